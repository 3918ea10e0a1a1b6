"""Counter-based random numbers for the oracle (test infrastructure only).

Philox4x64-10 is written out from its published definition (Salmon, Moraes,
Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4x64-bit
counter, a 2x64-bit key, ten rounds, each round two 64x64->128 multiplications
followed by a word permutation and a key xor; the key is advanced by the two
Weyl constants between rounds.  Pure-Python integers make the arithmetic
obviously exact.

Pinned by ``tests/test_oracle_rng.py`` against NumPy's own Philox bit generator
(an independent implementation of the same definition).

Stream layout used by every random decision of the method (both sides
implement it):

    key     = (seed, lattice_id)
    counter = (c0, c1, c2, tag)

with ``tag`` one of the TAG_* constants below.
"""

MASK64 = (1 << 64) - 1

# Philox4x64 multipliers and Weyl key increments (published constants).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B

TAG_INIT = 1       # Gaussian tensor initialisation: counter (param, 0, 0, TAG)
TAG_PERTURB = 2    # extra Gaussian perturbation:    counter (param, 0, 0, TAG)
TAG_SHUFFLE = 3    # Fisher-Yates start shuffle:     counter (chain, 0, i, TAG)
TAG_METRO = 4      # Metropolis uniform:             counter (chain, sweep, bond, TAG)
TAG_SGD = 5        # sign-gradient random step:      counter (param, step, 0, TAG)
TAG_PLAQ = 6       # plaquette proposal (word 0: propose, word 1: accept):
                   #                                 counter (chain, sweep, plaquette, TAG)


def philox4x64_10(counter, key):
    """One Philox4x64-10 block: four 64-bit words from a 4-word counter and 2-word key."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in counter)
    k0, k1 = (int(v) & MASK64 for v in key)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform53(word):
    """Uniform double in [0, 1): the top 53 bits of a 64-bit word times 2^-53 (exact)."""
    return float(int(word) >> 11) * (1.0 / 9007199254740992.0)


def gaussian(counter, key):
    """Standard normal by the Box-Muller transform (Box & Muller, 1958) of words 0 and 1."""
    import math
    w = philox4x64_10(counter, key)
    u1 = uniform53(w[0])
    u2 = uniform53(w[1])
    return math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)


def bounded_index(word, n):
    """floor(u * n) for u = uniform53(word), computed exactly in integers (n < 2^11)."""
    return ((int(word) >> 11) * int(n)) >> 53


def metropolis_uniform(seed, lattice_id, chain, sweep, bond):
    """The uniform r compared with the acceptance ratio at one visited bond."""
    w = philox4x64_10((chain, sweep, bond, TAG_METRO), (seed, lattice_id))
    return uniform53(w[0])


def plaquette_uniforms(seed, lattice_id, chain, sweep, plaquette):
    """(u_propose, u_accept) of the plaquette move q = y*(Lx-1) + x."""
    w = philox4x64_10((chain, sweep, plaquette, TAG_PLAQ), (seed, lattice_id))
    return uniform53(w[0]), uniform53(w[1])
