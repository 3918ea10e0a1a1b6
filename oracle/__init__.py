"""FP64 CPU oracle for variational Monte Carlo on finite open-boundary PEPS.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports, calls or
falls back to it, and this package shares no code with the HIP path.

It is a plain, slow, step-by-step statement of what the method computes
(Liu, Huang, Gong, Gu, "Accurate simulation for finite projected entangled pair
states in two dimensions"):

* ``philox``   -- the counter-based generator (Philox4x64-10 of Salmon et al.,
                  SC'11) written from its published definition, plus the
                  uniform / Gaussian / shuffle conversions built on it.
* ``lattice``  -- lattice geometry, tensor layout, Hamiltonian bonds and matrix
                  elements (Sec. II.A Eq. (3); App. C Eq. (Elocal)).
* ``peps``     -- single-layer contraction: boundary MPS with canonical QR/SVD
                  truncation (App. B), row networks with auxiliary tensors
                  (App. C), amplitudes, ratios, defect networks (Eqs. (4)-(7)).
* ``vmc``      -- fixed-configuration evaluation, the sequential bond-visiting
                  Metropolis sweep (Sec. II.A Eq. (9)), estimators (Eqs. (2),
                  (5)), the stochastic sign-gradient update (Eq. (10)) and a
                  stochastic-reconfiguration step.

Everything is float64 numpy; factorizations use LAPACK through numpy.

Parity status per function is stated in each module header.  Functions whose
output on truncated networks has no external truth (compression at Dc below the
exact rank) are pinned by invariants only; they say so in their docstrings.
"""
