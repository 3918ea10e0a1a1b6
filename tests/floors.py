"""Rounding floor of the oracle's truncated evaluation (test infrastructure).

The boundary compression (App. B) truncates at singular values that are close
together for the random networks of the benchmark workloads, so Psi, E_loc,
the pair ratios and the log-derivatives depend on the last bits of every
compression input.  No implementation that rounds differently can be expected
to agree with the oracle more closely than the oracle agrees with itself when
those inputs move by one unit in the last place.

``perturbed_eval`` runs the oracle's own ``eval_config`` with every input tensor
of every boundary compression multiplied by (1 + eps xi), xi ~ N(0, 1) i.i.d.
from a seeded stream (nothing else changes).  ``floor`` is the largest
deviation from the unperturbed evaluation over several seeds: the per-output
floor that the GPU parity bounds are derived from (a bound is a small multiple
of it, never below the float64 bounds of the small lattices).  The float64
floor perturbs the compression inputs at the float64 unit; the float32 floor
models float32 storage (``storage=True``): the site tensors, the compression
inputs and the compressed boundaries, each at the float32 unit.
"""
import numpy as np

from oracle import peps, vmc

F64_UNIT = 2.0 ** -52
F32_UNIT = 2.0 ** -24


def perturbed_eval(T, lat, spins, eps, seed, storage=False):
    """oracle.vmc.eval_config with every compression input (canonical or
    variational) scaled by (1 + eps xi).  With ``storage`` also the site
    tensors and every compression output: the model of an implementation that
    stores every tensor in a format of unit eps (the float32 path stores the
    site tensors, boundaries and environments in float32)."""
    exact, exact_fit = peps.compress, peps.compress_variational
    rng = np.random.default_rng(seed)

    def jitter(B):
        return [b * (1.0 + eps * rng.standard_normal(b.shape)) for b in B]

    def out(res):
        return (jitter(res[0]), res[1]) if storage else res

    def perturbed(B, Dc):
        return out(exact(jitter(B), Dc))

    def perturbed_fit(B, Dc, sweeps, **kw):
        return out(exact_fit(jitter(B), Dc, sweeps, **kw))

    if storage:
        T = np.asarray(T) * (1.0 + eps * rng.standard_normal(np.shape(T)))

    peps.compress, peps.compress_variational = perturbed, perturbed_fit
    vmc.compress = perturbed
    try:
        return vmc.eval_config(T, lat, spins)
    finally:
        peps.compress, peps.compress_variational = exact, exact_fit
        vmc.compress = exact


def deviations(a, b, n_sites):
    """Per-output deviation of evaluation ``a`` from ``b``: |dE|/site, |d log|Psi||,
    the largest relative ratio deviation (relative to max(1, |ratio|)) and the
    largest log-derivative deviation relative to max(1, max |G|)."""
    return dict(
        e_site=abs(a["e_loc"] - b["e_loc"]) / n_sites,
        log_abs_psi=abs(a["log_abs_psi"] - b["log_abs_psi"]),
        ratio=float(np.max(np.abs(a["ratios"] - b["ratios"]) / np.maximum(1.0, np.abs(b["ratios"])))
                    if len(b["ratios"]) else 0.0),
        dlnpsi=float(np.max(np.abs(a["dlnpsi"] - b["dlnpsi"])) / max(1.0, float(np.max(np.abs(b["dlnpsi"]))))),
    )


def floor(T, lat, spins, eps, seeds, base=None):
    """Largest deviation of each output over the perturbed evaluations with ``seeds``."""
    if base is None:
        base = vmc.eval_config(T, lat, spins)
    n = lat.Ly * lat.Lx
    out = dict(e_site=0.0, log_abs_psi=0.0, ratio=0.0, dlnpsi=0.0)
    for s in seeds:
        dv = deviations(perturbed_eval(T, lat, spins, eps, s), base, n)
        out = {k: max(out[k], dv[k]) for k in out}
    return out
