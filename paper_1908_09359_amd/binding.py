"""Thin ctypes binding of ``libvmcpeps.so`` (the C ABI in ``include/vmcpeps.h``).

Argument marshalling only: every step of the method runs in the HIP library.
Device buffers are torch tensors on the current HIP device; the functions pass
their ``data_ptr()`` and shapes.  Importing this module loads the library and
raises if it is missing; there is no CPU fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvmcpeps.so")

VP_OK, VP_ERR_ARG, VP_ERR_SHAPE, VP_ERR_OOM, VP_ERR_DEVICE = 0, 1, 2, 3, 4
VP_ERR_ZERO_AMPLITUDE, VP_ERR_NONFINITE, VP_ERR_UNSUPPORTED = 5, 6, 7
VP_COMPRESS_CANONICAL, VP_COMPRESS_VARIATIONAL = 0, 1
VP_GEOM_SQUARE, VP_GEOM_TRIANGULAR = 0, 1
VP_VERT_ROWPAIR, VP_VERT_COLUMN = 0, 1
VP_FP64, VP_FP32, VP_BF16 = 0, 1, 2
VP_SAMPLER_PAIR_SEQ, VP_SAMPLER_LEARNED_PLAQ, VP_SAMPLER_SIS_PAIR = 0, 1, 2
VP_SCHED_PHASES, VP_SCHED_PERSISTENT, VP_SCHED_GRAPH = 0, 1, 2
VP_TILE_DEFAULT, VP_TILE_SMALL, VP_TILE_LARGE, VP_N_TILES = 0, 1, 2, 3

STATUS_NAMES = {0: "VP_OK", 1: "VP_ERR_ARG", 2: "VP_ERR_SHAPE", 3: "VP_ERR_OOM", 4: "VP_ERR_DEVICE",
                5: "VP_ERR_ZERO_AMPLITUDE", 6: "VP_ERR_NONFINITE", 7: "VP_ERR_UNSUPPORTED"}

EXPORTED = ["vp_create", "vp_destroy", "vp_last_error", "vp_num_params", "vp_workspace_bytes",
            "vp_set_tensors", "vp_get_tensors", "vp_init_tensors", "vp_init_chains", "vp_sample",
            "vp_eval", "vp_gradient", "vp_sr_update", "vp_sign_sgd_update", "vp_sync",
            "vp_timing_enable", "vp_timing_read", "vp_stats_tau", "vp_trace_ratios", "vp_plaquette_ratios",
            "vp_proposal_num_params", "vp_proposal_set_weights", "vp_proposal_get_weights", "vp_proposal_forward",
            "vp_proposal_forward_noalloc", "vp_proposal_loss_grad", "vp_proposal_train", "vp_set_sampler", "vp_move_counts", "vp_set_schedule",
            "vp_sample_batch", "vp_autotune", "vp_sample_split", "vp_optimize", "vp_set_tile",
            "vp_autotune_tiles", "vp_eval_sis", "vp_simple_update", "vp_simple_update_lambdas",
            "vp_proposal_logits_sweep"]

PHASES = ["row3_envs", "hsweep", "row4_envs", "vsweep", "compress_up", "compress_down", "measure3",
          "measure4", "other"]


class vp_outputs(ctypes.Structure):
    _fields_ = [("log_abs_psi_dev", ctypes.c_void_p), ("sign_dev", ctypes.c_void_p), ("e_loc_dev", ctypes.c_void_p),
                ("dlnpsi_dev", ctypes.c_void_p), ("spins_out_dev", ctypes.c_void_p)]


class vp_lattice(ctypes.Structure):
    _fields_ = [("Ly", ctypes.c_int32), ("Lx", ctypes.c_int32), ("D", ctypes.c_int32), ("Dc", ctypes.c_int32),
                ("J1", ctypes.c_double), ("J2", ctypes.c_double), ("prec", ctypes.c_int32),
                ("n_chains", ctypes.c_int32), ("compress", ctypes.c_int32), ("fit_sweeps", ctypes.c_int32),
                ("geometry", ctypes.c_int32), ("vertical", ctypes.c_int32)]


class VPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    # torch's HIP runtime must be the one in the process: the library then
    # binds to it by soname instead of loading a second copy.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1908_09359_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    sig = {
        "vp_create": ([ctypes.POINTER(vp_lattice), I32, U64, P, ctypes.POINTER(P)], I32),
        "vp_destroy": ([P], I32),
        "vp_last_error": ([P], ctypes.c_char_p),
        "vp_num_params": ([ctypes.POINTER(vp_lattice)], I64),
        "vp_workspace_bytes": ([ctypes.POINTER(vp_lattice)], I64),
        "vp_set_tensors": ([P, I32, P], I32),
        "vp_get_tensors": ([P, I32, P], I32),
        "vp_init_tensors": ([P, I32, U64, D, D], I32),
        "vp_init_chains": ([P, I32, P], I32),
        "vp_sample": ([P, I32, I32, I32, P, P, P, P, P, P], I32),
        "vp_eval": ([P, I32, P, I32, P, P, P, P, P], I32),
        "vp_eval_sis": ([P, I32, P, I32, P, P, P, P], I32),
        "vp_gradient": ([P, I32, P, P, P, I64, P, P], I32),
        "vp_sr_update": ([P, I32, P, P, P, I64, D, D, P], I32),
        "vp_sign_sgd_update": ([P, I32, P, D, U64], I32),
        "vp_sync": ([P], I32),
        "vp_timing_enable": ([P, I32], I32),
        "vp_timing_read": ([P, P, P], I32),
        "vp_stats_tau": ([P, I32, I32, D, P, P, P], I32),
        "vp_trace_ratios": ([P, I32, P], I32),
        "vp_plaquette_ratios": ([P, I32, P, I32, P], I32),
        "vp_proposal_num_params": ([], I64),
        "vp_proposal_set_weights": ([P, I32, P], I32),
        "vp_proposal_get_weights": ([P, I32, P], I32),
        "vp_proposal_forward": ([P, I32, P, I32, P], I32),
        "vp_proposal_forward_noalloc": ([P, I32, P, I32, P], I32),
        "vp_proposal_logits_sweep": ([P, I32, P, I32, I32, P], I32),
        "vp_proposal_loss_grad": ([P, I32, P, P, I32, P, P], I32),
        "vp_proposal_train": ([P, I32, P, P, I64, I32, I32, D, U64, P], I32),
        "vp_set_sampler": ([P, I32, I32], I32),
        "vp_move_counts": ([P, I32, P], I32),
        "vp_set_schedule": ([P, I32, I32], I32),
        "vp_sample_batch": ([P, I32, P, I32, I32, P], I32),
        "vp_sample_split": ([P, I32, I32, I32, I32, P, P, P, P, P], I32),
        "vp_optimize": ([P, I32, I32, I32, I32, P, ctypes.c_uint64, P], I32),
        "vp_simple_update": ([P, I32, D, I32, P], I32),
        "vp_simple_update_lambdas": ([P, I32, P], I32),
        "vp_autotune": ([P, I32, I32, P, P], I32),
        "vp_set_tile": ([P, I32, I32], I32),
        "vp_autotune_tiles": ([P, I32, I32, P, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


LIB = _load()


def vp_proposal_num_params():
    return int(LIB.vp_proposal_num_params())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def lattice(Ly, Lx, D, Dc, J1=1.0, J2=0.0, prec=VP_FP64, n_chains=1, compress=0, fit_sweeps=0,
            geometry=0, vertical=0):
    """A vp_lattice; compress = VP_COMPRESS_CANONICAL (0) or VP_COMPRESS_VARIATIONAL (1);
    geometry = VP_GEOM_SQUARE (0) or VP_GEOM_TRIANGULAR (1); vertical = VP_VERT_ROWPAIR (0)
    or VP_VERT_COLUMN (1)."""
    return vp_lattice(Ly, Lx, D, Dc, J1, J2, prec, n_chains, compress, fit_sweeps, geometry, vertical)


def vp_num_params(lat):
    return int(LIB.vp_num_params(ctypes.byref(lat)))


def vp_workspace_bytes(lat):
    return int(LIB.vp_workspace_bytes(ctypes.byref(lat)))


def vp_stats_tau(series, c=5.0):
    """Per-chain tau_int, mean and tau-corrected standard error of a [n_chains][len] float64 array."""
    import numpy as np
    x = np.ascontiguousarray(series, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("series must be [n_chains][len]")
    tau = np.empty(x.shape[0])
    mean, err = ctypes.c_double(), ctypes.c_double()
    st = LIB.vp_stats_tau(x.ctypes.data_as(ctypes.c_void_p), x.shape[0], x.shape[1], c,
                          tau.ctypes.data_as(ctypes.c_void_p), ctypes.byref(mean), ctypes.byref(err))
    if st != VP_OK:
        raise VPError(st, LIB.vp_last_error(None).decode())
    return tau, mean.value, err.value


class Context:
    """Owns a vp_ctx; methods mirror the C functions of the same names."""

    def __init__(self, lats, seed=0, stream=None):
        if isinstance(lats, vp_lattice):
            lats = [lats]
        self.lats = list(lats)
        arr = (vp_lattice * len(self.lats))(*self.lats)
        h = ctypes.c_void_p()
        st = LIB.vp_create(arr, len(self.lats), ctypes.c_uint64(seed),
                           ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if st != VP_OK:
            raise VPError(st, LIB.vp_last_error(None).decode())
        self.h = h

    def _check(self, st):
        if st != VP_OK:
            raise VPError(st, LIB.vp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            LIB.vp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_params(self, lat=0):
        return vp_num_params(self.lats[lat])

    def vp_set_tensors(self, lat, T):
        self._check(LIB.vp_set_tensors(self.h, lat, _ptr(T)))

    def vp_get_tensors(self, lat, T):
        self._check(LIB.vp_get_tensors(self.h, lat, _ptr(T)))

    def vp_init_tensors(self, lat, seed, scale=0.0, perturb=0.0):
        self._check(LIB.vp_init_tensors(self.h, lat, ctypes.c_uint64(seed), scale, perturb))

    def vp_init_chains(self, lat, spins=None):
        self._check(LIB.vp_init_chains(self.h, lat, _ptr(spins)))

    def vp_sample(self, lat, n_burn, n_meas, log_abs_psi, sign, e_loc, dlnpsi=None, spins_out=None,
                  accept=None):
        self._check(LIB.vp_sample(self.h, lat, n_burn, n_meas, _ptr(log_abs_psi), _ptr(sign), _ptr(e_loc),
                                  _ptr(dlnpsi), _ptr(spins_out), _ptr(accept)))

    def vp_trace_ratios(self, lat, trace):
        """trace: float64 [n_chains, n_bonds, 2] device tensor (kept alive by the caller) or None."""
        self._trace = trace
        self._check(LIB.vp_trace_ratios(self.h, lat, _ptr(trace)))

    def vp_plaquette_ratios(self, lat, spins, n_cfg, ratios):
        self._check(LIB.vp_plaquette_ratios(self.h, lat, _ptr(spins), n_cfg, _ptr(ratios)))

    def vp_proposal_set_weights(self, lat, w):
        self._check(LIB.vp_proposal_set_weights(self.h, lat, _ptr(w)))

    def vp_proposal_get_weights(self, lat, w):
        self._check(LIB.vp_proposal_get_weights(self.h, lat, _ptr(w)))

    def vp_proposal_forward(self, lat, spins, n, logits):
        self._check(LIB.vp_proposal_forward(self.h, lat, _ptr(spins), n, _ptr(logits)))

    def vp_proposal_logits_sweep(self, lat, spins, n, flip, logits):
        self._check(LIB.vp_proposal_logits_sweep(self.h, lat, _ptr(spins), int(n), int(flip), _ptr(logits)))

    def vp_proposal_forward_noalloc(self, lat, spins, n, logits):
        self._check(LIB.vp_proposal_forward_noalloc(self.h, lat, _ptr(spins), n, _ptr(logits)))

    def vp_proposal_loss_grad(self, lat, spins, ratios, n, grad, loss):
        self._check(LIB.vp_proposal_loss_grad(self.h, lat, _ptr(spins), _ptr(ratios), n, _ptr(grad), _ptr(loss)))

    def vp_proposal_train(self, lat, spins, ratios, n, epochs, batch, lr, seed, loss=None):
        self._check(LIB.vp_proposal_train(self.h, lat, _ptr(spins), _ptr(ratios), n, epochs, batch, lr,
                                          ctypes.c_uint64(seed), _ptr(loss)))

    def vp_set_sampler(self, lat, sampler):
        self._check(LIB.vp_set_sampler(self.h, lat, sampler))

    def vp_set_schedule(self, lat, schedule):
        self._check(LIB.vp_set_schedule(self.h, lat, schedule))

    def vp_sample_batch(self, lats, n_burn, n_meas, outputs=None):
        """lats: lattice indices; outputs: one dict per lattice with log_abs_psi, sign, e_loc
        (and optionally dlnpsi, spins_out) device tensors, or None for unmeasured sweeps."""
        n = len(lats)
        idx = (ctypes.c_int32 * n)(*lats)
        outs = None
        if outputs is not None:
            outs = (vp_outputs * n)(*[vp_outputs(_ptr(o["log_abs_psi"]), _ptr(o["sign"]), _ptr(o["e_loc"]),
                                                 _ptr(o.get("dlnpsi")), _ptr(o.get("spins_out")))
                                      for o in outputs])
        self._check(LIB.vp_sample_batch(self.h, n, idx, n_burn, n_meas, outs))

    def vp_autotune(self, lat, sweeps):
        """Returns (chosen schedule, [ms per sweep of phases, persistent, graph])."""
        ms = (ctypes.c_double * 3)()
        pick = ctypes.c_int32()
        self._check(LIB.vp_autotune(self.h, lat, sweeps, ms, ctypes.byref(pick)))
        return pick.value, list(ms)

    def vp_set_tile(self, lat, tile):
        self._check(LIB.vp_set_tile(self.h, lat, tile))

    def vp_autotune_tiles(self, lat, sweeps):
        """Returns (chosen tile variant, [ms per sweep of VP_TILE_DEFAULT, VP_TILE_SMALL, VP_TILE_LARGE])."""
        ms = (ctypes.c_double * VP_N_TILES)()
        pick = ctypes.c_int32()
        self._check(LIB.vp_autotune_tiles(self.h, lat, sweeps, ms, ctypes.byref(pick)))
        return pick.value, list(ms)

    def vp_move_counts(self, lat, counts):
        self._check(LIB.vp_move_counts(self.h, lat, _ptr(counts)))

    def vp_sample_split(self, lat_sample, lat_measure, n_burn, n_meas, log_abs_psi, sign, e_loc, dlnpsi=None,
                        spins_out=None):
        self._check(LIB.vp_sample_split(self.h, lat_sample, lat_measure, n_burn, n_meas, _ptr(log_abs_psi),
                                        _ptr(sign), _ptr(e_loc), _ptr(dlnpsi), _ptr(spins_out)))

    def vp_optimize(self, lat, deltas, n_burn, n_meas, step0=0):
        """Algorithm 1 with step lengths `deltas` (one per step); returns the step energies (mean E_loc)."""
        d = (ctypes.c_double * len(deltas))(*[float(x) for x in deltas])
        e = (ctypes.c_double * len(deltas))()
        self._check(LIB.vp_optimize(self.h, lat, len(deltas), n_burn, n_meas, d, ctypes.c_uint64(step0), e))
        return list(e)

    def vp_simple_update(self, lat, dt, n_steps, change=None):
        self._check(LIB.vp_simple_update(self.h, lat, float(dt), int(n_steps), _ptr(change)))

    def vp_simple_update_lambdas(self, lat, lam):
        self._check(LIB.vp_simple_update_lambdas(self.h, lat, _ptr(lam)))

    def vp_eval(self, lat, spins, n_cfg, log_abs_psi, sign, e_loc, dlnpsi=None, ratios=None):
        self._check(LIB.vp_eval(self.h, lat, _ptr(spins), n_cfg, _ptr(log_abs_psi), _ptr(sign), _ptr(e_loc),
                                _ptr(dlnpsi), _ptr(ratios)))

    def vp_eval_sis(self, lat, spins, n_cfg, log_abs_phi, sign, e_loc, log_w):
        self._check(LIB.vp_eval_sis(self.h, lat, _ptr(spins), n_cfg, _ptr(log_abs_phi), _ptr(sign), _ptr(e_loc),
                                    _ptr(log_w)))

    def vp_gradient(self, lat, e_loc, dlnpsi, spins, n_samples, grad, e_mean):
        self._check(LIB.vp_gradient(self.h, lat, _ptr(e_loc), _ptr(dlnpsi), _ptr(spins), n_samples,
                                    _ptr(grad), _ptr(e_mean)))

    def vp_sr_update(self, lat, e_loc, dlnpsi, spins, n_samples, shift, lr, delta=None):
        self._check(LIB.vp_sr_update(self.h, lat, _ptr(e_loc), _ptr(dlnpsi), _ptr(spins), n_samples, shift, lr,
                                     _ptr(delta)))

    def vp_sign_sgd_update(self, lat, grad, step_len, step):
        self._check(LIB.vp_sign_sgd_update(self.h, lat, _ptr(grad), step_len, ctypes.c_uint64(step)))

    def vp_sync(self):
        self._check(LIB.vp_sync(self.h))

    def vp_timing_enable(self, enable=True):
        self._check(LIB.vp_timing_enable(self.h, 1 if enable else 0))

    def vp_timing_read(self):
        """Per-phase (milliseconds, launches) since the last vp_timing_enable, as dicts."""
        ms = (ctypes.c_double * len(PHASES))()
        n = (ctypes.c_int64 * len(PHASES))()
        self._check(LIB.vp_timing_read(self.h, ms, n))
        return dict(zip(PHASES, list(ms))), dict(zip(PHASES, list(n)))
