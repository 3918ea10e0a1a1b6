"""Throughput benchmark of the VMC-PEPS hot path on one MI355X.

One step = one sequential Metropolis sweep of every chain (top-down sampling
pass over all horizontal and vertical bonds -- plus, on the learned path, the
plaquette moves of every row pair -- then the bottom-up measurement pass),
producing Psi, E_loc and the log-derivatives dlnPsi/dT of every chain.

Two paths on the 16x16, D=8, Dc=16 Heisenberg workload:

* plain:   float32 contractions, nearest-neighbour pair sweeps;
* learned: bf16-operand 2-row steps and float64 3-line steps in the sampling
           pass over float64 storage, float64 measurement, pair
           sweeps plus learned plaquette moves; the proposal network is first
           trained (untimed) on configurations of the same chains.

    python bench.py [--steps K] [--warmup W] [--chains C] [--tau-sweeps S]

Prints one JSON line whose value is the learned path's samples/s; the plain
path is reported beside it.  After each path's timed region (untimed): tau_int
of its own E_loc/N and M_z^2 series, and the E/N bias of its measured
configurations against a float64 evaluation of the same configurations; for
the learned path also its bf16 sampling ratios and decisions against float64
along the same sweep.  From these, the time ratio at fixed dE (dE^2 = stderr^2
+ bias^2).  With --tau-sweeps S > 0 both paths also run S further measured
sweeps for a longer tau_int estimate.  Inputs are synthetic (seeded Gaussian
tensors of standard deviation 1/D^2, Philox-shuffled Neel starts) and resident
in HBM before the timed region.  The CPU baseline (the oracle, one process per
host core) runs first, before this process touches the GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "samples/s (psi, E_loc, dlnpsi) 16x16 D=8 Dc=16, learned+bf16 vs plain at fixed dE"

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "hbm": 8.0e12}

# HBM bytes per launch of the phases' kernels, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs (profiles/hbm_traffic_16x16_D8_Dc16_1024ch.md), each scaled by
# what the same counter reads for a device-to-device copy of known size.  They
# describe the kernel sources whose digest is `src`; for any other sources the
# benchmark reports no traffic.
TRAFFIC = {"src": "212d7b8258b52189",
           "bytes_per_launch": {
               # k_compress<double, 8, 16> (both directions): 1.880e+07 KiB fetched x 2.0, 1.818e+07 KiB written
               "learned": {"compress_up": 5.7122e+10, "compress_down": 5.7122e+10,
                           "measure4": 4.6200e+10, "vsweep": 4.3536e+10},
               # k_compress<float, 8, 16>: 1.850e+07 KiB fetched x 2.0, 1.797e+07 KiB written
               "plain": {"compress_up": 5.6288e+10, "compress_down": 5.6288e+10,
                         "measure4": 1.8356e+10, "vsweep": 1.2506e+10}}}


def kernel_source_digest():
    """sha256 over the sources of the phase kernels: vp_kernels.hip and every header it
    includes, directly or through other headers (names and contents)."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1908_09359_amd", "csrc")
    seen, todo = set(), ["vp_kernels.hip"]
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(os.path.join(csrc, f)):
            continue
        seen.add(f)
        with open(os.path.join(csrc, f)) as fh:
            todo += re.findall(r'#include "([^"/]+)"', fh.read())
    h = hashlib.sha256()
    for f in sorted(seen):
        h.update(f.encode())
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def phase_flops(Ly, Lx, D, Dc, nch, launches, anti_h=0, anti_v=0, fit_sweeps=None):
    """Algorithmic flops of each phase over the timed region (all chains, all launches).

    Column-step costs (multiply-adds, bulk dimensions):
      3-line step   D^4 Dc^2 + 2 D^2 Dc^3
      2-row step    2 D^5 Dc^2 + 2 D^3 Dc^3
      defect        D^4 Dc^2 + 2 D^2 Dc^3  ((Lp.A)(B.Rn), contracted over two bonds at a time)
      compression of one row (Gram steps, right-to-left carries, eigenproblems
      of order n = D Dc: tridiagonalisation 4/3 n^3 flops, back-transformation
      4 n^2 Dc flops)
    A measurement launch (one row, or one row pair) computes the right and left
    environments (Lx-1 steps each), the defects of the row's sites, and one ratio
    network per antiparallel pair: two 3-line steps for a horizontal pair, one
    2-row step for a vertical pair.  anti_h / anti_v are the numbers of
    antiparallel horizontal / vertical pairs in the configurations measured.
    With fit_sweeps (the variational fit instead of the canonical compression),
    a row's compression is (Lx-1)(1 + 2 S) 3-line environment steps, 2 S (Lx-1)
    + 1 optimal-site contractions (D^4 Dc^2 + 2 D^2 Dc^3 each) and Lx - 1 + 2 S
    (Lx - 1) Householder QRs of (D Dc) x Dc blocks (4 m n^2 - 4/3 n^3 flops,
    factorisation and Q).
    """
    c, d = Dc, D
    env3 = d ** 4 * c ** 2 + 2 * d ** 2 * c ** 3
    env4 = 2 * d ** 5 * c ** 2 + 2 * d ** 3 * c ** 3
    defect = d ** 4 * c ** 2 + 2 * d ** 2 * c ** 3
    n = d * c
    comp_mac = (Lx - 1) * env4 + Lx * (d ** 2 * c ** 3 + d ** 4 * c ** 2) + (Lx - 1) * (2 * n ** 3 + d ** 2 * c ** 3)
    comp = 2 * comp_mac + (Lx - 1) * (4.0 / 3.0 * n ** 3 + 4 * n ** 2 * c)
    if fit_sweeps is not None:
        S = fit_sweeps
        qr = 4.0 * n * c * c - 4.0 / 3.0 * c ** 3
        comp = 2.0 * ((Lx - 1) * (1 + 2 * S) * env3 + (2 * S * (Lx - 1) + 1) * env3) + (Lx - 1) * (1 + 2 * S) * qr
    per_launch = {"row3_envs": 2 * (Lx - 1) * env3, "row4_envs": 2 * (Lx - 1) * env4,
                  "compress_up": comp, "compress_down": comp}
    out = {k: v * nch * launches.get(k, 0) for k, v in per_launch.items()}
    out["measure3"] = 2.0 * (nch * launches.get("measure3", 0) * (2 * (Lx - 1) * env3 + Lx * defect)
                             + anti_h * 2 * env3)
    out["measure4"] = 2.0 * (nch * launches.get("measure4", 0) * 2 * (Lx - 1) * env4 + anti_v * env4)
    return out


def _oracle_chain_sweep(args):
    """One chain of the oracle: one sweep (sampling + measurement) of the workload, one thread; seconds."""
    Ly, Lx, D, Dc, seed, chain = args
    from threadpoolctl import threadpool_limits
    from oracle import lattice as olat
    from oracle import vmc
    from paper_1908_09359_amd import workloads as W
    lat = olat.Lattice(Ly, Lx, D, Dc)
    T = W.random_tensors(Ly, Lx, D, seed=seed)
    ch = vmc.Chain(lat, olat.neel_shuffled(lat, 9359, 0, chain), 9359, 0, chain)
    with threadpool_limits(limits=1):
        Dl = vmc._lower_boundaries(T, lat, ch.spins)
        t0 = time.perf_counter()
        U, _ = vmc._top_down_pass(T, lat, ch, Dl)
        vmc._measure(T, lat, ch.spins, U)
        return time.perf_counter() - t0


def cpu_baseline(Ly, Lx, D, Dc, seed, max_procs=16):
    """The oracle on the host's cores: one single-threaded process per core, each
    running one chain's sweep; samples/s = chains / the slowest chain's time."""
    import multiprocessing as mp
    procs = max(1, min(os.cpu_count() or 1, max_procs))
    with mp.get_context("spawn").Pool(procs) as pool:
        times = pool.map(_oracle_chain_sweep, [(Ly, Lx, D, Dc, seed, c) for c in range(procs)])
    wall = max(times)
    return {"value": procs / wall, "unit": "samples/s", "cores": procs, "kind": "oracle",
            "per_core": 1.0 / (sum(times) / len(times)),
            "sample": f"{procs} chains x 1 sweep (pair moves, sampling + measurement) of {Ly}x{Lx} D={D} Dc={Dc}, "
                      f"float64 numpy, one single-threaded process per core; {wall:.1f} s for the slowest chain",
            "paper": {"value_per_core": 0.044, "unit": "samples/s per core",
                      "hardware": "Intel E5-2620 (500 cores), 32x32 D=8, Dc 16 sampling / 24 measurement, "
                                  "derived from the optimisation wall time quoted in Sec. II.B (4 days, 170 steps "
                                  "x 45000 sweeps)"}}


def set_tensors(ctx, T=None):
    """The workload's tensors: given ones (a device tensor), or the seeded N(0,1)/D^2 draw."""
    if T is None:
        ctx.vp_init_tensors(0, seed=1908, scale=0.0, perturb=0.0)
    else:
        ctx.vp_set_tensors(0, T)


def correlated_tensors(B, torch, L, D, seed=7, steps=200, dt=0.05):
    """A correlated stand-in for the paper's optimised states: the simple-update state
    (App. A, the paper's initialisation before Algorithm 1) of the L x L Heisenberg
    lattice at bond dimension D, `steps` steps of dt from seeded N(0,1)/D^2 tensors."""
    import numpy as np
    t0 = time.perf_counter()
    dev = torch.device("cuda:0")
    ctx = B.Context(B.lattice(L, L, D, 4, 1.0, 0.0, B.VP_FP64, 1), seed=seed)
    ctx.vp_init_tensors(0, seed=seed, scale=0.0, perturb=0.0)
    ch = torch.zeros(steps, dtype=torch.float64, device=dev)
    ctx.vp_simple_update(0, dt, steps, ch)
    T = torch.empty(ctx.num_params(), dtype=torch.float64, device=dev)
    ctx.vp_get_tensors(0, T)
    ctx.vp_sync()
    c = ch.cpu().numpy()
    ctx.close()
    info = {"recipe": f"{L}x{L} D={D} simple-update state (App. A): seeded N(0,1)/D^2 tensors, {steps} steps of "
                      f"dt {dt}", "su_change_first": float(c[0]), "su_change_last": float(c[-1]),
            "seconds": time.perf_counter() - t0}
    return T, info


class Path:
    """One lattice context, its output buffers and the sweep loop of one path."""

    def __init__(self, B, torch, Ly, Lx, D, Dc, prec, nch, seed=9359, compress=0, fit_sweeps=0, T=None):
        self.B, self.torch = B, torch
        self.Ly, self.Lx, self.N = Ly, Lx, Ly * Lx
        self.prec, self.nch = prec, nch
        self.dev = torch.device("cuda:0")
        self.ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, prec, nch, compress, fit_sweeps), seed=seed)
        set_tensors(self.ctx, T)
        self.ctx.vp_init_chains(0, None)
        dt = torch.float32 if prec == B.VP_FP32 else torch.float64
        self.lp = torch.empty(nch, dtype=torch.float64, device=self.dev)
        self.sg = torch.empty(nch, dtype=torch.int8, device=self.dev)
        self.el = torch.empty(nch, dtype=torch.float64, device=self.dev)
        self.dl = torch.empty((nch, self.ctx.num_params() // 2), dtype=dt, device=self.dev)
        self.so = torch.empty((nch, self.N), dtype=torch.int8, device=self.dev)

    def sweep(self, spins=False):
        self.ctx.vp_sample(0, 0, 1, self.lp, self.sg, self.el, self.dl, self.so if spins else None)

    def train_proposal(self, sweeps, epochs, batch, lr):
        """Configurations of `sweeps` pair sweeps -> plaquette ratios -> Adam; chains resume after."""
        B, torch = self.B, self.torch
        from paper_1908_09359_amd.workloads import random_proposal_weights
        t0 = time.perf_counter()
        npl = (self.Ly - 1) * (self.Lx - 1)
        cfgs = torch.empty((sweeps * self.nch, self.N), dtype=torch.int8, device=self.dev)
        for s in range(sweeps):
            self.sweep(spins=True)
            cfgs[s * self.nch:(s + 1) * self.nch].copy_(self.so)
            if sweeps > 200 and (s + 1) % 500 == 0:
                self.ctx.vp_sync()
                print(f"training data: {(s + 1) * self.nch} configurations", file=sys.stderr, flush=True)
        last = self.so.clone()
        rho = torch.empty((sweeps * self.nch, npl), dtype=torch.float64, device=self.dev)
        for s in range(sweeps):
            self.ctx.vp_plaquette_ratios(0, cfgs[s * self.nch:(s + 1) * self.nch], self.nch,
                                         rho[s * self.nch:(s + 1) * self.nch])
            if sweeps > 200 and (s + 1) % 500 == 0:
                self.ctx.vp_sync()
                print(f"training targets: {(s + 1) * self.nch} configurations", file=sys.stderr, flush=True)
        w = torch.tensor(random_proposal_weights(seed=4), device=self.dev)
        self.ctx.vp_proposal_set_weights(0, w)
        loss = torch.empty(epochs, dtype=torch.float64, device=self.dev)
        self.ctx.vp_proposal_train(0, cfgs, rho, cfgs.shape[0], epochs, batch, lr, 11, loss)
        # evaluation reused the chain slots: the chains continue from their last states
        self.ctx.vp_init_chains(0, last)
        self.ctx.vp_set_sampler(0, B.VP_SAMPLER_LEARNED_PLAQ)
        self.ctx.vp_sync()
        return {"configs": int(cfgs.shape[0]), "epochs": epochs, "batch": batch, "lr": lr,
                "loss_first_epoch": float(loss[0].item()), "loss_last_epoch": float(loss[-1].item()),
                "seconds": time.perf_counter() - t0}

    def timed(self, warmup, steps):
        torch = self.torch
        for _ in range(warmup):
            self.sweep()
        self.ctx.vp_sync()
        torch.cuda.synchronize()
        cnt0 = self.counts()
        # the configurations measured in each step (an output of the sweep)
        so = torch.empty((steps, self.nch, self.N), dtype=torch.int8, device=self.dev)
        el = torch.empty((steps, self.nch), dtype=torch.float64, device=self.dev)
        self.ctx.vp_timing_enable(True)
        t0 = time.perf_counter()
        for s in range(steps):
            self.ctx.vp_sample(0, 0, 1, self.lp, self.sg, el[s], self.dl, so[s])
        self.ctx.vp_sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms, launches = self.ctx.vp_timing_read()
        self.ctx.vp_timing_enable(False)
        cnt = self.counts() - cnt0
        g = so.view(steps, self.nch, self.Ly, self.Lx)
        anti_h = int((g[..., :, 1:] != g[..., :, :-1]).sum().item())
        anti_v = int((g[..., 1:, :] != g[..., :-1, :]).sum().item())
        self.el.copy_(el[-1])
        self.last_spins, self.el_series, self.spin_series = so[-1], el, so
        return {"samples_per_s": self.nch * steps / dt, "ms_per_step": dt / steps * 1e3, "ms": ms,
                "launches": launches, "seconds": dt, "anti_h": anti_h, "anti_v": anti_v,
                "pair_accept": float(cnt[0] / max(cnt[1], 1)),
                "plaquette_accept": float(cnt[2] / cnt[3]) if cnt[3] else None,
                "plaquette_proposed_per_sweep": float(cnt[3] / self.nch / steps),
                "e_site_last_sweep": float(el[-1].mean().item()) / self.N}

    def series_stats(self):
        """tau_int (Sokal window 5) and variance per sample of the timed sweeps' own series:
        E_loc / N, and the squared staggered magnetisation M_z^2 (a function of the
        configuration alone)."""
        import numpy as np
        torch = self.torch
        x = self.el_series.t().contiguous().cpu().numpy() / self.N          # [chains][steps]
        g = self.spin_series.view(-1, self.nch, self.Ly, self.Lx).to(torch.float64)
        yy = torch.arange(self.Ly, device=self.dev).view(-1, 1)
        xx = torch.arange(self.Lx, device=self.dev).view(1, -1)
        stag = ((-1.0) ** (yy + xx)).to(torch.float64)
        mz = ((0.5 - g) * stag).sum(dim=(2, 3)) / self.N                   # [steps][chains]
        m2 = (mz * mz).t().contiguous().cpu().numpy()
        out = {"series_length": int(x.shape[1])}
        if x.shape[1] < 2:  # one timed sweep: no series to analyse
            return None
        for name, v in (("e_site", x), ("mz2", m2)):
            tau, mean, err = self.B.vp_stats_tau(v, 5.0)
            out[name] = {"tau_int_mean": float(np.mean(tau)), "mean": mean, "stderr": err,
                         "var_per_sample": float(np.mean(np.var(v, axis=1, ddof=1)))}
        return out

    def tau_run(self, sweeps):
        """`sweeps` measured sweeps: tau_int of E_loc/N per chain and the tau-corrected error of E/N."""
        import numpy as np
        torch = self.torch
        series = torch.empty((sweeps, self.nch), dtype=torch.float64, device=self.dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(sweeps):
            self.sweep()
            series[s].copy_(self.el)
            print(f"tau sweep {s + 1}/{sweeps}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        x = series.t().contiguous().cpu().numpy() / self.N
        tau, mean, err = self.B.vp_stats_tau(x, 5.0)
        var = float(np.mean(np.var(x, axis=1, ddof=1)))
        return {"sweeps": sweeps, "seconds": dt, "samples_per_s": self.nch * sweeps / dt,
                "tau_int_mean": float(np.mean(tau)), "e_site": mean, "e_site_stderr": err,
                "var_e_site_per_sample": var}

    def counts(self):
        c = self.torch.empty((self.nch, 4), dtype=self.torch.int64, device=self.dev)
        self.ctx.vp_move_counts(0, c)
        return c.sum(dim=0).cpu().numpy()

    def close(self):
        self.ctx.close()


def split_run(B, torch, Ly, Lx, D, Dc1, Dc2, nch, warmup, steps, seed=9359):
    """Two cutoffs: bf16-operand sampling at Dc1, float64 measurement at Dc2 (vp_sample_split)."""
    dev = torch.device("cuda:0")
    ctx = B.Context([B.lattice(Ly, Lx, D, Dc1, 1.0, 0.0, B.VP_BF16, nch),
                     B.lattice(Ly, Lx, D, Dc2, 1.0, 0.0, B.VP_BF16, nch)], seed=seed)
    ctx.vp_init_tensors(0, seed=1908, scale=0.0, perturb=0.0)
    T = torch.empty(ctx.num_params(0), dtype=torch.float64, device=dev)
    ctx.vp_get_tensors(0, T)
    ctx.vp_set_tensors(1, T)
    ctx.vp_init_chains(0, None)
    lp = torch.empty(nch * steps, dtype=torch.float64, device=dev)
    sg = torch.empty(nch * steps, dtype=torch.int8, device=dev)
    el = torch.empty(nch * steps, dtype=torch.float64, device=dev)
    dl = torch.empty((nch * steps, ctx.num_params(1) // 2), dtype=torch.float64, device=dev)
    ctx.vp_sample_split(0, 1, warmup, 1, lp[:nch], sg[:nch], el[:nch], dl[:nch])
    ctx.vp_sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.vp_sample_split(0, 1, 0, steps, lp, sg, el, dl)
    ctx.vp_sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    e = float(el.mean().item()) / (Ly * Lx)
    ctx.close()
    return {"workload": f"{Ly}x{Lx} Heisenberg D={D}, sampling Dc1={Dc1} (bf16-operand 2-row steps), "
                        f"measurement Dc2={Dc2} (float64), {nch} chains",
            "samples_per_s": nch * steps / dt, "ms_per_step": dt / steps * 1e3, "e_site_mean": e}


def fp64_reference(B, torch, Ly, Lx, D, Dc, spins, e_loc, n, compress=0, fit_sweeps=0, T=None):
    """The first n of a path's measured configurations re-evaluated in float64 (vp_eval, untimed,
    same truncation): the bias of the path's E_loc / N against the float64 evaluation of the same
    configurations."""
    import numpy as np
    dev = torch.device("cuda:0")
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, B.VP_FP64, n, compress, fit_sweeps), seed=1)
    set_tensors(ctx, T)  # the paths' tensors
    lp = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    ctx.vp_eval(0, spins[:n].contiguous(), n, lp, sg, el)
    ctx.vp_sync()
    d = (e_loc[:n].cpu().numpy() - el.cpu().numpy()) / (Ly * Lx)
    ctx.close()
    return {"configs": n, "bias_e_site": float(d.mean()), "bias_stderr": float(d.std(ddof=1) / np.sqrt(n)),
            "mean_abs_e_site": float(np.abs(d).mean()), "max_abs_e_site": float(np.abs(d).max())}


def bf16_decisions(B, torch, Ly, Lx, D, Dc, starts, seed=4242, compress=0, fit_sweeps=0, T=None):
    """One traced pair sweep from the same starts in float64 and with bf16-operand sampling
    steps, same seed: along each chain, until the first decision that differs (after which
    the configurations differ), the bf16 ratio's relative error against the float64 ratio of
    the same bond, and how often a decision differs."""
    import numpy as np
    dev = torch.device("cuda:0")
    n = starts.shape[0]
    nb = Ly * (Lx - 1) + (Ly - 1) * Lx
    tr = {}
    for prec in (B.VP_FP64, B.VP_BF16):
        ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, 0.0, prec, n, compress, fit_sweeps), seed=seed)
        set_tensors(ctx, T)
        ctx.vp_init_chains(0, starts.contiguous())
        t = torch.full((n, nb, 2), -1.0, dtype=torch.float64, device=dev)
        ctx.vp_trace_ratios(0, t)
        lp = torch.empty(n, dtype=torch.float64, device=dev)
        sg = torch.empty(n, dtype=torch.int8, device=dev)
        el = torch.empty(n, dtype=torch.float64, device=dev)
        ctx.vp_sample(0, 0, 1, lp, sg, el)
        ctx.vp_sync()
        tr[prec] = t.cpu().numpy()
        ctx.close()
    a, b = tr[B.VP_FP64], tr[B.VP_BF16]
    # bond k of row y: horizontal for k - y (2 Lx - 1) < Lx - 1, vertical otherwise
    vertical = np.array([(k % (2 * Lx - 1)) >= Lx - 1 for k in range(nb)])
    rel, vert, flips, agreed = [], [], 0, 0
    for c in range(n):
        for k in range(nb):
            if a[c, k, 1] != b[c, k, 1]:
                flips += 1
                break
            if a[c, k, 0] != 0.0:
                agreed += 1
                rel.append(abs(b[c, k, 0] - a[c, k, 0]) / abs(a[c, k, 0]))
                vert.append(vertical[k])
    rel, vert = np.array(rel), np.array(vert, dtype=bool)
    rv = rel[vert] if vert.any() else rel
    return {"chains": n, "bonds_compared": int(len(rel)), "rel_err_median": float(np.median(rel)),
            "rel_err_p95": float(np.quantile(rel, 0.95)),
            "vertical_bonds_compared": int(vert.sum()), "vertical_rel_err_median": float(np.median(rv)),
            "vertical_rel_err_p95": float(np.quantile(rv, 0.95)),
            "decisions_differing_per_proposal": flips / max(agreed + flips, 1)}


def fixed_de(plain, learned):
    """Time ratio plain / learned at the accuracy the plain path reached in its timed run.

    Per path: stderr^2 = v 2 tau / (rate t) (v: E_loc/N variance per sample, tau: its
    integrated autocorrelation time in sweeps), and dE^2 = stderr^2 + bias^2 with bias^2 the
    squared E/N bias against float64 less the variance of that estimate (floored at 0).  Target dE = the plain path's dE after its timed
    seconds; the learned path needs t = v 2 tau / (rate (dE^2 - bias^2)) to reach it.
    Both paths sample |Psi|^2 of the same tensors, so v is the same in expectation; its
    estimates from heavy-tailed E_loc series are noisy, so v is pooled over both paths
    (weighted by their sample counts; the per-path estimates are reported beside it).
    Also given: the same ratio without the bias terms, and with neither bias nor variance
    (2 tau / rate only)."""
    if plain["stats"] is None or learned["stats"] is None:
        return {"ratio": None, "ratio_without_bias": None, "ratio_tau_and_rate_only": None,
                "reason": "one timed sweep per chain: no series"}

    def parts(r):
        # the squared bias less the variance of its estimate (floored at 0): the mean of a few
        # hundred heavy-tailed differences carries its own noise
        st, ref = r["stats"]["e_site"], r["fp64_reference"]
        b2 = max(ref["bias_e_site"] ** 2 - ref["bias_stderr"] ** 2, 0.0)
        return st["var_per_sample"], st["tau_int_mean"], r["samples_per_s"], b2 ** 0.5
    vp, tp, rp, bp = parts(plain)
    vl, tl, rl, bl = parts(learned)
    if min(vp, tp, vl, tl) <= 0.0:
        # a few sweeps per chain: the windowed tau_int estimate can come out at or below zero
        return {"ratio": None, "ratio_without_bias": None, "ratio_tau_and_rate_only": None,
                "reason": f"tau_int or variance not positive (tau {tp:.3g} / {tl:.3g}, var {vp:.3g} / {vl:.3g}): "
                          "too few timed sweeps per chain"}
    t_plain = plain["seconds"]
    n_p, n_l = plain["samples_per_s"] * plain["seconds"], learned["samples_per_s"] * learned["seconds"]
    v = (vp * n_p + vl * n_l) / (n_p + n_l)
    se2 = v * 2 * tp / (rp * t_plain)
    de2 = se2 + bp * bp
    t_learned = v * 2 * tl / (rl * (de2 - bl * bl)) if de2 > bl * bl else float("inf")
    return {"target_dE_e_site": de2 ** 0.5, "plain_stderr": se2 ** 0.5, "plain_bias": bp, "learned_bias": bl,
            "var_per_sample_pooled": v, "var_per_sample_plain": vp, "var_per_sample_learned": vl,
            "plain_seconds": t_plain, "learned_seconds": t_learned, "ratio": t_plain / t_learned,
            "ratio_without_bias": (tp / rp) / (tl / rl), "ratio_tau_and_rate_only": (tp / rp) / (tl / rl)}


def roofline(ms, launches, flops, fp64_phases, path):
    """The phase with the largest share of the timed sweeps among those with an algorithmic
    flop count: its flops over the timed region / its summed live launch time."""
    timed = {k: v for k, v in ms.items() if k in flops and flops[k] > 0}
    dom = max(timed, key=lambda k: timed[k])
    achieved = flops[dom] / (ms[dom] / 1e3)
    peak = PEAK["fp64"] if dom in fp64_phases else PEAK["fp32"]
    traffic = None
    if TRAFFIC["src"] is not None and TRAFFIC["src"] == kernel_source_digest():
        traffic = TRAFFIC["bytes_per_launch"].get(path, {}).get(dom)
    return {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic, "traffic_unit": "HBM bytes per launch",
            "launches": launches[dom], "avg_launch_ms": ms[dom] / launches[dom]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chains", type=int, default=1024)
    ap.add_argument("--L", type=int, default=16)
    ap.add_argument("--D", type=int, default=8)
    ap.add_argument("--Dc", type=int, default=16)
    ap.add_argument("--train-sweeps", type=int, default=2)
    ap.add_argument("--train-epochs", type=int, default=4)
    ap.add_argument("--tau-sweeps", type=int, default=0)
    ap.add_argument("--split-dc2", type=int, default=0,
                    help="also time two-cutoff sampling (Dc1 = --Dc, Dc2 = this) on the --L, --D lattice")
    ap.add_argument("--only", choices=["both", "plain", "learned"], default="both")
    ap.add_argument("--compress", choices=["canonical", "variational"], default="canonical",
                    help="boundary truncation: canonical SVD compression or the variational fit (App. B)")
    ap.add_argument("--fit-sweeps", type=int, default=2, help="sweeps of the variational fit")
    ap.add_argument("--corr-chains", type=int, default=512,
                    help="chains of the correlated stand-in workload (0: skip it)")
    ap.add_argument("--corr-L", type=int, default=0, help="lattice of the correlated workload (0: --L)")
    ap.add_argument("--corr-D", type=int, default=0, help="its bond dimension (0: --D)")
    ap.add_argument("--corr-Dc", type=int, default=0, help="its cutoff (0: --Dc)")
    ap.add_argument("--corr-steps", type=int, default=0, help="its timed sweeps (0: --steps)")
    ap.add_argument("--corr-train-sweeps", type=int, default=0,
                    help="its training data: pair sweeps of every chain (0: --train-sweeps)")
    ap.add_argument("--corr-train-epochs", type=int, default=0, help="its training epochs (0: --train-epochs)")
    ap.add_argument("--corr-burn", type=int, default=20,
                    help="untimed sweeps from the chain starts before the correlated workload's timed region")
    ap.add_argument("--also-fit", type=int, default=2,
                    help="with the canonical compression, also time both paths with the variational fit of "
                         "this many sweeps for min(steps, 5) steps (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device three times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(chains shard across GPUs with no communication inside a sweep)", file=sys.stderr)
        sys.exit(2)

    # the oracle's processes start before anything in this process touches the GPU
    cpu = None
    if not args.no_cpu_baseline and not args.copy_probe:
        cpu = cpu_baseline(args.L, args.L, args.D, args.Dc, seed=1908)
        print(f"cpu baseline: {cpu['value']:.3f} samples/s on {cpu['cores']} cores", file=sys.stderr, flush=True)

    import torch
    if args.copy_probe:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 8, "copies": 3}), flush=True)
        return
    from paper_1908_09359_amd import binding as B

    Ly = Lx = args.L
    D, Dc, nch = args.D, args.Dc, args.chains
    cm = B.VP_COMPRESS_VARIATIONAL if args.compress == "variational" else B.VP_COMPRESS_CANONICAL
    fs = args.fit_sweeps if args.compress == "variational" else 0
    trunc = dict(compress=cm, fit_sweeps=fs)
    res = {}
    if args.only in ("both", "plain"):
        p = Path(B, torch, Ly, Lx, D, Dc, B.VP_FP32, nch, **trunc)
        r = p.timed(args.warmup, args.steps)
        print(f"plain: {r['samples_per_s']:.1f} samples/s", file=sys.stderr, flush=True)
        fl = phase_flops(Ly, Lx, D, Dc, nch, r["launches"], r["anti_h"], r["anti_v"],
                         fs if cm == B.VP_COMPRESS_VARIATIONAL else None)
        # the canonical compression runs in float64 in every precision, the fit in the working one
        r["roofline"] = roofline(r["ms"], r["launches"], fl,
                                 ("compress_up", "compress_down") if cm == B.VP_COMPRESS_CANONICAL else (), "plain")
        r["stats"] = p.series_stats()
        r["fp64_reference"] = fp64_reference(B, torch, Ly, Lx, D, Dc, p.last_spins, p.el, nch, **trunc)
        print(f"plain: E/N bias against float64 {r['fp64_reference']['bias_e_site']:.3e} "
              f"(mean |dE|/N {r['fp64_reference']['mean_abs_e_site']:.3e})", file=sys.stderr, flush=True)
        if args.tau_sweeps:
            r["tau"] = p.tau_run(args.tau_sweeps)
        p.close()
        del p
        torch.cuda.empty_cache()
        res["plain"] = r
    if args.only in ("both", "learned"):
        p = Path(B, torch, Ly, Lx, D, Dc, B.VP_BF16, nch, **trunc)
        tr = p.train_proposal(args.train_sweeps, args.train_epochs, 256, 3e-3)
        print(f"learned: trained in {tr['seconds']:.1f} s", file=sys.stderr, flush=True)
        r = p.timed(args.warmup, args.steps)
        print(f"learned: {r['samples_per_s']:.1f} samples/s", file=sys.stderr, flush=True)
        r["training"] = tr
        fl = phase_flops(Ly, Lx, D, Dc, nch, r["launches"], r["anti_h"], r["anti_v"],
                         fs if cm == B.VP_COMPRESS_VARIATIONAL else None)
        r["roofline"] = roofline(r["ms"], r["launches"], fl, ("compress_up", "compress_down", "measure3", "measure4"),
                                 "learned")
        r["stats"] = p.series_stats()
        r["fp64_reference"] = fp64_reference(B, torch, Ly, Lx, D, Dc, p.last_spins, p.el, nch, **trunc)
        r["bf16_sampling"] = bf16_decisions(B, torch, Ly, Lx, D, Dc, p.last_spins[:min(64, nch)], **trunc)
        print(f"learned: bf16 ratios rel err median {r['bf16_sampling']['vertical_rel_err_median']:.3e}, decisions differing "
              f"{r['bf16_sampling']['decisions_differing_per_proposal']:.4f}", file=sys.stderr, flush=True)
        if args.tau_sweeps:
            r["tau"] = p.tau_run(args.tau_sweeps)
        p.close()
        res["learned"] = r

    head = res.get("learned") or res["plain"]
    is_learned = "learned" in res
    out = {
        "metric": METRIC, "value": head["samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16/f64" if is_learned else "f32", "data": "synthetic",
        "config": {"workload": f"{Ly}x{Lx} Heisenberg D={D} Dc={Dc}, {nch} chains, "
                               + ("learned plaquette moves + pair sweeps, bf16-operand 2-row steps in the "
                                  "sampling pass, "
                                  "fp64 measurement" if is_learned else "plain pair sweeps, fp32 contractions")
                               + (" / fp64 canonical compression" if cm == B.VP_COMPRESS_CANONICAL else
                                  f" / variational boundary fit, {fs} sweeps"),
                   "Ly": Ly, "Lx": Lx, "D": D, "Dc": Dc, "chains": nch, "J2": 0.0, "compress": args.compress,
                   "parallelism": "chains (1 GPU)"},
        "roofline": head["roofline"],
        "phase_ms_per_step": {k: v / args.steps for k, v in head["ms"].items()},
    }
    for name, r in res.items():
        out[name] = {k: v for k, v in r.items() if k not in ("ms", "launches", "roofline", "anti_h", "anti_v")}
        out[name]["phase_ms_per_step"] = {k: v / args.steps for k, v in r["ms"].items()}
        out[name]["dominant_kernel"] = r["roofline"]
    if "plain" in res:
        out["plain_bias_e_site"] = res["plain"]["fp64_reference"]["bias_e_site"]
    if "learned" in res:
        # median relative error of the bf16-operand ratios (the 2-row steps: vertical bonds)
        out["bf16_ratio_err"] = res["learned"]["bf16_sampling"]["vertical_rel_err_median"]
    if "plain" in res and "learned" in res:
        out["learned_over_plain_raw"] = res["learned"]["samples_per_s"] / res["plain"]["samples_per_s"]
        out["fixed_dE"] = fixed_de(res["plain"], res["learned"])
        out["learned_over_plain_at_fixed_dE"] = out["fixed_dE"]["ratio"]
        if args.tau_sweeps:
            # time to a fixed standard error dE of E/site ~ var * 2 tau / (dE^2 * rate).  Both paths
            # sample |Psi|^2 of the same tensors, so var is the same in expectation; its sample
            # estimates are heavy-tailed (E_loc diverges near nodes of Psi) and are left out of
            # the ratio, which keeps tau_int and the rate only.
            def cost(t):
                return 2.0 * t["tau_int_mean"] / t["samples_per_s"]
            out["learned_over_plain_at_fixed_dE_long_run"] = cost(res["plain"]["tau"]) / cost(res["learned"]["tau"])
    cL, cD, cDc = args.corr_L or Ly, args.corr_D or D, args.corr_Dc or Dc
    c_steps = args.corr_steps or args.steps
    c_tsw, c_tep = args.corr_train_sweeps or args.train_sweeps, args.corr_train_epochs or args.train_epochs
    if args.corr_chains and args.compress == "canonical" and args.only == "both" and c_steps >= 2:
        Tc, info = correlated_tensors(B, torch, cL, cD)
        info.update({"L": cL, "D": cD, "Dc": cDc, "timed_sweeps": c_steps})
        print(f"correlated workload: simple update, lambda change {info['su_change_first']:.2e} -> "
              f"{info['su_change_last']:.2e} in {info['seconds']:.1f} s", file=sys.stderr, flush=True)
        cres = {}
        nc = args.corr_chains
        for name, prec in (("plain", B.VP_FP32), ("learned", B.VP_BF16)):
            p = Path(B, torch, cL, cL, cD, cDc, prec, nc, T=Tc)
            # equilibrate from the random starts before anything is trained or timed
            for _ in range(args.corr_burn):
                p.sweep()
            tr = None
            if name == "learned":
                tr = p.train_proposal(c_tsw, c_tep, 256, 3e-3)
                print(f"correlated learned: trained on {tr['configs']} configurations, loss {tr['loss_first_epoch']:.4f}"
                      f" -> {tr['loss_last_epoch']:.4f} in {tr['seconds']:.1f} s", file=sys.stderr, flush=True)
            r = p.timed(args.warmup, c_steps)
            r["stats"] = p.series_stats()
            r["fp64_reference"] = fp64_reference(B, torch, cL, cL, cD, cDc, p.last_spins, p.el, nc, T=Tc)
            if tr is not None:
                r["training"] = tr
            print(f"correlated {name}: {r['samples_per_s']:.1f} samples/s, tau_int(E) "
                  f"{r['stats']['e_site']['tau_int_mean']:.3f}, tau_int(Mz^2) {r['stats']['mz2']['tau_int_mean']:.3f}, "
                  f"E/N {r['stats']['e_site']['mean']:.5f} +- {r['stats']['e_site']['stderr']:.5f}",
                  file=sys.stderr, flush=True)
            cres[name] = {k: r[k] for k in ("samples_per_s", "ms_per_step", "seconds", "pair_accept",
                                             "plaquette_accept", "plaquette_proposed_per_sweep", "stats",
                                             "fp64_reference", "training") if k in r}
            p.close()
            del p
            torch.cuda.empty_cache()
        fd = fixed_de(cres["plain"], cres["learned"])
        ep, el_ = cres["plain"]["stats"]["e_site"], cres["learned"]["stats"]["e_site"]
        out["correlated"] = {"workload": info, "chains": nc, **cres, "fixed_dE": fd,
                             "learned_over_plain_at_fixed_dE": fd["ratio"],
                             "energies_agree_sigma": abs(ep["mean"] - el_["mean"]) /
                             max((ep["stderr"] ** 2 + el_["stderr"] ** 2) ** 0.5, 1e-300)}
        del Tc
        torch.cuda.empty_cache()
    if args.also_fit and args.compress == "canonical":
        fit = {}
        ft = dict(compress=B.VP_COMPRESS_VARIATIONAL, fit_sweeps=args.also_fit)
        fsteps = min(args.steps, 5)
        for name, prec in (("plain", B.VP_FP32), ("learned", B.VP_BF16)):
            if args.only not in ("both", name):
                continue
            p = Path(B, torch, Ly, Lx, D, Dc, prec, nch, **ft)
            if name == "learned":
                p.train_proposal(args.train_sweeps, args.train_epochs, 256, 3e-3)
            r = p.timed(min(args.warmup, 2), fsteps)
            fit[name] = {"samples_per_s": r["samples_per_s"], "ms_per_step": r["ms_per_step"], "steps": fsteps,
                         "phase_ms_per_step": {k: v / fsteps for k, v in r["ms"].items()}}
            print(f"{name} with the variational fit ({args.also_fit} sweeps): {r['samples_per_s']:.1f} samples/s",
                  file=sys.stderr, flush=True)
            p.close()
            del p
            torch.cuda.empty_cache()
        out["variational_fit"] = dict(fit_sweeps=args.also_fit, **fit)
    if args.split_dc2:
        out["split_cutoffs"] = split_run(B, torch, Ly, Lx, D, Dc, args.split_dc2, nch, args.warmup, args.steps)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
