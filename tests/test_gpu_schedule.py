"""Launch schedules and uneven batches on the GPU.

* the per-phase, persistent (work-queue) and graph-replay schedules give
  bit-identical float64 chains, measurements and move counts, over several
  vp_sample calls with eager work in between (every graph is replayed many
  times per call);
* one persistent launch over lattices of different sizes and couplings
  reproduces, lattice by lattice, the oracle's chains bit-exactly;
* the autotuner picks one of the schedules and leaves the sampler correct.
"""
import numpy as np
import pytest

from oracle import lattice as olat
from oracle import vmc
from paper_1908_09359_amd import workloads as W

pytestmark = pytest.mark.gpu


def _B():
    from paper_1908_09359_amd import binding as B
    return B


def _bufs(n, m, N, npar, dt):
    import torch
    dev = torch.device("cuda")
    return dict(log_abs_psi=torch.empty(n * m, dtype=torch.float64, device=dev),
                sign=torch.empty(n * m, dtype=torch.int8, device=dev),
                e_loc=torch.empty(n * m, dtype=torch.float64, device=dev),
                dlnpsi=torch.empty((n * m, npar // 2), dtype=dt, device=dev),
                spins_out=torch.empty((n * m, N), dtype=torch.int8, device=dev))


def _run(schedule, Ly, Lx, D, Dc, J2, n, T, seed, calls, learned=None, prec=None):
    import torch
    B = _B()
    ctx = B.Context(B.lattice(Ly, Lx, D, Dc, 1.0, J2, B.VP_FP64 if prec is None else prec, n), seed=seed)
    dev = torch.device("cuda")
    ctx.vp_set_tensors(0, torch.tensor(T, dtype=torch.float64, device=dev))
    ctx.vp_init_chains(0, None)
    if learned is not None:
        ctx.vp_proposal_set_weights(0, torch.tensor(learned, device=dev))
        ctx.vp_set_sampler(0, B.VP_SAMPLER_LEARNED_PLAQ)
    ctx.vp_set_schedule(0, schedule)
    outs = []
    for (nb, nm) in calls:
        b = _bufs(n, nm, Ly * Lx, ctx.num_params(), torch.float64)
        ctx.vp_sample(0, nb, nm, b["log_abs_psi"], b["sign"], b["e_loc"], b["dlnpsi"], b["spins_out"])
        # eager work between the calls (and between graph replays of consecutive calls)
        junk = torch.randn(1000, device=dev).sum()
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in b.items()})
        del junk
    cnt = torch.empty((n, 4), dtype=torch.int64, device=dev)
    ctx.vp_move_counts(0, cnt)
    ctx.vp_sync()
    c = cnt.cpu().numpy()
    ctx.close()
    return outs, c


FAULTED = ("a GPU memory fault was reported in this case once, on a build whose compression kernels also "
           "held the variational fit; the fit has since moved to a kernel of its own, but the fault's cause was "
           "not shown, so the case stays off the GPU until it is")


@pytest.mark.parametrize("Ly,Lx,D,Dc,J2,learn", [pytest.param(4, 4, 2, 4, 0.0, False, marks=pytest.mark.skip(reason=FAULTED)),
                                                 (6, 6, 4, 8, 0.5, False),
                                                 (4, 6, 3, 4, 0.0, True), (4, 6, 8, 16, 0.0, True)])
def test_schedules_agree_bit_exactly(Ly, Lx, D, Dc, J2, learn):
    B = _B()
    print(f"schedules {Ly}x{Lx} D={D} Dc={Dc} J2={J2} learned={learn}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=90 + D)
    th = W.random_proposal_weights(seed=91, scale=0.3, bias=0.5) if learn else None
    calls = [(1, 3), (0, 2), (2, 2)]
    ref, rc = _run(B.VP_SCHED_PHASES, Ly, Lx, D, Dc, J2, 5, T, 17, calls, th)
    for sch in (B.VP_SCHED_PERSISTENT, B.VP_SCHED_GRAPH):
        got, gc = _run(sch, Ly, Lx, D, Dc, J2, 5, T, 17, calls, th)
        for a, b in zip(ref, got):
            for k in a:
                assert np.array_equal(a[k], b[k]), (sch, k)
        assert np.array_equal(rc, gc), sch
    if learn:
        assert rc[:, 3].sum() > 0


def test_schedules_agree_bit_exactly_bf16_learned():
    """The bf16 sampling mode with learned moves (bf16 2-row steps, bf16 inference of
    the proposal network): phases, persistent queue and graph replay agree bit for bit."""
    B = _B()
    Ly, Lx, D, Dc = 4, 6, 8, 16
    print(f"schedules bf16 learned {Ly}x{Lx} D={D} Dc={Dc}", flush=True)
    T = W.random_tensors(Ly, Lx, D, seed=98)
    th = W.random_proposal_weights(seed=91, scale=0.3, bias=0.5)
    calls = [(1, 3), (0, 2), (2, 2)]
    ref, rc = _run(B.VP_SCHED_PHASES, Ly, Lx, D, Dc, 0.0, 5, T, 17, calls, th, B.VP_BF16)
    for sch in (B.VP_SCHED_PERSISTENT, B.VP_SCHED_GRAPH):
        got, gc = _run(sch, Ly, Lx, D, Dc, 0.0, 5, T, 17, calls, th, B.VP_BF16)
        for a, b in zip(ref, got):
            for k in a:
                assert np.array_equal(a[k], b[k]), (sch, k)
        assert np.array_equal(rc, gc), sch
    assert rc[:, 3].sum() > 0 and rc[:, 2].sum() > 0


def test_uneven_batch_matches_oracle():
    """Three lattices of different sizes and couplings in one persistent launch per sweep."""
    import torch
    B = _B()
    shapes = [(4, 4, 0.0, 3), (6, 4, 0.5, 2), (4, 6, 0.0, 2)]
    D, Dc, seed, nb, nm = 2, 4, 23, 1, 2
    print("uneven batch 4x4 + 6x4 (J2=0.5) + 4x6, D=2 Dc=4", flush=True)
    lats = [B.lattice(Ly, Lx, D, Dc, 1.0, J2, B.VP_FP64, n) for (Ly, Lx, J2, n) in shapes]
    ctx = B.Context(lats, seed=seed)
    dev = torch.device("cuda")
    Ts, outs = [], []
    for i, (Ly, Lx, J2, n) in enumerate(shapes):
        T = W.random_tensors(Ly, Lx, D, seed=100 + i)
        Ts.append(T)
        ctx.vp_set_tensors(i, torch.tensor(T, dtype=torch.float64, device=dev))
        ctx.vp_init_chains(i, None)
        outs.append(_bufs(n, nm, Ly * Lx, ctx.num_params(i), torch.float64))
    ctx.vp_sample_batch([0, 1, 2], nb, nm, outs)
    ctx.vp_sync()
    for i, (Ly, Lx, J2, n) in enumerate(shapes):
        lat = olat.Lattice(Ly, Lx, D, Dc, J2=J2)
        sp = outs[i]["spins_out"].cpu().numpy().reshape(n, nm, Ly * Lx)
        el = outs[i]["e_loc"].cpu().numpy().reshape(n, nm)
        lp = outs[i]["log_abs_psi"].cpu().numpy().reshape(n, nm)
        for c in range(n):
            ch = vmc.Chain(lat, olat.neel_shuffled(lat, seed, i, c), seed, i, c)
            o = vmc.run_chain(Ts[i], lat, ch, nb, nm)
            assert np.array_equal(sp[c], np.stack([x["spins"] for x in o])), (i, c)
            assert np.max(np.abs(el[c] - np.array([x["e_loc"] for x in o]))) / (Ly * Lx) <= 1e-10, (i, c)
            assert np.max(np.abs(lp[c] - np.array([x["log_abs_psi"] for x in o]))) <= 1e-10, (i, c)
    ctx.close()


def test_autotune_picks_a_schedule():
    import torch
    B = _B()
    print("autotune 6x6 D=4 Dc=8 fp32 64 chains", flush=True)
    ctx = B.Context(B.lattice(6, 6, 4, 8, 1.0, 0.0, B.VP_FP32, 64), seed=5)
    ctx.vp_init_tensors(0, seed=6, scale=0.0, perturb=0.0)
    ctx.vp_init_chains(0, None)
    pick, ms = ctx.vp_autotune(0, 2)
    print(f"autotune: pick {pick}, ms/sweep {ms}", flush=True)
    assert pick in (B.VP_SCHED_PHASES, B.VP_SCHED_PERSISTENT, B.VP_SCHED_GRAPH)
    assert all(m > 0 for m in ms) and ms[pick] == min(ms)
    b = _bufs(64, 1, 36, ctx.num_params(), torch.float32)
    ctx.vp_sample(0, 0, 1, b["log_abs_psi"], b["sign"], b["e_loc"], b["dlnpsi"], b["spins_out"])
    ctx.vp_sync()
    assert np.all(np.isfinite(b["e_loc"].cpu().numpy()))
    ctx.close()
