"""GPU tests of ragged batches (one persistent launch per stage for the whole
batch, per-iteration HIP graphs) and of the launch-shape autotuner.

A batch runs the same kernels as single designs but with per-design block
groups of other sizes, so reductions sum in another order: designs agree
with their single runs to rounding (the CG stopping point moves by rounding,
so compliance within 1e-7 and designs within 1e-6), and with the FP64 oracle
at the trajectory tolerance.  Graph replays run the captured launches with
the same arguments and agree with eager batched steps bit for bit.  Every
autotuner shape reproduces the oracle filter (1e-10 / 1e-4) and the assembly
bit for bit (each slot's sum has a fixed order)."""
from dataclasses import replace

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W
from oracle import filt as ofilt
from oracle import mesh as omesh
from oracle import sparse as osp
from oracle import element as oel
from oracle import topopt as otop


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_05436_amd import _lib
    _lib.load()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def ragged(precision="f64", beta=2.0):
    """Six designs of different sizes and both load cases, projection on."""
    out = []
    for i, (nx, ny, kind, load) in enumerate([(40, 20, "mbb", 7), (64, 32, "cantilever2d", 20), (30, 10, "mbb", 0),
                                              (50, 25, "cantilever2d", 3), (72, 24, "mbb", 40), (20, 16, "mbb", 19)]):
        out.append(W.Config(f"r{i}", kind, nx, ny, volfrac=0.3 + 0.03 * i, rmin=1.5 + 0.4 * i, ft=3, bc="D",
                            beta=beta, penal=3.0, iterations=10, precision=precision, load=load))
    return out


def test_batch_matches_single_runs():
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Batch, TopOpt
    cfgs = ragged()
    b = Batch(cfgs, autotune=False)
    singles = [TopOpt(c) for c in cfgs]
    info = b.info()
    assert info["designs"] == len(cfgs) and info["solve_blocks"] >= len(cfgs)
    for k in range(6):
        b.step()
        for g in singles:
            g.step()
        for gb, gs in zip(b.runs, singles):
            cb, cs = float(host(gb.c)[0]), float(host(gs.c)[0])
            assert abs(cb - cs) <= 1e-7 * abs(cs), (gb.cfg.name, k, cb, cs)
            assert np.abs(host(gb.x) - host(gs.x)).max() <= 1e-6
            sb = gb.stats()
            assert sb["solve_ok"] and sb["newton_ok"]
            assert gb.state.loop == gs.state.loop == k + 1


def test_batch_design_matches_oracle_trajectory():
    from paper_2005_05436_amd.driver import Batch
    cfgs = ragged()
    b = Batch(cfgs, autotune=True)
    refs = [otop.problem_from_config(c) for c in cfgs[:3]]
    states = [otop.State(p) for p in refs]
    for k in range(5):
        b.step()
        logs = [otop.step(p, st) for p, st in zip(refs, states)]
        for g, st, lg in zip(b.runs[:3], states, logs):
            c = float(host(g.c)[0])
            assert abs(c - lg["c"]) <= 1e-6 * abs(lg["c"]), (g.cfg.name, k, c, lg["c"])
            assert np.abs(host(g.xphys) - st.xphys).max() <= 1e-4


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_graph_replays_match_eager(precision):
    from paper_2005_05436_amd.driver import Batch
    cfgs = ragged(precision)
    be = Batch(cfgs, autotune=False)
    bg = Batch(cfgs, autotune=False)
    for k in range(4):
        be.step()
        bg.step(use_graph=True)
        torch.cuda.synchronize()
        junk = float(torch.ones(4096, device="cuda").sum().item())     # eager work between replays
        assert junk == 4096.0
        for ge, gg in zip(be.runs, bg.runs):
            np.testing.assert_array_equal(host(ge.x), host(gg.x))
            np.testing.assert_array_equal(host(ge.u), host(gg.u))
            assert float(host(ge.c)[0]) == float(host(gg.c)[0])
    info = bg.info()
    assert info["graph_captures"] == 1 and info["graph_launches"] == 4


def test_batch_graph_recaptures_on_continuation():
    from paper_2005_05436_amd.driver import Batch
    cfgs = [replace(c, beta=1.0, beta_sched=(1, 32.0, 2, 2.0, "mul")) for c in ragged()[:3]]
    be = Batch(cfgs, autotune=False)
    bg = Batch(cfgs, autotune=False)
    for k in range(5):
        be.step()
        bg.step(use_graph=True)
        for ge, gg in zip(be.runs, bg.runs):
            np.testing.assert_array_equal(host(ge.x), host(gg.x))
            assert ge.state.beta == gg.state.beta
    assert bg.runs[0].state.beta == 4.0
    assert bg.info()["graph_captures"] == 3      # beta 1, 2, 4


@pytest.mark.parametrize("dims,rmin,dt", [((120, 40), 4.0, 1), ((300, 100), 10.0, 0), ((61, 33), 2.5, 1)])
def test_autotune_shapes_reproduce_oracle(dims, rmin, dt):
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Plan
    P = Plan(2, dims[0], dims[1], 1, rmin, "D")
    I = P.info
    T = torch.float64 if dt == L.TO_F64 else torch.float32
    tol = 1e-10 if dt == L.TO_F64 else 1e-4
    M = omesh.Mesh(*dims)
    F = ofilt.Filter(M, rmin, "D")
    x = W.design_field(I.m, 3, 0.0, 1.0)
    g1 = W.design_field(I.m, 4, -1.0, 0.0)
    g2 = W.design_field(I.m, 5, 0.0, 1.0)
    s = W.design_field(I.m, 6, 0.5, 1.5)
    if dt == L.TO_F32:
        x, g1, g2, s = (a.astype(np.float32).astype(np.float64) for a in (x, g1, g2, s))
    ref_f = F.forward(x)
    ref_a1, ref_a2 = F.adjoint(g1, s), F.adjoint(g2, s)
    kval = torch.zeros(I.nnz_lower, dtype=T, device="cuda")
    t = L.to_plan_autotune(P.handle, dt, kval)
    assert t.tuned == 1 and t.filt_v in (4, 8) and t.asm_block in (128, 256, 512)
    kvals = []
    for v, parts, nt in [(8, 0, 256), (8, 8, 128), (4, 0, 512), (4, 4, 256), (t.filt_v, t.filt_parts, t.asm_block)]:
        L.to_plan_set_tuning(P.handle, v, parts, nt, 1)
        xd = torch.as_tensor(x, dtype=T).cuda()
        out = torch.zeros_like(xd)
        L.to_filter(P.handle, dt, L.TO_FILTER_FWD, xd, None, None, out, None)
        o1, o2 = torch.zeros_like(xd), torch.zeros_like(xd)
        L.to_filter(P.handle, dt, L.TO_FILTER_ADJ2, torch.as_tensor(g1, dtype=T).cuda(),
                    torch.as_tensor(g2, dtype=T).cuda(), torch.as_tensor(s, dtype=T).cuda(), o1, o2)
        for got, ref in ((out, ref_f), (o1, ref_a1), (o2, ref_a2)):
            g = host(got)
            assert np.abs(g - ref).max() <= tol * np.abs(ref).max(), (v, parts)
        L.to_assemble(P.handle, dt, xd, 3.0, kval)
        kvals.append(host(kval))
    for k in kvals[1:]:
        np.testing.assert_array_equal(k, kvals[0])


def test_batch64_ragged_configuration():
    """The 64-design ragged batch (nelx 100..400, nely = nelx / 2, both load
    cases, FP32 fields) for two graph-replayed iterations: every solve and
    Newton converges, every volume holds, and three sampled designs agree
    with their single runs."""
    from paper_2005_05436_amd.driver import Batch, TopOpt
    cfgs = W.batch_configs(64, 0)
    b = Batch(cfgs, autotune=True)
    for k in range(2):
        b.step(use_graph=True)
    torch.cuda.synchronize()
    for g in b.runs:
        s = g.stats()
        assert s["solve_ok"] and s["newton_ok"] and s["residual"] <= 1e-8, g.cfg.name
        assert abs(s["vol"] - g.cfg.volfrac) <= 1e-5, g.cfg.name
    for i in (0, 31, 63):
        gs = TopOpt(cfgs[i])
        gs.step()
        gs.step()
        cb, cs = float(host(b.runs[i].c)[0]), float(host(gs.c)[0])
        assert abs(cb - cs) <= 1e-5 * abs(cs), (i, cb, cs)


def _stage_check(b, x_before, penal):
    """Every stage a batched iteration ran through its batch-wide launches
    equals the single-design entry point on the same inputs: the stencil
    passes and the moduli / assembly / sensitivity fields bit for bit (same
    arithmetic per output), the compliance sum to rounding (another block
    split)."""
    from paper_2005_05436_amd import _lib as L
    for g, x0 in zip(b.runs, x_before):
        P, dt = g.plan.handle, g.dtype
        xt = torch.zeros_like(g.xtilde)
        L.to_filter(P, dt, L.TO_FILTER_FWD, x0, None, None, xt, None)
        np.testing.assert_array_equal(host(xt), host(g.xtilde), err_msg=g.cfg.name)
        kv = torch.zeros_like(g.kval)
        L.to_assemble(P, dt, g.xphys, penal, kv)
        np.testing.assert_array_equal(host(kv), host(g.kval), err_msg=g.cfg.name)
        dc = torch.zeros_like(g.dc)
        c = torch.zeros(1, dtype=torch.float64, device="cuda")
        L.to_sensitivity(P, dt, g.xphys, g.u, g.f, penal, dc, c)
        np.testing.assert_array_equal(host(dc), host(g.dc), err_msg=g.cfg.name)
        cs, cb = float(host(c)[0]), float(host(g.c)[0])
        assert abs(cs - cb) <= 1e-13 * abs(cs), (g.cfg.name, cs, cb)
        o1, o2 = torch.zeros_like(g.dcf), torch.zeros_like(g.dv0)
        L.to_filter(P, dt, L.TO_FILTER_ADJ2, g.dc, g.dv, g.dprj, o1, o2)
        np.testing.assert_array_equal(host(o1), host(g.dcf), err_msg=g.cfg.name)
        np.testing.assert_array_equal(host(o2), host(g.dv0), err_msg=g.cfg.name)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_stage_launches_match_single_entry_points(precision):
    """2D: the filter passes, moduli, assembly and sensitivities are one
    launch each for the whole batch; each design's outputs equal the
    single-design calls (eager and graph-replayed steps)."""
    from paper_2005_05436_amd.driver import Batch
    cfgs = ragged(precision)
    b = Batch(cfgs, autotune=False)
    info = b.info()
    assert info["filter_batched"] and info["element_blocks"] >= len(cfgs)
    for k in range(3):
        x_before = [g.x.clone() for g in b.runs]
        b.step(use_graph=(k > 0))
        torch.cuda.synchronize()
        _stage_check(b, x_before, 3.0)


def test_batch_3d_designs():
    """3D designs: per-design filter and assembly launches, batch-wide moduli
    and sensitivities; stages equal the single-design calls, and the designs
    follow their single runs to rounding."""
    from paper_2005_05436_amd.driver import Batch, TopOpt
    cfgs = [replace(W.C2_SMALL, name=f"b3_{i}", nelx=nx, nely=ny, nelz=nz, load=ld, rmin=rm)
            for i, (nx, ny, nz, ld, rm) in enumerate([(12, 6, 6, 0, 1.5), (16, 8, 4, 2, 2.0), (10, 6, 8, 5, 1.8)])]
    b = Batch(cfgs, autotune=False)
    assert not b.info()["filter_batched"]
    singles = [TopOpt(c) for c in cfgs]
    for k in range(3):
        x_before = [g.x.clone() for g in b.runs]
        b.step()
        for g in singles:
            g.step()
        torch.cuda.synchronize()
        _stage_check(b, x_before, 3.0)
        for gb, gs in zip(b.runs, singles):
            cb, cs = float(host(gb.c)[0]), float(host(gs.c)[0])
            assert abs(cb - cs) <= 1e-7 * abs(cs), (gb.cfg.name, k, cb, cs)
            assert np.abs(host(gb.x) - host(gs.x)).max() <= 1e-6
