"""FP32 fields through the continuation schedule, single stages at beta = 32
and penal = 3 from identical oracle states, the projection at the benchmark's
full size, and the 3D cantilever trajectory, against the FP64 oracle.

Tolerances (the survey's policy): FP32 fields 1e-4 relative (infinity norm)
on identical inputs, FP64 fields 1e-10; trajectories in FP32 compliance
within 1e-3 and 99% agreement on xphys > 0.5, in FP64 compliance within 1e-6.
FP32 inputs are promoted exactly to FP64 before the oracle sees them."""
import math
from dataclasses import replace

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W
from oracle import oc as ooc
from oracle import projection as oproj
from oracle import sensitivity as osens
from oracle import solve as osolve
from oracle import sparse as osp
from oracle import topopt as otop


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_05436_amd import _lib
    _lib.load()


def rel_inf(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


# the 300 x 100 schedule compressed to steps of 5 iterations on 90 x 30: beta
# reaches 32 at iteration 25, penal 3 at iteration 40
FAST = replace(W.C1[300], nelx=90, nely=30, rmin=3.0,
               penal_sched=(1, 3.0, 5, 0.25, "add"), beta_sched=(1, 32.0, 5, 2.0, "mul"))


@pytest.mark.parametrize("solve", ["auto", "mixed"])
def test_continuation_fp32_schedule(solve):
    """FP32 fields through beta 1 -> 32 and penal 1 -> 2.5 (30 iterations):
    compliance within 1e-3 of the FP64 oracle at every iteration and 99% of
    elements agree on xphys > 0.5 at the end."""
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    its = 30
    prob = otop.problem_from_config(FAST)
    st, log = otop.run(prob, its, solver="pcg")
    sp = L.TO_SOLVE_AUTO if solve == "auto" else L.TO_SOLVE_MIXED
    g = TopOpt(FAST, precision="f32", solve_precision=sp)
    worst = 0.0
    for i in range(its):
        g.step()
        s = g.stats()
        r = abs(s["c"] - log[i]["c"]) / log[i]["c"]
        worst = max(worst, r)
        print(f"it {i + 1:2d} beta {s['beta']:5.1f} penal {s['penal']:4.2f} c {s['c']:.6f} oracle {log[i]['c']:.6f} "
              f"rel {r:.2e} n_bs {s['n_bs']}/{log[i]['n_bs']} newton {s['n_newton']}/{log[i]['n_newton']}", flush=True)
        assert s["solve_ok"]
        assert s["penal"] == log[i]["penal"] and s["beta"] == log[i]["beta"]
        assert r <= 1e-3, (i + 1, s["c"], log[i]["c"])
    agree = np.mean((host(g.xphys) > 0.5) == (st.xphys > 0.5))
    print(f"worst rel {worst:.2e}, agreement {agree:.4f}")
    assert agree >= 0.99


@pytest.fixture(scope="module")
def late_state():
    """The oracle's FP64 state after 45 iterations of the compressed schedule
    (beta = 32, penal = 3)."""
    prob = otop.problem_from_config(FAST)
    st, log = otop.run(prob, 45, solver="pcg")
    assert st.beta == 32.0 and st.penal == 3.0
    return prob, st


def test_single_stages_fp32_beta32_penal3(late_state):
    """Every stage of one redesign iteration in FP32 at beta = 32, penal = 3,
    each fed the oracle's state rounded to FP32 (promoted exactly for the
    oracle): fields within 1e-4, equal Newton and bisection counts, the same
    bisection midpoint (the OC candidates and volume sums are FP64 on both
    sides, so no decision may flip)."""
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Plan, plan_for_config, read_struct
    prob, st = late_state
    P, f, _ = plan_for_config(FAST)
    m, n = P.info.m, P.info.n
    T = torch.float32
    dt = L.TO_F32
    cu = lambda a, t=T: torch.as_tensor(np.asarray(a), dtype=t).cuda()
    act = prob.act
    # forward filter
    x32 = f32(st.x)
    xd = cu(x32)
    xt = torch.zeros(m, dtype=T, device="cuda")
    L.to_filter(P.handle, dt, L.TO_FILTER_FWD, xd, None, None, xt, None)
    xt_ref = prob.filter.forward(x32)
    e_filter = rel_inf(host(xt), xt_ref)
    # projection with the Newton threshold from the oracle's eta
    xt_in = host(xt)
    xphys, dprj = torch.zeros(m, dtype=T, device="cuda"), torch.zeros(m, dtype=T, device="cuda")
    eta = torch.tensor([st.eta], dtype=torch.float64, device="cuda")
    pst = torch.zeros(48, dtype=torch.uint8, device="cuda")
    L.to_project(P.handle, dt, 3, xt, xd, xphys, dprj, 32.0, eta, FAST.volfrac, None, pst)
    ps = read_struct(pst, L.ProjectStats)
    xp_ref, dp_ref, eta_ref, nn_ref, ok = oproj.physical_density(xt_in, x32, act, 3, st.eta, 32.0, FAST.volfrac)
    e_xphys, e_dprj = rel_inf(host(xphys), xp_ref), rel_inf(host(dprj), dp_ref)
    # state solve on the FP32 design
    xp_in = host(xphys)
    kval = torch.zeros(P.info.nnz_lower, dtype=T, device="cuda")
    L.to_assemble(P.handle, dt, xphys, 3.0, kval)
    kl_ref = osp.assemble(xp_in, prob.ke_lower, prob.perm, prob.seg_ptr, 3.0, 1.0, 1e-9)
    e_kval = rel_inf(host(kval), kl_ref)
    K = osp.lower_to_full(prob.row_ptr, prob.col_idx, kl_ref, n)
    u_ref = osolve.solve_dense(K.toarray(), prob.f, prob.free) if n <= 3000 else \
        osolve.solve_pcg(K, prob.f, prob.free, np.zeros(n), 1e-12)[0]
    u = cu(st.u, torch.float64)
    sst = torch.zeros(64, dtype=torch.uint8, device="cuda")
    fd = cu(f, torch.float64)
    L.to_solve(P.handle, dt, kval, xphys, 3.0, fd, u, L.SolveOpts(1e-8, 0.1, 200000, L.TO_OP_ASSEMBLED,
                                                                   L.TO_SOLVE_AUTO, 0, 0, L.TO_PREC_JACOBI), sst)
    ss = read_struct(sst, L.SolveStats)
    u_h = host(u)
    c_ref = float(prob.f @ u_ref)
    e_c = abs(float(prob.f @ u_h) - c_ref) / c_ref
    res = osolve.true_residual(K, prob.f, prob.free, u_h)
    # sensitivity from the oracle's displacement
    dc = torch.zeros(m, dtype=T, device="cuda")
    cdev = torch.zeros(1, dtype=torch.float64, device="cuda")
    ud = cu(u_ref, torch.float64)
    L.to_sensitivity(P.handle, dt, xphys, ud, fd, 3.0, dc, cdev)
    dc_ref, _ = osens.sensitivity(xp_in, u_ref, prob.cmat, prob.ke_full, act, 3.0, 1.0, 1e-9)
    e_dc = rel_inf(host(dc), dc_ref)
    # fused back-filter of dc and dV through dprj
    dc_in, dp_in = host(dc), host(dprj)
    dv = cu(f32(prob.dv))
    dcf, dv0 = torch.zeros(m, dtype=T, device="cuda"), torch.zeros(m, dtype=T, device="cuda")
    L.to_filter(P.handle, dt, L.TO_FILTER_ADJ2, dc, dv, dprj, dcf, dv0)
    dcf_ref = prob.filter.adjoint(dc_in, dp_in)
    dv0_ref = prob.filter.adjoint(f32(prob.dv), dp_in)
    e_dcf, e_dv0 = rel_inf(host(dcf), dcf_ref), rel_inf(host(dv0), dv0_ref)
    # OC on the FP32 fields
    dcf_in, dv0_in = host(dcf), host(dv0)
    ost = torch.zeros(48, dtype=torch.uint8, device="cuda")
    L.to_oc_update(P.handle, dt, xd, dcf, dv0, FAST.volfrac, FAST.move, ost)
    os_ = read_struct(ost, L.OcStats)
    xo_ref, so = ooc.oc_update(x32, dcf_in, dv0_in, act, FAST.volfrac, FAST.move)
    flips = int(os_.n_bs != so["n_bs"]) + int(os_.lmid != so["lmid"])
    e_x = rel_inf(host(xd), xo_ref)
    print(f"beta 32 penal 3, FP32 stages: filter {e_filter:.2e} xphys {e_xphys:.2e} dprj {e_dprj:.2e} "
          f"eta {abs(ps.eta - eta_ref):.2e} newton {ps.n_newton}/{nn_ref} kval {e_kval:.2e} c {e_c:.2e} "
          f"residual {res:.2e} cg {ss.iterations} dc {e_dc:.2e} dcf {e_dcf:.2e} dv0 {e_dv0:.2e} "
          f"oc n_bs {os_.n_bs}/{so['n_bs']} lmid {os_.lmid!r}/{so['lmid']!r} decision flips {flips} x {e_x:.2e}")
    assert e_filter <= 1e-4 and e_xphys <= 1e-4 and e_dprj <= 1e-4
    assert ps.n_newton == nn_ref and abs(ps.eta - eta_ref) <= 1e-6
    assert e_kval <= 1e-6
    assert ss.converged and res <= 1e-8 and e_c <= 1e-7
    assert e_dc <= 1e-4 and e_dcf <= 1e-4 and e_dv0 <= 1e-4
    assert flips == 0
    assert e_x <= 1e-7


@pytest.mark.parametrize("dt", [1, 0])
@pytest.mark.parametrize("beta", [1.0, 32.0])
def test_project_full_size(dt, beta):
    """The projection with its Newton threshold at 1200 x 400 in the launch
    shape the benchmark uses (ft = 3, target volfrac), element by element
    against the oracle on the same (promoted) filtered field."""
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import plan_for_config, read_struct
    cfg = W.C1[1200]
    P, _, _ = plan_for_config(cfg)
    m = P.info.m
    T = torch.float64 if dt == 1 else torch.float32
    xt_h = W.smooth_design(cfg, 21)
    xt = torch.as_tensor(xt_h, dtype=T).cuda()
    x = torch.as_tensor(W.design_field(m, 22), dtype=T).cuda()
    xold = torch.as_tensor(W.design_field(m, 23), dtype=T).cuda()
    xphys, dprj = torch.zeros(m, dtype=T, device="cuda"), torch.zeros(m, dtype=T, device="cuda")
    eta0 = 0.47
    eta = torch.tensor([eta0], dtype=torch.float64, device="cuda")
    pst = torch.zeros(48, dtype=torch.uint8, device="cuda")
    L.to_project(P.handle, dt, 3, xt, x, xphys, dprj, beta, eta, cfg.volfrac, xold, pst)
    s = read_struct(pst, L.ProjectStats)
    xt_in, x_in, xo_in = host(xt), host(x), host(xold)
    act = np.ones(m, bool)
    xp, dp, eta_o, nn, ok = oproj.physical_density(xt_in, x_in, act, 3, eta0, beta, cfg.volfrac)
    tol = 1e-10 if dt == 1 else 1e-4
    print(f"1200x400 dt {dt} beta {beta}: newton {s.n_newton}/{nn} eta {s.eta!r}/{eta_o!r} "
          f"xphys {rel_inf(host(xphys), xp):.2e} dprj {rel_inf(host(dprj), dp):.2e}")
    assert ok and s.converged == 1 and s.n_newton == nn
    assert abs(s.eta - eta_o) <= (1e-12 if dt == 1 else 1e-6)
    assert rel_inf(host(xphys), xp) <= tol
    assert rel_inf(host(dprj), dp) <= tol
    assert abs(s.ch - oproj.change(host(xphys), xo_in)) <= 1e-12
    assert abs(s.vol - np.mean(xp)) <= 1e-9


@pytest.mark.parametrize("mode", ["f64", "f32-mixed"])
def test_cantilever3d_trajectory(mode):
    """The 3D cantilever (Sec. 4: clamped face, sine line load, 'N' filter,
    ft = 3, beta = 2) on 12 x 6 x 6 for 10 redesign iterations against the
    oracle, iteration by iteration: FP64 compliance within 1e-6, threshold
    within 1e-7, equal Newton and bisection counts, design within 1e-4 at
    the end; FP32 fields with the mixed-precision solve: compliance within
    1e-3 and 99% agreement on xphys > 0.5."""
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    cfg = W.C2_SMALL
    prob = otop.problem_from_config(cfg)
    st, log = otop.run(prob, cfg.iterations, solver="dense")
    if mode == "f64":
        g = TopOpt(cfg, precision="f64")
    else:
        g = TopOpt(cfg, precision="f32", solve_precision=L.TO_SOLVE_MIXED, op=L.TO_OP_MATFREE)
    for i in range(cfg.iterations):
        g.step()
        s = g.stats()
        r = abs(s["c"] - log[i]["c"]) / log[i]["c"]
        print(f"3D {mode} it {i + 1} c {s['c']:.8f} oracle {log[i]['c']:.8f} rel {r:.2e} "
              f"n_bs {s['n_bs']}/{log[i]['n_bs']} newton {s['n_newton']}/{log[i]['n_newton']}", flush=True)
        assert s["solve_ok"]
        if mode == "f64":
            assert r <= 1e-6
            assert abs(s["eta"] - log[i]["eta"]) <= 1e-7
            assert s["n_bs"] == log[i]["n_bs"] and s["n_newton"] == log[i]["n_newton"]
        else:
            assert r <= 1e-3
    if mode == "f64":
        assert np.abs(host(g.xphys) - st.xphys).max() <= 1e-4
    else:
        assert np.mean((host(g.xphys) > 0.5) == (st.xphys > 0.5)) >= 0.99
