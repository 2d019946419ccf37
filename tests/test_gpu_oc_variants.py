"""GPU tests of the OC variants against the FP64 oracle: the explicit
primal-dual update (Appendix A) and the bisection that filters and projects
every candidate (Sec. 3.2).

Primal-dual: the GPU sums the three sets in double-double, so the
multiplier agrees with the oracle's exactly rounded sums to 1e-12 and the
designs to 1e-12 (FP32: inputs rounded to FP32 first, designs rounded on
output, 1e-6).  Filtered bisection: the decisions are those of the oracle
(the candidate, the filter and the projection agree to rounding, far from
the decision margin), so the step count is equal and the midpoint agrees to
1e-14; in FP32 the filter runs in FP32, so the multiplier is compared at the
bisection tolerance.  Trajectories: to_step with each variant against the
oracle loop using the same variant."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W
from oracle import filt as ofilt
from oracle import mesh as omesh
from oracle import oc as ooc
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


def inputs(m, seed, passive, volfrac):
    r = np.random.default_rng(seed)
    x = 0.05 + 0.9 * r.random(m)
    dc = -np.exp(r.normal(0, 2, m))
    dv = np.exp(r.normal(0, 0.3, m)) / m / volfrac
    code = np.zeros(m, np.uint8)
    if passive:
        code[r.choice(m, m // 10, replace=False)] = 1
        code[r.choice(m, m // 10, replace=False)] = 2
        x[code == 1], x[code == 2] = 1.0, 0.0
    x[r.choice(m, m // 50, replace=False)] = 0.0       # exact lower-bound ties
    x[code == 1] = 1.0
    return x, dc, dv, code


def stats(t):
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import read_struct
    s = read_struct(t, L.OcStats)
    return dict(lmid=s.lmid, l1=s.l1, l2=s.l2, vol=s.vol, n_bs=s.n_bs, capped=s.capped, passes=s.passes)


@pytest.mark.parametrize("dims,dt,passive,volfrac", [
    ((60, 20), "f64", False, 0.5), ((61, 33), "f64", True, 0.5), ((300, 100), "f64", True, 0.45),
    ((1000, 600), "f64", False, 0.42), ((300, 100), "f32", True, 0.5), ((1000, 600), "f32", False, 0.4)])
def test_oc_pd_matches_oracle(dims, dt, passive, volfrac):
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Plan, _struct_tensor
    m = dims[0] * dims[1]
    x, dc, dv, code = inputs(m, 3, passive, volfrac)
    P = Plan(2, dims[0], dims[1], 1, 1.5, "D", passive=code if passive else None)
    T = torch.float64 if dt == "f64" else torch.float32
    dtype = L.TO_F64 if dt == "f64" else L.TO_F32
    if dt == "f32":
        x, dc, dv = (a.astype(np.float32).astype(np.float64) for a in (x, dc, dv))
    want, ref = ooc.oc_update_pd(x, dc, dv, code == 0, volfrac, 0.2)
    assert not ref["capped"]
    xd = torch.as_tensor(x, dtype=T).cuda()
    st = _struct_tensor(L.OcStats, "cuda")
    L.to_oc_update_pd(P.handle, dtype, xd, torch.as_tensor(dc, dtype=T).cuda(), torch.as_tensor(dv, dtype=T).cuda(),
                      volfrac, 0.2, st)
    s = stats(st)
    assert s["capped"] == 0 and abs(s["n_bs"] - ref["n_it"]) <= 1
    assert abs(s["lmid"] - ref["lm"]) <= 1e-12 * ref["lm"]
    tol = 1e-12 if dt == "f64" else 1e-6
    assert np.abs(host(xd) - want).max() <= tol
    assert abs(host(xd).mean() - volfrac) <= (1e-9 if dt == "f64" else 1e-6)


@pytest.mark.parametrize("dims,rmin,bc,ft,dt,passive", [
    ((60, 20), 2.5, "D", 1, "f64", False), ((61, 33), 3.0, "N", 2, "f64", True),
    ((120, 40), 4.5, "D", 3, "f64", True), ((300, 100), 8.75, "N", 2, "f64", False),
    ((300, 100), 8.75, "D", 2, "f32", True)])
def test_oc_filtered_matches_oracle(dims, rmin, bc, ft, dt, passive):
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Plan, _struct_tensor
    nelx, nely = dims
    m = nelx * nely
    x, dc, dv, code = inputs(m, 5, passive, 0.5)
    P = Plan(2, nelx, nely, 1, rmin, bc, passive=code if passive else None)
    T = torch.float64 if dt == "f64" else torch.float32
    dtype = L.TO_F64 if dt == "f64" else L.TO_F32
    if dt == "f32":
        x, dc, dv = (a.astype(np.float32).astype(np.float64) for a in (x, dc, dv))
    eta, beta = 0.47, 4.0
    F = ofilt.Filter(omesh.Mesh(nelx, nely), rmin, bc)
    want, ref = ooc.oc_update_filtered(x, dc, dv, code, 0.5, 0.2, F, ft, eta, beta)
    assert not ref["capped"] and ref["l1"] > 0
    xd = torch.as_tensor(x, dtype=T).cuda()
    st = _struct_tensor(L.OcStats, "cuda")
    d_eta = torch.tensor([eta], dtype=torch.float64, device="cuda")
    L.to_oc_update_filtered(P.handle, dtype, ft, xd, torch.as_tensor(dc, dtype=T).cuda(),
                            torch.as_tensor(dv, dtype=T).cuda(), 0.5, 0.2, beta, d_eta, st)
    s = stats(st)
    assert s["capped"] == 0
    if dt == "f64":
        assert s["n_bs"] == ref["n_bs"]
        assert abs(s["lmid"] - ref["lmid"]) <= 1e-14 * ref["lmid"]
        assert abs(s["vol"] - ref["vol"]) <= 1e-12
        assert np.abs(host(xd) - want).max() <= 1e-12
    else:
        assert abs(s["lmid"] - ref["lmid"]) <= 2e-4 * ref["lmid"]
        assert np.abs(host(xd) - want).max() <= 2e-4


def test_oc_filtered_rejects_bad_arguments():
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Plan, _struct_tensor
    P = Plan(2, 20, 10, 1, 1.5, "D")
    x = torch.full((200,), 0.5, dtype=torch.float64, device="cuda")
    st = _struct_tensor(L.OcStats, "cuda")
    with pytest.raises(L.ToError):
        L.to_oc_update_filtered(P.handle, L.TO_F64, 2, x, x, x, 0.5, 0.2, 2.0, None, st)     # ft 2 needs eta
    with pytest.raises(L.ToError):
        L.to_oc_update_filtered(P.handle, L.TO_F64, 4, x, x, x, 0.5, 0.2, 2.0, None, st)
    with pytest.raises(L.ToError):
        L.to_oc_update_pd(P.handle, L.TO_F64, x, x, x, 1.5, 0.2, st)


@pytest.mark.parametrize("method,ft,bc", [("pd", 1, "N"), ("filtered", 2, "D"), ("filtered", 3, "N")])
def test_step_with_oc_variant_matches_oracle(method, ft, bc):
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    cfg = W.Config("ocv", "mbb", 60, 20, volfrac=0.45, rmin=2.5, ft=ft, bc=bc, beta=2.0, eta=0.5, penal=3.0,
                   iterations=8, precision="f64")
    code = L.TO_OC_PD if method == "pd" else L.TO_OC_FILTERED
    g = TopOpt(cfg, oc=code)
    h = TopOpt(cfg, oc=code)
    prob = otop.problem_from_config(cfg)
    st = otop.State(prob)
    for k in range(8):
        lg = otop.step(prob, st, oc_method=method)
        g.step()
        h.step_stages()
        c = float(host(g.c)[0])
        assert abs(c - lg["c"]) <= 1e-6 * abs(lg["c"]), (k, c, lg["c"])
        assert np.abs(host(g.xphys) - st.xphys).max() <= 1e-5, k
        assert np.abs(host(g.x) - st.x).max() <= 1e-5, k
        assert np.abs(host(h.x) - host(g.x)).max() <= 1e-9, k
        s = g.stats()
        assert s["n_bs"] == lg["n_bs"] or method == "pd"


def test_batch_with_pd_matches_single_runs():
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Batch, TopOpt
    cfgs = [W.Config(f"b{i}", "mbb", nx, ny, volfrac=0.4 + 0.05 * i, rmin=2.0 + 0.5 * i, ft=1, bc="N",
                     iterations=4, precision="f64") for i, (nx, ny) in enumerate([(40, 20), (64, 32), (30, 10)])]
    b = Batch(cfgs, autotune=False, oc=L.TO_OC_PD)
    singles = [TopOpt(c, oc=L.TO_OC_PD) for c in cfgs]
    for k in range(4):
        b.step()
        for g in singles:
            g.step()
        for gb, gs in zip(b.runs, singles):
            assert np.abs(host(gb.x) - host(gs.x)).max() <= 1e-6
            assert abs(gb.stats()["vol"] - gs.stats()["vol"]) <= 1e-9
    with pytest.raises(L.ToError):
        Batch(cfgs[:1], autotune=False, oc=L.TO_OC_FILTERED)
