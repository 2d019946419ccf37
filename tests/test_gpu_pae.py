"""GPU tests of the periodic Anderson extrapolation of the OC iteration
(Section 3.3) against the FP64 oracle.

Step parity: the same sequence of (design before, design after the OC step)
pairs is fed to to_pae_step and to the oracle, with the oracle's output as
the next design before, over plain and extrapolated steps, early corrections
(q < m_r), passive elements and meshes that span many blocks with a ragged
tail.  The Gram matrix is summed in another order on the GPU, so FP64 agrees
to 1e-11 (the random histories are well conditioned); FP32 designs are
rounded on output (1e-6).  Trajectory parity: the whole redesign loop with
PAE on against the oracle loop followed by the oracle's PAE step."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W
from oracle import pae as opae
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


def passive_codes(m, seed):
    from paper_2005_05436_amd import _lib as L
    rng = np.random.default_rng(seed)
    code = np.zeros(m, np.uint8)
    code[rng.choice(m, m // 20, replace=False)] = L.TO_SOLID
    code[rng.choice(m, m // 20, replace=False)] = L.TO_VOID
    return code


@pytest.mark.parametrize("dims,dt,mr,q,q0,alpha,xi,passive", [
    ((60, 20), "f64", 4, 4, 3, 0.9, 1.0, False),
    ((60, 20), "f64", 4, 2, 0, 0.8, 0.7, True),          # early corrections, zero first column
    ((61, 33), "f64", 3, 1, 2, 0.9, 0.5, True),          # correction every step, wrap of the history
    ((300, 100), "f64", 8, 3, 5, 0.6, 1.0, False),
    ((300, 100), "f32", 4, 4, 1, 0.9, 1.0, True),
    ((1000, 600), "f32", 4, 4, 0, 0.9, 1.0, False),      # more elements than one pass of the grid
])
def test_pae_steps_match_oracle(dims, dt, mr, q, q0, alpha, xi, passive):
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Plan
    nelx, nely = dims
    m = nelx * nely
    code = passive_codes(m, 7) if passive else None
    P = Plan(2, nelx, nely, 1, 1.5, "D", passive=code)
    act = np.ones(m, bool) if code is None else code == L.TO_ACTIVE
    dtype = L.TO_F64 if dt == "f64" else L.TO_F32
    T = torch.float64 if dt == "f64" else torch.float32
    prm = L.PaeParams(mr, q, q0, 0, alpha, xi)
    ws = torch.zeros((L.to_pae_query(P.handle, prm) + 7) // 8, dtype=torch.float64, device="cuda")
    ref = opae.PAE(m, mr, q, q0, alpha, xi)
    rng = np.random.default_rng(11)
    x = rng.uniform(0.2, 0.8, m)
    if code is not None:
        x[code == L.TO_SOLID], x[code == L.TO_VOID] = 1.0, 0.0
    tol = 1e-11 if dt == "f64" else 1e-6
    for loop in range(q0 - 2, q0 + 4 * q + mr + 3):
        x_post = np.clip(x + 0.05 * rng.standard_normal(m) * np.exp(-0.1 * max(loop - q0, 0)), 0.0, 1.0)
        x_post[~act] = x[~act]
        if dt == "f32":
            x = x.astype(np.float32).astype(np.float64)
            x_post = x_post.astype(np.float32).astype(np.float64)
        want, used = ref.step(x, x_post, act, loop)
        xd = torch.as_tensor(x_post, dtype=T).cuda()
        L.to_pae_step(P.handle, dtype, xd, torch.as_tensor(x, dtype=T).cuda(), loop, prm, ws)
        got = host(xd)
        err = np.abs(got - want).max()
        assert err <= tol, (loop, used, err)
        assert np.array_equal(got[~act], x_post[~act])
        x = want


def test_pae_rejects_bad_arguments():
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Plan
    P = Plan(2, 20, 10, 1, 1.5, "D")
    x = torch.zeros(200, dtype=torch.float64, device="cuda")
    for bad in (L.PaeParams(9, 4, 0, 0, 0.9, 1.0), L.PaeParams(0, 4, 0, 0, 0.9, 1.0),
                L.PaeParams(4, 0, 0, 0, 0.9, 1.0), L.PaeParams(4, 4, -1, 0, 0.9, 1.0),
                L.PaeParams(4, 4, 0, 0, float("nan"), 1.0)):
        with pytest.raises(L.ToError):
            L.to_pae_query(P.handle, bad)
    prm = L.PaeParams(4, 4, 0, 0, 0.9, 1.0)
    ws = torch.zeros(L.to_pae_query(P.handle, prm) // 8 + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(L.ToError):
        L.to_pae_step(P.handle, L.TO_F64, x, x, 0, prm, ws)          # aliasing
    with pytest.raises(L.ToError):
        L.to_pae_step(P.handle, L.TO_F64, x, None, 0, prm, ws)
    y = x.clone()
    L.to_pae_step(P.handle, L.TO_F64, y, x, -5 + prm.q0, prm, ws)     # before q0: nothing
    assert torch.equal(y, x)


@pytest.mark.parametrize("ft,mr,q,q0", [(1, 4, 4, 3), (3, 4, 2, 2)])
def test_pae_trajectory_matches_oracle(ft, mr, q, q0):
    """MBB 60x20 (FP64, PCG to 1e-8 against the oracle's direct solve) with
    PAE on from loop q0: compliance and physical designs along 12 steps."""
    from paper_2005_05436_amd.driver import TopOpt
    cfg = W.Config("pae", "mbb", 60, 20, volfrac=0.4, rmin=2.5, ft=ft, bc="D", beta=2.0, penal=3.0,
                   iterations=12, precision="f64")
    g = TopOpt(cfg, pae=dict(mr=mr, q=q, q0=q0, alpha=0.9, xi=1.0))
    prob = otop.problem_from_config(cfg)
    st = otop.State(prob)
    ref = opae.PAE(prob.mesh.m, mr, q, q0, 0.9, 1.0)
    for k in range(12):
        x_pre = st.x.copy()
        lg = otop.step(prob, st)
        st.x, _ = ref.step(x_pre, st.x, prob.act, st.loop)
        g.step()
        c = float(host(g.c)[0])
        assert abs(c - lg["c"]) <= 1e-6 * abs(lg["c"]), (k, c, lg["c"])
        assert np.abs(host(g.xphys) - st.xphys).max() <= 1e-5, k
        assert np.abs(host(g.x) - st.x).max() <= 1e-5, k


def test_pae_step_stages_equals_step():
    """The single-stage sequence with PAE gives the same designs as to_step
    with PAE (same kernels, same order)."""
    from paper_2005_05436_amd.driver import TopOpt
    cfg = W.Config("pae", "mbb", 90, 30, volfrac=0.5, rmin=3.0, ft=3, bc="D", beta=2.0, penal=3.0,
                   iterations=8, precision="f64")
    a = TopOpt(cfg, pae=dict(mr=4, q=2, q0=2))
    b = TopOpt(cfg, pae=dict(mr=4, q=2, q0=2))
    for k in range(8):
        a.step()
        b.step_stages()
        assert np.abs(host(a.x) - host(b.x)).max() <= 1e-9, k
