"""Pins of the oracle's per-step arithmetic (CPU only): filter invariants and
brute force, projection closed forms and derivatives, assembly against the
dense definition, solve against a library factorisation, sensitivities
against finite differences, OC properties and App. A's primal-dual update,
the continuation schedule."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import (continuation, element, filt, mesh, oc, projection, sensitivity, solve,
                    sparse, topopt)

RNG = np.random.default_rng(1234)


# --- filter -----------------------------------------------------------------
@pytest.mark.parametrize("dims,rmin", [((7, 5), 2.0), ((9, 6), 3.3), ((4, 3, 5), 1.8), ((5, 4, 3), np.sqrt(3))])
@pytest.mark.parametrize("bc", ["D", "N"])
def test_filter_constant_field_is_fixed(dims, rmin, bc):
    F = filt.Filter(mesh.Mesh(*dims), rmin, bc)
    m = int(np.prod(dims))
    np.testing.assert_allclose(F.forward(np.full(m, 0.37)), 0.37, rtol=1e-14)


@pytest.mark.parametrize("dims,rmin", [((7, 5), 2.0), ((9, 6), 3.3), ((4, 3, 5), 1.8), ((3, 2), 4.5)])
def test_filter_neumann_preserves_volume(dims, rmin):
    """Mirror padding: Hs is the full kernel sum and every column of H sums to
    1, so the density filter is volume preserving (Sec. 3.2); the last case
    has a kernel wider than the mesh (repeated reflection)."""
    M = mesh.Mesh(*dims)
    F = filt.Filter(M, rmin, "N")
    h, _ = filt.kernel(rmin, M.dim)
    np.testing.assert_allclose(F.Hs, h.sum(), rtol=1e-14)
    x = RNG.random(M.m)
    assert abs(F.forward(x).sum() - x.sum()) < 1e-12 * x.sum()


@pytest.mark.parametrize("dims,rmin", [((6, 4), 2.0), ((7, 5), 2.7), ((3, 4, 2), 1.9)])
def test_filter_dirichlet_equals_brute_force_eq2(dims, rmin):
    M = mesh.Mesh(*dims)
    F = filt.Filter(M, rmin, "D")
    H = filt.brute_force_matrix_dirichlet(M, rmin)
    x = RNG.random(M.m)
    np.testing.assert_allclose(F.forward(x), H @ x, rtol=1e-13)
    g = RNG.standard_normal(M.m)
    np.testing.assert_allclose(F.adjoint(g), H.T @ g, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("bc", ["D", "N"])
@pytest.mark.parametrize("dims,rmin", [((8, 5), 2.4), ((3, 4, 5), 2.0), ((3, 2), 4.5)])
def test_filter_adjoint_identity(dims, rmin, bc):
    M = mesh.Mesh(*dims)
    F = filt.Filter(M, rmin, bc)
    x, g = RNG.random(M.m), RNG.standard_normal(M.m)
    lhs = F.forward(x) @ g
    rhs = x @ F.adjoint(g)
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + 1)


def test_filter_kernel_zero_at_rmin():
    """rmin = sqrt(3): the 3D corner offsets sit exactly at distance rmin and
    get weight exactly 0 (19 non-zero taps of 27)."""
    h, R = filt.kernel(np.sqrt(3.0), 3)
    assert R == 1 and np.count_nonzero(h) == 19


# --- projection -------------------------------------------------------------
@pytest.mark.parametrize("eta,beta", [(0.5, 1.0), (0.3, 8.0), (0.62, 32.0)])
def test_projection_endpoints_and_midpoint(eta, beta):
    assert projection.prj(np.array([0.0]), eta, beta)[0] == 0.0
    assert projection.prj(np.array([1.0]), eta, beta)[0] == 1.0
    t = math.tanh(beta * eta)
    assert abs(projection.prj(np.array([eta]), eta, beta)[0] - t / (t + math.tanh(beta * (1 - eta)))) < 1e-15
    v = np.linspace(0, 1, 101)
    assert np.all(np.diff(projection.prj(v, eta, beta)) >= 0)


def test_projection_small_beta_is_identity():
    v = np.linspace(0, 1, 11)
    np.testing.assert_allclose(projection.prj(v, 0.4, 1e-5), v, atol=1e-9)


@pytest.mark.parametrize("eta,beta", [(0.5, 1.0), (0.45, 4.0), (0.55, 32.0)])
def test_projection_derivatives_match_finite_differences(eta, beta):
    v = np.linspace(0.01, 0.99, 37)
    h = 1e-6
    fd_x = (projection.prj(v + h, eta, beta) - projection.prj(v - h, eta, beta)) / (2 * h)
    np.testing.assert_allclose(projection.dprj(v, eta, beta), fd_x, rtol=1e-6, atol=1e-8)
    fd_e = (projection.prj(v, eta + h, beta) - projection.prj(v, eta - h, beta)) / (2 * h)
    np.testing.assert_allclose(projection.deta(v, eta, beta), fd_e, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("beta", [1.0, 4.0, 32.0])
def test_newton_eta_volume_preserving(beta):
    """eq. (17): after Newton |mean(prj) - target| <= 1e-6; g is decreasing in
    eta (the uniqueness argument of Sec. 3.2)."""
    xt = np.clip(RNG.beta(0.6, 0.6, 4000), 0, 1)
    target = xt.mean()
    eta, steps, ok = projection.newton_eta(xt, 0.5, beta, target)
    assert ok and steps <= 10
    assert abs(projection.prj(xt, eta, beta).mean() - target) <= 1e-6
    assert np.mean(projection.deta(xt, eta, beta)) < 0
    assert 0.3 < eta < 0.7


# --- assembly ---------------------------------------------------------------
@pytest.mark.parametrize("dims", [(4, 2), (5, 3), (2, 3, 2)])
def test_assembly_equals_dense_definition(dims):
    M = mesh.Mesh(*dims)
    C = M.cmat()
    ke = element.element_matrix(M.dim, 0.3)
    row_ptr, col_idx, perm, seg_ptr = sparse.csr_pattern(sparse.reduced_index_set(C), M.n)
    x = RNG.random(M.m)
    kval = sparse.assemble(x, element.lower_vector(ke), perm, seg_ptr, 3.0, 1.0, 1e-9)
    Kd = sparse.dense_global(C, ke, sparse.simp_modulus(x, 3.0, 1.0, 1e-9), M.n)
    rows = np.repeat(np.arange(M.n), np.diff(row_ptr))
    np.testing.assert_allclose(kval, Kd[rows, col_idx], rtol=1e-13, atol=1e-16)
    # eq. (15) recovers the whole matrix
    np.testing.assert_allclose(sparse.lower_to_full(row_ptr, col_idx, kval, M.n).toarray(), Kd,
                               rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("dims", [(6, 3), (3, 2, 2)])
def test_assembled_matrix_annihilates_rigid_modes(dims):
    M = mesh.Mesh(*dims)
    C = M.cmat()
    ke = element.element_matrix(M.dim, 0.3)
    row_ptr, col_idx, perm, seg_ptr = sparse.csr_pattern(sparse.reduced_index_set(C), M.n)
    kval = sparse.assemble(RNG.random(M.m), element.lower_vector(ke), perm, seg_ptr, 3.0, 1.0, 1e-9)
    K = sparse.lower_to_full(row_ptr, col_idx, kval, M.n)
    nn = np.arange(M.nnode)
    iy = nn % (M.nely + 1)
    rest = nn // (M.nely + 1)
    if M.dim == 2:
        x, y = rest.astype(float), -iy.astype(float)
        modes = [np.column_stack([np.ones_like(x), 0 * x]), np.column_stack([0 * x, np.ones_like(x)]),
                 np.column_stack([-y, x])]
    else:
        iz, ix = rest % (M.nelz + 1), rest // (M.nelz + 1)
        P = np.column_stack([ix, -iy, iz]).astype(float)
        modes = [np.tile(np.eye(3)[k], (M.nnode, 1)) for k in range(3)]
        modes += [np.cross(np.eye(3)[k], P) for k in range(3)]
    for mo in modes:
        assert np.abs(K @ mo.reshape(-1)).max() < 1e-13


def test_simp_zero_power():
    """0^0 = 1 (p = 1 derivative at a void element)."""
    d = sensitivity.dsk(np.array([0.0, 0.5]), np.array([True, True]), 1.0, 1.0, 1e-9)
    np.testing.assert_allclose(d, -(1 - 1e-9))


# --- solve ------------------------------------------------------------------
def _mbb_problem(nelx, nely, **kw):
    M = mesh.Mesh(nelx, nely)
    f, fixed = mesh.mbb(M)
    return topopt.Problem(M, f, fixed, kw.pop("volfrac", 0.5), kw.pop("penal", 3.0),
                          kw.pop("rmin", 2.0), **kw)


def test_solvers_agree_with_library_factorisation():
    P = _mbb_problem(12, 6)
    x = 0.1 + 0.9 * RNG.random(P.mesh.m)
    kval = sparse.assemble(x, P.ke_lower, P.perm, P.seg_ptr, 3.0, 1.0, 1e-9)
    K = sparse.lower_to_full(P.row_ptr, P.col_idx, kval, P.mesh.n)
    ud = solve.solve_dense(K.toarray(), P.f, P.free)
    ref = np.zeros_like(P.f)
    ref[P.free] = spla.spsolve(K[P.free][:, P.free].tocsc(), P.f[P.free])
    np.testing.assert_allclose(ud, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    up, it, res, ok = solve.solve_pcg(K, P.f, P.free, np.zeros(P.mesh.n), rtol=1e-10)
    assert ok and res <= 1e-10
    np.testing.assert_allclose(up, ref, rtol=0, atol=1e-7 * np.abs(ref).max())
    # c = f^T u = u^T K u
    assert abs(P.f @ ud - ud @ (K @ ud)) < 1e-10 * abs(P.f @ ud)


# --- sensitivities by finite differences (4 x 2 MBB mesh) --------------------
def _compliance_of_x(P, x, eta, beta, penal):
    xt = P.filter.forward(x)
    xphys, dp, _, _, _ = projection.physical_density(xt, x, P.act, P.ft, eta, beta, P.volfrac)
    kval = sparse.assemble(xphys, P.ke_lower, P.perm, P.seg_ptr, penal, P.E0, P.Emin)
    K = sparse.lower_to_full(P.row_ptr, P.col_idx, kval, P.mesh.n).toarray()
    u = solve.solve_dense(K, P.f, P.free)
    return P.f @ u, xphys, dp, u


def test_elementwise_true_residual_matches_assembled_matrix():
    """The element-by-element residual that judges the full-size GPU solves
    equals the oracle's, formed with the assembled K of eq. (15), on a small
    MBB mesh with a random field (also a check of that helper's supports and
    element matrix orientation)."""
    import workloads as W
    from test_gpu_parity import _mbb_true_residual
    cfg = W.C0
    prob = topopt.problem_from_config(cfg)
    x = W.smooth_design(cfg, 3)
    kv = sparse.assemble(x, prob.ke_lower, prob.perm, prob.seg_ptr, cfg.penal, cfg.E0, cfg.Emin)
    K = sparse.lower_to_full(prob.row_ptr, prob.col_idx, kv, prob.mesh.n)
    u = RNG.normal(size=prob.mesh.n)
    u[prob.fixed] = 0.0
    want = solve.true_residual(K, prob.f, prob.free, u)
    assert abs(_mbb_true_residual(cfg, x, u) - want) <= 1e-12 * want
    uk = spla.spsolve(K[prob.free][:, prob.free].tocsc(), prob.f[prob.free])
    u2 = np.zeros(prob.mesh.n)
    u2[prob.free] = uk
    assert _mbb_true_residual(cfg, x, u2) <= 1e-10

@pytest.mark.parametrize("ft", [1, 2])
@pytest.mark.parametrize("bc", ["D", "N"])
def test_sensitivity_matches_finite_differences(ft, bc):
    """eq. (7)-(8), with eta fixed (the threshold's dependence on x is not
    differentiated by the method, so ft = 3 is not an FD case)."""
    P = _mbb_problem(4, 2, ft=ft, bc=bc, rmin=2.0)
    x = 0.2 + 0.6 * RNG.random(P.mesh.m)
    eta, beta, penal = 0.45, 4.0, 3.0
    c, xphys, dp, u = _compliance_of_x(P, x, eta, beta, penal)
    dc, ce = sensitivity.sensitivity(xphys, u, P.cmat, P.ke_full, P.act, penal, P.E0, P.Emin)
    # c = sum_e E_e ce_e
    assert abs(c - np.sum(sparse.simp_modulus(xphys, penal, P.E0, P.Emin) * ce)) < 1e-12 * c
    grad = P.filter.adjoint(dc, dp)
    fd = np.zeros(P.mesh.m)
    h = 1e-6
    for e in range(P.mesh.m):
        xp, xm = x.copy(), x.copy()
        xp[e] += h
        xm[e] -= h
        fd[e] = (_compliance_of_x(P, xp, eta, beta, penal)[0] - _compliance_of_x(P, xm, eta, beta, penal)[0]) / (2 * h)
    np.testing.assert_allclose(grad, fd, rtol=2e-6)
    # eq. (8) as typeset (dprj applied after H^T) is not the gradient
    if ft == 2:
        wrong = dp * P.filter.adjoint(dc)
        assert np.abs(wrong - fd).max() > 1e-3 * np.abs(fd).max()


# --- OC ---------------------------------------------------------------------
def _oc_inputs(m, seed):
    r = np.random.default_rng(seed)
    x = 0.05 + 0.9 * r.random(m)
    dc = -np.exp(r.normal(0, 2, m))
    dv = np.full(m, 1.0 / m / 0.5)
    return x, dc, dv


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oc_box_constraints_and_volume(seed):
    m = 5000
    x, dc, dv = _oc_inputs(m, seed)
    act = np.ones(m, bool)
    xn, st = oc.oc_update(x, dc, dv, act, 0.5, 0.2)
    assert np.all(xn >= np.maximum(0, x - 0.2) - 1e-15) and np.all(xn <= np.minimum(1, x + 0.2) + 1e-15)
    assert 13 <= st["n_bs"] <= 19
    assert st["l1"] > 0 and (st["l2"] - st["l1"]) / (st["l2"] + st["l1"]) <= 1e-4
    # the final x comes from the last lmid evaluated; the volume is within the
    # bracket's resolution of volfrac
    assert abs(st["vol"] - 0.5) < 2e-3


def test_oc_volume_monotone_in_lambda():
    m = 2000
    x, dc, dv = _oc_inputs(m, 7)
    ocp = x * np.sqrt(-dc / dv)
    lams = np.linspace(0.5, 50, 60)
    vols = [np.mean(np.clip(np.clip(ocp / l, x - 0.2, x + 0.2), 0, 1)) for l in lams]
    assert np.all(np.diff(vols) <= 0)


def test_oc_bisection_agrees_with_primal_dual_appendix_a():
    """Appendix A: for the density filter alone the multiplier has the
    explicit primal-dual fixed point; the bisection's sqrt(lambda) agrees to
    the bisection tolerance."""
    m = 4000
    x, dc, dv = _oc_inputs(m, 11)
    act = np.ones(m, bool)
    _, st = oc.oc_update(x, dc, dv, act, 0.5, 0.2)
    _, pd = oc.oc_update_pd(x, dc, dv, act, 0.5, 0.2)
    assert abs(st["lmid"] - pd["lm"]) / pd["lm"] < 2e-4


def test_oc_empty_bracket_keeps_design():
    m = 100
    x = np.full(m, 0.5)
    xn, st = oc.oc_update(x, np.zeros(m), np.full(m, 0.02), np.ones(m, bool), 0.5, 0.2)
    assert st["n_bs"] == 0
    np.testing.assert_array_equal(xn, x)


# --- continuation -------------------------------------------------------------
def test_continuation_schedules():
    penal, beta = 1.0, 1.0
    ps = (1, 3.0, 25, 0.25, "add")
    bs = (1, 32.0, 25, 2.0, "mul")
    for loop in range(1, 301):
        penal = continuation.cnt(penal, ps, loop)
        beta = continuation.cnt(beta, bs, loop)
        assert penal == min(3.0, 1 + 0.25 * (loop // 25))
        assert beta == min(32.0, 2.0 ** (loop // 25))
    assert continuation.cnt(3.0, ps, 25) == 3.0      # maxPar <= par switches it off


# --- whole loop ------------------------------------------------------------
def test_mbb_60x20_short_run_is_plausible():
    """Density filter, p = 3: compliance falls monotonically at first and the
    OC keeps mean(x) at volfrac."""
    P = _mbb_problem(60, 20, ft=1, bc="D")
    st, log = topopt.run(P, 12, solver="pcg")
    cs = [l["c"] for l in log]
    assert all(b < a for a, b in zip(cs[:8], cs[1:9]))
    assert abs(np.mean(st.x) - 0.5) < 1e-3
    assert all(l["residual"] <= 1e-8 for l in log)
    assert all(13 <= l["n_bs"] <= 19 for l in log)
