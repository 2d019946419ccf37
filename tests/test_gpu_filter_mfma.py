"""GPU parity of the matrix-core variant of the 2D FP32 filter (eq. (2) and
its adjoint) against the FP64 oracle, for each of its four tile shapes: the
forward filter, the adjoint and the fused double adjoint, both boundary
rules, meshes that span several tiles with ragged tails in both directions,
radii from one tap column to the benchmark's rmin 40, and a radius whose
two-field window does not fit in LDS (the stencil kernel takes over).  The
products are rounded to FP32 and summed in FP32 in another order than the
stencil kernel's, so the bound is the FP32 one (1e-4 relative)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W
from oracle import filt as ofilt
from oracle import mesh as omesh

TOL32 = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_05436_amd import _lib
    _lib.load()


def rel_inf(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def plan(dims, rmin, bc, shape):
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Plan
    P = Plan(2, dims[0], dims[1], 1, rmin, bc)
    L.to_plan_set_tuning(P.handle, 8, 0, 256, 1, filt_mfma=shape)
    t = L.to_plan_get_tuning(P.handle)
    assert t.filt_mfma == shape and t.filt_mfma2 == shape
    return P


CASES = [((60, 20), 1.5, "D"), ((60, 20), 2.0, "N"), ((7, 5), 4.5, "N"), ((150, 50), 5.0, "D"),
         ((130, 70), 10.0, "N"), ((97, 83), 13.3, "D"), ((300, 100), 10.0, "N")]


@pytest.mark.parametrize("shape", [1, 2, 3, 4])
@pytest.mark.parametrize("dims,rmin,bc", CASES)
def test_mfma_filter_matches_oracle(dims, rmin, bc, shape):
    from paper_2005_05436_amd import _lib as L
    P = plan(dims, rmin, bc, shape)
    M = omesh.Mesh(*dims)
    F = ofilt.Filter(M, rmin, bc)
    T = torch.float32
    xd = torch.as_tensor(W.design_field(M.m, 1), dtype=T).cuda()
    gd = torch.as_tensor(W.sensitivity_field(M.m, 2), dtype=T).cuda()
    g2d = torch.as_tensor(W.design_field(M.m, 3), dtype=T).cuda()
    sd = torch.as_tensor(W.design_field(M.m, 4, 0.1, 2.0), dtype=T).cuda()
    out, out2 = torch.zeros(M.m, dtype=T, device="cuda"), torch.zeros(M.m, dtype=T, device="cuda")
    L.to_filter(P.handle, L.TO_F32, L.TO_FILTER_FWD, xd, None, None, out, None)
    assert rel_inf(host(out), F.forward(host(xd))) < TOL32
    L.to_filter(P.handle, L.TO_F32, L.TO_FILTER_ADJ, gd, None, sd, out, None)
    assert rel_inf(host(out), F.adjoint(host(gd), host(sd))) < TOL32
    out.zero_()
    L.to_filter(P.handle, L.TO_F32, L.TO_FILTER_ADJ2, gd, g2d, sd, out, out2)
    assert rel_inf(host(out), F.adjoint(host(gd), host(sd))) < TOL32
    assert rel_inf(host(out2), F.adjoint(host(g2d), host(sd))) < TOL32


def _mirror(k, n):
    """Half-sample symmetric reflection into [0, n) (period 2 n)."""
    k = np.mod(k, 2 * n)
    return np.where(k >= n, 2 * n - 1 - k, k)


@pytest.mark.parametrize("shape,bc", [(1, "D"), (3, "D"), (2, "N")])
def test_mfma_filter_full_size_sampled(shape, bc):
    """1200 x 400 at rmin 40 (the benchmark filter): sampled outputs summed
    directly from eq. (2) with the boundary rule ('D': the window cut at the
    mesh edge, 'N': mirrored), and the whole field against the stencil
    kernel."""
    from paper_2005_05436_amd import _lib as L
    cfg = W.C1[1200]
    P = plan((cfg.nelx, cfg.nely), cfg.rmin, bc, shape)
    M = omesh.Mesh(cfg.nelx, cfg.nely)
    xd = torch.as_tensor(W.smooth_design(cfg, 5), dtype=torch.float32).cuda()
    out = torch.zeros(M.m, dtype=torch.float32, device="cuda")
    L.to_filter(P.handle, L.TO_F32, L.TO_FILTER_FWD, xd, None, None, out, None)
    got = host(out)
    xi = host(xd).reshape(M.shape, order="F")
    h, R = ofilt.kernel(cfg.rmin, 2)
    rng = np.random.default_rng(0)
    for e in np.concatenate([[0, M.m - 1, cfg.nely - 1], rng.integers(0, M.m, 200)]):
        iy, ix = e % cfg.nely, e // cfg.nely
        if bc == "D":
            y0, y1 = max(0, iy - R), min(cfg.nely, iy + R + 1)
            x0, x1 = max(0, ix - R), min(cfg.nelx, ix + R + 1)
            w = h[y0 - iy + R:y1 - iy + R, x0 - ix + R:x1 - ix + R]
            ref = (w * xi[y0:y1, x0:x1]).sum() / w.sum()
        else:
            ys = _mirror(np.arange(iy - R, iy + R + 1), cfg.nely)
            xs = _mirror(np.arange(ix - R, ix + R + 1), cfg.nelx)
            ref = (h * xi[np.ix_(ys, xs)]).sum() / h.sum()
        assert abs(got[e] - ref) <= TOL32, (e, got[e], ref)
    L.to_plan_set_tuning(P.handle, 8, 0, 256, 1, filt_mfma=0)
    ref = torch.zeros_like(out)
    L.to_filter(P.handle, L.TO_F32, L.TO_FILTER_FWD, xd, None, None, ref, None)
    assert rel_inf(got, host(ref)) < 1e-5


def test_mfma_filter_falls_back_where_the_tile_does_not_fit():
    """rmin 49 (R = 48): the two-field window of the 32 x 64 matrix-core
    tile exceeds the LDS, so the fused double adjoint runs on the stencil
    kernel and still matches the oracle; the one-field forward filter still
    fits the matrix-core tile."""
    from paper_2005_05436_amd import _lib as L
    dims, rmin = (150, 130), 49.0
    P = plan(dims, rmin, "N", 1)
    M = omesh.Mesh(*dims)
    F = ofilt.Filter(M, rmin, "N")
    gd = torch.as_tensor(W.sensitivity_field(M.m, 2), dtype=torch.float32).cuda()
    g2d = torch.as_tensor(W.design_field(M.m, 3), dtype=torch.float32).cuda()
    sd = torch.as_tensor(W.design_field(M.m, 4, 0.1, 2.0), dtype=torch.float32).cuda()
    out, out2 = torch.zeros_like(gd), torch.zeros_like(gd)
    L.to_filter(P.handle, L.TO_F32, L.TO_FILTER_FWD, g2d, None, None, out, None)
    assert rel_inf(host(out), F.forward(host(g2d))) < TOL32
    L.to_filter(P.handle, L.TO_F32, L.TO_FILTER_ADJ2, gd, g2d, sd, out, out2)
    assert rel_inf(host(out), F.adjoint(host(gd), host(sd))) < TOL32
    assert rel_inf(host(out2), F.adjoint(host(g2d), host(sd))) < TOL32


def test_mfma_filter_in_the_redesign_step_matches_stencil():
    """The whole redesign step with the matrix-core filters gives the
    designs of the stencil filters to FP32 rounding (MBB 300 x 100, rmin 10)."""
    from dataclasses import replace
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    cfg = replace(W.C1[300], iterations=6)
    a = TopOpt(cfg, autotune=False)
    b = TopOpt(cfg, autotune=False)
    L.to_plan_set_tuning(b.plan.handle, 8, 0, 256, 1, filt_mfma=1)
    for k in range(6):
        a.step()
        b.step()
        assert np.abs(host(a.xphys) - host(b.xphys)).max() <= 2e-4, k


@pytest.mark.parametrize("shape", [1, 2, 3, 4])
@pytest.mark.parametrize("dims,rmin,bc", [((60, 20), 2.0, "N"), ((150, 50), 5.0, "D"), ((97, 83), 13.3, "D"),
                                          ((130, 70), 10.0, "N"), ((1200, 400), 40.0, "D")])
def test_mfma_filter_fp64_matches_oracle(dims, rmin, bc, shape):
    """The same kernel in FP64 (v_mfma_f64_16x16x4_f64, FP64 weight table):
    forward, adjoint and double adjoint within 1e-12 of the oracle (FP64
    products summed in another order); where a tile does not fit in LDS the
    stencil kernel takes over (or, for two fields, two one-field passes)."""
    from paper_2005_05436_amd import _lib as L
    P = plan(dims, rmin, bc, shape)
    M = omesh.Mesh(*dims)
    F = ofilt.Filter(M, rmin, bc) if M.m <= 20000 else None
    T = torch.float64
    xd = torch.as_tensor(W.design_field(M.m, 1), dtype=T).cuda()
    gd = torch.as_tensor(W.sensitivity_field(M.m, 2), dtype=T).cuda()
    g2d = torch.as_tensor(W.design_field(M.m, 3), dtype=T).cuda()
    sd = torch.as_tensor(W.design_field(M.m, 4, 0.1, 2.0), dtype=T).cuda()
    out, out2 = torch.zeros(M.m, dtype=T, device="cuda"), torch.zeros(M.m, dtype=T, device="cuda")
    print(f"fp64 matrix-core filter {dims} rmin {rmin} {bc} shape {shape}", flush=True)
    L.to_filter(P.handle, L.TO_F64, L.TO_FILTER_FWD, xd, None, None, out, None)
    got_f = host(out)
    L.to_filter(P.handle, L.TO_F64, L.TO_FILTER_ADJ2, gd, g2d, sd, out, out2)
    got_a, got_a2 = host(out), host(out2)
    if F is not None:
        assert rel_inf(got_f, F.forward(host(xd))) < 1e-12
        assert rel_inf(got_a, F.adjoint(host(gd), host(sd))) < 1e-12
        assert rel_inf(got_a2, F.adjoint(host(g2d), host(sd))) < 1e-12
    else:
        # sampled outputs from eq. (2) directly, and the stencil kernel at full size
        L.to_plan_set_tuning(P.handle, 8, 0, 256, 1, filt_mfma=0)
        ref = torch.zeros(M.m, dtype=T, device="cuda")
        L.to_filter(P.handle, L.TO_F64, L.TO_FILTER_FWD, xd, None, None, ref, None)
        assert rel_inf(got_f, host(ref)) < 1e-12
        x = host(xd).reshape(dims[1], dims[0], order="F")
        h, R = ofilt.kernel(rmin, 2)
        rng = np.random.default_rng(5)
        for e in rng.integers(0, M.m, 12):
            iy, ix = int(e % dims[1]), int(e // dims[1])
            acc = wsum = 0.0
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    w = h[dy + R, dx + R]
                    if w == 0.0 or not (0 <= iy + dy < dims[1] and 0 <= ix + dx < dims[0]):
                        continue
                    acc += w * x[iy + dy, ix + dx]
                    wsum += w
            assert abs(got_f[e] - acc / wsum) <= 1e-12 * max(1.0, abs(acc / wsum))
