"""Pins of the network oracle (learned warm start of the state solve) against
library routines, closed forms and finite differences."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import unet


def test_bf16_round_known_values():
    # bfloat16 keeps 8 significand bits: 1 + 2^-7 is representable, 1 + 2^-8 is a tie -> even (1)
    vals = np.array([1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 3.0e38, 1e-40])
    want = np.array([1.0, 1.0 + 2 ** -7, 1.0, 1.0 + 2 ** -6, -2.5, 0.0, 2.0 ** 127 * (1 + 98 / 128), 0.0])
    got = unet.bf16_round(vals)
    assert got[0] == 1.0 and got[1] == 1.0 + 2 ** -7 and got[2] == 1.0 and got[3] == 1.0 + 2 ** -6
    assert got[4] == -2.5 and got[5] == 0.0
    assert got[6] == want[6]          # 3e38 = 2^127 (1 + 97.7 / 128) -> 98 / 128
    assert got[7] == 0.0 or abs(got[7]) < 1.2e-38
    # the result is always a float32 whose low 16 bits are zero
    r = np.random.default_rng(0).normal(size=1000) * 10.0 ** np.random.default_rng(1).integers(-20, 20, 1000)
    b = unet.bf16_round(r).astype(np.float32).view(np.uint32)
    assert np.all(b & 0xFFFF == 0)
    assert np.all(np.abs(unet.bf16_round(r) - r) <= np.abs(r) * 2.0 ** -8 * 1.0000001)


def test_conv3x3_equals_library_correlation():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(11, 7, 1))
    W = rng.normal(size=(9, 1, 1))
    y = unet.conv3x3(x, W)[..., 0]
    k = W[:, 0, 0].reshape(3, 3)
    ref = ndi.correlate(x[..., 0], k, mode="constant", cval=0.0)
    assert np.allclose(y, ref, atol=1e-13)


def test_conv3x3_channel_sum_and_bias():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(6, 5, 3))
    W = rng.normal(size=(9, 2, 3))
    b = np.array([0.5, -1.0])
    y = unet.conv3x3(x, W, b)
    for co in range(2):
        ref = sum(ndi.correlate(x[..., ci], W[:, co, ci].reshape(3, 3), mode="constant") for ci in range(3))
        assert np.allclose(y[..., co], ref + b[co], atol=1e-12)


def test_conv_adjoint_identities():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(8, 6, 4))
    W = rng.normal(size=(9, 3, 4))
    g = rng.normal(size=(8, 6, 3))
    # <conv(x, W), g> = <x, dgrad(g, W)> = <W, wgrad(x, g)>
    lhs = np.sum(unet.conv3x3(x, W) * g)
    assert np.isclose(lhs, np.sum(x * unet.conv3x3_dgrad(g, W)), rtol=1e-12)
    assert np.isclose(lhs, np.sum(W * unet.conv3x3_wgrad(x, g)), rtol=1e-12)


def test_parameter_count():
    assert 2.0e5 <= unet.n_params() <= 3.2e5


def _problem(seed, nelx=14, nely=6):
    rng = np.random.default_rng(seed)
    xt = rng.uniform(0.0, 1.0, nelx * nely)
    f = np.zeros(2 * (nelx + 1) * (nely + 1))
    f[2 * rng.integers(0, (nelx + 1) * (nely + 1)) + 1] = -1.0
    u = rng.normal(size=f.size)
    img = unet.features(nelx, nely, xt, f)
    return img, unet.target(nelx, nely, u), unet.node_mask(nelx, nely)


def _init(seed):
    rng = np.random.default_rng(seed)
    offs, P = unet.layer_offsets()
    p = np.zeros(P)
    for (name, ci, co, *_r), (ow, ob) in zip(unet.LAYERS, offs):
        p[ow:ob] = rng.normal(size=ob - ow) * np.sqrt(2.0 / (9 * ci))
        p[ob:ob + co] = rng.normal(size=co) * 0.1
    return p


def test_gradient_matches_finite_differences():
    img, tgt, mk = _problem(0)
    p = _init(1)
    loss, g = unet.loss_and_grad(p, img, tgt, mk)
    rng = np.random.default_rng(2)
    offs, P = unet.layer_offsets()
    # a few weights and a bias of every layer
    picks = []
    for (ow, ob), L in zip(offs, unet.LAYERS):
        picks += list(rng.integers(ow, ob, 2)) + [ob + int(rng.integers(0, L[2]))]
    for i in picks:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (unet.loss_and_grad(pp, img, tgt, mk)[0] - unet.loss_and_grad(pm, img, tgt, mk)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), abs(g[i]), 1e-3 * abs(g).max()), (i, fd, g[i])


def test_bf16_mode_is_close_to_fp64():
    img, tgt, mk = _problem(7)
    p = _init(8)
    o64, _ = unet.forward(p, img)
    o16, _ = unet.forward(p, img, bf16=True)
    rel = np.abs(o16 - o64).max() / np.abs(o64).max()
    assert 1e-5 < rel < 0.1


def test_adam_first_step_moves_by_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p, m, v = unet.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(p[:3], -0.01 * np.sign(g[:3]), rtol=1e-4)
    assert p[3] == 0.0


def test_adam_minimises_a_quadratic():
    target = np.array([1.0, -2.0, 0.5])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for k in range(1, 3001):
        p, m, v = unet.adam(p, 2 * (p - target), m, v, k, lr=0.01)
    assert np.allclose(p, target, atol=1e-3)


def test_features_density_is_node_average():
    nelx, nely = 5, 3
    xt = np.arange(nelx * nely, dtype=float)
    img = unet.features(nelx, nely, xt, np.zeros(2 * (nelx + 1) * (nely + 1)))
    xe = xt.reshape(nelx, nely)
    assert img[0, 0, 0] == xe[0, 0]
    assert img[2, 1, 0] == np.mean([xe[1, 0], xe[2, 0], xe[1, 1], xe[2, 1]])
    assert img.shape[:2] == (8, 8) and np.all(img[nelx + 1:, :, :] == 0)


def test_galerkin_start_minimises_energy():
    rng = np.random.default_rng(9)
    n = 40
    A = rng.normal(size=(n, n))
    K = A @ A.T + n * np.eye(n)
    f = rng.normal(size=n)
    ustar = np.linalg.solve(K, f)
    E = lambda u: 0.5 * u @ K @ u - f @ u
    up = ustar + 0.3 * rng.normal(size=n)
    uh = ustar + 0.5 * rng.normal(size=n)
    u0 = unet.galerkin_start(K, f, uh, up)
    for a in np.linspace(-1, 2, 7):
        for b in np.linspace(-1, 2, 7):
            assert E(u0) <= E(a * uh + b * up) + 1e-10
    # an exact prediction is recovered exactly; a zero previous field falls back
    assert np.allclose(unet.galerkin_start(K, f, ustar, up), ustar)
    assert np.allclose(unet.galerkin_start(K, f, uh, np.zeros(n)), (uh @ f) / (uh @ K @ uh) * uh)


# --- the 3D network (Hex8 meshes) --------------------------------------------

def test_conv3x3x3_equals_library_correlation():
    rng = np.random.default_rng(13)
    x = rng.normal(size=(6, 5, 7, 2))
    W = rng.normal(size=(27, 3, 2))
    b = np.array([0.25, -0.5, 1.0])
    y = unet.conv3x3(x, W, b)
    for co in range(3):
        ref = sum(ndi.correlate(x[..., ci], W[:, co, ci].reshape(3, 3, 3), mode="constant") for ci in range(2))
        assert np.allclose(y[..., co], ref + b[co], atol=1e-12)


def test_conv3d_adjoint_identities():
    rng = np.random.default_rng(14)
    x = rng.normal(size=(4, 6, 5, 3))
    W = rng.normal(size=(27, 2, 3))
    g = rng.normal(size=(4, 6, 5, 2))
    lhs = np.sum(unet.conv3x3(x, W) * g)
    assert np.isclose(lhs, np.sum(x * unet.conv3x3_dgrad(g, W)), rtol=1e-12)
    assert np.isclose(lhs, np.sum(W * unet.conv3x3_wgrad(x, g)), rtol=1e-12)


def test_pool_and_upsample_3d():
    rng = np.random.default_rng(15)
    x = rng.normal(size=(4, 6, 8, 2))
    p = unet.pool2(x)
    assert p.shape == (2, 3, 4, 2)
    assert np.isclose(p[1, 2, 3, 1], x[2:4, 4:6, 6:8, 1].mean())
    y = rng.normal(size=(2, 3, 4, 2))
    # up2 and sum2 are adjoint; pool2 = sum2 / 8
    assert np.isclose(np.sum(unet.up2(y) * x), np.sum(y * unet.sum2(x)), rtol=1e-12)
    assert np.allclose(unet.pool2(x), unet.sum2(x) / 8.0)
    assert np.all(unet.up2(y)[3, 5, 7] == y[1, 2, 3])


def test_parameter_count_3d():
    assert 2.0e5 <= unet.n_params(3) <= 3.2e5


def _problem3(seed, nelx=5, nely=4, nelz=3):
    rng = np.random.default_rng(seed)
    xt = rng.uniform(0.0, 1.0, nelx * nely * nelz)
    f = np.zeros(3 * (nelx + 1) * (nely + 1) * (nelz + 1))
    f[3 * rng.integers(0, f.size // 3) + 2] = -1.0
    u = rng.normal(size=f.size)
    img = unet.features3(nelx, nely, nelz, xt, f)
    return img, unet.target3(nelx, nely, nelz, u), unet.node_mask3(nelx, nely, nelz)


def _init3(seed):
    rng = np.random.default_rng(seed)
    offs, P = unet.layer_offsets(3)
    p = np.zeros(P)
    for (name, ci, co, *_r), (ow, ob) in zip(unet.LAYERS3, offs):
        p[ow:ob] = rng.normal(size=ob - ow) * np.sqrt(2.0 / (27 * ci))
        p[ob:ob + co] = rng.normal(size=co) * 0.1
    return p


def test_gradient_matches_finite_differences_3d():
    img, tgt, mk = _problem3(20)
    p = _init3(21)
    loss, g = unet.loss_and_grad(p, img, tgt, mk)
    rng = np.random.default_rng(22)
    offs, P = unet.layer_offsets(3)
    picks = []
    for (ow, ob), L in zip(offs, unet.LAYERS3):
        picks += list(rng.integers(ow, ob, 2)) + [ob + int(rng.integers(0, L[2]))]
    for i in picks:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (unet.loss_and_grad(pp, img, tgt, mk)[0] - unet.loss_and_grad(pm, img, tgt, mk)[0]) / (2 * h)
        # the central difference carries a rounding floor of about eps |loss| / h
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), abs(g[i])) + 1e-9, (i, fd, g[i])


def test_features3_density_and_load_layout():
    nelx, nely, nelz = 3, 4, 2
    xt = np.arange(nelx * nely * nelz, dtype=float)
    f = np.zeros(3 * (nelx + 1) * (nely + 1) * (nelz + 1))
    node = 2 + (nely + 1) * (1 + (nelz + 1) * 3)            # iy = 2, iz = 1, ix = 3
    f[3 * node + 2] = -7.0
    img = unet.features3(nelx, nely, nelz, xt, f)
    e = lambda iy, iz, ix: xt[iy + nely * (iz + nelz * ix)]
    assert img.shape == (8, 8, 8, 4)
    assert img[0, 0, 0, 0] == e(0, 0, 0)
    # node (iy 2, iz 1, ix 1): the eight elements around it
    want = np.mean([e(iy, iz, ix) for iy in (1, 2) for iz in (0, 1) for ix in (0, 1)])
    assert np.isclose(img[1, 1, 2, 0], want)
    assert img[3, 1, 2, 3] == -7.0 and np.count_nonzero(img[..., 1:]) == 1
