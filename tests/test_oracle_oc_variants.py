"""Pins of the two OC variants (oracle): the explicit primal-dual iteration
of Appendix A and the bisection that filters and projects every candidate
(Sec. 3.2).  Checked against a hand-solved case, the volume invariant of the
primal-dual fixed point, a library root finder on the monotone volume
function, the plain bisection (which the density filter with zero-Neumann
padding must reproduce, as it preserves the mean) and an independent filter
built on a library correlation."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
from scipy.optimize import brentq

from oracle import filt, mesh, oc, projection


def _inputs(m, seed, passive=False):
    r = np.random.default_rng(seed)
    x = 0.05 + 0.9 * r.random(m)
    dc = -np.exp(r.normal(0, 2, m))
    dv = np.full(m, 1.0 / m / 0.5)
    code = np.zeros(m, np.uint8)
    if passive:
        code[r.choice(m, m // 10, replace=False)] = 1
        code[r.choice(m, m // 10, replace=False)] = 2
        x[code == 1], x[code == 2] = 1.0, 0.0
    return x, dc, dv, code


def test_pd_hand_case():
    """Both elements stay inside their move limits: one dual update already
    gives the fixed point lm = sum ocP / (volfrac m)."""
    x = np.array([0.5, 0.5])
    dc = np.array([-1.0, -1.21])
    dv = np.array([1.0, 1.0])
    xn, st = oc.oc_update_pd(x, dc, dv, np.ones(2, bool), 0.5, 0.2)
    assert st["n_it"] == 1 and not st["capped"]
    assert st["lm"] == pytest.approx(1.05, rel=1e-15)
    np.testing.assert_allclose(xn, [0.5 / 1.05, 0.55 / 1.05], rtol=1e-15)
    assert math.fsum(xn) / 2 == pytest.approx(0.5, abs=1e-15)


@pytest.mark.parametrize("seed,passive,volfrac", [(0, False, 0.5), (1, True, 0.5), (2, True, 0.45)])
def test_pd_fixed_point_is_the_volume_root(seed, passive, volfrac):
    m = 3000
    x, dc, dv, code = _inputs(m, seed, passive)
    act = code == 0
    xn, st = oc.oc_update_pd(x, dc, dv, act, volfrac, 0.2)
    assert not st["capped"] and st["n_it"] < 60
    # the design meets the volume (mean over all elements) at the fixed point
    assert abs(math.fsum(xn) / m - volfrac) < 1e-9
    # the same multiplier as the root of the monotone volume function
    ocp = x[act] * np.sqrt(-dc[act] / dv[act])
    lo, hi = np.maximum(x[act] - 0.2, 0.0), np.minimum(x[act] + 0.2, 1.0)
    pas = x[~act].sum()
    vol = lambda lm: (np.clip(ocp / lm, lo, hi).sum() + pas) / m - volfrac
    root = brentq(vol, 1e-6, 1e6, xtol=1e-15, rtol=1e-15)
    assert abs(st["lm"] - root) <= 1e-9 * root
    # the box constraints hold and passive elements are untouched
    assert np.all(xn[act] >= lo - 1e-15) and np.all(xn[act] <= hi + 1e-15)
    np.testing.assert_array_equal(xn[~act], x[~act])


def test_pd_bound_ties_are_in_no_set():
    """x = 0 gives tmp = 0 = lower bound: the element is in none of the sets
    and stays 0; the others still meet the volume."""
    m = 400
    x, dc, dv, _ = _inputs(m, 5)
    x[:40] = 0.0
    xn, st = oc.oc_update_pd(x, dc, dv, np.ones(m, bool), 0.5, 0.2)
    assert np.all(xn[:40] == 0.0)
    assert abs(xn.mean() - 0.5) < 1e-9


def test_filtered_bisection_with_neumann_density_filter_is_the_plain_bisection():
    """The density filter with zero-Neumann padding preserves the mean, so the
    volume test on the filtered candidate takes the plain bisection's
    decisions."""
    M = mesh.Mesh(40, 24)
    F = filt.Filter(M, 3.0, "N")
    x, dc, dv, code = _inputs(M.m, 3)
    assert abs(F.forward(x).mean() - x.mean()) < 1e-14
    xa, sa = oc.oc_update(x, dc, dv, code == 0, 0.5, 0.2)
    xb, sb = oc.oc_update_filtered(x, dc, dv, code, 0.5, 0.2, F, 1, 0.5, 1.0)
    assert sb["n_bs"] == sa["n_bs"] and sb["lmid"] == sa["lmid"]
    np.testing.assert_array_equal(xa, xb)


def _independent_volume(x, code, nelx, nely, rmin, bc, ft, eta, beta):
    """mean of the projected filtered field with a library correlation."""
    R = math.ceil(rmin) - 1
    d = np.arange(-R, R + 1)
    h = np.maximum(0.0, rmin - np.sqrt(d[:, None] ** 2 + d[None, :] ** 2))
    mode = "constant" if bc == "D" else "reflect"
    img = x.reshape(nelx, nely).T
    xf = (ndi.correlate(img, h, mode=mode, cval=0.0) / ndi.correlate(np.ones_like(img), h, mode=mode, cval=0.0))
    xf = xf.T.reshape(-1)
    xf[code == 1], xf[code == 2] = 1.0, 0.0
    if ft > 1:
        xf = (np.tanh(beta * eta) + np.tanh(beta * (xf - eta))) / (np.tanh(beta * eta) + np.tanh(beta * (1 - eta)))
    return xf.mean()


@pytest.mark.parametrize("ft,bc,eta", [(2, "D", 0.45), (2, "N", 0.6), (1, "D", 0.5)])
def test_filtered_bisection_brackets_the_filtered_volume(ft, bc, eta):
    nelx, nely, rmin, beta = 36, 20, 2.5, 4.0
    M = mesh.Mesh(nelx, nely)
    F = filt.Filter(M, rmin, bc)
    x, dc, dv, code = _inputs(M.m, 7, passive=True)
    xn, st = oc.oc_update_filtered(x, dc, dv, code, 0.5, 0.2, F, ft, eta, beta)
    act = code == 0
    ocp = x[act] * np.sqrt(-dc[act] / dv[act])
    # both ends of the final bracket were decided (the root is inside [0, lm#])
    assert not st["capped"] and 0 < st["l1"] < st["l2"] < ocp.mean() / 0.5
    assert (st["l2"] - st["l1"]) / (st["l2"] + st["l1"]) <= 1e-4

    def cand(lm):
        y = x.copy()
        y[act] = np.clip(np.clip(ocp / lm, x[act] - 0.2, x[act] + 0.2), 0.0, 1.0)
        return y

    v1 = _independent_volume(cand(st["l1"]), code, nelx, nely, rmin, bc, ft, eta, beta)
    v2 = _independent_volume(cand(st["l2"]), code, nelx, nely, rmin, bc, ft, eta, beta)
    assert v1 > 0.5 >= v2
    np.testing.assert_allclose(xn, cand(st["lmid"]), rtol=0, atol=0)
    assert st["lmid"] in (st["l1"], st["l2"])


def test_pd_zero_sensitivities_keep_the_design():
    m = 50
    x = np.full(m, 0.5)
    xn, st = oc.oc_update_pd(x, np.zeros(m), np.full(m, 0.04), np.ones(m, bool), 0.5, 0.2)
    assert st["capped"] and st["n_it"] == 0
    np.testing.assert_array_equal(xn, x)
