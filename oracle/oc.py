"""Optimality-criteria update with bisection on sqrt(lambda) (oracle).
Test infrastructure only.

eq. (10)-(11) and block RL.4 of the 2D code; the bracket is eq. (19):
  on the active set  xU = x + move,  xL = x - move,
                     ocP = x sqrt(max(0, -dc / dV0))     (the codes take the
                     real part of the root, i.e. 0 for a negative argument),
  l1 = 0,  l2 = mean_active(ocP) / volfrac            (this l2 is sqrt(lambda#)),
  while (l2 - l1) / (l2 + l1) > 1e-4:
      lmid = (l1 + l2) / 2
      x_active = max(max(min(min(ocP / lmid, xU), 1), xL), 0)
      if mean_all(x) > volfrac: l1 = lmid  else: l2 = lmid.
The volume mean is over all elements (passive ones included) and is computed
with an exactly rounded sum (math.fsum).  The paper sets no cap on the number
of bisection steps; 200 is used and hitting it is reported.  When the bracket
is empty (l2 = 0, e.g. every ocP is 0) the stop ratio is 0/0 and the loop
does not run, as in the codes.
"""
import math
import numpy as np


def oc_update(x, dc, dv0, act, volfrac, move, tol=1e-4, cap=200):
    """Returns (x_new, stats) with stats = dict(lmid, n_bs, vol, l1, l2)."""
    x = np.array(x, dtype=np.float64)
    xt = x[act]
    xu, xl = xt + move, xt - move
    ocp = xt * np.sqrt(np.maximum(0.0, -dc[act] / dv0[act]))
    l1, l2 = 0.0, math.fsum(ocp) / ocp.size / volfrac
    m = x.size
    n_bs, lmid = 0, float("nan")
    while (l1 + l2) > 0.0 and (l2 - l1) / (l2 + l1) > tol and n_bs < cap:
        lmid = 0.5 * (l1 + l2)
        x[act] = np.maximum(np.maximum(np.minimum(np.minimum(ocp / lmid, xu), 1.0), xl), 0.0)
        if math.fsum(x) / m > volfrac:
            l1 = lmid
        else:
            l2 = lmid
        n_bs += 1
    return x, dict(lmid=lmid, n_bs=n_bs, vol=math.fsum(x) / m, l1=l1, l2=l2,
                   capped=n_bs >= cap)


def oc_update_pd(x, dc, dv0, act, volfrac, move, tol=1e-10, cap=200):
    """The explicit primal-dual iteration of Appendix A (eq. of the primal map
    and of the dual map, and the code given with them) for lm = sqrt(lambda):
      lm_0 = mean_active(ocP) / volfrac,  lm_old = 0,
      while |lm - lm_old| > 1e-10:
          tmp = ocP / lm;  U = {tmp > xU'},  L = {tmp < xL'},
          M = {sign(xL' - tmp) + sign(xU' - tmp) == 0}
          lm_old = lm;  lm = sum_M ocP / (volfrac m - sum_U xU' - sum_L xL')
      x = clip(ocP / lm, xL', xU'),
    with xU' = min(x + move, 1), xL' = max(x - move, 0) on the active set.
    An element with tmp exactly on a bound (x = 0 gives tmp = 0 = xL') is in
    none of the three sets, as in the code.  Reading: the code's constraint is
    the mean of the design over all m elements; passive elements keep their
    values, so their sum is moved to the right-hand side with the bounds (the
    code, written without passive elements, has volfrac m - sum_U - sum_L).
    A non-positive denominator stops the iteration (reported as capped); the
    cap on iterations is 200 (the paper sets none).  A multiplier that is not
    positive and finite (every ocP zero) leaves the design unchanged and is
    reported as capped (the paper does not treat the case).
    Returns (x_new, stats) with stats = dict(lm, lm_old, n_it, vol, capped)."""
    x = np.array(x, dtype=np.float64)
    act = np.asarray(act, bool)
    xt = x[act]
    up = np.minimum(xt + move, 1.0)
    lo = np.maximum(xt - move, 0.0)
    ocp = xt * np.sqrt(np.maximum(0.0, -dc[act] / dv0[act]))
    m = x.size
    pas = math.fsum(x[~act])
    lm, lm_old, it, bad = math.fsum(ocp) / ocp.size / volfrac, 0.0, 0, False
    vol = float("nan")
    while abs(lm - lm_old) > tol and it < cap:
        tmp = ocp / lm
        su, sl = tmp > up, tmp < lo
        sm = (np.sign(lo - tmp) + np.sign(up - tmp)) == 0
        bnd = math.fsum(up[su]) + math.fsum(lo[sl])
        summ = math.fsum(ocp[sm])
        vol = (summ / lm + bnd + pas) / m
        den = volfrac * m - pas - bnd
        it += 1
        if not den > 0.0:
            bad = True
            break
        lm_old, lm = lm, summ / den
    if not (lm > 0.0 and math.isfinite(lm)):
        return x, dict(lm=lm, lm_old=lm_old, n_it=it, vol=vol, capped=True)
    x[act] = np.maximum(np.maximum(np.minimum(np.minimum(ocp / lm, xt + move), 1.0), xt - move), 0.0)
    return x, dict(lm=lm, lm_old=lm_old, n_it=it, vol=vol, capped=bad or it >= cap)


def oc_update_filtered(x, dc, dv0, code, volfrac, move, filt, ft, eta, beta, tol=1e-4, cap=48):
    """Bisection whose volume test filters (and, for ft > 1, projects) every
    candidate design (Sec. 3.2, the code offered for a fixed threshold):
      candidate x(lmid) as in oc_update;  xf = filt.forward(x(lmid));
      xf = 1 on passive-solid, 0 on passive-void elements;
      if ft > 1: xf = prj(xf, eta, beta);
      if mean_all(xf) > volfrac: l1 = lmid  else: l2 = lmid.
    Readings: the forward filter is eq. (2) with the plan's boundary rule (the
    code writes the filter of x / Hs and no boundary argument); the bracket
    and the stop test are those of oc_update; the cap is 48 steps.
    code: element codes (0 active, 1 passive solid, 2 passive void).
    Returns (x_new, stats) with stats = dict(lmid, n_bs, vol, l1, l2, capped)."""
    from . import projection
    x = np.array(x, dtype=np.float64)
    code = np.asarray(code)
    act = code == 0
    xt = x[act]
    xu, xl = xt + move, xt - move
    ocp = xt * np.sqrt(np.maximum(0.0, -dc[act] / dv0[act]))
    l1, l2 = 0.0, math.fsum(ocp) / ocp.size / volfrac
    m = x.size
    n_bs, lmid, vol = 0, float("nan"), float("nan")
    xc = x.copy()
    while (l1 + l2) > 0.0 and (l2 - l1) / (l2 + l1) > tol and n_bs < cap:
        lmid = 0.5 * (l1 + l2)
        xc[act] = np.maximum(np.maximum(np.minimum(np.minimum(ocp / lmid, xu), 1.0), xl), 0.0)
        xf = filt.forward(xc)
        xf[code == 1] = 1.0
        xf[code == 2] = 0.0
        if ft > 1:
            xf = projection.prj(xf, eta, beta)
        vol = math.fsum(xf) / m
        if vol > volfrac:
            l1 = lmid
        else:
            l2 = lmid
        n_bs += 1
    return xc, dict(lmid=lmid, n_bs=n_bs, vol=vol, l1=l1, l2=l2, capped=n_bs >= cap)
