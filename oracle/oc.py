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


def primal_dual_lambda(xt, dc, dv0, volfrac, move, m, tol=1e-10, cap=1000):
    """The explicit primal-dual iteration of App. A (eq. (26)-(27)) for sqrt
    of the multiplier, used only as an independent cross-check of the
    bisection (no projection, all elements active)."""
    up = np.minimum(xt + move, 1.0)
    lo = np.maximum(xt - move, 0.0)
    ocp = xt * np.sqrt(np.maximum(0.0, -dc / dv0))
    lm = np.mean(ocp) / volfrac
    lm_old = 0.0
    it = 0
    while abs(lm - lm_old) > tol and it < cap:
        tmp = ocp / lm
        su, sl = tmp > up, tmp < lo
        mid = ~(su | sl)
        den = volfrac - (up[su].sum() + lo[sl].sum()) / m
        lm_old = lm
        lm = ocp[mid].sum() / den / m
        it += 1
    return lm
