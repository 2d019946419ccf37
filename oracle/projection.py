"""Heaviside projection and the volume-preserving threshold (oracle).
Test infrastructure only.

eq. (1): prj(x, eta, beta) = (tanh(beta eta) + tanh(beta (x - eta)))
                             / (tanh(beta eta) + tanh(beta (1 - eta))).
eq. (9): d prj / d x = beta (1 - tanh^2(beta (x - eta))) / (same denominator).
d prj / d eta: eq. (18) is garbled in the typeset text; the closed form used in
block PRE.4 of both codes is taken instead:
   -beta csch(beta) sech^2(beta (x - eta)) sinh(beta x) sinh(beta (1 - x)).
Sec. 3.2, eq. (17): for ft = 3 the threshold eta* is found by Newton's method
on g(eta) = mean(prj(xt, eta)) - target, warm-started from the previous eta,
to |g| <= 1e-6.  The codes use target = volfrac; eq. (17) uses the volume of
the filtered field.  Both are offered.  Newton is capped at 50 steps (the
paper sets no cap); a run that hits the cap is reported, not hidden.
"""
import numpy as np


def prj(v, eta, beta):
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return (np.tanh(beta * eta) + np.tanh(beta * (v - eta))) / den


def dprj(v, eta, beta):
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return beta * (1.0 - np.tanh(beta * (v - eta)) ** 2) / den


def deta(v, eta, beta):
    return (-beta / np.sinh(beta) / np.cosh(beta * (v - eta)) ** 2
            * np.sinh(v * beta) * np.sinh((1.0 - v) * beta))


def newton_eta(xpre, eta, beta, target, tol=1e-6, cap=50):
    """Volume-preserving threshold (Sec. 3.2).  xpre is the pre-projection
    field (filtered values on active elements, 0/1 on passive ones); means are
    over all elements.  Returns (eta, newton steps, converged flag)."""
    g = np.mean(prj(xpre, eta, beta)) - target
    steps = 0
    while abs(g) > tol and steps < cap:
        eta = eta - g / np.mean(deta(xpre, eta, beta))
        g = np.mean(prj(xpre, eta, beta)) - target
        steps += 1
    return eta, steps, abs(g) <= tol


def physical_density(xt, x, act, ft, eta, beta, volfrac, target=None):
    """Block RL.1 after the filter: returns (xphys, dprj, eta, n_newton, ok).
    ft = 1: density filter only (dprj = 1); ft = 2: projection with fixed eta;
    ft = 3: projection with the volume-preserving eta*."""
    xpre = np.array(x, dtype=np.float64)
    xpre[act] = xt[act]
    if ft <= 1:
        return xpre, np.ones_like(xpre), eta, 0, True
    steps, ok = 0, True
    if ft == 3:
        tgt = volfrac if target is None else target
        eta, steps, ok = newton_eta(xpre, eta, beta, tgt)
    return prj(xpre, eta, beta), dprj(xt, eta, beta), eta, steps, ok


def change(xphys, xold):
    """Design change ch = |xphys - xold|_2 / sqrt(m) (2D code, block RL.1)."""
    return float(np.linalg.norm(xphys - xold) / np.sqrt(xphys.size))
