"""Periodic Anderson extrapolation of the OC fixed-point iteration
(Section 3.3, eq. (20)-(23) and the code given there) -- oracle.
Test infrastructure only.

The OC step is read as a fixed-point map x_{k+1} = U(x_k) with residual
r_k = U(x_k) - x_k.  From iteration q0 on, the design after the OC step is
replaced by x_k + mix r_k - dp_k, where dp_k is the Anderson correction,
computed every q-th step from the last m_r differences of the designs
(X, columns x_i - x_{i-1}) and of the residuals (R, columns r_i - r_{i-1}):
gamma solves the least-squares problem min |r_k - R gamma| (normal
equations, as the code does), dp_k = (X + mix R) gamma.  The mixing weight is
xi on the steps (k - q0) that are multiples of q, alpha on the others.  The
result is clipped to [0, 1].  Only active elements take part.

Readings (the paper's formula for the second case of eq. (23) is garbled;
the code given with it is followed): the step counter it = loop - q0; the
history gains a column from it = 2 on (column (it - 1) mod m_r); the Anderson
correction is applied when it > 1 and (it - 1) mod q == 0; the history
arrays of the code grow to the largest column index written, so the
correction uses min(it, m_r) columns, the first of which is still zero
before it = m_r + 1; the normal equations are solved by Gaussian elimination
with partial pivoting, a zero pivot giving that coefficient 0 (so a zero
column drops out).
"""
import numpy as np


class PAE:
    """History of one run (the code keeps it in persistent variables)."""

    def __init__(self, m, mr=4, q=4, q0=20, alpha=0.9, xi=1.0):
        self.mr, self.q, self.q0, self.alpha, self.xi = mr, q, q0, alpha, xi
        self.X = np.zeros((m, mr))
        self.R = np.zeros((m, mr))
        self.xold = None
        self.rold = None

    def step(self, x_pre, x_post, act, loop):
        """x_pre: design before the OC step, x_post: after it; returns the
        design to continue from (x_post unchanged before q0) and the number
        of history columns used (0 when no Anderson correction was made)."""
        it = loop - self.q0
        if it < 0:
            return x_post.copy(), 0
        act = np.asarray(act, bool)
        x = np.where(act, x_pre, 0.0)
        r = np.where(act, x_post - x_pre, 0.0)
        sel = (it % self.q) == 0
        mix = self.xi if sel else self.alpha
        dp = np.zeros_like(x)
        used = 0
        if it > 1:
            k = (it - 1) % self.mr
            self.X[:, k] = x - self.xold
            self.R[:, k] = r - self.rold
            if (it - 1) % self.q == 0:
                nc = min(it, self.mr)
                Xc, Rc = self.X[:, :nc], self.R[:, :nc]
                gamma = solve_pivot(Rc.T @ Rc, Rc.T @ r)
                dp = (Xc + mix * Rc) @ gamma
                used = nc
        xnew = x + mix * r - dp
        self.xold, self.rold = x.copy(), r.copy()
        out = x_post.copy()
        out[act] = np.clip(xnew[act], 0.0, 1.0)
        return out, used


def solve_pivot(A, b):
    """Gaussian elimination with partial pivoting; a zero pivot sets that
    unknown to zero (singular system)."""
    A = np.array(A, dtype=np.float64)
    b = np.array(b, dtype=np.float64)
    n = len(b)
    piv = list(range(n))
    scale = max(np.abs(A).max(), 1e-300)
    for k in range(n):
        p = k + int(np.argmax(np.abs(A[k:, k])))
        if p != k:
            A[[k, p]] = A[[p, k]]
            b[[k, p]] = b[[p, k]]
        if abs(A[k, k]) <= 1e-14 * scale:
            A[k, :] = 0.0
            A[:, k] = 0.0
            A[k, k] = 1.0
            b[k] = 0.0
            continue
        for i in range(k + 1, n):
            f = A[i, k] / A[k, k]
            A[i, k:] -= f * A[k, k:]
            b[i] -= f * b[k]
    x = np.zeros(n)
    for k in range(n - 1, -1, -1):
        x[k] = (b[k] - A[k, k + 1:] @ x[k + 1:]) / A[k, k]
    return x
