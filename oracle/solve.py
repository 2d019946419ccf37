"""State equation K(free, free) u = f(free), eq. (5) (oracle).
Test infrastructure only.

Tiny meshes: dense Cholesky of the sliced matrix, the paper's own method
(block RL.2 of both codes).  Larger meshes: a plain Jacobi-preconditioned CG
in FP64 (textbook recurrences), which is the state solver of this build.
Stopping rule (the paper is silent, it uses a direct solver): stop when the
recursive residual satisfies |r|_2 <= rtol |f_free|_2 AND the residual
recomputed as f - K u also does; if only the recursive one does, CG restarts
from the recomputed residual.  Fixed DOFs hold u = 0.
"""
import numpy as np
import scipy.linalg as sla


def solve_dense(K_full, f, free):
    """Dense Cholesky on K(free, free) (tiny meshes)."""
    Kff = K_full[np.ix_(free, free)]
    L = np.linalg.cholesky(Kff)
    y = sla.solve_triangular(L, f[free], lower=True)
    u = np.zeros_like(f)
    u[free] = sla.solve_triangular(L.T, y, lower=False)
    return u


def pcg(A, b, diag, x0, rtol=1e-8, maxit=100000):
    """Jacobi-PCG on A x = b (A symmetric positive definite, any object with
    @).  Returns (x, iterations, true relative residual, converged)."""
    x = np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0, True
    r = b - A @ x
    z = r / diag
    p = z.copy()
    rz = r @ z
    it = 0
    while True:
        if np.linalg.norm(r) <= rtol * bnorm:
            r_true = b - A @ x
            if np.linalg.norm(r_true) <= rtol * bnorm:
                return x, it, np.linalg.norm(r_true) / bnorm, True
            r = r_true
            z = r / diag
            p = z.copy()
            rz = r @ z
        if it >= maxit:
            r_true = b - A @ x
            return x, it, np.linalg.norm(r_true) / bnorm, False
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = r / diag
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1


def solve_pcg(K_full_sparse, f, free, u0, rtol=1e-8, maxit=100000):
    """Jacobi-PCG on the sliced system, warm start u0[free]."""
    Kff = K_full_sparse[free][:, free].tocsr()
    diag = Kff.diagonal()
    uf, it, res, ok = pcg(Kff, f[free], diag, u0[free], rtol, maxit)
    u = np.zeros_like(f)
    u[free] = uf
    return u, it, res, ok


def true_residual(K_full_sparse, f, free, u):
    """|f - K u|_2 / |f|_2 over the free DOFs."""
    Kff = K_full_sparse[free][:, free]
    r = f[free] - Kff @ u[free]
    return float(np.linalg.norm(r) / np.linalg.norm(f[free]))
