"""Reduced index set, lower-triangular CSR pattern and assembly (oracle).
Test infrastructure only.

Sec. 3.1, eq. (14): only the lower triangle of each element matrix is
assembled.  For element e (ascending) and local pairs (i, j) taken column by
column (j = 0..d-1, i = j..d-1, the same order as the coefficient vector Ke),
the pair of global indices (C[e,i], C[e,j]) is sorted so that row >= col.
K^(s) = sparse(I_r, sK) sums duplicate (row, col) pairs; the paper leaves the
order of that summation to the sparse routine.  Reading adopted here: the
duplicates are summed in the order of a stable sort of I_r by (row, col), i.e.
in ascending (element, local pair) order.  All n DOFs keep their rows (the
paper assembles the whole matrix and slices the free DOFs at the solve).
"""
import numpy as np


def reduced_index_set(cmat):
    """I_r as an (m*d~) x 2 int64 array of (row, col), row >= col, eq. (14)."""
    m, d = cmat.shape
    ii, jj = [], []
    for j in range(d):
        for i in range(j, d):
            ii.append(i)
            jj.append(j)
    a = cmat[:, ii]            # m x d~   global DOF of local i
    b = cmat[:, jj]            # m x d~   global DOF of local j
    rows = np.maximum(a, b).reshape(-1)
    cols = np.minimum(a, b).reshape(-1)
    return np.stack([rows, cols], axis=1)


def csr_pattern(ir, n):
    """Lower CSR of K^(s): row_ptr (n+1), col_idx (nnz_L, ascending within a
    row), perm (stable argsort of I_r by (row, col)), seg_ptr (nnz_L+1)."""
    key = ir[:, 0].astype(np.int64) * n + ir[:, 1].astype(np.int64)
    perm = np.argsort(key, kind="stable")
    skey = key[perm]
    new = np.ones(len(skey), dtype=bool)
    new[1:] = skey[1:] != skey[:-1]
    starts = np.nonzero(new)[0]
    seg_ptr = np.append(starts, len(skey)).astype(np.int64)
    ukey = skey[starts]
    rows = ukey // n
    col_idx = (ukey % n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, col_idx, perm.astype(np.int64), seg_ptr


def simp_modulus(xphys, penal, E0, Emin):
    """eq. (6): E = Emin + xphys^p (E0 - Emin)."""
    return Emin + np.power(xphys, penal) * (E0 - Emin)


def assemble(xphys, ke_lower, perm, seg_ptr, penal, E0, Emin):
    """K^(s) values in CSR order: sK = vec(Ke) (x) E(xphys), then each CSR slot
    sums its duplicates sK[perm[t]], t = seg_ptr[s] .. seg_ptr[s+1]-1, in
    ascending t (the block RL.2 of both codes)."""
    E = simp_modulus(xphys, penal, E0, Emin)
    sk = (E[:, None] * ke_lower[None, :]).reshape(-1)
    vals = sk[perm]
    nnz = len(seg_ptr) - 1
    out = np.zeros(nnz)
    lens = np.diff(seg_ptr)
    # plain ordered summation: add the k-th member of every segment in turn
    for k in range(int(lens.max())):
        has = lens > k
        out[has] += vals[seg_ptr[:-1][has] + k]
    return out


def dense_global(cmat, ke_full, E, n):
    """K = sum_e E_e A_e^T Ke A_e, written out (tiny meshes only)."""
    K = np.zeros((n, n))
    for e in range(cmat.shape[0]):
        idx = cmat[e]
        K[np.ix_(idx, idx)] += E[e] * ke_full
    return K


def lower_to_full(row_ptr, col_idx, vals, n):
    """eq. (15): K = K^(s) + K^(s)^T - diag(K^(s)), as a scipy CSR matrix."""
    import scipy.sparse as sp
    L = sp.csr_matrix((vals, col_idx, row_ptr), shape=(n, n))
    return (L + L.T - sp.diags(L.diagonal())).tocsr()


def assemble_entry(cmat, ke_lower, E, row, col):
    """One value of K^(s) computed from its definition: every (element,
    local pair) whose sorted global pair is (row, col), summed in ascending
    (element, pair) order.  Cost O(elements containing both DOFs) after a
    scan of the connectivity; meant for sampled checks on large meshes."""
    d = cmat.shape[1]
    has_r = np.any(cmat == row, axis=1)
    has_c = np.any(cmat == col, axis=1)
    acc = 0.0
    for e in np.flatnonzero(has_r & has_c):
        k = 0
        for j in range(d):
            for i in range(j, d):
                a, b = cmat[e, i], cmat[e, j]
                if max(a, b) == row and min(a, b) == col:
                    acc += ke_lower[k] * E[e]
                k += 1
    return acc
