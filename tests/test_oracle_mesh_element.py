"""Pins of the oracle's numbering, element matrices and index sets against what
the paper prints or what the mathematics fixes (CPU only)."""
import math
import os

import numpy as np
import pytest

from oracle import element, mesh, sparse

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --- element matrices -------------------------------------------------------
def _printed(name, dim, nu):
    g = np.loadtxt(os.path.join(GOLD, name))
    if dim == 2:   # App. B, block PRE.2: Ke = (c1 + nu c2) / (24 (1 - nu^2))
        return (g[:, 0] + nu * g[:, 1]) / (24.0 * (1.0 - nu * nu))
    # App. C, block PRE.2: Ke = (k1 + nu k2) / ((1 + nu)(2 nu - 1) 144)
    return (g[:, 0] + nu * g[:, 1]) / ((1.0 + nu) * (2.0 * nu - 1.0) * 144.0)


@pytest.mark.parametrize("nu", [0.3, 0.0, 0.25, 0.45])
def test_ke_q4_matches_printed_coefficients(nu):
    v = element.lower_vector(element.ke_q4(nu))
    assert v.shape == (36,)
    np.testing.assert_allclose(v, _printed("ke2d_q4_printed.txt", 2, nu), rtol=0, atol=1e-15)


@pytest.mark.parametrize("nu", [0.3, 0.1, 0.4])
def test_ke_h8_matches_printed_coefficients(nu):
    v = element.lower_vector(element.ke_h8(nu))
    assert v.shape == (300,)
    np.testing.assert_allclose(v, _printed("ke3d_h8_printed.txt", 3, nu), rtol=0, atol=1e-15)


def _rigid_modes(dim):
    """Rigid-body modes from the corner coordinates of Fig. 1b."""
    if dim == 2:
        xy = np.array([(0, 0), (1, 0), (1, 1), (0, 1)], float)
        modes = [np.tile([1, 0], 4), np.tile([0, 1], 4),
                 np.column_stack([-xy[:, 1], xy[:, 0]]).reshape(-1)]
        return np.array(modes, float).T
    c = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                  (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)], float)
    modes = [np.tile(np.eye(3)[k], 8) for k in range(3)]
    for axis in range(3):
        w = np.zeros(3)
        w[axis] = 1.0
        modes.append(np.cross(w, c).reshape(-1))
    return np.array(modes).T


@pytest.mark.parametrize("dim", [2, 3])
def test_ke_symmetric_psd_nullspace_is_rigid_modes(dim):
    K = element.element_matrix(dim, 0.3)
    np.testing.assert_allclose(K, K.T, atol=1e-16)
    ev = np.linalg.eigvalsh(K)
    nzero = 3 if dim == 2 else 6
    assert np.all(ev[:nzero] < 1e-14 * ev[-1])
    assert ev[nzero] > 1e-3
    R = _rigid_modes(dim)
    assert np.linalg.matrix_rank(R) == nzero
    assert np.abs(K @ R).max() < 1e-14


def test_lower_vector_roundtrip():
    K = element.ke_h8(0.3)
    np.testing.assert_allclose(element.from_lower_vector(element.lower_vector(K), 24), K, rtol=0, atol=1e-16)


# --- numbering and connectivity -------------------------------------------
@pytest.mark.parametrize("nelx,nely", [(4, 2), (5, 3), (60, 20)])
def test_cmat_2d_matches_paper_offsets(nelx, nely):
    """Block PRE.2 of the 2D code builds C from 1-based node numbers N(iy,ix):
    first DOF 2N+1, offsets [0, 1, 2nely+2, 2nely+3, 2nely, 2nely+1, -2, -1]."""
    M = mesh.Mesh(nelx, nely)
    N1 = np.array([[iy + 1 + (nely + 1) * ix for ix in range(nelx)] for iy in range(nely)])
    cvec = (2 * N1 + 1).reshape(-1, order="F")
    off = np.array([0, 1, 2 * nely + 2, 2 * nely + 3, 2 * nely, 2 * nely + 1, -2, -1])
    np.testing.assert_array_equal(M.cmat(), cvec[:, None] + off[None, :] - 1)


@pytest.mark.parametrize("nelx,nely,nelz", [(2, 3, 2), (4, 2, 3)])
def test_cmat_3d_matches_paper_offsets(nelx, nely, nelz):
    """Block PRE.2 of the 3D code: first DOF 3N+1 with N(iy,iz,ix) 1-based."""
    M = mesh.Mesh(nelx, nely, nelz)
    cvec = np.zeros(M.m, int)
    for ix in range(nelx):
        for iz in range(nelz):
            for iy in range(nely):
                N = iy + 1 + (nely + 1) * iz + (nely + 1) * (nelz + 1) * ix
                cvec[iy + nely * (iz + nelz * ix)] = 3 * N + 1
    a, b = 3 * (nely + 1) * (nelz + 1), 3 * (nely + 1)
    c = 3 * (nely + 1) * (nelz + 2)
    off = np.array([0, 1, 2, a, a + 1, a + 2, a - 3, a - 2, a - 1, -3, -2, -1,
                    b, b + 1, b + 2, c, c + 1, c + 2, c - 3, c - 2, c - 1, b - 3, b - 2, b - 1])
    np.testing.assert_array_equal(M.cmat(), cvec[:, None] + off[None, :] - 1)


def test_corner_nodes_are_cell_corners_3d():
    M = mesh.Mesh(3, 2, 2)
    iy, ix, iz = M.element_grid()
    nodes = M.corner_nodes()
    ny1, nz1 = M.nely + 1, M.nelz + 1
    ny_, rest = nodes % ny1, nodes // ny1
    nz_, nx_ = rest % nz1, rest // nz1
    # physical coordinates (x = ix, y = -iy, z = iz) relative to the cell
    rel = np.stack([nx_ - ix[:, None], iy[:, None] + 1 - ny_, nz_ - iz[:, None]], -1)
    expect = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                       (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)])
    assert np.all(rel == expect[None])


# --- reduced index set and CSR --------------------------------------------
@pytest.mark.parametrize("side,expected", [(120, 1_036_800), (240, 4_147_200)])
def test_ir_size_table1_2d(side, expected):
    """Table 1 (H strategy) lists the entries of the two-column array I_r:
    2 m d(d+1)/2.  (eq. (14)'s printed d~ is wrong; the loops give d(d+1)/2.)"""
    M = mesh.Mesh(side, side)
    assert 2 * sparse.reduced_index_set(M.cmat()).shape[0] == expected


@pytest.mark.parametrize("side,expected", [(8, 307_200), (16, 2_457_600)])
def test_ir_size_table1_3d(side, expected):
    """Table 1, 3D.  The 16^3 entry is printed as 2,457,200: a typo for
    2 * 4096 * 300 = 2,457,600 (the memory column, 19.7 MB, agrees with it)."""
    M = mesh.Mesh(side, side, side)
    assert 2 * sparse.reduced_index_set(M.cmat()).shape[0] == expected


@pytest.mark.parametrize("dims", [(4, 2), (5, 3), (2, 2, 3)])
def test_csr_and_perm_brute_force(dims):
    M = mesh.Mesh(*dims)
    C = M.cmat()
    ir = sparse.reduced_index_set(C)
    # brute force: the pattern of tril(sum_e A_e^T 1 A_e)
    P = np.zeros((M.n, M.n), bool)
    for e in range(M.m):
        P[np.ix_(C[e], C[e])] = True
    P = np.tril(P)
    row_ptr, col_idx, perm, seg_ptr = sparse.csr_pattern(ir, M.n)
    assert row_ptr[-1] == P.sum() == len(col_idx) == len(seg_ptr) - 1
    for r in range(M.n):
        np.testing.assert_array_equal(col_idx[row_ptr[r]:row_ptr[r + 1]], np.nonzero(P[r])[0])
    # every pair sits in the slot of its (row, col), in ascending pair order
    slot_of = {}
    for s in range(len(col_idx)):
        r = np.searchsorted(row_ptr, s, side="right") - 1
        slot_of[(r, col_idx[s])] = s
    members = {s: [] for s in range(len(col_idx))}
    for t, (r, c) in enumerate(ir):
        assert r >= c
        members[slot_of[(r, c)]].append(t)
    for s in range(len(col_idx)):
        np.testing.assert_array_equal(perm[seg_ptr[s]:seg_ptr[s + 1]], members[s])


def test_nnz_closed_form_60x20():
    M = mesh.Mesh(60, 20)
    _, col_idx, _, _ = sparse.csr_pattern(sparse.reduced_index_set(M.cmat()), M.n)
    # lower triangle: 3 per node (2x2 diagonal block) + 4 per node-pair that
    # shares an element; node pairs: horizontal, vertical, 2 diagonals
    nx, ny = M.nelx, M.nely
    pairs = nx * (ny + 1) + (nx + 1) * ny + 2 * nx * ny
    assert len(col_idx) == 3 * M.nnode + 4 * pairs == 23_363


def test_frame_problem_matches_section_3_5():
    """Sec. 3.5: loads sum to the resultants of the two distributed loads,
    the passive sets have the sizes of the code's index ranges, the fixed
    DOFs are the corner ones, and the frame rows / columns are solid."""
    M = mesh.Mesh(150, 100)
    f, fixed, code = mesh.frame(M, -1.0)
    fy, fx = f[1::2], f[0::2]
    assert math.isclose(fy.sum(), -2.0, rel_tol=1e-13)
    assert math.isclose(fx.sum(), -(100 + 1) / (2 * 100), rel_tol=1e-13)
    assert np.count_nonzero(fy) == 151 and np.count_nonzero(fx) == 100       # iy = 0 carries 0
    assert fx[M.node(100, 150)] == pytest.approx(-1.0 / 100)
    assert list(fixed) == [0, 1, M.n - 1]
    img = code.reshape(100, 150, order="F")
    n_solid = 2 * 150 + 2 * 3 * (100 - 2)            # top 2 rows, 3 columns either side
    assert np.count_nonzero(img == 1) == n_solid
    assert np.count_nonzero(img == 2) == (100 - 40 + 1) * (150 - 30 - 60 + 1)   # rows 40..100, columns 60..120 (1-based)
    assert np.all(img[:2, :] == 1) and np.all(img[:, :3] == 1) and np.all(img[:, -3:] == 1)
    assert img[39, 59] == 2 and img[38, 59] == 0 and img[39, 58] == 0 and img[99, 119] == 2 and img[99, 120] == 0
    f2, _, code2 = mesh.frame(M, 1.0)
    np.testing.assert_array_equal(code2, code)
    np.testing.assert_array_equal(f2[0::2], -fx)
    with pytest.raises(ValueError):
        mesh.frame(mesh.Mesh(120, 100))


# --- loads and supports (block PRE.3 of both codes) ------------------------
def _node_nrs_2d(nelx, nely):
    """The 2D code's nodeNrs: 1-based node numbers filled column-major into a
    (1 + nely) x (1 + nelx) array (block PRE.2)."""
    return np.arange(1, (nelx + 1) * (nely + 1) + 1).reshape((nely + 1, nelx + 1), order="F")


def _node_nrs_3d(nelx, nely, nelz):
    """The 3D code's nodeNrs: (1 + nely) x (1 + nelz) x (1 + nelx), column-major."""
    n = (nelx + 1) * (nely + 1) * (nelz + 1)
    return np.arange(1, n + 1).reshape((nely + 1, nelz + 1, nelx + 1), order="F")


@pytest.mark.parametrize("nelx,nely", [(4, 2), (7, 3), (60, 20), (300, 100)])
def test_mbb_matches_listing_pre3(nelx, nely):
    """Block PRE.3 of the 2D code, transcribed with its 1-based indices:
    lcDof = 2 nodeNrs(1, 1); fixed = union(1:2:2(nely+1), 2 nodeNrs(end, end));
    F(lcDof) = -1.  The oracle's 0-based arrays are these minus one."""
    N = _node_nrs_2d(nelx, nely)
    lc = 2 * N[0, 0]
    fixed1 = np.union1d(np.arange(1, 2 * (nely + 1) + 1, 2), [2 * N[-1, -1]])
    M = mesh.Mesh(nelx, nely)
    f, fixed = mesh.mbb(M)
    F = np.zeros(M.n)
    F[lc - 1] = -1.0
    np.testing.assert_array_equal(f, F)
    np.testing.assert_array_equal(fixed, fixed1 - 1)


@pytest.mark.parametrize("nelx,nely,load_ix", [(10, 5, 0), (10, 5, 3), (40, 20, 39)])
def test_mbb_moved_load_is_top_edge_node(nelx, nely, load_ix):
    """Ragged-batch reading of the MBB load: the same unit downward load at the
    top node of column load_ix, i.e. DOF 2 nodeNrs(1, load_ix + 1) in the
    listing's indexing; supports unchanged."""
    N = _node_nrs_2d(nelx, nely)
    M = mesh.Mesh(nelx, nely)
    f, fixed = mesh.mbb(M, load_ix)
    assert np.flatnonzero(f).tolist() == [2 * N[0, load_ix] - 1] and f.sum() == -1.0
    np.testing.assert_array_equal(fixed, mesh.mbb(M)[1])


@pytest.mark.parametrize("nelx,nely,nelz", [(4, 2, 3), (6, 3, 3), (12, 6, 6), (96, 48, 48)])
def test_cantilever3d_matches_listing_pre3(nelx, nely, nelz):
    """Block PRE.3 of the 3D code, transcribed with its 1-based indices:
    lcDof = 3 nodeNrs(1:nely+1, 1, nelx+1); fixed = 1 : 3(nely+1)(nelz+1);
    F(lcDof) = -sin((0:nely)/nely pi)."""
    N = _node_nrs_3d(nelx, nely, nelz)
    lc = 3 * N[:, 0, nelx]
    F = np.zeros(3 * N.size)
    F[lc - 1] = -np.sin(np.arange(nely + 1) / nely * np.pi)
    fixed1 = np.arange(1, 3 * (nely + 1) * (nelz + 1) + 1)
    M = mesh.Mesh(nelx, nely, nelz)
    f, fixed = mesh.cantilever3d(M)
    np.testing.assert_array_equal(f, F)
    np.testing.assert_array_equal(fixed, fixed1 - 1)


@pytest.mark.parametrize("nelx,nely,load_iy", [(10, 5, 0), (10, 5, 5), (40, 20, 7)])
def test_cantilever2d_reading(nelx, nely, load_iy):
    """The 2D cantilever of the ragged batch (no listing of its own; read in
    the 2D code's indexing): fixed = 1 : 2(nely+1), the two DOFs of every
    node of the left edge; a unit downward load on DOF 2 nodeNrs(load_iy+1,
    nelx+1), a node of the free right edge."""
    N = _node_nrs_2d(nelx, nely)
    M = mesh.Mesh(nelx, nely)
    f, fixed = mesh.cantilever2d(M, load_iy)
    np.testing.assert_array_equal(fixed, np.arange(1, 2 * (nely + 1) + 1) - 1)
    assert np.flatnonzero(f).tolist() == [2 * N[load_iy, nelx] - 1] and f.sum() == -1.0
