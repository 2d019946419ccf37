"""Element stiffness matrices (oracle).  Test infrastructure only.

The paper prints the lower triangle of the unit-size element matrix for the
bilinear Q4 plane-stress element (App. B, block PRE.2) and the trilinear Hex8
element (App. C, block PRE.2) as integer coefficient vectors.  The oracle does
not retype them: it computes the matrices from their definition,
Ke = int B^T D B dV over the unit square / cube, by tensor Gauss quadrature
(2 points per direction integrate these polynomial integrands exactly), with
the corner order of Fig. 1b.  A test checks the result against the printed
coefficients.
"""
import numpy as np

_GAUSS = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))  # 2-pt rule on [0,1]

# corner coordinates in the element-matrix order (Fig. 1b): x right, y up
_Q4_CORNERS = [(0, 0), (1, 0), (1, 1), (0, 1)]
_H8_CORNERS = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
               (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]


def _lin(c, t):
    """1D linear shape function of the corner at c in {0,1}, and its slope."""
    return (t, 1.0) if c == 1 else (1.0 - t, -1.0)


def ke_q4(nu, E=1.0):
    """8x8 plane-stress Q4 stiffness, DOFs (ux, uy) per corner."""
    D = E / (1.0 - nu * nu) * np.array([[1.0, nu, 0.0],
                                         [nu, 1.0, 0.0],
                                         [0.0, 0.0, (1.0 - nu) / 2.0]])
    K = np.zeros((8, 8))
    for gx in _GAUSS:
        for gy in _GAUSS:
            B = np.zeros((3, 8))
            for a, (cx, cy) in enumerate(_Q4_CORNERS):
                nx, sx = _lin(cx, gx)
                ny, sy = _lin(cy, gy)
                dndx, dndy = sx * ny, nx * sy
                B[0, 2 * a] = dndx          # eps_xx
                B[1, 2 * a + 1] = dndy      # eps_yy
                B[2, 2 * a] = dndy          # gamma_xy
                B[2, 2 * a + 1] = dndx
            K += 0.25 * B.T @ D @ B        # weight of each point = 1/4
    return K


def ke_h8(nu, E=1.0):
    """24x24 Hex8 stiffness, DOFs (ux, uy, uz) per corner."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[[0, 1, 2], [0, 1, 2]] += 2.0 * mu
    D[[3, 4, 5], [3, 4, 5]] = mu
    K = np.zeros((24, 24))
    for gx in _GAUSS:
        for gy in _GAUSS:
            for gz in _GAUSS:
                B = np.zeros((6, 24))
                for a, (cx, cy, cz) in enumerate(_H8_CORNERS):
                    nx, sx = _lin(cx, gx)
                    ny, sy = _lin(cy, gy)
                    nz, sz = _lin(cz, gz)
                    d = (sx * ny * nz, nx * sy * nz, nx * ny * sz)
                    B[0, 3 * a] = d[0]
                    B[1, 3 * a + 1] = d[1]
                    B[2, 3 * a + 2] = d[2]
                    B[3, 3 * a], B[3, 3 * a + 1] = d[1], d[0]          # gamma_xy
                    B[4, 3 * a + 1], B[4, 3 * a + 2] = d[2], d[1]      # gamma_yz
                    B[5, 3 * a], B[5, 3 * a + 2] = d[2], d[0]          # gamma_zx
                K += 0.125 * B.T @ D @ B
    return K


def lower_vector(K):
    """Lower triangle of a symmetric matrix, columns taken in order and rows
    from the diagonal down (the V(K_e^(s)) vector of Sec. 3.1)."""
    d = K.shape[0]
    return np.array([K[i, j] for j in range(d) for i in range(j, d)])


def from_lower_vector(v, d):
    """Inverse of lower_vector: rebuild the full symmetric matrix, eq. (15)
    applied to one element (K = L + L^T - diag L)."""
    L = np.zeros((d, d))
    k = 0
    for j in range(d):
        for i in range(j, d):
            L[i, j] = v[k]
            k += 1
    return L + L.T - np.diag(np.diag(L))


def element_matrix(dim, nu):
    return ke_q4(nu) if dim == 2 else ke_h8(nu)
