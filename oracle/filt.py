"""Cone density filter, eq. (2) (oracle).  Test infrastructure only.

Sec. 2, eq. (2) and Sec. 3 (block PRE.5 / RL.1 / RL.3): the filter weight of
a neighbour at integer offset o is h(o) = max(0, rmin - |o|) with o ranging
over the box [-(ceil(rmin)-1), ceil(rmin)-1]^D; the filtered field is a
correlation with h divided by the correlation of the all-ones field,
Hs = h * 1.  Two boundary rules (the ftBC argument of Sec. 3):
  'D' -- zero padding outside the mesh (then Hs counts in-mesh weights only),
  'N' -- half-sample mirror padding (Matlab's 'symmetric'): index -1 reads 0,
         index N reads N-1; the reflection repeats with period 2N when the
         kernel is wider than the mesh.
Forward:  xt = (h * x) / Hs.
Adjoint:  H^T g = h * (g / Hs)  -- the correlation matrix is symmetric for
both rules, so the back-filter of eq. (8) (read as the chain rule, as the 2D
code does) is the same correlation applied to g / Hs.
The 3D code divides by Hs before correlating in the forward pass; eq. (2) is
followed here (identical for 'N', where Hs is constant).
"""
import numpy as np


def kernel(rmin, dim):
    """h over the offset box, built once in FP64; entries at distance >= rmin
    are exactly zero."""
    R = int(np.ceil(rmin)) - 1
    ax = np.arange(-R, R + 1, dtype=np.float64)
    grids = np.meshgrid(*([ax] * dim), indexing="ij")
    dist = np.sqrt(sum(g * g for g in grids))
    return np.maximum(0.0, rmin - dist), R


def _axis_map(N, o, bc):
    """Source index and validity for every target index along one axis."""
    k = np.arange(N) + o
    if bc == "D":
        ok = (k >= 0) & (k < N)
        return np.clip(k, 0, N - 1), ok
    k = np.mod(k, 2 * N)
    k = np.where(k >= N, 2 * N - 1 - k, k)
    return k, np.ones(N, dtype=bool)


def correlate(field, rmin, bc):
    """(h * field) with the chosen boundary rule; field has the mesh shape
    (nely, nelx) or (nely, nelz, nelx)."""
    field = np.asarray(field, dtype=np.float64)
    dim = field.ndim
    h, R = kernel(rmin, dim)
    out = np.zeros_like(field)
    offs = range(-R, R + 1)
    if dim == 2:
        for oy in offs:
            iy, vy = _axis_map(field.shape[0], oy, bc)
            for ox in offs:
                w = h[oy + R, ox + R]
                if w == 0.0:
                    continue
                ix, vx = _axis_map(field.shape[1], ox, bc)
                out += w * field[np.ix_(iy, ix)] * (vy[:, None] & vx[None, :])
    else:
        for oy in offs:
            iy, vy = _axis_map(field.shape[0], oy, bc)
            for oz in offs:
                iz, vz = _axis_map(field.shape[1], oz, bc)
                for ox in offs:
                    w = h[oy + R, oz + R, ox + R]
                    if w == 0.0:
                        continue
                    ix, vx = _axis_map(field.shape[2], ox, bc)
                    mask = vy[:, None, None] & vz[None, :, None] & vx[None, None, :]
                    out += w * field[np.ix_(iy, iz, ix)] * mask
    return out


class Filter:
    def __init__(self, mesh, rmin, bc):
        self.mesh, self.rmin, self.bc = mesh, float(rmin), bc
        self.shape = mesh.shape
        self.Hs = correlate(np.ones(self.shape), rmin, bc).reshape(-1, order="F")

    def _img(self, v):
        return np.asarray(v, dtype=np.float64).reshape(self.shape, order="F")

    def forward(self, x):
        """eq. (2): xt = (h * x) / Hs."""
        return correlate(self._img(x), self.rmin, self.bc).reshape(-1, order="F") / self.Hs

    def adjoint(self, g, scale=None):
        """H^T (scale . g) = h * (scale . g / Hs), the back-filter of eq. (8)."""
        g = np.asarray(g, dtype=np.float64)
        if scale is not None:
            g = g * scale
        return correlate(self._img(g / self.Hs), self.rmin, self.bc).reshape(-1, order="F")


def brute_force_matrix_dirichlet(mesh, rmin):
    """eq. (2) written out for tiny 2D/3D meshes: H[e,i] = h(e,i)/sum_i h(e,i)
    with h(e,i) = max(0, rmin - |c_e - c_i|) over element centroids inside the
    mesh (the 'D' rule)."""
    iy, ix, iz = mesh.element_grid()
    c = np.stack([ix, iy, iz], axis=1).astype(np.float64)
    dist = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(-1))
    w = np.maximum(0.0, rmin - dist)
    return w / w.sum(axis=1, keepdims=True)
