"""Problem definitions on the GPU-library side (block PRE.3 of the paper's
codes): load vectors and fixed DOFs in the library's numbering
(node n = iy + (nely+1) ix [+ (nely+1)(nelz+1)-strided z], DOF = dim n + c,
row iy = 0 on top).  Host numpy only; these are inputs of the C ABI.
"""
import numpy as np


def _node2(nely, iy, ix):
    return iy + (nely + 1) * ix


def _node3(nely, nelz, iy, ix, iz):
    return iy + (nely + 1) * (iz + (nelz + 1) * ix)


def mbb(nelx, nely, load_ix=0):
    """Half MBB beam: unit downward load at the top node of column load_ix,
    x-DOFs of the left edge and the y-DOF of the bottom-right node fixed."""
    n = 2 * (nelx + 1) * (nely + 1)
    f = np.zeros(n)
    f[2 * _node2(nely, 0, load_ix) + 1] = -1.0
    fixed = np.array([2 * _node2(nely, iy, 0) for iy in range(nely + 1)]
                     + [2 * _node2(nely, nely, nelx) + 1], dtype=np.int32)
    return f, np.unique(fixed)


def cantilever2d(nelx, nely, load_iy):
    """Left edge clamped, unit downward load on node (load_iy, nelx)."""
    n = 2 * (nelx + 1) * (nely + 1)
    f = np.zeros(n)
    f[2 * _node2(nely, load_iy, nelx) + 1] = -1.0
    iy = np.arange(nely + 1)
    fixed = np.concatenate([2 * _node2(nely, iy, 0), 2 * _node2(nely, iy, 0) + 1]).astype(np.int32)
    return f, np.unique(fixed)


def cantilever3d(nelx, nely, nelz, load_iz=0):
    """Face x = 0 clamped; downward line load sin(pi iy / nely) on u_z along
    the line iz = load_iz (0: the bottom edge, the paper's case) of the end
    x = nelx."""
    n = 3 * (nelx + 1) * (nely + 1) * (nelz + 1)
    f = np.zeros(n)
    iy = np.arange(nely + 1)
    f[3 * _node3(nely, nelz, iy, nelx, load_iz) + 2] = -np.sin(iy / nely * np.pi)
    nodes = np.arange((nely + 1) * (nelz + 1))          # ix = 0 face: the first nodes
    fixed = (3 * nodes[:, None] + np.arange(3)[None, :]).reshape(-1).astype(np.int32)
    return f, fixed


def frame(nelx, nely, sign=-1.0):
    """Frame reinforcement (Sec. 3.5): solid frame of thickness L/50 on top
    and at both sides, a void opening at the lower right of the middle, a
    uniform downward load of total 2 on the top nodes and a horizontal load
    sign * iy / nely^2 on the right-edge nodes; node 0 pinned, the last DOF
    (y of the bottom-right node) fixed.  Returns (f, fixed, element codes)."""
    if nelx % 50 or nely % 50:
        raise ValueError("frame: nelx and nely must be multiples of 50")
    n = 2 * (nelx + 1) * (nely + 1)
    f = np.zeros(n)
    ix = np.arange(nelx + 1)
    f[2 * _node2(nely, 0, ix) + 1] = -2.0 / (nelx + 1)
    iy = np.arange(nely + 1)
    f[2 * _node2(nely, iy, nelx)] = sign * iy / float(nely * nely)
    fixed = np.array([0, 1, n - 1], dtype=np.int32)
    ey, ex = np.meshgrid(np.arange(nely), np.arange(nelx), indexing="ij")
    solid = (ey < nely // 50) | (ex < nelx // 50) | (ex >= nelx - nelx // 50)
    void = (ey >= 2 * nely // 5 - 1) & (ex >= 2 * nelx // 5 - 1) & (ex < nelx - nelx // 5)
    code = np.where(solid, 1, np.where(void, 2, 0)).astype(np.uint8)
    return f, fixed, code.T.reshape(-1)          # element e = iy + nely * ix


def from_config(cfg):
    """(f, fixed, passive codes or None) for a workloads.Config."""
    if cfg.nelz:
        return cantilever3d(cfg.nelx, cfg.nely, cfg.nelz, cfg.load) + (None,)
    if cfg.kind == "mbb":
        return mbb(cfg.nelx, cfg.nely, cfg.load) + (None,)
    if cfg.kind == "frame":
        return frame(cfg.nelx, cfg.nely, -1.0 if cfg.load == 0 else 1.0)
    return cantilever2d(cfg.nelx, cfg.nely, cfg.load) + (None,)
