"""Structured-mesh bookkeeping (oracle).  Test infrastructure only.

Follows Sec. 3 (block PRE.2 / PRE.3 / PRE.6 of the 2D and 3D codes in
App. B and App. C) with 0-based indices:

* element e = iy + nely*ix (2D), e = iy + nely*(iz + nelz*ix) (3D): y runs
  fastest, so a field is a column-major nely x nelx (x nelz) image;
* node n = iy + (nely+1)*ix (2D), n = iy + (nely+1)*(iz + (nelz+1)*ix) (3D);
* DOF = dim*n + component, components (u_x, u_y[, u_z]).

Physical x follows ix, physical y points to smaller iy (row 0 is the top
edge, where the MBB load sits), physical z follows iz.  Each element lists its
corner nodes in the order the paper's element matrix expects (Fig. 1b):
lower-left, lower-right, upper-right, upper-left, and in 3D the same four on
the face iz, then on the face iz+1.
"""
import numpy as np


class Mesh:
    def __init__(self, nelx, nely, nelz=None):
        self.dim = 2 if nelz is None else 3
        self.nelx, self.nely = int(nelx), int(nely)
        self.nelz = 1 if nelz is None else int(nelz)
        if self.dim == 2:
            self.m = self.nelx * self.nely
            self.nnode = (self.nelx + 1) * (self.nely + 1)
            self.d = 8
        else:
            self.m = self.nelx * self.nely * self.nelz
            self.nnode = (self.nelx + 1) * (self.nely + 1) * (self.nelz + 1)
            self.d = 24
        self.n = self.dim * self.nnode
        self.shape = ((self.nely, self.nelx) if self.dim == 2
                      else (self.nely, self.nelz, self.nelx))

    # --- numbering ----------------------------------------------------------
    def node(self, iy, ix, iz=0):
        if self.dim == 2:
            return iy + (self.nely + 1) * ix
        return iy + (self.nely + 1) * (iz + (self.nelz + 1) * ix)

    def element(self, iy, ix, iz=0):
        if self.dim == 2:
            return iy + self.nely * ix
        return iy + self.nely * (iz + self.nelz * ix)

    def element_grid(self):
        """(iy, ix, iz) of every element, indexed by element number."""
        e = np.arange(self.m)
        iy = e % self.nely
        rest = e // self.nely
        if self.dim == 2:
            return iy, rest, np.zeros_like(iy)
        return iy, rest // self.nelz, rest % self.nelz

    def corner_nodes(self):
        """m x (2**dim) corner node numbers in the element-matrix order."""
        iy, ix, iz = self.element_grid()
        if self.dim == 2:
            corners = [(iy + 1, ix), (iy + 1, ix + 1), (iy, ix + 1), (iy, ix)]
            return np.stack([self.node(a, b) for a, b in corners], axis=1)
        corners = []
        for dz in (0, 1):
            corners += [(iy + 1, ix, iz + dz), (iy + 1, ix + 1, iz + dz),
                        (iy, ix + 1, iz + dz), (iy, ix, iz + dz)]
        return np.stack([self.node(a, b, c) for a, b, c in corners], axis=1)

    def cmat(self):
        """Connectivity C (m x d): global DOF of local DOF j of element e."""
        nodes = self.corner_nodes()
        comps = np.arange(self.dim)
        return (self.dim * nodes[:, :, None] + comps[None, None, :]).reshape(self.m, self.d)


# --- loads and supports ----------------------------------------------------
def mbb(mesh, load_ix=0):
    """Half MBB beam (Sec. 3 test setting, Fig. 2): unit downward load at the
    top node of column load_ix (the paper: the top-left node), x-DOFs of the
    left edge fixed (symmetry), y-DOF of the bottom-right node fixed."""
    assert mesh.dim == 2
    f = np.zeros(mesh.n)
    f[2 * mesh.node(0, load_ix) + 1] = -1.0
    fixed = [2 * mesh.node(iy, 0) for iy in range(mesh.nely + 1)]
    fixed.append(2 * mesh.node(mesh.nely, mesh.nelx) + 1)
    return f, np.array(sorted(set(fixed)), dtype=np.int64)


def cantilever2d(mesh, load_iy):
    """2D cantilever: every DOF of the left edge fixed, unit downward load on
    the node (load_iy, nelx) of the right edge."""
    assert mesh.dim == 2
    f = np.zeros(mesh.n)
    f[2 * mesh.node(load_iy, mesh.nelx) + 1] = -1.0
    fixed = [2 * mesh.node(iy, 0) + c for iy in range(mesh.nely + 1) for c in (0, 1)]
    return f, np.array(sorted(fixed), dtype=np.int64)


def cantilever3d(mesh, load_iz=0):
    """3D cantilever (Sec. 4, Fig. 7a, App. C block PRE.3): the face x = 0 is
    clamped; a line load along y on the bottom edge (iz = 0) of the free end
    x = nelx acts on u_z with magnitude sin((iy/nely)*pi), downward (the
    argument rounded in the code's order: the ratio first, then the
    product with pi).  load_iz moves the line up the free end (the random
    training instances of the learned warm start; 0 is the paper's case)."""
    assert mesh.dim == 3
    f = np.zeros(mesh.n)
    for iy in range(mesh.nely + 1):
        f[3 * mesh.node(iy, mesh.nelx, load_iz) + 2] = -np.sin(iy / mesh.nely * np.pi)
    fixed = [3 * mesh.node(iy, 0, iz) + c for iy in range(mesh.nely + 1)
             for iz in range(mesh.nelz + 1) for c in range(3)]
    return f, np.array(sorted(fixed), dtype=np.int64)


def frame(mesh, sign=-1.0):
    """Frame reinforcement problem (Sec. 3.5): a solid frame of thickness
    L/50 (the top nely/50 element rows and the nelx/50 element columns at
    either side) is passive solid; the elements with row index >= 2 nely/5 - 1
    and column index in [2 nelx/5 - 1, nelx - nelx/5 - 1] (0-based, the
    code's 1-based ranges) are passive void.  Loads: -2/(nelx + 1) on the
    y-DOF of every top node (a distributed load of density -2) and
    sign * iy / nely^2 on the x-DOF of the node (iy, nelx) of the right edge
    (a height-proportional load; the code gives sign = -1, the figures show
    both signs).  Fixed: both DOFs of node 0 and the last DOF of the mesh
    (the y-DOF of the bottom-right node).  nelx and nely must be multiples of
    50 (the code's ranges are integral only then).
    Returns (f, fixed, passive codes: 0 active, 1 solid, 2 void)."""
    assert mesh.dim == 2
    nelx, nely = mesh.nelx, mesh.nely
    if nelx % 50 or nely % 50:
        raise ValueError("the frame problem needs nelx and nely multiples of 50")
    f = np.zeros(mesh.n)
    for ix in range(nelx + 1):
        f[2 * mesh.node(0, ix) + 1] += -2.0 / (nelx + 1)
    for iy in range(nely + 1):
        f[2 * mesh.node(iy, nelx)] += sign * iy / nely ** 2
    fixed = np.array([0, 1, mesh.n - 1], dtype=np.int64)
    code = np.zeros((nely, nelx), dtype=np.uint8)       # [iy, ix]
    t_y, t_x = nely // 50, nelx // 50
    code[:t_y, :] = 1
    code[:, :t_x] = 1
    code[:, nelx - t_x:] = 1
    code[2 * nely // 5 - 1:, 2 * nelx // 5 - 1:nelx - nelx // 5] = 2
    return f, fixed, code.reshape(-1, order="F")


def free_dofs(mesh, fixed):
    mask = np.ones(mesh.n, dtype=bool)
    mask[np.asarray(fixed, dtype=np.int64)] = False
    return np.nonzero(mask)[0]


# --- design initialisation (block PRE.6) ----------------------------------
def initial_design(mesh, volfrac, passive=None):
    """x on the active set = (f*(m - |P0|) - |P1|)/|A|, 1 on passive solid,
    0 on passive void; dV = 1/(m*f) on the active set, 0 elsewhere.
    passive: None or per-element code 0 active, 1 solid, 2 void."""
    m = mesh.m
    code = np.zeros(m, dtype=np.int64) if passive is None else np.asarray(passive)
    act = code == 0
    n_solid = int(np.sum(code == 1))
    n_void = int(np.sum(code == 2))
    x = np.zeros(m)
    x[act] = (volfrac * (m - n_void) - n_solid) / np.sum(act)
    x[code == 1] = 1.0
    dv = np.zeros(m)
    dv[act] = 1.0 / m / volfrac
    return x, dv, act
