"""Learned warm start for the state solve: a small U-Net that maps the
filtered density and the load to a displacement field (oracle).
Test infrastructure only.

The paper has no network.  Its nearest relative is the acceleration of the
redesign loop in Section 3.3; the network here serves the solve of eq. (5)
only as a starting point, so the solve's true residual still decides the
answer.  The architecture is this build's own; the oracle defines it, and the
GPU kernels follow the oracle:

* image: node grid with rows = ix (0..nelx) and columns = iy (0..nely), both
  padded with zeros up to a multiple of 8, so pixel (ix, iy) is node
  iy + (nely + 1) ix and its two channels are that node's two DOFs;
* input channels: mean filtered density of the elements around the node,
  f_x, f_y;  output channels: u_x, u_y, normalised by the RMS of u over the
  real nodes (the solve only needs the direction: the warm start rescales);
* 'same' 3x3 cross-correlations with zero padding, bias, leaky ReLU with
  slope 1/8, 2x2 average pooling, nearest 2x upsampling, additive skips:

    e1a 3->16, e1b 16->16 | pool | e2a 16->32, e2b 32->32 | pool |
    e3a 32->64, e3b 64->64 | pool | ba 64->128, bb 128->64 |
    up, d3a 64->64 (+ e3b), d3b 64->32 | up, d2a 32->32 (+ e2b), d2b 32->16 |
    up, d1a 16->16 (+ e1b), d1b 16->16 | out 16->2 (no activation)

* loss: mean squared error over the real nodes and both channels;
* Adam with bias correction.

``bf16=True`` rounds to bfloat16 (round to nearest even) where the GPU
stores bfloat16: the weights, the input image, every activation after bias,
activation and skip, every pooled image, and the error signals fed to the
two products of the backward pass.  All sums stay in FP64.

Weights: flat FP64 vector, per layer W[t][co][ci] (t = 3 (dr + 1) + (dc + 1),
offset (dr, dc) along rows and columns) then b[co].

The 3D network (for Hex8 meshes) has the same structure with 3x3x3
cross-correlations, 2x2x2 average pooling and nearest 2x upsampling along
all three axes, half the channels (8, 16, 32, 64; about 2.2e5 parameters),
four input channels (density, f_x, f_y, f_z) and three outputs.  Its image
is [ix][iz][iy] (planes, rows, columns), each padded to a multiple of 8, so
pixel (ix, iz, iy) is node iy + (nely + 1) (iz + (nelz + 1) ix); tap
t = 9 (dp + 1) + 3 (dr + 1) + (dc + 1) for the offset (dp, dr, dc).  Every
function below takes 2D images [H, W, C] and 3D images [D, H, W, C] alike.
"""
import numpy as np

SLOPE = 0.125

# (name, c_in, c_out, level, activation, input: 'prev' | 'pool' | 'up', skip)
LAYERS = [
    ("e1a", 3, 16, 0, True, "prev", None),
    ("e1b", 16, 16, 0, True, "prev", None),
    ("e2a", 16, 32, 1, True, "pool", None),
    ("e2b", 32, 32, 1, True, "prev", None),
    ("e3a", 32, 64, 2, True, "pool", None),
    ("e3b", 64, 64, 2, True, "prev", None),
    ("ba", 64, 128, 3, True, "pool", None),
    ("bb", 128, 64, 3, True, "prev", None),
    ("d3a", 64, 64, 2, True, "up", "e3b"),
    ("d3b", 64, 32, 2, True, "prev", None),
    ("d2a", 32, 32, 1, True, "up", "e2b"),
    ("d2b", 32, 16, 1, True, "prev", None),
    ("d1a", 16, 16, 0, True, "up", "e1b"),
    ("d1b", 16, 16, 0, True, "prev", None),
    ("out", 16, 2, 0, False, "prev", None),
]


LAYERS3 = [
    ("e1a", 4, 8, 0, True, "prev", None),
    ("e1b", 8, 8, 0, True, "prev", None),
    ("e2a", 8, 16, 1, True, "pool", None),
    ("e2b", 16, 16, 1, True, "prev", None),
    ("e3a", 16, 32, 2, True, "pool", None),
    ("e3b", 32, 32, 2, True, "prev", None),
    ("ba", 32, 64, 3, True, "pool", None),
    ("bb", 64, 32, 3, True, "prev", None),
    ("d3a", 32, 32, 2, True, "up", "e3b"),
    ("d3b", 32, 16, 2, True, "prev", None),
    ("d2a", 16, 16, 1, True, "up", "e2b"),
    ("d2b", 16, 8, 1, True, "prev", None),
    ("d1a", 8, 8, 0, True, "up", "e1b"),
    ("d1b", 8, 8, 0, True, "prev", None),
    ("out", 8, 3, 0, False, "prev", None),
]


def layers(dim=2):
    return LAYERS if dim == 2 else LAYERS3


def taps(dim=2):
    return 9 if dim == 2 else 27


def offsets(dim):
    """Tap offsets in tap order: (dr, dc) in 2D, (dp, dr, dc) in 3D."""
    if dim == 2:
        return [(t // 3 - 1, t % 3 - 1) for t in range(9)]
    return [(t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1) for t in range(27)]


def layer_offsets(dim=2):
    """Offsets of each layer's W and b in the flat parameter vector."""
    offs, o = [], 0
    T = taps(dim)
    for (_, ci, co, *_rest) in layers(dim):
        offs.append((o, o + T * co * ci))
        o += T * co * ci + co
    return offs, o


def n_params(dim=2):
    return layer_offsets(dim)[1]


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    Values are first taken to float32, as on the GPU."""
    x = np.asarray(a, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((bits >> 16) & 1)
    r = ((bits + bias) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _rnd(a, on):
    return bf16_round(a) if on else a


def _shifted(x, o):
    """The zero-padded image x shifted by the offset o: out[p] = x[p + o]."""
    sp = x.shape[:-1]
    xp = np.zeros(tuple(n + 2 for n in sp) + (x.shape[-1],))
    xp[tuple(slice(1, -1) for _ in sp)] = x
    return xp[tuple(slice(1 + d, 1 + d + n) for d, n in zip(o, sp))]


def conv3x3(x, W, b=None):
    """'same' 3x3 (3x3x3) cross-correlation with zero padding: x [H, W, Ci]
    (or [D, H, W, Ci]), W [T, Co, Ci] -> [H, W, Co] (or [D, H, W, Co])."""
    dim = x.ndim - 1
    y = np.zeros(x.shape[:-1] + (W.shape[1],))
    for t, o in enumerate(offsets(dim)):
        y += _shifted(x, o) @ W[t].T
    if b is not None:
        y += b
    return y


def conv3x3_wgrad(x, dz):
    """d loss / d W for y = conv3x3(x, W): sum over pixels of x(p + o_t) dz(p)."""
    dim = x.ndim - 1
    offs = offsets(dim)
    g = np.zeros((len(offs), dz.shape[-1], x.shape[-1]))
    for t, o in enumerate(offs):
        xs = _shifted(x, o).reshape(-1, x.shape[-1])
        g[t] = dz.reshape(-1, dz.shape[-1]).T @ xs
    return g


def conv3x3_dgrad(dz, W):
    """d loss / d x for y = conv3x3(x, W): the correlation of dz with the
    flipped, transposed kernel."""
    T = W.shape[0]
    Wt = np.stack([W[T - 1 - t].T for t in range(T)])
    return conv3x3(dz, Wt)


def _corners(x):
    """The 2^dim sub-images x[a::2, b::2, ...] of the even/odd corners."""
    dim = x.ndim - 1
    out = []
    for k in range(2 ** dim):
        out.append(x[tuple(slice((k >> (dim - 1 - a)) & 1, None, 2) for a in range(dim))])
    return out


def pool2(x):
    c = _corners(x)
    s = c[0]
    for t in c[1:]:
        s = s + t
    return s / len(c)


def up2(x):
    for a in range(x.ndim - 1):
        x = np.repeat(x, 2, axis=a)
    return x


def sum2(x):
    """Sum over each 2x2 (2x2x2) block: the adjoint of up2."""
    c = _corners(x)
    s = c[0]
    for t in c[1:]:
        s = s + t
    return s


def leaky(z):
    return np.where(z > 0, z, SLOPE * z)


def leaky_grad(y):
    """Derivative of the leaky ReLU from its output (same sign as its input)."""
    return np.where(y > 0, 1.0, SLOPE)


def unpack(params, dim=2):
    offs, _ = layer_offsets(dim)
    T = taps(dim)
    out = []
    for (name, ci, co, *_r), (ow, ob) in zip(layers(dim), offs):
        out.append((params[ow:ob].reshape(T, co, ci), params[ob:ob + co]))
    return out


def forward(params, img, bf16=False):
    """Returns the output image ([H, W, 2] in 2D, [D, H, W, 3] in 3D) and the
    cache for backward()."""
    dim = img.ndim - 1
    wb = unpack(params, dim)
    cache = {"in": _rnd(img, bf16), "dim": dim}
    x = cache["in"]
    act = {}
    for (name, ci, co, lev, use_act, src, skip), (W, b) in zip(layers(dim), wb):
        W = _rnd(W, bf16)
        if src == "pool":
            x = _rnd(pool2(x), bf16)
        elif src == "up":
            x = up2(x)
        cache[name + ".x"] = x
        z = conv3x3(x, W, b)
        if use_act:
            a = leaky(z)
            y = a + act[skip] if skip else a
            a = _rnd(a, bf16)
            y = _rnd(y, bf16)
            cache[name + ".a"] = a
        else:
            y = z
        act[name] = y
        x = y
    return x, cache


def backward(params, cache, dout, bf16=False):
    """Gradient of a loss with d loss / d output = dout, for every weight."""
    dim = cache.get("dim", 2)
    LY = layers(dim)
    wb = unpack(params, dim)
    offs, P = layer_offsets(dim)
    grad = np.zeros(P)
    G = {"out": dout}
    prev = {}
    for i, L in enumerate(LY):
        prev[L[0]] = LY[i - 1][0] if i > 0 else None
    for i in range(len(LY) - 1, -1, -1):
        name, ci, co, lev, use_act, src, skip = LY[i]
        W, _ = wb[i]
        W = _rnd(W, bf16)
        g = G.pop(name)
        if skip:
            G[skip] = G.get(skip, 0.0) + g
        dz = g * leaky_grad(cache[name + ".a"]) if use_act else g
        dz = _rnd(dz, bf16)
        ow, ob = offs[i]
        x = cache[name + ".x"]
        grad[ow:ob] = conv3x3_wgrad(x, dz).ravel()
        grad[ob:ob + co] = dz.sum(axis=tuple(range(dim)))
        if i == 0:
            break
        gx = conv3x3_dgrad(dz, W)
        p = prev[name]
        if src == "pool":
            gx = up2(gx) / 2 ** dim
        elif src == "up":
            gx = sum2(gx)
        G[p] = G.get(p, 0.0) + gx
    return grad


def loss_and_grad(params, img, target, mask, bf16=False):
    """Mean squared error over the masked pixels (every output channel) and
    its gradient."""
    out, cache = forward(params, img, bf16)
    nc = target.shape[-1]
    cnt = nc * mask.sum()
    diff = (out[..., :nc] - target) * mask[..., None]
    loss = float((diff * diff).sum() / cnt)
    dout = 2.0 * diff / cnt
    return loss, backward(params, cache, dout, bf16)


def adam(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected moments); step counts from 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# --- features and targets on the node grid --------------------------------

def image_shape(nelx, nely):
    return ((nelx + 1 + 7) // 8 * 8, (nely + 1 + 7) // 8 * 8)


def features(nelx, nely, xtilde, f):
    """Input image: mean filtered density of the (1 to 4) elements around
    each node, and the nodal load."""
    H, Wd = image_shape(nelx, nely)
    img = np.zeros((H, Wd, 3))
    xe = np.asarray(xtilde, dtype=np.float64).reshape(nelx, nely)   # [ix, iy]
    s = np.zeros((nelx + 1, nely + 1))
    c = np.zeros((nelx + 1, nely + 1))
    for ax in (0, 1):
        for ay in (0, 1):
            s[ax:ax + nelx, ay:ay + nely] += xe
            c[ax:ax + nelx, ay:ay + nely] += 1.0
    img[:nelx + 1, :nely + 1, 0] = s / c
    fn = np.asarray(f, dtype=np.float64).reshape(nelx + 1, nely + 1, 2)
    img[:nelx + 1, :nely + 1, 1:3] = fn
    return img


def node_mask(nelx, nely):
    H, Wd = image_shape(nelx, nely)
    mk = np.zeros((H, Wd))
    mk[:nelx + 1, :nely + 1] = 1.0
    return mk


def target(nelx, nely, u):
    """u normalised by its RMS over the real DOFs, as an image."""
    H, Wd = image_shape(nelx, nely)
    u = np.asarray(u, dtype=np.float64)
    rms = np.sqrt(np.mean(u * u))
    t = np.zeros((H, Wd, 2))
    t[:nelx + 1, :nely + 1] = (u / rms if rms > 0 else u).reshape(nelx + 1, nely + 1, 2)
    return t


def prediction(nelx, nely, out, free):
    """Network output as a DOF vector (zero on fixed DOFs)."""
    u = out[:nelx + 1, :nely + 1, :2].reshape(-1).copy()
    u[~np.asarray(free, bool)] = 0.0
    return u


# --- Galerkin start on span{u_hat, u_prev} --------------------------------

def galerkin_start(K, f, uh, up):
    """Minimiser of the energy 1/2 u.K u - f.u over u = a uh + b up (K the
    free-DOF operator as anything supporting @).  Singular or one-sided
    cases fall back to the better one-vector fit."""
    Kh, Kp = K @ uh, K @ up
    A11, A12, A22 = uh @ Kh, uh @ Kp, up @ Kp
    r1, r2 = uh @ f, up @ f
    det = A11 * A22 - A12 * A12
    if A11 > 0 and A22 > 0 and det > 1e-12 * A11 * A22:
        a = (r1 * A22 - r2 * A12) / det
        b = (A11 * r2 - A12 * r1) / det
        return a * uh + b * up
    cands = []
    if A11 > 0:
        cands.append((-(r1 * r1) / (2 * A11), (r1 / A11) * uh))
    if A22 > 0:
        cands.append((-(r2 * r2) / (2 * A22), (r2 / A22) * up))
    if not cands:
        return np.zeros_like(f)
    return min(cands, key=lambda c: c[0])[1]


# --- the 3D image ([ix][iz][iy], node iy + (nely + 1) (iz + (nelz + 1) ix)) --

def image_shape3(nelx, nely, nelz):
    p8 = lambda n: (n + 1 + 7) // 8 * 8
    return (p8(nelx), p8(nelz), p8(nely))


def features3(nelx, nely, nelz, xtilde, f):
    """Input image of the 3D network: mean filtered density of the (1 to 8)
    elements around each node, and the nodal load (three components)."""
    D, H, Wd = image_shape3(nelx, nely, nelz)
    img = np.zeros((D, H, Wd, 4))
    # element e = iy + nely (iz + nelz ix)  ->  [ix, iz, iy]
    xe = np.asarray(xtilde, dtype=np.float64).reshape(nelx, nelz, nely)
    s = np.zeros((nelx + 1, nelz + 1, nely + 1))
    c = np.zeros((nelx + 1, nelz + 1, nely + 1))
    for a in (0, 1):
        for b in (0, 1):
            for d in (0, 1):
                s[a:a + nelx, b:b + nelz, d:d + nely] += xe
                c[a:a + nelx, b:b + nelz, d:d + nely] += 1.0
    img[:nelx + 1, :nelz + 1, :nely + 1, 0] = s / c
    fn = np.asarray(f, dtype=np.float64).reshape(nelx + 1, nelz + 1, nely + 1, 3)
    img[:nelx + 1, :nelz + 1, :nely + 1, 1:4] = fn
    return img


def node_mask3(nelx, nely, nelz):
    mk = np.zeros(image_shape3(nelx, nely, nelz))
    mk[:nelx + 1, :nelz + 1, :nely + 1] = 1.0
    return mk


def target3(nelx, nely, nelz, u):
    """u normalised by its RMS over the real DOFs, as a 3D image."""
    u = np.asarray(u, dtype=np.float64)
    rms = np.sqrt(np.mean(u * u))
    t = np.zeros(image_shape3(nelx, nely, nelz) + (3,))
    t[:nelx + 1, :nelz + 1, :nely + 1] = (u / rms if rms > 0 else u).reshape(nelx + 1, nelz + 1, nely + 1, 3)
    return t


def prediction3(nelx, nely, nelz, out, free):
    """3D network output as a DOF vector (zero on fixed DOFs)."""
    u = out[:nelx + 1, :nelz + 1, :nely + 1, :3].reshape(-1).copy()
    u[~np.asarray(free, bool)] = 0.0
    return u
