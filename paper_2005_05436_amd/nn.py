"""The learned warm start around the C ABI: the network's workspace and
parameters, training on the optimiser's own (design, displacement) pairs,
and the warm-started solve.  All arithmetic runs in libtopt's kernels."""
import torch

from . import _lib as L

# (c_in, c_out) of the 15 layers, in the library's parameter order (2D and 3D)
LAYERS = [(3, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 64),
          (64, 64), (64, 32), (32, 32), (32, 16), (16, 16), (16, 16), (16, 2)]
LAYERS3 = [(4, 8), (8, 8), (8, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 32),
           (32, 32), (32, 16), (16, 16), (16, 8), (8, 8), (8, 8), (8, 3)]
LEVELS = [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0]


def layers(dim):
    return LAYERS if dim == 2 else LAYERS3


class Net:
    """A U-Net bound to one plan (mesh size and free DOFs), 2D or 3D."""

    def __init__(self, plan):
        self.plan = plan
        self.dim = plan.dim
        self.ws_bytes, self.n_params = L.to_nn_query(plan.dim, plan.nelx, plan.nely, plan.nelz)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=plan.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) & ~255
        self.handle = L.to_nn_create(plan.handle, self.ws_ptr, self.ws_bytes)
        from .driver import track
        track("net", self)
        self.loss = torch.zeros(1, dtype=torch.float64, device=plan.device)
        p8 = lambda n: (n + 1 + 7) // 8 * 8
        if self.dim == 2:
            self.shape = (p8(plan.nelx), p8(plan.nely))
        else:
            self.shape = (p8(plan.nelx), p8(plan.nelz), p8(plan.nely))
        self.H, self.W = self.shape[-2], self.shape[-1]

    def close(self):
        if getattr(self, "handle", None):
            L.to_nn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p = torch.as_tensor(params, dtype=torch.float32).to(self.plan.device).contiguous()
        assert p.numel() == self.n_params
        L.to_nn_set_params(self.handle, p)

    def npix(self, level=0):
        n = 1
        for e in self.shape:
            n *= e >> level
        return n

    def get(self, what):
        n = self.npix() * 16 if what == L.TO_NN_OUTPUT else self.n_params
        out = torch.empty(n, dtype=torch.float32, device=self.plan.device)
        L.to_nn_get(self.handle, what, out)
        return out

    def layer(self, i, preskip=False):
        """bfloat16 output (or pre-skip activation) of layer i as float32,
        [(planes,) rows, cols, c_out padded]."""
        lev = LEVELS[i]
        cp = (layers(self.dim)[i][1] + 15) // 16 * 16
        n = self.npix(lev) * cp
        raw = torch.empty(n, dtype=torch.int16, device=self.plan.device)
        L.to_nn_get(self.handle, (L.TO_NN_PRESKIP if preskip else L.TO_NN_ACT) + i, raw)
        return (raw.to(torch.int32) << 16).view(torch.float32).reshape(*[e >> lev for e in self.shape], cp)

    def params(self):
        return self.get(L.TO_NN_PARAMS)

    def forward(self, dtype, xtilde, f, uhat=None):
        L.to_nn_forward(self.handle, dtype, xtilde, f, uhat)

    def backward(self, u):
        L.to_nn_backward(self.handle, u, self.loss)

    def train_step(self, dtype, xtilde, f, u, lr):
        L.to_nn_train_step(self.handle, dtype, xtilde, f, u, lr, self.loss)
