"""Plan and optimisation-loop objects around the C ABI.  PyTorch supplies
device memory and the stream; every step of the method runs in libtopt's
kernels (to_step and the single-step entry points)."""
import atexit
import ctypes as C
import math
import weakref

import numpy as np
import torch

from . import _lib as L
from . import problems


# Library objects still open when the interpreter exits are closed by an exit
# handler, while the HIP runtime is still up (destructors that run later, at
# module teardown, would call into a runtime that is already shut down).
_LIVE = {"batch": weakref.WeakSet(), "net": weakref.WeakSet(), "plan": weakref.WeakSet()}


def track(kind, obj):
    _LIVE[kind].add(obj)


@atexit.register
def _close_all():
    for kind in ("batch", "net", "plan"):
        for obj in list(_LIVE[kind]):
            try:
                obj.close()
            except Exception:
                pass


def _dev():
    if not torch.cuda.is_available():
        raise RuntimeError("libtopt needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch.device("cuda", torch.cuda.current_device())


def _struct_tensor(ctype, device):
    return torch.zeros(C.sizeof(ctype), dtype=torch.uint8, device=device)


def read_struct(t, ctype):
    """Copies a device stats struct to the host (synchronising)."""
    raw = t.cpu().numpy().tobytes()
    return ctype.from_buffer_copy(raw)


def struct_dict(s):
    return {k: getattr(s, k) for k, _ in s._fields_ if k != "pad"}


class Plan:
    """Owns the plan header and its device workspace."""

    def __init__(self, dim, nelx, nely, nelz=1, rmin=2.0, bc="D", fixed=(), passive=None,
                 E0=1.0, Emin=1e-9, nu=0.3, stream=None):
        self.device = _dev()
        self.fixed = np.ascontiguousarray(np.asarray(fixed, dtype=np.int32))
        self.passive = None if passive is None else np.ascontiguousarray(np.asarray(passive, dtype=np.uint8))
        self.desc = L.MeshDesc(dim, nelx, nely, nelz if dim == 3 else 1, E0, Emin, nu, rmin, bc.encode(),
                               L.ptr(self.passive), L.ptr(self.fixed), len(self.fixed))
        self.ws_bytes = L.to_plan_query(self.desc)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.handle = L.to_plan_create(self.desc, self.ws_ptr, self.ws_bytes, stream)
        track("plan", self)
        self.info = L.to_plan_get_info(self.handle)
        self.dim, self.nelx, self.nely, self.nelz = dim, nelx, nely, nelz if dim == 3 else 1

    def close(self):
        if getattr(self, "handle", None):
            L.to_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def export(self, what):
        I = self.info
        shapes = {L.TO_X_PAIRS: (np.int32, (I.n_pairs, 2)), L.TO_X_PERM: (np.int32, (I.n_pairs,)),
                  L.TO_X_SEGPTR: (np.int32, (I.nnz_lower + 1,)), L.TO_X_ROWPTR: (np.int32, (I.n + 1,)),
                  L.TO_X_COLIDX: (np.int32, (I.nnz_lower,)), L.TO_X_HS: (np.float64, (I.m,)),
                  L.TO_X_KE: (np.float64, (I.dtilde,)), L.TO_X_FREE: (np.uint8, (I.n,)),
                  L.TO_X_KERNEL: (np.float64, ((2 * I.filter_radius + 1) ** I.dim,))}
        dt, shape = shapes[what]
        out = np.empty(shape, dtype=dt)
        return L.to_plan_export(self.handle, what, out)


def plan_for_config(cfg, passive=None):
    """(plan, load vector, passive codes); the problem's own passive set
    (the frame) unless one is given."""
    f, fixed, own = problems.from_config(cfg)
    if passive is None:
        passive = own
    p = Plan(cfg.dim, cfg.nelx, cfg.nely, cfg.nelz or 1, cfg.rmin, cfg.bc, fixed, passive,
             cfg.E0, cfg.Emin, cfg.nu)
    return p, f, passive


def _sched(s):
    if s is None:
        return L.Sched(0, 1, 0.0, 0.0, 0, 0)
    istart, maxpar, isteps, delta, mode = s
    return L.Sched(istart, isteps, maxpar, delta, 1 if mode == "mul" else 0, 1)


class TopOpt:
    """The redesign loop on the GPU: state buffers + to_step."""

    def __init__(self, cfg, op=L.TO_OP_ASSEMBLED, rtol=1e-8, inner_rtol=0.1, maxit=200000,
                 precision=None, passive=None, solve_precision=L.TO_SOLVE_AUTO, grid_blocks=0, autotune=False,
                 precond=L.TO_PREC_JACOBI, pae=None, oc=L.TO_OC_BISECT, budget=0):
        self.cfg = cfg
        self.plan, f, passive = plan_for_config(cfg, passive)
        dev = self.plan.device
        I = self.plan.info
        prec = precision or cfg.precision
        self.dtype = L.TO_F64 if prec == "f64" else L.TO_F32
        tdt = torch.float64 if self.dtype == L.TO_F64 else torch.float32
        m, n = I.m, I.n
        mk = lambda: torch.zeros(m, dtype=tdt, device=dev)
        self.x, self.xtilde, self.xphys, self.xphys_old = mk(), mk(), mk(), mk()
        self.dprj, self.dc, self.dcf, self.dv, self.dv0 = mk(), mk(), mk(), mk(), mk()
        self.u = torch.zeros(n, dtype=torch.float64, device=dev)
        # block PRE.6 on the device: x, xphys, xphys_old = 1, dv, u = 0
        L.to_init_state(self.plan.handle, self.dtype, cfg.volfrac, self.x, self.xphys, self.xphys_old, self.dv,
                        self.u)
        self.kval = torch.zeros(I.nnz_lower, dtype=tdt, device=dev)
        self.f = torch.as_tensor(f, dtype=torch.float64).to(dev)
        self.eta = torch.tensor([cfg.eta], dtype=torch.float64, device=dev)
        self.c = torch.zeros(1, dtype=torch.float64, device=dev)
        self.pst = _struct_tensor(L.ProjectStats, dev)
        self.sst = _struct_tensor(L.SolveStats, dev)
        self.ost = _struct_tensor(L.OcStats, dev)
        self.state = L.StepState(*[L.ptr(t) for t in (self.x, self.xtilde, self.xphys, self.xphys_old,
                                                      self.dprj, self.dc, self.dcf, self.dv, self.dv0,
                                                      self.kval, self.u, self.f, self.eta, self.c,
                                                      self.pst, self.sst, self.ost)],
                                 cfg.penal, cfg.beta, 0, 0)
        self.params = L.StepParams(cfg.volfrac, cfg.move, cfg.ft, oc, math.nan, _sched(cfg.penal_sched),
                                   _sched(cfg.beta_sched),
                                   L.SolveOpts(rtol, inner_rtol, maxit, op, solve_precision, 0, grid_blocks,
                                               precond, budget))
        if autotune:
            self.tuning = L.to_plan_autotune(self.plan.handle, self.dtype, self.kval if op != L.TO_OP_MATFREE else None)
        self.pae = None
        if pae is not None:
            self.enable_pae(**pae)

    def enable_pae(self, mr=4, q=4, q0=20, alpha=0.9, xi=1.0):
        """Periodic Anderson extrapolation of the OC iteration from loop q0 on
        (Section 3.3; the defaults are the paper's m_r, q, alpha and a full
        step on the extrapolated iterations)."""
        self.pae = L.PaeParams(mr, q, q0, 0, alpha, xi)
        nbytes = L.to_pae_query(self.plan.handle, self.pae)
        dev = self.x.device
        self.pae_ws = torch.zeros((nbytes + 7) // 8, dtype=torch.float64, device=dev)
        self.pae_gamma = torch.zeros(8, dtype=torch.float64, device=dev)
        self.x_pre = torch.empty_like(self.x)

    def _pae_pre(self, stream):
        if self.pae is not None:
            with torch.cuda.stream(stream or torch.cuda.current_stream()):
                self.x_pre.copy_(self.x)

    def _pae_post(self, stream):
        if self.pae is not None:
            L.to_pae_step(self.plan.handle, self.dtype, self.x, self.x_pre, self.state.loop, self.pae, self.pae_ws,
                          self.pae_gamma, stream)

    @property
    def loop(self):
        return self.state.loop

    def step(self, stream=None):
        """Enqueues one redesign iteration (no host synchronisation); with
        PAE on, the extrapolation follows the OC update."""
        self._pae_pre(stream)
        L.to_step(self.plan.handle, self.dtype, self.state, self.params, stream)
        self._pae_post(stream)

    def step_stages(self, net=None, train_lr=None, stream=None, solve_events=None):
        """One redesign iteration through the single-stage entry points (the
        sequence to_step runs).  With a network: its prediction from the
        physical density and the load, combined with the previous displacement
        by the Galerkin start (to_warm_start), seeds the PCG; with train_lr the
        network then takes one Adam step on the converged displacement.
        solve_events: two torch events recorded before the network's
        prediction (or the solve) and after the solve."""
        h, dt, st, cfg = self.plan.handle, self.dtype, self.state, self.cfg
        self._pae_pre(stream)
        L.to_filter(h, dt, L.TO_FILTER_FWD, self.x, None, None, self.xtilde, None, stream)
        L.to_project(h, dt, cfg.ft, self.xtilde, self.x, self.xphys, self.dprj, st.beta, self.eta, cfg.volfrac,
                     self.xphys_old, self.pst, stream)
        if self.params.solve.op != L.TO_OP_MATFREE:
            L.to_assemble(h, dt, self.xphys, st.penal, self.kval, stream)
        sq = stream or torch.cuda.current_stream()
        if solve_events is not None:
            solve_events[0].record(sq)
        if net is not None:
            if not hasattr(self, "uhat"):
                self.uhat = torch.zeros_like(self.u)
                self.wcoef = torch.zeros(4, dtype=torch.float64, device=self.u.device)
            net.forward(dt, self.xphys, self.f, self.uhat)
            L.to_warm_start(h, dt, self.xphys, st.penal, self.f, self.uhat, self.u, self.u, self.wcoef, stream)
        L.to_solve(h, dt, self.kval, self.xphys, st.penal, self.f, self.u, self.params.solve, self.sst, stream)
        if solve_events is not None:
            solve_events[1].record(sq)
        if net is not None and train_lr:
            net.train_step(dt, self.xphys, self.f, self.u, train_lr)
        L.to_sensitivity(h, dt, self.xphys, self.u, self.f, st.penal, self.dc, self.c, stream)
        L.to_filter(h, dt, L.TO_FILTER_ADJ2, self.dc, self.dv, self.dprj, self.dcf, self.dv0, stream)
        oc = self.params.oc
        if oc == L.TO_OC_FILTERED:
            L.to_oc_update_filtered(h, dt, cfg.ft, self.x, self.dcf, self.dv0, cfg.volfrac, cfg.move, st.beta,
                                    self.eta, self.ost, stream)
        elif oc == L.TO_OC_PD:
            L.to_oc_update_pd(h, dt, self.x, self.dcf, self.dv0, cfg.volfrac, cfg.move, self.ost, stream)
        else:
            L.to_oc_update(h, dt, self.x, self.dcf, self.dv0, cfg.volfrac, cfg.move, self.ost, stream)
        self.xphys_old.copy_(self.xphys)
        st.loop += 1
        self._pae_post(stream)
        st.penal = L.to_continuation(st.penal, self.params.penal_sched, st.loop)
        st.beta = L.to_continuation(st.beta, self.params.beta_sched, st.loop)

    def stats(self):
        """Synchronising read of the last iteration's device statistics."""
        p = read_struct(self.pst, L.ProjectStats)
        s = read_struct(self.sst, L.SolveStats)
        o = read_struct(self.ost, L.OcStats)
        return dict(loop=self.state.loop, c=float(self.c.item()), vol=p.vol, ch=p.ch, eta=p.eta,
                    n_newton=p.n_newton, newton_ok=bool(p.converged), n_bs=o.n_bs, lmid=o.lmid,
                    oc_passes=o.passes, cg_it=s.iterations, residual=s.residual, solve_ok=bool(s.converged),
                    fallback=s.fallback, outer=s.outer, penal=self.state.penal, beta=self.state.beta)

    def run(self, iterations, log=False):
        out = []
        for _ in range(iterations):
            self.step()
            if log:
                out.append(self.stats())
        return out


class Batch:
    """Many independent designs advanced together (to_step_batched): one
    persistent launch per projection / solve / OC stage for the whole batch,
    optionally replayed from a HIP graph."""

    def __init__(self, cfgs, op=L.TO_OP_ASSEMBLED, rtol=1e-8, precision=None, solve_precision=L.TO_SOLVE_AUTO,
                 autotune=True, maxit=200000, oc=L.TO_OC_BISECT, precond=L.TO_PREC_JACOBI, budget=0):
        self.runs = [TopOpt(c, op=op, rtol=rtol, precision=precision, solve_precision=solve_precision, maxit=maxit,
                            oc=oc, precond=precond, budget=budget) for c in cfgs]
        dts = {g.dtype for g in self.runs}
        if len(dts) != 1:
            raise ValueError("all designs of a batch need the same precision")
        self.dtype = dts.pop()
        n = len(self.runs)
        self.states = (L.StepState * n)(*[g.state for g in self.runs])
        self.params = (L.StepParams * n)(*[g.params for g in self.runs])
        for i, g in enumerate(self.runs):          # the array is the live host state from now on
            g.state = self.states[i]
            g.params = self.params[i]
        self.ws_bytes = L.to_batch_query(n)
        dev = self.runs[0].plan.device
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        self.ws_ptr = (self.ws.data_ptr() + 255) & ~255
        self.handle = L.to_batch_create([g.plan.handle for g in self.runs], self.dtype, self.states, self.params,
                                        autotune, self.ws_ptr, self.ws_bytes)
        track("batch", self)

    def step(self, use_graph=False, stream=None):
        L.to_step_batched(self.handle, self.states, self.params, use_graph, stream)

    def info(self):
        return L.to_batch_get_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            L.to_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
