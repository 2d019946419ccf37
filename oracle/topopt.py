"""One redesign iteration and the whole optimisation loop (oracle).
Test infrastructure only.

Order of operations per iteration (blocks RL.1-RL.4 of both codes):
  filter -> physical density (projection, eta* by Newton if ft = 3) -> change
  -> SIMP moduli and assembly of K^(s) -> state solve -> sensitivities and
  compliance -> back-filter of dc and dV -> OC with bisection -> continuation.
The loop runs a fixed number of iterations (the ch < 1e-6 stop of the codes
is logged, not used, so that runs of equal length can be compared).
"""
import numpy as np

from . import mesh as _mesh
from . import element, sparse, filt, projection, solve, sensitivity, oc, continuation


class Problem:
    def __init__(self, mesh, f, fixed, volfrac, penal, rmin, ft=1, bc="D", eta=0.5,
                 beta=1.0, move=0.2, E0=1.0, Emin=1e-9, nu=0.3, passive=None,
                 penal_sched=None, beta_sched=None, target=None):
        self.mesh, self.f, self.fixed = mesh, np.asarray(f, float), np.asarray(fixed)
        self.free = _mesh.free_dofs(mesh, fixed)
        self.volfrac, self.penal0, self.rmin = volfrac, penal, rmin
        self.ft, self.bc, self.eta0, self.beta0, self.move = ft, bc, eta, beta, move
        self.E0, self.Emin, self.nu = E0, Emin, nu
        self.penal_sched, self.beta_sched, self.target = penal_sched, beta_sched, target
        self.cmat = mesh.cmat()
        self.ke_full = element.element_matrix(mesh.dim, nu)
        self.ke_lower = element.lower_vector(self.ke_full)
        self.ir = sparse.reduced_index_set(self.cmat)
        self.row_ptr, self.col_idx, self.perm, self.seg_ptr = sparse.csr_pattern(self.ir, mesh.n)
        self.filter = filt.Filter(mesh, rmin, bc)
        self.x0, self.dv, self.act = _mesh.initial_design(mesh, volfrac, passive)
        self.code = np.zeros(mesh.m, np.int64) if passive is None else np.asarray(passive)


class State:
    def __init__(self, prob):
        self.x = prob.x0.copy()
        self.xphys = prob.x0.copy()
        self.xold = np.ones(prob.mesh.m)
        self.u = np.zeros(prob.mesh.n)
        self.penal, self.beta, self.eta = prob.penal0, prob.beta0, prob.eta0
        self.loop = 0


def step(prob, st, solver="auto", rtol=1e-8, oc_method="bisect"):
    """One redesign iteration; mutates st and returns a stats dict.
    oc_method: 'bisect' (block RL.4), 'pd' (the primal-dual update of
    Appendix A) or 'filtered' (the bisection that filters and projects each
    candidate, Sec. 3.2, with this iteration's eta and beta)."""
    st.loop += 1
    m = prob.mesh.m
    xt = prob.filter.forward(st.x)
    xphys, dp, st.eta, n_newton, newton_ok = projection.physical_density(
        xt, st.x, prob.act, prob.ft, st.eta, st.beta, prob.volfrac, prob.target)
    ch = projection.change(xphys, st.xold)
    st.xold = xphys.copy()
    st.xphys = xphys
    kval = sparse.assemble(xphys, prob.ke_lower, prob.perm, prob.seg_ptr,
                           st.penal, prob.E0, prob.Emin)
    if solver == "auto":
        solver = "dense" if prob.mesh.n <= 3000 else "pcg"
    Kfull = sparse.lower_to_full(prob.row_ptr, prob.col_idx, kval, prob.mesh.n)
    if solver == "dense":
        st.u = solve.solve_dense(Kfull.toarray(), prob.f, prob.free)
        cg_it = 0
    else:
        st.u, cg_it, _, _ = solve.solve_pcg(Kfull, prob.f, prob.free, st.u, rtol)
    res = solve.true_residual(Kfull, prob.f, prob.free, st.u)
    c = sensitivity.compliance(prob.f, st.u)
    dc, _ = sensitivity.sensitivity(xphys, st.u, prob.cmat, prob.ke_full, prob.act,
                                    st.penal, prob.E0, prob.Emin)
    dcf = prob.filter.adjoint(dc, dp)
    dv0 = prob.filter.adjoint(prob.dv, dp)
    if oc_method == "pd":
        st.x, pd = oc.oc_update_pd(st.x, dcf, dv0, prob.act, prob.volfrac, prob.move)
        ocs = dict(n_bs=pd["n_it"], lmid=pd["lm"])
    elif oc_method == "filtered":
        st.x, ocs = oc.oc_update_filtered(st.x, dcf, dv0, prob.code, prob.volfrac, prob.move, prob.filter,
                                          prob.ft, st.eta, st.beta)
    else:
        st.x, ocs = oc.oc_update(st.x, dcf, dv0, prob.act, prob.volfrac, prob.move)
    st.penal = continuation.cnt(st.penal, prob.penal_sched, st.loop)
    st.beta = continuation.cnt(st.beta, prob.beta_sched, st.loop)
    return dict(loop=st.loop, c=c, vol=float(np.mean(xphys)), ch=ch, eta=st.eta,
                n_newton=n_newton, newton_ok=newton_ok, n_bs=ocs["n_bs"],
                lmid=ocs["lmid"], cg_it=cg_it, residual=res,
                penal=st.penal, beta=st.beta)


def run(prob, iterations, solver="auto", rtol=1e-8):
    st = State(prob)
    log = [step(prob, st, solver, rtol) for _ in range(iterations)]
    return st, log


def problem_from_config(cfg):
    """Build the oracle's Problem from a workloads.Config (parameters only)."""
    passive = None
    if cfg.nelz:
        M = _mesh.Mesh(cfg.nelx, cfg.nely, cfg.nelz)
        f, fixed = _mesh.cantilever3d(M, cfg.load)
    else:
        M = _mesh.Mesh(cfg.nelx, cfg.nely)
        if cfg.kind == "mbb":
            f, fixed = _mesh.mbb(M, cfg.load)
        elif cfg.kind == "frame":
            f, fixed, passive = _mesh.frame(M, -1.0 if cfg.load == 0 else 1.0)
        else:
            f, fixed = _mesh.cantilever2d(M, cfg.load)
    return Problem(M, f, fixed, cfg.volfrac, cfg.penal, cfg.rmin, ft=cfg.ft, bc=cfg.bc,
                   eta=cfg.eta, beta=cfg.beta, move=cfg.move, E0=cfg.E0, Emin=cfg.Emin,
                   nu=cfg.nu, passive=passive, penal_sched=cfg.penal_sched, beta_sched=cfg.beta_sched)
