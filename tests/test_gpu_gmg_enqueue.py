"""The multigrid-preconditioned solve in its enqueue-only form (a fixed
budget of outer iterations, each predicated on the device stop flag, no host
synchronisation): the same iterates as the host-checked form, recorded into a
caller's HIP graph and replayed, and inside ragged batches against the same
designs run one by one.  The solve is eq. (5); the true residual 1e-8 and the
oracle's compliance decide correctness."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W
from oracle import element as oel
from oracle import mesh as omesh
from oracle import solve as osolve
from oracle import sparse as osp


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_05436_amd import _lib
    _lib.load()


def _problem(dims, seed):
    from paper_2005_05436_amd import problems
    from paper_2005_05436_amd.driver import Plan
    if len(dims) == 2:
        M = omesh.Mesh(*dims)
        f, fixed = omesh.mbb(M, 0)
        P = Plan(2, dims[0], dims[1], 1, 2.0, "D", fixed)
    else:
        f, fixed = problems.cantilever3d(*dims)
        M = omesh.Mesh(*dims)
        P = Plan(3, dims[0], dims[1], dims[2], 1.5, "N", fixed)
    x = W.design_field(M.m, seed, 0.05, 1.0)
    return M, P, np.asarray(f, float), np.asarray(fixed), x


def _oracle_solution(M, f, fixed, x):
    ke = oel.element_matrix(M.dim, 0.3)
    free = np.ones(M.n, bool)
    free[fixed] = False
    ir = osp.reduced_index_set(M.cmat())
    rp, ci, perm, seg = osp.csr_pattern(ir, M.n)
    kl = osp.assemble(x, oel.lower_vector(ke), perm, seg, 3.0, 1.0, 1e-9)
    K = osp.lower_to_full(rp, ci, kl, M.n)
    # a sparse direct solve of the sliced system (the paper's own kind of solver)
    import scipy.sparse.linalg as spla
    u = np.zeros(M.n)
    u[free] = spla.spsolve(K[free][:, free].tocsc(), f[free])
    return u, K, free


def _solve(P, x, f, budget, u0=None):
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import read_struct
    u = torch.zeros(P.info.n, dtype=torch.float64, device="cuda") if u0 is None else u0.clone()
    st = torch.zeros(40, dtype=torch.uint8, device="cuda")
    opts = L.SolveOpts(1e-8, 0.1, 2000, L.TO_OP_MATFREE, L.TO_SOLVE_AUTO, 0, 0, L.TO_PREC_GMG, budget)
    L.to_solve(P.handle, L.TO_F64, None, x, 3.0, f, u, opts, st)
    torch.cuda.synchronize()
    return u, read_struct(st, L.SolveStats)


@pytest.mark.parametrize("dims,seed", [((120, 40), 1), ((61, 23), 2), ((12, 6, 6), 3), ((13, 7, 5), 4)])
def test_budget_matches_host_checked(dims, seed):
    """Budget mode takes exactly the host-checked mode's iterations (same
    kernels, predicated): bit-identical u, equal counts; the true residual
    and compliance against the oracle; a budget too small ends with
    converged = 0 and the next call from that u finishes the solve."""
    M, P, f, fixed, x = _problem(dims, seed)
    xd = torch.as_tensor(x).cuda()
    fd = torch.as_tensor(f).cuda()
    u_h, s_h = _solve(P, xd, fd, 0)
    u_b, s_b = _solve(P, xd, fd, 64)
    print(f"{dims}: host-checked {s_h.iterations} it, budget 64: {s_b.iterations} it, "
          f"residual {s_b.residual:.2e}", flush=True)
    assert s_h.converged and s_b.converged
    assert s_b.iterations == s_h.iterations
    np.testing.assert_array_equal(u_b.cpu().numpy(), u_h.cpu().numpy())
    u_ref, K, free = _oracle_solution(M, f, fixed, x)
    got = u_b.cpu().numpy()
    assert osolve.true_residual(K, f, free, got) <= 1e-8
    assert abs(f @ got - f @ u_ref) <= 1e-7 * abs(f @ u_ref)
    # too small a budget: not converged, and a second call continues
    u_s, s_s = _solve(P, xd, fd, 8)
    assert not s_s.converged and s_s.iterations == 8
    u_c, s_c = _solve(P, xd, fd, 64, u0=u_s)
    assert s_c.converged and osolve.true_residual(K, f, free, u_c.cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("dims", [(96, 32), (12, 6, 6)])
def test_budget_solve_captured_in_a_graph(dims):
    """to_solve (multigrid, budget 48) recorded into a HIP graph through the
    caller's stream capture, replayed four times with eager work and
    synchronisation between the replays: each replay gives the eager result
    bit for bit."""
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import read_struct
    M, P, f, fixed, x = _problem(dims, 5)
    xd = torch.as_tensor(x).cuda()
    fd = torch.as_tensor(f).cuda()
    u_e, s_e = _solve(P, xd, fd, 48)
    assert s_e.converged
    u = torch.zeros(P.info.n, dtype=torch.float64, device="cuda")
    st = torch.zeros(40, dtype=torch.uint8, device="cuda")
    opts = L.SolveOpts(1e-8, 0.1, 2000, L.TO_OP_MATFREE, L.TO_SOLVE_AUTO, 0, 0, L.TO_PREC_GMG, 48)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):     # one call before capture, on the capture stream
        L.to_solve(P.handle, L.TO_F64, None, xd, 3.0, fd, u, opts, st)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        L.to_solve(P.handle, L.TO_F64, None, xd, 3.0, fd, u, opts, st)
    for rep in range(4):
        u.zero_()                      # eager work between the replays
        st.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        s = read_struct(st, L.SolveStats)
        print(f"{dims} replay {rep}: {s.iterations} it, residual {s.residual:.2e}", flush=True)
        assert s.converged and s.iterations == s_e.iterations
        np.testing.assert_array_equal(u.cpu().numpy(), u_e.cpu().numpy())
    with pytest.raises(L.ToError):     # the host-checked form refuses capture
        g2 = torch.cuda.CUDAGraph()
        bad = L.SolveOpts(1e-8, 0.1, 2000, L.TO_OP_MATFREE, L.TO_SOLVE_AUTO, 0, 0, L.TO_PREC_GMG, 0)
        try:
            with torch.cuda.graph(g2, stream=side):
                L.to_solve(P.handle, L.TO_F64, None, xd, 3.0, fd, u, bad, st)
        finally:
            torch.cuda.synchronize()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_with_multigrid_matches_single_runs(use_graph):
    """Six ragged designs (MBB and cantilever, 100..400 elements wide) in one
    batch with multigrid solves (budget 48), eager and graph-replayed, over 4
    redesign iterations: compliance, design and solve statistics equal to the
    same designs advanced one by one with to_step."""
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Batch, TopOpt
    cfgs = W.batch_configs(6, seed=3)
    B = Batch(cfgs, autotune=False, precond=L.TO_PREC_GMG, budget=48, op=L.TO_OP_MATFREE)
    singles = [TopOpt(c, precond=L.TO_PREC_GMG, budget=48, op=L.TO_OP_MATFREE) for c in cfgs]
    for it in range(4):
        B.step(use_graph=use_graph)
        for g in singles:
            g.step()
        torch.cuda.synchronize()
        for i, (gb, gs) in enumerate(zip(B.runs, singles)):
            sb, ss = gb.stats(), gs.stats()
            assert sb["solve_ok"] and ss["solve_ok"], (it, i, sb, ss)
            assert sb["cg_it"] == ss["cg_it"] and sb["n_bs"] == ss["n_bs"]
            assert sb["c"] == ss["c"], (it, i, sb["c"], ss["c"])
            np.testing.assert_array_equal(gb.x.cpu().numpy(), gs.x.cpu().numpy())
        print(f"iteration {it + 1}: cg {[g.stats()['cg_it'] for g in B.runs]}", flush=True)
    with pytest.raises(L.ToError):
        Batch(cfgs[:2], autotune=False, precond=L.TO_PREC_GMG, budget=0, op=L.TO_OP_MATFREE)
