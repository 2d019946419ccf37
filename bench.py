"""Benchmark of the SIMP redesign iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--precision f32|f64] [--op assembled|matfree] [--no-cpu]

A step is one redesign iteration through the C ABI: filter, projection with
the volume-preserving threshold, assembly, Jacobi-PCG state solve,
sensitivities, back-filter, OC update, continuation.  The default workload is
the MBB half beam at 1200 x 400 (480,000 Q4 elements, rmin 40, beta 1 -> 32
and penal 1 -> 3 continuation, FP32 fields with FP64 solve vectors, dot
products and OC sums).  Inputs are synthetic (the paper's own test problem)
and resident in HBM before the timed region.

Printed: one JSON line.  value = elements per second through the non-solve
path (filter + projection + assembly + sensitivity + back-filter + OC),
m * K / (sum of those stage times); to_iters_per_s = whole iterations per
second including the Jacobi-preconditioned CG solve (the plain CG of the
metric); roofline = the persistent PCG kernel.  Also in the line: the same
steps with the multigrid-preconditioned CG (gmg, to_iters_per_s_gmg), with
the learned warm start for both solvers (nn_warm_start), the 64-design
ragged batch (batch64), test T2 of Table 4 with and without the periodic
Anderson extrapolation (pae_t2), the 900 x 900 frame problem (frame900), the
96 x 48 x 48 3D cantilever with three solvers (cantilever3d), the non-solve
stages on a 16 times larger mesh (stage_scaling) and the FP64 oracle on the
host (cpu_baseline).
Stage times come from HIP events recorded on the stream the kernels run on.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "elem/s assembly+filter+OC; TO iters/s plain vs NN-warm-start CG @rtol 1e-8"
HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
STAGES = ["filter", "project", "assemble", "solve", "sensitivity", "backfilter", "oc"]
NON_SOLVE = [s for s in STAGES if s != "solve"]


def workloads_by_name():
    import workloads as W
    out = {c.name: c for c in W.C1.values()}
    out[W.C0.name] = W.C0
    out[W.C2.name] = W.C2
    return out


def solve_path(cfg, op, solve):
    """Which solve kernel to_solve runs: (operator, vector precision)."""
    f32 = cfg.precision == "f32"
    mixed = f32 and solve == "mixed"
    assembled = op == "assembled" and (not f32 or mixed)
    return ("assembled" if assembled else "matfree"), ("f32" if mixed else "f64")


FP32_PEAK = 157.3e12          # flop/s, MI355X FP32 (matrix cores; also the vector rate with packed instructions)


def filter_flops(rmin):
    """2D cone filter work per element: (useful flops = 2 per non-zero tap,
    flops the matrix-core kernel issues = 2,048 per v_mfma_f32_16x16x4_f32,
    sum over the tap columns dx of ceil((16 + 2 lim(dx)) / 4) of them per
    16 x 16 outputs, lim(dx) = the largest |dy| with a non-zero weight)."""
    import math
    R = math.ceil(rmin) - 1
    taps, steps = 0, 0
    for dx in range(-R, R + 1):
        lim = -1
        for dy in range(-R, R + 1):
            if rmin - math.sqrt(dx * dx + dy * dy) > 0.0:
                taps += 1
                lim = max(lim, abs(dy))
        if lim >= 0:
            steps += (16 + 2 * lim + 3) // 4
    return 2.0 * taps, steps * 2048.0 / 256.0


def stage_bytes(cfg, info, dt_bytes, op, solve):
    """Algorithmic bytes per launch of each stage: every array the kernel must
    read or write counted once (no credit for caches, no charge for re-reads)."""
    m, n, nnz, npairs = info.m, info.n, info.nnz_lower, info.n_pairs
    F = dt_bytes
    b = {}
    b["filter"] = F * m + F * m + F * m                       # x in, Hs in, xtilde out
    b["project"] = F * m + 2 * F * m + m                      # xtilde in; xphys, dprj out; passive codes
    b["assemble"] = 4 * npairs + 4 * (nnz + 1) + F * nnz + F * m   # perm, seg_ptr, kval out, xphys in
    b["sensitivity"] = 8 * n + F * m * 2 + m + 8 * n          # u gather, xphys in, dc out, codes, f for f.u
    b["backfilter"] = 3 * F * m + F * m + 2 * F * m           # dc, dv, dprj, Hs in; dc~, dv~ out
    b["oc"] = F * m * 3 + m + F * m                           # x, dc~, dv~, codes in; x out
    # one CG iteration of the kernel to_solve runs (vectors in node-major DOF order)
    opk, vp = solve_path(cfg, op, solve)
    V = 4 if vp == "f32" else 8
    mat = (F * nnz + 4 * (n + 1)) if opk == "assembled" else V * m   # K^(s) values + row_ptr | moduli
    phase_a = mat + 2 * V * n + 2 * V * n + n                 # z, p_old in; p_new, q out; free mask
    phase_b = 5 * V * n + 3 * V * n                           # x, p, r, q, dinv in; x, r, z out
    if vp == "f32":
        phase_b += 2 * 4 * n                                  # the iterate u stays FP64
    b["solve_per_iter"] = phase_a + phase_b
    b["solve_kernel"] = {"operator": opk, "vectors": vp}
    return b


def measured_traffic(kernel_key):
    """HBM bytes per CG iteration from the committed counter summary, or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    fn = os.path.join(ROOT, "profiles", "solve_kernel_traffic.json")
    try:
        rec = json.load(open(fn))
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel_key:
        return None
    src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in rec["sources"])
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_cg_iteration"]


def cpu_baseline(cfg, budget_taps=1500):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload: one pass of projection, assembly, sensitivity and OC on the full
    mesh, and one filter application restricted to `budget_taps` of the
    kernel's non-zero taps, scaled to all taps and to the three filter
    applications of an iteration."""
    import numpy as np
    import workloads as W
    from oracle import filt, oc, projection, sensitivity, sparse, topopt
    prob_t0 = time.perf_counter()
    M = topopt._mesh.Mesh(cfg.nelx, cfg.nely)
    C = M.cmat()
    ke = topopt.element.element_matrix(2, cfg.nu)
    kl = topopt.element.lower_vector(ke)
    ir = sparse.reduced_index_set(C)
    row_ptr, col_idx, perm, seg_ptr = sparse.csr_pattern(ir, M.n)
    del ir
    setup_s = time.perf_counter() - prob_t0
    x = W.smooth_design(cfg, 3)
    act = np.ones(M.m, bool)
    t = {}
    # filter: a subset of the taps on the full field
    h, R = filt.kernel(cfg.rmin, 2)
    nz = np.argwhere(h > 0)
    rng = np.random.default_rng(0)
    pick = nz[rng.choice(len(nz), min(budget_taps, len(nz)), replace=False)]
    img = x.reshape(M.shape, order="F")
    out = np.zeros_like(img)
    t0 = time.perf_counter()
    for (a, b) in pick:
        iy, vy = filt._axis_map(M.nely, a - R, cfg.bc)
        ix, vx = filt._axis_map(M.nelx, b - R, cfg.bc)
        out += h[a, b] * img[np.ix_(iy, ix)] * (vy[:, None] & vx[None, :])
    t["filter"] = (time.perf_counter() - t0) * len(nz) / len(pick)
    xt = x
    t0 = time.perf_counter()
    xp, dp, eta, nn, ok = projection.physical_density(xt, x, act, 3, 0.5, 8.0, cfg.volfrac)
    t["project"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    sparse.assemble(xp, kl, perm, seg_ptr, 3.0, 1.0, 1e-9)
    t["assemble"] = time.perf_counter() - t0
    u = W.displacement_field(M.n, 4)
    t0 = time.perf_counter()
    dc, _ = sensitivity.sensitivity(xp, u, C, ke, act, 3.0, 1.0, 1e-9)
    t["sensitivity"] = time.perf_counter() - t0
    dv = np.full(M.m, 1.0 / M.m / cfg.volfrac)
    t0 = time.perf_counter()
    oc.oc_update(x, -np.abs(dc), dv, act, cfg.volfrac, cfg.move)
    t["oc"] = time.perf_counter() - t0
    t["backfilter"] = 2 * t["filter"]
    total = sum(t.values())
    return {"value": M.m / total, "unit": "elem/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 NumPy oracle on {cfg.name}: one pass of projection, assembly, sensitivity "
                       f"and OC on all {M.m} elements; the filter timed on {len(pick)} of its {len(nz)} "
                       f"non-zero taps over the full mesh and scaled to all taps and to 3 applications; "
                       f"numpy element-wise kernels run on one thread"),
            "stage_s": {k: round(v, 4) for k, v in t.items()}, "setup_s": round(setup_s, 2),
            "host_cpus": len(os.sched_getaffinity(0))}


def batch_run(args):
    """The 64-design ragged batch (nelx 100..400, nely = nelx / 2, MBB and
    cantilever loads, FP32 fields): graph-replayed batched iterations against
    the same designs advanced one by one with to_step."""
    import torch
    import workloads as W
    from paper_2005_05436_amd.driver import Batch, TopOpt
    cfgs = W.batch_configs(64, 0)
    m_total = sum(c.m for c in cfgs)
    b = Batch(cfgs, autotune=True)
    b.step(use_graph=True)                       # warm-up: capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        b.step(use_graph=True)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.batch_steps
    info = b.info()
    cg = sum(g.stats()["cg_it"] for g in b.runs)
    del b
    singles = [TopOpt(c) for c in cfgs]
    for g in singles:
        g.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        for g in singles:
            g.step()
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / args.batch_steps
    print(f"[bench] batch64: {1e3 * tb:.1f} ms per batched iteration, {1e3 * ts:.1f} ms one by one",
          file=sys.stderr, flush=True)
    return {"designs": len(cfgs), "elements": m_total, "steps": args.batch_steps,
            "ms_per_batched_step": round(1e3 * tb, 2), "ms_per_step_one_by_one": round(1e3 * ts, 2),
            "speedup": round(ts / tb, 2), "elem_iters_per_s": round(m_total / tb, 1),
            "cg_iterations_last_step": cg, "launch_blocks": {k: info[k] for k in ("project_blocks", "solve_blocks",
                                                                                  "oc_blocks")},
            "graph_captures": info["graph_captures"]}


def solver_run(args, cfg, op, sp, precond, net=None, zero_x0=False):
    """The same redesign iterations (steps warmup+1 .. warmup+K of the run)
    with another solve set-up: the multigrid preconditioner, the network warm
    start, or every solve started from u = 0 instead of the previous
    displacement.  Returns the rate and per-step CG statistics."""
    import torch
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    g = TopOpt(cfg, op=op, solve_precision=sp, autotune=True, precond=precond)
    g.params.solve.zero_x0 = 1 if zero_x0 else 0
    for _ in range(args.warmup):
        g.step_stages(net)
    K = args.steps
    hist = torch.zeros((K, g.sst.numel()), dtype=torch.uint8, device=g.sst.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        g.step_stages(net)
        hist[k].copy_(g.sst, non_blocking=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h = hist.cpu().numpy()
    st = [L.SolveStats.from_buffer_copy(h[k].tobytes()) for k in range(K)]
    its = [s.iterations for s in st]
    return {"to_iters_per_s": round(K / wall, 3), "ms_per_step": round(1e3 * wall / K, 3),
            "cg_iterations_per_step": round(sum(its) / K, 1), "cg_iterations": its,
            "all_converged": bool(all(s.converged for s in st)),
            "max_true_residual": max(s.residual for s in st)}


def train_net(args, cfg, op, sp, precond):
    """The warm-start network trained on the GPU (one Adam step per redesign
    iteration) on a run of the same problem (in-sample; held-out gains are
    measured by the test suite)."""
    import torch
    import workloads as W
    from paper_2005_05436_amd.driver import TopOpt
    from paper_2005_05436_amd.nn import LAYERS, Net
    t0 = time.perf_counter()
    gt = TopOpt(cfg, op=op, solve_precision=sp, autotune=True, precond=precond)
    net = Net(gt.plan)
    net.set_params(W.network_params(LAYERS, 0))
    for _ in range(args.nn_train_steps):
        gt.step_stages(net, train_lr=1e-3)
    torch.cuda.synchronize()
    return net, {"train_steps": args.nn_train_steps, "train_seconds": round(time.perf_counter() - t0, 2),
                 "last_train_loss": round(float(net.loss.item()), 5)}


def pae_run(args):
    """Test T2 of Table 4 (MBB 300 x 100, rmin 8.75, beta 2, volume-
    preserving projection, FP64, multigrid-preconditioned CG) with the
    periodic Anderson extrapolation (m_r = 4, q = 4, from iteration 20,
    alpha = 0.9) until |r|_2 / sqrt(m) < 1e-6 (at most --pae-cap
    iterations), and without it for the same number of iterations."""
    import torch
    import workloads as W
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    cfg = W.PAE_T["T2"]
    out = {"case": "T2", "paper_iterations": {"plain": "2500 (not converged)", "pae": 352}}
    n_pae = None
    for use in (True, False):
        g = TopOpt(cfg, precond=L.TO_PREC_GMG,
                   pae=dict(mr=4, q=4, q0=W.PAE_Q0["T2"], alpha=0.9, xi=1.0) if use else None)
        cap = args.pae_cap if use else n_pae
        ch = torch.zeros(cap, dtype=torch.float64, device=g.x.device)
        pv = g.pst.view(torch.float64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, conv = 0, None
        while it < cap and conv is None:
            for _ in range(min(50, cap - it)):
                g.step()
                ch[it:it + 1].copy_(pv[2:3])
                it += 1
            if use:
                hit = torch.nonzero(ch[:it] < 1e-6)
                if hit.numel():
                    conv = int(hit[0, 0]) + 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        n = conv or it
        s = g.stats()
        r = {"iterations": n, "converged": conv is not None, "residual": float(ch[n - 1].item()),
             "compliance": s["c"], "seconds": round(wall, 2), "ms_per_iteration": round(1e3 * wall / it, 3)}
        if use:
            n_pae = n
            out["pae"] = r
        else:
            out["plain_same_iterations"] = r
        print(f"[bench] T2 {'with' if use else 'without'} PAE: {r}", file=sys.stderr, flush=True)
    return out


def frame_run(args):
    """The frame reinforcement problem of Sec. 3.5 (900 x 900, 1.62e6 DOFs,
    ft = 3, beta = 2, FP64, multigrid-preconditioned CG): seconds per
    redesign iteration (the paper quotes about 10.8 s on its laptop)."""
    import torch
    import workloads as W
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    g = TopOpt(W.C4, precond=L.TO_PREC_GMG)
    for _ in range(2):
        g.step()
    K = args.frame_steps
    hist = torch.zeros((K, g.sst.numel()), dtype=torch.uint8, device=g.sst.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        g.step()
        hist[k].copy_(g.sst, non_blocking=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h = hist.cpu().numpy()
    st = [L.SolveStats.from_buffer_copy(h[k].tobytes()) for k in range(K)]
    out = {"workload": W.C4.name, "dofs": int(g.plan.info.n), "iterations_timed": f"3-{2 + K}",
           "ms_per_iteration": round(1e3 * wall / K, 2), "paper_s_per_iteration": 10.8,
           "cg_iterations": [s.iterations for s in st], "all_converged": bool(all(s.converged for s in st)),
           "compliance": g.stats()["c"]}
    print(f"[bench] frame900: {out}", file=sys.stderr, flush=True)
    return out


def stream_copy(nbytes=1 << 30, reps=5):
    """Achievable HBM bandwidth: a device-to-device copy of nbytes (read and
    written once), larger than the 256 MB last-level cache."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    s = a.elapsed_time(b) / reps * 1e-3
    gbps = 2 * nbytes / s / 1e9
    del src, dst
    return {"bytes_read_and_written": 2 * nbytes, "gbps": round(gbps, 1), "frac_of_peak": round(gbps * 1e9 / HBM_PEAK, 4)}


def cold_stages(g, cfg, sb, reps=5):
    """Each non-solve stage of the benchmark workload timed alone after
    streaming a 1 GiB buffer (the last-level cache holds none of its
    fields), median over reps."""
    import statistics
    import torch
    from paper_2005_05436_amd import _lib as L
    h, dt, st = g.plan.handle, g.dtype, g.state
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    stages = {
        "filter": lambda: L.to_filter(h, dt, L.TO_FILTER_FWD, g.x, None, None, g.xtilde, None),
        "project": lambda: L.to_project(h, dt, cfg.ft, g.xtilde, g.x, g.xphys, g.dprj, st.beta, g.eta, cfg.volfrac,
                                        g.xphys_old, g.pst),
        "assemble": lambda: L.to_assemble(h, dt, g.xphys, st.penal, g.kval),
        "sensitivity": lambda: L.to_sensitivity(h, dt, g.xphys, g.u, g.f, st.penal, g.dc, g.c),
        "backfilter": lambda: L.to_filter(h, dt, L.TO_FILTER_ADJ2, g.dc, g.dv, g.dprj, g.dcf, g.dv0),
        "oc": lambda: L.to_oc_update(h, dt, g.x, g.dcf, g.dv0, cfg.volfrac, cfg.move, g.ost),
    }
    out = {}
    for name, fn in stages.items():
        ts = []
        for _ in range(reps):
            flush.fill_(1.0)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        ms = statistics.median(ts)
        gbps = sb[name] / (ms * 1e-3) / 1e9
        out[name] = {"ms": round(ms, 4), "gbps": round(gbps, 1), "hbm_frac": round(gbps * 1e9 / HBM_PEAK, 4)}
    del flush
    return out


def stage_scaling(args):
    """The non-solve stages on a mesh 16 times the benchmark's (MBB 4800 x 1600,
    7.68e6 elements, rmin 3 so the filter is bandwidth-bound, FP32 fields,
    volume-preserving projection, beta 2): per-stage time and algorithmic
    bandwidth once the fields no longer fit in the caches (at 1200 x 400 a
    stage's fields are a few MB and its time is launch and grid-sum latency)."""
    import torch
    import workloads as W
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    cfg = W.Config("mbb4800x1600", "mbb", 4800, 1600, rmin=3.0, ft=3, bc="D", beta=2.0, penal=3.0,
                   precision="f32")
    g = TopOpt(cfg, autotune=True)
    I = g.plan.info
    h, dt, st = g.plan.handle, g.dtype, g.state
    g.x.copy_(torch.as_tensor(W.smooth_design(cfg, 5), dtype=torch.float32))
    g.u.copy_(torch.as_tensor(W.displacement_field(I.n, 6)))
    stages = {
        "filter": lambda: L.to_filter(h, dt, L.TO_FILTER_FWD, g.x, None, None, g.xtilde, None),
        "project": lambda: L.to_project(h, dt, cfg.ft, g.xtilde, g.x, g.xphys, g.dprj, st.beta, g.eta, cfg.volfrac,
                                        g.xphys_old, g.pst),
        "assemble": lambda: L.to_assemble(h, dt, g.xphys, st.penal, g.kval),
        "sensitivity": lambda: L.to_sensitivity(h, dt, g.xphys, g.u, g.f, st.penal, g.dc, g.c),
        "backfilter": lambda: L.to_filter(h, dt, L.TO_FILTER_ADJ2, g.dc, g.dv, g.dprj, g.dcf, g.dv0),
        "oc": lambda: L.to_oc_update(h, dt, g.x, g.dcf, g.dv0, cfg.volfrac, cfg.move, g.ost),
    }
    nb = stage_bytes(cfg, I, 4, "assembled", "auto")
    t = g.tuning
    out = {"workload": cfg.name, "elements": I.m, "rmin": cfg.rmin, "precision": "f32", "stages": {},
           "tuning": {k: getattr(t, k) for k in ("filt_v", "filt_parts", "filt_parts2", "filt_mfma", "filt_mfma2",
                                                 "asm_block", "asm_rows")}}
    reps = 5
    for name, fn in stages.items():
        fn()
        a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b2.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b2) / reps
        gbps = nb[name] / (ms * 1e-3) / 1e9
        out["stages"][name] = {"ms": round(ms, 4), "algorithmic_bytes": nb[name], "gbps": round(gbps, 1),
                               "hbm_frac": round(gbps * 1e9 / HBM_PEAK, 4)}
    total = sum(v["ms"] for v in out["stages"].values())
    out["elem_per_s"] = round(I.m / (total * 1e-3), 1)
    print(f"[bench] stage scaling {cfg.name}: {out}", file=sys.stderr, flush=True)
    del g
    return out


def c3d_run(args):
    """The 3D cantilever 96 x 48 x 48 (221,184 Hex8 elements, 6.9e5 DOFs,
    rmin sqrt(3), ft = 3, beta = 2): seconds per redesign iteration with the
    Jacobi-preconditioned CG in FP64 on the assembled K^(s) and on the
    matrix-free operator, with FP32 fields and the mixed-precision CG (FP64
    refinement), and with the multigrid-preconditioned CG (the paper's
    Table 5 quotes 14.2 s per iteration for its code with a multigrid-
    preconditioned CG at this size, rmin 2 sqrt(3), on its laptop)."""
    import torch
    import workloads as W
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    out = {"workload": W.C2.name, "elements": W.C2.m, "paper_s_per_iteration_mgcg": 14.2}
    for name, prec, sp, pc, op in (
            ("jacobi_f64_assembled", "f64", L.TO_SOLVE_AUTO, L.TO_PREC_JACOBI, L.TO_OP_ASSEMBLED),
            ("jacobi_f64_matfree", "f64", L.TO_SOLVE_AUTO, L.TO_PREC_JACOBI, L.TO_OP_MATFREE),
            ("jacobi_f32_mixed", "f32", L.TO_SOLVE_MIXED, L.TO_PREC_JACOBI, L.TO_OP_ASSEMBLED),
            ("gmg_f64", "f64", L.TO_SOLVE_AUTO, L.TO_PREC_GMG, L.TO_OP_ASSEMBLED)):
        g = TopOpt(W.C2, op=op, precision=prec, solve_precision=sp, precond=pc, autotune=True)
        g.step()
        K = args.c3d_steps
        hist = torch.zeros((K, g.sst.numel()), dtype=torch.uint8, device=g.sst.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(K):
            g.step()
            hist[k].copy_(g.sst, non_blocking=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        h = hist.cpu().numpy()
        st = [L.SolveStats.from_buffer_copy(h[k].tobytes()) for k in range(K)]
        out[name] = {"ms_per_iteration": round(1e3 * wall / K, 2), "iterations_timed": f"2-{1 + K}",
                     "cg_iterations": [s.iterations for s in st], "all_converged": bool(all(s.converged for s in st)),
                     "max_true_residual": max(s.residual for s in st), "compliance": g.stats()["c"]}
        print(f"[bench] cantilever 3D {name}: {out[name]}", file=sys.stderr, flush=True)
        del g
    # the paper's Fig. 7 values: 48 x 24 x 24 after 100 redesign steps
    from dataclasses import replace
    chk = {}
    for bc, paper_c in (("N", 3993.7), ("D", 4074.3)):
        cfg = replace(W.C2, name="cantilever48x24x24", nelx=48, nely=24, nelz=24, bc=bc, iterations=100)
        g = TopOpt(cfg, precond=L.TO_PREC_GMG)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(100):
            g.step()
        torch.cuda.synchronize()
        chk[bc] = {"compliance": round(g.stats()["c"], 2), "paper": paper_c,
                   "seconds_for_100_iterations": round(time.perf_counter() - t0, 2)}
        del g
    out["paper_check_48x24x24"] = chk
    print(f"[bench] cantilever 3D 48x24x24 after 100 steps: {chk}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mbb1200x400")
    ap.add_argument("--precision", default=None, choices=[None, "f32", "f64"])
    ap.add_argument("--op", default="assembled", choices=["assembled", "matfree"])
    ap.add_argument("--solve", default="auto", choices=["auto", "f64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--nn-train-steps", type=int, default=13,
                    help="redesign iterations used to train the warm-start network before its timed run "
                         "(0: skip the network-warm-started run)")
    ap.add_argument("--no-gmg", dest="gmg", action="store_false",
                    help="skip the run with the multigrid-preconditioned solve")
    ap.add_argument("--batch-steps", type=int, default=3,
                    help="redesign iterations of the 64-design ragged batch, batched (graph) and one by one "
                         "(0: skip)")
    ap.add_argument("--pae-cap", type=int, default=2500,
                    help="iteration cap of the T2 run with Anderson extrapolation (0: skip)")
    ap.add_argument("--frame-steps", type=int, default=10,
                    help="timed iterations of the 900 x 900 frame problem (0: skip)")
    ap.add_argument("--no-x0-zero", dest="x0_zero", action="store_false",
                    help="skip the runs whose solves start from u = 0")
    ap.add_argument("--no-scaling", dest="scaling", action="store_false",
                    help="skip the non-solve stages on the 4800 x 1600 mesh")
    ap.add_argument("--c3d-steps", type=int, default=3,
                    help="timed iterations of the 96 x 48 x 48 3D cantilever per solver (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size once (a counter calibration kernel)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (how it would shard is "
              "described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from dataclasses import replace
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt, read_struct

    cfg = workloads_by_name()[args.workload]
    if args.precision:
        cfg = replace(cfg, precision=args.precision)
    op = L.TO_OP_MATFREE if args.op == "matfree" else L.TO_OP_ASSEMBLED
    torch.cuda.set_device(0)
    sp = {"auto": L.TO_SOLVE_AUTO, "f64": L.TO_SOLVE_F64, "mixed": L.TO_SOLVE_MIXED}[args.solve]
    g = TopOpt(cfg, op=op, solve_precision=sp, autotune=True)
    I = g.plan.info
    stream = torch.cuda.current_stream()
    t = g.tuning
    print(f"[bench] {cfg.name} m={I.m} n={I.n} nnz_lower={I.nnz_lower} precision={cfg.precision} op={args.op} "
          f"tuning: filter columns {t.filt_v}, waves {t.filt_parts} / {t.filt_parts2}, matrix-core tile "
          f"{t.filt_mfma} / {t.filt_mfma2}, assembly block {t.asm_block}, rows {t.asm_rows}",
          file=sys.stderr, flush=True)

    sst_hist = torch.zeros((max(args.steps, 1), g.sst.numel()), dtype=torch.uint8, device=g.sst.device)
    pst_hist = torch.zeros((max(args.steps, 1), g.pst.numel()), dtype=torch.uint8, device=g.pst.device)
    ost_hist = torch.zeros((max(args.steps, 1), g.ost.numel()), dtype=torch.uint8, device=g.ost.device)

    def timed_step(ev, k=None):
        """One redesign iteration through the single-stage entry points (the
        same sequence to_step runs), with an event after each stage."""
        h, dt, st = g.plan.handle, g.dtype, g.state
        ev[0].record(stream)
        L.to_filter(h, dt, L.TO_FILTER_FWD, g.x, None, None, g.xtilde, None)
        ev[1].record(stream)
        L.to_project(h, dt, cfg.ft, g.xtilde, g.x, g.xphys, g.dprj, st.beta, g.eta, cfg.volfrac,
                     g.xphys_old, g.pst)
        ev[2].record(stream)
        if op == L.TO_OP_ASSEMBLED:
            L.to_assemble(h, dt, g.xphys, st.penal, g.kval)
        ev[3].record(stream)
        L.to_solve(h, dt, g.kval, g.xphys, st.penal, g.f, g.u, g.params.solve, g.sst)
        ev[4].record(stream)
        L.to_sensitivity(h, dt, g.xphys, g.u, g.f, st.penal, g.dc, g.c)
        ev[5].record(stream)
        L.to_filter(h, dt, L.TO_FILTER_ADJ2, g.dc, g.dv, g.dprj, g.dcf, g.dv0)
        ev[6].record(stream)
        L.to_oc_update(h, dt, g.x, g.dcf, g.dv0, cfg.volfrac, cfg.move, g.ost)
        ev[7].record(stream)
        if k is not None:                                  # device-to-device, after the timed stages
            sst_hist[k].copy_(g.sst, non_blocking=True)
            pst_hist[k].copy_(g.pst, non_blocking=True)
            ost_hist[k].copy_(g.ost, non_blocking=True)
        g.xphys_old.copy_(g.xphys)
        st.loop += 1
        st.penal = L.to_continuation(st.penal, g.params.penal_sched, st.loop)
        st.beta = L.to_continuation(st.beta, g.params.beta_sched, st.loop)

    for i in range(args.warmup):
        g.step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(8)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        timed_step(evs[k], k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    K = args.steps
    stage_ms = {s: 0.0 for s in STAGES}
    solve_launch_ms = []
    for k in range(K):
        for j, s in enumerate(STAGES):
            stage_ms[s] += evs[k][j].elapsed_time(evs[k][j + 1])
        solve_launch_ms.append(evs[k][3].elapsed_time(evs[k][4]))
    hist = sst_hist.cpu().numpy()
    solve_stats = [L.SolveStats.from_buffer_copy(hist[k].tobytes()) for k in range(K)]
    iters = [s.iterations for s in solve_stats]
    ph, oh = pst_hist.cpu().numpy(), ost_hist.cpu().numpy()
    newton = [L.ProjectStats.from_buffer_copy(ph[k].tobytes()).n_newton for k in range(K)]
    bisect = [L.OcStats.from_buffer_copy(oh[k].tobytes()).n_bs for k in range(K)]
    last = g.stats()
    print(f"[bench] timed {K} steps in {wall:.3f} s; cg iterations per step {iters}; last: {json.dumps(last)}",
          file=sys.stderr, flush=True)

    non_solve_s = sum(stage_ms[s] for s in NON_SOLVE) / 1e3
    value = I.m * K / non_solve_s
    ms_per_step = wall * 1e3 / K
    dt_bytes = 8 if cfg.precision == "f64" else 4
    sb = stage_bytes(cfg, I, dt_bytes, args.op, args.solve)
    avg_ms = {s: stage_ms[s] / K for s in STAGES}
    gbps = {s: sb[s] / (avg_ms[s] * 1e-3) / 1e9 for s in NON_SOLVE}
    # dominant kernel: the persistent PCG kernel (one launch per step); algorithmic bytes per
    # launch = bytes per CG iteration x the launch's iterations, over the launch's event time
    solve_bytes = sum(sb["solve_per_iter"] * it for it in iters)
    solve_s = sum(solve_launch_ms) / 1e3
    solve_gbps = solve_bytes / solve_s / 1e9
    per_iter_us = 1e6 * solve_s / max(sum(iters), 1)
    kern = sb["solve_kernel"]
    tpi = measured_traffic("solve_kernel<2, 1>") if (I.dim == 2 and kern["operator"] == "matfree"
                                                     and kern["vectors"] == "f64") else None
    traffic = None if tpi is None else round(tpi * sum(iters) / K)
    roof = {"kernel": f"solve_kernel ({kern['operator']} operator, {kern['vectors']} vectors)",
            "bound": "hbm", "achieved": round(solve_gbps, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": round(solve_gbps * 1e9 / HBM_PEAK, 4), "traffic": traffic,
            "avg_launch_ms": round(1e3 * solve_s / K, 3), "bytes_per_cg_iteration": int(sb["solve_per_iter"]),
            "cg_iterations_per_launch": round(sum(iters) / K, 1), "us_per_cg_iteration": round(per_iter_us, 2)}
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "elem/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if cfg.precision == "f32" else "f64",
        "data": "synthetic", "config": {"workload": cfg.name, "elements": I.m, "dofs": I.n, "rmin": cfg.rmin,
                                        "precision": cfg.precision, "operator": args.op, "solve": args.solve,
                                        "solve_vectors": "f64" if kern["vectors"] == "f64" else "f32+f64",
                                        "iterations_timed": f"{args.warmup + 1}-{args.warmup + K}"},
        "to_iters_per_s": round(1e3 / ms_per_step, 3),
        "stage_ms_per_step": {s: round(v, 4) for s, v in avg_ms.items()},
        "stage_gbps": {s: round(v, 1) for s, v in gbps.items()},
        "stage_hbm_frac": {s: round(v * 1e9 / HBM_PEAK, 4) for s, v in gbps.items()},
        "roofline": roof,
        "loop_counts": {"cg": iters, "newton": newton, "bisection": bisect},
        "tuning": {k: getattr(t, k) for k in ("filt_v", "filt_parts", "filt_parts2", "filt_mfma", "filt_mfma2",
                                              "asm_block", "asm_rows", "coop_launch")},
    }
    if I.dim == 2 and cfg.precision == "f32":
        useful, issued = filter_flops(cfg.rmin)
        fc = {}
        for stage, nf, shape in (("filter", 1, t.filt_mfma), ("backfilter", 2, t.filt_mfma2)):
            sec = avg_ms[stage] * 1e-3
            d = {"kernel": f"filter2d_mfma_kernel, tile shape {shape}" if shape else "filter2d_kernel (stencil)",
                 "useful_tflops": round(nf * useful * I.m / sec / 1e12, 1)}
            if shape:
                d["issued_tflops"] = round(nf * issued * I.m / sec / 1e12, 1)
            d["frac_of_fp32_peak"] = round(d.get("issued_tflops", d["useful_tflops"]) * 1e12 / FP32_PEAK, 4)
            fc[stage] = d
        line["filter_compute"] = fc
    sc = stream_copy()
    line["stream_copy"] = sc
    roof["frac_of_achievable"] = round(solve_gbps / sc["gbps"], 4)
    line["stage_cold_cache"] = cold_stages(g, cfg, sb)
    print(f"[bench] copy {sc}; cold-cache stages {line['stage_cold_cache']}", file=sys.stderr, flush=True)
    if I.dim == 2 and args.gmg:
        from paper_2005_05436_amd import _lib as L2
        r = solver_run(args, cfg, op, sp, L2.TO_PREC_GMG)
        print(f"[bench] multigrid run: cg iterations per step {r['cg_iterations']}", file=sys.stderr, flush=True)
        line["gmg"] = r
        line["to_iters_per_s_gmg"] = r["to_iters_per_s"]
    if args.x0_zero and I.dim == 2:
        from paper_2005_05436_amd import _lib as L2
        z = {"note": "every solve started from u = 0 (the other runs warm-start from the previous displacement)"}
        z["jacobi"] = solver_run(args, cfg, op, sp, L2.TO_PREC_JACOBI, zero_x0=True)
        if args.gmg:
            z["gmg"] = solver_run(args, cfg, op, sp, L2.TO_PREC_GMG, zero_x0=True)
        print(f"[bench] x0 = 0: cg iterations per step {z['jacobi']['cg_iterations']}", file=sys.stderr, flush=True)
        line["x0_zero"] = z
    if args.nn_train_steps > 0 and I.dim == 2:
        from paper_2005_05436_amd import _lib as L2
        out = {"note": "network trained on the first iterations of the same problem (in-sample); "
                       "held-out gains are measured by the test suite",
               "plain_cg_iterations_per_step": round(sum(iters) / K, 1)}
        net, info = train_net(args, cfg, op, sp, L2.TO_PREC_JACOBI)
        out.update(info)
        r = solver_run(args, cfg, op, sp, L2.TO_PREC_JACOBI, net)
        print(f"[bench] warm-started run: cg iterations per step {r['cg_iterations']}", file=sys.stderr, flush=True)
        out["jacobi"] = r
        if args.gmg:
            r = solver_run(args, cfg, op, sp, L2.TO_PREC_GMG, net)
            print(f"[bench] warm-started multigrid run: cg iterations per step {r['cg_iterations']}",
                  file=sys.stderr, flush=True)
            out["gmg"] = r
        line["nn_warm_start"] = out
    if args.batch_steps > 0:
        line["batch64"] = batch_run(args)
    if args.pae_cap > 0:
        line["pae_t2"] = pae_run(args)
    if args.frame_steps > 0:
        line["frame900"] = frame_run(args)
    if args.c3d_steps > 0:
        line["cantilever3d"] = c3d_run(args)
    if args.scaling:
        line["stage_scaling"] = stage_scaling(args)
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=g.sst.device)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = nb
        del src, dst
    if not args.no_cpu:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
