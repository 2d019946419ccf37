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
    """Which solve kernel to_solve runs: (operator, vector precision).  op:
    'assembled', 'matfree' or 'hybrid' (matrix-free FP64 operator, Jacobi
    diagonal from the assembled K^(s))."""
    f32 = cfg.precision == "f32"
    mixed = f32 and solve == "mixed"
    assembled = (op == "assembled" and (not f32 or mixed)) or (op == "hybrid" and mixed)
    return ("assembled" if assembled else "matfree"), ("f32" if mixed else "f64")


FP32_PEAK = 157.3e12          # flop/s, MI355X FP32 (matrix cores; also the vector rate with packed instructions)
FP64_PEAK = 78.6e12           # flop/s, MI355X FP64 (vector)


def filter_flops(rmin):
    """2D cone filter work per element: (useful flops = 2 per non-zero tap,
    flops the matrix-core kernel issues = 2,048 per 16 x 16 x 4 product,
    sum over the tap columns dx >= 0 of ceil((16 + 2 lim(dx)) / 4) of them
    per 16 x 16 outputs, lim(dx) = the largest |dy| with a non-zero weight;
    the columns dx and -dx share one product, their window values added
    first, so the useful rate counts taps the kernel did not multiply)."""
    import math
    R = math.ceil(rmin) - 1
    taps, steps = 0, 0
    for dx in range(-R, R + 1):
        lim = -1
        for dy in range(-R, R + 1):
            if rmin - math.sqrt(dx * dx + dy * dy) > 0.0:
                taps += 1
                lim = max(lim, abs(dy))
        if lim >= 0 and dx >= 0:
            steps += (16 + 2 * lim + 3) // 4
    return 2.0 * taps, steps * 2048.0 / 256.0


def stage_bytes(cfg, info, dt_bytes, op, solve):
    """Algorithmic bytes per launch of each stage: every array the kernel must
    read or write counted once (no credit for caches, no charge for re-reads).
    The state solve is priced per CG iteration as the method states it (the
    survey's CG row: the full FP64 CSR matrix at 12 B per non-zero, value and
    column index, plus 56 B per DOF for the vectors), and also by this
    kernel's own traffic model (the matrix-free operator reads moduli instead
    of a matrix)."""
    m, n, nnz, npairs = info.m, info.n, info.nnz_lower, info.n_pairs
    F = dt_bytes
    b = {}
    b["filter"] = F * m + F * m + F * m                       # x in, Hs in, xtilde out
    b["project"] = F * m + 2 * F * m + m                      # xtilde in; xphys, dprj out; passive codes
    b["assemble"] = 4 * npairs + 4 * (nnz + 1) + F * nnz + F * m   # perm, seg_ptr, kval out, xphys in
    b["sensitivity"] = 8 * n + F * m * 2 + m + 8 * n          # u gather, xphys in, dc out, codes, f for f.u
    b["backfilter"] = 3 * F * m + F * m + 2 * F * m           # dc, dv, dprj, Hs in; dc~, dv~ out
    b["oc"] = F * m * 3 + m + F * m                           # x, dc~, dv~, codes in; x out
    full_nnz = 2 * nnz - n                                    # eq. (15): K from its lower triangle
    b["solve_per_iter"] = 12 * full_nnz + 56 * n
    # the kernel's own model: one CG iteration of the kernel to_solve runs
    opk, vp = solve_path(cfg, op, solve)
    V = 4 if vp == "f32" else 8
    mat = (F * nnz + 4 * (n + 1)) if opk == "assembled" else V * m   # K^(s) values + row_ptr | moduli
    if info.dim == 2 and opk == "matfree" and vp == "f64":
        # the pipelined single-sum PCG with the own nodes' vectors on chip
        # (registers and LDS) for the whole solve: only the band moves through
        # memory -- each block stores w of its nodes within one band (ny + 2
        # nodes) of its range ends and loads that of the band on either side
        # of its range; every 100 iterations four more such exchanges
        # (x, r, p, s) recompute the recurrences
        import torch
        nnode, band = n // 2, cfg.nely + 2
        num_cu = torch.cuda.get_device_properties(0).multi_processor_count if torch.cuda.is_available() else 256
        nb = min(num_cu, -(-nnode // 1024))
        chunk = -(-nnode // nb)
        pub = rd = 0
        for bb in range(nb):
            lo = min(nnode, bb * chunk)
            hi = min(nnode, lo + chunk)
            pub += min(hi - lo, 2 * band)
            rd += (lo - max(0, lo - band)) + (min(nnode, hi + band) - hi)
        b["solve_per_iter_kernel_model"] = V * 2 * (pub + rd) * (1 + 4 / 100)
    else:
        phase_a = mat + 2 * V * n + 2 * V * n + n             # z, p_old in; p_new, q out; free mask
        phase_b = 5 * V * n + 3 * V * n                       # x, p, r, q, dinv in; x, r, z out
        if vp == "f32":
            phase_b += 2 * 4 * n                              # the iterate u stays FP64
        b["solve_per_iter_kernel_model"] = phase_a + phase_b
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


def host_info():
    """The host the oracle runs on: CPU model, logical CPUs, the CPUs this
    process may use, and the BLAS / OpenMP thread settings."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "threads_env": {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                                           "MKL_NUM_THREADS")}}


def cpu_sample(workload, strip_ny=25, stages=True):
    """The FP64 oracle on the host (runs in a child process, see cpu_baseline).

    (a) the non-solve stages of one redesign iteration of `workload` in the
        oracle's own calls, on a strip of the mesh (all of nelx, `strip_ny`
        rows, the same filter radius and parameters), each averaged over 3
        iterations and scaled by the ratio of elements (every stage's cost is
        linear in the elements; the filter's in elements x taps): forward
        filter, projection with the Newton threshold, assembly (ordered
        segmented sum), sensitivity, the two-field back-filter, OC bisection;
    (b) the whole 50-iteration run of the 60 x 20 MBB beam (dense Cholesky);
    (c) the oracle's Jacobi PCG at rtol 1e-8 from u = 0 on the 60 x 20 beam at
        a smooth design (whole solve), and 200 of its iterations on MBB
        300 x 100 (per-iteration cost of the smallest 2D configuration)."""
    import numpy as np
    import workloads as W
    from dataclasses import replace
    from oracle import oc, projection, sensitivity, solve, sparse, topopt
    cfg = workloads_by_name()[workload]
    out = {}
    if stages:
        out.update(_cpu_stages(cfg, strip_ny))
    # (b) the 60 x 20 beam, 50 iterations with the dense solve
    p0 = topopt.problem_from_config(W.C0)
    t0 = time.perf_counter()
    topopt.run(p0, W.C0.iterations, solver="dense")
    out["mbb60x20_to_iters_per_s"] = round(W.C0.iterations / (time.perf_counter() - t0), 2)
    # (c) the oracle's PCG
    for c, cap in ((W.C0, 100000), (W.C1[300], 200)):
        p = topopt.problem_from_config(c)
        xc = W.smooth_design(c, 7)
        kl = sparse.assemble(xc, p.ke_lower, p.perm, p.seg_ptr, 3.0, p.E0, p.Emin)
        K = sparse.lower_to_full(p.row_ptr, p.col_idx, kl, p.mesh.n)
        t0 = time.perf_counter()
        _, it, res, ok = solve.solve_pcg(K, p.f, p.free, np.zeros(p.mesh.n), 1e-8, maxit=cap)
        sec = time.perf_counter() - t0
        out[f"pcg_{c.name}"] = {"seconds": round(sec, 3), "iterations": int(it), "ms_per_cg_iteration":
                                round(1e3 * sec / max(int(it), 1), 3), "true_residual": float(res),
                                "converged": bool(ok), "cap": cap}
    return out


def _cpu_stages(cfg, strip_ny):
    import numpy as np
    import workloads as W
    from dataclasses import replace
    from oracle import oc, projection, sensitivity, sparse, topopt
    strip = replace(cfg, nely=min(cfg.nely, strip_ny))
    out = {"strip": f"{strip.nelx}x{strip.nely}"}
    t0 = time.perf_counter()
    prob = topopt.problem_from_config(strip)
    out["setup_s"] = round(time.perf_counter() - t0, 2)
    ms = prob.mesh.m
    scale = cfg.m / ms
    x = W.smooth_design(strip, 3)
    u = W.displacement_field(prob.mesh.n, 4)
    t = {k: [] for k in ("filter", "project", "assemble", "sensitivity", "backfilter", "oc")}
    for rep in range(3):
        t0 = time.perf_counter()
        xt = prob.filter.forward(x)
        t["filter"].append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        xp, dp, eta, nn, ok = projection.physical_density(xt, x, prob.act, cfg.ft, 0.5, 8.0, cfg.volfrac)
        t["project"].append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        sparse.assemble(xp, prob.ke_lower, prob.perm, prob.seg_ptr, 3.0, prob.E0, prob.Emin)
        t["assemble"].append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        dc, _ = sensitivity.sensitivity(xp, u, prob.cmat, prob.ke_full, prob.act, 3.0, prob.E0, prob.Emin)
        t["sensitivity"].append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        dcf = prob.filter.adjoint(-np.abs(dc), dp)
        dv0 = prob.filter.adjoint(prob.dv, dp)
        t["backfilter"].append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        oc.oc_update(x, dcf, dv0, prob.act, cfg.volfrac, cfg.move)
        t["oc"].append(time.perf_counter() - t0)
    stage = {k: scale * sum(v) / len(v) for k, v in t.items()}
    out["stage_s"] = {k: round(v, 4) for k, v in stage.items()}
    out["elem_per_s"] = cfg.m / sum(stage.values())
    return out


def cpu_baseline(workload):
    """cpu_sample in two child processes: BLAS / OpenMP limited to one thread,
    and at all the host's cores.  NumPy's element-wise kernels and SciPy's
    sparse products run on one thread either way, so the non-solve stages
    are timed in the one-thread run only; the thread setting reaches the
    dense Cholesky of the small beam."""
    import subprocess
    runs = {}
    ncpu = len(os.sched_getaffinity(0))
    for name, threads in (("one_thread", "1"), ("all_cores", str(ncpu))):
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = threads
        env["HIP_VISIBLE_DEVICES"] = ""       # the oracle needs no GPU
        # the element-wise stages run on one thread either way: timed once
        extra = [] if name == "one_thread" else ["--cpu-no-stages"]
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-sample", workload] + extra,
                           capture_output=True, text=True, env=env, timeout=900)
        if r.returncode != 0:
            raise RuntimeError(f"oracle sample failed:\n{r.stderr[-2000:]}")
        runs[name] = json.loads(r.stdout.strip().splitlines()[-1])
        runs[name]["threads"] = int(threads)
        print(f"[bench] cpu oracle ({name}): {runs[name]}", file=sys.stderr, flush=True)
    one = runs["one_thread"]
    return {"value": round(one["elem_per_s"], 1), "unit": "elem/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 NumPy oracle, {workload}: every non-solve stage by the oracle's own calls on a "
                       f"{one['strip']} strip of the mesh (same radius and parameters), mean of 3 iterations, "
                       f"scaled by the element ratio; one thread"),
            "host": host_info(), "runs": runs}


def batch_run(args):
    """The 64-design ragged batch (nelx 100..400, nely = nelx / 2, MBB and
    cantilever loads, FP32 fields): graph-replayed batched iterations against
    the same designs advanced one by one with to_step, with the Jacobi PCG
    (one persistent launch for all designs) and with the multigrid solve
    (enqueue-only budget, designs spread over side streams)."""
    import torch
    import workloads as W
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import Batch, TopOpt
    cfgs = W.batch_configs(64, 0)
    m_total = sum(c.m for c in cfgs)
    out = {"designs": len(cfgs), "elements": m_total, "steps": args.batch_steps}
    for name, kw in (("jacobi", {}), ("gmg", {"precond": L.TO_PREC_GMG, "budget": 64, "op": L.TO_OP_HYBRID})):
        b = Batch(cfgs, autotune=True, **kw)
        b.step(use_graph=True)                       # warm-up: capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            b.step(use_graph=True)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / args.batch_steps
        info = b.info()
        st = [g.stats() for g in b.runs]
        del b
        singles = [TopOpt(c, **kw) for c in cfgs]
        for g in singles:
            g.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            for g in singles:
                g.step()
        torch.cuda.synchronize()
        ts = (time.perf_counter() - t0) / args.batch_steps
        del singles
        out[name] = {"ms_per_batched_step": round(1e3 * tb, 2), "ms_per_step_one_by_one": round(1e3 * ts, 2),
                     "speedup": round(ts / tb, 2), "elem_iters_per_s": round(m_total / tb, 1),
                     "cg_iterations_last_step": sum(s["cg_it"] for s in st),
                     "all_converged": bool(all(s["solve_ok"] for s in st)),
                     "graph_captures": info["graph_captures"]}
        if name == "jacobi":
            out[name]["launch_blocks"] = {k: info[k] for k in ("project_blocks", "solve_blocks", "oc_blocks")}
        print(f"[bench] batch64 {name}: {out[name]}", file=sys.stderr, flush=True)
    return out


def nn_leg(args, dim=2):
    """The learned warm start in the regime of the survey's configuration:
    the network trained on the GPU, one Adam step per optimiser iteration, on
    the (physical density, displacement) pairs of `nn_train_iters` optimiser
    iterations over seeded random instances (100 iterations each, multigrid
    solves): in 2D the MBB beam at 300 x 100 with the load node and volfrac
    drawn per instance; in 3D the cantilever at `nn3_mesh` with the height
    of the sine line load and volfrac drawn per instance.  Then held-out
    instances run the same redesign iterations with the plain FP64 Jacobi
    PCG warm-started from the previous displacement and with the network's
    prediction combined with it by the Galerkin start.  Reported: CG
    iterations and solve time (prediction included) per instance for both,
    at true residual <= 1e-8."""
    import torch
    import workloads as W
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt, read_struct
    from paper_2005_05436_amd.nn import Net, layers
    per = 100
    if dim == 2:
        mesh = (300, 100)
        n_inst = max(1, args.nn_train_iters // per)
        train = W.warm_start_instances(n_inst, *mesh, 1000)
        held = W.warm_start_instances(3, *mesh, 2000)
        op = L.TO_OP_ASSEMBLED
    else:
        mesh = tuple(int(v) for v in args.nn3_mesh.split("x"))
        n_inst = max(1, args.nn3_train_iters // per)
        train = W.warm_start_instances3(n_inst, *mesh, 1000)
        held = W.warm_start_instances3(2, *mesh, 2000)
        op = L.TO_OP_MATFREE
    net = None
    t0 = time.perf_counter()
    for cfg in train:
        g = TopOpt(cfg, op=op, precond=L.TO_PREC_GMG, budget=64)
        if net is None:
            net = Net(g.plan)
            net.set_params(W.network_params(layers(dim), 0, taps=9 if dim == 2 else 27))
        for _ in range(per):
            g.step_stages(net, train_lr=1e-3)
        del g
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    out = {"dim": dim, "train": {"instances": n_inst, "iterations_per_instance": per, "mesh": "x".join(map(str, mesh)),
                                 "pairs": n_inst * per, "seconds": round(train_s, 1),
                                 "last_train_loss": round(float(net.loss.item()), 5), "params": net.n_params},
           "held_out": []}
    iters = args.nn_eval_iters
    tot = {"plain": [0, 0.0], "nn": [0, 0.0]}
    for cfg in held:
        row = {"instance": cfg.name, "volfrac": round(cfg.volfrac, 4), "load": cfg.load}
        for mode in ("plain", "nn"):
            g = TopOpt(cfg, op=op)
            cg, ms, ok = [], [], True
            for _ in range(iters):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                g.step_stages(net if mode == "nn" else None, solve_events=(a, b))
                torch.cuda.synchronize()
                s = read_struct(g.sst, L.SolveStats)
                ok = ok and bool(s.converged) and s.residual <= 1e-8
                cg.append(s.iterations)
                ms.append(a.elapsed_time(b))
            row[mode] = {"cg_iterations": sum(cg), "solve_ms": round(sum(ms), 2), "all_converged": ok,
                         "first": cg[0]}
            tot[mode][0] += sum(cg)
            tot[mode][1] += sum(ms)
            del g
        row["cg_gain"] = round(1.0 - row["nn"]["cg_iterations"] / row["plain"]["cg_iterations"], 4)
        out["held_out"].append(row)
        print(f"[bench] warm start {dim}D held-out {row}", file=sys.stderr, flush=True)
    out["iterations_per_instance"] = iters
    out["cg_gain"] = round(1.0 - tot["nn"][0] / tot["plain"][0], 4)
    out["solve_time_gain"] = round(1.0 - tot["nn"][1] / tot["plain"][1], 4)
    del net
    return out


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
    rmin sqrt(3), 'N', ft = 3, beta = 2, penal 3) over its `c3d_iters`
    redesign iterations, each solver timed stage by stage (HIP events):
    FP64 fields with the FP64 Jacobi PCG (matrix-free operator, diagonal from
    the assembled K^(s)); FP32 fields with the mixed-precision CG (FP32
    matrix-free inner operator, FP64 residual replacement to rtol 1e-8); FP64
    fields with the multigrid-preconditioned CG.  The paper's Table 5 quotes
    14.2 s per iteration for its code with a multigrid-preconditioned CG at
    this size (rmin 2 sqrt(3)) on its laptop.  Then the paper's Fig. 7 check:
    48 x 24 x 24 after 100 steps, both filter boundary rules."""
    import copy
    import torch
    import workloads as W
    from dataclasses import replace
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    a3 = copy.copy(args)
    a3.warmup, a3.steps = 1, max(1, args.c3d_iters - 1)
    out = {"workload": W.C2.name, "elements": W.C2.m, "iterations": a3.warmup + a3.steps,
           "paper_s_per_iteration_mgcg": 14.2}
    comp = {}
    for name, prec, op, solve, pc in (("jacobi_f64", "f64", "hybrid", "auto", L.TO_PREC_JACOBI),
                                      ("jacobi_f32_mixed", "f32", "matfree", "mixed", L.TO_PREC_JACOBI),
                                      ("gmg_f64", "f64", "hybrid", "auto", L.TO_PREC_GMG)):
        # multigrid: the host-checked form (runs to convergence at every step)
        rec, g, sb = run_leg(a3, replace(W.C2, precision=prec), op, solve, precond=pc, budget=0)
        c = g.stats()["c"]
        comp[name] = c
        lc = rec["loop_counts"]
        out[name] = {"ms_per_iteration": rec["ms_per_step"], "to_iters_per_s": rec["to_iters_per_s"],
                     "iterations_timed": rec["iterations_timed"],
                     "cg_iterations_per_step": round(sum(lc["cg"]) / len(lc["cg"]), 1),
                     "all_converged": lc["all_converged"], "max_true_residual": lc["max_true_residual"],
                     "us_per_cg_iteration": rec["solve"]["us_per_cg_iteration"],
                     "non_solve_elem_per_s": rec["value"], "stage_ms_per_step": rec["stage_ms_per_step"],
                     "stage_gbps": rec["stage_gbps"], "stage_hbm_frac": rec["stage_hbm_frac"],
                     "final_compliance": c}
        print(f"[bench] cantilever 3D {name}: {out[name]}", file=sys.stderr, flush=True)
        del g
    out["mixed_vs_f64_compliance_rel"] = abs(comp["jacobi_f32_mixed"] - comp["jacobi_f64"]) / abs(comp["jacobi_f64"])
    # the paper's Fig. 7 values: 48 x 24 x 24 after 100 redesign steps
    chk = {}
    for bc, paper_c in (("N", 3993.7), ("D", 4074.3)):
        cfg = replace(W.C2, name="cantilever48x24x24", nelx=48, nely=24, nelz=24, bc=bc, iterations=100)
        g = TopOpt(cfg, precond=L.TO_PREC_GMG, budget=0)
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


OPS = {"assembled": 0, "matfree": 1, "hybrid": 2}


def run_leg(args, cfg, op_name, solve="auto", precond=0, budget=None):
    """Warm-up iterations through to_step, then K timed redesign iterations
    through the single-stage entry points (the sequence to_step runs) with a
    HIP event after each stage on the launch stream.  Returns the leg's
    record, the run object and the stage byte model."""
    import torch
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt
    op = OPS[op_name]
    sp = {"auto": L.TO_SOLVE_AUTO, "f64": L.TO_SOLVE_F64, "mixed": L.TO_SOLVE_MIXED}[solve]
    g = TopOpt(cfg, op=op, solve_precision=sp, autotune=True, precond=precond,
               budget=(args.gmg_budget if budget is None else budget) if precond == L.TO_PREC_GMG else 0)
    I = g.plan.info
    stream = torch.cuda.current_stream()
    t = g.tuning
    print(f"[bench] {cfg.name} m={I.m} n={I.n} nnz_lower={I.nnz_lower} precision={cfg.precision} op={op_name} "
          f"tuning: filter columns {t.filt_v}, waves {t.filt_parts} / {t.filt_parts2}, matrix-core tile "
          f"{t.filt_mfma} / {t.filt_mfma2}, assembly block {t.asm_block}, rows {t.asm_rows}",
          file=sys.stderr, flush=True)
    K = args.steps
    sst_hist = torch.zeros((max(K, 1), g.sst.numel()), dtype=torch.uint8, device=g.sst.device)
    pst_hist = torch.zeros((max(K, 1), g.pst.numel()), dtype=torch.uint8, device=g.pst.device)
    ost_hist = torch.zeros((max(K, 1), g.ost.numel()), dtype=torch.uint8, device=g.ost.device)

    def timed_step(ev, k):
        h, dt, st = g.plan.handle, g.dtype, g.state
        ev[0].record(stream)
        L.to_filter(h, dt, L.TO_FILTER_FWD, g.x, None, None, g.xtilde, None)
        ev[1].record(stream)
        L.to_project(h, dt, cfg.ft, g.xtilde, g.x, g.xphys, g.dprj, st.beta, g.eta, cfg.volfrac,
                     g.xphys_old, g.pst)
        ev[2].record(stream)
        if op != L.TO_OP_MATFREE:
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
        sst_hist[k].copy_(g.sst, non_blocking=True)        # device-to-device, after the timed stages
        pst_hist[k].copy_(g.pst, non_blocking=True)
        ost_hist[k].copy_(g.ost, non_blocking=True)
        g.xphys_old.copy_(g.xphys)
        st.loop += 1
        st.penal = L.to_continuation(st.penal, g.params.penal_sched, st.loop)
        st.beta = L.to_continuation(st.beta, g.params.beta_sched, st.loop)

    for _ in range(args.warmup):
        g.step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(8)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        timed_step(evs[k], k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = {s: 0.0 for s in STAGES}
    solve_ms = []
    for k in range(K):
        for j, s in enumerate(STAGES):
            stage_ms[s] += evs[k][j].elapsed_time(evs[k][j + 1])
        solve_ms.append(evs[k][3].elapsed_time(evs[k][4]))
    sh, ph, oh = sst_hist.cpu().numpy(), pst_hist.cpu().numpy(), ost_hist.cpu().numpy()
    sst = [L.SolveStats.from_buffer_copy(sh[k].tobytes()) for k in range(K)]
    iters = [s.iterations for s in sst]
    newton = [L.ProjectStats.from_buffer_copy(ph[k].tobytes()).n_newton for k in range(K)]
    bisect = [L.OcStats.from_buffer_copy(oh[k].tobytes()).n_bs for k in range(K)]
    last = g.stats()
    print(f"[bench] {cfg.name} {cfg.precision}: timed {K} steps in {wall:.3f} s; cg iterations {iters}; "
          f"last: {json.dumps(last)}", file=sys.stderr, flush=True)
    dt_bytes = 8 if cfg.precision == "f64" else 4
    sb = stage_bytes(cfg, I, dt_bytes, op_name, solve)
    avg_ms = {s: stage_ms[s] / K for s in STAGES}
    non_solve_s = sum(stage_ms[s] for s in NON_SOLVE) / 1e3
    gbps = {s: sb[s] / (avg_ms[s] * 1e-3) / 1e9 for s in NON_SOLVE}
    solve_s = sum(solve_ms) / 1e3
    its = max(sum(iters), 1)
    kern = sb["solve_kernel"]
    rec = {"value": round(I.m * K / non_solve_s, 1), "ms_per_step": round(wall * 1e3 / K, 3),
           "to_iters_per_s": round(K / wall, 3),
           "iterations_timed": f"{args.warmup + 1}-{args.warmup + K}",
           "stage_ms_per_step": {s: round(v, 4) for s, v in avg_ms.items()},
           "stage_gbps": {s: round(v, 1) for s, v in gbps.items()},
           "stage_hbm_frac": {s: round(v * 1e9 / HBM_PEAK, 4) for s, v in gbps.items()},
           "loop_counts": {"cg": iters, "newton": newton, "bisection": bisect,
                           "all_converged": bool(all(s.converged for s in sst)),
                           "max_true_residual": max(s.residual for s in sst)},
           "solve": {"kernel": f"solve_kernel ({kern['operator']} operator, {kern['vectors']} vectors)",
                     "avg_launch_ms": round(1e3 * solve_s / K, 3), "cg_iterations_per_launch": round(its / K, 1),
                     "us_per_cg_iteration": round(1e6 * solve_s / its, 2),
                     "bytes_per_cg_iteration": int(sb["solve_per_iter"]),
                     "bytes_per_cg_iteration_kernel_model": int(sb["solve_per_iter_kernel_model"]),
                     "gbps": round(sb["solve_per_iter"] * its / solve_s / 1e9, 1),
                     "gbps_kernel_model": round(sb["solve_per_iter_kernel_model"] * its / solve_s / 1e9, 1)},
           "tuning": {k: getattr(t, k) for k in ("filt_v", "filt_parts", "filt_parts2", "filt_mfma", "filt_mfma2",
                                                 "asm_block", "asm_rows", "coop_launch")}}
    if I.dim == 2:
        useful, issued = filter_flops(cfg.rmin)
        fc = {}
        for stage, nf, shape in (("filter", 1, t.filt_mfma), ("backfilter", 2, t.filt_mfma2)):
            sec = avg_ms[stage] * 1e-3
            d = {"kernel": f"filter2d_mfma_kernel, tile shape {shape}" if shape else "filter2d_kernel (stencil)",
                 "useful_tflops": round(nf * useful * I.m / sec / 1e12, 1)}
            peak = FP32_PEAK if cfg.precision == "f32" else FP64_PEAK
            if shape:
                d["issued_tflops"] = round(nf * issued * I.m / sec / 1e12, 1)
            d["peak_tflops"] = peak / 1e12
            d["frac_of_peak"] = round(d.get("issued_tflops", d["useful_tflops"]) * 1e12 / peak, 4)
            fc[stage] = d
        rec["filter_compute"] = fc
    return rec, g, sb


def schedule_leg(args, cfg):
    """The workload's whole continuation schedule (beta 1 -> 32 x2 and penal
    1 -> 3 +0.25 every 25 iterations, 200 iterations) in FP64 fields.  The
    trajectory advances with the multigrid-preconditioned solve (enqueue-only
    budget); every iteration is timed (HIP events around to_step).  At
    `samples` iterations spread over the schedule (each continuation level
    included), the state solve of that iteration is also timed with the plain
    FP64 Jacobi PCG from the previous displacement, so the plain method's
    redesign rate over the schedule follows from the non-solve time of every
    iteration plus the Jacobi solve time interpolated between samples."""
    import numpy as np
    import torch
    from paper_2005_05436_amd import _lib as L
    from paper_2005_05436_amd.driver import TopOpt, read_struct
    n_it = cfg.iterations
    # the trajectory's multigrid solves check convergence on the host (their
    # iteration counts grow along the schedule), so every solve meets the tolerance
    g = TopOpt(cfg, op=L.TO_OP_HYBRID, precond=L.TO_PREC_GMG, budget=0, autotune=True)
    jac = L.SolveOpts(1e-8, 0.1, 400000, L.TO_OP_HYBRID, L.TO_SOLVE_AUTO, 0, 0, L.TO_PREC_JACOBI, 0)
    samples = sorted(set(int(round(v)) for v in np.linspace(1, n_it, args.schedule_samples)))
    stream = torch.cuda.current_stream()
    h, dt = g.plan.handle, g.dtype
    hist = torch.zeros((n_it, g.sst.numel()), dtype=torch.uint8, device=g.sst.device)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_it)]
    rows = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(n_it):
        it = k + 1
        st = g.state
        if it in samples:
            # the sample's Jacobi solve, on the state this iteration solves for
            eta0 = g.eta.clone()
            L.to_filter(h, dt, L.TO_FILTER_FWD, g.x, None, None, g.xtilde, None)
            L.to_project(h, dt, cfg.ft, g.xtilde, g.x, g.xphys, g.dprj, st.beta, g.eta, cfg.volfrac,
                         g.xphys_old, g.pst)
            L.to_assemble(h, dt, g.xphys, st.penal, g.kval)
            u_prev = g.u.clone()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            L.to_solve(h, dt, g.kval, g.xphys, st.penal, g.f, g.u, jac, g.sst)
            b.record(stream)
            torch.cuda.synchronize()
            s = read_struct(g.sst, L.SolveStats)
            rows.append({"iteration": it, "beta": st.beta, "penal": st.penal, "jacobi_ms": round(a.elapsed_time(b), 3),
                         "jacobi_cg": s.iterations, "jacobi_converged": bool(s.converged),
                         "jacobi_residual": s.residual})
            # restore the iteration's starting point (threshold and previous
            # displacement); to_step below redoes the iteration with the
            # multigrid solve
            g.u.copy_(u_prev)
            g.eta.copy_(eta0)
        ev[k][0].record(stream)
        g.step()
        ev[k][1].record(stream)
        hist[k].copy_(g.sst, non_blocking=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    step_ms = [a.elapsed_time(b) for a, b in ev]
    hh = hist.cpu().numpy()
    sst = [L.SolveStats.from_buffer_copy(hh[k].tobytes()) for k in range(n_it)]
    return g, rows, step_ms, sst, wall, samples


def schedule_record(args, cfg, non_solve_ms_per_it):
    """Runs schedule_leg and condenses it: the multigrid trajectory's measured
    redesign rate over the whole schedule, the Jacobi samples, and the plain
    Jacobi method's rate over the schedule (non-solve time of every iteration
    from the multigrid run's events minus its solve, plus the Jacobi solve
    time interpolated linearly between samples)."""
    import numpy as np
    g, rows, step_ms, sst, wall, samples = schedule_leg(args, cfg)
    n_it = len(step_ms)
    gmg_its = [s.iterations for s in sst]
    # the multigrid run: measured per iteration
    out = {"workload": cfg.name, "iterations": n_it, "precision": cfg.precision,
           "schedule": "beta 1 -> 32 (x2 every 25), penal 1 -> 3 (+0.25 every 25)",
           "gmg": {"to_iters_per_s": round(n_it / (sum(step_ms) * 1e-3), 2),
                   "wall_to_iters_per_s": round(n_it / wall, 2),
                   "cg_iterations_per_step": round(sum(gmg_its) / n_it, 1),
                   "all_converged": bool(all(s.converged for s in sst)),
                   "max_true_residual": max(s.residual for s in sst),
                   "final_compliance": g.stats()["c"]},
           "jacobi_samples": rows}
    xs = [r["iteration"] for r in rows]
    ys = [r["jacobi_ms"] for r in rows]
    jac_ms = np.interp(np.arange(1, n_it + 1), xs, ys)
    est = n_it / ((n_it * non_solve_ms_per_it + float(jac_ms.sum())) * 1e-3)
    out["jacobi"] = {"to_iters_per_s_estimated": round(est, 3),
                     "note": ("non-solve stages at the measured per-iteration time of the headline leg; Jacobi "
                              "PCG solve times measured at the sampled iterations (true residual <= 1e-8, warm "
                              "start from the previous displacement) and interpolated linearly in between"),
                     "cg_iterations_at_samples": [r["jacobi_cg"] for r in rows],
                     "all_converged": bool(all(r["jacobi_converged"] for r in rows))}
    print(f"[bench] schedule {cfg.name}: {out['gmg']}; jacobi samples {[(r['iteration'], r['jacobi_cg']) for r in rows]}"
          f" -> {est:.3f} it/s", file=sys.stderr, flush=True)
    del g
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mbb1200x400")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-no-stages", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-fp32", dest="fp32", action="store_false",
                    help="skip the second leg with FP32 fields")
    ap.add_argument("--schedule-samples", type=int, default=9,
                    help="iterations of the 200-iteration schedule at which the Jacobi solve is timed (0: skip "
                         "the schedule run)")
    ap.add_argument("--gmg-budget", type=int, default=48,
                    help="outer iterations enqueued per multigrid solve (enqueue-only form)")
    ap.add_argument("--nn-train-iters", type=int, default=2000,
                    help="optimiser iterations whose (design, displacement) pairs train the warm-start network "
                         "(0: skip the learned warm start)")
    ap.add_argument("--nn3-train-iters", type=int, default=500,
                    help="optimiser iterations that train the 3D network (0: skip the 3D learned warm start)")
    ap.add_argument("--nn3-mesh", default="48x24x24", help="mesh of the 3D learned warm start (nelx x nely x nelz)")
    ap.add_argument("--nn-eval-iters", type=int, default=30,
                    help="redesign iterations per held-out instance, plain and warm-started")
    ap.add_argument("--batch-steps", type=int, default=3,
                    help="redesign iterations of the 64-design ragged batch, batched (graph) and one by one "
                         "(0: skip)")
    ap.add_argument("--pae-cap", type=int, default=2500,
                    help="iteration cap of the T2 run with Anderson extrapolation (0: skip)")
    ap.add_argument("--frame-steps", type=int, default=10,
                    help="timed iterations of the 900 x 900 frame problem (0: skip)")
    ap.add_argument("--no-scaling", dest="scaling", action="store_false",
                    help="skip the non-solve stages on the 4800 x 1600 mesh")
    ap.add_argument("--c3d-iters", type=int, default=100,
                    help="redesign iterations of the 96 x 48 x 48 3D cantilever per solver (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size once (a counter calibration kernel)")
    args = ap.parse_args()
    if args.cpu_sample:
        print(json.dumps(cpu_sample(args.cpu_sample, stages=not args.cpu_no_stages)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (how it would shard is "
              "described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from dataclasses import replace

    cfg = workloads_by_name()[args.workload]
    torch.cuda.set_device(0)
    # headline: FP64 fields (the paper's precision); the solve is FP64 Jacobi
    # PCG on the matrix-free operator preconditioned by the assembled diagonal
    c64 = replace(cfg, precision="f64")
    rec, g, sb = run_leg(args, c64, "hybrid")
    I = g.plan.info
    K = args.steps
    sol = rec["solve"]
    tpi = measured_traffic("solve_kernel<2, 7>") if I.dim == 2 else None
    roof = {"kernel": sol["kernel"], "bound": "hbm", "achieved": sol["gbps"], "peak": HBM_PEAK / 1e9,
            "unit": "GB/s", "frac": round(sol["gbps"] * 1e9 / HBM_PEAK, 4),
            "traffic": None if tpi is None else round(tpi * sol["cg_iterations_per_launch"]),
            "algorithmic_bytes": "per CG iteration: 12 B per non-zero of the full FP64 CSR K + 56 B per DOF",
            "avg_launch_ms": sol["avg_launch_ms"], "bytes_per_cg_iteration": sol["bytes_per_cg_iteration"],
            "cg_iterations_per_launch": sol["cg_iterations_per_launch"],
            "us_per_cg_iteration": sol["us_per_cg_iteration"],
            "kernel_model": {"bytes_per_cg_iteration": sol["bytes_per_cg_iteration_kernel_model"],
                             "gbps": sol["gbps_kernel_model"],
                             "frac": round(sol["gbps_kernel_model"] * 1e9 / HBM_PEAK, 4)},
            "note": ("achieved prices a CG iteration at the survey's CG row (the full FP64 CSR K); the kernel "
                     "applies the matrix-free operator and never reads K, so that rate can pass the HBM peak; "
                     "kernel_model counts the arrays this kernel reads and writes, traffic the counted bytes")}
    line = {
        "metric": METRIC, "value": rec["value"], "unit": "elem/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": rec["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": c64.name, "elements": I.m, "dofs": I.n, "rmin": c64.rmin, "precision": "f64",
                   "operator": "matrix-free FP64 SpMV, Jacobi diagonal from the assembled FP64 K^(s)",
                   "solve": "FP64 Jacobi PCG, rtol 1e-8 (true residual), warm start from the previous u",
                   "iterations_timed": rec["iterations_timed"]},
        "to_iters_per_s": rec["to_iters_per_s"],
        "stage_ms_per_step": rec["stage_ms_per_step"], "stage_gbps": rec["stage_gbps"],
        "stage_hbm_frac": rec["stage_hbm_frac"], "roofline": roof, "loop_counts": rec["loop_counts"],
        "tuning": rec["tuning"], "filter_compute": rec.get("filter_compute"),
    }
    sc = stream_copy()
    line["stream_copy"] = sc
    roof["frac_of_achievable"] = round(sol["gbps"] / sc["gbps"], 4)
    line["stage_cold_cache"] = cold_stages(g, c64, sb)
    non_solve_ms = sum(rec["stage_ms_per_step"][s] for s in NON_SOLVE)
    del g
    print(f"[bench] FP64 headline {rec['value']:.4g} elem/s; copy {sc}", file=sys.stderr, flush=True)
    if args.fp32:
        r32, g32, _ = run_leg(args, replace(cfg, precision="f32"), "assembled")
        r32["config"] = {"precision": "f32 fields, FP64 dot products, solve vectors and OC sums",
                         "operator": "matrix-free FP64 SpMV, Jacobi diagonal from the assembled FP32 K^(s)"}
        line["fp32_fields"] = r32
        del g32
    if args.schedule_samples > 0:
        line["schedule"] = schedule_record(args, c64, non_solve_ms)
    if args.nn_train_iters > 0:
        line["nn_warm_start"] = nn_leg(args, 2)
    if args.nn3_train_iters > 0:
        line["nn_warm_start_3d"] = nn_leg(args, 3)
    if args.c3d_iters > 0:
        line["cantilever3d"] = c3d_run(args)
    if args.batch_steps > 0:
        line["batch64"] = batch_run(args)
    if args.pae_cap > 0:
        line["pae_t2"] = pae_run(args)
    if args.frame_steps > 0:
        line["frame900"] = frame_run(args)
    if args.scaling:
        line["stage_scaling"] = stage_scaling(args)
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = nb
        del src, dst
    if not args.no_cpu:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(c64.name)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
