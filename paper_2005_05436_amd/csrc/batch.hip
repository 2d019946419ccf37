// Ragged batches of independent designs, and the launch-shape autotuner.
//
// A batch advances many designs of different sizes by one redesign iteration
// (blocks RL.1-RL.4 for each) with one launch per persistent stage for the
// whole batch: the projection with its Newton threshold, the PCG solve and the
// OC bisection each run as one cooperative launch whose blocks are split into
// per-design groups (group sizes proportional to the design's size); each
// group synchronises and reduces on its own design's barrier words and
// partial buffers, so designs never wait for one another inside a stage and
// the solve of a small design does not hold back a large one until the
// launch ends.  The other stages are one ordinary launch each for the whole
// batch: the moduli, the 2D assembly and the sensitivities with per-design
// block groups of a fourth map, and the two 2D stencil passes over one list
// of the tiles of every design (3D designs filter and assemble per design).
// Every stage reads its per-design arguments from tables written once at
// creation, and the scalars that change during a run (beta, the threshold
// target, volfrac, move, penal) from a small device array refreshed at the
// start of each iteration.  Optionally the whole iteration is captured once into
// a HIP graph and replayed while every design's scalars (penal, beta,
// volfrac, move, threshold target) stay the same; a change recaptures it.
//
// The autotuner times the candidate launch shapes of the 2D filter (output
// columns per tile, waves per block) and of the assembly (threads per block)
// on the plan's own arrays and keeps the fastest.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

namespace topt {

constexpr int kDynChunk = 64;
constexpr int kDynStride = 5;    // beta, target, volfrac, move, penal
struct BatchDyn {
    int32_t first, n;
    double v[kDynChunk][kDynStride];
};

__global__ void batch_dyn_kernel(double* dyn, BatchDyn d) {
    const int t = threadIdx.x;
    if (t < kDynStride * d.n) dyn[kDynStride * (size_t)d.first + t] = d.v[t / kDynStride][t % kDynStride];
}

// Splits `blocks` among designs in proportion to `work`, at least one and at
// most `cap_i` each; returns the total used.
static int split_blocks(const std::vector<double>& work, const std::vector<int>& cap, int blocks,
                        std::vector<int32_t>& first, std::vector<int32_t>& count, std::vector<int32_t>& inst) {
    const int n = (int)work.size();
    double tot = 0.0;
    for (double w : work) tot += w;
    count.assign(n, 1);
    int used = n;
    // proportional share of the blocks left after the one each design gets
    for (int i = 0; i < n; ++i) {
        const int extra = (int)std::floor((blocks - n) * (work[i] / tot));
        const int c = std::max(1, std::min(cap[i], 1 + std::max(0, extra)));
        used += c - 1;
        count[i] = c;
    }
    while (used > blocks) {          // rounding can overshoot: take from the largest
        int j = 0;
        for (int i = 1; i < n; ++i) if (count[i] > count[j]) j = i;
        if (count[j] <= 1) break;
        --count[j];
        --used;
    }
    first.assign(n, 0);
    inst.clear();
    for (int i = 0; i < n; ++i) {
        first[i] = (int32_t)inst.size();
        for (int k = 0; k < count[i]; ++k) inst.push_back(i);
    }
    return used;
}

struct Batch {
    std::vector<Plan*> plans;
    std::vector<to_step_state> st0;     // device pointers fixed at creation
    std::vector<int> ft, oc;
    to_dtype dt = TO_F32;
    int n = 0, dim = 2, mode = 0;
    to_solve_opts solve{};
    char* proj_tab = nullptr;
    char* oc_tab = nullptr;
    char* solve_tab = nullptr;
    double* dyn = nullptr;
    BatchMap mp_proj{}, mp_oc{}, mp_solve{};
    // the stencil, moduli, assembly and sensitivity stages: one launch each
    // for the whole batch (filter and assembly for 2D designs; 3D designs
    // filter and assemble per design)
    char* filt_fwd = nullptr;
    char* filt_adj = nullptr;
    int32_t* tile0 = nullptr;
    int ntiles = 0, rmax = 0;
    bool filt_batched = false;
    unsigned* ctr = nullptr;
    char* asm_tab = nullptr;
    char* sens_tab = nullptr;
    BatchMap mp_elem{};
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<double> key;
    int graph_captures = 0, graph_launches = 0;
    // multigrid solves: one enqueue-only solve per design, spread over side
    // streams that fork from and join the batch's stream (parallel branches
    // when captured)
    bool gmg = false;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;     // ev[0] fork, ev[1 + j] join of side[j]
};
constexpr int kBatchSideStreams = 4;

struct BatchLayout {
    size_t proj, oc, solve, dyn, maps, filt, tile0, asmt, sens, ctr, total;
};
constexpr int kBatchMaps = 4;

static BatchLayout batch_layout(int count) {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    BatchLayout L{};
    size_t o = 0;
    const size_t pa = std::max(project_args_bytes(TO_F64), project_args_bytes(TO_F32));
    const size_t oa = std::max(oc_args_bytes(TO_F64), oc_args_bytes(TO_F32));
    L.proj = o; o += al(pa * count);
    L.oc = o; o += al(oa * count);
    L.solve = o; o += al(solve_args_bytes() * count);
    L.dyn = o; o += al(sizeof(double) * kDynStride * count);
    L.maps = o; o += al(kBatchMaps * sizeof(int32_t) * ((size_t)kMaxCoopBlocks + 2 * (size_t)count));
    L.filt = o; o += al(2 * filter_batch_entry_bytes() * count);
    L.tile0 = o; o += al(sizeof(int32_t) * (count + 1));
    L.asmt = o; o += al(asm_args_bytes() * count);
    L.sens = o; o += al(sens_args_bytes() * count);
    L.ctr = o; o += 256;
    L.total = o;
    return L;
}

static bool same_state(const to_step_state& a, const to_step_state& b) {
    return a.x == b.x && a.xtilde == b.xtilde && a.xphys == b.xphys && a.xphys_old == b.xphys_old &&
           a.dprj == b.dprj && a.dc == b.dc && a.dcf == b.dcf && a.dv == b.dv && a.dv0 == b.dv0 &&
           a.kval == b.kval && a.u == b.u && a.f == b.f && a.eta == b.eta && a.compliance == b.compliance &&
           a.pstats == b.pstats && a.sstats == b.sstats && a.ostats == b.ostats;
}

// One redesign iteration of every design, enqueued on s.
static to_status batch_enqueue(Batch* b, const to_step_state* st, const to_step_params* prm, hipStream_t s) {
    to_status r;
    const to_dtype dt = b->dt;
    for (int c0 = 0; c0 < b->n; c0 += kDynChunk) {
        BatchDyn d{};
        d.first = c0;
        d.n = std::min(kDynChunk, b->n - c0);
        for (int k = 0; k < d.n; ++k) {
            const to_step_params& p = prm[c0 + k];
            d.v[k][0] = st[c0 + k].beta;
            d.v[k][1] = std::isnan(p.target) ? p.volfrac : p.target;
            d.v[k][2] = p.volfrac;
            d.v[k][3] = p.move;
            d.v[k][4] = st[c0 + k].penal;
        }
        hipLaunchKernelGGL(batch_dyn_kernel, dim3(1), dim3(kDynStride * kDynChunk), 0, s, b->dyn, d);
    }
    const int num_cu = b->plans[0]->num_cu;
    if (b->filt_batched) {
        if ((r = launch_filter_batch(dt, TO_FILTER_FWD, b->filt_fwd, b->tile0, b->n, b->ntiles, b->rmax, num_cu,
                                     b->ctr, s)))
            return r;
    } else {
        for (int i = 0; i < b->n; ++i)
            if ((r = launch_filter(b->plans[i], dt, TO_FILTER_FWD, st[i].x, nullptr, nullptr, st[i].xtilde, nullptr,
                                   s)))
                return r;
    }
    if ((r = launch_project_batch(dt, b->proj_tab, b->mp_proj, s))) return r;
    if (b->gmg) {
        // per design: FP64 moduli, hierarchy set-up and a fixed budget of
        // predicated outer iterations (no host synchronisation)
        const int k = (int)b->side.size();
        TO_HIP(hipEventRecord(b->ev[0], s));
        for (int j = 0; j < k; ++j) TO_HIP(hipStreamWaitEvent(b->side[j], b->ev[0], 0));
        for (int i = 0; i < b->n; ++i)
            if ((r = launch_solve_gmg(b->plans[i], dt, st[i].xphys, st[i].penal, st[i].f, st[i].u, b->solve,
                                      st[i].sstats, b->side[i % k])))
                return r;
        for (int j = 0; j < k; ++j) {
            TO_HIP(hipEventRecord(b->ev[1 + j], b->side[j]));
            TO_HIP(hipStreamWaitEvent(s, b->ev[1 + j], 0));
        }
    } else {
        // the moduli (and the FP64 ones the mixed and hybrid operators use),
        // then the sums of K^(s)
        const bool assembled = b->solve.op != TO_OP_MATFREE;
        if (assembled || b->mode != 0) {
            if ((r = launch_moduli_batch(dt, b->asm_tab, b->dyn, kDynStride, b->mp_elem,
                                         dt == TO_F32 && b->mode != 0, s)))
                return r;
        }
        if (assembled) {
            if (b->dim == 2) {
                if ((r = launch_assemble_batch2d(dt, b->asm_tab, b->mp_elem, s))) return r;
            } else {
                for (int i = 0; i < b->n; ++i)
                    if ((r = launch_assemble_from_moduli(b->plans[i], dt, st[i].kval, s))) return r;
            }
        }
        if ((r = launch_solve_batch(b->dim, b->mode, b->solve_tab, b->mp_solve, s))) return r;
    }
    if ((r = launch_sensitivity_batch(b->dim, dt, b->sens_tab, b->dyn, kDynStride, b->mp_elem, s))) return r;
    if (b->filt_batched) {
        if ((r = launch_filter_batch(dt, TO_FILTER_ADJ2, b->filt_adj, b->tile0, b->n, b->ntiles, b->rmax, num_cu,
                                     b->ctr, s)))
            return r;
    } else {
        for (int i = 0; i < b->n; ++i)
            if ((r = launch_filter(b->plans[i], dt, TO_FILTER_ADJ2, st[i].dc, st[i].dv, st[i].dprj, st[i].dcf,
                                   st[i].dv0, s)))
                return r;
    }
    if ((r = launch_oc_batch(dt, b->oc_tab, b->mp_oc, s))) return r;
    for (int i = 0; i < b->n; ++i) {
        const size_t bytes = (dt == TO_F64 ? 8 : 4) * (size_t)b->plans[i]->info.m;
        TO_HIP(hipMemcpyAsync(st[i].xphys_old, st[i].xphys, bytes, hipMemcpyDeviceToDevice, s));
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

// --- autotuner ---------------------------------------------------------------
template <class F>
static float time_ms(hipStream_t s, F&& f, int reps) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return 1e30f;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return 1e30f; }
    f();                                               // warm-up (and first-launch costs)
    (void)hipEventRecord(a, s);
    for (int k = 0; k < reps; ++k) f();
    (void)hipEventRecord(b, s);
    float ms = 1e30f;
    if (hipEventSynchronize(b) == hipSuccess) (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

to_status plan_autotune(Plan* p, to_dtype dt, void* kval, hipStream_t s, to_tuning* out) {
    TO_HIP(hipStreamSynchronize(s));
    const void* Hs = dt == TO_F64 ? (const void*)p->Hs64 : (const void*)p->Hs32;
    void* scratch = dt == TO_F64 ? (void*)p->fx64 : (void*)p->fx32;
    Plan::Tune best = p->tune;
    if (p->dim == 2) {
        // one-field filter: columns per tile and waves per block
        struct Cand { int v, parts; };
        const Cand cands[] = {{8, 0}, {8, 8}, {4, 0}, {4, 4}};
        float tbest = 1e30f;
        p->tune.filt_mfma = p->tune.filt_mfma2 = best.filt_mfma = best.filt_mfma2 = 0;
        for (const Cand& c : cands) {
            p->tune.filt_v = c.v;
            p->tune.filt_parts = c.parts;
            to_status st = TO_OK;
            const float t = time_ms(s, [&] {
                if (st == TO_OK) st = launch_filter(p, dt, TO_FILTER_FWD, Hs, nullptr, nullptr, scratch, nullptr, s);
            }, 3);
            if (st != TO_OK) continue;          // e.g. the tile does not fit in LDS
            if (t < tbest) { tbest = t; best.filt_v = c.v; best.filt_parts = c.parts; }
        }
        {                                    // the matrix-core tiles (same columns and waves otherwise)
            p->tune.filt_v = best.filt_v;
            p->tune.filt_parts = best.filt_parts;
            for (int shape = 1; shape <= 4; ++shape) {
                p->tune.filt_mfma = shape;
                to_status st = TO_OK;
                const float t = time_ms(s, [&] {
                    if (st == TO_OK) st = launch_filter(p, dt, TO_FILTER_FWD, Hs, nullptr, nullptr, scratch, nullptr, s);
                }, 3);
                if (st == TO_OK && t < tbest) { tbest = t; best.filt_mfma = shape; }
            }
        }
        p->tune.filt_v = best.filt_v;
        p->tune.filt_parts = best.filt_parts;
        p->tune.filt_mfma = best.filt_mfma;
        // fused double adjoint: waves per block with the chosen columns
        void* scratch2 = dt == TO_F64 ? (void*)p->v64[7] : (void*)p->v32[7];   // n >= m entries
        tbest = 1e30f;
        for (int parts : {0, 8, 16}) {
            p->tune.filt_parts2 = parts;
            to_status st = TO_OK;
            const float t = time_ms(s, [&] {
                if (st == TO_OK) st = launch_filter(p, dt, TO_FILTER_ADJ2, Hs, Hs, nullptr, scratch, scratch2, s);
            }, 3);
            if (st != TO_OK) continue;
            if (t < tbest) { tbest = t; best.filt_parts2 = parts; }
        }
        {
            p->tune.filt_parts2 = best.filt_parts2;
            for (int shape = 1; shape <= 4; ++shape) {
                p->tune.filt_mfma2 = shape;
                to_status st = TO_OK;
                const float t = time_ms(s, [&] {
                    if (st == TO_OK) st = launch_filter(p, dt, TO_FILTER_ADJ2, Hs, Hs, nullptr, scratch, scratch2, s);
                }, 3);
                if (st == TO_OK && t < tbest) { tbest = t; best.filt_mfma2 = shape; }
            }
        }
        p->tune.filt_parts2 = best.filt_parts2;
        p->tune.filt_mfma2 = best.filt_mfma2;
    }
    if (kval) {
        float tbest = 1e30f;
        for (int rows : {0, 1, 2})
            for (int nt : {128, 256, 512}) {
                if (rows == 2 && p->dim != 2) continue;
                p->tune.asm_rows = rows;
                p->tune.asm_block = nt;
                to_status st = TO_OK;
                const float t = time_ms(s, [&] {
                    if (st == TO_OK) st = launch_assemble(p, dt, Hs, 3.0, kval, s);
                }, 3);
                if (st == TO_OK && t < tbest) { tbest = t; best.asm_block = nt; best.asm_rows = rows; }
            }
        p->tune.asm_block = best.asm_block;
        p->tune.asm_rows = best.asm_rows;
    }
    p->tune.tuned = 1;
    TO_HIP(hipStreamSynchronize(s));
    TO_HIP(hipGetLastError());
    if (out) {
        out->filt_v = p->tune.filt_v;
        out->filt_parts = p->tune.filt_parts;
        out->asm_block = p->tune.asm_block;
        out->tuned = p->tune.tuned;
        out->filt_parts2 = p->tune.filt_parts2;
        out->filt_mfma = p->tune.filt_mfma;
        out->filt_mfma2 = p->tune.filt_mfma2;
        out->coop_launch = p->tune.coop_launch;
        out->asm_rows = p->tune.asm_rows;
    }
    return TO_OK;
}

}  // namespace topt

// ---------------------------------------------------------------------------
// C ABI
using namespace topt;

struct to_batch {
    Batch impl;
};

extern "C" {

to_status to_plan_autotune(to_plan* plan, to_dtype dtype, void* kval, to_tuning* h_out, void* stream) {
    if (!plan) { set_error("to_plan_autotune: plan is NULL"); return TO_EINVAL; }
    if (dtype != TO_F32 && dtype != TO_F64) { set_error("to_plan_autotune: bad dtype"); return TO_EINVAL; }
    try {
        return plan_autotune(topt::P(plan), dtype, kval, (hipStream_t)stream, h_out);
    } catch (...) {
        set_error("to_plan_autotune: internal error");
        return TO_EINVAL;
    }
}

to_status to_plan_set_tuning(to_plan* plan, const to_tuning* t) {
    if (!plan || !t) { set_error("to_plan_set_tuning: NULL argument"); return TO_EINVAL; }
    if ((t->filt_v != 4 && t->filt_v != 8) || t->filt_parts < 0 || t->filt_parts > 16 || t->filt_parts2 < 0 ||
        t->filt_parts2 > 16 || t->filt_mfma < 0 || t->filt_mfma > 4 || t->filt_mfma2 < 0 || t->filt_mfma2 > 4 ||
        (t->coop_launch != 0 && t->coop_launch != 1) || (t->asm_rows < 0 || t->asm_rows > 2) ||
        (t->asm_block != 128 && t->asm_block != 256 && t->asm_block != 512)) {
        set_error("to_plan_set_tuning: filt_v must be 4 or 8, filt_parts 0..16, filt_mfma 0..4, coop_launch 0 or 1, "
                  "asm_rows 0, 1 or 2, asm_block 128, 256 or 512");
        return TO_EINVAL;
    }
    Plan* p = topt::P(plan);
    p->tune.filt_v = t->filt_v;
    p->tune.filt_parts = t->filt_parts;
    p->tune.filt_parts2 = t->filt_parts2;
    p->tune.asm_block = t->asm_block;
    p->tune.tuned = t->tuned;
    p->tune.filt_mfma = t->filt_mfma;
    p->tune.filt_mfma2 = t->filt_mfma2;
    p->tune.coop_launch = t->coop_launch;
    p->tune.asm_rows = t->asm_rows;
    return TO_OK;
}

to_status to_plan_get_tuning(const to_plan* plan, to_tuning* out) {
    if (!plan || !out) { set_error("to_plan_get_tuning: NULL argument"); return TO_EINVAL; }
    const Plan* p = topt::P(plan);
    out->filt_v = p->tune.filt_v;
    out->filt_parts = p->tune.filt_parts;
    out->filt_parts2 = p->tune.filt_parts2;
    out->asm_block = p->tune.asm_block;
    out->tuned = p->tune.tuned;
    out->filt_mfma = p->tune.filt_mfma;
    out->filt_mfma2 = p->tune.filt_mfma2;
    out->coop_launch = p->tune.coop_launch;
    out->asm_rows = p->tune.asm_rows;
    return TO_OK;
}

to_status to_batch_query(int32_t count, size_t* ws_bytes) {
    if (count < 1 || count > kMaxCoopBlocks || !ws_bytes) { set_error("to_batch_query: bad count or NULL"); return TO_EINVAL; }
    *ws_bytes = batch_layout(count).total;
    return TO_OK;
}

static to_status check_state(const to_step_state& st, const to_step_params& prm) {
    if (!st.x || !st.xtilde || !st.xphys || !st.xphys_old || !st.dprj || !st.dc || !st.dcf || !st.dv || !st.dv0 ||
        !st.u || !st.f || !st.eta || !st.compliance || !st.pstats || !st.sstats || !st.ostats) {
        set_error("batch: a state buffer is NULL");
        return TO_EINVAL;
    }
    if (prm.solve.op != TO_OP_MATFREE && !st.kval) { set_error("batch: kval is NULL"); return TO_EINVAL; }
    if (prm.ft < 1 || prm.ft > 3) { set_error("batch: ft must be 1, 2 or 3"); return TO_EINVAL; }
    if (prm.oc != TO_OC_BISECT && prm.oc != TO_OC_PD) {
        set_error("batch: oc must be TO_OC_BISECT or TO_OC_PD (the filtered bisection runs one design at a time)");
        return TO_EINVAL;
    }
    if (!(prm.volfrac > 0 && prm.volfrac < 1) || !(prm.move > 0 && prm.move <= 1)) {
        set_error("batch: volfrac must be in (0, 1) and move in (0, 1]");
        return TO_EINVAL;
    }
    return TO_OK;
}

to_status to_batch_create(to_plan* const* plans, int32_t count, to_dtype dtype, const to_step_state* states,
                          const to_step_params* params, int32_t autotune, void* ws, size_t ws_bytes, void* stream,
                          to_batch** out) {
    if (!plans || !states || !params || !ws || !out || count < 1) { set_error("to_batch_create: NULL argument"); return TO_EINVAL; }
    if (dtype != TO_F32 && dtype != TO_F64) { set_error("to_batch_create: bad dtype"); return TO_EINVAL; }
    if (((uintptr_t)ws & 255u) != 0) { set_error("to_batch_create: workspace not 256-byte aligned"); return TO_EINVAL; }
    const BatchLayout Ly = batch_layout(count);
    if (ws_bytes < Ly.total) { set_error("to_batch_create: workspace too small"); return TO_EWORKSPACE; }
    hipStream_t s = (hipStream_t)stream;
    try {
        to_batch* h = new (std::nothrow) to_batch;
        if (!h) { set_error("to_batch_create: out of host memory"); return TO_EINVAL; }
        Batch& b = h->impl;
        b.n = count;
        b.dt = dtype;
        b.solve = params[0].solve;
        for (int i = 0; i < count; ++i) {
            if (!plans[i]) { delete h; set_error("to_batch_create: a plan is NULL"); return TO_EINVAL; }
            to_status r = check_state(states[i], params[i]);
            if (r != TO_OK) { delete h; return r; }
            const to_solve_opts& o = params[i].solve;
            if (o.op != b.solve.op || o.precision != b.solve.precision || o.rtol != b.solve.rtol ||
                o.maxit != b.solve.maxit || o.inner_rtol != b.solve.inner_rtol || o.zero_x0 != b.solve.zero_x0) {
                delete h;
                set_error("to_batch_create: the solve options must be the same for every design");
                return TO_EINVAL;
            }
            b.plans.push_back(topt::P(plans[i]));
            b.st0.push_back(states[i]);
            b.ft.push_back(params[i].ft);
            b.oc.push_back(params[i].oc);
        }
        b.dim = b.plans[0]->dim;
        for (Plan* p : b.plans)
            if (p->dim != b.dim) { delete h; set_error("to_batch_create: designs must all be 2D or all 3D"); return TO_EINVAL; }
        for (int i = 0; i < count; ++i)
            if (params[i].solve.precond != b.solve.precond || params[i].solve.budget != b.solve.budget) {
                delete h;
                set_error("to_batch_create: the preconditioner and the multigrid budget must be the same for every design");
                return TO_EINVAL;
            }
        if (b.solve.precond == TO_PREC_GMG) {
            if (b.solve.budget <= 0) {
                delete h;
                set_error("to_batch_create: multigrid solves in a batch need a budget (to_solve_opts.budget > 0)");
                return TO_EINVAL;
            }
            for (Plan* p : b.plans)
                if (p->gmg.L < 2) {
                    delete h; set_error("to_batch_create: a mesh is too small for a multigrid hierarchy");
                    return TO_EUNSUPPORTED;
                }
            b.gmg = true;
        }
        if (b.solve.precision == TO_SOLVE_MIXED && dtype == TO_F64) {
            delete h; set_error("to_batch_create: the mixed solve needs TO_F32 fields"); return TO_EINVAL;
        }
        b.mode = solve_mode(dtype, b.solve);
        const int num_cu = b.plans[0]->num_cu;
        char* base = (char*)ws;
        b.proj_tab = base + Ly.proj;
        b.oc_tab = base + Ly.oc;
        b.solve_tab = base + Ly.solve;
        b.dyn = (double*)(base + Ly.dyn);
        // host images of the tables and maps
        const size_t pa = project_args_bytes(dtype), oa = oc_args_bytes(dtype), sa = solve_args_bytes();
        std::vector<char> hp(pa * count), ho(oa * count), hs(sa * count);
        const size_t aa = asm_args_bytes(), sn = sens_args_bytes(), fe = filter_batch_entry_bytes();
        std::vector<char> hasm(aa * count), hsens(sn * count), hfilt(2 * fe * count);
        std::vector<int32_t> tile0(count + 1, 0);
        b.filt_fwd = base + Ly.filt;
        b.filt_adj = base + Ly.filt + fe * count;
        b.tile0 = (int32_t*)(base + Ly.tile0);
        b.asm_tab = base + Ly.asmt;
        b.sens_tab = base + Ly.sens;
        b.ctr = (unsigned*)(base + Ly.ctr);
        for (int i = 0; i < count; ++i) {
            Plan* p = b.plans[i];
            const to_step_state& st = states[i];
            double* dyn = b.dyn + kDynStride * (size_t)i;
            project_args_fill(p, dtype, params[i].ft, st.xtilde, st.x, st.xphys, st.dprj, st.eta, st.xphys_old,
                              st.pstats, dyn, hp.data() + pa * i);
            oc_args_fill(p, dtype, st.x, st.dcf, st.dv0, st.ostats, dyn, params[i].oc, ho.data() + oa * i);
            solve_args_fill(p, dtype, st.kval, st.f, st.u, b.solve, st.sstats, hs.data() + sa * i);
            asm_args_fill(p, dtype, st.xphys, st.kval, hasm.data() + aa * i);
            sens_args_fill(p, dtype, st.xphys, st.u, st.f, st.dc, st.compliance, hsens.data() + sn * i);
            filter_batch_fill(p, dtype, st.x, nullptr, nullptr, st.xtilde, nullptr, hfilt.data() + fe * i);
            filter_batch_fill(p, dtype, st.dc, st.dv, st.dprj, st.dcf, st.dv0, hfilt.data() + fe * (count + i));
            tile0[i + 1] = tile0[i] + (b.dim == 2 ? filter_batch_tiles(p) : 0);
            b.rmax = std::max(b.rmax, p->R);
        }
        b.ntiles = tile0[count];
        b.filt_batched = b.dim == 2 && filter_batch_fits(dtype, b.rmax);
        std::vector<double> wm(count), wn(count);
        std::vector<int> cap_p(count), cap_o(count), cap_s(count), cap_e(count);
        for (int i = 0; i < count; ++i) {
            const Plan* p = b.plans[i];
            wm[i] = (double)p->info.m;
            // CG iterations grow with the mesh's linear size, so a design's
            // solve work goes as (nodes)^1.5
            wn[i] = std::pow((double)p->info.nnode, 1.5);
            cap_p[i] = (int)std::min<int64_t>(num_cu, (p->info.m + kBigBlock - 1) / kBigBlock);
            cap_o[i] = (int)std::min<int64_t>(512, (p->info.m + 511) / 512);
            const int sb = solve_block_size(b.dim, b.mode);
            cap_s[i] = (int)std::min<int64_t>(kMaxCoopBlocks, (p->info.nnode + sb - 1) / sb);
            // moduli, assembly and sensitivity blocks (one compliance partial
            // per block: at most sens_batch_cap)
            cap_e[i] = (int)std::min<int64_t>(sens_batch_cap(p), (p->info.m + kBlock - 1) / kBlock);
        }
        const int gp = std::min(project_batch_capacity(dtype, num_cu), kMaxCoopBlocks);
        const int go = std::min(oc_batch_capacity(dtype, num_cu), kMaxCoopBlocks);
        const int gs = std::min(solve_batch_capacity(b.dim, b.mode, num_cu), kMaxCoopBlocks);
        if (count > std::min(gp, std::min(go, gs))) {
            delete h;
            set_error("to_batch_create: more designs than blocks that can be co-resident");
            return TO_EUNSUPPORTED;
        }
        std::vector<int32_t> maps;
        auto add_map = [&](const std::vector<double>& w, const std::vector<int>& cap, int G, BatchMap& mp,
                           int32_t* dbase) {
            std::vector<int32_t> first, cnt, inst;
            const int used = split_blocks(w, cap, G, first, cnt, inst);
            const size_t off = maps.size();
            maps.insert(maps.end(), inst.begin(), inst.end());
            const size_t off_f = maps.size();
            maps.insert(maps.end(), first.begin(), first.end());
            const size_t off_c = maps.size();
            maps.insert(maps.end(), cnt.begin(), cnt.end());
            mp.inst = dbase + off;
            mp.first = dbase + off_f;
            mp.count = dbase + off_c;
            mp.blocks = used;
        };
        int32_t* dmaps = (int32_t*)(base + Ly.maps);
        add_map(wm, cap_p, gp, b.mp_proj, dmaps);
        add_map(wm, cap_o, go, b.mp_oc, dmaps);
        add_map(wn, cap_s, gs, b.mp_solve, dmaps);
        add_map(wm, cap_e, std::max(count, std::min(kMaxCoopBlocks, 8 * num_cu)), b.mp_elem, dmaps);
        TO_HIP(hipMemcpyAsync(b.proj_tab, hp.data(), hp.size(), hipMemcpyHostToDevice, s));
        TO_HIP(hipMemcpyAsync(b.oc_tab, ho.data(), ho.size(), hipMemcpyHostToDevice, s));
        TO_HIP(hipMemcpyAsync(b.solve_tab, hs.data(), hs.size(), hipMemcpyHostToDevice, s));
        TO_HIP(hipMemcpyAsync(dmaps, maps.data(), maps.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        TO_HIP(hipMemcpyAsync(b.asm_tab, hasm.data(), hasm.size(), hipMemcpyHostToDevice, s));
        TO_HIP(hipMemcpyAsync(b.sens_tab, hsens.data(), hsens.size(), hipMemcpyHostToDevice, s));
        TO_HIP(hipMemcpyAsync(b.filt_fwd, hfilt.data(), hfilt.size(), hipMemcpyHostToDevice, s));
        TO_HIP(hipMemcpyAsync(b.tile0, tile0.data(), tile0.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        TO_HIP(hipMemsetAsync(b.ctr, 0, 256, s));
        TO_HIP(hipStreamSynchronize(s));
        if (autotune) {
            for (int i = 0; i < count; ++i) {
                if (b.plans[i]->tune.tuned) continue;
                to_status r = plan_autotune(b.plans[i], dtype, b.solve.op != TO_OP_MATFREE ? states[i].kval : nullptr,
                                            s, nullptr);
                if (r != TO_OK) { delete h; return r; }
            }
        }
        TO_HIP(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
        if (b.gmg) {
            b.side.assign(kBatchSideStreams, nullptr);
            b.ev.assign(1 + kBatchSideStreams, nullptr);
            for (auto& q : b.side) TO_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
            for (auto& e : b.ev) TO_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
        *out = h;
        return TO_OK;
    } catch (...) {
        set_error("to_batch_create: internal error");
        return TO_EINVAL;
    }
}

void to_batch_destroy(to_batch* h) {
    if (!h) return;
    if (h->impl.exec) (void)hipGraphExecDestroy(h->impl.exec);
    if (h->impl.cap) (void)hipStreamDestroy(h->impl.cap);
    for (hipStream_t q : h->impl.side) if (q) (void)hipStreamDestroy(q);
    for (hipEvent_t e : h->impl.ev) if (e) (void)hipEventDestroy(e);
    delete h;
}

to_status to_step_batched(to_batch* h, to_step_state* states, const to_step_params* params, int32_t use_graph,
                          void* stream) {
    if (!h || !states || !params) { set_error("to_step_batched: NULL argument"); return TO_EINVAL; }
    Batch& b = h->impl;
    for (int i = 0; i < b.n; ++i) {
        to_status r = check_state(states[i], params[i]);
        if (r != TO_OK) return r;
        if (!same_state(states[i], b.st0[i])) {
            set_error("to_step_batched: state buffers differ from the ones the batch was created with");
            return TO_EINVAL;
        }
        if (params[i].ft != b.ft[i] || params[i].oc != b.oc[i] || params[i].solve.op != b.solve.op ||
            params[i].solve.precision != b.solve.precision) {
            set_error("to_step_batched: ft, the OC method and the solve operator / precision are fixed at batch "
                      "creation");
            return TO_EINVAL;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    try {
        if (!use_graph) {
            to_status r = batch_enqueue(&b, states, params, s);
            if (r != TO_OK) return r;
        } else {
            std::vector<double> key;
            key.reserve(6 * b.n);
            for (int i = 0; i < b.n; ++i) {
                key.push_back(states[i].penal);
                key.push_back(states[i].beta);
                key.push_back(params[i].volfrac);
                key.push_back(params[i].move);
                key.push_back(std::isnan(params[i].target) ? -1.0 : params[i].target);
                key.push_back((double)params[i].ft);
            }
            if (!b.exec || key != b.key) {
                if (b.exec) { TO_HIP(hipGraphExecDestroy(b.exec)); b.exec = nullptr; }
                TO_HIP(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
                to_status r = batch_enqueue(&b, states, params, b.cap);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(b.cap, &g);
                if (r != TO_OK) { if (g) (void)hipGraphDestroy(g); return r; }
                if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
                e = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) { b.exec = nullptr; return hip_fail(e, "hipGraphInstantiate"); }
                b.key = key;
                ++b.graph_captures;
            }
            TO_HIP(hipGraphLaunch(b.exec, s));
            ++b.graph_launches;
        }
    } catch (...) {
        set_error("to_step_batched: internal error");
        return TO_EINVAL;
    }
    for (int i = 0; i < b.n; ++i) {
        to_step_state& st = states[i];
        st.loop += 1;
        st.penal = to_continuation(st.penal, &params[i].penal_sched, st.loop);
        st.beta = to_continuation(st.beta, &params[i].beta_sched, st.loop);
    }
    return TO_OK;
}

to_status to_batch_get_info(const to_batch* h, int32_t* h_out) {
    if (!h || !h_out) { set_error("to_batch_get_info: NULL argument"); return TO_EINVAL; }
    const Batch& b = h->impl;
    h_out[0] = b.n;
    h_out[1] = b.mp_proj.blocks;
    h_out[2] = b.mp_solve.blocks;
    h_out[3] = b.mp_oc.blocks;
    h_out[4] = b.graph_captures;
    h_out[5] = b.graph_launches;
    h_out[6] = b.mp_elem.blocks;
    h_out[7] = b.filt_batched ? 1 : 0;
    return TO_OK;
}

}  // extern "C"
