// extern "C" entry points of libtopt: argument validation, error reporting,
// and the one-iteration driver to_step (blocks RL.1-RL.4 of both codes).
#include <cmath>
#include <exception>
#include <string>

#include "common.h"

namespace topt {

static thread_local std::string g_err;

void set_error(const std::string& s) { g_err = s; }

to_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return TO_EHIP;
}

to_status plan_query(const to_mesh_desc* desc, size_t* ws);
to_status plan_create(const to_mesh_desc* D, void* ws, size_t ws_bytes, hipStream_t stream, to_plan** out);
to_status plan_export(const to_plan* plan, int what, void* dst, size_t bytes, hipStream_t stream);
to_status plan_build_host(const to_mesh_desc* D, int what, void* dst, size_t bytes);

}  // namespace topt

using namespace topt;

#define TO_GUARD(expr)                                             \
    try {                                                          \
        return (expr);                                             \
    } catch (const std::exception& ex) {                           \
        set_error(std::string("internal error: ") + ex.what());    \
        return TO_EINVAL;                                          \
    } catch (...) {                                                \
        set_error("internal error");                               \
        return TO_EINVAL;                                          \
    }

#define NEED(ptr, name)                                            \
    do {                                                           \
        if (!(ptr)) { set_error(name " is NULL"); return TO_EINVAL; } \
    } while (0)

static inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

static to_status check_dtype(to_dtype d) {
    if (d != TO_F32 && d != TO_F64) { set_error("dtype must be TO_F32 or TO_F64"); return TO_EINVAL; }
    return TO_OK;
}

extern "C" {

const char* to_status_string(to_status s) {
    switch (s) {
    case TO_OK: return "ok";
    case TO_EINVAL: return "invalid argument";
    case TO_EHIP: return "HIP runtime error";
    case TO_EWORKSPACE: return "workspace too small or misaligned";
    case TO_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* to_last_error(void) { return g_err.c_str(); }

to_status to_plan_query(const to_mesh_desc* desc, size_t* ws_bytes) { TO_GUARD(plan_query(desc, ws_bytes)); }

to_status to_plan_create(const to_mesh_desc* desc, void* ws, size_t ws_bytes, void* stream, to_plan** out) {
    TO_GUARD(plan_create(desc, ws, ws_bytes, S(stream), out));
}

void to_plan_destroy(to_plan* plan) { delete P(plan); }

to_status to_plan_get_info(const to_plan* plan, to_plan_info* out) {
    NEED(plan, "plan");
    NEED(out, "out");
    *out = P(plan)->info;
    return TO_OK;
}

to_status to_plan_export(const to_plan* plan, int what, void* h_dst, size_t dst_bytes, void* stream) {
    TO_GUARD(plan_export(plan, what, h_dst, dst_bytes, S(stream)));
}

to_status to_plan_build_host(const to_mesh_desc* desc, int what, void* h_dst, size_t dst_bytes) {
    TO_GUARD(plan_build_host(desc, what, h_dst, dst_bytes));
}

to_status to_filter(const to_plan* plan, to_dtype dtype, int mode, const void* in, const void* in2,
                    const void* s, void* out, void* out2, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(in, "in");
    NEED(out, "out");
    if (mode == TO_FILTER_ADJ2) { NEED(in2, "in2"); NEED(out2, "out2"); }
    else if (mode != TO_FILTER_FWD && mode != TO_FILTER_ADJ) { set_error("bad filter mode"); return TO_EINVAL; }
    if (out == in || (mode == TO_FILTER_ADJ2 && (out2 == in || out2 == in2 || out == in2 || out == out2))) {
        set_error("filter outputs may not alias inputs"); return TO_EINVAL;
    }
    TO_GUARD(launch_filter(P(plan), dtype, mode, in, in2, s, out, out2, S(stream)));
}

to_status to_project(const to_plan* plan, to_dtype dtype, int ft, const void* xtilde, const void* x, void* xphys,
                     void* dprj, double beta, double* d_eta, double target, const void* xphys_old,
                     to_project_stats* d_stats, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(xtilde, "xtilde"); NEED(xphys, "xphys"); NEED(dprj, "dprj"); NEED(d_eta, "d_eta"); NEED(d_stats, "d_stats");
    if (ft < 1 || ft > 3) { set_error("ft must be 1, 2 or 3"); return TO_EINVAL; }
    if (ft >= 2 && !(beta > 0 && std::isfinite(beta))) { set_error("beta must be positive"); return TO_EINVAL; }
    if (xphys == xtilde || xphys == xphys_old) { set_error("xphys may not alias xtilde or xphys_old"); return TO_EINVAL; }
    TO_GUARD(launch_project(P(plan), dtype, ft, xtilde, x, xphys, dprj, beta, d_eta, target, xphys_old, d_stats,
                            S(stream)));
}

to_status to_assemble(const to_plan* plan, to_dtype dtype, const void* xphys, double penal, void* kval,
                      void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(xphys, "xphys"); NEED(kval, "kval");
    if (!(penal >= 0 && std::isfinite(penal))) { set_error("penal must be finite and >= 0"); return TO_EINVAL; }
    TO_GUARD(launch_assemble(P(plan), dtype, xphys, penal, kval, S(stream)));
}

static to_solve_opts default_opts() {
    to_solve_opts o;
    o.rtol = 1e-8; o.inner_rtol = 0.1; o.maxit = 200000; o.op = TO_OP_ASSEMBLED;
    o.precision = TO_SOLVE_AUTO; o.zero_x0 = 0; o.grid_blocks = 0; o.precond = TO_PREC_JACOBI;
    o.budget = 0; o.pad = 0;
    return o;
}

to_status to_solve(const to_plan* plan, to_dtype dtype, const void* kval, const void* xphys, double penal,
                   const double* f, double* u, const to_solve_opts* h_opts, to_solve_stats* d_stats, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(f, "f"); NEED(u, "u"); NEED(d_stats, "d_stats");
    to_solve_opts o = h_opts ? *h_opts : default_opts();
    if (!(o.rtol > 0) || !(o.inner_rtol > 0 && o.inner_rtol < 1) || o.maxit < 0 || o.grid_blocks < 0 ||
        (o.op != TO_OP_ASSEMBLED && o.op != TO_OP_MATFREE && o.op != TO_OP_HYBRID) ||
        (o.precision != TO_SOLVE_AUTO && o.precision != TO_SOLVE_F64 && o.precision != TO_SOLVE_MIXED) ||
        (o.precision == TO_SOLVE_MIXED && dtype == TO_F64) || (o.precond != TO_PREC_JACOBI && o.precond != TO_PREC_GMG) || o.budget < 0 || o.budget > 1000000) {
        set_error("bad solve options"); return TO_EINVAL;
    }
    if ((o.op != TO_OP_ASSEMBLED || dtype == TO_F32) && !xphys) { set_error("xphys is NULL"); return TO_EINVAL; }
    if ((const void*)f == (const void*)u) { set_error("f and u may not alias"); return TO_EINVAL; }
    TO_GUARD(launch_solve(P(plan), dtype, kval, xphys, penal, f, u, o, d_stats, S(stream)));
}

to_status to_warm_start(const to_plan* plan, to_dtype dtype, const void* xphys, double penal, const double* f,
                        const double* uhat, const double* uprev, double* u, double* d_coef, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(xphys, "xphys"); NEED(f, "f"); NEED(uhat, "uhat"); NEED(uprev, "uprev"); NEED(u, "u");
    if ((const void*)u == (const void*)uhat || (const void*)u == (const void*)f) {
        set_error("u may alias uprev only"); return TO_EINVAL;
    }
    TO_GUARD(launch_warm_start(P(plan), dtype, xphys, penal, f, uhat, uprev, u, d_coef, S(stream)));
}

to_status to_init_state(const to_plan* plan, to_dtype dtype, double volfrac, void* x, void* xphys, void* xphys_old,
                        void* dv, double* u, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(x, "x");
    if (!(volfrac > 0 && volfrac < 1)) { set_error("volfrac must be in (0, 1)"); return TO_EINVAL; }
    const to_plan_info& I = P(plan)->info;
    if (I.n_active == 0) { set_error("the plan has no active element"); return TO_EINVAL; }
    const double xa = (volfrac * (double)(I.m - I.n_void) - (double)I.n_solid) / (double)I.n_active;
    if (!(xa >= 0.0 && xa <= 1.0)) {
        set_error("volfrac cannot be met with designs in [0, 1] on the active set (passive elements fix too much)");
        return TO_EINVAL;
    }
    TO_GUARD(launch_init_state(P(plan), dtype, volfrac, x, xphys, xphys_old, dv, u, S(stream)));
}

to_status to_sensitivity(const to_plan* plan, to_dtype dtype, const void* xphys, const double* u, const double* f,
                         double penal, void* dc, double* d_compliance, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(xphys, "xphys"); NEED(u, "u"); NEED(dc, "dc");
    TO_GUARD(launch_sensitivity(P(plan), dtype, xphys, u, f, penal, dc, d_compliance, S(stream)));
}

to_status to_sensitivity_noalloc(const to_plan* plan, to_dtype dtype, const void* xphys, const double* u,
                                 const double* f, double penal, void* dc, double* d_compliance, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(xphys, "xphys"); NEED(u, "u"); NEED(dc, "dc");
    TO_GUARD(launch_sensitivity_noalloc(P(plan), dtype, xphys, u, f, penal, dc, d_compliance, S(stream)));
}

to_status to_oc_update(const to_plan* plan, to_dtype dtype, void* x, const void* dc, const void* dv, double volfrac,
                       double move, to_oc_stats* d_stats, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(x, "x"); NEED(dc, "dc"); NEED(dv, "dv"); NEED(d_stats, "d_stats");
    if (!(volfrac > 0 && volfrac < 1)) { set_error("volfrac must be in (0, 1)"); return TO_EINVAL; }
    if (!(move > 0 && move <= 1)) { set_error("move must be in (0, 1]"); return TO_EINVAL; }
    TO_GUARD(launch_oc(P(plan), dtype, x, dc, dv, volfrac, move, d_stats, S(stream)));
}

to_status to_oc_update_pd(const to_plan* plan, to_dtype dtype, void* x, const void* dc, const void* dv,
                          double volfrac, double move, to_oc_stats* d_stats, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(x, "x"); NEED(dc, "dc"); NEED(dv, "dv"); NEED(d_stats, "d_stats");
    if (!(volfrac > 0 && volfrac < 1)) { set_error("volfrac must be in (0, 1)"); return TO_EINVAL; }
    if (!(move > 0 && move <= 1)) { set_error("move must be in (0, 1]"); return TO_EINVAL; }
    TO_GUARD(launch_oc(P(plan), dtype, x, dc, dv, volfrac, move, d_stats, S(stream), TO_OC_PD));
}

to_status to_oc_update_filtered(const to_plan* plan, to_dtype dtype, int ft, void* x, const void* dc, const void* dv,
                                double volfrac, double move, double beta, const double* d_eta, to_oc_stats* d_stats,
                                void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(x, "x"); NEED(dc, "dc"); NEED(dv, "dv"); NEED(d_stats, "d_stats");
    if (ft < 1 || ft > 3) { set_error("ft must be 1, 2 or 3"); return TO_EINVAL; }
    if (ft > 1) NEED(d_eta, "d_eta");
    if (ft > 1 && !(beta > 0 && std::isfinite(beta))) { set_error("beta must be positive and finite"); return TO_EINVAL; }
    if (!(volfrac > 0 && volfrac < 1)) { set_error("volfrac must be in (0, 1)"); return TO_EINVAL; }
    if (!(move > 0 && move <= 1)) { set_error("move must be in (0, 1]"); return TO_EINVAL; }
    TO_GUARD(launch_oc_filtered(P(plan), dtype, ft, x, dc, dv, volfrac, move, beta, d_eta, d_stats, S(stream)));
}

static bool pae_params_ok(const to_pae_params* q) {
    return q && q->mr >= 1 && q->mr <= 8 && q->q >= 1 && q->q0 >= 0 && std::isfinite(q->alpha) &&
           std::isfinite(q->xi);
}

to_status to_pae_query(const to_plan* plan, const to_pae_params* prm, size_t* ws_bytes) {
    NEED(plan, "plan"); NEED(ws_bytes, "ws_bytes");
    if (!pae_params_ok(prm)) { set_error("pae: mr must be 1..8, q >= 1, q0 >= 0, alpha and xi finite"); return TO_EINVAL; }
    *ws_bytes = pae_workspace_bytes(P(plan)->info.m, prm->mr);
    return TO_OK;
}

to_status to_pae_step(const to_plan* plan, to_dtype dtype, void* x, const void* x_pre, int32_t loop,
                      const to_pae_params* prm, void* ws, double* d_gamma, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(x, "x"); NEED(x_pre, "x_pre"); NEED(ws, "ws");
    if (!pae_params_ok(prm)) { set_error("pae: mr must be 1..8, q >= 1, q0 >= 0, alpha and xi finite"); return TO_EINVAL; }
    if (x == x_pre) { set_error("pae: x and x_pre may not alias"); return TO_EINVAL; }
    TO_GUARD(launch_pae(P(plan), dtype, x, x_pre, loop, *prm, ws, d_gamma, S(stream)));
}

double to_continuation(double par, const to_sched* s, int32_t loop) {
    if (!s || !s->enabled || s->isteps <= 0) return par;
    if (loop >= s->istart && par < s->maxpar && loop % s->isteps == 0) return s->mul ? par * s->delta : par + s->delta;
    return par;
}

to_status to_step(const to_plan* plan, to_dtype dtype, to_step_state* st, const to_step_params* prm, void* stream) {
    NEED(plan, "plan");
    if (check_dtype(dtype)) return TO_EINVAL;
    NEED(st, "state"); NEED(prm, "params");
    NEED(st->x, "x"); NEED(st->xtilde, "xtilde"); NEED(st->xphys, "xphys"); NEED(st->xphys_old, "xphys_old");
    NEED(st->dprj, "dprj"); NEED(st->dc, "dc"); NEED(st->dcf, "dcf"); NEED(st->dv, "dv"); NEED(st->dv0, "dv0");
    NEED(st->u, "u"); NEED(st->f, "f"); NEED(st->eta, "eta"); NEED(st->compliance, "compliance");
    NEED(st->pstats, "pstats"); NEED(st->sstats, "sstats"); NEED(st->ostats, "ostats");
    if (prm->ft < 1 || prm->ft > 3) { set_error("ft must be 1, 2 or 3"); return TO_EINVAL; }
    if (prm->oc < TO_OC_BISECT || prm->oc > TO_OC_FILTERED) { set_error("oc must be TO_OC_BISECT, TO_OC_PD or TO_OC_FILTERED"); return TO_EINVAL; }
    // op TO_OP_ASSEMBLED or TO_OP_HYBRID: K^(s) is assembled every
    // iteration; it is the CG operator (TO_OP_ASSEMBLED with FP64 fields, or
    // the mixed scheme) or the source of the Jacobi preconditioner of the
    // matrix-free FP64 solve (TO_OP_HYBRID; TO_OP_ASSEMBLED with FP32 fields)
    const bool assembled = prm->solve.op != TO_OP_MATFREE;
    if (assembled) NEED(st->kval, "kval");
    try {
        Plan* p = P(plan);
        hipStream_t s = S(stream);
        to_status r;
        const size_t bytes = (dtype == TO_F64 ? 8 : 4) * (size_t)p->info.m;
        // RL.1: filter, projection, change
        if ((r = launch_filter(p, dtype, TO_FILTER_FWD, st->x, nullptr, nullptr, st->xtilde, nullptr, s))) return r;
        const double target = std::isnan(prm->target) ? prm->volfrac : prm->target;
        if ((r = launch_project(p, dtype, prm->ft, st->xtilde, st->x, st->xphys, st->dprj, st->beta, st->eta, target,
                                st->xphys_old, st->pstats, s)))
            return r;
        // RL.2: assembly and solve
        if (assembled && (r = launch_assemble(p, dtype, st->xphys, st->penal, st->kval, s))) return r;
        if ((r = launch_solve(p, dtype, st->kval, st->xphys, st->penal, st->f, st->u, prm->solve, st->sstats, s)))
            return r;
        // RL.3: sensitivities, compliance, back-filter of dc and dV
        if ((r = launch_sensitivity(p, dtype, st->xphys, st->u, st->f, st->penal, st->dc, st->compliance, s))) return r;
        if ((r = launch_filter(p, dtype, TO_FILTER_ADJ2, st->dc, st->dv, st->dprj, st->dcf, st->dv0, s))) return r;
        // RL.4: OC, then continuation
        if (prm->oc == TO_OC_FILTERED)
            r = launch_oc_filtered(p, dtype, prm->ft, st->x, st->dcf, st->dv0, prm->volfrac, prm->move, st->beta,
                                   st->eta, st->ostats, s);
        else
            r = launch_oc(p, dtype, st->x, st->dcf, st->dv0, prm->volfrac, prm->move, st->ostats, s, prm->oc);
        if (r) return r;
        TO_HIP(hipMemcpyAsync(st->xphys_old, st->xphys, bytes, hipMemcpyDeviceToDevice, s));
        st->loop += 1;
        st->penal = to_continuation(st->penal, &prm->penal_sched, st->loop);
        st->beta = to_continuation(st->beta, &prm->beta_sched, st->loop);
        return TO_OK;
    } catch (const std::exception& ex) {
        set_error(std::string("internal error: ") + ex.what());
        return TO_EINVAL;
    } catch (...) {
        set_error("internal error");
        return TO_EINVAL;
    }
}

}  // extern "C"
