"""ctypes binding of include/topt.h: argument marshalling only.

Every function keeps the C name.  Tensor arguments may be torch tensors
(their data_ptr() is passed) or plain integers (device addresses); host
arrays are numpy arrays.  A non-OK status raises ToError with the library's
own message.  There is no fallback: without the built library every call
fails loudly.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtopt.so")

TO_OK, TO_EINVAL, TO_EHIP, TO_EWORKSPACE, TO_EUNSUPPORTED = range(5)
TO_F32, TO_F64 = 0, 1
TO_ACTIVE, TO_SOLID, TO_VOID = 0, 1, 2
(TO_X_PAIRS, TO_X_PERM, TO_X_SEGPTR, TO_X_ROWPTR, TO_X_COLIDX, TO_X_HS, TO_X_KE, TO_X_FREE,
 TO_X_KERNEL) = range(9)
TO_FILTER_FWD, TO_FILTER_ADJ, TO_FILTER_ADJ2 = 0, 1, 2
TO_OP_ASSEMBLED, TO_OP_MATFREE, TO_OP_HYBRID = 0, 1, 2
TO_SOLVE_AUTO, TO_SOLVE_F64, TO_SOLVE_MIXED = 0, 1, 2
TO_OC_BISECT, TO_OC_PD, TO_OC_FILTERED = 0, 1, 2

EXPORTED = ["to_plan_query", "to_plan_create", "to_plan_destroy", "to_plan_get_info", "to_plan_export",
            "to_plan_build_host",
            "to_status_string", "to_last_error", "to_init_state", "to_filter", "to_project", "to_assemble", "to_solve",
            "to_sensitivity", "to_sensitivity_noalloc", "to_oc_update", "to_oc_update_pd", "to_oc_update_filtered", "to_step", "to_continuation", "to_warm_start",
            "to_nn_query", "to_nn_create", "to_nn_destroy", "to_nn_set_params", "to_nn_get", "to_nn_forward",
            "to_nn_backward", "to_nn_adam", "to_nn_train_step", "to_plan_autotune", "to_plan_set_tuning",
            "to_plan_get_tuning", "to_batch_query", "to_batch_create", "to_step_batched", "to_batch_get_info",
            "to_batch_destroy", "to_pae_query", "to_pae_step"]


class ToError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"topt status {status}: {msg}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nelx", C.c_int32), ("nely", C.c_int32), ("nelz", C.c_int32),
                ("E0", C.c_double), ("Emin", C.c_double), ("nu", C.c_double), ("rmin", C.c_double),
                ("bc", C.c_char), ("h_passive", C.c_void_p), ("h_fixed", C.c_void_p), ("n_fixed", C.c_int64)]


class PlanInfo(C.Structure):
    _fields_ = [("dim", C.c_int32), ("d", C.c_int32), ("dtilde", C.c_int32),
                ("m", C.c_int64), ("nnode", C.c_int64), ("n", C.c_int64), ("n_pairs", C.c_int64),
                ("nnz_lower", C.c_int64), ("n_active", C.c_int64), ("n_solid", C.c_int64),
                ("n_void", C.c_int64), ("n_free", C.c_int64), ("filter_radius", C.c_int32),
                ("coop_blocks", C.c_int32), ("workspace_bytes", C.c_size_t)]


class ProjectStats(C.Structure):
    _fields_ = [("eta", C.c_double), ("g", C.c_double), ("ch", C.c_double), ("vol", C.c_double),
                ("n_newton", C.c_int32), ("converged", C.c_int32), ("pad", C.c_int32 * 2)]


TO_PREC_JACOBI, TO_PREC_GMG = 0, 1


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("inner_rtol", C.c_double), ("maxit", C.c_int32),
                ("op", C.c_int32), ("precision", C.c_int32), ("zero_x0", C.c_int32),
                ("grid_blocks", C.c_int32), ("precond", C.c_int32), ("budget", C.c_int32), ("pad", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("residual", C.c_double), ("bnorm", C.c_double), ("iterations", C.c_int32),
                ("outer", C.c_int32), ("converged", C.c_int32), ("fallback", C.c_int32),
                ("restarts", C.c_int32), ("pad", C.c_int32)]


class OcStats(C.Structure):
    _fields_ = [("lmid", C.c_double), ("l1", C.c_double), ("l2", C.c_double), ("vol", C.c_double),
                ("n_bs", C.c_int32), ("capped", C.c_int32), ("passes", C.c_int32), ("pad", C.c_int32)]


class Sched(C.Structure):
    _fields_ = [("istart", C.c_int32), ("isteps", C.c_int32), ("maxpar", C.c_double),
                ("delta", C.c_double), ("mul", C.c_int32), ("enabled", C.c_int32)]


class StepParams(C.Structure):
    _fields_ = [("volfrac", C.c_double), ("move", C.c_double), ("ft", C.c_int32), ("oc", C.c_int32),
                ("target", C.c_double), ("penal_sched", Sched), ("beta_sched", Sched), ("solve", SolveOpts)]


class StepState(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "xtilde", "xphys", "xphys_old", "dprj", "dc", "dcf", "dv",
                                          "dv0", "kval", "u", "f", "eta", "compliance", "pstats", "sstats",
                                          "ostats")] + \
               [("penal", C.c_double), ("beta", C.c_double), ("loop", C.c_int32), ("pad", C.c_int32)]


_lib = None


class PaeParams(C.Structure):
    _fields_ = [("mr", C.c_int32), ("q", C.c_int32), ("q0", C.c_int32), ("pad", C.c_int32),
                ("alpha", C.c_double), ("xi", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("filt_v", C.c_int32), ("filt_parts", C.c_int32), ("asm_block", C.c_int32), ("tuned", C.c_int32),
                ("filt_parts2", C.c_int32), ("filt_mfma", C.c_int32), ("filt_mfma2", C.c_int32),
                ("coop_launch", C.c_int32), ("asm_rows", C.c_int32)]


def load():
    """Loads libtopt.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python -m paper_2005_05436_amd.build)")
    lib = C.CDLL(LIB_PATH)
    P, S = C.c_void_p, C.c_int
    sig = {
        "to_plan_query": (S, [C.POINTER(MeshDesc), C.POINTER(C.c_size_t)]),
        "to_plan_create": (S, [C.POINTER(MeshDesc), P, C.c_size_t, P, C.POINTER(P)]),
        "to_plan_destroy": (None, [P]),
        "to_plan_get_info": (S, [P, C.POINTER(PlanInfo)]),
        "to_plan_export": (S, [P, C.c_int, P, C.c_size_t, P]),
        "to_plan_build_host": (S, [C.POINTER(MeshDesc), C.c_int, P, C.c_size_t]),
        "to_status_string": (C.c_char_p, [S]),
        "to_last_error": (C.c_char_p, []),
        "to_init_state": (S, [P, S, C.c_double, P, P, P, P, P, P]),
        "to_filter": (S, [P, S, C.c_int, P, P, P, P, P, P]),
        "to_project": (S, [P, S, C.c_int, P, P, P, P, C.c_double, P, C.c_double, P, P, P]),
        "to_assemble": (S, [P, S, P, C.c_double, P, P]),
        "to_solve": (S, [P, S, P, P, C.c_double, P, P, C.POINTER(SolveOpts), P, P]),
        "to_sensitivity": (S, [P, S, P, P, P, C.c_double, P, P, P]),
        "to_sensitivity_noalloc": (S, [P, S, P, P, P, C.c_double, P, P, P]),
        "to_oc_update": (S, [P, S, P, P, P, C.c_double, C.c_double, P, P]),
        "to_oc_update_pd": (S, [P, S, P, P, P, C.c_double, C.c_double, P, P]),
        "to_oc_update_filtered": (S, [P, S, C.c_int, P, P, P, C.c_double, C.c_double, C.c_double, P, P, P]),
        "to_step": (S, [P, S, C.POINTER(StepState), C.POINTER(StepParams), P]),
        "to_continuation": (C.c_double, [C.c_double, C.POINTER(Sched), C.c_int32]),
        "to_warm_start": (S, [P, S, P, C.c_double, P, P, P, P, P, P]),
        "to_plan_autotune": (S, [P, S, P, C.POINTER(Tuning), P]),
        "to_plan_set_tuning": (S, [P, C.POINTER(Tuning)]),
        "to_plan_get_tuning": (S, [P, C.POINTER(Tuning)]),
        "to_batch_query": (S, [C.c_int32, C.POINTER(C.c_size_t)]),
        "to_batch_create": (S, [P, C.c_int32, S, P, P, C.c_int32, P, C.c_size_t, P, C.POINTER(P)]),
        "to_step_batched": (S, [P, P, P, C.c_int32, P]),
        "to_batch_get_info": (S, [P, C.POINTER(C.c_int32)]),
        "to_batch_destroy": (None, [P]),
        "to_pae_query": (S, [P, C.POINTER(PaeParams), C.POINTER(C.c_size_t)]),
        "to_pae_step": (S, [P, S, P, P, C.c_int32, C.POINTER(PaeParams), P, P, P]),
        "to_nn_query": (S, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_int64)]),
        "to_nn_create": (S, [P, P, C.c_size_t, C.POINTER(P)]),
        "to_nn_destroy": (None, [P]),
        "to_nn_set_params": (S, [P, P, P]),
        "to_nn_get": (S, [P, C.c_int, P, P]),
        "to_nn_forward": (S, [P, S, P, P, P, P]),
        "to_nn_backward": (S, [P, P, P, P]),
        "to_nn_adam": (S, [P, C.c_float, C.c_float, C.c_float, C.c_float, P]),
        "to_nn_train_step": (S, [P, S, P, P, P, C.c_float, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def ptr(t):
    """Device/host address of a torch tensor, numpy array or int (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    raise TypeError(f"cannot take the address of {type(t)}")


def check(status):
    if status != TO_OK:
        lib = load()
        raise ToError(status, lib.to_last_error().decode())


def stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# --- same-name wrappers ------------------------------------------------------
def to_plan_query(desc):
    n = C.c_size_t(0)
    check(load().to_plan_query(C.byref(desc), C.byref(n)))
    return n.value


def to_plan_create(desc, ws, ws_bytes, stream=None):
    out = C.c_void_p()
    check(load().to_plan_create(C.byref(desc), ptr(ws), ws_bytes, stream_ptr(stream), C.byref(out)))
    return out.value


def to_plan_destroy(plan):
    load().to_plan_destroy(plan)


def to_plan_get_info(plan):
    info = PlanInfo()
    check(load().to_plan_get_info(plan, C.byref(info)))
    return info


def to_plan_export(plan, what, dst, stream=None):
    check(load().to_plan_export(plan, what, ptr(dst), dst.nbytes, stream_ptr(stream)))
    return dst


def to_plan_build_host(desc, what, dst):
    check(load().to_plan_build_host(C.byref(desc), what, ptr(dst), dst.nbytes))
    return dst


def to_filter(plan, dtype, mode, inp, in2, s, out, out2, stream=None):
    check(load().to_filter(plan, dtype, mode, ptr(inp), ptr(in2), ptr(s), ptr(out), ptr(out2), stream_ptr(stream)))


def to_project(plan, dtype, ft, xtilde, x, xphys, dprj, beta, d_eta, target, xphys_old, d_stats, stream=None):
    check(load().to_project(plan, dtype, ft, ptr(xtilde), ptr(x), ptr(xphys), ptr(dprj), beta, ptr(d_eta),
                            target, ptr(xphys_old), ptr(d_stats), stream_ptr(stream)))


def to_assemble(plan, dtype, xphys, penal, kval, stream=None):
    check(load().to_assemble(plan, dtype, ptr(xphys), penal, ptr(kval), stream_ptr(stream)))


def to_solve(plan, dtype, kval, xphys, penal, f, u, opts, d_stats, stream=None):
    check(load().to_solve(plan, dtype, ptr(kval), ptr(xphys), penal, ptr(f), ptr(u),
                          C.byref(opts) if opts is not None else None, ptr(d_stats), stream_ptr(stream)))


def to_init_state(plan, dtype, volfrac, x, xphys, xphys_old, dv, u, stream=None):
    check(load().to_init_state(plan, dtype, volfrac, ptr(x), ptr(xphys), ptr(xphys_old), ptr(dv), ptr(u),
                               stream_ptr(stream)))


def to_sensitivity(plan, dtype, xphys, u, f, penal, dc, d_compliance, stream=None):
    check(load().to_sensitivity(plan, dtype, ptr(xphys), ptr(u), ptr(f), penal, ptr(dc), ptr(d_compliance),
                                stream_ptr(stream)))


def to_sensitivity_noalloc(plan, dtype, xphys, u, f, penal, dc, d_compliance, stream=None):
    check(load().to_sensitivity_noalloc(plan, dtype, ptr(xphys), ptr(u), ptr(f), penal, ptr(dc),
                                        ptr(d_compliance), stream_ptr(stream)))


def to_oc_update(plan, dtype, x, dc, dv, volfrac, move, d_stats, stream=None):
    check(load().to_oc_update(plan, dtype, ptr(x), ptr(dc), ptr(dv), volfrac, move, ptr(d_stats),
                              stream_ptr(stream)))


def to_oc_update_pd(plan, dtype, x, dc, dv, volfrac, move, d_stats, stream=None):
    check(load().to_oc_update_pd(plan, dtype, ptr(x), ptr(dc), ptr(dv), volfrac, move, ptr(d_stats),
                                 stream_ptr(stream)))


def to_oc_update_filtered(plan, dtype, ft, x, dc, dv, volfrac, move, beta, d_eta, d_stats, stream=None):
    check(load().to_oc_update_filtered(plan, dtype, ft, ptr(x), ptr(dc), ptr(dv), volfrac, move, beta, ptr(d_eta),
                                       ptr(d_stats), stream_ptr(stream)))


def to_step(plan, dtype, state, params, stream=None):
    check(load().to_step(plan, dtype, C.byref(state), C.byref(params), stream_ptr(stream)))


def to_continuation(par, sched, loop):
    return load().to_continuation(par, C.byref(sched), loop)


def to_warm_start(plan, dtype, xphys, penal, f, uhat, uprev, u, d_coef=None, stream=None):
    check(load().to_warm_start(plan, dtype, ptr(xphys), penal, ptr(f), ptr(uhat), ptr(uprev), ptr(u), ptr(d_coef),
                               stream_ptr(stream)))


def to_pae_query(plan, params):
    ws = C.c_size_t(0)
    check(load().to_pae_query(plan, C.byref(params), C.byref(ws)))
    return ws.value


def to_pae_step(plan, dtype, x, x_pre, loop, params, ws, d_gamma=None, stream=None):
    check(load().to_pae_step(plan, dtype, ptr(x), ptr(x_pre), loop, C.byref(params), ptr(ws), ptr(d_gamma),
                             stream_ptr(stream)))


TO_NN_PARAMS, TO_NN_GRAD, TO_NN_OUTPUT, TO_NN_ACT, TO_NN_PRESKIP = 0, 1, 2, 16, 32


def to_nn_query(dim, nelx, nely, nelz=1):
    ws = C.c_size_t(0)
    npar = C.c_int64(0)
    check(load().to_nn_query(dim, nelx, nely, nelz, C.byref(ws), C.byref(npar)))
    return ws.value, npar.value


def to_nn_create(plan, ws_ptr, ws_bytes):
    out = C.c_void_p()
    check(load().to_nn_create(plan, ws_ptr, ws_bytes, C.byref(out)))
    return out


def to_nn_destroy(nn):
    load().to_nn_destroy(nn)


def to_nn_set_params(nn, params, stream=None):
    check(load().to_nn_set_params(nn, ptr(params), stream_ptr(stream)))


def to_nn_get(nn, what, out, stream=None):
    check(load().to_nn_get(nn, what, ptr(out), stream_ptr(stream)))


def to_nn_forward(nn, dtype, xtilde, f, uhat, stream=None):
    check(load().to_nn_forward(nn, dtype, ptr(xtilde), ptr(f), ptr(uhat), stream_ptr(stream)))


def to_nn_backward(nn, u, d_loss=None, stream=None):
    check(load().to_nn_backward(nn, ptr(u), ptr(d_loss), stream_ptr(stream)))


def to_nn_adam(nn, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(load().to_nn_adam(nn, lr, beta1, beta2, eps, stream_ptr(stream)))


def to_nn_train_step(nn, dtype, xtilde, f, u, lr, d_loss=None, stream=None):
    check(load().to_nn_train_step(nn, dtype, ptr(xtilde), ptr(f), ptr(u), lr, ptr(d_loss), stream_ptr(stream)))


def to_plan_autotune(plan, dtype, kval=None, stream=None):
    t = Tuning()
    check(load().to_plan_autotune(plan, dtype, ptr(kval), C.byref(t), stream_ptr(stream)))
    return t


def to_plan_set_tuning(plan, filt_v=8, filt_parts=0, asm_block=256, tuned=0, filt_parts2=None, filt_mfma=0,
                       filt_mfma2=None, coop_launch=0, asm_rows=0):
    p2 = filt_parts if filt_parts2 is None else filt_parts2
    m2 = filt_mfma if filt_mfma2 is None else filt_mfma2
    check(load().to_plan_set_tuning(plan, C.byref(Tuning(filt_v, filt_parts, asm_block, tuned, p2, filt_mfma, m2,
                                                         coop_launch, asm_rows))))


def to_plan_get_tuning(plan):
    t = Tuning()
    check(load().to_plan_get_tuning(plan, C.byref(t)))
    return t


def to_batch_query(count):
    n = C.c_size_t(0)
    check(load().to_batch_query(count, C.byref(n)))
    return n.value


def to_batch_create(plans, dtype, states, params, autotune, ws_ptr, ws_bytes, stream=None):
    """plans: list of plan handles; states / params: ctypes arrays of StepState / StepParams."""
    arr = (C.c_void_p * len(plans))(*[p.value if isinstance(p, C.c_void_p) else p for p in plans])
    out = C.c_void_p()
    check(load().to_batch_create(arr, len(plans), dtype, C.cast(states, C.c_void_p), C.cast(params, C.c_void_p),
                                 1 if autotune else 0, ws_ptr, ws_bytes, stream_ptr(stream), C.byref(out)))
    return out


def to_step_batched(batch, states, params, use_graph=False, stream=None):
    check(load().to_step_batched(batch, C.cast(states, C.c_void_p), C.cast(params, C.c_void_p),
                                 1 if use_graph else 0, stream_ptr(stream)))


def to_batch_get_info(batch):
    out = (C.c_int32 * 8)()
    check(load().to_batch_get_info(batch, out))
    return dict(designs=out[0], project_blocks=out[1], solve_blocks=out[2], oc_blocks=out[3],
                graph_captures=out[4], graph_launches=out[5], element_blocks=out[6], filter_batched=bool(out[7]))


def to_batch_destroy(batch):
    load().to_batch_destroy(batch)
