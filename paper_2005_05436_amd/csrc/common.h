// Internal definitions shared by the HIP translation units of libtopt.
// Everything here is gfx950-only: 64-wide wavefronts, 256-thread blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <string>
#include <vector>

#include "../../include/topt.h"

namespace topt {

constexpr int kBlock = 256;             // threads per block (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxCoopBlocks = 4096;    // partial-sum slots reserved per reduction
constexpr int kPartialWidth = 32;       // doubles per block in the partial buffer
constexpr unsigned kSpinLimit = 1u << 27;   // grid-barrier spin cap (~several seconds)

// Device error bits written to plan->flags (never host-visible errors).
enum : unsigned { FLAG_BARRIER_TIMEOUT = 1u, FLAG_NONFINITE = 2u };

// ---------------------------------------------------------------------------
// Plan: host header with device views into the caller's workspace.
struct Plan {
    to_plan_info info{};
    int dim = 2, nelx = 0, nely = 0, nelz = 1, d = 8, dt = 36, R = 0;
    double E0 = 1, Emin = 1e-9, nu = 0.3, rmin = 1;
    char bc = 'D';
    int num_cu = 256;

    // mesh / sparse pattern (device)
    int32_t* perm = nullptr;      // n_pairs
    int32_t* seg_ptr = nullptr;   // nnz+1
    int32_t* row_ptr = nullptr;   // n+1
    int32_t* col_idx = nullptr;   // nnz
    int32_t* tptr = nullptr;      // n+1   strictly-lower entries grouped by column
    int32_t* tslot = nullptr;     // nnz-n slot of each strictly-lower entry, by column
    int32_t* trow = nullptr;      // nnz-n its row
    uint8_t* passive = nullptr;   // m
    uint8_t* freemask = nullptr;  // n
    // element matrix and filter (device)
    double* ke64 = nullptr;  float* ke32 = nullptr;      // d~ lower vector
    double* kf64 = nullptr;  float* kf32 = nullptr;      // d x d full
    double* h64 = nullptr;   float* h32 = nullptr;       // (2R+1)^dim, y fastest
    int32_t* hlim = nullptr;                             // per (x[,z]) column: max |dy| with h > 0
    double* Hs64 = nullptr;  float* Hs32 = nullptr;      // m
    // scratch (device)
    double* E64 = nullptr;   float* E32 = nullptr;       // m
    double* partial = nullptr;                           // kMaxCoopBlocks * kPartialWidth
    double* scal = nullptr;                              // 256 scalars
    unsigned* bar = nullptr;                             // barrier counters (16 words)
    double* v64[8] = {};                                 // n each
    float* v32[8] = {};                                  // n each
    double* fx64 = nullptr;  float* fx32 = nullptr;      // m (filter staging)

    // host copies
    std::vector<double> ke_lower, ke_full, h;
    std::vector<int32_t> hlim_host;
    size_t ws_bytes = 0;
};

inline Plan* P(const to_plan* p) { return reinterpret_cast<Plan*>(const_cast<to_plan*>(p)); }

// error reporting (api.cpp)
void set_error(const std::string& s);
to_status hip_fail(hipError_t e, const char* what);

#define TO_HIP(call)                                                    \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) return ::topt::hip_fail(_e, #call);       \
    } while (0)

// ---------------------------------------------------------------------------
// Device helpers
#if defined(__HIPCC__)

template <typename T> struct Acc { using type = T; };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Deterministic block sum; result valid in every thread.  `sh` holds kWaves doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) s += sh[i];
    return s;
}

// double-double (error-free) accumulation for the OC volume sums
struct dd { double hi, lo; };
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    double s = a.hi + b.hi;
    double bb = s - a.hi;
    double e = (a.hi - (s - bb)) + (b.hi - bb);
    e += a.lo + b.lo;
    double hi = s + e;
    return dd{hi, e - (hi - s)};
}
__device__ __forceinline__ dd dd_add1(dd a, double b) { return dd_add(a, dd{b, 0.0}); }
__device__ __forceinline__ dd dd_shfl_down(dd v, int off) {
    return dd{__shfl_down(v.hi, off, 64), __shfl_down(v.lo, off, 64)};
}
__device__ __forceinline__ dd wave_dd_sum(dd v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = dd_add(v, dd_shfl_down(v, off));
    return v;
}

__device__ __forceinline__ double ld_acq(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_acq_u(const unsigned* p) {
    return __hip_atomic_load(const_cast<unsigned*>(p), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier for cooperatively launched kernels (all blocks resident).
// bar[0] = arrival count, bar[1] = generation, bar[2] = abort flag, bar[3] = error bits.
// Returns false (in every thread of the block) once any block has timed out,
// so persistent loops can leave and every wave reaches the kernel's end.
__device__ __forceinline__ bool grid_sync(unsigned* bar) {
    __shared__ int ok_sh;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned g = ld_acq_u(&bar[1]);
        __threadfence();
        unsigned arrived = atomicAdd(&bar[0], 1u);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (ld_acq_u(&bar[1]) == g) {
                if (ld_acq_u(&bar[2]) != 0u) { ok = 0; break; }
                if (++spins > kSpinLimit) {
                    atomicOr(&bar[3], FLAG_BARRIER_TIMEOUT);
                    atomicExch(&bar[2], 1u);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __threadfence();
        if (ld_acq_u(&bar[2]) != 0u) ok = 0;
        ok_sh = ok;
    }
    __syncthreads();
    return ok_sh != 0;
}

// Sum of K partial columns written by every block: partial[b*kPartialWidth + k].
// Every block computes the identical result (same data, same order).
template <int K>
__device__ __forceinline__ void grid_reduce(const double* partial, double* out_sh, double* sh) {
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) s += ld_acq(&partial[b * kPartialWidth + k]);
        out_sh[k] = block_sum(s, sh);
    }
}

#endif  // __HIPCC__

// ---------------------------------------------------------------------------
// Host-side launchers implemented in the kernel translation units.
to_status launch_fill_hs(Plan* p, hipStream_t s);
to_status launch_filter(Plan* p, to_dtype dt, int mode, const void* in, const void* in2,
                        const void* sc, void* out, void* out2, hipStream_t s);
to_status launch_project(Plan* p, to_dtype dt, int ft, const void* xt, const void* x, void* xphys,
                         void* dprj, double beta, double* d_eta, double target,
                         const void* xold, to_project_stats* st, hipStream_t s);
to_status launch_assemble(Plan* p, to_dtype dt, const void* xphys, double penal, void* kval,
                          hipStream_t s);
to_status launch_moduli(Plan* p, to_dtype dt, const void* xphys, double penal, hipStream_t s, bool also64);
to_status launch_solve(Plan* p, to_dtype dt, const void* kval, const void* xphys, double penal,
                       const double* f, double* u, const to_solve_opts& o, to_solve_stats* st,
                       hipStream_t s);
to_status launch_sensitivity(Plan* p, to_dtype dt, const void* xphys, const double* u,
                             const double* f, double penal, void* dc, double* c, hipStream_t s);
to_status launch_oc(Plan* p, to_dtype dt, void* x, const void* dc, const void* dv, double volfrac,
                    double move, to_oc_stats* st, hipStream_t s);
int coop_blocks_for(const void* kernel, int block, size_t smem, int num_cu);

}  // namespace topt
