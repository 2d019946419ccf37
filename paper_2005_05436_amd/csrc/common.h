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
constexpr int kBigBlock = 512;          // persistent design-field kernels (8 wave64: 256 registers, no spills)
constexpr int kMaxCoopBlocks = 4096;    // partial-sum slots reserved per reduction
constexpr int kPartialWidth = 32;       // doubles per block in the partial buffer
constexpr unsigned kSpinLimit = 1u << 27;   // grid-barrier spin cap (~several seconds)
// Flagged partial sums (see FlagReduce): per region, block and value, two
// 64-bit words (32-bit half of the double, 32-bit tag).
constexpr int kLLVals = 4;
constexpr size_t kLLBytes = 2 * (size_t)kMaxCoopBlocks * kLLVals * 2 * 8;

// Geometric multigrid hierarchy: level l+1 has ceil(n_l / 2) elements per
// direction; coarsening stops once the level has at most kGmgCoarseMax DOFs
// (that level is inverted densely).
constexpr int kGmgMaxLevels = 16;
constexpr int kGmgCoarseMax = 128;
struct GmgShape {
    int L = 0;
    int nx[kGmgMaxLevels] = {}, ny[kGmgMaxLevels] = {}, nz[kGmgMaxLevels] = {};
};
inline int64_t gmg_dofs(int dim, int nx, int ny, int nz) {
    return (int64_t)dim * (nx + 1) * (ny + 1) * (dim == 3 ? nz + 1 : 1);
}
inline GmgShape gmg_shape(int dim, int nelx, int nely, int nelz) {
    GmgShape g;
    g.L = 1;
    g.nx[0] = nelx;
    g.ny[0] = nely;
    g.nz[0] = dim == 3 ? nelz : 1;
    while (g.L < kGmgMaxLevels) {
        const int nx = g.nx[g.L - 1], ny = g.ny[g.L - 1], nz = g.nz[g.L - 1];
        if ((gmg_dofs(dim, nx, ny, nz) <= kGmgCoarseMax && g.L >= 2) || (nx < 2 && ny < 2 && (dim == 2 || nz < 2)))
            break;
        g.nx[g.L] = (nx + 1) / 2;
        g.ny[g.L] = (ny + 1) / 2;
        g.nz[g.L] = dim == 3 ? (nz + 1) / 2 : 1;
        ++g.L;
    }
    const int t = g.L - 1;
    if (gmg_dofs(dim, g.nx[t], g.ny[t], g.nz[t]) > kGmgCoarseMax) g.L = 0;   // cannot coarsen far enough
    return g;
}
struct GmgLevel {
    int nx = 0, ny = 0, nz = 1;
    int64_t nnode = 0, n = 0, m = 0;
    double* K = nullptr;           // element matrices, (dim * 2^dim)^2 each (levels >= 1)
    double* S = nullptr;           // assembled node stencils, 3^dim * dim^2 per node, entry-major (levels >= 1)
    double *x = nullptr, *xt = nullptr, *b = nullptr, *r = nullptr, *dinv = nullptr;
};
// Device scalars of the outer flexible CG.  done: 0 iterating, 1 stopped
// (confirmed, or a cap reached), 2 breakdown.  check: the recursive residual
// reached the tolerance and waits for the true-residual confirmation.
// restart: the next direction update starts afresh (beta = 0).
struct GmgScal {
    double rz, pq, alpha, beta, rr, bnorm, tol, roz, rz_old;
    int32_t it, done, maxit, check, restarts, confirmed, restart, pad;
};
struct Gmg {
    int L = 0;
    GmgLevel lv[kGmgMaxLevels];
    double* Ainv = nullptr;        // dense inverse of the coarsest level
    GmgScal* scal = nullptr;
    // captured batches of outer iterations (first batch after a restart, and
    // the steady batch), valid for the (u, f) they were captured with
    hipStream_t cap = nullptr;
    hipGraphExec_t g_first = nullptr, g_steady = nullptr;
    const double* key_u = nullptr;
    const double* key_f = nullptr;
    ~Gmg() {
        if (g_first) (void)hipGraphExecDestroy(g_first);
        if (g_steady) (void)hipGraphExecDestroy(g_steady);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

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
    uint8_t* passive = nullptr;   // m
    uint8_t* freemask = nullptr;  // n
    // element matrix and filter (device)
    double* ke64 = nullptr;  float* ke32 = nullptr;      // d~ lower vector
    double* kf64 = nullptr;  float* kf32 = nullptr;      // d x d full
    double* h64 = nullptr;   float* h32 = nullptr;       // (2R+1)^dim, y fastest
    int32_t* hlim = nullptr;                             // per (x[,z]) column: max |dy| with h > 0
    double* hp64 = nullptr;  float* hp32 = nullptr;      // 2D: row dy of non-zero taps, zero padded
    int hp_stride = 0;
    float* hm32 = nullptr;                               // 2D: column dx of h, 16 zeros before, 19+ after
    double* hm64 = nullptr;                              // the same in FP64
    int hm_stride = 0;
    double* Hs64 = nullptr;  float* Hs32 = nullptr;      // m
    // scratch (device)
    double* E64 = nullptr;   float* E32 = nullptr;       // m
    double* partial = nullptr;                           // kMaxCoopBlocks * kPartialWidth
    unsigned long long* ll = nullptr;                    // flagged partial sums (kLLBytes)
    double* scal = nullptr;                              // 256 scalars
    unsigned* bar = nullptr;                             // barrier words (1024)
    double* v64[8] = {};                                 // n each
    float* v32[8] = {};                                  // n each
    double* fx64 = nullptr;  float* fx32 = nullptr;      // m (filter staging)

    Gmg gmg;                                             // multigrid hierarchy
    const unsigned* filt_skip = nullptr;                 // device flag: filter launches return at once when set

    // launch shapes chosen by the autotuner (or defaults)
    struct Tune {
        int filt_v = 8;        // 2D filter: output columns per tile (4 or 8)
        int filt_parts = 0;    // 2D filter: waves per block (0: automatic), one field
        int filt_parts2 = 0;   // 2D filter: waves per block for the fused double adjoint
        int asm_block = 256;   // assembly: threads per block (128, 256 or 512)
        int tuned = 0;
        int filt_mfma = 0;     // 2D FP32 filter on the matrix cores: 0 off, else the tile shape (1..4), one field
        int filt_mfma2 = 0;    // the same for the fused double adjoint
        int coop_launch = 0;   // projection and OC kernels: 0 plain launch, 1 cooperative launch
        int asm_rows = 0;      // assembly: 0 segmented sum over perm, 1 slots from the grid (no perm)
    } tune;

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

// Wave-wide sum through DPP lane moves (no LDS traffic): inclusive prefix
// sums inside each 16-lane row (shift right by 1, 2, 4, 8), then the row
// totals are carried across rows with the row broadcasts of lanes 15 and 31;
// lane 63 ends with the total, read back as a wave-uniform value.  The
// order of the additions is fixed.
template <int CTRL, int ROWS, bool BOUND>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xf, BOUND);
    const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xf, BOUND);
    return __hiloint2double(h2, l2);
}
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0x111, 0xf, true>(v);     // row_shr:1
    v += dpp_move<0x112, 0xf, true>(v);     // row_shr:2
    v += dpp_move<0x114, 0xf, true>(v);     // row_shr:4
    v += dpp_move<0x118, 0xf, true>(v);     // row_shr:8
    v += dpp_move<0x142, 0xa, false>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc, false>(v);    // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Deterministic block sum; result valid in every thread.  `sh` holds NB/64 doubles.
template <int NB = kBlock>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NB / 64; ++i) s += sh[i];
    return s;
}

// x^p with the small integer exponents of the SIMP continuation (0, 1, 2, 3)
// by products, any other exponent by pow
template <typename T>
__device__ __forceinline__ T simp_pow(T x, T p) {
    if (p == T(0)) return T(1);
    if (p == T(1)) return x;
    if (p == T(2)) return x * x;
    if (p == T(3)) return x * x * x;
    return pow(x, p);
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

// Device-coherent access without cache maintenance: relaxed atomics at agent
// scope are performed at the device coherence point (no stale L1/L2 copy),
// so data exchanged between blocks of one persistent kernel uses these and
// the grid barrier needs no agent-scope fence (on this multi-die part an
// agent-scope fence writes back and invalidates a whole L2, which made the
// barrier cost grow with the number of blocks).
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_acq(const double* p) { return ld_dev(p); }

// Reads a value that nothing writes while the kernel runs (the element
// matrix) through the constant address space: a wave-uniform address then
// becomes a scalar load even in kernels that also store to global memory,
// where the compiler cannot otherwise rule out that a store changed it.
template <typename T>
__device__ __forceinline__ T ld_const(const T* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}

// Wait until every global access this wave has issued has completed.  On gfx9
// the vector memory counter covers stores as well as loads, and a completed
// device-scope store (st_dev) is visible at the device coherence point.  A
// workgroup-scope release does not wait for it here (the waves of a block
// share one CU), so every wave that published data for other blocks waits
// before the block's arrival is signalled.  The "memory" clobber keeps the
// compiler from moving accesses across the wait.
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ unsigned ld_acq_u(const unsigned* p) { return ld_dev(p); }

// Grid-wide barrier for cooperatively launched kernels (all blocks resident).
//
// Data that crosses blocks is written and read with st_dev / ld_dev, so the
// barrier only has to order it: every wave waits for its own stores to
// complete (wait_stores) before the block arrives, and the arrival and
// release are relaxed device-scope atomics.
// Same-address atomics serialise, so arrivals are split over kBarGroups
// counters on separate cache lines (group = blockIdx % kBarGroups); the last
// arrival of a group resets it and arrives at the top word, whose low 20 bits
// count groups and high 12 bits hold the generation; the last group bumps the
// generation and clears the count with one atomic add.  Every block tracks
// the generation itself (read once at kernel start; each barrier adds one).
// Words of `bar`: [0] top, [2] abort flag, [3] error bits, [8] dot-product
// counter, [64 + 32 g] group g.
constexpr int kBarGroups = 16;

struct GridBar {
    unsigned* bar;
    unsigned gen;        // thread 0 only
    unsigned nblk, bid;  // blocks taking part and this block's index among them
    __device__ __forceinline__ void init(unsigned* b) { init(b, blockIdx.x, gridDim.x); }
    __device__ __forceinline__ void init(unsigned* b, unsigned block, unsigned nblocks) {
        bar = b;
        bid = block;
        nblk = nblocks;
        if (threadIdx.x == 0) gen = (ld_dev(&b[0]) >> 20) & 0xFFFu;
    }
    // Returns false in every thread once a block has timed out (then
    // persistent loops leave and every wave reaches the kernel's end).
    __device__ __forceinline__ bool sync() {
        __shared__ int ok_sh;
        wait_stores();
        __syncthreads();
        if (threadIdx.x == 0) {
            int ok = 1;
            const unsigned nb = nblk;
            const unsigned G = nb < (unsigned)kBarGroups ? nb : (unsigned)kBarGroups;
            const unsigned g = bid % G;
            const unsigned ng = nb / G + (g < nb % G ? 1u : 0u);
            unsigned* grp = &bar[64 + 32 * g];
            const unsigned old = atomicAdd(grp, 1u);
            if (old == ng - 1) {
                st_dev(grp, 0u);
                const unsigned o2 = atomicAdd(&bar[0], 1u);
                if ((o2 & 0xFFFFFu) == G - 1) atomicAdd(&bar[0], (1u << 20) - G);
            }
            const unsigned want = (gen + 1u) & 0xFFFu;
            unsigned spins = 0;
            while (((ld_dev(&bar[0]) >> 20) & 0xFFFu) != want) {
                if ((++spins & 255u) == 0u) {
                    if (ld_dev(&bar[2]) != 0u) { ok = 0; break; }
                    if (spins > kSpinLimit) {
                        atomicOr(&bar[3], FLAG_BARRIER_TIMEOUT);
                        atomicExch(&bar[2], 1u);
                        ok = 0;
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(1);
            }
            gen = want;
            ok_sh = ok;
        }
        __syncthreads();
        return ok_sh != 0;
    }
};

// Sum of K partial columns written by every block: partial[k*kMaxCoopBlocks + b]
// (value-major, so a wave's reads of one value from consecutive blocks coalesce).
// Every block computes the identical result (same data, same order).
// All loads are issued before the additions (one memory latency per
// reduction, not one per block); gridDim.x <= 4 * NB.
template <int K, int NB = kBlock>
__device__ __forceinline__ void grid_reduce(const double* partial, double* out_sh, double* sh, int nblocks) {
    double v[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = threadIdx.x + q * NB;
            v[k][q] = b < nblocks ? ld_acq(&partial[(size_t)k * kMaxCoopBlocks + b]) : 0.0;
        }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double s = ((v[k][0] + v[k][1]) + v[k][2]) + v[k][3];
        out_sh[k] = block_sum<NB>(s, sh);
    }
}

// Grid-wide sums without a separate barrier: every block publishes its K
// block sums as flagged words (the 32-bit halves of each double, each paired
// with a 32-bit tag in one 64-bit word, so a word is read whole or not at all)
// and every block polls all blocks' words until they carry the current tag,
// then sums them in block order (identical in every block).  Arrival and data
// travel together: one device round trip for the publication and one for the
// poll, instead of the counter atomics, the spin on the barrier word and the
// separate read of the partials.  Tags: a per-plan epoch word (bar[4]) read
// at kernel start, plus the reduction's running number; the kernel's block 0
// advances the epoch at the end.  Two regions alternate, so a block can
// publish reduction k+1 while a slower one still reads reduction k (it cannot
// get two ahead: reduction k+1 needs every block's k+1 words, written after
// that block finished reading k).
struct FlagReduce {
    unsigned long long* ll;
    unsigned* bar;
    unsigned epoch;
    int red;
    unsigned bid, nblk;
    __device__ __forceinline__ void init(unsigned long long* l, unsigned* b, unsigned block, unsigned nblocks) {
        ll = l; bar = b; bid = block; nblk = nblocks; red = 0;
        epoch = ld_dev(&b[4]);
    }
    __device__ __forceinline__ unsigned long long* region() const {
        return ll + (size_t)(red & 1) * kMaxCoopBlocks * kLLVals * 2;
    }
    __device__ __forceinline__ unsigned tag() const { return epoch + (unsigned)red + 1u; }
    __device__ __forceinline__ void waited(unsigned& spins, bool& ok) const {
        if ((++spins & 255u) == 0u) {
            if (ld_dev(&bar[2]) != 0u) ok = false;
            else if (spins > kSpinLimit) {
                atomicOr(&bar[3], FLAG_BARRIER_TIMEOUT);
                atomicExch(&bar[2], 1u);
                ok = false;
            }
        }
    }
    // Spins (one thread) until block b's record of the current grid sum
    // carries its tag: one word, the last its publisher writes (every block
    // polls every record, so the poll's request rate is what costs).
    template <int K>
    __device__ __forceinline__ void wait_record(unsigned b, bool& ok) const {
        const unsigned long long* wd = region() + (size_t)b * kLLVals * 2;
        const unsigned tg = tag();
        unsigned spins = 0;
        for (unsigned long long sent = ld_dev(wd + 2 * K - 1); ok && (unsigned)(sent >> 32) != tg;
             sent = ld_dev(wd + 2 * K - 1)) {
            waited(spins, ok);
            __builtin_amdgcn_s_sleep(2);
        }
    }
    // First half of a grid sum: the block's K partial sums (wave sums, then
    // waves in order) published as its flagged record, after every wave's
    // stores for other blocks completed (so a record also certifies them).
    // Every thread of the block calls it.
    template <int K>
    __device__ __forceinline__ void publish(const double (&v)[K]) {
        constexpr int NWMAX = 16;                      // up to 1024 threads
        __shared__ double shA[NWMAX][K];
        const int NW = (int)(blockDim.x >> 6);
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double s = wave_sum(v[k]);
            if (lane == 0) shA[w][k] = s;
        }
        // data the waves stored for other blocks (the halo band) must be
        // complete before this block's flagged words can be seen
        wait_stores();
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long* reg = region();
            const unsigned tg = tag();
#pragma unroll
            for (int k = 0; k < K; ++k) {
                double s = shA[0][k];
                for (int i = 1; i < NW; ++i) s += shA[i][k];
                const unsigned long long bits = (unsigned long long)__double_as_longlong(s);
                unsigned long long* wd = reg + ((size_t)bid * kLLVals + k) * 2;
                st_dev(wd, ((unsigned long long)tg << 32) | (bits & 0xFFFFFFFFull));
                st_dev(wd + 1, ((unsigned long long)tg << 32) | (bits >> 32));
            }
        }
    }
    // Second half: every block's record of the current grid sum, summed in
    // block order; results in out_sh[0..K) (valid in every thread); false if
    // the wait timed out or another block aborted.  A polling thread spins on
    // one word of its record, then loads the record's 2K words together and
    // reloads any without the tag.
    template <int K>
    __device__ __forceinline__ bool collect(double* out_sh, bool ok0 = true) {
        constexpr int NWMAX = 16;
        __shared__ double shB[NWMAX][K + 1];
        const int NW = (int)(blockDim.x >> 6), NB = (int)blockDim.x;
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const unsigned long long* reg = region();
        const unsigned tg = tag();
        bool ok = ok0;                                 // a caller's failed wait joins the verdict
        double acc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = 0.0;
        for (int b = threadIdx.x; b < (int)nblk; b += NB) {
            wait_record<K>((unsigned)b, ok);
            const unsigned long long* wd = reg + (size_t)b * kLLVals * 2;
            unsigned spins = 0;
            unsigned long long wv[2 * K];
#pragma unroll
            for (int h = 0; h < 2 * K; ++h) wv[h] = ld_dev(wd + h);
            while (ok) {
                bool ready = true;
#pragma unroll
                for (int h = 0; h < 2 * K; ++h) ready = ready && (unsigned)(wv[h] >> 32) == tg;
                if (ready) break;
                waited(spins, ok);
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int h = 0; h < 2 * K; ++h)
                    if ((unsigned)(wv[h] >> 32) != tg) wv[h] = ld_dev(wd + h);
            }
#pragma unroll
            for (int k = 0; k < K; ++k)
                acc[k] += __longlong_as_double((long long)((wv[2 * k + 1] << 32) | (wv[2 * k] & 0xFFFFFFFFull)));
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double s = wave_sum(acc[k]);
            if (lane == 0) shB[w][k] = s;
        }
        const bool wave_ok = __all(ok);
        if (lane == 0) shB[w][K] = wave_ok ? 1.0 : 0.0;
        __syncthreads();
        bool all_ok = true;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = shB[0][k];
            for (int i = 1; i < NW; ++i) s += shB[i][k];
            out_sh[k] = s;
        }
        for (int i = 0; i < NW; ++i) all_ok = all_ok && shB[i][K] != 0.0;
        ++red;
        return all_ok;
    }
    // K <= kLLVals; a whole grid sum: publish, then collect (two block
    // barriers).
    template <int K>
    __device__ __forceinline__ bool reduce(const double (&v)[K], double* out_sh, double* /*unused*/) {
        publish<K>(v);
        return collect<K>(out_sh);
    }
    // block 0 advances the epoch once every block has published its last sums
    __device__ __forceinline__ void finish() {
        if (bid == 0 && threadIdx.x == 0) st_dev(&bar[4], epoch + (unsigned)red);
    }
};

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
// Batched persistent kernels: block b of a launch works on instance inst[b],
// as block b - first[inst] of a group of count[inst] blocks.
struct BatchMap {
    const int32_t* inst;
    const int32_t* first;
    const int32_t* count;
    int blocks;
};
size_t project_args_bytes(to_dtype dt);
void project_args_fill(Plan* p, to_dtype dt, int ft, const void* xt, const void* x, void* xphys, void* dprj,
                       double* d_eta, const void* xold, to_project_stats* st, const double* dyn, void* dst);
int project_batch_capacity(to_dtype dt, int num_cu);
to_status launch_project_batch(to_dtype dt, const void* tab, const BatchMap& mp, hipStream_t s);
size_t oc_args_bytes(to_dtype dt);
void oc_args_fill(Plan* p, to_dtype dt, void* x, const void* dc, const void* dv, to_oc_stats* st, const double* dyn,
                  int method, void* dst);
int oc_batch_capacity(to_dtype dt, int num_cu);
to_status launch_oc_batch(to_dtype dt, const void* tab, const BatchMap& mp, hipStream_t s);
int solve_mode(to_dtype dt, const to_solve_opts& o);
to_status solve_prepare(Plan* p, to_dtype dt, const void* xphys, double penal, const to_solve_opts& o, hipStream_t s);
size_t solve_args_bytes();
void solve_args_fill(Plan* p, to_dtype dt, const void* kval, const double* f, double* u, const to_solve_opts& o,
                     to_solve_stats* st, void* dst);
int solve_batch_capacity(int dim, int mode, int num_cu);
int solve_block_size(int dim, int mode);
to_status launch_solve_batch(int dim, int mode, const void* tab, const BatchMap& mp, hipStream_t s);

// Stage launches covering every design of a batch (tables built once at
// batch creation; penal is the design's device scalar dyn[stride * i + 4]).
constexpr int kAsmBatchBlock = 256;
size_t filter_batch_entry_bytes();
int filter_batch_tiles(const Plan* p);
bool filter_batch_fits(to_dtype dt, int rmax);
void filter_batch_fill(Plan* p, to_dtype dt, const void* in, const void* in2, const void* sc, void* out, void* out2,
                       void* dst);
to_status launch_filter_batch(to_dtype dt, int mode, const void* tab, const int32_t* tile0, int n, int ntiles,
                              int rmax, int num_cu, unsigned* ctr, hipStream_t s);
size_t asm_args_bytes();
void asm_args_fill(Plan* p, to_dtype dt, const void* xphys, void* kval, void* dst);
to_status launch_moduli_batch(to_dtype dt, const void* tab, const double* dyn, int dyn_stride, const BatchMap& mp,
                              bool also64, hipStream_t s);
to_status launch_assemble_batch2d(to_dtype dt, const void* tab, const BatchMap& mp, hipStream_t s);
to_status launch_assemble_from_moduli(Plan* p, to_dtype dt, void* kval, hipStream_t s);
size_t sens_args_bytes();
int sens_batch_cap(const Plan* p);
void sens_args_fill(Plan* p, to_dtype dt, const void* xphys, const double* u, const double* f, void* dc, double* c,
                    void* dst);
to_status launch_sensitivity_batch(int dim, to_dtype dt, const void* tab, const double* dyn, int dyn_stride,
                                   const BatchMap& mp, hipStream_t s);

size_t pae_workspace_bytes(int64_t m, int mr);
to_status launch_pae(Plan* p, to_dtype dt, void* x, const void* xpre, int32_t loop, const to_pae_params& prm,
                     void* ws, double* d_gamma, hipStream_t s);
to_status plan_autotune(Plan* p, to_dtype dt, void* kval, hipStream_t s, to_tuning* out);
to_status launch_solve_gmg(Plan* p, to_dtype dt, const void* xphys, double penal, const double* f, double* u,
                           const to_solve_opts& o, to_solve_stats* st, hipStream_t s);
to_status launch_warm_start(Plan* p, to_dtype dt, const void* xphys, double penal, const double* f,
                            const double* uh, const double* up, double* u, double* coef, hipStream_t s);
to_status launch_solve(Plan* p, to_dtype dt, const void* kval, const void* xphys, double penal,
                       const double* f, double* u, const to_solve_opts& o, to_solve_stats* st,
                       hipStream_t s);
to_status launch_sensitivity(Plan* p, to_dtype dt, const void* xphys, const double* u,
                             const double* f, double penal, void* dc, double* c, hipStream_t s);
to_status launch_sensitivity_noalloc(Plan* p, to_dtype dt, const void* xphys, const double* u,
                                     const double* f, double penal, void* dc, double* c, hipStream_t s);
to_status launch_init_state(Plan* p, to_dtype dt, double volfrac, void* x, void* xphys, void* xold, void* dv,
                            double* u, hipStream_t s);
to_status launch_oc(Plan* p, to_dtype dt, void* x, const void* dc, const void* dv, double volfrac,
                    double move, to_oc_stats* st, hipStream_t s, int method = TO_OC_BISECT);
to_status launch_oc_filtered(Plan* p, to_dtype dt, int ft, void* x, const void* dc, const void* dv, double volfrac,
                             double move, double beta, const double* d_eta, to_oc_stats* st, hipStream_t s);
int coop_blocks_for(const void* kernel, int block, size_t smem, int num_cu);
// Launch of a persistent kernel whose blocks meet at grid barriers; `blocks`
// must not exceed coop_blocks_for (every block resident at once).  A plain
// launch by default (a cooperative launch costs about 17 us more here); with
// tune.coop_launch the runtime's cooperative launch, which also guarantees
// residency when other streams share the device.
hipError_t launch_resident(const Plan* p, const void* kernel, int blocks, int block, void** args, hipStream_t s);

}  // namespace topt
