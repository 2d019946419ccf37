// OC update with bisection on sqrt(lambda) (eq. (10)-(11), bracket from
// eq. (19); block RL.4 of the 2D code), as one persistent, cooperatively
// launched kernel.
//
// Bisection is a chain of decisions mean(x(lmid)) > volfrac.  Instead of one
// grid-wide reduction per step, each sweep over the design evaluates the 15
// midpoints of the next four levels of the bisection tree (each candidate's
// bracket follows from (l1, l2) by the same midpoint arithmetic the serial
// loop would do) and sums the candidate volumes; the blocks then walk the tree
// with the same stop test as the serial loop.  The decisions, the midpoints
// and the final design are therefore exactly those of plain bisection, with
// four times fewer grid barriers.  Volume sums are double-double, so every
// decision agrees with an exactly rounded sum except in exact ties.
#include <cmath>
#include <cstring>
#include <type_traits>

#include "common.h"

namespace topt {

constexpr int kLevels = 4;
constexpr int kCand = (1 << kLevels) - 1;   // 15 midpoints per sweep

__device__ __forceinline__ double oc_clamp(double ocp, double lm, double x, double move) {
    // max(max(min(min(ocP/lmid, xU), 1), xL), 0) with xU = x + move, xL = x - move
    double v = ocp / lm;
    v = fmin(v, x + move);
    v = fmin(v, 1.0);
    v = fmax(v, x - move);
    v = fmax(v, 0.0);
    return v;
}

constexpr int kOcBlock = 512;   // 15 double-double accumulators per lane need the register room

template <typename T>
struct OcArgs {
    int64_t m;
    const uint8_t* pas;
    T* x;
    const T* dc;
    const T* dv;
    double volfrac, move;
    double* ocp_buf;
    to_oc_stats* st;
    double* partial;
    unsigned* bar;
    const double* dyn;      // batch: device (volfrac, move) at dyn[2], dyn[3] (nullable)
};

// The update of one design, run by `nb` blocks of which this is `bid`.
template <typename T>
__device__ void oc_body(const OcArgs<T>& A, int bid, int nb) {
    constexpr int NB = kOcBlock, NW = NB / 64;
    __shared__ double wsum[NW * kCand * 2];
    __shared__ double gsum[NB * 2];
    __shared__ double tot[2 * kCand];
    const int64_t m = A.m;
    const uint8_t* __restrict__ pas = A.pas;
    T* __restrict__ x = A.x;
    const T* __restrict__ dc = A.dc;
    const T* __restrict__ dv = A.dv;
    const double volfrac = A.dyn ? A.dyn[2] : A.volfrac, move = A.dyn ? A.dyn[3] : A.move;
    double* __restrict__ ocp_buf = A.ocp_buf;
    double* partial = A.partial;
    const int64_t stride = (int64_t)nb * NB;
    const int64_t i0 = (int64_t)bid * NB + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    bool alive = true;
    int region = 0;
    GridBar gb;
    gb.init(A.bar, bid, nb);

    // Block-level double-double sums of K values (K compile-time, unrolled so
    // v stays in registers): every wave reduces all K with shuffles, one
    // barrier, then thread k combines the NW wave results of value k in wave
    // order and writes the block's partial.
    auto block_dd = [&](auto& v, auto kconst, double* reg) {
        constexpr int K = decltype(kconst)::value;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const dd s = wave_dd_sum(v[k]);
            if (lane == 0) { wsum[(w * K + k) * 2] = s.hi; wsum[(w * K + k) * 2 + 1] = s.lo; }
        }
        __syncthreads();
        if (threadIdx.x < K) {
            const int k = threadIdx.x;
            dd b{wsum[k * 2], wsum[k * 2 + 1]};
            for (int i = 1; i < NW; ++i) b = dd_add(b, dd{wsum[(i * K + k) * 2], wsum[(i * K + k) * 2 + 1]});
            st_dev(&reg[bid * kPartialWidth + 2 * k], b.hi);
            st_dev(&reg[bid * kPartialWidth + 2 * k + 1], b.lo);
        }
        __syncthreads();
    };
    // Identical fixed-order sum of the block partials in every block: thread
    // (k, j) with j < S = NB / K sums blocks j, j + S, ... of value k, then
    // thread k combines its S partial sums in order.
    auto grid_dd = [&](auto kconst, const double* reg) {
        constexpr int K = decltype(kconst)::value;
        constexpr int S = NB / K;
        if (threadIdx.x < K * S) {
            const int k = threadIdx.x / S, j = threadIdx.x % S;
            // all loads issued before the (dependent) additions: one memory
            // latency instead of one per block (at most kMaxPer blocks each)
            constexpr int kMaxPer = 32;
            double hv[kMaxPer], lv[kMaxPer];
#pragma unroll
            for (int q = 0; q < kMaxPer; ++q) {
                const int b = j + q * S;
                const bool ok = b < nb;
                hv[q] = ok ? ld_dev(&reg[b * kPartialWidth + 2 * k]) : 0.0;
                lv[q] = ok ? ld_dev(&reg[b * kPartialWidth + 2 * k + 1]) : 0.0;
            }
            dd a{0.0, 0.0};
#pragma unroll
            for (int q = 0; q < kMaxPer; ++q) a = dd_add(a, dd{hv[q], lv[q]});
            gsum[(k * S + j) * 2] = a.hi;
            gsum[(k * S + j) * 2 + 1] = a.lo;
        }
        __syncthreads();
        if (threadIdx.x < K) {
            const int k = threadIdx.x;
            dd b{gsum[k * S * 2], gsum[k * S * 2 + 1]};
            for (int j = 1; j < S; ++j) b = dd_add(b, dd{gsum[(k * S + j) * 2], gsum[(k * S + j) * 2 + 1]});
            tot[2 * k] = b.hi;
            tot[2 * k + 1] = b.lo;
        }
        __syncthreads();
    };

    // sweep 0: ocP on the active set, sum ocP, count active, sum passive x
    {
        dd v[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t e = i0; e < m; e += stride) {
            const double xe = (double)x[e];
            if (pas[e] == TO_ACTIVE) {
                const double q = xe * sqrt(fmax(0.0, -(double)dc[e] / (double)dv[e]));
                ocp_buf[e] = q;
                v[0] = dd_add1(v[0], q);
                v[1].hi += 1.0;
            } else {
                v[2] = dd_add1(v[2], xe);
            }
        }
        double* reg = partial + (size_t)region * kMaxCoopBlocks * kPartialWidth;
        block_dd(v, std::integral_constant<int, 3>{}, reg);
        alive = gb.sync() && alive;
        grid_dd(std::integral_constant<int, 3>{}, reg);
        region ^= 1;
    }
    const double n_act = tot[2] + tot[3];
    const dd pas_sum{tot[4], tot[5]};
    double l1 = 0.0, l2 = ((tot[0] + tot[1]) / n_act) / volfrac;
    double lmid = NAN, vol_last = NAN;
    int n_bs = 0, passes = 0;
    const int cap = 200;
    auto more = [&]() { return (l1 + l2) > 0.0 && (l2 - l1) / (l2 + l1) > 1e-4 && n_bs < cap; };

    while (alive && more()) {
        // candidate brackets of the next four levels (node j: children 2j+1 = "l1 = mid", 2j+2 = "l2 = mid")
        double lo[kCand], hi[kCand], mid[kCand];
        lo[0] = l1; hi[0] = l2;
#pragma unroll
        for (int j = 0; j < kCand; ++j) {
            mid[j] = 0.5 * (lo[j] + hi[j]);
            if (2 * j + 2 < kCand) {
                lo[2 * j + 1] = mid[j]; hi[2 * j + 1] = hi[j];
                lo[2 * j + 2] = lo[j];  hi[2 * j + 2] = mid[j];
            }
        }
        dd v[kCand];
#pragma unroll
        for (int j = 0; j < kCand; ++j) v[j] = dd{0.0, 0.0};
        for (int64_t e = i0; e < m; e += stride) {
            if (pas[e] != TO_ACTIVE) continue;
            const double q = ocp_buf[e], xe = (double)x[e];
#pragma unroll
            for (int j = 0; j < kCand; ++j) v[j] = dd_add1(v[j], oc_clamp(q, mid[j], xe, move));
        }
        double* reg = partial + (size_t)region * kMaxCoopBlocks * kPartialWidth;
        block_dd(v, std::integral_constant<int, kCand>{}, reg);
        alive = gb.sync() && alive;
        grid_dd(std::integral_constant<int, kCand>{}, reg);
        region ^= 1;
        ++passes;
        // walk the tree exactly as the serial loop would
        int j = 0;
        for (int lev = 0; lev < kLevels && more(); ++lev) {
            lmid = 0.5 * (l1 + l2);        // equals mid[j]: the same operands, the same rounding
            const dd s = dd_add(dd{tot[2 * j], tot[2 * j + 1]}, pas_sum);
            const double vol = (s.hi + s.lo) / (double)m;
            vol_last = vol;
            if (vol > volfrac) { l1 = lmid; j = 2 * j + 1; }
            else { l2 = lmid; j = 2 * j + 2; }
            ++n_bs;
        }
    }
    // final design from the last midpoint evaluated (unchanged if none)
    if (n_bs > 0 && alive)
        for (int64_t e = i0; e < m; e += stride)
            if (pas[e] == TO_ACTIVE) x[e] = (T)oc_clamp(ocp_buf[e], lmid, (double)x[e], move);
    if (bid == 0 && threadIdx.x == 0) {
        to_oc_stats s;
        s.lmid = lmid; s.l1 = l1; s.l2 = l2;
        s.vol = n_bs > 0 ? vol_last : NAN;
        s.n_bs = n_bs; s.capped = n_bs >= cap ? 1 : 0;
        s.passes = passes; s.pad = alive ? 0 : 1;
        *A.st = s;
    }
}

template <typename T>
__global__ __launch_bounds__(kOcBlock) void oc_kernel(OcArgs<T> a) {
    oc_body(a, blockIdx.x, gridDim.x);
}

// A batch of designs in one launch (block b: design inst[b], block b - first[inst] of count[inst]).
template <typename T>
__global__ __launch_bounds__(kOcBlock) void oc_batch_kernel(const OcArgs<T>* __restrict__ tab,
                                                            const int32_t* __restrict__ inst,
                                                            const int32_t* __restrict__ first,
                                                            const int32_t* __restrict__ count) {
    const int i = inst[blockIdx.x];
    oc_body(tab[i], (int)blockIdx.x - first[i], count[i]);
}

template <typename T>
static OcArgs<T> oc_args(Plan* p, T* x, const T* dc, const T* dv, double volfrac, double move, to_oc_stats* st) {
    OcArgs<T> a{};
    a.m = p->info.m; a.pas = p->passive; a.x = x; a.dc = dc; a.dv = dv;
    a.volfrac = volfrac; a.move = move; a.ocp_buf = p->fx64; a.st = st;
    a.partial = p->partial; a.bar = p->bar;
    return a;
}

template <typename T>
static to_status run_oc(Plan* p, T* x, const T* dc, const T* dv, double volfrac, double move, to_oc_stats* st,
                        hipStream_t s) {
    auto k = oc_kernel<T>;
    int64_t m = p->info.m;
    int maxb = coop_blocks_for((const void*)k, kOcBlock, 0, p->num_cu);
    // blocks <= (kOcBlock / 15) * 32 = 1088 keeps every block partial within the
    // unrolled gather of the grid reduction
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(maxb, 2 * p->num_cu), (m + kOcBlock - 1) / kOcBlock));
    blocks = std::min(blocks, 1024);
    OcArgs<T> a = oc_args<T>(p, x, dc, dv, volfrac, move, st);
    void* args[] = {&a};
    TO_HIP(hipLaunchCooperativeKernel((const void*)k, dim3(blocks), dim3(kOcBlock), args, 0, s));
    return TO_OK;
}

size_t oc_args_bytes(to_dtype dt) { return dt == TO_F64 ? sizeof(OcArgs<double>) : sizeof(OcArgs<float>); }

void oc_args_fill(Plan* p, to_dtype dt, void* x, const void* dc, const void* dv, to_oc_stats* st, const double* dyn,
                  void* dst) {
    if (dt == TO_F64) {
        OcArgs<double> a = oc_args<double>(p, (double*)x, (const double*)dc, (const double*)dv, 0.0, 0.0, st);
        a.dyn = dyn;
        std::memcpy(dst, &a, sizeof a);
    } else {
        OcArgs<float> a = oc_args<float>(p, (float*)x, (const float*)dc, (const float*)dv, 0.0, 0.0, st);
        a.dyn = dyn;
        std::memcpy(dst, &a, sizeof a);
    }
}

int oc_batch_capacity(to_dtype dt, int num_cu) {
    const void* k = dt == TO_F64 ? (const void*)oc_batch_kernel<double> : (const void*)oc_batch_kernel<float>;
    return std::min(coop_blocks_for(k, kOcBlock, 0, num_cu), 2 * num_cu);
}

to_status launch_oc_batch(to_dtype dt, const void* tab, const BatchMap& mp, hipStream_t s) {
    const void* k = dt == TO_F64 ? (const void*)oc_batch_kernel<double> : (const void*)oc_batch_kernel<float>;
    void* args[] = {(void*)&tab, (void*)&mp.inst, (void*)&mp.first, (void*)&mp.count};
    TO_HIP(hipLaunchCooperativeKernel(k, dim3(mp.blocks), dim3(kOcBlock), args, 0, s));
    return TO_OK;
}

to_status launch_oc(Plan* p, to_dtype dt, void* x, const void* dc, const void* dv, double volfrac, double move,
                    to_oc_stats* st, hipStream_t s) {
    if (dt == TO_F64) return run_oc<double>(p, (double*)x, (const double*)dc, (const double*)dv, volfrac, move, st, s);
    return run_oc<float>(p, (float*)x, (const float*)dc, (const float*)dv, volfrac, move, st, s);
}

}  // namespace topt

// ---------------------------------------------------------------------------
// Periodic Anderson extrapolation of the OC fixed-point iteration (Section
// 3.3, eq. (20)-(23) with the code given there): r = x_post - x_pre on the
// active elements; the history holds the last m_r differences of the
// pre-OC designs (X) and of the residuals (R) in FP64; every q-th step the
// correction dp = (X + mix R) gamma, gamma solving the normal equations
// R^T R gamma = R^T r; the design becomes clip(x_pre + mix r - dp, 0, 1).
// Kernel 1 updates the history column and, on correction steps, reduces the
// Gram matrix and right-hand side (block partials, the last block solves the
// small system by Gaussian elimination with partial pivoting); kernel 2
// applies the update.  The history has min(it, m_r) columns by the
// correction steps; before it = m_r + 1 the first is still zero (it was never
// written) and drops out through the zero-pivot rule.
namespace topt {

constexpr int kPaeMaxM = 8;

struct PaeArgs {
    int64_t m;
    const uint8_t* pas;
    int mr, col, nc, gram;      // history length, column to write (-1: none), columns used, correction?
    double mix;
    double* X; double* R; double* xold; double* rold;   // mr x m, mr x m, m, m
    double* gamma;                                      // kPaeMaxM
    double* partial;
    unsigned* counter;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void pae_history_kernel(PaeArgs a, const T* __restrict__ xpost,
                                                             const T* __restrict__ xpre) {
    constexpr int NV = kPaeMaxM * (kPaeMaxM + 1) / 2 + kPaeMaxM;
    __shared__ double sh[kWaves];
    __shared__ int last;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.m; i += (int64_t)gridDim.x * kBlock) {
        const bool act = a.pas[i] == TO_ACTIVE;
        const double x = act ? (double)xpre[i] : 0.0;
        const double r = act ? (double)xpost[i] - (double)xpre[i] : 0.0;
        if (a.col >= 0) {
            a.X[(size_t)a.col * a.m + i] = x - a.xold[i];
            a.R[(size_t)a.col * a.m + i] = r - a.rold[i];
        }
        if (a.gram) {
            double Rc[kPaeMaxM];
#pragma unroll
            for (int c = 0; c < kPaeMaxM; ++c) Rc[c] = c < a.nc ? a.R[(size_t)c * a.m + i] : 0.0;
            int t = 0;
#pragma unroll
            for (int c = 0; c < kPaeMaxM; ++c)
#pragma unroll
                for (int d = 0; d <= c; ++d) v[t++] += Rc[c] * Rc[d];
#pragma unroll
            for (int c = 0; c < kPaeMaxM; ++c) v[t++] += Rc[c] * r;
        }
    }
    if (!a.gram) return;
    // block partials, then the last block sums them in block order and solves
    double tot[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = block_sum(v[k], sh);
        if (threadIdx.x == 0) st_dev(&a.partial[(size_t)blockIdx.x * 64 + k], s);
    }
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        last = atomicAdd(a.counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) s += ld_dev(&a.partial[(size_t)b * 64 + k]);
        tot[k] = block_sum(s, sh);
    }
    if (threadIdx.x == 0) {
        const int n = a.nc;
        double A[kPaeMaxM][kPaeMaxM], b[kPaeMaxM], g[kPaeMaxM];
        int t = 0;
        for (int c = 0; c < kPaeMaxM; ++c)
            for (int d = 0; d <= c; ++d, ++t) { A[c][d] = tot[t]; A[d][c] = tot[t]; }
        for (int c = 0; c < kPaeMaxM; ++c) b[c] = tot[t++];
        double scale = 0.0;
        for (int c = 0; c < n; ++c)
            for (int d = 0; d < n; ++d) scale = fmax(scale, fabs(A[c][d]));
        scale = fmax(scale, 1e-300);
        for (int k = 0; k < n; ++k) {
            int p = k;
            for (int i = k + 1; i < n; ++i) if (fabs(A[i][k]) > fabs(A[p][k])) p = i;
            if (p != k) {
                for (int j = 0; j < n; ++j) { const double tmp = A[k][j]; A[k][j] = A[p][j]; A[p][j] = tmp; }
                const double tb = b[k]; b[k] = b[p]; b[p] = tb;
            }
            if (fabs(A[k][k]) <= 1e-14 * scale) {          // singular: this unknown is 0
                for (int j = 0; j < n; ++j) { A[k][j] = 0.0; A[j][k] = 0.0; }
                A[k][k] = 1.0;
                b[k] = 0.0;
                continue;
            }
            for (int i = k + 1; i < n; ++i) {
                const double f = A[i][k] / A[k][k];
                for (int j = k; j < n; ++j) A[i][j] -= f * A[k][j];
                b[i] -= f * b[k];
            }
        }
        for (int k = n - 1; k >= 0; --k) {
            double s = b[k];
            for (int j = k + 1; j < n; ++j) s -= A[k][j] * g[j];
            g[k] = s / A[k][k];
        }
        for (int k = 0; k < kPaeMaxM; ++k) a.gamma[k] = k < n ? g[k] : 0.0;
        st_dev(a.counter, 0u);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void pae_update_kernel(PaeArgs a, T* __restrict__ x, const T* __restrict__ xpre) {
    double g[kPaeMaxM];
#pragma unroll
    for (int c = 0; c < kPaeMaxM; ++c) g[c] = a.gram && c < a.nc ? a.gamma[c] : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.m; i += (int64_t)gridDim.x * kBlock) {
        const bool act = a.pas[i] == TO_ACTIVE;
        const double xp = act ? (double)xpre[i] : 0.0;
        const double r = act ? (double)x[i] - (double)xpre[i] : 0.0;
        double dp = 0.0;
        if (a.gram) {
#pragma unroll
            for (int c = 0; c < kPaeMaxM; ++c)
                if (c < a.nc) dp += g[c] * (a.X[(size_t)c * a.m + i] + a.mix * a.R[(size_t)c * a.m + i]);
        }
        a.xold[i] = xp;
        a.rold[i] = r;
        if (act) x[i] = (T)fmin(fmax(xp + a.mix * r - dp, 0.0), 1.0);
    }
}

size_t pae_workspace_bytes(int64_t m, int mr) { return sizeof(double) * ((size_t)(2 * mr + 2) * m + kPaeMaxM); }

to_status launch_pae(Plan* p, to_dtype dt, void* x, const void* xpre, int32_t loop, const to_pae_params& prm,
                     void* ws, double* d_gamma, hipStream_t s) {
    const int64_t m = p->info.m;
    const int it = loop - prm.q0;
    if (it < 0) return TO_OK;
    PaeArgs a{};
    a.m = m;
    a.pas = p->passive;
    a.mr = prm.mr;
    double* w = (double*)ws;
    a.X = w;
    a.R = w + (size_t)prm.mr * m;
    a.xold = w + (size_t)2 * prm.mr * m;
    a.rold = w + (size_t)(2 * prm.mr + 1) * m;
    a.gamma = d_gamma ? d_gamma : w + (size_t)(2 * prm.mr + 2) * m;
    a.partial = p->partial + (size_t)kMaxCoopBlocks * kPartialWidth;
    a.counter = p->bar + 14;
    a.mix = (it % prm.q == 0) ? prm.xi : prm.alpha;
    a.col = it > 1 ? (it - 1) % prm.mr : -1;
    a.gram = (it > 1 && (it - 1) % prm.q == 0) ? 1 : 0;
    a.nc = a.gram ? std::min(it, prm.mr) : 0;     // the history has grown to min(it, mr) columns
    const int blocks = (int)std::min<int64_t>(2048, (m + kBlock - 1) / kBlock);
    const bool hist = a.col >= 0 || a.gram;
    if (dt == TO_F64) {
        if (hist)
            hipLaunchKernelGGL(pae_history_kernel<double>, dim3(blocks), dim3(kBlock), 0, s, a, (const double*)x,
                               (const double*)xpre);
        hipLaunchKernelGGL(pae_update_kernel<double>, dim3(blocks), dim3(kBlock), 0, s, a, (double*)x,
                           (const double*)xpre);
    } else {
        if (hist)
            hipLaunchKernelGGL(pae_history_kernel<float>, dim3(blocks), dim3(kBlock), 0, s, a, (const float*)x,
                               (const float*)xpre);
        hipLaunchKernelGGL(pae_update_kernel<float>, dim3(blocks), dim3(kBlock), 0, s, a, (float*)x,
                           (const float*)xpre);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

}  // namespace topt
