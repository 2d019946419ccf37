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
