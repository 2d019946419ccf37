// OC update with bisection on sqrt(lambda) (eq. (10)-(11), bracket from
// eq. (19); block RL.4 of the 2D code), as one persistent, cooperatively
// launched kernel.
//
// Bisection is a chain of decisions mean(x(lmid)) > volfrac.  Instead of one
// grid-wide reduction per step, each sweep over the design evaluates the 31
// midpoints of the next five levels of the bisection tree (each candidate's
// bracket follows from (l1, l2) by the same midpoint arithmetic the serial
// loop would do) and sums the candidate volumes in FP64 together with a
// rigorous bound on their rounding error; the blocks then walk the tree with
// the same stop test as the serial loop.  A decision the bound cannot settle
// is taken on a double-double sum of that one candidate (one more sweep), so
// every decision agrees with the exactly rounded sum except in exact ties.
// The decisions, the midpoints and the final design are therefore exactly
// those of plain bisection, with up to five times fewer grid barriers.
//
// The same kernel runs the explicit primal-dual update of Appendix A instead
// of the bisection (TO_OC_PD).  Further down: the bisection whose volume test
// filters and projects each candidate (Sec. 3.2) and the periodic Anderson
// extrapolation of the OC iteration (Sec. 3.3).
#include <cmath>
#include <cstring>
#include <type_traits>

#include "common.h"

namespace topt {

constexpr int kLevels = 5;
constexpr int kCand = (1 << kLevels) - 1;   // 31 midpoints per sweep

__device__ __forceinline__ double oc_clamp(double ocp, double lm, double x, double move) {
    // max(max(min(min(ocP/lmid, xU), 1), xL), 0) with xU = x + move, xL = x - move
    double v = ocp / lm;
    v = fmin(v, x + move);
    v = fmin(v, 1.0);
    v = fmax(v, x - move);
    v = fmax(v, 0.0);
    return v;
}

// The same with the quotient ocp / lm formed from rlm = 1 / lm (correctly
// rounded, once per candidate): q = ocp rlm, then the remainder ocp - q lm
// (exact in one fma) corrects q to the correctly rounded quotient (the final
// step of Markstein's division; no overflow or underflow in the ranges of
// ocP and the multiplier), so the value equals oc_clamp's without a
// division per element.
__device__ __forceinline__ double oc_clamp_r(double ocp, double lm, double rlm, double x, double move) {
    const double q = ocp * rlm;
    const double r = fma(-q, lm, ocp);
    double v = fma(r, rlm, q);
    v = fmin(v, x + move);
    v = fmin(v, 1.0);
    v = fmax(v, x - move);
    v = fmax(v, 0.0);
    return v;
}

// Wave sums of 16 double-double values at once by a butterfly that halves
// the set at each of the first four levels (lane bit 5 keeps the upper or
// the lower half, then bits 4, 3, 2) and sums the last value over lane bits
// 1 and 0: 17 cross-lane exchanges instead of 16 x 6.  Lane 4 j ends with
// the sum of value j.
__device__ __forceinline__ dd dd_xor(dd a, int mask) {
    return dd{__shfl_xor(a.hi, mask, 64), __shfl_xor(a.lo, mask, 64)};
}
__device__ __forceinline__ dd dd_sel(bool c, dd a, dd b) { return c ? a : b; }
__device__ __forceinline__ dd wave_dd_sum16(const dd (&v)[16], int lane) {
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
    dd u1[8], u2[4], u3[2];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        u1[j] = dd_add(dd_sel(b5, v[8 + j], v[j]), dd_xor(dd_sel(b5, v[j], v[8 + j]), 32));
#pragma unroll
    for (int j = 0; j < 4; ++j)
        u2[j] = dd_add(dd_sel(b4, u1[4 + j], u1[j]), dd_xor(dd_sel(b4, u1[j], u1[4 + j]), 16));
#pragma unroll
    for (int j = 0; j < 2; ++j)
        u3[j] = dd_add(dd_sel(b3, u2[2 + j], u2[j]), dd_xor(dd_sel(b3, u2[j], u2[2 + j]), 8));
    dd u = dd_add(dd_sel(b2, u3[1], u3[0]), dd_xor(dd_sel(b2, u3[0], u3[1]), 4));
    u = dd_add(u, dd_xor(u, 2));
    return dd_add(u, dd_xor(u, 1));
}

// Wave sums of 32 FP64 values at once by the same halving butterfly (lane
// bits 5, 4, 3, 2, 1 halve the set, bit 0 sums the last value): 32
// cross-lane exchanges instead of 32 x 6.  Lane 2 j ends with the sum of
// value j.  The order of the additions is fixed.
__device__ __forceinline__ double f64_sel(bool c, double a, double b) { return c ? a : b; }
__device__ __forceinline__ double wave_sum32(const double (&v)[32], int lane) {
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
    double u1[16], u2[8], u3[4], u4[2];
#pragma unroll
    for (int j = 0; j < 16; ++j)
        u1[j] = f64_sel(b5, v[16 + j], v[j]) + __shfl_xor(f64_sel(b5, v[j], v[16 + j]), 32, 64);
#pragma unroll
    for (int j = 0; j < 8; ++j)
        u2[j] = f64_sel(b4, u1[8 + j], u1[j]) + __shfl_xor(f64_sel(b4, u1[j], u1[8 + j]), 16, 64);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        u3[j] = f64_sel(b3, u2[4 + j], u2[j]) + __shfl_xor(f64_sel(b3, u2[j], u2[4 + j]), 8, 64);
#pragma unroll
    for (int j = 0; j < 2; ++j)
        u4[j] = f64_sel(b2, u3[2 + j], u3[j]) + __shfl_xor(f64_sel(b2, u3[j], u3[2 + j]), 4, 64);
    double u = f64_sel(b1, u4[1], u4[0]) + __shfl_xor(f64_sel(b1, u4[0], u4[1]), 2, 64);
    return u + __shfl_xor(u, 1, 64);
}

constexpr int kOcBlock = 512;
constexpr int kMaxOcBlocks = 512;          // blocks of one design's OC launch (the grid sums gather this many)
// value-major partials (2 words per value, kMaxCoopBlocks blocks each) fit a partial region
// value-major partials: 31 FP64 values (the candidate sweeps) or 3 double-double
// values (the first sweep) per block fit a partial region
static_assert(kCand <= kPartialWidth && 6 <= kPartialWidth, "OC partials exceed a partial region");

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
    int method;             // TO_OC_BISECT or TO_OC_PD
};

// The update of one design, run by `nb` blocks of which this is `bid`.
template <typename T>
__device__ void oc_body(const OcArgs<T>& A, int bid, int nb) {
    constexpr int NB = kOcBlock, NW = NB / 64;
    __shared__ double wsum[NW * kCand * 2];
    __shared__ double gsum[NB * 2];
    __shared__ double tot[2 * kCand];
    __shared__ double smid[kCand], srmid[kCand];
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
        if constexpr (K > 8 && K <= 16) {
            dd v16[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v16[k] = k < K ? v[k] : dd{0.0, 0.0};
            const dd s = wave_dd_sum16(v16, lane);
            const int k = lane >> 2;
            if ((lane & 3) == 0 && k < K) { wsum[(w * K + k) * 2] = s.hi; wsum[(w * K + k) * 2 + 1] = s.lo; }
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const dd s = wave_dd_sum(v[k]);
                if (lane == 0) { wsum[(w * K + k) * 2] = s.hi; wsum[(w * K + k) * 2 + 1] = s.lo; }
            }
        }
        __syncthreads();
        if (threadIdx.x < K) {
            const int k = threadIdx.x;
            dd b{wsum[k * 2], wsum[k * 2 + 1]};
            for (int i = 1; i < NW; ++i) b = dd_add(b, dd{wsum[(i * K + k) * 2], wsum[(i * K + k) * 2 + 1]});
            // value-major: the words of one value from all blocks are
            // consecutive, so the grid sum's reads of a value coalesce
            st_dev(&reg[(size_t)(2 * k) * kMaxCoopBlocks + bid], b.hi);
            st_dev(&reg[(size_t)(2 * k + 1) * kMaxCoopBlocks + bid], b.lo);
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
            constexpr int kMaxPer = (kMaxOcBlocks + S - 1) / S;
            double hv[kMaxPer], lv[kMaxPer];
#pragma unroll
            for (int q = 0; q < kMaxPer; ++q) {
                const int b = j + q * S;
                const bool ok = b < nb;
                hv[q] = ok ? ld_dev(&reg[(size_t)(2 * k) * kMaxCoopBlocks + b]) : 0.0;
                lv[q] = ok ? ld_dev(&reg[(size_t)(2 * k + 1) * kMaxCoopBlocks + b]) : 0.0;
            }
            // the chains stop at the last existing block: adding the zeros of
            // missing blocks to a normalised pair leaves it unchanged
            const int qn = j < nb ? (nb - j + S - 1) / S : 0;
            dd a{0.0, 0.0};
#pragma unroll
            for (int q = 0; q < kMaxPer; ++q)
                if (q < qn) a = dd_add(a, dd{hv[q], lv[q]});
            gsum[(k * S + j) * 2] = a.hi;
            gsum[(k * S + j) * 2 + 1] = a.lo;
        }
        __syncthreads();
        if (threadIdx.x < K) {
            const int k = threadIdx.x;
            dd b{gsum[k * S * 2], gsum[k * S * 2 + 1]};
            const int jn = nb < S ? nb : S;
            for (int j = 1; j < jn; ++j) b = dd_add(b, dd{gsum[(k * S + j) * 2], gsum[(k * S + j) * 2 + 1]});
            tot[2 * k] = b.hi;
            tot[2 * k + 1] = b.lo;
        }
        __syncthreads();
    };

    // The same for K plain FP64 values (the candidate volumes): each wave
    // reduces 32 values with the halving butterfly, thread k adds the waves'
    // sums of value k in wave order; the grid sum is ordered as in grid_dd.
    auto block_f64 = [&](const double (&v)[32], double* reg) {
        const double sw = wave_sum32(v, lane);
        const int k = lane >> 1;
        if ((lane & 1) == 0 && k < kCand) wsum[w * kCand + k] = sw;
        __syncthreads();
        if (threadIdx.x < kCand) {
            const int k2 = threadIdx.x;
            double b = wsum[k2];
            for (int i = 1; i < NW; ++i) b += wsum[i * kCand + k2];
            st_dev(&reg[(size_t)k2 * kMaxCoopBlocks + bid], b);
        }
        __syncthreads();
    };
    auto grid_f64 = [&](const double* reg) {
        constexpr int K = kCand;
        constexpr int S = NB / K;
        if (threadIdx.x < K * S) {
            const int k = threadIdx.x / S, j = threadIdx.x % S;
            constexpr int kMaxPer = (kMaxOcBlocks + S - 1) / S;
            double hv[kMaxPer];
#pragma unroll
            for (int q = 0; q < kMaxPer; ++q) {
                const int b = j + q * S;
                hv[q] = b < nb ? ld_dev(&reg[(size_t)k * kMaxCoopBlocks + b]) : 0.0;
            }
            const int qn = j < nb ? (nb - j + S - 1) / S : 0;
            double a = 0.0;
#pragma unroll
            for (int q = 0; q < kMaxPer; ++q)
                if (q < qn) a += hv[q];
            gsum[k * S + j] = a;
        }
        __syncthreads();
        if (threadIdx.x < K) {
            const int k = threadIdx.x;
            double b = gsum[k * S];
            const int jn = nb < S ? nb : S;
            for (int j = 1; j < jn; ++j) b += gsum[k * S + j];
            tot[k] = b;
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
    if (A.method == TO_OC_PD) {
        // explicit primal-dual iteration (Appendix A): each pass sums ocP over
        // the free set M and the active bounds over U and L, then solves the
        // volume equation for lm; an element exactly on a bound (with
        // xL' < xU') is in none of the sets
        const double psum = pas_sum.hi + pas_sum.lo, md = (double)m;
        double lm = ((tot[0] + tot[1]) / n_act) / volfrac, lm_old = 0.0, vol = NAN;
        int it = 0, passes_pd = 0;
        bool bad = false;
        const int cap = 200;
        while (alive && fabs(lm - lm_old) > 1e-10 && it < cap) {
            dd v[2] = {{0, 0}, {0, 0}};
            for (int64_t e = i0; e < m; e += stride) {
                if (pas[e] != TO_ACTIVE) continue;
                const double q = ocp_buf[e], xe = (double)x[e];
                const double up = fmin(xe + move, 1.0), lo = fmax(xe - move, 0.0), tmp = q / lm;
                if (tmp > up) v[1] = dd_add1(v[1], up);
                else if (tmp < lo) v[1] = dd_add1(v[1], lo);
                else if (!((tmp == lo || tmp == up) && lo < up)) v[0] = dd_add1(v[0], q);
            }
            double* reg = partial + (size_t)region * kMaxCoopBlocks * kPartialWidth;
            block_dd(v, std::integral_constant<int, 2>{}, reg);
            alive = gb.sync() && alive;
            grid_dd(std::integral_constant<int, 2>{}, reg);
            region ^= 1;
            ++passes_pd;
            const double summ = tot[0] + tot[1], bnd = tot[2] + tot[3];
            ++it;
            vol = (summ / lm + bnd + psum) / md;
            const double den = volfrac * md - psum - bnd;
            if (!(den > 0.0)) { bad = true; break; }
            lm_old = lm;
            lm = summ / den;
        }
        // a multiplier that is not positive and finite (e.g. every ocP is 0)
        // leaves the design unchanged and is reported
        const bool ok = lm > 0.0 && lm < INFINITY;
        if (alive && ok)
            for (int64_t e = i0; e < m; e += stride)
                if (pas[e] == TO_ACTIVE) x[e] = (T)oc_clamp(ocp_buf[e], lm, (double)x[e], move);
        bad = bad || !ok;
        if (bid == 0 && threadIdx.x == 0) {
            to_oc_stats s;
            s.lmid = lm; s.l1 = lm_old; s.l2 = lm;
            s.vol = vol;
            s.n_bs = it; s.capped = (bad || it >= cap) ? 1 : 0;
            s.passes = passes_pd; s.pad = alive ? 0 : 1;
            *A.st = s;
        }
        return;
    }
    double l1 = 0.0, l2 = ((tot[0] + tot[1]) / n_act) / volfrac;
    double lmid = NAN, vol_last = NAN;
    int n_bs = 0, passes = 0;
    const int cap = 200;
    auto more = [&]() { return (l1 + l2) > 0.0 && (l2 - l1) / (l2 + l1) > 1e-4 && n_bs < cap; };

    // Rounding-error bound of the FP64 candidate sums: every term (x >= 0)
    // passes through at most d additions (its thread's elements, the wave
    // butterfly, the block's waves, the grid gather and the final
    // combination), so |sum - exact| <= d u exact / (1 - d u) <= err * sum.
    const int64_t per_thread = (m + stride - 1) / stride;
    const double err = (double)(per_thread + 6 + NW + (kMaxOcBlocks + NB / kCand - 1) / (NB / kCand) + NB / kCand + 4) *
                       0x1p-53 * (1.0 + 0x1p-20);
    while (alive && more()) {
        // candidate brackets of the next five levels (node j: children
        // 2j+1 = "l1 = mid", 2j+2 = "l2 = mid"); the midpoints and their
        // reciprocals are wave-uniform and read from LDS in the element loop
        if (threadIdx.x == 0) {
            double lo[kCand], hi[kCand];
            lo[0] = l1; hi[0] = l2;
            for (int j = 0; j < kCand; ++j) {
                const double mj = 0.5 * (lo[j] + hi[j]);
                smid[j] = mj;
                srmid[j] = 1.0 / mj;
                if (2 * j + 2 < kCand) {
                    lo[2 * j + 1] = mj; hi[2 * j + 1] = hi[j];
                    lo[2 * j + 2] = lo[j]; hi[2 * j + 2] = mj;
                }
            }
        }
        __syncthreads();
        double v[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = 0.0;
        for (int64_t e = i0; e < m; e += stride) {
            if (pas[e] != TO_ACTIVE) continue;
            const double q = ocp_buf[e], xe = (double)x[e];
#pragma unroll
            for (int j = 0; j < kCand; ++j) v[j] += oc_clamp_r(q, smid[j], srmid[j], xe, move);
        }
        double* reg = partial + (size_t)region * kMaxCoopBlocks * kPartialWidth;
        block_f64(v, reg);
        alive = gb.sync() && alive;
        grid_f64(reg);
        region ^= 1;
        ++passes;
        // walk the tree exactly as the serial loop would; a decision the
        // bound cannot settle is taken on the exactly summed volume
        int j = 0;
        for (int lev = 0; lev < kLevels && more(); ++lev) {
            lmid = 0.5 * (l1 + l2);        // equals mid[j]: the same operands, the same rounding
            const double tj = tot[j];
            const dd sl = dd_add(dd{tj - err * tj, 0.0}, pas_sum), sh = dd_add(dd{tj + err * tj, 0.0}, pas_sum);
            const double vlo = (sl.hi + sl.lo) / (double)m, vhi = (sh.hi + sh.lo) / (double)m;
            bool greater;
            if (vlo > volfrac) {
                greater = true;
                const dd s0 = dd_add(dd{tj, 0.0}, pas_sum);
                vol_last = (s0.hi + s0.lo) / (double)m;
            } else if (vhi <= volfrac) {
                greater = false;
                const dd s0 = dd_add(dd{tj, 0.0}, pas_sum);
                vol_last = (s0.hi + s0.lo) / (double)m;
            } else {
                // double-double sum of this candidate (agrees with the
                // exactly rounded sum except in exact ties)
                const double rl = 1.0 / lmid;
                dd ve[1] = {{0.0, 0.0}};
                for (int64_t e = i0; e < m; e += stride)
                    if (pas[e] == TO_ACTIVE)
                        ve[0] = dd_add1(ve[0], oc_clamp_r(ocp_buf[e], lmid, rl, (double)x[e], move));
                double* reg2 = partial + (size_t)region * kMaxCoopBlocks * kPartialWidth;
                block_dd(ve, std::integral_constant<int, 1>{}, reg2);
                alive = gb.sync() && alive;
                grid_dd(std::integral_constant<int, 1>{}, reg2);
                region ^= 1;
                ++passes;
                const dd s = dd_add(dd{tot[0], tot[1]}, pas_sum);
                vol_last = (s.hi + s.lo) / (double)m;
                greater = vol_last > volfrac;
                // the candidate sums of this sweep were overwritten: keep
                // walking from this level's decision only (the next sweep
                // starts from the new bracket)
                if (greater) l1 = lmid; else l2 = lmid;
                ++n_bs;
                break;
            }
            if (greater) { l1 = lmid; j = 2 * j + 1; }
            else { l2 = lmid; j = 2 * j + 2; }
            ++n_bs;
        }
    }
    // final design from the last midpoint evaluated (unchanged if none)
    if (n_bs > 0 && alive) {
        const double rl = 1.0 / lmid;
        for (int64_t e = i0; e < m; e += stride)
            if (pas[e] == TO_ACTIVE) x[e] = (T)oc_clamp_r(ocp_buf[e], lmid, rl, (double)x[e], move);
    }
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
                        hipStream_t s, int method) {
    auto k = oc_kernel<T>;
    int64_t m = p->info.m;
    int maxb = coop_blocks_for((const void*)k, kOcBlock, 0, p->num_cu);
    // blocks <= (kOcBlock / 15) * 32 = 1088 keeps every block partial within the
    // unrolled gather of the grid reduction
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(maxb, 2 * p->num_cu), (m + kOcBlock - 1) / kOcBlock));
    blocks = std::min(blocks, kMaxOcBlocks);
    OcArgs<T> a = oc_args<T>(p, x, dc, dv, volfrac, move, st);
    a.method = method;
    void* args[] = {&a};
    TO_HIP(launch_resident(p, (const void*)k, blocks, kOcBlock, args, s));
    return TO_OK;
}

size_t oc_args_bytes(to_dtype dt) { return dt == TO_F64 ? sizeof(OcArgs<double>) : sizeof(OcArgs<float>); }

void oc_args_fill(Plan* p, to_dtype dt, void* x, const void* dc, const void* dv, to_oc_stats* st, const double* dyn,
                  int method, void* dst) {
    if (dt == TO_F64) {
        OcArgs<double> a = oc_args<double>(p, (double*)x, (const double*)dc, (const double*)dv, 0.0, 0.0, st);
        a.dyn = dyn;
        a.method = method;
        std::memcpy(dst, &a, sizeof a);
    } else {
        OcArgs<float> a = oc_args<float>(p, (float*)x, (const float*)dc, (const float*)dv, 0.0, 0.0, st);
        a.dyn = dyn;
        a.method = method;
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
                    to_oc_stats* st, hipStream_t s, int method) {
    if (dt == TO_F64)
        return run_oc<double>(p, (double*)x, (const double*)dc, (const double*)dv, volfrac, move, st, s, method);
    return run_oc<float>(p, (float*)x, (const float*)dc, (const float*)dv, volfrac, move, st, s, method);
}

// ---------------------------------------------------------------------------
// Bisection whose volume test filters and (ft > 1) projects every candidate
// (Sec. 3.2, the code offered for a fixed projection threshold).  A candidate
// depends on the whole design through the filter, so each bisection step is
// three launches: the candidate design, the plan's LDS-tiled forward filter,
// and a volume kernel whose last block takes the step's decision on device.
// The host enqueues a fixed number of steps; once the stop test holds a
// device flag makes the remaining launches (the filter's included) return at
// once, so no host synchronisation is needed.
constexpr int kOcfCap = 48;

struct OcfState {
    double l1, l2, lmid, vol;
    unsigned done, n_bs, cap, pad;
};

__device__ __forceinline__ dd block_dd_sum(dd v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_dd_sum(v);
    if (lane == 0) { sh[2 * w] = v.hi; sh[2 * w + 1] = v.lo; }
    __syncthreads();
    dd s{sh[0], sh[1]};
    for (int i = 1; i < kBlock / 64; ++i) s = dd_add(s, dd{sh[2 * i], sh[2 * i + 1]});
    __syncthreads();
    return s;
}

// Block partials of two double-double sums, then the last block to arrive
// combines them in block order (deterministic) into out[0..1] (hi + lo).
__device__ __forceinline__ bool last_block_dd2(dd a, dd b, double* partial, unsigned* counter, double* sh,
                                               dd* out) {
    __shared__ int last;
    a = block_dd_sum(a, sh);
    b = block_dd_sum(b, sh);
    if (threadIdx.x == 0) {
        double* q = partial + (size_t)blockIdx.x * 4;
        st_dev(q, a.hi); st_dev(q + 1, a.lo); st_dev(q + 2, b.hi); st_dev(q + 3, b.lo);
        wait_stores();
        last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return false;
    // thread t combines blocks t, t + kBlock, ... in order, then the fixed
    // shuffle tree of block_dd_sum: the same order on every run
    dd sa{0.0, 0.0}, sb{0.0, 0.0};
    for (int k = threadIdx.x; k < (int)gridDim.x; k += kBlock) {
        const double* q = partial + (size_t)k * 4;
        sa = dd_add(sa, dd{ld_dev(q), ld_dev(q + 1)});
        sb = dd_add(sb, dd{ld_dev(q + 2), ld_dev(q + 3)});
    }
    sa = block_dd_sum(sa, sh);
    sb = block_dd_sum(sb, sh);
    if (threadIdx.x == 0) {
        out[0] = sa; out[1] = sb;
        st_dev(counter, 0u);
    }
    return true;
}

__device__ __forceinline__ bool ocf_more(double l1, double l2, unsigned n_bs, unsigned cap) {
    return (l1 + l2) > 0.0 && (l2 - l1) / (l2 + l1) > 1e-4 && n_bs < cap;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void ocf_init_kernel(int64_t m, const uint8_t* __restrict__ pas,
                                                          const T* __restrict__ x, const T* __restrict__ dc,
                                                          const T* __restrict__ dv, double volfrac,
                                                          double* __restrict__ ocp, double* partial,
                                                          unsigned* counter, OcfState* st) {
    __shared__ double sh[2 * kWaves];
    dd s{0.0, 0.0}, c{0.0, 0.0};
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock) {
        if (pas[e] != TO_ACTIVE) continue;
        const double q = (double)x[e] * sqrt(fmax(0.0, -(double)dc[e] / (double)dv[e]));
        ocp[e] = q;
        s = dd_add1(s, q);
        c.hi += 1.0;
    }
    dd tot[2];
    if (!last_block_dd2(s, c, partial, counter, sh, tot)) return;
    if (threadIdx.x == 0) {
        const double l2 = ((tot[0].hi + tot[0].lo) / (tot[1].hi + tot[1].lo)) / volfrac;
        st->l1 = 0.0;
        st->l2 = l2;
        st->lmid = NAN;
        st->vol = NAN;
        st->n_bs = 0;
        st->cap = kOcfCap;
        st->done = ocf_more(0.0, l2, 0, kOcfCap) ? 0u : 1u;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void ocf_cand_kernel(int64_t m, const uint8_t* __restrict__ pas,
                                                          const T* __restrict__ x, const double* __restrict__ ocp,
                                                          double move, const OcfState* __restrict__ st,
                                                          T* __restrict__ xc) {
    if (st->done) return;
    const double lmid = 0.5 * (st->l1 + st->l2);
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock)
        xc[e] = pas[e] == TO_ACTIVE ? (T)oc_clamp(ocp[e], lmid, (double)x[e], move) : x[e];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void ocf_vol_kernel(int64_t m, const uint8_t* __restrict__ pas,
                                                         const T* __restrict__ xf, int ft, double beta,
                                                         const double* __restrict__ d_eta, double volfrac,
                                                         double* partial, unsigned* counter, OcfState* st) {
    __shared__ double sh[2 * kWaves];
    if (st->done) return;
    double tbe = 0.0, den = 1.0, eta = 0.0;
    if (ft > 1) {
        eta = *d_eta;
        tbe = tanh(beta * eta);
        den = tbe + tanh(beta * (1.0 - eta));
    }
    dd s{0.0, 0.0}, z{0.0, 0.0};
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock) {
        const uint8_t c = pas[e];
        double v = c == TO_SOLID ? 1.0 : c == TO_VOID ? 0.0 : (double)xf[e];
        if (ft > 1) v = (tbe + tanh(beta * (v - eta))) / den;
        s = dd_add1(s, v);
    }
    dd tot[2];
    if (!last_block_dd2(s, z, partial, counter, sh, tot)) return;
    if (threadIdx.x == 0) {
        double l1 = st->l1, l2 = st->l2;
        const double lmid = 0.5 * (l1 + l2);
        const double vol = (tot[0].hi + tot[0].lo) / (double)m;
        if (vol > volfrac) l1 = lmid;
        else l2 = lmid;
        const unsigned n = st->n_bs + 1;
        st->l1 = l1;
        st->l2 = l2;
        st->lmid = lmid;
        st->vol = vol;
        st->n_bs = n;
        st->done = ocf_more(l1, l2, n, st->cap) ? 0u : 1u;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void ocf_final_kernel(int64_t m, const uint8_t* __restrict__ pas,
                                                           T* __restrict__ x, const double* __restrict__ ocp,
                                                           double move, const OcfState* __restrict__ st,
                                                           to_oc_stats* stats) {
    const unsigned n = st->n_bs;
    const double lmid = st->lmid;
    if (n > 0)
        for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock)
            if (pas[e] == TO_ACTIVE) x[e] = (T)oc_clamp(ocp[e], lmid, (double)x[e], move);
    if (stats && blockIdx.x == 0 && threadIdx.x == 0) {
        to_oc_stats s;
        s.lmid = n > 0 ? lmid : NAN; s.l1 = st->l1; s.l2 = st->l2;
        s.vol = n > 0 ? st->vol : NAN;
        s.n_bs = (int32_t)n; s.capped = n >= st->cap ? 1 : 0;
        s.passes = (int32_t)n; s.pad = 0;
        *stats = s;
    }
}

template <typename T>
static to_status run_oc_filtered(Plan* p, to_dtype dt, int ft, T* x, const T* dc, const T* dv, double volfrac,
                                 double move, double beta, const double* d_eta, to_oc_stats* stats, T* xc, T* xf,
                                 hipStream_t s) {
    const int64_t m = p->info.m;
    OcfState* fs = reinterpret_cast<OcfState*>(p->scal + 32);
    double* part = p->partial + (size_t)kMaxCoopBlocks * kPartialWidth;
    unsigned* ctr = p->bar + 20;
    // 256 blocks: the arrivals on the last-block counter serialise at one address
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(256, (m + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(ocf_init_kernel<T>, dim3(blocks), dim3(kBlock), 0, s, m, p->passive, x, dc, dv, volfrac,
                       p->fx64, part, ctr, fs);
    TO_HIP(hipGetLastError());
    p->filt_skip = &fs->done;
    to_status r = TO_OK;
    for (int k = 0; k < kOcfCap && r == TO_OK; ++k) {
        hipLaunchKernelGGL(ocf_cand_kernel<T>, dim3(blocks), dim3(kBlock), 0, s, m, p->passive, x, p->fx64, move,
                           fs, xc);
        r = launch_filter(p, dt, TO_FILTER_FWD, xc, nullptr, nullptr, xf, nullptr, s);
        if (r != TO_OK) break;
        hipLaunchKernelGGL(ocf_vol_kernel<T>, dim3(blocks), dim3(kBlock), 0, s, m, p->passive, xf, ft, beta, d_eta,
                           volfrac, part, ctr, fs);
    }
    p->filt_skip = nullptr;
    if (r != TO_OK) return r;
    hipLaunchKernelGGL(ocf_final_kernel<T>, dim3(blocks), dim3(kBlock), 0, s, m, p->passive, x, p->fx64, move, fs,
                       stats);
    TO_HIP(hipGetLastError());
    return TO_OK;
}

to_status launch_oc_filtered(Plan* p, to_dtype dt, int ft, void* x, const void* dc, const void* dv, double volfrac,
                             double move, double beta, const double* d_eta, to_oc_stats* st, hipStream_t s) {
    if (dt == TO_F64)
        return run_oc_filtered<double>(p, dt, ft, (double*)x, (const double*)dc, (const double*)dv, volfrac, move,
                                       beta, d_eta, st, p->v64[6], p->v64[7], s);
    return run_oc_filtered<float>(p, dt, ft, (float*)x, (const float*)dc, (const float*)dv, volfrac, move, beta,
                                  d_eta, st, p->v32[6], p->v32[7], s);
}

}  // namespace topt

// ---------------------------------------------------------------------------
// Periodic Anderson extrapolation of the OC fixed-point iteration (Section
// 3.3, eq. (20)-(23) with the code given there): r = x_post - x_pre on the
// active elements; the history holds the last m_r differences of the
// pre-OC designs (X) and of the residuals (R) in FP64; every q-th step the
// correction dp = (X + mix R) gamma, gamma solving the normal equations
// R^T R gamma = R^T r; the design becomes clip(x_pre + mix r - dp, 0, 1).
// The first kernel updates the history column and, on correction steps, forms
// block partials of the Gram matrix and right-hand side; a one-block kernel
// sums them in block order and solves the small system by Gaussian
// elimination with partial pivoting; the last kernel applies the update.  The history has min(it, m_r) columns by the
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
    double* partial;                                    // per block: kPaeMaxNV values
};

constexpr int kPaeMaxNV = kPaeMaxM * (kPaeMaxM + 1) / 2 + kPaeMaxM;   // Gram (lower) + right-hand side
constexpr int kPaeBlocks = 512;

// History column update and, on correction steps, block partials of the
// lower Gram matrix R^T R and of R^T r.  MR: compile-time bound on the
// columns (4 or 8), so the accumulators stay in registers.
template <typename T, int MR>
__global__ __launch_bounds__(kBlock) void pae_history_kernel(PaeArgs a, const T* __restrict__ xpost,
                                                             const T* __restrict__ xpre) {
    constexpr int NV = MR * (MR + 1) / 2 + MR;
    __shared__ double sh[kWaves];
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
            double Rc[MR];
#pragma unroll
            for (int c = 0; c < MR; ++c) Rc[c] = c < a.nc ? a.R[(size_t)c * a.m + i] : 0.0;
            int t = 0;
#pragma unroll
            for (int c = 0; c < MR; ++c)
#pragma unroll
                for (int d = 0; d <= c; ++d) v[t++] += Rc[c] * Rc[d];
#pragma unroll
            for (int c = 0; c < MR; ++c) v[t++] += Rc[c] * r;
        }
    }
    if (!a.gram) return;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = block_sum(v[k], sh);
        if (threadIdx.x == 0) a.partial[(size_t)blockIdx.x * kPaeMaxNV + k] = s;
    }
}

// One block: sums the partials in block order, then thread 0 solves the
// normal equations by Gaussian elimination with partial pivoting (a pivot
// below 1e-14 of the largest entry sets that coefficient to 0).
template <int MR>
__global__ __launch_bounds__(kBlock) void pae_solve_kernel(PaeArgs a, int nblocks) {
    constexpr int NV = MR * (MR + 1) / 2 + MR;
    constexpr int G = kBlock / 64;                      // block groups per value
    __shared__ double part[G][64];
    __shared__ double tot[64];
    const int k = threadIdx.x & 63, g = threadIdx.x >> 6;
    double s = 0.0;
    if (k < NV)
        for (int b = g; b < nblocks; b += G) s += a.partial[(size_t)b * kPaeMaxNV + k];
    part[g][k] = s;
    __syncthreads();
    if (threadIdx.x < 64) {
        double t = 0.0;
        for (int q = 0; q < G; ++q) t += part[q][threadIdx.x];
        tot[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int n = a.nc;
    double A[MR][MR], bv[MR], gv[MR];
    int t = 0;
    for (int c = 0; c < MR; ++c)
        for (int d = 0; d <= c; ++d, ++t) { A[c][d] = tot[t]; A[d][c] = tot[t]; }
    for (int c = 0; c < MR; ++c) bv[c] = tot[t++];
    double scale = 0.0;
    for (int c = 0; c < n; ++c)
        for (int d = 0; d < n; ++d) scale = fmax(scale, fabs(A[c][d]));
    scale = fmax(scale, 1e-300);
    for (int kk = 0; kk < n; ++kk) {
        int p = kk;
        for (int i = kk + 1; i < n; ++i) if (fabs(A[i][kk]) > fabs(A[p][kk])) p = i;
        if (p != kk) {
            for (int j = 0; j < n; ++j) { const double tmp = A[kk][j]; A[kk][j] = A[p][j]; A[p][j] = tmp; }
            const double tb = bv[kk]; bv[kk] = bv[p]; bv[p] = tb;
        }
        if (fabs(A[kk][kk]) <= 1e-14 * scale) {          // singular: this unknown is 0
            for (int j = 0; j < n; ++j) { A[kk][j] = 0.0; A[j][kk] = 0.0; }
            A[kk][kk] = 1.0;
            bv[kk] = 0.0;
            continue;
        }
        for (int i = kk + 1; i < n; ++i) {
            const double f = A[i][kk] / A[kk][kk];
            for (int j = kk; j < n; ++j) A[i][j] -= f * A[kk][j];
            bv[i] -= f * bv[kk];
        }
    }
    for (int kk = n - 1; kk >= 0; --kk) {
        double acc = bv[kk];
        for (int j = kk + 1; j < n; ++j) acc -= A[kk][j] * gv[j];
        gv[kk] = acc / A[kk][kk];
    }
    for (int c = 0; c < kPaeMaxM; ++c) a.gamma[c] = c < n ? gv[c] : 0.0;
}

template <typename T, int MR>
__global__ __launch_bounds__(kBlock) void pae_update_kernel(PaeArgs a, T* __restrict__ x, const T* __restrict__ xpre) {
    double g[MR];
#pragma unroll
    for (int c = 0; c < MR; ++c) g[c] = a.gram && c < a.nc ? a.gamma[c] : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.m; i += (int64_t)gridDim.x * kBlock) {
        const bool act = a.pas[i] == TO_ACTIVE;
        const double xp = act ? (double)xpre[i] : 0.0;
        const double r = act ? (double)x[i] - (double)xpre[i] : 0.0;
        double dp = 0.0;
        if (a.gram) {
#pragma unroll
            for (int c = 0; c < MR; ++c)
                if (c < a.nc) dp += g[c] * (a.X[(size_t)c * a.m + i] + a.mix * a.R[(size_t)c * a.m + i]);
        }
        a.xold[i] = xp;
        a.rold[i] = r;
        if (act) x[i] = (T)fmin(fmax(xp + a.mix * r - dp, 0.0), 1.0);
    }
}

template <typename T, int MR>
static void pae_launch(const PaeArgs& a, T* x, const T* xpre, int blocks, bool hist, hipStream_t s) {
    if (hist)
        hipLaunchKernelGGL((pae_history_kernel<T, MR>), dim3(blocks), dim3(kBlock), 0, s, a, (const T*)x, xpre);
    if (a.gram) hipLaunchKernelGGL(pae_solve_kernel<MR>, dim3(1), dim3(kBlock), 0, s, a, blocks);
    hipLaunchKernelGGL((pae_update_kernel<T, MR>), dim3(blocks), dim3(kBlock), 0, s, a, x, xpre);
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
    a.mix = (it % prm.q == 0) ? prm.xi : prm.alpha;
    a.col = it > 1 ? (it - 1) % prm.mr : -1;
    a.gram = (it > 1 && (it - 1) % prm.q == 0) ? 1 : 0;
    a.nc = a.gram ? std::min(it, prm.mr) : 0;     // the history has grown to min(it, mr) columns
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kPaeBlocks, (m + kBlock - 1) / kBlock));
    const bool hist = a.col >= 0 || a.gram;
    if (dt == TO_F64) {
        if (prm.mr <= 4) pae_launch<double, 4>(a, (double*)x, (const double*)xpre, blocks, hist, s);
        else pae_launch<double, kPaeMaxM>(a, (double*)x, (const double*)xpre, blocks, hist, s);
    } else {
        if (prm.mr <= 4) pae_launch<float, 4>(a, (float*)x, (const float*)xpre, blocks, hist, s);
        else pae_launch<float, kPaeMaxM>(a, (float*)x, (const float*)xpre, blocks, hist, s);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

}  // namespace topt
