// Physical density (block RL.1): Heaviside projection eq. (1), its derivative
// eq. (9), and the volume-preserving threshold of eq. (17) by Newton's method
// with the closed-form d prj / d eta of the codes.
//
// One persistent, cooperatively launched kernel does the whole block: each
// Newton step is one sweep that accumulates sum prj and sum d prj/d eta in
// FP64, a grid barrier, and an identical fixed-order reduction in every block
// (so every block takes the same Newton decision).  A final sweep writes
// xphys and dprj and accumulates the change and the volume.
#include <cmath>
#include <cstring>

#include "common.h"

namespace topt {

struct ProjCoef {
    double beta, eta, den, tbe, csch, chb;
    __device__ void set(double b, double e) {
        beta = b; eta = e;
        tbe = tanh(b * e);
        den = tbe + tanh(b * (1.0 - e));
        csch = 1.0 / sinh(b);
        chb = cosh(b);
    }
    // t(v) = tanh(beta (v - eta)), shared by the projection and both derivatives
    __device__ double th(double v) const { return tanh(beta * (v - eta)); }
    __device__ double prj_t(double t) const { return (tbe + t) / den; }
    __device__ double dprj_t(double t) const { return beta * (1.0 - t * t) / den; }
    // d prj / d eta of the codes, -beta csch(beta) sinh(v beta) sinh((1-v) beta)
    // / cosh^2(beta (v - eta)), with sinh a sinh b = (cosh(a+b) - cosh(a-b)) / 2
    // and 1 / cosh^2 = 1 - tanh^2: one more hyperbolic function per element
    // instead of three
    __device__ double deta_t(double v, double t) const {
        return -beta * csch * (1.0 - t * t) * 0.5 * (chb - cosh(beta * (2.0 * v - 1.0)));
    }
    __device__ double prj(double v) const { return prj_t(th(v)); }
    __device__ double dprj(double v) const { return dprj_t(th(v)); }
};

template <typename T>
__device__ __forceinline__ double pre_value(const T* xt, const T* x, const uint8_t* pas, int64_t e) {
    uint8_t c = pas[e];
    if (c == TO_ACTIVE) return (double)xt[e];
    if (x) return (double)x[e];
    return c == TO_SOLID ? 1.0 : 0.0;
}

template <typename T>
struct ProjArgs {
    int64_t m;
    int ft;
    const T* xt; const T* x; const uint8_t* pas;
    T* xphys; T* dprj;
    double beta;
    double* d_eta;
    double target;
    int mean_target;
    const T* xold;
    to_project_stats* st;
    double* partial;
    unsigned* bar;
    const double* dyn;      // batch: device (beta, target) replacing the fields above (nullable)
};

// The whole block for one design, run by `nb` blocks of which this is `bid`.
template <typename T>
__device__ void project_body(const ProjArgs<T>& a, int bid, int nb) {
    constexpr int NB = kBigBlock;
    __shared__ double sh[NB / 64];
    __shared__ double red[4];   // grid sums of up to four values
    const int64_t m = a.m;
    const T* __restrict__ xt = a.xt;
    const T* __restrict__ x = a.x;
    const uint8_t* __restrict__ pas = a.pas;
    // two partial regions used in turn: a block may write the next sums while
    // a slower one still reads the previous ones, so each grid sum needs one
    // barrier (a block cannot write a region again before every block has
    // passed the barrier that follows its reads)
    double* const part0 = a.partial;
    int region = 0;
    auto partial_now = [&]() { return part0 + (size_t)region * kMaxCoopBlocks * kPartialWidth; };
    const int64_t stride = (int64_t)nb * NB;
    const int64_t i0 = (int64_t)bid * NB + threadIdx.x;
    double eta = *a.d_eta;
    double target = a.dyn ? a.dyn[1] : a.target;
    const double beta = a.dyn ? a.dyn[0] : a.beta;
    const int mean_target = a.dyn ? (isnan(target) ? 1 : 0) : a.mean_target;
    const int ft = a.ft;
    bool alive = true;
    GridBar gb;
    gb.init(a.bar, bid, nb);

    if (ft == 3 && mean_target) {                   // eq. (17): target = volume of the pre-projection field
        double s = 0.0;
        for (int64_t e = i0; e < m; e += stride) s += pre_value(xt, x, pas, e);
        s = block_sum<NB>(s, sh);
        if (threadIdx.x == 0) st_dev(&partial_now()[bid], s);
        alive = gb.sync();
        grid_reduce<1, NB>(partial_now(), red, sh, nb);
        target = red[0] / (double)m;
        region ^= 1;
    }

    // One sweep writes xphys and dprj at the current threshold and sums the
    // change and the volume; with ft = 3 the same sweep also sums prj and
    // d prj / d eta for the Newton test.  If the test passes (|g| <= 1e-6),
    // the values just written are the final ones and no further sweep is
    // made; otherwise the threshold takes its Newton step and the next sweep
    // overwrites them.  The results are those of separate Newton and output
    // sweeps: every value is computed from the same operands.
    int steps = 0;
    double g = 0.0;
    ProjCoef P;
    double rsum[4] = {0.0, 0.0, 0.0, 0.0};   // change^2, volume, sum prj, sum d prj / d eta
    for (;;) {
        P.set(beta, eta);
        double sc = 0.0, sv = 0.0, sp = 0.0, sd = 0.0;
        if (alive)
            for (int64_t e = i0; e < m; e += stride) {
                const double v = pre_value(xt, x, pas, e);
                const double xte = (double)xt[e];
                double xp = v, dp = 1.0;
                if (ft >= 2) {
                    const double t = P.th(v);        // for active elements v is xtilde: one tanh serves all
                    xp = P.prj_t(t);
                    dp = P.dprj_t(v == xte ? t : P.th(xte));
                    if (ft == 3) {
                        sp += xp;
                        sd += P.deta_t(v, t);
                    }
                }
                const T xpT = (T)xp;
                a.xphys[e] = xpT;
                a.dprj[e] = (T)dp;
                if (a.xold) {
                    const double dlt = (double)xpT - (double)a.xold[e];
                    sc += dlt * dlt;
                }
                sv += (double)xpT;
            }
        sc = block_sum<NB>(sc, sh);
        sv = block_sum<NB>(sv, sh);
        if (ft == 3) {
            sp = block_sum<NB>(sp, sh);
            sd = block_sum<NB>(sd, sh);
        }
        if (threadIdx.x == 0) {
            double* pn = partial_now();
            st_dev(&pn[bid], sc);
            st_dev(&pn[kMaxCoopBlocks + bid], sv);
            if (ft == 3) {
                st_dev(&pn[2 * kMaxCoopBlocks + bid], sp);
                st_dev(&pn[3 * kMaxCoopBlocks + bid], sd);
            }
        }
        alive = gb.sync() && alive;
        if (ft == 3) grid_reduce<4, NB>(partial_now(), red, sh, nb);
        else grid_reduce<2, NB>(partial_now(), red, sh, nb);
        region ^= 1;
        for (int k = 0; k < 4; ++k) rsum[k] = red[k];
        if (ft != 3) break;
        g = rsum[2] / (double)m - target;
        if (!(fabs(g) > 1e-6) || steps >= 50 || !alive) break;
        eta = eta - g / (rsum[3] / (double)m);
        ++steps;
    }
    if (bid == 0 && threadIdx.x == 0) {
        to_project_stats s;
        s.eta = eta;
        s.g = g;
        s.ch = a.xold ? sqrt(rsum[0]) / sqrt((double)m) : NAN;
        s.vol = rsum[1] / (double)m;
        s.n_newton = steps;
        s.converged = (ft != 3 || fabs(g) <= 1e-6) && alive ? 1 : 0;
        s.pad[0] = s.pad[1] = 0;
        *a.st = s;
        *a.d_eta = eta;
    }
}

template <typename T>
__global__ __launch_bounds__(kBigBlock) void project_kernel(ProjArgs<T> a) {
    project_body(a, blockIdx.x, gridDim.x);
}

// A batch of designs in one launch: block b works on design inst[b], as block
// b - first[inst] of its group of count[inst] blocks.
template <typename T>
__global__ __launch_bounds__(kBigBlock) void project_batch_kernel(const ProjArgs<T>* __restrict__ tab,
                                                                  const int32_t* __restrict__ inst,
                                                                  const int32_t* __restrict__ first,
                                                                  const int32_t* __restrict__ count) {
    const int i = inst[blockIdx.x];
    project_body(tab[i], (int)blockIdx.x - first[i], count[i]);
}

int coop_blocks_for(const void* kernel, int block, size_t smem, int num_cu) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, smem) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return std::min(kMaxCoopBlocks, per_cu * num_cu);
}

hipError_t launch_resident(const Plan* p, const void* kernel, int blocks, int block, void** args, hipStream_t s) {
    if (p->tune.coop_launch) return hipLaunchCooperativeKernel(kernel, dim3(blocks), dim3(block), args, 0, s);
    return hipLaunchKernel(kernel, dim3(blocks), dim3(block), args, 0, s);
}

template <typename T>
static ProjArgs<T> proj_args(Plan* p, int ft, const void* xt, const void* x, void* xphys, void* dprj, double beta,
                             double* d_eta, double target, const void* xold, to_project_stats* st) {
    ProjArgs<T> a{};
    a.m = p->info.m; a.ft = ft;
    a.xt = (const T*)xt; a.x = (const T*)x; a.pas = p->passive;
    a.xphys = (T*)xphys; a.dprj = (T*)dprj;
    a.beta = beta; a.d_eta = d_eta; a.target = target; a.mean_target = std::isnan(target) ? 1 : 0;
    a.xold = (const T*)xold; a.st = st;
    a.partial = p->partial; a.bar = p->bar;
    return a;
}

template <typename T>
static to_status run_project(Plan* p, int ft, const void* xt, const void* x, void* xphys, void* dprj,
                             double beta, double* d_eta, double target, const void* xold,
                             to_project_stats* st, hipStream_t s) {
    auto k = project_kernel<T>;
    int64_t m = p->info.m;
    int maxb = coop_blocks_for((const void*)k, kBigBlock, 0, p->num_cu);
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(maxb, p->num_cu), (m + kBigBlock - 1) / kBigBlock));
    ProjArgs<T> a = proj_args<T>(p, ft, xt, x, xphys, dprj, beta, d_eta, target, xold, st);
    void* args[] = {&a};
    TO_HIP(launch_resident(p, (const void*)k, blocks, kBigBlock, args, s));
    return TO_OK;
}

size_t project_args_bytes(to_dtype dt) { return dt == TO_F64 ? sizeof(ProjArgs<double>) : sizeof(ProjArgs<float>); }

void project_args_fill(Plan* p, to_dtype dt, int ft, const void* xt, const void* x, void* xphys, void* dprj,
                       double* d_eta, const void* xold, to_project_stats* st, const double* dyn, void* dst) {
    if (dt == TO_F64) {
        ProjArgs<double> a = proj_args<double>(p, ft, xt, x, xphys, dprj, 0.0, d_eta, NAN, xold, st);
        a.dyn = dyn;
        std::memcpy(dst, &a, sizeof a);
    } else {
        ProjArgs<float> a = proj_args<float>(p, ft, xt, x, xphys, dprj, 0.0, d_eta, NAN, xold, st);
        a.dyn = dyn;
        std::memcpy(dst, &a, sizeof a);
    }
}

int project_batch_capacity(to_dtype dt, int num_cu) {
    const void* k = dt == TO_F64 ? (const void*)project_batch_kernel<double> : (const void*)project_batch_kernel<float>;
    return coop_blocks_for(k, kBigBlock, 0, num_cu);
}

to_status launch_project_batch(to_dtype dt, const void* tab, const BatchMap& mp, hipStream_t s) {
    const void* k = dt == TO_F64 ? (const void*)project_batch_kernel<double> : (const void*)project_batch_kernel<float>;
    void* args[] = {(void*)&tab, (void*)&mp.inst, (void*)&mp.first, (void*)&mp.count};
    TO_HIP(hipLaunchCooperativeKernel(k, dim3(mp.blocks), dim3(kBigBlock), args, 0, s));
    return TO_OK;
}

to_status launch_project(Plan* p, to_dtype dt, int ft, const void* xt, const void* x, void* xphys,
                         void* dprj, double beta, double* d_eta, double target, const void* xold,
                         to_project_stats* st, hipStream_t s) {
    if (dt == TO_F64) return run_project<double>(p, ft, xt, x, xphys, dprj, beta, d_eta, target, xold, st, s);
    return run_project<float>(p, ft, xt, x, xphys, dprj, beta, d_eta, target, xold, st, s);
}

}  // namespace topt
