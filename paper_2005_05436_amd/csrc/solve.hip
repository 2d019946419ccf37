// State solve K(free, free) u = f (eq. (5)) by Jacobi-preconditioned CG, in
// one persistent, cooperatively launched kernel per call.
//
// Operators (node-centric, gather only, deterministic):
//   Csr      the assembled K^(s) of eq. (14): row r of the full matrix (eq. (15))
//            is the lower row plus the strictly-lower entries of column r,
//            reached through the plan's transpose map (no atomics).
//   MatFree  K = sum_e E_e A_e^T Ke A_e applied node by node: each node sums
//            the rows of the (up to 4 or 8) adjacent element matrices, with
//            the element matrix indices fixed at compile time (scalar loads).
// Fixed DOFs: vectors are kept zero there; the operator's rows are masked.
//
// CG with two grid barriers per iteration: the SpMV builds the new direction
// p = z + beta p_old on the fly from z and the previous direction (double
// buffered), so no separate direction update phase is needed.  All dot
// products are FP64, reduced in a fixed order identical in every block.
//
// Mixed precision (FP32 fields): outer FP64 residual from the FP64 matrix-free
// operator, inner FP32 PCG, u += d; FP64 PCG fallback when the refinement
// stalls.
#include <cmath>

#include "common.h"

namespace topt {

struct Geo {
    int nx, ny, nz;
    int64_t nnode;
    __device__ __forceinline__ void coords(int64_t nd, int& iy, int& ix, int& iz, int dim) const {
        iy = (int)(nd % (ny + 1));
        int64_t rest = nd / (ny + 1);
        if (dim == 2) { ix = (int)rest; iz = 0; }
        else { iz = (int)(rest % (nz + 1)); ix = (int)(rest / (nz + 1)); }
    }
};

template <typename T> struct Src1 {
    const T* __restrict__ x;
    __device__ __forceinline__ T operator()(int64_t i) const { return x[i]; }
};
template <typename T> struct SrcZP {
    const T* __restrict__ z;
    const T* __restrict__ p;
    T beta;
    __device__ __forceinline__ T operator()(int64_t i) const { return z[i] + beta * p[i]; }
};

template <int DIM, typename T>
struct MatFree {
    const T* __restrict__ E;     // m moduli
    const T* __restrict__ ke;    // d x d, row major
    int nx, ny, nz;
    static constexpr int NC = DIM == 2 ? 4 : 8;
    static constexpr int D = DIM * NC;

    __device__ __forceinline__ int64_t node(int y, int x, int z) const {
        return DIM == 2 ? y + (int64_t)(ny + 1) * x : y + (int64_t)(ny + 1) * (z + (int64_t)(nz + 1) * x);
    }
    // The element loop is not unrolled: each pass gathers one element's D
    // source values into registers and applies this node's DIM rows of Ke,
    // whose (wave-uniform) entries come through the scalar cache.  Fully
    // unrolling it would keep all of Ke live in registers.
    template <class S>
    __device__ __forceinline__ void apply(int64_t, int iy, int ix, int iz, const S& src, T (&out)[DIM]) const {
        constexpr int CY[8] = {1, 1, 0, 0, 1, 1, 0, 0};
        constexpr int CX[8] = {0, 1, 1, 0, 0, 1, 1, 0};
        constexpr int CZ[8] = {0, 0, 0, 0, 1, 1, 1, 1};
#pragma unroll
        for (int c = 0; c < DIM; ++c) out[c] = T(0);
#pragma unroll 1
        for (int a = 0; a < NC; ++a) {
            const int ey = iy - CY[a], ex = ix - CX[a], ez = iz - CZ[a];
            const bool in = ey >= 0 && ey < ny && ex >= 0 && ex < nx && (DIM == 2 || (ez >= 0 && ez < nz));
            if (!in) continue;
            const int64_t e = DIM == 2 ? ey + (int64_t)ny * ex : ey + (int64_t)ny * (ez + (int64_t)nz * ex);
            const T Ee = E[e];
            T sv[D];
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                const int64_t q = node(ey + CY[b], ex + CX[b], DIM == 2 ? 0 : ez + CZ[b]);
#pragma unroll
                for (int c2 = 0; c2 < DIM; ++c2) sv[b * DIM + c2] = src(DIM * q + c2);
            }
            const T* kr = ke + (size_t)a * DIM * D;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                T acc = T(0);
#pragma unroll
                for (int j = 0; j < D; ++j) acc += kr[c * D + j] * sv[j];
                out[c] += Ee * acc;
            }
        }
    }
    __device__ __forceinline__ void diag(int64_t, int iy, int ix, int iz, T (&out)[DIM]) const {
        constexpr int CY[8] = {1, 1, 0, 0, 1, 1, 0, 0};
        constexpr int CX[8] = {0, 1, 1, 0, 0, 1, 1, 0};
        constexpr int CZ[8] = {0, 0, 0, 0, 1, 1, 1, 1};
#pragma unroll
        for (int c = 0; c < DIM; ++c) out[c] = T(0);
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            const int ey = iy - CY[a], ex = ix - CX[a], ez = iz - CZ[a];
            const bool in = ey >= 0 && ey < ny && ex >= 0 && ex < nx && (DIM == 2 || (ez >= 0 && ez < nz));
            if (!in) continue;
            const int64_t e = DIM == 2 ? ey + (int64_t)ny * ex : ey + (int64_t)ny * (ez + (int64_t)nz * ex);
            const T Ee = E[e];
#pragma unroll
            for (int c = 0; c < DIM; ++c) out[c] += Ee * ke[(a * DIM + c) * D + a * DIM + c];
        }
    }
};

template <int DIM, typename T>
struct Csr {
    const int32_t* __restrict__ rp;
    const int32_t* __restrict__ ci;
    const int32_t* __restrict__ tp;
    const int32_t* __restrict__ ts;
    const int32_t* __restrict__ tr;
    const T* __restrict__ kv;
    template <class S>
    __device__ __forceinline__ void apply(int64_t nd, int, int, int, const S& src, T (&out)[DIM]) const {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t r = DIM * nd + c;
            T acc = T(0);
            for (int32_t s = rp[r]; s < rp[r + 1]; ++s) acc += kv[s] * src(ci[s]);
            for (int32_t k = tp[r]; k < tp[r + 1]; ++k) acc += kv[ts[k]] * src(tr[k]);
            out[c] = acc;
        }
    }
    __device__ __forceinline__ void diag(int64_t nd, int, int, int, T (&out)[DIM]) const {
#pragma unroll
        for (int c = 0; c < DIM; ++c) out[c] = kv[rp[DIM * nd + c + 1] - 1];   // last lower entry
    }
};

struct SolveArgs {
    Geo geo;
    const uint8_t* freem;
    const int32_t *rp, *ci, *tp, *ts, *tr;
    const void* kval;
    const double* E64; const float* E32;
    const double* kf64; const float* kf32;
    const double* f; double* u;
    double* v64[8];
    float* v32[8];
    double rtol, inner_rtol;
    int maxit, max_outer, zero_x0;
    double* partial; unsigned* bar;
    to_solve_stats* st;
};

// per-kernel reduction context: double-buffered partial regions, so a fast
// block can write reduction k+1 while slow blocks still read reduction k
struct Ctx {
    double* partial;
    unsigned* bar;
    double* sh;
    double* res;     // shared results
    int red;
    bool alive;
    template <int K>
    __device__ __forceinline__ void reduce(const double (&v)[K]) {
        double* region = partial + (size_t)(red & 1) * kMaxCoopBlocks * kPartialWidth;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = block_sum(v[k], sh);
            if (threadIdx.x == 0) region[blockIdx.x * kPartialWidth + k] = s;
        }
        alive = grid_sync(bar) && alive;
        grid_reduce<K>(region, res, sh);
        ++red;
    }
};

template <int DIM, typename T, class Op>
struct Pcg {
    const Op& op;
    const Geo& g;
    const uint8_t* __restrict__ fm;
    Ctx& C;

    // r = b - A x (x = 0: r = b), z = dinv r; returns (r.z, r.r) in C.res
    __device__ void residual(const T* b, const T* x, bool x_zero, const T* dinv, T* r, T* z) {
        double v[2] = {0.0, 0.0};
        const int64_t stride = (int64_t)gridDim.x * kBlock;
        for (int64_t nd = (int64_t)blockIdx.x * kBlock + threadIdx.x; nd < g.nnode; nd += stride) {
            int iy, ix, iz;
            g.coords(nd, iy, ix, iz, DIM);
            T ax[DIM];
            if (!x_zero) op.apply(nd, iy, ix, iz, Src1<T>{x}, ax);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const int64_t i = DIM * nd + c;
                T ri = fm[i] ? (x_zero ? b[i] : b[i] - ax[c]) : T(0);
                T zi = dinv[i] * ri;
                r[i] = ri;
                z[i] = zi;
                v[0] += (double)ri * (double)zi;
                v[1] += (double)ri * (double)ri;
            }
        }
        C.reduce<2>(v);
    }

    // Solves A x = b from x (x_zero: from 0) until |r| <= tol; returns iterations.
    __device__ int run(const T* b, T* x, bool x_zero, const T* dinv, T* r, T* z, T* pa, T* pb, T* q,
                       double tol, int maxit, int& restarts) {
        const int64_t stride = (int64_t)gridDim.x * kBlock;
        const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
        if (x_zero)
            for (int64_t nd = i0; nd < g.nnode; nd += stride)
#pragma unroll
                for (int c = 0; c < DIM; ++c) x[DIM * nd + c] = T(0);
        residual(b, x, x_zero, dinv, r, z);
        double rz = C.res[0], rr = C.res[1];
        bool fresh = true;
        double beta = 0.0;
        T* pold = z;   // beta = 0: the first direction is z
        T* pnew = pa;
        int it = 0;
        while (C.alive) {
            if (rr <= tol * tol) {
                if (fresh) break;
                residual(b, x, false, dinv, r, z);   // confirm on the recomputed residual
                rz = C.res[0]; rr = C.res[1];
                fresh = true; beta = 0.0; pold = z; pnew = pa;
                if (rr <= tol * tol) break;
                ++restarts;
            }
            if (it >= maxit) break;
            fresh = false;
            // phase A: pnew = z + beta pold; q = A pnew
            double v1[1] = {0.0};
            const SrcZP<T> src{z, pold, (T)beta};
            for (int64_t nd = i0; nd < g.nnode; nd += stride) {
                int iy, ix, iz;
                g.coords(nd, iy, ix, iz, DIM);
                T ap[DIM];
                op.apply(nd, iy, ix, iz, src, ap);
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    const int64_t i = DIM * nd + c;
                    const T pi = src(i);
                    const T qi = fm[i] ? ap[c] : T(0);
                    pnew[i] = pi;
                    q[i] = qi;
                    v1[0] += (double)pi * (double)qi;
                }
            }
            C.reduce<1>(v1);
            const double pq = C.res[0];
            if (!(pq > 0.0)) break;        // breakdown (zero or non-finite direction)
            const double alpha = rz / pq;
            // phase B: x += alpha p; r -= alpha q; z = dinv r
            double v2[2] = {0.0, 0.0};
            const T a = (T)alpha;
            for (int64_t nd = i0; nd < g.nnode; nd += stride) {
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    const int64_t i = DIM * nd + c;
                    x[i] += a * pnew[i];
                    const T ri = r[i] - a * q[i];
                    const T zi = dinv[i] * ri;
                    r[i] = ri;
                    z[i] = zi;
                    v2[0] += (double)ri * (double)zi;
                    v2[1] += (double)ri * (double)ri;
                }
            }
            C.reduce<2>(v2);
            beta = C.res[0] / rz;
            rz = C.res[0];
            rr = C.res[1];
            T* t = pnew == pa ? pb : pa;
            pold = pnew;
            pnew = t;
            ++it;
        }
        if (!fresh && C.alive) residual(b, x, false, dinv, r, z);   // report the true residual
        return it;
    }
};

template <int DIM, typename T, class Op>
__device__ void jacobi(const Op& op, const Geo& g, const uint8_t* fm, T* dinv) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t nd = (int64_t)blockIdx.x * kBlock + threadIdx.x; nd < g.nnode; nd += stride) {
        int iy, ix, iz;
        g.coords(nd, iy, ix, iz, DIM);
        T dg[DIM];
        op.diag(nd, iy, ix, iz, dg);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t i = DIM * nd + c;
            dinv[i] = fm[i] && dg[c] != T(0) ? T(1) / dg[c] : T(0);
        }
    }
}

// MODE 0: FP64, assembled operator; 1: FP64, matrix-free;
//      2: mixed, FP32 assembled inner; 3: mixed, FP32 matrix-free inner.
template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void solve_kernel(SolveArgs A) {
    __shared__ double sh[kWaves];
    __shared__ double res[4];
    Ctx C{A.partial, A.bar, sh, res, 0, true};
    const Geo& g = A.geo;
    const int64_t n = g.nnode * DIM;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double* u = A.u;

    // |f_free|, and u = 0 on fixed DOFs (or everywhere when asked)
    {
        double v[1] = {0.0};
        for (int64_t i = i0; i < n; i += stride) {
            const bool fr = A.freem[i] != 0;
            if (!fr || A.zero_x0) u[i] = 0.0;
            const double fi = fr ? A.f[i] : 0.0;
            v[0] += fi * fi;
        }
        C.reduce<1>(v);
    }
    const double bnorm = sqrt(res[0]);
    const double tol = A.rtol * bnorm;
    int iters = 0, restarts = 0, outer = 0, fallback = 0;
    double resid = 0.0;

    MatFree<DIM, double> mf64{A.E64, A.kf64, g.nx, g.ny, g.nz};
    if (MODE <= 1) {
        double *r = A.v64[0], *z = A.v64[1], *pa = A.v64[2], *pb = A.v64[3], *q = A.v64[4], *dinv = A.v64[5];
        if (MODE == 0) {
            Csr<DIM, double> op{A.rp, A.ci, A.tp, A.ts, A.tr, (const double*)A.kval};
            jacobi<DIM, double>(op, g, A.freem, dinv);
            Pcg<DIM, double, Csr<DIM, double>> cg{op, g, A.freem, C};
            iters = cg.run(A.f, u, false, dinv, r, z, pa, pb, q, tol, A.maxit, restarts);
        } else {
            jacobi<DIM, double>(mf64, g, A.freem, dinv);
            Pcg<DIM, double, MatFree<DIM, double>> cg{mf64, g, A.freem, C};
            iters = cg.run(A.f, u, false, dinv, r, z, pa, pb, q, tol, A.maxit, restarts);
        }
        resid = sqrt(C.res[1]) / (bnorm > 0 ? bnorm : 1.0);
    } else {
        double *r64 = A.v64[0], *z64 = A.v64[1], *pa64 = A.v64[2], *pb64 = A.v64[3], *q64 = A.v64[4];
        double* dinv64 = A.v64[5];
        float *b32 = A.v32[0], *d32 = A.v32[1], *r32 = A.v32[2], *z32 = A.v32[3], *pa32 = A.v32[4];
        float *pb32 = A.v32[5], *q32 = A.v32[6], *dinv32 = A.v32[7];
        Csr<DIM, float> csr32{A.rp, A.ci, A.tp, A.ts, A.tr, (const float*)A.kval};
        MatFree<DIM, float> mf32{A.E32, A.kf32, g.nx, g.ny, g.nz};
        if (MODE == 2) jacobi<DIM, float>(csr32, g, A.freem, dinv32);
        else jacobi<DIM, float>(mf32, g, A.freem, dinv32);
        jacobi<DIM, double>(mf64, g, A.freem, dinv64);   // for the fallback
        Pcg<DIM, double, MatFree<DIM, double>> cg64{mf64, g, A.freem, C};
        double prev = INFINITY;
        int stall = 0;
        bool converged = false;
        for (;;) {
            // outer FP64 residual r = f - K64 u
            cg64.residual(A.f, u, false, dinv64, r64, z64);
            const double rn = sqrt(C.res[1]);
            resid = rn / (bnorm > 0 ? bnorm : 1.0);
            if (rn <= tol || !C.alive) { converged = rn <= tol; break; }
            stall = rn > 0.5 * prev ? stall + 1 : 0;
            if (outer >= A.max_outer || stall >= 2 || iters >= A.maxit) break;
            prev = rn;
            for (int64_t nd = i0; nd < g.nnode; nd += stride)
#pragma unroll
                for (int c = 0; c < DIM; ++c) b32[DIM * nd + c] = (float)r64[DIM * nd + c];
            const double itol = A.inner_rtol * rn;
            int left = A.maxit - iters;
            if (MODE == 2) {
                Pcg<DIM, float, Csr<DIM, float>> cg{csr32, g, A.freem, C};
                iters += cg.run(b32, d32, true, dinv32, r32, z32, pa32, pb32, q32, itol, left, restarts);
            } else {
                Pcg<DIM, float, MatFree<DIM, float>> cg{mf32, g, A.freem, C};
                iters += cg.run(b32, d32, true, dinv32, r32, z32, pa32, pb32, q32, itol, left, restarts);
            }
            for (int64_t nd = i0; nd < g.nnode; nd += stride)
#pragma unroll
                for (int c = 0; c < DIM; ++c) u[DIM * nd + c] += (double)d32[DIM * nd + c];
            C.alive = grid_sync(A.bar) && C.alive;
            ++outer;
        }
        if (!converged && C.alive) {
            fallback = 1;
            int left = A.maxit - iters;
            iters += cg64.run(A.f, u, false, dinv64, r64, z64, pa64, pb64, q64, tol, left > 0 ? left : 0, restarts);
            resid = sqrt(C.res[1]) / (bnorm > 0 ? bnorm : 1.0);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        to_solve_stats s;
        s.residual = resid;
        s.bnorm = bnorm;
        s.iterations = iters;
        s.outer = outer;
        s.converged = (resid <= A.rtol && C.alive) ? 1 : 0;
        s.fallback = fallback;
        s.restarts = restarts;
        s.pad = C.alive ? 0 : 1;
        *A.st = s;
    }
}

template <int DIM, int MODE>
static to_status launch_solve_t(Plan* p, SolveArgs& A, hipStream_t s) {
    auto k = solve_kernel<DIM, MODE>;
    int maxb = coop_blocks_for((const void*)k, kBlock, 0, p->num_cu);
    int64_t want = (A.geo.nnode + kBlock - 1) / kBlock;
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(maxb, 2 * p->num_cu), want));
    void* args[] = {&A};
    TO_HIP(hipLaunchCooperativeKernel((const void*)k, dim3(blocks), dim3(kBlock), args, 0, s));
    return TO_OK;
}

to_status launch_solve(Plan* p, to_dtype dt, const void* kval, const void* xphys, double penal,
                       const double* f, double* u, const to_solve_opts& o, to_solve_stats* st, hipStream_t s) {
    const bool assembled = o.op == TO_OP_ASSEMBLED;
    if (dt == TO_F32 && assembled && !kval) { set_error("kval is NULL"); return TO_EINVAL; }
    if (dt == TO_F64 && assembled && !kval) { set_error("kval is NULL"); return TO_EINVAL; }
    // moduli for the matrix-free operators (FP64 always; FP32 too in mixed mode)
    if (!(dt == TO_F64 && assembled)) {
        to_status r = launch_moduli(p, dt, xphys, penal, s, true);
        if (r != TO_OK) return r;
    }
    SolveArgs A{};
    A.geo = Geo{p->nelx, p->nely, p->nelz, p->info.nnode};
    A.freem = p->freemask;
    A.rp = p->row_ptr; A.ci = p->col_idx; A.tp = p->tptr; A.ts = p->tslot; A.tr = p->trow;
    A.kval = kval;
    A.E64 = p->E64; A.E32 = p->E32; A.kf64 = p->kf64; A.kf32 = p->kf32;
    A.f = f; A.u = u;
    for (int i = 0; i < 8; ++i) { A.v64[i] = p->v64[i]; A.v32[i] = p->v32[i]; }
    A.rtol = o.rtol; A.inner_rtol = o.inner_rtol; A.maxit = o.maxit; A.max_outer = o.max_outer;
    A.zero_x0 = o.zero_x0;
    A.partial = p->partial; A.bar = p->bar; A.st = st;
    const int mode = dt == TO_F64 ? (assembled ? 0 : 1) : (assembled ? 2 : 3);
    if (p->dim == 2) {
        switch (mode) {
        case 0: return launch_solve_t<2, 0>(p, A, s);
        case 1: return launch_solve_t<2, 1>(p, A, s);
        case 2: return launch_solve_t<2, 2>(p, A, s);
        default: return launch_solve_t<2, 3>(p, A, s);
        }
    }
    switch (mode) {
    case 0: return launch_solve_t<3, 0>(p, A, s);
    case 1: return launch_solve_t<3, 1>(p, A, s);
    case 2: return launch_solve_t<3, 2>(p, A, s);
    default: return launch_solve_t<3, 3>(p, A, s);
    }
}

}  // namespace topt
