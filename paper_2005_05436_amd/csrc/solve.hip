// State solve K(free, free) u = f (eq. (5)) by Jacobi-preconditioned CG, in
// one persistent, cooperatively launched kernel per call.
//
// Operators (node-centric, gather only, deterministic):
//   CsrS     the assembled K^(s) of eq. (14) in its CSR order, addressed through
//            the grid structure (full matrix by eq. (15), no atomics).
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
// Work split: block b owns the contiguous node range [lo, hi).  Vectors
// written by the owner and read by a neighbour node in another block (the
// iterate, z and the directions) are stored device-coherently (st_dev) only
// in the band of nodes within one neighbourhood of the range ends, and read
// device-coherently (ld_dev) only when the node is not the block's own; all
// other accesses are ordinary cached loads and stores.
//
// Mixed precision (FP32 fields): FP32 CG with FP64 residual replacement from
// the FP64 matrix-free operator; FP64 PCG fallback when it stalls.
#include <cmath>
#include <cstring>
#include <type_traits>

#include "common.h"
#include "operators.h"

namespace topt {

// The assembled K^(s) in the plan's CSR order, read with the structure of the
// grid instead of column indices.  The lower row of DOF (n, c) holds, for each
// existing neighbour q < n in ascending node order, the DIM entries of q, then
// components 0..c of n itself.  So the (n, q) block of the full matrix
// (eq. (15)) is found at row_ptr[DIM n + c] + DIM * rank_n(q) + c' for q < n,
// and, for q > n, as the transpose of the (q, n) block in q's rows at
// DIM * rank_q(n); the ranks are prefix counts of which neighbours exist
// (boundary nodes have fewer).  Only row_ptr and the values are read; each
// lower value is read once for its own row and once as a transposed entry.
template <int DIM, typename T>
struct CsrS {
    const int32_t* __restrict__ rp;
    const T* __restrict__ kv;
    int nx, ny, nz;
    static constexpr int NN = DIM == 2 ? 9 : 27;    // neighbourhood incl. the node itself
    static constexpr int SELF = NN / 2;
    // neighbour k in ascending node order: (dx, dz, dy) lexicographic
    __device__ __forceinline__ static void off(int k, int& dx, int& dy, int& dz) {
        if (DIM == 2) { dx = k / 3 - 1; dy = k % 3 - 1; dz = 0; }
        else { dx = k / 9 - 1; dz = (k / 3) % 3 - 1; dy = k % 3 - 1; }
    }
    __device__ __forceinline__ bool exists(int iy, int ix, int iz, int k) const {
        int dx, dy, dz;
        off(k, dx, dy, dz);
        const int y = iy + dy, x = ix + dx, z = iz + dz;
        return y >= 0 && y <= ny && x >= 0 && x <= nx && (DIM == 2 || (z >= 0 && z <= nz));
    }
    __device__ __forceinline__ int64_t delta(int k) const {
        int dx, dy, dz;
        off(k, dx, dy, dz);
        return DIM == 2 ? dy + (int64_t)(ny + 1) * dx : dy + (int64_t)(ny + 1) * (dz + (int64_t)(nz + 1) * dx);
    }
    // any node: existence tests on every neighbour, ranks counted
    template <class S>
    __device__ __forceinline__ void apply_general(int64_t nd, int iy, int ix, int iz, const S& src,
                                                  T (&out)[DIM]) const {
        int32_t row[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) { row[c] = rp[DIM * nd + c]; out[c] = T(0); }
        int rank = 0;
#pragma unroll
        for (int k = 0; k < SELF; ++k) {                       // lower neighbours
            if (!exists(iy, ix, iz, k)) continue;
            const int64_t q = nd + delta(k);
#pragma unroll
            for (int c2 = 0; c2 < DIM; ++c2) {
                const T sv = src(q, c2);
#pragma unroll
                for (int c = 0; c < DIM; ++c) out[c] += kv[row[c] + DIM * rank + c2] * sv;
            }
            ++rank;
        }
#pragma unroll
        for (int c2 = 0; c2 < DIM; ++c2) {                      // the node's own block
            const T sv = src(nd, c2);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const T kvv = c2 <= c ? kv[row[c] + DIM * rank + c2] : kv[row[c2] + DIM * rank + c];
                out[c] += kvv * sv;
            }
        }
#pragma unroll
        for (int k = SELF + 1; k < NN; ++k) {                  // upper neighbours: transposed blocks
            if (!exists(iy, ix, iz, k)) continue;
            int dx, dy, dz;
            off(k, dx, dy, dz);
            const int qy = iy + dy, qx = ix + dx, qz = iz + dz;
            const int64_t q = nd + delta(k);
            const int km = NN - 1 - k;                         // n seen from q
            int rq = 0;
#pragma unroll
            for (int j = 0; j < km; ++j) rq += exists(qy, qx, qz, j) ? 1 : 0;
#pragma unroll
            for (int c2 = 0; c2 < DIM; ++c2) {
                const T sv = src(q, c2);
                const int32_t rq0 = rp[DIM * q + c2] + DIM * rq;
#pragma unroll
                for (int c = 0; c < DIM; ++c) out[c] += kv[rq0 + c] * sv;
            }
        }
    }
    template <class S>
    __device__ __forceinline__ void apply(int64_t nd, int iy, int ix, int iz, const S& src, T (&out)[DIM]) const {
        // 2D FP64 only: there the loop form of the far case measured faster
        // than the unrolled general one (101 against 135 us per CG iteration
        // at 1200x400); in 3D (461 against 368 us at 96x48x48) and with FP32
        // values (103 against 98 us) slower
        constexpr bool kFar = DIM == 2 && sizeof(T) == 8;
        const bool far = kFar && iy >= 2 && iy <= ny - 2 && ix >= 2 && ix <= nx - 2;
        if (far) apply_far(nd, src, out);
        else apply_general(nd, iy, ix, iz, src, out);
    }
    // a node at least two layers from every boundary: all its neighbours and
    // all of theirs exist, so the rank of neighbour k in the node's row is k
    // and that of the node in the row of upper neighbour k is NN-1-k (no
    // existence tests, no rank counting); kept as rolled loops
    template <class S>
    __device__ __forceinline__ void apply_far(int64_t nd, const S& src, T (&out)[DIM]) const {
        int32_t row[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) { row[c] = rp[DIM * nd + c]; out[c] = T(0); }
#pragma unroll 1
        for (int k = 0; k < SELF; ++k) {                       // lower neighbours, rank k
            const int64_t q = nd + delta(k);
#pragma unroll
            for (int c2 = 0; c2 < DIM; ++c2) {
                const T sv = src(q, c2);
#pragma unroll
                for (int c = 0; c < DIM; ++c) out[c] += kv[row[c] + DIM * k + c2] * sv;
            }
        }
#pragma unroll
        for (int c2 = 0; c2 < DIM; ++c2) {                      // the node's own block, rank SELF
            const T sv = src(nd, c2);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const T kvv = c2 <= c ? kv[row[c] + DIM * SELF + c2] : kv[row[c2] + DIM * SELF + c];
                out[c] += kvv * sv;
            }
        }
#pragma unroll 1
        for (int k = SELF + 1; k < NN; ++k) {                  // upper neighbours: n has rank NN-1-k in q's row
            const int64_t q = nd + delta(k);
            const int rq = NN - 1 - k;
#pragma unroll
            for (int c2 = 0; c2 < DIM; ++c2) {
                const T sv = src(q, c2);
                const int32_t rq0 = rp[DIM * q + c2] + DIM * rq;
#pragma unroll
                for (int c = 0; c < DIM; ++c) out[c] += kv[rq0 + c] * sv;
            }
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
    const int32_t* rp;
    const void* kval;
    const float* kdiag32;       // FP32 assembled values for the Jacobi of the FP64 solve (nullable)
    const double* kdiag64;      // FP64 assembled values for the same (TO_OP_HYBRID; nullable)
    const double* E64; const float* E32;
    const double* kf64; const float* kf32;
    const double* f; double* u;
    double* v64[8];
    float* v32[8];
    double rtol, inner_rtol;
    int maxit, zero_x0;
    int stage;                  // 2D FP64 matrix-free: nodes of the LDS window of the SpMV source (0: off)
    int stage_own;              // with the window: own-node capacity of the LDS copies of dinv, x, p (0: off)
    int stage_e;                // with them: capacity of the LDS copy of the moduli the own nodes touch
    int follow;                 // 2D single-sum launch that continues a pipelined solve which handed over
    double* partial; unsigned* bar;
    unsigned long long* ll;
    to_solve_stats* st;
};

// per-kernel reduction context: double-buffered partial regions, so a fast
// block can write reduction k+1 while slow blocks still read reduction k
struct Ctx {
    double* partial;
    GridBar gb;
    double* sh;
    double* res;     // shared results
    int red;
    bool alive;
    Own o;
    FlagReduce fr;
    template <int K>
    __device__ __forceinline__ void reduce(const double (&v)[K]) {
        alive = fr.reduce<K>(v, res, sh) && alive;
        ++red;
    }
};

// Source of the SpMV read from the block's LDS window: nodes wlo ..
// wlo + wn - 1 (the block's own range and the band on either side), DIM
// values per node.
template <int DIM, typename T>
struct SrcLds {
    const T* w;
    int64_t wlo;
    __device__ __forceinline__ T operator()(int64_t q, int c) const { return w[DIM * (q - wlo) + c]; }
};

// 3D: the SpMV of nodes lo .. hi - 1 reads, in each of the x-planes ix - 1,
// ix, ix + 1, only the nodes within ny + 2 of the range shifted by one
// plane (P = (ny+1)(nz+1) nodes), so the window holds three segments of
// L = hi - lo + 2 (ny + 2) nodes: segment k starts at node wlo + k P
// (wlo = lo - (ny + 2) - P) and at slot k L.  Node q lies at rel = q - wlo
// in [k P, k P + L) for the k it is read with, k = [rel >= P] + [rel >= 2P];
// where segments overlap (L > P) both copies hold the same value.
template <typename T>
struct SrcSeg3 {
    const T* w;
    int64_t wlo;
    int P, S;                // S = P - L
    __device__ __forceinline__ T operator()(int64_t q, int c) const {
        const int rel = (int)(q - wlo);
        return w[3 * (rel - ((rel >= P) + (rel >= 2 * P)) * S) + c];
    }
};

// Hides per-node values from loop-invariant code motion: the neighbour
// masks and addresses derived from them are then recomputed where they are
// used, instead of being held in registers across the whole CG loop for
// every node a thread owns.
__device__ __forceinline__ void opaque(int& a, int& b, int& c, uint32_t& d) {
    asm volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
}

// Iterations between the pipelined PCG's recomputations of its recurrences
// (every 100 keeps the iteration count of PCG on the SIMP test meshes; every
// 400 lost 60%).
constexpr int kPipeReplace = 100;

template <int DIM, typename T, class Op>
struct Pcg {
    const Op& op;
    const Geo& g;
    const uint8_t* __restrict__ fm;
    Ctx& C;
    T* win = nullptr;            // LDS window of the direction (2D; nullptr: gather from memory)
    int64_t wlo = 0, wn = 0;
    int wP = 0, wS = 0;          // 3D: the window's segment shift P and P - L (SrcSeg3)
    T* own = nullptr;            // run1: LDS for x and p of the own nodes, their moduli and the band's dinv

    // r = b - A x (x = 0: r = b), z = dinv r; returns (r.z, r.r) in C.res
    __device__ __forceinline__ void residual(const T* b, const T* x, bool x_zero, const T* dinv, T* r, T* z) {
        double v[2] = {0.0, 0.0};
        const Own& o = C.o;
        for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x) {
            int iy, ix, iz;
            g.coords(nd, iy, ix, iz, DIM);
            T ax[DIM];
            if (!x_zero) op.apply(nd, iy, ix, iz, Src1<DIM, T>{x, o}, ax);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const int64_t i = DIM * nd + c;
                T ri = fm[i] ? (x_zero ? b[i] : b[i] - ax[c]) : T(0);
                T zi = dinv[i] * ri;
                r[i] = ri;
                o.st(z, nd, i, zi);
                v[0] += (double)ri * (double)zi;
                v[1] += (double)ri * (double)ri;
            }
        }
        C.reduce<2>(v);
    }

    // Solves A x = b from x (x_zero: from 0) until |r| <= tol; returns iterations.
    // confirm: accept convergence only when the recomputed residual b - A x
    // also meets tol (FP64 solves).  The inner FP32 solve of the mixed
    // scheme stops on the recursive residual: at high stiffness contrast the
    // FP32 recomputation of b - A x is dominated by cancellation, and the
    // outer FP64 residual is the judge anyway.
    template <bool WIN = true>
    __device__ __forceinline__ int run(const T* b, T* x, bool x_zero, const T* dinv, T* r, T* z, T* pa, T* pb, T* q,
                       double tol, int maxit, int& restarts, bool confirm = true) {
        const Own& o = C.o;
        if (x_zero)
            for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x)
#pragma unroll
                for (int c = 0; c < DIM; ++c) o.st(x, nd, DIM * nd + c, T(0));
        residual(b, x, x_zero, dinv, r, z);
        double rz = C.res[0], rr = C.res[1];
        bool fresh = true;
        double beta = 0.0;
        T* pold = z;   // beta = 0: the first direction is z
        T* pnew = pa;
        int it = 0;
        while (C.alive) {
            if (rr <= tol * tol) {
                if (fresh || !confirm) break;
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
            const SrcZP<DIM, T> src{z, pold, (T)beta, o};
            if (WIN && win) {
                // the direction over the window, staged once with coalesced
                // loads (the band from the neighbouring blocks' stores), then
                // the SpMV gathers from LDS
                // several values per thread and pass, their loads issued together
                // (one memory latency per pass, not per value)
                constexpr int U = DIM == 3 ? 8 : 2;
                const int64_t nwin = DIM * wn, bd = blockDim.x;
                const int L = (int)(wn / 3);     // 3D: the segment length
                for (int64_t i0 = threadIdx.x; i0 < nwin; i0 += U * bd) {
                    T val[U];
#pragma unroll
                    for (int k2 = 0; k2 < U; ++k2) {
                        const int64_t i = i0 + k2 * bd;
                        if constexpr (DIM == 3) {
                            // slot j of segment k holds node wlo + j + k (P - L); nodes
                            // outside the mesh (the first and last blocks) are never read
                            const int j = (int)(i / 3);
                            const int64_t nd = wlo + j + ((j >= L) + (j >= 2 * L)) * (int64_t)wS;
                            val[k2] = i < nwin && nd >= 0 && nd < g.nnode ? src(nd, (int)(i - 3 * j)) : T(0);
                        } else {
                            val[k2] = i < nwin ? src(wlo + i / DIM, (int)(i % DIM)) : T(0);
                        }
                    }
#pragma unroll
                    for (int k2 = 0; k2 < U; ++k2) {
                        const int64_t i = i0 + k2 * bd;
                        if (i < nwin) win[i] = val[k2];
                    }
                }
                __syncthreads();
                using SL = std::conditional_t<DIM == 3, SrcSeg3<T>, SrcLds<DIM, T>>;
                const SL sl = [&] {
                    if constexpr (DIM == 3) return SrcSeg3<T>{win, wlo, wP, wS};
                    else return SrcLds<DIM, T>{win, wlo};
                }();
                for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x) {
                    int iy, ix, iz;
                    g.coords(nd, iy, ix, iz, DIM);
                    T ap[DIM];
                    op.apply(nd, iy, ix, iz, sl, ap);
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        const int64_t i = DIM * nd + c;
                        const T pi = sl(nd, c);
                        const T qi = fm[i] ? ap[c] : T(0);
                        o.st(pnew, nd, i, pi);
                        q[i] = qi;
                        v1[0] += (double)pi * (double)qi;
                    }
                }
            } else {
                for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x) {
                    int iy, ix, iz;
                    g.coords(nd, iy, ix, iz, DIM);
                    T ap[DIM];
                    op.apply(nd, iy, ix, iz, src, ap);
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        const int64_t i = DIM * nd + c;
                        const T pi = src(nd, c);
                        const T qi = fm[i] ? ap[c] : T(0);
                        o.st(pnew, nd, i, pi);
                        q[i] = qi;
                        v1[0] += (double)pi * (double)qi;
                    }
                }
            }
            C.reduce<1>(v1);
            const double pq = C.res[0];
            if (!(pq > 0.0)) break;        // breakdown (zero or non-finite direction)
            const double alpha = rz / pq;
            // phase B: x += alpha p; r -= alpha q; z = dinv r
            double v2[2] = {0.0, 0.0};
            const T a = (T)alpha;
            for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x) {
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    const int64_t i = DIM * nd + c;
                    o.st(x, nd, i, x[i] + a * pnew[i]);
                    const T ri = r[i] - a * q[i];
                    const T zi = dinv[i] * ri;
                    r[i] = ri;
                    o.st(z, nd, i, zi);
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
        if (confirm && !fresh && C.alive) residual(b, x, false, dinv, r, z);   // report the true residual
        return it;
    }

    // The same solve with ONE grid sum per iteration (the Chronopoulos-Gear
    // arrangement of preconditioned CG; 2D, the SpMV source in the LDS
    // window).  With u = M^-1 r and w = A u, the recurrences
    //   p = u + beta p,  s = w + beta s  (s = A p),
    //   x += alpha p,    r -= alpha s,   u = M^-1 r,   w = A u,
    //   gamma = (r, u),  delta = (w, u),
    //   beta = gamma / gamma_old,  alpha = gamma / (delta - beta gamma / alpha_old)
    // give the iterates of PCG in exact arithmetic, and the three dot
    // products of an iteration (gamma, delta, |r|^2) are summed together.
    // The new u of the band nodes (owned by neighbouring blocks, which write
    // their new r and s meanwhile) is formed here from their previous r, w
    // and s, so r, w and s are double-buffered by iteration parity; the
    // operations are those of the owner, so every block sees the same u.
    //
    // Residency: thread t owns the nodes lo + t + j blockDim.x (j < J) for
    // the whole solve and keeps their coordinates, free flags, Jacobi
    // diagonal and r, w, s in registers, their x and p in LDS; the moduli of
    // the element columns around the own nodes and the band nodes' Jacobi
    // diagonal are staged in LDS once.  Only the own nodes within one band of
    // the range ends (those in a neighbour's window) publish r, w and s to
    // memory; the others never leave the CU.  x goes back to memory before
    // every true residual and at the end.  Convergence is confirmed on the
    // recomputed residual b - A x, and a failed confirmation restarts from x.
    template <int J>
    __device__ __forceinline__ int run1(const T* b, T* x, const T* dinv, T* R0, T* R1, T* W0, T* W1, T* S0, T* S1,
                                        double tol, int maxit, int& restarts) {
        const Own& o = C.o;
        const int bd = (int)blockDim.x;
        const int64_t whi = wlo + wn;
        const int nlo = (int)(2 * (o.lo - wlo)), nh = nlo + (int)(2 * (whi - o.hi));   // band values below / in total
        const int nown = (int)(2 * (o.hi - o.lo)), ohi = (int)(2 * (o.hi - wlo));
        // 32-bit value indices (the launch checks 2 nnode < 2^31)
        const uint32_t i0 = (uint32_t)(2 * o.lo), w0 = (uint32_t)(2 * wlo);
        T* const xl = own;
        T* const pl = own + nown;
        const int ny1 = g.ny + 1;
        const int64_t exl = o.lo / ny1 > 0 ? o.lo / ny1 - 1 : 0;
        const int64_t exh = (o.hi - 1) / ny1 < g.nx - 1 ? (o.hi - 1) / ny1 : g.nx - 1;
        const int64_t elo = exl * g.ny;
        const int ne = (int)((exh + 1) * g.ny - elo);
        T* const el = own + 2 * nown;
        T* const dband = el + ne;                 // filled after the first grid sum (below)
        for (int t = threadIdx.x; t < ne; t += bd) el[t] = op.E[elo + t];
        Op opl = op;
        opl.E = el;
        opl.e0 = elo;
        // per node: 2 nd, coordinates, and flags (bits 0, 1: free DOFs;
        // kPub: within one band of the range ends; kOn: an own node)
        constexpr int kPub = 4, kOn = 8;
        uint32_t gi[J];
        int iy[J], ix[J], fl[J];
        T d[J][2], r[J][2], w[J][2], s[J][2];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int64_t ndj = o.lo + threadIdx.x + (int64_t)j * bd;
            gi[j] = (uint32_t)(2 * ndj);
            iy[j] = ix[j] = fl[j] = 0;
#pragma unroll
            for (int c = 0; c < 2; ++c) d[j][c] = r[j][c] = w[j][c] = s[j][c] = T(0);
            if (ndj < o.hi) {
                int iz;
                g.coords(ndj, iy[j], ix[j], iz, 2);
                fl[j] = kOn | (o.edge(ndj) ? kPub : 0);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const uint32_t i = gi[j] + c;
                    fl[j] |= fm[i] ? 1 << c : 0;
                    d[j][c] = dinv[i];                // written by this thread (same node mapping)
                    xl[i - i0] = x[i];
                }
            }
        }
        __syncthreads();
        auto flush_x = [&]() {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (!(fl[j] & kOn)) continue;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const uint32_t i = gi[j] + c;
                    if (fl[j] & kPub) st_dev(x + i, xl[i - i0]);
                    else x[i] = xl[i - i0];
                }
            }
            C.alive = C.gb.sync() && C.alive;       // the band of x is read by the neighbours' residual
        };
        int it = 0;
        bool confirming = false, stop = false;
        while (C.alive) {
            // (re)start: r = b - A x (the true residual: it confirms the
            // previous pass's convergence, or is the one reported after a
            // breakdown or a spent budget), then u, w = A u
            {
                double v[2] = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    int f = fl[j], yy = iy[j], xx = ix[j];
                    uint32_t gg = gi[j];
                    opaque(f, yy, xx, gg);
                    if (!(f & kOn)) continue;
                    T ax[2];
                    opl.apply((int64_t)(gg >> 1), yy, xx, 0, Src1<2, T>{x, o}, ax);
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const uint32_t i = gg + c;
                        const T ri = (f >> c) & 1 ? b[i] - ax[c] : T(0);
                        r[j][c] = ri;
                        if (f & kPub) st_dev(R0 + i, ri);
                        v[0] += (double)ri * (double)(d[j][c] * ri);
                        v[1] += (double)ri * (double)ri;
                    }
                }
                C.reduce<2>(v);
            }
            double rr = C.res[1];
            if (rr <= tol * tol || !C.alive || stop) break;   // a fresh residual needs no confirmation
            if (confirming) ++restarts;                        // the recursive residual had met tol
            // the band's Jacobi diagonal, written by the neighbouring blocks
            // before the grid sum just taken (band nodes are never this
            // block's own); each value is read back by the thread that wrote it
            for (int t = threadIdx.x; t < nh; t += bd) {
                const int j = t < nlo ? t : t - nlo + ohi;
                dband[t] = ld_dev(dinv + w0 + j);
            }
            {
#pragma unroll
                for (int j = 0; j < J; ++j)
                    if (fl[j] & kOn)
#pragma unroll
                        for (int c = 0; c < 2; ++c) win[gi[j] + c - w0] = d[j][c] * r[j][c];
                for (int t = threadIdx.x; t < nh; t += bd) {
                    const int j = t < nlo ? t : t - nlo + ohi;
                    win[j] = dband[t] * ld_dev(R0 + w0 + j);
                }
                __syncthreads();
                const SrcLds<2, T> sl{win, wlo};
                double v[2] = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    int f = fl[j], yy = iy[j], xx = ix[j];
                    uint32_t gg = gi[j];
                    opaque(f, yy, xx, gg);
                    if (!(f & kOn)) continue;
                    T aw[2];
                    opl.apply((int64_t)(gg >> 1), yy, xx, 0, sl, aw);
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const T ui = d[j][c] * r[j][c], wi = (f >> c) & 1 ? aw[c] : T(0);
                        w[j][c] = wi;
                        if (f & kPub) st_dev(W0 + gg + c, wi);
                        v[0] += (double)r[j][c] * (double)ui;
                        v[1] += (double)wi * (double)ui;
                    }
                }
                C.reduce<2>(v);
            }
            double gamma = C.res[0], delta = C.res[1], gamma_old = 1.0, alpha_old = 1.0;
            int k = 0;
            bool ok = true;
            while (C.alive && rr > tol * tol && it < maxit) {
                double beta = 0.0, alpha;
                if (k == 0) {
                    alpha = gamma / delta;
                } else {
                    beta = gamma / gamma_old;
                    alpha = gamma / (delta - beta * gamma / alpha_old);
                }
                if (!(alpha > 0.0) || !(alpha < INFINITY)) { ok = false; break; }   // breakdown
                const bool odd = k & 1;
                const T* Rk = odd ? R1 : R0;
                T* Rn = odd ? R0 : R1;
                const T* Wk = odd ? W1 : W0;
                T* Wn = odd ? W0 : W1;
                T* Sk = odd ? S1 : S0;
                const T* So = odd ? S0 : S1;
                const T a = (T)alpha, bt = (T)beta;
                double v[3] = {0.0, 0.0, 0.0};        // gamma, delta, |r|^2
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    int f = fl[j], yy = iy[j], xx = ix[j];
                    uint32_t gg = gi[j];
                    opaque(f, yy, xx, gg);
                    if (!(f & kOn)) continue;
                    const uint32_t l = gg - i0;
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const T ui = d[j][c] * r[j][c];
                        const T pi = k == 0 ? ui : fma(bt, pl[l + c], ui);
                        const T si = k == 0 ? w[j][c] : fma(bt, s[j][c], w[j][c]);
                        const T rn = fma(-a, si, r[j][c]);
                        const T un = d[j][c] * rn;
                        pl[l + c] = pi;
                        xl[l + c] = fma(a, pi, xl[l + c]);
                        s[j][c] = si;
                        r[j][c] = rn;
                        if (f & kPub) {
                            st_dev(Sk + gg + c, si);
                            st_dev(Rn + gg + c, rn);
                        }
                        win[gg + c - w0] = un;
                        v[0] += (double)rn * (double)un;
                        v[2] += (double)rn * (double)rn;
                    }
                }
                // the band: a thread's loads (up to UB values) are all issued
                // before the first is used, one memory latency per pass
                constexpr int UB = 4;
                for (int t0 = threadIdx.x; t0 < nh; t0 += UB * bd) {
                    T rk[UB], wk[UB], so[UB];
#pragma unroll
                    for (int ub = 0; ub < UB; ++ub) {
                        const int t = t0 + ub * bd;
                        rk[ub] = wk[ub] = so[ub] = T(0);
                        if (t < nh) {
                            const uint32_t i = w0 + (uint32_t)(t < nlo ? t : t - nlo + ohi);
                            rk[ub] = ld_dev(Rk + i);
                            wk[ub] = ld_dev(Wk + i);
                            if (k > 0) so[ub] = ld_dev(So + i);
                        }
                    }
#pragma unroll
                    for (int ub = 0; ub < UB; ++ub) {
                        const int t = t0 + ub * bd;
                        if (t < nh) {
                            const T si = k == 0 ? wk[ub] : fma(bt, so[ub], wk[ub]);
                            win[t < nlo ? t : t - nlo + ohi] = dband[t] * fma(-a, si, rk[ub]);
                        }
                    }
                }
                __syncthreads();
                const SrcLds<2, T> sl{win, wlo};
                // the first and last node slots hold the band nodes, whose w
                // is stored for the neighbours: those go first, so that their
                // stores complete while the other nodes are computed
#pragma unroll
                for (int jj = 0; jj < J; ++jj) {
                    const int j = jj == 0 ? 0 : J - jj;
                    int f = fl[j], yy = iy[j], xx = ix[j];
                    uint32_t gg = gi[j];
                    opaque(f, yy, xx, gg);
                    if (!(f & kOn)) continue;
                    T aw[2];
                    opl.apply((int64_t)(gg >> 1), yy, xx, 0, sl, aw);
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const T wi = (f >> c) & 1 ? aw[c] : T(0);
                        w[j][c] = wi;
                        if (f & kPub) st_dev(Wn + gg + c, wi);
                        v[1] += (double)wi * (double)(d[j][c] * r[j][c]);
                    }
                }
                C.reduce<3>(v);
                gamma_old = gamma;
                alpha_old = alpha;
                gamma = C.res[0];
                delta = C.res[1];
                rr = C.res[2];
                ++k;
                ++it;
            }
            if (!C.alive) break;
            flush_x();
            confirming = ok && rr <= tol * tol;
            stop = !confirming;                                // breakdown or budget spent
        }
        return it;
    }

    // Pipelined PCG (the arrangement of Ghysels and Vanroose, 2014) of the
    // single-sum iteration above, with the same on-chip residency.  With
    // u = M^-1 r, w = A u, m = M^-1 w, n = A m and the extra recurrence
    // z = n + beta z (z = A M^-1 s):
    //   s = w + beta s,  p = u + beta p,  x += alpha p,  r -= alpha s,
    //   w -= alpha z,    u = M^-1 r,
    // the SpMV of an iteration (n = A m) no longer comes before its grid sum:
    // a block publishes its partial gamma = (r, u), delta = (w, u) and |r|^2,
    // applies A to m while the sums travel, and collects them afterwards.
    // The SpMV needs the neighbours' new w on the band, so a block first
    // waits only for the blocks whose nodes its window holds: their records
    // of the same grid sum, written after their band stores completed.  At
    // SIMP's stiffness contrast the recurrences for w, s and z drift from
    // A u, A p and A M^-1 s; every kPipeReplace iterations, and to confirm
    // convergence, r = b - A x, w, s and z are recomputed (four SpMVs with
    // their band exchanges), which keeps the iteration count that of PCG.
    // The w of the band nodes goes through memory double-buffered by the
    // parity of its publication (a block cannot publish twice more before
    // every reader has loaded it: that needs the readers' next grid sums).
    template <int J>
    __device__ __forceinline__ int run_pipe(const T* b, T* x, const T* dinv, T* WB0, T* WB1, T* EX0, T* EX1,
                                            double tol, int maxit, int& restarts, bool& handover) {
        const Own& o = C.o;
        const int bd = (int)blockDim.x;
        const int64_t whi = wlo + wn;
        const int nlo = (int)(2 * (o.lo - wlo)), nh = nlo + (int)(2 * (whi - o.hi));
        const int nown = (int)(2 * (o.hi - o.lo)), ohi = (int)(2 * (o.hi - wlo));
        const uint32_t i0 = (uint32_t)(2 * o.lo), w0 = (uint32_t)(2 * wlo);
        T* const xl = own;
        T* const pl = own + nown;
        const int ny1 = g.ny + 1;
        const int64_t exl = o.lo / ny1 > 0 ? o.lo / ny1 - 1 : 0;
        const int64_t exh = (o.hi - 1) / ny1 < g.nx - 1 ? (o.hi - 1) / ny1 : g.nx - 1;
        const int64_t elo = exl * g.ny;
        const int ne = (int)((exh + 1) * g.ny - elo);
        T* const el = own + 2 * nown;
        T* const dband = el + ne;
        for (int t = threadIdx.x; t < ne; t += bd) el[t] = op.E[elo + t];
        Op opl = op;
        opl.E = el;
        opl.e0 = elo;
        // the blocks whose nodes the window's bands hold (ranges of `chunk`
        // nodes, as the kernel deals them)
        const int64_t chunk = (g.nnode + C.fr.nblk - 1) / C.fr.nblk;
        const int nb_lo0 = (int)(wlo / chunk), nb_lo1 = o.lo > wlo ? (int)((o.lo - 1) / chunk) : -1;
        const int nb_hi0 = (int)(o.hi / chunk), nb_hi1 = whi > o.hi ? (int)((whi - 1) / chunk) : -1;
        const int n_lo = nb_lo1 >= nb_lo0 ? nb_lo1 - nb_lo0 + 1 : 0;
        const int n_nb = n_lo + (nb_hi1 >= nb_hi0 ? nb_hi1 - nb_hi0 + 1 : 0);
        constexpr int kPub = 4, kOn = 8;
        uint32_t gi[J];
        int iy[J], ix[J], fl[J];
        T d[J][2], r[J][2], w[J][2], s[J][2], z[J][2], nv[J][2];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int64_t ndj = o.lo + threadIdx.x + (int64_t)j * bd;
            gi[j] = (uint32_t)(2 * ndj);
            iy[j] = ix[j] = fl[j] = 0;
#pragma unroll
            for (int c = 0; c < 2; ++c) d[j][c] = r[j][c] = w[j][c] = s[j][c] = z[j][c] = nv[j][c] = T(0);
            if (ndj < o.hi) {
                int iz;
                g.coords(ndj, iy[j], ix[j], iz, 2);
                fl[j] = kOn | (o.edge(ndj) ? kPub : 0);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const uint32_t i = gi[j] + c;
                    fl[j] |= fm[i] ? 1 << c : 0;
                    d[j][c] = dinv[i];                // written by this thread (same node mapping)
                    xl[i - i0] = x[i];
                    pl[i - i0] = T(0);
                }
            }
        }
        __syncthreads();
        const SrcLds<2, T> sl{win, wlo};
        // the own values of a vector into the window (after the block's
        // previous SpMV: callers place a barrier before)
        auto own_to_window = [&](auto&& val) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                int f = fl[j], yy = 0, xx = 0;
                uint32_t gg = gi[j];
                opaque(f, yy, xx, gg);
                if (f & kOn)
#pragma unroll
                    for (int c = 0; c < 2; ++c) win[gg + c - w0] = val(j, c);
            }
        };
        auto publish_band = [&](T* buf, auto&& val) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                int f = fl[j], yy = 0, xx = 0;
                uint32_t gg = gi[j];
                opaque(f, yy, xx, gg);
                if (f & kPub)
#pragma unroll
                    for (int c = 0; c < 2; ++c) st_dev(buf + gg + c, val(j, c));
            }
        };
        // the band of the window from the neighbours' published values,
        // times their Jacobi diagonal when `scaled`; a thread's loads (UB per
        // pass) are issued together
        auto band_to_window = [&](const T* buf, bool scaled) {
            constexpr int UB = 4;
            for (int t0 = threadIdx.x; t0 < nh; t0 += UB * bd) {
                T bv[UB];
#pragma unroll
                for (int ub = 0; ub < UB; ++ub) {
                    const int t = t0 + ub * bd;
                    bv[ub] = T(0);
                    if (t < nh) bv[ub] = ld_dev(buf + w0 + (uint32_t)(t < nlo ? t : t - nlo + ohi));
                }
#pragma unroll
                for (int ub = 0; ub < UB; ++ub) {
                    const int t = t0 + ub * bd;
                    if (t < nh) win[t < nlo ? t : t - nlo + ohi] = scaled ? dband[t] * bv[ub] : bv[ub];
                }
            }
        };
        // out = A (window) on the own free DOFs; the band node slots first
        auto spmv = [&](T (&out)[J][2]) {
#pragma unroll
            for (int jj = 0; jj < J; ++jj) {
                const int j = jj == 0 ? 0 : J - jj;
                int f = fl[j], yy = iy[j], xx = ix[j];
                uint32_t gg = gi[j];
                opaque(f, yy, xx, gg);
                if (!(f & kOn)) continue;
                T a2[2];
                opl.apply((int64_t)(gg >> 1), yy, xx, 0, sl, a2);
#pragma unroll
                for (int c = 0; c < 2; ++c) out[j][c] = (f >> c) & 1 ? a2[c] : T(0);
            }
        };
        // the same on the nodes within one band of the range ends (near) or
        // on the others, whose stencils stay within the own range (!near)
        auto spmv_part = [&](T (&out)[J][2], bool near) {
#pragma unroll
            for (int jj = 0; jj < J; ++jj) {
                const int j = jj == 0 ? 0 : J - jj;
                int f = fl[j], yy = iy[j], xx = ix[j];
                uint32_t gg = gi[j];
                opaque(f, yy, xx, gg);
                if (!(f & kOn) || ((f & kPub) != 0) != near) continue;
                T a2[2];
                opl.apply((int64_t)(gg >> 1), yy, xx, 0, sl, a2);
#pragma unroll
                for (int c = 0; c < 2; ++c) out[j][c] = (f >> c) & 1 ? a2[c] : T(0);
            }
        };
        // one exchange and SpMV: out = A (M^-1 raw) when scaled, else A raw;
        // the band nodes' raw values go through buf
        auto exchange_spmv = [&](auto&& raw, T* buf, bool scaled, T (&out)[J][2]) {
            __syncthreads();                        // the previous SpMV's window reads are done
            own_to_window([&](int j, int c) { return scaled ? d[j][c] * raw(j, c) : raw(j, c); });
            publish_band(buf, raw);
            C.alive = C.gb.sync() && C.alive;       // the neighbours' band stores are complete
            band_to_window(buf, scaled);
            __syncthreads();
            spmv(out);
        };
        // r = b - A x, w = A M^-1 r, s = A p and z = A M^-1 s recomputed from
        // x and p (x and p through the window like the other sources)
        auto replace_all = [&]() {
            exchange_spmv([&](int j, int c) { return xl[gi[j] + c - i0]; }, EX0, false, nv);
#pragma unroll
            for (int j = 0; j < J; ++j) {
                int f = fl[j], yy = 0, xx = 0;
                uint32_t gg = gi[j];
                opaque(f, yy, xx, gg);
                if (f & kOn)
#pragma unroll
                    for (int c = 0; c < 2; ++c) r[j][c] = (f >> c) & 1 ? b[gg + c] - nv[j][c] : T(0);
            }
            exchange_spmv([&](int j, int c) { return r[j][c]; }, EX1, true, w);
            exchange_spmv([&](int j, int c) { return pl[gi[j] + c - i0]; }, EX0, false, s);
            exchange_spmv([&](int j, int c) { return s[j][c]; }, EX1, true, z);
        };
        auto partials = [&](double (&v)[3]) {
            v[0] = v[1] = v[2] = 0.0;
#pragma unroll
            for (int j = 0; j < J; ++j)
                if (fl[j] & kOn)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const T ui = d[j][c] * r[j][c];
                        v[0] += (double)r[j][c] * (double)ui;
                        v[1] += (double)w[j][c] * (double)ui;
                        v[2] += (double)r[j][c] * (double)r[j][c];
                    }
        };
        int it = 0, since = 0, pub = 0;
        bool fresh = false, stop = false, confirming = false, replace = true;
        double gamma_old = 1.0, alpha_old = 1.0, beta = 0.0, alpha = 0.0;
        // the smallest true residual so far; its x is kept in memory (x)
        double rr_best = INFINITY;
        handover = false;
        double v[3];
        // the band's Jacobi diagonal, written by the neighbouring blocks
        // before this barrier (each value read back by the thread that loads it)
        C.alive = C.gb.sync() && C.alive;
        for (int t = threadIdx.x; t < nh; t += bd) dband[t] = ld_dev(dinv + w0 + (uint32_t)(t < nlo ? t : t - nlo + ohi));
        while (C.alive) {
            if (replace) {
                // the recurrences' vectors recomputed (the true residual: it
                // confirms convergence, or is the one a spent budget or a
                // breakdown reports); p = s = z = 0 at the start
                replace_all();
                replace = false;
                fresh = true;
                since = 0;
            } else {
                const T a = (T)alpha, bt = (T)beta;
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    int f = fl[j], yy = 0, xx = 0;
                    uint32_t gg = gi[j];
                    opaque(f, yy, xx, gg);
                    if (!(f & kOn)) continue;
                    const uint32_t l = gg - i0;
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const T ui = d[j][c] * r[j][c];
                        z[j][c] = fma(bt, z[j][c], nv[j][c]);
                        s[j][c] = fma(bt, s[j][c], w[j][c]);
                        const T pi = fma(bt, pl[l + c], ui);
                        pl[l + c] = pi;
                        xl[l + c] = fma(a, pi, xl[l + c]);
                        r[j][c] = fma(-a, s[j][c], r[j][c]);
                        w[j][c] = fma(-a, z[j][c], w[j][c]);
                    }
                }
                fresh = false;
                ++it;
                ++since;
            }
            partials(v);
            publish_band(pub & 1 ? WB1 : WB0, [&](int j, int c) { return w[j][c]; });
            // m = M^-1 w into the window (own part), the partial sums out
            __syncthreads();
            own_to_window([&](int j, int c) { return d[j][c] * w[j][c]; });
            C.fr.template publish<3>(v);
            // n = A m while the sums travel: first on the nodes whose
            // stencils stay within the own range (the window's own part is
            // complete after the publication's barrier), while the
            // neighbours publish; then the band of m (wait for the blocks
            // that own it: a failed wait enters the grid sum's verdict) and
            // the nodes near the range ends
            spmv_part(nv, false);
            bool nb_ok = true;
            if ((int)threadIdx.x < n_nb) {
                const int t = threadIdx.x;
                C.fr.template wait_record<3>((unsigned)(t < n_lo ? nb_lo0 + t : nb_hi0 + t - n_lo), nb_ok);
            }
            __syncthreads();
            band_to_window(pub & 1 ? WB1 : WB0, true);
            ++pub;
            __syncthreads();
            spmv_part(nv, true);
            C.alive = C.fr.template collect<3>(C.res, nb_ok) && C.alive;
            if (!C.alive) break;
            const double gamma = C.res[0], delta = C.res[1], rr = C.res[2];
            if (fresh) {
                // near the attainable accuracy the recurrences can run away
                // (the true residual grows by orders of magnitude): hand the
                // solve over, from the best iterate, to the single-sum kernel
                if (!(rr <= 1e6 * rr_best)) { handover = true; break; }
                if (rr < rr_best) {
                    rr_best = rr;
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        if (!(fl[j] & kOn)) continue;
#pragma unroll
                        for (int c = 0; c < 2; ++c) x[gi[j] + c] = xl[gi[j] + c - i0];
                    }
                }
            }
            if (stop || (fresh && rr <= tol * tol)) break;
            if (fresh && confirming) ++restarts;        // the true residual missed tol
            confirming = rr <= tol * tol;
            if (confirming || it >= maxit || since >= kPipeReplace) {
                stop = it >= maxit;
                replace = true;
                continue;
            }
            if (it == 0) {
                beta = 0.0;
                alpha = gamma / delta;
            } else {
                beta = gamma / gamma_old;
                alpha = gamma / (delta - beta * gamma / alpha_old);
            }
            if (!(alpha > 0.0) || !(alpha < INFINITY)) {   // breakdown: hand over from the best iterate
                handover = true;
                break;
            }
            gamma_old = gamma;
            alpha_old = alpha;
        }
        // x of the own nodes back to memory (a hand-over leaves the best one)
        if (!handover)
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (!(fl[j] & kOn)) continue;
#pragma unroll
                for (int c = 0; c < 2; ++c) x[gi[j] + c] = xl[gi[j] + c - i0];
            }
        __syncthreads();
        if (threadIdx.x == 0) C.res[1] = handover ? rr_best : C.res[2];   // the caller reads |r|^2 there
        __syncthreads();
        return it;
    }
};

template <int DIM, typename T, class Op>
__device__ __forceinline__ void jacobi(const Op& op, const Geo& g, const Own& o, const uint8_t* fm, T* dinv) {
    for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x) {
        int iy, ix, iz;
        g.coords(nd, iy, ix, iz, DIM);
        T dg[DIM];
        op.diag(nd, iy, ix, iz, dg);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t i = DIM * nd + c;
            o.st(dinv, nd, i, fm[i] && dg[c] != T(0) ? T(1) / dg[c] : T(0));
        }
    }
}

// Mixed precision CG with reliable updates: the directions, the SpMV and the
// recursive residual are FP32 (FP32 operator and Jacobi), the iterate u is
// accumulated in FP64, and whenever the FP32 residual has dropped by the
// factor `drop` (opts.inner_rtol) since the last replacement, or every
// kReplaceEvery iterations, the residual is recomputed in FP64 from the FP64
// matrix-free operator, f - K64 u, and replaces the FP32 one without
// restarting the search direction.  Convergence is decided on those FP64
// residuals only.  The iterate with the smallest FP64 residual is kept (two
// buffers, swapped).  Returns false when the FP64 residual stops improving
// (three replacements without halving the best one), grows past twice the
// best, or half the iteration budget is spent; the caller then restores the
// best iterate and finishes in FP64.
constexpr int kReplaceEvery = 64;

template <int DIM, class Op32>
__device__ bool mixed_cg(Ctx& C, const Geo& g, const SolveArgs& A, const Op32& op32,
                         const MatFree<DIM, double>& mf64, double tol, int& iters, int& passes, double& rfinal,
                         double*& ubest) {
    const Own& o = C.o;
    const uint8_t* __restrict__ fm = A.freem;
    double* u = A.u;
    double* r64 = A.v64[0];
    double* cand = A.v64[6];
    float *r = A.v32[2], *z = A.v32[3], *pa = A.v32[4], *pb = A.v32[5], *q = A.v32[6], *dinv = A.v32[7];
    // FP64 residual replacement: r64 = f - K64 u, r = (float) r64, z = dinv r;
    // u is copied to the candidate buffer in the same sweep
    auto replace = [&](double& rz, double& rr64) {
        double v[2] = {0.0, 0.0};
        for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x) {
            int iy, ix, iz;
            g.coords(nd, iy, ix, iz, DIM);
            double ax[DIM];
            mf64.apply(nd, iy, ix, iz, Src1<DIM, double>{u, o}, ax);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const int64_t i = DIM * nd + c;
                cand[i] = u[i];                 // own range only
                const double ri = fm[i] ? A.f[i] - ax[c] : 0.0;
                r64[i] = ri;
                const float rf = (float)ri, zf = dinv[i] * rf;
                r[i] = rf;
                o.st(z, nd, i, zf);
                v[0] += (double)rf * (double)zf;
                v[1] += ri * ri;
            }
        }
        C.reduce<2>(v);
        rz = C.res[0];
        rr64 = C.res[1];
    };
    double rz, rr64;
    replace(rz, rr64);
    double rbest = sqrt(rr64), rlast = rbest;
    ubest = cand;
    cand = A.v64[7];
    rfinal = rbest;
    if (rbest <= tol) return true;
    const int budget = iters + A.maxit / 2;
    int stall = 0, since = 0;
    double beta = 0.0;
    float* pold = z;
    float* pnew = pa;
    const double drop = A.inner_rtol;
    while (C.alive && iters < budget) {
        double v1[1] = {0.0};
        const SrcZP<DIM, float> src{z, pold, (float)beta, o};
        for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x) {
            int iy, ix, iz;
            g.coords(nd, iy, ix, iz, DIM);
            float ap[DIM];
            op32.apply(nd, iy, ix, iz, src, ap);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const int64_t i = DIM * nd + c;
                const float pi = src(nd, c);
                const float qi = fm[i] ? ap[c] : 0.0f;
                o.st(pnew, nd, i, pi);
                q[i] = qi;
                v1[0] += (double)pi * (double)qi;
            }
        }
        C.reduce<1>(v1);
        const double pq = C.res[0];
        if (!(pq > 0.0)) return false;
        const double alpha = rz / pq;
        const float af = (float)alpha;
        double v2[2] = {0.0, 0.0};
        for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const int64_t i = DIM * nd + c;
                o.st(u, nd, i, u[i] + alpha * (double)pnew[i]);
                const float ri = r[i] - af * q[i];
                const float zi = dinv[i] * ri;
                r[i] = ri;
                o.st(z, nd, i, zi);
                v2[0] += (double)ri * (double)zi;
                v2[1] += (double)ri * (double)ri;
            }
        }
        C.reduce<2>(v2);
        ++iters;
        ++since;
        double rz_new = C.res[0];
        const double rn32 = sqrt(C.res[1]);
        if (rn32 <= drop * rlast || rn32 <= tol || since >= kReplaceEvery) {
            double rr;
            replace(rz_new, rr);
            ++passes;
            since = 0;
            const double rt = sqrt(rr);
            rfinal = rt;
            if (rt <= tol) { ubest = cand; return true; }
            if (rt < rbest) {
                stall = rt > 0.5 * rbest ? stall + 1 : 0;
                rbest = rt;
                double* t = ubest;
                ubest = cand;
                cand = t;
            } else {
                ++stall;
            }
            if (stall >= 3 || rt > 2.0 * rbest || !(rt == rt)) return false;
            rlast = rt;
        }
        beta = rz_new / rz;
        rz = rz_new;
        float* t = pnew == pa ? pb : pa;
        pold = pnew;
        pnew = t;
    }
    return false;
}

// MODE 0: FP64, assembled operator; 1: FP64, matrix-free;
//      2: mixed, FP32 assembled inner; 3: mixed, FP32 matrix-free inner;
//      kModeWindow: 2D FP64 matrix-free with the SpMV source in an LDS window
//      and one grid sum per iteration (Pcg::run1), the own nodes' vectors
//      held on chip (at most kRegNodes nodes per thread).
constexpr int kModeWindow = 4;
constexpr int kRegNodes = 4;
// kModePipe: the same residency with the pipelined iteration (Pcg::run_pipe).
constexpr int kModePipe = 7;
// kModeFallback: the FP64 PCG that finishes a mixed-precision solve which
// stalled (its own launch after the mixed kernel, so the two solvers do not
// share one kernel's registers); it returns at once when the mixed solve
// converged.
constexpr int kModeFallback = 5;
// kModeWindow3: 3D FP64 matrix-free with the SpMV source in an LDS window
// (the two-sum iteration of Pcg::run; 512-thread blocks, one per CU).
constexpr int kModeWindow3 = 6;
template <int DIM, int MODE>
__device__ __forceinline__ void solve_body(const SolveArgs& A, int bid, int nb) {
    if (MODE == kModeFallback && !(A.st->fallback == 1 && A.st->converged == 0)) return;   // uniform over the grid
    if (MODE == kModeWindow && A.follow && !(A.st->fallback == 1 && A.st->converged == 0)) return;
    const to_solve_stats prev_st = MODE == kModeWindow && A.follow ? *A.st : to_solve_stats{};
    __shared__ double sh[16];
    __shared__ double res[4];
    Ctx C{A.partial, GridBar{}, sh, res, 0, true, Own{}, FlagReduce{}};
    C.gb.init(A.bar, bid, nb);
    C.fr.init(A.ll, A.bar, bid, nb);
    {
        // contiguous node range of this block; band = largest node-index
        // distance between two nodes of one element
        const int64_t nn = A.geo.nnode;
        const int64_t chunk = (nn + nb - 1) / nb;
        C.o.lo = min(nn, (int64_t)bid * chunk);
        C.o.hi = min(nn, C.o.lo + chunk);
        C.o.band = DIM == 2 ? (int64_t)A.geo.ny + 2
                            : (int64_t)(A.geo.ny + 1) * (A.geo.nz + 1) + A.geo.ny + 2;
    }
    const Own& o = C.o;
    const Geo& g = A.geo;
    const int64_t n = g.nnode * DIM;
    double* u = A.u;

    if constexpr (MODE == kModeFallback) {
        // FP64 PCG from the restored iterate, with the mixed solve's Jacobi
        // diagonal, norm and remaining budget
        const to_solve_stats prev = *A.st;
        const double tol = A.rtol * prev.bnorm;
        MatFree<DIM, double> mf64{A.E64, A.kf64, A.geo.nx, A.geo.ny, A.geo.nz};
        Pcg<DIM, double, MatFree<DIM, double>> cg64{mf64, A.geo, A.freem, C};
        int restarts = prev.restarts;
        const int left = A.maxit - prev.iterations;
        const int it = cg64.run(A.f, A.u, false, A.v64[5], A.v64[0], A.v64[1], A.v64[2], A.v64[3], A.v64[4], tol,
                                left > 0 ? left : 0, restarts);
        const double resid = sqrt(C.res[1]) / (prev.bnorm > 0 ? prev.bnorm : 1.0);
        C.fr.finish();
        if (bid == 0 && threadIdx.x == 0) {
            to_solve_stats st2 = prev;
            st2.residual = resid;
            st2.iterations = prev.iterations + it;
            st2.converged = (resid <= A.rtol && C.alive) ? 1 : 0;
            st2.restarts = restarts;
            st2.pad = C.alive ? 0 : 1;
            *A.st = st2;
        }
        return;
    }
    // |f_free|, and u = 0 on fixed DOFs (or everywhere when asked)
    {
        double v[1] = {0.0};
        for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x)
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const int64_t i = DIM * nd + c;
                const bool fr = A.freem[i] != 0;
                if (!fr || (A.zero_x0 && !A.follow)) o.st(u, nd, i, 0.0);
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
    if (MODE <= 1 || MODE == kModeWindow || MODE == kModeWindow3 || MODE == kModePipe) {
        double *r = A.v64[0], *z = A.v64[1], *pa = A.v64[2], *pb = A.v64[3], *q = A.v64[4], *dinv = A.v64[5];
        if (MODE == 0) {
            CsrS<DIM, double> op{A.rp, (const double*)A.kval, g.nx, g.ny, g.nz};
            jacobi<DIM, double>(op, g, C.o, A.freem, dinv);
            Pcg<DIM, double, CsrS<DIM, double>> cg{op, g, A.freem, C};
            iters = cg.run(A.f, u, false, dinv, r, z, pa, pb, q, tol, A.maxit, restarts);
        } else {
            if (A.kdiag32 || A.kdiag64) {   // Jacobi from the assembled diagonal (last entry of each row)
                for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x)
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        const int64_t i = DIM * nd + c;
                        const int64_t k = A.rp[i + 1] - 1;
                        const double dg = A.kdiag64 ? A.kdiag64[k] : (double)A.kdiag32[k];
                        o.st(dinv, nd, i, A.freem[i] && dg != 0.0 ? 1.0 / dg : 0.0);
                    }
            } else {
                jacobi<DIM, double>(mf64, g, C.o, A.freem, dinv);
            }
            Pcg<DIM, double, MatFree<DIM, double>> cg{mf64, g, A.freem, C};
            if (DIM == 3 && A.stage > 0) {
                extern __shared__ double solve_win[];
                const int64_t P = ((int64_t)g.ny + 1) * (g.nz + 1), L = o.hi - o.lo + 2 * ((int64_t)g.ny + 2);
                cg.wlo = o.lo - (g.ny + 2) - P;
                cg.wn = 3 * L;
                cg.wP = (int)P;
                cg.wS = (int)(P - L);
                if (cg.wn <= A.stage) cg.win = solve_win;   // else (never, by the launch's sizing) gather
            } else if (A.stage > 0) {
                extern __shared__ double solve_win[];
                cg.wlo = o.lo - o.band > 0 ? o.lo - o.band : 0;
                const int64_t whi = o.hi + o.band < g.nnode ? o.hi + o.band : g.nnode;
                cg.wn = whi - cg.wlo;
                if (cg.wn <= A.stage) {                      // else (never, by the launch's sizing) gather
                    cg.win = solve_win;
                    if (DIM == 2 && A.stage_own > 0 && o.hi - o.lo <= A.stage_own)
                        cg.own = solve_win + 2 * (int64_t)A.stage;
                }
            }
            if constexpr (DIM == 2 && MODE == kModePipe) {
                bool handover = false;
                if (cg.win && cg.own && o.hi - o.lo <= (int64_t)kRegNodes * blockDim.x)
                    iters = cg.template run_pipe<kRegNodes>(A.f, u, dinv, r, z, pb, q, tol, A.maxit, restarts, handover);
                else C.alive = false;      // the launch sizes the LDS; a kernel without it reports failure
                fallback = handover ? 1 : 0;
            } else if constexpr (DIM == 2 && MODE == kModeWindow) {
                // as the follow-up of a pipelined solve: the remaining budget
                const int left = A.follow ? A.maxit - prev_st.iterations : A.maxit;
                if (cg.win && cg.own && o.hi - o.lo <= (int64_t)kRegNodes * blockDim.x)
                    iters = cg.template run1<kRegNodes>(A.f, u, dinv, r, z, pb, q, A.v64[6], A.v64[7], tol,
                                                        left > 0 ? left : 0, restarts);
                else C.alive = false;      // the launch sizes the LDS; a kernel without it reports failure
                if (A.follow) {
                    iters += prev_st.iterations;
                    restarts += prev_st.restarts;
                    fallback = 1;
                }
            } else if constexpr (DIM == 3 && MODE == 1) {
                // the gather kernel (the window kernel is kModeWindow3): no LDS path compiled in
                iters = cg.template run<false>(A.f, u, false, dinv, r, z, pa, pb, q, tol, A.maxit, restarts);
            } else {
                iters = cg.run(A.f, u, false, dinv, r, z, pa, pb, q, tol, A.maxit, restarts);
            }
        }
        resid = sqrt(C.res[1]) / (bnorm > 0 ? bnorm : 1.0);
    } else {
        double *r64 = A.v64[0], *z64 = A.v64[1], *pa64 = A.v64[2], *pb64 = A.v64[3], *q64 = A.v64[4];
        double* dinv64 = A.v64[5];
        CsrS<DIM, float> csr32{A.rp, (const float*)A.kval, g.nx, g.ny, g.nz};
        MatFree<DIM, float> mf32{A.E32, A.kf32, g.nx, g.ny, g.nz};
        jacobi<DIM, double>(mf64, g, C.o, A.freem, dinv64);   // for the fallback
        bool converged = false;
        double* ubest = A.v64[6];
        if (MODE == 2) {
            jacobi<DIM, float>(csr32, g, C.o, A.freem, A.v32[7]);
            converged = mixed_cg<DIM>(C, g, A, csr32, mf64, tol, iters, outer, resid, ubest);
        } else {
            jacobi<DIM, float>(mf32, g, C.o, A.freem, A.v32[7]);
            converged = mixed_cg<DIM>(C, g, A, mf32, mf64, tol, iters, outer, resid, ubest);
        }
        if (!converged && C.alive) {
            // the iterate with the smallest FP64 residual goes back into u;
            // the FP64 PCG of the next launch (kModeFallback) finishes from it
            fallback = 1;
            for (int64_t nd = o.lo + threadIdx.x; nd < o.hi; nd += (int64_t)blockDim.x)
#pragma unroll
                for (int c = 0; c < DIM; ++c) o.st(u, nd, DIM * nd + c, ubest[DIM * nd + c]);
        }
        resid /= (bnorm > 0 ? bnorm : 1.0);
    }
    C.fr.finish();
    if (bid == 0 && threadIdx.x == 0) {
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

// Threads per block of the persistent solve: 2D FP64 kernels fit in 128
// registers, so a block of 16 waves (one block per CU) hides the gather
// latency without adding blocks to every grid reduction; the others use 4.
constexpr int solve_block(int dim, int mode) {
    return dim == 2 && mode <= 1 ? 1024 : mode == 4 || mode == 6 || mode == 7 ? 512 : 256;
}
static_assert(solve_block(2, kModeFallback) == solve_block(2, 3) && solve_block(3, kModeFallback) == solve_block(3, 3),
              "a batch launches the fallback kernel with the mixed kernel's grid");
constexpr size_t kSolveLdsBytes = 158 * 1024;     // dynamic LDS of the windowed kernel (one block per CU)
constexpr bool kSolveWindow3 = true;              // the 3D windowed kernel where its window fits
constexpr bool kSolvePipe = true;                 // 2D on-chip kernel: the pipelined iteration

template <int DIM, int MODE>
__global__ __launch_bounds__(solve_block(DIM, MODE)) void solve_kernel(SolveArgs A) {
    solve_body<DIM, MODE>(A, blockIdx.x, gridDim.x);
}

// A batch of systems in one launch (block b: system inst[b], block b - first[inst] of count[inst]).
template <int DIM, int MODE>
__global__ __launch_bounds__(solve_block(DIM, MODE)) void solve_batch_kernel(const SolveArgs* __restrict__ tab,
                                                             const int32_t* __restrict__ inst,
                                                             const int32_t* __restrict__ first,
                                                             const int32_t* __restrict__ count) {
    const int i = inst[blockIdx.x];
    solve_body<DIM, MODE>(tab[i], (int)blockIdx.x - first[i], count[i]);
}

template <int DIM, int MODE>
static to_status launch_solve_t(Plan* p, SolveArgs& A, int req_blocks, hipStream_t s) {
    auto k = solve_kernel<DIM, MODE>;
    constexpr int SB = solve_block(DIM, MODE);
    int maxb = coop_blocks_for((const void*)k, SB, 0, p->num_cu);
    int64_t want = (A.geo.nnode + SB - 1) / SB;
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(maxb, p->num_cu), want));
    if (req_blocks > 0) blocks = std::min(req_blocks, maxb);
    blocks = std::min(blocks, kMaxCoopBlocks);
    A.stage = 0;
    A.stage_own = 0;
    A.stage_e = 0;
    A.follow = 0;
    if constexpr (DIM == 2 && MODE == 1) {
        // 2D matrix-free FP64: when the block's window (own nodes and the band
        // on either side) fits in LDS beside one block per CU, the kernel
        // with the window and one grid sum per iteration
        auto kw = kSolvePipe ? solve_kernel<2, kModePipe> : solve_kernel<2, kModeWindow>;
        const int64_t chunk = (A.geo.nnode + blocks - 1) / blocks;
        const int64_t wn = std::min<int64_t>(A.geo.nnode, chunk + 2 * ((int64_t)A.geo.ny + 2));
        const size_t win_bytes = (size_t)wn * 2 * sizeof(double);
        // x, p of the own nodes; the moduli of the element columns they touch
        // (at most chunk / (ny + 1) + 3 columns); the Jacobi diagonal of the
        // two bands
        const int64_t ecap = (int64_t)A.geo.ny * (chunk / ((int64_t)A.geo.ny + 1) + 3);
        const size_t own_bytes = (size_t)chunk * 4 * sizeof(double) + (size_t)ecap * sizeof(double) +
                                 (size_t)4 * ((size_t)A.geo.ny + 2) * sizeof(double);
        constexpr int SBW = solve_block(2, kModeWindow);
        auto fits = [&](size_t b) {
            return b <= kSolveLdsBytes && coop_blocks_for((const void*)kw, SBW, b, p->num_cu) >= blocks;
        };
        // the kernel keeps up to kRegNodes own nodes per thread on chip and
        // indexes vectors with 32-bit offsets
        if (chunk <= (int64_t)kRegNodes * SBW && 2 * A.geo.nnode < ((int64_t)1 << 31) &&
            fits(win_bytes + own_bytes)) {
            A.stage = (int)wn;
            A.stage_own = (int)chunk;
            A.stage_e = (int)ecap;
            void* args[] = {&A};
            TO_HIP(hipLaunchCooperativeKernel((const void*)kw, dim3(blocks), dim3(SBW), args, win_bytes + own_bytes, s));
            if (kSolvePipe) {
                // the single-sum kernel continues a pipelined solve that handed
                // over (it returns at once otherwise)
                A.follow = 1;
                TO_HIP(hipLaunchCooperativeKernel((const void*)solve_kernel<2, kModeWindow>, dim3(blocks), dim3(SBW), args,
                                                  win_bytes + own_bytes, s));
                A.follow = 0;
            }
            return TO_OK;
        }
        if (win_bytes <= kSolveLdsBytes && coop_blocks_for((const void*)k, SB, win_bytes, p->num_cu) >= blocks) {
            // the window alone: the two-sum iteration with the SpMV from LDS
            A.stage = (int)wn;
            void* args[] = {&A};
            TO_HIP(hipLaunchCooperativeKernel((const void*)k, dim3(blocks), dim3(SB), args, win_bytes, s));
            return TO_OK;
        }
    }
    if constexpr (DIM == 3 && MODE == 1) {
        // 3D matrix-free FP64: one 512-thread block per CU with the window of
        // the SpMV source in LDS, when it fits: the three segments of the own
        // range widened by ny + 2 nodes, in the planes ix - 1, ix, ix + 1
        auto kw = solve_kernel<3, kModeWindow3>;
        constexpr int SBW = solve_block(3, kModeWindow3);
        const int bw = req_blocks > 0 ? std::min(req_blocks, p->num_cu) : p->num_cu;
        const int64_t plane = ((int64_t)A.geo.ny + 1) * ((int64_t)A.geo.nz + 1);
        const int64_t chunk = (A.geo.nnode + bw - 1) / bw;
        const int64_t wn = 3 * (chunk + 2 * ((int64_t)A.geo.ny + 2));
        const size_t bytes = (size_t)wn * 3 * sizeof(double);
        if (kSolveWindow3 && bytes <= kSolveLdsBytes && 3 * plane < ((int64_t)1 << 30) &&
            coop_blocks_for((const void*)kw, SBW, bytes, p->num_cu) >= bw) {
            A.stage = (int)wn;
            void* args[] = {&A};
            TO_HIP(hipLaunchCooperativeKernel((const void*)kw, dim3(bw), dim3(SBW), args, bytes, s));
            return TO_OK;
        }
    }
    void* args[] = {&A};
    TO_HIP(hipLaunchCooperativeKernel((const void*)k, dim3(blocks), dim3(SB), args, 0, s));
    return TO_OK;
}

// Warm start of the solve from a predicted field: the minimiser of the
// energy 1/2 u.K u - f.u over span{uh, up} (a Galerkin projection onto two
// vectors; K the free-DOF operator of eq. (5)).  Block partials of
// uh.K uh, uh.K up, up.K up, uh.f, up.f; the last block to finish solves the
// 2x2 system (or, when it is singular or one vector is zero, takes the better
// one-vector fit) and writes (a, b, energy, case) to coef.
template <int DIM>
__global__ __launch_bounds__(kBlock) void galerkin_kernel(Geo g, MatFree<DIM, double> op, const uint8_t* __restrict__ fm,
                                                          const double* __restrict__ f, const double* __restrict__ uh,
                                                          const double* __restrict__ up, double* partial,
                                                          unsigned* counter, double* coef) {
    __shared__ double sh[kWaves];
    __shared__ int last;
    double v[5] = {0, 0, 0, 0, 0};
    for (int64_t nd = blockIdx.x * (int64_t)kBlock + threadIdx.x; nd < g.nnode; nd += (int64_t)gridDim.x * kBlock) {
        int iy, ix, iz;
        g.coords(nd, iy, ix, iz, DIM);
        double kh[DIM], kp[DIM];
        op.apply(nd, iy, ix, iz, SrcMask<DIM, double>{uh, fm}, kh);
        op.apply(nd, iy, ix, iz, SrcMask<DIM, double>{up, fm}, kp);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t i = DIM * nd + c;
            if (!fm[i]) continue;
            v[0] += uh[i] * kh[c];
            v[1] += uh[i] * kp[c];
            v[2] += up[i] * kp[c];
            v[3] += uh[i] * f[i];
            v[4] += up[i] * f[i];
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double s = block_sum(v[k], sh);
        if (threadIdx.x == 0) st_dev(&partial[blockIdx.x * 8 + k], s);
    }
    if (threadIdx.x == 0) {
        wait_stores();
        const unsigned done = atomicAdd(counter, 1u);
        last = done == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    double t[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) s += ld_dev(&partial[b * 8 + k]);
        t[k] = block_sum(s, sh);
    }
    if (threadIdx.x == 0) {
        const double A11 = t[0], A12 = t[1], A22 = t[2], r1 = t[3], r2 = t[4];
        const double det = A11 * A22 - A12 * A12;
        double a = 0.0, b = 0.0, E = 0.0, which = 0.0;
        if (A11 > 0.0 && A22 > 0.0 && det > 1e-12 * A11 * A22) {
            a = (r1 * A22 - r2 * A12) / det;
            b = (A11 * r2 - A12 * r1) / det;
            E = -0.5 * (a * r1 + b * r2);
            which = 3.0;
        } else {
            const double E1 = A11 > 0.0 ? -0.5 * r1 * r1 / A11 : INFINITY;
            const double E2 = A22 > 0.0 ? -0.5 * r2 * r2 / A22 : INFINITY;
            if (E1 <= E2 && A11 > 0.0) { a = r1 / A11; E = E1; which = 1.0; }
            else if (A22 > 0.0) { b = r2 / A22; E = E2; which = 2.0; }
        }
        coef[0] = a; coef[1] = b; coef[2] = E; coef[3] = which;
        st_dev(counter, 0u);
    }
}

template <int DIM>
__global__ void galerkin_combine_kernel(int64_t n, const uint8_t* __restrict__ fm, const double* uh, const double* up,
                                        const double* __restrict__ coef, double* u) {
    const double a = coef[0], b = coef[1];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        u[i] = fm[i] ? a * uh[i] + b * up[i] : 0.0;
}

to_status launch_warm_start(Plan* p, to_dtype dt, const void* xphys, double penal, const double* f,
                            const double* uh, const double* up, double* u, double* coef, hipStream_t s) {
    to_status r = launch_moduli(p, dt, xphys, penal, s, true);
    if (r != TO_OK) return r;
    const Geo g{p->nelx, p->nely, p->nelz, p->info.nnode};
    double* part = p->partial + (size_t)kMaxCoopBlocks * kPartialWidth;
    double* cf = coef ? coef : p->scal + 16;
    const int nb = (int)std::min<int64_t>(2048, (g.nnode + kBlock - 1) / kBlock);
    const int64_t n = p->info.n;
    const int nb2 = (int)std::min<int64_t>(4096, (n + kBlock - 1) / kBlock);
    if (p->dim == 2) {
        MatFree<2, double> op{p->E64, p->kf64, p->nelx, p->nely, p->nelz};
        hipLaunchKernelGGL(galerkin_kernel<2>, dim3(nb), dim3(kBlock), 0, s, g, op, p->freemask, f, uh, up, part,
                           p->bar + 10, cf);
        hipLaunchKernelGGL(galerkin_combine_kernel<2>, dim3(nb2), dim3(kBlock), 0, s, n, p->freemask, uh, up, cf, u);
    } else {
        MatFree<3, double> op{p->E64, p->kf64, p->nelx, p->nely, p->nelz};
        hipLaunchKernelGGL(galerkin_kernel<3>, dim3(nb), dim3(kBlock), 0, s, g, op, p->freemask, f, uh, up, part,
                           p->bar + 10, cf);
        hipLaunchKernelGGL(galerkin_combine_kernel<3>, dim3(nb2), dim3(kBlock), 0, s, n, p->freemask, uh, up, cf, u);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

int solve_mode(to_dtype dt, const to_solve_opts& o) {
    const bool mixed = dt == TO_F32 && o.precision == TO_SOLVE_MIXED;
    // TO_OP_HYBRID: the FP64 matrix-free operator with the assembled diagonal
    // (the mixed scheme keeps its FP32 assembled inner operator)
    const bool assembled = (o.op == TO_OP_ASSEMBLED && (dt == TO_F64 || mixed)) || (o.op == TO_OP_HYBRID && mixed);
    return !mixed ? (assembled ? 0 : 1) : (assembled ? 2 : 3);
}

// moduli for the matrix-free operators (FP64 always; FP32 too in mixed mode)
to_status solve_prepare(Plan* p, to_dtype dt, const void* xphys, double penal, const to_solve_opts& o, hipStream_t s) {
    if (solve_mode(dt, o) != 0) return launch_moduli(p, dt, xphys, penal, s, true);
    return TO_OK;
}

size_t solve_args_bytes() { return sizeof(SolveArgs); }

void solve_args_fill(Plan* p, to_dtype dt, const void* kval, const double* f, double* u, const to_solve_opts& o,
                     to_solve_stats* st, void* dst) {
    const int mode = solve_mode(dt, o);
    SolveArgs A{};
    A.geo = Geo{p->nelx, p->nely, p->nelz, p->info.nnode};
    A.freem = p->freemask;
    A.rp = p->row_ptr;
    A.kval = kval;
    A.kdiag32 = (dt == TO_F32 && mode == 1 && o.op != TO_OP_MATFREE) ? (const float*)kval : nullptr;
    A.kdiag64 = (dt == TO_F64 && mode == 1 && o.op == TO_OP_HYBRID) ? (const double*)kval : nullptr;
    A.E64 = p->E64; A.E32 = p->E32; A.kf64 = p->kf64; A.kf32 = p->kf32;
    A.f = f; A.u = u;
    for (int i = 0; i < 8; ++i) { A.v64[i] = p->v64[i]; A.v32[i] = p->v32[i]; }
    A.rtol = o.rtol; A.inner_rtol = o.inner_rtol; A.maxit = o.maxit;
    A.zero_x0 = o.zero_x0;
    A.partial = p->partial; A.bar = p->bar; A.ll = p->ll; A.st = st;
    std::memcpy(dst, &A, sizeof A);
}

to_status launch_solve(Plan* p, to_dtype dt, const void* kval, const void* xphys, double penal,
                       const double* f, double* u, const to_solve_opts& o, to_solve_stats* st, hipStream_t s) {
    if (o.precond == TO_PREC_GMG) return launch_solve_gmg(p, dt, xphys, penal, f, u, o, st, s);
    if (o.op != TO_OP_MATFREE && !kval) { set_error("kval is NULL"); return TO_EINVAL; }
    to_status r = solve_prepare(p, dt, xphys, penal, o, s);
    if (r != TO_OK) return r;
    SolveArgs A;
    solve_args_fill(p, dt, kval, f, u, o, st, &A);
    const int mode = solve_mode(dt, o);
    if (p->dim == 2) {
        switch (mode) {
        case 0: return launch_solve_t<2, 0>(p, A, o.grid_blocks, s);
        case 1: return launch_solve_t<2, 1>(p, A, o.grid_blocks, s);
        case 2: r = launch_solve_t<2, 2>(p, A, o.grid_blocks, s); break;
        default: r = launch_solve_t<2, 3>(p, A, o.grid_blocks, s); break;
        }
        // the mixed solve's FP64 fallback (returns at once unless it stalled)
        return r != TO_OK ? r : launch_solve_t<2, kModeFallback>(p, A, o.grid_blocks, s);
    }
    switch (mode) {
    case 0: return launch_solve_t<3, 0>(p, A, o.grid_blocks, s);
    case 1: return launch_solve_t<3, 1>(p, A, o.grid_blocks, s);
    case 2: r = launch_solve_t<3, 2>(p, A, o.grid_blocks, s); break;
    default: r = launch_solve_t<3, 3>(p, A, o.grid_blocks, s); break;
    }
    return r != TO_OK ? r : launch_solve_t<3, kModeFallback>(p, A, o.grid_blocks, s);
}

static const void* solve_batch_fn(int dim, int mode) {
    if (dim == 2) {
        switch (mode) {
        case 0: return (const void*)solve_batch_kernel<2, 0>;
        case 1: return (const void*)solve_batch_kernel<2, 1>;
        case 2: return (const void*)solve_batch_kernel<2, 2>;
        default: return (const void*)solve_batch_kernel<2, 3>;
        }
    }
    switch (mode) {
    case 0: return (const void*)solve_batch_kernel<3, 0>;
    case 1: return (const void*)solve_batch_kernel<3, 1>;
    case 2: return (const void*)solve_batch_kernel<3, 2>;
    default: return (const void*)solve_batch_kernel<3, 3>;
    }
}

int solve_block_size(int dim, int mode) { return solve_block(dim, mode); }

static const void* solve_batch_fallback_fn(int dim) {
    return dim == 2 ? (const void*)solve_batch_kernel<2, kModeFallback> : (const void*)solve_batch_kernel<3, kModeFallback>;
}

int solve_batch_capacity(int dim, int mode, int num_cu) {
    int c = coop_blocks_for(solve_batch_fn(dim, mode), solve_block(dim, mode), 0, num_cu);
    if (mode >= 2) c = std::min(c, coop_blocks_for(solve_batch_fallback_fn(dim), solve_block(dim, mode), 0, num_cu));
    return c;
}

to_status launch_solve_batch(int dim, int mode, const void* tab, const BatchMap& mp, hipStream_t s) {
    void* args[] = {(void*)&tab, (void*)&mp.inst, (void*)&mp.first, (void*)&mp.count};
    TO_HIP(hipLaunchCooperativeKernel(solve_batch_fn(dim, mode), dim3(mp.blocks), dim3(solve_block(dim, mode)), args,
                                      0, s));
    if (mode >= 2)        // the mixed solves' FP64 fallbacks, per design (each returns at once unless it stalled)
        TO_HIP(hipLaunchCooperativeKernel(solve_batch_fallback_fn(dim), dim3(mp.blocks), dim3(solve_block(dim, mode)),
                                          args, 0, s));
    return TO_OK;
}

}  // namespace topt
