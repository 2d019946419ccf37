// Geometric-multigrid preconditioned CG for the state solve (eq. (5)) in 2D
// and 3D, the solver the paper uses for its large 3D runs (Sec. 4).
//
// Hierarchy: level l+1 has ceil(n_l / 2) elements per direction; bi- or
// trilinear prolongation P (a fine node at an odd index takes the mean of its
// two coarse neighbours along that axis, so any element count coarsens; fine
// elements missing from a coarse element simply contribute nothing).  Coarse
// operators are Galerkin, A_{l+1} = P^T A_l P, formed element by element:
// inside a coarse element the prolongated field is the multilinear
// interpolation of its corners, so a coarse element matrix is the sum over
// its (up to 2^dim) child element matrices of P_c^T A_child P_c, with P_c the
// D x D local interpolation of child position c (D = 8 in 2D, 24 in 3D).  On
// the finest level the child matrices are E_e Ke with the rows and columns of
// fixed DOFs removed (the masked operator of eq. (5)), so the coarse spaces
// respect the supports.  Coarse element matrices are stored (D^2 doubles
// each); the coarsest level (at most kGmgCoarseMax DOFs) is inverted densely
// by Gauss-Jordan elimination in one block and applied as a dense
// matrix-vector product.
//
// V-cycle: Chebyshev smoothing of degree kGmgNu before and after (the same
// polynomial, so the preconditioner is symmetric), residual, restriction P^T,
// coarse correction, prolongation.  The smoother is the Chebyshev iteration
// for D1^-1 A on the interval [1 / kGmgChebRatio, 1], with D1 the element-wise
// l1 diagonal D1_ii = sum_e sum_j |A^e_ij|: D1 - A is diagonally dominant, so
// the spectrum of D1^-1 A lies in (0, 1] on every level, in 2D and 3D and for
// any design, and no damping weight has to be tuned (a Jacobi weight that
// suits Q4 elements, whose D^-1 A reaches about 2.9, diverges for Hex8
// elements, where it reaches about 4.8).  Outer iteration: flexible
// (Polak-Ribiere) PCG, FP64, convergence on the recursive residual confirmed
// by the true residual, like the Jacobi PCG.  All scalars live on the device;
// every kernel returns at once when the device `done` flag is set, so the host
// enqueues iterations in batches and reads the flag between batches.
#include <cmath>
#include <cstring>

#include "common.h"
#include "operators.h"

namespace topt {

constexpr int kGmgNu = 2;                    // Chebyshev degree of each smoothing
constexpr double kGmgChebRatio = 8.0;        // interval [1 / ratio, 1] of D1^-1 A

// Coefficients of the Chebyshev iteration for D1^-1 A on [lo, hi]
// (theta = (hi + lo) / 2, delta = (hi - lo) / 2, sigma = theta / delta):
// d_0 = D1^-1 r_0 / theta; d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) D1^-1 r_k,
// rho_0 = 1 / sigma, rho_k = 1 / (2 sigma - rho_{k-1}); x_{k+1} = x_k + d_k.
struct ChebStep { double cd, cr; };
static ChebStep cheb_step(int k) {
    const double hi = 1.0, lo = 1.0 / kGmgChebRatio;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    if (k == 0) return {0.0, 1.0 / theta};
    double rho = 1.0 / sigma, rho_prev = rho;
    for (int i = 1; i <= k; ++i) { rho_prev = rho; rho = 1.0 / (2.0 * sigma - rho); }
    return {rho * rho_prev, 2.0 * rho / delta};
}
constexpr int kGmgBatch = 8;           // iterations per captured batch (even: the directions alternate)
constexpr int kGmgMaxRestarts = 64;    // true-residual confirmations that may reopen the iteration


// --- deterministic block partials + last-block finish --------------------------
template <int K>
__device__ __forceinline__ bool last_block_sums(const double (&v)[K], double* partial, unsigned* counter,
                                                double (&tot)[K]) {
    __shared__ double sh[kWaves];
    __shared__ int last;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double s = block_sum(v[k], sh);
        if (threadIdx.x == 0) st_dev(&partial[blockIdx.x * 8 + k], s);
    }
    if (threadIdx.x == 0) {
        wait_stores();
        const unsigned done = atomicAdd(counter, 1u);
        last = done == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) s += ld_dev(&partial[b * 8 + k]);
        tot[k] = block_sum(s, sh);
    }
    if (threadIdx.x == 0) st_dev(counter, 0u);
    return true;
}

// Local corners of an element (2D: the first four): y, x and z offsets; the
// corner order is the one of the element matrices.
__device__ constexpr int kCY[8] = {1, 1, 0, 0, 1, 1, 0, 0};
__device__ constexpr int kCX[8] = {0, 1, 1, 0, 0, 1, 1, 0};
__device__ constexpr int kCZ[8] = {0, 0, 0, 0, 1, 1, 1, 1};

template <int DIM> struct Cell {
    static constexpr int NC = DIM == 2 ? 4 : 8;     // corners
    static constexpr int D = DIM * NC;              // element DOFs
};

struct LevelArgs {
    int nx, ny, nz;
    int64_t nnode;
    const double* K;          // stored element matrices (levels >= 1), else null
    const double* S;          // assembled node stencils (levels >= 1), else null
    const double* E;          // level 0: moduli
    const double* ke;         // level 0: element matrix
    const uint8_t* fm;        // level 0: free mask (null above)
};

template <int DIM>
__device__ __forceinline__ void node_coords(int64_t nd, int ny, int nz, int& iy, int& ix, int& iz) {
    iy = (int)(nd % (ny + 1));
    const int64_t rest = nd / (ny + 1);
    if (DIM == 2) { ix = (int)rest; iz = 0; }
    else { iz = (int)(rest % (nz + 1)); ix = (int)(rest / (nz + 1)); }
}
template <int DIM>
__device__ __forceinline__ int64_t node_at(int ny, int nz, int y, int x, int z) {
    return DIM == 2 ? y + (int64_t)(ny + 1) * x : y + (int64_t)(ny + 1) * (z + (int64_t)(nz + 1) * x);
}
template <int DIM>
__device__ __forceinline__ int64_t elem_at(int ny, int nz, int y, int x, int z) {
    return DIM == 2 ? y + (int64_t)ny * x : y + (int64_t)ny * (z + (int64_t)nz * x);
}
template <int DIM>
__device__ __forceinline__ bool elem_in(int nx, int ny, int nz, int y, int x, int z) {
    return y >= 0 && y < ny && x >= 0 && x < nx && (DIM == 2 || (z >= 0 && z < nz));
}

// --- level operators ----------------------------------------------------------
// y = A x at node nd from the assembled stencil: S holds, for neighbour k of
// the 3^DIM box (k = ((dx + 1) 3 + (dz + 1)) 3 + (dy + 1), dz absent in 2D)
// and components (c, c2), the block entry at S[((k DIM + c) DIM + c2) nnode + nd]
// (entry-major, so a wave reads consecutive nodes).  Each entry is read once
// per application, where element matrices would be read by every corner node.
template <int DIM>
__device__ __forceinline__ void stencil_apply(const double* __restrict__ S, int64_t nnode,
                                              const double* __restrict__ x, int nx, int ny, int nz, int64_t nd, int iy,
                                              int ix, int iz, double (&out)[DIM]) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) out[c] = 0.0;
    constexpr int ZR = DIM == 3 ? 1 : 0;
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx)
#pragma unroll
        for (int dz = -ZR; dz <= ZR; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int k = DIM == 2 ? (dx + 1) * 3 + (dy + 1) : ((dx + 1) * 3 + (dz + 1)) * 3 + (dy + 1);
                const bool ok = iy + dy >= 0 && iy + dy <= ny && ix + dx >= 0 && ix + dx <= nx &&
                                (DIM == 2 || (iz + dz >= 0 && iz + dz <= nz));
                if (!ok) continue;
                const int64_t q = node_at<DIM>(ny, nz, iy + dy, ix + dx, iz + dz);
#pragma unroll
                for (int c2 = 0; c2 < DIM; ++c2) {
                    const double xv = x[DIM * q + c2];
#pragma unroll
                    for (int c = 0; c < DIM; ++c) out[c] += S[((size_t)(k * DIM + c) * DIM + c2) * nnode + nd] * xv;
                }
            }
}

// plain source vector of the level-0 operator (the V-cycle's vectors are 0 on fixed DOFs)
template <int DIM> struct SrcPlain {
    const double* x;
    __device__ __forceinline__ double operator()(int64_t q, int c) const { return x[DIM * q + c]; }
};

// y = A x at node nd on level 0 (matrix-free, E_e Ke) or a stored level (stencil)
template <int DIM, bool STORED>
__device__ __forceinline__ void level_apply(const LevelArgs& L, const double* x, int64_t nd, int iy, int ix, int iz,
                                            double (&out)[DIM]) {
    if constexpr (STORED) {
        stencil_apply<DIM>(L.S, L.nnode, x, L.nx, L.ny, L.nz, nd, iy, ix, iz, out);
    } else {
        MatFree<DIM, double> op{L.E, L.ke, L.nx, L.ny, L.nz};
        op.apply(nd, iy, ix, iz, SrcPlain<DIM>{x}, out);
    }
}

// node stencils of a stored level from its element matrices: one thread per
// (node, neighbour k); the element contributions are summed in corner order
template <int DIM>
__global__ __launch_bounds__(kBlock) void gmg_stencil_kernel(int nx, int ny, int nz, int64_t nnode,
                                                             const double* __restrict__ K, double* __restrict__ S) {
    constexpr int NC = Cell<DIM>::NC, D = Cell<DIM>::D, NS = DIM == 2 ? 9 : 27;
    for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < nnode * NS; t += (int64_t)gridDim.x * kBlock) {
        const int64_t nd = t / NS;
        const int k = (int)(t % NS);
        const int dy = k % 3 - 1;
        const int dz = DIM == 3 ? (k / 3) % 3 - 1 : 0;
        const int dx = (DIM == 3 ? k / 9 : k / 3) - 1;
        int iy, ix, iz;
        node_coords<DIM>(nd, ny, nz, iy, ix, iz);
        double acc[DIM][DIM] = {};
        for (int a = 0; a < NC; ++a) {
            const int ey = iy - kCY[a], ex = ix - kCX[a], ez = iz - kCZ[a];
            if (!elem_in<DIM>(nx, ny, nz, ey, ex, ez)) continue;
            const int by = kCY[a] + dy, bx = kCX[a] + dx, bz = kCZ[a] + dz;
            if (by < 0 || by > 1 || bx < 0 || bx > 1 || bz < 0 || bz > (DIM == 3 ? 1 : 0)) continue;
            int b = 0;
            for (int q = 0; q < NC; ++q)
                if (kCY[q] == by && kCX[q] == bx && kCZ[q] == bz) b = q;
            const double* Ke = K + (size_t)elem_at<DIM>(ny, nz, ey, ex, ez) * D * D;
            for (int c = 0; c < DIM; ++c)
                for (int c2 = 0; c2 < DIM; ++c2) acc[c][c2] += Ke[(DIM * a + c) * D + DIM * b + c2];
        }
        for (int c = 0; c < DIM; ++c)
            for (int c2 = 0; c2 < DIM; ++c2) S[((size_t)(k * DIM + c) * DIM + c2) * nnode + nd] = acc[c][c2];
    }
}

// mode 0: y = b - A x (residual);
// mode 1: Chebyshev step  d = cd d + cr dinv (b - A x),  y = x + d;
// mode 2: the first step from x = 0:  d = cr dinv b,  y = d.
// d is updated in place (each entry by its own thread); y and x differ.
template <int DIM, bool STORED>
__global__ __launch_bounds__(kBlock) void gmg_sweep_kernel(LevelArgs L, int mode, const double* __restrict__ x,
                                                           const double* __restrict__ b, const double* __restrict__ dinv,
                                                           double* __restrict__ y, double* d, double cd, double cr,
                                                           const int32_t* done) {
    if (*done) return;
    for (int64_t nd = blockIdx.x * (int64_t)kBlock + threadIdx.x; nd < L.nnode; nd += (int64_t)gridDim.x * kBlock) {
        int iy, ix, iz;
        node_coords<DIM>(nd, L.ny, L.nz, iy, ix, iz);
        double ax[DIM] = {};
        if (mode != 2) level_apply<DIM, STORED>(L, x, nd, iy, ix, iz, ax);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t i = DIM * nd + c;
            const bool fr = !L.fm || L.fm[i];
            if (mode == 0) {
                y[i] = fr ? b[i] - ax[c] : 0.0;
            } else if (mode == 1) {
                const double dn = fr ? (cd == 0.0 ? 0.0 : cd * d[i]) + cr * dinv[i] * (b[i] - ax[c]) : 0.0;
                d[i] = dn;
                y[i] = fr ? x[i] + dn : 0.0;
            } else {
                const double dn = fr ? cr * dinv[i] * b[i] : 0.0;
                d[i] = dn;
                y[i] = dn;
            }
        }
    }
}

// dinv = 1 / D1, D1_ii = sum over the elements of node i of sum_j |A^e_ij|
template <int DIM>
__global__ __launch_bounds__(kBlock) void gmg_diag_kernel(LevelArgs L, double* __restrict__ dinv) {
    constexpr int NC = Cell<DIM>::NC, D = Cell<DIM>::D;
    for (int64_t nd = blockIdx.x * (int64_t)kBlock + threadIdx.x; nd < L.nnode; nd += (int64_t)gridDim.x * kBlock) {
        int iy, ix, iz;
        node_coords<DIM>(nd, L.ny, L.nz, iy, ix, iz);
        double d[DIM] = {};
        for (int a = 0; a < NC; ++a) {
            const int ey = iy - kCY[a], ex = ix - kCX[a], ez = iz - kCZ[a];
            if (!elem_in<DIM>(L.nx, L.ny, L.nz, ey, ex, ez)) continue;
            const int64_t e = elem_at<DIM>(L.ny, L.nz, ey, ex, ez);
            // columns of the element: level 0 leaves out fixed DOFs (the masked operator)
            unsigned live = ~0u;
            if (L.fm) {
                live = 0u;
                for (int b = 0; b < NC; ++b) {
                    const int64_t q = node_at<DIM>(L.ny, L.nz, ey + kCY[b], ex + kCX[b], ez + kCZ[b]);
                    for (int c2 = 0; c2 < DIM; ++c2)
                        if (L.fm[DIM * q + c2]) live |= 1u << (DIM * b + c2);
                }
            }
            for (int c = 0; c < DIM; ++c) {
                const int r = DIM * a + c;
                const double* row = L.K ? L.K + e * D * D + r * D : L.ke + r * D;
                double s = 0.0;
                for (int j = 0; j < D; ++j)
                    if ((live >> j) & 1u) s += fabs(row[j]);
                d[c] += L.K ? s : L.E[e] * s;
            }
        }
        for (int c = 0; c < DIM; ++c) {
            const int64_t i = DIM * nd + c;
            const bool fr = !L.fm || L.fm[i];
            dinv[i] = fr && d[c] > 0.0 ? 1.0 / d[c] : 0.0;
        }
    }
}

// coarse element matrices from the children (Galerkin, element by element):
// one thread per (coarse element, row of its D x D matrix)
template <int DIM>
__global__ __launch_bounds__(kBlock) void gmg_galerkin_kernel(int fnx, int fny, int fnz, int cnx, int cny, int cnz,
                                                              const double* __restrict__ E,
                                                              const double* __restrict__ ke,
                                                              const uint8_t* __restrict__ fm,
                                                              const double* __restrict__ Kf, double* __restrict__ Kc) {
    constexpr int NC = Cell<DIM>::NC, D = Cell<DIM>::D;
    const int64_t mc = (int64_t)cnx * cny * (DIM == 3 ? cnz : 1);
    for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < D * mc; t += (int64_t)gridDim.x * kBlock) {
        const int64_t E_c = t / D;
        const int row = (int)(t % D);                  // coarse DOF DIM a + k
        const int a = row / DIM, k = row % DIM;
        int ey, ex, ez;
        node_coords<DIM>(E_c, cny - 1, cnz - 1, ey, ex, ez);    // element grid = node grid of one less
        double acc[D];
#pragma unroll
        for (int i = 0; i < D; ++i) acc[i] = 0.0;
#pragma unroll 1
        for (int ch = 0; ch < NC; ++ch) {
            const int cx = ch / (NC / 2), cy = (ch / (DIM == 3 ? 2 : 1)) & 1, cz = DIM == 3 ? (ch & 1) : 0;
            const int fy = 2 * ey + cy, fx = 2 * ex + cx, fz = 2 * ez + cz;
            if (fy >= fny || fx >= fnx || (DIM == 3 && fz >= fnz)) continue;
            const int64_t fe = elem_at<DIM>(fny, fnz, fy, fx, fz);
            // interpolation weight of child corner b from coarse corner a' is
            // separable: W[0][CY[b]][CY[a']] W[1][CX[b]][CX[a']] W[2][CZ[b]][CZ[a']],
            // with W[d][s][t] = t ? pos : 1 - pos, pos = (child offset + s) / 2
            double W[3][2][2];
            const int co[3] = {cy, cx, cz};
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int sd = 0; sd < 2; ++sd) {
                    const double pos = 0.5 * (co[d] + sd);
                    W[d][sd][0] = 1.0 - pos;
                    W[d][sd][1] = pos;
                }
            auto w = [&](int b, int a2) {
                double v = W[0][kCY[b]][kCY[a2]] * W[1][kCX[b]][kCX[a2]];
                if (DIM == 3) v *= W[2][kCZ[b]][kCZ[a2]];
                return v;
            };
            unsigned live = 0;                  // bit j: DOF j of the child is free
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                const int64_t node = node_at<DIM>(fny, fnz, fy + kCY[b], fx + kCX[b], fz + kCZ[b]);
#pragma unroll
                for (int c = 0; c < DIM; ++c)
                    if (!fm || fm[DIM * node + c]) live |= 1u << (DIM * b + c);
            }
            const double Ee = E ? E[fe] : 1.0;
            const double* A = Kf ? Kf + fe * D * D : ke;
            // Kc[row][DIM a' + k'] += sum_{b, b'} w(b, a) A[DIM b + k][DIM b' + k'] w(b', a')
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                const int fr = DIM * b + k;
                const double wba = w(b, a);
                if (!((live >> fr) & 1u) || wba == 0.0) continue;
                const double wr = wba * Ee;
#pragma unroll
                for (int b2 = 0; b2 < NC; ++b2)
#pragma unroll
                    for (int k2 = 0; k2 < DIM; ++k2) {
                        const int fc = DIM * b2 + k2;
                        if (!((live >> fc) & 1u)) continue;
                        const double v = wr * A[fr * D + fc];
#pragma unroll
                        for (int a2 = 0; a2 < NC; ++a2) acc[DIM * a2 + k2] += v * w(b2, a2);
                    }
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) Kc[E_c * D * D + row * D + i] = acc[i];
    }
}

// b_c = P^T r_f
template <int DIM>
__global__ __launch_bounds__(kBlock) void gmg_restrict_kernel(int fnx, int fny, int fnz, int cnx, int cny, int cnz,
                                                              const double* __restrict__ rf, double* __restrict__ bc,
                                                              const int32_t* done) {
    if (*done) return;
    const int64_t nc = (int64_t)(cnx + 1) * (cny + 1) * (DIM == 3 ? cnz + 1 : 1);
    for (int64_t nd = blockIdx.x * (int64_t)kBlock + threadIdx.x; nd < nc; nd += (int64_t)gridDim.x * kBlock) {
        int I, J, Kz;
        node_coords<DIM>(nd, cny, cnz, I, J, Kz);
        double s[DIM] = {};
        for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy) {
                    const int fy = 2 * I + dy, fx = 2 * J + dx, fz = 2 * Kz + dz;
                    if (fy < 0 || fy > fny || fx < 0 || fx > fnx || (DIM == 3 && (fz < 0 || fz > fnz))) continue;
                    const double w = (dy ? 0.5 : 1.0) * (dx ? 0.5 : 1.0) * (dz ? 0.5 : 1.0);
                    const int64_t q = node_at<DIM>(fny, fnz, fy, fx, fz);
#pragma unroll
                    for (int c = 0; c < DIM; ++c) s[c] += w * rf[DIM * q + c];
                }
#pragma unroll
        for (int c = 0; c < DIM; ++c) bc[DIM * nd + c] = s[c];
    }
}

// x_f += P x_c (fixed DOFs of the finest level untouched)
template <int DIM>
__global__ __launch_bounds__(kBlock) void gmg_prolong_kernel(int fnx, int fny, int fnz, int cny, int cnz,
                                                             const double* __restrict__ xc,
                                                             const uint8_t* __restrict__ fm, double* __restrict__ xf,
                                                             const int32_t* done) {
    if (*done) return;
    const int64_t nf = (int64_t)(fnx + 1) * (fny + 1) * (DIM == 3 ? fnz + 1 : 1);
    for (int64_t nd = blockIdx.x * (int64_t)kBlock + threadIdx.x; nd < nf; nd += (int64_t)gridDim.x * kBlock) {
        int fy, fx, fz;
        node_coords<DIM>(nd, fny, fnz, fy, fx, fz);
        const int ys[2] = {fy >> 1, (fy + 1) >> 1}, xs[2] = {fx >> 1, (fx + 1) >> 1};
        const int zs[2] = {fz >> 1, (fz + 1) >> 1};
        const int ny_ = ys[0] == ys[1] ? 1 : 2, nx_ = xs[0] == xs[1] ? 1 : 2, nz_ = zs[0] == zs[1] ? 1 : 2;
        const double w = (ny_ == 1 ? 1.0 : 0.5) * (nx_ == 1 ? 1.0 : 0.5) * (nz_ == 1 ? 1.0 : 0.5);
        double s[DIM] = {};
        for (int k = 0; k < nz_; ++k)
            for (int i = 0; i < nx_; ++i)
                for (int j = 0; j < ny_; ++j) {
                    const int64_t q = node_at<DIM>(cny, cnz, ys[j], xs[i], zs[k]);
#pragma unroll
                    for (int c = 0; c < DIM; ++c) s[c] += w * xc[DIM * q + c];
                }
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t i = DIM * nd + c;
            if (!fm || fm[i]) xf[i] += s[c];
        }
    }
}

// dense coarsest matrix (rows of DOFs no element reaches stay 0: the
// inversion zeroes them)
template <int DIM>
__global__ __launch_bounds__(kBlock) void gmg_dense_kernel(int nx, int ny, int nz, const double* __restrict__ K,
                                                           int nc, double* __restrict__ A) {
    constexpr int NC = Cell<DIM>::NC, D = Cell<DIM>::D;
    for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < (int64_t)nc * nc;
         idx += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(idx / nc), j = (int)(idx % nc);
        const int ni = i / DIM, ci = i % DIM, nj = j / DIM, cj = j % DIM;
        int iy, ix, iz, jy, jx, jz;
        node_coords<DIM>(ni, ny, nz, iy, ix, iz);
        node_coords<DIM>(nj, ny, nz, jy, jx, jz);
        double s = 0.0;
        if (abs(iy - jy) <= 1 && abs(ix - jx) <= 1 && abs(iz - jz) <= 1) {
            for (int a = 0; a < NC; ++a) {
                const int ey = iy - kCY[a], ex = ix - kCX[a], ez = iz - kCZ[a];
                if (!elem_in<DIM>(nx, ny, nz, ey, ex, ez)) continue;
                for (int b = 0; b < NC; ++b) {
                    if (ey + kCY[b] != jy || ex + kCX[b] != jx || ez + kCZ[b] != jz) continue;
                    s += K[elem_at<DIM>(ny, nz, ey, ex, ez) * D * D + (DIM * a + ci) * D + DIM * b + cj];
                }
            }
        }
        A[idx] = s;
    }
}

// In-place inverse of the SPD coarsest matrix by Gauss-Jordan elimination in
// LDS (one block; no pivoting is needed for SPD matrices).  A zero pivot marks
// a DOF no coarse basis function reaches: its row and column become zero.
__global__ __launch_bounds__(1024) void gmg_invert_kernel(double* A, int n) {
    __shared__ double M[kGmgCoarseMax * kGmgCoarseMax];
    __shared__ double piv_row[kGmgCoarseMax];
    __shared__ double piv_col[kGmgCoarseMax];
    const int nn = n * n;
    for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) M[idx] = A[idx];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            piv_row[j] = M[k * n + j];
            piv_col[j] = M[j * n + k];
        }
        __syncthreads();
        const double p = piv_row[k];
        const double ip = p > 0.0 ? 1.0 / p : 0.0;
        for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
            const int i = idx / n, j = idx - i * n;
            double v;
            if (ip == 0.0) v = (i == k || j == k) ? 0.0 : M[idx];
            else if (i == k && j == k) v = ip;
            else if (i == k) v = piv_row[j] * ip;
            else if (j == k) v = -piv_col[i] * ip;
            else v = M[idx] - piv_col[i] * piv_row[j] * ip;
            M[idx] = v;
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) A[idx] = M[idx];
}

// x_c = A^{-1} b_c (the inverse is symmetric: thread i reads column i)
__global__ __launch_bounds__(kBlock) void gmg_coarse_solve_kernel(const double* __restrict__ Ainv, int n,
                                                                  const double* __restrict__ b, double* __restrict__ x,
                                                                  const int32_t* done) {
    if (*done) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;      // four chains: the loads overlap
        int j = 0;
        for (; j + 4 <= n; j += 4) {
            s0 += Ainv[(size_t)j * n + i] * b[j];
            s1 += Ainv[(size_t)(j + 1) * n + i] * b[j + 1];
            s2 += Ainv[(size_t)(j + 2) * n + i] * b[j + 2];
            s3 += Ainv[(size_t)(j + 3) * n + i] * b[j + 3];
        }
        for (; j < n; ++j) s0 += Ainv[(size_t)j * n + i] * b[j];
        x[i] = (s0 + s1) + (s2 + s3);
    }
}

// --- outer flexible PCG ---------------------------------------------------------
// r = f - A u on free DOFs, u = 0 on fixed ones; |f|, |r|.
// mode 1: the initial residual (also |f| and the counters);
// mode 2: the true-residual confirmation, run only while S->check is set:
//         accept (confirmed) if |r| meets the tolerance, else restart the
//         directions from this residual unless a cap has been reached.
template <int DIM>
__global__ __launch_bounds__(kBlock) void fcg_residual_kernel(LevelArgs L, const double* __restrict__ f, double* u,
                                                              double* __restrict__ r, double* partial,
                                                              unsigned* counter, GmgScal* S, int mode) {
    if (mode == 2 && !S->check) return;
    double v[2] = {0.0, 0.0};
    for (int64_t nd = blockIdx.x * (int64_t)kBlock + threadIdx.x; nd < L.nnode; nd += (int64_t)gridDim.x * kBlock) {
        int iy, ix, iz;
        node_coords<DIM>(nd, L.ny, L.nz, iy, ix, iz);
        double ax[DIM];
        MatFree<DIM, double> op{L.E, L.ke, L.nx, L.ny, L.nz};
        op.apply(nd, iy, ix, iz, SrcMask<DIM, double>{u, L.fm}, ax);     // u may hold values on fixed DOFs
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t i = DIM * nd + c;
            const bool fr = L.fm[i];
            const double ri = fr ? f[i] - ax[c] : 0.0;
            r[i] = ri;
            v[0] += fr ? f[i] * f[i] : 0.0;
            v[1] += ri * ri;
        }
    }
    double tot[2];
    if (last_block_sums<2>(v, partial, counter, tot) && threadIdx.x == 0) {
        S->rr = tot[1];
        if (mode == 1) {
            S->bnorm = sqrt(tot[0]);
            return;
        }
        S->check = 0;
        if (tot[1] <= S->tol * S->tol) {
            S->confirmed = 1;
        } else if (S->it < S->maxit && S->restarts < kGmgMaxRestarts) {
            S->done = 0;
            S->restart = 1;
            S->restarts += 1;
        }
    }
}

// z = M r finished: rz = r.z, roz = r_old.z; beta = (rz - roz) / rz_old (0 on restart)
__global__ __launch_bounds__(kBlock) void fcg_dots_kernel(int64_t n, const double* __restrict__ r,
                                                          const double* __restrict__ rold, const double* __restrict__ z,
                                                          double* partial, unsigned* counter, GmgScal* S) {
    if (S->done) return;
    // every block reads the flag before the last block (the last arrival)
    // clears it
    const int restart = S->restart;
    double v[2] = {0.0, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        v[0] += r[i] * z[i];
        if (!restart) v[1] += rold[i] * z[i];
    }
    double tot[2];
    if (last_block_sums<2>(v, partial, counter, tot) && threadIdx.x == 0) {
        S->beta = restart ? 0.0 : (tot[0] - tot[1]) / S->rz_old;
        S->rz = tot[0];
        S->rz_old = tot[0];
        S->restart = 0;
    }
}

// p = z + beta p (in place), q = A p; pq -> alpha
template <int DIM>
__global__ __launch_bounds__(kBlock) void fcg_dir_kernel(LevelArgs L, const double* __restrict__ z,
                                                         const double* __restrict__ pold, double* __restrict__ pnew,
                                                         double* __restrict__ q, double* partial, unsigned* counter,
                                                         GmgScal* S) {
    if (S->done) return;
    const double beta = S->beta;
    double v[1] = {0.0};
    for (int64_t nd = blockIdx.x * (int64_t)kBlock + threadIdx.x; nd < L.nnode; nd += (int64_t)gridDim.x * kBlock) {
        int iy, ix, iz;
        node_coords<DIM>(nd, L.ny, L.nz, iy, ix, iz);
        double ap[DIM];
        MatFree<DIM, double> op{L.E, L.ke, L.nx, L.ny, L.nz};
        op.apply(nd, iy, ix, iz, SrcZP<DIM, double>{z, pold, beta, Own{0, L.nnode, 0}}, ap);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t i = DIM * nd + c;
            const bool fr = L.fm[i];
            const double pi = fr ? z[i] + beta * pold[i] : 0.0;
            const double qi = fr ? ap[c] : 0.0;
            pnew[i] = pi;
            q[i] = qi;
            v[0] += pi * qi;
        }
    }
    double tot[1];
    if (last_block_sums<1>(v, partial, counter, tot) && threadIdx.x == 0) {
        S->pq = tot[0];
        S->alpha = tot[0] > 0.0 ? S->rz / tot[0] : 0.0;
        if (!(tot[0] > 0.0)) S->done = 2;            // breakdown: stop
    }
}

// u += alpha p; r_old = r; r -= alpha q; |r|
__global__ __launch_bounds__(kBlock) void fcg_update_kernel(int64_t n, const double* __restrict__ p,
                                                            const double* __restrict__ q, double* __restrict__ u,
                                                            double* __restrict__ r, double* __restrict__ rold,
                                                            double* partial, unsigned* counter, GmgScal* S) {
    if (S->done) return;
    const double a = S->alpha;
    double v[1] = {0.0};
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        u[i] += a * p[i];
        const double ri = r[i];
        rold[i] = ri;
        const double rn = ri - a * q[i];
        r[i] = rn;
        v[0] += rn * rn;
    }
    double tot[1];
    if (last_block_sums<1>(v, partial, counter, tot) && threadIdx.x == 0) {
        S->rr = tot[0];
        S->it += 1;
        if (tot[0] <= S->tol * S->tol) {
            S->done = 1;
            S->check = 1;            // confirmed on the true residual next
        } else if (S->it >= S->maxit) {
            S->done = 1;
        }
    }
}

__global__ void fcg_stats_kernel(const GmgScal* S, to_solve_stats* st, double rtol) {
    to_solve_stats s;
    const double bn = S->bnorm > 0.0 ? S->bnorm : 1.0;
    s.residual = sqrt(S->rr) / bn;
    s.bnorm = S->bnorm;
    s.iterations = S->it;
    s.outer = 0;
    s.converged = S->confirmed;
    s.fallback = 0;
    s.restarts = S->restarts;
    s.pad = 0;
    *st = s;
}

__global__ void fill_zero_f64_kernel(double* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void fcg_init_kernel(GmgScal* S, int maxit) {
    S->it = 0;
    S->done = 0;
    S->maxit = maxit;
    S->restarts = 0;
    S->rz_old = 1.0;
    S->check = 0;
    S->confirmed = 0;
    S->restart = 1;
}

// after the initial (true) residual: done at once if the start already meets
// the tolerance
__global__ void fcg_tol_kernel(GmgScal* S, double rtol) {
    S->tol = rtol * S->bnorm;
    const int ok = S->rr <= S->tol * S->tol ? 1 : 0;
    S->done = ok;
    S->confirmed = ok;
}

// --- host ------------------------------------------------------------------------
static int grid_of(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kBlock - 1) / kBlock)); }
// kernels that end in a last-block reduction: every block arrives on one
// counter, so fewer, fuller blocks (their arrivals serialise at one address)
static int grid_red(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + kBlock - 1) / kBlock)); }

static LevelArgs level_args(const Plan* p, int l) {
    const GmgLevel& v = p->gmg.lv[l];
    LevelArgs L{};
    L.nx = v.nx; L.ny = v.ny; L.nz = v.nz; L.nnode = v.nnode;
    if (l == 0) { L.K = nullptr; L.S = nullptr; L.E = p->E64; L.ke = p->kf64; L.fm = p->freemask; }
    else { L.K = v.K; L.S = v.S; L.E = nullptr; L.ke = nullptr; L.fm = nullptr; }
    return L;
}

// z = M r: one V-cycle from level l (x0 = 0); level-0 vectors b = r, x = z
template <int DIM>
static void vcycle(Plan* p, int l, const double* b, double* x, const int32_t* done, hipStream_t s) {
    Gmg& G = p->gmg;
    GmgLevel& v = G.lv[l];
    if (l == G.L - 1) {
        hipLaunchKernelGGL(gmg_coarse_solve_kernel, dim3(grid_of(v.n)), dim3(kBlock), 0, s, G.Ainv, (int)v.n, b, x,
                           done);
        return;
    }
    const LevelArgs L = level_args(p, l);
    const auto sweep = l == 0 ? gmg_sweep_kernel<DIM, false> : gmg_sweep_kernel<DIM, true>;
    double* t = v.xt;     // ping-pong partner of x
    double* r = v.r;
    const int g = grid_of(v.nnode);
    // pre-smoothing from x = 0: kGmgNu Chebyshev steps ending in x; the
    // step vector d lives in r (free until the residual below)
    double* cur = (kGmgNu % 2 == 1) ? x : t;
    double* nxt = (kGmgNu % 2 == 1) ? t : x;
    ChebStep cs = cheb_step(0);
    hipLaunchKernelGGL(sweep, dim3(g), dim3(kBlock), 0, s, L, 2, (const double*)nullptr, b, v.dinv,
                       cur, r, cs.cd, cs.cr, done);
    for (int k = 1; k < kGmgNu; ++k) {
        cs = cheb_step(k);
        hipLaunchKernelGGL(sweep, dim3(g), dim3(kBlock), 0, s, L, 1, cur, b, v.dinv, nxt, r, cs.cd,
                           cs.cr, done);
        std::swap(cur, nxt);
    }
    // residual, restriction, coarse correction, prolongation
    hipLaunchKernelGGL(sweep, dim3(g), dim3(kBlock), 0, s, L, 0, x, b, v.dinv, r, (double*)nullptr,
                       0.0, 0.0, done);
    GmgLevel& c = G.lv[l + 1];
    hipLaunchKernelGGL(gmg_restrict_kernel<DIM>, dim3(grid_of(c.nnode)), dim3(kBlock), 0, s, v.nx, v.ny, v.nz, c.nx,
                       c.ny, c.nz, r, c.b, done);
    vcycle<DIM>(p, l + 1, c.b, c.x, done, s);
    hipLaunchKernelGGL(gmg_prolong_kernel<DIM>, dim3(g), dim3(kBlock), 0, s, v.nx, v.ny, v.nz, c.ny, c.nz, c.x,
                       l == 0 ? p->freemask : nullptr, x, done);
    // post-smoothing: the same polynomial from x (r is free again)
    cur = x;
    nxt = t;
    for (int k = 0; k < kGmgNu; ++k) {
        cs = cheb_step(k);
        hipLaunchKernelGGL(sweep, dim3(g), dim3(kBlock), 0, s, L, 1, cur, b, v.dinv, nxt, r, cs.cd,
                           cs.cr, done);
        std::swap(cur, nxt);
    }
    if (cur != x) (void)hipMemcpyAsync(x, cur, 8 * v.n, hipMemcpyDeviceToDevice, s);
}

template <int DIM>
static to_status gmg_setup(Plan* p, hipStream_t s) {
    constexpr int D = Cell<DIM>::D;
    Gmg& G = p->gmg;
    for (int l = 0; l + 1 < G.L; ++l) {
        const GmgLevel& f = G.lv[l];
        GmgLevel& c = G.lv[l + 1];
        hipLaunchKernelGGL(gmg_galerkin_kernel<DIM>, dim3(grid_of(D * c.m)), dim3(kBlock), 0, s, f.nx, f.ny, f.nz,
                           c.nx, c.ny, c.nz, l == 0 ? p->E64 : nullptr, l == 0 ? p->kf64 : nullptr,
                           l == 0 ? p->freemask : nullptr, l == 0 ? nullptr : f.K, c.K);
    }
    for (int l = 1; l + 1 < G.L; ++l) {
        const GmgLevel& v = G.lv[l];
        hipLaunchKernelGGL(gmg_stencil_kernel<DIM>, dim3(grid_of(v.nnode * (DIM == 2 ? 9 : 27))), dim3(kBlock), 0, s,
                           v.nx, v.ny, v.nz, v.nnode, v.K, v.S);
    }
    for (int l = 0; l + 1 < G.L; ++l) {
        const LevelArgs L = level_args(p, l);
        hipLaunchKernelGGL(gmg_diag_kernel<DIM>, dim3(grid_of(G.lv[l].nnode)), dim3(kBlock), 0, s, L, G.lv[l].dinv);
    }
    const GmgLevel& cl = G.lv[G.L - 1];
    const int nc = (int)cl.n;
    hipLaunchKernelGGL(gmg_dense_kernel<DIM>, dim3(grid_of((int64_t)nc * nc)), dim3(kBlock), 0, s, cl.nx, cl.ny,
                       cl.nz, cl.K, nc, G.Ainv);
    hipLaunchKernelGGL(gmg_invert_kernel, dim3(1), dim3(1024), 0, s, G.Ainv, nc);
    TO_HIP(hipGetLastError());
    return TO_OK;
}

template <int DIM>
static to_status solve_gmg(Plan* p, const double* f, double* u, const to_solve_opts& o, to_solve_stats* st,
                           hipStream_t s) {
    Gmg& G = p->gmg;
    to_status r0 = gmg_setup<DIM>(p, s);
    if (r0 != TO_OK) return r0;
    GmgScal* S = G.scal;
    int32_t* done = &S->done;
    const int64_t n = p->info.n;
    double *r = p->v64[0], *z = p->v64[1], *pa = p->v64[2], *pb = p->v64[3], *q = p->v64[4], *rold = p->v64[5];
    double* part = p->partial + (size_t)kMaxCoopBlocks * kPartialWidth;
    unsigned* ctr = p->bar + 12;
    const LevelArgs L0 = level_args(p, 0);
    const int g0 = grid_red(p->info.nnode), gn = grid_red(n);
    if (o.zero_x0)
        hipLaunchKernelGGL(fill_zero_f64_kernel, dim3(gn), dim3(kBlock), 0, s, u, n);
    hipLaunchKernelGGL(fcg_init_kernel, dim3(1), dim3(1), 0, s, S, o.maxit);
    hipLaunchKernelGGL(fcg_residual_kernel<DIM>, dim3(g0), dim3(kBlock), 0, s, L0, f, u, r, part, ctr, S, 1);
    hipLaunchKernelGGL(fcg_tol_kernel, dim3(1), dim3(1), 0, s, S, o.rtol);
    // A batch of kGmgBatch outer iterations, each predicated on S->done and
    // followed by the (predicated) true-residual confirmation, which may
    // reopen the iteration with fresh directions.  The direction buffers
    // alternate with period 2, so every batch after the first has the same
    // launches; the first one starts from p_old = z (finite; beta is 0).
    auto enqueue_batch = [&](bool first, hipStream_t cs) {
        double* pold = first ? z : pb;
        double* pnew = pa;
        double* other = pb;
        for (int k = 0; k < kGmgBatch; ++k) {
            vcycle<DIM>(p, 0, r, z, done, cs);
            hipLaunchKernelGGL(fcg_dots_kernel, dim3(gn), dim3(kBlock), 0, cs, n, r, rold, z, part, ctr, S);
            hipLaunchKernelGGL(fcg_dir_kernel<DIM>, dim3(g0), dim3(kBlock), 0, cs, L0, z, pold, pnew, q, part, ctr, S);
            hipLaunchKernelGGL(fcg_update_kernel, dim3(gn), dim3(kBlock), 0, cs, n, pnew, q, u, r, rold, part, ctr, S);
            hipLaunchKernelGGL(fcg_residual_kernel<DIM>, dim3(g0), dim3(kBlock), 0, cs, L0, f, u, r, part, ctr, S, 2);
            pold = pnew;
            std::swap(pnew, other);
        }
    };
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    TO_HIP(hipStreamIsCapturing(s, &cst));
    const bool capturing = cst != hipStreamCaptureStatusNone;
    if (capturing && o.budget <= 0) {
        set_error("to_solve: a multigrid solve under stream capture needs a budget (to_solve_opts.budget > 0)");
        return TO_EINVAL;
    }
    if (capturing) {
        // the caller records this call into its own graph: the kernels go
        // straight into the capture (no private graph, no stream creation)
        const int nb = (o.budget + kGmgBatch - 1) / kGmgBatch;
        for (int b = 0; b < nb; ++b) enqueue_batch(b == 0, s);
    } else {
        // capture both batch kinds once per (u, f) and replay them
        if (!G.cap) TO_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
        if (G.key_u != u || G.key_f != f || !G.g_first || !G.g_steady) {
            for (hipGraphExec_t* ex : {&G.g_first, &G.g_steady}) {
                if (*ex) { TO_HIP(hipGraphExecDestroy(*ex)); *ex = nullptr; }
            }
            for (int kind = 0; kind < 2; ++kind) {
                TO_HIP(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
                enqueue_batch(kind == 0, G.cap);
                hipGraph_t gr = nullptr;
                hipError_t e = hipStreamEndCapture(G.cap, &gr);
                if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
                e = hipGraphInstantiate(kind == 0 ? &G.g_first : &G.g_steady, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
            }
            G.key_u = u;
            G.key_f = f;
        }
        if (o.budget > 0) {
            // enqueue-only: a fixed number of predicated outer iterations
            const int nb = (o.budget + kGmgBatch - 1) / kGmgBatch;
            for (int b = 0; b < nb; ++b) TO_HIP(hipGraphLaunch(b == 0 ? G.g_first : G.g_steady, s));
        } else {
            // host-checked: read the stop flag after every batch
            const int64_t max_batches = (int64_t)o.maxit / kGmgBatch + kGmgMaxRestarts + 2;
            for (int64_t b = 0; b < max_batches; ++b) {
                TO_HIP(hipGraphLaunch(b == 0 ? G.g_first : G.g_steady, s));
                int32_t h_done = 0;
                TO_HIP(hipMemcpyAsync(&h_done, &S->done, sizeof(int32_t), hipMemcpyDeviceToHost, s));
                TO_HIP(hipStreamSynchronize(s));
                if (h_done) break;
            }
        }
    }
    hipLaunchKernelGGL(fcg_stats_kernel, dim3(1), dim3(1), 0, s, S, st, o.rtol);
    TO_HIP(hipGetLastError());
    return TO_OK;
}

to_status launch_solve_gmg(Plan* p, to_dtype dt, const void* xphys, double penal, const double* f, double* u,
                           const to_solve_opts& o, to_solve_stats* st, hipStream_t s) {
    if (p->gmg.L < 2) {
        set_error("the mesh is too small for a multigrid hierarchy");
        return TO_EUNSUPPORTED;
    }
    // FP64 moduli of the design (the FP32 design promoted for TO_F32)
    to_status r0 = launch_moduli(p, dt, xphys, penal, s, true);
    if (r0 != TO_OK) return r0;
    return p->dim == 2 ? solve_gmg<2>(p, f, u, o, st, s) : solve_gmg<3>(p, f, u, o, st, s);
}

}  // namespace topt
