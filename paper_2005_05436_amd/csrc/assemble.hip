// Stiffness assembly on the reduced index set (block RL.2 of both codes,
// eq. (6) and (14)): K^(s)[s] = sum over t in seg(s) of Ke[perm_t mod d~] *
// E[perm_t div d~], in ascending t (the plan's fixed order), no atomics.
//
// The SIMP moduli E_e = Emin + xphys_e^p (E0 - Emin) are computed once per
// element by a first kernel (so the pow is not repeated for each of the d~
// pairs of an element).  The segmented reduction runs one slot per thread:
// the slots of a wave are consecutive, so their perm ranges form one
// contiguous stretch of memory and the wave's reads coalesce in L1/L2; Ke
// (d~ values) is staged in LDS.  A second kernel forms the same sums from the
// grid instead of the permutation, one thread per slot (the plan's tuning
// chooses).
#include <cstring>

#include "common.h"

namespace topt {

template <typename TX, typename T>
__global__ __launch_bounds__(kBlock) void moduli_kernel(int64_t m, const TX* __restrict__ x, T E0, T Emin,
                                                         T penal, T* __restrict__ E) {
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock)
        E[e] = Emin + simp_pow((T)x[e], penal) * (E0 - Emin);
}

template <typename T, int DT, int NT>
__global__ __launch_bounds__(NT) void assemble_kernel(int64_t nnz, const int32_t* __restrict__ seg,
                                                       const int32_t* __restrict__ perm,
                                                       const T* __restrict__ ke, const T* __restrict__ E,
                                                       T* __restrict__ kval) {
    __shared__ T ke_s[DT];
    for (int i = threadIdx.x; i < DT; i += NT) ke_s[i] = ke[i];
    __syncthreads();
    // a slot has at most MC contributions on a structured grid (the elements
    // that share both nodes: 4 in 2D, 8 in 3D); their perm and E loads are all
    // issued before the sum, which still runs in ascending t
    constexpr int MC = DT == 36 ? 4 : 8;
    for (int64_t s = blockIdx.x * (int64_t)NT + threadIdx.x; s < nnz; s += (int64_t)gridDim.x * NT) {
        const int32_t a = seg[s], b = seg[s + 1];
        uint32_t pk[MC];
        T ev[MC];
#pragma unroll
        for (int u = 0; u < MC; ++u) pk[u] = a + u < b ? (uint32_t)perm[a + u] : 0u;
#pragma unroll
        for (int u = 0; u < MC; ++u) ev[u] = a + u < b ? E[pk[u] / DT] : T(0);
        T acc = T(0);
#pragma unroll
        for (int u = 0; u < MC; ++u)
            if (a + u < b) acc += ke_s[pk[u] - (pk[u] / DT) * DT] * ev[u];
        for (int32_t t = a + MC; t < b; ++t) {             // longer segments (not produced by the plan)
            const uint32_t q = (uint32_t)perm[t];
            const uint32_t e = q / DT;
            acc += ke_s[q - e * DT] * E[e];
        }
        kval[s] = acc;
    }
}

// The same sums without the permutation.  On the structured grid the pairs t
// that land in slot (r, c) are those of the elements holding both nodes,
// and t = e * d~ + (local pair) grows with the element index e, so visiting
// those elements in ascending index and taking Ke at the lower-triangle
// position of the local pair adds the same terms in the same order as the
// segmented sum: the two kernels give identical values.  Reads: row_ptr and
// col_idx (4 B per slot) instead of seg_ptr and perm (about 12 B per slot),
// and the gathers of E.
// Node coordinates of a node index (32-bit: the plan keeps n below 2^31).
template <int DIM>
__device__ __forceinline__ void node_coords(uint32_t q, uint32_t ny1, uint32_t nz1, int& y, int& x, int& z) {
    const uint32_t rest = q / ny1;
    y = (int)(q - rest * ny1);
    if (DIM == 2) { x = (int)rest; z = 0; }
    else { const uint32_t xx = rest / nz1; x = (int)xx; z = (int)(rest - xx * nz1); }
}

// Value of slot (r, c), row r at node coordinates (iy, ix, iz) and DOF
// component cr.
template <typename T, int DIM>
__device__ __forceinline__ T grid_slot_value(int iy, int ix, int iz, int cr, int32_t c, int nelx, int nely, int nelz,
                                             const T* ke_s, const T* __restrict__ E) {
    constexpr int D = DIM == 2 ? 8 : 24;
    const uint32_t qc = (uint32_t)c / DIM;
    const int cc = (int)((uint32_t)c - qc * DIM);
    int jy, jx, jz;
    node_coords<DIM>(qc, nely + 1, nelz + 1, jy, jx, jz);
    // elements holding both nodes: e.x in [max(ix, jx) - 1, min(ix, jx)] within the
    // grid, likewise y and z; ascending element index = x outer, then z, then y
    const int x0 = max(max(ix, jx) - 1, 0), x1 = min(min(ix, jx), nelx - 1);
    const int y0 = max(max(iy, jy) - 1, 0), y1 = min(min(iy, jy), nely - 1);
    const int z0 = DIM == 2 ? 0 : max(max(iz, jz) - 1, 0), z1 = DIM == 2 ? 0 : min(min(iz, jz), nelz - 1);
    T acc = T(0);
    for (int ex = x0; ex <= x1; ++ex)
        for (int ez = z0; ez <= z1; ++ez)
            for (int ey = y0; ey <= y1; ++ey) {
                // corner of a node at offset (dy, dx, dz) in {0,1}^3 from the element's
                // origin: corners 0..3 at (1,0), (1,1), (0,1), (0,0) in (y, x), +4 at z + 1
                const int dyr = iy - ey, dxr = ix - ex, dyc = jy - ey, dxc = jx - ex;
                int br = dyr ? dxr : 3 - dxr, bc = dyc ? dxc : 3 - dxc;
                if (DIM == 3) { br += 4 * (iz - ez); bc += 4 * (jz - ez); }
                const int a = DIM * br + cr, b = DIM * bc + cc;
                const int j = min(a, b), i = max(a, b);
                const int k = j * D - ((j * (j - 1)) >> 1) + (i - j);
                const uint32_t e = (uint32_t)ey + (uint32_t)nely * (uint32_t)(DIM == 2 ? ex : ez + nelz * ex);
                acc += ke_s[k] * E[e];
            }
    return acc;
}

// One thread per slot: a block takes RB consecutive rows, stages their
// row_ptr entries and node coordinates in LDS, and every thread finds the row of its slot by a
// binary search there, so the slots (and the stores of kval) of a wave are
// consecutive.
template <typename T, int DIM, int NT>
__global__ __launch_bounds__(NT) void assemble_grid_kernel(int nelx, int nely, int nelz, int64_t n,
                                                            const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const T* __restrict__ ke, const T* __restrict__ E,
                                                            T* __restrict__ kval) {
    constexpr int D = DIM == 2 ? 8 : 24, DT = D * (D + 1) / 2;
    constexpr int RB = NT / (DIM == 2 ? 8 : 32);   // about 9.5 (2D) and 38 (3D) slots per row
    __shared__ T ke_s[DT];
    __shared__ int32_t rps[RB + 1];
    __shared__ int32_t ry[RB], rx[RB], rz[RB];
    for (int i = threadIdx.x; i < DT; i += NT) ke_s[i] = ke[i];
    for (int64_t R0 = blockIdx.x * (int64_t)RB; R0 < n; R0 += (int64_t)gridDim.x * RB) {
        const int nr = (int)std::min<int64_t>(RB, n - R0);
        __syncthreads();   // ke_s written; the previous group's rows no longer read
        if (threadIdx.x <= nr) rps[threadIdx.x] = rp[R0 + threadIdx.x];
        if (threadIdx.x < nr) {
            const uint32_t r = (uint32_t)(R0 + threadIdx.x);
            int y, x, z;
            node_coords<DIM>(r / DIM, nely + 1, nelz + 1, y, x, z);
            ry[threadIdx.x] = y;
            rx[threadIdx.x] = x;
            rz[threadIdx.x] = z;
        }
        __syncthreads();
        const int32_t S0 = rps[0], S1 = rps[nr];
        for (int32_t s = S0 + (int32_t)threadIdx.x; s < S1; s += NT) {
            int lo = 0, hi = nr;   // rps[lo] <= s < rps[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (rps[mid] <= s) lo = mid;
                else hi = mid;
            }
            const int cr = (int)((uint32_t)(R0 + lo) % DIM);
            kval[s] = grid_slot_value<T, DIM>(ry[lo], rx[lo], rz[lo], cr, ci[s], nelx, nely, nelz, ke_s, E);
        }
    }
}

// 2D, one thread per node: the node's two rows of K^(s) (up to 9 + 10
// slots) from the moduli of the (up to four) elements around it.  Row 2n
// holds the columns of the lower neighbours (iy-1, ix-1), (iy, ix-1),
// (iy+1, ix-1), (iy-1, ix) (both components each) and 2n itself; row 2n+1
// the same and 2n+1: the plan's ascending column order.  A slot's value
// sums, over the elements holding both nodes in ascending element index,
// Ke at the lower-triangle position of the local pair times E, so it equals
// the segmented sum bit for bit.  Every index is resolved at compile time
// except the boundary tests.  The values of a block's nodes are gathered in
// LDS and written out as one contiguous, coalesced stretch of kval (a
// block's nodes are consecutive, so their rows are).
template <typename T, int NT>
__device__ __forceinline__ void node2d_body(int nelx, int nely, int64_t nnode, const int32_t* __restrict__ rp,
                                            const T* __restrict__ ke, const T* __restrict__ E,
                                            T* __restrict__ kval, int bid, int nb) {
    constexpr int D = 8;
    __shared__ T ke_s[36];
    __shared__ T out_s[NT * 19];
    for (int i = threadIdx.x; i < 36; i += NT) ke_s[i] = ke[i];
    const int ny1 = nely + 1;
    for (int64_t n0 = bid * (int64_t)NT; n0 < nnode; n0 += (int64_t)nb * NT) {
        const int64_t nend = n0 + NT < nnode ? n0 + NT : nnode;
        const int64_t nd = n0 + threadIdx.x;
        __syncthreads();   // ke_s written; the previous stretch written out
        const int32_t base = rp[2 * n0], top = rp[2 * nend];
        if (nd < nend) {
            const int ix = (int)((uint32_t)nd / (uint32_t)ny1), iy = (int)nd - ix * ny1;
            // moduli of the elements (iy - 1 + ay, ix - 1 + bx), ay, bx in {0, 1}
            T Ev[2][2];
            bool ok[2][2];
#pragma unroll
            for (int ay = 0; ay < 2; ++ay)
#pragma unroll
                for (int bx = 0; bx < 2; ++bx) {
                    const int ey = iy - 1 + ay, ex = ix - 1 + bx;
                    ok[ay][bx] = ey >= 0 && ey < nely && ex >= 0 && ex < nelx;
                    Ev[ay][bx] = ok[ay][bx] ? E[ey + (int64_t)nely * ex] : T(0);
                }
            int pos = rp[2 * nd] - base;
#pragma unroll
            for (int cr = 0; cr < 2; ++cr)
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    // lower neighbour q at offset (a, b) in (y, x), ascending node index
                    const int a = q < 3 ? q - 1 : q - 4, b = q < 3 ? -1 : 0;
                    if (iy + a < 0 || iy + a > nely || ix + b < 0) continue;
#pragma unroll
                    for (int cc = 0; cc < 2; ++cc) {
                        if (q == 4 && cc > cr) continue;          // upper triangle of the diagonal block
                        T acc = T(0);
                        // shared elements, ascending element index: x outer, then y
#pragma unroll
                        for (int bx = 0; bx < 2; ++bx) {
                            if (b == -1 && bx == 1) continue;
#pragma unroll
                            for (int ay = 0; ay < 2; ++ay) {
                                if ((a == -1 && ay == 1) || (a == 1 && ay == 0)) continue;
                                if (!ok[ay][bx]) continue;
                                const int dyr = 1 - ay, dxr = 1 - bx;              // this node in the element
                                const int dyc = 1 - ay + a, dxc = 1 - bx + b;      // the neighbour
                                const int br = dyr ? dxr : 3 - dxr, bc = dyc ? dxc : 3 - dxc;
                                const int la = 2 * br + cr, lb = 2 * bc + cc;
                                const int j = la < lb ? la : lb, i = la < lb ? lb : la;
                                const int k = j * D - ((j * (j - 1)) >> 1) + (i - j);
                                acc += ke_s[k] * Ev[ay][bx];
                            }
                        }
                        out_s[pos++] = acc;
                    }
                }
        }
        __syncthreads();
        for (int32_t i = (int32_t)threadIdx.x; i < top - base; i += NT) kval[base + i] = out_s[i];
    }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void assemble_node2d_kernel(int nelx, int nely, int64_t nnode,
                                                              const int32_t* __restrict__ rp,
                                                              const T* __restrict__ ke, const T* __restrict__ E,
                                                              T* __restrict__ kval) {
    node2d_body<T, NT>(nelx, nely, nnode, rp, ke, E, kval, blockIdx.x, gridDim.x);
}

template <typename T, int NT>
static void assemble_node2d_nt(Plan* p, const T* ke, const T* E, T* kval, hipStream_t s) {
    const int64_t nn = p->info.nnode;
    const int blocks = (int)std::min<int64_t>(1 << 16, (nn + NT - 1) / NT);
    hipLaunchKernelGGL((assemble_node2d_kernel<T, NT>), dim3(blocks), dim3(NT), 0, s, p->nelx, p->nely, nn,
                       p->row_ptr, ke, E, kval);
}

template <typename T, int DIM, int NT>
static void assemble_grid_nt(Plan* p, const T* ke, const T* E, T* kval, hipStream_t s) {
    constexpr int RB = NT / (DIM == 2 ? 8 : 32);
    const int64_t n = p->info.n;
    const int blocks = (int)std::min<int64_t>(1 << 16, (n + RB - 1) / RB);
    hipLaunchKernelGGL((assemble_grid_kernel<T, DIM, NT>), dim3(blocks), dim3(NT), 0, s, p->nelx, p->nely,
                       DIM == 2 ? 1 : p->nelz, n, p->row_ptr, p->col_idx, ke, E, kval);
}

template <typename T, int DT, int NT>
static void assemble_nt(Plan* p, int64_t nnz, const T* ke, const T* E, T* kval, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>(1 << 16, (nnz + NT - 1) / NT);
    hipLaunchKernelGGL((assemble_kernel<T, DT, NT>), dim3(blocks), dim3(NT), 0, s, nnz, p->seg_ptr, p->perm, ke, E, kval);
}

template <typename T, int DT>
static void assemble_t(Plan* p, int64_t nnz, const T* ke, const T* E, T* kval, hipStream_t s) {
    constexpr int DIM = DT == 36 ? 2 : 3;
    if (DIM == 2 && p->tune.asm_rows == 2) {
        switch (p->tune.asm_block) {
        case 128: assemble_node2d_nt<T, 128>(p, ke, E, kval, s); break;
        case 512: assemble_node2d_nt<T, 512>(p, ke, E, kval, s); break;
        default: assemble_node2d_nt<T, 256>(p, ke, E, kval, s); break;
        }
        return;
    }
    if (p->tune.asm_rows) {
        switch (p->tune.asm_block) {
        case 128: assemble_grid_nt<T, DIM, 128>(p, ke, E, kval, s); break;
        case 512: assemble_grid_nt<T, DIM, 512>(p, ke, E, kval, s); break;
        default: assemble_grid_nt<T, DIM, 256>(p, ke, E, kval, s); break;
        }
        return;
    }
    switch (p->tune.asm_block) {
    case 128: assemble_nt<T, DT, 128>(p, nnz, ke, E, kval, s); break;
    case 512: assemble_nt<T, DT, 512>(p, nnz, ke, E, kval, s); break;
    default: assemble_nt<T, DT, 256>(p, nnz, ke, E, kval, s); break;
    }
}

// dt = the dtype of xphys.  TO_F64: E64 from double x.  TO_F32: E32 from float
// x, and with `also64` E64 from the same float x promoted (the FP64 operator
// of the mixed-precision refinement is built from the design the FP32 path used).
to_status launch_moduli(Plan* p, to_dtype dt, const void* xphys, double penal, hipStream_t s, bool also64) {
    const int64_t m = p->info.m;
    const int blocks = (int)std::min<int64_t>(4096, (m + kBlock - 1) / kBlock);
    if (dt == TO_F64) {
        hipLaunchKernelGGL((moduli_kernel<double, double>), dim3(blocks), dim3(kBlock), 0, s, m,
                           (const double*)xphys, p->E0, p->Emin, penal, p->E64);
    } else {
        hipLaunchKernelGGL((moduli_kernel<float, float>), dim3(blocks), dim3(kBlock), 0, s, m,
                           (const float*)xphys, (float)p->E0, (float)p->Emin, (float)penal, p->E32);
        if (also64)
            hipLaunchKernelGGL((moduli_kernel<float, double>), dim3(blocks), dim3(kBlock), 0, s, m,
                               (const float*)xphys, p->E0, p->Emin, penal, p->E64);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

to_status launch_assemble(Plan* p, to_dtype dt, const void* xphys, double penal, void* kval, hipStream_t s) {
    to_status st = launch_moduli(p, dt, xphys, penal, s, false);
    if (st != TO_OK) return st;
    return launch_assemble_from_moduli(p, dt, kval, s);
}

// The sums alone, from the moduli already in the plan's E array.
to_status launch_assemble_from_moduli(Plan* p, to_dtype dt, void* kval, hipStream_t s) {
    const int64_t nnz = p->info.nnz_lower;
    if (dt == TO_F64) {
        if (p->dim == 2) assemble_t<double, 36>(p, nnz, p->ke64, p->E64, (double*)kval, s);
        else assemble_t<double, 300>(p, nnz, p->ke64, p->E64, (double*)kval, s);
    } else {
        if (p->dim == 2) assemble_t<float, 36>(p, nnz, p->ke32, p->E32, (float*)kval, s);
        else assemble_t<float, 300>(p, nnz, p->ke32, p->E32, (float*)kval, s);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

// --- batches -----------------------------------------------------------------
// Arguments of one design: its moduli (E in the field type, and with the
// FP64 operator of the mixed solve also E64) and, for 2D designs, the
// node-centric sums.
template <typename T>
struct AsmArgs {
    int nelx, nely;
    int64_t m, nnode;
    const T* x;
    T* E;
    double* E64;
    const int32_t* rp;
    const T* ke;
    T* kval;
    double E0, Emin;
};

size_t asm_args_bytes() {
    static_assert(sizeof(AsmArgs<double>) == sizeof(AsmArgs<float>), "one table layout for both types");
    return sizeof(AsmArgs<double>);
}

void asm_args_fill(Plan* p, to_dtype dt, const void* xphys, void* kval, void* dst) {
    if (dt == TO_F64) {
        const AsmArgs<double> A{p->nelx, p->nely, p->info.m, p->info.nnode, (const double*)xphys, p->E64, p->E64,
                                p->row_ptr, p->ke64, (double*)kval, p->E0, p->Emin};
        std::memcpy(dst, &A, sizeof A);
    } else {
        const AsmArgs<float> A{p->nelx, p->nely, p->info.m, p->info.nnode, (const float*)xphys, p->E32, p->E64,
                               p->row_ptr, p->ke32, (float*)kval, p->E0, p->Emin};
        std::memcpy(dst, &A, sizeof A);
    }
}

// The moduli of every design (same arithmetic as moduli_kernel: the field
// type's pow and constants; with ALSO64 the FP64 moduli from the same x).
template <typename T, bool ALSO64>
__global__ __launch_bounds__(kBlock) void moduli_batch_kernel(const AsmArgs<T>* __restrict__ tab,
                                                               const double* __restrict__ dyn, int stride,
                                                               const int32_t* __restrict__ inst,
                                                               const int32_t* __restrict__ first,
                                                               const int32_t* __restrict__ count) {
    const int i = __builtin_amdgcn_readfirstlane(inst[blockIdx.x]);
    const AsmArgs<T> A = tab[i];
    const double penal = dyn[(size_t)stride * i + 4];
    const int bid = (int)blockIdx.x - first[i], nb = count[i];
    const T E0 = (T)A.E0, Emin = (T)A.Emin, pt = (T)penal;
    for (int64_t e = bid * (int64_t)kBlock + threadIdx.x; e < A.m; e += (int64_t)nb * kBlock) {
        const T x = A.x[e];
        A.E[e] = Emin + simp_pow(x, pt) * (E0 - Emin);
        if (ALSO64) A.E64[e] = A.Emin + simp_pow((double)x, penal) * (A.E0 - A.Emin);
    }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void assemble_node2d_batch_kernel(const AsmArgs<T>* __restrict__ tab,
                                                                    const int32_t* __restrict__ inst,
                                                                    const int32_t* __restrict__ first,
                                                                    const int32_t* __restrict__ count) {
    const int i = __builtin_amdgcn_readfirstlane(inst[blockIdx.x]);
    const AsmArgs<T> A = tab[i];
    node2d_body<T, NT>(A.nelx, A.nely, A.nnode, A.rp, A.ke, A.E, A.kval, (int)blockIdx.x - first[i], count[i]);
}

to_status launch_moduli_batch(to_dtype dt, const void* tab, const double* dyn, int dyn_stride, const BatchMap& mp,
                              bool also64, hipStream_t s) {
    if (dt == TO_F64)
        hipLaunchKernelGGL((moduli_batch_kernel<double, false>), dim3(mp.blocks), dim3(kBlock), 0, s,
                           (const AsmArgs<double>*)tab, dyn, dyn_stride, mp.inst, mp.first, mp.count);
    else if (also64)
        hipLaunchKernelGGL((moduli_batch_kernel<float, true>), dim3(mp.blocks), dim3(kBlock), 0, s,
                           (const AsmArgs<float>*)tab, dyn, dyn_stride, mp.inst, mp.first, mp.count);
    else
        hipLaunchKernelGGL((moduli_batch_kernel<float, false>), dim3(mp.blocks), dim3(kBlock), 0, s,
                           (const AsmArgs<float>*)tab, dyn, dyn_stride, mp.inst, mp.first, mp.count);
    TO_HIP(hipGetLastError());
    return TO_OK;
}

// 2D designs: the node-centric sums of every design in one launch (bit-identical
// to every other assembly kernel of this file).
to_status launch_assemble_batch2d(to_dtype dt, const void* tab, const BatchMap& mp, hipStream_t s) {
    if (dt == TO_F64)
        hipLaunchKernelGGL((assemble_node2d_batch_kernel<double, kAsmBatchBlock>), dim3(mp.blocks),
                           dim3(kAsmBatchBlock), 0, s, (const AsmArgs<double>*)tab, mp.inst, mp.first, mp.count);
    else
        hipLaunchKernelGGL((assemble_node2d_batch_kernel<float, kAsmBatchBlock>), dim3(mp.blocks),
                           dim3(kAsmBatchBlock), 0, s, (const AsmArgs<float>*)tab, mp.inst, mp.first, mp.count);
    TO_HIP(hipGetLastError());
    return TO_OK;
}

}  // namespace topt
