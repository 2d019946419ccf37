// Stiffness assembly on the reduced index set (block RL.2 of both codes,
// eq. (6) and (14)): K^(s)[s] = sum over t in seg(s) of Ke[perm_t mod d~] *
// E[perm_t div d~], in ascending t (the plan's fixed order), no atomics.
//
// The SIMP moduli E_e = Emin + xphys_e^p (E0 - Emin) are computed once per
// element by a first kernel (so the pow is not repeated for each of the d~
// pairs of an element).  The segmented reduction runs one slot per thread:
// the slots of a wave are consecutive, so their perm ranges form one
// contiguous stretch of memory and the wave's reads coalesce in L1/L2; Ke
// (d~ values) is staged in LDS.
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

template <typename T, int DT, int NT>
static void assemble_nt(Plan* p, int64_t nnz, const T* ke, const T* E, T* kval, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>(1 << 16, (nnz + NT - 1) / NT);
    hipLaunchKernelGGL((assemble_kernel<T, DT, NT>), dim3(blocks), dim3(NT), 0, s, nnz, p->seg_ptr, p->perm, ke, E, kval);
}

template <typename T, int DT>
static void assemble_t(Plan* p, int64_t nnz, const T* ke, const T* E, T* kval, hipStream_t s) {
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

}  // namespace topt
