// Compliance sensitivities, eq. (7) (block RL.3 of both codes):
//   dc_e = -p (E0 - Emin) xphys_e^(p-1) u_e^T Ke u_e   (0 on passive elements)
// and the compliance c = f^T u (a deterministic two-level FP64 reduction).
//
// One thread per element: its DOFs follow from the element index (structured
// grid, corner order of Fig. 1b), u_e is gathered in FP64 (adjacent threads
// read adjacent nodes), and Ke (d x d, FP64) is read with wave-uniform
// indices, i.e. through the scalar cache.
#include "common.h"

namespace topt {

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void sensitivity_kernel(int nx, int ny, int nz, const T* __restrict__ xphys,
                                                              const uint8_t* __restrict__ pas,
                                                              const double* __restrict__ u,
                                                              const double* __restrict__ ke, double penal,
                                                              double E0, double Emin, T* __restrict__ dc) {
    constexpr int NC = DIM == 2 ? 4 : 8, D = DIM * NC;
    constexpr int CY[8] = {1, 1, 0, 0, 1, 1, 0, 0};
    constexpr int CX[8] = {0, 1, 1, 0, 0, 1, 1, 0};
    constexpr int CZ[8] = {0, 0, 0, 0, 1, 1, 1, 1};
    const int64_t m = (int64_t)nx * ny * (DIM == 2 ? 1 : nz);
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock) {
        const int iy = (int)(e % ny);
        const int64_t rest = e / ny;
        const int ix = DIM == 2 ? (int)rest : (int)(rest / nz);
        const int iz = DIM == 2 ? 0 : (int)(rest % nz);
        double ue[D];
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            const int64_t q = DIM == 2 ? (iy + CY[b]) + (int64_t)(ny + 1) * (ix + CX[b])
                                       : (iy + CY[b]) + (int64_t)(ny + 1) * ((iz + CZ[b]) + (int64_t)(nz + 1) * (ix + CX[b]));
#pragma unroll
            for (int c = 0; c < DIM; ++c) ue[b * DIM + c] = u[DIM * q + c];
        }
        double ce = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double k_u = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) k_u += ke[i * D + j] * ue[j];
            ce += ue[i] * k_u;
        }
        double out = 0.0;
        if (pas[e] == TO_ACTIVE) out = -penal * (E0 - Emin) * pow((double)xphys[e], penal - 1.0) * ce;
        dc[e] = (T)out;
    }
}

// c = f^T u: block partials, then the last block to finish sums them in order.
__global__ __launch_bounds__(kBlock) void dot_kernel(int64_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b, double* partial,
                                                     unsigned* counter, double* out) {
    __shared__ double sh[kWaves];
    __shared__ int last;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        s += a[i] * b[i];
    s = block_sum(s, sh);
    // partials are exchanged with device-coherent accesses, so the arrival
    // needs only the block's own stores to have completed (no L2 writeback)
    if (threadIdx.x == 0) {
        st_dev(&partial[blockIdx.x], s);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        unsigned done = atomicAdd(counter, 1u);
        last = done == gridDim.x - 1;
    }
    __syncthreads();
    if (last) {
        double t = 0.0;
        for (int b2 = threadIdx.x; b2 < (int)gridDim.x; b2 += kBlock) t += ld_acq(&partial[b2]);
        t = block_sum(t, sh);
        if (threadIdx.x == 0) {
            *out = t;
            st_dev(counter, 0u);
        }
    }
}

to_status launch_sensitivity(Plan* p, to_dtype dt, const void* xphys, const double* u, const double* f,
                             double penal, void* dc, double* c, hipStream_t s) {
    const int64_t m = p->info.m;
    const int blocks = (int)std::min<int64_t>(8192, (m + kBlock - 1) / kBlock);
    if (p->dim == 2) {
        if (dt == TO_F64)
            hipLaunchKernelGGL((sensitivity_kernel<2, double>), dim3(blocks), dim3(kBlock), 0, s, p->nelx, p->nely, 1,
                               (const double*)xphys, p->passive, u, p->kf64, penal, p->E0, p->Emin, (double*)dc);
        else
            hipLaunchKernelGGL((sensitivity_kernel<2, float>), dim3(blocks), dim3(kBlock), 0, s, p->nelx, p->nely, 1,
                               (const float*)xphys, p->passive, u, p->kf64, penal, p->E0, p->Emin, (float*)dc);
    } else {
        if (dt == TO_F64)
            hipLaunchKernelGGL((sensitivity_kernel<3, double>), dim3(blocks), dim3(kBlock), 0, s, p->nelx, p->nely,
                               p->nelz, (const double*)xphys, p->passive, u, p->kf64, penal, p->E0, p->Emin,
                               (double*)dc);
        else
            hipLaunchKernelGGL((sensitivity_kernel<3, float>), dim3(blocks), dim3(kBlock), 0, s, p->nelx, p->nely,
                               p->nelz, (const float*)xphys, p->passive, u, p->kf64, penal, p->E0, p->Emin,
                               (float*)dc);
    }
    TO_HIP(hipGetLastError());
    if (f && c) {
        const int64_t n = p->info.n;
        // 256 blocks: the arrivals on the last-block counter serialise at one address
        const int nb = (int)std::min<int64_t>(256, (n + kBlock - 1) / kBlock);
        // partial slots: the second region of the partial buffer; counter: bar[8]
        double* part = p->partial + (size_t)kMaxCoopBlocks * kPartialWidth;
        hipLaunchKernelGGL(dot_kernel, dim3(nb), dim3(kBlock), 0, s, n, f, u, part, p->bar + 8, c);
        TO_HIP(hipGetLastError());
    }
    return TO_OK;
}

}  // namespace topt
