// Initial state of a run (block PRE.6 of both codes): the uniform design on
// the active set that meets the volume fraction over the whole domain, 1 on
// passive solid and 0 on passive void elements, the physical field equal to
// it, the previous physical field at 1, the constant volume derivative
// 1 / (m volfrac) on active elements (0 on passive ones), and a zero
// displacement.
#include "common.h"

namespace topt {

template <typename T>
__global__ __launch_bounds__(kBlock) void init_state_kernel(int64_t m, int64_t n, const uint8_t* __restrict__ pas,
                                                            double volfrac, int64_t n_act, int64_t n_solid,
                                                            int64_t n_void, T* __restrict__ x, T* __restrict__ xphys,
                                                            T* __restrict__ xold, T* __restrict__ dv,
                                                            double* __restrict__ u) {
    // the codes' value: (volfrac (m - |P0|) - |P1|) / |A|, in FP64, each
    // operation rounded on its own (no fused multiply-add), as the codes do
#pragma clang fp contract(off)
    const double xa = (volfrac * (double)(m - n_void) - (double)n_solid) / (double)n_act;
    const double dva = 1.0 / (double)m / volfrac;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += stride) {
        const uint8_t c = pas[e];
        const double v = c == TO_ACTIVE ? xa : (c == TO_SOLID ? 1.0 : 0.0);
        x[e] = (T)v;
        if (xphys) xphys[e] = (T)v;
        if (xold) xold[e] = (T)1.0;
        if (dv) dv[e] = (T)(c == TO_ACTIVE ? dva : 0.0);
    }
    if (u)
        for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += stride) u[i] = 0.0;
}

to_status launch_init_state(Plan* p, to_dtype dt, double volfrac, void* x, void* xphys, void* xold, void* dv,
                            double* u, hipStream_t s) {
    const int64_t m = p->info.m, n = p->info.n;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (std::max(m, u ? n : 0) + kBlock - 1) / kBlock));
    if (dt == TO_F64)
        hipLaunchKernelGGL(init_state_kernel<double>, dim3(blocks), dim3(kBlock), 0, s, m, n, p->passive, volfrac,
                           p->info.n_active, p->info.n_solid, p->info.n_void, (double*)x, (double*)xphys,
                           (double*)xold, (double*)dv, u);
    else
        hipLaunchKernelGGL(init_state_kernel<float>, dim3(blocks), dim3(kBlock), 0, s, m, n, p->passive, volfrac,
                           p->info.n_active, p->info.n_solid, p->info.n_void, (float*)x, (float*)xphys, (float*)xold,
                           (float*)dv, u);
    TO_HIP(hipGetLastError());
    return TO_OK;
}

}  // namespace topt
