// Compliance sensitivities, eq. (7) (block RL.3 of both codes):
//   dc_e = -p (E0 - Emin) xphys_e^(p-1) u_e^T Ke u_e   (0 on passive elements)
// and the compliance c = f^T u (a deterministic two-level FP64 reduction).
//
// One thread per element: its DOFs follow from the element index (structured
// grid, corner order of Fig. 1b), u_e is gathered in FP64 (adjacent threads
// read adjacent nodes), and Ke (d x d, FP64) is read with wave-uniform
// indices, i.e. through the scalar cache.
#include <cstring>
#include <mutex>

#include "common.h"

namespace topt {

// Words of the plan's barrier array used by the compliance sum: the top
// arrival counter and kDotGroups group counters on separate cache lines
// (clear of the grid barrier's words).
constexpr int kDotTop = 8, kDotGroup0 = 576, kDotGroupStride = 16, kDotGroups = 16;
// Blocks of a launch with the compliance sum, and the counter words it uses.
constexpr int kSensMaxBlocks = 1024;
constexpr int kSensBarWords = kDotGroup0 + kDotGroupStride * kDotGroups;
constexpr int kMaxDevices = 64;

// Arguments of one design's launch (penal is passed beside them: in a batch
// it is read from the design's device scalars).
template <typename T>
struct SensArgs {
    int nx, ny, nz;
    const T* xphys;
    const uint8_t* pas;
    const double* u;
    const double* ke;
    double E0, Emin;
    T* dc;
    const double* f;        // nullptr: no compliance sum
    int64_t n;
    double* partial;
    unsigned* bar;
    double* c_out;
};

// The work of block `bid` of the `nb` blocks given to one design.  With f
// given, the same blocks also sum c = f^T u: block partials, a two-level
// arrival (group counters, then the top counter, so no more than nb / 16
// arrivals meet at one address), and the last block sums the partials in
// block order.
template <int DIM, typename T>
__device__ __forceinline__ void sens_body(const SensArgs<T>& A, double penal, int bid, int nb) {
    constexpr int NC = DIM == 2 ? 4 : 8, D = DIM * NC;
    constexpr int CY[8] = {1, 1, 0, 0, 1, 1, 0, 0};
    constexpr int CX[8] = {0, 1, 1, 0, 0, 1, 1, 0};
    constexpr int CZ[8] = {0, 0, 0, 0, 1, 1, 1, 1};
    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const T* __restrict__ xphys = A.xphys;
    const uint8_t* __restrict__ pas = A.pas;
    const double* __restrict__ u = A.u;
    const double* __restrict__ ke = A.ke;
    const double E0 = A.E0, Emin = A.Emin;
    T* __restrict__ dc = A.dc;
    const int64_t m = (int64_t)nx * ny * (DIM == 2 ? 1 : nz);
    for (int64_t e = bid * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)nb * kBlock) {
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
            for (int j = 0; j < D; ++j) k_u += ld_const(ke + i * D + j) * ue[j];
            ce += ue[i] * k_u;
        }
        double out = 0.0;
        if (pas[e] == TO_ACTIVE) out = -penal * (E0 - Emin) * pow((double)xphys[e], penal - 1.0) * ce;
        dc[e] = (T)out;
    }
    const double* __restrict__ f = A.f;
    if (f == nullptr) return;
    const int64_t n = A.n;
    double* partial = A.partial;
    unsigned* bar = A.bar;
    __shared__ double sh[kWaves];
    __shared__ int last;
    double sd = 0.0;
    for (int64_t i = bid * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)nb * kBlock) sd += f[i] * u[i];
    sd = block_sum(sd, sh);
    // partials are exchanged with device-coherent accesses, so an arrival
    // needs only the block's own stores to have completed (no L2 writeback)
    if (threadIdx.x == 0) {
        st_dev(&partial[bid], sd);
        wait_stores();
        const unsigned G = nb < kDotGroups ? (unsigned)nb : (unsigned)kDotGroups;
        const unsigned g = (unsigned)bid % G;
        const unsigned ng = (unsigned)nb / G + (g < (unsigned)nb % G ? 1u : 0u);
        unsigned* grp = &bar[kDotGroup0 + kDotGroupStride * g];
        int is_last = 0;
        if (atomicAdd(grp, 1u) == ng - 1) {
            st_dev(grp, 0u);
            is_last = atomicAdd(&bar[kDotTop], 1u) == G - 1;
        }
        last = is_last;
    }
    __syncthreads();
    if (last) {
        double t = 0.0;
        for (int b2 = threadIdx.x; b2 < nb; b2 += kBlock) t += ld_acq(&partial[b2]);
        t = block_sum(t, sh);
        if (threadIdx.x == 0) {
            *A.c_out = t;
            st_dev(&bar[kDotTop], 0u);
        }
    }
}

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void sensitivity_kernel(SensArgs<T> A, double penal) {
    sens_body<DIM, T>(A, penal, blockIdx.x, gridDim.x);
}

// A batch: block b works for design inst[b] as block b - first[inst] of
// count[inst]; penal is the design's device scalar dyn[stride * inst + 4].
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void sensitivity_batch_kernel(const SensArgs<T>* __restrict__ tab,
                                                                    const double* __restrict__ dyn, int stride,
                                                                    const int32_t* __restrict__ inst,
                                                                    const int32_t* __restrict__ first,
                                                                    const int32_t* __restrict__ count) {
    const int i = __builtin_amdgcn_readfirstlane(inst[blockIdx.x]);
    const SensArgs<T> A = tab[i];
    sens_body<DIM, T>(A, dyn[(size_t)stride * i + 4], (int)blockIdx.x - first[i], count[i]);
}

// The launch itself, with the scratch (block partials, arrival counters)
// passed in: the plan's own region, or the per-device static array below.
// Blocks of the launch: with the compliance sum at most kSensMaxBlocks (64
// arrivals per group counter, one partial per block).
static int sens_blocks(const Plan* p, bool dot) {
    const int64_t work = dot ? std::max(p->info.m, p->info.n) : p->info.m;
    return (int)std::max<int64_t>(1, std::min<int64_t>(dot ? kSensMaxBlocks : 8192, (work + kBlock - 1) / kBlock));
}

template <typename T>
static SensArgs<T> sens_args(Plan* p, const void* xphys, const double* u, const double* f, void* dc, double* c,
                             double* part, unsigned* bar) {
    const bool dot = f && c;
    return SensArgs<T>{p->nelx, p->nely, p->dim == 2 ? 1 : p->nelz, (const T*)xphys, p->passive, u, p->kf64,
                       p->E0, p->Emin, (T*)dc, dot ? f : nullptr, p->info.n, part, bar, c};
}

static to_status sensitivity_enqueue(Plan* p, to_dtype dt, const void* xphys, const double* u, const double* f,
                                     double penal, void* dc, double* c, double* part, unsigned* bar, hipStream_t s) {
    const int blocks = sens_blocks(p, f && c);
    if (dt == TO_F64) {
        const SensArgs<double> A = sens_args<double>(p, xphys, u, f, dc, c, part, bar);
        if (p->dim == 2) hipLaunchKernelGGL((sensitivity_kernel<2, double>), dim3(blocks), dim3(kBlock), 0, s, A, penal);
        else hipLaunchKernelGGL((sensitivity_kernel<3, double>), dim3(blocks), dim3(kBlock), 0, s, A, penal);
    } else {
        const SensArgs<float> A = sens_args<float>(p, xphys, u, f, dc, c, part, bar);
        if (p->dim == 2) hipLaunchKernelGGL((sensitivity_kernel<2, float>), dim3(blocks), dim3(kBlock), 0, s, A, penal);
        else hipLaunchKernelGGL((sensitivity_kernel<3, float>), dim3(blocks), dim3(kBlock), 0, s, A, penal);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

to_status launch_sensitivity(Plan* p, to_dtype dt, const void* xphys, const double* u, const double* f,
                             double penal, void* dc, double* c, hipStream_t s) {
    // partial slots in the second region of the plan's partial buffer
    double* part = p->partial + (size_t)kMaxCoopBlocks * kPartialWidth;
    return sensitivity_enqueue(p, dt, xphys, u, f, penal, dc, c, part, p->bar, s);
}

// --- batches ---------------------------------------------------------------------
size_t sens_args_bytes() {
    static_assert(sizeof(SensArgs<double>) == sizeof(SensArgs<float>), "one table layout for both types");
    return sizeof(SensArgs<double>);
}

int sens_batch_cap(const Plan* p) { return sens_blocks(p, true); }

void sens_args_fill(Plan* p, to_dtype dt, const void* xphys, const double* u, const double* f, void* dc, double* c,
                    void* dst) {
    double* part = p->partial + (size_t)kMaxCoopBlocks * kPartialWidth;
    if (dt == TO_F64) {
        const SensArgs<double> A = sens_args<double>(p, xphys, u, f, dc, c, part, p->bar);
        std::memcpy(dst, &A, sizeof A);
    } else {
        const SensArgs<float> A = sens_args<float>(p, xphys, u, f, dc, c, part, p->bar);
        std::memcpy(dst, &A, sizeof A);
    }
}

// One launch for every design of a batch; block counts per design must not
// exceed sens_batch_cap (one partial slot per block).
to_status launch_sensitivity_batch(int dim, to_dtype dt, const void* tab, const double* dyn, int dyn_stride,
                                   const BatchMap& mp, hipStream_t s) {
    if (dt == TO_F64) {
        if (dim == 2)
            hipLaunchKernelGGL((sensitivity_batch_kernel<2, double>), dim3(mp.blocks), dim3(kBlock), 0, s,
                               (const SensArgs<double>*)tab, dyn, dyn_stride, mp.inst, mp.first, mp.count);
        else
            hipLaunchKernelGGL((sensitivity_batch_kernel<3, double>), dim3(mp.blocks), dim3(kBlock), 0, s,
                               (const SensArgs<double>*)tab, dyn, dyn_stride, mp.inst, mp.first, mp.count);
    } else {
        if (dim == 2)
            hipLaunchKernelGGL((sensitivity_batch_kernel<2, float>), dim3(mp.blocks), dim3(kBlock), 0, s,
                               (const SensArgs<float>*)tab, dyn, dyn_stride, mp.inst, mp.first, mp.count);
        else
            hipLaunchKernelGGL((sensitivity_batch_kernel<3, float>), dim3(mp.blocks), dim3(kBlock), 0, s,
                               (const SensArgs<float>*)tab, dyn, dyn_stride, mp.inst, mp.first, mp.count);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

// --- allocation-free variant ---------------------------------------------------
// Scratch of to_sensitivity_noalloc: kSensMaxBlocks block partials (FP64)
// followed by kSensBarWords arrival-counter words.  A file-scope device array
// exists once per device for the life of the process; host code must not pass
// its name to a kernel (on the host the name is only a stand-in): the device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchPartBytes = sizeof(double) * kSensMaxBlocks;
constexpr size_t kScratchBytes = kScratchPartBytes + sizeof(unsigned) * kSensBarWords;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Zeroes the arrival counters (the last block of a call leaves them at zero,
// but a call that never ran to its end would not).  A kernel rather than a
// memset, so the call stays capturable.
__global__ void sens_scratch_clear_kernel(unsigned* bar) {
    for (int i = threadIdx.x; i < kSensBarWords; i += blockDim.x) bar[i] = 0u;
}

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

to_status launch_sensitivity_noalloc(Plan* p, to_dtype dt, const void* xphys, const double* u, const double* f,
                                     double penal, void* dc, double* c, hipStream_t s) {
    int dev = -1;
    TO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("to_sensitivity_noalloc: device ordinal out of range");
        return TO_EINVAL;
    }
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* q = nullptr;
            hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
            g_scratch_ptr[dev] = q;
        }
        base = g_scratch_ptr[dev];
    }
    // one FP64 partial per block of the launch; the launch clamps its grid,
    // so any mesh fits, and this guards the bound if either side changes
    if ((f && c) && (size_t)sens_blocks(p, true) * sizeof(double) > kScratchPartBytes) {
        set_error("to_sensitivity_noalloc: the launch needs more block partials than the static scratch holds");
        return TO_EINVAL;
    }
    double* part = reinterpret_cast<double*>(base);
    unsigned* bar = reinterpret_cast<unsigned*>(reinterpret_cast<unsigned char*>(base) + kScratchPartBytes);
    if (f && c) {
        hipLaunchKernelGGL(sens_scratch_clear_kernel, dim3(1), dim3(kBlock), 0, s, bar);
        TO_HIP(hipGetLastError());
    }
    return sensitivity_enqueue(p, dt, xphys, u, f, penal, dc, c, part, bar, s);
}

}  // namespace topt
