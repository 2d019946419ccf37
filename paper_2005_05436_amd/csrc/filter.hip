// Cone density filter, eq. (2), and its adjoint (the back-filter of eq. (8),
// read as the chain rule), as LDS-tiled stencils with halo.
//
// Layout: fields are in element order (y fastest), i.e. column-major images.
// 2D tile: 64 rows (one wave's lanes, contiguous in memory) x 4*V columns (V
// per wave).  The block stages a (64+2R) x (4V+2R) window in LDS with the
// boundary rule applied while loading ('D': zeros outside, 'N': half-sample
// mirror, period 2N), so the tap loop itself is branch-free.  Every lane owns
// V outputs in one row; all lanes of a wave share the tap offset, so the
// weight is a wave-uniform (scalar) load.  Taps with zero weight are skipped
// per column through the plan's hlim table (the cone's support).
//
// Modes: RAW  out = h * in               (used once for Hs)
//        FWD  out = (h * in) / Hs
//        ADJ  out = h * (in . s / Hs)
//        ADJ2 out = h * (in . s / Hs), out2 = h * (in2 . s / Hs)  (one pass)
#include "common.h"

namespace topt {

enum { M_RAW = 0, M_FWD = 1, M_ADJ = 2, M_ADJ2 = 3 };

__device__ __forceinline__ int mirror_idx(int k, int N) {
    int p = 2 * N;
    k %= p;
    if (k < 0) k += p;
    return k >= N ? p - 1 - k : k;
}

template <typename T>
__device__ __forceinline__ T staged_value(int mode, const T* in, const T* sc, const T* Hs, int64_t e) {
    T v = in[e];
    if (mode >= M_ADJ) {
        if (sc) v = v * sc[e];
        v = v / Hs[e];
    }
    return v;
}

// ---------------------------------------------------------------------------
// 2D
template <typename T, int MODE, int V>
__global__ __launch_bounds__(kBlock) void filter2d_kernel(
    int nely, int nelx, int R, char bc, const T* __restrict__ h, const int32_t* __restrict__ hlim,
    const T* __restrict__ Hs, const T* __restrict__ in, const T* __restrict__ in2,
    const T* __restrict__ sc, T* __restrict__ out, T* __restrict__ out2) {
    extern __shared__ unsigned char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);
    constexpr int NF = MODE == M_ADJ2 ? 2 : 1;
    constexpr int TX = kWaves * V;
    const int W = 2 * R + 1;
    const int LY = 64 + 2 * R;           // LDS column height (y, contiguous)
    const int LX = TX + 2 * R;           // LDS columns (x)
    const int y0 = blockIdx.x * 64, x0 = blockIdx.y * TX;
    T* tile2 = tile + (size_t)LY * LX;

    // stage the window with the boundary rule
    for (int i = threadIdx.x; i < LY * LX; i += kBlock) {
        int ly = i % LY, lx = i / LY;
        int gy = y0 - R + ly, gx = x0 - R + lx;
        T v = T(0), v2 = T(0);
        bool inside = gy >= 0 && gy < nely && gx >= 0 && gx < nelx;
        if (bc == 'N' && !inside) {
            gy = mirror_idx(gy, nely);
            gx = mirror_idx(gx, nelx);
            inside = true;
        }
        if (inside) {
            int64_t e = gy + (int64_t)nely * gx;
            if (MODE == M_RAW) v = T(1);
            else v = staged_value<T>(MODE, in, sc, Hs, e);
            if (NF == 2) v2 = staged_value<T>(MODE, in2, sc, Hs, e);
        }
        tile[i] = v;
        if (NF == 2) tile2[i] = v2;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gy = y0 + lane;
    const int cx0 = wv * V;              // first owned column, tile-local
    T acc[V], acc2[V];
#pragma unroll
    for (int v = 0; v < V; ++v) { acc[v] = T(0); acc2[v] = T(0); }

    for (int dxi = 0; dxi < W; ++dxi) {
        const int lim = hlim[dxi];
        if (lim < 0) continue;
        const T* hc = h + (size_t)dxi * W + R;       // hc[dy], |dy| <= lim
        // LDS column of output v at this dx: cx0 + v + dxi (offset by R already)
        const T* col = tile + (size_t)(cx0 + dxi) * LY + lane + R;
        const T* colb = tile2 + (size_t)(cx0 + dxi) * LY + lane + R;
        for (int dy = -lim; dy <= lim; ++dy) {
            const T w = hc[dy];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                acc[v] += w * col[(size_t)v * LY + dy];
                if (NF == 2) acc2[v] += w * colb[(size_t)v * LY + dy];
            }
        }
    }
    if (gy < nely) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            int gx = x0 + cx0 + v;
            if (gx < nelx) {
                int64_t e = gy + (int64_t)nely * gx;
                T r = acc[v];
                if (MODE == M_FWD) r = r / Hs[e];
                out[e] = r;
                if (NF == 2) out2[e] = acc2[v];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 3D: tile of 64 (y) x 4 (z) x 4 (x) outputs, each thread 4 outputs along x.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void filter3d_kernel(
    int nely, int nelz, int nelx, int R, char bc, const T* __restrict__ h,
    const int32_t* __restrict__ hlim, const T* __restrict__ Hs, const T* __restrict__ in,
    const T* __restrict__ in2, const T* __restrict__ sc, T* __restrict__ out, T* __restrict__ out2) {
    extern __shared__ unsigned char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);
    constexpr int NF = MODE == M_ADJ2 ? 2 : 1;
    constexpr int TZ = 4, TXo = 4;
    const int W = 2 * R + 1;
    const int LY = 64 + 2 * R, LZ = TZ + 2 * R, LX = TXo + 2 * R;
    const int nzt = (nelz + TZ - 1) / TZ;
    const int y0 = blockIdx.x * 64, z0 = (blockIdx.y % nzt) * TZ, x0 = (blockIdx.y / nzt) * TXo;
    T* tile2 = tile + (size_t)LY * LZ * LX;
    for (int i = threadIdx.x; i < LY * LZ * LX; i += kBlock) {
        int ly = i % LY, r = i / LY, lz = r % LZ, lx = r / LZ;
        int gy = y0 - R + ly, gz = z0 - R + lz, gx = x0 - R + lx;
        T v = T(0), v2 = T(0);
        bool inside = gy >= 0 && gy < nely && gz >= 0 && gz < nelz && gx >= 0 && gx < nelx;
        if (bc == 'N' && !inside) {
            gy = mirror_idx(gy, nely); gz = mirror_idx(gz, nelz); gx = mirror_idx(gx, nelx);
            inside = true;
        }
        if (inside) {
            int64_t e = gy + (int64_t)nely * (gz + (int64_t)nelz * gx);
            if (MODE == M_RAW) v = T(1);
            else v = staged_value<T>(MODE, in, sc, Hs, e);
            if (NF == 2) v2 = staged_value<T>(MODE, in2, sc, Hs, e);
        }
        tile[i] = v;
        if (NF == 2) tile2[i] = v2;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;   // wv = z offset in the tile
    const int gy = y0 + lane, gz = z0 + wv;
    T acc[TXo], acc2[TXo];
#pragma unroll
    for (int v = 0; v < TXo; ++v) { acc[v] = T(0); acc2[v] = T(0); }
    for (int dxi = 0; dxi < W; ++dxi)
        for (int dzi = 0; dzi < W; ++dzi) {
            const int c = dxi * W + dzi;
            const int lim = hlim[c];
            if (lim < 0) continue;
            const T* hc = h + (size_t)c * W + R;
            for (int dy = -lim; dy <= lim; ++dy) {
                const T w = hc[dy];
#pragma unroll
                for (int v = 0; v < TXo; ++v) {
                    size_t li = (size_t)lane + R + dy + (size_t)LY * ((wv + dzi) + (size_t)LZ * (v + dxi));
                    acc[v] += w * tile[li];
                    if (NF == 2) acc2[v] += w * tile2[li];
                }
            }
        }
    if (gy < nely && gz < nelz) {
#pragma unroll
        for (int v = 0; v < TXo; ++v) {
            int gx = x0 + v;
            if (gx < nelx) {
                int64_t e = gy + (int64_t)nely * (gz + (int64_t)nelz * gx);
                T r = acc[v];
                if (MODE == M_FWD) r = r / Hs[e];
                out[e] = r;
                if (NF == 2) out2[e] = acc2[v];
            }
        }
    }
}

// ---------------------------------------------------------------------------
template <typename T, int MODE>
static to_status run_filter(Plan* p, const T* h, const T* Hs, const T* in, const T* in2, const T* sc,
                            T* out, T* out2, hipStream_t s) {
    constexpr int NF = MODE == M_ADJ2 ? 2 : 1;
    const int R = p->R;
    const size_t lds_max = 160 * 1024;
    if (p->dim == 2) {
        constexpr int V = 4;
        size_t lds = (size_t)NF * (64 + 2 * R) * (kWaves * V + 2 * R) * sizeof(T);
        if (lds > lds_max) { set_error("filter radius too large for the LDS tile"); return TO_EUNSUPPORTED; }
        auto k = filter2d_kernel<T, MODE, V>;
        TO_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        dim3 grid((p->nely + 63) / 64, (p->nelx + kWaves * V - 1) / (kWaves * V));
        hipLaunchKernelGGL(k, grid, dim3(kBlock), lds, s, p->nely, p->nelx, R, p->bc, h, p->hlim, Hs, in,
                           in2, sc, out, out2);
    } else {
        size_t lds = (size_t)NF * (64 + 2 * R) * (4 + 2 * R) * (4 + 2 * R) * sizeof(T);
        if (lds > lds_max) { set_error("3D filter radius too large for the LDS tile"); return TO_EUNSUPPORTED; }
        auto k = filter3d_kernel<T, MODE>;
        TO_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        int nzt = (p->nelz + 3) / 4, nxt = (p->nelx + 3) / 4;
        dim3 grid((p->nely + 63) / 64, nzt * nxt);
        hipLaunchKernelGGL(k, grid, dim3(kBlock), lds, s, p->nely, p->nelz, p->nelx, R, p->bc, h, p->hlim,
                           Hs, in, in2, sc, out, out2);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

__global__ void cast_f64_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

to_status launch_fill_hs(Plan* p, hipStream_t s) {
    to_status st = run_filter<double, M_RAW>(p, p->h64, nullptr, nullptr, nullptr, nullptr, p->Hs64, nullptr, s);
    if (st != TO_OK) return st;
    int64_t m = p->info.m ? p->info.m : (int64_t)p->nelx * p->nely * (p->dim == 3 ? p->nelz : 1);
    hipLaunchKernelGGL(cast_f64_to_f32, dim3(256), dim3(kBlock), 0, s, p->Hs64, p->Hs32, m);
    TO_HIP(hipGetLastError());
    return TO_OK;
}

to_status launch_filter(Plan* p, to_dtype dt, int mode, const void* in, const void* in2, const void* sc,
                        void* out, void* out2, hipStream_t s) {
    if (dt == TO_F64) {
        auto a = (const double*)in; auto b = (const double*)in2; auto c = (const double*)sc;
        auto o = (double*)out; auto o2 = (double*)out2;
        if (mode == TO_FILTER_FWD) return run_filter<double, M_FWD>(p, p->h64, p->Hs64, a, b, c, o, o2, s);
        if (mode == TO_FILTER_ADJ) return run_filter<double, M_ADJ>(p, p->h64, p->Hs64, a, b, c, o, o2, s);
        to_status st = run_filter<double, M_ADJ2>(p, p->h64, p->Hs64, a, b, c, o, o2, s);
        if (st == TO_EUNSUPPORTED) {   // two fields do not fit the LDS: two passes
            st = run_filter<double, M_ADJ>(p, p->h64, p->Hs64, a, nullptr, c, o, nullptr, s);
            if (st == TO_OK) st = run_filter<double, M_ADJ>(p, p->h64, p->Hs64, b, nullptr, c, o2, nullptr, s);
        }
        return st;
    }
    auto a = (const float*)in; auto b = (const float*)in2; auto c = (const float*)sc;
    auto o = (float*)out; auto o2 = (float*)out2;
    if (mode == TO_FILTER_FWD) return run_filter<float, M_FWD>(p, p->h32, p->Hs32, a, b, c, o, o2, s);
    if (mode == TO_FILTER_ADJ) return run_filter<float, M_ADJ>(p, p->h32, p->Hs32, a, b, c, o, o2, s);
    to_status st = run_filter<float, M_ADJ2>(p, p->h32, p->Hs32, a, b, c, o, o2, s);
    if (st == TO_EUNSUPPORTED) {
        st = run_filter<float, M_ADJ>(p, p->h32, p->Hs32, a, nullptr, c, o, nullptr, s);
        if (st == TO_OK) st = run_filter<float, M_ADJ>(p, p->h32, p->Hs32, b, nullptr, c, o2, nullptr, s);
    }
    return st;
}

}  // namespace topt
