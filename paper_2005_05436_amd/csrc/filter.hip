// Cone density filter, eq. (2), and its adjoint (the back-filter of eq. (8),
// read as the chain rule), as LDS-tiled stencils with halo.
//
// Layout: fields are in element order (y fastest), i.e. column-major images.
// 2D tile: 64 rows (one wave's lanes, contiguous in memory) x 4*V columns (V
// per wave).  The block stages a (64+2R) x (4V+2R+V) window in LDS with the
// boundary rule applied while loading ('D': zeros outside, 'N': half-sample
// mirror, period 2N), so the tap loop itself is branch-free.  Every lane owns
// V outputs in one row; all lanes of a wave share the tap offset, so the
// weight is a wave-uniform (scalar) load.  Taps with zero weight are skipped
// through the plan's hlim table (the cone's support).
//
// Modes: RAW  out = h * in               (used once for Hs)
//        FWD  out = (h * in) / Hs
//        ADJ  out = h * (in . s / Hs)
//        ADJ2 out = h * (in . s / Hs), out2 = h * (in2 . s / Hs)  (one pass)
#include <cstring>
#include <type_traits>

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
// 2D.  Work is cut into tiles of 64 rows (a wave's lanes, contiguous in memory)
// by V columns; the blocks are persistent (a few per CU) and take tiles from
// an atomic counter, so the ALU-bound large-radius case stays balanced over
// the CUs whatever the mesh size.  A block stages the tile's (64+2R) x
// (V+2R+V) window in LDS with the boundary rule applied while loading, then
// its `parts` waves split the tap rows dy (every parts-th row).  For a tap row
// a lane slides along x through its LDS row: the V outputs need V consecutive
// columns and one more tap to the right needs one new column, so a ring of V
// registers (indexed at compile time by unrolling V taps) turns each LDS read
// into V fused multiply-adds with one wave-uniform weight.  The cone weights
// are symmetric, so the per-column support table hlim also bounds each tap
// row; the last unrolled chunk of a row runs past it into the zero padding of
// the plan's padded row table (8 consecutive weights per scalar load) and the
// V spare window columns.  Partial sums of the parts are added through LDS.
constexpr int kFiltV = 8, kFiltMaxParts = 16;

// One chunk of V taps of a tap row: the window is cur[0..V) followed by
// nxt[0..V) (columns kV .. kV+2V-1 after the row's first column); while the
// FMAs run, the columns of the chunk after next are fetched into fut and the
// next chunk's weights into wnext.  The weights come through vector memory
// loads with a uniform address (a zero the compiler cannot see through keeps
// them off the scalar path): scalar loads share the LDS wait counter and may
// complete out of order, so waiting for a scalar weight would also wait for
// the column prefetch just issued.
template <typename T, int NF, int V, int LS>
__device__ __forceinline__ void filt_chunk(const T* __restrict__ hrow, int k, const T* col0, const T* col0b,
                                           int ls, int nch, T (&cur)[V], T (&nxt)[V], T (&fut)[V],
                                           T (&cur2)[V], T (&nxt2)[V], T (&fut2)[V], const T (&wk)[V],
                                           T (&wnext)[V], T (&acc)[V], T (&acc2)[V]) {
    const int stride = LS ? LS : ls;
    if (k + 1 < nch) {
        const T* p = col0 + (size_t)(k + 2) * V * stride;
#pragma unroll
        for (int u = 0; u < V; ++u) fut[u] = p[(size_t)u * stride];
        if (NF == 2) {
            const T* p2 = col0b + (size_t)(k + 2) * V * stride;
#pragma unroll
            for (int u = 0; u < V; ++u) fut2[u] = p2[(size_t)u * stride];
        }
#pragma unroll
        for (int u = 0; u < V; ++u) wnext[u] = hrow[(k + 1) * V + u];
    }
#pragma unroll
    for (int u = 0; u < V; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int j = u + v;
            acc[v] += wk[u] * (j < V ? cur[j] : nxt[j - V]);
            if (NF == 2) acc2[v] += wk[u] * (j < V ? cur2[j] : nxt2[j - V]);
        }
}

// LS: the LDS column stride when known at compile time (0: 64 + 2R at run
// time); a compile-time stride turns the V column reads of a chunk into one
// base address with immediate offsets.
// At most 16 waves per block in FP32; in FP64 at most 8, so the launch bound
// leaves 256 registers per lane (the ring, the weights and the accumulators
// of FP64 values take twice the registers).
template <typename T>
constexpr int filt_max_parts() { return sizeof(T) == 8 ? 8 : kFiltMaxParts; }

// One 64 x V tile t of one field set: stage the window with the boundary
// rule, run the tap rows of this wave's part, combine the parts in LDS and
// write the outputs.  Ends with a block barrier (the tile buffer is free
// again).
template <typename T>
struct Filt2dArgs {
    int nely, nelx, R;
    char bc;
    const T* hp;
    int hps;
    const int32_t* hlim;
    const T* Hs;
    const T* in;
    const T* in2;
    const T* sc;
    T* out;
    T* out2;
};

template <typename T, int MODE, int V, int LS>
__device__ __forceinline__ void filter2d_tile(const Filt2dArgs<T>& fa, int t, T* tile, int lane, int part, int parts) {
    constexpr int NF = MODE == M_ADJ2 ? 2 : 1;
    const int nely = fa.nely, nelx = fa.nelx, R = fa.R;
    const char bc = fa.bc;
    const T* __restrict__ hp = fa.hp;
    const int hps = fa.hps;
    const int32_t* __restrict__ hlim = fa.hlim;
    const T* __restrict__ Hs = fa.Hs;
    const T* __restrict__ in = fa.in;
    const T* __restrict__ in2 = fa.in2;
    const T* __restrict__ sc = fa.sc;
    T* __restrict__ out = fa.out;
    T* __restrict__ out2 = fa.out2;
    const int W = 2 * R + 1;
    const int LY = 64 + 2 * R;           // staged rows (y, contiguous)
    const int ls = LS ? LS : LY;         // column stride
    const int LX = V + 2 * R + V;        // LDS columns (x), V spare
    const int nty = (nely + 63) / 64;
    T* tile2 = tile + (size_t)ls * LX;
    const int y0 = (t % nty) * 64, x0 = (t / nty) * V;
    // stage the window with the boundary rule
    // (ly, lx) of element i = ly + LY lx, advanced without a division per element
    const int step_x = (int)blockDim.x / LY, step_y = (int)blockDim.x % LY;
    int ly = (int)threadIdx.x % LY, lx = (int)threadIdx.x / LY;
    for (int i = threadIdx.x; i < LY * LX; i += blockDim.x) {
        int gy = y0 - R + ly, gx = x0 - R + lx;
        T v = T(0), v2 = T(0);
        bool inside = gy >= 0 && gy < nely && gx >= 0 && gx < nelx;
        if (bc == 'N' && !inside) {
            gy = mirror_idx(gy, nely);
            gx = mirror_idx(gx, nelx);
            inside = true;
        }
        if (inside) {
            const int64_t e = gy + (int64_t)nely * gx;
            if (MODE == M_RAW) v = T(1);
            else v = staged_value<T>(MODE, in, sc, Hs, e);
            if (NF == 2) v2 = staged_value<T>(MODE, in2, sc, Hs, e);
        }
        tile[(size_t)lx * ls + ly] = v;
        if (NF == 2) tile2[(size_t)lx * ls + ly] = v2;
        ly += step_y;
        lx += step_x;
        if (ly >= LY) { ly -= LY; ++lx; }
    }
    __syncthreads();

    T acc[V], acc2[V];
#pragma unroll
    for (int v = 0; v < V; ++v) { acc[v] = T(0); acc2[v] = T(0); }
    for (int dyi = part; dyi < W; dyi += parts) {
        const int lim = hlim[dyi];
        if (lim < 0) continue;
        // hrow[t] = h(dy, t - lim), zero past 2 lim; read per lane (see filt_chunk)
        int zero;
        asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
        const T* hrow = hp + (size_t)dyi * hps + zero;
        // column R - lim of this lane's LDS row at this dy: output 0 at dx = -lim
        const T* col0 = tile + lane + dyi + (size_t)(R - lim) * ls;
        const T* col0b = tile2 + lane + dyi + (size_t)(R - lim) * ls;
        const int nch = (2 * lim + 1 + V - 1) / V;
        T A[V], B[V], C[V], A2[V], B2[V], C2[V], WA[V], WB[V], WC[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
            A[u] = col0[(size_t)u * ls];
            B[u] = col0[(size_t)(V + u) * ls];
            if (NF == 2) {
                A2[u] = col0b[(size_t)u * ls];
                B2[u] = col0b[(size_t)(V + u) * ls];
            }
            WA[u] = hrow[u];
        }
        // three buffers of columns and of weights rotate, so no register moves are needed
        for (int k = 0; k < nch; k += 3) {
            filt_chunk<T, NF, V, LS>(hrow, k, col0, col0b, ls, nch, A, B, C, A2, B2, C2, WA, WB, acc, acc2);
            if (k + 1 < nch)
                filt_chunk<T, NF, V, LS>(hrow, k + 1, col0, col0b, ls, nch, B, C, A, B2, C2, A2, WB, WC, acc,
                                         acc2);
            if (k + 2 < nch)
                filt_chunk<T, NF, V, LS>(hrow, k + 2, col0, col0b, ls, nch, C, A, B, C2, A2, B2, WC, WA, acc,
                                         acc2);
        }
    }
    // combine the parts' partial sums (the window is no longer needed)
    __syncthreads();
    T* red = tile;                                      // [part][field][v][lane]
    const int slab = NF * V * 64;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        red[part * slab + v * 64 + lane] = acc[v];
        if (NF == 2) red[part * slab + V * 64 + v * 64 + lane] = acc2[v];
    }
    __syncthreads();
    // wave q finishes output column q of the tile (q < V)
    if (part < V) {
        const int gy = y0 + lane, gx = x0 + part;
        T r = T(0), r2 = T(0);
        for (int q = 0; q < parts; ++q) {
            r += red[q * slab + part * 64 + lane];
            if (NF == 2) r2 += red[q * slab + V * 64 + part * 64 + lane];
        }
        if (gy < nely && gx < nelx) {
            const int64_t e = gy + (int64_t)nely * gx;
            if (MODE == M_FWD) r = r / Hs[e];
            out[e] = r;
            if (NF == 2) out2[e] = r2;
        }
    }
    __syncthreads();
}

template <typename T, int MODE, int V, int LS>
__global__ __launch_bounds__(64 * filt_max_parts<T>()) void filter2d_kernel(Filt2dArgs<T> A, unsigned* ctr,
                                                                          const unsigned* skip, int chunk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];   // 16-byte aligned: FP64 and wide LDS accesses
    __shared__ int tile_sh;
    if (skip && *skip) return;          // the whole launch is cancelled (the tile counter is untouched)
    T* tile = reinterpret_cast<T*>(smem_raw);
    const int nty = (A.nely + 63) / 64, ntiles = nty * ((A.nelx + V - 1) / V);
    const int lane = threadIdx.x & 63;
    // wave index made provably wave-uniform, so the tap loop's bounds and
    // weights are scalar loads (SGPRs) rather than per-lane loads
    const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int parts = blockDim.x >> 6;
    // tiles are claimed `chunk` at a time: every claim is an atomic on one
    // address, which at small radii (little work per tile) would serialise
    int t = 0, t_end = 0;
    for (;; ++t) {
        if (t >= t_end) {
            if (threadIdx.x == 0) tile_sh = (int)atomicAdd(&ctr[0], (unsigned)chunk);
            __syncthreads();
            t = tile_sh;
            t_end = min(t + chunk, ntiles);
        }
        if (t >= ntiles) break;
        filter2d_tile<T, MODE, V, LS>(A, t, tile, lane, part, parts);
    }
    // the last block to finish resets the tile counter for the next launch
    if (threadIdx.x == 0) {
        const unsigned done = atomicAdd(&ctr[1], 1u);
        if (done == gridDim.x - 1) {
            st_dev(&ctr[0], 0u);
            st_dev(&ctr[1], 0u);
        }
    }
}

// Many designs in one launch: the tiles of all designs form one list (design
// i owns tiles tile0[i] .. tile0[i+1]-1) claimed from one counter; each tile
// is filtered with its own design's arguments (a block-uniform lookup, so the
// table reads are scalar loads).
template <typename T, int MODE, int V, int LS>
__global__ __launch_bounds__(64 * filt_max_parts<T>()) void filter2d_batch_kernel(
    const Filt2dArgs<T>* __restrict__ tab, const int32_t* __restrict__ tile0, int ndesign, unsigned* ctr, int chunk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];   // 16-byte aligned: FP64 and wide LDS accesses
    __shared__ int tile_sh;
    T* tile = reinterpret_cast<T*>(smem_raw);
    const int ntiles = tile0[ndesign];
    const int lane = threadIdx.x & 63;
    const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int parts = blockDim.x >> 6;
    int t = 0, t_end = 0;
    for (;; ++t) {
        if (t >= t_end) {
            if (threadIdx.x == 0) tile_sh = (int)atomicAdd(&ctr[0], (unsigned)chunk);
            __syncthreads();
            t = __builtin_amdgcn_readfirstlane(tile_sh);
            t_end = min(t + chunk, ntiles);
        }
        if (t >= ntiles) break;
        int lo = 0, hi = ndesign;            // tile0[lo] <= t < tile0[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tile0[mid] <= t) lo = mid;
            else hi = mid;
        }
        filter2d_tile<T, MODE, V, LS>(tab[lo], t - tile0[lo], tile, lane, part, parts);
    }
    if (threadIdx.x == 0) {
        const unsigned done = atomicAdd(&ctr[1], 1u);
        if (done == gridDim.x - 1) {
            st_dev(&ctr[0], 0u);
            st_dev(&ctr[1], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// 2D, on the matrix cores (FP32 or FP64).  For one tap column dx the cone filter acts
// along y as a banded Toeplitz matrix: out[y0+i][x] += sum_t h(dx, t-i)
// in[y0+t][x+dx].  For 16 output rows and 16 output columns that is a
// (16 x K) band block of weights times a (K x 16) block of the staged
// window, K = 16 + 2 lim(dx) rounded up to 4, which v_mfma_f32_16x16x4_f32
// (v_mfma_f64_16x16x4_f64 for FP64 fields) takes four rows of K at a time (about 80% of the products are non-zero
// taps at large radii).  Operand lanes: A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k, D[4q+r][j] in register r of lane j + 16q.  Lane group k takes
// the contiguous rows k S .. k S + S - 1 of K (S = K / 4), so the weight of
// lane (i, k) at step s is h(dx, k S + s - lim - i), read from a per-column
// table with 16 zeros before and 19 or more after the taps (one copy per
// block in LDS).
//
// Block: 8 waves on a tile of TY = 16 MT rows by TX = 16 NB columns; wave w
// owns the 16-row strip w % MT of the tile (NB accumulators, so each weight
// register feeds NB products) and the tap columns dx = w / MT (mod 8 / MT);
// the parts are added in LDS.  Tiles are claimed like the stencil kernel's.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kFmUnroll = 4;           // MFMA steps whose operand reads issue together

// The 16 x 16 x 4 products in FP32 and FP64: the same operand layout
// (A[i][k] in lane i + 16k, B[k][j] in lane j + 16k); the results differ:
// D[4q+r][j] (FP32) and D[q+4r][j] (FP64) in register r of lane j + 16q.
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    using acc = f32x4;
    __device__ static acc step(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int q, int r) { return 4 * q + r; }
};
template <> struct Mfma<double> {
    using acc = f64x4;
    __device__ static acc step(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int q, int r) { return q + 4 * r; }
};

template <typename T, int MODE, int MT, int NB>
__global__ __launch_bounds__(512) void filter2d_mfma_kernel(
    int nely, int nelx, int R, char bc, const T* __restrict__ hm, int hms, const int32_t* __restrict__ hlim,
    const T* __restrict__ Hs, const T* __restrict__ in, const T* __restrict__ in2,
    const T* __restrict__ sc, T* __restrict__ out, T* __restrict__ out2, unsigned* ctr,
    const unsigned* skip, int chunk, int wofs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];   // 16-byte aligned: FP64 and wide LDS accesses
    __shared__ int tile_sh;
    if (skip && *skip) return;          // the whole launch is cancelled (the tile counter is untouched)
    constexpr int NF = MODE == M_ADJ2 ? 2 : 1;
    constexpr int NP = 8 / MT;           // tap-column parts
    constexpr int TY = 16 * MT, TX = 16 * NB;
    using Acc = typename Mfma<T>::acc;
    T* tile = reinterpret_cast<T*>(smem_raw);
    const int LY = TY + 2 * R + 3;       // rows y0-R .. y0+TY+R+2 (the last 3 meet zero weights only)
    const int ls = LY | 1;               // odd column stride: the 16 columns of a read fall in distinct banks
    const int LX = TX + 2 * R;
    T* tile2 = tile + (size_t)ls * LX;
    const int nty = (nely + TY - 1) / TY, ntiles = nty * ((nelx + TX - 1) / TX);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int mt = w % MT, part = w / MT;
    const int i16 = lane & 15, kq = lane >> 4;
    T* wtab = tile + wofs;           // the weight columns -R..0 (h is even in dx), for the whole launch
    for (int i = threadIdx.x; i < (R + 1) * hms; i += blockDim.x) wtab[i] = hm[i];

    int t = 0, t_end = 0;
    for (;; ++t) {
        if (t >= t_end) {
            if (threadIdx.x == 0) tile_sh = (int)atomicAdd(&ctr[0], (unsigned)chunk);
            __syncthreads();
            t = tile_sh;
            t_end = min(t + chunk, ntiles);
        }
        if (t >= ntiles) break;
        const int y0 = (t % nty) * TY, x0 = (t / nty) * TX;
        // (ly, lx) of element i = ly + LY lx, advanced without a division per element
        const int step_x = (int)blockDim.x / LY, step_y = (int)blockDim.x % LY;
        int ly = (int)threadIdx.x % LY, lx = (int)threadIdx.x / LY;
        for (int i = threadIdx.x; i < LY * LX; i += blockDim.x) {
            int gy = y0 - R + ly, gx = x0 - R + lx;
            T v = T(0), v2 = T(0);
            bool inside = gy >= 0 && gy < nely && gx >= 0 && gx < nelx;
            if (bc == 'N' && !inside) {
                gy = mirror_idx(gy, nely);
                gx = mirror_idx(gx, nelx);
                inside = true;
            }
            if (inside) {
                const int64_t e = gy + (int64_t)nely * gx;
                v = staged_value<T>(MODE, in, sc, Hs, e);
                if (NF == 2) v2 = staged_value<T>(MODE, in2, sc, Hs, e);
            }
            tile[(size_t)lx * ls + ly] = v;
            if (NF == 2) tile2[(size_t)lx * ls + ly] = v2;
            ly += step_y;
            lx += step_x;
            if (ly >= LY) { ly -= LY; ++lx; }
        }
        __syncthreads();

        Acc acc[NF][NB];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[f][nb] = Acc{T(0), T(0), T(0), T(0)};
        // h is even in dx: the columns +dx and -dx share their weights, so
        // their window values are added first and one product serves both
        // (half the matrix-core work; column dx = 0 alone)
        for (int dxa = part; dxa <= R; dxa += NP) {
            const int lim = hlim[R + dxa];
            if (lim < 0) continue;
            const int S = (16 + 2 * lim + 3) >> 2;
            const T* ap = wtab + (size_t)(R - dxa) * hms + (R + 16 - lim) + kq * S - i16;
            const size_t r0 = (size_t)mt * 16 + R - lim + kq * S;
            const size_t bpo = (size_t)(R + dxa + i16) * ls + r0, bmo = (size_t)(R - dxa + i16) * ls + r0;
            const T* bp = tile + bpo;
            const T* bm = tile + bmo;
            const T* bp2 = tile2 + bpo;
            const T* bm2 = tile2 + bmo;
            // MFMA is convergent, so the compiler will not unroll a loop of
            // unknown trip count: groups of kFmUnroll steps by hand (their
            // LDS reads issue together), then the rest one by one
            auto step = [&](int s, auto pair) {
                const T a = ap[s];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const size_t o = (size_t)nb * 16 * ls + s;
                    const T b1 = decltype(pair)::value ? bp[o] + bm[o] : bp[o];
                    acc[0][nb] = Mfma<T>::step(a, b1, acc[0][nb]);
                    if (NF == 2) {
                        const T b2 = decltype(pair)::value ? bp2[o] + bm2[o] : bp2[o];
                        acc[NF - 1][nb] = Mfma<T>::step(a, b2, acc[NF - 1][nb]);
                    }
                }
            };
            auto steps = [&](auto pair) {
                int s = 0;
                for (; s + kFmUnroll <= S; s += kFmUnroll) {
#pragma unroll
                    for (int u = 0; u < kFmUnroll; ++u) step(s + u, pair);
                }
                for (; s < S; ++s) step(s, pair);
            };
            if (dxa > 0) steps(std::true_type{});
            else steps(std::false_type{});
        }
        __syncthreads();                 // the window is no longer needed
        T* red = tile;                   // [part][field][column][row], TX x TY per slab
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    red[((size_t)(part * NF + f) * TX + nb * 16 + i16) * TY + mt * 16 + Mfma<T>::row(kq, r)] =
                        acc[f][nb][r];
        __syncthreads();
        for (int o = threadIdx.x; o < TY * TX; o += blockDim.x) {
            const int row = o % TY, col = o / TY;
            const int gy = y0 + row, gx = x0 + col;
            T r0 = T(0), r1 = T(0);
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                r0 += red[((size_t)(q * NF) * TX + col) * TY + row];
                if (NF == 2) r1 += red[((size_t)(q * NF + 1) * TX + col) * TY + row];
            }
            if (gy < nely && gx < nelx) {
                const int64_t e = gy + (int64_t)nely * gx;
                if (MODE == M_FWD) r0 = r0 / Hs[e];
                out[e] = r0;
                if (NF == 2) out2[e] = r1;
            }
        }
        __syncthreads();
    }
    // the last block to finish resets the tile counter for the next launch
    if (threadIdx.x == 0) {
        const unsigned done = atomicAdd(&ctr[1], 1u);
        if (done == gridDim.x - 1) {
            st_dev(&ctr[0], 0u);
            st_dev(&ctr[1], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// 3D: tile of 64 (y) x 4 (z) x 4 (x) outputs, each thread 4 outputs along x.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void filter3d_kernel(
    int nely, int nelz, int nelx, int R, char bc, const T* __restrict__ h,
    const int32_t* __restrict__ hlim, const T* __restrict__ Hs, const T* __restrict__ in,
    const T* __restrict__ in2, const T* __restrict__ sc, T* __restrict__ out, T* __restrict__ out2,
    const unsigned* skip) {
    extern __shared__ __align__(16) unsigned char smem_raw[];   // 16-byte aligned: FP64 and wide LDS accesses
    if (skip && *skip) return;          // the whole launch is cancelled
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
template <typename T, int MODE, int V, int LS>
static to_status run_filter2d_ls(Plan* p, const T* hp, const T* Hs, const T* in, const T* in2, const T* sc, T* out,
                                 T* out2, hipStream_t s) {
    constexpr int NF = MODE == M_ADJ2 ? 2 : 1;
    const int R = p->R;
    const size_t lds_max = 160 * 1024;
    const int W = 2 * R + 1;
    // waves per block: at least V (wave q finishes output column q); by
    // default 16 when there are enough tap rows to split, else V
    constexpr int maxp = filt_max_parts<T>();
    int parts = W >= 16 ? maxp : V;
    const int ptune = NF == 2 ? p->tune.filt_parts2 : p->tune.filt_parts;
    if (ptune > 0) parts = std::max(V, std::min(maxp, ptune));
    const int ls = LS ? LS : 64 + 2 * R;
    size_t lds = (size_t)NF * ls * (V + 2 * R + V) * sizeof(T);
    lds = std::max(lds, (size_t)parts * NF * V * 64 * sizeof(T));   // partial-sum reuse
    if (lds > lds_max) { set_error("filter radius too large for the LDS tile"); return TO_EUNSUPPORTED; }
    auto k = filter2d_kernel<T, MODE, V, LS>;
    TO_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k, 64 * parts, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int ntiles = ((p->nely + 63) / 64) * ((p->nelx + V - 1) / V);
    const int blocks = std::max(1, std::min(ntiles, per_cu * p->num_cu));
    // tiles per claim: about 8 claims per block at large radii (uneven work
    // near the boundary is balanced), 2 at small radii (the claims dominate)
    const int chunk = std::max(1, ntiles / (blocks * (W >= 16 ? 8 : 2)));
    Filt2dArgs<T> A{p->nely, p->nelx, R, p->bc, hp, p->hp_stride, p->hlim, Hs, in, in2, sc, out, out2};
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * parts), lds, s, A, p->bar + 16, p->filt_skip, chunk);
    TO_HIP(hipGetLastError());
    return TO_OK;
}

// the LDS column stride as a compile-time constant where the radius allows
template <typename T, int MODE, int V>
static to_status run_filter2d(Plan* p, const T* hp, const T* Hs, const T* in, const T* in2, const T* sc, T* out,
                              T* out2, hipStream_t s) {
    const int ly = 64 + 2 * p->R;
    if constexpr (V == kFiltV) {
        if (ly <= 96) return run_filter2d_ls<T, MODE, V, 96>(p, hp, Hs, in, in2, sc, out, out2, s);
        if (ly <= 160) return run_filter2d_ls<T, MODE, V, 160>(p, hp, Hs, in, in2, sc, out, out2, s);
        if (ly <= 224) return run_filter2d_ls<T, MODE, V, 224>(p, hp, Hs, in, in2, sc, out, out2, s);
    }
    return run_filter2d_ls<T, MODE, V, 0>(p, hp, Hs, in, in2, sc, out, out2, s);
}

// LDS bytes of the matrix-core kernel's tile shape (window or partial sums)
static size_t mfma_lds(int R, int NF, int MT, int NB, size_t tsz) {
    const int TY = 16 * MT, TX = 16 * NB;
    const size_t win = (size_t)NF * ((TY + 2 * R + 3) | 1) * (TX + 2 * R) * tsz;
    const size_t red = (size_t)(8 / MT) * NF * TY * TX * tsz;
    return std::max(win, red);
}

template <typename T, int MODE, int MT, int NB>
static to_status run_filter2d_mfma_shape(Plan* p, const T* Hs, const T* in, const T* in2,
                                         const T* sc, T* out, T* out2, hipStream_t s) {
    constexpr int NF = MODE == M_ADJ2 ? 2 : 1;
    const int R = p->R;
    const size_t lds0 = mfma_lds(R, NF, MT, NB, sizeof(T));
    const size_t lds = lds0 + (size_t)(R + 1) * p->hm_stride * sizeof(T);   // + the weight table
    if (lds > 160 * 1024 - 256) {        // the block also holds a few static words
        set_error("filter radius too large for the matrix-core tile");
        return TO_EUNSUPPORTED;
    }
    auto k = filter2d_mfma_kernel<T, MODE, MT, NB>;
    const T* hm;
    if constexpr (sizeof(T) == 8) hm = p->hm64; else hm = p->hm32;
    TO_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k, 512, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int ntiles = ((p->nely + 16 * MT - 1) / (16 * MT)) * ((p->nelx + 16 * NB - 1) / (16 * NB));
    const int blocks = std::max(1, std::min(ntiles, per_cu * p->num_cu));
    const int chunk = std::max(1, ntiles / (blocks * 4));
    hipLaunchKernelGGL(k, dim3(blocks), dim3(512), lds, s, p->nely, p->nelx, R, p->bc, hm, p->hm_stride,
                       p->hlim, Hs, in, in2, sc, out, out2, p->bar + 16, p->filt_skip, chunk, (int)(lds0 / sizeof(T)));
    TO_HIP(hipGetLastError());
    return TO_OK;
}

// shape 1: 32 x 64 tiles, 2: 16 x 64, 3: 32 x 32, 4: 16 x 32
template <typename T, int MODE>
static to_status run_filter2d_mfma(Plan* p, int shape, const T* Hs, const T* in, const T* in2,
                                   const T* sc, T* out, T* out2, hipStream_t s) {
    switch (shape) {
    case 1: return run_filter2d_mfma_shape<T, MODE, 2, 4>(p, Hs, in, in2, sc, out, out2, s);
    case 2: return run_filter2d_mfma_shape<T, MODE, 1, 4>(p, Hs, in, in2, sc, out, out2, s);
    case 3: return run_filter2d_mfma_shape<T, MODE, 2, 2>(p, Hs, in, in2, sc, out, out2, s);
    default: return run_filter2d_mfma_shape<T, MODE, 1, 2>(p, Hs, in, in2, sc, out, out2, s);
    }
}

template <typename T, int MODE>
static to_status run_filter(Plan* p, const T* h, const T* hp, const T* Hs, const T* in, const T* in2, const T* sc,
                            T* out, T* out2, hipStream_t s) {
    constexpr int NF = MODE == M_ADJ2 ? 2 : 1;
    const int R = p->R;
    const size_t lds_max = 160 * 1024;
    if (p->dim == 2) {
        if constexpr (MODE != M_RAW) {
            const int shape = NF == 2 ? p->tune.filt_mfma2 : p->tune.filt_mfma;
            if (shape > 0) {
                const to_status st = run_filter2d_mfma<T, MODE>(p, shape, Hs, in, in2, sc, out, out2, s);
                if (st != TO_EUNSUPPORTED) return st;   // else the tile does not fit: the stencil kernel below
            }
        }
        if (p->tune.filt_v == 4) return run_filter2d<T, MODE, 4>(p, hp, Hs, in, in2, sc, out, out2, s);
        return run_filter2d<T, MODE, kFiltV>(p, hp, Hs, in, in2, sc, out, out2, s);
    } else {
        size_t lds = (size_t)NF * (64 + 2 * R) * (4 + 2 * R) * (4 + 2 * R) * sizeof(T);
        if (lds > lds_max) { set_error("3D filter radius too large for the LDS tile"); return TO_EUNSUPPORTED; }
        auto k = filter3d_kernel<T, MODE>;
        TO_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        int nzt = (p->nelz + 3) / 4, nxt = (p->nelx + 3) / 4;
        dim3 grid((p->nely + 63) / 64, nzt * nxt);
        hipLaunchKernelGGL(k, grid, dim3(kBlock), lds, s, p->nely, p->nelz, p->nelx, R, p->bc, h, p->hlim,
                           Hs, in, in2, sc, out, out2, p->filt_skip);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

__global__ void cast_f64_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

to_status launch_fill_hs(Plan* p, hipStream_t s) {
    to_status st = run_filter<double, M_RAW>(p, p->h64, p->hp64, nullptr, nullptr, nullptr, nullptr, p->Hs64, nullptr, s);
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
        if (mode == TO_FILTER_FWD) return run_filter<double, M_FWD>(p, p->h64, p->hp64, p->Hs64, a, b, c, o, o2, s);
        if (mode == TO_FILTER_ADJ) return run_filter<double, M_ADJ>(p, p->h64, p->hp64, p->Hs64, a, b, c, o, o2, s);
        to_status st = run_filter<double, M_ADJ2>(p, p->h64, p->hp64, p->Hs64, a, b, c, o, o2, s);
        if (st == TO_EUNSUPPORTED) {   // two fields do not fit the LDS: two passes
            st = run_filter<double, M_ADJ>(p, p->h64, p->hp64, p->Hs64, a, nullptr, c, o, nullptr, s);
            if (st == TO_OK) st = run_filter<double, M_ADJ>(p, p->h64, p->hp64, p->Hs64, b, nullptr, c, o2, nullptr, s);
        }
        return st;
    }
    auto a = (const float*)in; auto b = (const float*)in2; auto c = (const float*)sc;
    auto o = (float*)out; auto o2 = (float*)out2;
    if (mode == TO_FILTER_FWD) return run_filter<float, M_FWD>(p, p->h32, p->hp32, p->Hs32, a, b, c, o, o2, s);
    if (mode == TO_FILTER_ADJ) return run_filter<float, M_ADJ>(p, p->h32, p->hp32, p->Hs32, a, b, c, o, o2, s);
    to_status st = run_filter<float, M_ADJ2>(p, p->h32, p->hp32, p->Hs32, a, b, c, o, o2, s);
    if (st == TO_EUNSUPPORTED) {
        st = run_filter<float, M_ADJ>(p, p->h32, p->hp32, p->Hs32, a, nullptr, c, o, nullptr, s);
        if (st == TO_OK) st = run_filter<float, M_ADJ>(p, p->h32, p->hp32, p->Hs32, b, nullptr, c, o2, nullptr, s);
    }
    return st;
}

// --- batches of 2D designs --------------------------------------------------
size_t filter_batch_entry_bytes() {
    static_assert(sizeof(Filt2dArgs<double>) == sizeof(Filt2dArgs<float>), "one table layout for both types");
    return sizeof(Filt2dArgs<double>);
}

int filter_batch_tiles(const Plan* p) { return ((p->nely + 63) / 64) * ((p->nelx + kFiltV - 1) / kFiltV); }

void filter_batch_fill(Plan* p, to_dtype dt, const void* in, const void* in2, const void* sc, void* out, void* out2,
                       void* dst) {
    if (dt == TO_F64) {
        Filt2dArgs<double> A{p->nely, p->nelx, p->R, p->bc, p->hp64, p->hp_stride, p->hlim, p->Hs64,
                             (const double*)in, (const double*)in2, (const double*)sc, (double*)out, (double*)out2};
        std::memcpy(dst, &A, sizeof A);
    } else {
        Filt2dArgs<float> A{p->nely, p->nelx, p->R, p->bc, p->hp32, p->hp_stride, p->hlim, p->Hs32,
                            (const float*)in, (const float*)in2, (const float*)sc, (float*)out, (float*)out2};
        std::memcpy(dst, &A, sizeof A);
    }
}

// LDS bytes of the batched stencil launch for the largest radius of a batch
template <typename T, int NF>
static size_t filter_batch_lds(int rmax) {
    constexpr int V = kFiltV;
    const int parts = 2 * rmax + 1 >= 16 ? filt_max_parts<T>() : V;
    const int ly = 64 + 2 * rmax;
    const int ls = ly <= 96 ? 96 : ly <= 160 ? 160 : ly <= 224 ? 224 : ly;
    const size_t lds = (size_t)NF * ls * (V + 2 * rmax + V) * sizeof(T);
    return std::max(lds, (size_t)parts * NF * V * 64 * sizeof(T));
}

bool filter_batch_fits(to_dtype dt, int rmax) {
    const size_t lds = dt == TO_F64 ? filter_batch_lds<double, 2>(rmax) : filter_batch_lds<float, 2>(rmax);
    return lds <= 160 * 1024;
}

template <typename T, int MODE, int LS>
static to_status run_filter_batch_ls(const void* tab, const int32_t* tile0, int n, int ntiles, int rmax, int num_cu,
                                     unsigned* ctr, hipStream_t s) {
    constexpr int NF = MODE == M_ADJ2 ? 2 : 1, V = kFiltV;
    constexpr int maxp = filt_max_parts<T>();
    const int W = 2 * rmax + 1;
    const int parts = W >= 16 ? maxp : V;
    // the largest radius sets the tile buffer (smaller radii use a part of it)
    const size_t lds = filter_batch_lds<T, NF>(rmax);
    if (lds > 160 * 1024) { set_error("filter radius too large for the LDS tile"); return TO_EUNSUPPORTED; }
    auto k = filter2d_batch_kernel<T, MODE, V, LS>;
    TO_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k, 64 * parts, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int blocks = std::max(1, std::min(ntiles, per_cu * num_cu));
    const int chunk = std::max(1, ntiles / (blocks * (W >= 16 ? 8 : 2)));
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * parts), lds, s, (const Filt2dArgs<T>*)tab, tile0, n, ctr, chunk);
    TO_HIP(hipGetLastError());
    return TO_OK;
}

// the LDS column stride as a compile-time constant where the largest radius allows
template <typename T, int MODE>
static to_status run_filter_batch(const void* tab, const int32_t* tile0, int n, int ntiles, int rmax, int num_cu,
                                  unsigned* ctr, hipStream_t s) {
    const int ly = 64 + 2 * rmax;
    if (ly <= 96) return run_filter_batch_ls<T, MODE, 96>(tab, tile0, n, ntiles, rmax, num_cu, ctr, s);
    if (ly <= 160) return run_filter_batch_ls<T, MODE, 160>(tab, tile0, n, ntiles, rmax, num_cu, ctr, s);
    if (ly <= 224) return run_filter_batch_ls<T, MODE, 224>(tab, tile0, n, ntiles, rmax, num_cu, ctr, s);
    return run_filter_batch_ls<T, MODE, 0>(tab, tile0, n, ntiles, rmax, num_cu, ctr, s);
}

to_status launch_filter_batch(to_dtype dt, int mode, const void* tab, const int32_t* tile0, int n, int ntiles,
                              int rmax, int num_cu, unsigned* ctr, hipStream_t s) {
    if (dt == TO_F64) {
        if (mode == TO_FILTER_FWD) return run_filter_batch<double, M_FWD>(tab, tile0, n, ntiles, rmax, num_cu, ctr, s);
        return run_filter_batch<double, M_ADJ2>(tab, tile0, n, ntiles, rmax, num_cu, ctr, s);
    }
    if (mode == TO_FILTER_FWD) return run_filter_batch<float, M_FWD>(tab, tile0, n, ntiles, rmax, num_cu, ctr, s);
    return run_filter_batch<float, M_ADJ2>(tab, tile0, n, ntiles, rmax, num_cu, ctr, s);
}

}  // namespace topt
