// Learned warm start of the state solve: a small U-Net on the node grid that
// maps (filtered density, load) to a displacement direction, with bfloat16
// weights and activations on the matrix cores (FP32 accumulation), its
// backward pass and Adam, all on the GPU.  The paper has no network; the
// prediction only seeds the CG of eq. (5) (see to_warm_start), so the solve's
// own residual still decides the answer.
//
// Image: planes x rows x columns x channels (channels innermost, padded to
// multiples of 16; each spatial extent padded to a multiple of 8).  2D: one
// plane, rows = ix, columns = iy, so pixel (ix, iy) holds the two DOFs of
// node iy + (nely + 1) ix.  3D: planes = ix, rows = iz, columns = iy, so
// pixel (ix, iz, iy) holds the three DOFs of node iy + (nely + 1) (iz +
// (nelz + 1) ix).  Layers (c_in -> c_out, level), 2D:
//   e1a 3->16 0, e1b 16->16 0 | pool | e2a 16->32 1, e2b 32->32 1 | pool |
//   e3a 32->64 2, e3b 64->64 2 | pool | ba 64->128 3, bb 128->64 3 |
//   up d3a 64->64 2 (+e3b), d3b 64->32 2 | up d2a 32->32 1 (+e2b), d2b 32->16 1 |
//   up d1a 16->16 0 (+e1b), d1b 16->16 0 | out 16->2 0 (no activation)
// and in 3D the same with half the channels (8, 16, 32, 64), 4 inputs
// (density, f_x, f_y, f_z) and 3 outputs.  'same' 3x3 (3x3x3)
// cross-correlation (zero padding), bias, leaky ReLU (slope 1/8), 2x2
// (2x2x2) average pooling, nearest 2x upsampling, additive skips.  Weights
// are kept as an FP32 master vector: per layer W[t][co][ci] (2D: t = 3 (dr+1)
// + (dc+1); 3D: t = 9 (dp+1) + 3 (dr+1) + (dc+1)) then b[co]; the matrix
// cores read bfloat16 copies, padded [T][co][ci] for the forward product and
// flipped-transposed [T][ci][co] for the input gradient.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x16_bf16: a wave owns
// 16 consecutive pixels of one image row and up to 64 output channels (four
// 16x16 accumulators); the K loop runs over the taps and the input channels
// in blocks of 16.  The weight gradient is a GEMM over pixels (M = c_out,
// N = c_in, K = pixels) per tap, reduced across waves in LDS; each block
// stores its partial product and a second kernel adds the blocks' partials in
// block order, so gradients (and training) are bitwise repeatable.  Every
// other sum of the backward pass is ordered the same way.
#include <cmath>
#include <new>

#include "common.h"

namespace topt {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kSlope = 0.125f;
constexpr int kNL = 15;
constexpr int kRedBlocks = 256;        // blocks of the two-level ordered reductions

struct LayerDef { int cin, cout, level, act, src, skip; };   // src: 0 previous, 1 pool, 2 up
static const LayerDef kLayers2[kNL] = {
    {3, 16, 0, 1, 0, -1},  {16, 16, 0, 1, 0, -1},  {16, 32, 1, 1, 1, -1}, {32, 32, 1, 1, 0, -1},
    {32, 64, 2, 1, 1, -1}, {64, 64, 2, 1, 0, -1},  {64, 128, 3, 1, 1, -1}, {128, 64, 3, 1, 0, -1},
    {64, 64, 2, 1, 2, 5},  {64, 32, 2, 1, 0, -1},  {32, 32, 1, 1, 2, 3},  {32, 16, 1, 1, 0, -1},
    {16, 16, 0, 1, 2, 1},  {16, 16, 0, 1, 0, -1},  {16, 2, 0, 0, 0, -1}};
static const LayerDef kLayers3[kNL] = {
    {4, 8, 0, 1, 0, -1},   {8, 8, 0, 1, 0, -1},    {8, 16, 1, 1, 1, -1},  {16, 16, 1, 1, 0, -1},
    {16, 32, 2, 1, 1, -1}, {32, 32, 2, 1, 0, -1},  {32, 64, 3, 1, 1, -1}, {64, 32, 3, 1, 0, -1},
    {32, 32, 2, 1, 2, 5},  {32, 16, 2, 1, 0, -1},  {16, 16, 1, 1, 2, 3},  {16, 8, 1, 1, 0, -1},
    {8, 8, 0, 1, 2, 1},    {8, 8, 0, 1, 0, -1},    {8, 3, 0, 0, 0, -1}};
static const LayerDef* layer_defs(int dim) { return dim == 2 ? kLayers2 : kLayers3; }

static inline int pad16(int c) { return (c + 15) / 16 * 16; }

// ---------------------------------------------------------------------------
// bfloat16 helpers (finite values; round to nearest even)
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// Tap t -> (plane, row, column) offsets: NT = 9 (2D, no plane offset) or 27.
template <int NT>
__device__ __forceinline__ void tap_offset(int t, int& dp, int& dr, int& dc) {
    if (NT == 9) { dp = 0; dr = t / 3 - 1; dc = t % 3 - 1; }
    else { dp = t / 9 - 1; dr = (t / 3) % 3 - 1; dc = t % 3 - 1; }
}

struct ConvArgs {
    const uint16_t* x;      // input [D'][H'][W'][cin] (D' = D / xs, ... ; D = 1 in 2D)
    int xs;                 // 1, or 2 = nearest-upsampled read of a half-size input
    int D, H, W, cin, cout; // output size; channel counts padded to 16
    const uint16_t* w;      // [T][cout][cin]
    const float* bias;      // [cout_true] or null
    int cout_true;
    int act;
    const uint16_t* skip;   // [D][H][W][cout] or null
    uint16_t* ya;           // activation before the skip (null: not kept)
    uint16_t* y;            // bfloat16 output (null: none)
    float* yf;              // FP32 output (null: none)
    int accum;              // yf += result
};

template <int NT>
__global__ __launch_bounds__(256) void conv_fwd_kernel(ConvArgs a) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int chunks = (a.W + 63) / 64;
    const int pr = blockIdx.x / chunks;                     // plane * H + row
    const int plane = pr / a.H, row = pr % a.H;
    const int c0 = (blockIdx.x % chunks) * 64 + wv * 16;
    const int co0 = blockIdx.y * 64;
    if (c0 >= a.W || plane >= a.D) return;                  // no block-wide synchronisation below
    const int ntn = min(4, (a.cout - co0) / 16);
    const int m = lane & 15, kq = lane >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int Hi = a.H / a.xs, Wi = a.W / a.xs;
    const int ncb = a.cin / 16;
    for (int t = 0; t < NT; ++t) {
        int dp, dr, dc;
        tap_offset<NT>(t, dp, dr, dc);
        const int p = plane + dp, r = row + dr;
        if (p < 0 || p >= a.D || r < 0 || r >= a.H) continue;
        const int col = c0 + m + dc;
        const bool ok = col >= 0 && col < a.W;
        const uint16_t* src = a.x + (((size_t)(p / a.xs) * Hi + r / a.xs) * Wi + (ok ? col / a.xs : 0)) * a.cin + kq * 4;
        const uint16_t* wt = a.w + ((size_t)t * a.cout + co0 + m) * a.cin + kq * 4;
        for (int cb = 0; cb < ncb; ++cb) {
            bf16x4 A = ok ? *(const bf16x4*)(src + cb * 16) : bf16x4{0, 0, 0, 0};
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                if (nt < ntn) {
                    const bf16x4 B = *(const bf16x4*)(wt + (size_t)nt * 16 * a.cin + cb * 16);
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[nt], 0, 0, 0);
                }
            }
        }
    }
    // lane holds D[4 kq + i][m]: pixel c0 + 4 kq + i, channel co0 + 16 nt + m
    const size_t rowbase = ((size_t)plane * a.H + row) * a.W;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        if (nt >= ntn) break;
        const int co = co0 + nt * 16 + m;
        const float b = (a.bias && co < a.cout_true) ? a.bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int col = c0 + kq * 4 + i;
            if (col >= a.W) continue;
            const size_t o = (rowbase + col) * a.cout + co;
            float v = acc[nt][i] + b;
            if (a.act) v = v > 0.f ? v : kSlope * v;
            if (a.ya) a.ya[o] = f2bf(v);
            if (a.skip) v += bf2f(a.skip[o]);
            if (a.y) a.y[o] = f2bf(v);
            if (a.yf) a.yf[o] = a.accum ? a.yf[o] + v : v;
        }
    }
}

// Partial weight gradient of one block: for its pixel rows and one (tap,
// 16-channel output tile), sum over pixels p of dz[p][co] x(p + o_t)[ci] (x
// read with upsampling xs), stored as part[(by gx + bx) 16 + co_local][cin].
struct WgradArgs {
    const uint16_t* x; int xs;
    const uint16_t* dz;
    int D, H, W, cin, cout;
    int rows_per_block;     // of the D H image rows
    float* part;
};

template <int NT>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(WgradArgs a) {
    __shared__ float red[4][8][64 * 4];      // [wave][ci tile][lane * 4 + i]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cot = a.cout / 16;
    const int t = blockIdx.y / cot, co0 = (blockIdx.y % cot) * 16;
    int dp, dr, dc;
    tap_offset<NT>(t, dp, dr, dc);
    const int m = lane & 15, kq = lane >> 4;
    const int nct = a.cin / 16;
    const int Hi = a.H / a.xs, Wi = a.W / a.xs;
    f32x4 acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nrows = a.D * a.H;
    const int r0 = blockIdx.x * a.rows_per_block;
    const int r1 = min(nrows, r0 + a.rows_per_block);
    const int cpr = (a.W + 15) / 16;                   // 16-pixel chunks per row
    const int nchunk = max(0, r1 - r0) * cpr;
    for (int q = wv; q < nchunk; q += 4) {
        const int prow = r0 + q / cpr, cb0 = (q % cpr) * 16;
        const int plane = prow / a.H, row = prow % a.H;
        bf16x4 A;
        const int ps = plane + dp, rs = row + dr;
        const bool rok = ps >= 0 && ps < a.D && rs >= 0 && rs < a.H;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = cb0 + kq * 4 + j;
            A[j] = col < a.W ? (short)a.dz[((size_t)prow * a.W + col) * a.cout + co0 + m] : (short)0;
        }
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) {
            if (ct >= nct) break;
            bf16x4 B;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = cb0 + kq * 4 + j, cs = col + dc;
                const bool ok = rok && col < a.W && cs >= 0 && cs < a.W;
                B[j] = ok ? (short)a.x[(((size_t)(ps / a.xs) * Hi + rs / a.xs) * Wi + cs / a.xs) * a.cin + ct * 16 + m]
                          : (short)0;
            }
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[ct], 0, 0, 0);
        }
    }
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
        if (ct >= nct) break;
#pragma unroll
        for (int i = 0; i < 4; ++i) red[wv][ct][lane * 4 + i] = acc[ct][i];
    }
    __syncthreads();
    // D[4 kq + i][m] of tile ct = dW[co0 + 4 kq + i][16 ct + m]
    float* out = a.part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 16 * a.cin;
    for (int e = threadIdx.x; e < nct * 256; e += 256) {
        const int ct = e / 256, li = e % 256, l = li / 4, i = li % 4;
        const float v = ((red[0][ct][li] + red[1][ct][li]) + red[2][ct][li]) + red[3][ct][li];
        out[(size_t)(4 * (l >> 4) + i) * a.cin + ct * 16 + (l & 15)] = v;
    }
}

// gw[t][co][ci] = sum over the blocks bx (in order) of their partials
__global__ void wgrad_reduce_kernel(const float* __restrict__ part, int gx, int T, int cin, int cout, int cin_true,
                                    int cout_true, float* __restrict__ gw) {
    const int64_t total = (int64_t)T * cout_true * cin_true;
    const int cot = cout / 16;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(i % cin_true);
        const int co = (int)((i / cin_true) % cout_true);
        const int t = (int)(i / ((int64_t)cin_true * cout_true));
        const int by = t * cot + co / 16;
        const float* p = part + ((size_t)by * gx * 16 + (co % 16)) * cin + ci;
        float s = 0.f;
        for (int bx = 0; bx < gx; ++bx) s += p[(size_t)bx * 16 * cin];
        gw[i] = s;
    }
}

// per-block channel sums of dz over a fixed pixel range: part[bx][c]
__global__ __launch_bounds__(256) void bias_grad_kernel(const uint16_t* dz, int64_t npix, int cout, float* part) {
    __shared__ float sh[256];
    const int c = threadIdx.x % cout;
    const int nsub = 256 / cout;
    const int sub = threadIdx.x / cout;
    float s = 0.f;
    if (sub < nsub) {
        const int64_t per = (npix + gridDim.x - 1) / gridDim.x;
        const int64_t p0 = (int64_t)blockIdx.x * per, p1 = min(npix, p0 + per);
        for (int64_t p = p0 + sub; p < p1; p += nsub) s += bf2f(dz[p * cout + c]);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < cout) {
        float t = 0.f;
        for (int k = 0; k < nsub; ++k) t += sh[k * cout + threadIdx.x];
        part[(size_t)blockIdx.x * cout + threadIdx.x] = t;
    }
}

__global__ void bias_reduce_kernel(const float* __restrict__ part, int nb, int cout, int cout_true,
                                   float* __restrict__ gb) {
    const int c = threadIdx.x;
    if (c >= cout_true) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * cout + c];
    gb[c] = s;
}

// ---------------------------------------------------------------------------
// element-wise kernels
// Image geometry shared by the element-wise kernels: padded extents and the
// mesh's node counts per axis (planes = ix, rows = iz in 3D / ix in 2D,
// columns = iy).
struct Img {
    int dim, D0, H0, W0;                  // padded extents (D0 = 1 in 2D)
    int nelx, nely, nelz;
};

template <typename T>
__global__ void prep_input_kernel(Img g, const T* __restrict__ xt, const double* __restrict__ f,
                                  uint16_t* __restrict__ x0, int64_t npix) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
        const int iy = (int)(p % g.W0);
        const int64_t pr = p / g.W0;
        float v[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = 0.f;
        if (g.dim == 2) {
            const int ix = (int)pr;
            if (ix <= g.nelx && iy <= g.nely) {
                double sm = 0.0;
                int n = 0;
                for (int ax = -1; ax <= 0; ++ax)
                    for (int ay = -1; ay <= 0; ++ay) {
                        const int ex = ix + ax, ey = iy + ay;
                        if (ex >= 0 && ex < g.nelx && ey >= 0 && ey < g.nely) {
                            sm += (double)xt[ey + (int64_t)g.nely * ex];
                            ++n;
                        }
                    }
                const int64_t node = iy + (int64_t)(g.nely + 1) * ix;
                v[0] = (float)(sm / n);
                v[1] = (float)f[2 * node];
                v[2] = (float)f[2 * node + 1];
            }
        } else {
            const int iz = (int)(pr % g.H0), ix = (int)(pr / g.H0);
            if (ix <= g.nelx && iz <= g.nelz && iy <= g.nely) {
                double sm = 0.0;
                int n = 0;
                for (int ax = -1; ax <= 0; ++ax)
                    for (int az = -1; az <= 0; ++az)
                        for (int ay = -1; ay <= 0; ++ay) {
                            const int ex = ix + ax, ez = iz + az, ey = iy + ay;
                            if (ex >= 0 && ex < g.nelx && ez >= 0 && ez < g.nelz && ey >= 0 && ey < g.nely) {
                                sm += (double)xt[ey + (int64_t)g.nely * (ez + (int64_t)g.nelz * ex)];
                                ++n;
                            }
                        }
                const int64_t node = iy + (int64_t)(g.nely + 1) * (iz + (int64_t)(g.nelz + 1) * ix);
                v[0] = (float)(sm / n);
                v[1] = (float)f[3 * node];
                v[2] = (float)f[3 * node + 1];
                v[3] = (float)f[3 * node + 2];
            }
        }
        uint16_t* o = x0 + p * 16;
#pragma unroll
        for (int c = 0; c < 16; ++c) o[c] = f2bf(v[c]);
    }
}

// average pooling of [D][H][W][C] (D, H, W: the input extents; the plane
// axis is pooled too in 3D); corner order: plane, row, column
__global__ void pool_kernel(const uint16_t* __restrict__ in, int dim, int D, int H, int W, int C,
                            uint16_t* __restrict__ out) {
    const int Do = dim == 3 ? D / 2 : 1, Ho = H / 2, Wo = W / 2;
    const int nd = dim == 3 ? 2 : 1;
    const float scale = dim == 3 ? 0.125f : 0.25f;
    const int64_t total = (int64_t)Do * Ho * Wo * C;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        const int w = (int)(p % Wo);
        const int64_t q = p / Wo;
        const int h = (int)(q % Ho), d = (int)(q / Ho);
        float s = 0.f;
        bool first = true;
        for (int a = 0; a < nd; ++a)
            for (int b = 0; b < 2; ++b)
                for (int e = 0; e < 2; ++e) {
                    const float v = bf2f(in[(((size_t)(nd * d + a) * H + 2 * h + b) * W + 2 * w + e) * C + c]);
                    s = first ? v : s + v;
                    first = false;
                }
        out[i] = f2bf(scale * s);
    }
}

// dz = bf16(g * leaky'(a)) (act) or bf16(g)
__global__ void act_bwd_kernel(const float* __restrict__ g, const uint16_t* __restrict__ a, int act, int64_t n,
                               uint16_t* __restrict__ dz) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float v = g[i];
        if (act && !(bf2f(a[i]) > 0.f)) v *= kSlope;
        dz[i] = f2bf(v);
    }
}

// g_prev[d][h][w] += s[d/2][h/2][w/2] / 2^dim  (gradient through the average
// pooling; D, H, W: the full-size extents)
__global__ void unpool_add_kernel(const float* __restrict__ s, int dim, int D, int H, int W, int C,
                                  float* __restrict__ g) {
    const int64_t total = (int64_t)D * H * W * C;
    const bool d3 = dim == 3;
    const float scale = d3 ? 0.125f : 0.25f;
    const int Hh = H / 2, Wh = W / 2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        const int w = (int)(p % W);
        const int64_t q = p / W;
        const int h = (int)(q % H), d = (int)(q / H);
        const int dh = d3 ? d / 2 : 0;
        g[i] += scale * s[(((size_t)dh * Hh + h / 2) * Wh + w / 2) * C + c];
    }
}

// g_prev[d][h][w] += sum of s over its 2x2 (2x2x2) block (gradient through
// the upsampling; D, H, W: the half-size extents)
__global__ void sumpool_add_kernel(const float* __restrict__ s, int dim, int D, int H, int W, int C,
                                   float* __restrict__ g) {
    const int64_t total = (int64_t)D * H * W * C;
    const bool d3 = dim == 3;
    const int H2 = 2 * H, W2 = 2 * W;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        const int w = (int)(p % W);
        const int64_t q = p / W;
        const int h = (int)(q % H), d = (int)(q / H);
        float acc = 0.f;
        bool first = true;
        for (int a = 0; a < (d3 ? 2 : 1); ++a)
            for (int b = 0; b < 2; ++b)
                for (int e = 0; e < 2; ++e) {
                    const size_t src = (((size_t)((d3 ? 2 * d : d) + a) * H2 + 2 * h + b) * W2 + 2 * w + e) * C + c;
                    acc = first ? s[src] : acc + s[src];
                    first = false;
                }
        g[i] += acc;
    }
}

__global__ void add_kernel(const float* __restrict__ s, int64_t n, float* __restrict__ g) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        g[i] += s[i];
}

__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// block partials of sum u^2 over a fixed range per block: part[bx]
__global__ __launch_bounds__(256) void sumsq_kernel(const double* __restrict__ u, int64_t n, double* part) {
    __shared__ double sh[kWaves];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(n, i0 + per);
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) s += u[i] * u[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[0] = sum of the nb partials in block order
__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ part, int nb, double* out) {
    __shared__ double sh[kWaves];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) s += part[b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *out = s;
}

// mean squared error against u / rms(u) over real nodes (block partials of
// the loss into part[bx]) and its gradient image
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ out, const double* __restrict__ u, Img g,
                                                   int64_t npix, const double* sumsq, int64_t n,
                                                   float* __restrict__ gout, double* part) {
    __shared__ double sh[kWaves];
    const double rms = sqrt(*sumsq / (double)n);
    const double inv = rms > 0.0 ? 1.0 / rms : 1.0;
    const int nc = g.dim;
    const double cnt = (double)n;                       // real nodes x components
    const int64_t per = (npix + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * per, p1 = min(npix, p0 + per);
    double s = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += kBlock) {
        const int iy = (int)(p % g.W0);
        const int64_t pr = p / g.W0;
        bool real;
        int64_t node;
        if (g.dim == 2) {
            const int ix = (int)pr;
            real = ix <= g.nelx && iy <= g.nely;
            node = iy + (int64_t)(g.nely + 1) * ix;
        } else {
            const int iz = (int)(pr % g.H0), ix = (int)(pr / g.H0);
            real = ix <= g.nelx && iz <= g.nelz && iy <= g.nely;
            node = iy + (int64_t)(g.nely + 1) * (iz + (int64_t)(g.nelz + 1) * ix);
        }
        for (int c = 0; c < nc; ++c) {
            double d = 0.0;
            if (real) d = (double)out[p * 16 + c] - u[(int64_t)nc * node + c] * inv;
            s += d * d;
            gout[p * 16 + c] = (float)(2.0 * d / cnt);
        }
        for (int c = nc; c < 16; ++c) gout[p * 16 + c] = 0.f;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s / cnt;
}

__global__ void out_to_dofs_kernel(const float* __restrict__ out, Img g, const uint8_t* __restrict__ freem,
                                   double* __restrict__ uh) {
    const int64_t nn = (int64_t)(g.nelx + 1) * (g.nely + 1) * (g.dim == 3 ? g.nelz + 1 : 1);
    const int nc = g.dim;
    for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < nn; node += (int64_t)gridDim.x * blockDim.x) {
        const int64_t iy = node % (g.nely + 1), rest = node / (g.nely + 1);
        int64_t p;
        if (g.dim == 2) p = rest * g.W0 + iy;
        else {
            const int64_t iz = rest % (g.nelz + 1), ix = rest / (g.nelz + 1);
            p = (ix * g.H0 + iz) * g.W0 + iy;
        }
        for (int c = 0; c < nc; ++c) {
            const int64_t i = (int64_t)nc * node + c;
            uh[i] = freem[i] ? (double)out[p * 16 + c] : 0.0;
        }
    }
}

// Adam with bias correction on the FP32 master vector
__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ mo, float* __restrict__ ve,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * mo[i] + (1.f - b1) * gi;
        const float vi = b2 * ve[i] + (1.f - b2) * gi * gi;
        mo[i] = mi;
        ve[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// bfloat16 weight copies of one layer: forward [T][cout_p][cin_p] and the
// flipped-transposed [T][cin_p][cout_p] for the input gradient
__global__ void pack_weights_kernel(const float* __restrict__ w, int T, int cin, int cout, int cin_p, int cout_p,
                                    uint16_t* __restrict__ wf, uint16_t* __restrict__ wb) {
    const int64_t total = (int64_t)T * cin_p * cout_p;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(i % cin_p);
        const int co = (int)((i / cin_p) % cout_p);
        const int t = (int)(i / ((int64_t)cin_p * cout_p));
        const uint16_t v = (ci < cin && co < cout) ? f2bf(w[((size_t)t * cout + co) * cin + ci]) : (uint16_t)0;
        wf[i] = v;
        wb[((size_t)(T - 1 - t) * cin_p + ci) * cout_p + co] = v;
    }
}

// ---------------------------------------------------------------------------
// host side
struct LayerBuf {
    int cin, cout, cin_p, cout_p, level, act, src, skip;
    int64_t w_off, b_off;              // in the master vector
    uint16_t *wf, *wb;                 // bfloat16 copies
    uint16_t *y, *a;                   // output (after skip) and activation before the skip
    float* g;                          // gradient of the output
};

struct Nn {
    const Plan* plan = nullptr;
    Img img{};
    int T = 9;                         // taps per convolution
    int64_t P = 0;
    LayerBuf L[kNL];
    float *master = nullptr, *mom = nullptr, *vel = nullptr, *grad = nullptr;
    uint16_t* x0 = nullptr;
    uint16_t* pooled[4] = {};          // pooled inputs of levels 1..3
    float* out = nullptr;              // final layer output (FP32, 16 channels)
    float* gtmp = nullptr;             // input-gradient staging
    uint16_t* dz = nullptr;            // bfloat16 error signal staging
    float* wpart = nullptr;            // per-block weight-gradient partials
    float* bpart = nullptr;            // per-block bias-gradient partials
    double* dpart = nullptr;           // per-block partials of the FP64 sums
    double* scal = nullptr;            // [0] sum u^2, [1] loss
    int64_t step = 0;
    // extents of level l
    int D(int l) const { return img.dim == 3 ? img.D0 >> l : 1; }
    int H(int l) const { return img.H0 >> l; }
    int W(int l) const { return img.W0 >> l; }
    int64_t px(int l) const { return (int64_t)D(l) * H(l) * W(l); }
    int64_t nodes() const {
        return (int64_t)(img.nelx + 1) * (img.nely + 1) * (img.dim == 3 ? img.nelz + 1 : 1);
    }
};

static int grid_for(int64_t n, int block = 256) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + block - 1) / block));
}

struct NnLayout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    }
};

// launch shape of a layer's weight-gradient kernel: (blocks over image rows,
// rows per block); blocks over (tap, output tile) = T cout_p / 16
static void wgrad_shape(const Nn& nn, int level, int cout_p, int& gx, int& rows) {
    const int nrows = nn.D(level) * nn.H(level);
    const int tiles = nn.T * (cout_p / 16);
    const int want_blocks = 2048;
    rows = (int)std::max<int64_t>(1, ((int64_t)nrows * tiles + want_blocks - 1) / want_blocks);
    gx = (nrows + rows - 1) / rows;
}

static Img make_img(int dim, int nelx, int nely, int nelz) {
    Img g{};
    g.dim = dim;
    g.nelx = nelx; g.nely = nely; g.nelz = dim == 3 ? nelz : 1;
    const auto p8 = [](int n) { return (n + 1 + 7) / 8 * 8; };
    if (dim == 2) { g.D0 = 1; g.H0 = p8(nelx); g.W0 = p8(nely); }
    else { g.D0 = p8(nelx); g.H0 = p8(nelz); g.W0 = p8(nely); }
    return g;
}

static size_t nn_layout(int dim, int nelx, int nely, int nelz, Nn* out, char* base) {
    Nn nn;
    nn.img = make_img(dim, nelx, nely, nelz);
    nn.T = dim == 2 ? 9 : 27;
    const LayerDef* defs = layer_defs(dim);
    NnLayout Ly;
    int64_t P = 0;
    int64_t woff[kNL], boff[kNL];
    for (int i = 0; i < kNL; ++i) {
        woff[i] = P;
        P += (int64_t)nn.T * defs[i].cin * defs[i].cout;
        boff[i] = P;
        P += defs[i].cout;
    }
    // staging sizes: the largest image a layer reads or writes, and the
    // largest weight-gradient partial set
    int64_t stage = 0;
    size_t wpart = 0;
    for (int i = 0; i < kNL; ++i) {
        const int ci = pad16(defs[i].cin), co = pad16(defs[i].cout);
        stage = std::max(stage, nn.px(defs[i].level) * std::max(ci, co));
        int gx, rows;
        wgrad_shape(nn, defs[i].level, co, gx, rows);
        wpart = std::max(wpart, (size_t)gx * nn.T * (co / 16) * 16 * ci);
    }
    size_t o_master = Ly.take(4 * P), o_m = Ly.take(4 * P), o_v = Ly.take(4 * P), o_g = Ly.take(4 * P);
    size_t o_x0 = Ly.take(2 * nn.px(0) * 16);
    size_t o_pool[4] = {0, 0, 0, 0};
    for (int l = 1; l < 4; ++l) {
        int c = 16;
        for (int i = 0; i < kNL; ++i)
            if (defs[i].src == 1 && defs[i].level == l) c = pad16(defs[i - 1].cout);
        o_pool[l] = Ly.take(2 * nn.px(l) * c);
    }
    size_t o_out = Ly.take(4 * nn.px(0) * 16);
    size_t o_gtmp = Ly.take(4 * stage);
    size_t o_dz = Ly.take(2 * stage);
    size_t o_wpart = Ly.take(4 * wpart);
    size_t o_bpart = Ly.take(4 * (size_t)kRedBlocks * 128);
    size_t o_dpart = Ly.take(8 * (size_t)kRedBlocks);
    size_t o_scal = Ly.take(64);
    size_t o_wf[kNL], o_wb[kNL], o_y[kNL], o_a[kNL], o_gl[kNL];
    for (int i = 0; i < kNL; ++i) {
        const LayerDef& d = defs[i];
        const int ci = pad16(d.cin), co = pad16(d.cout);
        o_wf[i] = Ly.take(2 * (size_t)nn.T * ci * co);
        o_wb[i] = Ly.take(2 * (size_t)nn.T * ci * co);
        o_y[i] = i == kNL - 1 ? 0 : Ly.take(2 * nn.px(d.level) * co);
        o_a[i] = d.skip >= 0 ? Ly.take(2 * nn.px(d.level) * co) : 0;
        o_gl[i] = Ly.take(4 * nn.px(d.level) * co);
    }
    if (out && base) {
        Nn& r = *out;
        r.img = nn.img; r.T = nn.T; r.P = P;
        r.master = (float*)(base + o_master); r.mom = (float*)(base + o_m);
        r.vel = (float*)(base + o_v); r.grad = (float*)(base + o_g);
        r.x0 = (uint16_t*)(base + o_x0);
        for (int l = 1; l < 4; ++l) r.pooled[l] = (uint16_t*)(base + o_pool[l]);
        r.out = (float*)(base + o_out);
        r.gtmp = (float*)(base + o_gtmp);
        r.dz = (uint16_t*)(base + o_dz);
        r.wpart = (float*)(base + o_wpart);
        r.bpart = (float*)(base + o_bpart);
        r.dpart = (double*)(base + o_dpart);
        r.scal = (double*)(base + o_scal);
        for (int i = 0; i < kNL; ++i) {
            const LayerDef& d = defs[i];
            LayerBuf& b = r.L[i];
            b.cin = d.cin; b.cout = d.cout; b.cin_p = pad16(d.cin); b.cout_p = pad16(d.cout);
            b.level = d.level; b.act = d.act; b.src = d.src; b.skip = d.skip;
            b.w_off = woff[i]; b.b_off = boff[i];
            b.wf = (uint16_t*)(base + o_wf[i]);
            b.wb = (uint16_t*)(base + o_wb[i]);
            b.y = i == kNL - 1 ? nullptr : (uint16_t*)(base + o_y[i]);
            b.a = d.skip >= 0 ? (uint16_t*)(base + o_a[i]) : b.y;
            b.g = (float*)(base + o_gl[i]);
        }
    }
    return Ly.off;
}

static int64_t nn_param_count(int dim) {
    const LayerDef* defs = layer_defs(dim);
    const int T = dim == 2 ? 9 : 27;
    int64_t P = 0;
    for (int i = 0; i < kNL; ++i) P += (int64_t)T * defs[i].cin * defs[i].cout + defs[i].cout;
    return P;
}

static void conv_launch(const Nn* nn, const ConvArgs& a, hipStream_t s) {
    dim3 grid((unsigned)(a.D * a.H * ((a.W + 63) / 64)), (unsigned)((a.cout + 63) / 64));
    if (nn->T == 9) hipLaunchKernelGGL(conv_fwd_kernel<9>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(conv_fwd_kernel<27>, grid, dim3(256), 0, s, a);
}

// the input a layer reads (and the upsampling factor of that read)
static const uint16_t* layer_input(const Nn* nn, int i, int& xs) {
    const LayerBuf& b = nn->L[i];
    xs = 1;
    if (i == 0) return nn->x0;
    if (b.src == 1) return nn->pooled[b.level];
    if (b.src == 2) xs = 2;
    return nn->L[i - 1].y;
}

static to_status nn_forward(Nn* nn, to_dtype dt, const void* xt, const double* f, hipStream_t s) {
    const int64_t npix0 = nn->px(0);
    if (dt == TO_F64)
        hipLaunchKernelGGL(prep_input_kernel<double>, dim3(grid_for(npix0)), dim3(256), 0, s, nn->img,
                           (const double*)xt, f, nn->x0, npix0);
    else
        hipLaunchKernelGGL(prep_input_kernel<float>, dim3(grid_for(npix0)), dim3(256), 0, s, nn->img,
                           (const float*)xt, f, nn->x0, npix0);
    const int dim = nn->img.dim;
    for (int i = 0; i < kNL; ++i) {
        LayerBuf& b = nn->L[i];
        const int l = b.level;
        if (b.src == 1) {
            const LayerBuf& pv = nn->L[i - 1];
            const int64_t tot = nn->px(l) * pv.cout_p;
            hipLaunchKernelGGL(pool_kernel, dim3(grid_for(tot)), dim3(256), 0, s, pv.y, dim, nn->D(l - 1), nn->H(l - 1),
                               nn->W(l - 1), pv.cout_p, nn->pooled[l]);
        }
        ConvArgs a{};
        a.x = layer_input(nn, i, a.xs);
        a.D = nn->D(l); a.H = nn->H(l); a.W = nn->W(l); a.cin = b.cin_p; a.cout = b.cout_p;
        a.w = b.wf;
        a.bias = nn->master + b.b_off;
        a.cout_true = b.cout;
        a.act = b.act;
        a.skip = b.skip >= 0 ? nn->L[b.skip].y : nullptr;
        a.ya = b.skip >= 0 ? b.a : nullptr;
        a.y = b.y;
        a.yf = i == kNL - 1 ? nn->out : nullptr;
        a.accum = 0;
        conv_launch(nn, a, s);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

static void zero_f32(float* p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, 0.f);
}

// loss and gradient of every weight for the sample the last forward pass saw
static to_status nn_backward(Nn* nn, const double* u, hipStream_t s) {
    const int64_t npix0 = nn->px(0);
    const int64_t n = (int64_t)nn->img.dim * nn->nodes();
    const int dim = nn->img.dim;
    hipLaunchKernelGGL(sumsq_kernel, dim3(kRedBlocks), dim3(kBlock), 0, s, u, n, nn->dpart);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kBlock), 0, s, nn->dpart, kRedBlocks, nn->scal);
    for (int i = 0; i < kNL - 1; ++i) {
        const LayerBuf& b = nn->L[i];
        zero_f32(b.g, nn->px(b.level) * b.cout_p, s);
    }
    LayerBuf& lo = nn->L[kNL - 1];
    hipLaunchKernelGGL(loss_kernel, dim3(kRedBlocks), dim3(kBlock), 0, s, nn->out, u, nn->img, npix0, nn->scal, n,
                       lo.g, nn->dpart);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kBlock), 0, s, nn->dpart, kRedBlocks, nn->scal + 1);
    for (int i = kNL - 1; i >= 0; --i) {
        LayerBuf& b = nn->L[i];
        const int l = b.level;
        const int64_t npix = nn->px(l), ne = npix * b.cout_p;
        if (b.skip >= 0)
            hipLaunchKernelGGL(add_kernel, dim3(grid_for(ne)), dim3(256), 0, s, b.g, ne, nn->L[b.skip].g);
        hipLaunchKernelGGL(act_bwd_kernel, dim3(grid_for(ne)), dim3(256), 0, s, b.g, b.a, b.act, ne, nn->dz);
        // weight and bias gradients: block partials, then ordered sums
        WgradArgs w{};
        w.x = layer_input(nn, i, w.xs);
        w.dz = nn->dz;
        w.D = nn->D(l); w.H = nn->H(l); w.W = nn->W(l); w.cin = b.cin_p; w.cout = b.cout_p;
        int gx, rows;
        wgrad_shape(*nn, l, b.cout_p, gx, rows);
        w.rows_per_block = rows;
        w.part = nn->wpart;
        const int tiles = nn->T * (b.cout_p / 16);
        if (nn->T == 9) hipLaunchKernelGGL(conv_wgrad_kernel<9>, dim3(gx, tiles), dim3(256), 0, s, w);
        else hipLaunchKernelGGL(conv_wgrad_kernel<27>, dim3(gx, tiles), dim3(256), 0, s, w);
        const int64_t nw = (int64_t)nn->T * b.cout * b.cin;
        hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(grid_for(nw)), dim3(256), 0, s, nn->wpart, gx, nn->T, b.cin_p,
                           b.cout_p, b.cin, b.cout, nn->grad + b.w_off);
        hipLaunchKernelGGL(bias_grad_kernel, dim3(kRedBlocks), dim3(256), 0, s, nn->dz, npix, b.cout_p, nn->bpart);
        hipLaunchKernelGGL(bias_reduce_kernel, dim3(1), dim3(128), 0, s, nn->bpart, kRedBlocks, b.cout_p, b.cout,
                           nn->grad + b.b_off);
        if (i == 0) break;
        // input gradient: correlation with the flipped, transposed kernel
        LayerBuf& pv = nn->L[i - 1];
        ConvArgs a{};
        a.x = nn->dz; a.xs = 1;
        a.D = nn->D(l); a.H = nn->H(l); a.W = nn->W(l); a.cin = b.cout_p; a.cout = b.cin_p;
        a.w = b.wb;
        a.cout_true = b.cin;
        a.act = 0;
        if (b.src == 0) {
            a.yf = pv.g; a.accum = 1;
            conv_launch(nn, a, s);
        } else {
            a.yf = nn->gtmp; a.accum = 0;
            conv_launch(nn, a, s);
            if (b.src == 1) {       // through the pooling: the previous level is twice the size
                const int64_t tot = nn->px(l - 1) * pv.cout_p;
                hipLaunchKernelGGL(unpool_add_kernel, dim3(grid_for(tot)), dim3(256), 0, s, nn->gtmp, dim,
                                   nn->D(l - 1), nn->H(l - 1), nn->W(l - 1), pv.cout_p, pv.g);
            } else {                // through the upsampling: the previous level is half the size
                const int64_t tot = nn->px(l + 1) * pv.cout_p;
                hipLaunchKernelGGL(sumpool_add_kernel, dim3(grid_for(tot)), dim3(256), 0, s, nn->gtmp, dim,
                                   nn->D(l + 1), nn->H(l + 1), nn->W(l + 1), pv.cout_p, pv.g);
            }
        }
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

static to_status nn_pack(Nn* nn, hipStream_t s) {
    for (int i = 0; i < kNL; ++i) {
        LayerBuf& b = nn->L[i];
        const int64_t tot = (int64_t)nn->T * b.cin_p * b.cout_p;
        hipLaunchKernelGGL(pack_weights_kernel, dim3(grid_for(tot)), dim3(256), 0, s, nn->master + b.w_off, nn->T,
                           b.cin, b.cout, b.cin_p, b.cout_p, b.wf, b.wb);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

}  // namespace topt

// ---------------------------------------------------------------------------
// C ABI
using namespace topt;

struct to_nn {
    Nn impl;
};

static void set_err(const char* m) { topt::set_error(m); }

extern "C" {

to_status to_nn_query(int32_t dim, int32_t nelx, int32_t nely, int32_t nelz, size_t* ws_bytes, int64_t* n_params) {
    if ((dim != 2 && dim != 3) || nelx < 1 || nely < 1 || (dim == 3 && nelz < 1) || !ws_bytes) {
        set_err("to_nn_query: bad dimension or size, or NULL ws_bytes");
        return TO_EINVAL;
    }
    const int64_t pix = (int64_t)(nelx + 8) * (nely + 8) * (dim == 3 ? nelz + 8 : 1);
    if (pix > (int64_t)1 << 28) { set_err("to_nn_query: mesh too large"); return TO_EINVAL; }
    *ws_bytes = nn_layout(dim, nelx, nely, nelz, nullptr, nullptr);
    if (n_params) *n_params = nn_param_count(dim);
    return TO_OK;
}

to_status to_nn_create(const to_plan* plan, void* ws, size_t ws_bytes, to_nn** out) {
    if (!plan || !ws || !out) { set_err("to_nn_create: NULL argument"); return TO_EINVAL; }
    const Plan* p = topt::P(plan);
    if (((uintptr_t)ws & 255u) != 0) { set_err("to_nn_create: workspace not 256-byte aligned"); return TO_EINVAL; }
    size_t need = nn_layout(p->dim, p->nelx, p->nely, p->nelz, nullptr, nullptr);
    if (ws_bytes < need) { set_err("to_nn_create: workspace too small"); return TO_EWORKSPACE; }
    to_nn* h = new (std::nothrow) to_nn;
    if (!h) { set_err("to_nn_create: out of host memory"); return TO_EINVAL; }
    h->impl.plan = p;
    nn_layout(p->dim, p->nelx, p->nely, p->nelz, &h->impl, (char*)ws);
    *out = h;
    return TO_OK;
}

void to_nn_destroy(to_nn* nn) { delete nn; }

to_status to_nn_set_params(to_nn* h, const float* params, void* stream) {
    if (!h || !params) { set_err("to_nn_set_params: NULL argument"); return TO_EINVAL; }
    Nn* nn = &h->impl;
    hipStream_t s = (hipStream_t)stream;
    TO_HIP(hipMemcpyAsync(nn->master, params, 4 * nn->P, hipMemcpyDeviceToDevice, s));
    zero_f32(nn->mom, nn->P, s);
    zero_f32(nn->vel, nn->P, s);
    nn->step = 0;
    return nn_pack(nn, s);
}

to_status to_nn_get(const to_nn* h, int what, void* out, void* stream) {
    if (!h || !out) { set_err("to_nn_get: NULL argument"); return TO_EINVAL; }
    const Nn* nn = &h->impl;
    hipStream_t s = (hipStream_t)stream;
    if (what == TO_NN_PARAMS) {
        TO_HIP(hipMemcpyAsync(out, nn->master, 4 * nn->P, hipMemcpyDeviceToDevice, s));
    } else if (what == TO_NN_GRAD) {
        TO_HIP(hipMemcpyAsync(out, nn->grad, 4 * nn->P, hipMemcpyDeviceToDevice, s));
    } else if (what == TO_NN_OUTPUT) {
        TO_HIP(hipMemcpyAsync(out, nn->out, 4 * nn->px(0) * 16, hipMemcpyDeviceToDevice, s));
    } else if (what >= TO_NN_ACT && what < TO_NN_ACT + kNL - 1) {
        const LayerBuf& b = nn->L[what - TO_NN_ACT];
        TO_HIP(hipMemcpyAsync(out, b.y, 2 * nn->px(b.level) * b.cout_p, hipMemcpyDeviceToDevice, s));
    } else if (what >= TO_NN_PRESKIP && what < TO_NN_PRESKIP + kNL - 1 && nn->L[what - TO_NN_PRESKIP].skip >= 0) {
        const LayerBuf& b = nn->L[what - TO_NN_PRESKIP];
        TO_HIP(hipMemcpyAsync(out, b.a, 2 * nn->px(b.level) * b.cout_p, hipMemcpyDeviceToDevice, s));
    } else {
        set_err("to_nn_get: unknown item");
        return TO_EINVAL;
    }
    return TO_OK;
}

to_status to_nn_forward(to_nn* h, to_dtype dtype, const void* xtilde, const double* f, double* uhat, void* stream) {
    if (!h || !xtilde || !f) { set_err("to_nn_forward: NULL argument"); return TO_EINVAL; }
    if (dtype != TO_F32 && dtype != TO_F64) { set_err("to_nn_forward: bad dtype"); return TO_EINVAL; }
    Nn* nn = &h->impl;
    hipStream_t s = (hipStream_t)stream;
    to_status r = nn_forward(nn, dtype, xtilde, f, s);
    if (r != TO_OK) return r;
    if (uhat) {
        hipLaunchKernelGGL(out_to_dofs_kernel, dim3(grid_for(nn->nodes())), dim3(256), 0, s, nn->out, nn->img,
                           nn->plan->freemask, uhat);
        TO_HIP(hipGetLastError());
    }
    return TO_OK;
}

to_status to_nn_backward(to_nn* h, const double* u, double* d_loss, void* stream) {
    if (!h || !u) { set_err("to_nn_backward: NULL argument"); return TO_EINVAL; }
    Nn* nn = &h->impl;
    hipStream_t s = (hipStream_t)stream;
    to_status r = nn_backward(nn, u, s);
    if (r != TO_OK) return r;
    if (d_loss) TO_HIP(hipMemcpyAsync(d_loss, nn->scal + 1, 8, hipMemcpyDeviceToDevice, s));
    return TO_OK;
}

to_status to_nn_adam(to_nn* h, float lr, float beta1, float beta2, float eps, void* stream) {
    if (!h) { set_err("to_nn_adam: NULL handle"); return TO_EINVAL; }
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f)) {
        set_err("to_nn_adam: bad hyper-parameters");
        return TO_EINVAL;
    }
    Nn* nn = &h->impl;
    hipStream_t s = (hipStream_t)stream;
    nn->step += 1;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)nn->step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)nn->step));
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(nn->P)), dim3(256), 0, s, nn->master, nn->mom, nn->vel, nn->grad,
                       nn->P, lr, beta1, beta2, eps, c1, c2);
    TO_HIP(hipGetLastError());
    return nn_pack(nn, s);
}

to_status to_nn_train_step(to_nn* h, to_dtype dtype, const void* xtilde, const double* f, const double* u,
                           float lr, double* d_loss, void* stream) {
    to_status r = to_nn_forward(h, dtype, xtilde, f, nullptr, stream);
    if (r != TO_OK) return r;
    r = to_nn_backward(h, u, d_loss, stream);
    if (r != TO_OK) return r;
    return to_nn_adam(h, lr, 0.9f, 0.999f, 1e-8f, stream);
}

}  // extern "C"
