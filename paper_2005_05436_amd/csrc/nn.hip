// Learned warm start of the state solve: a small U-Net on the node grid that
// maps (filtered density, load) to a displacement direction, with bfloat16
// weights and activations on the matrix cores (FP32 accumulation), its
// backward pass and Adam, all on the GPU.  The paper has no network; the
// prediction only seeds the CG of eq. (5) (see to_warm_start), so the solve's
// own residual still decides the answer.
//
// Image: rows = ix, columns = iy, both padded to multiples of 8, channels
// innermost (NHWC) and padded to multiples of 16, so pixel (ix, iy) holds the
// two DOFs of node iy + (nely + 1) ix.  Layers (c_in -> c_out, level):
//   e1a 3->16 0, e1b 16->16 0 | pool | e2a 16->32 1, e2b 32->32 1 | pool |
//   e3a 32->64 2, e3b 64->64 2 | pool | ba 64->128 3, bb 128->64 3 |
//   up d3a 64->64 2 (+e3b), d3b 64->32 2 | up d2a 32->32 1 (+e2b), d2b 32->16 1 |
//   up d1a 16->16 0 (+e1b), d1b 16->16 0 | out 16->2 0 (no activation)
// 'same' 3x3 cross-correlation (zero padding), bias, leaky ReLU (slope 1/8),
// 2x2 average pooling, nearest 2x upsampling, additive skips.  Weights are
// kept as an FP32 master vector: per layer W[t][co][ci] (t = 3 (dr+1) +
// (dc+1)) then b[co]; the matrix cores read bfloat16 copies, padded
// [9][co][ci] for the forward product and flipped-transposed [9][ci][co] for
// the input gradient.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x16_bf16: a wave owns
// 16 consecutive pixels of one image row and up to 64 output channels (four
// 16x16 accumulators); the K loop runs over the 9 taps and the input
// channels in blocks of 16.  The weight gradient is a GEMM over pixels
// (M = c_out, N = c_in, K = pixels) per tap, reduced across waves in LDS and
// across blocks with FP32 atomics.
#include <cmath>
#include <new>

#include "common.h"

namespace topt {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kSlope = 0.125f;
constexpr int kNL = 15;

struct LayerDef { int cin, cout, level, act, src, skip; };   // src: 0 previous, 1 pool, 2 up
static const LayerDef kLayers[kNL] = {
    {3, 16, 0, 1, 0, -1},  {16, 16, 0, 1, 0, -1},  {16, 32, 1, 1, 1, -1}, {32, 32, 1, 1, 0, -1},
    {32, 64, 2, 1, 1, -1}, {64, 64, 2, 1, 0, -1},  {64, 128, 3, 1, 1, -1}, {128, 64, 3, 1, 0, -1},
    {64, 64, 2, 1, 2, 5},  {64, 32, 2, 1, 0, -1},  {32, 32, 1, 1, 2, 3},  {32, 16, 1, 1, 0, -1},
    {16, 16, 0, 1, 2, 1},  {16, 16, 0, 1, 0, -1},  {16, 2, 0, 0, 0, -1}};

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
struct ConvArgs {
    const uint16_t* x;      // input [H'][W'][cin] (H' = H / xs)
    int xs;                 // 1, or 2 = nearest-upsampled read of a half-size input
    int H, W, cin, cout;    // output size; channel counts padded to 16
    const uint16_t* w;      // [9][cout][cin]
    const float* bias;      // [cout_true] or null
    int cout_true;
    int act;
    const uint16_t* skip;   // [H][W][cout] or null
    uint16_t* ya;           // activation before the skip (null: not kept)
    uint16_t* y;            // bfloat16 output (null: none)
    float* yf;              // FP32 output (null: none)
    int accum;              // yf += result
};

__global__ __launch_bounds__(256) void conv_fwd_kernel(ConvArgs a) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int chunks = (a.W + 63) / 64;
    const int row = blockIdx.x / chunks;
    const int c0 = (blockIdx.x % chunks) * 64 + wv * 16;
    const int co0 = blockIdx.y * 64;
    if (c0 >= a.W || row >= a.H) return;                    // no block-wide synchronisation below
    const int ntn = min(4, (a.cout - co0) / 16);
    const int m = lane & 15, kq = lane >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int Wi = a.W / a.xs;
    const int ncb = a.cin / 16;
    for (int t = 0; t < 9; ++t) {
        const int r = row + t / 3 - 1;
        if (r < 0 || r >= a.H) continue;
        const int col = c0 + m + t % 3 - 1;
        const bool ok = col >= 0 && col < a.W;
        const uint16_t* src = a.x + ((size_t)(r / a.xs) * Wi + (ok ? col / a.xs : 0)) * a.cin + kq * 4;
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
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        if (nt >= ntn) break;
        const int co = co0 + nt * 16 + m;
        const float b = (a.bias && co < a.cout_true) ? a.bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int col = c0 + kq * 4 + i;
            if (col >= a.W) continue;
            const size_t o = ((size_t)row * a.W + col) * a.cout + co;
            float v = acc[nt][i] + b;
            if (a.act) v = v > 0.f ? v : kSlope * v;
            if (a.ya) a.ya[o] = f2bf(v);
            if (a.skip) v += bf2f(a.skip[o]);
            if (a.y) a.y[o] = f2bf(v);
            if (a.yf) a.yf[o] = a.accum ? a.yf[o] + v : v;
        }
    }
}

// dW[t][co][ci] += sum over pixels p of dz[p][co] x(p + o_t)[ci] (x read with
// upsampling xs), into the flat FP32 gradient (true channel counts).
struct WgradArgs {
    const uint16_t* x; int xs;
    const uint16_t* dz;
    int H, W, cin, cout, cin_true, cout_true;
    int rows_per_block;
    float* gw;              // flat [9][cout_true][cin_true]
};

__global__ __launch_bounds__(256) void conv_wgrad_kernel(WgradArgs a) {
    __shared__ float red[4][8][64 * 4];      // [wave][ci tile][lane * 4 + i]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cot = a.cout / 16;
    const int t = blockIdx.y / cot, co0 = (blockIdx.y % cot) * 16;
    const int dr = t / 3 - 1, dc = t % 3 - 1;
    const int m = lane & 15, kq = lane >> 4;
    const int nct = a.cin / 16;
    const int Wi = a.W / a.xs;
    f32x4 acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int r0 = blockIdx.x * a.rows_per_block;
    const int r1 = min(a.H, r0 + a.rows_per_block);
    const int cpr = (a.W + 15) / 16;                   // 16-pixel chunks per row
    const int nchunk = (r1 - r0) * cpr;
    for (int q = wv; q < nchunk; q += 4) {
        const int row = r0 + q / cpr, cb0 = (q % cpr) * 16;
        bf16x4 A;
        const int rs = row + dr;
        const bool rok = rs >= 0 && rs < a.H;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = cb0 + kq * 4 + j;
            A[j] = col < a.W ? (short)a.dz[((size_t)row * a.W + col) * a.cout + co0 + m] : (short)0;
        }
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) {
            if (ct >= nct) break;
            bf16x4 B;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = cb0 + kq * 4 + j, cs = col + dc;
                const bool ok = rok && col < a.W && cs >= 0 && cs < a.W;
                B[j] = ok ? (short)a.x[((size_t)(rs / a.xs) * Wi + cs / a.xs) * a.cin + ct * 16 + m] : (short)0;
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
    for (int e = threadIdx.x; e < nct * 256; e += 256) {
        const int ct = e / 256, li = e % 256, l = li / 4, i = li % 4;
        const float v = red[0][ct][li] + red[1][ct][li] + red[2][ct][li] + red[3][ct][li];
        const int co = co0 + 4 * (l >> 4) + i, ci = ct * 16 + (l & 15);
        if (co < a.cout_true && ci < a.cin_true && v != 0.f)
            atomicAdd(&a.gw[((size_t)t * a.cout_true + co) * a.cin_true + ci], v);
    }
}

// db[co] += sum over pixels of dz[p][co]
__global__ __launch_bounds__(256) void bias_grad_kernel(const uint16_t* dz, int64_t npix, int cout, int cout_true,
                                                        float* gb) {
    const int c = threadIdx.x % cout;
    const int lanes = 256 / cout * cout;
    if (threadIdx.x >= lanes) return;
    const int sub = threadIdx.x / cout, nsub = 256 / cout;
    float s = 0.f;
    for (int64_t p = (int64_t)blockIdx.x * nsub + sub; p < npix; p += (int64_t)gridDim.x * nsub)
        s += bf2f(dz[p * cout + c]);
    if (c < cout_true && s != 0.f) atomicAdd(&gb[c], s);
}

// ---------------------------------------------------------------------------
// element-wise kernels
template <typename T>
__global__ void prep_input_kernel(int nelx, int nely, int W0, const T* __restrict__ xt, const double* __restrict__ f,
                                  uint16_t* __restrict__ x0, int64_t npix) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
        const int ix = (int)(p / W0), iy = (int)(p % W0);
        float v[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = 0.f;
        if (ix <= nelx && iy <= nely) {
            double s = 0.0;
            int n = 0;
            for (int ax = -1; ax <= 0; ++ax)
                for (int ay = -1; ay <= 0; ++ay) {
                    const int ex = ix + ax, ey = iy + ay;
                    if (ex >= 0 && ex < nelx && ey >= 0 && ey < nely) { s += (double)xt[ey + (int64_t)nely * ex]; ++n; }
                }
            const int64_t node = iy + (int64_t)(nely + 1) * ix;
            v[0] = (float)(s / n);
            v[1] = (float)f[2 * node];
            v[2] = (float)f[2 * node + 1];
        }
        uint16_t* o = x0 + p * 16;
#pragma unroll
        for (int c = 0; c < 16; ++c) o[c] = f2bf(v[c]);
    }
}

__global__ void pool_kernel(const uint16_t* __restrict__ in, int H, int W, int C, uint16_t* __restrict__ out) {
    const int64_t total = (int64_t)(H / 2) * (W / 2) * C;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        const int w = (int)(p % (W / 2)), h = (int)(p / (W / 2));
        const size_t b = ((size_t)(2 * h) * W + 2 * w) * C + c;
        const float s = ((bf2f(in[b]) + bf2f(in[b + C])) + bf2f(in[b + (size_t)W * C])) + bf2f(in[b + (size_t)W * C + C]);
        out[i] = f2bf(0.25f * s);
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

// g_prev[h][w] += 0.25 s[h/2][w/2]  (gradient through the average pooling)
__global__ void unpool_add_kernel(const float* __restrict__ s, int H, int W, int C, float* __restrict__ g) {
    const int64_t total = (int64_t)H * W * C;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        const int w = (int)(p % W), h = (int)(p / W);
        g[i] += 0.25f * s[((size_t)(h / 2) * (W / 2) + w / 2) * C + c];
    }
}

// g_prev[h][w] += sum of s over its 2x2 block (gradient through the upsampling)
__global__ void sumpool_add_kernel(const float* __restrict__ s, int H, int W, int C, float* __restrict__ g) {
    const int64_t total = (int64_t)H * W * C;     // H, W: the half-size grid
    const int W2 = 2 * W;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        const int w = (int)(p % W), h = (int)(p / W);
        const size_t b = ((size_t)(2 * h) * W2 + 2 * w) * C + c;
        g[i] += ((s[b] + s[b + C]) + s[b + (size_t)W2 * C]) + s[b + (size_t)W2 * C + C];
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

// sum of u^2 (FP64 atomics; the target scale)
__global__ __launch_bounds__(256) void sumsq_kernel(const double* __restrict__ u, int64_t n, double* out) {
    __shared__ double sh[kWaves];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) s += u[i] * u[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) atomicAdd(out, s);
}

// mean squared error against u / rms(u) over real nodes, its gradient image
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ out, const double* __restrict__ u,
                                                   int nelx, int nely, int W0, int64_t npix, const double* sumsq,
                                                   int64_t n, float* __restrict__ gout, double* loss) {
    __shared__ double sh[kWaves];
    const double rms = sqrt(*sumsq / (double)n);
    const double inv = rms > 0.0 ? 1.0 / rms : 1.0;
    const double cnt = 2.0 * (double)(nelx + 1) * (double)(nely + 1);
    double s = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < npix; p += (int64_t)gridDim.x * kBlock) {
        const int ix = (int)(p / W0), iy = (int)(p % W0);
        const bool real = ix <= nelx && iy <= nely;
        const int64_t node = iy + (int64_t)(nely + 1) * ix;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            double d = 0.0;
            if (real) d = (double)out[p * 16 + c] - u[2 * node + c] * inv;
            s += d * d;
            gout[p * 16 + c] = (float)(2.0 * d / cnt);
        }
#pragma unroll
        for (int c = 2; c < 16; ++c) gout[p * 16 + c] = 0.f;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) atomicAdd(loss, s / cnt);
}

__global__ void out_to_dofs_kernel(const float* __restrict__ out, int nelx, int nely, int W0,
                                   const uint8_t* __restrict__ freem, double* __restrict__ uh) {
    const int64_t nn = (int64_t)(nelx + 1) * (nely + 1);
    for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < nn; node += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ix = node / (nely + 1), iy = node % (nely + 1);
        const int64_t p = ix * W0 + iy;
#pragma unroll
        for (int c = 0; c < 2; ++c)
            uh[2 * node + c] = freem[2 * node + c] ? (double)out[p * 16 + c] : 0.0;
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

// bfloat16 weight copies of one layer: forward [9][cout_p][cin_p] and the
// flipped-transposed [9][cin_p][cout_p] for the input gradient
__global__ void pack_weights_kernel(const float* __restrict__ w, int cin, int cout, int cin_p, int cout_p,
                                    uint16_t* __restrict__ wf, uint16_t* __restrict__ wb) {
    const int64_t total = 9LL * cin_p * cout_p;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(i % cin_p);
        const int co = (int)((i / cin_p) % cout_p);
        const int t = (int)(i / ((int64_t)cin_p * cout_p));
        const uint16_t v = (ci < cin && co < cout) ? f2bf(w[((size_t)t * cout + co) * cin + ci]) : (uint16_t)0;
        wf[i] = v;
        wb[((size_t)(8 - t) * cin_p + ci) * cout_p + co] = v;
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
    int nelx = 0, nely = 0, H0 = 0, W0 = 0;
    int64_t P = 0;
    LayerBuf L[kNL];
    float *master = nullptr, *mom = nullptr, *vel = nullptr, *grad = nullptr;
    uint16_t* x0 = nullptr;
    uint16_t* pooled[4] = {};          // pooled inputs of levels 1..3
    float* out = nullptr;              // final layer output (FP32, 16 channels)
    float* gtmp = nullptr;             // input-gradient staging (largest level-0 image)
    uint16_t* dz = nullptr;            // bfloat16 error signal staging
    double* scal = nullptr;            // [0] sum u^2, [1] loss
    int64_t step = 0;
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

static size_t nn_layout(int nelx, int nely, Nn* nn, char* base) {
    NnLayout Ly;
    const int H0 = (nelx + 1 + 7) / 8 * 8, W0 = (nely + 1 + 7) / 8 * 8;
    int64_t P = 0;
    int64_t woff[kNL], boff[kNL];
    for (int i = 0; i < kNL; ++i) {
        woff[i] = P;
        P += 9LL * kLayers[i].cin * kLayers[i].cout;
        boff[i] = P;
        P += kLayers[i].cout;
    }
    auto px = [&](int lev) { return (size_t)(H0 >> lev) * (size_t)(W0 >> lev); };
    size_t o_master = Ly.take(4 * P), o_m = Ly.take(4 * P), o_v = Ly.take(4 * P), o_g = Ly.take(4 * P);
    size_t o_x0 = Ly.take(2 * px(0) * 16);
    size_t o_pool[4] = {0, 0, 0, 0};
    const int pool_c[4] = {0, 16, 32, 64};
    for (int l = 1; l < 4; ++l) o_pool[l] = Ly.take(2 * px(l) * pool_c[l]);
    size_t o_out = Ly.take(4 * px(0) * 16);
    size_t o_gtmp = Ly.take(4 * px(0) * 32);
    size_t o_dz = Ly.take(2 * px(0) * 32);
    size_t o_scal = Ly.take(64);
    size_t o_wf[kNL], o_wb[kNL], o_y[kNL], o_a[kNL], o_gl[kNL];
    for (int i = 0; i < kNL; ++i) {
        const LayerDef& d = kLayers[i];
        const int ci = pad16(d.cin), co = pad16(d.cout);
        o_wf[i] = Ly.take(2 * 9 * (size_t)ci * co);
        o_wb[i] = Ly.take(2 * 9 * (size_t)ci * co);
        o_y[i] = i == kNL - 1 ? 0 : Ly.take(2 * px(d.level) * co);
        o_a[i] = d.skip >= 0 ? Ly.take(2 * px(d.level) * co) : 0;
        o_gl[i] = Ly.take(4 * px(d.level) * co);
    }
    if (nn && base) {
        nn->nelx = nelx; nn->nely = nely; nn->H0 = H0; nn->W0 = W0; nn->P = P;
        nn->master = (float*)(base + o_master); nn->mom = (float*)(base + o_m);
        nn->vel = (float*)(base + o_v); nn->grad = (float*)(base + o_g);
        nn->x0 = (uint16_t*)(base + o_x0);
        for (int l = 1; l < 4; ++l) nn->pooled[l] = (uint16_t*)(base + o_pool[l]);
        nn->out = (float*)(base + o_out);
        nn->gtmp = (float*)(base + o_gtmp);
        nn->dz = (uint16_t*)(base + o_dz);
        nn->scal = (double*)(base + o_scal);
        for (int i = 0; i < kNL; ++i) {
            const LayerDef& d = kLayers[i];
            LayerBuf& b = nn->L[i];
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

static void conv_launch(const ConvArgs& a, hipStream_t s) {
    dim3 grid((unsigned)(a.H * ((a.W + 63) / 64)), (unsigned)((a.cout + 63) / 64));
    hipLaunchKernelGGL(conv_fwd_kernel, grid, dim3(256), 0, s, a);
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
    const int64_t npix0 = (int64_t)nn->H0 * nn->W0;
    if (dt == TO_F64)
        hipLaunchKernelGGL(prep_input_kernel<double>, dim3(grid_for(npix0)), dim3(256), 0, s, nn->nelx, nn->nely, nn->W0,
                           (const double*)xt, f, nn->x0, npix0);
    else
        hipLaunchKernelGGL(prep_input_kernel<float>, dim3(grid_for(npix0)), dim3(256), 0, s, nn->nelx, nn->nely, nn->W0,
                           (const float*)xt, f, nn->x0, npix0);
    for (int i = 0; i < kNL; ++i) {
        LayerBuf& b = nn->L[i];
        const int H = nn->H0 >> b.level, W = nn->W0 >> b.level;
        if (b.src == 1) {
            const LayerBuf& pv = nn->L[i - 1];
            const int64_t tot = (int64_t)(H * W) * pv.cout_p;
            hipLaunchKernelGGL(pool_kernel, dim3(grid_for(tot)), dim3(256), 0, s, pv.y, 2 * H, 2 * W, pv.cout_p,
                               nn->pooled[b.level]);
        }
        ConvArgs a{};
        a.x = layer_input(nn, i, a.xs);
        a.H = H; a.W = W; a.cin = b.cin_p; a.cout = b.cout_p;
        a.w = b.wf;
        a.bias = nn->master + b.b_off;
        a.cout_true = b.cout;
        a.act = b.act;
        a.skip = b.skip >= 0 ? nn->L[b.skip].y : nullptr;
        a.ya = b.skip >= 0 ? b.a : nullptr;
        a.y = b.y;
        a.yf = i == kNL - 1 ? nn->out : nullptr;
        a.accum = 0;
        conv_launch(a, s);
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

static void zero_f32(float* p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, 0.f);
}

// loss and gradient of every weight for the sample the last forward pass saw
static to_status nn_backward(Nn* nn, const double* u, hipStream_t s) {
    const int64_t npix0 = (int64_t)nn->H0 * nn->W0;
    const int64_t n = 2LL * (nn->nelx + 1) * (nn->nely + 1);
    hipLaunchKernelGGL(fill_f64_kernel, dim3(1), dim3(64), 0, s, nn->scal, (int64_t)2, 0.0);
    hipLaunchKernelGGL(sumsq_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, u, n, nn->scal);
    zero_f32(nn->grad, nn->P, s);
    for (int i = 0; i < kNL - 1; ++i) {
        const LayerBuf& b = nn->L[i];
        zero_f32(b.g, (int64_t)(nn->H0 >> b.level) * (nn->W0 >> b.level) * b.cout_p, s);
    }
    LayerBuf& lo = nn->L[kNL - 1];
    hipLaunchKernelGGL(loss_kernel, dim3(grid_for(npix0)), dim3(kBlock), 0, s, nn->out, u, nn->nelx, nn->nely, nn->W0,
                       npix0, nn->scal, n, lo.g, nn->scal + 1);
    for (int i = kNL - 1; i >= 0; --i) {
        LayerBuf& b = nn->L[i];
        const int H = nn->H0 >> b.level, W = nn->W0 >> b.level;
        const int64_t npix = (int64_t)H * W, ne = npix * b.cout_p;
        if (b.skip >= 0)
            hipLaunchKernelGGL(add_kernel, dim3(grid_for(ne)), dim3(256), 0, s, b.g, ne, nn->L[b.skip].g);
        hipLaunchKernelGGL(act_bwd_kernel, dim3(grid_for(ne)), dim3(256), 0, s, b.g, b.a, b.act, ne, nn->dz);
        // weight and bias gradients
        WgradArgs w{};
        w.x = layer_input(nn, i, w.xs);
        w.dz = nn->dz;
        w.H = H; w.W = W; w.cin = b.cin_p; w.cout = b.cout_p; w.cin_true = b.cin; w.cout_true = b.cout;
        const int tiles = 9 * (b.cout_p / 16);
        const int want_blocks = 2048;
        int rows = (int)std::max<int64_t>(1, ((int64_t)H * tiles + want_blocks - 1) / want_blocks);
        w.rows_per_block = rows;
        w.gw = nn->grad + b.w_off;
        hipLaunchKernelGGL(conv_wgrad_kernel, dim3((H + rows - 1) / rows, tiles), dim3(256), 0, s, w);
        hipLaunchKernelGGL(bias_grad_kernel, dim3(grid_for(npix, 256 / b.cout_p)), dim3(256), 0, s, nn->dz, npix,
                           b.cout_p, b.cout, nn->grad + b.b_off);
        if (i == 0) break;
        // input gradient: correlation with the flipped, transposed kernel
        LayerBuf& pv = nn->L[i - 1];
        ConvArgs a{};
        a.x = nn->dz; a.xs = 1;
        a.H = H; a.W = W; a.cin = b.cout_p; a.cout = b.cin_p;
        a.w = b.wb;
        a.cout_true = b.cin;
        a.act = 0;
        if (b.src == 0) {
            a.yf = pv.g; a.accum = 1;
            conv_launch(a, s);
        } else {
            a.yf = nn->gtmp; a.accum = 0;
            conv_launch(a, s);
            if (b.src == 1) {       // through the pooling: previous level is twice the size
                const int64_t tot = (int64_t)(2 * H) * (2 * W) * pv.cout_p;
                hipLaunchKernelGGL(unpool_add_kernel, dim3(grid_for(tot)), dim3(256), 0, s, nn->gtmp, 2 * H, 2 * W,
                                   pv.cout_p, pv.g);
            } else {                // through the upsampling: previous level is half the size
                const int64_t tot = (int64_t)(H / 2) * (W / 2) * pv.cout_p;
                hipLaunchKernelGGL(sumpool_add_kernel, dim3(grid_for(tot)), dim3(256), 0, s, nn->gtmp, H / 2, W / 2,
                                   pv.cout_p, pv.g);
            }
        }
    }
    TO_HIP(hipGetLastError());
    return TO_OK;
}

static to_status nn_pack(Nn* nn, hipStream_t s) {
    for (int i = 0; i < kNL; ++i) {
        LayerBuf& b = nn->L[i];
        const int64_t tot = 9LL * b.cin_p * b.cout_p;
        hipLaunchKernelGGL(pack_weights_kernel, dim3(grid_for(tot)), dim3(256), 0, s, nn->master + b.w_off, b.cin,
                           b.cout, b.cin_p, b.cout_p, b.wf, b.wb);
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

to_status to_nn_query(int32_t nelx, int32_t nely, size_t* ws_bytes, int64_t* n_params) {
    if (nelx < 1 || nely < 1 || !ws_bytes) { set_err("to_nn_query: bad size or NULL ws_bytes"); return TO_EINVAL; }
    if ((int64_t)(nelx + 8) * (nely + 8) > (int64_t)1 << 28) { set_err("to_nn_query: mesh too large"); return TO_EINVAL; }
    *ws_bytes = nn_layout(nelx, nely, nullptr, nullptr);
    if (n_params) {
        int64_t P = 0;
        for (int i = 0; i < kNL; ++i) P += 9LL * kLayers[i].cin * kLayers[i].cout + kLayers[i].cout;
        *n_params = P;
    }
    return TO_OK;
}

to_status to_nn_create(const to_plan* plan, void* ws, size_t ws_bytes, to_nn** out) {
    if (!plan || !ws || !out) { set_err("to_nn_create: NULL argument"); return TO_EINVAL; }
    const Plan* p = topt::P(plan);
    if (p->dim != 2) { set_err("to_nn_create: the network is defined for 2D meshes"); return TO_EUNSUPPORTED; }
    if (((uintptr_t)ws & 255u) != 0) { set_err("to_nn_create: workspace not 256-byte aligned"); return TO_EINVAL; }
    size_t need = nn_layout(p->nelx, p->nely, nullptr, nullptr);
    if (ws_bytes < need) { set_err("to_nn_create: workspace too small"); return TO_EWORKSPACE; }
    to_nn* h = new (std::nothrow) to_nn;
    if (!h) { set_err("to_nn_create: out of host memory"); return TO_EINVAL; }
    h->impl.plan = p;
    nn_layout(p->nelx, p->nely, &h->impl, (char*)ws);
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
    const int64_t npix0 = (int64_t)nn->H0 * nn->W0;
    if (what == TO_NN_PARAMS) {
        TO_HIP(hipMemcpyAsync(out, nn->master, 4 * nn->P, hipMemcpyDeviceToDevice, s));
    } else if (what == TO_NN_GRAD) {
        TO_HIP(hipMemcpyAsync(out, nn->grad, 4 * nn->P, hipMemcpyDeviceToDevice, s));
    } else if (what == TO_NN_OUTPUT) {
        TO_HIP(hipMemcpyAsync(out, nn->out, 4 * npix0 * 16, hipMemcpyDeviceToDevice, s));
    } else if (what >= TO_NN_ACT && what < TO_NN_ACT + kNL - 1) {
        const LayerBuf& b = nn->L[what - TO_NN_ACT];
        const size_t bytes = 2 * (size_t)(nn->H0 >> b.level) * (size_t)(nn->W0 >> b.level) * b.cout_p;
        TO_HIP(hipMemcpyAsync(out, b.y, bytes, hipMemcpyDeviceToDevice, s));
    } else if (what >= TO_NN_PRESKIP && what < TO_NN_PRESKIP + kNL - 1 && nn->L[what - TO_NN_PRESKIP].skip >= 0) {
        const LayerBuf& b = nn->L[what - TO_NN_PRESKIP];
        const size_t bytes = 2 * (size_t)(nn->H0 >> b.level) * (size_t)(nn->W0 >> b.level) * b.cout_p;
        TO_HIP(hipMemcpyAsync(out, b.a, bytes, hipMemcpyDeviceToDevice, s));
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
        const int64_t nn_nodes = (int64_t)(nn->nelx + 1) * (nn->nely + 1);
        hipLaunchKernelGGL(out_to_dofs_kernel, dim3(grid_for(nn_nodes)), dim3(256), 0, s, nn->out, nn->nelx, nn->nely,
                           nn->W0, nn->plan->freemask, uhat);
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
