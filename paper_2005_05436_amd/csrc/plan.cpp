// Plan builder (host C++): numbering, the reduced index set of eq. (14), the
// lower CSR pattern of K^(s), the stable (row, col) permutation, the element
// matrix by Gauss quadrature and the cone filter table.  This is the set-up phase of Sec. 3 (blocks PRE.2 and
// PRE.5 of both codes); it runs once per mesh.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "common.h"

namespace topt {

// ---------------------------------------------------------------------------
// Geometry helpers
struct Grid {
    int dim, nx, ny, nz;                  // elements per axis (nz = 1 in 2D)
    int64_t node(int iy, int ix, int iz) const {
        return dim == 2 ? iy + (int64_t)(ny + 1) * ix
                        : iy + (int64_t)(ny + 1) * (iz + (int64_t)(nz + 1) * ix);
    }
    int64_t m() const { return (int64_t)nx * ny * (dim == 2 ? 1 : nz); }
    int64_t nnode() const { return (int64_t)(nx + 1) * (ny + 1) * (dim == 2 ? 1 : nz + 1); }
    // Global DOFs of element e in the element-matrix order (corner order of
    // Fig. 1b: lower-left, lower-right, upper-right, upper-left; in 3D the face
    // iz then the face iz+1; "lower" = larger iy).
    void element_dofs(int64_t e, int32_t* g) const {
        int iy = (int)(e % ny);
        int64_t rest = e / ny;
        int ix, iz = 0;
        if (dim == 2) ix = (int)rest; else { iz = (int)(rest % nz); ix = (int)(rest / nz); }
        const int cy[4] = {1, 1, 0, 0}, cx[4] = {0, 1, 1, 0};
        int k = 0;
        for (int face = 0; face < (dim == 2 ? 1 : 2); ++face)
            for (int c = 0; c < 4; ++c) {
                int64_t nd = node(iy + cy[c], ix + cx[c], iz + face);
                for (int comp = 0; comp < dim; ++comp) g[k++] = (int32_t)(dim * nd + comp);
            }
    }
};

// Neighbour nodes (sharing an element) of node (iy, ix, iz) in ascending node
// order; returns the count (<= 27).
static int neighbours(const Grid& G, int iy, int ix, int iz, int64_t* out) {
    int k = 0;
    for (int dx = -1; dx <= 1; ++dx) {
        int jx = ix + dx;
        if (jx < 0 || jx > G.nx) continue;
        for (int dz = (G.dim == 3 ? -1 : 0); dz <= (G.dim == 3 ? 1 : 0); ++dz) {
            int jz = iz + dz;
            if (G.dim == 3 && (jz < 0 || jz > G.nz)) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                int jy = iy + dy;
                if (jy < 0 || jy > G.ny) continue;
                out[k++] = G.node(jy, jx, jz);
            }
        }
    }
    return k;
}

static void node_coords(const Grid& G, int64_t nd, int& iy, int& ix, int& iz) {
    iy = (int)(nd % (G.ny + 1));
    int64_t rest = nd / (G.ny + 1);
    if (G.dim == 2) { ix = (int)rest; iz = 0; }
    else { iz = (int)(rest % (G.nz + 1)); ix = (int)(rest / (G.nz + 1)); }
}

// Row lengths of the lower CSR of K^(s): the row of DOF dim*n + c holds every
// DOF of the neighbours q < n and components 0..c of n itself.
static void lower_pattern(const Grid& G, std::vector<int32_t>& row_ptr, std::vector<int32_t>* col_idx) {
    const int64_t nn = G.nnode(), n = G.dim * nn;
    row_ptr.assign(n + 1, 0);
    int64_t nb[27];
    for (int64_t nd = 0; nd < nn; ++nd) {
        int iy, ix, iz;
        node_coords(G, nd, iy, ix, iz);
        int k = neighbours(G, iy, ix, iz, nb);
        int below = 0;
        for (int i = 0; i < k; ++i) below += nb[i] < nd;
        for (int c = 0; c < G.dim; ++c) row_ptr[G.dim * nd + c + 1] = G.dim * below + c + 1;
    }
    for (int64_t r = 0; r < n; ++r) row_ptr[r + 1] += row_ptr[r];
    if (!col_idx) return;
    col_idx->resize(row_ptr[n]);
    for (int64_t nd = 0; nd < nn; ++nd) {
        int iy, ix, iz;
        node_coords(G, nd, iy, ix, iz);
        int k = neighbours(G, iy, ix, iz, nb);
        for (int c = 0; c < G.dim; ++c) {
            int32_t* out = col_idx->data() + row_ptr[G.dim * nd + c];
            for (int i = 0; i < k && nb[i] < nd; ++i)
                for (int cc = 0; cc < G.dim; ++cc) *out++ = (int32_t)(G.dim * nb[i] + cc);
            for (int cc = 0; cc <= c; ++cc) *out++ = (int32_t)(G.dim * nd + cc);
        }
    }
}

// ---------------------------------------------------------------------------
// Element stiffness by tensor Gauss quadrature (2 points per direction on the
// unit square / cube): Ke = int B^T D B.  Q4 plane stress, Hex8 isotropic.
static void element_matrix(int dim, double nu, std::vector<double>& K) {
    const int nc = dim == 2 ? 4 : 8, d = dim * nc;
    const int corner[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                              {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
    const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
    K.assign((size_t)d * d, 0.0);
    const int ns = dim == 2 ? 3 : 6;
    double D[6][6] = {};
    if (dim == 2) {
        double c = 1.0 / (1.0 - nu * nu);
        D[0][0] = D[1][1] = c; D[0][1] = D[1][0] = c * nu; D[2][2] = c * (1.0 - nu) / 2.0;
    } else {
        double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = 1.0 / (2.0 * (1.0 + nu));
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) D[i][j] = lam + (i == j ? 2.0 * mu : 0.0);
        D[3][3] = D[4][4] = D[5][5] = mu;
    }
    const double w = dim == 2 ? 0.25 : 0.125;
    for (int qz = 0; qz < (dim == 2 ? 1 : 2); ++qz)
        for (int qy = 0; qy < 2; ++qy)
            for (int qx = 0; qx < 2; ++qx) {
                double pt[3] = {gp[qx], gp[qy], gp[qz]};
                double B[6][24] = {};
                for (int a = 0; a < nc; ++a) {
                    double N[3], S[3];
                    for (int ax = 0; ax < dim; ++ax) {
                        bool one = corner[a][ax] == 1;
                        N[ax] = one ? pt[ax] : 1.0 - pt[ax];
                        S[ax] = one ? 1.0 : -1.0;
                    }
                    double g[3];
                    if (dim == 2) { g[0] = S[0] * N[1]; g[1] = N[0] * S[1]; }
                    else {
                        g[0] = S[0] * N[1] * N[2]; g[1] = N[0] * S[1] * N[2]; g[2] = N[0] * N[1] * S[2];
                    }
                    if (dim == 2) {
                        B[0][2 * a] = g[0]; B[1][2 * a + 1] = g[1];
                        B[2][2 * a] = g[1]; B[2][2 * a + 1] = g[0];
                    } else {
                        B[0][3 * a] = g[0]; B[1][3 * a + 1] = g[1]; B[2][3 * a + 2] = g[2];
                        B[3][3 * a] = g[1]; B[3][3 * a + 1] = g[0];
                        B[4][3 * a + 1] = g[2]; B[4][3 * a + 2] = g[1];
                        B[5][3 * a] = g[2]; B[5][3 * a + 2] = g[0];
                    }
                }
                double DB[6][24];
                for (int i = 0; i < ns; ++i)
                    for (int j = 0; j < d; ++j) {
                        double s = 0; for (int k = 0; k < ns; ++k) s += D[i][k] * B[k][j];
                        DB[i][j] = s;
                    }
                for (int i = 0; i < d; ++i)
                    for (int j = 0; j < d; ++j) {
                        double s = 0; for (int k = 0; k < ns; ++k) s += B[k][i] * DB[k][j];
                        K[(size_t)i * d + j] += w * s;
                    }
            }
    // exact symmetry (quadrature rounding can differ in the last bit)
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < i; ++j) {
            double a = 0.5 * (K[(size_t)i * d + j] + K[(size_t)j * d + i]);
            K[(size_t)i * d + j] = K[(size_t)j * d + i] = a;
        }
}

// ---------------------------------------------------------------------------
// Workspace layout
struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

struct Sizes {
    Grid G{};
    int64_t m = 0, nn = 0, n = 0, pairs = 0, nnz = 0;
    int d = 0, dt = 0, R = 0, taps = 0, cols = 0;
};

// Row stride of the padded 2D tap table: the non-zero taps of a row followed
// by zeros, so the filter's unrolled chunks of 8 taps read 8 consecutive
// weights without bounds tests.
static int pad_stride(int R) { return ((2 * R + 1 + 8) + 7) / 8 * 8; }
// column dx of the matrix-core filter table: dy = -R-16 .. R+19 and more
static int hm_stride(int R) { return (2 * R + 36 + 3) / 4 * 4; }

static to_status check_desc(const to_mesh_desc* D, Sizes& S) {
    if (!D) { set_error("desc is NULL"); return TO_EINVAL; }
    if (D->dim != 2 && D->dim != 3) { set_error("dim must be 2 or 3"); return TO_EINVAL; }
    if (D->nelx <= 0 || D->nely <= 0 || (D->dim == 3 && D->nelz <= 0)) {
        set_error("element counts must be positive"); return TO_EINVAL;
    }
    if (!(D->rmin > 0) || !std::isfinite(D->rmin) || D->rmin > 1000) { set_error("rmin must be in (0, 1000]"); return TO_EINVAL; }
    if (D->bc != 'D' && D->bc != 'N') { set_error("bc must be 'D' or 'N'"); return TO_EINVAL; }
    if (!(D->nu > -1.0 && D->nu < 0.5)) { set_error("nu must be in (-1, 0.5)"); return TO_EINVAL; }
    if (!(D->E0 > 0) || !(D->Emin >= 0) || !std::isfinite(D->E0) || !std::isfinite(D->Emin)) {
        set_error("E0 must be > 0 and Emin >= 0"); return TO_EINVAL;
    }
    if (D->n_fixed < 0 || (D->n_fixed > 0 && !D->h_fixed)) { set_error("bad fixed DOF list"); return TO_EINVAL; }
    S.G = Grid{D->dim, D->nelx, D->nely, D->dim == 3 ? D->nelz : 1};
    S.m = S.G.m(); S.nn = S.G.nnode(); S.n = D->dim * S.nn;
    S.d = D->dim == 2 ? 8 : 24; S.dt = S.d * (S.d + 1) / 2;
    S.pairs = S.m * S.dt;
    if (S.pairs >= INT32_MAX || S.n >= INT32_MAX / 2) { set_error("mesh too large for int32 indexing"); return TO_EINVAL; }
    for (int64_t i = 0; i < D->n_fixed; ++i)
        if (D->h_fixed[i] < 0 || D->h_fixed[i] >= S.n) { set_error("fixed DOF out of range"); return TO_EINVAL; }
    S.R = (int)std::ceil(D->rmin) - 1;
    const int w = 2 * S.R + 1;
    S.taps = D->dim == 2 ? w * w : w * w * w;
    S.cols = D->dim == 2 ? w : w * w;
    std::vector<int32_t> rp;
    lower_pattern(S.G, rp, nullptr);
    S.nnz = rp[S.n];
    return TO_OK;
}


// Cone filter table h(o) = max(0, rmin - |o|) over o in [-R, R]^dim, stored
// y fastest: index (col * (2R+1) + dy + R) with col = dx + R in 2D and
// col = (dx + R)(2R+1) + dz + R in 3D; lim[col] = largest |dy| with h > 0
// (-1 if the whole column is zero).
static void filter_table(const Sizes& S, double rmin, std::vector<double>& h, std::vector<int32_t>& lim) {
    const int w = 2 * S.R + 1;
    h.assign(S.taps, 0.0);
    lim.assign(S.cols, -1);
    for (int col = 0; col < S.cols; ++col) {
        const int dx = (S.G.dim == 2 ? col : col / w) - S.R;
        const int dz = S.G.dim == 2 ? 0 : col % w - S.R;
        for (int yy = 0; yy < w; ++yy) {
            const int dy = yy - S.R;
            const double v = std::max(0.0, rmin - std::sqrt((double)(dx * dx + dy * dy + dz * dz)));
            h[(size_t)col * w + yy] = v;
            if (v > 0.0) lim[col] = std::max(lim[col], std::abs(dy));
        }
    }
}

struct Offsets {
    size_t perm, seg, rowp, col, pas, freem, ke64, ke32, kf64, kf32, h64, h32,
        hlim, hp64, hp32, hm32, hm64, Hs64, Hs32, E64, E32, partial, ll, scal, bar, v64[8], v32[8], fx64, fx32, total;
    // multigrid hierarchy (2D)
    GmgShape gs;
    size_t gK[kGmgMaxLevels], gS[kGmgMaxLevels], gx[kGmgMaxLevels], gxt[kGmgMaxLevels], gb[kGmgMaxLevels], gr[kGmgMaxLevels],
        gd[kGmgMaxLevels], gAinv, gscal;
};

static Offsets layout(const Sizes& S) {
    Layout L;
    Offsets o{};
    o.perm = L.take(4 * S.pairs);
    o.seg = L.take(4 * (S.nnz + 1));
    o.rowp = L.take(4 * (S.n + 1));
    o.col = L.take(4 * S.nnz);
    o.pas = L.take(S.m);
    o.freem = L.take(S.n);
    o.ke64 = L.take(8 * S.dt);
    o.ke32 = L.take(4 * S.dt);
    o.kf64 = L.take(8 * S.d * S.d);
    o.kf32 = L.take(4 * S.d * S.d);
    o.h64 = L.take(8 * S.taps);
    o.h32 = L.take(4 * S.taps);
    o.hlim = L.take(4 * S.cols);
    o.hp64 = L.take(8 * (size_t)(2 * S.R + 1) * pad_stride(S.R));
    o.hp32 = L.take(4 * (size_t)(2 * S.R + 1) * pad_stride(S.R));
    o.hm32 = L.take(S.G.dim == 2 ? 4 * (size_t)(2 * S.R + 1) * hm_stride(S.R) : 0);
    o.hm64 = L.take(S.G.dim == 2 ? 8 * (size_t)(2 * S.R + 1) * hm_stride(S.R) : 0);
    o.Hs64 = L.take(8 * S.m);
    o.Hs32 = L.take(4 * S.m);
    o.E64 = L.take(8 * S.m);
    o.E32 = L.take(4 * S.m);
    o.partial = L.take(8 * 2 * (size_t)kMaxCoopBlocks * kPartialWidth);   // two regions
    o.ll = L.take(kLLBytes);
    o.scal = L.take(8 * 256);
    o.bar = L.take(4 * 1024);
    for (int i = 0; i < 8; ++i) o.v64[i] = L.take(8 * S.n);
    for (int i = 0; i < 8; ++i) o.v32[i] = L.take(4 * S.n);
    o.fx64 = L.take(8 * S.m);
    o.fx32 = L.take(4 * S.m);
    {
        const int dim = S.G.dim;
        const size_t D = (size_t)dim * (dim == 2 ? 4 : 8);
        o.gs = gmg_shape(dim, S.G.nx, S.G.ny, S.G.nz);
        for (int l = 0; l < o.gs.L; ++l) {
            const int64_t nx = o.gs.nx[l], ny = o.gs.ny[l], nz = o.gs.nz[l];
            const int64_t n = gmg_dofs(dim, (int)nx, (int)ny, (int)nz);
            o.gK[l] = l ? L.take(8 * D * D * (size_t)(nx * ny * nz)) : 0;
            o.gS[l] = l ? L.take(8 * (size_t)(dim == 2 ? 9 : 27) * dim * dim * (size_t)(n / dim)) : 0;
            o.gx[l] = l ? L.take(8 * n) : 0;
            o.gb[l] = l ? L.take(8 * n) : 0;
            o.gxt[l] = L.take(8 * n);
            o.gr[l] = L.take(8 * n);
            o.gd[l] = L.take(8 * n);
        }
        if (o.gs.L) {
            o.gAinv = L.take(8 * (size_t)kGmgCoarseMax * kGmgCoarseMax);
            o.gscal = L.take(sizeof(GmgScal));
        }
    }
    o.total = L.off;
    return o;
}

to_status plan_query(const to_mesh_desc* desc, size_t* ws) {
    if (!ws) { set_error("ws_bytes is NULL"); return TO_EINVAL; }
    Sizes S;
    to_status st = check_desc(desc, S);
    if (st != TO_OK) return st;
    *ws = layout(S).total;
    return TO_OK;
}

// Slot of every I_r pair: slot = row_ptr[row] + position of col in the row.
static void pair_slots(const Sizes& S, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci,
                       std::vector<int32_t>& slot) {
    slot.resize(S.pairs);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto work = [&](int64_t e0, int64_t e1) {
        int32_t g[24];
        for (int64_t e = e0; e < e1; ++e) {
            S.G.element_dofs(e, g);
            int64_t t = e * S.dt;
            for (int j = 0; j < S.d; ++j)
                for (int i = j; i < S.d; ++i, ++t) {
                    int32_t r = std::max(g[i], g[j]), c = std::min(g[i], g[j]);
                    const int32_t* b = ci.data() + rp[r];
                    const int32_t* en = ci.data() + rp[r + 1];
                    slot[t] = (int32_t)(std::lower_bound(b, en, c) - ci.data());
                }
        }
    };
    std::vector<std::thread> th;
    int64_t chunk = (S.m + nth - 1) / nth;
    for (unsigned k = 0; k < nth; ++k) {
        int64_t a = k * chunk, b = std::min<int64_t>(S.m, a + chunk);
        if (a < b) th.emplace_back(work, a, b);
    }
    for (auto& t : th) t.join();
}


// Lower CSR and the stable permutation of I_r with its segment pointers.
static void build_pattern(const Sizes& S, std::vector<int32_t>& rp, std::vector<int32_t>& ci,
                          std::vector<int32_t>& seg, std::vector<int32_t>& perm) {
    std::vector<int32_t> slot;
    lower_pattern(S.G, rp, &ci);
    pair_slots(S, rp, ci, slot);
    seg.assign(S.nnz + 1, 0);
    perm.resize(S.pairs);
    for (int64_t t = 0; t < S.pairs; ++t) seg[slot[t] + 1]++;
    for (int64_t s = 0; s < S.nnz; ++s) seg[s + 1] += seg[s];
    std::vector<int32_t> fill(seg.begin(), seg.end() - 1);
    for (int64_t t = 0; t < S.pairs; ++t) perm[fill[slot[t]]++] = (int32_t)t;   // stable
}

static void write_pairs(const Grid& G, int64_t m, int d, int32_t* o) {
    int32_t g[24];
    int64_t t = 0;
    for (int64_t e = 0; e < m; ++e) {
        G.element_dofs(e, g);
        for (int j = 0; j < d; ++j)
            for (int i = j; i < d; ++i, ++t) {
                o[2 * t] = std::max(g[i], g[j]);
                o[2 * t + 1] = std::min(g[i], g[j]);
            }
    }
}

// Same host code as to_plan_create, without a device (for host-side checks).
to_status plan_build_host(const to_mesh_desc* D, int what, void* dst, size_t bytes) {
    if (!dst) { set_error("dst is NULL"); return TO_EINVAL; }
    Sizes S;
    to_status st = check_desc(D, S);
    if (st != TO_OK) return st;
    auto put = [&](const void* src, size_t need) -> to_status {
        if (bytes < need) { set_error("destination too small"); return TO_EINVAL; }
        std::memcpy(dst, src, need);
        return TO_OK;
    };
    if (what == TO_X_PAIRS) {
        if (bytes < 8 * (size_t)S.pairs) { set_error("destination too small"); return TO_EINVAL; }
        write_pairs(S.G, S.m, S.d, (int32_t*)dst);
        return TO_OK;
    }
    if (what == TO_X_KE) {
        std::vector<double> K, v;
        element_matrix(S.G.dim, D->nu, K);
        for (int j = 0; j < S.d; ++j) for (int i = j; i < S.d; ++i) v.push_back(K[(size_t)i * S.d + j]);
        return put(v.data(), 8 * v.size());
    }
    if (what == TO_X_FREE) {
        std::vector<uint8_t> fm(S.n, 1);
        for (int64_t i = 0; i < D->n_fixed; ++i) fm[D->h_fixed[i]] = 0;
        return put(fm.data(), fm.size());
    }
    if (what == TO_X_KERNEL) {
        std::vector<double> h;
        std::vector<int32_t> lim;
        filter_table(S, D->rmin, h, lim);
        return put(h.data(), 8 * h.size());
    }
    if (what == TO_X_HS) { set_error("Hs is computed on the device"); return TO_EUNSUPPORTED; }
    std::vector<int32_t> rp, ci, seg, perm;
    if (what == TO_X_ROWPTR || what == TO_X_COLIDX) {
        lower_pattern(S.G, rp, &ci);
        return what == TO_X_ROWPTR ? put(rp.data(), 4 * rp.size()) : put(ci.data(), 4 * ci.size());
    }
    if (what != TO_X_PERM && what != TO_X_SEGPTR) { set_error("unknown export id"); return TO_EINVAL; }
    build_pattern(S, rp, ci, seg, perm);
    return what == TO_X_PERM ? put(perm.data(), 4 * perm.size()) : put(seg.data(), 4 * seg.size());
}

to_status plan_create(const to_mesh_desc* D, void* ws, size_t ws_bytes, hipStream_t stream, to_plan** out) {
    if (!out) { set_error("out is NULL"); return TO_EINVAL; }
    *out = nullptr;
    Sizes S;
    to_status st = check_desc(D, S);
    if (st != TO_OK) return st;
    Offsets o = layout(S);
    if (!ws || ws_bytes < o.total || ((uintptr_t)ws & 255u)) {
        set_error("workspace missing, too small or not 256-byte aligned");
        return TO_EWORKSPACE;
    }
    Plan* p = new Plan();
    p->dim = D->dim; p->nelx = D->nelx; p->nely = D->nely; p->nelz = S.G.nz;
    p->d = S.d; p->dt = S.dt; p->R = S.R;
    p->E0 = D->E0; p->Emin = D->Emin; p->nu = D->nu; p->rmin = D->rmin; p->bc = D->bc;
    p->ws_bytes = ws_bytes;
    char* base = (char*)ws;
    p->perm = (int32_t*)(base + o.perm); p->seg_ptr = (int32_t*)(base + o.seg);
    p->row_ptr = (int32_t*)(base + o.rowp); p->col_idx = (int32_t*)(base + o.col);
    p->passive = (uint8_t*)(base + o.pas); p->freemask = (uint8_t*)(base + o.freem);
    p->ke64 = (double*)(base + o.ke64); p->ke32 = (float*)(base + o.ke32);
    p->kf64 = (double*)(base + o.kf64); p->kf32 = (float*)(base + o.kf32);
    p->h64 = (double*)(base + o.h64); p->h32 = (float*)(base + o.h32); p->hlim = (int32_t*)(base + o.hlim);
    p->hp64 = (double*)(base + o.hp64); p->hp32 = (float*)(base + o.hp32); p->hp_stride = pad_stride(S.R);
    p->hm32 = (float*)(base + o.hm32); p->hm_stride = hm_stride(S.R);
    p->hm64 = (double*)(base + o.hm64);
    p->Hs64 = (double*)(base + o.Hs64); p->Hs32 = (float*)(base + o.Hs32);
    p->E64 = (double*)(base + o.E64); p->E32 = (float*)(base + o.E32);
    p->partial = (double*)(base + o.partial); p->scal = (double*)(base + o.scal);
    p->ll = (unsigned long long*)(base + o.ll);
    p->bar = (unsigned*)(base + o.bar);
    for (int i = 0; i < 8; ++i) { p->v64[i] = (double*)(base + o.v64[i]); p->v32[i] = (float*)(base + o.v32[i]); }
    p->fx64 = (double*)(base + o.fx64); p->fx32 = (float*)(base + o.fx32);
    p->gmg.L = o.gs.L;
    for (int l = 0; l < o.gs.L; ++l) {
        GmgLevel& v = p->gmg.lv[l];
        v.nx = o.gs.nx[l]; v.ny = o.gs.ny[l]; v.nz = o.gs.nz[l];
        v.nnode = (int64_t)(v.nx + 1) * (v.ny + 1) * (S.G.dim == 3 ? v.nz + 1 : 1);
        v.n = S.G.dim * v.nnode;
        v.m = (int64_t)v.nx * v.ny * v.nz;
        v.K = l ? (double*)(base + o.gK[l]) : nullptr;
        v.S = l ? (double*)(base + o.gS[l]) : nullptr;
        v.x = l ? (double*)(base + o.gx[l]) : nullptr;
        v.b = l ? (double*)(base + o.gb[l]) : nullptr;
        v.xt = (double*)(base + o.gxt[l]);
        v.r = (double*)(base + o.gr[l]);
        v.dinv = (double*)(base + o.gd[l]);
    }
    if (o.gs.L) {
        p->gmg.Ainv = (double*)(base + o.gAinv);
        p->gmg.scal = (GmgScal*)(base + o.gscal);
    }

    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete p; set_error("no HIP device"); return TO_EHIP;
    }
    p->num_cu = prop.multiProcessorCount;

    // --- sparse pattern, permutation, transpose map ------------------------
    std::vector<int32_t> rp, ci, seg, perm;
    build_pattern(S, rp, ci, seg, perm);
    // --- masks --------------------------------------------------------------
    std::vector<uint8_t> pas(S.m, TO_ACTIVE), fm(S.n, 1);
    if (D->h_passive) std::memcpy(pas.data(), D->h_passive, S.m);
    int64_t na = 0, ns = 0, nv = 0;
    for (auto c : pas) { if (c == TO_SOLID) ++ns; else if (c == TO_VOID) ++nv; else if (c == TO_ACTIVE) ++na; else {
        delete p; set_error("passive code must be 0, 1 or 2"); return TO_EINVAL; } }
    for (int64_t i = 0; i < D->n_fixed; ++i) fm[D->h_fixed[i]] = 0;
    int64_t nfree = 0;
    for (auto f : fm) nfree += f;
    // --- element matrix ------------------------------------------------------
    element_matrix(S.G.dim, D->nu, p->ke_full);
    p->ke_lower.clear();
    for (int j = 0; j < S.d; ++j) for (int i = j; i < S.d; ++i) p->ke_lower.push_back(p->ke_full[(size_t)i * S.d + j]);
    std::vector<float> ke32(p->ke_lower.begin(), p->ke_lower.end()), kf32(p->ke_full.begin(), p->ke_full.end());
    // --- filter table --------------------------------------------------------
    filter_table(S, D->rmin, p->h, p->hlim_host);
    std::vector<float> h32(p->h.begin(), p->h.end());
    // padded rows: hp[dyi][t] = h(dy, t - lim(dy)) for t <= 2 lim(dy), else 0
    // (the cone is symmetric, so lim of column dy bounds row dy)
    const int W2 = 2 * S.R + 1, WP = pad_stride(S.R);
    std::vector<double> hp(S.G.dim == 2 ? (size_t)W2 * WP : 1, 0.0);
    if (S.G.dim == 2)
        for (int dyi = 0; dyi < W2; ++dyi) {
            const int lim = p->hlim_host[dyi];
            for (int t = 0; t <= 2 * lim; ++t)
                hp[(size_t)dyi * WP + t] = p->h[(size_t)dyi * W2 + S.R + (t - lim)];
        }
    std::vector<float> hp32v(hp.begin(), hp.end());
    // hm[dxi][dy + R + 16] = h(dx, dy) in FP32, zero for |dy| > R
    const int HM = hm_stride(S.R);
    std::vector<float> hm(S.G.dim == 2 ? (size_t)W2 * HM : 0, 0.0f);
    std::vector<double> hm64(S.G.dim == 2 ? (size_t)W2 * HM : 0, 0.0);
    if (S.G.dim == 2)
        for (int dxi = 0; dxi < W2; ++dxi)
            for (int dyi = 0; dyi < W2; ++dyi) {
                hm[(size_t)dxi * HM + dyi + 16] = h32[(size_t)dxi * W2 + dyi];
                hm64[(size_t)dxi * HM + dyi + 16] = p->h[(size_t)dxi * W2 + dyi];
            }

    // --- upload ------------------------------------------------------------------
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream) : hipSuccess;
    };
    hipError_t e = hipSuccess;
#define UP(dst, vec) if (e == hipSuccess) e = up(dst, vec.data(), vec.size() * sizeof(vec[0]))
    UP(p->perm, perm); UP(p->seg_ptr, seg); UP(p->row_ptr, rp); UP(p->col_idx, ci);
    UP(p->passive, pas); UP(p->freemask, fm);
    UP(p->ke64, p->ke_lower); UP(p->ke32, ke32); UP(p->kf64, p->ke_full); UP(p->kf32, kf32);
    UP(p->h64, p->h); UP(p->h32, h32); UP(p->hlim, p->hlim_host);
    UP(p->hp64, hp); UP(p->hp32, hp32v); UP(p->hm32, hm); UP(p->hm64, hm64);
#undef UP
    if (e == hipSuccess) e = hipMemsetAsync(p->bar, 0, 4 * 1024, stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->ll, 0, kLLBytes, stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->scal, 0, 8 * 256, stream);
    if (e != hipSuccess) { delete p; return hip_fail(e, "plan upload"); }
    st = launch_fill_hs(p, stream);
    if (st != TO_OK) { delete p; return st; }
    e = hipStreamSynchronize(stream);   // host vectors above go out of scope
    if (e != hipSuccess) { delete p; return hip_fail(e, "plan upload sync"); }

    to_plan_info& I = p->info;
    I.dim = S.G.dim; I.d = S.d; I.dtilde = S.dt; I.m = S.m; I.nnode = S.nn; I.n = S.n;
    I.n_pairs = S.pairs; I.nnz_lower = S.nnz; I.n_active = na; I.n_solid = ns; I.n_void = nv;
    I.n_free = nfree; I.filter_radius = S.R; I.coop_blocks = 0; I.workspace_bytes = o.total;
    *out = reinterpret_cast<to_plan*>(p);
    return TO_OK;
}

to_status plan_export(const to_plan* plan, int what, void* dst, size_t bytes, hipStream_t stream) {
    Plan* p = P(plan);
    if (!p || !dst) { set_error("plan or dst is NULL"); return TO_EINVAL; }
    const to_plan_info& I = p->info;
    auto dl = [&](const void* src, size_t need) -> to_status {
        if (bytes < need) { set_error("destination too small"); return TO_EINVAL; }
        TO_HIP(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToHost, stream));
        TO_HIP(hipStreamSynchronize(stream));
        return TO_OK;
    };
    switch (what) {
    case TO_X_PAIRS: {
        if (bytes < 8 * (size_t)I.n_pairs) { set_error("destination too small"); return TO_EINVAL; }
        write_pairs(Grid{p->dim, p->nelx, p->nely, p->nelz}, I.m, p->d, (int32_t*)dst);
        return TO_OK;
    }
    case TO_X_PERM: return dl(p->perm, 4 * (size_t)I.n_pairs);
    case TO_X_SEGPTR: return dl(p->seg_ptr, 4 * (size_t)(I.nnz_lower + 1));
    case TO_X_ROWPTR: return dl(p->row_ptr, 4 * (size_t)(I.n + 1));
    case TO_X_COLIDX: return dl(p->col_idx, 4 * (size_t)I.nnz_lower);
    case TO_X_HS: return dl(p->Hs64, 8 * (size_t)I.m);
    case TO_X_KE: return dl(p->ke64, 8 * (size_t)p->dt);
    case TO_X_FREE: return dl(p->freemask, (size_t)I.n);
    case TO_X_KERNEL: return dl(p->h64, 8 * p->h.size());
    default: set_error("unknown export id"); return TO_EINVAL;
    }
}

}  // namespace topt
