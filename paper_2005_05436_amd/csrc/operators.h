// Node-centric operators of the state equation (eq. (5)) shared by the PCG
// solve and the multigrid preconditioner: the grid geometry, the block's
// node range with its device-coherent halo, source-vector adaptors and the
// matrix-free stiffness operator K = sum_e E_e A_e^T Ke A_e.
#pragma once

#include "common.h"

namespace topt {

struct Geo {
    int nx, ny, nz;
    int64_t nnode;
    __device__ __forceinline__ void coords(int64_t nd, int& iy, int& ix, int& iz, int dim) const {
        iy = (int)(nd % (ny + 1));
        int64_t rest = nd / (ny + 1);
        if (dim == 2) { ix = (int)rest; iz = 0; }
        else { iz = (int)(rest % (nz + 1)); ix = (int)(rest / (nz + 1)); }
    }
};

// The block's node range and its halo band (the largest node-index distance
// between two nodes of one element).
struct Own {
    int64_t lo, hi, band;
    __device__ __forceinline__ bool mine(int64_t q) const { return q >= lo && q < hi; }
    __device__ __forceinline__ bool edge(int64_t nd) const { return nd < lo + band || nd >= hi - band; }
    template <typename T>
    __device__ __forceinline__ T ld(const T* p, int64_t q, int64_t i) const { return mine(q) ? p[i] : ld_dev(p + i); }
    template <typename T>
    __device__ __forceinline__ void st(T* p, int64_t nd, int64_t i, T v) const {
        if (edge(nd)) st_dev(p + i, v);
        else p[i] = v;
    }
};

// Source vectors of the operators, read by node and component.
template <int DIM, typename T> struct Src1 {
    const T* x;
    Own o;
    __device__ __forceinline__ T operator()(int64_t q, int c) const { return o.ld(x, q, DIM * q + c); }
};
template <int DIM, typename T> struct SrcZP {
    const T* z;
    const T* p;
    T beta;
    Own o;
    __device__ __forceinline__ T operator()(int64_t q, int c) const {
        return o.ld(z, q, DIM * q + c) + beta * o.ld(p, q, DIM * q + c);
    }
};

template <int DIM, typename T>
struct MatFree {
    const T* __restrict__ E;     // m moduli
    const T* __restrict__ ke;    // d x d, row major
    int nx, ny, nz;
    static constexpr int NC = DIM == 2 ? 4 : 8;
    static constexpr int D = DIM * NC;

    __device__ __forceinline__ int64_t node(int y, int x, int z) const {
        return DIM == 2 ? y + (int64_t)(ny + 1) * x : y + (int64_t)(ny + 1) * (z + (int64_t)(nz + 1) * x);
    }
    // The element loop is not unrolled: each pass gathers one element's D
    // source values into registers and applies this node's DIM rows of Ke,
    // whose (wave-uniform) entries come through the scalar cache.  Fully
    // unrolling it would keep all of Ke live in registers.
    template <class S>
    __device__ __forceinline__ void apply(int64_t, int iy, int ix, int iz, const S& src, T (&out)[DIM]) const {
        constexpr int CY[8] = {1, 1, 0, 0, 1, 1, 0, 0};
        constexpr int CX[8] = {0, 1, 1, 0, 0, 1, 1, 0};
        constexpr int CZ[8] = {0, 0, 0, 0, 1, 1, 1, 1};
#pragma unroll
        for (int c = 0; c < DIM; ++c) out[c] = T(0);
#pragma unroll 1
        for (int a = 0; a < NC; ++a) {
            const int ey = iy - CY[a], ex = ix - CX[a], ez = iz - CZ[a];
            const bool in = ey >= 0 && ey < ny && ex >= 0 && ex < nx && (DIM == 2 || (ez >= 0 && ez < nz));
            if (!in) continue;
            const int64_t e = DIM == 2 ? ey + (int64_t)ny * ex : ey + (int64_t)ny * (ez + (int64_t)nz * ex);
            const T Ee = E[e];
            T sv[D];
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                const int64_t q = node(ey + CY[b], ex + CX[b], DIM == 2 ? 0 : ez + CZ[b]);
#pragma unroll
                for (int c2 = 0; c2 < DIM; ++c2) sv[b * DIM + c2] = src(q, c2);
            }
            const T* kr = ke + (size_t)a * DIM * D;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                T acc = T(0);
#pragma unroll
                for (int j = 0; j < D; ++j) acc += ld_const(kr + c * D + j) * sv[j];
                out[c] += Ee * acc;
            }
        }
    }
    __device__ __forceinline__ void diag(int64_t, int iy, int ix, int iz, T (&out)[DIM]) const {
        constexpr int CY[8] = {1, 1, 0, 0, 1, 1, 0, 0};
        constexpr int CX[8] = {0, 1, 1, 0, 0, 1, 1, 0};
        constexpr int CZ[8] = {0, 0, 0, 0, 1, 1, 1, 1};
#pragma unroll
        for (int c = 0; c < DIM; ++c) out[c] = T(0);
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            const int ey = iy - CY[a], ex = ix - CX[a], ez = iz - CZ[a];
            const bool in = ey >= 0 && ey < ny && ex >= 0 && ex < nx && (DIM == 2 || (ez >= 0 && ez < nz));
            if (!in) continue;
            const int64_t e = DIM == 2 ? ey + (int64_t)ny * ex : ey + (int64_t)ny * (ez + (int64_t)nz * ex);
            const T Ee = E[e];
#pragma unroll
            for (int c = 0; c < DIM; ++c) out[c] += Ee * ke[(a * DIM + c) * D + a * DIM + c];
        }
    }
};

// 2D: the node's 3x3 neighbourhood is gathered once (18 values of the source,
// one load per neighbour node and component) and the four adjacent element
// rows are applied from registers; element a of the node sees local corner b
// at neighbourhood offset (CY[b] - CY[a], CX[b] - CX[a]).  Fully unrolled, so
// the Ke entries are compile-time offsets into the (wave-uniform) matrix.
template <typename T>
struct MatFree<2, T> {
    const T* __restrict__ E;
    const T* __restrict__ ke;
    int nx, ny, nz;
    int64_t e0 = 0;              // E holds the moduli from element e0 on (a window of them)
    static constexpr int D = 8;

    template <class S>
    __device__ __forceinline__ void apply(int64_t nd, int iy, int ix, int, const S& src, T (&out)[2]) const {
        constexpr int CY[4] = {1, 1, 0, 0};
        constexpr int CX[4] = {0, 1, 1, 0};
        const int64_t col = ny + 1;
        T pv[3][3][2];                       // [dx + 1][dy + 1][component]
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const bool ok = iy + dy >= 0 && iy + dy <= ny && ix + dx >= 0 && ix + dx <= nx;
                const int64_t q = nd + dy + col * dx;
#pragma unroll
                for (int c = 0; c < 2; ++c) pv[dx + 1][dy + 1][c] = ok ? src(q, c) : T(0);
            }
        out[0] = T(0);
        out[1] = T(0);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int ey = iy - CY[a], ex = ix - CX[a];
            if (ey < 0 || ey >= ny || ex < 0 || ex >= nx) continue;
            const T Ee = E[ey + (int64_t)ny * ex - e0];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const T* kr = ke + (a * 2 + c) * D;
                T acc = T(0);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int dy = CY[b] - CY[a], dx = CX[b] - CX[a];
                    acc += ld_const(kr + 2 * b) * pv[dx + 1][dy + 1][0] + ld_const(kr + 2 * b + 1) * pv[dx + 1][dy + 1][1];
                }
                out[c] += Ee * acc;
            }
        }
    }
    __device__ __forceinline__ void diag(int64_t, int iy, int ix, int, T (&out)[2]) const {
        constexpr int CY[4] = {1, 1, 0, 0};
        constexpr int CX[4] = {0, 1, 1, 0};
        out[0] = T(0);
        out[1] = T(0);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int ey = iy - CY[a], ex = ix - CX[a];
            if (ey < 0 || ey >= ny || ex < 0 || ex >= nx) continue;
            const T Ee = E[ey + (int64_t)ny * ex - e0];
#pragma unroll
            for (int c = 0; c < 2; ++c) out[c] += Ee * ke[(a * 2 + c) * D + a * 2 + c];
        }
    }
};

template <int DIM, typename T> struct SrcMask {
    const T* x;
    const uint8_t* fm;
    __device__ __forceinline__ T operator()(int64_t q, int c) const {
        const int64_t i = DIM * q + c;
        return fm[i] ? x[i] : T(0);
    }
};

}  // namespace topt
