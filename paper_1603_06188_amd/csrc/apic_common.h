// Shared device/host definitions of libapic (gfx950).
//
// Method: Jiang, Schroeder, Teran, "An angular momentum conserving
// Affine-Particle-In-Cell method" (arXiv 1603.06188), explicit step at
// lambda = 0 (Sec. 3.2-3.5, lambda = 0 forms of Sec. 5.7).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apic {

// ---------------------------------------------------------------------------
// Workspace / grid description shared by host and device
// ---------------------------------------------------------------------------

// Grid nodes are stored tile-major: 4x4x4-node tiles in 3D, 8x8 in 2D, 64
// nodes per tile, tiles in x-fastest order.  Planes are `G` nodes long
// (node count padded to whole tiles).
struct GridDims {
    int dim, deg;
    int n[3];      // cells per axis
    int N[3];      // nodes per axis = n + 1
    int TN[3];     // tiles per axis
    int64_t tiles; // tile count
    int64_t G;     // padded node count = tiles * 64
};

template <typename T>
struct Parts {
    uint32_t *cell;
    T *off, *v, *B, *F, *m;
    int32_t *id;
    int64_t n, s;  // count, plane stride
};

template <typename T>
struct GridPlanes {
    T *m;      // 1 plane
    T *mv;     // dim planes: (m v)_i + dt f_i
    T *vt;     // dim planes: updated velocity
    T *cm;     // 1 plane error term of m  (compensated option)
    T *cmv;    // dim planes error term of mv
    uint32_t *flags;
    GridDims d;
    T dx, inv_dx;
};

template <typename T>
struct StepParams {
    T dt;
    T g[3];
    int model;
    int band[6];
    T mu, lam, inv_rho0;
};

enum : uint32_t {
    FLAG_OUT_OF_DOMAIN = 1u,
    FLAG_NONFINITE = 2u,
    FLAG_INVERTED = 4u,
    FLAG_CFL = 8u,
};

// ---------------------------------------------------------------------------
// Packed cell index and tiled node index
// ---------------------------------------------------------------------------

template <int DIM>
__device__ __forceinline__ void unpack_cell(uint32_t c, int *ci) {
    if constexpr (DIM == 3) {
        ci[0] = (int)(c & 1023u);
        ci[1] = (int)((c >> 10) & 1023u);
        ci[2] = (int)(c >> 20);
    } else {
        ci[0] = (int)(c & 0xFFFFu);
        ci[1] = (int)(c >> 16);
    }
}

template <int DIM>
__device__ __forceinline__ uint32_t pack_cell(const int *ci) {
    if constexpr (DIM == 3)
        return (uint32_t)ci[0] | ((uint32_t)ci[1] << 10) | ((uint32_t)ci[2] << 20);
    else
        return (uint32_t)ci[0] | ((uint32_t)ci[1] << 16);
}

template <int DIM>
__host__ __device__ __forceinline__ int64_t node_index(int ix, int iy, int iz, const int *TN) {
    if constexpr (DIM == 3) {
        int64_t t = (int64_t)(ix >> 2) + (int64_t)TN[0] * ((iy >> 2) + (int64_t)TN[1] * (iz >> 2));
        return t * 64 + ((ix & 3) | ((iy & 3) << 2) | ((iz & 3) << 4));
    } else {
        int64_t t = (int64_t)(ix >> 3) + (int64_t)TN[0] * (iy >> 3);
        return t * 64 + ((ix & 7) | ((iy & 7) << 3));
    }
}

// Inverse of node_index: tiled index -> node coordinates.
template <int DIM>
__host__ __device__ __forceinline__ void node_coords(int64_t i, const int *TN, int *c) {
    int64_t t = i >> 6;
    int l = (int)(i & 63);
    if constexpr (DIM == 3) {
        int tx = (int)(t % TN[0]);
        int64_t r = t / TN[0];
        int ty = (int)(r % TN[1]);
        int tz = (int)(r / TN[1]);
        c[0] = tx * 4 + (l & 3);
        c[1] = ty * 4 + ((l >> 2) & 3);
        c[2] = tz * 4 + (l >> 4);
    } else {
        int tx = (int)(t % TN[0]);
        int ty = (int)(t / TN[0]);
        c[0] = tx * 8 + (l & 7);
        c[1] = ty * 8 + (l >> 3);
    }
}

// ---------------------------------------------------------------------------
// Quadratic / cubic B-spline weights along one axis (Sec. 3.5), in cell
// units, relative to the base node of the kernel support.
//
// Quadratic: base = the node nearest below x/dx - 1/2; with c = x/dx - base - 1
// in [-1/2, 1/2), the three weights are 1/2 (1/2 - c)^2, 3/4 - c^2,
// 1/2 (1/2 + c)^2.  Cubic: base = cell - 1, u = offset in [0, 1), q = 1 - u:
// q^3/6, u^3/2 - u^2 + 2/3, q^3/2 - q^2 + 2/3, u^3/6.
// w[k]: weight of node base+k; dw[k]: d w[k] / d x_p (cell units);
// r[k]: (x_{base+k} - x_p) / dx.
// ---------------------------------------------------------------------------
template <typename T, int DEG>
struct Axis {
    int base;
    T w[DEG + 1], dw[DEG + 1], r[DEG + 1];
};

template <typename T, int DEG>
__device__ __forceinline__ void axis_weights(int cell, T off, Axis<T, DEG> &a) {
    if constexpr (DEG == 2) {
        const T half = T(0.5);
        bool lower = off < half;
        a.base = lower ? cell - 1 : cell;
        T c = lower ? off : off - T(1);
        T l = half - c, h = half + c;
        a.w[0] = half * l * l;
        a.w[1] = T(0.75) - c * c;
        a.w[2] = half * h * h;
        a.dw[0] = -l;
        a.dw[1] = T(-2) * c;
        a.dw[2] = h;
        a.r[0] = T(-1) - c;
        a.r[1] = -c;
        a.r[2] = T(1) - c;
    } else {
        const T u = off, q = T(1) - off;
        const T u2 = u * u, q2 = q * q;
        a.base = cell - 1;
        a.w[0] = q2 * q * T(1.0 / 6.0);
        a.w[1] = T(0.5) * u2 * u - u2 + T(2.0 / 3.0);
        a.w[2] = T(0.5) * q2 * q - q2 + T(2.0 / 3.0);
        a.w[3] = u2 * u * T(1.0 / 6.0);
        a.dw[0] = T(-0.5) * q2;
        a.dw[1] = T(1.5) * u2 - T(2) * u;
        a.dw[2] = T(2) * q - T(1.5) * q2;
        a.dw[3] = T(0.5) * u2;
        a.r[0] = T(-1) - u;
        a.r[1] = -u;
        a.r[2] = T(1) - u;
        a.r[3] = T(2) - u;
    }
}

// 1 / k with D_p = k dx^2 I: k = 1/4 (quadratic), 1/3 (cubic) (Sec. 5.6).
template <typename T, int DEG>
__host__ __device__ constexpr T inv_D_factor() {
    return DEG == 2 ? T(4) : T(3);
}

template <typename T>
__device__ __forceinline__ bool is_finite(T x) {
    return __builtin_isfinite(x);
}

template <typename T>
__device__ __forceinline__ T log_t(T x);
template <>
__device__ __forceinline__ float log_t<float>(float x) { return logf(x); }
template <>
__device__ __forceinline__ double log_t<double>(double x) { return log(x); }

template <typename T>
__device__ __forceinline__ T floor_t(T x);
template <>
__device__ __forceinline__ float floor_t<float>(float x) { return floorf(x); }
template <>
__device__ __forceinline__ double floor_t<double>(double x) { return floor(x); }

}  // namespace apic
