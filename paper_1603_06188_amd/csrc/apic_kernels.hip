// HIP kernels of libapic for gfx950 (wave64) and their host-side launchers.
//
// Method: Jiang, Schroeder, Teran, arXiv 1603.06188.  Explicit step at
// lambda = 0: transfer to grid (Sec. 3.2) with the force of Sec. 3.3 fused in,
// grid update (Sec. 3.3), transfer to particles (Sec. 3.4 in the lambda = 0
// form of Sec. 5.7), momenta of Sec. 3.1 / 5.3.
#include "apic_kernels.h"

namespace apic {

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------

static inline int grid_blocks(int64_t work, int threads, int cap = 65536) {
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

template <typename T>
__global__ void k_fill(T *p, int64_t count, T val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

template <typename T>
void launch_fill(T *p, int64_t count, T val, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_blocks(count, 256, 8192)), dim3(256), 0, st, p, count, val);
}
template void launch_fill<float>(float *, int64_t, float, hipStream_t);
template void launch_fill<double>(double *, int64_t, double, hipStream_t);
template void launch_fill<uint32_t>(uint32_t *, int64_t, uint32_t, hipStream_t);

// Grid accumulation: plain atomic add, or atomic add plus the exact rounding
// error of that add (two-sum on the value the atomic returned) into an
// error-term plane.
template <typename T, bool COMP>
__device__ __forceinline__ void accumulate(T *hi, T *lo, int64_t i, T x) {
    if constexpr (!COMP) {
        atomicAdd(hi + i, x);
    } else {
        T old = atomicAdd(hi + i, x);
        T s = old + x;
        T bp = s - old;
        T e = (old - (s - bp)) + (x - bp);
        if (e != T(0)) atomicAdd(lo + i, e);
    }
}

template <int DIM>
__device__ __forceinline__ bool support_inside(const int *base, const GridDims &d, int deg) {
    for (int a = 0; a < DIM; ++a)
        if (base[a] < 0 || base[a] + deg > d.n[a]) return false;
    return true;
}

// ---------------------------------------------------------------------------
// Transfer to grid (Sec. 3.2) + fused force (Sec. 3.3, lambda = 0)
// ---------------------------------------------------------------------------
//
// Per particle: Qc = m_p B_p D^{-1} dx (so that Qc * r_cell = m_p B_p D^{-1}
// (x_i - x_p)) and, for the neo-Hookean model, the Kirchhoff stress
// tau = P F^T = mu (F F^T - I) + lambda ln J I, Ac = -dt V_p tau / dx, so that
// Ac * grad_cell w = dt f-contribution -dt V_p P F^T grad w.
template <typename T, int DIM, int DEG, bool COMP>
__global__ __launch_bounds__(256) void k_p2g(Parts<T> P, GridPlanes<T> g, StepParams<T> prm) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    constexpr int K = DEG + 1;
    const int64_t s = P.s;
    int ci[3] = {0, 0, 0};
    unpack_cell<DIM>(P.cell[p], ci);
    T off[DIM], v[DIM], B[DIM * DIM], F[DIM * DIM];
    T m = P.m[p];
    bool finite = is_finite(m);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        off[a] = P.off[a * s + p];
        v[a] = P.v[a * s + p];
        finite = finite && is_finite(off[a]) && is_finite(v[a]);
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        B[k] = P.B[k * s + p];
        F[k] = P.F[k * s + p];
        finite = finite && is_finite(B[k]) && is_finite(F[k]);
    }
    if (!finite) {
        atomicOr(g.flags, FLAG_NONFINITE);
        return;
    }
    Axis<T, DEG> ax[DIM];
    int base[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        axis_weights<T, DEG>(ci[a], off[a], ax[a]);
        base[a] = ax[a].base;
    }
    if (!support_inside<DIM>(base, g.d, DEG)) {
        atomicOr(g.flags, FLAG_OUT_OF_DOMAIN);
        return;
    }
    // affine momentum matrix in cell units
    T Qc[DIM * DIM], Ac[DIM * DIM];
    const T qs = m * inv_D_factor<T, DEG>() * g.inv_dx;
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        Qc[k] = qs * B[k];
        Ac[k] = T(0);
    }
    if (prm.model == 1) {
        T J;
        if constexpr (DIM == 3)
            J = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
                F[2] * (F[3] * F[7] - F[4] * F[6]);
        else
            J = F[0] * F[3] - F[1] * F[2];
        if (J > T(0)) {
            const T lnJ = log_t(J);
            const T sc = -prm.dt * m * prm.inv_rho0 * g.inv_dx;
#pragma unroll
            for (int r = 0; r < DIM; ++r)
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    T ff = T(0);
#pragma unroll
                    for (int k = 0; k < DIM; ++k) ff += F[r * DIM + k] * F[c * DIM + k];
                    T tau = prm.mu * (ff - (r == c ? T(1) : T(0))) + (r == c ? prm.lam * lnJ : T(0));
                    Ac[r * DIM + c] = sc * tau;
                }
        } else {
            atomicOr(g.flags, FLAG_INVERTED);
        }
    }
    T mv0[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) mv0[a] = m * v[a];
    const int64_t G = g.d.G;
    if constexpr (DIM == 3) {
#pragma unroll
        for (int kz = 0; kz < K; ++kz)
#pragma unroll
            for (int ky = 0; ky < K; ++ky)
#pragma unroll
                for (int kx = 0; kx < K; ++kx) {
                    const T wyz = ax[1].w[ky] * ax[2].w[kz];
                    const T w = ax[0].w[kx] * wyz;
                    const T gw[3] = {ax[0].dw[kx] * wyz, ax[0].w[kx] * ax[1].dw[ky] * ax[2].w[kz],
                                     ax[0].w[kx] * ax[1].w[ky] * ax[2].dw[kz]};
                    const T rc[3] = {ax[0].r[kx], ax[1].r[ky], ax[2].r[kz]};
                    const int64_t i = node_index<3>(base[0] + kx, base[1] + ky, base[2] + kz, g.d.TN);
                    accumulate<T, COMP>(g.m, g.cm, i, w * m);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        T val = mv0[a] + Qc[a * 3 + 0] * rc[0] + Qc[a * 3 + 1] * rc[1] + Qc[a * 3 + 2] * rc[2];
                        val = w * val + Ac[a * 3 + 0] * gw[0] + Ac[a * 3 + 1] * gw[1] + Ac[a * 3 + 2] * gw[2];
                        accumulate<T, COMP>(g.mv + a * G, g.cmv + a * G, i, val);
                    }
                }
    } else {
#pragma unroll
        for (int ky = 0; ky < K; ++ky)
#pragma unroll
            for (int kx = 0; kx < K; ++kx) {
                const T w = ax[0].w[kx] * ax[1].w[ky];
                const T gw[2] = {ax[0].dw[kx] * ax[1].w[ky], ax[0].w[kx] * ax[1].dw[ky]};
                const T rc[2] = {ax[0].r[kx], ax[1].r[ky]};
                const int64_t i = node_index<2>(base[0] + kx, base[1] + ky, 0, g.d.TN);
                accumulate<T, COMP>(g.m, g.cm, i, w * m);
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    T val = mv0[a] + Qc[a * 2 + 0] * rc[0] + Qc[a * 2 + 1] * rc[1];
                    val = w * val + Ac[a * 2 + 0] * gw[0] + Ac[a * 2 + 1] * gw[1];
                    accumulate<T, COMP>(g.mv + a * G, g.cmv + a * G, i, val);
                }
            }
    }
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_p2g(const Parts<T> &P, const GridPlanes<T> &g, const StepParams<T> &prm, hipStream_t st) {
    const int64_t planes = 1 + DIM;
    launch_fill<T>(g.m, g.d.G, T(0), st);
    launch_fill<T>(g.mv, g.d.G * DIM, T(0), st);
    if (COMP) {
        launch_fill<T>(g.cm, g.d.G, T(0), st);
        launch_fill<T>(g.cmv, g.d.G * DIM, T(0), st);
    }
    (void)planes;
    if (P.n == 0) return;
    hipLaunchKernelGGL((k_p2g<T, DIM, DEG, COMP>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P, g,
                       prm);
}

// ---------------------------------------------------------------------------
// Grid update (Sec. 3.3 at lambda = 0)
// ---------------------------------------------------------------------------
template <typename T, int DIM, bool COMP>
__global__ __launch_bounds__(256) void k_grid_update(GridPlanes<T> g, StepParams<T> prm) {
    const int64_t G = g.d.G;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G; i += (int64_t)gridDim.x * blockDim.x) {
        int c[3] = {0, 0, 0};
        node_coords<DIM>(i, g.d.TN, c);
        bool valid = true;
        bool sticky = false;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            valid = valid && c[a] < g.d.N[a];
            sticky = sticky || c[a] < prm.band[2 * a] || c[a] > g.d.n[a] - prm.band[2 * a + 1];
        }
        T m = g.m[i];
        if (COMP) m += g.cm[i];
        const bool live = valid && m > T(0) && !sticky;
        const T inv_m = live ? T(1) / m : T(0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            T mv = g.mv[a * G + i];
            if (COMP) mv += g.cmv[a * G + i];
            g.vt[a * G + i] = live ? mv * inv_m + prm.dt * prm.g[a] : T(0);
        }
    }
}

template <typename T, int DIM, bool COMP>
void launch_grid_update(const GridPlanes<T> &g, const StepParams<T> &prm, hipStream_t st) {
    hipLaunchKernelGGL((k_grid_update<T, DIM, COMP>), dim3(grid_blocks(g.d.G, 256, 16384)), dim3(256), 0, st, g,
                       prm);
}

// ---------------------------------------------------------------------------
// Transfer to particles (Sec. 3.4, lambda = 0 forms of Sec. 5.7)
// ---------------------------------------------------------------------------
template <typename T, int DIM, int DEG>
__global__ __launch_bounds__(256) void k_g2p(Parts<T> P, GridPlanes<T> g, StepParams<T> prm) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    constexpr int K = DEG + 1;
    const int64_t s = P.s;
    int ci[3] = {0, 0, 0};
    unpack_cell<DIM>(P.cell[p], ci);
    T off[DIM], F[DIM * DIM];
    bool finite = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        off[a] = P.off[a * s + p];
        finite = finite && is_finite(off[a]);
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        F[k] = P.F[k * s + p];
        finite = finite && is_finite(F[k]);
    }
    if (!finite) {
        atomicOr(g.flags, FLAG_NONFINITE);
        return;
    }
    Axis<T, DEG> ax[DIM];
    int base[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        axis_weights<T, DEG>(ci[a], off[a], ax[a]);
        base[a] = ax[a].base;
    }
    if (!support_inside<DIM>(base, g.d, DEG)) {
        atomicOr(g.flags, FLAG_OUT_OF_DOMAIN);
        return;
    }
    const int64_t G = g.d.G;
    T vn[DIM], Bc[DIM * DIM], Gc[DIM * DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) vn[a] = T(0);
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        Bc[k] = T(0);
        Gc[k] = T(0);
    }
    if constexpr (DIM == 3) {
#pragma unroll
        for (int kz = 0; kz < K; ++kz)
#pragma unroll
            for (int ky = 0; ky < K; ++ky)
#pragma unroll
                for (int kx = 0; kx < K; ++kx) {
                    const T wyz = ax[1].w[ky] * ax[2].w[kz];
                    const T w = ax[0].w[kx] * wyz;
                    const T gw[3] = {ax[0].dw[kx] * wyz, ax[0].w[kx] * ax[1].dw[ky] * ax[2].w[kz],
                                     ax[0].w[kx] * ax[1].w[ky] * ax[2].dw[kz]};
                    const T rc[3] = {ax[0].r[kx], ax[1].r[ky], ax[2].r[kz]};
                    const int64_t i = node_index<3>(base[0] + kx, base[1] + ky, base[2] + kz, g.d.TN);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const T vt = g.vt[a * G + i];
                        const T wv = w * vt;
                        vn[a] += wv;
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            Bc[a * 3 + b] += wv * rc[b];
                            Gc[a * 3 + b] += vt * gw[b];
                        }
                    }
                }
    } else {
#pragma unroll
        for (int ky = 0; ky < K; ++ky)
#pragma unroll
            for (int kx = 0; kx < K; ++kx) {
                const T w = ax[0].w[kx] * ax[1].w[ky];
                const T gw[2] = {ax[0].dw[kx] * ax[1].w[ky], ax[0].w[kx] * ax[1].dw[ky]};
                const T rc[2] = {ax[0].r[kx], ax[1].r[ky]};
                const int64_t i = node_index<2>(base[0] + kx, base[1] + ky, 0, g.d.TN);
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const T vt = g.vt[a * G + i];
                    const T wv = w * vt;
                    vn[a] += wv;
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        Bc[a * 2 + b] += wv * rc[b];
                        Gc[a * 2 + b] += vt * gw[b];
                    }
                }
            }
    }
    // F <- (I + dt grad v) F with grad v = Gc / dx
    const T gs = prm.dt * g.inv_dx;
    T Fn[DIM * DIM];
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            T acc = F[r * DIM + c];
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc += gs * Gc[r * DIM + k] * F[k * DIM + c];
            Fn[r * DIM + c] = acc;
        }
    // x <- x + dt v, kept as cell index + offset
    bool cfl = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        T step = prm.dt * vn[a] * g.inv_dx;
        cfl = cfl || !(step <= T(1) && step >= T(-1));
        T o = off[a] + step;
        T fl = floor_t(o);
        int cc = ci[a] + (int)fl;
        o -= fl;
        if (o >= T(1)) {
            o -= T(1);
            cc += 1;
        }
        // keep the packed index representable; a particle that left the
        // grid is flagged by the next transfer that visits it
        ci[a] = cc < 0 ? 0 : (cc > g.d.n[a] - 1 ? g.d.n[a] - 1 : cc);
        off[a] = o;
    }
    if (cfl) atomicOr(g.flags, FLAG_CFL);
    P.cell[p] = pack_cell<DIM>(ci);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        P.off[a * s + p] = off[a];
        P.v[a * s + p] = vn[a];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        P.B[k * s + p] = Bc[k] * g.dx;
        P.F[k * s + p] = Fn[k];
    }
}

template <typename T, int DIM, int DEG>
void launch_g2p(const Parts<T> &P, const GridPlanes<T> &g, const StepParams<T> &prm, hipStream_t st) {
    if (P.n == 0) return;
    hipLaunchKernelGGL((k_g2p<T, DIM, DEG>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P, g, prm);
}

// ---------------------------------------------------------------------------
// Sort: stable counting sort by the tile-major index of the base node.
// ---------------------------------------------------------------------------
template <typename T, int DIM, int DEG>
__global__ __launch_bounds__(256) void k_sort_keys(Parts<T> P, GridDims d, uint32_t *keys, uint32_t *counts) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    int ci[3] = {0, 0, 0};
    unpack_cell<DIM>(P.cell[p], ci);
    int base[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        T o = P.off[a * P.s + p];
        ok = ok && is_finite(o);
        if constexpr (DEG == 2)
            base[a] = (o < T(0.5)) ? ci[a] - 1 : ci[a];
        else
            base[a] = ci[a] - 1;
        ok = ok && base[a] >= 0 && base[a] + DEG <= d.n[a];
    }
    uint32_t key = ok ? (uint32_t)node_index<DIM>(base[0], base[1], base[2], d.TN) : (uint32_t)d.G;
    keys[p] = key;
    atomicAdd(counts + key, 1u);
}

// Exclusive scan of `count` uint32 values in place; block sums go to `sums`.
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t *data, int64_t count, uint32_t *sums) {
    __shared__ uint32_t sh[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    uint32_t x = i < count ? data[i] : 0u;
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t y = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += y;
        __syncthreads();
    }
    if (i < count) data[i] = sh[threadIdx.x] - x;
    if (threadIdx.x == 1023) sums[blockIdx.x] = sh[1023];
}

// Single-block exclusive scan of the block sums (any length).
__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *sums, int64_t count) {
    __shared__ uint32_t sh[1024];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t start = 0; start < count; start += 1024) {
        const int64_t i = start + threadIdx.x;
        uint32_t x = i < count ? sums[i] : 0u;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            uint32_t y = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0u;
            __syncthreads();
            sh[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < count) sums[i] = sh[threadIdx.x] - x + carry;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_scan_add(uint32_t *data, int64_t count, const uint32_t *sums) {
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < count) data[i] += sums[blockIdx.x];
}

void launch_exclusive_scan(uint32_t *data, int64_t count, uint32_t *sums, hipStream_t st) {
    const int64_t nb = (count + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(1024), 0, st, data, count, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, sums, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(1024), 0, st, data, count, sums);
}

__global__ __launch_bounds__(256) void k_copy_u32(const uint32_t *src, uint32_t *dst, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_sort_slots(int64_t n, const uint32_t *keys, uint32_t *cursor,
                                                     uint32_t *perm) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t slot = atomicAdd(cursor + keys[p], 1u);
    perm[slot] = (uint32_t)p;
}

// Each key's segment [starts[k], starts[k+1]) is put in ascending particle
// order, which makes the counting sort stable and deterministic.
__global__ __launch_bounds__(256) void k_sort_fix(int64_t nkeys, const uint32_t *starts, uint32_t *perm) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nkeys) return;
    const uint32_t lo = starts[k], hi = starts[k + 1];
    for (uint32_t i = lo + 1; i < hi; ++i) {
        uint32_t x = perm[i];
        uint32_t j = i;
        while (j > lo && perm[j - 1] > x) {
            perm[j] = perm[j - 1];
            --j;
        }
        perm[j] = x;
    }
}

// dst[j] = src[perm[j]] for every plane.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_gather_state(Parts<T> src, Parts<T> dst, const uint32_t *perm) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= src.n) return;
    const int64_t p = perm[j];
    dst.cell[j] = src.cell[p];
    dst.m[j] = src.m[p];
    if (src.id) dst.id[j] = src.id[p];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        dst.off[a * dst.s + j] = src.off[a * src.s + p];
        dst.v[a * dst.s + j] = src.v[a * src.s + p];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        dst.B[k * dst.s + j] = src.B[k * src.s + p];
        dst.F[k * dst.s + j] = src.F[k * src.s + p];
    }
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_copy_state(Parts<T> src, Parts<T> dst) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= src.n) return;
    dst.cell[j] = src.cell[j];
    dst.m[j] = src.m[j];
    if (src.id) dst.id[j] = src.id[j];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        dst.off[a * dst.s + j] = src.off[a * src.s + j];
        dst.v[a * dst.s + j] = src.v[a * src.s + j];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        dst.B[k * dst.s + j] = src.B[k * src.s + j];
        dst.F[k * dst.s + j] = src.F[k * src.s + j];
    }
}

template <typename T, int DIM, int DEG>
void launch_sort(const Parts<T> &P, const Parts<T> &shadow, const GridDims &d, const SortBuffers &sb,
                 hipStream_t st) {
    if (P.n == 0) return;
    const int64_t nkeys = d.G + 1;  // key G collects particles that cannot be binned
    const unsigned pb = (unsigned)((P.n + 255) / 256);
    launch_fill<uint32_t>(sb.counts, nkeys + 1, 0u, st);
    hipLaunchKernelGGL((k_sort_keys<T, DIM, DEG>), dim3(pb), dim3(256), 0, st, P, d, sb.keys, sb.counts);
    launch_exclusive_scan(sb.counts, nkeys + 1, sb.sums, st);
    // cursor = starts (copy), then slots
    hipLaunchKernelGGL(k_copy_u32, dim3(grid_blocks(nkeys + 1, 256, 8192)), dim3(256), 0, st, sb.counts, sb.cursor,
                       nkeys + 1);
    hipLaunchKernelGGL(k_sort_slots, dim3(pb), dim3(256), 0, st, P.n, sb.keys, sb.cursor, sb.perm);
    hipLaunchKernelGGL(k_sort_fix, dim3(grid_blocks(nkeys, 256, 1 << 30)), dim3(256), 0, st, nkeys, sb.counts,
                       sb.perm);
    Parts<T> dst = shadow;
    dst.n = P.n;
    Parts<T> src = P;
    if (!P.id) {
        src.id = nullptr;
        dst.id = nullptr;
    }
    hipLaunchKernelGGL((k_gather_state<T, DIM>), dim3(pb), dim3(256), 0, st, src, dst, sb.perm);
    hipLaunchKernelGGL((k_copy_state<T, DIM>), dim3(pb), dim3(256), 0, st, dst, src);
}

// ---------------------------------------------------------------------------
// Binary64 totals (Sec. 3.1, Sec. 5.3)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_reduce8(double *acc, double *partials) {
    __shared__ double sh[8][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        double x = acc[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if (lane == 0) sh[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[threadIdx.x][w];
        partials[blockIdx.x * 8 + threadIdx.x] = t;
    }
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_diag_particles(Parts<T> P, double dx, double *partials) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P.n; p += (int64_t)gridDim.x * blockDim.x) {
        int ci[3] = {0, 0, 0};
        unpack_cell<DIM>(P.cell[p], ci);
        double x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, Bm[9];
        const double m = (double)P.m[p];
        for (int a = 0; a < DIM; ++a) {
            x[a] = ((double)ci[a] + (double)P.off[a * P.s + p]) * dx;
            v[a] = (double)P.v[a * P.s + p];
        }
        for (int k = 0; k < DIM * DIM; ++k) Bm[k] = (double)P.B[k * P.s + p];
        double mv[3] = {m * v[0], m * v[1], m * v[2]};
        acc[0] += mv[0];
        acc[1] += mv[1];
        acc[2] += mv[2];
        if constexpr (DIM == 3) {
            // x x m v + m (B^T : eps): components B_zy - B_yz, B_xz - B_zx, B_yx - B_xy
            acc[3] += x[1] * mv[2] - x[2] * mv[1] + m * (Bm[7] - Bm[5]);
            acc[4] += x[2] * mv[0] - x[0] * mv[2] + m * (Bm[2] - Bm[6]);
            acc[5] += x[0] * mv[1] - x[1] * mv[0] + m * (Bm[3] - Bm[1]);
        } else {
            acc[5] += x[0] * mv[1] - x[1] * mv[0] + m * (Bm[2] - Bm[1]);
        }
        double v2 = 0.0;
        for (int a = 0; a < DIM; ++a) v2 += v[a] * v[a];
        acc[6] += 0.5 * m * v2;
        acc[7] += m;
    }
    block_reduce8(acc, partials);
}

template <typename T, int DIM, bool COMP>
__global__ __launch_bounds__(256) void k_diag_grid(GridPlanes<T> g, int which, double dt, double *partials) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t G = g.d.G;
    const double dx = (double)g.dx;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G; i += (int64_t)gridDim.x * blockDim.x) {
        double m = (double)g.m[i];
        if (COMP) m += (double)g.cm[i];
        if (!(m > 0.0)) continue;
        int c[3] = {0, 0, 0};
        node_coords<DIM>(i, g.d.TN, c);
        double x[3] = {0, 0, 0}, mv[3] = {0, 0, 0};
        for (int a = 0; a < DIM; ++a) {
            x[a] = (double)c[a] * dx;
            if (which == 1) {
                mv[a] = (double)g.mv[a * G + i];
                if (COMP) mv[a] += (double)g.cmv[a * G + i];
            } else {
                const double vt = (double)g.vt[a * G + i];
                mv[a] = m * vt;
                x[a] += dt * vt;
            }
        }
        acc[0] += mv[0];
        acc[1] += mv[1];
        acc[2] += mv[2];
        if constexpr (DIM == 3) {
            acc[3] += x[1] * mv[2] - x[2] * mv[1];
            acc[4] += x[2] * mv[0] - x[0] * mv[2];
        }
        acc[5] += x[0] * mv[1] - x[1] * mv[0];
        double p2 = 0.0;
        for (int a = 0; a < DIM; ++a) p2 += mv[a] * mv[a];
        acc[6] += 0.5 * p2 / m;
        acc[7] += m;
    }
    block_reduce8(acc, partials);
}

__global__ void k_diag_final(const double *partials, int nb, double *out) {
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += partials[b * 8 + threadIdx.x];
        out[threadIdx.x] = t;
    }
}

template <typename T, int DIM>
void launch_diag_particles(const Parts<T> &P, double dx, double *partials, double *out, hipStream_t st) {
    const int nb = grid_blocks(P.n, 256, kDiagBlocks);
    hipLaunchKernelGGL((k_diag_particles<T, DIM>), dim3(nb), dim3(256), 0, st, P, dx, partials);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, st, partials, nb, out);
}

template <typename T, int DIM, bool COMP>
void launch_diag_grid(const GridPlanes<T> &g, int which, double dt, double *partials, double *out, hipStream_t st) {
    const int nb = grid_blocks(g.d.G, 256, kDiagBlocks);
    hipLaunchKernelGGL((k_diag_grid<T, DIM, COMP>), dim3(nb), dim3(256), 0, st, g, which, dt, partials);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, st, partials, nb, out);
}

// ---------------------------------------------------------------------------
// Grid export to a dense node-major buffer; position packing
// ---------------------------------------------------------------------------
template <typename T, int DIM, bool COMP>
__global__ __launch_bounds__(256) void k_grid_export(GridPlanes<T> g, int field, T *out) {
    int64_t count = 1;
    for (int a = 0; a < DIM; ++a) count *= g.d.N[a];
    const int comps = field == 0 ? 1 : DIM;
    const int64_t G = g.d.G;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += (int64_t)gridDim.x * blockDim.x) {
        int c[3] = {0, 0, 0};
        int64_t r = j;
        for (int a = 0; a < DIM; ++a) {
            c[a] = (int)(r % g.d.N[a]);
            r /= g.d.N[a];
        }
        const int64_t i = node_index<DIM>(c[0], c[1], c[2], g.d.TN);
        for (int k = 0; k < comps; ++k) {
            T val;
            if (field == 0) {
                val = g.m[i];
                if (COMP) val += g.cm[i];
            } else if (field == 1) {
                val = g.mv[k * G + i];
                if (COMP) val += g.cmv[k * G + i];
            } else {
                val = g.vt[k * G + i];
            }
            out[k * count + j] = val;
        }
    }
}

template <typename T, int DIM, bool COMP>
void launch_grid_export(const GridPlanes<T> &g, int field, T *out, hipStream_t st) {
    int64_t count = 1;
    for (int a = 0; a < DIM; ++a) count *= g.d.N[a];
    hipLaunchKernelGGL((k_grid_export<T, DIM, COMP>), dim3(grid_blocks(count, 256, 16384)), dim3(256), 0, st, g,
                       field, out);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_pack_positions(Parts<T> P, const double *x, double inv_dx) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    int ci[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) {
        const double sx = x[a * P.s + p] * inv_dx;
        double c = floor(sx);
        T o = (T)(sx - c);
        if (o >= T(1)) {
            o = T(0);
            c += 1.0;
        }
        ci[a] = (int)c;
        P.off[a * P.s + p] = o;
    }
    P.cell[p] = pack_cell<DIM>(ci);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_unpack_positions(Parts<T> P, double *x, double dx) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    int ci[3] = {0, 0, 0};
    unpack_cell<DIM>(P.cell[p], ci);
    for (int a = 0; a < DIM; ++a) x[a * P.s + p] = ((double)ci[a] + (double)P.off[a * P.s + p]) * dx;
}

template <typename T, int DIM>
void launch_pack_positions(const Parts<T> &P, const double *x, double dx, hipStream_t st) {
    if (P.n == 0) return;
    hipLaunchKernelGGL((k_pack_positions<T, DIM>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P, x,
                       1.0 / dx);
}

template <typename T, int DIM>
void launch_unpack_positions(const Parts<T> &P, double *x, double dx, hipStream_t st) {
    if (P.n == 0) return;
    hipLaunchKernelGGL((k_unpack_positions<T, DIM>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P, x,
                       dx);
}

// ---------------------------------------------------------------------------
// Explicit instantiations
// ---------------------------------------------------------------------------
#define APIC_INST_TD(T, DIM)                                                                                   \
    template void launch_diag_particles<T, DIM>(const Parts<T> &, double, double *, double *, hipStream_t);  \
    template void launch_diag_grid<T, DIM, false>(const GridPlanes<T> &, int, double, double *, double *,     \
                                                  hipStream_t);                                              \
    template void launch_diag_grid<T, DIM, true>(const GridPlanes<T> &, int, double, double *, double *,      \
                                                 hipStream_t);                                               \
    template void launch_grid_export<T, DIM, false>(const GridPlanes<T> &, int, T *, hipStream_t);            \
    template void launch_grid_export<T, DIM, true>(const GridPlanes<T> &, int, T *, hipStream_t);             \
    template void launch_grid_update<T, DIM, false>(const GridPlanes<T> &, const StepParams<T> &, hipStream_t); \
    template void launch_grid_update<T, DIM, true>(const GridPlanes<T> &, const StepParams<T> &, hipStream_t);  \
    template void launch_pack_positions<T, DIM>(const Parts<T> &, const double *, double, hipStream_t);        \
    template void launch_unpack_positions<T, DIM>(const Parts<T> &, double *, double, hipStream_t);

#define APIC_INST_TDK(T, DIM, DEG)                                                                             \
    template void launch_p2g<T, DIM, DEG, false>(const Parts<T> &, const GridPlanes<T> &, const StepParams<T> &, \
                                                 hipStream_t);                                               \
    template void launch_p2g<T, DIM, DEG, true>(const Parts<T> &, const GridPlanes<T> &, const StepParams<T> &,  \
                                                hipStream_t);                                                \
    template void launch_g2p<T, DIM, DEG>(const Parts<T> &, const GridPlanes<T> &, const StepParams<T> &,      \
                                          hipStream_t);                                                      \
    template void launch_sort<T, DIM, DEG>(const Parts<T> &, const Parts<T> &, const GridDims &,                \
                                           const SortBuffers &, hipStream_t);

APIC_INST_TD(float, 2)
APIC_INST_TD(float, 3)
APIC_INST_TD(double, 2)
APIC_INST_TD(double, 3)
APIC_INST_TDK(float, 2, 2)
APIC_INST_TDK(float, 2, 3)
APIC_INST_TDK(float, 3, 2)
APIC_INST_TDK(float, 3, 3)
APIC_INST_TDK(double, 2, 2)
APIC_INST_TDK(double, 2, 3)
APIC_INST_TDK(double, 3, 2)
APIC_INST_TDK(double, 3, 3)

}  // namespace apic
