// Implicit midpoint step (the lambda = 1/2 member of the grid update of
// Sec. 3.3), solved as the minimization of Sec. 4.1 with Newton's method and
// the mass-inner-product conjugate gradient of Sec. 4.2.  Binary64 throughout.
//
// Layout: dense node arrays (node ix + N0 (iy + N1 iz)), component-major
// vectors (component a of node i at a * nodes + i).  Once per step the
// particles are counting-sorted by base node and what the solve reads is
// copied in that order; particle kernels then write one matrix per particle
// and node kernels collect it over the sorted ranges of the base keys around
// each node (no atomics in the Newton loop).  Node kernels leave one partial
// sum per block, summed in a fixed order by k_mid_reduce.  The transfer to
// particles reads the caller's order.
#include "apic_kernels.h"

namespace apic {

namespace {

constexpr int kMidBlock = 256;
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * kMidBlock + threadIdx.x; }


// Sum of K values over the block; thread 0 writes them to part[blockIdx * K].
template <int K>
__device__ __forceinline__ void block_partials(double (&acc)[K], double *part) {
    __shared__ double red[K][kMidBlock / 64];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double v = acc[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        acc[k] = v;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[k][wave] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < kMidBlock / 64; ++w) s += red[k][w];
            part[(int64_t)blockIdx.x * K + k] = s;
        }
}

template <int DIM>
__device__ __forceinline__ void node_coords(int64_t i, const MidGrid &g, int *c) {
    c[0] = (int)(i % g.N[0]);
    const int64_t q = i / g.N[0];
    if constexpr (DIM == 3) {
        c[1] = (int)(q % g.N[1]);
        c[2] = (int)(q / g.N[1]);
    } else {
        c[1] = (int)q;
    }
}

// Per-axis weights of particle p; false when its support leaves the grid.
template <int DIM, int DEG>
__device__ __forceinline__ bool particle_axes(const Parts<double> &P, int64_t p, const MidGrid &g,
                                              Axis<double, DEG> (&ax)[DIM]) {
    int ci[3];
    unpack_cell<DIM>(P.cell[p], ci);
    bool ok = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        axis_weights<double, DEG>(ci[a], P.off[a * P.s + p], ax[a]);
        ok = ok && ax[a].base >= 0 && ax[a].base + DEG < g.N[a];
    }
    return ok;
}

// Visits the support: f(node index, w, grad w (cell units), r (cell units)).
template <int DIM, int DEG, typename Fn>
__device__ __forceinline__ void for_support(const Axis<double, DEG> (&ax)[DIM], const MidGrid &g, Fn &&fn) {
    constexpr int K = DEG + 1;
    if constexpr (DIM == 3) {
        // cubic: z rows one at a time (unrolling all 64 nodes hoists every load)
#pragma unroll (DEG == 2 ? K : 1)
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double wyz = ax[1].w[j] * ax[2].w[k];
                const int64_t row = (int64_t)g.N[0] * ((ax[1].base + j) + (int64_t)g.N[1] * (ax[2].base + k));
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const double w = ax[0].w[i] * wyz;
                    const double gw[3] = {ax[0].dw[i] * wyz, ax[0].w[i] * ax[1].dw[j] * ax[2].w[k],
                                          ax[0].w[i] * ax[1].w[j] * ax[2].dw[k]};
                    const double r[3] = {ax[0].r[i], ax[1].r[j], ax[2].r[k]};
                    fn(row + ax[0].base + i, w, gw, r);
                }
            }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t row = (int64_t)g.N[0] * (ax[1].base + j);
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const double w = ax[0].w[i] * ax[1].w[j];
                const double gw[2] = {ax[0].dw[i] * ax[1].w[j], ax[0].w[i] * ax[1].dw[j]};
                const double r[2] = {ax[0].r[i], ax[1].r[j]};
                fn(row + ax[0].base + i, w, gw, r);
            }
        }
    }
}

template <int DIM>
__device__ __forceinline__ void mat_mul(const double *A, const double *B, double *C) {
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) s += A[r * DIM + k] * B[k * DIM + c];
            C[r * DIM + c] = s;
        }
}

// det A and A^{-T}.
template <int DIM>
__device__ __forceinline__ double det_inv_t(const double *A, double *IT) {
    if constexpr (DIM == 2) {
        const double J = A[0] * A[3] - A[1] * A[2];
        const double q = 1.0 / J;
        IT[0] = A[3] * q;
        IT[1] = -A[2] * q;
        IT[2] = -A[1] * q;
        IT[3] = A[0] * q;
        return J;
    } else {
        const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
        const double c10 = A[2] * A[7] - A[1] * A[8], c11 = A[0] * A[8] - A[2] * A[6], c12 = A[1] * A[6] - A[0] * A[7];
        const double c20 = A[1] * A[5] - A[2] * A[4], c21 = A[2] * A[3] - A[0] * A[5], c22 = A[0] * A[4] - A[1] * A[3];
        const double J = A[0] * c00 + A[1] * c01 + A[2] * c02;
        const double q = 1.0 / J;
        // cofactor matrix / J = A^{-T}
        IT[0] = c00 * q; IT[1] = c01 * q; IT[2] = c02 * q;
        IT[3] = c10 * q; IT[4] = c11 * q; IT[5] = c12 * q;
        IT[6] = c20 * q; IT[7] = c21 * q; IT[8] = c22 * q;
        return J;
    }
}

// G = sum_i u_i grad w_ip^T (physical gradient = cell-unit gradient / dx).
template <int DIM, int DEG>
__device__ __forceinline__ void gather_grad(const Axis<double, DEG> (&ax)[DIM], const MidGrid &g, const double *gv,
                                            const double *dv, double cv, double cd, double *G) {
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) G[k] = 0.0;
    for_support<DIM, DEG>(ax, g, [&](int64_t i, double, const double *gw, const double *) {
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            const double u = cv * gv[r * g.nodes + i] + cd * dv[r * g.nodes + i];
#pragma unroll
            for (int c = 0; c < DIM; ++c) G[r * DIM + c] += u * gw[c];
        }
    });
    const double s = 1.0 / g.dx;
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) G[k] *= s;
}

template <int DIM>
__device__ __forceinline__ void load_mat(const double *plane, int64_t s, int64_t p, double *M) {
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) M[k] = plane[k * s + p];
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMidBlock) void k_mid_fill(double *a, int64_t n, double val) {
    const int64_t i = gtid();
    if (i < n) a[i] = val;
}

// --- particles sorted by base node (once per step) --------------------------
// Key = linear index of the particle's base node; particles whose support
// leaves the grid get no key (they take no part in the step).
template <int DIM, int DEG>
__global__ __launch_bounds__(kMidBlock) void k_mid_keys(Parts<double> P, MidGrid g, uint32_t *key, uint32_t *count,
                                                        uint32_t *flags) {
    const int64_t p = gtid();
    if (p >= P.n) return;
    Axis<double, DEG> ax[DIM];
    if (!particle_axes<DIM, DEG>(P, p, g, ax)) {
        key[p] = kNoKey;
        atomicOr(flags, (uint32_t)APIC_FLAG_OUT_OF_DOMAIN);
        return;
    }
    int64_t k = ax[DIM - 1].base;
#pragma unroll
    for (int a = DIM - 2; a >= 0; --a) k = k * g.N[a] + ax[a].base;
    key[p] = (uint32_t)k;
    atomicAdd(&count[k], 1u);
}

// Exclusive prefix sum of count[0, n) into start[0, n], start[n] = total:
// blocks of 1024 entries (scan1), the block totals in one block (scan2),
// then the block offsets added (scan3).
__global__ __launch_bounds__(kMidBlock) void k_mid_scan1(const uint32_t *count, int64_t n, uint32_t *start,
                                                         uint32_t *bsum) {
    __shared__ uint32_t sh[kMidBlock];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * 1024 + tid * 4;
    uint32_t v[4], tsum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = base + j < n ? count[base + j] : 0u;
        tsum += v[j];
    }
    sh[tid] = tsum;
    __syncthreads();
    for (int o = 1; o < kMidBlock; o <<= 1) {
        const uint32_t t = tid >= o ? sh[tid - o] : 0u;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    uint32_t run = sh[tid] - tsum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) start[base + j] = run;
        run += v[j];
    }
    if (tid == kMidBlock - 1) bsum[blockIdx.x] = sh[tid];
}

__global__ __launch_bounds__(kMidBlock) void k_mid_scan2(uint32_t *bsum, int64_t nb, uint32_t *start, int64_t n) {
    __shared__ uint32_t sh[kMidBlock];
    __shared__ uint32_t carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0u;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += kMidBlock) {
        const int64_t i = c0 + tid;
        const uint32_t v = i < nb ? bsum[i] : 0u;
        sh[tid] = v;
        __syncthreads();
        for (int o = 1; o < kMidBlock; o <<= 1) {
            const uint32_t t = tid >= o ? sh[tid - o] : 0u;
            __syncthreads();
            sh[tid] += t;
            __syncthreads();
        }
        const uint32_t excl = sh[tid] - v + carry;
        __syncthreads();
        if (i < nb) bsum[i] = excl;
        if (tid == kMidBlock - 1) carry += sh[tid];
        __syncthreads();
    }
    if (tid == 0) start[n] = carry;
}

__global__ __launch_bounds__(kMidBlock) void k_mid_scan3(uint32_t *start, int64_t n, const uint32_t *bsum) {
    const int64_t i = gtid();
    if (i < n) start[i] += bsum[i >> 10];
}

// perm[position] = particle, positions of one key in any order.
__global__ __launch_bounds__(kMidBlock) void k_mid_place(int64_t n, const uint32_t *key, const uint32_t *start,
                                                         uint32_t *cursor, uint32_t *perm) {
    const int64_t p = gtid();
    if (p >= n) return;
    const uint32_t k = key[p];
    if (k == kNoKey) return;
    perm[start[k] + atomicAdd(&cursor[k], 1u)] = (uint32_t)p;
}

// Sorted copies of what the solve reads (cell, offset, F, m) and the P2G
// terms: mv = m v and Q = m (k / dx) B, so that node i receives
// w (mv + Q r) with r = (x_i - x_p) / dx (B D^{-1} (x_i - x_p), D = dx^2 / k I).
template <int DIM, int DEG>
__global__ __launch_bounds__(kMidBlock) void k_mid_sort_state(Parts<double> P, MidSorted S) {
    const int64_t pos = gtid();
    if (pos >= S.n || pos >= (int64_t)S.start[S.nodes]) return;
    const int64_t q = S.perm[pos];
    S.cell[pos] = P.cell[q];
    const double m = P.m[q];
    S.m[pos] = m;
    const double kq = m * inv_D_factor<double, DEG>() / S.dx;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        S.off[a * S.n + pos] = P.off[a * P.s + q];
        S.mv[a * S.n + pos] = m * P.v[a * P.s + q];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        S.F[k * S.n + pos] = P.F[k * P.s + q];
        S.M[k * S.n + pos] = kq * P.B[k * P.s + q];
    }
}

template <int DIM, int DEG>
__device__ __forceinline__ void sorted_axes(const MidSorted &S, int64_t pos, Axis<double, DEG> (&ax)[DIM]) {
    int ci[3];
    unpack_cell<DIM>(S.cell[pos], ci);
#pragma unroll
    for (int a = 0; a < DIM; ++a) axis_weights<double, DEG>(ci[a], S.off[a * S.n + pos], ax[a]);
}

// v_i = (m v)_i / m_i on free nodes (mass, outside the sticky band); 0
// elsewhere.  mf_i = m_i on free nodes, 0 elsewhere.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_nodes(MidGrid g, const double *gm, double *gv, double *mf) {
    const int64_t i = gtid();
    if (i >= g.nodes) return;
    int c[3];
    node_coords<DIM>(i, g, c);
    bool sticky = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) sticky = sticky || c[a] < g.band[2 * a] || c[a] > g.N[a] - 1 - g.band[2 * a + 1];
    const double m = gm[i];
    const bool free_node = m > 0.0 && !sticky;
    mf[i] = free_node ? m : 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) gv[a * g.nodes + i] = free_node ? gv[a * g.nodes + i] / m : 0.0;
}

// Per sorted particle, the matrix that the node collect contracts with
// grad w (cell units): -V P(F_hat) F^T / dx for the force (DIFF = false;
// block partials of Phi = sum V Psi(F_hat)), -V (dP/dF(F_hat) : dF) F^T / dx
// for the force differential along du (DIFF = true), with
// F_hat = (I + sum_i u_i grad w^T) F, u_i = dt/2 v_i + dt/4 dv_i, and
// dF = (sum_i du_i grad w^T) F (Sec. 3.3, Sec. 4.1).
template <int DIM, int DEG, bool DIFF>
__global__ __launch_bounds__(kMidBlock) void k_mid_stress(MidSorted S, MidGrid g, MidMaterial mat, const double *gv,
                                                          const double *dv, double dt, const double *du, double *part,
                                                          uint32_t *flags) {
    const int64_t pos = gtid();
    double acc[1] = {0.0};
    if (pos < S.n && pos < (int64_t)S.start[S.nodes]) {
        Axis<double, DEG> ax[DIM];
        sorted_axes<DIM, DEG>(S, pos, ax);
        double F[DIM * DIM], G[DIM * DIM], Fh[DIM * DIM], IT[DIM * DIM], M[DIM * DIM];
#pragma unroll
        for (int k = 0; k < DIM * DIM; ++k) F[k] = S.F[k * S.n + pos];
        gather_grad<DIM, DEG>(ax, g, gv, dv, 0.5 * dt, 0.25 * dt, G);
#pragma unroll
        for (int a = 0; a < DIM; ++a) G[a * DIM + a] += 1.0;
        mat_mul<DIM>(G, F, Fh);
        const double J = det_inv_t<DIM>(Fh, IT);
        const double V = S.m[pos] / mat.rho0;
#pragma unroll
        for (int k = 0; k < DIM * DIM; ++k) M[k] = 0.0;
        if (!(J > 0.0)) {
            if (!DIFF) {
                atomicOr(flags, (uint32_t)APIC_FLAG_INVERTED);
                acc[0] = INFINITY;
            }
        } else {
            const double lnJ = log(J);
            double Pk[DIM * DIM];
            if constexpr (!DIFF) {
                double tr = 0.0;
#pragma unroll
                for (int k = 0; k < DIM * DIM; ++k) {
                    tr += Fh[k] * Fh[k];
                    Pk[k] = mat.mu * (Fh[k] - IT[k]) + mat.lambda * lnJ * IT[k];
                }
                acc[0] = V * (0.5 * mat.mu * (tr - DIM) - mat.mu * lnJ + 0.5 * mat.lambda * lnJ * lnJ);
            } else {
                double H[DIM * DIM], dF[DIM * DIM], dFt[DIM * DIM], T1[DIM * DIM], T2[DIM * DIM];
                gather_grad<DIM, DEG>(ax, g, du, du, 1.0, 0.0, H);
                mat_mul<DIM>(H, F, dF);
                // tr(F_hat^{-1} dF) = sum_ab IT_ab dF_ab;  T2 = F_hat^{-T} dF^T F_hat^{-T}
                double tr = 0.0;
#pragma unroll
                for (int k = 0; k < DIM * DIM; ++k) tr += IT[k] * dF[k];
#pragma unroll
                for (int r = 0; r < DIM; ++r)
#pragma unroll
                    for (int c = 0; c < DIM; ++c) dFt[r * DIM + c] = dF[c * DIM + r];
                mat_mul<DIM>(IT, dFt, T1);
                mat_mul<DIM>(T1, IT, T2);
                const double cT = mat.mu - mat.lambda * lnJ;
#pragma unroll
                for (int k = 0; k < DIM * DIM; ++k) Pk[k] = mat.mu * dF[k] + cT * T2[k] + mat.lambda * tr * IT[k];
            }
            // M = -V Pk F^T / dx
#pragma unroll
            for (int r = 0; r < DIM; ++r)
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    double sum = 0.0;
#pragma unroll
                    for (int k = 0; k < DIM; ++k) sum += Pk[r * DIM + k] * F[c * DIM + k];
                    M[r * DIM + c] = -V * sum / g.dx;
                }
        }
#pragma unroll
        for (int k = 0; k < DIM * DIM; ++k) S.M[k * S.n + pos] = M[k];
    }
    if constexpr (!DIFF) block_partials<1>(acc, part);
}

// Node collect, one block per tile of kRowTile nodes along x of one node row
// (fixed y, z).  The particles whose support holds a node of the row are
// those whose base key lies in rows y - DEG..y, z - DEG..z: DEG + 1 (2D) or
// (DEG + 1)^2 (3D) contiguous runs of the sorted order.  The block's lanes
// stride over each run (coalesced loads) and add each particle's terms for
// its DEG + 1 nodes of the row into LDS; the row tile is written once.
//   COLLECT_P2G:   gm_i = sum w m,  gv_i = sum w (mv + Q r)       (Sec. 3.2)
//   COLLECT_FORCE: f_i = sum M grad w                             (Sec. 3.3)
//   COLLECT_APPLY: df_i = sum M grad w, then s_i = p_i - dt^2/4 df_i / m_i on
//                  free nodes (0 elsewhere) and block partials of <p, s>_M
enum { COLLECT_P2G = 0, COLLECT_FORCE = 1, COLLECT_APPLY = 2 };
constexpr int kRowTile = 256;

template <int DIM>
__host__ __device__ __forceinline__ int64_t collect_blocks(const int *N) {
    const int64_t tiles = (N[0] + kRowTile - 1) / kRowTile;
    return DIM == 3 ? tiles * N[1] * N[2] : tiles * N[1];
}

template <int DIM, int DEG, int MODE>
__global__ __launch_bounds__(kMidBlock) void k_mid_collect(MidSorted S, MidGrid g, double *out_m, double *out_v,
                                                           const double *mf, const double *pv, double dt,
                                                           double *part) {
    constexpr int NC = MODE == COLLECT_P2G ? 1 + DIM : DIM;
    __shared__ double acc[kRowTile * NC];
    const int tid = threadIdx.x;
    const int ntile = (g.N[0] + kRowTile - 1) / kRowTile;
    const int64_t row = blockIdx.x / ntile;
    const int x0 = (int)(blockIdx.x % ntile) * kRowTile;
    const int x1 = (x0 + kRowTile < g.N[0] ? x0 + kRowTile : g.N[0]) - 1;
    const int cy = (int)(row % g.N[1]);
    const int cz = DIM == 3 ? (int)(row / g.N[1]) : 0;
    for (int k = tid; k < kRowTile * NC; k += kMidBlock) acc[k] = 0.0;
    __syncthreads();
    const int lo = x0 - DEG > 0 ? x0 - DEG : 0;
    const int hi = x1 < g.N[0] - 1 - DEG ? x1 : g.N[0] - 1 - DEG;
    constexpr int NZ = DIM == 3 ? DEG + 1 : 1;
#pragma unroll
    for (int dz = 0; dz < NZ; ++dz) {
        const int bz = cz - dz;
        if (DIM == 3 && (bz < 0 || bz + DEG > g.N[2] - 1)) continue;
#pragma unroll
        for (int dy = 0; dy <= DEG; ++dy) {
            const int by = cy - dy;
            if (by < 0 || by + DEG > g.N[1] - 1 || lo > hi) continue;
            const int64_t krow = (int64_t)g.N[0] * (by + (int64_t)g.N[1] * bz);
            const int64_t p1 = S.start[krow + hi + 1];
            for (int64_t pos = S.start[krow + lo] + tid; pos < p1; pos += kMidBlock) {
                Axis<double, DEG> ax[DIM];
                sorted_axes<DIM, DEG>(S, pos, ax);
                // the particle's weights along y (and z) at this row are fixed: index dy (dz)
                const double wy = ax[1].w[dy], dwy = ax[1].dw[dy], ry = ax[1].r[dy];
                const double wz = DIM == 3 ? ax[DIM - 1].w[dz] : 1.0;
                const double dwz = DIM == 3 ? ax[DIM - 1].dw[dz] : 0.0;
                const double rz = DIM == 3 ? ax[DIM - 1].r[dz] : 0.0;
                double Mq[DIM * DIM], mq = 0.0, mvq[DIM];
                if constexpr (MODE == COLLECT_P2G) {
                    mq = S.m[pos];
#pragma unroll
                    for (int a = 0; a < DIM; ++a) mvq[a] = S.mv[a * S.n + pos];
                }
#pragma unroll
                for (int k = 0; k < DIM * DIM; ++k) Mq[k] = S.M[k * S.n + pos];
#pragma unroll
                for (int kx = 0; kx <= DEG; ++kx) {
                    const int x = ax[0].base + kx;
                    if (x < x0 || x > x1) continue;
                    double* cell = acc + (x - x0) * NC;
                    const double w = ax[0].w[kx] * wy * wz;
                    if constexpr (MODE == COLLECT_P2G) {
                        double r[DIM];
                        r[0] = ax[0].r[kx];
                        r[1] = ry;
                        if constexpr (DIM == 3) r[2] = rz;
                        atomicAdd(&cell[0], w * mq);
#pragma unroll
                        for (int a = 0; a < DIM; ++a) {
                            double qr = 0.0;
#pragma unroll
                            for (int b = 0; b < DIM; ++b) qr += Mq[a * DIM + b] * r[b];
                            atomicAdd(&cell[1 + a], w * (mvq[a] + qr));
                        }
                    } else {
                        double gw[DIM];
                        gw[0] = ax[0].dw[kx] * wy * wz;
                        gw[1] = ax[0].w[kx] * dwy * wz;
                        if constexpr (DIM == 3) gw[2] = ax[0].w[kx] * wy * dwz;
#pragma unroll
                        for (int a = 0; a < DIM; ++a) {
                            double t = 0.0;
#pragma unroll
                            for (int b = 0; b < DIM; ++b) t += Mq[a * DIM + b] * gw[b];
                            atomicAdd(&cell[a], t);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    double part_acc[1] = {0.0};
    const int64_t rowbase = (int64_t)g.N[0] * row;
    for (int x = x0 + tid; x <= x1; x += kMidBlock) {
        const int64_t i = rowbase + x;
        const double *cell = acc + (x - x0) * NC;
        if constexpr (MODE == COLLECT_P2G) {
            out_m[i] = cell[0];
#pragma unroll
            for (int a = 0; a < DIM; ++a) out_v[a * g.nodes + i] = cell[1 + a];
        } else if constexpr (MODE == COLLECT_FORCE) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) out_v[a * g.nodes + i] = cell[a];
        } else {
            const double m = mf[i];
            const double cc = 0.25 * dt * dt;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const int64_t k = a * g.nodes + i;
                double sa = 0.0;
                if (m > 0.0) {
                    sa = pv[k] - cc * cell[a] / m;
                    part_acc[0] += m * pv[k] * sa;
                }
                out_v[k] = sa;
            }
        }
    }
    if constexpr (MODE == COLLECT_APPLY) block_partials<1>(part_acc, part);
}

// r_i = dv_i - dt (f_i / m_i + g) on free nodes (the gradient of E over
// m_i / 4); partials: sum m |r|^2 and sum m (|dv|^2 / 8 - dt/4 g.dv).
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_residual(MidGrid g, const double *mf, const double *f,
                                                            const double *dv, double dt, double3 grav, double *r,
                                                            double *part) {
    const int64_t i = gtid();
    double acc[2] = {0.0, 0.0};
    if (i < g.nodes) {
        const double m = mf[i];
        const double gr[3] = {grav.x, grav.y, grav.z};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + i;
            double ra = 0.0;
            if (m > 0.0) {
                ra = dv[k] - dt * (f[k] / m + gr[a]);
                acc[0] += m * ra * ra;
                acc[1] += m * (0.125 * dv[k] * dv[k] - 0.25 * dt * gr[a] * dv[k]);
            }
            r[k] = ra;
        }
    }
    block_partials<2>(acc, part);
}

// CG start: rc = b = -r, p = rc, delta = 0; partial <rc, rc>_M.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_cg_init(MidGrid g, const double *mf, const double *r,
                                                           double *delta, double *rc, double *pv, double *part) {
    const int64_t i = gtid();
    double acc[1] = {0.0};
    if (i < g.nodes) {
        const double m = mf[i];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + i;
            const double b = -r[k];
            rc[k] = b;
            pv[k] = b;
            delta[k] = 0.0;
            acc[0] += m * b * b;
        }
    }
    block_partials<1>(acc, part);
}

// delta += alpha p, rc -= alpha s; partial <rc, rc>_M.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_cg_step(MidGrid g, const double *mf, double alpha,
                                                           const double *pv, const double *s, double *delta,
                                                           double *rc, double *part) {
    const int64_t i = gtid();
    double acc[1] = {0.0};
    if (i < g.nodes) {
        const double m = mf[i];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + i;
            delta[k] += alpha * pv[k];
            const double ra = rc[k] - alpha * s[k];
            rc[k] = ra;
            acc[0] += m * ra * ra;
        }
    }
    block_partials<1>(acc, part);
}

// out = a + alpha b over n values.
__global__ __launch_bounds__(kMidBlock) void k_mid_axpy(int64_t n, const double *a, double alpha, const double *b,
                                                        double *out) {
    const int64_t i = gtid();
    if (i < n) out[i] = (a ? a[i] : 0.0) + alpha * b[i];
}

// vt_i = v_i + dv_i on free nodes (0 elsewhere); u_i = xt_i - x_i =
// dt (v_i + vt_i) / 2.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_finish(MidGrid g, const double *mf, const double *gv,
                                                          const double *dv, double dt, double *gvt, double *gu) {
    const int64_t i = gtid();
    if (i >= g.nodes) return;
    const bool free_node = mf[i] > 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int64_t k = a * g.nodes + i;
        const double vt = free_node ? gv[k] + dv[k] : 0.0;
        gvt[k] = vt;
        gu[k] = 0.5 * dt * (gv[k] + vt);
    }
}

// Transfer to particles with the general forms of Sec. 3.4, written with
// node displacements u_i = xt_i - x_i and U_p = x_p' - x_p = sum_i w u_i:
//   v_p' = sum_i w vt_i
//   B_p' = sum_i w vt_i r_i^T + 1/2 sum_i w (vt_i e_i^T - e_i vt_i^T),
//          r_i = x_i - x_p, e_i = u_i - U_p
//   F_p' = (I + sum_i u_i grad w^T) F_p,  x_p' = x_p + U_p.
template <int DIM, int DEG>
__global__ __launch_bounds__(kMidBlock) void k_mid_g2p(Parts<double> P, MidGrid g, const double *gvt,
                                                       const double *gu) {
    const int64_t p = gtid();
    if (p >= P.n) return;
    Axis<double, DEG> ax[DIM];
    if (!particle_axes<DIM, DEG>(P, p, g, ax)) return;
    double v[DIM] = {}, U[DIM] = {};
    for_support<DIM, DEG>(ax, g, [&](int64_t i, double w, const double *, const double *) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            v[a] += w * gvt[a * g.nodes + i];
            U[a] += w * gu[a * g.nodes + i];
        }
    });
    double B[DIM * DIM] = {}, G[DIM * DIM] = {};
    for_support<DIM, DEG>(ax, g, [&](int64_t i, double w, const double *gw, const double *r) {
        double vt[DIM], e[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            vt[a] = gvt[a * g.nodes + i];
            e[a] = gu[a * g.nodes + i] - U[a];
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = 0; b < DIM; ++b) {
                B[a * DIM + b] += w * (vt[a] * r[b] * g.dx + 0.5 * (vt[a] * e[b] - e[a] * vt[b]));
                G[a * DIM + b] += gu[a * g.nodes + i] * gw[b];
            }
    });
    double F[DIM * DIM], Fn[DIM * DIM];
    load_mat<DIM>(P.F, P.s, p, F);
    const double s = 1.0 / g.dx;
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) G[k] *= s;
#pragma unroll
    for (int a = 0; a < DIM; ++a) G[a * DIM + a] += 1.0;
    mat_mul<DIM>(G, F, Fn);
    int ci[3];
    unpack_cell<DIM>(P.cell[p], ci);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double o = P.off[a * P.s + p] + U[a] * s;
        const double c = floor(o);
        ci[a] += (int)c;
        P.off[a * P.s + p] = o - c;
        P.v[a * P.s + p] = v[a];
    }
    P.cell[p] = pack_cell<DIM>(ci);
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        P.B[k * P.s + p] = B[k];
        P.F[k * P.s + p] = Fn[k];
    }
}

// out[k] = sum over nblk blocks of part[b * K + k], in block order per thread
// stride, then a fixed tree (deterministic for a given nblk).
__global__ __launch_bounds__(kMidBlock) void k_mid_reduce(const double *part, int64_t nblk, int K, double *out) {
    __shared__ double red[kMidBlock];
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int64_t b = threadIdx.x; b < nblk; b += kMidBlock) s += part[b * K + k];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = kMidBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kMidBlock - 1) / kMidBlock); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_mid_fill(double *a, int64_t n, double val, hipStream_t st) {
    if (n > 0) k_mid_fill<<<blocks_for(n), kMidBlock, 0, st>>>(a, n, val);
}

void launch_mid_reduce(const double *part, int64_t nblk, int K, double *out, hipStream_t st) {
    k_mid_reduce<<<1, kMidBlock, 0, st>>>(part, nblk, K, out);
}

void launch_mid_axpy(int64_t n, const double *a, double alpha, const double *b, double *out, hipStream_t st) {
    if (n > 0) k_mid_axpy<<<blocks_for(n), kMidBlock, 0, st>>>(n, a, alpha, b, out);
}

// flags |= trial, trial = 0: the flag bits of the iterate the line search
// accepted join the call's flags (rejected trials leave none).
__global__ void k_mid_flags_accept(uint32_t *flags, uint32_t *trial) {
    if (threadIdx.x == 0) {
        flags[0] |= trial[0];
        trial[0] = 0u;
    }
}

void launch_mid_flags_accept(uint32_t *flags, uint32_t *trial, hipStream_t st) {
    k_mid_flags_accept<<<1, 64, 0, st>>>(flags, trial);
}

int64_t mid_particle_blocks(int64_t n) { return blocks_for(n); }
int64_t mid_node_blocks(int64_t nodes) { return blocks_for(nodes); }
int64_t mid_scan_blocks(int64_t nodes) { return (nodes + 1023) / 1024; }
int64_t mid_collect_blocks(int dim, const int *N) { return dim == 3 ? collect_blocks<3>(N) : collect_blocks<2>(N); }

template <int DIM, int DEG>
void launch_mid_sort(const Parts<double> &P, const MidGrid &g, const MidSorted &S, uint32_t *key, uint32_t *count,
                     uint32_t *cursor, uint32_t *bsum, uint32_t *flags, hipStream_t st) {
    launch_fill<uint32_t>(count, g.nodes, 0u, st);
    launch_fill<uint32_t>(cursor, g.nodes, 0u, st);
    if (P.n > 0) k_mid_keys<DIM, DEG><<<blocks_for(P.n), kMidBlock, 0, st>>>(P, g, key, count, flags);
    const int64_t nb = mid_scan_blocks(g.nodes);
    uint32_t *start = const_cast<uint32_t *>(S.start);
    k_mid_scan1<<<(unsigned)nb, kMidBlock, 0, st>>>(count, g.nodes, start, bsum);
    k_mid_scan2<<<1, kMidBlock, 0, st>>>(bsum, nb, start, g.nodes);
    k_mid_scan3<<<blocks_for(g.nodes), kMidBlock, 0, st>>>(start, g.nodes, bsum);
    if (P.n > 0) {
        k_mid_place<<<blocks_for(P.n), kMidBlock, 0, st>>>(P.n, key, S.start, cursor, const_cast<uint32_t *>(S.perm));
        k_mid_sort_state<DIM, DEG><<<blocks_for(P.n), kMidBlock, 0, st>>>(P, S);
    }
}

template <int DIM>
void launch_mid_nodes(const MidGrid &g, const double *gm, double *gv, double *mf, hipStream_t st) {
    k_mid_nodes<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, gm, gv, mf);
}

template <int DIM, int DEG, bool DIFF>
void launch_mid_stress(const MidSorted &S, const MidGrid &g, const MidMaterial &mat, const double *gv,
                       const double *dv, double dt, const double *du, double *part, uint32_t *flags, hipStream_t st) {
    if (S.n > 0) k_mid_stress<DIM, DEG, DIFF><<<blocks_for(S.n), kMidBlock, 0, st>>>(S, g, mat, gv, dv, dt, du, part,
                                                                                     flags);
}

template <int DIM, int DEG>
void launch_mid_collect_p2g(const MidSorted &S, const MidGrid &g, double *gm, double *gmv, hipStream_t st) {
    k_mid_collect<DIM, DEG, COLLECT_P2G><<<(unsigned)collect_blocks<DIM>(g.N), kMidBlock, 0, st>>>(S, g, gm, gmv, nullptr, nullptr,
                                                                                    0.0, nullptr);
}

template <int DIM, int DEG>
void launch_mid_collect_force(const MidSorted &S, const MidGrid &g, double *f, hipStream_t st) {
    k_mid_collect<DIM, DEG, COLLECT_FORCE><<<(unsigned)collect_blocks<DIM>(g.N), kMidBlock, 0, st>>>(S, g, nullptr, f, nullptr,
                                                                                      nullptr, 0.0, nullptr);
}

template <int DIM, int DEG>
void launch_mid_collect_apply(const MidSorted &S, const MidGrid &g, const double *mf, const double *pv, double dt,
                              double *s, double *part, hipStream_t st) {
    k_mid_collect<DIM, DEG, COLLECT_APPLY><<<(unsigned)collect_blocks<DIM>(g.N), kMidBlock, 0, st>>>(S, g, nullptr, s, mf, pv, dt,
                                                                                      part);
}

template <int DIM>
void launch_mid_residual(const MidGrid &g, const double *mf, const double *f, const double *dv, double dt,
                         const double *grav, double *r, double *part, hipStream_t st) {
    const double3 gr = make_double3(grav[0], grav[1], grav[2]);
    k_mid_residual<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, mf, f, dv, dt, gr, r, part);
}

template <int DIM>
void launch_mid_cg_init(const MidGrid &g, const double *mf, const double *r, double *delta, double *rc, double *pv,
                        double *part, hipStream_t st) {
    k_mid_cg_init<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, mf, r, delta, rc, pv, part);
}

template <int DIM>
void launch_mid_cg_step(const MidGrid &g, const double *mf, double alpha, const double *pv, const double *s,
                        double *delta, double *rc, double *part, hipStream_t st) {
    k_mid_cg_step<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, mf, alpha, pv, s, delta, rc, part);
}

template <int DIM>
void launch_mid_finish(const MidGrid &g, const double *mf, const double *gv, const double *dv, double dt, double *gvt,
                       double *gu, hipStream_t st) {
    k_mid_finish<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, mf, gv, dv, dt, gvt, gu);
}

template <int DIM, int DEG>
void launch_mid_g2p(const Parts<double> &P, const MidGrid &g, const double *gvt, const double *gu, hipStream_t st) {
    if (P.n > 0) k_mid_g2p<DIM, DEG><<<blocks_for(P.n), kMidBlock, 0, st>>>(P, g, gvt, gu);
}

#define APIC_MID_INST_DD(DIM, DEG)                                                                                   \
    template void launch_mid_sort<DIM, DEG>(const Parts<double> &, const MidGrid &, const MidSorted &, uint32_t *,   \
                                            uint32_t *, uint32_t *, uint32_t *, uint32_t *, hipStream_t);            \
    template void launch_mid_stress<DIM, DEG, false>(const MidSorted &, const MidGrid &, const MidMaterial &,         \
                                                     const double *, const double *, double, const double *,         \
                                                     double *, uint32_t *, hipStream_t);                             \
    template void launch_mid_stress<DIM, DEG, true>(const MidSorted &, const MidGrid &, const MidMaterial &,          \
                                                    const double *, const double *, double, const double *,          \
                                                    double *, uint32_t *, hipStream_t);                              \
    template void launch_mid_collect_p2g<DIM, DEG>(const MidSorted &, const MidGrid &, double *, double *,           \
                                                   hipStream_t);                                                     \
    template void launch_mid_collect_force<DIM, DEG>(const MidSorted &, const MidGrid &, double *, hipStream_t);     \
    template void launch_mid_collect_apply<DIM, DEG>(const MidSorted &, const MidGrid &, const double *,             \
                                                     const double *, double, double *, double *, hipStream_t);       \
    template void launch_mid_g2p<DIM, DEG>(const Parts<double> &, const MidGrid &, const double *, const double *,   \
                                           hipStream_t);
#define APIC_MID_INST_D(DIM)                                                                                          \
    template void launch_mid_nodes<DIM>(const MidGrid &, const double *, double *, double *, hipStream_t);           \
    template void launch_mid_residual<DIM>(const MidGrid &, const double *, const double *, const double *, double,  \
                                           const double *, double *, double *, hipStream_t);                         \
    template void launch_mid_cg_init<DIM>(const MidGrid &, const double *, const double *, double *, double *,       \
                                          double *, double *, hipStream_t);                                          \
    template void launch_mid_cg_step<DIM>(const MidGrid &, const double *, double, const double *, const double *,   \
                                          double *, double *, double *, hipStream_t);                                \
    template void launch_mid_finish<DIM>(const MidGrid &, const double *, const double *, const double *, double,    \
                                         double *, double *, hipStream_t);

APIC_MID_INST_DD(2, 2)
APIC_MID_INST_DD(2, 3)
APIC_MID_INST_DD(3, 2)
APIC_MID_INST_DD(3, 3)
APIC_MID_INST_D(2)
APIC_MID_INST_D(3)

}  // namespace apic
