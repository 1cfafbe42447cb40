// Implicit midpoint step (the lambda = 1/2 member of the grid update of
// Sec. 3.3), solved as the minimization of Sec. 4.1 with Newton's method and
// the mass-inner-product conjugate gradient of Sec. 4.2.  Binary64 throughout.
//
// Layout.  Nodes are grouped in tiles of 64 (4^3 in 3D, 8^2 in 2D); node
// vectors are component-major over the node slots (64 tile + place in tile).
// A particle's key is its base node.  Once per step the particles are
// counting-sorted by key, the key tiles that hold particles and the node tiles
// their regions touch are listed (a key tile's region is the tile plus DEG
// nodes up each axis: the support of every particle keyed in it), and what
// the solve reads is copied level-major per key tile.
//
// Particle terms.  One wavefront per listed key tile, one lane per key, walks
// the levels: it gathers node values of the region, staged in LDS, computes
// the particle's term and adds it into an LDS copy of the region.  Within one
// add every lane targets a different node (the lanes hold different base
// nodes and visit the support in the same order), so each node's sum has a
// fixed order.  The region sums go to the tile's slab.
//
// Node passes.  One wavefront per listed node tile, one lane per node, adds
// the (at most 2^dim) slabs that cover the node in a fixed order and finishes
// the node's update.  Reductions leave one partial per block; the kernel that
// needs the total has every block sum the partials in the same fixed order
// (one-block kernels where only the host or the next solve reads it), so the
// conjugate gradient's scalars are formed on the device and no iteration
// waits for the host.
//
// The transfer to particles writes the particles back to the caller's planes
// in the solve's order (ids move with them), those outside the grid last.
#include <hip/hip_ext.h>

#include "apic_kernels.h"

namespace apic {

namespace {

constexpr int kMidBlock = 256;  // node passes: four node tiles per block
constexpr int kNodeTilesPerBlock = kMidBlock / 64;

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * kMidBlock + threadIdx.x; }

template <int DIM>
__host__ __device__ constexpr int tile_edge() {
    return DIM == 3 ? 4 : 8;
}
template <int DIM, int DEG>
__host__ __device__ constexpr int region_edge() {
    return tile_edge<DIM>() + DEG;
}
template <int DIM, int DEG>
__host__ __device__ constexpr int region_nodes() {
    return DIM == 3 ? region_edge<DIM, DEG>() * region_edge<DIM, DEG>() * region_edge<DIM, DEG>()
                    : region_edge<DIM, DEG>() * region_edge<DIM, DEG>();
}

template <int DIM>
__device__ __forceinline__ int64_t tile_index(const MidGrid &g, const int *tc) {
    return DIM == 3 ? tc[0] + (int64_t)g.T[0] * (tc[1] + (int64_t)g.T[1] * tc[2]) : tc[0] + (int64_t)g.T[0] * tc[1];
}

// Slot of node (x, y, z).
template <int DIM>
__device__ __forceinline__ int64_t node_slot(const MidGrid &g, int x, int y, int z) {
    if constexpr (DIM == 3) {
        const int tc[3] = {x >> 2, y >> 2, z >> 2};
        return tile_index<3>(g, tc) * 64 + ((x & 3) | ((y & 3) << 2) | ((z & 3) << 4));
    } else {
        const int tc[3] = {x >> 3, y >> 3, 0};
        return tile_index<2>(g, tc) * 64 + ((x & 7) | ((y & 7) << 3));
    }
}

template <int DIM>
__device__ __forceinline__ void tile_coords(const MidGrid &g, int64_t t, int *tc) {
    tc[0] = (int)(t % g.T[0]);
    const int64_t q = t / g.T[0];
    if constexpr (DIM == 3) {
        tc[1] = (int)(q % g.T[1]);
        tc[2] = (int)(q / g.T[1]);
    } else {
        tc[1] = (int)q;
        tc[2] = 0;
    }
}

template <int DIM>
__device__ __forceinline__ void local_coords(int l, int *lc) {
    if constexpr (DIM == 3) {
        lc[0] = l & 3;
        lc[1] = (l >> 2) & 3;
        lc[2] = l >> 4;
    } else {
        lc[0] = l & 7;
        lc[1] = l >> 3;
        lc[2] = 0;
    }
}

// Sum over the block's threads of a[b * K + k] for b < n (each thread its
// stride of b in order, then a fixed tree); every thread returns the total.
__device__ __forceinline__ double block_total(const double *a, int64_t n, int K, int k) {
    __shared__ double red[kMidBlock];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < n; b += kMidBlock) s += a[b * K + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kMidBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// Block sums of K values to part[blockIdx * K + k] (thread 0 writes them).
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

template <int DIM, int DEG>
__device__ __forceinline__ void sorted_axes(const MidSorted &S, int64_t pos, Axis<double, DEG> (&ax)[DIM]) {
    int ci[3];
    unpack_cell<DIM>(S.cell[pos], ci);
#pragma unroll
    for (int a = 0; a < DIM; ++a) axis_weights<double, DEG>(ci[a], S.off[a * S.n + pos], ax[a]);
}

// Visits the support: f(w, grad w (cell units), r (cell units), i, j, k),
// (i, j, k) the offsets from the base node.  In 3D the z planes are a loop
// unless ZFULL (unrolling all of them lets the compiler hoist every load and
// keep every weight product live); the plane's z weights are rotated into
// element 0, so no register array is indexed dynamically.
template <int DIM, int DEG, bool ZFULL = false, typename Fn>
__device__ __forceinline__ void for_support(const Axis<double, DEG> (&ax)[DIM], Fn &&fn) {
    constexpr int K = DEG + 1;
    if constexpr (DIM == 3 && ZFULL) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double wyz = ax[1].w[j] * ax[DIM - 1].w[k];
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const double w = ax[0].w[i] * wyz;
                    const double gw[3] = {ax[0].dw[i] * wyz, ax[0].w[i] * ax[1].dw[j] * ax[DIM - 1].w[k],
                                          ax[0].w[i] * ax[1].w[j] * ax[DIM - 1].dw[k]};
                    const double r[3] = {ax[0].r[i], ax[1].r[j], ax[DIM - 1].r[k]};
                    fn(w, gw, r, i, j, k);
                }
            }
    } else if constexpr (DIM == 3) {
        double wz[K], dwz[K], rz[K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            wz[q] = ax[2].w[q];
            dwz[q] = ax[2].dw[q];
            rz[q] = ax[2].r[q];
        }
#pragma unroll 1
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double wyz = ax[1].w[j] * wz[0];
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const double w = ax[0].w[i] * wyz;
                    const double gw[3] = {ax[0].dw[i] * wyz, ax[0].w[i] * ax[1].dw[j] * wz[0],
                                          ax[0].w[i] * ax[1].w[j] * dwz[0]};
                    const double r[3] = {ax[0].r[i], ax[1].r[j], rz[0]};
                    fn(w, gw, r, i, j, k);
                }
            }
#pragma unroll
            for (int q = 0; q + 1 < K; ++q) {
                wz[q] = wz[q + 1];
                dwz[q] = dwz[q + 1];
                rz[q] = rz[q + 1];
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const double w = ax[0].w[i] * ax[1].w[j];
                const double gw[2] = {ax[0].dw[i] * ax[1].w[j], ax[0].w[i] * ax[1].dw[j]};
                const double r[2] = {ax[0].r[i], ax[1].r[j]};
                fn(w, gw, r, i, j, 0);
            }
    }
}

// Visits the support row by row (a row: the DEG + 1 nodes along x at the
// y, z offsets j, k): f(j, k, c0, c1, c2, ry, rz) with c0 = w_j w_k,
// c1 = dw_j w_k, c2 = w_j dw_k (y, z factors of w and of the gradient's
// components; in 2D c0 = w_j, c1 = dw_j, c2 = 0) and ry, rz the row's
// offsets from the particle (cell units).  3D planes as in for_support.
template <int DIM, int DEG, typename Fn>
__device__ __forceinline__ void for_rows(const Axis<double, DEG> (&ax)[DIM], Fn &&fn) {
    constexpr int K = DEG + 1;
    if constexpr (DIM == 3) {
        double wz[K], dwz[K], rz[K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            wz[q] = ax[DIM - 1].w[q];
            dwz[q] = ax[DIM - 1].dw[q];
            rz[q] = ax[DIM - 1].r[q];
        }
#pragma unroll 1
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int j = 0; j < K; ++j)
                fn(j, k, ax[1].w[j] * wz[0], ax[1].dw[j] * wz[0], ax[1].w[j] * dwz[0], ax[1].r[j], rz[0]);
#pragma unroll
            for (int q = 0; q + 1 < K; ++q) {
                wz[q] = wz[q + 1];
                dwz[q] = dwz[q + 1];
                rz[q] = rz[q + 1];
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) fn(j, 0, ax[1].w[j], ax[1].dw[j], 0.0, ax[1].r[j], 0.0);
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

// Key (place in the tile) that a lane walks.  Lanes are processed in groups
// of 16 by LDS; the maps put, in each group, keys whose region addresses
// (x + RE y + RE^2 z, in doubles) differ modulo 16, so that a group's LDS
// accesses at one support offset fall in different bank pairs: 3D quadratic,
// a group is one y layer; 3D cubic, the keys with y ^ z = group; 2D
// quadratic, the rows y = group, group + 4 (x = key mod 4 / 8 in 3D / 2D).
template <int DIM, int DEG>
__device__ __forceinline__ int lane_key(int lane) {
    if constexpr (DIM == 3) {
        const int x = lane & 3, z = (lane >> 2) & 3, g = lane >> 4;
        const int y = DEG == 3 ? g ^ z : g;
        return x | (y << 2) | (z << 4);
    } else if constexpr (DEG == 2) {
        const int x = lane & 7, y = (lane >> 4) | (((lane >> 3) & 1) << 2);
        return x | (y << 3);
    } else {
        return lane;
    }
}

// Walks the particles of key tile t level by level, in the lane of each
// particle's key: fn(sorted position, level, first key-major position of the
// key).  Positions of one level are consecutive, in lane order.
template <int DIM, int DEG, typename Fn>
__device__ __forceinline__ void for_levels(const uint32_t *start, int64_t t, Fn &&fn) {
    const int lane = threadIdx.x & 63;
    const int64_t key = t * 64 + lane_key<DIM, DEG>(lane);
    const uint32_t k0 = start[key];
    const uint32_t cnt = start[key + 1] - k0;
    uint32_t maxc = cnt;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t other = __shfl_xor(maxc, o, 64);
        maxc = other > maxc ? other : maxc;
    }
    int64_t pos0 = start[t * 64];
    const uint64_t below = (1ull << lane) - 1ull;
    for (uint32_t r = 0; r < maxc; ++r) {
        const bool act = r < cnt;
        const uint64_t bal = ballot(act);
        if (act) fn(pos0 + __popcll(bal & below), r, k0);
        pos0 += __popcll(bal);
    }
}

// ---------------------------------------------------------------------------
// Sort (once per step)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMidBlock) void k_mid_fill_u32(uint32_t *a, int64_t n) {
    const int64_t i = gtid();
    if (i < n) a[i] = 0u;
}

// Key = slot of the particle's base node; particles whose support leaves the
// grid take no part in the step and get the key `nodes`, after every node.
template <int DIM, int DEG>
__global__ __launch_bounds__(kMidBlock) void k_mid_keys(Parts<double> P, MidGrid g, uint32_t *key, uint32_t *count,
                                                        uint32_t *flags) {
    const int64_t p = gtid();
    if (p >= P.n) return;
    Axis<double, DEG> ax[DIM];
    if (!particle_axes<DIM, DEG>(P, p, g, ax)) {
        key[p] = (uint32_t)g.nodes;  // the bucket after every node: particles that take no part
        atomicAdd(&count[g.nodes], 1u);
        atomicOr(flags, (uint32_t)APIC_FLAG_OUT_OF_DOMAIN);
        return;
    }
    const int64_t k = node_slot<DIM>(g, ax[0].base, ax[1].base, DIM == 3 ? ax[DIM - 1].base : 0);
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

// perm[position] = particle; the positions of one key in any order (the
// level-major copy orders them).
__global__ __launch_bounds__(kMidBlock) void k_mid_place(int64_t n, const uint32_t *key, const uint32_t *start,
                                                         uint32_t *cursor, uint32_t *perm) {
    const int64_t p = gtid();
    if (p >= n) return;
    const uint32_t k = key[p];
    perm[start[k] + atomicAdd(&cursor[k], 1u)] = (uint32_t)p;
}

// Tile lists: klist = tiles holding particles, nlist = tiles t with a tile
// holding particles among t - d, d in {0, 1}^dim (the regions reach one tile
// up each axis), both ascending; slot[t] = index in klist or -1.  Flags per
// tile, their prefix sums (the scan kernels above), then the placement.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_tile_flags(MidGrid g, const uint32_t *start, uint32_t *kf,
                                                              uint32_t *nf, uint32_t *hf) {
    const int64_t t = gtid();
    if (t >= g.tiles) return;
    int tc[3];
    tile_coords<DIM>(g, t, tc);
    bool nact = false;
#pragma unroll
    for (int d = 0; d < (1 << DIM); ++d) {
        const int u[3] = {tc[0] - (d & 1), tc[1] - ((d >> 1) & 1), DIM == 3 ? tc[2] - (d >> 2) : 0};
        if (u[0] < 0 || u[1] < 0 || u[2] < 0) continue;
        const int64_t ut = tile_index<DIM>(g, u);
        nact = nact || start[ut * 64 + 64] > start[ut * 64];
    }
    const uint32_t np = start[t * 64 + 64] - start[t * 64];
    kf[t] = np > 0u ? 1u : 0u;
    hf[t] = np >= kFullTile ? 1u : 0u;
    nf[t] = nact ? 1u : 0u;
}

// Key tiles of at least kFullTile particles take the first places of the
// list (in tile order), the others follow (in tile order), so that the tile
// passes, one block per listed key tile in list order, end with the short
// tiles.
__global__ __launch_bounds__(kMidBlock) void k_mid_tile_place(int64_t tiles, const uint32_t *kf, const uint32_t *nf,
                                                              const uint32_t *hf, const uint32_t *ks,
                                                              const uint32_t *ns, const uint32_t *hs, MidTiles tl,
                                                              int32_t *counts) {
    const int64_t t = gtid();
    if (t == 0) {
        counts[0] = (int32_t)ks[tiles];
        counts[1] = (int32_t)ns[tiles];
    }
    if (t >= tiles) return;
    const uint32_t pos = hf[t] ? hs[t] : hs[tiles] + (ks[t] - hs[t]);
    tl.slot[t] = kf[t] ? (int32_t)pos : -1;
    if (kf[t]) tl.klist[pos] = (int32_t)t;
    if (nf[t]) tl.nlist[ns[t]] = (int32_t)t;
}

// Level-major copies of what the solve reads (cell, offset, F, m) and the
// transfer-to-grid terms mv = m v and Q = m (k / dx) B, so that node i
// receives w (mv + Q r) with r = (x_i - x_p) / dx (the B D^{-1} (x_i - x_p)
// term of Sec. 3.2 with D = dx^2 / k I).  A key's particles are first put in
// ascending index order, so the copy and every sum after it are the same on
// every run.
// A lane's walk over the levels of its key in a key tile: position of level
// r (consecutive positions per level, in lane order) and the level count.
struct LevelWalk {
    int64_t pos0;
    uint32_t maxc;
    uint64_t below;
};

__device__ __forceinline__ LevelWalk level_walk(const uint32_t *start, int64_t t, uint32_t cnt) {
    const int lane = threadIdx.x & 63;
    LevelWalk w;
    w.maxc = cnt;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t other = __shfl_xor(w.maxc, o, 64);
        w.maxc = other > w.maxc ? other : w.maxc;
    }
    w.pos0 = start[t * 64];
    w.below = (1ull << lane) - 1ull;
    return w;
}

// What the sort copy moves of one particle.
template <int DIM>
struct SortRow {
    uint32_t cell, id;
    double m, off[DIM], v[DIM], F[DIM * DIM], B[DIM * DIM];
};

template <int DIM>
__device__ __forceinline__ void sort_row_load(const Parts<double> &P, int64_t q, bool with_id, SortRow<DIM> &w) {
    w.cell = P.cell[q];
    w.id = with_id ? P.id[q] : 0u;
    w.m = P.m[q];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        w.off[a] = P.off[a * P.s + q];
        w.v[a] = P.v[a * P.s + q];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        w.F[k] = P.F[k * P.s + q];
        w.B[k] = P.B[k * P.s + q];
    }
}

// Level-major copies of what the solve reads (cell, offset, F, m) and the
// transfer-to-grid terms mv = m v and Q = m (k / dx) B, so that node i
// receives w (mv + Q r) with r = (x_i - x_p) / dx (the B D^{-1} (x_i - x_p)
// term of Sec. 3.2 with D = dx^2 / k I).  A key's particles are first put in
// ascending index order, so the copy and every sum after it are the same on
// every run: up to kSortLds of them in the lane's own LDS column (all loads
// in flight together, insertion sort in LDS), more with a Shell sort of the
// segment in place.  The copy loads level r + 1 before it stores level r.
constexpr uint32_t kSortLds = 32;

template <int DIM, int DEG>
__global__ __launch_bounds__(64) void k_mid_sort_state(Parts<double> P, MidSorted S, MidTiles tl) {
    __shared__ uint32_t col[kSortLds * 64];
    const int lane = threadIdx.x;
    const int64_t t = tl.klist[blockIdx.x];
    const int64_t key = t * 64 + lane_key<DIM, DEG>(lane);
    const uint32_t k0 = S.start[key], cnt = S.start[key + 1] - k0;
    uint32_t *seg = S.perm + k0;
    const bool in_lds = cnt <= kSortLds;
    if (in_lds) {
#pragma unroll 8
        for (uint32_t i = 0; i < cnt; ++i) col[i * 64 + lane] = seg[i];
        for (uint32_t i = 1; i < cnt; ++i) {
            const uint32_t v = col[i * 64 + lane];
            uint32_t j = i;
            while (j > 0 && col[(j - 1) * 64 + lane] > v) {
                col[j * 64 + lane] = col[(j - 1) * 64 + lane];
                --j;
            }
            col[j * 64 + lane] = v;
        }
    } else {
        // Shell sort (gaps 701, 301, 132, 57, 23, 10, 4, 1, then 2.25x
        // above): about cnt^1.3 steps, not cnt^2
        uint32_t gap = 1;
        while (gap < cnt / 3) gap = gap < 701 ? (gap < 4 ? 4 : gap < 10 ? 10 : gap < 23 ? 23 : gap < 57 ? 57 :
                                                 gap < 132 ? 132 : gap < 301 ? 301 : 701)
                                              : gap * 9 / 4;
        for (;; gap = gap > 701 ? max(gap * 4 / 9, 701u) : (gap == 701 ? 301 : gap == 301 ? 132 : gap == 132 ? 57 :
                                                    gap == 57 ? 23 : gap == 23 ? 10 : gap == 10 ? 4 : 1)) {
            for (uint32_t i = gap; i < cnt; ++i) {
                const uint32_t v = seg[i];
                uint32_t j = i;
                while (j >= gap && seg[j - gap] > v) {
                    seg[j] = seg[j - gap];
                    j -= gap;
                }
                seg[j] = v;
            }
            if (gap == 1) break;
        }
    }
    auto index_of = [&](uint32_t r) -> int64_t { return in_lds ? col[r * 64 + lane] : seg[r]; };
    const double kD = inv_D_factor<double, DEG>() / S.dx;
    const bool with_id = S.id != nullptr;
    LevelWalk lw = level_walk(S.start, t, cnt);
    SortRow<DIM> cur, nxt;
    if (cnt > 0) sort_row_load<DIM>(P, index_of(0), with_id, cur);
    for (uint32_t r = 0; r < lw.maxc; ++r) {
        const bool act = r < cnt;
        const uint64_t bal = ballot(act);
        if (r + 1 < cnt) sort_row_load<DIM>(P, index_of(r + 1), with_id, nxt);
        if (act) {
            const int64_t pos = lw.pos0 + __popcll(bal & lw.below);
            S.cell[pos] = cur.cell;
            if (with_id) S.id[pos] = cur.id;
            S.m[pos] = cur.m;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                S.off[a * S.n + pos] = cur.off[a];
                S.mv[a * S.n + pos] = cur.m * cur.v[a];
            }
#pragma unroll
            for (int k = 0; k < DIM * DIM; ++k) {
                S.F[k * S.n + pos] = cur.F[k];
                S.M[k * S.n + pos] = cur.m * kD * cur.B[k];
            }
        }
        lw.pos0 += __popcll(bal);
        cur = nxt;
    }
}

// Full copies of the particles that take no part (positions after every
// keyed one): v into the m v planes, B into the first d^2 M planes, for the
// transfer to particles to put back after the others.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_sort_dead(Parts<double> P, MidSorted S, int64_t nodes) {
    const int64_t pos = (int64_t)S.start[nodes] + gtid();
    if (pos >= (int64_t)S.start[nodes + 1]) return;
    const int64_t q = S.perm[pos];
    S.cell[pos] = P.cell[q];
    S.m[pos] = P.m[q];
    if (S.id) S.id[pos] = P.id ? P.id[q] : (uint32_t)q;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        S.off[a * S.n + pos] = P.off[a * P.s + q];
        S.mv[a * S.n + pos] = P.v[a * P.s + q];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        S.F[k * S.n + pos] = P.F[k * P.s + q];
        S.M[k * S.n + pos] = P.B[k * P.s + q];
    }
}

// ---------------------------------------------------------------------------
// Particle terms, one wavefront per listed key tile
// ---------------------------------------------------------------------------
//   TILE_P2G:   node i receives w m and w (mv + Q r)                     (Sec. 3.2)
//   TILE_FORCE: F_hat = (I + sum_i u_i grad w^T) F with u_i = dt/2 v_i + dt/4 dv_i
//               (staged), the energy V Psi(F_hat) and node i receives
//               -V P(F_hat) F^T grad w / dx; F_hat is kept for TILE_APPLY (Sec. 3.3, 4.1)
//   TILE_APPLY: dF = (sum_i p_i grad w^T) F (p staged) and node i receives
//               -V (dP/dF(F_hat) : dF) F^T grad w / dx                       (Sec. 4.2)
enum { TILE_P2G = 0, TILE_FORCE = 1, TILE_APPLY = 2 };

// Waves per SIMD the register allocation of a tile kernel aims at (1: no
// target).
template <int DIM, int DEG, int MODE>
constexpr int tile_waves() {
    return MODE == TILE_APPLY && DIM == 3 && DEG == 2 ? 3 : 1;
}

template <int DIM, int DEG, int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(tile_waves<DIM, DEG, MODE>()))) void k_mid_tile(
    MidSorted S, MidGrid g, MidTiles tl, MidMaterial mat, const double *va, const double *vb, double ca, double cb,
    double *epart, uint32_t *flags, const MidCg *cg) {
    constexpr int R = region_nodes<DIM, DEG>(), RE = region_edge<DIM, DEG>(), E = tile_edge<DIM>();
    constexpr int CIN = MODE == TILE_P2G ? 0 : DIM;
    constexpr int COUT = MODE == TILE_P2G ? 1 + DIM : DIM;
    constexpr int D2 = DIM * DIM;
    __shared__ double acc[COUT * R];
    __shared__ double stage[(CIN > 0 ? CIN : 1) * R];
    if constexpr (MODE == TILE_APPLY) {
        if (cg->done) return;
    }
    const int lane = threadIdx.x;
    const int64_t t = tl.klist[blockIdx.x];
    int tc[3];
    tile_coords<DIM>(g, t, tc);
    const int org[3] = {tc[0] * E, tc[1] * E, tc[2] * E};
    for (int k = lane; k < COUT * R; k += 64) acc[k] = 0.0;
    if constexpr (CIN > 0) {
        for (int k = lane; k < R; k += 64) {
            const int rx = k % RE, ry = DIM == 3 ? (k / RE) % RE : k / RE, rz = DIM == 3 ? k / (RE * RE) : 0;
            const int x = org[0] + rx, y = org[1] + ry, z = org[2] + rz;
            const bool in = x < g.N[0] && y < g.N[1] && (DIM == 2 || z < g.N[2]);
            const int64_t i = in ? node_slot<DIM>(g, x, y, z) : 0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                double u = 0.0;
                if (in) {
                    u = ca * va[a * g.nodes + i];
                    if (vb) u += cb * vb[a * g.nodes + i];
                }
                stage[a * R + k] = u;
            }
        }
    }
    __syncthreads();
    double energy = 0.0;
    const double inv_dx = 1.0 / g.dx, inv_rho0 = 1.0 / mat.rho0;
    for_levels<DIM, DEG>(S.start, t, [&](int64_t pos, uint32_t, uint32_t) {
        Axis<double, DEG> ax[DIM];
        sorted_axes<DIM, DEG>(S, pos, ax);
        const int rb[3] = {ax[0].base - org[0], ax[1].base - org[1], DIM == 3 ? ax[DIM - 1].base - org[2] : 0};
        // region index of the first node of support row (j, k)
        auto row_start = [&](int j, int k) {
            return DIM == 3 ? rb[0] + RE * ((rb[1] + j) + RE * (rb[2] + k)) : rb[0] + RE * (rb[1] + j);
        };
        if constexpr (MODE == TILE_P2G) {
            // node i receives w m and w (mv + Q r): per row, mv + Q r without the x term
            double Q[D2], mvq[DIM];
            const double mq = S.m[pos];
#pragma unroll
            for (int a = 0; a < DIM; ++a) mvq[a] = S.mv[a * S.n + pos];
#pragma unroll
            for (int k = 0; k < D2; ++k) Q[k] = S.M[k * S.n + pos];
            for_rows<DIM, DEG>(ax, [&](int j, int k, double wr, double, double, double ry, double rz) {
                const int r0 = row_start(j, k);
                double base[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    base[a] = mvq[a] + Q[a * DIM + 1] * ry;
                    if constexpr (DIM == 3) base[a] += Q[a * DIM + 2] * rz;
                }
#pragma unroll
                for (int i = 0; i <= DEG; ++i) {
                    const double w = ax[0].w[i] * wr;
                    atomicAdd(&acc[r0 + i], w * mq);
#pragma unroll
                    for (int a = 0; a < DIM; ++a)
                        atomicAdd(&acc[(1 + a) * R + r0 + i], w * (base[a] + Q[a * DIM] * ax[0].r[i]));
                }
            });
        } else {
            double F[D2], G[D2], IT[D2], Pk[D2];
#pragma unroll
            for (int k = 0; k < D2; ++k) {
                F[k] = S.F[k * S.n + pos];
                G[k] = 0.0;
            }
            // G = sum_i u_i grad w^T over the staged node values (cell units),
            // per row: the x sums of w u and dw u, then the row's y, z factors
            for_rows<DIM, DEG>(ax, [&](int j, int k, double c0, double c1, double c2, double, double) {
                const int r0 = row_start(j, k);
                double sw[DIM], sdw[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    sw[a] = 0.0;
                    sdw[a] = 0.0;
                }
#pragma unroll
                for (int i = 0; i <= DEG; ++i)
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        const double u = stage[a * R + r0 + i];
                        sw[a] += ax[0].w[i] * u;
                        sdw[a] += ax[0].dw[i] * u;
                    }
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    G[a * DIM] += sdw[a] * c0;
                    G[a * DIM + 1] += sw[a] * c1;
                    if constexpr (DIM == 3) G[a * DIM + 2] += sw[a] * c2;
                }
            });
#pragma unroll
            for (int k = 0; k < D2; ++k) G[k] *= inv_dx;
            const double V = S.m[pos] * inv_rho0;
            bool ok;
            if constexpr (MODE == TILE_FORCE) {
                double Fh[D2];
#pragma unroll
                for (int a = 0; a < DIM; ++a) G[a * DIM + a] += 1.0;
                mat_mul<DIM>(G, F, Fh);
                const double J = det_inv_t<DIM>(Fh, IT);
                ok = J > 0.0;
                if (!ok) {
                    atomicOr(flags, (uint32_t)APIC_FLAG_INVERTED);
                    energy = INFINITY;
                } else {
                    const double lnJ = log(J);
                    double tr = 0.0;
#pragma unroll
                    for (int k = 0; k < D2; ++k) {
                        tr += Fh[k] * Fh[k];
                        Pk[k] = mat.mu * (Fh[k] - IT[k]) + mat.lambda * lnJ * IT[k];
                    }
                    energy += V * (0.5 * mat.mu * (tr - DIM) - mat.mu * lnJ + 0.5 * mat.lambda * lnJ * lnJ);
                    // kept for the differential: F_hat^{-T} and mu - lambda ln J
#pragma unroll
                    for (int k = 0; k < D2; ++k) S.M[k * S.n + pos] = IT[k];
                    S.M[D2 * S.n + pos] = mat.mu - mat.lambda * lnJ;
                }
            } else {
                // dP = mu dF + (mu - lambda ln J) F_hat^{-T} dF^T F_hat^{-T} + lambda tr(F_hat^{-1} dF) F_hat^{-T}
                // (an inverted F_hat was rejected by the line search: its element is not kept)
#pragma unroll
                for (int k = 0; k < D2; ++k) IT[k] = S.M[k * S.n + pos];
                const double cT = S.M[D2 * S.n + pos];
                ok = true;
                double dF[D2], dFt[D2], T1[D2], T2[D2];
                mat_mul<DIM>(G, F, dF);
                double tr = 0.0;
#pragma unroll
                for (int k = 0; k < D2; ++k) tr += IT[k] * dF[k];
#pragma unroll
                for (int r = 0; r < DIM; ++r)
#pragma unroll
                    for (int c = 0; c < DIM; ++c) dFt[r * DIM + c] = dF[c * DIM + r];
                mat_mul<DIM>(IT, dFt, T1);
                mat_mul<DIM>(T1, IT, T2);
#pragma unroll
                for (int k = 0; k < D2; ++k) Pk[k] = mat.mu * dF[k] + cT * T2[k] + mat.lambda * tr * IT[k];
            }
            if (ok) {
                // M = -V Pk F^T / dx; node i receives M grad w = dw_x (M e_x) c0 + w_x (M_y c1 + M_z c2)
                double M[D2];
                const double cm = -V * inv_dx;
#pragma unroll
                for (int r = 0; r < DIM; ++r)
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        double sum = 0.0;
#pragma unroll
                        for (int k = 0; k < DIM; ++k) sum += Pk[r * DIM + k] * F[c * DIM + k];
                        M[r * DIM + c] = cm * sum;
                    }
                for_rows<DIM, DEG>(ax, [&](int j, int k, double c0, double c1, double c2, double, double) {
                    const int r0 = row_start(j, k);
                    double A[DIM], Bv[DIM];
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        A[a] = M[a * DIM] * c0;
                        Bv[a] = M[a * DIM + 1] * c1;
                        if constexpr (DIM == 3) Bv[a] += M[a * DIM + 2] * c2;
                    }
#pragma unroll
                    for (int i = 0; i <= DEG; ++i)
#pragma unroll
                        for (int a = 0; a < DIM; ++a)
                            atomicAdd(&acc[a * R + r0 + i], ax[0].dw[i] * A[a] + ax[0].w[i] * Bv[a]);
                });
            }
        }
    });
    __syncthreads();
    double *sl = tl.slab + (int64_t)blockIdx.x * COUT * R;
    for (int k = lane; k < COUT * R; k += 64) sl[k] = acc[k];
    if constexpr (MODE == TILE_FORCE) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) energy += __shfl_xor(energy, o, 64);
        if (lane == 0) epart[blockIdx.x] = energy;
    }
}

// ---------------------------------------------------------------------------
// Node passes, one wavefront per listed node tile
// ---------------------------------------------------------------------------
struct NodeAt {
    int64_t i;         // slot
    int c[3], tc[3], lc[3];  // node, tile and in-tile coordinates
};

template <int DIM>
__device__ __forceinline__ bool node_at(const MidGrid &g, const MidTiles &tl, NodeAt &n) {
    constexpr int E = tile_edge<DIM>();
    const int64_t li = (int64_t)blockIdx.x * kNodeTilesPerBlock + (threadIdx.x >> 6);
    if (li >= tl.nn) return false;
    const int64_t u = tl.nlist[li];
    tile_coords<DIM>(g, u, n.tc);
    local_coords<DIM>(threadIdx.x & 63, n.lc);
#pragma unroll
    for (int a = 0; a < 3; ++a) n.c[a] = n.tc[a] * E + n.lc[a];
    n.i = u * 64 + (threadIdx.x & 63);
    return true;
}

// Sum of the COUT region sums that cover the node, over the key tiles
// tc - d, d in {0, 1}^dim, in that order.
template <int DIM, int DEG, int COUT>
__device__ __forceinline__ void slab_sum(const MidGrid &g, const MidTiles &tl, const NodeAt &n, double *out) {
    constexpr int R = region_nodes<DIM, DEG>(), RE = region_edge<DIM, DEG>(), E = tile_edge<DIM>();
#pragma unroll
    for (int c = 0; c < COUT; ++c) out[c] = 0.0;
#pragma unroll
    for (int d = 0; d < (1 << DIM); ++d) {
        const int dd[3] = {d & 1, (d >> 1) & 1, DIM == 3 ? d >> 2 : 0};
        int T[3], rc[3];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T[a] = n.tc[a] - dd[a];
            rc[a] = n.lc[a] + E * dd[a];
            ok = ok && T[a] >= 0 && (a >= DIM || rc[a] < RE);
        }
        if (!ok) continue;
        const int32_t s = tl.slot[tile_index<DIM>(g, T)];
        if (s < 0) continue;
        const int ri = DIM == 3 ? rc[0] + RE * (rc[1] + RE * rc[2]) : rc[0] + RE * rc[1];
        const double *sl = tl.slab + (int64_t)s * COUT * R + ri;
#pragma unroll
        for (int c = 0; c < COUT; ++c) out[c] += sl[c * R];
    }
}

// mf_i = m_i and v_i = (m v)_i / m_i on free nodes (mass, outside the sticky
// band); 0 elsewhere.
template <int DIM, int DEG>
__global__ __launch_bounds__(kMidBlock) void k_mid_node_p2g(MidGrid g, MidTiles tl, double *mf, double *gv) {
    NodeAt n;
    if (!node_at<DIM>(g, tl, n)) return;
    double sum[1 + DIM];
    slab_sum<DIM, DEG, 1 + DIM>(g, tl, n, sum);
    bool sticky = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        sticky = sticky || n.c[a] < g.band[2 * a] || n.c[a] > g.N[a] - 1 - g.band[2 * a + 1];
    const double m = sum[0];
    const bool free_node = m > 0.0 && !sticky;
    mf[n.i] = free_node ? m : 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) gv[a * g.nodes + n.i] = free_node ? sum[1 + a] / m : 0.0;
}

// r_i = dv_i - dt (f_i / m_i + g) on free nodes (the gradient of E over
// m_i / 4, Sec. 4.1); block partials of sum m |r|^2 and sum m (|dv|^2 / 8 -
// dt/4 g.dv).
template <int DIM, int DEG, bool ELASTIC>
__global__ __launch_bounds__(kMidBlock) void k_mid_node_force(MidGrid g, MidTiles tl, const double *mf,
                                                              const double *dv, double dt, double3 grav, double *r,
                                                              double *part) {
    double acc[2] = {0.0, 0.0};
    NodeAt n;
    if (node_at<DIM>(g, tl, n)) {
        double f[DIM];
        if constexpr (ELASTIC)
            slab_sum<DIM, DEG, DIM>(g, tl, n, f);
        else
#pragma unroll
            for (int a = 0; a < DIM; ++a) f[a] = 0.0;
        const double m = mf[n.i];
        const double gr[3] = {grav.x, grav.y, grav.z};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + n.i;
            double ra = 0.0;
            if (m > 0.0) {
                ra = dv[k] - dt * (f[a] / m + gr[a]);
                acc[0] += m * ra * ra;
                acc[1] += m * (0.125 * dv[k] * dv[k] - 0.25 * dt * gr[a] * dv[k]);
            }
            r[k] = ra;
        }
    }
    block_partials<2>(acc, part);
}

// s_i = p_i - dt^2/4 (df/dx p)_i / m_i on free nodes (0 elsewhere); block
// partials of <p, s>_M.
template <int DIM, int DEG, bool ELASTIC>
__global__ __launch_bounds__(kMidBlock) void k_mid_node_apply(MidGrid g, MidTiles tl, const double *mf,
                                                              const double *pv, double dt, double *s, double *part,
                                                              const MidCg *cg) {
    if (cg->done) return;
    double acc[1] = {0.0};
    NodeAt n;
    if (node_at<DIM>(g, tl, n)) {
        double df[DIM];
        if constexpr (ELASTIC)
            slab_sum<DIM, DEG, DIM>(g, tl, n, df);
        else
#pragma unroll
            for (int a = 0; a < DIM; ++a) df[a] = 0.0;
        const double m = mf[n.i];
        const double cc = 0.25 * dt * dt;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + n.i;
            double sa = 0.0;
            if (m > 0.0) {
                sa = pv[k] - cc * df[a] / m;
                acc[0] += m * pv[k] * sa;
            }
            s[k] = sa;
        }
    }
    block_partials<1>(acc, part);
}

// CG start: rc = b = -r, p = rc, delta = 0; block partials of <rc, rc>_M.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_cg_init(MidGrid g, MidTiles tl, const double *mf, const double *r,
                                                           double *delta, double *rc, double *pv, double *part) {
    double acc[1] = {0.0};
    NodeAt n;
    if (node_at<DIM>(g, tl, n)) {
        const double m = mf[n.i];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + n.i;
            const double b = -r[k];
            rc[k] = b;
            pv[k] = b;
            delta[k] = 0.0;
            acc[0] += m * b * b;
        }
    }
    block_partials<1>(acc, part);
}

// CG iteration `it`, after the operator application.  Every block sums the
// partials of <p, s>_M (nps blocks) in the same fixed order, so all take the
// same alpha = gamma / <p, s>_M; then delta += alpha p, rc -= alpha s, and
// block partials of <rc, rc>_M.  A non-positive <p, s>_M stops the CG (the
// direction has no positive curvature): at the first iteration delta = -r,
// the steepest-descent direction, instead.  Block 0 counts the iteration and
// raises the stop for the next kernel (no block of this one reads either).
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_cg_step(MidGrid g, MidTiles tl, const double *mf, const double *r,
                                                           const double *pv, const double *s, double *delta,
                                                           double *rc, const double *part_ps, int64_t nps,
                                                           double *part, MidCg *cg, int it) {
    if (cg->done) return;
    const double ps = block_total(part_ps, nps, 1, 0);
    NodeAt n;
    const bool have = node_at<DIM>(g, tl, n);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!(ps > 0.0)) {
        if (it == 0 && have)
#pragma unroll
            for (int a = 0; a < DIM; ++a) delta[a * g.nodes + n.i] = -r[a * g.nodes + n.i];
        if (lead) {
            cg->iters += 1;
            cg->stop = 1;
        }
        return;
    }
    const double alpha = cg->gamma[it & 1] / ps;
    double acc[1] = {0.0};
    if (have) {
        const double m = mf[n.i];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + n.i;
            delta[k] += alpha * pv[k];
            const double ra = rc[k] - alpha * s[k];
            rc[k] = ra;
            acc[0] += m * ra * ra;
        }
    }
    block_partials<1>(acc, part);
    if (lead) cg->iters += 1;
}

// CG iteration `it`, last kernel: every block sums the partials of
// kappa = <rc, rc>_M in the same fixed order; beta = kappa / gamma; unless the
// CG stops (tolerance, iteration cap, or the curvature stop raised by the
// step kernel) p = rc + beta p.  Block 0 stores kappa as the next gamma (the
// other slot of two: this kernel's blocks read the current one) and the stop
// flag; a block that starts after it and sees the flag skips the update,
// which it would skip anyway.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_cg_dir(MidGrid g, MidTiles tl, const double *rc, double *pv,
                                                          const double *part, int64_t nblk, MidCg *cg, int it) {
    if (cg->done) return;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (cg->stop) {
        if (lead) cg->done = 1;
        return;
    }
    const double kappa = block_total(part, nblk, 1, 0);
    const double beta = kappa / cg->gamma[it & 1];
    const bool stop = kappa <= cg->tol2 * cg->gamma0 || (uint32_t)it + 1u >= cg->max_iters;
    if (lead) {
        cg->gamma[(it + 1) & 1] = kappa;
        if (stop) cg->done = 1;
    }
    if (stop) return;
    NodeAt n;
    if (!node_at<DIM>(g, tl, n)) return;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int64_t k = a * g.nodes + n.i;
        pv[k] = rc[k] + beta * pv[k];
    }
}

// Scalars from the block partials of the node pass before it (one block; the
// partials are summed in block order per thread stride, then a fixed tree):
//   SC_EVAL:  out[0] = sum m |r|^2, out[1] = E = sum m (|dv|^2/8 - dt/4 g.dv)
//             + sum V Psi (the key tiles' energy partials)
//   SC_INIT:  gamma = gamma0 = <rc, rc>_M; stop at once when gamma0 is 0 or
//             no iteration is allowed
enum { SC_EVAL = 0, SC_INIT = 1 };

template <int OP>
__global__ __launch_bounds__(kMidBlock) void k_mid_scalars(const double *part, int64_t nblk, const double *epart,
                                                           int64_t nk, double *out, MidCg *cg, double tol2,
                                                           uint32_t max_iters) {
    if constexpr (OP == SC_EVAL) {
        const double res2 = block_total(part, nblk, 2, 0);
        const double kin = block_total(part, nblk, 2, 1);
        const double phi = epart ? block_total(epart, nk, 1, 0) : 0.0;
        if (threadIdx.x == 0) {
            out[0] = res2;
            out[1] = kin + phi;
        }
    } else {
        const double t = block_total(part, nblk, 1, 0);
        if (threadIdx.x != 0) return;
        cg->gamma[0] = t;
        cg->gamma0 = t;
        cg->tol2 = tol2;
        cg->stop = 0;
        cg->max_iters = max_iters;
        cg->done = (t <= tol2 * t || max_iters == 0) ? 1u : 0u;
    }
}

template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_axpy(MidGrid g, MidTiles tl, const double *a, double alpha,
                                                        const double *b, double *out) {
    NodeAt n;
    if (!node_at<DIM>(g, tl, n)) return;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const int64_t k = c * g.nodes + n.i;
        out[k] = (a ? a[k] : 0.0) + alpha * b[k];
    }
}

// vt_i = v_i + dv_i on free nodes (0 elsewhere); u_i = xt_i - x_i =
// dt (v_i + vt_i) / 2.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_finish(MidGrid g, MidTiles tl, const double *mf, const double *gv,
                                                          const double *dv, double dt, double *gvt, double *gu) {
    NodeAt n;
    if (!node_at<DIM>(g, tl, n)) return;
    const bool free_node = mf[n.i] > 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int64_t k = a * g.nodes + n.i;
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
// One wavefront per listed key tile, vt and u of the tile's region staged in
// LDS, the particles walked level by level as in the particle passes: the
// old state comes from the sorted copies and the new state goes to the
// caller's planes at the particle's sorted position, so the particles leave
// the step in the solve's order (the next step's sort reads them nearly in
// place).
// What the transfer to particles reads of one particle of the sorted copy.
template <int DIM>
struct MidRow {
    uint32_t cell, id;
    double m, off[DIM], F[DIM * DIM];
};

template <int DIM>
__device__ __forceinline__ void mid_row_load(const MidSorted &S, int64_t p, bool with_id, MidRow<DIM> &w) {
    w.cell = S.cell[p];
    w.id = with_id ? S.id[p] : 0u;
    w.m = S.m[p];
#pragma unroll
    for (int a = 0; a < DIM; ++a) w.off[a] = S.off[a * S.n + p];
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) w.F[k] = S.F[k * S.n + p];
}

template <int DIM, int DEG>
__global__ __launch_bounds__(64) void k_mid_g2p(Parts<double> P, MidSorted S, MidGrid g, MidTiles tl,
                                                const double *gvt, const double *gu) {
    constexpr int R = region_nodes<DIM, DEG>(), RE = region_edge<DIM, DEG>(), E = tile_edge<DIM>();
    constexpr int D2 = DIM * DIM;
    __shared__ double stage[2 * DIM * R];  // vt planes, then u planes
    const int lane = threadIdx.x;
    const int64_t t = tl.klist[blockIdx.x];
    int tc[3];
    tile_coords<DIM>(g, t, tc);
    const int org[3] = {tc[0] * E, tc[1] * E, tc[2] * E};
    for (int k = lane; k < R; k += 64) {
        const int rx = k % RE, ry = DIM == 3 ? (k / RE) % RE : k / RE, rz = DIM == 3 ? k / (RE * RE) : 0;
        const int x = org[0] + rx, y = org[1] + ry, z = org[2] + rz;
        const bool in = x < g.N[0] && y < g.N[1] && (DIM == 2 || z < g.N[2]);
        const int64_t i = in ? node_slot<DIM>(g, x, y, z) : 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            stage[a * R + k] = in ? gvt[a * g.nodes + i] : 0.0;
            stage[(DIM + a) * R + k] = in ? gu[a * g.nodes + i] : 0.0;
        }
    }
    __syncthreads();
    const double s = 1.0 / g.dx;
    // level r + 1 of the sorted copy loads while level r is computed and stored
    const bool with_id = P.id != nullptr && S.id != nullptr;
    const int64_t key = t * 64 + lane_key<DIM, DEG>(lane);
    const uint32_t cnt = S.start[key + 1] - S.start[key];
    LevelWalk lw = level_walk(S.start, t, cnt);
    MidRow<DIM> cur, nxt;
    const uint64_t bal0 = ballot(cnt > 0);
    if (cnt > 0) mid_row_load<DIM>(S, lw.pos0 + __popcll(bal0 & lw.below), with_id, cur);
    for (uint32_t lr = 0; lr < lw.maxc; ++lr) {
        const bool act = lr < cnt;
        const uint64_t bal = ballot(act);
        const uint64_t bal_n = ballot(lr + 1 < cnt);
        const int64_t p = lw.pos0 + __popcll(bal & lw.below);
        lw.pos0 += __popcll(bal);
        if (lr + 1 < cnt) mid_row_load<DIM>(S, lw.pos0 + __popcll(bal_n & lw.below), with_id, nxt);
        if (!act) continue;
        Axis<double, DEG> ax[DIM];
        int ci[3];
        unpack_cell<DIM>(cur.cell, ci);
#pragma unroll
        for (int a = 0; a < DIM; ++a) axis_weights<double, DEG>(ci[a], cur.off[a], ax[a]);
        const int rb[3] = {ax[0].base - org[0], ax[1].base - org[1], DIM == 3 ? ax[DIM - 1].base - org[2] : 0};
        auto region = [&](int i, int j, int k) {
            return DIM == 3 ? (rb[0] + i) + RE * ((rb[1] + j) + RE * (rb[2] + k)) : (rb[0] + i) + RE * (rb[1] + j);
        };
        double v[DIM] = {}, U[DIM] = {};
        for_support<DIM, DEG>(ax, [&](double w, const double *, const double *, int i, int j, int k) {
            const int ri = region(i, j, k);
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                v[a] += w * stage[a * R + ri];
                U[a] += w * stage[(DIM + a) * R + ri];
            }
        });
        double B[D2] = {}, G[D2] = {};
        for_support<DIM, DEG>(ax, [&](double w, const double *gw, const double *r, int i, int j, int k) {
            const int ri = region(i, j, k);
            double vt[DIM], e[DIM], un[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                vt[a] = stage[a * R + ri];
                un[a] = stage[(DIM + a) * R + ri];
                e[a] = un[a] - U[a];
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) {
                    B[a * DIM + b] += w * (vt[a] * r[b] * g.dx + 0.5 * (vt[a] * e[b] - e[a] * vt[b]));
                    G[a * DIM + b] += un[a] * gw[b];
                }
        });
        double Fn[D2];
#pragma unroll
        for (int k = 0; k < D2; ++k) G[k] *= s;
#pragma unroll
        for (int a = 0; a < DIM; ++a) G[a * DIM + a] += 1.0;
        mat_mul<DIM>(G, cur.F, Fn);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double o = cur.off[a] + U[a] * s;
            const double c = floor(o);
            ci[a] += (int)c;
            P.off[a * P.s + p] = o - c;
            P.v[a * P.s + p] = v[a];
        }
        P.cell[p] = pack_cell<DIM>(ci);
        P.m[p] = cur.m;
        if (with_id) P.id[p] = cur.id;
#pragma unroll
        for (int k = 0; k < D2; ++k) {
            P.B[k * P.s + p] = B[k];
            P.F[k * P.s + p] = Fn[k];
        }
        cur = nxt;
    }
}

// The particles that took no part, back after all others, unchanged (staged
// by k_mid_sort_dead: v in the m v planes, B in the first d^2 M planes).
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_put_dead(Parts<double> P, MidSorted S, int64_t nodes) {
    const int64_t p = (int64_t)S.start[nodes] + gtid();
    if (p >= (int64_t)S.start[nodes + 1]) return;
    P.cell[p] = S.cell[p];
    P.m[p] = S.m[p];
    if (P.id) P.id[p] = S.id[p];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        P.off[a * P.s + p] = S.off[a * S.n + p];
        P.v[a * P.s + p] = S.mv[a * S.n + p];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        P.B[k * P.s + p] = S.M[k * S.n + p];
        P.F[k * P.s + p] = S.F[k * S.n + p];
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kMidBlock - 1) / kMidBlock); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
MidGrid mid_grid(int dim, const int *cells, const int *band, double dx) {
    MidGrid g{};
    const int E = dim == 3 ? tile_edge<3>() : tile_edge<2>();
    g.tiles = 1;
    for (int a = 0; a < 3; ++a) {
        g.N[a] = a < dim ? cells[a] + 1 : 1;
        g.T[a] = a < dim ? (g.N[a] + E - 1) / E : 1;
        g.tiles *= g.T[a];
    }
    for (int k = 0; k < 6; ++k) g.band[k] = band[k];
    g.nodes = g.tiles * 64;
    g.dx = dx;
    return g;
}

int mid_region_nodes(int dim, int degree) {
    if (dim == 3) return degree == 2 ? region_nodes<3, 2>() : region_nodes<3, 3>();
    return degree == 2 ? region_nodes<2, 2>() : region_nodes<2, 3>();
}

int64_t mid_node_blocks(int64_t nn) { return (nn + kNodeTilesPerBlock - 1) / kNodeTilesPerBlock; }
int64_t mid_scan_blocks(int64_t nodes) { return (nodes + 1023) / 1024; }

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

template <int DIM, int DEG>
void launch_mid_sort(const Parts<double> &P, const MidGrid &g, const MidSorted &S, const MidTiles &tl, uint32_t *key,
                     uint32_t *count, uint32_t *cursor, uint32_t *bsum, int32_t *counts, uint32_t *flags,
                     hipStream_t st) {
    // buckets: one per node slot, then one for the particles that take no part
    const int64_t nbk = g.nodes + 1;
    k_mid_fill_u32<<<blocks_for(nbk), kMidBlock, 0, st>>>(count, nbk);
    k_mid_fill_u32<<<blocks_for(nbk), kMidBlock, 0, st>>>(cursor, nbk);
    if (P.n > 0) k_mid_keys<DIM, DEG><<<blocks_for(P.n), kMidBlock, 0, st>>>(P, g, key, count, flags);
    const int64_t nb = mid_scan_blocks(nbk);
    uint32_t *start = const_cast<uint32_t *>(S.start);
    k_mid_scan1<<<(unsigned)nb, kMidBlock, 0, st>>>(count, nbk, start, bsum);
    k_mid_scan2<<<1, kMidBlock, 0, st>>>(bsum, nb, start, nbk);
    k_mid_scan3<<<blocks_for(nbk), kMidBlock, 0, st>>>(start, nbk, bsum);
    if (P.n > 0) k_mid_place<<<blocks_for(P.n), kMidBlock, 0, st>>>(P.n, key, S.start, cursor, S.perm);
    // count and cursor are free again: tile flags and their prefix sums
    uint32_t *kf = count, *nf = count + g.tiles, *hf = count + 2 * g.tiles;
    uint32_t *ks = cursor, *ns = cursor + g.tiles + 1, *hs = cursor + 2 * (g.tiles + 1);
    const int64_t tb = mid_scan_blocks(g.tiles);
    k_mid_tile_flags<DIM><<<blocks_for(g.tiles), kMidBlock, 0, st>>>(g, S.start, kf, nf, hf);
    for (int q = 0; q < 3; ++q) {
        const uint32_t *f = q == 0 ? kf : (q == 1 ? nf : hf);
        uint32_t *sc = q == 0 ? ks : (q == 1 ? ns : hs);
        k_mid_scan1<<<(unsigned)tb, kMidBlock, 0, st>>>(f, g.tiles, sc, bsum);
        k_mid_scan2<<<1, kMidBlock, 0, st>>>(bsum, tb, sc, g.tiles);
        k_mid_scan3<<<blocks_for(g.tiles), kMidBlock, 0, st>>>(sc, g.tiles, bsum);
    }
    k_mid_tile_place<<<blocks_for(g.tiles), kMidBlock, 0, st>>>(g.tiles, kf, nf, hf, ks, ns, hs, tl, counts);
}

template <int DIM, int DEG>
void launch_mid_sort_state(const Parts<double> &P, const MidSorted &S, const MidTiles &tl, int64_t nodes,
                           hipStream_t st) {
    if (tl.nk > 0) k_mid_sort_state<DIM, DEG><<<(unsigned)tl.nk, 64, 0, st>>>(P, S, tl);
    if (P.n > 0) k_mid_sort_dead<DIM><<<blocks_for(P.n), kMidBlock, 0, st>>>(P, S, nodes);
}

template <int DIM, int DEG>
void launch_mid_p2g(const MidSorted &S, const MidGrid &g, const MidTiles &tl, double *mf, double *gv, hipStream_t st) {
    if (tl.nk == 0) return;
    k_mid_tile<DIM, DEG, TILE_P2G><<<(unsigned)tl.nk, 64, 0, st>>>(S, g, tl, MidMaterial{}, nullptr, nullptr, 0.0, 0.0,
                                                                   nullptr, nullptr, nullptr);
    k_mid_node_p2g<DIM, DEG><<<(unsigned)mid_node_blocks(tl.nn), kMidBlock, 0, st>>>(g, tl, mf, gv);
}

template <int DIM, int DEG>
void launch_mid_force_tiles(const MidSorted &S, const MidGrid &g, const MidTiles &tl, const MidMaterial &mat,
                            const double *gv, const double *dv, double dt, double *epart, uint32_t *flags,
                            hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    if (tl.nk == 0) return;
    hipExtLaunchKernelGGL(k_mid_tile<DIM, DEG, TILE_FORCE>, dim3((unsigned)tl.nk), dim3(64), 0, st, ev0, ev1, 0, S, g,
                          tl, mat, gv, dv, 0.5 * dt, 0.25 * dt, epart, flags, (const MidCg *)nullptr);
}

template <int DIM, int DEG>
void launch_mid_force_nodes(const MidGrid &g, const MidTiles &tl, bool elastic, const double *dv, double dt,
                            const double *grav, const double *mf, double *r, const double *epart, double *part,
                            double *out, hipStream_t st) {
    if (tl.nk == 0) return;
    const double3 gr = make_double3(grav[0], grav[1], grav[2]);
    const int64_t nb = mid_node_blocks(tl.nn);
    if (elastic)
        k_mid_node_force<DIM, DEG, true><<<(unsigned)nb, kMidBlock, 0, st>>>(g, tl, mf, dv, dt, gr, r, part);
    else
        k_mid_node_force<DIM, DEG, false><<<(unsigned)nb, kMidBlock, 0, st>>>(g, tl, mf, dv, dt, gr, r, part);
    k_mid_scalars<SC_EVAL><<<1, kMidBlock, 0, st>>>(part, nb, elastic ? epart : nullptr, tl.nk, out, nullptr, 0.0, 0);
}

template <int DIM, int DEG>
void launch_mid_apply_tiles(const MidSorted &S, const MidGrid &g, const MidTiles &tl, const MidMaterial &mat,
                            const double *pv, MidCg *cg, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    if (tl.nk == 0) return;
    hipExtLaunchKernelGGL(k_mid_tile<DIM, DEG, TILE_APPLY>, dim3((unsigned)tl.nk), dim3(64), 0, st, ev0, ev1, 0, S, g,
                          tl, mat, pv, (const double *)nullptr, 1.0, 0.0, (double *)nullptr, (uint32_t *)nullptr,
                          (const MidCg *)cg);
}

template <int DIM, int DEG>
void launch_mid_apply_nodes(const MidGrid &g, const MidTiles &tl, bool elastic, const double *pv, const double *mf,
                            double dt, double *s, double *part, MidCg *cg, hipStream_t st) {
    if (tl.nk == 0) return;
    const int64_t nb = mid_node_blocks(tl.nn);
    if (elastic)
        k_mid_node_apply<DIM, DEG, true><<<(unsigned)nb, kMidBlock, 0, st>>>(g, tl, mf, pv, dt, s, part, cg);
    else
        k_mid_node_apply<DIM, DEG, false><<<(unsigned)nb, kMidBlock, 0, st>>>(g, tl, mf, pv, dt, s, part, cg);
}

template <int DIM>
void launch_mid_cg_init(const MidGrid &g, const MidTiles &tl, const double *mf, const double *r, double *delta,
                        double *rc, double *pv, double *part, MidCg *cg, double tol2, uint32_t max_iters,
                        hipStream_t st) {
    if (tl.nn == 0) return;
    const int64_t nb = mid_node_blocks(tl.nn);
    k_mid_cg_init<DIM><<<(unsigned)nb, kMidBlock, 0, st>>>(g, tl, mf, r, delta, rc, pv, part);
    k_mid_scalars<SC_INIT><<<1, kMidBlock, 0, st>>>(part, nb, nullptr, 0, nullptr, cg, tol2, max_iters);
}

template <int DIM>
void launch_mid_cg_step(const MidGrid &g, const MidTiles &tl, const double *mf, const double *r, const double *pv,
                        const double *s, double *delta, double *rc, const double *part_ps, double *part, MidCg *cg,
                        int it, hipStream_t st) {
    if (tl.nn == 0) return;
    const int64_t nb = mid_node_blocks(tl.nn);
    k_mid_cg_step<DIM><<<(unsigned)nb, kMidBlock, 0, st>>>(g, tl, mf, r, pv, s, delta, rc, part_ps, nb, part, cg, it);
}

template <int DIM>
void launch_mid_cg_dir(const MidGrid &g, const MidTiles &tl, const double *rc, double *pv, const double *part,
                       MidCg *cg, int it, hipStream_t st) {
    if (tl.nn == 0) return;
    const int64_t nb = mid_node_blocks(tl.nn);
    k_mid_cg_dir<DIM><<<(unsigned)nb, kMidBlock, 0, st>>>(g, tl, rc, pv, part, nb, cg, it);
}

template <int DIM>
void launch_mid_axpy(const MidGrid &g, const MidTiles &tl, const double *a, double alpha, const double *b, double *out,
                     hipStream_t st) {
    if (tl.nn == 0) return;
    k_mid_axpy<DIM><<<(unsigned)mid_node_blocks(tl.nn), kMidBlock, 0, st>>>(g, tl, a, alpha, b, out);
}

template <int DIM>
void launch_mid_finish(const MidGrid &g, const MidTiles &tl, const double *mf, const double *gv, const double *dv,
                       double dt, double *gvt, double *gu, hipStream_t st) {
    if (tl.nn == 0) return;
    k_mid_finish<DIM><<<(unsigned)mid_node_blocks(tl.nn), kMidBlock, 0, st>>>(g, tl, mf, gv, dv, dt, gvt, gu);
}

template <int DIM, int DEG>
void launch_mid_g2p(const Parts<double> &P, const MidSorted &S, const MidGrid &g, const MidTiles &tl,
                    const double *gvt, const double *gu, hipStream_t st) {
    if (tl.nk > 0) k_mid_g2p<DIM, DEG><<<(unsigned)tl.nk, 64, 0, st>>>(P, S, g, tl, gvt, gu);
    if (P.n > 0) k_mid_put_dead<DIM><<<blocks_for(P.n), kMidBlock, 0, st>>>(P, S, g.nodes);
}

#define APIC_MID_INST_DD(DIM, DEG)                                                                                    \
    template void launch_mid_sort<DIM, DEG>(const Parts<double> &, const MidGrid &, const MidSorted &,                \
                                            const MidTiles &, uint32_t *, uint32_t *, uint32_t *, uint32_t *,         \
                                            int32_t *, uint32_t *, hipStream_t);                                      \
    template void launch_mid_sort_state<DIM, DEG>(const Parts<double> &, const MidSorted &, const MidTiles &,         \
                                                  int64_t, hipStream_t);                                              \
    template void launch_mid_p2g<DIM, DEG>(const MidSorted &, const MidGrid &, const MidTiles &, double *, double *,  \
                                           hipStream_t);                                                              \
    template void launch_mid_force_tiles<DIM, DEG>(const MidSorted &, const MidGrid &, const MidTiles &,              \
                                                   const MidMaterial &, const double *, const double *, double,       \
                                                   double *, uint32_t *, hipStream_t, hipEvent_t, hipEvent_t);        \
    template void launch_mid_force_nodes<DIM, DEG>(const MidGrid &, const MidTiles &, bool, const double *, double,   \
                                                   const double *, const double *, double *, const double *,          \
                                                   double *, double *, hipStream_t);                                  \
    template void launch_mid_apply_tiles<DIM, DEG>(const MidSorted &, const MidGrid &, const MidTiles &,              \
                                                   const MidMaterial &, const double *, MidCg *, hipStream_t,         \
                                                   hipEvent_t, hipEvent_t);                                           \
    template void launch_mid_apply_nodes<DIM, DEG>(const MidGrid &, const MidTiles &, bool, const double *,           \
                                                   const double *, double, double *, double *, MidCg *, hipStream_t); \
    template void launch_mid_g2p<DIM, DEG>(const Parts<double> &, const MidSorted &, const MidGrid &,                 \
                                           const MidTiles &, const double *, const double *, hipStream_t);
#define APIC_MID_INST_D(DIM)                                                                                          \
    template void launch_mid_cg_init<DIM>(const MidGrid &, const MidTiles &, const double *, const double *,          \
                                          double *, double *, double *, double *, MidCg *, double, uint32_t,          \
                                          hipStream_t);                                                               \
    template void launch_mid_cg_step<DIM>(const MidGrid &, const MidTiles &, const double *, const double *,          \
                                          const double *, const double *, double *, double *, const double *,         \
                                          double *, MidCg *, int, hipStream_t);                                       \
    template void launch_mid_cg_dir<DIM>(const MidGrid &, const MidTiles &, const double *, double *, const double *, \
                                         MidCg *, int, hipStream_t);                                                  \
    template void launch_mid_axpy<DIM>(const MidGrid &, const MidTiles &, const double *, double, const double *,     \
                                       double *, hipStream_t);                                                        \
    template void launch_mid_finish<DIM>(const MidGrid &, const MidTiles &, const double *, const double *,           \
                                         const double *, double, double *, double *, hipStream_t);

APIC_MID_INST_DD(2, 2)
APIC_MID_INST_DD(2, 3)
APIC_MID_INST_DD(3, 2)
APIC_MID_INST_DD(3, 3)
APIC_MID_INST_D(2)
APIC_MID_INST_D(3)

}  // namespace apic
