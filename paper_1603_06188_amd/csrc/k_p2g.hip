// Transfer to grid (Sec. 3.2) with the force of Sec. 3.3 fused in (lambda = 0).
//
// One wavefront per listed tile, one lane per key (base node).  Every
// particle of a key touches the same K^DIM nodes, so a lane accumulates its
// particles' contributions to those nodes in registers, then the 64 lanes add
// their sums into the tile's slab in LDS in K^DIM rounds (within a round the
// lanes hit distinct nodes: plain read-modify-write, no atomics), and the
// slab is stored with plain coalesced writes.
//
// Per particle, in cell units (r = (x_i - x_p)/dx, grad w in 1/cell):
//   m_i     += w m_p
//   (mv)_i  += w (m_p v_p + Qc r) + Ac grad w
//   Qc = m_p B_p D^{-1} dx        with D = k dx^2 I, 1/k = 4 (quadratic), 3 (cubic)
//   Ac = -dt V_p tau_p / dx       tau = P F^T = mu (F F^T - I) + lambda ln J I
// so Ac grad w is dt times the force contribution -V_p P F^T grad w of Sec. 3.3.
// The K^DIM node terms are factored axis by axis (tensor-product weights).
#include "apic_bin_device.h"
#include "apic_kernels.h"

namespace apic {

template <typename T, int DIM, int DEG>
struct P2GParticle {
    Axis<T, DEG> ax[DIM];
    T m;
    T p[DIM];              // m v
    T Qc[DIM * DIM];
    T Ac[DIM * DIM];
};

// Raw state of one particle as stored (loaded one level ahead of its use).
template <typename T, int DIM>
struct P2GRaw {
    uint32_t cell;
    T m, off[DIM], v[DIM], B[DIM * DIM], F[DIM * DIM];
};

template <typename T, int DIM>
__device__ __forceinline__ void p2g_load(const Parts<T> &P, uint32_t q, P2GRaw<T, DIM> &r) {
    const int64_t s = P.s;
    const uint32_t qb = q * (uint32_t)sizeof(T);
    r.cell = P.cell[q];
    r.m = plane_at(P.m, qb);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        r.off[a] = plane_at(P.off + a * s, qb);
        r.v[a] = plane_at(P.v + a * s, qb);
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        r.B[k] = plane_at(P.B + k * s, qb);
        r.F[k] = plane_at(P.F + k * s, qb);
    }
}

// Checks a loaded particle and forms its per-particle terms.  Returns false
// (and sets a flag) when the particle must be skipped.
template <typename T, int DIM, int DEG>
__device__ __forceinline__ bool p2g_prepare(const P2GRaw<T, DIM> &r, const int *key, const StepParams<T> &prm,
                                            T inv_dx, uint32_t *flags, P2GParticle<T, DIM, DEG> &pp) {
    int ci[3] = {0, 0, 0};
    unpack_cell<DIM>(r.cell, ci);
    T off[DIM], v[DIM], B[DIM * DIM], F[DIM * DIM];
    const T m = r.m;
    bool finite = is_finite(m);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        off[a] = r.off[a];
        v[a] = r.v[a];
        finite = finite && is_finite(off[a]) && is_finite(v[a]);
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        B[k] = r.B[k];
        F[k] = r.F[k];
        finite = finite && is_finite(B[k]) && is_finite(F[k]);
    }
    if (!finite) {
        atomicOr(flags, FLAG_NONFINITE);
        return false;
    }
    bool same = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        axis_weights<T, DEG>(ci[a], off[a], pp.ax[a]);
        same = same && pp.ax[a].base == key[a];
    }
    if (!same) {
        atomicOr(flags, FLAG_UNSORTED);
        return false;
    }
    pp.m = m;
    const T qs = m * inv_D_factor<T, DEG>() * inv_dx;
#pragma unroll
    for (int a = 0; a < DIM; ++a) pp.p[a] = m * v[a];
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        pp.Qc[k] = qs * B[k];
        pp.Ac[k] = T(0);
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
            const T sc = -prm.dt * m * prm.inv_rho0 * inv_dx;
#pragma unroll
            for (int r = 0; r < DIM; ++r)
#pragma unroll
                for (int c = r; c < DIM; ++c) {
                    T ff = T(0);
#pragma unroll
                    for (int k = 0; k < DIM; ++k) ff += F[r * DIM + k] * F[c * DIM + k];
                    const T tau = r == c ? prm.mu * (ff - T(1)) + prm.lam * lnJ : prm.mu * ff;
                    pp.Ac[r * DIM + c] = sc * tau;
                    pp.Ac[c * DIM + r] = sc * tau;
                }
        } else {
            atomicOr(flags, FLAG_INVERTED);
        }
    }
    return true;
}

// Adds one particle's contributions to the nodes of z-slices [C0, C0+CZ)
// (3D) of its support.  acc_m[(c-C0)][b][a], acc_v[k][(c-C0)][b][a].
//
// With w = wx wy wz, r = (rx, ry, rz), grad w = (dx wy wz, wx dy wz, wx wy dz)
// the momentum contribution to node (a,b,c), component k, is
//   w p_k + w (Qc r)_k + (Ac grad w)_k
//   = X0_k(a) (wy wz)(b,c) + Yb_k(b) (wx wz)(a,c) + Zc_k(c) (wx wy)(a,b)
// with X0_k = wx p_k + wx rx Qc_k0 + dx Ac_k0, Yb_k = wy ry Qc_k1 + dy Ac_k1,
// Zc_k = wz rz Qc_k2 + dz Ac_k2: three multiply-adds per node and component.
template <typename T, int DEG, int C0, int CZ>
__device__ __forceinline__ void p2g_accumulate3(const P2GParticle<T, 3, DEG> &pp, T (&acc_m)[CZ][DEG + 1][DEG + 1],
                                                T (&acc_v)[3][CZ][DEG + 1][DEG + 1]) {
    constexpr int K = DEG + 1;
    const Axis<T, DEG> &X = pp.ax[0], &Y = pp.ax[1], &Z = pp.ax[2];
    T X0[3][K], Yb[3][K], Mx[K], Rxy[K][K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const T wrx = X.w[a] * X.r[a], wry = Y.w[a] * Y.r[a];
        Mx[a] = pp.m * X.w[a];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            X0[k][a] = X.w[a] * pp.p[k] + wrx * pp.Qc[k * 3 + 0] + X.dw[a] * pp.Ac[k * 3 + 0];
            Yb[k][a] = wry * pp.Qc[k * 3 + 1] + Y.dw[a] * pp.Ac[k * 3 + 1];
        }
#pragma unroll
        for (int b = 0; b < K; ++b) Rxy[a][b] = X.w[a] * Y.w[b];
    }
    // slice by slice: the slice's own factors, then its K*K nodes
#pragma unroll
    for (int cc = 0; cc < CZ; ++cc) {
        const int c = C0 + cc;
        const T wrz = Z.w[c] * Z.r[c];
        T Zc[3], Pyz[K], Qxz[K];
#pragma unroll
        for (int k = 0; k < 3; ++k) Zc[k] = wrz * pp.Qc[k * 3 + 2] + Z.dw[c] * pp.Ac[k * 3 + 2];
#pragma unroll
        for (int b = 0; b < K; ++b) {
            Pyz[b] = Y.w[b] * Z.w[c];
            Qxz[b] = X.w[b] * Z.w[c];
        }
#pragma unroll
        for (int b = 0; b < K; ++b)
#pragma unroll
            for (int a = 0; a < K; ++a) {
                acc_m[cc][b][a] += Mx[a] * Pyz[b];
                // separate multiply-adds into the accumulator (one FMA each)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    acc_v[k][cc][b][a] += X0[k][a] * Pyz[b];
                    acc_v[k][cc][b][a] += Yb[k][b] * Qxz[a];
                    acc_v[k][cc][b][a] += Zc[k] * Rxy[a][b];
                }
            }
        // the slice is accumulated here, not deferred (bounds live factors)
#pragma unroll
        for (int b = 0; b < K; ++b)
#pragma unroll
            for (int a = 0; a < K; ++a) {
                asm volatile("" : "+v"(acc_m[cc][b][a]));
#pragma unroll
                for (int k = 0; k < 3; ++k) asm volatile("" : "+v"(acc_v[k][cc][b][a]));
            }
    }
}

// 2D: contribution = X0_k(a) wy(b) + Yb_k(b) wx(a).
template <typename T, int DEG>
__device__ __forceinline__ void p2g_accumulate2(const P2GParticle<T, 2, DEG> &pp, T (&acc_m)[DEG + 1][DEG + 1],
                                                T (&acc_v)[2][DEG + 1][DEG + 1]) {
    constexpr int K = DEG + 1;
    const Axis<T, DEG> &X = pp.ax[0], &Y = pp.ax[1];
    T X0[2][K], Yb[2][K], Mx[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const T wrx = X.w[a] * X.r[a], wry = Y.w[a] * Y.r[a];
        Mx[a] = pp.m * X.w[a];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            X0[k][a] = X.w[a] * pp.p[k] + wrx * pp.Qc[k * 2 + 0] + X.dw[a] * pp.Ac[k * 2 + 0];
            Yb[k][a] = wry * pp.Qc[k * 2 + 1] + Y.dw[a] * pp.Ac[k * 2 + 1];
        }
    }
#pragma unroll
    for (int b = 0; b < K; ++b)
#pragma unroll
        for (int a = 0; a < K; ++a) {
            acc_m[b][a] += Mx[a] * Y.w[b];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                acc_v[k][b][a] += X0[k][a] * Y.w[b];
                acc_v[k][b][a] += Yb[k][b] * X.w[a];
            }
        }
}

// Slab planes in LDS, padded so that the 64 lanes of one round (a 4x4x4 or
// 8x8 block of distinct nodes) fall in distinct banks of each half-wave:
// 3D x + 8 y + 68 z, 2D x + 40 y.  The slab in global memory is compact.
template <int DIM, int DEG>
struct SlabLds {
    static constexpr int RE = Geo<DIM, DEG>::RE;
    static constexpr int SY = DIM == 3 ? 8 : 40;
    static constexpr int SZ = DIM == 3 ? 68 : 0;
    static constexpr int PLANE = DIM == 3 ? SZ * RE : SY * RE;
    __device__ static constexpr int at(int x, int y, int z) { return x + SY * y + SZ * z; }
    // compact index (x + RE (y + RE z)) -> padded index
    __device__ static int from_compact(int i) {
        const int x = i % RE, y = (i / RE) % RE, z = i / (RE * RE);
        return at(x, y, DIM == 3 ? z : 0);
    }
};

// Slab (LDS) update of one node from this lane: plain, or two-sum with an
// error plane when compensated.
template <typename T, bool COMP, int RN, int NC>
__device__ __forceinline__ void slab_add(T *lds, int comp, int idx, T x) {
    T *hi = lds + comp * RN + idx;
    if constexpr (!COMP) {
        *hi += x;
    } else {
        const T a = *hi;
        const T s = a + x;
        *hi = s;
        lds[(NC + comp) * RN + idx] += two_sum_err(a, x, s);
    }
}

// z-slices per pass: keeps the register accumulators near 128 VGPRs.
template <typename T, int DIM, int DEG>
constexpr int p2g_slices() {
    constexpr int K = DEG + 1;
    constexpr int per_slice = K * K * (1 + DIM) * (int)(sizeof(T) / 4);
    return DIM == 2 ? K : (per_slice * K <= 128 ? K : (per_slice * 2 <= 128 ? 2 : 1));
}

template <typename T, int DEG, bool COMP, int C0, int CZ>
__device__ __forceinline__ void p2g_pass3(const Parts<T> &P, const int *key, int lcoord[3], uint32_t start,
                                          uint32_t kstart, uint32_t cnt, uint32_t maxc, const StepParams<T> &prm,
                                          T inv_dx, uint32_t *flags, T *lds) {
    using Gm = Geo<3, DEG>;
    using SL = SlabLds<3, DEG>;
    constexpr int K = DEG + 1, NC = Gm::NC, LP = SL::PLANE;
    const int lane = lane_id();
    T acc_m[CZ][K][K], acc_v[3][CZ][K][K];
#pragma unroll
    for (int c = 0; c < CZ; ++c)
#pragma unroll
        for (int b = 0; b < K; ++b)
#pragma unroll
            for (int a = 0; a < K; ++a) {
                acc_m[c][b][a] = T(0);
                acc_v[0][c][b][a] = acc_v[1][c][b][a] = acc_v[2][c][b][a] = T(0);
            }
    // level j's particle is loaded while level j-1 is accumulated
    uint32_t level = 0;
    uint64_t mask = ballot(cnt > 0);
    P2GRaw<T, 3> raw;
    if (cnt > 0) p2g_load<T, 3>(P, (uint32_t)particle_at(start, kstart, 0, mask, 0, maxc, lane), raw);
    for (uint32_t j = 0; j < maxc; ++j) {
        const uint32_t level_n = level + (uint32_t)popc64(mask);
        const uint64_t mask_n = ballot(cnt > j + 1);
        P2GRaw<T, 3> raw_n;
        if (cnt > j + 1)
            p2g_load<T, 3>(P, (uint32_t)particle_at(start, kstart, level_n, mask_n, j + 1, maxc, lane), raw_n);
        if (cnt > j) {
            P2GParticle<T, 3, DEG> pp;
            if (p2g_prepare<T, 3, DEG>(raw, key, prm, inv_dx, flags, pp))
                p2g_accumulate3<T, DEG, C0, CZ>(pp, acc_m, acc_v);
        }
        raw = raw_n;
        level = level_n;
        mask = mask_n;
    }
    // K*K*CZ rounds; lanes of one round touch distinct nodes
#pragma unroll
    for (int c = 0; c < CZ; ++c)
#pragma unroll
        for (int b = 0; b < K; ++b)
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const int idx = SL::at(lcoord[0] + a, lcoord[1] + b, lcoord[2] + C0 + c);
                slab_add<T, COMP, LP, NC>(lds, 0, idx, acc_m[c][b][a]);
                slab_add<T, COMP, LP, NC>(lds, 1, idx, acc_v[0][c][b][a]);
                slab_add<T, COMP, LP, NC>(lds, 2, idx, acc_v[1][c][b][a]);
                slab_add<T, COMP, LP, NC>(lds, 3, idx, acc_v[2][c][b][a]);
                wave_lds_sync();
            }
}

template <typename T, int DIM, int DEG, bool COMP>
__device__ __forceinline__ void p2g_body(const Parts<T> &P, const BinLists &cur, const BinLists &nxt,
                                         const TileTables &tab, const Slabs<T> &slabs, const GridState<T> &g,
                                         const StepParams<T> &prm, uint32_t blk, uint32_t nblk) {
    using Gm = Geo<DIM, DEG>;
    using SL = SlabLds<DIM, DEG>;
    constexpr int K = Gm::K, RN = Gm::RN, NC = Gm::NC, LP = SL::PLANE;
    constexpr int NPL = NC * (COMP ? 2 : 1);      // planes
    constexpr int SLAB = NPL * RN;                // compact, in global memory
    constexpr int LSLAB = NPL * LP;               // padded, in LDS
    __shared__ T lds_all[4 * LSLAB];
    T *lds = lds_all + (threadIdx.x >> 6) * LSLAB;
    const int lane = lane_id();
    int lcoord[3] = {0, 0, 0};
    local_coords<DIM>(lane, lcoord);
    if (blk == 0) {
        // the grid update that follows raises these bounds of max |vt|, and
        // the layout the following G2P builds starts from empty lists
        for (int i = (int)threadIdx.x; i < kBuckets; i += (int)blockDim.x) {
            g.vmax[i] = 0u;
            nxt.rec_count[i] = 0u;
            nxt.tot[i] = 0u;
        }
        if (threadIdx.x == 0) nxt.dead[0] = 0u;
    }
    const TileWalk walk = tile_walk(cur);
    for (uint32_t r = blk * 4 + (threadIdx.x >> 6); r < walk.nrec; r += nblk * 4) {
        uint32_t start, cnt, maxc, kstart;
        const uint32_t t = tile_of_record(walk, r, cur, tab, start, cnt, maxc, kstart);
        int key[3] = {0, 0, 0};
        tile_origin<DIM>(t, g.d.TN, key);
#pragma unroll
        for (int a = 0; a < DIM; ++a) key[a] += lcoord[a];
        for (int i = lane; i < LSLAB; i += 64) lds[i] = T(0);
        wave_lds_sync();
        if constexpr (DIM == 3) {
            constexpr int CZ = p2g_slices<T, 3, DEG>();
            p2g_pass3<T, DEG, COMP, 0, CZ>(P, key, lcoord, start, kstart, cnt, maxc, prm, g.inv_dx, g.flags, lds);
            if constexpr (CZ < K) p2g_pass3<T, DEG, COMP, CZ, (2 * CZ <= K ? CZ : K - CZ)>(
                P, key, lcoord, start, kstart, cnt, maxc, prm, g.inv_dx, g.flags, lds);
            if constexpr (2 * CZ < K) p2g_pass3<T, DEG, COMP, 2 * CZ, (3 * CZ <= K ? CZ : K - 2 * CZ)>(
                P, key, lcoord, start, kstart, cnt, maxc, prm, g.inv_dx, g.flags, lds);
            if constexpr (3 * CZ < K) p2g_pass3<T, DEG, COMP, 3 * CZ, K - 3 * CZ>(
                P, key, lcoord, start, kstart, cnt, maxc, prm, g.inv_dx, g.flags, lds);
        } else {
            T acc_m[K][K], acc_v[2][K][K];
#pragma unroll
            for (int bb = 0; bb < K; ++bb)
#pragma unroll
                for (int a = 0; a < K; ++a) acc_m[bb][a] = acc_v[0][bb][a] = acc_v[1][bb][a] = T(0);
            uint32_t level = 0;
            for (uint32_t jj = 0; jj < maxc; ++jj) {
                const uint64_t mask = ballot(cnt > jj);
                if (cnt > jj) {
                    const int64_t q = particle_at(start, kstart, level, mask, jj, maxc, lane);
                    P2GRaw<T, 2> raw;
                    p2g_load<T, 2>(P, (uint32_t)q, raw);
                    P2GParticle<T, 2, DEG> pp;
                    if (p2g_prepare<T, 2, DEG>(raw, key, prm, g.inv_dx, g.flags, pp))
                        p2g_accumulate2<T, DEG>(pp, acc_m, acc_v);
                }
                level += (uint32_t)popc64(mask);
            }
#pragma unroll
            for (int bb = 0; bb < K; ++bb)
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    const int idx = SL::at(lcoord[0] + a, lcoord[1] + bb, 0);
                    slab_add<T, COMP, LP, NC>(lds, 0, idx, acc_m[bb][a]);
                    slab_add<T, COMP, LP, NC>(lds, 1, idx, acc_v[0][bb][a]);
                    slab_add<T, COMP, LP, NC>(lds, 2, idx, acc_v[1][bb][a]);
                    wave_lds_sync();
                }
        }
        T *out = slabs.v + (int64_t)r * slabs.stride;
        for (int i = lane; i < SLAB; i += 64) out[i] = lds[(i / RN) * LP + SL::from_compact(i % RN)];
        wave_lds_sync();
    }
}

template <typename T, int DIM, int DEG, bool COMP>
__global__ __launch_bounds__(256) void k_p2g(Parts<T> P, BinLists cur, BinLists nxt, TileTables tab, Slabs<T> slabs,
                                             GridState<T> g, StepParams<T> prm) {
    p2g_body<T, DIM, DEG, COMP>(P, cur, nxt, tab, slabs, g, prm, blockIdx.x, gridDim.x);
}

template <typename T, int DIM, int DEG, bool COMP>
__global__ __launch_bounds__(256) void k_p2g_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k) {
    const BatchStep<T> b = batch_step<T>(descs, start, n, k);
    const SceneDesc<T> &d = *b.d;
    p2g_body<T, DIM, DEG, COMP>(d.bufs[b.sp.src], b.cur, b.nxt, d.tab[b.sp.cur], d.slabs, d.g, d.prm, b.blk, b.nblk);
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_p2g_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, int blocks, hipStream_t st) {
    hipLaunchKernelGGL((k_p2g_batch<T, DIM, DEG, COMP>), dim3((unsigned)blocks), dim3(256), 0, st, descs, start, n, k);
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_p2g(const Parts<T> &P, const BinLists &cur, const BinLists &nxt, const TileTables &tab,
                const Slabs<T> &slabs, const GridState<T> &g, const StepParams<T> &prm, int64_t max_records,
                hipStream_t st) {
    int64_t blocks = (max_records + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_p2g<T, DIM, DEG, COMP>), dim3((unsigned)blocks), dim3(256), 0, st, P, cur, nxt, tab, slabs,
                       g, prm);
}

#define APIC_P2G_INST(T, DIM, DEG)                                                                                \
    template void launch_p2g_batch<T, DIM, DEG, false>(const SceneDesc<T> *, const int32_t *, int, int, int,        \
                                                       hipStream_t);                                              \
    template void launch_p2g_batch<T, DIM, DEG, true>(const SceneDesc<T> *, const int32_t *, int, int, int,         \
                                                      hipStream_t);                                               \
    template void launch_p2g<T, DIM, DEG, false>(const Parts<T> &, const BinLists &, const BinLists &,           \
                                                 const TileTables &, const Slabs<T> &, const GridState<T> &,     \
                                                 const StepParams<T> &, int64_t, hipStream_t);                   \
    template void launch_p2g<T, DIM, DEG, true>(const Parts<T> &, const BinLists &, const BinLists &,            \
                                                const TileTables &, const Slabs<T> &, const GridState<T> &,      \
                                                const StepParams<T> &, int64_t, hipStream_t);
APIC_P2G_INST(float, 2, 2)
APIC_P2G_INST(float, 2, 3)
APIC_P2G_INST(float, 3, 2)
APIC_P2G_INST(float, 3, 3)
APIC_P2G_INST(double, 2, 2)
APIC_P2G_INST(double, 2, 3)
APIC_P2G_INST(double, 3, 2)
APIC_P2G_INST(double, 3, 3)

}  // namespace apic
