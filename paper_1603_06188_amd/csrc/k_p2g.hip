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

// Loads particle `q`, checks it and forms its per-particle terms.  Returns
// false (and sets a flag) when the particle must be skipped.
template <typename T, int DIM, int DEG>
__device__ __forceinline__ bool p2g_prepare(const Parts<T> &P, int64_t q, const int *key, const StepParams<T> &prm,
                                            T inv_dx, uint32_t *flags, P2GParticle<T, DIM, DEG> &pp) {
    const int64_t s = P.s;
    int ci[3] = {0, 0, 0};
    unpack_cell<DIM>(P.cell[q], ci);
    T off[DIM], v[DIM], B[DIM * DIM], F[DIM * DIM];
    const T m = P.m[q];
    bool finite = is_finite(m);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        off[a] = P.off[a * s + q];
        v[a] = P.v[a * s + q];
        finite = finite && is_finite(off[a]) && is_finite(v[a]);
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        B[k] = P.B[k * s + q];
        F[k] = P.F[k * s + q];
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
    T X0[3][K], Yb[3][K], Zc[3][CZ], Mx[K];
    T Pyz[K][CZ], Qxz[K][CZ], Rxy[K][K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const T wrx = X.w[a] * X.r[a], wry = Y.w[a] * Y.r[a];
        Mx[a] = pp.m * X.w[a];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            X0[k][a] = X.w[a] * pp.p[k] + wrx * pp.Qc[k * 3 + 0] + X.dw[a] * pp.Ac[k * 3 + 0];
            Yb[k][a] = wry * pp.Qc[k * 3 + 1] + Y.dw[a] * pp.Ac[k * 3 + 1];
        }
    }
#pragma unroll
    for (int cc = 0; cc < CZ; ++cc) {
        const int c = C0 + cc;
        const T wrz = Z.w[c] * Z.r[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) Zc[k][cc] = wrz * pp.Qc[k * 3 + 2] + Z.dw[c] * pp.Ac[k * 3 + 2];
#pragma unroll
        for (int b = 0; b < K; ++b) {
            Pyz[b][cc] = Y.w[b] * Z.w[c];
            Qxz[b][cc] = X.w[b] * Z.w[c];
        }
    }
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int b = 0; b < K; ++b) Rxy[a][b] = X.w[a] * Y.w[b];
#pragma unroll
    for (int cc = 0; cc < CZ; ++cc)
#pragma unroll
        for (int b = 0; b < K; ++b)
#pragma unroll
            for (int a = 0; a < K; ++a) {
                acc_m[cc][b][a] += Mx[a] * Pyz[b][cc];
                // separate multiply-adds into the accumulator (one FMA each)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    acc_v[k][cc][b][a] += X0[k][a] * Pyz[b][cc];
                    acc_v[k][cc][b][a] += Yb[k][b] * Qxz[a][cc];
                    acc_v[k][cc][b][a] += Zc[k][cc] * Rxy[a][b];
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

// Index of the jj-th particle of this lane's key: level-major layout
// (start + offset of level jj + rank among the keys present in it), or
// key-major (kstart + jj) for tiles busier than kMaxLevels.
__device__ __forceinline__ int64_t particle_at(uint32_t start, uint32_t kstart, uint32_t level, uint64_t mask,
                                               uint32_t jj, uint32_t maxc, int lane) {
    return maxc > (uint32_t)kMaxLevels ? (int64_t)kstart + jj
                                       : (int64_t)start + level + (uint32_t)popc64(mask & lanes_below(lane));
}

template <typename T, int DEG, bool COMP, int C0, int CZ>
__device__ __forceinline__ void p2g_pass3(const Parts<T> &P, const int *key, int lcoord[3], uint32_t start,
                                          uint32_t kstart, uint32_t cnt, uint32_t maxc, const StepParams<T> &prm,
                                          T inv_dx, uint32_t *flags, T *lds) {
    using Gm = Geo<3, DEG>;
    constexpr int K = DEG + 1, RE = Gm::RE, RN = Gm::RN, NC = Gm::NC;
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
    uint32_t level = 0;
    for (uint32_t j = 0; j < maxc; ++j) {
        const uint64_t mask = ballot(cnt > j);
        if (cnt > j) {
            const int64_t q = particle_at(start, kstart, level, mask, j, maxc, lane);
            P2GParticle<T, 3, DEG> pp;
            if (p2g_prepare<T, 3, DEG>(P, q, key, prm, inv_dx, flags, pp))
                p2g_accumulate3<T, DEG, C0, CZ>(pp, acc_m, acc_v);
        }
        level += (uint32_t)popc64(mask);
    }
    // K*K*CZ rounds; lanes of one round touch distinct nodes
#pragma unroll
    for (int c = 0; c < CZ; ++c)
#pragma unroll
        for (int b = 0; b < K; ++b)
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const int idx = (lcoord[0] + a) + RE * ((lcoord[1] + b) + RE * (lcoord[2] + C0 + c));
                slab_add<T, COMP, RN, NC>(lds, 0, idx, acc_m[c][b][a]);
                slab_add<T, COMP, RN, NC>(lds, 1, idx, acc_v[0][c][b][a]);
                slab_add<T, COMP, RN, NC>(lds, 2, idx, acc_v[1][c][b][a]);
                slab_add<T, COMP, RN, NC>(lds, 3, idx, acc_v[2][c][b][a]);
                wave_lds_sync();
            }
}

template <typename T, int DIM, int DEG, bool COMP>
__global__ __launch_bounds__(256) void k_p2g(Parts<T> P, BinLists cur, BinLists nxt, TileTables tab, Slabs<T> slabs,
                                             GridState<T> g, StepParams<T> prm) {
    using Gm = Geo<DIM, DEG>;
    constexpr int K = Gm::K, RE = Gm::RE, RN = Gm::RN, NC = Gm::NC;
    constexpr int SLAB = NC * RN * (COMP ? 2 : 1);
    __shared__ T lds_all[4 * SLAB];
    T *lds = lds_all + (threadIdx.x >> 6) * SLAB;
    const int lane = lane_id();
    int lcoord[3] = {0, 0, 0};
    local_coords<DIM>(lane, lcoord);
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        // the grid update that follows raises these bounds of max |vt|, and
        // the layout the following G2P builds starts from empty lists
        g.vmax[threadIdx.x] = 0u;
        nxt.rec_count[threadIdx.x] = 0u;
        nxt.tot[threadIdx.x] = 0u;
        nxt.node_count[threadIdx.x] = 0u;
        if (threadIdx.x == 0) nxt.dead[0] = 0u;
    }
    uint32_t total_recs, rcnt, live, bmine;
    const uint32_t rpre = wave_bucket_prefix(cur.rec_count, total_recs, rcnt);
    const uint32_t bbase = wave_bucket_prefix(cur.tot, live, bmine);
    for (uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6); r < total_recs; r += gridDim.x * 4) {
        uint32_t b, j;
        bucket_locate(r, rpre, rcnt, b, j);
        const uint32_t t = cur.rec_list[(int64_t)b * cur.rcap + j];
        int key[3] = {0, 0, 0};
        tile_origin<DIM>(t, g.d.TN, key);
#pragma unroll
        for (int a = 0; a < DIM; ++a) key[a] += lcoord[a];
        const uint32_t start = __shfl(bbase, (int)b, 64) + tab.off[t];
        const uint32_t cnt = tab.kcount[(int64_t)t * 64 + lane];
        const uint32_t maxc = tab.maxc[t];
        // first particle of this lane's key in key-major order (busy tiles)
        const uint32_t kstart = maxc > (uint32_t)kMaxLevels ? start + tab.kprefix[(int64_t)t * 64 + lane] : 0u;
        for (int i = lane; i < SLAB; i += 64) lds[i] = T(0);
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
                    P2GParticle<T, 2, DEG> pp;
                    if (p2g_prepare<T, 2, DEG>(P, q, key, prm, g.inv_dx, g.flags, pp))
                        p2g_accumulate2<T, DEG>(pp, acc_m, acc_v);
                }
                level += (uint32_t)popc64(mask);
            }
#pragma unroll
            for (int bb = 0; bb < K; ++bb)
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    const int idx = (lcoord[0] + a) + RE * (lcoord[1] + bb);
                    slab_add<T, COMP, RN, NC>(lds, 0, idx, acc_m[bb][a]);
                    slab_add<T, COMP, RN, NC>(lds, 1, idx, acc_v[0][bb][a]);
                    slab_add<T, COMP, RN, NC>(lds, 2, idx, acc_v[1][bb][a]);
                    wave_lds_sync();
                }
        }
        T *out = slabs.v + (int64_t)r * slabs.stride;
        for (int i = lane; i < SLAB; i += 64) out[i] = lds[i];
        wave_lds_sync();
    }
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
