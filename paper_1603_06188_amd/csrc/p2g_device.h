// Device helpers of the transfer to grid (Sec. 3.2) with the force of
// Sec. 3.3 fused in, shared by the P2G kernels: a particle's per-particle
// terms, the factored tensor-product accumulation of its node contributions
// into a key's register sums, and the padded LDS slab.
#pragma once
#include "apic_bin_device.h"

namespace apic {

template <typename T, int DIM, int DEG>
struct P2GParticle {
    Axis<T, DEG> ax[DIM];
    T m;
    T p[DIM];              // m (v - uref): momentum relative to the tile's reference velocity
    T Qc[DIM * DIM];
    T Ac[DIM * DIM];
};

// Raw state of one particle as stored (loaded one level ahead of its use).
template <typename T, int DIM>
struct P2GRaw {
    uint32_t cell;
    T m, off[DIM], v[DIM], B[DIM * DIM], F[DIM * DIM];
};

// ABS: absolute positions in the offset planes; the cell plane is not read.
template <typename T, int DIM, bool ABS = false>
__device__ __forceinline__ void p2g_load(const Parts<T> &P, uint32_t q, P2GRaw<T, DIM> &r) {
    const int64_t s = P.s;
    const uint32_t qb = q * (uint32_t)sizeof(T);
    r.cell = ABS ? 0u : P.cell[q];
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

// Checks a loaded particle and forms its per-particle terms, its momentum
// relative to the reference velocity uref of its tile.  Returns false (and
// sets a flag) when the particle must be skipped.
template <typename T, int DIM, int DEG, bool ABS = false>
__device__ __forceinline__ bool p2g_prepare(const P2GRaw<T, DIM> &r, const int *key, const StepParams<T> &prm,
                                            T inv_dx, uint32_t *flags, const T *uref,
                                            P2GParticle<T, DIM, DEG> &pp) {
    int ci[3] = {0, 0, 0};
    T off[DIM], v[DIM], B[DIM * DIM], F[DIM * DIM];
    const T m = r.m;
    // x * 0 is NaN exactly when x is infinite or NaN, and +-0 otherwise, so
    // the sum of all of them is zero exactly when every value is finite (one
    // multiply-add per value instead of a class test and a mask merge)
    T z = m * T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        v[a] = r.v[a];
        z = fma_t(r.off[a], T(0), z);
        z = fma_t(v[a], T(0), z);
    }
    particle_cells<T, DIM, ABS>(r.cell, r.off, inv_dx, ci, off);
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        B[k] = r.B[k];
        F[k] = r.F[k];
        z = fma_t(B[k], T(0), z);
        z = fma_t(F[k], T(0), z);
    }
    const bool finite = z == T(0);
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
    // Q = m C in cell units of r: C = B D^{-1} = B inv_D / dx^2 (quadratic,
    // cubic); multilinear carries the lagged C itself (Sec. 5.9)
    T qs;
    if constexpr (DEG == 1)
        qs = m / inv_dx;
    else
        qs = m * inv_D_factor<T, DEG>() * inv_dx;
#pragma unroll
    for (int a = 0; a < DIM; ++a) pp.p[a] = m * (v[a] - uref[a]);
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
//   = wz(c) S_k(a,b) + Zc_k(c) Rxy(a,b)
// with X0_k = wx p_k + wx rx Qc_k0 + dx Ac_k0, Yb_k = wy ry Qc_k1 + dy Ac_k1,
// Zc_k = wz rz Qc_k2 + dz Ac_k2, S_k(a,b) = X0_k(a) wy(b) + Yb_k(b) wx(a)
// (independent of the slice) and Rxy = wx wy: two multiply-adds per node
// and component, one for the mass (m wx wy) wz.
template <typename T, int DEG, int C0, int CZ>
__device__ __forceinline__ void p2g_accumulate3(const P2GParticle<T, 3, DEG> &pp, T (&acc_m)[CZ][DEG + 1][DEG + 1],
                                                T (&acc_v)[3][CZ][DEG + 1][DEG + 1]) {
    constexpr int K = DEG + 1;
    const Axis<T, DEG> &X = pp.ax[0], &Y = pp.ax[1], &Z = pp.ax[2];
    T X0[3][K], Yb[3][K], Zc[3][CZ];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const T wrx = X.w[a] * X.r[a], wry = Y.w[a] * Y.r[a];
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
    }
    // column by column (a, b): its own factors, then its CZ nodes
#pragma unroll
    for (int b = 0; b < K; ++b)
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const T Rxy = X.w[a] * Y.w[b], Mxy = pp.m * Rxy;
            T S[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) S[k] = X0[k][a] * Y.w[b] + Yb[k][b] * X.w[a];
#pragma unroll
            for (int cc = 0; cc < CZ; ++cc) {
                const T wz = Z.w[C0 + cc];
                acc_m[cc][b][a] += Mxy * wz;
                // separate multiply-adds into the accumulator (one FMA each)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    acc_v[k][cc][b][a] += wz * S[k];
                    acc_v[k][cc][b][a] += Zc[k][cc] * Rxy;
                }
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
// 3D x + 8 y + 68 z, 2D x + 40 y.  The slab in global memory is compact, in
// the block order of SlabMap.
template <int DIM, int DEG>
struct SlabLds {
    static constexpr int RE = Geo<DIM, DEG>::RE;
    static constexpr int SY = DIM == 3 ? 8 : 40;
    static constexpr int SZ = DIM == 3 ? 68 : 0;
    static constexpr int PLANE = DIM == 3 ? SZ * RE : SY * RE;
    __device__ static constexpr int at(int x, int y, int z) { return x + SY * y + SZ * z; }
    // global position j -> padded index
    __device__ static int from_global(int j) {
        int c[3] = {0, 0, 0};
        SlabMap<DIM, DEG>::coords(j, c);
        return at(c[0], c[1], c[2]);
    }
};

// All NC planes of one node: every read first, then the sums and writes
// (one wait for the LDS per node instead of one per plane).
template <typename T, bool COMP, int LP, int NC>
__device__ __forceinline__ void slab_add_node(T *lds, int idx, const T (&x)[NC]) {
    T hi[NC], lo[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        hi[q] = lds[q * LP + idx];
        if constexpr (COMP) lo[q] = lds[(NC + q) * LP + idx];
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const T sum = hi[q] + x[q];
        lds[q * LP + idx] = sum;
        if constexpr (COMP) lds[(NC + q) * LP + idx] = lo[q] + two_sum_err(hi[q], x[q], sum);
    }
}

// z-slices per pass: keeps the register accumulators near 128 VGPRs.
template <typename T, int DIM, int DEG>
constexpr int p2g_slices() {
    constexpr int K = DEG + 1;
    constexpr int per_slice = K * K * (1 + DIM) * (int)(sizeof(T) / 4);
    return DIM == 2 ? K : (per_slice * K <= 128 ? K : (per_slice * 2 <= 128 ? 2 : 1));
}

// Adds a lane's register sums for z-slices [C0, C0+CZ) of its key's support
// into the slab in K*K*CZ rounds; the lanes of one round touch distinct
// nodes (distinct keys), so a plain read-modify-write is safe.
template <typename T, int DEG, bool COMP, int C0, int CZ>
__device__ __forceinline__ void slab_flush3(const int *lcoord, const T (&acc_m)[CZ][DEG + 1][DEG + 1],
                                            const T (&acc_v)[3][CZ][DEG + 1][DEG + 1], T *lds) {
    using Gm = Geo<3, DEG>;
    using SL = SlabLds<3, DEG>;
    constexpr int K = DEG + 1, NC = Gm::NC, LP = SL::PLANE;
#pragma unroll
    for (int c = 0; c < CZ; ++c)
#pragma unroll
        for (int b = 0; b < K; ++b)
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const int idx = SL::at(lcoord[0] + a, lcoord[1] + b, lcoord[2] + C0 + c);
                const T x[NC] = {acc_m[c][b][a], acc_v[0][c][b][a], acc_v[1][c][b][a], acc_v[2][c][b][a]};
                slab_add_node<T, COMP, LP, NC>(lds, idx, x);
                wave_lds_sync();
            }
}

// Slab planes between the padded LDS layout and the compact global one
// (one wavefront): the lane's padded indices are formed once and serve every
// plane.
template <typename T, int DIM, int DEG, bool COMP>
__device__ __forceinline__ void slab_store(const T *lds, T *out) {
    using Gm = Geo<DIM, DEG>;
    using SL = SlabLds<DIM, DEG>;
    constexpr int RN = Gm::RN, LP = SL::PLANE, NP = Gm::NC * (COMP ? 2 : 1), R = (RN + 63) / 64;
    const int lane = lane_id();
    int pad[R];
#pragma unroll
    for (int k = 0; k < R; ++k) pad[k] = SL::from_global(lane + 64 * k);
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (lane + 64 * k < RN) out[q * RN + lane + 64 * k] = lds[q * LP + pad[k]];
}

template <typename T, int DIM, int DEG, bool COMP>
__device__ __forceinline__ void slab_load(const T *in, T *lds) {
    using Gm = Geo<DIM, DEG>;
    using SL = SlabLds<DIM, DEG>;
    constexpr int RN = Gm::RN, LP = SL::PLANE, NP = Gm::NC * (COMP ? 2 : 1), R = (RN + 63) / 64;
    const int lane = lane_id();
    int pad[R];
#pragma unroll
    for (int k = 0; k < R; ++k) pad[k] = SL::from_global(lane + 64 * k);
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (lane + 64 * k < RN) lds[q * LP + pad[k]] = in[q * RN + lane + 64 * k];
}

// Reference velocity of a tile (wave-wide) from the velocities v of the
// particles at level 0 of its keys (lanes with has = true): their mean,
// rounded by quantize_ref; every lane gets the same value (the butterfly adds
// the same pairs on every lane).  0 for a tile without particles.
template <typename T, int DIM>
__device__ __forceinline__ void reference_of_level0(const T *v, bool has, T *uref) {
    const uint64_t mask = ballot(has);
    const T inv_n = mask ? T(1) / (T)popc64(mask) : T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        T x = has ? v[a] : T(0);
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o, 64);
        uref[a] = wave_uniform(quantize_ref(x * inv_n));
    }
}

// The same with the level-0 velocities loaded here (lanes with act > 0).
template <typename T, int DIM>
__device__ __forceinline__ void tile_reference(const Parts<T> &P, uint32_t start, uint32_t kstart, uint32_t act,
                                               uint32_t maxc, T *uref) {
    const int lane = lane_id();
    const uint64_t mask = ballot(act > 0);
    T v[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) v[a] = T(0);
    if (act > 0) {
        const uint32_t q = (uint32_t)particle_at(start, kstart, 0, mask, 0, maxc, lane);
#pragma unroll
        for (int a = 0; a < DIM; ++a) v[a] = P.v[a * P.s + q];
    }
    reference_of_level0<T, DIM>(v, act > 0, uref);
}

// Reference velocity the slab of key tile t was formed with.
template <typename T, int DIM>
__device__ __forceinline__ void tile_uref(uint32_t t, const GridState<T> &g, T *uref) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) uref[k] = g.uref[k * g.d.tiles + t];
}

// Register sums of a key's particles (cnt per key, maxc the tile's busiest)
// for z-slices [C0, C0+CZ), added into the slab.  MOV: only the first `act`
// particles of each key (its movers), levels [0, jend).  Momenta are taken
// relative to the tile's reference velocity uref; DERIVE: uref is first set
// from the level-0 particles this pass loads (reference_of_level0).
template <typename T, int DEG, bool COMP, int C0, int CZ, bool MOV = false, bool DERIVE = false, bool ABS = false>
__device__ __forceinline__ void p2g_pass3(const Parts<T> &P, const int *key, int lcoord[3], uint32_t start,
                                          uint32_t kstart, uint32_t cnt, uint32_t maxc, uint32_t act, uint32_t jend,
                                          const StepParams<T> &prm, T inv_dx, uint32_t *flags, T *uref,
                                          T *lds) {
    constexpr int K = DEG + 1;
    const int lane = lane_id();
    const uint32_t n_act = MOV ? act : cnt, j_end = MOV ? jend : maxc;
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
    if (n_act > 0) p2g_load<T, 3, ABS>(P, (uint32_t)particle_at(start, kstart, 0, mask, 0, maxc, lane), raw);
    if constexpr (DERIVE) reference_of_level0<T, 3>(raw.v, n_act > 0, uref);
    // level j from cur while level j + 1 loads into nxt; two levels per trip
    // with the buffers swapped, so no registers are copied between levels
    P2GRaw<T, 3> raw_b;
    auto level_step = [&](const P2GRaw<T, 3> &cur, P2GRaw<T, 3> &nxt, uint32_t j) {
        const uint32_t level_n = level + (uint32_t)popc64(mask);
        const uint64_t mask_n = ballot(cnt > j + 1);
        if (n_act > j + 1)
            p2g_load<T, 3, ABS>(P, (uint32_t)particle_at(start, kstart, level_n, mask_n, j + 1, maxc, lane), nxt);
        if (n_act > j) {
            P2GParticle<T, 3, DEG> pp;
            if (p2g_prepare<T, 3, DEG, ABS>(cur, key, prm, inv_dx, flags, uref, pp))
                p2g_accumulate3<T, DEG, C0, CZ>(pp, acc_m, acc_v);
        }
        level = level_n;
        mask = mask_n;
    };
    for (uint32_t j = 0; j < j_end; j += 2) {
        level_step(raw, raw_b, j);
        if (j + 1 < j_end) level_step(raw_b, raw, j + 1);
    }
    slab_flush3<T, DEG, COMP, C0, CZ>(lcoord, acc_m, acc_v, lds);
}

}  // namespace apic
