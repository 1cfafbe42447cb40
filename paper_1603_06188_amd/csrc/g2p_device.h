// Device helpers of the transfer to particles (Sec. 3.4, lambda = 0 form of
// Sec. 5.7) shared by the G2P kernels: weights and the new velocity in a
// fixed operation sequence, the advected position, the key-keeping test, the
// LDS region of grid velocities around a key tile and the particle loads.
#pragma once
#include "apic_bin_device.h"

namespace apic {

// Weights along one axis with a fixed operation sequence (see axis_weights).
template <typename T, int DEG>
__device__ __forceinline__ int axis_w_fixed(int cell, T off, T *w) {
#pragma clang fp contract(off)
    if constexpr (DEG == 1) {
        w[0] = T(1) - off;
        w[1] = off;
        return cell;
    } else if constexpr (DEG == 2) {
        const bool lower = off < T(0.5);
        const T c = lower ? off : off - T(1);
        const T l = T(0.5) - c, h = T(0.5) + c;
        w[0] = T(0.5) * (l * l);
        w[1] = T(0.75) - c * c;
        w[2] = T(0.5) * (h * h);
        return lower ? cell - 1 : cell;
    } else {
        const T u = off, q = T(1) - off;
        const T u2 = u * u, q2 = q * q;
        w[0] = (q2 * q) * T(1.0 / 6.0);
        w[1] = (T(0.5) * (u2 * u) - u2) + T(2.0 / 3.0);
        w[2] = (T(0.5) * (q2 * q) - q2) + T(2.0 / 3.0);
        w[3] = (u2 * u) * T(1.0 / 6.0);
        return cell - 1;
    }
}

// New velocity v = sum_i w_i vt_i with a fixed operation sequence, shared
// by both passes: first the x-axis sums Tx_k(a) = sum_{c,b} (wy(b) wz(c))
// (vt_k(a,b,c) - c_k), nodes in (c, b) order, then
// v_k = c_k + sum_a wx(a) Tx_k(a).  The reference velocity c (the grid
// velocity at the support node nearest the particle, see nearest_node) is
// taken out of every node value before the sums: with sum_i w_i = 1,
// sum_i w_i (x_i - x_p) = 0 and sum_i grad w_i = 0 (Sec. 3.5) it changes
// none of v, B or grad v, but a large common velocity no longer costs
// binary32 digits in B and grad v, which are differences of such sums.
// The nearest node carries a weight of at least 1/8 (quadratic, 3D) or
// about 1/9 (cubic), so c is never far out of scale with v: a corner node
// can have a weight near zero and, if nothing else reaches it, a velocity
// thousands of times larger than v, whose rounding would then dominate v.
template <typename T, int DIM, int DEG>
__device__ __forceinline__ void velocity_from_tx(const T (&tx)[DIM][DEG + 1], const T (&w)[DIM][DEG + 1],
                                                 const T *cref, T *vn) {
#pragma clang fp contract(off)
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < DEG + 1; ++a) s = fma_t(w[0][a], tx[k][a], s);
        vn[k] = cref[k] + s;
    }
}

// Position x + dt v as cell index + offset in [0, 1), fixed operation order;
// cfl is set when the step exceeds one cell.
template <typename T, int DIM>
__device__ __forceinline__ void move_position(const int *ci, const T *off, const T *vn, T dt_inv_dx, int *cn, T *on,
                                              bool &cfl) {
#pragma clang fp contract(off)
    cfl = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T step = dt_inv_dx * vn[a];
        cfl = cfl || !(step <= T(1) && step >= T(-1));
        T o = off[a] + step;
        const T fl = floor_t(o);
        int cc = ci[a] + (int)fl;
        o = o - fl;
        if (o >= T(1)) {
            o = o - T(1);
            cc += 1;
        }
        cn[a] = cc;
        on[a] = o;
    }
}

// The same for absolute binary32 positions (APIC_OPT_ABSOLUTE_POSITIONS):
// xn = x + dt v in absolute coordinates, then its cell and offset as
// cell_of_absolute derives them; fixed operation order.
template <typename T, int DIM>
__device__ __forceinline__ void move_absolute(const T *x, const T *vn, T dt, T inv_dx, T *xn, int *cn, T *on,
                                              bool &cfl) {
#pragma clang fp contract(off)
    cfl = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T step = dt * vn[a];
        const T cells = step * inv_dx;
        cfl = cfl || !(cells <= T(1) && cells >= T(-1));
        xn[a] = x[a] + step;
        cell_of_absolute(xn[a], inv_dx, cn[a], on[a]);
    }
}

// The CFL quantity of Sec. 4.3 of one particle's new state, |v| + c |B|_F,
// evaluated in the state's precision and folded into a running maximum (a
// NaN state propagates).  The bound passes over particles (first step of a
// call, apic_cfl_dt) evaluate it in binary64.
template <typename T, int DIM>
__device__ __forceinline__ void cfl_fold(const T *v, const T *B, double c, T &m) {
    T vv = T(0), bb = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) vv += v[a] * v[a];
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) bb += B[k] * B[k];
    const T u = sqrt(vv) + (T)c * sqrt(bb);
    m = u > m || u != u ? u : m;
}

// The same in binary64 (the bound passes over particles).
template <typename T, int DIM>
__device__ __forceinline__ void cfl_fold64(const T *v, const T *B, double c, double &m) {
    double vv = 0.0, bb = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) vv += (double)v[a] * (double)v[a];
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) bb += (double)B[k] * (double)B[k];
    const double u = sqrt(vv) + c * sqrt(bb);
    m = u > m || u != u ? u : m;
}

// Wave-wide: the maximum of m over the wavefront raised into one of the
// kVmaxSlots bound slots (non-negative binary64 values order as their bits;
// a NaN's bits exceed every finite value's).
__device__ __forceinline__ void cfl_raise(unsigned long long *slots, uint32_t slot, double m) {
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_xor(m, o, 64);
        m = y > m || y != y ? y : m;
    }
    if (lane_id() == 0 && m != 0.0)
        atomicMax(slots + slot % (uint32_t)kVmaxSlots, (unsigned long long)__double_as_longlong(m));
}

// Support index of the node nearest the particle along one axis, from the
// axis weights: the heavier of the two for multilinear (weight >= 1/2), the
// middle node for quadratic (weight >= 1/2), the heavier of the middle two
// for cubic (weight >= 0.479).
template <typename T, int DEG>
__device__ __forceinline__ int nearest_node(const T (&w)[DEG + 1]) {
    if constexpr (DEG == 1)
        return w[0] >= w[1] ? 0 : 1;
    else if constexpr (DEG == 2)
        return 1;
    else
        return w[1] >= w[2] ? 1 : 2;
}

// Bound of max_i |vt_i| over the slots the grid update raised (wave-wide).
__device__ __forceinline__ float wave_vmax(const uint32_t *slots) {
    static_assert(kVmaxSlots == 16 * 64, "16 slots per lane");
    const uint4 *q = (const uint4 *)(slots + 16 * lane_id());
    uint32_t m = 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 v = q[i];
        const uint32_t a = v.x > v.y ? v.x : v.y, c = v.z > v.w ? v.z : v.w;
        m = m > a ? m : a;
        m = m > c ? m : c;
    }
    return __uint_as_float(wave_max_u32(m));
}

// Largest displacement this step in cell units, with a margin for rounding:
// |v_p| <= max_i |vt_i| since the weights are a partition of unity.
template <typename T>
__device__ __forceinline__ T step_reach(float vbound, const StepParams<T> &prm, T inv_dx) {
    return (T)vbound * prm.dt * inv_dx * T(1.0001) + T(1e-6);
}

// True when the particle is farther than `reach` from every offset where its
// base node changes (1/2 for quadratic, 0 and 1 for cubic): it keeps its key.
template <typename T, int DIM, int DEG>
__device__ __forceinline__ bool keeps_key(const T *off, T reach) {
    bool far = reach < T(0.5);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T dist = DEG == 2 ? (off[a] < T(0.5) ? T(0.5) - off[a] : off[a] - T(0.5))
                                : (off[a] < T(0.5) ? off[a] : T(1) - off[a]);
        far = far && dist > reach;
    }
    return far;
}

// Dead particles of the current layout are walked in chunks of 64 after the
// listed tiles.
__device__ __forceinline__ uint32_t dead_chunks(int64_t n, uint32_t live) {
    return (uint32_t)((n - (int64_t)live + 63) / 64);
}

// Grid velocities of the 2^DIM node tiles from the key tile on, in LDS:
// 3D 8x8x8 nodes at x + 8 y + 68 z (the z pad spreads a wavefront's 4x4x4
// reads over the banks), 2D 16x16 nodes at x + 16 y; component-major.
// Grid velocities of the 2^DIM node tiles from the key tile on, in LDS:
// 3D 8x8x8 nodes at x + 8 y + 68 z (the z pad spreads a wavefront's 4x4x4
// reads over the banks), 2D 16x16 nodes at x + 16 y; component-major.
template <int DIM>
struct VtRegion {
    static constexpr int SY = DIM == 3 ? 8 : 16;
    static constexpr int SZ = DIM == 3 ? 68 : 0;
    static constexpr int SIZE = DIM == 3 ? 8 * 68 : 256;
    __device__ static constexpr int at(int x, int y, int z) { return x + SY * y + SZ * z; }
};

template <typename T, int DIM>
__device__ __forceinline__ void stage_velocities(uint32_t t, const GridState<T> &g, T *reg) {
    using R = VtRegion<DIM>;
    constexpr int TE = DIM == 3 ? 4 : 8;
    const int lane = lane_id();
    const int64_t G = g.d.G;
    int tc[3] = {0, 0, 0}, lc[3] = {0, 0, 0};
    tc[0] = (int)(t % (uint32_t)g.d.TN[0]);
    if constexpr (DIM == 3) {
        tc[1] = (int)((t / (uint32_t)g.d.TN[0]) % (uint32_t)g.d.TN[1]);
        tc[2] = (int)(t / ((uint32_t)g.d.TN[0] * (uint32_t)g.d.TN[1]));
    } else {
        tc[1] = (int)(t / (uint32_t)g.d.TN[0]);
    }
    local_coords<DIM>(lane, lc);
#pragma unroll
    for (int corner = 0; corner < (1 << DIM); ++corner) {
        bool ok = true;
        int64_t tau = 0, mul = 1;
        int rc[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int bit = (corner >> a) & 1;
            ok = ok && tc[a] + bit < g.d.TN[a];
            tau += (int64_t)(tc[a] + bit) * mul;
            mul *= g.d.TN[a];
            rc[a] = bit * TE + lc[a];
        }
        const int idx = R::at(rc[0], rc[1], rc[2]);
#pragma unroll
        for (int k = 0; k < DIM; ++k) reg[k * R::SIZE + idx] = ok ? g.vt[k * G + tau * 64 + lane] : T(0);
    }
}

// Occupancy target: binary32 quadratic 3D fits 128 registers (4 waves per
// SIMD); binary64 cubic 3D runs at 2 (256 registers, a few spilled) rather
// than the compiler's 1; other variants are left to the compiler.
template <typename T, int DIM, int DEG>
constexpr int g2p_min_waves() {
    if (sizeof(T) == 4 && DEG == 2) return 4;
    return (sizeof(T) == 8 && DIM == 3 && DEG == 3) ? 2 : 1;
}

// What G2P reads of a particle (loaded one chunk ahead of its use).
template <typename T, int DIM>
struct G2PRaw {
    uint32_t cell;
    int32_t id;
    T m, off[DIM], F[DIM * DIM];
};

template <typename T, int DIM, bool ABS = false>
__device__ __forceinline__ void g2p_load(const Parts<T> &src, uint32_t p, G2PRaw<T, DIM> &r) {
    const int64_t ss = src.s;
    const uint32_t pb = p * (uint32_t)sizeof(T);
    r.cell = ABS ? 0u : src.cell[p];
    r.m = plane_at(src.m, pb);
    r.id = src.id ? plane_at(src.id, p * 4u) : 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) r.off[a] = plane_at(src.off + a * ss, pb);
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) r.F[k] = plane_at(src.F + k * ss, pb);
}

// The update of one particle from the grid velocities staged in LDS around
// its key tile (`origin`: the tile's first node): new cell index and offset,
// velocity, B (stored units) and F, and its base node relative to the tile
// (lk).  Raises FLAG_CFL when the step exceeds one cell along an axis.
// B keeps the part of the affine field the transfer carries (APIC_TRANSFER_*).
// ABS (absolute binary32 positions): `xs` receives the new coordinates (what
// the offset planes store), and on/cn the cell and offset derived from them;
// otherwise xs = on.
template <typename T, int DIM, int DEG, bool ABS = false>
__device__ __forceinline__ void g2p_update(const G2PRaw<T, DIM> &raw, const T *reg, const int *origin,
                                           const GridState<T> &g, T dt_inv_dx, T gs, int *lk, int *cn, T *on, T *vn,
                                           T *Bs, T *Fn, int transfer, T *xs = nullptr, T dt = T(0)) {
    constexpr int K = DEG + 1;
    using R = VtRegion<DIM>;
    int ci[3] = {0, 0, 0};
    T off[DIM], wf[DIM][K], Bc[DIM * DIM];
    particle_cells<T, DIM, ABS>(raw.cell, raw.off, g.inv_dx, ci, off);
#pragma unroll
    for (int a = 0; a < DIM; ++a) lk[a] = axis_w_fixed<T, DEG>(ci[a], off[a], wf[a]) - origin[a];
    // One sweep over the support nodes (c, b, a) from LDS: the
    // axis-pair sums Tx_k(a) = sum_{b,c} wy wz vt_k (in the
    // sequence of pass 1), Ty_k(b) = sum_{a,c} wx wz vt_k and
    // Tz_k(c) = sum_{a,b} wx wy vt_k, from which
    //   v_k = sum_a wx Tx_k(a),
    //   B_k0 = sum_a wx rx Tx_k(a), grad v_k0 = sum_a dwx Tx_k(a),
    // and likewise along y and z.
    T Tx[DIM][K], Ty[DIM][K], Tz[DIM][K], cref[DIM];
    const int ic = R::at(lk[0] + nearest_node<T, DEG>(wf[0]), lk[1] + nearest_node<T, DEG>(wf[1]),
                         DIM == 3 ? lk[2] + nearest_node<T, DEG>(wf[DIM - 1]) : 0);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        cref[k] = reg[k * R::SIZE + ic];
#pragma unroll
        for (int ii = 0; ii < K; ++ii) Tx[k][ii] = Ty[k][ii] = Tz[k][ii] = T(0);
    }
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int c = 0; c < (DIM == 3 ? K : 1); ++c)
#pragma unroll
            for (int b = 0; b < K; ++b) {
                const T wyz = DIM == 3 ? wf[1][b] * wf[2][c] : wf[1][b];
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    const T wxz = DIM == 3 ? wf[0][a] * wf[2][c] : wf[0][a];
                    const T wxy = DIM == 3 ? wf[0][a] * wf[1][b] : T(0);
                    const int idx = R::at(lk[0] + a, lk[1] + b, DIM == 3 ? lk[2] + c : 0);
#pragma unroll
                    for (int k = 0; k < DIM; ++k) {
                        const T x = reg[k * R::SIZE + idx] - cref[k];
                        Tx[k][a] = fma_t(wyz, x, Tx[k][a]);
                        Ty[k][b] = fma_t(wxz, x, Ty[k][b]);
                        if constexpr (DIM == 3) Tz[k][c] = fma_t(wxy, x, Tz[k][c]);
                    }
                }
                // the sums are formed here, row by row, not sunk to
                // their later use (which would keep every LDS value
                // of the sweep in registers)
#pragma unroll
                for (int k = 0; k < DIM; ++k)
#pragma unroll
                    for (int ii = 0; ii < K; ++ii) {
                        asm volatile("" : "+v"(Ty[k][ii]));
                        if constexpr (DIM == 3) asm volatile("" : "+v"(Tz[k][ii]));
                    }
            }
    }
    velocity_from_tx<T, DIM, DEG>(Tx, wf, cref, vn);
    // B and grad v (cell units) from the axis sums; weight
    // derivatives and node offsets from the offsets
    T Gc[DIM * DIM];
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) Bc[k] = Gc[k] = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        Axis<T, DEG> ax;
        axis_weights<T, DEG>(ci[a], off[a], ax);
#pragma unroll
        for (int ii = 0; ii < K; ++ii) {
            const T wr = wf[a][ii] * ax.r[ii];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const T tk = a == 0 ? Tx[k][ii] : (a == 1 ? Ty[k][ii] : Tz[k][ii]);
                Bc[k * DIM + a] += wr * tk;
                Gc[k * DIM + a] += ax.dw[ii] * tk;
            }
        }
    }
    // F <- (I + dt grad v) F, grad v = Gc / dx
    T F[DIM * DIM];
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) F[k] = raw.F[k];
#pragma unroll
    for (int rr = 0; rr < DIM; ++rr)
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc += Gc[rr * DIM + k] * F[k * DIM + c];
            Fn[rr * DIM + c] = F[rr * DIM + c] + gs * acc;
        }
    bool cfl;
    if constexpr (ABS)
        move_absolute<T, DIM>(raw.off, vn, dt, g.inv_dx, xs, cn, on, cfl);
    else
        move_position<T, DIM>(ci, off, vn, dt_inv_dx, cn, on, cfl);
    if (cfl) atomicOr(g.flags, FLAG_CFL);
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) Bs[k] = DEG == 1 ? Gc[k] * g.inv_dx : Bc[k] * g.dx;
    keep_affine<T, DIM>(transfer, Bs);
}

// Dead particles (chunk `c` of the dead region after `live` listed ones) are
// carried over unchanged to their places after the new layout's live ones.
template <typename T, int DIM>
__device__ __forceinline__ void carry_dead(const Parts<T> &src, const Parts<T> &dst, const BinScratch &sc,
                                           uint32_t live, uint32_t live_nxt, uint32_t c) {
    const int64_t ss = src.s, ds = dst.s;
    const int64_t p = (int64_t)live + (int64_t)c * 64 + lane_id();
    if (p >= src.n) return;
    const int64_t q = (int64_t)live_nxt + sc.prank[p];
    dst.cell[q] = src.cell[p];
    dst.m[q] = src.m[p];
    if (src.id) dst.id[q] = src.id[p];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        dst.off[a * ds + q] = src.off[a * ss + p];
        dst.v[a * ds + q] = src.v[a * ss + p];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        dst.B[k * ds + q] = src.B[k * ss + p];
        dst.F[k * ds + q] = src.F[k * ss + p];
    }
}

// New velocity from the grid velocities staged in LDS (base node at lk
// relative to the region): x-axis sums Tx_k(a) over the nodes in (c, b)
// order, then velocity_from_tx -- the operation sequence of the G2P sweep,
// so both give the same bits.
template <typename T, int DIM, int DEG>
__device__ __forceinline__ void velocity_lds(const T *reg, const int *lk, const T (&w)[DIM][DEG + 1], T *vn) {
#pragma clang fp contract(off)
    constexpr int K = DEG + 1;
    using R = VtRegion<DIM>;
    T tx[DIM][K], cref[DIM];
    const int ic = R::at(lk[0] + nearest_node<T, DEG>(w[0]), lk[1] + nearest_node<T, DEG>(w[1]),
                         DIM == 3 ? lk[2] + nearest_node<T, DEG>(w[DIM - 1]) : 0);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        cref[k] = reg[k * R::SIZE + ic];
#pragma unroll
        for (int a = 0; a < K; ++a) tx[k][a] = T(0);
    }
#pragma unroll
    for (int c = 0; c < (DIM == 3 ? K : 1); ++c)
#pragma unroll
        for (int b = 0; b < K; ++b) {
            const T wyz = DIM == 3 ? w[1][b] * w[2][c] : w[1][b];
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const int idx = R::at(lk[0] + a, lk[1] + b, DIM == 3 ? lk[2] + c : 0);
#pragma unroll
                for (int k = 0; k < DIM; ++k)
                    tx[k][a] = fma_t(wyz, reg[k * R::SIZE + idx] - cref[k], tx[k][a]);
            }
        }
    velocity_from_tx<T, DIM, DEG>(tx, w, cref, vn);
}

}  // namespace apic
