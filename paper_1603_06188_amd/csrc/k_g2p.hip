// Transfer to particles (Sec. 3.4) in its lambda = 0 form (Sec. 5.7), with
// the weights of time n, fused with the re-binning of the particles:
//   v_p = sum_i w_ip vt_i
//   B_p = sum_i w_ip vt_i (x_i - x_p)^T
//   F_p = (I + dt sum_i vt_i grad w_ip^T) F_p
//   x_p = x_p + dt v_p          (cell index + offset)
// Pass 1 (k_bin_keys_moved) computes every particle's new position to find
// its new key and rank; pass 2 (k_g2p) computes the whole update and writes
// the particle at its place in the new layout.  Both passes get the new
// position from `advect`, whose operation sequence is fixed (no contraction
// freedom), so the two agree bit for bit.
#include "apic_bin_device.h"
#include "apic_kernels.h"

namespace apic {

// Weights along one axis with a fixed operation sequence (see axis_weights).
template <typename T, int DEG>
__device__ __forceinline__ int axis_w_fixed(int cell, T off, T *w) {
#pragma clang fp contract(off)
    if constexpr (DEG == 2) {
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

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Support-node velocities of a particle: vt[node][k], node = a + K (b + K c).
template <typename T, int DIM, int DEG>
__device__ __forceinline__ void load_support(const int *base, const GridState<T> &g,
                                             T (&vt)[Geo<DIM, DEG>::NODES][DIM]) {
    constexpr int K = DEG + 1;
    const int64_t G = g.d.G;
#pragma unroll
    for (int c = 0; c < (DIM == 3 ? K : 1); ++c)
#pragma unroll
        for (int b = 0; b < K; ++b)
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const int nc[3] = {base[0] + a, base[1] + b, DIM == 3 ? base[2] + c : 0};
                const int64_t i = node_index<DIM>(nc, g.d.TN);
#pragma unroll
                for (int k = 0; k < DIM; ++k) vt[a + K * (b + K * c)][k] = g.vt[k * G + i];
            }
}

// New velocity sum_i w vt_i and position x + dt v, fixed operation order.
template <typename T, int DIM, int DEG>
__device__ __forceinline__ void advect(const int *ci, const T *off, const T (&vt)[Geo<DIM, DEG>::NODES][DIM],
                                       const T (&w)[DIM][DEG + 1], T dt_inv_dx, T *vn, int *cn, T *on,
                                       bool &cfl) {
#pragma clang fp contract(off)
    constexpr int K = DEG + 1;
#pragma unroll
    for (int k = 0; k < DIM; ++k) vn[k] = T(0);
#pragma unroll
    for (int c = 0; c < (DIM == 3 ? K : 1); ++c)
#pragma unroll
        for (int b = 0; b < K; ++b) {
            const T wyz = DIM == 3 ? w[1][b] * w[2][c] : w[1][b];
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const T wn = w[0][a] * wyz;
#pragma unroll
                for (int k = 0; k < DIM; ++k) vn[k] = fma_t(wn, vt[a + K * (b + K * c)][k], vn[k]);
            }
        }
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

// Bound of max_i |vt_i| over the slots the grid update raised (wave-wide).
__device__ __forceinline__ float wave_vmax(const uint32_t *slots) {
    return __uint_as_float(wave_max_u32(slots[lane_id() & (kVmaxSlots - 1)]));
}

// --- pass 1: keys at the advected positions -----------------------------------------
template <typename T, int DIM, int DEG>
__global__ __launch_bounds__(256) void k_bin_keys_moved(Parts<T> P, BinLists cur, GridState<T> g, StepParams<T> prm,
                                                        BinLists nxt, BinScratch sc) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = p < P.n;
    // particles at or beyond the live total of the current layout are dead
    uint32_t live_cur, unused;
    (void)wave_bucket_prefix(cur.tot, live_cur, unused);
    // Largest displacement this step in cell units, with a margin for
    // rounding: |v_p| <= max_i |vt_i| since the weights are a partition of
    // unity.  A particle farther than that from every boundary where its
    // base node changes (offset 1/2 for quadratic, offset 0 or 1 for cubic)
    // keeps its key; only the others need the gather.
    const float vbound = wave_vmax(g.vmax);
    const T reach = (T)vbound * prm.dt * g.inv_dx * T(1.0001) + T(1e-6);
    uint32_t key = kDeadKey;
    if (active && p < (int64_t)live_cur) {
        int ci[3] = {0, 0, 0}, base[3] = {0, 0, 0}, cn[3] = {0, 0, 0};
        unpack_cell<DIM>(P.cell[p], ci);
        T off[DIM], w[DIM][DEG + 1], on[DIM], vn[DIM];
        bool far = reach < T(0.5);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            off[a] = P.off[a * P.s + p];
            const T dist = DEG == 2 ? (off[a] < T(0.5) ? T(0.5) - off[a] : off[a] - T(0.5))
                                    : (off[a] < T(0.5) ? off[a] : T(1) - off[a]);
            far = far && dist > reach;
        }
        bool finite;
        if (far) {
            key = key_of<T, DIM, DEG>(ci, off, g.d, finite);
        } else {
#pragma unroll
            for (int a = 0; a < DIM; ++a) base[a] = axis_w_fixed<T, DEG>(ci[a], off[a], w[a]);
            T vt[Geo<DIM, DEG>::NODES][DIM];
            load_support<T, DIM, DEG>(base, g, vt);
            bool cfl;
            advect<T, DIM, DEG>(ci, off, vt, w, prm.dt * g.inv_dx, vn, cn, on, cfl);
            key = key_of<T, DIM, DEG>(cn, on, g.d, finite);
        }
        if (key == kDeadKey) atomicOr(g.flags, finite ? FLAG_OUT_OF_DOMAIN : FLAG_NONFINITE);
    }
    const uint32_t rank = bin_take_slot(key, active, nxt, sc);
    if (active) {
        sc.pkey[p] = key;
        sc.prank[p] = rank;
    }
}

template <typename T, int DIM, int DEG>
void launch_bin_keys_moved(const Parts<T> &P, const BinLists &cur, const GridState<T> &g, const StepParams<T> &prm,
                           const BinLists &nxt, const BinScratch &sc, hipStream_t st) {
    if (P.n == 0) return;
    hipLaunchKernelGGL((k_bin_keys_moved<T, DIM, DEG>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P,
                       cur, g, prm, nxt, sc);
}

// --- pass 2: the transfer, written to the new layout ----------------------------------
template <typename T, int DIM, int DEG>
__global__ __launch_bounds__(256) void k_g2p(Parts<T> src, Parts<T> dst, BinLists cur, BinLists nxt, TileTables tab,
                                             BinScratch sc, GridState<T> g, StepParams<T> prm) {
    constexpr int K = DEG + 1;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = p < src.n;
    uint32_t live_cur, live_nxt, unused;
    (void)wave_bucket_prefix(cur.tot, live_cur, unused);
    const uint32_t bbase = wave_bucket_prefix(nxt.tot, live_nxt, unused);
    const uint32_t key = active ? sc.pkey[p] : kDeadKey;
    const uint32_t rank = active ? sc.prank[p] : 0u;
    const int64_t q = bin_destination(key, rank, tab, bbase, live_nxt);
    if (!active) return;
    const int64_t ss = src.s, ds = dst.s;
    dst.m[q] = src.m[p];
    if (src.id) dst.id[q] = src.id[p];
    if (p >= (int64_t)live_cur) {
        dst.cell[q] = src.cell[p];
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
        return;
    }
    int ci[3] = {0, 0, 0}, base[3] = {0, 0, 0}, cn[3] = {0, 0, 0};
    unpack_cell<DIM>(src.cell[p], ci);
    T off[DIM], wf[DIM][K], on[DIM], vn[DIM], F[DIM * DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        off[a] = src.off[a * ss + p];
        base[a] = axis_w_fixed<T, DEG>(ci[a], off[a], wf[a]);
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) F[k] = src.F[k * ss + p];
    T vt[Geo<DIM, DEG>::NODES][DIM];
    load_support<T, DIM, DEG>(base, g, vt);
    bool cfl;
    advect<T, DIM, DEG>(ci, off, vt, wf, prm.dt * g.inv_dx, vn, cn, on, cfl);
    if (cfl) atomicOr(g.flags, FLAG_CFL);

    // B (cell units) and grad v (1/cell) from the tensor-product weights
    Axis<T, DEG> ax[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) axis_weights<T, DEG>(ci[a], off[a], ax[a]);
    T Bc[DIM * DIM], Gc[DIM * DIM];
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) Bc[k] = Gc[k] = T(0);
    // Axis-pair grouping: with Tx_k(a) = sum_{b,c} wy wz vt, Ty_k(b) =
    // sum_{a,c} wx wz vt, Tz_k(c) = sum_{a,b} wx wy vt (three multiply-adds
    // per node and component),
    //   B_k0 = sum_a wx rx Tx_k(a),  grad v_k0 = sum_a dx Tx_k(a), and the
    // same along y with Ty and along z with Tz.
    if constexpr (DIM == 3) {
        T Pyz[K][K], Qxz[K][K], Rxy[K][K];
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                Pyz[i][j] = ax[1].w[i] * ax[2].w[j];
                Qxz[i][j] = ax[0].w[i] * ax[2].w[j];
                Rxy[i][j] = ax[0].w[i] * ax[1].w[j];
            }
        T Tx[3][K], Ty[3][K], Tz[3][K];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < K; ++i) Tx[k][i] = Ty[k][i] = Tz[k][i] = T(0);
#pragma unroll
        for (int c = 0; c < K; ++c)
#pragma unroll
            for (int b = 0; b < K; ++b)
#pragma unroll
                for (int a = 0; a < K; ++a)
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const T x = vt[a + K * (b + K * c)][k];
                        Tx[k][a] += Pyz[b][c] * x;
                        Ty[k][b] += Qxz[a][c] * x;
                        Tz[k][c] += Rxy[a][b] * x;
                    }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const T wrx = ax[0].w[i] * ax[0].r[i], wry = ax[1].w[i] * ax[1].r[i], wrz = ax[2].w[i] * ax[2].r[i];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                Bc[k * 3 + 0] += wrx * Tx[k][i];
                Gc[k * 3 + 0] += ax[0].dw[i] * Tx[k][i];
                Bc[k * 3 + 1] += wry * Ty[k][i];
                Gc[k * 3 + 1] += ax[1].dw[i] * Ty[k][i];
                Bc[k * 3 + 2] += wrz * Tz[k][i];
                Gc[k * 3 + 2] += ax[2].dw[i] * Tz[k][i];
            }
        }
    } else {
        T Tx[2][K], Ty[2][K];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int i = 0; i < K; ++i) Tx[k][i] = Ty[k][i] = T(0);
#pragma unroll
        for (int b = 0; b < K; ++b)
#pragma unroll
            for (int a = 0; a < K; ++a)
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const T x = vt[a + K * b][k];
                    Tx[k][a] += ax[1].w[b] * x;
                    Ty[k][b] += ax[0].w[a] * x;
                }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const T wrx = ax[0].w[i] * ax[0].r[i], wry = ax[1].w[i] * ax[1].r[i];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                Bc[k * 2 + 0] += wrx * Tx[k][i];
                Gc[k * 2 + 0] += ax[0].dw[i] * Tx[k][i];
                Bc[k * 2 + 1] += wry * Ty[k][i];
                Gc[k * 2 + 1] += ax[1].dw[i] * Ty[k][i];
            }
        }
    }
    // F <- (I + dt grad v) F, grad v = Gc / dx
    const T gs = prm.dt * g.inv_dx;
    T Fn[DIM * DIM];
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc += Gc[r * DIM + k] * F[k * DIM + c];
            Fn[r * DIM + c] = F[r * DIM + c] + gs * acc;
        }
    // keep the packed index representable; a particle that left the grid is
    // in the dead region of the new layout and is not transferred again
#pragma unroll
    for (int a = 0; a < DIM; ++a) cn[a] = cn[a] < 0 ? 0 : (cn[a] > g.d.n[a] - 1 ? g.d.n[a] - 1 : cn[a]);
    dst.cell[q] = pack_cell<DIM>(cn);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        dst.off[a * ds + q] = on[a];
        dst.v[a * ds + q] = vn[a];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        dst.B[k * ds + q] = Bc[k] * g.dx;
        dst.F[k * ds + q] = Fn[k];
    }
}

template <typename T, int DIM, int DEG>
void launch_g2p(const Parts<T> &src, const Parts<T> &dst, const BinLists &cur, const BinLists &nxt,
                const TileTables &tab, const BinScratch &sc, const GridState<T> &g, const StepParams<T> &prm,
                hipStream_t st) {
    if (src.n == 0) return;
    Parts<T> s2 = src, d2 = dst;
    if (!src.id || !dst.id) s2.id = d2.id = nullptr;
    hipLaunchKernelGGL((k_g2p<T, DIM, DEG>), dim3((unsigned)((src.n + 255) / 256)), dim3(256), 0, st, s2, d2, cur, nxt,
                       tab, sc, g, prm);
}

#define APIC_G2P_INST(T, DIM, DEG)                                                                               \
    template void launch_bin_keys_moved<T, DIM, DEG>(const Parts<T> &, const BinLists &, const GridState<T> &,   \
                                                     const StepParams<T> &, const BinLists &, const BinScratch &, \
                                                     hipStream_t);                                               \
    template void launch_g2p<T, DIM, DEG>(const Parts<T> &, const Parts<T> &, const BinLists &, const BinLists &, \
                                          const TileTables &, const BinScratch &, const GridState<T> &,          \
                                          const StepParams<T> &, hipStream_t);
APIC_G2P_INST(float, 2, 2)
APIC_G2P_INST(float, 2, 3)
APIC_G2P_INST(float, 3, 2)
APIC_G2P_INST(float, 3, 3)
APIC_G2P_INST(double, 2, 2)
APIC_G2P_INST(double, 2, 3)
APIC_G2P_INST(double, 3, 2)
APIC_G2P_INST(double, 3, 3)

}  // namespace apic
