// Transfer to particles (Sec. 3.4) in its lambda = 0 form (Sec. 5.7), with
// the weights of time n, fused with the re-binning of the particles:
//   v_p = sum_i w_ip vt_i
//   B_p = sum_i w_ip vt_i (x_i - x_p)^T
//   F_p = (I + dt sum_i vt_i grad w_ip^T) F_p
//   x_p = x_p + dt v_p          (cell index + offset)
// Both passes walk the listed tiles of the current layout, one wavefront per
// tile and one lane per key, through the key's particles level by level.
// Pass 1 (k_bin_keys_moved) finds every particle's new key: a particle whose
// key does not change ("stayer") only adds to its key's stayer count; one
// that changes key ("mover", rare) takes a rank in its new key by a counter.
// Pass 2 (k_g2p) stages the grid velocities around the tile in LDS, computes
// the whole update and writes each particle at its place in the new layout
// (movers first within a key, then stayers in their old order).  Both passes
// get the new position through the same fixed operation sequence (no
// contraction freedom), so they agree bit for bit on every key.
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

// New velocity v = sum_i w_i vt_i with a fixed operation sequence, shared
// by both passes: first the x-axis sums Tx_k(a) = sum_{c,b} (wy(b) wz(c))
// vt_k(a,b,c), nodes in (c, b) order, then v_k = sum_a wx(a) Tx_k(a).
template <typename T, int DIM, int DEG>
__device__ __forceinline__ void velocity_from_tx(const T (&tx)[DIM][DEG + 1], const T (&w)[DIM][DEG + 1], T *vn) {
#pragma clang fp contract(off)
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        vn[k] = T(0);
#pragma unroll
        for (int a = 0; a < DEG + 1; ++a) vn[k] = fma_t(w[0][a], tx[k][a], vn[k]);
    }
}

// Pass 1: x-axis sums from support-node velocities held in registers.
template <typename T, int DIM, int DEG>
__device__ __forceinline__ void gather_velocity(const T (&vt)[Geo<DIM, DEG>::NODES][DIM], const T (&w)[DIM][DEG + 1],
                                                T *vn) {
#pragma clang fp contract(off)
    constexpr int K = DEG + 1;
    T tx[DIM][K];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int a = 0; a < K; ++a) tx[k][a] = T(0);
#pragma unroll
    for (int c = 0; c < (DIM == 3 ? K : 1); ++c)
#pragma unroll
        for (int b = 0; b < K; ++b) {
            const T wyz = DIM == 3 ? w[1][b] * w[2][c] : w[1][b];
#pragma unroll
            for (int a = 0; a < K; ++a)
#pragma unroll
                for (int k = 0; k < DIM; ++k) tx[k][a] = fma_t(wyz, vt[a + K * (b + K * c)][k], tx[k][a]);
        }
    velocity_from_tx<T, DIM, DEG>(tx, w, vn);
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

// --- pass 1: new keys ---------------------------------------------------------------------
// One wavefront per listed tile walks the tile's particles in chunks of 64.
// A particle farther from every key boundary than this step can move keeps
// its key and only adds to its key's stayer count (LDS).  The others are
// queued in LDS and resolved 64 at a time with the gather, so the gather
// runs about once per tile instead of once per chunk.

// Base-node key, local index within its tile, of a particle at (ci, off).
template <typename T, int DIM, int DEG>
__device__ __forceinline__ int local_key(const int *ci, const T *off) {
    int base[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) base[a] = base_of<T, DEG>(ci[a], off[a]);
    return local_of<DIM>(base);
}

// Resolves queued particles lane < count: stayers add to their key's count,
// movers take a rank in their new key (or among the dead).  Wave-wide.
template <typename T, int DIM, int DEG>
__device__ __forceinline__ void resolve_near(const Parts<T> &P, const GridState<T> &g, const StepParams<T> &prm,
                                             const BinLists &nxt, const BinScratch &sc, const uint32_t *queue,
                                             uint32_t count, uint32_t t, uint32_t *stay) {
    const int lane = lane_id();
    const bool act = (uint32_t)lane < count;
    uint32_t nkey = kDeadKey, q = 0;
    bool mover = false;
    if (act) {
        q = queue[lane];
        int ci[3] = {0, 0, 0}, base[3] = {0, 0, 0}, cn[3] = {0, 0, 0};
        unpack_cell<DIM>(P.cell[q], ci);
        T off[DIM], w[DIM][DEG + 1], vn[DIM], on[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            off[a] = P.off[a * P.s + q];
            base[a] = axis_w_fixed<T, DEG>(ci[a], off[a], w[a]);
        }
        const uint32_t mykey = t * 64 + (uint32_t)local_of<DIM>(base);
        T vt[Geo<DIM, DEG>::NODES][DIM];
        load_support<T, DIM, DEG>(base, g, vt);
        gather_velocity<T, DIM, DEG>(vt, w, vn);
        bool cfl, finite;
        move_position<T, DIM>(ci, off, vn, prm.dt * g.inv_dx, cn, on, cfl);
        nkey = key_of<T, DIM, DEG>(cn, on, g.d, finite);
        if (nkey == kDeadKey) atomicOr(g.flags, finite ? FLAG_OUT_OF_DOMAIN : FLAG_NONFINITE);
        if (nkey == mykey)
            atomicAdd(stay + (mykey & 63u), 1u);
        else
            mover = true;
    }
    const uint32_t rank = bin_take_slot(nkey, mover, nxt, sc);
    if (mover) {
        sc.pkey[q] = nkey;
        sc.prank[q] = rank;
    }
}

template <typename T, int DIM, int DEG>
__device__ __forceinline__ void keys_body(const Parts<T> &P, const BinLists &cur, const TileTables &ctab,
                                          const GridState<T> &g, const StepParams<T> &prm, const BinLists &nxt,
                                          const BinScratch &sc, uint32_t blk, uint32_t nblk) {
    __shared__ uint32_t lds_stay[4][64];
    __shared__ uint32_t lds_queue[4][128];
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    uint32_t *stay = lds_stay[wv], *queue = lds_queue[wv];
    const TileWalk walk = tile_walk(cur);
    const T reach = step_reach<T>(wave_vmax(g.vmax), prm, g.inv_dx);
    const uint32_t items = walk.nrec + dead_chunks(P.n, walk.live);
    for (uint32_t r = blk * 4 + (uint32_t)wv; r < items; r += nblk * 4) {
        if (r >= walk.nrec) {
            // particles that could not be binned stay in the dead region
            const int64_t p = (int64_t)walk.live + (int64_t)(r - walk.nrec) * 64 + lane;
            if (p < P.n) sc.prank[p] = atomicAdd(nxt.dead, 1u);
            continue;
        }
        uint32_t start, total;
        const uint32_t t = tile_range(walk, r, cur, ctab, start, total);
        stay[lane] = 0u;
        wave_lds_sync();
        uint32_t queued = 0, c0 = 0;
        // cell and offset of the current chunk; the next chunk's are loaded
        // while this one is classified
        uint32_t cell = 0;
        T off[DIM];
        if ((uint32_t)lane < total) {
            cell = P.cell[start + lane];
#pragma unroll
            for (int a = 0; a < DIM; ++a) off[a] = P.off[a * P.s + start + lane];
        }
        for (;;) {
            if (c0 < total) {
                const uint32_t i = c0 + (uint32_t)lane;
                uint32_t cell_n = 0;
                T off_n[DIM];
                if (i + 64 < total) {
                    cell_n = P.cell[start + i + 64];
#pragma unroll
                    for (int a = 0; a < DIM; ++a) off_n[a] = P.off[a * P.s + start + i + 64];
                }
                bool near = false;
                if (i < total) {
                    int ci[3] = {0, 0, 0};
                    unpack_cell<DIM>(cell, ci);
                    if (keeps_key<T, DIM, DEG>(off, reach))
                        atomicAdd(stay + local_key<T, DIM, DEG>(ci, off), 1u);
                    else
                        near = true;
                }
                const uint64_t nm = ballot(near);
                if (near) queue[queued + (uint32_t)popc64(nm & lanes_below(lane))] = start + i;
                queued += (uint32_t)popc64(nm);
                cell = cell_n;
#pragma unroll
                for (int a = 0; a < DIM; ++a) off[a] = off_n[a];
            }
            c0 += 64;
            const bool read_all = c0 >= total;
            if (queued >= 64 || (read_all && queued > 0)) {
                // resolve up to 64 queued particles, keep the rest queued
                const uint32_t take = queued < 64 ? queued : 64u;
                wave_lds_sync();
                resolve_near<T, DIM, DEG>(P, g, prm, nxt, sc, queue, take, t, stay);
                const uint32_t rest = queued - take;
                const uint32_t moved = (uint32_t)lane < rest ? queue[64 + lane] : 0u;
                wave_lds_sync();
                if ((uint32_t)lane < rest) queue[lane] = moved;
                queued = rest;
            }
            if (read_all && queued == 0) break;
        }
        wave_lds_sync();
        const uint32_t s = stay[lane];
        sc.scount[t * 64 + (uint32_t)lane] = s;
        if (ballot(s > 0u) != 0ull && lane == 0) list_tile(t, nxt);
        wave_lds_sync();
    }
}

template <typename T, int DIM, int DEG>
__global__ __launch_bounds__(256) void k_bin_keys_moved(Parts<T> P, BinLists cur, TileTables ctab, GridState<T> g,
                                                        StepParams<T> prm, BinLists nxt, BinScratch sc) {
    keys_body<T, DIM, DEG>(P, cur, ctab, g, prm, nxt, sc, blockIdx.x, gridDim.x);
}

template <typename T, int DIM, int DEG>
__global__ __launch_bounds__(256) void k_bin_keys_moved_batch(const SceneDesc<T> *descs, const int32_t *start, int n,
                                                              int k) {
    const BatchStep<T> b = batch_step<T>(descs, start, n, k);
    const SceneDesc<T> &d = *b.d;
    keys_body<T, DIM, DEG>(d.bufs[b.sp.src], b.cur, d.tab[b.sp.cur], d.g, d.prm, b.nxt, d.sc, b.blk, b.nblk);
}

template <typename T, int DIM, int DEG>
void launch_bin_keys_moved_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, int blocks,
                                 hipStream_t st) {
    hipLaunchKernelGGL((k_bin_keys_moved_batch<T, DIM, DEG>), dim3((unsigned)blocks), dim3(256), 0, st, descs, start,
                       n, k);
}

template <typename T, int DIM, int DEG>
void launch_bin_keys_moved(const Parts<T> &P, const BinLists &cur, const TileTables &ctab, const GridState<T> &g,
                           const StepParams<T> &prm, const BinLists &nxt, const BinScratch &sc, int64_t max_records,
                           hipStream_t st) {
    int64_t blocks = (max_records + (P.n + 63) / 64 + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL((k_bin_keys_moved<T, DIM, DEG>), dim3((unsigned)blocks), dim3(256), 0, st, P, cur, ctab, g,
                       prm, nxt, sc);
}

// --- pass 2: the transfer, written to the new layout ------------------------------------
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
// SIMD); other variants are left to the compiler.
template <typename T, int DIM, int DEG>
constexpr int g2p_min_waves() {
    return (sizeof(T) == 4 && DEG == 2) ? 4 : 1;
}

// What G2P reads of a particle (loaded one chunk ahead of its use).
template <typename T, int DIM>
struct G2PRaw {
    uint32_t cell;
    int32_t id;
    T m, off[DIM], F[DIM * DIM];
};

template <typename T, int DIM>
__device__ __forceinline__ void g2p_load(const Parts<T> &src, uint32_t p, G2PRaw<T, DIM> &r) {
    const int64_t ss = src.s;
    const uint32_t pb = p * (uint32_t)sizeof(T);
    r.cell = src.cell[p];
    r.m = plane_at(src.m, pb);
    r.id = src.id ? plane_at(src.id, p * 4u) : 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) r.off[a] = plane_at(src.off + a * ss, pb);
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) r.F[k] = plane_at(src.F + k * ss, pb);
}

// One wavefront per listed tile walks the tile's particles in chunks of 64
// (every lane busy).  A stayer's rank in its key continues from the key's
// mover count (LDS counter); a mover takes the key and rank of pass 1.
template <typename T, int DIM, int DEG>
__device__ __forceinline__ void g2p_body(const Parts<T> &src, const Parts<T> &dst, const BinLists &cur,
                                         const TileTables &ctab, const BinLists &nxt, const TileTables &ntab,
                                         const BinScratch &sc, const GridState<T> &g, const StepParams<T> &prm,
                                         uint32_t blk, uint32_t nblk) {
    constexpr int K = DEG + 1;
    constexpr int TE = DIM == 3 ? 4 : 8;
    using R = VtRegion<DIM>;
    __shared__ T lds_vt[4 * DIM * R::SIZE];
    __shared__ uint32_t lds_rank[4][64];
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    T *reg = lds_vt + wv * (DIM * R::SIZE);
    uint32_t *rankc = lds_rank[wv];
    const TileWalk walk = tile_walk(cur);
    const uint32_t *bases = nxt.bpre;
    const uint32_t live_nxt = nxt.bpre[kBuckets];
    const T reach = step_reach<T>(wave_vmax(g.vmax), prm, g.inv_dx);
    const T dt_inv_dx = prm.dt * g.inv_dx, gs = prm.dt * g.inv_dx;
    const uint32_t items = walk.nrec + dead_chunks(src.n, walk.live);
    const int64_t ss = src.s, ds = dst.s;
    for (uint32_t r = blk * 4 + (uint32_t)wv; r < items; r += nblk * 4) {
        if (r >= walk.nrec) {
            // dead particles are carried over unchanged
            const int64_t p = (int64_t)walk.live + (int64_t)(r - walk.nrec) * 64 + lane;
            if (p < src.n) {
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
            continue;
        }
        uint32_t start, total;
        const uint32_t t = tile_range(walk, r, cur, ctab, start, total);
        int origin[3] = {0, 0, 0};
        tile_origin<DIM>(t, g.d.TN, origin);
        stage_velocities<T, DIM>(t, g, reg);
        // stayers of a key follow its movers in the new layout
        rankc[lane] = ntab.kmov[t * 64 + (uint32_t)lane];
        const uint32_t tbase = bases[bucket_of(t)];
        wave_lds_sync();
        G2PRaw<T, DIM> raw;
        if ((uint32_t)lane < total) g2p_load<T, DIM>(src, start + (uint32_t)lane, raw);
        for (uint32_t c0 = 0; c0 < total; c0 += 64) {
            const uint32_t i = c0 + (uint32_t)lane;
            // the next chunk is in flight while this one is computed
            G2PRaw<T, DIM> raw_n;
            if (i + 64 < total) g2p_load<T, DIM>(src, start + i + 64, raw_n);
            if (i < total) {
                const uint32_t p = start + i;
                int ci[3] = {0, 0, 0}, cn[3] = {0, 0, 0}, lk[3] = {0, 0, 0};
                unpack_cell<DIM>(raw.cell, ci);
                T off[DIM], wf[DIM][K], on[DIM], vn[DIM], Bc[DIM * DIM], Fn[DIM * DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    off[a] = raw.off[a];
                    lk[a] = axis_w_fixed<T, DEG>(ci[a], off[a], wf[a]) - origin[a];
                }
                // One sweep over the support nodes (c, b, a) from LDS: the
                // axis-pair sums Tx_k(a) = sum_{b,c} wy wz vt_k (in the
                // sequence of pass 1), Ty_k(b) = sum_{a,c} wx wz vt_k and
                // Tz_k(c) = sum_{a,b} wx wy vt_k, from which
                //   v_k = sum_a wx Tx_k(a),
                //   B_k0 = sum_a wx rx Tx_k(a), grad v_k0 = sum_a dwx Tx_k(a),
                // and likewise along y and z.
                T Tx[DIM][K], Ty[DIM][K], Tz[DIM][K];
#pragma unroll
                for (int k = 0; k < DIM; ++k)
#pragma unroll
                    for (int ii = 0; ii < K; ++ii) Tx[k][ii] = Ty[k][ii] = Tz[k][ii] = T(0);
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
                                    const T x = reg[k * R::SIZE + idx];
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
                velocity_from_tx<T, DIM, DEG>(Tx, wf, vn);
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
                move_position<T, DIM>(ci, off, vn, dt_inv_dx, cn, on, cfl);
                if (cfl) atomicOr(g.flags, FLAG_CFL);
                const uint32_t mykey = t * 64 + (uint32_t)local_of<DIM>(lk);
                bool stays = keeps_key<T, DIM, DEG>(off, reach);
                if (!stays) {
                    bool finite;
                    stays = key_of<T, DIM, DEG>(cn, on, g.d, finite) == mykey;
                }
                uint32_t dkey, drank, base;
                if (stays) {
                    dkey = mykey;
                    drank = atomicAdd(rankc + (mykey & 63u), 1u);
                    base = tbase;
                } else {
                    dkey = sc.pkey[p];
                    drank = sc.prank[p];
                    base = bucket_base_of(dkey, bases);
                }
                const uint32_t q = bin_destination(dkey, drank, ntab, base, live_nxt);
                // keep the packed index representable; a particle that left
                // the grid is in the dead region and is not transferred again
#pragma unroll
                for (int a = 0; a < DIM; ++a) cn[a] = cn[a] < 0 ? 0 : (cn[a] > g.d.n[a] - 1 ? g.d.n[a] - 1 : cn[a]);
                const uint32_t qb = q * (uint32_t)sizeof(T), q4 = q * 4u;
                plane_at(dst.cell, q4) = pack_cell<DIM>(cn);
                plane_at(dst.m, qb) = raw.m;
                if (src.id) plane_at(dst.id, q4) = raw.id;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    plane_at(dst.off + a * ds, qb) = on[a];
                    plane_at(dst.v + a * ds, qb) = vn[a];
                }
#pragma unroll
                for (int k = 0; k < DIM * DIM; ++k) {
                    plane_at(dst.B + k * ds, qb) = Bc[k] * g.dx;
                    plane_at(dst.F + k * ds, qb) = Fn[k];
                }
            }
            raw = raw_n;
        }
        wave_lds_sync();
    }
    (void)TE;
}

template <typename T, int DIM, int DEG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(g2p_min_waves<T, DIM, DEG>()))) void k_g2p(
    Parts<T> src, Parts<T> dst, BinLists cur, TileTables ctab, BinLists nxt, TileTables ntab, BinScratch sc,
    GridState<T> g, StepParams<T> prm) {
    g2p_body<T, DIM, DEG>(src, dst, cur, ctab, nxt, ntab, sc, g, prm, blockIdx.x, gridDim.x);
}

template <typename T, int DIM, int DEG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(g2p_min_waves<T, DIM, DEG>()))) void k_g2p_batch(
    const SceneDesc<T> *descs, const int32_t *start, int n, int k) {
    const BatchStep<T> b = batch_step<T>(descs, start, n, k);
    const SceneDesc<T> &d = *b.d;
    Parts<T> src = d.bufs[b.sp.src], dst = d.bufs[b.sp.src ^ 1];
    if (!src.id || !dst.id) src.id = dst.id = nullptr;
    g2p_body<T, DIM, DEG>(src, dst, b.cur, d.tab[b.sp.cur], b.nxt, d.tab[b.sp.nxt], d.sc, d.g, d.prm, b.blk, b.nblk);
}

template <typename T, int DIM, int DEG>
void launch_g2p_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, int blocks, hipStream_t st) {
    hipLaunchKernelGGL((k_g2p_batch<T, DIM, DEG>), dim3((unsigned)blocks), dim3(256), 0, st, descs, start, n, k);
}

template <typename T, int DIM, int DEG>
void launch_g2p(const Parts<T> &src, const Parts<T> &dst, const BinLists &cur, const TileTables &ctab,
                const BinLists &nxt, const TileTables &ntab, const BinScratch &sc, const GridState<T> &g,
                const StepParams<T> &prm, int64_t max_records, hipStream_t st) {
    if (src.n == 0) return;
    Parts<T> s2 = src, d2 = dst;
    if (!src.id || !dst.id) s2.id = d2.id = nullptr;
    int64_t blocks = (max_records + (src.n + 63) / 64 + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_g2p<T, DIM, DEG>), dim3((unsigned)blocks), dim3(256), 0, st, s2, d2, cur, ctab, nxt, ntab,
                       sc, g, prm);
}

#define APIC_G2P_INST(T, DIM, DEG)                                                                               \
    template void launch_bin_keys_moved_batch<T, DIM, DEG>(const SceneDesc<T> *, const int32_t *, int, int, int,  \
                                                           hipStream_t);                                          \
    template void launch_g2p_batch<T, DIM, DEG>(const SceneDesc<T> *, const int32_t *, int, int, int,             \
                                                hipStream_t);                                                     \
    template void launch_bin_keys_moved<T, DIM, DEG>(const Parts<T> &, const BinLists &, const TileTables &,     \
                                                     const GridState<T> &, const StepParams<T> &,                \
                                                     const BinLists &, const BinScratch &, int64_t, hipStream_t); \
    template void launch_g2p<T, DIM, DEG>(const Parts<T> &, const Parts<T> &, const BinLists &,                  \
                                          const TileTables &, const BinLists &, const TileTables &,              \
                                          const BinScratch &, const GridState<T> &, const StepParams<T> &,       \
                                          int64_t, hipStream_t);
APIC_G2P_INST(float, 2, 2)
APIC_G2P_INST(float, 2, 3)
APIC_G2P_INST(float, 3, 2)
APIC_G2P_INST(float, 3, 3)
APIC_G2P_INST(double, 2, 2)
APIC_G2P_INST(double, 2, 3)
APIC_G2P_INST(double, 3, 2)
APIC_G2P_INST(double, 3, 3)

}  // namespace apic
