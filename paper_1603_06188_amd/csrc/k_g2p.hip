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
// (within a key the stayers first, in their old order, then the movers that
// entered it).  Both passes get the new position through the same fixed
// operation sequence (no contraction freedom), so they agree bit for bit on
// every key.
#include "apic_kernels.h"
#include "g2p_device.h"

namespace apic {

// --- pass 1: new keys ---------------------------------------------------------------------
// One wavefront per listed tile loads the tile's particles in groups of
// kKeyChunks chunks of 64 (all loads of a group in flight together).  A
// particle farther from every key boundary than this step can move keeps its
// key and only adds to its key's stayer count (LDS).  The others are queued
// in LDS and resolved 64 at a time from the grid velocities around the tile,
// staged in LDS when the tile first needs them.

// Base-node key, local index within its tile, of a particle at (ci, off).
template <typename T, int DIM, int DEG>
__device__ __forceinline__ int local_key(const int *ci, const T *off) {
    int base[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) base[a] = base_of<T, DEG>(ci[a], off[a]);
    return local_of<DIM>(base);
}

// Resolves queued particles lane < count: stayers add to their key's count,
// movers take a rank in their new key (or among the dead).  The grid
// velocities around tile t (first node `origin`) are staged in `reg`.
// Wave-wide.
template <typename T, int DIM, int DEG, bool ABS>
__device__ __forceinline__ void resolve_near(const Parts<T> &P, const GridState<T> &g, const StepParams<T> &prm,
                                             const BinLists &nxt, const BinScratch &sc, const uint32_t *queue,
                                             uint32_t count, uint32_t t, uint32_t start, const int *origin,
                                             const T *reg, uint32_t *stay) {
    const int lane = lane_id();
    const bool act = (uint32_t)lane < count;
    uint32_t nkey = kDeadKey, q = 0;
    bool mover = false;
    if (act) {
        q = queue[lane];
        int ci[3] = {0, 0, 0}, base[3] = {0, 0, 0}, lk[3] = {0, 0, 0}, cn[3] = {0, 0, 0};
        T x[DIM], off[DIM], w[DIM][DEG + 1], vn[DIM], on[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) x[a] = P.off[a * P.s + q];
        particle_cells<T, DIM, ABS>(ABS ? 0u : P.cell[q], x, g.inv_dx, ci, off);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            base[a] = axis_w_fixed<T, DEG>(ci[a], off[a], w[a]);
            lk[a] = base[a] - origin[a];
        }
        const uint32_t mykey = t * 64 + (uint32_t)local_of<DIM>(base);
        velocity_lds<T, DIM, DEG>(reg, lk, w, vn);
        bool cfl, finite;
        if constexpr (ABS) {
            T xn[DIM];
            move_absolute<T, DIM>(x, vn, prm.dt, g.inv_dx, xn, cn, on, cfl);
        } else {
            move_position<T, DIM>(ci, off, vn, prm.dt * g.inv_dx, cn, on, cfl);
        }
        nkey = key_of<T, DIM, DEG>(cn, on, g.d, finite);
        if (nkey == kDeadKey) atomicOr(g.flags, finite ? FLAG_OUT_OF_DOMAIN : FLAG_NONFINITE);
        if (nkey == mykey)
            atomicAdd(stay + (mykey & 63u), 1u);
        else
            mover = true;
    }
    const uint32_t rank = bin_take_slot(nkey, mover, q, tile_order(t, q - start), nxt, sc);
    if (mover) {
        sc.pkey[q] = nkey;
        sc.prank[q] = rank;
    }
}

template <typename T, int DIM, int DEG, bool ABS>
__device__ __forceinline__ void keys_body(const Parts<T> &P, const BinLists &cur, const TileTables &ctab,
                                          const GridState<T> &g, const StepParams<T> &prm_in, const BinLists &nxt,
                                          const BinScratch &sc, uint32_t blk, uint32_t nblk) {
    const StepParams<T> prm = with_step_dt(prm_in);
    using R = VtRegion<DIM>;
    __shared__ uint32_t lds_stay[4][64];
    __shared__ uint32_t lds_queue[4][64 * kKeyChunks];
    __shared__ T lds_vt[4 * DIM * R::SIZE];
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    uint32_t *stay = lds_stay[wv], *queue = lds_queue[wv];
    T *reg = lds_vt + wv * (DIM * R::SIZE);
    const TileWalk walk = tile_walk(cur);
    const T reach = step_reach<T>(wave_vmax(g.vmax), prm, g.inv_dx);
    const uint32_t items = walk.nrec + dead_chunks(P.n, walk.live);
    for (uint32_t r = blk * 4 + (uint32_t)wv; r < items; r += nblk * 4) {
        if (r >= walk.nrec) {
            // particles that could not be binned stay in the dead region
            const int64_t p = (int64_t)walk.live + (int64_t)(r - walk.nrec) * 64 + lane;
            if (p < P.n) sc.prank[p] = atomicAdd(nxt.ctr + kCtrDead, 1u);
            continue;
        }
        uint32_t start, total;
        const uint32_t t = tile_range(walk, r, cur, ctab, start, total);
        int origin[3] = {0, 0, 0};
        tile_origin<DIM>(t, g.d.TN, origin);
        bool staged = false;  // grid velocities around the tile, on first use
        stay[lane] = 0u;
        // the tile is claimed in the new layout now (its particles nearly all
        // stay) and appended at the end, so the claim's round trip overlaps
        // the tile's loads; a tile all of whose particles leave is listed
        // empty, which every later pass walks as a tile without particles
        uint32_t claim = nxt.gen;
        if (lane == 0 && total > 0u) claim = atomicExch(nxt.tile_gen + t, nxt.gen);
        wave_lds_sync();
        uint32_t queued = 0;
        // groups of kKeyChunks chunks of 64: every load of a group is in
        // flight at once, then its chunks are classified in order
        for (uint32_t g0 = 0; g0 < total; g0 += 64u * kKeyChunks) {
            uint32_t cell[kKeyChunks];
            T off[kKeyChunks][DIM];
#pragma unroll
            for (int u = 0; u < kKeyChunks; ++u) {
                const uint32_t i = g0 + 64u * u + (uint32_t)lane;
                cell[u] = 0u;
                if (i < total) {
                    if constexpr (!ABS) cell[u] = P.cell[start + i];
#pragma unroll
                    for (int a = 0; a < DIM; ++a) off[u][a] = P.off[a * P.s + start + i];
                }
            }
#pragma unroll
            for (int u = 0; u < kKeyChunks; ++u) {
                const uint32_t i = g0 + 64u * u + (uint32_t)lane;
                if (g0 + 64u * u >= total) break;
                bool near = false;
                if (i < total) {
                    int ci[3] = {0, 0, 0};
                    T o[DIM];
                    particle_cells<T, DIM, ABS>(cell[u], off[u], g.inv_dx, ci, o);
                    if (keeps_key<T, DIM, DEG>(o, reach))
                        atomicAdd(stay + local_key<T, DIM, DEG>(ci, o), 1u);
                    else
                        near = true;
                }
                const uint64_t nm = ballot(near);
                if (near) queue[queued + (uint32_t)popc64(nm & lanes_below(lane))] = start + i;
                queued += (uint32_t)popc64(nm);
            }
            // the group's queued particles, 64 at a time
            for (uint32_t q0 = 0; q0 < queued; q0 += 64u) {
                if (!staged) {
                    stage_velocities<T, DIM>(t, g, reg);
                    staged = true;
                }
                wave_lds_sync();
                const uint32_t take = queued - q0 < 64u ? queued - q0 : 64u;
                resolve_near<T, DIM, DEG, ABS>(P, g, prm, nxt, sc, queue + q0, take, t, start, origin, reg, stay);
            }
            queued = 0;
            wave_lds_sync();
        }
        wave_lds_sync();
        const uint32_t s = stay[lane];
        sc.scount[t * 64 + (uint32_t)lane] = s;
        if (lane == 0 && claim != nxt.gen) append_tile(t, nxt);
        wave_lds_sync();
    }
}

// Three waves per SIMD (at most 168 VGPRs) for binary32 3D quadratic, whose
// resolve loop otherwise takes 170 VGPRs (two waves): the latency of the
// queue's LDS traffic needs the third wave.  The other variants are left to
// the compiler (the hint slowed the cubic pass by 40 % at the same occupancy).
template <typename T, int DIM, int DEG>
constexpr int keys_min_waves() {
    return (sizeof(T) == 4 && DIM == 3 && DEG == 2) ? 3 : 1;
}

template <typename T, int DIM, int DEG, bool ABS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(keys_min_waves<T, DIM, DEG>()))) void k_bin_keys_moved(
    Parts<T> P, BinLists cur, TileTables ctab, GridState<T> g, StepParams<T> prm, BinLists nxt, BinScratch sc) {
    keys_body<T, DIM, DEG, ABS>(P, cur, ctab, g, prm, nxt, sc, blockIdx.x, gridDim.x);
}

template <typename T, int DIM, int DEG, bool QUEUE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QUEUE ? 1 : keys_min_waves<T, DIM, DEG>()))) void k_bin_keys_moved_batch(
    const SceneDesc<T> *descs, const int32_t *start, int n, int k, BatchQueue q) {
    batch_items<QUEUE>(q, [&](uint32_t it) {
        const BatchStep<T> b = batch_step<T>(descs, start, n, k, it);
        const SceneDesc<T> &d = *b.d;
        // the scene's structs as values: read through the table they would be
        // read again after every store the compiler cannot prove apart
        const Parts<T> P = d.bufs[b.sp.src];
        const TileTables ctab = d.tab[b.sp.cur];
        const GridState<T> g = d.g;
        const StepParams<T> prm = d.prm;
        const BinScratch sc = d.sc;
        keys_body<T, DIM, DEG, false>(P, b.cur, ctab, g, prm, b.nxt, sc, b.blk, b.nblk);
    });
}

template <typename T, int DIM, int DEG>
void launch_bin_keys_moved_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, const BatchQueue &q,
                                 int blocks, hipStream_t st) {
    if (q.ctr)
        hipLaunchKernelGGL((k_bin_keys_moved_batch<T, DIM, DEG, true>), dim3((unsigned)blocks), dim3(256), 0, st,
                           descs, start, n, k, q);
    else
        hipLaunchKernelGGL((k_bin_keys_moved_batch<T, DIM, DEG, false>), dim3((unsigned)blocks), dim3(256), 0, st,
                           descs, start, n, k, q);
}

template <typename T, int DIM, int DEG, bool ABS>
void launch_bin_keys_moved(const Parts<T> &P, const BinLists &cur, const TileTables &ctab, const GridState<T> &g,
                           const StepParams<T> &prm, const BinLists &nxt, const BinScratch &sc, int64_t max_records,
                           hipStream_t st) {
    int64_t blocks = (max_records + (P.n + 63) / 64 + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL((k_bin_keys_moved<T, DIM, DEG, ABS>), dim3((unsigned)blocks), dim3(256), 0, st, P, cur, ctab,
                       g, prm, nxt, sc);
}

// --- pass 2: the transfer, written to the new layout ------------------------------------
// One wavefront per listed tile walks the tile's particles in chunks of 64
// (every lane busy).  A stayer's rank in its key comes from an LDS counter
// from 0; a mover takes the key of pass 1 and its rank there after the key's
// stayers.
// ADAPT: the step's dt comes from the device and the CFL bound of the
// written state is folded into g.cfl (adaptive steps); a separate
// instantiation, so that fixed steps carry none of it.
template <typename T, int DIM, int DEG, bool ADAPT, bool ABS = false>
__device__ __forceinline__ void g2p_body(const Parts<T> &src, const Parts<T> &dst, const BinLists &cur,
                                         const TileTables &ctab, const BinLists &nxt, const TileTables &ntab,
                                         const BinScratch &sc, const GridState<T> &g, const StepParams<T> &prm_in,
                                         uint32_t blk, uint32_t nblk) {
    const StepParams<T> prm = ADAPT ? with_step_dt(prm_in) : prm_in;
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
    T cmax = T(0);  // CFL bound of the particles this lane writes (when asked)
    for (uint32_t r = blk * 4 + (uint32_t)wv; r < items; r += nblk * 4) {
        if (r >= walk.nrec) {
            carry_dead<T, DIM>(src, dst, sc, walk.live, live_nxt, r - walk.nrec);
            continue;
        }
        uint32_t start, total;
        const uint32_t t = tile_range(walk, r, cur, ctab, start, total);
        int origin[3] = {0, 0, 0};
        tile_origin<DIM>(t, g.d.TN, origin);
        // chunks of 64 start on 32-particle boundaries (128 B in binary32)
        // of the tile's place in the new layout: the particles keep their
        // order there up to the few that change key, so each chunk writes
        // whole cache lines (the writes move twice the bytes of the reads,
        // which now start mid-line), and the next step's transfer to grid
        // reads lines written whole.  The first chunk is in flight while the
        // grid velocities are staged.
        const uint32_t head = (nxt.bpre[bucket_of(t)] + ntab.off[t]) & 31u, span = total + head,
                       first = start - head;
        G2PRaw<T, DIM> raw;
        if ((uint32_t)lane >= head && (uint32_t)lane < span) g2p_load<T, DIM, ABS>(src, first + (uint32_t)lane, raw);
        stage_velocities<T, DIM>(t, g, reg);
        // a key's stayers keep their levels in the new layout: they take the
        // first ranks, the movers entering the key the ranks after them
        rankc[lane] = 0u;
        const uint32_t tbase = bases[bucket_of(t)];
        wave_lds_sync();
        for (uint32_t c0 = 0; c0 < span; c0 += 64) {
            const uint32_t e = c0 + (uint32_t)lane;
            // the next chunk is in flight while this one is computed
            G2PRaw<T, DIM> raw_n;
            if (e + 64 < span) g2p_load<T, DIM, ABS>(src, first + e + 64, raw_n);
            if (e >= head && e < span) {
                const uint32_t p = first + e;
                int cn[3] = {0, 0, 0}, lk[3] = {0, 0, 0};
                T on[DIM], vn[DIM], Bs[DIM * DIM], Fn[DIM * DIM], xs[DIM];
                g2p_update<T, DIM, DEG, ABS>(raw, reg, origin, g, dt_inv_dx, gs, lk, cn, on, vn, Bs, Fn, prm.transfer,
                                             xs, prm.dt);
                T off[DIM];
                if constexpr (ABS) {
                    int ci[3];
                    particle_cells<T, DIM, true>(0u, raw.off, g.inv_dx, ci, off);
                } else {
#pragma unroll
                    for (int a = 0; a < DIM; ++a) off[a] = raw.off[a];
                }
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
                    drank = sc.prank[p] + (dkey == kDeadKey ? 0u : ntab.kcount[dkey] - ntab.kmov[dkey]);
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
                    plane_at(dst.off + a * ds, qb) = ABS ? xs[a] : on[a];
                    plane_at(dst.v + a * ds, qb) = vn[a];
                }
#pragma unroll
                for (int k = 0; k < DIM * DIM; ++k) {
                    plane_at(dst.B + k * ds, qb) = Bs[k];
                    plane_at(dst.F + k * ds, qb) = Fn[k];
                }
                // after the stores, when the particle's other values are dead
                if constexpr (ADAPT) cfl_fold<T, DIM>(vn, Bs, g.cfl_c, cmax);
            }
            raw = raw_n;
        }
        wave_lds_sync();
    }
    if constexpr (ADAPT) cfl_raise(g.cfl, blk * 4 + (uint32_t)wv, (double)cmax);
    (void)cmax;
    (void)TE;
}

template <typename T, int DIM, int DEG, bool ADAPT, bool ABS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ADAPT ? 1 : g2p_min_waves<T, DIM, DEG>()))) void k_g2p(
    Parts<T> src, Parts<T> dst, BinLists cur, TileTables ctab, BinLists nxt, TileTables ntab, BinScratch sc,
    GridState<T> g, StepParams<T> prm) {
    g2p_body<T, DIM, DEG, ADAPT, ABS>(src, dst, cur, ctab, nxt, ntab, sc, g, prm, blockIdx.x, gridDim.x);
}

template <typename T, int DIM, int DEG, bool ADAPT, bool QUEUE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QUEUE ? 1 : g2p_min_waves<T, DIM, DEG>()))) void k_g2p_batch(
    const SceneDesc<T> *descs, const int32_t *start, int n, int k, BatchQueue q) {
    batch_items<QUEUE>(q, [&](uint32_t it) {
        const BatchStep<T> b = batch_step<T>(descs, start, n, k, it);
        const SceneDesc<T> &d = *b.d;
        Parts<T> src = d.bufs[b.sp.src], dst = d.bufs[b.sp.src ^ 1];
        if (!src.id || !dst.id) src.id = dst.id = nullptr;
        // the scene's structs as values: read through the table they would be
        // read again after every store the compiler cannot prove apart
        const TileTables ctab = d.tab[b.sp.cur], ntab = d.tab[b.sp.nxt];
        const BinScratch sc = d.sc;
        const GridState<T> g = d.g;
        const StepParams<T> prm = d.prm;
        g2p_body<T, DIM, DEG, ADAPT>(src, dst, b.cur, ctab, b.nxt, ntab, sc, g, prm, b.blk, b.nblk);
    });
}

template <typename T, int DIM, int DEG>
void launch_g2p_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, const BatchQueue &q, int blocks,
                      bool adapt, hipStream_t st) {
    const dim3 grid((unsigned)blocks), block(256);
    if (adapt && q.ctr)
        hipLaunchKernelGGL((k_g2p_batch<T, DIM, DEG, true, true>), grid, block, 0, st, descs, start, n, k, q);
    else if (adapt)
        hipLaunchKernelGGL((k_g2p_batch<T, DIM, DEG, true, false>), grid, block, 0, st, descs, start, n, k, q);
    else if (q.ctr)
        hipLaunchKernelGGL((k_g2p_batch<T, DIM, DEG, false, true>), grid, block, 0, st, descs, start, n, k, q);
    else
        hipLaunchKernelGGL((k_g2p_batch<T, DIM, DEG, false, false>), grid, block, 0, st, descs, start, n, k, q);
}

// --- adaptive batched steps (Sec. 4.3) ---------------------------------------------
// One block per scene: zero its bound slots.
template <typename T>
__global__ __launch_bounds__(256) void k_cfl_clear_batch(const SceneDesc<T> *descs) {
    unsigned long long *slots = descs[blockIdx.x].g.cfl;
    for (int i = (int)threadIdx.x; i < kVmaxSlots; i += (int)blockDim.x) slots[i] = 0ull;
}

// Blocks by particle count (start): each scene's bound over the particles
// it starts the call with, raised into its slots.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_cfl_bound_batch(const SceneDesc<T> *descs, const int32_t *start, int n) {
    const int s = scene_of_block(start, n, blockIdx.x);
    const SceneDesc<T> &d = descs[s];
    const Parts<T> P = d.bufs[d.where0];
    const uint32_t b = blockIdx.x - (uint32_t)start[s], nb = (uint32_t)(start[s + 1] - start[s]);
    double m = 0.0;
    for (int64_t p = (int64_t)b * 256 + threadIdx.x; p < P.n; p += (int64_t)nb * 256) {
        T v[DIM], B[DIM * DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) v[a] = P.v[a * P.s + p];
#pragma unroll
        for (int q = 0; q < DIM * DIM; ++q) B[q] = P.B[q * P.s + p];
        cfl_fold64<T, DIM>(v, B, d.g.cfl_c, m);
    }
    cfl_raise(d.g.cfl, b * 4 + (threadIdx.x >> 6), m);
}

// One wavefront per scene: dt = min(dt_cap, nu_dx / bound) from its slots
// (bound 0 or NaN: dt_cap), recorded with the running time; slots zeroed.
template <typename T>
__global__ __launch_bounds__(64) void k_adapt_dt_batch(const SceneDesc<T> *descs) {
    const SceneDesc<T> &d = descs[blockIdx.x];
    const int lane = (int)threadIdx.x;
    unsigned long long *slots = d.g.cfl;
    double bnd = 0.0;
    for (int i = lane; i < kVmaxSlots; i += 64) {
        const double y = __longlong_as_double((long long)slots[i]);
        bnd = y > bnd || y != y ? y : bnd;
        slots[i] = 0ull;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_xor(bnd, o, 64);
        bnd = y > bnd || y != y ? y : bnd;
    }
    if (lane == 0) {
        double dt = d.dt_cap;
        if (bnd > 0.0) {
            const double c = d.nu_dx / bnd;
            dt = c < dt ? c : dt;
        }
        double *state = const_cast<double *>(d.prm.dt_dev);
        state[0] = dt;
        state[1] += dt;
    }
}

template <typename T, int DIM>
void launch_adapt_dt_batch(const SceneDesc<T> *descs, const int32_t *copy_start, int n, int copy_blocks, bool first,
                           hipStream_t st) {
    if (first) {
        hipLaunchKernelGGL((k_cfl_clear_batch<T>), dim3((unsigned)n), dim3(256), 0, st, descs);
        hipLaunchKernelGGL((k_cfl_bound_batch<T, DIM>), dim3((unsigned)copy_blocks), dim3(256), 0, st, descs,
                           copy_start, n);
    }
    hipLaunchKernelGGL((k_adapt_dt_batch<T>), dim3((unsigned)n), dim3(64), 0, st, descs);
}

template <typename T, int DIM, int DEG, bool ABS>
void launch_g2p(const Parts<T> &src, const Parts<T> &dst, const BinLists &cur, const TileTables &ctab,
                const BinLists &nxt, const TileTables &ntab, const BinScratch &sc, const GridState<T> &g,
                const StepParams<T> &prm, int64_t max_records, hipStream_t st) {
    if (src.n == 0) return;
    Parts<T> s2 = src, d2 = dst;
    if (!src.id || !dst.id) s2.id = d2.id = nullptr;
    int64_t blocks = (max_records + (src.n + 63) / 64 + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    if constexpr (!ABS) {
        if (g.cfl) {
            hipLaunchKernelGGL((k_g2p<T, DIM, DEG, true, false>), dim3((unsigned)blocks), dim3(256), 0, st, s2, d2,
                               cur, ctab, nxt, ntab, sc, g, prm);
            return;
        }
    }
    hipLaunchKernelGGL((k_g2p<T, DIM, DEG, false, ABS>), dim3((unsigned)blocks), dim3(256), 0, st, s2, d2, cur, ctab,
                       nxt, ntab, sc, g, prm);
}

#define APIC_G2P_INST(T, DIM, DEG)                                                                               \
    template void launch_bin_keys_moved_batch<T, DIM, DEG>(const SceneDesc<T> *, const int32_t *, int, int,           \
                                                           const BatchQueue &, int,                                   \
                                                           hipStream_t);                                          \
    template void launch_g2p_batch<T, DIM, DEG>(const SceneDesc<T> *, const int32_t *, int, int,                      \
                                                const BatchQueue &, int, bool,                                        \
                                                hipStream_t);                                                     \
    template void launch_bin_keys_moved<T, DIM, DEG, false>(const Parts<T> &, const BinLists &, const TileTables &, \
                                                            const GridState<T> &, const StepParams<T> &,         \
                                                            const BinLists &, const BinScratch &, int64_t,       \
                                                            hipStream_t);                                         \
    template void launch_g2p<T, DIM, DEG, false>(const Parts<T> &, const Parts<T> &, const BinLists &,           \
                                                 const TileTables &, const BinLists &, const TileTables &,       \
                                                 const BinScratch &, const GridState<T> &, const StepParams<T> &, \
                                                 int64_t, hipStream_t);
APIC_G2P_INST(float, 2, 1)
APIC_G2P_INST(float, 3, 1)
APIC_G2P_INST(double, 2, 1)
APIC_G2P_INST(double, 3, 1)
APIC_G2P_INST(float, 2, 2)
APIC_G2P_INST(float, 2, 3)
APIC_G2P_INST(float, 3, 2)
APIC_G2P_INST(float, 3, 3)
APIC_G2P_INST(double, 2, 2)
APIC_G2P_INST(double, 2, 3)
APIC_G2P_INST(double, 3, 2)
APIC_G2P_INST(double, 3, 3)

// absolute binary32 positions: binary32, quadratic and cubic, fixed steps
#define APIC_G2P_ABS_INST(DIM, DEG)                                                                               \
    template void launch_bin_keys_moved<float, DIM, DEG, true>(                                                   \
        const Parts<float> &, const BinLists &, const TileTables &, const GridState<float> &,                    \
        const StepParams<float> &, const BinLists &, const BinScratch &, int64_t, hipStream_t);                  \
    template void launch_g2p<float, DIM, DEG, true>(const Parts<float> &, const Parts<float> &, const BinLists &, \
                                                    const TileTables &, const BinLists &, const TileTables &,    \
                                                    const BinScratch &, const GridState<float> &,                \
                                                    const StepParams<float> &, int64_t, hipStream_t);
APIC_G2P_ABS_INST(2, 2)
APIC_G2P_ABS_INST(2, 3)
APIC_G2P_ABS_INST(3, 2)
APIC_G2P_ABS_INST(3, 3)

template void launch_adapt_dt_batch<float, 2>(const SceneDesc<float> *, const int32_t *, int, int, bool, hipStream_t);
template void launch_adapt_dt_batch<float, 3>(const SceneDesc<float> *, const int32_t *, int, int, bool, hipStream_t);
template void launch_adapt_dt_batch<double, 2>(const SceneDesc<double> *, const int32_t *, int, int, bool,
                                               hipStream_t);
template void launch_adapt_dt_batch<double, 3>(const SceneDesc<double> *, const int32_t *, int, int, bool,
                                               hipStream_t);

}  // namespace apic
