// One step's transfer to particles (Sec. 3.4, lambda = 0 form of Sec. 5.7)
// fused with the next step's transfer to grid (Sec. 3.2 with the force of
// Sec. 3.3), for binary32 quadratic 3D.
//
// k_g2p2g: one block of two wavefronts per listed tile of the current
// layout, lane = key in both.  Wavefront 0 walks the key's particles level by
// level (loads two levels ahead), updates each one from the grid velocities
// staged in LDS with the same code as k_g2p and writes it to its place in
// the new layout.  A particle that keeps its key (nearly all of them in a
// step) is in the same tile and key of the new layout: wavefront 0 hands its
// new state to wavefront 1 through a double-buffered LDS slot (one barrier
// per level), and wavefront 1 adds its P2G terms to the lane's register sums
// of the key's 27 x 4 node values, then adds the sums into the tile's slab of
// the new layout (conflict-free LDS rounds, as in k_p2g) and stores it.  The
// two roles run on different wavefronts, so the G2P sweep and the register
// sums never hold registers at the same time, and the G2P memory traffic
// overlaps the P2G arithmetic.
//
// k_p2g_movers: one wavefront per listed tile of the new layout that took in
// movers: it loads the tile's slab (stored by k_g2p2g when the tile was
// listed before, zero otherwise), adds the register sums of its movers (the
// first ranks of each key, read back from the new layout) and stores it.
//
// The P2G terms of a particle are formed from exactly the values written to
// the new layout, so the slabs equal those of a P2G pass over it up to the
// order of the sums.
#include "apic_kernels.h"
#include "g2p_device.h"
#include "p2g_device.h"

namespace apic {

constexpr int kHandFields = 25;  // m, off[3], v[3], B[9], F[9] (the cell travels apart)

// The LDS of one k_g2p2g block.
template <typename T, int DEG, bool COMP>
struct PairLds {
    static constexpr int VT = 3 * VtRegion<3>::SIZE;
    static constexpr int SLAB = Geo<3, DEG>::NC * (COMP ? 2 : 1) * SlabLds<3, DEG>::PLANE;
    T vt[VT];                         // grid velocities around the tile (wavefront 0)
    T slab[SLAB];                     // slab of the new layout (wavefront 1)
    T hand[2][kHandFields][64];       // new state of the level's stayers
    uint32_t hcell[2][64];
    uint64_t hmask[2];                // lanes whose particle stayed
};

template <typename T, int DEG, bool COMP>
__device__ __forceinline__ void g2p2g_body(const Parts<T> &src, const Parts<T> &dst, const BinLists &cur,
                                           const TileTables &ctab, const BinLists &nxt, const TileTables &ntab,
                                           const BinScratch &sc, const Slabs<T> &slabs, const GridState<T> &g,
                                           const StepParams<T> &prm_in, uint32_t blk, uint32_t nblk) {
    const StepParams<T> &prm = prm_in;  // fixed dt: never used by adaptive steps
    constexpr int K = DEG + 1;
    static_assert(p2g_slices<T, 3, DEG>() == K, "the register sums of all support nodes fit in one pass");
    __shared__ PairLds<T, DEG, COMP> L;
    const int lane = lane_id();
    const bool producer = threadIdx.x < 64;
    int lcoord[3] = {0, 0, 0};
    local_coords<3>(lane, lcoord);
    const TileWalk walk = tile_walk(cur);
    const uint32_t *bases = nxt.bpre;
    const uint32_t live_nxt = nxt.bpre[kBuckets];
    const uint32_t items = walk.nrec + dead_chunks(src.n, walk.live);
    const T dt_inv_dx = prm.dt * g.inv_dx, gs = prm.dt * g.inv_dx;
    const T reach = step_reach<T>(wave_vmax(g.vmax), prm, g.inv_dx);
    const int64_t ds = dst.s;
    uint32_t hj = 0;  // hand-over slots used so far (alternating buffers)
    for (uint32_t r = blk; r < items; r += nblk) {
        if (r >= walk.nrec) {
            if (producer) carry_dead<T, 3>(src, dst, sc, walk.live, live_nxt, r - walk.nrec);
            continue;
        }
        uint32_t start, cnt, maxc, kstart;
        const uint32_t t = tile_of_record(walk, r, cur, ctab, start, cnt, maxc, kstart);
        int origin[3] = {0, 0, 0};
        tile_origin<3>(t, g.d.TN, origin);
        if (producer) {
            // --- wavefront 0: G2P, write, hand the stayers over ---------------------
            stage_velocities<T, 3>(t, g, L.vt);
            // stayers of a key follow its movers, in their old order (the
            // mover pass after this one walks the lowest levels)
            uint32_t srank = ntab.kmov[t * 64 + (uint32_t)lane];
            const uint32_t tbase = bases[bucket_of(t)];
            wave_lds_sync();
            uint32_t level = 0, p = 0;
            uint64_t mask = ballot(cnt > 0);
            G2PRaw<T, 3> raw;
            if (cnt > 0) {
                p = (uint32_t)particle_at(start, kstart, 0, mask, 0, maxc, lane);
                g2p_load<T, 3>(src, p, raw);
            }
            for (uint32_t j = 0; j < maxc; ++j, ++hj) {
                // level j + 1 is in flight while level j is computed
                const uint32_t level_n = level + (uint32_t)popc64(mask);
                const uint64_t mask_n = ballot(cnt > j + 1);
                G2PRaw<T, 3> raw_n;
                uint32_t p_n = 0;
                if (cnt > j + 1) {
                    p_n = (uint32_t)particle_at(start, kstart, level_n, mask_n, j + 1, maxc, lane);
                    g2p_load<T, 3>(src, p_n, raw_n);
                }
                bool stays = false;
                const uint32_t hb = hj & 1u;
                if (cnt > j) {
                    int cn[3] = {0, 0, 0}, lk[3] = {0, 0, 0};
                    T on[3], vn[3], Bs[9], Fn[9];
                    g2p_update<T, 3, DEG>(raw, L.vt, origin, g, dt_inv_dx, gs, lk, cn, on, vn, Bs, Fn, prm.transfer);
                    const uint32_t mykey = t * 64 + (uint32_t)local_of<3>(lk);
                    stays = keeps_key<T, 3, DEG>(raw.off, reach);
                    if (!stays) {
                        bool finite;
                        stays = key_of<T, 3, DEG>(cn, on, g.d, finite) == mykey;
                    }
                    uint32_t dkey, drank, base;
                    if (stays) {
                        dkey = mykey;
                        drank = srank++;
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
                    for (int a = 0; a < 3; ++a)
                        cn[a] = cn[a] < 0 ? 0 : (cn[a] > g.d.n[a] - 1 ? g.d.n[a] - 1 : cn[a]);
                    const uint32_t packed = pack_cell<3>(cn);
                    const uint32_t qb = q * (uint32_t)sizeof(T), q4 = q * 4u;
                    plane_at(dst.cell, q4) = packed;
                    plane_at(dst.m, qb) = raw.m;
                    if (src.id) plane_at(dst.id, q4) = raw.id;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        plane_at(dst.off + a * ds, qb) = on[a];
                        plane_at(dst.v + a * ds, qb) = vn[a];
                    }
#pragma unroll
                    for (int k = 0; k < 9; ++k) {
                        plane_at(dst.B + k * ds, qb) = Bs[k];
                        plane_at(dst.F + k * ds, qb) = Fn[k];
                    }
                    if (stays) {
                        T(&h)[kHandFields][64] = L.hand[hb];
                        L.hcell[hb][lane] = packed;
                        h[0][lane] = raw.m;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            h[1 + a][lane] = on[a];
                            h[4 + a][lane] = vn[a];
                        }
#pragma unroll
                        for (int k = 0; k < 9; ++k) {
                            h[7 + k][lane] = Bs[k];
                            h[16 + k][lane] = Fn[k];
                        }
                    }
                }
                const uint64_t stayed = ballot(stays);
                if (lane == 0) L.hmask[hb] = stayed;
                __syncthreads();
                raw = raw_n;
                p = p_n;
                level = level_n;
                mask = mask_n;
            }
        } else {
            // --- wavefront 1: register sums of the stayers, slab ---------------------
            const int key[3] = {origin[0] + lcoord[0], origin[1] + lcoord[1], origin[2] + lcoord[2]};
            // the tile keeps its reference velocity: the slab this pass forms
            // for the new layout holds momenta relative to the same uref[t]
            T uref[3];
            tile_uref<T, 3>(t, g, uref);
            // the tile in the new layout: listed there when a particle stays in it
            const bool listed = nxt.tile_gen[t] == nxt.gen;
            const uint32_t rnew = nxt.slot[t];
            for (int i = lane; i < PairLds<T, DEG, COMP>::SLAB; i += 64) L.slab[i] = T(0);
            T acc_m[K][K][K], acc_v[3][K][K][K];
#pragma unroll
            for (int c = 0; c < K; ++c)
#pragma unroll
                for (int b = 0; b < K; ++b)
#pragma unroll
                    for (int a = 0; a < K; ++a) {
                        acc_m[c][b][a] = T(0);
                        acc_v[0][c][b][a] = acc_v[1][c][b][a] = acc_v[2][c][b][a] = T(0);
                    }
            for (uint32_t j = 0; j < maxc; ++j, ++hj) {
                __syncthreads();
                const uint32_t hb = hj & 1u;
                if ((L.hmask[hb] >> lane) & 1ull) {
                    const T(&h)[kHandFields][64] = L.hand[hb];
                    P2GRaw<T, 3> pr;
                    pr.cell = L.hcell[hb][lane];
                    pr.m = h[0][lane];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        pr.off[a] = h[1 + a][lane];
                        pr.v[a] = h[4 + a][lane];
                    }
#pragma unroll
                    for (int k = 0; k < 9; ++k) {
                        pr.B[k] = h[7 + k][lane];
                        pr.F[k] = h[16 + k][lane];
                    }
                    P2GParticle<T, 3, DEG> pp;
                    if (p2g_prepare<T, 3, DEG>(pr, key, prm, g.inv_dx, g.flags, uref, pp))
                        p2g_accumulate3<T, DEG, 0, K>(pp, acc_m, acc_v);
                }
            }
            if (listed) {
                wave_lds_sync();
                slab_flush3<T, DEG, COMP, 0, K>(lcoord, acc_m, acc_v, L.slab);
                slab_store<T, 3, DEG, COMP>(L.slab, slabs.v + (int64_t)rnew * slabs.stride);
            }
            wave_lds_sync();
        }
    }
}

template <typename T, int DEG, bool COMP>
__device__ __forceinline__ void p2g_movers_body(const Parts<T> &P, const BinLists &cur, const BinLists &nxt,
                                                const TileTables &ntab, const Slabs<T> &slabs,
                                                const GridState<T> &g, const StepParams<T> &prm_in, uint32_t blk,
                                                uint32_t nblk) {
    const StepParams<T> &prm = prm_in;  // fixed dt: never used by adaptive steps
    constexpr int K = DEG + 1;
    using Gm = Geo<3, DEG>;
    using SL = SlabLds<3, DEG>;
    constexpr int LSLAB = Gm::NC * (COMP ? 2 : 1) * SL::PLANE;
    __shared__ T lds_all[4 * LSLAB];
    T *lds = lds_all + (threadIdx.x >> 6) * LSLAB;
    const int lane = lane_id();
    int lcoord[3] = {0, 0, 0};
    local_coords<3>(lane, lcoord);
    if (blk == 0) {
        // the next grid update raises these bounds of max |vt|, and the
        // layout the next step builds (the one just read) starts from empty
        // lists
        for (int i = (int)threadIdx.x; i < kBuckets; i += (int)blockDim.x) {
            g.vmax[i] = 0u;
            cur.rec_count[i] = 0u;
            cur.nfull[i] = 0u;
            cur.nsparse[i] = 0u;
            cur.tot[i] = 0u;
        }
        if (threadIdx.x < kCtrCount) cur.ctr[threadIdx.x] = 0u;
    }
    const TileWalk walk = tile_walk(nxt);
    for (uint32_t r = blk * 4 + (threadIdx.x >> 6); r < walk.nrec; r += nblk * 4) {
        uint32_t start, cnt, maxc, kstart;
        const uint32_t t = tile_of_record(walk, r, nxt, ntab, start, cnt, maxc, kstart);
        const uint32_t mov = ntab.kmov[t * 64 + (uint32_t)lane];
        const uint32_t jend = wave_max_u32(mov);
        if (jend == 0u) continue;
        int key[3] = {0, 0, 0};
        tile_origin<3>(t, g.d.TN, key);
#pragma unroll
        for (int a = 0; a < 3; ++a) key[a] += lcoord[a];
        T *slab = slabs.v + (int64_t)r * slabs.stride;
        T uref[3];
        if (cur.tile_gen[t] == cur.gen) {
            // listed before: its slab (stored by k_g2p2g) and its reference
            slab_load<T, 3, DEG, COMP>(slab, lds);
            tile_uref<T, 3>(t, g, uref);
        } else {
            // new in this layout (only movers): the reference of its movers
            for (int i = lane; i < LSLAB; i += 64) lds[i] = T(0);
            tile_reference<T, 3>(P, start, kstart, mov, maxc, uref);
            if (lane == 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) g.uref[a * g.d.tiles + t] = uref[a];
            }
        }
        wave_lds_sync();
        constexpr int CZ = p2g_slices<T, 3, DEG>();
        p2g_pass3<T, DEG, COMP, 0, CZ, true>(P, key, lcoord, start, kstart, cnt, maxc, mov, jend, prm, g.inv_dx,
                                             g.flags, uref, lds);
        if constexpr (CZ < K) p2g_pass3<T, DEG, COMP, CZ, (2 * CZ <= K ? CZ : K - CZ), true>(
            P, key, lcoord, start, kstart, cnt, maxc, mov, jend, prm, g.inv_dx, g.flags, uref, lds);
        if constexpr (2 * CZ < K) p2g_pass3<T, DEG, COMP, 2 * CZ, (3 * CZ <= K ? CZ : K - 2 * CZ), true>(
            P, key, lcoord, start, kstart, cnt, maxc, mov, jend, prm, g.inv_dx, g.flags, uref, lds);
        if constexpr (3 * CZ < K) p2g_pass3<T, DEG, COMP, 3 * CZ, K - 3 * CZ, true>(
            P, key, lcoord, start, kstart, cnt, maxc, mov, jend, prm, g.inv_dx, g.flags, uref, lds);
        slab_store<T, 3, DEG, COMP>(lds, slab);
        wave_lds_sync();
    }
}

template <typename T, int DEG, bool COMP>
__global__ __launch_bounds__(128) void k_g2p2g(Parts<T> src, Parts<T> dst, BinLists cur, TileTables ctab,
                                               BinLists nxt, TileTables ntab, BinScratch sc, Slabs<T> slabs,
                                               GridState<T> g, StepParams<T> prm) {
    g2p2g_body<T, DEG, COMP>(src, dst, cur, ctab, nxt, ntab, sc, slabs, g, prm, blockIdx.x, gridDim.x);
}

template <typename T, int DEG, bool COMP>
__global__ __launch_bounds__(256) void k_p2g_movers(Parts<T> P, BinLists cur, BinLists nxt, TileTables ntab,
                                                    Slabs<T> slabs, GridState<T> g, StepParams<T> prm) {
    p2g_movers_body<T, DEG, COMP>(P, cur, nxt, ntab, slabs, g, prm, blockIdx.x, gridDim.x);
}

template <typename T, int DEG, bool COMP>
void launch_g2p2g(const Parts<T> &src, const Parts<T> &dst, const BinLists &cur, const TileTables &ctab,
                  const BinLists &nxt, const TileTables &ntab, const BinScratch &sc, const Slabs<T> &slabs,
                  const GridState<T> &g, const StepParams<T> &prm, int64_t max_records, hipStream_t st) {
    Parts<T> s2 = src, d2 = dst;
    if (!src.id || !dst.id) s2.id = d2.id = nullptr;
    // one block of two wavefronts per record or dead chunk
    int64_t blocks = max_records + (src.n + 63) / 64;
    if (blocks < 1) blocks = 1;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((k_g2p2g<T, DEG, COMP>), dim3((unsigned)blocks), dim3(128), 0, st, s2, d2, cur, ctab, nxt,
                       ntab, sc, slabs, g, prm);
}

template <typename T, int DEG, bool COMP>
void launch_p2g_movers(const Parts<T> &P, const BinLists &cur, const BinLists &nxt, const TileTables &ntab,
                       const Slabs<T> &slabs, const GridState<T> &g, const StepParams<T> &prm, int64_t max_records,
                       hipStream_t st) {
    int64_t blocks = (max_records + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_p2g_movers<T, DEG, COMP>), dim3((unsigned)blocks), dim3(256), 0, st, P, cur, nxt, ntab,
                       slabs, g, prm);
}

#define APIC_G2P2G_INST(T, DEG, COMP)                                                                          \
    template void launch_g2p2g<T, DEG, COMP>(const Parts<T> &, const Parts<T> &, const BinLists &,            \
                                             const TileTables &, const BinLists &, const TileTables &,        \
                                             const BinScratch &, const Slabs<T> &, const GridState<T> &,      \
                                             const StepParams<T> &, int64_t, hipStream_t);                    \
    template void launch_p2g_movers<T, DEG, COMP>(const Parts<T> &, const BinLists &, const BinLists &,       \
                                                  const TileTables &, const Slabs<T> &, const GridState<T> &, \
                                                  const StepParams<T> &, int64_t, hipStream_t);
APIC_G2P2G_INST(float, 2, false)
APIC_G2P2G_INST(float, 2, true)

}  // namespace apic
