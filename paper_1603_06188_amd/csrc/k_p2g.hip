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
#include "apic_kernels.h"
#include "p2g_device.h"

namespace apic {

template <typename T, int DIM, int DEG, bool COMP, bool ABS = false>
__device__ __forceinline__ void p2g_body(const Parts<T> &P, const BinLists &cur, const BinLists &nxt,
                                         const TileTables &tab, const Slabs<T> &slabs, const GridState<T> &g,
                                         const StepParams<T> &prm_in, uint32_t blk, uint32_t nblk) {
    const StepParams<T> prm = with_step_dt(prm_in);
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
            nxt.nfull[i] = 0u;
            nxt.nsparse[i] = 0u;
            nxt.tot[i] = 0u;
        }
        if (threadIdx.x < kCtrCount) nxt.ctr[threadIdx.x] = 0u;
    }
    const TileWalk walk = tile_walk(cur);
    for (uint32_t r = blk * 4 + (threadIdx.x >> 6); r < walk.nrec; r += nblk * 4) {
        uint32_t start, cnt, maxc, kstart;
        const uint32_t t = tile_of_record(walk, r, cur, tab, start, cnt, maxc, kstart);
        int key[3] = {0, 0, 0};
        tile_origin<DIM>(t, g.d.TN, key);
#pragma unroll
        for (int a = 0; a < DIM; ++a) key[a] += lcoord[a];
        // the tile's reference velocity (the first pass derives it from the
        // level-0 particles it loads): the slab holds momenta relative to it
        T uref[DIM];
        for (int i = lane; i < LSLAB; i += 64) lds[i] = T(0);
        wave_lds_sync();
        if constexpr (DIM == 3) {
            constexpr int CZ = p2g_slices<T, 3, DEG>();
            p2g_pass3<T, DEG, COMP, 0, CZ, false, true, ABS>(P, key, lcoord, start, kstart, cnt, maxc, cnt, maxc,
                                                             prm, g.inv_dx, g.flags, uref, lds);
            if constexpr (CZ < K) p2g_pass3<T, DEG, COMP, CZ, (2 * CZ <= K ? CZ : K - CZ), false, false, ABS>(
                P, key, lcoord, start, kstart, cnt, maxc, cnt, maxc, prm, g.inv_dx, g.flags, uref, lds);
            if constexpr (2 * CZ < K)
                p2g_pass3<T, DEG, COMP, 2 * CZ, (3 * CZ <= K ? CZ : K - 2 * CZ), false, false, ABS>(
                    P, key, lcoord, start, kstart, cnt, maxc, cnt, maxc, prm, g.inv_dx, g.flags, uref, lds);
            if constexpr (3 * CZ < K) p2g_pass3<T, DEG, COMP, 3 * CZ, K - 3 * CZ, false, false, ABS>(
                P, key, lcoord, start, kstart, cnt, maxc, cnt, maxc, prm, g.inv_dx, g.flags, uref, lds);
        } else {
            tile_reference<T, DIM>(P, start, kstart, cnt, maxc, uref);
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
                    p2g_load<T, 2, ABS>(P, (uint32_t)q, raw);
                    P2GParticle<T, 2, DEG> pp;
                    if (p2g_prepare<T, 2, DEG, ABS>(raw, key, prm, g.inv_dx, g.flags, uref, pp))
                        p2g_accumulate2<T, DEG>(pp, acc_m, acc_v);
                }
                level += (uint32_t)popc64(mask);
            }
#pragma unroll
            for (int bb = 0; bb < K; ++bb)
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    const int idx = SL::at(lcoord[0] + a, lcoord[1] + bb, 0);
                    const T x[NC] = {acc_m[bb][a], acc_v[0][bb][a], acc_v[1][bb][a]};
                    slab_add_node<T, COMP, LP, NC>(lds, idx, x);
                    wave_lds_sync();
                }
        }
        if (lane == 0) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) g.uref[a * g.d.tiles + t] = uref[a];
        }
        slab_store<T, DIM, DEG, COMP>(lds, slabs.v + (int64_t)r * slabs.stride);
        wave_lds_sync();
    }
}

// Binary32 3D cubic: two waves per SIMD (256 VGPRs, a few spilled) instead
// of one; its accumulation issues VALU for under half of its time at one.
template <typename T, int DIM, int DEG>
constexpr int p2g_min_waves() {
    return (sizeof(T) == 4 && DIM == 3 && DEG == 3) ? 2 : 1;
}

template <typename T, int DIM, int DEG, bool COMP, bool ABS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(p2g_min_waves<T, DIM, DEG>()))) void k_p2g(
    Parts<T> P, BinLists cur, BinLists nxt, TileTables tab, Slabs<T> slabs, GridState<T> g, StepParams<T> prm) {
    p2g_body<T, DIM, DEG, COMP, ABS>(P, cur, nxt, tab, slabs, g, prm, blockIdx.x, gridDim.x);
}

template <typename T, int DIM, int DEG, bool COMP, bool QUEUE>
__global__ __launch_bounds__(256) void k_p2g_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k,
                                                   BatchQueue q) {
    batch_items<QUEUE>(q, [&](uint32_t it) {
        const BatchStep<T> b = batch_step<T>(descs, start, n, k, it);
        const SceneDesc<T> &d = *b.d;
        // the scene's structs as values: read through the table they would be
        // read again after every store the compiler cannot prove apart
        const Parts<T> P = d.bufs[b.sp.src];
        const TileTables tab = d.tab[b.sp.cur];
        const Slabs<T> slabs = d.slabs;
        const GridState<T> g = d.g;
        const StepParams<T> prm = d.prm;
        p2g_body<T, DIM, DEG, COMP>(P, b.cur, b.nxt, tab, slabs, g, prm, b.blk, b.nblk);
    });
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_p2g_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, const BatchQueue &q, int blocks,
                      hipStream_t st) {
    if (q.ctr)
        hipLaunchKernelGGL((k_p2g_batch<T, DIM, DEG, COMP, true>), dim3((unsigned)blocks), dim3(256), 0, st, descs,
                           start, n, k, q);
    else
        hipLaunchKernelGGL((k_p2g_batch<T, DIM, DEG, COMP, false>), dim3((unsigned)blocks), dim3(256), 0, st, descs,
                           start, n, k, q);
}

template <typename T, int DIM, int DEG, bool COMP, bool ABS>
void launch_p2g(const Parts<T> &P, const BinLists &cur, const BinLists &nxt, const TileTables &tab,
                const Slabs<T> &slabs, const GridState<T> &g, const StepParams<T> &prm, int64_t max_records,
                hipStream_t st) {
    int64_t blocks = (max_records + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_p2g<T, DIM, DEG, COMP, ABS>), dim3((unsigned)blocks), dim3(256), 0, st, P, cur, nxt, tab,
                       slabs, g, prm);
}

#define APIC_P2G_INST(T, DIM, DEG)                                                                                \
    template void launch_p2g_batch<T, DIM, DEG, false>(const SceneDesc<T> *, const int32_t *, int, int,               \
                                                       const BatchQueue &, int,                                       \
                                                       hipStream_t);                                              \
    template void launch_p2g_batch<T, DIM, DEG, true>(const SceneDesc<T> *, const int32_t *, int, int,                \
                                                      const BatchQueue &, int,                                        \
                                                      hipStream_t);                                               \
    template void launch_p2g<T, DIM, DEG, false, false>(const Parts<T> &, const BinLists &, const BinLists &,    \
                                                        const TileTables &, const Slabs<T> &, const GridState<T> &, \
                                                        const StepParams<T> &, int64_t, hipStream_t);            \
    template void launch_p2g<T, DIM, DEG, true, false>(const Parts<T> &, const BinLists &, const BinLists &,     \
                                                       const TileTables &, const Slabs<T> &, const GridState<T> &, \
                                                       const StepParams<T> &, int64_t, hipStream_t);
APIC_P2G_INST(float, 2, 1)
APIC_P2G_INST(float, 3, 1)
APIC_P2G_INST(double, 2, 1)
APIC_P2G_INST(double, 3, 1)
APIC_P2G_INST(float, 2, 2)
APIC_P2G_INST(float, 2, 3)
APIC_P2G_INST(float, 3, 2)
APIC_P2G_INST(float, 3, 3)
APIC_P2G_INST(double, 2, 2)
APIC_P2G_INST(double, 2, 3)
APIC_P2G_INST(double, 3, 2)
APIC_P2G_INST(double, 3, 3)

// absolute binary32 positions: binary32, quadratic and cubic
#define APIC_P2G_ABS_INST(DIM, DEG)                                                                                \
    template void launch_p2g<float, DIM, DEG, false, true>(const Parts<float> &, const BinLists &,              \
                                                           const BinLists &, const TileTables &,                 \
                                                           const Slabs<float> &, const GridState<float> &,       \
                                                           const StepParams<float> &, int64_t, hipStream_t);     \
    template void launch_p2g<float, DIM, DEG, true, true>(const Parts<float> &, const BinLists &, const BinLists &, \
                                                          const TileTables &, const Slabs<float> &,              \
                                                          const GridState<float> &, const StepParams<float> &,   \
                                                          int64_t, hipStream_t);
APIC_P2G_ABS_INST(2, 2)
APIC_P2G_ABS_INST(2, 3)
APIC_P2G_ABS_INST(3, 2)
APIC_P2G_ABS_INST(3, 3)

}  // namespace apic
