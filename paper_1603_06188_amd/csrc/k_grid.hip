// Grid evolution at lambda = 0 (Sec. 3.3) and grid observation.
//
// A node's mass and momentum are the sum of the slabs of the (at most
// 2^DIM) listed key tiles whose slab covers it, visited in a fixed order.
#include "apic_bin_device.h"
#include "apic_kernels.h"

namespace apic {

static inline int blocks_for(int64_t work, int threads, int cap) {
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// Mass and momentum of node `nc`: out[0] = m, out[1..DIM] = (m v) + dt f
// (each slab's momentum plus its mass times the reference velocity of its
// key tile).
template <typename T, int DIM, int DEG, bool COMP>
__device__ __forceinline__ void gather_node(const int *nc, const BinLists &gm, const Slabs<T> &slabs,
                                            const GridDims &d, const T *uref, T *out) {
    using Gm = Geo<DIM, DEG>;
    constexpr int TE = Gm::TE, RE = Gm::RE, RN = Gm::RN, NC = Gm::NC;
    T hi[NC], lo[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) hi[k] = lo[k] = T(0);
#pragma unroll
    for (int corner = 0; corner < (1 << DIM); ++corner) {
        int kt[3] = {0, 0, 0}, loc[3] = {0, 0, 0};
        bool ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            kt[a] = nc[a] / TE - ((corner >> a) & 1);
            loc[a] = nc[a] - kt[a] * TE;
            ok = ok && kt[a] >= 0 && loc[a] < RE;
        }
        if (!ok) continue;
        int64_t t = kt[0];
        if constexpr (DIM == 3)
            t += (int64_t)d.TN[0] * (kt[1] + (int64_t)d.TN[1] * kt[2]);
        else
            t += (int64_t)d.TN[0] * kt[1];
        // membership tag and record index are independent loads
        const uint32_t tag = gm.tile_gen[t], rec = gm.slot[t];
        if (tag != gm.gen) continue;
        int lb[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) lb[a] = loc[a] - ((corner >> a) & 1) * TE;
        const int idx = SlabMap<DIM, DEG>::in_block(corner, lb);
        const T *s = slabs.v + (int64_t)rec * slabs.stride;
        const T ms = s[idx], ms_lo = COMP ? s[NC * RN + idx] : T(0);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const T u = k == 0 ? T(0) : uref[(k - 1) * d.tiles + t];
            const T x = s[k * RN + idx] + ms * u;
            if constexpr (COMP) {
                const T sum = hi[k] + x;
                lo[k] += two_sum_err(hi[k], x, sum) + (s[(NC + k) * RN + idx] + ms_lo * u);
                hi[k] = sum;
            } else {
                hi[k] += x;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) out[k] = COMP ? hi[k] + lo[k] : hi[k];
}

// Node tile tau is updated by exactly one wavefront: the one of the first
// listed key tile, in the order e = 0, 1, ..., 2^DIM - 1, among the key tiles
// tau - e whose slabs cover it.  In the interior every tile owns itself.
// One load of 64 lanes (lane = corner c * 2^DIM + e) fetches the membership
// tags and slab records of all key tiles around all 2^DIM candidate node
// tiles t + c; they decide ownership and feed the slab gathers.
template <typename T, int DIM, int DEG, bool COMP>
__device__ __forceinline__ void grid_update_body(const BinLists &cur, const Slabs<T> &slabs, const GridState<T> &g,
                                                 const StepParams<T> &prm_in, uint32_t blk, uint32_t nblk) {
    const StepParams<T> prm = with_step_dt(prm_in);
    using Gm = Geo<DIM, DEG>;
    constexpr int TE = Gm::TE, RN = Gm::RN, NC = Gm::NC, NCOR = 1 << DIM;
    // slab values in flight per group: at most 32 registers
    constexpr int NP = NC * (COMP ? 2 : 1), REGS = NP * (int)(sizeof(T) / 4);
    constexpr int GE = REGS * NCOR <= 32 ? NCOR : (REGS * NCOR / 2 <= 32 ? NCOR / 2 : NCOR / 4);
    const int lane = lane_id();
    const int64_t G = g.d.G;
    __shared__ uint32_t wave_bits[4];
    const uint32_t nrec = cur.rpre[kBuckets];
    uint32_t bits = 0u;  // wave maximum so far of the bounds below
    const WaveWalk ww = wave_walk(blk, nblk, nrec);
    int lc[3] = {0, 0, 0};
    local_coords<DIM>(lane, lc);
    const int my_c = lane / NCOR, my_e = lane % NCOR;
    for (uint32_t r = ww.first; r < nrec; r += ww.stride) {
        const uint32_t t = cur.rec_tile[r];
        int tc[3] = {0, 0, 0};
        tc[0] = (int)(t % (uint32_t)g.d.TN[0]);
        if constexpr (DIM == 3) {
            tc[1] = (int)((t / (uint32_t)g.d.TN[0]) % (uint32_t)g.d.TN[1]);
            tc[2] = (int)(t / ((uint32_t)g.d.TN[0] * (uint32_t)g.d.TN[1]));
        } else {
            tc[1] = (int)(t / (uint32_t)g.d.TN[0]);
        }
        // lane (c, e): key tile (t + c) - e
        bool node_in = my_c < NCOR, key_in = my_c < NCOR;
        int64_t k = 0, mul = 1;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int nt = tc[a] + ((my_c >> a) & 1);
            const int kt = nt - ((my_e >> a) & 1);
            node_in = node_in && nt < g.d.TN[a];
            key_in = key_in && nt < g.d.TN[a] && kt >= 0;
            k += (int64_t)kt * mul;
            mul *= g.d.TN[a];
        }
        uint32_t rec = 0u;
        bool listed = false;
        T ur[DIM];  // reference velocity of the key tile (read as is; used only when listed)
#pragma unroll
        for (int a = 0; a < DIM; ++a) ur[a] = T(0);
        if (key_in) {
            listed = cur.tile_gen[k] == cur.gen;
            rec = cur.slot[k];
#pragma unroll
            for (int a = 0; a < DIM; ++a) ur[a] = g.uref[a * g.d.tiles + k];
        }
        // this wave's key tile t owns the node tiles it updates: their
        // reference is t's (lane (0, 0) holds it)
        T own[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) own[a] = wave_uniform(ur[a]);
        const uint64_t lmask = ballot(listed);
        const uint64_t nmask = ballot(node_in && my_e == 0);
        for (int c = 0; c < NCOR; ++c) {
            const uint32_t lst = (uint32_t)(lmask >> (c * NCOR)) & ((1u << NCOR) - 1u);
            // owned: node tile inside, and no listed key tile before e = c
            if (!((nmask >> (c * NCOR)) & 1ull) || (lst & ((1u << c) - 1u)) != 0u) continue;
            int nc[3] = {0, 0, 0};
            int64_t tau = 0, tmul = 1;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const int ta = tc[a] + ((c >> a) & 1);
                tau += (int64_t)ta * tmul;
                tmul *= g.d.TN[a];
                nc[a] = ta * TE + lc[a];
            }
            bool valid = true, sticky = false;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                valid = valid && nc[a] < g.d.N[a];
                sticky = sticky || nc[a] < prm.band[2 * a] || nc[a] > g.d.n[a] - prm.band[2 * a + 1];
            }
            // sum of the covering slabs, e in increasing order, each slab's
            // momentum moved to this node tile's reference (the difference of
            // two references is exact).  The slabs are fetched in groups of
            // GE, every load of a group issued before the first is used (a
            // lane without a slab of that e reads the first slab and drops it)
            T hi[NC], lo[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) hi[q] = lo[q] = T(0);
#pragma unroll
            for (int e0 = 0; e0 < NCOR; e0 += GE) {
                T val[GE][NP];
                bool use[GE];
#pragma unroll
                for (int j = 0; j < GE; ++j) {
                    const int e = e0 + j;
                    const uint32_t srec = __shfl(rec, c * NCOR + e, 64);
                    // block e of the slab (one contiguous run per plane): the
                    // nodes within DEG of the tile's low faces along e's axes
                    bool ok = valid && ((lst >> e) & 1u);
#pragma unroll
                    for (int a = 0; a < DIM; ++a) ok = ok && lc[a] < SlabMap<DIM, DEG>::edge(e, a);
                    use[j] = ok;
                    const T *sp = slabs.v + (ok ? (int64_t)srec * slabs.stride + SlabMap<DIM, DEG>::in_block(e, lc) : 0);
#pragma unroll
                    for (int q = 0; q < NP; ++q) val[j][q] = sp[q * RN];
                }
#pragma unroll
                for (int j = 0; j < GE; ++j) {
                    const int e = e0 + j;
                    T du[DIM];
#pragma unroll
                    for (int a = 0; a < DIM; ++a) du[a] = __shfl(ur[a], c * NCOR + e, 64) - own[a];
                    if (!use[j]) continue;
                    const T ms = val[j][0], ms_lo = COMP ? val[j][NC] : T(0);
#pragma unroll
                    for (int q = 0; q < NC; ++q) {
                        const T u = q == 0 ? T(0) : du[q - 1];
                        const T x = val[j][q] + ms * u;
                        if constexpr (COMP) {
                            const T sum = hi[q] + x;
                            lo[q] += two_sum_err(hi[q], x, sum) + (val[j][NC + q] + ms_lo * u);
                            hi[q] = sum;
                        } else {
                            hi[q] += x;
                        }
                    }
                }
            }
            T mm[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) mm[q] = COMP ? hi[q] + lo[q] : hi[q];
            const bool live = valid && mm[0] > T(0) && !sticky;
            const T inv_m = live ? T(1) / mm[0] : T(0);
            const int64_t node = tau * 64 + lane;
            float vabs = 0.f;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                // the node tile's reference added back last
                const T vt = live ? (mm[1 + a] * inv_m + prm.dt * prm.g[a]) + own[a] : T(0);
                g.vt[a * G + node] = vt;
                // binary32 value not below |vt| (NaN propagates as the largest bits)
                const T va = vt < T(0) ? -vt : vt;
                float f = (float)va;
                if ((T)f < va) f = __uint_as_float(__float_as_uint(f) + 1u);  // next binary32 up
                vabs = (f > vabs || f != f) ? f : vabs;
            }
            // non-negative binary32 values order like their bit patterns
            const uint32_t mine = __float_as_uint(vabs);
            bits = mine > bits ? mine : bits;
        }
    }
    // one atomic per block, blocks spread over the slots
    bits = wave_max_u32(bits);
    if (lane == 0) wave_bits[threadIdx.x >> 6] = bits;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = wave_bits[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = wave_bits[k] > m ? wave_bits[k] : m;
        if (m != 0u) atomicMax(g.vmax + (blk % (uint32_t)kVmaxSlots), m);
    }
}

template <typename T, int DIM, int DEG, bool COMP>
__global__ __launch_bounds__(256) void k_grid_update(BinLists cur, Slabs<T> slabs, GridState<T> g,
                                                     StepParams<T> prm) {
    grid_update_body<T, DIM, DEG, COMP>(cur, slabs, g, prm, blockIdx.x, gridDim.x);
}

template <typename T, int DIM, int DEG, bool COMP, bool QUEUE>
__global__ __launch_bounds__(256) void k_grid_update_batch(const SceneDesc<T> *descs, const int32_t *start, int n,
                                                           int k, BatchQueue q) {
    batch_items<QUEUE>(q, [&](uint32_t it) {
        const BatchStep<T> b = batch_step<T>(descs, start, n, k, it);
        const SceneDesc<T> &d = *b.d;
        // the scene's structs as values: read through the table they would be
        // read again after every store the compiler cannot prove apart
        const Slabs<T> slabs = d.slabs;
        const GridState<T> g = d.g;
        const StepParams<T> prm = d.prm;
        grid_update_body<T, DIM, DEG, COMP>(b.cur, slabs, g, prm, b.blk, b.nblk);
    });
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_grid_update_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, const BatchQueue &q,
                              int blocks, hipStream_t st) {
    if (q.ctr)
        hipLaunchKernelGGL((k_grid_update_batch<T, DIM, DEG, COMP, true>), dim3((unsigned)blocks), dim3(256), 0, st,
                           descs, start, n, k, q);
    else
        hipLaunchKernelGGL((k_grid_update_batch<T, DIM, DEG, COMP, false>), dim3((unsigned)blocks), dim3(256), 0, st,
                           descs, start, n, k, q);
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_grid_update(const BinLists &cur, const Slabs<T> &slabs, const GridState<T> &g, const StepParams<T> &prm,
                        int64_t max_records, hipStream_t st) {
    const int blocks = blocks_for(max_records, 4, 4096);
    hipLaunchKernelGGL((k_grid_update<T, DIM, DEG, COMP>), dim3(blocks), dim3(256), 0, st, cur, slabs, g, prm);
}

// --- export: dense node-major copy of one field ------------------------------------
template <typename T, int DIM, int DEG, bool COMP>
__global__ __launch_bounds__(256) void k_grid_export(BinLists gm, Slabs<T> slabs, GridState<T> g, int field, T *out) {
    int64_t count = 1;
    for (int a = 0; a < DIM; ++a) count *= g.d.N[a];
    const int64_t G = g.d.G;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += (int64_t)gridDim.x * blockDim.x) {
        int nc[3] = {0, 0, 0};
        int64_t r = j;
        for (int a = 0; a < DIM; ++a) {
            nc[a] = (int)(r % g.d.N[a]);
            r /= g.d.N[a];
        }
        T mm[1 + DIM];
        gather_node<T, DIM, DEG, COMP>(nc, gm, slabs, g.d, g.uref, mm);
        if (field == 0) {
            out[j] = mm[0];
        } else if (field == 1) {
            for (int a = 0; a < DIM; ++a) out[a * count + j] = mm[1 + a];
        } else {
            const int64_t node = node_index<DIM>(nc, g.d.TN);
            for (int a = 0; a < DIM; ++a) out[a * count + j] = mm[0] > T(0) ? g.vt[a * G + node] : T(0);
        }
    }
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_grid_export(const BinLists &gm, const Slabs<T> &slabs, const GridState<T> &g, int field, T *out,
                        hipStream_t st) {
    int64_t count = 1;
    for (int a = 0; a < DIM; ++a) count *= g.d.N[a];
    hipLaunchKernelGGL((k_grid_export<T, DIM, DEG, COMP>), dim3(blocks_for(count, 256, 16384)), dim3(256), 0, st, gm,
                       slabs, g, field, out);
}

// --- binary64 grid totals (Sec. 3.1 momenta) ---------------------------------------
__device__ __forceinline__ void block_reduce8(double *acc, double *partials) {
    __shared__ double sh[8][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        double x = acc[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if (lane == 0) sh[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[threadIdx.x][w];
        partials[blockIdx.x * 8 + threadIdx.x] = t;
    }
}

template <typename T, int DIM, int DEG, bool COMP>
__global__ __launch_bounds__(256) void k_diag_grid(BinLists gm, Slabs<T> slabs, GridState<T> g, int which, double dt,
                                                   double *partials) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t count = 1;
    for (int a = 0; a < DIM; ++a) count *= g.d.N[a];
    const int64_t G = g.d.G;
    const double dx = (double)g.dx;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += (int64_t)gridDim.x * blockDim.x) {
        int nc[3] = {0, 0, 0};
        int64_t r = j;
        for (int a = 0; a < DIM; ++a) {
            nc[a] = (int)(r % g.d.N[a]);
            r /= g.d.N[a];
        }
        T mm[1 + DIM];
        gather_node<T, DIM, DEG, COMP>(nc, gm, slabs, g.d, g.uref, mm);
        const double m = (double)mm[0];
        if (!(m > 0.0)) continue;
        const int64_t node = node_index<DIM>(nc, g.d.TN);
        double x[3] = {0, 0, 0}, mv[3] = {0, 0, 0};
        for (int a = 0; a < DIM; ++a) {
            x[a] = (double)nc[a] * dx;
            if (which == 1) {
                mv[a] = (double)mm[1 + a];
            } else {
                const double vt = (double)g.vt[a * G + node];
                mv[a] = m * vt;
                x[a] += dt * vt;
            }
        }
        acc[0] += mv[0];
        acc[1] += mv[1];
        acc[2] += mv[2];
        if constexpr (DIM == 3) {
            acc[3] += x[1] * mv[2] - x[2] * mv[1];
            acc[4] += x[2] * mv[0] - x[0] * mv[2];
        }
        acc[5] += x[0] * mv[1] - x[1] * mv[0];
        double p2 = 0.0;
        for (int a = 0; a < DIM; ++a) p2 += mv[a] * mv[a];
        acc[6] += 0.5 * p2 / m;
        acc[7] += m;
    }
    block_reduce8(acc, partials);
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_diag_grid(const BinLists &gm, const Slabs<T> &slabs, const GridState<T> &g, int which, double dt,
                      double *partials, double *out, hipStream_t st) {
    int64_t count = 1;
    for (int a = 0; a < DIM; ++a) count *= g.d.N[a];
    const int nb = blocks_for(count, 256, kDiagBlocks);
    hipLaunchKernelGGL((k_diag_grid<T, DIM, DEG, COMP>), dim3(nb), dim3(256), 0, st, gm, slabs, g, which, dt,
                       partials);
    launch_diag_final(partials, nb, out, st);
}

#define APIC_GRID_INST(T, DIM, DEG, COMP)                                                                         \
    template void launch_grid_update_batch<T, DIM, DEG, COMP>(const SceneDesc<T> *, const int32_t *, int, int,        \
                                                              const BatchQueue &, int,                                \
                                                              hipStream_t);                                       \
    template void launch_grid_update<T, DIM, DEG, COMP>(const BinLists &, const Slabs<T> &, const GridState<T> &, \
                                                        const StepParams<T> &, int64_t, hipStream_t);            \
    template void launch_grid_export<T, DIM, DEG, COMP>(const BinLists &, const Slabs<T> &, const GridState<T> &, \
                                                        int, T *, hipStream_t);                                  \
    template void launch_diag_grid<T, DIM, DEG, COMP>(const BinLists &, const Slabs<T> &, const GridState<T> &,   \
                                                      int, double, double *, double *, hipStream_t);
#define APIC_GRID_INST2(T, DIM, DEG) APIC_GRID_INST(T, DIM, DEG, false) APIC_GRID_INST(T, DIM, DEG, true)
APIC_GRID_INST2(float, 2, 1)
APIC_GRID_INST2(float, 3, 1)
APIC_GRID_INST2(double, 2, 1)
APIC_GRID_INST2(double, 3, 1)
APIC_GRID_INST2(float, 2, 2)
APIC_GRID_INST2(float, 2, 3)
APIC_GRID_INST2(float, 3, 2)
APIC_GRID_INST2(float, 3, 3)
APIC_GRID_INST2(double, 2, 2)
APIC_GRID_INST2(double, 2, 3)
APIC_GRID_INST2(double, 3, 2)
APIC_GRID_INST2(double, 3, 3)

}  // namespace apic
