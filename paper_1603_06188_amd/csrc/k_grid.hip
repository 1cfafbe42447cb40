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

// Mass and momentum of node `nc`: out[0] = m, out[1..DIM] = (m v) + dt f.
template <typename T, int DIM, int DEG, bool COMP>
__device__ __forceinline__ void gather_node(const int *nc, const BinLists &gm, const Slabs<T> &slabs,
                                            const GridDims &d, T *out) {
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
        const int idx = DIM == 3 ? loc[0] + RE * (loc[1] + RE * loc[2]) : loc[0] + RE * loc[1];
        const T *s = slabs.v + (int64_t)rec * slabs.stride;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const T x = s[k * RN + idx];
            if constexpr (COMP) {
                const T sum = hi[k] + x;
                lo[k] += two_sum_err(hi[k], x, sum) + s[(NC + k) * RN + idx];
                hi[k] = sum;
            } else {
                hi[k] += x;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) out[k] = COMP ? hi[k] + lo[k] : hi[k];
}

template <typename T, int DIM, int DEG, bool COMP>
__device__ __forceinline__ void grid_update_body(const BinLists &cur, const Slabs<T> &slabs, const GridState<T> &g,
                                                 const StepParams<T> &prm, uint32_t blk, uint32_t nblk) {
    const int lane = lane_id();
    const int64_t G = g.d.G;
    uint32_t ntiles, ncnt;
    const uint32_t npre = wave_bucket_prefix(cur.node_count, ntiles, ncnt);
    uint32_t bits = 0u;  // wave maximum so far of the bounds below
    const uint32_t wave = blk * 4 + (threadIdx.x >> 6);
    for (uint32_t i = wave; i < ntiles; i += nblk * 4) {
        uint32_t b, j;
        bucket_locate(i, npre, ncnt, b, j);
        const uint32_t tau = cur.node_list[(int64_t)b * cur.rcap + j];
        int nc[3] = {0, 0, 0}, lc[3] = {0, 0, 0};
        tile_origin<DIM>(tau, g.d.TN, nc);
        local_coords<DIM>(lane, lc);
        bool valid = true, sticky = false;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            nc[a] += lc[a];
            valid = valid && nc[a] < g.d.N[a];
            sticky = sticky || nc[a] < prm.band[2 * a] || nc[a] > g.d.n[a] - prm.band[2 * a + 1];
        }
        T mm[1 + DIM];
#pragma unroll
        for (int k = 0; k <= DIM; ++k) mm[k] = T(0);
        if (valid) gather_node<T, DIM, DEG, COMP>(nc, cur, slabs, g.d, mm);
        const bool live = valid && mm[0] > T(0) && !sticky;
        const T inv_m = live ? T(1) / mm[0] : T(0);
        const int64_t node = (int64_t)tau * 64 + lane;
        float vabs = 0.f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const T vt = live ? mm[1 + a] * inv_m + prm.dt * prm.g[a] : T(0);
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
    bits = wave_max_u32(bits);
    if (lane == 0 && bits != 0u) atomicMax(g.vmax + (wave & (kVmaxSlots - 1)), bits);
}

template <typename T, int DIM, int DEG, bool COMP>
__global__ __launch_bounds__(256) void k_grid_update(BinLists cur, Slabs<T> slabs, GridState<T> g,
                                                     StepParams<T> prm) {
    grid_update_body<T, DIM, DEG, COMP>(cur, slabs, g, prm, blockIdx.x, gridDim.x);
}

template <typename T, int DIM, int DEG, bool COMP>
__global__ __launch_bounds__(256) void k_grid_update_batch(const SceneDesc<T> *descs, const int32_t *start, int n,
                                                           int k) {
    const BatchStep<T> b = batch_step<T>(descs, start, n, k);
    const SceneDesc<T> &d = *b.d;
    grid_update_body<T, DIM, DEG, COMP>(b.cur, d.slabs, d.g, d.prm, b.blk, b.nblk);
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_grid_update_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, int blocks,
                              hipStream_t st) {
    hipLaunchKernelGGL((k_grid_update_batch<T, DIM, DEG, COMP>), dim3((unsigned)blocks), dim3(256), 0, st, descs,
                       start, n, k);
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_grid_update(const BinLists &cur, const Slabs<T> &slabs, const GridState<T> &g, const StepParams<T> &prm,
                        int64_t max_node_tiles, hipStream_t st) {
    const int blocks = blocks_for(max_node_tiles, 4, 8192);
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
        gather_node<T, DIM, DEG, COMP>(nc, gm, slabs, g.d, mm);
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
        gather_node<T, DIM, DEG, COMP>(nc, gm, slabs, g.d, mm);
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

__global__ void k_diag_final_grid(const double *partials, int nb, double *out) {
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += partials[b * 8 + threadIdx.x];
        out[threadIdx.x] = t;
    }
}

template <typename T, int DIM, int DEG, bool COMP>
void launch_diag_grid(const BinLists &gm, const Slabs<T> &slabs, const GridState<T> &g, int which, double dt,
                      double *partials, double *out, hipStream_t st) {
    int64_t count = 1;
    for (int a = 0; a < DIM; ++a) count *= g.d.N[a];
    const int nb = blocks_for(count, 256, kDiagBlocks);
    hipLaunchKernelGGL((k_diag_grid<T, DIM, DEG, COMP>), dim3(nb), dim3(256), 0, st, gm, slabs, g, which, dt,
                       partials);
    hipLaunchKernelGGL(k_diag_final_grid, dim3(1), dim3(64), 0, st, partials, nb, out);
}

#define APIC_GRID_INST(T, DIM, DEG, COMP)                                                                         \
    template void launch_grid_update_batch<T, DIM, DEG, COMP>(const SceneDesc<T> *, const int32_t *, int, int, int, \
                                                              hipStream_t);                                       \
    template void launch_grid_update<T, DIM, DEG, COMP>(const BinLists &, const Slabs<T> &, const GridState<T> &, \
                                                        const StepParams<T> &, int64_t, hipStream_t);            \
    template void launch_grid_export<T, DIM, DEG, COMP>(const BinLists &, const Slabs<T> &, const GridState<T> &, \
                                                        int, T *, hipStream_t);                                  \
    template void launch_diag_grid<T, DIM, DEG, COMP>(const BinLists &, const Slabs<T> &, const GridState<T> &,   \
                                                      int, double, double *, double *, hipStream_t);
#define APIC_GRID_INST2(T, DIM, DEG) APIC_GRID_INST(T, DIM, DEG, false) APIC_GRID_INST(T, DIM, DEG, true)
APIC_GRID_INST2(float, 2, 2)
APIC_GRID_INST2(float, 2, 3)
APIC_GRID_INST2(float, 3, 2)
APIC_GRID_INST2(float, 3, 3)
APIC_GRID_INST2(double, 2, 2)
APIC_GRID_INST2(double, 2, 3)
APIC_GRID_INST2(double, 3, 2)
APIC_GRID_INST2(double, 3, 3)

}  // namespace apic
