// Binning of particles by base node (apic_sort, and the shared passes of the
// re-binning done by apic_g2p).  Integer work only: counts, prefix sums and
// permutations; the result does not depend on the method's arithmetic.
#include "apic_bin_device.h"
#include "apic_kernels.h"

namespace apic {

static inline int blocks_for(int64_t work, int threads, int cap) {
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// --- clearing the buffers a new layout is built in ---------------------------
__global__ __launch_bounds__(256) void k_bin_clear(BinMeta nxt, BinScratch sc, int64_t bound) {
    const uint32_t nrec = nxt.count[0];
    const uint32_t nnode = sc.node_count[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bound; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < nrec) nxt.map[nxt.tile[i]] = -1;
        if (i < nnode) sc.node_flag[sc.node_list[i]] = 0u;
    }
}

__global__ void k_bin_reset(BinMeta nxt, BinScratch sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        nxt.count[0] = 0u;
        nxt.count[1] = 0u;
        sc.node_count[0] = 0u;
    }
}

void launch_bin_begin(const BinMeta &nxt, const BinScratch &sc, const Bounds &b, hipStream_t st) {
    const int64_t bound = b.max_records > b.tiles ? b.max_records : b.tiles;
    hipLaunchKernelGGL(k_bin_clear, dim3(blocks_for(bound, 256, 4096)), dim3(256), 0, st, nxt, sc, bound);
    hipLaunchKernelGGL(k_bin_reset, dim3(1), dim3(64), 0, st, nxt, sc);
}

// --- keys of particles at their current position -----------------------------
template <typename T, int DIM, int DEG>
__global__ __launch_bounds__(256) void k_bin_keys_static(Parts<T> P, GridDims d, BinMeta nxt, BinScratch sc,
                                                         uint32_t *flags) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = p < P.n;
    uint32_t key = kDeadKey;
    if (active) {
        int ci[3] = {0, 0, 0};
        unpack_cell<DIM>(P.cell[p], ci);
        T off[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) off[a] = P.off[a * P.s + p];
        bool finite;
        key = key_of<T, DIM, DEG>(ci, off, d, finite);
        if (key == kDeadKey) atomicOr(flags, finite ? FLAG_OUT_OF_DOMAIN : FLAG_NONFINITE);
    }
    const uint32_t rank = bin_take_slot(key, active, nxt, sc);
    if (!active) return;
    sc.pkey[p] = key;
    sc.prank[p] = rank;
}

template <typename T, int DIM, int DEG>
void launch_bin_keys_static(const Parts<T> &P, const GridDims &d, const BinMeta &nxt, const BinScratch &sc,
                            uint32_t *flags, hipStream_t st) {
    if (P.n == 0) return;
    hipLaunchKernelGGL((k_bin_keys_static<T, DIM, DEG>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P,
                       d, nxt, sc, flags);
}

// --- per-record counts ------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t &total) {
    const int lane = lane_id();
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    total = __shfl(inc, 63, 64);
    return inc - x;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t y = __shfl_xor(x, o, 64);
        x = x > y ? x : y;
    }
    return x;
}

__global__ __launch_bounds__(256) void k_bin_records(BinMeta nxt, BinScratch sc) {
    const int lane = lane_id();
    const uint32_t nrec = nxt.count[0];
    for (uint32_t rec = blockIdx.x * 4 + (threadIdx.x >> 6); rec < nrec; rec += gridDim.x * 4) {
        const uint32_t t = nxt.tile[rec];
        const uint32_t key = t * 64 + lane;
        const uint32_t c = sc.key_count[key];
        sc.key_count[key] = 0u;
        uint32_t total;
        const uint32_t pre = wave_excl_scan(c, total);
        const uint32_t mx = wave_max(c);
        nxt.kcount[rec * 64 + lane] = c;
        nxt.kprefix[rec * 64 + lane] = pre;
        if (lane == 0) {
            nxt.base[rec] = total;
            nxt.maxc[rec] = mx;
            nxt.map[t] = (int32_t)rec;
            sc.tile_flag[t] = 0u;
            if (rec == 0) nxt.base[nrec] = 0u;
        }
    }
}

// --- exclusive scan of nxt.base[0 .. count] (count read on the device) ------
__global__ __launch_bounds__(1024) void k_scan_blocks_dev(uint32_t *data, const uint32_t *count, uint32_t *sums) {
    __shared__ uint32_t sh[1024];
    const int64_t n = (int64_t)count[0] + 1;
    const int64_t start = (int64_t)blockIdx.x * 1024;
    if (start >= n) {
        if (threadIdx.x == 0) sums[blockIdx.x] = 0u;
        return;
    }
    const int64_t i = start + threadIdx.x;
    uint32_t x = i < n ? data[i] : 0u;
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t y = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
        __syncthreads();
        sh[threadIdx.x] += y;
        __syncthreads();
    }
    if (i < n) data[i] = sh[threadIdx.x] - x;
    if (threadIdx.x == 1023) sums[blockIdx.x] = sh[1023];
}

__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *sums, int64_t count) {
    __shared__ uint32_t sh[1024];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t start = 0; start < count; start += 1024) {
        const int64_t i = start + threadIdx.x;
        uint32_t x = i < count ? sums[i] : 0u;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            uint32_t y = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
            __syncthreads();
            sh[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < count) sums[i] = sh[threadIdx.x] - x + carry;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_scan_add_dev(uint32_t *data, const uint32_t *count, const uint32_t *sums) {
    const int64_t n = (int64_t)count[0] + 1;
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < n) data[i] += sums[blockIdx.x];
}

// --- level-major destinations, tile map and node tiles of the grid update ------
template <int DIM>
__global__ __launch_bounds__(256) void k_bin_levels(BinMeta nxt, BinScratch sc, GridDims d) {
    const int lane = lane_id();
    const uint32_t nrec = nxt.count[0];
    for (uint32_t rec = blockIdx.x * 4 + (threadIdx.x >> 6); rec < nrec; rec += gridDim.x * 4) {
        const uint32_t base = nxt.base[rec];
        const uint32_t c = nxt.kcount[rec * 64 + lane];
        const uint32_t kp = nxt.kprefix[rec * 64 + lane];
        const uint32_t mx = nxt.maxc[rec];
        uint32_t level = 0;
        for (uint32_t j = 0; j < mx; ++j) {
            const uint64_t mask = ballot(c > j);
            if (c > j) sc.perm[base + kp + j] = base + level + (uint32_t)popc64(mask & lanes_below(lane));
            level += (uint32_t)popc64(mask);
        }
        // node tiles whose nodes this record's slab covers: t + {0,1}^DIM
        if (lane < (1 << DIM)) {
            const int64_t t = nxt.tile[rec];
            int tc[3] = {0, 0, 0};
            tc[0] = (int)(t % d.TN[0]);
            if constexpr (DIM == 3) {
                tc[1] = (int)((t / d.TN[0]) % d.TN[1]);
                tc[2] = (int)(t / ((int64_t)d.TN[0] * d.TN[1]));
            } else {
                tc[1] = (int)(t / d.TN[0]);
            }
            bool ok = true;
            int64_t tau = 0, mul = 1;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const int c2 = tc[a] + ((lane >> a) & 1);
                ok = ok && c2 < d.TN[a];
                tau += c2 * mul;
                mul *= d.TN[a];
            }
            if (ok && atomicOr(sc.node_flag + tau, 1u) == 0u) {
                const uint32_t idx = atomicAdd(sc.node_count, 1u);
                sc.node_list[idx] = (uint32_t)tau;
            }
        }
    }
}

template <int DIM>
void launch_bin_finish(const GridDims &d, const BinMeta &nxt, const BinScratch &sc, const Bounds &b,
                       hipStream_t st) {
    const int wave_blocks = blocks_for(b.max_records, 4, 4096);
    hipLaunchKernelGGL(k_bin_records, dim3(wave_blocks), dim3(256), 0, st, nxt, sc);
    const int64_t nb = (b.max_records + 1 + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_blocks_dev, dim3((unsigned)nb), dim3(1024), 0, st, nxt.base, nxt.count, sc.sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, sc.sums, nb);
    hipLaunchKernelGGL(k_scan_add_dev, dim3((unsigned)nb), dim3(1024), 0, st, nxt.base, nxt.count, sc.sums);
    hipLaunchKernelGGL((k_bin_levels<DIM>), dim3(wave_blocks), dim3(256), 0, st, nxt, sc, d);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_bin_scatter_copy(Parts<T> src, Parts<T> dst, BinMeta nxt, BinScratch sc) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= src.n) return;
    const int64_t q = bin_destination(sc.pkey[p], sc.prank[p], nxt, sc);
    dst.cell[q] = src.cell[p];
    dst.m[q] = src.m[p];
    if (src.id) dst.id[q] = src.id[p];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        dst.off[a * dst.s + q] = src.off[a * src.s + p];
        dst.v[a * dst.s + q] = src.v[a * src.s + p];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        dst.B[k * dst.s + q] = src.B[k * src.s + p];
        dst.F[k * dst.s + q] = src.F[k * src.s + p];
    }
}

template <typename T, int DIM>
void launch_bin_scatter_copy(const Parts<T> &src, const Parts<T> &dst, const BinMeta &nxt, const BinScratch &sc,
                             hipStream_t st) {
    if (src.n == 0) return;
    Parts<T> s2 = src, d2 = dst;
    if (!src.id || !dst.id) s2.id = d2.id = nullptr;
    hipLaunchKernelGGL((k_bin_scatter_copy<T, DIM>), dim3((unsigned)((src.n + 255) / 256)), dim3(256), 0, st, s2, d2,
                       nxt, sc);
}

// --- instantiations -------------------------------------------------------------------
template void launch_bin_finish<2>(const GridDims &, const BinMeta &, const BinScratch &, const Bounds &, hipStream_t);
template void launch_bin_finish<3>(const GridDims &, const BinMeta &, const BinScratch &, const Bounds &, hipStream_t);

#define APIC_BIN_INST(T, DIM)                                                                                    \
    template void launch_bin_scatter_copy<T, DIM>(const Parts<T> &, const Parts<T> &, const BinMeta &,            \
                                                  const BinScratch &, hipStream_t);                               \
    template void launch_bin_keys_static<T, DIM, 2>(const Parts<T> &, const GridDims &, const BinMeta &,          \
                                                    const BinScratch &, uint32_t *, hipStream_t);                 \
    template void launch_bin_keys_static<T, DIM, 3>(const Parts<T> &, const GridDims &, const BinMeta &,          \
                                                    const BinScratch &, uint32_t *, hipStream_t);
APIC_BIN_INST(float, 2)
APIC_BIN_INST(float, 3)
APIC_BIN_INST(double, 2)
APIC_BIN_INST(double, 3)

}  // namespace apic
