// Binning of particles by base node (apic_sort, and the passes shared with
// the re-binning done by apic_g2p).  Integer work only: counts, prefix sums,
// lists and destinations; nothing here depends on the method's arithmetic.
#include "apic_bin_device.h"
#include "apic_kernels.h"

namespace apic {

static inline int blocks_for(int64_t work, int threads, int cap) {
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// --- counters of a layout about to be built ---------------------------------------
__global__ void k_bin_reset(BinLists nxt) {
    for (int t = (int)threadIdx.x; t < kBuckets; t += (int)blockDim.x) {
        nxt.rec_count[t] = 0u;
        nxt.nfull[t] = 0u;
        nxt.nsparse[t] = 0u;
        nxt.tot[t] = 0u;
    }
    if (threadIdx.x < kCtrCount) nxt.ctr[threadIdx.x] = 0u;
}

void launch_bin_reset(const BinLists &nxt, hipStream_t st) {
    hipLaunchKernelGGL(k_bin_reset, dim3(1), dim3(256), 0, st, nxt);
}

// --- keys of particles at their current position (apic_sort); every particle
// counts as a mover, so ranks come from the per-key counters ---------------------
template <typename T, int DIM, int DEG, bool ABS>
__global__ __launch_bounds__(256) void k_bin_keys_static(Parts<T> P, GridDims d, BinLists nxt, BinScratch sc,
                                                         uint32_t *flags, T inv_dx) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = p < P.n;
    uint32_t key = kDeadKey;
    if (active) {
        int ci[3] = {0, 0, 0};
        T x[DIM], off[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) x[a] = P.off[a * P.s + p];
        particle_cells<T, DIM, ABS>(ABS ? 0u : P.cell[p], x, inv_dx, ci, off);
        bool finite;
        key = key_of<T, DIM, DEG>(ci, off, d, finite);
        if (key == kDeadKey) atomicOr(flags, finite ? FLAG_OUT_OF_DOMAIN : FLAG_NONFINITE);
    }
    const uint32_t rank = bin_take_slot(key, active, (uint32_t)p, (uint64_t)p, nxt, sc);
    if (active) {
        sc.pkey[p] = key;
        sc.prank[p] = rank;
    }
}

template <typename T, int DIM, int DEG, bool ABS>
void launch_bin_keys_static(const Parts<T> &P, const GridDims &d, const BinLists &nxt, const BinScratch &sc,
                            uint32_t *flags, T inv_dx, hipStream_t st) {
    if (P.n == 0) return;
    hipLaunchKernelGGL((k_bin_keys_static<T, DIM, DEG, ABS>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st,
                       P, d, nxt, sc, flags, inv_dx);
}

// --- per listed tile: counts, prefix sums, tile offset, level table ------------------
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t &total) {
    const int lane = lane_id();
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    total = __shfl(inc, 63, 64);
    return inc - x;
}

template <int DIM>
__device__ __forceinline__ void records_body(const BinLists &nxt, const TileTables &tab, const BinScratch &sc,
                                             const GridDims &d, uint32_t blk, uint32_t nblk) {
    __shared__ uint32_t rpre[kBuckets + 4];
    const int lane = lane_id();
    const uint32_t total_recs = block_bucket_prefix(nxt.rec_count, rpre, rpre + kBuckets);
    for (uint32_t r = blk * 4 + (threadIdx.x >> 6); r < total_recs; r += nblk * 4) {
        const uint32_t b = bucket_find(rpre, r);
        const uint32_t t = nxt.rec_list[(int64_t)b * nxt.rcap + (r - rpre[b])];
        const int64_t key = (int64_t)t * 64 + lane;
        const uint32_t mov = sc.key_count[key];
        const uint32_t c = mov + sc.scount[key];
        sc.key_count[key] = 0u;
        sc.scount[key] = 0u;
        if (mov) rank_movers(sc.head + key, mov, sc);
        uint32_t total;
        const uint32_t kp = wave_excl_scan(c, total);
        const uint32_t mx = wave_max_u32(c);
        tab.kcount[key] = c;
        tab.kmov[key] = mov;
        tab.kprefix[key] = kp;
        if (lane == 0) {
            tab.maxc[t] = mx;
            tab.tcount[t] = total;
            tab.off[t] = atomicAdd(nxt.tot + b, total);
            // rank among the bucket's tiles of its class (high bit: fewer
            // than kFullTile particles); the finalize pass makes it the
            // tile's record number
            nxt.slot[t] = total >= kFullTile ? atomicAdd(nxt.nfull + b, 1u)
                                             : (0x80000000u | atomicAdd(nxt.nsparse + b, 1u));
        }
        if (mx <= (uint32_t)kMaxLevels) {
            // level jj holds the jj-th particle of every key with more than jj
            uint32_t level = 0, my_off = 0;
            uint64_t my_mask = 0;
            for (uint32_t jj = 0; jj < mx; ++jj) {
                const uint64_t mask = ballot(c > jj);
                if ((uint32_t)lane == jj) {
                    my_off = level;
                    my_mask = mask;
                }
                level += (uint32_t)popc64(mask);
            }
            if ((uint32_t)lane < mx) {
                tab.lvl_off[(int64_t)t * kMaxLevels + lane] = my_off;
                tab.lvl_mask[(int64_t)t * kMaxLevels + lane] = my_mask;
            }
        }
    }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_bin_records(BinLists nxt, TileTables tab, BinScratch sc, GridDims d) {
    records_body<DIM>(nxt, tab, sc, d, blockIdx.x, gridDim.x);
}

template <typename T, int DIM, bool QUEUE>
__global__ __launch_bounds__(256) void k_bin_records_batch(const SceneDesc<T> *descs, const int32_t *start, int n,
                                                           int k, BatchQueue q) {
    batch_items<QUEUE>(q, [&](uint32_t it) {
        const BatchStep<T> b = batch_step<T>(descs, start, n, k, it);
        const SceneDesc<T> &d = *b.d;
        // the scene's structs as values: read through the table they would be
        // read again after every store the compiler cannot prove apart
        const TileTables tab = d.tab[b.sp.nxt];
        const BinScratch sc = d.sc;
        const GridDims dims = d.g.d;
        records_body<DIM>(b.nxt, tab, sc, dims, b.blk, b.nblk);
    });
}

template <typename T, int DIM>
void launch_bin_records_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, const BatchQueue &q,
                              int blocks, hipStream_t st) {
    if (q.ctr)
        hipLaunchKernelGGL((k_bin_records_batch<T, DIM, true>), dim3((unsigned)blocks), dim3(256), 0, st, descs, start,
                           n, k, q);
    else
        hipLaunchKernelGGL((k_bin_records_batch<T, DIM, false>), dim3((unsigned)blocks), dim3(256), 0, st, descs,
                           start, n, k, q);
}

// copies the particles of every scene that ended in the workspace shadow
// back to the caller's planes
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_copy_back_batch(const SceneDesc<T> *descs, const int32_t *start, int n,
                                                         int k) {
    const BatchStep<T> b = batch_step<T>(descs, start, n, k, blockIdx.x);
    if (b.sp.src != 1) return;
    const Parts<T> &src = b.d->bufs[1], &dst = b.d->bufs[0];
    for (int64_t j = (int64_t)b.blk * blockDim.x + threadIdx.x; j < src.n; j += (int64_t)b.nblk * blockDim.x) {
        dst.cell[j] = src.cell[j];
        dst.m[j] = src.m[j];
        if (src.id && dst.id) dst.id[j] = src.id[j];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            dst.off[a * dst.s + j] = src.off[a * src.s + j];
            dst.v[a * dst.s + j] = src.v[a * src.s + j];
        }
#pragma unroll
        for (int q = 0; q < DIM * DIM; ++q) {
            dst.B[q * dst.s + j] = src.B[q * src.s + j];
            dst.F[q * dst.s + j] = src.F[q * src.s + j];
        }
    }
}

template <typename T, int DIM>
void launch_copy_back_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, int blocks,
                            hipStream_t st) {
    hipLaunchKernelGGL((k_copy_back_batch<T, DIM>), dim3((unsigned)blocks), dim3(256), 0, st, descs, start, n, k);
}

// --- prefix tables and record numbers of a finished layout --------------------------
// Every block forms the bucket prefixes in LDS (block 0 also stores them).
// Record numbers: the tiles of at least kFullTile particles first, in bucket
// order and then by their rank in the bucket, then the others the same way,
// so that every tile walk takes the short tiles last.

// Last bucket whose exclusive prefix is <= i (pre[kBuckets] = total > i).
__device__ __forceinline__ uint32_t bucket_search(const uint32_t *pre, uint32_t i) {
    uint32_t lo = 0, hi = kBuckets;
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void finalize_body(const BinLists &nxt, uint32_t blk, uint32_t nblk) {
    __shared__ uint32_t rpre[kBuckets + 1], fpre[kBuckets + 1], bpre[kBuckets + 1], part[12];
    const uint32_t nrec = block_bucket_prefix(nxt.rec_count, rpre, part);
    const uint32_t nfull = block_bucket_prefix(nxt.nfull, fpre, part + 4);
    if (threadIdx.x == 0) rpre[kBuckets] = nrec;
    if (blk == 0) {
        const uint32_t live = block_bucket_prefix(nxt.tot, bpre, part + 8);
        for (int i = (int)threadIdx.x; i < kBuckets; i += (int)blockDim.x) {
            nxt.rpre[i] = rpre[i];
            nxt.bpre[i] = bpre[i];
        }
        if (threadIdx.x == 0) {
            nxt.rpre[kBuckets] = nrec;
            nxt.bpre[kBuckets] = live;
        }
    }
    __syncthreads();
    for (uint32_t i = blk * blockDim.x + threadIdx.x; i < nrec; i += nblk * blockDim.x) {
        const uint32_t b = bucket_search(rpre, i);
        const uint32_t t = nxt.rec_list[(int64_t)b * nxt.rcap + (i - rpre[b])];
        const uint32_t v = nxt.slot[t];
        const uint32_t rec = (v & 0x80000000u) ? nfull + (rpre[b] - fpre[b]) + (v & 0x7FFFFFFFu) : fpre[b] + v;
        nxt.slot[t] = rec;
        nxt.rec_tile[rec] = t;
    }
}

__global__ __launch_bounds__(256) void k_bin_finalize(BinLists nxt) { finalize_body(nxt, blockIdx.x, gridDim.x); }

void launch_bin_finalize(const BinLists &nxt, int64_t max_records, hipStream_t st) {
    hipLaunchKernelGGL(k_bin_finalize, dim3(blocks_for(max_records, 256, 128)), dim3(256), 0, st, nxt);
}

template <typename T>
__global__ __launch_bounds__(256) void k_bin_finalize_batch(const SceneDesc<T> *descs, const int32_t *start, int n,
                                                            int k) {
    const BatchStep<T> b = batch_step<T>(descs, start, n, k, blockIdx.x);
    finalize_body(b.nxt, b.blk, b.nblk);
}

template <typename T>
void launch_bin_finalize_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, int blocks,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_bin_finalize_batch<T>, dim3((unsigned)blocks), dim3(256), 0, st, descs, start, n, k);
}
template void launch_bin_finalize_batch<float>(const SceneDesc<float> *, const int32_t *, int, int, int, hipStream_t);
template void launch_bin_finalize_batch<double>(const SceneDesc<double> *, const int32_t *, int, int, int,
                                                hipStream_t);

template <int DIM>
void launch_bin_records(const GridDims &d, const BinLists &nxt, const TileTables &tab, const BinScratch &sc,
                        int64_t max_records, hipStream_t st) {
    hipLaunchKernelGGL((k_bin_records<DIM>), dim3(blocks_for(max_records, 4, 2048)), dim3(256), 0, st, nxt, tab, sc,
                       d);
}

// --- moves every particle to its binned position (apic_sort) ------------------------
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_bin_scatter_copy(Parts<T> src, Parts<T> dst, BinLists nxt, TileTables tab,
                                                          BinScratch sc) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= src.n) return;
    const uint32_t live = nxt.bpre[kBuckets];
    const uint32_t key = sc.pkey[p];
    const uint32_t rank = sc.prank[p];
    const int64_t q = bin_destination(key, rank, tab, bucket_base_of(key, nxt.bpre), live);
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
void launch_bin_scatter_copy(const Parts<T> &src, const Parts<T> &dst, const BinLists &nxt, const TileTables &tab,
                             const BinScratch &sc, hipStream_t st) {
    if (src.n == 0) return;
    Parts<T> s2 = src, d2 = dst;
    if (!src.id || !dst.id) s2.id = d2.id = nullptr;
    hipLaunchKernelGGL((k_bin_scatter_copy<T, DIM>), dim3((unsigned)((src.n + 255) / 256)), dim3(256), 0, st, s2, d2,
                       nxt, tab, sc);
}

// --- instantiations ---------------------------------------------------------------------
template void launch_bin_records<2>(const GridDims &, const BinLists &, const TileTables &, const BinScratch &,
                                    int64_t, hipStream_t);
template void launch_bin_records<3>(const GridDims &, const BinLists &, const TileTables &, const BinScratch &,
                                    int64_t, hipStream_t);

#define APIC_BIN_INST(T, DIM)                                                                                    \
    template void launch_bin_records_batch<T, DIM>(const SceneDesc<T> *, const int32_t *, int, int,                   \
                                                   const BatchQueue &, int,                                           \
                                                   hipStream_t);                                                  \
    template void launch_copy_back_batch<T, DIM>(const SceneDesc<T> *, const int32_t *, int, int, int,            \
                                                 hipStream_t);                                                    \
    template void launch_bin_scatter_copy<T, DIM>(const Parts<T> &, const Parts<T> &, const BinLists &,           \
                                                  const TileTables &, const BinScratch &, hipStream_t);           \
    template void launch_bin_keys_static<T, DIM, 1, false>(const Parts<T> &, const GridDims &, const BinLists &,  \
                                                           const BinScratch &, uint32_t *, T, hipStream_t);      \
    template void launch_bin_keys_static<T, DIM, 2, false>(const Parts<T> &, const GridDims &, const BinLists &,  \
                                                           const BinScratch &, uint32_t *, T, hipStream_t);      \
    template void launch_bin_keys_static<T, DIM, 3, false>(const Parts<T> &, const GridDims &, const BinLists &,  \
                                                           const BinScratch &, uint32_t *, T, hipStream_t);
APIC_BIN_INST(float, 2)
APIC_BIN_INST(float, 3)
APIC_BIN_INST(double, 2)
APIC_BIN_INST(double, 3)
template void launch_bin_keys_static<float, 2, 2, true>(const Parts<float> &, const GridDims &, const BinLists &,
                                                        const BinScratch &, uint32_t *, float, hipStream_t);
template void launch_bin_keys_static<float, 2, 3, true>(const Parts<float> &, const GridDims &, const BinLists &,
                                                        const BinScratch &, uint32_t *, float, hipStream_t);
template void launch_bin_keys_static<float, 3, 2, true>(const Parts<float> &, const GridDims &, const BinLists &,
                                                        const BinScratch &, uint32_t *, float, hipStream_t);
template void launch_bin_keys_static<float, 3, 3, true>(const Parts<float> &, const GridDims &, const BinLists &,
                                                        const BinScratch &, uint32_t *, float, hipStream_t);

}  // namespace apic
