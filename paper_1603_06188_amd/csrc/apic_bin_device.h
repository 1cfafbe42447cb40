// Device helpers shared by the binning passes and the kernels that read a
// binned layout.  Wave helpers must be called by all 64 lanes.
#pragma once

#include "apic_common.h"

namespace apic {

__device__ __forceinline__ uint32_t bucket_of(uint32_t tile) { return tile & (kBuckets - 1); }

// Block-wide (every thread of a 256-thread block must call): exclusive
// prefix sums of the per-bucket counts v[0..kBuckets) into the LDS table
// pre[0..kBuckets); returns the total.  Thread i owns buckets [4i, 4i + 4);
// `part` is LDS scratch of 4 words.
__device__ __forceinline__ uint32_t block_bucket_prefix(const uint32_t *v, uint32_t *pre, uint32_t *part) {
    static_assert(kBuckets == 4 * 256, "one uint4 of buckets per thread");
    const int tid = (int)threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint4 q = ((const uint4 *)v)[tid];
    const uint32_t own = q.x + q.y + q.z + q.w;
    uint32_t inc = own;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) part[w] = inc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) before += k < w ? part[k] : 0u;
    const uint32_t total = part[0] + part[1] + part[2] + part[3];
    const uint32_t e = before + inc - own;
    pre[4 * tid + 0] = e;
    pre[4 * tid + 1] = e + q.x;
    pre[4 * tid + 2] = e + q.x + q.y;
    pre[4 * tid + 3] = e + q.x + q.y + q.z;
    __syncthreads();
    return total;
}

// Bucket of list index r (r below the table's total): the last bucket whose
// exclusive prefix is <= r (it holds r).  Wave-wide, r wave-uniform.
__device__ __forceinline__ uint32_t bucket_find(const uint32_t *pre, uint32_t r) {
    const int lane = lane_id();
    const int grp = popc64(ballot(pre[16 * lane] <= r)) - 1;
    const uint64_t m = ballot(lane < 16 && pre[16 * grp + lane] <= r);
    return (uint32_t)(16 * grp + popc64(m) - 1);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(x, o, 64);
        x = x > y ? x : y;
    }
    return x;
}

// True for exactly one lane among the active lanes holding each value of t.
__device__ __forceinline__ bool first_lane_of_value(uint32_t t, bool active) {
    const int lane = lane_id();
    uint64_t pending = ballot(active);
    bool leader = false;
    while (pending) {
        const int first = __ffsll((unsigned long long)pending) - 1;
        const uint32_t tf = __shfl(t, first, 64);
        pending &= ~ballot(active && t == tf);
        leader = leader || lane == first;
    }
    return leader;
}

// Base of the bucket of `key` from a block table of bucket bases.
__device__ __forceinline__ uint32_t bucket_base_of(uint32_t key, const uint32_t *bases) {
    return key == kDeadKey ? 0u : bases[bucket_of(key >> 6)];
}

// Position of particle (key, rank) in the layout described by `tab`, given
// the base of the key's bucket and the live total (dead particles follow it).
__device__ __forceinline__ uint32_t bin_destination(uint32_t key, uint32_t rank, const TileTables &tab,
                                                    uint32_t base, uint32_t live_total) {
    if (key == kDeadKey) return live_total + rank;
    const uint32_t t = key >> 6, l = key & 63;
    const uint32_t start = base + tab.off[t];
    if (tab.maxc[t] <= (uint32_t)kMaxLevels) {
        const uint64_t mask = tab.lvl_mask[(int64_t)t * kMaxLevels + rank];
        return start + tab.lvl_off[(int64_t)t * kMaxLevels + rank] + (uint32_t)popc64(mask & lanes_below((int)l));
    }
    return start + tab.kprefix[(int64_t)t * 64 + l] + rank;
}

// Appends tile t to its bucket's list of `nxt`.
__device__ __forceinline__ void append_tile(uint32_t t, const BinLists &nxt) {
    const uint32_t b = bucket_of(t);
    const uint32_t j = atomicAdd(nxt.rec_count + b, 1u);
    nxt.rec_list[(int64_t)b * nxt.rcap + j] = t;
}

// Lists tile t in `nxt` unless already listed in this generation.
__device__ __forceinline__ void list_tile(uint32_t t, const BinLists &nxt) {
    if (nxt.tile_gen[t] != nxt.gen && atomicExch(nxt.tile_gen + t, nxt.gen) != nxt.gen) append_tile(t, nxt);
}

// Index of the jj-th particle of a lane's key within a listed tile: level-
// major (start + offset of level jj + rank among the keys present in it,
// given the running level offset and the level's key mask), or key-major
// (kstart + jj) for tiles whose busiest key holds more than kMaxLevels.
__device__ __forceinline__ int64_t particle_at(uint32_t start, uint32_t kstart, uint32_t level, uint64_t mask,
                                               uint32_t jj, uint32_t maxc, int lane) {
    return maxc > (uint32_t)kMaxLevels ? (int64_t)kstart + jj
                                       : (int64_t)start + level + (uint32_t)popc64(mask & lanes_below(lane));
}

// Listed tiles of a finished layout, enumerated as records r = 0, 1, ... in
// bucket order, with the bases of its particle buckets (prefix tables written
// once per layout by the finalize pass).
struct TileWalk {
    const uint32_t *rpre, *bbase;  // [kBuckets] record prefix, particle base per bucket
    uint32_t nrec, live;           // records, live particles
};

__device__ __forceinline__ TileWalk tile_walk(const BinLists &lists) {
    TileWalk w;
    w.rpre = lists.rpre;
    w.bbase = lists.bpre;
    w.nrec = lists.rpre[kBuckets];
    w.live = lists.bpre[kBuckets];
    return w;
}

// Record r of the walk: tile id, first particle and particle count.
__device__ __forceinline__ uint32_t tile_range(const TileWalk &w, uint32_t r, const BinLists &lists,
                                               const TileTables &tab, uint32_t &start, uint32_t &total) {
    const uint32_t t = lists.rec_tile[r];
    start = w.bbase[bucket_of(t)] + tab.off[t];
    total = tab.tcount[t];
    return t;
}

// Record r of the walk: tile id, first particle, this lane's key count,
// busiest key count and (busy tiles) first particle of this lane's key.
__device__ __forceinline__ uint32_t tile_of_record(const TileWalk &w, uint32_t r, const BinLists &lists,
                                                   const TileTables &tab, uint32_t &start, uint32_t &cnt,
                                                   uint32_t &maxc, uint32_t &kstart) {
    const int lane = lane_id();
    const uint32_t t = lists.rec_tile[r];
    start = w.bbase[bucket_of(t)] + tab.off[t];
    cnt = tab.kcount[(int64_t)t * 64 + lane];
    maxc = tab.maxc[t];
    kstart = maxc > (uint32_t)kMaxLevels ? start + tab.kprefix[(int64_t)t * 64 + lane] : 0u;
    return t;
}

// Lists the key's tile in `nxt` on first touch (generation tag + bucketed
// append), takes a provisional rank within the key and pushes the mover (old
// position p, order value ord) on the key's list for its final rank; dead
// particles take a rank in the dead region.  `active` false for lanes
// without a particle.  Wave-wide.
__device__ __forceinline__ uint32_t bin_take_slot(uint32_t key, bool active, uint32_t p, uint64_t ord,
                                                  const BinLists &nxt, const BinScratch &sc) {
    const bool live = active && key != kDeadKey;
    const uint32_t t = key >> 6;
    // the rank and list atomics are issued before the tile listing, whose
    // probe and claim depend on each other, so their round trips overlap
    uint32_t rank = 0u;
    if (active) {
        if (key == kDeadKey) {
            rank = atomicAdd(nxt.ctr + kCtrDead, 1u);
        } else {
            sc.pord[p] = ord;
            const uint32_t nx = atomicExch(sc.head + key, p + 1u);
            rank = atomicAdd(sc.key_count + key, 1u);
            sc.next[p] = nx;
        }
    }
    if (first_lane_of_value(t, live)) list_tile(t, nxt);
    return rank;
}

// Final ranks of the n movers on a key's list (head: first old position +
// 1): each mover's rank is the number of movers on the list with a smaller
// order value.  Clears the list.
__device__ __forceinline__ void rank_movers(uint32_t *head, uint32_t n, const BinScratch &sc) {
    const uint32_t h = *head;
    if (!h) return;
    *head = 0u;
    if (n == 1u) {
        sc.prank[h - 1] = 0u;
        return;
    }
    for (uint32_t a = h; a; a = sc.next[a - 1]) {
        const uint64_t oa = sc.pord[a - 1];
        uint32_t r = 0u;
        for (uint32_t b = h; b; b = sc.next[b - 1]) r += sc.pord[b - 1] < oa ? 1u : 0u;
        sc.prank[a - 1] = r;
    }
}

// One scene's view of step k of a batched launch: its descriptor, the lists
// being read and built (with their generations) and its share of blocks.
template <typename T>
struct BatchStep {
    const SceneDesc<T> *d;
    StepParity sp;
    BinLists cur, nxt;
    uint32_t blk, nblk;
};

// Runs fn(item) for the block's work items: item blockIdx.x, or (QUEUE)
// items taken from the device counter until none is left.  The taken item
// passes through LDS behind block barriers, so every thread of the block
// takes part.  (Two kernels rather than one with a run-time test: the loop
// keeps more registers live than the one-item body needs.)
template <bool QUEUE, typename Fn>
__device__ __forceinline__ void batch_items(const BatchQueue &q, Fn &&fn) {
    if constexpr (!QUEUE) {
        fn((uint32_t)blockIdx.x);
    } else {
        __shared__ uint32_t item;
        for (;;) {
            __syncthreads();
            if (threadIdx.x == 0) item = atomicAdd(q.ctr, 1u) - q.base;
            __syncthreads();
            const uint32_t it = item;
            if (it >= q.items) break;
            fn(it);
        }
    }
}

template <typename T>
__device__ __forceinline__ BatchStep<T> batch_step(const SceneDesc<T> *descs, const int32_t *start, int n, int k,
                                                   uint32_t item) {
    BatchStep<T> b;
    const int s = scene_of_block(start, n, item);
    b.d = descs + s;
    const uint32_t gen0[2] = {b.d->lists[0].gen, b.d->lists[1].gen};
    b.sp = step_parity(b.d->cur0, b.d->where0, gen0, k);
    b.cur = b.d->lists[b.sp.cur];
    b.cur.gen = b.sp.gen_cur;
    b.nxt = b.d->lists[b.sp.nxt];
    b.nxt.gen = b.sp.gen_nxt;
    b.blk = item - (uint32_t)start[s];
    b.nblk = (uint32_t)(start[s + 1] - start[s]);
    return b;
}

// Key (base node) of a particle at cell `ci`, offset `off`, or kDeadKey when
// its support leaves the grid or the offset is not finite.
template <typename T, int DIM, int DEG>
__device__ __forceinline__ uint32_t key_of(const int *ci, const T *off, const GridDims &d, bool &finite) {
    int base[3] = {0, 0, 0};
    bool inside = true;
    finite = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        finite = finite && is_finite(off[a]);
        base[a] = base_of<T, DEG>(ci[a], off[a]);
        inside = inside && base[a] >= 0 && base[a] + DEG <= d.n[a];
    }
    return (finite && inside) ? (uint32_t)node_index<DIM>(base, d.TN) : kDeadKey;
}

}  // namespace apic
