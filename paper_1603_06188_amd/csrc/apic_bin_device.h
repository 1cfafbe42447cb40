// Device helpers shared by the binning passes and the kernels that read a
// binned layout.  Wave helpers must be called by all 64 lanes.
#pragma once

#include "apic_common.h"

namespace apic {

__device__ __forceinline__ uint32_t bucket_of(uint32_t tile) { return tile & (kBuckets - 1); }

// Lane b receives the exclusive prefix of v[0..kBuckets) at b; `total` the sum.
__device__ __forceinline__ uint32_t wave_bucket_prefix(const uint32_t *v, uint32_t &total, uint32_t &mine) {
    const int lane = lane_id();
    mine = v[lane];
    uint32_t inc = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    total = __shfl(inc, 63, 64);
    return inc - mine;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(x, o, 64);
        x = x > y ? x : y;
    }
    return x;
}

// Index r in [0, total) of a bucketed list -> (bucket, position in bucket),
// given every lane's exclusive prefix `pre` and count `cnt` of bucket = lane.
__device__ __forceinline__ void bucket_locate(uint32_t r, uint32_t pre, uint32_t cnt, uint32_t &bucket,
                                              uint32_t &j) {
    bucket = (uint32_t)popc64(ballot(pre + cnt <= r));
    j = r - __shfl(pre, (int)bucket, 64);
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

// Lists the key's tile in `nxt` on first touch (generation tag + bucketed
// append) and takes a rank within the key; dead particles take a rank in
// the dead region.  `active` false for lanes without a particle.
__device__ __forceinline__ uint32_t bin_take_slot(uint32_t key, bool active, const BinLists &nxt,
                                                  const BinScratch &sc) {
    const bool live = active && key != kDeadKey;
    const uint32_t t = key >> 6;
    if (first_lane_of_value(t, live) && nxt.tile_gen[t] != nxt.gen && atomicExch(nxt.tile_gen + t, nxt.gen) != nxt.gen) {
        const uint32_t b = bucket_of(t);
        const uint32_t j = atomicAdd(nxt.rec_count + b, 1u);
        nxt.rec_list[(int64_t)b * nxt.rcap + j] = t;
    }
    if (!active) return 0u;
    if (key == kDeadKey) return atomicAdd(nxt.dead, 1u);
    return atomicAdd(sc.key_count + key, 1u);
}

// Position of particle (key, rank) in the layout described by `tab`, given
// this lane's bucket base of bucket = lane (`bbase`) and the live total.
__device__ __forceinline__ uint32_t bin_destination(uint32_t key, uint32_t rank, const TileTables &tab,
                                                    uint32_t bbase, uint32_t live_total) {
    const uint32_t t = key >> 6;
    const uint32_t base = __shfl(bbase, (int)bucket_of(key == kDeadKey ? 0u : t), 64);
    if (key == kDeadKey) return live_total + rank;
    const uint32_t l = key & 63;
    const uint32_t start = base + tab.off[t];
    if (tab.maxc[t] <= (uint32_t)kMaxLevels) {
        const uint64_t mask = tab.lvl_mask[(int64_t)t * kMaxLevels + rank];
        return start + tab.lvl_off[(int64_t)t * kMaxLevels + rank] + (uint32_t)popc64(mask & lanes_below((int)l));
    }
    return start + tab.kprefix[(int64_t)t * 64 + l] + rank;
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
