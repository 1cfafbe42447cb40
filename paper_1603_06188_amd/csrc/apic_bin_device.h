// Device helpers shared by the binning passes (apic_sort and apic_g2p).
#pragma once

#include "apic_common.h"

namespace apic {

// True for exactly one lane among the active lanes holding each value of t.
// Must be called by the whole wavefront.
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

// Appends the key's tile to the record list on first touch and takes a rank
// within the key; dead particles take a rank in the dead region.  Must be
// called by the whole wavefront (`active` false for lanes without a particle).
__device__ __forceinline__ uint32_t bin_take_slot(uint32_t key, bool active, const BinMeta &nxt,
                                                  const BinScratch &sc) {
    const bool live = active && key != kDeadKey;
    const uint32_t t = key >> 6;
    // one lane per distinct tile of the wavefront; a plain read skips the
    // atomic for tiles already listed (a stale 0 only costs the atomic)
    if (first_lane_of_value(t, live) && sc.tile_flag[t] == 0u && atomicOr(sc.tile_flag + t, 1u) == 0u) {
        const uint32_t rec = atomicAdd(nxt.count, 1u);
        nxt.tile[rec] = t;
    }
    if (!active) return 0u;
    if (key == kDeadKey) return atomicAdd(nxt.count + 1, 1u);
    return atomicAdd(sc.key_count + key, 1u);
}

// Position of a particle (key, rank) in the level-major layout `nxt`.
__device__ __forceinline__ uint32_t bin_destination(uint32_t key, uint32_t rank, const BinMeta &nxt,
                                                    const BinScratch &sc) {
    if (key == kDeadKey) return nxt.base[nxt.count[0]] + rank;
    const int32_t rec = nxt.map[key >> 6];
    const uint32_t s = nxt.base[rec] + nxt.kprefix[rec * 64 + (key & 63)] + rank;
    return sc.perm[s];
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
