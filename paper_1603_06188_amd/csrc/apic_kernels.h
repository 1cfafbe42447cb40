// Host-side launchers of the libapic kernels.
#pragma once

#include "apic_common.h"

namespace apic {

constexpr int kDiagBlocks = 1024;

// Work bounds known on the host (device-side counts are never read back).
struct Bounds {
    int64_t max_records;   // upper bound of listed tiles
    int64_t tiles;         // tile count of the grid
};

// --- generic ---------------------------------------------------------------
template <typename T>
void launch_fill(T *p, int64_t count, T val, hipStream_t st);

template <typename T, int DIM>
void launch_copy_state(const Parts<T> &src, const Parts<T> &dst, hipStream_t st);

// --- binning (apic_sort and the re-binning inside apic_g2p) ----------------
// Clears the stale entries of `nxt` and the node list, then resets counters.
void launch_bin_begin(const BinMeta &nxt, const BinScratch &sc, const Bounds &b, hipStream_t st);

// Keys of particles at their current positions (apic_sort).
template <typename T, int DIM, int DEG>
void launch_bin_keys_static(const Parts<T> &P, const GridDims &d, const BinMeta &nxt, const BinScratch &sc,
                            uint32_t *flags, hipStream_t st);

// Per-record counts, prefix sums, scan of record sizes, level-major
// destinations, tile map and node list of the next grid update.
template <int DIM>
void launch_bin_finish(const GridDims &d, const BinMeta &nxt, const BinScratch &sc, const Bounds &b,
                       hipStream_t st);

// Moves every particle to its binned position (apic_sort).
template <typename T, int DIM>
void launch_bin_scatter_copy(const Parts<T> &src, const Parts<T> &dst, const BinMeta &nxt, const BinScratch &sc,
                             hipStream_t st);

// --- transfers ----------------------------------------------------------------
template <typename T, int DIM, int DEG, bool COMP>
void launch_p2g(const Parts<T> &P, const BinMeta &cur, const Slabs<T> &slabs, const GridState<T> &g,
                const StepParams<T> &prm, const Bounds &b, hipStream_t st);

template <typename T, int DIM, int DEG, bool COMP>
void launch_grid_update(const BinMeta &cur, const BinScratch &sc, const Slabs<T> &slabs, const GridState<T> &g,
                        const StepParams<T> &prm, const Bounds &b, hipStream_t st);

// Keys of particles at their positions after G2P (first pass of apic_g2p).
template <typename T, int DIM, int DEG>
void launch_bin_keys_moved(const Parts<T> &P, const BinMeta &cur, const GridState<T> &g, const StepParams<T> &prm,
                           const BinMeta &nxt, const BinScratch &sc, hipStream_t st);

// G2P proper, writing each particle to its new binned position.
template <typename T, int DIM, int DEG>
void launch_g2p(const Parts<T> &src, const Parts<T> &dst, const BinMeta &cur, const BinMeta &nxt,
                const BinScratch &sc, const GridState<T> &g, const StepParams<T> &prm, hipStream_t st);

// --- observation ----------------------------------------------------------------
template <typename T, int DIM>
void launch_diag_particles(const Parts<T> &P, double dx, double *partials, double *out, hipStream_t st);

template <typename T, int DIM, int DEG, bool COMP>
void launch_diag_grid(const BinMeta &gm, const Slabs<T> &slabs, const GridState<T> &g, int which, double dt,
                      double *partials, double *out, hipStream_t st);

template <typename T, int DIM, int DEG, bool COMP>
void launch_grid_export(const BinMeta &gm, const Slabs<T> &slabs, const GridState<T> &g, int field, T *out,
                        hipStream_t st);

template <typename T, int DIM>
void launch_pack_positions(const Parts<T> &P, const double *x, double dx, hipStream_t st);

template <typename T, int DIM>
void launch_unpack_positions(const Parts<T> &P, double *x, double dx, hipStream_t st);

}  // namespace apic
