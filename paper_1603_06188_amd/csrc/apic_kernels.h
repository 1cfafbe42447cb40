// Host-side launchers of the libapic kernels (definitions in apic_kernels.hip).
#pragma once

#include "apic_common.h"

namespace apic {

constexpr int kDiagBlocks = 1024;

struct SortBuffers {
    uint32_t *keys;    // n
    uint32_t *perm;    // n
    uint32_t *counts;  // G + 2: per-key counts, then exclusive starts
    uint32_t *cursor;  // G + 2
    uint32_t *sums;    // scan block sums
};

template <typename T>
void launch_fill(T *p, int64_t count, T val, hipStream_t st);

template <typename T, int DIM, int DEG, bool COMP>
void launch_p2g(const Parts<T> &P, const GridPlanes<T> &g, const StepParams<T> &prm, hipStream_t st);

template <typename T, int DIM, bool COMP>
void launch_grid_update(const GridPlanes<T> &g, const StepParams<T> &prm, hipStream_t st);

template <typename T, int DIM, int DEG>
void launch_g2p(const Parts<T> &P, const GridPlanes<T> &g, const StepParams<T> &prm, hipStream_t st);

template <typename T, int DIM, int DEG>
void launch_sort(const Parts<T> &P, const Parts<T> &shadow, const GridDims &d, const SortBuffers &sb,
                 hipStream_t st);

template <typename T, int DIM>
void launch_diag_particles(const Parts<T> &P, double dx, double *partials, double *out, hipStream_t st);

template <typename T, int DIM, bool COMP>
void launch_diag_grid(const GridPlanes<T> &g, int which, double dt, double *partials, double *out, hipStream_t st);

template <typename T, int DIM, bool COMP>
void launch_grid_export(const GridPlanes<T> &g, int field, T *out, hipStream_t st);

template <typename T, int DIM>
void launch_pack_positions(const Parts<T> &P, const double *x, double dx, hipStream_t st);

template <typename T, int DIM>
void launch_unpack_positions(const Parts<T> &P, double *x, double dx, hipStream_t st);

}  // namespace apic
