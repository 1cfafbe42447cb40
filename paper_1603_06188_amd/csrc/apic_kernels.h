// Host-side launchers of the libapic kernels.
#pragma once

#include "apic_common.h"

namespace apic {

constexpr int kDiagBlocks = 1024;

// --- generic ---------------------------------------------------------------
template <typename T>
void launch_fill(T *p, int64_t count, T val, hipStream_t st);

template <typename T, int DIM>
void launch_copy_state(const Parts<T> &src, const Parts<T> &dst, hipStream_t st);

// --- binning (apic_sort and the re-binning inside apic_g2p) ----------------
// Zeroes the counters of the lists a layout is about to be built in.
void launch_bin_reset(const BinLists &nxt, hipStream_t st);

// Keys of particles at their current positions (apic_sort).
template <typename T, int DIM, int DEG, bool ABS = false>
void launch_bin_keys_static(const Parts<T> &P, const GridDims &d, const BinLists &nxt, const BinScratch &sc,
                            uint32_t *flags, T inv_dx, hipStream_t st);

// Per listed tile of `nxt`: key counts and prefix sums, the tile's place in
// its bucket, its record index, level tables and the node tiles of the
// next grid update.
template <int DIM>
void launch_bin_records(const GridDims &d, const BinLists &nxt, const TileTables &tab, const BinScratch &sc,
                        int64_t max_records, hipStream_t st);

// Prefix tables (records and particle bases per bucket) of a finished layout.
void launch_bin_finalize(const BinLists &nxt, int64_t max_records, hipStream_t st);
template <typename T>
void launch_bin_finalize_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, int blocks,
                               hipStream_t st);

// Moves every particle to its binned position (apic_sort).
template <typename T, int DIM>
void launch_bin_scatter_copy(const Parts<T> &src, const Parts<T> &dst, const BinLists &nxt, const TileTables &tab,
                             const BinScratch &sc, hipStream_t st);

// --- transfers ----------------------------------------------------------------
// P2G over the layout `cur`; also zeroes the counters of `nxt` and the
// bounds of max |vt| for the grid update and re-binning that follow.
template <typename T, int DIM, int DEG, bool COMP, bool ABS = false>
void launch_p2g(const Parts<T> &P, const BinLists &cur, const BinLists &nxt, const TileTables &tab,
                const Slabs<T> &slabs, const GridState<T> &g, const StepParams<T> &prm, int64_t max_records,
                hipStream_t st);

template <typename T, int DIM, int DEG, bool COMP>
void launch_grid_update(const BinLists &cur, const Slabs<T> &slabs, const GridState<T> &g, const StepParams<T> &prm,
                        int64_t max_records, hipStream_t st);

// New keys of the particles of layout `cur` after G2P (first pass of
// apic_g2p): stayer counts per key, movers' keys and ranks, dead ranks.
template <typename T, int DIM, int DEG, bool ABS = false>
void launch_bin_keys_moved(const Parts<T> &P, const BinLists &cur, const TileTables &ctab, const GridState<T> &g,
                           const StepParams<T> &prm, const BinLists &nxt, const BinScratch &sc, int64_t max_records,
                           hipStream_t st);

// G2P proper, writing each particle to its place in layout `nxt`.
template <typename T, int DIM, int DEG, bool ABS = false>
void launch_g2p(const Parts<T> &src, const Parts<T> &dst, const BinLists &cur, const TileTables &ctab,
                const BinLists &nxt, const TileTables &ntab, const BinScratch &sc, const GridState<T> &g,
                const StepParams<T> &prm, int64_t max_records, hipStream_t st);

// G2P fused with the next step's P2G (binary32 quadratic 3D): writes each
// particle to its place in layout `nxt` and the slabs of `nxt` with the
// contributions of the particles that kept their key.
template <typename T, int DEG, bool COMP>
void launch_g2p2g(const Parts<T> &src, const Parts<T> &dst, const BinLists &cur, const TileTables &ctab,
                  const BinLists &nxt, const TileTables &ntab, const BinScratch &sc, const Slabs<T> &slabs,
                  const GridState<T> &g, const StepParams<T> &prm, int64_t max_records, hipStream_t st);

// Adds the contributions of the particles that changed key into the slabs
// of layout `nxt` (after launch_g2p2g); zeroes the bounds of max |vt| and
// the counters of layout `cur`, which the next step builds.
template <typename T, int DEG, bool COMP>
void launch_p2g_movers(const Parts<T> &P, const BinLists &cur, const BinLists &nxt, const TileTables &ntab,
                       const Slabs<T> &slabs, const GridState<T> &g, const StepParams<T> &prm, int64_t max_records,
                       hipStream_t st);

// --- batched steps: one launch per phase for every scene of a batch -------------
// `start` holds, per scene, its first work item (n + 1 entries); `k` is the
// step index within the batched call; `q` says how the `blocks` blocks of
// the launch take the items (one each, or from a device queue).
template <typename T, int DIM, int DEG, bool COMP>
void launch_p2g_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, const BatchQueue &q, int blocks,
                      hipStream_t st);
template <typename T, int DIM, int DEG, bool COMP>
void launch_grid_update_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, const BatchQueue &q,
                              int blocks, hipStream_t st);
template <typename T, int DIM, int DEG>
void launch_bin_keys_moved_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, const BatchQueue &q,
                                 int blocks, hipStream_t st);
template <typename T, int DIM>
void launch_bin_records_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, const BatchQueue &q,
                              int blocks, hipStream_t st);
template <typename T, int DIM, int DEG>
void launch_g2p_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, const BatchQueue &q, int blocks,
                      bool adapt, hipStream_t st);
// Adaptive batched steps: before each step, every scene's dt from its bound
// slots (first: the slots cleared and raised by a pass over the particles
// each scene starts the call with; blocks as the copy-back table).
template <typename T, int DIM>
void launch_adapt_dt_batch(const SceneDesc<T> *descs, const int32_t *copy_start, int n, int copy_blocks, bool first,
                           hipStream_t st);
// after k steps: scenes whose particles are in the shadow copy them back
template <typename T, int DIM>
void launch_copy_back_batch(const SceneDesc<T> *descs, const int32_t *start, int n, int k, int blocks,
                            hipStream_t st);

// The caller's B in the form the transfer carries (RPIC: skew part, PIC:
// zero), in place; nothing for APIC.
template <typename T, int DIM>
void launch_keep_affine(const Parts<T> &P, int transfer, hipStream_t st);

// --- observation ----------------------------------------------------------------
// out[k] = sum over b < nb of partials[8 b + k], k < 8, in a fixed order.
void launch_diag_final(const double *partials, int nb, double *out, hipStream_t st);

template <typename T, int DIM>
// affine: include the m_p B_p^T : eps term (not for the lagged C_p of the
// multilinear kernel)
void launch_diag_particles(const Parts<T> &P, double dx, bool affine, double *partials, double *out,
                           hipStream_t st, bool absolute = false);

// Kinetic and neo-Hookean potential energy of the particles in binary64:
// out[0] T, out[1] Phi (0 for model 0), out[2] T + Phi, out[7] mass.
template <typename T, int DIM>
void launch_diag_energy(const Parts<T> &P, int model, double mu, double lam, double rho0, double *partials,
                        double *out, hipStream_t st);

// max_p (|v_p| + c |B_p|_F) in binary64 into out[0] (Sec. 4.3; c from the
// grid's degree and dx).
template <typename T, int DIM>
void launch_cfl_bound(const Parts<T> &P, double c, double *partials, double *out, hipStream_t st);
// The same bound per block into partials[0..nb); returns nb.
template <typename T, int DIM>
int launch_cfl_partials(const Parts<T> &P, double c, double *partials, hipStream_t st);
// Adaptive step: dt = min(cap, nu_dx / max src[0..n)) (cap when the bound
// is 0) into state[0], added to state[1]; zeroes the kVmaxSlots bound slots.
void launch_adapt_dt(const double *src, int n, unsigned long long *slots, double cap, double nu_dx, double *state,
                     hipStream_t st);

template <typename T, int DIM, int DEG, bool COMP>
void launch_diag_grid(const BinLists &gm, const Slabs<T> &slabs, const GridState<T> &g, int which, double dt,
                      double *partials, double *out, hipStream_t st);

template <typename T, int DIM, int DEG, bool COMP>
void launch_grid_export(const BinLists &gm, const Slabs<T> &slabs, const GridState<T> &g, int field, T *out,
                        hipStream_t st);

template <typename T, int DIM>
void launch_pack_positions(const Parts<T> &P, const double *x, double dx, hipStream_t st, bool absolute);

template <typename T, int DIM>
void launch_unpack_positions(const Parts<T> &P, double *x, double dx, hipStream_t st, bool absolute);

// --- implicit midpoint (binary64, node vectors in tiles of 64 nodes) --------
// Node (x, y, z) has slot 64 t + l: t is its tile (4^3 nodes in 3D, 8^2 in 2D),
// l its place in the tile (x fastest).  Node vectors are component-major over
// the slots (component a of slot i at a * nodes + i).
struct MidGrid {
    int N[3];        // nodes per axis (N[2] = 1 in 2D)
    int T[3];        // tiles per axis (T[2] = 1 in 2D)
    int band[6];     // sticky band widths in nodes
    int64_t tiles;   // T[0] T[1] T[2]
    int64_t nodes;   // node slots: 64 tiles
    double dx;
};

// Host-side geometry of the tiled node layout.
MidGrid mid_grid(int dim, const int *cells, const int *band, double dx);
// Nodes in the region of one key tile (the tile plus DEG nodes up each axis).
int mid_region_nodes(int dim, int degree);
// Blocks (and block partials) of a node pass over nn node tiles.
int64_t mid_node_blocks(int64_t nn);
int64_t mid_scan_blocks(int64_t nodes);

// Particles counting-sorted by base node (key = the base node's slot; the
// particles that take no part follow every node's, at positions
// start[nodes] .. start[nodes + 1] - 1); the copies are level-major within a
// key tile: level r holds, in lane order, the r-th particle (ascending index)
// of every key of the tile with more than r.
struct MidSorted {
    uint32_t *perm;         // key-major position -> particle
    const uint32_t *start;  // nodes + 2 entries: first position of each key (and of the rest)
    uint32_t *cell;         // packed cell
    double *off;            // dim planes
    double *F;              // dim*dim planes
    double *m;
    double *mv;             // dim planes: m v
    double *M;              // dim*dim + 1 planes: m (k / dx) B for the transfer to grid, then F_hat^{-T} and
                            // mu - lambda ln J of the last force pass
    uint32_t *id;           // particle ids (the caller's, else the particle's index); null: not kept
    int64_t n;              // plane stride
    double dx;
};

// Key tiles that hold particles and the node tiles within their reach.
struct MidTiles {
    int32_t *klist;   // key tiles holding particles, ascending
    int32_t *nlist;   // node tiles that some listed key tile's region touches, ascending
    int32_t *slot;    // per tile: its index in klist, -1 when it holds no particle
    double *slab;     // per listed key tile: the sums over its region, component planes of mid_region_nodes
    int64_t nk, nn;   // list lengths (host copies)
};

// Conjugate-gradient scalars, formed and kept on the device.
struct MidCg {
    double gamma[2];  // <rc, rc>_M of the current iteration in slot it & 1 (the next one is written to the other)
    double gamma0, tol2;
    uint32_t done;    // the CG has stopped
    uint32_t stop;    // stop raised by an iteration's step kernel, made `done` by its direction kernel
    uint32_t iters;   // iterations run in the call
    uint32_t max_iters;
};

struct MidMaterial {
    double mu, lambda, rho0;
};

void launch_mid_flags_accept(uint32_t *flags, uint32_t *trial, hipStream_t st);
// Keys, counting sort and tile lists; counts[0] = nk, counts[1] = nn.
template <int DIM, int DEG>
void launch_mid_sort(const Parts<double> &P, const MidGrid &g, const MidSorted &S, const MidTiles &tl, uint32_t *key,
                     uint32_t *count, uint32_t *cursor, uint32_t *bsum, int32_t *counts, uint32_t *flags,
                     hipStream_t st);
// Level-major copies of the particles of the nk listed key tiles, and full
// copies of the particles that take no part.
template <int DIM, int DEG>
void launch_mid_sort_state(const Parts<double> &P, const MidSorted &S, const MidTiles &tl, int64_t nodes,
                           hipStream_t st);
// Transfer to grid: free-node mass mf and velocity gv.
template <int DIM, int DEG>
void launch_mid_p2g(const MidSorted &S, const MidGrid &g, const MidTiles &tl, double *mf, double *gv, hipStream_t st);
// Force evaluation at the iterate dv: the particle pass (F_hat, energy
// partials, force slabs; ev0 / ev1, when given, take the kernel's start and
// end times) and the node pass (residual r, out[0] = |r|_M^2,
// out[1] = E(dv)).
template <int DIM, int DEG>
void launch_mid_force_tiles(const MidSorted &S, const MidGrid &g, const MidTiles &tl, const MidMaterial &mat,
                            const double *gv, const double *dv, double dt, double *epart, uint32_t *flags,
                            hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <int DIM, int DEG>
void launch_mid_force_nodes(const MidGrid &g, const MidTiles &tl, bool elastic, const double *dv, double dt,
                            const double *grav, const double *mf, double *r, const double *epart, double *part,
                            double *out, hipStream_t st);
// One application of the Newton operator to the search direction pv (s = A pv): the
// particle pass (force-differential slabs) and the node pass (s and partials of <p, s>_M).
template <int DIM, int DEG>
void launch_mid_apply_tiles(const MidSorted &S, const MidGrid &g, const MidTiles &tl, const MidMaterial &mat,
                            const double *pv, MidCg *cg, hipStream_t st, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr);
template <int DIM, int DEG>
void launch_mid_apply_nodes(const MidGrid &g, const MidTiles &tl, bool elastic, const double *pv, const double *mf,
                            double dt, double *s, double *part, MidCg *cg, hipStream_t st);
template <int DIM>
void launch_mid_cg_init(const MidGrid &g, const MidTiles &tl, const double *mf, const double *r, double *delta,
                        double *rc, double *pv, double *part, MidCg *cg, double tol2, uint32_t max_iters,
                        hipStream_t st);
// CG iteration `it` after the operator application: alpha from the partials
// of <p, s>_M (part_ps), delta and rc updated, partials of <rc, rc>_M (part);
// then beta and the direction from those partials.
template <int DIM>
void launch_mid_cg_step(const MidGrid &g, const MidTiles &tl, const double *mf, const double *r, const double *pv,
                        const double *s, double *delta, double *rc, const double *part_ps, double *part, MidCg *cg,
                        int it, hipStream_t st);
template <int DIM>
void launch_mid_cg_dir(const MidGrid &g, const MidTiles &tl, const double *rc, double *pv, const double *part,
                       MidCg *cg, int it, hipStream_t st);
// out = a + alpha b on the listed node tiles (a = nullptr reads as 0).
template <int DIM>
void launch_mid_axpy(const MidGrid &g, const MidTiles &tl, const double *a, double alpha, const double *b, double *out,
                     hipStream_t st);
template <int DIM>
void launch_mid_finish(const MidGrid &g, const MidTiles &tl, const double *mf, const double *gv, const double *dv,
                       double dt, double *gvt, double *gu, hipStream_t st);
// Transfer to particles from the sorted copies (one wavefront per listed key
// tile), written to P in the sorted order; the particles outside the grid last.
template <int DIM, int DEG>
void launch_mid_g2p(const Parts<double> &P, const MidSorted &S, const MidGrid &g, const MidTiles &tl,
                    const double *gvt, const double *gu, hipStream_t st);

}  // namespace apic
