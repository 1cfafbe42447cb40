// Shared device/host definitions of libapic (gfx950, wave64).
//
// Method: Jiang, Schroeder, Teran, "An angular momentum conserving
// Affine-Particle-In-Cell method" (arXiv 1603.06188), explicit step at
// lambda = 0 (Sec. 3.2-3.5, lambda = 0 forms of Sec. 5.7).
//
// Data layout
//   Keys.  A particle's key is its base grid node: the lowest node of its
//   kernel support (quadratic: the node below x/dx - 1/2; cubic: cell - 1).
//   Keys and nodes are grouped in tiles of 64 (4x4x4 in 3D, 8x8 in 2D); a
//   tile is handled by one wavefront, one lane per key / node.
//   Grid.  Node values (velocity planes) are stored tile-major: node
//   (x, y, z) at tile(x/4, y/4, z/4) * 64 + (x%4) + 4 (y%4) + 16 (z%4).
//   Particles.  Structure of arrays.  After binning, the particles of every
//   listed tile are contiguous and stored level by level: level j holds the
//   j-th particle of every key of the tile that has more than j particles, in
//   key order, so the wavefront that owns the tile reads each level with
//   one coalesced load per field (a tile whose busiest key holds more than
//   kMaxLevels particles is stored key by key instead).  Particles that
//   cannot be binned (support outside the grid, non-finite state) follow all
//   tiles ("dead" region).
//   Lists.  Listed tiles are kept in kBuckets append lists (bucket = tile id mod kBuckets) so appends do
//   not contend on one counter; membership is a generation tag per tile, so
//   nothing needs clearing between steps.  A tile's particles start at
//   bucket_base[bucket] + off[tile], bucket_base being the exclusive prefix
//   of the per-bucket particle totals.
//   Slabs.  P2G writes, per listed tile, the mass and momentum of the
//   (4+K-1)^3 nodes its keys touch (K = kernel support width) to the slab of
//   the tile's record index; the grid update sums the at most 8 slabs that
//   cover a node.  No float atomics anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apic.h"

namespace apic {

constexpr int kBuckets = 1024;   // 4 per thread of a 256-thread block
constexpr int kMaxLevels = 32;
constexpr int kVmaxSlots = 1024;
constexpr int kKeyChunks = 8;     // key pass: chunks of 64 particles loaded together

struct GridDims {
    int dim, deg;
    int n[3];      // cells per axis
    int N[3];      // nodes per axis = n + 1
    int TN[3];     // tiles per axis
    int64_t tiles; // tile count
    int64_t G;     // padded node count = tiles * 64
};

template <typename T>
struct Parts {
    uint32_t *cell;
    T *off, *v, *B, *F, *m;
    int32_t *id;
    int64_t n, s;  // count, plane stride
};

// Lists of one binned layout (double-buffered: the layout being read and the
// one being built).
struct BinLists {
    uint32_t gen;          // generation tag of this layout
    uint32_t *tile_gen;    // [tiles] == gen: tile listed
    uint32_t *slot;        // [tiles] record index of a listed tile (its slab; its rank in its
                           // bucket's class between the records and finalize passes)
    uint32_t *rec_count;   // [kBuckets] listed tiles per bucket
    uint32_t *nfull;       // [kBuckets] of them holding >= kFullTile particles
    uint32_t *nsparse;     // [kBuckets] the others
    uint32_t *rec_list;    // [kBuckets * rcap] tile ids, bucket b from b * rcap
    uint32_t *tot;         // [kBuckets] particles per bucket
    uint32_t *rpre;        // [kBuckets + 1] exclusive prefix of rec_count; [kBuckets] = records
    uint32_t *rec_tile;    // [records] tile id of record r (tiles of >= kFullTile particles first)
    uint32_t *bpre;        // [kBuckets + 1] exclusive prefix of tot; [kBuckets] = live particles
    uint32_t *ctr;         // [kCtrCount] counters of a build, zero when it starts
    int64_t rcap;          // list capacity per bucket: ceil(tiles / kBuckets)
};

// Counters of a build: dead particles.
enum : int { kCtrDead = 0, kCtrCount = 4 };
// Tiles of at least this many particles (four per key on average) take the
// first record numbers, so every tile walk ends with the short tiles.
constexpr uint32_t kFullTile = 4 * 64;

// Per-tile tables of one layout (dense, indexed by tile id; entries of tiles
// not listed are stale and never read).  Within a key, the particles that
// stayed keep their old order and the particles that came from other keys
// (movers) are ranked among themselves in the order of their positions in the
// layout they came from; the G2P places the stayers first (ranks [0, kcount -
// kmov)) so that they keep their levels, the fused G2P -> P2G pass the movers
// first (ranks [0, kmov), the levels its mover pass walks).  Either way a
// layout is a function of the one before it, whatever order the device's
// atomics ran in.
struct TileTables {
    uint32_t *kcount;      // [tiles * 64] particles per key
    uint32_t *kmov;        // [tiles * 64] of which movers
    uint32_t *kprefix;     // [tiles * 64] exclusive prefix of kcount in the tile
    uint32_t *maxc;        // [tiles] largest per-key count
    uint32_t *tcount;      // [tiles] particles in the tile
    uint32_t *off;         // [tiles] first particle relative to the bucket base
    uint32_t *lvl_off;     // [tiles * kMaxLevels] first particle of level j in the tile
    uint64_t *lvl_mask;    // [tiles * kMaxLevels] keys present in level j
};

// Scratch of the binning passes (counters are zero between passes).  A
// mover takes a provisional rank in its new key from a counter (the order
// the device runs its atomics in) and is pushed on its new key's list; the
// records pass walks each key's list and gives every mover its final rank:
// the number of movers into the key that precede it in the old layout's
// order.  The order value of a particle is (tile << 32 | index within the
// tile) for a re-binning (tiles sit in the particle planes in the order their
// counters ran, so absolute positions would not do) and its position for a
// binning from scratch.
struct BinScratch {
    uint32_t *key_count;  // [G]   movers entering each key
    uint32_t *scount;     // [G]   particles staying in each key
    uint32_t *head;       // [G]   list of the movers entering each key: first old position + 1 (0: none)
    uint32_t *pkey;       // [cap] new key of a mover (kDeadKey: dead)
    uint32_t *prank;      // [cap] rank of a mover within its key / among the dead
    uint32_t *next;       // [cap] next mover of the same key's list, old position + 1 (0: end)
    uint64_t *pord;       // [cap] order value of a mover
};

// Order value of the particle at index i within tile t of a layout.
__host__ __device__ __forceinline__ uint64_t tile_order(uint32_t t, uint32_t i) {
    return ((uint64_t)t << 32) | (uint64_t)i;
}

template <typename T>
struct Slabs {
    T *v;               // [records][NC * RN] (+ error terms when compensated)
    int64_t stride;     // elements per record
};

// The transfer to grid sums momenta relative to a reference velocity per
// listed key tile, uref[t] (chosen by the transfer to grid that forms the
// tile's slab): the slab holds m_i and sum w m_p (v_p - uref[t]) + ...; the
// grid update moves each slab's sums to the reference of the node tile it
// updates (a difference of two references) and adds that reference back to
// the velocity it stores.  References are multiples of kRefQuantum below
// kRefMax in magnitude, so their differences are exact in binary32, and the
// rounding of the sums scales with |v - reference| instead of |v| (a body
// that moves fast as a whole keeps the digits of its velocity differences,
// which B and grad v are made of).  Mathematically nothing changes.
constexpr float kRefQuantum = 1.0f / 1024.0f;
constexpr float kRefMax = 4096.0f;

__device__ __forceinline__ float rint_t(float x) { return __builtin_rintf(x); }
__device__ __forceinline__ double rint_t(double x) { return __builtin_rint(x); }

// Reference velocity from a velocity: rounded to a multiple of kRefQuantum;
// 0 when not finite or not below kRefMax in magnitude.
template <typename T>
__device__ __forceinline__ T quantize_ref(T x) {
    return (x == x && x < T(kRefMax) && x > -T(kRefMax)) ? rint_t(x * T(1024)) * T(kRefQuantum) : T(0);
}

template <typename T>
struct GridState {
    T *vt;              // dim planes of G nodes: updated velocity
    T *uref;            // dim planes of `tiles`: reference velocity of each listed key tile
    uint32_t *flags;
    uint32_t *vmax;     // [kVmaxSlots] binary32 bits; their max bounds max_i |vt_i|
    // [kVmaxSlots] binary64 bits; the transfer to particles raises them to
    // max_p (|v_p| + cfl_c |B_p|_F) of the state it writes (null: it does not)
    unsigned long long *cfl;
    double cfl_c;       // 6 sqrt(d) / dx (Sec. 4.3)
    GridDims d;
    T dx, inv_dx;
};

template <typename T>
struct StepParams {
    T dt;
    T g[3];
    int model;
    int transfer;  // APIC_TRANSFER_*
    int band[6];
    T mu, lam, inv_rho0;
    const double *dt_dev;  // non-null: the step's dt is *dt_dev (chosen on the device)
};

// The parameters with the step's dt resolved: a step whose dt is chosen on
// the device reads it once per kernel.
template <typename T>
__device__ __forceinline__ StepParams<T> with_step_dt(const StepParams<T> &prm) {
    StepParams<T> q = prm;
    if (prm.dt_dev) q.dt = (T)*prm.dt_dev;
    return q;
}

// Everything the step kernels need for one scene of a batch (the caller's
// particle planes and the workspace shadow, both list parities, tables,
// slabs, grid and parameters), as of the start of a batched call: the
// layout being read is lists[cur0] and the particles are in bufs[where0].
template <typename T>
struct SceneDesc {
    Parts<T> bufs[2];
    BinLists lists[2];     // gen: generation of the last build in each parity
    TileTables tab[2];
    BinScratch sc;
    Slabs<T> slabs;
    GridState<T> g;
    StepParams<T> prm;
    int64_t rc;            // record capacity
    int32_t cur0, where0;
    double dt_cap, nu_dx;  // adaptive steps: dt = min(dt_cap, nu_dx / bound)
};

// Kernels of a batched step; per kind, scene s owns work items
// [start[s], start[s + 1]) of the launch (item j: the j-th block of the
// scene's share).
enum BatchKernel : int { BK_P2G = 0, BK_GRID = 1, BK_KEYS = 2, BK_RECORDS = 3, BK_G2P = 4, BK_COPY = 5,
                         BK_FINAL = 6, BK_COUNT = 7 };

// How the blocks of a batched launch find their work items.  ctr null: one
// block per item, item = block index.  Otherwise a persistent launch: every
// block takes items from the device counter *ctr (a queue over (scene, share
// block) items) until they run out; this launch's items are the counter
// values base .. base + items - 1, and each block takes one value past them
// on its way out, so the next launch on the counter starts at base + items +
// (blocks of this launch).
struct BatchQueue {
    uint32_t *ctr;
    uint32_t base, items;
};

// Layout parities and generations at step k of a batched call: step k
// reads parity (cur0 + k) & 1 and builds the other one; the j-th build of a
// call into parity p gets generation gen0[p] + 1 + j.
struct StepParity {
    int cur, nxt, src;
    uint32_t gen_cur, gen_nxt;
};

__host__ __device__ __forceinline__ StepParity step_parity(int cur0, int where0, const uint32_t *gen0, int k) {
    StepParity sp;
    sp.cur = (cur0 + k) & 1;
    sp.nxt = sp.cur ^ 1;
    sp.src = (where0 + k) & 1;
    sp.gen_cur = k == 0 ? gen0[sp.cur] : gen0[sp.cur] + 1u + (uint32_t)((k - 1) / 2);
    sp.gen_nxt = gen0[sp.nxt] + 1u + (uint32_t)(k / 2);
    return sp;
}

enum : uint32_t {
    FLAG_OUT_OF_DOMAIN = 1u,
    FLAG_NONFINITE = 2u,
    FLAG_INVERTED = 4u,
    FLAG_CFL = 8u,
    FLAG_UNSORTED = 16u,
};

constexpr uint32_t kDeadKey = 0xFFFFFFFFu;

// The affine state a transfer carries (Sec. 5.6): all of B (APIC), its skew
// part (RPIC, Sec. 2.1: B = omega^* D with D a multiple of I) or none (PIC).
template <typename T, int DIM>
__device__ __forceinline__ void keep_affine(int transfer, T *B) {
    if (transfer == APIC_TRANSFER_RPIC) {
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            B[r * DIM + r] = T(0);
#pragma unroll
            for (int c = r + 1; c < DIM; ++c) {
                const T w = T(0.5) * (B[r * DIM + c] - B[c * DIM + r]);
                B[r * DIM + c] = w;
                B[c * DIM + r] = -w;
            }
        }
    } else if (transfer == APIC_TRANSFER_PIC) {
#pragma unroll
        for (int k = 0; k < DIM * DIM; ++k) B[k] = T(0);
    }
}

// ---------------------------------------------------------------------------
// Compile-time geometry per (DIM, DEG)
// ---------------------------------------------------------------------------
template <int DIM, int DEG>
struct Geo {
    static constexpr int TE = DIM == 3 ? 4 : 8;          // tile edge
    static constexpr int K = DEG + 1;                     // support width
    static constexpr int RE = TE + DEG;                   // slab edge (nodes)
    static constexpr int RN = DIM == 3 ? RE * RE * RE : RE * RE;
    static constexpr int NODES = DIM == 3 ? K * K * K : K * K;  // support nodes
    static constexpr int NC = 1 + DIM;                    // m, mv
};

// Order of a key tile's slab (its RE^DIM region) in global memory: 2^DIM
// blocks, block e holding the nodes that lie past the tile's own TE nodes
// (in the DEG nodes beyond it) exactly along the axes whose bit is set in e;
// blocks in increasing e, x fastest inside a block.  Block e is the part of
// the slab that node tile (key tile + e) adds up, so each gather of a node
// tile reads one contiguous run of every plane.
template <int DIM, int DEG>
struct SlabMap {
    static constexpr int TE = Geo<DIM, DEG>::TE;
    __host__ __device__ static constexpr int edge(int e, int a) { return ((e >> a) & 1) ? DEG : TE; }
    __host__ __device__ static constexpr int size(int e) {
        int s = 1;
        for (int a = 0; a < DIM; ++a) s *= edge(e, a);
        return s;
    }
    __host__ __device__ static constexpr int start(int e) {
        int s = 0;
        for (int b = 0; b < e; ++b) s += size(b);
        return s;
    }
    // position of the node at l (coordinates within block e)
    __host__ __device__ static constexpr int in_block(int e, const int *l) {
        return DIM == 3 ? start(e) + l[0] + edge(e, 0) * (l[1] + edge(e, 1) * l[2])
                        : start(e) + l[0] + edge(e, 0) * l[1];
    }
    // position of region node c (0 <= c[a] < RE)
    __host__ __device__ static int at(const int *c) {
        int e = 0, l[3] = {0, 0, 0};
        for (int a = 0; a < DIM; ++a) {
            const bool past = c[a] >= TE;
            e |= (int)past << a;
            l[a] = past ? c[a] - TE : c[a];
        }
        int pos = 0;
        for (int b = 0; b < (1 << DIM); ++b)
            if (b == e) pos = in_block(b, l);
        return pos;
    }
    // region coordinates of position j (0 <= j < RN); c is left as is for j >= RN
    __host__ __device__ static void coords(int j, int *c) {
#pragma unroll
        for (int e = 0; e < (1 << DIM); ++e) {
            if (j >= start(e) && j < start(e) + size(e)) {
                int l = j - start(e);
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    c[a] = l % edge(e, a) + (((e >> a) & 1) ? TE : 0);
                    l /= edge(e, a);
                }
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Packed cell index and tiled node index
// ---------------------------------------------------------------------------
template <int DIM>
__host__ __device__ __forceinline__ void unpack_cell(uint32_t c, int *ci) {
    if constexpr (DIM == 3) {
        ci[0] = (int)(c & 1023u);
        ci[1] = (int)((c >> 10) & 1023u);
        ci[2] = (int)(c >> 20);
    } else {
        ci[0] = (int)(c & 0xFFFFu);
        ci[1] = (int)(c >> 16);
    }
}

template <int DIM>
__host__ __device__ __forceinline__ uint32_t pack_cell(const int *ci) {
    if constexpr (DIM == 3)
        return (uint32_t)ci[0] | ((uint32_t)ci[1] << 10) | ((uint32_t)ci[2] << 20);
    else
        return (uint32_t)ci[0] | ((uint32_t)ci[1] << 16);
}

template <int DIM>
__host__ __device__ __forceinline__ int64_t tile_of(const int *c, const int *TN) {
    if constexpr (DIM == 3)
        return (int64_t)(c[0] >> 2) + (int64_t)TN[0] * ((c[1] >> 2) + (int64_t)TN[1] * (c[2] >> 2));
    else
        return (int64_t)(c[0] >> 3) + (int64_t)TN[0] * (c[1] >> 3);
}

template <int DIM>
__host__ __device__ __forceinline__ int local_of(const int *c) {
    if constexpr (DIM == 3)
        return (c[0] & 3) | ((c[1] & 3) << 2) | ((c[2] & 3) << 4);
    else
        return (c[0] & 7) | ((c[1] & 7) << 3);
}

template <int DIM>
__host__ __device__ __forceinline__ int64_t node_index(const int *c, const int *TN) {
    return tile_of<DIM>(c, TN) * 64 + local_of<DIM>(c);
}

// tile id -> coordinates of its first node / key
template <int DIM>
__host__ __device__ __forceinline__ void tile_origin(int64_t t, const int *TN, int *c) {
    // tile ids fit 32 bits: the padded node count 64 x tiles is below 2^32 (checked on the host)
    constexpr int TE = DIM == 3 ? 4 : 8;
    const uint32_t u = (uint32_t)t, n0 = (uint32_t)TN[0];
    c[0] = (int)(u % n0) * TE;
    if constexpr (DIM == 3) {
        const uint32_t r = u / n0, n1 = (uint32_t)TN[1];
        c[1] = (int)(r % n1) * TE;
        c[2] = (int)(r / n1) * TE;
    } else {
        c[1] = (int)(u / n0) * TE;
    }
}

// local index 0..63 -> offset inside the tile
template <int DIM>
__host__ __device__ __forceinline__ void local_coords(int l, int *c) {
    if constexpr (DIM == 3) {
        c[0] = l & 3;
        c[1] = (l >> 2) & 3;
        c[2] = l >> 4;
    } else {
        c[0] = l & 7;
        c[1] = l >> 3;
    }
}

// ---------------------------------------------------------------------------
// Quadratic / cubic B-spline weights along one axis (Sec. 3.5), in cell
// units, relative to the base node of the kernel support.
//
// Multilinear (Sec. 5.9): base = cell, weights 1 - u, u with u the offset;
// the derivative is taken from above at a node (base = cell).
// Quadratic: base = node below x/dx - 1/2; with c = x/dx - base - 1 in
// [-1/2, 1/2) the weights are 1/2 (1/2 - c)^2, 3/4 - c^2, 1/2 (1/2 + c)^2.
// Cubic: base = cell - 1, u = offset in [0, 1), q = 1 - u:
// q^3/6, u^3/2 - u^2 + 2/3, q^3/2 - q^2 + 2/3, u^3/6.
// w[k]: weight of node base+k; dw[k]: d w[k] / d x_p (cell units);
// r[k]: (x_{base+k} - x_p) / dx.
// ---------------------------------------------------------------------------
template <typename T, int DEG>
struct Axis {
    int base;
    T w[DEG + 1], dw[DEG + 1], r[DEG + 1];
};

template <typename T, int DEG>
__device__ __forceinline__ int base_of(int cell, T off) {
    if constexpr (DEG == 1)
        return cell;
    else if constexpr (DEG == 2)
        return off < T(0.5) ? cell - 1 : cell;
    else
        return cell - 1;
}

template <typename T, int DEG>
__device__ __forceinline__ void axis_weights(int cell, T off, Axis<T, DEG> &a) {
    if constexpr (DEG == 1) {
        a.base = cell;
        a.w[0] = T(1) - off;
        a.w[1] = off;
        a.dw[0] = T(-1);
        a.dw[1] = T(1);
        a.r[0] = -off;
        a.r[1] = T(1) - off;
    } else if constexpr (DEG == 2) {
        const T half = T(0.5);
        bool lower = off < half;
        a.base = lower ? cell - 1 : cell;
        T c = lower ? off : off - T(1);
        T l = half - c, h = half + c;
        a.w[0] = half * l * l;
        a.w[1] = T(0.75) - c * c;
        a.w[2] = half * h * h;
        a.dw[0] = -l;
        a.dw[1] = T(-2) * c;
        a.dw[2] = h;
        a.r[0] = T(-1) - c;
        a.r[1] = -c;
        a.r[2] = T(1) - c;
    } else {
        const T u = off, q = T(1) - off;
        const T u2 = u * u, q2 = q * q;
        a.base = cell - 1;
        a.w[0] = q2 * q * T(1.0 / 6.0);
        a.w[1] = T(0.5) * u2 * u - u2 + T(2.0 / 3.0);
        a.w[2] = T(0.5) * q2 * q - q2 + T(2.0 / 3.0);
        a.w[3] = u2 * u * T(1.0 / 6.0);
        a.dw[0] = T(-0.5) * q2;
        a.dw[1] = T(1.5) * u2 - T(2) * u;
        a.dw[2] = T(2) * q - T(1.5) * q2;
        a.dw[3] = T(0.5) * u2;
        a.r[0] = T(-1) - u;
        a.r[1] = -u;
        a.r[2] = T(1) - u;
        a.r[3] = T(2) - u;
    }
}

// 1 / k with D_p = k dx^2 I: k = 1/4 (quadratic), 1/3 (cubic) (Sec. 5.6).
// Multilinear D_p is not a multiple of I (and is singular on grid lines);
// that kernel carries C_p instead of B_p and never uses this.
template <typename T, int DEG>
__host__ __device__ constexpr T inv_D_factor() {
    static_assert(DEG == 2 || DEG == 3, "quadratic and cubic only");
    return DEG == 2 ? T(4) : T(3);
}

template <typename T>
__device__ __forceinline__ bool is_finite(T x) {
    return __builtin_isfinite(x);
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
    if constexpr (sizeof(T) == 4)
        return __builtin_fmaf(a, b, c);
    else
        return __builtin_fma(a, b, c);
}

template <typename T>
__device__ __forceinline__ T log_t(T x);
template <>
__device__ __forceinline__ float log_t<float>(float x) { return logf(x); }
template <>
__device__ __forceinline__ double log_t<double>(double x) { return log(x); }

template <typename T>
__device__ __forceinline__ T floor_t(T x);
template <>
__device__ __forceinline__ float floor_t<float>(float x) { return floorf(x); }
template <>
__device__ __forceinline__ double floor_t<double>(double x) { return floor(x); }

// Absolute binary32 positions (APIC_OPT_ABSOLUTE_POSITIONS): the offset
// planes hold the coordinate x_p itself, and the cell index and offset follow
// from it as a plain binary32 code computes them: s = x / dx (one rounding),
// c = floor(s), o = s - c (exact).
template <typename T>
__device__ __forceinline__ void cell_of_absolute(T x, T inv_dx, int &c, T &o) {
    const T s = x * inv_dx;
    const T f = floor_t(s);
    c = (int)f;
    o = s - f;
}

// Cell index and offset of a particle: from the packed cell and the offset
// planes, or (ABS) from the absolute coordinates in the offset planes.
template <typename T, int DIM, bool ABS>
__device__ __forceinline__ void particle_cells(uint32_t cell, const T *x, T inv_dx, int *ci, T *off) {
    if constexpr (ABS) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) cell_of_absolute(x[a], inv_dx, ci[a], off[a]);
    } else {
        unpack_cell<DIM>(cell, ci);
#pragma unroll
        for (int a = 0; a < DIM; ++a) off[a] = x[a];
    }
}

// wave64 helpers
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
// A value that is the same on every lane, held once per wavefront (scalar
// register) instead of once per lane.
__device__ __forceinline__ float wave_uniform(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double wave_uniform(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xFFFFFFFFll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ uint64_t lanes_below(int lane) { return lane == 0 ? 0ull : (~0ull >> (64 - lane)); }

// Scene of block b in a batched launch: the largest s < n with
// start[s] <= b (start ascending, start[0] = 0).  Wave-wide: the 64 lanes
// test 64 evenly spaced entries of the remaining range at once, so the
// search takes ceil(log64 n) dependent loads (two up to 4096 scenes).
__device__ __forceinline__ int scene_of_block(const int32_t *start, int n, uint32_t b) {
    const int lane = lane_id();
    int lo = 0, len = n;  // the answer lies in [lo, lo + len)
    while (len > 1) {
        const int step = (len + 63) / 64;
        const int idx = lo + lane * step;
        const uint64_t m = ballot(idx < lo + len && (uint32_t)start[idx] <= b);
        const int k = 63 - __builtin_clzll(m);  // lane 0 holds start[lo] <= b
        const int end = lo + len;
        lo += k * step;
        len = end - lo < step ? end - lo : step;
    }
    return lo;
}

// Workgroups go to the 8 XCDs round-robin (hardware block b on XCD b % 8),
// and each XCD has an L2 of its own.  This renumbering gives the blocks of
// one XCD one contiguous range of logical indices, so that neighbouring work
// items (which read the same slabs and node tiles) meet in the same L2.  It
// is a bijection of [0, nblk) for any nblk, and it only needs the blocks of a
// range to be consecutive hardware blocks.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t blk, uint32_t nblk) {
    const uint32_t c = blk % kXcds, q = nblk / kXcds, rem = nblk % kXcds;
    return c * q + (c < rem ? c : rem) + blk / kXcds;
}

// A walk over `items` work items, one per wavefront of 256-thread blocks.
// Launches are sized for the capacity, so only the first
// min(nblk, ceil(items / 4)) blocks take part, renumbered by xcd_block among
// themselves; `first` is this wave's first item (items when it has none).
// When the items outnumber the waves the walk is strided and left in
// hardware order, which spreads the extra items over all XCDs.
struct WaveWalk {
    uint32_t first, stride;
};
__device__ __forceinline__ WaveWalk wave_walk(uint32_t blk, uint32_t nblk, uint32_t items) {
    const uint32_t need = (uint32_t)(((uint64_t)items + 3u) / 4u);
    const uint32_t nb = need < nblk ? need : nblk;
    WaveWalk w;
    w.stride = nb * 4u;
    const uint32_t lb = need <= nblk ? xcd_block(blk, nb) : blk;
    w.first = blk < nb ? lb * 4u + (uint32_t)(threadIdx.x >> 6) : items;
    return w;
}

// Element of a particle plane at byte offset `boff` (index * sizeof(T)); the
// plane pointer is wave-uniform, so plane + 32-bit offset addressing keeps
// one offset register per particle for all planes.
template <typename T>
__device__ __forceinline__ T &plane_at(T *plane, uint32_t boff) {
    return *(T *)((char *)plane + boff);
}

// Exact error of a + b (Knuth two-sum).
template <typename T>
__device__ __forceinline__ T two_sum_err(T a, T b, T s) {
    T bp = s - a;
    return (a - (s - bp)) + (b - bp);
}

// Compiler and LDS ordering point between dependent rounds of one wavefront.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace apic
