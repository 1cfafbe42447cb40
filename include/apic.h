/*
 * apic.h -- C ABI of libapic, an MI355X (gfx950) implementation of the
 * explicit Affine-Particle-In-Cell / MPM step of Jiang, Schroeder and Teran,
 * "An angular momentum conserving Affine-Particle-In-Cell method"
 * (arXiv 1603.06188).
 *
 * One step is
 *   apic_sort         (optional, every k steps)  bin particles by cell
 *   apic_p2g          Sec. 3.2 transfer to grid + fused force of Sec. 3.3
 *   apic_grid_update  Sec. 3.3 grid evolution at lambda = 0 (symplectic Euler)
 *   apic_g2p          Sec. 3.4 transfer to particles (lambda = 0 forms of Sec. 5.7)
 * and apic_step runs whole steps for one or many scenes.  Variants: the
 * affine part the transfers carry (apic_params.transfer: APIC, RPIC of
 * Sec. 2.1, PIC; Sec. 5.6), multilinear weights with the lagged affine
 * matrix (APIC_MULTILINEAR, Sec. 5.9) and steps whose dt follows the CFL
 * rule of Sec. 4.3 (APIC_OPT_ADAPTIVE_DT).
 *
 * Conventions shared by every call
 *   - Every pointer inside the structs below is a DEVICE pointer owned by the
 *     caller; the library borrows it for the duration of the call (and of the
 *     work that call enqueues).  The library never allocates device memory.
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     Every call is asynchronous on that stream except apic_diagnostics,
 *     apic_cfl_dt, apic_step_time and apic_get_flags, which synchronize it.
 *   - Errors: a call returns APIC_OK or a negative apic_status.  Argument
 *     errors are detected on the host before anything is enqueued and leave
 *     all buffers untouched; apic_last_error() then returns a message (per
 *     host thread).  Problems found on the device (a particle whose kernel
 *     support leaves the grid, a non-finite value, an inverted element) never
 *     abort: they set sticky bits in the scene's flag word (apic_get_flags)
 *     and the offending particle is skipped by the transfer that found it.
 *   - Floating point planes hold binary32 (APIC_F32) or binary64 (APIC_F64)
 *     values as selected by apic_grid_desc.precision.
 *
 * Grid: n[a] cells and n[a]+1 nodes per axis, node i at x_i = i*dx, origin 0
 * (a fixed Cartesian grid, Sec. 3.3).  A particle must keep its whole kernel
 * support inside the grid: quadratic needs 0.5 <= x/dx < n-0.5, cubic needs
 * 1 <= x/dx < n-1 on every axis.
 *
 * Particles: structure of arrays.  A "plane" is one scalar field for all n
 * particles; consecutive planes of one field are `stride` elements apart.
 * Any stride >= n works; a multiple of 64 keeps every plane on the first
 * plane's 256-byte alignment, so that the transfers' aligned runs of 64
 * particles cover whole cache lines in every plane.
 * Position = packed cell index + offset inside the cell in cell units:
 *   3D: cell = cx | cy << 10 | cz << 20   (cells per axis <= 1024)
 *   2D: cell = cx | cy << 16              (cells per axis <= 65535)
 *   x_p[a] = (c_a + off[a]) * dx, 0 <= off[a] < 1.
 */
#ifndef APIC_H
#define APIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t apic_status;
enum {
    APIC_OK = 0,
    APIC_E_INVAL = -1,        /* bad argument (message in apic_last_error)    */
    APIC_E_UNSUPPORTED = -2,  /* valid but not implemented combination        */
    APIC_E_HIP = -3,          /* a HIP runtime call failed                    */
    APIC_E_WORKSPACE = -4     /* workspace missing, misaligned or too small   */
};

/* B-spline degree (Sec. 3.5).  APIC_MULTILINEAR (Sec. 5.9): 2 nodes per
 * axis; its D_p is singular on grid lines, so the particle carries the lagged
 * affine matrix C_p in the B planes instead of B_p: the transfer to grid adds
 * w m_p (v_p + C_p (x_i - x_p)) and the transfer to particles stores
 * C_p = sum_i vt_i grad w_ip^T.  APIC transfer only; its CFL quantity is
 * |v_p| + sqrt(d) dx |C_p|_F, and the particle angular momentum of
 * apic_diagnostics has no affine term for it. */
enum { APIC_MULTILINEAR = 1, APIC_QUADRATIC = 2, APIC_CUBIC = 3 };
enum { APIC_F32 = 0, APIC_F64 = 1 };              /* element type of planes    */
enum { APIC_MODEL_NONE = 0, APIC_MODEL_NEO_HOOKEAN = 1 };

/*
 * apic_params.transfer: the affine part C_p of the particle velocity field
 * that the transfers carry (Sec. 5.6: full, skew or zero).
 *   APIC_TRANSFER_APIC  C_p = B_p D_p^{-1} (Sec. 3.2, Sec. 3.4).
 *   APIC_TRANSFER_RPIC  rigid: C_p is the angular velocity omega_p^* that
 *                       conserves the grid's angular momentum (Sec. 2.1);
 *                       B_p holds omega_p^* D_p, the skew part of what APIC
 *                       would store.
 *   APIC_TRANSFER_PIC   C_p = 0: B_p = 0.
 * apic_p2g, apic_step and apic_step_batch first put the caller's B_p in that
 * form, in place (RPIC: its skew part, PIC: zero); the transfers to
 * particles store it so.
 * Positions and F are updated the same way in all three.
 */
enum { APIC_TRANSFER_APIC = 0, APIC_TRANSFER_RPIC = 1, APIC_TRANSFER_PIC = 2 };

/* apic_grid_desc.options bits */
enum {
    APIC_OPT_COMPENSATED = 1, /* accumulate grid mass/momentum with an error
                                 term per node (two-sum), folded in by
                                 apic_grid_update                            */
    APIC_OPT_FUSED_TRANSFER = 2, /* apic_step, binary32 quadratic 3D only:
                                 the transfer to particles of each step but
                                 the last of a call also forms the next
                                 step's grid sums (Sec. 3.4 fused with
                                 Sec. 3.2); same results up to the order of
                                 the sums.  Ignored by other combinations
                                 and with APIC_OPT_ADAPTIVE_DT.              */
    APIC_OPT_ADAPTIVE_DT = 4, /* apic_step and apic_step_batch: every step
                                 of every scene chooses its own dt on the
                                 device by the CFL rule of Sec. 4.3,
                                   dt_k = min(prm.dt, prm.cfl * dx / b_k),
                                   b_k  = max_p (|v_p| + 6 sqrt(d)/dx |B_p|_F)
                                 over the state the step starts from (b_k = 0:
                                 prm.dt).  The first step of a call bounds all
                                 particles in a pass of its own; each later
                                 step takes b_k from the transfer to particles
                                 that wrote the state (fused into it,
                                 evaluated in the state's precision).  The
                                 steps' dt are read back by apic_step_time. */
    APIC_OPT_ABSOLUTE_POSITIONS = 8, /* binary32, quadratic or cubic weights,
                                 not with APIC_OPT_ADAPTIVE_DT nor in
                                 apic_step_batch: the position is held as the
                                 plain binary32 coordinate x_p in the `off`
                                 planes (world units, not cell units), the
                                 way a plain binary32 code stores it, and the
                                 kernels derive cell and offset from it
                                 (s = x / dx, c = floor(s), o = s - c) and
                                 write x + dt v back.  `cell` must still
                                 point to a plane of n entries; the library
                                 writes the derived cell there and never
                                 reads it.  A comparison mode: cell + offset
                                 keeps the position to ~2^-24 dx, this one to
                                 ~2^-24 |x| (Sec. 5.3: the particle's angular
                                 momentum uses x_p and B_p).                 */
    APIC_OPT_BATCH_GRAPH = 16   /* apic_step_batch (set on every scene): the
                                 K-step launch sequence of a call is captured
                                 in a HIP graph once per scene set, step
                                 count and launch plan, and replayed by later
                                 calls with the same set (the scene table is
                                 still written per call, ahead of the
                                 replay).  Results equal the launches'.
                                 Ignored while kernel timing is enabled.     */
};

/* Sticky device flag bits (apic_get_flags). */
enum {
    APIC_FLAG_OUT_OF_DOMAIN = 1, /* a kernel support left the grid: skipped   */
    APIC_FLAG_NONFINITE = 2,     /* NaN/Inf in a particle's state: skipped    */
    APIC_FLAG_INVERTED = 4,      /* det F <= 0: the particle's force skipped  */
    APIC_FLAG_CFL = 8,           /* a particle moved more than one cell       */
    APIC_FLAG_UNSORTED = 16      /* a particle was not where the binning put
                                    it (particle data changed without
                                    apic_sort): skipped by apic_p2g           */
};

typedef struct {
    int32_t dim;        /* 2 or 3                                        */
    int32_t degree;     /* APIC_MULTILINEAR, APIC_QUADRATIC or APIC_CUBIC */
    int32_t precision;  /* APIC_F32 or APIC_F64                          */
    int32_t options;    /* APIC_OPT_* bits                               */
    int32_t cells[3];   /* cells per axis; cells[2] ignored in 2D        */
    double dx;          /* grid spacing (> 0)                            */
} apic_grid_desc;

typedef struct {
    int64_t n;          /* particle count: 0 <= n, n * element size < 2^32  */
    int64_t stride;     /* elements between planes of one field (>= n)     */
    uint32_t *cell;     /* 1 plane, packed cell index                       */
    void *off;          /* dim planes: offset in the cell, cell units       */
    void *v;            /* dim planes: velocity v_p                         */
    void *B;            /* dim*dim planes, row-major: plane r*dim+c = B_rc  */
    void *F;            /* dim*dim planes, row-major: deformation gradient  */
    void *mass;         /* 1 plane: m_p                                     */
    int32_t *id;        /* optional (NULL): carried along by apic_sort      */
} apic_particles;

typedef struct {
    double dt;          /* time step (>= 0); dt = 0 gives pure transfers    */
    double gravity[3];  /* added to the velocity of nodes with mass         */
    int32_t model;      /* APIC_MODEL_*                                     */
    int32_t band[6];    /* sticky band width in nodes: -x,+x,-y,+y,-z,+z    */
    int32_t transfer;   /* APIC_TRANSFER_*                                  */
    double mu;          /* Lame mu of the neo-Hookean model                 */
    double lambda;      /* Lame lambda of the neo-Hookean model             */
    double rho0;        /* rest density: particle volume V_p = m_p / rho0   */
    double cfl;         /* CFL number nu of Sec. 4.3 for APIC_OPT_ADAPTIVE_DT
                           (0 < nu <= 1); prm.dt is then the largest step   */
} apic_params;

typedef struct {
    apic_grid_desc grid;
    apic_particles p;
    apic_params prm;
    void *workspace;          /* device, 256-byte aligned, caller-owned     */
    size_t workspace_bytes;   /* >= apic_workspace_bytes(grid, p.n)         */
} apic_scene;

/* Grid fields for apic_grid_export. */
enum {
    APIC_GRID_MASS = 0,       /* m_i                                 (1)     */
    APIC_GRID_MOMENTUM = 1,   /* (m v)_i + dt f_i after apic_p2g    (dim)   */
    APIC_GRID_VELOCITY = 2    /* vt_i after apic_grid_update        (dim)   */
};

/* Totals for apic_diagnostics. */
enum {
    APIC_DIAG_PARTICLES = 0,  /* p, l (with the B term of Sec. 5.3), KE, M    */
    APIC_DIAG_GRID = 1,       /* p, l, KE, M of (m v)_i + dt f_i at x_i       */
    APIC_DIAG_GRID_NEW = 2,   /* p, l, KE, M of m_i vt_i at x_i + dt vt_i     */
    APIC_DIAG_ENERGY = 3      /* energies of the particle state, see below     */
};

/*
 * Device workspace needed for a grid and up to max_particles particles.
 * *bytes receives the size.  The workspace holds the grid (mass, momentum,
 * velocity and their error terms), sort buffers, a shadow copy of the
 * particle state used when reordering, flags and reduction partials.  The
 * library keeps state across calls in it (e.g. the grid from apic_p2g is
 * what apic_grid_update reads): one workspace per scene.
 */
apic_status apic_workspace_bytes(const apic_grid_desc *grid, int64_t max_particles, size_t *bytes);

/*
 * Clears the scene's workspace (grid, flags, counters, binning state).  Call
 * once after allocating a workspace (the first call on an unknown workspace
 * also does it).
 */
apic_status apic_reset(apic_scene *scene, void *stream);

/*
 * Bins the particles in place by base grid node (the lowest node of a
 * particle's kernel support).  Base nodes are grouped in tiles of 64 (4x4x4
 * in 3D, 8x8 in 2D); the particles of a tile become contiguous and are stored
 * level by level (level j holds the j-th particle of every base node of the
 * tile with more than j particles, in node order).  Particles whose support
 * leaves the grid, or whose position is not finite, are moved after all
 * tiles and skipped by the transfers.  Every plane, and p.id when non-NULL,
 * is permuted; the order of particles sharing a base node is unspecified.
 * apic_g2p keeps the particles binned, so apic_sort is needed only after the
 * caller changes particle data or count (apic_p2g bins unbinned particles
 * itself).
 */
apic_status apic_sort(apic_scene *scene, void *stream);

/*
 * Transfer to grid, Sec. 3.2, with D_p = (dx^2/4) I (quadratic) or (dx^2/3) I
 * (cubic) (Sec. 5.6):
 *   m_i       = sum_p w_ip m_p
 *   (m v)_i   = sum_p w_ip m_p (v_p + B_p D_p^{-1} (x_i - x_p)) + dt f_i
 * where f_i = -sum_p V_p P(F_p) F_p^T grad w_ip is the force of Sec. 3.3 at
 * F^{n+lambda} = F^n (lambda = 0), fused into the momentum (model 1 only;
 * P is neo-Hookean).  Overwrites the workspace grid; no float atomics, and
 * the grid values do not depend on the order of the tiles.
 */
apic_status apic_p2g(apic_scene *scene, void *stream);

/*
 * Grid update, Sec. 3.3 at lambda = 0: for m_i > 0,
 *   vt_i = ((m v)_i + dt f_i) / m_i + dt g, zero inside sticky bands;
 * vt_i = 0 where m_i = 0.  (The grid position x~_i = x_i + dt vt_i stays
 * implicit: the grid is fixed.)
 */
apic_status apic_grid_update(apic_scene *scene, void *stream);

/*
 * Transfer to particles, Sec. 3.4, in its lambda = 0 form (Sec. 5.7), with the
 * weights of time n:
 *   v_p = sum_i w_ip vt_i
 *   B_p = sum_i w_ip vt_i (x_i - x_p)^T
 *   F_p = (I + dt sum_i vt_i grad w_ip^T) F_p
 *   x_p = x_p + dt v_p   (cell index and offset updated together)
 * Overwrites cell, off, v, B, F and re-bins the particles for the next
 * apic_p2g (particles are permuted as by apic_sort; p.id follows them).
 * Requires apic_p2g and apic_grid_update on the same particles before it.
 */
apic_status apic_g2p(apic_scene *scene, void *stream);

/*
 * Runs n_steps whole steps (P2G, grid update, G2P) for each of n_scenes
 * independent scenes (host array of scenes, each with its own workspace and
 * particles).  Equivalent to the per-call sequence above, but the particle
 * state alternates between the caller's planes and the workspace instead of
 * being copied back after every step; it ends in the caller's planes.
 * sort_every > 0 additionally re-bins from scratch every sort_every steps
 * (never needed for correctness).
 */
apic_status apic_step(apic_scene *scenes, int32_t n_scenes, int32_t n_steps, int32_t sort_every,
                      void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * steps as apic_step(scene, 1, n_steps, 0, stream) on one scene, without a
 * caller workspace.  scene->workspace and scene->workspace_bytes are
 * ignored; the library uses a device array of its own instead, one per GPU,
 * of apic_noalloc_max_bytes() bytes (128 MiB), which it holds until the
 * process ends.  The call allocates nothing: no hipMalloc, no hipFree, no
 * allocating library routine, no timing events (apic_timing_enable does not
 * apply to it).
 *   - Limit: the scene's workspace (apic_workspace_bytes for its grid and
 *     particle count) must fit in that array, else APIC_E_WORKSPACE before
 *     anything is enqueued (a 64^3-cell grid with 262,144 binary32
 *     particles fits; the 128^3 cube with 2M does not).
 *   - Every call starts from a cleared array (a fill kernel on `stream`) and
 *     bins the particles from scratch, so nothing carries over between calls;
 *     the results are those of apic_step on a freshly reset workspace.
 *   - All calls on one GPU share its array: calls whose work overlaps on the
 *     device (different streams, or threads without ordering) race and
 *     corrupt each other.  Order them on one stream.  The host part of the
 *     call is serialized by a lock.
 * Particles end in the caller's planes (binned, as after apic_step).
 */
apic_status apic_noalloc_max_bytes(size_t *bytes);
apic_status apic_step_noalloc(apic_scene *scene, int32_t n_steps, void *stream);

/*
 * Batched steps: the same computation as apic_step for n_scenes independent
 * scenes, but each phase of a step (P2G, grid update, keys, records, G2P)
 * is ONE kernel launch covering every scene, so many small scenes fill the
 * GPU and pay one launch per phase instead of one per scene.  All scenes
 * must share dim, degree, precision and options (else APIC_E_INVAL) and
 * have distinct workspaces.  `batch_ws` is a device buffer of at least
 * apic_batch_workspace_bytes(n_scenes) bytes, 256-byte aligned, owned by the
 * caller; it holds the scene table of the call, written on `stream`, so
 * calls that share a batch_ws must be ordered (same stream).  Results
 * are those of apic_step on each scene alone (same kernels; a scene never
 * reads another scene's memory).  Ends with every scene's particles in the
 * caller's planes.  Kernel timing (apic_timing_enable) records each batched
 * launch once under its phase.
 */
apic_status apic_batch_workspace_bytes(int32_t n_scenes, size_t *bytes);
apic_status apic_step_batch(apic_scene *scenes, int32_t n_scenes, int32_t n_steps, void *batch_ws,
                            size_t batch_ws_bytes, void *stream);

/*
 * Launch plans of apic_step_batch.  A plan fixes how many particles one
 * block of a scene's share covers (the share: ceil(n / particles) blocks,
 * capped per kernel) and how blocks find their work: one block per
 * (scene, share block) item, or a persistent launch of blocks_per_cu blocks
 * per compute unit that take items from a device queue until none is left.
 * Every plan computes the same results (each item's work is the same).
 *
 * By default the plan is tuned: per (precision, dim, degree, options,
 * scene-count and particle-count octaves) the first calls each run one
 * plan, timed with HIP events around their steps (each plan twice, the
 * faster time kept), and later calls use the plan with the least time per
 * particle-step.  apic_batch_set_plan(p) forces plan p for every later call
 * (-1: back to tuning).  apic_batch_plan_info describes plan p.
 * apic_batch_tuning reports, for the key a call with these scenes would
 * use, the chosen plan (-1 while tuning) and the measured nanoseconds per
 * particle-step of each plan (+inf if not measured) in ns[count].
 */
apic_status apic_batch_plan_count(int32_t *count);
apic_status apic_batch_plan_info(int32_t plan, int32_t *particles_per_block, int32_t *blocks_per_cu);
apic_status apic_batch_set_plan(int32_t plan);
apic_status apic_batch_tuning(const apic_scene *scenes, int32_t n_scenes, int32_t *plan, double *ns);

/*
 * Copies one grid field (APIC_GRID_*) into `out`, a device buffer of
 * node_count * components elements of the scene precision, component-major
 * (component c of node i at out[c*node_count + i]), nodes in the order
 * ix + N0*(iy + N1*iz), N_a = cells[a]+1.  Error terms are folded in.
 */
apic_status apic_grid_export(const apic_scene *scene, int32_t field, void *out, void *stream);

/*
 * Binary64 totals (Sec. 3.1 momenta; Sec. 5.3 particle angular momentum):
 * out[0..2] linear momentum, out[3..5] angular momentum about the origin (in
 * 2D the scalar is out[5]), out[6] kinetic energy 1/2 sum m |v|^2, out[7]
 * mass.  APIC_DIAG_ENERGY instead gives the energies of the particle state:
 * out[0] kinetic energy 1/2 sum_p m_p |v_p|^2 (Sec. 3.1, with the factor
 * 1/2), out[1] potential energy Phi = sum_p V_p Psi(F_p) of Sec. 3.3 with the
 * neo-Hookean density Psi = mu/2 (tr F^T F - d) - mu ln J + lambda/2 (ln J)^2
 * and V_p = m_p / rho0 (0 for APIC_MODEL_NONE, +inf if some det F_p <= 0),
 * out[2] = out[0] + out[1], out[3..6] = 0, out[7] mass.  `out` is a HOST
 * array of 8 doubles.  Synchronizes `stream`.
 */
apic_status apic_diagnostics(const apic_scene *scene, int32_t which, double *out, void *stream);

/*
 * Largest time step the CFL rule of Sec. 4.3 admits for the scene's current
 * particle state:
 *   *dt_out = nu * dx / max_p (|v_p| + (6 sqrt(d) / dx) |B_p|_F)
 * (the paper bounds every grid velocity the next transfer can produce by
 * that maximum; kappa dx / k = 6 sqrt(d) / dx for quadratic and cubic
 * weights; APIC_MULTILINEAR uses |v_p| + sqrt(d) dx |C_p|_F for its lagged
 * C_p), evaluated in binary64 over all n particles.  *dt_out is +inf when
 * every particle is at rest.  nu must be positive and finite.  Synchronizes
 * `stream`.
 */
apic_status apic_cfl_dt(const apic_scene *scene, double nu, double *dt_out, void *stream);

/*
 * Time advanced by the adaptive steps (APIC_OPT_ADAPTIVE_DT) of the scene
 * since its apic_reset: *t_out the sum of their dt, *dt_last the dt of the
 * most recent one (0 before any).  Host doubles.  Synchronizes `stream`.
 */
apic_status apic_step_time(const apic_scene *scene, double *dt_last, double *t_out, void *stream);

/* Reads (host *flags) / clears the sticky flag word.  get synchronizes. */
apic_status apic_get_flags(const apic_scene *scene, uint32_t *flags, void *stream);
apic_status apic_clear_flags(apic_scene *scene, void *stream);

/*
 * Converts absolute binary64 positions (device, dim planes of p.stride
 * elements) into p.cell / p.off, and back.
 */
apic_status apic_positions_from_absolute(apic_scene *scene, const double *x, void *stream);
apic_status apic_positions_to_absolute(const apic_scene *scene, double *x, void *stream);

/*
 * Kernel timing, for benchmarks.  While enabled, apic_step brackets each of
 * its phases (per scene and step), and apic_step_midpoint the particle pass
 * of each force evaluation and CG iteration, with a pair of HIP events on the
 * call's stream.  apic_timing_read waits for the recorded events, writes per phase
 * (index APIC_PHASE_*) the number of recorded launches to counts[] and their
 * mean duration in milliseconds to mean_ms[] (host arrays of
 * APIC_PHASE_COUNT entries), and forgets the records.  Events are created by
 * the library (no device memory is allocated).
 */
enum {
    APIC_PHASE_P2G = 0,          /* transfer to grid                         */
    APIC_PHASE_GRID_UPDATE = 1,  /* grid update                              */
    APIC_PHASE_BIN = 2,          /* keys at the advected positions + binning */
    APIC_PHASE_G2P = 3,          /* transfer to particles (re-binned write)  */
    APIC_PHASE_SORT = 4,         /* full re-bin from positions               */
    APIC_PHASE_MID_FORCE = 5,    /* midpoint: particle pass of a force evaluation */
    APIC_PHASE_MID_APPLY = 6,    /* midpoint: particle pass of one CG operator
                                    application (launches after the CG stopped
                                    are left out of the records)             */
    APIC_PHASE_COUNT = 7
};
apic_status apic_timing_enable(int32_t enable);
apic_status apic_timing_read(int64_t *counts, double *mean_ms);

/* Message of the last failed call on this host thread ("" if none). */
const char *apic_last_error(void);

/* Library version string. */
const char *apic_version(void);

/*
 * Implicit midpoint steps (the lambda = 1/2 member of the grid update of
 * Sec. 3.3, the integrator the paper uses for its examples), binary64 only.
 *
 * Each step: the transfer to grid of mass and momentum (Sec. 3.2); grid
 * velocities v_i = (m v)_i / m_i; then dv_i = vt_i - v_i solves the midpoint
 * equations m_i dv_i = dt f_i(x_i + dt/2 v_i + dt/4 dv_i) + dt m_i g
 * (Sec. 4.1), found as the minimizer of
 *   E(dv) = sum_i m_i/8 |dv_i|^2 - dt/4 sum_i m_i g.dv_i + Phi(x_i + dt/2 v_i + dt/4 dv_i)
 * by Newton's method: each Newton step solves
 *   (I - dt^2/4 M^{-1} df/dx) delta = -r,  r_i = dv_i - dt (f_i / m_i + g),
 * with the conjugate gradient of Sec. 4.2 in the mass inner product
 * <a, b> = sum_i m_i a_i.b_i (the operator is symmetric in it and keeps every
 * vector velocity-like), stopping at |r_cg|_M <= cg_tol |r_cg,0|_M or at
 * non-positive curvature (then the iterate so far; -r on the first
 * iteration), and is followed by a backtracking line search (halving from
 * 1, at most 30 times, until E does not increase or |r|_M decreases: near the
 * minimum E is flat to within its rounding).  Newton stops when
 * |r|_M <= newton_tol |r_0|_M.  Then vt_i = v_i + dv_i,
 * xt_i = x_i + dt (v_i + vt_i)/2, and the transfer to particles of Sec. 3.4
 * in its general form updates x, v, B, F (APIC transfer).
 *
 * Nodes without mass and nodes in the sticky band are not unknowns: they
 * keep v_i = vt_i = 0 (a sticky node does not move during the step).  The
 * force is that of the neo-Hookean model (APIC_MODEL_NEO_HOOKEAN) at
 * F_hat_p = (I + sum_i u_i grad w_ip^T) F_p, u_i = xt_i/2 - x_i/2 (its
 * derivative products use dP/dF of that model); APIC_MODEL_NONE has no force
 * (dv_i = dt g exactly).
 *
 * Precision APIC_F64, degree 2 or 3, transfer APIC, no APIC_OPT_ADAPTIVE_DT:
 * else APIC_E_UNSUPPORTED.  Particles need not be sorted.  Each step leaves
 * them in the caller's planes reordered by base node (tiles of 4^3 base
 * nodes, 8^2 in 2D), ids (when p.id is given) moving with them; particles
 * whose support leaves the grid take no part, keep their state, follow all
 * others and set APIC_FLAG_OUT_OF_DOMAIN in stats->flags.  The scene's
 * workspace must hold apic_midpoint_workspace_bytes (node vectors over tiles
 * of 64 nodes, per-particle sorted copies, per-tile slabs); the step uses it
 * as scratch, so the explicit entry points see a fresh workspace afterwards
 * (their binning and grid are rebuilt on their next call).  The CG's scalars
 * stay on the device; the call synchronizes the stream once per step (tile
 * counts), once per energy evaluation (E and |r|_M for the line search) and
 * when it looks at the CG's stop flag (first after 8 iterations, then after
 * the iterations the convergence rate so far says are left).  A trial iterate with some
 * det F_hat <= 0 has E = +inf and the line search halves it (it is never
 * accepted while a halving is left); APIC_FLAG_INVERTED is raised only when
 * an accepted iterate (the start of a step, or the 30th trial) is inverted.
 */
typedef struct {
    double newton_tol;   /* relative Newton tolerance, 0 = default 1e-10      */
    double cg_tol;       /* relative CG tolerance, 0 = default 1e-8            */
    int32_t max_newton;  /* Newton iterations per step, 0 = default 20         */
    int32_t max_cg;      /* CG iterations per Newton step, 0 = default 500     */
} apic_midpoint_opts;

typedef struct {
    int32_t newton_iters;   /* summed over the steps of the call             */
    int32_t cg_iters;       /* summed over the steps of the call             */
    int32_t halvings;       /* line-search halvings, summed                  */
    int32_t converged;      /* 1 when every step met newton_tol              */
    uint32_t flags;         /* APIC_FLAG_* raised during the call            */
    int32_t reserved;
    double res0;            /* |r|_M at dv = 0, last step                     */
    double res;             /* |r|_M at the end, last step                    */
} apic_midpoint_stats;

/* Workspace bytes apic_step_midpoint needs for a grid and particle count. */
apic_status apic_midpoint_workspace_bytes(const apic_grid_desc *grid, int64_t max_particles, size_t *bytes);

/* n_steps implicit midpoint steps of dt = prm.dt.  opts may be NULL
 * (defaults); stats receives the solver counts (required). */
apic_status apic_step_midpoint(apic_scene *scene, int32_t n_steps, const apic_midpoint_opts *opts,
                               apic_midpoint_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* APIC_H */
