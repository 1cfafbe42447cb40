/*
 * FP64 CPU oracle for one explicit APIC-MPM step.
 *
 * Method: Jiang, Schroeder, Teran, "An angular momentum conserving
 * Affine-Particle-In-Cell method" (arXiv 1603.06188).  The step is the
 * symplectic-Euler member (lambda = 0) of the grid-update family of Sec. 3.3,
 * written with the general transfers of Sec. 3.2 (particle to grid) and
 * Sec. 3.4 (grid to particle) and the interpolation weights of Sec. 3.5.
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  It is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header or table with the GPU library.
 *
 * Conventions
 *   dim d in {2,3}; degree 1 = multilinear, 2 = quadratic, 3 = cubic B-spline.
 *   The grid has n[a] cells and n[a]+1 nodes along axis a; node i sits at
 *   x_i = i * dx (origin 0).  Node linear index: ix + N0*(iy + N1*iz),
 *   N_a = n[a]+1.  Grid vectors are stored node-major: g[node*d + a].
 *   Particle vectors are stored particle-major: x[p*d + a],
 *   matrices row-major: B[p*d*d + r*d + c].
 *   All arithmetic is IEEE binary64; build with -ffp-contract=off.
 *   The transfers run on one thread unless oracle_set_threads asks for more
 *   (the CPU baseline of the benchmark): particles are then split into
 *   contiguous blocks, one per thread, and the transfer to grid sums the
 *   threads' private grids in thread order.  The tests use one thread.
 *
 * Readings of the paper that this file takes (each listed in the design notes):
 *   - N is the tensor product of the cardinal quadratic / cubic B-spline
 *     scaled by dx (Sec. 3.5 asks only for partition of unity and linear
 *     reproduction; Sec. 5.4 and 5.6 name quadratic and cubic B-splines).
 *   - grad w_ip is the gradient of N evaluated at x_p - x_i, i.e. the
 *     derivative with respect to the particle position (Sec. 3.5).
 *   - The force is minus the gradient of the potential of Sec. 3.3,
 *     f_i = -sum_p V_p P(F_p) F_p^T grad w_ip; the printed formula lacks the
 *     minus sign, which the midpoint objective of Sec. 4.1 implies.
 *   - V_p is the particle's initial volume, passed in.
 *   - Neo-Hookean energy (named, not written, in Sec. 6):
 *       Psi = mu/2 (tr(F^T F) - d) - mu ln J + lambda/2 (ln J)^2,
 *       P   = mu (F - F^{-T}) + lambda ln J F^{-T}.
 *   - Gravity and sticky walls are not in the paper: gravity adds dt*g to the
 *     grid velocity of every node with positive mass; a node inside a sticky
 *     band gets zero velocity.  A node with zero mass gets zero velocity.
 *   - Transfer variants (Sec. 2.1, Sec. 5.6): the particle-to-grid form is
 *     (m v)_ip = m_ip (v_p + C_p (x_i - x_p)) with C_p full (APIC), skew
 *     (RPIC) or zero (PIC).  The particle state keeps the APIC variable B_p
 *     with C_p = B_p D_p^{-1}; an RPIC particle stores B_p = omega_p^* D_p,
 *     and a state whose C_p is not skew is read through its rotation:
 *     omega_p = 1/2 sum eps_abc C_cb.  RPIC's grid to particle solves
 *     omega_p = K_p^{-1} l_p; the factor m_p of K_p and l_p cancels and is
 *     left out.  PIC stores B_p = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_DOMAIN (-2)     /* a particle's kernel support leaves the grid  */
#define OR_E_SINGULAR (-3)   /* D_p or F_p could not be inverted             */
#define OR_E_INVERTED (-4)   /* det F_p <= 0: ln J undefined                 */
#define OR_E_NOMEM (-5)

/* Transfer variants of Sec. 5.6: C_p full, skew or zero. */
#define OR_TRANSFER_APIC 0
#define OR_TRANSFER_RPIC 1
#define OR_TRANSFER_PIC 2

/* Threads of oracle_p2g and oracle_g2p (1: the plain serial checker). */
static int g_threads = 1;

void oracle_set_threads(int t) { g_threads = t < 1 ? 1 : t; }
int oracle_get_threads(void) { return g_threads; }

typedef struct {
    int32_t dim;       /* 2 or 3 */
    int32_t degree;    /* 1 multilinear, 2 quadratic, 3 cubic */
    int32_t n[3];      /* cells per axis */
    double dx;         /* grid spacing */
} oracle_grid;

/* ------------------------------------------------------------------------ */
/* Interpolation kernel (Sec. 3.5).                                          */
/* ------------------------------------------------------------------------ */

/* Cardinal B-spline of the given degree, argument in cell units. */
double oracle_bspline(int degree, double t)
{
    double a = fabs(t);
    if (degree == 1) return a < 1.0 ? 1.0 - a : 0.0;
    if (degree == 2) {
        if (a < 0.5) return 0.75 - a * a;
        if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
        return 0.0;
    }
    if (degree == 3) {
        if (a < 1.0) return 0.5 * a * a * a - a * a + 2.0 / 3.0;
        if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
        return 0.0;
    }
    return 0.0;
}

/* Derivative of oracle_bspline with respect to t. */
double oracle_bspline_deriv(int degree, double t)
{
    double a = fabs(t);
    double s = (t < 0.0) ? -1.0 : 1.0;
    if (degree == 1) return a < 1.0 ? -s : 0.0; /* one-sided (from above) at t = 0 */
    if (degree == 2) {
        if (a < 0.5) return -2.0 * t;
        if (a < 1.5) return -(1.5 - a) * s;
        return 0.0;
    }
    if (degree == 3) {
        if (a < 1.0) return (1.5 * a * a - 2.0 * a) * s;
        if (a < 2.0) return -0.5 * (2.0 - a) * (2.0 - a) * s;
        return 0.0;
    }
    return 0.0;
}

static double support_half_width(int degree) { return degree == 1 ? 1.0 : (degree == 2 ? 1.5 : 2.0); }

static int nodes_per_axis(const oracle_grid *g, int a) { return g->n[a] + 1; }

static int64_t node_count(const oracle_grid *g)
{
    int64_t c = 1;
    for (int a = 0; a < g->dim; ++a) c *= nodes_per_axis(g, a);
    return c;
}

static int64_t node_linear(const oracle_grid *g, const int *idx)
{
    int64_t lin = 0;
    for (int a = g->dim - 1; a >= 0; --a) lin = lin * nodes_per_axis(g, a) + idx[a];
    return lin;
}

/* One node of a particle's kernel support. */
typedef struct {
    int64_t node;      /* linear node index                               */
    double w;          /* w_ip = N(x_p - x_i)                             */
    double gw[3];      /* grad w_ip = grad N(x_p - x_i)                   */
    double xi[3];      /* node position x_i                               */
} stencil_entry;

#define MAX_STENCIL 125 /* 5^3: the cubic support with a tie on every axis */

/*
 * All grid nodes at which N(x_p - x_i) or its gradient is non-zero: along each
 * axis, the integer nodes i with |x_p/dx - i| <= support half-width.  A node
 * exactly at the support edge has zero weight and zero gradient and is kept
 * harmlessly.  Returns the entry count, or OR_E_DOMAIN when a node carrying
 * non-zero weight or gradient lies outside the grid.
 */
static int particle_stencil(const oracle_grid *g, const double *xp, stencil_entry *out)
{
    const int d = g->dim;
    const double h = support_half_width(g->degree);
    int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
    double ns[3][5], dns[3][5];
    for (int a = 0; a < d; ++a) {
        double s = xp[a] / g->dx;
        lo[a] = (int)ceil(s - h);
        int hi = (int)floor(s + h);
        cnt[a] = hi - lo[a] + 1;
        if (cnt[a] > 5 || cnt[a] < 1) return OR_E_DOMAIN;
        for (int k = 0; k < cnt[a]; ++k) {
            double t = s - (double)(lo[a] + k);
            ns[a][k] = oracle_bspline(g->degree, t);
            dns[a][k] = oracle_bspline_deriv(g->degree, t) / g->dx;
        }
    }
    int m = 0;
    int k[3];
    for (k[2] = 0; k[2] < (d == 3 ? cnt[2] : 1); ++k[2])
        for (k[1] = 0; k[1] < cnt[1]; ++k[1])
            for (k[0] = 0; k[0] < cnt[0]; ++k[0]) {
                int idx[3];
                double w = 1.0, gw[3];
                for (int a = 0; a < d; ++a) {
                    idx[a] = lo[a] + k[a];
                    w *= ns[a][k[a]];
                }
                for (int a = 0; a < d; ++a) {
                    gw[a] = dns[a][k[a]];
                    for (int b = 0; b < d; ++b)
                        if (b != a) gw[a] *= ns[b][k[b]];
                }
                int inside = 1;
                for (int a = 0; a < d; ++a)
                    if (idx[a] < 0 || idx[a] > g->n[a]) inside = 0;
                if (!inside) {
                    int zero = (w == 0.0);
                    for (int a = 0; a < d; ++a) zero = zero && (gw[a] == 0.0);
                    if (!zero) return OR_E_DOMAIN;
                    continue;
                }
                if (m >= MAX_STENCIL) return OR_E_DOMAIN;
                stencil_entry *e = &out[m++];
                e->node = node_linear(g, idx);
                e->w = w;
                for (int a = 0; a < 3; ++a) {
                    e->gw[a] = (a < d) ? gw[a] : 0.0;
                    e->xi[a] = (a < d) ? (double)idx[a] * g->dx : 0.0;
                }
            }
    return m;
}

/*
 * Weights and gradients of one particle over its support, for tests.
 * nodes[] receives linear node indices, w[] the weights, gw[] the gradients
 * (d per entry).  Returns the entry count or a negative error.
 */
int oracle_weights(const oracle_grid *g, const double *xp, int64_t *nodes, double *w, double *gw)
{
    stencil_entry st[MAX_STENCIL];
    int m = particle_stencil(g, xp, st);
    if (m < 0) return m;
    for (int j = 0; j < m; ++j) {
        nodes[j] = st[j].node;
        w[j] = st[j].w;
        for (int a = 0; a < g->dim; ++a) gw[j * g->dim + a] = st[j].gw[a];
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra (d <= 3).                                      */
/* ------------------------------------------------------------------------ */

/* Gauss-Jordan elimination with partial pivoting: inv = A^{-1}, *det = det A.
   Returns 0, or OR_E_SINGULAR when a pivot is exactly zero. */
static int mat_inverse(int d, const double *A, double *inv, double *det)
{
    double M[3][6];
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < 2 * d; ++c)
            M[r][c] = (c < d) ? A[r * d + c] : (c - d == r ? 1.0 : 0.0);
    double dt = 1.0;
    for (int col = 0; col < d; ++col) {
        int piv = col;
        for (int r = col + 1; r < d; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (M[piv][col] == 0.0) return OR_E_SINGULAR;
        if (piv != col) {
            for (int c = 0; c < 2 * d; ++c) {
                double t = M[col][c];
                M[col][c] = M[piv][c];
                M[piv][c] = t;
            }
            dt = -dt;
        }
        double p = M[col][col];
        dt *= p;
        for (int c = 0; c < 2 * d; ++c) M[col][c] /= p;
        for (int r = 0; r < d; ++r) {
            if (r == col) continue;
            double f = M[r][col];
            for (int c = 0; c < 2 * d; ++c) M[r][c] -= f * M[col][c];
        }
    }
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) inv[r * d + c] = M[r][c + d];
    if (det) *det = dt;
    return OR_OK;
}

static double mat_det(int d, const double *A)
{
    double inv[9], det = 0.0;
    if (mat_inverse(d, A, inv, &det) != OR_OK) return 0.0;
    return det;
}

/* C = A * B (d x d). */
static void mat_mul(int d, const double *A, const double *B, double *C)
{
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += A[r * d + k] * B[k * d + c];
            C[r * d + c] = s;
        }
}

static void mat_transpose(int d, const double *A, double *T)
{
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) T[c * d + r] = A[r * d + c];
}

/* ------------------------------------------------------------------------ */
/* Neo-Hookean energy density and first Piola-Kirchhoff stress (Sec. 3.1).   */
/* ------------------------------------------------------------------------ */

int oracle_neo_hookean_psi(int d, const double *F, double mu, double lam, double *psi)
{
    double Finv[9], J;
    int rc = mat_inverse(d, F, Finv, &J);
    if (rc != OR_OK) return rc;
    if (!(J > 0.0)) return OR_E_INVERTED;
    double tr = 0.0;
    for (int k = 0; k < d * d; ++k) tr += F[k] * F[k];
    double lnJ = log(J);
    *psi = 0.5 * mu * (tr - (double)d) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
    return OR_OK;
}

int oracle_neo_hookean_P(int d, const double *F, double mu, double lam, double *P)
{
    double Finv[9], FinvT[9], J;
    int rc = mat_inverse(d, F, Finv, &J);
    if (rc != OR_OK) return rc;
    if (!(J > 0.0)) return OR_E_INVERTED;
    mat_transpose(d, Finv, FinvT);
    double lnJ = log(J);
    for (int k = 0; k < d * d; ++k) P[k] = mu * (F[k] - FinvT[k]) + lam * lnJ * FinvT[k];
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Rigid rotations (Sec. 2.1).                                               */
/* ------------------------------------------------------------------------ */

static double levi_civita(int a, int b, int c);
static void cross3(int d, const double *a, const double *b, double *out);

/* The 3x3 matrix u^* with u^* y = u x y for every y. */
static void cross_matrix(const double *u, double *M)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            M[r * 3 + c] = 0.0;
            for (int a = 0; a < 3; ++a) M[r * 3 + c] += levi_civita(r, a, c) * u[a];
        }
}

/* omega with omega^* the skew part of the d x d matrix C (d = 2: about z). */
static void rotation_of(int d, const double *C, double *omega)
{
    double C3[9] = {0};
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) C3[r * 3 + c] = C[r * d + c];
    for (int a = 0; a < 3; ++a) {
        omega[a] = 0.0;
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) omega[a] += 0.5 * levi_civita(a, b, c) * C3[c * 3 + b];
    }
}

/* The d x d block of omega^*. */
static void skew_from_rotation(int d, const double *omega, double *C)
{
    double M[9];
    cross_matrix(omega, M);
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) C[r * d + c] = M[r * 3 + c];
}

/* ------------------------------------------------------------------------ */
/* Particle to grid (Sec. 3.2) and the force of Sec. 3.3 at F^{n+0} = F^n.    */
/* ------------------------------------------------------------------------ */

/*
 * For every particle: D_p = sum_i w_ip (x_i - x_p)(x_i - x_p)^T, then
 *   m_i       += w_ip m_p
 *   (m v)_i   += w_ip m_p (v_p + B_p D_p^{-1} (x_i - x_p))
 *   f_i       += -V_p P(F_p) F_p^T grad w_ip          (model == 1 only)
 * with B_p D_p^{-1} replaced by its rotation omega_p^* (RPIC, Sec. 2.1) or
 * by zero (PIC), as the transfer selects (Sec. 5.6).  Multilinear weights
 * (degree 1, Sec. 5.9): D_p can be singular, and the particle carries the
 * lagged affine matrix C_p itself, so the B planes hold C_p and
 *   (m v)_i   += w_ip m_p (v_p + C_p (x_i - x_p)).
 * Grid arrays are overwritten (zeroed first).  Particles are visited in
 * ascending order.  dp_out, when non-NULL, receives D_p (d*d per particle).
 */
/* Adds the contributions of particles [p0, p1), in ascending order, to the
 * grid arrays (which the caller zeroed). */
static int p2g_range(const oracle_grid *g, int64_t p0, int64_t p1, const double *x, const double *v,
                     const double *B, const double *F, const double *m, const double *V,
                     int model, double mu, double lam, int transfer,
                     double *gm, double *gmv, double *gf, double *dp_out)
{
    const int d = g->dim;
    stencil_entry st[MAX_STENCIL];
    for (int64_t p = p0; p < p1; ++p) {
        const double *xp = x + p * d;
        int cnt = particle_stencil(g, xp, st);
        if (cnt < 0) return cnt;
        double D[9] = {0}, Dinv[9], C[9], PFt[9] = {0};
        for (int j = 0; j < cnt; ++j)
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < d; ++c)
                    D[r * d + c] += st[j].w * (st[j].xi[r] - xp[r]) * (st[j].xi[c] - xp[c]);
        int rc = OR_OK;
        if (dp_out)
            for (int k = 0; k < d * d; ++k) dp_out[p * d * d + k] = D[k];
        if (g->degree == 1) {
            for (int k = 0; k < d * d; ++k) C[k] = B[p * d * d + k];
        } else {
            rc = mat_inverse(d, D, Dinv, NULL);
            if (rc != OR_OK) return rc;
            mat_mul(d, B + p * d * d, Dinv, C);
        }
        if (transfer == OR_TRANSFER_RPIC) {
            double omega[3];
            rotation_of(d, C, omega);
            skew_from_rotation(d, omega, C);
        } else if (transfer == OR_TRANSFER_PIC) {
            for (int k = 0; k < d * d; ++k) C[k] = 0.0;
        }
        if (model == 1) {
            double P[9], Ft[9];
            rc = oracle_neo_hookean_P(d, F + p * d * d, mu, lam, P);
            if (rc != OR_OK) return rc;
            mat_transpose(d, F + p * d * d, Ft);
            mat_mul(d, P, Ft, PFt);
        }
        for (int j = 0; j < cnt; ++j) {
            const stencil_entry *e = &st[j];
            double r[3];
            for (int a = 0; a < d; ++a) r[a] = e->xi[a] - xp[a];
            gm[e->node] += e->w * m[p];
            for (int a = 0; a < d; ++a) {
                double cr = 0.0;
                for (int b = 0; b < d; ++b) cr += C[a * d + b] * r[b];
                gmv[e->node * d + a] += e->w * m[p] * (v[p * d + a] + cr);
            }
            if (model == 1 && gf) {
                for (int a = 0; a < d; ++a) {
                    double s = 0.0;
                    for (int b = 0; b < d; ++b) s += PFt[a * d + b] * e->gw[b];
                    gf[e->node * d + a] += -V[p] * s;
                }
            }
        }
    }
    return OR_OK;
}

int oracle_p2g(const oracle_grid *g, int64_t np, const double *x, const double *v,
               const double *B, const double *F, const double *m, const double *V,
               int model, double mu, double lam, int transfer,
               double *gm, double *gmv, double *gf, double *dp_out)
{
    const int d = g->dim;
    if (d < 2 || d > 3 || g->degree < 1 || g->degree > 3 || !(g->dx > 0.0)) return OR_E_ARG;
    if (transfer < OR_TRANSFER_APIC || transfer > OR_TRANSFER_PIC) return OR_E_ARG;
    if (g->degree == 1 && transfer != OR_TRANSFER_APIC) return OR_E_ARG;
    const int64_t nn = node_count(g);
    memset(gm, 0, sizeof(double) * nn);
    memset(gmv, 0, sizeof(double) * nn * d);
    if (gf) memset(gf, 0, sizeof(double) * nn * d);
    const int T = g_threads;
    if (T <= 1 || np < 2)
        return p2g_range(g, 0, np, x, v, B, F, m, V, model, mu, lam, transfer, gm, gmv, gf, dp_out);
    /* T threads: thread t adds the contiguous particle range
     * [t np / T, (t+1) np / T) into a grid of its own; the grids are then
     * summed in thread order, so the result depends on T only through the
     * grouping of the sums. */
    const int64_t per = nn * (1 + 2 * d);
    double *priv = (double *)calloc((size_t)T * (size_t)per, sizeof(double));
    int *rcs = (int *)calloc((size_t)T, sizeof(int));
    if (!priv || !rcs) {
        free(priv);
        free(rcs);
        return OR_E_NOMEM;
    }
#pragma omp parallel for num_threads(T) schedule(static, 1)
    for (int t = 0; t < T; ++t) {
        double *pm = priv + (int64_t)t * per, *pmv = pm + nn, *pf = pmv + nn * d;
        rcs[t] = p2g_range(g, np * t / T, np * (t + 1) / T, x, v, B, F, m, V, model, mu, lam, transfer, pm,
                           pmv, gf ? pf : NULL, dp_out);
    }
    int rc = OR_OK;
    for (int t = 0; t < T && rc == OR_OK; ++t) rc = rcs[t];
    if (rc == OR_OK) {
#pragma omp parallel for num_threads(T) schedule(static)
        for (int64_t i = 0; i < nn; ++i)
            for (int t = 0; t < T; ++t) {
                const double *pm = priv + (int64_t)t * per, *pmv = pm + nn, *pf = pmv + nn * d;
                gm[i] += pm[i];
                for (int a = 0; a < d; ++a) {
                    gmv[i * d + a] += pmv[i * d + a];
                    if (gf) gf[i * d + a] += pf[i * d + a];
                }
            }
    }
    free(priv);
    free(rcs);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Grid evolution at lambda = 0 (Sec. 3.3).                                  */
/* ------------------------------------------------------------------------ */

static int node_in_band(const oracle_grid *g, const int *idx, const int32_t *band)
{
    if (!band) return 0;
    for (int a = 0; a < g->dim; ++a) {
        if (idx[a] < band[2 * a]) return 1;
        if (idx[a] > g->n[a] - band[2 * a + 1]) return 1;
    }
    return 0;
}

/*
 * v_i = (m v)_i / m_i;  vt_i = v_i + dt f_i / m_i (+ dt g);
 * xt_i = x_i + dt (lambda v_i + (1 - lambda) vt_i) with lambda = 0.
 * Nodes with m_i <= 0 get v = vt = 0.  gf may be NULL (no force).
 */
int oracle_grid_update(const oracle_grid *g, const double *gm, const double *gmv, const double *gf,
                       double dt, const double *gravity, const int32_t *band,
                       double *gv, double *gvt, double *gxt)
{
    const int d = g->dim;
    const double lambda = 0.0;
    int idx[3] = {0, 0, 0};
    for (idx[2] = 0; idx[2] < (d == 3 ? nodes_per_axis(g, 2) : 1); ++idx[2])
        for (idx[1] = 0; idx[1] < nodes_per_axis(g, 1); ++idx[1])
            for (idx[0] = 0; idx[0] < nodes_per_axis(g, 0); ++idx[0]) {
                int64_t i = node_linear(g, idx);
                int sticky = node_in_band(g, idx, band);
                for (int a = 0; a < d; ++a) {
                    double vi = 0.0, vti = 0.0;
                    if (gm[i] > 0.0) {
                        vi = gmv[i * d + a] / gm[i];
                        vti = vi + (gf ? dt * gf[i * d + a] / gm[i] : 0.0);
                        if (gravity) vti += dt * gravity[a];
                        if (sticky) vti = 0.0;
                    }
                    gv[i * d + a] = vi;
                    gvt[i * d + a] = vti;
                    gxt[i * d + a] = (double)idx[a] * g->dx + dt * (lambda * vi + (1.0 - lambda) * vti);
                }
            }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Grid to particle (Sec. 3.4), with the weights of time n.                  */
/* ------------------------------------------------------------------------ */

/*
 *   v_p' = sum_i w_ip vt_i
 *   x_p' = sum_i w_ip xt_i
 *   B_p' = 1/2 sum_i w_ip [ vt_i (x_i - x_p + xt_i - x_p')^T
 *                          + (x_i - x_p - xt_i + x_p') vt_i^T ]
 *   F_p' = (I + sum_i (xt_i - x_i) grad w_ip^T) F_p
 * for APIC.  RPIC (Sec. 2.1, its grid-to-particle step as written out in
 * Sec. 5.1) replaces B_p' by omega^* D_p with
 *   K_p = sum_i w_ip (x_i - x_p)^* (x_i - x_p)^{*T},
 *   l_p = sum_i w_ip (x_i - x_p) x vt_i,   omega = K_p^{-1} l_p
 * (vectors embedded in 3D when d = 2); PIC stores B_p' = 0.  Multilinear
 * weights (degree 1, Sec. 5.9) store the lagged C_p' = sum_i vt_i grad w_ip^T
 * (the paper's form of sum_i w_ip vt_i (D_p^{-1} (x_i - x_p))^T for these
 * weights), APIC only.
 */
int oracle_g2p(const oracle_grid *g, int64_t np, const double *x, const double *F,
               const double *gvt, const double *gxt, int transfer,
               double *x_out, double *v_out, double *B_out, double *F_out)
{
    const int d = g->dim;
    if (transfer < OR_TRANSFER_APIC || transfer > OR_TRANSFER_PIC) return OR_E_ARG;
    if (g->degree == 1 && transfer != OR_TRANSFER_APIC) return OR_E_ARG;
    /* particles are independent: with several threads each takes a block
     * of them and the results are the same bits as with one; the error of
     * the lowest failing particle is returned */
    int64_t bad = np;
    int bad_rc = OR_OK;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int64_t p = 0; p < np; ++p) {
        stencil_entry st[MAX_STENCIL];
        const double *xp = x + p * d;
        int cnt = particle_stencil(g, xp, st);
        if (cnt < 0) {
#pragma omp critical(oracle_g2p_err)
            if (p < bad) {
                bad = p;
                bad_rc = cnt;
            }
            continue;
        }
        double vn[3] = {0, 0, 0}, xn[3] = {0, 0, 0}, Bn[9] = {0}, G[9] = {0};
        for (int j = 0; j < cnt; ++j) {
            const stencil_entry *e = &st[j];
            for (int a = 0; a < d; ++a) {
                vn[a] += e->w * gvt[e->node * d + a];
                xn[a] += e->w * gxt[e->node * d + a];
            }
        }
        for (int j = 0; j < cnt; ++j) {
            const stencil_entry *e = &st[j];
            const double *vt = gvt + e->node * d;
            const double *xt = gxt + e->node * d;
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < d; ++c) {
                    double left = vt[r] * ((e->xi[c] - xp[c]) + (xt[c] - xn[c]));
                    double right = ((e->xi[r] - xp[r]) - (xt[r] - xn[r])) * vt[c];
                    Bn[r * d + c] += 0.5 * e->w * (left + right);
                    G[r * d + c] += (xt[r] - e->xi[r]) * e->gw[c];
                }
        }
        if (transfer == OR_TRANSFER_RPIC) {
            double K[9] = {0}, Kinv[9], l[3] = {0, 0, 0}, D[9] = {0}, C[9];
            for (int j = 0; j < cnt; ++j) {
                const stencil_entry *e = &st[j];
                double r3[3] = {0, 0, 0}, R[9], lr[3];
                for (int a = 0; a < d; ++a) r3[a] = e->xi[a] - xp[a];
                cross_matrix(r3, R);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        for (int c = 0; c < 3; ++c) K[a * 3 + b] += e->w * R[a * 3 + c] * R[b * 3 + c];
                cross3(d, r3, gvt + e->node * d, lr);
                for (int a = 0; a < 3; ++a) l[a] += e->w * lr[a];
                for (int r = 0; r < d; ++r)
                    for (int c = 0; c < d; ++c) D[r * d + c] += e->w * r3[r] * r3[c];
            }
            int rc = mat_inverse(3, K, Kinv, NULL);
            if (rc != OR_OK) {
#pragma omp critical(oracle_g2p_err)
                if (p < bad) {
                    bad = p;
                    bad_rc = rc;
                }
                continue;
            }
            double omega[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) omega[a] += Kinv[a * 3 + b] * l[b];
            skew_from_rotation(d, omega, C);
            mat_mul(d, C, D, Bn);
        } else if (transfer == OR_TRANSFER_PIC) {
            for (int k = 0; k < d * d; ++k) Bn[k] = 0.0;
        }
        if (g->degree == 1) {
            for (int k = 0; k < d * d; ++k) Bn[k] = 0.0;
            for (int j = 0; j < cnt; ++j)
                for (int r = 0; r < d; ++r)
                    for (int c = 0; c < d; ++c) Bn[r * d + c] += gvt[st[j].node * d + r] * st[j].gw[c];
        }
        for (int a = 0; a < d; ++a) G[a * d + a] += 1.0;
        double Fn[9];
        mat_mul(d, G, F + p * d * d, Fn);
        for (int a = 0; a < d; ++a) {
            x_out[p * d + a] = xn[a];
            v_out[p * d + a] = vn[a];
        }
        for (int k = 0; k < d * d; ++k) {
            B_out[p * d * d + k] = Bn[k];
            F_out[p * d * d + k] = Fn[k];
        }
    }
    return bad < np ? bad_rc : OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Momenta and energies (Sec. 3.1, Sec. 5.2, Sec. 5.3).                      */
/* ------------------------------------------------------------------------ */

static double levi_civita(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0.0;
    /* even permutations of (0,1,2) */
    if ((a == 0 && b == 1 && c == 2) || (a == 1 && b == 2 && c == 0) || (a == 2 && b == 0 && c == 1))
        return 1.0;
    return -1.0;
}

/* cross product embedded in 3D: a and b have d components, out has 3 */
static void cross3(int d, const double *a, const double *b, double *out)
{
    double A[3] = {0, 0, 0}, Bv[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) {
        A[k] = a[k];
        Bv[k] = b[k];
    }
    for (int c = 0; c < 3; ++c) {
        out[c] = 0.0;
        for (int a2 = 0; a2 < 3; ++a2)
            for (int b2 = 0; b2 < 3; ++b2) out[c] += levi_civita(a2, b2, c) * A[a2] * Bv[b2];
    }
}

/*
 * Particle totals: out[0..2] = p = sum m v;
 * out[3..5] = l = sum x x m v + m B^T : eps  (the B term of Sec. 5.3, with
 * (A : eps)_g = A_ab eps_abg); out[6] = kinetic energy 1/2 sum m |v|^2;
 * out[7] = total mass.  In 2D the angular momentum is out[5].
 */
void oracle_particle_totals(int d, int64_t np, const double *x, const double *v, const double *B,
                            const double *m, double *out)
{
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        double mv[3] = {0, 0, 0}, c[3];
        for (int a = 0; a < d; ++a) mv[a] = m[p] * v[p * d + a];
        cross3(d, x + p * d, mv, c);
        for (int a = 0; a < 3; ++a) {
            out[a] += mv[a];
            out[3 + a] += c[a];
        }
        if (B) {
            for (int gam = 0; gam < 3; ++gam) {
                double s = 0.0;
                for (int al = 0; al < d; ++al)
                    for (int be = 0; be < d; ++be)
                        s += B[p * d * d + be * d + al] * levi_civita(al, be, gam);
                out[3 + gam] += m[p] * s;
            }
        }
        double v2 = 0.0;
        for (int a = 0; a < d; ++a) v2 += v[p * d + a] * v[p * d + a];
        out[6] += 0.5 * m[p] * v2;
        out[7] += m[p];
    }
}

/*
 * Grid totals for velocities gvel at positions gpos (node-major, d per node):
 * p = sum m_i v_i, l = sum x_i x m_i v_i, KE, mass.  gpos NULL means x_i.
 */
void oracle_grid_totals(const oracle_grid *g, const double *gm, const double *gvel, const double *gpos,
                        double *out)
{
    const int d = g->dim;
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    int idx[3] = {0, 0, 0};
    for (idx[2] = 0; idx[2] < (d == 3 ? nodes_per_axis(g, 2) : 1); ++idx[2])
        for (idx[1] = 0; idx[1] < nodes_per_axis(g, 1); ++idx[1])
            for (idx[0] = 0; idx[0] < nodes_per_axis(g, 0); ++idx[0]) {
                int64_t i = node_linear(g, idx);
                double xi[3] = {0, 0, 0}, mv[3] = {0, 0, 0}, c[3];
                for (int a = 0; a < d; ++a) {
                    xi[a] = gpos ? gpos[i * d + a] : (double)idx[a] * g->dx;
                    mv[a] = gm[i] * gvel[i * d + a];
                }
                cross3(d, xi, mv, c);
                double v2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    out[a] += mv[a];
                    out[3 + a] += c[a];
                }
                for (int a = 0; a < d; ++a) v2 += gvel[i * d + a] * gvel[i * d + a];
                out[6] += 0.5 * gm[i] * v2;
                out[7] += gm[i];
            }
}

/* Total potential energy Phi = sum_p V_p Psi(F_p) (Sec. 3.3). */
int oracle_potential(int d, int64_t np, const double *F, const double *V, double mu, double lam,
                     double *phi)
{
    double s = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        double psi;
        int rc = oracle_neo_hookean_psi(d, F + p * d * d, mu, lam, &psi);
        if (rc != OR_OK) return rc;
        s += V[p] * psi;
    }
    *phi = s;
    return OR_OK;
}

/*
 * Largest time step the CFL rule of Sec. 4.3 admits:
 *   dt <= nu dx / max_p (|v_p| + (6 sqrt(d) / dx) |B_p|_F).
 * Returns +inf when every particle is at rest.
 */
double oracle_cfl_dt(int d, double dx, double nu, int64_t np, const double *v, const double *B)
{
    double worst = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        double vv = 0.0, bb = 0.0;
        for (int a = 0; a < d; ++a) vv += v[p * d + a] * v[p * d + a];
        for (int k = 0; k < d * d; ++k) bb += B[p * d * d + k] * B[p * d * d + k];
        double s = sqrt(vv) + 6.0 * sqrt((double)d) / dx * sqrt(bb);
        if (s > worst) worst = s;
    }
    if (worst == 0.0) return INFINITY;
    return nu * dx / worst;
}

/*
 * The same rule for multilinear weights with the lagged C_p of Sec. 5.9:
 * every grid velocity a particle contributes, v_p + C_p (x_i - x_p), has
 * |x_i - x_p| <= sqrt(d) dx, so
 *   dt <= nu dx / max_p (|v_p| + sqrt(d) dx |C_p|_F).
 */
double oracle_cfl_dt_lagged(int d, double dx, double nu, int64_t np, const double *v, const double *C)
{
    double worst = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        double vv = 0.0, cc = 0.0;
        for (int a = 0; a < d; ++a) vv += v[p * d + a] * v[p * d + a];
        for (int k = 0; k < d * d; ++k) cc += C[p * d * d + k] * C[p * d * d + k];
        double s = sqrt(vv) + sqrt((double)d) * dx * sqrt(cc);
        if (s > worst) worst = s;
    }
    if (worst == 0.0) return INFINITY;
    return nu * dx / worst;
}

/* ------------------------------------------------------------------------ */
/* One whole step: P2G, grid update, G2P.                                     */
/* ------------------------------------------------------------------------ */

/*
 * Grid outputs (node-major, caller-allocated with node_count entries times d
 * where vector-valued): gm, gmv, gf, gv, gvt, gxt.  Particle outputs: x_out,
 * v_out, B_out, F_out.  Inputs are never modified.
 */
int oracle_step(const oracle_grid *g, int64_t np, const double *x, const double *v, const double *B,
                const double *F, const double *m, const double *V, int model, double mu, double lam,
                double dt, const double *gravity, const int32_t *band, int transfer,
                double *gm, double *gmv, double *gf, double *gv, double *gvt, double *gxt,
                double *x_out, double *v_out, double *B_out, double *F_out)
{
    int rc = oracle_p2g(g, np, x, v, B, F, m, V, model, mu, lam, transfer, gm, gmv, gf, NULL);
    if (rc != OR_OK) return rc;
    rc = oracle_grid_update(g, gm, gmv, model == 1 ? gf : NULL, dt, gravity, band, gv, gvt, gxt);
    if (rc != OR_OK) return rc;
    return oracle_g2p(g, np, x, F, gvt, gxt, transfer, x_out, v_out, B_out, F_out);
}

/* ------------------------------------------------------------------------ */
/* Implicit midpoint pieces (Sec. 3.3 at lambda = 1/2, Sec. 4.1).            */
/* ------------------------------------------------------------------------ */

/*
 * Differential of the neo-Hookean first Piola-Kirchhoff stress,
 * dP = dP/dF : dF, the product the force derivative of Sec. 3.3 needs:
 * from P = mu (F - F^{-T}) + lam ln J F^{-T}, d(F^{-T}) = -F^{-T} dF^T F^{-T}
 * and d(ln J) = tr(F^{-1} dF),
 *   dP = mu dF + (mu - lam ln J) F^{-T} dF^T F^{-T} + lam tr(F^{-1} dF) F^{-T}.
 */
int oracle_neo_hookean_dP(int d, const double *F, double mu, double lam, const double *dF, double *dP)
{
    double Finv[9], FinvT[9], dFT[9], T1[9], T2[9], J;
    int rc = mat_inverse(d, F, Finv, &J);
    if (rc != OR_OK) return rc;
    if (!(J > 0.0)) return OR_E_INVERTED;
    mat_transpose(d, Finv, FinvT);
    mat_transpose(d, dF, dFT);
    mat_mul(d, FinvT, dFT, T1);
    mat_mul(d, T1, FinvT, T2);
    double tr = 0.0;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) tr += Finv[a * d + b] * dF[b * d + a];
    double lnJ = log(J);
    for (int k = 0; k < d * d; ++k) dP[k] = mu * dF[k] + (mu - lam * lnJ) * T2[k] + lam * tr * FinvT[k];
    return OR_OK;
}

/* F_hat = (I + sum_i u_i grad w_ip^T) F_p for a node displacement field u. */
static void displaced_F(int d, const stencil_entry *st, int cnt, const double *u, const double *Fp, double *Fh)
{
    double G[9] = {0};
    for (int j = 0; j < cnt; ++j)
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) G[r * d + c] += u[st[j].node * d + r] * st[j].gw[c];
    for (int a = 0; a < d; ++a) G[a * d + a] += 1.0;
    mat_mul(d, G, Fp, Fh);
}

/*
 * Grid forces and potential energy with the nodes moved to x_i + u_i
 * (Sec. 3.3): F_hat_p as above, Phi = sum_p V_p Psi(F_hat_p) and
 * f_i = -dPhi/dx_i = -sum_p V_p P(F_hat_p) F_p^T grad w_ip.  f (node-major,
 * node_count * d) is overwritten.  Returns OR_E_INVERTED when some
 * det F_hat_p <= 0 (Phi is then +infinity).
 */
int oracle_forces_at(const oracle_grid *g, int64_t np, const double *x, const double *F, const double *V,
                     double mu, double lam, const double *u, double *f, double *phi)
{
    const int d = g->dim;
    stencil_entry st[MAX_STENCIL];
    for (int64_t i = 0; i < node_count(g) * d; ++i) f[i] = 0.0;
    *phi = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        int cnt = particle_stencil(g, x + p * d, st);
        if (cnt < 0) return cnt;
        const double *Fp = F + p * d * d;
        double Fh[9], P[9], FT[9], PFT[9], psi;
        displaced_F(d, st, cnt, u, Fp, Fh);
        int rc = oracle_neo_hookean_psi(d, Fh, mu, lam, &psi);
        if (rc == OR_OK) rc = oracle_neo_hookean_P(d, Fh, mu, lam, P);
        if (rc != OR_OK) {
            *phi = INFINITY;
            return rc;
        }
        *phi += V[p] * psi;
        mat_transpose(d, Fp, FT);
        mat_mul(d, P, FT, PFT);
        for (int j = 0; j < cnt; ++j)
            for (int r = 0; r < d; ++r) {
                double s = 0.0;
                for (int c = 0; c < d; ++c) s += PFT[r * d + c] * st[j].gw[c];
                f[st[j].node * d + r] -= V[p] * s;
            }
    }
    return OR_OK;
}

/*
 * Product of the force derivative with a node vector du at the displaced
 * state (Sec. 3.3, force derivative and its helper):
 *   dF_p = (sum_j du_j grad w_jp^T) F_p,  A_p = dP/dF(F_hat_p) : dF_p,
 *   df_i = sum_j (df_i/dx_j) du_j = -sum_p V_p A_p F_p^T grad w_ip.
 * df is overwritten.
 */
int oracle_force_differential(const oracle_grid *g, int64_t np, const double *x, const double *F,
                              const double *V, double mu, double lam, const double *u, const double *du,
                              double *df)
{
    const int d = g->dim;
    stencil_entry st[MAX_STENCIL];
    for (int64_t i = 0; i < node_count(g) * d; ++i) df[i] = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        int cnt = particle_stencil(g, x + p * d, st);
        if (cnt < 0) return cnt;
        const double *Fp = F + p * d * d;
        double Fh[9], G[9] = {0}, dF[9], A[9], FT[9], AFT[9];
        displaced_F(d, st, cnt, u, Fp, Fh);
        for (int j = 0; j < cnt; ++j)
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < d; ++c) G[r * d + c] += du[st[j].node * d + r] * st[j].gw[c];
        mat_mul(d, G, Fp, dF);
        int rc = oracle_neo_hookean_dP(d, Fh, mu, lam, dF, A);
        if (rc != OR_OK) return rc;
        mat_transpose(d, Fp, FT);
        mat_mul(d, A, FT, AFT);
        for (int j = 0; j < cnt; ++j)
            for (int r = 0; r < d; ++r) {
                double s = 0.0;
                for (int c = 0; c < d; ++c) s += AFT[r * d + c] * st[j].gw[c];
                df[st[j].node * d + r] -= V[p] * s;
            }
    }
    return OR_OK;
}

/* 1 when node idx lies in the sticky band (the rule of oracle_grid_update). */
int oracle_node_in_band(const oracle_grid *g, const int *idx, const int32_t *band)
{
    return node_in_band(g, idx, band);
}

int64_t oracle_node_count(const oracle_grid *g) { return node_count(g); }

double oracle_matrix_det(int d, const double *A) { return mat_det(d, A); }
