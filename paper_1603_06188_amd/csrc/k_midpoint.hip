// Implicit midpoint step (the lambda = 1/2 member of the grid update of
// Sec. 3.3), solved as the minimization of Sec. 4.1 with Newton's method and
// the mass-inner-product conjugate gradient of Sec. 4.2.  Binary64 throughout.
//
// Layout: dense node arrays (node ix + N0 (iy + N1 iz)), component-major
// vectors (component a of node i at a * nodes + i).  Particle kernels run one
// thread per particle in the caller's order (no binning) and scatter with
// binary64 atomics; node kernels run one thread per node and leave one
// partial sum per block, summed in a fixed order by k_mid_reduce.
#include "apic_kernels.h"

namespace apic {

namespace {

constexpr int kMidBlock = 256;

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * kMidBlock + threadIdx.x; }

// Particle of thread t in the scattering kernels: (t * pstride) mod n with
// pstride coprime to n (a bijection).  Particles stored cell by cell put the
// lanes of a wave on the same few nodes, whose binary64 atomics then
// serialize; the stride spreads a wave's lanes over the whole body.
__device__ __forceinline__ int64_t spread(int64_t t, const MidGrid &g, int64_t n) { return (t * g.pstride) % n; }

// Sum of K values over the block; thread 0 writes them to part[blockIdx * K].
template <int K>
__device__ __forceinline__ void block_partials(double (&acc)[K], double *part) {
    __shared__ double red[K][kMidBlock / 64];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double v = acc[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        acc[k] = v;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[k][wave] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < kMidBlock / 64; ++w) s += red[k][w];
            part[(int64_t)blockIdx.x * K + k] = s;
        }
}

template <int DIM>
__device__ __forceinline__ void node_coords(int64_t i, const MidGrid &g, int *c) {
    c[0] = (int)(i % g.N[0]);
    const int64_t q = i / g.N[0];
    if constexpr (DIM == 3) {
        c[1] = (int)(q % g.N[1]);
        c[2] = (int)(q / g.N[1]);
    } else {
        c[1] = (int)q;
    }
}

// Per-axis weights of particle p; false when its support leaves the grid.
template <int DIM, int DEG>
__device__ __forceinline__ bool particle_axes(const Parts<double> &P, int64_t p, const MidGrid &g,
                                              Axis<double, DEG> (&ax)[DIM]) {
    int ci[3];
    unpack_cell<DIM>(P.cell[p], ci);
    bool ok = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        axis_weights<double, DEG>(ci[a], P.off[a * P.s + p], ax[a]);
        ok = ok && ax[a].base >= 0 && ax[a].base + DEG < g.N[a];
    }
    return ok;
}

// Visits the support: f(node index, w, grad w (cell units), r (cell units)).
template <int DIM, int DEG, typename Fn>
__device__ __forceinline__ void for_support(const Axis<double, DEG> (&ax)[DIM], const MidGrid &g, Fn &&fn) {
    constexpr int K = DEG + 1;
    if constexpr (DIM == 3) {
        // z rows one at a time: unrolling all K^3 nodes hoists every load
#pragma unroll 1
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double wyz = ax[1].w[j] * ax[2].w[k];
                const int64_t row = (int64_t)g.N[0] * ((ax[1].base + j) + (int64_t)g.N[1] * (ax[2].base + k));
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const double w = ax[0].w[i] * wyz;
                    const double gw[3] = {ax[0].dw[i] * wyz, ax[0].w[i] * ax[1].dw[j] * ax[2].w[k],
                                          ax[0].w[i] * ax[1].w[j] * ax[2].dw[k]};
                    const double r[3] = {ax[0].r[i], ax[1].r[j], ax[2].r[k]};
                    fn(row + ax[0].base + i, w, gw, r);
                }
            }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t row = (int64_t)g.N[0] * (ax[1].base + j);
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const double w = ax[0].w[i] * ax[1].w[j];
                const double gw[2] = {ax[0].dw[i] * ax[1].w[j], ax[0].w[i] * ax[1].dw[j]};
                const double r[2] = {ax[0].r[i], ax[1].r[j]};
                fn(row + ax[0].base + i, w, gw, r);
            }
        }
    }
}

template <int DIM>
__device__ __forceinline__ void mat_mul(const double *A, const double *B, double *C) {
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) s += A[r * DIM + k] * B[k * DIM + c];
            C[r * DIM + c] = s;
        }
}

// det A and A^{-T}.
template <int DIM>
__device__ __forceinline__ double det_inv_t(const double *A, double *IT) {
    if constexpr (DIM == 2) {
        const double J = A[0] * A[3] - A[1] * A[2];
        const double q = 1.0 / J;
        IT[0] = A[3] * q;
        IT[1] = -A[2] * q;
        IT[2] = -A[1] * q;
        IT[3] = A[0] * q;
        return J;
    } else {
        const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
        const double c10 = A[2] * A[7] - A[1] * A[8], c11 = A[0] * A[8] - A[2] * A[6], c12 = A[1] * A[6] - A[0] * A[7];
        const double c20 = A[1] * A[5] - A[2] * A[4], c21 = A[2] * A[3] - A[0] * A[5], c22 = A[0] * A[4] - A[1] * A[3];
        const double J = A[0] * c00 + A[1] * c01 + A[2] * c02;
        const double q = 1.0 / J;
        // cofactor matrix / J = A^{-T}
        IT[0] = c00 * q; IT[1] = c01 * q; IT[2] = c02 * q;
        IT[3] = c10 * q; IT[4] = c11 * q; IT[5] = c12 * q;
        IT[6] = c20 * q; IT[7] = c21 * q; IT[8] = c22 * q;
        return J;
    }
}

// G = sum_i u_i grad w_ip^T (physical gradient = cell-unit gradient / dx).
template <int DIM, int DEG>
__device__ __forceinline__ void gather_grad(const Axis<double, DEG> (&ax)[DIM], const MidGrid &g, const double *gv,
                                            const double *dv, double cv, double cd, double *G) {
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) G[k] = 0.0;
    for_support<DIM, DEG>(ax, g, [&](int64_t i, double, const double *gw, const double *) {
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            const double u = cv * gv[r * g.nodes + i] + cd * dv[r * g.nodes + i];
#pragma unroll
            for (int c = 0; c < DIM; ++c) G[r * DIM + c] += u * gw[c];
        }
    });
    const double s = 1.0 / g.dx;
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) G[k] *= s;
}

template <int DIM>
__device__ __forceinline__ void load_mat(const double *plane, int64_t s, int64_t p, double *M) {
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) M[k] = plane[k * s + p];
}

// Scatters -V (M F^T) grad w_ip into out (component-major node vectors).
template <int DIM, int DEG>
__device__ __forceinline__ void scatter_stress(const Axis<double, DEG> (&ax)[DIM], const MidGrid &g, const double *M,
                                               const double *F, double V, double *out) {
    double MFt[DIM * DIM];
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) s += M[r * DIM + k] * F[c * DIM + k];
            MFt[r * DIM + c] = -V * s / g.dx;
        }
    for_support<DIM, DEG>(ax, g, [&](int64_t i, double, const double *gw, const double *) {
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s += MFt[r * DIM + c] * gw[c];
            atomicAdd(&out[r * g.nodes + i], s);
        }
    });
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMidBlock) void k_mid_fill(double *a, int64_t n, double val) {
    const int64_t i = gtid();
    if (i < n) a[i] = val;
}

// Transfer to grid of mass and affine momentum (Sec. 3.2).
template <int DIM, int DEG>
__global__ __launch_bounds__(kMidBlock) void k_mid_p2g(Parts<double> P, MidGrid g, double *gm, double *gmv,
                                                       uint32_t *flags) {
    const int64_t t = gtid();
    if (t >= P.n) return;
    const int64_t p = spread(t, g, P.n);
    Axis<double, DEG> ax[DIM];
    if (!particle_axes<DIM, DEG>(P, p, g, ax)) {
        atomicOr(flags, (uint32_t)APIC_FLAG_OUT_OF_DOMAIN);
        return;
    }
    const double m = P.m[p];
    double v[DIM], B[DIM * DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) v[a] = P.v[a * P.s + p];
    load_mat<DIM>(P.B, P.s, p, B);
    // B D^{-1} (x_i - x_p) with D = dx^2 / k I and x_i - x_p = r dx
    const double q = inv_D_factor<double, DEG>() / g.dx;
    for_support<DIM, DEG>(ax, g, [&](int64_t i, double w, const double *, const double *r) {
        const double wm = w * m;
        atomicAdd(&gm[i], wm);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double br = 0.0;
#pragma unroll
            for (int b = 0; b < DIM; ++b) br += B[a * DIM + b] * r[b];
            atomicAdd(&gmv[a * g.nodes + i], wm * (v[a] + q * br));
        }
    });
}

// v_i = (m v)_i / m_i on free nodes (mass, outside the sticky band); 0
// elsewhere.  mf_i = m_i on free nodes, 0 elsewhere.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_nodes(MidGrid g, const double *gm, double *gv, double *mf) {
    const int64_t i = gtid();
    if (i >= g.nodes) return;
    int c[3];
    node_coords<DIM>(i, g, c);
    bool sticky = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) sticky = sticky || c[a] < g.band[2 * a] || c[a] > g.N[a] - 1 - g.band[2 * a + 1];
    const double m = gm[i];
    const bool free_node = m > 0.0 && !sticky;
    mf[i] = free_node ? m : 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) gv[a * g.nodes + i] = free_node ? gv[a * g.nodes + i] / m : 0.0;
}

// Forces at the displaced nodes x_i + u_i, u_i = dt/2 v_i + dt/4 dv_i
// (Sec. 4.1), and Phi = sum_p V_p Psi(F_hat_p) (Sec. 3.3).
template <int DIM, int DEG>
__global__ __launch_bounds__(kMidBlock) void k_mid_force(Parts<double> P, MidGrid g, MidMaterial mat,
                                                         const double *gv, const double *dv, double dt, double *f,
                                                         double *part, uint32_t *flags) {
    const int64_t t = gtid();
    const int64_t p = t < P.n ? spread(t, g, P.n) : 0;
    double acc[1] = {0.0};
    Axis<double, DEG> ax[DIM];
    if (t < P.n && particle_axes<DIM, DEG>(P, p, g, ax)) {
        double F[DIM * DIM], G[DIM * DIM], Fh[DIM * DIM], IT[DIM * DIM];
        load_mat<DIM>(P.F, P.s, p, F);
        gather_grad<DIM, DEG>(ax, g, gv, dv, 0.5 * dt, 0.25 * dt, G);
#pragma unroll
        for (int a = 0; a < DIM; ++a) G[a * DIM + a] += 1.0;
        mat_mul<DIM>(G, F, Fh);
        const double J = det_inv_t<DIM>(Fh, IT);
        const double V = P.m[p] / mat.rho0;
        if (!(J > 0.0)) {
            atomicOr(flags, (uint32_t)APIC_FLAG_INVERTED);
            acc[0] = INFINITY;
        } else {
            const double lnJ = log(J);
            double tr = 0.0, Pk[DIM * DIM];
#pragma unroll
            for (int k = 0; k < DIM * DIM; ++k) {
                tr += Fh[k] * Fh[k];
                Pk[k] = mat.mu * (Fh[k] - IT[k]) + mat.lambda * lnJ * IT[k];
            }
            acc[0] = V * (0.5 * mat.mu * (tr - DIM) - mat.mu * lnJ + 0.5 * mat.lambda * lnJ * lnJ);
            scatter_stress<DIM, DEG>(ax, g, Pk, F, V, f);
        }
    }
    block_partials<1>(acc, part);
}

// Force differential at the displaced state for the node vector du
// (Sec. 3.3): dF_p = (sum_j du_j grad w_jp^T) F_p,
// A_p = mu dF + (mu - lam ln J) F_hat^{-T} dF^T F_hat^{-T} + lam tr(F_hat^{-1} dF) F_hat^{-T},
// df_i = -sum_p V_p A_p F_p^T grad w_ip.
template <int DIM, int DEG>
__global__ __launch_bounds__(kMidBlock) void k_mid_dforce(Parts<double> P, MidGrid g, MidMaterial mat,
                                                          const double *gv, const double *dv, double dt,
                                                          const double *du, double *df) {
    const int64_t t = gtid();
    if (t >= P.n) return;
    const int64_t p = spread(t, g, P.n);
    Axis<double, DEG> ax[DIM];
    if (!particle_axes<DIM, DEG>(P, p, g, ax)) return;
    double F[DIM * DIM], G[DIM * DIM], H[DIM * DIM], Fh[DIM * DIM], dF[DIM * DIM], IT[DIM * DIM];
    load_mat<DIM>(P.F, P.s, p, F);
    gather_grad<DIM, DEG>(ax, g, gv, dv, 0.5 * dt, 0.25 * dt, G);
    gather_grad<DIM, DEG>(ax, g, du, du, 1.0, 0.0, H);
#pragma unroll
    for (int a = 0; a < DIM; ++a) G[a * DIM + a] += 1.0;
    mat_mul<DIM>(G, F, Fh);
    mat_mul<DIM>(H, F, dF);
    const double J = det_inv_t<DIM>(Fh, IT);
    if (!(J > 0.0)) return;
    const double lnJ = log(J);
    // tr(F_hat^{-1} dF) = sum_{a,b} IT[b][a] ... with F_hat^{-1} = IT^T: sum_ab IT[a][b] dF[a][b]
    double tr = 0.0;
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) tr += IT[k] * dF[k];
    // T = IT dF^T IT
    double T1[DIM * DIM], T2[DIM * DIM], dFt[DIM * DIM];
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c) dFt[r * DIM + c] = dF[c * DIM + r];
    mat_mul<DIM>(IT, dFt, T1);
    mat_mul<DIM>(T1, IT, T2);
    double A[DIM * DIM];
    const double cT = mat.mu - mat.lambda * lnJ;
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) A[k] = mat.mu * dF[k] + cT * T2[k] + mat.lambda * tr * IT[k];
    scatter_stress<DIM, DEG>(ax, g, A, F, P.m[p] / mat.rho0, df);
}

// r_i = dv_i - dt (f_i / m_i + g) on free nodes (the gradient of E over
// m_i / 4); partials: sum m |r|^2 and sum m (|dv|^2 / 8 - dt/4 g.dv).
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_residual(MidGrid g, const double *mf, const double *f,
                                                            const double *dv, double dt, double3 grav, double *r,
                                                            double *part) {
    const int64_t i = gtid();
    double acc[2] = {0.0, 0.0};
    if (i < g.nodes) {
        const double m = mf[i];
        const double gr[3] = {grav.x, grav.y, grav.z};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + i;
            double ra = 0.0;
            if (m > 0.0) {
                ra = dv[k] - dt * (f[k] / m + gr[a]);
                acc[0] += m * ra * ra;
                acc[1] += m * (0.125 * dv[k] * dv[k] - 0.25 * dt * gr[a] * dv[k]);
            }
            r[k] = ra;
        }
    }
    block_partials<2>(acc, part);
}

// CG start: rc = b = -r, p = rc, delta = 0; partial <rc, rc>_M.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_cg_init(MidGrid g, const double *mf, const double *r,
                                                           double *delta, double *rc, double *pv, double *part) {
    const int64_t i = gtid();
    double acc[1] = {0.0};
    if (i < g.nodes) {
        const double m = mf[i];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + i;
            const double b = -r[k];
            rc[k] = b;
            pv[k] = b;
            delta[k] = 0.0;
            acc[0] += m * b * b;
        }
    }
    block_partials<1>(acc, part);
}

// s = A p = p - dt^2/4 M^{-1} (df/dx) p on free nodes; partial <p, s>_M.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_apply(MidGrid g, const double *mf, const double *pv,
                                                         const double *df, double dt, double *s, double *part) {
    const int64_t i = gtid();
    double acc[1] = {0.0};
    if (i < g.nodes) {
        const double m = mf[i];
        const double c = 0.25 * dt * dt;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + i;
            double sa = 0.0;
            if (m > 0.0) {
                sa = pv[k] - c * df[k] / m;
                acc[0] += m * pv[k] * sa;
            }
            s[k] = sa;
        }
    }
    block_partials<1>(acc, part);
}

// delta += alpha p, rc -= alpha s; partial <rc, rc>_M.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_cg_step(MidGrid g, const double *mf, double alpha,
                                                           const double *pv, const double *s, double *delta,
                                                           double *rc, double *part) {
    const int64_t i = gtid();
    double acc[1] = {0.0};
    if (i < g.nodes) {
        const double m = mf[i];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int64_t k = a * g.nodes + i;
            delta[k] += alpha * pv[k];
            const double ra = rc[k] - alpha * s[k];
            rc[k] = ra;
            acc[0] += m * ra * ra;
        }
    }
    block_partials<1>(acc, part);
}

// out = a + alpha b over n values.
__global__ __launch_bounds__(kMidBlock) void k_mid_axpy(int64_t n, const double *a, double alpha, const double *b,
                                                        double *out) {
    const int64_t i = gtid();
    if (i < n) out[i] = (a ? a[i] : 0.0) + alpha * b[i];
}

// vt_i = v_i + dv_i on free nodes (0 elsewhere); u_i = xt_i - x_i =
// dt (v_i + vt_i) / 2.
template <int DIM>
__global__ __launch_bounds__(kMidBlock) void k_mid_finish(MidGrid g, const double *mf, const double *gv,
                                                          const double *dv, double dt, double *gvt, double *gu) {
    const int64_t i = gtid();
    if (i >= g.nodes) return;
    const bool free_node = mf[i] > 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int64_t k = a * g.nodes + i;
        const double vt = free_node ? gv[k] + dv[k] : 0.0;
        gvt[k] = vt;
        gu[k] = 0.5 * dt * (gv[k] + vt);
    }
}

// Transfer to particles with the general forms of Sec. 3.4, written with
// node displacements u_i = xt_i - x_i and U_p = x_p' - x_p = sum_i w u_i:
//   v_p' = sum_i w vt_i
//   B_p' = sum_i w vt_i r_i^T + 1/2 sum_i w (vt_i e_i^T - e_i vt_i^T),
//          r_i = x_i - x_p, e_i = u_i - U_p
//   F_p' = (I + sum_i u_i grad w^T) F_p,  x_p' = x_p + U_p.
template <int DIM, int DEG>
__global__ __launch_bounds__(kMidBlock) void k_mid_g2p(Parts<double> P, MidGrid g, const double *gvt,
                                                       const double *gu) {
    const int64_t p = gtid();
    if (p >= P.n) return;
    Axis<double, DEG> ax[DIM];
    if (!particle_axes<DIM, DEG>(P, p, g, ax)) return;
    double v[DIM] = {}, U[DIM] = {};
    for_support<DIM, DEG>(ax, g, [&](int64_t i, double w, const double *, const double *) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            v[a] += w * gvt[a * g.nodes + i];
            U[a] += w * gu[a * g.nodes + i];
        }
    });
    double B[DIM * DIM] = {}, G[DIM * DIM] = {};
    for_support<DIM, DEG>(ax, g, [&](int64_t i, double w, const double *gw, const double *r) {
        double vt[DIM], e[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            vt[a] = gvt[a * g.nodes + i];
            e[a] = gu[a * g.nodes + i] - U[a];
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = 0; b < DIM; ++b) {
                B[a * DIM + b] += w * (vt[a] * r[b] * g.dx + 0.5 * (vt[a] * e[b] - e[a] * vt[b]));
                G[a * DIM + b] += gu[a * g.nodes + i] * gw[b];
            }
    });
    double F[DIM * DIM], Fn[DIM * DIM];
    load_mat<DIM>(P.F, P.s, p, F);
    const double s = 1.0 / g.dx;
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) G[k] *= s;
#pragma unroll
    for (int a = 0; a < DIM; ++a) G[a * DIM + a] += 1.0;
    mat_mul<DIM>(G, F, Fn);
    int ci[3];
    unpack_cell<DIM>(P.cell[p], ci);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double o = P.off[a * P.s + p] + U[a] * s;
        const double c = floor(o);
        ci[a] += (int)c;
        P.off[a * P.s + p] = o - c;
        P.v[a * P.s + p] = v[a];
    }
    P.cell[p] = pack_cell<DIM>(ci);
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        P.B[k * P.s + p] = B[k];
        P.F[k * P.s + p] = Fn[k];
    }
}

// out[k] = sum over nblk blocks of part[b * K + k], in block order per thread
// stride, then a fixed tree (deterministic for a given nblk).
__global__ __launch_bounds__(kMidBlock) void k_mid_reduce(const double *part, int64_t nblk, int K, double *out) {
    __shared__ double red[kMidBlock];
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int64_t b = threadIdx.x; b < nblk; b += kMidBlock) s += part[b * K + k];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = kMidBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kMidBlock - 1) / kMidBlock); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_mid_fill(double *a, int64_t n, double val, hipStream_t st) {
    if (n > 0) k_mid_fill<<<blocks_for(n), kMidBlock, 0, st>>>(a, n, val);
}

void launch_mid_reduce(const double *part, int64_t nblk, int K, double *out, hipStream_t st) {
    k_mid_reduce<<<1, kMidBlock, 0, st>>>(part, nblk, K, out);
}

void launch_mid_axpy(int64_t n, const double *a, double alpha, const double *b, double *out, hipStream_t st) {
    if (n > 0) k_mid_axpy<<<blocks_for(n), kMidBlock, 0, st>>>(n, a, alpha, b, out);
}

int64_t mid_particle_blocks(int64_t n) { return blocks_for(n); }
int64_t mid_node_blocks(int64_t nodes) { return blocks_for(nodes); }

template <int DIM, int DEG>
void launch_mid_p2g(const Parts<double> &P, const MidGrid &g, double *gm, double *gmv, uint32_t *flags,
                    hipStream_t st) {
    if (P.n > 0) k_mid_p2g<DIM, DEG><<<blocks_for(P.n), kMidBlock, 0, st>>>(P, g, gm, gmv, flags);
}

template <int DIM>
void launch_mid_nodes(const MidGrid &g, const double *gm, double *gv, double *mf, hipStream_t st) {
    k_mid_nodes<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, gm, gv, mf);
}

template <int DIM, int DEG>
void launch_mid_force(const Parts<double> &P, const MidGrid &g, const MidMaterial &mat, const double *gv,
                      const double *dv, double dt, double *f, double *part, uint32_t *flags, hipStream_t st) {
    k_mid_force<DIM, DEG><<<blocks_for(P.n), kMidBlock, 0, st>>>(P, g, mat, gv, dv, dt, f, part, flags);
}

template <int DIM, int DEG>
void launch_mid_dforce(const Parts<double> &P, const MidGrid &g, const MidMaterial &mat, const double *gv,
                       const double *dv, double dt, const double *du, double *df, hipStream_t st) {
    if (P.n > 0) k_mid_dforce<DIM, DEG><<<blocks_for(P.n), kMidBlock, 0, st>>>(P, g, mat, gv, dv, dt, du, df);
}

template <int DIM>
void launch_mid_residual(const MidGrid &g, const double *mf, const double *f, const double *dv, double dt,
                         const double *grav, double *r, double *part, hipStream_t st) {
    const double3 gr = make_double3(grav[0], grav[1], grav[2]);
    k_mid_residual<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, mf, f, dv, dt, gr, r, part);
}

template <int DIM>
void launch_mid_cg_init(const MidGrid &g, const double *mf, const double *r, double *delta, double *rc, double *pv,
                        double *part, hipStream_t st) {
    k_mid_cg_init<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, mf, r, delta, rc, pv, part);
}

template <int DIM>
void launch_mid_apply(const MidGrid &g, const double *mf, const double *pv, const double *df, double dt, double *s,
                      double *part, hipStream_t st) {
    k_mid_apply<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, mf, pv, df, dt, s, part);
}

template <int DIM>
void launch_mid_cg_step(const MidGrid &g, const double *mf, double alpha, const double *pv, const double *s,
                        double *delta, double *rc, double *part, hipStream_t st) {
    k_mid_cg_step<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, mf, alpha, pv, s, delta, rc, part);
}

template <int DIM>
void launch_mid_finish(const MidGrid &g, const double *mf, const double *gv, const double *dv, double dt, double *gvt,
                       double *gu, hipStream_t st) {
    k_mid_finish<DIM><<<blocks_for(g.nodes), kMidBlock, 0, st>>>(g, mf, gv, dv, dt, gvt, gu);
}

template <int DIM, int DEG>
void launch_mid_g2p(const Parts<double> &P, const MidGrid &g, const double *gvt, const double *gu, hipStream_t st) {
    if (P.n > 0) k_mid_g2p<DIM, DEG><<<blocks_for(P.n), kMidBlock, 0, st>>>(P, g, gvt, gu);
}

#define APIC_MID_INST_DD(DIM, DEG)                                                                                   \
    template void launch_mid_p2g<DIM, DEG>(const Parts<double> &, const MidGrid &, double *, double *, uint32_t *,   \
                                           hipStream_t);                                                             \
    template void launch_mid_force<DIM, DEG>(const Parts<double> &, const MidGrid &, const MidMaterial &,            \
                                             const double *, const double *, double, double *, double *, uint32_t *, \
                                             hipStream_t);                                                           \
    template void launch_mid_dforce<DIM, DEG>(const Parts<double> &, const MidGrid &, const MidMaterial &,           \
                                              const double *, const double *, double, const double *, double *,      \
                                              hipStream_t);                                                          \
    template void launch_mid_g2p<DIM, DEG>(const Parts<double> &, const MidGrid &, const double *, const double *,   \
                                           hipStream_t);
#define APIC_MID_INST_D(DIM)                                                                                          \
    template void launch_mid_nodes<DIM>(const MidGrid &, const double *, double *, double *, hipStream_t);           \
    template void launch_mid_residual<DIM>(const MidGrid &, const double *, const double *, const double *, double,  \
                                           const double *, double *, double *, hipStream_t);                         \
    template void launch_mid_cg_init<DIM>(const MidGrid &, const double *, const double *, double *, double *,       \
                                          double *, double *, hipStream_t);                                          \
    template void launch_mid_apply<DIM>(const MidGrid &, const double *, const double *, const double *, double,     \
                                        double *, double *, hipStream_t);                                            \
    template void launch_mid_cg_step<DIM>(const MidGrid &, const double *, double, const double *, const double *,   \
                                          double *, double *, double *, hipStream_t);                                \
    template void launch_mid_finish<DIM>(const MidGrid &, const double *, const double *, const double *, double,    \
                                         double *, double *, hipStream_t);

APIC_MID_INST_DD(2, 2)
APIC_MID_INST_DD(2, 3)
APIC_MID_INST_DD(3, 2)
APIC_MID_INST_DD(3, 3)
APIC_MID_INST_D(2)
APIC_MID_INST_D(3)

}  // namespace apic
