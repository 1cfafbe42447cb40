// Fills, state copies, binary64 particle totals and position conversion.
#include "apic_kernels.h"

namespace apic {

static inline int blocks_for(int64_t work, int threads, int cap) {
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

template <typename T>
__global__ void k_fill(T *p, int64_t count, T val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

template <typename T>
void launch_fill(T *p, int64_t count, T val, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(count, 256, 8192)), dim3(256), 0, st, p, count, val);
}
template void launch_fill<float>(float *, int64_t, float, hipStream_t);
template void launch_fill<double>(double *, int64_t, double, hipStream_t);
template void launch_fill<uint32_t>(uint32_t *, int64_t, uint32_t, hipStream_t);
template void launch_fill<int32_t>(int32_t *, int64_t, int32_t, hipStream_t);

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_copy_state(Parts<T> src, Parts<T> dst) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= src.n) return;
    dst.cell[j] = src.cell[j];
    dst.m[j] = src.m[j];
    if (src.id) dst.id[j] = src.id[j];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        dst.off[a * dst.s + j] = src.off[a * src.s + j];
        dst.v[a * dst.s + j] = src.v[a * src.s + j];
    }
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) {
        dst.B[k * dst.s + j] = src.B[k * src.s + j];
        dst.F[k * dst.s + j] = src.F[k * src.s + j];
    }
}

template <typename T, int DIM>
void launch_copy_state(const Parts<T> &src, const Parts<T> &dst, hipStream_t st) {
    if (src.n == 0) return;
    Parts<T> s2 = src, d2 = dst;
    if (!src.id || !dst.id) s2.id = d2.id = nullptr;
    hipLaunchKernelGGL((k_copy_state<T, DIM>), dim3((unsigned)((src.n + 255) / 256)), dim3(256), 0, st, s2, d2);
}

// --- binary64 particle totals (Sec. 3.1; B term of Sec. 5.3) -------------------
__device__ __forceinline__ void block_reduce8p(double *acc, double *partials) {
    __shared__ double sh[8][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        double x = acc[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if (lane == 0) sh[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[threadIdx.x][w];
        partials[blockIdx.x * 8 + threadIdx.x] = t;
    }
}

template <typename T, int DIM, bool ABS>
__global__ __launch_bounds__(256) void k_diag_particles(Parts<T> P, double dx, double affine, double *partials) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P.n; p += (int64_t)gridDim.x * blockDim.x) {
        int ci[3] = {0, 0, 0};
        if constexpr (!ABS) unpack_cell<DIM>(P.cell[p], ci);
        double x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, Bm[9];
        const double m = (double)P.m[p];
        for (int a = 0; a < DIM; ++a) {
            x[a] = ABS ? (double)P.off[a * P.s + p] : ((double)ci[a] + (double)P.off[a * P.s + p]) * dx;
            v[a] = (double)P.v[a * P.s + p];
        }
        for (int k = 0; k < DIM * DIM; ++k) Bm[k] = affine * (double)P.B[k * P.s + p];
        const double mv[3] = {m * v[0], m * v[1], m * v[2]};
        acc[0] += mv[0];
        acc[1] += mv[1];
        acc[2] += mv[2];
        if constexpr (DIM == 3) {
            // x x m v + m (B^T : eps): B_zy - B_yz, B_xz - B_zx, B_yx - B_xy
            acc[3] += x[1] * mv[2] - x[2] * mv[1] + m * (Bm[7] - Bm[5]);
            acc[4] += x[2] * mv[0] - x[0] * mv[2] + m * (Bm[2] - Bm[6]);
            acc[5] += x[0] * mv[1] - x[1] * mv[0] + m * (Bm[3] - Bm[1]);
        } else {
            acc[5] += x[0] * mv[1] - x[1] * mv[0] + m * (Bm[2] - Bm[1]);
        }
        double v2 = 0.0;
        for (int a = 0; a < DIM; ++a) v2 += v[a] * v[a];
        acc[6] += 0.5 * m * v2;
        acc[7] += m;
    }
    block_reduce8p(acc, partials);
}

// One wavefront: lane l sums the partials of blocks l, l + 64, ... in that
// order, then a fixed shuffle tree adds the lanes, so the result does not
// depend on timing.
__global__ __launch_bounds__(64) void k_diag_final(const double *partials, int nb, double *out) {
    const int lane = (int)threadIdx.x;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        double t = 0.0;
        for (int b = lane; b < nb; b += 64) t += partials[b * 8 + k];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o, 64);
        if (lane == 0) out[k] = t;
    }
}

void launch_diag_final(const double *partials, int nb, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, st, partials, nb, out);
}

template <typename T, int DIM>
void launch_diag_particles(const Parts<T> &P, double dx, bool affine, double *partials, double *out,
                           hipStream_t st, bool absolute) {
    const int nb = blocks_for(P.n, 256, kDiagBlocks);
    if (absolute)
        hipLaunchKernelGGL((k_diag_particles<T, DIM, true>), dim3(nb), dim3(256), 0, st, P, dx, affine ? 1.0 : 0.0,
                           partials);
    else
        hipLaunchKernelGGL((k_diag_particles<T, DIM, false>), dim3(nb), dim3(256), 0, st, P, dx, affine ? 1.0 : 0.0,
                           partials);
    launch_diag_final(partials, nb, out, st);
}

// --- binary64 energies (Sec. 3.1 kinetic, Sec. 3.3 potential) -------------
// acc[0] = 1/2 sum m |v|^2, acc[1] = Phi = sum V_p Psi(F_p) with the
// neo-Hookean density Psi = mu/2 (tr F^T F - d) - mu ln J + lambda/2 (ln J)^2
// (V_p = m_p / rho0; 0 without a model; +inf for det F <= 0), acc[2] their
// sum, acc[7] the mass.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_diag_energy(Parts<T> P, int model, double mu, double lam, double inv_rho0,
                                                     double *partials) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P.n; p += (int64_t)gridDim.x * blockDim.x) {
        const double m = (double)P.m[p];
        double v2 = 0.0;
        for (int a = 0; a < DIM; ++a) {
            const double x = (double)P.v[a * P.s + p];
            v2 += x * x;
        }
        const double ke = 0.5 * m * v2;
        double phi = 0.0;
        if (model == APIC_MODEL_NEO_HOOKEAN) {
            double F[DIM * DIM], tr = 0.0;
            for (int k = 0; k < DIM * DIM; ++k) {
                F[k] = (double)P.F[k * P.s + p];
                tr += F[k] * F[k];
            }
            double J;
            if constexpr (DIM == 3)
                J = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
                    F[2] * (F[3] * F[7] - F[4] * F[6]);
            else
                J = F[0] * F[3] - F[1] * F[2];
            if (J > 0.0) {
                const double lj = log(J);
                phi = m * inv_rho0 * (0.5 * mu * (tr - (double)DIM) - mu * lj + 0.5 * lam * lj * lj);
            } else {
                phi = INFINITY;
            }
        }
        acc[0] += ke;
        acc[1] += phi;
        acc[2] += ke + phi;
        acc[7] += m;
    }
    block_reduce8p(acc, partials);
}

template <typename T, int DIM>
void launch_diag_energy(const Parts<T> &P, int model, double mu, double lam, double rho0, double *partials,
                        double *out, hipStream_t st) {
    const int nb = blocks_for(P.n, 256, kDiagBlocks);
    hipLaunchKernelGGL((k_diag_energy<T, DIM>), dim3(nb), dim3(256), 0, st, P, model, mu, lam,
                       rho0 > 0.0 ? 1.0 / rho0 : 0.0, partials);
    launch_diag_final(partials, nb, out, st);
}

// --- CFL bound (Sec. 4.3) -----------------------------------------------------------
// max_p (|v_p| + c |B_p|_F), c = 6 sqrt(d) / dx, in binary64: per block into
// partials[block], then one block reduces them into out[0].
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_cfl_bound(Parts<T> P, double c, double *partials) {
    __shared__ double sh[4];
    double worst = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P.n; p += (int64_t)gridDim.x * blockDim.x) {
        double vv = 0.0, bb = 0.0;
        for (int a = 0; a < DIM; ++a) {
            const double x = (double)P.v[a * P.s + p];
            vv += x * x;
        }
        for (int k = 0; k < DIM * DIM; ++k) {
            const double x = (double)P.B[k * P.s + p];
            bb += x * x;
        }
        const double u = sqrt(vv) + c * sqrt(bb);
        worst = u > worst || u != u ? u : worst;  // a NaN state propagates
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_down(worst, o, 64);
        worst = y > worst || y != y ? y : worst;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = worst;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = sh[w] > m || sh[w] != sh[w] ? sh[w] : m;
        partials[blockIdx.x] = m;
    }
}

// One wavefront: a lane-strided max, then a shuffle tree (max is exact in any order).
__global__ __launch_bounds__(64) void k_cfl_final(const double *partials, int nb, double *out) {
    const int lane = (int)threadIdx.x;
    double m = 0.0;
    for (int b = lane; b < nb; b += 64) {
        const double y = partials[b];
        m = y > m || y != y ? y : m;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_down(m, o, 64);
        m = y > m || y != y ? y : m;
    }
    if (lane == 0) out[0] = m;
}

template <typename T, int DIM>
void launch_cfl_bound(const Parts<T> &P, double c, double *partials, double *out, hipStream_t st) {
    const int nb = blocks_for(P.n, 256, kDiagBlocks);
    hipLaunchKernelGGL((k_cfl_bound<T, DIM>), dim3(nb), dim3(256), 0, st, P, c, partials);
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(64), 0, st, partials, nb, out);
}

// --- transfer variants (Sec. 5.6) -------------------------------------------------
// The caller's B planes in the form the transfer carries (skew part for
// RPIC, zero for PIC), in place, once per call: the transfers to particles
// store that form themselves, so the transfers to grid can read B as is.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_keep_affine(Parts<T> P, int transfer) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    T B[DIM * DIM];
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) B[k] = P.B[k * P.s + p];
    keep_affine<T, DIM>(transfer, B);
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) P.B[k * P.s + p] = B[k];
}

template <typename T, int DIM>
void launch_keep_affine(const Parts<T> &P, int transfer, hipStream_t st) {
    if (P.n == 0 || transfer == APIC_TRANSFER_APIC) return;
    hipLaunchKernelGGL((k_keep_affine<T, DIM>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P, transfer);
}

// --- adaptive step (Sec. 4.3) ------------------------------------------------------
// One wavefront: b = max of src[0..n) (binary64; NaN propagates), then
//   dt = b > 0 ? min(cap, nu_dx / b) : cap      (a NaN bound gives cap: the
// flags of the transfers report a non-finite state), state[0] = dt,
// state[1] += dt, and the kVmaxSlots bound slots are zeroed for the next
// transfer to particles (src may be those slots: each lane reads its
// entries before it clears them).
__global__ __launch_bounds__(64) void k_adapt_dt(const double *src, int n, unsigned long long *slots, double cap,
                                                  double nu_dx, double *state) {
    const int lane = (int)threadIdx.x;
    double b = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double y = src[i];
        b = y > b || y != y ? y : b;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_xor(b, o, 64);
        b = y > b || y != y ? y : b;
    }
    for (int i = lane; i < kVmaxSlots; i += 64) slots[i] = 0ull;
    if (lane == 0) {
        double dt = cap;
        if (b > 0.0) {
            const double c = nu_dx / b;
            dt = c < cap ? c : cap;
        }
        state[0] = dt;
        state[1] += dt;
    }
}

void launch_adapt_dt(const double *src, int n, unsigned long long *slots, double cap, double nu_dx, double *state,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_adapt_dt, dim3(1), dim3(64), 0, st, src, n, slots, cap, nu_dx, state);
}

// Binary64 bound of every particle into partials[0..nb) (the first pass of
// launch_cfl_bound); returns nb.
template <typename T, int DIM>
int launch_cfl_partials(const Parts<T> &P, double c, double *partials, hipStream_t st) {
    const int nb = blocks_for(P.n, 256, kDiagBlocks);
    hipLaunchKernelGGL((k_cfl_bound<T, DIM>), dim3(nb), dim3(256), 0, st, P, c, partials);
    return nb;
}

// --- absolute positions <-> cell + offset ---------------------------------------
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_pack_positions(Parts<T> P, const double *x, double inv_dx, int absolute) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    int ci[3] = {0, 0, 0};
    if (absolute) {
        // the coordinate itself, rounded to the plane's type (the cell plane
        // gets the cell that rounded coordinate lies in)
        for (int a = 0; a < DIM; ++a) {
            const T xa = (T)x[a * P.s + p];
            T o;
            cell_of_absolute(xa, (T)inv_dx, ci[a], o);
            const int lim = DIM == 3 ? 1023 : 65535;
            ci[a] = ci[a] < 0 ? 0 : (ci[a] > lim ? lim : ci[a]);
            P.off[a * P.s + p] = xa;
        }
        P.cell[p] = pack_cell<DIM>(ci);
        return;
    }
    for (int a = 0; a < DIM; ++a) {
        const double sx = x[a * P.s + p] * inv_dx;
        double c = floor(sx);
        T o = (T)(sx - c);
        if (o >= T(1)) {
            o = T(0);
            c += 1.0;
        }
        const int lim = DIM == 3 ? 1023 : 65535;
        ci[a] = c < 0.0 ? 0 : (c > lim ? lim : (int)c);
        P.off[a * P.s + p] = o;
    }
    P.cell[p] = pack_cell<DIM>(ci);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_unpack_positions(Parts<T> P, double *x, double dx, int absolute) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    if (absolute) {
        for (int a = 0; a < DIM; ++a) x[a * P.s + p] = (double)P.off[a * P.s + p];
        return;
    }
    int ci[3] = {0, 0, 0};
    unpack_cell<DIM>(P.cell[p], ci);
    for (int a = 0; a < DIM; ++a) x[a * P.s + p] = ((double)ci[a] + (double)P.off[a * P.s + p]) * dx;
}

template <typename T, int DIM>
void launch_pack_positions(const Parts<T> &P, const double *x, double dx, hipStream_t st, bool absolute) {
    if (P.n == 0) return;
    hipLaunchKernelGGL((k_pack_positions<T, DIM>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P, x,
                       1.0 / dx, absolute ? 1 : 0);
}

template <typename T, int DIM>
void launch_unpack_positions(const Parts<T> &P, double *x, double dx, hipStream_t st, bool absolute) {
    if (P.n == 0) return;
    hipLaunchKernelGGL((k_unpack_positions<T, DIM>), dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, P, x, dx,
                       absolute ? 1 : 0);
}

#define APIC_MISC_INST(T, DIM)                                                                                  \
    template void launch_copy_state<T, DIM>(const Parts<T> &, const Parts<T> &, hipStream_t);                    \
    template void launch_diag_particles<T, DIM>(const Parts<T> &, double, bool, double *, double *, hipStream_t,  \
                                                bool);                                                            \
    template void launch_diag_energy<T, DIM>(const Parts<T> &, int, double, double, double, double *, double *,    \
                                             hipStream_t);                                                     \
    template void launch_cfl_bound<T, DIM>(const Parts<T> &, double, double *, double *, hipStream_t);         \
    template int launch_cfl_partials<T, DIM>(const Parts<T> &, double, double *, hipStream_t);                  \
    template void launch_keep_affine<T, DIM>(const Parts<T> &, int, hipStream_t);                                \
    template void launch_pack_positions<T, DIM>(const Parts<T> &, const double *, double, hipStream_t, bool);   \
    template void launch_unpack_positions<T, DIM>(const Parts<T> &, double *, double, hipStream_t, bool);
APIC_MISC_INST(float, 2)
APIC_MISC_INST(float, 3)
APIC_MISC_INST(double, 2)
APIC_MISC_INST(double, 3)

}  // namespace apic
