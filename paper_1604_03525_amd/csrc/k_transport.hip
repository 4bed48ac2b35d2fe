// Transport coupling helpers (Sec. 6, velocities as in Sec. 7):
//
//   v_nk,a = Re [U_k^dag (dH/dk_a) U_k]_nn,
//       dH/dk_a = Hermitised sum_R i R_a exp(2 pi i k.R) H(R)/ndeg(R)  (R Cartesian)
//   averaged over bands whose sorted energies differ by < deg_tol;
//
//   alpha^2 F(w_j) = (1/2) (1/N_q) sum_q,nu omega_q,nu lambda_q,nu delta_s(w_j - omega_q,nu)   (Eqs. (12), (54))
//
//   rho n e^2 / m_e = (4 pi / (k_B T)) int dw w a2F(w) n(w) [1 + n(w)]     (Eq. (53)),
//   trapezoid rule on the grid with the integrand 0 for w <= 0.
#include <hip/hip_runtime.h>

#include "epw_internal.h"
#include "kernels.h"

namespace epw {
namespace {

struct Vectors {
    double a[3][3];
};

constexpr int VEL_THREADS = 256;
constexpr int VEL_CHUNK = 1024;          // R vectors whose phases are staged in LDS at a time
constexpr int VEL_PER_THREAD = (3 * EPW_MAX_NB * EPW_MAX_NB + VEL_THREADS - 1) / VEL_THREADS;

// One block per point.  Per chunk of R vectors: phases in LDS, then the
// entries (a, i, j) of dH/dk_a accumulated over the threads; then the
// Hermitised matrices are rotated into the band basis and the diagonals
// averaged over degenerate bands.
__global__ __launch_bounds__(VEL_THREADS) void velocity_kernel(int nb, int nR, const int32_t* __restrict__ R,
                                                               const int32_t* __restrict__ ndeg,
                                                               const double2* __restrict__ HR, Vectors V,
                                                               const double* __restrict__ kfrac,
                                                               const double* __restrict__ eps,
                                                               const double2* __restrict__ U, double deg_tol,
                                                               double* __restrict__ vel)
{
    __shared__ double2 ph[VEL_CHUNK];
    __shared__ double Rc[VEL_CHUNK][3];
    __shared__ double2 dH[3][EPW_MAX_NB][EPW_MAX_NB];
    __shared__ double d[3][EPW_MAX_NB];
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    const double k0 = kfrac[3 * (size_t)p], k1 = kfrac[3 * (size_t)p + 1], k2 = kfrac[3 * (size_t)p + 2];
    const int nb2 = nb * nb;
    double sr[VEL_PER_THREAD], si[VEL_PER_THREAD];
#pragma unroll
    for (int u = 0; u < VEL_PER_THREAD; ++u) {
        sr[u] = 0.0;
        si[u] = 0.0;
    }
    for (int r0 = 0; r0 < nR; r0 += VEL_CHUNK) {
        const int nc = min(VEL_CHUNK, nR - r0);
        __syncthreads();                                 // previous chunk no longer read
        for (int c = tid; c < nc; c += VEL_THREADS) {
            const int r = r0 + c;
            double x = k0 * R[3 * r] + k1 * R[3 * r + 1] + k2 * R[3 * r + 2];
            x -= rint(x);
            double sn, cs;
            sincospi(2.0 * x, &sn, &cs);
            const double w = 1.0 / (double)ndeg[r];
            ph[c] = make_double2(cs * w, sn * w);
            for (int a = 0; a < 3; ++a)
                Rc[c][a] = R[3 * r] * V.a[0][a] + R[3 * r + 1] * V.a[1][a] + R[3 * r + 2] * V.a[2][a];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < VEL_PER_THREAD; ++u) {
            const int e = tid + u * VEL_THREADS;
            if (e >= 3 * nb2) break;
            const int a = e / nb2, ij = e % nb2;
            for (int c = 0; c < nc; ++c) {
                const double2 h = HR[(size_t)(r0 + c) * nb2 + ij];
                const double2 f = ph[c];
                // i R_a f h
                const double pr = f.x * h.x - f.y * h.y, pi = f.x * h.y + f.y * h.x;
                sr[u] -= Rc[c][a] * pi;
                si[u] += Rc[c][a] * pr;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < VEL_PER_THREAD; ++u) {
        const int e = tid + u * VEL_THREADS;
        if (e >= 3 * nb2) break;
        const int a = e / nb2, ij = e % nb2;
        dH[a][ij / nb][ij % nb] = make_double2(sr[u], si[u]);
    }
    __syncthreads();
    // diagonal of U^dag ((dH + dH^dag)/2) U, per (a, n)
    if (tid < 3 * nb) {
        const int a = tid / nb, n = tid % nb;
        const double2* u = U + (size_t)p * nb2;
        double acc = 0.0;
        for (int i = 0; i < nb; ++i) {
            const double2 ui = u[i * nb + n];
            for (int j = 0; j < nb; ++j) {
                const double2 uj = u[j * nb + n];
                const double2 x = dH[a][i][j], y = dH[a][j][i];
                const double hr = 0.5 * (x.x + y.x), hi = 0.5 * (x.y - y.y);
                // Re(conj(ui) h uj)
                const double tr = hr * uj.x - hi * uj.y, ti = hr * uj.y + hi * uj.x;
                acc += ui.x * tr + ui.y * ti;
            }
        }
        d[a][n] = acc;
    }
    __syncthreads();
    if (tid < 3) {
        const int a = tid;
        const double* e = eps + (size_t)p * nb;
        int start = 0;
        while (start < nb) {
            int stop = start + 1;
            while (stop < nb && fabs(e[stop] - e[stop - 1]) < deg_tol) ++stop;
            double t = 0.0;
            for (int n = start; n < stop; ++n) t += d[a][n];
            t /= (double)(stop - start);
            for (int n = start; n < stop; ++n) vel[((size_t)p * nb + n) * 3 + a] = t;
            start = stop;
        }
    }
}

// dHR3[a][r][ij] = i R_a(r) H(R)[ij], R Cartesian
__global__ void velocity_operands_kernel(int nb2, int nR, const int32_t* __restrict__ R,
                                         const double2* __restrict__ HR, Vectors V, double2* __restrict__ out)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t per = (size_t)nR * nb2;
    if (idx >= 3 * per) return;
    const int a = (int)(idx / per);
    const size_t rij = idx % per;
    const int r = (int)(rij / nb2);
    const double Ra = R[3 * r] * V.a[0][a] + R[3 * r + 1] * V.a[1][a] + R[3 * r + 2] * V.a[2][a];
    const double2 h = HR[rij];
    out[idx] = make_double2(-Ra * h.y, Ra * h.x);
}

// One wave per pair: v_m,a = Re [U^dag ((dH_a + dH_a^dag)/2) U]_mm, then the
// average over degenerate bands.
__global__ __launch_bounds__(64) void pair_velocity_kernel(int nb, long ld, const double2* __restrict__ dH3,
                                                           const double2* __restrict__ U,
                                                           const double* __restrict__ eps, double deg_tol,
                                                           double* __restrict__ vel)
{
    __shared__ double d[3][EPW_MAX_NB];
    const long p = blockIdx.x;
    const int tid = threadIdx.x;
    const int nb2 = nb * nb;
    if (tid < 3 * nb) {
        const int a = tid / nb, m = tid % nb;
        const double2* h = dH3 + ((size_t)a * ld + p) * nb2;
        const double2* u = U + (size_t)p * nb2;
        double acc = 0.0;
        for (int i = 0; i < nb; ++i) {
            const double2 ui = u[i * nb + m];
            for (int j = 0; j < nb; ++j) {
                const double2 uj = u[j * nb + m];
                const double2 x = h[i * nb + j], y = h[j * nb + i];
                const double hr = 0.5 * (x.x + y.x), hi = 0.5 * (x.y - y.y);
                const double tr = hr * uj.x - hi * uj.y, ti = hr * uj.y + hi * uj.x;
                acc += ui.x * tr + ui.y * ti;
            }
        }
        d[a][m] = acc;
    }
    __syncthreads();
    if (tid < 3) {
        const int a = tid;
        const double* e = eps + (size_t)p * nb;
        int start = 0;
        while (start < nb) {
            int stop = start + 1;
            while (stop < nb && fabs(e[stop] - e[stop - 1]) < deg_tol) ++stop;
            double t = 0.0;
            for (int n = start; n < stop; ++n) t += d[a][n];
            t /= (double)(stop - start);
            for (int n = start; n < stop; ++n) vel[((size_t)p * nb + n) * 3 + a] = t;
            start = stop;
        }
    }
}

__global__ void eliashberg_kernel(int ncb, const double* __restrict__ omega, const double* __restrict__ lam,
                                  double inv_nq, int nw, const double* __restrict__ wgrid, double sigma,
                                  double* __restrict__ a2f)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nw) return;
    const double w = wgrid[j];
    const double inv_s = 1.0 / sigma;
    constexpr double kPi = 3.141592653589793;
    double acc = 0.0;
    for (int t = 0; t < ncb; ++t) {
        const double y = (w - omega[t]) * inv_s;
        acc += omega[t] * lam[t] * exp(-y * y);
    }
    a2f[j] = 0.5 * inv_nq * acc * inv_s / sqrt(kPi);
}

__global__ void ziman_kernel(int nw, const double* __restrict__ wgrid, const double* __restrict__ a2f, int nT,
                             const double* __restrict__ T, double* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nT) return;
    constexpr double kPi = 3.141592653589793;
    const double kT = 8.617333262e-5 * T[i];
    if (!(kT > 0.0)) {
        out[i] = 0.0;
        return;
    }
    double acc = 0.0, prev = 0.0;
    for (int j = 0; j < nw; ++j) {
        const double w = wgrid[j];
        double f = 0.0;
        if (w > 0.0) {
            const double n = 1.0 / expm1(w / kT);
            f = w * a2f[j] * n * (1.0 + n);
        }
        if (j > 0) acc += 0.5 * (prev + f) * (w - wgrid[j - 1]);
        prev = f;
    }
    out[i] = 4.0 * kPi / kT * acc;
}

}  // namespace

void launch_velocities(int nb, int nR, const int32_t* R, const int32_t* ndeg, const void* HR, const double* vectors9,
                       int np, const double* kfrac, const double* eps, const void* U, double deg_tol, double* vel,
                       hipStream_t stream) {
    if (np == 0) return;
    Vectors V;
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) V.a[i][a] = vectors9[3 * i + a];
    velocity_kernel<<<np, VEL_THREADS, 0, stream>>>(nb, nR, R, ndeg, (const double2*)HR, V, kfrac, eps,
                                                    (const double2*)U, deg_tol, vel);
    launch_check("velocity_kernel");
}

void launch_velocity_operands(int nb, int nR, const int32_t* R, const void* HR, const double* vectors9, void* dHR3,
                              hipStream_t stream) {
    const size_t n = 3 * (size_t)nR * nb * nb;
    if (n == 0) return;
    Vectors V;
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) V.a[i][a] = vectors9[3 * i + a];
    velocity_operands_kernel<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(nb * nb, nR, R, (const double2*)HR, V,
                                                                             (double2*)dHR3);
    launch_check("velocity_operands_kernel");
}

void launch_pair_velocities(int nb, int np, long ld, const void* dH3, const void* U, const double* eps, double deg_tol,
                            double* vel, hipStream_t stream) {
    if (np == 0) return;
    pair_velocity_kernel<<<(unsigned)np, 64, 0, stream>>>(nb, ld, (const double2*)dH3, (const double2*)U, eps,
                                                         deg_tol, vel);
    launch_check("pair_velocity_kernel");
}

void launch_eliashberg(int nq, int nm, const double* omega, const double* lam, double nq_norm, int nw,
                       const double* wgrid, double sigma, double* a2f, hipStream_t stream) {
    if (nw == 0) return;
    eliashberg_kernel<<<(nw + 127) / 128, 128, 0, stream>>>(nq * nm, omega, lam, 1.0 / nq_norm, nw, wgrid, sigma,
                                                           a2f);
    launch_check("eliashberg_kernel");
}

void launch_ziman(int nw, const double* wgrid, const double* a2f, int nT, const double* T, double* out,
                  hipStream_t stream) {
    if (nT == 0) return;
    ziman_kernel<<<(nT + 63) / 64, 64, 0, stream>>>(nw, wgrid, a2f, nT, T, out);
    launch_check("ziman_kernel");
}

}  // namespace epw
