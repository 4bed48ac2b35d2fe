// Long-range (polar) factor of the electron-phonon vertex, Sec. 4:
//
//   L_nu(q) = i C sc_nu(q) sum_kappa M_kappa^(-1/2) sum_{K = q + G != 0}
//             exp(-K.eps.K/(4 alpha)) / (K.eps.K) (K . Z*_kappa . e_kappa,nu(q)) exp(-i K . tau_kappa)
//
// with sc = 1/sqrt(2 omega) (0 for cut modes).  One block per q: the G box
// is strided over the threads, each thread keeps its partial sums for every
// mode, and the block sums them in fixed order (bit-reproducible).  The mode
// rotation then adds L_nu(q) delta_ij at R_e = 0, which becomes
// L_nu(q) [U_k+q^dagger U_k]_mn after the band rotation.
#include <hip/hip_runtime.h>

#include "epw_internal.h"
#include "kernels.h"

namespace epw {
namespace {

constexpr int POLAR_THREADS = 128;

__global__ __launch_bounds__(POLAR_THREADS) void polar_factor_kernel(PolarDev P, int nm,
                                                                     const double* __restrict__ qfrac,
                                                                     const double2* __restrict__ evec,
                                                                     const double* __restrict__ sc,
                                                                     double2* __restrict__ L)
{
    __shared__ double2 red[POLAR_THREADS][EPW_MAX_NM];
    const int q = blockIdx.x;
    const int tid = threadIdx.x;
    double qr[3];
    for (int a = 0; a < 3; ++a) {
        const double x = qfrac[3 * (size_t)q + a];
        qr[a] = x - floor(x + 0.5);                 // the sum over all G is periodic in q
    }
    double2 acc[EPW_MAX_NM];
#pragma unroll
    for (int v = 0; v < EPW_MAX_NM; ++v) acc[v] = make_double2(0.0, 0.0);
    const double2* e = evec + (size_t)q * nm * nm;
    const int w = 2 * P.gmax + 1;
    const long nG = (long)w * w * w;
    for (long t = tid; t < nG; t += POLAR_THREADS) {
        const double g0 = (double)(t / (w * w)) - P.gmax, g1 = (double)((t / w) % w) - P.gmax,
                     g2 = (double)(t % w) - P.gmax;
        double K[3];
        for (int a = 0; a < 3; ++a)
            K[a] = (qr[0] + g0) * P.B[0][a] + (qr[1] + g1) * P.B[1][a] + (qr[2] + g2) * P.B[2][a];
        double x = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) x += K[a] * P.eps[a][b] * K[b];
        const double kk = K[0] * K[0] + K[1] * K[1] + K[2] * K[2];
        if (!(kk > 1e-24) || !(x / (4.0 * P.alpha) < P.cutoff)) continue;
        const double f = exp(-x / (4.0 * P.alpha)) / x;
        for (int kap = 0; kap < P.nat; ++kap) {
            double zK[3];
            for (int b = 0; b < 3; ++b)
                zK[b] = K[0] * P.zstar[kap][0][b] + K[1] * P.zstar[kap][1][b] + K[2] * P.zstar[kap][2][b];
            double sn, cs;
            sincos(-(K[0] * P.tau[kap][0] + K[1] * P.tau[kap][1] + K[2] * P.tau[kap][2]), &sn, &cs);
            const double fr = f * P.rsm[kap] * cs, fi = f * P.rsm[kap] * sn;
#pragma unroll
            for (int v = 0; v < EPW_MAX_NM; ++v) {
                if (v >= nm) break;
                double zr = 0.0, zi = 0.0;
                for (int b = 0; b < 3; ++b) {
                    const double2 ev = e[(size_t)(3 * kap + b) * nm + v];
                    zr += zK[b] * ev.x;
                    zi += zK[b] * ev.y;
                }
                acc[v].x += fr * zr - fi * zi;
                acc[v].y += fr * zi + fi * zr;
            }
        }
    }
#pragma unroll
    for (int v = 0; v < EPW_MAX_NM; ++v) red[tid][v] = acc[v];
    __syncthreads();
    if (tid < nm) {
        double sr = 0.0, si = 0.0;
        for (int u = 0; u < POLAR_THREADS; ++u) {
            sr += red[u][tid].x;
            si += red[u][tid].y;
        }
        // times i C sc
        const double s = P.prefactor * sc[(size_t)q * nm + tid];
        L[(size_t)q * nm + tid] = make_double2(-s * si, s * sr);
    }
}

}  // namespace

void launch_polar_factor(const PolarDev& P, int qc, int nm, const double* qfrac, const void* evec,
                         const double* sc, void* L, hipStream_t stream) {
    if (qc == 0) return;
    polar_factor_kernel<<<qc, POLAR_THREADS, 0, stream>>>(P, nm, qfrac, (const double2*)evec, sc, (double2*)L);
    launch_check("polar_factor_kernel");
}

}  // namespace epw
