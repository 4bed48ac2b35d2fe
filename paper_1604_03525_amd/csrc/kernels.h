// Launchers of the libepw device kernels (one place for all signatures).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace epw {

// ---- k_eigh.hip ----
// Interpolate n x n matrices at np points from nR real-space matrices and
// diagonalise them in float64.  real_in: X(R) real (dynamical matrix);
// sqrt_out: eigenvalues l -> sign(l) sqrt|l|.  evecs: [np][n][n] c128.
void launch_interp_eigh(bool real_in, bool sqrt_out, int n, int nR, const int32_t* R,
                        const int32_t* ndeg, const double* XR, int np, const double* pts,
                        double* evals, void* evecs, hipStream_t stream);

// ---- k_vertex.hip ----
enum class Prec { F64 = 0, F32 = 1, BF16X2 = 2 };

// exp(2 pi i p.R)/ndeg(R) -> [np][ld] complex in `prec` (columns >= nR zero).
// F64/F32 write interleaved complex; BF16X2 writes four bf16 planes
// (re_hi, re_lo, im_hi, im_lo), each [np][ld].
void launch_phase_table(Prec prec, int np, const double* pts, int nR, const int32_t* R,
                        const int32_t* ndeg, int ld, void* out, hipStream_t stream);

// complex128 -> complex64 copy (n elements)
void launch_c128_to_c64(size_t n, const void* in, void* out, hipStream_t stream);

// Per-chunk phonon factors: sc[q][nu] = 1/sqrt(2 omega) (0 when omega < cut),
// nbose[q][nu] = Bose factor (0 when cut).
void launch_phonon_factors(int nq, int nm, const double* omega, double omega_cut, double T,
                           double* sc, double* nbose, hipStream_t stream);

// f[i] = Fermi-Dirac(eps[i]) for n values.
void launch_fermi_table(size_t n, const double* eps, double mu, double T, double* f,
                        hipStream_t stream);

// a5: g(R_e, q) = sum_p Phi_q[q][p] g(R_e, R_p): out[e][q][col], col < ncol.
void launch_gemm_rp(Prec prec, int nq, int ne, int np_, int ncol, const void* phi_q, int ldphi,
                    const void* gR, void* out, hipStream_t stream);

// a6: out[e][q][nu][i][j] (NBP-padded) = sum_a in[e][q][a][i][j] e_q[a][nu] sc[q][nu]
void launch_mode_rotate(Prec prec, int ne, int nq, int nm, int nb, int nbp, const void* in,
                        const void* evec, const double* sc, void* out, hipStream_t stream);

struct FusedArgs {
    int nk, ne, nb, nbp, nm;
    int qc;            // q points in this chunk
    int q0;            // global index of the first q of the chunk
    int nq_total;      // row length of kq
    const void* phi_k; // [nk][ldk] complex in prec
    int ldk;
    const void* B;     // [ne][qc*nm*nbp*nbp] complex in prec
    const double* eps; // [nk][nb]
    const void* U;     // [nk][nb][nb] c128
    const double* ftab;// [nk][nb]
    const int32_t* kq; // [nk][nq_total]
    const double* omega;   // [qc][nm] (chunk-local)
    const double* nbose;   // [qc][nm] (chunk-local)
    const double* sc;      // [qc][nm] (chunk-local)
    double sigma;
    double* part;      // [S][nk][nb] partial sums (imsigma mode)
    int S;             // number of slices
    void* gkq;         // [nk][nq_total][nm][nb][nb] c128 (store mode)
};
// a7 + a8 + a9 (imsigma mode) or a7 + a8 (store mode, gkq != nullptr)
void launch_fused_k(Prec prec, const FusedArgs& a, int num_cu, hipStream_t stream);
int fused_slices(int nk, int nbp, int ncols_tiles, int num_cu);

// imsig[k][n] = (acc ? imsig : 0) + scale * sum_s part[s][k][n]
void launch_reduce_partials(int nk, int nb, int S, const double* part, double scale,
                            int accumulate, double* imsig, hipStream_t stream);
// average over bands whose consecutive energies differ by < tol
void launch_degenerate_average(int nk, int nb, const double* eps, double tol, double* v,
                               hipStream_t stream);

}  // namespace epw
