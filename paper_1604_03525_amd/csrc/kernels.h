// Launchers of the libepw device kernels (one place for all signatures).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "epw.h"

namespace epw {

// ---- k_eigh.hip ----
// Interpolate n x n matrices at np points from nR real-space matrices and
// diagonalise them in float64.  real_in: X(R) real (dynamical matrix);
// sqrt_out: eigenvalues l -> sign(l) sqrt|l|.  evecs: [np][n][n] c128.
// Pair mode (pts2 != nullptr): point p is pts[p / n2] + pts2[p % n2].
void launch_interp_eigh(bool real_in, bool sqrt_out, int n, int nR, const int32_t* R,
                        const int32_t* ndeg, const double* XR, int np, const double* pts,
                        double* evals, void* evecs, hipStream_t stream,
                        const double* pts2 = nullptr, int n2 = 1);

// Eigendecomposition (float64, Hermitised first) of np given n x n complex
// matrices X [np][n][n]; evals ascending [np][n], evecs [np][n][n] c128.
// packed: X holds only the upper triangles ([np][n(n+1)/2], row by row from the diagonal)
void launch_eigh_given(int n, int np, const void* X, double* evals, void* evecs, hipStream_t stream,
                       bool packed = false);
// P[r] = upper triangle, in the packed order above, of the Hermitian part
// (X(R) + ndeg(R)/ndeg(-R) X(-R)^dag)/2 of nR complex n x n matrices on a WS set
// closed under R -> -R (a sum of these over R gives the Hermitised interpolated
// matrix); neg [nR] int32 scratch receives the index of -R (entries of a vector
// whose negative is missing become NaN)
// halved R list of the folded R_e -> k contraction: neg[nR] (index of -R or
// -1), half[nR], pair[nR], R_half[nR][3], kh[1] = the list's length
void launch_half_list(int nR, const int32_t* R, int32_t* neg, int32_t* half, int32_t* pair, int32_t* R_half,
                      int32_t* kh, hipStream_t stream);
void launch_pack_upper(int n, int nR, const int32_t* R, const int32_t* ndeg, const void* X, int32_t* neg, void* P,
                       hipStream_t stream);

// ---- k_vertex.hip ----
enum class Prec { F64 = 0, F32 = 1, BF16X2 = 2 };

// exp(2 pi i p.R)/ndeg(R) -> [np][ld] complex in `prec` (columns >= nR zero;
// ndeg == nullptr: weight 1).
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

// a6: out[e][q][nu][i][j] (NBP-padded) = sum_a in[e][q][a][i][j] e_q[a][nu] sc[q][nu]
// ndeg_fold (optional): also multiply row e by 1/ndeg_fold[e] (the phase table
// of the following R_e -> k contraction then carries no 1/ndeg).
// Lq (optional, [nq][nm] c128, with Re): add Lq[q][nu] to the diagonal i == j
// of the row with R_e = 0 (the polar long-range term, in the Wannier basis).
void launch_mode_rotate(Prec prec, int ne, int nq, int nm, int nb, int nbp, const void* in,
                        const void* evec, const double* sc, void* out, hipStream_t stream,
                        const int32_t* ndeg_fold = nullptr, const void* Lq = nullptr,
                        const int32_t* Re = nullptr);

// a6 with the R_e rows folded by the pairs (R, -R) of the halved list (half,
// pair, kh as from launch_half_list): out holds B+ in row half[h] and B- in
// row pair[h] (B alone for an entry without a partner), each B(R) with its
// 1/ndeg[R]; the result of launch_mode_rotate with ndeg_fold = ndeg followed by
// the fold B+ = B(R) + B(-R), B- = B(R) - B(-R), in one pass
void launch_mode_rotate_fold(Prec prec, int ne, int nq, int nm, int nb, int nbp, const void* in, const void* evec,
                             const double* sc, const int32_t* ndeg, const int32_t* kh, const int32_t* half,
                             const int32_t* pair, const void* Lq, const int32_t* Re, void* out, hipStream_t stream);

// a6 for split-bf16: float32 g(R_e,q) [ne][qc][nm*nb*nb] -> four bf16 planes
// [4][qc*nm*nbp*nbp][kpad] (R_e contiguous), scaled by sc and rotated by e_q.
void launch_mode_rotate_bf16(int ne, int qc, int nm, int nb, int nbp, int kpad, const void* in, const void* evec,
                             const double* sc, void* out, hipStream_t stream, const int32_t* ndeg_fold = nullptr,
                             const void* Lq = nullptr, const int32_t* Re = nullptr);

// Split-bf16 complex GEMM C[m][n] (+)= sum_k A[m][k] B[n][k]: both operands
// as four bf16 planes (re_hi, re_lo, im_hi, im_lo) with K contiguous and
// zero-padded to Kpad (a multiple of 32); A plane p row m at A + p*aplane +
// m*lda (likewise B); C complex64 with row stride ldc.
struct Bf16GemmDesc {
    int M = 0;
    long N = 0;
    int Kpad = 0;
    const uint16_t* A = nullptr;
    long lda = 0, aplane = 0;
    const uint16_t* B = nullptr;
    long ldb = 0, bplane = 0;
    float2* C = nullptr;
    long ldc = 0;
    int accumulate = 0;
};
void launch_bf16_gemm(const Bf16GemmDesc& d, hipStream_t stream);
// conj(exp(2 pi i p.R)/ndeg(R)) split into four bf16 planes [4][nR][ld], the
// point index contiguous (zero for p >= np)
void launch_phase_planes_t(int np, const double* pts, int nR, const int32_t* R, const int32_t* ndeg, int ld,
                           void* out, hipStream_t stream);
// complex64 X [K][N] -> four bf16 planes [4][N][Kpad] (K contiguous, zero-padded)
void launch_split_transpose(int K, long N, const void* X, int Kpad, void* out, hipStream_t stream);

// Polar long-range factor L_nu(q) (k_polar.hip): the per-q Gaussian-damped
// sum over G of Sec. 4, for a chunk of q points.
struct PolarDev {
    int nat, gmax;
    double B[3][3];          // reciprocal vectors (rows, Cartesian)
    double tau[EPW_MAX_ATOMS][3];
    double zstar[EPW_MAX_ATOMS][3][3];
    double eps[3][3];
    double rsm[EPW_MAX_ATOMS];   // 1/sqrt(M_kappa)
    double prefactor, alpha, cutoff;
};
void launch_polar_factor(const PolarDev& P, int qc, int nm, const double* qfrac, const void* evec,
                         const double* sc, void* L, hipStream_t stream);

struct FusedArgs {
    int nk, ne, nb, nbp, nm;
    int qc;            // q points in this chunk
    int q0;            // global index of the first q of the chunk
    int nq_total;      // row length of kq
    const void* phi_k; // [nk][ldk] complex in prec (split-bf16: [4][nk][ldk] planes)
    int ldk;
    // phases generated in the kernel (nmax > 0) from per-axis factors
    // exp(2 pi i k_a n), |n| <= nmax, instead of read from phi_k
    int nmax;
    const int32_t* Re;     // [ne][3]
    const int32_t* ndeg_e; // [ne]
    const double* kfrac;   // [nk][3]
    int ldk_b;         // split-bf16: row length (kpad) of the B planes [4][cols][kpad]
    int kpad;          // split-bf16: K padded to a multiple of 32
    const void* B;     // [ne][qc*nm*nbp*nbp] complex in prec
    const double* eps; // [nk][nb]
    const void* U;     // [nk][nb][nb] c128
    const double* ftab;// [nk][nb]
    const int32_t* kq; // [nk][nq_total], or nullptr: per-pair states below
    const double* eps_pair;  // [nk][qc][nb]      eps at k+q (kq == nullptr)
    const void* U_pair;      // [nk][qc][nb][nb]  U at k+q (c128)
    const double* f_pair;    // [nk][qc][nb]      Fermi factors at k+q
    const double* omega;   // [qc][nm] (chunk-local)
    const double* nbose;   // [qc][nm] (chunk-local)
    const double* sc;      // [qc][nm] (chunk-local)
    double sigma;
    double mu;         // chemical potential (phonon mode)
    double* part;      // [S or 2 S][nk][nb] partial sums (imsigma mode): slot s of slice s,
                       // slot S + s of its tail when helper blocks run (fused_part_slots)
    int S;             // number of slices
    int helpers = 0;   // helper blocks beyond the tiles_m * S regular ones (fused_balance)
    int keep = 0x7fffffff;   // column tiles of its slice a regular block runs when helpers > 0
    void* gkq;         // [nk][nq_total][nm][nb][nb] c128 (store mode)
    double* part_ph;   // [2][tiles_m][qc*nm] per-row-tile sums (phonon mode): Eq. (9), Eq. (11)
    double* part2;     // [S or 2 S][nk][nb] second partials (real-part mode: Sigma' at omega = 0; part
                       // then holds Sigma' on shell)
    double* rec;       // [nk][qc][nm][nb] pole records of 4 + nbp doubles (pole mode)
    const double* vel; // [nk][nb][3] band velocities of the k set (transport mode, with part_ph)
    const double* vel_pair;  // [nk][qc][nb][3] velocities at k+q per pair (transport mode, off-grid)
    // folded R_e -> k contraction (fused_fold_c): B holds (B+, B-) in rows
    // (half[h], pair[h]) and phi_k the phases of R_half; kh[0] = number of
    // entries h
    const int32_t* half = nullptr;
    const int32_t* pair = nullptr;
    const int32_t* kh = nullptr;
    void* gout = nullptr;    // [nk][qc*nm*nbp*nbp] complex in prec: the Wannier-basis g_nu(k,q)
                             // itself (no rotation or reduction; float64 / float32, phase table)
};
// a7 alone (gout != nullptr: the adjoint's recomputed vertex), a7 + a8 + a9 (imsigma mode), a7 + a8 (store mode, gkq != nullptr),
// a7 + a8 + the phonon-linewidth sums (phonon mode, part_ph != nullptr), or
// a7 + a8 + the real-part sums of Eq. (3) (real-part mode, part2 != nullptr)
void launch_fused_k(Prec prec, const FusedArgs& a, int num_cu, hipStream_t stream);
int fused_slices(int nk, int nbp, int ncols_tiles, int num_cu, Prec prec);
// helper blocks and the regular blocks' share of their slices (a.helpers,
// a.keep) for a launch whose sizes and a.S are set; slots of a.part then
void fused_balance(FusedArgs& a, Prec prec, int num_cu);
inline int fused_part_slots(const FusedArgs& a) { return a.helpers > 0 ? 2 * a.S : a.S; }
// fused-kernel instantiations that run helper blocks: float32, and every
// precision at 16 padded bands (mode 0 float64, 1 float32, 2 split-bf16)
constexpr bool fused_balanced_c(int nbp, int mode) { return mode == 1 || nbp >= 16; }
// fused-kernel instantiations that fold the R_e -> k sum by pairs (R, -R):
// float64, and float32 up to 8 padded bands (at 16 its stages and the row
// indices would not fit two blocks per CU)
constexpr bool fused_fold_c(int nbp, int mode) { return mode == 0 || (mode == 1 && nbp <= 8); }
// columns and k rows per tile of the fused kernel for a padded band count:
// whole band blocks, at least 64 columns; 4096 complex entries, 8192 for
// float32 and split-bf16 at 16 bands (32 x 256); `wide` = not float64
constexpr int fused_tile_cols_c(int nbp, bool wide) { return nbp * nbp >= 64 ? nbp * nbp : 64; }
constexpr int fused_tile_rows_c(int nbp, bool wide) {
    return (wide && fused_tile_cols_c(nbp, wide) >= 256 ? 8192 : 4096) / fused_tile_cols_c(nbp, wide);
}
inline int fused_tile_cols(int nbp, Prec prec) { return fused_tile_cols_c(nbp, prec != Prec::F64); }
inline int fused_tile_rows(int nbp, Prec prec) { return fused_tile_rows_c(nbp, prec != Prec::F64); }
// raw[0] = sum_i exp(-((eps_i - mu)/sigma)^2) over n values (fixed order)
void launch_dos_raw(size_t n, const double* eps, double mu, double sigma, double* raw, hipStream_t stream);
// Pi''[q][nu] = 2 pi / (N_k sigma sqrt pi) sum_t part[0][t][q][nu];
// lam[q][nu] = sum_t part[1][t][q][nu] / (sigma sqrt(pi) raw_dos omega) (0 for cut modes or raw_dos = 0)
void launch_phonon_finalize(int qc, int nm, int tiles_m, const double* part_ph, const double* omega,
                            double omega_cut, const double* raw_dos, int nk, double sigma, double* pi_im,
                            double* lam, hipStream_t stream, double* lam_tr = nullptr);

// ---- k_gemm.hip ----
// C(m, n) (+)= sum_k A(m, k) B(k, n), complex in `prec` (F64 or F32).
//   A(m, k) = conj_trans_a ? conj(A[k*lda + m]) : A[m*lda + k]
//   n = e*ncb + c:  B(k, n) = B[e*sBe + k*sBk + c],  C(m, n) = C[e*sCe + m*sCm + c]
struct GemmDesc {
    int M = 0, N = 0, K = 0;
    const void* A = nullptr;
    long lda = 0;
    int conj_trans_a = 0;
    const void* B = nullptr;
    long sBe = 0, sBk = 0;
    int ncb = 1;
    void* C = nullptr;
    long sCe = 0, sCm = 0;
    int accumulate = 0;
    // pair operand (A2 != nullptr): A(m, k) = A[(r / n2) * lda + k] * A2[(r % n2) * lda + k] with
    // r = row0 + m -- the phases of the sum k + q of a point pair; with conj_trans_a,
    // A(m, k) = conj(A[(r / n2) * lda + m] * A2[(r % n2) * lda + m]) with r = row0 + k
    const void* A2 = nullptr;
    int n2 = 1;
    long row0 = 0;
    int kchunk = 0;    // split K: blockIdx.z covers [z*kchunk, (z+1)*kchunk) (0: all of K)
    long sCz = 0;      // C offset between the split-K partial outputs
    // folded sum (float64, pair operand, no conj_trans_a, no split K): K runs over
    // the kh[0] entries h of a halved R list (read on the device), A(m, h) = c + i s
    // is the pair operand over that list, B holds B+ rows and B2 the B- rows
    // (launch_fold_gather); C = sum_h c B+ + i s B-
    const int32_t* kh = nullptr;
    const void* B2 = nullptr;
};
// kparts > 1 launches that many K slices (d.kchunk must cover K)
void launch_cgemm(Prec prec, const GemmDesc& d, hipStream_t stream, int kparts = 1);
// B+ and B- rows of the halved R list for a folded float64 GEMM: for h < kh[0],
// x = B[half[h]] / ndeg[half[h]] and y = B[pair[h]] / ndeg[pair[h]] (rows of
// `cols` complex entries), Bp[h] = x + y and Bm[h] = x - y, or both x for an
// entry without a partner (pair[h] == half[h])
void launch_fold_gather(int nR, const int32_t* kh, const int32_t* half, const int32_t* pair, const int32_t* ndeg,
                        long cols, const void* B, void* Bp, void* Bm, hipStream_t stream);
// number of K slices launch_cgemm_splitk uses for an M x N x K product
int splitk_parts(int M, int N, int K);
// the same for products with very few output tiles (up to max_parts slices)
int splitk_parts_wide(int M, int N, int K, int max_parts);
// C (+)= A B as `parts` K slices into scratch ([parts][M][N] complex in prec),
// summed in fixed order into C; needs a single column slab (d.ncb == d.N)
void launch_cgemm_splitk(Prec prec, const GemmDesc& d, int parts, void* scratch, hipStream_t stream);

// the adjoint's sum over k folded by the pairs of the halved R list:
// C[e][col] = sum_k conj(Phi_k(R_e)) G[k][col] / ndeg(R_e) for every row e of
// C [ne][ncols], with phi the unweighted phases of R_half ([nk][ld]);
// `parts` K slices in scratch ([parts][ne][ncols]) summed in fixed order
struct KsumFoldDesc {
    int nk = 0, ne = 0;
    long ncols = 0;
    const void* phi = nullptr;
    int ld = 0;
    const void* G = nullptr;
    const int32_t* half = nullptr;
    const int32_t* pair = nullptr;
    const int32_t* kh = nullptr;
    const int32_t* ndeg = nullptr;
    void* out = nullptr;     // set by the launcher
    int kchunk = 0;          // set by the launcher
};
void launch_ksum_fold(Prec prec, const KsumFoldDesc& d, int parts, void* scratch, void* C, hipStream_t stream);

// ---- k_backward.hip (adjoint of L = sum_nk w_nk Im Sigma_nk) ----
struct PairBwdArgs {
    int nk, nb, nbp, nm;
    int qc, q0, nq_total;
    void* G;               // [nk][qc*nm*nbp*nbp] complex(prec): Wannier-basis g_nu(k,q) in,
                           // adjoint Gbar out (in place)
    const double* eps;     // [nk][nb]
    const void* U;         // [nk][nb][nb] c128
    const double* ftab;    // [nk][nb]
    const double* wbar;    // [nk][nb] degenerate-averaged loss weights
    const int32_t* kq;     // [nk][nq_total], or nullptr: per-pair states below
    const double* eps_pair;  // [nk][qc][nb]
    const void* U_pair;      // [nk][qc][nb][nb] c128
    const double* f_pair;    // [nk][qc][nb]
    const double* omega;   // [qc][nm]
    const double* nbose;   // [qc][nm]
    const double* sc;      // [qc][nm]
    double sigma, kT, C;   // C = pi / (N_q sigma sqrt(pi))
    double* ek_c;          // [nk][qc][nb]      d/d eps_nk
    void* Uk_c;            // [nk][qc][nb][nb]  d/dU_k
    double* ekq_c;         // [nk][qc][nb]      d/d eps_m,k+q
    void* Ukq_c;           // [nk][qc][nb][nb]  d/dU_k+q
    double* om_c;          // [nk][qc][nm]      d/d omega
};
void launch_pair_bwd(Prec prec, const PairBwdArgs& a, hipStream_t stream);
// inv[k'][j] = k with kq[k][q0+j] = k', else -1   (j < qc)
void launch_kq_inverse(int nk, int qc, int q0, int nq_total, const int32_t* kq, int32_t* inv,
                       hipStream_t stream);
// ebar[k] += sum_j ek_c[k][j] + ekq_c[inv[k][j]][j];  Ubar likewise (fixed order);
// inv == nullptr: the k side only (off-grid runs, whose k+q states are per pair)
void launch_gather_state_adjoint(int nk, int nb, int qc, const int32_t* inv, const double* ek_c,
                                 const void* Uk_c, const double* ekq_c, const void* Ukq_c,
                                 double* ebar, void* Ubar, hipStream_t stream);
// domega[q][nu] (+)= sum_k om_c[k][q][nu] (fixed order)
void launch_reduce_omega(int nk, int qc, int nm, const double* om_c, int accumulate, double* domega,
                         hipStream_t stream);
// gbar_a[e][q][a][i][j] = sum_nu conj(e_q[a][nu]) sc[q][nu] gbar_nu[e][q][nu][i][j]  (i, j < nb)
void launch_mode_rotate_adjoint(Prec prec, int ne, int nq, int nm, int nb, int nbp, const void* gnu,
                                const void* evec, const double* sc, void* ga, hipStream_t stream);
// Xbar(k) from (eps, U, ebar, Ubar): Hermitian part of U (F o U^dag Ubar + diag ebar) U^dag
void launch_eigh_adjoint(int nk, int nb, const double* eps, const void* U, const double* ebar,
                         const void* Ubar, double deg_tol, void* Xbar, hipStream_t stream);
// f64 fill
void launch_fill(size_t n, double v, double* p, hipStream_t stream);
// dst[i] += src[i] (n doubles)
void launch_add_f64(size_t n, const double* src, double* dst, hipStream_t stream);
// convert c64 -> c128 with optional accumulate
void launch_c64_to_c128(size_t n, const void* in, int accumulate, void* out, hipStream_t stream);

// imsig[k][n] = (acc ? imsig : 0) + scale * sum_s part[s][k][n]
void launch_reduce_partials(int nk, int nb, int S, const double* part, double scale,
                            int accumulate, double* imsig, hipStream_t stream);
// out[k][n] = (acc ? out : 0) + scale * sum_s (A[s][k][n] - B[s][k][n])  (fixed order)
void launch_reduce_partials_diff(int nk, int nb, int S, const double* A, const double* B, double scale,
                                 int accumulate, double* out, hipStream_t stream);
// average over bands whose consecutive energies differ by < tol
// Frequency-resolved Eq. (3) from pole records (k_spectral.hip): slices of
// the pole list per (k, frequency tile), their fixed-order reduction (with the
// degenerate average, scaled, accumulated into out [nk][nb][nw] c128 and, for
// omega = 0, out0 [nk][nb] c128), and Eq. (10).
int sigma_omega_slices(int nk, int nw, long npole);
void launch_sigma_omega(int nk, int nb, long npole, int nw, const double* wgrid, double delta, const double* rec,
                        int S, void* part, hipStream_t stream);
void launch_sigma_omega_reduce(int nk, int nb, int nw, int S, const void* part, const double* eps, double tol,
                               double scale, int acc, void* out, void* out0, hipStream_t stream);
void launch_spectral_function(int nk, int nb, int nw, const double* eps, double mu, const double* wgrid,
                              const void* sig, const void* sig0, double* A, hipStream_t stream);

// k-outer pole records: from the Wannier-basis vertex C[k][q][nm][nb][nb]
// (complex, float64 or float32), the mode rotation (with 1/sqrt(2 omega) and
// the polar term), the band rotation and the record layout of the fused
// kernel's pole mode (4 + nbp doubles per (k, q, nu, m)).
struct PairPoleArgs {
    int nk, nb, nbp, nm, qc, q0, nq_total;
    const void* C;
    int c64;
    const void* U;              // [nk][nb][nb] c128
    const int32_t* kq;          // [nk][nq_total] or NULL (then the pair states)
    const double* eps;          // [nk][nb]
    const double* ftab;         // [nk][nb]
    const double* eps_pair;     // [nk][qc][nb]
    const double* f_pair;       // [nk][qc][nb]
    const void* U_pair;         // [nk][qc][nb][nb] c128
    const double* omega;        // [qc][nm]
    const double* nbose;        // [qc][nm]
    const double* sc;           // [qc][nm]
    const void* evec;           // [qc][nm][nm] c128
    const void* Lq;             // [qc][nm] c128 or NULL
    double mu;
    double* rec;
};
void launch_pair_pole(const PairPoleArgs& a, hipStream_t stream);

// Transport (k_transport.hip): band velocities v_nk = Re diag(U^dag dH/dk U),
// averaged over degenerate bands, at np points (vectors: Cartesian primitive
// rows); alpha^2 F on a frequency grid; the Ziman resistivity integral.
void launch_velocities(int nb, int nR, const int32_t* R, const int32_t* ndeg, const void* HR, const double* vectors9,
                       int np, const double* kfrac, const double* eps, const void* U, double deg_tol, double* vel,
                       hipStream_t stream);
// i R_a H(R) for a = x, y, z (R Cartesian): [3][nR][nb][nb] c128
void launch_velocity_operands(int nb, int nR, const int32_t* R, const void* HR, const double* vectors9, void* dHR3,
                              hipStream_t stream);
// velocities of np pairs from dH/dk_a [3][ld][nb][nb] (ld = batch stride),
// eigenvectors U [np][nb][nb] and energies eps [np][nb] (degenerate average)
void launch_pair_velocities(int nb, int np, long ld, const void* dH3, const void* U, const double* eps, double deg_tol,
                            double* vel, hipStream_t stream);
void launch_eliashberg(int nq, int nm, const double* omega, const double* lam, double nq_norm, int nw,
                       const double* wgrid, double sigma, double* a2f, hipStream_t stream);
void launch_ziman(int nw, const double* wgrid, const double* a2f, int nT, const double* T, double* out,
                  hipStream_t stream);
void launch_degenerate_average(int nk, int nb, const double* eps, double tol, double* v,
                               hipStream_t stream);

// ---- k_check.hip (epw_check_inputs) ----
struct CheckRecord {
    int32_t nonfinite;          // bits: 1 H, 2 D, 4 g, 8 points, 16 given phonon states
    int32_t ndeg_bad;           // bits: 1 R_e, 2 R_p (ndeg < 1)
    int32_t nmax_bad;           // 1: a component of R_e exceeds nmax_e
    int32_t not_closed;         // bits: 1 R_e, 2 R_p (-R missing)
    int32_t kq_range;           // 1: a kq entry outside [0, nk)
    int32_t kq_not_bijective;   // 1: for some q, k -> kq[k][q] is not one-to-one
    unsigned long long h_dev, h_max, d_dev, d_max;   // bit patterns of non-negative doubles
};
void launch_check_clear(CheckRecord* rec, hipStream_t st);
void launch_check_finite(size_t n, const double* x, int bit, CheckRecord* rec, hipStream_t st);
void launch_check_ws(int nR, const int32_t* R, const int32_t* ndeg, int nmax, int bit, int32_t* neg,
                     CheckRecord* rec, hipStream_t st);
void launch_check_herm(bool cplx, int n, int nR, const double* X, const int32_t* neg, unsigned long long* dev_slot,
                       unsigned long long* max_slot, hipStream_t st);
void launch_check_kq(int nk, int qc, int q0, int nq_total, const int32_t* kq, int32_t* inv, CheckRecord* rec,
                     hipStream_t st);

}  // namespace epw
