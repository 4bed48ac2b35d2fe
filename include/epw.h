/*
 * epw.h - C ABI of libepw: Wannier-Fourier interpolation of electrons,
 * phonons and the electron-phonon vertex onto fine k/q points, and the
 * imaginary electron self-energy (linewidth) of the EPW method
 * (Ponce, Margine, Verdi, Giustino, arXiv:1604.03525), for AMD MI355X
 * (gfx950).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Array arguments marked "device" are HIP device pointers owned by the
 *    caller; "host" arrays live in host memory.  The library never frees
 *    or retains a pointer after the call returns.
 *  - Arrays are C-contiguous (row-major).  Complex numbers are interleaved
 *    (re, im) pairs of double ("c128").
 *  - Device calls are enqueued on the caller's stream (a hipStream_t passed
 *    as void*, NULL = the default stream) and return before the work ends.
 *  - Every call returns an int status: EPW_OK (0) or a negative code; the
 *    message of the last failure on the calling thread is returned by
 *    epw_last_error().  Argument checks happen before anything is enqueued,
 *    so a failed call leaves outputs untouched.
 *  - The library allocates no device memory.  Calls that need scratch take
 *    a caller-allocated device workspace (ws, ws_bytes); its size comes
 *    from epw_workspace_size().  Concurrent calls must use distinct
 *    workspaces.  (epw_imsigma_noalloc instead uses a static device array
 *    of the library, see there.)
 *  - Units: energies in eV, temperature in K, hbar = 1.  Points are in
 *    fractional (reciprocal-lattice) coordinates, real-space vectors in
 *    integer lattice coordinates.
 *  - Interpolation convention (the paper cites it, Sec. 1 and Sec. 8 step
 *    (iii), without printing it): X(p) = sum_R exp(+2 pi i p.R) X(R)/ndeg(R)
 *    over the Wigner-Seitz vectors R with degeneracy weights ndeg.
 */
#ifndef EPW_H
#define EPW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define EPW_OK        0
#define EPW_EINVAL   -1   /* NULL pointer or invalid scalar parameter            */
#define EPW_ESHAPE   -2   /* unsupported or inconsistent sizes                   */
#define EPW_EDTYPE   -3   /* unknown precision selector                          */
#define EPW_ENOTHERM -4   /* H(-R) != H(R)^dag or D(-R) != D(R)^T beyond tolerance */
#define EPW_ENOMEM   -5   /* workspace (or host capacity) too small              */
#define EPW_EHIP     -6   /* the HIP runtime reported an error                   */

/* ---- precision of the contractions and rotations ----
 * Eigensolves, phase arguments k.R, occupations and the degenerate-subspace
 * logic are float64 in every mode. */
#define EPW_FP64        0   /* complex float64 on MFMA                              */
#define EPW_FP32        1   /* complex float32 on MFMA, float32 accumulation        */
#define EPW_SPLIT_BF16  2   /* x = hi + lo in bfloat16, three products per real
                               product on MFMA, float32 accumulation               */

/* ---- size limits ---- */
#define EPW_MAX_NB  16      /* Wannier bands                                        */
#define EPW_MAX_NM  16      /* phonon modes (3 x atoms)                             */
#define EPW_MAX_NW  (1 << 20) /* frequencies of epw_selfenergy_omega                  */
#define EPW_MAX_ATOMS 5     /* atoms of the polar long-range term (3 x 5 <= 16)   */
#define EPW_MAX_GMAX  24    /* half-width of the G box of the polar term          */

/* Message of the last failed call on this thread ("" if none). */
const char* epw_last_error(void);

/* Library version, 100*major + minor. */
int epw_version(void);

/* ======================================================================
 * Host-side integer steps (no GPU involved, bit-exact)
 * ====================================================================== */

/* Wigner-Seitz vectors of the ncell[0] x ncell[1] x ncell[2] supercell
 * (the real-space support of the interpolation; Sec. 1, Sec. 8 step (ii)).
 *  metric  host [9]  integer metric G_ab = a_a.a_b of the primitive vectors
 *                    (any common positive scale), row-major, positive definite
 *  ncell   host [3]  supercell size N_a >= 1 (the coarse k/q grid)
 *  R       host [cap][3] out: vectors n with |n|_G <= |n - T|_G for every
 *                    supercell vector T = (N1 t1, N2 t2, N3 t3), t in {-2..2}^3,
 *                    lexicographically ascending
 *  ndeg    host [cap] out: number of T attaining equality (T = 0 included)
 *  cap     capacity of R and ndeg; *count receives the number of vectors.
 * Errors: EPW_EINVAL (NULL, N_a < 1, metric not positive definite),
 *         EPW_ENOMEM (cap < count; *count is still set). */
int epw_ws_vectors(const int64_t metric[9], const int32_t ncell[3],
                   int32_t* R, int32_t* ndeg, int32_t cap, int32_t* count);

/* Gamma-centred grid n[0] x n[1] x n[2] (Sec. 8, Sec. 10.2): point
 * i = (i1*n1 + i2)*n2 + i3 gets (i1/n0, i2/n1, i3/n2).
 *  out host [n0*n1*n2][3] double.  Errors: EPW_EINVAL. */
int epw_grid_points(const int32_t n[3], double* out);

/* Index of k+q (folded into [0,1)^3) in the k grid for Gamma-centred grids
 * with kgrid[a] a multiple of qgrid[a]:
 *  out host [Nk][Nq] int32, k and q in the C order of epw_grid_points.
 * Errors: EPW_EINVAL (NULL), EPW_ESHAPE (incommensurate grids). */
int epw_kq_index(const int32_t kgrid[3], const int32_t qgrid[3], int32_t* out);

/* ======================================================================
 * Device steps
 * ====================================================================== */

/* Electron bands at arbitrary points: H(k) = sum_R exp(2 pi i k.R) H(R)/ndeg,
 * Hermitised, diagonalised in float64 (Jacobi) -> eps ascending, U columns.
 * (The paper obtains the rotation matrices U_k at arbitrary k from the
 * interpolated Hamiltonian: Sec. 4, after the overlap formula.)
 *  nb              bands, 1..EPW_MAX_NB
 *  nR, R, ndeg     device [nR][3] int32, [nR] int32 (WS set, ndeg >= 1)
 *  HR              device [nR][nb][nb] c128
 *  nk, kfrac       device [nk][3] double
 *  eps             device [nk][nb] double out
 *  U               device [nk][nb][nb] c128 out (U[k][i][n]: orbital i of band n)
 * Errors: EPW_EINVAL, EPW_ESHAPE, EPW_EHIP. */
int epw_interp_bands(int nb, int nR, const int32_t* R, const int32_t* ndeg,
                     const void* HR, int nk, const double* kfrac,
                     double* eps, void* U, void* stream);

/* Phonons at arbitrary points: D(q) = sum_R exp(2 pi i q.R) D(R)/ndeg with
 * the masses folded into D (Sec. 3, after Eq. (2)), Hermitised and
 * diagonalised in float64; omega = sign(l) sqrt|l| per eigenvalue l.
 *  nm              modes, 1..EPW_MAX_NM
 *  DR              device [nR][nm][nm] double (real force constants / masses)
 *  omega           device [nq][nm] double out (ascending)
 *  evec            device [nq][nm][nm] c128 out (columns)
 * Errors: EPW_EINVAL, EPW_ESHAPE, EPW_EHIP. */
int epw_interp_phonons(int nm, int nR, const int32_t* R, const int32_t* ndeg,
                       const double* DR, int nq, const double* qfrac,
                       double* omega, void* evec, void* stream);

/* Long-range (polar) part of the vertex, Sec. 4:
 *   g_mn,nu(k,q) = g^S_mn,nu(k,q) + L_nu(q) [U_k+q^dagger U_k]_mn
 *   L_nu(q) = i C sum_kappa (2 M_kappa omega_q,nu)^(-1/2) sum_{G, K = q+G != 0}
 *             exp(-K.eps.K/(4 alpha)) / (K.eps.K) (K . Z*_kappa . e_kappa,nu(q))
 *             exp(-i K . tau_kappa)
 * (the overlap in the small-(q+G) form of Sec. 4; the Gaussian damping, the
 * atomic phase and the overall factor C = 4 pi e^2 / Omega are those of the
 * method the paper cites, absent from its printed equation).  The
 * interpolated g(R_e,R_p) is then the short-range part g^S.  Host struct,
 * copied into the kernel arguments; all vectors Cartesian in one length unit
 * (K in the inverse unit, 2 pi included). */
typedef struct {
    int32_t nat;                          /* atoms, 3 nat = nm, 1..EPW_MAX_ATOMS  */
    int32_t reserved;
    double vectors[3][3];                 /* primitive lattice vectors a_i (rows) */
    double tau[EPW_MAX_ATOMS][3];         /* atomic positions in the cell         */
    double zstar[EPW_MAX_ATOMS][3][3];    /* Born charges Z*_kappa[a][b]: K_a Z_ab e_b */
    double eps_inf[3][3];                 /* dielectric tensor (symmetric, > 0)   */
    double mass[EPW_MAX_ATOMS];           /* M_kappa (> 0), the mass unit of D    */
    double prefactor;                     /* C                                    */
    double alpha;                         /* Gaussian parameter (> 0)             */
    double cutoff;                        /* keep terms with K.eps.K/(4 alpha) <
                                             cutoff (> 0); the G box this needs
                                             must fit EPW_MAX_GMAX               */
} epw_polar;

/* Real-space system shared by the vertex and self-energy calls. */
typedef struct {
    int32_t nb;            /* Wannier bands (1..EPW_MAX_NB)                      */
    int32_t nm;            /* phonon modes = 3 x atoms (1..EPW_MAX_NM)           */
    int32_t nRe;           /* electron WS vectors                                */
    int32_t nRp;           /* phonon WS vectors                                  */
    const int32_t* Re;     /* device [nRe][3]                                    */
    const int32_t* ndeg_e; /* device [nRe]                                       */
    const int32_t* Rp;     /* device [nRp][3]                                    */
    const int32_t* ndeg_p; /* device [nRp]                                       */
    const void* HR;        /* device [nRe][nb][nb] c128                          */
    const double* DR;      /* device [nRp][nm][nm] double; may be NULL when
                              phonon states are given in epw_points              */
    const void* gR;        /* device [nRe][nRp][nm][nb][nb] c128: g_{ka}(R_e,R_p),
                              row index = Wannier function on the k+q side      */
    int32_t nmax_e;        /* optional: max |Re[r][a]| over all r, a.  When set
                              (1..EPW_MAX_NMAX) the electron phases of the R_e -> k
                              contraction are generated in the kernel from
                              per-axis factors exp(2 pi i k_a n) instead of being
                              streamed from a table; 0 = use the table.  A value
                              smaller than the true maximum gives wrong results. */
    int32_t reserved;
    const epw_polar* polar;  /* optional long-range term, NULL = none: used by
                              every forward call and by the adjoint             */
} epw_system;

#define EPW_MAX_NMAX 8

/* Fine points. */
typedef struct {
    int32_t nk;            /* number of k points                                 */
    int32_t nq;            /* number of q points                                 */
    const double* kfrac;   /* device [nk][3]                                     */
    const double* qfrac;   /* device [nq][3]                                     */
    const int32_t* kq;     /* device [nk][nq]: index in the k set of the point
                              equal to k+q modulo a reciprocal lattice vector
                              (grid runs), or NULL: the k+q states are then
                              interpolated and diagonalised for every pair       */
    const double* omega;   /* device [nq][nm] or NULL: given phonon frequencies  */
    const void* evec;      /* device [nq][nm][nm] c128 or NULL: given modes.  When
                              both are set, DR is not used.                      */
} epw_points;

/* Physical and numerical parameters of Eq. (8). */
typedef struct {
    double T;              /* temperature (K), >= 0                              */
    double mu;             /* chemical potential = Fermi level (eV)              */
    double sigma;          /* Gaussian width (eV), > 0: delta(x) ->
                              exp(-x^2/sigma^2)/(sigma sqrt(pi))                  */
    double omega_cut;      /* modes with omega < omega_cut contribute 0 (eV)      */
    double deg_tol;        /* bands closer than this are averaged (eV), >= 0     */
    double nq_norm;        /* N_q of the BZ mean (1/N_q) sum_q; 0 -> nq          */
    int32_t dtype;         /* EPW_FP64 / EPW_FP32 / EPW_SPLIT_BF16               */
    int32_t chunk_q;       /* q points per chunk (0 = choose from the workspace) */
    int32_t accumulate;    /* 0: overwrite the output, 1: add to it              */
    int32_t order;         /* contraction order of epw_selfenergy_omega (other
                              calls ignore it): EPW_ORDER_AUTO, EPW_ORDER_K_INNER
                              (per q chunk R_p -> q, then R_e -> k fused with the
                              rotation) or EPW_ORDER_K_OUTER (R_e -> k once for
                              all k, then R_p -> q per chunk and a per-pair
                              rotation; cheaper when n_k is small against N_e) */
} epw_params;

#define EPW_ORDER_AUTO     0   /* k-outer when 4 n_k <= N_e */
#define EPW_ORDER_K_INNER  1
#define EPW_ORDER_K_OUTER  2

/* Electron-phonon vertex in the band/mode basis (Sec. 3 Eq. (2)):
 *   g_mn,nu(k,q) = [U_{k+q}^dag (sum_ka g_ka(k,q) e_ka,nu(q)) U_k]_mn / sqrt(2 omega_q,nu)
 *   g_ka(k,q)   = sum_{R_e,R_p} exp(2 pi i (k.R_e + q.R_p)) g_ka(R_e,R_p)/(ndeg_e ndeg_p)
 * materialised for every pair (meant for small sizes and tests); modes with
 * omega < par->omega_cut are set to 0.  Only par->dtype and par->omega_cut
 * are read.
 *  gkq  device [nk][nq][nm][nb][nb] c128 out
 * The band-basis vertex depends on the eigenvector gauge; gauge-invariant
 * combinations (sums of |g|^2 over degenerate states) are what compare
 * between implementations.
 * Errors: EPW_EINVAL, EPW_ESHAPE, EPW_EDTYPE, EPW_ENOMEM, EPW_EHIP. */
int epw_interp_g(const epw_system* sys, const epw_points* pts, const epw_params* par,
                 void* gkq, void* ws, size_t ws_bytes, void* stream);

/* Imaginary electron self-energy on shell, Sec. 3 Eq. (8):
 *   Im Sigma_nk = (pi/N_q) sum_q sum_m,nu |g_mn,nu(k,q)|^2
 *       { [n_q,nu + f_m,k+q] delta(eps_nk - eps_m,k+q + omega_q,nu)
 *       + [n_q,nu + 1 - f_m,k+q] delta(eps_nk - eps_m,k+q - omega_q,nu) }
 * with n the Bose and f the Fermi-Dirac function at T, then averaged over
 * bands degenerate within deg_tol.  The scattering rate of the Sec. 10.2
 * example is 2 Im Sigma.
 *  imsig  device [nk][nb] double out (overwritten or accumulated)
 * Errors: EPW_EINVAL, EPW_ESHAPE, EPW_EDTYPE, EPW_ENOMEM, EPW_EHIP. */
int epw_imsigma(const epw_system* sys, const epw_points* pts, const epw_params* par,
                double* imsig, void* ws, size_t ws_bytes, void* stream);

/* Im Sigma exactly as epw_imsigma, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): there is no workspace argument and the call allocates nothing.
 * Its scratch is a library-owned device array of EPW_NOALLOC_SCRATCH_BYTES
 * on each GPU, held from the first call on that GPU until the process ends.
 *  - The array of the current device (hipGetDevice) is used: the stream and
 *    every pointer must belong to that device.
 *  - par->chunk_q = 0 takes the largest q chunk whose scratch fits the array;
 *    a given chunk_q must fit as it is.  Sizes that do not fit (even one q
 *    point at a time, or the given chunk) fail with EPW_ENOMEM before any
 *    device work.
 *  - Every call on one GPU shares that GPU's array, which keeps the last
 *    call's contents (nothing in it is assumed to start at zero).  Calls
 *    ordered on one stream are safe; calls that overlap on one GPU (other
 *    streams, or host threads with no ordering between them) race on the
 *    array and give wrong results.
 * Errors: as epw_imsigma. */
#define EPW_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int epw_imsigma_noalloc(const epw_system* sys, const epw_points* pts, const epw_params* par,
                        double* imsig, void* stream);

/* Real part of the electron self-energy, Sec. 3 Eq. (3), on shell, and its
 * Fermi-level-referenced form, Sec. 3 Eq. (5):
 *   Sigma'_nk(omega) = (1/N_q) sum_q sum_m,nu |g_mn,nu(k,q)|^2 Re{
 *       [n_q,nu + f_m,k+q] / (omega - (eps_m,k+q - eps_F) + omega_q,nu + i delta)
 *     + [n_q,nu + 1 - f_m,k+q] / (omega - (eps_m,k+q - eps_F) - omega_q,nu + i delta) }
 *   re_shell = Sigma'_nk(eps_nk - eps_F),  re_tilde = re_shell - Sigma'_nk(0)
 * with eps_F = mu and delta = par->sigma; occupations, nq_norm, omega_cut,
 * chunking, accumulate and the degenerate average as for epw_imsigma.
 *  re_shell  device [nk][nb] double out
 *  re_tilde  device [nk][nb] double out, or NULL to skip
 * Errors: as epw_imsigma. */
int epw_resigma(const epw_system* sys, const epw_points* pts, const epw_params* par, double* re_shell,
                double* re_tilde, void* ws, size_t ws_bytes, void* stream);

/* The complex electron self-energy of Sec. 3 Eq. (3) on a frequency grid:
 *   Sigma_nk(omega) = (1/N_q) sum_q sum_m,nu |g_mn,nu(k,q)|^2 {
 *       [n_q,nu + f_m,k+q] / (omega - (eps_m,k+q - eps_F) + omega_q,nu + i delta)
 *     + [n_q,nu + 1 - f_m,k+q] / (omega - (eps_m,k+q - eps_F) - omega_q,nu + i delta) }
 * with omega measured from eps_F = mu and delta = par->sigma, at every
 * wgrid[j] and at omega = 0 (the Sigma'(eps_F) of Eq. (5)).  Each q chunk
 * writes one record per (k, q, nu, m) to the workspace (8 (4 + nb) bytes),
 * then a second kernel sums the records per frequency.  Occupations,
 * nq_norm, omega_cut, chunking, accumulate and the degenerate average (at
 * every frequency) as for epw_imsigma; the precision selects the contraction
 * arithmetic, the frequency sums are float64.
 *  nw       frequencies, 0..EPW_MAX_NW
 *  wgrid    device [nw] double (eV, from eps_F)
 *  sigma_w  device [nk][nb][nw] c128 out (overwritten or accumulated)
 *  sigma0   device [nk][nb] c128 out: Sigma_nk(omega = 0)
 *  ws       workspace of epw_workspace_size_omega() bytes
 * Errors: as epw_imsigma; EPW_ESHAPE for nw out of range. */
int epw_selfenergy_omega(const epw_system* sys, const epw_points* pts, const epw_params* par, int nw,
                         const double* wgrid, void* sigma_w, void* sigma0, void* ws, size_t ws_bytes,
                         void* stream);

/* Workspace bytes of epw_selfenergy_omega for nw frequencies (0 on error). */
size_t epw_workspace_size_omega(const epw_system* sys, const epw_points* pts, const epw_params* par, int nw);

/* The electronic spectral function of Sec. 3 Eq. (10) from a frequency-
 * resolved self-energy, with Sigma~' of Sec. 3 Eq. (5):
 *   A_nk(omega) = (1/pi) |Sigma''| / ((omega - (eps_nk - mu) - Sigma~')^2 + Sigma''^2)
 *   Sigma~' = Re Sigma_nk(omega) - Re Sigma_nk(0),  Sigma'' = Im Sigma_nk(omega)
 * (the squared Sigma'' of the denominator makes A a normalised density).
 *  eps      device [nk][nb] double: band energies at the k points (eV)
 *  wgrid    device [nw] double (eV, from eps_F = mu)
 *  sigma_w  device [nk][nb][nw] c128, sigma0 device [nk][nb] c128 (as
 *           written by epw_selfenergy_omega)
 *  A        device [nk][nb][nw] double out (1/eV)
 * Errors: EPW_ESHAPE, EPW_EINVAL (NULL pointer, mu not finite), EPW_EHIP. */
int epw_spectral_function(int nk, int nb, int nw, const double* eps, double mu, const double* wgrid,
                          const void* sigma_w, const void* sigma0, double* A, void* stream);

/* Band velocities for the transport coupling (Sec. 6; the analytic
 * derivative of the interpolated bands, the Wannier route Sec. 7 names):
 *   v_nk,a = Re [U_k^dag (dH/dk_a) U_k]_nn,
 *   dH/dk_a = Hermitised sum_R i R_a exp(2 pi i k.R) H(R)/ndeg(R), R Cartesian
 * (R_cart = R . vectors), averaged over bands whose sorted energies differ
 * by < deg_tol (the trace over a degenerate subspace is basis independent).
 *  vectors  host [3][3] double: primitive lattice vectors (rows, Cartesian)
 *  eps, U   device out, as epw_interp_bands
 *  vel      device [nk][nb][3] double out (energy x length)
 * Errors: EPW_ESHAPE, EPW_EINVAL, EPW_EHIP. */
int epw_band_velocities(int nb, int nR, const int32_t* R, const int32_t* ndeg, const void* HR,
                        const double* vectors, int nk, const double* kfrac, double deg_tol, double* eps,
                        void* U, double* vel, void* stream);

/* Mode-resolved transport coupling strength, Sec. 6 Eq. (55):
 *   lambda_tr,q,nu = 1 / (N(eps_F) omega_q,nu) (1/N_k) sum_k sum_mn |g_mn,nu(k,q)|^2
 *       delta(eps_nk - eps_F) delta(eps_m,k+q - eps_F) (1 - v_nk . v_m,k+q / |v_nk|^2)
 * with the velocities of epw_band_velocities (the factor is 1 where
 * |v_nk|^2 <= 1e-18), N(eps_F), the deltas and the degenerate-mode average
 * as for lambda_q,nu (epw_phonon_selfenergy), which comes out of the same
 * pass together with Pi''.  Without a k+q map the velocities at k+q are
 * formed per pair, from dH/dk at k+q summed like H(k+q).
 *  vectors  host [3][3] double: primitive lattice vectors (rows, Cartesian)
 *  lam_tr   device [nq][nm] double out; lam, pi_im device [nq][nm] or NULL
 * Errors: as epw_phonon_selfenergy. */
int epw_transport_coupling(const epw_system* sys, const epw_points* pts, const epw_params* par,
                           const double* vectors, double* lam_tr, double* lam, double* pi_im, void* ws,
                           size_t ws_bytes, void* stream);

/* Eliashberg function, Sec. 3 Eq. (12) (from lambda_q,nu) or its transport
 * form Sec. 6 Eq. (54) (from lambda_tr,q,nu), on a frequency grid:
 *   a2F(w_j) = (1/2) (1/nq_norm) sum_q,nu omega_q,nu lambda_q,nu delta_s(w_j - omega_q,nu)
 * with the Gaussian delta_s(x) = exp(-x^2/s^2)/(s sqrt(pi)), s = sigma.
 *  omega, lam  device [nq][nm] double; wgrid device [nw]; a2f device [nw] out
 * Errors: EPW_ESHAPE, EPW_EINVAL, EPW_EHIP. */
int epw_eliashberg_function(int nq, int nm, const double* omega, const double* lam, double nq_norm, int nw,
                            const double* wgrid, double sigma, double* a2f, void* stream);

/* Ziman resistivity, Sec. 6 Eq. (53), without its material prefactor:
 *   out[i] = rho(T_i) n e^2 / m_e = (4 pi / (k_B T_i)) int dw w a2F_tr(w) n(w) [1 + n(w)]
 * by the trapezoid rule over the grid (integrand 0 for w <= 0; out = 0 at
 * T = 0); energies in eV, k_B in eV/K, hbar = 1.
 *  wgrid, a2f_tr device [nw]; T device [nT] (K); out device [nT] out
 * Errors: EPW_ESHAPE, EPW_EINVAL, EPW_EHIP. */
int epw_ziman_resistivity(int nw, const double* wgrid, const double* a2f_tr, int nT, const double* T,
                          double* out, void* stream);

/* Phonon linewidth, Sec. 3 Eq. (9), on shell (omega = omega_q,nu), and the
 * mode-resolved electron-phonon coupling strength, Sec. 3 Eq. (11):
 *   Pi''_q,nu = (2 pi / N_k) sum_k sum_mn |g_mn,nu(k,q)|^2
 *                  [f_nk - f_m,k+q] delta(eps_nk - eps_m,k+q - omega_q,nu)
 *   lambda_q,nu = 1/(N(eps_F) omega_q,nu N_k) sum_k sum_mn |g_mn,nu(k,q)|^2
 *                  delta(eps_nk - mu) delta(eps_m,k+q - mu)
 *   N(eps_F) = (1/N_k) sum_nk delta(eps_nk - mu)   (per spin, on the k set)
 * with eps_F = mu, the Gaussian delta and the Fermi-Dirac f of epw_imsigma.
 * The sign is that of the printed delta argument (the magnitude is the
 * linewidth).  Modes with omega < omega_cut give 0; lambda is 0 where
 * N(eps_F) = 0.  Both are averaged over modes of one q whose frequencies
 * differ by less than deg_tol.  The k sum is over the whole k set of the
 * call (par->nq_norm and par->accumulate are not used); q is chunked as in
 * epw_imsigma; grid (kq) and off-grid k+q as in epw_imsigma.
 *  pi_im  device [nq][nm] double out (overwritten)
 *  lam    device [nq][nm] double out (overwritten), or NULL to skip
 * Errors: EPW_EINVAL, EPW_ESHAPE (also for an empty k set), EPW_EDTYPE,
 * EPW_ENOMEM, EPW_EHIP. */
int epw_phonon_selfenergy(const epw_system* sys, const epw_points* pts, const epw_params* par,
                          double* pi_im, double* lam, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of L = sum_nk w_nk Im Sigma_nk (the forward of epw_imsigma) with
 * respect to g(R_e,R_p), H(R_e) and omega_q,nu.  Complex gradients are
 * dL/dRe + i dL/dIm; H(k) is the Hermitised sum, so every entry of H(R) is
 * an independent complex parameter; dL/domega is taken at fixed e_q (through
 * the Bose factor, the Gaussians and 1/sqrt(2 omega)) and is 0 for cut
 * modes.  The rotated vertex is recomputed, not stored.
 *  w       device [nk][nb] double
 *  dgR     device [nRe][nRp][nm][nb][nb] c128 out (NULL to skip)
 *  dHR     device [nRe][nb][nb] c128 out (NULL to skip).  On grids it is
 *          the k-set eigen-adjoint contracted back to R_e; off-grid (no kq
 *          map) it adds, for every (k, q) pair, the eigen-adjoint of the
 *          interpolated H(k+q) contracted back with the conjugate of the
 *          phase that formed it.
 *  domega  device [nq][nm] double out (NULL to skip)
 * Outputs are overwritten (par->accumulate = 1 adds instead).
 * par->dtype: EPW_FP64; EPW_FP32 (the contractions, rotations and the
 * per-pair adjoint in complex64); EPW_SPLIT_BF16 (the R_e <-> k
 * contractions on split-bf16 operands with float32 accumulation, the
 * R_p <-> q sums and the per-pair adjoint as in EPW_FP32).  In every
 * precision the eigen-adjoints, the dL/dH(R_e) contraction and all outputs
 * are float64.
 * Errors: as epw_imsigma. */
int epw_imsigma_backward(const epw_system* sys, const epw_points* pts, const epw_params* par,
                         const double* w, void* dgR, void* dHR, double* domega,
                         void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for the call `which` (EPW_WS_INTERP_G, EPW_WS_IMSIGMA,
 * EPW_WS_IMSIGMA_BACKWARD, EPW_WS_PHONON, EPW_WS_RESIGMA, EPW_WS_TRANSPORT,
 * EPW_WS_CHECK for epw_check_inputs) with these sizes and parameters; device pointers
 * inside sys/pts are not dereferenced and may be NULL.  Returns 0 and sets
 * the error message on invalid arguments. */
#define EPW_WS_INTERP_G          1
#define EPW_WS_IMSIGMA           2
#define EPW_WS_IMSIGMA_BACKWARD  3
#define EPW_WS_PHONON            4
#define EPW_WS_RESIGMA           5
#define EPW_WS_TRANSPORT         6
#define EPW_WS_CHECK             7
size_t epw_workspace_size(int which, const epw_system* sys, const epw_points* pts,
                          const epw_params* par);

/* Validation of a system and point set, meant to run once before the calls
 * above, which check sizes and scalar parameters only and take the arrays
 * as they are.  Synchronous: the check kernels run on `stream` and the call
 * waits for them.  The first failed check, in this order, is returned:
 *  1. every entry of H(R_e), D(R_p) (when given), g(R_e,R_p), the k and q
 *     points and given omega / evec is finite                 -> EPW_EINVAL
 *  2. ndeg >= 1 in both WS sets, and nmax_e (when set) >= every |component|
 *     of R_e (the in-kernel phase generation relies on it)    -> EPW_EINVAL
 *  3. both WS sets are closed under R -> -R (off-grid runs need it for R_e;
 *     epw_ws_vectors always returns such sets)                 -> EPW_ESHAPE
 *  4. max |H(-R) - H(R)^dag| <= herm_tol max |H| and
 *     max |D(-R) - D(R)^T| <= herm_tol max |D| over all R and entries: the
 *     interpolated H(k) and D(q) are then Hermitian before their
 *     symmetrisation (the Wannier Hamiltonian and force constants of a real
 *     crystal are; every call Hermitises the interpolated matrices, so a
 *     violation is a symptom of bad input, not a failure)    -> EPW_ENOTHERM
 *  5. the k+q map (when given): every entry in [0, nk), and for every q the
 *     map k -> kq[k][q] is one-to-one (as on a full grid)     -> EPW_EINVAL
 *  herm_tol  >= 0 (1e-12 suits float64 inputs built with the symmetry)
 *  ws        device workspace of epw_workspace_size(EPW_WS_CHECK, ...) bytes
 *            (the params of the size query are only checked for validity)
 * Errors: as listed, plus EPW_EINVAL (NULL, bad herm_tol), EPW_ESHAPE,
 * EPW_ENOMEM (workspace), EPW_EHIP. */
int epw_check_inputs(const epw_system* sys, const epw_points* pts, double herm_tol, void* ws, size_t ws_bytes,
                     void* stream);

/* ======================================================================
 * Stage timing (diagnostics)
 * ====================================================================== */

/* When enabled, every launch of the kernels of a stage is bracketed by a
 * pair of HIP events recorded on the launch's own stream.  The library's
 * only process-wide state; guarded by a mutex.  Stages: */
#define EPW_STAGE_EIGH      0   /* interpolation + eigensolve of H(k), D(q),
                                   phase tables of the off-grid pairs            */
#define EPW_STAGE_GEMM_RP   1   /* R_p -> q contraction                          */
#define EPW_STAGE_MODEROT   2   /* mode rotation and 1/sqrt(2 omega)             */
#define EPW_STAGE_FUSED     3   /* R_e -> k contraction + rotation + reduction   */
#define EPW_STAGE_BACKWARD  4   /* adjoint kernels                               */
#define EPW_STAGE_SPECTRAL  5   /* frequency-resolved sum over pole records      */
#define EPW_STAGE_PAIR_GEMM 6   /* off-grid: H(k+q) of every pair (phase GEMM)   */
#define EPW_STAGE_PAIR_EIGH 7   /* off-grid: eigensolve of every H(k+q)          */
#define EPW_STAGE_BWD_GEMM  8   /* adjoint: recomputed and transposed contractions
                                   (also counted in EPW_STAGE_BACKWARD)          */
#define EPW_NUM_STAGES      9

/* enable != 0 starts recording (and discards earlier records); 0 stops. */
int epw_timing_enable(int enable);

/* Waits for the recorded events of `stage`, returns the summed duration in
 * milliseconds and the number of launches, and discards those records.
 * Errors: EPW_EINVAL (bad stage or NULL), EPW_EHIP. */
int epw_timing_read(int stage, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* EPW_H */
