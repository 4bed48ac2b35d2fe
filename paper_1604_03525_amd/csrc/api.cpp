// C ABI entry points: argument checks, workspace layout and the order of
// kernel launches for each call.  All device work goes to the caller's
// stream; nothing here blocks on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "epw_internal.h"
#include "kernels.h"

namespace epw {
namespace {

constexpr int SLICE_CUS = 256;          // column-slice count is sized for 256 CUs
constexpr size_t AUTO_CHUNK_BYTES = (size_t)8 << 30;

// Automatic q chunk: as many q as the per-q scratch budget allows, then
// evened out over the chunks that takes, so no launch runs a small tail.
long auto_chunk(long nq, size_t budget, size_t per_q) {
    long Q = (long)(budget / (per_q > 0 ? per_q : 1));
    if (Q < 1) Q = 1;
    if (nq <= Q) return nq > 0 ? nq : 1;
    const long nchunks = (nq + Q - 1) / Q;
    return (nq + nchunks - 1) / nchunks;
}

size_t cbytes(Prec p) { return p == Prec::F64 ? 16 : 8; }

// Smallest eigenvalue of a symmetric 3 x 3 matrix (cyclic Jacobi).
double sym3_min_eig(const double (&m)[3][3]) {
    double a[3][3];
    std::memcpy(a, m, sizeof(a));
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = std::fabs(a[0][1]) + std::fabs(a[0][2]) + std::fabs(a[1][2]);
        if (off < 1e-300) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                const double th = 0.5 * std::atan2(2.0 * a[p][q], a[q][q] - a[p][p]);
                const double c = std::cos(th), sn = std::sin(th);
                for (int k = 0; k < 3; ++k) {           // A <- A J
                    const double x = a[k][p], y = a[k][q];
                    a[k][p] = c * x - sn * y;
                    a[k][q] = sn * x + c * y;
                }
                for (int k = 0; k < 3; ++k) {           // A <- J^T A
                    const double x = a[p][k], y = a[q][k];
                    a[p][k] = c * x - sn * y;
                    a[q][k] = sn * x + c * y;
                }
            }
    }
    return std::min(a[0][0], std::min(a[1][1], a[2][2]));
}

// Device copy of the polar data: reciprocal vectors, 1/sqrt(M) and the half-
// width of a G box holding every K = q + G (q reduced to [-1/2, 1/2)^3) with
// K.eps.K/(4 alpha) < cutoff.  Returns an error message or nullptr.
const char* polar_device(const epw_polar* pp, int nm, PolarDev& P) {
    if (pp->nat < 1 || pp->nat > EPW_MAX_ATOMS || 3 * pp->nat != nm) return "polar: nat must be nm / 3 (1..EPW_MAX_ATOMS)";
    if (!(pp->alpha > 0.0) || !(pp->cutoff > 0.0) || !std::isfinite(pp->alpha) || !std::isfinite(pp->cutoff))
        return "polar: alpha and cutoff must be > 0";
    if (!std::isfinite(pp->prefactor)) return "polar: prefactor not finite";
    const double(&A)[3][3] = pp->vectors;
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                       A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (!(std::fabs(det) > 1e-300) || !std::isfinite(det)) return "polar: singular lattice vectors";
    // B = 2 pi (A^-1)^T: row i of B is 2 pi times column i of A^-1
    double inv[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            inv[j][i] = (A[i1][j1] * A[i2][j2] - A[i1][j2] * A[i2][j1]) / det;   // cofactor transpose
        }
    P.nat = pp->nat;
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) P.B[i][a] = 2.0 * M_PI * inv[a][i];
    double mx = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            if (!std::isfinite(pp->eps_inf[a][b])) return "polar: eps_inf not finite";
            mx = std::max(mx, std::fabs(pp->eps_inf[a][b]));
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (std::fabs(pp->eps_inf[a][b] - pp->eps_inf[b][a]) > 1e-12 * mx) return "polar: eps_inf not symmetric";
    const double lmin = sym3_min_eig(pp->eps_inf);
    if (!(lmin > 0.0)) return "polar: eps_inf not positive definite";
    std::memcpy(P.eps, pp->eps_inf, sizeof(P.eps));
    for (int k = 0; k < pp->nat; ++k) {
        if (!(pp->mass[k] > 0.0) || !std::isfinite(pp->mass[k])) return "polar: masses must be > 0";
        P.rsm[k] = 1.0 / std::sqrt(pp->mass[k]);
        for (int a = 0; a < 3; ++a) {
            P.tau[k][a] = pp->tau[k][a];
            for (int b = 0; b < 3; ++b) P.zstar[k][a][b] = pp->zstar[k][a][b];
        }
    }
    P.prefactor = pp->prefactor;
    P.alpha = pp->alpha;
    P.cutoff = pp->cutoff;
    const double kmax = std::sqrt(4.0 * pp->alpha * pp->cutoff / lmin);
    double qmax = 0.0, amax = 0.0;
    for (int i = 0; i < 3; ++i) {
        for (int a = 0; a < 3; ++a) qmax += 0.5 * std::fabs(P.B[i][a]);
        amax = std::max(amax, std::sqrt(A[i][0] * A[i][0] + A[i][1] * A[i][1] + A[i][2] * A[i][2]));
    }
    const double g = std::ceil(amax * (kmax + qmax) / (2.0 * M_PI)) + 1.0;
    if (!(g <= EPW_MAX_GMAX)) return "polar: the G box for this cutoff exceeds EPW_MAX_GMAX";
    P.gmax = (int)g;
    return nullptr;
}

int check_common(const epw_system* s, const epw_points* p, const epw_params* par, const char* fn) {
    if (!s || !p || !par) return fail(EPW_EINVAL, "%s: NULL argument", fn);
    if (s->nb < 1 || s->nb > EPW_MAX_NB) return fail(EPW_ESHAPE, "%s: nb = %d not in 1..%d", fn, s->nb, EPW_MAX_NB);
    if (s->nm < 1 || s->nm > EPW_MAX_NM) return fail(EPW_ESHAPE, "%s: nm = %d not in 1..%d", fn, s->nm, EPW_MAX_NM);
    if (s->nRe < 1 || s->nRp < 1) return fail(EPW_ESHAPE, "%s: empty WS set", fn);
    if (s->nRe > (1 << 20) || s->nRp > (1 << 20)) return fail(EPW_ESHAPE, "%s: WS set too large", fn);
    if (p->nk < 0 || p->nq < 0) return fail(EPW_ESHAPE, "%s: negative point count", fn);
    if (par->dtype != EPW_FP64 && par->dtype != EPW_FP32 && par->dtype != EPW_SPLIT_BF16)
        return fail(EPW_EDTYPE, "%s: unknown dtype %d", fn, par->dtype);
    if (!(par->sigma > 0.0) || !std::isfinite(par->sigma)) return fail(EPW_EINVAL, "%s: sigma must be > 0", fn);
    if (!(par->T >= 0.0) || !std::isfinite(par->T)) return fail(EPW_EINVAL, "%s: T must be >= 0", fn);
    if (!std::isfinite(par->mu)) return fail(EPW_EINVAL, "%s: mu not finite", fn);
    if (!(par->deg_tol >= 0.0)) return fail(EPW_EINVAL, "%s: deg_tol must be >= 0", fn);
    if (!(par->nq_norm >= 0.0)) return fail(EPW_EINVAL, "%s: nq_norm must be >= 0", fn);
    if (!std::isfinite(par->omega_cut)) return fail(EPW_EINVAL, "%s: omega_cut not finite", fn);
    if (par->chunk_q < 0) return fail(EPW_EINVAL, "%s: chunk_q < 0", fn);
    if (par->order < EPW_ORDER_AUTO || par->order > EPW_ORDER_K_OUTER)
        return fail(EPW_EINVAL, "%s: unknown contraction order %d", fn, par->order);
    if (s->nmax_e < 0 || s->nmax_e > EPW_MAX_NMAX)
        return fail(EPW_EINVAL, "%s: nmax_e = %d not in 0..%d", fn, s->nmax_e, EPW_MAX_NMAX);
    if (s->polar) {
        PolarDev P;
        const char* msg = polar_device(s->polar, s->nm, P);
        if (msg) return fail(EPW_EINVAL, "%s: %s", fn, msg);
    }
    const bool given = p->omega && p->evec;
    if ((p->omega != nullptr) != (p->evec != nullptr))
        return fail(EPW_EINVAL, "%s: omega and evec must be given together", fn);
    if (p->nk > 0 && p->nq > 0) {
        if (!s->Re || !s->ndeg_e || !s->Rp || !s->ndeg_p || !s->HR || !s->gR)
            return fail(EPW_EINVAL, "%s: NULL pointer in epw_system", fn);
        if (!given && !s->DR) return fail(EPW_EINVAL, "%s: DR is NULL and no phonon states given", fn);
        if (!p->kfrac || !p->qfrac) return fail(EPW_EINVAL, "%s: NULL point array", fn);
    }
    return EPW_OK;
}

// Off-grid k+q: H(k+q) of every (k, q) pair of a chunk is formed as an FP64
// GEMM over R_e whose A operand is the product of the k and q phase tables
// (e^{2 pi i (k+q).R} = e^{2 pi i k.R} e^{2 pi i q.R}), in batches of pairs,
// then diagonalised.  Scratch: both phase tables and one batch of matrices.
constexpr long PAIR_BATCH = 65536;

struct PairScratch {
    void* phi_k = nullptr;   // [N_k][N_e] c128, 1/ndeg_e included
    void* phi_q = nullptr;   // [Q][N_e] c128
    void* H = nullptr;       // [batch][n_b (n_b + 1) / 2] c128: upper triangles of H(k+q)
    void* HRu = nullptr;     // [N_e][n_b (n_b + 1) / 2] c128: upper triangles of the Hermitian part of H(R_e)
    int32_t* negR = nullptr; // [N_e] index of -R_e
    // the H(k+q) product folded by the pairs (R, -R): halved R list, its phase
    // tables without weights, and the B+ / B- rows of HRu (1/ndeg_e included)
    int32_t* fneg = nullptr;
    int32_t* fhalf = nullptr;
    int32_t* fpair = nullptr;
    int32_t* fR = nullptr;
    int32_t* fkh = nullptr;
    void* fphi_k = nullptr;  // [N_k][N_e] c128 (rows of the halved list)
    void* fphi_q = nullptr;  // [Q][N_e] c128
    void* HRp = nullptr;     // [N_e][n_b (n_b + 1) / 2] c128
    void* HRm = nullptr;
    long batch = 0;
    // band velocities at k+q (transport mode): i R_a H(R) for a = x, y, z,
    // their Fourier sums for one batch, and the velocities of every pair
    void* dHR3 = nullptr;    // [3][N_e][n_b][n_b] c128
    void* dH3 = nullptr;     // [3][batch][n_b][n_b] c128
    double* vel_pair = nullptr;  // [N_k][Q][n_b][3]
    const double* vectors9 = nullptr;
};

// what a forward pass produces
enum class Out { IMSIGMA, STORE, PHONON, RESIGMA, OMEGA, TRANSPORT };

struct Layout {
    Prec prec;
    Out out;
    int nbp, Q, nchunks, S, kpad, tiles_m;
    // fixed tables
    double* eps = nullptr;
    void* U = nullptr;
    double* ftab = nullptr;
    void* phi_k = nullptr;
    void* gR_t = nullptr;
    // per chunk
    double* omega_c = nullptr;
    void* evec_c = nullptr;
    double* sc = nullptr;
    double* nbose = nullptr;
    void* phi_q = nullptr;
    void* gq = nullptr;
    void* Bnu = nullptr;
    double* part = nullptr;
    double* part2 = nullptr;     // [S][nk][nb] (real-part mode: Sigma' at eps_F)
    double* part_ph = nullptr;   // [2][tiles_m][Q nm] (phonon mode)
    double* dos_raw = nullptr;   // [1] (phonon mode)
    int nw = 0;                  // frequency-grid mode: grid size,
    double* rec = nullptr;       // [nk][Q][nm][nb] pole records of 4 + nbp doubles (+ 2),
    void* spart = nullptr;       // [S_w][nk][nb][nw + 1] c128 slice partials
    int Sw = 1;
    void* polar_L = nullptr;     // [Q][nm] c128 long-range factors (polar systems)
    double* vel = nullptr;       // [nk][nb][3] band velocities (transport mode)
    // folded R_e -> k contraction (float64 / float32): -R index, halved R
    // list, partner rows, its R vectors and length
    bool fold = false;
    int32_t* fneg = nullptr;
    int32_t* fhalf = nullptr;
    int32_t* fpair = nullptr;
    int32_t* fR = nullptr;
    int32_t* fkh = nullptr;
    // k-outer order (frequency-grid mode): R_e -> k once, R_p -> q per chunk
    bool kouter = false;
    void* phi_e = nullptr;       // [nk][N_e] phases with 1/ndeg_e
    void* Gk = nullptr;          // [N_p][nk][nm nb nb] g(k, R_p)
    void* Cq = nullptr;          // [nk][Q][nm nb nb] g(k, q), Wannier basis
    // per pair states at k+q when no k+q map is given
    double* eps_pair = nullptr;
    void* U_pair = nullptr;
    double* f_pair = nullptr;
    PairScratch ps;
};

// bytes per q point of the per-pair k+q states (off-grid runs)
size_t pair_bytes_per_q(const epw_system* s, const epw_points* p) {
    if (p->kq) return 0;
    return (size_t)p->nk * (16 * (size_t)s->nb + 16 * (size_t)s->nb * s->nb) + 32 * (size_t)s->nRe;
}

// extra bytes per q point of the k+q velocities (off-grid transport runs)
size_t pair_vel_bytes_per_q(const epw_system* s, const epw_points* p) {
    return p->kq ? 0 : (size_t)p->nk * 24 * (size_t)s->nb;
}

void take_pair_states(const epw_system* s, const epw_points* p, int Q, Arena& A, double*& eps_pair, void*& U_pair,
                      double*& f_pair, PairScratch& ps, bool velocities = false) {
    if (p->kq) return;
    const size_t n = (size_t)p->nk * Q;
    const size_t nbb = (size_t)s->nb * s->nb;
    eps_pair = (double*)A.take(8 * n * s->nb);
    U_pair = A.take(16 * n * nbb);
    f_pair = (double*)A.take(8 * n * s->nb);
    ps.phi_k = A.take(16 * (size_t)p->nk * s->nRe);
    ps.phi_q = A.take(16 * (size_t)Q * s->nRe);
    ps.batch = std::min<long>(PAIR_BATCH, (long)n);
    ps.H = A.take(16 * (size_t)ps.batch * nbb);
    ps.HRu = A.take(16 * (size_t)s->nRe * (s->nb * (s->nb + 1) / 2));
    ps.negR = (int32_t*)A.take(4 * (size_t)s->nRe);
    ps.fneg = (int32_t*)A.take(4 * (size_t)s->nRe);
    ps.fhalf = (int32_t*)A.take(4 * (size_t)s->nRe);
    ps.fpair = (int32_t*)A.take(4 * (size_t)s->nRe);
    ps.fR = (int32_t*)A.take(12 * (size_t)s->nRe);
    ps.fkh = (int32_t*)A.take(4);
    ps.fphi_k = A.take(16 * (size_t)p->nk * s->nRe);
    ps.fphi_q = A.take(16 * (size_t)Q * s->nRe);
    ps.HRp = A.take(16 * (size_t)s->nRe * (s->nb * (s->nb + 1) / 2));
    ps.HRm = A.take(16 * (size_t)s->nRe * (s->nb * (s->nb + 1) / 2));
    if (velocities) {
        ps.dHR3 = A.take(16 * 3 * (size_t)s->nRe * nbb);
        ps.dH3 = A.take(16 * 3 * (size_t)ps.batch * nbb);
        ps.vel_pair = (double*)A.take(8 * 3 * n * s->nb);
    }
}

// eps, U and f at k+q for every (k, q) of a chunk (off-grid runs); pair
// index k*qc + q.  The k phase table is built with the first chunk.
void pair_states(const epw_system* s, const epw_points* p, const epw_params* par, int q0, int qc, double* eps_pair,
                 void* U_pair, double* f_pair, const PairScratch& ps, hipStream_t st) {
    if (p->kq) return;
    const int nb = s->nb, ne = s->nRe, nbb = nb * nb;
    // H(k+q) is Hermitian: only its upper triangle is formed, from the upper
    // triangles of the Hermitian part of H(R_e) (exact for any H(R_e)), summed
    // over the pairs (R, -R) of R_e: sum_h c (B(R) + B(-R)) + i s (B(R) - B(-R))
    // with c + i s = exp(2 pi i (k+q).R) and B(R) = HRu(R) / ndeg(R)
    const int ntri = nb * (nb + 1) / 2;
    {
        StageTimer t(EPW_STAGE_EIGH, st);
        if (q0 == 0) {
            launch_phase_table(Prec::F64, p->nk, p->kfrac, ne, s->Re, s->ndeg_e, ne, ps.phi_k, st);
            launch_pack_upper(nb, ne, s->Re, s->ndeg_e, s->HR, ps.negR, ps.HRu, st);
            launch_half_list(ne, s->Re, ps.fneg, ps.fhalf, ps.fpair, ps.fR, ps.fkh, st);
            launch_phase_table(Prec::F64, p->nk, p->kfrac, ne, ps.fR, nullptr, ne, ps.fphi_k, st);
            launch_fold_gather(ne, ps.fkh, ps.fhalf, ps.fpair, s->ndeg_e, ntri, ps.HRu, ps.HRp, ps.HRm, st);
        }
        if (q0 == 0 && ps.dHR3) launch_velocity_operands(nb, ne, s->Re, s->HR, ps.vectors9, ps.dHR3, st);
        launch_phase_table(Prec::F64, qc, p->qfrac + 3 * (size_t)q0, ne, s->Re, nullptr, ne, ps.phi_q, st);
        launch_phase_table(Prec::F64, qc, p->qfrac + 3 * (size_t)q0, ne, ps.fR, nullptr, ne, ps.fphi_q, st);
    }
    const long npair = (long)p->nk * qc;
    for (long b0 = 0; b0 < npair; b0 += ps.batch) {
        const int nbt = (int)std::min(ps.batch, npair - b0);
        GemmDesc d;   // H(k+q)[pair][i <= j] = sum_R Phi_k[k][R] Phi_q[q][R] H(R)[i <= j]
        d.M = nbt;
        d.N = ntri;
        d.K = ne;
        d.A = ps.phi_k;
        d.lda = ne;
        d.A2 = ps.phi_q;
        d.n2 = qc;
        d.row0 = b0;
        d.B = ps.HRu;
        d.ncb = ntri;
        d.sBk = ntri;
        d.C = ps.H;
        d.sCm = ntri;
        {
            StageTimer t(EPW_STAGE_PAIR_GEMM, st);
            GemmDesc df = d;   // the same sum folded by the pairs (R, -R)
            df.A = ps.fphi_k;
            df.A2 = ps.fphi_q;
            df.B = ps.HRp;
            df.B2 = ps.HRm;
            df.kh = ps.fkh;
            launch_cgemm(Prec::F64, df, st);
        }
        {
            StageTimer t(EPW_STAGE_PAIR_EIGH, st);
            launch_eigh_given(nb, nbt, ps.H, eps_pair + (size_t)b0 * nb, (char*)U_pair + 16 * (size_t)b0 * nbb, st,
                              true);
        }
        if (ps.vel_pair) {
            StageTimer t(EPW_STAGE_PAIR_GEMM, st);
            // dH/dk_a(k+q) = sum_R Phi_k Phi_q (i R_a H(R)), then the band velocities (full matrices)
            for (int a = 0; a < 3; ++a) {
                GemmDesc dv = d;
                dv.N = nbb;
                dv.ncb = nbb;
                dv.sBk = nbb;
                dv.sCm = nbb;
                dv.B = (const char*)ps.dHR3 + 16 * (size_t)a * ne * nbb;
                dv.C = (char*)ps.dH3 + 16 * (size_t)a * ps.batch * nbb;
                launch_cgemm(Prec::F64, dv, st);
            }
            launch_pair_velocities(nb, nbt, ps.batch, ps.dH3, (const char*)U_pair + 16 * (size_t)b0 * nbb,
                                   eps_pair + (size_t)b0 * nb, par->deg_tol, ps.vel_pair + 3 * (size_t)b0 * nb, st);
        }
    }
    launch_fermi_table((size_t)p->nk * qc * nb, eps_pair, par->mu, par->T, f_pair, st);
}

int tiles_n_for(int qc, int nm, int nbp, Prec prec) {
    const long ncols = (long)qc * nm * nbp * nbp;
    const int BN = fused_tile_cols(nbp, prec);
    return (int)((ncols + BN - 1) / BN);
}

// Carve the workspace (or count its size when A.dry).
void plan(const epw_system* s, const epw_points* p, const epw_params* par, Out out, Arena& A, Layout& L,
          int nw = 0) {
    const bool store = out == Out::STORE;
    const bool omg = out == Out::OMEGA;
    L.out = out;
    L.prec = (Prec)par->dtype;
    L.nbp = pow2_at_least(s->nb);
    const size_t cb = cbytes(L.prec);
    const int nk = p->nk, nq = p->nq, nb = s->nb, nm = s->nm, ne = s->nRe, np_ = s->nRp;
    const bool given = p->omega && p->evec;
    const bool bf = L.prec == Prec::BF16X2;
    L.kpad = (ne + 31) / 32 * 32;
    const size_t bcol_bytes = bf ? 8 * (size_t)L.kpad : cb * (size_t)ne;   // B bytes per column
    const size_t X = (size_t)nm * nb * nb;
    L.kouter = omg && (par->order == EPW_ORDER_K_OUTER || (par->order == EPW_ORDER_AUTO && 4L * nk <= ne));
    // chunk size
    const size_t per_q = cb * np_ + (given ? 0 : 8 * (size_t)nm + 16 * (size_t)nm * nm) + 16 * (size_t)nm +
                         pair_bytes_per_q(s, p) + (omg ? 8 * (size_t)nk * nm * nb * (4 + L.nbp) : 0) +
                         (out == Out::TRANSPORT ? pair_vel_bytes_per_q(s, p) : 0) +
                         (L.kouter ? cb * (size_t)nk * X : cb * (size_t)ne * X + bcol_bytes * nm * L.nbp * L.nbp);
    long Q = par->chunk_q > 0 ? par->chunk_q : auto_chunk(nq, AUTO_CHUNK_BYTES, per_q);
    if (Q < 1) Q = 1;
    if (Q > nq) Q = nq > 0 ? nq : 1;
    L.Q = (int)Q;
    L.nchunks = nq > 0 ? (int)((nq + Q - 1) / Q) : 0;
    L.S = (store || omg) ? 0 : fused_slices(nk, L.nbp, tiles_n_for(L.Q, nm, L.nbp, L.prec), SLICE_CUS, L.prec);
    L.eps = (double*)A.take(8 * (size_t)nk * nb);
    L.U = A.take(16 * (size_t)nk * nb * nb);
    L.ftab = (double*)A.take(8 * (size_t)nk * nb);
    if (!L.kouter) L.phi_k = A.take(bf ? 8 * (size_t)nk * L.kpad : cb * (size_t)nk * ne);
    L.fold = !L.kouter && fused_fold_c(L.nbp, (int)L.prec);
    if (L.fold) {
        L.fneg = (int32_t*)A.take(4 * (size_t)ne);
        L.fhalf = (int32_t*)A.take(4 * (size_t)ne);
        L.fpair = (int32_t*)A.take(4 * (size_t)ne);
        L.fR = (int32_t*)A.take(12 * (size_t)ne);
        L.fkh = (int32_t*)A.take(4);
    }
    if (L.prec != Prec::F64) L.gR_t = A.take(cb * (size_t)ne * np_ * nm * nb * nb);
    if (!given) {
        L.omega_c = (double*)A.take(8 * (size_t)L.Q * nm);
        L.evec_c = A.take(16 * (size_t)L.Q * nm * nm);
    }
    L.sc = (double*)A.take(8 * (size_t)L.Q * nm);
    L.nbose = (double*)A.take(8 * (size_t)L.Q * nm);
    L.phi_q = A.take(cb * (size_t)L.Q * np_);
    if (L.kouter) {
        L.phi_e = A.take(cb * (size_t)nk * ne);
        L.Gk = A.take(cb * (size_t)np_ * nk * X);
        L.Cq = A.take(cb * (size_t)nk * L.Q * X);
    } else {
        L.gq = A.take(cb * (size_t)ne * L.Q * X);
        L.Bnu = A.take(bcol_bytes * L.Q * nm * L.nbp * L.nbp);
    }
    if (s->polar) L.polar_L = A.take(16 * (size_t)L.Q * nm);
    L.tiles_m = (nk + fused_tile_rows(L.nbp, L.prec) - 1) / fused_tile_rows(L.nbp, L.prec);
    // two slots per slice: the slice's own and its tail's (helper blocks)
    if (out == Out::IMSIGMA || out == Out::RESIGMA) L.part = (double*)A.take(16 * (size_t)L.S * nk * nb);
    if (out == Out::RESIGMA) L.part2 = (double*)A.take(16 * (size_t)L.S * nk * nb);
    if (omg) {
        L.nw = nw;
        // two records of padding: the frequency kernel reads two records ahead
        L.rec = (double*)A.take(8 * ((size_t)nk * L.Q * nm * nb + 2) * (4 + L.nbp));
        // slice count of the largest chunk bounds every chunk's
        int smax = 1;
        for (int qc : {L.Q, nq % L.Q}) {
            if (qc <= 0) continue;
            const int sw = sigma_omega_slices(nk, nw, (long)qc * nm * nb);
            if (sw > smax) smax = sw;
        }
        L.Sw = smax;
        L.spart = A.take(16 * (size_t)smax * nk * nb * ((size_t)nw + 1));
    }
    if (out == Out::PHONON || out == Out::TRANSPORT) {
        const int kinds = out == Out::TRANSPORT ? 3 : 2;
        L.part_ph = (double*)A.take(8 * kinds * (size_t)L.tiles_m * L.Q * nm);
        L.dos_raw = (double*)A.take(8);
    }
    if (out == Out::TRANSPORT) L.vel = (double*)A.take(8 * 3 * (size_t)nk * nb);
    take_pair_states(s, p, L.Q, A, L.eps_pair, L.U_pair, L.f_pair, L.ps, out == Out::TRANSPORT);
}

// a5 as a strided GEMM: out[e][q][c] = sum_p phi_q[q][p] gR[e][p][c]
GemmDesc rp_desc(int qc, int ne, int np_, int ncol, const void* phi_q, const void* gR, void* out) {
    GemmDesc d;
    d.M = qc;
    d.N = ne * ncol;
    d.K = np_;
    d.A = phi_q;
    d.lda = np_;
    d.B = gR;
    d.ncb = ncol;
    d.sBe = (long)np_ * ncol;
    d.sBk = ncol;
    d.C = out;
    d.sCe = (long)qc * ncol;
    d.sCm = ncol;
    return d;
}

// Shared forward pipeline: store mode writes g_mn,nu(k,q) to gkq, phonon
// mode writes Pi''_q,nu and lambda_q,nu to pi_im / lam, otherwise Im Sigma
// goes to imsig.
// What a forward call writes (unused members stay NULL).
struct Outputs {
    double* imsig = nullptr;            // Im Sigma, or Sigma' on shell (real-part mode)
    void* gkq = nullptr;                // g_mn,nu(k,q) (store mode)
    double* pi_im = nullptr;            // Pi'' (phonon and transport modes)
    double* lam = nullptr;              // lambda
    double* re_tilde = nullptr;         // Sigma~' (real-part mode)
    const double* wgrid = nullptr;      // frequencies (frequency-grid mode)
    void* sig_w = nullptr;              // Sigma(omega)
    void* sig0 = nullptr;               // Sigma(0)
    double* lam_tr = nullptr;           // lambda_tr (transport mode)
    const double* vectors9 = nullptr;   // lattice vectors (transport mode)
};

void run_forward(const epw_system* s, const epw_points* p, const epw_params* par, Layout& L, const Outputs& o,
                 hipStream_t st) {
    double* imsig = o.imsig;
    void* gkq = o.gkq;
    double* pi_im = o.pi_im;
    double* lam = o.lam;
    double* re_tilde = o.re_tilde;
    const double* wgrid = o.wgrid;
    void* sig_w = o.sig_w;
    void* sig0 = o.sig0;
    double* lam_tr = o.lam_tr;
    const double* vectors9 = o.vectors9;
    const bool trans = L.out == Out::TRANSPORT;
    const bool phon = L.out == Out::PHONON || trans;
    const bool omg = L.out == Out::OMEGA;
    const bool re = L.out == Out::RESIGMA;     // imsig then receives Sigma' on shell
    const int nk = p->nk, nq = p->nq, nb = s->nb, nm = s->nm, ne = s->nRe, np_ = s->nRp;
    const Prec prec = L.prec;
    const bool given = p->omega && p->evec;
    // electrons on the k set (the k+q states are members of the k set)
    {
        StageTimer t(EPW_STAGE_EIGH, st);
        launch_interp_eigh(false, false, nb, ne, s->Re, s->ndeg_e, (const double*)s->HR, nk, p->kfrac,
                           L.eps, L.U, st);
    }
    launch_fermi_table((size_t)nk * nb, L.eps, par->mu, par->T, L.ftab, st);
    if (phon) launch_dos_raw((size_t)nk * nb, L.eps, par->mu, par->sigma, L.dos_raw, st);
    if (trans) {
        launch_velocities(nb, ne, s->Re, s->ndeg_e, s->HR, vectors9, nk, p->kfrac, L.eps, L.U, par->deg_tol, L.vel,
                          st);
        L.ps.vectors9 = vectors9;
    }
    const bool bf = prec == Prec::BF16X2;
    const Prec rprec = bf ? Prec::F32 : prec;      // precision of the R_p -> q step
    // Phases of the R_e -> k contraction: generated inside the fused kernel
    // from per-axis factors for the split-BF16 path up to 8 padded bands (its
    // short main loop would otherwise wait on the table; realistic workload
    // 248 -> 219 ms per 4000-q launch), read from a table for FP64 and FP32,
    // where the extra VALU work of generating them costs more than the table
    // reads (FP32: 322 -> 291 ms per launch with the table), and for
    // split-BF16 at 16 padded bands, whose 32-row tiles amortise the
    // generation over few rows (mobility-shaped shard: 129 -> 121 ms per
    // launch with the table).  Generation needs the R_e offsets of a tile in
    // LDS, hence the bound on ne.  The 1/ndeg weights of R_e are folded into
    // the B operand (mode rotation) in both cases.
    // FP32 up to 8 padded bands folds the sum over R_e by pairs (R, -R)
    // (cfold_mainloop): its table holds the phases of the halved list.
    const bool gen = prec == Prec::BF16X2 && L.nbp < 16 && s->nmax_e > 0 && ne <= 4096;
    if (L.fold) {
        launch_half_list(ne, s->Re, L.fneg, L.fhalf, L.fpair, L.fR, L.fkh, st);
        launch_phase_table(prec, nk, p->kfrac, ne, L.fR, nullptr, ne, L.phi_k, st);
    } else if (!gen && !L.kouter) {
        launch_phase_table(prec, nk, p->kfrac, ne, s->Re, nullptr, bf ? L.kpad : ne, L.phi_k, st);
    }
    const void* gsrc = s->gR;
    if (prec != Prec::F64) {
        launch_c128_to_c64((size_t)ne * np_ * nm * nb * nb, s->gR, L.gR_t, st);
        gsrc = L.gR_t;
    }
    const int X = nm * nb * nb;
    if (L.kouter) {
        // k-outer: g(k, R_p)[p][k][x] = sum_e Phi_k[k][e] g(R_e, R_p)[e][p][x], once for all chunks
        StageTimer t(EPW_STAGE_GEMM_RP, st);
        const Prec kp = prec == Prec::BF16X2 ? Prec::F32 : prec;
        launch_phase_table(kp, nk, p->kfrac, ne, s->Re, s->ndeg_e, ne, L.phi_e, st);
        GemmDesc d;
        d.M = nk;
        d.N = np_ * X;
        d.K = ne;
        d.A = L.phi_e;
        d.lda = ne;
        d.B = gsrc;
        d.ncb = X;
        d.sBe = X;
        d.sBk = (long)np_ * X;
        d.C = L.Gk;
        d.sCe = (long)nk * X;
        d.sCm = X;
        launch_cgemm(kp, d, st);
    }
    const double nqn = par->nq_norm > 0.0 ? par->nq_norm : (double)nq;
    const double scale = M_PI / (nqn * par->sigma * std::sqrt(M_PI));
    for (int c = 0; c < L.nchunks; ++c) {
        const int q0 = c * L.Q;
        const int qc = (q0 + L.Q <= nq) ? L.Q : nq - q0;
        const double* om;
        const void* ev;
        if (given) {
            om = p->omega + (size_t)q0 * nm;
            ev = (const char*)p->evec + 16 * (size_t)q0 * nm * nm;
        } else {
            StageTimer t(EPW_STAGE_EIGH, st);
            launch_interp_eigh(true, true, nm, np_, s->Rp, s->ndeg_p, s->DR, qc, p->qfrac + 3 * (size_t)q0,
                               L.omega_c, L.evec_c, st);
            om = L.omega_c;
            ev = L.evec_c;
        }
        launch_phonon_factors(qc, nm, om, par->omega_cut, par->T, L.sc, L.nbose, st);
        if (s->polar) {
            StageTimer t(EPW_STAGE_MODEROT, st);
            PolarDev P;
            polar_device(s->polar, nm, P);          // validated by check_common
            launch_polar_factor(P, qc, nm, p->qfrac + 3 * (size_t)q0, ev, L.sc, L.polar_L, st);
        }
        pair_states(s, p, par, q0, qc, L.eps_pair, L.U_pair, L.f_pair, L.ps, st);
        launch_phase_table(rprec, qc, p->qfrac + 3 * (size_t)q0, np_, s->Rp, s->ndeg_p, np_, L.phi_q, st);
        if (L.kouter) {
            {
                // g(k, q)[k][q][x] = sum_p Phi_q[q][p] g(k, R_p)[p][k][x]
                StageTimer t(EPW_STAGE_GEMM_RP, st);
                GemmDesc d;
                d.M = qc;
                d.N = nk * X;
                d.K = np_;
                d.A = L.phi_q;
                d.lda = np_;
                d.B = L.Gk;
                d.ncb = X;
                d.sBe = X;
                d.sBk = (long)nk * X;
                d.C = L.Cq;
                d.sCe = (long)qc * X;
                d.sCm = X;
                launch_cgemm(rprec, d, st);
            }
            {
                StageTimer t(EPW_STAGE_FUSED, st);
                PairPoleArgs pa;
                pa.nk = nk;
                pa.nb = nb;
                pa.nbp = L.nbp;
                pa.nm = nm;
                pa.qc = qc;
                pa.q0 = q0;
                pa.nq_total = nq;
                pa.C = L.Cq;
                pa.c64 = rprec == Prec::F64 ? 0 : 1;
                pa.U = L.U;
                pa.kq = p->kq;
                pa.eps = L.eps;
                pa.ftab = L.ftab;
                pa.eps_pair = L.eps_pair;
                pa.f_pair = L.f_pair;
                pa.U_pair = L.U_pair;
                pa.omega = om;
                pa.nbose = L.nbose;
                pa.sc = L.sc;
                pa.evec = ev;
                pa.Lq = L.polar_L;
                pa.mu = par->mu;
                pa.rec = L.rec;
                launch_pair_pole(pa, st);
            }
            const long npole = (long)qc * nm * nb;
            const int sw = sigma_omega_slices(nk, L.nw, npole);
            {
                StageTimer t(EPW_STAGE_SPECTRAL, st);
                launch_sigma_omega(nk, nb, npole, L.nw, wgrid, par->sigma, L.rec, sw, L.spart, st);
            }
            launch_sigma_omega_reduce(nk, nb, L.nw, sw, L.spart, L.eps, par->deg_tol, 1.0 / nqn,
                                      (c > 0 || par->accumulate) ? 1 : 0, sig_w, sig0, st);
            continue;
        }
        {
            StageTimer t(EPW_STAGE_GEMM_RP, st);
            launch_cgemm(rprec, rp_desc(qc, ne, np_, nm * nb * nb, L.phi_q, gsrc, L.gq), st);
        }
        {
            StageTimer t(EPW_STAGE_MODEROT, st);
            if (bf)
                launch_mode_rotate_bf16(ne, qc, nm, nb, L.nbp, L.kpad, L.gq, ev, L.sc, L.Bnu, st, s->ndeg_e,
                                        L.polar_L, s->Re);
            else if (L.fold)
                launch_mode_rotate_fold(prec, ne, qc, nm, nb, L.nbp, L.gq, ev, L.sc, s->ndeg_e, L.fkh, L.fhalf,
                                        L.fpair, L.polar_L, s->Re, L.Bnu, st);
            else
                launch_mode_rotate(prec, ne, qc, nm, nb, L.nbp, L.gq, ev, L.sc, L.Bnu, st, s->ndeg_e, L.polar_L,
                                   s->Re);
        }
        FusedArgs a;
        a.nk = nk;
        a.ne = ne;
        a.nb = nb;
        a.nbp = L.nbp;
        a.nm = nm;
        a.qc = qc;
        a.q0 = q0;
        a.nq_total = nq;
        a.phi_k = L.phi_k;
        a.ldk = bf ? L.kpad : ne;
        a.nmax = gen ? s->nmax_e : 0;
        a.Re = s->Re;
        a.ndeg_e = s->ndeg_e;
        a.kfrac = p->kfrac;
        a.ldk_b = L.kpad;
        a.kpad = L.kpad;
        a.B = L.Bnu;
        a.eps = L.eps;
        a.U = L.U;
        a.ftab = L.ftab;
        a.kq = p->kq;
        a.eps_pair = L.eps_pair;
        a.U_pair = L.U_pair;
        a.f_pair = L.f_pair;
        a.omega = om;
        a.nbose = L.nbose;
        a.sc = L.sc;
        a.sigma = par->sigma;
        a.mu = par->mu;
        a.part = L.part;
        a.half = L.fold ? L.fhalf : nullptr;
        a.pair = L.fold ? L.fpair : nullptr;
        a.kh = L.fold ? L.fkh : nullptr;
        // (pole mode: the slices only spread the column tiles over blocks)
        a.S = gkq ? 1 : fused_slices(nk, L.nbp, tiles_n_for(qc, nm, L.nbp, prec), SLICE_CUS, prec);
        fused_balance(a, prec, SLICE_CUS);
        a.gkq = gkq;
        a.part_ph = phon ? L.part_ph : nullptr;
        a.vel = trans ? L.vel : nullptr;
        a.vel_pair = trans ? L.ps.vel_pair : nullptr;
        a.part2 = re ? L.part2 : nullptr;
        a.rec = omg ? L.rec : nullptr;
        {
            StageTimer t(EPW_STAGE_FUSED, st);
            launch_fused_k(prec, a, SLICE_CUS, st);
        }
        if (omg) {
            const long npole = (long)qc * nm * nb;
            const int sw = sigma_omega_slices(nk, L.nw, npole);
            {
                StageTimer t(EPW_STAGE_SPECTRAL, st);
                launch_sigma_omega(nk, nb, npole, L.nw, wgrid, par->sigma, L.rec, sw, L.spart, st);
            }
            launch_sigma_omega_reduce(nk, nb, L.nw, sw, L.spart, L.eps, par->deg_tol, 1.0 / nqn,
                                      (c > 0 || par->accumulate) ? 1 : 0, sig_w, sig0, st);
        } else if (phon) {
            double* pi_c = pi_im ? pi_im + (size_t)q0 * nm : nullptr;
            double* lam_c = lam ? lam + (size_t)q0 * nm : nullptr;
            double* ltr_c = (trans && lam_tr) ? lam_tr + (size_t)q0 * nm : nullptr;
            launch_phonon_finalize(qc, nm, L.tiles_m, L.part_ph, om, par->omega_cut, L.dos_raw, nk, par->sigma,
                                   pi_c, lam_c, st, ltr_c);
            // average over degenerate modes of each q
            if (pi_c) launch_degenerate_average(qc, nm, om, par->deg_tol, pi_c, st);
            if (lam_c) launch_degenerate_average(qc, nm, om, par->deg_tol, lam_c, st);
            if (ltr_c) launch_degenerate_average(qc, nm, om, par->deg_tol, ltr_c, st);
        } else if (re) {
            // Eq. (3) carries no pi: the BZ mean only
            const int acc = (c > 0 || par->accumulate) ? 1 : 0;
            launch_reduce_partials(nk, nb, fused_part_slots(a), L.part, 1.0 / nqn, acc, imsig, st);
            if (re_tilde)
                launch_reduce_partials_diff(nk, nb, fused_part_slots(a), L.part, L.part2, 1.0 / nqn, acc, re_tilde, st);
        } else if (!gkq) {
            launch_reduce_partials(nk, nb, fused_part_slots(a), L.part, scale, (c > 0 || par->accumulate) ? 1 : 0,
                                   imsig, st);
        }
    }
    if (omg) {
        if (L.nchunks == 0 && !par->accumulate && nk > 0) {
            launch_fill(2 * (size_t)nk * nb * L.nw, 0.0, (double*)sig_w, st);
            launch_fill(2 * (size_t)nk * nb, 0.0, (double*)sig0, st);
        }
    } else if (!gkq && !phon) {
        if (L.nchunks == 0 && !par->accumulate && nk > 0) {
            launch_fill((size_t)nk * nb, 0.0, imsig, st);
            if (re_tilde) launch_fill((size_t)nk * nb, 0.0, re_tilde, st);
        }
        launch_degenerate_average(nk, nb, L.eps, par->deg_tol, imsig, st);
        if (re_tilde) launch_degenerate_average(nk, nb, L.eps, par->deg_tol, re_tilde, st);
    }
}

// ---------------------------------------------------------------- adjoint

struct BwdLayout {
    Prec prec;
    int nbp, Q, nchunks;
    double* eps = nullptr;
    void* U = nullptr;
    double* ftab = nullptr;
    double* wbar = nullptr;
    void* phi_k = nullptr;
    double* ebar = nullptr;
    void* Ubar = nullptr;
    void* Xbar = nullptr;
    double* omega_c = nullptr;
    void* evec_c = nullptr;
    double* sc = nullptr;
    double* nbose = nullptr;
    void* phi_q = nullptr;
    void* gq = nullptr;      // a5 output, reused for the mode-basis adjoint
    void* Bnu = nullptr;     // a6 output, reused for gbar_nu(R_e,q)
    // folded sums over R_e <-> k (float64 / float32): the halved R list (as
    // in the forward) and its unweighted phases serve the sum over k
    // (ksum_fold_kernel) at every band count (fold_tab) and the recompute of G
    // on the fused kernel's tiling below 16 padded bands (fold), where B then
    // carries the 1/ndeg weights
    bool fold_tab = false;
    bool fold = false;
    int32_t* fneg = nullptr;
    int32_t* fhalf = nullptr;
    int32_t* fpair = nullptr;
    int32_t* fR = nullptr;
    int32_t* fkh = nullptr;
    void* phi_f = nullptr;
    void* G = nullptr;       // recomputed Wannier-basis g(k,q), overwritten by its adjoint
    double* ek_c = nullptr;
    double* ekq_c = nullptr;
    void* Uk_c = nullptr;
    void* Ukq_c = nullptr;
    double* om_c = nullptr;
    int32_t* inv = nullptr;
    double* eps_pair = nullptr;
    void* U_pair = nullptr;
    double* f_pair = nullptr;
    PairScratch ps;
    // float32 runs: g(R_e,R_p) and dL/dg(R_e,R_p) in complex64, and a float64
    // phase table for the dL/dH(R_e) contraction
    void* gR_t = nullptr;
    void* dgR_t = nullptr;
    void* phi_k64 = nullptr;
    // split-bf16 runs: the R_e <-> k contractions on bf16 planes (K contiguous)
    int kpad = 0;            // N_e padded to a multiple of 32
    int nkpad = 0;           // N_k padded to a multiple of 32
    void* Bpl = nullptr;     // [4][Q n_m NBP^2][kpad] mode-rotated vertex (recompute B)
    void* phiT = nullptr;    // [4][N_e][nkpad] conj phases (adjoint A)
    void* Gt = nullptr;      // [4][Q n_m NBP^2][nkpad] adjoint Gbar, transposed (adjoint B)
    void* polar_L = nullptr; // [Q][nm] c128 long-range factors (polar systems)
    int kparts = 1;          // split-K slices of the sum over k (conjugate-transposed GEMM)
    void* kpart = nullptr;   // [kparts][N_e][Q n_m NBP^2] partial products
    // off-grid dL/dH(R_e): per-pair eigen-adjoints of one batch, their sum
    // over pairs (split over pairs, then reduced), and the running total
    void* Xbar_pair = nullptr;   // [batch][n_b][n_b] c128
    int hparts = 1;
    void* hpart = nullptr;       // [hparts][N_e][n_b n_b] c128
    double* dHR_pair = nullptr;  // [N_e][n_b][n_b] c128
};

// automatic q chunk of the adjoint: its per-q scratch holds the recomputed
// vertex of every k (77 MB per q on the fcc 20^3 workload); 32 GB gives ~440 q
// per chunk there (FP64 adjoint 2071 -> 2019 ms against a 16 GB budget)
constexpr size_t AUTO_BWD_CHUNK_BYTES = (size_t)32 << 30;

void plan_bwd(const epw_system* s, const epw_points* p, const epw_params* par, Arena& A, BwdLayout& L) {
    L.prec = (Prec)par->dtype;
    L.nbp = pow2_at_least(s->nb);
    const size_t cb = cbytes(L.prec);
    const int nk = p->nk, nq = p->nq, nb = s->nb, nm = s->nm, ne = s->nRe, np_ = s->nRp;
    const bool given = p->omega && p->evec;
    const bool bf = L.prec == Prec::BF16X2;
    const size_t nbp2 = (size_t)L.nbp * L.nbp;
    L.kpad = (ne + 31) / 32 * 32;
    L.nkpad = (nk + 31) / 32 * 32;
    const size_t per_q = cb * ((size_t)nk * nm * nbp2 + 6 * (size_t)ne * nm * nbp2 + np_) +
                         (bf ? 8 * ((size_t)L.kpad + L.nkpad) * nm * nbp2 : 0) +
                         (size_t)nk * (16 * nb + 32 * (size_t)nb * nb + 8 * nm + 4) +
                         (given ? 0 : 8 * (size_t)nm + 16 * (size_t)nm * nm) + 16 * (size_t)nm +
                         pair_bytes_per_q(s, p);
    long Q = par->chunk_q > 0 ? par->chunk_q : auto_chunk(nq, AUTO_BWD_CHUNK_BYTES, per_q);
    if (Q < 1) Q = 1;
    if (Q > nq) Q = nq > 0 ? nq : 1;
    L.Q = (int)Q;
    L.nchunks = nq > 0 ? (int)((nq + Q - 1) / Q) : 0;
    L.eps = (double*)A.take(8 * (size_t)nk * nb);
    L.U = A.take(16 * (size_t)nk * nb * nb);
    L.ftab = (double*)A.take(8 * (size_t)nk * nb);
    L.wbar = (double*)A.take(8 * (size_t)nk * nb);
    L.phi_k = A.take(bf ? 8 * (size_t)nk * L.kpad : cb * (size_t)nk * ne);
    L.fold_tab = !bf;
    L.fold = L.fold_tab && L.nbp < 16 && fused_fold_c(L.nbp, (int)L.prec);
    if (L.fold_tab) {
        L.fneg = (int32_t*)A.take(4 * (size_t)ne);
        L.fhalf = (int32_t*)A.take(4 * (size_t)ne);
        L.fpair = (int32_t*)A.take(4 * (size_t)ne);
        L.fR = (int32_t*)A.take(12 * (size_t)ne);
        L.fkh = (int32_t*)A.take(4);
        L.phi_f = A.take(cb * (size_t)nk * ne);
    }
    L.ebar = (double*)A.take(8 * (size_t)nk * nb);
    L.Ubar = A.take(16 * (size_t)nk * nb * nb);
    L.Xbar = A.take(16 * (size_t)nk * nb * nb);
    if (!given) {
        L.omega_c = (double*)A.take(8 * (size_t)L.Q * nm);
        L.evec_c = A.take(16 * (size_t)L.Q * nm * nm);
    }
    L.sc = (double*)A.take(8 * (size_t)L.Q * nm);
    L.nbose = (double*)A.take(8 * (size_t)L.Q * nm);
    L.phi_q = A.take(cb * (size_t)L.Q * np_);
    L.gq = A.take(cb * (size_t)ne * L.Q * nm * nb * nb);
    L.Bnu = A.take(cb * (size_t)ne * L.Q * nm * nbp2);
    if (s->polar) L.polar_L = A.take(16 * (size_t)L.Q * nm);
    L.G = A.take(cb * (size_t)nk * L.Q * nm * nbp2);
    L.ek_c = (double*)A.take(8 * (size_t)nk * L.Q * nb);
    L.ekq_c = (double*)A.take(8 * (size_t)nk * L.Q * nb);
    L.Uk_c = A.take(16 * (size_t)nk * L.Q * nb * nb);
    L.Ukq_c = A.take(16 * (size_t)nk * L.Q * nb * nb);
    L.om_c = (double*)A.take(8 * (size_t)nk * L.Q * nm);
    L.inv = (int32_t*)A.take(4 * (size_t)nk * L.Q);
    take_pair_states(s, p, L.Q, A, L.eps_pair, L.U_pair, L.f_pair, L.ps);
    if (!p->kq) {
        const size_t nbb = (size_t)nb * nb;
        L.Xbar_pair = A.take(16 * (size_t)L.ps.batch * nbb);
        L.hparts = splitk_parts_wide(ne, (int)nbb, (int)L.ps.batch, 32);
        if (L.hparts > 1) L.hpart = A.take(16 * (size_t)L.hparts * ne * nbb);
        L.dHR_pair = (double*)A.take(16 * (size_t)ne * nbb);
    }
    L.kparts = bf ? 1 : splitk_parts(ne, (int)((size_t)L.Q * nm * nbp2), nk);
    if (L.kparts > 1) L.kpart = A.take(cb * (size_t)L.kparts * ne * L.Q * nm * nbp2);
    if (L.prec != Prec::F64) {
        const size_t ng = (size_t)ne * np_ * nm * nb * nb;
        L.gR_t = A.take(8 * ng);
        L.dgR_t = A.take(8 * ng);
        L.phi_k64 = A.take(16 * (size_t)nk * ne);
    }
    if (bf) {
        const size_t cols = (size_t)L.Q * nm * nbp2;
        L.Bpl = A.take(8 * cols * L.kpad);
        L.phiT = A.take(8 * (size_t)ne * L.nkpad);
        L.Gt = A.take(8 * cols * L.nkpad);
    }
}

void run_backward(const epw_system* s, const epw_points* p, const epw_params* par, BwdLayout& L, const double* w,
                  void* dgR, void* dHR, double* domega, hipStream_t st) {
    const int nk = p->nk, nq = p->nq, nb = s->nb, nm = s->nm, ne = s->nRe, np_ = s->nRp;
    const Prec prec = L.prec;
    const bool given = p->omega && p->evec;
    const int acc0 = par->accumulate ? 1 : 0;
    const size_t ncol_g = (size_t)nm * nb * nb;
    {
        StageTimer t(EPW_STAGE_EIGH, st);
        launch_interp_eigh(false, false, nb, ne, s->Re, s->ndeg_e, (const double*)s->HR, nk, p->kfrac, L.eps,
                           L.U, st);
    }
    launch_fermi_table((size_t)nk * nb, L.eps, par->mu, par->T, L.ftab, st);
    EPW_HIP(hipMemcpyAsync(L.wbar, w, 8 * (size_t)nk * nb, hipMemcpyDeviceToDevice, st));
    launch_degenerate_average(nk, nb, L.eps, par->deg_tol, L.wbar, st);
    const bool bf = prec == Prec::BF16X2;
    // contraction precision of everything but the R_e <-> k sums (split-bf16
    // runs those on bf16 planes and the rest in float32, as the forward does)
    const Prec cprec = bf ? Prec::F32 : prec;
    if (bf) {
        launch_phase_table(Prec::BF16X2, nk, p->kfrac, ne, s->Re, s->ndeg_e, L.kpad, L.phi_k, st);
        launch_phase_planes_t(nk, p->kfrac, ne, s->Re, s->ndeg_e, L.nkpad, L.phiT, st);
    } else {
        launch_phase_table(prec, nk, p->kfrac, ne, s->Re, s->ndeg_e, ne, L.phi_k, st);
    }
    if (L.fold_tab) {
        launch_half_list(ne, s->Re, L.fneg, L.fhalf, L.fpair, L.fR, L.fkh, st);
        launch_phase_table(prec, nk, p->kfrac, ne, L.fR, nullptr, ne, L.phi_f, st);
    }
    launch_fill((size_t)nk * nb, 0.0, L.ebar, st);
    launch_fill(2 * (size_t)nk * nb * nb, 0.0, (double*)L.Ubar, st);
    if (dgR && (L.nchunks == 0) && !acc0)
        launch_fill(2 * (size_t)ne * np_ * ncol_g, 0.0, (double*)dgR, st);
    const bool offgrid = !p->kq;
    if (dHR && offgrid) launch_fill(2 * (size_t)ne * nb * nb, 0.0, L.dHR_pair, st);
    const double nqn = par->nq_norm > 0.0 ? par->nq_norm : (double)nq;
    const double C = M_PI / (nqn * par->sigma * std::sqrt(M_PI));
    const double kT = 8.617333262e-5 * par->T;
    const bool f32 = prec != Prec::F64;    // float32 storage of g, dL/dg and the vertex
    const void* gsrc = s->gR;
    if (f32) {
        launch_c128_to_c64((size_t)ne * np_ * ncol_g, s->gR, L.gR_t, st);
        gsrc = L.gR_t;
    }
    for (int c = 0; c < L.nchunks; ++c) {
        const int q0 = c * L.Q;
        const int qc = (q0 + L.Q <= nq) ? L.Q : nq - q0;
        const double* om;
        const void* ev;
        if (given) {
            om = p->omega + (size_t)q0 * nm;
            ev = (const char*)p->evec + 16 * (size_t)q0 * nm * nm;
        } else {
            StageTimer t(EPW_STAGE_EIGH, st);
            launch_interp_eigh(true, true, nm, np_, s->Rp, s->ndeg_p, s->DR, qc, p->qfrac + 3 * (size_t)q0,
                               L.omega_c, L.evec_c, st);
            om = L.omega_c;
            ev = L.evec_c;
        }
        launch_phonon_factors(qc, nm, om, par->omega_cut, par->T, L.sc, L.nbose, st);
        if (s->polar) {
            // the long-range part is proportional to 1/sqrt(2 omega) like the rest of g, so
            // the per-pair omega adjoint (|g|^2 ~ 1/omega) covers it; it depends on g(R_e,R_p)
            // and H(R_e) only through the rotations
            PolarDev P;
            polar_device(s->polar, nm, P);
            launch_polar_factor(P, qc, nm, p->qfrac + 3 * (size_t)q0, ev, L.sc, L.polar_L, st);
        }
        launch_phase_table(cprec, qc, p->qfrac + 3 * (size_t)q0, np_, s->Rp, s->ndeg_p, np_, L.phi_q, st);
        pair_states(s, p, par, q0, qc, L.eps_pair, L.U_pair, L.f_pair, L.ps, st);
        const long ncols = (long)qc * nm * L.nbp * L.nbp;
        StageTimer tb(EPW_STAGE_BACKWARD, st);
        {
            StageTimer tg(EPW_STAGE_BWD_GEMM, st);
            launch_cgemm(cprec, rp_desc(qc, ne, np_, (int)ncol_g, L.phi_q, gsrc, L.gq), st);
        }
        if (bf) {
            // recompute G = Phi_k B on bf16 planes (the forward's R_e -> k arithmetic)
            launch_mode_rotate_bf16(ne, qc, nm, nb, L.nbp, L.kpad, L.gq, ev, L.sc, L.Bpl, st, nullptr, L.polar_L,
                                    s->Re);
            Bf16GemmDesc d;
            d.M = nk;
            d.N = ncols;
            d.Kpad = L.kpad;
            d.A = (const uint16_t*)L.phi_k;
            d.lda = L.kpad;
            d.aplane = (long)nk * L.kpad;
            d.B = (const uint16_t*)L.Bpl;
            d.ldb = L.kpad;
            d.bplane = ncols * L.kpad;
            d.C = (float2*)L.G;
            d.ldc = ncols;
            StageTimer tg(EPW_STAGE_BWD_GEMM, st);
            launch_bf16_gemm(d, st);
        } else {
            // the folded recompute takes the 1/ndeg weights in B (its phases are
            // unweighted), the generic GEMM in the phase table
            if (L.fold)
                launch_mode_rotate_fold(prec, ne, qc, nm, nb, L.nbp, L.gq, ev, L.sc, s->ndeg_e, L.fkh, L.fhalf,
                                        L.fpair, L.polar_L, s->Re, L.Bnu, st);
            else
                launch_mode_rotate(prec, ne, qc, nm, nb, L.nbp, L.gq, ev, L.sc, L.Bnu, st, nullptr, L.polar_L, s->Re);
        }
        if (!bf && L.nbp >= 16) {   // recompute G = Phi_k B (Wannier basis, all k of the chunk)
            GemmDesc d;
            d.M = nk;
            d.N = (int)ncols;
            d.K = ne;
            d.A = L.phi_k;
            d.lda = ne;
            d.B = L.Bnu;
            d.ncb = (int)ncols;
            d.sBk = ncols;
            d.C = L.G;
            d.sCm = ncols;
            StageTimer tg(EPW_STAGE_BWD_GEMM, st);
            launch_cgemm(prec, d, st);
        } else if (!bf) {
            // recompute G on the forward's R_e -> k tiling (64 x 64 up to 8
            // padded bands), without its epilogue (the 16 x 256 tiles of 16
            // bands are slower than the generic GEMM's 64 x 64)
            FusedArgs a;
            a.nk = nk;
            a.ne = ne;
            a.nb = nb;
            a.nbp = L.nbp;
            a.nm = nm;
            a.qc = qc;
            a.q0 = q0;
            a.nq_total = nq;
            a.phi_k = L.phi_f;
            a.half = L.fhalf;
            a.pair = L.fpair;
            a.kh = L.fkh;
            a.ldk = ne;
            a.nmax = 0;
            a.Re = s->Re;
            a.ndeg_e = s->ndeg_e;
            a.kfrac = p->kfrac;
            a.ldk_b = ne;
            a.kpad = ne;
            a.B = L.Bnu;
            a.eps = L.eps;
            a.U = L.U;
            a.ftab = L.ftab;
            a.kq = p->kq;
            a.eps_pair = L.eps_pair;
            a.U_pair = L.U_pair;
            a.f_pair = L.f_pair;
            a.omega = om;
            a.nbose = L.nbose;
            a.sc = L.sc;
            a.sigma = par->sigma;
            a.mu = par->mu;
            a.part = nullptr;
            a.S = fused_slices(nk, L.nbp, tiles_n_for(qc, nm, L.nbp, prec), SLICE_CUS, prec);
            fused_balance(a, prec, SLICE_CUS);
            a.gkq = nullptr;
            a.part_ph = nullptr;
            a.part2 = nullptr;
            a.rec = nullptr;
            a.vel = nullptr;
            a.vel_pair = nullptr;
            a.gout = L.G;
            StageTimer tg(EPW_STAGE_BWD_GEMM, st);
            launch_fused_k(prec, a, SLICE_CUS, st);
        }
        PairBwdArgs a;
        a.nk = nk;
        a.nb = nb;
        a.nbp = L.nbp;
        a.nm = nm;
        a.qc = qc;
        a.q0 = q0;
        a.nq_total = nq;
        a.G = L.G;
        a.eps = L.eps;
        a.U = L.U;
        a.ftab = L.ftab;
        a.wbar = L.wbar;
        a.kq = p->kq;
        a.eps_pair = L.eps_pair;
        a.U_pair = L.U_pair;
        a.f_pair = L.f_pair;
        a.omega = om;
        a.nbose = L.nbose;
        a.sc = L.sc;
        a.sigma = par->sigma;
        a.kT = kT;
        a.C = C;
        a.ek_c = L.ek_c;
        a.Uk_c = L.Uk_c;
        a.ekq_c = L.ekq_c;
        a.Ukq_c = L.Ukq_c;
        a.om_c = L.om_c;
        launch_pair_bwd(cprec, a, st);
        if (dHR && !offgrid) {
            launch_kq_inverse(nk, qc, q0, nq, p->kq, L.inv, st);
            launch_gather_state_adjoint(nk, nb, qc, L.inv, L.ek_c, L.Uk_c, L.ekq_c, L.Ukq_c, L.ebar, L.Ubar, st);
        } else if (dHR) {
            // k side summed over the chunk's q; the k+q side stays per pair: the
            // eigen-adjoint of every H(k+q), contracted back to R_e through the
            // conjugate of the pair phases e^{2 pi i (k+q).R}/ndeg that formed it
            launch_gather_state_adjoint(nk, nb, qc, nullptr, L.ek_c, L.Uk_c, nullptr, nullptr, L.ebar, L.Ubar, st);
            const long npair = (long)nk * qc;
            const size_t nbb = (size_t)nb * nb;
            for (long b0 = 0; b0 < npair; b0 += L.ps.batch) {
                const int nbt = (int)std::min(L.ps.batch, npair - b0);
                launch_eigh_adjoint(nbt, nb, L.eps_pair + (size_t)b0 * nb, (const char*)L.U_pair + 16 * (size_t)b0 * nbb,
                                    L.ekq_c + (size_t)b0 * nb, (const char*)L.Ukq_c + 16 * (size_t)b0 * nbb,
                                    par->deg_tol, L.Xbar_pair, st);
                GemmDesc d;   // dHR_pair[e][ij] += sum_pair conj(Phi_k[k][e] Phi_q[q][e]) Xbar[pair][ij]
                d.M = ne;
                d.N = (int)nbb;
                d.K = nbt;
                d.A = L.ps.phi_k;
                d.lda = ne;
                d.A2 = L.ps.phi_q;
                d.n2 = qc;
                d.row0 = b0;
                d.conj_trans_a = 1;
                d.B = L.Xbar_pair;
                d.ncb = (int)nbb;
                d.sBk = (long)nbb;
                d.C = L.dHR_pair;
                d.sCm = (long)nbb;
                d.accumulate = 1;
                launch_cgemm_splitk(Prec::F64, d, std::min(L.hparts, splitk_parts_wide(ne, (int)nbb, nbt, 32)),
                                    L.hpart, st);
            }
        }
        if (domega) launch_reduce_omega(nk, qc, nm, L.om_c, acc0, domega + (size_t)q0 * nm, st);
        if (dgR && bf) {
            // gbar_nu(R_e, q) = sum_k conj(Phi_k[k][R_e]) Gbar[k][col] on bf16 planes
            launch_split_transpose(nk, ncols, L.G, L.nkpad, L.Gt, st);
            Bf16GemmDesc d;
            d.M = ne;
            d.N = ncols;
            d.Kpad = L.nkpad;
            d.A = (const uint16_t*)L.phiT;
            d.lda = L.nkpad;
            d.aplane = (long)ne * L.nkpad;
            d.B = (const uint16_t*)L.Gt;
            d.ldb = L.nkpad;
            d.bplane = ncols * L.nkpad;
            d.C = (float2*)L.Bnu;
            d.ldc = ncols;
            StageTimer tg(EPW_STAGE_BWD_GEMM, st);
            launch_bf16_gemm(d, st);
        } else if (dgR && L.fold_tab) {
            // gbar_nu(R_e, q) = sum_k conj(Phi_k[k][R_e]) Gbar[k][col] / ndeg(R_e) over the
            // pairs (R, -R): a real-by-complex product of the halved list
            KsumFoldDesc d;
            d.nk = nk;
            d.ne = ne;
            d.ncols = ncols;
            d.phi = L.phi_f;
            d.ld = ne;
            d.G = L.G;
            d.half = L.fhalf;
            d.pair = L.fpair;
            d.kh = L.fkh;
            d.ndeg = s->ndeg_e;
            StageTimer tg(EPW_STAGE_BWD_GEMM, st);
            launch_ksum_fold(prec, d, std::min(splitk_parts(ne, (int)ncols, nk), L.kparts), L.kpart, L.Bnu, st);
        } else if (dgR) {
            GemmDesc d;   // gbar_nu(R_e, q) = sum_k conj(Phi_k[k][R_e]) Gbar[k][col]
            d.M = ne;
            d.N = (int)ncols;
            d.K = nk;
            d.A = L.phi_k;
            d.lda = ne;
            d.conj_trans_a = 1;
            d.B = L.G;
            d.ncb = (int)ncols;
            d.sBk = ncols;
            d.C = L.Bnu;
            d.sCm = ncols;
            // K = N_k is long and M = N_e short: split the sum over k so the grid fills the chip
            StageTimer tg(EPW_STAGE_BWD_GEMM, st);
            launch_cgemm_splitk(prec, d, std::min(splitk_parts(d.M, d.N, d.K), L.kparts), L.kpart, st);
        }
        if (dgR) {
            launch_mode_rotate_adjoint(cprec, ne, qc, nm, nb, L.nbp, L.Bnu, ev, L.sc, L.gq, st);
            GemmDesc e;   // dgR[e][p][c] (+)= sum_q conj(Phi_q[q][p]) gbar_a[e][q][c]
            e.M = np_;
            e.N = (int)(ne * ncol_g);
            e.K = qc;
            e.A = L.phi_q;
            e.lda = np_;
            e.conj_trans_a = 1;
            e.B = L.gq;
            e.ncb = (int)ncol_g;
            e.sBe = (long)qc * ncol_g;
            e.sBk = (long)ncol_g;
            // float32: accumulated over chunks in complex64, converted at the end
            e.C = f32 ? L.dgR_t : dgR;
            e.sCe = (long)np_ * ncol_g;
            e.sCm = (long)ncol_g;
            e.accumulate = (c > 0 || (acc0 && !f32)) ? 1 : 0;
            StageTimer tg(EPW_STAGE_BWD_GEMM, st);
            launch_cgemm(cprec, e, st);
        }
    }
    if (dgR && f32 && L.nchunks > 0) launch_c64_to_c128((size_t)ne * np_ * ncol_g, L.dgR_t, acc0, dgR, st);
    if (dHR) {
        launch_eigh_adjoint(nk, nb, L.eps, L.U, L.ebar, L.Ubar, par->deg_tol, L.Xbar, st);
        if (f32) launch_phase_table(Prec::F64, nk, p->kfrac, ne, s->Re, s->ndeg_e, ne, L.phi_k64, st);
        GemmDesc d;   // dHR[e][ij] (+)= sum_k conj(Phi_k[k][R_e]) Xbar[k][ij]
        d.M = ne;
        d.N = nb * nb;
        d.K = nk;
        d.A = f32 ? L.phi_k64 : L.phi_k;
        d.lda = ne;
        d.conj_trans_a = 1;
        d.B = L.Xbar;
        d.ncb = nb * nb;
        d.sBk = nb * nb;
        d.C = dHR;
        d.sCm = nb * nb;
        d.accumulate = acc0;
        launch_cgemm(Prec::F64, d, st);
        if (offgrid) launch_add_f64(2 * (size_t)ne * nb * nb, L.dHR_pair, (double*)dHR, st);
    }
}

template <class F>
int guarded(const char* fn, F body) {
    try {
        return body();
    } catch (const HipFailure& e) {
        return fail(EPW_EHIP, "%s: HIP error %d (%s) in %s at %s:%d", fn, e.code,
                    hipGetErrorString((hipError_t)e.code), e.call, e.file, e.line);
    } catch (...) {
        return fail(EPW_EINVAL, "%s: unexpected host exception", fn);
    }
}

}  // namespace
}  // namespace epw

using namespace epw;

extern "C" int epw_interp_bands(int nb, int nR, const int32_t* R, const int32_t* ndeg, const void* HR,
                                int nk, const double* kfrac, double* eps, void* U, void* stream) {
    clear_error();
    if (nb < 1 || nb > EPW_MAX_NB) return fail(EPW_ESHAPE, "epw_interp_bands: nb = %d not in 1..%d", nb, EPW_MAX_NB);
    if (nR < 1 || nk < 0) return fail(EPW_ESHAPE, "epw_interp_bands: nR = %d, nk = %d", nR, nk);
    if (nk == 0) return EPW_OK;
    if (!R || !ndeg || !HR || !kfrac || !eps || !U) return fail(EPW_EINVAL, "epw_interp_bands: NULL argument");
    return guarded("epw_interp_bands", [&]() {
        launch_interp_eigh(false, false, nb, nR, R, ndeg, (const double*)HR, nk, kfrac, eps, U,
                           (hipStream_t)stream);
        return EPW_OK;
    });
}

extern "C" int epw_interp_phonons(int nm, int nR, const int32_t* R, const int32_t* ndeg, const double* DR,
                                  int nq, const double* qfrac, double* omega, void* evec, void* stream) {
    clear_error();
    if (nm < 1 || nm > EPW_MAX_NM) return fail(EPW_ESHAPE, "epw_interp_phonons: nm = %d not in 1..%d", nm, EPW_MAX_NM);
    if (nR < 1 || nq < 0) return fail(EPW_ESHAPE, "epw_interp_phonons: nR = %d, nq = %d", nR, nq);
    if (nq == 0) return EPW_OK;
    if (!R || !ndeg || !DR || !qfrac || !omega || !evec) return fail(EPW_EINVAL, "epw_interp_phonons: NULL argument");
    return guarded("epw_interp_phonons", [&]() {
        launch_interp_eigh(true, true, nm, nR, R, ndeg, DR, nq, qfrac, omega, evec, (hipStream_t)stream);
        return EPW_OK;
    });
}

// Size queries run the shape checks on copies of the structs whose missing
// pointers are replaced by placeholders (never dereferenced).
int size_query_checks(const epw_system* sys, const epw_points* pts, const epw_params* par, const char* fn,
                      epw_system& s, epw_points& p) {
    if (!sys || !pts || !par) return fail(EPW_EINVAL, "%s: NULL argument", fn);
    p = *pts;
    s = *sys;
    static const int32_t dummy_i = 0;
    static const double dummy_d = 0.0;
    if (!p.kfrac) p.kfrac = &dummy_d;
    if (!p.qfrac) p.qfrac = &dummy_d;
    if (!s.Re) s.Re = &dummy_i;
    if (!s.Rp) s.Rp = &dummy_i;
    if (!s.ndeg_e) s.ndeg_e = &dummy_i;
    if (!s.ndeg_p) s.ndeg_p = &dummy_i;
    if (!s.HR) s.HR = &dummy_d;
    if (!s.gR) s.gR = &dummy_d;
    if (!s.DR && !(p.omega && p.evec)) s.DR = &dummy_d;
    return check_common(&s, &p, par, fn);
}

// Shared tail of the forward entry points: size the workspace, carve it and
// run the pipeline, with HIP failures turned into status codes.
int planned_forward(const char* fn, const epw_system* sys, const epw_points* pts, const epw_params* par, Out out,
                    int nw, void* ws, size_t ws_bytes, void* stream, const Outputs& o) {
    Arena dry;
    dry.dry = true;
    Layout L;
    plan(sys, pts, par, out, dry, L, nw);
    if (!ws || ws_bytes < dry.used + 256)
        return fail(EPW_ENOMEM, "%s: workspace %zu bytes, need %zu", fn, ws_bytes, dry.used + 256);
    return guarded(fn, [&]() {
        Arena A;
        A.base = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
        A.cap = ws_bytes;
        plan(sys, pts, par, out, A, L, nw);
        run_forward(sys, pts, par, L, o, (hipStream_t)stream);
        return EPW_OK;
    });
}

namespace epw {
namespace {

// q points per pass of the k+q map check (its inverse map is [nk][Qc] int32)
int check_kq_chunk(const epw_points* p) {
    if (!p->kq || p->nk <= 0 || p->nq <= 0) return 0;
    const long q = std::max<long>(1, (4L << 20) / p->nk);
    return (int)std::min<long>(q, p->nq);
}

size_t check_ws_bytes(const epw_system* s, const epw_points* p) {
    Arena A;
    A.dry = true;
    A.take(sizeof(CheckRecord));
    A.take(4 * (size_t)s->nRe);
    A.take(4 * (size_t)s->nRp);
    A.take(4 * (size_t)std::max(p->nk, 0) * check_kq_chunk(p));
    return A.used + 256;
}

// parameters that pass check_common (epw_check_inputs has none of its own)
epw_params neutral_params() {
    epw_params q;
    std::memset(&q, 0, sizeof(q));
    q.sigma = 1.0;
    q.dtype = EPW_FP64;
    return q;
}

}  // namespace
}  // namespace epw

namespace epw {

// Im Sigma in a fixed device buffer of `cap` bytes (the no-allocation entry
// point).  With par->chunk_q = 0 the largest q chunk whose workspace fits is
// taken; a given chunk_q must fit as it is.  Argument and size checks run
// before anything touches the device; `base` is asked for only once they
// have passed.
int imsigma_in_buffer(const char* fn, const epw_system* sys, const epw_points* pts, const epw_params* par,
                      double* imsig, size_t cap, void* (*base)(int* rc), void* stream) {
    int rc = check_common(sys, pts, par, fn);
    if (rc != EPW_OK) return rc;
    if (pts->nk == 0) return EPW_OK;
    if (!imsig) return fail(EPW_EINVAL, "%s: NULL output", fn);
    auto need = [&](int q) {
        epw_params t = *par;
        t.chunk_q = q;
        Arena dry;
        dry.dry = true;
        Layout L;
        plan(sys, pts, &t, Out::IMSIGMA, dry, L);
        return dry.used + 256;
    };
    epw_params fitted = *par;
    if (par->chunk_q > 0) {
        const size_t n = need(par->chunk_q);
        if (n > cap)
            return fail(EPW_ENOMEM, "%s: chunk_q = %d needs %zu bytes of scratch, the library's buffer holds %zu", fn,
                        par->chunk_q, n, cap);
    } else {
        const size_t n1 = need(1);
        if (n1 > cap)
            return fail(EPW_ENOMEM, "%s: these sizes need %zu bytes of scratch even one q point at a time, the "
                        "library's buffer holds %zu", fn, n1, cap);
        // the workspace grows with the chunk; take the largest chunk that fits
        int lo = 1, hi = pts->nq > 1 ? pts->nq : 1;
        while (lo < hi) {
            const int mid = lo + (hi - lo + 1) / 2;
            if (need(mid) <= cap) lo = mid;
            else hi = mid - 1;
        }
        while (lo > 1 && need(lo) > cap) --lo;
        fitted.chunk_q = lo;
    }
    int brc = EPW_OK;
    void* ws = base(&brc);
    if (brc != EPW_OK) return brc;
    Outputs o;
    o.imsig = imsig;
    return planned_forward(fn, sys, pts, &fitted, Out::IMSIGMA, 0, ws, cap, stream, o);
}

}  // namespace epw

extern "C" size_t epw_workspace_size(int which, const epw_system* sys, const epw_points* pts,
                                     const epw_params* par) {
    clear_error();
    if (which != EPW_WS_INTERP_G && which != EPW_WS_IMSIGMA && which != EPW_WS_IMSIGMA_BACKWARD &&
        which != EPW_WS_PHONON && which != EPW_WS_RESIGMA && which != EPW_WS_TRANSPORT && which != EPW_WS_CHECK) {
        fail(EPW_EINVAL, "epw_workspace_size: unknown call id %d", which);
        return 0;
    }
    epw_system s;
    epw_points p;
    if (size_query_checks(sys, pts, par, "epw_workspace_size", s, p) != EPW_OK) return 0;
    if (which == EPW_WS_CHECK) return check_ws_bytes(&s, &p);
    Arena A;
    A.dry = true;
    if (which == EPW_WS_IMSIGMA_BACKWARD) {
        BwdLayout L;
        plan_bwd(&s, &p, par, A, L);
    } else {
        Layout L;
        const Out o = which == EPW_WS_INTERP_G ? Out::STORE
                      : which == EPW_WS_PHONON ? Out::PHONON
                      : which == EPW_WS_RESIGMA ? Out::RESIGMA
                      : which == EPW_WS_TRANSPORT ? Out::TRANSPORT : Out::IMSIGMA;
        plan(&s, &p, par, o, A, L);
    }
    return A.used + 256;
}

extern "C" int epw_check_inputs(const epw_system* sys, const epw_points* pts, double herm_tol, void* ws,
                                size_t ws_bytes, void* stream) {
    clear_error();
    const char* fn = "epw_check_inputs";
    const epw_params np0 = neutral_params();
    int rc = check_common(sys, pts, &np0, fn);
    if (rc != EPW_OK) return rc;
    if (!(herm_tol >= 0.0) || !std::isfinite(herm_tol)) return fail(EPW_EINVAL, "%s: herm_tol must be >= 0", fn);
    if (!sys->Re || !sys->ndeg_e || !sys->Rp || !sys->ndeg_p || !sys->HR || !sys->gR)
        return fail(EPW_EINVAL, "%s: NULL pointer in epw_system", fn);
    if ((pts->nk > 0 && !pts->kfrac) || (pts->nq > 0 && !pts->qfrac)) return fail(EPW_EINVAL, "%s: NULL point array", fn);
    const size_t need = check_ws_bytes(sys, pts);
    if (!ws || ws_bytes < need) return fail(EPW_ENOMEM, "%s: workspace %zu bytes, need %zu", fn, ws_bytes, need);
    CheckRecord h;
    rc = guarded(fn, [&]() {
        hipStream_t st = (hipStream_t)stream;
        Arena A;
        A.base = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
        A.cap = ws_bytes;
        CheckRecord* rec = (CheckRecord*)A.take(sizeof(CheckRecord));
        int32_t* negE = (int32_t*)A.take(4 * (size_t)sys->nRe);
        int32_t* negP = (int32_t*)A.take(4 * (size_t)sys->nRp);
        const int qck = check_kq_chunk(pts);
        int32_t* inv = (int32_t*)A.take(4 * (size_t)std::max(pts->nk, 0) * qck);
        const size_t nb = sys->nb, nm = sys->nm, ne = sys->nRe, np_ = sys->nRp;
        launch_check_clear(rec, st);
        launch_check_finite(2 * ne * nb * nb, (const double*)sys->HR, 1, rec, st);
        if (sys->DR) launch_check_finite(np_ * nm * nm, sys->DR, 2, rec, st);
        launch_check_finite(2 * ne * np_ * nm * nb * nb, (const double*)sys->gR, 4, rec, st);
        launch_check_finite(3 * (size_t)pts->nk, pts->kfrac, 8, rec, st);
        launch_check_finite(3 * (size_t)pts->nq, pts->qfrac, 8, rec, st);
        if (pts->omega) launch_check_finite((size_t)pts->nq * nm, pts->omega, 16, rec, st);
        if (pts->evec) launch_check_finite(2 * (size_t)pts->nq * nm * nm, (const double*)pts->evec, 16, rec, st);
        launch_check_ws(sys->nRe, sys->Re, sys->ndeg_e, sys->nmax_e, 1, negE, rec, st);
        launch_check_ws(sys->nRp, sys->Rp, sys->ndeg_p, 0, 2, negP, rec, st);
        launch_check_herm(true, sys->nb, sys->nRe, (const double*)sys->HR, negE, &rec->h_dev, &rec->h_max, st);
        if (sys->DR) launch_check_herm(false, sys->nm, sys->nRp, sys->DR, negP, &rec->d_dev, &rec->d_max, st);
        for (int q0 = 0; qck > 0 && q0 < pts->nq; q0 += qck) {
            const int qc = std::min(qck, pts->nq - q0);
            launch_check_kq(pts->nk, qc, q0, pts->nq, pts->kq, inv, rec, st);
        }
        EPW_HIP(hipMemcpyAsync(&h, rec, sizeof(h), hipMemcpyDeviceToHost, st));
        EPW_HIP(hipStreamSynchronize(st));
        return EPW_OK;
    });
    if (rc != EPW_OK) return rc;
    auto bits = [](unsigned long long b) {
        double v;
        std::memcpy(&v, &b, sizeof(v));
        return v;
    };
    static const char* const what[] = {"H(R_e)", "D(R_p)", "g(R_e,R_p)", "the k or q points",
                                       "the given phonon frequencies or modes"};
    for (int b = 0; b < 5; ++b)
        if (h.nonfinite & (1 << b)) return fail(EPW_EINVAL, "%s: non-finite entries in %s", fn, what[b]);
    if (h.ndeg_bad) return fail(EPW_EINVAL, "%s: a WS degeneracy of %s is < 1", fn, (h.ndeg_bad & 1) ? "R_e" : "R_p");
    if (h.nmax_bad)
        return fail(EPW_EINVAL, "%s: nmax_e = %d is smaller than a component of R_e", fn, sys->nmax_e);
    if (h.not_closed)
        return fail(EPW_ESHAPE, "%s: the WS set %s is not closed under R -> -R", fn,
                    (h.not_closed & 1) ? "R_e" : "R_p");
    const double hd = bits(h.h_dev), hm = bits(h.h_max), dd = bits(h.d_dev), dm = bits(h.d_max);
    if (hd > herm_tol * hm)
        return fail(EPW_ENOTHERM, "%s: max |H(-R) - H(R)^dag| = %.3e exceeds %.3e x max |H| = %.3e", fn, hd,
                    herm_tol, hm);
    if (dd > herm_tol * dm)
        return fail(EPW_ENOTHERM, "%s: max |D(-R) - D(R)^T| = %.3e exceeds %.3e x max |D| = %.3e", fn, dd, herm_tol,
                    dm);
    if (h.kq_range) return fail(EPW_EINVAL, "%s: a kq entry lies outside [0, nk)", fn);
    if (h.kq_not_bijective) return fail(EPW_EINVAL, "%s: for some q the map k -> kq[k][q] is not one-to-one", fn);
    return EPW_OK;
}

extern "C" int epw_interp_g(const epw_system* sys, const epw_points* pts, const epw_params* par, void* gkq,
                            void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    int rc = check_common(sys, pts, par, "epw_interp_g");
    if (rc != EPW_OK) return rc;
    if (pts->nk == 0 || pts->nq == 0) return EPW_OK;
    if (!gkq) return fail(EPW_EINVAL, "epw_interp_g: NULL output");
    Outputs o;
    o.gkq = gkq;
    return planned_forward("epw_interp_g", sys, pts, par, Out::STORE, 0, ws, ws_bytes, stream, o);
}

extern "C" int epw_imsigma(const epw_system* sys, const epw_points* pts, const epw_params* par, double* imsig,
                           void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    int rc = check_common(sys, pts, par, "epw_imsigma");
    if (rc != EPW_OK) return rc;
    if (pts->nk == 0) return EPW_OK;
    if (!imsig) return fail(EPW_EINVAL, "epw_imsigma: NULL output");
    Outputs o;
    o.imsig = imsig;
    return planned_forward("epw_imsigma", sys, pts, par, Out::IMSIGMA, 0, ws, ws_bytes, stream, o);
}

extern "C" size_t epw_workspace_size_omega(const epw_system* sys, const epw_points* pts, const epw_params* par,
                                           int nw) {
    clear_error();
    if (nw < 0 || nw > EPW_MAX_NW) {
        fail(EPW_ESHAPE, "epw_workspace_size_omega: nw = %d not in 0..%d", nw, EPW_MAX_NW);
        return 0;
    }
    epw_system s;
    epw_points p;
    if (size_query_checks(sys, pts, par, "epw_workspace_size_omega", s, p) != EPW_OK) return 0;
    Arena A;
    A.dry = true;
    Layout L;
    plan(&s, &p, par, Out::OMEGA, A, L, nw);
    return A.used + 256;
}

extern "C" int epw_selfenergy_omega(const epw_system* sys, const epw_points* pts, const epw_params* par, int nw,
                                    const double* wgrid, void* sigma_w, void* sigma0, void* ws, size_t ws_bytes,
                                    void* stream) {
    clear_error();
    if (nw < 0 || nw > EPW_MAX_NW) return fail(EPW_ESHAPE, "epw_selfenergy_omega: nw = %d not in 0..%d", nw, EPW_MAX_NW);
    int rc = check_common(sys, pts, par, "epw_selfenergy_omega");
    if (rc != EPW_OK) return rc;
    if (pts->nk == 0) return EPW_OK;
    if (!sigma0 || (nw > 0 && (!sigma_w || !wgrid))) return fail(EPW_EINVAL, "epw_selfenergy_omega: NULL output or grid");
    Outputs o;
    o.wgrid = wgrid;
    o.sig_w = sigma_w;
    o.sig0 = sigma0;
    return planned_forward("epw_selfenergy_omega", sys, pts, par, Out::OMEGA, nw, ws, ws_bytes, stream, o);
}

extern "C" int epw_spectral_function(int nk, int nb, int nw, const double* eps, double mu, const double* wgrid,
                                     const void* sigma_w, const void* sigma0, double* A, void* stream) {
    clear_error();
    if (nk < 0 || nw < 0 || nb < 1 || nb > EPW_MAX_NB)
        return fail(EPW_ESHAPE, "epw_spectral_function: nk = %d, nb = %d, nw = %d", nk, nb, nw);
    if (!std::isfinite(mu)) return fail(EPW_EINVAL, "epw_spectral_function: mu not finite");
    if (nk == 0 || nw == 0) return EPW_OK;
    if (!eps || !wgrid || !sigma_w || !sigma0 || !A) return fail(EPW_EINVAL, "epw_spectral_function: NULL argument");
    return guarded("epw_spectral_function", [&]() {
        launch_spectral_function(nk, nb, nw, eps, mu, wgrid, sigma_w, sigma0, A, (hipStream_t)stream);
        return EPW_OK;
    });
}

extern "C" int epw_resigma(const epw_system* sys, const epw_points* pts, const epw_params* par, double* re_shell,
                           double* re_tilde, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    int rc = check_common(sys, pts, par, "epw_resigma");
    if (rc != EPW_OK) return rc;
    if (pts->nk == 0) return EPW_OK;
    if (!re_shell) return fail(EPW_EINVAL, "epw_resigma: NULL output");
    Outputs o;
    o.imsig = re_shell;
    o.re_tilde = re_tilde;
    return planned_forward("epw_resigma", sys, pts, par, Out::RESIGMA, 0, ws, ws_bytes, stream, o);
}

extern "C" int epw_transport_coupling(const epw_system* sys, const epw_points* pts, const epw_params* par,
                                      const double* vectors, double* lam_tr, double* lam, double* pi_im, void* ws,
                                      size_t ws_bytes, void* stream) {
    clear_error();
    int rc = check_common(sys, pts, par, "epw_transport_coupling");
    if (rc != EPW_OK) return rc;
    if (pts->nq == 0) return EPW_OK;
    if (!lam_tr || !vectors) return fail(EPW_EINVAL, "epw_transport_coupling: NULL output or lattice vectors");
    if (pts->nk == 0) return fail(EPW_ESHAPE, "epw_transport_coupling: the k set is empty");
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(vectors[i])) return fail(EPW_EINVAL, "epw_transport_coupling: lattice vectors not finite");
    Outputs o;
    o.pi_im = pi_im;
    o.lam = lam;
    o.lam_tr = lam_tr;
    o.vectors9 = vectors;
    return planned_forward("epw_transport_coupling", sys, pts, par, Out::TRANSPORT, 0, ws, ws_bytes, stream, o);
}

extern "C" int epw_band_velocities(int nb, int nR, const int32_t* R, const int32_t* ndeg, const void* HR,
                                   const double* vectors, int nk, const double* kfrac, double deg_tol, double* eps,
                                   void* U, double* vel, void* stream) {
    clear_error();
    if (nb < 1 || nb > EPW_MAX_NB || nR < 1 || nk < 0)
        return fail(EPW_ESHAPE, "epw_band_velocities: nb = %d, nR = %d, nk = %d", nb, nR, nk);
    if (nk == 0) return EPW_OK;
    if (!R || !ndeg || !HR || !vectors || !kfrac || !eps || !U || !vel)
        return fail(EPW_EINVAL, "epw_band_velocities: NULL argument");
    if (!(deg_tol >= 0.0)) return fail(EPW_EINVAL, "epw_band_velocities: deg_tol must be >= 0");
    return guarded("epw_band_velocities", [&]() {
        launch_interp_eigh(false, false, nb, nR, R, ndeg, (const double*)HR, nk, kfrac, eps, U, (hipStream_t)stream);
        launch_velocities(nb, nR, R, ndeg, HR, vectors, nk, kfrac, eps, U, deg_tol, vel, (hipStream_t)stream);
        return EPW_OK;
    });
}

extern "C" int epw_eliashberg_function(int nq, int nm, const double* omega, const double* lam, double nq_norm,
                                       int nw, const double* wgrid, double sigma, double* a2f, void* stream) {
    clear_error();
    if (nq < 0 || nm < 1 || nm > EPW_MAX_NM || nw < 0)
        return fail(EPW_ESHAPE, "epw_eliashberg_function: nq = %d, nm = %d, nw = %d", nq, nm, nw);
    if (!(sigma > 0.0) || !(nq_norm > 0.0)) return fail(EPW_EINVAL, "epw_eliashberg_function: sigma and nq_norm must be > 0");
    if (nw == 0) return EPW_OK;
    if (!wgrid || !a2f || (nq > 0 && (!omega || !lam))) return fail(EPW_EINVAL, "epw_eliashberg_function: NULL argument");
    return guarded("epw_eliashberg_function", [&]() {
        launch_eliashberg(nq, nm, omega, lam, nq_norm, nw, wgrid, sigma, a2f, (hipStream_t)stream);
        return EPW_OK;
    });
}

extern "C" int epw_ziman_resistivity(int nw, const double* wgrid, const double* a2f_tr, int nT, const double* T,
                                     double* out, void* stream) {
    clear_error();
    if (nw < 0 || nT < 0) return fail(EPW_ESHAPE, "epw_ziman_resistivity: nw = %d, nT = %d", nw, nT);
    if (nT == 0) return EPW_OK;
    if (!T || !out || (nw > 0 && (!wgrid || !a2f_tr))) return fail(EPW_EINVAL, "epw_ziman_resistivity: NULL argument");
    return guarded("epw_ziman_resistivity", [&]() {
        launch_ziman(nw, wgrid, a2f_tr, nT, T, out, (hipStream_t)stream);
        return EPW_OK;
    });
}

extern "C" int epw_phonon_selfenergy(const epw_system* sys, const epw_points* pts, const epw_params* par,
                                     double* pi_im, double* lam, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    int rc = check_common(sys, pts, par, "epw_phonon_selfenergy");
    if (rc != EPW_OK) return rc;
    if (pts->nq == 0) return EPW_OK;
    if (!pi_im) return fail(EPW_EINVAL, "epw_phonon_selfenergy: NULL output");
    if (pts->nk == 0) return fail(EPW_ESHAPE, "epw_phonon_selfenergy: the k set is empty");
    Outputs o;
    o.pi_im = pi_im;
    o.lam = lam;
    return planned_forward("epw_phonon_selfenergy", sys, pts, par, Out::PHONON, 0, ws, ws_bytes, stream, o);
}

extern "C" int epw_imsigma_backward(const epw_system* sys, const epw_points* pts, const epw_params* par,
                                    const double* w, void* dgR, void* dHR, double* domega, void* ws,
                                    size_t ws_bytes, void* stream) {
    clear_error();
    int rc = check_common(sys, pts, par, "epw_imsigma_backward");
    if (rc != EPW_OK) return rc;
    if (pts->nk == 0) return EPW_OK;
    if (!w) return fail(EPW_EINVAL, "epw_imsigma_backward: NULL weights");
    Arena dry;
    dry.dry = true;
    BwdLayout L;
    plan_bwd(sys, pts, par, dry, L);
    if (!ws || ws_bytes < dry.used + 256)
        return fail(EPW_ENOMEM, "epw_imsigma_backward: workspace %zu bytes, need %zu", ws_bytes, dry.used + 256);
    return guarded("epw_imsigma_backward", [&]() {
        Arena A;
        A.base = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
        A.cap = ws_bytes;
        plan_bwd(sys, pts, par, A, L);
        run_backward(sys, pts, par, L, w, dgR, dHR, domega, (hipStream_t)stream);
        return EPW_OK;
    });
}
