// Interpolation of small Hermitian matrices (H(k), D(q)) from real space and
// their float64 eigendecomposition, four points per wavefront.
//
// X(p) = sum_R exp(2 pi i p.R) X(R)/ndeg(R): the phases of a block of R
// vectors are staged in LDS; lanes split the (entry, R) work, partial sums
// are reduced in a fixed order (bit-reproducible).  The matrix is then
// Hermitised and diagonalised by the cyclic complex Jacobi method with the
// round-robin (tournament) ordering: every round applies n/2 disjoint plane
// rotations at once.  The two-sided update J^H A J of a round is block-wise:
// the 2 x 2 block of rows of one pair and columns of another depends only
// on itself, so each lane updates one block in a single step (no barrier
// between the column and the row rotations) and no two lanes touch the same
// entry; only the blocks above the diagonal are computed (A stays exactly
// Hermitian).  The eigenvector matrix V <- V J stays in registers, one row per
// lane: the pairs of each round are compile-time constants, so the rotation
// of a row needs no indexing at run time and only A passes through LDS.
// Jacobi is used because it reaches full float64 accuracy for eigenvalues and
// eigenvectors at these sizes (n <= 16) and maps onto a wave without serial
// Householder steps.
#include <hip/hip_runtime.h>

#include "epw_internal.h"
#include "kernels.h"

#include <utility>

namespace epw {
namespace {

constexpr int MAXN = 16;         // largest matrix
constexpr int RBLK = 256;         // R vectors staged per pass
constexpr int MAX_SWEEPS = 24;

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// pair i of round r of the round-robin schedule on N2 indices (8 or 16):
// index N2 - 1 stays fixed, the others rotate (r < N2 - 1, i < N2 / 2).  A
// matrix of size n <= N2 runs on N2 indices, those at or beyond n being zero
// rows and columns whose pairs are not rotated; a sweep (N2 - 1 rounds) still
// meets every pair of indices below n once.  constexpr: with r and i known at
// compile time the indices are constants, which keeps the rows of V in
// registers.
template <int N2>
__host__ __device__ constexpr int rr_p(int r, int i) {
    const int m = N2 - 1;
    const int a = (r + i) % m;
    const int b = i == 0 ? m : (r - i + m) % m;
    return a < b ? a : b;
}
template <int N2>
__host__ __device__ constexpr int rr_q(int r, int i) {
    const int m = N2 - 1;
    const int a = (r + i) % m;
    const int b = i == 0 ? m : (r - i + m) % m;
    return a < b ? b : a;
}
template <int N2>
__device__ inline void rr_pair(int r, int i, int& p, int& q) {
    const int m = N2 - 1;
    int a = r + i;
    if (a >= m) a -= m;
    int b = r - i + m;
    if (b >= m) b -= m;
    if (i == 0) b = m;
    p = a < b ? a : b;
    q = a < b ? b : a;
}

// 1/x and 1/sqrt(x) for positive normal x: the hardware estimates (relative
// error near 5e-8) refined by two Newton-Raphson steps, each of which squares
// the relative error, so the results are within a few units in the last
// place, like the correctly rounded division and square root they replace
// (which cost several times more issue cycles).
__device__ __forceinline__ double rcp_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsqrt_pos(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);   // y (3 - x y^2) / 2
    return y;
}

// sum over the N2 lanes of one matrix (lanes N2 h .. N2 h + N2 - 1); every
// lane of the group receives the same value
template <int N2>
__device__ inline double group_sum(double v) {
#pragma unroll
    for (int m = N2 / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// V <- V J for round R on one row v of V (registers): the columns (p, q) of
// each pair U, with the pair's parameters rt[U] = {c, s, cos phi, sin phi}.
template <int N2, int R, int U>
__device__ __forceinline__ void vrot_pair(double2 (&v)[N2], const double (*rt)[4]) {
    constexpr int p = rr_p<N2>(R, U), q = rr_q<N2>(R, U);
    const double c = rt[U][0], s = rt[U][1];
    const double2 e = make_double2(rt[U][2], -rt[U][3]);
    const double2 w = cmul(v[q], e);
    const double2 x = v[p];
    v[p] = make_double2(c * x.x - s * w.x, c * x.y - s * w.y);
    v[q] = make_double2(s * x.x + c * w.x, s * x.y + c * w.y);
}
template <int N2, int R, int... U>
__device__ __forceinline__ void vrot_round(double2 (&v)[N2], const double (*rt)[4],
                                           std::integer_sequence<int, U...>) {
    (vrot_pair<N2, R, U>(v, rt), ...);
}
template <int N2, int... R>
__device__ __forceinline__ void vrot(int r, double2 (&v)[N2], const double (*rt)[4],
                                     std::integer_sequence<int, R...>) {
    ((r == R ? vrot_round<N2, R>(v, rt, std::make_integer_sequence<int, N2 / 2>{}) : void()), ...);
}

// 64 / N2 matrices per wave (matrix h of a block is point MPW blockIdx.x + h):
// four on the 16-index schedule (n > 8), eight on the 8-index one.  A is in
// LDS as its upper triangle (entry (i, j), i <= j, at tri(i, j); an entry
// below the diagonal is read and written as the conjugate of its mirror);
// lane N2 h + i holds row i of V of matrix h in registers.  A Jacobi round:
//   - lane NPAIR h + u (32 lanes) computes the rotation of pair u of matrix h
//     and writes the pair's own 2 x 2 diagonal block in closed form
//     (a_pp - t |b|, a_qq + t |b|, exact zeros off the diagonal);
//   - the off-diagonal blocks (pairs P1 < P2; 4 x 28 or 8 x 6) are rotated
//     in APASS passes over the 64 lanes; each block's four entries lie in
//     four distinct places of the triangle that no other block touches;
//   - every lane rotates its row of V by all pairs of the round.
// A matrix that has converged takes identity rotations, which change nothing
// (exactly), so its result does not depend on the other matrices of its wave.
// offset of entry (lo, hi), lo <= hi, in the row-major upper triangle of N2 x N2
template <int N2>
__device__ __forceinline__ int tri(int lo, int hi) {
    return (lo * (2 * N2 - 1 - lo) >> 1) + hi;
}

template <int N2> struct JacobiShape {
    static constexpr int MPW = 64 / N2;
    static constexpr int NPAIR = N2 / 2;
    static constexpr int NBLK = NPAIR * (NPAIR - 1) / 2;
    static constexpr int APASS = (MPW * NBLK + 63) / 64;
    static constexpr int NT = N2 * (N2 + 1) / 2;  // entries of the upper triangle
    static_assert(N2 == 8 || N2 == 16, "schedules on 8 or 16 indices");
    static_assert(MPW * NPAIR == 32, "32 rotation-parameter lanes");
};

// REAL_IN: X(R) is real (dynamical matrix); else complex interleaved.
// SQRT_OUT: write omega = sign(l) sqrt|l| instead of the eigenvalue l.
// Pair mode (pts2 != nullptr): point p is pts[p / npts2] + pts2[p % npts2].
// GIVEN: the matrices are given ([np][n][n] complex at XR), no Fourier sum;
// with PACKED only their upper triangles ([np][n(n+1)/2], rows i with columns
// j >= i in turn), the lower triangle being the conjugate.
template <int N2, bool REAL_IN, bool SQRT_OUT, bool GIVEN = false, bool PACKED = false>
__global__ __launch_bounds__(64, N2 == 16 ? (GIVEN ? 3 : 2) : 4) void interp_eigh_kernel(
    int n, int nR, const int32_t* __restrict__ R, const int32_t* __restrict__ ndeg,
    const double* __restrict__ XR, int np, const double* __restrict__ pts,
    const double* __restrict__ pts2, int npts2,
    double* __restrict__ evals, double2* __restrict__ evecs)
{
    typedef JacobiShape<N2> S;
    constexpr int MPW = S::MPW, NPAIR = S::NPAIR, NBLK = S::NBLK, APASS = S::APASS;
    constexpr int NT = S::NT;
    __shared__ double2 A[MPW][NT];
    __shared__ double2 ph[GIVEN ? 1 : RBLK];
    __shared__ double2 red[GIVEN ? 1 : 64];
    __shared__ double rot[MPW][NPAIR][4];
    __shared__ int rpq[MPW][NPAIR][2];
    __shared__ int rk[MPW][N2];

    const int lane = threadIdx.x;
    const int p0 = blockIdx.x * MPW;
    if (p0 >= np) return;
    const int nmat = min(MPW, np - p0);
    for (int e = lane; e < MPW * NT; e += 64) A[e / NT][e % NT] = make_double2(0.0, 0.0);
    __syncthreads();
    if constexpr (GIVEN) {
        // the given matrices of the block's points -> A[h], one after the other
        for (int h = 0; h < nmat; ++h) {
            const int p = p0 + h;
            if constexpr (PACKED) {
                const double2* X = reinterpret_cast<const double2*>(XR) + (size_t)p * (n * (n + 1) / 2);
                for (int e = lane; e < n * n; e += 64) {
                    const int i = e / n, j = e % n;
                    if (i > j) continue;
                    A[h][tri<N2>(i, j)] = X[i * n - i * (i - 1) / 2 + (j - i)];
                }
            } else {
                // the Hermitian part (X + X^dag) / 2
                const double2* X = reinterpret_cast<const double2*>(XR) + (size_t)p * n * n;
                for (int e = lane; e < n * n; e += 64) {
                    const int i = e / n, j = e % n;
                    if (i > j) continue;
                    const double2 x = X[e], y = X[j * n + i];
                    A[h][tri<N2>(i, j)] = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
                }
            }
        }
    } else {
        // the Fourier sums of the block's points together: every entry of X(R)
        // read from memory feeds all of them.  Point p is pts[p], or the sum
        // pts[p / npts2] + pts2[p % npts2] in pair mode; an absent point (past np)
        // gets zero phases.
        constexpr int EPLMAX = (N2 * N2 + 63) / 64;     // entries per lane, at most
        constexpr int RB = RBLK / MPW;                  // R vectors per staging pass
        const int E = n * n;
        const int P = (E >= 64) ? 1 : 64 / E;           // R partitions per entry
        const int EPL = (E + 63) / 64;                  // entries per lane when P == 1
        double2 acc[EPLMAX][MPW];
#pragma unroll
        for (int j = 0; j < EPLMAX; ++j)
#pragma unroll
            for (int h = 0; h < MPW; ++h) acc[j][h] = make_double2(0.0, 0.0);

        for (int r0 = 0; r0 < nR; r0 += RB) {
            const int cnt = min(RB, nR - r0);
            __syncthreads();
            for (int t = lane; t < MPW * cnt; t += 64) {
                const int h = t / cnt, r = t - h * cnt;
                double2 f = make_double2(0.0, 0.0);
                if (h < nmat) {
                    const size_t pp = (size_t)p0 + h;
                    const size_t ia = pts2 ? pp / npts2 : pp;
                    double k0 = pts[3 * ia + 0];
                    double k1 = pts[3 * ia + 1];
                    double k2 = pts[3 * ia + 2];
                    if (pts2) {
                        const size_t ib = pp % npts2;
                        k0 += pts2[3 * ib + 0];
                        k1 += pts2[3 * ib + 1];
                        k2 += pts2[3 * ib + 2];
                    }
                    const int idx = r0 + r;
                    double x = k0 * (double)R[3 * idx] + k1 * (double)R[3 * idx + 1] +
                               k2 * (double)R[3 * idx + 2];
                    x -= rint(x);
                    double sn, cs;
                    sincospi(2.0 * x, &sn, &cs);
                    const double w = 1.0 / (double)ndeg[idx];
                    f = make_double2(cs * w, sn * w);
                }
                ph[h * RB + r] = f;
            }
            __syncthreads();
            // acc[j][h] += phase(h, R) X_e(R) for the lane's entries e
            auto accumulate = [&](int j, int e, int r) {
                if (REAL_IN) {
                    const double x = XR[(size_t)(r0 + r) * E + e];
#pragma unroll
                    for (int h = 0; h < MPW; ++h) {
                        const double2 f = ph[h * RB + r];
                        acc[j][h].x += f.x * x;
                        acc[j][h].y += f.y * x;
                    }
                } else {
                    const double2 x = reinterpret_cast<const double2*>(XR)[(size_t)(r0 + r) * E + e];
#pragma unroll
                    for (int h = 0; h < MPW; ++h) {
                        const double2 t = cmul(ph[h * RB + r], x);
                        acc[j][h].x += t.x;
                        acc[j][h].y += t.y;
                    }
                }
            };
            if (P > 1) {
                const int e = lane % E, part = lane / E;
                if (part < P)
                    for (int r = part; r < cnt; r += P) accumulate(0, e, r);
            } else {
#pragma unroll
                for (int j = 0; j < EPLMAX; ++j) {
                    const int e = lane + 64 * j;
                    if (j < EPL && e < E)
                        for (int r = 0; r < cnt; ++r) accumulate(j, e, r);
                }
            }
        }
        // point h's raw matrix (the partitions' partial sums added in a fixed
        // order) -> ph as [n][n], then its Hermitian part -> the triangle of A[h]
#pragma unroll
        for (int h = 0; h < MPW; ++h) {
            if (h >= nmat) break;
            __syncthreads();
            if (P > 1) {
                red[lane] = acc[0][h];
                __syncthreads();
                if (lane < E) {
                    double2 sum = make_double2(0.0, 0.0);
                    for (int part = 0; part < P; ++part) {
                        sum.x += red[lane + E * part].x;
                        sum.y += red[lane + E * part].y;
                    }
                    ph[lane] = sum;
                }
            } else {
#pragma unroll
                for (int j = 0; j < EPLMAX; ++j) {
                    const int e = lane + 64 * j;
                    if (j < EPL && e < E) ph[e] = acc[j][h];
                }
            }
            __syncthreads();
            for (int e = lane; e < E; e += 64) {
                const int i = e / n, j = e % n;
                if (i > j) continue;
                const double2 x = ph[e], y = ph[j * n + i];
                A[h][tri<N2>(i, j)] = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
            }
        }
    }
    __syncthreads();

    // row `vr` of V of matrix `vh` in registers
    const int vh = lane / N2, vr = lane % N2;
    double2 v[N2];
#pragma unroll
    for (int j = 0; j < N2; ++j) v[j] = make_double2(j == vr ? 1.0 : 0.0, 0.0);
    // rotation parameters: lane NPAIR ph_h + ph_u, for the 32 lanes below 32
    const int ph_h = lane / NPAIR, ph_u = lane % NPAIR;
    // off-diagonal blocks of the two passes: matrix, pairs (B1 < B2)
    int bh[APASS], b1[APASS], b2[APASS];
    bool bv[APASS];
#pragma unroll
    for (int k = 0; k < APASS; ++k) {
        const int item = lane + 64 * k;
        bv[k] = item < MPW * NBLK;
        bh[k] = item / NBLK;
        int w = item - bh[k] * NBLK;
        b1[k] = 0;
        b2[k] = 0;
        for (int a = 0; a < NPAIR - 1; ++a) {
            const int cnt = NPAIR - 1 - a;
            if (w >= 0 && w < cnt) {
                b1[k] = a;
                b2[k] = a + 1 + w;
            }
            w -= cnt;
        }
    }
    for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
        // convergence of matrix vh: off-diagonal mass against the whole matrix,
        // lane vr summing row vr
        double off = 0.0, dia = 0.0;
        if (vr < n) {
#pragma unroll
            for (int j = 0; j < N2; ++j) {
                if (j >= n) continue;
                const double2 a = A[vh][vr <= j ? tri<N2>(vr, j) : tri<N2>(j, vr)];
                const double m2 = a.x * a.x + a.y * a.y;
                if (j == vr) dia += m2; else off += m2;
            }
        }
        const double so = group_sum<N2>(off), sd = group_sum<N2>(dia);
        const bool done = so <= 1e-30 * (so + sd);   // the same decision in the N2 lanes of a matrix
        const unsigned long long dmask = __ballot(done);
        if (dmask == ~0ull) break;
        const bool ph_done = (dmask >> (N2 * ph_h)) & 1ull;
        // rounds kept rolled: unrolled, their schedules overlap and the registers
        // double (one wave per SIMD); each round picks its V rotation by a branch
#pragma unroll 1
        for (int r = 0; r < N2 - 1; ++r) {
            // rotation of pair ph_u: J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on
            // indices (p, q), which zeroes A[p][q] = |b| e^{i phi} of J^H A J.  A pair
            // with q >= n (zero row and column) and a converged matrix keep J = 1.
            if (lane < MPW * NPAIR) {
                int pp, qq;
                rr_pair<N2>(r, ph_u, pp, qq);
                double c = 1.0, s = 0.0, cph = 1.0, sph = 0.0;
                if (!ph_done && qq < n) {
                    const double app = A[ph_h][tri<N2>(pp, pp)].x, aqq = A[ph_h][tri<N2>(qq, qq)].x;
                    const double2 b = A[ph_h][tri<N2>(pp, qq)];
                    double tb = 0.0;                          // t |b|
                    // b = |b| e^{i phi} with b scaled by max(|Re b|, |Im b|) first, so that the
                    // phase keeps unit modulus down to the smallest normal numbers; a coupling
                    // below 1e-300 is taken as zero (no rotation)
                    const double mb = fmax(fabs(b.x), fabs(b.y));
                    if (mb > 1e-300) {
                        const double im = rcp_pos(mb);
                        const double bx = b.x * im, by = b.y * im;
                        const double nb2 = fma(bx, bx, by * by);
                        const double ir = rsqrt_pos(nb2);
                        cph = bx * ir;
                        sph = by * ir;
                        // tau = (a_qq - a_pp) / (2 |b|); the smaller root t of t^2 + 2 tau t = 1,
                        // t = sign(tau) / (|tau| + sqrt(1 + tau^2)); beyond |tau| = 1e150 the
                        // denominator is 2 |tau| to rounding
                        const double tau = 0.5 * (aqq - app) * im * ir;
                        const double at = fabs(tau);
                        double t;
                        if (at < 1e150) {
                            const double w = fma(at, at, 1.0);
                            t = rcp_pos(at + w * rsqrt_pos(w));
                        } else {
                            t = 0.5 * rcp_pos(at);
                        }
                        if (tau < 0.0) t = -t;
                        c = rsqrt_pos(fma(t, t, 1.0));
                        s = t * c;
                        tb = t * (mb * (nb2 * ir));               // |b| = mb sqrt(nb2)
                    }
                    // the pair's own block after the rotation: a real diagonal, exact zeros
                    // off it
                    A[ph_h][tri<N2>(pp, pp)] = make_double2(app - tb, 0.0);
                    A[ph_h][tri<N2>(qq, qq)] = make_double2(aqq + tb, 0.0);
                    A[ph_h][tri<N2>(pp, qq)] = make_double2(0.0, 0.0);
                }
                rot[ph_h][ph_u][0] = c;
                rot[ph_h][ph_u][1] = s;
                rot[ph_h][ph_u][2] = cph;
                rot[ph_h][ph_u][3] = sph;
                rpq[ph_h][ph_u][0] = pp;
                rpq[ph_h][ph_u][1] = qq;
            }
            __syncthreads();
            // off-diagonal blocks: rows (p1, q1) of pair B1, columns (p2, q2) of pair B2.
            // Columns first: col_p' = c col_p - s e^{-i phi} col_q,
            //                col_q' = s col_p + c e^{-i phi} col_q (pair B2);
            // then rows:     row_p' = c row_p - s e^{i phi} row_q,
            //                row_q' = s row_p + c e^{i phi} row_q (pair B1).
#pragma unroll
            for (int k = 0; k < APASS; ++k) {
                if (!bv[k]) continue;
                const int h = bh[k], B1 = b1[k], B2 = b2[k];
                const int p1 = rpq[h][B1][0], q1 = rpq[h][B1][1], p2 = rpq[h][B2][0], q2 = rpq[h][B2][1];
                const double c1 = rot[h][B1][0], s1 = rot[h][B1][1];
                const double2 e1 = make_double2(rot[h][B1][2], rot[h][B1][3]);
                const double c2 = rot[h][B2][0], s2 = rot[h][B2][1];
                const double2 e2 = make_double2(rot[h][B2][2], -rot[h][B2][3]);
                // the block's entries (row, column): offset in the triangle and whether
                // the entry lies below the diagonal (stored as its mirror's conjugate)
                auto at = [&](int i, int j, int& off) -> bool {
                    const bool low = i > j;
                    off = low ? tri<N2>(j, i) : tri<N2>(i, j);
                    return low;
                };
                auto rd = [&](int off, bool low) -> double2 {
                    const double2 v = A[h][off];
                    return make_double2(v.x, low ? -v.y : v.y);
                };
                auto wr = [&](int off, bool low, double2 v) { A[h][off] = make_double2(v.x, low ? -v.y : v.y); };
                int opp, opq, oqp, oqq;
                const bool lpp = at(p1, p2, opp), lpq = at(p1, q2, opq), lqp = at(q1, p2, oqp), lqq = at(q1, q2, oqq);
                const double2 xpp = rd(opp, lpp), xpq = rd(opq, lpq), xqp = rd(oqp, lqp), xqq = rd(oqq, lqq);
                const double2 wp = cmul(xpq, e2), wq = cmul(xqq, e2);
                const double2 ypp = make_double2(c2 * xpp.x - s2 * wp.x, c2 * xpp.y - s2 * wp.y);
                const double2 ypq = make_double2(s2 * xpp.x + c2 * wp.x, s2 * xpp.y + c2 * wp.y);
                const double2 yqp = make_double2(c2 * xqp.x - s2 * wq.x, c2 * xqp.y - s2 * wq.y);
                const double2 yqq = make_double2(s2 * xqp.x + c2 * wq.x, s2 * xqp.y + c2 * wq.y);
                const double2 up = cmul(yqp, e1), uq = cmul(yqq, e1);
                const double2 zpp = make_double2(c1 * ypp.x - s1 * up.x, c1 * ypp.y - s1 * up.y);
                const double2 zqp = make_double2(s1 * ypp.x + c1 * up.x, s1 * ypp.y + c1 * up.y);
                const double2 zpq = make_double2(c1 * ypq.x - s1 * uq.x, c1 * ypq.y - s1 * uq.y);
                const double2 zqq = make_double2(s1 * ypq.x + c1 * uq.x, s1 * ypq.y + c1 * uq.y);
                wr(opp, lpp, zpp);
                wr(opq, lpq, zpq);
                wr(oqp, lqp, zqp);
                wr(oqq, lqq, zqq);
            }
            // V <- V J on the lane's row (the round's pair indices are constants)
            vrot<N2>(r, v, rot[vh], std::make_integer_sequence<int, N2 - 1>{});
            __syncthreads();
        }
    }
    // ascending order with a stable rank; eigenvector i is column i of V
    if (vr < n) {
        const double li = A[vh][tri<N2>(vr, vr)].x;
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[vh][tri<N2>(j, j)].x;
            rank += (lj < li) || (lj == li && j < vr);
        }
        rk[vh][vr] = rank;
        if (vh < nmat) {
            double out = li;
            if (SQRT_OUT) out = (li < 0.0 ? -1.0 : 1.0) * sqrt(fabs(li));
            evals[((size_t)p0 + vh) * n + rank] = out;
        }
    }
    __syncthreads();
    if (vr < n && vh < nmat) {
        double2* row = evecs + (((size_t)p0 + vh) * n + vr) * n;
#pragma unroll
        for (int j = 0; j < N2; ++j)
            if (j < n) row[rk[vh][j]] = v[j];
    }
}

}  // namespace

// matrices of size n <= 8 run on the 8-index schedule (eight per wave), the
// others on the 16-index one (four per wave); sizes are 1..16 (checked by the
// entry points)
template <int N2>
static void launch_given_t(int n, int np, const void* X, double* evals, void* evecs, hipStream_t stream, bool packed) {
    const dim3 grid((np + JacobiShape<N2>::MPW - 1) / JacobiShape<N2>::MPW), block(64);
    const double* x = reinterpret_cast<const double*>(X);
    double2* ev = reinterpret_cast<double2*>(evecs);
    if (packed)
        interp_eigh_kernel<N2, false, false, true, true><<<grid, block, 0, stream>>>(n, 0, nullptr, nullptr, x, np,
                                                                                    nullptr, nullptr, 1, evals, ev);
    else
        interp_eigh_kernel<N2, false, false, true><<<grid, block, 0, stream>>>(n, 0, nullptr, nullptr, x, np,
                                                                              nullptr, nullptr, 1, evals, ev);
}

void launch_eigh_given(int n, int np, const void* X, double* evals, void* evecs, hipStream_t stream, bool packed) {
    if (np <= 0) return;
    if (n <= 8)
        launch_given_t<8>(n, np, X, evals, evecs, stream, packed);
    else
        launch_given_t<16>(n, np, X, evals, evecs, stream, packed);
    launch_check("interp_eigh_kernel (given)");
}

// neg[r] = index of -R[r] in the set, or -1 when the set has no such vector
__global__ void neg_index_kernel(int nR, const int32_t* __restrict__ R, int32_t* __restrict__ neg) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nR) return;
    const int a = -R[3 * r], b = -R[3 * r + 1], c = -R[3 * r + 2];
    int found = -1;
    for (int t = 0; t < nR; ++t)
        if (R[3 * t] == a && R[3 * t + 1] == b && R[3 * t + 2] == c) {
            found = t;
            break;
        }
    neg[r] = found;
}

// The halved R list of the folded contraction (cfold_mainloop): in order of
// the set, every vector that is not the second member of a pair (R, -R),
// with pair[h] its partner's row, or its own row when it has none (R = 0, a
// vector whose negative is missing, a duplicate); kh[0] = the list's length.
// Entries h >= kh repeat the last member's rows with a zero R (never read by
// the contraction, kept finite for the phase table).  A pair needs neg to
// map each member to the other, so any R list gives an exact fold.  One
// thread: the list is a few thousand vectors at most.
__global__ void half_list_kernel(int nR, const int32_t* __restrict__ R, const int32_t* __restrict__ neg,
                                 int32_t* __restrict__ half, int32_t* __restrict__ pair,
                                 int32_t* __restrict__ R_half, int32_t* __restrict__ kh) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int h = 0;
    for (int e = 0; e < nR; ++e) {
        const int t = neg[e];
        const bool mutual = t >= 0 && t < nR && neg[t] == e;
        if (mutual && t < e) continue;               // second member of a pair
        half[h] = e;
        pair[h] = (mutual && t > e) ? t : e;
        for (int a = 0; a < 3; ++a) R_half[3 * h + a] = R[3 * e + a];
        ++h;
    }
    kh[0] = h;
    for (int j = h; j < nR; ++j) {
        half[j] = h > 0 ? half[h - 1] : 0;
        pair[j] = h > 0 ? pair[h - 1] : 0;
        for (int a = 0; a < 3; ++a) R_half[3 * j + a] = 0;
    }
}

// Upper triangles (rows i with columns j >= i in turn) of the Hermitian part
// of the interpolation: with Phi_R = exp(2 pi i p.R)/ndeg(R) and the set
// closed under R -> -R,
//   ((S + S^dag)/2)_ij = sum_R Phi_R (X_ij(R) + ndeg(R)/ndeg(-R) conj(X_ji(-R)))/2,
// so a sum over these triangles gives the Hermitised matrix exactly, whatever
// X(-R) is.  A vector whose negative is missing makes its entries NaN (the
// triangle cannot represent the sum; the results then show it).
__global__ void pack_upper_kernel(int n, int nR, const double2* __restrict__ X, const int32_t* __restrict__ ndeg,
                                  const int32_t* __restrict__ neg, double2* __restrict__ P) {
    const int nt = n * (n + 1) / 2;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nR * n * n) return;
    const int e = (int)(idx % (n * n));
    const long r = idx / (n * n);
    const int i = e / n, j = e % n;
    if (i > j) return;
    const int t = neg[r];
    double2 v;
    if (t >= 0) {
        const double2 x = X[idx];
        const double2 y = X[(long)t * n * n + j * n + i];
        const double w = (double)ndeg[r] / (double)ndeg[t];
        v = make_double2(0.5 * (x.x + w * y.x), 0.5 * (x.y - w * y.y));
    } else {
        v = make_double2(__builtin_nan(""), __builtin_nan(""));
    }
    P[r * nt + i * n - i * (i - 1) / 2 + (j - i)] = v;
}

void launch_half_list(int nR, const int32_t* R, int32_t* neg, int32_t* half, int32_t* pair, int32_t* R_half,
                      int32_t* kh, hipStream_t stream) {
    if (nR <= 0) return;
    neg_index_kernel<<<dim3((unsigned)((nR + 255) / 256)), dim3(256), 0, stream>>>(nR, R, neg);
    launch_check("neg_index_kernel");
    half_list_kernel<<<dim3(1), dim3(64), 0, stream>>>(nR, R, neg, half, pair, R_half, kh);
    launch_check("half_list_kernel");
}

void launch_pack_upper(int n, int nR, const int32_t* R, const int32_t* ndeg, const void* X, int32_t* neg, void* P,
                       hipStream_t stream) {
    const long total = (long)nR * n * n;
    if (total <= 0) return;
    neg_index_kernel<<<dim3((unsigned)((nR + 255) / 256)), dim3(256), 0, stream>>>(nR, R, neg);
    launch_check("neg_index_kernel");
    pack_upper_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream>>>(
        n, nR, reinterpret_cast<const double2*>(X), ndeg, neg, reinterpret_cast<double2*>(P));
    launch_check("pack_upper_kernel");
}

template <int N2>
static void launch_interp_t(bool real_in, bool sqrt_out, int n, int nR, const int32_t* R, const int32_t* ndeg,
                     const double* XR, int np, const double* pts, double* evals, void* evecs, hipStream_t stream,
                     const double* pts2, int n2) {
    const dim3 grid((np + JacobiShape<N2>::MPW - 1) / JacobiShape<N2>::MPW), block(64);
    double2* ev = reinterpret_cast<double2*>(evecs);
    if (real_in && sqrt_out)
        interp_eigh_kernel<N2, true, true><<<grid, block, 0, stream>>>(n, nR, R, ndeg, XR, np, pts, pts2, n2, evals, ev);
    else if (real_in)
        interp_eigh_kernel<N2, true, false><<<grid, block, 0, stream>>>(n, nR, R, ndeg, XR, np, pts, pts2, n2, evals, ev);
    else if (sqrt_out)
        interp_eigh_kernel<N2, false, true><<<grid, block, 0, stream>>>(n, nR, R, ndeg, XR, np, pts, pts2, n2, evals, ev);
    else
        interp_eigh_kernel<N2, false, false><<<grid, block, 0, stream>>>(n, nR, R, ndeg, XR, np, pts, pts2, n2, evals,
                                                                         ev);
}

void launch_interp_eigh(bool real_in, bool sqrt_out, int n, int nR, const int32_t* R,
                        const int32_t* ndeg, const double* XR, int np, const double* pts,
                        double* evals, void* evecs, hipStream_t stream, const double* pts2, int n2)
{
    if (np <= 0) return;
    if (n <= 8)
        launch_interp_t<8>(real_in, sqrt_out, n, nR, R, ndeg, XR, np, pts, evals, evecs, stream, pts2, n2);
    else
        launch_interp_t<16>(real_in, sqrt_out, n, nR, R, ndeg, XR, np, pts, evals, evecs, stream, pts2, n2);
    launch_check("interp_eigh_kernel");
}

}  // namespace epw
