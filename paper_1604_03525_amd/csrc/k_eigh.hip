// Interpolation of small Hermitian matrices (H(k), D(q)) from real space and
// their float64 eigendecomposition, one wavefront per point.
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
// entry.  Jacobi is used because it reaches full float64 accuracy
// for eigenvalues and eigenvectors at these sizes (n <= 16) and maps onto a
// single wave without serial Householder steps.
#include <hip/hip_runtime.h>

#include "epw_internal.h"
#include "kernels.h"

namespace epw {
namespace {

constexpr int MAXN = 16;
constexpr int LDA = MAXN + 1;     // padded leading dimension in LDS
constexpr int RBLK = 256;         // R vectors staged per pass
constexpr int MAX_SWEEPS = 24;
// work items of the rotation updates are decoded with shifts over the fixed
// MAXN x MAXN layout (no division by the runtime size)
constexpr int LOGN = 4;
static_assert((1 << LOGN) == MAXN, "MAXN is a power of two");

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// pair i of round r of the round-robin schedule on n2 (even) indices:
// index n2 - 1 stays fixed, the others rotate (r < n2 - 1, i < n2 / 2, so
// one conditional subtraction does the reduction mod n2 - 1)
__device__ inline void rr_pair(int n2, int r, int i, int& p, int& q) {
    const int m = n2 - 1;
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

// sum over the 64 lanes of the wave; every lane receives the same value
// (each butterfly step adds the same two operands in every lane)
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// REAL_IN: X(R) is real (dynamical matrix); else complex interleaved.
// SQRT_OUT: write omega = sign(l) sqrt|l| instead of the eigenvalue l.
// Pair mode (pts2 != nullptr): point p is pts[p / npts2] + pts2[p % npts2].
// GIVEN: the matrices are given ([np][n][n] complex at XR), no Fourier sum;
// with PACKED only their upper triangles ([np][n(n+1)/2], rows i with columns
// j >= i in turn), the lower triangle being the conjugate.
template <bool REAL_IN, bool SQRT_OUT, bool GIVEN = false, bool PACKED = false>
__global__ __launch_bounds__(64) void interp_eigh_kernel(
    int n, int nR, const int32_t* __restrict__ R, const int32_t* __restrict__ ndeg,
    const double* __restrict__ XR, int np, const double* __restrict__ pts,
    const double* __restrict__ pts2, int npts2,
    double* __restrict__ evals, double2* __restrict__ evecs)
{
    __shared__ double2 A[MAXN + 1][LDA];
    __shared__ double2 V[MAXN + 1][LDA];
    __shared__ double2 ph[RBLK];
    __shared__ double2 red[64];
    __shared__ double rot[MAXN / 2][4];
    __shared__ int rpq[MAXN / 2][2];

    const int lane = threadIdx.x;
    const int p = blockIdx.x;
    if (p >= np) return;
    if constexpr (GIVEN && PACKED) {
        const double2* X = reinterpret_cast<const double2*>(XR) + (size_t)p * (n * (n + 1) / 2);
        for (int e = lane; e < n * n; e += 64) {
            const int i = e / n, j = e % n;
            if (i > j) continue;
            const double2 x = X[i * n - i * (i - 1) / 2 + (j - i)];
            V[i][j] = x;
            if (i < j) V[j][i] = make_double2(x.x, -x.y);
        }
    } else if constexpr (GIVEN) {
        const double2* X = reinterpret_cast<const double2*>(XR) + (size_t)p * n * n;
        for (int e = lane; e < n * n; e += 64) V[e / n][e % n] = X[e];
    } else {
        // point p, or the sum pts[p / npts2] + pts2[p % npts2] in pair mode
        const size_t ia = pts2 ? (size_t)(p / npts2) : (size_t)p;
        double k0 = pts[3 * ia + 0];
        double k1 = pts[3 * ia + 1];
        double k2 = pts[3 * ia + 2];
        if (pts2) {
            const size_t ib = (size_t)(p % npts2);
            k0 += pts2[3 * ib + 0];
            k1 += pts2[3 * ib + 1];
            k2 += pts2[3 * ib + 2];
        }
        const int E = n * n;
        const int P = (E >= 64) ? 1 : 64 / E;          // R partitions per entry
        const int EPL = (E + 63) / 64;                   // entries per lane when P == 1

        double2 acc[4];
        for (int j = 0; j < 4; ++j) acc[j] = make_double2(0.0, 0.0);

        for (int r0 = 0; r0 < nR; r0 += RBLK) {
            const int cnt = min(RBLK, nR - r0);
            __syncthreads();
            for (int r = lane; r < cnt; r += 64) {
                const int idx = r0 + r;
                double x = k0 * (double)R[3 * idx] + k1 * (double)R[3 * idx + 1] +
                           k2 * (double)R[3 * idx + 2];
                x -= rint(x);
                double s, c;
                sincospi(2.0 * x, &s, &c);
                const double w = 1.0 / (double)ndeg[idx];
                ph[r] = make_double2(c * w, s * w);
            }
            __syncthreads();
            if (P > 1) {
                const int e = lane % E, part = lane / E;
                if (part < P) {
                    for (int r = part; r < cnt; r += P) {
                        const double2 f = ph[r];
                        if (REAL_IN) {
                            const double x = XR[(size_t)(r0 + r) * E + e];
                            acc[0].x += f.x * x;
                            acc[0].y += f.y * x;
                        } else {
                            const double2 x = reinterpret_cast<const double2*>(XR)[(size_t)(r0 + r) * E + e];
                            const double2 t = cmul(f, x);
                            acc[0].x += t.x;
                            acc[0].y += t.y;
                        }
                    }
                }
            } else {
                for (int j = 0; j < EPL; ++j) {
                    const int e = lane + 64 * j;
                    if (e >= E) break;
                    for (int r = 0; r < cnt; ++r) {
                        const double2 f = ph[r];
                        if (REAL_IN) {
                            const double x = XR[(size_t)(r0 + r) * E + e];
                            acc[j].x += f.x * x;
                            acc[j].y += f.y * x;
                        } else {
                            const double2 x = reinterpret_cast<const double2*>(XR)[(size_t)(r0 + r) * E + e];
                            const double2 t = cmul(f, x);
                            acc[j].x += t.x;
                            acc[j].y += t.y;
                        }
                    }
                }
            }
        }
        // raw interpolated matrix -> V (scratch)
        if (P > 1) {
            red[lane] = acc[0];
            __syncthreads();
            if (lane < E) {
                double2 s = make_double2(0.0, 0.0);
                for (int part = 0; part < P; ++part) {
                    s.x += red[lane + E * part].x;
                    s.y += red[lane + E * part].y;
                }
                V[lane / n][lane % n] = s;
            }
        } else {
            for (int j = 0; j < EPL; ++j) {
                const int e = lane + 64 * j;
                if (e < E) V[e / n][e % n] = acc[j];
            }
        }
    }   // Fourier sum
    __syncthreads();
    // Hermitise into A; V <- identity; padding row/column of zeros
    const int n2 = n + (n & 1);
    for (int e = lane; e < n2 * n2; e += 64) {
        const int i = e / n2, j = e % n2;
        double2 a = make_double2(0.0, 0.0);
        if (i < n && j < n) {
            const double2 x = V[i][j], y = V[j][i];
            a = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
        }
        A[i][j] = a;
    }
    __syncthreads();
    for (int e = lane; e < n2 * n2; e += 64) {
        const int i = e / n2, j = e % n2;
        V[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();

    const int npair = n2 / 2;
    for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
        // convergence: off-diagonal mass against the whole matrix
        double off = 0.0, dia = 0.0;
        for (int e = lane; e < MAXN * MAXN; e += 64) {
            const int i = e >> LOGN, j = e & (MAXN - 1);
            if (i >= n || j >= n) continue;
            const double2 a = A[i][j];
            const double m2 = a.x * a.x + a.y * a.y;
            if (i == j) dia += m2; else off += m2;
        }
        const double so = wave_sum(off), sd = wave_sum(dia);
        if (so <= 1e-30 * (so + sd)) break;   // the same decision in every lane
        for (int r = 0; r < n2 - 1; ++r) {
            // rotation of pair `lane`: J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on
            // indices (p, q), which zeroes A[p][q] = |b| e^{i phi} of J^H A J.
            // An inactive pair (q is the padding index of odd n) keeps J = 1.
            if (lane < npair) {
                int pp, qq;
                rr_pair(n2, r, lane, pp, qq);
                double c = 1.0, s = 0.0, cph = 1.0, sph = 0.0;
                if (qq < n) {
                    const double app = A[pp][pp].x, aqq = A[qq][qq].x;
                    const double2 b = A[pp][qq];
                    // b = |b| e^{i phi} with b scaled by max(|Re b|, |Im b|) first, so that the
                    // phase keeps unit modulus down to the smallest normal numbers; a coupling
                    // below 1e-300 is taken as zero (no rotation)
                    const double mb = fmax(fabs(b.x), fabs(b.y));
                    if (mb > 1e-300) {
                        const double im = rcp_pos(mb);
                        const double bx = b.x * im, by = b.y * im;
                        const double ir = rsqrt_pos(fma(bx, bx, by * by));
                        cph = bx * ir;
                        sph = by * ir;
                        // tau = (a_qq - a_pp) / (2 |b|); the smaller root t of t^2 + 2 tau t = 1,
                        // t = sign(tau) / (|tau| + sqrt(1 + tau^2)); beyond |tau| = 1e150 the
                        // denominator is 2 |tau| to rounding
                        const double tau = 0.5 * (aqq - app) * im * ir;
                        const double at = fabs(tau);
                        double t;
                        if (at < 1e150) {
                            const double u = fma(at, at, 1.0);
                            t = rcp_pos(at + u * rsqrt_pos(u));
                        } else {
                            t = 0.5 * rcp_pos(at);
                        }
                        if (tau < 0.0) t = -t;
                        c = rsqrt_pos(fma(t, t, 1.0));
                        s = t * c;
                    }
                }
                rot[lane][0] = c;
                rot[lane][1] = s;
                rot[lane][2] = cph;
                rot[lane][3] = sph;
                rpq[lane][0] = pp;
                rpq[lane][1] = qq;
            }
            __syncthreads();
            // A <- J^H A J in one step: lane (P1, P2) owns the 2 x 2 block of rows
            // (p1, q1) and columns (p2, q2), which depends on no other block.
            // Columns first: col_p' = c col_p - s e^{-i phi} col_q,
            //                col_q' = s col_p + c e^{-i phi} col_q (pair P2);
            // then rows:     row_p' = c row_p - s e^{i phi} row_q,
            //                row_q' = s row_p + c e^{i phi} row_q (pair P1).
            // The same lane applies the column rotation of pair P2 to rows 2 P1 and
            // 2 P1 + 1 of V (V <- V J), reusing the parameters it already holds;
            // with 2 npair = n2 >= n those rows cover every row of V.
            {
                const int P1 = lane >> (LOGN - 1), P2 = lane & (MAXN / 2 - 1);
                if (P1 < npair && P2 < npair) {
                    const int p1 = rpq[P1][0], q1 = rpq[P1][1], p2 = rpq[P2][0], q2 = rpq[P2][1];
                    const double c1 = rot[P1][0], s1 = rot[P1][1];
                    const double2 e1 = make_double2(rot[P1][2], rot[P1][3]);
                    const double c2 = rot[P2][0], s2 = rot[P2][1];
                    const double2 e2 = make_double2(rot[P2][2], -rot[P2][3]);
                    const double2 xpp = A[p1][p2], xpq = A[p1][q2], xqp = A[q1][p2], xqq = A[q1][q2];
                    const int i1 = 2 * P1, i2 = 2 * P1 + 1;
                    const double2 v1p = V[i1][p2], v1q = V[i1][q2], v2p = V[i2][p2], v2q = V[i2][q2];
                    // columns (pair P2) on rows p1 and q1
                    const double2 wp = cmul(xpq, e2), wq = cmul(xqq, e2);
                    const double2 ypp = make_double2(c2 * xpp.x - s2 * wp.x, c2 * xpp.y - s2 * wp.y);
                    const double2 ypq = make_double2(s2 * xpp.x + c2 * wp.x, s2 * xpp.y + c2 * wp.y);
                    const double2 yqp = make_double2(c2 * xqp.x - s2 * wq.x, c2 * xqp.y - s2 * wq.y);
                    const double2 yqq = make_double2(s2 * xqp.x + c2 * wq.x, s2 * xqp.y + c2 * wq.y);
                    // rows (pair P1) on columns p2 and q2
                    const double2 up = cmul(yqp, e1), uq = cmul(yqq, e1);
                    double2 zpp = make_double2(c1 * ypp.x - s1 * up.x, c1 * ypp.y - s1 * up.y);
                    double2 zqp = make_double2(s1 * ypp.x + c1 * up.x, s1 * ypp.y + c1 * up.y);
                    double2 zpq = make_double2(c1 * ypq.x - s1 * uq.x, c1 * ypq.y - s1 * uq.y);
                    double2 zqq = make_double2(s1 * ypq.x + c1 * uq.x, s1 * ypq.y + c1 * uq.y);
                    if (P1 == P2 && q1 < n) {
                        // the rotated pair: exact zeros off the diagonal, a real diagonal
                        zpq = make_double2(0.0, 0.0);
                        zqp = make_double2(0.0, 0.0);
                        zpp.y = 0.0;
                        zqq.y = 0.0;
                    }
                    A[p1][p2] = zpp;
                    A[p1][q2] = zpq;
                    A[q1][p2] = zqp;
                    A[q1][q2] = zqq;
                    // V: columns (pair P2) on rows i1 and i2 (an inactive pair has J = 1)
                    const double2 w1 = cmul(v1q, e2), w2 = cmul(v2q, e2);
                    V[i1][p2] = make_double2(c2 * v1p.x - s2 * w1.x, c2 * v1p.y - s2 * w1.y);
                    V[i1][q2] = make_double2(s2 * v1p.x + c2 * w1.x, s2 * v1p.y + c2 * w1.y);
                    V[i2][p2] = make_double2(c2 * v2p.x - s2 * w2.x, c2 * v2p.y - s2 * w2.y);
                    V[i2][q2] = make_double2(s2 * v2p.x + c2 * w2.x, s2 * v2p.y + c2 * w2.y);
                }
            }
            __syncthreads();
        }
    }
    // ascending order with a stable rank; eigenvector i is column i of V
    if (lane < n) {
        const double li = A[lane][lane].x;
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[j][j].x;
            rank += (lj < li) || (lj == li && j < lane);
        }
        double out = li;
        if (SQRT_OUT) out = (li < 0.0 ? -1.0 : 1.0) * sqrt(fabs(li));
        evals[(size_t)p * n + rank] = out;
        for (int row = 0; row < n; ++row)
            evecs[((size_t)p * n + row) * n + rank] = V[row][lane];
    }
}

}  // namespace

void launch_eigh_given(int n, int np, const void* X, double* evals, void* evecs, hipStream_t stream, bool packed) {
    if (np <= 0) return;
    if (packed)
        interp_eigh_kernel<false, false, true, true><<<dim3(np), dim3(64), 0, stream>>>(
            n, 0, nullptr, nullptr, reinterpret_cast<const double*>(X), np, nullptr, nullptr, 1, evals,
            reinterpret_cast<double2*>(evecs));
    else
        interp_eigh_kernel<false, false, true><<<dim3(np), dim3(64), 0, stream>>>(
            n, 0, nullptr, nullptr, reinterpret_cast<const double*>(X), np, nullptr, nullptr, 1, evals,
            reinterpret_cast<double2*>(evecs));
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

void launch_interp_eigh(bool real_in, bool sqrt_out, int n, int nR, const int32_t* R,
                        const int32_t* ndeg, const double* XR, int np, const double* pts,
                        double* evals, void* evecs, hipStream_t stream, const double* pts2, int n2)
{
    if (np <= 0) return;
    dim3 grid(np), block(64);
    double2* ev = reinterpret_cast<double2*>(evecs);
    if (real_in && sqrt_out)
        interp_eigh_kernel<true, true><<<grid, block, 0, stream>>>(n, nR, R, ndeg, XR, np, pts, pts2, n2, evals, ev);
    else if (real_in)
        interp_eigh_kernel<true, false><<<grid, block, 0, stream>>>(n, nR, R, ndeg, XR, np, pts, pts2, n2, evals, ev);
    else if (sqrt_out)
        interp_eigh_kernel<false, true><<<grid, block, 0, stream>>>(n, nR, R, ndeg, XR, np, pts, pts2, n2, evals, ev);
    else
        interp_eigh_kernel<false, false><<<grid, block, 0, stream>>>(n, nR, R, ndeg, XR, np, pts, pts2, n2, evals, ev);
    launch_check("interp_eigh_kernel");
}

}  // namespace epw
