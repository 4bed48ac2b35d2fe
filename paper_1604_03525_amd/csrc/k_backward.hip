// Adjoint of L = sum_nk w_nk Im Sigma_nk (Sec. 3 Eq. (8)) with respect to
// g(R_e,R_p), H(R_e) and omega_q,nu; the k+q states are members of the k set
// (grid runs) or per pair (off-grid runs).
//
// Per (k, q) pair and mode nu, with X = g_nu(k,q) in the Wannier basis
// (recomputed by the R_e -> k GEMM), T = X U_k, g' = U_{k+q}^dag T:
//   gbar'_mn   = 2 C wbar_n W_mn g'_mn                (C = pi/(N_q sigma sqrt pi))
//   Y          = U_{k+q} gbar'
//   Gbar       = Y U_k^dag                              -> R_e <- k contraction
//   Ubar_k    += X^dag Y,   Ubar_{k+q} += T gbar'^dag
//   epsbar_nk += C wbar_n sum |g'|^2 dW/dx,   x = eps_nk - eps_m,k+q
//   epsbar_m,k+q += C wbar_n |g'|^2 (-dW/dx + (e1 - e2) f'(eps_m,k+q))
//   omegabar  += C wbar_n |g'|^2 (dW/domega - W/omega)  (the last term is the
//                 1/sqrt(2 omega) of Eq. (2), the partial at fixed e_q)
// where W = (n+f) e1 + (n+1-f) e2, e1,2 = exp(-((x +- omega)/sigma)^2).
// Contributions are written per (k, q) and summed afterwards in a fixed
// order, so the adjoint is bit-reproducible like the forward.
#include <hip/hip_runtime.h>

#include "epw_internal.h"
#include "kernels.h"

#include <type_traits>

namespace epw {
namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {   // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cmul_bc(double2 a, double2 b) {  // a * conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

template <typename CT> __device__ inline double2 to_d2(CT v) { return make_double2((double)v.x, (double)v.y); }
template <typename CT> __device__ inline CT from_d2(double2 v);
template <> __device__ inline double2 from_d2<double2>(double2 v) { return v; }
template <> __device__ inline float2 from_d2<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }

// One block per (k, q) pair; thread e owns matrix element (e / P, e % P) of
// every per-pair matrix (P = padded band count: 64 threads for P <= 8, one
// wave, or P^2 = 256 for P = 16).  The per-pair matrices live in LDS; the
// accumulated adjoints of U_k and U_k+q stay in the registers of the element's
// thread, and the sums over a row or a column of the band-pair weights are
// lane butterflies inside the wave (LDS tree sums for P = 16), so no thread
// walks a row of LDS values one dependent load at a time.
template <int P> __device__ inline double sum_rows_of_column(double v) {   // over e / P, same e % P
#pragma unroll
    for (int m = P; m < P * P; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}
template <int P> __device__ inline double sum_columns_of_row(double v) {   // over e % P, same e / P
#pragma unroll
    for (int m = 1; m < P; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}
template <int P> __device__ inline double sum_all(double v) {
#pragma unroll
    for (int m = 1; m < P * P; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <typename CT, int P>
__global__ __launch_bounds__(P * P > 64 ? P * P : 64) void pair_bwd_kernel(PairBwdArgs a)
{
    constexpr bool WAVE = P * P <= 64;             // every element in one wave
    __shared__ double2 Uk[P][P + 1];
    __shared__ double2 Uq[P][P + 1];
    __shared__ double2 X[P][P + 1];
    __shared__ double2 Tm[P][P + 1];
    __shared__ double2 gb[P][P + 1];
    __shared__ double2 Y[P][P + 1];
    __shared__ double red[WAVE ? 1 : 3][P][P + 1];  // row / column / total sums (P = 16)

    const int lane = threadIdx.x;
    const int r = lane / P, c = lane % P;
    const int ql = blockIdx.x;
    const int k = blockIdx.y;
    const int nb = a.nb, nm = a.nm, nbp = a.nbp;
    const int nb2 = nb * nb;
    const bool act = lane < P * P;                        // lanes beyond P^2 (P < 8) hold no element
    const bool el = act && r < nb && c < nb;              // a true element (not padding)
    const int q = a.q0 + ql;
    const size_t pair = (size_t)k * a.qc + ql;
    const double2* U = reinterpret_cast<const double2*>(a.U);
    // states at k+q: a member of the k set (grid runs) or per pair
    const int kq = a.kq ? a.kq[(size_t)k * a.nq_total + q] : 0;
    const bool valid = a.kq ? (unsigned)kq < (unsigned)a.nk : true;
    const double2* Uqs = a.kq ? U + (size_t)kq * nb * nb : reinterpret_cast<const double2*>(a.U_pair) + pair * nb * nb;
    const double* eqs = a.kq ? a.eps + (size_t)kq * nb : a.eps_pair + pair * nb;
    const double* fqs = a.kq ? a.ftab + (size_t)kq * nb : a.f_pair + pair * nb;
    CT* G = reinterpret_cast<CT*>(a.G);
    const size_t ncols = (size_t)a.qc * nm * nbp * nbp;
    const double2 zero = make_double2(0.0, 0.0);

    if (act) {
        Uk[r][c] = (el && valid) ? U[((size_t)k * nb + r) * nb + c] : zero;
        Uq[r][c] = (el && valid) ? Uqs[r * nb + c] : zero;
    }
    // this thread's band energies and occupation (element (m, n) = (r, c))
    const double en = el ? a.eps[(size_t)k * nb + c] : 0.0;
    const double em = el && valid ? eqs[r] : 0.0;
    const double f = el && valid ? fqs[r] : 0.0;
    const double wb = el ? a.wbar[(size_t)k * nb + c] : 0.0;
    const double fp = a.kT > 0.0 ? -f * (1.0 - f) / a.kT : 0.0;
    double2 ukA = zero, uqA = zero;       // dL/dU_k[r][c], dL/dU_k+q[r][c]
    double ekA = 0.0, eqA = 0.0;          // dL/deps_k[c] (held where r == 0), dL/deps_k+q[r] (where c == 0)
    __syncthreads();
    const double inv_s2 = 1.0 / (a.sigma * a.sigma);
    for (int nu = 0; nu < nm; ++nu) {
        CT* Gb = G + (size_t)k * ncols + ((size_t)ql * nm + nu) * nbp * nbp;
        const double scv = a.sc[(size_t)ql * nm + nu];
        if (!valid || scv == 0.0) {
            // no contribution: the adjoint of this block is zero
            if (el) Gb[r * nbp + c] = from_d2<CT>(zero);
            if (lane == 0) a.om_c[pair * nm + nu] = 0.0;
            continue;
        }
        if (act) X[r][c] = el ? to_d2(Gb[r * nbp + c]) : zero;
        __syncthreads();
        double2 t = zero;                  // T = X U_k
#pragma unroll
        for (int j = 0; j < P; ++j) {
            if (!act) break;
            const double2 p = cmul(X[r][j], Uk[j][c]);
            t.x += p.x;
            t.y += p.y;
        }
        if (act) Tm[r][c] = t;
        __syncthreads();
        const double w = a.omega[(size_t)ql * nm + nu];
        const double nB = a.nbose[(size_t)ql * nm + nu];
        const double dnB = a.kT > 0.0 ? -nB * (nB + 1.0) / a.kT : 0.0;
        double2 g = zero;                  // g' = U_kq^dag T, element (m, n) = (r, c)
#pragma unroll
        for (int i = 0; i < P; ++i) {
            if (!act) break;
            const double2 p = cmulc(Uq[i][r], Tm[i][c]);
            g.x += p.x;
            g.y += p.y;
        }
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        double2 gbv = zero;
        if (el) {
            const double x = en - em;
            const double e1 = exp(-(x + w) * (x + w) * inv_s2);
            const double e2 = exp(-(x - w) * (x - w) * inv_s2);
            const double A1 = nB + f, A2 = nB + 1.0 - f;
            const double Wv = A1 * e1 + A2 * e2;
            const double dWdx = -2.0 * inv_s2 * (A1 * (x + w) * e1 + A2 * (x - w) * e2);
            const double dWdw = dnB * (e1 + e2) - 2.0 * inv_s2 * (A1 * (x + w) * e1 - A2 * (x - w) * e2);
            const double cw = a.C * wb;
            const double amp = g.x * g.x + g.y * g.y;
            gbv = make_double2(2.0 * cw * Wv * g.x, 2.0 * cw * Wv * g.y);
            s1 = cw * amp * dWdx;
            s2 = cw * amp * (-dWdx + (e1 - e2) * fp);
            s3 = cw * amp * (dWdw - Wv / w);
        }
        if (act) gb[r][c] = gbv;
        // eps_k[n] gets the column sums over m, eps_k+q[m] the row sums over n,
        // omega the total (fixed order: lane butterflies, or LDS sums for P = 16)
        double colsum, rowsum, total;
        if constexpr (WAVE) {
            colsum = sum_rows_of_column<P>(s1);
            rowsum = sum_columns_of_row<P>(s2);
            total = sum_all<P>(s3);
        } else {
            red[0][r][c] = s1;
            red[1][r][c] = s2;
            red[2][r][c] = s3;
        }
        __syncthreads();
        if constexpr (!WAVE) {
            colsum = 0.0;
            rowsum = 0.0;
            total = 0.0;
            if (r == 0) {
                for (int m = 0; m < P; ++m) colsum += red[0][m][c];
            }
            if (c == 0) {
                for (int n = 0; n < P; ++n) rowsum += red[1][r][n];
                red[2][r][P] = 0.0;
                double t3 = 0.0;
                for (int n = 0; n < P; ++n) t3 += red[2][r][n];
                red[2][r][P] = t3;
            }
        }
        if (r == 0) ekA += colsum;
        if (c == 0) eqA += rowsum;
        double2 y = zero, u = zero;        // Y = U_kq gbar'; dL/dU_kq += T gbar'^dag
#pragma unroll
        for (int m = 0; m < P; ++m) {
            if (!act) break;
            const double2 p = cmul(Uq[r][m], gb[m][c]);
            y.x += p.x;
            y.y += p.y;
        }
#pragma unroll
        for (int n = 0; n < P; ++n) {
            if (!act) break;
            const double2 p = cmul_bc(Tm[r][n], gb[c][n]);
            u.x += p.x;
            u.y += p.y;
        }
        uqA.x += u.x;
        uqA.y += u.y;
        if (act) Y[r][c] = y;
        __syncthreads();
        if constexpr (!WAVE) {
            if (lane == 0) {
                for (int m = 0; m < P; ++m) total += red[2][m][P];
            }
        }
        if (lane == 0) a.om_c[pair * nm + nu] = total;
        double2 uk = zero, gbar = zero;    // dL/dU_k += X^dag Y; Gbar = Y U_k^dag
#pragma unroll
        for (int i = 0; i < P; ++i) {
            if (!act) break;
            const double2 p = cmulc(X[i][r], Y[i][c]);
            uk.x += p.x;
            uk.y += p.y;
        }
#pragma unroll
        for (int n = 0; n < P; ++n) {
            if (!act) break;
            const double2 p = cmul_bc(Y[r][n], Uk[c][n]);
            gbar.x += p.x;
            gbar.y += p.y;
        }
        ukA.x += uk.x;
        ukA.y += uk.y;
        if (el) Gb[r * nbp + c] = from_d2<CT>(gbar);
        __syncthreads();                   // X, Tm, gb, Y are rewritten by the next mode
    }
    double2* Ukc = reinterpret_cast<double2*>(a.Uk_c);
    double2* Uqc = reinterpret_cast<double2*>(a.Ukq_c);
    if (el) {
        Ukc[pair * nb2 + r * nb + c] = ukA;
        Uqc[pair * nb2 + r * nb + c] = uqA;
    }
    if (r == 0 && c < nb) a.ek_c[pair * nb + c] = ekA;
    if (c == 0 && r < nb) a.ekq_c[pair * nb + r] = eqA;
}

__global__ void fill_i32_kernel(size_t n, int32_t v, int32_t* p) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_f64_kernel(size_t n, double v, double* p) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void kq_inverse_kernel(int nk, int qc, int q0, int nq_total, const int32_t* __restrict__ kq,
                                  int32_t* __restrict__ inv) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nk * qc) return;
    const int k = (int)(idx / qc), j = (int)(idx % qc);
    const int t = kq[(size_t)k * nq_total + q0 + j];
    if ((unsigned)t < (unsigned)nk) inv[(size_t)t * qc + j] = k;
}

__global__ void gather_state_adjoint_kernel(int nk, int nb, int qc, const int32_t* __restrict__ inv,
                                            const double* __restrict__ ek_c, const double2* __restrict__ Uk_c,
                                            const double* __restrict__ ekq_c, const double2* __restrict__ Ukq_c,
                                            double* __restrict__ ebar, double2* __restrict__ Ubar) {
    const int per = nb + nb * nb;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nk * per) return;
    const int k = (int)(idx / per), e = (int)(idx % per);
    if (e < nb) {
        double s = 0.0;
        for (int j = 0; j < qc; ++j) {
            s += ek_c[((size_t)k * qc + j) * nb + e];
            const int src = inv ? inv[(size_t)k * qc + j] : -1;
            if (src >= 0) s += ekq_c[((size_t)src * qc + j) * nb + e];
        }
        ebar[(size_t)k * nb + e] += s;
    } else {
        const int f = e - nb, nb2 = nb * nb;
        double2 s = make_double2(0.0, 0.0);
        for (int j = 0; j < qc; ++j) {
            const double2 v = Uk_c[((size_t)k * qc + j) * nb2 + f];
            s.x += v.x;
            s.y += v.y;
            const int src = inv ? inv[(size_t)k * qc + j] : -1;
            if (src >= 0) {
                const double2 u = Ukq_c[((size_t)src * qc + j) * nb2 + f];
                s.x += u.x;
                s.y += u.y;
            }
        }
        double2& o = Ubar[(size_t)k * nb2 + f];
        o.x += s.x;
        o.y += s.y;
    }
}

// one block per (q, nu): 256-way split over k, then a fixed-order tree
__global__ __launch_bounds__(256) void reduce_omega_kernel(int nk, int qc, int nm, const double* __restrict__ om_c,
                                                           int accumulate, double* __restrict__ out) {
    __shared__ double red[256];
    const int qv = blockIdx.x;          // q * nm + nu
    double s = 0.0;
    for (int k = threadIdx.x; k < nk; k += 256) s += om_c[(size_t)k * qc * nm + qv];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[qv] = (accumulate ? out[qv] : 0.0) + red[0];
}

template <typename CT>
__global__ void mode_rotate_adjoint_kernel(int ne, int nq, int nm, int nb, int nbp, const CT* __restrict__ gnu,
                                           const double2* __restrict__ evec, const double* __restrict__ sc,
                                           CT* __restrict__ ga) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nb2 = nb * nb;
    if (idx >= (size_t)ne * nq * nb2) return;
    const int ij = (int)(idx % nb2);
    const size_t eq = idx / nb2;
    const int q = (int)(eq % nq);
    const int i = ij / nb, j = ij % nb;
    const CT* src = gnu + eq * (size_t)nm * nbp * nbp + i * nbp + j;
    for (int aa = 0; aa < nm; ++aa) {
        double re = 0.0, im = 0.0;
        for (int v = 0; v < nm; ++v) {
            const double s = sc[(size_t)q * nm + v];
            if (s == 0.0) continue;
            const double2 ev = evec[((size_t)q * nm + aa) * nm + v];
            const CT g = src[(size_t)v * nbp * nbp];
            // conj(ev) * g * s
            re += s * (ev.x * (double)g.x + ev.y * (double)g.y);
            im += s * (ev.x * (double)g.y - ev.y * (double)g.x);
        }
        CT o;
        o.x = re;
        o.y = im;
        ga[(eq * nm + aa) * nb2 + ij] = o;
    }
}

// one 64-thread block per k (runs once per call: sized for the largest band count)
constexpr int PMAX = 16;
__global__ __launch_bounds__(64) void eigh_adjoint_kernel(int nk, int nb, const double* __restrict__ eps,
                                                          const double2* __restrict__ U,
                                                          const double* __restrict__ ebar,
                                                          const double2* __restrict__ Ubar, double tol,
                                                          double2* __restrict__ Xbar) {
    __shared__ double2 Us[PMAX][PMAX + 1], Ub[PMAX][PMAX + 1], M[PMAX][PMAX + 1], H[PMAX][PMAX + 1];
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    const int nb2 = nb * nb;
    for (int e = lane; e < nb2; e += 64) {
        Us[e / nb][e % nb] = U[(size_t)k * nb2 + e];
        Ub[e / nb][e % nb] = Ubar[(size_t)k * nb2 + e];
    }
    __syncthreads();
    for (int e = lane; e < nb2; e += 64) {   // M = F o (U^dag Ubar) + diag(ebar)
        const int i = e / nb, j = e % nb;
        double2 z = make_double2(0.0, 0.0);
        for (int r = 0; r < nb; ++r) {
            const double2 p = cmulc(Us[r][i], Ub[r][j]);
            z.x += p.x;
            z.y += p.y;
        }
        double2 m = make_double2(0.0, 0.0);
        if (i == j) {
            m.x = ebar[(size_t)k * nb + i];
        } else {
            const double d = eps[(size_t)k * nb + j] - eps[(size_t)k * nb + i];
            if (fabs(d) >= tol && d != 0.0) m = make_double2(z.x / d, z.y / d);
        }
        M[i][j] = m;
    }
    __syncthreads();
    for (int e = lane; e < nb2; e += 64) {   // H = U M
        const int i = e / nb, j = e % nb;
        double2 h = make_double2(0.0, 0.0);
        for (int r = 0; r < nb; ++r) {
            const double2 p = cmul(Us[i][r], M[r][j]);
            h.x += p.x;
            h.y += p.y;
        }
        H[i][j] = h;
    }
    __syncthreads();
    for (int e = lane; e < nb2; e += 64) {   // Hbar = H U^dag; Xbar = (Hbar + Hbar^dag)/2
        const int i = e / nb, j = e % nb;
        double2 h1 = make_double2(0.0, 0.0), h2 = make_double2(0.0, 0.0);
        for (int r = 0; r < nb; ++r) {
            const double2 p = cmul_bc(H[i][r], Us[j][r]);   // (H U^dag)_ij
            const double2 t = cmul_bc(H[j][r], Us[i][r]);   // (H U^dag)_ji
            h1.x += p.x;
            h1.y += p.y;
            h2.x += t.x;
            h2.y += t.y;
        }
        Xbar[(size_t)k * nb2 + e] = make_double2(0.5 * (h1.x + h2.x), 0.5 * (h1.y - h2.y));
    }
}

__global__ void add_f64_kernel(size_t n, const double* __restrict__ src, double* __restrict__ dst) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] += src[i];
}

__global__ void c64_to_c128_kernel(size_t n, const float2* __restrict__ in, int acc, double2* __restrict__ out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 v = make_double2((double)in[i].x, (double)in[i].y);
    if (acc) {
        v.x += out[i].x;
        v.y += out[i].y;
    }
    out[i] = v;
}

inline unsigned nblk(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_pair_bwd(Prec prec, const PairBwdArgs& a, hipStream_t stream) {
    if (a.nk == 0 || a.qc == 0) return;
    dim3 grid((unsigned)a.qc, (unsigned)a.nk);
    auto go = [&](auto tag) {
        constexpr int P = decltype(tag)::value;
        if (prec == Prec::F64)
            pair_bwd_kernel<double2, P><<<grid, P * P > 64 ? P * P : 64, 0, stream>>>(a);
        else
            pair_bwd_kernel<float2, P><<<grid, P * P > 64 ? P * P : 64, 0, stream>>>(a);
    };
    switch (a.nbp) {
        case 1: go(std::integral_constant<int, 1>()); break;
        case 2: go(std::integral_constant<int, 2>()); break;
        case 4: go(std::integral_constant<int, 4>()); break;
        case 8: go(std::integral_constant<int, 8>()); break;
        default: go(std::integral_constant<int, 16>()); break;
    }
    launch_check("pair_bwd_kernel");
}

void launch_kq_inverse(int nk, int qc, int q0, int nq_total, const int32_t* kq, int32_t* inv, hipStream_t stream) {
    const size_t n = (size_t)nk * qc;
    if (n == 0) return;
    fill_i32_kernel<<<nblk(n, 256), 256, 0, stream>>>(n, -1, inv);
    kq_inverse_kernel<<<nblk(n, 256), 256, 0, stream>>>(nk, qc, q0, nq_total, kq, inv);
    launch_check("kq_inverse_kernel");
}

void launch_gather_state_adjoint(int nk, int nb, int qc, const int32_t* inv, const double* ek_c, const void* Uk_c,
                                 const double* ekq_c, const void* Ukq_c, double* ebar, void* Ubar,
                                 hipStream_t stream) {
    const size_t n = (size_t)nk * (nb + nb * nb);
    if (n == 0 || qc == 0) return;
    gather_state_adjoint_kernel<<<nblk(n, 128), 128, 0, stream>>>(nk, nb, qc, inv, ek_c, (const double2*)Uk_c, ekq_c,
                                                                  (const double2*)Ukq_c, ebar, (double2*)Ubar);
    launch_check("gather_state_adjoint_kernel");
}

void launch_reduce_omega(int nk, int qc, int nm, const double* om_c, int accumulate, double* domega,
                         hipStream_t stream) {
    if (qc * nm == 0) return;
    reduce_omega_kernel<<<qc * nm, 256, 0, stream>>>(nk, qc, nm, om_c, accumulate, domega);
    launch_check("reduce_omega_kernel");
}

void launch_mode_rotate_adjoint(Prec prec, int ne, int nq, int nm, int nb, int nbp, const void* gnu,
                                const void* evec, const double* sc, void* ga, hipStream_t stream) {
    const size_t n = (size_t)ne * nq * nb * nb;
    if (n == 0) return;
    if (prec == Prec::F64)
        mode_rotate_adjoint_kernel<double2><<<nblk(n, 256), 256, 0, stream>>>(
            ne, nq, nm, nb, nbp, (const double2*)gnu, (const double2*)evec, sc, (double2*)ga);
    else
        mode_rotate_adjoint_kernel<float2><<<nblk(n, 256), 256, 0, stream>>>(
            ne, nq, nm, nb, nbp, (const float2*)gnu, (const double2*)evec, sc, (float2*)ga);
    launch_check("mode_rotate_adjoint_kernel");
}

void launch_eigh_adjoint(int nk, int nb, const double* eps, const void* U, const double* ebar, const void* Ubar,
                         double deg_tol, void* Xbar, hipStream_t stream) {
    if (nk == 0) return;
    eigh_adjoint_kernel<<<nk, 64, 0, stream>>>(nk, nb, eps, (const double2*)U, ebar, (const double2*)Ubar, deg_tol,
                                               (double2*)Xbar);
    launch_check("eigh_adjoint_kernel");
}

void launch_fill(size_t n, double v, double* p, hipStream_t stream) {
    if (n == 0) return;
    fill_f64_kernel<<<nblk(n, 256), 256, 0, stream>>>(n, v, p);
    launch_check("fill_f64_kernel");
}

void launch_add_f64(size_t n, const double* src, double* dst, hipStream_t stream) {
    if (n == 0) return;
    add_f64_kernel<<<nblk(n, 256), 256, 0, stream>>>(n, src, dst);
    launch_check("add_f64_kernel");
}

void launch_c64_to_c128(size_t n, const void* in, int accumulate, void* out, hipStream_t stream) {
    if (n == 0) return;
    c64_to_c128_kernel<<<nblk(n, 256), 256, 0, stream>>>(n, (const float2*)in, accumulate, (double2*)out);
    launch_check("c64_to_c128_kernel");
}

}  // namespace epw
