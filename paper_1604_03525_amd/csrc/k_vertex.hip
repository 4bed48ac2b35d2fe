// Vertex interpolation and the fused self-energy reduction (float64 and
// float32 complex paths on MFMA 16x16x4).
//
//   a5  g(R_e,q)      = sum_{R_p} Phi_q[q][R_p] g(R_e,R_p)         complex GEMM
//   a6  g_nu(R_e,q)   = sum_ka g_ka(R_e,q) e_ka,nu(q) / sqrt(2 w)   per-q mode rotation
//   a7  g_nu(k,q)     = sum_{R_e} Phi_k[k][R_e] g_nu(R_e,q)         complex GEMM (hot loop)
//   a8  g_mn,nu(k,q)  = [U_{k+q}^dag g_nu(k,q) U_k]_mn              fused epilogue
//   a9  Im Sigma_nk  += |g_mn,nu|^2 {(n+f) d(x+w) + (n+1-f) d(x-w)}  fused epilogue
//
// Phi tables already carry the 1/ndeg weights.  Complex products use four
// real MFMAs (re.re, -im.im into the real accumulator, re.im, im.re into the
// imaginary one); the four are interleaved over the wave's four C blocks so
// consecutive MFMAs never depend on each other.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include "cgemm.h"
#include "epw_internal.h"
#include "kernels.h"

namespace epw {
namespace {

// ------------------------------------------------------------ phase tables

__global__ void phase_table_kernel(int np, const double* __restrict__ pts, int nR,
                                   const int32_t* __restrict__ R, const int32_t* __restrict__ ndeg,
                                   int ld, int prec, void* __restrict__ out)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)np * ld;
    if (idx >= total) return;
    const int p = (int)(idx / ld), r = (int)(idx % ld);
    double c = 0.0, s = 0.0;
    if (r < nR) {
        double x = pts[3 * (size_t)p] * (double)R[3 * r] + pts[3 * (size_t)p + 1] * (double)R[3 * r + 1] +
                   pts[3 * (size_t)p + 2] * (double)R[3 * r + 2];
        x -= rint(x);
        sincospi(2.0 * x, &s, &c);
        const double w = 1.0 / (double)ndeg[r];
        c *= w;
        s *= w;
    }
    if (prec == 0) {
        reinterpret_cast<double2*>(out)[idx] = make_double2(c, s);
    } else if (prec == 1) {
        reinterpret_cast<float2*>(out)[idx] = make_float2((float)c, (float)s);
    } else {
        __hip_bfloat16* o = reinterpret_cast<__hip_bfloat16*>(out);
        const __hip_bfloat16 ch = __float2bfloat16((float)c);
        const __hip_bfloat16 cl = __float2bfloat16((float)(c - (double)__bfloat162float(ch)));
        const __hip_bfloat16 sh = __float2bfloat16((float)s);
        const __hip_bfloat16 sl = __float2bfloat16((float)(s - (double)__bfloat162float(sh)));
        o[idx] = ch;
        o[total + idx] = cl;
        o[2 * total + idx] = sh;
        o[3 * total + idx] = sl;
    }
}

__global__ void c128_to_c64_kernel(size_t n, const double2* __restrict__ in, float2* __restrict__ out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

__global__ void phonon_factors_kernel(int n, const double* __restrict__ omega, double cut, double kT,
                                      double* __restrict__ sc, double* __restrict__ nb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double w = omega[i];
    if (w < cut) {
        sc[i] = 0.0;
        nb[i] = 0.0;
        return;
    }
    sc[i] = 1.0 / sqrt(2.0 * w);
    nb[i] = (kT > 0.0) ? 1.0 / expm1(w / kT) : 0.0;
}

__global__ void fermi_kernel(size_t n, const double* __restrict__ eps, double mu, double kT,
                             double* __restrict__ f) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double e = eps[i];
    if (kT > 0.0) {
        f[i] = 1.0 / (exp((e - mu) / kT) + 1.0);
    } else {
        f[i] = e < mu ? 1.0 : (e > mu ? 0.0 : 0.5);
    }
}

// ------------------------------------------------------------ a5: R_p -> q

template <typename T>
__global__ __launch_bounds__(256) void gemm_rp_kernel(int nq, int ne, int np_, int ncol,
                                                      const typename Cx<T>::type* __restrict__ phi, int ldphi,
                                                      const typename Cx<T>::type* __restrict__ gR,
                                                      typename Cx<T>::type* __restrict__ out)
{
    typedef typename Cx<T>::type CT;
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ Stage<T, BM, BN, BK> st;
    const int m0 = blockIdx.y * BM;
    const long n0 = (long)blockIdx.x * BN;
    const long N = (long)ne * ncol;
    auto afetch = [&](int m, int k) -> CT {
        const int q = m0 + m;
        if (q < nq && k < np_) return phi[(size_t)q * ldphi + k];
        return cz<T>();
    };
    auto bfetch = [&](int k, int n) -> CT {
        const long col = n0 + n;
        if (k < np_ && col < N) {
            const long e = col / ncol, c = col % ncol;
            return gR[((size_t)e * np_ + k) * ncol + c];
        }
        return cz<T>();
    };
    typename Cx<T>::acc cr[4], ci[4];
    cgemm_mainloop<T, BM, BN, BK>(st, np_, afetch, bfetch, cr, ci);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = 0; c < 4; ++c) {
        const long col = n0 + c * 16 + (lane & 15);
        if (col >= N) continue;
        const long e = col / ncol, cc = col % ncol;
        for (int i = 0; i < 4; ++i) {
            const int q = m0 + wave * 16 + crow<T>(lane, i);
            if (q >= nq) continue;
            CT v;
            v.x = cr[c][i];
            v.y = ci[c][i];
            out[((size_t)e * nq + q) * ncol + cc] = v;
        }
    }
}

// ------------------------------------------------------------ a6: modes

template <typename T>
__global__ void mode_rotate_kernel(int ne, int nq, int nm, int nb, int nbp,
                                   const typename Cx<T>::type* __restrict__ in,
                                   const double2* __restrict__ evec, const double* __restrict__ sc,
                                   typename Cx<T>::type* __restrict__ out)
{
    typedef typename Cx<T>::type CT;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nbp2 = nbp * nbp;
    const size_t total = (size_t)ne * nq * nbp2;
    if (idx >= total) return;
    const int ij = (int)(idx % nbp2);
    const size_t eq = idx / nbp2;
    const int q = (int)(eq % nq);
    const int i = ij / nbp, j = ij % nbp;
    CT* o = out + eq * (size_t)nm * nbp2 + ij;
    if (i >= nb || j >= nb) {
        for (int v = 0; v < nm; ++v) o[(size_t)v * nbp2] = cz<T>();
        return;
    }
    const CT* x = in + eq * (size_t)nm * nb * nb + i * nb + j;
    for (int v = 0; v < nm; ++v) {
        const double s = sc[(size_t)q * nm + v];
        T re = T(0), im = T(0);
        if (s != 0.0) {
            for (int a = 0; a < nm; ++a) {
                const double2 ev = evec[((size_t)q * nm + a) * nm + v];
                const CT g = x[(size_t)a * nb * nb];
                re += g.x * (T)ev.x - g.y * (T)ev.y;
                im += g.x * (T)ev.y + g.y * (T)ev.x;
            }
            re *= (T)s;
            im *= (T)s;
        }
        CT r;
        r.x = re;
        r.y = im;
        o[(size_t)v * nbp2] = r;
    }
}

// ------------------------------------------------------------ a7+a8+a9
//
// Block (mt, s): k rows [mt*BM, mt*BM+BM), column tiles nt = s, s+S, ...
// Columns are (q_local, nu, i, j) with i, j < NBP; a tile holds whole band
// blocks (BN is a multiple of NBP^2), so the rotation and the reduction run
// on the LDS copy of the C tile.  Im Sigma contributions are accumulated in
// registers across all of the block's tiles and written once per block to
// part[s][k][n]: the cross-block sum is a separate fixed-order reduction.

template <int NBP> struct FusedShape {
    static constexpr int BN = NBP * NBP >= 64 ? NBP * NBP : 64;
    static constexpr int BM = 4096 / BN;          // 64 x 64 or 16 x 256
};

template <typename T, int NBP, bool STORE>
__global__ __launch_bounds__(256) void fused_k_kernel(FusedArgs a, int tiles_m, int tiles_n)
{
    typedef typename Cx<T>::type CT;
    constexpr int BM = FusedShape<NBP>::BM, BN = FusedShape<NBP>::BN, BK = 16;
    constexpr int NB2 = NBP * NBP;
    constexpr int NBLK = BN / NB2;                 // band blocks per tile
    constexpr int TPR = 256 / BM;                  // threads per k row
    constexpr int JN = (NBP + TPR - 1) / TPR;      // n values per thread when nb > TPR
    typedef Stage<T, BM, BN, BK> St;
    constexpr size_t CBYTES = sizeof(CT) * BM * BN;
    constexpr size_t SBYTES = sizeof(St) > CBYTES ? sizeof(St) : CBYTES;
    __shared__ __attribute__((aligned(16))) char smem[SBYTES];
    __shared__ double red[256];
    St& st = *reinterpret_cast<St*>(smem);
    CT* Cs = reinterpret_cast<CT*>(smem);

    // XCD-aware remap: consecutive workgroup ids land on different XCDs
    // (round-robin over 8); give each XCD a contiguous range of (s, mt)
    // so blocks sharing a column slice run on the same L2.
    const int G = gridDim.x;
    const int bid = blockIdx.x;
    const int per = G / 8;
    const int lin = (bid % 8) * per + bid / 8;
    if (lin >= tiles_m * a.S) return;
    const int s = lin / tiles_m;
    const int mt = lin % tiles_m;
    const int m0 = mt * BM;

    const int nb = a.nb, nm = a.nm;
    const int tid = threadIdx.x;
    const int r = tid / TPR, sub = tid % TPR;
    const int k = m0 + r;
    const long ncols = (long)a.qc * nm * NB2;
    const long ldb = ncols;
    const CT* phi = reinterpret_cast<const CT*>(a.phi_k);
    const CT* Bm = reinterpret_cast<const CT*>(a.B);
    const double2* U = reinterpret_cast<const double2*>(a.U);

    // thread -> (n, block subset)
    const bool fewn = nb <= TPR;
    const int NT = fewn ? TPR / nb : 1;               // threads per n value
    const int n_single = fewn ? sub / NT : 0;
    const int bsub = fewn ? sub % NT : 0;
    const bool active_row = k < a.nk;
    const bool active_thr = active_row && (!fewn || n_single < nb);

    double acc[JN];
    for (int j = 0; j < JN; ++j) acc[j] = 0.0;

    const double inv_sig = 1.0 / a.sigma;
    double eps_k[JN];
    double2 Uk[JN][NBP];
    for (int j = 0; j < JN; ++j) {
        const int n = fewn ? n_single : sub + j * TPR;
        eps_k[j] = 0.0;
        for (int jj = 0; jj < NBP; ++jj) Uk[j][jj] = make_double2(0.0, 0.0);
        if (active_thr && n < nb) {
            eps_k[j] = a.eps[(size_t)k * nb + n];
            for (int jj = 0; jj < nb; ++jj) Uk[j][jj] = U[((size_t)k * nb + jj) * nb + n];
        }
    }

    for (int nt = s; nt < tiles_n; nt += a.S) {
        const long n0 = (long)nt * BN;
        auto afetch = [&](int m, int kk) -> CT {
            const int row = m0 + m;
            if (row < a.nk && kk < a.ne) return phi[(size_t)row * a.ldk + kk];
            return cz<T>();
        };
        auto bfetch = [&](int kk, int n) -> CT {
            const long col = n0 + n;
            if (kk < a.ne && col < ncols) return Bm[(size_t)kk * ldb + col];
            return cz<T>();
        };
        typename Cx<T>::acc cr[4], ci[4];
        cgemm_mainloop<T, BM, BN, BK>(st, a.ne, afetch, bfetch, cr, ci);
        // C fragments -> LDS tile [BM][BN]
        {
            const int lane = tid & 63, wave = tid >> 6;
            constexpr int WN = BN / 64;
            const int wm = wave / WN, wn = wave % WN;
            for (int c = 0; c < 4; ++c)
                for (int i = 0; i < 4; ++i) {
                    const int row = wm * 16 + crow<T>(lane, i);
                    const int col = wn * 64 + c * 16 + (lane & 15);
                    CT v;
                    v.x = cr[c][i];
                    v.y = ci[c][i];
                    Cs[row * BN + col] = v;
                }
        }
        __syncthreads();
        if (active_thr) {
            for (int b = 0; b < NBLK; ++b) {
                if (fewn && (b % NT) != bsub) continue;
                const long gblk = n0 / NB2 + b;            // (q_local, nu)
                const int ql = (int)(gblk / nm), nu = (int)(gblk % nm);
                if (ql >= a.qc) break;
                const double scv = a.sc[(size_t)ql * nm + nu];
                if (scv == 0.0 && !STORE) continue;
                const int q = a.q0 + ql;
                const int kq = a.kq[(size_t)k * a.nq_total + q];
                if ((unsigned)kq >= (unsigned)a.nk) continue;   // invalid map entry: no access
                const double w = a.omega[(size_t)ql * nm + nu];
                const double nB = a.nbose[(size_t)ql * nm + nu];
                const CT* G = Cs + r * BN + b * NB2;
                for (int j = 0; j < JN; ++j) {
                    const int n = fewn ? n_single : sub + j * TPR;
                    if (n >= nb) continue;
                    // v = G U_k[:, n]
                    double2 v[NBP];
#pragma unroll
                    for (int i = 0; i < NBP; ++i) {
                        double vr = 0.0, vi = 0.0;
                        if (i < nb) {
#pragma unroll
                            for (int jj = 0; jj < NBP; ++jj) {
                                if (jj < nb) {
                                    const CT g = G[i * NBP + jj];
                                    const double2 u = Uk[j][jj];
                                    vr += (double)g.x * u.x - (double)g.y * u.y;
                                    vi += (double)g.x * u.y + (double)g.y * u.x;
                                }
                            }
                        }
                        v[i] = make_double2(vr, vi);
                    }
                    for (int m = 0; m < nb; ++m) {
                        double gr = 0.0, gi = 0.0;
#pragma unroll
                        for (int i = 0; i < NBP; ++i) {
                            if (i < nb) {
                                const double2 u = U[((size_t)kq * nb + i) * nb + m];
                                // conj(u) * v_i
                                gr += u.x * v[i].x + u.y * v[i].y;
                                gi += u.x * v[i].y - u.y * v[i].x;
                            }
                        }
                        if (STORE) {
                            reinterpret_cast<double2*>(a.gkq)
                                [((((size_t)k * a.nq_total + q) * nm + nu) * nb + m) * nb + n] =
                                make_double2(gr, gi);
                        } else {
                            const double em = a.eps[(size_t)kq * nb + m];
                            const double fm = a.ftab[(size_t)kq * nb + m];
                            const double x = eps_k[j] - em;
                            const double y1 = (x + w) * inv_sig, y2 = (x - w) * inv_sig;
                            const double W = (nB + fm) * exp(-y1 * y1) + (nB + 1.0 - fm) * exp(-y2 * y2);
                            acc[j] += (gr * gr + gi * gi) * W;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (STORE) return;
    // fixed-order reduction of the NT partial sums of each (k, n)
    if (fewn) {
        red[tid] = acc[0];
        __syncthreads();
        if (active_thr && bsub == 0) {
            double t = 0.0;
            for (int u = 0; u < NT; ++u) t += red[r * TPR + n_single * NT + u];
            a.part[((size_t)s * a.nk + k) * nb + n_single] = t;
        }
    } else if (active_row) {
        for (int j = 0; j < JN; ++j) {
            const int n = sub + j * TPR;
            if (n < nb) a.part[((size_t)s * a.nk + k) * nb + n] = acc[j];
        }
    }
}

__global__ void reduce_partials_kernel(int nk, int nb, int S, const double* __restrict__ part,
                                       double scale, int accumulate, double* __restrict__ out)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)nk * nb;
    if (idx >= total) return;
    double t = 0.0;
    for (int s = 0; s < S; ++s) t += part[(size_t)s * total + idx];
    out[idx] = (accumulate ? out[idx] : 0.0) + scale * t;
}

__global__ void degenerate_average_kernel(int nk, int nb, const double* __restrict__ eps, double tol,
                                          double* __restrict__ v)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nk) return;
    const double* e = eps + (size_t)k * nb;
    double* x = v + (size_t)k * nb;
    int start = 0;
    while (start < nb) {
        int stop = start + 1;
        while (stop < nb && fabs(e[stop] - e[stop - 1]) < tol) ++stop;
        if (stop - start > 1) {
            double t = 0.0;
            for (int i = start; i < stop; ++i) t += x[i];
            t /= (double)(stop - start);
            for (int i = start; i < stop; ++i) x[i] = t;
        }
        start = stop;
    }
}

inline unsigned blocks_for(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T, int NBP>
void launch_fused_t(const FusedArgs& a, int num_cu, hipStream_t stream) {
    constexpr int BM = FusedShape<NBP>::BM, BN = FusedShape<NBP>::BN;
    const int tiles_m = (a.nk + BM - 1) / BM;
    const long ncols = (long)a.qc * a.nm * NBP * NBP;
    const int tiles_n = (int)((ncols + BN - 1) / BN);
    const long total = (long)tiles_m * a.S;
    const long G = ((total + 7) / 8) * 8;
    (void)num_cu;
    (void)tiles_n;
    if (a.gkq)
        fused_k_kernel<T, NBP, true><<<dim3((unsigned)G), dim3(256), 0, stream>>>(a, tiles_m, tiles_n);
    else
        fused_k_kernel<T, NBP, false><<<dim3((unsigned)G), dim3(256), 0, stream>>>(a, tiles_m, tiles_n);
    launch_check("fused_k_kernel");
}

template <typename T>
void launch_fused_nbp(const FusedArgs& a, int num_cu, hipStream_t stream) {
    switch (a.nbp) {
        case 1: launch_fused_t<T, 1>(a, num_cu, stream); break;
        case 2: launch_fused_t<T, 2>(a, num_cu, stream); break;
        case 4: launch_fused_t<T, 4>(a, num_cu, stream); break;
        case 8: launch_fused_t<T, 8>(a, num_cu, stream); break;
        case 16: launch_fused_t<T, 16>(a, num_cu, stream); break;
        default: break;
    }
}

}  // namespace

void launch_phase_table(Prec prec, int np, const double* pts, int nR, const int32_t* R,
                        const int32_t* ndeg, int ld, void* out, hipStream_t stream) {
    const size_t total = (size_t)np * ld;
    if (total == 0) return;
    phase_table_kernel<<<blocks_for(total, 256), 256, 0, stream>>>(np, pts, nR, R, ndeg, ld, (int)prec, out);
    launch_check("phase_table_kernel");
}

void launch_c128_to_c64(size_t n, const void* in, void* out, hipStream_t stream) {
    if (n == 0) return;
    c128_to_c64_kernel<<<blocks_for(n, 256), 256, 0, stream>>>(n, (const double2*)in, (float2*)out);
    launch_check("c128_to_c64_kernel");
}

void launch_phonon_factors(int nq, int nm, const double* omega, double omega_cut, double T,
                           double* sc, double* nbose, hipStream_t stream) {
    const int n = nq * nm;
    if (n == 0) return;
    const double kT = 8.617333262e-5 * T;
    phonon_factors_kernel<<<blocks_for(n, 256), 256, 0, stream>>>(n, omega, omega_cut, kT, sc, nbose);
    launch_check("phonon_factors_kernel");
}

void launch_fermi_table(size_t n, const double* eps, double mu, double T, double* f, hipStream_t stream) {
    if (n == 0) return;
    fermi_kernel<<<blocks_for(n, 256), 256, 0, stream>>>(n, eps, mu, 8.617333262e-5 * T, f);
    launch_check("fermi_kernel");
}

void launch_gemm_rp(Prec prec, int nq, int ne, int np_, int ncol, const void* phi_q, int ldphi,
                    const void* gR, void* out, hipStream_t stream) {
    const long N = (long)ne * ncol;
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((nq + 63) / 64));
    if (prec == Prec::F64)
        gemm_rp_kernel<double><<<grid, 256, 0, stream>>>(nq, ne, np_, ncol, (const double2*)phi_q, ldphi,
                                                         (const double2*)gR, (double2*)out);
    else
        gemm_rp_kernel<float><<<grid, 256, 0, stream>>>(nq, ne, np_, ncol, (const float2*)phi_q, ldphi,
                                                        (const float2*)gR, (float2*)out);
    launch_check("gemm_rp_kernel");
}

void launch_mode_rotate(Prec prec, int ne, int nq, int nm, int nb, int nbp, const void* in,
                        const void* evec, const double* sc, void* out, hipStream_t stream) {
    const size_t total = (size_t)ne * nq * nbp * nbp;
    if (total == 0) return;
    if (prec == Prec::F64)
        mode_rotate_kernel<double><<<blocks_for(total, 256), 256, 0, stream>>>(
            ne, nq, nm, nb, nbp, (const double2*)in, (const double2*)evec, sc, (double2*)out);
    else
        mode_rotate_kernel<float><<<blocks_for(total, 256), 256, 0, stream>>>(
            ne, nq, nm, nb, nbp, (const float2*)in, (const double2*)evec, sc, (float2*)out);
    launch_check("mode_rotate_kernel");
}

int fused_slices(int nk, int nbp, int tiles_n, int num_cu) {
    const int BM = (nbp * nbp >= 64) ? 4096 / (nbp * nbp) : 64;
    const int tiles_m = (nk + BM - 1) / BM;
    if (tiles_m <= 0 || tiles_n <= 0) return 1;
    // about four resident blocks per CU, in whole multiples of the k tiles
    long want = 4L * (num_cu > 0 ? num_cu : 256);
    long S = (want + tiles_m - 1) / tiles_m;
    if (S > tiles_n) S = tiles_n;
    if (S < 1) S = 1;
    return (int)S;
}

void launch_fused_k(Prec prec, const FusedArgs& a, int num_cu, hipStream_t stream) {
    if (a.nk == 0 || a.qc == 0) return;
    if (prec == Prec::F64)
        launch_fused_nbp<double>(a, num_cu, stream);
    else
        launch_fused_nbp<float>(a, num_cu, stream);
}

void launch_reduce_partials(int nk, int nb, int S, const double* part, double scale, int accumulate,
                            double* imsig, hipStream_t stream) {
    const size_t total = (size_t)nk * nb;
    if (total == 0) return;
    reduce_partials_kernel<<<blocks_for(total, 256), 256, 0, stream>>>(nk, nb, S, part, scale, accumulate, imsig);
    launch_check("reduce_partials_kernel");
}

void launch_degenerate_average(int nk, int nb, const double* eps, double tol, double* v, hipStream_t stream) {
    if (nk == 0 || nb < 2) return;
    degenerate_average_kernel<<<blocks_for(nk, 128), 128, 0, stream>>>(nk, nb, eps, tol, v);
    launch_check("degenerate_average_kernel");
}

}  // namespace epw
