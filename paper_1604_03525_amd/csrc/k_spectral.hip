// Frequency-resolved electron self-energy (Sec. 3 Eq. (3)) and the electronic
// spectral function (Sec. 3 Eq. (10)).
//
// The fused kernel's pole mode leaves, per k and q chunk, one record per pole
// family (q, nu, m):  {c1, c2, A1, A2, |g_mn|^2 for n < nb, zeros up to the
// padded band count} with
// c1 = xi_m - omega_q,nu, c2 = xi_m + omega_q,nu, A1 = n + f, A2 = n + 1 - f.
// The braces of Eq. (3) do not depend on the band n at k, so one evaluation
// of the two complex poles at a frequency serves every n:
//
//   Sigma_n(w) += |g_mn|^2 [A1 / (w - c1 + i d) + A2 / (w - c2 + i d)]
//   1/(x + i d) = (x - i d) / (x^2 + d^2)
//
// One wave per (frequency tile of 64, k, pole slice): lane j owns frequency
// j of the tile and all n; the records are read at wave-uniform addresses
// (scalar loads), so the VALU does only the pole arithmetic.  Slices are
// summed in fixed order by the reduction kernel, which also averages over
// degenerate bands and accumulates the chunk into the output.
#include <hip/hip_runtime.h>

#include "epw_internal.h"
#include "kernels.h"

namespace epw {
namespace {

// 1/d for d > 0 of moderate range: the hardware reciprocal estimate (relative
// error below 5e-8, measured) refined by one Newton-Raphson step
// r <- r + r (1 - d r), which squares the relative error (below 3e-15).
__device__ __forceinline__ double recip_pos(double d) {
    const double r = __builtin_amdgcn_rcp(d);
    return fma(r, fma(-d, r, 1.0), r);
}

template <int NBT>
__global__ __launch_bounds__(64) void sigma_omega_kernel(int nk, int nb, long npole, int nw, int nwt,
                                                         const double* __restrict__ wgrid, double delta,
                                                         const double* __restrict__ rec, int S,
                                                         double2* __restrict__ part)
{
    constexpr int RS = 4 + NBT;                        // record: c1, c2, A1, A2, |g|^2 [NBT]
    const int wt = blockIdx.x % nwt;
    const int k = blockIdx.x / nwt;
    const int s = blockIdx.y;
    const int j = wt * 64 + threadIdx.x;               // frequency index; j == nw is omega = 0
    const double w = j < nw ? wgrid[j] : 0.0;
    const long p0 = npole * s / S, p1 = npole * (s + 1) / S;
    const double d2 = delta * delta;
    double are[NBT], aim[NBT];
#pragma unroll
    for (int n = 0; n < NBT; ++n) {
        are[n] = 0.0;
        aim[n] = 0.0;
    }
    // records at wave-uniform addresses, two at a time, the next two read
    // ahead (the buffer holds two records of padding past the last)
    const double* r = rec + ((size_t)k * npole + p0) * RS;
    auto pole = [&](const double* c) {
        const double x1 = w - c[0], x2 = w - c[1];
        const double t1 = c[2] * recip_pos(fma(x1, x1, d2));
        const double t2 = c[3] * recip_pos(fma(x2, x2, d2));
        const double wre = fma(t1, x1, t2 * x2);       // real part of the braces
        const double wim = t1 + t2;                    // imaginary part is -d wim
#pragma unroll
        for (int n = 0; n < NBT; ++n) {
            are[n] = fma(c[4 + n], wre, are[n]);
            aim[n] = fma(c[4 + n], wim, aim[n]);
        }
    };
    double c0[RS], c1[RS];
#pragma unroll
    for (int i = 0; i < RS; ++i) {
        c0[i] = r[i];
        c1[i] = r[RS + i];
    }
    long p = p0;
    for (; p + 1 < p1; p += 2) {
        r += 2 * RS;
        double n0[RS], n1[RS];
#pragma unroll
        for (int i = 0; i < RS; ++i) {
            n0[i] = r[i];
            n1[i] = r[RS + i];
        }
        pole(c0);
        pole(c1);
#pragma unroll
        for (int i = 0; i < RS; ++i) {
            c0[i] = n0[i];
            c1[i] = n1[i];
        }
    }
    if (p < p1) pole(c0);
    if (j > nw) return;
    const size_t ld = (size_t)nw + 1;
#pragma unroll
    for (int n = 0; n < NBT; ++n) {
        if (n >= nb) break;
        part[(((size_t)s * nk + k) * nb + n) * ld + j] = make_double2(are[n], -delta * aim[n]);
    }
}

// out[k][n][j] (+)= scale x (degenerate average over n of) sum_s part[s][k][n][j];
// column j == nw goes to out0[k][n].
template <int NBT>
__global__ void sigma_omega_reduce_kernel(int nk, int nb, int nw, int S, const double2* __restrict__ part,
                                          const double* __restrict__ eps, double tol, double scale, int acc,
                                          double2* __restrict__ out, double2* __restrict__ out0)
{
    const size_t ld = (size_t)nw + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nk * ld) return;
    const int k = (int)(idx / ld), j = (int)(idx % ld);
    double vr[NBT], vi[NBT];
#pragma unroll
    for (int n = 0; n < NBT; ++n) {
        vr[n] = 0.0;
        vi[n] = 0.0;
        if (n >= nb) continue;
        for (int s = 0; s < S; ++s) {
            const double2 v = part[(((size_t)s * nk + k) * nb + n) * ld + j];
            vr[n] += v.x;
            vi[n] += v.y;
        }
        vr[n] *= scale;
        vi[n] *= scale;
    }
    // average over runs of bands whose sorted energies differ by < tol
    const double* e = eps + (size_t)k * nb;
    int start = 0;
    while (start < nb) {
        int stop = start + 1;
        while (stop < nb && fabs(e[stop] - e[stop - 1]) < tol) ++stop;
        if (stop - start > 1) {
            double tr = 0.0, ti = 0.0;
#pragma unroll
            for (int n = 0; n < NBT; ++n)
                if (n >= start && n < stop) {
                    tr += vr[n];
                    ti += vi[n];
                }
            tr /= (double)(stop - start);
            ti /= (double)(stop - start);
#pragma unroll
            for (int n = 0; n < NBT; ++n)
                if (n >= start && n < stop) {
                    vr[n] = tr;
                    vi[n] = ti;
                }
        }
        start = stop;
    }
#pragma unroll
    for (int n = 0; n < NBT; ++n) {
        if (n >= nb) break;
        double2* o = j < nw ? out + ((size_t)k * nb + n) * nw + j : out0 + (size_t)k * nb + n;
        double2 v = make_double2(vr[n], vi[n]);
        if (acc) {
            const double2 old = *o;
            v.x += old.x;
            v.y += old.y;
        }
        *o = v;
    }
}

// Eq. (10) with Sigma~' of Eq. (5): A = (1/pi) |S''| / ((w - xi - S~')^2 + S''^2)
__global__ void spectral_function_kernel(int nk, int nb, int nw, const double* __restrict__ eps, double mu,
                                         const double* __restrict__ wgrid, const double2* __restrict__ sig,
                                         const double2* __restrict__ sig0, double* __restrict__ A)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nk * nb * nw) return;
    const size_t kn = idx / nw;
    const int j = (int)(idx % nw);
    const double2 s = sig[idx];
    const double im = fabs(s.y);
    const double x = wgrid[j] - (eps[kn] - mu) - (s.x - sig0[kn].x);
    A[idx] = im / (M_PI * (x * x + im * im));
}

// One block (one wave) per (k, q) pair: for each mode nu, the Wannier-basis
// g_nu[i][j] = sc_nu sum_a C[a][i][j] e[a][nu] (+ L_nu delta_ij), then
// T = g_nu U_k and h = U_k+q^dag T, written as the pole records of (k, q, nu, m).
template <typename CT>
__global__ __launch_bounds__(64) void pair_pole_kernel(PairPoleArgs a)
{
    __shared__ double2 Uk[EPW_MAX_NB * EPW_MAX_NB], Uq[EPW_MAX_NB * EPW_MAX_NB];
    __shared__ double2 Gv[EPW_MAX_NB * EPW_MAX_NB], Tm[EPW_MAX_NB * EPW_MAX_NB];
    __shared__ double emq[EPW_MAX_NB], fmq[EPW_MAX_NB];
    const long pr = blockIdx.x;                      // k * qc + ql
    const int k = (int)(pr / a.qc), ql = (int)(pr % a.qc);
    const int tid = threadIdx.x;
    const int nb = a.nb, nb2 = nb * nb, nm = a.nm, RS = 4 + a.nbp;
    double* rec0 = a.rec + (size_t)pr * nm * nb * RS;
    const double2* Uqs;
    const double* eq;
    const double* fq;
    if (a.kq) {
        const int kq = a.kq[(size_t)k * a.nq_total + a.q0 + ql];
        if ((unsigned)kq >= (unsigned)a.nk) {        // invalid map entry: zero records
            for (int t = tid; t < nm * nb * RS; t += 64) rec0[t] = 0.0;
            return;
        }
        Uqs = reinterpret_cast<const double2*>(a.U) + (size_t)kq * nb2;
        eq = a.eps + (size_t)kq * nb;
        fq = a.ftab + (size_t)kq * nb;
    } else {
        Uqs = reinterpret_cast<const double2*>(a.U_pair) + (size_t)pr * nb2;
        eq = a.eps_pair + (size_t)pr * nb;
        fq = a.f_pair + (size_t)pr * nb;
    }
    const double2* Uks = reinterpret_cast<const double2*>(a.U) + (size_t)k * nb2;
    for (int t = tid; t < nb2; t += 64) {
        Uk[t] = Uks[t];
        Uq[t] = Uqs[t];
    }
    if (tid < nb) {
        emq[tid] = eq[tid];
        fmq[tid] = fq[tid];
    }
    const CT* C = reinterpret_cast<const CT*>(a.C) + (size_t)pr * nm * nb2;
    const double2* ev = reinterpret_cast<const double2*>(a.evec) + (size_t)ql * nm * nm;
    for (int nu = 0; nu < nm; ++nu) {
        const double s = a.sc[(size_t)ql * nm + nu];
        __syncthreads();                             // Gv, Tm of the previous mode no longer read
        for (int t = tid; t < nb2; t += 64) {
            double gr = 0.0, gi = 0.0;
            if (s != 0.0) {
                for (int m = 0; m < nm; ++m) {
                    const CT c = C[(size_t)m * nb2 + t];
                    const double2 e = ev[(size_t)m * nm + nu];
                    gr += (double)c.x * e.x - (double)c.y * e.y;
                    gi += (double)c.x * e.y + (double)c.y * e.x;
                }
                gr *= s;
                gi *= s;
            }
            if (a.Lq && t / nb == t % nb) {
                const double2 l = reinterpret_cast<const double2*>(a.Lq)[(size_t)ql * nm + nu];
                gr += l.x;
                gi += l.y;
            }
            Gv[t] = make_double2(gr, gi);
        }
        __syncthreads();
        for (int t = tid; t < nb2; t += 64) {        // T[i][n] = sum_j Gv[i][j] Uk[j][n]
            const int i = t / nb, n = t % nb;
            double tr = 0.0, ti = 0.0;
            for (int j = 0; j < nb; ++j) {
                const double2 g = Gv[i * nb + j], u = Uk[j * nb + n];
                tr += g.x * u.x - g.y * u.y;
                ti += g.x * u.y + g.y * u.x;
            }
            Tm[t] = make_double2(tr, ti);
        }
        __syncthreads();
        const double w = a.omega[(size_t)ql * nm + nu];
        const double nB = a.nbose[(size_t)ql * nm + nu];
        for (int t = tid; t < nb2; t += 64) {        // h[m][n] = sum_i conj(Uq[i][m]) T[i][n]
            const int m = t / nb, n = t % nb;
            double hr = 0.0, hi = 0.0;
            for (int i = 0; i < nb; ++i) {
                const double2 u = Uq[i * nb + m], x = Tm[i * nb + n];
                hr += u.x * x.x + u.y * x.y;
                hi += u.x * x.y - u.y * x.x;
            }
            double* rec = rec0 + ((size_t)nu * nb + m) * RS;
            rec[4 + n] = hr * hr + hi * hi;
            if (n == 0) {
                const double xi = emq[m] - a.mu;
                const bool kept = s != 0.0;
                rec[0] = xi - w;
                rec[1] = xi + w;
                rec[2] = kept ? nB + fmq[m] : 0.0;
                rec[3] = kept ? nB + 1.0 - fmq[m] : 0.0;
                for (int j = nb; j < a.nbp; ++j) rec[4 + j] = 0.0;
            }
        }
    }
}

}  // namespace

void launch_pair_pole(const PairPoleArgs& a, hipStream_t stream) {
    const long pairs = (long)a.nk * a.qc;
    if (pairs == 0) return;
    if (a.c64)
        pair_pole_kernel<float2><<<(unsigned)pairs, 64, 0, stream>>>(a);
    else
        pair_pole_kernel<double2><<<(unsigned)pairs, 64, 0, stream>>>(a);
    launch_check("pair_pole_kernel");
}

int sigma_omega_slices(int nk, int nw, long npole) {
    const long waves = (long)nk * ((nw + 1 + 63) / 64);
    if (waves <= 0 || npole <= 0) return 1;
    long S = (8192 + waves - 1) / waves;              // about 8 waves per SIMD
    const long cap = npole / 64 > 0 ? npole / 64 : 1;  // at least 64 poles per wave
    if (S > cap) S = cap;
    if (S > 1024) S = 1024;
    return S < 1 ? 1 : (int)S;
}

void launch_sigma_omega(int nk, int nb, long npole, int nw, const double* wgrid, double delta, const double* rec,
                        int S, void* part, hipStream_t stream) {
    if (nk == 0 || npole == 0) return;
    const int nwt = (nw + 1 + 63) / 64;
    const dim3 grid((unsigned)(nk * nwt), (unsigned)S);
    double2* p = (double2*)part;
    switch (pow2_at_least(nb)) {
        case 1: sigma_omega_kernel<1><<<grid, 64, 0, stream>>>(nk, nb, npole, nw, nwt, wgrid, delta, rec, S, p); break;
        case 2: sigma_omega_kernel<2><<<grid, 64, 0, stream>>>(nk, nb, npole, nw, nwt, wgrid, delta, rec, S, p); break;
        case 4: sigma_omega_kernel<4><<<grid, 64, 0, stream>>>(nk, nb, npole, nw, nwt, wgrid, delta, rec, S, p); break;
        case 8: sigma_omega_kernel<8><<<grid, 64, 0, stream>>>(nk, nb, npole, nw, nwt, wgrid, delta, rec, S, p); break;
        case 16: sigma_omega_kernel<16><<<grid, 64, 0, stream>>>(nk, nb, npole, nw, nwt, wgrid, delta, rec, S, p); break;
        default: break;
    }
    launch_check("sigma_omega_kernel");
}

void launch_sigma_omega_reduce(int nk, int nb, int nw, int S, const void* part, const double* eps, double tol,
                               double scale, int acc, void* out, void* out0, hipStream_t stream) {
    const size_t n = (size_t)nk * (nw + 1);
    if (n == 0) return;
    const unsigned blocks = (unsigned)((n + 127) / 128);
    const double2* p = (const double2*)part;
    double2* o = (double2*)out;
    double2* o0 = (double2*)out0;
    switch (pow2_at_least(nb)) {
        case 1: sigma_omega_reduce_kernel<1><<<blocks, 128, 0, stream>>>(nk, nb, nw, S, p, eps, tol, scale, acc, o, o0); break;
        case 2: sigma_omega_reduce_kernel<2><<<blocks, 128, 0, stream>>>(nk, nb, nw, S, p, eps, tol, scale, acc, o, o0); break;
        case 4: sigma_omega_reduce_kernel<4><<<blocks, 128, 0, stream>>>(nk, nb, nw, S, p, eps, tol, scale, acc, o, o0); break;
        case 8: sigma_omega_reduce_kernel<8><<<blocks, 128, 0, stream>>>(nk, nb, nw, S, p, eps, tol, scale, acc, o, o0); break;
        case 16: sigma_omega_reduce_kernel<16><<<blocks, 128, 0, stream>>>(nk, nb, nw, S, p, eps, tol, scale, acc, o, o0); break;
        default: break;
    }
    launch_check("sigma_omega_reduce_kernel");
}

void launch_spectral_function(int nk, int nb, int nw, const double* eps, double mu, const double* wgrid,
                              const void* sig, const void* sig0, double* A, hipStream_t stream) {
    const size_t n = (size_t)nk * nb * nw;
    if (n == 0) return;
    spectral_function_kernel<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(
        nk, nb, nw, eps, mu, wgrid, (const double2*)sig, (const double2*)sig0, A);
    launch_check("spectral_function_kernel");
}

}  // namespace epw
