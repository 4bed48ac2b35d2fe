// Vertex interpolation and the fused self-energy reduction (float64 and
// float32 complex paths on MFMA 16x16x4).
//
//   a5  g(R_e,q)      = sum_{R_p} Phi_q[q][R_p] g(R_e,R_p)         complex GEMM
//   a6  g_nu(R_e,q)   = sum_ka g_ka(R_e,q) e_ka,nu(q) / sqrt(2 w)   per-q mode rotation
//   a7  g_nu(k,q)     = sum_{R_e} Phi_k[k][R_e] g_nu(R_e,q)         complex GEMM (hot loop)
//   a8  g_mn,nu(k,q)  = [U_{k+q}^dag g_nu(k,q) U_k]_mn              fused epilogue
//   a9  Im Sigma_nk  += |g_mn,nu|^2 {(n+f) d(x+w) + (n+1-f) d(x-w)}  fused epilogue
//
// The 1/ndeg weights of R_e are folded into the B operand by a6.  Float64 (at
// every band count) and float32 (up to 8 padded bands) run the a7 sum folded
// by the pairs (R, -R) of the R_e list: with c and s the cosine and sine of a
// pair's phase, the pair contributes c (B(R) + B(-R)) + i s (B(R) - B(-R)),
// two real MFMAs per original R vector (cfold_mainloop, cgemm.h; a vector
// without its negative enters alone).  Float32 at 16 padded bands uses Gauss's
// three-multiplication form (three real MFMAs per complex block product), the
// split-bf16 path four real products of three split terms each.  The MFMAs of
// one K step are interleaved over the wave's C blocks so consecutive ones
// never depend on each other.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include "cgemm.h"
#include "epw_internal.h"
#include "kernels.h"

#include <type_traits>

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
        const double w = ndeg ? 1.0 / (double)ndeg[r] : 1.0;
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

// (a5, the R_p -> q contraction, runs on the generic complex GEMM of k_gemm.hip)

// ------------------------------------------------------------ a6: modes

template <typename T>
__global__ void mode_rotate_kernel(int ne, int nq, int nm, int nb, int nbp,
                                   const typename Cx<T>::type* __restrict__ in,
                                   const double2* __restrict__ evec, const double* __restrict__ sc,
                                   const int32_t* __restrict__ ndeg_fold,
                                   const double2* __restrict__ Lq, const int32_t* __restrict__ Re,
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
    const double wfold = ndeg_fold ? 1.0 / (double)ndeg_fold[eq / nq] : 1.0;
    for (int v = 0; v < nm; ++v) {
        const double s = sc[(size_t)q * nm + v] * wfold;
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
        if (Lq && i == j) {
            // polar long-range term: L_nu(q) delta_ij at R_e = 0, where the
            // phase is 1 for every k and the degeneracy is 1
            const int32_t* rv = Re + 3 * (eq / nq);
            if ((rv[0] | rv[1] | rv[2]) == 0) {
                const double2 l = Lq[(size_t)q * nm + v];
                re += (T)l.x;
                im += (T)l.y;
            }
        }
        CT r;
        r.x = re;
        r.y = im;
        o[(size_t)v * nbp2] = r;
    }
}

// a6 and the fold of the R_e rows by the pairs (R, -R) in one pass: thread
// (h, q, i, j) rotates rows half[h] and pair[h] of g(R_e, q), each with its
// 1/ndeg, and writes B+ = B(R) + B(-R) to row half[h] and B- = B(R) - B(-R)
// to row pair[h], or B(R) alone for an entry without a partner; the same
// values as mode_rotate_kernel (with the ndeg weights) followed by the fold.
template <typename T, int NMX>
__global__ void mode_rotate_fold_kernel(int ne, int nq, int nm, int nb, int nbp,
                                        const typename Cx<T>::type* __restrict__ in,
                                        const double2* __restrict__ evec, const double* __restrict__ sc,
                                        const int32_t* __restrict__ ndeg, const int32_t* __restrict__ kh,
                                        const int32_t* __restrict__ half, const int32_t* __restrict__ pair,
                                        const double2* __restrict__ Lq, const int32_t* __restrict__ Re,
                                        typename Cx<T>::type* __restrict__ out)
{
    typedef typename Cx<T>::type CT;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nbp2 = nbp * nbp;
    const size_t total = (size_t)ne * nq * nbp2;
    if (idx >= total) return;
    const int ij = (int)(idx % nbp2);
    const size_t hq = idx / nbp2;
    const int q = (int)(hq % nq);
    const int h = (int)(hq / nq);
    if (h >= kh[0]) return;
    const int e1 = half[h], e2 = pair[h];
    const bool two = e2 != e1;
    CT* o1 = out + ((size_t)e1 * nq + q) * nm * nbp2 + ij;
    CT* o2 = out + ((size_t)e2 * nq + q) * nm * nbp2 + ij;
    const int i = ij / nbp, j = ij % nbp;
    if (i >= nb || j >= nb) {
        for (int v = 0; v < nm; ++v) {
            o1[(size_t)v * nbp2] = cz<T>();
            if (two) o2[(size_t)v * nbp2] = cz<T>();
        }
        return;
    }
    // NMX > 0: the row's nm entries loaded once into registers (NMX >= nm, indices
    // known at compile time); NMX == 0 (more than 8 modes): read in the mode loop
    const CT* x1 = in + ((size_t)e1 * nq + q) * nm * nb * nb + i * nb + j;
    const CT* x2 = in + ((size_t)e2 * nq + q) * nm * nb * nb + i * nb + j;
    constexpr int NG = NMX > 0 ? NMX : 1;
    CT g1[NG], g2[NG];
#pragma unroll
    for (int a = 0; a < NG; ++a) {
        g1[a] = cz<T>();
        g2[a] = cz<T>();
        if (NMX > 0 && a < nm) {
            g1[a] = x1[(size_t)a * nb * nb];
            if (two) g2[a] = x2[(size_t)a * nb * nb];
        }
    }
    const double w1 = 1.0 / (double)ndeg[e1], w2 = 1.0 / (double)ndeg[e2];
    // the polar long-range term sits on the row with R_e = 0 (its own partner)
    const bool z1 = Lq && i == j && (Re[3 * e1] | Re[3 * e1 + 1] | Re[3 * e1 + 2]) == 0;
    const bool z2 = Lq && i == j && (Re[3 * e2] | Re[3 * e2 + 1] | Re[3 * e2 + 2]) == 0;
    for (int v = 0; v < nm; ++v) {
        const double s = sc[(size_t)q * nm + v];
        T ar = T(0), ai = T(0), br = T(0), bi = T(0);
        if (s != 0.0) {
            if constexpr (NMX > 0) {
#pragma unroll
                for (int a = 0; a < NMX; ++a) {
                    if (a >= nm) break;
                    const double2 ev = evec[((size_t)q * nm + a) * nm + v];
                    ar += g1[a].x * (T)ev.x - g1[a].y * (T)ev.y;
                    ai += g1[a].x * (T)ev.y + g1[a].y * (T)ev.x;
                    br += g2[a].x * (T)ev.x - g2[a].y * (T)ev.y;
                    bi += g2[a].x * (T)ev.y + g2[a].y * (T)ev.x;
                }
            } else {
                for (int a = 0; a < nm; ++a) {
                    const double2 ev = evec[((size_t)q * nm + a) * nm + v];
                    const CT g = x1[(size_t)a * nb * nb];
                    ar += g.x * (T)ev.x - g.y * (T)ev.y;
                    ai += g.x * (T)ev.y + g.y * (T)ev.x;
                    if (two) {
                        const CT f = x2[(size_t)a * nb * nb];
                        br += f.x * (T)ev.x - f.y * (T)ev.y;
                        bi += f.x * (T)ev.y + f.y * (T)ev.x;
                    }
                }
            }
            ar *= (T)(s * w1);
            ai *= (T)(s * w1);
            br *= (T)(s * w2);
            bi *= (T)(s * w2);
        }
        if (z1 || z2) {
            const double2 l = Lq[(size_t)q * nm + v];
            if (z1) {
                ar += (T)l.x;
                ai += (T)l.y;
            }
            if (z2) {
                br += (T)l.x;
                bi += (T)l.y;
            }
        }
        CT r;
        r.x = ar + br;
        r.y = ai + bi;
        if (two) {
            CT m;
            m.x = ar - br;
            m.y = ai - bi;
            o2[(size_t)v * nbp2] = m;
        } else {
            r.x = ar;
            r.y = ai;
        }
        o1[(size_t)v * nbp2] = r;
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

// 64 x 64 (4096 complex entries) up to 8 padded bands; at 16 bands one band
// block is 256 columns wide: 16 x 256 in float64, 32 x 256 in float32 and
// split-bf16, where a 16-row tile uses each B column for too few k rows to
// keep the main loop fed (the mobility-scale shard's split-bf16 fused stage
// 5.3 -> 3.7 s); the float64 C tile of 32 rows would not leave room in LDS
// for a second resident block
template <int MODE, int NBP> struct FusedShape {
    static constexpr int BN = NBP * NBP >= 64 ? NBP * NBP : 64;
    static constexpr int BM = (MODE != 0 && BN >= 256 ? 8192 : 4096) / BN;
};

// ---- split-bf16 tile: x = hi + lo (bf16 each), products hi.hi + hi.lo + lo.hi
// on MFMA 16x16x32 bf16 with float32 accumulation.  Operands are four bf16
// planes (re_hi, re_lo, im_hi, im_lo), K contiguous: A [4][rows][lda],
// B [4][cols][ldb]; K is padded with zeros to a multiple of 32.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline bf16x8 as_bf8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ inline uint4 neg_bf8(uint4 v) {
    v.x ^= 0x80008000u;
    v.y ^= 0x80008000u;
    v.z ^= 0x80008000u;
    v.w ^= 0x80008000u;
    return v;
}
__device__ inline f4 mfma_bf(uint4 a, uint4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a), as_bf8(b), c, 0, 0, 0);
}

template <int BM, int BN>
struct BfStage {
    static constexpr int BKP = 40;                 // 32 + 8 bf16 of padding per row
    uint16_t a[4][BM][BKP];
    uint16_t b[4][BN][BKP];
};

// Computes the BM x BN complex tile and leaves it in registers (same
// fragment layout as the f32 MFMA: element i of lane l is row 4(l/16)+i).
// split x into bf16 hi + lo, packed pairwise into 32-bit words
__device__ inline void split_pack(float x0, float x1, uint32_t& hi, uint32_t& lo) {
    const __hip_bfloat16 h0 = __float2bfloat16(x0), h1 = __float2bfloat16(x1);
    const __hip_bfloat16 l0 = __float2bfloat16(x0 - __bfloat162float(h0));
    const __hip_bfloat16 l1 = __float2bfloat16(x1 - __bfloat162float(h1));
    hi = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
    lo = (uint32_t)__builtin_bit_cast(uint16_t, l0) | ((uint32_t)__builtin_bit_cast(uint16_t, l1) << 16);
}

// GEN: the A operand (phases) is produced by agen(local_row, k) -> float2
// instead of being loaded; thread t < 4 BM generates row t/4, k = k0 + 8 (t%4) .. +7.
// B is staged in 16-byte chunks (8 bf16 of K); for tiles 256 or more columns
// wide, chunk e of thread t is chunk e * 256 + t, so that consecutive lanes
// read consecutive chunks (18 % faster at 16 bands), narrower tiles keep BCH
// consecutive chunks per thread (the other order was 6 % slower at 64 columns).
// Waves: WN = BN/64 across the columns, 4/WN across the rows; each wave owns
// RB row blocks of 16 x 64 (accumulator index rb * 4 + column block).
template <int BM, int BN> struct BfWaves {
    static constexpr int WN = BN / 64;
    static constexpr int RB = BM * WN / 64;
};
template <int BM, int BN, bool GEN, class AG>
__device__ inline void bf16_mainloop(BfStage<BM, BN>& st, const uint16_t* __restrict__ A, long lda, long aplane,
                                     int arows, int m0, const uint16_t* __restrict__ B, long ldb, long bplane,
                                     long bcols, long n0, int Kpad, AG agen, f4 (&cr)[4 * BfWaves<BM, BN>::RB],
                                     f4 (&ci)[4 * BfWaves<BM, BN>::RB])
{
    constexpr int WN = BfWaves<BM, BN>::WN;
    constexpr int RB = BfWaves<BM, BN>::RB;
    static_assert(RB >= 1 && 16 * RB * (4 / WN) == BM && 4 * BM <= 256, "split-bf16 wave layout");
    constexpr int ACH0 = 4 * BM * 4 / 256;         // 16-byte chunks per thread
    constexpr int ACH = GEN ? 4 : ACH0;
    constexpr int BCH = 4 * BN * 4 / 256;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    uint4 ra[ACH], rb[BCH];
    for (int c = 0; c < 4 * RB; ++c)
        for (int i = 0; i < 4; ++i) {
            cr[c][i] = 0.f;
            ci[c][i] = 0.f;
        }
    auto gload = [&](int k0) {
        if constexpr (GEN) {
            if (tid < 4 * BM) {
                const int row = tid >> 2, part = tid & 3;
                uint32_t w[4][4];
#pragma unroll
                for (int t = 0; t < 8; t += 2) {
                    const float2 p0 = agen(row, k0 + part * 8 + t);
                    const float2 p1 = agen(row, k0 + part * 8 + t + 1);
                    split_pack(p0.x, p1.x, w[0][t >> 1], w[1][t >> 1]);
                    split_pack(p0.y, p1.y, w[2][t >> 1], w[3][t >> 1]);
                }
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) ra[pl] = make_uint4(w[pl][0], w[pl][1], w[pl][2], w[pl][3]);
            }
        } else {
#pragma unroll
            for (int e = 0; e < ACH; ++e) {
                const int c = tid * ACH + e;
                const int p = c / (BM * 4), row = (c / 4) % BM, part = c % 4;
                const int grow = m0 + row;
                ra[e] = grow < arows ? *reinterpret_cast<const uint4*>(A + p * aplane + (size_t)grow * lda + k0 + part * 8)
                                     : make_uint4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int e = 0; e < BCH; ++e) {
            const int c = BN >= 256 ? e * 256 + tid : tid * BCH + e;
            const int p = c / (BN * 4), col = (c / 4) % BN, part = c % 4;
            const long gcol = n0 + col;
            rb[e] = gcol < bcols ? *reinterpret_cast<const uint4*>(B + p * bplane + (size_t)gcol * ldb + k0 + part * 8)
                                 : make_uint4(0, 0, 0, 0);
        }
    };
    auto sstore = [&]() {
        if constexpr (GEN) {
            if (tid < 4 * BM) {
                const int row = tid >> 2, part = tid & 3;
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) *reinterpret_cast<uint4*>(&st.a[pl][row][part * 8]) = ra[pl];
            }
        } else {
#pragma unroll
            for (int e = 0; e < ACH; ++e) {
                const int c = tid * ACH + e;
                const int p = c / (BM * 4), row = (c / 4) % BM, part = c % 4;
                *reinterpret_cast<uint4*>(&st.a[p][row][part * 8]) = ra[e];
            }
        }
#pragma unroll
        for (int e = 0; e < BCH; ++e) {
            const int c = BN >= 256 ? e * 256 + tid : tid * BCH + e;
            const int p = c / (BN * 4), col = (c / 4) % BN, part = c % 4;
            *reinterpret_cast<uint4*>(&st.b[p][col][part * 8]) = rb[e];
        }
    };
    gload(0);
    sstore();
    __syncthreads();
    const int koff = 8 * (lane >> 4);
    for (int k0 = 0; k0 < Kpad; k0 += 32) {
        const bool more = k0 + 32 < Kpad;
        if (more) gload(k0 + 32);
        if constexpr (RB == 1) {
            const int arow = wm * 16 + (lane & 15);
            const uint4 arh = *reinterpret_cast<const uint4*>(&st.a[0][arow][koff]);
            const uint4 arl = *reinterpret_cast<const uint4*>(&st.a[1][arow][koff]);
            const uint4 aih = *reinterpret_cast<const uint4*>(&st.a[2][arow][koff]);
            const uint4 ail = *reinterpret_cast<const uint4*>(&st.a[3][arow][koff]);
            const uint4 naih = neg_bf8(aih), nail = neg_bf8(ail);
            uint4 brh[4], brl[4], bih[4], bil[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int bcol = wn * 64 + c * 16 + (lane & 15);
                brh[c] = *reinterpret_cast<const uint4*>(&st.b[0][bcol][koff]);
                brl[c] = *reinterpret_cast<const uint4*>(&st.b[1][bcol][koff]);
                bih[c] = *reinterpret_cast<const uint4*>(&st.b[2][bcol][koff]);
                bil[c] = *reinterpret_cast<const uint4*>(&st.b[3][bcol][koff]);
            }
            // the four column blocks interleaved: consecutive MFMAs never share an accumulator
#pragma unroll
            for (int c = 0; c < 4; ++c) cr[c] = mfma_bf(arh, brh[c], cr[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) ci[c] = mfma_bf(arh, bih[c], ci[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) cr[c] = mfma_bf(arh, brl[c], cr[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) ci[c] = mfma_bf(arh, bil[c], ci[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) cr[c] = mfma_bf(arl, brh[c], cr[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) ci[c] = mfma_bf(arl, bih[c], ci[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) cr[c] = mfma_bf(naih, bih[c], cr[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) ci[c] = mfma_bf(aih, brh[c], ci[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) cr[c] = mfma_bf(naih, bil[c], cr[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) ci[c] = mfma_bf(aih, brl[c], ci[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) cr[c] = mfma_bf(nail, bih[c], cr[c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) ci[c] = mfma_bf(ail, brh[c], ci[c]);
        } else {
            // RB row blocks share each B fragment; the A fragments of all row
            // blocks stay in registers over the four column blocks, the B
            // fragments of one column block at a time
            uint4 arh[RB], arl[RB], aih[RB], ail[RB], naih[RB], nail[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int arow = wm * 16 * RB + q * 16 + (lane & 15);
                arh[q] = *reinterpret_cast<const uint4*>(&st.a[0][arow][koff]);
                arl[q] = *reinterpret_cast<const uint4*>(&st.a[1][arow][koff]);
                aih[q] = *reinterpret_cast<const uint4*>(&st.a[2][arow][koff]);
                ail[q] = *reinterpret_cast<const uint4*>(&st.a[3][arow][koff]);
                naih[q] = neg_bf8(aih[q]);
                nail[q] = neg_bf8(ail[q]);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int bcol = wn * 64 + c * 16 + (lane & 15);
                const uint4 brh = *reinterpret_cast<const uint4*>(&st.b[0][bcol][koff]);
                const uint4 brl = *reinterpret_cast<const uint4*>(&st.b[1][bcol][koff]);
                const uint4 bih = *reinterpret_cast<const uint4*>(&st.b[2][bcol][koff]);
                const uint4 bil = *reinterpret_cast<const uint4*>(&st.b[3][bcol][koff]);
                // real and imaginary accumulators of the RB row blocks taken in
                // turn, so that consecutive MFMAs never share an accumulator
                auto step = [&](const uint4 (&ar)[RB], uint4 br, const uint4 (&ai)[RB], uint4 bi) {
#pragma unroll
                    for (int q = 0; q < RB; ++q) {
                        cr[q * 4 + c] = mfma_bf(ar[q], br, cr[q * 4 + c]);
                        ci[q * 4 + c] = mfma_bf(ai[q], bi, ci[q * 4 + c]);
                    }
                };
                step(arh, brh, arh, bih);
                step(arh, brl, arh, bil);
                step(arl, brh, arl, bih);
                step(naih, bih, aih, brh);
                step(naih, bil, aih, brl);
                step(nail, bih, ail, brh);
            }
        }
        __syncthreads();
        if (more) {
            sstore();
            __syncthreads();
        }
    }
}

// MODE 0: float64 MFMA, float64 epilogue.  MODE 1: float32 MFMA, MODE 2:
// split-bf16 MFMA; both with a float32 rotation and float32 weights from
// float64 energy differences, accumulated in float64.
template <int MODE> struct ModeTypes;
template <> struct ModeTypes<0> { typedef double T; typedef double2 CT; typedef double TE; typedef double2 CE; };
template <> struct ModeTypes<1> { typedef float T; typedef float2 CT; typedef float TE; typedef float2 CE; };
template <> struct ModeTypes<2> { typedef float T; typedef float2 CT; typedef float TE; typedef float2 CE; };

__device__ inline double2 mk2(double x, double y) { return make_double2(x, y); }
__device__ inline float2 mk2(float x, float y) { return make_float2(x, y); }
__device__ inline double fexp(double x) { return exp(x); }
__device__ inline float fexp(float x) { return __expf(x); }

__device__ inline double2 cmulx(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cmulx(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// GEN: the electron phases exp(2 pi i k.R_e) are generated from per-axis
// factors exp(2 pi i k_a n), |n| <= nmax, kept in (dynamic) LDS for the
// block's k rows: three complex products per element instead of a table
// streamed from memory once per column tile.  The 1/ndeg weights are then
// carried by the B operand.
// KIND 0: Im Sigma (Eq. (8)) partial sums per (k, n); 1: store g_mn,nu(k,q);
// 2: the sums of the phonon linewidth (Eq. (9)) and of the coupling strength
// (Eq. (11)) per (q, nu), reduced over the tile's k rows in fixed order;
// 3: the real part of Eq. (3) per (k, n), on shell and at omega = eps_F;
// 4: one pole record of 4 + NBP doubles per (k, q, nu, m) for the
// frequency-resolved Eq. (3): {xi_m - omega, xi_m + omega, n + f, n + 1 - f,
// |g_mn|^2 for n < nb, 0 up to NBP}, with xi_m = eps_m,k+q - mu (the records
// of modes below omega_cut carry zero weights);
// 5: mode 2 plus the transport coupling sum of Eq. (55) (the Eq. (11) weight
// times 1 - v_nk . v_m,k+q / |v_nk|^2; velocities of the k set, and per pair
// at k+q for off-grid runs).
template <int MODE, int NBP, int KIND, bool GEN>
__global__ __launch_bounds__(256, 2) void fused_k_kernel(FusedArgs a, int tiles_m, int tiles_n)
{
    constexpr bool STORE = KIND == 1;
    constexpr bool WSTORE = KIND == 6;
    static_assert(!WSTORE || MODE != 2, "the Wannier-basis store runs in float64 / float32");
    constexpr bool TR = KIND == 5;
    constexpr bool PH = KIND == 2 || TR;
    constexpr bool RE = KIND == 3;
    constexpr bool POLE = KIND == 4;
    typedef typename ModeTypes<MODE>::T T;
    typedef typename ModeTypes<MODE>::CT CT;
    typedef typename ModeTypes<MODE>::TE TE;
    typedef typename ModeTypes<MODE>::CE CE;
    constexpr int BM = FusedShape<MODE, NBP>::BM, BN = FusedShape<MODE, NBP>::BN;
    // folded R_e -> k contraction (cfold_mainloop): float64, and float32 up
    // to 8 padded bands, every kind (the adjoint's recompute included).
    // fcc 20^3: FP32 278 -> 226 ms per 4000-q launch, FP64 256 -> 204 ms per
    // 2000-q launch (K steps of 8 halved entries in two LDS stages: with
    // steps of 16 in one stage, as unfolded, the fold ran slower, 256 -> 288
    // ms, the doubled B staging of each step standing between its two
    // barriers); mobility shard at 16 bands: FP64 205 -> 168 ms per launch
    // (K steps of 4 in two stages), FP32 131 -> 155 ms with one stage, and
    // two stages with the row indices exceed the LDS of two blocks.
    constexpr bool FOLD = fused_fold_c(NBP, MODE) && !GEN;
    // K step: 8 for the float64 16 x 256 tile, whose B stage (16 complex
    // doubles per thread at K step 16) would not fit beside its accumulators,
    // and for the folded float64 loop below 16 bands; 4 for the folded one
    // at 16 bands
    constexpr int BK = (MODE == 0 && NBP >= 16 && FOLD) ? 4 : (MODE == 0 && (NBP >= 16 || FOLD)) ? 8 : 16;
    constexpr int NB2 = NBP * NBP;
    constexpr int TPR = 256 / BM;                  // threads per k row
    // Epilogue work items of a row: (band block b, band x), x < NBP; thread
    // `sub` of the row owns items sub*JI .. sub*JI + JI - 1, in runs of RUN
    // consecutive items that share one band block.
    constexpr int JI = BN / (NBP * TPR);
    constexpr int RUN = JI < NBP ? JI : NBP;
    constexpr int NRUN = JI / RUN;
    // bands of a run taken together in phase 2: one for split-bf16, float32 at
    // 16 bands and the float64 Im Sigma reduction, whose k+q eigenvector
    // columns then leave its accumulators in registers (fcc 20^3: 116 bytes
    // per lane of spills, 29 GB of spill stores per launch -> none; 203 -> 191
    // ms per 2000-q launch; the phonon kind ran 3.5 % slower so and keeps RUN)
    constexpr int RT = (MODE == 2 || (MODE == 1 && NBP >= 16) || (MODE == 0 && KIND == 0)) ? 1 : RUN;
    static_assert(JI * NBP * TPR == BN && JI % RUN == 0 && NBP % RUN == 0, "epilogue split");
    constexpr int LDC = BN + 1;                    // C tile row stride: rows start on different LDS banks
    typedef typename PickType<FOLD, FoldStage<T, BM, BN, BK>, Stage<T, BM, BN, BK>>::type St;
    typedef BfStage<BM, BN> Sb;
    constexpr size_t CBYTES = sizeof(CT) * BM * LDC;
    // two LDS stages (one barrier per K step) for float32, where they fit
    // beside a second resident block; the float64 loop measured faster with
    // a single stage
    constexpr int NS = ((sizeof(T) == 4 && 2 * sizeof(St) <= 72 * 1024) || (MODE == 0 && FOLD)) ? 2 : 1;
    constexpr size_t STB = MODE == 2 ? sizeof(Sb) : NS * sizeof(St);
    constexpr size_t SBYTES = STB > CBYTES ? STB : CBYTES;
    static_assert(SBYTES >= sizeof(double) * 256 * NBP, "row reduction buffer");
    __shared__ __attribute__((aligned(16))) char smem[SBYTES];
    extern __shared__ __attribute__((aligned(16))) char dsm[];
    CT* Cs = reinterpret_cast<CT*>(smem);
    CE* Et = reinterpret_cast<CE*>(dsm);          // [3][BM][2 nmax + 1] when GEN
    int* Roff = reinterpret_cast<int*>(dsm + (size_t)3 * BM * (2 * a.nmax + 1) * sizeof(CE));  // [ne]

    // XCD-aware remap: consecutive workgroup ids land on different XCDs
    // (round-robin over 8); each XCD gets a contiguous range of lin, i.e. a
    // band of row tiles with all S column slices, so that its L2 serves the
    // A strips of few row tiles and each B tile to several row tiles (with
    // the slice index outermost, an XCD ran ~64 row tiles of one slice and
    // fetched both operands of every tile from beyond its L2).
    const int G = gridDim.x;
    const int bid = blockIdx.x;
    const int per = G / 8;
    const int lin = (bid % 8) * per + bid / 8;
    const int R = tiles_m * a.S;                  // regular blocks: one per (row tile, slice)
    int kh = 0;                                   // entries of the folded sum
    int* Hs = reinterpret_cast<int*>(dsm);        // [ne] rows of B+ (FOLD)
    int* Ps = Hs + a.ne;                          // [ne] rows of B-
    if constexpr (FOLD) {
        kh = a.kh[0];
        for (int i = threadIdx.x; i < kh; i += 256) {
            Hs[i] = a.half[i];
            Ps[i] = a.pair[i];
        }
        __syncthreads();
    }
    if (lin >= R + a.helpers) return;
    const int NE = 2 * a.nmax + 1;
    if constexpr (GEN) {
        // table offsets of each R_e, packed 8 bits per axis
        for (int r = threadIdx.x; r < a.ne; r += 256) {
            const int* rr = a.Re + 3 * r;
            Roff[r] = (rr[0] + a.nmax) | ((rr[1] + a.nmax) << 8) | ((rr[2] + a.nmax) << 16);
        }
    }
    // Segments.  A regular block (lin < R) runs the first `keep` column tiles
    // of slice s of row tile mt and writes its partial sums to slot s; helper
    // h = lin - R runs the remaining tiles of the slices of regular blocks
    // [h R / H, (h + 1) R / H) in turn and writes theirs to slot S + s.  When
    // the regular blocks leave some of the two slots per CU empty, the helpers
    // fill them and `keep` evens out the work of the two kinds of block.
    // Only the instantiations in BAL take helpers (fused_balance): in the
    // float64 and split-bf16 ones below 16 bands the segment state cost more
    // registers than the balance saved (fcc 20^3: FP64 254 -> 269 ms per
    // launch, split-BF16 219 -> 237), elsewhere it gained 3-9 %.
    constexpr bool BAL = fused_balanced_c(NBP, MODE);
    const bool helper = BAL && lin >= R;
    const int rb0 = helper ? (int)((long)(lin - R) * R / a.helpers) : lin;
    const int rb1 = helper ? (int)((long)(lin - R + 1) * R / a.helpers) : lin + 1;
    for (int rb = rb0; rb < rb1; ++rb) {
        if (rb > rb0) __syncthreads();                // the previous segment is done with LDS
        const int s = rb % a.S;
        const int mt = rb / a.S;
        const int slot = helper ? a.S + s : s;
        const int j0 = helper ? a.keep : 0;
        const int j1 = BAL ? (helper ? 0x7fffffff : a.keep) : 0x7fffffff;
        const int m0 = mt * BM;
        if constexpr (GEN) {
            for (int idx = threadIdx.x; idx < 3 * BM * NE; idx += 256) {
                const int ax = idx / (BM * NE), rem = idx % (BM * NE);
                const int row = rem / NE, j = rem % NE;
                const int kr = m0 + row;
                double x = kr < a.nk ? a.kfrac[3 * (size_t)kr + ax] * (double)(j - a.nmax) : 0.0;
                x -= rint(x);
                double sn, cs;
                sincospi(2.0 * x, &sn, &cs);
                Et[idx] = mk2((TE)cs, (TE)sn);
            }
            __syncthreads();
        }
        // phase of (local row m, R_e index kk), zero outside the valid range
        auto phase = [&](int m, int kk) -> CE {
            if (m0 + m >= a.nk || kk >= a.ne) return mk2(TE(0), TE(0));
            const int off = Roff[kk];
            const CE p0 = Et[(0 * BM + m) * NE + (off & 255)];
            const CE p1 = Et[(1 * BM + m) * NE + ((off >> 8) & 255)];
            const CE p2 = Et[(2 * BM + m) * NE + (off >> 16)];
            return cmulx(cmulx(p0, p1), p2);
        };

        const int nb = a.nb, nm = a.nm;
        const int tid = threadIdx.x;
        const int r = tid / TPR, sub = tid % TPR;
        const int k = m0 + r;
        const long ncols = (long)a.qc * nm * NB2;
        const double2* U = reinterpret_cast<const double2*>(a.U);
        const bool active_row = k < a.nk;
        // a Gaussian factor exp(-y^2) is exactly zero in TE beyond this y^2
        const double ylim = sizeof(TE) == 8 ? 750.0 : 110.0;

        // Items of one run are bands x0 .. x0 + RUN - 1 of one band block, with
        // x0 = (sub*JI) % NBP the same for every run of the thread.
        const int x0 = (sub * JI) % NBP;
        // U_k columns x0 .. x0 + RUN - 1 (phase 1), in TE
        auto load_uk = [&](CE (&uk)[RUN][NBP]) {
#pragma unroll
            for (int t = 0; t < RUN; ++t)
#pragma unroll
                for (int jj = 0; jj < NBP; ++jj) {
                    const int n = x0 + t;
                    const double2 u = (active_row && n < nb && jj < nb) ? U[((size_t)k * nb + jj) * nb + n]
                                                                        : make_double2(0.0, 0.0);
                    uk[t][jj] = mk2((TE)u.x, (TE)u.y);
                }
        };
        // Per-row state kept over the block's tiles: the Im Sigma accumulators of
        // the row's bands and, in the float32 modes, eps_nk and the U_k columns
        // (the float64 mode reloads those per tile to stay within its registers).
        constexpr bool HOIST = (MODE == 1 && NBP < 16) || (MODE == 2 && RUN * NBP <= 16);
        double acc[NBP], acc2[RE ? NBP : 1];
        double eps_h[HOIST ? NBP : 1];
        CE uk_h[HOIST ? RUN : 1][NBP];
#pragma unroll
        for (int n = 0; n < NBP; ++n) acc[n] = 0.0;
        if constexpr (RE) {
#pragma unroll
            for (int n = 0; n < NBP; ++n) acc2[n] = 0.0;
        }
        if constexpr (HOIST) {
#pragma unroll
            for (int n = 0; n < NBP; ++n) eps_h[n] = (active_row && n < nb) ? a.eps[(size_t)k * nb + n] : 0.0;
            load_uk(uk_h);
        }
        const double inv_sig = 1.0 / a.sigma;

        for (int j = j0, nt = s + j0 * a.S; j < j1 && nt < tiles_n; ++j, nt += a.S) {
            const long n0 = (long)nt * BN;
            // The main loop runs at raised wave priority and the epilogue at the
            // normal one: where one resident block is in its main loop and the
            // other in its epilogue, the SIMD's arbiter then keeps the MFMA stream
            // fed first and fills the gaps with the epilogue (FP64 170 -> 163 ms per
            // 1260-q launch, FP32 -2 %, split-BF16 -2 %).
            __builtin_amdgcn_s_setprio(1);
            if constexpr (MODE == 2) {
                constexpr int RB = BfWaves<BM, BN>::RB;
                f4 cr[4 * RB], ci[4 * RB];
                const uint16_t* Ap = reinterpret_cast<const uint16_t*>(a.phi_k);
                const uint16_t* Bp = reinterpret_cast<const uint16_t*>(a.B);
                auto agen = [&](int m, int kk) -> float2 { return phase(m, kk); };
                bf16_mainloop<BM, BN, GEN>(*reinterpret_cast<Sb*>(smem), Ap, a.ldk, (long)a.nk * a.ldk, a.nk, m0, Bp,
                                           a.ldk_b, ncols * a.ldk_b, ncols, n0, a.kpad, agen, cr, ci);
                const int lane = tid & 63, wave = tid >> 6;
                constexpr int WN = BN / 64;
                const int wm = wave / WN, wn = wave % WN;
                for (int q = 0; q < RB; ++q)
                    for (int c = 0; c < 4; ++c)
                        for (int i = 0; i < 4; ++i) {
                            const int row = wm * 16 * RB + q * 16 + 4 * (lane >> 4) + i;
                            const int col = wn * 64 + c * 16 + (lane & 15);
                            Cs[row * LDC + col] = make_float2(cr[q * 4 + c][i], ci[q * 4 + c][i]);
                        }
            } else {
                const CT* phi = reinterpret_cast<const CT*>(a.phi_k);
                const CT* Bm = reinterpret_cast<const CT*>(a.B);
                auto afetch = [&](int m, int kk) -> CT {
                    if constexpr (GEN) {
                        return phase(m, kk);
                    } else {
                        const int row = m0 + m;
                        if (row < a.nk && kk < a.ne) return phi[(size_t)row * a.ldk + kk];
                        return cz<T>();
                    }
                };
                auto bfetch = [&](int kk, int n) -> CT {
                    const long col = n0 + n;
                    if (kk < a.ne && col < ncols) return Bm[(size_t)kk * ncols + col];
                    return cz<T>();
                };
                constexpr int RB = CWaves<BM, BN>::RB;
                typename Cx<T>::acc cr[4 * RB], ci[4 * RB];
                if constexpr (FOLD) {
                    // entry h of the halved sum: B+ in row half[h], B- in row pair[h]
                    auto bfold = [&](int h, int n) -> CPair<CT> {
                        const long col = n0 + n;
                        CPair<CT> v;
                        if (h < kh && col < ncols) {
                            v.p = Bm[(size_t)Hs[h] * ncols + col];
                            v.m = Bm[(size_t)Ps[h] * ncols + col];
                        } else {
                            v.p = cz<T>();
                            v.m = cz<T>();
                        }
                        return v;
                    };
                    auto afold = [&](int m, int h) -> CT {
                        const int row = m0 + m;
                        if (row < a.nk && h < kh) return phi[(size_t)row * a.ldk + h];
                        return cz<T>();
                    };
                    cfold_mainloop<T, BM, BN, BK, decltype(afold), decltype(bfold), NS>(
                        reinterpret_cast<St*>(smem), kh, afold, bfold, cr, ci);
                } else {
                    cgemm_mainloop<T, BM, BN, BK, decltype(afetch), decltype(bfetch), false, NS>(
                        reinterpret_cast<St*>(smem), a.ne, afetch, bfetch, cr, ci);
                }
                const int lane = tid & 63, wave = tid >> 6;
                constexpr int WN = BN / 64;
                const int wm = wave / WN, wn = wave % WN;
                if constexpr (WSTORE) {
                    // the Wannier-basis tile itself, straight to memory (the main
                    // loop's last barrier has released the LDS stage)
                    CT* G = reinterpret_cast<CT*>(a.gout);
                    for (int q = 0; q < RB; ++q)
                        for (int c = 0; c < 4; ++c) {
                            const long col = n0 + wn * 64 + c * 16 + (lane & 15);
                            for (int i = 0; i < 4; ++i) {
                                const int row = m0 + wm * 16 * RB + q * 16 + crow<T>(lane, i);
                                if (row >= a.nk || col >= ncols) continue;
                                CT v;
                                v.x = cr[q * 4 + c][i];
                                v.y = ci[q * 4 + c][i];
                                G[(size_t)row * ncols + col] = v;
                            }
                        }
                    __builtin_amdgcn_s_setprio(0);
                    continue;
                }
                for (int q = 0; q < RB; ++q)
                    for (int c = 0; c < 4; ++c)
                        for (int i = 0; i < 4; ++i) {
                            const int row = wm * 16 * RB + q * 16 + crow<T>(lane, i);
                            const int col = wn * 64 + c * 16 + (lane & 15);
                            CT v;
                            v.x = cr[q * 4 + c][i];
                            v.y = ci[q * 4 + c][i];
                            Cs[row * LDC + col] = v;
                        }
            }
            __builtin_amdgcn_s_setprio(0);
            __syncthreads();
            // The band loops of both phases stop at nb for up to 8 padded bands; at
            // 16 they run over the zero padding (G, U_k and the k+q columns are
            // zero there), so they unroll completely and their arrays stay in
            // registers instead of scratch.
            // phase 1: V = G U_k for the thread's items (b, n), all rows i of V,
            // written over G in LDS.  With JI >= NBP a thread owns whole band
            // blocks; otherwise the TPR threads of a row share the single block
            // and wait for each other between reading G and writing V.
            {
                CE uk[RUN][NBP];
                if constexpr (HOIST) {
#pragma unroll
                    for (int t = 0; t < RUN; ++t)
#pragma unroll
                        for (int jj = 0; jj < NBP; ++jj) uk[t][jj] = uk_h[t][jj];
                } else {
                    load_uk(uk);
                }
#pragma unroll
                for (int rr = 0; rr < NRUN; ++rr) {
                    const int b = (sub * JI + rr * RUN) / NBP;
                    CT* Gt = Cs + r * LDC + b * NB2;
                    CE v[RUN][NBP];
#pragma unroll
                    for (int t = 0; t < RUN; ++t)
#pragma unroll
                        for (int i = 0; i < NBP; ++i) v[t][i] = mk2(TE(0), TE(0));
                    if (active_row) {
#pragma unroll
                        for (int i = 0; i < NBP; ++i) {
                            if (NBP < 16 && i >= nb) break;
#pragma unroll
                            for (int jj = 0; jj < NBP; ++jj) {
                                if (NBP < 16 && jj >= nb) break;
                                const CT g = Gt[i * NBP + jj];
                                const TE gx = (TE)g.x, gy = (TE)g.y;
#pragma unroll
                                for (int t = 0; t < RUN; ++t) {
                                    const CE u = uk[t][jj];
                                    v[t][i].x += gx * u.x - gy * u.y;
                                    v[t][i].y += gx * u.y + gy * u.x;
                                }
                            }
                        }
                    }
                    if constexpr (JI < NBP) __syncthreads();   // all of G has been read
                    if (active_row) {
#pragma unroll
                        for (int t = 0; t < RUN; ++t) {
                            const int n = x0 + t;
                            if (n >= nb) break;
#pragma unroll
                            for (int i = 0; i < NBP; ++i) {
                                if (NBP < 16 && i >= nb) break;
                                CT o;
                                o.x = (T)v[t][i].x;
                                o.y = (T)v[t][i].y;
                                Gt[i * NBP + n] = o;
                            }
                        }
                    }
                }
                if constexpr (JI < NBP) __syncthreads();
            }
            // phase 2: g_mn = sum_i conj(U_k+q[i][m]) V[i][n] for the thread's
            // items (b, m), all n; weights and |g|^2 accumulated per n (Im Sigma)
            // or per run (phonon sums)
            double pp[NRUN], pl[NRUN], pt[TR ? NRUN : 1];
#pragma unroll
            for (int rr = 0; rr < NRUN; ++rr) {
                pp[rr] = 0.0;
                pl[rr] = 0.0;
                if constexpr (TR) pt[rr] = 0.0;
            }
            if (active_row) {
#pragma unroll
                for (int rr = 0; rr < NRUN; ++rr) {
                    const int b = (sub * JI + rr * RUN) / NBP;
                    if (x0 >= nb) continue;
                    const long gblk = n0 / NB2 + b;            // (q_local, nu)
                    const int ql = (int)(gblk / nm), nu = (int)(gblk % nm);
                    if (ql >= a.qc) continue;
                    const double scv = a.sc[(size_t)ql * nm + nu];
                    if (scv == 0.0 && !STORE && !POLE) continue;
                    const int q = a.q0 + ql;
                    // states at k+q: a member of the k set (grid runs) or per pair
                    const double2* Uq;
                    const double* eq;
                    const double* fq;
                    const double* vq = nullptr;   // velocities at k+q (transport mode, grid runs)
                    if (a.kq) {
                        const int kq = a.kq[(size_t)k * a.nq_total + q];
                        if ((unsigned)kq >= (unsigned)a.nk) {           // invalid map entry: no access
                            if constexpr (POLE) {
                                for (int t = 0; t < RUN; ++t) {
                                    if (x0 + t >= nb) break;
                                    double* rec = a.rec + ((((size_t)k * a.qc + ql) * nm + nu) * nb + x0 + t) * (4 + NBP);
                                    for (int j = 0; j < 4 + NBP; ++j) rec[j] = 0.0;
                                }
                            }
                            continue;
                        }
                        Uq = U + (size_t)kq * nb * nb;
                        eq = a.eps + (size_t)kq * nb;
                        fq = a.ftab + (size_t)kq * nb;
                        if constexpr (TR) vq = a.vel + (size_t)kq * nb * 3;
                    } else {
                        const size_t pr = (size_t)k * a.qc + ql;
                        Uq = reinterpret_cast<const double2*>(a.U_pair) + pr * nb * nb;
                        eq = a.eps_pair + pr * nb;
                        fq = a.f_pair + pr * nb;
                        if constexpr (TR) vq = a.vel_pair + pr * nb * 3;
                    }
                    const double w = a.omega[(size_t)ql * nm + nu];
                    const double nB = a.nbose[(size_t)ql * nm + nu];
                    // the run's bands in groups of RT: split-bf16 takes one band at a time so
                    // its k+q eigenvector column and sums fit beside the wider main loop's state
#pragma unroll 1
                    for (int tb = 0; tb < RUN; tb += RT) {
                        CE uq[RT][NBP];
                        double em[RT], fm[RT], dm[RT];
                        double vm[TR ? RT : 1][3];
                        bool mv[RT];
#pragma unroll
                        for (int t = 0; t < RT; ++t) {
                            const int m = x0 + tb + t;
                            mv[t] = m < nb;
                            em[t] = mv[t] ? eq[m] : 0.0;
                            fm[t] = mv[t] ? fq[m] : 0.0;
                            if constexpr (PH) {
                                const double ym = (em[t] - a.mu) * inv_sig;
                                dm[t] = mv[t] ? exp(-ym * ym) : 0.0;
                            }
                            if constexpr (TR) {
                                for (int c = 0; c < 3; ++c) vm[t][c] = mv[t] ? vq[3 * m + c] : 0.0;
                            }
#pragma unroll
                            for (int i = 0; i < NBP; ++i) {
                                const double2 u = (mv[t] && i < nb) ? Uq[i * nb + m] : make_double2(0.0, 0.0);
                                uq[t][i] = mk2((TE)u.x, (TE)u.y);
                            }
                        }
                        const CT* Vt = Cs + r * LDC + b * NB2;
#pragma unroll
                        for (int n = 0; n < NBP; ++n) {
                            if (n >= nb) break;
                            double epsn;
                            if constexpr (HOIST) epsn = eps_h[n]; else epsn = a.eps[(size_t)k * nb + n];
                            TE W[RT], WL[RT], WT[TR ? RT : 1];
                            bool need = STORE || POLE;
                            if constexpr (PH) {
                                // Eq. (9): [f_nk - f_m,k+q] exp(-((eps_nk - eps_m,k+q - omega)/sigma)^2);
                                // Eq. (11): exp(-((eps_nk - mu)/sigma)^2) exp(-((eps_m,k+q - mu)/sigma)^2)
                                const double fn = a.ftab[(size_t)k * nb + n];
                                const double yn = (epsn - a.mu) * inv_sig;
                                const double dn = exp(-yn * yn);
                                // Eq. (55): 1 - v_nk . v_m,k+q / |v_nk|^2, 1 at a zero velocity
                                double vn[3] = {0.0, 0.0, 0.0}, inv_vv = 0.0;
                                if constexpr (TR) {
                                    for (int c = 0; c < 3; ++c) vn[c] = a.vel[((size_t)k * nb + n) * 3 + c];
                                    const double vv = vn[0] * vn[0] + vn[1] * vn[1] + vn[2] * vn[2];
                                    inv_vv = vv > 1e-18 ? 1.0 / vv : 0.0;
                                }
#pragma unroll
                                for (int t = 0; t < RT; ++t) {
                                    W[t] = TE(0);
                                    WL[t] = TE(0);
                                    if constexpr (TR) WT[t] = TE(0);
                                    if (!mv[t]) continue;
                                    const double y = (epsn - em[t] - w) * inv_sig;
                                    const double s1 = y * y;
                                    if (s1 < ylim) W[t] = (TE)(fn - fm[t]) * fexp((TE)(-s1));
                                    WL[t] = (TE)(dn * dm[t]);
                                    if constexpr (TR) {
                                        const double fac = inv_vv > 0.0
                                            ? 1.0 - (vn[0] * vm[t][0] + vn[1] * vm[t][1] + vn[2] * vm[t][2]) * inv_vv
                                            : 1.0;
                                        WT[t] = (TE)(dn * dm[t] * fac);
                                    }
                                    need = need || (s1 < ylim) || (WL[t] != TE(0));
                                }
                            } else if constexpr (RE) {
                                // Eq. (3), Re 1/(x + i delta) = x/(x^2 + delta^2), delta = sigma:
                                // on shell x = eps_nk - eps_m,k+q +- omega; at eps_F x = mu - eps_m,k+q +- omega
                                const double d2 = a.sigma * a.sigma;
                                need = true;
#pragma unroll
                                for (int t = 0; t < RT; ++t) {
                                    W[t] = TE(0);
                                    WL[t] = TE(0);
                                    if (!mv[t]) continue;
                                    const double A1 = nB + fm[t], A2 = nB + 1.0 - fm[t];
                                    const double x1 = epsn - em[t] + w, x2 = epsn - em[t] - w;
                                    const double y1 = a.mu - em[t] + w, y2 = a.mu - em[t] - w;
                                    W[t] = (TE)(A1 * x1 / (x1 * x1 + d2) + A2 * x2 / (x2 * x2 + d2));
                                    WL[t] = (TE)(A1 * y1 / (y1 * y1 + d2) + A2 * y2 / (y2 * y2 + d2));
                                }
                            } else {
#pragma unroll
                                for (int t = 0; t < RT; ++t) {
                                    W[t] = TE(0);
                                    WL[t] = TE(0);
                                    if (STORE || POLE || !mv[t]) continue;
                                    const double x = epsn - em[t];
                                    const double y1 = (x + w) * inv_sig, y2 = (x - w) * inv_sig;
                                    const double s1 = y1 * y1, s2 = y2 * y2;
                                    if (s1 < ylim) W[t] += (TE)(nB + fm[t]) * fexp((TE)(-s1));
                                    if (s2 < ylim) W[t] += (TE)(nB + 1.0 - fm[t]) * fexp((TE)(-s2));
                                    need = need || (s1 < ylim) || (s2 < ylim);
                                }
                            }
                            if (!need) continue;
                            TE gr[RT], gi[RT];
#pragma unroll
                            for (int t = 0; t < RT; ++t) {
                                gr[t] = TE(0);
                                gi[t] = TE(0);
                            }
#pragma unroll
                            for (int i = 0; i < NBP; ++i) {
                                if (NBP < 16 && i >= nb) break;
                                const CT vv = Vt[i * NBP + n];
                                const TE vx = (TE)vv.x, vy = (TE)vv.y;
#pragma unroll
                                for (int t = 0; t < RT; ++t) {
                                    // conj(u) * v
                                    gr[t] += uq[t][i].x * vx + uq[t][i].y * vy;
                                    gi[t] += uq[t][i].x * vy - uq[t][i].y * vx;
                                }
                            }
#pragma unroll
                            for (int t = 0; t < RT; ++t) {
                                if (!mv[t]) continue;
                                if (STORE) {
                                    reinterpret_cast<double2*>(a.gkq)
                                        [((((size_t)k * a.nq_total + q) * nm + nu) * nb + x0 + tb + t) * nb + n] =
                                        make_double2((double)gr[t], (double)gi[t]);
                                } else if (PH) {
                                    const TE g2 = gr[t] * gr[t] + gi[t] * gi[t];
                                    pp[rr] += (double)(g2 * W[t]);
                                    pl[rr] += (double)(g2 * WL[t]);
                                    if constexpr (TR) pt[rr] += (double)(g2 * WT[TR ? t : 0]);
                                } else if (RE) {
                                    const TE g2 = gr[t] * gr[t] + gi[t] * gi[t];
                                    acc[n] += (double)(g2 * W[t]);
                                    acc2[n] += (double)(g2 * WL[t]);
                                } else if (POLE) {
                                    double* rec = a.rec + ((((size_t)k * a.qc + ql) * nm + nu) * nb + x0 + tb + t) * (4 + NBP);
                                    rec[4 + n] = (double)(gr[t] * gr[t] + gi[t] * gi[t]);
                                    if (n == 0) {
                                        const double xi = em[t] - a.mu;
                                        const bool kept = scv != 0.0;
                                        rec[0] = xi - w;
                                        rec[1] = xi + w;
                                        rec[2] = kept ? nB + fm[t] : 0.0;
                                        rec[3] = kept ? nB + 1.0 - fm[t] : 0.0;
                                        for (int j = nb; j < NBP; ++j) rec[4 + j] = 0.0;   // padded bands
                                    }
                                } else {
                                    acc[n] += (double)((gr[t] * gr[t] + gi[t] * gi[t]) * W[t]);
                                }
                            }
                            // keep the scheduler from overlapping band iterations (register pressure)
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                }
            }
            if constexpr (PH) {
                // fixed-order sums over the tile's k rows, per band block (q, nu):
                // slot (b, r, j) holds run j of row r; rows are summed after the
                // slots of each row, for Eq. (9) and then Eq. (11)
                constexpr int NBLK = BN / NB2;
                constexpr int SPB = NBP / RUN;                  // runs per band block and row
                static_assert(SBYTES >= sizeof(double) * NBLK * BM * SPB, "phonon reduction buffer");
                double* red = reinterpret_cast<double*>(smem);
                const int jslot = x0 / RUN;
                const size_t ncb = (size_t)a.qc * nm;
#pragma unroll
                for (int kind = 0; kind < (TR ? 3 : 2); ++kind) {
                    __syncthreads();                            // V, or the previous pass, no longer read
#pragma unroll
                    for (int rr = 0; rr < NRUN; ++rr) {
                        const int b = (sub * JI + rr * RUN) / NBP;
                        double val = kind == 0 ? pp[rr] : pl[rr];
                        if constexpr (TR) val = kind == 2 ? pt[rr] : val;
                        red[((size_t)b * BM + r) * SPB + jslot] = val;
                    }
                    __syncthreads();
                    for (int t = tid; t < NBLK * BM; t += 256) {
                        double v = 0.0;
                        for (int j = 0; j < SPB; ++j) v += red[(size_t)t * SPB + j];
                        red[(size_t)t * SPB] = v;
                    }
                    __syncthreads();
                    for (int b = tid; b < NBLK; b += 256) {
                        const long gblk = n0 / NB2 + b;         // q_local * nm + nu
                        if (gblk >= (long)ncb) continue;
                        double v = 0.0;
                        for (int rw = 0; rw < BM; ++rw) v += red[((size_t)b * BM + rw) * SPB];
                        a.part_ph[((size_t)kind * tiles_m + mt) * ncb + gblk] = v;
                    }
                }
            }
            __syncthreads();
        }
        if constexpr (KIND == 1 || KIND == 2 || KIND == 4 || KIND == 5 || KIND == 6) continue;
        // fixed-order reduction over the TPR threads of each row (real-part
        // mode: the on-shell sums, then the sums at eps_F)
        double* red = reinterpret_cast<double*>(smem);   // [BM][TPR][NBP]
#pragma unroll
        for (int pass = 0; pass < (RE ? 2 : 1); ++pass) {
            if (pass) __syncthreads();
#pragma unroll
            for (int n = 0; n < NBP; ++n) red[(size_t)tid * NBP + n] = pass ? acc2[RE ? n : 0] : acc[n];
            __syncthreads();
            double* dst = pass ? a.part2 : a.part;
            if (active_row) {
                for (int n = sub; n < nb; n += TPR) {
                    double t = 0.0;
                    for (int u = 0; u < TPR; ++u) t += red[((size_t)r * TPR + u) * NBP + n];
                    dst[((size_t)slot * a.nk + k) * nb + n] = t;
                }
            }
        }
    }   // segments
}

// a6 for the split-bf16 path: float32 g(R_e,q) [ne][qc][nm*nb*nb] ->
// four bf16 planes [4][qc*nm*NBP*NBP][kpad] with R_e contiguous (the K index
// of the R_e -> k contraction), transposed through LDS in 64 x 64 tiles.
__global__ __launch_bounds__(256) void mode_rotate_bf16_kernel(int ne, int qc, int nm, int nb, int nbp, int kpad,
                                                              const float2* __restrict__ in,
                                                              const double2* __restrict__ evec,
                                                              const double* __restrict__ sc,
                                                              const int32_t* __restrict__ ndeg_fold,
                                                              const double2* __restrict__ Lq,
                                                              const int32_t* __restrict__ Re,
                                                              uint16_t* __restrict__ out)
{
    __shared__ float2 tile[64][65];
    const int q = blockIdx.x;
    const int e0 = blockIdx.y * 64;
    const int nbp2 = nbp * nbp;
    const long ncols = (long)qc * nm * nbp2;
    const long plane = ncols * kpad;
    const int tid = threadIdx.x;
    for (int nu = 0; nu < nm; ++nu) {
        const float s = (float)sc[(size_t)q * nm + nu];
        for (int ij0 = 0; ij0 < nbp2; ij0 += 64) {
            // compute: item (e_local, ij_local), ij fastest for coalesced reads
            for (int it = tid; it < 64 * 64; it += 256) {
                const int el = it / 64, il = it % 64;
                const int e = e0 + el, ij = ij0 + il;
                float2 v = make_float2(0.f, 0.f);
                if (ij < nbp2 && e < ne && s != 0.f) {
                    const int i = ij / nbp, j = ij % nbp;
                    const float wf = ndeg_fold ? s / (float)ndeg_fold[e] : s;
                    if (i < nb && j < nb) {
                        const float2* x = in + ((size_t)e * qc + q) * nm * nb * nb + i * nb + j;
                        float re = 0.f, im = 0.f;
                        for (int aa = 0; aa < nm; ++aa) {
                            const double2 ev = evec[((size_t)q * nm + aa) * nm + nu];
                            const float2 g = x[(size_t)aa * nb * nb];
                            re += g.x * (float)ev.x - g.y * (float)ev.y;
                            im += g.x * (float)ev.y + g.y * (float)ev.x;
                        }
                        v = make_float2(re * wf, im * wf);
                    }
                }
                if (Lq && ij < nbp2 && e < ne) {
                    const int i = ij / nbp, j = ij % nbp;
                    const int32_t* rv = Re + 3 * (size_t)e;
                    if (i == j && i < nb && (rv[0] | rv[1] | rv[2]) == 0) {
                        const double2 l = Lq[(size_t)q * nm + nu];
                        v.x += (float)l.x;
                        v.y += (float)l.y;
                    }
                }
                tile[il][el] = v;
            }
            __syncthreads();
            // write: row (column of B) ij, 8 consecutive R_e per item
            for (int it = tid; it < 64 * 8; it += 256) {
                const int il = it / 8, part = it % 8;
                const int ij = ij0 + il;
                if (ij >= nbp2) continue;
                const int eb = e0 + part * 8;
                if (eb >= kpad) continue;
                const long col = ((long)q * nm + nu) * nbp2 + ij;
                uint32_t hr[4], lr[4], hi[4], li[4];
                for (int t = 0; t < 4; ++t) {
                    hr[t] = lr[t] = hi[t] = li[t] = 0u;
                }
                for (int t = 0; t < 8; ++t) {
                    const float2 v = tile[il][part * 8 + t];
                    const __hip_bfloat16 xh = __float2bfloat16(v.x);
                    const __hip_bfloat16 xl = __float2bfloat16(v.x - __bfloat162float(xh));
                    const __hip_bfloat16 yh = __float2bfloat16(v.y);
                    const __hip_bfloat16 yl = __float2bfloat16(v.y - __bfloat162float(yh));
                    const int sh = 16 * (t & 1);
                    hr[t >> 1] |= (uint32_t)__builtin_bit_cast(uint16_t, xh) << sh;
                    lr[t >> 1] |= (uint32_t)__builtin_bit_cast(uint16_t, xl) << sh;
                    hi[t >> 1] |= (uint32_t)__builtin_bit_cast(uint16_t, yh) << sh;
                    li[t >> 1] |= (uint32_t)__builtin_bit_cast(uint16_t, yl) << sh;
                }
                uint16_t* o = out + (size_t)col * kpad + eb;
                *reinterpret_cast<uint4*>(o) = make_uint4(hr[0], hr[1], hr[2], hr[3]);
                *reinterpret_cast<uint4*>(o + plane) = make_uint4(lr[0], lr[1], lr[2], lr[3]);
                *reinterpret_cast<uint4*>(o + 2 * plane) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
                *reinterpret_cast<uint4*>(o + 3 * plane) = make_uint4(li[0], li[1], li[2], li[3]);
            }
            __syncthreads();
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

__global__ void reduce_partials_diff_kernel(int nk, int nb, int S, const double* __restrict__ A,
                                            const double* __restrict__ B, double scale, int accumulate,
                                            double* __restrict__ out)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)nk * nb;
    if (idx >= total) return;
    double t = 0.0;
    for (int s = 0; s < S; ++s) t += A[(size_t)s * total + idx] - B[(size_t)s * total + idx];
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

// raw[0] = sum_i exp(-((eps_i - mu)/sigma)^2): one block, strided partial
// sums then a fixed tree (bit-reproducible)
__global__ __launch_bounds__(256) void dos_raw_kernel(size_t n, const double* __restrict__ eps, double mu,
                                                     double inv_sig, double* __restrict__ raw)
{
    __shared__ double part[256];
    double t = 0.0;
    for (size_t i = threadIdx.x; i < n; i += 256) {
        const double y = (eps[i] - mu) * inv_sig;
        t += exp(-y * y);
    }
    part[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) raw[0] = part[0];
}

// Eq. (9) and Eq. (11) from the per-row-tile sums: fixed-order sum over row
// tiles, then the normalisations (the Gaussian 1/(sigma sqrt pi) per delta,
// 2 pi / N_k for Pi'', 1/(N(eps_F) omega N_k) for lambda with
// N(eps_F) = raw / (N_k sigma sqrt pi))
__global__ void phonon_finalize_kernel(int qc, int nm, int tiles_m, const double* __restrict__ part_ph,
                                       const double* __restrict__ omega, double omega_cut,
                                       const double* __restrict__ raw_dos, int nk, double sigma,
                                       double* __restrict__ pi_im, double* __restrict__ lam,
                                       double* __restrict__ lam_tr)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncb = qc * nm;
    if (idx >= ncb) return;
    double P = 0.0, L = 0.0, Lt = 0.0;
    for (int t = 0; t < tiles_m; ++t) {
        P += part_ph[(size_t)t * ncb + idx];
        L += part_ph[((size_t)tiles_m + t) * ncb + idx];
        if (lam_tr) Lt += part_ph[((size_t)2 * tiles_m + t) * ncb + idx];
    }
    const double w = omega[idx];
    const bool keep = w >= omega_cut;
    constexpr double kPi = 3.141592653589793;
    const double gnorm = 1.0 / (sigma * sqrt(kPi));
    if (pi_im) pi_im[idx] = keep ? 2.0 * kPi * gnorm * P / (double)nk : 0.0;
    const double raw = raw_dos[0];
    if (lam) lam[idx] = (keep && raw > 0.0) ? gnorm * L / (raw * w) : 0.0;
    if (lam_tr) lam_tr[idx] = (keep && raw > 0.0) ? gnorm * Lt / (raw * w) : 0.0;
}

inline unsigned blocks_for(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <int MODE, int NBP>
void launch_fused_t(const FusedArgs& a, int num_cu, hipStream_t stream) {
    constexpr int BM = FusedShape<MODE, NBP>::BM, BN = FusedShape<MODE, NBP>::BN;
    static_assert(BM == fused_tile_rows_c(NBP, MODE != 0), "tile rows known to the host code");
    const int tiles_m = (a.nk + BM - 1) / BM;
    const long ncols = (long)a.qc * a.nm * NBP * NBP;
    const int tiles_n = (int)((ncols + BN - 1) / BN);
    const long total = (long)tiles_m * a.S + a.helpers;
    const long G = ((total + 7) / 8) * 8;
    (void)num_cu;
    (void)tiles_n;
    // the float64 path always reads its phases from a table
    if (MODE == 0 && a.nmax > 0) throw HipFailure{(int)hipErrorInvalidValue, "fused_k_kernel (f64, nmax > 0)", __FILE__, __LINE__};
    constexpr bool CAN_GEN = MODE != 0;
    const bool gen = CAN_GEN && a.nmax > 0;
    // the folding instantiations read the halved R list (kh, half, pair)
    if (fused_fold_c(NBP, MODE) && !(a.kh && a.half && a.pair))
        throw HipFailure{(int)hipErrorInvalidValue, "fused_k_kernel (folded sum without its R list)", __FILE__,
                         __LINE__};
    const bool fold = fused_fold_c(NBP, MODE);
    const size_t dyn = gen ? (size_t)3 * BM * (2 * a.nmax + 1) * 8 + 4 * (size_t)a.ne
                           : fold ? 8 * (size_t)a.ne : 0;
    const dim3 grid((unsigned)G), block(256);
    auto go = [&](auto kind) {
        constexpr int K = decltype(kind)::value;
        if (gen)
            fused_k_kernel<MODE, NBP, K, CAN_GEN><<<grid, block, dyn, stream>>>(a, tiles_m, tiles_n);
        else
            fused_k_kernel<MODE, NBP, K, false><<<grid, block, dyn, stream>>>(a, tiles_m, tiles_n);
    };
    if constexpr (MODE != 2) {
        if (a.gout) {
            go(std::integral_constant<int, 6>());
            launch_check("fused_k_kernel");
            return;
        }
    }
    if (a.gkq) go(std::integral_constant<int, 1>());
    else if (a.rec) go(std::integral_constant<int, 4>());
    else if (a.part_ph && a.vel) go(std::integral_constant<int, 5>());
    else if (a.part_ph) go(std::integral_constant<int, 2>());
    else if (a.part2) go(std::integral_constant<int, 3>());
    else go(std::integral_constant<int, 0>());
    launch_check("fused_k_kernel");
}

template <int MODE>
void launch_fused_nbp(const FusedArgs& a, int num_cu, hipStream_t stream) {
    switch (a.nbp) {
        case 1: launch_fused_t<MODE, 1>(a, num_cu, stream); break;
        case 2: launch_fused_t<MODE, 2>(a, num_cu, stream); break;
        case 4: launch_fused_t<MODE, 4>(a, num_cu, stream); break;
        case 8: launch_fused_t<MODE, 8>(a, num_cu, stream); break;
        case 16: launch_fused_t<MODE, 16>(a, num_cu, stream); break;
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

void launch_mode_rotate(Prec prec, int ne, int nq, int nm, int nb, int nbp, const void* in,
                        const void* evec, const double* sc, void* out, hipStream_t stream,
                        const int32_t* ndeg_fold, const void* Lq, const int32_t* Re) {
    const size_t total = (size_t)ne * nq * nbp * nbp;
    if (total == 0) return;
    if (prec == Prec::F64)
        mode_rotate_kernel<double><<<blocks_for(total, 256), 256, 0, stream>>>(
            ne, nq, nm, nb, nbp, (const double2*)in, (const double2*)evec, sc, ndeg_fold, (const double2*)Lq, Re,
            (double2*)out);
    else
        mode_rotate_kernel<float><<<blocks_for(total, 256), 256, 0, stream>>>(
            ne, nq, nm, nb, nbp, (const float2*)in, (const double2*)evec, sc, ndeg_fold, (const double2*)Lq, Re,
            (float2*)out);
    launch_check("mode_rotate_kernel");
}

void launch_mode_rotate_fold(Prec prec, int ne, int nq, int nm, int nb, int nbp, const void* in, const void* evec,
                             const double* sc, const int32_t* ndeg, const int32_t* kh, const int32_t* half,
                             const int32_t* pair, const void* Lq, const int32_t* Re, void* out, hipStream_t stream) {
    const size_t total = (size_t)ne * nq * nbp * nbp;
    if (total == 0) return;
    // up to 8 modes: the mode count rounded up to 4 or 8, entries in registers
    auto go = [&](auto nmx) {
        constexpr int NMX = decltype(nmx)::value;
        if (prec == Prec::F64)
            mode_rotate_fold_kernel<double, NMX><<<blocks_for(total, 256), 256, 0, stream>>>(
                ne, nq, nm, nb, nbp, (const double2*)in, (const double2*)evec, sc, ndeg, kh, half, pair,
                (const double2*)Lq, Re, (double2*)out);
        else
            mode_rotate_fold_kernel<float, NMX><<<blocks_for(total, 256), 256, 0, stream>>>(
                ne, nq, nm, nb, nbp, (const float2*)in, (const double2*)evec, sc, ndeg, kh, half, pair,
                (const double2*)Lq, Re, (float2*)out);
    };
    if (nm <= 4) go(std::integral_constant<int, 4>{});
    else if (nm <= 8) go(std::integral_constant<int, 8>{});
    else go(std::integral_constant<int, 0>{});
    launch_check("mode_rotate_fold_kernel");
}

int fused_slices(int nk, int nbp, int tiles_n, int num_cu, Prec prec) {
    const int BM = fused_tile_rows(nbp, prec);
    const int tiles_m = (nk + BM - 1) / BM;
    if (tiles_m <= 0 || tiles_n <= 0) return 1;
    // one round of resident blocks (two per CU): every block gets the same
    // number of column tiles and no partial second round is left over
    const long slots = 2L * (num_cu > 0 ? num_cu : 256);
    long S = slots / tiles_m;
    if (S > tiles_n) S = tiles_n;
    if (S < 1) S = 1;
    return (int)S;
}

void fused_balance(FusedArgs& a, Prec prec, int num_cu) {
    a.helpers = 0;
    a.keep = 0x7fffffff;
    const int BM = fused_tile_rows(a.nbp, prec), BN = fused_tile_cols(a.nbp, prec);
    const long tiles_m = (a.nk + BM - 1) / BM;
    const long tiles_n = ((long)a.qc * a.nm * a.nbp * a.nbp + BN - 1) / BN;
    const long R = tiles_m * a.S;
    const long H = 2L * (num_cu > 0 ? num_cu : 256) - R;   // empty slots of one round
    const long J = (tiles_n + a.S - 1) / a.S;               // tiles of the longest slice
    if (!fused_balanced_c(a.nbp, (int)prec) || H <= 0 || R <= 0 || J < 32) return;
    // a helper runs at most c tails of J - keep tiles: keep = c (J - keep)
    const long c = (R + H - 1) / H;
    const long keep = (c * J + c) / (c + 1);
    if (keep >= J) return;
    a.helpers = (int)H;
    a.keep = (int)keep;
}

void launch_fused_k(Prec prec, const FusedArgs& a, int num_cu, hipStream_t stream) {
    if (a.nk == 0 || a.qc == 0) return;
    if (prec == Prec::F64)
        launch_fused_nbp<0>(a, num_cu, stream);
    else if (prec == Prec::F32)
        launch_fused_nbp<1>(a, num_cu, stream);
    else
        launch_fused_nbp<2>(a, num_cu, stream);
}

void launch_dos_raw(size_t n, const double* eps, double mu, double sigma, double* raw, hipStream_t stream) {
    dos_raw_kernel<<<1, 256, 0, stream>>>(n, eps, mu, 1.0 / sigma, raw);
    launch_check("dos_raw_kernel");
}

void launch_phonon_finalize(int qc, int nm, int tiles_m, const double* part_ph, const double* omega,
                            double omega_cut, const double* raw_dos, int nk, double sigma, double* pi_im,
                            double* lam, hipStream_t stream, double* lam_tr) {
    const int n = qc * nm;
    if (n == 0) return;
    phonon_finalize_kernel<<<blocks_for(n, 256), 256, 0, stream>>>(qc, nm, tiles_m, part_ph, omega, omega_cut,
                                                                  raw_dos, nk, sigma, pi_im, lam, lam_tr);
    launch_check("phonon_finalize_kernel");
}

void launch_reduce_partials(int nk, int nb, int S, const double* part, double scale, int accumulate,
                            double* imsig, hipStream_t stream) {
    const size_t total = (size_t)nk * nb;
    if (total == 0) return;
    reduce_partials_kernel<<<blocks_for(total, 256), 256, 0, stream>>>(nk, nb, S, part, scale, accumulate, imsig);
    launch_check("reduce_partials_kernel");
}

void launch_reduce_partials_diff(int nk, int nb, int S, const double* A, const double* B, double scale,
                                 int accumulate, double* out, hipStream_t stream) {
    const size_t total = (size_t)nk * nb;
    if (total == 0) return;
    reduce_partials_diff_kernel<<<blocks_for(total, 256), 256, 0, stream>>>(nk, nb, S, A, B, scale, accumulate,
                                                                            out);
    launch_check("reduce_partials_diff_kernel");
}

void launch_degenerate_average(int nk, int nb, const double* eps, double tol, double* v, hipStream_t stream) {
    if (nk == 0 || nb < 2) return;
    degenerate_average_kernel<<<blocks_for(nk, 128), 128, 0, stream>>>(nk, nb, eps, tol, v);
    launch_check("degenerate_average_kernel");
}

}  // namespace epw

namespace epw {
namespace {

// ------------------------------------------------------------ split-bf16 GEMM
// C[m][n] (+)= sum_k A[m][k] B[n][k] (complex), both operands four bf16
// planes with K contiguous and zero-padded to Kpad (a multiple of 32); float32
// accumulation on MFMA 16x16x32, the product form of the fused kernel's main
// loop; C is complex64.  Used by the split-bf16 adjoint for the R_e <-> k
// contractions.
__global__ __launch_bounds__(256) void bf16_gemm_kernel(Bf16GemmDesc d)
{
    __shared__ BfStage<64, 64> st;
    const int tiles_m = (d.M + 63) / 64;
    const long tiles_n = (d.N + 63) / 64;
    const long bx = blockIdx.x;
    const int mt = tiles_m <= 8 ? (int)(bx % tiles_m) : (int)(bx / tiles_n);
    const long nt = tiles_m <= 8 ? bx / tiles_m : bx % tiles_n;
    const int m0 = mt * 64;
    const long n0 = nt * 64;
    f4 cr[4], ci[4];
    auto nogen = [](int, int) { return make_float2(0.f, 0.f); };
    bf16_mainloop<64, 64, false>(st, d.A, d.lda, d.aplane, d.M, m0, d.B, d.ldb, d.bplane, d.N, n0, d.Kpad, nogen, cr,
                                 ci);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = 0; c < 4; ++c) {
        const long col = n0 + c * 16 + (lane & 15);
        if (col >= d.N) continue;
        for (int i = 0; i < 4; ++i) {
            const int row = m0 + wave * 16 + 4 * (lane >> 4) + i;
            if (row >= d.M) continue;
            float2* dst = d.C + (size_t)row * d.ldc + col;
            float2 v = make_float2(cr[c][i], ci[c][i]);
            if (d.accumulate) {
                const float2 o = *dst;
                v.x += o.x;
                v.y += o.y;
            }
            *dst = v;
        }
    }
}

__device__ inline void split_bf(float x, uint16_t& h, uint16_t& l) {
    const __hip_bfloat16 xh = __float2bfloat16(x);
    const __hip_bfloat16 xl = __float2bfloat16(x - __bfloat162float(xh));
    h = __builtin_bit_cast(uint16_t, xh);
    l = __builtin_bit_cast(uint16_t, xl);
}

// conj(exp(2 pi i p.R_r) / ndeg_r) as planes [4][nR][ld] (point index p
// contiguous, zero for p >= np): the A operand of a sum over points
__global__ void phase_planes_t_kernel(int np, const double* __restrict__ pts, int nR, const int32_t* __restrict__ R,
                                      const int32_t* __restrict__ ndeg, int ld, uint16_t* __restrict__ out)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)nR * ld;
    if (idx >= total) return;
    const int r = (int)(idx / ld), p = (int)(idx % ld);
    float c = 0.f, sn = 0.f;
    if (p < np) {
        double x = pts[3 * (size_t)p] * (double)R[3 * r] + pts[3 * (size_t)p + 1] * (double)R[3 * r + 1] +
                   pts[3 * (size_t)p + 2] * (double)R[3 * r + 2];
        x -= rint(x);
        double s, cc;
        sincospi(2.0 * x, &s, &cc);
        const double w = ndeg ? 1.0 / (double)ndeg[r] : 1.0;
        c = (float)(cc * w);
        sn = (float)(-s * w);
    }
    uint16_t h, l;
    split_bf(c, h, l);
    out[idx] = h;
    out[total + idx] = l;
    split_bf(sn, h, l);
    out[2 * total + idx] = h;
    out[3 * total + idx] = l;
}

// complex64 X [K][N] -> planes [4][N][Kpad] (K contiguous, zero for k >= K),
// transposed through LDS in 64 x 64 tiles
__global__ __launch_bounds__(256) void split_transpose_kernel(int K, long N, const float2* __restrict__ X, int Kpad,
                                                              uint16_t* __restrict__ out)
{
    __shared__ float2 tile[64][65];
    const long n0 = (long)blockIdx.x * 64;
    const int k0 = blockIdx.y * 64;
    const int tid = threadIdx.x;
    for (int it = tid; it < 64 * 64; it += 256) {
        const int kl = it / 64, nl = it % 64;
        const int k = k0 + kl;
        const long n = n0 + nl;
        tile[nl][kl] = (k < K && n < N) ? X[(size_t)k * N + n] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const long plane = N * (long)Kpad;
    for (int it = tid; it < 64 * 8; it += 256) {
        const int nl = it / 8, part = it % 8;
        const long n = n0 + nl;
        const int kb = k0 + part * 8;
        if (n >= N || kb >= Kpad) continue;
        uint32_t hr[4] = {0u, 0u, 0u, 0u}, lr[4] = {0u, 0u, 0u, 0u}, hi[4] = {0u, 0u, 0u, 0u},
                 li[4] = {0u, 0u, 0u, 0u};
        for (int t = 0; t < 8; ++t) {
            const float2 v = tile[nl][part * 8 + t];
            uint16_t a, b, c2, d2;
            split_bf(v.x, a, b);
            split_bf(v.y, c2, d2);
            const int sh = 16 * (t & 1);
            hr[t >> 1] |= (uint32_t)a << sh;
            lr[t >> 1] |= (uint32_t)b << sh;
            hi[t >> 1] |= (uint32_t)c2 << sh;
            li[t >> 1] |= (uint32_t)d2 << sh;
        }
        uint16_t* o = out + (size_t)n * Kpad + kb;
        *reinterpret_cast<uint4*>(o) = make_uint4(hr[0], hr[1], hr[2], hr[3]);
        *reinterpret_cast<uint4*>(o + plane) = make_uint4(lr[0], lr[1], lr[2], lr[3]);
        *reinterpret_cast<uint4*>(o + 2 * plane) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        *reinterpret_cast<uint4*>(o + 3 * plane) = make_uint4(li[0], li[1], li[2], li[3]);
    }
}

}  // namespace

void launch_bf16_gemm(const Bf16GemmDesc& d, hipStream_t stream) {
    if (d.M <= 0 || d.N <= 0) return;
    if (d.Kpad % 32 != 0 || d.lda % 8 != 0 || d.ldb % 8 != 0 || d.aplane % 8 != 0 || d.bplane % 8 != 0)
        throw HipFailure{(int)hipErrorInvalidValue, "bf16 GEMM descriptor (K padding / 16-byte rows)", __FILE__,
                         __LINE__};
    const long tiles = (long)((d.N + 63) / 64) * ((d.M + 63) / 64);
    bf16_gemm_kernel<<<dim3((unsigned)tiles), 256, 0, stream>>>(d);
    launch_check("bf16_gemm_kernel");
}

void launch_phase_planes_t(int np, const double* pts, int nR, const int32_t* R, const int32_t* ndeg, int ld,
                           void* out, hipStream_t stream) {
    const size_t total = (size_t)nR * ld;
    if (total == 0) return;
    phase_planes_t_kernel<<<(unsigned)((total + 255) / 256), 256, 0, stream>>>(np, pts, nR, R, ndeg, ld,
                                                                              (uint16_t*)out);
    launch_check("phase_planes_t_kernel");
}

void launch_split_transpose(int K, long N, const void* X, int Kpad, void* out, hipStream_t stream) {
    if (N <= 0 || Kpad <= 0) return;
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((Kpad + 63) / 64));
    split_transpose_kernel<<<grid, 256, 0, stream>>>(K, N, (const float2*)X, Kpad, (uint16_t*)out);
    launch_check("split_transpose_kernel");
}

}  // namespace epw

namespace epw {
void launch_mode_rotate_bf16(int ne, int qc, int nm, int nb, int nbp, int kpad, const void* in, const void* evec,
                             const double* sc, void* out, hipStream_t stream, const int32_t* ndeg_fold,
                             const void* Lq, const int32_t* Re) {
    if (qc == 0) return;
    dim3 grid((unsigned)qc, (unsigned)((kpad + 63) / 64));
    mode_rotate_bf16_kernel<<<grid, 256, 0, stream>>>(ne, qc, nm, nb, nbp, kpad, (const float2*)in,
                                                     (const double2*)evec, sc, ndeg_fold, (const double2*)Lq, Re,
                                                     (uint16_t*)out);
    launch_check("mode_rotate_bf16_kernel");
}
}  // namespace epw
