// Generic strided complex GEMM on MFMA (float64 / float32):
//   C(m, n) (+)= sum_k A(m, k) B(k, n)
// with A read row-major or conjugate-transposed, and the column index n split
// as n = e * ncb + c so that batched slabs (one per Wannier vector R_e) are
// addressed without copies.  Used for the R_p -> q contraction, the
// recomputation of the vertex in the adjoint, and the transposed
// contractions of the adjoint.  The float64 pair-operand product (H(k+q)
// from H(R_e)) also runs folded by the pairs (R, -R): A = c + i s over a
// halved R list, C = sum_h c B+ + i s B- (cfold_mainloop), two real MFMAs
// per original R vector instead of three.
#include <hip/hip_runtime.h>

#include "cgemm.h"
#include "epw_internal.h"
#include "kernels.h"

namespace epw {
namespace {

template <typename T, bool CONJ_TRANS_A, bool FOLD = false>
__global__ __launch_bounds__(256, 2) void cgemm_generic_kernel(GemmDesc d)
{
    static_assert(!FOLD || (!CONJ_TRANS_A && sizeof(T) == 8), "folded sums: float64, row-major pair operand");
    typedef typename Cx<T>::type CT;
    // the folded stage holds six planes: K steps of 8 keep two stages per block
    // within the LDS of two resident blocks
    constexpr int BM = 64, BN = 64, BK = FOLD ? 8 : 16;
    // 1-D grid: with few row tiles the row tile varies fastest, so the blocks
    // sharing a column tile of B run together and share it in L2
    const int tiles_m = (d.M + BM - 1) / BM;
    const long tiles_n = ((long)d.N + BN - 1) / BN;
    const long bx = blockIdx.x;
    const int mt = tiles_m <= 8 ? (int)(bx % tiles_m) : (int)(bx / tiles_n);
    const long nt = tiles_m <= 8 ? bx / tiles_m : bx % tiles_n;
    const int m0 = mt * BM;
    const long n0 = nt * BN;
    // split K: block z covers k in [kb, kb + Kz) and writes its own partial C
    const int kb = d.kchunk > 0 ? (int)blockIdx.z * d.kchunk : 0;
    const int Kz = FOLD ? d.kh[0] : d.kchunk > 0 ? min(d.kchunk, d.K - kb) : d.K;
    const CT* A = reinterpret_cast<const CT*>(d.A);
    const CT* B = reinterpret_cast<const CT*>(d.B);
    CT* C = reinterpret_cast<CT*>(d.C) + (size_t)blockIdx.z * d.sCz;
    // Index arithmetic that does not change along K is done once per tile, so
    // that the K loop has no integer division.  Row-major A: the AE elements
    // a thread fetches per K step lie in one row (AE divides BK), whose two
    // phase rows the pair operand needs.  B: the thread fetches BE consecutive
    // columns from nbase on; the slab index and offset of the first one are
    // kept, the others are at most one slab boundary further.
    constexpr int AE = BM * BK / 256, BE = BK * BN / 256;
    static_assert(BK % AE == 0 && BN < 256 && BN % BE == 0, "fetch order of the 64 x 64 tile");
    const CT* arow1 = A;
    const CT* arow2 = reinterpret_cast<const CT*>(d.A2);
    if (!CONJ_TRANS_A && d.A2) {
        const int my_row = min(m0 + (int)threadIdx.x * AE / BK, d.M - 1);
        const long r = d.row0 + my_row;
        arow1 = A + (size_t)(r / d.n2) * d.lda;
        arow2 += (size_t)(r % d.n2) * d.lda;
    }
    const int nbase = (int)(threadIdx.x * BE) % BN;
    const long colbase = n0 + nbase;
    const long e_base = colbase / d.ncb;
    const int c_base = (int)(colbase % d.ncb);
    auto afetch = [&](int m, int kl) -> CT {
        const int row = m0 + m, k = kb + kl;
        if (row < d.M && kl < Kz) {
            if (CONJ_TRANS_A) {
                CT v;
                if (d.A2) {
                    // conj of the pair operand: GEMM index k is the pair row0 + k
                    const unsigned r = (unsigned)(d.row0 + k);
                    const unsigned i1 = r / (unsigned)d.n2, i2 = r - i1 * (unsigned)d.n2;
                    const CT x = A[(size_t)i1 * d.lda + row];
                    const CT y = reinterpret_cast<const CT*>(d.A2)[(size_t)i2 * d.lda + row];
                    v.x = x.x * y.x - x.y * y.y;
                    v.y = x.x * y.y + x.y * y.x;
                } else {
                    v = A[(size_t)k * d.lda + row];
                }
                v.y = -v.y;
                return v;
            }
            if (d.A2) {
                const CT x = arow1[k];
                const CT y = arow2[k];
                CT v;
                v.x = x.x * y.x - x.y * y.y;
                v.y = x.x * y.y + x.y * y.x;
                return v;
            }
            return A[(size_t)row * d.lda + k];
        }
        return cz<T>();
    };
    auto bfetch = [&](int kl, int n) -> CT {
        const long col = n0 + n;
        if (kl < Kz && col < d.N) {
            long e = e_base;
            int c = c_base + (n - nbase);      // n - nbase < BE
            while (c >= d.ncb) {
                c -= d.ncb;
                ++e;
            }
            return B[(size_t)e * d.sBe + (size_t)(kb + kl) * d.sBk + c];
        }
        return cz<T>();
    };
    typename Cx<T>::acc cr[4], ci[4];
    if constexpr (FOLD) {
        // B+ and B- of entry h of the halved list, same column decoding as bfetch
        const CT* B2 = reinterpret_cast<const CT*>(d.B2);
        auto bfold = [&](int kl, int n) -> CPair<CT> {
            CPair<CT> v;
            v.p = cz<T>();
            v.m = cz<T>();
            const long col = n0 + n;
            if (kl < Kz && col < d.N) {
                long e = e_base;
                int c = c_base + (n - nbase);
                while (c >= d.ncb) {
                    c -= d.ncb;
                    ++e;
                }
                const size_t off = (size_t)e * d.sBe + (size_t)kl * d.sBk + c;
                v.p = B[off];
                v.m = B2[off];
            }
            return v;
        };
        __shared__ FoldStage<T, BM, BN, BK> fst[2];
        cfold_mainloop<T, BM, BN, BK, decltype(afetch), decltype(bfold), 2>(fst, Kz, afetch, bfold, cr, ci);
    } else {
        __shared__ Stage<T, BM, BN, BK> st[2];
        cgemm_mainloop<T, BM, BN, BK, decltype(afetch), decltype(bfetch), CONJ_TRANS_A, 2>(st, Kz, afetch, bfetch, cr,
                                                                                          ci);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = 0; c < 4; ++c) {
        const long col = n0 + c * 16 + (lane & 15);
        if (col >= d.N) continue;
        const long e = col / d.ncb, cc = col % d.ncb;
        for (int i = 0; i < 4; ++i) {
            const int row = m0 + wave * 16 + crow<T>(lane, i);
            if (row >= d.M) continue;
            CT* dst = C + (size_t)e * d.sCe + (size_t)row * d.sCm + cc;
            CT v;
            v.x = cr[c][i];
            v.y = ci[c][i];
            if (d.accumulate) {
                const CT o = *dst;
                v.x += o.x;
                v.y += o.y;
            }
            *dst = v;
        }
    }
}

// C[m][n] (+)= sum_z P[z][m][n] in fixed z order (split-K partials, C with row stride ldc)
template <typename CT>
__global__ void splitk_reduce_kernel(int M, int N, int parts, const CT* __restrict__ P, long ldc, int accumulate,
                                     CT* __restrict__ C)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t MN = (size_t)M * N;
    if (idx >= MN) return;
    const size_t m = idx / N, n = idx % N;
    CT v = P[idx];
    for (int z = 1; z < parts; ++z) {
        const CT p = P[(size_t)z * MN + idx];
        v.x += p.x;
        v.y += p.y;
    }
    CT* dst = C + m * ldc + n;
    if (accumulate) {
        v.x += dst->x;
        v.y += dst->y;
    }
    *dst = v;
}

}  // namespace

int splitk_parts_wide(int M, int N, int K, int max_parts) {
    // about four rounds of two resident blocks per CU on 256 CUs, at least
    // 512 K values per part
    const long blocks = (long)((N + 63) / 64) * ((M + 63) / 64);
    long parts = blocks > 0 ? (2048 + blocks - 1) / blocks : 1;
    const long kmax = K / 512;
    if (parts > kmax) parts = kmax;
    if (parts > max_parts) parts = max_parts;
    return parts < 1 ? 1 : (int)parts;
}

int splitk_parts(int M, int N, int K) {
    // enough blocks for ~8 rounds of two resident blocks per CU on 256 CUs,
    // at least 512 K values per part, at most 4 parts
    const long blocks = (long)((N + 63) / 64) * ((M + 63) / 64);
    long parts = blocks > 0 ? (4096 + blocks - 1) / blocks : 1;
    const long kmax = K / 512;
    if (parts > kmax) parts = kmax;
    if (parts > 4) parts = 4;
    return parts < 1 ? 1 : (int)parts;
}

// The adjoint's sum over k, gbar(R_e, col) = sum_k conj(Phi_k(R_e)) Gbar[k][col]
// / ndeg(R_e), folded by the pairs (R, -R) of the halved R list: with
// c + i s = Phi_k(R_h) (unweighted), P = sum_k c Gbar_k and Q = sum_k s Gbar_k,
//   gbar(R_h) = (P - i Q) / ndeg(R_h),   gbar(-R_h) = (P + i Q) / ndeg(-R_h),
// a real-by-complex product of 2 kh rows: two real MFMAs per block where the
// complex form takes three over N_e rows.  A 64-row tile holds P and Q of 32
// entries h, placed so that both land in the same lane of the MFMA result
// (each 16-row block: 8 entries, P and Q), where they are unfolded.
template <typename T>
__global__ __launch_bounds__(256, 2) void ksum_fold_kernel(KsumFoldDesc d)
{
    typedef typename Cx<T>::type CT;
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ RStage<T, BM, BN, BK> st[2];
    const int kh = d.kh[0];
    const int tiles_m = (d.ne + 31) / 32;
    const long bx = blockIdx.x;
    const int mt = (int)(bx % tiles_m);
    const long nt = bx / tiles_m;
    const int h0 = mt * 32;
    if (h0 >= kh) return;
    const long n0 = nt * BN;
    const int kb = d.kchunk > 0 ? (int)blockIdx.z * d.kchunk : 0;
    const int Kz = d.kchunk > 0 ? min(d.kchunk, d.nk - kb) : d.nk;
    const CT* phi = reinterpret_cast<const CT*>(d.phi);
    const CT* G = reinterpret_cast<const CT*>(d.G);
    // row m of the tile: entry h and part (0: P, from c; 1: Q, from s)
    auto rowmap = [&](int m, int& h, int& part) {
        const int b = m >> 4, l = m & 15;
        if (sizeof(T) == 8) {        // f64 result rows l/16 + 4i: i and i + 1 hold P and Q
            h = h0 + 8 * b + (l & 3) + 4 * (l >> 3);
            part = (l >> 2) & 1;
        } else {                     // f32 result rows 4 (l/16) + i
            h = h0 + 8 * b + 2 * (l >> 2) + ((l & 3) >> 1);
            part = l & 1;
        }
    };
    auto afetch = [&](int m, int kl) -> T {
        int h, part;
        rowmap(m, h, part);
        if (h < kh && kl < Kz) {
            const CT v = phi[(size_t)(kb + kl) * d.ld + h];
            return part ? v.y : v.x;
        }
        return T(0);
    };
    auto bfetch = [&](int kl, int n) -> CT {
        const long col = n0 + n;
        if (kl < Kz && col < d.ncols) return G[(size_t)(kb + kl) * d.ncols + col];
        return cz<T>();
    };
    typename Cx<T>::acc cr[4], ci[4];
    rgemm_mainloop<T, BM, BN, BK, decltype(afetch), decltype(bfetch), 2>(st, Kz, afetch, bfetch, cr, ci);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    CT* out = reinterpret_cast<CT*>(d.out) + (size_t)blockIdx.z * d.ne * d.ncols;
    for (int c = 0; c < 4; ++c) {
        const long col = n0 + c * 16 + (lane & 15);
        if (col >= d.ncols) continue;
        for (int i = 0; i < 4; i += 2) {
            int h, part;
            rowmap(wave * 16 + crow<T>(lane, i), h, part);   // part 0; element i + 1 holds Q
            if (h >= kh) continue;
            const T pr = cr[c][i], pim = ci[c][i], qr = cr[c][i + 1], qim = ci[c][i + 1];
            const int e1 = d.half[h], e2 = d.pair[h];
            const T w1 = T(1) / (T)d.ndeg[e1];
            CT v;
            v.x = (pr + qim) * w1;
            v.y = (pim - qr) * w1;
            out[(size_t)e1 * d.ncols + col] = v;
            if (e2 != e1) {
                const T w2 = T(1) / (T)d.ndeg[e2];
                v.x = (pr - qim) * w2;
                v.y = (pim + qr) * w2;
                out[(size_t)e2 * d.ncols + col] = v;
            }
        }
    }
}

namespace {
// B+ / B- rows of a halved R list (launch_fold_gather); rows h >= kh[0] are zero
__global__ void fold_gather_kernel(const int32_t* __restrict__ kh, const int32_t* __restrict__ half,
                                   const int32_t* __restrict__ pair, const int32_t* __restrict__ ndeg, long cols,
                                   const double2* __restrict__ B, double2* __restrict__ Bp, double2* __restrict__ Bm) {
    const long h = blockIdx.y;
    const long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= cols) return;
    double2 p = make_double2(0.0, 0.0), m = p;
    if (h < kh[0]) {
        const long r1 = half[h], r2 = pair[h];
        const double w1 = 1.0 / (double)ndeg[r1];
        const double2 x = B[r1 * cols + col];
        p = make_double2(x.x * w1, x.y * w1);
        m = p;
        if (r2 != r1) {
            const double w2 = 1.0 / (double)ndeg[r2];
            const double2 y = B[r2 * cols + col];
            const double2 yw = make_double2(y.x * w2, y.y * w2);
            p = make_double2(x.x * w1 + yw.x, x.y * w1 + yw.y);
            m = make_double2(x.x * w1 - yw.x, x.y * w1 - yw.y);
        }
    }
    Bp[h * cols + col] = p;
    Bm[h * cols + col] = m;
}
}  // namespace

void launch_fold_gather(int nR, const int32_t* kh, const int32_t* half, const int32_t* pair, const int32_t* ndeg,
                        long cols, const void* B, void* Bp, void* Bm, hipStream_t stream) {
    if (nR <= 0 || cols <= 0) return;
    const dim3 grid((unsigned)((cols + 255) / 256), (unsigned)nR);
    fold_gather_kernel<<<grid, 256, 0, stream>>>(kh, half, pair, ndeg, cols, (const double2*)B, (double2*)Bp,
                                                 (double2*)Bm);
    launch_check("fold_gather_kernel");
}

void launch_cgemm_splitk(Prec prec, const GemmDesc& d, int parts, void* scratch, hipStream_t stream) {
    if (d.M <= 0 || d.N <= 0) return;
    if (parts <= 1 || d.ncb != d.N || d.kchunk != 0) {
        launch_cgemm(prec, d, stream);
        return;
    }
    GemmDesc e = d;
    e.kchunk = ((d.K + parts - 1) / parts + 15) / 16 * 16;
    const int nz = (d.K + e.kchunk - 1) / e.kchunk;
    e.C = scratch;
    e.sCe = 0;
    e.sCm = d.N;
    e.sCz = (long)d.M * d.N;
    e.accumulate = 0;
    launch_cgemm(prec, e, stream, nz);
    const size_t MN = (size_t)d.M * d.N;
    const unsigned nb = (unsigned)((MN + 255) / 256);
    if (prec == Prec::F64)
        splitk_reduce_kernel<double2><<<nb, 256, 0, stream>>>(d.M, d.N, nz, (const double2*)scratch, d.sCm,
                                                               d.accumulate, (double2*)d.C);
    else
        splitk_reduce_kernel<float2><<<nb, 256, 0, stream>>>(d.M, d.N, nz, (const float2*)scratch, d.sCm,
                                                             d.accumulate, (float2*)d.C);
    launch_check("splitk_reduce_kernel");
}

void launch_ksum_fold(Prec prec, const KsumFoldDesc& desc, int parts, void* scratch, void* C, hipStream_t stream) {
    if (desc.ne <= 0 || desc.ncols <= 0) return;
    KsumFoldDesc d = desc;
    int nz = 1;
    if (parts > 1 && d.nk > 16) {
        d.kchunk = ((d.nk + parts - 1) / parts + 15) / 16 * 16;
        nz = (d.nk + d.kchunk - 1) / d.kchunk;
    } else {
        d.kchunk = 0;
    }
    d.out = nz > 1 ? scratch : C;
    const long tiles = (long)((d.ne + 31) / 32) * ((d.ncols + 63) / 64);
    const dim3 grid((unsigned)tiles, 1, (unsigned)nz);
    if (prec == Prec::F64) ksum_fold_kernel<double><<<grid, 256, 0, stream>>>(d);
    else ksum_fold_kernel<float><<<grid, 256, 0, stream>>>(d);
    launch_check("ksum_fold_kernel");
    if (nz > 1) {
        const size_t MN = (size_t)d.ne * d.ncols;
        const unsigned nb = (unsigned)((MN + 255) / 256);
        if (prec == Prec::F64)
            splitk_reduce_kernel<double2><<<nb, 256, 0, stream>>>(d.ne, (int)d.ncols, nz, (const double2*)scratch,
                                                                   d.ncols, 0, (double2*)C);
        else
            splitk_reduce_kernel<float2><<<nb, 256, 0, stream>>>(d.ne, (int)d.ncols, nz, (const float2*)scratch,
                                                                 d.ncols, 0, (float2*)C);
        launch_check("splitk_reduce_kernel");
    }
}

void launch_cgemm(Prec prec, const GemmDesc& d, hipStream_t stream, int kparts) {
    if (d.M <= 0 || d.N <= 0) return;
    // the kernel walks column slabs of width ncb and splits pair rows by n2
    if (d.ncb < 1 || d.n2 < 1) throw HipFailure{(int)hipErrorInvalidValue, "cgemm descriptor (ncb, n2)", __FILE__, __LINE__};
    const long tiles = (long)((d.N + 63) / 64) * ((d.M + 63) / 64);
    dim3 grid((unsigned)tiles, 1, (unsigned)(kparts > 1 ? kparts : 1));
    if (d.kh) {
        if (prec != Prec::F64 || d.conj_trans_a || !d.A2 || !d.B2 || d.kchunk != 0 || kparts > 1)
            throw HipFailure{(int)hipErrorInvalidValue, "folded cgemm descriptor", __FILE__, __LINE__};
        cgemm_generic_kernel<double, false, true><<<grid, 256, 0, stream>>>(d);
    } else if (prec == Prec::F64) {
        if (d.conj_trans_a) cgemm_generic_kernel<double, true><<<grid, 256, 0, stream>>>(d);
        else cgemm_generic_kernel<double, false><<<grid, 256, 0, stream>>>(d);
    } else {
        if (d.conj_trans_a) cgemm_generic_kernel<float, true><<<grid, 256, 0, stream>>>(d);
        else cgemm_generic_kernel<float, false><<<grid, 256, 0, stream>>>(d);
    }
    launch_check("cgemm_generic_kernel");
}

}  // namespace epw
