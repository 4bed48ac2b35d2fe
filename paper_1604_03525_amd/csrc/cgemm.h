// Complex GEMM building blocks on MFMA 16x16x4 (float64 and float32),
// shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace epw {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Cx;
template <> struct Cx<double> { typedef double2 type; typedef d4 acc; };
template <> struct Cx<float> { typedef float2 type; typedef f4 acc; };

__device__ inline d4 mfma4(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma4(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <bool B, class X, class Y> struct PickType { typedef X type; };
template <class X, class Y> struct PickType<false, X, Y> { typedef Y type; };

template <typename T> __device__ inline typename Cx<T>::type cz() {
    typename Cx<T>::type z;
    z.x = T(0);
    z.y = T(0);
    return z;
}


// ------------------------------------------------------------ GEMM main loop
//
// Block tile BM x BN (complex), K step BK, 256 threads = 4 waves; each wave
// owns a 16 x 64 sub-tile = four 16x16 MFMA blocks.  Operands are staged
// global -> registers -> LDS (split into re/im planes, K-major) with the
// next K step's global loads issued before the current step's MFMAs.
//
// MFMA 16x16x4 operand layout (f64 and f32): lane l holds A[l%16][l/16] and
// B[l/16][l%16].  Accumulator element i of lane l is C[crow][l%16] with
// crow = l/16 + 4i for f64 and 4*(l/16) + i for f32 (measured on gfx950).
template <typename T> __device__ inline int crow(int lane, int i);
template <> __device__ inline int crow<double>(int lane, int i) { return (lane >> 4) + 4 * i; }
template <> __device__ inline int crow<float>(int lane, int i) { return 4 * (lane >> 4) + i; }

// Rows are padded by 16 elements: the four K rows one MFMA operand read
// touches then start in different LDS bank ranges.
template <typename T, int BM, int BN, int BK>
struct Stage {
    static constexpr int PAD = 16;
    T a_re[BK][BM + PAD];
    T a_im[BK][BM + PAD];
    T b_re[BK][BN + PAD];
    T b_im[BK][BN + PAD];
};

// B elements per thread: for tiles 256 or more columns wide, element e of
// thread t is entry e * 256 + t, so that one load instruction of a wave reads
// 64 consecutive columns of one K row (512 contiguous bytes in float32) and
// the LDS stores are conflict-free; narrower tiles keep BE consecutive
// columns per thread (measured faster there: the consecutive-lane order was
// 29 % slower for 64-wide float64 tiles, and 18 % faster for 256-wide ones).
// A_KMAJOR selects which index of the A tile varies fastest across threads
// when it is fetched: k (row-major A, default) or m (A read transposed).
// NS = 1: one LDS stage, two barriers per K step; NS = 2: the next K step is
// stored into the other stage while this one is read, one barrier per step.
// Waves: WN = BN / 64 across the columns, 4 / WN across the rows; each wave
// owns RB row blocks of 16 x 64 (accumulator index rb * 4 + column block), so
// a wave reads each B fragment once for RB row blocks.
template <int BM, int BN> struct CWaves {
    static constexpr int WN = BN / 64;
    static constexpr int RB = BM * WN / 64;
};
template <typename T, int BM, int BN, int BK, class AF, class BF, bool A_KMAJOR = false, int NS = 1>
__device__ inline void cgemm_mainloop(Stage<T, BM, BN, BK>* stages, int K, AF afetch, BF bfetch,
                                      typename Cx<T>::acc (&cr)[4 * CWaves<BM, BN>::RB],
                                      typename Cx<T>::acc (&ci)[4 * CWaves<BM, BN>::RB])
{
    static_assert(NS == 1 || NS == 2, "one or two LDS stages");
    typedef typename Cx<T>::type CT;
    constexpr int WN = CWaves<BM, BN>::WN;
    constexpr int RB = CWaves<BM, BN>::RB;
    static_assert(RB >= 1 && 16 * RB * (4 / WN) == BM, "wave layout");
    // A tiles smaller than the block (16 rows at K step 8) load one element
    // on the first BM * BK threads only
    constexpr int AN = BM * BK;
    constexpr int AE = AN >= 256 ? AN / 256 : 1;
    constexpr int BE = BK * BN / 256;
    static_assert((AN >= 256 ? AE * 256 == AN : 256 % AN == 0) && BE >= 1 && BE * 256 == BK * BN,
                  "tile too small for 256 threads");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    CT ra[AE], rb[BE];
    for (int c = 0; c < 4 * RB; ++c) {
        for (int i = 0; i < 4; ++i) {
            cr[c][i] = T(0);
            ci[c][i] = T(0);
        }
    }
    auto gload = [&](int k0) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = tid * AE + e;
            if (AN < 256 && idx >= AN) break;
            if (A_KMAJOR)
                ra[e] = afetch(idx % BM, k0 + idx / BM);
            else
                ra[e] = afetch(idx / BK, k0 + idx % BK);
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = BN >= 256 ? e * 256 + tid : tid * BE + e;
            rb[e] = bfetch(k0 + idx / BN, idx % BN);
        }
    };
    auto sstore = [&](Stage<T, BM, BN, BK>& st) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = tid * AE + e;
            if (AN < 256 && idx >= AN) break;
            const int m = A_KMAJOR ? idx % BM : idx / BK;
            const int k = A_KMAJOR ? idx / BM : idx % BK;
            st.a_re[k][m] = ra[e].x;
            st.a_im[k][m] = ra[e].y;
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = BN >= 256 ? e * 256 + tid : tid * BE + e;
            st.b_re[idx / BN][idx % BN] = rb[e].x;
            st.b_im[idx / BN][idx % BN] = rb[e].y;
        }
    };
    // Gauss's three-multiplication complex product: with P1 = sum ar br,
    // P2 = sum ai bi, P3 = sum (ar + ai)(br + bi):  re = P1 - P2,
    // im = P3 - P1 - P2.  Three real MFMAs per complex block product instead
    // of four; the operand sums are formed in registers from the LDS planes.
    typename Cx<T>::acc cm[4 * RB];
    for (int c = 0; c < 4 * RB; ++c)
        for (int i = 0; i < 4; ++i) cm[c][i] = T(0);
    gload(0);
    sstore(stages[0]);
    __syncthreads();
    for (int k0 = 0, it = 0; k0 < K; k0 += BK, ++it) {
        const bool more = k0 + BK < K;
        if (more) gload(k0 + BK);
        const Stage<T, BM, BN, BK>& st = stages[NS == 2 ? (it & 1) : 0];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            // the K tail in float32: sub-steps that start at or beyond K would
            // only add zero rows (279 R vectors: 2 of the last step's 4 run;
            // FP32 fused launch 287 -> 284 ms).  The float64 loop is left
            // without the test, which stops the compiler from reading the next
            // sub-step's operands under the current MFMAs there (255 -> 351 ms).
            if (sizeof(T) == 4 && BK > 8 && k0 + kk >= K) break;
            const int kr = kk + (lane >> 4);
            T ar[RB], ai[RB], as[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                ar[q] = st.a_re[kr][wm * 16 * RB + q * 16 + (lane & 15)];
                ai[q] = st.a_im[kr][wm * 16 * RB + q * 16 + (lane & 15)];
                as[q] = ar[q] + ai[q];
            }
            T br[4], bi[4], bs[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                br[c] = st.b_re[kr][wn * 64 + c * 16 + (lane & 15)];
                bi[c] = st.b_im[kr][wn * 64 + c * 16 + (lane & 15)];
                bs[c] = br[c] + bi[c];
            }
            // consecutive MFMAs cycle over the 4 RB accumulators of a product
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) cr[q * 4 + c] = mfma4(ar[q], br[c], cr[q * 4 + c]);
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) cm[q * 4 + c] = mfma4(ai[q], bi[c], cm[q * 4 + c]);
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) ci[q * 4 + c] = mfma4(as[q], bs[c], ci[q * 4 + c]);
        }
        if constexpr (NS == 2) {
            // the other stage was last read in the previous step, before its barrier
            if (more) sstore(stages[(it + 1) & 1]);
            __syncthreads();
        } else {
            __syncthreads();
            if (more) {
                sstore(stages[0]);
                __syncthreads();
            }
        }
    }
    for (int c = 0; c < 4 * RB; ++c)
        for (int i = 0; i < 4; ++i) {
            const T p1 = cr[c][i], p2 = cm[c][i];
            cr[c][i] = p1 - p2;
            ci[c][i] = ci[c][i] - p1 - p2;
        }
}


// ------------------------------------------------ folded contraction main loop
//
// For a K set that pairs every vector R with -R, a sum of Phi(R) B(R) with
// Phi(-R) = conj(Phi(R)) regroups over one member of each pair:
//   sum_R Phi(R) B(R) = sum_h [c_h B+_h + i s_h B-_h],
// c + i s = Phi(R_h), B+ = B(R_h) + B(-R_h), B- = B(R_h) - B(-R_h); a vector
// without a partner (and R = 0) enters with B+ = B- = B(R_h).  Per K entry of
// the halved sum the real and imaginary parts take two real MFMAs each:
//   re += c B+re - s B-im,   im += c B+im + s B-re,
// i.e. two real products per original vector instead of three (Gauss) or
// four.  B- im is stored negated so that both updates are plain MFMAs.
template <typename T, int BM, int BN, int BK>
struct FoldStage {
    static constexpr int PAD = 16;
    T a_re[BK][BM + PAD];      // c
    T a_im[BK][BM + PAD];      // s
    T bp_re[BK][BN + PAD];     // B+ re
    T bp_im[BK][BN + PAD];     // B+ im
    T bm_re[BK][BN + PAD];     // B- re
    T bm_ni[BK][BN + PAD];     // -B- im
};
template <typename CT> struct CPair {
    CT p, m;   // B+ and B- entries
};

// Main loop over the halved K (Kh entries): afetch(m, h) gives c + i s of
// row m, bfetch(h, n) the pair {B+, B-} of column n (zeros beyond Kh).  The
// same block, wave and staging layout as cgemm_mainloop; the accumulators
// are C re and C im.
template <typename T, int BM, int BN, int BK, class AF, class BF, int NS = 1>
__device__ inline void cfold_mainloop(FoldStage<T, BM, BN, BK>* stages, int Kh, AF afetch, BF bfetch,
                                      typename Cx<T>::acc (&cr)[4 * CWaves<BM, BN>::RB],
                                      typename Cx<T>::acc (&ci)[4 * CWaves<BM, BN>::RB])
{
    static_assert(NS == 1 || NS == 2, "one or two LDS stages");
    typedef typename Cx<T>::type CT;
    constexpr int WN = CWaves<BM, BN>::WN;
    constexpr int RB = CWaves<BM, BN>::RB;
    static_assert(RB >= 1 && 16 * RB * (4 / WN) == BM, "wave layout");
    constexpr int AN = BM * BK;
    constexpr int AE = AN >= 256 ? AN / 256 : 1;
    constexpr int BE = BK * BN / 256;
    static_assert((AN >= 256 ? AE * 256 == AN : 256 % AN == 0) && BE >= 1 && BE * 256 == BK * BN,
                  "tile too small for 256 threads");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    CT ra[AE];
    CPair<CT> rb[BE];
    for (int c = 0; c < 4 * RB; ++c)
        for (int i = 0; i < 4; ++i) {
            cr[c][i] = T(0);
            ci[c][i] = T(0);
        }
    auto gload = [&](int k0) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = tid * AE + e;
            if (AN < 256 && idx >= AN) break;
            ra[e] = afetch(idx / BK, k0 + idx % BK);
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = BN >= 256 ? e * 256 + tid : tid * BE + e;
            rb[e] = bfetch(k0 + idx / BN, idx % BN);
        }
    };
    auto sstore = [&](FoldStage<T, BM, BN, BK>& st) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = tid * AE + e;
            if (AN < 256 && idx >= AN) break;
            st.a_re[idx % BK][idx / BK] = ra[e].x;
            st.a_im[idx % BK][idx / BK] = ra[e].y;
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = BN >= 256 ? e * 256 + tid : tid * BE + e;
            st.bp_re[idx / BN][idx % BN] = rb[e].p.x;
            st.bp_im[idx / BN][idx % BN] = rb[e].p.y;
            st.bm_re[idx / BN][idx % BN] = rb[e].m.x;
            st.bm_ni[idx / BN][idx % BN] = -rb[e].m.y;
        }
    };
    gload(0);
    sstore(stages[0]);
    __syncthreads();
    for (int k0 = 0, it = 0; k0 < Kh; k0 += BK, ++it) {
        const bool more = k0 + BK < Kh;
        if (more) gload(k0 + BK);
        const FoldStage<T, BM, BN, BK>& st = stages[NS == 2 ? (it & 1) : 0];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4);
            T ac[RB], as[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                ac[q] = st.a_re[kr][wm * 16 * RB + q * 16 + (lane & 15)];
                as[q] = st.a_im[kr][wm * 16 * RB + q * 16 + (lane & 15)];
            }
            T pr[4], pi[4], mr[4], mn[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int col = wn * 64 + c * 16 + (lane & 15);
                pr[c] = st.bp_re[kr][col];
                pi[c] = st.bp_im[kr][col];
                mr[c] = st.bm_re[kr][col];
                mn[c] = st.bm_ni[kr][col];
            }
            // each accumulator's second update follows its first by 4 RB MFMAs
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) cr[q * 4 + c] = mfma4(ac[q], pr[c], cr[q * 4 + c]);
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) ci[q * 4 + c] = mfma4(ac[q], pi[c], ci[q * 4 + c]);
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) cr[q * 4 + c] = mfma4(as[q], mn[c], cr[q * 4 + c]);
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) ci[q * 4 + c] = mfma4(as[q], mr[c], ci[q * 4 + c]);
        }
        if constexpr (NS == 2) {
            if (more) sstore(stages[(it + 1) & 1]);
            __syncthreads();
        } else {
            __syncthreads();
            if (more) {
                sstore(stages[0]);
                __syncthreads();
            }
        }
    }
}

// ---------------------------------------- real A times complex B main loop
//
// C (complex) = A (real) B (complex): two real MFMAs per block product
// (A B re, A B im).  afetch(m, k) gives the real A entry, bfetch(k, n) the
// complex B entry; the same block, wave and staging layout as cgemm_mainloop
// (64-column tiles).
template <typename T, int BM, int BN, int BK>
struct RStage {
    static constexpr int PAD = 16;
    T a[BK][BM + PAD];
    T b_re[BK][BN + PAD];
    T b_im[BK][BN + PAD];
};
template <typename T, int BM, int BN, int BK, class AF, class BF, int NS = 2>
__device__ inline void rgemm_mainloop(RStage<T, BM, BN, BK>* stages, int K, AF afetch, BF bfetch,
                                      typename Cx<T>::acc (&cr)[4 * CWaves<BM, BN>::RB],
                                      typename Cx<T>::acc (&ci)[4 * CWaves<BM, BN>::RB])
{
    static_assert(NS == 1 || NS == 2, "one or two LDS stages");
    typedef typename Cx<T>::type CT;
    constexpr int WN = CWaves<BM, BN>::WN;
    constexpr int RB = CWaves<BM, BN>::RB;
    static_assert(RB >= 1 && 16 * RB * (4 / WN) == BM && BN < 256, "wave layout");
    constexpr int AE = BM * BK / 256;
    constexpr int BE = BK * BN / 256;
    static_assert(AE >= 1 && AE * 256 == BM * BK && BE >= 1 && BE * 256 == BK * BN, "tile for 256 threads");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    T ra[AE];
    CT rb[BE];
    for (int c = 0; c < 4 * RB; ++c)
        for (int i = 0; i < 4; ++i) {
            cr[c][i] = T(0);
            ci[c][i] = T(0);
        }
    // A is fetched k-fastest across threads (its source is K-major: a phase
    // table [k][h]), B as in cgemm_mainloop
    auto gload = [&](int k0) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = tid * AE + e;
            ra[e] = afetch(idx % BM, k0 + idx / BM);
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = tid * BE + e;
            rb[e] = bfetch(k0 + idx / BN, idx % BN);
        }
    };
    auto sstore = [&](RStage<T, BM, BN, BK>& st) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = tid * AE + e;
            st.a[idx / BM][idx % BM] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = tid * BE + e;
            st.b_re[idx / BN][idx % BN] = rb[e].x;
            st.b_im[idx / BN][idx % BN] = rb[e].y;
        }
    };
    gload(0);
    sstore(stages[0]);
    __syncthreads();
    for (int k0 = 0, it = 0; k0 < K; k0 += BK, ++it) {
        const bool more = k0 + BK < K;
        if (more) gload(k0 + BK);
        const RStage<T, BM, BN, BK>& st = stages[NS == 2 ? (it & 1) : 0];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4);
            T av[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) av[q] = st.a[kr][wm * 16 * RB + q * 16 + (lane & 15)];
            T br[4], bi[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                br[c] = st.b_re[kr][wn * 64 + c * 16 + (lane & 15)];
                bi[c] = st.b_im[kr][wn * 64 + c * 16 + (lane & 15)];
            }
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) cr[q * 4 + c] = mfma4(av[q], br[c], cr[q * 4 + c]);
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) ci[q * 4 + c] = mfma4(av[q], bi[c], ci[q * 4 + c]);
        }
        if constexpr (NS == 2) {
            if (more) sstore(stages[(it + 1) & 1]);
            __syncthreads();
        } else {
            __syncthreads();
            if (more) {
                sstore(stages[0]);
                __syncthreads();
            }
        }
    }
}

}  // namespace
}  // namespace epw
