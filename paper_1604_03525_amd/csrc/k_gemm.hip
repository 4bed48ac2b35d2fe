// Generic strided complex GEMM on MFMA (float64 / float32):
//   C(m, n) (+)= sum_k A(m, k) B(k, n)
// with A read row-major or conjugate-transposed, and the column index n split
// as n = e * ncb + c so that batched slabs (one per Wannier vector R_e) are
// addressed without copies.  Used for the R_p -> q contraction, the
// recomputation of the vertex in the adjoint, and the transposed
// contractions of the adjoint.
#include <hip/hip_runtime.h>

#include "cgemm.h"
#include "epw_internal.h"
#include "kernels.h"

namespace epw {
namespace {

template <typename T, bool CONJ_TRANS_A>
__global__ __launch_bounds__(256) void cgemm_generic_kernel(GemmDesc d)
{
    typedef typename Cx<T>::type CT;
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ Stage<T, BM, BN, BK> st[2];
    const int m0 = blockIdx.y * BM;
    const long n0 = (long)blockIdx.x * BN;
    const CT* A = reinterpret_cast<const CT*>(d.A);
    const CT* B = reinterpret_cast<const CT*>(d.B);
    CT* C = reinterpret_cast<CT*>(d.C);
    auto afetch = [&](int m, int k) -> CT {
        const int row = m0 + m;
        if (row < d.M && k < d.K) {
            if (CONJ_TRANS_A) {
                CT v = A[(size_t)k * d.lda + row];
                v.y = -v.y;
                return v;
            }
            return A[(size_t)row * d.lda + k];
        }
        return cz<T>();
    };
    auto bfetch = [&](int k, int n) -> CT {
        const long col = n0 + n;
        if (k < d.K && col < d.N) {
            const long e = col / d.ncb, c = col % d.ncb;
            return B[(size_t)e * d.sBe + (size_t)k * d.sBk + c];
        }
        return cz<T>();
    };
    typename Cx<T>::acc cr[4], ci[4];
    cgemm_mainloop<T, BM, BN, BK, decltype(afetch), decltype(bfetch), CONJ_TRANS_A, 2>(st, d.K, afetch, bfetch, cr, ci);
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

}  // namespace

void launch_cgemm(Prec prec, const GemmDesc& d, hipStream_t stream) {
    if (d.M <= 0 || d.N <= 0) return;
    dim3 grid((unsigned)((d.N + 63) / 64), (unsigned)((d.M + 63) / 64));
    if (prec == Prec::F64) {
        if (d.conj_trans_a) cgemm_generic_kernel<double, true><<<grid, 256, 0, stream>>>(d);
        else cgemm_generic_kernel<double, false><<<grid, 256, 0, stream>>>(d);
    } else {
        if (d.conj_trans_a) cgemm_generic_kernel<float, true><<<grid, 256, 0, stream>>>(d);
        else cgemm_generic_kernel<float, false><<<grid, 256, 0, stream>>>(d);
    }
    launch_check("cgemm_generic_kernel");
}

}  // namespace epw
