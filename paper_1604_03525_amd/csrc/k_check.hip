// Input validation kernels (epw_check_inputs): finiteness of every array,
// Wigner-Seitz set properties, the Hermiticity relations H(-R) = H(R)^dag and
// D(-R) = D(R)^T that make the interpolated H(k), D(q) Hermitian before
// their symmetrisation, and the k+q map.  Findings are or-ed into flag words
// and maxima of non-negative doubles (compared as their bit patterns, which
// order like the values) in a small device record.
#include <hip/hip_runtime.h>

#include "epw_internal.h"
#include "kernels.h"

namespace epw {
namespace {

inline unsigned nblk(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ inline void max_bits(unsigned long long* slot, double v) {
    atomicMax(slot, (unsigned long long)__double_as_longlong(v));
}

__global__ void finite_kernel(size_t n, const double* __restrict__ x, int bit, CheckRecord* rec) {
    bool bad = false;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[i]);
    if (bad) atomicOr(&rec->nonfinite, bit);
}

// neg[r] = index of -R[r] (or -1, flagged); ndeg >= 1; |R components| <= nmax when nmax > 0
__global__ void ws_set_kernel(int nR, const int32_t* __restrict__ R, const int32_t* __restrict__ ndeg, int nmax,
                              int bit, int32_t* __restrict__ neg, CheckRecord* rec) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nR) return;
    const int a = R[3 * r], b = R[3 * r + 1], c = R[3 * r + 2];
    if (ndeg[r] < 1) atomicOr(&rec->ndeg_bad, bit);
    if (nmax > 0 && (abs(a) > nmax || abs(b) > nmax || abs(c) > nmax)) atomicOr(&rec->nmax_bad, bit);
    int found = -1;
    for (int t = 0; t < nR; ++t)
        if (R[3 * t] == -a && R[3 * t + 1] == -b && R[3 * t + 2] == -c) {
            found = t;
            break;
        }
    neg[r] = found;
    if (found < 0) atomicOr(&rec->not_closed, bit);
}

// |X_ij(-R) - conj(X_ji(R))| (complex) or |X_ij(-R) - X_ji(R)| (real) and |X_ij(R)|
template <bool CPLX>
__global__ void herm_kernel(int n, int nR, const double* __restrict__ X, const int32_t* __restrict__ neg,
                            unsigned long long* dev_slot, unsigned long long* max_slot) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nn = (size_t)n * n;
    if (idx >= (size_t)nR * nn) return;
    const int r = (int)(idx / nn), e = (int)(idx % nn), i = e / n, j = e % n;
    const int t = neg[r];
    double mag, dev = 0.0;
    if (CPLX) {
        const double2* Z = reinterpret_cast<const double2*>(X);
        const double2 x = Z[idx];
        mag = sqrt(x.x * x.x + x.y * x.y);
        if (t >= 0) {
            const double2 y = Z[(size_t)t * nn + (size_t)j * n + i];
            const double dx = y.x - x.x, dy = y.y + x.y;     // X_ji(-R) - conj(X_ij(R))
            dev = sqrt(dx * dx + dy * dy);
        }
    } else {
        const double x = X[idx];
        mag = fabs(x);
        if (t >= 0) dev = fabs(X[(size_t)t * nn + (size_t)j * n + i] - x);
    }
    max_bits(max_slot, mag);
    max_bits(dev_slot, dev);
}

// for q in [q0, q0 + qc): range of kq[k][q]; inv[t][j] = k
__global__ void kq_scatter_kernel(int nk, int qc, int q0, int nq_total, const int32_t* __restrict__ kq,
                                  int32_t* __restrict__ inv, CheckRecord* rec) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nk * qc) return;
    const int k = (int)(idx / qc), j = (int)(idx % qc);
    const int t = kq[(size_t)k * nq_total + q0 + j];
    if ((unsigned)t >= (unsigned)nk) {
        atomicOr(&rec->kq_range, 1);
        return;
    }
    inv[(size_t)t * qc + j] = k;
}

// every target hit: nk sources on nk targets, so a target never hit means two
// sources share one (the map of that q is not one-to-one)
__global__ void kq_cover_kernel(int nk, int qc, const int32_t* __restrict__ inv, CheckRecord* rec) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nk * qc) return;
    if (inv[idx] < 0) atomicOr(&rec->kq_not_bijective, 1);
}

__global__ void fill_i32(size_t n, int32_t v, int32_t* p) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void clear_record(CheckRecord* rec) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *rec = CheckRecord{};
}

}  // namespace

void launch_check_clear(CheckRecord* rec, hipStream_t st) {
    clear_record<<<1, 64, 0, st>>>(rec);
    launch_check("clear_record");
}

void launch_check_finite(size_t n, const double* x, int bit, CheckRecord* rec, hipStream_t st) {
    if (n == 0 || !x) return;
    const unsigned g = std::min<unsigned>(nblk(n, 256), 4096);
    finite_kernel<<<g, 256, 0, st>>>(n, x, bit, rec);
    launch_check("finite_kernel");
}

void launch_check_ws(int nR, const int32_t* R, const int32_t* ndeg, int nmax, int bit, int32_t* neg,
                     CheckRecord* rec, hipStream_t st) {
    if (nR <= 0) return;
    ws_set_kernel<<<nblk(nR, 128), 128, 0, st>>>(nR, R, ndeg, nmax, bit, neg, rec);
    launch_check("ws_set_kernel");
}

void launch_check_herm(bool cplx, int n, int nR, const double* X, const int32_t* neg, unsigned long long* dev_slot,
                       unsigned long long* max_slot, hipStream_t st) {
    const size_t total = (size_t)nR * n * n;
    if (total == 0 || !X) return;
    if (cplx) herm_kernel<true><<<nblk(total, 256), 256, 0, st>>>(n, nR, X, neg, dev_slot, max_slot);
    else herm_kernel<false><<<nblk(total, 256), 256, 0, st>>>(n, nR, X, neg, dev_slot, max_slot);
    launch_check("herm_kernel");
}

void launch_check_kq(int nk, int qc, int q0, int nq_total, const int32_t* kq, int32_t* inv, CheckRecord* rec,
                     hipStream_t st) {
    const size_t n = (size_t)nk * qc;
    if (n == 0) return;
    fill_i32<<<nblk(n, 256), 256, 0, st>>>(n, -1, inv);
    kq_scatter_kernel<<<nblk(n, 256), 256, 0, st>>>(nk, qc, q0, nq_total, kq, inv, rec);
    kq_cover_kernel<<<nblk(n, 256), 256, 0, st>>>(nk, qc, inv, rec);
    launch_check("kq check kernels");
}

}  // namespace epw
