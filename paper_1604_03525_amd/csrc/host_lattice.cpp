// Host-side integer steps: Wigner-Seitz vectors, Gamma-centred grids and the
// k+q index map.  Exact integer arithmetic; no GPU involvement.
#include <cstdint>
#include <cstring>
#include <vector>

#include "epw_internal.h"

namespace {

int64_t norm2(const int64_t G[9], int64_t a, int64_t b, int64_t c) {
    const int64_t v[3] = {a, b, c};
    int64_t s = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s += G[3 * i + j] * v[i] * v[j];
    return s;
}

bool positive_definite(const int64_t G[9]) {
    // Sylvester's criterion on the leading minors, in integers.
    const int64_t m1 = G[0];
    const int64_t m2 = G[0] * G[4] - G[1] * G[3];
    const int64_t m3 = G[0] * (G[4] * G[8] - G[5] * G[7]) -
                       G[1] * (G[3] * G[8] - G[5] * G[6]) +
                       G[2] * (G[3] * G[7] - G[4] * G[6]);
    const bool sym = G[1] == G[3] && G[2] == G[6] && G[5] == G[7];
    return sym && m1 > 0 && m2 > 0 && m3 > 0;
}

}  // namespace

extern "C" int epw_ws_vectors(const int64_t metric[9], const int32_t ncell[3],
                              int32_t* R, int32_t* ndeg, int32_t cap, int32_t* count) {
    using namespace epw;
    clear_error();
    if (!metric || !ncell || !count) return fail(EPW_EINVAL, "epw_ws_vectors: NULL argument");
    if (cap > 0 && (!R || !ndeg)) return fail(EPW_EINVAL, "epw_ws_vectors: NULL output");
    for (int a = 0; a < 3; ++a)
        if (ncell[a] < 1 || ncell[a] > 4096)
            return fail(EPW_EINVAL, "epw_ws_vectors: ncell[%d] = %d out of range", a, ncell[a]);
    if (!positive_definite(metric))
        return fail(EPW_EINVAL, "epw_ws_vectors: metric is not symmetric positive definite");
    const int64_t N[3] = {ncell[0], ncell[1], ncell[2]};
    // the 125 supercell translations T = (N1 t1, N2 t2, N3 t3), t in {-2..2}^3
    std::vector<int64_t> T;
    for (int t1 = -2; t1 <= 2; ++t1)
        for (int t2 = -2; t2 <= 2; ++t2)
            for (int t3 = -2; t3 <= 2; ++t3) {
                T.push_back(N[0] * t1);
                T.push_back(N[1] * t2);
                T.push_back(N[2] * t3);
            }
    int32_t n = 0;
    for (int64_t a = -2 * N[0]; a <= 2 * N[0]; ++a)
        for (int64_t b = -2 * N[1]; b <= 2 * N[1]; ++b)
            for (int64_t c = -2 * N[2]; c <= 2 * N[2]; ++c) {
                const int64_t d0 = norm2(metric, a, b, c);
                int32_t deg = 0;
                bool inside = true;
                for (size_t t = 0; t < T.size(); t += 3) {
                    const int64_t d = norm2(metric, a - T[t], b - T[t + 1], c - T[t + 2]);
                    if (d < d0) { inside = false; break; }
                    if (d == d0) ++deg;
                }
                if (!inside) continue;
                if (n < cap) {
                    R[3 * n + 0] = (int32_t)a;
                    R[3 * n + 1] = (int32_t)b;
                    R[3 * n + 2] = (int32_t)c;
                    ndeg[n] = deg;
                }
                ++n;
            }
    *count = n;
    if (n > cap) return fail(EPW_ENOMEM, "epw_ws_vectors: %d vectors, capacity %d", n, cap);
    return EPW_OK;
}

extern "C" int epw_grid_points(const int32_t n[3], double* out) {
    using namespace epw;
    clear_error();
    if (!n || !out) return fail(EPW_EINVAL, "epw_grid_points: NULL argument");
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1) return fail(EPW_EINVAL, "epw_grid_points: n[%d] = %d", a, n[a]);
    int64_t i = 0;
    for (int32_t i1 = 0; i1 < n[0]; ++i1)
        for (int32_t i2 = 0; i2 < n[1]; ++i2)
            for (int32_t i3 = 0; i3 < n[2]; ++i3, ++i) {
                out[3 * i + 0] = (double)i1 / (double)n[0];
                out[3 * i + 1] = (double)i2 / (double)n[1];
                out[3 * i + 2] = (double)i3 / (double)n[2];
            }
    return EPW_OK;
}

extern "C" int epw_kq_index(const int32_t kgrid[3], const int32_t qgrid[3], int32_t* out) {
    using namespace epw;
    clear_error();
    if (!kgrid || !qgrid || !out) return fail(EPW_EINVAL, "epw_kq_index: NULL argument");
    int64_t K[3], Q[3], ratio[3];
    for (int a = 0; a < 3; ++a) {
        K[a] = kgrid[a];
        Q[a] = qgrid[a];
        if (K[a] < 1 || Q[a] < 1) return fail(EPW_EINVAL, "epw_kq_index: grid size < 1");
        if (K[a] % Q[a] != 0)
            return fail(EPW_ESHAPE, "epw_kq_index: q grid %lld does not divide k grid %lld on axis %d",
                        (long long)Q[a], (long long)K[a], a);
        ratio[a] = K[a] / Q[a];
    }
    const int64_t nk = K[0] * K[1] * K[2], nq = Q[0] * Q[1] * Q[2];
    if (nk * nq > (int64_t)1 << 40) return fail(EPW_ESHAPE, "epw_kq_index: map too large");
    for (int64_t ik = 0; ik < nk; ++ik) {
        const int64_t i1 = ik / (K[1] * K[2]), i2 = (ik / K[2]) % K[1], i3 = ik % K[2];
        int32_t* row = out + ik * nq;
        for (int64_t iq = 0; iq < nq; ++iq) {
            const int64_t j1 = iq / (Q[1] * Q[2]), j2 = (iq / Q[2]) % Q[1], j3 = iq % Q[2];
            const int64_t s1 = (i1 + j1 * ratio[0]) % K[0];
            const int64_t s2 = (i2 + j2 * ratio[1]) % K[1];
            const int64_t s3 = (i3 + j3 * ratio[2]) % K[2];
            row[iq] = (int32_t)((s1 * K[1] + s2) * K[2] + s3);
        }
    }
    return EPW_OK;
}
