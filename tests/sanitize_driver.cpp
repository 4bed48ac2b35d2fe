// Host-side checks of the library's integer steps and error reporting, built
// with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py (no GPU involved).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "epw.h"

int main() {
    const int64_t metrics[2][9] = {{1, 0, 0, 0, 1, 0, 0, 0, 1}, {2, 1, 1, 1, 2, 1, 1, 1, 2}};
    int bad = 0;
    for (int mi = 0; mi < 2; ++mi)
        for (int n = 1; n <= 6; ++n) {
            const int32_t nc[3] = {n, n, n + 1};
            int32_t count = 0;
            // a zero capacity reports the count and EPW_ENOMEM
            if (epw_ws_vectors(metrics[mi], nc, nullptr, nullptr, 0, &count) != EPW_ENOMEM || count <= 0) bad++;
            std::vector<int32_t> R(3 * (size_t)count), nd(count);
            if (epw_ws_vectors(metrics[mi], nc, R.data(), nd.data(), count, &count) != EPW_OK) bad++;
            double s = 0.0;
            for (int i = 0; i < count; ++i) s += 1.0 / nd[i];
            if (std::fabs(s - (double)n * n * (n + 1)) > 1e-9) bad++;     // sum rule: cells of the supercell
        }
    const int32_t g[3] = {4, 3, 2};
    std::vector<double> pts(3 * 24);
    if (epw_grid_points(g, pts.data()) != EPW_OK) bad++;
    std::vector<int32_t> kq(24 * 24);
    if (epw_kq_index(g, g, kq.data()) != EPW_OK) bad++;
    for (int v : kq)
        if (v < 0 || v >= 24) bad++;
    const int32_t g3[3] = {3, 3, 2};
    if (epw_kq_index(g, g3, kq.data()) != EPW_ESHAPE) bad++;          // q grid not a divisor
    if (std::strlen(epw_last_error()) == 0) bad++;
    const int64_t singular[9] = {1, 0, 0, 0, 1, 0, 0, 0, 0};
    const int32_t nc[3] = {2, 2, 2};
    int32_t count = 0;
    if (epw_ws_vectors(singular, nc, nullptr, nullptr, 0, &count) != EPW_EINVAL) bad++;
    const int32_t zero[3] = {0, 2, 2};
    if (epw_ws_vectors(metrics[0], zero, nullptr, nullptr, 0, &count) != EPW_EINVAL) bad++;
    if (epw_version() < 100) bad++;
    std::printf("sanitize_driver bad=%d\n", bad);
    return bad != 0;
}
