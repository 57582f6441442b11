// mc_capmat.hpp -- host-side linear algebra of the metal-mask correction:
// the list of mask nodes among the Poisson unknowns and the in-place inverse
// of the (small, dense) capacitance matrix.  Pure host C++, no device calls.
#pragma once
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

namespace mc {

// Mask nodes among the unknowns (0 <= i <= nr-2, 1 <= j <= nz-2), node order.
inline std::vector<int32_t> mask_unknowns(const uint8_t *mask, int32_t nr, int32_t nz) {
    std::vector<int32_t> v;
    if (!mask) return v;
    for (int32_t j = 1; j <= nz - 2; ++j)
        for (int32_t i = 0; i <= nr - 2; ++i)
            if (mask[(int64_t)j * nr + i]) v.push_back(j * nr + i);
    return v;
}

// In-place inverse of the row-major n x n matrix a (Gauss-Jordan with partial
// pivoting); false if a pivot vanishes.
inline bool invert_in_place(std::vector<double> &a, int32_t n) {
    std::vector<int32_t> perm(n);
    for (int32_t k = 0; k < n; ++k) perm[k] = k;
    for (int32_t k = 0; k < n; ++k) {
        int32_t p = k;
        double best = std::fabs(a[(int64_t)k * n + k]);
        for (int32_t r = k + 1; r < n; ++r) {
            const double v = std::fabs(a[(int64_t)r * n + k]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (!(best > 0.0) || !std::isfinite(best)) return false;
        if (p != k) {
            for (int32_t c = 0; c < n; ++c) std::swap(a[(int64_t)k * n + c], a[(int64_t)p * n + c]);
            std::swap(perm[k], perm[p]);
        }
        double *rk = &a[(int64_t)k * n];
        const double inv = 1.0 / rk[k];
        rk[k] = 1.0;
        for (int32_t c = 0; c < n; ++c) rk[c] *= inv;
        for (int32_t r = 0; r < n; ++r) {
            if (r == k) continue;
            double *rr = &a[(int64_t)r * n];
            const double f = rr[k];
            if (f == 0.0) continue;
            rr[k] = 0.0;
            for (int32_t c = 0; c < n; ++c) rr[c] -= f * rk[c];
        }
    }
    // undo the row interchanges on the columns of the inverse
    std::vector<double> col(n);
    for (int32_t r = 0; r < n; ++r) {
        double *rr = &a[(int64_t)r * n];
        for (int32_t k = 0; k < n; ++k) col[perm[k]] = rr[k];
        for (int32_t k = 0; k < n; ++k) rr[k] = col[k];
    }
    return true;
}

}  // namespace mc
