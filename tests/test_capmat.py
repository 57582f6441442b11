"""Host linear algebra of the metal-mask correction (mc_capmat.hpp), compiled
on the CPU with g++: the list of mask nodes among the Poisson unknowns, and
the in-place Gauss-Jordan inverse against the identity A A^-1 = I on random
matrices, on matrices that need row interchanges (zero leading diagonal,
permuted identities) and on a singular matrix."""
import os
import subprocess

HARNESS = r'''
#include "mc_capmat.hpp"
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
using namespace mc;
static double check(const std::vector<double> &a, const std::vector<double> &inv, int n) {
    double worst = 0;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            double s = 0;
            for (int k = 0; k < n; ++k) s += a[(size_t)r * n + k] * inv[(size_t)k * n + c];
            worst = std::fmax(worst, std::fabs(s - (r == c ? 1.0 : 0.0)));
        }
    return worst;
}
int main() {
    std::mt19937_64 rng(11);
    std::uniform_real_distribution<double> u(-1, 1);
    for (int n : {1, 2, 3, 7, 40, 130}) {
        std::vector<double> a((size_t)n * n);
        for (auto &x : a) x = u(rng);
        for (int k = 0; k < n; ++k) a[(size_t)k * n + k] += (k % 3 == 0) ? 0.0 : 2.0;
        if (n > 1) a[0] = 0.0;  // forces a row interchange at the first pivot
        auto inv = a;
        if (!invert_in_place(inv, n) || check(a, inv, n) > 1e-10) { std::printf("FAIL random %d\n", n); return 1; }
        // a permutation matrix: its inverse is its transpose
        std::vector<int> perm(n);
        for (int k = 0; k < n; ++k) perm[k] = k;
        std::shuffle(perm.begin(), perm.end(), rng);
        std::vector<double> p((size_t)n * n, 0.0);
        for (int k = 0; k < n; ++k) p[(size_t)k * n + perm[k]] = 1.0;
        auto pinv = p;
        if (!invert_in_place(pinv, n)) { std::puts("FAIL perm"); return 1; }
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c)
                if (pinv[(size_t)r * n + c] != p[(size_t)c * n + r]) { std::puts("FAIL perm inverse"); return 1; }
    }
    std::vector<double> sing = {1, 2, 3, 2, 4, 6, 1, 0, 1};
    if (invert_in_place(sing, 3)) { std::puts("FAIL singular accepted"); return 1; }
    // mask nodes: boundary rows j = 0, nz-1 and the outer column i = nr-1 are excluded
    const int nr = 5, nz = 6;
    std::vector<uint8_t> mask(nr * nz, 0);
    mask[0 * nr + 1] = 1;              // j = 0: boundary
    mask[2 * nr + 0] = 1;              // axis node, kept
    mask[3 * nr + 4] = 1;              // i = nr-1: boundary
    mask[4 * nr + 2] = 1;              // kept
    mask[5 * nr + 2] = 1;              // j = nz-1: boundary
    auto v = mask_unknowns(mask.data(), nr, nz);
    if (v.size() != 2 || v[0] != 2 * nr + 0 || v[1] != 4 * nr + 2) { std::puts("FAIL mask nodes"); return 1; }
    if (!mask_unknowns(nullptr, nr, nz).empty()) { std::puts("FAIL null mask"); return 1; }
    std::puts("OK");
    return 0;
}
'''


def test_capacitance_linear_algebra(tmp_path):
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2609_31258_amd", "csrc")
    src = tmp_path / "capmat_test.cpp"
    src.write_text(HARNESS.replace("#include <vector>\n", "#include <vector>\n#include <algorithm>\n", 1))
    exe = tmp_path / "capmat_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Xlinker", "--no-as-needed", "-fsanitize=address,undefined",
                    "-I" + csrc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.strip()
    assert out == "OK"
