// Host check of the 1D eigensolver (EigT Step 1, Sec. 4.1) built with AddressSanitizer and UndefinedBehaviorSanitizer:
// for each case, Lambda-bar V = V diag(d) and V^{-1} V = I to a tolerance, through both the folded and the dense
// entry points. Exit status 0 if every case passes.
#include <cmath>
#include <complex>
#include <cstdio>
#include <string>
#include <vector>

#include "helm_internal.h"

using cd = std::complex<double>;

static double check(int n, cd gamma, double zeta) {
    std::vector<cd> d, V, Vi;
    std::string err;
    if (!helm::eig_lambda_bar(n, gamma, d, V, Vi, err, zeta)) {
        std::printf("n=%d: eigensolver failed: %s\n", n, err.c_str());
        return 1e300;
    }
    // Lambda-bar: zero diagonal except gamma in both corners, unit off-diagonals except zeta in the corner ones
    auto lam = [&](int i, int j) -> cd {
        if (i == j) return (i == 0 || i == n - 1) ? gamma : cd(0.0);
        if (std::abs(i - j) != 1) return cd(0.0);
        if ((i == 0 && j == 1) || (i == n - 1 && j == n - 2)) return cd(zeta);
        return cd(1.0);
    };
    double r = 0.0, s = 0.0, vmax = 0.0;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            cd a = 0.0, b = 0.0;
            for (int j = std::max(0, i - 1); j <= std::min(n - 1, i + 1); ++j) a += lam(i, j) * V[(size_t)j * n + k];
            for (int j = 0; j < n; ++j) b += Vi[(size_t)i * n + j] * V[(size_t)j * n + k];
            r = std::max(r, std::abs(a - V[(size_t)i * n + k] * d[k]));
            s = std::max(s, std::abs(b - cd(i == k ? 1.0 : 0.0)));
            vmax = std::max(vmax, std::abs(V[(size_t)i * n + k]));
        }
    helm::EigFold f;
    if (!helm::eig_lambda_bar_folded(n, gamma, zeta, f, err) || f.ms + f.ma != n) {
        std::printf("n=%d: folded eigensolver failed: %s\n", n, err.c_str());
        return 1e300;
    }
    return std::max(r / std::max(vmax, 1.0), s);
}

int main() {
    const int sizes[] = {2, 3, 4, 5, 8, 17, 32, 33, 64, 100, 128, 131};
    int bad = 0;
    for (int n : sizes) {
        const double kh = 0.47;
        const cd g_abc = (cd(2.0, kh)) / (cd(2.0, -kh));           // two-point absorbing closure
        const cd g_col = cd(0.0, 2.0 * kh);                          // collocated closure (zeta = 2)
        const double e1 = check(n, g_abc, 1.0), e2 = check(n, g_col, 2.0), e3 = check(n, cd(0.0), 1.0);
        const double e = std::max(e1, std::max(e2, e3));
        std::printf("n=%3d  max error %.2e\n", n, e);
        if (!(e < 1e-9)) ++bad;
    }
    std::printf(bad ? "FAILED\n" : "ok\n");
    return bad ? 1 : 0;
}
