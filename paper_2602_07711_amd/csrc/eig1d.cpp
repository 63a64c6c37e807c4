// Host 1D eigen-decomposition of Lambda-bar (EigT Step 1, Sec. 4.1 eq. EIG_SOLVER; matrix of eq.
// lambda_mat_definition): the N x N tridiagonal with zero diagonal, unit off-diagonals, gamma in both corners
// and zeta in the corner off-diagonals (row 1 column 2 and row N column N-1). With S = diag(sqrt(zeta), 1, ...,
// 1, sqrt(zeta)), B = S^{-1} Lambda-bar S is complex symmetric (sqrt(zeta) on both corner off-diagonals); B is
// decomposed as W diag(d) W^{-1} and Lambda-bar = (S W) diag(d) (W^{-1} S^{-1}). For zeta = 1, S = I. B is
// complex symmetric but not Hermitian, so W is non-unitary.
//
//   1. eigenvalues: shifted QR iteration (Wilkinson shift, unitary Givens rotations) on the dense upper
//      Hessenberg copy of the matrix, with deflation on small subdiagonal entries;
//   2. eigenvectors: inverse iteration with the tridiagonal matrix (LU with partial pivoting), alternating
//      with the two-sided Rayleigh quotient x^T A x / x^T x (left = right eigenvector for a complex
//      symmetric matrix), which also polishes each eigenvalue;
//   3. V^{-1}: LU with partial pivoting of the dense V;
//   4. checks: ||A V - V D||_max and ||V^{-1} V - I||_max.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "helm_internal.h"

namespace helm {

using cd = std::complex<double>;

namespace {

// Givens rotation [[c, s], [-conj(s), c]] mapping (a, b) to (r, 0), c real.
inline void givens(cd a, cd b, double &c, cd &s) {
    double aa = std::abs(a), bb = std::abs(b);
    if (bb == 0.0) { c = 1.0; s = 0.0; return; }
    if (aa == 0.0) { c = 0.0; s = 1.0; return; }
    double t = std::hypot(aa, bb);
    c = aa / t;
    s = (a / aa) * std::conj(b) / t;
}

// Eigenvalues of a dense upper Hessenberg matrix H (row-major, n x n), destroyed on exit.
bool hessenberg_qr_eigenvalues(std::vector<cd> &H, int n, std::vector<cd> &ev) {
    const double eps = 2.220446049250313e-16;
    ev.assign(n, cd(0.0));
    auto at = [&](int i, int j) -> cd & { return H[(size_t)i * n + j]; };
    std::vector<double> cs(n);
    std::vector<cd> sn(n);
    int hi = n - 1;
    int total_iter = 0;
    while (hi >= 0) {
        int iter = 0;
        for (;;) {
            int lo = hi;
            while (lo > 0) {
                double tst = std::abs(at(lo - 1, lo - 1)) + std::abs(at(lo, lo));
                if (tst == 0.0) tst = 1.0;
                if (std::abs(at(lo, lo - 1)) <= eps * tst) break;
                --lo;
            }
            if (lo > 0) at(lo, lo - 1) = 0.0;
            if (lo == hi) { ev[hi] = at(hi, hi); --hi; break; }
            if (++iter > 60 || ++total_iter > 60 * n) return false;
            // Wilkinson shift from the trailing 2x2 block of the active window
            cd a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
            cd mu;
            if (iter % 11 == 10) {
                mu = d + cd(std::abs(c), 0.0) * 0.75;   // exceptional shift
            } else {
                cd half = (a - d) * 0.5;
                cd disc = std::sqrt(half * half + b * c);
                cd m1 = (a + d) * 0.5 + disc, m2 = (a + d) * 0.5 - disc;
                mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
            }
            // explicit single-shift QR step on rows/cols lo..hi: H - mu I = Q R, H <- R Q + mu I
            for (int k = lo; k <= hi; ++k) at(k, k) -= mu;
            for (int k = lo; k < hi; ++k) {
                givens(at(k, k), at(k + 1, k), cs[k], sn[k]);
                for (int j = k; j <= hi; ++j) {
                    cd x = at(k, j), y = at(k + 1, j);
                    at(k, j) = cs[k] * x + sn[k] * y;
                    at(k + 1, j) = -std::conj(sn[k]) * x + cs[k] * y;
                }
            }
            for (int k = lo; k < hi; ++k) {
                int rmax = std::min(k + 2, hi);
                for (int i = lo; i <= rmax; ++i) {
                    cd p = at(i, k), q = at(i, k + 1);
                    at(i, k) = p * cs[k] + q * std::conj(sn[k]);
                    at(i, k + 1) = -p * sn[k] + q * cs[k];
                }
            }
            for (int k = lo; k <= hi; ++k) at(k, k) += mu;
        }
    }
    return true;
}

// Solve (T - lam I) x = b for the tridiagonal T (sub-diagonal lo, diagonal di, super-diagonal up) by
// Gaussian elimination with partial pivoting; b is overwritten with x.
void tridiag_shifted_solve(const std::vector<cd> &lo, const std::vector<cd> &di, const std::vector<cd> &up,
                           cd lam, std::vector<cd> &b, double tiny) {
    int n = (int)di.size();
    // U has up to two super-diagonals after pivoting
    std::vector<cd> u0(n), u1(n, 0.0), u2(n, 0.0);
    std::vector<cd> l(n, 0.0);
    std::vector<int> piv(n, 0);
    // working rows: current row k holds (u0[k], u1[k], u2[k]) in columns k, k+1, k+2
    std::vector<cd> rowd(n), rowu(n);
    for (int k = 0; k < n; ++k) { rowd[k] = di[k] - lam; rowu[k] = (k + 1 < n) ? up[k] : cd(0.0); }
    cd cur0 = rowd[0], cur1 = (n > 1) ? rowu[0] : cd(0.0), cur2 = 0.0;
    for (int k = 0; k < n - 1; ++k) {
        cd sub = lo[k];                  // entry (k+1, k)
        cd nxt0 = rowd[k + 1], nxt1 = (k + 2 < n) ? rowu[k + 1] : cd(0.0), nxt2 = 0.0;
        if (std::abs(sub) > std::abs(cur0)) {
            // swap rows k and k+1
            piv[k] = 1;
            std::swap(b[k], b[k + 1]);
            cd t0 = cur0, t1 = cur1, t2 = cur2;
            cur0 = sub; cur1 = nxt0; cur2 = nxt1;
            nxt0 = t0; nxt1 = t1; nxt2 = t2;
            // the old row k had zero in column k+2 beyond cur2 (cur2 is column k+2)
            cd m = nxt0 / cur0;
            l[k] = m;
            nxt0 = nxt1 - m * cur1;      // column k+1
            nxt1 = nxt2 - m * cur2;      // column k+2
            b[k + 1] -= m * b[k];
        } else {
            if (cur0 == cd(0.0)) cur0 = tiny;
            cd m = sub / cur0;
            l[k] = m;
            nxt0 = nxt0 - m * cur1;
            nxt1 = nxt1 - m * cur2;
            b[k + 1] -= m * b[k];
        }
        u0[k] = cur0; u1[k] = cur1; u2[k] = cur2;
        cur0 = nxt0; cur1 = nxt1; cur2 = 0.0;
    }
    if (cur0 == cd(0.0) || std::abs(cur0) < tiny) cur0 = (cur0 == cd(0.0)) ? cd(tiny) : cur0 / std::abs(cur0) * tiny;
    u0[n - 1] = cur0; u1[n - 1] = 0.0; u2[n - 1] = 0.0;
    for (int k = n - 1; k >= 0; --k) {
        cd s = b[k];
        if (k + 1 < n) s -= u1[k] * b[k + 1];
        if (k + 2 < n) s -= u2[k] * b[k + 2];
        cd d0 = u0[k];
        if (std::abs(d0) < tiny) d0 = tiny;
        b[k] = s / d0;
    }
}

// In-place inverse of a dense n x n complex matrix (row-major) by LU with partial pivoting.
bool invert(std::vector<cd> &A, int n) {
    std::vector<cd> inv((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::abs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = std::abs(A[(size_t)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) return false;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
                std::swap(inv[(size_t)k * n + j], inv[(size_t)p * n + j]);
            }
        }
        cd piv = A[(size_t)k * n + k];
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            cd m = A[(size_t)i * n + k] / piv;
            if (m == cd(0.0)) continue;
            for (int j = k; j < n; ++j) A[(size_t)i * n + j] -= m * A[(size_t)k * n + j];
            for (int j = 0; j < n; ++j) inv[(size_t)i * n + j] -= m * inv[(size_t)k * n + j];
        }
        for (int j = k; j < n; ++j) A[(size_t)k * n + j] /= piv;
        for (int j = 0; j < n; ++j) inv[(size_t)k * n + j] /= piv;
    }
    A.swap(inv);
    return true;
}

}  // namespace

bool eig_lambda_bar(int n, cd gamma, std::vector<cd> &d, std::vector<cd> &V, std::vector<cd> &Vinv,
                    std::string &err, double zeta) {
    if (n < 2) { err = "eig1d: n must be >= 2"; return false; }
    if (!(zeta > 0.0)) { err = "eig1d: zeta must be positive"; return false; }
    // tridiagonal entries of the symmetrised B
    const double sz = std::sqrt(zeta);
    std::vector<cd> lo(n - 1, 1.0), up(n - 1, 1.0), di(n, 0.0);
    di[0] += gamma;
    di[n - 1] += gamma;
    lo[0] = up[0] = sz;
    lo[n - 2] = up[n - 2] = sz;
    std::vector<cd> H((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        H[(size_t)i * n + i] = di[i];
        if (i + 1 < n) { H[(size_t)i * n + i + 1] = up[i]; H[(size_t)(i + 1) * n + i] = lo[i]; }
    }
    std::vector<cd> ev;
    if (!hessenberg_qr_eigenvalues(H, n, ev)) { err = "eig1d: QR iteration did not converge"; return false; }

    auto apply = [&](const std::vector<cd> &x, std::vector<cd> &y) {
        for (int i = 0; i < n; ++i) {
            cd s = di[i] * x[i];
            if (i > 0) s += lo[i - 1] * x[i - 1];
            if (i + 1 < n) s += up[i] * x[i + 1];
            y[i] = s;
        }
    };
    const double anorm = 2.0 * sz + std::abs(gamma);
    const double tiny = 1e-300 + anorm * 1e-18;
    V.assign((size_t)n * n, 0.0);
    d.assign(n, 0.0);
    std::vector<cd> x(n), y(n);
    for (int k = 0; k < n; ++k) {
        cd lam = ev[k];
        // deterministic start vector with no special symmetry
        for (int i = 0; i < n; ++i) x[i] = cd(1.0 + 0.37 * std::sin(1.3 * i + 0.7 * k), 0.11 * std::cos(2.1 * i));
        for (int it = 0; it < 4; ++it) {
            tridiag_shifted_solve(lo, di, up, lam, x, tiny);
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) nrm += std::norm(x[i]);
            nrm = std::sqrt(nrm);
            for (int i = 0; i < n; ++i) x[i] /= nrm;
            if (it >= 1) {   // two-sided Rayleigh quotient (complex symmetric: left vector = x^T)
                apply(x, y);
                cd num = 0.0, den = 0.0;
                for (int i = 0; i < n; ++i) { num += x[i] * y[i]; den += x[i] * x[i]; }
                if (std::abs(den) > 1e-8) lam = num / den;
            }
        }
        d[k] = lam;
        for (int i = 0; i < n; ++i) V[(size_t)i * n + k] = x[i];
    }
    // checks: ||A V - V D||_max relative to ||A|| and ||V^{-1} V - I||_max
    double res = 0.0;
    for (int k = 0; k < n; ++k) {
        for (int i = 0; i < n; ++i) x[i] = V[(size_t)i * n + k];
        apply(x, y);
        for (int i = 0; i < n; ++i) res = std::max(res, std::abs(y[i] - d[k] * x[i]));
    }
    if (!(res <= 1e-11 * anorm)) { err = "eig1d: eigenpair residual too large"; return false; }
    Vinv = V;
    if (!invert(Vinv, n)) { err = "eig1d: eigenvector matrix is singular"; return false; }
    double ortho = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            cd s = 0.0;
            for (int k = 0; k < n; ++k) s += Vinv[(size_t)i * n + k] * V[(size_t)k * n + j];
            ortho = std::max(ortho, std::abs(s - (i == j ? cd(1.0) : cd(0.0))));
        }
    }
    if (!(ortho <= 1e-9)) { err = "eig1d: V^{-1} V differs from I"; return false; }
    if (zeta != 1.0) {              // V = S W, V^{-1} = W^{-1} S^{-1}
        for (int k = 0; k < n; ++k) {
            V[k] *= sz;
            V[(size_t)(n - 1) * n + k] *= sz;
            Vinv[(size_t)k * n] /= sz;
            Vinv[(size_t)k * n + n - 1] /= sz;
        }
    }
    return true;
}

}  // namespace helm
