// Host 1D eigen-decomposition of Lambda-bar (EigT Step 1, Sec. 4.1 eq. EIG_SOLVER; matrix of eq.
// lambda_mat_definition): the N x N tridiagonal with zero diagonal, unit off-diagonals, gamma in both corners
// and zeta in the corner off-diagonals (row 1 column 2 and row N column N-1). With S = diag(sqrt(zeta), 1, ...,
// 1, sqrt(zeta)), B = S^{-1} Lambda-bar S is complex symmetric (sqrt(zeta) on both corner off-diagonals); B is
// decomposed as W diag(d) W^{-1} and Lambda-bar = (S W) diag(d) (W^{-1} S^{-1}). For zeta = 1, S = I. B is
// complex symmetric but not Hermitian, so W is non-unitary.
//
// Both ends carry the same closure, so B is centrosymmetric (J B J = B, J the exchange matrix). With the
// orthogonal Q whose columns are (e_i + e_{N-1-i})/sqrt(2) (symmetric half, plus e_m in the middle for odd
// N) and (e_i - e_{N-1-i})/sqrt(2) (skew half), Q^T B Q = diag(B_s, B_a): two tridiagonal blocks of sizes
// ceil(N/2) and floor(N/2). For even N = 2m they are the leading m x m block of B with b_{m-1,m} added to
// (B_s) or subtracted from (B_a) its last diagonal entry; for odd N = 2m+1, B_s is the leading (m+1) x
// (m+1) block with its last off-diagonal scaled by sqrt(2) and B_a the leading m x m block. Each block is
// decomposed separately and V = S Q diag(W_s, W_a) = Q diag(S_h W_s, S_h W_a), S_h = diag(sqrt(zeta), 1,
// ..., 1); the modes are ordered [symmetric | skew]. The preconditioner's transforms apply Q and the two
// half-size blocks instead of the dense V (half the flops); the dense V and V^{-1} are assembled for the
// other users.
//
// Per block:
//   1. eigenvalues: shifted QR iteration (Wilkinson shift, unitary Givens rotations) on the dense upper
//      Hessenberg copy of the matrix, with deflation on small subdiagonal entries;
//   2. eigenvectors: inverse iteration with the tridiagonal matrix (LU with partial pivoting), alternating
//      with the two-sided Rayleigh quotient x^T A x / x^T x (left = right eigenvector for a complex
//      symmetric matrix), which also polishes each eigenvalue;
//   3. W^{-1}: LU with partial pivoting of the dense W;
//   4. checks: ||B W - W D||_max and ||W^{-1} W - I||_max.
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

// Eigen-decomposition B = W diag(d) W^{-1} of the complex symmetric tridiagonal B with diagonal di and
// off-diagonal off (both sides). Returns false with err set when the QR iteration fails or a check fails.
bool eig_sym_tridiag(const std::vector<cd> &di, const std::vector<cd> &off, std::vector<cd> &d, std::vector<cd> &W,
                     std::vector<cd> &Winv, std::string &err) {
    const int n = (int)di.size();
    const std::vector<cd> &lo = off, &up = off;
    std::vector<cd> H((size_t)n * n, 0.0);
    double anorm = 0.0;
    for (int i = 0; i < n; ++i) {
        H[(size_t)i * n + i] = di[i];
        if (i + 1 < n) { H[(size_t)i * n + i + 1] = up[i]; H[(size_t)(i + 1) * n + i] = lo[i]; }
        double row = std::abs(di[i]) + (i > 0 ? std::abs(off[i - 1]) : 0.0) + (i + 1 < n ? std::abs(off[i]) : 0.0);
        anorm = std::max(anorm, row);
    }
    if (anorm == 0.0) anorm = 1.0;
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
    const double tiny = 1e-300 + anorm * 1e-18;
    W.assign((size_t)n * n, 0.0);
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
        for (int i = 0; i < n; ++i) W[(size_t)i * n + k] = x[i];
    }
    // checks: ||B W - W D||_max relative to ||B|| and ||W^{-1} W - I||_max
    double res = 0.0;
    for (int k = 0; k < n; ++k) {
        for (int i = 0; i < n; ++i) x[i] = W[(size_t)i * n + k];
        apply(x, y);
        for (int i = 0; i < n; ++i) res = std::max(res, std::abs(y[i] - d[k] * x[i]));
    }
    if (!(res <= 1e-11 * anorm)) { err = "eig1d: eigenpair residual too large"; return false; }
    Winv = W;
    if (!invert(Winv, n)) { err = "eig1d: eigenvector matrix is singular"; return false; }
    double ortho = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            cd s = 0.0;
            for (int k = 0; k < n; ++k) s += Winv[(size_t)i * n + k] * W[(size_t)k * n + j];
            ortho = std::max(ortho, std::abs(s - (i == j ? cd(1.0) : cd(0.0))));
        }
    }
    if (!(ortho <= 1e-9)) { err = "eig1d: V^{-1} V differs from I"; return false; }
    return true;
}

}  // namespace

bool eig_lambda_bar_folded(int n, cd gamma, double zeta, EigFold &f, std::string &err) {
    if (n < 2) { err = "eig1d: n must be >= 2"; return false; }
    if (!(zeta > 0.0)) { err = "eig1d: zeta must be positive"; return false; }
    const double sz = std::sqrt(zeta);
    // tridiagonal entries of the symmetrised B
    std::vector<cd> di(n, 0.0), off(n - 1, 1.0);
    di[0] += gamma;
    di[n - 1] += gamma;
    off[0] = sz;
    off[n - 2] = sz;
    if (n == 2) off[0] = zeta;   // both corners are the one off-diagonal pair and S = sqrt(zeta) I
    const int m = n / 2;
    f.n = n;
    f.ms = n - m;
    f.ma = m;
    // the two blocks of Q^T B Q (B is centrosymmetric)
    std::vector<cd> ds(di.begin(), di.begin() + f.ms), da(di.begin(), di.begin() + m);
    std::vector<cd> os(off.begin(), off.begin() + (f.ms - 1)), oa(off.begin(), off.begin() + (m - 1));
    if (n % 2 == 0) {
        ds[m - 1] += off[m - 1];
        da[m - 1] -= off[m - 1];
    } else {
        os[m - 1] = std::sqrt(2.0) * off[m - 1];
    }
    if (!eig_sym_tridiag(ds, os, f.ds, f.Vs, f.Vsi, err)) return false;
    if (!eig_sym_tridiag(da, oa, f.da, f.Va, f.Vai, err)) return false;
    if (zeta != 1.0) {   // block position 0 is the corner of both halves: V = S W, V^{-1} = W^{-1} S^{-1}
        for (int k = 0; k < f.ms; ++k) { f.Vs[k] *= sz; f.Vsi[(size_t)k * f.ms] /= sz; }
        for (int k = 0; k < f.ma; ++k) { f.Va[k] *= sz; f.Vai[(size_t)k * f.ma] /= sz; }
    }
    return true;
}

void eig_fold_dense(const EigFold &f, std::vector<cd> &d, std::vector<cd> &V, std::vector<cd> &Vinv) {
    // V = Q diag(Vs, Va), V^{-1} = diag(Vs^{-1}, Va^{-1}) Q^T; modes ordered [symmetric | skew]
    const int n = f.n, ms = f.ms, ma = f.ma;
    const double r = 1.0 / std::sqrt(2.0);
    d.assign(n, 0.0);
    V.assign((size_t)n * n, 0.0);
    Vinv.assign((size_t)n * n, 0.0);
    for (int k = 0; k < ms; ++k) d[k] = f.ds[k];
    for (int k = 0; k < ma; ++k) d[ms + k] = f.da[k];
    for (int i = 0; i < ma; ++i) {
        for (int k = 0; k < ms; ++k) {
            V[(size_t)i * n + k] = f.Vs[(size_t)i * ms + k] * r;
            V[(size_t)(n - 1 - i) * n + k] = f.Vs[(size_t)i * ms + k] * r;
            Vinv[(size_t)k * n + i] = f.Vsi[(size_t)k * ms + i] * r;
            Vinv[(size_t)k * n + n - 1 - i] = f.Vsi[(size_t)k * ms + i] * r;
        }
        for (int k = 0; k < ma; ++k) {
            V[(size_t)i * n + ms + k] = f.Va[(size_t)i * ma + k] * r;
            V[(size_t)(n - 1 - i) * n + ms + k] = -f.Va[(size_t)i * ma + k] * r;
            Vinv[(size_t)(ms + k) * n + i] = f.Vai[(size_t)k * ma + i] * r;
            Vinv[(size_t)(ms + k) * n + n - 1 - i] = -f.Vai[(size_t)k * ma + i] * r;
        }
    }
    if (ms > ma) {   // odd n: the middle position belongs to the symmetric half only
        for (int k = 0; k < ms; ++k) {
            V[(size_t)ma * n + k] = f.Vs[(size_t)ma * ms + k];
            Vinv[(size_t)k * n + ma] = f.Vsi[(size_t)k * ms + ma];
        }
    }
}

bool eig_lambda_bar(int n, cd gamma, std::vector<cd> &d, std::vector<cd> &V, std::vector<cd> &Vinv,
                    std::string &err, double zeta) {
    EigFold f;
    if (!eig_lambda_bar_folded(n, gamma, zeta, f, err)) return false;
    eig_fold_dense(f, d, V, Vinv);
    return true;
}

}  // namespace helm
