// Host FP64 symmetric eigensolver for the C x C feature covariance of the PCA
// step (Sec. 3.3).  The problem is tiny next to the feature map (C <= 2048),
// so it runs on the host: Householder reduction to tridiagonal form, then the
// implicit QL iteration with shifts (Bowdler, Martin, Reinsch and Wilkinson,
// 1968).  sym_eig accumulates the whole orthogonal transform; sym_eig_top,
// which the fit uses, keeps the reflectors instead, takes all eigenvalues
// from the root-free form of QL, the k leading eigenvectors of the tridiagonal
// matrix by inverse iteration (Wilkinson; vectors of close eigenvalues
// orthogonalised against each other, as in LAPACK's dstein), and applies the
// reflectors to those k vectors only: O(C^3) for the reduction instead of
// the several C^3 of accumulating every rotation.
//
// Host code only, compiled as plain C++ (no device pass).
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

namespace qfca {

// Declared for the library in qfca_internal.h.
int sym_eig(double* A, int n, double* evals, double* vecs);
int sym_eig_top(double* A, int n, int k, double* evals, double* vecs);

namespace {

// Reduce symmetric A (n x n, row-major, destroyed) to tridiagonal T = Q^T A Q.
// d[i] = T[i][i], e[i] = T[i][i+1] (e[n-1] = 0).  Q = H_0 H_1 ... H_{n-3},
// H_k = I - beta_k v_k v_k^T acting on indices k+1 .. n-1: accumulated
// row-major into Q when Q is given; when H is given, v_k is kept in
// H[k n + k + 1 ..] and beta_k in beta[k] (0 for a skipped step).
void householder_tridiag(double* A, int n, double* d, double* e, double* Q, double* H = nullptr,
                         double* beta_out = nullptr) {
    if (Q)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Q[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    if (beta_out)
        for (int i = 0; i < n; ++i) beta_out[i] = 0.0;
    std::vector<double> v(n), p(n), qv(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;  // entries A[k+1..n-1][k]
        double nrm2 = 0.0;
        for (int t = 0; t < len; ++t) {
            const double x = A[(size_t)(k + 1 + t) * n + k];
            nrm2 += x * x;
        }
        if (nrm2 == 0.0) continue;
        const double x0 = A[(size_t)(k + 1) * n + k];
        const double alpha = (x0 > 0.0) ? -sqrt(nrm2) : sqrt(nrm2);
        for (int t = 0; t < len; ++t) v[t] = A[(size_t)(k + 1 + t) * n + k];
        v[0] -= alpha;
        double vn2 = 0.0;
        for (int t = 0; t < len; ++t) vn2 += v[t] * v[t];
        if (vn2 == 0.0) continue;
        const double beta = 2.0 / vn2;
        // p = beta * A_sub v, A_sub = A[k+1.., k+1..]
        double vp = 0.0;
        for (int a = 0; a < len; ++a) {
            const double* row = A + (size_t)(k + 1 + a) * n + (k + 1);
            double s = 0.0;
            for (int b = 0; b < len; ++b) s += row[b] * v[b];
            p[a] = beta * s;
            vp += v[a] * p[a];
        }
        const double K = 0.5 * beta * vp;
        for (int a = 0; a < len; ++a) qv[a] = p[a] - K * v[a];
        // A_sub <- A_sub - v q^T - q v^T
        for (int a = 0; a < len; ++a) {
            double* row = A + (size_t)(k + 1 + a) * n + (k + 1);
            const double va = v[a], qa = qv[a];
            for (int b = 0; b < len; ++b) row[b] -= va * qv[b] + qa * v[b];
        }
        A[(size_t)(k + 1) * n + k] = alpha;
        A[(size_t)k * n + (k + 1)] = alpha;
        for (int t = 1; t < len; ++t) {
            A[(size_t)(k + 1 + t) * n + k] = 0.0;
            A[(size_t)k * n + (k + 1 + t)] = 0.0;
        }
        if (H) {
            for (int t = 0; t < len; ++t) H[(size_t)k * n + k + 1 + t] = v[t];
            beta_out[k] = beta;
        }
        if (!Q) continue;
        // Q[:, k+1..] <- Q[:, k+1..] (I - beta v v^T)
        for (int rI = 0; rI < n; ++rI) {
            double* row = Q + (size_t)rI * n + (k + 1);
            double s = 0.0;
            for (int b = 0; b < len; ++b) s += row[b] * v[b];
            s *= beta;
            for (int b = 0; b < len; ++b) row[b] -= s * v[b];
        }
    }
    for (int i = 0; i < n; ++i) {
        d[i] = A[(size_t)i * n + i];
        e[i] = (i + 1 < n) ? A[(size_t)i * n + i + 1] : 0.0;
    }
}

// The same reduction working on the lower triangle of A only (A[i][j],
// j <= i, row-major; the upper triangle is neither read nor written), with the
// reflectors kept in H and beta: the symmetric product p = beta A v reads each
// stored entry once (a dot product along the row and an update of p along
// the same row), and the rank-2 update A -= v q^T + q v^T touches the stored
// half only, so a step costs about 4 len^2 operations instead of 6.  The
// row loops are contiguous; the dot products keep four partial sums.
// Compiled twice, for AVX2 and for the baseline, the first taken at load time
// where the processor has it (the row loops then run four doubles wide).
__attribute__((target_clones("avx2", "default"))) void householder_tridiag_lower(double* A, int n, double* d,
                                                                                 double* e, double* H,
                                                                                 double* beta_out) {
    for (int i = 0; i < n; ++i) beta_out[i] = 0.0;
    for (int i = 0; i < n; ++i) e[i] = 0.0;
    std::vector<double> v(n), p(n), qv(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;  // entries A[k+1..n-1][k]
        double nrm2 = 0.0;
        for (int t = 0; t < len; ++t) {
            const double x = A[(size_t)(k + 1 + t) * n + k];
            nrm2 += x * x;
        }
        if (nrm2 == 0.0) {
            e[k] = 0.0;
            continue;
        }
        const double x0 = A[(size_t)(k + 1) * n + k];
        const double alpha = (x0 > 0.0) ? -sqrt(nrm2) : sqrt(nrm2);
        for (int t = 0; t < len; ++t) v[t] = A[(size_t)(k + 1 + t) * n + k];
        v[0] -= alpha;
        double vn2 = 0.0;
        for (int t = 0; t < len; ++t) vn2 += v[t] * v[t];
        e[k] = alpha;
        if (vn2 == 0.0) continue;
        const double beta = 2.0 / vn2;
        // p = A_sub v from the lower triangle: row a contributes
        // sum_{b<a} A[a][b] v[b] to p[a] and A[a][b] v[a] to every p[b], b < a
        double* __restrict__ pp = p.data();
        const double* __restrict__ vv = v.data();
        for (int a = 0; a < len; ++a) pp[a] = 0.0;
        for (int a = 0; a < len; ++a) {
            const double* __restrict__ row = A + (size_t)(k + 1 + a) * n + (k + 1);
            const double va = vv[a];
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int b = 0;
            for (; b + 4 <= a; b += 4) {
                s0 += row[b] * vv[b];
                s1 += row[b + 1] * vv[b + 1];
                s2 += row[b + 2] * vv[b + 2];
                s3 += row[b + 3] * vv[b + 3];
                pp[b] += row[b] * va;
                pp[b + 1] += row[b + 1] * va;
                pp[b + 2] += row[b + 2] * va;
                pp[b + 3] += row[b + 3] * va;
            }
            for (; b < a; ++b) {
                s0 += row[b] * vv[b];
                pp[b] += row[b] * va;
            }
            pp[a] += (s0 + s1) + (s2 + s3) + row[a] * va;
        }
        double vp = 0.0;
        for (int a = 0; a < len; ++a) {
            pp[a] *= beta;
            vp += vv[a] * pp[a];
        }
        const double K = 0.5 * beta * vp;
        double* __restrict__ qq = qv.data();
        for (int a = 0; a < len; ++a) qq[a] = pp[a] - K * vv[a];
        // A_sub <- A_sub - v q^T - q v^T, lower triangle
        for (int a = 0; a < len; ++a) {
            double* __restrict__ row = A + (size_t)(k + 1 + a) * n + (k + 1);
            const double va = vv[a], qa = qq[a];
            for (int b = 0; b <= a; ++b) row[b] -= va * qq[b] + qa * vv[b];
        }
        for (int t = 0; t < len; ++t) H[(size_t)k * n + k + 1 + t] = v[t];
        beta_out[k] = beta;
    }
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
    if (n >= 2) e[n - 2] = A[(size_t)(n - 1) * n + (n - 2)];
    e[n - 1] = 0.0;
}

// sqrt(a^2 + b^2): the plain formula wherever the sum of squares neither
// overflows nor underflows (within two units in the last place of the
// library's hypot, several times faster), else the library's scaled hypot.
inline double fast_hypot(double a, double b) {
    const double s = a * a + b * b;
    if (s > 1e-290 && s < 1e290) return sqrt(s);
    return hypot(a, b);
}

// Implicit QL on the tridiagonal (d, e); ZT, when given, accumulates the
// rotations, held transposed (row i of ZT is column i of the transform) so
// that each rotation updates two contiguous rows.  Returns 0 on success, -1
// if an eigenvalue fails to converge.
int tridiag_ql(double* d, double* e, int n, double* ZT) {
    const double eps = 2.220446049250313e-16;
    // An off-diagonal entry is negligible next to its diagonal neighbours or,
    // as in EISPACK's tql2, next to the matrix norm: without the latter a
    // cluster of (numerically) zero eigenvalues, whose entries are all
    // rounding noise, never deflates.
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i) tnorm = std::max(tnorm, fabs(d[i]) + fabs(e[i]));
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= eps * dd || fabs(e[m]) <= eps * tnorm) break;
            }
            if (m == l) break;
            if (++iter > 100) return -1;
            // shift from the eigenvalue of the leading 2 x 2 block closer to d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double rr = fast_hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? fabs(rr) : -fabs(rr)));
            double s = 1.0, c = 1.0, p = 0.0;
            bool early = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                rr = fast_hypot(f, g);
                e[i + 1] = rr;
                if (rr == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = true;
                    break;
                }
                const double ir = 1.0 / rr;
                s = f * ir;
                c = g * ir;
                g = d[i + 1] - p;
                rr = (d[i] - g) * s + 2.0 * c * b;
                p = s * rr;
                d[i + 1] = g + p;
                g = c * rr - b;
                if (!ZT) continue;
                double* __restrict__ zi = ZT + (size_t)i * n;
                double* __restrict__ zj = ZT + (size_t)(i + 1) * n;
                for (int k = 0; k < n; ++k) {
                    const double t = zj[k];
                    zj[k] = s * zi[k] + c * t;
                    zi[k] = c * zi[k] - s * t;
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return 0;
}

// Eigenvalues only of the tridiagonal (d, e): the same shifted QL sweeps as
// tridiag_ql, carried on the squares e_i^2 of the off-diagonal so that a
// sweep takes no square root (the root-free form of Pal, Walker and Kahan,
// as presented in Parlett, The Symmetric Eigenvalue Problem, 1980).  With
// c and s the squared cosine and sine of a rotation, a sweep from the
// bottom m of the unreduced block up to its top l carries gamma (the
// rotated diagonal entry less the shift) and p = gamma^2 / c; the shift is
// the eigenvalue of the leading 2 x 2 block nearer to d[l], as in
// tridiag_ql.  e is destroyed; d receives the eigenvalues (unsorted).
// Returns 0, or -1 if an eigenvalue fails to converge.
int tridiag_eigvals(double* d, double* e, int n) {
    const double eps = 2.220446049250313e-16, eps2 = eps * eps;
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i) tnorm = std::max(tnorm, fabs(d[i]) + fabs(e[i]));
    const double tn2 = eps2 * tnorm * tnorm;
    std::vector<double> e2(n);
    for (int i = 0; i < n; ++i) e2[i] = e[i] * e[i];
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            // negligible off-diagonal below the block (next to its diagonal
            // neighbours, or next to the matrix norm, as in tridiag_ql)
            int m = l;
            for (; m + 1 < n; ++m)
                if (e2[m] <= eps2 * fabs(d[m]) * fabs(d[m + 1]) || e2[m] <= tn2) break;
            if (m == l) break;
            if (++iter > 100) return -1;
            const double rte = sqrt(e2[l]);
            double g = (d[l + 1] - d[l]) / (2.0 * rte);
            const double rr = fast_hypot(g, 1.0);
            const double sigma = d[l] - rte / (g + (g >= 0.0 ? rr : -rr));
            double c = 1.0, sn = 0.0;
            double gamma = d[m] - sigma;
            double p = gamma * gamma;
            for (int i = m - 1; i >= l; --i) {
                const double bb = e2[i];
                const double r = p + bb;
                if (i != m - 1) e2[i + 1] = sn * r;
                const double oldc = c;
                c = p / r;
                sn = bb / r;
                const double oldgam = gamma;
                const double alpha = d[i];
                gamma = c * (alpha - sigma) - sn * oldgam;
                d[i + 1] = oldgam + (alpha - gamma);
                p = c != 0.0 ? (gamma * gamma) / c : oldc * bb;
            }
            e2[l] = sn * p;
            d[l] = sigma + gamma;
        }
    }
    return 0;
}

// One solve of (T - sigma I) x = b for the symmetric tridiagonal T = (d, e)
// by Gaussian elimination with partial pivoting (the factor has up to two
// superdiagonals); a zero pivot is replaced by `tiny`.  b is overwritten.
struct TridiagLU {
    std::vector<double> u0, u1, u2, l;
    std::vector<char> piv;
    void factor(const double* d, const double* e, int n, double sigma, double tiny) {
        u0.assign(n, 0.0); u1.assign(n, 0.0); u2.assign(n, 0.0); l.assign(n, 0.0); piv.assign(n, 0);
        double ad = d[0] - sigma, au = n > 1 ? e[0] : 0.0;  // the pending row: columns i, i + 1
        for (int i = 0; i + 1 < n; ++i) {
            const double cc = e[i], ad1 = d[i + 1] - sigma, au1 = (i + 2 < n) ? e[i + 1] : 0.0;
            if (fabs(cc) > fabs(ad)) {  // row i + 1 becomes the pivot row
                const double mult = ad / cc;
                u0[i] = cc; u1[i] = ad1; u2[i] = au1;
                l[i] = mult; piv[i] = 1;
                ad = au - mult * ad1;
                au = -mult * au1;
            } else {
                if (ad == 0.0) ad = tiny;
                const double mult = cc / ad;
                u0[i] = ad; u1[i] = au; u2[i] = 0.0;
                l[i] = mult; piv[i] = 0;
                ad = ad1 - mult * au;
                au = au1;
            }
        }
        u0[n - 1] = (ad == 0.0) ? tiny : ad;
    }
    void solve(double* b, int n) const {
        for (int i = 0; i + 1 < n; ++i) {
            if (piv[i]) {
                const double bi = b[i];
                b[i] = b[i + 1];
                b[i + 1] = bi - l[i] * b[i];
            } else {
                b[i + 1] -= l[i] * b[i];
            }
        }
        b[n - 1] /= u0[n - 1];
        if (n > 1) b[n - 2] = (b[n - 2] - u1[n - 2] * b[n - 1]) / u0[n - 2];
        for (int i = n - 3; i >= 0; --i) b[i] = (b[i] - u1[i] * b[i + 1] - u2[i] * b[i + 2]) / u0[i];
    }
};

double norm2(const double* x, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += x[i] * x[i];
    return sqrt(s);
}

}  // namespace

// AVX2 and baseline builds, as householder_tridiag_lower.
__attribute__((target_clones("avx2", "default"))) int sym_eig_top(double* A, int n, int k, double* evals,
                                                                 double* vecs) {
    if (n <= 0 || k < 0 || k > n) return -1;
    std::vector<double> A0(A, A + (size_t)n * n);  // for the fallback below
    // When the inverse iteration cannot deliver (a large cluster of zero
    // eigenvalues among the k leading ones, whose solves overflow), the full
    // solver runs instead; such a cluster's vectors are any basis of it.
    auto fallback = [&]() -> int {
        std::vector<double> all((size_t)n * n);
        if (sym_eig(A0.data(), n, evals, all.data()) != 0) return -1;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < k; ++j) vecs[(size_t)i * k + j] = all[(size_t)i * n + j];
        return 0;
    };
    std::vector<double> d(n), e(n), H((size_t)n * n, 0.0), beta(n, 0.0);
    householder_tridiag_lower(A, n, d.data(), e.data(), H.data(), beta.data());
    std::vector<double> dt(d), et(e);  // T, kept for the inverse iteration
    if (tridiag_eigvals(d.data(), e.data(), n) != 0) return -1;
    std::sort(d.begin(), d.end(), [](double a, double b) { return a > b; });
    for (int j = 0; j < n; ++j) evals[j] = d[j];
    if (k == 0) return 0;
    double tnorm = 0.0;  // max row sum of |T|
    for (int i = 0; i < n; ++i)
        tnorm = std::max(tnorm, fabs(dt[i]) + (i > 0 ? fabs(et[i - 1]) : 0.0) + (i + 1 < n ? fabs(et[i]) : 0.0));
    if (tnorm == 0.0) tnorm = 1.0;
    const double eps = 2.220446049250313e-16;
    const double ortol = 1e-3 * tnorm;  // eigenvalues this close form a cluster
    const double tiny = eps * tnorm;
    std::vector<double> X((size_t)k * n);  // eigenvectors of T, one per row
    TridiagLU lu;
    int cl0 = 0;  // first vector of the current cluster
    double sigma_prev = 0.0;
    uint64_t rng = 0x9E3779B97F4A7C15ull;
    for (int j = 0; j < k; ++j) {
        double sigma = d[j];
        if (j > 0 && d[j - 1] - d[j] > ortol) cl0 = j;
        // equal eigenvalues get slightly different shifts (then each solve
        // favours a different direction; the orthogonalisation does the rest)
        if (j > cl0 && sigma_prev - sigma < 10.0 * eps * std::max(fabs(sigma), tnorm))
            sigma = sigma_prev - 10.0 * eps * std::max(fabs(sigma), tnorm);
        sigma_prev = sigma;
        lu.factor(dt.data(), et.data(), n, sigma, tiny);
        double* x = X.data() + (size_t)j * n;
        for (int i = 0; i < n; ++i) {  // fixed pseudo-random start (xorshift)
            rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
            x[i] = (double)(rng >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        }
        for (int it = 0; it < 4; ++it) {
            lu.solve(x, n);
            for (int q = cl0; q < j; ++q) {  // modified Gram-Schmidt within the cluster
                const double* y = X.data() + (size_t)q * n;
                double s = 0.0;
                for (int i = 0; i < n; ++i) s += y[i] * x[i];
                for (int i = 0; i < n; ++i) x[i] -= s * y[i];
            }
            const double nr = norm2(x, n);
            if (!(nr > 0.0) || !isfinite(nr)) return fallback();
            for (int i = 0; i < n; ++i) x[i] /= nr;
        }
    }
    // back to the basis of A: y = H_0 H_1 ... H_{n-3} x for all k vectors at
    // once, reflector by reflector (each reflector read once, the k vectors
    // held as rows of Y [n][k] so that the k dot products and updates of a
    // row run along contiguous memory), then the sign fixed so that the
    // entry of largest magnitude is positive
    std::vector<double> Y((size_t)n * k), dots(k);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < k; ++j) Y[(size_t)i * k + j] = X[(size_t)j * n + i];
    for (int s = n - 3; s >= 0; --s) {
        if (beta[s] == 0.0) continue;
        const double* v = H.data() + (size_t)s * n;
        std::fill(dots.begin(), dots.end(), 0.0);
        for (int i = s + 1; i < n; ++i) {
            const double vi = v[i];
            const double* __restrict__ yi = Y.data() + (size_t)i * k;
            double* __restrict__ dt = dots.data();
            for (int j = 0; j < k; ++j) dt[j] += vi * yi[j];
        }
        for (int j = 0; j < k; ++j) dots[j] *= beta[s];
        for (int i = s + 1; i < n; ++i) {
            const double vi = v[i];
            double* __restrict__ yi = Y.data() + (size_t)i * k;
            const double* __restrict__ dt = dots.data();
            for (int j = 0; j < k; ++j) yi[j] -= dt[j] * vi;
        }
    }
    for (int j = 0; j < k; ++j) {
        int arg = 0;
        for (int i = 1; i < n; ++i)
            if (fabs(Y[(size_t)i * k + j]) > fabs(Y[(size_t)arg * k + j])) arg = i;
        const double sg = Y[(size_t)arg * k + j] < 0.0 ? -1.0 : 1.0;
        for (int i = 0; i < n; ++i) vecs[(size_t)i * k + j] = sg * Y[(size_t)i * k + j];
    }
    return 0;
}

int sym_eig(double* A, int n, double* evals, double* vecs) {
    if (n <= 0) return -1;
    std::vector<double> d(n), e(n), Q((size_t)n * n);
    householder_tridiag(A, n, d.data(), e.data(), Q.data());
    std::vector<double> QT((size_t)n * n);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) QT[(size_t)c * n + r] = Q[(size_t)r * n + c];
    if (tridiag_ql(d.data(), e.data(), n, QT.data()) != 0) return -1;
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] > d[b]; });
    for (int j = 0; j < n; ++j) {
        const int col = idx[j];
        evals[j] = d[col];
        // sign convention: the entry of largest magnitude is positive
        const double* q = QT.data() + (size_t)col * n;  // eigenvector `col`, contiguous
        int arg = 0;
        for (int rI = 1; rI < n; ++rI)
            if (fabs(q[rI]) > fabs(q[arg])) arg = rI;
        const double sg = q[arg] < 0.0 ? -1.0 : 1.0;
        for (int rI = 0; rI < n; ++rI) vecs[(size_t)rI * n + j] = sg * q[rI];
    }
    return 0;
}

}  // namespace qfca

extern "C" int qfca_host_sym_eig(double* A, int32_t n, double* evals, double* vecs) {
    return qfca::sym_eig(A, n, evals, vecs);
}

extern "C" int qfca_host_sym_eig_top(double* A, int32_t n, int32_t k, double* evals, double* vecs) {
    return qfca::sym_eig_top(A, n, k, evals, vecs);
}
