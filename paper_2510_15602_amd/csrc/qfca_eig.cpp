// Host FP64 symmetric eigensolver for the C x C feature covariance of the PCA
// step (Sec. 3.3).  The problem is tiny next to the feature map (C <= 2048),
// so it runs on the host: Householder reduction to tridiagonal form, then the
// implicit QL iteration with shifts (Bowdler, Martin, Reinsch and Wilkinson,
// 1968) applied to the accumulated orthogonal transform.
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

namespace {

// Reduce symmetric A (n x n, row-major, destroyed) to tridiagonal T = Q^T A Q.
// d[i] = T[i][i], e[i] = T[i][i+1] (e[n-1] = 0), Q row-major.
void householder_tridiag(double* A, int n, double* d, double* e, double* Q) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Q[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
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

// Implicit QL on the tridiagonal (d, e); ZT accumulates the rotations, held
// transposed (row i of ZT is column i of the transform) so that each
// rotation updates two contiguous rows.  Returns 0 on success, -1 if an
// eigenvalue fails to converge.
int tridiag_ql(double* d, double* e, int n, double* ZT) {
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++iter > 100) return -1;
            // shift from the eigenvalue of the leading 2 x 2 block closer to d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double rr = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? fabs(rr) : -fabs(rr)));
            double s = 1.0, c = 1.0, p = 0.0;
            bool early = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                rr = hypot(f, g);
                e[i + 1] = rr;
                if (rr == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = true;
                    break;
                }
                s = f / rr;
                c = g / rr;
                g = d[i + 1] - p;
                rr = (d[i] - g) * s + 2.0 * c * b;
                p = s * rr;
                d[i + 1] = g + p;
                g = c * rr - b;
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

}  // namespace

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
