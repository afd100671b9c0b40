/*
 * qfca_oracle.c -- slow, plain FP64 CPU oracle for the QFCA score-map path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * It follows "Quantized FCA: Efficient Zero-Shot Texture Anomaly Detection"
 * (Ardelean, Rueckbeil, Weyrich) step by step, with no blocking, running sums
 * or reordering:
 *   - PCA residual preprocessing, F = W - PCA^-1(PCA(W))        (Sec. 3.3)
 *   - per-channel quantisation into N equally spaced values      (Sec. 3.1)
 *   - a T x T window histogram per pixel, counted directly       (Sec. 3.1)
 *   - the per-bin patch mismatch of Alg. 1, written as the monotone coupling
 *     of the two cumulative histograms it walks                  (Alg. 1, proof)
 *   - error-to-pixel association: box mean (sigma_p = infinity) or Gaussian
 *     weights over a patch-sized kernel (finite sigma_p)          (Eq. 2, Sec. 3.1, Sec. 4.5.4)
 *   - channel mean and the final Gaussian blur sigma_s           (Eq. 1, Sec. 4.5.4)
 *   - the four reference choices: median -> quan (the default), mean -> quan,
 *     quan -> median, quan -> mean                               (Sec. 3.2, Sec. 4.5.3, Tab. 3)
 * and, beside the method itself:
 *   - histograms of the k principal coordinates scored by the window
 *     1-Wasserstein distance, box smoothed                        (Sec. 3.3, Sec. 3.1)
 *   - FCA's sort-based comparison of real values, the method QFCA quantises
 *                                                                 (Sec. 3.1, proof)
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - windows are clipped at the image border; patch and reference histograms
 *     are brought to equal mass by scaling P by the reference mass and R by n_p;
 *   - quantisation range is [q_lo, q_hi] type-7 quantiles of each channel,
 *     edges rounded to float32 and a value equal to an edge goes to the upper bin;
 *   - medians over an even number of windows are lower medians;
 *   - references use every full (unclipped) window;
 *   - the association averages over the in-image windows that contain a pixel
 *     (with finite sigma_p, weighted and renormalised over those windows);
 *   - errors are in feature units (bin distance times the channel's bin width);
 *   - channels are averaged; the final blur has radius ceil(3 sigma_s) and is
 *     renormalised over in-image taps;
 *   - FCA orders equal values by raster position inside the window.
 *
 * Parity pins for every function live in tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* PCA (Sec. 3.3): mean, covariance, cyclic Jacobi eigen-decomposition.      */

/* Cyclic Jacobi on a symmetric n x n matrix A (row-major, destroyed).
 * On return evals[i] holds the eigenvalues and V (row-major, V[r*n+i]) the
 * eigenvectors as columns, unsorted.  Returns the number of sweeps. */
static int jacobi_eig(double* A, int n, double* evals, double* V) {
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) V[i * n + j] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int i = 0; i < n * n; i++) fro += A[i] * A[i];
    fro = sqrt(fro);
    int sweep = 0;
    for (sweep = 0; sweep < 100; sweep++) {
        double off = 0.0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) off += A[p * n + q] * A[p * n + q];
        if (sqrt(2.0 * off) <= 1e-15 * fro || off == 0.0) break;
        for (int p = 0; p < n; p++) {
            for (int q = p + 1; q < n; q++) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                double app = A[p * n + p], aqq = A[q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with J the rotation in the (p, q) plane. */
                for (int k = 0; k < n; k++) {
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; k++) {
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; k++) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int i = 0; i < n; i++) evals[i] = A[i * n + i];
    return sweep;
}

/* X: [C][N] float32 features (N = H*W pixels).  Outputs:
 *   mu[C]; V[C*k] (row-major [C][k]: column j is the j-th principal axis);
 *   evals[C] all eigenvalues of the 1/N covariance, descending.
 * Eigenvector signs are fixed so the entry of largest magnitude is positive.
 * Returns the Jacobi sweep count, or -1 on bad arguments. */
int orc_pca(const float* X, int C, long N, int k, double* mu, double* V, double* evals) {
    if (C <= 0 || N <= 0 || k < 0 || k > C) return -1;
    for (int c = 0; c < C; c++) {
        double s = 0.0;
        for (long i = 0; i < N; i++) s += (double)X[(long)c * N + i];
        mu[c] = s / (double)N;
    }
    double* S = (double*)calloc((size_t)C * C, sizeof(double));
    double* E = (double*)malloc((size_t)C * C * sizeof(double));
    double* ev = (double*)malloc((size_t)C * sizeof(double));
    #pragma omp parallel for schedule(dynamic)
    for (int a = 0; a < C; a++) {
        for (int b = a; b < C; b++) {
            double s = 0.0;
            for (long i = 0; i < N; i++)
                s += ((double)X[(long)a * N + i] - mu[a]) * ((double)X[(long)b * N + i] - mu[b]);
            S[a * C + b] = S[b * C + a] = s / (double)N;
        }
    }
    int sweeps = jacobi_eig(S, C, ev, E);
    /* sort descending (selection sort on indices; C is small) */
    int* idx = (int*)malloc((size_t)C * sizeof(int));
    for (int i = 0; i < C; i++) idx[i] = i;
    for (int i = 0; i < C; i++) {
        int best = i;
        for (int j = i + 1; j < C; j++)
            if (ev[idx[j]] > ev[idx[best]]) best = j;
        int t = idx[i]; idx[i] = idx[best]; idx[best] = t;
    }
    for (int i = 0; i < C; i++) evals[i] = ev[idx[i]];
    for (int j = 0; j < k; j++) {
        int col = idx[j];
        int arg = 0;
        for (int r = 1; r < C; r++)
            if (fabs(E[r * C + col]) > fabs(E[arg * C + col])) arg = r;
        double sg = E[arg * C + col] < 0 ? -1.0 : 1.0;
        for (int r = 0; r < C; r++) V[r * k + j] = sg * E[r * C + col];
    }
    free(idx); free(ev); free(E); free(S);
    return sweeps;
}

/* r(x) = (x - mu) - V V^T (x - mu) for every pixel; R is [C][N] double.
 * With preproc == 0 (plain QFCA) r = x unchanged. */
void orc_residual(const float* X, int C, long N, const double* mu, const double* V, int k,
                  int preproc, double* R) {
    if (!preproc) {
        for (long i = 0; i < (long)C * N; i++) R[i] = (double)X[i];
        return;
    }
    #pragma omp parallel
    {
        double* d = (double*)malloc((size_t)C * sizeof(double));
        double* z = (double*)malloc((size_t)(k > 0 ? k : 1) * sizeof(double));
        #pragma omp for schedule(static)
        for (long i = 0; i < N; i++) {
            for (int c = 0; c < C; c++) d[c] = (double)X[(long)c * N + i] - mu[c];
            for (int j = 0; j < k; j++) {
                double s = 0.0;
                for (int c = 0; c < C; c++) s += V[c * k + j] * d[c];
                z[j] = s;
            }
            for (int c = 0; c < C; c++) {
                double s = 0.0;
                for (int j = 0; j < k; j++) s += V[c * k + j] * z[j];
                R[(long)c * N + i] = d[c] - s;
            }
        }
        free(z); free(d);
    }
}

/* ------------------------------------------------------------------------ */
/* Quantisation (Sec. 3.1).                                                  */

/* Type-7 (linear interpolation) quantile of n values; v is not modified. */
double orc_quantile(const double* v, long n, double q) {
    double* s = (double*)malloc((size_t)n * sizeof(double));
    memcpy(s, v, (size_t)n * sizeof(double));
    qsort(s, (size_t)n, sizeof(double), cmp_double);
    double h = (double)(n - 1) * q;
    long lo = (long)floor(h);
    double out = s[lo];
    if (lo + 1 < n) out = s[lo] + (h - (double)lo) * (s[lo + 1] - s[lo]);
    free(s);
    return out;
}

/* Per channel: lo = quantile(q_lo), hi = quantile(q_hi), delta = (hi-lo)/B and
 * the B-1 inner edges lo + m*delta (m = 1..B-1) rounded to float32.  A channel
 * with hi <= lo is degenerate: delta = 0 and every edge is +inf (all bin 0). */
void orc_edges(const double* R, int C, long N, int B, double qlo, double qhi,
               double* lo, double* hi, double* delta, float* edges) {
    #pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < C; c++) {
        double l = orc_quantile(R + (long)c * N, N, qlo);
        double h = orc_quantile(R + (long)c * N, N, qhi);
        lo[c] = l; hi[c] = h;
        if (!(h > l)) {
            delta[c] = 0.0;
            for (int m = 1; m < B; m++) edges[(long)c * (B - 1) + (m - 1)] = INFINITY;
        } else {
            double d = (h - l) / (double)B;
            delta[c] = d;
            for (int m = 1; m < B; m++) edges[(long)c * (B - 1) + (m - 1)] = (float)(l + (double)m * d);
        }
    }
}

/* bin = #{m : r >= e_m}, compared in double precision against the stored
 * float32 edges. */
void orc_quantize(const double* R, int C, long N, int B, const float* edges, uint8_t* bins) {
    #pragma omp parallel for schedule(static)
    for (int c = 0; c < C; c++) {
        const float* e = edges + (long)c * (B - 1);
        for (long i = 0; i < N; i++) {
            double r = R[(long)c * N + i];
            int b = 0;
            for (int m = 0; m < B - 1; m++)
                if (r >= (double)e[m]) b++;
            bins[(long)c * N + i] = (uint8_t)b;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Per-bin patch mismatch (Sec. 3.1, Alg. 1; supplementary proof).           */

/* P, R: nonnegative bin weights of the patch and the reference with equal
 * total mass, N bins, Q_i = i (bin units).  The optimal 1-D transport between
 * them is the monotone (rank) coupling: the patch bin i occupies the mass
 * interval (cP_{i-1}, cP_i] of the cumulative weights, the reference bin j
 * occupies (cR_{j-1}, cR_j], and the mass moved from i to j is the length of
 * the intersection of the two intervals.  The numerator of bin i is
 *   I_i = sum_j |i - j| |(cP_{i-1}, cP_i] n (cR_{j-1}, cR_j]|
 * and its mismatch E_i = I_i / P_i (0 where P_i = 0): the bin's share of the
 * Wasserstein distance averaged over the mass of the bin, which is what the
 * two-pointer walk of Alg. 1 accumulates.  I (may be NULL) receives the
 * numerators.  Returns the number of (i, j) pairs that carry mass (at most
 * 2N - 1, the length of a monotone staircase). */
int orc_bin_mismatch(const double* P, const double* R, int N, double* E, double* I) {
    double* cP = (double*)malloc((size_t)N * sizeof(double));
    double* cR = (double*)malloc((size_t)N * sizeof(double));
    double a = 0.0, b = 0.0;
    for (int i = 0; i < N; i++) {
        a += P[i];
        b += R[i];
        cP[i] = a;
        cR[i] = b;
    }
    int cells = 0;
    for (int i = 0; i < N; i++) {
        double lo = i > 0 ? cP[i - 1] : 0.0, hi = cP[i];
        double s = 0.0;
        if (hi > lo) {
            /* first reference bin whose interval ends above lo */
            int j0 = 0, j1 = N - 1;
            while (j0 < j1) {
                int mid = (j0 + j1) / 2;
                if (cR[mid] > lo) j1 = mid; else j0 = mid + 1;
            }
            for (int j = j0; j < N; j++) {
                double rl = j > 0 ? cR[j - 1] : 0.0;
                if (rl >= hi) break;
                double ov = fmin(hi, cR[j]) - fmax(lo, rl);
                if (ov > 0.0) {
                    s += (double)(i > j ? i - j : j - i) * ov;
                    cells++;
                }
            }
        }
        if (I) I[i] = s;
        E[i] = P[i] > 0.0 ? s / P[i] : 0.0;
    }
    free(cR);
    free(cP);
    return cells;
}

/* ------------------------------------------------------------------------ */
/* Reference (Sec. 3.2, Sec. 4.5.3 and Tab. 3).                               */

static int cmp_double_q(const void* a, const void* b) { return cmp_double(a, b); }

/* Every full T x T window of channel plane Rc, sorted: out [nw][T*T], windows
 * in raster order of their top-left corner.  Returns nw. */
static long sorted_windows(const double* Rc, int H, int W, int T, double* out) {
    int n = T * T;
    long w = 0;
    for (int py = 0; py + T <= H; py++)
        for (int px = 0; px + T <= W; px++, w++) {
            double* s = out + w * n;
            int t = 0;
            for (int dy = 0; dy < T; dy++)
                for (int dx = 0; dx < T; dx++) s[t++] = Rc[(long)(py + dy) * W + px + dx];
            qsort(s, (size_t)n, sizeof(double), cmp_double_q);
        }
    return w;
}

/* Full-precision reference vectors (Sec. 3.2): for every channel and every
 * rank rho of the sorted full windows, the lower median (kind 0: the
 * ceil(nw/2)-th smallest over the nw windows) or the mean (kind 1) of the
 * rank-rho values.  Y: [C][T*T], nondecreasing in rho. */
void orc_reference_values(const double* R, int C, int H, int W, int T, int kind, double* Y) {
    int n = T * T;
    long nw = (long)(H - T + 1) * (W - T + 1);
    long h = (nw + 1) / 2;
    #pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < C; c++) {
        double* sorted = (double*)malloc((size_t)nw * n * sizeof(double));
        double* col = (double*)malloc((size_t)nw * sizeof(double));
        sorted_windows(R + (long)c * H * W, H, W, T, sorted);
        for (int rho = 0; rho < n; rho++) {
            for (long q = 0; q < nw; q++) col[q] = sorted[q * n + rho];
            if (kind == 0) {
                qsort(col, (size_t)nw, sizeof(double), cmp_double_q);
                Y[(long)c * n + rho] = col[h - 1];
            } else {
                double s = 0.0;
                for (long q = 0; q < nw; q++) s += col[q];
                Y[(long)c * n + rho] = s / (double)nw;
            }
        }
        free(col);
        free(sorted);
    }
}

/* "median -> quan" (kind 0, the default) and "mean -> quan" (kind 1):
 * the full-precision reference vector of orc_reference_values, quantised with
 * the channel's edges.  cR[C][B]: cumulative reference histogram
 * (cR[B-1] = T*T). */
void orc_reference_literal(const double* R, int C, int H, int W, int T, int B,
                           const float* edges, int kind, int* cR) {
    int n = T * T;
    double* Y = (double*)malloc((size_t)C * n * sizeof(double));
    orc_reference_values(R, C, H, W, T, kind, Y);
    for (int c = 0; c < C; c++) {
        int* hist = (int*)calloc((size_t)B, sizeof(int));
        const float* e = edges + (long)c * (B - 1);
        for (int rho = 0; rho < n; rho++) {
            double ref = Y[(long)c * n + rho];
            int b = 0;
            for (int m = 0; m < B - 1; m++)
                if (ref >= (double)e[m]) b++;
            hist[b]++;
        }
        int acc = 0;
        for (int i = 0; i < B; i++) { acc += hist[i]; cR[(long)c * B + i] = acc; }
        free(hist);
    }
    free(Y);
}

/* Histogram of the window of side T centred at (py, px), clipped to the
 * image: P[B] counts; returns the number of pixels n_p. */
static long window_hist(const uint8_t* bc, int H, int W, int T, int B, int py, int px, long* P) {
    int r = T / 2;
    long np = 0;
    for (int i = 0; i < B; i++) P[i] = 0;
    for (int y = py - r; y <= py + r; y++) {
        if (y < 0 || y >= H) continue;
        for (int x = px - r; x <= px + r; x++) {
            if (x < 0 || x >= W) continue;
            P[bc[(long)y * W + x]]++;
            np++;
        }
    }
    return np;
}

/* The median -> quan reference from the bins alone: cR(i) is the
 * ceil(nw/2)-th largest of the full-window cumulative counts cP_p(i).  This
 * follows because quantisation is monotone and commutes with order
 * statistics (a derivation, pinned against orc_reference_literal). */
void orc_reference_cdf(const uint8_t* bins, int C, int H, int W, int T, int B, int* cR) {
    int n = T * T, r = T / 2;
    long nw = (long)(H - T + 1) * (W - T + 1);
    long h = (nw + 1) / 2;
    #pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < C; c++) {
        const uint8_t* bc = bins + (long)c * H * W;
        long* cnt = (long*)calloc((size_t)B * (n + 1), sizeof(long));
        long* P = (long*)malloc((size_t)B * sizeof(long));
        for (int py = r; py + r < H; py++)
            for (int px = r; px + r < W; px++) {
                window_hist(bc, H, W, T, B, py, px, P);
                long acc = 0;
                for (int i = 0; i < B; i++) { acc += P[i]; cnt[(long)i * (n + 1) + acc]++; }
            }
        for (int i = 0; i < B; i++) {
            long seen = 0;
            int v = n;
            for (v = n; v >= 0; v--) {
                seen += cnt[(long)i * (n + 1) + v];
                if (seen >= h) break;
            }
            cR[(long)c * B + i] = v;
        }
        free(P); free(cnt);
    }
}

/* References taken after the quantisation, bin by bin over the full-window
 * histograms P_p (Tab. 3): "quan -> median" (kind 0) takes for every bin i
 * the lower median over windows of P_p(i) (the ceil(nw/2)-th smallest; the
 * medians need not add up to T*T, so the reference mass is their sum);
 * "quan -> mean" (kind 1) takes the mean of P_p(i) (mass T*T, fractional
 * counts).  cR[C][B]: cumulative reference weights (double). */
void orc_reference_hist(const uint8_t* bins, int C, int H, int W, int T, int B, int kind, double* cR) {
    int n = T * T, r = T / 2;
    long nw = (long)(H - T + 1) * (W - T + 1);
    long h = (nw + 1) / 2;
    #pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < C; c++) {
        const uint8_t* bc = bins + (long)c * H * W;
        long* cnt = (long*)calloc((size_t)B * (n + 1), sizeof(long));  /* [bin][count value] */
        long* P = (long*)malloc((size_t)B * sizeof(long));
        for (int py = r; py + r < H; py++)
            for (int px = r; px + r < W; px++) {
                window_hist(bc, H, W, T, B, py, px, P);
                for (int i = 0; i < B; i++) cnt[(long)i * (n + 1) + P[i]]++;
            }
        double acc = 0.0;
        for (int i = 0; i < B; i++) {
            double v = 0.0;
            if (kind == 0) {
                long seen = 0;
                int t;
                for (t = 0; t <= n; t++) {
                    seen += cnt[(long)i * (n + 1) + t];
                    if (seen >= h) break;
                }
                v = (double)t;
            } else {
                double s = 0.0;
                for (int t = 0; t <= n; t++) s += (double)t * (double)cnt[(long)i * (n + 1) + t];
                v = s / (double)nw;
            }
            acc += v;
            cR[(long)c * B + i] = acc;
        }
        free(P); free(cnt);
    }
}

/* ------------------------------------------------------------------------ */
/* Patch statistics comparison and association for one channel.             */

/* Per-bin mismatch of the window centred at (py, px) against a reference
 * given by its cumulative weights cR_c[B] (total M_R = cR_c[B-1], any
 * nonnegative reals).  The patch histogram P (mass n_p) and the reference R
 * (mass M_R) are brought to equal mass as P~ = P M_R and R~ = R n_p.
 * e_out[B]: E_i of orc_bin_mismatch (bin units); I_out [B] (may be NULL):
 * the numerators I_i (in units of the scaled masses); Pt_out [B] (may be
 * NULL): P~.  Returns the number of transport cells. */
int orc_window_errors(const uint8_t* bc, int H, int W, int T, int B, const double* cR_c,
                      int py, int px, double* e_out, double* I_out, double* Pt_out) {
    long* P = (long*)malloc((size_t)B * sizeof(long));
    double* Pt = (double*)malloc((size_t)B * sizeof(double));
    double* Rt = (double*)malloc((size_t)B * sizeof(double));
    long np = window_hist(bc, H, W, T, B, py, px, P);
    double MR = cR_c[B - 1];
    for (int i = 0; i < B; i++) {
        double Ri = cR_c[i] - (i > 0 ? cR_c[i - 1] : 0.0);
        Pt[i] = (double)P[i] * MR;
        Rt[i] = Ri * (double)np;
    }
    int cells = orc_bin_mismatch(Pt, Rt, B, e_out, I_out);
    if (Pt_out) memcpy(Pt_out, Pt, (size_t)B * sizeof(double));
    free(Rt); free(Pt); free(P);
    return cells;
}

/* Spatial weight of a window whose centre is (dy, dx) away from the pixel
 * (Eq. 2's G_sigma_p over a kernel the size of the patch, Sec. 3.1 and
 * Sec. 4.5.4): 1 for sigma_p = infinity (box), else exp(-(dx^2 + dy^2) /
 * (2 sigma_p^2)). */
static double assoc_weight(int dy, int dx, double sigma_p) {
    if (isinf(sigma_p)) return 1.0;
    return exp(-(double)(dx * dx + dy * dy) / (2.0 * sigma_p * sigma_p));
}

/* bins_c: [H][W]; cR_c: cumulative reference weights [B] (see
 * orc_window_errors).  Ac[H][W] (bin units): the sigma_p-weighted mean, over
 * the windows p containing x, of e_p(b(x)) (the error of the pixel's own bin
 * in that window).  W1c[H][W] (bin units, may be NULL): window
 * 1-Wasserstein distance sum_k |cP~_k - cR~_k| / (n_p M_R).  Returns the
 * largest number of transport cells met. */
int orc_channel_map(const uint8_t* bc, int H, int W, int T, int B, const double* cR_c,
                    double sigma_p, double* Ac, double* W1c) {
    int r = T / 2;
    double* e = (double*)malloc((size_t)H * W * B * sizeof(double));
    double* Pt = (double*)malloc((size_t)B * sizeof(double));
    long* P = (long*)malloc((size_t)B * sizeof(long));
    int maxcells = 0;
    double MR = cR_c[B - 1];
    for (int py = 0; py < H; py++) {
        for (int px = 0; px < W; px++) {
            double* ep = e + ((long)py * W + px) * B;
            int cells = orc_window_errors(bc, H, W, T, B, cR_c, py, px, ep, NULL, Pt);
            if (cells > maxcells) maxcells = cells;
            if (W1c) {
                long np = window_hist(bc, H, W, T, B, py, px, P);
                double a = 0.0, s = 0.0;
                for (int k = 0; k < B; k++) {
                    a += Pt[k];
                    s += fabs(a - cR_c[k] * (double)np);
                }
                W1c[(long)py * W + px] = MR > 0.0 ? s / ((double)np * MR) : 0.0;
            }
        }
    }
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            int b = bc[(long)y * W + x];
            double s = 0.0, wsum = 0.0;
            for (int py = y - r; py <= y + r; py++) {
                if (py < 0 || py >= H) continue;
                for (int px = x - r; px <= x + r; px++) {
                    if (px < 0 || px >= W) continue;
                    double w = assoc_weight(py - y, px - x, sigma_p);
                    s += w * e[((long)py * W + px) * B + b];
                    wsum += w;
                }
            }
            Ac[(long)y * W + x] = s / wsum;
        }
    }
    free(P); free(Pt); free(e);
    return maxcells;
}

/* Final low-pass (Sec. 4.5.4): direct 2-D Gaussian convolution, radius
 * ceil(3 sigma), weights exp(-(dx^2+dy^2)/(2 sigma^2)) renormalised over the
 * in-image taps.  sigma <= 0 copies. */
void orc_blur(const double* A, int H, int W, double sigma, double* out) {
    if (!(sigma > 0.0)) {
        memcpy(out, A, (size_t)H * W * sizeof(double));
        return;
    }
    int R = (int)ceil(3.0 * sigma);
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            double s = 0.0, wsum = 0.0;
            for (int dy = -R; dy <= R; dy++) {
                int yy = y + dy;
                if (yy < 0 || yy >= H) continue;
                for (int dx = -R; dx <= R; dx++) {
                    int xx = x + dx;
                    if (xx < 0 || xx >= W) continue;
                    double w = exp(-(double)(dx * dx + dy * dy) / (2.0 * sigma * sigma));
                    s += w * A[(long)yy * W + xx];
                    wsum += w;
                }
            }
            out[(long)y * W + x] = s / wsum;
        }
    }
}

/* Full score: A(x) = (1/C) sum_c delta_c Ac_c(x); score = blur(A).
 * cR: [C][B] cumulative reference weights.  Achan (may be NULL) receives the
 * per-channel maps delta_c Ac_c [C][H][W]; W1 (may be NULL) the channel mean
 * of delta_c W1c_c.  Returns the largest number of transport cells met. */
int orc_score(const uint8_t* bins, int C, int H, int W, int T, int B, const double* cR,
              const double* delta, double sigma_p, double sigma_s, double* A, double* score,
              double* W1, double* Achan) {
    long N = (long)H * W;
    double* Aall = (double*)malloc((size_t)C * N * sizeof(double));
    double* Wall = W1 ? (double*)malloc((size_t)C * N * sizeof(double)) : NULL;
    int maxcells = 0;
    #pragma omp parallel for schedule(dynamic) reduction(max : maxcells)
    for (int c = 0; c < C; c++) {
        int s = orc_channel_map(bins + (long)c * N, H, W, T, B, cR + (long)c * B, sigma_p,
                                Aall + (long)c * N, Wall ? Wall + (long)c * N : NULL);
        if (s > maxcells) maxcells = s;
    }
    for (long i = 0; i < N; i++) {
        double s = 0.0, w = 0.0;
        for (int c = 0; c < C; c++) {
            s += delta[c] * Aall[(long)c * N + i];
            if (Wall) w += delta[c] * Wall[(long)c * N + i];
        }
        A[i] = s / (double)C;
        if (W1) W1[i] = w / (double)C;
    }
    if (Achan)
        for (int c = 0; c < C; c++)
            for (long i = 0; i < N; i++) Achan[(long)c * N + i] = delta[c] * Aall[(long)c * N + i];
    orc_blur(A, H, W, sigma_s, score);
    free(Aall);
    if (Wall) free(Wall);
    return maxcells;
}

/* A(x) at a list of pixels only, each from its definition (for sampled checks
 * on maps too large for orc_score).  Achan_out may be NULL or [npix][C]. */
void orc_amap_pixels(const uint8_t* bins, int C, int H, int W, int T, int B, const double* cR,
                     const double* delta, double sigma_p, int npix, const int* ys, const int* xs,
                     double* A_out, double* Achan_out) {
    int r = T / 2;
    long N = (long)H * W;
    #pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < npix; t++) {
        int y = ys[t], x = xs[t];
        double* E = (double*)malloc((size_t)B * sizeof(double));
        double acc = 0.0;
        for (int c = 0; c < C; c++) {
            const uint8_t* bc = bins + (long)c * N;
            int b = bc[(long)y * W + x];
            double s = 0.0, wsum = 0.0;
            for (int py = y - r; py <= y + r; py++) {
                if (py < 0 || py >= H) continue;
                for (int px = x - r; px <= x + r; px++) {
                    if (px < 0 || px >= W) continue;
                    orc_window_errors(bc, H, W, T, B, cR + (long)c * B, py, px, E, NULL, NULL);
                    double w = assoc_weight(py - y, px - x, sigma_p);
                    s += w * E[b];
                    wsum += w;
                }
            }
            double v = delta[c] * s / wsum;
            if (Achan_out) Achan_out[(long)t * C + c] = v;
            acc += v;
        }
        A_out[t] = acc / (double)C;
        free(E);
    }
}

/* ------------------------------------------------------------------------ */
/* Histograms of the k principal coordinates scored by the window            */
/* 1-Wasserstein distance (the reading of the problem in which the PCA       */
/* projection itself is histogrammed, Sec. 3.3 "PCA(W)").                    */

/* z_j(x) = sum_c V[c][j] (x_c - mu_c): the k principal coordinates of every
 * pixel, Z [k][N] double. */
void orc_project(const float* X, int C, long N, const double* mu, const double* V, int k, double* Z) {
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < N; i++) {
        for (int j = 0; j < k; j++) {
            double s = 0.0;
            for (int c = 0; c < C; c++) s += V[c * k + j] * ((double)X[(long)c * N + i] - mu[c]);
            Z[(long)j * N + i] = s;
        }
    }
}

/* bins [K][H][W] (one plane per coordinate), cR [K][B] integer cumulative
 * references (mass T*T), delta [K].  For every window p the window W1
 * distance of coordinate j, W1_j(p) = delta_j sum_k |cP~_k - cR~_k| /
 * (n_p T^2) with the equal-mass scaling of orc_window_errors; the map is its
 * mean over the windows that contain the pixel (box smoothing) averaged over
 * the K coordinates, then blurred with sigma_s.  A and score: [H][W]. */
void orc_w1_score(const uint8_t* bins, int K, int H, int W, int T, int B, const int* cR,
                  const double* delta, double sigma_s, double* A, double* score) {
    long N = (long)H * W;
    int r = T / 2;
    double nR = (double)T * T;
    double* Aall = (double*)calloc((size_t)K * N, sizeof(double));
    #pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < K; j++) {
        const uint8_t* bc = bins + (long)j * N;
        double* w1 = (double*)malloc((size_t)N * sizeof(double));
        long* P = (long*)malloc((size_t)B * sizeof(long));
        for (int py = 0; py < H; py++)
            for (int px = 0; px < W; px++) {
                long np = window_hist(bc, H, W, T, B, py, px, P);
                double a = 0.0, s = 0.0;
                for (int b = 0; b < B; b++) {
                    a += (double)P[b] * nR;
                    s += fabs(a - (double)cR[(long)j * B + b] * (double)np);
                }
                w1[(long)py * W + px] = delta[j] * s / ((double)np * nR);
            }
        for (int y = 0; y < H; y++)
            for (int x = 0; x < W; x++) {
                double s = 0.0;
                long cnt = 0;
                for (int py = y - r; py <= y + r; py++) {
                    if (py < 0 || py >= H) continue;
                    for (int px = x - r; px <= x + r; px++) {
                        if (px < 0 || px >= W) continue;
                        s += w1[(long)py * W + px];
                        cnt++;
                    }
                }
                Aall[(long)j * N + (long)y * W + x] = s / (double)cnt;
            }
        free(P);
        free(w1);
    }
    for (long i = 0; i < N; i++) {
        double s = 0.0;
        for (int j = 0; j < K; j++) s += Aall[(long)j * N + i];
        A[i] = s / (double)K;
    }
    orc_blur(A, H, W, sigma_s, score);
    free(Aall);
}

/* ------------------------------------------------------------------------ */
/* FCA's sort-based comparison (Sec. 3.1, the method QFCA quantises).        */

/* Per-element mismatch of the window centred at (py, px) of channel plane
 * Rc against the sorted full-precision reference Y[T*T]: the window's n_p
 * values are sorted (equal values ordered by their raster position in the
 * window), the element of rank rho gets |x - Y_rho| when n_p = T*T; for a
 * window clipped at the border the masses are equalised as for the
 * histograms (each window element carries T*T, each reference element n_p)
 * and an element's error is the mass-weighted mean of |x - Y_k| over the
 * reference elements its mass is matched to in rank order.  err[n_p]: the
 * errors in raster order of the window's pixels.  Returns n_p. */
int orc_fca_window(const double* Rc, int H, int W, int T, const double* Y, int py, int px, double* err) {
    int r = T / 2, n = T * T;
    int np = 0;
    double vals[63 * 63];
    int order[63 * 63];
    for (int y = py - r; y <= py + r; y++) {
        if (y < 0 || y >= H) continue;
        for (int x = px - r; x <= px + r; x++) {
            if (x < 0 || x >= W) continue;
            vals[np] = Rc[(long)y * W + x];
            order[np] = np;
            np++;
        }
    }
    /* insertion sort of the indices by (value, raster position) */
    for (int i = 1; i < np; i++) {
        int t = order[i];
        int j = i - 1;
        while (j >= 0 && vals[order[j]] > vals[t]) {
            order[j + 1] = order[j];
            j--;
        }
        order[j + 1] = t;
    }
    for (int rho = 0; rho < np; rho++) {
        int idx = order[rho];
        double x = vals[idx];
        double e = 0.0;
        if (np == n) {
            e = fabs(x - Y[rho]);
        } else {
            /* element mass interval (rho n, (rho + 1) n]; reference element k
             * holds (k np, (k + 1) np] */
            double lo = (double)rho * n, hi = lo + (double)n;
            for (int k = 0; k < n; k++) {
                double rl = (double)k * np, rh = rl + (double)np;
                double ov = fmin(hi, rh) - fmax(lo, rl);
                if (ov > 0.0) e += ov * fabs(x - Y[k]);
            }
            e /= (double)n;
        }
        err[idx] = e;
    }
    return np;
}

/* FCA map of one channel: A_c(x) = mean over the windows p containing x of
 * the error of x's element in window p (sigma_p = infinity). */
static void fca_channel(const double* Rc, int H, int W, int T, const double* Y, double* Ac) {
    int r = T / 2;
    double err[63 * 63];
    for (long i = 0; i < (long)H * W; i++) Ac[i] = 0.0;
    int* cnt = (int*)calloc((size_t)H * W, sizeof(int));
    for (int py = 0; py < H; py++)
        for (int px = 0; px < W; px++) {
            orc_fca_window(Rc, H, W, T, Y, py, px, err);
            int t = 0;
            for (int y = py - r; y <= py + r; y++) {
                if (y < 0 || y >= H) continue;
                for (int x = px - r; x <= px + r; x++) {
                    if (x < 0 || x >= W) continue;
                    Ac[(long)y * W + x] += err[t++];
                    cnt[(long)y * W + x]++;
                }
            }
        }
    for (long i = 0; i < (long)H * W; i++) Ac[i] /= (double)cnt[i];
    free(cnt);
}

/* FCA score: R [C][H][W] real features, Y [C][T*T] sorted references;
 * A(x) = (1/C) sum_c A_c(x) (feature units) and score = blur(A, sigma_s).
 * Achan (may be NULL): [C][H][W]. */
void orc_fca_score(const double* R, int C, int H, int W, int T, const double* Y, double sigma_s,
                   double* A, double* score, double* Achan) {
    long N = (long)H * W;
    double* Aall = (double*)malloc((size_t)C * N * sizeof(double));
    #pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < C; c++)
        fca_channel(R + (long)c * N, H, W, T, Y + (long)c * T * T, Aall + (long)c * N);
    for (long i = 0; i < N; i++) {
        double s = 0.0;
        for (int c = 0; c < C; c++) s += Aall[(long)c * N + i];
        A[i] = s / (double)C;
    }
    if (Achan) memcpy(Achan, Aall, (size_t)C * N * sizeof(double));
    orc_blur(A, H, W, sigma_s, score);
    free(Aall);
}
