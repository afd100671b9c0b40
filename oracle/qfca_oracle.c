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
 *   - Algorithm 1, the two-pointer quantised patch mismatch      (Alg. 1)
 *   - error-to-pixel association, sigma_p = infinity (box mean)  (Sec. 3.1, Sec. 4.5.4)
 *   - channel mean and the final Gaussian blur sigma_s           (Eq. 1, Sec. 4.5.4)
 *   - the median reference, computed at full precision and then
 *     quantised ("median -> quan")                                (Sec. 3.2, Tab. 3)
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - windows are clipped at the image border; patch and reference histograms
 *     are brought to equal mass by scaling P by n_R and R by n_p;
 *   - quantisation range is [q_lo, q_hi] type-7 quantiles of each channel,
 *     edges rounded to float32 and a value equal to an edge goes to the upper bin;
 *   - the reference median over an even number of patches is the lower median;
 *   - the reference uses every full (unclipped) window;
 *   - the association averages over the in-image windows that contain a pixel;
 *   - errors are in feature units (bin distance times the channel's bin width);
 *   - channels are averaged; the final blur has radius ceil(3 sigma_s) and is
 *     renormalised over in-image taps.
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
/* Algorithm 1: quantised patch mismatch.                                    */

/* P, R: histogram weights (equal total mass), N bins, Q_i = i (bin units).
 * E[i] receives the per-bin mismatch after the division by the original
 * P_i (0 where P_i = 0).  Returns the number of loop iterations. */
int orc_alg1(const long long* Pin, const long long* Rin, int N, double* E) {
    long long* P = (long long*)malloc((size_t)N * sizeof(long long));
    long long* R = (long long*)malloc((size_t)N * sizeof(long long));
    memcpy(P, Pin, (size_t)N * sizeof(long long));
    memcpy(R, Rin, (size_t)N * sizeof(long long));
    for (int i = 0; i < N; i++) E[i] = 0.0;
    int i = 0, j = 0, steps = 0;
    while (i < N && j < N) {
        steps++;
        double dist = (double)(i > j ? i - j : j - i);
        if (P[i] < R[j]) {
            E[i] += (double)P[i] * dist;
            R[j] -= P[i];
            i++;
        } else {
            E[i] += (double)R[j] * dist;
            P[i] -= R[j];
            j++;
        }
    }
    for (int t = 0; t < N; t++) E[t] = Pin[t] > 0 ? E[t] / (double)Pin[t] : 0.0;
    free(P); free(R);
    return steps;
}

/* ------------------------------------------------------------------------ */
/* Reference (Sec. 3.2): per-rank median over patches, then quantised.       */

static int cmp_double_q(const void* a, const void* b) { return cmp_double(a, b); }

/* Literal "median -> quan": every full T x T window's values are sorted; for
 * every rank the lower median over windows is taken at full precision; the
 * resulting reference vector is quantised with the channel's edges.  Output
 * cR[C][B] is the cumulative reference histogram (cR[B-1] = T*T). */
void orc_reference_literal(const double* R, int C, int H, int W, int T, int B,
                           const float* edges, int* cR) {
    int n = T * T;
    long nw = (long)(H - T + 1) * (W - T + 1);
    long h = (nw + 1) / 2; /* lower median: the ceil(nw/2)-th smallest */
    #pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < C; c++) {
        const double* Rc = R + (long)c * H * W;
        double* sorted = (double*)malloc((size_t)nw * n * sizeof(double));
        long w = 0;
        for (int py = 0; py + T <= H; py++)
            for (int px = 0; px + T <= W; px++, w++) {
                double* s = sorted + w * n;
                int t = 0;
                for (int dy = 0; dy < T; dy++)
                    for (int dx = 0; dx < T; dx++) s[t++] = Rc[(long)(py + dy) * W + px + dx];
                qsort(s, (size_t)n, sizeof(double), cmp_double_q);
            }
        double* col = (double*)malloc((size_t)nw * sizeof(double));
        int* hist = (int*)calloc((size_t)B, sizeof(int));
        const float* e = edges + (long)c * (B - 1);
        for (int rho = 0; rho < n; rho++) {
            for (long q = 0; q < nw; q++) col[q] = sorted[q * n + rho];
            qsort(col, (size_t)nw, sizeof(double), cmp_double_q);
            double ref = col[h - 1];
            int b = 0;
            for (int m = 0; m < B - 1; m++)
                if (ref >= (double)e[m]) b++;
            hist[b]++;
        }
        int acc = 0;
        for (int i = 0; i < B; i++) { acc += hist[i]; cR[(long)c * B + i] = acc; }
        free(hist); free(col); free(sorted);
    }
}

/* The same reference from the bins alone: cR(i) is the ceil(nw/2)-th largest
 * of the full-window cumulative counts cP_p(i).  This follows because
 * quantisation is monotone and commutes with order statistics (a derivation,
 * pinned against orc_reference_literal).  Window counts are taken directly. */
void orc_reference_cdf(const uint8_t* bins, int C, int H, int W, int T, int B, int* cR) {
    int n = T * T;
    long nw = (long)(H - T + 1) * (W - T + 1);
    long h = (nw + 1) / 2;
    #pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < C; c++) {
        const uint8_t* bc = bins + (long)c * H * W;
        long* cnt = (long*)calloc((size_t)B * (n + 1), sizeof(long));
        int* P = (int*)malloc((size_t)B * sizeof(int));
        for (int py = 0; py + T <= H; py++)
            for (int px = 0; px + T <= W; px++) {
                for (int i = 0; i < B; i++) P[i] = 0;
                for (int dy = 0; dy < T; dy++)
                    for (int dx = 0; dx < T; dx++) P[bc[(long)(py + dy) * W + px + dx]]++;
                int acc = 0;
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

/* ------------------------------------------------------------------------ */
/* Patch statistics comparison and association for one channel.             */

/* bins_c: [H][W]; cR_c: cumulative reference histogram [B] (total T*T).
 * Ac[H][W] (bin units): mean over the windows p containing x of e_p(b(x)).
 * W1c[H][W] (bin units, may be NULL): window 1-Wasserstein distance between
 * the window histogram and the reference, sum_k |cP~_k - cR~_k| / (n_p n_R).
 * Returns the largest Alg. 1 step count met. */
int orc_channel_map(const uint8_t* bc, int H, int W, int T, int B, const int* cR_c,
                    double* Ac, double* W1c) {
    int r = T / 2;
    long nR = (long)T * T;
    double* e = (double*)malloc((size_t)H * W * B * sizeof(double));
    long long* P = (long long*)malloc((size_t)B * sizeof(long long));
    long long* Rt = (long long*)malloc((size_t)B * sizeof(long long));
    double* E = (double*)malloc((size_t)B * sizeof(double));
    int maxsteps = 0;
    for (int py = 0; py < H; py++) {
        for (int px = 0; px < W; px++) {
            for (int i = 0; i < B; i++) P[i] = 0;
            long np = 0;
            for (int y = py - r; y <= py + r; y++) {
                if (y < 0 || y >= H) continue;
                for (int x = px - r; x <= px + r; x++) {
                    if (x < 0 || x >= W) continue;
                    P[bc[(long)y * W + x]]++;
                    np++;
                }
            }
            /* equal-mass scaling: P~ = P n_R, R~ = R n_p */
            for (int i = 0; i < B; i++) {
                long Ri = cR_c[i] - (i > 0 ? cR_c[i - 1] : 0);
                P[i] *= nR;
                Rt[i] = Ri * np;
            }
            int steps = orc_alg1(P, Rt, B, E);
            if (steps > maxsteps) maxsteps = steps;
            double* ep = e + ((long)py * W + px) * B;
            for (int i = 0; i < B; i++) ep[i] = E[i];
            if (W1c) {
                long a = 0, b = 0;
                double s = 0.0;
                for (int k = 0; k < B; k++) {
                    a += P[k];
                    b += Rt[k];
                    s += (double)llabs(a - b);
                }
                W1c[(long)py * W + px] = s / ((double)np * (double)nR);
            }
        }
    }
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            int b = bc[(long)y * W + x];
            double s = 0.0;
            long cnt = 0;
            for (int py = y - r; py <= y + r; py++) {
                if (py < 0 || py >= H) continue;
                for (int px = x - r; px <= x + r; px++) {
                    if (px < 0 || px >= W) continue;
                    s += e[((long)py * W + px) * B + b];
                    cnt++;
                }
            }
            Ac[(long)y * W + x] = s / (double)cnt;
        }
    }
    free(E); free(Rt); free(P); free(e);
    return maxsteps;
}

/* The per-window mismatch vector e_p (bin units) of one window, as used by
 * orc_channel_map; exposed for pins.  Returns the Alg. 1 step count. */
int orc_window_errors(const uint8_t* bc, int H, int W, int T, int B, const int* cR_c,
                      int py, int px, double* e_out) {
    int r = T / 2;
    long nR = (long)T * T;
    long long* P = (long long*)calloc((size_t)B, sizeof(long long));
    long long* Rt = (long long*)malloc((size_t)B * sizeof(long long));
    long np = 0;
    for (int y = py - r; y <= py + r; y++) {
        if (y < 0 || y >= H) continue;
        for (int x = px - r; x <= px + r; x++) {
            if (x < 0 || x >= W) continue;
            P[bc[(long)y * W + x]]++;
            np++;
        }
    }
    for (int i = 0; i < B; i++) {
        long Ri = cR_c[i] - (i > 0 ? cR_c[i - 1] : 0);
        P[i] *= nR;
        Rt[i] = Ri * np;
    }
    int steps = orc_alg1(P, Rt, B, e_out);
    free(Rt); free(P);
    return steps;
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
 * Achan (may be NULL) receives the per-channel maps delta_c Ac_c [C][H][W];
 * W1 (may be NULL) the channel mean of delta_c W1c_c.  Returns the largest
 * Alg. 1 step count. */
int orc_score(const uint8_t* bins, int C, int H, int W, int T, int B, const int* cR,
              const double* delta, double sigma_s, double* A, double* score, double* W1,
              double* Achan) {
    long N = (long)H * W;
    double* Aall = (double*)malloc((size_t)C * N * sizeof(double));
    double* Wall = W1 ? (double*)malloc((size_t)C * N * sizeof(double)) : NULL;
    int maxsteps = 0;
    #pragma omp parallel for schedule(dynamic) reduction(max : maxsteps)
    for (int c = 0; c < C; c++) {
        int s = orc_channel_map(bins + (long)c * N, H, W, T, B, cR + (long)c * B,
                                Aall + (long)c * N, Wall ? Wall + (long)c * N : NULL);
        if (s > maxsteps) maxsteps = s;
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
    return maxsteps;
}

/* A(x) at a list of pixels only, each from its definition (for sampled checks
 * on maps too large for orc_score).  Achan_out may be NULL or [npix][C]. */
void orc_amap_pixels(const uint8_t* bins, int C, int H, int W, int T, int B, const int* cR,
                     const double* delta, int npix, const int* ys, const int* xs,
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
            double s = 0.0;
            long cnt = 0;
            for (int py = y - r; py <= y + r; py++) {
                if (py < 0 || py >= H) continue;
                for (int px = x - r; px <= x + r; px++) {
                    if (px < 0 || px >= W) continue;
                    orc_window_errors(bc, H, W, T, B, cR + (long)c * B, py, px, E);
                    s += E[b];
                    cnt++;
                }
            }
            double v = delta[c] * s / (double)cnt;
            if (Achan_out) Achan_out[(long)t * C + c] = v;
            acc += v;
        }
        A_out[t] = acc / (double)C;
        free(E);
    }
}
