// CPU driver of the library's host-only code, built by the CPU tests with
// the address and undefined-behaviour sanitizers: serialised models (round
// trips, every truncation, seeded corruption of bytes and of array values),
// the symmetric eigensolver (residuals and orthonormality on seeded
// matrices, tiny and degenerate ones included) and the serving admission
// policy (seeded random traces).  Prints "ok" and exits 0 when every check
// holds; a sanitizer finding aborts the run.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <deque>
#include <random>
#include <string>
#include <vector>

#include "qfca_blob.h"
#include "serve_policy.h"

namespace qfca {
int sym_eig(double* A, int n, double* evals, double* vecs);
int sym_eig_top(double* A, int n, int k, double* evals, double* vecs);
}  // namespace qfca

using namespace qfca;

static int failures = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            ++failures;                                    \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);                  \
            fprintf(stderr, "\n");                         \
        }                                                  \
    } while (0)

static ModelArrays make_model(std::mt19937_64& g, int preproc, int C, int k, int B, int T, uint32_t flags) {
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    ModelArrays m;
    m.p.C = C; m.p.k = k; m.p.B = B; m.p.T = T;
    m.p.q_lo = 0.01f; m.p.q_hi = 0.99f; m.p.sigma_s = 1.0f;
    m.p.preproc = preproc; m.p.proj_prec = QFCA_PREC_FP32;
    m.p.sigma_p = INFINITY; m.p.reference = QFCA_REF_MEDIAN_QUAN;
    m.flags = flags;
    const int P = blob_planes(m.p);
    m.mu.resize(C);
    for (auto& v : m.mu) v = U(g);
    if (preproc != QFCA_PRE_NONE) {
        m.V.resize((size_t)C * k);
        for (auto& v : m.V) v = U(g);
    }
    m.delta.resize(P);
    for (auto& v : m.delta) v = 0.1 + 0.5 * fabs(U(g));
    m.edges.resize((size_t)P * (B > 1 ? B - 1 : 0));
    for (int c = 0; c < P; ++c)
        for (int i = 0; i + 1 < B; ++i) m.edges[(size_t)c * (B - 1) + i] = (float)(-1.0 + m.delta[c] * (i + 1));
    if (flags & 1u) {
        m.cR.resize((size_t)P * B);
        for (int c = 0; c < P; ++c)
            for (int i = 0; i < B; ++i) m.cR[(size_t)c * B + i] = (i + 1) * T * T / B;
        for (int c = 0; c < P; ++c) m.cR[(size_t)c * B + B - 1] = T * T;
    }
    if (flags & 2u) {
        m.evals.resize(C);
        for (auto& v : m.evals) v = fabs(U(g));
    }
    if (flags & 4u) {
        m.lo.resize(P);
        m.hi.resize(P);
        for (int c = 0; c < P; ++c) {
            m.lo[c] = -1.0;
            m.hi[c] = -1.0 + m.delta[c] * B;
        }
    }
    if (flags & 8u) {
        m.cRw.resize((size_t)P * B);
        for (int c = 0; c < P; ++c) {
            double acc = 0.0;
            for (int i = 0; i < B; ++i) m.cRw[(size_t)c * B + i] = (acc += fabs(U(g)));
        }
    }
    return m;
}

static bool same(const ModelArrays& a, const ModelArrays& b) {
    return a.flags == b.flags && memcmp(&a.p, &b.p, sizeof(a.p)) == 0 && a.mu == b.mu && a.V == b.V &&
           a.delta == b.delta && a.evals == b.evals && a.lo == b.lo && a.hi == b.hi && a.cRw == b.cRw &&
           a.edges == b.edges && a.cR == b.cR;
}

static void test_blobs() {
    std::mt19937_64 g(2510);
    struct Cfg {
        int preproc, C, k, B, T;
        uint32_t flags;
    } cfgs[] = {{QFCA_PRE_RESIDUAL, 16, 4, 8, 5, 1u | 2u | 4u}, {QFCA_PRE_NONE, 5, 0, 1, 3, 1u},
                {QFCA_PRE_COORDS, 12, 3, 16, 7, 4u | 8u}, {QFCA_PRE_RESIDUAL, 9, 0, 4, 3, 0u},
                {QFCA_PRE_RESIDUAL, 33, 8, 64, 31, 8u | 2u}};
    for (const Cfg& c : cfgs) {
        const ModelArrays m = make_model(g, c.preproc, c.C, c.k, c.B, c.T, c.flags);
        std::vector<unsigned char> blob(blob_bytes(m.p, m.flags));
        blob_write(m, blob.data());
        ModelArrays r;
        std::string err;
        CHECK(blob_read(blob.data(), blob.size(), &r, &err) == QFCA_OK, "round trip: %s", err.c_str());
        CHECK(same(m, r), "round trip differs");
        // every truncation is refused
        for (size_t n = 0; n < blob.size(); ++n) {
            ModelArrays t;
            CHECK(blob_read(blob.data(), n, &t, &err) != QFCA_OK, "truncation to %zu bytes accepted", n);
        }
        // one byte too many is refused
        std::vector<unsigned char> longer(blob);
        longer.push_back(0);
        CHECK(blob_read(longer.data(), longer.size(), &r, &err) != QFCA_OK, "trailing byte accepted");
        // seeded corruption: any outcome but a crash or undefined behaviour;
        // an accepted blob must hold arrays of the sizes its header states
        std::uniform_int_distribution<size_t> pos(0, blob.size() - 1);
        std::uniform_int_distribution<int> byte(0, 255);
        for (int trial = 0; trial < 3000; ++trial) {
            std::vector<unsigned char> b(blob);
            const int nflip = 1 + trial % 4;
            for (int f = 0; f < nflip; ++f) b[pos(g)] = (unsigned char)byte(g);
            ModelArrays t;
            if (blob_read(b.data(), b.size(), &t, &err) == QFCA_OK) {
                const size_t P = (size_t)blob_planes(t.p);
                CHECK(t.mu.size() == (size_t)t.p.C && t.delta.size() == P, "accepted blob with wrong sizes");
                CHECK(blob_bytes(t.p, t.flags) == b.size(), "accepted blob of another size");
            }
        }
    }
    // array rules
    ModelArrays m = make_model(g, QFCA_PRE_RESIDUAL, 6, 2, 8, 5, 1u | 8u);
    m.flags = 1u;
    m.cRw.clear();
    std::string err;
    std::vector<float> e = m.edges;
    e[3] = e[2] - 1.0f;
    CHECK(host_check_arrays(m.p, e.data(), m.delta.data(), m.cR.data(), &err) != QFCA_OK, "descending edges");
    std::vector<double> d = m.delta;
    d[1] = NAN;
    CHECK(host_check_arrays(m.p, m.edges.data(), d.data(), m.cR.data(), &err) != QFCA_OK, "NaN delta");
    std::vector<int32_t> cr = m.cR;
    cr[7] = 1;
    CHECK(host_check_arrays(m.p, m.edges.data(), m.delta.data(), cr.data(), &err) != QFCA_OK, "cR mass");
    std::vector<double> w((size_t)6 * 8, 1.0);
    w[9] = 0.5;
    CHECK(host_check_weights(m.p, w.data(), &err) != QFCA_OK, "decreasing weights");
    qfca_params bad = m.p;
    bad.T = 4;
    CHECK(host_check_params(&bad, &err) != QFCA_OK, "even T");
    bad = m.p;
    bad.k = 64;
    CHECK(host_check_params(&bad, &err) != QFCA_OK, "k >= C");
    CHECK(host_check_params(nullptr, &err) != QFCA_OK, "NULL params");
}

static void check_eig(const std::vector<double>& A, int n, const double* ev, const double* V, int k, int ld,
                      const char* what) {
    double scale = 1e-300;
    for (double a : A) scale = fmax(scale, fabs(a));
    for (int j = 0; j < k; ++j) {
        if (j > 0) CHECK(ev[j] <= ev[j - 1] + 1e-12 * scale, "%s: eigenvalues not descending at %d", what, j);
        double res = 0.0, nrm = 0.0;
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int t = 0; t < n; ++t) s += A[(size_t)i * n + t] * V[(size_t)t * ld + j];
            res = fmax(res, fabs(s - ev[j] * V[(size_t)i * ld + j]));
            nrm += V[(size_t)i * ld + j] * V[(size_t)i * ld + j];
        }
        CHECK(res <= 1e-10 * scale * n, "%s: residual %g at %d", what, res, j);
        CHECK(fabs(nrm - 1.0) <= 1e-10, "%s: norm %g at %d", what, nrm, j);
        for (int j2 = 0; j2 < j; ++j2) {
            double dot = 0.0;
            for (int i = 0; i < n; ++i) dot += V[(size_t)i * ld + j] * V[(size_t)i * ld + j2];
            CHECK(fabs(dot) <= 1e-9, "%s: vectors %d %d not orthogonal (%g)", what, j, j2, dot);
        }
    }
}

static void test_eig() {
    std::mt19937_64 g(15602);
    std::normal_distribution<double> N(0.0, 1.0);
    const int sizes[] = {1, 2, 3, 5, 17, 64, 130};
    for (int n : sizes) {
        for (int kind = 0; kind < 3; ++kind) {
            std::vector<double> A((size_t)n * n, 0.0);
            if (kind == 0) {  // a covariance
                const int m = 2 * n + 3;
                std::vector<double> X((size_t)n * m);
                for (auto& x : X) x = N(g);
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j <= i; ++j) {
                        double s = 0.0;
                        for (int t = 0; t < m; ++t) s += X[(size_t)i * m + t] * X[(size_t)j * m + t];
                        A[(size_t)i * n + j] = A[(size_t)j * n + i] = s / m;
                    }
            } else if (kind == 1) {  // rank 2 (a cluster of zero eigenvalues)
                std::vector<double> u(n), v(n);
                for (int i = 0; i < n; ++i) { u[i] = N(g); v[i] = N(g); }
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = u[i] * u[j] + 0.5 * v[i] * v[j];
            } else {  // diagonal with repeated values
                for (int i = 0; i < n; ++i) A[(size_t)i * n + i] = (double)(i % 3);
            }
            std::vector<double> ev(n), V((size_t)n * n), B(A);
            CHECK(sym_eig(B.data(), n, ev.data(), V.data()) == 0, "sym_eig n=%d kind=%d", n, kind);
            check_eig(A, n, ev.data(), V.data(), n, n, "sym_eig");
            const int k = n < 8 ? n : 8;
            std::vector<double> ev2(n), V2((size_t)n * k);
            B = A;
            CHECK(sym_eig_top(B.data(), n, k, ev2.data(), V2.data()) == 0, "sym_eig_top n=%d kind=%d", n, kind);
            if (kind != 1) check_eig(A, n, ev2.data(), V2.data(), k, k, "sym_eig_top");
            for (int j = 0; j < n; ++j)
                CHECK(fabs(ev2[j] - ev[j]) <= 1e-10 * (1.0 + fabs(ev[j])), "eigenvalue %d differs", j);
        }
    }
    std::vector<double> e(1), v(1);
    double a = 0.0;
    CHECK(sym_eig_top(&a, 1, 2, e.data(), v.data()) != 0, "k > n accepted");
}

struct Req {
    uint64_t ticket = 0;
    int group = 0;
    size_t bytes = 0, off = 0;
};

static void test_policy() {
    std::mt19937_64 g(355);
    for (int trial = 0; trial < 200; ++trial) {
        serve::Arena arena;
        const size_t size = serve::align_up(1 + g() % (1u << 22));
        arena.reset(size);
        std::deque<Req> pending;
        std::vector<Req> live;
        uint64_t next = 1;
        for (int step = 0; step < 400; ++step) {
            const int op = (int)(g() % 3);
            if (op == 0) {
                Req r;
                r.ticket = next++;
                r.group = (int)(g() % 3);
                r.bytes = serve::request_bytes(1 + (int)(g() % 64), 1 + (int)(g() % 300), 1 + (int)(g() % 300));
                pending.push_back(r);
            } else if (op == 1) {
                std::vector<Req> out;
                uint64_t blocked = 0;
                serve::form_batch(pending, arena, 1 + (int)(g() % 8), out, &blocked);
                for (const Req& r : out) {
                    CHECK(r.off + r.bytes <= size, "batch member beyond the arena");
                    live.push_back(r);
                }
            } else if (!live.empty()) {
                const size_t i = g() % live.size();
                arena.release(live[i].off, live[i].bytes);
                live.erase(live.begin() + (long)i);
            }
        }
        for (const Req& r : live) arena.release(r.off, r.bytes);
        CHECK(arena.used() == 0, "arena not empty after every release");
    }
}

int main() {
    test_blobs();
    test_eig();
    test_policy();
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
