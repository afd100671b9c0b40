// Host-only model checks and the serialised model format (see qfca_blob.h).
// Compiled as plain C++ (no device pass).
#include "qfca_blob.h"

#include <math.h>
#include <string.h>

namespace qfca {
namespace {

constexpr char kModelMagic[8] = {'Q', 'F', 'C', 'A', 'M', 'D', 'L', '\0'};
constexpr size_t kParamBytes[3] = {0, 40, 44};

size_t model_header(uint32_t version) { return 8 + 4 + 4 + kParamBytes[version]; }

struct Sizes {
    size_t mu, V, edges, delta, cR, evals, lohi, cRw, total;
};

Sizes blob_sizes(const qfca_params& p, uint32_t flags, uint32_t version) {
    Sizes z;
    const size_t C = (size_t)p.C;
    const size_t P = (size_t)blob_planes(p);
    z.mu = C * 8;
    z.V = p.preproc != QFCA_PRE_NONE ? C * (size_t)p.k * 8 : 0;
    z.edges = P * (size_t)(p.B > 1 ? p.B - 1 : 0) * 4;
    z.delta = P * 8;
    z.cR = (flags & 1u) ? P * (size_t)p.B * 4 : 0;
    z.evals = (flags & 2u) ? C * 8 : 0;
    z.lohi = (flags & 4u) ? P * 16 : 0;
    z.cRw = (flags & 8u) ? P * (size_t)p.B * 8 : 0;
    z.total = model_header(version) + z.mu + z.V + z.edges + z.delta + z.cR + z.evals + z.lohi + z.cRw;
    return z;
}

void put_params(unsigned char* d, const qfca_params& p) {
    const int32_t iv[4] = {p.C, p.k, p.B, p.T};
    const float fv[3] = {p.q_lo, p.q_hi, p.sigma_s};
    const int32_t jv[2] = {p.preproc, p.proj_prec};
    memcpy(d, iv, 16);
    memcpy(d + 16, fv, 12);
    memcpy(d + 28, jv, 8);
    memcpy(d + 36, &p.sigma_p, 4);
    memcpy(d + 40, &p.reference, 4);
}

qfca_params get_params(const unsigned char* d, uint32_t version) {
    int32_t iv[4];
    float fv[3];
    int32_t jv[2];
    memcpy(iv, d, 16);
    memcpy(fv, d + 16, 12);
    memcpy(jv, d + 28, 8);
    qfca_params p{};
    p.C = iv[0]; p.k = iv[1]; p.B = iv[2]; p.T = iv[3];
    p.q_lo = fv[0]; p.q_hi = fv[1]; p.sigma_s = fv[2];
    p.preproc = jv[0]; p.proj_prec = jv[1];
    p.sigma_p = INFINITY;
    p.reference = QFCA_REF_MEDIAN_QUAN;
    if (version >= 2) {
        memcpy(&p.sigma_p, d + 36, 4);
        memcpy(&p.reference, d + 40, 4);
    }
    return p;
}

qfca_status bad(qfca_status s, std::string* err, const char* msg) {
    if (err) *err = msg;
    return s;
}

}  // namespace

qfca_status host_check_params(const qfca_params* p, std::string* err) {
    if (!p) return bad(QFCA_E_ARG, err, "params is NULL");
    if (p->C < 1 || p->C > 2048) return bad(QFCA_E_ARG, err, "C must be in [1, 2048]");
    if (p->B < 1 || p->B > 64) return bad(QFCA_E_UNSUPPORTED, err, "B must be in [1, 64]");
    if (p->T < 1 || p->T > 63 || (p->T % 2) == 0) return bad(QFCA_E_UNSUPPORTED, err, "T must be odd, 1..63");
    if (p->preproc != QFCA_PRE_NONE && p->preproc != QFCA_PRE_RESIDUAL && p->preproc != QFCA_PRE_COORDS)
        return bad(QFCA_E_ARG, err, "unknown preproc");
    if (p->proj_prec != QFCA_PREC_FP32 && p->proj_prec != QFCA_PREC_BF16)
        return bad(QFCA_E_ARG, err, "unknown proj_prec");
    if (p->preproc == QFCA_PRE_RESIDUAL && (p->k < 0 || p->k > 64 || p->k > p->C - 1))
        return bad(QFCA_E_UNSUPPORTED, err, "k must be in [0, min(64, C-1)]");
    if (p->preproc == QFCA_PRE_COORDS && (p->k < 1 || p->k > 64 || p->k > p->C))
        return bad(QFCA_E_UNSUPPORTED, err, "k must be in [1, min(64, C)] for principal coordinates");
    if (!(p->q_lo >= 0.f && p->q_lo < p->q_hi && p->q_hi <= 1.f))
        return bad(QFCA_E_ARG, err, "need 0 <= q_lo < q_hi <= 1");
    if (!(p->sigma_s >= 0.f && p->sigma_s <= 5.f)) return bad(QFCA_E_ARG, err, "sigma_s must be in [0, 5]");
    if (!(p->sigma_p > 0.f)) return bad(QFCA_E_ARG, err, "sigma_p must be > 0 (INFINITY: plain mean)");
    if (p->reference < QFCA_REF_MEDIAN_QUAN || p->reference > QFCA_REF_QUAN_MEAN)
        return bad(QFCA_E_ARG, err, "unknown reference");
    return QFCA_OK;
}

qfca_status host_check_arrays(const qfca_params& p, const float* edges, const double* delta, const int32_t* cR,
                              std::string* err) {
    const int B = p.B, T = p.T, P = blob_planes(p);
    if ((B > 1 && !edges) || !delta) return bad(QFCA_E_ARG, err, "edges and delta are required");
    for (int c = 0; c < P; ++c) {
        if (!(delta[c] >= 0.0) || !isfinite(delta[c])) return bad(QFCA_E_ARG, err, "delta must be finite, >= 0");
        for (int i = 1; i + 1 < B; ++i)
            if (!(edges[(size_t)c * (B - 1) + i] >= edges[(size_t)c * (B - 1) + i - 1]))
                return bad(QFCA_E_ARG, err, "edges must be nondecreasing per channel");
    }
    if (cR) {
        for (int c = 0; c < P; ++c) {
            if (cR[(size_t)c * B + B - 1] != T * T) return bad(QFCA_E_ARG, err, "cR[c][B-1] must equal T*T");
            for (int i = 0; i < B; ++i) {
                const int32_t v = cR[(size_t)c * B + i];
                if (v < 0 || (i > 0 && v < cR[(size_t)c * B + i - 1]))
                    return bad(QFCA_E_ARG, err, "cR must be nondecreasing and >= 0");
            }
        }
    }
    return QFCA_OK;
}

qfca_status host_check_weights(const qfca_params& p, const double* cRw, std::string* err) {
    const size_t n = (size_t)blob_planes(p) * (size_t)p.B;
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(cRw[i]) || cRw[i] < 0.0 || (i % (size_t)p.B && cRw[i] < cRw[i - 1]))
            return bad(QFCA_E_ARG, err, "malformed reference weights");
    return QFCA_OK;
}

size_t blob_bytes(const qfca_params& p, uint32_t flags) { return blob_sizes(p, flags, kModelVersion).total; }

void blob_write(const ModelArrays& m, unsigned char* d) {
    const Sizes z = blob_sizes(m.p, m.flags, kModelVersion);
    memcpy(d, kModelMagic, 8);
    memcpy(d + 8, &kModelVersion, 4);
    memcpy(d + 12, &m.flags, 4);
    put_params(d + 16, m.p);
    size_t o = model_header(kModelVersion);
    auto put = [&](const void* src, size_t n) {
        if (n) memcpy(d + o, src, n);
        o += n;
    };
    put(m.mu.data(), z.mu);
    put(m.V.data(), z.V);
    put(m.edges.data(), z.edges);
    put(m.delta.data(), z.delta);
    put(m.cR.data(), z.cR);
    put(m.evals.data(), z.evals);
    if (z.lohi) {
        put(m.lo.data(), z.lohi / 2);
        put(m.hi.data(), z.lohi / 2);
    }
    put(m.cRw.data(), z.cRw);
}

qfca_status blob_read(const void* buf, size_t bytes, ModelArrays* out, std::string* err) {
    if (!buf || !out) return bad(QFCA_E_ARG, err, "NULL argument");
    const unsigned char* d = (const unsigned char*)buf;
    if (bytes < model_header(1) || memcmp(d, kModelMagic, 8) != 0) return bad(QFCA_E_ARG, err, "not a serialised model");
    uint32_t version = 0, flags = 0;
    memcpy(&version, d + 8, 4);
    memcpy(&flags, d + 12, 4);
    if (version < 1 || version > kModelVersion) return bad(QFCA_E_UNSUPPORTED, err, "unknown model format version");
    if (bytes < model_header(version)) return bad(QFCA_E_ARG, err, "not a serialised model");
    if (flags & ~15u) return bad(QFCA_E_ARG, err, "unknown model flags");
    if ((flags & 1u) && (flags & 8u)) return bad(QFCA_E_ARG, err, "two references in one model");
    ModelArrays m;
    m.p = get_params(d + 16, version);
    m.flags = flags;
    qfca_status st = host_check_params(&m.p, err);
    if (st != QFCA_OK) return st;
    const Sizes z = blob_sizes(m.p, flags, version);
    if (bytes != z.total) return bad(QFCA_E_ARG, err, "byte count does not match the serialised model");
    size_t o = model_header(version);
    auto take = [&](auto& v, size_t n) {
        v.resize(n / sizeof(v[0]));
        if (n) memcpy(v.data(), d + o, n);
        o += n;
    };
    take(m.mu, z.mu);
    take(m.V, z.V);
    take(m.edges, z.edges);
    take(m.delta, z.delta);
    take(m.cR, z.cR);
    take(m.evals, z.evals);
    take(m.lo, z.lohi / 2);
    take(m.hi, z.lohi / 2);
    take(m.cRw, z.cRw);
    st = host_check_arrays(m.p, z.edges ? m.edges.data() : nullptr, m.delta.data(), z.cR ? m.cR.data() : nullptr,
                           err);
    if (st != QFCA_OK) return st;
    if (z.cRw && (st = host_check_weights(m.p, m.cRw.data(), err)) != QFCA_OK) return st;
    *out = std::move(m);
    return QFCA_OK;
}

}  // namespace qfca
