// C ABI of libqfca: argument validation, contexts, models and the order of
// kernel launches for the fit, quantisation and score-map calls.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "qfca_blob.h"
#include "qfca_internal.h"

namespace qfca {
namespace {
thread_local std::string g_err;
}
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace qfca

using namespace qfca;

enum Slot {
    SL_ASUM = 0, SL_W1SUM, SL_SCORE, SL_RESID, SL_BINS, SL_COUNTS, SL_SEL,
    SL_COV, SL_MU, SL_RANKS, SL_CR, SL_CRW, SL_RMPART, SL_BBINS, SL_BASUM, SL_COUNT
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

enum { K_SCORE = 0, K_PROJ, K_FINISH, K_COUNT };

struct qfca_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    DevBuf scratch[SL_COUNT];
    std::map<long long, ScoreTile> tiles;  // tile-configuration cache
    ScoreTile tile_override{0, 0, 0, 0};   // Ws == 0: automatic
    uint32_t profile_mask = 0;  // bit k: time kernel k
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed[K_COUNT];
    std::vector<hipEvent_t> event_pool;
    // batched path
    BatchHeader* d_hdr = nullptr;
    BatchJob* d_jobs = nullptr;
    BatchHeader* h_hdr = nullptr;  // pinned staging
    BatchJob* h_jobs = nullptr;
    hipEvent_t staged = nullptr;   // the last upload from the staging buffers
    hipStream_t capture = nullptr; // private stream used only to capture graphs
    std::map<long long, GraphEntry> graphs;
    std::map<long long, ScoreTile> tuned;  // autotuned tiles keyed by (T, B)
    int ncu = 0;            // compute units of the device (0: not read yet)
    size_t lds_per_cu = 0;  // bytes of LDS per compute unit
};

struct qfca_model_s {
    qfca_params p{};
    int device = 0;
    int KP = 0;  // projection width (k padded to 8/16/32/64)
    int Bp = 8;  // lanes per channel in the score kernel
    int m = 1;   // T*T
    std::vector<double> mu, V, evals, lo, hi, delta;
    std::vector<float> edges;
    std::vector<int32_t> cR;   // integer reference of mass T*T (the fast path)
    std::vector<double> cRw;   // the reference as cumulative weights (any reference)
    bool has_ref = false, has_evals = false, has_lohi = false;
    bool ref_general = false;  // the reference is not integer of mass T*T
    float* d_mu = nullptr;
    float* d_V = nullptr;
    void* d_V1 = nullptr;  // MFMA operand tables of the projection (nullptr: VALU path)
    void* d_V2 = nullptr;
    void* d_V1b = nullptr;  // the same padded for the batch kernel (batch_combo), or nullptr
    void* d_V2b = nullptr;
    uint16_t* d_Vbf = nullptr;
    float* d_edges = nullptr;
    float* d_lo = nullptr;
    float* d_invd = nullptr;
    float* d_fastd = nullptr;
    double* d_delta = nullptr;
    int32_t* d_cR = nullptr;
    ScoreTables tab;
    std::vector<void*> owned;
    ~qfca_model_s() {
        for (void* q : owned) (void)hipFree(q);
    }
};

namespace {

qfca_status fail(qfca_status s, const std::string& msg) {
    set_error(msg);
    return s;
}

qfca_status hip_fail(hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(e == hipErrorOutOfMemory ? QFCA_E_NOMEM : QFCA_E_DEVICE, m);
}

#define HIP_TRY(expr)                                       \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return hip_fail(_e, #expr);   \
    } while (0)

qfca_status check_params(const qfca_params* p) {
    std::string err;
    const qfca_status st = host_check_params(p, &err);
    return st == QFCA_OK ? st : fail(st, err);
}

// Histogrammed planes of a model: the C channels (PRE_NONE, PRE_RESIDUAL) or
// the k principal coordinates (PRE_COORDS).
int planes(const qfca_params& p) { return p.preproc == QFCA_PRE_COORDS ? p.k : p.C; }

qfca_status check_shape(int H, int W, int C) {
    if (H < 1 || W < 1) return fail(QFCA_E_SHAPE, "H and W must be >= 1");
    if ((long long)H * W > (1LL << 30)) return fail(QFCA_E_SHAPE, "H*W too large");
    if ((long long)H * W * C > (1LL << 40)) return fail(QFCA_E_SHAPE, "C*H*W too large");
    return QFCA_OK;
}

template <class Tp>
hipError_t scratch(qfca_ctx ctx, Slot s, size_t bytes, Tp** out) {
    DevBuf& b = ctx->scratch[s];
    if (b.bytes < bytes) {
        if (b.p) {
            hipError_t e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) return e;
            (void)hipFree(b.p);
            b.p = nullptr;
            b.bytes = 0;
        }
        hipError_t e = hipMalloc(&b.p, bytes);
        if (e != hipSuccess) return e;
        b.bytes = bytes;
    }
    *out = (Tp*)b.p;
    return hipSuccess;
}

template <class Tp>
hipError_t upload(qfca_model m, Tp** dst, const Tp* src, size_t n) {
    if (!*dst) {
        hipError_t e = hipMalloc((void**)dst, std::max<size_t>(n, 1) * sizeof(Tp));
        if (e != hipSuccess) return e;
        m->owned.push_back(*dst);
    }
    if (n) return hipMemcpy(*dst, src, n * sizeof(Tp), hipMemcpyHostToDevice);
    return hipSuccess;
}

uint16_t f32_to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);  // inf / nan
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;  // round to nearest even
    return (uint16_t)(u >> 16);
}

size_t align16c(size_t x) { return (x + 15) & ~size_t(15); }

int pow2_at_least(int v, int lo) {
    int p = lo;
    while (p < v) p <<= 1;
    return p;
}

// Upload mu and V (float32, V padded to KP columns, plus a bf16 copy).
qfca_status upload_projection(qfca_model m) {
    const int C = m->p.C, k = m->p.k;
    const bool pre = m->p.preproc != QFCA_PRE_NONE;
    m->KP = (!pre || k == 0) ? 0 : (k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64);
    std::vector<float> muf(C, 0.f), Vf((size_t)C * std::max(m->KP, 1), 0.f);
    std::vector<uint16_t> Vb(Vf.size(), 0);
    if (pre) {
        for (int c = 0; c < C; ++c) muf[c] = (float)m->mu[c];
        for (int c = 0; c < C; ++c)
            for (int j = 0; j < k; ++j) {
                Vf[(size_t)c * m->KP + j] = (float)m->V[(size_t)c * k + j];
                Vb[(size_t)c * m->KP + j] = f32_to_bf16(Vf[(size_t)c * m->KP + j]);
            }
    }
    HIP_TRY(upload(m, &m->d_mu, muf.data(), muf.size()));
    HIP_TRY(upload(m, &m->d_V, Vf.data(), Vf.size()));
    HIP_TRY(upload(m, &m->d_Vbf, Vb.data(), Vb.size()));
    m->d_V1 = m->d_V2 = nullptr;
    m->d_V1b = m->d_V2b = nullptr;
    if (pre && k > 0 && mfma_cmax(C, m->p.proj_prec) && mfma_kt(k, m->p.proj_prec)) {
        std::vector<float> Vk((size_t)C * k);
        for (size_t i = 0; i < Vk.size(); ++i) Vk[i] = (float)m->V[i];
        std::vector<uint16_t> Vkb(Vk.size());
        for (size_t i = 0; i < Vk.size(); ++i) Vkb[i] = f32_to_bf16(Vk[i]);
        const bool bf = m->p.proj_prec == QFCA_PREC_BF16;
        // tables padded to (CM, KT): uploads them, returns the two device pointers
        auto tables = [&](int CM, int KT, void** d1, void** d2) -> qfca_status {
            if (bf) {
                std::vector<uint16_t> T1, T2;
                mfma_tables_bf16_at(Vkb.data(), C, k, CM, KT, T1, T2);
                uint16_t *p1 = nullptr, *p2 = nullptr;
                HIP_TRY(upload(m, &p1, T1.data(), T1.size()));
                HIP_TRY(upload(m, &p2, T2.data(), T2.size()));
                *d1 = p1;
                *d2 = p2;
            } else {
                std::vector<float> T1, T2;
                mfma_tables_f32_at(Vk.data(), C, k, CM, KT, T1, T2);
                float *p1 = nullptr, *p2 = nullptr;
                HIP_TRY(upload(m, &p1, T1.data(), T1.size()));
                HIP_TRY(upload(m, &p2, T2.data(), T2.size()));
                *d1 = p1;
                *d2 = p2;
            }
            return QFCA_OK;
        };
        const int CM = mfma_cmax(C, m->p.proj_prec), KT = mfma_kt(k, m->p.proj_prec);
        qfca_status st = tables(CM, KT, &m->d_V1, &m->d_V2);
        if (st != QFCA_OK) return st;
        // the persistent batch kernel is instantiated for fewer paddings: its
        // own copy of the tables when its padding differs
        int CMb = 0, KTb = 0;
        if (m->p.preproc == QFCA_PRE_RESIDUAL && batch_combo(C, k, m->p.proj_prec, &CMb, &KTb)) {
            if (CMb == CM && KTb == KT) {
                m->d_V1b = m->d_V1;
                m->d_V2b = m->d_V2;
            } else if ((st = tables(CMb, KTb, &m->d_V1b, &m->d_V2b)) != QFCA_OK) {
                return st;
            }
        }
    } else if (pre && k > 0 && m->p.proj_prec == QFCA_PREC_BF16) {
        return fail(QFCA_E_UNSUPPORTED, "the BF16 projection needs C <= 512");
    }
    return QFCA_OK;
}

// Upload edges, lo, 1/delta and delta.
qfca_status upload_quant(qfca_model m) {
    const int C = planes(m->p), B = m->p.B;
    std::vector<float> lof(C), invd(C);
    for (int c = 0; c < C; ++c) {
        lof[c] = (float)m->lo[c];
        invd[c] = m->delta[c] > 0.0 ? (float)(1.0 / m->delta[c]) : 0.f;
    }
    // Margin of the arithmetic bin guess t = (r - lo) * (1/delta) (FP32 on the
    // device, three roundings: relative error below 3.1e-7 of |t|): with
    // dev = max_m |(e_m - lo) / delta - m| over the stored edges, a value
    // whose t lies farther than dev + (B + 2) * 2.4e-7 from every integer
    // has bin floor(t) (clamped).  The shortcut is off for a channel whose
    // margin would be one half or more, or whose 1/delta is zero: its margin
    // is +infinity, which no distance reaches.
    std::vector<float> fastd(C, INFINITY);
    for (int c = 0; c < C; ++c) {
        const double dl = m->delta[c];
        if (!(dl > 0.0) || B < 2 || invd[c] == 0.f) continue;
        double dev = 0.0;
        for (int mm = 1; mm < B; ++mm) {
            const double e = (double)m->edges[(size_t)c * (B - 1) + mm - 1];
            dev = std::max(dev, fabs((e - (double)lof[c]) / dl - (double)mm));
        }
        const double fd = dev + (double)(B + 2) * 2.4e-7 + 1e-6;
        if (fd < 0.5) fastd[c] = nextafterf((float)fd, 1.f);
    }
    std::vector<float> e = m->edges;
    if (e.empty()) e.push_back(0.f);
    HIP_TRY(upload(m, &m->d_edges, e.data(), e.size()));
    HIP_TRY(upload(m, &m->d_lo, lof.data(), lof.size()));
    HIP_TRY(upload(m, &m->d_invd, invd.data(), invd.size()));
    HIP_TRY(upload(m, &m->d_fastd, fastd.data(), fastd.size()));
    HIP_TRY(upload(m, &m->d_delta, m->delta.data(), m->delta.size()));
    return QFCA_OK;
}

// Fixed-point scale of the channel sums (see KArgs): the largest power of two
// s with s (B - 1) sum_c delta_c <= 2^62, so that the sum over channels of
// per-channel values v_c <= (B - 1) delta_c, each rounded to llrint(v_c s),
// stays below 2^63 with room for the float32 rounding of v_c.
double fixed_point_scale(const std::vector<double>& delta, int B) {
    double vmax = 0.0;
    for (double d : delta) vmax += d;
    vmax *= (double)std::max(B - 1, 0);
    if (!(vmax > 0.0) || !std::isfinite(vmax)) return 1.0;
    return ldexp(1.0, (int)floor(log2(ldexp(1.0, 62) / vmax)));
}

// Reference-dependent tables of the score kernel (see ScoreTables).
qfca_status upload_tables(qfca_model m) {
    const int C = planes(m->p), B = m->p.B, T = m->p.T;
    const int mm = T * T, Bp = m->Bp;
    std::vector<int2> psig((size_t)C * (mm + 1));
    std::vector<int32_t> cRm1((size_t)C * Bp, 0), Dm1((size_t)C * Bp, 0), cRl((size_t)C * Bp, 0);
    for (int c = 0; c < C; ++c) {
        const int32_t* cr = &m->cR[(size_t)c * B];
        int2* ps = &psig[(size_t)c * (mm + 1)];
        int kk = 0;  // #{k < B-1 : cR_k <= t}
        long long psi = 0;
        for (int t = 0; t <= mm; ++t) {
            while (kk < B - 1 && cr[kk] <= t) ++kk;
            ps[t] = make_int2((int)psi, kk);
            psi += kk;
        }
        for (int i = 0; i < Bp; ++i) {
            if (i >= 1 && i < B) {
                cRm1[(size_t)c * Bp + i] = cr[i - 1];
                Dm1[(size_t)c * Bp + i] = ps[cr[i - 1]].x;
            }
            if (i < B - 1) cRl[(size_t)c * Bp + i] = cr[i];
        }
    }
    std::vector<float> rcp(mm + 1);
    rcp[0] = 0.f;
    for (int t = 1; t <= mm; ++t) rcp[t] = (float)(1.0 / (double)t);
    HIP_TRY(upload(m, &m->tab.psig, psig.data(), psig.size()));
    HIP_TRY(upload(m, &m->tab.cRm1, cRm1.data(), cRm1.size()));
    HIP_TRY(upload(m, &m->tab.Dm1, Dm1.data(), Dm1.size()));
    HIP_TRY(upload(m, &m->tab.cRl, cRl.data(), cRl.size()));
    HIP_TRY(upload(m, &m->tab.rcp, rcp.data(), rcp.size()));
    HIP_TRY(upload(m, &m->d_cR, m->cR.data(), m->cR.size()));
    m->tab.delta = m->d_delta;
    m->tab.Bp = Bp;
    m->tab.fxs = fixed_point_scale(m->delta, B);
    m->tab.cRw = nullptr;
    m->cRw.assign(m->cR.begin(), m->cR.end());
    m->ref_general = false;
    m->has_ref = true;
    return QFCA_OK;
}

// Sets the reference from cumulative weights (validated by the caller):
// integer weights of mass T*T go to the integer tables, any other reference
// to the column-walk kernel's double weights.
qfca_status set_reference_weights(qfca_model m, const double* cRw) {
    const int C = planes(m->p), B = m->p.B, mm = m->p.T * m->p.T;
    bool integral = true;
    for (size_t i = 0; i < (size_t)C * B && integral; ++i)
        integral = cRw[i] == floor(cRw[i]) && cRw[i] <= (double)mm;
    for (int c = 0; c < C && integral; ++c) integral = cRw[(size_t)c * B + B - 1] == (double)mm;
    if (integral) {
        m->cR.assign((size_t)C * B, 0);
        for (size_t i = 0; i < m->cR.size(); ++i) m->cR[i] = (int32_t)cRw[i];
        return upload_tables(m);
    }
    // the scaled masses P M_R and R n_p must stay exact in double
    for (int c = 0; c < C; ++c)
        if (cRw[(size_t)c * B + B - 1] * (double)mm > 1e15)
            return fail(QFCA_E_UNSUPPORTED, "reference mass too large");
    m->cRw.assign(cRw, cRw + (size_t)C * B);
    m->cR.clear();
    HIP_TRY(upload(m, &m->tab.cRw, m->cRw.data(), m->cRw.size()));
    m->tab.delta = m->d_delta;
    m->tab.Bp = m->Bp;
    m->tab.fxs = fixed_point_scale(m->delta, B);
    m->ref_general = true;
    m->has_ref = true;
    return QFCA_OK;
}

// Association weights w(d) = exp(-d^2 / (2 sigma_p^2)), d = -r .. r, of a
// finite sigma_p (float32, one table per model).
qfca_status upload_assoc_weights(qfca_model m) {
    m->tab.wgt = nullptr;
    if (std::isinf(m->p.sigma_p)) return QFCA_OK;
    const int T = m->p.T, r = T / 2;
    const double sp = (double)m->p.sigma_p;
    std::vector<float> w(T);
    for (int i = 0; i < T; ++i) w[i] = (float)exp(-(double)((i - r) * (i - r)) / (2.0 * sp * sp));
    HIP_TRY(upload(m, &m->tab.wgt, w.data(), w.size()));
    return QFCA_OK;
}

qfca_model new_model(qfca_ctx ctx, const qfca_params* p) {
    qfca_model m = new (std::nothrow) qfca_model_s();
    if (!m) return nullptr;
    m->p = *p;
    m->device = ctx->device;
    m->m = p->T * p->T;
    m->Bp = pow2_at_least(p->B, 8);
    return m;
}

hipEvent_t take_event(qfca_ctx ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records events around one kernel launch when profiling is on.
struct KernelTimer {
    qfca_ctx ctx;
    int kernel;
    hipEvent_t a = nullptr, b = nullptr;
    KernelTimer(qfca_ctx c, int k) : ctx(c), kernel(k) {
        if (ctx->profile_mask & (1u << kernel)) {
            a = take_event(ctx);
            b = take_event(ctx);
            if (a) (void)hipEventRecord(a, ctx->stream);
        }
    }
    ~KernelTimer() {
        if (a && b) {
            (void)hipEventRecord(b, ctx->stream);
            ctx->timed[kernel].push_back({a, b});
        } else {
            if (a) ctx->event_pool.push_back(a);
            if (b) ctx->event_pool.push_back(b);
        }
    }
};

// Compute units of the context's device (read once).
int device_cus(qfca_ctx ctx) {
    if (!ctx->ncu) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return 0;
        ctx->ncu = prop.multiProcessorCount;
        ctx->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
    }
    return ctx->ncu;
}

ScoreTile choose_tile(qfca_ctx ctx, int C, int H, int W, int T, int B, int Bp) {
    auto tn = ctx->tuned.find((long long)T * 128 + B);
    if (tn != ctx->tuned.end()) return tn->second;
    const long long key =
        ((((long long)T * 128 + B) * 4096 + std::min(W, 4095)) * 4096 + std::min(H, 4095)) * 8192 + std::min(C, 8191);
    auto it = ctx->tiles.find(key);
    if (it != ctx->tiles.end()) return it->second;
    ScoreTile t;
    t.S = 64 / Bp;
    t.variant = score_has_block_kernel(T) ? 1 : 0;
    if (t.variant) t.S = std::min(t.S, score_block_max_S(T));
    // block walk: strips of 3 T columns (a multiple of T, so that blocks sit
    // at the same image columns in every strip; 3T + 2r patch columns fill
    // four blocks of T but one)
    t.Ws = t.variant ? 3 * T : 64;
    t.Hb = 128;
    // prefer at most 64 KiB per wavefront (occupancy); very large windows may
    // use up to the 160 KiB of a compute unit
    while (score_lds_bytes(T, Bp, t.S, t.Ws, t.variant) > 65536 && t.S > 1) t.S >>= 1;
    while (score_lds_bytes(T, Bp, t.S, t.Ws, t.variant) > 65536 && t.Ws > 8)
        t.Ws = t.variant ? (t.Ws > T ? t.Ws - T : 8) : t.Ws >> 1;
    if (t.variant == 1 && t.Ws < T) t.variant = 0;  // the block walk needs strips of at least T columns
    if (t.variant == 1) {
        // Bands: the tallest (least halo: a band walks 2r rows beyond its own)
        // that still gives at least three tiles per SIMD, so that the
        // dispatcher can even out the SIMDs' loads (with one or two long
        // tiles per SIMD, some SIMDs run one wavefront and others two)
        const long long nsimd = 4LL * std::max(1, device_cus(ctx));
        const long long cols = (long long)((W + t.Ws - 1) / t.Ws) * ((C + t.S - 1) / t.S);
        t.Hb = 32;
        for (int hb : {256, 192, 128, 96, 64, 48}) {
            if (cols * ((H + hb - 1) / hb) >= 3 * nsimd) {
                t.Hb = hb;
                break;
            }
        }
    }
    ctx->tiles[key] = t;
    return t;
}

}  // namespace

// The score launch sequence of qfca_score_map on caller-given fixed-point
// buffers asum [H][W] (and w1sum [H][W] when w1 is wanted): zero them, score
// tiles, channel mean and blur.  Arguments checked by score_map_check.
qfca_status qfca::score_map_into(qfca_ctx ctx, qfca_model m, const uint8_t* bins, int32_t H, int32_t W,
                                 float* score, float* amap, float* w1, float* achan, long long* asum,
                                 long long* w1sum, int* dbg_cp, int* dbg_I) {
    const bool coords = m->p.preproc == QFCA_PRE_COORDS;
    ScoreLaunch L;
    L.dbg_cp = dbg_cp; L.dbg_I = dbg_I;
    L.bins = bins; L.C = planes(m->p); L.H = H; L.W = W; L.T = m->p.T; L.B = m->p.B;
    L.tab = m->tab;
    L.fxs = m->tab.fxs;
    if (coords) {
        // principal coordinates: window W1 of every window into asum, its box
        // mean into amap (or the w1sum buffer used as float scratch), blur
        if (achan) return fail(QFCA_E_UNSUPPORTED, "principal-coordinate models have no per-channel maps");
        if (!amap && !w1sum) return fail(QFCA_E_ARG, "internal: no scratch for the box-mean map");
        L.asum = asum; L.w1sum = asum; L.achan = nullptr; L.w1only = true;
    } else {
        L.asum = asum; L.w1sum = w1 ? w1sum : nullptr; L.achan = achan;
    }
    if (ctx->tile_override.Ws > 0) {
        L.tile = ctx->tile_override;
        if (L.tile.S * m->Bp > 64) return fail(QFCA_E_UNSUPPORTED, "S * lanes per channel exceeds 64");
        if (L.tile.variant == 1 && (!score_has_block_kernel(m->p.T) || L.tile.S > score_block_max_S(m->p.T) ||
                                    L.tile.Ws < m->p.T))
            L.tile.variant = 0;
        if (score_lds_bytes(m->p.T, m->Bp, L.tile.S, L.tile.Ws, L.tile.variant) > 160 * 1024)
            return fail(QFCA_E_UNSUPPORTED, "tile does not fit in LDS");
    } else {
        L.tile = choose_tile(ctx, L.C, H, W, m->p.T, m->p.B, m->Bp);
        // the window-W1 walk has no halo rows: bands of 16 rows cost nothing
        // extra and give the few coordinate planes enough tiles
        if (coords) L.tile.Hb = 16;
    }
    if (dbg_cp && L.tile.variant != 1)
        return fail(QFCA_E_UNSUPPORTED, "window inspection needs the block walk (T in 3..31, S within its limit)");
    {
        KernelTimer kt(ctx, K_SCORE);
        HIP_TRY(launch_score(L, ctx->stream));
    }
    {
        KernelTimer kt(ctx, K_FINISH);
        const double inv = 1.0 / (m->tab.fxs * (double)L.C);
        if (coords)
            HIP_TRY(launch_finish_w1(asum, inv, H, W, m->p.T, m->p.sigma_s, amap ? amap : (float*)w1sum, w1, score,
                                     ctx->stream));
        else
            HIP_TRY(launch_finish(asum, L.w1sum, inv, H, W, m->p.sigma_s, amap, w1, score, ctx->stream));
    }
    return QFCA_OK;
}

qfca_status qfca::score_map_check(qfca_ctx ctx, qfca_model m, const uint8_t* bins, int32_t H, int32_t W,
                                  const float* score) {
    if (!ctx || !m || !bins || !score) return fail(QFCA_E_ARG, "NULL argument");
    qfca_status st = check_shape(H, W, m->p.C);
    if (st != QFCA_OK) return st;
    if (!m->has_ref) return fail(QFCA_E_STATE, "model has no reference");
    if (m->device != ctx->device) return fail(QFCA_E_ARG, "model and context are on different devices");
    HIP_TRY(hipSetDevice(ctx->device));
    return QFCA_OK;
}

int qfca::ctx_device(qfca_ctx ctx) { return ctx->device; }

qfca_status qfca::status_fail(qfca_status s, const std::string& msg) { return fail(s, msg); }

namespace {


}  // namespace

// ---------------------------------------------------------------------------

extern "C" {

const char* qfca_status_str(qfca_status s) {
    switch (s) {
        case QFCA_OK: return "ok";
        case QFCA_E_ARG: return "invalid argument";
        case QFCA_E_SHAPE: return "invalid shape";
        case QFCA_E_NOMEM: return "out of memory";
        case QFCA_E_DEVICE: return "device error";
        case QFCA_E_STATE: return "invalid state";
        case QFCA_E_NONFINITE: return "non-finite input";
        case QFCA_E_UNSUPPORTED: return "unsupported parameters";
    }
    return "unknown status";
}

const char* qfca_last_error(void) { return g_err.c_str(); }

int32_t qfca_version(void) { return 100; }

qfca_status qfca_ctx_create(int32_t device, void* hip_stream, qfca_ctx* out) {
    if (!out) return fail(QFCA_E_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(QFCA_E_ARG, "no such device");
    HIP_TRY(hipSetDevice(device));
    qfca_ctx c = new (std::nothrow) qfca_ctx_s();
    if (!c) return fail(QFCA_E_NOMEM, "context allocation failed");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    // the device address of this device's allocation-free scratch (once per device)
    const hipError_t e = noalloc_init(device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipGetSymbolAddress (scratch)");
    }
    *out = c;
    return QFCA_OK;
}

qfca_status qfca_ctx_set_stream(qfca_ctx ctx, void* hip_stream) {
    if (!ctx) return fail(QFCA_E_ARG, "ctx is NULL");
    ctx->stream = (hipStream_t)hip_stream;
    return QFCA_OK;
}

qfca_status qfca_ctx_set_tile(qfca_ctx ctx, int32_t Ws, int32_t Hb, int32_t S, int32_t variant) {
    if (!ctx) return fail(QFCA_E_ARG, "ctx is NULL");
    if (Ws == 0) {
        ctx->tile_override = ScoreTile();
        ctx->tile_override.Ws = 0;
        return QFCA_OK;
    }
    if (Ws < 1 || Ws > 1024 || Hb < 1 || S < 1 || S > 64 || (variant != 0 && variant != 1))
        return fail(QFCA_E_ARG, "bad tile");
    ctx->tile_override.Ws = Ws;
    ctx->tile_override.Hb = Hb;
    ctx->tile_override.S = S;
    ctx->tile_override.variant = variant;
    return QFCA_OK;
}

qfca_status qfca_ctx_profile(qfca_ctx ctx, int32_t enable) {
    if (!ctx) return fail(QFCA_E_ARG, "ctx is NULL");
    ctx->profile_mask = (uint32_t)enable;
    return QFCA_OK;
}

qfca_status qfca_ctx_profile_read(qfca_ctx ctx, int32_t kernel, double* total_ms, int64_t* launches) {
    if (!ctx || !total_ms || !launches) return fail(QFCA_E_ARG, "NULL argument");
    if (kernel < 0 || kernel >= K_COUNT) return fail(QFCA_E_ARG, "unknown kernel id");
    HIP_TRY(hipSetDevice(ctx->device));
    double tot = 0.0;
    int64_t n = 0;
    for (auto& pr : ctx->timed[kernel]) {
        HIP_TRY(hipEventSynchronize(pr.second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
        tot += ms;
        ++n;
        ctx->event_pool.push_back(pr.first);
        ctx->event_pool.push_back(pr.second);
    }
    ctx->timed[kernel].clear();
    *total_ms = tot;
    *launches = n;
    return QFCA_OK;
}

qfca_status qfca_ctx_destroy(qfca_ctx ctx) {
    if (!ctx) return QFCA_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& g : ctx->graphs) {
        if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
        if (g.second.graph) (void)hipGraphDestroy(g.second.graph);
    }
    if (ctx->d_hdr) (void)hipFree(ctx->d_hdr);
    if (ctx->d_jobs) (void)hipFree(ctx->d_jobs);
    if (ctx->h_hdr) (void)hipHostFree(ctx->h_hdr);
    if (ctx->h_jobs) (void)hipHostFree(ctx->h_jobs);
    if (ctx->staged) (void)hipEventDestroy(ctx->staged);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    for (auto& v : ctx->timed)
        for (auto& pr : v) ctx->event_pool.push_back(pr.first), ctx->event_pool.push_back(pr.second);
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    for (auto& b : ctx->scratch)
        if (b.p) (void)hipFree(b.p);
    delete ctx;
    return QFCA_OK;
}

qfca_status qfca_model_destroy(qfca_model m) {
    if (!m) return QFCA_OK;
    (void)hipSetDevice(m->device);
    delete m;  // hipFree of its arrays waits for the device (see qfca.h)
    return QFCA_OK;
}

qfca_status qfca_model_params(qfca_model m, qfca_params* out) {
    if (!m || !out) return fail(QFCA_E_ARG, "NULL argument");
    *out = m->p;
    return QFCA_OK;
}

qfca_status qfca_model_read(qfca_model m, int32_t field, void* dst, size_t bytes) {
    if (!m || !dst) return fail(QFCA_E_ARG, "NULL argument");
    const int C = m->p.C, k = m->p.k, B = m->p.B, P = planes(m->p);
    std::vector<float> tmp;
    const void* src = nullptr;
    size_t need = 0;
    bool ok = true;
    switch (field) {
        case 0:
            tmp.resize(C);
            for (int c = 0; c < C; ++c) tmp[c] = m->mu.empty() ? 0.f : (float)m->mu[c];
            src = tmp.data(); need = (size_t)C * 4; break;
        case 1:
            tmp.resize((size_t)C * k);
            ok = m->p.preproc != QFCA_PRE_NONE && m->V.size() == tmp.size();
            for (size_t i = 0; ok && i < tmp.size(); ++i) tmp[i] = (float)m->V[i];
            src = tmp.data(); need = tmp.size() * 4; break;
        case 2: src = m->edges.data(); need = (size_t)P * (B - 1) * 4; break;
        case 3: src = m->delta.data(); need = (size_t)P * 8; break;
        case 4: ok = m->has_ref && !m->ref_general; src = m->cR.data(); need = (size_t)P * B * 4; break;
        case 8: ok = m->has_ref; src = m->cRw.data(); need = (size_t)P * B * 8; break;
        case 5: ok = m->has_evals; src = m->evals.data(); need = (size_t)C * 8; break;
        case 6: ok = m->has_lohi; src = m->lo.data(); need = (size_t)P * 8; break;
        case 7: ok = m->has_lohi; src = m->hi.data(); need = (size_t)P * 8; break;
        default: return fail(QFCA_E_ARG, "unknown field");
    }
    if (!ok) return fail(QFCA_E_STATE, "field not set on this model");
    if (bytes != need) return fail(QFCA_E_ARG, "byte count does not match the field size");
    if (need) memcpy(dst, src, need);
    return QFCA_OK;
}

}  // extern "C"

namespace {

// Builds a model from host arrays (mu and V in double precision); lo, when
// given, is taken as is (a fitted or exported model), otherwise derived from
// the first edge.  Validates everything before any allocation.
qfca_status build_model(qfca_ctx ctx, const qfca_params* p, const double* mu, const double* V,
                        const float* edges, const double* delta, const int32_t* cR, const double* lo,
                        qfca_model* out) {
    if (!ctx || !out) return fail(QFCA_E_ARG, "NULL argument");
    *out = nullptr;
    qfca_status st = check_params(p);
    if (st != QFCA_OK) return st;
    const int C = p->C, k = p->k, B = p->B, T = p->T, P = planes(*p);
    const bool pre = p->preproc != QFCA_PRE_NONE;
    if (pre && k > 0 && (!mu || !V)) return fail(QFCA_E_ARG, "mu and V are required for k > 0");
    {
        std::string err;
        if ((st = host_check_arrays(*p, edges, delta, cR, &err)) != QFCA_OK) return fail(st, err);
    }
    (void)T;
    HIP_TRY(hipSetDevice(ctx->device));
    std::unique_ptr<qfca_model_s> m(new_model(ctx, p));
    if (!m) return fail(QFCA_E_NOMEM, "model allocation failed");
    m->mu.assign(C, 0.0);
    if (pre) {
        if (mu)
            for (int c = 0; c < C; ++c) m->mu[c] = mu[c];
        m->V.assign((size_t)C * k, 0.0);
        for (size_t i = 0; i < m->V.size(); ++i) m->V[i] = V[i];
    }
    if (B > 1) m->edges.assign(edges, edges + (size_t)P * (B - 1));
    m->delta.assign(delta, delta + P);
    m->lo.assign(P, 0.0);
    for (int c = 0; c < P; ++c)
        m->lo[c] = lo ? lo[c]
                      : ((B > 1 && m->delta[c] > 0.0) ? (double)m->edges[(size_t)c * (B - 1)] - m->delta[c] : 0.0);
    if ((st = upload_projection(m.get())) != QFCA_OK) return st;
    if ((st = upload_quant(m.get())) != QFCA_OK) return st;
    if ((st = upload_assoc_weights(m.get())) != QFCA_OK) return st;
    if (cR) {
        m->cR.assign(cR, cR + (size_t)P * B);
        if ((st = upload_tables(m.get())) != QFCA_OK) return st;
    }
    *out = m.release();
    return QFCA_OK;
}

// The serialised model format is described in qfca_blob.h.

}  // namespace

extern "C" {

qfca_status qfca_model_create(qfca_ctx ctx, const qfca_params* p, const float* mu, const float* V,
                              const float* edges, const double* delta, const int32_t* cR,
                              qfca_model* out) {
    if (!p) return fail(QFCA_E_ARG, "NULL argument");
    std::vector<double> mud, Vd;
    if (mu && p->C > 0) mud.assign(mu, mu + p->C);
    if (V && p->C > 0 && p->k > 0) Vd.assign(V, V + (size_t)p->C * p->k);
    return build_model(ctx, p, mu ? mud.data() : nullptr, V ? Vd.data() : nullptr, edges, delta, cR, nullptr,
                       out);
}

qfca_status qfca_model_export(qfca_model m, void* host_buf, size_t* inout_bytes) {
    if (!m || !inout_bytes) return fail(QFCA_E_ARG, "NULL argument");
    const uint32_t flags = ((m->has_ref && !m->ref_general) ? 1u : 0u) | (m->has_evals ? 2u : 0u) |
                           (m->has_lohi ? 4u : 0u) | ((m->has_ref && m->ref_general) ? 8u : 0u);
    const size_t total = blob_bytes(m->p, flags);
    if (!host_buf) {
        *inout_bytes = total;
        return QFCA_OK;
    }
    if (*inout_bytes < total) {
        *inout_bytes = total;
        return fail(QFCA_E_ARG, "buffer smaller than the serialised model");
    }
    ModelArrays a;
    a.p = m->p;
    a.flags = flags;
    a.mu.assign(m->p.C, 0.0);
    for (int c = 0; c < m->p.C && c < (int)m->mu.size(); ++c) a.mu[c] = m->mu[c];
    a.V = m->V;
    a.edges = m->edges;
    a.delta = m->delta;
    if (flags & 1u) a.cR = m->cR;
    if (flags & 2u) a.evals = m->evals;
    if (flags & 4u) {
        a.lo = m->lo;
        a.hi = m->hi;
    }
    if (flags & 8u) a.cRw = m->cRw;
    blob_write(a, (unsigned char*)host_buf);
    *inout_bytes = total;
    return QFCA_OK;
}

qfca_status qfca_model_import(qfca_ctx ctx, const void* host_buf, size_t bytes, qfca_model* out) {
    if (!ctx || !host_buf || !out) return fail(QFCA_E_ARG, "NULL argument");
    *out = nullptr;
    ModelArrays a;
    {
        std::string err;
        const qfca_status st = blob_read(host_buf, bytes, &a, &err);
        if (st != QFCA_OK) return fail(st, err);
    }
    const bool pca = a.p.preproc != QFCA_PRE_NONE;
    qfca_model m = nullptr;
    qfca_status st = build_model(ctx, &a.p, a.mu.data(), pca ? a.V.data() : nullptr,
                                 a.edges.empty() ? nullptr : a.edges.data(), a.delta.data(),
                                 a.cR.empty() ? nullptr : a.cR.data(), a.lo.empty() ? nullptr : a.lo.data(), &m);
    if (st != QFCA_OK) return st;
    if (a.flags & 2u) {
        m->evals = a.evals;
        m->has_evals = true;
    }
    if (a.flags & 4u) {
        m->hi = a.hi;
        m->has_lohi = true;
    }
    if (a.flags & 8u) {
        if ((st = set_reference_weights(m, a.cRw.data())) != QFCA_OK) {
            delete m;
            return st;
        }
    }
    *out = m;
    return QFCA_OK;
}

qfca_status qfca_quantize(qfca_ctx ctx, qfca_model m, const float* X, int32_t H, int32_t W,
                          uint8_t* bins, float* resid) {
    if (!ctx || !m || !X || (!bins && !resid)) return fail(QFCA_E_ARG, "NULL argument");
    qfca_status st = check_shape(H, W, m->p.C);
    if (st != QFCA_OK) return st;
    if (m->device != ctx->device) return fail(QFCA_E_ARG, "model and context are on different devices");
    HIP_TRY(hipSetDevice(ctx->device));
    ProjLaunch L;
    L.X = X; L.C = m->p.C; L.N = H * W; L.k = m->p.k; L.B = m->p.B;
    L.preproc = m->p.preproc; L.prec = m->p.proj_prec;
    L.mu = m->d_mu; L.V = m->d_V; L.Vbf = m->d_Vbf; L.edges = m->d_edges; L.lo = m->d_lo;
    L.inv_delta = m->d_invd; L.fastd = m->d_fastd; L.bins = bins; L.resid = resid;
    L.V1 = m->d_V1; L.V2 = m->d_V2;
    KernelTimer kt(ctx, K_PROJ);
    if (m->p.preproc == QFCA_PRE_COORDS) {
        if (!m->d_V1) return fail(QFCA_E_UNSUPPORTED, "principal coordinates need C <= 512");
        HIP_TRY(launch_coords(L, ctx->stream));
    } else {
        HIP_TRY(launch_proj(L, ctx->stream));
    }
    return QFCA_OK;
}

qfca_status qfca_fit_reference(qfca_ctx ctx, qfca_model m, const uint8_t* bins, int32_t H, int32_t W) {
    if (!ctx || !m || !bins) return fail(QFCA_E_ARG, "NULL argument");
    qfca_status st = check_shape(H, W, m->p.C);
    if (st != QFCA_OK) return st;
    const int C = planes(m->p), B = m->p.B, T = m->p.T, mm = T * T;
    if (H < T || W < T) return fail(QFCA_E_SHAPE, "the reference needs H, W >= T");
    if (m->p.reference == QFCA_REF_MEAN_QUAN)
        return fail(QFCA_E_UNSUPPORTED, "the mean -> quan reference needs the features: use qfca_fit_pca");
    HIP_TRY(hipSetDevice(ctx->device));
    uint32_t* counts = nullptr;
    HIP_TRY(scratch(ctx, SL_COUNTS, (size_t)C * B * (mm + 1) * 4, &counts));
    const long long P = (long long)(H - T + 1) * (W - T + 1);
    if (m->p.reference == QFCA_REF_QUAN_MEDIAN || m->p.reference == QFCA_REF_QUAN_MEAN) {
        // bin-wise statistics of the full windows' bin counts (Tab. 3)
        double* dw = nullptr;
        HIP_TRY(scratch(ctx, SL_CRW, (size_t)C * B * 8, &dw));
        HIP_TRY(launch_refcount(bins, C, H, W, T, B, counts, ctx->stream, 1));
        HIP_TRY(launch_refstat(counts, C, B, mm, P, m->p.reference == QFCA_REF_QUAN_MEDIAN ? 0 : 1, dw,
                               ctx->stream));
        std::vector<double> w((size_t)C * B);
        HIP_TRY(hipMemcpyAsync(w.data(), dw, w.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        return set_reference_weights(m, w.data());
    }
    int32_t* dcR = nullptr;
    HIP_TRY(scratch(ctx, SL_CR, (size_t)C * B * 4, &dcR));
    HIP_TRY(launch_refmedian(bins, C, H, W, T, B, counts, (P + 1) / 2, dcR, ctx->stream));
    m->cR.assign((size_t)C * B, 0);
    HIP_TRY(hipMemcpyAsync(m->cR.data(), dcR, (size_t)C * B * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return upload_tables(m);
}

qfca_status qfca_model_set_reference(qfca_ctx ctx, qfca_model m, const double* cRw) {
    if (!ctx || !m || !cRw) return fail(QFCA_E_ARG, "NULL argument");
    if (m->device != ctx->device) return fail(QFCA_E_ARG, "model and context are on different devices");
    const int C = planes(m->p), B = m->p.B;
    for (int c = 0; c < C; ++c)
        for (int i = 0; i < B; ++i) {
            const double v = cRw[(size_t)c * B + i];
            if (!std::isfinite(v) || v < 0.0 || (i > 0 && v < cRw[(size_t)c * B + i - 1]))
                return fail(QFCA_E_ARG, "reference weights must be finite, >= 0 and nondecreasing");
        }
    HIP_TRY(hipSetDevice(ctx->device));
    return set_reference_weights(m, cRw);
}

qfca_status qfca_fit_pca(qfca_ctx ctx, const qfca_params* p, const float* X, int32_t H, int32_t W,
                         qfca_model* out) {
    if (!ctx || !X || !out) return fail(QFCA_E_ARG, "NULL argument");
    *out = nullptr;
    qfca_status st = check_params(p);
    if (st != QFCA_OK) return st;
    if ((st = check_shape(H, W, p->C)) != QFCA_OK) return st;
    if (H < p->T || W < p->T) return fail(QFCA_E_SHAPE, "the fit needs H, W >= T");
    HIP_TRY(hipSetDevice(ctx->device));
    const int C = p->C, k = p->k, B = p->B, P = planes(*p);
    const long N = (long)H * W;
    const bool pre = p->preproc != QFCA_PRE_NONE;
    const bool coords = p->preproc == QFCA_PRE_COORDS;
    std::unique_ptr<qfca_model_s> m(new_model(ctx, p));
    if (!m) return fail(QFCA_E_NOMEM, "model allocation failed");
    hipStream_t s = ctx->stream;

    // 1. mean (also the finiteness check) and covariance, FP64 on the GPU
    double* dmu = nullptr;
    HIP_TRY(scratch(ctx, SL_MU, (size_t)C * 8, &dmu));
    HIP_TRY(launch_mean(X, C, N, dmu, s));
    // the covariance is queued behind the mean before either comes back (a
    // copy to pageable memory may wait for the stream); the features'
    // finiteness (a non-finite mean) is checked once both are back
    std::vector<double> cov;
    double* dcov = nullptr;
    if (pre) {
        cov.resize((size_t)C * C);
        HIP_TRY(scratch(ctx, SL_COV, (size_t)C * C * 8, &dcov));
        HIP_TRY(launch_cov(X, C, N, dmu, dcov, s));
    }
    m->mu.assign(C, 0.0);
    HIP_TRY(hipMemcpyAsync(m->mu.data(), dmu, (size_t)C * 8, hipMemcpyDeviceToHost, s));
    if (pre) HIP_TRY(hipMemcpyAsync(cov.data(), dcov, cov.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int c = 0; c < C; ++c)
        if (!isfinite(m->mu[c])) return fail(QFCA_E_NONFINITE, "non-finite value in the features");
    if (pre) {
        std::vector<double> vecs((size_t)C * k);
        m->evals.assign(C, 0.0);
        // 2. eigenvectors of the k largest eigenvalues (host, FP64)
        if (sym_eig_top(cov.data(), C, k, m->evals.data(), vecs.data()) != 0)
            return fail(QFCA_E_DEVICE, "eigensolver did not converge");
        m->has_evals = true;
        m->V = vecs;  // [C][k], column j the eigenvector of the j-th largest eigenvalue
    } else {
        std::fill(m->mu.begin(), m->mu.end(), 0.0);
    }
    if ((st = upload_projection(m.get())) != QFCA_OK) return st;

    // 3. residual and its per-channel type-7 quantiles (exact order statistics)
    float* resid = nullptr;
    HIP_TRY(scratch(ctx, SL_RESID, (size_t)C * N * 4, &resid));
    {
        ProjLaunch L;
        L.X = X; L.C = C; L.N = (int)N; L.k = k; L.B = B; L.preproc = p->preproc;
        L.prec = p->proj_prec; L.mu = m->d_mu; L.V = m->d_V; L.Vbf = m->d_Vbf;
        L.edges = nullptr; L.lo = nullptr; L.inv_delta = nullptr; L.fastd = nullptr; L.bins = nullptr;
        L.resid = resid;
        L.V1 = m->d_V1; L.V2 = m->d_V2;
        if (coords) {
            if (!m->d_V1) return fail(QFCA_E_UNSUPPORTED, "principal coordinates need C <= 512");
            HIP_TRY(launch_coords(L, s));  // the k coordinates z into resid [k][N]
        } else {
            HIP_TRY(launch_proj(L, s));
        }
    }
    const double hq[2] = {(double)(N - 1) * (double)p->q_lo, (double)(N - 1) * (double)p->q_hi};
    long long ranks[4];
    for (int q = 0; q < 2; ++q) {
        const long long f = (long long)floor(hq[q]);
        ranks[2 * q] = f;
        ranks[2 * q + 1] = std::min<long long>(f + 1, N - 1);
    }
    long long* dranks = nullptr;
    float* dsel = nullptr;
    HIP_TRY(scratch(ctx, SL_RANKS, sizeof(ranks), &dranks));
    HIP_TRY(scratch(ctx, SL_SEL, (size_t)P * 4 * 4, &dsel));
    HIP_TRY(hipMemcpyAsync(dranks, ranks, sizeof(ranks), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_select(resid, P, N, dranks, 4, dsel, s));
    std::vector<float> sel((size_t)P * 4);
    HIP_TRY(hipMemcpyAsync(sel.data(), dsel, sel.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    m->lo.assign(P, 0.0);
    m->hi.assign(P, 0.0);
    m->delta.assign(P, 0.0);
    m->edges.assign((size_t)P * (B - 1), 0.f);
    for (int c = 0; c < P; ++c) {
        double qv[2];
        for (int q = 0; q < 2; ++q) {
            const double a = sel[(size_t)c * 4 + 2 * q], b = sel[(size_t)c * 4 + 2 * q + 1];
            const double f = floor(hq[q]);
            qv[q] = (ranks[2 * q] + 1 < N) ? a + (hq[q] - f) * (b - a) : a;
        }
        if (!isfinite(qv[0]) || !isfinite(qv[1])) return fail(QFCA_E_NONFINITE, "non-finite residual");
        m->lo[c] = qv[0];
        m->hi[c] = qv[1];
        if (!(qv[1] > qv[0])) {
            m->delta[c] = 0.0;
            for (int i = 1; i < B; ++i) m->edges[(size_t)c * (B - 1) + i - 1] = INFINITY;
        } else {
            const double d = (qv[1] - qv[0]) / (double)B;
            m->delta[c] = d;
            for (int i = 1; i < B; ++i) m->edges[(size_t)c * (B - 1) + i - 1] = (float)(qv[0] + (double)i * d);
        }
    }
    m->has_lohi = true;
    if ((st = upload_quant(m.get())) != QFCA_OK) return st;

    if ((st = upload_assoc_weights(m.get())) != QFCA_OK) return st;

    // 4. bins with the final edges, then the reference
    uint8_t* bins = nullptr;
    HIP_TRY(scratch(ctx, SL_BINS, (size_t)P * N, &bins));
    if ((st = qfca_quantize(ctx, m.get(), X, H, W, bins, nullptr)) != QFCA_OK) return st;
    if (p->reference == QFCA_REF_MEAN_QUAN) {
        // rank-wise mean of the sorted full windows of the residual, quantised
        int nparts = 0, NP = 0;
        double* part = nullptr;
        int32_t* dcR = nullptr;
        HIP_TRY(scratch(ctx, SL_RMPART, refmean_part_bytes(P, p->T, &nparts, &NP), &part));
        HIP_TRY(scratch(ctx, SL_CR, (size_t)P * B * 4, &dcR));
        HIP_TRY(launch_refmean(resid, P, H, W, p->T, m->d_edges, B, part, dcR, s));
        m->cR.assign((size_t)P * B, 0);
        HIP_TRY(hipMemcpyAsync(m->cR.data(), dcR, (size_t)P * B * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if ((st = upload_tables(m.get())) != QFCA_OK) return st;
    } else if ((st = qfca_fit_reference(ctx, m.get(), bins, H, W)) != QFCA_OK) {
        return st;
    }
    *out = m.release();
    return QFCA_OK;
}

qfca_status qfca_inspect_windows(qfca_ctx ctx, qfca_model m, const uint8_t* bins, int32_t H, int32_t W,
                                 int32_t* cp, int32_t* I) {
    if (!ctx || !m || !bins || !cp || !I) return fail(QFCA_E_ARG, "NULL argument");
    qfca_status st = check_shape(H, W, m->p.C);
    if (st != QFCA_OK) return st;
    if (!m->has_ref) return fail(QFCA_E_STATE, "model has no reference");
    if (m->device != ctx->device) return fail(QFCA_E_ARG, "model and context are on different devices");
    if (!score_has_block_kernel(m->p.T) || m->ref_general || !std::isinf(m->p.sigma_p) ||
        m->p.preproc == QFCA_PRE_COORDS)
        return fail(QFCA_E_UNSUPPORTED, "window inspection needs T in 3..31, sigma_p = INFINITY and an integer "
                                        "reference of mass T*T");
    HIP_TRY(hipSetDevice(ctx->device));
    const size_t N = (size_t)H * W;
    long long* asum = nullptr;
    float* score = nullptr;
    HIP_TRY(scratch(ctx, SL_ASUM, N * 8, &asum));
    HIP_TRY(scratch(ctx, SL_SCORE, N * 4, &score));
    return score_map_into(ctx, m, bins, H, W, score, nullptr, nullptr, nullptr, asum, nullptr, cp, I);
}

qfca_status qfca_score_map(qfca_ctx ctx, qfca_model m, const uint8_t* bins, int32_t H, int32_t W,
                           float* score, float* amap, float* w1, float* achan) {
    qfca_status st = score_map_check(ctx, m, bins, H, W, score);
    if (st != QFCA_OK) return st;
    const size_t N = (size_t)H * W;
    long long* asum = nullptr;
    long long* w1sum = nullptr;
    HIP_TRY(scratch(ctx, SL_ASUM, N * 8, &asum));
    if (w1 || (m->p.preproc == QFCA_PRE_COORDS && !amap)) HIP_TRY(scratch(ctx, SL_W1SUM, N * 8, &w1sum));
    return score_map_into(ctx, m, bins, H, W, score, amap, w1, achan, asum, w1sum);
}

}  // extern "C"

namespace {

int batch_lanes(int B) { return pow2_at_least(B, 8); }

ScoreTile batch_tile(qfca_ctx ctx, const qfca_params& p) {
    const int Bp = batch_lanes(p.B);
    ScoreTile t = choose_tile(ctx, p.C, 256, 256, p.T, p.B, Bp);
    if (ctx->tile_override.Ws > 0) t = ctx->tile_override;
    t.variant = 1;
    t.Ws = score_block_ws(p.T, t.Ws);
    t.S = std::min(std::min(t.S, 64 / Bp), score_block_max_S(p.T));
    if (t.S < 1) t.S = 1;
    // four wavefront regions and the shared reciprocal table must fit in LDS:
    // narrow the strip one window width at a time (keeping whole blocks)
    while (batch_head_bytes(p.T) + 4 * align16c(batch_wave_lds(p.T, t.S, t.Ws)) > 160 * 1024 && t.Ws > p.T + 1)
        t.Ws -= p.T;
    return t;
}

}  // namespace

extern "C" {

qfca_status qfca_score_batch(qfca_ctx ctx, const qfca_job* jobs, int32_t n) {
    return score_batch_ext(ctx, jobs, n, nullptr, nullptr);
}

}  // extern "C"

qfca_status qfca::batch_job_check(qfca_ctx ctx, const qfca_job& J, const qfca_params& p) {
    if (!J.model || !J.X || !J.score) return fail(QFCA_E_ARG, "job with a NULL model, X or score");
    const qfca_params& q = J.model->p;
    if (q.C != p.C || q.k != p.k || q.B != p.B || q.T != p.T || q.preproc != p.preproc ||
        q.proj_prec != p.proj_prec || q.sigma_s != p.sigma_s || !(q.sigma_p == p.sigma_p))
        return fail(QFCA_E_ARG, "all jobs of a batch must share C, k, B, T, sigma_s, preproc, proj_prec");
    if (!J.model->has_ref) return fail(QFCA_E_STATE, "model without reference");
    if (J.model->ref_general || !std::isinf(q.sigma_p))
        return fail(QFCA_E_UNSUPPORTED, "batched path: needs sigma_p = INFINITY and an integer reference of mass T*T");
    if (J.model->device != ctx->device) return fail(QFCA_E_ARG, "model on another device");
    qfca_status st = check_shape(J.H, J.W, p.C);
    if (st != QFCA_OK) return st;
    int CM = 0, KT = 0;
    if (p.preproc != QFCA_PRE_RESIDUAL || !batch_combo(p.C, p.k, p.proj_prec, &CM, &KT) ||
        !batch_supported(p.T, CM, KT, p.proj_prec) || !J.model->d_V1b)
        return fail(QFCA_E_UNSUPPORTED, "batched path: needs the PCA residual, T odd in 3..31, C <= 512 and "
                                        "k in 1..64");
    return QFCA_OK;
}

qfca_status qfca::score_batch_ext(qfca_ctx ctx, const qfca_job* jobs, int32_t n, long long* const* asum_ext,
                                  int32_t* err_host) {
    if (!ctx || !jobs) return fail(QFCA_E_ARG, "NULL argument");
    if (n < 1 || n > BATCH_MAXJ) return fail(QFCA_E_ARG, "n must be in [1, 256]");
    const qfca_model m0 = jobs[0].model;
    if (!m0) return fail(QFCA_E_ARG, "job 0 has no model");
    const qfca_params p = m0->p;
    for (int i = 0; i < n; ++i) {
        qfca_status st = batch_job_check(ctx, jobs[i], p);
        if (st != QFCA_OK) return st;
        if (asum_ext && !asum_ext[i]) return fail(QFCA_E_ARG, "NULL channel-sum buffer");
    }
    int CM = 0, KT = 0;
    batch_combo(p.C, p.k, p.proj_prec, &CM, &KT);
    HIP_TRY(hipSetDevice(ctx->device));
    const ScoreTile tile = batch_tile(ctx, p);
    const int Bp = batch_lanes(p.B);
    const size_t wave_lds = align16c(batch_wave_lds(p.T, tile.S, tile.Ws));
    const size_t lds = batch_head_bytes(p.T) + std::max((size_t)4 * wave_lds, batch_proj_lds(CM, KT));
    if (lds > 160 * 1024) return fail(QFCA_E_UNSUPPORTED, "batch tile does not fit in LDS");

    // device + pinned staging buffers
    if (!ctx->d_hdr) {
        HIP_TRY(hipMalloc((void**)&ctx->d_hdr, sizeof(BatchHeader)));
        HIP_TRY(hipMalloc((void**)&ctx->d_jobs, sizeof(BatchJob) * BATCH_MAXJ));
        HIP_TRY(hipHostMalloc((void**)&ctx->h_hdr, sizeof(BatchHeader), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&ctx->h_jobs, sizeof(BatchJob) * BATCH_MAXJ, hipHostMallocDefault));
        HIP_TRY(hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming));
        HIP_TRY(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
    } else {
        HIP_TRY(hipEventSynchronize(ctx->staged));  // previous upload has left the staging buffers
    }
    // scratch for bins and the fixed-point channel sums
    size_t nb = 0, na = 0;
    for (int i = 0; i < n; ++i) {
        const size_t N = (size_t)jobs[i].H * jobs[i].W;
        if (!jobs[i].bins) nb += (size_t)p.C * N;
        if (!asum_ext) na += N;
    }
    uint8_t* sb = nullptr;
    long long* sa = nullptr;
    HIP_TRY(scratch(ctx, SL_BBINS, std::max<size_t>(nb, 1), &sb));
    HIP_TRY(scratch(ctx, SL_BASUM, std::max<size_t>(na, 1) * 8, &sa));
    BatchHeader& h = *ctx->h_hdr;
    memset(&h, 0, sizeof(h));
    h.n = n;
    const int S = tile.S;
    const int cgroups = (p.C + S - 1) / S;
    int np = 0, ns = 0;
    size_t ob = 0, oa = 0;
    for (int i = 0; i < n; ++i) {
        const qfca_job& J = jobs[i];
        const qfca_model m = J.model;
        BatchJob& b = ctx->h_jobs[i];
        memset(&b, 0, sizeof(b));
        const int N = J.H * J.W;
        uint8_t* bins = J.bins ? J.bins : sb + ob;
        if (!J.bins) ob += (size_t)p.C * N;
        long long* asum = asum_ext ? asum_ext[i] : sa + oa;
        if (!asum_ext) oa += (size_t)N;
        b.pa.X = J.X; b.pa.C = p.C; b.pa.N = N; b.pa.k = p.k; b.pa.B = p.B;
        b.pa.mu = m->d_mu; b.pa.V1 = m->d_V1b; b.pa.V2 = m->d_V2b; b.pa.edges = m->d_edges;
        b.pa.lo = m->d_lo; b.pa.inv_delta = m->d_invd; b.pa.fastd = m->d_fastd; b.pa.bins = bins;
        b.pa.resid = nullptr;
        b.pa.ntiles = (N + 15) / 16;
        b.sa.bins = bins; b.sa.C = p.C; b.sa.H = J.H; b.sa.W = J.W; b.sa.T = p.T; b.sa.B = p.B;
        b.sa.Bp = Bp; b.sa.S = S; b.sa.r = p.T / 2; b.sa.m = p.T * p.T; b.sa.Ws = tile.Ws;
        b.sa.Hb = tile.Hb; b.sa.WbA = tile.Ws + 4 * (p.T / 2);
        b.sa.psig = m->tab.psig; b.sa.cRm1 = m->tab.cRm1; b.sa.Dm1 = m->tab.Dm1; b.sa.cRl = m->tab.cRl;
        b.sa.rcp = m->tab.rcp; b.sa.delta = m->d_delta;
        b.sa.fxs = m->tab.fxs; b.sa.asum = asum; b.sa.w1sum = nullptr; b.sa.achan = J.achan;
        b.ntiles_proj = b.pa.ntiles;
        b.nstrips = (J.W + tile.Ws - 1) / tile.Ws;
        b.nbands = (J.H + tile.Hb - 1) / tile.Hb;
        b.asum = asum;
        b.inv_scale = 1.0 / (m->tab.fxs * (double)p.C);
        b.amap = J.amap;
        b.score = J.score;
        h.proj_prefix[i] = np;
        h.score_prefix[i] = ns;
        np += b.ntiles_proj;
        ns += b.nstrips * b.nbands * ((cgroups + 3) / 4);
    }
    h.proj_prefix[n] = np;
    h.score_prefix[n] = ns;
    h.nproj = np;
    h.nitems = np + ns;
    const float sig = p.sigma_s;
    h.blur_R = sig > 0.f ? (int)ceil(3.0 * (double)sig) : 0;
    for (int d = 0; d <= 16; ++d)
        h.blur_w[d] = (d <= h.blur_R) ? (sig > 0.f ? exp(-(double)(d * d) / (2.0 * (double)sig * sig)) : 1.0) : 0.0;
    HIP_TRY(hipMemcpyAsync(ctx->d_jobs, ctx->h_jobs, sizeof(BatchJob) * n, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->d_hdr, ctx->h_hdr, sizeof(BatchHeader), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipEventRecord(ctx->staged, ctx->stream));

    // grid: as many resident blocks as fit
    if (!device_cus(ctx)) return fail(QFCA_E_DEVICE, "cannot read the device properties");
    const int ncu = ctx->ncu;
    const int per_cu = std::min(2, std::max(1, (int)(ctx->lds_per_cu / std::max<size_t>(lds, 1))));
    const int grid = ncu * per_cu;
    int maxn = 1;
    while (maxn < n) maxn <<= 1;
    const long long key = ((((long long)p.T * 1024 + CM) * 8 + KT) * 2 + p.proj_prec) * 1000003LL +
                          ((long long)lds * 64 + maxn) * 4096 + grid;
    GraphEntry& ge = ctx->graphs[key];
    if (!ge.exec) {
        HIP_TRY(prepare_batch(p.T, CM, KT, p.proj_prec, lds));
        HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
        hipError_t le = launch_batch(p.T, CM, KT, p.proj_prec, ctx->d_hdr, ctx->d_jobs, (int)wave_lds, lds,
                                     grid, maxn, ctx->capture);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(ctx->capture, &g);
        if (le != hipSuccess) return hip_fail(le, "launch_batch (capture)");
        if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
        ge.graph = g;
        HIP_TRY(hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0));
    }
    {
        KernelTimer kt(ctx, K_SCORE);
        HIP_TRY(hipGraphLaunch(ge.exec, ctx->stream));
    }
    if (err_host)
        HIP_TRY(hipMemcpyAsync(err_host, &ctx->d_hdr->error, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    return QFCA_OK;
}

extern "C" {

qfca_status qfca_batch_error(qfca_ctx ctx, int32_t* failed) {
    if (!ctx || !failed) return fail(QFCA_E_ARG, "NULL argument");
    *failed = 0;
    if (!ctx->d_hdr) return QFCA_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    int v = 0;
    HIP_TRY(hipMemcpyAsync(&v, &ctx->d_hdr->error, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    *failed = v;
    return QFCA_OK;
}

qfca_status qfca_autotune(qfca_ctx ctx, const qfca_job* jobs, int32_t n, int32_t* best_Ws,
                          int32_t* best_Hb, double* best_ms) {
    if (!ctx || !jobs || n < 1 || !best_Ws || !best_Hb || !jobs[0].model) return fail(QFCA_E_ARG, "NULL argument");
    const qfca_params p = jobs[0].model->p;
    const int T = p.T, Bp = batch_lanes(p.B);
    // the tile override and the two events are restored and released on
    // every exit, including the early returns of HIP_TRY
    struct Guard {
        qfca_ctx ctx;
        ScoreTile saved;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Guard() {
            ctx->tile_override = saved;
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } g{ctx, ctx->tile_override};
    HIP_TRY(hipEventCreate(&g.e0));
    HIP_TRY(hipEventCreate(&g.e1));
    double best = 1e30;
    ScoreTile bt;
    bool found = false;
    for (int kmul = 2; kmul <= 8; ++kmul) {
        const int Ws = kmul * T;  // a multiple of T (see score_block_ws)
        if (Ws < 8 || Ws > 256) continue;
        for (int Hb : {64, 128, 256}) {
            ScoreTile t;
            t.Ws = Ws;
            t.Hb = Hb;
            t.variant = 1;
            t.S = std::min(64 / Bp, score_block_max_S(T));
            if (batch_head_bytes(T) + 4 * align16c(batch_wave_lds(T, t.S, t.Ws)) > 160 * 1024) continue;
            ctx->tile_override = t;
            qfca_status st = qfca_score_batch(ctx, jobs, n);  // warm-up (and graph capture)
            if (st != QFCA_OK) continue;
            HIP_TRY(hipEventRecord(g.e0, ctx->stream));
            for (int rep = 0; rep < 2; ++rep)
                if ((st = qfca_score_batch(ctx, jobs, n)) != QFCA_OK) break;
            HIP_TRY(hipEventRecord(g.e1, ctx->stream));
            HIP_TRY(hipEventSynchronize(g.e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, g.e0, g.e1));
            if (st == QFCA_OK && ms / 2 < best) {
                best = ms / 2;
                bt = t;
                found = true;
            }
        }
    }
    if (!found) return fail(QFCA_E_UNSUPPORTED, "no candidate tile ran");
    ctx->tuned[(long long)T * 128 + p.B] = bt;
    ctx->tiles.clear();
    *best_Ws = bt.Ws;
    *best_Hb = bt.Hb;
    if (best_ms) *best_ms = best;
    return QFCA_OK;
}

}  // extern "C"
