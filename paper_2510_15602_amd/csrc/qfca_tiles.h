// Device-side tile routines shared by the standalone kernels and the
// persistent batch kernel (internal header of libqfca).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qfca {
namespace tiles {

__device__ __forceinline__ int lane_prev(int v) {
    // Value held by lane-1 (DPP wave_shr:1); lane 0 receives 0.
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }


// Same computation as k_score with the window side T fixed at compile time,
// organised for instruction-level parallelism.  Per row of patch centres:
//   1. the vertical counts vc of every bin column are updated in place (one
//      pass, dword-wide; the counts of lane (s, j) for a T-column block are
//      T consecutive bytes padded to a multiple of 4);
//   2. the row is walked in blocks of T patch columns: the T counts of the
//      block are read, the running window sums formed in registers, and then
//      the T table reads, the T neighbour exchanges and the T reciprocal reads
//      are each issued together; the values leaving the running sums T
//      columns later (counts, per-bin errors) stay in register rings;
//   3. the horizontal window sums of the block's T output columns are written
//      to a small LDS buffer and gathered into the pending rows' accumulators
//      by all lanes at once, one (channel, column, pending row) triple per
//      lane.
template <int T>
struct BLayout {
    static constexpr int r = T / 2, m = T * T, T1 = T + 1, TP = (T + 3) & ~3;
    int nblk, rowb, vs4;
    size_t vc, ring, acc, hrow, psig, rcp, total;
    __host__ __device__ BLayout(int S, int Ws) {
        nblk = (Ws + 2 * r + T - 1) / T;  // blocks of patch columns
        rowb = (nblk + 1) * TP;           // bin columns [x0-2r, x0-2r+(nblk+1)T)
        vs4 = rowb / 4;
        if ((vs4 & 1) == 0) vs4 += 1;  // odd dword stride between lanes
        size_t off = 0;
        vc = off;   off += align16((size_t)64 * vs4 * 4);
        ring = off; off += align16((size_t)T1 * S * rowb);
        acc = off;  off += align16((size_t)T * S * Ws * 4 + 64 * 4);
        hrow = off; off += align16((size_t)T * 64 * 4);
        psig = off; off += align16((size_t)S * (m + 1) * 8);
        rcp = off;  off += align16((size_t)(m + 1) * 4);
        total = off;
    }
};

// One (strip bx, band by, channel group bz) tile, run by one wavefront whose
// lanes are `lane`, with its private LDS region `smem`.  Every wavefront of a
// block must run a tile of the same geometry (the barriers are block-wide).
template <int T>
__device__ __forceinline__ void score_tile(const KArgs& a, int bx, int by, int bz, int lane,
                                           unsigned char* smem) {
    using BL = BLayout<T>;
    constexpr int r = BL::r, m = BL::m, T1 = BL::T1, TP = BL::TP;
    const int Bp = a.Bp, S = a.S, H = a.H, W = a.W, Ws = a.Ws;
    const int s = lane / Bp;
    const int sa = s < S ? s : S - 1;
    const int j = lane - s * Bp;
    const int x0 = bx * Ws;
    const int xe = min(W, x0 + Ws);
    const int ws = xe - x0;
    const int y0 = by * a.Hb;
    const int ye = min(H, y0 + a.Hb);
    const int cbase = bz * S;
    const int c = cbase + s;
    const bool cval = (s < S) && (c < a.C);
    const int Wb = ws + 4 * r;  // used bin columns [x0-2r, xe+2r)
    const int xb0 = x0 - 2 * r;
    const BL L(S, Ws);
    const int np = ws + 2 * r;  // patch columns [x0-r, xe+r)
    const int nblk = (np + T - 1) / T;
    const int rowb = L.rowb;

    uint32_t* vc32 = (uint32_t*)(smem + L.vc);   // [64 lanes][vs4 dwords]
    uint8_t* vcl = (uint8_t*)(vc32 + lane * L.vs4);
    uint8_t* ring = smem + L.ring;               // [T1][S][rowb]
    float* acc = (float*)(smem + L.acc);         // [T][S][Ws] + 64 trash slots
    float* trash = acc + T * S * Ws;
    float* hrow = (float*)(smem + L.hrow);       // [T][64]
    int2* psig = (int2*)(smem + L.psig);
    float* rcp = (float*)(smem + L.rcp);

    for (int t = lane; t < S * (m + 1); t += 64) {
        const int ss = t / (m + 1), tt = t - ss * (m + 1);
        const int cc = cbase + ss;
        psig[t] = (cc < a.C) ? a.psig[(size_t)cc * (m + 1) + tt] : make_int2(0, 0);
    }
    for (int t = lane; t <= m; t += 64) rcp[t] = a.rcp[t];
    for (int t = lane; t < 64 * L.vs4; t += 64) vc32[t] = 0u;
    for (int t = lane; t < T * S * Ws + 64; t += 64) acc[t] = 0.f;
    const int ci = cval ? c : 0;
    const int crm1 = a.cRm1[ci * Bp + j];
    const int dm1 = a.Dm1[ci * Bp + j];
    const int crl = a.cRl[ci * Bp + j];
    const float binf = (cval && (j < a.B)) ? 1.f : 0.f;
    const bool w1ok = cval && (j < a.B - 1);
    const bool want_w1 = a.w1chan != nullptr;
    constexpr float inv_m = 1.0f / (float)m;
    __syncthreads();

    // bin column q sits at byte (q / T) * TP + q % T of a row
    auto load_row = [&](int yy) {
        uint8_t* dst = ring + (size_t)(yy % T1) * S * rowb;
        for (int t = lane; t < S * rowb; t += 64) {
            const int ss = t / rowb, o = t - ss * rowb;
            const int blk = o / TP, k = o - blk * TP;
            const int q = blk * T + k;
            const int cc = cbase + ss, xx = xb0 + q;
            // bins are < 64; 0x7F marks columns outside the image or padding
            // (never counted by the 7-bit comparison below)
            uint8_t v = 0x7F;
            if (k < T && cc < a.C && q < Wb && xx >= 0 && xx < W)
                v = a.bins[((size_t)cc * H + yy) * W + xx] & 0x7F;
            dst[t] = v;
        }
    };
    // vc[q] += [bin(row ya, q) <= j] - [bin(row yr, q) <= j], four columns per
    // dword: for 7-bit bytes b and j < 64, 0x80 + j - b never borrows across
    // bytes and its top bit is set exactly when b <= j.
    const uint32_t jhi = ((uint32_t)j * 0x01010101u) | 0x80808080u;
    auto update_vc = [&](int ya, int yr, bool add, bool rem) {
        const uint32_t* ra = (const uint32_t*)(ring + (size_t)(ya % T1) * S * rowb + sa * rowb);
        const uint32_t* rr = (const uint32_t*)(ring + (size_t)((yr + T1) % T1) * S * rowb + sa * rowb);
        uint32_t* v = vc32 + lane * L.vs4;
        const uint32_t ma = add ? 0xFFFFFFFFu : 0u, mr = rem ? 0xFFFFFFFFu : 0u;
        for (int d = 0; d < rowb / 4; ++d) {
            const uint32_t ia = (((jhi - ra[d]) & 0x80808080u) >> 7) & ma;
            const uint32_t ir = (((jhi - rr[d]) & 0x80808080u) >> 7) & mr;
            v[d] = v[d] + ia - ir;
        }
    };

    // gather work items of a block: item it*64+lane -> (channel slot, column k, pending row t)
    constexpr int SMAX = (T <= 9) ? 4 : 2;  // channels per wavefront the gather budget covers
    constexpr int NIT = (T * T * SMAX + 63) / 64;
    const int nit = (S * T * T + 63) / 64;

    const int ys = max(0, y0 - r);
    const int yend = min(H, ye + r);
    const int lo_add = max(0, ys - r);
    const int hi_add = min(H, ys + r);
    for (int yy = lo_add; yy < hi_add; ++yy) {
        load_row(yy);
        __syncthreads();
        update_vc(yy, yy, true, false);
        __syncthreads();
    }

    for (int y = ys; y < yend; ++y) {
        const bool add = (y + r) < H;
        const bool rem = (y - r - 1) >= lo_add;
        if (add) load_row(y + r);
        __syncthreads();
        update_vc(y + r, y - r - 1, add, rem);
        const int ny = min(H - 1, y + r) - max(0, y - r) + 1;
        const bool row_full = (ny == T);
        const bool own_row = (y >= y0) && (y < ye);
        // gather items of this row: item it*64+lane = (channel slot, step k,
        // pending row t); their LDS offsets do not change along the row
        // packed: w0 = ring offset | hrow offset << 16,
        //         w1 = (acc offset + 64) | k << 16 | ok << 31
        uint32_t g_w0[NIT], g_w1[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int idx = it * 64 + lane;
            const int ss = idx / (T * T);
            const int rem2 = idx - ss * (T * T);
            const int k = rem2 / T, t = rem2 - k * T;
            const int yo = y - r + t;
            const bool ok = (it < nit) && (ss < S) && (cbase + ss < a.C) && (yo >= y0) && (yo < ye);
            const int ssc = (ss < S) ? ss : 0;
            const int yoc = ok ? yo : y0;
            const uint32_t ro = (uint32_t)((yoc % T1) * S * rowb + ssc * rowb + k);
            const uint32_t ho = (uint32_t)(k * 64 + ssc * Bp);
            const uint32_t ao = (uint32_t)(((yoc % T) * S + ssc) * Ws + k - 2 * r + 64);
            g_w0[it] = ro | (ho << 16);
            g_w1[it] = ao | ((uint32_t)k << 16) | (ok ? 0x80000000u : 0u);
        }
        // Step i walks patch column p = x0 - r + i; its window covers bin
        // columns q in [i, i + 2r].  The count entering at step i is vc[i + 2r]
        // and the one leaving is vc[i - 1], which entered T steps earlier.
        int vring[T];
        double ering[T];
        int cP = 0;
        vring[0] = 0;
#pragma unroll
        for (int k = 1; k < T; ++k) {
            vring[k] = vcl[k - 1];  // bin columns 0 .. 2r-1 (layout block 0)
            cP += vring[k];
        }
#pragma unroll
        for (int k = 0; k < T; ++k) ering[k] = 0.0;
        double hs = 0.0;
        for (int blk = 0; blk < nblk; ++blk) {
            const int i0 = blk * T;
            const int p0 = x0 - r + i0;  // patch column of the block's first step
            const bool full = row_full && (i0 + T <= np) && (p0 >= r) && (p0 + T - 1 <= W - 1 - r);
            // 1. counts entering the window and the running cumulative counts
            int cpv[T], cm1[T];
            const uint8_t* vb = vcl + blk * TP;
#pragma unroll
            for (int k = 0; k < T; ++k) {
                // bin column i0 + k + 2r = (blk + 1) T + k - 1
                const int v = (k == 0) ? (int)vb[T - 1] : (int)vb[TP + k - 1];
                cP += v - vring[k];
                vring[k] = v;
                cpv[k] = cP;
            }
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const int u = lane_prev(cpv[k]);
                cm1[k] = (j == 0) ? 0 : u;
            }
            float ev[T];
            if (full) {
                int psv[T];
#pragma unroll
                for (int k = 0; k < T; ++k) psv[k] = psig[sa * (m + 1) + cpv[k]].x;
                float rc[T];
#pragma unroll
                for (int k = 0; k < T; ++k) rc[k] = rcp[cpv[k] - cm1[k]];
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    const int pu = lane_prev(psv[k]);
                    const int psu = (j == 0) ? 0 : pu;
                    const int u = cm1[k], vv = cpv[k];
                    const int sc = min(max(crm1, u), vv);
                    const int pss = (crm1 <= u) ? psu : ((crm1 >= vv) ? psv[k] : dm1);
                    const int I = (psv[k] - pss) + (psu - pss) + __mul24(j, 2 * sc - u - vv);
                    ev[k] = (float)I * rc[k] * binf;
                }
            } else {
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    const int i = i0 + k;
                    const int p = x0 - r + i;
                    const bool pval = (i < np) && (p >= 0) && (p < W);
                    const int nx = max(1, min(W - 1, p + r) - max(0, p - r) + 1);
                    const int n = ny * nx;
                    const int cPk = cpv[k], cPm1 = cm1[k];
                    const int av = __mul24(cPk, m);
                    int q0d = (int)((float)av * rcp[min(n, m)]);
                    q0d = max(0, min(q0d, m));
                    if (q0d < m && __mul24(q0d + 1, n) <= av) q0d++;
                    if (q0d > 0 && __mul24(q0d, n) > av) q0d--;
                    const int2 ps = psig[sa * (m + 1) + q0d];
                    const int phia = __mul24(n, ps.x) + __mul24(av - __mul24(q0d, n), ps.y);
                    const int pu = lane_prev(phia);
                    const int phiu = (j == 0) ? 0 : pu;
                    const int au = __mul24(cPm1, m);
                    const int cm = __mul24(crm1, n);
                    const int sc = min(max(cm, au), av);
                    const int phis = (cm <= au) ? phiu : ((cm >= av) ? phia : __mul24(n, dm1));
                    const int I = (phia - phis) + (phiu - phis) + __mul24(j, 2 * sc - au - av);
                    const int P = min(max(cPk - cPm1, 0), m);
                    ev[k] = pval ? (float)I * rcp[P] * inv_m * binf : 0.f;
                }
            }
            if (want_w1 && own_row) {
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    const int p = x0 - r + i0 + k;
                    if (p >= x0 && p < xe) {
                        const int nx = min(W - 1, p + r) - max(0, p - r) + 1;
                        const int n = ny * nx;
                        int d = w1ok ? abs(cpv[k] * m - crl * n) : 0;
                        for (int o = Bp >> 1; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
                        if (cval && j == 0)
                            a.w1chan[((size_t)c * H + y) * W + p] =
                                (float)(a.delta[c] * (double)d / ((double)n * (double)m));
                    }
                }
            }
            // 2. horizontal window sums; after step i the sum covers patch
            //    steps [i - 2r, i], i.e. output column o = i - 2r
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const double ed = (double)ev[k];
                hs += ed - ering[k];
                ering[k] = ed;
                hrow[k * 64 + lane] = (float)hs;
            }
            __syncthreads();
            // 3. gather the pixel's own bin into the accumulators of the T
            //    pending output rows; the output column of step k is
            //    o = i0 + k - 2r, whose bin column i0 + k sits at byte blk*TP + k
            if (i0 + T - 1 >= 2 * r) {
#pragma unroll
                for (int it = 0; it < NIT; ++it) {
                    const uint32_t w0 = g_w0[it], w1 = g_w1[it];
                    const int xo = i0 + (int)((w1 >> 16) & 0x7FFFu) - 2 * r;
                    const bool ok = (w1 >> 31) && (xo >= 0) && (xo < ws);
                    const int b = ring[(w0 & 0xFFFFu) + blk * TP];
                    const float h = hrow[(w0 >> 16) + (b & (Bp - 1))];
                    float* dst = ok ? (acc + (int)(w1 & 0xFFFFu) - 64 + i0) : (trash + lane);
                    *dst += h;
                }
            }
            __syncthreads();
        }
        int yo_lo = y - r, yo_hi = (y < H - 1) ? y - r : H - 1;
        yo_lo = max(yo_lo, y0);
        yo_hi = min(yo_hi, ye - 1);
        for (int yo = yo_lo; yo <= yo_hi; ++yo) {
            const int nyo = min(H - 1, yo + r) - max(0, yo - r) + 1;
            for (int t = lane; t < S * ws; t += 64) {
                const int ss = t / ws, xo = t - ss * ws;
                const int cc = cbase + ss;
                float* ap = acc + ((yo % T) * S + ss) * Ws + xo;
                if (cc < a.C) {
                    const int xg = x0 + xo;
                    const int nxo = min(W - 1, xg + r) - max(0, xg - r) + 1;
                    a.achan[((size_t)cc * H + yo) * W + xg] =
                        (float)((double)(*ap) * a.delta[cc] / (double)(nyo * nxo));
                }
                *ap = 0.f;
            }
        }
        __syncthreads();
    }
}


typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));


__device__ __forceinline__ int bin_of_m(float rr, const float* __restrict__ e, float lo, float idl, int B) {
    if (idl == 0.f) return 0;
    int b = (int)floorf((rr - lo) * idl);
    b = b < 0 ? 0 : (b > B - 1 ? B - 1 : b);
    while (b > 0 && rr < e[b - 1]) --b;
    while (b < B - 1 && rr >= e[b]) ++b;
    return b;
}

__device__ __forceinline__ void emit(const MArgs& a, int c, int px, float r, const float* slo,
                                     const float* sid) {
    if (a.resid) a.resid[(size_t)c * a.N + px] = r;
    if (a.bins)
        a.bins[(size_t)c * a.N + px] =
            (uint8_t)bin_of_m(r, a.edges + (size_t)c * (a.B - 1), slo[c], sid[c], a.B);
}

template <int CMAX, int KT>
__device__ __forceinline__ void proj_tile_f32(const MArgs& a, int tile, int w, int lane,
        const float* __restrict__ V1, const float* __restrict__ V2, const float* smu, const float* slo,
        const float* sid, float* zp) {
    constexpr int NSW = CMAX / 16;
    constexpr int NTW = CMAX / 64;
    constexpr int NU = 4 * KT;
    const int g = lane >> 4, n = lane & 15;
    const int px = tile * 16 + n;
    const bool pxok = px < a.N;
    float d[NSW];
    floatx4 z[KT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) z[kt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < NSW; ++i) {
        const int s = w * NSW + i;
        const int c = 4 * s + g;
        const float x = (pxok && c < a.C) ? a.X[(size_t)c * a.N + px] : 0.f;
        d[i] = (c < a.C) ? x - smu[c] : 0.f;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
            z[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(V1[((s * KT + kt) * 4 + g) * 16 + n], d[i],
                                                         z[kt], 0, 0, 0);
        if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int v = 0; v < 4; ++v) zp[((w * KT + kt) * 4 + v) * 64 + lane] = z[kt][v];
    __syncthreads();
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float acc = zp[((0 * KT + kt) * 4 + v) * 64 + lane];
            acc += zp[((1 * KT + kt) * 4 + v) * 64 + lane];
            acc += zp[((2 * KT + kt) * 4 + v) * 64 + lane];
            acc += zp[((3 * KT + kt) * 4 + v) * 64 + lane];
            z[kt][v] = acc;
        }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NTW; ++i) {
        const int t = w * NTW + i;
        floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < NU; ++u)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(V2[((t * NU + u) * 4 + g) * 16 + n],
                                                       z[u >> 2][u & 3], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = 16 * t + 4 * v + g;
            const float r = d[4 * i + v] - acc[v];
            if (pxok && c < a.C) emit(a, c, px, r, slo, sid);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int CMAX, int KT>
__device__ __forceinline__ void proj_tile_bf16(const MArgs& a, int tile, int w, int lane,
        const bf16x8* __restrict__ V1, const bf16x8* __restrict__ V2, const float* smu, const float* slo,
        const float* sid, float* zp) {
    constexpr int NSW = CMAX / 128;
    constexpr int NU = KT / 2;
    const int g = lane >> 4, n = lane & 15;
    const int px = tile * 16 + n;
    const bool pxok = px < a.N;
    float d[NSW][8];
    floatx4 z[KT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) z[kt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < NSW; ++i) {
        const int s = w * NSW + i;
        bf16x8 bv;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int c = 32 * s + 8 * g + t;
            const float x = (pxok && c < a.C) ? a.X[(size_t)c * a.N + px] : 0.f;
            d[i][t] = (c < a.C) ? x - smu[c] : 0.f;
            bv[t] = (__bf16)d[i][t];
        }
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
            z[kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(V1[((s * KT + kt) * 4 + g) * 16 + n], bv,
                                                            z[kt], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int v = 0; v < 4; ++v) zp[((w * KT + kt) * 4 + v) * 64 + lane] = z[kt][v];
    __syncthreads();
    bf16x8 zb[NU];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float acc = zp[((0 * KT + kt) * 4 + v) * 64 + lane];
            acc += zp[((1 * KT + kt) * 4 + v) * 64 + lane];
            acc += zp[((2 * KT + kt) * 4 + v) * 64 + lane];
            acc += zp[((3 * KT + kt) * 4 + v) * 64 + lane];
            zb[kt >> 1][4 * (kt & 1) + v] = (__bf16)acc;
        }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NSW; ++i) {
        const int s = w * NSW + i;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t2 = 2 * s + h;
            floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int u = 0; u < NU; ++u)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(V2[((t2 * NU + u) * 4 + g) * 16 + n],
                                                              zb[u], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = 32 * s + 8 * g + 4 * h + v;
                const float r = d[i][4 * h + v] - acc[v];
                if (pxok && c < a.C) emit(a, c, px, r, slo, sid);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

}  // namespace tiles
}  // namespace qfca
