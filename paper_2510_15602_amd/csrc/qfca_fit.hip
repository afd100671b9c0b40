// Fit-side kernels for gfx950: mean and covariance of the features (PCA of
// Sec. 3.3, FP64 accumulation), exact per-channel order statistics for the
// quantisation range (Sec. 3.1), the median reference of Sec. 3.2 as an
// integer selection over full-window cumulative counts, and the projection +
// quantisation kernel (residual W - PCA^-1(PCA(W)) then the bin index).
#include <algorithm>

#include "qfca_internal.h"
#include "qfca_tiles.h"

namespace qfca {
namespace {
using tiles::lane_prev;
using tiles::wave_sync;

// ------------------------------------------------------------------------
// Mean: one block per channel, FP64 tree reduction in a fixed order.
__global__ __launch_bounds__(256) void k_mean(const float* __restrict__ X, long N,
                                              double* __restrict__ mu) {
    __shared__ double red[256];
    const int c = blockIdx.x;
    const float* x = X + (size_t)c * N;
    double s = 0.0;
    for (long i = threadIdx.x; i < N; i += 256) s += (double)x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) mu[c] = red[0] / (double)N;
}

// Covariance partials: block (tile ta, tile tb >= ta, chunk) accumulates
// sum_i (x_a - mu_a)(x_b - mu_b) over its pixel chunk for a 64 x 64 tile in
// FP64 on the matrix cores: the centred values of a stage are staged in LDS
// as doubles, and wavefront w computes the 32 x 32 quadrant (w / 2, w % 2)
// as 2 x 2 blocks of v_mfma_f64_16x16x4 (lane (g, n) gives row n of A and
// column n of B at pixel g of each group of four; it ends with rows
// 4 e + g, e = 0 .. 3, of column n: the FP64 form's output order, unlike
// the FP32 16x16x4 form's 4 g + e).  Partials are reduced over chunks in a fixed order
// by k_cov_reduce (deterministic).
constexpr int CT = 64;   // tile side
constexpr int CK = 16;   // pixels per LDS stage (a multiple of 4)
typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_cov_partial(const float* __restrict__ X, int C, long N,
                                                     const double* __restrict__ mu, int ntile,
                                                     long chunk, double* __restrict__ part) {
    __shared__ double As[CK][CT + 1];
    __shared__ double Bs[CK][CT + 1];
    // decode upper-triangular tile pair
    int pair = blockIdx.x, ta = 0;
    while (pair >= ntile - ta) { pair -= ntile - ta; ++ta; }
    const int tb = ta + pair;
    const long i0 = (long)blockIdx.y * chunk;
    const long i1 = min(N, i0 + chunk);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int qa = (w >> 1) * 32, qb = (w & 1) * 32;
    dbl4 acc[2][2];
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) acc[u][v] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (long ib = i0; ib < i1; ib += CK) {
        for (int t = threadIdx.x; t < CK * CT; t += 256) {
            const int kk = t % CK, row = t / CK;
            const long i = ib + kk;
            const int ca = ta * CT + row, cb = tb * CT + row;
            As[kk][row] = (i < i1 && ca < C) ? (double)X[(size_t)ca * N + i] - mu[ca] : 0.0;
            Bs[kk][row] = (i < i1 && cb < C) ? (double)X[(size_t)cb * N + i] - mu[cb] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k0 = 0; k0 < CK; k0 += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) av[u] = As[k0 + g][qa + 16 * u + n];
#pragma unroll
            for (int v = 0; v < 2; ++v) bv[v] = Bs[k0 + g][qb + 16 * v + n];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[v], acc[u][v], 0, 0, 0);
        }
        __syncthreads();
    }
    double* out = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * CT * CT;
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v)
            for (int e = 0; e < 4; ++e) out[(qa + 16 * u + 4 * e + g) * CT + qb + 16 * v + n] = acc[u][v][e];
}

// One thread per entry of a tile pair (grid: pairs x entry blocks); the
// chunk partials are added in chunk order, U loads in flight at a time.
__global__ __launch_bounds__(256) void k_cov_reduce(const double* __restrict__ part, int C, long N, int ntile,
                                                    int npair, int nchunk, double* __restrict__ cov) {
    const int pair0 = blockIdx.x;
    int pair = pair0, ta = 0;
    while (pair >= ntile - ta) { pair -= ntile - ta; ++ta; }
    const int tb = ta + pair;
    const int t = blockIdx.y * blockDim.x + threadIdx.x;
    if (t >= CT * CT) return;
    const double* p = part + (size_t)pair0 * CT * CT + t;
    const size_t stride = (size_t)npair * CT * CT;
    double s = 0.0;
    constexpr int U = 8;
    int k0 = 0;
    for (; k0 + U <= nchunk; k0 += U) {
        double x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = p[(size_t)(k0 + u) * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) s += x[u];
    }
    for (; k0 < nchunk; ++k0) s += p[(size_t)k0 * stride];
    const int a = ta * CT + t / CT, b = tb * CT + t % CT;
    if (a < C && b < C) {
        cov[(size_t)a * C + b] = s / (double)N;
        cov[(size_t)b * C + a] = s / (double)N;
    }
}

// ------------------------------------------------------------------------
// Exact order statistics by MSB-first radix selection on order-preserving
// 32-bit keys, 4 passes of 8 bits, all requested ranks of a channel at once.
constexpr int MAXR = 8;

__device__ __forceinline__ uint32_t fkey(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float funkey(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return __uint_as_float(u);
}

constexpr int SEL_THREADS = 1024;  // per channel: enough loads in flight to cover the memory latency

__global__ __launch_bounds__(SEL_THREADS) void k_select(const float* __restrict__ vals, long N,
                                                const long long* __restrict__ ranks, int nr,
                                                float* __restrict__ out) {
    __shared__ uint32_t hist[MAXR][256];
    __shared__ uint32_t prefix[MAXR];
    __shared__ long long remaining[MAXR];
    const int c = blockIdx.x;
    const float* v = vals + (size_t)c * N;
    if (threadIdx.x < nr) {
        prefix[threadIdx.x] = 0u;
        remaining[threadIdx.x] = ranks[threadIdx.x];
    }
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        const uint32_t mask = pass == 0 ? 0u : (0xFFFFFFFFu << (32 - 8 * pass));
        for (int t = threadIdx.x; t < MAXR * 256; t += SEL_THREADS) (&hist[0][0])[t] = 0u;
        __syncthreads();
        uint32_t pf[MAXR];
#pragma unroll
        for (int q = 0; q < MAXR; ++q) pf[q] = q < nr ? prefix[q] : 0u;
        // U loads per thread in flight before their histogram updates
        constexpr int U = 16;
        for (long i0 = threadIdx.x; i0 < N; i0 += SEL_THREADS * U) {
            float x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const long i = i0 + (long)u * SEL_THREADS;
                x[u] = v[i < N ? i : N - 1];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (i0 + (long)u * SEL_THREADS >= N) break;
                const uint32_t k = fkey(x[u]);
#pragma unroll
                for (int q = 0; q < MAXR; ++q)
                    if (q < nr && (k & mask) == pf[q]) atomicAdd(&hist[q][(k >> shift) & 255u], 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x < nr) {
            const int q = threadIdx.x;
            long long rem = remaining[q];
            int d = 0;
            for (d = 0; d < 256; ++d) {
                if (rem < (long long)hist[q][d]) break;
                rem -= hist[q][d];
            }
            prefix[q] |= ((uint32_t)min(d, 255)) << shift;
            remaining[q] = rem;
        }
        __syncthreads();
    }
    if (threadIdx.x < nr) out[(size_t)c * nr + threadIdx.x] = funkey(prefix[threadIdx.x]);
}

// ------------------------------------------------------------------------
// Reference: count table counts[c][i][t] = #{full windows p : cP_p(i) = t}.
// Lane (s, j) owns bin j of channel s.  Per row of window centres:
//   1. the entering and leaving image rows of the S channels are staged in
//      LDS (0x7F outside the image, never counted);
//   2. each lane's vertical counts #{rows of the window : bin <= j} of every
//      column, four columns per dword, are updated with one SWAR step per
//      dword: for 7-bit bytes b and j < 64, 0x80 + j - b never borrows across
//      bytes and its top bit is set exactly when b <= j;
//   3. the lane walks the columns with a running window sum cP and counts
//      each full window's cP in its bin's table of uint16 counters, two per
//      word, by LDS atomic adds that return nothing (no wait per window).
// The four wavefronts of a block (one band each) share the tables; their
// counts (at most 4 Ws Hb = 16384 windows) fit in 16 bits and are flushed
// with global atomics at the end.
struct RArgs {
    const uint8_t* bins;
    int C, H, W, T, B, Bp, S, r, m, Ws, Hb, nsplit;
    int perbin;  // 1: count the windows' bin counts P(j) instead of their cumulative counts cP(j)
    // what a window's count v in [0, m] adds to: mode 0 its own counter v
    // (mcnt = m); mode 1 the counter v >> sh (coarse pass of a median,
    // mcnt = m >> sh); mode 2, only when v >> sh equals sel[c][j], the
    // counter v & (2^sh - 1) (fine pass, mcnt = 2^sh - 1)
    int mode, sh, mcnt;
    const int32_t* sel;
    uint32_t* counts;  // [C][B][mcnt + 1]
};

__host__ __device__ inline size_t ralign16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS of a k_refcount block of nw wavefronts: the count table shared by the
// block, then each wavefront's column counts and staged rows.
struct RefLayout {
    int WbP, vsd, mw;
    size_t cnt, wave, total;
    __host__ __device__ RefLayout(int Ws, int r, int S, int per, int m, int nw) {
        const int WbMax = Ws + 2 * r;       // bin columns of the widest tile
        WbP = (WbMax + 3) & ~3;
        vsd = WbP / 4;
        if ((vsd & 1) == 0) vsd += 1;       // odd dword stride between lanes
        mw = (m + 2) / 2;                   // words holding counters 0 .. m
        cnt = ralign16((size_t)S * per * mw * 4);
        wave = ralign16((size_t)64 * vsd * 4) + ralign16((size_t)2 * S * WbP);
        total = cnt + (size_t)nw * wave;
    }
    __host__ __device__ size_t vc(int w) const { return cnt + (size_t)w * wave; }
    __host__ __device__ size_t rows(int w) const { return vc(w) + ralign16((size_t)64 * vsd * 4); }
};

// MODE: what a window's count adds to (RArgs::mode); PERBIN: RArgs::perbin.
// A block of nw wavefronts (blockDim.x / 64, at most 4) shares one count
// table: wavefront w walks band blockIdx.y * nw + w of the strip with its own
// column counts and staged rows, synchronising with itself only, and adds to
// the shared counters with LDS atomics; the block adds the table to the
// global one at the end.
template <int MODE, bool PERBIN>
__global__ __launch_bounds__(256) void k_refcount(RArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int nw = (int)blockDim.x >> 6;
    const int Bp = a.Bp, S = a.S, T = a.T, r = a.r, m = a.m, H = a.H, W = a.W;
    const int s = lane / Bp, j = lane - s * Bp;
    const int sa = s < S ? s : S - 1;
    const int x0 = blockIdx.x * a.Ws, xe = min(W, x0 + a.Ws), ws = xe - x0;
    const int y0 = ((int)blockIdx.y * nw + w) * a.Hb, ye = min(H, y0 + a.Hb);
    const int split = blockIdx.z % a.nsplit;
    const int cbase = (blockIdx.z / a.nsplit) * S;
    const int c = cbase + s;
    const bool cv = (s < S) && (c < a.C);
    const int per = Bp / a.nsplit;
    const int jlo = split * per;
    const bool counting = cv && (j < a.B) && (j >= jlo) && (j < jlo + per);
    const int mcnt = a.mcnt;
    const int selj = (a.mode == 2 && counting) ? a.sel[(size_t)c * a.B + j] : -1;
    const RefLayout L(a.Ws, r, S, per, mcnt, nw);
    const int WbP = L.WbP;
    const int Wb = ws + 2 * r;  // bin columns [x0-r, xe+r)
    const int xb0 = x0 - r;
    uint32_t* cnt = (uint32_t*)smem;               // [S][per][mw], shared
    uint32_t* vc32 = (uint32_t*)(smem + L.vc(w));  // [64 lanes][vsd]
    uint8_t* rows = smem + L.rows(w);              // [2][S][WbP]
    for (int t = lane; t < 64 * L.vsd; t += 64) vc32[t] = 0u;
    for (int t = threadIdx.x; t < S * per * L.mw; t += blockDim.x) cnt[t] = 0u;
    __syncthreads();
    uint32_t* mycnt = cnt + ((size_t)sa * per + (counting ? j - jlo : 0)) * L.mw;
    const uint32_t jhi = ((uint32_t)j * 0x01010101u) | 0x80808080u;
    // Full-window centres owned by this tile: rows [ys, yend), columns
    // [max(x0, r), min(xe, W - r)).
    const int ys = max(y0, r), yend = min(ye, H - r);
    const int pxlo = max(x0, r), pxhi = min(xe, W - r);
    if (ys < yend && pxlo < pxhi) {
        // Image row yy into staging slot h (0 entering, 1 leaving), one pass
        // for the S channels.  When a slot fits LR bytes per lane, each lane's
        // source offsets are fixed for the tile (channel ss, column q of byte
        // t = lane + 64 i: ss H W + x, offset 0 and bit i of lmark clear where
        // the byte lies outside the image), and a row is loaded into
        // registers (issue) a row before it is written to the slot (commit),
        // so the loads overlap the previous row's counting.  Every load is
        // issued from a valid address; markers and rows outside the image
        // become 0x7F when committed.
        constexpr int LR = 4;
        const bool lfast = (S * WbP <= 64 * LR) && ((long long)S * H * W < 0x7FFFFFFFLL);
        int loff[LR];
        uint32_t lmark = 0;
#pragma unroll
        for (int i = 0; i < LR; ++i) {
            const int t = lane + 64 * i;
            const int ss = t / WbP, q = t - ss * WbP;
            const int cc = cbase + ss, xl = xb0 + q;
            const bool ok = lfast && t < S * WbP && q < Wb && cc < a.C && xl >= 0 && xl < W;
            loff[i] = ok ? ss * H * W + xl : 0;
            lmark |= ok ? (1u << i) : 0u;
        }
        const uint8_t* gbase = a.bins + (size_t)cbase * H * W;
        auto issue = [&](uint32_t (&pre)[LR], int yy) {
            const uint8_t* rowp = gbase + (size_t)(yy >= 0 && yy < H ? yy : 0) * W;
#pragma unroll
            for (int i = 0; i < LR; ++i) pre[i] = rowp[loff[i]];
        };
        auto commit = [&](const uint32_t (&pre)[LR], int h, int yy) {
            const bool yok = yy >= 0 && yy < H;
#pragma unroll
            for (int i = 0; i < LR; ++i) {
                const int t = lane + 64 * i;
                if (t < S * WbP)
                    rows[(size_t)h * S * WbP + t] = (yok && ((lmark >> i) & 1u)) ? (uint8_t)(pre[i] & 0x7Fu) : (uint8_t)0x7F;
            }
        };
        auto stage = [&](int h, int yy) {
            for (int t = lane; t < S * WbP; t += 64) {
                const int ss = t / WbP, q = t - ss * WbP;
                const int cc = cbase + ss, xl = xb0 + q;
                uint8_t v = 0x7F;
                if (q < Wb && cc < a.C && xl >= 0 && xl < W && yy >= 0 && yy < H)
                    v = a.bins[((size_t)cc * H + yy) * W + xl] & 0x7F;
                rows[(size_t)(h * S + ss) * WbP + q] = v;
            }
        };
        uint32_t pa[LR], pr[LR];  // the next row's entering and leaving bytes
        // the lane's counts += [entering bin <= j] (ADD), -= [leaving bin <= j]
        // (REM); the loads of a chunk are issued before its stores
        auto update = [&](bool add, bool rem) {
            const uint32_t* __restrict__ ra = (const uint32_t*)(rows + (size_t)sa * WbP);
            const uint32_t* __restrict__ rr = (const uint32_t*)(rows + (size_t)(S + sa) * WbP);
            uint32_t* __restrict__ v = vc32 + lane * L.vsd;
            const int nd = WbP / 4;
            constexpr int CH = 8;
            for (int d0 = 0; d0 < nd; d0 += CH) {
                uint32_t xv[CH], xa[CH], xr[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int d = min(d0 + i, nd - 1);
                    xv[i] = v[d];
                    xa[i] = ra[d];
                    xr[i] = rr[d];
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    uint32_t x = xv[i];
                    if (add) x += ((jhi - xa[i]) & 0x80808080u) >> 7;
                    if (rem) x -= ((jhi - xr[i]) & 0x80808080u) >> 7;
                    if (d0 + i < nd) v[d0 + i] = x;
                }
            }
        };
        if (lfast) issue(pa, ys - r);
        for (int yy = ys - r; yy < ys + r; ++yy) {
            wave_sync();
            if (lfast) {
                commit(pa, 0, yy);
                issue(pa, yy + 1);  // the next warm-up row, or row ys + r
            } else {
                stage(0, yy);
            }
            wave_sync();
            update(true, false);
        }
        const uint8_t* __restrict__ vb = (const uint8_t*)(vc32 + lane * L.vsd);
        for (int yc = ys; yc < yend; ++yc) {
            const bool rem = yc > ys;
            wave_sync();
            if (lfast) {
                commit(pa, 0, yc + r);
                if (rem) commit(pr, 1, yc - r - 1);
                if (yc + 1 < yend) {
                    issue(pa, yc + 1 + r);
                    issue(pr, yc - r);
                }
            } else {
                stage(0, yc + r);
                if (rem) stage(1, yc - r - 1);
            }
            wave_sync();
            update(true, rem);
            wave_sync();
            // window sums along the row: cP = sum of the counts of columns
            // [q - T + 1, q]; the window ending at column q is centred on
            // image column xb0 + q - r, and is counted for q in [qc0, qc1)
            // (a full window of the tile's own centres)
            const int qc0 = max(T - 1, pxlo - xb0 + r), qc1 = min(Wb, pxhi - xb0 + r);
            const uint32_t* __restrict__ vw = vc32 + lane * L.vsd;
            auto count = [&](int cP) __attribute__((always_inline)) {
                // the bin's own count: its cumulative count minus the previous
                // bin's (the neighbouring lane of the channel); the exchange
                // runs in every lane
                const int pv = lane_prev(cP);
                const int cv0 = PERBIN ? cP - (j == 0 ? 0 : pv) : cP;
                if constexpr (MODE == 2) {
                    if (counting && (cv0 >> a.sh) == selj) {
                        const int cu = cv0 & ((1 << a.sh) - 1);
                        atomicAdd(mycnt + (cu >> 1), 1u << ((cu & 1) << 4));
                    }
                } else {
                    // lanes that do not count add zero to a counter of their
                    // own channel's table (every cu lies in [0, mcnt])
                    const int cu = MODE == 0 ? cv0 : cv0 >> a.sh;
                    atomicAdd(mycnt + (cu >> 1), counting ? 1u << ((cu & 1) << 4) : 0u);
                }
            };
            int cP = 0;
            for (int q = qc0 - T + 1; q <= qc0; ++q) cP += (int)vb[q];
            count(cP);
            // then four columns per step: the entering bytes are one dword,
            // the leaving ones (T columns back) the dword pair's bytes at a
            // fixed offset
            int q = qc0 + 1;
            for (; q < qc1 && (q & 3); ++q) {
                cP += (int)vb[q] - (int)vb[q - T];
                count(cP);
            }
            const int osh = (4 - (T & 3)) & 3;  // (q - T) & 3 for q a multiple of 4
            for (; q + 4 <= qc1; q += 4) {
                const uint32_t xn = vw[q >> 2];
                const int qo = q - T - osh;  // a multiple of 4
                const uint32_t lo = vw[qo >> 2], hi = vw[(qo >> 2) + 1];
                const uint32_t xo = osh ? __builtin_amdgcn_alignbyte(hi, lo, osh) : lo;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    cP += (int)((xn >> (8 * i)) & 0xFFu) - (int)((xo >> (8 * i)) & 0xFFu);
                    count(cP);
                }
            }
            for (; q < qc1; ++q) {
                cP += (int)vb[q] - (int)vb[q - T];
                count(cP);
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < S * per * L.mw; t += blockDim.x) {
        const int ss = t / (per * L.mw);
        const int rest = t - ss * per * L.mw;
        const int jj = rest / L.mw + jlo, w = rest - (rest / L.mw) * L.mw;
        const int cc = cbase + ss;
        const uint32_t v = cnt[t];
        if (v && cc < a.C && jj < a.B) {
            uint32_t* dst = a.counts + ((size_t)cc * a.B + jj) * (mcnt + 1) + 2 * w;
            if (v & 0xFFFFu) atomicAdd(dst, v & 0xFFFFu);
            if ((v >> 16) && 2 * w + 1 <= mcnt) atomicAdd(dst + 1, v >> 16);
        }
    }
}

// References taken bin by bin over the full-window histograms (Sec. 4.5.3,
// Tab. 3), from the count table of the windows' bin counts: for every
// channel (one thread each) and bin i, the lower median over windows of
// P(i) (kind 0: the h-th smallest, h = ceil(P_w / 2)) or its mean (kind 1),
// accumulated into cumulative weights cRw [C][B] (double).
__global__ void k_refstat(const uint32_t* __restrict__ counts, int C, int B, int m, long long nw, int kind,
                          double* __restrict__ cRw) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const long long h = (nw + 1) / 2;
    double acc = 0.0;
    for (int i = 0; i < B; ++i) {
        const uint32_t* cnt = counts + ((size_t)c * B + i) * (m + 1);
        double v = 0.0;
        if (kind == 0) {
            long long seen = 0;
            int t = 0;
            for (t = 0; t < m; ++t) {
                seen += cnt[t];
                if (seen >= h) break;
            }
            v = (double)t;
        } else {
            double sum = 0.0;  // integer-valued, exact below 2^53
            for (int t = 1; t <= m; ++t) sum += (double)t * (double)cnt[t];
            v = sum / (double)nw;
        }
        acc += v;
        cRw[(size_t)c * B + i] = acc;
    }
}

// Rank-wise mean of the sorted full windows (Sec. 3.2 "mean -> quan"):
// for channel c (blockIdx.y) and a slice of the window-centre rows
// (blockIdx.x), every wavefront sorts its windows' T*T values in its LDS
// region (bitonic, padded to NP = 2^k >= T*T with +inf) and adds the value of
// rank rho to its running double sum (lane l holds ranks l, l + 64, ...).
// The sums go to part[(c * gridDim.x + blockIdx.x) * 4 + wave][rho], reduced
// afterwards in a fixed order.
template <int NP>
__global__ __launch_bounds__(256) void k_refmean(const float* __restrict__ R, int C, int H, int W, int T,
                                                 double* __restrict__ part) {
    extern __shared__ __align__(16) unsigned char smem_rm[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float* v = (float*)smem_rm + (size_t)wv * NP;
    const int c = blockIdx.y, r = T / 2, n = T * T;
    const int ny = H - T + 1, nx = W - T + 1;
    const int rows_per = (ny + gridDim.x - 1) / gridDim.x;
    const int py0 = r + blockIdx.x * rows_per, py1 = min(r + ny, py0 + rows_per);
    constexpr int PER = NP / 64;
    double sum[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) sum[i] = 0.0;
    const float* Rc = R + (size_t)c * H * W;
    // windows of the slice, one per wavefront in turn
    const int nwin = (py1 > py0) ? (py1 - py0) * nx : 0;
    for (int wi = wv; wi < nwin; wi += 4) {
        const int py = py0 + wi / nx, px = r + wi % nx;
        for (int t = lane; t < NP; t += 64) {
            float x = INFINITY;
            if (t < n) {
                const int dy = t / T, dx = t - dy * T;
                x = Rc[(size_t)(py - r + dy) * W + (px - r + dx)];
            }
            v[t] = x;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int k = 2; k <= NP; k <<= 1) {
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                for (int pi = lane; pi < NP / 2; pi += 64) {
                    const int i = ((pi & ~(jj - 1)) << 1) | (pi & (jj - 1));
                    const int q = i | jj;
                    const float a = v[i], b = v[q];
                    const bool up = (i & k) == 0;
                    const bool sw = up ? (a > b) : (a < b);
                    v[i] = sw ? b : a;
                    v[q] = sw ? a : b;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int rho = lane + 64 * i;
            if (rho < n) sum[i] += (double)v[rho];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    double* dst = part + (((size_t)c * gridDim.x + blockIdx.x) * 4 + wv) * NP;
#pragma unroll
    for (int i = 0; i < PER; ++i) dst[lane + 64 * i] = sum[i];
}

// Y[c][rho] = (sum over the slices and wavefronts, in order) / P_w, then the
// reference histogram of Y quantised with the float32 edges (a value equal
// to an edge goes to the upper bin), cumulated: cR [C][B] (one thread per
// channel).
__global__ void k_refmean_finish(const double* __restrict__ part, int C, int nparts, int NP, int n, double nw,
                                 const float* __restrict__ edges, int B, int32_t* __restrict__ cR) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    int hist[64];
    for (int i = 0; i < 64; ++i) hist[i] = 0;
    for (int rho = 0; rho < n; ++rho) {
        double s = 0.0;
        for (int pw = 0; pw < nparts * 4; ++pw) s += part[((size_t)c * nparts * 4 + pw) * NP + rho];
        const double y = s / nw;
        int b = 0;
        for (int e = 0; e < B - 1; ++e) b += (y >= (double)edges[(size_t)c * (B - 1) + e]) ? 1 : 0;
        hist[b] += 1;
    }
    int acc = 0;
    for (int i = 0; i < B; ++i) {
        acc += hist[i];
        cR[(size_t)c * B + i] = acc;
    }
}

__global__ void k_refselect(const uint32_t* __restrict__ counts, int C, int B, int m, long long h,
                            int32_t* __restrict__ cR) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * B) return;
    const uint32_t* cnt = counts + (size_t)t * (m + 1);
    long long seen = 0;
    int v = m;
    for (v = m; v > 0; --v) {
        seen += cnt[v];
        if (seen >= h) break;
    }
    cR[t] = v;
}

// Two-pass median, pass 1: for every (channel, bin), the coarse bucket
// (count >> sh) that holds the h-th largest window count, and that count's
// rank among the bucket's windows (counted from the top).
__global__ void k_refsel_coarse(const uint32_t* __restrict__ counts, int C, int B, int nb, long long h,
                                int32_t* __restrict__ sel, long long* __restrict__ hrem) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * B) return;
    const uint32_t* cnt = counts + (size_t)t * nb;
    long long seen = 0;
    int b = nb - 1;
    for (; b > 0; --b) {
        if (seen + cnt[b] >= h) break;
        seen += cnt[b];
    }
    sel[t] = b;
    hrem[t] = h - seen;
}

// Pass 2: the h'-th largest of the counts in the selected bucket, from the
// bucket's fine table (count & (2^sh - 1)).
__global__ void k_refsel_fine(const uint32_t* __restrict__ counts, int C, int B, int sh,
                              const int32_t* __restrict__ sel, const long long* __restrict__ hrem,
                              int32_t* __restrict__ cR) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * B) return;
    const int nf = 1 << sh;
    const uint32_t* cnt = counts + (size_t)t * nf;
    const long long h = hrem[t];
    long long seen = 0;
    int v = nf - 1;
    for (; v > 0; --v) {
        seen += cnt[v];
        if (seen >= h) break;
    }
    cR[t] = (sel[t] << sh) + v;
}

// ------------------------------------------------------------------------
// Projection + quantisation, FP32 on the vector ALUs: one thread per pixel;
// z = V^T (x - mu) (KP accumulators, V zero-padded to KP columns), then
// r_c = (x_c - mu_c) - sum_j V[c][j] z_j, then the bin index.
struct PArgs {
    const float* X;
    int C, N, k, B, preproc;
    const float* mu;
    const float* V;  // [C][KP]
    const float* edges;
    const float* lo;
    const float* inv_delta;
    uint8_t* bins;
    float* resid;
};

// bin = #{m : rr >= e[m]} for the channel's ascending edges e: a guess from
// (rr - lo) / delta corrected edge by edge (a zero-width channel, idl = 0,
// has no guess and walks the edges from bin 0).
__device__ __forceinline__ int bin_of(float rr, const float* __restrict__ e, float lo, float idl, int B) {
    int b = idl == 0.f ? 0 : (int)floorf((rr - lo) * idl);
    b = b < 0 ? 0 : (b > B - 1 ? B - 1 : b);
    while (b > 0 && rr < e[b - 1]) --b;
    while (b < B - 1 && rr >= e[b]) ++b;
    return b;
}

template <int KP>
__global__ __launch_bounds__(256) void k_proj_fp32(PArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const size_t N = (size_t)a.N;
    float z[KP > 0 ? KP : 1];
#pragma unroll
    for (int q = 0; q < (KP > 0 ? KP : 1); ++q) z[q] = 0.f;
    if (a.preproc && KP > 0) {
        for (int c = 0; c < a.C; ++c) {
            const float d = a.X[(size_t)c * N + i] - a.mu[c];
            const float* vr = a.V + (size_t)c * KP;
#pragma unroll
            for (int q = 0; q < KP; ++q) z[q] = fmaf(vr[q], d, z[q]);
        }
    }
    for (int c = 0; c < a.C; ++c) {
        float rr = a.X[(size_t)c * N + i];
        if (a.preproc) {
            rr -= a.mu[c];
            const float* vr = a.V + (size_t)c * KP;
            float rec = 0.f;
#pragma unroll
            for (int q = 0; q < KP; ++q) rec = fmaf(vr[q], z[q], rec);
            rr -= rec;
        }
        if (a.resid) a.resid[(size_t)c * N + i] = rr;
        if (a.bins)
            a.bins[(size_t)c * N + i] =
                (uint8_t)bin_of(rr, a.edges + (size_t)c * (a.B - 1), a.lo[c], a.inv_delta[c], a.B);
    }
}

}  // namespace

hipError_t launch_mean(const float* X, int C, long N, double* mu, hipStream_t st) {
    hipLaunchKernelGGL(k_mean, dim3(C), dim3(256), 0, st, X, N, mu);
    return hipGetLastError();
}

hipError_t launch_cov(const float* X, int C, long N, const double* mu, double* cov, hipStream_t st) {
    const int ntile = (C + CT - 1) / CT;
    const int npair = ntile * (ntile + 1) / 2;
    int nchunk = (int)std::max(1L, std::min(512L, 1024L / npair));
    nchunk = (int)std::min<long>(nchunk, std::max(1L, N / CK));
    const long chunk = ((N + nchunk - 1) / nchunk + CK - 1) / CK * CK;
    nchunk = (int)((N + chunk - 1) / chunk);
    double* part = nullptr;
    hipError_t e = hipMallocAsync((void**)&part, (size_t)nchunk * npair * CT * CT * sizeof(double), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cov_partial, dim3(npair, nchunk), dim3(256), 0, st, X, C, N, mu, ntile,
                       chunk, part);
    hipLaunchKernelGGL(k_cov_reduce, dim3(npair, (CT * CT + 255) / 256), dim3(256), 0, st, part, C, N, ntile,
                       npair, nchunk, cov);
    e = hipGetLastError();
    const hipError_t e2 = hipFreeAsync(part, st);
    return e != hipSuccess ? e : e2;
}

hipError_t launch_select(const float* vals, int C, long N, const long long* ranks_dev, int nr,
                         float* out, hipStream_t st) {
    if (nr > MAXR) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_select, dim3(C), dim3(SEL_THREADS), 0, st, vals, N, ranks_dev, nr, out);
    return hipGetLastError();
}

// Count-table pass: mode, shift and selected buckets as in RArgs; counts
// [C][B][mcnt + 1] is zeroed first.  nsplit_out (if given) receives the bin
// splits the mode-0 table needs to fit in LDS.
static hipError_t refcount_pass(const uint8_t* bins, int C, int H, int W, int T, int B, uint32_t* counts,
                                hipStream_t st, int perbin, int mode, int sh, const int32_t* sel,
                                int* nsplit_out, bool launch) {
    RArgs a;
    a.bins = bins; a.C = C; a.H = H; a.W = W; a.T = T; a.B = B;
    a.perbin = perbin;
    int Bp = 8;
    while (Bp < B) Bp <<= 1;
    a.Bp = Bp;
    a.r = T / 2; a.m = T * T;
    a.mode = mode; a.sh = sh; a.sel = sel;
    a.mcnt = mode == 0 ? a.m : (mode == 1 ? (a.m >> sh) : (1 << sh) - 1);
    a.Ws = 64; a.Hb = 64;
    a.counts = counts;
    // channels per wave and bin splits so the private histograms fit in LDS;
    // a tile's counters are 16 bits wide
    int S = 64 / Bp, nsplit = 1;
    auto lds = [&](int S_, int ns_, int nw_) { return RefLayout(a.Ws, a.r, S_, Bp / ns_, a.mcnt, nw_).total; };
    while (lds(S, nsplit, 1) > 60000 && S > 1) S >>= 1;
    while (lds(S, nsplit, 1) > 60000 && nsplit < Bp) nsplit <<= 1;
    if (lds(S, nsplit, 1) > 65536) return hipErrorInvalidValue;
    // four wavefronts share a table where it fits (a counter then sees at
    // most 4 Ws Hb windows, within its 16 bits)
    const int nw = lds(S, nsplit, 4) <= 60000 ? 4 : 1;
    if ((long)nw * a.Ws * a.Hb >= 65536) return hipErrorInvalidValue;
    if (nsplit_out) *nsplit_out = nsplit;
    if (!launch) return hipSuccess;
    hipError_t e = hipMemsetAsync(counts, 0, (size_t)C * B * (a.mcnt + 1) * sizeof(uint32_t), st);
    if (e != hipSuccess) return e;
    a.S = S; a.nsplit = nsplit;
    dim3 grid((W + a.Ws - 1) / a.Ws, (H + a.Hb * nw - 1) / (a.Hb * nw), ((C + S - 1) / S) * nsplit);
    const size_t ldsb = lds(S, nsplit, nw);
    const dim3 block(64 * nw);
    if (mode == 0 && !perbin)
        hipLaunchKernelGGL((k_refcount<0, false>), grid, block, ldsb, st, a);
    else if (mode == 0)
        hipLaunchKernelGGL((k_refcount<0, true>), grid, block, ldsb, st, a);
    else if (mode == 1 && !perbin)
        hipLaunchKernelGGL((k_refcount<1, false>), grid, block, ldsb, st, a);
    else if (mode == 1)
        hipLaunchKernelGGL((k_refcount<1, true>), grid, block, ldsb, st, a);
    else if (!perbin)
        hipLaunchKernelGGL((k_refcount<2, false>), grid, block, ldsb, st, a);
    else
        hipLaunchKernelGGL((k_refcount<2, true>), grid, block, ldsb, st, a);
    return hipGetLastError();
}

hipError_t launch_refcount(const uint8_t* bins, int C, int H, int W, int T, int B,
                           uint32_t* counts, hipStream_t st, int perbin) {
    return refcount_pass(bins, C, H, W, T, B, counts, st, perbin, 0, 0, nullptr, nullptr, true);
}

hipError_t launch_refmedian(const uint8_t* bins, int C, int H, int W, int T, int B, uint32_t* counts,
                            long long h, int32_t* cR, hipStream_t st) {
    const int m = T * T;
    int nsplit = 1;
    hipError_t e = refcount_pass(bins, C, H, W, T, B, counts, st, 0, 0, 0, nullptr, &nsplit, false);
    if (e != hipSuccess) return e;
    if (nsplit == 1) {
        // the whole table of counts 0 .. m fits: one pass
        if ((e = launch_refcount(bins, C, H, W, T, B, counts, st)) != hipSuccess) return e;
        return launch_refselect(counts, C, B, m, h, cR, st);
    }
    // Two passes over the map with small tables instead of nsplit passes with
    // the whole one: buckets of 2^sh counts (at most 64 buckets, 64 counts
    // each), then the counts inside each (channel, bin)'s median bucket.
    int sh = 0;
    while ((m >> sh) + 1 > 64) ++sh;
    const size_t n = (size_t)C * B;
    // carved from the caller's table of n (m + 1) words (m + 1 > 128 here)
    uint32_t* c1 = counts;
    uint32_t* c2 = counts + n * 64;
    int32_t* sel = (int32_t*)(counts + n * 128);
    long long* hrem = (long long*)(counts + n * 130);  // 8-byte aligned: n * 130 words from an aligned base
    if ((size_t)m + 1 < 134) return hipErrorInvalidValue;
    if ((e = refcount_pass(bins, C, H, W, T, B, c1, st, 0, 1, sh, nullptr, nullptr, true)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_refsel_coarse, dim3((int)((n + 255) / 256)), dim3(256), 0, st, c1, C, B, (m >> sh) + 1, h,
                       sel, hrem);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = refcount_pass(bins, C, H, W, T, B, c2, st, 0, 2, sh, sel, nullptr, true)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_refsel_fine, dim3((int)((n + 255) / 256)), dim3(256), 0, st, c2, C, B, sh, sel, hrem, cR);
    return hipGetLastError();
}

hipError_t launch_refstat(const uint32_t* counts, int C, int B, int m, long long nw, int kind, double* cRw,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_refstat, dim3((C + 63) / 64), dim3(64), 0, st, counts, C, B, m, nw, kind, cRw);
    return hipGetLastError();
}

size_t refmean_part_bytes(int C, int T, int* nparts, int* NP) {
    int np2 = 64;
    while (np2 < T * T) np2 <<= 1;
    *NP = np2;
    *nparts = 32;
    return (size_t)C * 32 * 4 * np2 * sizeof(double);
}

hipError_t launch_refmean(const float* R, int C, int H, int W, int T, const float* edges, int B, double* part,
                          int32_t* cR, hipStream_t st) {
    int nparts = 0, NP = 0;
    (void)refmean_part_bytes(C, T, &nparts, &NP);
    const size_t lds = (size_t)4 * NP * sizeof(float);
    dim3 grid(nparts, C);
    auto go = [&](const void* k, auto launch) -> hipError_t {
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        launch();
        return hipGetLastError();
    };
    hipError_t e = hipErrorInvalidValue;
    switch (NP) {
#define QFCA_RM(NPV) \
        case NPV: e = go((const void*)k_refmean<NPV>, [&] { \
            hipLaunchKernelGGL(k_refmean<NPV>, grid, dim3(256), lds, st, R, C, H, W, T, part); }); break;
        QFCA_RM(64) QFCA_RM(128) QFCA_RM(256) QFCA_RM(512) QFCA_RM(1024) QFCA_RM(2048) QFCA_RM(4096)
#undef QFCA_RM
        default: break;
    }
    if (e != hipSuccess) return e;
    const double nw = (double)(H - T + 1) * (double)(W - T + 1);
    hipLaunchKernelGGL(k_refmean_finish, dim3((C + 63) / 64), dim3(64), 0, st, (const double*)part, C, nparts,
                       NP, T * T, nw, edges, B, cR);
    return hipGetLastError();
}

hipError_t launch_refselect(const uint32_t* counts, int C, int B, int m, long long h, int32_t* cR,
                            hipStream_t st) {
    const int n = C * B;
    hipLaunchKernelGGL(k_refselect, dim3((n + 255) / 256), dim3(256), 0, st, counts, C, B, m, h, cR);
    return hipGetLastError();
}

hipError_t launch_proj(const ProjLaunch& L, hipStream_t st) {
    if (L.preproc && L.k > 0 && L.V1 && L.V2) return launch_proj_mfma(L, L.V1, L.V2, st);
    if (L.prec == QFCA_PREC_BF16 && L.preproc && L.k > 0) return hipErrorInvalidValue;
    PArgs a;
    a.X = L.X; a.C = L.C; a.N = L.N; a.k = L.k; a.B = L.B; a.preproc = L.preproc;
    a.mu = L.mu; a.V = L.V; a.edges = L.edges; a.lo = L.lo; a.inv_delta = L.inv_delta;
    a.bins = L.bins; a.resid = L.resid;
    const int KP = (!L.preproc || L.k == 0) ? 0 : (L.k <= 8 ? 8 : L.k <= 16 ? 16 : L.k <= 32 ? 32 : 64);
    if (L.preproc && L.k > 64) return hipErrorInvalidValue;
    dim3 grid((L.N + 255) / 256);
    switch (KP) {
        case 0: hipLaunchKernelGGL(k_proj_fp32<0>, grid, dim3(256), 0, st, a); break;
        case 8: hipLaunchKernelGGL(k_proj_fp32<8>, grid, dim3(256), 0, st, a); break;
        case 16: hipLaunchKernelGGL(k_proj_fp32<16>, grid, dim3(256), 0, st, a); break;
        case 32: hipLaunchKernelGGL(k_proj_fp32<32>, grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL(k_proj_fp32<64>, grid, dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

}  // namespace qfca
