// Patch statistics comparison (Sec. 3.1, Alg. 1), error-to-pixel association
// with sigma_p = infinity (Sec. 3.1, Sec. 4.5.4), channel mean (Eq. 1) and the
// final sigma_s blur (Sec. 4.5.4) for gfx950.
//
// Work decomposition of k_score: one wavefront per (column strip, row band,
// group of S channels).  Lane (s, j) owns bin j of channel s; lanes walk the
// strip left to right, one row of patch centres at a time, streaming down the
// band:
//   * vc[x][lane]: the number of pixels of column x inside the current T-row
//     window whose bin is <= j (updated by one add and one remove per row),
//   * cP: running horizontal sum of vc, i.e. the window's cumulative count at
//     bin j,
//   * Algorithm 1's per-bin transport numerator I_j is evaluated in closed
//     form from cP_{j-1}, cP_j (the previous lane) and the reference tables:
//     with a_i = cP_i m, c_k = cR_k n (equal-mass scaling, m = T^2 reference
//     mass, n in-image window mass) and Phi(t) = sum_{k<B-1} (t - c_k)^+,
//     the bin's mass occupies quantiles (a_{j-1}, a_j] and is sent to the
//     reference bin J(u) = #{k : c_k < u}, so
//       I_j = int_{a_{j-1}}^{a_j} |j - J(u)| du
//           = Phi(a_{j-1}) + Phi(a_j) - 2 Phi(s) + j (2 s - a_{j-1} - a_j),
//     s = clamp(c_{j-1}, a_{j-1}, a_j).  This is exactly what the two-pointer
//     loop of Alg. 1 accumulates; e_j = I_j / (P_j m) in bin units.
//   * e is summed over the T patch columns around each output column (in
//     this generic kernel each window sum is formed afresh, in image-column
//     order, in double precision; the block-walk kernel k_score_t sums in an
//     order fixed by the image columns too, so either kernel's maps are the
//     same for every tiling), and the result for the pixel's own bin is
//     gathered across lanes and added to the pixel's accumulator for each of
//     the T patch rows that cover it (rows in image order).
// All counts are exact integers; each per-channel value is rounded once to
// 64-bit fixed point and added to the channel sum with an integer atomic
// (order-free); k_finish turns the sum into the channel mean and blurs it.
#include <algorithm>
#include <atomic>

#include "qfca_internal.h"
#include "qfca_tiles.h"

namespace qfca {
namespace {
using namespace tiles;

struct Lds {
    size_t vc, ring, acc, psig, rcp, ering, crw, wgt, total;
};

// WbA: allocated bin columns per row (>= Ws + 4r; the block-walk kernel
// rounds it up to a multiple of T).
__host__ __device__ inline Lds lds_layout(int T, int Bp, int S, int Ws, int WbA) {
    (void)Bp;
    const int m = T * T;
    const size_t WbMax = (size_t)WbA;
    Lds L;
    size_t off = 0;
    L.vc = off;    off += align16(WbMax * 64);
    L.ring = off;  off += align16((size_t)(T + 1) * S * WbMax);
    L.acc = off;   off += align16((size_t)T * S * Ws * 4);
    L.psig = off;  off += align16((size_t)S * (m + 1) * 8);
    L.rcp = off;   off += align16((size_t)(m + 1) * 4);
    L.ering = off; off += align16((size_t)T * 64 * 4);
    L.crw = off;   off += align16((size_t)S * 64 * 8);  // general reference weights (B <= 64)
    L.wgt = off;   off += align16((size_t)T * 4);       // association weights (finite sigma_p)
    L.total = off;
    return L;
}

__global__ __launch_bounds__(64) void k_score(KArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int Bp = a.Bp, S = a.S, T = a.T, r = a.r, m = a.m, H = a.H, W = a.W;
    const int T1 = T + 1;
    const int s = lane / Bp;
    const int sa = s < S ? s : S - 1;
    const int j = lane - s * Bp;
    const int x0 = blockIdx.x * a.Ws;
    const int xe = min(W, x0 + a.Ws);
    const int ws = xe - x0;
    const int y0 = blockIdx.y * a.Hb;
    const int ye = min(H, y0 + a.Hb);
    const int cbase = blockIdx.z * S;
    const int c = cbase + s;
    const bool cval = (s < S) && (c < a.C);
    const int WbMax = a.WbA;
    const int Wb = ws + 4 * r;
    const int xb0 = x0 - 2 * r;

    const Lds L = lds_layout(T, Bp, S, a.Ws, a.WbA);
    uint8_t* vc = smem + L.vc;
    uint8_t* ring = smem + L.ring;
    float* acc = (float*)(smem + L.acc);
    int2* psig = (int2*)(smem + L.psig);
    float* rcp = (float*)(smem + L.rcp);
    float* ering = (float*)(smem + L.ering);
    double* crw = (double*)(smem + L.crw);  // [S][B] cumulative reference weights (general reference)
    float* wgt = (float*)(smem + L.wgt);    // [T] association weights w(d), d = -r .. r
    const bool gen = a.cRw != nullptr, gauss = a.wgt != nullptr;
    const int B = a.B;
    for (int t = lane; t < S * B; t += 64) {
        const int ss = t / B, cc = cbase + ss;
        crw[t] = (gen && cc < a.C) ? a.cRw[(size_t)cc * B + (t - ss * B)] : 0.0;
    }
    for (int t = lane; t < T; t += 64) wgt[t] = gauss ? a.wgt[t] : 1.f;

    // the integer tables exist only for an integer reference of mass T*T (a
    // general reference has none: nothing is read from them then)
    for (int t = lane; t < S * (m + 1); t += 64) {
        const int ss = t / (m + 1), tt = t - ss * (m + 1);
        const int cc = cbase + ss;
        psig[t] = (!gen && cc < a.C) ? a.psig[(size_t)cc * (m + 1) + tt] : make_int2(0, 0);
    }
    for (int t = lane; t <= m; t += 64) rcp[t] = gen ? 0.f : a.rcp[t];
    for (int t = lane; t < WbMax * 16; t += 64) ((uint32_t*)vc)[t] = 0u;
    for (int t = lane; t < T * S * a.Ws; t += 64) acc[t] = 0.f;
    const int ci = cval ? c : 0;
    const int crm1 = gen ? 0 : a.cRm1[ci * Bp + j];
    const int dm1 = gen ? 0 : a.Dm1[ci * Bp + j];
    const int crl = gen ? 0 : a.cRl[ci * Bp + j];
    const bool binok = cval && (j < a.B);
    const bool w1ok = cval && (j < a.B - 1);
    const bool want_w1 = a.w1sum != nullptr;
    const float inv_m = 1.0f / (float)m;
    __syncthreads();

    auto load_row = [&](int yy) {
        uint8_t* dst = ring + (size_t)(yy % T1) * S * WbMax;
        for (int t = lane; t < S * Wb; t += 64) {
            const int ss = t / Wb, q = t - ss * Wb;
            const int cc = cbase + ss, xx = xb0 + q;
            uint8_t v = 0xFF;  // out of the image: never counted
            if (cc < a.C && xx >= 0 && xx < W) v = a.bins[((size_t)cc * H + yy) * W + xx];
            dst[ss * WbMax + q] = v;
        }
    };

    const int ys = max(0, y0 - r);
    const int yend = min(H, ye + r);
    const int lo_add = max(0, ys - r);
    const int hi_add = min(H, ys + r);
    // Bring the vertical window of the first processed row up to date.
    for (int yy = lo_add; yy < hi_add; ++yy) {
        load_row(yy);
        __syncthreads();
        const uint8_t* row = ring + (size_t)(yy % T1) * S * WbMax + sa * WbMax;
        for (int q = 0; q < Wb; ++q) {
            const int xl = xb0 + q;
            if (xl >= 0 && xl < W) vc[q * 64 + lane] += (row[q] <= j) ? 1 : 0;
        }
        __syncthreads();
    }

    for (int y = ys; y < yend; ++y) {
        const bool add = (y + r) < H;
        const bool rem = (y - r - 1) >= lo_add;
        if (add) load_row(y + r);
        __syncthreads();
        const uint8_t* rowA = ring + (size_t)((y + r) % T1) * S * WbMax + sa * WbMax;
        const uint8_t* rowR = ring + (size_t)((y - r - 1 + T1) % T1) * S * WbMax + sa * WbMax;
        const int ny = min(H - 1, y + r) - max(0, y - r) + 1;
        const bool own_row = (y >= y0) && (y < ye);
        int cP = 0;
        int slot = 0;
        for (int q = 0; q < Wb; ++q) {
            const int xl = xb0 + q;
            int v = 0;
            if (xl >= 0 && xl < W) {
                v = vc[q * 64 + lane];
                if (add) v += (rowA[q] <= j) ? 1 : 0;
                if (rem) v -= (rowR[q] <= j) ? 1 : 0;
                vc[q * 64 + lane] = (uint8_t)v;
            }
            const int vold = (q >= T) ? (int)vc[(q - T) * 64 + lane] : 0;
            cP += v - vold;
            const int p = xl - r;  // patch-centre column
            float e = 0.f;
            if (q >= 2 * r && p >= 0 && p < W) {
                const int nx = min(W - 1, p + r) - max(0, p - r) + 1;
                const int n = ny * nx;
                int cPm1 = lane_prev(cP);
                if (j == 0) cPm1 = 0;
                const int P = cP - cPm1;
                if (gen) {
                    // General reference (any nonnegative weights, mass M_R):
                    // a = cP M_R, c_k = cR_k n, Phi(t) = sum_{k<B-1} (t - c_k)^+
                    // summed directly in double precision.
                    const double* cr = crw + sa * B;
                    const double MR = cr[B - 1], dn = (double)n;
                    const double au = (double)cPm1 * MR, av = (double)cP * MR;
                    const double cm = (j >= 1 && j < B) ? dn * cr[j - 1] : 0.0;
                    const double sc = fmin(fmax(cm, au), av);
                    double pu = 0.0, pv = 0.0, ps = 0.0;
                    for (int k = 0; k < B - 1; ++k) {
                        const double ck = dn * cr[k];
                        pu += fmax(au - ck, 0.0);
                        pv += fmax(av - ck, 0.0);
                        ps += fmax(sc - ck, 0.0);
                    }
                    const double I = (pu + pv - 2.0 * ps) + (double)j * (2.0 * sc - au - av);
                    e = (binok && P > 0 && MR > 0.0) ? (float)(I / ((double)P * MR)) : 0.f;
                } else if (n == m) {
                    // Interior window: equal masses, Phi(c P) = m Psi(cP).
                    const int psv = psig[sa * (m + 1) + cP].x;
                    int psu = lane_prev(psv);
                    if (j == 0) psu = 0;
                    const int u = cPm1, vv = cP;
                    const int sc = min(max(crm1, u), vv);
                    const int pss = (crm1 <= u) ? psu : ((crm1 >= vv) ? psv : dm1);
                    const int I = (psv - pss) + (psu - pss) + j * (2 * sc - u - vv);
                    e = (binok && P > 0) ? (float)I * rcp[P] : 0.f;
                } else {
                    // Clipped window: a = cP m, c = cR n, Phi(a) = n Psi(t) with
                    // t = a / n, evaluated by linear interpolation of Psi.
                    const int av = cP * m;
                    int q0 = (int)((float)av * rcp[n]);
                    if ((q0 + 1) * n <= av) q0++;
                    if (q0 * n > av) q0--;
                    const int2 ps = psig[sa * (m + 1) + q0];
                    const int phia = n * ps.x + (av - q0 * n) * ps.y;
                    int phiu = lane_prev(phia);
                    if (j == 0) phiu = 0;
                    const int au = cPm1 * m;
                    const int cm = crm1 * n;
                    const int sc = min(max(cm, au), av);
                    const int phis = (cm <= au) ? phiu : ((cm >= av) ? phia : n * dm1);
                    const int I = (phia - phis) + (phiu - phis) + j * (2 * sc - au - av);
                    e = (binok && P > 0) ? (float)I * rcp[P] * inv_m : 0.f;
                }
                if (want_w1 && own_row && p >= x0 && p < xe) {
                    if (gen) {
                        const double* cr = crw + sa * B;
                        const double MR = cr[B - 1];
                        double d = w1ok ? fabs((double)cP * MR - cr[j] * (double)n) : 0.0;
                        for (int o = Bp >> 1; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
                        if (cval && j == 0 && MR > 0.0) {
                            const double v = (d * (a.delta[c] * a.fxs)) / ((double)n * MR);
                            __hip_atomic_fetch_add(&a.w1sum[(size_t)y * W + p], __double2ll_rn(v),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    } else {
                        int d = w1ok ? abs(cP * m - crl * n) : 0;
                        for (int o = Bp >> 1; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
                        if (cval && j == 0) {
                            const double v = ((double)d * (a.delta[c] * a.fxs)) / ((double)n * (double)m);
                            __hip_atomic_fetch_add(&a.w1sum[(size_t)y * W + p], __double2ll_rn(v),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                }
            }
            // Horizontal window sum of e over the T patch columns around
            // output column p - r (weighted by w(d) for a finite sigma_p),
            // summed afresh in double from the oldest column to the newest,
            // an order fixed by the image columns.
            ering[slot * 64 + lane] = e;
            slot = (slot + 1 == T) ? 0 : slot + 1;
            const int xo = q - 4 * r;  // local output column
            if (xo >= 0) {
                double hs = 0.0;
                for (int i = 0, sl = slot; i < T; ++i, sl = (sl + 1 == T) ? 0 : sl + 1)
                    hs += gauss ? (double)wgt[i] * (double)ering[sl * 64 + lane] : (double)ering[sl * 64 + lane];
                const float hf = (float)hs;
                for (int tc = 0; tc < T; tc += Bp) {
                    const int t = tc + j;
                    const int yo = y - r + t;
                    const bool ok = cval && (t < T) && (yo >= y0) && (yo < ye);
                    int b = 0;
                    if (ok) b = ring[(size_t)(yo % T1) * S * WbMax + sa * WbMax + xo + 2 * r];
                    const float hv = __shfl(hf, sa * Bp + b, 64);
                    if (ok) {
                        float* ap = acc + ((yo % T) * S + sa) * a.Ws + xo;
                        *ap = gauss ? __builtin_fmaf(wgt[t], hv, *ap) : *ap + hv;
                    }
                }
            }
        }
        // Output rows whose last covering patch row is y.
        int yo_lo = y - r, yo_hi = (y < H - 1) ? y - r : H - 1;
        yo_lo = max(yo_lo, y0);
        yo_hi = min(yo_hi, ye - 1);
        __syncthreads();
        // in-image weight of the windows along one axis around position x
        // (their count for the box, the sum of w(d) for a finite sigma_p)
        auto axis_weight = [&](int x, int len) -> double {
            if (!gauss) return (double)(min(len - 1, x + r) - max(0, x - r) + 1);
            double w = 0.0;
            for (int i = 0; i < T; ++i)
                if (x - r + i >= 0 && x - r + i < len) w += (double)wgt[i];
            return w;
        };
        for (int yo = yo_lo; yo <= yo_hi; ++yo) {
            const double rny = 1.0 / axis_weight(yo, H);
            for (int t = lane; t < S * ws; t += 64) {
                const int ss = t / ws, xo = t - ss * ws;
                const int cc = cbase + ss;
                float* ap = acc + ((yo % T) * S + ss) * a.Ws + xo;
                const float av = *ap;
                *ap = 0.f;
                if (cc < a.C) {
                    const int xg = x0 + xo;
                    const double v = (((double)av * (a.delta[cc] * a.fxs)) * (1.0 / axis_weight(xg, W))) * rny;
                    if (a.achan) a.achan[((size_t)cc * H + yo) * W + xg] = (float)(v * (1.0 / a.fxs));
                    __hip_atomic_fetch_add(&a.asum[(size_t)yo * W + xg], __double2ll_rn(v), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        __syncthreads();
    }
}

template <int T>
__global__ __launch_bounds__(64) void k_score_t(KArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    // block-shared, at LDS address 0: the kernel has no static LDS (its
    // launcher checks that), so the dynamic LDS starts there
    float* rcp4 = (float*)smem;
    fill_rcp4<T>(rcp4, a.rcp, threadIdx.x, 64);
    const int y0 = blockIdx.y * a.Hb;
    score_tile<T, false, true>(a, blockIdx.x, y0, min(a.H, y0 + a.Hb), blockIdx.z, threadIdx.x,
                               smem + BLayout<T>::RCP_BYTES, rcp4);
}

// The block walk with a finite sigma_p (Gaussian association weights a.wgt).
template <int T>
__global__ __launch_bounds__(64) void k_score_tg(KArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* rcp4 = (float*)smem;
    fill_rcp4<T>(rcp4, a.rcp, threadIdx.x, 64);
    const int y0 = blockIdx.y * a.Hb;
    score_tile<T, false, true, false, false, true>(a, blockIdx.x, y0, min(a.H, y0 + a.Hb), blockIdx.z, threadIdx.x,
                                                   smem + BLayout<T>::RCP_BYTES, rcp4);
}

// Separable Gaussian, radius R, renormalised over in-image taps (the 2-D
// renormalisation factorises because the in-image tap set is a rectangle).
constexpr int BT = 16;
constexpr int RMAX = 16;

struct BlurW {
    double w[RMAX + 1];
};

// Box mean over the windows holding each pixel (radius r, clipped to the
// image) of the window-W1 map W = (float)(w1sum * inv): amap (float) and,
// when w1 is given, W itself.  Separable, in double, in a fixed order.
constexpr int BOXT = 16, BOXR = 31;
__global__ __launch_bounds__(256) void k_box(const long long* __restrict__ w1sum, double inv, int H, int W, int r,
                                             float* __restrict__ amap, float* __restrict__ w1) {
    __shared__ double tile[BOXT + 2 * BOXR][BOXT + 2 * BOXR];
    __shared__ double hp[BOXT + 2 * BOXR][BOXT];
    const int tx = threadIdx.x % BOXT, ty = threadIdx.x / BOXT;
    const int bx = blockIdx.x * BOXT, by = blockIdx.y * BOXT;
    const int TS = BOXT + 2 * r;
    for (int t = threadIdx.x; t < TS * TS; t += 256) {
        const int ly = t / TS, lx = t - ly * TS;
        const int gy = by + ly - r, gx = bx + lx - r;
        tile[ly][lx] = (gy >= 0 && gy < H && gx >= 0 && gx < W)
                           ? (double)(float)((double)w1sum[(size_t)gy * W + gx] * inv) : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < TS * BOXT; t += 256) {
        const int ly = t / BOXT, lx = t - ly * BOXT;
        double sacc = 0.0;
        for (int d = 0; d <= 2 * r; ++d) sacc += tile[ly][lx + d];
        hp[ly][lx] = sacc;
    }
    __syncthreads();
    const int gy = by + ty, gx = bx + tx;
    if (gy >= H || gx >= W) return;
    double sacc = 0.0;
    for (int d = 0; d <= 2 * r; ++d) sacc += hp[ty + d][tx];
    const int nx = min(W - 1, gx + r) - max(0, gx - r) + 1, ny = min(H - 1, gy + r) - max(0, gy - r) + 1;
    amap[(size_t)gy * W + gx] = (float)(sacc / ((double)nx * (double)ny));
    if (w1) w1[(size_t)gy * W + gx] = (float)tile[ty + r][tx + r];
}

// Separable Gaussian (radius R) of a float map, renormalised over the
// in-image taps.
__global__ __launch_bounds__(256) void k_blur_f32(const float* __restrict__ in, int H, int W, int R, BlurW wts,
                                                  float* __restrict__ out) {
    __shared__ double tile[BT + 2 * RMAX][BT + 2 * RMAX];
    __shared__ double hpass[BT + 2 * RMAX][BT];
    __shared__ double w[RMAX + 1];
    const int tx = threadIdx.x % BT, ty = threadIdx.x / BT;
    const int bx = blockIdx.x * BT, by = blockIdx.y * BT;
    const int TS = BT + 2 * R;
    if (threadIdx.x <= R) w[threadIdx.x] = wts.w[threadIdx.x];
    for (int t = threadIdx.x; t < TS * TS; t += 256) {
        const int ly = t / TS, lx = t - ly * TS;
        const int gy = by + ly - R, gx = bx + lx - R;
        tile[ly][lx] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? (double)in[(size_t)gy * W + gx] : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < TS * BT; t += 256) {
        const int ly = t / BT, lx = t - ly * BT;
        const int gx = bx + lx;
        double sacc = 0.0, ws = 0.0;
        for (int d = -R; d <= R; ++d) {
            if (gx + d < 0 || gx + d >= W) continue;
            const double wd = w[d < 0 ? -d : d];
            sacc += wd * tile[ly][lx + R + d];
            ws += wd;
        }
        hpass[ly][lx] = sacc / ws;
    }
    __syncthreads();
    const int gy = by + ty, gx = bx + tx;
    if (gy >= H || gx >= W) return;
    double sacc = 0.0, ws = 0.0;
    for (int d = -R; d <= R; ++d) {
        if (gy + d < 0 || gy + d >= H) continue;
        const double wd = w[d < 0 ? -d : d];
        sacc += wd * hpass[ty + R + d][tx];
        ws += wd;
    }
    out[(size_t)gy * W + gx] = (float)(sacc / ws);
}

__global__ __launch_bounds__(256) void k_zero64(long long* __restrict__ a, long long* __restrict__ b, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        a[i] = 0;
        if (b) b[i] = 0;
    }
}

// Window 1-Wasserstein distances of every window (the principal-coordinate
// variant of the score), summed over channels into a.w1sum.
template <int T>
__global__ __launch_bounds__(64) void k_score_w1(KArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* rcp4 = (float*)smem;
    fill_rcp4<T>(rcp4, a.rcp, threadIdx.x, 64);
    const int y0 = blockIdx.y * a.Hb;
    score_tile<T, false, true, false, true>(a, blockIdx.x, y0, min(a.H, y0 + a.Hb), blockIdx.z, threadIdx.x,
                                            smem + BLayout<T>::RCP_BYTES, rcp4);
}

// Inspection build of k_score_t: the same tile code, also storing every
// window's cumulative counts and transport numerators.
template <int T>
__global__ __launch_bounds__(64) void k_score_dbg(KArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* rcp4 = (float*)smem;
    fill_rcp4<T>(rcp4, a.rcp, threadIdx.x, 64);
    const int y0 = blockIdx.y * a.Hb;
    score_tile<T, false, true, true>(a, blockIdx.x, y0, min(a.H, y0 + a.Hb), blockIdx.z, threadIdx.x,
                                     smem + BLayout<T>::RCP_BYTES, rcp4);
}

// The channel mean A = (float)(asum * inv) of the fixed-point channel sum
// (written to amap when given) and its separable Gaussian blur; with w1 and
// w1sum given, also w1 = (float)(w1sum * inv).  R = 0 copies A.
__global__ __launch_bounds__(256) void k_finish(const long long* __restrict__ asum,
                                                const long long* __restrict__ w1sum, double inv, int H,
                                                int W, int R, BlurW wts, float* __restrict__ amap,
                                                float* __restrict__ w1, float* __restrict__ out) {
    __shared__ double tile[BT + 2 * RMAX][BT + 2 * RMAX];
    __shared__ double hpass[BT + 2 * RMAX][BT];
    __shared__ double w[RMAX + 1];
    const int tx = threadIdx.x % BT, ty = threadIdx.x / BT;
    const int bx = blockIdx.x * BT, by = blockIdx.y * BT;
    const int TS = BT + 2 * R;
    if (threadIdx.x <= R) w[threadIdx.x] = wts.w[threadIdx.x];
    for (int t = threadIdx.x; t < TS * TS; t += 256) {
        const int ly = t / TS, lx = t - ly * TS;
        const int gy = by + ly - R, gx = bx + lx - R;
        tile[ly][lx] = (gy >= 0 && gy < H && gx >= 0 && gx < W)
                           ? (double)(float)((double)asum[(size_t)gy * W + gx] * inv) : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < TS * BT; t += 256) {
        const int ly = t / BT, lx = t - ly * BT;
        const int gx = bx + lx;
        double s = 0.0, ws = 0.0;
        for (int d = -R; d <= R; ++d) {
            const int xx = gx + d;
            if (xx < 0 || xx >= W) continue;
            const double wd = w[d < 0 ? -d : d];
            s += wd * tile[ly][lx + R + d];
            ws += wd;
        }
        hpass[ly][lx] = s / ws;
    }
    __syncthreads();
    const int gy = by + ty, gx = bx + tx;
    if (gy >= H || gx >= W) return;
    const size_t g = (size_t)gy * W + gx;
    if (amap) amap[g] = (float)tile[ty + R][tx + R];
    if (w1 && w1sum) w1[g] = (float)((double)w1sum[g] * inv);
    double s = 0.0, ws = 0.0;
    for (int d = -R; d <= R; ++d) {
        const int yy = gy + d;
        if (yy < 0 || yy >= H) continue;
        const double wd = w[d < 0 ? -d : d];
        s += wd * hpass[ty + R + d][tx];
        ws += wd;
    }
    out[g] = (float)(s / ws);
}

}  // namespace

bool score_has_block_kernel(int T) { return T >= 3 && T <= 31 && (T & 1); }
int score_block_max_S(int T) { return T <= 9 ? 4 : 2; }
int score_block_ws(int T, int Ws) { return T < 1 ? Ws : std::max(T, Ws / T * T); }

static int alloc_cols(int T, int Ws, int variant) {
    (void)variant;
    return Ws + 4 * (T / 2);
}

template <int T>
static size_t blayout_bytes(int S, int Ws) { return BLayout<T>::RCP_BYTES + BLayout<T>(S, Ws).total; }

size_t score_rcp_bytes(int T) { return align16((size_t)(T * T + 1) * 4); }

size_t score_lds_bytes(int T, int Bp, int S, int Ws, int variant) {
    if (variant == 1 && score_has_block_kernel(T)) {
        Ws = score_block_ws(T, Ws);
        switch (T) {
#define QFCA_T_LDS(TT) case TT: return blayout_bytes<TT>(S, Ws);
            QFCA_T_LDS(3) QFCA_T_LDS(5) QFCA_T_LDS(7) QFCA_T_LDS(9) QFCA_T_LDS(11) QFCA_T_LDS(13)
            QFCA_T_LDS(15) QFCA_T_LDS(17) QFCA_T_LDS(19) QFCA_T_LDS(21) QFCA_T_LDS(23) QFCA_T_LDS(25)
            QFCA_T_LDS(27) QFCA_T_LDS(29) QFCA_T_LDS(31)
#undef QFCA_T_LDS
            default: break;
        }
    }
    return lds_layout(T, Bp, S, Ws, alloc_cols(T, Ws, 0)).total;
}

// k_score_t<T> addresses its reciprocal table as LDS address 0, which holds
// while the kernel has no static LDS: checked once per window size, on the
// first launch.
static hipError_t no_static_lds(const void* k, int T) {
    static std::atomic<int> state[32];  // by T / 2: 0 unknown, 1 none, 2 some
    std::atomic<int>& s = state[(T / 2) & 31];
    int v = s.load(std::memory_order_relaxed);
    if (v == 0) {
        hipFuncAttributes fa;
        const hipError_t e = hipFuncGetAttributes(&fa, k);
        if (e != hipSuccess) return e;
        v = fa.sharedSizeBytes == 0 ? 1 : 2;
        s.store(v, std::memory_order_relaxed);
    }
    return v == 1 ? hipSuccess : hipErrorInvalidDeviceFunction;
}

static hipError_t no_static_lds_uncached(const void* k) {
    hipFuncAttributes fa;
    const hipError_t e = hipFuncGetAttributes(&fa, k);
    if (e != hipSuccess) return e;
    return fa.sharedSizeBytes == 0 ? hipSuccess : hipErrorInvalidDeviceFunction;
}

hipError_t launch_score(const ScoreLaunch& L, hipStream_t st) {
    KArgs a;
    a.bins = L.bins;
    a.C = L.C; a.H = L.H; a.W = L.W; a.T = L.T; a.B = L.B;
    a.Bp = L.tab.Bp;
    a.S = L.tile.S;
    a.r = L.T / 2;
    a.m = L.T * L.T;
    a.Hb = L.tile.Hb;
    // a general reference runs the column walk; a finite sigma_p runs the
    // block walk with Gaussian weights where the tile allows it
    const bool generic_only = L.tab.cRw != nullptr;
    const bool gauss = L.tab.wgt != nullptr;
    const int variant =
        (!generic_only && L.tile.variant == 1 && score_has_block_kernel(L.T) &&
         L.tile.S <= score_block_max_S(L.T) && L.tile.Ws >= L.T) ? 1 : 0;
    a.Ws = variant ? score_block_ws(L.T, L.tile.Ws) : L.tile.Ws;
    a.WbA = alloc_cols(L.T, a.Ws, variant);
    a.psig = L.tab.psig; a.cRm1 = L.tab.cRm1; a.Dm1 = L.tab.Dm1; a.cRl = L.tab.cRl;
    a.rcp = L.tab.rcp; a.delta = L.tab.delta;
    a.fxs = L.fxs; a.asum = L.asum; a.w1sum = L.w1sum; a.achan = L.achan;
    a.dbg_cp = L.dbg_cp; a.dbg_I = L.dbg_I;
    a.cRw = L.tab.cRw; a.wgt = L.tab.wgt;
    const bool dbg = L.dbg_cp != nullptr;
    if (dbg && (!L.dbg_I || variant != 1 || gauss)) return hipErrorInvalidValue;
    const bool w1o = L.w1only && variant == 1;
    if (L.w1only && !a.w1sum) return hipErrorInvalidValue;
    if (a.S < 1 || a.S * a.Bp > 64 || !a.asum) return hipErrorInvalidValue;
    const size_t lds = score_lds_bytes(a.T, a.Bp, a.S, a.Ws, variant);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    dim3 grid((L.W + a.Ws - 1) / a.Ws, (L.H + a.Hb - 1) / a.Hb, (L.C + a.S - 1) / a.S);
    {
        const size_t n = (size_t)L.H * L.W;
        const int zb = (int)std::min<size_t>((n + 255) / 256, 1024);
        hipLaunchKernelGGL(k_zero64, dim3(zb), dim3(256), 0, st, a.asum, a.w1sum, n);
    }
    // more than 64 KiB of dynamic LDS has to be allowed per kernel
    auto allow = [&](const void* k) -> hipError_t {
        return lds > 65536 ? hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                           : hipSuccess;
    };
    if (variant == 0) {
        hipError_t e = allow((const void*)k_score);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_score, grid, dim3(64), lds, st, a);
        return hipGetLastError();
    }
    switch (a.T) {
#define QFCA_T_CASE(TT)                                                          \
        case TT: {                                                               \
            const bool gs = gauss && !dbg && !w1o;                               \
            const void* kf = dbg ? (const void*)k_score_dbg<TT>                  \
                                 : (w1o ? (const void*)k_score_w1<TT>            \
                                        : (gs ? (const void*)k_score_tg<TT> : (const void*)k_score_t<TT>)); \
            hipError_t e = (dbg || w1o || gs) ? no_static_lds_uncached(kf) : no_static_lds(kf, TT); \
            if (e == hipSuccess) e = allow(kf);                                  \
            if (e != hipSuccess) return e;                                       \
            if (dbg)                                                             \
                hipLaunchKernelGGL(k_score_dbg<TT>, grid, dim3(64), lds, st, a); \
            else if (w1o)                                                        \
                hipLaunchKernelGGL(k_score_w1<TT>, grid, dim3(64), lds, st, a);  \
            else if (gs)                                                         \
                hipLaunchKernelGGL(k_score_tg<TT>, grid, dim3(64), lds, st, a);  \
            else                                                                 \
                hipLaunchKernelGGL(k_score_t<TT>, grid, dim3(64), lds, st, a);   \
        } break;
        QFCA_T_CASE(3) QFCA_T_CASE(5) QFCA_T_CASE(7) QFCA_T_CASE(9) QFCA_T_CASE(11)
        QFCA_T_CASE(13) QFCA_T_CASE(15) QFCA_T_CASE(17) QFCA_T_CASE(19) QFCA_T_CASE(21)
        QFCA_T_CASE(23) QFCA_T_CASE(25) QFCA_T_CASE(27) QFCA_T_CASE(29) QFCA_T_CASE(31)
#undef QFCA_T_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finish_w1(const long long* w1sum, double inv_scale, int H, int W, int T, float sigma,
                            float* amap, float* w1, float* score, hipStream_t st) {
    const int r = T / 2;
    if (r > BOXR) return hipErrorInvalidValue;
    dim3 grid((W + BOXT - 1) / BOXT, (H + BOXT - 1) / BOXT);
    hipLaunchKernelGGL(k_box, grid, dim3(256), 0, st, w1sum, inv_scale, H, W, r, amap, w1);
    const int R = sigma > 0.f ? (int)ceil(3.0 * (double)sigma) : 0;
    if (R > RMAX) return hipErrorInvalidValue;
    BlurW wts;
    for (int d = 0; d <= RMAX; ++d)
        wts.w[d] = d <= R ? (R > 0 ? exp(-(double)(d * d) / (2.0 * (double)sigma * (double)sigma)) : 1.0) : 0.0;
    dim3 g2((W + BT - 1) / BT, (H + BT - 1) / BT);
    hipLaunchKernelGGL(k_blur_f32, g2, dim3(256), 0, st, (const float*)amap, H, W, R, wts, score);
    return hipGetLastError();
}

hipError_t launch_finish(const long long* asum, const long long* w1sum, double inv_scale, int H, int W,
                         float sigma, float* amap, float* w1, float* score, hipStream_t st) {
    const int R = sigma > 0.f ? (int)ceil(3.0 * (double)sigma) : 0;
    if (R > RMAX) return hipErrorInvalidValue;
    BlurW wts;
    for (int d = 0; d <= RMAX; ++d)
        wts.w[d] = d <= R ? (R > 0 ? exp(-(double)(d * d) / (2.0 * (double)sigma * (double)sigma)) : 1.0) : 0.0;
    dim3 grid((W + BT - 1) / BT, (H + BT - 1) / BT);
    hipLaunchKernelGGL(k_finish, grid, dim3(256), 0, st, asum, w1sum, inv_scale, H, W, R, wts, amap, w1, score);
    return hipGetLastError();
}

}  // namespace qfca
