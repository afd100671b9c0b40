// Batched QFCA for images of different sizes (gfx950): one persistent kernel
// drains a device work queue of projection tiles (16 pixels of one image:
// residual + bins) and score tiles (a strip x band of one image for 4 channel
// groups: window histograms, Alg. 1, association, fixed-point channel sum),
// followed by a batched kernel for the channel mean and the blur.  The launch sequence is captured once in a
// hipGraph whose kernels read every per-batch quantity from device-resident
// descriptors, so one graph replays any batch within its capacity.
//
// Ordering: every projection item precedes every score item in the queue.
// A block that takes a score item of image i waits (bounded spin) until all
// projection items of image i are done; those items were taken earlier by
// blocks that are already running, so the wait always ends.  Projection
// blocks publish with a device-scope release (fence + atomic add), score
// blocks acquire with an atomic load and a fence before reading the bins.
#include <algorithm>

#include "qfca_batch_impl.h"

namespace qfca {

namespace {
using namespace tiles;

__global__ void k_batch_reset(BatchHeader* h, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        h->head = 0;
        h->error = 0;
    }
    if (i < n) h->done[i] = 0;
}


// Channel mean A = (float)(asum * inv_scale) of every image (written to its
// amap when given) and its separable Gaussian blur, radius R <= 16 (grid:
// tiles, images).
__global__ __launch_bounds__(256) void k_batch_blur(const BatchHeader* hdr, const BatchJob* jobs) {
    constexpr int BT = 16, RM = 16;
    __shared__ double tile[BT + 2 * RM][BT + 2 * RM];
    __shared__ double hp[BT + 2 * RM][BT];
    const int jb = blockIdx.z;
    if (jb >= hdr->n) return;
    const BatchJob& J = jobs[jb];
    const int H = J.sa.H, W = J.sa.W, R = hdr->blur_R;
    const int ntx = (W + BT - 1) / BT, nty = (H + BT - 1) / BT;
    const int tx = threadIdx.x % BT, ty = threadIdx.x / BT, TS = BT + 2 * R;
    for (int tb = blockIdx.x; tb < ntx * nty; tb += gridDim.x) {
        const int bx = (tb % ntx) * BT, by = (tb / ntx) * BT;
        __syncthreads();
        for (int t = threadIdx.x; t < TS * TS; t += 256) {
            const int ly = t / TS, lx = t - ly * TS;
            const int gy = by + ly - R, gx = bx + lx - R;
            tile[ly][lx] = (gy >= 0 && gy < H && gx >= 0 && gx < W)
                               ? (double)(float)((double)J.asum[(size_t)gy * W + gx] * J.inv_scale) : 0.0;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < TS * BT; t += 256) {
            const int ly = t / BT, lx = t - ly * BT;
            const int gx = bx + lx;
            double s = 0.0, ws = 0.0;
            for (int d = -R; d <= R; ++d) {
                const int xx = gx + d;
                if (xx < 0 || xx >= W) continue;
                const double wd = hdr->blur_w[d < 0 ? -d : d];
                s += wd * tile[ly][lx + R + d];
                ws += wd;
            }
            hp[ly][lx] = ws > 0.0 ? s / ws : 0.0;
        }
        __syncthreads();
        const int gy = by + ty, gx = bx + tx;
        if (gy < H && gx < W) {
            if (J.amap) J.amap[(size_t)gy * W + gx] = (float)tile[ty + R][tx + R];
            double s = 0.0, ws = 0.0;
            for (int d = -R; d <= R; ++d) {
                const int yy = gy + d;
                if (yy < 0 || yy >= H) continue;
                const double wd = hdr->blur_w[d < 0 ? -d : d];
                s += wd * hp[ty + R + d][tx];
                ws += wd;
            }
            J.score[(size_t)gy * W + gx] = (float)(s / ws);
        }
    }
}

}  // namespace

#define QFCA_BATCH_ALL_T(X) X(3) X(5) X(7) X(9) X(11) X(13) X(15) X(17) X(19) X(21) X(23) X(25) X(27) X(29) X(31)

size_t batch_wave_lds(int T, int S, int Ws) {
    switch (T) {
#define QFCA_BL(TT) case TT: return BLayout<TT>(S, Ws).total;
        QFCA_BATCH_ALL_T(QFCA_BL)
#undef QFCA_BL
        default: return 0;
    }
}

bool batch_combo(int C, int k, int prec, int* CM, int* KT) {
    static const int f32[3][2] = {{64, 1}, {256, 2}, {512, 4}};
    static const int bf16[2][2] = {{256, 2}, {512, 4}};
    const bool bf = prec == QFCA_PREC_BF16;
    const int n = bf ? 2 : 3;
    if (C < 1 || k < 1 || k > 64) return false;
    for (int i = 0; i < n; ++i) {
        const int cm = bf ? bf16[i][0] : f32[i][0], kt = bf ? bf16[i][1] : f32[i][1];
        if (cm >= C && 16 * kt >= k) {
            *CM = cm;
            *KT = kt;
            return true;
        }
    }
    return false;
}

bool batch_supported(int T, int CMAX, int KT, int prec) {
    if (T < 3 || T > 31 || !(T & 1)) return false;
    if (prec == QFCA_PREC_BF16) return (CMAX == 256 && KT == 2) || (CMAX == 512 && KT == 4);
    return (CMAX == 64 && KT == 1) || (CMAX == 256 && KT == 2) || (CMAX == 512 && KT == 4);
}

size_t batch_proj_lds(int CMAX, int KT) { return (size_t)4 * CMAX * 4 + (size_t)4 * KT * 4 * 64 * 4; }

size_t batch_head_bytes(int T) { return score_rcp_bytes(T) + BATCH_CTL_BYTES; }

// Dispatch over T to the instantiation of qfca_batch_t*.hip.
static hipError_t batch_main_any(int T, int CMAX, int KT, int prec, BatchHeader* hdr, const BatchJob* jobs,
                                 int wave_lds, size_t lds, int grid, hipStream_t st, bool prepare_only) {
    const bool bf = prec == QFCA_PREC_BF16;
    switch (T) {
#define QFCA_BM(TT) \
        case TT: return batchk::batch_main<TT>(CMAX, KT, bf, hdr, jobs, wave_lds, lds, grid, st, prepare_only);
        QFCA_BATCH_ALL_T(QFCA_BM)
#undef QFCA_BM
        default: return hipErrorInvalidValue;
    }
}

// Allows the kernel's dynamic LDS and checks that it has no static LDS (its
// reciprocal table is addressed as LDS address 0).
hipError_t prepare_batch(int T, int CMAX, int KT, int prec, size_t lds) {
    return batch_main_any(T, CMAX, KT, prec, nullptr, nullptr, 0, lds, 0, nullptr, true);
}

hipError_t launch_batch(int T, int CMAX, int KT, int prec, BatchHeader* hdr, const BatchJob* jobs,
                        int wave_lds, size_t lds, int grid, int maxn, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_reset, dim3((maxn + 255) / 256), dim3(256), 0, st, hdr, maxn);
    hipError_t e = batch_main_any(T, CMAX, KT, prec, hdr, jobs, wave_lds, lds, grid, st, false);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_blur, dim3(256, 1, maxn), dim3(256), 0, st, (const BatchHeader*)hdr, jobs);
    return hipGetLastError();
}

}  // namespace qfca
