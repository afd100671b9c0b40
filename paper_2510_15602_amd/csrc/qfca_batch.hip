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

#include "qfca_internal.h"
#include "qfca_tiles.h"

namespace qfca {

namespace {
using namespace tiles;

constexpr int SPIN_LIMIT = 1 << 22;

__global__ void k_batch_reset(BatchHeader* h, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        h->head = 0;
        h->error = 0;
    }
    if (i < n) h->done[i] = 0;
}

__device__ int find_job(const int* prefix, int n, int item) {
    // largest j with prefix[j] <= item (prefix[0] = 0, nondecreasing)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int T, int CMAX, int KT, bool BF>
__device__ __forceinline__ void batch_body(BatchHeader* hdr, const BatchJob* jobs, int wave_lds) {
    // LDS: the block-shared reciprocal table of the score tiles (it depends
    // on T only), the block's control words (item, job, ready flag), then
    // either the projection scratch or 4 wave regions.  The kernel declares
    // no static LDS (prepare_batch checks it), so the table sits at LDS
    // address 0.
    extern __shared__ __align__(16) unsigned char smem_all[];
    constexpr size_t RCP = BLayout<T>::RCP_BYTES;
    float* rcp4 = (float*)smem_all;
    int* ctl = (int*)(smem_all + RCP);
    int& s_item = ctl[0];
    int& s_job = ctl[1];
    int& s_ok = ctl[2];
    unsigned char* smem = smem_all + RCP + BATCH_CTL_BYTES;
    // the wavefront index is uniform across the wavefront: held in a scalar
    // register, offsets derived from it fold into instruction offsets
    const int lane0 = threadIdx.x & 63, w0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = hdr->n, nproj = hdr->nproj, nitems = hdr->nitems;
    if (n > 0) fill_rcp4<T>(rcp4, jobs[0].sa.rcp, threadIdx.x, 256);
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) {
            const int it = atomicAdd(&hdr->head, 1);
            s_item = it;
            s_job = it < nproj ? find_job(hdr->proj_prefix, n, it)
                               : (it < nitems ? find_job(hdr->score_prefix, n, it - nproj) : 0);
        }
        __syncthreads();
        const int item = s_item, jb = s_job;
        if (item >= nitems) break;
        // lane-derived values are recomputed per item rather than held in
        // registers across items (the hidden copies keep them from being hoisted)
        int lane = lane0, w = w0;
        asm volatile("" : "+v"(lane), "+s"(w));
        const BatchJob& J = jobs[jb];
        if (item < nproj) {
            const int tile = item - hdr->proj_prefix[jb];
            float* smu = (float*)smem;
            float* slo = smu + CMAX;
            float* sid = slo + CMAX;
            float* sfd = sid + CMAX;
            float* zp = sfd + CMAX;
            for (int i = threadIdx.x; i < CMAX; i += 256) {
                // loads before stores (see proj_prologue)
                const bool ok = i < J.pa.C;
                const float vm = ok ? J.pa.mu[i] : 0.f;
                const float vl = ok ? J.pa.lo[i] : 0.f;
                const float vi = ok ? J.pa.inv_delta[i] : 0.f;
                const float vf = ok ? J.pa.fastd[i] : 1.f;
                smu[i] = vm;
                slo[i] = vl;
                sid[i] = vi;
                sfd[i] = vf;
            }
            __syncthreads();
            if constexpr (BF) {
                float x[CMAX / 128][8];
                proj_load_bf16<CMAX>(J.pa, tile, w, lane, x);
                proj_tile_bf16<CMAX, KT>(J.pa, tile, w, lane, (const bf16x8*)J.pa.V1, (const bf16x8*)J.pa.V2,
                                         smu, slo, sid, sfd, zp, x, J.pa.edges, nullptr);
            } else {
                float x[CMAX / 16];
                proj_load_f32<CMAX>(J.pa, tile, w, lane, x);
                proj_tile_f32<CMAX, KT>(J.pa, tile, w, lane, (const float*)J.pa.V1, (const float*)J.pa.V2,
                                        smu, slo, sid, sfd, zp, x, J.pa.edges, nullptr);
            }
            // the tile's pixels start the image's fixed-point channel sum at 0
            // (published with the bins by the release below)
            if (threadIdx.x < 16) {
                const int px = tile * 16 + threadIdx.x;
                if (px < J.pa.N) J.asum[px] = 0;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                __threadfence();
                atomicAdd(&hdr->done[jb], 1);
            }
        } else {
            const int local = item - nproj - hdr->score_prefix[jb];
            if (threadIdx.x == 0) {
                const int need = J.ntiles_proj;
                int ok = 0;
                for (int sp = 0; sp < SPIN_LIMIT; ++sp) {
                    if (__hip_atomic_load(&hdr->done[jb], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= need) {
                        ok = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
                if (!ok) atomicOr(&hdr->error, 1);
                s_ok = ok;
            }
            __syncthreads();
            __threadfence();
            if (s_ok) {
                // local = ((gz * nbands) + by) * nstrips + bx
                const int bx = local % J.nstrips;
                const int rest = local / J.nstrips;
                const int by = rest % J.nbands;
                const int gz = rest / J.nbands;
                score_tile<T, true, true>(J.sa, bx, by, 4 * gz + w, lane, smem + (size_t)w * wave_lds, rcp4);
            }
        }
        __syncthreads();
    }
}

// The persistent kernel.  Up to T = 15 the register budget is held to two
// wavefronts per SIMD (the projection and score tiles then fit without
// spilling); larger windows keep the full register file.
constexpr int BATCH_TWO_WAVES_MAX_T = 15;

template <int T, int CMAX, int KT, bool BF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_batch2(
        BatchHeader* hdr, const BatchJob* jobs, int wave_lds) {
    batch_body<T, CMAX, KT, BF>(hdr, jobs, wave_lds);
}

template <int T, int CMAX, int KT, bool BF>
__global__ __launch_bounds__(256) void k_batch1(BatchHeader* hdr, const BatchJob* jobs, int wave_lds) {
    batch_body<T, CMAX, KT, BF>(hdr, jobs, wave_lds);
}

template <int T, int CMAX, int KT, bool BF>
const void* batch_kernel() {
    if constexpr (T <= BATCH_TWO_WAVES_MAX_T) return (const void*)k_batch2<T, CMAX, KT, BF>;
    else return (const void*)k_batch1<T, CMAX, KT, BF>;
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

template <int T, int CMAX, int KT, bool BF>
hipError_t run_batch(BatchHeader* hdr, const BatchJob* jobs, int wave_lds, size_t lds, int grid,
                     int maxn, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_reset, dim3((maxn + 255) / 256), dim3(256), 0, st, hdr, maxn);
    if constexpr (T <= BATCH_TWO_WAVES_MAX_T)
        hipLaunchKernelGGL((k_batch2<T, CMAX, KT, BF>), dim3(grid), dim3(256), lds, st, hdr, jobs, wave_lds);
    else
        hipLaunchKernelGGL((k_batch1<T, CMAX, KT, BF>), dim3(grid), dim3(256), lds, st, hdr, jobs, wave_lds);
    hipLaunchKernelGGL(k_batch_blur, dim3(256, 1, maxn), dim3(256), 0, st, (const BatchHeader*)hdr, jobs);
    return hipGetLastError();
}

}  // namespace

size_t batch_wave_lds(int T, int S, int Ws) {
    switch (T) {
#define QFCA_BL(TT) case TT: return BLayout<TT>(S, Ws).total;
        QFCA_BL(5) QFCA_BL(7) QFCA_BL(9) QFCA_BL(11) QFCA_BL(15) QFCA_BL(31)
#undef QFCA_BL
        default: return 0;
    }
}

bool batch_supported(int T, int CMAX, int KT, int prec) {
    const bool t_ok = T == 5 || T == 7 || T == 9 || T == 11 || T == 15 || T == 31;
    if (!t_ok) return false;
    if (prec == QFCA_PREC_BF16) return (CMAX == 256 && KT == 2) || (CMAX == 512 && KT == 4);
    return (CMAX == 64 && KT == 1) || (CMAX == 256 && KT == 2) || (CMAX == 512 && KT == 4);
}

size_t batch_proj_lds(int CMAX, int KT) { return (size_t)4 * CMAX * 4 + (size_t)4 * KT * 4 * 64 * 4; }

// Allows the kernel's dynamic LDS and checks that it has no static LDS (its
// reciprocal table is addressed as LDS address 0).
static hipError_t prepare_kernel(const void* k, size_t lds) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipFuncAttributes fa;
    e = hipFuncGetAttributes(&fa, k);
    if (e != hipSuccess) return e;
    return fa.sharedSizeBytes == 0 ? hipSuccess : hipErrorInvalidDeviceFunction;
}

size_t batch_head_bytes(int T) { return score_rcp_bytes(T) + BATCH_CTL_BYTES; }

hipError_t prepare_batch(int T, int CMAX, int KT, int prec, size_t lds) {
    const bool bf = prec == QFCA_PREC_BF16;
#define QFCA_PREP_CASE(TT, CM, KK, BFV)                                                    \
    if (T == TT && CMAX == CM && KT == KK && bf == BFV)                                    \
        return prepare_kernel(batch_kernel<TT, CM, KK, BFV>(), lds);
#define QFCA_PREP_T(TT) QFCA_PREP_CASE(TT, 64, 1, false) QFCA_PREP_CASE(TT, 256, 2, false) \
    QFCA_PREP_CASE(TT, 512, 4, false) QFCA_PREP_CASE(TT, 256, 2, true) QFCA_PREP_CASE(TT, 512, 4, true)
    QFCA_PREP_T(5) QFCA_PREP_T(7) QFCA_PREP_T(9) QFCA_PREP_T(11) QFCA_PREP_T(15) QFCA_PREP_T(31)
#undef QFCA_PREP_T
#undef QFCA_PREP_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_batch(int T, int CMAX, int KT, int prec, BatchHeader* hdr, const BatchJob* jobs,
                        int wave_lds, size_t lds, int grid, int maxn, hipStream_t st) {
    const bool bf = prec == QFCA_PREC_BF16;
#define QFCA_BATCH_CASE(TT, CM, KK, BFV)                                                   \
    if (T == TT && CMAX == CM && KT == KK && bf == BFV)                                    \
        return run_batch<TT, CM, KK, BFV>(hdr, jobs, wave_lds, lds, grid, maxn, st);
#define QFCA_BATCH_T(TT) QFCA_BATCH_CASE(TT, 64, 1, false) QFCA_BATCH_CASE(TT, 256, 2, false) \
    QFCA_BATCH_CASE(TT, 512, 4, false) QFCA_BATCH_CASE(TT, 256, 2, true) QFCA_BATCH_CASE(TT, 512, 4, true)
    QFCA_BATCH_T(5) QFCA_BATCH_T(7) QFCA_BATCH_T(9) QFCA_BATCH_T(11) QFCA_BATCH_T(15) QFCA_BATCH_T(31)
#undef QFCA_BATCH_T
#undef QFCA_BATCH_CASE
    return hipErrorInvalidValue;
}

}  // namespace qfca
