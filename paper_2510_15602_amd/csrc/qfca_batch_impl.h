// Persistent batch kernel templates (internal header of libqfca): one
// instantiation per window side T, channel padding CMAX, component tiles KT
// and projection precision.  Each T is instantiated in its own translation
// unit (qfca_batch_t*.hip) through QFCA_BATCH_INSTANTIATE, so the kernels
// compile in parallel.
#pragma once
#include "qfca_internal.h"
#include "qfca_tiles.h"

namespace qfca {
namespace batchk {
using namespace tiles;

constexpr int SPIN_LIMIT = 1 << 22;

__device__ inline int find_job(const int* prefix, int n, int item) {
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
                const float vf = ok ? J.pa.fastd[i] : INFINITY;
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
                score_tile<T, true, true>(J.sa, bx, by * J.sa.Hb, min(J.sa.H, (by + 1) * J.sa.Hb), 4 * gz + w, lane,
                                          smem + (size_t)w * wave_lds, rcp4);
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

// Launches (or, with prepare_only, prepares: allows the dynamic LDS and
// checks that the kernel has no static LDS) the persistent kernel for
// (T, CMAX, KT, precision); hipErrorInvalidValue for a shape with no
// instantiation.
template <int T>
hipError_t batch_main(int CMAX, int KT, bool bf, BatchHeader* hdr, const BatchJob* jobs, int wave_lds,
                      size_t lds, int grid, hipStream_t st, bool prepare_only) {
    auto go = [&](const void* k, auto launch) -> hipError_t {
        if (prepare_only) {
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            hipFuncAttributes fa;
            e = hipFuncGetAttributes(&fa, k);
            if (e != hipSuccess) return e;
            return fa.sharedSizeBytes == 0 ? hipSuccess : hipErrorInvalidDeviceFunction;
        }
        launch();
        return hipGetLastError();
    };
#define QFCA_BMAIN(CM, KK, BFV)                                                                    \
    if (CMAX == CM && KT == KK && bf == BFV) {                                                     \
        const void* k = batch_kernel<T, CM, KK, BFV>();                                            \
        return go(k, [&] {                                                                         \
            if constexpr (T <= BATCH_TWO_WAVES_MAX_T)                                              \
                hipLaunchKernelGGL((k_batch2<T, CM, KK, BFV>), dim3(grid), dim3(256), lds, st, hdr, jobs, \
                                   wave_lds);                                                      \
            else                                                                                   \
                hipLaunchKernelGGL((k_batch1<T, CM, KK, BFV>), dim3(grid), dim3(256), lds, st, hdr, jobs, \
                                   wave_lds);                                                      \
        });                                                                                        \
    }
    QFCA_BMAIN(64, 1, false) QFCA_BMAIN(256, 2, false) QFCA_BMAIN(512, 4, false)
    QFCA_BMAIN(256, 2, true) QFCA_BMAIN(512, 4, true)
#undef QFCA_BMAIN
    return hipErrorInvalidValue;
}

}  // namespace batchk
}  // namespace qfca

#define QFCA_BATCH_INSTANTIATE(TT)                                                                   \
    template hipError_t qfca::batchk::batch_main<TT>(int, int, bool, qfca::BatchHeader*,              \
                                                     const qfca::BatchJob*, int, size_t, int, hipStream_t, bool);
