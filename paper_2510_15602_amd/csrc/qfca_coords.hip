// Principal coordinates and their bins for gfx950: z = V^T (x - mu) (the
// "PCA(W)" of Sec. 3.3 taken as the histogrammed quantity), then
// bin = #{m : z_j >= edge_{j,m}} per coordinate j.  The variant of the method
// that histograms the k coordinates instead of the C residual channels and
// scores each window by its 1-Wasserstein distance to the reference.
//
// The product is the first GEMM of the residual projection (qfca_proj.hip)
// alone: one block of four wavefronts owns a 16-pixel tile, wave w forms the
// partial Z of its channel quarter on MFMA (FP32 v_mfma_f32_16x16x4f32 or
// BF16 v_mfma_f32_16x16x32_bf16 with FP32 accumulation), the partials are
// added through LDS in a fixed order, and wave w < KT then quantises the 16
// components 16 w .. 16 w + 15 of the 16 pixels.  The grid is persistent
// (contiguous runs of tiles per block), the operand table sits in LDS, and
// the next tile's features are loaded while the current one is computed.
// The only HBM traffic is the features in (4 C bytes per pixel) and k bytes
// of bins out (plus 4 k bytes of coordinates when they are asked for).
#include <algorithm>
#include <atomic>

#include "qfca_internal.h"
#include "qfca_tiles.h"

namespace qfca {
namespace {
using namespace tiles;

constexpr size_t CO_LDS_MAX = 160 * 1024;
constexpr size_t CO_LDS_TWO_BLOCKS = 80 * 1024;

// LDS: mu [CMAX]; lo, 1/delta, margin [64] each; Z partials [4][KT][4][64];
// bin staging [64][16] bytes; the operand table.
__host__ __device__ inline size_t co_lds(int CMAX, int KT, int elt) {
    return (size_t)CMAX * 4 + 3 * 64 * 4 + (size_t)4 * KT * 4 * 64 * 4 + 64 * 16 + (size_t)CMAX * KT * 16 * elt;
}

// Quantises the 16 components of wave w (< KT) for the tile's 16 pixels
// from the reduced Z (register v of lane (g, n): component 16 w + 4 g + v,
// pixel n) and stores the bins (and the coordinates when a.resid is set).
__device__ __forceinline__ void co_emit(const MArgs& a, int tile, int w, int lane, const floatx4& zw,
                                        const float* slo, const float* sid, const float* sfd, uint8_t* stg) {
    const int g = lane >> 4, n = lane & 15;
    const int px = tile * 16 + n;
    int cs[4];
    float rv[4];
    bool valid[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int j = 16 * w + 4 * g + v;
        cs[v] = j;
        rv[v] = zw[v];
        valid[v] = px < a.N && j < a.k;
    }
    emit_values<4>(a, px, cs, rv, valid, slo, sid, sfd, a.edges, stg);
}

// Bins of the tile from the staging area, one 16-byte row per component.
__device__ __forceinline__ void co_store(const MArgs& a, int tile, const uint8_t* stg) {
    const int p0 = tile * 16;
    const int j = threadIdx.x;
    if (j >= a.k) return;
    if (p0 + 16 <= a.N && (a.N & 15) == 0 && (((uintptr_t)a.bins & 15) == 0)) {
        *(uint4*)(a.bins + (size_t)j * a.N + p0) = *(const uint4*)(stg + j * 16);
    } else {
        uint8_t* dst = a.bins + (size_t)j * a.N + p0;
        for (int q = 0; q < 16 && p0 + q < a.N; ++q) dst[q] = stg[j * 16 + q];
    }
}

template <int CMAX, int KT, bool BF>
__device__ __forceinline__ void coords_body(const MArgs& a) {
    constexpr int ELT = BF ? 2 : 4;
    constexpr int VSZ = CMAX * KT * 16;  // table elements
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float* smu = (float*)lds_raw;
    float* slo = smu + CMAX;
    float* sid = slo + 64;
    float* sfd = sid + 64;
    float* zp = sfd + 64;  // [4 waves][KT][4][64]
    uint8_t* stg = (uint8_t*)(zp + 4 * KT * 4 * 64);
    void* stab = stg + 64 * 16;
    for (int i = threadIdx.x; i < CMAX; i += blockDim.x) {
        const float vm = i < a.C ? a.mu[i] : 0.f;
        smu[i] = vm;
    }
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        const bool ok = i < a.k;
        const float vl = ok && a.lo ? a.lo[i] : 0.f;
        const float vi = ok && a.inv_delta ? a.inv_delta[i] : 0.f;
        const float vf = ok && a.fastd ? a.fastd[i] : INFINITY;
        slo[i] = vl;
        sid[i] = vi;
        sfd[i] = vf;
    }
    {
        const uint4* src = (const uint4*)a.V1;
        uint4* dst = (uint4*)stab;
        constexpr int NU = VSZ * ELT / 16;
        for (int u = threadIdx.x; u < NU; u += blockDim.x) dst[u] = src[u];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int per = (a.ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    int tile = blockIdx.x * per;
    const int tend = min(a.ntiles, tile + per);
    if constexpr (BF) {
        constexpr int NSW = CMAX / 128;
        float x[NSW][8];
        if (tile < tend) proj_load_bf16<CMAX>(a, tile, w, lane, x);
        for (; tile < tend; ++tile) {
            int lt = lane, wt = w;
            asm volatile("" : "+v"(lt), "+s"(wt));
            float xn[NSW][8];
            const int nt = tile + 1;
            proj_load_bf16<CMAX>(a, nt < tend ? nt : tend - 1, wt, lt, xn);
            const bf16x8* V1 = opaque_lds((const bf16x8*)stab);
            const int g = lt >> 4, n = lt & 15;
            floatx4 z[KT];
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) z[kt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < NSW; ++i) {
                const int s = wt * NSW + i;
                bf16x8 bv;
#pragma unroll
                for (int t = 0; t < 8; ++t) bv[t] = (__bf16)(x[i][t] - smu[32 * s + 8 * g + t]);
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
                    z[kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(V1[((s * KT + kt) * 4 + g) * 16 + n], bv,
                                                                    z[kt], 0, 0, 0);
            }
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                for (int v = 0; v < 4; ++v) zp[((wt * KT + kt) * 4 + v) * 64 + lt] = z[kt][v];
            block_sync_lds();
            if (wt < KT) {
                floatx4 zw;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float acc = zp[((0 * KT + wt) * 4 + v) * 64 + lt];
                    acc += zp[((1 * KT + wt) * 4 + v) * 64 + lt];
                    acc += zp[((2 * KT + wt) * 4 + v) * 64 + lt];
                    acc += zp[((3 * KT + wt) * 4 + v) * 64 + lt];
                    zw[v] = acc;
                }
                co_emit(a, tile, wt, lt, zw, opaque_lds(slo), opaque_lds(sid), opaque_lds(sfd), stg);
            }
            block_sync_lds();
            if (a.bins) co_store(a, tile, stg);
#pragma unroll
            for (int i = 0; i < NSW; ++i)
#pragma unroll
                for (int t = 0; t < 8; ++t) x[i][t] = xn[i][t];
        }
    } else {
        constexpr int NSW = CMAX / 16;
        float x[NSW];
        if (tile < tend) proj_load_f32<CMAX>(a, tile, w, lane, x);
        for (; tile < tend; ++tile) {
            int lt = lane, wt = w;
            asm volatile("" : "+v"(lt), "+s"(wt));
            float xn[NSW];
            const int nt = tile + 1;
            proj_load_f32<CMAX>(a, nt < tend ? nt : tend - 1, wt, lt, xn);
            const float* V1 = opaque_lds((const float*)stab);
            const int g = lt >> 4, n = lt & 15;
            floatx4 z[KT];
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) z[kt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < NSW; ++i) {
                const int s = wt * NSW + i;
                const float d = x[i] - smu[4 * s + g];
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
                    z[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(V1[((s * KT + kt) * 4 + g) * 16 + n], d, z[kt], 0,
                                                                 0, 0);
                if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                for (int v = 0; v < 4; ++v) zp[((wt * KT + kt) * 4 + v) * 64 + lt] = z[kt][v];
            block_sync_lds();
            if (wt < KT) {
                floatx4 zw;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float acc = zp[((0 * KT + wt) * 4 + v) * 64 + lt];
                    acc += zp[((1 * KT + wt) * 4 + v) * 64 + lt];
                    acc += zp[((2 * KT + wt) * 4 + v) * 64 + lt];
                    acc += zp[((3 * KT + wt) * 4 + v) * 64 + lt];
                    zw[v] = acc;
                }
                co_emit(a, tile, wt, lt, zw, opaque_lds(slo), opaque_lds(sid), opaque_lds(sfd), stg);
            }
            block_sync_lds();
            if (a.bins) co_store(a, tile, stg);
#pragma unroll
            for (int i = 0; i < NSW; ++i) x[i] = xn[i];
        }
    }
}

template <int CMAX, int KT, bool BF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_coords(MArgs a) {
    coords_body<CMAX, KT, BF>(a);
}

// Whole-tile kernel for 512 channels in BF16: every wavefront computes the
// full Z of its own 16-pixel tiles (all channels, so no partials are added
// across wavefronts), sixteen wavefronts per block (four per SIMD) share the
// operand table and the parameters in LDS, and a block's wavefronts take
// interleaved tiles of one contiguous run, meeting at a bare barrier at the
// start of each round.
// The centred features are not needed after the product, so they stream
// through a ring of PF + 1 register groups: step s + PF is loaded while step
// s is multiplied.  Lane (g, n) ends with components 16 kt + 4 g + v of pixel
// n; the bins of those four consecutive components are packed in a dword,
// byte-transposed across each lane quad and written four pixels per dword.
// LDS: mu [CMAX]; lo, 1/delta, margin [64] each; the operand table.
// CS_WAVES wavefronts per block, CS_BLOCKS blocks per compute unit (four
// wavefronts per SIMD; two blocks of ten, five per SIMD, ran no faster and
// spilled).
constexpr int CS_WAVES = 16, CS_BLOCKS = 1;
__host__ __device__ inline size_t cs_lds(int CMAX, int KT) {
    return (size_t)4 * CMAX + 3 * 64 * 4 + (size_t)CMAX * KT * 16 * 2;
}

template <int CMAX, int KT, int NW, int WPE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void k_coords_solo(MArgs a) {
    constexpr int NS = CMAX / 32;        // product K steps (32 channels each)
    constexpr int QS = NS / 4;           // K steps of one quarter (one wavefront's share in k_coords)
    constexpr int VSZ = CMAX * KT * 16;  // bf16 table elements
    constexpr int PF = 4;                // steps of features in flight ahead
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float* smu = (float*)lds_raw;
    float* slo = smu + CMAX;
    float* sid = slo + 64;
    float* sfd = sid + 64;
    bf16x8* stab = (bf16x8*)(lds_raw + 4 * CMAX + 3 * 64 * 4);
    for (int i = threadIdx.x; i < CMAX; i += blockDim.x) {
        const float vm = i < a.C ? a.mu[i] : 0.f;
        smu[i] = vm;
    }
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        const bool ok = i < a.k;
        const float vl = ok && a.lo ? a.lo[i] : 0.f;
        const float vi = ok && a.inv_delta ? a.inv_delta[i] : 0.f;
        const float vf = ok && a.fastd ? a.fastd[i] : INFINITY;
        slo[i] = vl;
        sid[i] = vi;
        sfd[i] = vf;
    }
    {
        constexpr int NUNIT = VSZ / 8;
        const uint4* src = (const uint4*)a.V1;
        uint4* dst = (uint4*)stab;
        for (int u0 = threadIdx.x; u0 < NUNIT; u0 += 4 * 64 * NW) {
            uint4 t[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (u0 + 64 * NW * i < NUNIT) t[i] = src[u0 + 64 * NW * i];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (u0 + 64 * NW * i < NUNIT) dst[u0 + 64 * NW * i] = t[i];
        }
    }
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int per = ((a.ntiles + (int)gridDim.x - 1) / (int)gridDim.x + NW - 1) / NW * NW;
    const int b0 = (int)blockIdx.x * per;
    const int tend = min(a.ntiles, b0 + per);
    const bool rows_dw = ((a.N & 3) == 0) && (((uintptr_t)a.bins & 3) == 0);
    // every wavefront of the block runs the same number of rounds and meets
    // the others at the start of each (a bare barrier), so the block's
    // stores to a line of bins come close together in time
    const int nround = tend > b0 ? (tend - b0 + NW - 1) / NW : 0;
    int tile = b0 + w;
    for (int rd = 0; rd < nround; ++rd, tile += NW) {
        __builtin_amdgcn_s_barrier();
        if (tile >= tend) continue;
        // lane index and bases opaque per tile (nothing lane- or base-derived
        // is hoisted out of the loop into registers)
        int lane = threadIdx.x & 63;
        asm volatile("" : "+v"(lane));
        const float* Xt = a.X;
        float* Rt = a.resid;
        uint8_t* Bt = a.bins;
        const float* Et = a.edges;
        asm volatile("" : "+s"(Xt), "+s"(Rt), "+s"(Bt), "+s"(Et));
        const int g = lane >> 4, n = lane & 15, p = n & 3, qd = n >> 2;
        const uint32_t selA = (p & 1) ? 0x07030501u : 0x02060004u;
        const uint32_t selB = (p & 2) ? 0x07060302u : 0x01000504u;
        const int px = tile * 16 + n;
        const bool pxok = px < a.N;
        const int pxc = pxok ? px : a.N - 1;
        // channel 32 s + t + 8 g of pixel pxc: the uniform row base of channel
        // 32 s + t plus the lane's 32-bit byte offset (channels past C read a
        // real row; their table rows are zero)
        const uint32_t voff = ((uint32_t)(8 * g) * (uint32_t)a.N + (uint32_t)pxc) * 4u;
        const uint32_t voff0 = (uint32_t)pxc * 4u;
        float ring[PF + 1][8];
        auto load = [&](auto sc) __attribute__((always_inline)) {
            constexpr int s = decltype(sc)::value;
            if constexpr (s < NS) {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int cu = 32 * s + t;
                    const char* rb = (const char*)(Xt + (size_t)(cu < a.C ? cu : a.C - 1) * a.N);
                    ring[s % (PF + 1)][t] = *(const float*)(rb + (cu + 8 * g < a.C ? voff : voff0));
                }
            }
        };
        StaticFor<0, PF>::run(load);
        const bf16x8* V1 = opaque_lds((const bf16x8*)stab);
        const float* mu = opaque_lds((const float*)smu);
        // Z in the order of the block-split kernel: four quarters of the K
        // steps, each a chain from zero, the quarters added in order
        floatx4 z[KT], zq[KT];
        auto step = [&](auto sc) __attribute__((always_inline)) {
            constexpr int s = decltype(sc)::value;
            if constexpr (s % QS == 0) {
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) zq[kt] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
            load(std::integral_constant<int, s + PF>{});
            const float4 m0 = *(const float4*)(mu + 32 * s + 8 * g);
            const float4 m1 = *(const float4*)(mu + 32 * s + 8 * g + 4);
            const float mv[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
            bf16x8 bv;
#pragma unroll
            for (int t = 0; t < 8; ++t) bv[t] = (__bf16)(ring[s % (PF + 1)][t] - mv[t]);
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
                zq[kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(V1[((s * KT + kt) * 4 + g) * 16 + n], bv, zq[kt], 0,
                                                                 0, 0);
            if constexpr (s % QS == QS - 1) {
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) z[kt][v] = (s == QS - 1) ? zq[kt][v] : z[kt][v] + zq[kt][v];
            }
        };
        StaticFor<0, NS>::run(step);
        const float* plo = opaque_lds((const float*)slo);
        const float* pid = opaque_lds((const float*)sid);
        const float* pfd = opaque_lds((const float*)sfd);
        const int B = a.B;
        const float top = (float)max(B - 1, 0);
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            const int j0 = 16 * kt + 4 * g;  // components j0 .. j0 + 3 of pixel px
            if (Rt) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (pxok && j0 + v < a.k) Rt[(size_t)(j0 + v) * a.N + px] = z[kt][v];
            }
            if (!Bt) continue;
            const float4 l4 = *(const float4*)(plo + j0);
            const float4 i4 = *(const float4*)(pid + j0);
            const float4 f4 = *(const float4*)(pfd + j0);
            const float lov[4] = {l4.x, l4.y, l4.z, l4.w};
            const float idv[4] = {i4.x, i4.y, i4.z, i4.w};
            const float dlv[4] = {f4.x, f4.y, f4.z, f4.w};
            uint32_t bq[4];
            uint32_t need = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float tt = (z[kt][v] - lov[v]) * idv[v];
                const float near = __builtin_amdgcn_fmed3f(rintf(tt), 1.f, top);
                const bool dec = fabsf(tt - near) >= dlv[v];  // +infinity: the shortcut is off
                bq[v] = (uint32_t)__builtin_amdgcn_fmed3f(floorf(tt), 0.f, top);
                need |= ((!dec) & pxok & (j0 + v < a.k) & (B > 1)) ? (1u << v) : 0u;
            }
            if (__ballot(need != 0u)) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (need & (1u << v))
                        bq[v] = (uint32_t)bin_fast(z[kt][v], Et + (size_t)(j0 + v) * (B - 1), lov[v], idv[v], B);
            }
            const uint32_t tr = quad_transpose_bytes(bq[0] | (bq[1] << 8) | (bq[2] << 16) | (bq[3] << 24), selA, selB);
            // lane (g, 4 qd + p): component j0' + p, pixels 4 qd .. 4 qd + 3
            const int jw = 16 * kt + 4 * g + p;
            const int pw = tile * 16 + 4 * qd;
            if (jw < a.k) {
                uint8_t* dst = Bt + (size_t)jw * a.N + pw;
                if (rows_dw && pw + 3 < a.N) {
                    *(uint32_t*)dst = tr;
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (pw + i < a.N) dst[i] = (uint8_t)(tr >> (8 * i));
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_coords(const ProjLaunch& L, hipStream_t st) {
    const int CM = mfma_cmax(L.C, L.prec), KT = mfma_kt(L.k, L.prec);
    if (!CM || !KT || !L.V1 || L.k > 64) return hipErrorInvalidValue;
    MArgs a;
    a.X = L.X; a.C = L.C; a.N = L.N; a.k = L.k; a.B = L.B;
    a.mu = L.mu; a.V1 = L.V1; a.V2 = nullptr;
    a.edges = L.edges; a.lo = L.lo; a.inv_delta = L.inv_delta; a.fastd = L.fastd;
    a.bins = L.bins; a.resid = L.resid;
    a.ntiles = (L.N + 15) / 16;
    const bool bf = L.prec == QFCA_PREC_BF16;
    if (bf && CM == 512 && (KT == 2 || KT == 4) && (unsigned long long)L.N * 100ULL < (1ULL << 32)) {
        // whole tiles per wavefront (32-bit lane offsets of the feature loads)
        int ncu = 0, dev0 = 0;
        hipError_t e0 = hipGetDevice(&dev0);
        if (e0 != hipSuccess) return e0;
        if ((e0 = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev0)) != hipSuccess) return e0;
        const size_t lds = cs_lds(CM, KT);
        constexpr int NW = CS_WAVES;
        constexpr int WPE = NW * CS_BLOCKS / 4;
        const void* kf =
            KT == 4 ? (const void*)k_coords_solo<512, 4, NW, WPE> : (const void*)k_coords_solo<512, 2, NW, WPE>;
        if ((e0 = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
            return e0;
        const int blocks = std::max(1, std::min((a.ntiles + NW - 1) / NW, ncu * CS_BLOCKS));
        if (KT == 4)
            hipLaunchKernelGGL((k_coords_solo<512, 4, NW, WPE>), dim3(blocks), dim3(64 * NW), lds, st, a);
        else
            hipLaunchKernelGGL((k_coords_solo<512, 2, NW, WPE>), dim3(blocks), dim3(64 * NW), lds, st, a);
        return hipGetLastError();
    }
    const size_t lds = co_lds(CM, KT, bf ? 2 : 4);
    if (lds > CO_LDS_MAX) return hipErrorInvalidValue;
    static std::atomic<int> ncu_cache[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int ncu = ncu_cache[dev & 63].load(std::memory_order_relaxed);
    if (!ncu) {
        e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        ncu_cache[dev & 63].store(ncu, std::memory_order_relaxed);
    }
    const int per_cu = lds <= CO_LDS_TWO_BLOCKS ? 2 : 1;
    const int grid = std::max(1, std::min(a.ntiles, ncu * per_cu));
    auto go = [&](const void* k, auto launch) -> hipError_t {
        if (lds > 65536) {
            hipError_t e2 = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e2 != hipSuccess) return e2;
        }
        launch();
        return hipGetLastError();
    };
#define QFCA_CO(CMV, KTV, BFV)                                                                   \
    if (CM == CMV && KT == KTV && bf == BFV)                                                     \
        return go((const void*)k_coords<CMV, KTV, BFV>,                                          \
                  [&] { hipLaunchKernelGGL((k_coords<CMV, KTV, BFV>), dim3(grid), dim3(256), lds, st, a); });
    QFCA_CO(64, 1, false) QFCA_CO(64, 2, false) QFCA_CO(64, 4, false)
    QFCA_CO(128, 1, false) QFCA_CO(128, 2, false) QFCA_CO(128, 4, false)
    QFCA_CO(256, 1, false) QFCA_CO(256, 2, false) QFCA_CO(256, 4, false)
    QFCA_CO(512, 1, false) QFCA_CO(512, 2, false) QFCA_CO(512, 4, false)
    QFCA_CO(128, 2, true) QFCA_CO(128, 4, true) QFCA_CO(256, 2, true) QFCA_CO(256, 4, true)
    QFCA_CO(512, 2, true) QFCA_CO(512, 4, true)
#undef QFCA_CO
    return hipErrorInvalidValue;
}

}  // namespace qfca
