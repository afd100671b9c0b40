// Projection + quantisation on MFMA for gfx950 (Sec. 3.3 residual, Sec. 3.1
// bins): r = (x - mu) - V (V^T (x - mu)), then bin = #{m : r >= edge_m}.
//
// One wavefront owns 16 pixels.  Their centred features d stay in registers
// for the whole pixel tile, laid out as the B operand of the first product
// (Z = V^T D, K = channels).  Because the summation order over K is free, the
// channel order of that product and the row order of the second product
// (V Z, M = channels) are chosen so that every output of the second product
// lands in the lane and register that already hold the same channel's d:
// the residual is formed with no data movement.  Likewise the component order
// of the second product's K dimension is the one in which Z comes out of the
// first.  V is stored twice on the device in exactly these operand orders
// (built on the host with the model), so every operand load is contiguous.
//
// FP32 path: v_mfma_f32_16x16x4f32.  Lane l = n + 16 g feeds A[n][g] and
//   B[g][n] and receives D[4 g + v][n] in register v.
//   GEMM1 step s: lane group g supplies channel 4 s + g.
//   GEMM2 tile t: output row 4 g + v is channel 16 t + 4 v + g (held in d[4 t + v]);
//   K step u supplies component 16 (u / 4) + 4 g + (u % 4) (held in z[u / 4][u % 4]).
// BF16 path: v_mfma_f32_16x16x32_bf16, 8 K values per lane, FP32 accumulation;
//   GEMM1 step s: lane group g supplies channels 32 s + 8 g + t (t < 8);
//   GEMM2 tile 2 s + h: output row 4 g + v is channel 32 s + 8 g + 4 h + v;
//   K step u supplies components 16 (2 u + t / 4) + 4 g + (t % 4).
// The subtraction, the comparisons with the edges and all counting stay FP32.
#include <algorithm>
#include <atomic>

#include "qfca_internal.h"
#include "qfca_tiles.h"

namespace qfca {
namespace {
using namespace tiles;

// ------------------------------------------------------------------------
// Standalone kernels.  The four wavefronts of a block share one 16-pixel
// tile: wave w owns the channel quarter [w CMAX/4, (w+1) CMAX/4) in both
// products, and the partial Z of the four quarters are added through LDS in
// a fixed order.  The blocks are persistent: a block copies the operand
// tables (VLDS) and the edge table (ELDS) into LDS once, when they fit, then
// walks tiles blockIdx.x, blockIdx.x + gridDim.x, ..., loading the next
// tile's features into registers while it computes the current one.  The
// bins of a tile are staged in LDS and written one 16-byte channel row per
// thread.
//
// LDS: mu, lo, 1/delta, bin margin [CMAX] each; Z partials [4 waves][KT][4]
// [64]; bin staging [CMAX][16] bytes; the two operand tables (VLDS); the
// edges [C][B-1] (ELDS).
struct ProjLds {
    size_t stg, tab, edges, total;
};

__host__ __device__ inline ProjLds proj_lds(int CMAX, int KT, int elt, bool vlds, bool elds, int C, int B) {
    ProjLds L;
    size_t off = ((size_t)4 * CMAX + (size_t)4 * KT * 4 * 64) * 4;
    L.stg = off;
    off += (size_t)CMAX * 16;
    L.tab = off;
    if (vlds) off += (size_t)2 * CMAX * KT * 16 * elt;
    L.edges = off;
    if (elds) off += (size_t)C * (B > 1 ? B - 1 : 0) * 4;
    L.total = (off + 15) & ~(size_t)15;
    return L;
}

__device__ __forceinline__ void proj_prologue(const MArgs& a, int CMAX, float* smu, float* slo, float* sid,
                                              float* sfd, float* sedge, bool elds) {
    for (int i = threadIdx.x; i < CMAX; i += blockDim.x) {
        // the four loads are issued before the stores (the sources are not
        // known not to alias LDS, so interleaved each load would wait)
        const bool ok = i < a.C;
        const float vm = ok ? a.mu[i] : 0.f;
        const float vl = ok && a.lo ? a.lo[i] : 0.f;
        const float vi = ok && a.inv_delta ? a.inv_delta[i] : 0.f;
        const float vf = ok && a.fastd ? a.fastd[i] : INFINITY;
        smu[i] = vm;
        slo[i] = vl;
        sid[i] = vi;
        sfd[i] = vf;
    }
    if (elds && a.bins) {
        const int ne = a.C * (a.B > 1 ? a.B - 1 : 0);
        for (int i = threadIdx.x; i < ne; i += blockDim.x) sedge[i] = a.edges[i];
    }
}

// Copies two operand tables of NU 16-byte units each into LDS: every thread
// issues up to eight loads of each table before it stores any, so the copy
// costs about one memory latency per eight units instead of one per unit.
template <int NU>
__device__ __forceinline__ void copy_tables(const void* g1, const void* g2, void* s1, void* s2) {
    const uint4* a1 = (const uint4*)g1;
    const uint4* a2 = (const uint4*)g2;
    uint4* d1 = (uint4*)s1;
    uint4* d2 = (uint4*)s2;
    constexpr int PER = (NU + 255) / 256;
    constexpr int G = PER < 8 ? PER : 8;
#pragma unroll
    for (int i0 = 0; i0 < PER; i0 += G) {
        uint4 t1[G], t2[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int u = threadIdx.x + 256 * (i0 + i);
            if (i0 + i < PER && u < NU) {
                t1[i] = a1[u];
                t2[i] = a2[u];
            }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int u = threadIdx.x + 256 * (i0 + i);
            if (i0 + i < PER && u < NU) {
                d1[u] = t1[i];
                d2[u] = t2[i];
            }
        }
    }
}

template <int CMAX, int KT, bool VLDS, bool ELDS>
__device__ __forceinline__ void proj_f32_body(const MArgs& a) {
    constexpr int NSW = CMAX / 16;   // GEMM1 K steps per wave (4 channels each)
    constexpr int VSZ = CMAX * KT * 16;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ProjLds L = proj_lds(CMAX, KT, 4, VLDS, ELDS, a.C, a.B);
    float* smu = (float*)lds_raw;
    float* slo = smu + CMAX;
    float* sid = slo + CMAX;
    float* sfd = sid + CMAX;
    float* zp = sfd + CMAX;              // [4 waves][KT][4][64]
    uint8_t* stg = lds_raw + L.stg;
    float* sv1 = (float*)(lds_raw + L.tab);
    float* sv2 = sv1 + VSZ;
    float* sedge = (float*)(lds_raw + L.edges);
    proj_prologue(a, CMAX, smu, slo, sid, sfd, sedge, ELDS);
    const float* V1 = (const float*)a.V1;
    const float* V2 = (const float*)a.V2;
    if (VLDS) {
        copy_tables<VSZ / 4>(V1, V2, sv1, sv2);
        V1 = sv1;
        V2 = sv2;
    }
    const float* edges = ELDS ? (const float*)sedge : a.edges;
    __syncthreads();
    // the wavefront index is uniform across the wavefront: held in a scalar
    // register, offsets derived from it fold into instruction offsets
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float x[NSW];
    // a contiguous run of tiles per block: neighbouring tiles share cache
    // lines, which then stay in one L2
    const int per = (a.ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    int tile = blockIdx.x * per;
    const int tend = min(a.ntiles, tile + per);
    if (tile < tend) proj_load_f32<CMAX>(a, tile, w, lane, x);
    for (; tile < tend; ++tile) {
        // Everything a tile derives from the lane and wavefront indices
        // (channels, masks, addresses) and the tables it reads are computed
        // and re-read per tile rather than held in registers across tiles:
        // the hidden copies below keep the compiler from hoisting them.
        int lt = lane, wt = w;
        asm volatile("" : "+v"(lt), "+s"(wt));
        float xn[NSW];
        const int nt = tile + 1;
        proj_load_f32<CMAX>(a, nt < tend ? nt : tend - 1, wt, lt, xn);  // the last one repeats a tile
        const float* V1t = VLDS ? opaque_lds(V1) : V1;
        const float* V2t = VLDS ? opaque_lds(V2) : V2;
        proj_tile_f32<CMAX, KT>(a, tile, wt, lt, V1t, V2t, opaque_lds(smu), opaque_lds(slo), opaque_lds(sid),
                                opaque_lds(sfd), zp, x, edges, stg);
        if (a.bins) {
            block_sync_lds();
            proj_store_bins<CMAX>(a, tile, stg);
        }
#pragma unroll
        for (int i = 0; i < NSW; ++i) x[i] = xn[i];
    }
}

template <int CMAX, int KT, bool VLDS, bool ELDS>
__device__ __forceinline__ void proj_bf16_body(const MArgs& a) {
    constexpr int NSW = CMAX / 128;  // GEMM1 K steps per wave (32 channels each)
    constexpr int VSZ = CMAX * KT * 16;  // bf16 elements per table
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ProjLds L = proj_lds(CMAX, KT, 2, VLDS, ELDS, a.C, a.B);
    float* smu = (float*)lds_raw;
    float* slo = smu + CMAX;
    float* sid = slo + CMAX;
    float* sfd = sid + CMAX;
    float* zp = sfd + CMAX;              // [4 waves][KT][4][64]
    uint8_t* stg = lds_raw + L.stg;
    bf16x8* sv1 = (bf16x8*)(lds_raw + L.tab);
    bf16x8* sv2 = sv1 + VSZ / 8;
    float* sedge = (float*)(lds_raw + L.edges);
    proj_prologue(a, CMAX, smu, slo, sid, sfd, sedge, ELDS);
    const bf16x8* V1 = (const bf16x8*)a.V1;
    const bf16x8* V2 = (const bf16x8*)a.V2;
    if (VLDS) {
        copy_tables<VSZ / 8>(V1, V2, sv1, sv2);
        V1 = sv1;
        V2 = sv2;
    }
    const float* edges = ELDS ? (const float*)sedge : a.edges;
    __syncthreads();
    // the wavefront index is uniform across the wavefront: held in a scalar
    // register, offsets derived from it fold into instruction offsets
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float x[NSW][8];
    const int per = (a.ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    int tile = blockIdx.x * per;
    const int tend = min(a.ntiles, tile + per);
    if (tile < tend) proj_load_bf16<CMAX>(a, tile, w, lane, x);
    for (; tile < tend; ++tile) {
        int lt = lane, wt = w;
        asm volatile("" : "+v"(lt), "+s"(wt));
        float xn[NSW][8];
        const int nt = tile + 1;
        proj_load_bf16<CMAX>(a, nt < tend ? nt : tend - 1, wt, lt, xn);  // the last one repeats a tile
        const bf16x8* V1t = VLDS ? opaque_lds(V1) : V1;
        const bf16x8* V2t = VLDS ? opaque_lds(V2) : V2;
        proj_tile_bf16<CMAX, KT>(a, tile, wt, lt, V1t, V2t, opaque_lds(smu), opaque_lds(slo), opaque_lds(sid),
                                 opaque_lds(sfd), zp, x, edges, stg);
        if (a.bins) {
            block_sync_lds();
            proj_store_bins<CMAX>(a, tile, stg);
        }
#pragma unroll
        for (int i = 0; i < NSW; ++i)
#pragma unroll
            for (int t = 0; t < 8; ++t) x[i][t] = xn[i][t];
    }
}

// Up to 256 channels the kernels are compiled for two wavefronts per SIMD;
// 512 channels keep the full register file (they would spill otherwise).
template <int CMAX, int KT, bool VLDS, bool ELDS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_proj_f32_mfma(MArgs a) {
    proj_f32_body<CMAX, KT, VLDS, ELDS>(a);
}
template <int CMAX, int KT, bool VLDS, bool ELDS>
__global__ __launch_bounds__(256) void k_proj_f32_mfma_wide(MArgs a) {
    proj_f32_body<CMAX, KT, VLDS, ELDS>(a);
}
template <int CMAX, int KT, bool VLDS, bool ELDS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_proj_bf16_mfma(MArgs a) {
    proj_bf16_body<CMAX, KT, VLDS, ELDS>(a);
}
template <int CMAX, int KT, bool VLDS, bool ELDS>
__global__ __launch_bounds__(256) void k_proj_bf16_mfma_wide(MArgs a) {
    proj_bf16_body<CMAX, KT, VLDS, ELDS>(a);
}

// ------------------------------------------------------------------------
// BF16 kernel for the widest maps (CMAX = 512): every wavefront runs whole
// 16-pixel tiles on its own, all channels in both products, so there are no
// Z partials to add across wavefronts.  The NW wavefronts of a block (two
// per SIMD, which hide each other's memory and LDS latency) share the
// operand tables and the per-channel parameters in LDS and take interleaved
// tiles of one contiguous run, meeting at bare barriers (see the loop).  Lane (g, n) holds the
// channels 32 s + 8 g + t of pixel n in d[s][t] (the first product's B
// operand), and the second product's outputs land on the same channels.
// The bins of four consecutive channels of a pixel (one lane) are packed in
// a dword and transposed within each group of four lanes (two quad-permute
// exchanges and two byte permutes), so that a lane holds four consecutive
// pixels of one channel and writes them with one dword store.
//
// LDS: mu, lo, 1/delta, bin margin [CMAX] each; the two operand tables.
// Wavefronts per block of k_proj_bf16_solo (a multiple of 4: NW / 4 per SIMD).
// Eight take 128 pixels a round, one whole 128-byte line of every channel's
// bins, so with the per-step barriers no line is split between rounds
// (1024x1024x512, k = 64: eight 0.86 ms, twelve 1.04 ms, sixteen, which
// spill at 128 registers, 1.71 ms).
#ifndef SOLO_WAVES
#define SOLO_WAVES 8
#endif
__host__ __device__ inline size_t solo_lds(int CMAX, int KT) {
    return (size_t)16 * CMAX + (size_t)2 * CMAX * KT * 16 * 2;
}

template <int CMAX, int KT, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW / 4, NW / 4))) void k_proj_bf16_solo(
    MArgs a) {
    constexpr int NS = CMAX / 32;        // first-product K steps (32 channels each)
    constexpr int QS = NS / 4;           // K steps of one quarter (one wavefront's share in k_proj_bf16_mfma)
    constexpr int SB = 1;                // second-product steps between the block's barriers
    constexpr int NU = KT / 2;           // second-product K steps (32 components each)
    constexpr int VSZ = CMAX * KT * 16;  // bf16 elements per table
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float* smu = (float*)lds_raw;
    float* slo = smu + CMAX;
    float* sid = slo + CMAX;
    float* sfd = sid + CMAX;
    bf16x8* sv1 = (bf16x8*)(lds_raw + 16 * CMAX);
    bf16x8* sv2 = sv1 + VSZ / 8;
    for (int i = threadIdx.x; i < CMAX; i += blockDim.x) {
        const bool ok = i < a.C;
        const float vm = ok ? a.mu[i] : 0.f;
        const float vl = ok && a.lo ? a.lo[i] : 0.f;
        const float vi = ok && a.inv_delta ? a.inv_delta[i] : 0.f;
        const float vf = ok && a.fastd ? a.fastd[i] : INFINITY;
        smu[i] = vm;
        slo[i] = vl;
        sid[i] = vi;
        sfd[i] = vf;
    }
    {
        // tables: 16-byte units, eight loads per thread in flight before
        // their stores
        constexpr int NUNIT = VSZ / 8;
        const uint4* g1 = (const uint4*)a.V1;
        const uint4* g2 = (const uint4*)a.V2;
        uint4* d1 = (uint4*)sv1;
        uint4* d2 = (uint4*)sv2;
        for (int u0 = threadIdx.x; u0 < NUNIT; u0 += 4 * 64 * NW) {
            uint4 t1[4], t2[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = u0 + 64 * NW * i;
                if (u < NUNIT) {
                    t1[i] = g1[u];
                    t2[i] = g2[u];
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = u0 + 64 * NW * i;
                if (u < NUNIT) {
                    d1[u] = t1[i];
                    d2[u] = t2[i];
                }
            }
        }
    }
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // A block walks a contiguous run of tiles, its NW wavefronts interleaved
    // (wave w takes tiles w, w + NW, ...): the block's current tiles are
    // 16 NW consecutive pixels, so its bin stores fill whole 128-byte lines
    // of each channel row and its feature loads whole lines too.
    const int per = ((a.ntiles + (int)gridDim.x - 1) / (int)gridDim.x + NW - 1) / NW * NW;
    const int b0 = (int)blockIdx.x * per;
    const int tend = min(a.ntiles, b0 + per);
    int tile = b0 + w;
    const bool rows_dw = ((a.N & 3) == 0) && (((uintptr_t)a.bins & 3) == 0);
    // features of a tile: channel 32 s + t + 8 g of pixel px is at the uniform
    // row base of channel 32 s + t plus the lane's 32-bit byte offset
    // (8 g N + px) 4.  A lane whose channel is past C reads the uniform
    // channel's row, or channel C - 1 when that is past C too: real features
    // that meet zero table rows and whose residuals are never stored.
    // d[s] of the next tile is loaded as soon as the current tile's step s
    // has used it, so the loads of a tile are in flight during the previous
    // one's second product and quantisation.
    auto load_row = [&](float (&dr)[8], int s, const float* Xb, uint32_t vo, uint32_t vo0, int gg)
        __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int cu = 32 * s + t;  // uniform part of the channel
            const char* rb = (const char*)(Xb + (size_t)(cu < a.C ? cu : a.C - 1) * a.N);
            dr[t] = *(const float*)(rb + (cu + 8 * gg < a.C ? vo : vo0));
        }
    };
    float d[NS][8];
    if (tile < tend) {
        const int lane = threadIdx.x & 63;
        const int g = lane >> 4;
        const int pxc = min(tile * 16 + (lane & 15), a.N - 1);
        const uint32_t vo = ((uint32_t)(8 * g) * (uint32_t)a.N + (uint32_t)pxc) * 4u;
#pragma unroll
        for (int s = 0; s < NS; ++s) load_row(d[s], s, a.X, vo, (uint32_t)pxc * 4u, g);
    }
    // Every wavefront of the block runs the same number of rounds and meets
    // the others at the start of each (a bare barrier: loads in flight stay
    // in flight), so the block's stores to a line of bins, and its loads of a
    // line of features, come close together in time.
    const int nround = tend > b0 ? (tend - b0 + NW - 1) / NW : 0;
    for (int rd = 0; rd < nround; ++rd, tile += NW) {
        __builtin_amdgcn_s_barrier();
        if (tile >= tend) {
            // the barriers of the steps the others run
#pragma unroll
            for (int i = 0; i < NS / SB - 1; ++i) __builtin_amdgcn_s_barrier();
            continue;
        }
        // the lane index made opaque per tile: every address and test derived
        // from the lane's channels is formed in the loop where it is used
        // (hoisted out of it, the 128 channels' offsets and tests would take
        // far more registers than the wavefront has)
        int lane = threadIdx.x & 63;
        asm volatile("" : "+v"(lane));
        const int g = lane >> 4, n = lane & 15, p = n & 3, qd = n >> 2;
        // byte selectors of the quad transpose (first exchange with lane
        // p ^ 1, then with lane p ^ 2; own dword is the first perm source)
        const uint32_t selA = (p & 1) ? 0x07030501u : 0x02060004u;
        const uint32_t selB = (p & 2) ? 0x07060302u : 0x01000504u;
        const int px = tile * 16 + n;
        const bool pxok = px < a.N;
        const bool more = tile + NW < tend;
        const int pxn = min((tile + NW) * 16 + n, a.N - 1);
        const uint32_t von = ((uint32_t)(8 * g) * (uint32_t)a.N + (uint32_t)pxn) * 4u;
        const uint32_t von0 = (uint32_t)pxn * 4u;
        // the base made opaque per tile, as the lane index
        const float* Xt = a.X;
        asm volatile("" : "+s"(Xt));
        const bf16x8* V1 = opaque_lds((const bf16x8*)sv1);
        const bf16x8* V2 = opaque_lds((const bf16x8*)sv2);
        const float* mu = opaque_lds((const float*)smu);
        // Z in the order of the block-split kernels (and of the batch
        // kernel): four quarters of the K steps, each a chain from zero, the
        // quarters added in order, so that every path gives the same bits
        floatx4 z[KT], zq[KT];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s % QS == 0) {
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) zq[kt] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
            // mu of the lane's eight channels: two 16-byte reads
            const float4 m0 = *(const float4*)(mu + 32 * s + 8 * g);
            const float4 m1 = *(const float4*)(mu + 32 * s + 8 * g + 4);
            const float mv[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
            bf16x8 bv;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                d[s][t] -= mv[t];
                bv[t] = (__bf16)d[s][t];
            }
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
                zq[kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(V1[((s * KT + kt) * 4 + g) * 16 + n], bv, zq[kt], 0,
                                                                 0, 0);
            if (s % QS == QS - 1) {
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) z[kt][v] = (s == QS - 1) ? zq[kt][v] : z[kt][v] + zq[kt][v];
            }
            // keeps the scheduler from hoisting later steps' table reads
            // (all of them in flight at once would not fit the registers)
            __builtin_amdgcn_sched_barrier(0);
        }
        bf16x8 zb[NU];
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int v = 0; v < 4; ++v) zb[kt >> 1][4 * (kt & 1) + v] = (__bf16)z[kt][v];
        const float* plo = opaque_lds((const float*)slo);
        const float* pid = opaque_lds((const float*)sid);
        const float* pfd = opaque_lds((const float*)sfd);
        const int B = a.B;
        const float top = (float)max(B - 1, 0);
        const uint32_t needmask = B > 1 ? 0xFu : 0u;  // one bin: every value's bin is 0
        // the other bases opaque per tile too, for the same reason
        const float* Et = a.edges;
        float* Rt = a.resid;
        uint8_t* Bt = a.bins;
        asm volatile("" : "+s"(Et), "+s"(Rt), "+s"(Bt));
        auto step = [&](auto sc) __attribute__((always_inline)) {
            constexpr int s = decltype(sc)::value;
            // the block's wavefronts meet every SB steps, so that their
            // stores to each channel's line of bins stay close in time
            if constexpr (s > 0 && s % SB == 0) __builtin_amdgcn_s_barrier();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int u = 0; u < NU; ++u)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(V2[(((2 * s + h) * NU + u) * 4 + g) * 16 + n],
                                                                  zb[u], acc, 0, 0, 0);
                const int c0 = 32 * s + 8 * g + 4 * h;  // channels c0 .. c0 + 3 of pixel px
                float rv[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) rv[v] = d[s][4 * h + v] - acc[v];
                if (Rt) {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (pxok && c0 + v < a.C) Rt[(size_t)(c0 + v) * a.N + px] = rv[v];
                }
                if (!Bt) continue;
                // bin = #{m : r >= e_m}, decided by the margin test or, next
                // to an edge, by the edge search (as emit_values)
                // the four channels' parameters: one 16-byte read each (c0 is a
                // multiple of 4); tests combined without branches
                const float4 l4 = *(const float4*)(plo + c0);
                const float4 i4 = *(const float4*)(pid + c0);
                const float4 f4 = *(const float4*)(pfd + c0);
                const float lov[4] = {l4.x, l4.y, l4.z, l4.w};
                const float idv[4] = {i4.x, i4.y, i4.z, i4.w};
                const float dlv[4] = {f4.x, f4.y, f4.z, f4.w};
                uint32_t bq[4];
                uint32_t need = 0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float tt = (rv[v] - lov[v]) * idv[v];
                    const float near = __builtin_amdgcn_fmed3f(rintf(tt), 1.f, top);
                    const bool dec = fabsf(tt - near) >= dlv[v];  // +infinity: the shortcut is off
                    bq[v] = (uint32_t)__builtin_amdgcn_fmed3f(floorf(tt), 0.f, top);
                    need |= ((!dec) & pxok & (c0 + v < a.C)) ? (1u << v) : 0u;
                }
                need &= needmask;
                if (__ballot(need != 0u)) {
                    // one edge search per round for the lowest flagged value
                    // of each lane (one copy of the search code per step)
                    uint32_t nd = need;
                    while (__ballot(nd != 0u)) {
                        const int v = nd ? __builtin_ctz(nd) : 0;
                        const float r = v == 0 ? rv[0] : (v == 1 ? rv[1] : (v == 2 ? rv[2] : rv[3]));
                        const int c = c0 + v;
                        const uint32_t b = nd ? (uint32_t)bin_fast(r, Et + (size_t)c * (B - 1), plo[c], pid[c], B)
                                              : 0u;
                        if (nd) {
                            bq[0] = v == 0 ? b : bq[0];
                            bq[1] = v == 1 ? b : bq[1];
                            bq[2] = v == 2 ? b : bq[2];
                            bq[3] = v == 3 ? b : bq[3];
                        }
                        nd &= nd - 1u;
                    }
                }
                const uint32_t pk = bq[0] | (bq[1] << 8) | (bq[2] << 16) | (bq[3] << 24);
                // lane (g, 4 qd + p) now holds channel c0' + p, pixels 4 qd .. 4 qd + 3
                const uint32_t tr = quad_transpose_bytes(pk, selA, selB);
                const int cw = 32 * s + 8 * g + 4 * h + p;
                const int pw = tile * 16 + 4 * qd;
                if (cw < a.C) {
                    uint8_t* dst = Bt + (size_t)cw * a.N + pw;
                    if (rows_dw && pw + 3 < a.N) {
                        *(uint32_t*)dst = tr;
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (pw + i < a.N) dst[i] = (uint8_t)(tr >> (8 * i));
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if (more) load_row(d[s], s, Xt, von, von0, g);
        };
        StaticFor<0, NS>::run(step);
    }
}

constexpr size_t LDS_MAX = 160 * 1024;
constexpr size_t LDS_TWO_BLOCKS = 80 * 1024;

// Launches a persistent grid: as many blocks as fit on the device (at most
// two per compute unit, the register limit), never more than there are tiles.
// Compute units of the current device, queried once per device; callers may
// launch from several host threads.
hipError_t device_cus(int* out) {
    static std::atomic<int> cache[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64) {
        const int v = cache[dev].load(std::memory_order_relaxed);
        if (v > 0) {
            *out = v;
            return hipSuccess;
        }
    }
    int n = 0;
    e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (n < 1) return hipErrorInvalidValue;
    if (dev >= 0 && dev < 64) cache[dev].store(n, std::memory_order_relaxed);
    *out = n;
    return hipSuccess;
}

template <class K>
hipError_t go(K kern, const MArgs& a, size_t lds, hipStream_t st) {
    int ncu = 0;
    {
        const hipError_t e = device_cus(&ncu);
        if (e != hipSuccess) return e;
    }
    if (lds > LDS_MAX) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int per_cu = lds <= LDS_TWO_BLOCKS ? 2 : 1;
    const int blocks = std::max(1, std::min(a.ntiles, ncu * per_cu));
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, st, a);
    return hipGetLastError();
}

}  // namespace

int mfma_cmax(int C, int prec) {
    int cm = prec == QFCA_PREC_BF16 ? 128 : 64;
    while (cm < C) cm <<= 1;
    return cm <= 512 ? cm : 0;
}

int mfma_kt(int k, int prec) {
    if (k <= 0 || k > 64) return 0;
    int kt = (k + 15) / 16;
    if (prec == QFCA_PREC_BF16) kt = (kt + 1) / 2 * 2;
    return kt == 3 ? 4 : kt;
}

// Operand tables: see the file comment.  V: host [C][k] (float), padded to
// CM channels and KT component tiles (zero rows and columns).
void mfma_tables_f32(const float* V, int C, int k, std::vector<float>& V1, std::vector<float>& V2) {
    mfma_tables_f32_at(V, C, k, mfma_cmax(C, QFCA_PREC_FP32), mfma_kt(k, QFCA_PREC_FP32), V1, V2);
}

void mfma_tables_bf16(const uint16_t* Vb, int C, int k, std::vector<uint16_t>& V1, std::vector<uint16_t>& V2) {
    mfma_tables_bf16_at(Vb, C, k, mfma_cmax(C, QFCA_PREC_BF16), mfma_kt(k, QFCA_PREC_BF16), V1, V2);
}

void mfma_tables_f32_at(const float* V, int C, int k, int CM, int KT, std::vector<float>& V1,
                        std::vector<float>& V2) {
    const int NU = 4 * KT;
    V1.assign((size_t)CM * KT * 16, 0.f);
    V2.assign((size_t)CM * KT * 16, 0.f);
    auto at = [&](int c, int j) { return (c < C && j < k) ? V[(size_t)c * k + j] : 0.f; };
    for (int s = 0; s < CM / 4; ++s)
        for (int kt = 0; kt < KT; ++kt)
            for (int g = 0; g < 4; ++g)
                for (int n = 0; n < 16; ++n) V1[((s * KT + kt) * 4 + g) * 16 + n] = at(4 * s + g, 16 * kt + n);
    for (int t = 0; t < CM / 16; ++t)
        for (int u = 0; u < NU; ++u)
            for (int g = 0; g < 4; ++g)
                for (int n = 0; n < 16; ++n)
                    V2[((t * NU + u) * 4 + g) * 16 + n] =
                        at(16 * t + 4 * (n % 4) + n / 4, 16 * (u / 4) + 4 * g + (u % 4));
}

void mfma_tables_bf16_at(const uint16_t* Vb, int C, int k, int CM, int KT, std::vector<uint16_t>& V1,
                         std::vector<uint16_t>& V2) {
    const int NU = KT / 2;
    V1.assign((size_t)CM * KT * 16, 0);
    V2.assign((size_t)CM * KT * 16, 0);
    auto at = [&](int c, int j) -> uint16_t { return (c < C && j < k) ? Vb[(size_t)c * k + j] : (uint16_t)0; };
    for (int s = 0; s < CM / 32; ++s)
        for (int kt = 0; kt < KT; ++kt)
            for (int g = 0; g < 4; ++g)
                for (int n = 0; n < 16; ++n)
                    for (int t = 0; t < 8; ++t)
                        V1[(((s * KT + kt) * 4 + g) * 16 + n) * 8 + t] = at(32 * s + 8 * g + t, 16 * kt + n);
    for (int s = 0; s < CM / 32; ++s)
        for (int h = 0; h < 2; ++h)
            for (int u = 0; u < NU; ++u)
                for (int g = 0; g < 4; ++g)
                    for (int n = 0; n < 16; ++n)
                        for (int t = 0; t < 8; ++t)
                            V2[((((2 * s + h) * NU + u) * 4 + g) * 16 + n) * 8 + t] =
                                at(32 * s + 8 * (n / 4) + 4 * h + (n % 4), 16 * (2 * u + t / 4) + 4 * g + (t % 4));
}

hipError_t launch_proj_mfma(const ProjLaunch& L, const void* V1, const void* V2, hipStream_t st) {
    MArgs a;
    a.X = L.X; a.C = L.C; a.N = L.N; a.k = L.k; a.B = L.B;
    a.mu = L.mu; a.V1 = V1; a.V2 = V2;
    a.edges = L.edges; a.lo = L.lo; a.inv_delta = L.inv_delta; a.fastd = L.fastd;
    a.bins = L.bins; a.resid = L.resid;
    a.ntiles = (L.N + 15) / 16;
    const int CM = mfma_cmax(L.C, L.prec), KT = mfma_kt(L.k, L.prec);
    if (!CM || !KT) return hipErrorInvalidValue;
    const bool bf = L.prec == QFCA_PREC_BF16;
    const int elt = bf ? 2 : 4;
    // (the lane byte offsets of its feature loads are 32-bit: (24 N + N) 4 < 2^32)
    if (bf && CM == 512 && (KT == 2 || KT == 4) && (unsigned long long)L.N * 100ULL < (1ULL << 32)) {
        // whole tiles per wavefront, eight wavefronts per block, one block per CU
        int ncu = 0;
        const hipError_t e = device_cus(&ncu);
        if (e != hipSuccess) return e;
        const size_t lds = solo_lds(CM, KT);
        constexpr int NW = SOLO_WAVES;
        const void* kf =
            KT == 4 ? (const void*)k_proj_bf16_solo<512, 4, NW> : (const void*)k_proj_bf16_solo<512, 2, NW>;
        const hipError_t ea = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (ea != hipSuccess) return ea;
        const int blocks = std::max(1, std::min((a.ntiles + NW - 1) / NW, ncu));
        if (KT == 4)
            hipLaunchKernelGGL((k_proj_bf16_solo<512, 4, NW>), dim3(blocks), dim3(64 * NW), lds, st, a);
        else
            hipLaunchKernelGGL((k_proj_bf16_solo<512, 2, NW>), dim3(blocks), dim3(64 * NW), lds, st, a);
        return hipGetLastError();
    }
    // tables in LDS when they fit; the edges are read through the cache
    // (the bin decision needs them only for values next to an edge)
    const bool vl = proj_lds(CM, KT, elt, true, false, L.C, L.B).total <= LDS_MAX;
    const bool el = false;
    (void)el;
    const size_t lds = proj_lds(CM, KT, elt, vl, el, L.C, L.B).total;
#define QFCA_PJ(KERN, CMV, KTV)                                                          \
    {                                                                                    \
        if (vl) return go(KERN<CMV, KTV, true, false>, a, lds, st);                      \
        return go(KERN<CMV, KTV, false, false>, a, lds, st);                             \
    }
    // one block per compute unit (one wavefront per SIMD) when the LDS allows
    // no second: the register file is then the wavefront's alone, so the
    // variant without the two-wavefront register cap runs
    const bool one_block = lds > LDS_TWO_BLOCKS;
#define QFCA_PJ2(KERN, CMV, KTV)                                                         \
    {                                                                                    \
        if (one_block) QFCA_PJ(KERN##_wide, CMV, KTV)                                    \
        QFCA_PJ(KERN, CMV, KTV)                                                          \
    }
#define QFCA_F32_CASE(CMV, KTV) if (!bf && CM == CMV && KT == KTV) QFCA_PJ2(k_proj_f32_mfma, CMV, KTV)
#define QFCA_BF_CASE(CMV, KTV) if (bf && CM == CMV && KT == KTV) QFCA_PJ2(k_proj_bf16_mfma, CMV, KTV)
#define QFCA_F32_CM(CMV) QFCA_F32_CASE(CMV, 1) QFCA_F32_CASE(CMV, 2) QFCA_F32_CASE(CMV, 4)
#define QFCA_BF_CM(CMV) QFCA_BF_CASE(CMV, 2) QFCA_BF_CASE(CMV, 4)
#define QFCA_F32W_CASE(CMV, KTV) if (!bf && CM == CMV && KT == KTV) QFCA_PJ(k_proj_f32_mfma_wide, CMV, KTV)
#define QFCA_BFW_CASE(CMV, KTV) if (bf && CM == CMV && KT == KTV) QFCA_PJ(k_proj_bf16_mfma_wide, CMV, KTV)
    QFCA_F32_CM(64) QFCA_F32_CM(128) QFCA_F32_CM(256)
    QFCA_F32W_CASE(512, 1) QFCA_F32W_CASE(512, 2) QFCA_F32W_CASE(512, 4)
    QFCA_BF_CM(128) QFCA_BF_CM(256)
    QFCA_BFW_CASE(512, 2) QFCA_BFW_CASE(512, 4)
#undef QFCA_BFW_CASE
#undef QFCA_PJ2
#undef QFCA_F32W_CASE
#undef QFCA_BF_CM
#undef QFCA_F32_CM
#undef QFCA_BF_CASE
#undef QFCA_F32_CASE
#undef QFCA_PJ
    return hipErrorInvalidValue;
}

}  // namespace qfca
