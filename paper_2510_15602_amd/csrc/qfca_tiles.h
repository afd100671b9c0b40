// Device-side tile routines shared by the standalone kernels and the
// persistent batch kernel (internal header of libqfca).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace qfca {
namespace tiles {

__device__ __forceinline__ int lane_prev(int v) {
    // Value held by lane-1 (DPP wave_shr:1); lane 0 receives 0 (bound_ctrl).
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// Sum of v over each aligned group of g lanes (g = 8, 16, 32 or 64), held
// by every lane of the group: mirrored and quad-permuted DPP adds within
// rows of 16 lanes, then exchanges across rows.  Called by all lanes.
__device__ __forceinline__ int group_sum(int v, int g) {
    v += __builtin_amdgcn_mov_dpp(v, 0x141, 0xf, 0xf, false);  // row_half_mirror: lanes l, 7 - l
    v += __builtin_amdgcn_mov_dpp(v, 0x4E, 0xf, 0xf, false);   // quad_perm [2, 3, 0, 1]
    v += __builtin_amdgcn_mov_dpp(v, 0xB1, 0xf, 0xf, false);   // quad_perm [1, 0, 3, 2]: 8-lane sums
    if (g >= 16) v += __builtin_amdgcn_mov_dpp(v, 0x140, 0xf, 0xf, false);  // row_mirror: 16-lane sums
    if (g >= 32) v += __shfl_xor(v, 16, 64);
    if (g >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

// A compile-time boolean passed as a value (selects code paths of a lambda).
template <bool V>
struct bconst {
    static constexpr bool value = V;
};

// LDS (address space 3) views: loads through these take a 32-bit LDS byte
// address held in a register, so constant parts of an address fold into the
// instruction's offset field.
typedef __attribute__((address_space(3))) const char* lds_cptr;
typedef __attribute__((address_space(3))) const int* lds_iptr;
typedef __attribute__((address_space(3))) const float* lds_fptr;

// Orders one wavefront's LDS accesses before it against those after it.  A
// score tile's LDS region is private to its wavefront, and the LDS performs
// the operations of one wavefront in program order, so a wavefront-scope
// fence (which keeps the compiler from moving accesses across it) is all
// the synchronisation the tile needs.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block barrier for data exchanged through LDS only: this wavefront's LDS
// operations complete (lgkmcnt 0), then s_barrier.  Unlike __syncthreads it
// does not wait for outstanding global loads, so a prefetch stays in flight
// across it.  The signal fences keep the compiler from moving memory
// accesses across the barrier.
__device__ __forceinline__ void block_sync_lds() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt 63, expcnt 7, lgkmcnt 0
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ int lds_addr(const void* p) { return (int)(uintptr_t)(lds_cptr)(const char*)p; }
__device__ __forceinline__ int lds_load_i(int addr) { return *(lds_iptr)(uintptr_t)addr; }
__device__ __forceinline__ float lds_load_f(int addr) { return *(lds_fptr)(uintptr_t)addr; }
__device__ __forceinline__ void lds_store_f(int addr, float v) {
    *(__attribute__((address_space(3))) float*)(uintptr_t)addr = v;
}


// Same computation as k_score with the window side T fixed at compile time,
// organised for instruction-level parallelism.  Per row of patch centres:
//   1. the vertical counts vc of every bin column are updated in place (one
//      pass, dword-wide; the counts of lane (s, j) for a T-column block are
//      T consecutive bytes padded to a multiple of 4);
//   2. the row is walked in blocks of T patch columns.  Window cumulative
//      counts are carried times 4 and offset by the LDS address of the
//      lane's per-channel table psi4[t] = 4 Psi(t), so that they are directly
//      the addresses of its entries, and differences of two of them are the
//      addresses of the block-shared table rcp4[P] = 1 / (4 P) at the start
//      of the block's LDS.  For a full window (n = T*T)
//      the transport numerator of bin j is, with g(t) = Psi(t) - j t (convex,
//      smallest at the reference crossing c = cR_{j-1}):
//        I_j = g(u) + g(v) - 2 min_{[u, v]} g,  u = cP_{j-1}, v = cP_j,
//      where the minimum is g(u) if c <= u, g(v) if c >= v and g(c) otherwise;
//      the neighbour lane supplies g(u) (its own g of u, shifted by u).
//      The T table reads, neighbour exchanges and reciprocal reads of a block
//      are each issued together;
//   3. the horizontal window sum of each step is the suffix sum of the
//      previous block plus the prefix sum of the current one (FP32, in an
//      order fixed by the block, so deterministic for a given tile); the
//      sums are written to a small LDS buffer and gathered into the pending
//      rows' accumulators by all lanes at once, one (channel, pending row,
//      column) triple per lane.
// Throughout, LDS loads of a step are written before its stores: the regions
// of a tile never overlap, but the compiler cannot prove it, and a load that
// follows a store in program order waits for it (one LDS round trip per
// element instead of one per group).
template <int T>
struct BLayout {
    static constexpr int r = T / 2, m = T * T, T1 = T + 1, TP = (T + 3) & ~3;
    static constexpr int PSI = m + 2;  // psi4 entries per channel (t = 0 .. m + 1)
    static constexpr int HS = T + 2;   // odd row stride of the horizontal-sum buffer [64][HS]
    // block-shared 1/(4P) table, P = 0 .. m, at the start of the block's LDS
    static constexpr size_t RCP_BYTES = ((size_t)(m + 1) * 4 + 15) & ~(size_t)15;
    int nblk, rowb, vs4;
    size_t vc, ring, acc, hrow, psi, total;
    __host__ __device__ BLayout(int S, int Ws) {
        nblk = (Ws + 2 * r + T - 1) / T;  // blocks of patch columns
        rowb = (nblk + 1) * TP;           // bin columns [x0-2r, x0-2r+(nblk+1)T)
        vs4 = rowb / 4;
        if ((vs4 & 1) == 0) vs4 += 1;  // odd dword stride between lanes
        size_t off = 0;
        vc = off;   off += align16((size_t)64 * vs4 * 4);
        ring = off; off += align16((size_t)T1 * S * rowb);
        acc = off;  off += align16((size_t)T * S * Ws * 4);
        hrow = off; off += align16((size_t)64 * HS * 4);
        psi = off;  off += align16((size_t)S * PSI * 4);
        total = off;
        // the gather packs ring and accumulator offsets, one row past their
        // ring's end included, into 16 bits, and tells accumulator rows apart
        // only when a strip is at least T columns wide: a layout beyond that
        // reports a size no LDS limit admits
        if ((size_t)(T1 + 1) * S * rowb >= 65536 || (size_t)(T + 1) * S * Ws >= 65536 || Ws < T)
            total = (size_t)1 << 30;
    }
};

// Fills the block-shared table rcp4[P] = rcp[P] / 4 (exact) for P = 0 .. T*T.
// The loads of a chunk are all issued before its stores (the global source
// is not known not to alias LDS, so one load per store would each wait).
template <int T>
__device__ __forceinline__ void fill_rcp4(float* rcp4, const float* rcp, int tid, int nthreads) {
    constexpr int N = T * T + 1;
    for (int t0 = tid; t0 < N; t0 += 8 * nthreads) {
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int t = t0 + i * nthreads;
            v[i] = t < N ? rcp[t] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int t = t0 + i * nthreads;
            if (t < N) rcp4[t] = 0.25f * v[i];
        }
    }
}

// One (strip bx, output rows [y0, ye), channel group bz) tile, run by one
// wavefront whose lanes are `lane`, with its private LDS region `smem`
// (BLayout) and the block-shared table rcp4 (fill_rcp4, visible to the wave
// before the call).  Every map is the same for any split of the rows.
// The tile synchronises only its own wavefront, so the wavefronts of a block
// may run tiles of different geometry.
//   FASTG: blocks whose output columns all lie inside the strip take a
//   gather with no column test (a gain in the persistent batch kernel, a
//   small loss in the one-tile kernel, whose registers it crowds).
//   RCP0: the caller guarantees that rcp4 sits at LDS address 0 (a kernel
//   with no static LDS whose dynamic LDS starts with it), so the byte offset
//   4P of rcp4[P] is its address and costs no add.
//   DBG: inspection build of the same code that also stores, for every
//   window of the tile's own outputs, the cumulative count cP_j and the
//   transport numerator I_j of every bin (a.dbg_cp, a.dbg_I, [C][H][W][B]).
//   W1O: window 1-Wasserstein distances only: for each of the tile's own
//   windows, sum_j |cP_j m - cR_j n| / (n m) weighted by delta_c, added over
//   the channel group into a.w1sum (fixed point); no per-bin errors, no
//   association, no halo rows.
//   GS: finite sigma_p (Eq. 2 weights w(d) = a.wgt[d + r], separable): the
//   horizontal sums are the w-weighted sums of the T steps around each
//   output column (fixed order), the gather adds w(dy) times them, and an
//   output is divided by the in-image weight sums along both axes instead of
//   the window counts.
template <int T, bool FASTG, bool RCP0, bool DBG = false, bool W1O = false, bool GS = false>
__device__ __forceinline__ void score_tile(const KArgs& a, int bx, int y0, int ye, int bz, int lane,
                                           unsigned char* smem, const float* rcp4) {
    using BL = BLayout<T>;
    constexpr int r = BL::r, m = BL::m, T1 = BL::T1, TP = BL::TP, PSI = BL::PSI, HS = BL::HS;
    const int Bp = a.Bp, S = a.S, H = a.H, W = a.W, Ws = a.Ws;
    const int s = lane / Bp;
    const int sa = s < S ? s : S - 1;
    const int j = lane - s * Bp;
    const bool j0 = (j == 0);
    const int x0 = bx * Ws;
    const int xe = min(W, x0 + Ws);
    const int ws = xe - x0;
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
    float* acc = (float*)(smem + L.acc);         // [T][S][Ws]
    float* hrow = (float*)(smem + L.hrow);       // [64 lanes][HS]: the block's T window sums per lane
    // the gather's stores of items with no output go to column T of the
    // lane's own hrow row (padding, never read)
    float* trash_l = hrow + lane * HS + T;
    int* psi = (int*)(smem + L.psi);             // [S][PSI]: 4 Psi_c(t)

    // psi4[t] = 4 Psi(t) for t <= m, and 4 Psi(m + 1) = 4 (Psi(m) + sigma(m));
    // eight loads per lane in flight before their stores
    for (int t0 = lane; t0 < S * PSI; t0 += 8 * 64) {
        int v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int t = t0 + 64 * i;
            const int ss = t / PSI, tt = t - ss * PSI;
            const int cc = cbase + ss;
            v[i] = 0;
            if (t < S * PSI && cc < a.C) {
                const int2 p = a.psig[(size_t)cc * (m + 1) + min(tt, m)];
                v[i] = 4 * (tt <= m ? p.x : p.x + p.y);
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (t0 + 64 * i < S * PSI) psi[t0 + 64 * i] = v[i];
    }
    for (int t = lane; t < 64 * L.vs4; t += 64) vc32[t] = 0u;
    for (int t = lane; t < T * S * Ws; t += 64) acc[t] = 0.f;
    const int ci = cval ? c : 0;
    const int crm1 = a.cRm1[ci * Bp + j];
    const int dm1 = a.Dm1[ci * Bp + j];
    const int crl4 = 4 * a.cRl[ci * Bp + j];
    // The running counts carry the LDS address `bias` of this lane's psi4
    // table: cpb = 4 cP + bias is the address of psi4[cP], and the difference
    // of two such counts, 4P, is the offset of rcp4[P] from rcp4.  The g
    // values below are all shifted by the same per-lane constant -j bias,
    // which cancels in I.
    const int* psl = psi + sa * PSI;
    const int bias = lds_addr(psl);
    const int rbase = lds_addr(rcp4);
    const int crmb = 4 * crm1 + bias;              // 4 c + bias, c = cR_{j-1}
    const int gcb = 4 * dm1 - j * (4 * crm1 + bias);  // 4 g(c) - j bias
    const int dm1_4 = 4 * dm1;
    const int negj = -j;
    const bool w1ok = cval && (j < a.B - 1);
    const bool want_w1 = a.w1sum != nullptr;
    constexpr float inv_m = 1.0f / (float)m;
    wave_sync();

    // bin column q sits at byte (q / T) * TP + q % T of a ring row; a ring
    // row holds the S channels' rows back to back (nlb bytes).  Bins are
    // < 64; 0x7F marks columns outside the image or padding (never counted
    // by the 7-bit comparison below).  When the row fits LRN bytes per lane,
    // each lane's source offsets (relative to the group's first channel at
    // the row) are fixed for the tile: s H W + x, clamped to offset 0 for a
    // marker byte (bit i of lmark), and the row entering next is loaded into
    // registers one row ahead (issue_row) and written to the ring when it
    // enters (commit_row).  Every load is issued and its value used (ORed
    // with 0x7F for a marker), so no branch hides a load from the compiler's
    // count of loads in flight.
    const int nlb = S * rowb;
    constexpr int LRN = 4;
    const bool lfast = (nlb <= 64 * LRN) && ((long long)S * H * W < 0x7FFFFFFFLL);
    int loff[LRN];
    uint32_t lmark = 0;
#pragma unroll
    for (int i = 0; i < LRN; ++i) {
        const int t = lane + 64 * i;
        const int ss = t / rowb, o = t - ss * rowb;
        const int blk = o / TP, k = o - blk * TP;
        const int q = blk * T + k;
        const int cc = cbase + ss, xx = xb0 + q;
        const bool v = lfast && t < nlb && k < T && cc < a.C && q < Wb && xx >= 0 && xx < W;
        loff[i] = v ? ss * H * W + xx : 0;
        lmark |= v ? 0u : (1u << i);
    }
    uint32_t pre[LRN];
    auto issue_row = [&](int yy) {
        const uint8_t* rowp = a.bins + ((size_t)cbase * H + yy) * W;
#pragma unroll
        for (int i = 0; i < LRN; ++i) pre[i] = (uint32_t)rowp[loff[i]];
    };
    auto commit_row = [&](int yy) {
        uint8_t* dst = ring + (size_t)(yy % T1) * nlb;
#pragma unroll
        for (int i = 0; i < LRN; ++i)
            if (lane + 64 * i < nlb) dst[lane + 64 * i] = (uint8_t)((pre[i] | (((lmark >> i) & 1u) * 0x7Fu)) & 0x7Fu);
    };
    auto load_row = [&](int yy) {
        if (lfast) {
            issue_row(yy);
            commit_row(yy);
            return;
        }
        uint8_t* dst = ring + (size_t)(yy % T1) * nlb;
        for (int t = lane; t < nlb; t += 64) {
            const int ss = t / rowb, o = t - ss * rowb;
            const int blk = o / TP, k = o - blk * TP;
            const int q = blk * T + k;
            const int cc = cbase + ss, xx = xb0 + q;
            uint8_t v = 0x7F;
            if (k < T && cc < a.C && q < Wb && xx >= 0 && xx < W)
                v = a.bins[((size_t)cc * H + yy) * W + xx] & 0x7F;
            dst[t] = v;
        }
    };
    // vc[q] += [bin(row ya, q) <= j] - [bin(row yr, q) <= j], four columns per
    // dword: for 7-bit bytes b and j < 64, 0x80 + j - b never borrows across
    // bytes and its top bit is set exactly when b <= j.  ADD / REM select at
    // compile time whether a row enters and whether one leaves.
    const uint32_t jhi = ((uint32_t)j * 0x01010101u) | 0x80808080u;
    // The ring rows and the lane's count row never overlap: declared so, and
    // taken in chunks whose loads are all issued before any store, so a row
    // costs a few LDS round trips rather than one per dword.
    auto update_vc = [&](int ya, int yr, auto addc, auto remc) {
        constexpr bool ADD = decltype(addc)::value, REM = decltype(remc)::value;
        const uint32_t* __restrict__ ra = (const uint32_t*)(ring + (size_t)(ya % T1) * nlb + sa * rowb);
        const uint32_t* __restrict__ rr = (const uint32_t*)(ring + (size_t)((yr + T1) % T1) * nlb + sa * rowb);
        uint32_t* __restrict__ v = vc32 + lane * L.vs4;
        const int nd = rowb / 4;
        constexpr int CH = 8;
        for (int d0 = 0; d0 < nd; d0 += CH) {
            uint32_t xv[CH], xa[CH], xr[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int d = min(d0 + i, nd - 1);  // the tail rereads the last dword
                xv[i] = v[d];
                if (ADD) xa[i] = ra[d];
                if (REM) xr[i] = rr[d];
            }
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                uint32_t x = xv[i];
                if (ADD) x += ((jhi - xa[i]) & 0x80808080u) >> 7;
                if (REM) x -= ((jhi - xr[i]) & 0x80808080u) >> 7;
                if (d0 + i < nd) v[d0 + i] = x;
            }
        }
    };

    // gather work items of a block: item it*64+lane -> (channel slot, column k, pending row t)
    constexpr int SMAX = (T <= 9) ? 4 : 2;  // channels per wavefront the gather budget covers
    constexpr int NIT = (T * T * SMAX + 63) / 64;
    // read the gather's operands ahead of each block where the extra
    // registers leave the occupancy unchanged (T = 13 and T >= 17 would lose
    // a wavefront per SIMD)
    constexpr bool GATHER_AHEAD = (T <= 11) || (T == 15);

    const int ys = W1O ? y0 : max(0, y0 - r);
    const int yend = W1O ? ye : min(H, ye + r);
    const int lo_add = max(0, ys - r);
    const int hi_add = min(H, ys + r);

    // Gather items of a row: item it*64+lane = (channel slot ss, pending row
    // t, step k), k fastest, so that neighbouring lanes read neighbouring
    // bin bytes of one ring row and neighbouring accumulators.  Pending row
    // t of image row y is output row yo = y - r + t, whose bins sit in ring
    // row yo mod T1 and whose sums go to accumulator row yo mod T.  Packed:
    //   w0 = ring offset (block 0) << 16 | hrow offset
    //   w1 = (accumulator row + channel offset + k) << 16 | valid << 15 | k
    // where step k of the block starting at step i0 adds to output column
    // i0 + k - 2r of that row.
    // From one image row to the next both offsets move by one row, minus a
    // whole ring (accumulator) period when they pass its end: the smaller of
    // the two unsigned candidates, because the other one wraps below zero.
    // Rows outside the band accumulate too: those above it are cleared once
    // complete, those below are never output (the accumulator ring of T rows
    // holds exactly the T pending rows).
    uint32_t g_w0[NIT], g_w1[NIT];
    // GS: the weights w(d - r), d = 0 .. T - 1 (uniform), and the vertical
    // weight of a gather item, w(r - t) = w(t - r) for pending row t
    float gw[GS ? T : 1];
    if constexpr (GS) {
#pragma unroll
        for (int d = 0; d < T; ++d) gw[d] = a.wgt[d];
    }
    float gwt[GS ? NIT : 1];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = it * 64 + lane;
        const int ss = idx / (T * T);
        const int rem2 = idx - ss * (T * T);
        const int t = rem2 / T, k = rem2 - t * T;
        if constexpr (GS) gwt[it] = a.wgt[t];
        const bool ok = (ss < S) && (cbase + ss < a.C);
        const int ssc = (ss < S) ? ss : 0;
        const int yo = ys - r + t;
        const int rrow = ((yo % T1) + T1) % T1, arow = ((yo % T) + T) % T;
        const uint32_t ro = (uint32_t)(rrow * nlb + ssc * rowb + k);
        const uint32_t ho = (uint32_t)(ssc * Bp * HS + k);
        const uint32_t ao = (uint32_t)((arow * S + ssc) * Ws + k);
        g_w0[it] = (ro << 16) | ho;
        g_w1[it] = (ao << 16) | (ok ? 0x8000u : 0u) | (uint32_t)k;
    }
    const uint32_t gstep0 = (uint32_t)nlb << 16, gwrap0 = (uint32_t)(T1 * nlb) << 16;
    const uint32_t gstep1 = (uint32_t)(S * Ws) << 16, gwrap1 = (uint32_t)(T * S * Ws) << 16;

    // Output columns of a row: column t = lane + 64 i of the strip (t < ws),
    // with 1 / n_x of its global column; fixed for the tile.  An output of
    // channel c at (yo, xg) is v = ((acc * delta_c fxs) * (1 / n_x)) * (1 / n_y),
    // rounded once to an integer and added to the channel sum: the S channel
    // values of a column are summed in the lane first (integer adds), so one
    // atomic add per column carries the wavefront's channels.
    constexpr int OSL = 4;
    constexpr int OSM = (T <= 9) ? 4 : 2;  // channels per wavefront (score_block_max_S)
    const bool ofast = (ws <= 64 * OSL) && (S <= OSM);
    // in-image weight of the windows around position x along one axis: their
    // count for the box, the sum of w(d) for a finite sigma_p (fixed order)
    auto axis_weight = [&](int x, int len) -> double {
        if constexpr (GS) {
            double sw = 0.0;
            for (int d = 0; d < T; ++d)
                if (x - r + d >= 0 && x - r + d < len) sw += (double)a.wgt[d];
            return sw > 0.0 ? sw : 1.0;
        } else {
            return (double)max(min(len - 1, x + r) - max(0, x - r) + 1, 1);
        }
    };
    double orx[OSL];
#pragma unroll
    for (int i = 0; i < OSL; ++i) orx[i] = 1.0 / axis_weight(x0 + lane + 64 * i, W);
    const double inv_fxs = 1.0 / a.fxs;

    for (int yy = lo_add; yy < hi_add; ++yy) {
        load_row(yy);
        wave_sync();
        update_vc(yy, yy, bconst<true>(), bconst<false>());
        wave_sync();
    }
    if (lfast && ys + r < H) issue_row(ys + r);

    for (int y = ys; y < yend; ++y) {
        const bool add = (y + r) < H;
        const bool rem = (y - r - 1) >= lo_add;
        if (add) {
            if (lfast)
                commit_row(y + r);  // loaded during the previous row
            else
                load_row(y + r);
        }
        wave_sync();
        if (add && rem)
            update_vc(y + r, y - r - 1, bconst<true>(), bconst<true>());
        else if (add)
            update_vc(y + r, y - r - 1, bconst<true>(), bconst<false>());
        else if (rem)
            update_vc(y + r, y - r - 1, bconst<false>(), bconst<true>());
        // the row entering next goes to the ring slot of row y - r - 1, which
        // the update above has just consumed; its loads overlap this row
        if (lfast && y + 1 < yend && y + r + 1 < H) issue_row(y + r + 1);
        const int ny = min(H - 1, y + r) - max(0, y - r) + 1;
        const bool row_full = (ny == T);
        const bool own_row = (y >= y0) && (y < ye);
        // inspection stores (DBG only): step i is patch column x0 - r + i;
        // cpv carries 4 cP + bias and I4 = 4 I
        // (full windows compute I with unscaled masses: the stored value is
        // brought to the scaled masses P T^2, R n of the clipped windows)
        auto dbg_store = [&](int i, int cpb_k, int I4, bool full_w) {
            const int p = x0 - r + i;
            if (own_row && cval && j < a.B && p >= x0 && p < xe) {
                const size_t o = (((size_t)c * H + y) * W + p) * a.B + j;
                a.dbg_cp[o] = (cpb_k - bias) >> 2;
                a.dbg_I[o] = full_w ? (I4 >> 2) * m : (I4 >> 2);
            }
        };
        (void)dbg_store;
        // Step i walks patch column p = x0 - r + i; its window covers bin
        // columns q in [i, i + 2r].  The count entering at step i is vc[i + 2r]
        // and the one leaving is vc[i - 1].
        // bin columns 0 .. 2r-1 (layout block 0): byte sums of whole dwords
        uint32_t c0 = 0;
        {
            const uint32_t* vw = vc32 + lane * L.vs4;
#pragma unroll
            for (int d = 0; d < (T - 1) / 4; ++d) c0 = __builtin_amdgcn_sad_u8(vw[d], 0u, c0);
            if ((T - 1) % 4)
                c0 = __builtin_amdgcn_sad_u8(vw[(T - 1) / 4] & ((1u << (8 * ((T - 1) % 4))) - 1u), 0u, c0);
        }
        int cpb = 4 * (int)c0 + bias;
        // Block blk reads the count bytes [blk TP, blk TP + TP + T - 1) of the
        // lane's row, which the next block's range overlaps by TP bytes: a
        // window of 2 TPD dwords is kept in registers, and the TPD dwords the
        // next block adds are loaded while this block computes (the counts do
        // not change during the walk).  Windows above T = 21 would not fit the
        // registers; they read the bytes from LDS in each block.
        constexpr bool WIN = T <= 21;
        constexpr int TPD = TP / 4;
        const uint32_t* vw = vc32 + lane * L.vs4;
        uint32_t win[WIN ? 2 * TPD : 1], nxt[WIN ? TPD : 1];
        if constexpr (WIN) {
#pragma unroll
            for (int i = 0; i < 2 * TPD; ++i) win[i] = vw[i];
        }
        int ent0 = 0;  // count that entered at step k = 0 of the previous block
        // suffix sums of the previous block's errors (suf[k] = sum over
        // k' >= k); with GS the previous block's errors themselves
        float suf[T];
#pragma unroll
        for (int k = 0; k < T; ++k) suf[k] = 0.f;
        for (int blk = 0; blk < nblk; ++blk) {
            const int i0 = blk * T;
            const int p0 = x0 - r + i0;  // patch column of the block's first step
            // (decided by the block's image columns only, so that a block of
            // patch columns takes the same path in every tiling; steps past
            // the strip's last patch column feed no output)
            const bool full = row_full && (p0 >= r) && (p0 + T - 1 <= W - 1 - r);
            // 0. the gather's bin bytes and accumulators, read ahead: neither
            //    is written during the block (the ring rows are fixed within a
            //    row, and the accumulator columns of different blocks are
            //    disjoint), so their latency hides behind steps 1 and 2.
            //    The output column of step k is o = i0 + k - 2r, whose bin
            //    column i0 + k sits at byte blk*TP + k.
            //    When every step's output column lies inside the strip (gin),
            //    only the channel of an item decides whether it is stored.
            const bool gat = (i0 + T - 1 >= 2 * r);
            const bool gin = (i0 >= 2 * r) && (i0 + T - 1 - 2 * r < ws);
            int gbin[NIT], gdst[NIT];
            float gacc[NIT];
            auto gather_ahead = [&](auto inner) {
                constexpr bool IN = decltype(inner)::value;
#pragma unroll
                for (int it = 0; it < NIT; ++it) {
                    const uint32_t w0 = g_w0[it], w1 = g_w1[it];
                    const int xo = i0 + (int)(w1 & 63u) - 2 * r;
                    const bool ok = IN ? (w1 & 0x8000u) != 0u : ((w1 & 0x8000u) && (xo >= 0) && (xo < ws));
                    const float* dst = ok ? (acc + (int)(w1 >> 16) + (i0 - 2 * r)) : trash_l;
                    gbin[it] = ring[(w0 >> 16) + blk * TP];
                    gdst[it] = lds_addr(dst);
                    gacc[it] = *dst;
                }
            };
            if (!W1O && GATHER_AHEAD && gat) {
                if (FASTG && gin)
                    gather_ahead(bconst<true>());
                else
                    gather_ahead(bconst<false>());
            }
            if (WIN && blk + 1 < nblk) {
#pragma unroll
                for (int i = 0; i < TPD; ++i) nxt[WIN ? i : 0] = vw[(blk + 2) * TPD + i];
            }
            // 1. counts entering and leaving the window, running cumulative counts
            int cpv[T], cmv[T];
            const uint8_t* vb = vcl + blk * TP;
            auto vbyte = [&](int q) {
                if constexpr (WIN)
                    return (int)((win[q >> 2] >> (8 * (q & 3))) & 0xFFu);
                else
                    return (int)vb[q];
            };
#pragma unroll
            for (int k = 0; k < T; ++k) {
                // entering: bin column i0 + k + 2r = (blk + 1) T + k - 1;
                // leaving:  bin column i0 + k - 1 = blk T + k - 1
                const int ve = (k == 0) ? vbyte(T - 1) : vbyte(TP + k - 1);
                const int vl = (k == 0) ? ent0 : vbyte(k - 1);
                if (k == 0) ent0 = ve;
                cpb += (ve - vl) << 2;
                cpv[k] = cpb;
            }
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const int u = lane_prev(cpv[k]);
                cmv[k] = j0 ? bias : u;
            }
            if constexpr (W1O) {
                // each lane's |4 (cP_j m - cR_j n)| (bins j < B - 1), summed over
                // the channel's Bp lanes by cross-lane adds (every lane of the
                // group ends with the sum), scaled by the group's first lane
                // and added to the channel sum of the patch
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    const int p = x0 - r + i0 + k;
                    const int nx = max(1, min(W - 1, p + r) - max(0, p - r) + 1);
                    const int n = ny * nx;
                    int d = w1ok ? abs((cpv[k] - bias) * m - crl4 * n) : 0;
                    d = group_sum(d, Bp);
                    if (j0 && cval && p >= x0 && p < xe) {
                        const double v = ((double)d * (a.delta[c] * a.fxs * 0.25)) / ((double)n * (double)m);
                        __hip_atomic_fetch_add(&a.w1sum[(size_t)y * W + p], __double2ll_rn(v), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            } else {
            float ev[T];
            if (full) {
                int gv[T];
                float rc[T];
#pragma unroll
                for (int k = 0; k < T; ++k) gv[k] = lds_load_i(cpv[k]);
#pragma unroll
                for (int k = 0; k < T; ++k) rc[k] = lds_load_f(RCP0 ? cpv[k] - cmv[k] : rbase + (cpv[k] - cmv[k]));
#pragma unroll
                for (int k = 0; k < T; ++k) gv[k] += __mul24(negj, cpv[k]);  // 4 g(v) - j bias
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    const int un = lane_prev(gv[k]);  // the neighbour's 4 g(u) - (j - 1) bias, plus 4u
                    const int gu = j0 ? 0 : un - cmv[k];
                    const int mn = (crmb <= cmv[k]) ? gu : ((crmb >= cpv[k]) ? gv[k] : gcb);
                    const int I4 = (gu + gv[k]) - (mn << 1);
                    ev[k] = (float)I4 * rc[k];
                    if constexpr (DBG) dbg_store(i0 + k, cpv[k], I4, true);
                }
            } else {
                // Windows clipped at the image border (or rows with fewer than
                // T window rows): the general equal-mass form.  Columns go in
                // groups of G whose table reads are issued together, so a group
                // costs one round of LDS reads instead of several per column;
                // q = floor(a / n) comes from a reciprocal estimate corrected to
                // the exact integer (the estimate is within one of it).
                const float* rcf = rcp4;
                constexpr int G = (T <= 8) ? 4 : 5;  // keeps T = 7 within three wavefronts per SIMD and T = 15 within two
#pragma unroll
                for (int k0 = 0; k0 < T; k0 += G) {
                    // a group whose patch columns all lie outside the image
                    // contributes nothing (the same zeros its steps would give)
                    const int pg = x0 - r + i0 + k0;
                    if (pg + G - 1 < 0 || pg >= W) {
#pragma unroll
                        for (int kk = 0; kk < G; ++kk)
                            if (k0 + kk < T) ev[k0 + kk] = 0.f;
                        continue;
                    }
                    int gn[G], gav[G], gq[G], gP[G], gau[G], gps0[G], gps1[G];
                    float grc[G];
#pragma unroll
                    for (int kk = 0; kk < G; ++kk) {
                        const int k = k0 + kk;
                        if (k < T) {
                            const int p = x0 - r + i0 + k;
                            const int nx = max(1, min(W - 1, p + r) - max(0, p - r) + 1);
                            const int n = ny * nx;
                            const int cPk = (cpv[k] - bias) >> 2, cPm1 = (cmv[k] - bias) >> 2;
                            const int av = __mul24(cPk, m);
                            int q = (int)((float)av * __builtin_amdgcn_rcpf((float)n));
                            q = max(0, min(q, m));
                            q += (q < m && __mul24(q + 1, n) <= av) ? 1 : 0;
                            q -= (q > 0 && __mul24(q, n) > av) ? 1 : 0;
                            gn[kk] = n;
                            gav[kk] = av;
                            gq[kk] = q;
                            gau[kk] = __mul24(cPm1, m);
                            gP[kk] = min(max(cPk - cPm1, 0), m);
                        }
                    }
#pragma unroll
                    for (int kk = 0; kk < G; ++kk) {
                        if (k0 + kk < T) {
                            gps0[kk] = psl[gq[kk]];  // 4 Psi(q)
                            gps1[kk] = psl[gq[kk] + 1];  // 4 Psi(q + 1)
                            grc[kk] = rcf[gP[kk]];
                        }
                    }
#pragma unroll
                    for (int kk = 0; kk < G; ++kk) {
                        const int k = k0 + kk;
                        if (k < T) {
                            const int i = i0 + k;
                            const int p = x0 - r + i;
                            const bool pval = (i < np) && (p >= 0) && (p < W);
                            const int n = gn[kk], av = gav[kk], au = gau[kk];
                            const int phia = __mul24(n, gps0[kk]) + __mul24(av - __mul24(gq[kk], n), gps1[kk] - gps0[kk]);
                            const int pu = lane_prev(phia);
                            const int phiu = j0 ? 0 : pu;
                            const int cm = __mul24(crm1, n);
                            const int sc = min(max(cm, au), av);
                            const int phis = (cm <= au) ? phiu : ((cm >= av) ? phia : __mul24(n, dm1_4));
                            const int I4 = (phia - phis) + (phiu - phis) + __mul24(4 * j, 2 * sc - au - av);
                            ev[k] = pval ? (float)I4 * grc[kk] * inv_m : 0.f;
                            if constexpr (DBG) dbg_store(i, cpv[k], I4, false);
                        }
                    }
                }
            }
            if (want_w1 && own_row) {
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    const int p = x0 - r + i0 + k;
                    if (p >= x0 && p < xe) {
                        const int nx = min(W - 1, p + r) - max(0, p - r) + 1;
                        const int n = ny * nx;
                        int d = w1ok ? abs((cpv[k] - bias) * m - crl4 * n) : 0;
                        for (int o = Bp >> 1; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
                        if (cval && j == 0) {
                            const double v = ((double)d * (a.delta[c] * a.fxs * 0.25)) / ((double)n * (double)m);
                            __hip_atomic_fetch_add(&a.w1sum[(size_t)y * W + p], __double2ll_rn(v), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                }
            }
            // 2. horizontal window sums: after step i0 + k the window holds
            //    steps [i0 + k - 2r, i0 + k] = previous block's k+1 .. T-1 and
            //    this block's 0 .. k; output column o = i0 + k - 2r
            if constexpr (GS) {
                // suf holds the previous block's errors; step i0 + k - 2r + d
                // has weight w(d - r) for the output of step k
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    float h = 0.f;
#pragma unroll
                    for (int d = 0; d < T; ++d) {
                        const int si = k - 2 * r + d;
                        h = __builtin_fmaf(gw[d], si < 0 ? suf[si + T] : ev[si], h);
                    }
                    hrow[lane * HS + k] = h;
                }
#pragma unroll
                for (int k = 0; k < T; ++k) suf[k] = ev[k];
            } else {
                float pre = 0.f;
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    pre += ev[k];
                    hrow[lane * HS + k] = (k < T - 1) ? suf[k + 1] + pre : pre;
                }
                float sf = 0.f;
#pragma unroll
                for (int k = T - 1; k >= 1; --k) {
                    sf += ev[k];
                    suf[k] = sf;
                }
            }
            wave_sync();
            // 3. gather the pixel's own bin into the accumulators of the T
            //    pending output rows
            //    (every read is issued before any accumulator store: the
            //    regions are disjoint, which the compiler cannot see, and one
            //    item at a time would cost an LDS round trip each)
            if (GATHER_AHEAD && gat) {
                float hv[NIT];
#pragma unroll
                for (int it = 0; it < NIT; ++it) hv[it] = hrow[(g_w0[it] & 0xFFFFu) + (gbin[it] & (Bp - 1)) * HS];
#pragma unroll
                for (int it = 0; it < NIT; ++it)
                    lds_store_f(gdst[it], GS ? __builtin_fmaf(gwt[GS ? it : 0], hv[it], gacc[it]) : gacc[it] + hv[it]);
            } else if (gat) {
                constexpr int CHK = 8;  // items per round of reads
                auto gather_chunks = [&](auto inner) {
                    constexpr bool IN = decltype(inner)::value;
#pragma unroll
                    for (int c0 = 0; c0 < NIT; c0 += CHK) {
                        int bv[CHK], da[CHK];
                        float hv[CHK], av[CHK];
#pragma unroll
                        for (int q = 0; q < CHK; ++q) {
                            if (c0 + q < NIT) {
                                const uint32_t w0 = g_w0[c0 + q], w1 = g_w1[c0 + q];
                                const int xo = i0 + (int)(w1 & 63u) - 2 * r;
                                const bool ok =
                                    IN ? (w1 & 0x8000u) != 0u : ((w1 & 0x8000u) && (xo >= 0) && (xo < ws));
                                bv[q] = ring[(w0 >> 16) + blk * TP];
                                da[q] = lds_addr(ok ? (acc + (int)(w1 >> 16) + (i0 - 2 * r)) : trash_l);
                            }
                        }
#pragma unroll
                        for (int q = 0; q < CHK; ++q) {
                            if (c0 + q < NIT) {
                                hv[q] = hrow[(g_w0[c0 + q] & 0xFFFFu) + (bv[q] & (Bp - 1)) * HS];
                                av[q] = lds_load_f(da[q]);
                            }
                        }
#pragma unroll
                        for (int q = 0; q < CHK; ++q)
                            if (c0 + q < NIT)
                                lds_store_f(da[q], GS ? __builtin_fmaf(gwt[GS ? c0 + q : 0], hv[q], av[q]) : av[q] + hv[q]);
                    }
                };
                if (FASTG && gin)
                    gather_chunks(bconst<true>());
                else
                    gather_chunks(bconst<false>());
            }
            wave_sync();
            }
            if constexpr (WIN) {
#pragma unroll
                for (int i = 0; i < TPD; ++i) {
                    win[i] = win[TPD + i];
                    win[TPD + i] = nxt[i];
                }
            }
        }
        if constexpr (!W1O) {
        // the pending rows move down by one
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const uint32_t u0 = g_w0[it] + gstep0, u1 = g_w1[it] + gstep1;
            g_w0[it] = min(u0, u0 - gwrap0);
            g_w1[it] = min(u1, u1 - gwrap1);
        }
        // row y - r is complete: above the band it is only cleared
        if (y - r < y0) {
            float* ap = acc + ((((y - r) % T) + T) % T) * S * Ws;
            for (int t = lane; t < S * Ws; t += 64) ap[t] = 0.f;
        }
        int yo_lo = y - r, yo_hi = (y < H - 1) ? y - r : H - 1;
        yo_lo = max(yo_lo, y0);
        yo_hi = min(yo_hi, ye - 1);
        for (int yo = yo_lo; yo <= yo_hi; ++yo) {
            const double rny = 1.0 / axis_weight(yo, H);
            float* ar = acc + (yo % T) * S * Ws;
            if (ofast) {
                // every read of the row before the stores that clear it
                float ov[OSL][OSM];
#pragma unroll
                for (int i = 0; i < OSL; ++i)
#pragma unroll
                    for (int ss = 0; ss < OSM; ++ss)
                        ov[i][ss] = (lane + 64 * i < ws && ss < S) ? ar[ss * Ws + lane + 64 * i] : 0.f;
#pragma unroll
                for (int i = 0; i < OSL; ++i)
#pragma unroll
                    for (int ss = 0; ss < OSM; ++ss)
                        if (lane + 64 * i < ws && ss < S) ar[ss * Ws + lane + 64 * i] = 0.f;
#pragma unroll
                for (int i = 0; i < OSL; ++i) {
                    if (lane + 64 * i < ws) {
                        const int xg = x0 + lane + 64 * i;
                        long long qs = 0;
#pragma unroll
                        for (int ss = 0; ss < OSM; ++ss) {
                            const int cc = cbase + ss;
                            if (ss < S && cc < a.C) {
                                const double v = (((double)ov[i][ss] * (a.delta[cc] * a.fxs)) * orx[i]) * rny;
                                qs += __double2ll_rn(v);
                                if (a.achan) a.achan[((size_t)cc * H + yo) * W + xg] = (float)(v * inv_fxs);
                            }
                        }
                        __hip_atomic_fetch_add(&a.asum[(size_t)yo * W + xg], qs, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                continue;
            }
            for (int t = lane; t < S * ws; t += 64) {
                const int ss = t / ws, xo = t - ss * ws;
                const int cc = cbase + ss;
                float* ap = ar + ss * Ws + xo;
                const float av = *ap;
                *ap = 0.f;
                if (cc < a.C) {
                    const int xg = x0 + xo;
                    const double v = (((double)av * (a.delta[cc] * a.fxs)) * (1.0 / axis_weight(xg, W))) * rny;
                    if (a.achan) a.achan[((size_t)cc * H + yo) * W + xg] = (float)(v * inv_fxs);
                    __hip_atomic_fetch_add(&a.asum[(size_t)yo * W + xg], __double2ll_rn(v), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        }
        wave_sync();
    }
}


typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));


__device__ __forceinline__ int bin_of_m(float rr, const float* __restrict__ e, float lo, float idl, int B) {
    int b = idl == 0.f ? 0 : (int)floorf((rr - lo) * idl);  // zero width: walk from bin 0
    b = b < 0 ? 0 : (b > B - 1 ? B - 1 : b);
    while (b > 0 && rr < e[b - 1]) --b;
    while (b < B - 1 && rr >= e[b]) ++b;
    return b;
}

// bin = #{m : rr >= e[m]} (B >= 2): the arithmetic guess from (rr - lo) / delta
// is checked against its two neighbouring edges (read together); only when
// that moves it is the search continued edge by edge.  A zero-width channel
// (idl = 0) starts the search at bin 0.
__device__ __forceinline__ int bin_fast(float rr, const float* __restrict__ e, float lo, float idl, int B) {
    int b = idl == 0.f ? 0 : (int)floorf((rr - lo) * idl);
    b = b < 0 ? 0 : (b > B - 1 ? B - 1 : b);
    const float el = e[b > 0 ? b - 1 : 0];
    const float eh = e[b < B - 1 ? b : B - 2];
    const int b1 = b - ((b > 0 && rr < el) ? 1 : 0) + ((b < B - 1 && rr >= eh) ? 1 : 0);
    if (b1 != b) {
        b = b1;
        while (b > 0 && rr < e[b - 1]) --b;
        while (b < B - 1 && rr >= e[b]) ++b;
    }
    return b;
}

// Residuals and bins of NE values of one pixel px (channels cs[e], residuals
// rv[e]); `valid` marks the values whose pixel and channel exist.  edges:
// the [C][B-1] edge table (read only for values next to an edge).  slo, sid,
// sfd: per-channel lo, 1/delta and margin dl in LDS (arrays of the block's
// channel capacity, so every cs[e] may be read).  stg: the block's bin
// staging area [CMAX][16] in LDS (the caller writes it out; bytes of invalid
// values are never stored), or nullptr to store each bin directly.
// bin = #{m : r >= e[m]}: t = (r - lo) / delta decides it on its own when t
// lies at least dl from every integer edge position 1 .. B-1 (dl bounds
// the stored edges' distance from the grid lo + m delta plus the FP32
// rounding of t; a margin of one half or more disables this): floor(t) in
// range, 0 below the grid, B-1 above it.  The test is made without branches
// for all NE values; the edge search (bin_fast) runs only when some lane of
// the wavefront has a value next to an edge, and then only for such values.
template <int NE>
__device__ __forceinline__ void emit_values(const MArgs& a, int px, const int (&cs)[NE], const float (&rv)[NE],
                                            const bool (&valid)[NE], const float* slo, const float* sid,
                                            const float* sfd, const float* edges, uint8_t* stg) {
    if (a.resid) {
#pragma unroll
        for (int e = 0; e < NE; ++e)
            if (valid[e]) a.resid[(size_t)cs[e] * a.N + px] = rv[e];
    }
    if (!a.bins) return;
    const int B = a.B;
    int bq[NE];
    uint32_t need = 0;
    if (B > 1) {
        const float top = (float)(B - 1);
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int c = cs[e];
            const float lo = slo[c], idl = sid[c], dl = sfd[c];
            const float t = (rv[e] - lo) * idl;
            // the edge position nearest to t is rint(t) clamped to [1, B-1];
            // t is decided when it lies at least dl from it, and its bin is
            // then floor(t) clamped to [0, B-1] (NaN is never decided)
            const float near = __builtin_amdgcn_fmed3f(rintf(t), 1.f, top);
            const bool dec = fabsf(t - near) >= dl;  // +infinity: the shortcut is off
            bq[e] = (int)__builtin_amdgcn_fmed3f(floorf(t), 0.f, top);
            need |= (!dec && valid[e]) ? (1u << e) : 0u;
        }
        if (__ballot(need != 0u)) {
#pragma unroll
            for (int e = 0; e < NE; ++e)
                if (need & (1u << e)) {
                    const int c = cs[e];
                    bq[e] = bin_fast(rv[e], edges + (size_t)c * (B - 1), slo[c], sid[c], B);
                }
        }
    } else {
#pragma unroll
        for (int e = 0; e < NE; ++e) bq[e] = 0;
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        if (stg)
            stg[cs[e] * 16 + (px & 15)] = (uint8_t)bq[e];
        else if (valid[e])
            a.bins[(size_t)cs[e] * a.N + px] = (uint8_t)bq[e];
    }
}

// Calls f(std::integral_constant<int, S>) for S = I .. N - 1 in order: an
// unrolled loop whose index is a constant in every copy of the body (a body
// too large for the loop unroller would otherwise index register arrays at
// run time, which puts them in scratch memory).
template <int I, int N>
struct StaticFor {
    template <class F>
    __device__ __forceinline__ static void run(F& f) {
        f(std::integral_constant<int, I>{});
        StaticFor<I + 1, N>::run(f);
    }
};
template <int N>
struct StaticFor<N, N> {
    template <class F>
    __device__ __forceinline__ static void run(F&) {}
};

// Transposes the 4x4 bytes of a lane quad: lane p's byte v becomes lane v's
// byte p.
__device__ __forceinline__ uint32_t quad_transpose_bytes(uint32_t d, uint32_t selA, uint32_t selB) {
    const uint32_t pa = (uint32_t)__builtin_amdgcn_mov_dpp((int)d, 0xB1, 0xf, 0xf, false);  // lane p ^ 1
    const uint32_t a1 = __builtin_amdgcn_perm(d, pa, selA);
    const uint32_t pb = (uint32_t)__builtin_amdgcn_mov_dpp((int)a1, 0x4E, 0xf, 0xf, false);  // lane p ^ 2
    return __builtin_amdgcn_perm(a1, pb, selB);
}

// Hides an LDS pointer's value from the optimiser, so that loads through it
// inside a loop are not hoisted out of it (keeping every table entry of a
// tile live across iterations would take more registers than reloading).
template <class T>
__device__ __forceinline__ const T* opaque_lds(const T* p) {
    uint32_t v = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const T*)p;
    asm volatile("" : "+s"(v));
    return (const T*)(__attribute__((address_space(3))) const T*)(uintptr_t)v;
}

// Writes a block's (256 threads) staged bins of one 16-pixel tile: one
// 16-byte channel row per thread, without per-thread branches (threads past
// the last channel write that channel's row again, the same bytes), so the
// compiler can count the memory operations in flight exactly; byte by byte
// for a ragged last tile or a width that is not a multiple of 16.  Called by
// all threads of the block after a barrier.
template <int CMAX>
__device__ __forceinline__ void proj_store_bins(const MArgs& a, int tile, const uint8_t* stg) {
    const int p0 = tile * 16;
    const bool whole = (p0 + 16 <= a.N) && ((a.N & 15) == 0) && (((uintptr_t)a.bins & 15) == 0);
    if (whole) {
#pragma unroll
        for (int r = 0; r < (CMAX + 255) / 256; ++r) {
            const int c = threadIdx.x + 256 * r;
            const int cs = c < a.C ? c : a.C - 1;
            *(uint4*)(a.bins + (size_t)cs * a.N + p0) = *(const uint4*)(stg + cs * 16);
        }
    } else {
        for (int c = threadIdx.x; c < CMAX && c < a.C; c += blockDim.x) {
            uint8_t* dst = a.bins + (size_t)c * a.N + p0;
            for (int q = 0; q < 16 && p0 + q < a.N; ++q) dst[q] = stg[c * 16 + q];
        }
    }
}

// Features of one 16-pixel tile for wave w: the FP32 tile's GEMM1 B operands
// (channel 4 s + g, s = w NSW + i, pixel n) and the BF16 tile's (channels
// 32 s + 8 g + t).  Loaded separately so that a caller can prefetch them.
// Every load is issued, from a clamped, valid address, and its value is
// used as loaded: with no branch around a load the compiler knows how many
// are in flight and waits only for the ones it needs.  Lanes of pixels past
// the map compute on a real pixel's features and are never stored; channels
// past C meet zero rows of the operand tables (and their residuals are never
// stored), so the features they load do not enter any result.
template <int CMAX>
__device__ __forceinline__ void proj_load_f32(const MArgs& a, int tile, int w, int lane, float (&x)[CMAX / 16]) {
    constexpr int NSW = CMAX / 16;
    const int g = lane >> 4, n = lane & 15;
    const int px = tile * 16 + n;
    const bool pxok = px < a.N;
    const int pxc = pxok ? px : a.N - 1;
#pragma unroll
    for (int i = 0; i < NSW; ++i) {
        const int c = 4 * (w * NSW + i) + g;
        const int cc = c < a.C ? c : a.C - 1;
        x[i] = a.X[(size_t)cc * a.N + pxc];
    }
}

template <int CMAX>
__device__ __forceinline__ void proj_load_bf16(const MArgs& a, int tile, int w, int lane,
                                               float (&x)[CMAX / 128][8]) {
    constexpr int NSW = CMAX / 128;
    const int g = lane >> 4, n = lane & 15;
    const int px = tile * 16 + n;
    const bool pxok = px < a.N;
    const int pxc = pxok ? px : a.N - 1;
#pragma unroll
    for (int i = 0; i < NSW; ++i)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int c = 32 * (w * NSW + i) + 8 * g + t;
            const int cc = c < a.C ? c : a.C - 1;
            x[i][t] = a.X[(size_t)cc * a.N + pxc];
        }
}

template <int CMAX, int KT>
__device__ __forceinline__ void proj_tile_f32(const MArgs& a, int tile, int w, int lane,
        const float* __restrict__ V1, const float* __restrict__ V2, const float* smu, const float* slo,
        const float* sid, const float* sfd, float* zp, const float (&x)[CMAX / 16], const float* edges,
        uint8_t* stg) {
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
        d[i] = x[i] - smu[c];
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
    block_sync_lds();
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
    block_sync_lds();
    int cs[NSW];
    float rv[NSW];
    bool valid[NSW];
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
            cs[4 * i + v] = c;
            rv[4 * i + v] = d[4 * i + v] - acc[v];
            valid[4 * i + v] = pxok && c < a.C;
        }
    }
    emit_values<NSW>(a, px, cs, rv, valid, slo, sid, sfd, edges, stg);
}

template <int CMAX, int KT>
__device__ __forceinline__ void proj_tile_bf16(const MArgs& a, int tile, int w, int lane,
        const bf16x8* __restrict__ V1, const bf16x8* __restrict__ V2, const float* smu, const float* slo,
        const float* sid, const float* sfd, float* zp, const float (&x)[CMAX / 128][8], const float* edges,
        uint8_t* stg) {
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
            d[i][t] = x[i][t] - smu[c];
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
    block_sync_lds();
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
    block_sync_lds();
    int cs[NSW * 8];
    float rv[NSW * 8];
    bool valid[NSW * 8];
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
                const int e = 8 * i + 4 * h + v;
                cs[e] = c;
                rv[e] = d[i][4 * h + v] - acc[v];
                valid[e] = pxok && c < a.C;
            }
        }
    }
    emit_values<NSW * 8>(a, px, cs, rv, valid, slo, sid, sfd, edges, stg);
}


}  // namespace tiles
}  // namespace qfca
