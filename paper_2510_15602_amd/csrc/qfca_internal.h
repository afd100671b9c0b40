// Internal declarations shared by the libqfca translation units (not part of
// the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/qfca.h"

namespace qfca {

// Arguments of one score tile (see qfca_tiles.h).
// The channel sum of the per-channel maps is accumulated in 64-bit fixed
// point: every (channel, pixel) value v is rounded once to llrint(v * fxs)
// and added with an integer atomic, so the sum does not depend on the order
// in which tiles, channel groups or batch items finish.  fxs is a power of
// two chosen per model so that the sum over all channels stays below 2^62
// (every per-channel value is at most (B - 1) delta_c).
struct KArgs {
    const uint8_t* bins;
    int C, H, W, T, B, Bp, S, r, m, Ws, Hb, WbA;
    const int2* psig;
    const int32_t* cRm1;
    const int32_t* Dm1;
    const int32_t* cRl;
    const float* rcp;
    const double* delta;
    double fxs;        // fixed-point scale of asum and w1sum
    long long* asum;   // [H][W] sum over channels of A_c, fixed point (atomic adds)
    long long* w1sum;  // [H][W] sum over channels of W1_c, fixed point, or nullptr
    float* achan;      // [C][H][W] per-channel maps A_c (inspection output), or nullptr
    const double* cRw; // generic kernel: [C][B] cumulative weights of a general reference, or nullptr
    const float* wgt;  // generic kernel: [T] association weights for a finite sigma_p, or nullptr
    int* dbg_cp;       // inspection kernel only: [C][H][W][B] window cumulative counts cP_j
    int* dbg_I;        // inspection kernel only: [C][H][W][B] transport numerators I_j
};

// Arguments of the MFMA projection (see qfca_tiles.h).
struct MArgs {
    const float* X;
    int C, N, k, B;
    const float* mu;
    const void* V1;  // GEMM1 A operands
    const void* V2;  // GEMM2 A operands
    const float* edges;
    const float* lo;
    const float* inv_delta;
    const float* fastd;  // [C] margin of the arithmetic bin guess (see ProjLaunch)
    uint8_t* bins;
    float* resid;
    int ntiles;
};

// Batched path: one descriptor per image and one header per batch, both in
// device memory.
constexpr int BATCH_MAXJ = 256;
struct BatchJob {
    MArgs pa;             // projection of this image
    KArgs sa;             // score tiles of this image
    int ntiles_proj;      // projection items of this image
    int nstrips, nbands;  // score item grid (x strips, y bands; z = channel groups / 4)
    long long* asum;      // [H][W] fixed-point channel sum (zeroed by the projection items)
    double inv_scale;     // 1 / (fxs * C): asum to the channel mean
    float* amap;          // [H][W] channel mean, or nullptr
    float* score;         // [H][W] blurred score
};
struct BatchHeader {
    int head;             // next queue item
    int error;            // set if a wait gave up (never expected)
    int n, nproj, nitems, blur_R;
    double blur_w[17];
    int done[BATCH_MAXJ];
    int proj_prefix[BATCH_MAXJ + 1];
    int score_prefix[BATCH_MAXJ + 1];
};
size_t batch_wave_lds(int T, int S, int Ws);
size_t score_rcp_bytes(int T);  // block-shared reciprocal table of the score tiles
constexpr size_t BATCH_CTL_BYTES = 16;  // batch kernel: control words after the table
size_t batch_head_bytes(int T);  // batch kernel: table and control words, before the wave regions
size_t batch_proj_lds(int CMAX, int KT);
bool batch_supported(int T, int CMAX, int KT, int prec);
hipError_t prepare_batch(int T, int CMAX, int KT, int prec, size_t lds);
hipError_t launch_batch(int T, int CMAX, int KT, int prec, BatchHeader* hdr, const BatchJob* jobs,
                        int wave_lds, size_t lds, int grid, int maxn, hipStream_t st);

// Batched launch (the body of qfca_score_batch).  asum: per-job fixed-point
// channel-sum buffers of H*W int64, or nullptr for context scratch.
// err_host: pinned host word that receives the batch's wait-failure flag
// (stream-ordered after the batch), or nullptr.
qfca_status score_batch_ext(qfca_ctx ctx, const qfca_job* jobs, int32_t n, long long* const* asum,
                            int32_t* err_host);
// qfca_score_map's checks (and hipSetDevice), and its launch sequence on
// caller-given fixed-point buffers (dbg_cp, dbg_I: inspection outputs).
qfca_status score_map_check(qfca_ctx ctx, qfca_model m, const uint8_t* bins, int32_t H, int32_t W,
                            const float* score);
qfca_status score_map_into(qfca_ctx ctx, qfca_model m, const uint8_t* bins, int32_t H, int32_t W,
                           float* score, float* amap, float* w1, float* achan, long long* asum,
                           long long* w1sum, int* dbg_cp = nullptr, int* dbg_I = nullptr);
int ctx_device(qfca_ctx ctx);
qfca_status status_fail(qfca_status s, const std::string& msg);  // sets the message, returns s
// Allocation-free entry point: resolves the device address of the static
// scratch array on `device` (current), once per device.
hipError_t noalloc_init(int device);

// Validation of one job against the parameters p of its batch.
qfca_status batch_job_check(qfca_ctx ctx, const qfca_job& job, const qfca_params& p);

// Per-thread last error message, set by the API layer.
void set_error(const std::string& msg);

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Tile shape of the score kernel: strip width (output columns), band height
// (output rows) and channels per wavefront.
struct ScoreTile {
    int Ws = 64;
    int Hb = 64;
    int S = 1;
    int variant = 1;  // 0: runtime-T column walk, 1: compile-time-T block walk (T = 3..31)
};

// Device-resident tables of a model that the score kernel reads.  For the
// cumulative reference cR of channel c (total m = T*T):
//   psig[c][t] = (Psi_c(t), sigma_c(t)), t in [0, m], where
//     Psi_c(t)   = sum_{k<B-1} max(0, t - cR_c[k])   (integral of the reference
//                  bin index over the first t units of reference mass) and
//     sigma_c(t) = #{k < B-1 : cR_c[k] <= t}        (its slope on [t, t+1]);
//   cRm1[c][i] = cR_c[i-1] (0 for i = 0), Dm1[c][i] = Psi_c(cRm1[c][i]),
//   cRl[c][i] = cR_c[i] for i < B-1 and 0 otherwise (window W1 by-product);
//   rcp[P] = 1/P as float32 (rcp[0] = 0).
struct ScoreTables {
    int2* psig = nullptr;
    int32_t* cRm1 = nullptr;
    int32_t* Dm1 = nullptr;
    int32_t* cRl = nullptr;
    float* rcp = nullptr;
    double* delta = nullptr;  // [C]
    int Bp = 0;               // lanes per channel (power of two, >= 8)
    double fxs = 1.0;         // fixed-point scale of the channel sums (see KArgs)
    double* cRw = nullptr;    // [C][B] general reference weights (column-walk kernel), or nullptr
    float* wgt = nullptr;     // [T] association weights of a finite sigma_p (column-walk kernel), or nullptr
};

struct ScoreLaunch {
    const uint8_t* bins;  // [C][H][W]
    int C, H, W, T, B;
    ScoreTables tab;
    double fxs;           // fixed-point scale (ScoreTables::fxs of the model)
    long long* asum;      // [H][W] fixed-point channel sum (zeroed by the launcher)
    long long* w1sum;     // [H][W] or nullptr
    float* achan;         // [C][H][W] out or nullptr
    bool w1only = false;    // window W1 only (principal-coordinate models): w1sum required
    int* dbg_cp = nullptr;  // inspection kernel: [C][H][W][B] out (with dbg_I), or nullptr
    int* dbg_I = nullptr;
    ScoreTile tile;
};

size_t score_lds_bytes(int T, int Bp, int S, int Ws, int variant);
bool score_has_block_kernel(int T);
int score_block_max_S(int T);  // channels per wavefront the block walk supports
// Strip width the block walk runs for a requested Ws: a multiple of T (at
// least T), so that its blocks of T patch columns sit at the same image
// columns whatever the tiling.
int score_block_ws(int T, int Ws);
// Zeroes asum (and w1sum when given), then launches the score tiles.
hipError_t launch_score(const ScoreLaunch& L, hipStream_t st);
// Channel mean A = asum * inv_scale (written to amap when given), its
// sigma-blurred score, and the W1 channel mean w1 = w1sum * inv_scale when
// both are given.
// Principal-coordinate score: the plane mean of the window W1 map
// (w1sum * inv_scale; to w1 when given), its box mean over the windows
// holding each pixel (amap, required), and amap's sigma blur (score).
hipError_t launch_finish_w1(const long long* w1sum, double inv_scale, int H, int W, int T, float sigma,
                            float* amap, float* w1, float* score, hipStream_t st);
hipError_t launch_finish(const long long* asum, const long long* w1sum, double inv_scale, int H, int W,
                         float sigma, float* amap, float* w1, float* score, hipStream_t st);

// Reference fit: count table [C][B][m+1] (uint32, zeroed by the launcher) of
// full-window cumulative counts, then the selection of cR.
// perbin = 1 counts the windows' bin counts P(i) instead (for the
// references taken after the quantisation).
hipError_t launch_refcount(const uint8_t* bins, int C, int H, int W, int T, int B,
                           uint32_t* counts, hipStream_t st, int perbin = 0);
// From the perbin count table: cumulative reference weights cRw [C][B] of the
// bin-wise lower median (kind 0) or mean (kind 1) over the nw full windows.
hipError_t launch_refstat(const uint32_t* counts, int C, int B, int m, long long nw, int kind, double* cRw,
                          hipStream_t st);
// Rank-wise mean of the sorted full windows of the residual R [C][H][W],
// quantised with edges [C][B-1]: cumulative reference cR [C][B] (mass T*T).
// part: device scratch of refmean_part_bytes(C, T, ...) bytes.
size_t refmean_part_bytes(int C, int T, int* nparts, int* NP);
hipError_t launch_refmean(const float* R, int C, int H, int W, int T, const float* edges, int B, double* part,
                          int32_t* cR, hipStream_t st);
hipError_t launch_refselect(const uint32_t* counts, int C, int B, int m, long long h,
                            int32_t* cR, hipStream_t st);
// The median -> quan reference in one call: cR [C][B] = the h-th largest
// full-window cumulative count per (channel, bin).  counts: scratch of
// C B (T^2 + 1) words.  One pass with the whole count table when it fits
// in LDS, else a coarse pass (buckets of counts) and a fine pass inside each
// (channel, bin)'s median bucket.
hipError_t launch_refmedian(const uint8_t* bins, int C, int H, int W, int T, int B, uint32_t* counts,
                            long long h, int32_t* cR, hipStream_t st);

// Projection + quantisation.
struct ProjLaunch {
    const float* X;  // [C][N]
    int C, N, k, B;
    int preproc, prec;
    const float* mu;        // [C]
    const float* V;         // [C][k] float32
    const uint16_t* Vbf;    // [C][k] bf16 bits
    const float* edges;     // [C][B-1]
    const float* lo;        // [C]
    const float* inv_delta; // [C] (0 for a degenerate channel)
    // [C] margin, in bin units, beyond which t = (r - lo) * inv_delta in FP32
    // determines the bin on its own: the largest distance of a stored edge
    // from the grid lo + m delta plus the rounding bound of t; >= 0.5 when
    // the edges must always be consulted
    const float* fastd;
    uint8_t* bins;          // [C][N] or nullptr
    float* resid;           // [C][N] or nullptr
    const void* V1 = nullptr;  // MFMA operand tables (precision of prec), or nullptr
    const void* V2 = nullptr;
};
hipError_t launch_proj(const ProjLaunch& L, hipStream_t st);
// Principal coordinates z = V^T (x - mu) (k of them, L.k <= 64) and their
// bins against the coordinate edges (qfca_coords.hip): L.bins [k][N], L.resid
// [k][N] (the coordinates) when set; L.V1 the GEMM1 operand table.
hipError_t launch_coords(const ProjLaunch& L, hipStream_t st);

// MFMA projection: padded channel count (0 if C > 512), number of 16-wide
// component tiles (0 if k is 0 or > 64), host builders of the operand
// tables, and the launcher.
int mfma_cmax(int C, int prec);
int mfma_kt(int k, int prec);
void mfma_tables_f32(const float* V, int C, int k, std::vector<float>& V1, std::vector<float>& V2);
void mfma_tables_bf16(const uint16_t* Vb, int C, int k, std::vector<uint16_t>& V1,
                      std::vector<uint16_t>& V2);
// The same tables padded to CM channels and KT 16-wide component tiles
// (CM >= C, 16 KT >= k; KT even in BF16).
void mfma_tables_f32_at(const float* V, int C, int k, int CM, int KT, std::vector<float>& V1,
                        std::vector<float>& V2);
void mfma_tables_bf16_at(const uint16_t* Vb, int C, int k, int CM, int KT, std::vector<uint16_t>& V1,
                         std::vector<uint16_t>& V2);
// Channel and component padding of the persistent batch kernel for (C, k):
// the smallest of its instantiated shapes (64, 1), (256, 2), (512, 4) (FP32)
// or (256, 2), (512, 4) (BF16) that holds C channels and k components;
// false if none does (C > 512 or k outside 1..64).
bool batch_combo(int C, int k, int prec, int* CM, int* KT);
hipError_t launch_proj_mfma(const ProjLaunch& L, const void* V1, const void* V2, hipStream_t st);

// Fit statistics.
hipError_t launch_mean(const float* X, int C, long N, double* mu, hipStream_t st);
hipError_t launch_cov(const float* X, int C, long N, const double* mu, double* cov,
                      hipStream_t st);
// Exact order statistics: for every channel c and every j < nr, out[c*nr+j] =
// the ranks[j]-th smallest (0-based) value of vals[c][0..N).
hipError_t launch_select(const float* vals, int C, long N, const long long* ranks_dev, int nr,
                         float* out, hipStream_t st);

// Host FP64 symmetric eigensolver: A [n][n] row-major (destroyed); evals
// descending; vecs [n][n] row-major with column j the j-th eigenvector.
int sym_eig(double* A, int n, double* evals, double* vecs);
// The same eigenvalues with only the k leading eigenvectors: vecs [n][k].
int sym_eig_top(double* A, int n, int k, double* evals, double* vecs);

}  // namespace qfca
