// Allocation-free variant of qfca_score_map, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  Its only scratch, the two fixed-point
// channel-sum maps, lives in a file-scope device array of fixed size that
// every GPU the library runs on holds until the process ends.
#include <mutex>

#include "qfca_internal.h"

namespace qfca {
namespace {

// Largest map the variant accepts (H * W pixels): 2048 x 2048.
constexpr size_t NOALLOC_MAX_PIXELS = (size_t)1 << 22;

// [0, MAX): channel sum of A_c; [MAX, 2 MAX): channel sum of W1_c.  64 MiB.
// In host code this name is a stand-in, not a device address: kernels and
// copies get the per-device address resolved by noalloc_init.
static __device__ __align__(256) long long scratch[2 * NOALLOC_MAX_PIXELS];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
long long* g_ptr[MAX_DEVICES] = {};

}  // namespace

hipError_t noalloc_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = (long long*)p;
    return hipSuccess;
}

}  // namespace qfca

using namespace qfca;

extern "C" qfca_status qfca_score_map_noalloc(qfca_ctx ctx, qfca_model m, const uint8_t* bins, int32_t H,
                                              int32_t W, float* score, float* amap, float* w1, float* achan) {
    qfca_status st = score_map_check(ctx, m, bins, H, W, score);
    if (st != QFCA_OK) return st;
    if ((size_t)H * (size_t)W > NOALLOC_MAX_PIXELS)
        return status_fail(QFCA_E_UNSUPPORTED, "qfca_score_map_noalloc: H * W exceeds 4194304 pixels");
    const int dev = ctx_device(ctx);
    long long* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = (dev >= 0 && dev < MAX_DEVICES) ? g_ptr[dev] : nullptr;
    }
    if (!base) return status_fail(QFCA_E_STATE, "qfca_score_map_noalloc: scratch not resolved for this device");
    // the second half carries the W1 channel sum (or, for a principal-
    // coordinate model, the box-mean map when amap is NULL)
    return score_map_into(ctx, m, bins, H, W, score, amap, w1, achan, base, base + NOALLOC_MAX_PIXELS);
}
