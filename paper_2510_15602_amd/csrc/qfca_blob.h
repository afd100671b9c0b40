// Host-only part of the model lifecycle: parameter and array checks and the
// serialised model format (internal header of libqfca).  Plain C++ with no
// device code, so that the CPU tests can build it on its own under the
// address and undefined-behaviour sanitizers.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/qfca.h"

namespace qfca {

// Histogrammed planes of a model: the C channels (PRE_NONE, PRE_RESIDUAL) or
// the k principal coordinates (PRE_COORDS).
inline int blob_planes(const qfca_params& p) { return p.preproc == QFCA_PRE_COORDS ? p.k : p.C; }

// Parameter ranges of the library (QFCA_OK, or a status with *err set).
qfca_status host_check_params(const qfca_params* p, std::string* err);

// The arrays a model is built from: delta [P] finite and >= 0, edges [P][B-1]
// nondecreasing per plane, and (when given) the integer reference cR [P][B]
// nondecreasing, >= 0, ending at T*T.  P = blob_planes(p).
qfca_status host_check_arrays(const qfca_params& p, const float* edges, const double* delta, const int32_t* cR,
                              std::string* err);

// General reference weights cRw [P][B]: finite, >= 0, nondecreasing per plane.
qfca_status host_check_weights(const qfca_params& p, const double* cRw, std::string* err);

// A serialised model: an 8-byte magic, u32 version, u32 flags (bit 0 integer
// reference, bit 1 eigenvalues, bit 2 lo/hi, bit 3 general reference), the
// parameters (C k B T as int32, q_lo q_hi sigma_s as float32, preproc
// proj_prec as int32, then in version 2 sigma_p as float32 and reference as
// int32), then mu [C] f64, V [C][k] f64 (PCA models only), edges [P][B-1]
// f32, delta [P] f64, and, by flag, cR [P][B] i32, eigenvalues [C] f64, lo
// [P] f64, hi [P] f64 and the general reference weights [P][B] f64.  Host
// byte order.  Version 1 (no sigma_p, reference) is read with sigma_p =
// INFINITY and the median -> quan reference.
constexpr uint32_t kModelVersion = 2;

struct ModelArrays {
    qfca_params p{};
    uint32_t flags = 0;
    std::vector<double> mu, V, delta, evals, lo, hi, cRw;
    std::vector<float> edges;
    std::vector<int32_t> cR;
};

// Bytes of the current version's blob of a model with these parameters and
// flags.
size_t blob_bytes(const qfca_params& p, uint32_t flags);

// Writes m (its arrays sized as its parameters and flags say) into d, which
// holds blob_bytes(m.p, m.flags) bytes.
void blob_write(const ModelArrays& m, unsigned char* d);

// Reads and checks a blob of `bytes` bytes (every size, range and array rule
// above); QFCA_OK fills *out.
qfca_status blob_read(const void* buf, size_t bytes, ModelArrays* out, std::string* err);

}  // namespace qfca
