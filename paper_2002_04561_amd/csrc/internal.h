// Internal declarations shared by the mialign HIP sources (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mialign.h"

namespace mialign {

constexpr int kMaxAlphabet = 32;
constexpr int kPad = 32;        // code used for positions past the end of a sequence or invalid codes
constexpr int kTab = 33;        // substitution table side: 32 letters + pad
constexpr int32_t kNeg32 = -(1 << 30);  // stands for -infinity in 32-bit lanes
constexpr int32_t kBig32 = (1 << 29);   // |sigma| of the pad letter; exact scores stay below this

// Scoring constants handed to every kernel by value.
struct KParams {
  int32_t mode;
  int32_t alphabet;
  int32_t go;     // gap open (<= 0)
  int32_t ge;     // gap extend (< 0)
  int32_t goe;    // go + ge
  int32_t match;
  int32_t mismatch;
  int32_t use_table;
  int32_t sigma_max;
  int32_t sigma_min;
  int8_t sig[kMaxAlphabet * kMaxAlphabet];  // row-major sigma(q, s) over the real alphabet
};

// Device workspace layout for the batch path.
struct BatchPlan {
  int64_t n_pairs;
  int64_t max_n, max_m;
  int32_t strips;       // ceil(max_n / R)
  int32_t n_waves;      // persistent waves of the launch
  size_t rowbuf_bytes;  // per wave
  size_t dirs_bytes;    // per wave (traceback only)
  size_t total_bytes;
};

aln_status_t make_params(const aln_scoring_t* sc, KParams* kp);
int device_cu_count();

// batch_i32.hip
aln_status_t plan_batch_i32(const KParams& kp, int64_t n_pairs, int64_t max_n, int64_t max_m, bool traceback,
                            BatchPlan* plan);
aln_status_t launch_batch_i32(const KParams& kp, const BatchPlan& plan, const uint8_t* q, const int64_t* q_off,
                              const uint8_t* s, const int64_t* s_off, bool traceback, aln_result_t* out,
                              uint32_t* cigar, const int64_t* cigar_off, void* ws, hipStream_t stream);

}  // namespace mialign
