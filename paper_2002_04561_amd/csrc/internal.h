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
  int64_t spin_dev;  // polls of device memory a bounded wait makes before giving up
  int64_t spin_lds;  // polls of LDS a bounded wait makes before giving up
  int8_t sig[kMaxAlphabet * kMaxAlphabet];  // row-major sigma(q, s) over the real alphabet
};

// Traceback slabs of the one-pair-per-lane kernels hold every cell's code for the waves in flight; a batch
// of large pairs runs fewer waves rather than asking for more than this.
constexpr int64_t kTbSlabBudget = (int64_t)16 << 30;
// Codes of the pairs a traceback batch sends to the band wavefront are held in an arena of at most this.
constexpr int64_t kTbArenaBytes = (int64_t)16 << 30;
// ... namely every pair of at least kTbMinCells cells or longer than kTbLaneDim on a side.
constexpr int64_t kTbMinCells = (int64_t)1 << 18;
constexpr int64_t kTbLaneDim = 1024;

constexpr int64_t kSpinDevDefault = 1ll << 22;  // ~0.1-0.5 s of polling device memory
constexpr int64_t kSpinLdsDefault = 1ll << 26;  // ~1-2 s of polling LDS

// Device workspace layout for the batch path.
struct BatchPlan {
  int64_t n_pairs;
  int64_t max_n, max_m;
  int32_t strips;       // ceil(max_n / R)
  int32_t n_waves;      // persistent waves of the launch
  size_t rowbuf_bytes;  // per wave
  size_t letters_bytes; // per wave
  size_t dirs_bytes;    // per wave (traceback only)
  size_t total_bytes;
};

// Brackets the kernels enqueued in its lifetime with timing events when profiling is enabled.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t stream);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  int token_;
  hipStream_t stream_;
};

// One pair handled by the wavefront engine.  With `flip` set the problem is relaxed transposed:
// the rows are the subject (read from the subject array at q_off) and the columns the query (from
// the query array at s_off); n and m are then the subject and query lengths.  Scores are unchanged
// and optima are compared in the original (i, j) order.
struct WfPair {
  int64_t q_off, s_off;  // offsets of the row / column sequence in its concatenated array
  int32_t n, m;          // rows, columns as relaxed
  int32_t nb;            // bands of the pair
  int32_t out_idx;       // index of the pair's aln_result_t
  int32_t flip;          // 1: rows are the subject (score-only calls)
  int32_t pad_;
  int64_t item0;         // global index of the pair's first band
  int64_t row_off;       // offset (int2 units) of the pair's two bottom-row slots, 2 * (m + 1)
  int64_t code_off;      // traceback: offset (uint16 units) of the pair's predecessor codes
};

// Device views of the wavefront engine's workspace.
struct WfWs {
  WfPair* pairs;     // [n_pairs], item0 ascending
  int2* rows;        // row slots of all pairs
  int* flags;        // [n_items] columns of each band's bottom row published so far
  int* item_pair;    // [n_items] index in `pairs` of each band's pair
  int4* band_res;    // [n_items] (score, i, j, flags) optimum of each band
  int64_t* ticket;   // item dispenser
  int64_t* n_items;  // total bands (device value, written by the planner)
  int* n_pairs;      // pairs in the table (device value)
  int* error;        // set when a bounded wait gives up
  uint16_t* codes;   // traceback: [band][lane][column] codes of 4 rows (4 bits each)
  int2* ckcols;      // checkpointed forward pass (one pair), else null: [k][row - 1] Hb and Fb of column
                     // (k + 1) * kTileCols; its row slots hold every group's bottom row
  int64_t ck_ld;     // rows of a checkpoint column (a multiple of the band height)
  int one_pair;      // aln_align_long: one pair, its bands spread over the whole device
  int64_t* order;    // [n_items] per-band engine: the item handed out at each ticket (see wf_order_kernel)
  int* lv;           // [2 * n_lv - 1] per-band engine: level counts, positions and cursors of that order
  int n_lv;          // more than the largest band count of any pair
};

struct WfOffsets {
  size_t pairs, rows, flags, item_pair, res, misc, codes, order, lv;
  int64_t n_lv;
};

struct LongPlan {
  int64_t nb;
  int n_waves;
  bool tb;
  WfOffsets off;
  size_t total_bytes;
};

constexpr int kWfR = 4;             // rows per lane in the wavefront engine
constexpr int kWfBand = 64 * kWfR;  // rows per band
constexpr int kTileCols = 2048;     // linear-space traceback: columns of a recomputed tile (a power of 2)
constexpr int kTileRows = 4 * kWfBand;  // rows of a recomputed tile: one workgroup's 4 bands

aln_status_t make_params(const aln_scoring_t* sc, KParams* kp);
int device_cu_count();

// batch_i32.hip
aln_status_t plan_batch_i32(const KParams& kp, int64_t n_pairs, int64_t max_n, int64_t max_m, bool traceback,
                            BatchPlan* plan);
aln_status_t launch_batch_i32(const KParams& kp, const BatchPlan& plan, const uint8_t* q, const int64_t* q_off,
                              const uint8_t* s, const int64_t* s_off, bool traceback, aln_result_t* out,
                              uint32_t* cigar, const int64_t* cigar_off, void* ws, const int* idx,
                              const int* idx_count, uint32_t extra_flags, int* ticket, hipStream_t stream,
                              const aln_result_t* fwd = nullptr);

// batch_i16.hip
struct BatchPlan16 {
  int64_t n_pairs, max_n, max_m;
  int R;
  int n_waves;
  size_t rowbuf_bytes, letters_bytes, slab_bytes, total_bytes;
};
struct I16Args {
  const uint8_t* q;
  const int64_t* q_off;
  const uint8_t* s;
  const int64_t* s_off;
  aln_result_t* out;
  uint32_t* cigar;
  const int64_t* cigar_off;
  void* ws;
  const int* idx;
  const int* idx_count;
  int* redo_idx;
  int* redo_cnt;
  int* ticket;  // group dispenser, zero before the launch
};
aln_status_t plan_batch_i16(const KParams& kp, int64_t n_pairs, int64_t max_n, int64_t max_m, bool tb,
                            BatchPlan16* plan);
aln_status_t launch_batch_i16(const KParams& kp, const BatchPlan16& plan, const I16Args& args, bool tb,
                              hipStream_t stream);

// wf_i32.hip
constexpr int kWfWavesPerCUDefault = 16;
constexpr int kWfGroupBands = 4;  // bands (compute waves) of a workgroup of the grouped wavefront engine
constexpr int kWfWavesPerCUMax = 32;
int wf_waves(int per_cu);
size_t wf_layout(int64_t max_pairs, int64_t max_items, int64_t row_words, int64_t code_words, WfOffsets* o);
WfWs wf_view(void* base, const WfOffsets& o);
// grouped: workgroups of 4 consecutive bands with LDS hand-offs and a courier wave for HBM
// p16: grouped score-only local bands over alphabets of up to 4 letters may use packed 16-bit cells
// where the scoring's step bound keeps them exact
// cigar_off: batches, each pair's CIGAR room (cigar[cigar_off[k] .. cigar_off[k + 1]]); else one pair with
// cigar_cap words at cigar
aln_status_t launch_wf_i32(const KParams& kp, const WfWs& W, const uint8_t* q, const uint8_t* s, aln_result_t* out,
                           int max_waves, bool grouped, bool tb, bool p16, uint32_t* cigar, int64_t cigar_cap,
                           hipStream_t stream, const int64_t* cigar_off = nullptr);
aln_status_t plan_long(int64_t n, int64_t m, bool tb, LongPlan* plan);
void launch_single_pair(const WfWs& W, int n, int m, hipStream_t stream);

// tb_tiles.hip: linear-space traceback of one pair (checkpointed forward pass, tiles relaxed again)
struct LongLsPlan {
  int64_t nb;        // bands of the forward pass
  int n_waves;       // its waves
  WfOffsets off;     // its workspace (row slots: one per group of 4 bands)
  int64_t ck_ld;     // rows of a checkpoint column
  int strips;        // tiles across the columns
  int64_t seg_rows;  // rows of a segment
  int nseg;          // segments
  size_t off_ckcols, off_codes, off_walk, total_bytes;
};
constexpr int64_t kLsCodeBudget = (int64_t)4 << 30;  // codes of one segment
aln_status_t plan_long_ls(int64_t n, int64_t m, int64_t code_budget, LongLsPlan* plan);
aln_status_t launch_long_ls(const KParams& kp, const LongLsPlan& plan, const uint8_t* q, int64_t n, const uint8_t* s,
                            int64_t m, aln_result_t* out, uint32_t* cigar, int64_t cigar_cap, void* ws,
                            hipStream_t stream);
aln_status_t launch_long(const KParams& kp, const LongPlan& plan, const uint8_t* q, int64_t n, const uint8_t* s,
                         int64_t m, aln_result_t* out, uint32_t* cigar, int64_t cigar_cap, void* ws,
                         hipStream_t stream);

// batch_plan.hip
struct SplitPlan {
  int64_t big_cells;  // pairs with n*m >= big_cells go to the wavefront engine
  int orient;         // wavefront pair orientation: 1 longer sequence along the rows, 0 as given, 2 cheaper
  int64_t item_cap, row_cap;  // bands and row-slot entries the workspace holds
  bool grouped;               // the wavefront engine runs workgroups of 4 consecutive bands
  bool wf_p16;                // grouped score-only local bands may use packed 16-bit cells
  bool tb;                    // a traceback call
  int64_t lane_dim;           // traceback calls: pairs longer than this on a side go to the wavefront
  int64_t code_cap;           // traceback calls: 16-bit code words the wavefront's arena holds (0: none)
  bool code_exact;            // the arena holds the codes of every pair that goes to the wavefront
  WfOffsets wf;
  size_t off_small_idx, off_small_cnt, off_keys, off_hist, off_code_off, off_code_used, wf_base, total_bytes;
  int wf_waves;
};
// Resolved execution choices of a batch call (defaults filled in).
struct BatchCfg {
  int64_t wf_min_cells;  // 0: by the batch's size (plan_split)
  int wf_group;  // 0: by the batch's size, 1: bands on their own, 4: groups of 4 bands
  int wf_waves_per_cu;
  bool waves_given;  // wf_waves_per_cu came from the caller
  int orient;  // 1 longer along the rows, 0 as given, 2 the cheaper of the two
  bool small16;
  bool wf_p16;  // packed 16-bit wavefront bands where exact
  int64_t tb_arena;  // most bytes of a traceback call's code arena (aln_set_batch_code_arena)
};
// Process-wide bound on a traceback batch's code arena (default kTbArenaBytes).
extern int64_t g_tb_arena_bytes;
BatchCfg resolve_cfg(const aln_batch_config_t* c);
// The planner's routing rule: a pair runs on the band wavefront when n*m >= *min_cells or n or m >
// *lane_dim (INT64_MAX: no such bound); cus = the device's compute units.
void route_rule(int64_t n_pairs, bool tb, const BatchCfg& cfg, int cus, int64_t* min_cells, int64_t* lane_dim);
aln_status_t plan_split(int64_t n_pairs, int64_t total_q, int64_t total_s, bool tb, int64_t max_n, int64_t max_m,
                        const BatchCfg& cfg, SplitPlan* sp);
void launch_split(const SplitPlan& sp, int64_t n_pairs, const int64_t* q_off, const int64_t* s_off, int64_t max_n,
                  int64_t max_m, aln_result_t* out, void* ws, hipStream_t stream);

}  // namespace mialign
