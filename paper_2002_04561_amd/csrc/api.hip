// C-ABI entry points of mialign: argument validation, workspace sizing and dispatch.
#include <cstring>
#include <mutex>

#include "internal.h"

namespace mialign {

int device_cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  return cus;
}

// Poll counts of the bounded device-side waits (aln_set_wait_limits); process-wide.
static int64_t g_spin_dev = kSpinDevDefault;
static int64_t g_spin_lds = kSpinLdsDefault;

aln_status_t make_params(const aln_scoring_t* sc, KParams* kp) {
  if (!sc || !kp) return ALN_E_INVALID;
  if (sc->mode < ALN_GLOBAL || sc->mode > ALN_SEMIGLOBAL) return ALN_E_INVALID;
  if (sc->alphabet_size < 2 || sc->alphabet_size > kMaxAlphabet) return ALN_E_ALPHABET;
  if (sc->gap_open > 0 || sc->gap_extend >= 0) return ALN_E_SCORING;
  if (sc->gap_open < -(1 << 16) || sc->gap_extend < -(1 << 16)) return ALN_E_SCORING;
  std::memset(kp, 0, sizeof(*kp));
  kp->mode = sc->mode;
  kp->alphabet = sc->alphabet_size;
  kp->go = sc->gap_open;
  kp->ge = sc->gap_extend;
  kp->goe = sc->gap_open + sc->gap_extend;
  kp->spin_dev = g_spin_dev;
  kp->spin_lds = g_spin_lds;
  const int A = sc->alphabet_size;
  int smax = -1000, smin = 1000;
  if (sc->subst) {
    kp->use_table = 1;
    for (int a = 0; a < A; ++a)
      for (int b = 0; b < A; ++b) {
        const int v = sc->subst[a * A + b];
        kp->sig[a * kMaxAlphabet + b] = (int8_t)v;
        smax = v > smax ? v : smax;
        smin = v < smin ? v : smin;
      }
    kp->match = 0;
    kp->mismatch = 0;
  } else {
    if (sc->match > 127 || sc->match < -127 || sc->mismatch > 127 || sc->mismatch < -127) return ALN_E_SCORING;
    kp->use_table = 0;
    kp->match = sc->match;
    kp->mismatch = sc->mismatch;
    for (int a = 0; a < A; ++a)
      for (int b = 0; b < A; ++b) kp->sig[a * kMaxAlphabet + b] = (int8_t)(a == b ? sc->match : sc->mismatch);
    smax = sc->match > sc->mismatch ? sc->match : sc->mismatch;
    smin = sc->match < sc->mismatch ? sc->match : sc->mismatch;
  }
  kp->sigma_max = smax;
  kp->sigma_min = smin;
  return ALN_OK;
}

// Every exact score of an n x m problem lies in [3*go + (n+m)*ge, min(n,m)*max(sigma_max, 0)];
// the 32-bit lanes need both ends well inside +-2^29 (the pad letter scores -2^29).
// The wavefront engine also adds a row bias of up to rows*|ge| to every value, and relaxes a pair
// transposed when that puts the longer sequence along the rows.
static bool fits_i32(const KParams& kp, int64_t max_n, int64_t max_m) {
  const int64_t mn = max_n < max_m ? max_n : max_m;
  const int64_t mx = max_n < max_m ? max_m : max_n;
  const int64_t up = mn * (kp.sigma_max > 0 ? kp.sigma_max : 0) - mx * (int64_t)kp.ge;
  const int64_t lo = 3 * (int64_t)kp.go + (max_n + max_m) * (int64_t)kp.ge;
  const int64_t lim = (int64_t)1 << 28;
  return up < lim && -lo < lim;
}

}  // namespace mialign

using namespace mialign;

extern "C" {

const char* aln_version(void) { return "mialign 0.2 (gfx950)"; }

aln_status_t aln_set_wait_limits(int64_t device_polls, int64_t lds_polls) {
  if (device_polls < 0 || lds_polls < 0) return ALN_E_INVALID;
  g_spin_dev = device_polls ? device_polls : kSpinDevDefault;
  g_spin_lds = lds_polls ? lds_polls : kSpinLdsDefault;
  return ALN_OK;
}

const char* aln_status_string(aln_status_t st) {
  switch (st) {
    case ALN_OK:
      return "ok";
    case ALN_E_INVALID:
      return "invalid argument";
    case ALN_E_ALPHABET:
      return "alphabet_size must be in 2..32";
    case ALN_E_SCORING:
      return "invalid scoring (gap_open > 0, gap_extend >= 0, or scores too large for exact integer lanes)";
    case ALN_E_WORKSPACE:
      return "workspace too small";
    case ALN_E_DEVICE:
      return "HIP device error";
    case ALN_E_UNSUPPORTED:
      return "unsupported combination";
    default:
      return "unknown status";
  }
}

__global__ void fill_i32_kernel(int* p, int n, int v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// Workspace of a batch call:
//   [slabs: shared by the 16-bit kernel and the 32-bit kernel, which run one after the other]
//   [redo list: n_pairs ints + counter]
//   [split plan + wavefront engine, with a code arena for traceback calls]
struct BatchLayout {
  BatchPlan bp;
  BatchPlan16 bp16;
  SplitPlan sp;
  bool use16;
  size_t off_redo, off_redo_cnt, off_split, total;
};

static aln_status_t batch_layout(const KParams& kp, int64_t n_pairs, int64_t max_n, int64_t max_m, int64_t total_q,
                                 int64_t total_s, uint32_t flags, const BatchCfg& cfg, BatchLayout* L) {
  const bool tb = (flags & ALN_TRACEBACK) != 0;
  aln_status_t st = plan_split(n_pairs, total_q, total_s, tb, max_n, max_m, cfg, &L->sp);
  if (st != ALN_OK) return st;
  // The one-pair-per-lane kernels of a traceback call meet pairs up to kTbLaneDim on each side when the
  // wavefront's code arena takes every longer pair; their slabs are sized for that.
  const bool lanes_bounded = tb && L->sp.code_exact;
  const int64_t lane_n = lanes_bounded ? std::min(max_n, kTbLaneDim) : max_n;
  const int64_t lane_m = lanes_bounded ? std::min(max_m, kTbLaneDim) : max_m;
  st = plan_batch_i32(kp, n_pairs, lane_n, lane_m, tb, &L->bp);
  if (st != ALN_OK) return st;
  L->use16 = !(flags & ALN_FORCE_INT32) && cfg.small16 && lane_m < 32767;
  size_t slabs = L->bp.total_bytes;
  if (L->use16) {
    st = plan_batch_i16(kp, n_pairs, lane_n, lane_m, tb, &L->bp16);
    if (st != ALN_OK) return st;
    if (L->bp16.total_bytes > slabs) slabs = L->bp16.total_bytes;
  }
  size_t off = (slabs + 255) & ~(size_t)255;
  L->off_redo = off;
  off += ((size_t)(n_pairs + 1) * sizeof(int) + 255) & ~(size_t)255;
  L->off_redo_cnt = off;
  off += 256;
  L->off_split = off;
  off += L->sp.total_bytes;
  L->total = off;
  return ALN_OK;
}

aln_status_t aln_batch_workspace_size(const aln_scoring_t* scoring, int64_t n_pairs, int64_t max_n, int64_t max_m,
                                      int64_t total_q, int64_t total_s, uint32_t flags, size_t* bytes) {
  if (!bytes || n_pairs < 0 || max_n < 0 || max_m < 0 || total_q < 0 || total_s < 0) return ALN_E_INVALID;
  if (flags & ~(ALN_TRACEBACK | ALN_FORCE_INT32 | ALN_FORCE_INT16)) return ALN_E_INVALID;
  KParams kp;
  aln_status_t st = make_params(scoring, &kp);
  if (st != ALN_OK) return st;
  if (!fits_i32(kp, max_n, max_m)) return ALN_E_SCORING;
  // the slab sizes do not depend on the config; the 16-bit slabs are sized whenever they may be used
  BatchLayout L;
  st = batch_layout(kp, n_pairs, max_n, max_m, total_q, total_s, flags, resolve_cfg(nullptr), &L);
  if (st != ALN_OK) return st;
  *bytes = L.total;
  return ALN_OK;
}

static bool cfg_valid(const aln_batch_config_t* c) {
  if (!c) return true;
  if (c->wf_waves_per_cu < 0 || c->wf_waves_per_cu > kWfWavesPerCUMax) return false;
  if (c->wf_orient < -1 || c->wf_orient > 2) return false;
  if (c->small_bits != 0 && c->small_bits != 16 && c->small_bits != 32) return false;
  if (c->wf_group != 0 && c->wf_group != 1 && c->wf_group != 4) return false;
  if (c->wf_bits != 0 && c->wf_bits != 16 && c->wf_bits != 32) return false;
  if (c->reserved != 0) return false;
  return true;
}

aln_status_t aln_batch_route(int64_t n_pairs, uint32_t flags, const aln_batch_config_t* config, int64_t* min_cells,
                             int64_t* max_side) {
  if (!min_cells || !max_side || n_pairs < 0) return ALN_E_INVALID;
  if (flags & ~(ALN_TRACEBACK | ALN_FORCE_INT32 | ALN_FORCE_INT16)) return ALN_E_INVALID;
  if (!cfg_valid(config)) return ALN_E_INVALID;
  const int cus = device_cu_count();
  if (cus <= 0) return ALN_E_DEVICE;
  route_rule(n_pairs, (flags & ALN_TRACEBACK) != 0, resolve_cfg(config), cus, min_cells, max_side);
  return ALN_OK;
}

aln_status_t aln_align_batch(const aln_scoring_t* scoring, int64_t n_pairs, const uint8_t* q, const int64_t* q_off,
                             const uint8_t* s, const int64_t* s_off, int64_t max_n, int64_t max_m, int64_t total_q,
                             int64_t total_s, uint32_t flags, aln_result_t* out, uint32_t* cigar,
                             const int64_t* cigar_off, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  return aln_align_batch_ex(scoring, n_pairs, q, q_off, s, s_off, max_n, max_m, total_q, total_s, flags, nullptr,
                            out, cigar, cigar_off, workspace, workspace_bytes, stream);
}

aln_status_t aln_align_batch_ex(const aln_scoring_t* scoring, int64_t n_pairs, const uint8_t* q,
                                const int64_t* q_off, const uint8_t* s, const int64_t* s_off, int64_t max_n,
                                int64_t max_m, int64_t total_q, int64_t total_s, uint32_t flags,
                                const aln_batch_config_t* config, aln_result_t* out, uint32_t* cigar,
                                const int64_t* cigar_off, void* workspace, size_t workspace_bytes,
                                hipStream_t stream) {
  if (n_pairs < 0 || max_n < 0 || max_m < 0 || total_q < 0 || total_s < 0) return ALN_E_INVALID;
  if (flags & ~(ALN_TRACEBACK | ALN_FORCE_INT32 | ALN_FORCE_INT16)) return ALN_E_INVALID;
  if (!cfg_valid(config)) return ALN_E_INVALID;
  const BatchCfg cfg = resolve_cfg(config);
  KParams kp;
  aln_status_t st = make_params(scoring, &kp);
  if (st != ALN_OK) return st;
  if (n_pairs == 0) return ALN_OK;
  if (!q_off || !s_off || !out) return ALN_E_INVALID;
  if ((!q && max_n > 0) || (!s && max_m > 0)) return ALN_E_INVALID;
  if (n_pairs >= (1ll << 31)) return ALN_E_INVALID;
  const bool tb = (flags & ALN_TRACEBACK) != 0;
  if (tb && (!cigar || !cigar_off)) return ALN_E_INVALID;
  if (!fits_i32(kp, max_n, max_m)) return ALN_E_SCORING;
  BatchLayout L;
  st = batch_layout(kp, n_pairs, max_n, max_m, total_q, total_s, flags, cfg, &L);
  if (st != ALN_OK) return st;
  if (!workspace || workspace_bytes < L.total) return ALN_E_WORKSPACE;
  char* base = static_cast<char*>(workspace);
  int* redo_idx = reinterpret_cast<int*>(base + L.off_redo);
  int* redo_cnt = reinterpret_cast<int*>(base + L.off_redo_cnt);

  // The inter-sequence kernels see a shape-sorted list of the small pairs; the large ones go to the
  // wavefront engine (in a traceback call, those whose codes found room in its arena).
  char* split_ws = base + L.off_split;
  launch_split(L.sp, n_pairs, q_off, s_off, max_n, max_m, out, split_ws, stream);
  if (!tb || L.sp.code_cap > 0) {
    WfWs W = wf_view(split_ws + L.sp.wf_base, L.sp.wf);
    st = launch_wf_i32(kp, W, q, s, out, L.sp.wf_waves, L.sp.grouped, tb, !tb && L.sp.wf_p16, cigar, 0, stream,
                       tb ? cigar_off : nullptr);
    if (st != ALN_OK) return st;
  }
  const int* list = reinterpret_cast<const int*>(split_ws + L.sp.off_small_idx);
  const int* list_cnt = reinterpret_cast<const int*>(split_ws + L.sp.off_small_cnt);
  // the redo counter and the group tickets of the 16- and 32-bit launches start at zero
  int* ticket16 = redo_cnt + 16;
  int* ticket32 = redo_cnt + 32;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, stream, redo_cnt, 48, 0);
  if (!L.use16)
    return launch_batch_i32(kp, L.bp, q, q_off, s, s_off, tb, out, cigar, cigar_off, workspace, list, list_cnt, 0u,
                            ticket32, stream);
  I16Args a;
  a.q = q;
  a.q_off = q_off;
  a.s = s;
  a.s_off = s_off;
  a.out = out;
  a.cigar = cigar;
  a.cigar_off = cigar_off;
  a.ws = workspace;
  a.idx = list;
  a.idx_count = list_cnt;
  a.redo_idx = redo_idx;
  a.redo_cnt = redo_cnt;
  a.ticket = ticket16;
  st = launch_batch_i16(kp, L.bp16, a, tb, stream);
  if (st != ALN_OK) return st;
  // pairs whose 16-bit range was not provably exact, or that saturated, are recomputed in 32 bits
  return launch_batch_i32(kp, L.bp, q, q_off, s, s_off, tb, out, cigar, cigar_off, workspace, redo_idx, redo_cnt,
                          ALN_RES_INT32_REDO, ticket32, stream);
}

// Device scratch of aln_align_batch_noalloc: the workspace of calls that cannot allocate.  Each device the
// library runs on holds its own copy for the life of the process.  In host code `scratch` names a host-side
// stand-in, never the device memory: the device address is taken once per device with hipGetSymbolAddress
// and kept in g_scratch_ptr, and only that address is handed to kernels.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static aln_status_t scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ALN_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ALN_E_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ALN_OK;
}

aln_status_t aln_align_batch_noalloc(const aln_scoring_t* scoring, int64_t n_pairs, const uint8_t* q,
                                     const int64_t* q_off, const uint8_t* s, const int64_t* s_off, int64_t max_n,
                                     int64_t max_m, int64_t total_q, int64_t total_s, uint32_t flags,
                                     const aln_batch_config_t* config, aln_result_t* out, uint32_t* cigar,
                                     const int64_t* cigar_off, hipStream_t stream) {
  size_t need = 0;
  aln_status_t st = aln_batch_workspace_size(scoring, n_pairs, max_n, max_m, total_q, total_s, flags, &need);
  if (st != ALN_OK) return st;
  if (need > kScratchBytes) return ALN_E_WORKSPACE;
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st != ALN_OK) return st;
  // the batch path clears every counter and ticket it uses with small kernels, so the scratch's
  // contents from an earlier call do not matter
  return aln_align_batch_ex(scoring, n_pairs, q, q_off, s, s_off, max_n, max_m, total_q, total_s, flags, config, out,
                            cigar, cigar_off, ws, kScratchBytes, stream);
}

size_t aln_noalloc_scratch_bytes(void) { return kScratchBytes; }

// aln_traceback: the 32-bit one-pair-per-lane slabs, then the group ticket.
static aln_status_t tb_layout(const KParams& kp, int64_t n_pairs, int64_t max_n, int64_t max_m, BatchPlan* bp,
                              size_t* off_ticket, size_t* total) {
  aln_status_t st = plan_batch_i32(kp, n_pairs, max_n, max_m, true, bp);
  if (st != ALN_OK) return st;
  *off_ticket = (bp->total_bytes + 255) & ~(size_t)255;
  *total = *off_ticket + 256;
  return ALN_OK;
}

aln_status_t aln_traceback_workspace_size(const aln_scoring_t* scoring, int64_t n_pairs, int64_t max_n,
                                          int64_t max_m, size_t* bytes) {
  if (!bytes || n_pairs < 0 || max_n < 0 || max_m < 0) return ALN_E_INVALID;
  KParams kp;
  aln_status_t st = make_params(scoring, &kp);
  if (st != ALN_OK) return st;
  if (!fits_i32(kp, max_n, max_m)) return ALN_E_SCORING;
  BatchPlan bp;
  size_t off_ticket = 0;
  st = tb_layout(kp, n_pairs, max_n, max_m, &bp, &off_ticket, bytes);
  return st;
}

aln_status_t aln_traceback(const aln_scoring_t* scoring, int64_t n_pairs, const uint8_t* q, const int64_t* q_off,
                           const uint8_t* s, const int64_t* s_off, int64_t max_n, int64_t max_m,
                           const aln_result_t* fwd, aln_result_t* out, uint32_t* cigar, const int64_t* cigar_off,
                           void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (n_pairs < 0 || max_n < 0 || max_m < 0) return ALN_E_INVALID;
  KParams kp;
  aln_status_t st = make_params(scoring, &kp);
  if (st != ALN_OK) return st;
  if (n_pairs == 0) return ALN_OK;
  if (!q_off || !s_off || !fwd || !out || !cigar || !cigar_off) return ALN_E_INVALID;
  if ((!q && max_n > 0) || (!s && max_m > 0)) return ALN_E_INVALID;
  if (n_pairs >= (1ll << 31)) return ALN_E_INVALID;
  if (!fits_i32(kp, max_n, max_m)) return ALN_E_SCORING;
  BatchPlan bp;
  size_t off_ticket = 0, total = 0;
  st = tb_layout(kp, n_pairs, max_n, max_m, &bp, &off_ticket, &total);
  if (st != ALN_OK) return st;
  if (!workspace || workspace_bytes < total) return ALN_E_WORKSPACE;
  int* ticket = reinterpret_cast<int*>(static_cast<char*>(workspace) + off_ticket);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, stream, ticket, 1, 0);
  return launch_batch_i32(kp, bp, q, q_off, s, s_off, true, out, cigar, cigar_off, workspace, nullptr, nullptr, 0u,
                          ticket, stream, fwd);
}

aln_status_t aln_cigar_to_gapped(const uint8_t* q, int64_t n, const uint8_t* s, int64_t m,
                                 const aln_result_t* result, const uint32_t* cigar, const char* letters,
                                 char* q_aln, char* s_aln, int64_t capacity) {
  if ((!q && n > 0) || (!s && m > 0) || !result || !q_aln || !s_aln || capacity < 1 || n < 0 || m < 0)
    return ALN_E_INVALID;
  if (result->cigar_len < 0 || (result->cigar_len > 0 && !cigar)) return ALN_E_INVALID;
  int64_t i = result->q_begin, j = result->s_begin, len = 0;
  if (i < 0 || j < 0 || i > n || j > m) return ALN_E_INVALID;
  const int64_t nl = letters ? (int64_t)std::strlen(letters) : 26;
  auto letter = [&](uint8_t c) -> char {
    if (c >= nl) return '?';
    return letters ? letters[c] : (char)('A' + c);
  };
  for (int32_t k = 0; k < result->cigar_len; ++k) {
    const uint32_t op = cigar[k] & 15u, run = cigar[k] >> 4;
    if (op > ALN_CIGAR_D) return ALN_E_INVALID;
    if (len + (int64_t)run + 1 > capacity) return ALN_E_INVALID;
    if ((op != ALN_CIGAR_D && i + run > n) || (op != ALN_CIGAR_I && j + run > m)) return ALN_E_INVALID;
    for (uint32_t r = 0; r < run; ++r, ++len) {
      q_aln[len] = op == ALN_CIGAR_D ? '-' : letter(q[i++]);
      s_aln[len] = op == ALN_CIGAR_I ? '-' : letter(s[j++]);
    }
  }
  q_aln[len] = 0;
  s_aln[len] = 0;
  return ALN_OK;
}

// Traceback of one long pair stores 4 bits per cell for pairs of at most kLsAutoCells cells (or with
// ALN_STORED_CODES) while that fits under kMaxLongCodeBytes; otherwise (or with ALN_LINEAR_SPACE) the
// pair is traced back in linear space from checkpoints.
static const int64_t kMaxLongCodeBytes = (int64_t)64 << 30;

static const int64_t kLsAutoCells = (int64_t)1 << 24;

static bool long_linear_space(int64_t n, int64_t m, uint32_t flags) {
  if (!(flags & ALN_TRACEBACK)) return false;
  if (flags & ALN_LINEAR_SPACE) return true;
  // codes that would not fit; and above 2^24 cells the linear-space traceback is faster (the forward
  // pass writes no code per cell, and the tiles relax only a window around the path)
  return (n + kWfBand) / 2 * m > kMaxLongCodeBytes || (!(flags & ALN_STORED_CODES) && n * m > kLsAutoCells);
}

static const uint32_t kLongFlags =
    ALN_TRACEBACK | ALN_FORCE_INT32 | ALN_FORCE_INT16 | ALN_LINEAR_SPACE | ALN_STORED_CODES;

// Bytes of predecessor codes a linear-space traceback holds at once (aln_set_traceback_budget).
static int64_t g_ls_budget = kLsCodeBudget;

aln_status_t aln_set_batch_code_arena(int64_t bytes) {
  if (bytes < 0) return ALN_E_INVALID;
  g_tb_arena_bytes = bytes ? bytes : kTbArenaBytes;
  return ALN_OK;
}

aln_status_t aln_set_traceback_budget(int64_t bytes) {
  if (bytes < 0) return ALN_E_INVALID;
  g_ls_budget = bytes ? bytes : kLsCodeBudget;
  return ALN_OK;
}

aln_status_t aln_long_workspace_size(const aln_scoring_t* scoring, int64_t n, int64_t m, uint32_t flags,
                                     size_t* bytes) {
  if (!bytes || n < 0 || m < 0 || n >= (1ll << 31) || m >= (1ll << 31)) return ALN_E_INVALID;
  if (flags & ~kLongFlags) return ALN_E_INVALID;
  const bool tb = (flags & ALN_TRACEBACK) != 0;
  KParams kp;
  aln_status_t st = make_params(scoring, &kp);
  if (st != ALN_OK) return st;
  if (!fits_i32(kp, n, m)) return ALN_E_SCORING;
  if (long_linear_space(n, m, flags)) {
    LongLsPlan pl;
    st = plan_long_ls(n, m, g_ls_budget, &pl);
    if (st != ALN_OK) return st;
    *bytes = pl.total_bytes;
    return ALN_OK;
  }
  LongPlan pl;
  st = plan_long(n, m, tb, &pl);
  if (st != ALN_OK) return st;
  *bytes = pl.total_bytes;
  return ALN_OK;
}

aln_status_t aln_align_long(const aln_scoring_t* scoring, const uint8_t* q, int64_t n, const uint8_t* s, int64_t m,
                            uint32_t flags, aln_result_t* out, uint32_t* cigar, int64_t cigar_capacity,
                            void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (n < 0 || m < 0 || n >= (1ll << 31) || m >= (1ll << 31) || !out) return ALN_E_INVALID;
  if ((n > 0 && !q) || (m > 0 && !s)) return ALN_E_INVALID;
  if (flags & ~kLongFlags) return ALN_E_INVALID;
  const bool tb = (flags & ALN_TRACEBACK) != 0;
  if (tb && (!cigar || cigar_capacity < 0)) return ALN_E_INVALID;
  KParams kp;
  aln_status_t st = make_params(scoring, &kp);
  if (st != ALN_OK) return st;
  if (!fits_i32(kp, n, m)) return ALN_E_SCORING;
  if (long_linear_space(n, m, flags)) {
    LongLsPlan pl;
    st = plan_long_ls(n, m, g_ls_budget, &pl);
    if (st != ALN_OK) return st;
    if (!workspace || workspace_bytes < pl.total_bytes) return ALN_E_WORKSPACE;
    return launch_long_ls(kp, pl, q, n, s, m, out, cigar, cigar_capacity, workspace, stream);
  }
  LongPlan pl;
  st = plan_long(n, m, tb, &pl);
  if (st != ALN_OK) return st;
  if (!workspace || workspace_bytes < pl.total_bytes) return ALN_E_WORKSPACE;
  return launch_long(kp, pl, q, n, s, m, out, cigar, tb ? cigar_capacity : 0, workspace, stream);
}

}  // extern "C"
