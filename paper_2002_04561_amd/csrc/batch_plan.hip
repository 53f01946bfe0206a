// Device-side planning of a batch: routes each pair to the inter-sequence kernels (one pair per
// lane) or, when its matrix is large, to the intra-sequence wavefront engine (one band per wave),
// and orders both lists with one counting sort:
//   - inter-sequence pairs by shape, so that the 64 or 128 pairs sharing a wave have similar n and
//     m (a wave runs max n x max m steps for all of its pairs).  Shapes are binned on a log scale
//     with 8 bins per octave of n and of m, largest first, so long pairs start first;
//   - wavefront pairs by cell count, largest first (longest-processing-time order for the queue),
//     each oriented with its longer sequence along the band rows when the call allows it.
// Everything runs on the device: a batch needs no host copy of its lengths and stays capturable
// in a HIP graph.
#include "internal.h"

namespace mialign {
namespace {

constexpr int kShapeBins = 128;                 // per dimension
constexpr int kSmallKeys = kShapeBins * kShapeBins;
constexpr int kBigKeys = 1024;                  // cell-count bins of wavefront pairs
constexpr int kKeys = kSmallKeys + kBigKeys;    // sort keys; big pairs sort above every small one
constexpr int kScanThreads = 1024;
static_assert(kKeys % kScanThreads == 0, "keys per scan thread");

struct SplitView {
  int* small_idx;  // sorted inter-sequence list
  int* counters;   // [0] small pairs, [1] big pairs
  int* keys;       // per pair: sort key
  int* hist;       // [kKeys] counts, then cursors
  int64_t* code_off;                 // traceback calls: per pair, offset of its codes in the code arena
  unsigned long long* code_used;     // traceback calls: code words reserved so far
};

// 8 bins per octave: floor(8 * log2(x)) - 16 for x >= 8, x itself below.
__device__ __forceinline__ int log_bin_wide(int64_t x) {
  if (x < 8) return (int)(x < 0 ? 0 : x);
  const int e = 63 - __builtin_clzll((unsigned long long)x);
  const int frac = (int)((x >> (e - 3)) & 7);
  return e * 8 + frac - 16;  // x = 8 gives 8
}
__device__ __forceinline__ int log_bin(int64_t x) {
  const int b = log_bin_wide(x);
  return b < kShapeBins ? b : kShapeBins - 1;
}

// Wave-steps the band wavefront spends on a rows x cols problem: one band per 256 rows, each
// sweeping cols + 63 steps plus about 192 steps of start-up (ticket, pair lookup, profile) and of
// waiting for the band above to publish its first columns.
__device__ __forceinline__ int64_t band_steps(int64_t rows, int64_t cols) {
  return (rows + kWfBand - 1) / kWfBand * (cols + 63 + 192);
}

// Whether a wavefront pair runs transposed.  Row slots (2 (columns + 1) entries) are reserved from
// the subject total, so a pair of two or more bands may only be flipped to shorter columns; a
// one-band pair needs no slots.
__device__ __forceinline__ bool orient_flip(int64_t n, int64_t m, int orient) {
  if (orient == 1) return m > n;
  if (orient == 2) return band_steps(m, n) < band_steps(n, m) && (n <= m || m <= kWfBand);
  return false;
}

__global__ void split_reset_kernel(SplitView V) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < kKeys; k += gridDim.x * blockDim.x) V.hist[k] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 2) V.counters[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *V.code_used = 0;
}

// Blocks of the classify and scatter passes each own one contiguous chunk of pairs and count its
// keys in an LDS histogram first, so a batch whose pairs share a few shapes does not serialise on
// a few global counters.
constexpr int kPlanThreads = 1024;

__device__ __forceinline__ void chunk_of_block(int64_t n_pairs, int64_t* p0, int64_t* p1) {
  const int64_t per = (n_pairs + gridDim.x - 1) / gridDim.x;
  *p0 = (int64_t)blockIdx.x * per;
  *p1 = *p0 + per < n_pairs ? *p0 + per : n_pairs;
}

__global__ __launch_bounds__(kPlanThreads) void split_classify_kernel(int64_t n_pairs,
                                                                      const int64_t* __restrict__ q_off,
                                                                      const int64_t* __restrict__ s_off,
                                                                      int64_t max_n, int64_t max_m,
                                                                      int64_t big_cells, int64_t lane_dim, int orient,
                                                                      bool tb, int64_t code_cap, SplitView V) {
  __shared__ int h[kKeys];
  __shared__ int n_big;
  for (int k = threadIdx.x; k < kKeys; k += blockDim.x) h[k] = 0;
  if (threadIdx.x == 0) n_big = 0;
  __syncthreads();
  int64_t p0, p1;
  chunk_of_block(n_pairs, &p0, &p1);
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const int64_t n = q_off[p + 1] - q_off[p], m = s_off[p + 1] - s_off[p];
    const bool fits = n >= 0 && m >= 0 && n <= max_n && m <= max_m;
    int key;
    // (a traceback call's pair longer than lane_dim on a side goes to the wavefront even with the
    // other side empty: it then has no bands, and the finish pass gives its result)
    bool big = fits && ((n > 0 && m > 0 && n * m >= big_cells) || n > lane_dim || m > lane_dim);
    if (big && tb) {
      // a traceback call: the pair's 4-bit codes (one 16-bit word per band lane and column) must fit the
      // code arena; pairs are given room in the order they reserve it.  A pair that finds no room runs
      // one pair per lane instead, with the same result: the planner sizes the lanes' slabs for every
      // pair whenever the arena may fall short.
      const unsigned long long words = (unsigned long long)((n + kWfBand - 1) / kWfBand) * 64ull * (unsigned long long)m;
      const unsigned long long at = code_cap > 0 ? atomicAdd(V.code_used, words) : 0ull;
      big = code_cap > 0 && at + words <= (unsigned long long)code_cap;
      if (big) V.code_off[p] = (int64_t)at;
    }
    if (big) {
      // wavefront pairs by band work, bands x (columns + 63), largest first: a workgroup relaxes
      // kWfWavesPerBlock consecutive bands, which then take about the same time
      const bool flip = orient_flip(n, m, orient);
      const int64_t rows = flip ? m : n, cols = flip ? n : m;
      const int b = log_bin_wide((rows + kWfBand - 1) / kWfBand * (cols + 63));
      key = kSmallKeys + (b < kBigKeys ? b : kBigKeys - 1);
      atomicAdd(&n_big, 1);
    } else {
      key = log_bin(n) * kShapeBins + log_bin(m);
    }
    V.keys[p] = key;
    atomicAdd(&h[key], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kKeys; k += blockDim.x)
    if (h[k]) atomicAdd(&V.hist[k], h[k]);
  if (threadIdx.x == 0 && n_big) atomicAdd(&V.counters[1], n_big);
}

// One block: turns the key histogram into cursors, largest keys first, and counts the small list.
__global__ __launch_bounds__(kScanThreads) void sort_scan_kernel(SplitView V) {
  __shared__ int part[kScanThreads];
  constexpr int per = kKeys / kScanThreads;
  int local[per];
  int sum = 0;
  // thread t owns keys kKeys-1-(t*per) ... descending
  for (int k = 0; k < per; ++k) {
    local[k] = V.hist[kKeys - 1 - (threadIdx.x * per + k)];
    sum += local[k];
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const int a = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += a;
    __syncthreads();
  }
  int run = part[threadIdx.x] - sum;
  for (int k = 0; k < per; ++k) {
    V.hist[kKeys - 1 - (threadIdx.x * per + k)] = run;
    run += local[k];
  }
  if (threadIdx.x == kScanThreads - 1) V.counters[0] = part[kScanThreads - 1] - V.counters[1];
}

// Places every pair at its sorted position: big pairs (positions 0 .. n_big-1) become entries of
// the wavefront pair table, small ones entries of the inter-sequence list.
__global__ __launch_bounds__(kPlanThreads) void sort_scatter_kernel(int64_t n_pairs,
                                                                    const int64_t* __restrict__ q_off,
                                                                    const int64_t* __restrict__ s_off, int orient,
                                                                    int64_t code_cap, SplitView V, WfWs W) {
  __shared__ int h[kKeys];  // this chunk's count per key, then its next position per key
  const int n_big = V.counters[1];
  for (int k = threadIdx.x; k < kKeys; k += blockDim.x) h[k] = 0;
  __syncthreads();
  int64_t p0, p1;
  chunk_of_block(n_pairs, &p0, &p1);
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) atomicAdd(&h[V.keys[p]], 1);
  __syncthreads();
  for (int k = threadIdx.x; k < kKeys; k += blockDim.x)
    if (h[k]) h[k] = atomicAdd(&V.hist[k], h[k]);  // reserve the chunk's range of each key
  __syncthreads();
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const int key = V.keys[p];
    const int pos = atomicAdd(&h[key], 1);
    if (key < kSmallKeys) {
      V.small_idx[pos - n_big] = (int)p;
      continue;
    }
    const int64_t qb = q_off[p], sb = s_off[p];
    const int32_t n = (int32_t)(q_off[p + 1] - qb), m = (int32_t)(s_off[p + 1] - sb);
    const bool flip = orient_flip(n, m, orient);
    WfPair pr;
    pr.q_off = flip ? sb : qb;
    pr.s_off = flip ? qb : sb;
    pr.n = flip ? m : n;
    pr.m = flip ? n : m;
    pr.nb = (pr.n + kWfBand - 1) / kWfBand;
    pr.out_idx = (int32_t)p;
    pr.flip = flip ? 1 : 0;
    pr.pad_ = 0;
    pr.item0 = 0;
    pr.row_off = 0;
    pr.code_off = code_cap > 0 ? V.code_off[p] : 0;
    W.pairs[pos] = pr;
  }
}

// One block: exclusive prefix sums of the bands (item0) and row slots (row_off) of the big pairs.
// Should the totals exceed what the workspace was sized for (the caller understated total_q or
// total_s), the wavefront pairs are dropped and their results flagged instead.
__global__ __launch_bounds__(1024) void split_scan_kernel(SplitView V, WfWs W, int64_t item_cap, int64_t row_cap,
                                                          aln_result_t* __restrict__ out) {
  __shared__ int64_t s_items[1024], s_rows[1024];
  const int np = V.counters[1];
  int64_t base_items = 0, base_rows = 0;
  for (int c0 = 0; c0 < np; c0 += 1024) {
    const int k = c0 + threadIdx.x;
    int64_t it = 0, rw = 0;
    if (k < np) {
      it = W.pairs[k].nb;
      rw = it >= 2 ? 2 * ((int64_t)W.pairs[k].m + 1) : 0;  // one band: no hand-off
    }
    s_items[threadIdx.x] = it;
    s_rows[threadIdx.x] = rw;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t a = threadIdx.x >= o ? s_items[threadIdx.x - o] : 0;
      const int64_t b = threadIdx.x >= o ? s_rows[threadIdx.x - o] : 0;
      __syncthreads();
      s_items[threadIdx.x] += a;
      s_rows[threadIdx.x] += b;
      __syncthreads();
    }
    if (k < np) {
      W.pairs[k].item0 = base_items + s_items[threadIdx.x] - it;
      W.pairs[k].row_off = base_rows + s_rows[threadIdx.x] - rw;
    }
    base_items += s_items[1023];
    base_rows += s_rows[1023];
    __syncthreads();
  }
  const bool fits = base_items <= item_cap && base_rows <= row_cap;
  if (!fits) {
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
      aln_result_t r;
      r.score = 0;
      r.q_begin = r.s_begin = -1;
      r.q_end = r.s_end = 0;
      r.cigar_len = 0;
      r.flags = ALN_RES_DEVICE_ERROR;
      r.reserved = 0;
      out[W.pairs[k].out_idx] = r;
    }
  }
  if (threadIdx.x == 0) {
    *W.n_items = fits ? base_items : 0;
    *W.n_pairs = fits ? np : 0;
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int64_t g_tb_arena_bytes = kTbArenaBytes;

BatchCfg resolve_cfg(const aln_batch_config_t* c) {
  BatchCfg r;
  r.tb_arena = g_tb_arena_bytes;
  r.wf_min_cells = 0;
  r.wf_group = 0;
  r.wf_waves_per_cu = kWfWavesPerCUDefault;
  r.waves_given = false;
  r.orient = 0;
  r.small16 = true;
  r.wf_p16 = false;
  if (!c) return r;
  if (c->wf_min_cells < 0) r.wf_min_cells = INT64_MAX;
  if (c->wf_min_cells > 0) r.wf_min_cells = c->wf_min_cells;
  if (c->wf_waves_per_cu > 0) {
    r.wf_waves_per_cu = c->wf_waves_per_cu;
    r.waves_given = true;
  }
  if (c->wf_group > 0) r.wf_group = c->wf_group;
  if (c->wf_orient < 0) r.orient = 0;
  if (c->wf_orient == 1) r.orient = 1;
  if (c->wf_orient == 2) r.orient = 2;
  if (c->small_bits == 32) r.small16 = false;
  if (c->wf_bits == 16) r.wf_p16 = true;
  return r;
}

void route_rule(int64_t n_pairs, bool tb, const BatchCfg& cfg, int cus, int64_t* min_cells, int64_t* lane_dim) {
  int64_t mc = cfg.wf_min_cells;
  if (tb) {
    // Traceback calls send pairs from kTbMinCells cells up to the band wavefront, with their codes in an
    // arena: the one-pair-per-lane kernels hold a code slab per wave for the largest pair they may meet,
    // so such pairs would cost every wave their size.  The rule is fixed, so that the workspace does
    // not depend on the call's configuration.
    mc = kTbMinCells;
  } else if (mc == 0) {
    // The one-pair-per-lane kernels keep 8 waves of 128 pairs (16-bit lanes) on each compute unit.
    // A batch with fewer pairs leaves waves idle there, and each wave pads its pairs to the largest n
    // and m among them, so such a batch sends its pairs from 2^12 cells up to the band wavefront,
    // whose bands spread over every compute unit.
    const int64_t fill = (int64_t)128 * 8 * (cus > 0 ? cus : 1);
    mc = n_pairs >= fill ? (int64_t)1 << 16 : (int64_t)1 << 12;
  }
  *min_cells = mc;
  // A traceback call also sends every pair longer than kTbLaneDim on either side to the wavefront.
  *lane_dim = tb ? kTbLaneDim : INT64_MAX;
}

aln_status_t plan_split(int64_t n_pairs, int64_t total_q, int64_t total_s, bool tb, int64_t max_n, int64_t max_m,
                        const BatchCfg& cfg, SplitPlan* sp) {
  const int cus = device_cu_count();
  int64_t min_cells = 0;
  route_rule(n_pairs, tb, cfg, cus, &min_cells, &sp->lane_dim);
  sp->tb = tb;
  sp->big_cells = min_cells;
  // a traceback walks its pair as given: no transposed pairs
  sp->orient = tb ? 0 : cfg.orient;
  // Code arena of a traceback call.  A wavefront pair takes ceil(n / 256) x 64 x m words, at most
  // n m / 4 + 64 m; summed over the batch that is at most min(total_q max_m, total_s max_n) / 4 +
  // 64 total_s.  The arena holds that bound when it fits the arena budget (cfg.tb_arena bytes): then
  // every wavefront pair finds room (code_exact), and the lanes' slabs need only hold pairs up to
  // kTbLaneDim on each side.  Otherwise the arena is the budget and the lanes' slabs are sized for the
  // largest pair.  None when no pair within the bounds can reach the wavefront.
  sp->code_cap = 0;
  sp->code_exact = true;
  if (tb && max_n > 0 && max_m > 0 &&
      (max_n * max_m >= min_cells || max_n > kTbLaneDim || max_m > kTbLaneDim)) {
    const int64_t cells = std::min(total_q * max_m, total_s * max_n);
    const int64_t words = cells / 4 + (int64_t)kWfBand / 4 * (total_s + 1);
    const int64_t cap = cfg.tb_arena / 2;
    sp->code_exact = words <= cap;
    sp->code_cap = std::min<int64_t>(words, cap);
  }
  size_t off = 0;
  sp->off_small_idx = off;
  off += align256((size_t)(n_pairs + 1) * sizeof(int));
  sp->off_small_cnt = off;
  off += 256;
  sp->off_keys = off;
  off += align256((size_t)(n_pairs + 1) * sizeof(int));
  sp->off_hist = off;
  off += align256((size_t)kKeys * sizeof(int));
  sp->off_code_off = off;
  off += sp->code_cap > 0 ? align256((size_t)(n_pairs + 1) * sizeof(int64_t)) : 0;
  sp->off_code_used = off;
  off += 256;
  sp->wf_base = off;
  // bands run along the longer side when oriented: at most (n + m) / band + 1 per pair
  const int64_t max_items = (total_q + total_s) / kWfBand + n_pairs + 1;
  // the per-band engine's hand-out order keeps item positions and level counts in 32 bits
  if (max_items > (int64_t)INT32_MAX - 2) return ALN_E_INVALID;
  // a pair of two or more bands has row slots over its columns, never more than m + 1 of them
  sp->item_cap = max_items;
  sp->row_cap = 2 * (total_s + n_pairs);
  off += wf_layout(n_pairs + 1, max_items, sp->row_cap, sp->code_cap, &sp->wf);
  sp->total_bytes = off;
  sp->wf_waves = wf_waves(cfg.wf_waves_per_cu);
  // Groups of bands pay off when the batch has few bands per SIMD: then each compute wave is alone
  // on its SIMD and nothing hides its device-memory waits.  Bands are estimated from the letters
  // (rows along the longer sequence, 256 per band).  On uneven protein batches the per-band engine
  // (bands handed out level by level) overtakes between 46 and 70 estimated bands per compute unit.
  const int64_t est_bands = (total_q + total_s) / (2 * kWfBand);
  sp->grouped = cfg.wf_group == 4 || (cfg.wf_group == 0 && est_bands < (int64_t)56 * (cus > 0 ? cus : 1));
  if (sp->grouped && !cfg.waves_given && cus > 0) {
    // Workgroups take their groups in the order they start, wherever they sit, so a grid with more
    // workgroups than groups can stack several working ones on a compute unit while others idle.
    // By default the grid holds as many workgroups per compute unit as the estimated groups need
    // (1..4; a workgroup is 4 compute waves).
    const int64_t groups = (est_bands + kWfGroupBands - 1) / kWfGroupBands;
    const int64_t per_cu = std::min<int64_t>(std::max<int64_t>((groups + cus - 1) / cus, 1), 4);
    sp->wf_waves = wf_waves((int)(kWfGroupBands * per_cu));
  }
  sp->wf_p16 = cfg.wf_p16;
  return sp->wf_waves > 0 ? ALN_OK : ALN_E_DEVICE;
}

void launch_split(const SplitPlan& sp, int64_t n_pairs, const int64_t* q_off, const int64_t* s_off, int64_t max_n,
                  int64_t max_m, aln_result_t* out, void* ws, hipStream_t stream) {
  char* base = static_cast<char*>(ws);
  SplitView V;
  V.small_idx = reinterpret_cast<int*>(base + sp.off_small_idx);
  V.counters = reinterpret_cast<int*>(base + sp.off_small_cnt);
  V.keys = reinterpret_cast<int*>(base + sp.off_keys);
  V.hist = reinterpret_cast<int*>(base + sp.off_hist);
  V.code_off = reinterpret_cast<int64_t*>(base + sp.off_code_off);
  V.code_used = reinterpret_cast<unsigned long long*>(base + sp.off_code_used);
  WfWs W = wf_view(base + sp.wf_base, sp.wf);
  ProfScope prof("plan", stream);
  hipLaunchKernelGGL(split_reset_kernel, dim3(68), dim3(256), 0, stream, V);
  // one chunk of at least 4096 pairs per block, at most 512 blocks
  int64_t blocks = (n_pairs + 4095) / 4096;
  blocks = blocks < 1 ? 1 : (blocks > 512 ? 512 : blocks);
  hipLaunchKernelGGL(split_classify_kernel, dim3((unsigned)blocks), dim3(kPlanThreads), 0, stream, n_pairs, q_off,
                     s_off, max_n, max_m, sp.big_cells, sp.lane_dim, sp.orient, sp.tb, sp.code_cap, V);
  hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, V);
  hipLaunchKernelGGL(sort_scatter_kernel, dim3((unsigned)blocks), dim3(kPlanThreads), 0, stream, n_pairs, q_off,
                     s_off, sp.orient, sp.code_cap, V, W);
  hipLaunchKernelGGL(split_scan_kernel, dim3(1), dim3(1024), 0, stream, V, W, sp.item_cap, sp.row_cap, out);
}

}  // namespace mialign
