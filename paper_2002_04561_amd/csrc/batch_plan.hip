// Device-side planning of a batch: routes each pair to the inter-sequence kernels (one pair per
// lane) or, when its matrix is large, to the intra-sequence wavefront engine (one band per wave),
// and sorts the inter-sequence pairs by shape so that the 64 or 128 pairs sharing a wave have
// similar n and m (a wave runs max n x max m steps for all of its pairs).  Shapes are binned on a
// log scale with 8 bins per octave of n and of m; a counting sort lays the bins out from the
// largest to the smallest, so long pairs start first.  Everything runs on the device: a batch
// needs no host copy of its lengths and stays capturable in a HIP graph.
#include "internal.h"

namespace mialign {
namespace {

constexpr int kShapeBins = 128;                     // per dimension
constexpr int kKeys = kShapeBins * kShapeBins;      // sort keys

struct SplitView {
  int* small_idx;  // sorted inter-sequence list
  int* counters;   // [0] small pairs, [1] big pairs
  int* keys;       // per pair: shape key, or -1 for a big pair
  int* hist;       // [kKeys] counts, then cursors
};

// 8 bins per octave: floor(8 * log2(x)) for x >= 8, x itself below.
__device__ __forceinline__ int log_bin(int64_t x) {
  if (x < 8) return (int)(x < 0 ? 0 : x);
  const int e = 63 - __builtin_clzll((unsigned long long)x);
  const int frac = (int)((x >> (e - 3)) & 7);
  const int b = e * 8 + frac - 16;  // x = 8 gives 8
  return b < kShapeBins ? b : kShapeBins - 1;
}

__global__ void split_reset_kernel(SplitView V) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < kKeys; k += gridDim.x * blockDim.x) V.hist[k] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 2) V.counters[threadIdx.x] = 0;
}

__global__ void split_classify_kernel(int64_t n_pairs, const int64_t* __restrict__ q_off,
                                      const int64_t* __restrict__ s_off, int64_t max_n, int64_t max_m,
                                      int64_t big_cells, SplitView V, WfWs W) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t qb = q_off[p], sb = s_off[p];
    const int64_t n = q_off[p + 1] - qb, m = s_off[p + 1] - sb;
    const bool fits = n >= 0 && m >= 0 && n <= max_n && m <= max_m;
    if (fits && n > 0 && m > 0 && n * m >= big_cells) {
      const int k = atomicAdd(&V.counters[1], 1);
      WfPair pr;
      pr.q_off = qb;
      pr.s_off = sb;
      pr.n = (int32_t)n;
      pr.m = (int32_t)m;
      pr.nb = (int32_t)((n + kWfBand - 1) / kWfBand);
      pr.out_idx = (int32_t)p;
      pr.item0 = 0;
      pr.row_off = 0;
      pr.code_off = 0;
      W.pairs[k] = pr;
      V.keys[p] = -1;
    } else {
      const int key = log_bin(n) * kShapeBins + log_bin(m);
      V.keys[p] = key;
      atomicAdd(&V.hist[key], 1);
    }
  }
}

// One block: turns the key histogram into cursors, largest shapes first, and counts the list.
__global__ __launch_bounds__(1024) void sort_scan_kernel(SplitView V) {
  __shared__ int part[1024];
  constexpr int per = kKeys / 1024;
  int local[per];
  int sum = 0;
  // thread t owns keys kKeys-1-(t*per) ... descending
  for (int k = 0; k < per; ++k) {
    local[k] = V.hist[kKeys - 1 - (threadIdx.x * per + k)];
    sum += local[k];
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
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
  if (threadIdx.x == 1023) V.counters[0] = part[1023];
}

__global__ void sort_scatter_kernel(int64_t n_pairs, SplitView V) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int key = V.keys[p];
    if (key < 0) continue;
    const int pos = atomicAdd(&V.hist[key], 1);
    V.small_idx[pos] = (int)p;
  }
}

// One block: exclusive prefix sums of the bands (item0) and row slots (row_off) of the big pairs.
__global__ __launch_bounds__(1024) void split_scan_kernel(SplitView V, WfWs W) {
  __shared__ int64_t s_items[1024], s_rows[1024];
  const int np = V.counters[1];
  int64_t base_items = 0, base_rows = 0;
  for (int c0 = 0; c0 < np; c0 += 1024) {
    const int k = c0 + threadIdx.x;
    int64_t it = 0, rw = 0;
    if (k < np) {
      it = W.pairs[k].nb;
      rw = 2 * ((int64_t)W.pairs[k].m + 1);
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
  if (threadIdx.x == 0) {
    *W.n_items = base_items;
    *W.n_pairs = np;
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

aln_status_t plan_split(int64_t n_pairs, int64_t total_q, int64_t total_s, bool route_big, SplitPlan* sp) {
  sp->big_cells = route_big ? ((int64_t)1 << 20) : INT64_MAX;
  size_t off = 0;
  sp->off_small_idx = off;
  off += align256((size_t)(n_pairs + 1) * sizeof(int));
  sp->off_small_cnt = off;
  off += 256;
  sp->off_keys = off;
  off += align256((size_t)(n_pairs + 1) * sizeof(int));
  sp->off_hist = off;
  off += align256((size_t)kKeys * sizeof(int));
  sp->wf_base = off;
  const int64_t max_items = total_q / kWfBand + n_pairs + 1;
  off += wf_layout(n_pairs + 1, max_items, 2 * (total_s + n_pairs), 0, &sp->wf);
  sp->total_bytes = off;
  sp->wf_waves = wf_waves();
  return sp->wf_waves > 0 ? ALN_OK : ALN_E_DEVICE;
}

void launch_split(const SplitPlan& sp, int64_t n_pairs, const int64_t* q_off, const int64_t* s_off, int64_t max_n,
                  int64_t max_m, void* ws, hipStream_t stream) {
  char* base = static_cast<char*>(ws);
  SplitView V;
  V.small_idx = reinterpret_cast<int*>(base + sp.off_small_idx);
  V.counters = reinterpret_cast<int*>(base + sp.off_small_cnt);
  V.keys = reinterpret_cast<int*>(base + sp.off_keys);
  V.hist = reinterpret_cast<int*>(base + sp.off_hist);
  WfWs W = wf_view(base + sp.wf_base, sp.wf);
  ProfScope prof("plan", stream);
  hipLaunchKernelGGL(split_reset_kernel, dim3(64), dim3(256), 0, stream, V);
  const int64_t blocks = (n_pairs + 255) / 256;
  const dim3 grid((unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096));
  hipLaunchKernelGGL(split_classify_kernel, grid, dim3(256), 0, stream, n_pairs, q_off, s_off, max_n, max_m,
                     sp.big_cells, V, W);
  hipLaunchKernelGGL(split_scan_kernel, dim3(1), dim3(1024), 0, stream, V, W);
  hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(1024), 0, stream, V);
  hipLaunchKernelGGL(sort_scatter_kernel, grid, dim3(256), 0, stream, n_pairs, V);
}

}  // namespace mialign
