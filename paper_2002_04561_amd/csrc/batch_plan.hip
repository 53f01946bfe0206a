// Device-side planning of a batch: routes each pair to the inter-sequence kernel (one pair per
// lane) or, when its matrix is large, to the intra-sequence wavefront engine (one band per wave).
// Everything runs on the device, so a batch needs no host copy of its lengths and stays
// capturable in a HIP graph.
#include "internal.h"

namespace mialign {
namespace {

struct SplitView {
  int* small_idx;
  int* counters;  // [0] small pairs, [1] big pairs
};

__global__ void split_reset_kernel(SplitView V) {
  if (threadIdx.x < 2) V.counters[threadIdx.x] = 0;
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
      W.pairs[k] = pr;
    } else {
      const int k = atomicAdd(&V.counters[0], 1);
      V.small_idx[k] = (int)p;
    }
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

aln_status_t plan_split(int64_t n_pairs, int64_t total_q, int64_t total_s, SplitPlan* sp) {
  sp->big_cells = (int64_t)1 << 20;
  size_t off = 0;
  sp->off_small_idx = off;
  off += align256((size_t)(n_pairs + 1) * sizeof(int));
  sp->off_small_cnt = off;
  off += 256;
  sp->wf_base = off;
  const int64_t max_items = total_q / kWfBand + n_pairs + 1;
  off += wf_layout(n_pairs + 1, max_items, 2 * (total_s + n_pairs), &sp->wf);
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
  WfWs W = wf_view(base + sp.wf_base, sp.wf);
  hipLaunchKernelGGL(split_reset_kernel, dim3(1), dim3(64), 0, stream, V);
  const int64_t blocks = (n_pairs + 255) / 256;
  hipLaunchKernelGGL(split_classify_kernel, dim3((unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096)),
                     dim3(256), 0, stream, n_pairs, q_off, s_off, max_n, max_m, sp.big_cells, V, W);
  hipLaunchKernelGGL(split_scan_kernel, dim3(1), dim3(1024), 0, stream, V, W);
}

}  // namespace mialign
