// Canonical traceback walk over stored 4-bit predecessor codes (device side).
//
// Code of cell (i,j): bits 0-1 = which term gave H (0 diagonal, 1 E, 2 F, 3 the
// local zero), bit 2 = E(i,j) extended E(i-1,j) rather than opening from
// H(i-1,j), bit 3 = F(i,j) extended F(i,j-1).  (The relaxation function of
// AnySeq Sec. III-B records the predecessor of H; the two extension bits add
// what the affine model needs.)  The walk starts at the optimum in state H and
// follows, by priority, diagonal, then E, then F; inside a gap it stops the run
// when the gap was opened at that cell.  Local walks stop at a cell whose H is
// 0, semi-global walks on row 0 or column 0, global walks finish along row 0 or
// column 0 with one gap run.
#pragma once
#include "internal.h"

namespace mialign {

// code(i, j) returns the 4-bit code of cell (i, j), i, j >= 1.  The CIGAR is written forward into
// cig[0..runs) when it fits in cap words; *n_runs receives the number of runs either way.
template <int MODE, typename CodeFn>
__device__ void walk_back(CodeFn code, int i, int j, uint32_t* cig, int64_t cap, int* q_begin, int* s_begin,
                          int* n_runs) {
  int state = 0;  // 0 = H, 1 = E, 2 = F
  int64_t runs = 0;
  uint32_t cur_op = 0xffu, cur_len = 0;
  auto push_n = [&](uint32_t op, uint32_t len) {
    if (op == cur_op) {
      cur_len += len;
      return;
    }
    if (cur_len) {
      if (runs < cap) cig[runs] = (cur_len << 4) | cur_op;
      ++runs;
    }
    cur_op = op;
    cur_len = len;
  };
  auto push = [&](uint32_t op) { push_n(op, 1); };
  for (;;) {
    if (state == 0) {
      if (i == 0 || j == 0) {
        if (MODE == ALN_GLOBAL) {
          if (j > 0) push_n(ALN_CIGAR_D, (uint32_t)j);
          if (i > 0) push_n(ALN_CIGAR_I, (uint32_t)i);
          i = 0;
          j = 0;
        }
        break;
      }
      // The next kDiag cells along the diagonal are read together, so their loads are in flight at
      // once; the walk takes the diagonal moves among them up to the first cell that is not one (or
      // the matrix border), which it then handles from the code already read.
      constexpr int kDiag = 8;
      const int lim = min(min(i, j), kDiag);
      uint32_t hs[kDiag];
#pragma unroll
      for (int t = 0; t < kDiag; ++t) hs[t] = t < lim ? (code(i - t, j - t) & 3u) : 0u;
      int k = 0;
      uint32_t stop = 0u;
#pragma unroll
      for (int t = kDiag - 1; t >= 0; --t)
        if (t < lim && hs[t] != 0u) {
          k = t;
          stop = hs[t];
        }
      if (stop == 0u) k = lim;  // every cell read is a diagonal move
      if (k > 0) push_n(ALN_CIGAR_M, (uint32_t)k);
      i -= k;
      j -= k;
      if (stop == 3u) break;
      if (stop != 0u) state = (int)stop;
    } else if (state == 1) {
      const uint32_t c = code(i, j);
      push(ALN_CIGAR_I);
      if (!(c & 4u)) state = 0;
      --i;
      if (i == 0) state = 0;
    } else {
      const uint32_t c = code(i, j);
      push(ALN_CIGAR_D);
      if (!(c & 8u)) state = 0;
      --j;
      if (j == 0) state = 0;
    }
  }
  if (cur_len) {
    if (runs < cap) cig[runs] = (cur_len << 4) | cur_op;
    ++runs;
  }
  if (runs <= cap) {
    for (int64_t a = 0, b = runs - 1; a < b; ++a, --b) {
      const uint32_t t = cig[a];
      cig[a] = cig[b];
      cig[b] = t;
    }
  }
  *q_begin = i;
  *s_begin = j;
  *n_runs = (int)runs;
}

__device__ __forceinline__ int wave_max_i32(int v) {
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

}  // namespace mialign
