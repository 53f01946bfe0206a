// Canonical traceback walk by a whole wave over 4-bit predecessor codes held in device memory.
//
// The walk of walk.h (the canonical rule: diagonal, then E, then F in the no-gap state; inside a gap
// the gap-open predecessor wins ties; local walks stop at a cell whose H is 0, semi-global ones on
// row 0 or column 0, global ones finish along row 0 or column 0), taken by one wave: the codes are
// read from an LDS window of kWalkGroups row groups x kWalkCols columns ending at the current cell,
// diagonal runs are taken up to 64 cells at a time (lane t looks at cell (i - t, j - t), and the first
// lane whose cell is not a diagonal move, or lies outside the window or the codes, ends the run), and
// gap runs are taken the same way along their column or row.  Every lane runs the same walk and
// stores the same runs.
//
// The codes may cover only a segment of rows, r0 + 1 .. r0 + rows: the walk then stops when it
// reaches row r0 (in the no-gap state or inside a vertical gap), and a later call with the segment
// above continues it.  This is the linear-space traceback of AnySeq Sec. III-A: the segments are
// relaxed again one at a time from stored rows, so only one segment's codes are held at once.  They
// may also cover only the columns right of cb: the walk then stops when it reaches column cb, and a
// later call with the columns left of it continues.
#pragma once
#include "internal.h"

namespace mialign {

constexpr int kWalkGroups = 32;  // row groups (of kWfR rows) in a traceback window
constexpr int kWalkCols = 128;   // columns in a traceback window

// A walk in progress.  Runs are stored last to first while walking; walk_finish reverses them.
struct WalkState {
  int32_t i, j;      // current cell (the begin cell once done)
  int32_t state;     // 0 = H, 1 = E (vertical gap, CIGAR I), 2 = F (horizontal gap, CIGAR D)
  int32_t done;      // the walk has reached the alignment's first cell
  uint32_t cur_op;   // the run being built (0xff: none yet)
  uint32_t cur_len;
  int64_t runs;      // runs stored so far
  int32_t stuck;     // the walk did not end within its bound of turns (never, for valid codes)
  int32_t pad_;
};

__device__ __forceinline__ void walk_start(WalkState& S, int i, int j) {
  S.i = i;
  S.j = j;
  S.state = 0;
  S.done = 0;
  S.cur_op = 0xffu;
  S.cur_len = 0;
  S.runs = 0;
  S.stuck = 0;
  S.pad_ = 0;
}

// Walks from S through the codes of rows r0 + 1 .. and columns cb + 1 .. (row group g of the segment,
// column c at codes[g * ld + c - 1]).  Returns when the walk is done or has reached row r0 > 0 or
// column cb > 0.
template <int MODE>
__device__ void walk_core(const uint16_t* __restrict__ codes, int64_t ld, int r0, int cb, WalkState& S,
                          uint16_t* __restrict__ win, int lane, uint32_t* __restrict__ cig, int64_t cap) {
  if (S.done) return;
  // Every lane holds the same walk state; saying so lets the compiler keep it in scalar registers
  // and branch on it with scalar branches.
  int i = __builtin_amdgcn_readfirstlane(S.i);
  int j = __builtin_amdgcn_readfirstlane(S.j);
  int state = __builtin_amdgcn_readfirstlane(S.state);
  uint32_t cur_op = (uint32_t)__builtin_amdgcn_readfirstlane((int)S.cur_op);
  uint32_t cur_len = (uint32_t)__builtin_amdgcn_readfirstlane((int)S.cur_len);
  int64_t runs = S.runs;
  bool done = false;
  // The window holds row groups g0-kWalkGroups+1..g0 of the segment and columns c0-kWalkCols+1..c0; it is
  // loaded at the walk's cell, in row group g0 and column c0.  The walk only moves up and left, so every
  // later cell is inside it as long as it lies at or below row ilo and at or right of column jlo (the
  // window's first row and column inside the segment).  Before the first load nothing is inside.
  int g0 = 0, c0 = 0, ilo = 0x7fffffff, jlo = 0x7fffffff;
  auto load = [&](int ii, int jj) {
    g0 = (ii - r0 - 1) / kWfR;
    c0 = jj;
    ilo = r0 + max(1, (g0 - kWalkGroups + 1) * kWfR + 1);
    jlo = max(cb + 1, c0 - kWalkCols + 1);
    // Every load of the window is issued before the first LDS write, so the reload costs one memory
    // latency rather than one per code.  A window cell outside the segment (row group < 0 or column
    // < 1) loads the in-bounds cell (g0, c0) instead; it lies before row ilo or column jlo, so code()
    // never reads it.  The loads carry no branches, so all of them stay in flight together.
    constexpr int kPer = kWalkGroups * kWalkCols / 64;
    uint32_t v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = lane + 64 * u;
      const int gg = g0 - k / kWalkCols, cc = c0 - k % kWalkCols;
      const bool ok = gg >= 0 && cc >= 1;
      v[u] = codes[(size_t)(ok ? gg : g0) * (size_t)ld + (size_t)((ok ? cc : c0) - 1)];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) win[lane + 64 * u] = (uint16_t)v[u];
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");  // the window is in LDS before it is read
  };
  // the code of a cell inside the window
  auto code = [&](int ii, int jj) -> uint32_t {
    const unsigned r = (unsigned)(ii - r0 - 1);
    const uint32_t w = win[(g0 - (int)(r / kWfR)) * kWalkCols + (c0 - jj)];
    return (w >> (4 * (r % kWfR))) & 15u;
  };
  auto push = [&](uint32_t op, uint32_t len) {
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
  int64_t turns = 2 * ((int64_t)i + j) + 64;
  for (; turns > 0; --turns) {
    if (state == 0) {
      if (i == 0 || j == 0) {
        if (MODE == ALN_GLOBAL) {
          if (j > 0) push(ALN_CIGAR_D, (uint32_t)j);
          if (i > 0) push(ALN_CIGAR_I, (uint32_t)i);
          i = 0;
          j = 0;
        }
        done = true;
        break;
      }
      if (i == r0) break;  // the segment above holds this cell
      if (cb > 0 && j == cb) break;  // the columns left of cb hold it
      if (i < ilo || j < jlo) load(i, j);
      // lanes t <= lim look at cells inside the window; the others read (i, j) and count as a
      // non-diagonal code, which ends the run
      const int lim = min(i - ilo, j - jlo);
      const bool in = lane <= lim;
      const int t = in ? lane : 0;
      const uint32_t ct = code(i - t, j - t);
      const uint32_t pc = in ? ct : 3u;
      const unsigned long long stop = __builtin_amdgcn_ballot_w64((pc & 3u) != 0u);
      const int k = stop ? __builtin_ctzll(stop) : 64;
      if (k > 0) {
        push(ALN_CIGAR_M, (uint32_t)k);
        i -= k;
        j -= k;
        continue;
      }
      // lane 0 looked at (i, j) itself, which the window holds; its code also gives the first gap
      // step, taken below without reading the cell again
      const uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane((int)pc);
      if ((c & 3u) == 3u) {
        done = true;
        break;
      }
      state = (int)(c & 3u);
      if (state == 1) {
        push(ALN_CIGAR_I, 1);
        if (!(c & 4u) || i == 1) state = 0;
        --i;
      } else {
        push(ALN_CIGAR_D, 1);
        if (!(c & 8u) || j == 1) state = 0;
        --j;
      }
    } else {
      if (state == 1 && i == r0) break;  // the vertical gap goes on in the segment above
      if (cb > 0 && j == cb) break;       // the gap goes on in (or ends at) a column left of cb
      // A gap run, up to 64 steps at a time: lane t looks at the t-th cell of the run.  The run goes
      // on through a cell whose extension bit is set and which is not in row (column) 1; the first
      // cell that ends it is stepped through and returns the walk to H, unless it lies outside the
      // window, where the walk stops short of it and reloads.
      if (i < ilo || j < jlo) load(i, j);
      const bool vert = state == 1;
      const int lim = vert ? i - ilo : j - jlo;  // lanes t <= lim look at cells inside the window
      const bool in = lane <= lim;
      const int t = in ? lane : 0;
      const int ii = vert ? i - t : i, jj = vert ? j : j - t;
      const uint32_t pc = code(ii, jj);
      const bool more = in && (pc & (vert ? 4u : 8u)) != 0u && (vert ? ii : jj) > 1;
      const unsigned long long stop = __builtin_amdgcn_ballot_w64(!more);
      const int k = stop ? __builtin_ctzll(stop) : 64;
      const bool ends = k < 64 && k <= lim;
      const int steps = k + (ends ? 1 : 0);
      push(vert ? ALN_CIGAR_I : ALN_CIGAR_D, (uint32_t)steps);
      if (vert)
        i -= steps;
      else
        j -= steps;
      if (ends) state = 0;
    }
  }
  if (turns <= 0) {
    S.stuck = 1;
    done = true;
  }
  S.i = i;
  S.j = j;
  S.state = state;
  S.done = done ? 1 : 0;
  S.cur_op = cur_op;
  S.cur_len = cur_len;
  S.runs = runs;
}

// Ends a walk: stores the last run and reverses the runs (last to first while walking) with the whole
// wave.  Lane l swaps the pairs (a, runs-1-a) with a = l, l+64, ...: no two lanes touch the same run,
// and each lane's loads are its own earlier stores' addresses only through the walk, which has
// completed.  Returns the number of runs.
__device__ inline int64_t walk_finish(WalkState& S, int lane, uint32_t* __restrict__ cig, int64_t cap) {
  int64_t runs = S.runs;
  if (S.cur_len) {
    if (runs < cap) cig[runs] = (S.cur_len << 4) | S.cur_op;
    ++runs;
  }
  S.cur_len = 0;
  S.runs = runs;
  if (runs <= cap) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const int64_t half = runs / 2;
    for (int64_t a = lane; a < half; a += 64) {
      const int64_t b = runs - 1 - a;
      const uint32_t x = cig[a], y = cig[b];
      cig[a] = y;
      cig[b] = x;
    }
  }
  return runs;
}

}  // namespace mialign
