// Linear-space traceback of one long pair.
//
// AnySeq (Sec. III-A) traces back in linear space by relaxing the matrix again, at the cost of at most
// doubling the cells relaxed.  Here the forward pass (the grouped band wavefront, score only) also keeps
// checkpoints: the bottom row (H, E) of every workgroup of 4 bands (every kTileRows rows) and the column
// (H, F) of every kTileCols-th column, all rows.  Any tile of kTileRows x kTileCols cells can then be
// relaxed again on its own from the row above it and the column left of it, replaying exactly the
// forward pass's integers.  The walk goes back through segments of rows, bottom first.  For each
// segment, the tiles at or above the walk's row and left of its column, within a window as wide as the
// rows the walk has left in the segment plus kTbWinMargin columns, are relaxed again in parallel (one
// workgroup of 4 band waves per tile), storing the 4-bit predecessor codes of walk.h for the segment
// only; then one wave walks the segment (walk_wave.h).  A near-diagonal path crosses the segment inside
// the window; a walk that reaches the window's left edge first stops there, the tiles left of the
// window are relaxed again, and the walk goes on.  The walk then hands its position to the next
// segment up.  Each cell is relaxed again at most once, so the whole traceback relaxes at most twice
// the cells of the matrix; memory is one segment of codes plus the checkpoints, not a code per cell.
#include "band.h"
#include "internal.h"
#include "walk_wave.h"

namespace mialign {
namespace {

constexpr int kTBlk = 32;      // steps between lane-0 input refills
constexpr int kTRing = 256;    // columns held by the ring between two bands of a tile
constexpr int kTWaves = kTileRows / kWfBand;  // bands (waves) of a tile
constexpr int kTbWinMargin = 2 * kTileCols;   // window columns beyond the rows the walk has left

// Profile kinds of the band wavefront (band.h): register bytes for up to 4 letters, else the LDS table.

__device__ __forceinline__ int t_dpp_shr1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xf, 0xf, false);  // wave_shr:1, lane 0 keeps old
}
__device__ __forceinline__ int t_dpp_shl1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x130, 0xf, 0xf, false);  // wave_shl:1, lane 63 keeps old
}

struct TbView {
  int n, m;            // rows (query) and columns (subject) of the pair
  int seg_rows;        // rows of a segment, a multiple of kTileRows
  int strips;          // tiles across the columns, ceil(m / kTileCols)
  const int2* ckrows;  // [g][c] (stride m + 1): Hb, Eb of row (g + 1) * kTileRows, columns 1..m
  const int2* ckcols;  // [k][i - 1] (stride ck_ld): Hb, Fb of column (k + 1) * kTileCols
  int64_t ck_ld;
  uint16_t* codes;     // the current segment's codes: [row group][column - 1], stride m
  WalkState* walk;
  int* error;          // set when a bounded wait gives up
  int* win_lo;         // the current segment's window: its first tile column
};

// First tile column of the window of a segment whose tiles are relaxed again from the walk at (i, j):
// the walk's column minus the rows it has left in the segment and a margin.
__device__ __forceinline__ int tb_window_lo(int i, int j, int seg_r0) {
  const int c = j - (i - seg_r0) - kTbWinMargin;
  return c > 0 ? c / kTileCols : 0;
}

// One tile of the segment `seg`, relaxed again with the codes stored.  Values carry the row bias of
// the band wavefront (Hb = H - i*ge, likewise E and F), so they are the forward pass's own integers.
// Phase 0 relaxes the tiles of the window, phase 1 (after a walk that stopped at the window's left
// edge) those left of it.
template <int MODE, bool AFFINE, int PROF>
__global__ __launch_bounds__(64 * kTWaves) void tb_tile_kernel(const KParams P, const uint8_t* __restrict__ Q,
                                                              const uint8_t* __restrict__ S, TbView V, int seg,
                                                              int phase) {
  constexpr int R = kWfR, BLK = kTBlk;
  __shared__ int32_t tab[kTab * kTab];
  __shared__ int4 stage[kTWaves][3][BLK / 4];  // lane-0 inputs of BLK steps: H, E, letter
  __shared__ int2 ring[kTWaves][kTRing];       // ring w carries band w-1's bottom row to band w
  __shared__ int pub[kTWaves], con[kTWaves];
  __shared__ int s_err;
  for (int k = threadIdx.x; k < kTab * kTab; k += blockDim.x) {
    const int a = k / kTab, b = k % kTab;
    tab[k] = (a >= P.alphabet || b >= P.alphabet) ? -kBig32 : (int32_t)P.sig[a * kMaxAlphabet + b] - P.ge;
  }
  if (threadIdx.x < kTWaves) {
    pub[threadIdx.x] = 0;
    con[threadIdx.x] = 0;
  }
  if (threadIdx.x == 0) s_err = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wib = threadIdx.x >> 6;
  const int n = V.n, m = V.m;
  const int i_w = V.walk->i, j_w = V.walk->j, w_done = V.walk->done;
  const int seg_r0 = seg * V.seg_rows;
  const int tr = blockIdx.x / V.strips, sc = blockIdx.x % V.strips;
  const int R0 = seg_r0 + tr * kTileRows, C0 = sc * kTileCols;
  // only tiles at or above the walk's row and left of its column, in the segment it is in, and in
  // (phase 0) or left of (phase 1) the segment's window
  if (w_done || i_w <= seg_r0 || R0 >= i_w || C0 >= j_w) return;
  const int lo = phase == 0 ? tb_window_lo(i_w, j_w, seg_r0) : *V.win_lo;
  if (phase == 0 ? sc < lo : sc >= lo) return;
  const int rows_hi = min(n, i_w);
  const int cols = min(C0 + kTileCols, j_w) - C0;  // tile columns C0+1 .. C0+cols
  const int i0 = R0 + wib * kWfBand;               // this band's rows i0+1 .. i0+kWfBand
  if (i0 >= rows_hi) return;                       // the bands below it return too; none waits on it
  const bool has_out = wib + 1 < kTWaves && i0 + kWfBand < rows_hi;
  const int32_t go = P.go, ge = P.ge, goe = P.goe;
  int* st_h = reinterpret_cast<int*>(&stage[wib][0][0]);
  int* st_e = reinterpret_cast<int*>(&stage[wib][1][0]);
  int* st_c = reinterpret_cast<int*>(&stage[wib][2][0]);
  auto give_up = [&]() {
    if (lane == 0) {
      __hip_atomic_store(&s_err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_store(V.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  auto lds_wait_ge = [&](int* p, int v) -> bool {
    long long spins = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < v) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > P.spin_lds || __hip_atomic_load(&s_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
        give_up();
        return false;
      }
    }
    return true;
  };

  // rows of this lane, their letters and profile entries
  int prof[R];
  int32_t hl[R], f[R], nu[R];
  const int irow0 = i0 + lane * R;  // the row just above this lane's first row
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = irow0 + r + 1;
    int c = kPad;
    if (i <= n) {
      c = Q[i - 1];
      if (c >= P.alphabet) c = kPad;
    }
    if (PROF == kProfReg) {
      uint32_t w = 0;
      for (int a = 0; a < 4; ++a) {
        const int v = (c < P.alphabet && a < P.alphabet) ? tab[c * kTab + a] : -128;
        w |= ((uint32_t)(v & 0xff)) << (8 * a);
      }
      prof[r] = (int)w;
    } else {
      prof[r] = c * kTab;
    }
    nu[r] = -i * ge;  // local floor: H = 0
  }
  // the column left of the tile (the matrix border, or a checkpoint column), and the cell above-left
  // of each lane's first row
  int32_t diag;
  if (C0 == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = irow0 + r + 1;
      hl[r] = (MODE == ALN_GLOBAL) ? go : -i * ge;  // Hb(i, 0)
      f[r] = kNeg32;
    }
    diag = (MODE == ALN_GLOBAL) ? (irow0 > 0 ? go : 0) : -irow0 * ge;  // Hb(irow0, 0)
  } else {
    const int2* cc = V.ckcols + (int64_t)(C0 / kTileCols - 1) * V.ck_ld;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int2 v = cc[irow0 + r];
      hl[r] = v.x;
      f[r] = v.y;
    }
    if (irow0 > R0)
      diag = cc[irow0 - 1].x;
    else if (R0 == 0)
      diag = (MODE == ALN_GLOBAL) ? go + C0 * ge : 0;  // H(0, C0)
    else
      diag = V.ckrows[(int64_t)(R0 / kTileRows - 1) * (m + 1) + C0].x;
  }
  uint16_t* __restrict__ codes = V.codes + (int64_t)((irow0 - seg_r0) / R) * m + C0;
  int32_t bot_h = 0, bot_e = kNeg32, cur_c = 0, out_h = 0, out_e = 0;
  int2* __restrict__ rin = ring[wib];
  int2* __restrict__ rout = ring[has_out ? wib + 1 : wib];
  const uint8_t* __restrict__ s = S + C0;
  auto letter_idx = [&](int col) -> int {
    if (col > cols) return 0;
    int c = s[col - 1];
    if (c >= P.alphabet) c = PROF == kProfTable ? kPad : 0;
    return PROF == kProfReg ? c * 8 : c;
  };

  const int steps = cols + 63;
  for (int tb = 0; tb < steps; tb += BLK) {
    // lane-0 inputs for steps tb..tb+BLK-1 (tile columns tb+1..tb+BLK), held by lanes < BLK
    const int col_in = tb + 1 + lane;
    const int sreg = lane < BLK ? letter_idx(col_in) : 0;
    int32_t th = 0, te = kNeg32;
    if (wib == 0) {
      if (lane < BLK && col_in <= cols) {
        if (R0 == 0) {
          th = (MODE == ALN_GLOBAL) ? go + (C0 + col_in) * ge : 0;
        } else {
          const int2 v = V.ckrows[(int64_t)(R0 / kTileRows - 1) * (m + 1) + C0 + col_in];
          th = v.x;
          te = v.y;
        }
      }
    } else {
      const int need = min(tb + BLK, cols);
      if (!lds_wait_ge(&pub[wib], need)) break;
      if (lane < BLK && col_in <= cols) {
        const int2 v = rin[col_in % kTRing];
        th = v.x;
        te = v.y;
      }
      // the ring reads are complete before their slots are released to the band above
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      if (lane == 0) __hip_atomic_store(&con[wib], need, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (lane < BLK) {
      st_h[lane] = th;
      st_e[lane] = te;
      st_c[lane] = sreg;
    }
    // One step: lane l relaxes tile column jt = t - l + 1 for its R rows and stores their codes.
    auto step = [&](int t, int in_top_h, int in_top_e, int in_top_c, auto checked) {
      const int jt = t - lane + 1;
      const int in_h = t_dpp_shr1(in_top_h, bot_h);
      const int in_e = t_dpp_shr1(in_top_e, bot_e);
      const int in_c = t_dpp_shr1(in_top_c, cur_c);
      cur_c = in_c;
      if (!decltype(checked)::value || (jt >= 1 && jt <= cols)) {
        int32_t hup = in_h, eup = in_e, hn = 0, unused_bv[R];
        int unused_bj[R];
        uint32_t word = 0;
        band_column<MODE, AFFINE, PROF, true, decltype(checked)::value, R, false>(
            tab, prof, in_c, 0, go, ge, goe, nu, hl, f, unused_bv, unused_bj, nullptr, jt, -1, diag, hup, eup, hn,
            word);
        codes[jt - 1] = (uint16_t)word;
        bot_h = hup;
        bot_e = eup;
        diag = in_h;
      }
      out_h = t_dpp_shl1(bot_h, out_h);
      out_e = t_dpp_shl1(bot_e, out_e);
    };
    for (int g4 = 0; g4 < BLK / 4; ++g4) {
      const int t0 = tb + 4 * g4;
      const int4 vh = reinterpret_cast<const int4*>(st_h)[g4];
      const int4 ve = reinterpret_cast<const int4*>(st_e)[g4];
      const int4 vc = reinterpret_cast<const int4*>(st_c)[g4];
      if (t0 >= 63 && t0 + 3 < cols) {
        step(t0, vh.x, ve.x, vc.x, std::false_type());
        step(t0 + 1, vh.y, ve.y, vc.y, std::false_type());
        step(t0 + 2, vh.z, ve.z, vc.z, std::false_type());
        step(t0 + 3, vh.w, ve.w, vc.w, std::false_type());
      } else {
        step(t0, vh.x, ve.x, vc.x, std::true_type());
        step(t0 + 1, vh.y, ve.y, vc.y, std::true_type());
        step(t0 + 2, vh.z, ve.z, vc.z, std::true_type());
        step(t0 + 3, vh.w, ve.w, vc.w, std::true_type());
      }
    }
    // lanes 64-BLK.. hold lane 63's outputs of steps tb..tb+BLK-1, i.e. tile columns tb-62..tb+BLK-63
    if (has_out) {
      const int hi = min(tb + BLK - 63, cols);
      const int col_out = tb + (lane - (64 - BLK)) - 62;
      const bool mine = lane >= 64 - BLK && col_out >= 1 && col_out <= cols;
      if (hi >= 1) {
        // the band below has read what this overwrites
        if (!lds_wait_ge(&con[wib + 1], hi - kTRing)) break;
        if (mine) rout[col_out % kTRing] = make_int2(out_h, out_e);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (lane == 0) __hip_atomic_store(&pub[wib + 1], hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
}

// One wave walks the codes of segment `seg` from where the walk stands, if it stands in it: in phase 0
// up to the window's left edge (recorded for phase 1's tiles), in phase 1 on from there.
template <int MODE>
__global__ __launch_bounds__(64) void tb_walk_kernel(TbView V, int seg, int phase, uint32_t* __restrict__ cig,
                                                     int64_t cap) {
  __shared__ uint16_t win[kWalkGroups * kWalkCols];
  const int lane = threadIdx.x;
  WalkState S = *V.walk;
  const int seg_r0 = seg * V.seg_rows;
  if (S.done || S.i <= seg_r0) return;
  int cb = 0;
  if (phase == 0) {
    const int lo = tb_window_lo(S.i, S.j, seg_r0);
    cb = lo * kTileCols;
    if (lane == 0) *V.win_lo = lo;
  }
  walk_core<MODE>(V.codes, V.m, seg_r0, cb, S, win, lane, cig, cap);
  __syncthreads();  // every lane has read the state before lane 0 writes it
  if (lane == 0) *V.walk = S;
}

// Starts the walk at the forward pass's optimum (its aln_result_t).  A walk that starts on row 0 or
// column 0 ends there at once (global alignments against an empty prefix take their gap run here).
template <int MODE>
__global__ __launch_bounds__(64) void tb_init_kernel(const aln_result_t* __restrict__ out, TbView V,
                                                     uint32_t* __restrict__ cig, int64_t cap) {
  __shared__ uint16_t win[1];  // never loaded: the walk below starts on row 0 or column 0
  const int lane = threadIdx.x;
  const aln_result_t r = *out;
  WalkState S;
  walk_start(S, r.q_end, r.s_end);
  if (r.flags) {
    S.done = 1;  // no CIGAR for a failed forward pass
  } else if (r.q_end == 0 || r.s_end == 0) {
    walk_core<MODE>(nullptr, 0, 0, 0, S, win, lane, cig, cap);
  }
  if (lane == 0) {
    *V.walk = S;
    *V.error = 0;
  }
}

// Ends the walk: reverses the runs and completes the pair's result.
__global__ __launch_bounds__(64) void tb_final_kernel(aln_result_t* __restrict__ out, TbView V,
                                                      uint32_t* __restrict__ cig, int64_t cap) {
  const int lane = threadIdx.x;
  aln_result_t r = *out;
  if (r.flags) return;
  WalkState S = *V.walk;
  if (!S.done || S.stuck || __hip_atomic_load(V.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    if (lane == 0) out->flags = r.flags | ALN_RES_DEVICE_ERROR;
    return;
  }
  const int64_t runs = walk_finish(S, lane, cig, cap);
  if (lane == 0) {
    r.q_begin = S.i;
    r.s_begin = S.j;
    r.cigar_len = (int)runs;
    if (runs > cap) r.flags |= ALN_RES_CIGAR_TRUNC;
    *out = r;
  }
}

template <int MODE, bool AFFINE, int PROF>
void launch_tiles(const KParams& kp, const uint8_t* q, const uint8_t* s, const TbView& V, int seg, int phase,
                  hipStream_t stream) {
  const int tiles = V.seg_rows / kTileRows * V.strips;
  hipLaunchKernelGGL((tb_tile_kernel<MODE, AFFINE, PROF>), dim3(tiles), dim3(64 * kTWaves), 0, stream, kp, q, s, V,
                     seg, phase);
}

template <int MODE>
void launch_rounds(const KParams& kp, const uint8_t* q, const uint8_t* s, const TbView& V, int nseg,
                   aln_result_t* out, uint32_t* cigar, int64_t cap, hipStream_t stream) {
  hipLaunchKernelGGL((tb_init_kernel<MODE>), dim3(1), dim3(64), 0, stream, out, V, cigar, cap);
  const bool bytes = kp.sigma_max - kp.ge <= 127 && kp.sigma_min - kp.ge >= -127;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    for (int phase = 0; phase < 2; ++phase) {
      {
        ProfScope prof("traceback_tiles", stream);
        if (kp.go != 0) {
          if (bytes && kp.alphabet <= 4)
            launch_tiles<MODE, true, kProfReg>(kp, q, s, V, seg, phase, stream);
          else
            launch_tiles<MODE, true, kProfTable>(kp, q, s, V, seg, phase, stream);
        } else {
          if (bytes && kp.alphabet <= 4)
            launch_tiles<MODE, false, kProfReg>(kp, q, s, V, seg, phase, stream);
          else
            launch_tiles<MODE, false, kProfTable>(kp, q, s, V, seg, phase, stream);
        }
      }
      ProfScope prof("traceback_walk", stream);
      hipLaunchKernelGGL((tb_walk_kernel<MODE>), dim3(1), dim3(64), 0, stream, V, seg, phase, cigar, cap);
    }
  }
  hipLaunchKernelGGL(tb_final_kernel, dim3(1), dim3(64), 0, stream, out, V, cigar, cap);
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Workspace of the linear-space traceback of an n x m pair, after the forward pass's:
//   [checkpoint columns][one segment's codes][walk state, error flag]
aln_status_t plan_long_ls(int64_t n, int64_t m, int64_t code_budget, LongLsPlan* pl) {
  pl->nb = (n + kWfBand - 1) / kWfBand;
  const int64_t groups = (pl->nb + kWfGroupBands - 1) / kWfGroupBands;
  const int nw = wf_waves(kWfWavesPerCUDefault);
  if (nw <= 0) return ALN_E_DEVICE;
  int64_t waves = nw;
  const int64_t want = groups * kWfGroupBands;
  if (want < waves) waves = want;
  if (waves < kWfGroupBands) waves = kWfGroupBands;
  pl->n_waves = (int)waves;
  // the forward pass keeps every group's bottom row in a slot of its own
  size_t off = wf_layout(1, pl->nb, groups * (m + 1), 0, &pl->off);
  pl->ck_ld = pl->nb * kWfBand;
  pl->strips = (int)((m + kTileCols - 1) / kTileCols);
  const int64_t ncols = pl->strips > 0 ? pl->strips - 1 : 0;
  pl->off_ckcols = off;
  off += a256((size_t)ncols * (size_t)pl->ck_ld * sizeof(int2));
  // rows per segment: as many tile rows as the code budget allows, at least one.  A segment's window
  // is about as wide as its rows, so shorter segments would relax fewer cells, but a tile takes its
  // 2048 steps whatever the number of tiles beside it: taller segments keep more tiles in flight per
  // launch (at 262144^2, segments of 8192 rows took 48.8 ms of tiles per traceback, of 32768 rows 20.1)
  const int64_t rows_all = groups * kTileRows;
  int64_t seg = m > 0 ? code_budget * 2 / m / kTileRows * kTileRows : rows_all;
  if (seg < kTileRows) seg = kTileRows;
  if (seg > rows_all) seg = rows_all > 0 ? rows_all : kTileRows;
  pl->seg_rows = seg;
  pl->nseg = (int)((n + seg - 1) / seg);
  pl->off_codes = off;
  off += a256((size_t)(seg / kWfR) * (size_t)m * sizeof(uint16_t));
  pl->off_walk = off;
  off += 256;
  pl->total_bytes = off;
  return ALN_OK;
}

aln_status_t launch_long_ls(const KParams& kp, const LongLsPlan& pl, const uint8_t* q, int64_t n, const uint8_t* s,
                            int64_t m, aln_result_t* out, uint32_t* cigar, int64_t cigar_cap, void* ws,
                            hipStream_t stream) {
  char* base = static_cast<char*>(ws);
  WfWs W = wf_view(ws, pl.off);
  W.ckcols = reinterpret_cast<int2*>(base + pl.off_ckcols);
  W.ck_ld = pl.ck_ld;
  launch_single_pair(W, (int)n, (int)m, stream);
  // the forward pass: score, end cell and the checkpoints (grouped bands)
  aln_status_t st = launch_wf_i32(kp, W, q, s, out, pl.n_waves, true, false, false, nullptr, 0, stream);
  if (st != ALN_OK) return st;
  TbView V;
  V.n = (int)n;
  V.m = (int)m;
  V.seg_rows = (int)pl.seg_rows;
  V.strips = pl.strips;
  V.ckrows = W.rows;
  V.ckcols = W.ckcols;
  V.ck_ld = pl.ck_ld;
  V.codes = reinterpret_cast<uint16_t*>(base + pl.off_codes);
  V.walk = reinterpret_cast<WalkState*>(base + pl.off_walk);
  V.error = reinterpret_cast<int*>(base + pl.off_walk + 128);
  V.win_lo = reinterpret_cast<int*>(base + pl.off_walk + 192);
  switch (kp.mode) {
    case ALN_GLOBAL:
      launch_rounds<ALN_GLOBAL>(kp, q, s, V, pl.nseg, out, cigar, cigar_cap, stream);
      break;
    case ALN_LOCAL:
      launch_rounds<ALN_LOCAL>(kp, q, s, V, pl.nseg, out, cigar, cigar_cap, stream);
      break;
    default:
      launch_rounds<ALN_SEMIGLOBAL>(kp, q, s, V, pl.nseg, out, cigar, cigar_cap, stream);
      break;
  }
  return hipGetLastError() == hipSuccess ? ALN_OK : ALN_E_DEVICE;
}

}  // namespace mialign
