// Inter-sequence batch kernel, 32-bit lanes.
//
// One lane aligns one pair (inter-sequence parallelism).  The lane relaxes its
// DP matrix in strips of R query rows held in registers, sweeping the subject
// column by column; the bottom row (H, E) of a strip is kept in a per-wave row
// buffer in the workspace, interleaved [column][lane] so the 64 lanes of a
// wave touch one contiguous 512-byte line per column.  This is the strip
// relaxation of AnySeq Sec. III-A (a strip needs its top row computed before
// and publishes its last row) applied per lane.
//
// With traceback, every cell also records the 4-bit predecessor code of
// walk.h (the NextStep.predc of Sec. III-B plus the two gap-extension bits of
// the affine model).
// The R codes of one column of a strip form one 32-bit word.  The same wave
// then walks each pair back from its optimum and writes the CIGAR.
#include "internal.h"
#include "walk.h"

namespace mialign {
namespace {

constexpr int R = 8;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = 64 * kWavesPerBlock;
constexpr int kWavesPerCU = 8;

// Persistent waves take groups of pairs from a device ticket; the groups come in the planner's
// order (largest shapes first), so the waves drain the list evenly whatever number of them is
// resident.
__device__ __forceinline__ int64_t next_group(int* ticket, int lane) {
  int g = 0;
  if (lane == 0) g = atomicAdd(ticket, 1);
  return (int64_t)__shfl(g, 0, 64);
}

// TBK: 0 score only; 1 traceback from the optimum; 2 traceback from the end cell a forward pass found
// (fwd[p].q_end, fwd[p].s_end): the pair is relaxed only up to that cell, whose H must equal fwd[p].score.
template <int MODE, bool AFFINE, int TBK>
__global__ __launch_bounds__(kBlock) void batch_i32_kernel(
    const KParams P, const uint8_t* __restrict__ q, const int64_t* __restrict__ q_off, const uint8_t* __restrict__ s,
    const int64_t* __restrict__ s_off, int64_t n_pairs, int64_t max_n, int64_t max_m, aln_result_t* __restrict__ out,
    uint32_t* __restrict__ cigar, const int64_t* __restrict__ cigar_off, char* __restrict__ ws, size_t slab_bytes,
    size_t letters_off, size_t dirs_off, const int* __restrict__ idx, const int* __restrict__ idx_count,
    uint32_t extra_flags,
    int* __restrict__ ticket, const aln_result_t* __restrict__ fwd) {
  constexpr bool TB = TBK != 0;
  constexpr bool FIXED = TBK == 2;
  __shared__ int32_t tab[kTab * kTab];
  for (int k = threadIdx.x; k < kTab * kTab; k += blockDim.x) {
    const int a = k / kTab, b = k % kTab;
    int32_t v;
    if (a >= P.alphabet || b >= P.alphabet)
      v = -kBig32;
    else
      v = P.use_table ? (int32_t)P.sig[a * kMaxAlphabet + b] : (a == b ? P.match : P.mismatch);
    tab[k] = v;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  char* slab = ws + wave * slab_bytes;
  int2* __restrict__ rowbuf = reinterpret_cast<int2*>(slab);
  // the subject letters of the wave's pairs as table indices, [column][lane], written once per group so
  // that every strip reads one coalesced row per column instead of a byte of 64 different subjects
  uint8_t* __restrict__ letters = reinterpret_cast<uint8_t*>(slab + letters_off);
  uint32_t* __restrict__ dirs = reinterpret_cast<uint32_t*>(slab + dirs_off);
  // pairs come in input order, or from an index list whose length is a device value
  const int64_t count = idx ? (int64_t)*idx_count : n_pairs;
  const int64_t groups = (count + 63) / 64;
  const int32_t go = P.go, ge = P.ge, goe = P.goe;

  for (int64_t g = next_group(ticket, lane); g < groups; g = next_group(ticket, lane)) {
    const int64_t slot = g * 64 + lane;
    const bool active = slot < count;
    const int64_t p = active ? (idx ? (int64_t)idx[slot] : slot) : 0;
    int64_t qb = 0, sb = 0;
    int n = 0, m = 0;
    uint32_t flags = 0;
    aln_result_t fw{};
    if (active) {
      qb = q_off[p];
      sb = s_off[p];
      const int64_t nn = q_off[p + 1] - qb, mm = s_off[p + 1] - sb;
      if (nn > max_n || mm > max_m || nn < 0 || mm < 0) {
        flags |= ALN_RES_TOO_LONG;
      } else {
        n = (int)nn;
        m = (int)mm;
      }
      if (FIXED) {
        // the forward pass's result: its failures carry over; otherwise only the rectangle up to its
        // end cell is relaxed (the values there are those of the whole matrix)
        fw = fwd[p];
        flags |= fw.flags & (ALN_RES_BAD_CODE | ALN_RES_TOO_LONG | ALN_RES_DEVICE_ERROR);
        if (!flags && (fw.q_end < 0 || fw.q_end > n || fw.s_end < 0 || fw.s_end > m)) flags |= ALN_RES_BAD_END;
        if (flags) {
          n = 0;
          m = 0;
        } else {
          n = fw.q_end;
          m = fw.s_end;
        }
      }
    }
    const int nmax = wave_max_i32(n), mmax = wave_max_i32(m);
    const int strips = (nmax + R - 1) / R;
    bool bad = false;
    // letters of columns 1..mmax (kPad past the subject's end), 8 columns per round so that the byte
    // loads of a round are in flight together
    for (int j0 = 1; j0 <= mmax; j0 += 8) {
      int lc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) lc[u] = j0 + u <= m ? (int)s[sb + j0 + u - 1] : kPad;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int c = lc[u];
        if (j0 + u <= m && c >= P.alphabet) {
          bad = true;
          c = kPad;
        }
        if (j0 + u <= mmax) letters[(size_t)(j0 + u - 1) * 64 + lane] = (uint8_t)c;
      }
    }

    // optimum bookkeeping
    int32_t best = 0;
    int bi = 0, bj = 0;
    if (MODE == ALN_SEMIGLOBAL) bj = m;   // first candidate in row-major order: (0, m)
    int32_t brow = 0;                     // semi: best of row n so far, starting at (n, 0)
    int browj = 0;
    int32_t hfinal = 0;                   // global: H(n, m)

    for (int k = 0; k < strips; ++k) {
      const int i0 = k * R;  // this strip holds rows i0+1 .. i0+R
      int qcb[R];
      int32_t hl[R], f[R], bv[R], cap[R];
      int bjr[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = i0 + 1 + r;
        int c = kPad;
        if (i <= n) {
          c = q[qb + i - 1];
          if (c >= P.alphabet) {
            bad = true;
            c = kPad;
          }
        }
        qcb[r] = c * kTab;
        hl[r] = (MODE == ALN_GLOBAL) ? go + i * ge : 0;
        f[r] = kNeg32;
        bv[r] = kNeg32;
        bjr[r] = 0;
        cap[r] = 0;
      }
      int32_t hdiag = (MODE == ALN_GLOBAL && i0 > 0) ? go + i0 * ge : 0;  // H(i0, 0)
      const bool has_n = (i0 < n) && (n <= i0 + R);
      const int rn = n - 1 - i0;
      for (int j = 1; j <= mmax; ++j) {
        const int c = letters[(size_t)(j - 1) * 64 + lane];
        int32_t hup, eup;
        if (k == 0) {
          hup = (MODE == ALN_GLOBAL) ? go + j * ge : 0;
          eup = kNeg32;
        } else {
          const int2 v = rowbuf[(size_t)j * 64 + lane];
          hup = v.x;
          eup = v.y;
        }
        int32_t hd = hdiag;
        hdiag = hup;
        uint32_t word = 0;
        int32_t hn = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int32_t hlo = hl[r];
          const int32_t e = AFFINE ? max(eup + ge, hup + goe) : hup + ge;
          const int32_t ff = AFFINE ? max(f[r] + ge, hlo + goe) : hlo + ge;
          const int32_t d = hd + tab[qcb[r] + c];
          int32_t h = max(d, max(e, ff));
          if (MODE == ALN_LOCAL) h = max(h, 0);
          if (TB) {
            uint32_t src;
            if (MODE == ALN_LOCAL && h == 0)
              src = 3u;
            else if (d == h)
              src = 0u;
            else if (e == h)
              src = 1u;
            else
              src = 2u;
            const uint32_t ee = AFFINE ? (uint32_t)(hup + goe != e) : 0u;
            const uint32_t fe = AFFINE ? (uint32_t)(hlo + goe != ff) : 0u;
            word |= (src | (ee << 2) | (fe << 3)) << (4 * r);
          }
          if (MODE == ALN_LOCAL && !FIXED) {
            if (h > bv[r]) {
              bv[r] = h;
              bjr[r] = j;
            }
          } else {
            if (j == m) cap[r] = h;
            if (MODE == ALN_SEMIGLOBAL && !FIXED && r == rn) hn = h;
          }
          f[r] = ff;
          hl[r] = h;
          hd = hlo;
          hup = h;
          eup = e;
        }
        if (k + 1 < strips) rowbuf[(size_t)j * 64 + lane] = make_int2(hup, eup);
        if (TB) dirs[((size_t)k * (size_t)max_m + (size_t)(j - 1)) * 64 + lane] = word;
        if (MODE == ALN_SEMIGLOBAL && !FIXED && has_n && j <= m && hn > brow) {
          brow = hn;
          browj = j;
        }
      }
      // merge this strip's rows into the optimum, in row order
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = i0 + 1 + r;
        if (FIXED) {
          if (i == n) hfinal = cap[r];
        } else if (MODE == ALN_LOCAL) {
          if (bv[r] > best) {
            best = bv[r];
            bi = i;
            bj = bjr[r];
          }
        } else if (MODE == ALN_SEMIGLOBAL) {
          if (i < n && cap[r] > best) {
            best = cap[r];
            bi = i;
            bj = m;
          }
        } else {
          if (i == n) hfinal = cap[r];
        }
      }
    }

    if (FIXED) {
      // H at the given end cell; on row 0 or column 0 it is the mode's border value
      bi = n;
      bj = m;
      if (n == 0 || m == 0)
        best = (MODE == ALN_GLOBAL && n + m > 0) ? go + (n + m) * ge : 0;
      else
        best = hfinal;
      if (active && !flags && best != fw.score) flags |= ALN_RES_BAD_END;
    } else if (MODE == ALN_SEMIGLOBAL) {
      if (n == 0 || m == 0) {
        best = 0;
        bi = 0;
        bj = 0;
      } else if (brow > best) {
        best = brow;
        bi = n;
        bj = browj;
      }
    } else if (MODE == ALN_GLOBAL) {
      bi = n;
      bj = m;
      if (n == 0 || m == 0)
        best = (n + m > 0) ? go + (n + m) * ge : 0;
      else
        best = hfinal;
    }

    if (!active) continue;
    aln_result_t res;
    res.score = best;
    res.q_begin = -1;
    res.q_end = bi;
    res.s_begin = -1;
    res.s_end = bj;
    res.cigar_len = 0;
    res.reserved = 0;
    if (bad) flags |= ALN_RES_BAD_CODE;
    if (flags) {
      res.score = 0;
      res.q_end = 0;
      res.s_end = 0;
    } else if (TB) {
      const int64_t c0 = cigar_off[p];
      const int64_t capw = cigar_off[p + 1] - c0;
      int qbeg, sbeg, runs;
      auto code = [&](int ii, int jj) -> uint32_t {
        const uint32_t w = dirs[((size_t)((ii - 1) / R) * (size_t)max_m + (size_t)(jj - 1)) * 64 + lane];
        return (w >> (4 * ((ii - 1) % R))) & 15u;
      };
      walk_back<MODE>(code, bi, bj, cigar + c0, capw, &qbeg, &sbeg, &runs);
      res.q_begin = qbeg;
      res.s_begin = sbeg;
      res.cigar_len = runs;
      if (runs > capw) flags |= ALN_RES_CIGAR_TRUNC;
    }
    res.flags = flags | extra_flags;
    out[p] = res;
  }
}

template <int MODE, bool AFFINE, int TBK>
void launch_one(const KParams& kp, const BatchPlan& pl, const uint8_t* q, const int64_t* q_off, const uint8_t* s,
                const int64_t* s_off, aln_result_t* out, uint32_t* cigar, const int64_t* cigar_off, void* ws,
                const int* idx, const int* idx_count, uint32_t extra_flags, int* ticket, const aln_result_t* fwd,
                hipStream_t stream) {
  const size_t slab = pl.rowbuf_bytes + pl.letters_bytes + pl.dirs_bytes;
  const int blocks = (pl.n_waves + kWavesPerBlock - 1) / kWavesPerBlock;
  ProfScope prof(TBK == 2 ? "batch_i32_traceback_from_end" : (TBK ? "batch_i32_traceback" : "batch_i32_score"),
                 stream);
  hipLaunchKernelGGL((batch_i32_kernel<MODE, AFFINE, TBK>), dim3(blocks), dim3(kBlock), 0, stream, kp, q, q_off, s,
                     s_off, pl.n_pairs, pl.max_n, pl.max_m, out, cigar, cigar_off, static_cast<char*>(ws), slab,
                     pl.rowbuf_bytes, pl.rowbuf_bytes + pl.letters_bytes, idx, idx_count, extra_flags, ticket, fwd);
}

template <int MODE, bool AFFINE>
void launch_tb(const KParams& kp, const BatchPlan& pl, const uint8_t* q, const int64_t* q_off, const uint8_t* s,
               const int64_t* s_off, bool tb, aln_result_t* out, uint32_t* cigar, const int64_t* cigar_off, void* ws,
               const int* idx, const int* idx_count, uint32_t extra_flags, int* ticket, const aln_result_t* fwd,
               hipStream_t stream) {
  if (fwd)
    launch_one<MODE, AFFINE, 2>(kp, pl, q, q_off, s, s_off, out, cigar, cigar_off, ws, idx, idx_count, extra_flags,
                                ticket, fwd, stream);
  else if (tb)
    launch_one<MODE, AFFINE, 1>(kp, pl, q, q_off, s, s_off, out, cigar, cigar_off, ws, idx, idx_count, extra_flags,
                                ticket, nullptr, stream);
  else
    launch_one<MODE, AFFINE, 0>(kp, pl, q, q_off, s, s_off, out, cigar, cigar_off, ws, idx, idx_count, extra_flags,
                                ticket, nullptr, stream);
}

template <int MODE>
void launch_mode(const KParams& kp, const BatchPlan& pl, const uint8_t* q, const int64_t* q_off, const uint8_t* s,
                 const int64_t* s_off, bool tb, aln_result_t* out, uint32_t* cigar, const int64_t* cigar_off,
                 void* ws, const int* idx, const int* idx_count, uint32_t extra_flags, int* ticket,
                 const aln_result_t* fwd, hipStream_t stream) {
  if (kp.go != 0)
    launch_tb<MODE, true>(kp, pl, q, q_off, s, s_off, tb, out, cigar, cigar_off, ws, idx, idx_count, extra_flags,
                          ticket, fwd, stream);
  else
    launch_tb<MODE, false>(kp, pl, q, q_off, s, s_off, tb, out, cigar, cigar_off, ws, idx, idx_count, extra_flags,
                           ticket, fwd, stream);
}

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

aln_status_t plan_batch_i32(const KParams& kp, int64_t n_pairs, int64_t max_n, int64_t max_m, bool traceback,
                            BatchPlan* plan) {
  (void)kp;
  BatchPlan pl{};
  pl.n_pairs = n_pairs;
  pl.max_n = max_n;
  pl.max_m = max_m;
  pl.strips = (int32_t)((max_n + R - 1) / R);
  const int64_t groups = (n_pairs + 63) / 64;
  const int cus = device_cu_count();
  if (cus <= 0) return ALN_E_DEVICE;
  int64_t waves = (int64_t)cus * kWavesPerCU;
  if (groups < waves) waves = groups;
  if (waves < 1) waves = 1;
  waves = (waves + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock;  // every launched wave owns a slab
  pl.n_waves = (int32_t)waves;
  pl.rowbuf_bytes = round256((size_t)(max_m + 1) * 64 * sizeof(int2));
  pl.letters_bytes = round256((size_t)(max_m + 1) * 64);
  pl.dirs_bytes = traceback ? round256((size_t)pl.strips * (size_t)max_m * 64 * sizeof(uint32_t)) : 0;
  if (traceback) {
    // fewer waves in flight when every wave's codes would exceed the budget (at least one workgroup)
    const int64_t slab = (int64_t)(pl.rowbuf_bytes + pl.letters_bytes + pl.dirs_bytes);
    const int64_t fit = kTbSlabBudget / slab / kWavesPerBlock * kWavesPerBlock;
    if (fit < waves) pl.n_waves = (int32_t)(fit > kWavesPerBlock ? fit : kWavesPerBlock);
  }
  pl.total_bytes = (size_t)pl.n_waves * (pl.rowbuf_bytes + pl.letters_bytes + pl.dirs_bytes);
  *plan = pl;
  return ALN_OK;
}

aln_status_t launch_batch_i32(const KParams& kp, const BatchPlan& pl, const uint8_t* q, const int64_t* q_off,
                              const uint8_t* s, const int64_t* s_off, bool tb, aln_result_t* out, uint32_t* cigar,
                              const int64_t* cigar_off, void* ws, const int* idx, const int* idx_count,
                              uint32_t extra_flags, int* ticket, hipStream_t stream, const aln_result_t* fwd) {
  if (pl.n_pairs == 0) return ALN_OK;
  switch (kp.mode) {
    case ALN_GLOBAL:
      launch_mode<ALN_GLOBAL>(kp, pl, q, q_off, s, s_off, tb, out, cigar, cigar_off, ws, idx, idx_count, extra_flags,
                              ticket, fwd, stream);
      break;
    case ALN_LOCAL:
      launch_mode<ALN_LOCAL>(kp, pl, q, q_off, s, s_off, tb, out, cigar, cigar_off, ws, idx, idx_count, extra_flags,
                             ticket, fwd, stream);
      break;
    default:
      launch_mode<ALN_SEMIGLOBAL>(kp, pl, q, q_off, s, s_off, tb, out, cigar, cigar_off, ws, idx, idx_count,
                                  extra_flags, ticket, fwd, stream);
      break;
  }
  return hipGetLastError() == hipSuccess ? ALN_OK : ALN_E_DEVICE;
}

}  // namespace mialign
