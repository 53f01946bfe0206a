// The cell recurrence of the band wavefronts (the grouped and per-band engines of wf_i32.hip and the
// traceback tiles of tb_tiles.hip): one column of a lane's rows.
#pragma once
#include "internal.h"

namespace mialign {

// Where a band's substitution scores sigma(row letter, column letter) - ge come from:
//   kProfTable  a 32-bit LDS table indexed by both letters (any score range);
//   kProfReg    alphabets of up to 4 letters: one register per row holds the scores of the row's
//               letter against the 4 letters as signed bytes, picked with a bit-field extract;
//   kProfLane   alphabets of up to 32 letters: per letter, every lane keeps the scores of its
//               R = 4 rows as 4 signed bytes in one LDS word, so a step reads one word.
// The byte forms need every sigma - ge in -127..127 (-128 marks rows past the end).
constexpr int kProfTable = 0, kProfReg = 1, kProfLane = 2;

// The R cells of one column of a lane's rows: Eqs. (1), (4), (5) with the row bias Hb = H - i*ge (likewise
// E and F), shared by both wavefront engines.  On entry hup and eup are the Hb and Eb of the row above the
// lane's first row, hd that row's Hb one column left; on return hup and eup hold the lane's last row.
// With TRACK, local alignments track each row's best cell (CHECKED: cell by cell) or hand the H values to
// the caller's 4-step tracking (hk), and semi-global bands report row n's H (rn: its index among the lane's
// rows); with TB the 4-bit codes of walk.h are packed into word.
// FLOOR_E (local affine, score-only): E is taken as max(E above, H above + go, the row's floor), one v_max3,
// so that H's max has three terms instead of four.  H is unchanged: the floor is one of its terms anyway, and an E raised
// to row i's floor stays below the floor of every row beneath it (the row bias raises the floor by |ge|
// per row and E's extension keeps its value).  Only E differs, so kernels that store predecessor codes or
// rows of E do not use it.
template <int MODE, bool AFFINE, int PROF, bool TB, bool CHECKED, int R, bool TRACK = true, bool FLOOR_E = false>
__device__ __forceinline__ void band_column(const int32_t* tab, const int (&prof)[R], int in_c, int pw,
                                            int32_t go, int32_t ge, int32_t goe, const int32_t (&nu)[R],
                                            int32_t (&hl)[R], int32_t (&f)[R], int32_t (&bv)[R], int (&bj)[R],
                                            int32_t* hk, int j, int rn, int32_t hd, int32_t& hup, int32_t& eup,
                                            int32_t& hn, uint32_t& word) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    static_assert(!FLOOR_E || (MODE == ALN_LOCAL && AFFINE && !TB), "the E floor: local affine, score-only");
    const int32_t hlo = hl[r];
    const int32_t e = FLOOR_E ? max(max(eup, hup + go), nu[r]) : (AFFINE ? max(eup, hup + go) : hup);
    const int32_t ff = AFFINE ? max(f[r] + ge, hlo + goe) : hlo + ge;
    const int32_t sg = PROF == kProfReg    ? __builtin_amdgcn_sbfe(prof[r], in_c, 8)
                       : PROF == kProfLane ? __builtin_amdgcn_sbfe(pw, 8 * r, 8)
                                           : tab[prof[r] + in_c];
    const int32_t d = hd + sg;
    int32_t h = max(d, max(e, ff));
    if (MODE == ALN_LOCAL && !FLOOR_E) h = max(h, nu[r]);
    if (TB) {
      uint32_t src = (d == h) ? 0u : ((e == h) ? 1u : 2u);
      if (MODE == ALN_LOCAL && h == nu[r]) src = 3u;
      const uint32_t xe = AFFINE ? (uint32_t)(hup + go != e) : 0u;
      const uint32_t xf = AFFINE ? (uint32_t)(hlo + goe != ff) : 0u;
      word |= (src | (xe << 2) | (xf << 3)) << (4 * r);
    }
    if (MODE == ALN_LOCAL && TRACK) {
      if (CHECKED) {
        if (h > bv[r]) {
          bv[r] = h;
          bj[r] = j;
        }
      } else {
        hk[r] = h;
      }
    }
    if (MODE == ALN_SEMIGLOBAL && TRACK && r == rn) hn = h;
    f[r] = ff;
    hl[r] = h;
    hd = hlo;
    hup = h;
    eup = e;
  }
}

}  // namespace mialign
