// Inter-sequence batch kernel, packed 16-bit lanes: two pairs per lane.
//
// Lane l of a wave carries pair slot l in the low halves and slot 64+l in the
// high halves of every register, so one v_pk_* instruction relaxes a cell of
// two independent pairs (the inter-task vectorisation of AnySeq Sec. IV-A with
// 16-bit scores, Sec. V).  Each lane walks its two matrices in strips of R
// query rows.  The substitution scores of a strip come from a query profile in
// LDS -- for every letter c, the R scores sigma(q_i, c) as int16 -- so one
// 16-byte LDS read per pair and column delivers eight rows, and one v_perm
// merges the two pairs' scores of a row.
//
// All arithmetic saturates, so -infinity is -32768 and never wraps.  Exactness:
// a global or semi-global pair keeps its 16-bit result only when its score
// range provably fits (every value lies in [3*go + (n+m)*ge,
// min(n,m)*max(sigma_max,0)], the 16-bit bound of Sec. IV-A made explicit);
// otherwise it goes to a redo list that the 32-bit kernel recomputes exactly.
// A local pair keeps its result whenever its best score stayed below 32767,
// whatever the bound says: every H is then below 32767 and at least 0, so no H
// saturated, and a value clamped at -32768 (an E or F far below 0) loses every
// maximum it enters, as its true value would.  A local pair that reached 32767
// may have saturated and is redone.
#include "internal.h"
#include "walk.h"

namespace mialign {
namespace {

typedef short s2 __attribute__((ext_vector_type(2)));
typedef unsigned short u2 __attribute__((ext_vector_type(2)));

constexpr int kI16WavesPerBlock = 2;
constexpr int kI16Block = 64 * kI16WavesPerBlock;
constexpr int kI16WavesPerCU = 8;
constexpr int kPadSigma16 = -16384;
constexpr int kBound16 = 32000;

__device__ __forceinline__ s2 adds(s2 a, s2 b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ s2 subs(s2 a, s2 b) { return __builtin_elementwise_sub_sat(a, b); }
__device__ __forceinline__ s2 mx(s2 a, s2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ s2 mn(s2 a, s2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ s2 sp(int v) {
  s2 r = {(short)v, (short)v};
  return r;
}
__device__ __forceinline__ s2 pk(int lo, int hi) {
  s2 r = {(short)lo, (short)hi};
  return r;
}
__device__ __forceinline__ uint32_t bits(s2 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ s2 from_bits(uint32_t x) { return __builtin_bit_cast(s2, x); }
__device__ __forceinline__ int lo16(s2 x) { return (int)x.x; }
__device__ __forceinline__ int hi16(s2 x) { return (int)x.y; }
// a * b + c on unsigned halves (small non-negative values)
__device__ __forceinline__ s2 mad_u(s2 a, s2 b, s2 c) {
  const u2 r = __builtin_bit_cast(u2, a) * __builtin_bit_cast(u2, b) + __builtin_bit_cast(u2, c);
  return __builtin_bit_cast(s2, r);
}
// The same as one v_pk_mad_u16 where b is a constant: the compiler would otherwise turn a power-of-two
// b into a shift and an add.
__device__ __forceinline__ s2 mad_u1(s2 a, s2 b, s2 c) {
  uint32_t r;
  asm("v_pk_mad_u16 %0, %1, %2, %3" : "=v"(r) : "v"(bits(a)), "v"(bits(b)), "v"(bits(c)));
  return from_bits(r);
}
// Per 16-bit half, x[k] with k given by its bits: kb[b] holds 0xffff in the half whose index has bit b
// set.  A tree of N - 1 bit-field inserts (v_bfi_b32) picks both halves' entries at once, instead of a
// compare and a select per entry and half.
template <int N>
__device__ __forceinline__ uint32_t tree_pick(const uint32_t* x, const uint32_t* kb) {
  static_assert(N == 4 || N == 8 || N == 16, "row counts of the 16-bit kernel");
  uint32_t t[N / 2];
#pragma unroll
  for (int q = 0; q < N / 2; ++q) t[q] = (x[2 * q + 1] & kb[0]) | (x[2 * q] & ~kb[0]);
#pragma unroll
  for (int lvl = 1, w = N / 2; w > 1; ++lvl, w /= 2) {
#pragma unroll
    for (int q = 0; q < w / 2; ++q) t[q] = (t[2 * q + 1] & kb[lvl]) | (t[2 * q] & ~kb[lvl]);
  }
  return t[0];
}

// LDS query profile of one wave, in 32-bit words.  For letter c, the R scores of a pair slot are
// W = R/2 words, cut into chunks of CW words (one ds_read_b128, or b64 when R = 4); chunk k of every
// slot of a letter lies in one block, [letter][chunk][slot][CW words].  Each letter block spans a
// whole number of 64-word bank sweeps, so the chunk a lane reads sits in the same banks whatever
// letter it reads, and the lanes of a read cover the banks once: no bank conflicts.  After the AP
// letter blocks comes one pad row (the W words of kPadSigma16 pairs that every slot reads past its
// subject's end, the same address for all lanes), padded to a bank sweep.  The profiles start at a
// 256-byte boundary after the substitution table.
constexpr int kI16ProfBase = (kTab * kTab * 4 + 255) & ~255;
__host__ __device__ constexpr int i16_chunk_words(int R) { return R / 2 < 4 ? R / 2 : 4; }
__host__ __device__ constexpr int i16_wave_prof_words(int AP, int R) { return AP * 128 * (R / 2) + 64; }
static_assert(kI16ProfBase % 256 == 0, "profiles start on a bank sweep");

// biased: values carry the row bias of the global and semi-global recurrence (Hb = H - i*ge), which
// lifts them by at most n*|ge|
__device__ __forceinline__ bool fits16(const KParams& P, int n, int m, bool biased) {
  const int mn = n < m ? n : m;
  const long long up = (long long)mn * (P.sigma_max > 0 ? P.sigma_max : 0) - (biased ? (long long)n * P.ge : 0);
  const long long lo = 3ll * P.go + (long long)(n + m) * P.ge;
  return up <= kBound16 && lo >= -kBound16 && m < 32767;
}

// Persistent waves take groups of pairs from a device ticket; the groups come in the planner's
// order (largest shapes first), so the waves drain the list evenly whatever number of them is
// resident.
__device__ __forceinline__ int64_t next_group(int* ticket, int lane) {
  int g = 0;
  if (lane == 0) g = atomicAdd(ticket, 1);
  return (int64_t)__shfl(g, 0, 64);
}

template <int MODE, bool AFFINE, bool TB, int R>
__global__ __launch_bounds__(kI16Block) void batch_i16_kernel(
    const KParams P, const uint8_t* __restrict__ q, const int64_t* __restrict__ q_off, const uint8_t* __restrict__ s,
    const int64_t* __restrict__ s_off, int64_t n_pairs, int64_t max_n, int64_t max_m, aln_result_t* __restrict__ out,
    uint32_t* __restrict__ cigar, const int64_t* __restrict__ cigar_off, char* __restrict__ ws, size_t slab_bytes,
    size_t letters_off, size_t dirs_off, const int* __restrict__ idx, const int* __restrict__ idx_count,
    int* __restrict__ redo_idx, int* __restrict__ redo_cnt, int* __restrict__ ticket) {
  static_assert(R % 8 == 0 || R == 4, "R must be 4 or a multiple of 8");
  // Global and semi-global pairs keep their values with a row bias, Hb(i, j) = H(i, j) - i*ge (and so
  // E and F): then Eb(i, j) = max(Eb(i-1, j), Hb(i-1, j) + go) extends a vertical gap with no add,
  // Hb(i, j) = max(Hb(i-1, j-1) + sigma - ge, Eb, Fb), and Fb is unchanged -- Eqs. (1), (4), (5) with
  // every term of row i shifted by the same constant.  Local pairs, whose floor H = 0 would become a
  // per-row constant, keep plain values.
  constexpr bool kBias = MODE != ALN_LOCAL;
  extern __shared__ char smem[];
  int32_t* tab = reinterpret_cast<int32_t*>(smem);
  for (int k = threadIdx.x; k < kTab * kTab; k += blockDim.x) {
    const int a = k / kTab, b = k % kTab;
    int32_t v;
    if (a >= P.alphabet || b >= P.alphabet)
      v = kPadSigma16;
    else
      v = (P.use_table ? (int32_t)P.sig[a * kMaxAlphabet + b] : (a == b ? P.match : P.mismatch)) -
          (kBias ? P.ge : 0);
    tab[k] = v;
  }
  __syncthreads();
  const int AP = P.alphabet;  // profile letters per pair; past a subject's end, the shared pad row
  constexpr int W = R / 2, CW = i16_chunk_words(R), NCH = W / CW, SCH = 128 * CW;
  const int SC = 128 * W;  // words per letter block
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  uint32_t* __restrict__ profw =
      reinterpret_cast<uint32_t*>(smem + kI16ProfBase) + (size_t)wib * i16_wave_prof_words(AP, R);
  uint32_t* __restrict__ padw = profw + (size_t)AP * SC;
  if (lane < W) padw[lane] = (0xffffu & (uint32_t)kPadSigma16) | ((uint32_t)kPadSigma16 << 16);  // read by this wave only

  const int64_t wave = (int64_t)blockIdx.x * kI16WavesPerBlock + wib;
  char* slab = ws + wave * slab_bytes;
  uint2* __restrict__ rowbuf = reinterpret_cast<uint2*>(slab);
  // the subject letters of the wave's pairs, [column][lane] with pair A's profile index in the low byte
  // and pair B's in the high one, written once per group: every strip then reads one coalesced row per
  // column instead of a byte of 128 different subjects
  uint16_t* __restrict__ letters = reinterpret_cast<uint16_t*>(slab + letters_off);
  uint32_t* __restrict__ dirs = reinterpret_cast<uint32_t*>(slab + dirs_off);
  constexpr int RW = (R + 3) / 4;  // direction words per column (4 rows x 2 pairs per word)
  // Global and semi-global traceback with 8 or 16 rows per strip store the codes as flags: for each
  // group of 8 rows a pair of words, the first with "not diagonal" and "not E" and the second with
  // "E extended" and "F extended", one byte per (flag, pair), bit b for row b of the group.  A flag is
  // the sign of a packed difference, spread to a byte mask by v_perm's sign selectors and merged with
  // one and-or: 8 operations per row and step instead of 10.  Same words per column as the nibbles.
  constexpr bool kFlagCodes = TB && MODE != ALN_LOCAL && R % 8 == 0;
  const int64_t count = idx ? (int64_t)*idx_count : n_pairs;
  const int64_t groups = (count + 127) / 128;
  const s2 ge2 = sp(P.ge), goe2 = sp(P.goe), go2 = sp(P.go), one = sp(1), zero = sp(0);
  const s2 neg2 = sp(-32768);

  for (int64_t g = next_group(ticket, lane); g < groups; g = next_group(ticket, lane)) {
    int64_t pp[2];
    int nn[2], mm[2];
    bool act[2], ok16[2], bad[2];
    int64_t qb[2], sb[2];
    uint32_t flg[2];
    for (int h = 0; h < 2; ++h) {
      const int64_t slot = g * 128 + h * 64 + lane;
      act[h] = slot < count;
      pp[h] = act[h] ? (idx ? (int64_t)idx[slot] : slot) : 0;
      nn[h] = 0;
      mm[h] = 0;
      qb[h] = 0;
      sb[h] = 0;
      flg[h] = 0;
      bad[h] = false;
      ok16[h] = true;
      if (act[h]) {
        qb[h] = q_off[pp[h]];
        sb[h] = s_off[pp[h]];
        const int64_t a = q_off[pp[h] + 1] - qb[h], b = s_off[pp[h] + 1] - sb[h];
        if (a > max_n || b > max_m || a < 0 || b < 0) {
          flg[h] = ALN_RES_TOO_LONG;
        } else {
          nn[h] = (int)a;
          mm[h] = (int)b;
          const bool f = fits16(P, nn[h], mm[h], kBias);
          ok16[h] = f || (MODE == ALN_LOCAL && mm[h] < 32767);
        }
      }
    }
    const int nmax = wave_max_i32(max(nn[0], nn[1])), mmax = wave_max_i32(max(mm[0], mm[1]));
    const int strips = (nmax + R - 1) / R;
    // Letters of columns 1..mmax (the pad letter P.alphabet past a subject's end), 8 columns per round
    // so that the byte loads of a round are in flight together.
    for (int j0 = 1; j0 <= mmax; j0 += 8) {
      int la[8], lb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + u;
        la[u] = j <= mm[0] ? (int)s[sb[0] + j - 1] : -1;
        lb[u] = j <= mm[1] ? (int)s[sb[1] + j - 1] : -1;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int ca = P.alphabet, cb = P.alphabet;
        if (la[u] >= 0) {
          if (la[u] < P.alphabet)
            ca = la[u];
          else
            bad[0] = true;
        }
        if (lb[u] >= 0) {
          if (lb[u] < P.alphabet)
            cb = lb[u];
          else
            bad[1] = true;
        }
        if (j0 + u <= mmax) letters[(size_t)(j0 + u - 1) * 64 + lane] = (uint16_t)(ca | (cb << 8));
      }
    }

    // optimum bookkeeping per pair (scalars)
    int best[2] = {0, 0}, bi[2] = {0, 0}, bj[2] = {0, 0};
    if (MODE == ALN_SEMIGLOBAL) {
      bj[0] = mm[0];
      bj[1] = mm[1];
    }
    int brow[2] = {0, 0}, browj[2] = {0, 0}, hfin[2] = {0, 0};

    for (int k = 0; k < strips; ++k) {
      const int i0 = k * R;
      // query profile of this strip for both pairs: row r of letter c is sigma(q_{i0+r+1}, c)
      for (int h = 0; h < 2; ++h) {
        uint32_t* pr = profw + (size_t)(h * 64 + lane) * CW;
        int qc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = i0 + 1 + r;
          int c = kPad;
          if (i <= nn[h]) {
            c = q[qb[h] + i - 1];
            if (c >= P.alphabet) {
              bad[h] = true;
              c = kPad;
            }
          }
          qc[r] = c * kTab;
        }
        for (int c = 0; c < AP; ++c) {
          const int cc = c < P.alphabet ? c : kPad;
          uint32_t w[W];
#pragma unroll
          for (int r = 0; r < R; r += 2)
            w[r / 2] = (uint32_t)(tab[qc[r] + cc] & 0xffff) | ((uint32_t)tab[qc[r + 1] + cc] << 16);
          uint32_t* dst = pr + (size_t)c * SC;
#pragma unroll
          for (int k = 0; k < NCH; ++k) {
            if constexpr (CW == 4)
              *reinterpret_cast<uint4*>(dst + k * SCH) = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
            else
              *reinterpret_cast<uint2*>(dst + k * SCH) = make_uint2(w[2 * k], w[2 * k + 1]);
          }
        }
      }
      s2 hl[R], f[R], bv[R], bjr[R], cap[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = i0 + 1 + r;
        hl[r] = sp((MODE == ALN_GLOBAL) ? P.go + (kBias ? 0 : i * P.ge) : (kBias ? -i * P.ge : 0));
        f[r] = neg2;
        bv[r] = sp(-32768);
        bjr[r] = zero;
        cap[r] = zero;
      }
      // H(i0, 0), with the row bias where it applies
      s2 hdiag = sp((MODE == ALN_GLOBAL && i0 > 0) ? P.go + (kBias ? 0 : i0 * P.ge) : (kBias ? -i0 * P.ge : 0));
      const int rnA = nn[0] - 1 - i0, rnB = nn[1] - 1 - i0;
      const bool lastA = rnA >= 0 && rnA < R, lastB = rnB >= 0 && rnB < R;
      const bool track_last = (MODE == ALN_SEMIGLOBAL) && __any(lastA || lastB);
      // bits of row n's index in this strip, pair A's in the low half and pair B's in the high half
      constexpr int kRB = R == 16 ? 4 : (R == 8 ? 3 : 2);
      uint32_t rnb[kRB];
#pragma unroll
      for (int b = 0; b < kRB; ++b)
        rnb[b] = (((rnA >> b) & 1) ? 0x0000ffffu : 0u) | (((rnB >> b) & 1) ? 0xffff0000u : 0u);
      // Letters and top-row inputs of column j (the pad letter of the profile past a subject's end).
      auto fetch = [&](int j, int& ca, int& cb, uint2& top) {
        const uint32_t l2 = j <= mmax ? (uint32_t)letters[(size_t)(j - 1) * 64 + lane] : 0u;
        ca = j <= mmax ? (int)(l2 & 0xffu) : P.alphabet;
        cb = j <= mmax ? (int)(l2 >> 8) : P.alphabet;
        if (k == 0)
          top = make_uint2(bits(sp((MODE == ALN_GLOBAL) ? P.go + j * P.ge : 0)), bits(neg2));
        else
          top = (j <= mmax) ? rowbuf[(size_t)j * 64 + lane] : make_uint2(0u, 0u);
      };
      // One column of the strip for both pairs.
      auto column = [&](int j, int ca, int cb, uint2 top) {
        s2 hup = from_bits(top.x), eup = from_bits(top.y);
        s2 hd = hdiag;
        hdiag = hup;
        // chunk k of a slot's letter is SCH words after chunk k-1; the pad row's chunks are adjacent
        const uint32_t* pa = ca < AP ? profw + (size_t)ca * SC + (size_t)lane * CW : padw;
        const uint32_t* pb = cb < AP ? profw + (size_t)cb * SC + (size_t)(64 + lane) * CW : padw;
        const int sa = ca < AP ? SCH : CW, sb2 = cb < AP ? SCH : CW;
        uint32_t wa[W], wb[W];
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
          if constexpr (CW == 4) {
            const uint4 va = *reinterpret_cast<const uint4*>(pa + k * sa);
            const uint4 vb = *reinterpret_cast<const uint4*>(pb + k * sb2);
            wa[4 * k] = va.x, wa[4 * k + 1] = va.y, wa[4 * k + 2] = va.z, wa[4 * k + 3] = va.w;
            wb[4 * k] = vb.x, wb[4 * k + 1] = vb.y, wb[4 * k + 2] = vb.z, wb[4 * k + 3] = vb.w;
          } else {
            const uint2 va = *reinterpret_cast<const uint2*>(pa + k * sa);
            const uint2 vb = *reinterpret_cast<const uint2*>(pb + k * sb2);
            wa[2 * k] = va.x, wa[2 * k + 1] = va.y;
            wb[2 * k] = vb.x, wb[2 * k + 1] = vb.y;
          }
        }
        uint32_t acc[RW];
#pragma unroll
        for (int w = 0; w < RW; ++w) acc[w] = 0;
        const s2 jj = sp(j);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const s2 sg = from_bits(__builtin_amdgcn_perm(wb[r / 2], wa[r / 2], (r & 1) ? 0x07060302u : 0x05040100u));
          const s2 hlo = hl[r];
          const s2 d = adds(hd, sg);
          const s2 tup = adds(hup, kBias ? go2 : goe2);
          const s2 e = AFFINE ? mx(kBias ? eup : adds(eup, ge2), tup) : (kBias ? hup : adds(hup, ge2));
          const s2 tle = adds(hlo, goe2);
          const s2 ff = AFFINE ? mx(adds(f[r], ge2), tle) : adds(hlo, ge2);
          s2 hv = mx(mx(d, e), ff);
          if (MODE == ALN_LOCAL) hv = mx(hv, zero);
          if (kFlagCodes) {
            // words 2g and 2g + 1 of the column hold row group g; byte order (pair A, pair B) per flag
            const uint32_t bit = 0x01010101u << (r & 7);
            const uint32_t nd_ne = __builtin_amdgcn_perm(bits(subs(e, hv)), bits(subs(d, hv)), 0x0b0a0908u);
            acc[2 * (r >> 3)] = (nd_ne & bit) | acc[2 * (r >> 3)];
            if (AFFINE) {
              const uint32_t xe_xf = __builtin_amdgcn_perm(bits(subs(tle, ff)), bits(subs(tup, e)), 0x0b0a0908u);
              acc[2 * (r >> 3) + 1] = (xe_xf & bit) | acc[2 * (r >> 3) + 1];
            }
          } else if (TB) {
            const s2 bd = mn(subs(hv, d), one);
            const s2 be = mn(subs(hv, e), one);
            s2 hs = mad_u(bd, be, bd);
            if (MODE == ALN_LOCAL) hs = mx(hs, mad_u(subs(one, mn(hv, one)), sp(3), zero));
            s2 nib = hs;
            if (AFFINE) {
              nib = mad_u1(mn(subs(e, tup), one), sp(4), nib);
              nib = mad_u1(mn(subs(ff, tle), one), sp(8), nib);
            }
            acc[r / 4] |= bits(nib) << (4 * (r & 3));
          }
          if (MODE == ALN_LOCAL) {
            const s2 gt = mn(mx(subs(hv, bv[r]), zero), one);
            bjr[r] = mad_u(gt, subs(jj, bjr[r]), bjr[r]);
            bv[r] = mx(bv[r], hv);
          }
          f[r] = ff;
          hl[r] = hv;
          hd = hlo;
          hup = hv;
          eup = e;
        }
        if (MODE != ALN_LOCAL && (j == mm[0] || j == mm[1])) {
          const uint32_t msk = (j == mm[0] ? 0x0000ffffu : 0u) | (j == mm[1] ? 0xffff0000u : 0u);
#pragma unroll
          for (int r = 0; r < R; ++r) cap[r] = from_bits((bits(cap[r]) & ~msk) | (bits(hl[r]) & msk));
        }
        if (track_last) {
          // row n of each pair, picked by the bits of its index (any row where the pair has none here)
          uint32_t hw[R];
#pragma unroll
          for (int r = 0; r < R; ++r) hw[r] = bits(hl[r]);
          const s2 hn = from_bits(tree_pick<R>(hw, rnb));
          const int va = lo16(hn) + (kBias ? nn[0] * P.ge : 0), vb = hi16(hn) + (kBias ? nn[1] * P.ge : 0);
          if (lastA && j <= mm[0] && va > brow[0]) {
            brow[0] = va;
            browj[0] = j;
          }
          if (lastB && j <= mm[1] && vb > brow[1]) {
            brow[1] = vb;
            browj[1] = j;
          }
        }
        if (k + 1 < strips) rowbuf[(size_t)j * 64 + lane] = make_uint2(bits(hup), bits(eup));
        if (kFlagCodes) {
          uint2* __restrict__ d2 = reinterpret_cast<uint2*>(dirs);
#pragma unroll
          for (int g = 0; g < R / 8; ++g)
            d2[(((size_t)k * (R / 8) + g) * (size_t)max_m + (size_t)(j - 1)) * 64 + lane] =
                make_uint2(acc[2 * g], acc[2 * g + 1]);
        } else if (TB) {
#pragma unroll
          for (int w = 0; w < RW; ++w)
            dirs[(((size_t)k * RW + w) * (size_t)max_m + (size_t)(j - 1)) * 64 + lane] = acc[w];
        }
      };
      // Software pipeline over groups of 4 columns: the next group's global loads are issued
      // before the current group is relaxed, so their latency hides behind the arithmetic.
      int ca[4], cb[4];
      uint2 top[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) fetch(1 + u, ca[u], cb[u], top[u]);
      for (int j0 = 1; j0 <= mmax; j0 += 4) {
        int nca[4], ncb[4];
        uint2 ntop[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) fetch(j0 + 4 + u, nca[u], ncb[u], ntop[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (j0 + u <= mmax) column(j0 + u, ca[u], cb[u], top[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ca[u] = nca[u];
          cb[u] = ncb[u];
          top[u] = ntop[u];
        }
      }
      // merge this strip's rows in row order
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = i0 + 1 + r;
        for (int h = 0; h < 2; ++h) {
          if (MODE == ALN_LOCAL) {
            const int v = h ? hi16(bv[r]) : lo16(bv[r]);
            if (i <= nn[h] && v > best[h]) {
              best[h] = v;
              bi[h] = i;
              bj[h] = h ? hi16(bjr[r]) : lo16(bjr[r]);
            }
          } else {
            const int v = (h ? hi16(cap[r]) : lo16(cap[r])) + (kBias ? i * P.ge : 0);
            if (MODE == ALN_SEMIGLOBAL && i < nn[h] && v > best[h]) {
              best[h] = v;
              bi[h] = i;
              bj[h] = mm[h];
            }
            if (MODE == ALN_GLOBAL && i == nn[h]) hfin[h] = v;
          }
        }
      }
    }

    for (int h = 0; h < 2; ++h) {
      if (!act[h]) continue;
      const int n = nn[h], m = mm[h];
      int sc = best[h], ei = bi[h], ej = bj[h];
      if (MODE == ALN_SEMIGLOBAL) {
        if (n == 0 || m == 0) {
          sc = 0;
          ei = 0;
          ej = 0;
        } else if (brow[h] > sc) {
          sc = brow[h];
          ei = n;
          ej = browj[h];
        }
      } else if (MODE == ALN_GLOBAL) {
        ei = n;
        ej = m;
        sc = (n == 0 || m == 0) ? ((n + m > 0) ? P.go + (n + m) * P.ge : 0) : hfin[h];
      }
      const bool saturated = (MODE == ALN_LOCAL) && sc >= 32767;
      if (!flg[h] && !bad[h] && (!ok16[h] || saturated)) {
        const int k = atomicAdd(redo_cnt, 1);
        redo_idx[k] = (int)pp[h];
        continue;  // the 32-bit kernel writes this pair's result
      }
      aln_result_t res;
      res.score = sc;
      res.q_begin = -1;
      res.q_end = ei;
      res.s_begin = -1;
      res.s_end = ej;
      res.cigar_len = 0;
      res.reserved = 0;
      uint32_t fl = flg[h];
      if (bad[h]) fl |= ALN_RES_BAD_CODE;
      if (fl) {
        res.score = 0;
        res.q_end = 0;
        res.s_end = 0;
      } else if (TB) {
        const int64_t c0 = cigar_off[pp[h]];
        const int64_t capw = cigar_off[pp[h] + 1] - c0;
        const int shift = 16 * h;
        auto code = [&](int ii, int jx) -> uint32_t {
          const int kk = (ii - 1) / R, rr = (ii - 1) % R;
          if constexpr (kFlagCodes) {
            // the 4-bit code of walk.h from the row's four flags
            const uint2 w = reinterpret_cast<const uint2*>(
                dirs)[(((size_t)kk * (R / 8) + (rr >> 3)) * (size_t)max_m + (size_t)(jx - 1)) * 64 + lane];
            const int sh = 8 * h + (rr & 7);
            const uint32_t nd = (w.x >> sh) & 1u, ne = (w.x >> (sh + 16)) & 1u;
            const uint32_t xe = (w.y >> sh) & 1u, xf = (w.y >> (sh + 16)) & 1u;
            return (nd ? (ne ? 2u : 1u) : 0u) | (xe << 2) | (xf << 3);
          } else {
            const uint32_t w = dirs[(((size_t)kk * RW + rr / 4) * (size_t)max_m + (size_t)(jx - 1)) * 64 + lane];
            return (w >> (shift + 4 * (rr & 3))) & 15u;
          }
        };
        int qbeg, sbeg, runs;
        walk_back<MODE>(code, ei, ej, cigar + c0, capw, &qbeg, &sbeg, &runs);
        res.q_begin = qbeg;
        res.s_begin = sbeg;
        res.cigar_len = runs;
        if (runs > capw) fl |= ALN_RES_CIGAR_TRUNC;
      }
      res.flags = fl;
      out[pp[h]] = res;
    }
  }
}

template <int MODE, bool AFFINE, bool TB, int R>
void launch_i16_t(const KParams& kp, const BatchPlan16& pl, const I16Args& a, hipStream_t stream) {
  const int blocks = (pl.n_waves + kI16WavesPerBlock - 1) / kI16WavesPerBlock;
  const size_t lds = (size_t)kI16ProfBase + (size_t)kI16WavesPerBlock * i16_wave_prof_words(kp.alphabet, R) * 4;
  ProfScope prof(TB ? "batch_i16_traceback" : "batch_i16_score", stream);
  hipLaunchKernelGGL((batch_i16_kernel<MODE, AFFINE, TB, R>), dim3(blocks), dim3(kI16Block), lds, stream, kp, a.q,
                     a.q_off, a.s, a.s_off, pl.n_pairs, pl.max_n, pl.max_m, a.out, a.cigar, a.cigar_off,
                     static_cast<char*>(a.ws), pl.slab_bytes, pl.rowbuf_bytes, pl.rowbuf_bytes + pl.letters_bytes,
                     a.idx, a.idx_count, a.redo_idx,
                     a.redo_cnt, a.ticket);
}

template <int MODE, bool AFFINE, bool TB>
void launch_i16_r(const KParams& kp, const BatchPlan16& pl, const I16Args& a, hipStream_t st) {
  if (pl.R == 16)
    launch_i16_t<MODE, AFFINE, TB, 16>(kp, pl, a, st);
  else if (pl.R == 8)
    launch_i16_t<MODE, AFFINE, TB, 8>(kp, pl, a, st);
  else
    launch_i16_t<MODE, AFFINE, TB, 4>(kp, pl, a, st);
}

template <int MODE>
void launch_i16_m(const KParams& kp, const BatchPlan16& pl, const I16Args& a, bool tb, hipStream_t st) {
  const bool affine = kp.go != 0;
  if (affine) {
    if (tb)
      launch_i16_r<MODE, true, true>(kp, pl, a, st);
    else
      launch_i16_r<MODE, true, false>(kp, pl, a, st);
  } else {
    if (tb)
      launch_i16_r<MODE, false, true>(kp, pl, a, st);
    else
      launch_i16_r<MODE, false, false>(kp, pl, a, st);
  }
}

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

aln_status_t plan_batch_i16(const KParams& kp, int64_t n_pairs, int64_t max_n, int64_t max_m, bool tb,
                            BatchPlan16* pl) {
  pl->n_pairs = n_pairs;
  pl->max_n = max_n;
  pl->max_m = max_m;
  // rows per strip: the LDS query profile holds 128 pairs x (alphabet+1) letters x R rows per wave
  pl->R = kp.alphabet <= 4 ? 16 : (kp.alphabet <= 12 ? 8 : 4);
  const int64_t strips = (max_n + pl->R - 1) / pl->R;
  const int RW = (pl->R + 3) / 4;
  const int64_t groups = (n_pairs + 127) / 128;
  const int cus = device_cu_count();
  if (cus <= 0) return ALN_E_DEVICE;
  int64_t waves = (int64_t)cus * kI16WavesPerCU;
  if (groups < waves) waves = groups;
  if (waves < 1) waves = 1;
  waves = (waves + kI16WavesPerBlock - 1) / kI16WavesPerBlock * kI16WavesPerBlock;
  pl->n_waves = (int)waves;
  pl->rowbuf_bytes = round256((size_t)(max_m + 1) * 64 * sizeof(uint2));
  pl->letters_bytes = round256((size_t)(max_m + 1) * 64 * sizeof(uint16_t));
  pl->slab_bytes = pl->rowbuf_bytes + pl->letters_bytes +
                   (tb ? round256((size_t)strips * RW * (size_t)max_m * 64 * 4) : 0);
  if (tb) {
    // fewer waves in flight when every wave's codes would exceed the budget (at least one workgroup)
    const int64_t fit = kTbSlabBudget / (int64_t)pl->slab_bytes / kI16WavesPerBlock * kI16WavesPerBlock;
    if (fit < waves) pl->n_waves = (int)(fit > kI16WavesPerBlock ? fit : kI16WavesPerBlock);
  }
  pl->total_bytes = (size_t)pl->n_waves * pl->slab_bytes;
  return ALN_OK;
}

aln_status_t launch_batch_i16(const KParams& kp, const BatchPlan16& pl, const I16Args& a, bool tb,
                              hipStream_t stream) {
  if (pl.n_pairs == 0) return ALN_OK;
  switch (kp.mode) {
    case ALN_GLOBAL:
      launch_i16_m<ALN_GLOBAL>(kp, pl, a, tb, stream);
      break;
    case ALN_LOCAL:
      launch_i16_m<ALN_LOCAL>(kp, pl, a, tb, stream);
      break;
    default:
      launch_i16_m<ALN_SEMIGLOBAL>(kp, pl, a, tb, stream);
      break;
  }
  return hipGetLastError() == hipSuccess ? ALN_OK : ALN_E_DEVICE;
}

}  // namespace mialign
