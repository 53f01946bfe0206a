// Intra-sequence wavefront engine, 32-bit lanes: bands of rows relaxed as anti-diagonal fronts.
//
// A work item is one band (BH = 64*R rows) of one pair.  A wave relaxes a band: lane l owns R
// consecutive rows and works on column j = t - l + 1 at step t, so the 64 lanes sweep the band as an
// anti-diagonal front (cells on one anti-diagonal are independent, AnySeq Sec. III-A).  The lane
// above hands its bottom-row H and E (and the subject letter) down with a DPP wave_shr:1 move each
// step; lane 0 reads the band's top row from an LDS stage refilled every kBlk steps, and lane 63's
// outputs collect in a DPP wave_shl:1 shift register that is written out every kBlk steps.
//
// Work is handed out in groups of kWfWavesPerBlock consecutive items from one atomic ticket, so
// several pairs of different sizes share the device the way the paper's dynamic wavefront shares
// its queue between alignments (Sec. IV-A).  A workgroup relaxes one group: its compute waves take
// the group's bands, and the band below of a pair reads the band above's bottom row from an LDS ring
// with LDS progress counters -- the tile border publication of Sec. IV-B, without device memory.
// Where a pair continues into the next group, the workgroup's courier wave copies the last band's
// row to the pair's row slot in HBM and publishes a per-band progress counter once the stores have
// completed (device-coherent sc1 accesses); the next group's courier streams it into its first
// band's ring.  Only couriers wait on device memory, so the compute waves run at the rate of the
// recurrence.  Groups are handed out in order, so every group a courier waits on is already running;
// every wait is bounded -- a wave that waits too long raises an error flag and leaves its band, and
// all waves still meet at the group's barriers, so the grid always drains.
#include <type_traits>

#include "internal.h"
#include "band.h"
#include "walk.h"
#include "walk_wave.h"

extern "C" __device__ __attribute__((const)) int __ockl_wfred_max_i32(int);  // maximum over the wave

namespace mialign {
namespace {

// A workgroup is a group of kWfWavesPerBlock compute waves, which relax consecutive bands, plus one
// courier wave.  Consecutive bands of a pair hand their rows to each other through LDS rings; the
// courier streams the group's first input row from HBM and its last output row to HBM, so only the
// courier ever waits on device memory.
constexpr int kWfWavesPerBlock = kWfGroupBands;       // compute waves (bands) per workgroup
constexpr int kWfBlock = 64 * (kWfWavesPerBlock + 1);  // plus the courier
constexpr int kRing = 256;                            // columns held by one LDS ring
constexpr int kBlkGrouped = 32;                       // steps between lane-0 input refills, grouped
constexpr int kCourierChunk = 32;                     // columns a courier moves between HBM and LDS at once
constexpr int kWfBlockAlone = 64 * kWfWavesPerBlock;  // bands on their own: no courier


__device__ __forceinline__ int dpp_shr1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xf, 0xf, false);  // wave_shr:1, lane 0 keeps old
}
__device__ __forceinline__ int dpp_shl1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x130, 0xf, 0xf, false);  // wave_shl:1, lane 63 keeps old
}

// Local alignment: every row keeps the best biased score it has seen (bv) and the first column that
// reached it.  The pair's optimum -- the first cell in (score, i, j) order -- scores at least as high
// as every real cell, so once per block each row's running value is raised to the largest score seen
// so far minus one (ties still pass, also for transposed pairs, whose caller rows run along the band):
// the best of the band's top-row inputs, which are cells of an earlier row, and the best its own rows
// have recorded.  Rows then record only cells that may still be the optimum.  On related sequences
// the top row stays ahead of the values that climb towards the diagonal inside the band; on unrelated
// ones the band's best over all its rows is rarely beaten; either way the exact per-cell update runs
// in a small fraction of the 4-step groups.  A raised value never wins: it is below a real cell,
// which some band records or beats.  top_h is the top-row Hb (row i0's bias) of the block's columns,
// or 0 (at most H = 0) on lanes without one.  Rows past n need no mask: with gap scores <= 0 their
// values come from row n's minus penalties, or from the floor H = 0, so they never exceed the
// optimum either.  Every lane of the wave calls this.
template <int R>
__device__ __forceinline__ void raise_local_floors(int32_t (&bv)[R], const int32_t (&nu)[R], int32_t top_h, int i0,
                                                   int32_t ge) {
  static_assert(R % 2 == 0, "rows are folded in pairs");
  int32_t v = top_h + i0 * ge;  // H of the top-row cell
#pragma unroll
  for (int r = 0; r < R; r += 2) v = max(max(v, bv[r] - nu[r]), bv[r + 1] - nu[r + 1]);
  const int32_t fl = __ockl_wfred_max_i32(v) - 1;
#pragma unroll
  for (int r = 0; r < R; ++r) bv[r] = max(bv[r], fl + nu[r]);
}

// Per lane, a where the lane's bit of mask is set, else b: one v_cndmask, never a branch.
__device__ __forceinline__ int mask_select(unsigned long long mask, int a, int b) {
  int r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mask));
  return r;
}

// c ? a : b as one v_cndmask on the lane mask of c, so the compiler cannot turn the choice into a
// branch around the computation of a
__device__ __forceinline__ int lane_select(bool c, int a, int b) {
  const unsigned long long mask = __builtin_amdgcn_ballot_w64(c);
  int r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mask));
  return r;
}

// Packed 16-bit bands (local alignment, score only; register profiles for up to 4 letters, per-lane LDS
// profiles of two 16-bit rows per half for up to 32).  A 32-bit lane
// register holds two 16-bit cells: rows of the band's upper half (HB = 128 rows) in its low half and
// rows of the lower half in its high half, the lower half running kP16Delay steps behind so that the
// two are independent within a step -- the two halves are independent submatrices sharing one vector
// lane, as in the paper's inter-task vectorisation (Sec. IV-A), and each keeps its scores as 16-bit
// differences from an offset of its own, as the paper does within a block (Sec. IV-A): the offset is
// the half's top-row score at the first column of each block of steps.
typedef short s2 __attribute__((ext_vector_type(2)));
constexpr int kP16Half = 128;   // rows per half band
constexpr int kP16Delay = 96;   // steps between the upper and the lower half
constexpr int kDelayRing = 256; // columns of the upper half's bottom row kept for the lower half
constexpr int kNeg16 = -32768;  // stands for -infinity; sums saturate, so it stays far below real scores
// The lower half's lane 0 reads columns up to j + kBlkGrouped - 1 - kP16Delay at the start of the block
// of step j; the upper half's lane 63 has written them by then only if the delay covers a block plus
// lane 63's 63 steps.  The delay line must also keep a column until the lower half has read it.
static_assert(kP16Delay >= kBlkGrouped + 63, "the delay between the halves must cover a block and the lanes");
static_assert(kDelayRing >= kP16Delay + kBlkGrouped, "the delay line must hold the columns in flight");

__device__ __forceinline__ s2 as_s2(int x) { return __builtin_bit_cast(s2, x); }
__device__ __forceinline__ int as_int(s2 x) { return __builtin_bit_cast(int, x); }
__device__ __forceinline__ int sat16(int x) { return min(max(x, -32768), 32767); }
__device__ __forceinline__ int pack16(int lo, int hi) { return (int)(((uint32_t)lo & 0xffffu) | ((uint32_t)hi << 16)); }
__device__ __forceinline__ int lo16(int x) { return (int)(int16_t)(x & 0xffff); }
__device__ __forceinline__ int hi16(int x) { return x >> 16; }
__device__ __forceinline__ int padd(int a, int b) { return as_int(__builtin_elementwise_add_sat(as_s2(a), as_s2(b))); }
__device__ __forceinline__ int psub(int a, int b) { return as_int(__builtin_elementwise_sub_sat(as_s2(a), as_s2(b))); }
__device__ __forceinline__ int pmax(int a, int b) { return as_int(__builtin_elementwise_max(as_s2(a), as_s2(b))); }
// a 16-bit relative score back to an absolute 32-bit one (-infinity stays -infinity)
__device__ __forceinline__ int unrel16(int rel, int base) { return rel == kNeg16 ? kNeg32 : rel + base; }

// (score, i, j) order of optima: larger score, then smaller i, then smaller j.
__device__ __forceinline__ bool better(int s1, int i1, int j1, int s2, int i2, int j2) {
  return s1 > s2 || (s1 == s2 && (i1 < i2 || (i1 == i2 && j1 < j2)));
}

// Bands on their own (one wave per band, hand-offs through HBM), handed out level by level (wf_order_kernel).
//
// Values are kept with a row bias: Hb(i,j) = H(i,j) - i*ge, and likewise E and F.  Then
//   Eb(i,j) = max(Eb(i-1,j), Hb(i-1,j) + go)          (extension costs nothing: one add less)
//   Fb(i,j) = max(Fb(i,j-1) + ge, Hb(i,j-1) + go + ge)
//   Hb(i,j) = max(Hb(i-1,j-1) + sigma - ge, Eb, Fb [, -i*ge for local])
// which is Eqs. (1), (4), (5) with every term shifted by the same per-row constant.
template <int MODE, bool AFFINE, int PROF, bool TB, int R>
__global__ __launch_bounds__(kWfBlockAlone) void wf_i32_kernel(const KParams P, const uint8_t* __restrict__ Q,
                                                          const uint8_t* __restrict__ S, WfWs W) {
  static_assert(PROF != kProfLane || R == 4, "a lane profile word holds 4 rows");
  // sigma - ge by (query letter, subject letter); also the source of the byte profiles
  __shared__ int32_t tab[kTab * kTab];
  __shared__ int4 stage[kWfWavesPerBlock][3][16];  // lane-0 inputs of 64 steps: H, E, letter
  extern __shared__ uint32_t lprof[];               // kProfLane: [wave][letter][lane], alphabet letters
  for (int k = threadIdx.x; k < kTab * kTab; k += blockDim.x) {
    const int a = k / kTab, b = k % kTab;
    tab[k] = (a >= P.alphabet || b >= P.alphabet) ? -kBig32 : (int32_t)P.sig[a * kMaxAlphabet + b] - P.ge;
  }
  __syncthreads();
  constexpr int BH = 64 * R;
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  int* st_h = reinterpret_cast<int*>(&stage[wib][0][0]);
  int* st_e = reinterpret_cast<int*>(&stage[wib][1][0]);
  int* st_c = reinterpret_cast<int*>(&stage[wib][2][0]);
  const int32_t go = P.go, ge = P.ge, goe = P.goe;
  const int np = *W.n_pairs;
  const int64_t n_items = *W.n_items;

  for (;;) {
    int64_t t = 0;
    if (lane == 0) t = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(W.ticket), 1ull);
    t = __shfl(t, 0, 64);
    if (t >= n_items) break;
    if (__hip_atomic_load(W.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    t = W.order[t];  // the item (pair-major band index) this ticket hands out
    const WfPair pr = W.pairs[np == 1 ? 0 : W.item_pair[t]];
    const int b = (int)(t - pr.item0);
    const int n = pr.n, m = pr.m, nb = pr.nb;
    // rows come from the query array, columns from the subject array, or the reverse when flipped
    const bool flip = pr.flip != 0;
    const uint8_t* __restrict__ q = (flip ? S : Q) + pr.q_off;
    const uint8_t* __restrict__ s = (flip ? Q : S) + pr.s_off;
    const int64_t ld = (int64_t)m + 1;
    // sigma - ge of a (row letter, column letter) pair, taken in the call's (query, subject) order
    auto sig_rc = [&](int cr, int cc) -> int { return flip ? tab[cc * kTab + cr] : tab[cr * kTab + cc]; };

    const int i0 = b * BH;
    int prof[R];  // kProfReg: 4 bytes sigma - ge against letters 0..3; kProfTable: table offset of the letter
    int32_t hl[R], f[R], bv[R], nu[R];
    int bj[R];
    int rowc[R];
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + lane * R + r + 1;
      int c = kPad;
      if (i <= n) {
        c = q[i - 1];
        if (c >= P.alphabet) {
          bad = true;
          c = kPad;
        }
      }
      rowc[r] = c;
      if (PROF == kProfReg) {
        uint32_t w = 0;
        for (int a = 0; a < 4; ++a) {
          const int v = (c < P.alphabet && a < P.alphabet) ? sig_rc(c, a) : -128;
          w |= ((uint32_t)(v & 0xff)) << (8 * a);
        }
        prof[r] = (int)w;
      } else if (PROF == kProfTable) {
        prof[r] = flip ? c : c * kTab;  // the table is indexed [query letter][subject letter]
      } else {
        prof[r] = 0;
      }
      hl[r] = (MODE == ALN_GLOBAL) ? go : -i * ge;  // Hb(i, 0)
      f[r] = kNeg32;
      nu[r] = -i * ge;                                // local floor: H = 0
      bv[r] = kNeg32;
      bj[r] = 0;
    }
    uint32_t* __restrict__ lp = lprof + (PROF == kProfLane ? wib * P.alphabet * 64 + lane : 0);
    if (PROF == kProfLane) {
      // this lane's word per column letter; each lane reads only its own words, so no barrier
      for (int a = 0; a < P.alphabet; ++a) {
        uint32_t w = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int v = rowc[r] < P.alphabet ? sig_rc(rowc[r], a) : -128;
          w |= ((uint32_t)(v & 0xff)) << (8 * r);
        }
        lp[a * 64] = w;
      }
    }
    const int irow0 = i0 + lane * R;  // the row just above this lane's first row
    int32_t diag = (MODE == ALN_GLOBAL) ? (irow0 > 0 ? go : 0) : -irow0 * ge;  // Hb(irow0, 0)
    uint16_t* __restrict__ codes = TB ? W.codes + pr.code_off + (size_t)(b * 64 + lane) * (size_t)m : nullptr;
    int32_t bot_h = 0, bot_e = kNeg32, cur_c = 0, out_h = 0, out_e = 0;
    // semi-global: the band holding row n tracks row n's running maximum
    const bool last_band = (b == nb - 1);
    int32_t brow = -n * ge;  // Hb(n, 0), i.e. H(n, 0) = 0
    int browj = 0;
    const int rn = n - 1 - irow0;  // index of row n among this lane's rows

    int2* __restrict__ prev = W.rows + pr.row_off + (int64_t)((b + 1) & 1) * ld;
    int2* __restrict__ cur = W.rows + pr.row_off + (int64_t)(b & 1) * ld;
    bool failed = false;

    int seen = 0;  // columns of the previous band known to be published
    constexpr int BLK = 64;

    const int steps = m + 63;
    for (int tb = 0; tb < steps; tb += BLK) {
      // lane-0 inputs for steps tb..tb+63 (columns tb+1..tb+64)
      const int col_in = tb + 1 + lane;
      int sreg = 0;
      if (col_in <= m) {
        sreg = s[col_in - 1];
        if (sreg >= P.alphabet) {
          bad = true;
          sreg = PROF == kProfTable ? kPad : 0;
        }
      }
      if (PROF == kProfReg) sreg *= 8;
      if (PROF == kProfLane) sreg *= 64;
      if (PROF == kProfTable && flip) sreg *= kTab;
      int32_t th, te;
      if (b == 0) {
        th = (MODE == ALN_GLOBAL) ? go + col_in * ge : 0;
        te = kNeg32;
      } else {
        const int need = min(tb + BLK, m);
        if (seen < need) {
          int v = 0;
          if (lane == 0) {
            long long spins = 0;
            for (;;) {
              v = __hip_atomic_load(W.flags + (t - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              if (v >= need) break;
              if (++spins > P.spin_dev || __hip_atomic_load(W.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                v = -1;
                break;
              }
              __builtin_amdgcn_s_sleep(1);
            }
          }
          v = __shfl(v, 0, 64);
          if (v < 0) {
            if (lane == 0) __hip_atomic_store(W.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            failed = true;
            break;
          }
          // The row data below is read with device-coherent (sc1) loads issued after the flag load has
          // returned, so they observe the producer's sc1 stores that completed before its flag store.
          asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
          seen = v;
        }
        th = 0;
        te = kNeg32;
        if (col_in <= m) {
          const long long pv = __hip_atomic_load(reinterpret_cast<long long*>(prev + col_in), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
          th = (int32_t)(pv & 0xffffffffll);
          te = (int32_t)(pv >> 32);
        }
      }
      if (MODE == ALN_LOCAL) raise_local_floors<R>(bv, nu, th, i0, ge);
      st_h[lane] = th;
      st_e[lane] = te;
      st_c[lane] = sreg;
      // One step: lane l relaxes column j = t - l + 1 for its R rows.
      auto step = [&](int t, int in_top_h, int in_top_e, int in_top_c, auto checked, int32_t* hk) {
        const int j = t - lane + 1;
        const int in_h = dpp_shr1(in_top_h, bot_h);
        const int in_e = dpp_shr1(in_top_e, bot_e);
        const int in_c = dpp_shr1(in_top_c, cur_c);
        cur_c = in_c;
        if (!decltype(checked)::value || (j >= 1 && j <= m)) {
          int32_t hd = diag, hup = in_h, eup = in_e;
          int32_t hn = 0;
          uint32_t word = 0;
          const int pw = PROF == kProfLane ? (int)lp[in_c] : 0;
          // local affine score-only bands fold the floor into E (band.h)
          constexpr bool kFloorE = MODE == ALN_LOCAL && AFFINE && !TB;
          band_column<MODE, AFFINE, PROF, TB, decltype(checked)::value, R, true, kFloorE>(
              tab, prof, in_c, pw, go, ge, goe, nu, hl, f, bv, bj, hk, j, rn, hd, hup, eup, hn, word);
          if (TB) codes[j - 1] = (uint16_t)word;
          if (MODE == ALN_SEMIGLOBAL && last_band && rn >= 0 && rn < R && hn > brow) {
            brow = hn;
            browj = j;
          }
          bot_h = hup;
          bot_e = eup;
          diag = in_h;
        }
        out_h = dpp_shl1(bot_h, out_h);
        out_e = dpp_shl1(bot_e, out_e);
      };
      for (int g4 = 0; g4 < BLK / 4; ++g4) {
        const int t0 = tb + 4 * g4;
        const int4 vh = reinterpret_cast<const int4*>(st_h)[g4];
        const int4 ve = reinterpret_cast<const int4*>(st_e)[g4];
        const int4 vc = reinterpret_cast<const int4*>(st_c)[g4];
        if (t0 >= 63 && t0 + 3 < m) {
          // every lane is inside the matrix: no range test; local optima are tracked per 4 steps
          int32_t hk[4][R];
          step(t0, vh.x, ve.x, vc.x, std::false_type(), hk[0]);
          step(t0 + 1, vh.y, ve.y, vc.y, std::false_type(), hk[1]);
          step(t0 + 2, vh.z, ve.z, vc.z, std::false_type(), hk[2]);
          step(t0 + 3, vh.w, ve.w, vc.w, std::false_type(), hk[3]);
          if (MODE == ALN_LOCAL) {
            int32_t mk[R];
            bool imp = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              mk[r] = max(max(hk[0][r], hk[1][r]), max(hk[2][r], hk[3][r]));
              imp |= mk[r] > bv[r];
            }
            if (imp) {
              // a row that beat its best takes the group's maximum at the first of the 4 steps that
              // reached it, as a cell-by-cell strict update would
#pragma unroll
              for (int r = 0; r < R; ++r) {
                int k = hk[2][r] == mk[r] ? 2 : 3;
                k = hk[1][r] == mk[r] ? 1 : k;
                k = hk[0][r] == mk[r] ? 0 : k;
                bj[r] = lane_select(mk[r] > bv[r], t0 - lane + 1 + k, bj[r]);
                bv[r] = max(bv[r], mk[r]);
              }
            }
          }
        } else {
          step(t0, vh.x, ve.x, vc.x, std::true_type(), nullptr);
          step(t0 + 1, vh.y, ve.y, vc.y, std::true_type(), nullptr);
          step(t0 + 2, vh.z, ve.z, vc.z, std::true_type(), nullptr);
          step(t0 + 3, vh.w, ve.w, vc.w, std::true_type(), nullptr);
        }
      }
      // lane u now holds lane 63's outputs of step tb+u, i.e. column tb+u-62
      if (b + 1 < nb) {
        const int col_out = tb + lane - 62;
        if (col_out >= 1 && col_out <= m) {
          const long long pv = ((long long)(uint32_t)out_h) | ((long long)out_e << 32);
          __hip_atomic_store(reinterpret_cast<long long*>(cur + col_out), pv, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        }
        const int published = min(tb + 1, m);
        // Publication: the row stores above are device-coherent (sc1) atomics; waiting for their
        // completion before the sc1 flag store orders them without an L2 write-back (an agent-scope
        // release fence would emit buffer_wbl2 on every publication).
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if (published >= 1 && lane == 0)
          __hip_atomic_store(W.flags + t, published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    // band optimum: (score, i, j) over this lane's rows, then across the wave
    int bs = kNeg32, bi = 0, bjj = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = irow0 + r + 1;
      if (i > n) continue;
      int sc = 0, jj = 0;
      bool cand = false;
      if (MODE == ALN_LOCAL) {
        sc = bv[r] + i * ge;
        jj = bj[r];
        cand = sc > 0;
      } else if (MODE == ALN_SEMIGLOBAL) {
        sc = hl[r] + i * ge;  // H(i, m): last-column candidate; row n is handled below
        jj = m;
        cand = (i < n);
      } else {
        sc = hl[r] + i * ge;
        jj = m;
        cand = (i == n);
      }
      // a flipped pair's cell (i, jj) is the call's cell (jj, i)
      const int ci = flip ? jj : i, cj = flip ? i : jj;
      if (cand && better(sc, ci, cj, bs, bi, bjj)) {
        bs = sc;
        bi = ci;
        bjj = cj;
      }
    }
    if (MODE == ALN_SEMIGLOBAL && last_band && rn >= 0 && rn < R) {
      // row n: (n, 0) with H = 0 first, then its running maximum over j in column order
      const int rowv = (browj > 0) ? brow + n * ge : 0;
      const int ci = flip ? browj : n, cj = flip ? n : browj;
      if (better(rowv, ci, cj, bs, bi, bjj)) {
        bs = rowv;
        bi = ci;
        bjj = cj;
      }
    }
    for (int o = 32; o >= 1; o >>= 1) {
      const int s2 = __shfl_xor(bs, o, 64), i2 = __shfl_xor(bi, o, 64), j2 = __shfl_xor(bjj, o, 64);
      if (better(s2, i2, j2, bs, bi, bjj)) {
        bs = s2;
        bi = i2;
        bjj = j2;
      }
    }
    const bool anybad = __any(bad);
    if (lane == 0) W.band_res[t] = make_int4(bs, bi, bjj, (anybad ? 1 : 0) | (failed ? 2 : 0));
  }
}

// Bands in groups (workgroups of kWfWavesPerBlock bands and a courier), same recurrence.
// Values are kept with a row bias: Hb(i,j) = H(i,j) - i*ge, and likewise E and F.  Then
//   Eb(i,j) = max(Eb(i-1,j), Hb(i-1,j) + go)          (extension costs nothing: one add less)
//   Fb(i,j) = max(Fb(i,j-1) + ge, Hb(i,j-1) + go + ge)
//   Hb(i,j) = max(Hb(i-1,j-1) + sigma - ge, Eb, Fb [, -i*ge for local])
// which is Eqs. (1), (4), (5) with every term shifted by the same per-row constant.
// CKPT: also store checkpoints for a linear-space traceback (one pair, groups aligned with its bands):
// every group's bottom row stays in its own row slot instead of two rotating ones, and every
// kTileCols-th column's H and F of all rows go to W.ckcols.
template <int MODE, bool AFFINE, int PROF, bool TB, int R, bool P16, bool CKPT, bool LAZY>
__global__ __launch_bounds__(kWfBlock) void wf_i32_group_kernel(const KParams P, const uint8_t* __restrict__ Q,
                                                          const uint8_t* __restrict__ S, WfWs W) {
  static_assert(PROF != kProfLane || R == 4, "a lane profile word holds 4 rows");
  // sigma - ge by (query letter, subject letter); also the source of the byte profiles
  __shared__ int32_t tab[kTab * kTab];
  constexpr int BLK = kBlkGrouped;
  __shared__ int4 stage[kWfWavesPerBlock][3][BLK / 4];  // lane-0 inputs of BLK steps: H, E, letter
  // ring k carries the rows feeding compute wave k; ring kWfWavesPerBlock feeds the courier
  __shared__ int2 ring[kWfWavesPerBlock + 1][kRing];
  __shared__ int pub[kWfWavesPerBlock + 1];  // columns written into each ring
  __shared__ int con[kWfWavesPerBlock + 1];  // columns read out of each ring
  __shared__ long long s_t0;                 // first item of the group
  __shared__ int s_err;
  extern __shared__ uint32_t lprof[];        // kProfLane: [wave][letter][lane], alphabet letters
  static_assert(!P16 || (MODE == ALN_LOCAL && (PROF == kProfReg || PROF == kProfLane) && !TB && R == 4),
                "packed bands: local, score only, register or per-lane profiles");
  static_assert(!CKPT || (!TB && !P16 && R == 4), "checkpoints: 32-bit score-only bands");
  static_assert(!LAZY || (MODE == ALN_LOCAL && !TB && !P16 && !CKPT), "kept groups: local 32-bit score-only bands");
  // packed bands: the upper half's bottom row (absolute H, E) on its way to the lower half
  __shared__ int2 dline[P16 ? kWfWavesPerBlock : 1][P16 ? kDelayRing : 1];
  for (int k = threadIdx.x; k < kTab * kTab; k += blockDim.x) {
    const int a = k / kTab, b = k % kTab;
    tab[k] = (a >= P.alphabet || b >= P.alphabet) ? -kBig32 : (int32_t)P.sig[a * kMaxAlphabet + b] - P.ge;
  }
  __syncthreads();
  constexpr int BH = 64 * R;
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  const int cw = wib < kWfWavesPerBlock ? wib : 0;  // the courier borrows wave 0's stage pointers
  int* st_h = reinterpret_cast<int*>(&stage[cw][0][0]);
  int* st_e = reinterpret_cast<int*>(&stage[cw][1][0]);
  int* st_c = reinterpret_cast<int*>(&stage[cw][2][0]);
  const int32_t go = P.go, ge = P.ge, goe = P.goe;
  const int np = *W.n_pairs;
  const int64_t n_items = *W.n_items;

  // Bounded waits.  A wave that gives up raises the group's and the launch's error flags and leaves
  // its band; every wave still meets the group's barriers, so the grid drains.
  auto give_up = [&]() {
    if (lane == 0) {
      __hip_atomic_store(&s_err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_store(W.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

  // The courier: for the group's first band (if it has a band above, in another group) it streams
  // that band's bottom row from HBM into ring 0, kCourierChunk columns at a time, once the band above has
  // published them; for the group's last band (if its band below is in another group) it copies
  // ring kWfWavesPerBlock to the pair's row slot in HBM and publishes the band's progress counter
  // once those stores have completed.  HBM rows and counters use device-coherent (sc1) accesses.
  auto courier = [&](int64_t t0) {
    const int64_t tin = t0, tout = t0 + kWfWavesPerBlock - 1;
    bool in_on = false, out_on = false;
    int m_in = 0, m_out = 0;
    const int2* src = nullptr;
    int2* dst = nullptr;
    if (tin < n_items) {
      const WfPair a = W.pairs[np == 1 ? 0 : W.item_pair[tin]];
      const int b = (int)(tin - a.item0);
      if (b > 0) {
        in_on = true;
        m_in = a.m;
        const int64_t slot = CKPT ? b / kWfWavesPerBlock - 1 : ((b + 1) & 1);
        src = W.rows + a.row_off + slot * ((int64_t)a.m + 1);
      }
    }
    if (tout < n_items) {
      const WfPair a = W.pairs[np == 1 ? 0 : W.item_pair[tout]];
      const int b = (int)(tout - a.item0);
      if (b + 1 < a.nb) {
        out_on = true;
        m_out = a.m;
        const int64_t slot = CKPT ? b / kWfWavesPerBlock : (b & 1);
        dst = W.rows + a.row_off + slot * ((int64_t)a.m + 1);
      }
    }
    int in_done = 0, out_done = 0, seen = 0;
    long long idle = 0;
    while ((in_on && in_done < m_in) || (out_on && out_done < m_out)) {
      bool moved = false;
      if (in_on && in_done < m_in) {
        const int want = min(in_done + kCourierChunk, m_in);
        if (seen < want) seen = __hip_atomic_load(W.flags + (tin - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (seen >= want &&
            __hip_atomic_load(&con[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= want - kRing) {
          // the row loads are issued after the counter load has returned (device-coherent loads)
          const int col = in_done + 1 + lane;
          if (col <= want) {
            const long long v = __hip_atomic_load(reinterpret_cast<const long long*>(src + col), __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            ring[0][col % kRing] = make_int2((int32_t)(v & 0xffffffffll), (int32_t)(v >> 32));
          }
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
          if (lane == 0) __hip_atomic_store(&pub[0], want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          in_done = want;
          moved = true;
        }
      }
      if (out_on && out_done < m_out) {
        const int want = min(out_done + kCourierChunk, m_out);
        if (__hip_atomic_load(&pub[kWfWavesPerBlock], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= want) {
          const int col = out_done + 1 + lane;
          if (col <= want) {
            const int2 v = ring[kWfWavesPerBlock][col % kRing];
            const long long pv = ((long long)(uint32_t)v.x) | ((long long)v.y << 32);
            __hip_atomic_store(reinterpret_cast<long long*>(dst + col), pv, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          }
          // stores complete (device-coherent) before the counter that announces them; the ring
          // values were read before the stores were issued, so the slots can be released too
          asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
          if (lane == 0) {
            __hip_atomic_store(W.flags + tout, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&con[kWfWavesPerBlock], want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
          out_done = want;
          moved = true;
        }
      }
      if (moved) {
        idle = 0;
      } else {
        __builtin_amdgcn_s_sleep(1);
        if (++idle > P.spin_dev || __hip_atomic_load(&s_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) ||
            __hip_atomic_load(W.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          give_up();
          break;
        }
      }
    }
  };


  // Packed 16-bit band t (see kP16Half): lane l holds rows i0 + 2l + 1, i0 + 2l + 2 of the upper half
  // in the low 16 bits and the same rows plus kP16Half in the high 16 bits.  The upper half works on
  // column j = t - l + 1 at step t, the lower half on j - kP16Delay.  Values are the row-biased Hb of
  // the 32-bit kernel minus the half's offset; each block re-bases both halves on their top-row
  // scores at the block's first column, so every value of a block stays within a few thousand of its
  // offset (adjacent cells differ by at most max|sigma| + |go| + 2|ge|, which the host bounds).  The
  // band's inputs and outputs are absolute 32-bit rows, as for the 32-bit bands.
  auto p16_band = [&](auto t_) {
    const int64_t t = t_;
    const WfPair pr = W.pairs[np == 1 ? 0 : W.item_pair[t]];
    const int b = (int)(t - pr.item0);
    const int n = pr.n, m = pr.m, nb = pr.nb;
    const bool flip = pr.flip != 0;
    const uint8_t* __restrict__ q = (flip ? S : Q) + pr.q_off;
    const uint8_t* __restrict__ s = (flip ? Q : S) + pr.s_off;
    auto sig_rc = [&](int cr, int cc) -> int { return flip ? tab[cc * kTab + cr] : tab[cr * kTab + cc]; };
    constexpr int HB = kP16Half, D = kP16Delay, BH = 64 * R;
    const int i0 = b * BH;
    // half h (0 upper, 1 lower), row r (0, 1): i = i0 + h * HB + 2 lane + r + 1
    int prof[2][2];
    int rowc[2][2];
    int32_t nuA[2][2], bvA[2][2];
    int bjA[2][2];
    bool bad = false;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int i = i0 + h * HB + 2 * lane + r + 1;
        int c = kPad;
        if (i <= n) {
          c = q[i - 1];
          if (c >= P.alphabet) {
            bad = true;
            c = kPad;
          }
        }
        rowc[h][r] = c;
        uint32_t w = 0;
        if (PROF == kProfReg) {
          for (int a = 0; a < 4; ++a) {
            const int v = (c < P.alphabet && a < P.alphabet) ? sig_rc(c, a) : -128;
            w |= ((uint32_t)(v & 0xff)) << (8 * a);
          }
        }
        prof[h][r] = (int)w;
        nuA[h][r] = -i * ge;  // Hb(i, j) of H = 0, also Hb(i, 0)
        bvA[h][r] = kNeg32;
        bjA[h][r] = 0;
      }
    // kProfLane: per column letter, this lane's two rows of each half as 16-bit sigma - ge, the upper
    // half's in lpu[letter * 64] and the lower half's in lpl[letter * 64]; each lane reads only its own
    // words, so no barrier
    const uint32_t* __restrict__ lpu = lprof + (PROF == kProfLane ? (size_t)wib * 2 * P.alphabet * 64 + lane : 0);
    const uint32_t* __restrict__ lpl = lpu + (PROF == kProfLane ? (size_t)P.alphabet * 64 : 0);
    if (PROF == kProfLane) {
      uint32_t* wu = lprof + (size_t)wib * 2 * P.alphabet * 64 + lane;
      for (int a = 0; a < P.alphabet; ++a) {
        uint32_t hw[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int v0 = rowc[h][0] < P.alphabet ? sig_rc(rowc[h][0], a) : -128;
          const int v1 = rowc[h][1] < P.alphabet ? sig_rc(rowc[h][1], a) : -128;
          hw[h] = (uint32_t)(v0 & 0xffff) | ((uint32_t)v1 << 16);
        }
        wu[a * 64] = hw[0];
        wu[(P.alphabet + a) * 64] = hw[1];
      }
    }
    int32_t B0 = -i0 * ge, B1 = -(i0 + HB) * ge;  // offsets: Hb of each half's top row at column 0
    int hl[2], f[2], nu[2], bvr[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      hl[r] = pack16(sat16(nuA[0][r] - B0), sat16(nuA[1][r] - B1));
      f[r] = pack16(kNeg16, kNeg16);
      nu[r] = hl[r];
      bvr[r] = pack16(kNeg16, kNeg16);
    }
    int diag = pack16(sat16(-(i0 + 2 * lane) * ge - B0), sat16(-(i0 + HB + 2 * lane) * ge - B1));
    int bot_h = 0, bot_e = pack16(kNeg16, kNeg16), cur_c = 0, out_h = 0, out_e = 0;
    const int go2 = pack16(go, go), ge2 = pack16(ge, ge), goe2 = pack16(goe, goe);
    bool failed = false;
    int2* __restrict__ rin = ring[wib];
    int2* __restrict__ rout = ring[wib + 1];
    int2* __restrict__ dl = dline[wib];
    const bool has_out = b + 1 < nb;
    auto letter_raw = [&](int col) -> int { return (col >= 1 && col <= m) ? (int)s[col - 1] : -1; };
    auto letter_idx = [&](int c) -> int {
      if (c < 0) return 0;
      if (c >= P.alphabet) {
        bad = true;
        c = 0;
      }
      return PROF == kProfLane ? c * 64 : c * 8;
    };
    int cn0 = lane < BLK ? letter_raw(1 + lane) : -1;
    int cn1 = lane < BLK ? letter_raw(1 + lane - D) : -1;

    const int steps = m + 63 + D;  // lane 63's lower half reaches column m at step m + 62 + D
    for (int tb = 0; tb < steps; tb += BLK) {
      const int col0 = tb + 1 + lane, col1 = col0 - D;  // lane-0 input columns of the two halves
      const int c0 = letter_idx(cn0), c1 = letter_idx(cn1);
      asm volatile("" ::"v"(c0), "v"(c1) : "memory");
      cn0 = lane < BLK ? letter_raw(col0 + BLK) : -1;
      cn1 = lane < BLK ? letter_raw(col1 + BLK) : -1;
      int32_t th0 = 0, te0 = kNeg32, th1 = 0, te1 = kNeg32;
      if (b > 0) {
        const int need = min(tb + BLK, m);
        if (!lds_wait_ge(&pub[wib], need)) {
          failed = true;
          break;
        }
        if (lane < BLK && col0 <= m) {
          const int2 v = rin[col0 % kRing];
          th0 = v.x;
          te0 = v.y;
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (lane == 0) __hip_atomic_store(&con[wib], need, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      if (lane < BLK && col1 >= 1 && col1 <= m) {
        const int2 v = dl[col1 % kDelayRing];
        th1 = v.x;
        te1 = v.y;
      }
      // re-base each half on its top-row score at the block's first column while it is in the matrix
      const int nB0 = (tb + 1 <= m) ? __builtin_amdgcn_readfirstlane(th0) : B0;
      const int nB1 = (tb + 1 - D >= 1 && tb + 1 - D <= m) ? __builtin_amdgcn_readfirstlane(th1) : B1;
      if (nB0 != B0 || nB1 != B1) {
        const int dd = pack16(sat16(nB0 - B0), sat16(nB1 - B1));
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          hl[r] = psub(hl[r], dd);
          f[r] = psub(f[r], dd);
        }
        bot_h = psub(bot_h, dd);
        bot_e = psub(bot_e, dd);
        diag = psub(diag, dd);
        B0 = nB0;
        B1 = nB1;
      }
      {
        // floors (see raise_local_floors): the best of both halves' top-row inputs and recorded optima
        int v = max(th0 + i0 * ge, th1 + (i0 + HB) * ge);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 2; ++r) v = max(v, bvA[h][r] - nuA[h][r]);
        const int fl = __ockl_wfred_max_i32(v) - 1;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 2; ++r) bvA[h][r] = max(bvA[h][r], fl + nuA[h][r]);
      }
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        nu[r] = pack16(sat16(nuA[0][r] - B0), sat16(nuA[1][r] - B1));
        bvr[r] = pack16(sat16(bvA[0][r] - B0), sat16(bvA[1][r] - B1));
      }
      if (lane < BLK) {
        st_h[lane] = pack16(sat16(th0 - B0), sat16(th1 - B1));
        st_e[lane] = pack16(sat16(te0 - B0), sat16(te1 - B1));
        st_c[lane] = c0 | (c1 << 16);
      }
      // One step: lane l relaxes its two rows of each half, the upper at column j = tt - l + 1 and the
      // lower at j - D.  Near the matrix edges (CK) a half outside it keeps its state unchanged.
      auto step = [&](int tt, int in_top_h, int in_top_e, int in_top_c, auto checked, int* hk) {
        constexpr bool CK = decltype(checked)::value;
        const int j0 = tt - lane + 1, j1 = j0 - D;
        const int in_h = dpp_shr1(in_top_h, bot_h);
        const int in_e = dpp_shr1(in_top_e, bot_e);
        const int in_c = dpp_shr1(in_top_c, cur_c);
        cur_c = in_c;
        const int c1s = (int)((uint32_t)in_c >> 16);
        const uint32_t wu = PROF == kProfLane ? lpu[in_c & 0xffff] : 0u;
        const uint32_t wl = PROF == kProfLane ? lpl[c1s] : 0u;
        const bool ok0 = !CK || (j0 >= 1 && j0 <= m), ok1 = !CK || (j1 >= 1 && j1 <= m);
        const int keep = (ok0 ? 0 : 0xffff) | (ok1 ? 0 : (int)0xffff0000u);  // bits left unchanged
        auto sel = [&](int old, int nw) { return CK ? ((keep & old) | (~keep & nw)) : nw; };
        int hd = diag, hup = in_h, eup = in_e;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const int hlo = hl[r];
          const int e = AFFINE ? pmax(eup, padd(hup, go2)) : hup;
          const int ff = AFFINE ? pmax(padd(f[r], ge2), padd(hlo, goe2)) : padd(hlo, ge2);
          // sigma - ge of both halves' cells side by side: register bytes picked by bit-field extracts
          // (kProfReg), or the 16-bit halves of the two halves' profile words (kProfLane)
          int sg;
          if constexpr (PROF == kProfLane) {
            sg = (int)__builtin_amdgcn_perm(wl, wu, r ? 0x07060302u : 0x05040100u);
          } else {
            sg = (int)__builtin_amdgcn_perm((uint32_t)__builtin_amdgcn_sbfe(prof[1][r], c1s, 8),
                                            (uint32_t)__builtin_amdgcn_sbfe(prof[0][r], in_c, 8), 0x05040100u);
          }
          const int d = padd(hd, sg);
          const int h = pmax(pmax(d, pmax(e, ff)), nu[r]);
          if (CK) {
            // exact cell-by-cell optimum tracking, per half
            const int v0 = lo16(h), v1 = hi16(h);
            if (ok0 && v0 > lo16(bvr[r])) {
              bvA[0][r] = v0 + B0;
              bjA[0][r] = j0;
              bvr[r] = pack16(v0, hi16(bvr[r]));
            }
            if (ok1 && v1 > hi16(bvr[r])) {
              bvA[1][r] = v1 + B1;
              bjA[1][r] = j1;
              bvr[r] = pack16(lo16(bvr[r]), v1);
            }
          } else {
            hk[r] = h;
          }
          f[r] = sel(f[r], ff);
          hl[r] = sel(hlo, h);
          hd = hlo;
          hup = h;
          eup = e;
        }
        bot_h = sel(bot_h, hup);
        bot_e = sel(bot_e, eup);
        diag = sel(diag, in_h);
        out_h = dpp_shl1(bot_h, out_h);
        out_e = dpp_shl1(bot_e, out_e);
      };
      for (int g4 = 0; g4 < BLK / 4; ++g4) {
        const int t0 = tb + 4 * g4;
        const int4 vh = reinterpret_cast<const int4*>(st_h)[g4];
        const int4 ve = reinterpret_cast<const int4*>(st_e)[g4];
        const int4 vc = reinterpret_cast<const int4*>(st_c)[g4];
        if (t0 >= 63 + D && t0 + 3 < m) {
          // both halves of every lane inside the matrix: optima tracked per 4 steps
          int hk[4][2];
          step(t0, vh.x, ve.x, vc.x, std::false_type(), hk[0]);
          step(t0 + 1, vh.y, ve.y, vc.y, std::false_type(), hk[1]);
          step(t0 + 2, vh.z, ve.z, vc.z, std::false_type(), hk[2]);
          step(t0 + 3, vh.w, ve.w, vc.w, std::false_type(), hk[3]);
          int mk[2];
          bool imp = false;
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            mk[r] = pmax(pmax(hk[0][r], hk[1][r]), pmax(hk[2][r], hk[3][r]));
            imp |= pmax(mk[r], bvr[r]) != bvr[r];
          }
          if (imp) {
#pragma unroll
            for (int r = 0; r < 2; ++r) {
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                auto half = [&](int x) { return h ? hi16(x) : lo16(x); };
                const int mv = half(mk[r]);
                int k = half(hk[2][r]) == mv ? 2 : 3;
                k = half(hk[1][r]) == mv ? 1 : k;
                k = half(hk[0][r]) == mv ? 0 : k;
                const bool up = mv > half(bvr[r]);
                bjA[h][r] = lane_select(up, t0 - lane + 1 - (h ? D : 0) + k, bjA[h][r]);
                bvA[h][r] = max(bvA[h][r], mv + (h ? B1 : B0));
              }
              bvr[r] = pmax(bvr[r], mk[r]);
            }
          }
        } else {
          step(t0, vh.x, ve.x, vc.x, std::true_type(), nullptr);
          step(t0 + 1, vh.y, ve.y, vc.y, std::true_type(), nullptr);
          step(t0 + 2, vh.z, ve.z, vc.z, std::true_type(), nullptr);
          step(t0 + 3, vh.w, ve.w, vc.w, std::true_type(), nullptr);
        }
      }
      // lanes 64-BLK.. hold lane 63's outputs of steps tb..tb+BLK-1: the upper half's bottom row at
      // columns step - 62 (kept for the lower half) and the band's bottom row at step - 62 - D
      const int so = tb + (lane - (64 - BLK));
      const bool inw = lane >= 64 - BLK;
      const int cu = so - 62, cl = so - 62 - D;
      if (inw && cu >= 1 && cu <= m) dl[cu % kDelayRing] = make_int2(unrel16(lo16(out_h), B0), unrel16(lo16(out_e), B0));
      if (has_out) {
        const int hi = min(tb + BLK - 63 - D, m);
        if (hi >= 1) {
          if (!lds_wait_ge(&con[wib + 1], hi - kRing)) {  // the band below has read what this overwrites
            failed = true;
            break;
          }
          if (inw && cl >= 1 && cl <= m)
            rout[cl % kRing] = make_int2(unrel16(hi16(out_h), B1), unrel16(hi16(out_e), B1));
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
          if (lane == 0) __hip_atomic_store(&pub[wib + 1], hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }

    // band optimum: (score, i, j) over this lane's rows, then across the wave
    int bs = kNeg32, bi = 0, bjj = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int i = i0 + h * HB + 2 * lane + r + 1;
        if (i > n) continue;
        const int sc = bvA[h][r] + i * ge;
        const int jj = bjA[h][r];
        const int ci = flip ? jj : i, cj = flip ? i : jj;
        if (sc > 0 && better(sc, ci, cj, bs, bi, bjj)) {
          bs = sc;
          bi = ci;
          bjj = cj;
        }
      }
    for (int o = 32; o >= 1; o >>= 1) {
      const int s2_ = __shfl_xor(bs, o, 64), i2 = __shfl_xor(bi, o, 64), j2 = __shfl_xor(bjj, o, 64);
      if (better(s2_, i2, j2, bs, bi, bjj)) {
        bs = s2_;
        bi = i2;
        bjj = j2;
      }
    }
    const bool anybad = __any(bad);
    if (lane == 0) W.band_res[t] = make_int4(bs, bi, bjj, (anybad ? 1 : 0) | (failed ? 2 : 0));
  };

  for (;;) {
    if (threadIdx.x == 0) {
      s_t0 = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(W.ticket), (unsigned long long)kWfWavesPerBlock);
      for (int k = 0; k <= kWfWavesPerBlock; ++k) {
        pub[k] = 0;
        con[k] = 0;
      }
      s_err = 0;
    }
    __syncthreads();
    const int64_t t0g = s_t0;
    if (t0g >= n_items) break;  // the same for the whole workgroup
    const bool launch_err = __hip_atomic_load(W.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    if (!launch_err && wib == kWfWavesPerBlock) {
      courier(t0g);
    } else if (!launch_err && t0g + wib < n_items) {
    if constexpr (P16) {
      p16_band(t0g + wib);
    } else {
    const int64_t t = t0g + wib;
    const WfPair pr = W.pairs[np == 1 ? 0 : W.item_pair[t]];
    const int b = (int)(t - pr.item0);
    const int n = pr.n, m = pr.m, nb = pr.nb;
    // rows come from the query array, columns from the subject array, or the reverse when flipped
    const bool flip = pr.flip != 0;
    const uint8_t* __restrict__ q = (flip ? S : Q) + pr.q_off;
    const uint8_t* __restrict__ s = (flip ? Q : S) + pr.s_off;
    // sigma - ge of a (row letter, column letter) pair, taken in the call's (query, subject) order
    auto sig_rc = [&](int cr, int cc) -> int { return flip ? tab[cc * kTab + cr] : tab[cr * kTab + cc]; };

    const int i0 = b * BH;
    int prof[R];  // kProfReg: 4 bytes sigma - ge against letters 0..3; kProfTable: table offset of the letter
    int32_t hl[R], f[R], bv[R], nu[R];
    int bj[R];
    int rowc[R];
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + lane * R + r + 1;
      int c = kPad;
      if (i <= n) {
        c = q[i - 1];
        if (c >= P.alphabet) {
          bad = true;
          c = kPad;
        }
      }
      rowc[r] = c;
      if (PROF == kProfReg) {
        uint32_t w = 0;
        for (int a = 0; a < 4; ++a) {
          const int v = (c < P.alphabet && a < P.alphabet) ? sig_rc(c, a) : -128;
          w |= ((uint32_t)(v & 0xff)) << (8 * a);
        }
        prof[r] = (int)w;
      } else if (PROF == kProfTable) {
        prof[r] = flip ? c : c * kTab;  // the table is indexed [query letter][subject letter]
      } else {
        prof[r] = 0;
      }
      hl[r] = (MODE == ALN_GLOBAL) ? go : -i * ge;  // Hb(i, 0)
      f[r] = kNeg32;
      nu[r] = -i * ge;                                // local floor: H = 0
      bv[r] = kNeg32;
      bj[r] = 0;
    }
    uint32_t* __restrict__ lp = lprof + (PROF == kProfLane ? wib * P.alphabet * 64 + lane : 0);
    if (PROF == kProfLane) {
      // this lane's word per column letter; each lane reads only its own words, so no barrier
      for (int a = 0; a < P.alphabet; ++a) {
        uint32_t w = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int v = rowc[r] < P.alphabet ? sig_rc(rowc[r], a) : -128;
          w |= ((uint32_t)(v & 0xff)) << (8 * r);
        }
        lp[a * 64] = w;
      }
    }
    const int irow0 = i0 + lane * R;  // the row just above this lane's first row
    int32_t diag = (MODE == ALN_GLOBAL) ? (irow0 > 0 ? go : 0) : -irow0 * ge;  // Hb(irow0, 0)
    uint16_t* __restrict__ codes = TB ? W.codes + pr.code_off + (size_t)(b * 64 + lane) * (size_t)m : nullptr;
    int32_t bot_h = 0, bot_e = kNeg32, cur_c = 0, out_h = 0, out_e = 0;
    // semi-global: the band holding row n tracks row n's running maximum
    const bool last_band = (b == nb - 1);
    int32_t brow = -n * ge;  // Hb(n, 0), i.e. H(n, 0) = 0
    int browj = 0;
    const int rn = n - 1 - irow0;  // index of row n among this lane's rows

    bool failed = false;
    int2* __restrict__ rin = ring[wib];       // rows of the band above (b > 0)
    int2* __restrict__ rout = ring[wib + 1];  // this band's bottom row, for the band below
    const bool has_out = b + 1 < nb;
    // Subject letters are loaded one block ahead and turned into profile indices only when their block
    // starts, so the load's latency hides behind a block of steps: the raw letter of column col (-1 past
    // the end), then the index the profile kind uses (0 past the end).
    auto letter_raw = [&](int col) -> int { return col <= m ? (int)s[col - 1] : -1; };
    auto letter_idx = [&](int c) -> int {
      if (c < 0) return 0;
      if (c >= P.alphabet) {
        bad = true;
        c = PROF == kProfTable ? kPad : 0;
      }
      if (PROF == kProfReg) c *= 8;
      if (PROF == kProfLane) c *= 64;
      if (PROF == kProfTable && flip) c *= kTab;
      return c;
    };
    int c_next = lane < BLK ? letter_raw(1 + lane) : -1;

    // LAZY (local, score-only): a row that beats its best in a group of 4 steps keeps that group (its
    // first step sg and its 4 H values sv) instead of finding the first maximal step at once; resolve()
    // turns the kept group into the row's column before any cell-by-cell update and after the band's
    // last step.  The result is the same (a later strict improvement replaces the kept group, as it
    // would replace the column), and the improving groups -- hundreds per band where the bands meet
    // the alignment's diagonal -- cost 20 selects instead of a search.  Every step a band spends there
    // also delays each band below it, which is what the selects save.
    int32_t sv[4][R];
    int sg[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      sg[r] = -1;
      sv[0][r] = sv[1][r] = sv[2][r] = sv[3][r] = 0;
    }
    auto resolve = [&]() {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (sg[r] >= 0) {
          const int32_t mx = max(max(sv[0][r], sv[1][r]), max(sv[2][r], sv[3][r]));
          int k = sv[2][r] == mx ? 2 : 3;
          k = sv[1][r] == mx ? 1 : k;
          k = sv[0][r] == mx ? 0 : k;
          bj[r] = sg[r] - lane + 1 + k;
          sg[r] = -1;
        }
      }
    };

    const int steps = m + 63;
    for (int tb = 0; tb < steps; tb += BLK) {
      // lane-0 inputs for steps tb..tb+BLK-1 (columns tb+1..tb+BLK), held by lanes < BLK
      const int col_in = tb + 1 + lane;
      const int sreg = letter_idx(c_next);
      // consume the previous block's load before issuing the next one: memory counters drain in order,
      // so waiting for the old letter must not also wait for the new load
      asm volatile("" ::"v"(sreg) : "memory");
      c_next = lane < BLK ? letter_raw(col_in + BLK) : -1;
      // The band below's consumption, read together with the input counter: it only grows, so a value
      // that already allows this block's output spares the wait at the block's end.
      const int con_seen =
          has_out ? __hip_atomic_load(&con[wib + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0;
      int32_t th = 0, te = kNeg32;
      if (b == 0) {
        th = (MODE == ALN_GLOBAL) ? go + col_in * ge : 0;
      } else {
        const int need = min(tb + BLK, m);
        if (!lds_wait_ge(&pub[wib], need)) {
          failed = true;
          break;
        }
        if (lane < BLK && col_in <= m) {
          const int2 v = rin[col_in % kRing];
          th = v.x;
          te = v.y;
        }
        // the ring reads are complete before their slots are released to the band above
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (lane == 0) __hip_atomic_store(&con[wib], need, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      if (MODE == ALN_LOCAL) raise_local_floors<R>(bv, nu, th, i0, ge);
      if (lane < BLK) {
        st_h[lane] = th;
        st_e[lane] = te;
        st_c[lane] = sreg;
      }
      // One step: lane l relaxes column j = t - l + 1 for its R rows.  With ckc (checkpointing, wave-uniform)
      // a lane whose column is a multiple of kTileCols also stores its rows' H and F there.
      auto step = [&](int t, int in_top_h, int in_top_e, int in_top_c, auto checked, int32_t* hk, bool ckc) {
        const int j = t - lane + 1;
        const int in_h = dpp_shr1(in_top_h, bot_h);
        const int in_e = dpp_shr1(in_top_e, bot_e);
        const int in_c = dpp_shr1(in_top_c, cur_c);
        cur_c = in_c;
        if (!decltype(checked)::value || (j >= 1 && j <= m)) {
          int32_t hd = diag, hup = in_h, eup = in_e;
          int32_t hn = 0;
          uint32_t word = 0;
          const int pw = PROF == kProfLane ? (int)lp[in_c] : 0;
          // local affine score-only bands fold the floor into E (band.h).  Checkpoint rows then hold the
          // raised E too; the tiles relaxed again from them reproduce every H, and every E on the alignment's
          // path (a local path's E is at least 0, the floor), so the walk reads the same codes.
          constexpr bool kFloorE = MODE == ALN_LOCAL && AFFINE && !TB;
          band_column<MODE, AFFINE, PROF, TB, decltype(checked)::value, R, true, kFloorE>(
              tab, prof, in_c, pw, go, ge, goe, nu, hl, f, bv, bj, hk, j, rn, hd, hup, eup, hn, word);
          if (TB) codes[j - 1] = (uint16_t)word;
          if (MODE == ALN_SEMIGLOBAL && last_band && rn >= 0 && rn < R && hn > brow) {
            brow = hn;
            browj = j;
          }
          if (CKPT && ckc && (j & (kTileCols - 1)) == 0 && j >= kTileCols && j < m) {
            // rows irow0+1..irow0+4 of column j: Hb and Fb, 32 contiguous bytes
            int4* dst = reinterpret_cast<int4*>(W.ckcols + (int64_t)(j / kTileCols - 1) * W.ck_ld + irow0);
            dst[0] = make_int4(hl[0], f[0], hl[1], f[1]);
            dst[1] = make_int4(hl[2], f[2], hl[3], f[3]);
          }
          bot_h = hup;
          bot_e = eup;
          diag = in_h;
        }
        out_h = dpp_shl1(bot_h, out_h);
        out_e = dpp_shl1(bot_e, out_e);
      };
      for (int g4 = 0; g4 < BLK / 4; ++g4) {
        const int t0 = tb + 4 * g4;
        const int4 vh = reinterpret_cast<const int4*>(st_h)[g4];
        const int4 ve = reinterpret_cast<const int4*>(st_e)[g4];
        const int4 vc = reinterpret_cast<const int4*>(st_c)[g4];
        // With checkpoints, some lane's column in these 4 steps is a multiple of kTileCols only when
        // (t0 + 1) mod kTileCols is below 64 or within 3 of kTileCols (a wave-uniform test); such
        // groups take the checked path, which stores the checkpoints, and the fast path stays as is.
        const int u = (t0 + 1) & (kTileCols - 1);
        const bool ck_group = CKPT && (u < 64 || u > kTileCols - 4);
        if (t0 >= 63 && t0 + 3 < m && !ck_group) {
          // every lane is inside the matrix: no range test; local optima are tracked per 4 steps
          int32_t hk[4][R];
          step(t0, vh.x, ve.x, vc.x, std::false_type(), hk[0], false);
          step(t0 + 1, vh.y, ve.y, vc.y, std::false_type(), hk[1], false);
          step(t0 + 2, vh.z, ve.z, vc.z, std::false_type(), hk[2], false);
          step(t0 + 3, vh.w, ve.w, vc.w, std::false_type(), hk[3], false);
          if (MODE == ALN_LOCAL) {
            int32_t mk[R];
            bool imp = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              mk[r] = max(max(hk[0][r], hk[1][r]), max(hk[2][r], hk[3][r]));
              imp |= mk[r] > bv[r];
            }
            if (LAZY && imp) {
              // a row that beat its best keeps the group (resolved later, see resolve)
#pragma unroll
              for (int r = 0; r < R; ++r) {
                const unsigned long long up = __builtin_amdgcn_ballot_w64(mk[r] > bv[r]);
#pragma unroll
                for (int x = 0; x < 4; ++x) sv[x][r] = mask_select(up, hk[x][r], sv[x][r]);
                sg[r] = mask_select(up, t0, sg[r]);
                bv[r] = max(bv[r], mk[r]);
              }
            } else if (imp) {
              // a row that beat its best takes the group's maximum at the first of the 4 steps that
              // reached it, as a cell-by-cell strict update would
#pragma unroll
              for (int r = 0; r < R; ++r) {
                int k = hk[2][r] == mk[r] ? 2 : 3;
                k = hk[1][r] == mk[r] ? 1 : k;
                k = hk[0][r] == mk[r] ? 0 : k;
                bj[r] = lane_select(mk[r] > bv[r], t0 - lane + 1 + k, bj[r]);
                bv[r] = max(bv[r], mk[r]);
              }
            }
          }
        } else {
          if (LAZY) resolve();
          step(t0, vh.x, ve.x, vc.x, std::true_type(), nullptr, CKPT);
          step(t0 + 1, vh.y, ve.y, vc.y, std::true_type(), nullptr, CKPT);
          step(t0 + 2, vh.z, ve.z, vc.z, std::true_type(), nullptr, CKPT);
          step(t0 + 3, vh.w, ve.w, vc.w, std::true_type(), nullptr, CKPT);
        }
      }
      // lanes 64-BLK.. hold lane 63's outputs of steps tb..tb+BLK-1, i.e. columns tb-62..tb+BLK-63
      if (has_out) {
        const int hi = min(tb + BLK - 63, m);
        const int col_out = tb + (lane - (64 - BLK)) - 62;
        const bool mine = lane >= 64 - BLK && col_out >= 1 && col_out <= m;
        if (hi >= 1) {
          // the band below has read what this overwrites
          if (con_seen < hi - kRing && !lds_wait_ge(&con[wib + 1], hi - kRing)) {
            failed = true;
            break;
          }
          if (mine) rout[col_out % kRing] = make_int2(out_h, out_e);
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
          if (lane == 0) __hip_atomic_store(&pub[wib + 1], hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }

    if (LAZY) resolve();
    // band optimum: (score, i, j) over this lane's rows, then across the wave
    int bs = kNeg32, bi = 0, bjj = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = irow0 + r + 1;
      if (i > n) continue;
      int sc = 0, jj = 0;
      bool cand = false;
      if (MODE == ALN_LOCAL) {
        sc = bv[r] + i * ge;
        jj = bj[r];
        cand = sc > 0;
      } else if (MODE == ALN_SEMIGLOBAL) {
        sc = hl[r] + i * ge;  // H(i, m): last-column candidate; row n is handled below
        jj = m;
        cand = (i < n);
      } else {
        sc = hl[r] + i * ge;
        jj = m;
        cand = (i == n);
      }
      // a flipped pair's cell (i, jj) is the call's cell (jj, i)
      const int ci = flip ? jj : i, cj = flip ? i : jj;
      if (cand && better(sc, ci, cj, bs, bi, bjj)) {
        bs = sc;
        bi = ci;
        bjj = cj;
      }
    }
    if (MODE == ALN_SEMIGLOBAL && last_band && rn >= 0 && rn < R) {
      // row n: (n, 0) with H = 0 first, then its running maximum over j in column order
      const int rowv = (browj > 0) ? brow + n * ge : 0;
      const int ci = flip ? browj : n, cj = flip ? n : browj;
      if (better(rowv, ci, cj, bs, bi, bjj)) {
        bs = rowv;
        bi = ci;
        bjj = cj;
      }
    }
    for (int o = 32; o >= 1; o >>= 1) {
      const int s2 = __shfl_xor(bs, o, 64), i2 = __shfl_xor(bi, o, 64), j2 = __shfl_xor(bjj, o, 64);
      if (better(s2, i2, j2, bs, bi, bjj)) {
        bs = s2;
        bi = i2;
        bjj = j2;
      }
    }
    const bool anybad = __any(bad);
    if (lane == 0) W.band_res[t] = make_int4(bs, bi, bjj, (anybad ? 1 : 0) | (failed ? 2 : 0));
    }
    }
    __syncthreads();  // the group's rings and ticket are reused by the next group
  }
}

// One wave per pair: reduces the pair's band optima into its aln_result_t.
// cigar_off, when given, is a batch call's: pair out_idx owns cigar[cigar_off[out_idx] .. cigar_off[out_idx + 1]];
// otherwise the single pair owns cigar_cap words at cigar.
template <int MODE, bool TB>
__global__ __launch_bounds__(256) void wf_finish_kernel(const KParams P, WfWs W, const uint8_t* __restrict__ q,
                                                        const uint8_t* __restrict__ s,
                                                        aln_result_t* __restrict__ out,
                                                        uint32_t* __restrict__ cigar, int64_t cigar_cap,
                                                        const int64_t* __restrict__ cigar_off) {
  __shared__ uint16_t walk_win[TB ? 4 : 1][TB ? kWalkGroups * kWalkCols : 1];
  const int lane = threadIdx.x & 63;
  const int np = *W.n_pairs;
  const bool err = __hip_atomic_load(W.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  for (int k = blockIdx.x * 4 + (threadIdx.x >> 6); k < np; k += gridDim.x * 4) {
    const WfPair pr = W.pairs[k];
    int bs = kNeg32, bi = 0, bj = 0, flag = 0;
    for (int b = lane; b < pr.nb; b += 64) {
      const int4 v = W.band_res[pr.item0 + b];
      flag |= v.w;
      if (better(v.x, v.y, v.z, bs, bi, bj)) {
        bs = v.x;
        bi = v.y;
        bj = v.z;
      }
    }
    if (pr.nb == 0) {
      // a pair with an empty side has no bands, whose relaxation checks the letters: check them here
      const uint8_t* rq = (pr.flip ? s : q) + pr.q_off;  // the pair's row and column letters
      const uint8_t* rs = (pr.flip ? q : s) + pr.s_off;
      for (int k = lane; k < pr.n; k += 64)
        if (rq[k] >= P.alphabet) flag |= 1;
      for (int k = lane; k < pr.m; k += 64)
        if (rs[k] >= P.alphabet) flag |= 1;
    }
    for (int o = 32; o >= 1; o >>= 1) {
      const int s2 = __shfl_xor(bs, o, 64), i2 = __shfl_xor(bi, o, 64), j2 = __shfl_xor(bj, o, 64);
      flag |= __shfl_xor(flag, o, 64);
      if (better(s2, i2, j2, bs, bi, bj)) {
        bs = s2;
        bi = i2;
        bj = j2;
      }
    }
    // every lane now holds the same optimum; the result is computed by all and written by lane 0
    const int n = pr.flip ? pr.m : pr.n, m = pr.flip ? pr.n : pr.m;  // the call's query and subject lengths
    aln_result_t r;
    r.q_begin = -1;
    r.s_begin = -1;
    r.cigar_len = 0;
    r.reserved = 0;
    r.flags = 0;
    if (P.mode == ALN_GLOBAL) {
      r.q_end = n;
      r.s_end = m;
      r.score = (n == 0 || m == 0) ? ((n + m > 0) ? P.go + (n + m) * P.ge : 0) : bs;
    } else if (n == 0 || m == 0 || bs < 0 || (bs == 0 && P.mode == ALN_LOCAL)) {
      // local: the empty alignment at (0,0); semi-global: the first candidate (0, m), or (0, 0) if a side is empty
      r.score = 0;
      r.q_end = 0;
      r.s_end = (P.mode == ALN_SEMIGLOBAL && n > 0) ? m : 0;
    } else if (P.mode == ALN_SEMIGLOBAL && bs == 0) {
      r.score = 0;  // (0, m) precedes every other candidate in row-major order
      r.q_end = 0;
      r.s_end = m;
    } else {
      r.score = bs;
      r.q_end = bi;
      r.s_end = bj;
    }
    if (err || (flag & 2)) r.flags |= ALN_RES_DEVICE_ERROR;
    if (flag & 1) {
      r.flags |= ALN_RES_BAD_CODE;
      r.score = 0;
      r.q_end = 0;
      r.s_end = 0;
    }
    if (TB && r.flags == 0) {
      // The codes form a [row group][column] array of 16-bit words, 4 rows per word (band bb, lane L
      // is row group bb * 64 + L); walk_core walks them with the whole wave.
      uint32_t* cg = cigar;
      int64_t cap = cigar_cap;
      if (cigar_off) {
        const int64_t c0 = cigar_off[pr.out_idx];
        cg = cigar + c0;
        cap = cigar_off[pr.out_idx + 1] - c0;
      }
      WalkState S;
      walk_start(S, r.q_end, r.s_end);
      walk_core<MODE>(W.codes + pr.code_off, m, 0, 0, S, walk_win[threadIdx.x >> 6], lane, cg, cap);
      const int64_t runs = walk_finish(S, lane, cg, cap);
      r.q_begin = S.i;
      r.s_begin = S.j;
      r.cigar_len = (int)runs;
      if (runs > cap) r.flags |= ALN_RES_CIGAR_TRUNC;
      if (S.stuck) r.flags |= ALN_RES_DEVICE_ERROR;
    }
    if (lane == 0) out[pr.out_idx] = r;
  }
}

// Before a wavefront launch: clears the progress counter of every item and the ticket, and maps
// every item to its pair.
__global__ void wf_reset_kernel(WfWs W) {
  const int64_t n_items = *W.n_items;
  const int np = *W.n_pairs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_items; k += stride) W.flags[k] = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 2 * (int64_t)W.n_lv - 1; k += stride)
    W.lv[k] = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < np; k += stride) {
    const WfPair pr = W.pairs[k];
    for (int b = 0; b < pr.nb; ++b) W.item_pair[pr.item0 + b] = (int)k;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *W.ticket = 0;
    *W.error = 0;
  }
}

// The order in which the per-band engine hands out its items: level by level, band 0 of every pair
// (in the planner's order, largest band work first), then band 1 of every pair, and so on.  Pair-major
// order handed out all the bands of a pair at once, and band b then waited about b lags for the bands
// above it, idle -- a fifth of the waves' time on square pairs, whatever their size -- while other
// pairs' bands could have run.  Level by level, a band is handed out only after every band of the
// level above, so band b - 1 of its pair is always already running (no deadlock, whatever the
// residency) and usually far ahead.  On the uneven protein batch this took the call from 250 to 175 ms;
// chunks of 64 to 16384 pairs ordered this way, one chunk after the other, gave 230 to 177.
//
// W.lv: [0] the largest band count, [1 .. L] the pairs with exactly b bands, then the first position
// of level b, [L + 1 ..] the level cursors (L = W.n_lv - 1 entries each, cleared by wf_reset_kernel).
__global__ __launch_bounds__(256) void wf_level_hist_kernel(WfWs W) {
  const int np = *W.n_pairs;
  const int L = W.n_lv - 1;
  const int lane = threadIdx.x & 63;
  int mx = 0;
  for (int64_t p0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); p0 < np;
       p0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = p0 + lane;
    const int nb = p < np ? W.pairs[p].nb : 0;
    mx = max(mx, nb);
    // one atomic per distinct band count among the wave's pairs (the planner's order keeps them few)
    bool left = nb > 0 && nb <= L;
    while (__builtin_amdgcn_ballot_w64(left) != 0) {
      const unsigned long long lm = __builtin_amdgcn_ballot_w64(left);
      const int first = (int)__builtin_ctzll(lm);
      const int v = __shfl(nb, first, 64);
      const bool same = left && nb == v;
      const unsigned long long sm = __builtin_amdgcn_ballot_w64(same);
      if (lane == first) atomicAdd(&W.lv[v], (int)__builtin_popcountll(sm));
      left = left && !same;
    }
  }
  mx = __ockl_wfred_max_i32(mx);
  if (lane == 0 && mx > 0) atomicMax(&W.lv[0], min(mx, L));
}

// One block: level b holds the pairs with more than b bands; its items start after those of levels
// 0 .. b - 1.  Overwrites the histogram with the first position of every level.
__global__ __launch_bounds__(1024) void wf_level_scan_kernel(WfWs W) {
  __shared__ int64_t part[1024];
  const int L = min(W.lv[0], W.n_lv - 1);
  // cnt(b) = pairs with more than b bands = sum of hist[h], h > b; then the exclusive prefix of cnt
  int64_t run_cnt = 0;  // pairs with more than the current chunk's bands (suffix sum so far)
  // levels in chunks of 1024, from the top: cnt needs a suffix sum over the histogram
  const int chunks = (L + 1023) / 1024;
  // pass 1: cnt(b) in place of hist(b + 1) (hist(b + 1) is read before it is overwritten)
  for (int c = chunks - 1; c >= 0; --c) {
    const int b = c * 1024 + threadIdx.x;  // level b counts hist[b + 1 .. L]
    const int64_t h = (b < L) ? (int64_t)W.lv[b + 1] : 0;
    part[threadIdx.x] = h;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // suffix sums within the chunk
      const int64_t a = threadIdx.x + o < 1024 ? part[threadIdx.x + o] : 0;
      __syncthreads();
      part[threadIdx.x] += a;
      __syncthreads();
    }
    const int64_t cnt = part[threadIdx.x] + run_cnt;
    const int64_t chunk_total = part[0];
    __syncthreads();
    if (b < L) W.lv[b + 1] = (int)cnt;  // now cnt(b) at lv[b + 1]
    run_cnt += chunk_total;
    __syncthreads();
  }
  // pass 2: exclusive prefix of cnt over the levels: the first position of level b, at lv[b + 1]
  int64_t run = 0;
  for (int c = 0; c < chunks; ++c) {
    const int b = c * 1024 + threadIdx.x;
    const int64_t v = (b < L) ? (int64_t)W.lv[b + 1] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t a = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
      __syncthreads();
      part[threadIdx.x] += a;
      __syncthreads();
    }
    const int64_t incl = part[threadIdx.x];
    const int64_t total = part[1023];
    __syncthreads();
    if (b < L) W.lv[b + 1] = (int)(run + incl - v);
    run += total;
    __syncthreads();
  }
}

// One wave per 64 consecutive pairs: each level's items of the wave's pairs get consecutive positions
// from the level's cursor, in pair order.
__global__ __launch_bounds__(256) void wf_order_kernel(WfWs W) {
  const int np = *W.n_pairs;
  const int L = W.n_lv - 1;
  const int lane = threadIdx.x & 63;
  const int64_t nchunks = ((int64_t)np + 63) / 64;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int64_t waves = (int64_t)gridDim.x * blockDim.x / 64;
  int* cur = W.lv + 1 + L;
  for (int64_t c = wave0; c < nchunks; c += waves) {
    const int64_t p = c * 64 + lane;
    int nb = 0;
    int64_t it0 = 0;
    if (p < np) {
      const WfPair pr = W.pairs[p];
      nb = pr.nb <= L ? pr.nb : 0;
      it0 = pr.item0;
    }
    const int wmax = __ockl_wfred_max_i32(nb);
    // 64 levels at a time: lane u counts the wave's pairs at level b0 + u, reserves their places with one
    // atomic (all lanes' atomics in one instruction) and reads the level's first position
    for (int b0 = 0; b0 < wmax; b0 += 64) {
      const int nl = min(64, wmax - b0);
      int mycnt = 0;
      for (int u = 0; u < nl; ++u) {
        const int cnt = (int)__builtin_popcountll(__builtin_amdgcn_ballot_w64(b0 + u < nb));
        if (lane == u) mycnt = cnt;
      }
      int mybase = 0;
      if (lane < nl && mycnt > 0) mybase = W.lv[1 + b0 + lane] + atomicAdd(&cur[b0 + lane], mycnt);
      for (int u = 0; u < nl; ++u) {
        const int b = b0 + u;
        const bool has = b < nb;
        const unsigned long long mask = __builtin_amdgcn_ballot_w64(has);
        const int at = __shfl(mybase, u, 64);
        const int rank = (int)__builtin_popcountll(mask & ((1ull << lane) - 1ull));
        if (has) W.order[(int64_t)at + rank] = it0 + b;
      }
    }
  }
}

// align_long: describes the single pair as the only entry of the pair table.
__global__ void wf_single_pair_kernel(WfWs W, int n, int m, int band_rows) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    WfPair p;
    p.q_off = 0;
    p.s_off = 0;
    p.n = n;
    p.m = m;
    p.nb = (n > 0 && m > 0) ? (n + band_rows - 1) / band_rows : 0;
    p.item0 = 0;
    p.row_off = 0;
    p.code_off = 0;
    p.out_idx = 0;
    p.flip = 0;
    p.pad_ = 0;
    W.pairs[0] = p;
    *W.n_pairs = 1;
    *W.n_items = p.nb;
  }
}

// Packed 16-bit bands are exact when a block's scores stay within int16 of its offsets: a block's
// cells lie within 128 rows and 63 + 32 columns of the offset's cell, and the block's own 32 steps
// move the offset's column by at most 32 more; adjacent cells differ by at most max|sigma| + |go| +
// 2|ge| (row bias included), and E, F lie within |go + ge| of a neighbouring H.  Bounding that step
// by 32 keeps every value of a block within (128 + 95 + 32) x 32 = 8,160 of its offset, far from the
// -32,768 that stands for -infinity.
bool p16_exact(const KParams& kp) {
  const int64_t smax = kp.sigma_max > -kp.sigma_min ? kp.sigma_max : -(int64_t)kp.sigma_min;
  const int64_t step = smax - kp.go - 2 * (int64_t)kp.ge;
  return step <= 32;
}

template <int MODE, bool AFFINE, int PROF, bool TB>
void launch_wf_t(const KParams& kp, const uint8_t* q, const uint8_t* s, const WfWs& W, int n_waves, bool grouped,
                 bool p16, hipStream_t stream) {
  const int blocks = (n_waves + kWfWavesPerBlock - 1) / kWfWavesPerBlock;
  const size_t lds = PROF == kProfLane ? (size_t)kWfWavesPerBlock * kp.alphabet * 64 * sizeof(uint32_t) : 0;
  constexpr bool kCanPack = MODE == ALN_LOCAL && (PROF == kProfReg || PROF == kProfLane) && !TB;
  if (kCanPack && grouped && p16 && p16_exact(kp)) {
    // packed bands keep two 16-bit rows of each half per letter and lane: twice the words
    ProfScope prof("wavefront_p16", stream);
    hipLaunchKernelGGL((wf_i32_group_kernel<MODE, AFFINE, PROF, TB, kWfR, kCanPack, false, false>), dim3(blocks),
                       dim3(kWfBlock), 2 * lds, stream, kp, q, s, W);
    return;
  }
  if (!TB && W.ckcols) {
    ProfScope prof("wavefront_i32_checkpoints", stream);
    hipLaunchKernelGGL((wf_i32_group_kernel<MODE, AFFINE, PROF, false, kWfR, false, !TB, false>), dim3(blocks),
                       dim3(kWfBlock), lds, stream, kp, q, s, W);
    return;
  }
  ProfScope prof(TB ? "wavefront_i32_traceback" : "wavefront_i32", stream);
  // one long pair, local and score-only: improving groups are kept and resolved later (LAZY)
  constexpr bool kLazy = MODE == ALN_LOCAL && !TB;
  if (grouped && kLazy && W.one_pair)
    hipLaunchKernelGGL((wf_i32_group_kernel<MODE, AFFINE, PROF, TB, kWfR, false, false, kLazy>), dim3(blocks),
                       dim3(kWfBlock), lds, stream, kp, q, s, W);
  else if (grouped)
    hipLaunchKernelGGL((wf_i32_group_kernel<MODE, AFFINE, PROF, TB, kWfR, false, false, false>), dim3(blocks),
                       dim3(kWfBlock), lds, stream, kp, q, s, W);
  else
    hipLaunchKernelGGL((wf_i32_kernel<MODE, AFFINE, PROF, TB, kWfR>), dim3(blocks), dim3(kWfBlockAlone), lds,
                       stream, kp, q, s, W);
}

template <int MODE, bool AFFINE, bool TB>
void launch_wf_p(const KParams& kp, const uint8_t* q, const uint8_t* s, const WfWs& W, int nw, bool grouped, bool p16,
                 hipStream_t st) {
  const bool bytes = kp.sigma_max - kp.ge <= 127 && kp.sigma_min - kp.ge >= -127;
  if (bytes && kp.alphabet <= 4)
    launch_wf_t<MODE, AFFINE, kProfReg, TB>(kp, q, s, W, nw, grouped, p16, st);
  else if (bytes)
    launch_wf_t<MODE, AFFINE, kProfLane, TB>(kp, q, s, W, nw, grouped, p16, st);
  else
    launch_wf_t<MODE, AFFINE, kProfTable, TB>(kp, q, s, W, nw, grouped, false, st);
}

template <int MODE, bool TB>
void launch_wf_m(const KParams& kp, const uint8_t* q, const uint8_t* s, const WfWs& W, int nw, bool grouped, bool p16,
                 hipStream_t st) {
  if (kp.go != 0)
    launch_wf_p<MODE, true, TB>(kp, q, s, W, nw, grouped, p16, st);
  else
    launch_wf_p<MODE, false, TB>(kp, q, s, W, nw, grouped, p16, st);
}

template <int MODE>
void launch_wf_mode(const KParams& kp, const uint8_t* q, const uint8_t* s, const WfWs& W, int nw, bool grouped, bool tb,
                    bool p16, aln_result_t* out, uint32_t* cigar, int64_t cap, const int64_t* cigar_off,
                    hipStream_t st) {
  if (tb) {
    launch_wf_m<MODE, true>(kp, q, s, W, nw, grouped, false, st);
    hipLaunchKernelGGL((wf_finish_kernel<MODE, true>), dim3(256), dim3(256), 0, st, kp, W, q, s, out, cigar, cap,
                       cigar_off);
  } else {
    launch_wf_m<MODE, false>(kp, q, s, W, nw, grouped, p16, st);
    hipLaunchKernelGGL((wf_finish_kernel<MODE, false>), dim3(256), dim3(256), 0, st, kp, W, q, s, out, cigar, cap,
                       cigar_off);
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int wf_waves(int per_cu) {
  const int cus = device_cu_count();
  if (per_cu < 1 || per_cu > kWfWavesPerCUMax) return -1;
  return cus > 0 ? cus * per_cu : -1;
}

size_t wf_layout(int64_t max_pairs, int64_t max_items, int64_t row_words, int64_t code_words, WfOffsets* o) {
  size_t off = 0;
  o->pairs = off;
  off += align256((size_t)max_pairs * sizeof(WfPair));
  o->rows = off;
  off += align256((size_t)row_words * sizeof(int2));
  o->flags = off;
  off += align256((size_t)(max_items + 1) * sizeof(int));
  o->item_pair = off;
  off += align256((size_t)(max_items + 1) * sizeof(int));
  o->res = off;
  off += align256((size_t)(max_items + 1) * sizeof(int4));
  o->misc = off;
  off += 256;
  o->codes = off;
  off += align256((size_t)code_words * sizeof(uint16_t));
  o->order = off;
  off += align256((size_t)(max_items + 1) * sizeof(int64_t));
  // a pair has at most max_items bands
  o->n_lv = max_items + 2;
  o->lv = off;
  off += align256((size_t)(2 * o->n_lv - 1) * sizeof(int));
  return off;
}

WfWs wf_view(void* base_, const WfOffsets& o) {
  char* base = static_cast<char*>(base_);
  WfWs W;
  W.pairs = reinterpret_cast<WfPair*>(base + o.pairs);
  W.rows = reinterpret_cast<int2*>(base + o.rows);
  W.flags = reinterpret_cast<int*>(base + o.flags);
  W.item_pair = reinterpret_cast<int*>(base + o.item_pair);
  W.band_res = reinterpret_cast<int4*>(base + o.res);
  W.ticket = reinterpret_cast<int64_t*>(base + o.misc);
  W.n_items = reinterpret_cast<int64_t*>(base + o.misc + 8);
  W.n_pairs = reinterpret_cast<int*>(base + o.misc + 16);
  W.error = reinterpret_cast<int*>(base + o.misc + 20);
  W.codes = reinterpret_cast<uint16_t*>(base + o.codes);
  W.ckcols = nullptr;
  W.ck_ld = 0;
  W.one_pair = 0;
  W.order = reinterpret_cast<int64_t*>(base + o.order);
  W.lv = reinterpret_cast<int*>(base + o.lv);
  W.n_lv = (int)o.n_lv;
  return W;
}

aln_status_t launch_wf_i32(const KParams& kp, const WfWs& W, const uint8_t* q, const uint8_t* s,
                           aln_result_t* out, int max_waves, bool grouped, bool tb, bool p16, uint32_t* cigar,
                           int64_t cigar_cap, hipStream_t stream, const int64_t* cigar_off) {
  hipLaunchKernelGGL(wf_reset_kernel, dim3(256), dim3(256), 0, stream, W);
  if (!grouped) {
    hipLaunchKernelGGL(wf_level_hist_kernel, dim3(256), dim3(256), 0, stream, W);
    hipLaunchKernelGGL(wf_level_scan_kernel, dim3(1), dim3(1024), 0, stream, W);
    hipLaunchKernelGGL(wf_order_kernel, dim3(256), dim3(256), 0, stream, W);
  }
  switch (kp.mode) {
    case ALN_GLOBAL:
      launch_wf_mode<ALN_GLOBAL>(kp, q, s, W, max_waves, grouped, tb, p16, out, cigar, cigar_cap, cigar_off, stream);
      break;
    case ALN_LOCAL:
      launch_wf_mode<ALN_LOCAL>(kp, q, s, W, max_waves, grouped, tb, p16, out, cigar, cigar_cap, cigar_off, stream);
      break;
    default:
      launch_wf_mode<ALN_SEMIGLOBAL>(kp, q, s, W, max_waves, grouped, tb, p16, out, cigar, cigar_cap, cigar_off,
                                     stream);
      break;
  }
  return hipGetLastError() == hipSuccess ? ALN_OK : ALN_E_DEVICE;
}

// ---------------------------------------------------------------------------------------------
// aln_align_long: the engine on one pair.
// ---------------------------------------------------------------------------------------------
aln_status_t plan_long(int64_t n, int64_t m, bool tb, LongPlan* pl) {
  pl->nb = (n + kWfBand - 1) / kWfBand;
  pl->tb = tb;
  const int nw = wf_waves(kWfWavesPerCUDefault);
  if (nw <= 0) return ALN_E_DEVICE;
  int64_t waves = nw;
  const int64_t want = (pl->nb + kWfWavesPerBlock - 1) / kWfWavesPerBlock * kWfWavesPerBlock;
  if (want < waves) waves = want;
  if (waves < kWfWavesPerBlock) waves = kWfWavesPerBlock;
  pl->n_waves = (int)waves;
  const int64_t code_words = tb ? pl->nb * 64 * m : 0;
  pl->total_bytes = wf_layout(1, pl->nb, 2 * (m + 1), code_words, &pl->off);
  return ALN_OK;
}

void launch_single_pair(const WfWs& W, int n, int m, hipStream_t stream) {
  hipLaunchKernelGGL(wf_single_pair_kernel, dim3(1), dim3(64), 0, stream, W, n, m, kWfBand);
}

aln_status_t launch_long(const KParams& kp, const LongPlan& pl, const uint8_t* q, int64_t n, const uint8_t* s,
                         int64_t m, aln_result_t* out, uint32_t* cigar, int64_t cigar_cap, void* ws,
                         hipStream_t stream) {
  WfWs W = wf_view(ws, pl.off);
  W.one_pair = 1;
  hipLaunchKernelGGL(wf_single_pair_kernel, dim3(1), dim3(64), 0, stream, W, (int)n, (int)m, kWfBand);
  // one pair: its bands are few per SIMD, so the grouped engine (no device-memory stalls in the
  // compute waves) is the faster one
  return launch_wf_i32(kp, W, q, s, out, pl.n_waves, true, pl.tb, false, cigar, cigar_cap, stream);
}

}  // namespace mialign
