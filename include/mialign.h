/*
 * mialign -- pairwise sequence alignment on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library.  Every entry point computes the dynamic-programming
 * recurrence of AnySeq Sec. III-A:
 *
 *   H(i,j) = max{ H(i-1,j-1) + sigma(q_i,s_j), E(i,j), F(i,j), nu }     Eq. (1)
 *   E(i,j) = max{ E(i-1,j) + ge, H(i-1,j) + go + ge }                    Eq. (4)
 *   F(i,j) = max{ F(i,j-1) + ge, H(i,j-1) + go + ge }                    Eq. (5)
 *
 * for query Q = q_1..q_n (rows i) and subject S = s_1..s_m (columns j).
 * Scores are signed and added: a gap of length k scores go + k*ge, with
 * go <= 0 and ge < 0 (the paper writes subtracted positive penalties; its
 * experiments use this signed form, Sec. V).  go == 0 is the linear gap model
 * of Eqs. (2)-(3).  The three modes follow the initialisation and optimum
 * rules of Sec. III-A:
 *   ALN_GLOBAL     H(i,0) = go + i*ge, H(0,j) = go + j*ge, nu = -inf, optimum H(n,m);
 *   ALN_LOCAL      H(i,0) = H(0,j) = 0, nu = 0, optimum anywhere;
 *   ALN_SEMIGLOBAL H(i,0) = H(0,j) = 0, nu = -inf, optimum in row n or column m.
 *
 * Conventions where the paper leaves a choice open (all results are unique):
 *   - optimum ties: smallest i, then smallest j; local with best score 0 is
 *     the empty alignment at (0,0);
 *   - traceback priority in the no-gap state: diagonal, then the vertical gap
 *     E (CIGAR I, consumes the query), then the horizontal gap F (CIGAR D),
 *     the order of the relaxation function in Sec. III-B; inside a gap the
 *     gap-open predecessor wins ties; local alignments start at the first
 *     cell with H = 0, semi-global ones on row 0 or column 0.
 *
 * Memory and execution model:
 *   - Pointers documented as DEVICE point to memory the caller allocated on
 *     the current HIP device; HOST pointers are ordinary host memory.
 *   - The library never allocates device memory in aln_align_batch,
 *     aln_align_long or aln_traceback: the caller passes a workspace whose
 *     size it obtains from the matching *_workspace_size call.  All calls are
 *     asynchronous on `stream` and capturable in a HIP graph.
 *   - Host-detectable errors return a negative aln_status_t and enqueue no
 *     device work.  Problems found on the device are reported per pair in
 *     aln_result_t.flags.
 */
#ifndef MIALIGN_H
#define MIALIGN_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t aln_status_t;
#define ALN_OK 0
#define ALN_E_INVALID (-1)     /* a null pointer, negative size or inconsistent argument */
#define ALN_E_ALPHABET (-2)    /* alphabet_size outside 2..32 */
#define ALN_E_SCORING (-3)     /* gap_open > 0, gap_extend >= 0, or scores too large to be exact */
#define ALN_E_WORKSPACE (-4)   /* workspace smaller than the size query returned */
#define ALN_E_DEVICE (-5)      /* a HIP call failed (launch or device query) */
#define ALN_E_UNSUPPORTED (-6) /* a combination the library does not provide */

#define ALN_GLOBAL 0
#define ALN_LOCAL 1
#define ALN_SEMIGLOBAL 2

/* Scoring scheme (Sec. III-C composes a substitution function with a gap scheme). */
typedef struct {
  int32_t mode;          /* ALN_GLOBAL / ALN_LOCAL / ALN_SEMIGLOBAL */
  int32_t alphabet_size; /* 2..32; sequence codes must lie in 0..alphabet_size-1 */
  const int8_t* subst;   /* HOST, alphabet_size^2 row-major sigma(q,s); NULL => match/mismatch */
  int32_t match;         /* sigma(a,a) when subst == NULL */
  int32_t mismatch;      /* sigma(a,b), a != b, when subst == NULL */
  int32_t gap_open;      /* go <= 0; 0 selects the linear model */
  int32_t gap_extend;    /* ge < 0; a gap of length k scores go + k*ge */
} aln_scoring_t;

/* One result per pair, 32 bytes, written by the device. */
typedef struct {
  int32_t score;
  int32_t q_begin, q_end; /* aligned query part is q[q_begin:q_end] (0-based, half-open);
                             q_end is the DP row of the optimum; q_begin = -1 when score-only */
  int32_t s_begin, s_end; /* same for the subject */
  int32_t cigar_len;      /* CIGAR words written, or required when ALN_RES_CIGAR_TRUNC; 0 if score-only */
  uint32_t flags;         /* ALN_RES_* */
  int32_t reserved;
} aln_result_t;

/* call flags */
#define ALN_SCORE_ONLY 0u
#define ALN_TRACEBACK 1u   /* aln_align_batch: also write the canonical CIGAR of every pair */
#define ALN_FORCE_INT32 2u /* skip the packed 16-bit path */
#define ALN_FORCE_INT16 4u /* accepted, no effect: local pairs run in 16 bits under the saturation check
                              (best < 32767) whatever the a-priori bound; kept for existing callers */
#define ALN_LINEAR_SPACE 8u /* aln_align_long with ALN_TRACEBACK: trace back in linear space (checkpoints and
                               tiles relaxed again) also for pairs of at most 2^24 cells */
#define ALN_STORED_CODES 16u /* aln_align_long with ALN_TRACEBACK: store a code per cell also above 2^24 cells
                               (while the codes take at most 64 GiB); ignored with ALN_LINEAR_SPACE */

/* result flags */
#define ALN_RES_INT32_REDO 1u  /* the 16-bit pass saturated; the pair was recomputed in 32 bits */
#define ALN_RES_CIGAR_TRUNC 2u /* CIGAR capacity too small; cigar_len holds the required count */
#define ALN_RES_BAD_CODE 4u    /* a sequence code >= alphabet_size; no score computed */
#define ALN_RES_TOO_LONG 8u    /* n > max_n or m > max_m (the bounds the workspace was sized for) */
#define ALN_RES_DEVICE_ERROR 16u /* a bounded device-side wait gave up; the result is not valid */
#define ALN_RES_BAD_END 32u    /* aln_traceback: the given end cell lies outside the pair's matrix, or H there
                                  differs from the given score; no CIGAR written */

/* CIGAR words: (run_length << 4) | op, op 0 = M (match or mismatch), 1 = I (query letter
 * against a gap), 2 = D (subject letter against a gap), in alignment order. */
#define ALN_CIGAR_M 0u
#define ALN_CIGAR_I 1u
#define ALN_CIGAR_D 2u

/* Bytes of device workspace aln_align_batch needs for n_pairs pairs whose lengths are at most
 * max_n (queries) and max_m (subjects) and sum to total_q / total_s letters, for the given flags.
 * Returns ALN_OK and sets *bytes. */
aln_status_t aln_batch_workspace_size(const aln_scoring_t* scoring, int64_t n_pairs, int64_t max_n,
                                      int64_t max_m, int64_t total_q, int64_t total_s, uint32_t flags,
                                      size_t* bytes);

/* Aligns n_pairs independent pairs.  Small pairs run one pair per lane (inter-sequence parallelism,
 * Sec. VI); in score-only calls, pairs with n*m >= 2^16 run on the band wavefront of aln_align_long
 * instead, all of them sharing one device-wide work queue (the dynamic wavefront of Sec. IV-A),
 * largest first.  The routing is decided on the device, so the host needs no copy of the lengths;
 * aln_align_batch_ex sets the threshold and the other execution choices.
 * In traceback calls the rule is fixed: pairs with n*m >= 2^18, or longer than 1024 on either side,
 * run on the band wavefront and store their 4-bit predecessor codes in an arena of the workspace (about
 * n*m/2 bytes each); the one-pair-per-lane kernels then hold code slabs for pairs up to 1024 x 1024
 * only.  The arena is sized by a bound from max_n, max_m, total_q and total_s; where that bound exceeds
 * the arena budget (aln_set_batch_code_arena, 16 GiB by default) the arena is the budget, pairs take
 * room in the order they reach it, those that find none run one pair per lane, and the lanes' slabs are
 * sized for max_n x max_m (fewer waves in flight, at most 16 GiB of slabs).  Results are identical
 * either way.
 *   q, s          DEVICE  concatenated uint8 codes of all queries / subjects
 *   q_off, s_off  DEVICE  int64[n_pairs+1]; pair k is q[q_off[k]:q_off[k+1]] vs s[s_off[k]:s_off[k+1]]
 *   max_n, max_m  upper bounds of the lengths (pairs above them get ALN_RES_TOO_LONG)
 *   total_q, total_s  q_off[n_pairs] and s_off[n_pairs] (upper bounds suffice)
 *   flags         ALN_SCORE_ONLY or ALN_TRACEBACK, optionally | ALN_FORCE_INT32 / ALN_FORCE_INT16
 *   out           DEVICE  aln_result_t[n_pairs]
 *   cigar         DEVICE  uint32 CIGAR words; pair k owns cigar[cigar_off[k]:cigar_off[k+1]]
 *                         (n + m words always suffice); both NULL unless ALN_TRACEBACK
 *   cigar_off     DEVICE  int64[n_pairs+1]
 *   workspace     DEVICE  at least aln_batch_workspace_size(...) bytes, 256-byte aligned
 * Ownership: the caller owns every buffer; nothing is retained after the call's work completes. */
aln_status_t aln_align_batch(const aln_scoring_t* scoring, int64_t n_pairs, const uint8_t* q, const int64_t* q_off,
                             const uint8_t* s, const int64_t* s_off, int64_t max_n, int64_t max_m, int64_t total_q,
                             int64_t total_s, uint32_t flags, aln_result_t* out, uint32_t* cigar,
                             const int64_t* cigar_off, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Execution choices of a batch call.  None of them changes any result, only how the work is laid
 * out on the device; an autotuner (paper_2002_04561_amd/tune.py) searches them per workload.  A
 * zero field selects the default.
 *   wf_min_cells     score-only calls: pairs with n*m >= wf_min_cells run on the band wavefront
 *                    engine, the others one pair per lane.  0 => 2^16 for a batch of at least
 *                    1024 pairs per compute unit (enough to fill the one-pair-per-lane kernels),
 *                    else 2^12; negative => no pair.
 *   wf_waves_per_cu  persistent waves per compute unit of the wavefront engine, 1..32; 0 => 16,
 *                    or for grouped bands 4 per estimated 4-band group per compute unit, 4..16
 *                    (waves beyond what a compute unit holds start as others finish).
 *   wf_orient        score-only calls: how a wavefront pair is laid out.  The transposed problem
 *                    has the same optimum, and ties are still resolved in the (i, j) order of the
 *                    call.  1 => longer sequence along the band rows; -1 => as given; 2 => whichever
 *                    takes fewer band steps, ceil(rows / 256) * (columns + 255), except that a pair
 *                    of several bands is never laid out with the longer sequence as columns.
 *                    0 => -1.
 *   small_bits       one-pair-per-lane kernels: 16 => packed 16-bit lanes where provably exact,
 *                    with the 32-bit redo; 32 => 32-bit lanes only.  0 => 16.
 *   wf_group         wavefront engine: 1 => every band on its own wave, hand-offs through HBM;
 *                    4 => workgroups of 4 consecutive bands handing rows over in LDS, with a courier
 *                    wave for the hand-offs to and from other workgroups.  0 => 4 when the batch has
 *                    fewer than 56 bands per compute unit (estimated from total_q + total_s), else 1.
 *                    aln_align_long always uses 4.
 *   wf_bits          wavefront engine, grouped bands of score-only local alignments over alphabets
 *                    of up to 32 letters: 16 => packed 16-bit cells (two half bands per lane, scores
 *                    relative to per-block offsets) where the scores' step bound keeps them exact
 *                    (max|sigma| + |gap_open| + 2 |gap_extend| <= 32), else 32-bit lanes; 32 =>
 *                    32-bit lanes only.  0 => 32.  Results are identical either way; the packed
 *                    cells are slower on MI355X (one long pair and the uneven protein batch alike),
 *                    so aln_align_long uses 32. */
typedef struct {
  int64_t wf_min_cells;
  int32_t wf_waves_per_cu;
  int32_t wf_orient;
  int32_t small_bits;
  int32_t wf_group;
  int32_t wf_bits;
  int32_t reserved; /* must be zero */
} aln_batch_config_t;

/* The routing rule aln_align_batch(_ex) applies on the device to a batch of n_pairs pairs with these flags
 * and config (NULL: the defaults): a pair runs on the band wavefront when n*m >= *min_cells or when n or m
 * exceeds *max_side, else one pair per lane.  *min_cells = INT64_MAX means never by cells, *max_side =
 * INT64_MAX no bound on the sides.  Defaults: score-only 2^12 cells, or 2^16 once the batch fills the
 * per-lane kernels (128 pairs x 8 waves per compute unit); traceback 2^18 cells or a side above 1024,
 * whatever the config.  Host only (reads the device's compute-unit count).  Returns ALN_E_INVALID for
 * bad arguments, ALN_E_DEVICE without a device. */
aln_status_t aln_batch_route(int64_t n_pairs, uint32_t flags, const aln_batch_config_t* config, int64_t* min_cells,
                             int64_t* max_side);

/* aln_align_batch with explicit execution choices; config == NULL is aln_align_batch.  The
 * workspace size does not depend on the config.  Returns ALN_E_INVALID for a field out of range. */
aln_status_t aln_align_batch_ex(const aln_scoring_t* scoring, int64_t n_pairs, const uint8_t* q,
                                const int64_t* q_off, const uint8_t* s, const int64_t* s_off, int64_t max_n,
                                int64_t max_m, int64_t total_q, int64_t total_s, uint32_t flags,
                                const aln_batch_config_t* config, aln_result_t* out, uint32_t* cigar,
                                const int64_t* cigar_off, void* workspace, size_t workspace_bytes,
                                hipStream_t stream);

/* aln_align_batch_ex for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, hosts that forbid allocation): the same arguments without a workspace, whose place
 * takes a device scratch array the library holds on each device for the life of the process
 * (aln_noalloc_scratch_bytes(), 64 MiB).  Nothing is allocated: the scratch's device address is looked up
 * once per device.  Returns ALN_E_WORKSPACE, with no device work, when the batch needs more than the
 * scratch (aln_batch_workspace_size); otherwise as aln_align_batch_ex.  Every call on a device shares
 * that device's scratch: calls that overlap on one device (on different streams, or from different
 * threads) race and must not be made. */
aln_status_t aln_align_batch_noalloc(const aln_scoring_t* scoring, int64_t n_pairs, const uint8_t* q,
                                     const int64_t* q_off, const uint8_t* s, const int64_t* s_off, int64_t max_n,
                                     int64_t max_m, int64_t total_q, int64_t total_s, uint32_t flags,
                                     const aln_batch_config_t* config, aln_result_t* out, uint32_t* cigar,
                                     const int64_t* cigar_off, hipStream_t stream);

/* Bytes of the device scratch of aln_align_batch_noalloc. */
size_t aln_noalloc_scratch_bytes(void);

/* Bytes of device workspace aln_traceback needs for n_pairs pairs whose lengths are at most max_n and
 * max_m.  Returns ALN_OK and sets *bytes. */
aln_status_t aln_traceback_workspace_size(const aln_scoring_t* scoring, int64_t n_pairs, int64_t max_n,
                                          int64_t max_m, size_t* bytes);

/* Re-emits the canonical alignment of pairs whose optimum a forward call already found (the traceback
 * of AnySeq Sec. III-A, started from the given end cell; Sec. III-C returns the alignment beside the
 * score).  Pair k's matrix is relaxed again only up to its end cell (fwd[k].q_end, fwd[k].s_end):
 * every value there equals that of the whole matrix, so the walk back from that cell is the one
 * aln_align_batch with ALN_TRACEBACK takes.  Typical use: a batch run score-only, or one whose
 * CIGAR buffers were too small (ALN_RES_CIGAR_TRUNC, cigar_len = the words needed), is traced back
 * for the affected pairs only, into resized buffers.
 *   q, q_off, s, s_off, max_n, max_m   as for aln_align_batch (DEVICE arrays)
 *   fwd           DEVICE  aln_result_t[n_pairs] from aln_align_batch / aln_align_long: score and end cell
 *   out           DEVICE  aln_result_t[n_pairs]; may be the same array as fwd.  score, q_end and s_end
 *                         are fwd's; q_begin, s_begin, cigar_len and flags are set.  A pair whose fwd
 *                         carries ALN_RES_BAD_CODE, ALN_RES_TOO_LONG or ALN_RES_DEVICE_ERROR keeps
 *                         that flag and gets no CIGAR; ALN_RES_BAD_END is set when the end cell lies
 *                         outside the matrix or H there is not fwd's score.
 *   cigar, cigar_off  DEVICE  as for aln_align_batch; ALN_RES_CIGAR_TRUNC when a pair's room is short
 *   workspace     DEVICE  at least aln_traceback_workspace_size(...) bytes, 256-byte aligned
 * Pairs run one per lane in 32-bit lanes, in the order given. */
aln_status_t aln_traceback(const aln_scoring_t* scoring, int64_t n_pairs, const uint8_t* q, const int64_t* q_off,
                           const uint8_t* s, const int64_t* s_off, int64_t max_n, int64_t max_m,
                           const aln_result_t* fwd, aln_result_t* out, uint32_t* cigar, const int64_t* cigar_off,
                           void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Renders an alignment as the two gapped strings of AnySeq's C interface (Sec. III-C): q_aln and
 * s_aln receive the aligned parts of the query and the subject, letters mapped through `letters`
 * (letter k is letters[k]; codes outside it render as '?') and '-' where the other sequence has a
 * letter against a gap.  HOST only; no device work.
 *   q, s            HOST  the pair's codes (the whole sequences)
 *   result          HOST  the pair's result (q_begin, s_begin and cigar_len are used)
 *   cigar           HOST  result->cigar_len CIGAR words
 *   q_aln, s_aln    HOST  buffers of `capacity` chars each; both are NUL-terminated
 * Returns ALN_OK, or ALN_E_INVALID if a pointer is NULL, the CIGAR runs past the sequences, or the
 * alignment (length + 1) does not fit in capacity. */
aln_status_t aln_cigar_to_gapped(const uint8_t* q, int64_t n, const uint8_t* s, int64_t m,
                                 const aln_result_t* result, const uint32_t* cigar, const char* letters,
                                 char* q_aln, char* s_aln, int64_t capacity);

/* Bytes of device workspace aln_align_long needs for an n x m problem and the given flags. */
aln_status_t aln_long_workspace_size(const aln_scoring_t* scoring, int64_t n, int64_t m, uint32_t flags,
                                     size_t* bytes);

/* Aligns one long pair with intra-sequence parallelism: the matrix is relaxed in bands of 256 rows
 * that move as a wavefront across the device (AnySeq Sec. IV-B: tiles relaxed along anti-diagonals,
 * each publishing its last row to the next), all bands drawn from one device-side work queue.
 *   q             DEVICE  n uint8 codes;  s  DEVICE  m uint8 codes
 *   flags         ALN_SCORE_ONLY, or ALN_TRACEBACK to also write the canonical CIGAR, optionally
 *                 | ALN_LINEAR_SPACE or | ALN_STORED_CODES
 *   out           DEVICE  one aln_result_t (q_begin = s_begin = -1 when score-only)
 *   cigar         DEVICE  CIGAR words, cigar_capacity of them (n + m always suffice); NULL when
 *                         score-only.  A short buffer gives ALN_RES_CIGAR_TRUNC and the required count.
 *   workspace     DEVICE  at least aln_long_workspace_size(...) bytes, 256-byte aligned: two bottom-row
 *                         slots of (m + 1) * 8 bytes, plus, with ALN_TRACEBACK, either the 4-bit
 *                         predecessor code of every cell (about n * m / 2 bytes: pairs of at most 2^24
 *                         cells, or with ALN_STORED_CODES while that is at most 64 GiB), or the
 *                         linear-space traceback's checkpoints (the H and E of every 1024th row and the H
 *                         and F of every 2048th column, about n * m / 85 bytes) and one segment of codes
 *                         (aln_set_traceback_budget).  Above 2^24 cells the linear-space traceback is
 *                         also the faster one on MI355X (it writes no code for most cells).
 * Traceback in linear space (Sec. III-A): the forward pass keeps the checkpoints; the walk then goes back
 * through segments of rows, bottom first, relaxing each segment's tiles again from the checkpoints (the
 * same integers as the forward pass) and walking its codes.  At most twice the cells are relaxed.
 * Exactness: 32-bit lanes; the call returns ALN_E_SCORING if the score range of an n x m problem
 * could leave +-2^28. */
aln_status_t aln_align_long(const aln_scoring_t* scoring, const uint8_t* q, int64_t n, const uint8_t* s, int64_t m,
                            uint32_t flags, aln_result_t* out, uint32_t* cigar, int64_t cigar_capacity,
                            void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Most bytes the code arena of a traceback batch (aln_align_batch with ALN_TRACEBACK) may take; the arena
 * holds the predecessor codes of the pairs that run on the band wavefront.  0 restores the default of
 * 16 GiB.  Process-wide; read when a size query or align call is made, so the same value must hold for
 * both.  Returns ALN_E_INVALID for a negative size. */
aln_status_t aln_set_batch_code_arena(int64_t bytes);

/* Bytes of 4-bit predecessor codes a linear-space traceback (aln_align_long with ALN_TRACEBACK above 2^24
 * cells, or with ALN_LINEAR_SPACE) holds at once: the rows of a segment that the traceback relaxes again in one go
 * are as many as fit (at least 1024).  A smaller budget means more segments, each relaxed and walked in
 * turn.  0 restores the default of 4 GiB.  Process-wide; read when a size query or align call is made,
 * so the same value must hold for both.  Returns ALN_E_INVALID for a negative size. */
aln_status_t aln_set_traceback_budget(int64_t bytes);

/* Kernel timing, a profiling aid.  While enabled, every kernel the library enqueues is bracketed by
 * HIP events recorded on the same stream; aln_profile_read waits for those events and returns, per
 * kernel family, the number of launches and their summed device time since the last reset.  Not for
 * use under graph capture (it records events).  Host-side only; returns ALN_OK or ALN_E_INVALID. */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
} aln_profile_entry_t;
aln_status_t aln_profile_enable(int on);
aln_status_t aln_profile_reset(void);
aln_status_t aln_profile_read(aln_profile_entry_t* entries, int32_t max_entries, int32_t* n_entries);

/* Diagnostic aid: how many times a bounded device-side wait polls before it gives up (device-memory
 * waits of the band wavefront's hand-offs, and LDS waits between the bands of a workgroup).  A wait
 * that gives up sets ALN_RES_DEVICE_ERROR on the pairs of its launch instead of blocking; every wave
 * still leaves its kernel.  0 restores a default (2^22 device-memory polls, 2^26 LDS polls, on the
 * order of a second each).  The limits are process-wide and read when an align call is enqueued; a
 * small limit makes waits that would have succeeded give up, which is how tests check that every
 * kernel exits on that path.  Returns ALN_E_INVALID for a negative count. */
aln_status_t aln_set_wait_limits(int64_t device_polls, int64_t lds_polls);

/* Human-readable text of a status code (static storage). */
const char* aln_status_string(aln_status_t status);

/* Library version string. */
const char* aln_version(void);

#ifdef __cplusplus
}
#endif
#endif
