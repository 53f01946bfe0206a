/*
 * Reference oracle for pairwise alignment: TEST INFRASTRUCTURE ONLY.
 * Loaded by the test suite, the smoke check and the benchmark's CPU-baseline
 * leg; never by the product library.  See oracle.c for what it computes and
 * which passage of the paper each part follows.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GLOBAL = 0, ORC_LOCAL = 1, ORC_SEMIGLOBAL = 2 };
enum { ORC_OP_M = 0, ORC_OP_I = 1, ORC_OP_D = 2 };
enum { ORC_CIGAR_TRUNC = 2, ORC_BAD_CODE = 4 };

typedef struct {
  int32_t mode;          /* ORC_GLOBAL / ORC_LOCAL / ORC_SEMIGLOBAL */
  int32_t alphabet_size; /* codes are 0..alphabet_size-1 */
  const int32_t* sigma;  /* alphabet_size^2, row-major sigma[q*A + s] */
  int64_t gap_open;      /* <= 0 */
  int64_t gap_extend;    /* < 0; a gap of length k scores gap_open + k*gap_extend */
} orc_scoring;

typedef struct {
  int64_t score;
  int64_t q_begin, q_end; /* aligned query region q[q_begin:q_end]; begin = -1 when score-only */
  int64_t s_begin, s_end;
  int64_t cigar_len;      /* runs written (or required when truncated) */
  int64_t flags;          /* ORC_CIGAR_TRUNC | ORC_BAD_CODE */
} orc_result;

/* Full H/E/F matrices in int64; traceback when want_cigar.  Returns 0, or -1 on allocation failure. */
int orc_align_affine_full(const orc_scoring* sc, const uint8_t* q, int64_t n, const uint8_t* s, int64_t m,
                          int want_cigar, orc_result* res, uint32_t* cigar, int64_t cigar_cap);
/* The same results as orc_align_affine_full with a traceback, in linear space: every block_rows-th row of
 * H and E kept by the forward pass, one block of full matrices recomputed at a time for the walk.
 * Returns 0, -1 on allocation failure, -2 for block_rows < 1. */
int orc_align_affine_checkpointed(const orc_scoring* sc, const uint8_t* q, int64_t n, const uint8_t* s, int64_t m,
                                  int64_t block_rows, orc_result* res, uint32_t* cigar, int64_t cigar_cap);
/* One-matrix linear-gap DP (requires gap_open == 0, else returns -2). */
int orc_align_linear_full(const orc_scoring* sc, const uint8_t* q, int64_t n, const uint8_t* s, int64_t m,
                          int want_cigar, orc_result* res, uint32_t* cigar, int64_t cigar_cap);
/* Score and end cell only, two rows of memory. */
int orc_score_affine_linear_space(const orc_scoring* sc, const uint8_t* q, int64_t n, const uint8_t* s,
                                  int64_t m, orc_result* res);
/* Independent pairs over n_threads POSIX threads (full matrices when want_cigar, else linear space). */
int orc_align_batch(const orc_scoring* sc, int64_t n_pairs, const uint8_t* q, const int64_t* q_off,
                    const uint8_t* s, const int64_t* s_off, int want_cigar, orc_result* res, uint32_t* cigar,
                    const int64_t* cigar_off, int n_threads);

#ifdef __cplusplus
}
#endif
#endif
