/*
 * Reference oracle for pairwise alignment: TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct scalar C.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load this file's library; the
 * product (the HIP library and its Python binding) never does.  It shares no
 * code, header, table or helper with the HIP path.
 *
 * What it computes (AnySeq, Sec. III-A "Pairwise Sequence Alignment"):
 *   H(i,j) = max{ H(i-1,j-1) + sigma(q_i,s_j), E(i,j), F(i,j), nu }      Eq. (1)
 *   E(i,j) = max{ E(i-1,j) + ge, H(i-1,j) + go + ge }                     Eq. (4)
 *   F(i,j) = max{ F(i,j-1) + ge, H(i,j-1) + go + ge }                     Eq. (5)
 * with signed, added gap scores: a gap of length k scores go + k*ge (the
 * paper writes positive penalties that are subtracted; its experiments use
 * the signed form, Sec. V).  Linear gaps (Eqs. (2)-(3)) are go = 0, and a
 * separate one-matrix implementation of Eqs. (2)-(3) is kept below so the
 * two can be tested against each other.
 *
 * Initialisation and optimum per mode (Sec. III-A, the three paragraphs on
 * local, global and semi-global alignment):
 *   global: H(0,0)=0, H(i,0)=go+i*ge, H(0,j)=go+j*ge, nu=-inf, optimum H(n,m)
 *   local : H(i,0)=H(0,j)=0, nu=0, optimum anywhere
 *   semi  : H(i,0)=H(0,j)=0, nu=-inf (reading: the paper gives semi-global
 *           the local initialisation only), optimum in the last row or column
 *   E(0,j) = F(i,0) = -inf in every mode.
 *
 * Readings where the paper is silent (each is a stated convention):
 *   - optimum ties (local, semi): smallest i, then smallest j, i.e. the first
 *     strict improvement in a row-major scan; local with best 0 ends at (0,0);
 *   - predecessor priority in state H: diagonal, then E (vertical gap, a query
 *     letter against '-', CIGAR I), then F (horizontal gap, CIGAR D), following
 *     the order of the relaxation function in Sec. III-B (substitution first,
 *     a gap replaces it only when strictly better, subject gap before query gap);
 *   - in state E/F the gap-open predecessor wins ties against extension;
 *   - local traceback stops at the first cell in state H whose H is 0; semi
 *     stops on row 0 or column 0; global walks to (0,0), finishing along row 0
 *     or column 0 with one gap run;
 *   - -inf is NEG = -2^40 in int64.
 *
 * CIGAR words are (run_length << 4) | op with op 0 = M, 1 = I (consumes the
 * query), 2 = D (consumes the subject).
 */
#include "oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define NEG ((int64_t)(-(((int64_t)1) << 40)))

static int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

static int check_codes(const uint8_t* x, int64_t len, int32_t alphabet) {
  for (int64_t k = 0; k < len; ++k)
    if ((int32_t)x[k] >= alphabet) return 0;
  return 1;
}

/* Reverses the backward op list and merges equal neighbours into runs. */
static int64_t emit_cigar(const uint8_t* ops_rev, int64_t n_ops, uint32_t* cigar, int64_t cap,
                          int* truncated) {
  int64_t runs = 0;
  int64_t k = n_ops - 1;
  *truncated = 0;
  while (k >= 0) {
    uint8_t op = ops_rev[k];
    int64_t len = 0;
    while (k >= 0 && ops_rev[k] == op) {
      ++len;
      --k;
    }
    if (runs < cap && cigar)
      cigar[runs] = (uint32_t)((len << 4) | op);
    else
      *truncated = 1;
    ++runs;
  }
  return runs;
}

/* ---------------------------------------------------------------------- */
/* Affine (Gotoh) DP with full H/E/F matrices; optional traceback.         */
/* ---------------------------------------------------------------------- */
int orc_align_affine_full(const orc_scoring* sc, const uint8_t* q, int64_t n, const uint8_t* s, int64_t m,
                          int want_cigar, orc_result* res, uint32_t* cigar, int64_t cigar_cap) {
  const int64_t go = sc->gap_open, ge = sc->gap_extend;
  const int32_t A = sc->alphabet_size;
  memset(res, 0, sizeof(*res));
  res->q_begin = res->s_begin = -1;
  if (!check_codes(q, n, A) || !check_codes(s, m, A)) {
    res->flags = ORC_BAD_CODE;
    return 0;
  }
  const int64_t W = m + 1;
  const int64_t cells = (n + 1) * W;
  int64_t* Hm = (int64_t*)malloc(sizeof(int64_t) * cells);
  int64_t* Em = (int64_t*)malloc(sizeof(int64_t) * cells);
  int64_t* Fm = (int64_t*)malloc(sizeof(int64_t) * cells);
  if (!Hm || !Em || !Fm) {
    free(Hm);
    free(Em);
    free(Fm);
    return -1;
  }
#define H_(i, j) Hm[(i) * W + (j)]
#define E_(i, j) Em[(i) * W + (j)]
#define F_(i, j) Fm[(i) * W + (j)]
  /* borders */
  for (int64_t i = 0; i <= n; ++i) {
    E_(i, 0) = NEG;
    F_(i, 0) = NEG;
    H_(i, 0) = (sc->mode == ORC_GLOBAL && i > 0) ? go + i * ge : 0;
  }
  for (int64_t j = 0; j <= m; ++j) {
    E_(0, j) = NEG;
    F_(0, j) = NEG;
    H_(0, j) = (sc->mode == ORC_GLOBAL && j > 0) ? go + j * ge : 0;
  }
  /* recurrence, Eqs. (1), (4), (5) */
  for (int64_t i = 1; i <= n; ++i) {
    for (int64_t j = 1; j <= m; ++j) {
      int64_t e = max2(E_(i - 1, j) + ge, H_(i - 1, j) + go + ge);
      int64_t f = max2(F_(i, j - 1) + ge, H_(i, j - 1) + go + ge);
      int64_t d = H_(i - 1, j - 1) + sc->sigma[q[i - 1] * A + s[j - 1]];
      int64_t h = max2(max2(d, e), f);
      if (sc->mode == ORC_LOCAL) h = max2(h, 0);
      E_(i, j) = e;
      F_(i, j) = f;
      H_(i, j) = h;
    }
  }
  /* optimum */
  int64_t bi = n, bj = m, best = H_(n, m);
  if (sc->mode == ORC_LOCAL) {
    best = H_(0, 0);
    bi = 0;
    bj = 0;
    for (int64_t i = 0; i <= n; ++i)
      for (int64_t j = 0; j <= m; ++j)
        if (H_(i, j) > best) {
          best = H_(i, j);
          bi = i;
          bj = j;
        }
  } else if (sc->mode == ORC_SEMIGLOBAL) {
    int first = 1;
    for (int64_t i = 0; i <= n; ++i)
      for (int64_t j = 0; j <= m; ++j) {
        if (i != n && j != m) continue;
        if (first || H_(i, j) > best) {
          best = H_(i, j);
          bi = i;
          bj = j;
          first = 0;
        }
      }
  }
  res->score = best;
  res->q_end = bi;
  res->s_end = bj;
  if (!want_cigar) {
    free(Hm);
    free(Em);
    free(Fm);
    return 0;
  }
  /* canonical traceback */
  uint8_t* ops = (uint8_t*)malloc((size_t)(n + m + 1));
  int64_t n_ops = 0;
  int64_t i = bi, j = bj;
  int state = 0; /* 0 = H, 1 = E, 2 = F */
  for (;;) {
    if (state == 0) {
      if (sc->mode == ORC_LOCAL && H_(i, j) == 0) break;
      if (sc->mode == ORC_SEMIGLOBAL && (i == 0 || j == 0)) break;
      if (sc->mode == ORC_GLOBAL) {
        if (i == 0 && j == 0) break;
        if (i == 0) {
          while (j > 0) {
            ops[n_ops++] = ORC_OP_D;
            --j;
          }
          break;
        }
        if (j == 0) {
          while (i > 0) {
            ops[n_ops++] = ORC_OP_I;
            --i;
          }
          break;
        }
      }
      int64_t d = H_(i - 1, j - 1) + sc->sigma[q[i - 1] * A + s[j - 1]];
      if (d == H_(i, j)) {
        ops[n_ops++] = ORC_OP_M;
        --i;
        --j;
      } else if (E_(i, j) == H_(i, j)) {
        state = 1;
      } else {
        state = 2;
      }
    } else if (state == 1) {
      ops[n_ops++] = ORC_OP_I;
      if (H_(i - 1, j) + go + ge == E_(i, j)) state = 0;
      --i;
    } else {
      ops[n_ops++] = ORC_OP_D;
      if (H_(i, j - 1) + go + ge == F_(i, j)) state = 0;
      --j;
    }
  }
  res->q_begin = i;
  res->s_begin = j;
  int trunc = 0;
  res->cigar_len = emit_cigar(ops, n_ops, cigar, cigar_cap, &trunc);
  if (trunc) res->flags |= ORC_CIGAR_TRUNC;
  free(ops);
  free(Hm);
  free(Em);
  free(Fm);
#undef H_
#undef E_
#undef F_
  return 0;
}

/* ---------------------------------------------------------------------- */
/* The same alignment in linear space (Sec. III-A: the traceback can run in */
/* linear space at the cost of recomputing the matrix).  The forward pass   */
/* keeps two rows, finds the optimum by the same row-major scan as above,   */
/* and keeps the H and E of every block_rows-th row.  The walk then goes    */
/* back block by block: the block holding the walk's row is recomputed from */
/* the kept row above it, as full H/E/F matrices up to the walk's cell, and */
/* the walk takes exactly the steps of orc_align_affine_full until it       */
/* reaches the block's first row, where the block above takes over.        */
/* ---------------------------------------------------------------------- */
int orc_align_affine_checkpointed(const orc_scoring* sc, const uint8_t* q, int64_t n, const uint8_t* s, int64_t m,
                                  int64_t block_rows, orc_result* res, uint32_t* cigar, int64_t cigar_cap) {
  const int64_t go = sc->gap_open, ge = sc->gap_extend;
  const int32_t A = sc->alphabet_size;
  const int64_t K = block_rows;
  memset(res, 0, sizeof(*res));
  res->q_begin = res->s_begin = -1;
  if (K < 1) return -2;
  if (!check_codes(q, n, A) || !check_codes(s, m, A)) {
    res->flags = ORC_BAD_CODE;
    return 0;
  }
  const int64_t W = m + 1;
  const int64_t nck = n / K + 1; /* kept rows 0, K, 2K, ... */
  int64_t* ckH = (int64_t*)malloc(sizeof(int64_t) * nck * W);
  int64_t* ckE = (int64_t*)malloc(sizeof(int64_t) * nck * W);
  int64_t* pH = (int64_t*)malloc(sizeof(int64_t) * W);
  int64_t* pE = (int64_t*)malloc(sizeof(int64_t) * W);
  int64_t* cH = (int64_t*)malloc(sizeof(int64_t) * W);
  int64_t* cE = (int64_t*)malloc(sizeof(int64_t) * W);
  const int64_t rows_b = (K < n ? K : n) + 1;
  int64_t* Hm = (int64_t*)malloc(sizeof(int64_t) * rows_b * W);
  int64_t* Em = (int64_t*)malloc(sizeof(int64_t) * rows_b * W);
  int64_t* Fm = (int64_t*)malloc(sizeof(int64_t) * rows_b * W);
  uint8_t* ops = (uint8_t*)malloc((size_t)(n + m + 1));
  if (!ckH || !ckE || !pH || !pE || !cH || !cE || !Hm || !Em || !Fm || !ops) {
    free(ckH), free(ckE), free(pH), free(pE), free(cH), free(cE), free(Hm), free(Em), free(Fm), free(ops);
    return -1;
  }
  /* forward pass; the optimum scan visits the cells in the order of orc_align_affine_full's */
  int64_t bi = n, bj = m, best = 0;
  int first = 1;
  for (int64_t i = 0; i <= n; ++i) {
    if (i == 0) {
      for (int64_t j = 0; j <= m; ++j) {
        cH[j] = (sc->mode == ORC_GLOBAL && j > 0) ? go + j * ge : 0;
        cE[j] = NEG;
      }
    } else {
      int64_t fl = NEG; /* F(i, j - 1) */
      cH[0] = (sc->mode == ORC_GLOBAL) ? go + i * ge : 0;
      cE[0] = NEG;
      for (int64_t j = 1; j <= m; ++j) {
        int64_t e = max2(pE[j] + ge, pH[j] + go + ge);
        int64_t f = max2(fl + ge, cH[j - 1] + go + ge);
        int64_t d = pH[j - 1] + sc->sigma[q[i - 1] * A + s[j - 1]];
        int64_t h = max2(max2(d, e), f);
        if (sc->mode == ORC_LOCAL) h = max2(h, 0);
        cE[j] = e;
        fl = f;
        cH[j] = h;
      }
    }
    for (int64_t j = 0; j <= m; ++j) {
      if (sc->mode == ORC_LOCAL) {
        if (i == 0 && j == 0) {
          best = cH[0];
          bi = 0;
          bj = 0;
        } else if (cH[j] > best) {
          best = cH[j];
          bi = i;
          bj = j;
        }
      } else if (sc->mode == ORC_SEMIGLOBAL) {
        if (i != n && j != m) continue;
        if (first || cH[j] > best) {
          best = cH[j];
          bi = i;
          bj = j;
          first = 0;
        }
      }
    }
    if (sc->mode == ORC_GLOBAL && i == n) best = cH[m];
    if (i % K == 0) {
      memcpy(ckH + (i / K) * W, cH, sizeof(int64_t) * W);
      memcpy(ckE + (i / K) * W, cE, sizeof(int64_t) * W);
    }
    int64_t* t = pH;
    pH = cH;
    cH = t;
    t = pE;
    pE = cE;
    cE = t;
  }
  res->score = best;
  res->q_end = bi;
  res->s_end = bj;
  /* the walk, block by block */
  int64_t n_ops = 0, i = bi, j = bj;
  int state = 0; /* 0 = H, 1 = E, 2 = F */
  for (;;) {
    /* the borders, as in orc_align_affine_full (local walks stop there too: H is 0) */
    if (state == 0 && (i == 0 || j == 0)) {
      if (sc->mode == ORC_GLOBAL) {
        while (j > 0) {
          ops[n_ops++] = ORC_OP_D;
          --j;
        }
        while (i > 0) {
          ops[n_ops++] = ORC_OP_I;
          --i;
        }
      }
      break;
    }
    /* recompute the block of row i: rows r0 .. i, columns 0 .. j */
    const int64_t b = (i - 1) / K, r0 = b * K;
#define BH(r, c) Hm[((r) - r0) * W + (c)]
#define BE(r, c) Em[((r) - r0) * W + (c)]
#define BF(r, c) Fm[((r) - r0) * W + (c)]
    for (int64_t c = 0; c <= j; ++c) {
      BH(r0, c) = ckH[b * W + c];
      BE(r0, c) = ckE[b * W + c];
      BF(r0, c) = NEG; /* never read: the walk leaves the block before a step on row r0 */
    }
    for (int64_t r = r0 + 1; r <= i; ++r) {
      BH(r, 0) = (sc->mode == ORC_GLOBAL) ? go + r * ge : 0;
      BE(r, 0) = NEG;
      BF(r, 0) = NEG;
      for (int64_t c = 1; c <= j; ++c) {
        int64_t e = max2(BE(r - 1, c) + ge, BH(r - 1, c) + go + ge);
        int64_t f = max2(BF(r, c - 1) + ge, BH(r, c - 1) + go + ge);
        int64_t d = BH(r - 1, c - 1) + sc->sigma[q[r - 1] * A + s[c - 1]];
        int64_t h = max2(max2(d, e), f);
        if (sc->mode == ORC_LOCAL) h = max2(h, 0);
        BE(r, c) = e;
        BF(r, c) = f;
        BH(r, c) = h;
      }
    }
    /* the steps of orc_align_affine_full, inside the block */
    int done = 0;
    for (;;) {
      if (state != 2 && i == r0 && r0 > 0) break; /* the block above holds the next step */
      if (state == 0) {
        if (i == 0 || j == 0) break;                     /* the borders, above */
        if (sc->mode == ORC_LOCAL && BH(i, j) == 0) {
          done = 1;
          break;
        }
        int64_t d = BH(i - 1, j - 1) + sc->sigma[q[i - 1] * A + s[j - 1]];
        if (d == BH(i, j)) {
          ops[n_ops++] = ORC_OP_M;
          --i;
          --j;
        } else if (BE(i, j) == BH(i, j)) {
          state = 1;
        } else {
          state = 2;
        }
      } else if (state == 1) {
        ops[n_ops++] = ORC_OP_I;
        if (BH(i - 1, j) + go + ge == BE(i, j)) state = 0;
        --i;
      } else {
        ops[n_ops++] = ORC_OP_D;
        if (BH(i, j - 1) + go + ge == BF(i, j)) state = 0;
        --j;
      }
    }
#undef BH
#undef BE
#undef BF
    if (done) break;
  }
  res->q_begin = i;
  res->s_begin = j;
  int trunc = 0;
  res->cigar_len = emit_cigar(ops, n_ops, cigar, cigar_cap, &trunc);
  if (trunc) res->flags |= ORC_CIGAR_TRUNC;
  free(ckH), free(ckE), free(pH), free(pE), free(cH), free(cE), free(Hm), free(Em), free(Fm), free(ops);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Linear gap, Eqs. (2)-(3): one matrix H; priority diag > up (I) > left.  */
/* ---------------------------------------------------------------------- */
int orc_align_linear_full(const orc_scoring* sc, const uint8_t* q, int64_t n, const uint8_t* s, int64_t m,
                          int want_cigar, orc_result* res, uint32_t* cigar, int64_t cigar_cap) {
  const int64_t g = sc->gap_extend;
  const int32_t A = sc->alphabet_size;
  memset(res, 0, sizeof(*res));
  res->q_begin = res->s_begin = -1;
  if (sc->gap_open != 0) return -2;
  if (!check_codes(q, n, A) || !check_codes(s, m, A)) {
    res->flags = ORC_BAD_CODE;
    return 0;
  }
  const int64_t W = m + 1;
  int64_t* Hm = (int64_t*)malloc(sizeof(int64_t) * (n + 1) * W);
  if (!Hm) return -1;
#define H_(i, j) Hm[(i) * W + (j)]
  for (int64_t i = 0; i <= n; ++i) H_(i, 0) = (sc->mode == ORC_GLOBAL) ? i * g : 0;
  for (int64_t j = 0; j <= m; ++j) H_(0, j) = (sc->mode == ORC_GLOBAL) ? j * g : 0;
  for (int64_t i = 1; i <= n; ++i)
    for (int64_t j = 1; j <= m; ++j) {
      int64_t h = H_(i - 1, j - 1) + sc->sigma[q[i - 1] * A + s[j - 1]];
      h = max2(h, H_(i - 1, j) + g);
      h = max2(h, H_(i, j - 1) + g);
      if (sc->mode == ORC_LOCAL) h = max2(h, 0);
      H_(i, j) = h;
    }
  int64_t bi = n, bj = m, best = H_(n, m);
  if (sc->mode == ORC_LOCAL) {
    best = 0;
    bi = bj = 0;
    for (int64_t i = 0; i <= n; ++i)
      for (int64_t j = 0; j <= m; ++j)
        if (H_(i, j) > best) {
          best = H_(i, j);
          bi = i;
          bj = j;
        }
  } else if (sc->mode == ORC_SEMIGLOBAL) {
    int first = 1;
    for (int64_t i = 0; i <= n; ++i)
      for (int64_t j = 0; j <= m; ++j) {
        if (i != n && j != m) continue;
        if (first || H_(i, j) > best) {
          best = H_(i, j);
          bi = i;
          bj = j;
          first = 0;
        }
      }
  }
  res->score = best;
  res->q_end = bi;
  res->s_end = bj;
  if (want_cigar) {
    uint8_t* ops = (uint8_t*)malloc((size_t)(n + m + 1));
    int64_t n_ops = 0, i = bi, j = bj;
    for (;;) {
      if (sc->mode == ORC_LOCAL && H_(i, j) == 0) break;
      if (sc->mode == ORC_SEMIGLOBAL && (i == 0 || j == 0)) break;
      if (i == 0 && j == 0) break;
      if (i == 0) {
        ops[n_ops++] = ORC_OP_D;
        --j;
        continue;
      }
      if (j == 0) {
        ops[n_ops++] = ORC_OP_I;
        --i;
        continue;
      }
      if (H_(i - 1, j - 1) + sc->sigma[q[i - 1] * A + s[j - 1]] == H_(i, j)) {
        ops[n_ops++] = ORC_OP_M;
        --i;
        --j;
      } else if (H_(i - 1, j) + g == H_(i, j)) {
        ops[n_ops++] = ORC_OP_I;
        --i;
      } else {
        ops[n_ops++] = ORC_OP_D;
        --j;
      }
    }
    res->q_begin = i;
    res->s_begin = j;
    int trunc = 0;
    res->cigar_len = emit_cigar(ops, n_ops, cigar, cigar_cap, &trunc);
    if (trunc) res->flags |= ORC_CIGAR_TRUNC;
    free(ops);
  }
  free(Hm);
#undef H_
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Score-only affine DP in linear space (Sec. III-A: only the previous row */
/* is kept).  Same optimum and tie rule as the full version.              */
/* ---------------------------------------------------------------------- */
int orc_score_affine_linear_space(const orc_scoring* sc, const uint8_t* q, int64_t n, const uint8_t* s,
                                  int64_t m, orc_result* res) {
  const int64_t go = sc->gap_open, ge = sc->gap_extend;
  const int32_t A = sc->alphabet_size;
  memset(res, 0, sizeof(*res));
  res->q_begin = res->s_begin = -1;
  if (!check_codes(q, n, A) || !check_codes(s, m, A)) {
    res->flags = ORC_BAD_CODE;
    return 0;
  }
  /* Hrow[j], Erow[j] hold row i-1 until overwritten with row i. */
  int64_t* Hrow = (int64_t*)malloc(sizeof(int64_t) * (m + 1));
  int64_t* Erow = (int64_t*)malloc(sizeof(int64_t) * (m + 1));
  if (!Hrow || !Erow) {
    free(Hrow);
    free(Erow);
    return -1;
  }
  for (int64_t j = 0; j <= m; ++j) {
    Hrow[j] = (sc->mode == ORC_GLOBAL && j > 0) ? go + j * ge : 0;
    Erow[j] = NEG;
  }
  int64_t best = 0, bi = 0, bj = 0;
  int have = 0;
  for (int64_t i = 0; i <= n; ++i) {
    if (i > 0) {
      int64_t hdiag = Hrow[0];
      int64_t hleft = (sc->mode == ORC_GLOBAL) ? go + i * ge : 0;
      int64_t f = NEG;
      Hrow[0] = hleft;
      for (int64_t j = 1; j <= m; ++j) {
        int64_t e = max2(Erow[j] + ge, Hrow[j] + go + ge);
        f = max2(f + ge, hleft + go + ge);
        int64_t d = hdiag + sc->sigma[q[i - 1] * A + s[j - 1]];
        int64_t h = max2(max2(d, e), f);
        if (sc->mode == ORC_LOCAL) h = max2(h, 0);
        hdiag = Hrow[j];
        Hrow[j] = h;
        Erow[j] = e;
        hleft = h;
      }
    }
    /* candidates of row i, scanned in row-major order with strict '>' */
    for (int64_t j = 0; j <= m; ++j) {
      int cand = (sc->mode == ORC_LOCAL) || (sc->mode == ORC_SEMIGLOBAL && (i == n || j == m));
      if (cand && (!have || Hrow[j] > best)) {
        best = Hrow[j];
        bi = i;
        bj = j;
        have = 1;
      }
    }
  }
  if (sc->mode == ORC_GLOBAL) {
    best = Hrow[m];
    bi = n;
    bj = m;
  }
  res->score = best;
  res->q_end = bi;
  res->s_end = bj;
  free(Hrow);
  free(Erow);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Batch driver: independent pairs over a pool of POSIX threads.           */
/* ---------------------------------------------------------------------- */
typedef struct {
  const orc_scoring* sc;
  int64_t n_pairs;
  const uint8_t *q, *s;
  const int64_t *q_off, *s_off;
  int want_cigar;
  orc_result* res;
  uint32_t* cigar;
  const int64_t* cigar_off;
  int64_t next;
  pthread_mutex_t mu;
  int status;
} batch_ctx;

static void* batch_worker(void* arg) {
  batch_ctx* c = (batch_ctx*)arg;
  for (;;) {
    pthread_mutex_lock(&c->mu);
    int64_t k = c->next++;
    pthread_mutex_unlock(&c->mu);
    if (k >= c->n_pairs) break;
    const uint8_t* q = c->q + c->q_off[k];
    const uint8_t* s = c->s + c->s_off[k];
    int64_t n = c->q_off[k + 1] - c->q_off[k], m = c->s_off[k + 1] - c->s_off[k];
    int rc;
    if (c->want_cigar) {
      int64_t cap = c->cigar_off[k + 1] - c->cigar_off[k];
      rc = orc_align_affine_full(c->sc, q, n, s, m, 1, &c->res[k], c->cigar + c->cigar_off[k], cap);
    } else {
      rc = orc_score_affine_linear_space(c->sc, q, n, s, m, &c->res[k]);
    }
    if (rc != 0) {
      pthread_mutex_lock(&c->mu);
      c->status = rc;
      pthread_mutex_unlock(&c->mu);
    }
  }
  return 0;
}

int orc_align_batch(const orc_scoring* sc, int64_t n_pairs, const uint8_t* q, const int64_t* q_off,
                    const uint8_t* s, const int64_t* s_off, int want_cigar, orc_result* res, uint32_t* cigar,
                    const int64_t* cigar_off, int n_threads) {
  batch_ctx c;
  c.sc = sc;
  c.n_pairs = n_pairs;
  c.q = q;
  c.s = s;
  c.q_off = q_off;
  c.s_off = s_off;
  c.want_cigar = want_cigar;
  c.res = res;
  c.cigar = cigar;
  c.cigar_off = cigar_off;
  c.next = 0;
  c.status = 0;
  pthread_mutex_init(&c.mu, 0);
  if (n_threads < 1) n_threads = 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
  for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], 0, batch_worker, &c);
  for (int t = 0; t < n_threads; ++t) pthread_join(th[t], 0);
  free(th);
  pthread_mutex_destroy(&c.mu);
  return c.status;
}
