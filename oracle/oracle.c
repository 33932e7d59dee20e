/*
 * oracle.c -- plain, slow CPU reference for the ABFT-protected one-sided
 * decompositions (Chen et al., "Improving Energy Saving of One-sided Matrix
 * Decompositions on CPU-GPU Heterogeneous Systems", PPoPP'23).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code with the GPU
 * path.
 *
 * What it computes (paper section "State-of-the-art matrix decompositions"):
 * a blocked decomposition walks the matrix from the top-left corner to the
 * bottom-right one; each iteration does a panel decomposition (PD), a panel
 * update (PU) and a trailing-matrix update (TMU).  Cholesky, LU with partial
 * pivoting and Householder QR all follow this shape.
 *
 * ABFT (paper section "Design of ABFT-OC"): checksums are encoded before an
 * operation, the same operation is applied to the checksums, and the checksum
 * relation is verified afterwards.  Full checksums encode both rows and
 * columns; every b x b block carries its own checksums and at most one fault
 * per block per detection interval (one iteration) is tolerated.  The paper
 * gives only these principles; the concrete algebra below (weights, carry
 * rules, thresholds, locate/correct rule) is this project's reading of them
 * and is written out in the design notes.
 *
 * Arithmetic is plain IEEE binary64 with no contraction (built with
 * -ffp-contract=off).  The mixed-precision forms emulate binary32 data by
 * rounding every stored result to float, and bf16/fp16 GEMM operands by
 * round-to-nearest-even to that format.
 *
 * Storage: column-major, element (i,j) at A[i + j*lda].
 *
 * Threads: the loops over independent output elements (tiles, columns,
 * rows of a block of rows) are spread over OpenMP threads.  Every element
 * is still computed by one thread with the same operations in the same
 * order as a plain serial loop, so the results are bitwise independent of
 * the thread count (a test runs the same factorization with 1 and with
 * several threads).  Report events are emitted in the serial order.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define AT(A, i, j, ld) ((A)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

/* ------------------------------------------------------------------ */
/* Public structs (mirrored by the Python loader).                     */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t iter;   /* iteration after whose trailing update the flip lands */
  int32_t target; /* 0 = matrix, 1 = column checksums, 2 = row checksums */
  int64_t row, col;
  int32_t bit;    /* 0..63 of the binary64 pattern */
  int32_t pad;
} orc_fault;

typedef struct {
  int32_t iter, kind; /* kind: 1 corrected, 2 checksum repaired, 3 uncorrectable, 4 panel flag */
  int64_t row, col;
} orc_event;

#define ORC_MAX_EV 16
typedef struct {
  int64_t flagged_tiles, corrected, checksum_repaired, uncorrectable, panel_flags;
  int32_t first_flag_iter, status; /* status bits: 1 corrected, 2 repaired, 4 uncorrectable, 8 panel */
  double max_ratio;                /* max |d|/tau over unflagged compared entries */
  int32_t nev, pad;
  orc_event ev[ORC_MAX_EV];
} orc_report;

enum { PR64 = 0, PR32 = 1, PRBF16 = 2, PRF16 = 3 };

/* ------------------------------------------------------------------ */
/* Precision emulation.                                                */
/* ------------------------------------------------------------------ */
static inline double rs(int prec, double x) { return prec == PR64 ? x : (double)(float)x; }

/* round-to-nearest-even of x to a binary format with `mant` fraction bits and
   normal exponent range [emin, emax] (subnormals kept, overflow to inf) */
static double round_fmt(double x, int mant, int emin, int emax) {
  if (!isfinite(x) || x == 0.0) return x;
  int e;
  frexp(x, &e);
  int ex = e - 1;
  if (ex < emin) ex = emin;
  double ulp = ldexp(1.0, ex - mant);
  double y = nearbyint(x / ulp) * ulp;
  double maxv = ldexp(2.0 - ldexp(1.0, -mant), emax);
  if (fabs(y) > maxv) return copysign(INFINITY, x);
  return y;
}
double orc_round_bf16(double x) { return round_fmt((double)(float)x, 7, -126, 127); }
double orc_round_fp16(double x) { return round_fmt((double)(float)x, 10, -14, 15); }

/* operand rounding applied to the trailing-update GEMM inputs */
static inline double rop(int prec, double x) {
  switch (prec) {
    case PR32: return (double)(float)x;
    case PRBF16: return orc_round_bf16(x);
    case PRF16: return orc_round_fp16(x);
    default: return x;
  }
}
static inline double unit_round(int prec) { return prec == PR64 ? ldexp(1.0, -53) : ldexp(1.0, -24); }

void orc_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }
static inline int imin(int a, int b) { return a < b ? a : b; }
static inline int imax(int a, int b) { return a > b ? a : b; }

/* Compensated accumulator (value s + c): Knuth's two-sum for additions and
   an FMA-based two-product for products, so checksum sums and checksum
   updates carry almost no rounding of their own and the comparison sees the
   rounding of the data alone. */
typedef struct { double s, c; } acc_t;
static inline void acc_add(acc_t* a, double x) {
  double t = a->s + x, bp = t - a->s;
  a->c += (a->s - (t - bp)) + (x - bp);
  a->s = t;
}
static inline void acc_fma(acc_t* a, double x, double y) {
  double p = x * y;
  double e = fma(x, y, -p);
  acc_add(a, p);
  a->c += e;
}
static inline double acc_val(acc_t a) { return a.s + a.c; }

/* ------------------------------------------------------------------ */
/* Unblocked reference factorizations (used for brute-force checks).   */
/* ------------------------------------------------------------------ */

/* Cholesky-Crout, lower: L(j,j) = sqrt(a_jj - sum_p L(j,p)^2),
   L(i,j) = (a_ij - sum_p L(i,p) L(j,p)) / L(j,j).  Returns info (0 or j+1). */
int orc_potrf_unb(int n, double* A, int lda) {
  for (int j = 0; j < n; ++j) {
    double d = AT(A, j, j, lda);
    for (int p = 0; p < j; ++p) d -= AT(A, j, p, lda) * AT(A, j, p, lda);
    if (!(d > 0.0)) return j + 1;
    d = sqrt(d);
    AT(A, j, j, lda) = d;
    for (int i = j + 1; i < n; ++i) {
      double s = AT(A, i, j, lda);
      for (int p = 0; p < j; ++p) s -= AT(A, i, p, lda) * AT(A, j, p, lda);
      AT(A, i, j, lda) = s / d;
    }
  }
  return 0;
}

/* pivot choice shared by all LU variants: first index of the largest |a| */
static int pick_pivot(const double* A, int lda, int col, int r0, int m) {
  int p = r0;
  double best = fabs(AT(A, r0, col, lda));
  for (int i = r0 + 1; i < m; ++i) {
    double v = fabs(AT(A, i, col, lda));
    if (v > best) { best = v; p = i; }
  }
  return p;
}

static void swap_rows(double* A, int lda, int r, int p, int c0, int c1) {
  if (r == p) return;
  for (int j = c0; j < c1; ++j) {
    double t = AT(A, r, j, lda);
    AT(A, r, j, lda) = AT(A, p, j, lda);
    AT(A, p, j, lda) = t;
  }
}

/* LU with partial pivoting, right-looking rank-1 form (getf2), whole-row swaps.
   ipiv is 1-based.  info = first j+1 with U(j,j) == 0 (factorization continues). */
int orc_getrf_unb(int n, double* A, int lda, int32_t* ipiv) {
  int info = 0;
  for (int j = 0; j < n; ++j) {
    int p = pick_pivot(A, lda, j, j, n);
    ipiv[j] = p + 1;
    swap_rows(A, lda, j, p, 0, n);
    double piv = AT(A, j, j, lda);
    if (piv == 0.0) {
      if (!info) info = j + 1;
      continue;
    }
    for (int i = j + 1; i < n; ++i) AT(A, i, j, lda) = AT(A, i, j, lda) / piv;
    for (int c = j + 1; c < n; ++c) {
      double u = AT(A, j, c, lda);
      for (int i = j + 1; i < n; ++i) AT(A, i, c, lda) -= AT(A, i, j, lda) * u;
    }
  }
  return info;
}

/* Householder reflector in the LAPACK dlarfg convention: given alpha and the
   sub-column x (norm^2 = sigma2), H = I - tau v v^T with v(0) = 1 maps
   [alpha; x] to [beta; 0].  Returns beta and writes tau and the scale
   1/(alpha - beta) that turns x into v(1:). */
static double householder(double alpha, double sigma2, double* tau, double* scale) {
  if (sigma2 == 0.0) {
    *tau = 0.0;
    *scale = 0.0;
    return alpha;
  }
  double beta = -copysign(sqrt(alpha * alpha + sigma2), alpha);
  *tau = (beta - alpha) / beta;
  *scale = 1.0 / (alpha - beta);
  return beta;
}

/* Householder QR of columns [c0,c1) over rows [c0,m) (geqr2).  R overwrites
   the upper part, v(1:) the part below the diagonal. */
static void geqr2_cols(int m, double* A, int lda, double* tau, int c0, int c1) {
  for (int j = c0; j < c1; ++j) {
    double s2 = 0.0;
    for (int i = j + 1; i < m; ++i) s2 += AT(A, i, j, lda) * AT(A, i, j, lda);
    double t, sc;
    double beta = householder(AT(A, j, j, lda), s2, &t, &sc);
    tau[j] = t;
    if (t == 0.0) continue;
    for (int i = j + 1; i < m; ++i) AT(A, i, j, lda) *= sc;
    AT(A, j, j, lda) = beta;
#pragma omp parallel for schedule(static) if ((size_t)(c1 - j) * (size_t)(m - j) > ((size_t)1 << 16))
    for (int c = j + 1; c < c1; ++c) {
      double w = AT(A, j, c, lda);
      for (int i = j + 1; i < m; ++i) w += AT(A, i, j, lda) * AT(A, i, c, lda);
      w *= t;
      AT(A, j, c, lda) -= w;
      for (int i = j + 1; i < m; ++i) AT(A, i, c, lda) -= w * AT(A, i, j, lda);
    }
  }
}

void orc_geqrf_unb(int n, double* A, int lda, double* tau) { geqr2_cols(n, A, lda, tau, 0, n); }

/* ------------------------------------------------------------------ */
/* ABFT state.                                                         */
/*   colchk: (2N) x n, ld 2N.  Row 2I holds sum_{i in tile-row I} a_ij, */
/*           row 2I+1 holds sum (i - I*nb + 1) a_ij.                    */
/*   rowchk: n x (2N), ld n.  Column 2J holds sum_{j in tile-col J} a_ij*/
/*           column 2J+1 holds sum (j - J*nb + 1) a_ij.                 */
/*   gc/gr : same shapes; per-entry magnitude of this iteration's update*/
/* ------------------------------------------------------------------ */
typedef struct {
  int n, nb, N, sym, prec, protect;
  double u, ts;
  double *cc, *rc, *gc, *gr;
  int ldc, ldr;
  orc_report* rep;
  int iter;
  int level; /* protection of the current iteration: 0 none, 1 column side only, 2 both sides */
} ctx_t;

static inline int tlen(const ctx_t* c, int I) { int r = c->n - I * c->nb; return r < c->nb ? r : c->nb; }

/* symmetric view for Cholesky diagonal tiles (lower storage) */
static inline double S(const ctx_t* c, const double* A, int lda, int i, int j) {
  if (c->sym && i < j) return AT(A, j, i, lda);
  return AT(A, i, j, lda);
}

static void add_event(orc_report* r, int iter, int kind, int64_t row, int64_t col) {
  if (r->nev < ORC_MAX_EV) {
    r->ev[r->nev].iter = iter;
    r->ev[r->nev].kind = kind;
    r->ev[r->nev].row = row;
    r->ev[r->nev].col = col;
  }
  r->nev++;
}

static void note_flag(ctx_t* c) {
  if (c->rep->first_flag_iter < 0) c->rep->first_flag_iter = c->iter;
}

/* all sums of one tile (symmetric view when c->sym and I == J), with the
   compensated accumulators they are formed in */
typedef struct {
  double ce[1024], cw[1024], ca[1024], cwa[1024];
  double re[1024], rw[1024], ra[1024], rwa[1024];
  acc_t ace[1024], acw[1024], are[1024], arw[1024];
} tsums_t;

static void tile_sums(const ctx_t* c, const double* A, int lda, int I, int J, tsums_t* t) {
  int r0 = I * c->nb, h = tlen(c, I), c0 = J * c->nb, w = tlen(c, J);
  acc_t *ce = t->ace, *cw = t->acw, *re = t->are, *rw = t->arw;
  for (int j = 0; j < w; ++j) { ce[j].s = ce[j].c = cw[j].s = cw[j].c = 0.0; t->ca[j] = t->cwa[j] = 0.0; }
  for (int i = 0; i < h; ++i) { re[i].s = re[i].c = rw[i].s = rw[i].c = 0.0; t->ra[i] = t->rwa[i] = 0.0; }
  for (int j = 0; j < w; ++j)
    for (int i = 0; i < h; ++i) {
      double v = (c->sym && I == J) ? S(c, A, lda, r0 + i, c0 + j) : AT(A, r0 + i, c0 + j, lda);
      acc_add(&ce[j], v);
      acc_fma(&cw[j], (double)(i + 1), v);
      t->ca[j] += fabs(v);
      t->cwa[j] += (double)(i + 1) * fabs(v);
      acc_add(&re[i], v);
      acc_fma(&rw[i], (double)(j + 1), v);
      t->ra[i] += fabs(v);
      t->rwa[i] += (double)(j + 1) * fabs(v);
    }
  for (int j = 0; j < w; ++j) { t->ce[j] = acc_val(ce[j]); t->cw[j] = acc_val(cw[j]); }
  for (int i = 0; i < h; ++i) { t->re[i] = acc_val(re[i]); t->rw[i] = acc_val(rw[i]); }
}

static void store_sums(ctx_t* c, int I, int J, const tsums_t* t) {
  int r0 = I * c->nb, h = tlen(c, I), c0 = J * c->nb, w = tlen(c, J);
  for (int j = 0; j < w; ++j) {
    AT(c->cc, 2 * I, c0 + j, c->ldc) = t->ce[j];
    AT(c->cc, 2 * I + 1, c0 + j, c->ldc) = t->cw[j];
  }
  for (int i = 0; i < h; ++i) {
    AT(c->rc, r0 + i, 2 * J, c->ldr) = t->re[i];
    AT(c->rc, r0 + i, 2 * J + 1, c->ldr) = t->rw[i];
  }
}

/* Verify threshold for trailing tiles.  With compensated checksum
   arithmetic the carried/recomputed gap is made of the data's own rounding:
   about one ulp of each stored element (covered by the 4 a term, a = sum of
   |a_ij| over the checksum's support) plus the accumulation error of the
   update's dot products (covered by g = sum |x||y| of the same products). */
static inline double tau_of(const ctx_t* c, double a, double g) { return (4.0 * c->ts * c->u) * a + (c->ts * c->u) * g; }
/* a comparison fails when |d| exceeds tau, when d is NaN, and when the
   threshold itself is not finite (Inf or overflowed magnitudes in the data) */
static inline int bad(double d, double tau) { return !(fabs(d) <= tau) || !(tau <= 1.79e308); }
/* Panel threshold: the factorization's backward error enters through dot
   products of length up to nb, hence the extra sqrt(nb). */
static inline double tau_panel(const ctx_t* c, double mag) { return (2.0 * c->ts * c->u * sqrt((double)c->nb)) * mag; }

typedef struct { int fe[1024], fw[1024], ge[1024], gw[1024]; double de[1024], dw[1024], he[1024], hw[1024]; } tflags_t;

/* A rebuilt element (tile-relative ci, cj) is known only to the tolerance of
   the column checksum it was rebuilt from, te_c.  When a tile is rechecked
   after a correction, every sum that contains the element (twice in the
   symmetric view of a diagonal tile: at (ci, cj) and at its mirror) may
   differ by its weight in that sum times te_c.  These give the weight of the
   element in column j / row i of the tile, 0 where it does not occur. */
typedef struct { int ci, cj, diag; double tec; } slack_t;
static double slack_col(const slack_t* s, int j) {
  if (!s) return 0.0;
  if (j == s->cj) return (s->ci + 1) * s->tec;
  if (s->diag && j == s->ci) return (s->cj + 1) * s->tec;
  return 0.0;
}
static double slack_row(const slack_t* s, int i) {
  if (!s) return 0.0;
  if (i == s->ci) return (s->cj + 1) * s->tec;
  if (s->diag && i == s->cj) return (s->ci + 1) * s->tec;
  return 0.0;
}
static double slack_one(const slack_t* s, int hit) { return (s && hit) ? s->tec : 0.0; }
/* After a whole row (column) of a tile was rebuilt from the checksums of
   the other side, each rebuilt element is known to the tolerance of the
   checksum it came from; the additions to the plain (e) and weighted (w)
   tolerances of every column and row sum of the tile. */
typedef struct { double ce[1024], cw[1024], re[1024], rw[1024]; } lslack_t;

/* compare recomputed sums with carried checksums; returns number of flags.
   sl (may be NULL) widens the comparisons that contain a rebuilt element. */
static int tile_flags(ctx_t* c, int I, int J, const tsums_t* t, tflags_t* f, double* maxr, const slack_t* sl,
                      const lslack_t* ls) {
  int r0 = I * c->nb, h = tlen(c, I), c0 = J * c->nb, w = tlen(c, J);
  int nflag = 0;
  for (int j = 0; j < w; ++j) {
    double de = t->ce[j] - AT(c->cc, 2 * I, c0 + j, c->ldc);
    double dw = t->cw[j] - AT(c->cc, 2 * I + 1, c0 + j, c->ldc);
    double te = tau_of(c, t->ca[j], AT(c->gc, 2 * I, c0 + j, c->ldc));
    double tw = tau_of(c, t->cwa[j], AT(c->gc, 2 * I + 1, c0 + j, c->ldc));
    double sw = slack_col(sl, j);
    te += slack_one(sl, sw > 0.0);
    tw += sw;
    if (ls) { te += ls->ce[j]; tw += ls->cw[j]; }
    f->de[j] = de;
    f->dw[j] = dw;
    f->fe[j] = bad(de, te);
    f->fw[j] = bad(dw, tw);
    nflag += f->fe[j] + f->fw[j];
    if (maxr) {
      if (!f->fe[j] && te > 0) { double r = fabs(de) / te; if (r > *maxr) *maxr = r; }
      if (!f->fw[j] && tw > 0) { double r = fabs(dw) / tw; if (r > *maxr) *maxr = r; }
    }
  }
  for (int i = 0; i < h; ++i) {
    if (c->level == 1) { /* single side: the row checksums are not compared */
      f->he[i] = f->hw[i] = 0.0;
      f->ge[i] = f->gw[i] = 0;
      continue;
    }
    double de = t->re[i] - AT(c->rc, r0 + i, 2 * J, c->ldr);
    double dw = t->rw[i] - AT(c->rc, r0 + i, 2 * J + 1, c->ldr);
    double te = tau_of(c, t->ra[i], AT(c->gr, r0 + i, 2 * J, c->ldr));
    double tw = tau_of(c, t->rwa[i], AT(c->gr, r0 + i, 2 * J + 1, c->ldr));
    double sw = slack_row(sl, i);
    te += slack_one(sl, sw > 0.0);
    tw += sw;
    if (ls) { te += ls->re[i]; tw += ls->rw[i]; }
    f->he[i] = de;
    f->hw[i] = dw;
    f->ge[i] = bad(de, te);
    f->gw[i] = bad(dw, tw);
    nflag += f->ge[i] + f->gw[i];
    if (maxr) {
      if (!f->ge[i] && te > 0) { double r = fabs(de) / te; if (r > *maxr) *maxr = r; }
      if (!f->gw[i] && tw > 0) { double r = fabs(dw) / tw; if (r > *maxr) *maxr = r; }
    }
  }
  return nflag;
}

/* whether the weighted / plain difference ratio exists (it does not when a
   difference is not finite or the weighted one overflowed) */
static int ratio_finite(double dw, double de) { return de != 0.0 && isfinite(dw / de); }

/* locate a row (column) from the weighted / plain difference ratio */
static int ratio_index(double dw, double de, int len) {
  if (!(de != 0.0) || !isfinite(dw / de)) return -1;
  double r = dw / de;
  double k = floor(r + 0.5);
  if (fabs(r - k) > 0.25) return -1;
  if (k < 1.0 || k > (double)len) return -1;
  return (int)k - 1;
}

/* Rebuild a whole line of a tile (1D error: one row or one column of the
   tile is wrong): line 1 = row idx, each element from its column's plain
   checksum with the rest of the column left out; line 2 = column idx, each
   element from its row's plain checksum.  The tile is then rechecked with
   the rebuilt elements' tolerances added where they occur; on failure the
   old values come back.  Returns 1 when the recheck passes. */
static int rebuild_line(ctx_t* c, double* A, int lda, int I, int J, int line, int idx, tsums_t* t, tflags_t* f) {
  int r0 = I * c->nb, h = tlen(c, I), c0 = J * c->nb, w = tlen(c, J);
  double* old = malloc(sizeof(double) * 1024);
  if (line == 1) {
    for (int j = 0; j < w; ++j) {
      double s = AT(c->cc, 2 * I, c0 + j, c->ldc);
      for (int i = 0; i < h; ++i) {
        if (i == idx) continue;
        s -= AT(A, r0 + i, c0 + j, lda);
      }
      old[j] = AT(A, r0 + idx, c0 + j, lda);
      AT(A, r0 + idx, c0 + j, lda) = s;
    }
  } else {
    for (int i = 0; i < h; ++i) {
      double s = AT(c->rc, r0 + i, 2 * J, c->ldr);
      for (int j = 0; j < w; ++j) {
        if (j == idx) continue;
        s -= AT(A, r0 + i, c0 + j, lda);
      }
      old[i] = AT(A, r0 + i, c0 + idx, lda);
      AT(A, r0 + i, c0 + idx, lda) = s;
    }
  }
  tile_sums(c, A, lda, I, J, t);
  lslack_t* ls = calloc(1, sizeof(lslack_t));
  if (line == 1) {
    for (int j = 0; j < w; ++j) {
      double tec = tau_of(c, t->ca[j], AT(c->gc, 2 * I, c0 + j, c->ldc));
      ls->ce[j] = tec;
      ls->cw[j] = (double)(idx + 1) * tec;
      ls->re[idx] += tec;
      ls->rw[idx] += (double)(j + 1) * tec;
    }
  } else {
    for (int i = 0; i < h; ++i) {
      double ter = tau_of(c, t->ra[i], AT(c->gr, r0 + i, 2 * J, c->ldr));
      ls->re[i] = ter;
      ls->rw[i] = (double)(idx + 1) * ter;
      ls->ce[idx] += ter;
      ls->cw[idx] += (double)(i + 1) * ter;
    }
  }
  int ok = tile_flags(c, I, J, t, f, NULL, NULL, ls) == 0;
  if (!ok) {
    if (line == 1) for (int j = 0; j < w; ++j) AT(A, r0 + idx, c0 + j, lda) = old[j];
    else for (int i = 0; i < h; ++i) AT(A, r0 + i, c0 + idx, lda) = old[i];
  }
  free(ls);
  free(old);
  return ok;
}

/* Locate and correct one flagged tile (0D model: one fault per tile per
   iteration).  The element is recomputed from its column checksum with the
   element itself left out, so huge, Inf or NaN values are repaired too. */
static void correct_tile(ctx_t* c, double* A, int lda, int I, int J) {
  int r0 = I * c->nb, h = tlen(c, I), c0 = J * c->nb, w = tlen(c, J);
  int diag = c->sym && I == J;
  tsums_t* tp = malloc(sizeof(tsums_t));
  tflags_t* fp = malloc(sizeof(tflags_t));
#define t (*tp)
#define f (*fp)
  tile_sums(c, A, lda, I, J, &t);
  int nf = tile_flags(c, I, J, &t, &f, NULL, NULL, NULL);
  if (nf == 0) { free(tp); free(fp); return; }
  int nFe = 0, nGe = 0, nFw = 0, nGw = 0, jf[2] = {-1, -1}, ig = -1;
  for (int j = 0; j < w; ++j) {
    if (f.fe[j]) { if (nFe < 2) jf[nFe] = j; nFe++; }
    nFw += f.fw[j];
  }
  for (int i = 0; i < h; ++i) {
    if (f.ge[i]) { ig = i; nGe++; }
    nGw += f.gw[i];
  }
  int ci = -1, cj = -1; /* candidate stored element (tile-relative) */
  int repair = 0;
  int line = 0; /* 1D: 1 = rebuild row ig from the column checksums, 2 = column jf[0] from the row checksums */
  if (diag) {
    /* In the symmetric view an off-diagonal element shows in two columns
       (itself and its mirror), a diagonal one in one.  Two flagged columns
       therefore name the element by the pattern alone (the ratios would only
       confirm it, and near the threshold they carry the weighted sums'
       rounding noise); the recheck after the rebuild rejects any other
       cause.  One flagged column: the ratio names the row (the element, or
       its mirror when the other column stayed below its threshold); where
       the ratio does not exist (a non-finite value, or a weighted sum that
       overflowed) it is the diagonal element. */
    if (nFe == 1) {
      int a = jf[0], i = ratio_index(f.dw[a], f.de[a], h);
      if (i >= 0) { ci = i > a ? i : a; cj = i > a ? a : i; }
      else if (!ratio_finite(f.dw[a], f.de[a])) { ci = a; cj = a; }
      else if (nGe == 0 && !f.fw[a]) repair = 1; /* a flipped e entry of the column checksums */
    } else if (nFe == 2) {
      ci = jf[1]; cj = jf[0];
    } else if (nFe == 0) {
      repair = 1;
    }
  } else {
    /* a checksum entry is taken for wrong only when its data side is
       consistent: a plain column (row) difference with an unflagged weighted
       one (a flipped e entry), or weighted differences alone */
    if (nFe == 1 && nGe == 1) {
      ci = ig; cj = jf[0];
    } else if (nFe == 1 && nGe == 0) {
      int i = ratio_index(f.dw[jf[0]], f.de[jf[0]], h);
      if (i >= 0) { ci = i; cj = jf[0]; }
      else if (nGw == 0 && !f.fw[jf[0]]) repair = 1;
    } else if (nFe == 0 && nGe == 1) {
      int j = ratio_index(f.hw[ig], f.he[ig], w);
      if (j >= 0) { ci = ig; cj = j; }
      else if (nFw == 0 && !f.gw[ig]) repair = 1;
    } else if (nFe == 0 && nGe == 0) {
      repair = 1;
    } else if (c->level == 2 && nGe == 1 && nFe >= 2) {
      line = 1; /* one row of the tile is wrong in several columns */
    } else if (c->level == 2 && nFe == 1 && nGe >= 2) {
      line = 2; /* one column is wrong in several rows */
    }
  }
  int kind = 3;
  if (ci >= 0) {
    /* recompute the element from the carried column-e checksum of column cj */
    double s = AT(c->cc, 2 * I, c0 + cj, c->ldc);
    for (int i = 0; i < h; ++i) {
      if (i == ci) continue;
      s -= diag ? S(c, A, lda, r0 + i, c0 + cj) : AT(A, r0 + i, c0 + cj, lda);
    }
    double old = AT(A, r0 + ci, c0 + cj, lda);
    AT(A, r0 + ci, c0 + cj, lda) = s;
    tile_sums(c, A, lda, I, J, &t);
    slack_t sl = {ci, cj, diag, tau_of(c, t.ca[cj], AT(c->gc, 2 * I, c0 + cj, c->ldc))};
    if (tile_flags(c, I, J, &t, &f, NULL, &sl, NULL) == 0) {
      kind = 1;
    } else {
      AT(A, r0 + ci, c0 + cj, lda) = old;
    }
  } else if (line) {
    if (rebuild_line(c, A, lda, I, J, line, line == 1 ? ig : jf[0], &t, &f)) kind = 4 + line;
  } else if (repair) {
    kind = 2;
  }
  if (kind == 1) { c->rep->corrected++; c->rep->status |= 1; add_event(c->rep, c->iter, 1, r0 + ci, c0 + cj); }
  else if (kind == 5) { c->rep->corrected++; c->rep->status |= 1; add_event(c->rep, c->iter, 5, r0 + ig, c0); }
  else if (kind == 6) { c->rep->corrected++; c->rep->status |= 1; add_event(c->rep, c->iter, 6, r0, c0 + jf[0]); }
  else if (kind == 2) { c->rep->checksum_repaired++; c->rep->status |= 2; add_event(c->rep, c->iter, 2, r0, c0); }
  else { c->rep->uncorrectable++; c->rep->status |= 4; add_event(c->rep, c->iter, 3, r0, c0); }
  /* refresh the tile's checksums from the (corrected) data */
  tile_sums(c, A, lda, I, J, &t);
  store_sums(c, I, J, &t);
#undef t
#undef f
  free(tp);
  free(fp);
}

/* the tiles I >= Ia, J >= Ja (lower tiles only when sym), in the serial
   visiting order: tile-columns left to right, tile-rows top to bottom */
static int tile_list(const ctx_t* c, int Ia, int Ja, int* IJ) {
  int nt = 0;
  for (int J = Ja; J < c->N; ++J)
    for (int I = Ia; I < c->N; ++I) {
      if (c->sym && I < J) continue;
      IJ[2 * nt] = I;
      IJ[2 * nt + 1] = J;
      nt++;
    }
  return nt;
}

/* verify tiles I >= Ia, J >= Ja (lower tiles only when sym); flagged tiles go
   to correction, clean ones get their checksums refreshed from the data.
   Tiles are independent: their sums and comparisons run in parallel, the
   flagged ones are then corrected one by one in the visiting order. */
static void verify_region(ctx_t* c, double* A, int lda, int Ia, int Ja) {
  int* IJ = malloc(sizeof(int) * 2 * (size_t)c->N * c->N + 2);
  int nt = tile_list(c, Ia, Ja, IJ);
  int* flagged = calloc((size_t)nt + 1, sizeof(int));
  double* mr = calloc((size_t)nt + 1, sizeof(double));
#pragma omp parallel
  {
    tsums_t* t = malloc(sizeof(tsums_t));
    tflags_t* f = malloc(sizeof(tflags_t));
#pragma omp for schedule(dynamic, 1)
    for (int q = 0; q < nt; ++q) {
      int I = IJ[2 * q], J = IJ[2 * q + 1];
      tile_sums(c, A, lda, I, J, t);
      double m = 0.0;
      if (tile_flags(c, I, J, t, f, &m, NULL, NULL)) flagged[q] = 1;
      else { mr[q] = m; store_sums(c, I, J, t); }
    }
    free(t);
    free(f);
  }
  for (int q = 0; q < nt; ++q) {
    if (flagged[q]) {
      c->rep->flagged_tiles++;
      note_flag(c);
      correct_tile(c, A, lda, IJ[2 * q], IJ[2 * q + 1]);
    } else if (mr[q] > c->rep->max_ratio) {
      c->rep->max_ratio = mr[q];
    }
  }
  free(IJ);
  free(flagged);
  free(mr);
}

/* encode tiles I >= Ia, J >= Ja (lower tiles only when sym) from the data:
   the start of a protected stretch of iterations; the magnitude terms of the
   previous update are cleared */
static void encode_region(ctx_t* c, const double* A, int lda, int Ia, int Ja) {
  int* IJ = malloc(sizeof(int) * 2 * (size_t)c->N * c->N + 2);
  int nt = tile_list(c, Ia, Ja, IJ);
#pragma omp parallel
  {
    tsums_t* t = malloc(sizeof(tsums_t));
#pragma omp for schedule(dynamic, 1)
    for (int q = 0; q < nt; ++q) {
      tile_sums(c, A, lda, IJ[2 * q], IJ[2 * q + 1], t);
      store_sums(c, IJ[2 * q], IJ[2 * q + 1], t);
    }
    free(t);
  }
  free(IJ);
  memset(c->gc, 0, (size_t)c->ldc * c->n * sizeof(double));
  memset(c->gr, 0, (size_t)c->n * 2 * c->N * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* X / Y checksum vectors for the carry rules.                         */
/* X is the left factor of an update (rows [xr0,n), nb columns from    */
/* column xc0); for rows inside tile-row `dI` it is read through a mask*/
/* (0 full, 1 lower with diagonal, 2 unit lower).                      */
/* ------------------------------------------------------------------ */
enum { XM_FULL = 0, XM_LOWER = 1, XM_UNIT = 2 };

static inline double xval(const double* A, int lda, int i, int p, int xc0, int dI_r0, int dI_r1, int mode) {
  if (i >= dI_r0 && i < dI_r1 && mode != XM_FULL) {
    int ii = i - dI_r0;
    if (ii < p) return 0.0;
    if (ii == p && mode == XM_UNIT) return 1.0;
  }
  return AT(A, i, xc0 + p, lda);
}

typedef struct { double *e, *w, *a, *wa; } vec4_t; /* each N x nb, index [I*nb + p] */

static void x_colsums(ctx_t* c, const double* A, int lda, int I0, int xc0, int kw, int dI, int mode, vec4_t* s) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int I = I0; I < c->N; ++I) {
    int r0 = I * c->nb, h = tlen(c, I);
    for (int p = 0; p < kw; ++p) {
      acc_t e = {0, 0}, w = {0, 0};
      double a = 0, wa = 0;
      for (int i = 0; i < h; ++i) {
        double v = rop(c->prec, xval(A, lda, r0 + i, p, xc0, dI * c->nb, dI * c->nb + tlen(c, dI), mode));
        acc_add(&e, v); acc_fma(&w, (double)(i + 1), v); a += fabs(v); wa += (double)(i + 1) * fabs(v);
      }
      s->e[I * c->nb + p] = acc_val(e); s->w[I * c->nb + p] = acc_val(w); s->a[I * c->nb + p] = a; s->wa[I * c->nb + p] = wa;
    }
  }
}

/* Generic carry for C -= X*Y over tiles I >= I0, J >= J0 (I >= J when sym).
   Y(p, j) is given by yfun.  Column side: colchk -= [e;w]^T X_I * Y.
   Row side: rowchk -= X * (Y_J [e, w]).  gc / gr receive the matching
   magnitudes (|.|-sums of the same products) used by the thresholds. */
typedef double (*yfun_t)(const void* ctx, int p, int j);

static void carry(ctx_t* c, const double* A, int lda, int I0, int J0, int xc0, int kw, int dI, int mode,
                  yfun_t Y, const void* yctx) {
  int N = c->N, nb = c->nb, n = c->n;
  vec4_t s;
  s.e = calloc((size_t)N * nb, sizeof(double)); s.w = calloc((size_t)N * nb, sizeof(double));
  s.a = calloc((size_t)N * nb, sizeof(double)); s.wa = calloc((size_t)N * nb, sizeof(double));
  vec4_t t;
  t.e = calloc((size_t)N * nb, sizeof(double)); t.w = calloc((size_t)N * nb, sizeof(double));
  t.a = calloc((size_t)N * nb, sizeof(double)); t.wa = calloc((size_t)N * nb, sizeof(double));
  x_colsums(c, A, lda, I0, xc0, kw, dI, mode, &s);
  /* row sums of Y over each tile-column J */
#pragma omp parallel for schedule(dynamic, 1)
  for (int J = J0; J < N; ++J) {
    int c0 = J * nb, w = tlen(c, J);
    for (int p = 0; p < kw; ++p) {
      acc_t e = {0, 0}, ww = {0, 0};
      double a = 0, wa = 0;
      for (int j = 0; j < w; ++j) {
        double v = rop(c->prec, Y(yctx, p, c0 + j));
        acc_add(&e, v); acc_fma(&ww, (double)(j + 1), v); a += fabs(v); wa += (double)(j + 1) * fabs(v);
      }
      t.e[J * nb + p] = acc_val(e); t.w[J * nb + p] = acc_val(ww); t.a[J * nb + p] = a; t.wa[J * nb + p] = wa;
    }
  }
  /* column side */
#pragma omp parallel for schedule(dynamic, 16)
  for (int j = J0 * nb; j < n; ++j) {
    int Jj = j / nb;
    for (int I = I0; I < N; ++I) {
      if (c->sym && I < Jj) continue;
      acc_t ue = {AT(c->cc, 2 * I, j, c->ldc), 0}, uw = {AT(c->cc, 2 * I + 1, j, c->ldc), 0};
      double ga = 0, gwa = 0;
      for (int p = 0; p < kw; ++p) {
        double y = rop(c->prec, Y(yctx, p, j));
        acc_fma(&ue, -s.e[I * nb + p], y); acc_fma(&uw, -s.w[I * nb + p], y);
        ga += s.a[I * nb + p] * fabs(y); gwa += s.wa[I * nb + p] * fabs(y);
      }
      AT(c->cc, 2 * I, j, c->ldc) = acc_val(ue);
      AT(c->cc, 2 * I + 1, j, c->ldc) = acc_val(uw);
      AT(c->gc, 2 * I, j, c->ldc) = ga;
      AT(c->gc, 2 * I + 1, j, c->ldc) = gwa;
    }
  }
  /* row side (full checksums only) */
  int dr0 = dI * nb, dr1 = dI * nb + tlen(c, dI);
  if (c->level == 2) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = I0 * nb; i < n; ++i) {
      int Ii = i / nb;
      for (int J = J0; J < N; ++J) {
        if (c->sym && Ii < J) continue;
        acc_t ue = {AT(c->rc, i, 2 * J, c->ldr), 0}, uw = {AT(c->rc, i, 2 * J + 1, c->ldr), 0};
        double ga = 0, gwa = 0;
        for (int p = 0; p < kw; ++p) {
          double x = rop(c->prec, xval(A, lda, i, p, xc0, dr0, dr1, mode));
          acc_fma(&ue, -x, t.e[J * nb + p]); acc_fma(&uw, -x, t.w[J * nb + p]);
          ga += fabs(x) * t.a[J * nb + p]; gwa += fabs(x) * t.wa[J * nb + p];
        }
        AT(c->rc, i, 2 * J, c->ldr) = acc_val(ue);
        AT(c->rc, i, 2 * J + 1, c->ldr) = acc_val(uw);
        AT(c->gr, i, 2 * J, c->ldr) = ga;
        AT(c->gr, i, 2 * J + 1, c->ldr) = gwa;
      }
    }
  }
  free(s.e); free(s.w); free(s.a); free(s.wa);
  free(t.e); free(t.w); free(t.a); free(t.wa);
}

/* Panel / PU check (detection only): the carried column checksums of tile
   rows I in [I0, N) over columns [j0, j1) must equal [e;w]^T X_I * M(:, j)
   (+ an optional exact term).  M(p, j) and |M|-magnitudes come from mfun. */
typedef void (*mfun_t)(const void* ctx, int I, int p, int j, double* m, double* mabs);
typedef void (*efun_t)(const void* ctx, int I, int j, double* ee, double* ew, double* ea, double* ewa);

static void panel_check(ctx_t* c, const double* A, int lda, int I0, int I1, int xc0, int kw, int dI, int mode,
                        int j0, int j1, mfun_t M, efun_t E, const void* mctx) {
  int N = c->N, nb = c->nb;
  vec4_t s;
  s.e = calloc((size_t)N * nb, sizeof(double)); s.w = calloc((size_t)N * nb, sizeof(double));
  s.a = calloc((size_t)N * nb, sizeof(double)); s.wa = calloc((size_t)N * nb, sizeof(double));
  x_colsums(c, A, lda, I0, xc0, kw, dI, mode, &s);
  int* flagged = calloc((size_t)N + 1, sizeof(int));
  double* mr = calloc((size_t)N + 1, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
  for (int I = I0; I < I1; ++I) {
    for (int j = j0; j < j1; ++j) {
      double ce = AT(c->cc, 2 * I, j, c->ldc), cw = AT(c->cc, 2 * I + 1, j, c->ldc);
      acc_t xe = {ce, 0}, xw = {cw, 0};
      double ge = 0, gw = 0;
      for (int p = 0; p < kw; ++p) {
        double m, ma;
        M(mctx, I, p, j, &m, &ma);
        acc_fma(&xe, -s.e[I * nb + p], m); acc_fma(&xw, -s.w[I * nb + p], m);
        ge += s.a[I * nb + p] * ma; gw += s.wa[I * nb + p] * ma;
      }
      if (E) {
        double ee, ew, ea, ewa;
        E(mctx, I, j, &ee, &ew, &ea, &ewa);
        acc_add(&xe, -ee); acc_add(&xw, -ew); ge += ea; gw += ewa;
      }
      double de = acc_val(xe), dw = acc_val(xw);
      double te = tau_panel(c, fabs(ce) + ge), tw = tau_panel(c, fabs(cw) + gw);
      if (bad(de, te) || bad(dw, tw)) flagged[I] = 1;
      else {
        if (te > 0 && fabs(de) / te > mr[I]) mr[I] = fabs(de) / te;
        if (tw > 0 && fabs(dw) / tw > mr[I]) mr[I] = fabs(dw) / tw;
      }
    }
  }
  for (int I = I0; I < I1; ++I) {
    if (mr[I] > c->rep->max_ratio) c->rep->max_ratio = mr[I];
    if (flagged[I]) {
      c->rep->panel_flags++;
      c->rep->status |= 8;
      note_flag(c);
      add_event(c->rep, c->iter, 4, (int64_t)I * nb, j0);
    }
  }
  free(flagged);
  free(mr);
  free(s.e); free(s.w); free(s.a); free(s.wa);
}

/* fault injection: XOR one bit of a binary64 element */
static void flip(double* p, int bit) {
  uint64_t u;
  memcpy(&u, p, 8);
  u ^= (uint64_t)1 << bit;
  memcpy(p, &u, 8);
}

static void inject(ctx_t* c, double* A, int lda, const orc_fault* f, int nf, int iter) {
  for (int q = 0; q < nf; ++q) {
    if (f[q].iter != iter) continue;
    if (f[q].target == 0) flip(&AT(A, f[q].row, f[q].col, lda), f[q].bit);
    else if (f[q].target == 1 && c->cc) flip(&AT(c->cc, f[q].row, f[q].col, c->ldc), f[q].bit);
    else if (f[q].target == 2 && c->rc) flip(&AT(c->rc, f[q].row, f[q].col, c->ldr), f[q].bit);
  }
}

/* Faults in an operand of the trailing-update product (target 3: an element
   of the left operand, L21 or V, at its matrix position; target 4: of the
   right operand, U12 at its matrix position, or QR's W2 at (p, column)):
   the stored element is flipped for the duration of that product only, as
   a fault in the product's read of it would be, so the error spreads along
   a row (left operand) or a column (right operand) of the updated matrix
   while the operand itself and the checksum carry stay intact.  Called once
   before and once after the product (the flip undoes itself). */
static void flip_operands(double* A, int lda, double* W2, int ldw, const orc_fault* f, int nf, int iter) {
  for (int q = 0; q < nf; ++q) {
    if (f[q].iter != iter) continue;
    if (f[q].target == 3) flip(&AT(A, f[q].row, f[q].col, lda), f[q].bit);
    else if (f[q].target == 4) {
      if (W2) flip(&W2[(size_t)f[q].row + (size_t)f[q].col * (size_t)ldw], f[q].bit);
      else flip(&AT(A, f[q].row, f[q].col, lda), f[q].bit);
    }
  }
}

/* protection level of iteration k: the caller's per-iteration levels, or
   the call's level for every iteration */
static int level_of(const int8_t* levels, int k, int protect) {
  int v = levels ? levels[k] : protect;
  return v < 0 ? 0 : (v > 2 ? 2 : v);
}

static int ctx_init(ctx_t* c, int n, int nb, int sym, int prec, int protect, double ts, orc_report* rep) {
  memset(c, 0, sizeof(*c));
  c->n = n; c->nb = nb; c->N = (n + nb - 1) / nb; c->sym = sym; c->prec = prec; c->protect = protect;
  c->u = unit_round(prec); c->ts = ts; c->rep = rep;
  memset(rep, 0, sizeof(*rep));
  rep->first_flag_iter = -1;
  if (nb > 1024) return -1;
  if (protect) {
    c->ldc = 2 * c->N; c->ldr = n;
    c->cc = calloc((size_t)c->ldc * n, sizeof(double));
    c->gc = calloc((size_t)c->ldc * n, sizeof(double));
    c->rc = calloc((size_t)n * 2 * c->N, sizeof(double));
    c->gr = calloc((size_t)n * 2 * c->N, sizeof(double));
  }
  return 0;
}

static void ctx_free(ctx_t* c) { free(c->cc); free(c->gc); free(c->rc); free(c->gr); }

static void zero_g(ctx_t* c) {
  if (!c->protect) return;
  memset(c->gc, 0, (size_t)c->ldc * c->n * sizeof(double));
  memset(c->gr, 0, (size_t)c->n * 2 * c->N * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* Update loops shared by the decompositions.  Rows are split into     */
/* blocks of RB handled by one thread each; inside a block every       */
/* element still sees its operations in the plain serial order.        */
/* ------------------------------------------------------------------ */
#define RB 256
typedef double v4d __attribute__((vector_size(32)));  /* four independent lanes */

/* C(i, j) -= sum_p X(i, p) Y(p, j) for rows i in [0, mr) and columns j in
   [0, nc) (only i >= j when lower): element (i, j) accumulates its products
   over p = 0, 1, ..., kw-1 (rounded to prec after every step), then C(i, j)
   becomes rs(C(i, j) - acc).  X is column-major with leading dimension
   ldx, Y(p, j) = Y[p + j*ldy]. */
static void update_rows(int prec, int mr, int nc, int kw, const double* X, int ldx, const double* Y, int ldy,
                        double* C, int ldc, int lower) {
#pragma omp parallel
  {
    double* acc = malloc(sizeof(double) * 4 * RB);
#pragma omp for schedule(dynamic, 1)
    for (int ib = 0; ib < mr; ib += RB) {
      int ie = imin(ib + RB, mr);
      int jend = lower ? imin(nc, ie) : nc;
      /* four columns at a time; rows [i0, ie) of the block, where rows above
         a column's diagonal (lower) are computed but not stored */
      for (int j0 = 0; j0 < jend; j0 += 4) {
        int nj = imin(4, jend - j0);
        int i0 = lower ? imax(ib, j0) : ib;
        int i = i0;
        if (prec == PR64 && nj == 4) {
          /* 8 rows x 4 columns of accumulators held in registers: each lane
             of a v4d is one element's own running sum */
          const double* y0 = Y + (size_t)j0 * ldy;
          for (; i + 8 <= ie; i += 8) {
            v4d a[4][2];
            for (int jj = 0; jj < 4; ++jj) a[jj][0] = a[jj][1] = (v4d){0.0, 0.0, 0.0, 0.0};
            for (int p = 0; p < kw; ++p) {
              v4d x0, x1;
              memcpy(&x0, X + (size_t)p * ldx + i, sizeof x0);
              memcpy(&x1, X + (size_t)p * ldx + i + 4, sizeof x1);
              for (int jj = 0; jj < 4; ++jj) {
                double y = y0[p + (size_t)jj * ldy];
                a[jj][0] = a[jj][0] + x0 * y;
                a[jj][1] = a[jj][1] + x1 * y;
              }
            }
            for (int jj = 0; jj < 4; ++jj) {
              memcpy(acc + jj * RB + (i - ib), &a[jj][0], sizeof(v4d));
              memcpy(acc + jj * RB + (i - ib) + 4, &a[jj][1], sizeof(v4d));
            }
          }
        }
        /* the remaining rows, one accumulator per element */
        for (int jj = 0; jj < nj; ++jj)
          for (int r = i; r < ie; ++r) acc[jj * RB + (r - ib)] = 0.0;
        for (int p = 0; p < kw; ++p) {
          const double* x = X + (size_t)p * ldx;
          for (int jj = 0; jj < nj; ++jj) {
            double y = Y[p + (size_t)(j0 + jj) * ldy];
            double* aj = acc + jj * RB - ib;
            for (int r = i; r < ie; ++r) aj[r] = rs(prec, aj[r] + x[r] * y);
          }
        }
        for (int jj = 0; jj < nj; ++jj) {
          int j = j0 + jj;
          double* cj = C + (size_t)j * ldc;
          const double* aj = acc + jj * RB - ib;
          for (int r = lower ? imax(i0, j) : i0; r < ie; ++r) cj[r] = rs(prec, cj[r] - aj[r]);
        }
      }
    }
    free(acc);
  }
}

/* operand copies of an update, rounded as the update's inputs are:
   X[i + p*m] = rop(A(r0 + i, c0 + p)) and Y[p + j*kw] = rop(A(yr0 + p, yc0 + j))
   (ty = 0) or rop(A(yc0 + j, yr0 + p)) (ty = 1, a transposed operand) */
static double* copy_x(int prec, const double* A, int lda, int r0, int m, int c0, int kw) {
  double* X = malloc(sizeof(double) * ((size_t)m * kw + 1));
#pragma omp parallel for schedule(static)
  for (int p = 0; p < kw; ++p)
    for (int i = 0; i < m; ++i) X[i + (size_t)p * m] = rop(prec, AT(A, r0 + i, c0 + p, lda));
  return X;
}
static double* copy_y(int prec, const double* A, int lda, int yr0, int kw, int yc0, int nc, int ty) {
  double* Y = malloc(sizeof(double) * ((size_t)nc * kw + 1));
#pragma omp parallel for schedule(static)
  for (int j = 0; j < nc; ++j)
    for (int p = 0; p < kw; ++p)
      Y[p + (size_t)j * kw] = rop(prec, ty ? AT(A, yc0 + j, yr0 + p, lda) : AT(A, yr0 + p, yc0 + j, lda));
  return Y;
}

/* ------------------------------------------------------------------ */
/* Blocked right-looking Cholesky (lower) with ABFT.                  */
/* ------------------------------------------------------------------ */
typedef struct { const double* A; int lda; int c0; } lctx_t;
/* Y = L21^T : Y(p, j) = L(j, c0 + p) */
static double y_lt(const void* v, int p, int j) { const lctx_t* l = v; return AT(l->A, j, l->c0 + p, l->lda); }
/* panel check matrix M = L_kk^T : M(p, j) = L(j, c0 + p) for p <= j - c0 */
static void m_lkkT(const void* v, int I, int p, int j, double* m, double* ma) {
  const lctx_t* l = v;
  (void)I;
  int jj = j - l->c0;
  double x = (p <= jj) ? AT(l->A, j, l->c0 + p, l->lda) : 0.0;
  *m = x; *ma = fabs(x);
}

int orc_abft_potrf(int n, int nb, double* A, int lda, int prec, int protect, double tau_scale,
                   const orc_fault* faults, int nfaults, const int8_t* levels, orc_report* rep) {
  ctx_t c;
  if (ctx_init(&c, n, nb, 1, prec, protect || levels, tau_scale, rep)) return -2;
  if (prec != PR64)
    for (int j = 0; j < n; ++j) for (int i = j; i < n; ++i) AT(A, i, j, lda) = rs(prec, AT(A, i, j, lda));
  int info = 0, prev = 0;
  for (int k = 0; k < c.N; ++k) {
    c.iter = k;
    /* protection of this iteration; a protected stretch starts from
       checksums encoded from the data */
    int lev = level_of(levels, k, protect);
    c.level = lev;
    if (lev > prev) encode_region(&c, A, lda, k, k);
    prev = lev;
    int c0 = k * nb, w = tlen(&c, k), c1 = c0 + w;
    /* PD: Cholesky of the diagonal tile (right-looking inside the tile) */
    for (int j = c0; j < c1 && !info; ++j) {
      double d = AT(A, j, j, lda);
      if (!(d > 0.0)) { info = j + 1; break; }
      d = rs(prec, sqrt(d));
      AT(A, j, j, lda) = d;
      for (int i = j + 1; i < c1; ++i) AT(A, i, j, lda) = rs(prec, AT(A, i, j, lda) / d);
      for (int jj = j + 1; jj < c1; ++jj)
        for (int i = jj; i < c1; ++i)
          AT(A, i, jj, lda) = rs(prec, AT(A, i, jj, lda) - AT(A, i, j, lda) * AT(A, jj, j, lda));
    }
    if (info) break;
    /* PU: L21 = A21 * L_kk^{-T}, forward substitution along each row:
       element (i, j) subtracts L(i, p) L(j, p) for p = c0 .. j-1 in order,
       then is divided by L(j, j) */
#pragma omp parallel for schedule(dynamic, 1)
    for (int ib = c1; ib < n; ib += RB) {
      int ie = imin(ib + RB, n);
      for (int j = c0; j < c1; ++j) {
        double* aj = &AT(A, 0, j, lda);
        for (int p = c0; p < j; ++p) {
          const double* ap = &AT(A, 0, p, lda);
          double ljp = AT(A, j, p, lda);
          for (int i = ib; i < ie; ++i) aj[i] = rs(prec, aj[i] - ap[i] * ljp);
        }
        double d = AT(A, j, j, lda);
        for (int i = ib; i < ie; ++i) aj[i] = rs(prec, aj[i] / d);
      }
    }
    lctx_t l = {A, lda, c0};
    if (lev) {
      /* panel check: e^T A_Ik = (e^T L_I) L_kk^T for every tile-row I >= k */
      panel_check(&c, A, lda, k, c.N, c0, w, k, XM_LOWER, c0, c1, m_lkkT, NULL, &l);
    }
    if (c1 >= n) break;
    /* TMU: A22 -= L21 L21^T (lower part), operands rounded for MP forms */
    {
      int m = n - c1;
      flip_operands(A, lda, NULL, 0, faults, nfaults, k);
      double* X = copy_x(prec, A, lda, c1, m, c0, w);
      double* Y = copy_y(prec, A, lda, c0, w, c1, m, 1);
      flip_operands(A, lda, NULL, 0, faults, nfaults, k);
      update_rows(prec, m, m, w, X, m, Y, w, &AT(A, c1, c1, lda), lda, 1);
      free(X);
      free(Y);
    }
    if (lev) {
      zero_g(&c);
      carry(&c, A, lda, k + 1, k + 1, c0, w, k, XM_LOWER, y_lt, &l);
    }
    inject(&c, A, lda, faults, nfaults, k);
    if (lev) verify_region(&c, A, lda, k + 1, k + 1);
  }
  ctx_free(&c);
  return info;
}

/* ------------------------------------------------------------------ */
/* Blocked right-looking LU with partial pivoting and ABFT.           */
/* ------------------------------------------------------------------ */
typedef struct { const double* A; int lda; int c0, c1; } uctx_t;
/* Y = U12 : Y(p, j) = A(c0 + p, j) */
static double y_u12(const void* v, int p, int j) { const uctx_t* u = v; return AT(u->A, u->c0 + p, j, u->lda); }
/* panel check M = U_kk (upper incl. diagonal) */
static void m_ukk(const void* v, int I, int p, int j, double* m, double* ma) {
  const uctx_t* u = v;
  (void)I;
  double x = (p <= j - u->c0) ? AT(u->A, u->c0 + p, j, u->lda) : 0.0;
  *m = x; *ma = fabs(x);
}
static void m_u12(const void* v, int I, int p, int j, double* m, double* ma) {
  const uctx_t* u = v;
  (void)I;
  double x = AT(u->A, u->c0 + p, j, u->lda);
  *m = x; *ma = fabs(x);
}

int orc_abft_getrf(int n, int nb, double* A, int lda, int32_t* ipiv, int prec, int protect, double tau_scale,
                   const orc_fault* faults, int nfaults, const int8_t* levels, orc_report* rep) {
  ctx_t c;
  if (ctx_init(&c, n, nb, 0, prec, protect || levels, tau_scale, rep)) return -2;
  if (prec != PR64)
    for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i) AT(A, i, j, lda) = rs(prec, AT(A, i, j, lda));
  int info = 0, prev = 0;
  double* porig = (protect || levels) ? malloc((size_t)n * nb * sizeof(double)) : NULL;
  for (int k = 0; k < c.N; ++k) {
    c.iter = k;
    int lev = level_of(levels, k, protect);
    c.level = lev;
    if (lev > prev) encode_region(&c, A, lda, k, k);
    prev = lev;
    int c0 = k * nb, w = tlen(&c, k), c1 = c0 + w;
    int mp = n - c0;
    if (lev)
      for (int j = 0; j < w; ++j) for (int i = 0; i < mp; ++i) porig[i + (size_t)j * mp] = AT(A, c0 + i, c0 + j, lda);
    /* PD: getf2 on the panel.  Each interchange is applied to the panel
       columns at once and to the other columns after the panel (column by
       column, in the panel's order): nothing else reads those columns in
       between, so every value is the same as with whole-row swaps. */
    for (int j = c0; j < c1; ++j) {
      int p = pick_pivot(A, lda, j, j, n);
      ipiv[j] = p + 1;
      if (p != j) {
        if (lev) {
          /* checksum fix-up of the panel columns, from the original panel
             values; row checksums move with their rows */
          int Ir = j / nb, Ip = p / nb;
          double wr = (double)(j - Ir * nb + 1), wp = (double)(p - Ip * nb + 1);
          for (int jj = c0; jj < c1; ++jj) {
            double ar = porig[(j - c0) + (size_t)(jj - c0) * mp], ap = porig[(p - c0) + (size_t)(jj - c0) * mp];
            AT(c.cc, 2 * Ir, jj, c.ldc) += ap - ar;
            AT(c.cc, 2 * Ir + 1, jj, c.ldc) += wr * (ap - ar);
            AT(c.cc, 2 * Ip, jj, c.ldc) += ar - ap;
            AT(c.cc, 2 * Ip + 1, jj, c.ldc) += wp * (ar - ap);
          }
          for (int jj = 0; jj < w; ++jj) {
            double t = porig[(j - c0) + (size_t)jj * mp];
            porig[(j - c0) + (size_t)jj * mp] = porig[(p - c0) + (size_t)jj * mp];
            porig[(p - c0) + (size_t)jj * mp] = t;
          }
          swap_rows(c.rc, c.ldr, j, p, 0, 2 * c.N);
        }
        swap_rows(A, lda, j, p, c0, c1);
      }
      double piv = AT(A, j, j, lda);
      if (piv == 0.0) { if (!info) info = j + 1; continue; }
      for (int i = j + 1; i < n; ++i) AT(A, i, j, lda) = rs(prec, AT(A, i, j, lda) / piv);
#pragma omp parallel for schedule(static) if ((size_t)(c1 - j) * (size_t)(n - j) > ((size_t)1 << 16))
      for (int cc = j + 1; cc < c1; ++cc) {
        double u = AT(A, j, cc, lda);
        for (int i = j + 1; i < n; ++i) AT(A, i, cc, lda) = rs(prec, AT(A, i, cc, lda) - AT(A, i, j, lda) * u);
      }
    }
    /* the panel's interchanges on the columns left and right of it; each
       trailing column's checksum fix-up uses the column's current values at
       each interchange */
#pragma omp parallel for schedule(dynamic, 16)
    for (int jj = 0; jj < n; ++jj) {
      if (jj >= c0 && jj < c1) continue;
      for (int j = c0; j < c1; ++j) {
        int p = ipiv[j] - 1;
        if (p == j) continue;
        double ar = AT(A, j, jj, lda), ap = AT(A, p, jj, lda);
        if (lev && jj >= c1) {
          int Ir = j / nb, Ip = p / nb;
          double wr = (double)(j - Ir * nb + 1), wp = (double)(p - Ip * nb + 1);
          AT(c.cc, 2 * Ir, jj, c.ldc) += ap - ar;
          AT(c.cc, 2 * Ir + 1, jj, c.ldc) += wr * (ap - ar);
          AT(c.cc, 2 * Ip, jj, c.ldc) += ar - ap;
          AT(c.cc, 2 * Ip + 1, jj, c.ldc) += wp * (ar - ap);
        }
        AT(A, j, jj, lda) = ap;
        AT(A, p, jj, lda) = ar;
      }
    }
    uctx_t u = {A, lda, c0, c1};
    if (lev) panel_check(&c, A, lda, k, c.N, c0, w, k, XM_UNIT, c0, c1, m_ukk, NULL, &u);
    if (c1 >= n) break;
    /* PU: U12 = L11^{-1} A12, unit lower forward substitution per column:
       element (i, j) subtracts L(i, p) U(p, j) for p = c0 .. i-1 in order */
#pragma omp parallel for schedule(dynamic, 16)
    for (int j = c1; j < n; ++j)
      for (int p = c0; p < c1; ++p) {
        double u = AT(A, p, j, lda);
        for (int i = p + 1; i < c1; ++i) AT(A, i, j, lda) = rs(prec, AT(A, i, j, lda) - AT(A, i, p, lda) * u);
      }
    /* PU check: (e^T L11) U12 = e^T A12 on tile-row k */
    if (lev) panel_check(&c, A, lda, k, k + 1, c0, w, k, XM_UNIT, c1, n, m_u12, NULL, &u);
    /* TMU: A22 -= L21 U12 */
    {
      int m = n - c1;
      flip_operands(A, lda, NULL, 0, faults, nfaults, k);
      double* X = copy_x(prec, A, lda, c1, m, c0, w);
      double* Y = copy_y(prec, A, lda, c0, w, c1, m, 0);
      flip_operands(A, lda, NULL, 0, faults, nfaults, k);
      update_rows(prec, m, m, w, X, m, Y, w, &AT(A, c1, c1, lda), lda, 0);
      free(X);
      free(Y);
    }
    if (lev) {
      zero_g(&c);
      carry(&c, A, lda, k + 1, k + 1, c0, w, k, XM_FULL, y_u12, &u);
    }
    inject(&c, A, lda, faults, nfaults, k);
    if (lev) verify_region(&c, A, lda, k + 1, k + 1);
  }
  free(porig);
  ctx_free(&c);
  return info;
}

/* ------------------------------------------------------------------ */
/* Blocked Householder QR with ABFT (FP64).                            */
/* ------------------------------------------------------------------ */
/* T factor, forward columnwise: T(j,j) = tau_j,
   T(0:j, j) = -tau_j T(0:j,0:j) (V(:,0:j)^T v_j); V unit lower from (c0,c0) */
static void larft(int n, const double* A, int lda, const double* tau, int c0, int w, double* T) {
  for (int j = 0; j < w; ++j) {
    for (int i = 0; i < w; ++i) T[i + j * w] = 0.0;
    T[j + j * w] = tau[c0 + j];
    double* g = malloc(sizeof(double) * (j + 1));
#pragma omp parallel for schedule(static) if ((size_t)j * (size_t)(n - c0) > ((size_t)1 << 16))
    for (int q = 0; q < j; ++q) {
      /* V(:,q)^T V(:,j), V(c0+j, j) = 1, rows above c0+j of column j are 0 */
      double s = AT(A, c0 + j, c0 + q, lda); /* V(c0+j, q) * 1 */
      for (int i = c0 + j + 1; i < n; ++i) s += AT(A, i, c0 + q, lda) * AT(A, i, c0 + j, lda);
      g[q] = s;
    }
    for (int i = 0; i < j; ++i) {
      double s = 0.0;
      for (int q = i; q < j; ++q) s += T[i + q * w] * g[q];
      T[i + j * w] = -tau[c0 + j] * s;
    }
    free(g);
  }
}

/* W = V^T C and W2 = T^T W for C = columns [c1, n) of rows [c0, n):
   W(p, j) = C(c0+p, j) + sum over i > c0+p of V(i, p) C(i, j), each a plain
   running sum over i in ascending order, then
   W2(p, j) = sum over q <= p of T(q, p) W(q, j) in ascending q.
   Blocks of 8 values of p and 4 columns advance their 32 independent sums
   together (lanes of a v4d are the 4 columns of one p), which changes no
   sum's order. */
static void qr_w(int n, const double* A, int lda, int c0, int w, int c1, const double* T, double* W2) {
  int ncol = n - c1;
#pragma omp parallel
  {
    double* wv = malloc(sizeof(double) * 4 * (size_t)w);
    double* ct = malloc(sizeof(double) * 4 * (size_t)(n - c0) + 32);
#pragma omp for schedule(dynamic, 1)
    for (int jb = 0; jb < ncol; jb += 4) {
      int nj = imin(4, ncol - jb);
      /* rows of the 4-column block side by side: ct[4 (i - c0) + jj] = C(i, j) */
      for (int i = c0; i < n; ++i)
        for (int jj = 0; jj < 4; ++jj) ct[4 * (size_t)(i - c0) + jj] = jj < nj ? AT(A, i, c1 + jb + jj, lda) : 0.0;
      for (int p0 = 0; p0 < w; p0 += 8) {
        int np = imin(8, w - p0);
        double sacc[8][4];
        for (int q = 0; q < np; ++q)
          for (int jj = 0; jj < 4; ++jj) sacc[q][jj] = ct[4 * (size_t)(p0 + q) + jj];
        /* rows inside the block of p: only the sums that have started */
        for (int i = c0 + p0 + 1; i < c0 + p0 + np && i < n; ++i)
          for (int q = 0; q < np; ++q)
            if (c0 + p0 + q < i)
              for (int jj = 0; jj < 4; ++jj) sacc[q][jj] += AT(A, i, c0 + p0 + q, lda) * ct[4 * (size_t)(i - c0) + jj];
        if (np == 8) {
          v4d a[8];
          for (int q = 0; q < 8; ++q) memcpy(&a[q], sacc[q], sizeof(v4d));
          for (int i = c0 + p0 + 8; i < n; ++i) {
            v4d cv;
            memcpy(&cv, ct + 4 * (size_t)(i - c0), sizeof cv);
            for (int q = 0; q < 8; ++q) a[q] = a[q] + AT(A, i, c0 + p0 + q, lda) * cv;
          }
          for (int q = 0; q < 8; ++q) memcpy(sacc[q], &a[q], sizeof(v4d));
        } else {
          for (int i = c0 + p0 + np; i < n; ++i)
            for (int q = 0; q < np; ++q)
              for (int jj = 0; jj < 4; ++jj) sacc[q][jj] += AT(A, i, c0 + p0 + q, lda) * ct[4 * (size_t)(i - c0) + jj];
        }
        for (int q = 0; q < np; ++q)
          for (int jj = 0; jj < 4; ++jj) wv[(p0 + q) + (size_t)jj * w] = sacc[q][jj];
      }
      for (int jj = 0; jj < nj; ++jj)
        for (int p = 0; p < w; ++p) {
          double s = 0.0;
          for (int q = 0; q <= p; ++q) s += T[q + p * w] * wv[q + (size_t)jj * w];
          W2[p + (size_t)(c1 + jb + jj) * w] = s;
        }
    }
    free(wv);
    free(ct);
  }
}

typedef struct { const double* A; int lda; int c0, w, n, nb, k; const double* T; double* W2; const double* Z; const double* Zabs; } qctx_t;
static double y_w2(const void* v, int p, int j) { const qctx_t* q = v; return q->W2[p + (size_t)(j) * q->w]; }
/* panel check for QR: colchk(A)_I = [I==k] e^T R_kk - ([e;w]^T V_I) Z, Z = T V1^T R_kk */
static void m_qz(const void* v, int I, int p, int j, double* m, double* ma) {
  const qctx_t* q = v;
  (void)I;
  int jj = j - q->c0;
  *m = -q->Z[p + jj * q->w];
  *ma = q->Zabs[p + jj * q->w];
}
static void e_qr(const void* v, int I, int j, double* ee, double* ew, double* ea, double* ewa) {
  const qctx_t* q = v;
  *ee = *ew = *ea = *ewa = 0.0;
  int jj = j - q->c0;
  double nrm2 = 0.0;
  for (int i = 0; i <= jj; ++i) nrm2 += AT(q->A, q->c0 + i, j, q->lda) * AT(q->A, q->c0 + i, j, q->lda);
  /* backward-error allowance of the Householder panel: sqrt(m) ||R(:,j)|| */
  double bt = sqrt((double)(q->n - q->c0)) * sqrt(nrm2);
  *ea = bt;
  *ewa = bt * (double)q->nb;
  if (I == q->k) {
    for (int i = 0; i <= jj; ++i) {
      double r = AT(q->A, q->c0 + i, j, q->lda);
      *ee += r; *ew += (double)(i + 1) * r; *ea += fabs(r); *ewa += (double)(i + 1) * fabs(r);
    }
  }
}

int orc_abft_geqrf(int n, int nb, double* A, int lda, double* tau, int protect, double tau_scale,
                   const orc_fault* faults, int nfaults, const int8_t* levels, orc_report* rep) {
  ctx_t c;
  if (ctx_init(&c, n, nb, 0, PR64, protect || levels, tau_scale, rep)) return -2;
  int prev = 0;
  double* T = malloc(sizeof(double) * nb * nb);
  double* W2 = malloc(sizeof(double) * (size_t)nb * n);
  double* Z = malloc(sizeof(double) * nb * nb);
  double* Zabs = malloc(sizeof(double) * nb * nb);
  for (int k = 0; k < c.N; ++k) {
    c.iter = k;
    int lev = level_of(levels, k, protect);
    c.level = lev;
    if (lev > prev) encode_region(&c, A, lda, k, k);
    prev = lev;
    int c0 = k * nb, w = tlen(&c, k), c1 = c0 + w;
    geqr2_cols(n, A, lda, tau, c0, c1);
    larft(n, A, lda, tau, c0, w, T);
    qctx_t q = {A, lda, c0, w, n, nb, k, T, W2, Z, Zabs};
    if (lev) {
      /* Z = T * (V1^T R_kk) and its magnitude |T| (|V1|^T |R_kk|) */
      for (int j = 0; j < w; ++j) {
        double* y = malloc(sizeof(double) * w);
        double* ya = malloc(sizeof(double) * w);
        for (int p = 0; p < w; ++p) {
          double s = 0, sa = 0;
          for (int i = p; i <= j; ++i) {
            double vip = (i == p) ? 1.0 : AT(A, c0 + i, c0 + p, lda);
            double r = AT(A, c0 + i, c0 + j, lda);
            s += vip * r; sa += fabs(vip) * fabs(r);
          }
          y[p] = s; ya[p] = sa;
        }
        for (int p = 0; p < w; ++p) {
          double s = 0, sa = 0;
          for (int q2 = p; q2 < w; ++q2) { s += T[p + q2 * w] * y[q2]; sa += fabs(T[p + q2 * w]) * ya[q2]; }
          Z[p + j * w] = s; Zabs[p + j * w] = sa;
        }
        free(y); free(ya);
      }
      panel_check(&c, A, lda, k, c.N, c0, w, k, XM_UNIT, c0, c1, m_qz, e_qr, &q);
    }
    if (c1 >= n) break;
    /* TMU (larfb): W = V^T C, W2 = T^T W, C -= V W2 over rows [c0,n), cols [c1,n) */
    qr_w(n, A, lda, c0, w, c1, T, W2);
    flip_operands(A, lda, W2, w, faults, nfaults, k);
    /* C(i, j) -= sum over p <= min(i - c0, w - 1) of V(i, p) W2(p, j), with
       V(c0 + p, p) = 1, accumulated in ascending p: the rows of V's unit
       triangle term by term, the rows below it (all w terms, no unit
       entry) with the update loop above */
    {
      int mt = imin(w, n - c0);
#pragma omp parallel for schedule(dynamic, 16)
      for (int j = c1; j < n; ++j) {
        const double* y = W2 + (size_t)j * w;
        for (int i = c0; i < c0 + mt; ++i) {
          double acc = 0.0;
          for (int p = 0; p <= i - c0; ++p) acc += (i - c0 == p ? 1.0 : AT(A, i, c0 + p, lda)) * y[p];
          AT(A, i, j, lda) -= acc;
        }
      }
      if (n - c0 > w) {
        double* X = copy_x(PR64, A, lda, c0 + w, n - c0 - w, c0, w);
        update_rows(PR64, n - c0 - w, n - c1, w, X, n - c0 - w, W2 + (size_t)c1 * w, w, &AT(A, c0 + w, c1, lda), lda,
                    0);
        free(X);
      }
    }
    flip_operands(A, lda, W2, w, faults, nfaults, k);
    if (lev) {
      zero_g(&c);
      carry(&c, A, lda, k, k + 1, c0, w, k, XM_UNIT, y_w2, &q);
    }
    inject(&c, A, lda, faults, nfaults, k);
    if (lev) verify_region(&c, A, lda, k, k + 1);
  }
  free(T); free(W2); free(Z); free(Zabs);
  ctx_free(&c);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Standalone encode / verify (same checksum layout as above, general */
/* m x n, full tiles, no symmetric view).                              */
/* ------------------------------------------------------------------ */
void orc_encode(int m, int n, const double* A, int lda, int nb, double* colchk, int ldc, double* rowchk, int ldr) {
  int Tr = (m + nb - 1) / nb, Tc = (n + nb - 1) / nb;
  for (int j = 0; j < n; ++j)
    for (int I = 0; I < Tr; ++I) {
      acc_t e = {0, 0}, w = {0, 0};
      for (int i = I * nb; i < m && i < (I + 1) * nb; ++i) { acc_add(&e, AT(A, i, j, lda)); acc_fma(&w, (double)(i - I * nb + 1), AT(A, i, j, lda)); }
      AT(colchk, 2 * I, j, ldc) = acc_val(e);
      AT(colchk, 2 * I + 1, j, ldc) = acc_val(w);
    }
  for (int i = 0; i < m; ++i)
    for (int J = 0; J < Tc; ++J) {
      acc_t e = {0, 0}, w = {0, 0};
      for (int j = J * nb; j < n && j < (J + 1) * nb; ++j) { acc_add(&e, AT(A, i, j, lda)); acc_fma(&w, (double)(j - J * nb + 1), AT(A, i, j, lda)); }
      AT(rowchk, i, 2 * J, ldr) = acc_val(e);
      AT(rowchk, i, 2 * J + 1, ldr) = acc_val(w);
    }
}

/* returns the number of flagged tiles; flags[I + J*Tr] = 1 for flagged tiles */
int orc_verify(int m, int n, const double* A, int lda, int nb, const double* colchk, int ldc, const double* rowchk,
               int ldr, double tau_scale, int32_t* flags, double* max_ratio) {
  int Tr = (m + nb - 1) / nb, Tc = (n + nb - 1) / nb;
  double u = ldexp(1.0, -53), mr = 0.0;
  int nfl = 0;
  for (int J = 0; J < Tc; ++J)
    for (int I = 0; I < Tr; ++I) {
      int fl = 0;
      int r0 = I * nb, r1 = (I + 1) * nb < m ? (I + 1) * nb : m, c0 = J * nb, c1 = (J + 1) * nb < n ? (J + 1) * nb : n;
      for (int j = c0; j < c1; ++j) {
        acc_t e = {-AT(colchk, 2 * I, j, ldc), 0}, w = {-AT(colchk, 2 * I + 1, j, ldc), 0};
        double a = 0, wa = 0;
        for (int i = r0; i < r1; ++i) {
          double v = AT(A, i, j, lda);
          acc_add(&e, v); acc_fma(&w, (double)(i - r0 + 1), v); a += fabs(v); wa += (double)(i - r0 + 1) * fabs(v);
        }
        double de = acc_val(e), dw = acc_val(w);
        double te = (tau_scale * u * 4.0) * a, tw = (tau_scale * u * 4.0) * wa;
        if (!(fabs(de) <= te) || !(fabs(dw) <= tw) || !(te <= 1.79e308) || !(tw <= 1.79e308)) fl = 1;
        else { if (te > 0 && fabs(de) / te > mr) mr = fabs(de) / te; if (tw > 0 && fabs(dw) / tw > mr) mr = fabs(dw) / tw; }
      }
      for (int i = r0; i < r1; ++i) {
        acc_t e = {-AT(rowchk, i, 2 * J, ldr), 0}, w = {-AT(rowchk, i, 2 * J + 1, ldr), 0};
        double a = 0, wa = 0;
        for (int j = c0; j < c1; ++j) {
          double v = AT(A, i, j, lda);
          acc_add(&e, v); acc_fma(&w, (double)(j - c0 + 1), v); a += fabs(v); wa += (double)(j - c0 + 1) * fabs(v);
        }
        double de = acc_val(e), dw = acc_val(w);
        double te = (tau_scale * u * 4.0) * a, tw = (tau_scale * u * 4.0) * wa;
        if (!(fabs(de) <= te) || !(fabs(dw) <= tw) || !(te <= 1.79e308) || !(tw <= 1.79e308)) fl = 1;
        else { if (te > 0 && fabs(de) / te > mr) mr = fabs(de) / te; if (tw > 0 && fabs(dw) / tw > mr) mr = fabs(dw) / tw; }
      }
      if (flags) flags[I + J * Tr] = fl;
      nfl += fl;
    }
  if (max_ratio) *max_ratio = mr;
  return nfl;
}

/* Verify a square matrix against its per-tile checksums and send flagged
   tiles through the locate / correct rules of the factorizations (the
   detection interval here is the single call).  colchk is (2N) x n with
   ld 2N, rowchk n x (2N) with ld n; both are refreshed in place: clean and
   corrected tiles get sums recomputed from the data. */
int orc_verify_correct(int n, int nb, double* A, int lda, double* colchk, double* rowchk, double tau_scale,
                       orc_report* rep) {
  ctx_t c;
  if (ctx_init(&c, n, nb, 0, PR64, 2, tau_scale, rep)) return -2;
  c.level = 2;
  memcpy(c.cc, colchk, sizeof(double) * (size_t)c.ldc * n);
  memcpy(c.rc, rowchk, sizeof(double) * (size_t)c.ldr * 2 * c.N);
  c.iter = 0;
  verify_region(&c, A, lda, 0, 0);
  memcpy(colchk, c.cc, sizeof(double) * (size_t)c.ldc * n);
  memcpy(rowchk, c.rc, sizeof(double) * (size_t)c.ldr * 2 * c.N);
  ctx_free(&c);
  return (int)rep->flagged_tiles;
}

/* ------------------------------------------------------------------ */
/* Solves and iterative refinement.                                   */
/* ------------------------------------------------------------------ */
/* x := U^{-1} L^{-1} P b with LU factors from getrf (prec-emulated) */
static void lu_solve(int n, const double* LU, int lda, const int32_t* ipiv, double* x, int prec) {
  for (int i = 0; i < n; ++i) {
    int p = ipiv[i] - 1;
    if (p != i) { double t = x[i]; x[i] = x[p]; x[p] = t; }
  }
  for (int i = 0; i < n; ++i) {
    double s = x[i];
    for (int p = 0; p < i; ++p) s = rs(prec, s - AT(LU, i, p, lda) * x[p]);
    x[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int p = i + 1; p < n; ++p) s = rs(prec, s - AT(LU, i, p, lda) * x[p]);
    x[i] = rs(prec, s / AT(LU, i, i, lda));
  }
}

/* x := L^{-T} L^{-1} b with the Cholesky factor */
static void chol_solve(int n, const double* L, int lda, double* x, int prec) {
  for (int i = 0; i < n; ++i) {
    double s = x[i];
    for (int p = 0; p < i; ++p) s = rs(prec, s - AT(L, i, p, lda) * x[p]);
    x[i] = rs(prec, s / AT(L, i, i, lda));
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int p = i + 1; p < n; ++p) s = rs(prec, s - AT(L, p, i, lda) * x[p]);
    x[i] = rs(prec, s / AT(L, i, i, lda));
  }
}

void orc_getrs(int n, const double* LU, int lda, const int32_t* ipiv, double* x) { lu_solve(n, LU, lda, ipiv, x, PR64); }
void orc_potrs(int n, const double* L, int lda, double* x) { chol_solve(n, L, lda, x, PR64); }

typedef struct {
  int32_t iters, converged, failed_reason, pad; /* reason: 0 ok, 1 no contraction, 2 non-finite, 3 max iter, 4 factor info */
  double resid_norm, x_norm, a_norm, last_dx;
} orc_ir_report;

static double inf_norm_vec(int n, const double* x) {
  double m = 0.0;
  for (int i = 0; i < n; ++i) { double a = fabs(x[i]); if (!(a <= m)) m = a; }
  return m;
}
static double inf_norm_mat(int n, const double* A, int lda) {
  double m = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += fabs(AT(A, i, j, lda));
    if (s > m) m = s;
  }
  return m;
}

/* Mixed-precision solve with FP64 iterative refinement.  The factorization
   runs in binary32 with trailing-update operands rounded per `prec`; the
   residual r = b - A x and the update x += d are FP64; the correction solve
   uses the low-precision factors on r scaled by its infinity norm.
   Converged when ||d|| <= u ||x|| or ||r|| <= u ||A|| ||x||; failed on a
   non-finite value, on ||d_i|| > ||d_{i-1}||/2 (i >= 2) while still far from
   converged, or after max_iter corrections. */
int orc_gesv_mp(int n, int nb, const double* A, int lda, const double* b, double* x, int prec, int chol,
                int max_iter, orc_ir_report* ir) {
  memset(ir, 0, sizeof(*ir));
  double* F = malloc(sizeof(double) * (size_t)n * n);
  int32_t* ipiv = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i) F[i + (size_t)j * n] = AT(A, i, j, lda);
  orc_report rep;
  int info = chol ? orc_abft_potrf(n, nb, F, n, prec, 0, 4.0, NULL, 0, NULL, &rep)
                  : orc_abft_getrf(n, nb, F, n, ipiv, prec, 0, 4.0, NULL, 0, NULL, &rep);
  if (info) { ir->failed_reason = 4; free(F); free(ipiv); return info; }
  double u = ldexp(1.0, -53);
  double an = inf_norm_mat(n, A, lda);
  ir->a_norm = an;
  double* r = malloc(sizeof(double) * n);
  double* d = malloc(sizeof(double) * n);
  for (int i = 0; i < n; ++i) d[i] = rs(PR32, b[i]);
  if (chol) chol_solve(n, F, n, d, PR32); else lu_solve(n, F, n, ipiv, d, PR32);
  for (int i = 0; i < n; ++i) x[i] = d[i];
  double prev = INFINITY;
  int it;
  for (it = 1; it <= max_iter; ++it) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      double s = b[i];
      for (int j = 0; j < n; ++j) s -= AT(A, i, j, lda) * x[j];
      r[i] = s;
    }
    double rn = inf_norm_vec(n, r), xn = inf_norm_vec(n, x);
    ir->resid_norm = rn; ir->x_norm = xn;
    if (!isfinite(rn) || !isfinite(xn)) { ir->failed_reason = 2; break; }
    if (rn <= u * an * xn) { ir->converged = 1; break; }
    double sc = rn > 0 ? rn : 1.0;
    for (int i = 0; i < n; ++i) d[i] = rs(PR32, r[i] / sc);
    if (chol) chol_solve(n, F, n, d, PR32); else lu_solve(n, F, n, ipiv, d, PR32);
    for (int i = 0; i < n; ++i) d[i] *= sc;
    double dn = inf_norm_vec(n, d);
    ir->last_dx = dn;
    for (int i = 0; i < n; ++i) x[i] += d[i];
    ir->iters = it;
    if (!isfinite(dn)) { ir->failed_reason = 2; break; }
    if (dn <= u * inf_norm_vec(n, x)) { ir->converged = 1; break; }
    if (it >= 2 && dn > 0.5 * prev && dn > 1e3 * u * inf_norm_vec(n, x)) { ir->failed_reason = 1; break; }
    prev = dn;
  }
  if (!ir->converged && !ir->failed_reason) ir->failed_reason = 3;
  free(F); free(ipiv); free(r); free(d);
  return 0;
}

/* Reference solution of the stored system: FP64 LU + refinement whose
   residual is accumulated in double-double (error-free transformations of
   Knuth's two-sum and an FMA-based two-product). */
static inline void two_sum(double a, double b, double* s, double* e) {
  double x = a + b, bv = x - a, av = x - bv;
  *s = x;
  *e = (a - av) + (b - bv);
}
void orc_solve_ref(int n, const double* A, int lda, const double* b, double* x, int iters) {
  double* F = malloc(sizeof(double) * (size_t)n * n);
  int32_t* ipiv = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i) F[i + (size_t)j * n] = AT(A, i, j, lda);
  orc_report rep;
  orc_abft_getrf(n, 64, F, n, ipiv, PR64, 0, 4.0, NULL, 0, NULL, &rep);
  for (int i = 0; i < n; ++i) x[i] = b[i];
  lu_solve(n, F, n, ipiv, x, PR64);
  double* r = malloc(sizeof(double) * n);
  for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      double hi = b[i], lo = 0.0;
      for (int j = 0; j < n; ++j) {
        double a = AT(A, i, j, lda), p = -a * x[j];
        double pe = fma(-a, x[j], -p);
        double s, e;
        two_sum(hi, p, &s, &e);
        hi = s;
        lo += e + pe;
      }
      r[i] = hi + lo;
    }
    lu_solve(n, F, n, ipiv, r, PR64);
    for (int i = 0; i < n; ++i) x[i] += r[i];
  }
  free(F); free(ipiv); free(r);
}
