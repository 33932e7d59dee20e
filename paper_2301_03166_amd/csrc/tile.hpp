// Per-tile checksum sums, comparison and locate/correct (device functions
// shared by the per-iteration kernels and the batched factorizations).
#pragma once
#include "common.hpp"

namespace abft {

constexpr int MAXNB = 512;
constexpr int QROWS = MAXNB / 64;

template <typename T>
__device__ __forceinline__ double ld(const T* p) {
  return (double)*p;
}

// LDS scratch of one tile's sums (40 KB)
struct TileSums {
  double ce[MAXNB], cw[MAXNB], ca[MAXNB], cwa[MAXNB];
  double res[MAXNB], rec[MAXNB], rws[MAXNB], rwc[MAXNB], ra[MAXNB], rwa[MAXNB];
};

// All column and row sums of tile (r0, c0, h x w); in the symmetric view an
// element above the diagonal is read from its mirror below it.  Waves take
// columns round-robin and lanes walk the rows (coalesced); each lane keeps
// its rows' partial row sums, merged across waves in a fixed order.
template <typename T>
__device__ void tile_sums(const T* A, int64_t lda, int64_t r0, int64_t c0, int h, int w, bool sym, TileSums& ts) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  acc2 pe[QROWS], pw[QROWS];
  double pa[QROWS], pwa[QROWS];
#pragma unroll
  for (int q = 0; q < QROWS; ++q) { pe[q] = {0, 0}; pw[q] = {0, 0}; pa[q] = 0; pwa[q] = 0; }
  for (int j = wv; j < w; j += 4) {
    acc2 se{0, 0}, sw{0, 0};
    double sa = 0, swa = 0;
    const double wj = (double)(j + 1);
    double vq[QROWS];
    // all loads of the column first (QROWS independent requests in flight)
#pragma unroll
    for (int q = 0; q < QROWS; ++q) {
      int i = lane + 64 * q;
      vq[q] = 0.0;
      if (i < h) vq[q] = (sym && i < j) ? ld(A + (r0 + j) + (c0 + i) * lda) : ld(A + (r0 + i) + (c0 + j) * lda);
    }
#pragma unroll
    for (int q = 0; q < QROWS; ++q) {
      int i = lane + 64 * q;
      if (i < h) {
        const double v = vq[q];
        double wi = (double)(i + 1), av = fabs(v);
        cadd(se, v);
        cfma(sw, wi, v);
        sa += av;
        swa += wi * av;
        cadd(pe[q], v);
        cfma(pw[q], wj, v);
        pa[q] += av;
        pwa[q] += wj * av;
      }
    }
    se = wave_csum(se);
    sw = wave_csum(sw);
    sa = wave_sum(sa);
    swa = wave_sum(swa);
    if (lane == 0) {
      ts.ce[j] = cval(se);
      ts.cw[j] = cval(sw);
      ts.ca[j] = sa;
      ts.cwa[j] = swa;
    }
  }
  for (int s = 0; s < 4; ++s) {
    if (wv == s) {
#pragma unroll
      for (int q = 0; q < QROWS; ++q) {
        int i = lane + 64 * q;
        if (i < h) {
          if (s == 0) {
            ts.res[i] = pe[q].s; ts.rec[i] = pe[q].c;
            ts.rws[i] = pw[q].s; ts.rwc[i] = pw[q].c;
            ts.ra[i] = pa[q]; ts.rwa[i] = pwa[q];
          } else {
            acc2 e{ts.res[i], ts.rec[i]}, ww{ts.rws[i], ts.rwc[i]};
            cmerge(e, pe[q]);
            cmerge(ww, pw[q]);
            ts.res[i] = e.s; ts.rec[i] = e.c;
            ts.rws[i] = ww.s; ts.rwc[i] = ww.c;
            ts.ra[i] += pa[q]; ts.rwa[i] += pwa[q];
          }
        }
      }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < h; i += blockDim.x) {
    ts.res[i] = ts.res[i] + ts.rec[i];
    ts.rws[i] = ts.rws[i] + ts.rwc[i];
  }
  __syncthreads();
}

__device__ __forceinline__ void tile_geom(int bid, int I0, int J0, int nI, int nb, int64_t nr, int64_t nc, int& I,
                                          int& J, int& h, int& w) {
  I = I0 + bid % nI;
  J = J0 + bid / nI;
  h = (int)min((int64_t)nb, nr - (int64_t)I * nb);
  w = (int)min((int64_t)nb, nc - (int64_t)J * nb);
}

// write the sums of a tile into the checksum arrays
__device__ void store_sums(const TileSums& ts, int I, int J, int nb, int h, int w, double* colchk, int64_t ldc,
                           double* rowchk, int64_t ldr) {
  int64_t r0 = (int64_t)I * nb, c0 = (int64_t)J * nb;
  for (int j = threadIdx.x; j < w; j += blockDim.x) {
    colchk[2 * I + (c0 + j) * ldc] = ts.ce[j];
    colchk[2 * I + 1 + (c0 + j) * ldc] = ts.cw[j];
  }
  for (int i = threadIdx.x; i < h; i += blockDim.x) {
    rowchk[(r0 + i) + (2 * J) * ldr] = ts.res[i];
    rowchk[(r0 + i) + (2 * J + 1) * ldr] = ts.rws[i];
  }
}

// flags of every column / row of a tile against the carried checksums
struct TileFlags {
  double de[MAXNB], dw[MAXNB], he[MAXNB], hw[MAXNB];
  unsigned char fe[MAXNB], fw[MAXNB], ge[MAXNB], gw[MAXNB];
  int nflag;
  double maxr;
};

// A rebuilt element (tile-relative sci, scj) is known only to the tolerance
// tec of the column checksum it was rebuilt from; after a correction every
// sum containing it (twice in the symmetric view of a diagonal tile: the
// element and its mirror) may differ by its weight in that sum times tec.
__device__ __forceinline__ double slack_w(int line, int a, int b, bool sdiag, double tec) {
  if (line == b) return (a + 1) * tec;
  if (sdiag && line == a) return (b + 1) * tec;
  return 0.0;
}

// sci < 0: plain comparison; otherwise widen the sums that hold element
// (sci, scj) as described above.  level 1 (column checksums only) leaves the
// row side out.  line 1 / 2: row / column lidx of the tile was rebuilt from
// the checksums of the other side; every rebuilt element is known to the
// tolerance of the checksum it came from (column j: te_j, row i: te_i), so
// each sum through it is widened by its weight there times that tolerance,
// and the rebuilt line's own sums by lsum = sum of them (lwsum: weighted).
__device__ void tile_compare(const TileSums& ts, TileFlags& tf, int I, int J, int nb, int h, int w,
                             const double* colchk, int64_t ldc, const double* rowchk, int64_t ldr, const double* gc,
                             const double* gr, double tsu, int sci = -1, int scj = -1, bool sdiag = false,
                             int level = 2, int line = 0, int lidx = -1, double lsum = 0.0, double lwsum = 0.0) {
  int64_t r0 = (int64_t)I * nb, c0 = (int64_t)J * nb;
  if (threadIdx.x == 0) { tf.nflag = 0; tf.maxr = 0.0; }
  __syncthreads();
  const double tec =
      sci >= 0 ? tau_verify(tsu, ts.ca[scj], gc ? gc[2 * I + (c0 + scj) * ldc] : 0.0) : 0.0;
  int nfl = 0;
  double mr = 0.0;
  for (int j = threadIdx.x; j < w; j += blockDim.x) {
    int64_t o = 2 * I + (c0 + j) * ldc;
    double de = ts.ce[j] - colchk[o], dw = ts.cw[j] - colchk[o + 1];
    double te = tau_verify(tsu, ts.ca[j], gc ? gc[o] : 0.0), tw = tau_verify(tsu, ts.cwa[j], gc ? gc[o + 1] : 0.0);
    if (sci >= 0) {
      const double sw = slack_w(j, sci, scj, sdiag, tec);
      if (sw > 0.0) { te += tec; tw += sw; }
    }
    if (line == 1) {  // this column's element in row lidx came from this column's checksum
      const double tl = tau_verify(tsu, ts.ca[j], gc ? gc[o] : 0.0);
      te += tl;
      tw += (double)(lidx + 1) * tl;
    } else if (line == 2 && j == lidx) {
      te += lsum;
      tw += lwsum;
    }
    bool be = bad(de, te), bw = bad(dw, tw);
    tf.de[j] = de; tf.dw[j] = dw; tf.fe[j] = be; tf.fw[j] = bw;
    nfl += be + bw;
    if (!be && te > 0) mr = fmax(mr, fabs(de) / te);
    if (!bw && tw > 0) mr = fmax(mr, fabs(dw) / tw);
  }
  for (int i = threadIdx.x; i < h; i += blockDim.x) {
    if (level == 1) {  // single side: the row checksums are not compared
      tf.he[i] = tf.hw[i] = 0.0;
      tf.ge[i] = tf.gw[i] = 0;
      continue;
    }
    int64_t o = (r0 + i) + (2 * J) * ldr;
    double de = ts.res[i] - rowchk[o], dw = ts.rws[i] - rowchk[o + ldr];
    double te = tau_verify(tsu, ts.ra[i], gr ? gr[o] : 0.0), tw = tau_verify(tsu, ts.rwa[i], gr ? gr[o + ldr] : 0.0);
    if (sci >= 0) {
      const double sw = slack_w(i, scj, sci, sdiag, tec);
      if (sw > 0.0) { te += tec; tw += sw; }
    }
    if (line == 2) {  // this row's element in column lidx came from this row's checksum
      const double tl = tau_verify(tsu, ts.ra[i], gr ? gr[o] : 0.0);
      te += tl;
      tw += (double)(lidx + 1) * tl;
    } else if (line == 1 && i == lidx) {
      te += lsum;
      tw += lwsum;
    }
    bool be = bad(de, te), bw = bad(dw, tw);
    tf.he[i] = de; tf.hw[i] = dw; tf.ge[i] = be; tf.gw[i] = bw;
    nfl += be + bw;
    if (!be && te > 0) mr = fmax(mr, fabs(de) / te);
    if (!bw && tw > 0) mr = fmax(mr, fabs(dw) / tw);
  }
  if (nfl) atomicAdd(&tf.nflag, nfl);
  // max over the workgroup: wave max then one LDS atomic per wave (order-free)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mr = fmax(mr, __shfl_xor(mr, o));
  if ((threadIdx.x & 63) == 0 && mr > 0)
    atomicMax(reinterpret_cast<unsigned long long*>(&tf.maxr), (unsigned long long)__double_as_longlong(mr));
  __syncthreads();
}

// whether the weighted / plain difference ratio exists (it does not when a
// difference is not finite or the weighted one overflowed)
__device__ __forceinline__ bool ratio_finite(double dw, double de) {
  return de != 0.0 && fabs(dw / de) <= 1.79e308;
}
__device__ __forceinline__ int ratio_index(double dw, double de, int len) {
  if (!(de != 0.0)) return -1;
  double r = dw / de;
  if (!(fabs(r) <= 1.79e308)) return -1;
  double k = floor(r + 0.5);
  if (fabs(r - k) > 0.25) return -1;
  if (k < 1.0 || k > (double)len) return -1;
  return (int)k - 1;
}

// Locate and correct one flagged tile (one fault per tile per iteration).
// Decision rules: intersection of a single flagged column and row; a single
// flagged line located by the ratio of its weighted and plain differences; a
// lone weighted-checksum mismatch is a checksum error; anything else is
// uncorrectable.  The element is recomputed from its column checksum with
// itself left out, so huge, Inf or NaN values are repaired too.  Every
// outcome ends with the tile's checksums re-encoded from the data.
struct CorrState {
  int ci, cj, kind;  // kind: 0 clean, 1 element, 2 checksum repair, 3 uncorrectable, 5 / 6 row / column rebuilt
  int lidx;          // the rebuilt row (kind 5) or column (kind 6)
  double old, lsum, lwsum;
  double part[4][2];     // per-wave partial sums of the rebuilt line's tolerances
  double oldv[MAXNB];    // the rebuilt line's previous values
};

// A 1D error (one row or one column of the tile wrong in several places,
// as an error in an operand of the update leaves it) with full checksums:
// the row (column) is rebuilt element by element from the checksums of the
// other side, each element from its own column (row) with the rest of that
// column (row) left out; the tile is then rechecked with the rebuilt
// elements' tolerances (tile_compare, line 1 / 2) and the old values come
// back when the recheck fails.  Returns through cs.kind (3 on failure).
template <typename T>
__device__ void rebuild_line_dev(T* A, int64_t lda, int I, int J, int nb, int h, int w, const double* colchk,
                                 int64_t ldc, const double* rowchk, int64_t ldr, const double* gc, const double* gr,
                                 double tsu, TileSums& ts, TileFlags& tf, CorrState& cs) {
  const int64_t r0 = (int64_t)I * nb, c0 = (int64_t)J * nb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int line = cs.kind == 5 ? 1 : 2, idx = cs.lidx;
  if (line == 1) {  // row idx: one column per wave
    for (int j = wv; j < w; j += 4) {
      acc2 sacc{0, 0};
      for (int i = lane; i < h; i += 64)
        if (i != idx) cadd(sacc, (double)A[(r0 + i) + (c0 + j) * lda]);
      sacc = wave_csum(sacc);
      if (lane == 0) {
        T* p = A + (r0 + idx) + (c0 + j) * lda;
        cs.oldv[j] = (double)*p;
        *p = (T)(colchk[2 * I + (c0 + j) * ldc] - cval(sacc));
      }
    }
  } else {  // column idx: one row per wave
    for (int i = wv; i < h; i += 4) {
      acc2 sacc{0, 0};
      for (int j = lane; j < w; j += 64)
        if (j != idx) cadd(sacc, (double)A[(r0 + i) + (c0 + j) * lda]);
      sacc = wave_csum(sacc);
      if (lane == 0) {
        T* p = A + (r0 + i) + (c0 + idx) * lda;
        cs.oldv[i] = (double)*p;
        *p = (T)(rowchk[(r0 + i) + (2 * J) * ldr] - cval(sacc));
      }
    }
  }
  __syncthreads();
  tile_sums(A, lda, r0, c0, h, w, false, ts);
  // the rebuilt line's own sums hold every rebuilt element once
  double p0 = 0.0, p1 = 0.0;
  if (line == 1) {
    for (int j = threadIdx.x; j < w; j += blockDim.x) {
      const double tl = tau_verify(tsu, ts.ca[j], gc ? gc[2 * I + (c0 + j) * ldc] : 0.0);
      p0 += tl;
      p1 += (double)(j + 1) * tl;
    }
  } else {
    for (int i = threadIdx.x; i < h; i += blockDim.x) {
      const double tl = tau_verify(tsu, ts.ra[i], gr ? gr[(r0 + i) + (2 * J) * ldr] : 0.0);
      p0 += tl;
      p1 += (double)(i + 1) * tl;
    }
  }
  p0 = wave_sum(p0);
  p1 = wave_sum(p1);
  if (lane == 0) {
    cs.part[wv][0] = p0;
    cs.part[wv][1] = p1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    cs.lsum = ((cs.part[0][0] + cs.part[1][0]) + cs.part[2][0]) + cs.part[3][0];
    cs.lwsum = ((cs.part[0][1] + cs.part[1][1]) + cs.part[2][1]) + cs.part[3][1];
  }
  __syncthreads();
  tile_compare(ts, tf, I, J, nb, h, w, colchk, ldc, rowchk, ldr, gc, gr, tsu, -1, -1, false, 2, line, idx, cs.lsum,
               cs.lwsum);
  if (tf.nflag != 0) {
    if (line == 1) {
      for (int j = threadIdx.x; j < w; j += blockDim.x) A[(r0 + idx) + (c0 + j) * lda] = (T)cs.oldv[j];
    } else {
      for (int i = threadIdx.x; i < h; i += blockDim.x) A[(r0 + i) + (c0 + idx) * lda] = (T)cs.oldv[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) cs.kind = 3;
  }
  __syncthreads();
}

// level: 2 full checksums (0D and 1D rules), 1 column checksums only (0D)
template <typename T>
__device__ void correct_tile_dev(T* A, int64_t lda, int I, int J, int nb, int h, int w, bool diag, double* colchk,
                                 int64_t ldc, double* rowchk, int64_t ldr, const double* gc, const double* gr,
                                 double tsu, abft_report* rep, int iter, TileSums& ts, TileFlags& tf, CorrState& cs,
                                 int level = 2) {
  const int64_t r0 = (int64_t)I * nb, c0 = (int64_t)J * nb;
  tile_sums(A, lda, r0, c0, h, w, diag, ts);
  tile_compare(ts, tf, I, J, nb, h, w, colchk, ldc, rowchk, ldr, gc, gr, tsu, -1, -1, false, level);
  if (threadIdx.x == 0) {
    int nFe = 0, nGe = 0, nFw = 0, nGw = 0, jf0 = -1, jf1 = -1, ig = -1;
    for (int j = 0; j < w; ++j) {
      if (tf.fe[j]) {
        if (nFe == 0) jf0 = j; else if (nFe == 1) jf1 = j;
        nFe++;
      }
      nFw += tf.fw[j];
    }
    for (int i = 0; i < h; ++i) {
      if (tf.ge[i]) { ig = i; nGe++; }
      nGw += tf.gw[i];
    }
    int ci = -1, cj = -1, repair = 0, line = 0;
    if (tf.nflag == 0) {
      repair = -1;
    } else if (diag) {
      // symmetric view: an off-diagonal element shows in two columns (itself
      // and its mirror), a diagonal one in one.  Two flagged columns name the
      // element by the pattern (the recheck rejects any other cause); one
      // flagged column: the ratio names the row (the element or its mirror),
      // and where it does not exist (non-finite value, overflowed weighted
      // sum) it is the diagonal element
      if (nFe == 1) {
        const int i = ratio_index(tf.dw[jf0], tf.de[jf0], h);
        if (i >= 0) {
          ci = i > jf0 ? i : jf0;
          cj = i > jf0 ? jf0 : i;
        } else if (!ratio_finite(tf.dw[jf0], tf.de[jf0])) {
          ci = cj = jf0;
        } else if (nGe == 0 && !tf.fw[jf0]) {
          repair = 1;  // a flipped e entry of the column checksums
        }
      } else if (nFe == 2) {
        ci = jf1;
        cj = jf0;
      } else if (nFe == 0) {
        repair = 1;
      }
    } else {
      // a checksum entry is taken for wrong only when its data side is
      // consistent: a plain difference with an unflagged weighted one (a
      // flipped e entry), or weighted differences alone
      if (nFe == 1 && nGe == 1) {
        ci = ig; cj = jf0;
      } else if (nFe == 1 && nGe == 0) {
        int i = ratio_index(tf.dw[jf0], tf.de[jf0], h);
        if (i >= 0) { ci = i; cj = jf0; } else if (nGw == 0 && !tf.fw[jf0]) repair = 1;
      } else if (nFe == 0 && nGe == 1) {
        int j = ratio_index(tf.hw[ig], tf.he[ig], w);
        if (j >= 0) { ci = ig; cj = j; } else if (nFw == 0 && !tf.gw[ig]) repair = 1;
      } else if (nFe == 0 && nGe == 0) {
        repair = 1;
      } else if (level == 2 && nGe == 1 && nFe >= 2) {
        line = 1;  // one row wrong in several columns
      } else if (level == 2 && nFe == 1 && nGe >= 2) {
        line = 2;  // one column wrong in several rows
      }
    }
    cs.ci = ci;
    cs.cj = cj;
    cs.lidx = line == 1 ? ig : jf0;
    cs.kind = (repair == -1) ? 0 : (ci >= 0 ? 1 : (line ? 4 + line : (repair ? 2 : 3)));
  }
  __syncthreads();
  if (cs.kind == 5 || cs.kind == 6)
    rebuild_line_dev(A, lda, I, J, nb, h, w, colchk, ldc, rowchk, ldr, gc, gr, tsu, ts, tf, cs);
  if (cs.kind == 1) {
    const int ci = cs.ci, cj = cs.cj;
    if (threadIdx.x < 64) {
      acc2 sacc{0, 0};
      for (int i = threadIdx.x; i < h; i += 64) {
        if (i == ci) continue;
        double v = (diag && i < cj) ? (double)A[(r0 + cj) + (c0 + i) * lda] : (double)A[(r0 + i) + (c0 + cj) * lda];
        cadd(sacc, v);
      }
      sacc = wave_csum(sacc);
      if (threadIdx.x == 0) {
        double val = colchk[2 * I + (c0 + cj) * ldc] - cval(sacc);
        T* p = A + (r0 + ci) + (c0 + cj) * lda;
        cs.old = (double)*p;
        *p = (T)val;
      }
    }
    __syncthreads();
    tile_sums(A, lda, r0, c0, h, w, diag, ts);
    tile_compare(ts, tf, I, J, nb, h, w, colchk, ldc, rowchk, ldr, gc, gr, tsu, ci, cj, diag, level);
    if (tf.nflag != 0) {
      if (threadIdx.x == 0) {
        A[(r0 + ci) + (c0 + cj) * lda] = (T)cs.old;
        cs.kind = 3;
      }
      __syncthreads();
    }
  }
  if (cs.kind == 0) return;
  tile_sums(A, lda, r0, c0, h, w, diag, ts);
  store_sums(ts, I, J, nb, h, w, colchk, ldc, rowchk, ldr);
  if (threadIdx.x == 0 && rep) {
    if (cs.kind == 1) {
      atomicAdd((unsigned long long*)&rep->corrected, 1ull);
      atomicOr(&rep->status, (int)ABFT_ST_CORRECTED);
      rep_event(rep, iter, 1, r0 + cs.ci, c0 + cs.cj);
    } else if (cs.kind == 5 || cs.kind == 6) {
      atomicAdd((unsigned long long*)&rep->corrected, 1ull);
      atomicOr(&rep->status, (int)ABFT_ST_CORRECTED);
      if (cs.kind == 5) rep_event(rep, iter, 5, r0 + cs.lidx, c0);
      else rep_event(rep, iter, 6, r0, c0 + cs.lidx);
    } else if (cs.kind == 2) {
      atomicAdd((unsigned long long*)&rep->checksum_repaired, 1ull);
      atomicOr(&rep->status, (int)ABFT_ST_REPAIRED);
      rep_event(rep, iter, 2, r0, c0);
    } else {
      atomicAdd((unsigned long long*)&rep->uncorrectable, 1ull);
      atomicOr(&rep->status, (int)ABFT_ST_UNCORRECTABLE);
      rep_event(rep, iter, 3, r0, c0);
    }
  }
  __syncthreads();
}

}  // namespace abft
