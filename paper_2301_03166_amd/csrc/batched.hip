// Batched ABFT-protected Cholesky and LU of many small matrices of uneven
// orders (n <= 512) in ONE persistent kernel.
//
// Every workgroup repeatedly takes the next matrix from a largest-first
// queue (the host-visible order is sorted on the device) and factors it
// completely: for each 32-wide block step the panel lives in LDS (pivot
// search, interchanges, scaling and the rank-1 updates, or the diagonal
// Cholesky and the row solves), the panel update and the trailing update run
// from LDS-staged operands with 4x4 register tiles per thread, the per-tile
// checksums of the trailing matrix are carried through the update, and the
// trailing tiles are verified and, if flagged, located and corrected --
// exactly the per-iteration protocol of the large factorizations, with one
// detection interval per block step.  The queue order depends on the
// scheduling, the arithmetic of each matrix does not.
#include "common.hpp"
#include "kernels.hpp"
#include "tile.hpp"

namespace abft {

constexpr int BNB = 32;        // block size = checksum tile size of the batched path
constexpr int BMAX = 512;      // largest matrix order
constexpr int BN = BMAX / BNB; // largest number of tile rows

struct BatchChk {  // per-matrix checksum workspace (fixed stride)
  double *colchk, *rowchk, *gc, *gr, *S, *Sa, *Tm, *Ta;
};
__host__ __device__ constexpr size_t batch_chk_doubles() {
  return (size_t)4 * 2 * BN * BMAX + (size_t)4 * 2 * BN * BNB;
}
__device__ BatchChk chk_of(double* base, int mi) {
  BatchChk c;
  double* p = base + (size_t)mi * batch_chk_doubles();
  c.colchk = p; p += 2 * BN * BMAX;
  c.rowchk = p; p += 2 * BN * BMAX;
  c.gc = p; p += 2 * BN * BMAX;
  c.gr = p; p += 2 * BN * BMAX;
  c.S = p; p += 2 * BN * BNB;
  c.Sa = p; p += 2 * BN * BNB;
  c.Tm = p; p += 2 * BN * BNB;
  c.Ta = p;
  return c;
}

// largest-first order of the matrices (bitonic sort of (n, index) in LDS)
__global__ void k_batch_order(const int32_t* dn, int batch, int* order, unsigned* queue) {
  __shared__ int key[8192];
  __shared__ int idx[8192];
  int P = 1;
  while (P < batch) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    key[i] = i < batch ? dn[i] : -1;
    idx[i] = i;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        int l = i ^ j;
        if (l > i) {
          // descending by n, ascending by index on ties
          bool desc = (i & k) == 0;
          bool gt = key[i] < key[l] || (key[i] == key[l] && idx[i] > idx[l]);
          if (gt == desc) {
            int t = key[i]; key[i] = key[l]; key[l] = t;
            t = idx[i]; idx[i] = idx[l]; idx[l] = t;
          }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < batch; i += blockDim.x) order[i] = idx[i];
  if (threadIdx.x == 0) *queue = 0u;
}

template <typename T>
__device__ __forceinline__ T fms_b(T a, T b, T c) {
  return a - b * c;
}
template <>
__device__ __forceinline__ float fms_b<float>(float a, float b, float c) {
  return __fmaf_rn(-b, c, a);
}

// checksum carry of the batched trailing update  A22 -= X Y  over tile-rows
// and tile-columns > k: X rows (i >= c1) from the LDS panel P (row i - c0),
// Y(p, j) from ymat (LU: U12 in A; Cholesky: the transpose of X).
template <typename T, int CHOL>
__device__ void batch_carry(const T* A, int64_t lda, int n, int k, int w, const T* P, int ldp, const BatchChk& c) {
  const int N = (n + BNB - 1) / BNB;
  const int c0 = k * BNB, c1 = c0 + w;
  const int ldc = 2 * BN;
  // S: sums of X over each tile-row I > k (compensated); Sa: |.|-sums
  for (int e = threadIdx.x; e < (N - k - 1) * w; e += blockDim.x) {
    int I = k + 1 + e / w, p = e % w;
    acc2 se{0, 0}, sw{0, 0};
    double sa = 0, swa = 0;
    for (int i = I * BNB; i < min(n, (I + 1) * BNB); ++i) {
      double v = (double)P[(i - c0) * ldp + p], wi = (double)(i - I * BNB + 1);
      cadd(se, v);
      cfma(sw, wi, v);
      sa += fabs(v);
      swa += wi * fabs(v);
    }
    c.S[2 * I + p * ldc] = cval(se);
    c.S[2 * I + 1 + p * ldc] = cval(sw);
    c.Sa[2 * I + p * ldc] = sa;
    c.Sa[2 * I + 1 + p * ldc] = swa;
  }
  if (!CHOL) {
    // Tm: row sums of U12 over each tile-column J > k
    for (int e = threadIdx.x; e < (N - k - 1) * w; e += blockDim.x) {
      int J = k + 1 + e / w, p = e % w;
      acc2 se{0, 0}, sw{0, 0};
      double sa = 0, swa = 0;
      for (int j = J * BNB; j < min(n, (J + 1) * BNB); ++j) {
        double v = (double)A[(c0 + p) + (int64_t)j * lda], wj = (double)(j - J * BNB + 1);
        cadd(se, v);
        cfma(sw, wj, v);
        sa += fabs(v);
        swa += wj * fabs(v);
      }
      c.Tm[p + (2 * J) * BNB] = cval(se);
      c.Tm[p + (2 * J + 1) * BNB] = cval(sw);
      c.Ta[p + (2 * J) * BNB] = sa;
      c.Ta[p + (2 * J + 1) * BNB] = swa;
    }
  }
  __syncthreads();
  // column side: colchk(2I+e, j) -= S(2I+e, :) y(:, j);  gc = Sa |y|
  for (int e = threadIdx.x; e < (n - c1) * (N - k - 1); e += blockDim.x) {
    int j = c1 + e % (n - c1), I = k + 1 + e / (n - c1);
    if (CHOL && I < j / BNB) continue;
    acc2 ue{c.colchk[2 * I + (int64_t)j * ldc], 0}, uw{c.colchk[2 * I + 1 + (int64_t)j * ldc], 0};
    double ga = 0, gwa = 0;
    for (int p = 0; p < w; ++p) {
      double y = CHOL ? (double)P[(j - c0) * ldp + p] : (double)A[(c0 + p) + (int64_t)j * lda];
      cfma(ue, -c.S[2 * I + p * ldc], y);
      cfma(uw, -c.S[2 * I + 1 + p * ldc], y);
      ga += c.Sa[2 * I + p * ldc] * fabs(y);
      gwa += c.Sa[2 * I + 1 + p * ldc] * fabs(y);
    }
    c.colchk[2 * I + (int64_t)j * ldc] = cval(ue);
    c.colchk[2 * I + 1 + (int64_t)j * ldc] = cval(uw);
    c.gc[2 * I + (int64_t)j * ldc] = ga;
    c.gc[2 * I + 1 + (int64_t)j * ldc] = gwa;
  }
  // row side: rowchk(i, 2J+e) -= x(i, :) t(:, 2J+e);  gr = |x| t_abs
  for (int e = threadIdx.x; e < (n - c1) * (N - k - 1); e += blockDim.x) {
    int i = c1 + e % (n - c1), J = k + 1 + e / (n - c1);
    if (CHOL && i / BNB < J) continue;
    acc2 ue{c.rowchk[i + (int64_t)(2 * J) * BMAX], 0}, uw{c.rowchk[i + (int64_t)(2 * J + 1) * BMAX], 0};
    double ga = 0, gwa = 0;
    for (int p = 0; p < w; ++p) {
      double x = (double)P[(i - c0) * ldp + p];
      double te = CHOL ? c.S[2 * J + p * ldc] : c.Tm[p + (2 * J) * BNB];
      double tw = CHOL ? c.S[2 * J + 1 + p * ldc] : c.Tm[p + (2 * J + 1) * BNB];
      double ta = CHOL ? c.Sa[2 * J + p * ldc] : c.Ta[p + (2 * J) * BNB];
      double twa = CHOL ? c.Sa[2 * J + 1 + p * ldc] : c.Ta[p + (2 * J + 1) * BNB];
      cfma(ue, -x, te);
      cfma(uw, -x, tw);
      ga += fabs(x) * ta;
      gwa += fabs(x) * twa;
    }
    c.rowchk[i + (int64_t)(2 * J) * BMAX] = cval(ue);
    c.rowchk[i + (int64_t)(2 * J + 1) * BMAX] = cval(uw);
    c.gr[i + (int64_t)(2 * J) * BMAX] = ga;
    c.gr[i + (int64_t)(2 * J + 1) * BMAX] = gwa;
  }
  __syncthreads();
}

// trailing update A[c1:n, c1:n] -= X Y, X = rows of the LDS panel below the
// diagonal block, Y = U12 (staged chunk by chunk) or X^T (Cholesky, lower
// part only).  16 x 16 threads, each with a 4 x 4 register tile of a 64 x 64
// output block.
template <typename T, int CHOL>
__device__ void batch_tmu(T* A, int64_t lda, int n, int c0, int w, const T* P, int ldp, T* Uc) {
  const int c1 = c0 + w, m = n - c1;
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  for (int jb = 0; jb < m; jb += 64) {
    const int jn = min(64, m - jb);
    if (!CHOL) {
      __syncthreads();
      for (int e = threadIdx.x; e < w * 64; e += blockDim.x) {
        int p = e % w, jj = e / w;
        Uc[p * 65 + jj] = jj < jn ? A[(c0 + p) + (int64_t)(c1 + jb + jj) * lda] : (T)0;
      }
      __syncthreads();
    }
    for (int ib = CHOL ? jb : 0; ib < m; ib += 64) {
      T acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (T)0;
      for (int p = 0; p < w; ++p) {
        T xa[4], yb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          int i = ib + tr + 16 * a;
          xa[a] = i < m ? P[(w + i) * ldp + p] : (T)0;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          int jj = tc + 16 * b;
          if (CHOL) yb[b] = (jb + jj < m) ? P[(w + jb + jj) * ldp + p] : (T)0;
          else yb[b] = Uc[p * 65 + jj];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = acc[a][b] + xa[a] * yb[b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          int i = ib + tr + 16 * a, jj = jb + tc + 16 * b;
          if (i < m && jj < m && (!CHOL || i >= jj)) {
            T* q = A + (c1 + i) + (int64_t)(c1 + jj) * lda;
            *q = *q - acc[a][b];
          }
        }
    }
  }
  __syncthreads();
}

template <typename T, int CHOL>
__device__ void factor_one(int mi, int n, T* A, int64_t lda, int32_t* ipiv, BatchChk c, int protect, double tsu,
                           const abft_fault* faults, int nfaults, int32_t* info, abft_report* rep,
                           unsigned char* smem) {
  const int tid = threadIdx.x;
  const int N = (n + BNB - 1) / BNB;
  const int ldc = 2 * BN;
  T* P = reinterpret_cast<T*>(smem);  // panel: (n - c0) x ldp
  const int ldp = BNB + 1;
  T* Uc = P + (size_t)BMAX * ldp;                                  // U12 chunk: BNB x 65
  TileSums& ts = *reinterpret_cast<TileSums*>(smem);              // verify phase (reuses the panel space)
  TileFlags& tf = *reinterpret_cast<TileFlags*>(smem + sizeof(TileSums));
  __shared__ CorrState cs;
  __shared__ int swp[BNB];
  __shared__ double wv_val[4];
  __shared__ int wv_idx[4];
  __shared__ int s_fail;
  if (tid == 0) {
    rep->flagged_tiles = rep->corrected = rep->checksum_repaired = rep->uncorrectable = rep->panel_flags = 0;
    rep->first_flag_iter = 0x7fffffff;
    rep->status = 0;
    rep->max_ratio = 0.0;
    rep->nev = 0;
    *info = 0;
    s_fail = 0;
  }
  __syncthreads();
  if (protect) {
    for (int J = 0; J < N; ++J)
      for (int I = CHOL ? J : 0; I < N; ++I) {
        int h = min(BNB, n - I * BNB), w = min(BNB, n - J * BNB);
        tile_sums(A, lda, (int64_t)I * BNB, (int64_t)J * BNB, h, w, CHOL && I == J, ts);
        store_sums(ts, I, J, BNB, h, w, c.colchk, ldc, c.rowchk, BMAX);
        __syncthreads();
      }
  }
  for (int k = 0; k < N; ++k) {
    const int c0 = k * BNB, w = min(BNB, n - c0), c1 = c0 + w, mrows = n - c0;
    // ---- panel into LDS
    for (int e = tid; e < mrows * w; e += blockDim.x) {
      int i = e % mrows, j = e / mrows;
      P[i * ldp + j] = A[(c0 + i) + (int64_t)(c0 + j) * lda];
    }
    __syncthreads();
    if (CHOL) {
      // diagonal block, right-looking
      for (int j = 0; j < w; ++j) {
        if (tid == 0) {
          T d = P[j * ldp + j];
          if (!(d > (T)0) && !s_fail) {
            s_fail = 1;
            *info = c0 + j + 1;
          }
          P[j * ldp + j] = sqrt(d);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < w; i += blockDim.x) P[i * ldp + j] = P[i * ldp + j] / P[j * ldp + j];
        __syncthreads();
        const int r = w - j - 1;
        for (int e = tid; e < r * r; e += blockDim.x) {
          int i = j + 1 + e % r, jj = j + 1 + e / r;
          if (i >= jj) P[i * ldp + jj] = fms_b(P[i * ldp + jj], P[i * ldp + j], P[jj * ldp + j]);
        }
        __syncthreads();
      }
      // rows below: x L^T = a, one thread per row
      for (int i = w + tid; i < mrows; i += blockDim.x)
        for (int j = 0; j < w; ++j) {
          T sacc = P[i * ldp + j];
          for (int p = 0; p < j; ++p) sacc = fms_b(sacc, P[i * ldp + p], P[j * ldp + p]);
          P[i * ldp + j] = sacc / P[j * ldp + j];
        }
      __syncthreads();
    } else {
      for (int j = 0; j < w; ++j) {
        double bv = -1.0;
        int bi = 0x7fffffff;
        for (int i = j + tid; i < mrows; i += blockDim.x) {
          double v = fabs((double)P[i * ldp + j]);
          if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          double ov = __shfl_xor(bv, o);
          int oi = __shfl_xor(bi, o);
          if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if ((tid & 63) == 0) { wv_val[tid >> 6] = bv; wv_idx[tid >> 6] = bi; }
        __syncthreads();
        if (tid == 0) {
          for (int q = 1; q < 4; ++q)
            if (wv_val[q] > bv || (wv_val[q] == bv && wv_idx[q] < bi)) { bv = wv_val[q]; bi = wv_idx[q]; }
          if (bi == 0x7fffffff) bi = j;
          swp[j] = bi;
          ipiv[c0 + j] = c0 + bi + 1;
        }
        __syncthreads();
        const int p = swp[j];
        if (p != j && tid < w) {
          T t = P[j * ldp + tid];
          P[j * ldp + tid] = P[p * ldp + tid];
          P[p * ldp + tid] = t;
        }
        __syncthreads();
        const T piv = P[j * ldp + j];
        if (piv == (T)0) {
          if (tid == 0 && !s_fail) { s_fail = 1; *info = c0 + j + 1; }
        } else {
          for (int i = j + 1 + tid; i < mrows; i += blockDim.x) {
            T l = P[i * ldp + j] / piv;
            P[i * ldp + j] = l;
            for (int cc = j + 1; cc < w; ++cc) P[i * ldp + cc] = fms_b(P[i * ldp + cc], l, P[j * ldp + cc]);
          }
        }
        __syncthreads();
      }
    }
    // ---- panel back to memory
    for (int e = tid; e < mrows * w; e += blockDim.x) {
      int i = e % mrows, j = e / mrows;
      if (!CHOL || i >= j) A[(c0 + i) + (int64_t)(c0 + j) * lda] = P[i * ldp + j];
    }
    __syncthreads();
    if (!CHOL) {
      // interchanges outside the panel, one at a time (checksums follow the rows)
      for (int j = 0; j < w; ++j) {
        const int r = c0 + j, q = c0 + swp[j];
        if (q != r) {
          const int Ir = r / BNB, Iq = q / BNB;
          const double wr = r - Ir * BNB + 1, wq = q - Iq * BNB + 1;
          for (int col = tid; col < n; col += blockDim.x) {
            if (col >= c0 && col < c1) continue;
            T ar = A[r + (int64_t)col * lda], aq = A[q + (int64_t)col * lda];
            if (protect && col >= c1) {
              double d = (double)aq - (double)ar;
              c.colchk[2 * Ir + (int64_t)col * ldc] += d;
              c.colchk[2 * Ir + 1 + (int64_t)col * ldc] += wr * d;
              c.colchk[2 * Iq + (int64_t)col * ldc] -= d;
              c.colchk[2 * Iq + 1 + (int64_t)col * ldc] -= wq * d;
            }
            A[r + (int64_t)col * lda] = aq;
            A[q + (int64_t)col * lda] = ar;
          }
          if (protect)
            for (int cc = tid; cc < 2 * N; cc += blockDim.x) {
              double t = c.rowchk[r + (int64_t)cc * BMAX];
              c.rowchk[r + (int64_t)cc * BMAX] = c.rowchk[q + (int64_t)cc * BMAX];
              c.rowchk[q + (int64_t)cc * BMAX] = t;
            }
        }
        __syncthreads();
      }
    }
    if (c1 >= n) break;
    if (!CHOL) {
      // panel update U12 = L11^{-1} A12, one thread per column
      for (int col = c1 + tid; col < n; col += blockDim.x) {
        T x[BNB];
#pragma unroll
        for (int i = 0; i < BNB; ++i) x[i] = i < w ? A[(c0 + i) + (int64_t)col * lda] : (T)0;
#pragma unroll
        for (int i = 1; i < BNB; ++i)
          for (int p = 0; p < i; ++p)
            if (i < w) x[i] = fms_b(x[i], P[i * ldp + p], x[p]);
#pragma unroll
        for (int i = 0; i < BNB; ++i)
          if (i < w) A[(c0 + i) + (int64_t)col * lda] = x[i];
      }
      __syncthreads();
    }
    // ---- trailing update and checksum carry
    batch_tmu<T, CHOL>(A, lda, n, c0, w, P, ldp, Uc);
    if (protect) batch_carry<T, CHOL>(A, lda, n, k, w, P, ldp, c);
    // ---- planned faults of this matrix and iteration
    if (tid == 0)
      for (int f = 0; f < nfaults; ++f) {
        const abft_fault& F = faults[f];
        if (F.matrix != mi || F.iter != k || F.row < 0 || F.row >= n || F.col < 0 || F.col >= n) continue;
        T* p = A + F.row + (int64_t)F.col * lda;
        if (sizeof(T) == 8) {
          unsigned long long u = (unsigned long long)__double_as_longlong((double)*p) ^ (1ull << (F.bit & 63));
          *p = (T)__longlong_as_double((long long)u);
        } else {
          unsigned u = __float_as_uint((float)*p) ^ (1u << (F.bit & 31));
          *p = (T)__uint_as_float(u);
        }
      }
    __syncthreads();
    // ---- verify (and correct) the trailing tiles
    if (protect) {
      for (int J = k + 1; J < N; ++J)
        for (int I = CHOL ? J : k + 1; I < N; ++I) {
          int h = min(BNB, n - I * BNB), wj = min(BNB, n - J * BNB);
          bool diag = CHOL && I == J;
          tile_sums(A, lda, (int64_t)I * BNB, (int64_t)J * BNB, h, wj, diag, ts);
          tile_compare(ts, tf, I, J, BNB, h, wj, c.colchk, ldc, c.rowchk, BMAX, c.gc, c.gr, tsu);
          if (tf.nflag == 0) {
            store_sums(ts, I, J, BNB, h, wj, c.colchk, ldc, c.rowchk, BMAX);
            if (tid == 0 && tf.maxr > 0) rep_max_ratio(rep, tf.maxr);
          } else {
            if (tid == 0) {
              rep->flagged_tiles++;
              if (rep->first_flag_iter > k) rep->first_flag_iter = k;
            }
            correct_tile_dev(A, lda, I, J, BNB, h, wj, diag, c.colchk, ldc, c.rowchk, BMAX, c.gc, c.gr, tsu, rep, k,
                             ts, tf, cs);
          }
          __syncthreads();
        }
    }
  }
  if (tid == 0) {
    if (rep->first_flag_iter == 0x7fffffff) rep->first_flag_iter = -1;
    if (rep->nev > ABFT_MAX_EVENTS) rep->nev = ABFT_MAX_EVENTS;
  }
  __syncthreads();
}

template <typename T, int CHOL>
__global__ __launch_bounds__(256) void k_batched(int batch, const int32_t* dn, void* const* dA, const int32_t* dlda,
                                                 int32_t* const* dipiv, const int* order, unsigned* queue,
                                                 double* chkbase, int protect, double tsu, const abft_fault* faults,
                                                 int nfaults, int32_t* dinfo, abft_report* dreps) {
  extern __shared__ unsigned char smem[];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= batch) break;
    const int mi = order[item];
    const int n = dn[mi];
    if (n <= 0 || n > BMAX) {
      if (threadIdx.x == 0) {
        dinfo[mi] = n == 0 ? 0 : -1;
        dreps[mi].status = 0;
        dreps[mi].nev = 0;
        dreps[mi].first_flag_iter = -1;
      }
      continue;
    }
    factor_one<T, CHOL>(mi, n, (T*)dA[mi], (int64_t)dlda[mi], CHOL ? nullptr : dipiv[mi], chk_of(chkbase, mi), protect,
                        tsu, faults, nfaults, dinfo + mi, dreps + mi, smem);
  }
}

// ---------------------------------------------------------------------------
size_t batched_ws_bytes(int batch) {
  return (size_t)batch * batch_chk_doubles() * sizeof(double) + (size_t)batch * sizeof(int) + 256 +
         (size_t)4096 * sizeof(abft_fault);
}

int batched_factor(hipStream_t s, int chol, int prec, int batch, const int32_t* dn, void* const* dA,
                   const int32_t* dlda, int32_t* const* dipiv, void* dwork, int protect, double ts,
                   const abft_fault* hfaults, int nfaults, int32_t* dinfo, abft_report* dreps, int wgs) {
  if (batch > 8192) return ABFT_ERR_UNSUPPORTED;
  char* base = (char*)dwork;
  double* chk = (double*)base;
  size_t off = (size_t)batch * batch_chk_doubles() * sizeof(double);
  int* order = (int*)(base + off);
  off += ((size_t)batch * sizeof(int) + 255) & ~(size_t)255;
  unsigned* queue = (unsigned*)(base + off);
  off += 256;
  abft_fault* dfaults = (abft_fault*)(base + off);
  if (nfaults > 4096) return ABFT_ERR_UNSUPPORTED;
  if (nfaults > 0 &&
      hipMemcpyAsync(dfaults, hfaults, (size_t)nfaults * sizeof(abft_fault), hipMemcpyHostToDevice, s) != hipSuccess)
    return ABFT_ERR_HIP;
  hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, dn, batch, order, queue);
  if (hipGetLastError() != hipSuccess) return ABFT_ERR_HIP;
  const double u = prec == ABFT_F64 ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
  const size_t elem = prec == ABFT_F64 ? 8 : 4;
  size_t shm = std::max((size_t)BMAX * (BNB + 1) * elem + (size_t)BNB * 65 * elem, sizeof(TileSums) + sizeof(TileFlags));
  shm = (shm + 255) & ~(size_t)255;
  dim3 grid(std::min(batch, wgs));  // persistent workgroups; extra ones wait for a free CU
#define BLAUNCH(T_, C_)                                                                                            \
  hipLaunchKernelGGL((k_batched<T_, C_>), grid, dim3(256), shm, s, batch, dn, dA, dlda, dipiv, order, queue, chk,   \
                     protect, ts * u, nfaults ? dfaults : nullptr, nfaults, dinfo, dreps)
  if (prec == ABFT_F64) {
    if (chol) BLAUNCH(double, 1); else BLAUNCH(double, 0);
  } else {
    if (chol) BLAUNCH(float, 1); else BLAUNCH(float, 0);
  }
#undef BLAUNCH
  return hipGetLastError() == hipSuccess ? 0 : ABFT_ERR_HIP;
}

}  // namespace abft
