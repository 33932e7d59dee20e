// Panel kernels: Cholesky diagonal leaf, the two triangular-solve leaves,
// the cooperative LU and Householder leaves, and the row-interchange kernels.
//
// Leaves are at most 32 columns wide; the host recursion (panel.cpp side of
// the driver) splits wider panels and applies the updates between halves with
// the MFMA GEMM, so the work inside a leaf is small and latency-bound.
//
// The LU and QR leaves hold the whole m x 32 leaf in the LDS of G co-resident
// workgroups (cooperative launch); each column costs one grid barrier: every
// workgroup publishes its candidate (pivot) or its partial Gram row (QR) to
// a slot array, waits at the barrier, then all of them reduce the slots in
// the same fixed order, so every workgroup takes the same decision.
#include "common.hpp"
#include "kernels.hpp"

namespace abft {

constexpr int LEAF = 32;   // width of the triangular leaf kernels (potrf / trsm)
constexpr int CLEAF = 64;  // widest cooperative LU / QR leaf

template <typename T>
__device__ __forceinline__ T fms(T a, T b, T c) {  // a - b*c as the reference arithmetic does it
  return a - b * c;
}
template <>
__device__ __forceinline__ float fms<float>(float a, float b, float c) {
  return __fmaf_rn(-b, c, a);
}

// Row update Ld[c] -= f[c] * v for c in [cb, w) (a - b*c rounding, as the
// reference arithmetic), eight columns per step with every load issued
// before the first use (an LDS round trip per eight elements, not per one).
template <typename T, typename F>
__device__ __forceinline__ void row_axpy(T* __restrict__ x, const F* __restrict__ f, T v, int cb, int w) {
  int c = cb;
  for (; c + 8 <= w; c += 8) {
    T xv[8];
    F fv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      xv[u] = x[c + u];
      fv[u] = f[c + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) x[c + u] = fms(xv[u], (T)fv[u], v);
  }
  for (; c < w; ++c) x[c] = fms(x[c], (T)f[c], v);
}

// ---------------------------------------------------------------------------
// Cholesky of the w x w diagonal block at (c0, c0), w <= 32, right-looking in
// LDS.  info records the first non-positive pivot (global column + 1).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_potrf_leaf(T* A, int64_t lda, int64_t c0, int w, int32_t* info) {
  __shared__ T L[LEAF][LEAF + 1];
  __shared__ int fail;
  const int tid = threadIdx.x;
  if (tid == 0) fail = 0;
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    int i = idx % w, j = idx / w;
    if (i >= j) L[i][j] = A[(c0 + i) + (c0 + j) * lda];
  }
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    if (tid == 0) {
      T d = L[j][j];
      if (!(d > (T)0)) {
        if (!fail && info) atomicCAS(info, 0, (int32_t)(c0 + j + 1));
        fail = 1;
      }
      L[j][j] = sqrt(d);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < w; i += blockDim.x) L[i][j] = L[i][j] / L[j][j];
    __syncthreads();
    const int r = w - j - 1;
    for (int idx = tid; idx < r * r; idx += blockDim.x) {
      int i = j + 1 + idx % r, jj = j + 1 + idx / r;
      if (i >= jj) L[i][jj] = fms(L[i][jj], L[i][j], L[jj][j]);
    }
    __syncthreads();
  }
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    int i = idx % w, j = idx / w;
    if (i >= j) A[(c0 + i) + (c0 + j) * lda] = L[i][j];
  }
}

// X = B L^{-T} for rows [r0, r1) and columns [c0, c0+w): L the factored
// diagonal block at (c0, c0) (non-unit lower).  One thread per row.
template <typename T>
__global__ __launch_bounds__(256) void k_trsm_rlt_leaf(T* A, int64_t lda, int64_t r0, int64_t r1, int64_t c0, int w) {
  __shared__ T L[LEAF][LEAF + 1];
  __shared__ T B[256][LEAF + 1];
  const int tid = threadIdx.x;
  const int64_t rb = r0 + (int64_t)blockIdx.x * 256;
  for (int idx = tid; idx < w * w; idx += 256) {
    int i = idx % w, j = idx / w;
    L[i][j] = (i >= j) ? A[(c0 + i) + (c0 + j) * lda] : (T)0;
  }
  for (int idx = tid; idx < 256 * w; idx += 256) {
    int i = idx % 256, j = idx / 256;
    if (rb + i < r1) B[i][j] = A[(rb + i) + (c0 + j) * lda];
  }
  __syncthreads();
  if (rb + tid < r1) {
    if (w == LEAF) {  // the row in registers, fully unrolled (same operation order)
      T x[LEAF];
#pragma unroll
      for (int j = 0; j < LEAF; ++j) x[j] = B[tid][j];
#pragma unroll
      for (int j = 0; j < LEAF; ++j) {
        T s = x[j];
#pragma unroll
        for (int p = 0; p < j; ++p) s = fms(s, x[p], L[j][p]);
        x[j] = s / L[j][j];
      }
#pragma unroll
      for (int j = 0; j < LEAF; ++j) B[tid][j] = x[j];
    } else {
      for (int j = 0; j < w; ++j) {
        T s = B[tid][j];
        for (int p = 0; p < j; ++p) s = fms(s, B[tid][p], L[j][p]);
        B[tid][j] = s / L[j][j];
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < 256 * w; idx += 256) {
    int i = idx % 256, j = idx / 256;
    if (rb + i < r1) A[(rb + i) + (c0 + j) * lda] = B[i][j];
  }
}

// X = L^{-1} B for the w rows [c0, c0+w) of columns [j0, j1): L unit lower at
// (c0, c0).  One thread per column.
template <typename T>
__global__ __launch_bounds__(256) void k_trsm_llu_leaf(T* A, int64_t lda, int64_t c0, int w, int64_t j0, int64_t j1) {
  __shared__ T L[LEAF][LEAF + 1];
  __shared__ T B[256][LEAF + 1];
  const int tid = threadIdx.x;
  const int64_t jb = j0 + (int64_t)blockIdx.x * 256;
  for (int idx = tid; idx < w * w; idx += 256) {
    int i = idx % w, j = idx / w;
    L[i][j] = (i > j) ? A[(c0 + i) + (c0 + j) * lda] : (T)0;
  }
  for (int idx = tid; idx < 256 * w; idx += 256) {
    int i = idx % w, c = idx / w;
    if (jb + c < j1) B[c][i] = A[(c0 + i) + (jb + c) * lda];
  }
  __syncthreads();
  if (jb + tid < j1) {
    if (w == LEAF) {  // the column in registers, fully unrolled (same operation order)
      T x[LEAF];
#pragma unroll
      for (int i = 0; i < LEAF; ++i) x[i] = B[tid][i];
#pragma unroll
      for (int i = 1; i < LEAF; ++i) {
        T s = x[i];
#pragma unroll
        for (int p = 0; p < i; ++p) s = fms(s, L[i][p], x[p]);
        x[i] = s;
      }
#pragma unroll
      for (int i = 0; i < LEAF; ++i) B[tid][i] = x[i];
    } else {
      for (int i = 0; i < w; ++i) {
        T s = B[tid][i];
        for (int p = 0; p < i; ++p) s = fms(s, L[i][p], B[tid][p]);
        B[tid][i] = s;
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < 256 * w; idx += 256) {
    int i = idx % w, c = idx / w;
    if (jb + c < j1) A[(c0 + i) + (jb + c) * lda] = B[c][i];
  }
}

// ---------------------------------------------------------------------------
// Cooperative LU leaf: columns [c0, c0+w), rows [c0, m); workgroup g owns
// rows [c0 + g R, c0 + (g+1) R) in LDS.  Partial pivoting with the first
// index on ties; row interchanges inside the leaf columns only (the caller
// applies them to the other columns).
// ---------------------------------------------------------------------------
#ifdef ABFT_LEAF_TIMING
#define LT_DECL unsigned long long lt_t = __builtin_amdgcn_s_memtime(), lt_acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#define LT_MARK(k)                                        \
  do {                                                    \
    unsigned long long lt_n = __builtin_amdgcn_s_memtime(); \
    lt_acc[k] += lt_n - lt_t;                             \
    lt_t = lt_n;                                          \
  } while (0)
#define LT_PRINT(name)                                                                                          \
  if (blockIdx.x == 0 && threadIdx.x == 0 && c0 < 64)                                                          \
    printf("%s c0=%ld G=%d R=%d w=%d: %llu %llu %llu %llu %llu %llu %llu %llu\n", name, (long)c0, (int)gridDim.x, R, w, \
           lt_acc[0], lt_acc[1], lt_acc[2], lt_acc[3], lt_acc[4], lt_acc[5], lt_acc[6], lt_acc[7]);
#else
#define LT_DECL
#define LT_MARK(k)
#define LT_PRINT(name)
#endif

template <typename T>
__device__ __forceinline__ bool better(double a, int64_t ia, double b, int64_t ib) {
  return a > b || (a == b && ia < ib);
}

template <typename T>
__global__ __launch_bounds__(256) void k_getrf_leaf(T* A, int64_t lda, int64_t m, int64_t c0, int w, int R,
                                                    int32_t* ipiv, int32_t* info, double* slots, unsigned* ctr,
                                                    unsigned ctr_base, abft_report* rep) {
  extern __shared__ unsigned char smem_raw[];
  LT_DECL
  T* Ld = reinterpret_cast<T*>(smem_raw);  // R x (w+1)
  const int ldl = w + 1;
  __shared__ double prow[CLEAF], orow[CLEAF];
  __shared__ double wv_val[4];
  __shared__ int64_t wv_idx[4];
  __shared__ int wv_g[4];
  __shared__ int64_t s_piv, s_loc;
  __shared__ int s_pg;
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t rbeg = c0 + (int64_t)g * R;
  const int rows = (int)max((int64_t)0, min((int64_t)R, m - rbeg));
  const int slot_stride = G * (w + 2) + w;

  for (int idx = tid; idx < rows * w; idx += 256) {
    int i = idx % rows, j = idx / rows;
    Ld[i * ldl + j] = A[(rbeg + i) + (c0 + j) * lda];
  }
  __syncthreads();

  for (int j = 0; j < w; ++j) {
    const int64_t d = c0 + j;  // diagonal row
    double* sj = slots + (size_t)j * slot_stride;
    // local argmax of |a(i, j)| over owned rows i >= d
    double bv = -1.0;
    int64_t bi = INT64_MAX;
    for (int i = tid; i < rows; i += 256) {
      int64_t gi = rbeg + i;
      if (gi < d) continue;
      double v = fabs((double)Ld[i * ldl + j]);
      if (better<T>(v, gi, bv, bi)) { bv = v; bi = gi; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      double ov = __shfl_xor(bv, o);
      int64_t oi = __shfl_xor(bi, o);
      if (better<T>(ov, oi, bv, bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { wv_val[wv] = bv; wv_idx[wv] = bi; }
    __syncthreads();
    if (tid == 0) {
      for (int q = 1; q < 4; ++q)
        if (better<T>(wv_val[q], wv_idx[q], bv, bi)) { bv = wv_val[q]; bi = wv_idx[q]; }
      sj[g * (w + 2) + 0] = bv;
      sj[g * (w + 2) + 1] = (double)bi;
      s_loc = bi;
    }
    __syncthreads();
    // candidate row (values of the leaf columns) and, from workgroup 0, row d
    if (tid < w) {
      const int64_t bl = s_loc;
      double val = 0.0;
      if (bl != INT64_MAX) val = (double)Ld[(bl - rbeg) * ldl + tid];
      sj[g * (w + 2) + 2 + tid] = val;
      if (g == 0) sj[G * (w + 2) + tid] = (double)Ld[(d - rbeg) * ldl + tid];
    }
    LT_MARK(0);
    grid_barrier(ctr, ctr_base + (unsigned)(j + 1) * G, rep, nullptr);
    LT_MARK(1);
    // every workgroup picks the same winner: one slot per thread, then a
    // block argmax (largest |value|, first row index on ties; the row index
    // identifies its workgroup, so the choice does not depend on the order)
    {
      double v = -1.0;
      int64_t ii = INT64_MAX;
      int gq = 0;
      for (int q = tid; q < G; q += 256) {
        const double vq = sj[q * (w + 2) + 0];
        const int64_t iq = vq < 0 ? INT64_MAX : (int64_t)sj[q * (w + 2) + 1];
        if (vq >= 0 && better<T>(vq, iq, v, ii)) { v = vq; ii = iq; gq = q; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o);
        const int64_t oi = __shfl_xor(ii, o);
        const int og = __shfl_xor(gq, o);
        if (better<T>(ov, oi, v, ii)) { v = ov; ii = oi; gq = og; }
      }
      if (lane == 0) { wv_val[wv] = v; wv_idx[wv] = ii; wv_g[wv] = gq; }
      __syncthreads();
      if (tid == 0) {
        double best = wv_val[0];
        int64_t bidx = wv_idx[0];
        int bg = wv_g[0];
        for (int q = 1; q < 4; ++q)
          if (better<T>(wv_val[q], wv_idx[q], best, bidx)) { best = wv_val[q]; bidx = wv_idx[q]; bg = wv_g[q]; }
        if (bidx == INT64_MAX) { bidx = d; bg = 0; }
        s_piv = bidx;
        s_pg = bg;
      }
      __syncthreads();
    }
    LT_MARK(2);
    const int64_t p = s_piv;
    const int pg = s_pg;
    if (tid < w) {
      prow[tid] = sj[pg * (w + 2) + 2 + tid];
      orow[tid] = sj[G * (w + 2) + tid];
    }
    __syncthreads();
    LT_MARK(3);
    if (p != d) {
      if (g == 0 && tid < w) Ld[(d - rbeg) * ldl + tid] = (T)prow[tid];
      if (p >= rbeg && p < rbeg + rows && tid < w) Ld[(p - rbeg) * ldl + tid] = (T)orow[tid];
    }
    __syncthreads();
    if (g == 0 && tid == 0) {
      ipiv[d] = (int32_t)(p + 1);
      if (prow[j] == 0.0 && info) atomicCAS(info, 0, (int32_t)(d + 1));
    }
    const T piv = (T)prow[j];
    if (piv != (T)0) {
      for (int i = tid; i < rows; i += 256) {
        int64_t gi = rbeg + i;
        if (gi <= d) continue;
        T l = Ld[i * ldl + j] / piv;
        Ld[i * ldl + j] = l;
        row_axpy(Ld + i * ldl, prow, l, j + 1, w);  // a(i,c) - l * u(c)
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < rows * w; idx += 256) {
    int i = idx % rows, j = idx / rows;
    A[(rbeg + i) + (c0 + j) * lda] = Ld[i * ldl + j];
  }
  LT_MARK(4);
  LT_PRINT("lu_leaf")
}

// ---------------------------------------------------------------------------
// Cooperative Householder leaf: columns [c0, c0+w), rows [c0, m) (LAPACK
// dlarfg convention), plus the leaf's triangular factor T (forward,
// columnwise) written at T[toff + toff*ldt].
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_geqrf_leaf(double* A, int64_t lda, int64_t m, int64_t c0, int w, int R,
                                                    double* tau, double* Tm, int ldt, int toff, double* slots,
                                                    unsigned* ctr, unsigned ctr_base, abft_report* rep) {
  extern __shared__ unsigned char smem_raw[];
  LT_DECL
  double* Ld = reinterpret_cast<double*>(smem_raw);  // R x (w+1)
  const int ldl = w + 1;
  __shared__ double part[4][CLEAF];
  __shared__ double qpart[256 / CLEAF][CLEAF];
  __shared__ double svec[CLEAF], orow[CLEAF], fvec[CLEAF];
  __shared__ double s_beta, s_tau, s_scale;
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int64_t rbeg = c0 + (int64_t)g * R;
  const int rows = (int)max((int64_t)0, min((int64_t)R, m - rbeg));
  // per column: G workgroup partial Gram rows, then row d (w values each)
  const size_t slot_stride = (size_t)(G + 1) * w;

  for (int idx = tid; idx < rows * w; idx += 256) {
    int i = idx % rows, j = idx / rows;
    Ld[i * ldl + j] = A[(rbeg + i) + (c0 + j) * lda];
  }
  __syncthreads();

  // sum of the G records of len values (src + r * len) for entries e <
  // len: QG threads share an entry (records r = gq, gq + QG, ...), eight
  // loads in flight each; the parts are added in a fixed order.  The result
  // goes to dst[e] (LDS).
  constexpr int QG = 256 / CLEAF;
  auto sum_slots = [&](const double* src, int len, double* dst) {
    for (int e0 = 0; e0 < len; e0 += CLEAF) {
      const int c = tid % CLEAF, gq = tid / CLEAF, e = e0 + c;
      double pp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (e < len) {
        int r = gq;
        for (; r + 7 * QG < G; r += 8 * QG) {
#pragma unroll
          for (int u = 0; u < 8; ++u) pp[u] += src[(size_t)(r + u * QG) * len + e];
        }
        for (int u = 0; r < G; r += QG, ++u) pp[u] += src[(size_t)r * len + e];
      }
      double t = pp[0];
#pragma unroll
      for (int u = 1; u < 8; ++u) t += pp[u];
      qpart[gq][c] = t;
      __syncthreads();
      if (tid < CLEAF && e0 + tid < len) {
        double v = qpart[0][tid];
        for (int u = 1; u < QG; ++u) v += qpart[u][tid];
        dst[e0 + tid] = v;
      }
      __syncthreads();
    }
  };

  for (int j = 0; j < w; ++j) {
    const int64_t d = c0 + j;
    double* sj = slots + (size_t)j * slot_stride;
    double* rowd = sj + (size_t)G * w;
    // partial Gram row: s_c = sum_{i > d} a(i,j) a(i,c), c = j..w-1; thread
    // (q, cl) takes column c = j + cl over the rows i = q (mod 4) of the LDS
    // panel, and the four row classes are added in order
    {
      const int cl = tid & 63, q = tid >> 6, c = j + cl;
      double acc = 0.0;
      if (c < w) {
        const int i0 = (int)max((int64_t)0, d + 1 - rbeg);
        int i = i0 + ((q - i0 % 4) + 4) % 4;
        for (; i + 28 < rows; i += 32) {  // eight rows per step, loads first
          double xa[8], xb[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            xa[u] = Ld[(i + 4 * u) * ldl + j];
            xb[u] = Ld[(i + 4 * u) * ldl + c];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) acc += xa[u] * xb[u];
        }
        for (; i < rows; i += 4) acc += Ld[i * ldl + j] * Ld[i * ldl + c];
      }
      part[q][cl] = acc;
    }
    __syncthreads();
    LT_MARK(0);
    if (tid < w) {
      double v = 0.0;
      if (tid >= j) v = ((part[0][tid - j] + part[1][tid - j]) + part[2][tid - j]) + part[3][tid - j];
      sj[(size_t)g * w + tid] = v;
      if (g == 0) rowd[tid] = Ld[(d - rbeg) * ldl + tid];
    }
    LT_MARK(1);
    grid_barrier(ctr, ctr_base + (unsigned)(j + 1) * G, rep, nullptr);
    LT_MARK(2);
    // every workgroup: Gram row = sum of the G partial rows, and row d
    if (tid < w) orow[tid] = rowd[tid];
    sum_slots(sj, w, svec);
    LT_MARK(3);
    if (tid == 0) {
      double alpha = orow[j], s2 = svec[j];
      if (s2 == 0.0) {
        s_tau = 0.0; s_scale = 0.0; s_beta = alpha;
      } else {
        double beta = -copysign(sqrt(alpha * alpha + s2), alpha);
        s_tau = (beta - alpha) / beta;
        s_scale = 1.0 / (alpha - beta);
        s_beta = beta;
      }
      if (g == 0) tau[d] = s_tau;
    }
    __syncthreads();
    const double t = s_tau, sc = s_scale;
    if (t != 0.0) {
      if (tid < w && tid > j) fvec[tid] = t * (orow[tid] + sc * svec[tid]);
      __syncthreads();
      for (int i = tid; i < rows; i += 256) {
        int64_t gi = rbeg + i;
        if (gi < d) continue;
        if (gi == d) {
          Ld[i * ldl + j] = s_beta;
          for (int c = j + 1; c < w; ++c) Ld[i * ldl + c] -= fvec[c];
        } else {
          double v = Ld[i * ldl + j] * sc;
          Ld[i * ldl + j] = v;
          row_axpy(Ld + i * ldl, fvec, v, j + 1, w);  // a(i,c) - f(c) * v
        }
      }
    }
    __syncthreads();
    LT_MARK(4);
  }
  // T factor of the leaf from the Gram matrix of V (unit diagonal, zeros above)
  double* sg = slots + (size_t)w * slot_stride;  // G partial Gram matrices (w*w each)
  for (int e = tid; e < w * w; e += 256) {
    int q = e % w, jj = e / w;
    double acc = 0.0;
    if (q < jj) {
      // rows inside the leaf's top w x w block carry the unit diagonal and
      // the zeros above it; the rows below are plain (eight per step)
      const int itop = (int)min((int64_t)rows, max((int64_t)0, c0 + w - rbeg));
      for (int i = 0; i < itop; ++i) {
        int64_t li = rbeg + i - c0;  // row index relative to the leaf top
        double vq = (li < q) ? 0.0 : (li == q ? 1.0 : Ld[i * ldl + q]);
        double vj = (li < jj) ? 0.0 : (li == jj ? 1.0 : Ld[i * ldl + jj]);
        acc += vq * vj;
      }
      int i = itop;
      for (; i + 8 <= rows; i += 8) {
        double xa[8], xb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          xa[u] = Ld[(i + u) * ldl + q];
          xb[u] = Ld[(i + u) * ldl + jj];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += xa[u] * xb[u];
      }
      for (; i < rows; ++i) acc += Ld[i * ldl + q] * Ld[i * ldl + jj];
    }
    sg[(size_t)g * w * w + e] = acc;
  }
  // the panel goes back to A first: workgroup 0 then reuses its LDS for the
  // Gram matrix and T (2 w (w+1) doubles <= R (w+1), since R >= 2w)
  for (int idx = tid; idx < rows * w; idx += 256) {
    int i = idx % rows, j = idx / rows;
    A[(rbeg + i) + (c0 + j) * lda] = Ld[i * ldl + j];
  }
  LT_MARK(5);
  grid_barrier(ctr, ctr_base + (unsigned)(w + 1) * G, rep, nullptr);
  LT_MARK(6);
  if (g == 0) {
    double* Gm = Ld;                 // Gm[q * ldl + j]
    double* Tl = Ld + w * ldl;       // Tl[q * ldl + j]
    // the Gram matrix (sum of the G partials), staged in Tl's space: one
    // entry per thread, eight loads in flight, parts added in order
    for (int e = tid; e < w * w; e += 256) {
      double pp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int r = 0;
      for (; r + 8 <= G; r += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) pp[u] += sg[(size_t)(r + u) * w * w + e];
      }
      for (int u = 0; r < G; ++r, ++u) pp[u] += sg[(size_t)r * w * w + e];
      double t = pp[0];
#pragma unroll
      for (int u = 1; u < 8; ++u) t += pp[u];
      Tl[e] = t;
    }
    __syncthreads();
    for (int e = tid; e < w * w; e += 256) {
      Gm[(e % w) * ldl + e / w] = Tl[e];
    }
    __syncthreads();
    for (int e = tid; e < w * w; e += 256) Tl[(e % w) * ldl + e / w] = 0.0;
    __syncthreads();
    for (int jj = 0; jj < w; ++jj) {
      double tj = tau[c0 + jj];
      if (tid == 0) Tl[jj * ldl + jj] = tj;
      if (tid < jj) {
        double sacc = 0.0;
        int q = tid;
        for (; q + 8 <= jj; q += 8) {
          double ta[8], gb[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            ta[u] = Tl[tid * ldl + q + u];
            gb[u] = Gm[(q + u) * ldl + jj];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) sacc += ta[u] * gb[u];
        }
        for (; q < jj; ++q) sacc += Tl[tid * ldl + q] * Gm[q * ldl + jj];
        Tl[tid * ldl + jj] = -tj * sacc;
      }
      __syncthreads();
    }
    for (int e = tid; e < w * w; e += 256)
      Tm[(toff + e % w) + (int64_t)(toff + e / w) * ldt] = Tl[(e % w) * ldl + e / w];
  }
  LT_MARK(7);
  LT_PRINT("qr_leaf")
}

// ---------------------------------------------------------------------------
// Row interchanges.  k_perm_build turns the interchanges ipiv[c0..c0+w) into
// the list of moved rows (dst <- src), sorted by dst.  k_laswp applies the
// moves to columns [j0, j1) through a staging buffer; with a column-checksum
// array it also adds, per tile-row, the change of the column sums and of the
// weighted column sums (compensated, in the moves' fixed order).
// ---------------------------------------------------------------------------
// The table holds, for every row r in [c0, n), the original row now stored at
// r (-1: unchanged).  Rows [c0, n) of the panel bound the table (<= 36864
// rows in LDS); one thread replays the interchanges, then a block-wide
// compaction lists the moved rows in increasing order.
// Move list of the w row interchanges of a panel starting at row c0: after
// the swaps, row dst holds the original row src; moves = {count, dst0, src0,
// dst1, src1, ...} in increasing dst.  Only the panel's own rows [0, w) and
// the distinct pivot rows at or below w (relative to c0) can move, so the
// replay works on a compact table of at most 2w entries: entry t < w is row
// t, entry w + f is the pivot row first named by interchange f.
constexpr int PB_W = 512;  // largest panel width (block size)
__global__ __launch_bounds__(2 * PB_W) void k_perm_build(const int32_t* ipiv, int64_t c0, int w, int64_t n,
                                                        int* moves) {
  __shared__ int pv[PB_W], sidx[PB_W];
  __shared__ int key[2 * PB_W], cur[2 * PB_W];
  __shared__ int nmoved;
  const int tid = threadIdx.x;
  const int rows = (int)min<int64_t>(n - c0, 0x7fffffff);
  if (tid < w) {
    int p = ipiv[c0 + tid] - 1 - (int)c0;
    if (p < 0 || p >= rows) p = tid;  // not produced by the panel; no interchange
    pv[tid] = p;
  }
  if (tid == 0) nmoved = 0;
  __syncthreads();
  if (tid < w) {
    const int p = pv[tid];
    int f = tid;
    if (p >= w)
      for (int t = 0; t < tid; ++t)
        if (pv[t] == p) { f = t; break; }
    sidx[tid] = p < w ? p : w + f;
    key[tid] = tid;
    key[w + tid] = (p >= w && f == tid) ? p : -1;
  }
  __syncthreads();
  for (int i = tid; i < 2 * w; i += blockDim.x) cur[i] = key[i];
  __syncthreads();
  if (tid == 0)
    for (int t = 0; t < w; ++t) {
      const int b = sidx[t];
      if (b != t) {
        const int x = cur[t];
        cur[t] = cur[b];
        cur[b] = x;
      }
    }
  __syncthreads();
  // rank every moved entry by its row (rows are distinct) and emit in order
  for (int i = tid; i < 2 * w; i += blockDim.x) {
    const int ki = key[i];
    if (ki < 0 || cur[i] == ki) continue;
    int r = 0;
    for (int q = 0; q < 2 * w; ++q) {
      const int kq = key[q];
      r += (kq >= 0 && cur[q] != kq && kq < ki);
    }
    moves[1 + 2 * r] = (int)(c0 + ki);
    moves[2 + 2 * r] = (int)(c0 + cur[i]);
    atomicAdd(&nmoved, 1);
  }
  __syncthreads();
  if (tid == 0) moves[0] = nmoved;
}

// Row interchanges on columns [j0, j1).  TPC threads share a column (the
// column's moves are dealt round-robin; TPC = 1 for wide ranges); all moved
// values are read (in batches of independent loads) and parked in `stage`
// before any is written, so cycles of moves need no ordering.  With colchk
// (TPC = 1), the column checksums of every tile-row that receives a new value
// are corrected by the plain and position-weighted differences (moves arrive
// in increasing destination row, so each tile-row's corrections are
// contiguous).
constexpr int LASWP_BATCH = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_laswp(T* __restrict__ A, int64_t lda, int64_t j0, int64_t j1,
                                               const int* __restrict__ moves, T* __restrict__ stage,
                                               double* __restrict__ colchk, int64_t ldc, int nb, int tpc) {
  __shared__ int mv[4 * PB_W];
  const int nm = moves[0];
  for (int t = threadIdx.x; t < 2 * nm; t += blockDim.x) mv[t] = moves[1 + t];
  __syncthreads();
  const int cpb = (int)blockDim.x / tpc, sub = threadIdx.x % tpc;
  const int64_t j = j0 + (int64_t)blockIdx.x * cpb + threadIdx.x / tpc;
  const bool active = j < j1;
  const int64_t nc = j1 - j0, jj = j - j0;
  T* __restrict__ col = A + (active ? j : j0) * lda;
  acc2 e{0, 0}, ww{0, 0};
  int curI = -1;
  auto flush = [&]() {
    if (curI >= 0) {
      acc2 c0{colchk[2 * curI + j * ldc], 0}, c1{colchk[2 * curI + 1 + j * ldc], 0};
      cmerge(c0, e);
      cmerge(c1, ww);
      colchk[2 * curI + j * ldc] = cval(c0);
      colchk[2 * curI + 1 + j * ldc] = cval(c1);
    }
  };
  if (active) {
    for (int t0 = sub; t0 < nm; t0 += LASWP_BATCH * tpc) {
      T vs[LASWP_BATCH], vd[LASWP_BATCH];
#pragma unroll
      for (int u = 0; u < LASWP_BATCH; ++u) {
        const int t = t0 + u * tpc;
        if (t < nm) {
          vs[u] = col[mv[2 * t + 1]];
          if (colchk) vd[u] = col[mv[2 * t]];
        }
      }
#pragma unroll
      for (int u = 0; u < LASWP_BATCH; ++u) {
        const int t = t0 + u * tpc;
        if (t < nm) {
          stage[(int64_t)t * nc + jj] = vs[u];
          if (colchk) {
            const int dst = mv[2 * t];
            const int I = dst / nb;
            if (I != curI) {
              flush();
              curI = I;
              e = {0, 0};
              ww = {0, 0};
            }
            const double wr = (double)(dst - I * nb + 1);
            cadd(e, (double)vs[u]);
            cadd(e, -(double)vd[u]);
            cfma(ww, wr, (double)vs[u]);
            cfma(ww, -wr, (double)vd[u]);
          }
        }
      }
    }
    if (colchk) flush();
  }
  if (tpc > 1) __syncthreads();  // every value of the column is staged before any is written
  if (active) {
    for (int t0 = sub; t0 < nm; t0 += LASWP_BATCH * tpc) {
      T v[LASWP_BATCH];
#pragma unroll
      for (int u = 0; u < LASWP_BATCH; ++u) {
        const int t = t0 + u * tpc;
        if (t < nm) v[u] = stage[(int64_t)t * nc + jj];
      }
#pragma unroll
      for (int u = 0; u < LASWP_BATCH; ++u) {
        const int t = t0 + u * tpc;
        if (t < nm) col[mv[2 * t]] = v[u];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
#define CHECK_LAUNCH() return hipGetLastError() == hipSuccess ? 0 : ABFT_ERR_HIP

template <typename T>
int potrf_leaf(hipStream_t s, T* A, int64_t lda, int64_t c0, int w, int32_t* info) {
  hipLaunchKernelGGL(k_potrf_leaf<T>, dim3(1), dim3(256), 0, s, A, lda, c0, w, info);
  CHECK_LAUNCH();
}
template <typename T>
int trsm_rlt_leaf(hipStream_t s, T* A, int64_t lda, int64_t r0, int64_t r1, int64_t c0, int w) {
  if (r1 <= r0) return 0;
  hipLaunchKernelGGL(k_trsm_rlt_leaf<T>, dim3((unsigned)((r1 - r0 + 255) / 256)), dim3(256), 0, s, A, lda, r0, r1, c0, w);
  CHECK_LAUNCH();
}
template <typename T>
int trsm_llu_leaf(hipStream_t s, T* A, int64_t lda, int64_t c0, int w, int64_t j0, int64_t j1) {
  if (j1 <= j0) return 0;
  hipLaunchKernelGGL(k_trsm_llu_leaf<T>, dim3((unsigned)((j1 - j0 + 255) / 256)), dim3(256), 0, s, A, lda, c0, w, j0, j1);
  CHECK_LAUNCH();
}

// rows per workgroup of a cooperative leaf: enough workgroups to spread m
// rows, at least w rows in workgroup 0, at most `maxg` workgroups
static inline void coop_shape(int64_t rows, int w, int maxg, int max_rows, int& G, int& R) {
  int64_t r = (rows + maxg - 1) / maxg;
  if (r < 256) r = 256;
  if (r < w) r = w;
  if (r > max_rows) r = max_rows;
  G = (int)((rows + r - 1) / r);
  if (G < 1) G = 1;
  R = (int)r;
}

template <typename T>
int getrf_leaf(hipStream_t s, T* A, int64_t lda, int64_t m, int64_t c0, int w, int32_t* ipiv, int32_t* info,
               double* slots, unsigned* ctr, unsigned* ctr_base, abft_report* rep, int maxg) {
  int G, R;
  const int max_rows = (int)((144 * 1024) / ((w + 1) * sizeof(T)));
  coop_shape(m - c0, w, maxg, max_rows, G, R);
  if ((int64_t)G * R < m - c0) return ABFT_ERR_UNSUPPORTED;
  size_t shm = (size_t)R * (w + 1) * sizeof(T);
  void* args[] = {&A, &lda, &m, &c0, &w, &R, &ipiv, &info, &slots, &ctr, ctr_base, &rep};
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_getrf_leaf<T>, dim3(G), dim3(256), args, shm, s);
  *ctr_base += (unsigned)w * G;
  return e == hipSuccess ? 0 : ABFT_ERR_HIP;
}

int geqrf_leaf(hipStream_t s, double* A, int64_t lda, int64_t m, int64_t c0, int w, double* tau, double* Tm, int ldt,
               int toff, double* slots, unsigned* ctr, unsigned* ctr_base, abft_report* rep, int maxg) {
  int G, R;
  const int max_rows = (int)((140 * 1024) / ((w + 1) * sizeof(double)));
  coop_shape(m - c0, w, maxg, max_rows, G, R);
  if ((int64_t)G * R < m - c0) return ABFT_ERR_UNSUPPORTED;
  size_t shm = (size_t)R * (w + 1) * sizeof(double);
  void* args[] = {&A, &lda, &m, &c0, &w, &R, &tau, &Tm, &ldt, &toff, &slots, &ctr, ctr_base, &rep};
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_geqrf_leaf, dim3(G), dim3(256), args, shm, s);
  *ctr_base += (unsigned)(w + 1) * G;
  return e == hipSuccess ? 0 : ABFT_ERR_HIP;
}

int perm_build(hipStream_t s, const int32_t* ipiv, int64_t c0, int w, int64_t n, int* moves) {
  if (w < 0 || w > PB_W) return ABFT_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k_perm_build, dim3(1), dim3(2 * PB_W), 0, s, ipiv, c0, w, n, moves);
  CHECK_LAUNCH();
}
template <typename T>
int laswp(hipStream_t s, T* A, int64_t lda, int64_t j0, int64_t j1, const int* moves, T* stage, double* colchk,
          int64_t ldc, int nb) {
  if (j1 <= j0) return 0;
  // Every moved value is its own cache line (rows are scattered), so the
  // work is spread over as many CUs as possible: without checksums 16
  // threads per column (4 for wide ranges) share a column's moves; with
  // checksums (one thread per column) 64-thread workgroups.
  int tpc = 1, bs = 64;
  if (!colchk) {
    tpc = (j1 - j0) >= 4096 ? 4 : 16;
    bs = 256;
  }
  const int64_t cpb = bs / tpc;
  hipLaunchKernelGGL(k_laswp<T>, dim3((unsigned)((j1 - j0 + cpb - 1) / cpb)), dim3(bs), 0, s, A, lda, j0, j1, moves,
                     stage, colchk, ldc, nb, tpc);
  CHECK_LAUNCH();
}

template int potrf_leaf<double>(hipStream_t, double*, int64_t, int64_t, int, int32_t*);
template int potrf_leaf<float>(hipStream_t, float*, int64_t, int64_t, int, int32_t*);
template int trsm_rlt_leaf<double>(hipStream_t, double*, int64_t, int64_t, int64_t, int64_t, int);
template int trsm_rlt_leaf<float>(hipStream_t, float*, int64_t, int64_t, int64_t, int64_t, int);
template int trsm_llu_leaf<double>(hipStream_t, double*, int64_t, int64_t, int, int64_t, int64_t);
template int trsm_llu_leaf<float>(hipStream_t, float*, int64_t, int64_t, int, int64_t, int64_t);
template int getrf_leaf<double>(hipStream_t, double*, int64_t, int64_t, int64_t, int, int32_t*, int32_t*, double*,
                                unsigned*, unsigned*, abft_report*, int);
template int getrf_leaf<float>(hipStream_t, float*, int64_t, int64_t, int64_t, int, int32_t*, int32_t*, double*,
                               unsigned*, unsigned*, abft_report*, int);
template int laswp<double>(hipStream_t, double*, int64_t, int64_t, int64_t, const int*, double*, double*, int64_t, int);
template int laswp<float>(hipStream_t, float*, int64_t, int64_t, int64_t, const int*, float*, double*, int64_t, int);

}  // namespace abft
