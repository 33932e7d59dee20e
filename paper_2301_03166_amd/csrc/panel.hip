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

typedef double f64x4 __attribute__((ext_vector_type(4)));

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
// X = L^{-1} B in one launch, L unit lower w x w at (c0, c0) (w <= 512), B
// rows [c0, c0+w) of columns [j0, j1).  A workgroup keeps a strip of
// TRS_CB columns of B in LDS and walks the 32-row blocks of L: the diagonal
// block's substitution runs in registers (one thread per column, the
// elimination order of the 32-wide leaf), its solution is copied row-major,
// and the rows below subtract its products with the block's 32 columns of L
// (read straight from memory, shared by all strips through L2) on FP64 MFMA
// tiles of 16 rows x 16 strip columns.
// ---------------------------------------------------------------------------
constexpr int TRS_CB = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_trsm_llu_blk(T* A, int64_t lda, int64_t c0, int w, int64_t j0, int64_t j1) {
  extern __shared__ unsigned char trs_raw[];
  const int wp = (w + LEAF - 1) / LEAF * LEAF;  // rows padded with zeros to whole blocks
  const int ldb = wp + 1;
  T* Bs = reinterpret_cast<T*>(trs_raw);  // Bs[c * ldb + i]
  __shared__ T Ls[LEAF][LEAF + 1];
  __shared__ __attribute__((aligned(16))) T Xs[LEAF][TRS_CB];  // solved block, row-major
  const int tid = threadIdx.x;
  const int64_t jb = j0 + (int64_t)blockIdx.x * TRS_CB;
  const int ncol = (int)min((int64_t)TRS_CB, j1 - jb);
  for (int idx = tid; idx < wp * TRS_CB; idx += 256) {
    const int i = idx % wp, c = idx / wp;
    Bs[c * ldb + i] = (c < ncol && i < w) ? A[(c0 + i) + (jb + c) * lda] : (T)0;
  }
  for (int r0 = 0; r0 < w; r0 += LEAF) {
    const int bw = min(LEAF, w - r0);
    for (int idx = tid; idx < LEAF * LEAF; idx += 256) {
      const int i = idx % LEAF, p = idx / LEAF;
      Ls[i][p] = (i < bw && p < i) ? A[(c0 + r0 + i) + (c0 + r0 + p) * lda] : (T)0;
    }
    __syncthreads();
    if (tid < TRS_CB) {
      // (rows past w are zero and their L rows too: no guards needed)
      T x[LEAF];
#pragma unroll
      for (int i = 0; i < LEAF; ++i) x[i] = Bs[tid * ldb + r0 + i];
#pragma unroll
      for (int i = 1; i < LEAF; ++i) {
        T sacc = x[i];
#pragma unroll
        for (int p = 0; p < i; ++p) sacc = fms(sacc, Ls[i][p], x[p]);
        x[i] = sacc;
      }
#pragma unroll
      for (int i = 0; i < LEAF; ++i) {
        Bs[tid * ldb + r0 + i] = x[i];
        Xs[i][tid] = x[i];
      }
    }
    __syncthreads();
    // rows below the block, 16-row tiles per wave on FP64 MFMA (16x16x4):
    // lane (il, kl) feeds L(row il, column kl of the k-step) and X(row kl,
    // column il), and holds rows il, columns 4r + kl of the tile in reg r
    {
      const int lane = tid & 63, wv = tid >> 6, il = lane & 15, kl = lane >> 4;
      for (int rt = r0 + bw + 16 * wv; rt < w; rt += 64) {
        const bool rin = rt + il < w;
        f64x4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = rin ? (double)Bs[(4 * r + kl) * ldb + rt + il] : 0.0;
#pragma unroll
        for (int p0 = 0; p0 < LEAF; p0 += 4) {
          const int p = p0 + kl;
          const double a = (rin && p < bw) ? -(double)A[(c0 + rt + il) + (c0 + r0 + p) * lda] : 0.0;
          const double b = p < bw ? (double)Xs[p][il] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, acc, 0, 0, 0);
        }
        if (rin) {
#pragma unroll
          for (int r = 0; r < 4; ++r) Bs[(4 * r + kl) * ldb + rt + il] = (T)acc[r];
        }
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < w * TRS_CB; idx += 256) {
    const int i = idx % w, c = idx / w;
    if (c < ncol) A[(c0 + i) + (jb + c) * lda] = Bs[c * ldb + i];
  }
}

// ---------------------------------------------------------------------------
// Cooperative LU leaf: columns [c0, c0+w), rows [c0, m); workgroup g owns
// rows [c0 + g R, c0 + (g+1) R) in LDS.  Partial pivoting with the first
// index on ties; row interchanges inside the leaf columns only (the caller
// applies them to the other columns).
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ bool better(double a, int64_t ia, double b, int64_t ib) {
  return a > b || (a == b && ia < ib);
}

// Wave arg-max of (v, i) under `better` (larger v, then smaller i), result in
// every lane.  Lanes exchange values with DPP moves inside each row of 16
// (quad permutations, then the half-row and row mirrors: a few cycles each,
// against an LDS round trip per step for a general shuffle); the four row
// results are then read with readlane and combined.  `better` is a total
// order, so the result does not depend on the combining order.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  return __hiloint2double(dpp_i<CTRL>(__double2hiint(x)), dpp_i<CTRL>(__double2loint(x)));
}
__device__ __forceinline__ double readlane_d(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}
template <int CTRL>
__device__ __forceinline__ void argmax_step(double& v, int& i) {
  const double ov = dpp_d<CTRL>(v);
  const int oi = dpp_i<CTRL>(i);
  if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
}
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  argmax_step<0xB1>(v, i);   // quad_perm [1, 0, 3, 2]
  argmax_step<0x4E>(v, i);   // quad_perm [2, 3, 0, 1]
  argmax_step<0x141>(v, i);  // row_half_mirror
  argmax_step<0x140>(v, i);  // row_mirror
  double bv = readlane_d(v, 0);
  int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) {
    const double ov = readlane_d(v, r);
    const int oi = __builtin_amdgcn_readlane(i, r);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  v = bv;
  i = bi;
}

// Exchange records of the LU leaf.  Every 64-bit word carries 32 bits of
// payload (high half) and the sequence number of the column that wrote it
// (low half), so a reader polls the very word it needs: a word is valid
// once its sequence number matches, with no barrier or fence between
// writer and reader (single-copy atomicity of aligned 64-bit accesses at
// device scope).  Sequence numbers are unique within a factorization, and
// the record area is cleared before the factorization starts.
__device__ __forceinline__ void ll_put(uint64_t* p, uint32_t payload, uint32_t seq) {
  __hip_atomic_store(p, ((uint64_t)payload << 32) | seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ll_put2(uint64_t* p, double v, uint32_t seq) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  ll_put(p, (uint32_t)(u >> 32), seq);
  ll_put(p + 1, (uint32_t)u, seq);
}
// bounded poll of a word already loaded once: on expiry the error is
// recorded and whatever was read is used
__device__ __forceinline__ void ll_poll(const uint64_t* p, uint64_t& v, uint32_t seq, abft_report* rep) {
  long spins = 0;
  while ((uint32_t)v != seq) {
    __builtin_amdgcn_s_sleep(1);
    v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (++spins > (1L << 21)) {
      if (rep) atomicOr(&rep->status, (int)ABFT_ST_INTERNAL);
      break;
    }
  }
}
__device__ __forceinline__ double ll_dbl(uint64_t hi, uint64_t lo) {
  return __longlong_as_double((long long)((hi & 0xffffffff00000000ull) | (lo >> 32)));
}
// both words of a double: the two loads are issued before either is polled
__device__ __forceinline__ double ll_get2b(const uint64_t* p, uint32_t seq, abft_report* rep) {
  uint64_t hi = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint64_t lo = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  ll_poll(p, hi, seq, rep);
  ll_poll(p + 1, lo, seq, rep);
  return ll_dbl(hi, lo);
}
constexpr uint32_t LL_NONE = 0xffffffffu;  // no candidate row in this workgroup

// Records of one column: per workgroup 3 + 2w words (|pivot| candidate, its
// row index, its row), then the 2w words of row d.  Two columns' records
// alternate: a workgroup writes column j + 2 only after every workgroup has
// published column j + 1, which each does only after it has read everything
// of column j it needs.
__host__ __device__ constexpr int64_t lu_rec_words(int G, int w) { return (int64_t)G * (3 + 2 * w) + 2 * w; }

template <typename T>
__global__ __launch_bounds__(256) void k_getrf_leaf(T* A, int64_t lda, int64_t m, int64_t c0, int w, int R,
                                                    int32_t* ipiv, int32_t* info, uint64_t* recs, uint32_t seq0,
                                                    abft_report* rep) {
  extern __shared__ unsigned char smem_raw[];
  T* Ld = reinterpret_cast<T*>(smem_raw);  // R x (w+1)
  const int ldl = w + 1;
  __shared__ double prow[CLEAF], orow[CLEAF];
  __shared__ double wv_val[4];
  __shared__ int64_t wv_idx[4];
  __shared__ int64_t s_piv, s_loc;
  __shared__ int s_pg;
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t rbeg = c0 + (int64_t)g * R;
  const int rows = (int)max((int64_t)0, min((int64_t)R, m - rbeg));
  const int rw = 3 + 2 * w;
  const int64_t cstride = lu_rec_words(G, w);

  for (int idx = tid; idx < rows * w; idx += 256) {
    int i = idx % rows, j = idx / rows;
    Ld[i * ldl + j] = A[(rbeg + i) + (c0 + j) * lda];
  }
  __syncthreads();

  for (int j = 0; j < w; ++j) {
    const int64_t d = c0 + j;  // diagonal row (in workgroup 0: R >= w)
    const uint32_t seq = seq0 + (uint32_t)j;
    uint64_t* rj = recs + (size_t)(j & 1) * cstride;
    uint64_t* rowd = rj + (size_t)G * rw;
    // local argmax of |a(i, j)| over owned rows i >= d (row indices fit in
    // 32 bits: the exchange records carry them so)
    double bv = -1.0;
    int bi32 = INT_MAX;
    for (int i = tid; i < rows; i += 256) {
      const int gi = (int)(rbeg + i);
      if (gi < d) continue;
      const double v = fabs((double)Ld[i * ldl + j]);
      if (better<T>(v, gi, bv, bi32)) { bv = v; bi32 = gi; }
    }
    wave_argmax(bv, bi32);
    int64_t bi = bi32 == INT_MAX ? INT64_MAX : (int64_t)bi32;
    if (lane == 0) { wv_val[wv] = bv; wv_idx[wv] = bi; }
    __syncthreads();
    uint64_t* mine = rj + (size_t)g * rw;
    if (tid == 0) {
      for (int q = 1; q < 4; ++q)
        if (better<T>(wv_val[q], wv_idx[q], bv, bi)) { bv = wv_val[q]; bi = wv_idx[q]; }
      ll_put2(mine, bv, seq);
      ll_put(mine + 2, bi == INT64_MAX ? LL_NONE : (uint32_t)bi, seq);
      s_loc = bi;
    }
    __syncthreads();
    // candidate row (values of the leaf columns) and, from workgroup 0, row d
    if (tid < w) {
      const int64_t bl = s_loc;
      ll_put2(mine + 3 + 2 * tid, bl == INT64_MAX ? 0.0 : (double)Ld[(bl - rbeg) * ldl + tid], seq);
      if (g == 0) ll_put2(rowd + 2 * tid, (double)Ld[(d - rbeg) * ldl + tid], seq);
    }
    // every workgroup picks the same winner: one record per thread (its three
    // words loaded together), then a block argmax (largest |value|, first
    // row index on ties; the row index identifies its workgroup, so the
    // choice does not depend on the order)
    {
      double v = -1.0;
      int ii = INT_MAX;
      for (int q = tid; q < G; q += 256) {
        const uint64_t* rq = rj + (size_t)q * rw;
        uint64_t wd[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) wd[u] = __hip_atomic_load(rq + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int u = 0; u < 3; ++u) ll_poll(rq + u, wd[u], seq, rep);
        const double vq = ll_dbl(wd[0], wd[1]);
        const uint32_t iq32 = (uint32_t)(wd[2] >> 32);
        // a record that expired unwritten (ABFT_ST_INTERNAL already set) may
        // decode to any index: only rows [d, m) count as candidates
        const int iq = (iq32 == LL_NONE || (int64_t)iq32 < d || (int64_t)iq32 >= m) ? INT_MAX : (int)iq32;
        if (vq >= 0 && better<T>(vq, iq, v, ii)) { v = vq; ii = iq; }
      }
      wave_argmax(v, ii);
      if (lane == 0) { wv_val[wv] = v; wv_idx[wv] = ii == INT_MAX ? INT64_MAX : (int64_t)ii; }
      __syncthreads();
      if (tid == 0) {
        double best = wv_val[0];
        int64_t bidx = wv_idx[0];
        for (int q = 1; q < 4; ++q)
          if (better<T>(wv_val[q], wv_idx[q], best, bidx)) { best = wv_val[q]; bidx = wv_idx[q]; }
        // the winning row names its workgroup (rows [c0 + g R, c0 + (g+1) R))
        int bg = bidx == INT64_MAX ? 0 : (int)((bidx - c0) / R);
        if (bidx == INT64_MAX || bg < 0 || bg >= G) {  // (bounds kept on the degraded path too)
          bidx = d;
          bg = 0;
        }
        s_piv = bidx;
        s_pg = bg;
      }
      __syncthreads();
    }
    const int64_t p = s_piv;
    const int pg = s_pg;
    const bool own_p = p != d && p >= rbeg && p < rbeg + rows;
    if (tid < w) {
      prow[tid] = ll_get2b(rj + (size_t)pg * rw + 3 + 2 * tid, seq, rep);
      if (own_p) orow[tid] = ll_get2b(rowd + 2 * tid, seq, rep);
    }
    __syncthreads();
    if (p != d) {
      if (g == 0 && tid < w) Ld[(d - rbeg) * ldl + tid] = (T)prow[tid];
      if (own_p && tid < w) Ld[(p - rbeg) * ldl + tid] = (T)orow[tid];
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
}

// ---------------------------------------------------------------------------
// Cooperative Householder leaf: columns [c0, c0+w), rows [c0, m) (LAPACK
// dlarfg convention), plus the leaf's triangular factor T (forward,
// columnwise) written at T[toff + toff*ldt].
//
// Per column j every workgroup forms the partial Gram row
// S_c = sum over its rows i > d of a(i,j) a(i,c) for every c < w.  The G
// partial rows are added in two levels through self-validating exchange
// records (as in the LU leaf; no barrier, no fence): the first workgroup of
// each group of 8 (16 beyond 128 workgroups) adds its members' rows in
// member order and publishes the group sum, then every workgroup adds the
// group sums in group order, so all hold the same Gram row.  Entries c >= j give the column norm and the
// reflector's dot products with the trailing columns; entries c < j give
// v_c . v_j = v_c(d) + scale S_c, the inputs of T's column j, which
// workgroup 0 stages in T's strictly upper part.  After the loop workgroup
// 0 runs T's recurrence in LDS.  Records of two columns alternate: a
// workgroup rewrites column j's records only after it has read every group
// sum of column j + 1, which no group publishes before its members have
// finished column j.
// ---------------------------------------------------------------------------
// groups of 8 workgroups up to 128 workgroups, of 16 beyond: at most 16
// group sums, four per thread of the second level
__host__ __device__ constexpr int qr_group(int G) { return G <= 128 ? 8 : 16; }
__host__ __device__ constexpr int64_t qr_rec_words(int G, int w) {
  return (int64_t)(G + (G + qr_group(G) - 1) / qr_group(G) + 1) * 2 * w;
}

__global__ __launch_bounds__(256) void k_geqrf_leaf(double* A, int64_t lda, int64_t m, int64_t c0, int w, int R,
                                                    double* tau, double* Tm, int ldt, int toff, uint64_t* recs,
                                                    uint32_t seq0, abft_report* rep) {
  extern __shared__ unsigned char smem_raw[];
  double* Ld = reinterpret_cast<double*>(smem_raw);  // R x (w+1)
  const int ldl = w + 1;
  __shared__ double part[4][CLEAF];
  __shared__ double qpart[4][CLEAF], gpart[4][CLEAF];
  __shared__ double orow[CLEAF], fvec[CLEAF];
  __shared__ double s_beta, s_tau, s_scale;
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, e = tid & 63, wq = tid >> 6;
  const int grp = qr_group(G), NG = (G + grp - 1) / grp;
  const int64_t rbeg = c0 + (int64_t)g * R;
  const int rows = (int)max((int64_t)0, min((int64_t)R, m - rbeg));
  const int64_t cstride = qr_rec_words(G, w);

  for (int idx = tid; idx < rows * w; idx += 256) {
    int i = idx % rows, j = idx / rows;
    Ld[i * ldl + j] = A[(rbeg + i) + (c0 + j) * lda];
  }
  __syncthreads();

  // sum of up to four records (q0, q0 + 4, ... < q1) of 2w words at base:
  // entry e of this thread, all loads issued before any is polled
  auto sum4 = [&](const uint64_t* base, int q0, int q1, uint32_t seq) {
    double acc = 0.0;
    if (e < w) {
      uint64_t wd[8];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = q0 + 4 * k;
        if (q < q1) {
          const uint64_t* pr = base + (size_t)q * 2 * w + 2 * e;
          wd[2 * k] = __hip_atomic_load(pr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          wd[2 * k + 1] = __hip_atomic_load(pr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = q0 + 4 * k;
        if (q < q1) {
          const uint64_t* pr = base + (size_t)q * 2 * w + 2 * e;
          ll_poll(pr, wd[2 * k], seq, rep);
          ll_poll(pr + 1, wd[2 * k + 1], seq, rep);
          acc += ll_dbl(wd[2 * k], wd[2 * k + 1]);
        }
      }
    }
    return acc;
  };

  for (int j = 0; j < w; ++j) {
    const int64_t d = c0 + j;
    const uint32_t seq = seq0 + (uint32_t)j;
    uint64_t* r1 = recs + (size_t)(j & 1) * cstride;  // G partial rows
    uint64_t* r2 = r1 + (size_t)G * 2 * w;           // NG group sums
    uint64_t* rdw = r2 + (size_t)NG * 2 * w;         // row d
    // partial Gram row: thread (q, c) takes column c over the rows i = q
    // (mod 4) below d of the LDS panel, eight rows per step, loads first
    {
      const int c = e, q = wq;
      double acc = 0.0;
      if (c < w) {
        const int i0 = (int)max((int64_t)0, d + 1 - rbeg);
        int i = i0 + ((q - i0 % 4) + 4) % 4;
        for (; i + 28 < rows; i += 32) {
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
      part[q][c] = acc;
    }
    __syncthreads();
    if (tid < w) {
      ll_put2(r1 + (size_t)g * 2 * w + 2 * tid, ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid], seq);
      if (g == 0) ll_put2(rdw + 2 * tid, Ld[(d - rbeg) * ldl + tid], seq);
    }
    // level 1: the group's first workgroup adds its members' rows
    if (g % grp == 0) {
      qpart[wq][e] = sum4(r1, g + wq, min(G, g + grp), seq);
      __syncthreads();
      if (tid < w)
        ll_put2(r2 + (size_t)(g / grp) * 2 * w + 2 * tid,
                ((qpart[0][tid] + qpart[1][tid]) + qpart[2][tid]) + qpart[3][tid], seq);
    }
    // level 2: every workgroup adds the group sums (and reads row d)
    gpart[wq][e] = sum4(r2, wq, NG, seq);
    if (tid < w) orow[tid] = ll_get2b(rdw + 2 * tid, seq, rep);
    __syncthreads();
    double sv = 0.0;
    if (tid < w) sv = ((gpart[0][tid] + gpart[1][tid]) + gpart[2][tid]) + gpart[3][tid];
    if (tid < w) fvec[tid] = sv;  // the Gram row, for thread 0's reflector
    __syncthreads();
    if (tid == 0) {
      const double alpha = orow[j], s2 = fvec[j];
      if (s2 == 0.0) {
        s_tau = 0.0; s_scale = 0.0; s_beta = alpha;
      } else {
        const double beta = -copysign(sqrt(alpha * alpha + s2), alpha);
        s_tau = (beta - alpha) / beta;
        s_scale = 1.0 / (alpha - beta);
        s_beta = beta;
      }
      if (g == 0) tau[d] = s_tau;
    }
    __syncthreads();
    const double t = s_tau, sc = s_scale;
    if (g == 0 && tid < j)  // v_c . v_j for c < j, staged in T's strictly upper part
      Tm[(toff + tid) + (int64_t)(toff + j) * ldt] = orow[tid] + sc * sv;
    if (t != 0.0) {
      if (tid < w && tid > j) fvec[tid] = t * (orow[tid] + sc * sv);
      __syncthreads();
      for (int i = tid; i < rows; i += 256) {
        int64_t gi = rbeg + i;
        if (gi < d) continue;
        if (gi == d) {
          Ld[i * ldl + j] = s_beta;
          row_axpy(Ld + i * ldl, fvec, 1.0, j + 1, w);  // a(d,c) - f(c)
        } else {
          double v = Ld[i * ldl + j] * sc;
          Ld[i * ldl + j] = v;
          row_axpy(Ld + i * ldl, fvec, v, j + 1, w);  // a(i,c) - f(c) * v
        }
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < rows * w; idx += 256) {
    int i = idx % rows, j = idx / rows;
    A[(rbeg + i) + (c0 + j) * lda] = Ld[i * ldl + j];
  }
  if (g == 0) {
    // T from the staged dot products: T(0:j, j) = -tau_j T(0:j, 0:j) z_j
    __syncthreads();
    double* Gm = Ld;            // Gm[q * ldl + j] = v_q . v_j, q < j
    double* Tl = Ld + w * ldl;  // Tl[q * ldl + j]
    for (int e = tid; e < w * w; e += 256) {
      const int q = e % w, jj = e / w;
      Gm[q * ldl + jj] = q < jj ? Tm[(toff + q) + (int64_t)(toff + jj) * ldt] : 0.0;
      Tl[q * ldl + jj] = 0.0;
    }
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
}

// ---------------------------------------------------------------------------
// Row interchanges.  k_perm_build turns the interchanges ipiv[c0..c0+w) into
// the list of moved rows (dst <- src), sorted by dst.  k_laswp applies the
// moves to columns [j0, j1); with a column-checksum array it also adds, per
// tile-row, the change of the column sums and of the weighted column sums
// (compensated).
// ---------------------------------------------------------------------------
// Move list of the w row interchanges of a panel starting at row c0: after
// the swaps, row dst holds the original row src; moves = {count, dst0, src0,
// dst1, src1, ...} in increasing dst.  Only the panel's own rows [0, w) and
// the distinct pivot rows at or below w (relative to c0) can move, so the
// work is on a compact table of at most 2w slots: slot t < w is row t, slot
// w + f is the pivot row first named by interchange f.  The interchanges are
// resolved in parallel (no serial replay): see the chain rule below.
constexpr int PB_W = 512;  // largest panel width (block size)
__global__ __launch_bounds__(2 * PB_W) void k_perm_build(const int32_t* ipiv, int64_t c0, int w, int64_t n,
                                                        int* moves) {
  // (scans read four entries per LDS access)
  __shared__ __attribute__((aligned(16))) int pv[PB_W], sidx[PB_W], ptr[PB_W];
  __shared__ __attribute__((aligned(16))) int key[2 * PB_W], mflag[2 * PB_W];
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
  // table slot of each step's pivot row (b_t >= t), and the row each slot starts with
  if (tid < w) {
    const int p = pv[tid];
    int f = tid;
    if (p >= w) {
      int t = 0;
      for (; t + 4 <= tid; t += 4) {
        const int4 q = *reinterpret_cast<const int4*>(&pv[t]);
        if (q.x == p) { f = t; break; }
        if (q.y == p) { f = t + 1; break; }
        if (q.z == p) { f = t + 2; break; }
        if (q.w == p) { f = t + 3; break; }
      }
      if (f == tid)
        for (; t < tid; ++t)
          if (pv[t] == p) { f = t; break; }
    }
    sidx[tid] = p < w ? p : w + f;
    key[tid] = tid;
    key[w + tid] = (p >= w && f == tid) ? p : -1;
  }
  __syncthreads();
  // Step t swaps slots t and b_t, after which slot t never changes.  With
  // D(t) the row in slot t just before step t: D(t) = D(t') for the last
  // step t' < t with b_t' = t (it moved D(t') into slot t), else row t; so
  // D(t) is the root of the chain t -> t'.  Slot t ends with D(t) when
  // b_t = t, else with what slot b_t held before step t: D(t*) for the last
  // step t* < t with b_t* = b_t, else that slot's first row; an outer slot
  // ends with D of the last step that names it, else its own row.
  int ts = -1, tl = -1;
  if (tid < w) {
    const int b = sidx[tid];
    int pr = -1, t2 = 0;
    for (; t2 + 4 <= tid; t2 += 4) {
      const int4 q = *reinterpret_cast<const int4*>(&sidx[t2]);
      pr = q.w == tid ? t2 + 3 : (q.z == tid ? t2 + 2 : (q.y == tid ? t2 + 1 : (q.x == tid ? t2 : pr)));
      ts = q.w == b ? t2 + 3 : (q.z == b ? t2 + 2 : (q.y == b ? t2 + 1 : (q.x == b ? t2 : ts)));
    }
    for (; t2 < tid; ++t2) {
      const int s2 = sidx[t2];
      if (s2 == tid) pr = t2;
      if (s2 == b) ts = t2;
    }
    ptr[tid] = pr >= 0 ? pr : tid;
  } else if (tid < 2 * w) {
    int t = 0;
    for (; t + 4 <= w; t += 4) {
      const int4 q = *reinterpret_cast<const int4*>(&sidx[t]);
      tl = q.w == tid ? t + 3 : (q.z == tid ? t + 2 : (q.y == tid ? t + 1 : (q.x == tid ? t : tl)));
    }
    for (; t < w; ++t)
      if (sidx[t] == tid) tl = t;
  }
  __syncthreads();
  for (int r = 0; r < 10; ++r) {  // pointer jumping: chains are shorter than 2^10 > PB_W
    const int nxt = tid < w ? ptr[ptr[tid]] : 0;
    __syncthreads();
    if (tid < w) ptr[tid] = nxt;
    __syncthreads();
  }
  int fin = -1;
  if (tid < w) {
    const int b = sidx[tid];
    fin = b == tid ? ptr[tid] : (ts >= 0 ? ptr[ts] : key[b]);
  } else if (tid < 2 * w) {
    fin = tl >= 0 ? ptr[tl] : key[tid];
  }
  const int moved = tid < 2 * w && key[tid] >= 0 && fin != key[tid];
  mflag[tid] = moved;
  if (moved) atomicAdd(&nmoved, 1);
  __syncthreads();
  // rank by destination row: the panel's own rows (slots < w, in order)
  // come before the outer pivot rows
  if (moved) {
    int r = 0;
    const int lim = tid < w ? tid : w;  // moved panel rows before this one
    int q = 0;
    for (; q + 4 <= lim; q += 4) {
      const int4 f4 = *reinterpret_cast<const int4*>(&mflag[q]);
      r += f4.x + f4.y + f4.z + f4.w;
    }
    for (; q < lim; ++q) r += mflag[q];
    if (tid >= w) {  // and the moved outer rows with a smaller row index
      const int kx = key[tid];
      q = w;
      for (; q < 2 * w && (q & 3); ++q) r += (mflag[q] && key[q] < kx);
      for (; q + 4 <= 2 * w; q += 4) {
        const int4 f4 = *reinterpret_cast<const int4*>(&mflag[q]);
        const int4 k4 = *reinterpret_cast<const int4*>(&key[q]);
        r += (f4.x && k4.x < kx) + (f4.y && k4.y < kx) + (f4.z && k4.z < kx) + (f4.w && k4.w < kx);
      }
      for (; q < 2 * w; ++q) r += (mflag[q] && key[q] < kx);
    }
    moves[1 + 2 * r] = (int)(c0 + key[tid]);
    moves[2 + 2 * r] = (int)(c0 + fin);
  }
  if (tid == 0) moves[0] = nmoved;
}

// Row interchanges on columns [j0, j1), in one kernel with no staging in
// HBM: a workgroup takes cpw consecutive columns and every move of each;
// pair (move t, column c) goes to thread (t + nm c) mod 256, so the lanes of
// a wave touch consecutive moves of one column (the panel's own rows are
// contiguous).  Every value is loaded into registers before the workgroup
// barrier and stored after it, so cycles of moves need no ordering.  With a
// column-checksum array, the new and old values of the moved elements go to
// LDS and, per column, the thread at the start of each run of moves into one
// tile-row adds the run's plain and position-weighted differences
// (compensated, in the moves' order: increasing destination row) to that
// tile-row's column checksums.
constexpr int LASWP_PAIRS = 8;                       // (move, column) pairs per thread
constexpr int LASWP_CPW = 256 * LASWP_PAIRS / 1024;  // columns per workgroup (up to 1024 moves)
constexpr int LASWP_NBK = 1024 / 16;                 // blocks of 16 moves per column
template <typename T>
__global__ __launch_bounds__(256) void k_laswp(T* __restrict__ A, int64_t lda, int64_t j0, int64_t j1,
                                               const int* __restrict__ moves, double* __restrict__ colchk,
                                               int64_t ldc, int nb, int cpw) {
  extern __shared__ double dl[];  // with colchk: new values [ncol][nm], then old values [ncol][nm]
  __shared__ int mv[4 * PB_W];
  const int nm = moves[0];
  for (int t = threadIdx.x; t < 2 * nm; t += blockDim.x) mv[t] = moves[1 + t];
  __syncthreads();
  const int64_t cb = j0 + (int64_t)blockIdx.x * cpw;
  const int ncol = (int)min((int64_t)cpw, j1 - cb);
  const int np = nm * ncol;
  T vs[LASWP_PAIRS], vd[LASWP_PAIRS];
#pragma unroll
  for (int k = 0; k < LASWP_PAIRS; ++k) {
    const int p = threadIdx.x + 256 * k;
    if (p < np) {
      const int t = p % nm, c = p / nm;
      const T* col = A + (cb + c) * lda;
      vs[k] = col[mv[2 * t + 1]];
      if (colchk) vd[k] = col[mv[2 * t]];
    }
  }
  __syncthreads();  // every value of the workgroup's columns is loaded before any is written
#pragma unroll
  for (int k = 0; k < LASWP_PAIRS; ++k) {
    const int p = threadIdx.x + 256 * k;
    if (p < np) {
      const int t = p % nm, c = p / nm;
      A[(cb + c) * lda + mv[2 * t]] = vs[k];
      if (colchk) {
        dl[c * nm + t] = (double)vs[k];
        dl[(ncol + c) * nm + t] = (double)vd[k];
      }
    }
  }
  if (!colchk) return;
  __syncthreads();
  // Checksum fix-up.  The moves of a column are cut into blocks of 16; one
  // thread per (column, block) sums each piece of a run (the moves into one
  // tile-row) that lies in its block.  A run inside one block updates the
  // checksums directly; the pieces of a run that crosses blocks are merged
  // in block order by the thread of the block where the run starts.
  __shared__ acc2 hd[LASWP_CPW][LASWP_NBK][2], tl[LASWP_CPW][LASWP_NBK][2];
  const int nbk = (nm + 15) / 16;
  auto tile_of = [&](int t) { return mv[2 * t] / nb; };
  auto fix = [&](int c, int I, const acc2& e, const acc2& ww) {
    const int64_t j = cb + c;
    acc2 c0{colchk[2 * I + j * ldc], 0}, c1{colchk[2 * I + 1 + j * ldc], 0};
    cmerge(c0, e);
    cmerge(c1, ww);
    colchk[2 * I + j * ldc] = cval(c0);
    colchk[2 * I + 1 + j * ldc] = cval(c1);
  };
  for (int p = threadIdx.x; p < ncol * nbk; p += blockDim.x) {
    const int c = p / nbk, b = p % nbk, t0 = 16 * b, t1 = min(nm, t0 + 16);
    for (int t = t0; t < t1;) {
      const int I = tile_of(t);
      const bool from_before = t == t0 && t0 > 0 && tile_of(t0 - 1) == I;  // run begun in an earlier block
      acc2 e{0, 0}, ww{0, 0};
      int u = t;
      for (; u < t1 && tile_of(u) == I; ++u) {
        const double wr = (double)(mv[2 * u] - I * nb + 1), vn = dl[c * nm + u], vo = dl[(ncol + c) * nm + u];
        cadd(e, vn);
        cadd(e, -vo);
        cfma(ww, wr, vn);
        cfma(ww, -wr, vo);
      }
      const bool ends_here = u < t1 || t1 == nm || tile_of(t1) != I;
      if (!from_before && ends_here) {
        fix(c, I, e, ww);  // the whole run
      } else if (from_before) {
        hd[c][b][0] = e;  // head or middle piece of a run begun earlier
        hd[c][b][1] = ww;
      } else {
        tl[c][b][0] = e;  // first piece of a run that continues
        tl[c][b][1] = ww;
      }
      t = u;
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < ncol * nbk; p += blockDim.x) {
    const int c = p / nbk, b = p % nbk, t0 = 16 * b, t1 = min(nm, t0 + 16);
    const int I = tile_of(t1 - 1);
    const bool continues = t1 < nm && tile_of(t1) == I;
    const bool began_before = tile_of(t0) == I && t0 > 0 && tile_of(t0 - 1) == I;
    if (!continues || began_before) continue;  // this block does not hold the start of a crossing run
    acc2 e = tl[c][b][0], ww = tl[c][b][1];
    for (int bb = b + 1; bb < nbk; ++bb) {
      cmerge(e, hd[c][bb][0]);
      cmerge(ww, hd[c][bb][1]);
      const int u1 = min(nm, 16 * bb + 16);
      if (u1 == nm || tile_of(u1) != I) break;
    }
    fix(c, I, e, ww);
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
int trsm_llu_blk(hipStream_t s, T* A, int64_t lda, int64_t c0, int w, int64_t j0, int64_t j1) {
  if (j1 <= j0 || w <= 0) return 0;
  if (w > PB_W) return ABFT_ERR_UNSUPPORTED;
  const size_t shm = (size_t)((w + LEAF - 1) / LEAF * LEAF + 1) * TRS_CB * sizeof(T);
  hipLaunchKernelGGL(k_trsm_llu_blk<T>, dim3((unsigned)((j1 - j0 + TRS_CB - 1) / TRS_CB)), dim3(256), shm, s, A, lda, c0,
                     w, j0, j1);
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
  (void)ctr;
  int G, R;
  const int max_rows = (int)((144 * 1024) / ((w + 1) * sizeof(T)));
  coop_shape(m - c0, w, maxg, max_rows, G, R);
  if ((int64_t)G * R < m - c0) return ABFT_ERR_UNSUPPORTED;
  if (w > CLEAF || (size_t)(2 * lu_rec_words(G, w)) > SLOT_WORDS) return ABFT_ERR_UNSUPPORTED;
  size_t shm = (size_t)R * (w + 1) * sizeof(T);
  uint64_t* recs = reinterpret_cast<uint64_t*>(slots);
  uint32_t seq0 = *ctr_base + 1;
  void* args[] = {&A, &lda, &m, &c0, &w, &R, &ipiv, &info, &recs, &seq0, &rep};
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_getrf_leaf<T>, dim3(G), dim3(256), args, shm, s);
  *ctr_base += (unsigned)w;
  return e == hipSuccess ? 0 : ABFT_ERR_HIP;
}

int geqrf_leaf(hipStream_t s, double* A, int64_t lda, int64_t m, int64_t c0, int w, double* tau, double* Tm, int ldt,
               int toff, double* slots, unsigned* ctr, unsigned* ctr_base, abft_report* rep, int maxg) {
  (void)ctr;
  int G, R;
  const int max_rows = (int)((140 * 1024) / ((w + 1) * sizeof(double)));
  coop_shape(m - c0, w, maxg, max_rows, G, R);
  if ((int64_t)G * R < m - c0) return ABFT_ERR_UNSUPPORTED;
  if (w > CLEAF || G > 256 || (size_t)(2 * qr_rec_words(G, w)) > SLOT_WORDS) return ABFT_ERR_UNSUPPORTED;
  size_t shm = (size_t)R * (w + 1) * sizeof(double);
  uint64_t* recs = reinterpret_cast<uint64_t*>(slots);
  uint32_t seq0 = *ctr_base + 1;
  void* args[] = {&A, &lda, &m, &c0, &w, &R, &tau, &Tm, &ldt, &toff, &recs, &seq0, &rep};
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_geqrf_leaf, dim3(G), dim3(256), args, shm, s);
  *ctr_base += (unsigned)w;
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
  (void)stage;
  if (j1 <= j0) return 0;
  // the move count is on the device: size for the largest list (2 x panel
  // width) unless the range is narrow
  const int nmax = 2 * PB_W;
  const int cpw = LASWP_CPW;
  const size_t shm = colchk ? (size_t)2 * cpw * nmax * sizeof(double) : 0;
  hipLaunchKernelGGL(k_laswp<T>, dim3((unsigned)((j1 - j0 + cpw - 1) / cpw)), dim3(256), shm, s, A, lda, j0, j1, moves,
                     colchk, ldc, nb, cpw);
  CHECK_LAUNCH();
}

template int potrf_leaf<double>(hipStream_t, double*, int64_t, int64_t, int, int32_t*);
template int potrf_leaf<float>(hipStream_t, float*, int64_t, int64_t, int, int32_t*);
template int trsm_rlt_leaf<double>(hipStream_t, double*, int64_t, int64_t, int64_t, int64_t, int);
template int trsm_rlt_leaf<float>(hipStream_t, float*, int64_t, int64_t, int64_t, int64_t, int);
template int trsm_llu_leaf<double>(hipStream_t, double*, int64_t, int64_t, int, int64_t, int64_t);
template int trsm_llu_blk<double>(hipStream_t, double*, int64_t, int64_t, int, int64_t, int64_t);
template int trsm_llu_blk<float>(hipStream_t, float*, int64_t, int64_t, int, int64_t, int64_t);
template int trsm_llu_leaf<float>(hipStream_t, float*, int64_t, int64_t, int, int64_t, int64_t);
template int getrf_leaf<double>(hipStream_t, double*, int64_t, int64_t, int64_t, int, int32_t*, int32_t*, double*,
                                unsigned*, unsigned*, abft_report*, int);
template int getrf_leaf<float>(hipStream_t, float*, int64_t, int64_t, int64_t, int, int32_t*, int32_t*, double*,
                               unsigned*, unsigned*, abft_report*, int);
template int laswp<double>(hipStream_t, double*, int64_t, int64_t, int64_t, const int*, double*, double*, int64_t, int);
template int laswp<float>(hipStream_t, float*, int64_t, int64_t, int64_t, const int*, float*, double*, int64_t, int);

}  // namespace abft
