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
constexpr int BMAXFL = BN * (BN + 1) / 2;  // most trailing tiles of one step (lower part)

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

// LDS writes of one wave made visible to its other lanes
__device__ __forceinline__ void wave_sync_b() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ T fms_b(T a, T b, T c) {
  return a - b * c;
}
template <>
__device__ __forceinline__ float fms_b<float>(float a, float b, float c) {
  return __fmaf_rn(-b, c, a);
}

typedef double bf64x4 __attribute__((ext_vector_type(4)));
typedef float bf32x4 __attribute__((ext_vector_type(4)));

// A small FP64 product on the matrix cores, D (R x C) = sum_k a(r, k) b(k, c)
// for k < K, with its magnitude twin Dm = sum_k |a|(r, k) |b|(k, c): 16 x 16
// output tiles dealt to the workgroup's four waves, K in steps of 4
// (v_mfma_f64_16x16x4).  fa(r, k, v, vm) / fb(k, c, v, vm) return an operand
// and its magnitude-side value (0 outside the bounds); epi(r, c, d, dm)
// consumes each output inside R x C.
template <typename FA, typename FB, typename EPI>
__device__ void small_mma(int R, int C, int K, FA fa, FB fb, EPI epi) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, il = lane & 15, kl = lane >> 4;
  const int tr = (R + 15) / 16, tc = (C + 15) / 16;
  for (int t = wv; t < tr * tc; t += 4) {
    const int r0 = (t % tr) * 16, q0 = (t / tr) * 16;
    bf64x4 acc{0, 0, 0, 0}, accm{0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      double a, am, b, bm;
      fa(r0 + il, k0 + kl, a, am);
      fb(k0 + kl, q0 + il, b, bm);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      accm = __builtin_amdgcn_mfma_f64_16x16x4f64(am, bm, accm, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = r0 + 4 * r + kl, j = q0 + il;  // D[i][j]: lane j + 16 (i % 4), register i / 4
      if (i < R && j < C) epi(i, j, acc[r], accm[r]);
    }
  }
}

// checksum carry of the batched trailing update  A22 -= X Y  over tile-rows
// and tile-columns > k: X rows (i >= c1) from the LDS panel P (row i - c0),
// Y(p, j) from ymat (LU: U12 in A; Cholesky: the transpose of X).  The
// per-tile-row sums of X (S, Sa), and for LU the per-tile-column sums of
// U12 (Tm, Ta), are formed in the LDS block sl (2 x 2 BN x BNB doubles,
// compensated, in index order); the carries themselves are the products
// colchk -= S Y, gc = Sa |Y| and rowchk -= X T, gr = |X| Ta (T = S for
// Cholesky's symmetric update) on the matrix cores, as in the blocked path.
template <typename T, int CHOL>
__device__ void batch_carry(const T* A, int64_t lda, int n, int k, int w, const T* P, int ldp, const BatchChk& c,
                            double* sl) {
  const int N = (n + BNB - 1) / BNB;
  const int c0 = k * BNB, c1 = c0 + w, m = n - c1;
  const int ldc = 2 * BN;
  const int M = N - k - 1, R = 2 * M;  // checksum rows (columns) of the trailing tile-rows (tile-columns)
  double* Sl = sl;                 // [2I + e][p]
  double* Sal = sl + 2 * BN * BNB;  // magnitudes
  // S: sums of X over each tile-row I > k (compensated); Sa: |.|-sums
  for (int e = threadIdx.x; e < M * BNB; e += blockDim.x) {
    const int I = k + 1 + e / BNB, p = e % BNB;
    acc2 se{0, 0}, sw{0, 0};
    double sa = 0, swa = 0;
    if (p < w)
      for (int i = I * BNB; i < min(n, (I + 1) * BNB); ++i) {
        const double v = (double)P[(i - c0) * ldp + p], wi = (double)(i - I * BNB + 1);
        cadd(se, v);
        cfma(sw, wi, v);
        sa += fabs(v);
        swa += wi * fabs(v);
      }
    Sl[(2 * I) * BNB + p] = cval(se);
    Sl[(2 * I + 1) * BNB + p] = cval(sw);
    Sal[(2 * I) * BNB + p] = sa;
    Sal[(2 * I + 1) * BNB + p] = swa;
  }
  __syncthreads();
  const int q0 = 2 * (k + 1);  // first checksum row (column) of the trailing tiles
  // column side: colchk(2I+e, j) -= S(2I+e, :) y(:, j);  gc = Sa |y|
  small_mma(
      R, m, w,
      [&](int r, int p, double& v, double& vm) {
        const bool in = r < R && p < w;
        v = in ? Sl[(q0 + r) * BNB + p] : 0.0;
        vm = in ? Sal[(q0 + r) * BNB + p] : 0.0;
      },
      [&](int p, int jj, double& v, double& vm) {
        double y = 0.0;
        if (p < w && jj < m)
          y = CHOL ? (double)P[(c1 + jj - c0) * ldp + p] : (double)A[(c0 + p) + (int64_t)(c1 + jj) * lda];
        v = y;
        vm = fabs(y);
      },
      [&](int r, int jj, double d, double dm) {
        const int I = k + 1 + r / 2, j = c1 + jj;
        if (CHOL && I < j / BNB) return;  // (lower tiles only)
        double* ce = &c.colchk[(q0 + r) + (int64_t)j * ldc];
        *ce = *ce - d;
        c.gc[(q0 + r) + (int64_t)j * ldc] = dm;
      });
  __syncthreads();
  if (!CHOL) {
    // Tm: row sums of U12 over each tile-column J > k (the S block is free now)
    for (int e = threadIdx.x; e < M * BNB; e += blockDim.x) {
      const int J = k + 1 + e / BNB, p = e % BNB;
      acc2 se{0, 0}, sw{0, 0};
      double sa = 0, swa = 0;
      if (p < w) {
        const int j0 = J * BNB, jn = min(n, j0 + BNB) - j0;
        for (int t = 0; t < jn; ++t) {
          const double u = (double)A[(c0 + p) + (int64_t)(j0 + t) * lda], wj = (double)(t + 1);
          cadd(se, u);
          cfma(sw, wj, u);
          sa += fabs(u);
          swa += wj * fabs(u);
        }
      }
      Sl[(2 * J) * BNB + p] = cval(se);
      Sl[(2 * J + 1) * BNB + p] = cval(sw);
      Sal[(2 * J) * BNB + p] = sa;
      Sal[(2 * J + 1) * BNB + p] = swa;
    }
    __syncthreads();
  }
  // row side: rowchk(i, 2J+e) -= x(i, :) t(:, 2J+e);  gr = |x| t_abs
  // (t = S for Cholesky: the symmetric update, t = Tm for LU)
  small_mma(
      m, R, w,
      [&](int ii, int p, double& v, double& vm) {
        const double x = (ii < m && p < w) ? (double)P[(c1 + ii - c0) * ldp + p] : 0.0;
        v = x;
        vm = fabs(x);
      },
      [&](int p, int q, double& v, double& vm) {
        const bool in = p < w && q < R;
        v = in ? Sl[(q0 + q) * BNB + p] : 0.0;
        vm = in ? Sal[(q0 + q) * BNB + p] : 0.0;
      },
      [&](int ii, int q, double d, double dm) {
        const int i = c1 + ii, J = k + 1 + q / 2;
        if (CHOL && J > i / BNB) return;
        double* re = &c.rowchk[i + (int64_t)(q0 + q) * BMAX];
        *re = *re - d;
        c.gr[i + (int64_t)(q0 + q) * BMAX] = dm;
      });
  __syncthreads();
}

// trailing update A[c1:n, c1:n] -= X Y, X = rows of the LDS panel below the
// diagonal block, Y = U12 (staged chunk by chunk) or X^T (Cholesky, lower
// part only), on the matrix cores: per 64 x 64 output block each of the four
// waves computes a 32 x 32 quadrant as 2 x 2 tiles of 16 x 16 MFMA products
// over K = w in steps of 4 (binary64: v_mfma_f64_16x16x4, binary32:
// v_mfma_f32_16x16x4).  The operand roles are swapped (the MFMA's first
// operand is the Y side) so that the product is the transposed block and a
// register holds one column of it: sixteen lanes then read and write sixteen
// consecutive rows.  The block's C values are read before its products.
template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  typedef bf64x4 V;
  __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // column (within the 16-wide tile) of register r in lane group kl
  __device__ static int col(int r, int kl) { return 4 * r + kl; }
};
template <>
struct MfmaAcc<float> {
  typedef bf32x4 V;
  __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int col(int r, int kl) { return 4 * kl + r; }
};

template <typename T, int CHOL>
__device__ void batch_tmu(T* A, int64_t lda, int n, int c0, int w, const T* P, int ldp, T* Uc) {
  typedef MfmaAcc<T> M;
  const int c1 = c0 + w, m = n - c1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wm = wv & 1, wn = wv >> 1;
  const int il = lane & 15, kl = lane >> 4;
  auto inside = [&](int i, int jj) { return i < m && jj < m && (!CHOL || i >= jj); };
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
      const int r0 = ib + wm * 32, q0 = jb + wn * 32;  // this wave's quadrant (rows, columns of the trailing matrix)
      if (CHOL && r0 + 31 < q0) continue;            // strictly above the diagonal
      T cv[2][2][4];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = r0 + 16 * a + il, jj = q0 + 16 * b + M::col(r, kl);
            cv[b][a][r] = inside(i, jj) ? A[(c1 + i) + (int64_t)(c1 + jj) * lda] : (T)0;
          }
      typename M::V acc[2][2];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[b][a] = typename M::V{0, 0, 0, 0};
      for (int k0 = 0; k0 < w; k0 += 4) {
        const int k = k0 + kl;
        T xf[2], yf[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int i = r0 + 16 * a + il;
          xf[a] = (k < w && i < m) ? P[(w + i) * ldp + k] : (T)0;
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int jj = q0 + 16 * b + il;
          if (CHOL) yf[b] = (k < w && jj < m) ? P[(w + jj) * ldp + k] : (T)0;
          else yf[b] = k < w ? Uc[k * 65 + (jj - jb)] : (T)0;
        }
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int a = 0; a < 2; ++a) acc[b][a] = M::mma(yf[b], xf[a], acc[b][a]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = r0 + 16 * a + il, jj = q0 + 16 * b + M::col(r, kl);
            if (inside(i, jj)) A[(c1 + i) + (int64_t)(c1 + jj) * lda] = cv[b][a][r] - (T)acc[b][a][r];
          }
    }
  }
  __syncthreads();
}

// One wave checks one tile (h x w <= 32 x 32): the tile goes to a
// wave-private LDS block (padded, conflict-free both ways), then lane j < 32
// sums column j and lane 32 + i sums row i, both in index order with
// compensated plain and position-weighted sums and plain magnitudes.
// mode 0: store the sums as the tile's checksums (encode).  mode 1: compare
// with the carried checksums (thresholds from the magnitudes and the carried
// magnitude bounds); a clean tile's checksums are refreshed from the sums.
// Returns the number of flagged sums; *maxr gets the largest |d|/tau of the
// clean comparisons.  (frow, fcol): an element planted by a fault plan in
// this iteration (-1: none); the |d| and tau of the plain column checksum
// that covers it go to rep.
template <typename T>
__device__ int wave_tile32(const T* A, int64_t lda, int I, int J, int h, int w, bool sym, int mode, double* colchk,
                           int ldc, double* rowchk, int ldr, const double* gc, const double* gr, double tsu,
                           double* lds, double* maxr, int64_t frow = -1, int64_t fcol = -1,
                           abft_report* rep = nullptr) {
  const int lane = threadIdx.x & 63;
  const int64_t r0 = (int64_t)I * BNB, c0 = (int64_t)J * BNB;
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = lane + 64 * q, i = e & 31, j = e >> 5;
    double x = 0.0;
    if (i < h && j < w) x = (sym && i < j) ? (double)A[(r0 + j) + (c0 + i) * lda] : (double)A[(r0 + i) + (c0 + j) * lda];
    v[q] = x;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = lane + 64 * q;
    lds[(e & 31) + 33 * (e >> 5)] = v[q];
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const bool col = lane < 32;
  const int x = lane & 31;  // column (col) or row index
  acc2 se{0, 0}, sw{0, 0};
  double sa = 0.0, swa = 0.0;
  for (int t = 0; t < 32; ++t) {
    const double val = col ? lds[t + 33 * x] : lds[x + 33 * t], wt = (double)(t + 1), av = fabs(val);
    cadd(se, val);
    cfma(sw, wt, val);
    sa += av;
    swa += wt * av;
  }
  __builtin_amdgcn_wave_barrier();
  const bool live = col ? x < w : x < h;
  double* pe = col ? &colchk[2 * I + (c0 + x) * ldc] : &rowchk[(r0 + x) + (2 * J) * ldr];
  double* pw = col ? pe + 1 : pe + ldr;
  const double e = cval(se), ww = cval(sw);
  if (mode == 0) {
    if (live) { *pe = e; *pw = ww; }
    return 0;
  }
  int nfl = 0;
  double mr = 0.0;
  if (live) {
    const double ge = col ? (gc ? gc[2 * I + (c0 + x) * ldc] : 0.0) : (gr ? gr[(r0 + x) + (2 * J) * ldr] : 0.0);
    const double gw = col ? (gc ? gc[2 * I + 1 + (c0 + x) * ldc] : 0.0) : (gr ? gr[(r0 + x) + (2 * J + 1) * ldr] : 0.0);
    const double de = e - *pe, dw = ww - *pw;
    const double te = tau_verify(tsu, sa, ge), tw = tau_verify(tsu, swa, gw);
    const bool be = bad(de, te), bw = bad(dw, tw);
    nfl = be + bw;
    if (!be && te > 0) mr = fmax(mr, fabs(de) / te);
    if (!bw && tw > 0) mr = fmax(mr, fabs(dw) / tw);
    if (rep && col && c0 + x == fcol && frow >= r0 && frow < r0 + h) {
      rep->fault_d = fabs(de);
      rep->fault_tau = te;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    nfl += __shfl_xor(nfl, o);
    mr = fmax(mr, __shfl_xor(mr, o));
  }
  if (nfl == 0 && live) { *pe = e; *pw = ww; }
  *maxr = mr;
  return nfl;
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
  __shared__ int s_nflag;
  __shared__ int s_flagged[BMAXFL];
  __shared__ int64_t s_frow, s_fcol;  // element planted in this iteration (-1: none)
  if (tid == 0) {
    rep->flagged_tiles = rep->corrected = rep->checksum_repaired = rep->uncorrectable = rep->panel_flags = 0;
    rep->first_flag_iter = 0x7fffffff;
    rep->status = 0;
    rep->max_ratio = 0.0;
    rep->nev = 0;
    rep->fault_delta = 0.0;
    rep->fault_d = rep->fault_tau = -1.0;
    *info = 0;
    s_fail = 0;
  }
  __syncthreads();
  double* wlds = reinterpret_cast<double*>(smem) + (tid >> 6) * (BNB * (BNB + 1));  // this wave's tile block
  if (protect) {
    // encode: one tile per wave
    const int nt = CHOL ? N * (N + 1) / 2 : N * N;
    for (int t = tid >> 6; t < nt; t += 4) {
      int I, J;
      if (CHOL) {  // lower tiles, column by column
        J = 0;
        int r = t;
        while (r >= N - J) { r -= N - J; ++J; }
        I = J + r;
      } else {
        I = t % N;
        J = t / N;
      }
      double mr;
      wave_tile32(A, lda, I, J, min(BNB, n - I * BNB), min(BNB, n - J * BNB), CHOL && I == J, 0, c.colchk, ldc,
                  c.rowchk, BMAX, nullptr, nullptr, 0.0, wlds, &mr);
    }
    __syncthreads();
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
      // diagonal block, right-looking, by wave 0 alone (no workgroup barriers)
      if (tid < 64) {
        for (int j = 0; j < w; ++j) {
          if (tid == 0) {
            T d = P[j * ldp + j];
            if (!(d > (T)0) && !s_fail) {
              s_fail = 1;
              *info = c0 + j + 1;
            }
            P[j * ldp + j] = sqrt(d);
          }
          wave_sync_b();
          for (int i = j + 1 + tid; i < w; i += 64) P[i * ldp + j] = P[i * ldp + j] / P[j * ldp + j];
          wave_sync_b();
          const int r = w - j - 1;
          for (int e = tid; e < r * r; e += 64) {
            int i = j + 1 + e % r, jj = j + 1 + e / r;
            if (i >= jj) P[i * ldp + jj] = fms_b(P[i * ldp + jj], P[i * ldp + j], P[jj * ldp + j]);
          }
          wave_sync_b();
        }
      }
      __syncthreads();
      // rows below: x L^T = a, one thread per row, the row in registers
      // (same operation order as the plain substitution)
      for (int i = w + tid; i < mrows; i += blockDim.x) {
        T x[BNB];
#pragma unroll
        for (int j = 0; j < BNB; ++j) x[j] = j < w ? P[i * ldp + j] : (T)0;
#pragma unroll
        for (int j = 0; j < BNB; ++j) {
          if (j < w) {
            T sacc = x[j];
#pragma unroll
            for (int p = 0; p < j; ++p) sacc = fms_b(sacc, x[p], P[j * ldp + p]);
            x[j] = sacc / P[j * ldp + j];
          }
        }
#pragma unroll
        for (int j = 0; j < BNB; ++j)
          if (j < w) P[i * ldp + j] = x[j];
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
      // interchanges outside the panel: every thread applies all of them, in
      // order, to its own columns (checksums follow the rows), so no barrier
      // is needed between them; the changes of tile-row k (every row r of the
      // panel lies in it) are gathered in registers
      for (int col = tid; col < n; col += blockDim.x) {
        if (col >= c0 && col < c1) continue;
        T* colp = A + (int64_t)col * lda;
        const bool chk = protect && col >= c1;
        double dk = 0.0, dkw = 0.0;
        for (int j = 0; j < w; ++j) {
          const int r = c0 + j, q = c0 + swp[j];
          if (q == r) continue;
          const T ar = colp[r], aq = colp[q];
          if (chk) {
            const int Iq = q / BNB;
            const double d = (double)aq - (double)ar, wr = (double)(j + 1), wq = (double)(q - Iq * BNB + 1);
            dk += d;
            dkw += wr * d;
            c.colchk[2 * Iq + (int64_t)col * ldc] -= d;
            c.colchk[2 * Iq + 1 + (int64_t)col * ldc] -= wq * d;
          }
          colp[r] = aq;
          colp[q] = ar;
        }
        if (chk) {
          c.colchk[2 * k + (int64_t)col * ldc] += dk;
          c.colchk[2 * k + 1 + (int64_t)col * ldc] += dkw;
        }
      }
      if (protect)
        for (int cc = tid; cc < 2 * N; cc += blockDim.x)
          for (int j = 0; j < w; ++j) {
            const int r = c0 + j, q = c0 + swp[j];
            if (q == r) continue;
            const double t = c.rowchk[r + (int64_t)cc * BMAX];
            c.rowchk[r + (int64_t)cc * BMAX] = c.rowchk[q + (int64_t)cc * BMAX];
            c.rowchk[q + (int64_t)cc * BMAX] = t;
          }
      __syncthreads();
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
    if (protect) batch_carry<T, CHOL>(A, lda, n, k, w, P, ldp, c, reinterpret_cast<double*>(Uc));
    // ---- planned faults of this matrix and iteration (the last one planted
    // is recorded: |new - old|, +Inf when either is not finite)
    if (tid == 0) {
      s_frow = s_fcol = -1;
      for (int f = 0; f < nfaults; ++f) {
        const abft_fault& F = faults[f];
        if (F.matrix != mi || F.iter != k || F.row < 0 || F.row >= n || F.col < 0 || F.col >= n) continue;
        T* p = A + F.row + (int64_t)F.col * lda;
        const double before = (double)*p;
        if (sizeof(T) == 8) {
          unsigned long long u = (unsigned long long)__double_as_longlong((double)*p) ^ (1ull << (F.bit & 63));
          *p = (T)__longlong_as_double((long long)u);
        } else {
          unsigned u = __float_as_uint((float)*p) ^ (1u << (F.bit & 31));
          *p = (T)__uint_as_float(u);
        }
        const double d = fabs((double)*p - before);
        rep->fault_delta = (d <= 1.79e308) ? d : __builtin_inf();
        s_frow = F.row;
        s_fcol = F.col;
      }
    }
    __syncthreads();
    // ---- verify (and correct) the trailing tiles
    if (protect) {
      // one trailing tile per wave; flagged tiles are listed and corrected
      // afterwards by the whole workgroup, in tile order
      const int M = N - k - 1;
      const int nt = CHOL ? M * (M + 1) / 2 : M * M;
      if (tid == 0) s_nflag = 0;
      __syncthreads();
      double wmax = 0.0;
      for (int t = tid >> 6; t < nt; t += 4) {
        int I, J;
        if (CHOL) {
          J = 0;
          int r = t;
          while (r >= M - J) { r -= M - J; ++J; }
          I = J + r;
        } else {
          I = t % M;
          J = t / M;
        }
        I += k + 1;
        J += k + 1;
        double mr;
        const int nfl = wave_tile32(A, lda, I, J, min(BNB, n - I * BNB), min(BNB, n - J * BNB), CHOL && I == J, 1,
                                    c.colchk, ldc, c.rowchk, BMAX, c.gc, c.gr, tsu, wlds, &mr, s_frow, s_fcol, rep);
        if (nfl) {
          if ((tid & 63) == 0) {
            const int slot = atomicAdd(&s_nflag, 1);
            if (slot < BMAXFL) s_flagged[slot] = t;
          }
        } else {
          wmax = fmax(wmax, mr);
        }
      }
      if ((tid & 63) == 0 && wmax > 0) rep_max_ratio(rep, wmax);
      __syncthreads();
      const int nf = min(s_nflag, BMAXFL);
      if (nf > 0) {
        // tile order (the workgroup's waves listed them in any order)
        if (tid == 0)
          for (int a = 1; a < nf; ++a)
            for (int b2 = a; b2 > 0 && s_flagged[b2 - 1] > s_flagged[b2]; --b2) {
              const int tmp = s_flagged[b2];
              s_flagged[b2] = s_flagged[b2 - 1];
              s_flagged[b2 - 1] = tmp;
            }
        __syncthreads();
        for (int f = 0; f < nf; ++f) {
          const int t = s_flagged[f];
          int I, J;
          if (CHOL) {
            J = 0;
            int r = t;
            while (r >= M - J) { r -= M - J; ++J; }
            I = J + r;
          } else {
            I = t % M;
            J = t / M;
          }
          I += k + 1;
          J += k + 1;
          if (tid == 0) {
            rep->flagged_tiles++;
            if (rep->first_flag_iter > k) rep->first_flag_iter = k;
          }
          correct_tile_dev(A, lda, I, J, BNB, min(BNB, n - I * BNB), min(BNB, n - J * BNB), CHOL && I == J, c.colchk,
                           ldc, c.rowchk, BMAX, c.gc, c.gr, tsu, rep, k, ts, tf, cs);
          __syncthreads();
        }
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
        dreps[mi].fault_delta = 0.0;
        dreps[mi].fault_d = dreps[mi].fault_tau = -1.0;
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
  // panel, then the U12 chunk / the carry's sum block, or the verify scratch
  const size_t tail = std::max((size_t)BNB * 65 * elem, (size_t)4 * BN * BNB * sizeof(double));
  size_t shm = std::max((size_t)BMAX * (BNB + 1) * elem + tail, sizeof(TileSums) + sizeof(TileFlags));
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
