// Kernels of the mixed-precision solve with FP64 iterative refinement:
// precision conversion, the row permutation of LU, blocked triangular solves
// (one launch per solve, sync-free between row blocks), the FP64 residual
// r = b - A x and the vector updates / infinity norms the refinement reads.
#include "common.hpp"
#include "kernels.hpp"

namespace abft {

constexpr int TB = 64;  // rows per block of the triangular solves

__global__ void k_convert(const double* __restrict__ A, int64_t lda, float* __restrict__ B, int64_t ldb, int64_t m,
                          int64_t n) {
  const int64_t j = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    B[i + j * ldb] = (float)A[i + j * lda];
}

// final row permutation of the LU interchanges: row i of P A is row perm[i] of A
__global__ void k_perm_vector(const int32_t* ipiv, int n, int* perm) {
  extern __shared__ int pv[];
  for (int i = threadIdx.x; i < n; i += blockDim.x) pv[i] = i;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < n; ++j) {
      int q = ipiv[j] - 1;
      int t = pv[j];
      pv[j] = pv[q];
      pv[q] = t;
    }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) perm[i] = pv[i];
}

// y[i] = (float) (x[perm[i]] * scale)   (perm may be null)
__global__ void k_gather_scale(const double* x, const int* perm, double scale, float* y, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    y[i] = (float)(x[perm ? perm[i] : i] * scale);
}
__global__ void k_gather64(const double* x, const int* perm, double* y, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[i] = x[perm ? perm[i] : i];
}

// Triangular solve x := M^{-1} x in place (M n x n, stored in the factor
// array F): KIND 0 = unit lower (LU's L), 1 = upper (LU's U), 2 = lower
// (Cholesky L), 3 = upper given as the transpose of the stored lower
// Cholesky factor.  Workgroups take 64-row blocks in solve order from a
// counter.  A solved block is published as self-validating words in xw
// (each 64-bit word = 32 bits of the value and the call's sequence number
// seq; one word per binary32 value, two per binary64 value), so a later
// block polls the very values it needs, with no flag and no fence between
// writer and reader.  A block first subtracts the products of every earlier
// block: its 64 x 64 coefficient blocks do not depend on the solution and
// are read ahead, and each wave takes every earlier block whose first word
// is already published in one go.  One wave then solves the diagonal block
// with its row of the block in registers: substitution, one lane broadcast
// per step, the reciprocals of the diagonal formed up front.  The
// accumulation order is fixed, so results are reproducible.
template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c);
template <>
__device__ __forceinline__ float fmat<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fmat<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T lane_bcast(T v, int j);
template <>
__device__ __forceinline__ float lane_bcast<float>(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
template <>
__device__ __forceinline__ double lane_bcast<double>(double v, int j) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, j), hi = __builtin_amdgcn_readlane((int)(u >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// words per value and the encode / poll of one value
template <typename T>
constexpr int xw_words() { return sizeof(T) == 4 ? 1 : 2; }
__device__ __forceinline__ void xw_put(uint64_t* p, uint32_t payload, uint32_t seq) {
  __hip_atomic_store(p, ((uint64_t)payload << 32) | seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void xw_store(uint64_t* xw, int64_t i, T v, uint32_t seq) {
  if (sizeof(T) == 4) {
    xw_put(xw + i, __float_as_uint((float)v), seq);
  } else {
    const uint64_t u = (uint64_t)__double_as_longlong((double)v);
    xw_put(xw + 2 * i, (uint32_t)(u >> 32), seq);
    xw_put(xw + 2 * i + 1, (uint32_t)u, seq);
  }
}
__device__ __forceinline__ uint64_t xw_poll(const uint64_t* p, uint32_t seq, long& spins, abft_report* rep) {
  uint64_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while ((uint32_t)v != seq) {
    __builtin_amdgcn_s_sleep(1);
    v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (++spins > (1L << 22)) {
      if (rep) atomicOr(&rep->status, (int)ABFT_ST_INTERNAL);
      break;
    }
  }
  return v;
}

template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_trsv(const T* __restrict__ F, int64_t ld, int n, T* x, unsigned* counter,
                                              uint64_t* xw, uint32_t seq, abft_report* rep) {
  constexpr bool LOWER = KIND == 0 || KIND == 2, TR = KIND == 3;
  constexpr int WPV = xw_words<T>();
  __shared__ T part[4][TB];
  __shared__ T D[TB][TB + 1];
  __shared__ int s_blk;
  const int nblk = (n + TB - 1) / TB;
  if (threadIdx.x == 0) s_blk = (int)atomicAdd(counter, 1u);
  __syncthreads();
  const int ord = s_blk;
  if (ord >= nblk) return;
  const int b = LOWER ? ord : nblk - 1 - ord;
  const int64_t r0 = (int64_t)b * TB;
  const int rows = (int)min((int64_t)TB, (int64_t)n - r0);
  const int r = threadIdx.x & (TB - 1), q = threadIdx.x >> 6;
  // element (i, j) of the diagonal block of M
  for (int idx = threadIdx.x; idx < TB * TB; idx += 256) {
    const int i = TR ? idx / TB : idx % TB, j = TR ? idx % TB : idx / TB;
    T v = (T)0;
    if (i < rows && j < rows) v = TR ? F[(r0 + j) + (r0 + i) * ld] : F[(r0 + i) + (r0 + j) * ld];
    D[i][j] = v;
  }
  // earlier block k of the solve order, its coefficients in row r0 + r and
  // this wave's 16 columns [16 q, 16 q + 16)
  auto pred = [&](int k) { return LOWER ? k : nblk - 1 - k; };
  auto load_m = [&](int k, T(&m)[16]) {
    const int64_t c0 = (int64_t)pred(k) * TB;
    const int cl = (int)min((int64_t)TB, (int64_t)n - c0) - 16 * q;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int64_t col = c0 + 16 * q + s;
      m[s] = (r < rows && s < cl) ? (TR ? F[col + (r0 + r) * ld] : F[(r0 + r) + col * ld]) : (T)0;
    }
  };
  long spins = 0;
  T acc = (T)0;
  auto accum = [&](int k, const T(&m)[16]) {
    const int64_t c0 = (int64_t)pred(k) * TB;
    const int cl = (int)min((int64_t)TB, (int64_t)n - c0) - 16 * q;
    uint64_t wd[16 * WPV];
#pragma unroll
    for (int s = 0; s < 16; ++s)
#pragma unroll
      for (int u = 0; u < WPV; ++u)
        wd[s * WPV + u] = s < cl ? __hip_atomic_load(xw + WPV * (c0 + 16 * q + s) + u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                                 : (uint64_t)seq;
    T xs[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      if (s < cl) {
#pragma unroll
        for (int u = 0; u < WPV; ++u)
          if ((uint32_t)wd[s * WPV + u] != seq) wd[s * WPV + u] = xw_poll(xw + WPV * (c0 + 16 * q + s) + u, seq, spins, rep);
        if (sizeof(T) == 4)
          xs[s] = (T)__uint_as_float((uint32_t)(wd[s * WPV] >> 32));
        else
          xs[s] = (T)__longlong_as_double(
              (long long)((wd[s * WPV] & 0xffffffff00000000ull) | (wd[s * WPV + WPV - 1] >> 32)));
      } else {
        xs[s] = (T)0;
      }
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) acc = fmat(m[s], xs[s], acc);
  };
  T mp[16];
  if (ord > 0) load_m(0, mp);
  for (int k = 0; k < ord;) {
    // earlier blocks k, k+1, ... whose first value is published (lane l looks at k + l)
    int nr;
    for (;;) {
      const int kl = k + r;
      int f = 1;
      if (kl < ord) {
        const uint64_t v = __hip_atomic_load(xw + WPV * ((int64_t)pred(kl) * TB), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        f = (uint32_t)v == seq;
      }
      const unsigned long long waiting = __ballot(f == 0);
      nr = min(waiting ? (int)__builtin_ctzll(waiting) : TB, ord - k);
      if (nr > 0) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1L << 22)) {
        if (r == 0 && rep) atomicOr(&rep->status, (int)ABFT_ST_INTERNAL);
        nr = ord - k;
        break;
      }
    }
    accum(k, mp);
    int kk = k + 1;
    for (; kk + 1 < k + nr; kk += 2) {
      T m0[16], m1[16];
      load_m(kk, m0);
      load_m(kk + 1, m1);
      accum(kk, m0);
      accum(kk + 1, m1);
    }
    if (kk < k + nr) {
      T m0[16];
      load_m(kk, m0);
      accum(kk, m0);
    }
    k += nr;
    if (k < ord) load_m(k, mp);
  }
  part[q][r] = acc;
  __syncthreads();
  if (q != 0) return;
  // diagonal block: wave 0, lane r holds row r
  T xv = (T)0, dr[TB];
  if (r < rows) xv = x[r0 + r] - (((part[0][r] + part[1][r]) + part[2][r]) + part[3][r]);
#pragma unroll
  for (int j = 0; j < TB; ++j) dr[j] = D[r][j];
  const T rd = (KIND != 0 && r < rows) ? (T)1 / D[r][r] : (T)1;
#pragma unroll
  for (int s = 0; s < TB; ++s) {
    const int j = LOWER ? s : TB - 1 - s;
    if (j < rows) {
      T xj = lane_bcast(xv, j);
      if (KIND != 0) xj *= lane_bcast(rd, j);
      if (r == j) xv = xj;
      else if (LOWER ? r > j : r < j) xv = fmat(-dr[j], xj, xv);
    }
  }
  if (r < rows) {
    xw_store(xw, r0 + r, xv, seq);
    x[r0 + r] = xv;
  }
}

// residual partials: part[s][i] = sum over column chunk s of A(i, j) x(j)
__global__ __launch_bounds__(256) void k_resid_part(const double* __restrict__ A, int64_t lda, int n,
                                                    const double* __restrict__ x, int chunk, double* part) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  const int j0 = s * chunk, j1 = min(n, j0 + chunk);
  __shared__ double xs[256];
  double acc = 0.0;
  for (int jb = j0; jb < j1; jb += 256) {
    __syncthreads();
    if (jb + threadIdx.x < j1) xs[threadIdx.x] = x[jb + threadIdx.x];
    __syncthreads();
    const int je = min(256, j1 - jb);
    if (i < n)
      for (int jj = 0; jj < je; ++jj) acc += A[i + (int64_t)(jb + jj) * lda] * xs[jj];
  }
  if (i < n) part[(int64_t)s * n + i] = acc;
}

__device__ __forceinline__ void max_bits(double* p, double v) {
  if (!(v <= 1.79e308)) v = __longlong_as_double(0x7ff0000000000000ll);  // NaN / Inf -> +Inf
  atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

// r = b - sum_s part[s]; norms[0] = max |r|, norms[1] = max |x|
__global__ void k_resid_fin(const double* part, int nsplit, const double* b, const double* x, double* r, int n,
                            double* norms) {
  double mr = 0.0, mx = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < nsplit; ++q) s += part[(int64_t)q * n + i];
    double v = b[i] - s;
    r[i] = v;
    mr = fmax(mr, fabs(v));
    if (!(fabs(v) <= 1.79e308)) mr = __longlong_as_double(0x7ff0000000000000ll);
    mx = fmax(mx, fabs(x[i]));
    if (!(fabs(x[i]) <= 1.79e308)) mx = __longlong_as_double(0x7ff0000000000000ll);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mr = fmax(mr, __shfl_xor(mr, o));
    mx = fmax(mx, __shfl_xor(mx, o));
  }
  if ((threadIdx.x & 63) == 0) {
    max_bits(&norms[0], mr);
    max_bits(&norms[1], mx);
  }
}

// x += scale * (double) d32; norms[2] = max |scale d|, norms[3] = max |x|
__global__ void k_update(double* x, const float* d32, double scale, int n, double* norms) {
  double md = 0.0, mx = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double d = scale * (double)d32[i];
    double v = x[i] + d;
    x[i] = v;
    md = fmax(md, fabs(d));
    if (!(fabs(d) <= 1.79e308)) md = __longlong_as_double(0x7ff0000000000000ll);
    mx = fmax(mx, fabs(v));
    if (!(fabs(v) <= 1.79e308)) mx = __longlong_as_double(0x7ff0000000000000ll);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    md = fmax(md, __shfl_xor(md, o));
    mx = fmax(mx, __shfl_xor(mx, o));
  }
  if ((threadIdx.x & 63) == 0) {
    max_bits(&norms[2], md);
    max_bits(&norms[3], mx);
  }
}

// infinity norm of A (max row |.|-sum) into norms[4], in two passes: row
// sums over column chunks (part[s][i], chunk s), then their fixed-order sums
__global__ __launch_bounds__(256) void k_anorm_part(const double* __restrict__ A, int64_t lda, int n, int chunk,
                                                    double* part) {
  const int i = blockIdx.x * 256 + threadIdx.x, s = blockIdx.y;
  const int j0 = s * chunk, j1 = min(n, j0 + chunk);
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < n) {
    int j = j0;
    for (; j + 7 < j1; j += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += fabs(A[i + (int64_t)(j + u) * lda]);
    }
    for (int u = 0; j < j1; ++j, ++u) a[u] += fabs(A[i + (int64_t)j * lda]);
    part[(int64_t)s * n + i] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
}
__global__ void k_anorm_fin(const double* part, int nsplit, int n, double* norms) {
  double m = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int q = 0; q < nsplit; ++q) v += part[(int64_t)q * n + i];
    if (!(v <= 1.79e308)) v = __longlong_as_double(0x7ff0000000000000ll);
    m = fmax(m, v);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) max_bits(&norms[4], m);
}

__global__ void k_copy_f64(const double* a, double* b, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = a[i];
}
__global__ void k_f32_to_f64(const float* a, double* b, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = (double)a[i];
}

// ---------------------------------------------------------------------------
#define LAUNCH_OK return hipGetLastError() == hipSuccess ? 0 : ABFT_ERR_HIP
static inline unsigned g1(int64_t n) { return (unsigned)std::min<int64_t>(4096, (n + 255) / 256); }

int convert_f64_f32(hipStream_t s, const double* A, int64_t lda, float* B, int64_t ldb, int64_t m, int64_t n) {
  if (m <= 0 || n <= 0) return 0;
  hipLaunchKernelGGL(k_convert, dim3(g1(m), (unsigned)n), dim3(256), 0, s, A, lda, B, ldb, m, n);
  LAUNCH_OK;
}
int perm_vector(hipStream_t s, const int32_t* ipiv, int n, int* perm) {
  if ((size_t)n * sizeof(int) > 150 * 1024) return ABFT_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k_perm_vector, dim3(1), dim3(256), (size_t)n * sizeof(int), s, ipiv, n, perm);
  LAUNCH_OK;
}
int gather_scale(hipStream_t s, const double* x, const int* perm, double scale, float* y, int n) {
  hipLaunchKernelGGL(k_gather_scale, dim3(g1(n)), dim3(256), 0, s, x, perm, scale, y, n);
  LAUNCH_OK;
}
int gather64(hipStream_t s, const double* x, const int* perm, double* y, int n) {
  hipLaunchKernelGGL(k_gather64, dim3(g1(n)), dim3(256), 0, s, x, perm, y, n);
  LAUNCH_OK;
}
template <typename T>
int trsv(hipStream_t s, const T* F, int64_t ld, int n, int kind, T* x, unsigned* counter, uint64_t* xw,
         uint32_t seq, abft_report* rep) {
  if (n <= 0) return 0;
  if (kind < 0 || kind > 3 || seq == 0) return ABFT_ERR_UNSUPPORTED;
  const int nblk = (n + TB - 1) / TB;
  if (fill_zero(s, counter, 4)) return ABFT_ERR_HIP;
  switch (kind) {
    case 0: hipLaunchKernelGGL((k_trsv<T, 0>), dim3(nblk), dim3(256), 0, s, F, ld, n, x, counter, xw, seq, rep); break;
    case 1: hipLaunchKernelGGL((k_trsv<T, 1>), dim3(nblk), dim3(256), 0, s, F, ld, n, x, counter, xw, seq, rep); break;
    case 2: hipLaunchKernelGGL((k_trsv<T, 2>), dim3(nblk), dim3(256), 0, s, F, ld, n, x, counter, xw, seq, rep); break;
    default: hipLaunchKernelGGL((k_trsv<T, 3>), dim3(nblk), dim3(256), 0, s, F, ld, n, x, counter, xw, seq, rep);
  }
  LAUNCH_OK;
}
template int trsv<float>(hipStream_t, const float*, int64_t, int, int, float*, unsigned*, uint64_t*, uint32_t,
                         abft_report*);
template int trsv<double>(hipStream_t, const double*, int64_t, int, int, double*, unsigned*, uint64_t*, uint32_t,
                          abft_report*);

int residual(hipStream_t s, const double* A, int64_t lda, int n, const double* x, const double* b, double* r,
             double* part, int nsplit, double* norms) {
  const int chunk = (n + nsplit - 1) / nsplit;
  hipLaunchKernelGGL(k_resid_part, dim3((n + 255) / 256, nsplit), dim3(256), 0, s, A, lda, n, x, chunk, part);
  if (hipGetLastError() != hipSuccess) return ABFT_ERR_HIP;
  hipLaunchKernelGGL(k_resid_fin, dim3(g1(n)), dim3(256), 0, s, part, nsplit, b, x, r, n, norms);
  LAUNCH_OK;
}
int update_x(hipStream_t s, double* x, const float* d32, double scale, int n, double* norms) {
  hipLaunchKernelGGL(k_update, dim3(g1(n)), dim3(256), 0, s, x, d32, scale, n, norms);
  LAUNCH_OK;
}
int anorm(hipStream_t s, const double* A, int64_t lda, int n, double* part, int nsplit, double* norms) {
  if (n <= 0) return 0;
  const int chunk = (n + nsplit - 1) / nsplit;
  hipLaunchKernelGGL(k_anorm_part, dim3((n + 255) / 256, nsplit), dim3(256), 0, s, A, lda, n, chunk, part);
  if (hipGetLastError() != hipSuccess) return ABFT_ERR_HIP;
  hipLaunchKernelGGL(k_anorm_fin, dim3(g1(n)), dim3(256), 0, s, part, nsplit, n, norms);
  LAUNCH_OK;
}
int copy_f64(hipStream_t s, const double* a, double* b, int n) {
  hipLaunchKernelGGL(k_copy_f64, dim3(g1(n)), dim3(256), 0, s, a, b, n);
  LAUNCH_OK;
}
int f32_to_f64(hipStream_t s, const float* a, double* b, int n) {
  hipLaunchKernelGGL(k_f32_to_f64, dim3(g1(n)), dim3(256), 0, s, a, b, n);
  LAUNCH_OK;
}

}  // namespace abft
