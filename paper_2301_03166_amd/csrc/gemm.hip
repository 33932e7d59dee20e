// FP64 MFMA GEMM for gfx950:  C = beta*C + alpha*op(A)*op(B), column-major.
//
// One 256-thread workgroup computes a 128x128 tile of C with four waves in a
// 2x2 arrangement (64x64 each, 4x4 blocks of v_mfma_f64_16x16x4_f64).  K is
// walked in steps of 16 through double-buffered LDS: the next step's global
// loads are in flight while the current step's MFMAs run.  The MFMA's
// row/column roles are swapped (its "A" operand is the B tile): the
// instruction's result D[i][j] sits in lane j + 16 (i % 4), register i / 4
// (measured on gfx950), so with D = C^T each register of a lane maps to one
// column of C and sixteen lanes write sixteen consecutive rows -- every store
// instruction writes 128-byte column segments.
//
// Operand options (template): transposition, a unit-lower mask on the stored
// operand (Householder vectors with their implicit unit diagonal), |.| of the
// operand (magnitude products for checksum thresholds), binary32 operands
// with optional bf16/fp16 rounding (checksum updates of mixed-precision
// factorizations), and a lower-triangular write mask (symmetric updates).
// Workgroups are remapped so that each XCD receives a contiguous range of
// tiles in column-major tile order, keeping B panels L2-resident per XCD.
#include "common.hpp"
#include "kernels.hpp"

#include <hip/hip_fp16.h>

#include <algorithm>

namespace abft {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float round_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;  // Inf / NaN unchanged
  u += 0x7fffu + ((u >> 16) & 1u);                 // round to nearest, ties to even
  return __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ float round_fp16(float x) { return __half2float(__float2half_rn(x)); }

template <int RND>
__device__ __forceinline__ double load_op(const double* p) {
  return *p;
}
template <int RND>
__device__ __forceinline__ double load_op(const float* p) {
  float v = *p;
  if (RND == 1) v = round_bf16(v);
  if (RND == 2) v = round_fp16(v);
  return (double)v;
}

// Split-K (kc > 0): workgroup y takes K range [y*kc, min(K, (y+1)*kc)) and
// writes alpha * its partial product to P + y*M*N (leading dimension M);
// k_splitk_reduce then adds the partials in a fixed order.
template <typename AT, typename BT, int TA, int TB, int FA, int FB, int LOWER, int RND>
__global__ __launch_bounds__(256) void k_gemm64(int M, int N, int K, double alpha, const AT* __restrict__ A,
                                                int64_t lda, const BT* __restrict__ B, int64_t ldb, double beta,
                                                double* __restrict__ C, int64_t ldc, int64_t doff, int kc,
                                                double* __restrict__ P) {
  constexpr int BM = 128, BN = 128, BK = 16, PAD = 4;
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][BN + PAD];

  const int tilesM = (M + BM - 1) / BM, tilesN = (N + BN - 1) / BN;
  const int nt = tilesM * tilesN;
  int wg = blockIdx.x;
  if ((nt & 7) == 0) wg = (wg & 7) * (nt >> 3) + (wg >> 3);
  const int tm = wg % tilesM, tn = wg / tilesM;
  const int m0 = tm * BM, n0 = tn * BN;
  if (LOWER && (int64_t)(m0 + BM - 1) + doff < (int64_t)n0) return;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv & 1, wn = wv >> 1;
  const int kbeg = kc > 0 ? (int)blockIdx.y * kc : 0;
  const int kend = kc > 0 ? min(K, kbeg + kc) : K;
  if (kc > 0) {
    C = P + (int64_t)blockIdx.y * M * N;
    ldc = M;
    beta = 0.0;
  }

  double ra[8], rb[8];
  auto loadA = [&](int k0) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      int idx = tid + 256 * s;
      int i, p;
      if (TA == 0) { i = idx % BM; p = idx / BM; } else { p = idx % BK; i = idx / BK; }
      int gi = m0 + i, gp = k0 + p;
      double v = 0.0;
      if (gi < M && gp < kend) {
        int64_t r = TA == 0 ? gi : gp, c = TA == 0 ? gp : gi;
        v = load_op<RND>(A + r + c * lda);
        if (FA == 1 || FA == 3) v = (r < c) ? 0.0 : ((r == c) ? 1.0 : v);
        if (FA == 2 || FA == 3) v = fabs(v);
      }
      ra[s] = v;
    }
  };
  auto loadB = [&](int k0) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      int idx = tid + 256 * s;
      int j, p;
      if (TB == 0) { p = idx % BK; j = idx / BK; } else { j = idx % BN; p = idx / BN; }
      int gj = n0 + j, gp = k0 + p;
      double v = 0.0;
      if (gj < N && gp < kend) {
        int64_t r = TB == 0 ? gp : gj, c = TB == 0 ? gj : gp;
        v = load_op<RND>(B + r + c * ldb);
        if (FB == 1) v = (r < c) ? 0.0 : ((r == c) ? 1.0 : v);
        if (FB == 2) v = fabs(v);
      }
      rb[s] = v;
    }
  };
  auto storeAB = [&](int buf) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      int idx = tid + 256 * s;
      if (TA == 0) As[buf][idx / BM][idx % BM] = ra[s]; else As[buf][idx % BK][idx / BK] = ra[s];
      if (TB == 0) Bs[buf][idx % BK][idx / BK] = rb[s]; else Bs[buf][idx / BN][idx % BN] = rb[s];
    }
  };

  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

  const int KT = (kend - kbeg + BK - 1) / BK;
  if (KT > 0) {
    loadA(kbeg);
    loadB(kbeg);
    storeAB(0);
  }
  __syncthreads();
  const int kl = lane >> 4, il = lane & 15;
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) {
      loadA(kbeg + (kt + 1) * BK);
      loadB(kbeg + (kt + 1) * BK);
    }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      double af[4], bf[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        af[q] = As[cur][kk * 4 + kl][wm * 64 + q * 16 + il];
        bf[q] = Bs[cur][kk * 4 + kl][wn * 64 + q * 16 + il];
      }
#pragma unroll
      for (int ci = 0; ci < 4; ++ci)
#pragma unroll
        for (int ri = 0; ri < 4; ++ri)
          acc[ci][ri] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[ci], af[ri], acc[ci][ri], 0, 0, 0);
    }
    if (kt + 1 < KT) storeAB(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int ci = 0; ci < 4; ++ci)
#pragma unroll
    for (int ri = 0; ri < 4; ++ri)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gi = m0 + wm * 64 + ri * 16 + il;
        int gj = n0 + wn * 64 + ci * 16 + 4 * r + kl;
        if (gi < M && gj < N && (!LOWER || (int64_t)gi + doff >= (int64_t)gj)) {
          double* p = C + gi + (int64_t)gj * ldc;
          double v = alpha * acc[ci][ri][r];
          *p = (beta == 0.0) ? v : beta * (*p) + v;
        }
      }
}

__global__ void k_splitk_reduce(const double* __restrict__ P, int S, int M, int N, double beta, double* C,
                                int64_t ldc) {
  const int64_t tot = (int64_t)M * N;
  const bool narrow = tot <= 0x7fffffff;  // (32-bit index arithmetic)
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i, j;
    if (narrow) {
      const uint32_t jj = (uint32_t)e / (uint32_t)M;
      j = jj;
      i = (int64_t)((uint32_t)e - jj * (uint32_t)M);
    } else {
      j = e / M;
      i = e - j * M;
    }
    // the partials in order, sixteen requested before the first is added
    double acc = 0.0;
    for (int q = 0; q < S; q += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = q + u < S ? P[(int64_t)(q + u) * tot + e] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (q + u < S) acc += v[u];
    }
    double* c = C + i + j * ldc;
    *c = (beta == 0.0) ? acc : beta * (*c) + acc;
  }
}

int splitk_reduce(hipStream_t s, const double* P, int S, int m, int n, double beta, double* C, int64_t ldc) {
  unsigned rg = (unsigned)std::min<int64_t>(4096, ((int64_t)m * n + 255) / 256);
  hipLaunchKernelGGL(k_splitk_reduce, dim3(rg), dim3(256), 0, s, P, S, m, n, beta, C, ldc);
  return hipGetLastError() == hipSuccess ? 0 : ABFT_ERR_HIP;
}

// ---------------------------------------------------------------------------
// host dispatcher
// ---------------------------------------------------------------------------
#define GEMM_CASE(AT_, BT_, TA_, TB_, FA_, FB_, LO_, RN_)                                                        \
  if (ta == TA_ && tb == TB_ && fa == FA_ && fb == FB_ && lower == LO_ && rnd == RN_) {                            \
    hipLaunchKernelGGL((k_gemm64<AT_, BT_, TA_, TB_, FA_, FB_, LO_, RN_>), dim3((unsigned)grid, S), dim3(256), 0, s, \
                       m, n, k, alpha, (const AT_*)A, lda, (const BT_*)B, ldb, beta, C, ldc, doff, kc, ws);        \
    if (hipGetLastError() != hipSuccess) return ABFT_ERR_HIP;                                                      \
    if (kc > 0) {                                                                                                  \
      unsigned rg = (unsigned)std::min<int64_t>(4096, ((int64_t)m * n + 255) / 256);                              \
      hipLaunchKernelGGL(k_splitk_reduce, dim3(rg), dim3(256), 0, s, ws, (int)S, m, n, beta, C, ldc);               \
      if (hipGetLastError() != hipSuccess) return ABFT_ERR_HIP;                                                    \
    }                                                                                                              \
    return 0;                                                                                                      \
  }

int gemm64(hipStream_t s, int ta, int tb, int fa, int fb, int lower, int m, int n, int k, double alpha, const void* A,
           int64_t lda, const void* B, int64_t ldb, double beta, double* C, int64_t ldc, int64_t doff, int atype,
           int btype, int rnd, double* ws, size_t ws_elems, int role, int* split_out) {
  if (m <= 0 || n <= 0) return 0;
  if (k <= 0 && beta == 1.0) return 0;
  int64_t grid = (int64_t)((m + 127) / 128) * ((n + 127) / 128);
  // few output tiles and a long K: split K over extra workgroups (about two
  // per CU, K ranges of at least 128, as many as the partials buffer holds)
  unsigned S = 1;
  int kc = 0;
  // (a trailing-update launch splits only when its caller reduces the
  // partials itself, so that the launch stays one kernel)
  if (split_out) *split_out = 0;
  const int64_t slots = 512;  // resident product workgroups: two per CU
  int64_t want = 1;
  if (ws && !lower && (!role || split_out) && grid < slots && k >= 1024) {
    want = std::min<int64_t>(64, std::min<int64_t>((slots + grid - 1) / grid, k / 128));
  } else if (ws && !lower && split_out && grid % slots != 0 && k >= 2048) {
    // several rounds of long-K tiles with a partial last round: the split
    // (2..4) with the least time in rounds per unit of K
    double best = (double)((grid + slots - 1) / slots);
    for (int64_t sp = 2; sp <= 4 && k / sp >= 512; ++sp) {
      const double cost = (double)((grid * sp + slots - 1) / slots) / (double)sp;
      if (cost < 0.95 * best) {
        best = cost;
        want = sp;
      }
    }
  }
  want = std::min<int64_t>(want, (int64_t)(ws_elems / ((size_t)m * n)));
  if (want >= 2) {
    int64_t kcl = ((k + want - 1) / want + 31) / 32 * 32;
    int64_t sp = (k + kcl - 1) / kcl;
    if (sp >= 2 && (size_t)sp * m * n <= ws_elems) {
      S = (unsigned)sp;
      kc = (int)kcl;
    }
  }
  if (atype == 0 && btype == 0 && rnd == 0) {
    const int r = dgemm_fast(s, ta, tb, fa, fb, lower, m, n, k, alpha, (const double*)A, lda, (const double*)B, ldb,
                             beta, C, ldc, doff, (int)S, kc, ws, role);
    if (r < 0) return r;
    if (r == 1) {
      if (kc > 0) {
        if (split_out) {
          *split_out = (int)S;
          return 0;
        }
        return splitk_reduce(s, ws, (int)S, m, n, beta, C, ldc);
      }
      return 0;
    }
  }
  if (atype == 0 && btype == 0) {
    GEMM_CASE(double, double, 0, 0, 0, 0, 0, 0)  // LU trailing update, TRSM updates, checksum carries
    GEMM_CASE(double, double, 0, 1, 0, 0, 0, 0)  // X * Y^T
    GEMM_CASE(double, double, 0, 1, 0, 0, 1, 0)  // symmetric (lower) trailing update
    GEMM_CASE(double, double, 1, 0, 1, 0, 0, 0)  // V^T C
    GEMM_CASE(double, double, 0, 0, 1, 0, 0, 0)  // V W
    GEMM_CASE(double, double, 1, 0, 0, 0, 0, 0)  // T^T W
    GEMM_CASE(double, double, 1, 0, 0, 1, 0, 0)  // V1^T V2 (rows below V1's block)
    GEMM_CASE(double, double, 0, 0, 0, 2, 0, 0)  // magnitudes Sa * |Y|
    GEMM_CASE(double, double, 0, 1, 0, 2, 0, 0)  // magnitudes Sa * |X|^T
    GEMM_CASE(double, double, 0, 0, 2, 0, 0, 0)  // |X| * Ta
    GEMM_CASE(double, double, 0, 1, 2, 0, 0, 0)  // |X| * Sa^T
    GEMM_CASE(double, double, 0, 0, 3, 0, 0, 0)  // |V| * Ta (unit-lower V)
    GEMM_CASE(double, double, 1, 0, 2, 2, 0, 0)  // |V|^T |R| (QR panel check, odd widths)
  }
  if (atype == 0 && btype == 1) {  // double S times binary32 Y (mixed-precision checksum carry)
    GEMM_CASE(double, float, 0, 0, 0, 0, 0, 0)
    GEMM_CASE(double, float, 0, 0, 0, 0, 0, 1)
    GEMM_CASE(double, float, 0, 0, 0, 0, 0, 2)
    GEMM_CASE(double, float, 0, 0, 0, 2, 0, 0)
    GEMM_CASE(double, float, 0, 0, 0, 2, 0, 1)
    GEMM_CASE(double, float, 0, 0, 0, 2, 0, 2)
    GEMM_CASE(double, float, 0, 1, 0, 0, 0, 0)
    GEMM_CASE(double, float, 0, 1, 0, 0, 0, 1)
    GEMM_CASE(double, float, 0, 1, 0, 0, 0, 2)
    GEMM_CASE(double, float, 0, 1, 0, 2, 0, 0)
    GEMM_CASE(double, float, 0, 1, 0, 2, 0, 1)
    GEMM_CASE(double, float, 0, 1, 0, 2, 0, 2)
  }
  if (atype == 1 && btype == 0) {  // binary32 X times double T
    GEMM_CASE(float, double, 0, 0, 0, 0, 0, 0)
    GEMM_CASE(float, double, 0, 0, 0, 0, 0, 1)
    GEMM_CASE(float, double, 0, 0, 0, 0, 0, 2)
    GEMM_CASE(float, double, 0, 0, 2, 0, 0, 0)
    GEMM_CASE(float, double, 0, 0, 2, 0, 0, 1)
    GEMM_CASE(float, double, 0, 0, 2, 0, 0, 2)
    GEMM_CASE(float, double, 0, 1, 0, 0, 0, 0)
    GEMM_CASE(float, double, 0, 1, 0, 0, 0, 1)
    GEMM_CASE(float, double, 0, 1, 0, 0, 0, 2)
    GEMM_CASE(float, double, 0, 1, 2, 0, 0, 0)
    GEMM_CASE(float, double, 0, 1, 2, 0, 0, 1)
    GEMM_CASE(float, double, 0, 1, 2, 0, 0, 2)
  }
  return ABFT_ERR_UNSUPPORTED;
}

}  // namespace abft
