// Binary32-data GEMM for the mixed-precision trailing update on gfx950:
//   C = beta*C + alpha*op(A)*op(B), C/A/B float, column-major,
// with the products on FP32 MFMA (v_mfma_f32_16x16x4_f32) or on bf16 / fp16
// MFMA (16x16x16, FP32 accumulation) after round-to-nearest-even of the
// operands.  Tile and pipeline shape follow the FP64 kernel: 128x128 tiles,
// four waves of 64x64, K in steps of 16 through double-buffered LDS,
// XCD-aware workgroup order.  For these MFMAs the result D[i][j] sits in lane
// j + 16 (i / 4), register i % 4 (measured on gfx950; the FP64 instruction
// interleaves the other way), so with D = C^T a lane's four registers are four
// consecutive columns of C.  The bf16/fp16 form is bound by the FP32 read
// and write of C (arithmetic intensity ~ nb/4 flop per byte), the FP32 form
// by the MFMA rate.
#include "common.hpp"
#include "kernels.hpp"

namespace abft {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

template <int TA, int TB, int PREC, int LOWER>
__global__ __launch_bounds__(256) void k_gemm32(int M, int N, int K, float alpha, const float* __restrict__ A,
                                                int64_t lda, const float* __restrict__ B, int64_t ldb, float beta,
                                                float* __restrict__ C, int64_t ldc, int64_t doff) {
  constexpr int BM = 128, BN = 128, BK = 16, PAD = 4;
  __shared__ float As[2][BK][BM + PAD];
  __shared__ float Bs[2][BK][BN + PAD];
  const int tilesM = (M + BM - 1) / BM, tilesN = (N + BN - 1) / BN;
  const int nt = tilesM * tilesN;
  int wg = blockIdx.x;
  if ((nt & 7) == 0) wg = (wg & 7) * (nt >> 3) + (wg >> 3);
  const int tm = wg % tilesM, tn = wg / tilesM;
  const int m0 = tm * BM, n0 = tn * BN;
  if (LOWER && (int64_t)(m0 + BM - 1) + doff < (int64_t)n0) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv & 1, wn = wv >> 1;

  float ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      int idx = tid + 256 * s;
      int i, p;
      if (TA == 0) { i = idx % BM; p = idx / BM; } else { p = idx % BK; i = idx / BK; }
      int gi = m0 + i, gp = k0 + p;
      float v = 0.f;
      if (gi < M && gp < K) v = TA == 0 ? A[gi + (int64_t)gp * lda] : A[gp + (int64_t)gi * lda];
      ra[s] = v;
      int j;
      if (TB == 0) { p = idx % BK; j = idx / BK; } else { j = idx % BN; p = idx / BN; }
      int gj = n0 + j;
      gp = k0 + p;
      v = 0.f;
      if (gj < N && gp < K) v = TB == 0 ? B[gp + (int64_t)gj * ldb] : B[gj + (int64_t)gp * ldb];
      rb[s] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      int idx = tid + 256 * s;
      if (TA == 0) As[buf][idx / BM][idx % BM] = ra[s]; else As[buf][idx % BK][idx / BK] = ra[s];
      if (TB == 0) Bs[buf][idx % BK][idx / BK] = rb[s]; else Bs[buf][idx / BN][idx % BN] = rb[s];
    }
  };

  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int KT = (K + BK - 1) / BK;
  if (KT > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int kl = lane >> 4, il = lane & 15;
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) load((kt + 1) * BK);
    if (PREC == ABFT_F32) {
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        float af[4], bf[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          af[q] = As[cur][kk * 4 + kl][wm * 64 + q * 16 + il];
          bf[q] = Bs[cur][kk * 4 + kl][wn * 64 + q * 16 + il];
        }
#pragma unroll
        for (int ci = 0; ci < 4; ++ci)
#pragma unroll
          for (int ri = 0; ri < 4; ++ri)
            acc[ci][ri] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[ci], af[ri], acc[ci][ri], 0, 0, 0);
      }
    } else if (PREC == ABFT_BF16) {
      s16x4 af[4], bf[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          af[q][e] = bf16_bits(As[cur][kl * 4 + e][wm * 64 + q * 16 + il]);
          bf[q][e] = bf16_bits(Bs[cur][kl * 4 + e][wn * 64 + q * 16 + il]);
        }
#pragma unroll
      for (int ci = 0; ci < 4; ++ci)
#pragma unroll
        for (int ri = 0; ri < 4; ++ri)
          acc[ci][ri] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bf[ci], af[ri], acc[ci][ri], 0, 0, 0);
    } else {
      f16x4 af[4], bf[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          af[q][e] = (_Float16)As[cur][kl * 4 + e][wm * 64 + q * 16 + il];
          bf[q][e] = (_Float16)Bs[cur][kl * 4 + e][wn * 64 + q * 16 + il];
        }
#pragma unroll
      for (int ci = 0; ci < 4; ++ci)
#pragma unroll
        for (int ri = 0; ri < 4; ++ri)
          acc[ci][ri] = __builtin_amdgcn_mfma_f32_16x16x16f16(bf[ci], af[ri], acc[ci][ri], 0, 0, 0);
    }
    if (kt + 1 < KT) store(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int ci = 0; ci < 4; ++ci)
#pragma unroll
    for (int ri = 0; ri < 4; ++ri)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gi = m0 + wm * 64 + ri * 16 + il;
        int gj = n0 + wn * 64 + ci * 16 + 4 * kl + r;
        if (gi < M && gj < N && (!LOWER || (int64_t)gi + doff >= (int64_t)gj)) {
          float* p = C + gi + (int64_t)gj * ldc;
          float v = alpha * acc[ci][ri][r];
          *p = (beta == 0.f) ? v : beta * (*p) + v;
        }
      }
}

#define G32_CASE(TA_, TB_, PR_, LO_)                                                                             \
  if (ta == TA_ && tb == TB_ && prec == PR_ && lower == LO_) {                                                   \
    hipLaunchKernelGGL((k_gemm32<TA_, TB_, PR_, LO_>), dim3(grid), dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb, \
                       beta, C, ldc, doff);                                                                       \
    return hipGetLastError() == hipSuccess ? 0 : ABFT_ERR_HIP;                                                   \
  }

int gemm32(hipStream_t s, int prec, int ta, int tb, int lower, int m, int n, int k, float alpha, const float* A,
           int64_t lda, const float* B, int64_t ldb, float beta, float* C, int64_t ldc, int64_t doff) {
  if (m <= 0 || n <= 0) return 0;
  if (k <= 0 && beta == 1.f) return 0;
  int64_t grid = (int64_t)((m + 127) / 128) * ((n + 127) / 128);
  G32_CASE(0, 0, ABFT_F32, 0)
  G32_CASE(0, 1, ABFT_F32, 0)
  G32_CASE(0, 1, ABFT_F32, 1)
  G32_CASE(0, 0, ABFT_BF16, 0)
  G32_CASE(0, 1, ABFT_BF16, 1)
  G32_CASE(0, 0, ABFT_F16, 0)
  G32_CASE(0, 1, ABFT_F16, 1)
  return ABFT_ERR_UNSUPPORTED;
}

}  // namespace abft
