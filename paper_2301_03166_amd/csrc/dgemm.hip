// FP64 MFMA GEMM for the large products of the factorizations (trailing
// updates and the reflector products of the blocked QR):
//   C = beta*C + alpha*op(A)*op(B), column-major, A/B 16-byte aligned with
//   even leading dimensions (the host dispatcher checks this).
//
// Tile 128x128 per 256-thread workgroup, four waves in 2x2 of 64x64, each a
// 4x4 block of v_mfma_f64_16x16x4_f64; K walked through double-buffered LDS
// in steps of BK: BK = 32 (~2 x 72 KB of LDS, one workgroup per CU, C read
// ahead during the last K step) or BK = 16 (~2 x 36 KB and at most 256
// registers per lane, so two workgroups share a CU and one's prologue and
// epilogue overlap the other's products).  Interior tiles load with 16-byte
// global loads and no bounds tests; edge tiles, the K tail and split-K
// remainders take the same data path with per-element guards.
//
// Workgroup order: the hardware deals workgroups round-robin to the eight
// XCDs; the index is remapped so that each XCD owns a contiguous chunk of a
// grouped order (groups of 8 tile-rows, column-major inside a group), so the
// 8 row-blocks of A a chunk reads stay in that XCD's L2 while it sweeps the
// columns.  For the symmetric (lower) update only the tiles on or below the
// diagonal are enumerated, column by column, so the chunks carry equal work.
//
// Operand options: op(A) = A or A^T, op(B) = B or B^T, a unit-lower mask on
// the stored A (Householder vectors with their implicit unit diagonal),
// magnitudes |op(A)| / |op(B)| (the checksum carries' threshold products),
// and a lower-triangular write mask on C.
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

namespace abft {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int DG_BM = 128, DG_BN = 128, DG_GM = 8;
// LDS image of an operand tile (R = 128 rows of op(X), BK values of k): an
// operand read from memory along R is kept k-major with row stride
// SKR = R + 16 (its 16-byte stores are sequential, and the MFMA's reads of
// four k-rows x 16 consecutive r fall in disjoint bank halves); an operand
// read along K is kept r-major with row stride SRK = BK + 2 (its 16-byte
// stores are sequential, and lane (r, k) of the MFMA read hits bank pair
// ((BK + 2) r + k) mod 32 -- a bijection over each half-wave for BK = 16, 32).
constexpr int SKR = DG_BM + 16;
template <int BK, bool ALONG_R>
__host__ __device__ constexpr int lds_elems() {
  return ALONG_R ? BK * SKR : DG_BM * (BK + 2);
}
template <int BK, bool ALONG_R>
__device__ __forceinline__ int lidx(int k, int r) {
  return ALONG_R ? k * SKR + r : r * (BK + 2) + k;
}

// Stage of one operand tile (R x BK logical, R = 128) held in registers as
// BK/4 pairs per thread.  ALONG_R: the pairs run along the tile's R
// dimension (stored operand contiguous in R); else along K.
template <int BK, bool ALONG_R>
struct Stage {
  f64x2 v[BK / 4];
};

// Stored element (r, c) of a unit-lower operand: 0 above, 1 on the diagonal.
__device__ __forceinline__ double unit_lower(double v, int64_t r, int64_t c) {
  return r < c ? 0.0 : (r == c ? 1.0 : v);
}

// Load the R x BK block of op(X) starting at (x0, k0) where op(X)[i][p] is
// X[x0+i + (k0+p)*ld] (ALONG_R) or X[k0+p + (x0+i)*ld] (!ALONG_R).
// FULL: no bounds tests (the block lies inside [0,R) x [k0,kend)).
// MASK: apply the unit-lower mask of the stored operand.
template <int BK, bool ALONG_R, bool FULL, bool MASK>
__device__ __forceinline__ void stage_load(Stage<BK, ALONG_R>& st, const double* __restrict__ X, int64_t ld, int x0,
                                           int xlim, int k0, int kend) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < BK / 4; ++s) {
    const int v = tid + 256 * s;
    int i0, i1, p0, p1;
    if (ALONG_R) {
      i0 = 2 * (v & 63);
      i1 = i0 + 1;
      p0 = p1 = v >> 6;
    } else {
      p0 = 2 * (v & (BK / 2 - 1));
      p1 = p0 + 1;
      i0 = i1 = v / (BK / 2);
    }
    const int gi0 = x0 + i0, gi1 = x0 + i1, gp0 = k0 + p0, gp1 = k0 + p1;
    // stored coordinates (row, column) of the two elements
    const int64_t r0 = ALONG_R ? gi0 : gp0, c0 = ALONG_R ? gp0 : gi0;
    const int64_t r1 = ALONG_R ? gi1 : gp1, c1 = ALONG_R ? gp1 : gi1;
    f64x2 val;
    if (FULL) {
      val = *reinterpret_cast<const f64x2*>(X + r0 + c0 * ld);
    } else {
      val[0] = (gi0 < xlim && gp0 < kend) ? X[r0 + c0 * ld] : 0.0;
      val[1] = (gi1 < xlim && gp1 < kend) ? X[r1 + c1 * ld] : 0.0;
    }
    if (MASK) {
      val[0] = unit_lower(val[0], r0, c0);
      val[1] = unit_lower(val[1], r1, c1);
      if (!FULL) {
        if (!(gi0 < xlim && gp0 < kend)) val[0] = 0.0;
        if (!(gi1 < xlim && gp1 < kend)) val[1] = 0.0;
      }
    }
    st.v[s] = val;
  }
}

// LDS image of a tile (layout lidx): element (p, i), p in [0, BK), i in [0, R);
// ABS stores magnitudes (|.| products for checksum thresholds)
template <int BK, bool ALONG_R, bool ABS>
__device__ __forceinline__ void stage_store(const Stage<BK, ALONG_R>& st, double* S) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < BK / 4; ++s) {
    const int v = tid + 256 * s;
    f64x2 x = st.v[s];
    if (ABS) {
      x[0] = fabs(x[0]);
      x[1] = fabs(x[1]);
    }
    if (ALONG_R) {
      *reinterpret_cast<f64x2*>(&S[lidx<BK, true>(v >> 6, 2 * (v & 63))]) = x;
    } else {
      const int p = 2 * (v & (BK / 2 - 1)), i = v / (BK / 2);
      *reinterpret_cast<f64x2*>(&S[lidx<BK, false>(p, i)]) = x;
    }
  }
}

// inverse of the column-major enumeration of the lower tiles of a T x T grid:
// column c holds T - c tiles, S(c) = c*T - c(c-1)/2 precede it
__device__ __forceinline__ void lower_tile(int lin, int T, int& tm, int& tn) {
  const double b = 2.0 * T + 1.0;
  int c = (int)((b - sqrt(b * b - 8.0 * lin)) * 0.5);
  c = max(0, min(c, T - 1));
  auto S = [&](int x) { return (int)((int64_t)x * T - ((int64_t)x * (x - 1)) / 2); };
  while (c > 0 && S(c) > lin) --c;
  while (c + 1 < T && S(c + 1) <= lin) ++c;
  tn = c;
  tm = c + (lin - S(c));
}

}  // namespace

// FA: operand modes, bit 0 the unit-lower mask on the stored A, bit 1 |op(A)|,
// bit 2 |op(B)| (magnitude products), bit 3 the unit-lower mask on the
// stored B.  TRI: the grid enumerates only the
// lower tiles of a square T x T grid (requires LOWER, M == N, doff == 0).
// ROLE only separates the launches of the trailing-matrix update (1) from
// the other products (0) in profiles.
template <int TA, int TB, int FA, int LOWER, int TRI, int ROLE, int BK>
__global__ __launch_bounds__(256, BK == 16 ? 2 : 1) void k_dgemm(int M, int N, int K, double alpha,
                                                                 const double* __restrict__ A, int64_t lda,
                                                                 const double* __restrict__ B, int64_t ldb,
                                                                 double beta, double* __restrict__ C, int64_t ldc,
                                                                 int64_t doff, int kc, double* __restrict__ P) {
  constexpr int BM = DG_BM, BN = DG_BN;
  __shared__ __attribute__((aligned(16))) double As[2][lds_elems<BK, TA == 0>()];
  __shared__ __attribute__((aligned(16))) double Bs[2][lds_elems<BK, TB == 1>()];

  const int tilesM = (M + BM - 1) / BM, tilesN = (N + BN - 1) / BN;
  const int nt = TRI ? tilesM * (tilesM + 1) / 2 : tilesM * tilesN;
  int lin = blockIdx.x;
  if ((nt & 7) == 0) lin = (lin & 7) * (nt >> 3) + (lin >> 3);
  int tm, tn;
  if (TRI) {
    lower_tile(lin, tilesM, tm, tn);
  } else {
    const int g = lin / (DG_GM * tilesN);
    const int rbase = g * DG_GM;
    const int rows = min(DG_GM, tilesM - rbase);
    const int rem = lin - g * DG_GM * tilesN;
    tm = rbase + rem % rows;
    tn = rem / rows;
  }
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
  const bool inner = (m0 + BM <= M) && (n0 + BN <= N);

  Stage<BK, TA == 0> sa;
  Stage<BK, TB == 1> sb;
  // A's stored operand needs its mask only where the tile meets the diagonal
  auto load = [&](int k0) {
    const bool full = inner && (k0 + BK <= kend);
    const bool needmask =
        (FA & 1) && (TA == 0 ? (m0 < k0 + BK) : (k0 < m0 + BM));  // some stored row <= stored column
    const bool needmask_b =
        (FA & 8) && (TB == 0 ? (k0 < n0 + BN) : (n0 < k0 + BK));  // (same test on the stored B)
    if (full) {
      if ((FA & 1) && needmask)
        stage_load<BK, TA == 0, true, true>(sa, A, lda, m0, M, k0, kend);
      else
        stage_load<BK, TA == 0, true, false>(sa, A, lda, m0, M, k0, kend);
      if ((FA & 8) && needmask_b)
        stage_load<BK, TB == 1, true, true>(sb, B, ldb, n0, N, k0, kend);
      else
        stage_load<BK, TB == 1, true, false>(sb, B, ldb, n0, N, k0, kend);
    } else {
      stage_load<BK, TA == 0, false, (FA & 1) != 0>(sa, A, lda, m0, M, k0, kend);
      stage_load<BK, TB == 1, false, (FA & 8) != 0>(sb, B, ldb, n0, N, k0, kend);
    }
  };
  auto store = [&](int buf) {
    stage_store<BK, TA == 0, (FA & 2) != 0>(sa, As[buf]);
    stage_store<BK, TB == 1, (FA & 4) != 0>(sb, Bs[buf]);
  };

  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

  const int KT = (kend - kbeg + BK - 1) / BK;
  if (KT > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  const int kl = lane >> 4, il = lane & 15;
  // D = C^T layout: acc[ci][ri][r] is C(gi, gj) with gi = m0 + wm*64 + ri*16 + il,
  // gj = n0 + wn*64 + ci*16 + 4r + kl; sixteen lanes write 128 contiguous bytes.
  // Interior tiles read their C values during the last K step (the epilogue
  // then finds them in registers instead of waiting on memory).
  const bool straddle = LOWER && (int64_t)m0 + doff < (int64_t)(n0 + BN - 1);
  // (read ahead only with one workgroup per CU: with two, the other one's
  // products cover the wait, and the registers are needed)
  const bool fastC = BK == 32 && inner && !straddle && beta != 0.0;
  double cpre[4][4][4];
  auto loadC = [&]() {
#pragma unroll
    for (int ci = 0; ci < 4; ++ci)
#pragma unroll
      for (int ri = 0; ri < 4; ++ri)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = m0 + wm * 64 + ri * 16 + il, gj = n0 + wn * 64 + ci * 16 + 4 * r + kl;
          cpre[ci][ri][r] = C[gi + (int64_t)gj * ldc];
        }
  };
  auto step = [&](int cur) {
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      double af[4], bf[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        af[q] = As[cur][lidx<BK, TA == 0>(kk * 4 + kl, wm * 64 + q * 16 + il)];
        bf[q] = Bs[cur][lidx<BK, TB == 1>(kk * 4 + kl, wn * 64 + q * 16 + il)];
      }
#pragma unroll
      for (int ci = 0; ci < 4; ++ci)
#pragma unroll
        for (int ri = 0; ri < 4; ++ri)
          acc[ci][ri] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[ci], af[ri], acc[ci][ri], 0, 0, 0);
    }
    // the scheduler's MFMA / LDS-read interleave for one wave's GEMM loop
    // (measured with 16-deep steps: +11% on the long-K V^T C product, +1% on
    // the K = nb ones; with 32-deep steps it cost 10-15%, so those keep the
    // default schedule)
    if constexpr (BK == 16) __builtin_amdgcn_iglp_opt(1);
  };
  for (int kt = 0; kt + 1 < KT; ++kt) {
    const int cur = kt & 1;
    load(kbeg + (kt + 1) * BK);
    step(cur);
    store(cur ^ 1);
    __syncthreads();
  }
  // last K step (peeled: no operand loads in flight, C's values instead)
  if (fastC) loadC();
  if (KT > 0) step((KT - 1) & 1);

  if (inner && !straddle) {
#pragma unroll
    for (int ci = 0; ci < 4; ++ci)
#pragma unroll
      for (int ri = 0; ri < 4; ++ri)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = m0 + wm * 64 + ri * 16 + il, gj = n0 + wn * 64 + ci * 16 + 4 * r + kl;
          const double v = alpha * acc[ci][ri][r];
          C[gi + (int64_t)gj * ldc] = fastC ? beta * cpre[ci][ri][r] + v : (beta == 0.0 ? v : beta * C[gi + (int64_t)gj * ldc] + v);
        }
  } else {
#pragma unroll
    for (int ci = 0; ci < 4; ++ci)
#pragma unroll
      for (int ri = 0; ri < 4; ++ri)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = m0 + wm * 64 + ri * 16 + il, gj = n0 + wn * 64 + ci * 16 + 4 * r + kl;
          if (gi < M && gj < N && (!LOWER || (int64_t)gi + doff >= (int64_t)gj)) {
            double* p = C + gi + (int64_t)gj * ldc;
            const double v = alpha * acc[ci][ri][r];
            *p = (beta == 0.0) ? v : beta * (*p) + v;
          }
        }
  }
}

// Returns 1 when the product was launched here, 0 when the caller should use
// the general kernel (unsupported option combination or alignment), <0 on error.
// fa: 0 plain, 1 unit-lower A, 2 |A|, 3 |unit-lower A|; fb: 0 plain, 1
// unit-lower B, 2 |B|.
int dgemm_fast(hipStream_t s, int ta, int tb, int fa, int fb, int lower, int m, int n, int k, double alpha,
               const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
               int64_t doff, int S, int kc, double* ws, int role) {
  if (fa < 0 || fa > 3 || fb < 0 || fb > 2) return 0;
  const int modes = fa | (fb == 2 ? 4 : 0) | (fb == 1 ? 8 : 0);
  if ((reinterpret_cast<uintptr_t>(A) & 15) || (reinterpret_cast<uintptr_t>(B) & 15) || (lda & 1) || (ldb & 1))
    return 0;
  const int64_t tM = (m + DG_BM - 1) / DG_BM, tN = (n + DG_BN - 1) / DG_BN;
  const bool tri = lower && m == n && doff == 0 && S == 1;
  const int64_t nt = tri ? tM * (tM + 1) / 2 : tM * tN;
  if (nt > 0x7fffffff) return 0;
  const dim3 grid((unsigned)nt, (unsigned)S), block(256);
#define DG_LAUNCH(TA_, TB_, FA_, LO_, TRI_, RO_, BK_)                                                             \
  hipLaunchKernelGGL((k_dgemm<TA_, TB_, FA_, LO_, TRI_, RO_, BK_>), grid, block, 0, s, m, n, k, alpha, A, lda, B, ldb, \
                     beta, C, ldc, doff, kc, ws)
#define DG_CASE(TA_, TB_, FA_, LO_)                                                                              \
  if (ta == TA_ && tb == TB_ && modes == FA_ && lower == LO_) {                                                    \
    if (LO_ && tri) {                                                                                              \
      if (role) DG_LAUNCH(TA_, TB_, FA_, LO_, LO_, 1, 16); else DG_LAUNCH(TA_, TB_, FA_, LO_, LO_, 0, 16);         \
    } else {                                                                                                       \
      if (role) DG_LAUNCH(TA_, TB_, FA_, LO_, 0, 1, 16); else DG_LAUNCH(TA_, TB_, FA_, LO_, 0, 0, 16);             \
    }                                                                                                              \
    return hipGetLastError() == hipSuccess ? 1 : ABFT_ERR_HIP;                                                     \
  }
  // trailing-update products with 32-deep K tiles (role 2; split-K launches keep 16)
#define DG_CASE32(TA_, TB_, FA_, LO_)                                                                            \
  if (role == 2 && S == 1 && ta == TA_ && tb == TB_ && modes == FA_ && lower == LO_) {                           \
    if (LO_ && tri) DG_LAUNCH(TA_, TB_, FA_, LO_, LO_, 1, 32); else DG_LAUNCH(TA_, TB_, FA_, LO_, 0, 1, 32);       \
    return hipGetLastError() == hipSuccess ? 1 : ABFT_ERR_HIP;                                                     \
  }
  DG_CASE32(0, 0, 0, 0)
  DG_CASE32(0, 1, 0, 1)
  DG_CASE32(1, 0, 1, 0)
  DG_CASE32(0, 0, 1, 0)
  DG_CASE(0, 0, 0, 0)  // C -= L21 U12 (LU), TRSM block updates
  DG_CASE(0, 1, 0, 1)  // C -= L21 L21^T, lower part (Cholesky)
  DG_CASE(0, 1, 0, 0)  // X Y^T
  DG_CASE(1, 0, 1, 0)  // W = V^T C (QR)
  DG_CASE(0, 0, 1, 0)  // C -= V W (QR)
  DG_CASE(0, 0, 4, 0)  // magnitude products of the checksum carries: S |Y|
  DG_CASE(0, 1, 4, 0)  //   S |Y^T| (symmetric update)
  DG_CASE(0, 0, 2, 0)  //   |X| T
  DG_CASE(0, 1, 2, 0)  //   |X| S^T (symmetric update)
  DG_CASE(0, 0, 3, 0)  //   |V| T (unit-lower V)
  DG_CASE(1, 0, 0, 0)  // T^T W (QR)
  DG_CASE(1, 0, 8, 0)  // V1^T V2, V2 unit lower (QR T merge)
  DG_CASE(1, 0, 6, 0)  // |V|^T |R| (QR panel check)
#undef DG_CASE
#undef DG_CASE32
#undef DG_LAUNCH
  return 0;
}

}  // namespace abft
