// Device helpers shared by the gfx950 kernels of the ABFT library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/abft.h"

namespace abft {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Compensated accumulation (value s + c).  Knuth's two-sum and an FMA-based
// two-product keep the checksum arithmetic free of its own rounding, so a
// carried-vs-recomputed comparison sees the data's rounding only.  The whole
// library is compiled with -ffp-contract=off, so no product is fused behind
// the back of these error-free transformations.
// ---------------------------------------------------------------------------
struct acc2 {
  double s, c;
};
__device__ __forceinline__ void cadd(acc2& a, double x) {
  double t = a.s + x;
  double bp = t - a.s;
  a.c += (a.s - (t - bp)) + (x - bp);
  a.s = t;
}
__device__ __forceinline__ void cfma(acc2& a, double x, double y) {
  double p = x * y;
  double e = __fma_rn(x, y, -p);
  cadd(a, p);
  a.c += e;
}
__device__ __forceinline__ void cmerge(acc2& a, const acc2& b) {
  cadd(a, b.s);
  a.c += b.c;
}
__device__ __forceinline__ double cval(const acc2& a) { return a.s + a.c; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ acc2 wave_csum(acc2 a) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    acc2 b;
    b.s = __shfl_xor(a.s, o);
    b.c = __shfl_xor(a.c, o);
    cmerge(a, b);
  }
  return a;
}

// threshold of a trailing-tile comparison: tau = ts*u*(4a + g); a comparison
// fails when |d| > tau, when d is NaN, or when tau is not finite
__device__ __forceinline__ double tau_verify(double tsu, double a, double g) { return (4.0 * tsu) * a + tsu * g; }
__device__ __forceinline__ bool bad(double d, double tau) { return !(fabs(d) <= tau) || !(tau <= 1.79e308); }

// report updates (device-resident abft_report)
__device__ __forceinline__ void rep_max_ratio(abft_report* r, double v) {
  if (!(v >= 0.0) || !(v <= 1.79e308)) return;
  atomicMax(reinterpret_cast<unsigned long long*>(&r->max_ratio), (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ void rep_event(abft_report* r, int iter, int kind, int64_t row, int64_t col) {
  int slot = atomicAdd(&r->nev, 1);
  if (slot < ABFT_MAX_EVENTS) {
    r->ev[slot].iter = iter;
    r->ev[slot].kind = kind;
    r->ev[slot].row = row;
    r->ev[slot].col = col;
  }
}
__device__ __forceinline__ void rep_flag_iter(abft_report* r, int iter) { atomicMin(&r->first_flag_iter, iter); }

}  // namespace abft
