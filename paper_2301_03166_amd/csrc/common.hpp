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

// ---------------------------------------------------------------------------
// Grid-wide barrier for cooperative launches (every workgroup resident), on
// one flag word per workgroup: workgroup g stores the barrier's sequence
// number into flags[g] (release), then waits until every flag has reached it
// (one flag per polling thread, so there is no contended read-modify-write).
// Only thread 0 releases: after the workgroup barrier its agent-scope
// release (L2 write-back) covers the whole workgroup's completed stores; the
// acquire fence after the wait (L2 invalidate) covers the following loads.
// Sequence numbers increase within a use of the flags (cleared before), so a
// flag already past `seq` also counts.  The wait is bounded; on expiry the
// workgroup records ABFT_ST_INTERNAL and carries on, so every wave always
// reaches the end of the kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void flag_barrier(unsigned* flags, unsigned seq, abft_report* rep) {
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(&flags[blockIdx.x], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  for (unsigned t = threadIdx.x; t < gridDim.x; t += blockDim.x) {
    long spins = 0;
    while (__hip_atomic_load(&flags[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < seq) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1L << 21)) {
        if (rep) atomicOr(&rep->status, (int)ABFT_ST_INTERNAL);
        break;
      }
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

}  // namespace abft
