// Block-level accumulation of the diagnostics slots (float64 sums, ordered-key minima and
// maxima, integer counts): every thread folds its values into an Acc, then one call reduces
// the block (wavefront shuffles, then LDS) and issues one atomic per slot that received data
// into one of kStripes copies of the accumulator (block index mod kStripes, each copy on its
// own 128-byte line), so that thousands of blocks do not serialise on one cache line.  The
// one-block finalize kernel folds the copies together.
#pragma once

#include "sipf_internal.h"

namespace sipf {

struct Acc {
  double sum[3];                 // D_SUM_A, D_SUM_U, D_SUM_M
  double mn[8];                  // D_MIN_V .. D_MIN_U in DiagSlot order (max slots negated)
  unsigned long long cnt[3];     // D_NAN, D_NEG_M, D_NEG_W
};

// index of slot s in Acc::mn (s in [D_MIN_V, D_MIN_U]); max slots store -value
__device__ __forceinline__ bool slot_is_max(int s) {
  return s == D_MAX_M || s == D_MAX_W || s == D_MAX_A;
}

__device__ __forceinline__ void acc_init(Acc& a) {
  const double inf = __builtin_inf();
#pragma unroll
  for (int k = 0; k < 3; ++k) a.sum[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) a.mn[k] = inf;
#pragma unroll
  for (int k = 0; k < 3; ++k) a.cnt[k] = 0ull;
}

// fold a value into a min or max slot
__device__ __forceinline__ void acc_min(Acc& a, int slot, double v) {
  const int k = slot - D_MIN_V;
  a.mn[k] = fmin(a.mn[k], slot_is_max(slot) ? -v : v);
}

__device__ __forceinline__ void acc_flush(Acc& a, unsigned long long* g) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) a.sum[k] += __shfl_xor(a.sum[k], m, 64);
#pragma unroll
    for (int k = 0; k < 8; ++k) a.mn[k] = fmin(a.mn[k], __shfl_xor(a.mn[k], m, 64));
#pragma unroll
    for (int k = 0; k < 3; ++k) a.cnt[k] += __shfl_xor(a.cnt[k], m, 64);
  }
  __shared__ Acc part[kThreads / 64];
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) part[wid] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      for (int k = 0; k < 3; ++k) a.sum[k] += part[w].sum[k];
      for (int k = 0; k < 8; ++k) a.mn[k] = fmin(a.mn[k], part[w].mn[k]);
      for (int k = 0; k < 3; ++k) a.cnt[k] += part[w].cnt[k];
    }
    const double inf = __builtin_inf();
    for (int k = 0; k < 3; ++k)
      if (a.sum[k] != 0.0) unsafeAtomicAdd(reinterpret_cast<double*>(&g[D_SUM_A + k]), a.sum[k]);
    for (int k = 0; k < 8; ++k) {
      if (a.mn[k] < inf) {
        const int slot = D_MIN_V + k;
        if (slot_is_max(slot))
          atomicMax(&g[slot], order_key(-a.mn[k]));
        else
          atomicMin(&g[slot], order_key(a.mn[k]));
      }
    }
    for (int k = 0; k < 3; ++k)
      if (a.cnt[k]) atomicAdd(&g[D_NAN + k], a.cnt[k]);
  }
}

// accumulator copy of this block
template <typename T>
__device__ __forceinline__ unsigned long long* diag_stripe(SimC<T>& d) {
  return d.diag + (blockIdx.x & (kStripes - 1)) * kStripeWords;
}

}  // namespace sipf
