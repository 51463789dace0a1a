// Diagnostics of the SIPF-W state on gfx950: float64 mass sums (Corollary mass: total particle
// mass; partition of unity: h^3 sum ubar equals it), minima / maxima for the positivity
// lemma and Lemma mass, and counts of non-finite and negative values.
//
// The diagnostics describe the state they are read from, so they are reduced when they are
// read: one pass over the particles (masses, positions), the deposited density ubar and the
// fields v, m, w folds into striped accumulator copies, and a one-block kernel folds the
// copies into the result words and clears them.  The step's own passes carry no reduction
// (the particle pass and the z passes are bound by instruction issue, and ubar is complete
// only after the particle pass's last atomic); the kernel that ends a step only advances the
// step index.
#include "diag_acc.h"

namespace sipf {

__device__ __forceinline__ unsigned long long slot_identity(int sl) {
  if (sl >= D_MIN_V && sl <= D_MIN_U && !slot_is_max(sl)) return ~0ull;
  return 0ull;
}

// Fold the accumulator copies into the result words and clear them (one block of
// kStripes * kStripeWords threads per simulation: every thread loads one word); with
// step_end, only advance the step index.
constexpr int kFinThreads = kStripes * kStripeWords;

template <typename T>
__global__ void __launch_bounds__(kFinThreads) k_diag_finalize(Batch<T> bt, int step_end) {
  SimC<T>& d = sim_view(bt, (int)blockIdx.x);
  if (step_end) {
    if (threadIdx.x == 0) *d.step += 1;
    return;
  }
  __shared__ unsigned long long w[kFinThreads];
  const int t = threadIdx.x;
  const int sl = t % kStripeWords;
  w[t] = d.diag[t];
  d.diag[t] = slot_identity(sl);
  __syncthreads();
  // one wavefront per slot, lane c holding stripe c's word, reduced across the lanes
  static_assert(kStripes == 64 && D_COUNT <= kFinThreads / 64, "one stripe per lane");
  const int slot = t >> 6, lane = t & 63;
  if (slot < D_COUNT) {
    unsigned long long r = w[lane * kStripeWords + slot];
    if (slot < D_MIN_V) {
      double x;
      __builtin_memcpy(&x, &r, 8);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      __builtin_memcpy(&r, &x, 8);
    } else {
      const bool mx = slot_is_max(slot), cnt = slot > D_MIN_U;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long v = (unsigned long long)__shfl_xor((long long)r, o, 64);
        r = cnt ? r + v : (mx ? (v > r ? v : r) : (v < r ? v : r));
      }
    }
    if (lane == 0) d.diag[kDiagResult + slot] = r;
  }
}

// Clear every word of the diagnostics area.
template <typename T>
__global__ void k_diag_clear(Batch<T> bt) {
  SimC<T>& d = sim_view(bt, (int)blockIdx.x);
  for (int e = threadIdx.x; e < kDiagWords; e += blockDim.x)
    d.diag[e] = slot_identity(e % kStripeWords);
}

// Full reduction into the accumulator copies of what the bits of `what` select.
constexpr int kDiagParticles = 1;  // masses and positions
constexpr int kDiagGrid = 2;       // v, m, w
constexpr int kDiagU = 4;          // ubar
template <typename T>
__global__ void __launch_bounds__(kThreads) k_diag_full(Batch<T> bt, int what) {
  int lb;
  const int s = find_sim(bt, K_DIAG, lb);
  SimC<T>& d = sim_view(bt, s);
  const int* off = bt.blk + K_DIAG * (bt.nsims + 1);
  const int nb = off[s + 1] - off[s];
  Acc a;
  acc_init(a);
  const int64_t stride = (int64_t)nb * kThreads;
  const bool state = what & kDiagGrid, u = what & kDiagU;
  if (what & kDiagParticles) {
    for (int64_t i = (int64_t)lb * kThreads + threadIdx.x; i < d.P; i += stride) {
      const double am = d.as[0][i];
      const bool bad = !isfinite(am) || !isfinite((double)d.xs[0][i]) ||
                       !isfinite((double)d.ys[0][i]) ||
                       (d.dim == 3 && !isfinite((double)d.zs[0][i]));
      if (bad) {
        a.cnt[0] += 1;
      } else {
        a.sum[0] += am;
        acc_min(a, D_MIN_A, am);
        acc_min(a, D_MAX_A, am);
      }
    }
  }
  const int64_t G = d.G;
  const T* const ub = d.ubar[(uint32_t)(*d.step) & 1u];  // the state's deposit
  for (int64_t i = (int64_t)lb * kThreads + threadIdx.x; i < G; i += stride) {
    if (u) {
      const double uu = ub[i];
      if (!isfinite(uu)) {
        a.cnt[0] += 1;
      } else {
        a.sum[1] += uu;
        acc_min(a, D_MIN_U, uu);
      }
    }
    if (state) {
      const double v = d.v[i], m = d.m[i], w = d.w[i];
      if (!isfinite(v) || !isfinite(m) || !isfinite(w)) {
        a.cnt[0] += 1;
        continue;
      }
      a.sum[2] += m;
      acc_min(a, D_MIN_V, v);
      acc_min(a, D_MIN_M, m);
      acc_min(a, D_MAX_M, m);
      acc_min(a, D_MIN_W, w);
      acc_min(a, D_MAX_W, w);
      a.cnt[1] += m < 0.0;
      a.cnt[2] += w < 0.0;
    }
  }
  acc_flush(a, diag_stripe(d));
}

template <typename T>
void launch_diag_clear(const Batch<T>& b, int nsims, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_clear<T>, dim3(nsims), dim3(256), 0, st, b);
}

template <typename T>
void launch_diag_read(const Batch<T>& b, int nblk, int nsims, hipStream_t st) {
  if (nblk > 0)
    hipLaunchKernelGGL(k_diag_full<T>, dim3(nblk), dim3(kThreads), 0, st, b,
                       kDiagParticles | kDiagGrid | kDiagU);
  hipLaunchKernelGGL(k_diag_finalize<T>, dim3(nsims), dim3(kFinThreads), 0, st, b, 0);
}

template <typename T>
void launch_finalize(const Batch<T>& b, int nsims, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_finalize<T>, dim3(nsims), dim3(64), 0, st, b, 1);
}

template void launch_diag_clear<double>(const Batch<double>&, int, hipStream_t);
template void launch_diag_clear<float>(const Batch<float>&, int, hipStream_t);
template void launch_diag_read<double>(const Batch<double>&, int, int, hipStream_t);
template void launch_diag_read<float>(const Batch<float>&, int, int, hipStream_t);
template void launch_finalize<double>(const Batch<double>&, int, hipStream_t);
template void launch_finalize<float>(const Batch<float>&, int, hipStream_t);

}  // namespace sipf
