// Diagnostics of the SIPF-W state on gfx950: float64 mass sums (Corollary mass: total particle
// mass; partition of unity: h^3 sum ubar equals it), minima / maxima for the positivity
// lemma and Lemma mass, and counts of non-finite and negative values.
//
// One reset kernel (one block per simulation) advances the device step counter when asked
// and clears the accumulators; the reduction kernel then folds every particle and node into
// per-block partials (wavefront shuffles, then LDS) and one atomic per block and slot.
#include "sipf_internal.h"

namespace sipf {

template <typename T>
__global__ void k_diag_reset(Batch<T> bt, int advance_step) {
  const SimDev<T>& d = bt.sims[blockIdx.x];
  if (threadIdx.x == 0 && advance_step) *d.step += 1;
  if (threadIdx.x < D_COUNT) {
    unsigned long long v = 0ull;
    const int sl = threadIdx.x;
    if (sl == D_MIN_V || sl == D_MIN_M || sl == D_MIN_W || sl == D_MIN_A || sl == D_MIN_U)
      v = ~0ull;
    d.diag[sl] = v;
  }
}

struct Acc {
  double sa, su, sm;
  double mnv, mnm, mnw, mxm, mxw, mna, mxa, mnu;
  unsigned long long nan, negm, negw;
};

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ unsigned long long shfl_xor_u(unsigned long long v, int m) {
  return __shfl_xor(v, m, 64);
}

__device__ void wave_reduce(Acc& a) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    a.sa += shfl_xor_d(a.sa, m);
    a.su += shfl_xor_d(a.su, m);
    a.sm += shfl_xor_d(a.sm, m);
    a.mnv = fmin(a.mnv, shfl_xor_d(a.mnv, m));
    a.mnm = fmin(a.mnm, shfl_xor_d(a.mnm, m));
    a.mnw = fmin(a.mnw, shfl_xor_d(a.mnw, m));
    a.mxm = fmax(a.mxm, shfl_xor_d(a.mxm, m));
    a.mxw = fmax(a.mxw, shfl_xor_d(a.mxw, m));
    a.mna = fmin(a.mna, shfl_xor_d(a.mna, m));
    a.mxa = fmax(a.mxa, shfl_xor_d(a.mxa, m));
    a.mnu = fmin(a.mnu, shfl_xor_d(a.mnu, m));
    a.nan += shfl_xor_u(a.nan, m);
    a.negm += shfl_xor_u(a.negm, m);
    a.negw += shfl_xor_u(a.negw, m);
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_diag(Batch<T> bt) {
  int lb;
  const int s = find_sim(bt, K_DIAG, lb);
  const SimDev<T>& d = bt.sims[s];
  const int* off = bt.blk + K_DIAG * (bt.nsims + 1);
  const int nb = off[s + 1] - off[s];
  const double inf = __builtin_inf();
  Acc a = {0, 0, 0, inf, inf, inf, -inf, -inf, inf, -inf, inf, 0ull, 0ull, 0ull};
  const int64_t stride = (int64_t)nb * kThreads;
  for (int64_t i = (int64_t)lb * kThreads + threadIdx.x; i < d.P; i += stride) {
    const double am = d.as[0][i];
    const bool bad = !isfinite(am) || !isfinite((double)d.xs[0][i]) ||
                     !isfinite((double)d.ys[0][i]) || !isfinite((double)d.zs[0][i]);
    if (bad) {
      a.nan += 1;
    } else {
      a.sa += am;
      a.mna = fmin(a.mna, am);
      a.mxa = fmax(a.mxa, am);
    }
  }
  const int64_t G = (int64_t)d.N * d.N * d.N;
  for (int64_t i = (int64_t)lb * kThreads + threadIdx.x; i < G; i += stride) {
    const double u = d.ubar[i], v = d.v[i], m = d.m[i], w = d.w[i];
    if (!isfinite(u) || !isfinite(v) || !isfinite(m) || !isfinite(w)) {
      a.nan += 1;
      continue;
    }
    a.su += u;
    a.sm += m;
    a.mnu = fmin(a.mnu, u);
    a.mnv = fmin(a.mnv, v);
    a.mnm = fmin(a.mnm, m);
    a.mnw = fmin(a.mnw, w);
    a.mxm = fmax(a.mxm, m);
    a.mxw = fmax(a.mxw, w);
    a.negm += m < 0.0;
    a.negw += w < 0.0;
  }
  wave_reduce(a);
  __shared__ Acc part[kThreads / 64];
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) part[wid] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    Acc r = part[0];
    for (int k = 1; k < kThreads / 64; ++k) {
      const Acc& o = part[k];
      r.sa += o.sa; r.su += o.su; r.sm += o.sm;
      r.mnv = fmin(r.mnv, o.mnv); r.mnm = fmin(r.mnm, o.mnm); r.mnw = fmin(r.mnw, o.mnw);
      r.mxm = fmax(r.mxm, o.mxm); r.mxw = fmax(r.mxw, o.mxw);
      r.mna = fmin(r.mna, o.mna); r.mxa = fmax(r.mxa, o.mxa); r.mnu = fmin(r.mnu, o.mnu);
      r.nan += o.nan; r.negm += o.negm; r.negw += o.negw;
    }
    unsigned long long* g = d.diag;
    unsafeAtomicAdd(reinterpret_cast<double*>(&g[D_SUM_A]), r.sa);
    unsafeAtomicAdd(reinterpret_cast<double*>(&g[D_SUM_U]), r.su);
    unsafeAtomicAdd(reinterpret_cast<double*>(&g[D_SUM_M]), r.sm);
    if (r.mnv < inf) atomicMin(&g[D_MIN_V], order_key(r.mnv));
    if (r.mnm < inf) atomicMin(&g[D_MIN_M], order_key(r.mnm));
    if (r.mnw < inf) atomicMin(&g[D_MIN_W], order_key(r.mnw));
    if (r.mxm > -inf) atomicMax(&g[D_MAX_M], order_key(r.mxm));
    if (r.mxw > -inf) atomicMax(&g[D_MAX_W], order_key(r.mxw));
    if (r.mna < inf) atomicMin(&g[D_MIN_A], order_key(r.mna));
    if (r.mxa > -inf) atomicMax(&g[D_MAX_A], order_key(r.mxa));
    if (r.mnu < inf) atomicMin(&g[D_MIN_U], order_key(r.mnu));
    if (r.nan) atomicAdd(&g[D_NAN], r.nan);
    if (r.negm) atomicAdd(&g[D_NEG_M], r.negm);
    if (r.negw) atomicAdd(&g[D_NEG_W], r.negw);
  }
}

template <typename T>
void launch_diag(const Batch<T>& b, int nblk, int nsims, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_reset<T>, dim3(nsims), dim3(64), 0, st, b, 0);
  if (nblk > 0) hipLaunchKernelGGL(k_diag<T>, dim3(nblk), dim3(kThreads), 0, st, b);
}

// variant used inside a step: also advances the step counter
template <typename T>
void launch_diag_step(const Batch<T>& b, int nblk, int nsims, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_reset<T>, dim3(nsims), dim3(64), 0, st, b, 1);
  if (nblk > 0) hipLaunchKernelGGL(k_diag<T>, dim3(nblk), dim3(kThreads), 0, st, b);
}

template void launch_diag<double>(const Batch<double>&, int, int, hipStream_t);
template void launch_diag<float>(const Batch<float>&, int, int, hipStream_t);
template void launch_diag_step<double>(const Batch<double>&, int, int, hipStream_t);
template void launch_diag_step<float>(const Batch<float>&, int, int, hipStream_t);

}  // namespace sipf
