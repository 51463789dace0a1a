// Residual resampling (Alg. res_res) of one simulation's particles on gfx950.
//
// The P weighted particles are replaced by P particles of mass a0 = (1/P) sum_p a_p: particle
// p is copied k_p = floor(a_p / a0) times and the P - sum_p k_p others are drawn with
// probabilities proportional to the residuals r_p = a_p - k_p a0.  To make the particle list
// a function of the input alone (not of the order of floating-point reductions):
//
//   * the mass sum is exact: every a_p is added as an integer multiple of a power of two into
//     a 256-bit fixed-point accumulator anchored 160 binades below the largest mass, and the
//     total is rounded once (to nearest, ties to even) before the division by P;
//   * the residual of particle p is carried as R_p = floor((q_p - k_p) 2^32), q_p = a_p / a0,
//     i.e. r_p / a0 in 32-bit fixed point, so its prefix sums are exact integers;
//   * draw j takes two Philox4x32-10 words at counter (j, n, sim_lo, sim_hi | 2^31), key
//     (seed_lo, seed_hi), u = r0 + 2^32 r1, target t = floor(u R_tot / 2^64), and selects the
//     particle whose prefix-sum interval holds t.
//
// The output list is the deterministic copies in particle order, then the drawn particles in
// draw order.  Particle order is the input order given at initialisation (the particle
// index), not the tile order the step keeps: the particles are first scattered back to it.
//
// Kernels, in launch order (all on the simulation's stream):
//   k_rs_unsort   set 0 (tile order) -> set 1 (particle order); largest mass; input checks
//   k_rs_sum      exact fixed-point sum of the masses
//   k_rs_mean     one thread: round the sum, a0 = S / P
//   k_rs_blocks   per block of kScanBlock particles: sum of k_p and of R_p
//   k_rs_offsets  one block: exclusive scan of the block sums, totals
//   k_rs_prefix   per particle: exclusive prefix of k (into set 1's index array) and
//                 inclusive prefix of R (into the binning key array)
//   k_rs_gather   output particle i -> its source by binary search, written into set 0
#include "sipf_internal.h"

namespace sipf {

namespace {

constexpr int kRsThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanBlock = kRsThreads * kScanPer;  // particles per scan block
constexpr int kAnchor = 160;                        // binades kept below the largest mass
constexpr int kDigits = 8;                          // 32-bit digits of the accumulator

__device__ __forceinline__ uint64_t wave_max(uint64_t x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const uint64_t y = __shfl_xor(x, m, 64);
    x = y > x ? y : x;
  }
  return x;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

// inclusive prefix sum over the lanes of a wavefront
__device__ __forceinline__ uint64_t wave_scan(uint64_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Inclusive prefix over the block of two counters; returns the block totals in tk, tr.
// Every thread of the block must call it.
template <int NT>
__device__ __forceinline__ void block_scan2(uint64_t& k, uint64_t& r, uint64_t& tk, uint64_t& tr) {
  __shared__ uint64_t wk[NT / 64], wr[NT / 64];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  k = wave_scan(k);
  r = wave_scan(r);
  __syncthreads();
  if (lane == 63) {
    wk[wid] = k;
    wr[wid] = r;
  }
  __syncthreads();
  uint64_t ok = 0, orr = 0;
  tk = 0;
  tr = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wid) {
      ok += wk[w];
      orr += wr[w];
    }
    tk += wk[w];
    tr += wr[w];
  }
  k += ok;
  r += orr;
}

// Split of a non-negative double into m 2^(e - 1075), e >= 1 (subnormals: e = 1).
__device__ __forceinline__ void decompose(double a, uint64_t& m, int& e) {
  const uint64_t b = (uint64_t)__double_as_longlong(a);
  e = (int)(b >> 52);
  m = b & ((1ull << 52) - 1);
  if (e == 0)
    e = 1;
  else
    m |= 1ull << 52;
}

// q_p, k_p and R_p of one mass
__device__ __forceinline__ void split_mass(double a, double a0, uint32_t& k, uint32_t& R) {
  const double q = a / a0;  // IEEE division (correctly rounded)
  const double fk = floor(q);
  k = (uint32_t)fk;
  R = (uint32_t)floor((q - fk) * 4294967296.0);  // q - k is exact; the product too
}

template <typename T>
__global__ void __launch_bounds__(kRsThreads)
    k_rs_unsort(const T* __restrict__ x0, const T* __restrict__ y0, const T* __restrict__ z0,
                const double* __restrict__ a0, const uint32_t* __restrict__ id0, T* x1, T* y1,
                T* z1, double* a1, int64_t P, unsigned long long* rs) {
  uint64_t mx = 0;
  unsigned long long bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)kRsThreads + threadIdx.x; e < P;
       e += (int64_t)gridDim.x * kRsThreads) {
    const uint32_t p = id0[e];
    const double a = a0[e];
    x1[p] = x0[e];
    y1[p] = y0[e];
    if (z0) z1[p] = z0[e];  // no z coordinate in 2D
    a1[p] = a;
    if (!(a >= 0.0) || !isfinite(a)) {
      bad |= RS_BAD_VALUE;
    } else {
      const uint64_t b = (uint64_t)__double_as_longlong(a);
      mx = b > mx ? b : mx;
    }
  }
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0 && mx) atomicMax(&rs[RS_MAXBITS], (unsigned long long)mx);
  if (bad) atomicOr(&rs[RS_FLAGS], bad);
}

// Exact sum: mass m 2^(e-1075) enters as m << (e - B) with B = E_max - kAnchor, spread over
// three 32-bit digits; each block normalises its carries before adding its digits.
__global__ void __launch_bounds__(kRsThreads)
    k_rs_sum(const double* __restrict__ a1, int64_t P, unsigned long long* rs) {
  const int emax = (int)(rs[RS_MAXBITS] >> 52);
  const int base = emax - kAnchor;
  uint64_t acc[kDigits];
#pragma unroll
  for (int k = 0; k < kDigits; ++k) acc[k] = 0;
  unsigned long long bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)kRsThreads + threadIdx.x; e < P;
       e += (int64_t)gridDim.x * kRsThreads) {
    const double a = a1[e];
    if (!(a > 0.0) || !isfinite(a)) continue;  // zeros add nothing; bad values are flagged
    uint64_t m;
    int ex;
    decompose(a, m, ex);
    const int s = ex - base;
    if (s < 0) {
      bad |= RS_BAD_RANGE;
      continue;
    }
    const int d = s >> 5, off = s & 31;
    const uint64_t lo = m << off;
    const uint64_t hi = off ? (m >> (64 - off)) : 0;
    const uint64_t c0 = lo & 0xFFFFFFFFull, c1 = lo >> 32, c2 = hi;
#pragma unroll
    for (int k = 0; k < kDigits; ++k) {
      acc[k] += k == d ? c0 : 0;
      acc[k] += k == d + 1 ? c1 : 0;
      acc[k] += k == d + 2 ? c2 : 0;
    }
  }
  __shared__ uint64_t part[kRsThreads / 64][kDigits];
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kDigits; ++k) acc[k] = wave_sum(acc[k]);
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < kDigits; ++k) part[wid][k] = acc[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t carry = 0;
    for (int k = 0; k < kDigits; ++k) {
      uint64_t t = carry;
      for (int w = 0; w < kRsThreads / 64; ++w) t += part[w][k];
      const uint64_t dgt = t & 0xFFFFFFFFull;
      carry = t >> 32;
      if (dgt) atomicAdd(&rs[RS_DIGITS + k], (unsigned long long)dgt);
    }
    if (carry) bad |= RS_BAD_RANGE;  // cannot happen below 2^31 particles
  }
  if (bad) atomicOr(&rs[RS_FLAGS], bad);
}

// Round the fixed-point sum to the nearest double (ties to even) and divide by P.
__global__ void k_rs_mean(int64_t P, unsigned long long* rs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int emax = (int)(rs[RS_MAXBITS] >> 52);
  // the sum must stay a normal double: largest mass in [2^-775, 2^990)
  if (emax < 300 || emax > 2013) {
    atomicOr(&rs[RS_FLAGS], RS_BAD_RANGE);
    return;
  }
  uint32_t dg[kDigits];
  uint64_t carry = 0;
  for (int k = 0; k < kDigits; ++k) {
    const uint64_t t = rs[RS_DIGITS + k] + carry;
    dg[k] = (uint32_t)t;
    carry = t >> 32;
  }
  if (carry) {
    atomicOr(&rs[RS_FLAGS], RS_BAD_RANGE);
    return;
  }
  int top = -1;  // index of the highest set bit
  for (int k = kDigits - 1; k >= 0 && top < 0; --k)
    if (dg[k]) top = 32 * k + 31 - __builtin_clz(dg[k]);
  if (top < 0) {  // every mass is zero
    atomicOr(&rs[RS_FLAGS], RS_BAD_VALUE);
    return;
  }
  auto bit = [&](int i) -> uint64_t { return i < 0 ? 0 : (dg[i >> 5] >> (i & 31)) & 1u; };
  int exp2 = top - 52;  // the sum is mant 2^exp2 (in units of the accumulator's lowest bit)
  uint64_t mant = 0;
  if (exp2 <= 0) {  // at most 53 significant bits: exact
    for (int i = top; i >= 0; --i) mant = (mant << 1) | bit(i);
    exp2 = 0;
  } else {
    for (int i = top; i >= exp2; --i) mant = (mant << 1) | bit(i);
    const uint64_t guard = bit(exp2 - 1);
    uint64_t sticky = 0;
    for (int i = exp2 - 2; i >= 0; --i) sticky |= bit(i);
    if (guard && (sticky || (mant & 1))) {  // round to nearest, ties to even
      mant += 1;
      if (mant >> 53) {
        mant >>= 1;
        exp2 += 1;
      }
    }
  }
  const double S = ldexp((double)mant, exp2 + (emax - kAnchor) - 1075);
  const double a0 = S / (double)P;
  rs[RS_A0] = (unsigned long long)__double_as_longlong(a0);
}

__global__ void __launch_bounds__(kRsThreads)
    k_rs_blocks(const double* __restrict__ a1, int64_t P, unsigned long long* rs) {
  const double a0 = __longlong_as_double((long long)rs[RS_A0]);
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint64_t sk = 0, sr = 0;
#pragma unroll 4
  for (int r = 0; r < kScanPer; ++r) {
    const int64_t e = base + r * kRsThreads + threadIdx.x;
    if (e < P) {
      uint32_t k, R;
      split_mass(a1[e], a0, k, R);
      sk += k;
      sr += R;
    }
  }
  uint64_t tk, tr;
  block_scan2<kRsThreads>(sk, sr, tk, tr);
  if (threadIdx.x == 0) {
    rs[RS_BLOCKS + 2 * blockIdx.x] = tk;
    rs[RS_BLOCKS + 2 * blockIdx.x + 1] = tr;
  }
}

constexpr int kOffThreads = 1024;

__global__ void __launch_bounds__(kOffThreads) k_rs_offsets(int nb, unsigned long long* rs) {
  uint64_t ck = 0, cr = 0;
  for (int c = 0; c < nb; c += kOffThreads) {
    const int b = c + threadIdx.x;
    uint64_t k = b < nb ? rs[RS_BLOCKS + 2 * b] : 0;
    uint64_t r = b < nb ? rs[RS_BLOCKS + 2 * b + 1] : 0;
    const uint64_t k0 = k, r0 = r;
    uint64_t tk, tr;
    block_scan2<kOffThreads>(k, r, tk, tr);
    if (b < nb) {  // exclusive prefix
      rs[RS_BLOCKS + 2 * b] = ck + k - k0;
      rs[RS_BLOCKS + 2 * b + 1] = cr + r - r0;
    }
    ck += tk;
    cr += tr;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    rs[RS_KTOT] = ck;
    rs[RS_RTOT] = cr;
  }
}

__global__ void __launch_bounds__(kRsThreads)
    k_rs_prefix(const double* __restrict__ a1, int64_t P, const unsigned long long* rs,
                uint32_t* kex, uint64_t* rin) {
  const double a0 = __longlong_as_double((long long)rs[RS_A0]);
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint64_t ok = rs[RS_BLOCKS + 2 * blockIdx.x], orr = rs[RS_BLOCKS + 2 * blockIdx.x + 1];
  for (int r = 0; r < kScanPer; ++r) {
    const int64_t e = base + r * kRsThreads + threadIdx.x;
    uint32_t k = 0, R = 0;
    if (e < P) split_mass(a1[e], a0, k, R);
    uint64_t ik = k, ir = R, tk, tr;
    block_scan2<kRsThreads>(ik, ir, tk, tr);
    if (e < P) {
      kex[e] = (uint32_t)(ok + ik - k);  // exclusive: first output slot of particle e
      rin[e] = orr + ir;                 // inclusive
    }
    ok += tk;
    orr += tr;
  }
}

template <typename T>
__global__ void __launch_bounds__(kRsThreads)
    k_rs_gather(const T* __restrict__ x1, const T* __restrict__ y1, const T* __restrict__ z1,
                const uint32_t* __restrict__ kex, const uint64_t* __restrict__ rin, int64_t P,
                const unsigned long long* rs, const uint64_t* step, uint32_t seed_lo,
                uint32_t seed_hi, uint32_t sim_lo, uint32_t sim_hi, T* x0, T* y0, T* z0,
                double* a0s, uint32_t* id0) {
  const int64_t i = blockIdx.x * (int64_t)kRsThreads + threadIdx.x;
  if (i >= P) return;
  const uint64_t ktot = rs[RS_KTOT], rtot = rs[RS_RTOT];
  const int64_t kdet = ktot < (uint64_t)P ? (int64_t)ktot : P;
  int64_t src;
  if (i < kdet) {
    // last particle whose first slot is <= i
    int64_t lo = 0, hi = P;  // kex[lo] <= i < kex[hi] (kex[P] taken as +inf)
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (kex[mid] <= (uint64_t)i)
        lo = mid;
      else
        hi = mid;
    }
    src = lo;
  } else {
    uint32_t c0 = (uint32_t)(i - kdet), c1 = (uint32_t)*step, c2 = sim_lo,
             c3 = sim_hi | 0x80000000u;
    philox4x32_10(c0, c1, c2, c3, seed_lo, seed_hi);
    const uint64_t u = (uint64_t)c0 | ((uint64_t)c1 << 32);
    if (rtot > 0) {
      const uint64_t t = __umul64hi(u, rtot);
      // first particle whose inclusive prefix exceeds t
      int64_t lo = -1, hi = P - 1;  // rin[lo] <= t < rin[hi]
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (rin[mid] > t)
          hi = mid;
        else
          lo = mid;
      }
      src = hi;
    } else {
      src = (int64_t)__umul64hi(u, (uint64_t)P);
    }
  }
  x0[i] = x1[src];
  y0[i] = y1[src];
  if (z0) z0[i] = z1[src];
  a0s[i] = __longlong_as_double((long long)rs[RS_A0]);
  id0[i] = (uint32_t)i;
}

int grid_for(int64_t n) {
  const int64_t b = (n + kRsThreads - 1) / kRsThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

}  // namespace

size_t resample_scratch_words(int64_t P) {
  return RS_BLOCKS + 2 * (size_t)((P + kScanBlock - 1) / kScanBlock + 1);
}

template <typename T>
void launch_resample_stats(const SimDev<T>& d, unsigned long long* rs, hipStream_t st) {
  const int64_t P = d.P;
  const bool z = d.dim == 3;
  hipLaunchKernelGGL(k_rs_unsort<T>, dim3(grid_for(P)), dim3(kRsThreads), 0, st, d.xs[0],
                     d.ys[0], z ? d.zs[0] : nullptr, d.as[0], d.ids[0], d.xs[1], d.ys[1],
                     z ? d.zs[1] : nullptr, d.as[1], P, rs);
  hipLaunchKernelGGL(k_rs_sum, dim3(grid_for(P)), dim3(kRsThreads), 0, st, d.as[1], P, rs);
  hipLaunchKernelGGL(k_rs_mean, dim3(1), dim3(64), 0, st, P, rs);
}

template <typename T>
void launch_resample_apply(const SimDev<T>& d, unsigned long long* rs, hipStream_t st) {
  const int64_t P = d.P;
  const int nb = (int)((P + kScanBlock - 1) / kScanBlock);
  uint32_t* kex = d.ids[1];
  uint64_t* rin = reinterpret_cast<uint64_t*>(d.key);
  hipLaunchKernelGGL(k_rs_blocks, dim3(nb), dim3(kRsThreads), 0, st, d.as[1], P, rs);
  hipLaunchKernelGGL(k_rs_offsets, dim3(1), dim3(kOffThreads), 0, st, nb, rs);
  hipLaunchKernelGGL(k_rs_prefix, dim3(nb), dim3(kRsThreads), 0, st, d.as[1], P, rs, kex, rin);
  const int ng = (int)((P + kRsThreads - 1) / kRsThreads);
  const bool z = d.dim == 3;
  hipLaunchKernelGGL(k_rs_gather<T>, dim3(ng), dim3(kRsThreads), 0, st, d.xs[1], d.ys[1],
                     z ? d.zs[1] : nullptr, kex, rin, P, rs, d.step, d.seed_lo, d.seed_hi,
                     d.sim_lo, d.sim_hi, d.xs[0], d.ys[0], z ? d.zs[0] : nullptr, d.as[0],
                     d.ids[0]);
}

template void launch_resample_stats<double>(const SimDev<double>&, unsigned long long*,
                                            hipStream_t);
template void launch_resample_stats<float>(const SimDev<float>&, unsigned long long*,
                                           hipStream_t);
template void launch_resample_apply<double>(const SimDev<double>&, unsigned long long*,
                                            hipStream_t);
template void launch_resample_apply<float>(const SimDev<float>&, unsigned long long*,
                                           hipStream_t);

}  // namespace sipf
