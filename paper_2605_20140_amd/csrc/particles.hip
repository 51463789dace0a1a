// Particle half of the SIPF-W step on gfx950: grid-to-particle gather (Alg. g2p), Philox
// Wiener increments, Euler-Maruyama push and mass update (eq. u_hat_update, eq. SDE), and the
// particle-to-grid deposit (Alg. p2g) of the new state, fused in one pass over the particles;
// plus the tile binning that makes that pass local.
//
// Particles are structure of arrays: x, y, z in the working precision T, masses a in
// float64, and a 32-bit particle index id that keys the noise stream, so results do not
// depend on the storage order.  Set 0 holds the state; binning scatters set 0 into set 1 by
// tile, and the particle pass that follows reads set 1 and writes its results back into
// set 0, which stays tile-ordered until the next binning.
//
// Trilinear stencil: s = x / h, i = floor(s), f = s - i; node weights (1 - f, f) per axis
// (K_h = h^3 R_h); R_h = K_h / h^3 for the deposit.  Node indices wrap modulo N.
//
// Particle pass: one block per (tile, chunk of <= kChunk particles).  The block stages the
// gather array of its tile's nodes plus a drift margin in LDS, gathers from LDS,
// deposits the new state into an LDS accumulator, and flushes every non-zero accumulator
// node to the global density with one atomic.  A particle whose stencil leaves the region
// (it drifted more than a cell since the last binning) uses global memory instead.
#include "diag_acc.h"

namespace sipf {

template <typename T>
struct Stencil {
  int c[3];  // cell index (lower node), in [0, N)
  T f[3];    // fractional offsets
};

template <typename T>
__device__ __forceinline__ Stencil<T> make_stencil(T x, T y, T z, T inv_h, int N) {
  Stencil<T> st;
  const T s[3] = {x * inv_h, y * inv_h, z * inv_h};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T fl = floor(s[j]);
    st.f[j] = s[j] - fl;
    st.c[j] = ((int)fl) & (N - 1);
  }
  return st;
}

// flat index of node (a, b, c) on the N^3 grid; 32-bit arithmetic, since N <= 512 in 3D keeps
// every index below 2^27
__device__ __forceinline__ uint32_t node(int a, int b, int c, int N) {
  return ((uint32_t)a * (uint32_t)N + (uint32_t)b) * (uint32_t)N + (uint32_t)c;
}

// Box-Muller normals from one Philox block.  float64: exact uniforms (r + 1/2) 2^-32 and
// ocml log / sqrt / sincospi.  float32: the same uniforms rounded to float32 and the
// hardware transcendentals (log2, and sin / cos that take their argument in turns).
__device__ __forceinline__ void box_muller(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3,
                                           double z[3]) {
  const double u0 = fma((double)r0, 0x1p-32, 0x1p-33);
  const double u1 = fma((double)r1, 0x1p-32, 0x1p-33);
  const double u2 = fma((double)r2, 0x1p-32, 0x1p-33);
  const double u3 = fma((double)r3, 0x1p-32, 0x1p-33);
  const double ra = sqrt(-2.0 * log(u0));
  const double rb = sqrt(-2.0 * log(u2));
  double s1, c1;
  sincospi(2.0 * u1, &s1, &c1);
  z[0] = ra * c1;
  z[1] = ra * s1;
  z[2] = rb * cospi(2.0 * u3);
}

__device__ __forceinline__ void box_muller(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3,
                                           float z[3]) {
  const float u0 = fmaf((float)r0, 0x1p-32f, 0x1p-33f);
  const float u1 = fmaf((float)r1, 0x1p-32f, 0x1p-33f);
  const float u2 = fmaf((float)r2, 0x1p-32f, 0x1p-33f);
  const float u3 = fmaf((float)r3, 0x1p-32f, 0x1p-33f);
  const float ln2x2 = -2.0f * 0.69314718055994531f;
  const float ra = __builtin_amdgcn_sqrtf(ln2x2 * __builtin_amdgcn_logf(u0));
  const float rb = __builtin_amdgcn_sqrtf(ln2x2 * __builtin_amdgcn_logf(u2));
  z[0] = ra * __builtin_amdgcn_cosf(u1);
  z[1] = ra * __builtin_amdgcn_sinf(u1);
  z[2] = rb * __builtin_amdgcn_cosf(u3);
}

// rho(w) = 2w / (1 + w) of the mass update: float64 exactly rounded; float32 with the
// hardware reciprocal (about 1 ulp), since rho enters only through exp(dt (rho - 1))
__device__ __forceinline__ double rho_of(double w) { return 2.0 * w / (1.0 + w); }
__device__ __forceinline__ float rho_of(float w) {
  return 2.0f * w * __builtin_amdgcn_rcpf(1.0f + w);
}

// Keep a loop-invariant value in a register for the whole pass.  Values read from the
// descriptor (constant address space) would otherwise be re-read inside the particle loop,
// and every scalar load is followed by a wait on the counter it shares with LDS operations,
// so the next particle would wait for the previous one's deposit atomics to drain.
// (The values are uniform; readfirstlane moves one that was computed in a vector register.)
template <typename U>
__device__ __forceinline__ U keep_in_sgpr(U v) {
  static_assert(sizeof(U) == 4 || sizeof(U) == 8, "32- or 64-bit values");
  if constexpr (sizeof(U) == 4) {
    uint32_t b = (uint32_t)__builtin_amdgcn_readfirstlane((int)__builtin_bit_cast(uint32_t, v));
    asm volatile("" : "+s"(b));
    return __builtin_bit_cast(U, b);
  } else {
    const uint64_t w = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)w);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(w >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return __builtin_bit_cast(U, (uint64_t)lo | ((uint64_t)hi << 32));
  }
}

// exp(x) for the float32 mass update outside |x| <= 1/2: x log2(e) = k + f with k an integer
// and |f| <= 1/2, 2^f by the hardware float32 exp2 (about 1 ulp) and 2^k exactly by a
// float64 ldexp, so that the result neither overflows nor underflows before float64 does.
// Relative error about (|x| + 2) 2^-24, from rounding x log2(e) to float32.  (No float64
// polynomial: its constants would occupy registers for the whole particle loop.)
__device__ __forceinline__ double exp_wide(float x) {
  if (__builtin_isinf(x)) return x > 0.0f ? (double)x : 0.0;
  const float t = x * 1.44269504088896341f;
  const float k = __builtin_rintf(t);
  return ldexp((double)__builtin_amdgcn_exp2f(t - k), (int)k);
}

// Mass update a' = a exp(x), x = tau (rho - 1).  float64: the exact exponential.  float32
// form: a' = a + a expm1(x) with expm1 by its Taylor polynomial to degree 8 in float32
// (relative truncation error below 1e-8 for |x| <= 1/2, the range of tau |rho - 1| <= tau
// <= 1/2 for w >= 0) and one float64 multiply-add, so that the mass itself is accumulated
// in float64 and the relative error of a step's factor is about |x| 2^-24; outside that
// range (w < 0 at a node of the implicit solve's small negative lobes, or non-finite)
// exp_wide.
__device__ __forceinline__ double mass_factor_update(double a, double x) {
  return a * exp(x);
}
__device__ __forceinline__ double mass_factor_update(double a, float x) {
  if (!(fabsf(x) <= 0.5f)) return a * exp_wide(x);
  float e = 1.0f / 40320.0f;
  e = fmaf(e, x, 1.0f / 5040.0f);
  e = fmaf(e, x, 1.0f / 720.0f);
  e = fmaf(e, x, 1.0f / 120.0f);
  e = fmaf(e, x, 1.0f / 24.0f);
  e = fmaf(e, x, 1.0f / 6.0f);
  e = fmaf(e, x, 0.5f);
  e = fmaf(e, x, 1.0f);
  e *= x;
  return fma(a, (double)e, a);
}

template <typename T>
__device__ __forceinline__ T wrap_periodic(T x, T L) {
  if (x < (T)0) x += L;
  if (x >= L) x -= L;
  return x;
}

// LDS region of one tile for deposit order ORDER: the tile's kTile^3 cells, the nodes their
// stencils reach (one more for the trilinear stencil; one before and two after for the
// fourth-order one) and a one-cell drift margin.  The gather is trilinear at every order, so
// the gather array always covers the order-2 region (11^3 nodes) and only the deposit
// accumulator grows to 13^3 at order 4 (38.9 KB of LDS instead of 52.7 KB in float32: four
// blocks per CU instead of three).
template <int ORDER>
struct Reg {
  static constexpr int M = ORDER == 4 ? 2 : 1;  // nodes before the tile's first node
  static constexpr int R = kTile + 2 * M + 1;   // nodes per axis
  static constexpr int R3 = R * R * R;
};

// Region of one tile: node (ox + r1, oy + r2, oz + r3), r in [0, R)^3, wrapped.
struct Region {
  int o[3];
};

// Local lower-node coordinates of a stencil in the region; true if the trilinear stencil
// (nodes l .. l+1 per axis) lies inside.
template <int R, typename T>
__device__ __forceinline__ bool in_region(const Stencil<T>& st, const Region& rg, int N,
                                          int l[3]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    l[j] = (st.c[j] - rg.o[j]) & (N - 1);
    ok = ok && (l[j] <= R - 2);
  }
  return ok;
}

// Same for the fourth-order stencil (nodes l-1 .. l+2 per axis).
template <int R, typename T>
__device__ __forceinline__ bool in_region4(const Stencil<T>& st, const Region& rg, int N,
                                           int l[3]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    l[j] = (st.c[j] - rg.o[j]) & (N - 1);
    ok = ok && (l[j] >= 1) && (l[j] <= R - 3);
  }
  return ok;
}

// node (a, b, c) of an R^3 region; 24-bit multiplies (full rate), indices are below R^3
template <int R>
__device__ __forceinline__ int rindex(int a, int b, int c) {
  return (int)__umul24(__umul24((unsigned)a, R) + (unsigned)b, R) + c;
}

template <typename T>
__device__ __forceinline__ void weights(const Stencil<T>& st, T wx[2], T wy[2], T wz[2]) {
  wx[0] = (T)1 - st.f[0];
  wx[1] = st.f[0];
  wy[0] = (T)1 - st.f[1];
  wy[1] = st.f[1];
  wz[0] = (T)1 - st.f[2];
  wz[1] = st.f[2];
}

template <typename T>
__device__ __forceinline__ void deposit_global(T* ubar, const Stencil<T>& st, T q, int N) {
  T wx[2], wy[2], wz[2];
  weights(st, wx, wy, wz);
  const int ix[2] = {st.c[0], (st.c[0] + 1) & (N - 1)};
  const int iy[2] = {st.c[1], (st.c[1] + 1) & (N - 1)};
  const int iz[2] = {st.c[2], (st.c[2] + 1) & (N - 1)};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        unsafeAtomicAdd(&ubar[node(ix[a], iy[b], iz[c], N)], q * wx[a] * wy[b] * wz[c]);
}

// ---- particle pass ----------------------------------------------------------------------
// deposit_only != 0: deposit the current state of set 0 and change nothing else (used once
// at initialisation for ubar^0).
//
// The deposit accumulator in LDS is float64 in both precisions: float64 LDS atomics are
// far cheaper than float32 ones under the same-address contention of dense cells, and the
// wider sum loses nothing when the block's total is rounded into the global density.
constexpr int kPer = kChunk / kThreads;  // particles per thread
// s_waitcnt operand for vmcnt(0) alone (expcnt and lgkmcnt at their no-wait maxima)
constexpr int kWaitVmcnt0 = 0x0F70;
// type of the LDS deposit accumulator (float64 in both forms: a tile's sums mix up to
// thousands of contributions per node)
template <typename T> struct LdsAccT { using type = double; };
template <typename T> using LdsAcc = typename LdsAccT<T>::type;

// Particles per load batch: four in the 3D pass of both forms.  The float32 pass issues the
// batch's gather loads before its noise is drawn and fits in 84 VGPRs, so that five waves per
// SIMD run, as many as the 32-KB LDS region of a 4-wave block allows on one CU.  The 2D pass
// keeps eight in float32 (LoadBatch2).
template <typename T> struct LoadBatch { static constexpr int n = 4; };
// float32 3D pass: gather loads issued before the noise is drawn
constexpr bool kEarlyGather = true;
template <> struct LoadBatch<double> { static constexpr int n = 4; };
template <typename T> struct LoadBatch2 { static constexpr int n = 8; };
template <> struct LoadBatch2<double> { static constexpr int n = 4; };
// gather-region nodes per thread whose loads are in flight together (24 VGPRs of data)
template <typename T> struct kStageGroup { static constexpr int n = 24 / (int)sizeof(T); };

template <int R, typename T>
__device__ __forceinline__ void deposit_lds(LdsAcc<T>* acc, const Stencil<T>& st, const int l[3],
                                            T q) {
  T wx[2], wy[2], wz[2];
  weights(st, wx, wy, wz);
  // one address; the eight nodes sit at constant offsets from it
  LdsAcc<T>* const a0 = acc + rindex<R>(l[0], l[1], l[2]);
#pragma unroll
  for (int aa = 0; aa < 2; ++aa)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int cc = 0; cc < 2; ++cc)
        atomicAdd(&a0[(aa * R + bb) * R + cc], (LdsAcc<T>)(q * wx[aa] * wy[bb] * wz[cc]));
}

// Fourth-order assignment R_h^(4) (Sec. 2.2.1) in factored form.  With f the fractional
// offset on one axis, the distances of nodes c-1, c, c+1, c+2 are 1+f, f, 1-f, 2-f.  Inner
// nodes (both inner on every axis) weigh prod(1 - p) (1 + sum_j f_j (1 - f_j) / 2); a node
// outer on exactly one axis j weighs -(1/6) (p_j - 1)(2 - p_j)(3 - p_j) prod_{k != j} (1 - p_k),
// i.e. -(1/6) f (1-f) (2-f) at c-1 and -(1/6) f (1-f) (1+f) at c+2.  32 nodes in all.
template <typename T>
struct W4 {
  T u[3][2];  // inner factors 1 - p at nodes c, c+1
  T o[3][2];  // outer factors at nodes c-1, c+2
  T inner;    // 1 + sum_j f_j (1 - f_j) / 2
};

template <typename T>
__device__ __forceinline__ W4<T> weights4(const Stencil<T>& st) {
  W4<T> w;
  T sig = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T f = st.f[j], g = (T)1 - f, fg = f * g;
    w.u[j][0] = g;
    w.u[j][1] = f;
    w.o[j][0] = -fg * ((T)2 - f) / (T)6;
    w.o[j][1] = -fg * ((T)1 + f) / (T)6;
    sig += fg;
  }
  w.inner = (T)1 + sig / (T)2;
  return w;
}

// visit the 32 nodes: fn(d1, d2, d3, weight) with node offsets d in {-1, 0, 1, 2}
template <typename T, typename F>
__device__ __forceinline__ void for_r4(const W4<T>& w, F&& fn) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) fn(a, b, c, w.u[0][a] * w.u[1][b] * w.u[2][c] * w.inner);
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const int dq = o ? 2 : -1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        fn(dq, a, b, w.o[0][o] * w.u[1][a] * w.u[2][b]);
        fn(a, dq, b, w.o[1][o] * w.u[0][a] * w.u[2][b]);
        fn(a, b, dq, w.o[2][o] * w.u[0][a] * w.u[1][b]);
      }
  }
}

template <int R, typename T>
__device__ __forceinline__ void deposit4_lds(LdsAcc<T>* acc, const Stencil<T>& st, const int l[3],
                                             T q) {
  const W4<T> w = weights4(st);
  // one address (node l - 1 on every axis, inside the region); the 32 nodes at constant
  // offsets from it
  LdsAcc<T>* const a0 = acc + rindex<R>(l[0] - 1, l[1] - 1, l[2] - 1);
  for_r4(w, [&](int a, int b, int c, T wt) {
    atomicAdd(&a0[((a + 1) * R + (b + 1)) * R + (c + 1)], (LdsAcc<T>)(q * wt));
  });
}

template <typename T>
__device__ __forceinline__ void deposit4_global(T* ubar, const Stencil<T>& st, T q, int N) {
  const W4<T> w = weights4(st);
  for_r4(w, [&](int a, int b, int c, T wt) {
    unsafeAtomicAdd(&ubar[node((st.c[0] + a) & (N - 1), (st.c[1] + b) & (N - 1),
                               (st.c[2] + c) & (N - 1), N)],
                    q * wt);
  });
}

// deposit of one particle with the assignment of order ORDER
template <int ORDER, int R, typename T>
__device__ __forceinline__ void deposit_one(T* ubar, LdsAcc<T>* acc, const Stencil<T>& st,
                                            const Region& rg, bool use_region, int N, T q) {
  int l[3];
  if (ORDER == 4) {
    if (use_region && in_region4<R>(st, rg, N, l))
      deposit4_lds<R>(acc, st, l, q);
    else
      deposit4_global(ubar, st, q, N);
  } else {
    if (use_region && in_region<R>(st, rg, N, l))
      deposit_lds<R>(acc, st, l, q);
    else
      deposit_global(ubar, st, q, N);
  }
}

template <typename T, int ORDER>
__global__ void __launch_bounds__(kThreads)
    __attribute__((amdgpu_waves_per_eu(ORDER == 2 && sizeof(T) == 4 ? 5 : 1)))
    k_particles(Batch<T> bt, int src_set, int deposit_only) {
  constexpr int R = Reg<ORDER>::R;  // deposit accumulator region
  constexpr int R3 = Reg<ORDER>::R3;
  constexpr int RG = Reg<2>::R;     // gather region: the gather is trilinear at every order
  constexpr int RG3 = Reg<2>::R3;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim<kPartRun>(bt, K_PART, lb);
  SimC<T>& d = sim_view(bt, s);
  const int nchunks = (int)d.coff[d.ntiles];
  const uint4 ci = d.cinfo[lb];  // lb < max_chunks; both loads in flight together
  if (lb >= nchunks) return;
  // uniform: every array below is based at the chunk's first particle, so that accesses
  // take a scalar base and a small per-thread offset (no 64-bit address arithmetic)
  const uint32_t start = __builtin_amdgcn_readfirstlane(ci.x);
  const uint32_t cnt = __builtin_amdgcn_readfirstlane(ci.y) - start;
  const int tile = (int)__builtin_amdgcn_readfirstlane(ci.z);
  const int N = d.N;
  const int nt = d.ntile1;
  Region rg;
  rg.o[0] = (tile / (nt * nt)) * kTile - Reg<ORDER>::M;
  rg.o[1] = ((tile / nt) % nt) * kTile - Reg<ORDER>::M;
  rg.o[2] = (tile % nt) * kTile - Reg<ORDER>::M;
  Region rgg;  // origin of the gather region (rg itself at order 2)
#pragma unroll
  for (int j = 0; j < 3; ++j) rgg.o[j] = rg.o[j] + (Reg<ORDER>::M - Reg<2>::M);
  const bool use_region = d.use_region;
  // buffers of step n: gather array g4[n & 1]; the deposit goes to ubar[(n + 1) & 1] (the
  // state's own ubar[n & 1] when only depositing)
  const uint32_t n = (uint32_t)(*d.step);
  const vec4<T>* const g4 = d.g4[n & 1u];
  T* const ubar = d.ubar[deposit_only ? (n & 1u) : ((n & 1u) ^ 1u)];

  const T* xi = d.xs[src_set] + start;
  const T* yi = d.ys[src_set] + start;
  const T* zi = d.zs[src_set] + start;
  const double* ai = d.as[src_set] + start;
  const uint32_t* idi = d.ids[src_set] + start;
  constexpr int kB = LoadBatch<T>::n;
  T px[kB], py[kB], pz[kB];
  double pa[kB];
  uint32_t pid[kB];
  // issue the loads of kB particles before any arithmetic on them
  auto load_batch = [&](int j0) {
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const uint32_t i = threadIdx.x + (j0 + j) * kThreads;  // within the chunk
      if (i < cnt) {
        px[j] = xi[i];
        py[j] = yi[i];
        pz[j] = zi[i];
        pa[j] = ai[i];
        pid[j] = deposit_only ? 0u : idi[i];
      }
    }
  };
  load_batch(0);  // in flight while the region is staged

  vec4<T>* gl = reinterpret_cast<vec4<T>*>(smem_raw);  // gather array (RG^3 nodes)
  LdsAcc<T>* acc = reinterpret_cast<LdsAcc<T>*>(gl + RG3);  // deposit accumulator (R^3)
  if (use_region) {
    // groups of kStageGroup nodes per thread: all loads of a group in flight together
    constexpr int kS = (R3 + kThreads - 1) / kThreads;
    constexpr int kG = kStageGroup<T>::n;
#pragma unroll
    for (int k0 = 0; k0 < kS; k0 += kG) {
      T s0[kG], s1[kG], s2[kG], s3[kG];  // components, so that they stay in registers
      if (!deposit_only) {
#pragma unroll
        for (int k = 0; k < kG; ++k) {
          const int e = threadIdx.x + (k0 + k) * kThreads;
          if (k0 + k < kS && e < RG3) {
            const int rz = e % RG, ry = (e / RG) % RG, rx = e / (RG * RG);
            const vec4<T> q = g4[node((rgg.o[0] + rx) & (N - 1), (rgg.o[1] + ry) & (N - 1),
                                        (rgg.o[2] + rz) & (N - 1), N)];
            s0[k] = q.x;
            s1[k] = q.y;
            s2[k] = q.z;
            s3[k] = q.w;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kG; ++k) {
        const int e = threadIdx.x + (k0 + k) * kThreads;
        if (k0 + k < kS && e < R3) {  // R3 >= RG3
          if (!deposit_only && e < RG3) gl[e] = vec4<T>{s0[k], s1[k], s2[k], s3[k]};
          acc[e] = (LdsAcc<T>)0;
        }
      }
    }
    __syncthreads();
  }

  // loop invariants held in scalar registers (see keep_in_sgpr); float64 pins only the two
  // it always held, the others would take twice the registers and spill
  constexpr bool kPin = sizeof(T) == 4;
  const T inv_h = keep_in_sgpr(d.inv_h);
  const T inv_h3 = keep_in_sgpr(d.inv_h3);
  const T drift_s = kPin ? keep_in_sgpr(d.drift) : (T)0;
  const T noise_amp_s = kPin ? keep_in_sgpr(d.noise_amp) : (T)0;
  const T L_s = kPin ? keep_in_sgpr(d.L) : (T)0;
  const double dt_s = kPin ? keep_in_sgpr(d.dt) : 0.0;
  const uint32_t sim_lo_s = kPin ? keep_in_sgpr(d.sim_lo) : 0u;
  const uint32_t sim_hi_s = kPin ? keep_in_sgpr(d.sim_hi) : 0u;
  const uint32_t seed_lo_s = kPin ? keep_in_sgpr(d.seed_lo) : 0u;
  const uint32_t seed_hi_s = kPin ? keep_in_sgpr(d.seed_hi) : 0u;
#define SIPF_INV(name, field) (kPin ? name##_s : d.field)
  // outputs at 32-bit byte offsets from the chunk's first particle (scalar base + vector
  // offset addressing)
  unsigned char* const xo = reinterpret_cast<unsigned char*>(d.xs[0] + start);
  unsigned char* const yo = reinterpret_cast<unsigned char*>(d.ys[0] + start);
  unsigned char* const zo = reinterpret_cast<unsigned char*>(d.zs[0] + start);
  unsigned char* const ao = reinterpret_cast<unsigned char*>(d.as[0] + start);
  unsigned char* const ido = reinterpret_cast<unsigned char*>(d.ids[0] + start);
  const bool linear_mass = d.flags & SIPF_FLAG_LINEAR_MASS;
  const bool noise = !(d.flags & SIPF_FLAG_NO_NOISE);

  for (int j0 = 0; j0 < kPer; j0 += kB) {
    // The batch's loads were issued together, so waiting for all of them costs about what
    // waiting for the first does; afterwards no particle of the batch waits for memory (the
    // compiler would otherwise wait for every outstanding access, including the previous
    // particle's stores, before each use of a loaded value).
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const uint32_t i = threadIdx.x + (j0 + j) * kThreads;  // within the chunk
      if (i >= cnt) continue;
      __builtin_amdgcn_sched_barrier(0);
      const T x = px[j], y = py[j], z = pz[j];
      const double a = pa[j];
      int l[3];
      if (deposit_only) {
        const Stencil<T> s0 = make_stencil(x, y, z, inv_h, N);
        deposit_one<ORDER, R>(ubar, acc, s0, rg, use_region, N, (T)a * inv_h3);
        continue;
      }
      // gather (d1 v, d2 v, d3 v, w) at the old position.  float32: the eight LDS loads are
      // issued first and used after the noise is drawn, so that their latency (and that of
      // the previous particle's deposit atomics, which the LDS completes in order) overlaps
      // the Philox rounds; a stencil outside the staged region loads the region's first
      // nodes instead and is gathered from global memory below.  (float64: 64 registers of
      // loads in flight would cost occupancy; its loads follow the noise.)
      const Stencil<T> st = make_stencil(x, y, z, inv_h, N);
      const bool inr = use_region && in_region<RG>(st, rgg, N, l);
      constexpr bool kEarly = sizeof(T) == 4 && kEarlyGather;
      vec4<T> q[kEarly ? 8 : 1];
      const int b0 = inr ? rindex<RG>(l[0], l[1], l[2]) : 0;
      if constexpr (kEarly) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
          q[k] = gl[b0 + ((k >> 2) * RG + ((k >> 1) & 1)) * RG + (k & 1)];
      }

      // Wiener increment: Philox counter (particle index, step, simulation)
      T zn[3] = {0, 0, 0};
      if (noise) {
        uint32_t c0 = pid[j], c1 = n, c2 = SIPF_INV(sim_lo, sim_lo), c3 = SIPF_INV(sim_hi, sim_hi);
        philox4x32_10(c0, c1, c2, c3, SIPF_INV(seed_lo, seed_lo), SIPF_INV(seed_hi, seed_hi));
        box_muller(c0, c1, c2, c3, zn);
      }

      T wx[2], wy[2], wz[2];
      weights(st, wx, wy, wz);
      T g0 = 0, g1 = 0, g2 = 0, gw = 0;
      if constexpr (kEarly) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const T wgt = wx[k >> 2] * wy[(k >> 1) & 1] * wz[k & 1];
          g0 += wgt * q[k].x;
          g1 += wgt * q[k].y;
          g2 += wgt * q[k].z;
          gw += wgt * q[k].w;
        }
      } else if (inr) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const vec4<T> qk = gl[b0 + ((k >> 2) * RG + ((k >> 1) & 1)) * RG + (k & 1)];
          const T wgt = wx[k >> 2] * wy[(k >> 1) & 1] * wz[k & 1];
          g0 += wgt * qk.x;
          g1 += wgt * qk.y;
          g2 += wgt * qk.z;
          gw += wgt * qk.w;
        }
      }
      if (!inr) {
        // the stencil leaves the staged region (or there is none): one corner at a time, so
        // that this rare path does not raise the register count of the whole kernel
        g0 = g1 = g2 = gw = (T)0;
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
          const int aa = k >> 2, bb = (k >> 1) & 1, cc = k & 1;
          const vec4<T> qg = g4[node((st.c[0] + aa) & (N - 1), (st.c[1] + bb) & (N - 1),
                                     (st.c[2] + cc) & (N - 1), N)];
          const T wgt = (aa ? wx[1] : wx[0]) * (bb ? wy[1] : wy[0]) * (cc ? wz[1] : wz[0]);
          g0 += wgt * qg.x;
          g1 += wgt * qg.y;
          g2 += wgt * qg.z;
          gw += wgt * qg.w;
        }
      }

      // push and mass update
      const T drift = SIPF_INV(drift, drift), noise_amp = SIPF_INV(noise_amp, noise_amp);
      const T Lbox = SIPF_INV(L, L);
      const double dt = SIPF_INV(dt, dt);
      const T xn = wrap_periodic(x + drift * g0 + noise_amp * zn[0], Lbox);
      const T yn = wrap_periodic(y + drift * g1 + noise_amp * zn[1], Lbox);
      const T zz = wrap_periodic(z + drift * g2 + noise_amp * zn[2], Lbox);
      const T rho = rho_of(gw);
      const double an = linear_mass ? a * (1.0 + dt * (double)rho - dt)
                                    : mass_factor_update(a, (T)dt * (rho - (T)1));
      const uint32_t bo = i * (uint32_t)sizeof(T);
      *reinterpret_cast<T*>(xo + bo) = xn;
      *reinterpret_cast<T*>(yo + bo) = yn;
      *reinterpret_cast<T*>(zo + bo) = zz;
      *reinterpret_cast<double*>(ao + i * 8u) = an;
      if (src_set) *reinterpret_cast<uint32_t*>(ido + i * 4u) = pid[j];

      // deposit of the new state: ubar^{n+1}
      const Stencil<T> sn = make_stencil(xn, yn, zz, inv_h, N);
      deposit_one<ORDER, R>(ubar, acc, sn, rg, use_region, N, (T)an * inv_h3);
    }
    // Next batch, if the chunk has one.  Its loads are issued here, after an explicit wait
    // for this batch's stores: the compiler cannot tell that the exec-masked loads of the
    // previous batch were all consumed, and would otherwise wait for every outstanding
    // access before each particle's loads, so that a batch cost one round trip per particle.
    if (j0 + kB >= kPer || (uint32_t)((j0 + kB) * kThreads) >= cnt) break;
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    load_batch(j0 + kB);
  }

  if (use_region) {
    __syncthreads();
    for (int e = threadIdx.x; e < R3; e += kThreads) {
      const LdsAcc<T> v = acc[e];
      if (v != (LdsAcc<T>)0) {
        const int rz = e % R, ry = (e / R) % R, rx = e / (R * R);
        unsafeAtomicAdd(&ubar[node((rg.o[0] + rx) & (N - 1), (rg.o[1] + ry) & (N - 1),
                                     (rg.o[2] + rz) & (N - 1), N)],
                        (T)v);
      }
    }
  }
}

#undef SIPF_INV

// ---- two-dimensional particle pass ---------------------------------------------------------
// The same pass on an N^2 grid (the paper's two-dimensional example): bilinear stencils,
// square tiles of kTile2^2 cells with a (kTile2 + 3)^2-node LDS region, two Wiener
// components (the first two normals of the Philox block).  The gather array holds
// (d1 v, -, d2 v, w) per node.
constexpr int kR2 = kTile2 + 2 * kM2 + 1;  // nodes per axis of a 2D region
constexpr int kR2sq = kR2 * kR2;

template <typename T>
__device__ __forceinline__ Stencil<T> make_stencil2(T x, T y, T inv_h, int N) {
  Stencil<T> st;
  const T s[2] = {x * inv_h, y * inv_h};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const T fl = floor(s[j]);
    st.f[j] = s[j] - fl;
    st.c[j] = ((int)fl) & (N - 1);
  }
  st.f[2] = (T)0;
  st.c[2] = 0;
  return st;
}

template <typename T>
__device__ __forceinline__ bool in_region2(const Stencil<T>& st, const Region& rg, int N,
                                           int l[2]) {
  l[0] = (st.c[0] - rg.o[0]) & (N - 1);
  l[1] = (st.c[1] - rg.o[1]) & (N - 1);
  return l[0] <= kR2 - 2 && l[1] <= kR2 - 2;
}

__device__ __forceinline__ void box_muller2(uint32_t r0, uint32_t r1, double z[2]) {
  const double u0 = fma((double)r0, 0x1p-32, 0x1p-33);
  const double u1 = fma((double)r1, 0x1p-32, 0x1p-33);
  const double ra = sqrt(-2.0 * log(u0));
  double s1, c1;
  sincospi(2.0 * u1, &s1, &c1);
  z[0] = ra * c1;
  z[1] = ra * s1;
}

__device__ __forceinline__ void box_muller2(uint32_t r0, uint32_t r1, float z[2]) {
  const float u0 = fmaf((float)r0, 0x1p-32f, 0x1p-33f);
  const float u1 = fmaf((float)r1, 0x1p-32f, 0x1p-33f);
  const float ra = __builtin_amdgcn_sqrtf(-2.0f * 0.69314718055994531f * __builtin_amdgcn_logf(u0));
  z[0] = ra * __builtin_amdgcn_cosf(u1);
  z[1] = ra * __builtin_amdgcn_sinf(u1);
}

template <typename T>
__device__ __forceinline__ void deposit2(T* ubar, LdsAcc<T>* acc, const Stencil<T>& st,
                                         const Region& rg, bool use_region, int N, T q) {
  const T wx[2] = {(T)1 - st.f[0], st.f[0]};
  const T wy[2] = {(T)1 - st.f[1], st.f[1]};
  int l[2];
  if (use_region && in_region2(st, rg, N, l)) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        atomicAdd(&acc[(l[0] + a) * kR2 + l[1] + b], (LdsAcc<T>)(q * wx[a] * wy[b]));
  } else {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        unsafeAtomicAdd(&ubar[(int64_t)((st.c[0] + a) & (N - 1)) * N + ((st.c[1] + b) & (N - 1))],
                        q * wx[a] * wy[b]);
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_particles2(Batch<T> bt, int src_set,
                                                         int deposit_only) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim<kPartRun>(bt, K_PART, lb);
  SimC<T>& d = sim_view(bt, s);
  const int nchunks = (int)d.coff[d.ntiles];
  const uint4 ci = d.cinfo[lb];  // lb < max_chunks; both loads in flight together
  if (lb >= nchunks) return;
  // uniform: every array below is based at the chunk's first particle, so that accesses
  // take a scalar base and a small per-thread offset (no 64-bit address arithmetic)
  const uint32_t start = __builtin_amdgcn_readfirstlane(ci.x);
  const uint32_t cnt = __builtin_amdgcn_readfirstlane(ci.y) - start;
  const int tile = (int)__builtin_amdgcn_readfirstlane(ci.z);
  const int N = d.N;
  const int nt = d.ntile1;
  Region rg;
  rg.o[0] = (tile / nt) * kTile2 - kM2;
  rg.o[1] = (tile % nt) * kTile2 - kM2;
  rg.o[2] = 0;
  const bool use_region = d.use_region;
  // buffers of step n: gather array g4[n & 1]; the deposit goes to ubar[(n + 1) & 1] (the
  // state's own ubar[n & 1] when only depositing)
  const uint32_t n = (uint32_t)(*d.step);
  const vec4<T>* const g4 = d.g4[n & 1u];
  T* const ubar = d.ubar[deposit_only ? (n & 1u) : ((n & 1u) ^ 1u)];
  const T* xi = d.xs[src_set] + start;
  const T* yi = d.ys[src_set] + start;
  const double* ai = d.as[src_set] + start;
  const uint32_t* idi = d.ids[src_set] + start;
  T* xo = d.xs[0] + start;
  T* yo = d.ys[0] + start;
  double* ao = d.as[0] + start;
  uint32_t* ido = d.ids[0] + start;
  constexpr int kB = LoadBatch2<T>::n;
  T px[kB], py[kB];
  double pa[kB];
  uint32_t pid[kB];
  // the loads of kB particles are issued before any arithmetic on them
  auto load_batch = [&](int j0) {
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const uint32_t i = threadIdx.x + (j0 + j) * kThreads;  // within the chunk
      if (i < cnt) {
        px[j] = xi[i];
        py[j] = yi[i];
        pa[j] = ai[i];
        pid[j] = deposit_only ? 0u : idi[i];
      }
    }
  };
  load_batch(0);  // in flight while the region is staged

  vec4<T>* gl = reinterpret_cast<vec4<T>*>(smem_raw);
  LdsAcc<T>* acc = reinterpret_cast<LdsAcc<T>*>(gl + kR2sq);
  if (use_region) {
    constexpr int kS = (kR2sq + kThreads - 1) / kThreads;
    T s0[kS], s1[kS], s2[kS], s3[kS];
    if (!deposit_only) {
#pragma unroll
      for (int k = 0; k < kS; ++k) {
        const int e = threadIdx.x + k * kThreads;
        if (e < kR2sq) {
          const int ry = e % kR2, rx = e / kR2;
          const vec4<T> q =
              g4[(int64_t)((rg.o[0] + rx) & (N - 1)) * N + ((rg.o[1] + ry) & (N - 1))];
          s0[k] = q.x;
          s1[k] = q.y;
          s2[k] = q.z;
          s3[k] = q.w;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kS; ++k) {
      const int e = threadIdx.x + k * kThreads;
      if (e < kR2sq) {
        if (!deposit_only) gl[e] = vec4<T>{s0[k], s1[k], s2[k], s3[k]};
        acc[e] = (LdsAcc<T>)0;
      }
    }
    __syncthreads();
  }
  const T inv_h = keep_in_sgpr(d.inv_h);
  const T inv_h3 = keep_in_sgpr(d.inv_h3);
  const bool linear_mass = d.flags & SIPF_FLAG_LINEAR_MASS;
  const bool noise = !(d.flags & SIPF_FLAG_NO_NOISE);
  for (int j0 = 0; j0 < kPer; j0 += kB) {
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);  // the batch's loads, as in the 3D pass
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const uint32_t i = threadIdx.x + (j0 + j) * kThreads;  // within the chunk
      if (i >= cnt) continue;
      __builtin_amdgcn_sched_barrier(0);
      const T x = px[j], y = py[j];
      const double a = pa[j];
      if (deposit_only) {
        deposit2(ubar, acc, make_stencil2(x, y, inv_h, N), rg, use_region, N,
                 (T)a * inv_h3);
        continue;
      }
      const Stencil<T> st = make_stencil2(x, y, inv_h, N);
      const T wx[2] = {(T)1 - st.f[0], st.f[0]};
      const T wy[2] = {(T)1 - st.f[1], st.f[1]};
      T g0 = 0, g1 = 0, gw = 0;
      int l[2];
      const bool inside = use_region && in_region2(st, rg, N, l);
      // separate LDS and global branches: a load through a pointer selected between the two
      // would be a flat access
      if (inside) {
#pragma unroll
        for (int aa = 0; aa < 2; ++aa)
#pragma unroll
          for (int bb = 0; bb < 2; ++bb) {
            const vec4<T> q = gl[(l[0] + aa) * kR2 + l[1] + bb];
            const T wgt = wx[aa] * wy[bb];
            g0 += wgt * q.x;
            g1 += wgt * q.z;
            gw += wgt * q.w;
          }
      } else {
        // outside the staged region (or none): one node at a time, as in the 3D pass
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
          const int aa = k >> 1, bb = k & 1;
          const vec4<T> q =
              g4[(int64_t)((st.c[0] + aa) & (N - 1)) * N + ((st.c[1] + bb) & (N - 1))];
          const T wgt = (aa ? wx[1] : wx[0]) * (bb ? wy[1] : wy[0]);
          g0 += wgt * q.x;
          g1 += wgt * q.z;
          gw += wgt * q.w;
        }
      }
      T zn[2] = {0, 0};
      if (noise) {
        uint32_t c0 = pid[j], c1 = n, c2 = d.sim_lo, c3 = d.sim_hi;
        philox4x32_10(c0, c1, c2, c3, d.seed_lo, d.seed_hi);
        box_muller2(c0, c1, zn);
      }
      const T xn = wrap_periodic(x + d.drift * g0 + d.noise_amp * zn[0], d.L);
      const T yn = wrap_periodic(y + d.drift * g1 + d.noise_amp * zn[1], d.L);
      const T rho = rho_of(gw);
      const double an = linear_mass ? a * (1.0 + d.dt * (double)rho - d.dt)
                                    : mass_factor_update(a, (T)d.dt * (rho - (T)1));
      xo[i] = xn;
      yo[i] = yn;
      ao[i] = an;
      if (src_set) ido[i] = pid[j];
      deposit2(ubar, acc, make_stencil2(xn, yn, inv_h, N), rg, use_region, N,
               (T)an * inv_h3);
    }
    if (j0 + kB >= kPer || (uint32_t)((j0 + kB) * kThreads) >= cnt) break;
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);  // see the 3D pass
    load_batch(j0 + kB);
  }
  if (use_region) {
    __syncthreads();
    for (int e = threadIdx.x; e < kR2sq; e += kThreads) {
      const LdsAcc<T> v = acc[e];
      if (v != (LdsAcc<T>)0) {
        const int ry = e % kR2, rx = e / kR2;
        unsafeAtomicAdd(&ubar[(int64_t)((rg.o[0] + rx) & (N - 1)) * N +
                                ((rg.o[1] + ry) & (N - 1))],
                        (T)v);
      }
    }
  }
}

// ---- binning ----------------------------------------------------------------------------
// Tile of every particle of set 0 and its rank among the particles of that tile.  A block
// takes kBinChunk consecutive particles: wavefronts aggregate their first tile (one LDS
// atomic), the other lanes count themselves, into a block-local hash table; then the block
// adds each distinct tile's count to the global counter with one atomic and derives global
// ranks.  Set 0 is tile-ordered after the first binning, so a block sees one or two tiles
// and the global counters see few atomics.  Tiles that do not fit the table count on the
// global counter directly.
constexpr int kBinChunk = kBinBlock;
constexpr int kBinPer = kBinChunk / kThreads;
constexpr int kHash = 512;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kGlobalFlag = 0x80000000u;

// Slot of tile t in a block's open-addressing hash table (claimed on first use), or kEmpty
// when 16 probes find no free slot.
__device__ __forceinline__ uint32_t hash_slot(uint32_t* hkey, uint32_t t) {
  uint32_t h = (t * 2654435761u) >> 23;  // 9-bit multiplicative hash
  for (int probe = 0; probe < 16; ++probe, h = (h + 1) & (kHash - 1)) {
    const uint32_t k = atomicCAS(&hkey[h], kEmpty, t);
    if (k == kEmpty || k == t) return h;
  }
  return kEmpty;
}

// Tile of a particle (row-major tile index, z fastest; a cell index N - 1 beyond the last
// full tile joins the last tile).  The count and the scatter compute it from the same
// positions, so the binning keys hold only the rank within the tile.
template <typename T, int DIM>
__device__ __forceinline__ uint32_t tile_of(T x, T y, T z, T inv_h, int N, int nt) {
  if (DIM == 2) {
    const Stencil<T> st = make_stencil2(x, y, inv_h, N);
    const int tx = st.c[0] / kTile2, ty = st.c[1] / kTile2;
    return (uint32_t)((tx < nt ? tx : nt - 1) * nt + (ty < nt ? ty : nt - 1));
  }
  const Stencil<T> st = make_stencil(x, y, z, inv_h, N);
  const int tx = st.c[0] / kTile, ty = st.c[1] / kTile, tz = st.c[2] / kTile;
  return (uint32_t)(((tx < nt ? tx : nt - 1) * nt + (ty < nt ? ty : nt - 1)) * nt +
                    (tz < nt ? tz : nt - 1));
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kThreads) k_bin_count(Batch<T> bt) {
  int lb;
  const int s = find_sim<kFieldRun>(bt, K_SCOUNT, lb);
  SimC<T>& d = sim_view(bt, s);
  __shared__ uint32_t hkey[kHash], hcnt[kHash], hbase[kHash];
  for (int e = threadIdx.x; e < kHash; e += kThreads) {
    hkey[e] = kEmpty;
    hcnt[e] = 0;
  }
  __syncthreads();
  const int N = d.N, nt = d.ntile1;
  const int lane = threadIdx.x & 63;
  const int64_t i0 = (int64_t)lb * kBinChunk + threadIdx.x;
  uint32_t slot[kBinPer], lrank[kBinPer];
  // positions of all kBinPer particles loaded before the first tile is aggregated (the
  // aggregation loop would otherwise put one memory round trip between consecutive loads)
  T px[kBinPer], py[kBinPer], pz[kBinPer];
#pragma unroll
  for (int j = 0; j < kBinPer; ++j) {
    const int64_t i = i0 + (int64_t)j * kThreads;
    if (i < d.P) {
      px[j] = d.xs[0][i];
      py[j] = d.ys[0][i];
      if (DIM == 3) pz[j] = d.zs[0][i];
    }
  }
#pragma unroll
  for (int j = 0; j < kBinPer; ++j) {
    const int64_t i = i0 + (int64_t)j * kThreads;
    const bool valid = i < d.P;
    const uint32_t tile =
        valid ? tile_of<T, DIM>(px[j], py[j], DIM == 3 ? pz[j] : (T)0, d.inv_h, N, nt) : 0u;
    slot[j] = kEmpty;
    lrank[j] = 0;
    // The wavefront's first tile (usually shared by most lanes: set 0 is tile-ordered) is
    // aggregated by one leader lane; the lanes whose particle has moved to another tile then
    // take their ranks on their own, all in one pass, rather than one pass per tile.
    const unsigned long long pending = __ballot(valid);
    if (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const uint32_t lt = __shfl(tile, leader, 64);
      const unsigned long long same = __ballot(valid && tile == lt) & pending;
      uint32_t sl = kEmpty, base = 0;
      if (lane == leader) {
        sl = hash_slot(hkey, lt);
        if (sl != kEmpty) {
          base = atomicAdd(&hcnt[sl], (uint32_t)__popcll(same));
        } else {
          base = atomicAdd(&d.tcount[lt], (uint32_t)__popcll(same));
          sl = kGlobalFlag;
        }
      }
      sl = __shfl(sl, leader, 64);
      base = __shfl(base, leader, 64);
      if ((same >> lane) & 1ull) {
        slot[j] = sl;
        lrank[j] = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
      } else if (valid) {
        uint32_t so = hash_slot(hkey, tile);
        if (so != kEmpty) {
          lrank[j] = atomicAdd(&hcnt[so], 1u);
        } else {
          lrank[j] = atomicAdd(&d.tcount[tile], 1u);
          so = kGlobalFlag;
        }
        slot[j] = so;
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kHash; e += kThreads) {
    const uint32_t k = hkey[e];
    if (k != kEmpty) hbase[e] = atomicAdd(&d.tcount[k], hcnt[e]);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kBinPer; ++j) {
    const int64_t i = i0 + (int64_t)j * kThreads;
    if (i < d.P) {
      const uint32_t r = slot[j] == kGlobalFlag ? lrank[j] : hbase[slot[j]] + lrank[j];
      d.key[i] = r;  // rank within the tile
    }
  }
}

// Exclusive scan of the tile counts (tile offsets, in tile order) and the chunk table, with
// the chunks in decreasing size: a tile of c particles has floor(c / kChunk) full chunks and,
// if c mod kChunk > 0, one smaller chunk.  The table holds the full chunks first (in tile
// order), then the smaller ones by size class (halving from kChunk / 2 to kChunk / 16, and
// a last class below that), each class in tile order.  The particle pass takes chunks in
// table order as CUs free up, so the large chunks start first and the small ones fill the
// end of the pass, which shortens its tail (longest-first list scheduling).  With more than
// kSizeOrderMax chunks the tail is a small part of the pass, and the table stays in tile order
// (all chunks of a tile together, neighbouring tiles next to each other).
// One block per segment of kSegTiles tiles: every block sums the counts of all segments
// (class totals, for the class bases) and of the earlier ones (its carries), then scans its
// own segment.  The counts are cleared for the next binning by the scatter, after every block
// has read them.
constexpr int kScanSeg = 16;                    // tiles per thread in a segment
constexpr int kSegTiles = kScanSeg * kThreads;  // tiles per segment (block)
constexpr int kClasses = 6;                     // size classes of the chunk table
constexpr uint32_t kSizeOrderMax = 8192;        // chunks up to which they go by size

// size class of a chunk of n particles, 0 < n <= kChunk
__device__ __forceinline__ int chunk_class(uint32_t n) {
  int c = 0;
#pragma unroll
  for (int k = 0; k < kClasses - 1; ++k) c += n < (uint32_t)(kChunk >> k);
  return c;
}

// chunks of each class contributed by a tile of c particles
struct ClassCount {
  uint32_t n[kClasses];
};
__device__ __forceinline__ void add_tile(ClassCount& a, uint32_t c) {
  a.n[0] += c / kChunk;
  const uint32_t r = c % kChunk;
  const int cl = chunk_class(r);
#pragma unroll
  for (int k = 1; k < kClasses; ++k) a.n[k] += (r != 0u && cl == k) ? 1u : 0u;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_bin_scan(Batch<T> bt) {
  int lb;
  const int s = find_sim(bt, K_SSCAN, lb);
  SimC<T>& d = sim_view(bt, s);
  const int nt = d.ntiles;
  const int s0 = lb * kSegTiles;
  __shared__ uint32_t cnt[kSegTiles];
  __shared__ uint32_t sh[kClasses + 1][kThreads];  // scan arrays: classes, then particles
  __shared__ uint32_t base[kClasses];              // first table entry of each class, here
  __shared__ uint32_t carry_all;                   // chunks of the earlier segments
  __shared__ uint32_t by_size;                     // table by size class (else tile order)
  // class totals over all segments and carries (chunks per class, particles) of the earlier
  // ones; kScanSeg loads per thread in flight together per segment
  ClassCount tot{}, car{};
  uint32_t ap = 0;
  for (int e0 = 0; e0 < nt; e0 += kSegTiles) {
    uint32_t v[kScanSeg];
#pragma unroll
    for (int j = 0; j < kScanSeg; ++j) {
      const int t = e0 + (int)threadIdx.x + j * kThreads;
      v[j] = t < nt ? d.tcount[t] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kScanSeg; ++j) {
      add_tile(tot, v[j]);
      if (e0 < s0) {
        add_tile(car, v[j]);
        ap += v[j];
      }
    }
  }
  // block sums: totals into sh[0..kClasses), then carries (and particles) the same way
  for (int pass = 0; pass < 2; ++pass) {
    const ClassCount& a = pass ? car : tot;
#pragma unroll
    for (int k = 0; k < kClasses; ++k) sh[k][threadIdx.x] = a.n[k];
    sh[kClasses][threadIdx.x] = ap;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
#pragma unroll
        for (int k = 0; k <= kClasses; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (pass == 0) {
        uint32_t b = 0;  // exclusive scan of the class totals: class bases
        for (int k = 0; k < kClasses; ++k) {
          base[k] = b;
          b += sh[k][0];
        }
        by_size = b <= kSizeOrderMax ? 1u : 0u;
        if (s0 + kSegTiles >= nt) d.coff[nt] = b;  // number of chunks
      } else {
        uint32_t ca = 0;
        for (int k = 0; k < kClasses; ++k) {
          base[k] += sh[k][0];  // + this block's carries
          ca += sh[k][0];
        }
        carry_all = ca;
      }
    }
    if (pass == 1) ap = sh[kClasses][0];
    __syncthreads();
  }
  const uint32_t carry_p = ap;
  // this segment: counts into LDS (coalesced), kScanSeg consecutive tiles per thread
  {
    uint32_t v[kScanSeg];
#pragma unroll
    for (int j = 0; j < kScanSeg; ++j) {
      const int t = s0 + (int)threadIdx.x + j * kThreads;
      v[j] = t < nt ? d.tcount[t] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kScanSeg; ++j) cnt[threadIdx.x + j * kThreads] = v[j];
  }
  __syncthreads();
  const int b0 = (int)threadIdx.x * kScanSeg;
  ClassCount mine{};
  uint32_t sp = 0;
#pragma unroll
  for (int j = 0; j < kScanSeg; ++j) {
    const uint32_t c = cnt[b0 + j];
    sp += c;
    add_tile(mine, c);
  }
#pragma unroll
  for (int k = 0; k < kClasses; ++k) sh[k][threadIdx.x] = mine.n[k];
  sh[kClasses][threadIdx.x] = sp;
  __syncthreads();
  // inclusive Hillis-Steele scan of the per-thread sums
  for (int off = 1; off < kThreads; off <<= 1) {
    uint32_t x[kClasses + 1];
#pragma unroll
    for (int k = 0; k <= kClasses; ++k)
      x[k] = (int)threadIdx.x >= off ? sh[k][threadIdx.x - off] : 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k <= kClasses; ++k) sh[k][threadIdx.x] += x[k];
    __syncthreads();
  }
  uint32_t rp = carry_p + (threadIdx.x ? sh[kClasses][threadIdx.x - 1] : 0u);
  uint32_t nx[kClasses];  // next table entry of each class for this thread's tiles
  uint32_t na = carry_all;  // next entry in tile order
#pragma unroll
  for (int k = 0; k < kClasses; ++k) {
    nx[k] = base[k] + (threadIdx.x ? sh[k][threadIdx.x - 1] : 0u);
    na += threadIdx.x ? sh[k][threadIdx.x - 1] : 0u;
  }
  if (!by_size) {
    for (int j = 0; j < kScanSeg; ++j) {
      const int t = s0 + b0 + j;
      if (t >= nt) break;
      const uint32_t c = cnt[b0 + j];
      d.toff[t] = rp;
      for (uint32_t k = 0; k * kChunk < c; ++k) {
        const uint32_t cs = rp + k * kChunk;
        d.cinfo[na++] = uint4{cs, cs + kChunk < rp + c ? cs + kChunk : rp + c, (uint32_t)t, 0u};
      }
      rp += c;
    }
  }
  for (int j = 0; j < kScanSeg && by_size; ++j) {
    const int t = s0 + b0 + j;
    if (t >= nt) break;
    const uint32_t c = cnt[b0 + j];
    d.toff[t] = rp;
    const uint32_t full = c / kChunk, r = c % kChunk;
    for (uint32_t k = 0; k < full; ++k)
      d.cinfo[nx[0]++] = uint4{rp + k * kChunk, rp + (k + 1) * kChunk, (uint32_t)t, 0u};
    if (r != 0u) {
      const int cl = chunk_class(r);
      uint32_t at = 0;
#pragma unroll
      for (int k = 1; k < kClasses; ++k)
        if (cl == k) at = nx[k]++;
      d.cinfo[at] = uint4{rp + full * kChunk, rp + c, (uint32_t)t, 0u};
    }
    rp += c;
  }
  if (s0 + kSegTiles >= nt && threadIdx.x == kThreads - 1)  // the last segment closes toff
    d.toff[nt] = carry_p + sh[kClasses][kThreads - 1];
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kThreads) k_bin_scatter(Batch<T> bt) {
  int lb;
  const int s = find_sim<kFieldRun>(bt, K_SSCATTER, lb);
  SimC<T>& d = sim_view(bt, s);
  const int64_t i = (int64_t)lb * kThreads + threadIdx.x;
  // tile counts cleared for the next binning (the scan has read them all)
  if (i < d.ntiles) d.tcount[i] = 0;
  if (i >= d.P) return;
  const T x = d.xs[0][i], y = d.ys[0][i], z = DIM == 3 ? d.zs[0][i] : (T)0;
  const uint32_t dst = d.toff[tile_of<T, DIM>(x, y, z, d.inv_h, d.N, d.ntile1)] + d.key[i];
  d.xs[1][dst] = x;
  d.ys[1][dst] = y;
  if (DIM == 3) d.zs[1][dst] = z;
  d.as[1][dst] = d.as[0][i];
  d.ids[1][dst] = d.ids[0][i];
}

template <typename T, int ORDER>
size_t particle_lds_bytes() {
  return Reg<2>::R3 * sizeof(vec4<T>) + Reg<ORDER>::R3 * sizeof(LdsAcc<T>);
}

template <typename T>
void launch_particles(const Batch<T>& b, int nblk, int src_set, int deposit_only, int order,
                      int dim, hipStream_t st) {
  if (nblk <= 0) return;
  if (dim == 2) {
    hipLaunchKernelGGL(k_particles2<T>, dim3(nblk), dim3(kThreads),
                       kR2sq * (sizeof(vec4<T>) + sizeof(LdsAcc<T>)), st, b, src_set, deposit_only);
    return;
  }
  auto kern = order == 4 ? k_particles<T, 4> : k_particles<T, 2>;
  const size_t lds = order == 4 ? particle_lds_bytes<T, 4>() : particle_lds_bytes<T, 2>();
  hipLaunchKernelGGL(kern, dim3(nblk), dim3(kThreads), lds, st, b, src_set, deposit_only);
}
template <typename T>
void launch_binning(const Batch<T>& b, const int* tot, int nsims, int dim, hipStream_t st) {
  if (tot[K_SCOUNT] > 0) {
    if (dim == 2)
      hipLaunchKernelGGL((k_bin_count<T, 2>), dim3(tot[K_SCOUNT]), dim3(kThreads), 0, st, b);
    else
      hipLaunchKernelGGL((k_bin_count<T, 3>), dim3(tot[K_SCOUNT]), dim3(kThreads), 0, st, b);
  }
  hipLaunchKernelGGL(k_bin_scan<T>, dim3(tot[K_SSCAN]), dim3(kThreads), 0, st, b);
  if (tot[K_SSCATTER] > 0) {
    if (dim == 2)
      hipLaunchKernelGGL((k_bin_scatter<T, 2>), dim3(tot[K_SSCATTER]), dim3(kThreads), 0, st, b);
    else
      hipLaunchKernelGGL((k_bin_scatter<T, 3>), dim3(tot[K_SSCATTER]), dim3(kThreads), 0, st, b);
  }
}
// raise the dynamic LDS limit of the particle kernel of this order (call outside capture)
template <typename T>
void configure_particles(int order, int dim) {
  if (dim == 2) return;  // its region fits the default limit
  if (order == 4)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_particles<T, 4>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)particle_lds_bytes<T, 4>());
  else
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_particles<T, 2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)particle_lds_bytes<T, 2>());
}
template void configure_particles<double>(int, int);
template void configure_particles<float>(int, int);

template void launch_particles<double>(const Batch<double>&, int, int, int, int, int,
                                       hipStream_t);
template void launch_particles<float>(const Batch<float>&, int, int, int, int, int, hipStream_t);
template void launch_binning<double>(const Batch<double>&, const int*, int, int, hipStream_t);
template void launch_binning<float>(const Batch<float>&, const int*, int, int, hipStream_t);

}  // namespace sipf
