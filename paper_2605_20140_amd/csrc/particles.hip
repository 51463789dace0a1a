// Particle half of the SIPF-W step on gfx950: grid-to-particle gather (Alg. g2p), Philox
// Wiener increments, Euler-Maruyama push and mass update (eq. u_hat_update, eq. SDE), and the
// particle-to-grid deposit (Alg. p2g) of the new state, fused in one pass over the particles.
//
// Particles are structure of arrays: x, y, z in the working precision T, masses a in
// float64, and a 32-bit particle index id that keys the noise stream, so results do not
// depend on the storage order.
//
// Trilinear stencil: s = x / h, i = floor(s), f = s - i; node weights (1 - f, f) per axis
// (K_h = h^3 R_h); R_h = K_h / h^3 for the deposit.  Node indices wrap modulo N.
#include "sipf_internal.h"

namespace sipf {

template <typename T>
struct Stencil {
  int i0[3], i1[3];
  T f[3];
};

template <typename T>
__device__ __forceinline__ Stencil<T> make_stencil(T x, T y, T z, T inv_h, int N) {
  Stencil<T> st;
  const T s[3] = {x * inv_h, y * inv_h, z * inv_h};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T fl = floor(s[j]);
    st.f[j] = s[j] - fl;
    const int i = (int)fl;
    st.i0[j] = i & (N - 1);
    st.i1[j] = (i + 1) & (N - 1);
  }
  return st;
}

__device__ __forceinline__ int64_t node(int a, int b, int c, int N) {
  return ((int64_t)a * N + b) * N + c;
}

template <typename T>
__device__ __forceinline__ void deposit_stencil(T* ubar, const Stencil<T>& st, T q, int N) {
  const T wx[2] = {(T)1 - st.f[0], st.f[0]};
  const T wy[2] = {(T)1 - st.f[1], st.f[1]};
  const T wz[2] = {(T)1 - st.f[2], st.f[2]};
  const int ix[2] = {st.i0[0], st.i1[0]};
  const int iy[2] = {st.i0[1], st.i1[1]};
  const int iz[2] = {st.i0[2], st.i1[2]};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        unsafeAtomicAdd(&ubar[node(ix[a], iy[b], iz[c], N)], q * wx[a] * wy[b] * wz[c]);
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

template <typename T>
__device__ __forceinline__ T wrap_periodic(T x, T L) {
  if (x < (T)0) x += L;
  if (x >= L) x -= L;
  return x;
}

// One thread per particle.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_particles(Batch<T> bt) {
  int lb;
  const int s = find_sim(bt, K_PART, lb);
  const SimDev<T>& d = bt.sims[s];
  const int64_t i = (int64_t)lb * kThreads + threadIdx.x;
  if (i >= d.P) return;
  const int N = d.N;
  const uint32_t n = (uint32_t)(*d.step);
  const T x = d.x[i], y = d.y[i], z = d.z[i];
  const double a = d.a[i];
  const uint32_t id = d.id[i];

  // gather (d1 v, d2 v, d3 v, w) at the old position
  const Stencil<T> st = make_stencil(x, y, z, d.inv_h, N);
  const T wx[2] = {(T)1 - st.f[0], st.f[0]};
  const T wy[2] = {(T)1 - st.f[1], st.f[1]};
  const T wz[2] = {(T)1 - st.f[2], st.f[2]};
  const int ix[2] = {st.i0[0], st.i1[0]};
  const int iy[2] = {st.i0[1], st.i1[1]};
  const int iz[2] = {st.i0[2], st.i1[2]};
  T g0 = 0, g1 = 0, g2 = 0, gw = 0;
#pragma unroll
  for (int aa = 0; aa < 2; ++aa)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const vec4<T> q = d.g4[node(ix[aa], iy[bb], iz[cc], N)];
        const T wgt = wx[aa] * wy[bb] * wz[cc];
        g0 += wgt * q.x;
        g1 += wgt * q.y;
        g2 += wgt * q.z;
        gw += wgt * q.w;
      }

  // Wiener increment
  T zn[3] = {0, 0, 0};
  if (!(d.flags & SIPF_FLAG_NO_NOISE)) {
    uint32_t c0 = id, c1 = n, c2 = d.sim_lo, c3 = d.sim_hi;
    philox4x32_10(c0, c1, c2, c3, d.seed_lo, d.seed_hi);
    box_muller(c0, c1, c2, c3, zn);
  }

  // push and mass update
  const T xn = wrap_periodic(x + d.drift * g0 + d.noise_amp * zn[0], d.L);
  const T yn = wrap_periodic(y + d.drift * g1 + d.noise_amp * zn[1], d.L);
  const T zz = wrap_periodic(z + d.drift * g2 + d.noise_amp * zn[2], d.L);
  const T rho = (T)2 * gw / ((T)1 + gw);
  double an;
  if (d.flags & SIPF_FLAG_LINEAR_MASS)
    an = a * (1.0 + d.dt * (double)rho - d.dt);
  else
    an = a * exp(d.dt * ((double)rho - 1.0));
  d.x[i] = xn;
  d.y[i] = yn;
  d.z[i] = zz;
  d.a[i] = an;

  // deposit of the new state: ubar^{n+1}
  const Stencil<T> sn = make_stencil(xn, yn, zz, d.inv_h, N);
  deposit_stencil(d.ubar, sn, (T)an * d.inv_h3, N);
}

// Standalone deposit of the current particles (initialisation).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_deposit(Batch<T> bt) {
  int lb;
  const int s = find_sim(bt, K_DEPOSIT, lb);
  const SimDev<T>& d = bt.sims[s];
  const int64_t i = (int64_t)lb * kThreads + threadIdx.x;
  if (i >= d.P) return;
  const Stencil<T> st = make_stencil(d.x[i], d.y[i], d.z[i], d.inv_h, d.N);
  deposit_stencil(d.ubar, st, (T)d.a[i] * d.inv_h3, d.N);
}

template <typename T>
void launch_particles(const Batch<T>& b, int nblk, hipStream_t st) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(k_particles<T>, dim3(nblk), dim3(kThreads), 0, st, b);
}
template <typename T>
void launch_deposit(const Batch<T>& b, int nblk, hipStream_t st) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(k_deposit<T>, dim3(nblk), dim3(kThreads), 0, st, b);
}
template void launch_particles<double>(const Batch<double>&, int, hipStream_t);
template void launch_particles<float>(const Batch<float>&, int, hipStream_t);
template void launch_deposit<double>(const Batch<double>&, int, hipStream_t);
template void launch_deposit<float>(const Batch<float>&, int, hipStream_t);

}  // namespace sipf
