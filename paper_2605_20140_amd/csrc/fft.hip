// Grid half of the SIPF-W step on gfx950: explicit reaction, three-dimensional real FFTs,
// implicit diffusion-decay solves for m and w, and the spectral gradient of v.
//
// Data layout.  Real fields are N^3 row-major [i1][i2][i3].  Spectra are half spectra in
// the transposed layout S[k3][i1][i2] with k3 in [0, N/2]: the z (i3) transform is done
// first on contiguous rows and writes k3-major, so that every later pass reads and writes
// contiguous runs (y lines are contiguous, x lines are strided by N with runs of
// consecutive i2 per block).
//
// Passes per step (each one kernel; transforms in LDS, radix 2):
//   zfwd : reaction (eq. g_hat_phy with S of eq. g_t) on (ubar, m, v, w) at time n, writes
//          v^{n+1} and clears ubar; real z transforms of m*, w* (packed as m* + i w*) and of
//          v^n (two rows packed) -> SM, SW, SV.
//   yfwd : y transforms of SM, SW, SV (in place).
//   xpass: x transforms, the diagonal multipliers of eq. k_q_tilde_update (m: decay beta,
//          diffusion D_m; w: decay 1, diffusion D_w) and the x-derivative multiplier of
//          eq. gradv (i (2 pi/L) q_1, Nyquist zeroed), inverse x transforms -> SM, SW, SGx.
//   yinv : inverse y transforms of SM, SW, SGx, and of SV together with the y-derivative
//          spectrum SGy = i (2 pi/L) q_2 SV.  SV is transformed along y and z only (x stays
//          in physical space), so the derivatives formed from it carry 1/N^2.
//   zinv : forms the z-derivative spectrum i (2 pi/L) q_3 SV, inverse real z transforms of
//          (SM, SW), (SGx, SGy) and of row pairs of the z derivative; writes m^{n+1},
//          w^{n+1} and the gather array g4 = (d1 v^n, d2 v^n, d3 v^n, w^n).
// Forward transforms are decimation in time (bit-reversed input order, natural output);
// inverse transforms are decimation in frequency (natural input, bit-reversed output), so
// no transform needs an explicit reordering step.  Inverse transforms are unnormalised; the
// 1/N^3 factor is folded into the multipliers.
#include "diag_acc.h"

namespace sipf {

template <> int elems_per_block<double>() { return 1024; }
template <> int elems_per_block<float>() { return 2048; }

template <typename T>
void block_counts(const SimDev<T>& d, int c[K_COUNT]) {
  const int64_t N = d.N;
  const int64_t H = N / 2 + 1;
  const int64_t lines = H * N;
  const int64_t Bl = d.lines_per_blk;
  const int64_t ny = (lines + Bl - 1) / Bl;
  const int64_t ny2 = (lines + Bl / 2 - 1) / (Bl / 2);
  c[K_ZFWD] = (int)(N * N / d.rows_per_blk);
  c[K_YFWD] = (int)(3 * ny);
  c[K_XPASS] = (int)(3 * H * (N / d.cols_per_blk));
  c[K_YINV] = (int)(3 * ny + ny2);
  c[K_ZINV] = c[K_ZFWD];
  const int64_t pb = (d.P + kThreads - 1) / kThreads;
  c[K_PART] = d.max_chunks;  // bound on the number of (tile, chunk) items
  c[K_SCOUNT] = (int)((d.P + kBinBlock - 1) / kBinBlock);
  c[K_SSCAN] = 1;
  c[K_SSCATTER] = (int)pb;
  const int64_t work = d.P > N * N * N ? d.P : N * N * N;
  int64_t db = (work + kThreads * 8 - 1) / (kThreads * 8);
  if (db < 1) db = 1;
  if (db > 1024) db = 1024;
  c[K_DIAG] = (int)db;
}
template void block_counts<double>(const SimDev<double>&, int*);
template void block_counts<float>(const SimDev<float>&, int*);

// ---- radix-2 transforms of many lines held in LDS -----------------------------------------
// Lines of length N = 2^lg are stored back to back.  tw[k] = exp(-2 pi i k / N), k < N/2.
// Decimation in time: input in bit-reversed order, output natural.  sgn = +1 forward
// (exp(-i)), -1 inverse (exp(+i)).
template <typename T>
__device__ void fft_dit(cplx<T>* buf, int nlines, int N, int lg, const cplx<T>* tw, T sgn) {
  const int half = N >> 1;
  const int nbf = nlines * half;
  for (int s = 0; s < lg; ++s) {
    __syncthreads();
    const int hs = 1 << s;
    const int tstep = half >> s;
    for (int b = threadIdx.x; b < nbf; b += kThreads) {
      const int line = b >> (lg - 1);
      const int j = b & (half - 1);
      const int k = j & (hs - 1);
      const int i0 = ((j >> s) << (s + 1)) + k;
      cplx<T> w = tw[k * tstep];
      w.y *= sgn;
      cplx<T>* Lp = buf + line * N;
      const cplx<T> a = Lp[i0];
      const cplx<T> t = cmul(Lp[i0 + hs], w);
      Lp[i0] = cadd(a, t);
      Lp[i0 + hs] = csub(a, t);
    }
  }
  __syncthreads();
}

// Decimation in frequency: input natural, output in bit-reversed order.
template <typename T>
__device__ void fft_dif(cplx<T>* buf, int nlines, int N, int lg, const cplx<T>* tw, T sgn) {
  const int half = N >> 1;
  const int nbf = nlines * half;
  for (int s = lg - 1; s >= 0; --s) {
    __syncthreads();
    const int hs = 1 << s;
    const int tstep = half >> s;
    for (int b = threadIdx.x; b < nbf; b += kThreads) {
      const int line = b >> (lg - 1);
      const int j = b & (half - 1);
      const int k = j & (hs - 1);
      const int i0 = ((j >> s) << (s + 1)) + k;
      cplx<T> w = tw[k * tstep];
      w.y *= sgn;
      cplx<T>* Lp = buf + line * N;
      const cplx<T> a = Lp[i0];
      const cplx<T> b2 = Lp[i0 + hs];
      Lp[i0] = cadd(a, b2);
      Lp[i0 + hs] = cmul(csub(a, b2), w);
    }
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* tw, const SimDev<T>& d) {
  for (int k = threadIdx.x; k < (d.N >> 1); k += kThreads) tw[k] = d.tw[k];
}

// signed derivative frequency for index k of an N-point axis (Nyquist -> 0)
__device__ __forceinline__ int deriv_freq(int k, int N) {
  return k < (N >> 1) ? k : (k == (N >> 1) ? 0 : k - N);
}
// signed frequency for |q|^2 (Nyquist kept as -N/2)
__device__ __forceinline__ int lap_freq(int k, int N) { return k < (N >> 1) ? k : k - N; }

// ---- zfwd ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads) k_zfwd(Batch<T> bt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim(bt, K_ZFWD, lb);
  const SimDev<T>& d = bt.sims[s];
  const int N = d.N, lg = d.log2N, B = d.rows_per_blk;
  const int64_t N2 = (int64_t)N * N;
  const int64_t r0 = (int64_t)lb * B;
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);  // B lines: m* + i w*
  cplx<T>* Vp = A + B * N;                             // B/2 lines: v(row 2q) + i v(row 2q+1)
  cplx<T>* tw = Vp + (B >> 1) * N;
  load_twiddles(tw, d);
  const T dt = (T)d.dt, gam = (T)d.gamma, adt = (T)(d.alpha * d.dt);
  const bool freeze_v = d.flags & SIPF_FLAG_FREEZE_V;
  const bool impl_v = d.flags & SIPF_FLAG_IMPLICIT_V;
  Acc acc;
  acc_init(acc);
  for (int e = threadIdx.x; e < B * N; e += kThreads) {
    const int rr = e >> lg, iz = e & (N - 1);
    const int64_t g = (r0 + rr) * N + iz;
    const T u = d.ubar[g], mm = d.m[g], vv = d.v[g], ww = d.w[g];
    const T ms = mm + dt * u;
    const T eta = (T)2 * u / ((T)1 + u);
    const T wsr = ww + dt * (gam * vv - eta * ww);
    T vn = vv;
    if (!freeze_v) {
      vn = impl_v ? vv / ((T)1 + adt * mm) : vv * exp(-adt * mm);
      d.v[g] = vn;
    }
    if (isfinite((double)vn)) acc_min(acc, D_MIN_V, (double)vn); else acc.cnt[0] += 1;
    d.ubar[g] = (T)0;
    const int br = bitrev(iz, lg);
    A[rr * N + br] = cplx<T>{ms, wsr};
    T* vp = reinterpret_cast<T*>(&Vp[(rr >> 1) * N + br]);
    vp[rr & 1] = vv;
  }
  fft_dit(A, B + (B >> 1), N, lg, tw, (T)1);
  const int H = (N >> 1) + 1;
  for (int e = threadIdx.x; e < H * B; e += kThreads) {
    const int kz = e / B, rr = e - kz * B;
    const int kc = (N - kz) & (N - 1);
    const int64_t o = (int64_t)kz * N2 + r0 + rr;
    const cplx<T> Z = A[rr * N + kz], Zc = cconj(A[rr * N + kc]);
    const cplx<T> Ms = cscale(cadd(Z, Zc), (T)0.5);
    const cplx<T> Dm = cscale(csub(Z, Zc), (T)0.5);
    d.SM[o] = Ms;
    d.SW[o] = cplx<T>{Dm.y, -Dm.x};
    const cplx<T> Y = Vp[(rr >> 1) * N + kz], Yc = cconj(Vp[(rr >> 1) * N + kc]);
    cplx<T> Vv;
    if (rr & 1) {
      const cplx<T> Dv = cscale(csub(Y, Yc), (T)0.5);
      Vv = cplx<T>{Dv.y, -Dv.x};
    } else {
      Vv = cscale(cadd(Y, Yc), (T)0.5);
    }
    d.SV[o] = Vv;
  }
  acc_flush(acc, diag_stripe(d));
}

// ---- y passes -------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads) k_yfwd(Batch<T> bt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim(bt, K_YFWD, lb);
  const SimDev<T>& d = bt.sims[s];
  const int N = d.N, lg = d.log2N, Bl = d.lines_per_blk;
  const int64_t lines = (int64_t)((N >> 1) + 1) * N;
  const int nbf = (int)((lines + Bl - 1) / Bl);
  const int f = lb / nbf;
  const int64_t l0 = (int64_t)(lb - f * nbf) * Bl;
  const int nl = (int)((lines - l0) < Bl ? (lines - l0) : Bl);
  cplx<T>* S = f == 0 ? d.SM : (f == 1 ? d.SW : d.SV);
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tw = buf + Bl * N;
  load_twiddles(tw, d);
  const cplx<T>* src = S + l0 * N;
  for (int e = threadIdx.x; e < nl * N; e += kThreads) {
    const int line = e >> lg, j = e & (N - 1);
    buf[line * N + bitrev(j, lg)] = src[e];
  }
  fft_dit(buf, nl, N, lg, tw, (T)1);
  cplx<T>* dst = S + l0 * N;
  for (int e = threadIdx.x; e < nl * N; e += kThreads) dst[e] = buf[e];
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_yinv(Batch<T> bt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim(bt, K_YINV, lb);
  const SimDev<T>& d = bt.sims[s];
  const int N = d.N, lg = d.log2N, Bl = d.lines_per_blk;
  const int64_t lines = (int64_t)((N >> 1) + 1) * N;
  const int nb1 = (int)((lines + Bl - 1) / Bl);
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tw = buf + Bl * N;
  load_twiddles(tw, d);
  if (lb < 3 * nb1) {
    const int f = lb / nb1;
    const int64_t l0 = (int64_t)(lb - f * nb1) * Bl;
    const int nl = (int)((lines - l0) < Bl ? (lines - l0) : Bl);
    cplx<T>* S = (f == 0 ? d.SM : (f == 1 ? d.SW : d.SGx)) + l0 * N;
    for (int e = threadIdx.x; e < nl * N; e += kThreads) buf[e] = S[e];
    fft_dif(buf, nl, N, lg, tw, (T)-1);
    for (int e = threadIdx.x; e < nl * N; e += kThreads) {
      const int line = e >> lg, j = e & (N - 1);
      S[e] = buf[line * N + bitrev(j, lg)];
    }
  } else {
    // SV lines: transform SV and form + transform SGy = i (2 pi/L) q2 SV / N^3
    const int Bh = Bl >> 1;
    const int64_t l0 = (int64_t)(lb - 3 * nb1) * Bh;
    const int nl = (int)((lines - l0) < Bh ? (lines - l0) : Bh);
    const cplx<T>* SV = d.SV + l0 * N;
    // SV is never transformed along x, so its round trip scales by N^2 only
    const T c = d.two_pi_over_L * d.inv_n2;
    for (int e = threadIdx.x; e < nl * N; e += kThreads) {
      const int line = e >> lg, j = e & (N - 1);
      const cplx<T> V = SV[e];
      const T kk = c * (T)deriv_freq(j, N);
      buf[(2 * line) * N + j] = V;
      buf[(2 * line + 1) * N + j] = cplx<T>{-kk * V.y, kk * V.x};
    }
    fft_dif(buf, 2 * nl, N, lg, tw, (T)-1);
    cplx<T>* dV = d.SV + l0 * N;
    cplx<T>* dG = d.SGy + l0 * N;
    for (int e = threadIdx.x; e < nl * N; e += kThreads) {
      const int line = e >> lg, j = e & (N - 1);
      const int br = bitrev(j, lg);
      dV[e] = buf[(2 * line) * N + br];
      dG[e] = buf[(2 * line + 1) * N + br];
    }
  }
}

// ---- x pass: forward x transform, multipliers, inverse x transform ------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads) k_xpass(Batch<T> bt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim(bt, K_XPASS, lb);
  const SimDev<T>& d = bt.sims[s];
  const int N = d.N, lg = d.log2N, Bx = d.cols_per_blk;
  const int H = (N >> 1) + 1;
  const int ncb = N / Bx;
  const int per_field = H * ncb;
  const int f = lb / per_field;
  const int rem = lb - f * per_field;
  const int kz = rem / ncb;
  const int y0 = (rem - kz * ncb) * Bx;
  const int64_t N2 = (int64_t)N * N;
  const cplx<T>* src = (f == 0 ? d.SM : (f == 1 ? d.SW : d.SV)) + (int64_t)kz * N2;
  cplx<T>* dst = (f == 0 ? d.SM : (f == 1 ? d.SW : d.SGx)) + (int64_t)kz * N2;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);  // Bx lines of N along i1
  cplx<T>* tw = buf + Bx * N;
  load_twiddles(tw, d);
  for (int e = threadIdx.x; e < Bx * N; e += kThreads) {
    const int c = e % Bx, ix = e / Bx;
    buf[c * N + bitrev(ix, lg)] = src[(int64_t)ix * N + y0 + c];
  }
  fft_dit(buf, Bx, N, lg, tw, (T)1);
  const int qz = lap_freq(kz, N);
  const T k0 = d.two_pi_over_L;
  for (int e = threadIdx.x; e < Bx * N; e += kThreads) {
    const int c = e >> lg, kx = e & (N - 1);
    const int ky = y0 + c;
    T mult;
    cplx<T> val = buf[e];
    if (f < 2) {
      const T D = (T)(f == 0 ? d.D_m : d.D_w);
      const T decay = (T)(f == 0 ? d.beta : 1.0);
      if (d.mult_kind == 0) {
        const int qx = lap_freq(kx, N), qy = lap_freq(ky, N);
        const T k2 = k0 * k0 * (T)(qx * qx + qy * qy + qz * qz);
        mult = (T)1 / ((T)1 + (T)d.dt * (decay + D * k2));
      } else {
        const T* tab = d.mtab + f * N;
        mult = (T)exp(-(T)d.dt * decay) * tab[kx] * tab[ky] * tab[kz];
      }
      mult *= d.inv_n3;
      if (d.use_lowpass) {
        const T* lp = d.mtab + 2 * N;
        mult *= lp[kx] * lp[ky] * lp[kz];
      }
      val = cscale(val, mult);
    } else {
      T kk = k0 * (T)deriv_freq(kx, N) * d.inv_n3;
      if (d.use_lowpass) {
        const T* lp = d.mtab + 2 * N;
        kk *= lp[kx] * lp[ky] * lp[kz];
      }
      val = cplx<T>{-kk * val.y, kk * val.x};
    }
    buf[e] = val;
  }
  fft_dif(buf, Bx, N, lg, tw, (T)-1);
  for (int e = threadIdx.x; e < Bx * N; e += kThreads) {
    const int c = e % Bx, ix = e / Bx;
    dst[(int64_t)ix * N + y0 + c] = buf[c * N + bitrev(ix, lg)];
  }
}

// ---- zinv ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads) k_zinv(Batch<T> bt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim(bt, K_ZINV, lb);
  const SimDev<T>& d = bt.sims[s];
  const int N = d.N, lg = d.log2N, B = d.rows_per_blk;
  const int64_t N2 = (int64_t)N * N;
  const int64_t r0 = (int64_t)lb * B;
  const int Bh = B >> 1;
  cplx<T>* MW = reinterpret_cast<cplx<T>*>(smem_raw);  // B lines: m + i w
  cplx<T>* GG = MW + B * N;                            // B lines: d1 v + i d2 v
  cplx<T>* GZ = GG + B * N;                            // B/2 lines: d3 v rows 2q + i 2q+1
  cplx<T>* tw = GZ + Bh * N;
  load_twiddles(tw, d);
  const int H = (N >> 1) + 1;
  const T cz = d.two_pi_over_L * d.inv_n2;  // SV: y and z round trips only
  for (int e = threadIdx.x; e < H * Bh; e += kThreads) {
    const int kz = e / Bh, q = e - kz * Bh;
    const int kc = N - kz;
    const bool mirror = kz > 0 && kz < (N >> 1);
    const T kk = cz * (T)deriv_freq(kz, N);
    cplx<T> gz[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rr = 2 * q + h;
      const int64_t o = (int64_t)kz * N2 + r0 + rr;
      const cplx<T> M = d.SM[o], W = d.SW[o], Gx = d.SGx[o], Gy = d.SGy[o], V = d.SV[o];
      MW[rr * N + kz] = cplx<T>{M.x - W.y, M.y + W.x};
      GG[rr * N + kz] = cplx<T>{Gx.x - Gy.y, Gx.y + Gy.x};
      if (mirror) {
        MW[rr * N + kc] = cplx<T>{M.x + W.y, W.x - M.y};
        GG[rr * N + kc] = cplx<T>{Gx.x + Gy.y, Gy.x - Gx.y};
      }
      gz[h] = cplx<T>{-kk * V.y, kk * V.x};
    }
    GZ[q * N + kz] = cplx<T>{gz[0].x - gz[1].y, gz[0].y + gz[1].x};
    if (mirror) GZ[q * N + kc] = cplx<T>{gz[0].x + gz[1].y, gz[1].x - gz[0].y};
  }
  fft_dif(MW, 2 * B + Bh, N, lg, tw, (T)-1);
  const bool freeze_m = d.flags & SIPF_FLAG_FREEZE_M;
  const bool freeze_w = d.flags & SIPF_FLAG_FREEZE_W;
  Acc acc;
  acc_init(acc);
  for (int e = threadIdx.x; e < B * N; e += kThreads) {
    const int rr = e >> lg, iz = e & (N - 1);
    const int br = bitrev(iz, lg);
    const int64_t g = (r0 + rr) * N + iz;
    const cplx<T> mw = MW[rr * N + br];
    const cplx<T> gg = GG[rr * N + br];
    const cplx<T> gzp = GZ[(rr >> 1) * N + br];
    const T wold = d.w[g];
    d.g4[g] = vec4<T>{gg.x, gg.y, (rr & 1) ? gzp.y : gzp.x, wold};
    T mn = mw.x, wn = mw.y;
    if (!freeze_m) d.m[g] = mn; else mn = d.m[g];
    if (!freeze_w) d.w[g] = wn; else wn = wold;
    const double md = mn, wd = wn;
    if (isfinite(md) && isfinite(wd)) {
      acc.sum[2] += md;
      acc_min(acc, D_MIN_M, md);
      acc_min(acc, D_MAX_M, md);
      acc_min(acc, D_MIN_W, wd);
      acc_min(acc, D_MAX_W, wd);
      acc.cnt[1] += md < 0.0;
      acc.cnt[2] += wd < 0.0;
    } else {
      acc.cnt[0] += 1;
    }
  }
  acc_flush(acc, diag_stripe(d));
}

// ---- LDS sizes and launchers ----------------------------------------------------------------
template <typename T>
size_t fft_lds_bytes(int kind) {
  const size_t E = (size_t)elems_per_block<T>();
  const size_t c = sizeof(cplx<T>);
  const size_t tw = 256 * c;  // N/2 <= 256
  switch (kind) {
    case K_ZFWD: return (E + E / 2) * c + tw;
    case K_YFWD: return E * c + tw;
    case K_YINV: return E * c + tw;
    case K_XPASS: return E * c + tw;
    case K_ZINV: return (2 * E + E / 2) * c + tw;
    default: return 0;
  }
}
template size_t fft_lds_bytes<double>(int);
template size_t fft_lds_bytes<float>(int);

#define SIPF_LAUNCH(KER, KIND)                                                              \
  template <typename T>                                                                     \
  void launch_##KER(const Batch<T>& b, int nblk, hipStream_t st) {                          \
    if (nblk <= 0) return;                                                                  \
    hipLaunchKernelGGL(k_##KER<T>, dim3(nblk), dim3(kThreads), fft_lds_bytes<T>(KIND), st, \
                       b);                                                                  \
  }                                                                                         \
  template void launch_##KER<double>(const Batch<double>&, int, hipStream_t);               \
  template void launch_##KER<float>(const Batch<float>&, int, hipStream_t);

SIPF_LAUNCH(zfwd, K_ZFWD)
SIPF_LAUNCH(yfwd, K_YFWD)
SIPF_LAUNCH(xpass, K_XPASS)
SIPF_LAUNCH(yinv, K_YINV)
SIPF_LAUNCH(zinv, K_ZINV)

}  // namespace sipf
