// Grid half of the SIPF-W step on gfx950: explicit reaction, three-dimensional real FFTs,
// implicit diffusion-decay solves for m and w, and the spectral gradient of v.
//
// Data layout.  Real fields are N^3 row-major [i1][i2][i3].  Spectra are half spectra in
// the transposed layout S[k3][i1][i2] with k3 in [0, N/2]: the z (i3) transform is done
// first on contiguous rows and writes k3-major, so that every later pass reads and writes
// contiguous runs (y lines are contiguous, x lines are strided by N with runs of
// consecutive i2 per block).  Along y the spectra are kept in the order the forward line
// transform leaves them in (see below); the multipliers map positions to frequencies.
//
// Passes per step (each one kernel):
//   zfwd : reaction (eq. g_hat_phy with S of eq. g_t) on (ubar, m, v, w) at time n, writes
//          v^{n+1} and, for the solves in change form (float32), m* (into m) and w* (into
//          ubar^n's array; float64 clears that array here); real z transforms of m*, w*
//          (packed as m* + i w*) and of v^{n+1} (two rows packed) -> SM, SW, SV.
//   yfwd : y transforms of SM and SW (in place).  V needs only its three derivatives, each a
//          round trip along its own axis after the z transform: this pass makes the y one,
//          SGy = inverse y (i (2 pi/L) q_2 y transform of SV).
//   xpass: x transforms, the diagonal multipliers of eq. k_q_tilde_update (M - 1 in change
//          form; m: decay beta, diffusion D_m; w: decay 1, diffusion D_w) and, for SV, the
//          x-derivative multiplier of eq. gradv (i (2 pi/L) q_1, Nyquist zeroed), inverse x
//          transforms -> SM, SW, SGx.
//   yinv : inverse y transforms of SM and SW.
//          With the low-pass filter exp(-2 pi^2 |q|^2 / H0^2) (Alg. p2g text, Alg. sipf-pic)
//          V needs its full transform: yfwd transforms SV in place like SM and SW, the filter
//          multiplies the m, w and d1 v spectra in the x pass, a fourth x-pass job writes the
//          filtered V (x round trip undone) into a buffer of its own, SVg, and yinv also
//          transforms SGx back and forms, from SVg, the y-derivative spectrum
//          SGy = i (2 pi/L) q_2 SVg.  Without the filter SVg is SV itself.  Either way SVg
//          leaves x (and, without the filter, y) in physical space, which sets the scale of
//          the derivatives formed from it (gz_scale).
//   zinv : forms the z-derivative spectrum i (2 pi/L) q_3 SVg, inverse real z transforms of
//          (SM, SW), (SGx, SGy) and of row pairs of the z derivative; writes m^{n+1} and
//          w^{n+1} (in change form m* + change and w* + change, then clearing ubar^n's array
//          for the next step's deposit; see the solves below), and the gather array of the
//          next step g4 = (d1 v^{n+1}, d2 v^{n+1}, d3 v^{n+1}, w^{n+1}).
// The particle pass of step n gathers (grad v^n, w^n) from the array the previous step's
// passes formed (at initialisation, these passes run once in gradient-only mode on v^0, w^0),
// so the field passes and the particle pass of one step are independent and run side by
// side; the gather array and ubar are double-buffered by the parity of n.
//
// Line transforms (length N = N1 N2, held in LDS): four-step.  Forward: N1 transforms of
// length N2 over stride-N1 subsequences, twiddles W_N^{n1 k2}, then N2 transforms of length N1
// over contiguous runs; each sub-transform runs in registers (unrolled radix 2).  The result
// X[k2 + N2 k1] stays at position k1 + N1 k2 (fpos).  The inverse takes exactly that order and
// returns natural order, so transform -> multiply -> inverse needs no reordering.  Two LDS
// barriers per transform.  Inverse transforms are unnormalised; the 1/N^3 (or 1/N^2) factor
// is folded into the multipliers.
#include <algorithm>

#include "sipf_internal.h"

namespace sipf {

// elements per thread whose global loads the z passes issue before any of their stores:
// all of a block's elements (B N = elems_per_block, over kThreads threads) in one batch
template <typename T> struct ZBatch { static constexpr int n = sizeof(T) == 4 ? 8 : 4; };

template <> int elems_per_block<double>() { return 1024; }
template <> int elems_per_block<float>() { return 2048; }

template <typename T>
void block_counts(const SimDev<T>& d, int c[K_COUNT]) {
  const int64_t N = d.N;
  const int64_t H = N / 2 + 1;
  const int64_t lines = H * N;
  // y passes (3D only; there N <= 512, so at least two lines per block)
  const int64_t Bl = d.lines_per_blk > 1 ? d.lines_per_blk : 2;
  const int64_t ny = (lines + Bl - 1) / Bl;
  const int64_t ny2 = (lines + Bl / 2 - 1) / (Bl / 2);
  c[K_ZFWD] = (int)(d.nrows / d.rows_per_blk);
  const int64_t nlp = d.use_lowpass ? 1 : 0;  // filtered copy of V as an extra job
  if (d.dim == 2) {  // row pass, one column pass (k_xpass), inverse row pass
    c[K_YFWD] = 0;
    c[K_XPASS] = (int)((3 + nlp) * ((H + d.cols_per_blk - 1) / d.cols_per_blk));
    c[K_YINV] = 0;
    c[K_PLANE] = 0;
  } else {
    c[K_YFWD] = d.use_plane ? 0 : (int)(3 * ny);
    c[K_XPASS] = d.use_plane ? 0 : (int)((3 + nlp) * H * (N / d.cols_per_blk));
    // inverse y of M and W; with the filter also of d1 V and of the filtered V (+ d2 V)
    c[K_YINV] = d.use_plane ? 0 : (int)(nlp ? 3 * ny + ny2 : 2 * ny);
    // plane jobs: M, W and one for both V derivatives; with the filter M, W, d1 V, d2 V, V
    c[K_PLANE] = d.use_plane ? (int)((nlp ? 5 : 3) * H) : 0;
  }
  c[K_ZINV] = (int)(d.nrows / d.rows_zinv);
  const int64_t pb = (d.P + kThreads - 1) / kThreads;
  c[K_PART] = d.max_chunks;  // bound on the number of (tile, chunk) items
  c[K_SCOUNT] = (int)((d.P + kBinBlock - 1) / kBinBlock);
  // one scan block per segment of 16 kThreads tiles; the scatter also clears the tile counts
  c[K_SSCAN] = (int)((d.ntiles + 16 * kThreads - 1) / (16 * kThreads));
  const int64_t tb = (d.ntiles + kThreads - 1) / kThreads;
  c[K_SSCATTER] = (int)(pb > tb ? pb : tb);
  const int64_t work = d.P > d.G ? d.P : d.G;
  int64_t db = (work + kThreads * 8 - 1) / (kThreads * 8);
  if (db < 1) db = 1;
  if (db > 1024) db = 1024;
  c[K_DIAG] = (int)db;
}
template void block_counts<double>(const SimDev<double>&, int*);
template void block_counts<float>(const SimDev<float>&, int*);

// ---- register transforms ----------------------------------------------------------------
// exp(2 pi i k / 32) for k < 16, correctly rounded
struct W32 {
  double c, s;
};
__device__ constexpr W32 kW32[16] = {
    {1.0, 0.0},
    {0.9807852804032304, 0.19509032201612828},
    {0.9238795325112867, 0.3826834323650898},
    {0.8314696123025452, 0.5555702330196022},
    {0.7071067811865476, 0.7071067811865476},
    {0.5555702330196022, 0.8314696123025452},
    {0.3826834323650898, 0.9238795325112867},
    {0.19509032201612828, 0.9807852804032304},
    {0.0, 1.0},
    {-0.19509032201612828, 0.9807852804032304},
    {-0.3826834323650898, 0.9238795325112867},
    {-0.5555702330196022, 0.8314696123025452},
    {-0.7071067811865476, 0.7071067811865476},
    {-0.8314696123025452, 0.5555702330196022},
    {-0.9238795325112867, 0.3826834323650898},
    {-0.9807852804032304, 0.19509032201612828},
};

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }
constexpr int brevc(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
  return r;
}

// In-register DFT of length R <= 32, natural order in and out.  DIR = +1: exp(-2 pi i jk/R);
// DIR = -1: exp(+2 pi i jk/R).
template <typename T, int R, int DIR>
__device__ __forceinline__ void reg_dft(cplx<T> (&a)[R]) {
  constexpr int LR = ilog2c(R);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = brevc(i, LR);
    if (j > i) {
      const cplx<T> t = a[i];
      a[i] = a[j];
      a[j] = t;
    }
  }
#pragma unroll
  for (int s = 0; s < LR; ++s) {
    const int hs = 1 << s;
#pragma unroll
    for (int j = 0; j < R / 2; ++j) {
      const int k = j & (hs - 1);
      const int i0 = ((j >> s) << (s + 1)) + k;
      const int ti = k * (32 >> (s + 1));
      const cplx<T> u = a[i0];
      cplx<T> v = a[i0 + hs];
      if (ti == 8)  // the twiddle is -DIR i: a swap of the parts and one sign, no products
        v = DIR > 0 ? cplx<T>{v.y, -v.x} : cplx<T>{-v.y, v.x};
      else if (k != 0)
        v = cmul(v, cplx<T>{(T)kW32[ti].c, (T)(-DIR * kW32[ti].s)});
      a[i0] = cadd(u, v);
      a[i0 + hs] = csub(u, v);
    }
  }
}

template <int LG>
struct Split {
  static constexpr int L1 = LG / 2, L2 = LG - LG / 2;
  static constexpr int N1 = 1 << L1, N2 = 1 << L2, N = 1 << LG;
};

// The z and y passes read and write their lines across rows (one row per thread when
// packing spectra), so they pad by one complex value (an odd stride spreads consecutive rows
// over all LDS banks) and map consecutive threads to consecutive lines in the transforms.
template <int LG>
constexpr int zy_stride() {
  return (1 << LG) + 1;
}
inline int zy_stride_rt(int lg) { return (1 << lg) + 1; }
// The plane kernel transforms rows and columns of one plane with one line per thread; a
// stride of N + 2 spreads consecutive rows over the LDS banks and keeps rows 16-byte aligned.
template <int LG>
constexpr int plane_stride() {
  return (1 << LG) + 2;
}
// Lines whose sub-transforms run one per thread on consecutive threads (the x pass, the 2D
// column pass) are stored skewed: position p at p + floor(p / N1), one gap after every group
// of N1.  The second stage's threads then read their groups N1 + 1 values apart instead of
// N1, which spreads them over the LDS banks (N1 apart, 16 threads of a wavefront met on the
// same banks).  The odd line stride N + N2 + 1 holds the N2 - 1 gaps.
template <int LG, bool SKEW>
constexpr int group_stride() {
  return Split<LG>::N1 + (SKEW ? 1 : 0);
}
template <int LG, bool SKEW>
__device__ __forceinline__ int skp(int p) {
  return SKEW ? p + (p >> Split<LG>::L1) : p;
}
template <int LG>
constexpr int skew_stride() {
  return (1 << LG) + Split<LG>::N2 + 1;
}
inline int skew_stride_rt(int lg) { return (1 << lg) + (1 << (lg - lg / 2)) + 1; }

// position of frequency k after a forward line transform, and its inverse map
template <int LG>
__device__ __forceinline__ int fpos(int k) {
  using S = Split<LG>;
  return (k >> S::L2) + ((k & (S::N2 - 1)) << S::L1);
}
template <int LG>
__device__ __forceinline__ int ufpos(int p) {
  using S = Split<LG>;
  return (p >> S::L1) + ((p & (S::N1 - 1)) << S::L2);
}

// Entries of a pass's twiddle table in LDS: all N powers W_N^k up to N = 512, so that a
// twiddle is one load; at N = 1024 (the 2D form's largest rows) the N/2 of the first half
// only, which keeps its blocks' LDS within the occupancy they have (the second half is the
// first negated).
template <int LG>
constexpr int tw_len() {
  return LG <= 9 ? (1 << LG) : (1 << LG) >> 1;
}
inline int tw_len_rt(int lg) { return lg <= 9 ? (1 << lg) : (1 << lg) >> 1; }

// W_N^e (DIR +1) or W_N^{-e} (DIR -1) for 0 <= e < N from the table tw[k] = W_N^k
template <typename T, int LG, int DIR>
__device__ __forceinline__ cplx<T> twid(const cplx<T>* tw, int e) {
  constexpr int H = (1 << LG) >> 1;
  cplx<T> w;
  if (tw_len<LG>() == (1 << LG))
    w = tw[e];
  else
    w = e < H ? tw[e] : cplx<T>{-tw[e - H].x, -tw[e - H].y};
  if (DIR < 0) w.y = -w.y;
  return w;
}

// Line transforms over nlines lines of buf: element n of line l at buf[l * ls + n * es].
// NT threads cooperate.  LINE_FAST maps consecutive threads to consecutive lines (for
// columns, es > 1, so that a wavefront touches consecutive LDS words); otherwise to
// consecutive elements of one line.
template <int LG, bool LINE_FAST>
struct TaskMap {
  // task t -> (line, sub-index < R) for sub-transforms of R = 2^LR
  template <int LR>
  __device__ static __forceinline__ void map(int t, int nlines, int& line, int& j) {
    if (LINE_FAST) {
      line = t % nlines;
      j = t / nlines;
    } else {
      line = t >> LR;
      j = t & ((1 << LR) - 1);
    }
  }
};

// Four-step line transforms (N = N1 N2).  Forward, first stage: N2-point transforms of the
// N1 strided subsequences, times the twiddles; second stage: N1-point transforms of
// contiguous groups, leaving frequency k at position fpos(k).  The inverse takes that order
// and runs the stages the other way round.  Each stage ends at a barrier.
template <typename T, int LG, bool LINE_FAST, int NT, bool SKEW = false>
__device__ __forceinline__ void fwd_stage1(cplx<T>* buf, int nlines, int ls, int es,
                                           const cplx<T>* tw) {
  using S = Split<LG>;
  constexpr int GS = group_stride<LG, SKEW>();
  for (int t = threadIdx.x; t < nlines * S::N1; t += NT) {
    int line, n1;
    TaskMap<LG, LINE_FAST>::template map<S::L1>(t, nlines, line, n1);
    cplx<T>* Lp = buf + line * ls + n1 * es;
    cplx<T> a[S::N2];
#pragma unroll
    for (int n2 = 0; n2 < S::N2; ++n2) a[n2] = Lp[n2 * GS * es];
    reg_dft<T, S::N2, 1>(a);
    Lp[0] = a[0];
#pragma unroll
    for (int k2 = 1; k2 < S::N2; ++k2)
      Lp[k2 * GS * es] = cmul(a[k2], twid<T, LG, 1>(tw, n1 * k2));
  }
  __syncthreads();
}
template <typename T, int LG, bool LINE_FAST, int NT, bool SKEW = false>
__device__ __forceinline__ void fwd_stage2(cplx<T>* buf, int nlines, int ls, int es) {
  using S = Split<LG>;
  constexpr int GS = group_stride<LG, SKEW>();
  for (int t = threadIdx.x; t < nlines * S::N2; t += NT) {
    int line, k2;
    TaskMap<LG, LINE_FAST>::template map<S::L2>(t, nlines, line, k2);
    cplx<T>* Lp = buf + line * ls + k2 * GS * es;
    cplx<T> a[S::N1];
#pragma unroll
    for (int n1 = 0; n1 < S::N1; ++n1) a[n1] = Lp[n1 * es];
    reg_dft<T, S::N1, 1>(a);
#pragma unroll
    for (int k1 = 0; k1 < S::N1; ++k1) Lp[k1 * es] = a[k1];
  }
  __syncthreads();
}
template <typename T, int LG, bool LINE_FAST, int NT, bool SKEW = false>
__device__ __forceinline__ void inv_stage1(cplx<T>* buf, int nlines, int ls, int es,
                                           const cplx<T>* tw) {
  using S = Split<LG>;
  constexpr int GS = group_stride<LG, SKEW>();
  for (int t = threadIdx.x; t < nlines * S::N2; t += NT) {
    int line, a2;
    TaskMap<LG, LINE_FAST>::template map<S::L2>(t, nlines, line, a2);
    cplx<T>* Lp = buf + line * ls + a2 * GS * es;
    cplx<T> v[S::N1];
#pragma unroll
    for (int b = 0; b < S::N1; ++b) v[b] = Lp[b * es];
    reg_dft<T, S::N1, -1>(v);
    Lp[0] = v[0];
#pragma unroll
    for (int c = 1; c < S::N1; ++c) Lp[c * es] = cmul(v[c], twid<T, LG, -1>(tw, c * a2));
  }
  __syncthreads();
}
template <typename T, int LG, bool LINE_FAST, int NT, bool SKEW = false>
__device__ __forceinline__ void inv_stage2(cplx<T>* buf, int nlines, int ls, int es) {
  using S = Split<LG>;
  constexpr int GS = group_stride<LG, SKEW>();
  for (int t = threadIdx.x; t < nlines * S::N1; t += NT) {
    int line, c;
    TaskMap<LG, LINE_FAST>::template map<S::L1>(t, nlines, line, c);
    cplx<T>* Lp = buf + line * ls + c * es;
    cplx<T> v[S::N2];
#pragma unroll
    for (int a2 = 0; a2 < S::N2; ++a2) v[a2] = Lp[a2 * GS * es];
    reg_dft<T, S::N2, -1>(v);
#pragma unroll
    for (int dd = 0; dd < S::N2; ++dd) Lp[dd * GS * es] = v[dd];
  }
  __syncthreads();
}

// forward transforms: natural order -> fpos order
template <typename T, int LG, bool LINE_FAST = false, int NT = kThreads>
__device__ __forceinline__ void line_fwd(cplx<T>* buf, int nlines, int ls, int es, const cplx<T>* tw) {
  fwd_stage1<T, LG, LINE_FAST, NT>(buf, nlines, ls, es, tw);
  fwd_stage2<T, LG, LINE_FAST, NT>(buf, nlines, ls, es);
}
// inverse transforms (unnormalised): fpos order -> natural order
template <typename T, int LG, bool LINE_FAST = false, int NT = kThreads, bool SKEW = false>
__device__ __forceinline__ void line_inv(cplx<T>* buf, int nlines, int ls, int es, const cplx<T>* tw) {
  inv_stage1<T, LG, LINE_FAST, NT, SKEW>(buf, nlines, ls, es, tw);
  inv_stage2<T, LG, LINE_FAST, NT, SKEW>(buf, nlines, ls, es);
}

// Forward transform, pointwise multiplier and inverse transform of nlines lines.  The
// forward second stage and the inverse first stage work on the same groups of N1 elements
// with the same thread mapping, so the multiplier is applied in registers between them: one
// LDS pass and one barrier less than the transforms alone, and no pass for the multiplier.
// mul(line, p, v) returns v times the multiplier of position p (frequency ufpos(p)).
// (Above 128 points the two transforms and the multiplier in registers cost more registers
// than the pass saves - the x pass at 256 points went from 7 to 3 waves per SIMD in float32
// - so there the multiplier is a pass of its own.)
template <typename T, int LG, bool LINE_FAST, int NT, bool SKEW = false, typename Mul>
__device__ __forceinline__ void line_round_trip(cplx<T>* buf, int nlines, int ls, int es,
                                                const cplx<T>* tw, const Mul& mul) {
  using S = Split<LG>;
  constexpr int GS = group_stride<LG, SKEW>();
  fwd_stage1<T, LG, LINE_FAST, NT, SKEW>(buf, nlines, ls, es, tw);
  if (LG > 7) {
    fwd_stage2<T, LG, LINE_FAST, NT, SKEW>(buf, nlines, ls, es);
    if (NT % (1 << LG) == 0) {  // each thread keeps one position p on every line it visits
      const int p = threadIdx.x & ((1 << LG) - 1);
      for (int line = threadIdx.x >> LG; line < nlines; line += NT >> LG) {
        cplx<T>* q = buf + line * ls + skp<LG, SKEW>(p) * es;
        *q = mul(line, p, *q);
      }
    } else {
      for (int e = threadIdx.x; e < (nlines << LG); e += NT) {
        const int line = e >> LG, p = e & ((1 << LG) - 1);
        cplx<T>* q = buf + line * ls + skp<LG, SKEW>(p) * es;
        *q = mul(line, p, *q);
      }
    }
    __syncthreads();
    line_inv<T, LG, LINE_FAST, NT, SKEW>(buf, nlines, ls, es, tw);
    return;
  }
  for (int t = threadIdx.x; t < nlines * S::N2; t += NT) {
    int line, k2;
    TaskMap<LG, LINE_FAST>::template map<S::L2>(t, nlines, line, k2);
    cplx<T>* Lp = buf + line * ls + k2 * GS * es;
    cplx<T> a[S::N1];
#pragma unroll
    for (int n1 = 0; n1 < S::N1; ++n1) a[n1] = Lp[n1 * es];
    reg_dft<T, S::N1, 1>(a);
#pragma unroll
    for (int k1 = 0; k1 < S::N1; ++k1) a[k1] = mul(line, (k2 << S::L1) + k1, a[k1]);
    reg_dft<T, S::N1, -1>(a);
    Lp[0] = a[0];
#pragma unroll
    for (int c = 1; c < S::N1; ++c) Lp[c * es] = cmul(a[c], twid<T, LG, -1>(tw, c * k2));
  }
  __syncthreads();
  inv_stage2<T, LG, LINE_FAST, NT, SKEW>(buf, nlines, ls, es);
}

// The pass's LDS twiddle table (tw_len entries) from the N/2 values W_N^k, k < N/2, in
// global memory: W_N^{k + N/2} = -W_N^k.
template <typename T, int LG>
__device__ __forceinline__ void load_twiddles(cplx<T>* tw, SimC<T>& d) {
  constexpr int H = (1 << LG) >> 1;
  for (int k = threadIdx.x; k < H; k += kThreads) {
    const cplx<T> v = d.tw[k];
    tw[k] = v;
    if (tw_len<LG>() > H) tw[k + H] = cplx<T>{-v.x, -v.y};
  }
}

// The N/2 twiddles in two steps, so that their loads join a batch of other loads: issue them
// into registers, then (after the batch) write them to LDS.
template <typename T, int LG, int NT>
struct TwiddleRegs {
  static constexpr int K = (((1 << LG) >> 1) + NT - 1) / NT;
  T x[K], y[K];
  __device__ __forceinline__ void load(const cplx<T>* twg) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int t = threadIdx.x + k * NT;
      if (t < ((1 << LG) >> 1)) {
        const cplx<T> v = twg[t];
        x[k] = v.x;
        y[k] = v.y;
      }
    }
  }
  __device__ __forceinline__ void store(cplx<T>* twl) const {
    constexpr int H = (1 << LG) >> 1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int t = threadIdx.x + k * NT;
      if (t < H) {
        twl[t] = cplx<T>{x[k], y[k]};
        if (tw_len<LG>() > H) twl[t + H] = cplx<T>{-x[k], -y[k]};
      }
    }
  }
};

// values per thread whose global loads a copy into LDS keeps in flight together
template <typename T> struct CopyBatch { static constexpr int n = 32 / (int)sizeof(T); };

// n consecutive complex values from global memory into LDS rows of N values at stride LS,
// and (unless twg is null) the N/2 twiddles into twl.  The loads of CopyBatch values per thread (and of the
// twiddles) are in flight together: a plain loop waits for each load before its LDS store,
// one memory round trip per value.  Component arrays keep the batch in registers.
template <typename T, int LG, int NT, bool SKEW = false>
__device__ __forceinline__ void rows_in(cplx<T>* buf, int LS, const cplx<T>* src, int n,
                                        cplx<T>* twl, const cplx<T>* twg) {
  constexpr int N = 1 << LG;
  constexpr int B = CopyBatch<T>::n;
  TwiddleRegs<T, LG, NT> tr;
  if (twg) tr.load(twg);
  for (int e0 = threadIdx.x; e0 < n; e0 += B * NT) {
    T vx[B], vy[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int e = e0 + k * NT;
      if (e < n) {
        const cplx<T> v = src[e];
        vx[k] = v.x;
        vy[k] = v.y;
      }
    }
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int e = e0 + k * NT;
      if (e < n) buf[(e >> LG) * LS + skp<LG, SKEW>(e & (N - 1))] = cplx<T>{vx[k], vy[k]};
    }
  }
  if (twg) tr.store(twl);
}

// signed derivative frequency for index k of an N-point axis (Nyquist -> 0)
__device__ __forceinline__ int deriv_freq(int k, int N) {
  return k < (N >> 1) ? k : (k == (N >> 1) ? 0 : k - N);
}
// signed frequency for |q|^2 (Nyquist kept as -N/2)
__device__ __forceinline__ int lap_freq(int k, int N) { return k < (N >> 1) ? k : k - N; }

// The diffusion-decay solves (eq. k_q_tilde_update), for f = m, w, with M the solve's
// multiplier of one Fourier mode times the low-pass factor lp (1 without the filter).
// Float32 takes them in change form, f^{n+1} = f* + IFFT((M - 1) FFT(f*)): the inverse pass
// adds f* back, so that the rounding of the transforms, relative to the transformed values,
// is scaled by the small M - 1 instead of reaching f^{n+1} in full at every step (it would
// accumulate in m and w, and through v' = v exp(-alpha tau m) in v).  Float64, whose
// transforms round five hundred million times finer, takes the plain form
// f^{n+1} = IFFT(M FFT(f*)), so that m* and w* need not go through HBM between the passes.
template <typename T> constexpr bool change_form() { return sizeof(T) == 4; }
// Implicit multiplier, c = tau (R + D |k|^2): M = lp / (1 + c); in change form
// M - 1 = (lp - 1 - c) / (1 + c).  In float32 the quotient takes the hardware reciprocal
// (within 1 ulp; 1 + c >= 1) instead of the correctly rounded division sequence: about ten
// instructions less per mode.
template <typename T>
__device__ __forceinline__ T solve_multiplier(T c, T lp) {
  static_assert(!change_form<T>(), "float32 is specialised below");
  return lp / ((T)1 + c);
}
template <>
__device__ __forceinline__ float solve_multiplier<float>(float c, float lp) {
  return (lp - 1.0f - c) * __builtin_amdgcn_rcpf(1.0f + c);
}
// the same for a tabulated multiplier M (exponential or aliased kernel)
template <typename T>
__device__ __forceinline__ T table_multiplier(T M, T lp) {
  return change_form<T>() ? M * lp - (T)1 : M * lp;
}

// ---- zfwd ---------------------------------------------------------------------------------
template <typename T, int LG>
__device__ __forceinline__ void zfwd_body(SimC<T>& d, int lb, unsigned char* smem, int mode) {
  constexpr int N = 1 << LG;
  const int B = d.rows_per_blk;
  const int64_t N2 = d.nrows;  // rows per k3 plane of the spectra (N^2; N in 2D)
  const int64_t r0 = (int64_t)lb * B;
  constexpr int LS = zy_stride<LG>();
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);  // B lines: m* + i w*
  cplx<T>* Vp = A + B * LS;                       // B/2 lines: v(row 2q) + i v(row 2q+1)
  cplx<T>* tw = Vp + (B >> 1) * LS;
  TwiddleRegs<T, LG, kThreads> tr;
  tr.load(d.tw);  // in flight with the first batch of field loads
  const T dt = (T)d.dt, gam = (T)d.gamma, adt = (T)(d.alpha * d.dt);
  const bool freeze_v = d.flags & SIPF_FLAG_FREEZE_V;
  const bool freeze_m = d.flags & SIPF_FLAG_FREEZE_M;
  const bool impl_v = d.flags & SIPF_FLAG_IMPLICIT_V;
  const bool grad_only = mode == kGradOnly;
  T* const ub = d.ubar[(uint32_t)(*d.step) & 1u];  // ubar^n
  // ZBatch elements per thread have their loads in flight together (the stores to v and ubar
  // would otherwise order each element's loads after the previous element's stores)
  constexpr int ZB = ZBatch<T>::n;
  const int nel = B * N;
  const int64_t g0 = r0 * N;  // first node of the block's rows
  for (int e0 = threadIdx.x; e0 < nel; e0 += ZB * kThreads) {
    T u[ZB], mm[ZB], vv[ZB], ww[ZB];
#pragma unroll
    for (int k = 0; k < ZB; ++k) {
      const int e = e0 + k * kThreads;
      if (e < nel) {
        vv[k] = d.v[g0 + e];
        if (!grad_only) {
          u[k] = ub[g0 + e];
          mm[k] = d.m[g0 + e];
          ww[k] = d.w[g0 + e];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < ZB; ++k) {
      const int e = e0 + k * kThreads;
      if (e < nel && grad_only) {  // v^n itself; the m and w lines are not used
        const int rr = e >> LG, iz = e & (N - 1);
        A[rr * LS + iz] = cplx<T>{(T)0, (T)0};
        reinterpret_cast<T*>(&Vp[(rr >> 1) * LS + iz])[rr & 1] = vv[k];
      } else if (e < nel) {
        const int rr = e >> LG, iz = e & (N - 1);
        const T ms = mm[k] + dt * u[k];
        // change form: m* in place of m, for the inverse pass to add the solve's change to
        if (change_form<T>() && !freeze_m) d.m[g0 + e] = ms;
        const T eta = (T)2 * u[k] / ((T)1 + u[k]);
        const T wsr = ww[k] + dt * (gam * vv[k] - eta * ww[k]);
        T vn = vv[k];
        if (!freeze_v) {
          // v' = v exp(-y) (or v / (1 + y)), y = alpha tau m, written as v plus its small
          // decrement: the factor itself, rounded next to 1, would carry an absolute error of
          // up to half an ulp of 1 every step, which float32 v accumulates step after step
          const T y = adt * mm[k];
          vn = impl_v ? vv[k] - vv[k] * (y / ((T)1 + y)) : fma(vv[k], expm1(-y), vv[k]);
          d.v[g0 + e] = vn;
        }
        // ubar^n's array, which this step needs no more, is the next step's deposit target: in
        // change form it holds w* until the inverse pass has added it to the solve's change
        // and cleared the array; in plain form it is cleared here
        ub[g0 + e] = change_form<T>() ? wsr : (T)0;
        A[rr * LS + iz] = cplx<T>{ms, wsr};
        // v^{n+1}: its gradient is the next step's gather array
        T* vp = reinterpret_cast<T*>(&Vp[(rr >> 1) * LS + iz]);
        vp[rr & 1] = vn;
      }
    }
  }
  tr.store(tw);
  __syncthreads();
  line_fwd<T, LG, true>(A, B + (B >> 1), LS, 1, tw);
  constexpr int H = (N >> 1) + 1;
  const int lgB = __builtin_ctz((unsigned)B);  // B is a power of two: no vector division
  for (int e = threadIdx.x; e < H * B; e += kThreads) {
    const int kz = e >> lgB, rr = e & (B - 1);
    const int pk = fpos<LG>(kz), pc = fpos<LG>((N - kz) & (N - 1));
    const int64_t o = (int64_t)kz * N2 + r0 + rr;
    const cplx<T> Z = A[rr * LS + pk], Zc = cconj(A[rr * LS + pc]);
    const cplx<T> Ms = cscale(cadd(Z, Zc), (T)0.5);
    const cplx<T> Dm = cscale(csub(Z, Zc), (T)0.5);
    d.SM[o] = Ms;
    d.SW[o] = cplx<T>{Dm.y, -Dm.x};
    const cplx<T> Y = Vp[(rr >> 1) * LS + pk], Yc = cconj(Vp[(rr >> 1) * LS + pc]);
    cplx<T> Vv;
    if (rr & 1) {
      const cplx<T> Dv = cscale(csub(Y, Yc), (T)0.5);
      Vv = cplx<T>{Dv.y, -Dv.x};
    } else {
      Vv = cscale(cadd(Y, Yc), (T)0.5);
    }
    d.SV[o] = Vv;
  }
}

template <typename T, int LG>
__global__ void __launch_bounds__(kThreads) k_zfwd(Batch<T> bt, int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim<kFieldRun>(bt, K_ZFWD, lb);
  zfwd_body<T, LG>(sim_view(bt, s), lb, smem_raw, mode);
}

// ---- y passes -------------------------------------------------------------------------------
// Along y the spectra stay in fpos order between yfwd and yinv.
template <typename T, int LG>
__device__ __forceinline__ void yfwd_body(SimC<T>& d, int lb, unsigned char* smem) {
  constexpr int N = 1 << LG;
  const int Bl = d.lines_per_blk;
  const int64_t lines = (int64_t)((N >> 1) + 1) * N;
  const int nbf = (int)((lines + Bl - 1) / Bl);
  const int fj = lb / nbf;
  const int64_t l0 = (int64_t)(lb - fj * nbf) * Bl;
  // without the filter the V blocks come first, so that the x pass that follows starts on M
  // and W as the last blocks of this pass left them (x pass at 256^3 float32 117.5 ->
  // 104.7 us, y inverse 57 -> 54 us; the step unchanged)
  const int f = d.use_lowpass ? fj : (fj == 0 ? 2 : fj - 1);
  const int nl = (int)((lines - l0) < Bl ? (lines - l0) : Bl);
  const cplx<T>* S = (f == 0 ? d.SM : (f == 1 ? d.SW : d.SV)) + l0 * N;
  // Without the filter V needs no y transform of its own: only its derivative along y,
  // a y round trip of SV with the multiplier i (2 pi/L) q2 into SGy (1/N^2 undoes the z
  // and y round trips).  With the filter V is transformed in place like M and W.
  const bool vround = f == 2 && !d.use_lowpass;
  cplx<T>* dst = (vround ? d.SGy : (f == 0 ? d.SM : (f == 1 ? d.SW : d.SV))) + l0 * N;
  constexpr int LS = zy_stride<LG>();
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = buf + Bl * LS;
  rows_in<T, LG, kThreads>(buf, LS, S, nl * N, tw, d.tw);
  __syncthreads();
  if (vround) {
    const T c = d.two_pi_over_L * d.inv_n2;
    const auto deriv = [c](int, int p, cplx<T> v) {
      const T kk = c * (T)deriv_freq(ufpos<LG>(p), N);
      return cplx<T>{-kk * v.y, kk * v.x};
    };
    line_round_trip<T, LG, true, kThreads>(buf, nl, LS, 1, tw, deriv);
  } else {
    line_fwd<T, LG, true>(buf, nl, LS, 1, tw);
  }
  for (int e = threadIdx.x; e < nl * N; e += kThreads) dst[e] = buf[(e >> LG) * LS + (e & (N - 1))];
}

template <typename T, int LG>
__global__ void __launch_bounds__(kThreads) k_yfwd(Batch<T> bt, int /*mode*/) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim<kFieldRun>(bt, K_YFWD, lb);
  yfwd_body<T, LG>(sim_view(bt, s), lb, smem_raw);
}

template <typename T, int LG>
__device__ __forceinline__ void yinv_body(SimC<T>& d, int lb, unsigned char* smem) {
  constexpr int N = 1 << LG;
  const int Bl = d.lines_per_blk;
  const int64_t lines = (int64_t)((N >> 1) + 1) * N;
  const int nb1 = (int)((lines + Bl - 1) / Bl);
  constexpr int LS = zy_stride<LG>();
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = buf + Bl * LS;
  // jobs M and W; with the filter also d1 V (SGx) and, below, the filtered V lines (the
  // launch has 2 nb1 blocks without the filter)
  if (lb < 3 * nb1) {
    const int f = lb / nb1;
    const int64_t l0 = (int64_t)(lb - f * nb1) * Bl;
    const int nl = (int)((lines - l0) < Bl ? (lines - l0) : Bl);
    cplx<T>* S = (f == 0 ? d.SM : (f == 1 ? d.SW : d.SGx)) + l0 * N;
    rows_in<T, LG, kThreads>(buf, LS, S, nl * N, tw, d.tw);
    __syncthreads();
    line_inv<T, LG, true>(buf, nl, LS, 1, tw);
    for (int e = threadIdx.x; e < nl * N; e += kThreads)
      S[e] = buf[(e >> LG) * LS + (e & (N - 1))];
  } else {
    // filtered V lines (with the filter only): transform SVg and form + transform
    // SGy = i (2 pi/L) q2 SVg / N^2 (SVg is never transformed along x, so its round trip
    // scales by N^2 only)
    const int Bh = Bl >> 1;
    const int64_t l0 = (int64_t)(lb - 3 * nb1) * Bh;
    const int nl = (int)((lines - l0) < Bh ? (lines - l0) : Bh);
    const cplx<T>* SV = d.SVg + l0 * N;
    const T c = d.two_pi_over_L * d.inv_n2;
    TwiddleRegs<T, LG, kThreads> tr;
    tr.load(d.tw);
    // CopyBatch loads per thread in flight together, as in rows_in
    constexpr int CB = CopyBatch<T>::n;
    const int n = nl * N;
    for (int e0 = threadIdx.x; e0 < n; e0 += CB * kThreads) {
      cplx<T> V[CB];
#pragma unroll
      for (int k = 0; k < CB; ++k) {
        const int e = e0 + k * kThreads;
        if (e < n) V[k] = SV[e];
      }
#pragma unroll
      for (int k = 0; k < CB; ++k) {
        const int e = e0 + k * kThreads;
        if (e < n) {
          const int line = e >> LG, p = e & (N - 1);
          const T kk = c * (T)deriv_freq(ufpos<LG>(p), N);
          buf[(2 * line) * LS + p] = V[k];
          buf[(2 * line + 1) * LS + p] = cplx<T>{-kk * V[k].y, kk * V[k].x};
        }
      }
    }
    tr.store(tw);
    __syncthreads();
    line_inv<T, LG, true>(buf, 2 * nl, LS, 1, tw);
    cplx<T>* dV = d.SVg + l0 * N;
    cplx<T>* dG = d.SGy + l0 * N;
    for (int e = threadIdx.x; e < nl * N; e += kThreads) {
      const int line = e >> LG, j = e & (N - 1);
      dV[e] = buf[(2 * line) * LS + j];
      dG[e] = buf[(2 * line + 1) * LS + j];
    }
  }
}

template <typename T, int LG>
__global__ void __launch_bounds__(kThreads) k_yinv(Batch<T> bt, int /*mode*/) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim<kFieldRun>(bt, K_YINV, lb);
  yinv_body<T, LG>(sim_view(bt, s), lb, smem_raw);
}

// ---- x pass: forward x transform, multipliers, inverse x transform ------------------------
template <typename T, int LG>
__device__ __forceinline__ void xpass_body(SimC<T>& d, int lb, unsigned char* smem) {
  constexpr int N = 1 << LG;
  const int Bx = d.cols_per_blk;
  constexpr int H = (N >> 1) + 1;
  const int ncb = N / Bx;
  const int per_field = H * ncb;
  const int f = lb / per_field;
  const int rem = lb - f * per_field;
  const int kz = rem / ncb;
  const int y0 = (rem - kz * ncb) * Bx;
  const int lbx = __builtin_ctz((unsigned)Bx);  // Bx is a power of two: no vector division
  const int64_t N2 = (int64_t)N * N;
  const cplx<T>* src = (f == 0 ? d.SM : (f == 1 ? d.SW : d.SV)) + (int64_t)kz * N2;
  cplx<T>* dst = (f == 0 ? d.SM : (f == 1 ? d.SW : (f == 2 ? d.SGx : d.SVg))) + (int64_t)kz * N2;
  constexpr int LS = skew_stride<LG>();
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);  // Bx lines of N along i1, skewed
  cplx<T>* tw = buf + Bx * LS;
  load_twiddles<T, LG>(tw, d);
  {  // columns of the plane into LDS lines, CopyBatch loads per thread in flight together
    constexpr int CB = CopyBatch<T>::n;
    const int n = Bx * N;
    for (int e0 = threadIdx.x; e0 < n; e0 += CB * kThreads) {
      T vx[CB], vy[CB];
#pragma unroll
      for (int k = 0; k < CB; ++k) {
        const int e = e0 + k * kThreads;
        if (e < n) {
          const int c = e & (Bx - 1), ix = e >> lbx;
          const cplx<T> v = src[(int64_t)ix * N + y0 + c];
          vx[k] = v.x;
          vy[k] = v.y;
        }
      }
#pragma unroll
      for (int k = 0; k < CB; ++k) {
        const int e = e0 + k * kThreads;
        if (e < n) buf[(e & (Bx - 1)) * LS + skp<LG, true>(e >> lbx)] = cplx<T>{vx[k], vy[k]};
      }
    }
  }
  __syncthreads();
  const int qz = lap_freq(kz, N);
  const T k0 = d.two_pi_over_L;
  const T D = (T)(f == 0 ? d.D_m : d.D_w);
  const T decay = (T)(f == 0 ? d.beta : 1.0);
  const T dt = (T)d.dt, inv_n3 = d.inv_n3, inv_n2 = d.inv_n2;
  const bool use_lp = d.use_lowpass, implicit = d.mult_kind == 0;
  const T* lpt = d.mtab + 2 * N;
  const T* tab = d.mtab + (f < 2 ? f : 0) * N;
  const T e_dec = implicit ? (T)0 : (T)exp(-dt * decay);
  // multiplier at position p (frequency along x) of the line c (y = y0 + c, plane kz)
  const auto mul = [=](int c, int p, cplx<T> val) {
    const int kx = ufpos<LG>(p);
    const int ky = ufpos<LG>(y0 + c);
    if (f < 2) {
      const T lp = use_lp ? lpt[kx] * lpt[ky] * lpt[kz] : (T)1;
      T mult;
      if (implicit) {
        const int qx = lap_freq(kx, N), qy = lap_freq(ky, N);
        const T k2 = k0 * k0 * (T)(qx * qx + qy * qy + qz * qz);
        mult = solve_multiplier(dt * (decay + D * k2), lp);
      } else {
        mult = table_multiplier(e_dec * tab[kx] * tab[ky] * tab[kz], lp);
      }
      return cscale(val, mult * inv_n3);
    } else if (f == 2) {
      // d1 v: with the filter V went through all three transforms, without it through the
      // z transform only (this x round trip adds the second N)
      T kk = k0 * (T)deriv_freq(kx, N) * (use_lp ? inv_n3 : inv_n2);
      if (use_lp) kk *= lpt[kx] * lpt[ky] * lpt[kz];
      return cplx<T>{-kk * val.y, kk * val.x};
    }
    // low-pass filtered V for the y and z derivatives; 1/N undoes this x round trip
    return cscale(val, lpt[kx] * lpt[ky] * lpt[kz] / (T)N);
  };
  line_round_trip<T, LG, false, kThreads, true>(buf, Bx, LS, 1, tw, mul);
  for (int e = threadIdx.x; e < Bx * N; e += kThreads) {
    const int c = e & (Bx - 1), ix = e >> lbx;
    dst[(int64_t)ix * N + y0 + c] = buf[c * LS + skp<LG, true>(ix)];
  }
}

// ---- two-dimensional column pass ---------------------------------------------------------
// In 2D the spectra are S[k2][i1] (k2 in [0, N/2]): after the row pass every k2 line along
// i1 is contiguous.  Per line: forward transform, the multipliers of eq. k_q_tilde_update
// with |k|^2 = (2 pi/L)^2 (q1^2 + q2^2) (m, w), the d1 multiplier (V -> SGx), or with the
// low-pass filter the filtered V (1/N undoes this round trip) into SVg; inverse transform.
// The d2 derivative is formed by the inverse row pass from SVg, as d3 is in 3D.
template <typename T, int LG>
__device__ __forceinline__ void col2d_body(SimC<T>& d, int lb, unsigned char* smem) {
  constexpr int N = 1 << LG;
  constexpr int H = (N >> 1) + 1;
  const int Bl = d.cols_per_blk;
  const int nbf = (H + Bl - 1) / Bl;
  const int f = lb / nbf;
  const int kl0 = (lb - f * nbf) * Bl;
  const int nl = H - kl0 < Bl ? H - kl0 : Bl;
  const cplx<T>* src = (f == 0 ? d.SM : (f == 1 ? d.SW : d.SV)) + (int64_t)kl0 * N;
  cplx<T>* dst = (f == 0 ? d.SM : (f == 1 ? d.SW : (f == 2 ? d.SGx : d.SVg))) + (int64_t)kl0 * N;
  constexpr int LS = skew_stride<LG>();
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);  // nl lines, skewed
  cplx<T>* tw = buf + Bl * LS;
  rows_in<T, LG, kThreads, true>(buf, LS, src, nl * N, tw, d.tw);
  __syncthreads();
  const T k0 = d.two_pi_over_L;
  const T D = (T)(f == 0 ? d.D_m : d.D_w);
  const T decay = (T)(f == 0 ? d.beta : 1.0);
  const T dt = (T)d.dt, inv_nd = d.inv_nd;
  const bool use_lp = d.use_lowpass, implicit = d.mult_kind == 0;
  const T* lpt = d.mtab + 2 * N;
  const T* tab = d.mtab + (f < 2 ? f : 0) * N;
  const T e_dec = implicit ? (T)0 : (T)exp(-dt * decay);
  // multiplier at position p (frequency along i1) of the line k2 = kl0 + line
  const auto mul = [=](int line, int p, cplx<T> val) {
    const int k1 = ufpos<LG>(p), k2 = kl0 + line;
    const T lp = use_lp ? lpt[k1] * lpt[k2] : (T)1;
    if (f < 2) {
      T mult;
      if (implicit) {
        const int q1 = lap_freq(k1, N), q2 = lap_freq(k2, N);
        mult = solve_multiplier(dt * (decay + D * k0 * k0 * (T)(q1 * q1 + q2 * q2)), lp);
      } else {
        mult = table_multiplier(e_dec * tab[k1] * tab[k2], lp);
      }
      return cscale(val, mult * inv_nd);
    } else if (f == 2) {
      const T kk = k0 * (T)deriv_freq(k1, N) * inv_nd * lp;
      return cplx<T>{-kk * val.y, kk * val.x};
    }
    return cscale(val, lp / (T)N);
  };
  line_round_trip<T, LG, false, kThreads, true>(buf, nl, LS, 1, tw, mul);
  for (int e = threadIdx.x; e < nl * N; e += kThreads)
    dst[e] = buf[(e >> LG) * LS + skp<LG, true>(e & (N - 1))];
}

template <typename T, int LG>
__global__ void __launch_bounds__(kThreads) k_xpass(Batch<T> bt, int /*mode*/) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim<kFieldRun>(bt, K_XPASS, lb);
  SimC<T>& d = sim_view(bt, s);
  if (d.dim == 2)
    col2d_body<T, LG>(d, lb, smem_raw);
  else
    xpass_body<T, LG>(d, lb, smem_raw);
}

// ---- plane pass: y, x, multipliers, x^-1, y^-1 on one k3 plane in LDS --------------------
// Replaces yfwd + xpass + yinv when a k3 plane of a half spectrum (N^2 complex values,
// contiguous in the S[k3][i1][i2] layout) fits in LDS.  Three jobs per plane: M, W (2D
// transforms and the diffusion multipliers), and one that forms both derivative spectra of V
// with 1D transforms only (x for d1 v, then y for d2 v: a derivative needs only its own
// axis), so that one block per job and plane fits the chip in a single round.  V itself is
// not written: it stays transformed along z only, and zinv forms the z derivative from it
// (scale 1/N).  With the low-pass filter (which needs both axes) the jobs are M, W, d1 V,
// d2 V with full 2D transforms, and a fifth writes the filtered V plane (x, y round trip
// undone) into SVg, from which zinv then forms the z derivative.
template <typename T, int LG>
__device__ __forceinline__ void plane_body(SimC<T>& d, int lb, unsigned char* smem) {
  constexpr int N = 1 << LG;
  constexpr int NN = N * N;
  constexpr int NT = kPlaneThreads;
  const int nj = d.use_lowpass ? 5 : 3;
  const int kz = lb / nj, job = lb - kz * nj;
  const int64_t off = (int64_t)kz * NN;
  if (!d.use_lowpass && job == 2) {
    // d1 v and d2 v need only the transform along their own axis: x round trip for SGx,
    // then (from a fresh copy of the plane) y round trip for SGy; 1/N^2 undoes the z and
    // own-axis round trips
    constexpr int LSv = plane_stride<LG>();
    cplx<T>* Q = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* twv = Q + N * LSv;
    const T c = d.two_pi_over_L * d.inv_n2;
    for (int pass = 0; pass < 2; ++pass) {
      const cplx<T>* twg = pass == 0 ? (const cplx<T>*)d.tw : nullptr;  // loaded once
      rows_in<T, LG, NT>(Q, LSv, d.SV + off, NN, twv, twg);
      __syncthreads();
      // i (2 pi / L) q v along the pass's axis (position p on a line of that axis)
      const auto deriv = [c](int, int p, cplx<T> v) {
        const T kk = c * (T)deriv_freq(ufpos<LG>(p), N);
        return cplx<T>{-kk * v.y, kk * v.x};
      };
      if (pass == 0)
        line_round_trip<T, LG, true, NT>(Q, N, 1, LSv, twv, deriv);  // along i1
      else
        line_round_trip<T, LG, true, NT>(Q, N, LSv, 1, twv, deriv);  // along i2
      cplx<T>* dst = (pass == 0 ? d.SGx : d.SGy) + off;
      for (int e = threadIdx.x; e < NN; e += NT) dst[e] = Q[(e >> LG) * LSv + (e & (N - 1))];
      __syncthreads();
    }
    return;
  }
  const cplx<T>* src = (job == 0 ? d.SM : (job == 1 ? d.SW : d.SV)) + off;
  cplx<T>* dst =
      (job == 0 ? d.SM : (job == 1 ? d.SW : (job == 2 ? d.SGx : (job == 3 ? d.SGy : d.SVg)))) +
      off;
  constexpr int LS = plane_stride<LG>();
  cplx<T>* P = reinterpret_cast<cplx<T>*>(smem);  // P[i1 * LS + i2]
  cplx<T>* tw = P + N * LS;
  rows_in<T, LG, NT>(P, LS, src, NN, tw, d.tw);
  __syncthreads();
  line_fwd<T, LG, true, NT>(P, N, LS, 1, tw);  // along i2 (rows)
  const int qz = lap_freq(kz, N);
  const T k0 = d.two_pi_over_L;
  const T D = (T)(job == 0 ? d.D_m : d.D_w);
  const T decay = (T)(job == 0 ? d.beta : 1.0);
  const T dt = (T)d.dt, inv_n3 = d.inv_n3, inv_n2 = d.inv_n2;
  const bool use_lp = d.use_lowpass, implicit = d.mult_kind == 0;
  const T* lpt = d.mtab + 2 * N;
  const T* tab = d.mtab + (job < 2 ? job : 0) * N;
  const T lpz = use_lp ? lpt[kz] : (T)1;
  const T sep_z = implicit ? (T)0 : (T)exp(-dt * decay) * tab[kz];
  // multiplier at column position p (frequency along i1) of the line i2 (frequency along
  // i2 from the row transforms)
  const auto mul = [=](int i2, int p, cplx<T> val) {
    const int kx = ufpos<LG>(p), ky = ufpos<LG>(i2);
    const T lp = use_lp ? lpt[kx] * lpt[ky] * lpz : (T)1;
    if (job < 2) {
      T mult;
      if (implicit) {
        const int qx = lap_freq(kx, N), qy = lap_freq(ky, N);
        const T k2 = k0 * k0 * (T)(qx * qx + qy * qy + qz * qz);
        mult = solve_multiplier(dt * (decay + D * k2), lp);
      } else {
        mult = table_multiplier(sep_z * tab[kx] * tab[ky], lp);
      }
      return cscale(val, mult * inv_n3);
    } else if (job < 4) {
      const T kk = k0 * (T)deriv_freq(job == 2 ? kx : ky, N) * inv_n3 * lp;
      return cplx<T>{-kk * val.y, kk * val.x};
    }
    // low-pass filtered V for the z derivative; 1/N^2 undoes this x, y round trip
    return cscale(val, lp * inv_n2);
  };
  line_round_trip<T, LG, true, NT>(P, N, 1, LS, tw, mul);  // along i1 (columns)
  line_inv<T, LG, true, NT>(P, N, LS, 1, tw);
  for (int e = threadIdx.x; e < NN; e += NT) dst[e] = P[(e >> LG) * LS + (e & (N - 1))];
}

template <typename T, int LG>
__global__ void __launch_bounds__(kPlaneThreads) k_plane(Batch<T> bt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim(bt, K_PLANE, lb);
  plane_body<T, LG>(sim_view(bt, s), lb, smem_raw);
}

// ---- zinv ---------------------------------------------------------------------------------
// Elements per thread of a z inverse block: ZB loads per batch, ZR batches, ZR ZB = 8 in
// both precisions, so a block holds up to zinv_max_elems() = 2048 nodes (float32 blocks of
// up to 2048 nodes; float64 blocks of 1024, and of two 1024-node rows in the 2D form); the
// host checks rows_zinv N against it.
template <typename T> struct ZBatches { static constexpr int n = sizeof(T) == 4 ? 1 : 2; };
static_assert(ZBatch<float>::n * ZBatches<float>::n * kThreads == zinv_max_elems() &&
                  ZBatch<double>::n * ZBatches<double>::n * kThreads == zinv_max_elems(),
              "z inverse elements per block");

// Two half spectra A, B (k3 in [0, N/2]) of real rows a, b into the full spectrum of the
// complex row a + i b on line rr: A + i B at position fpos(k3) and, for 0 < k3 < N/2,
// conj(A) + i conj(B) at the mirrored position fpos(N - k3).
template <typename T, int LG>
__device__ __forceinline__ void put_pair(cplx<T>* L, int rr, int pk, int pc, bool mirror,
                                         cplx<T> A, cplx<T> Bv) {
  constexpr int LS = zy_stride<LG>();
  L[rr * LS + pk] = cplx<T>{A.x - Bv.y, A.y + Bv.x};
  if (mirror) L[rr * LS + pc] = cplx<T>{A.x + Bv.y, Bv.x - A.y};
}

template <typename T, int LG>
__device__ __forceinline__ void zinv_body(SimC<T>& d, int lb, unsigned char* smem, int mode) {
  constexpr int N = 1 << LG;
  const int B = d.rows_zinv;
  const int64_t N2 = d.nrows;  // rows per k3 plane of the spectra (N^2; N in 2D)
  const int64_t r0 = (int64_t)lb * B;
  const int Bh = B >> 1;
  const int lgBh = __builtin_ctz((unsigned)Bh);  // B is a power of two: no vector division
  constexpr int LS = zy_stride<LG>();
  // Two phases over one LDS area of 1.5 B lines, so that more blocks share a CU: first the
  // m and w lines (B lines of m + i w), then the gradient lines (B lines of d1 v + i d2 v and
  // B/2 lines of d3 v, rows 2q + i 2q+1).
  cplx<T>* MW = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* GG = MW;
  cplx<T>* GZ = GG + B * LS;
  cplx<T>* tw = GZ + Bh * LS;
  const bool freeze_m = d.flags & SIPF_FLAG_FREEZE_M;
  const bool freeze_w = d.flags & SIPF_FLAG_FREEZE_W;
  const bool grad_only = mode == kGradOnly;
  const uint32_t par = (uint32_t)(*d.step) & 1u;
  T* const ub = d.ubar[par];  // holds w* in change form (see zfwd)
  // the gather array of step n + 1, or with grad_only that of step n
  vec4<T>* const gout = d.g4[grad_only ? par : par ^ 1u];
  constexpr int ZB = ZBatch<T>::n, ZR = ZBatches<T>::n;
  const int nel = B * N;
  const int64_t g0 = r0 * N;
  constexpr int H = (N >> 1) + 1;
  const int n1 = H * Bh;  // (k3, row pair) items
  // spectra of IB items per thread loaded together
  constexpr int IB = sizeof(T) == 4 ? 2 : 1;
  // m* and w* of the first ZB elements per thread (change form only; w^n instead of w* when
  // w is frozen or only the gradient is formed, in both forms; m* not at all when m is
  // frozen) are loaded first: they are needed only after the transforms, so their loads
  // overlap everything before.  wk keeps w of every element of the thread for the gather
  // array.
  const bool need_wold = grad_only || freeze_w, write_m = !grad_only && !freeze_m;
  const bool need_m = change_form<T>() && write_m, need_wst = change_form<T>() && !need_wold;
  T wold[ZB], mold[ZB], wst[ZB], wk[ZR * ZB];
#pragma unroll
  for (int k = 0; k < ZB; ++k) {
    const int e = threadIdx.x + k * kThreads;
    if (e < nel) {
      if (need_wold) wold[k] = d.w[g0 + e];
      if (need_m) mold[k] = d.m[g0 + e];
      if (need_wst) wst[k] = ub[g0 + e];
    }
  }
  TwiddleRegs<T, LG, kThreads> tr;
  tr.load(d.tw);
  // ---- first phase: m and w ----
  if (!grad_only) {
    for (int e0 = threadIdx.x; e0 < n1; e0 += IB * kThreads) {
      cplx<T> sv[IB][2][2];  // (M, W) of rows 2q and 2q + 1
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) {
        const int e = e0 + ib * kThreads;
        if (e < n1) {
          const int kz = e >> lgBh, q = e & (Bh - 1);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int64_t o = (int64_t)kz * N2 + r0 + 2 * q + h;
            sv[ib][h][0] = d.SM[o];
            sv[ib][h][1] = d.SW[o];
          }
        }
      }
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) {
        const int e = e0 + ib * kThreads;
        if (e < n1) {
          const int kz = e >> lgBh, q = e & (Bh - 1);
          const bool mirror = kz > 0 && kz < (N >> 1);
          const int pk = fpos<LG>(kz), pc = fpos<LG>((N - kz) & (N - 1));
#pragma unroll
          for (int h = 0; h < 2; ++h)
            put_pair<T, LG>(MW, 2 * q + h, pk, pc, mirror, sv[ib][h][0], sv[ib][h][1]);
        }
      }
    }
  }
  tr.store(tw);
  __syncthreads();
  if (!grad_only) line_inv<T, LG, true>(MW, B, LS, 1, tw);
#pragma unroll
  for (int r = 0; r < ZR; ++r) {
    const int e0 = threadIdx.x + r * ZB * kThreads;
    if (r > 0) {  // elements beyond the first ZB per thread
#pragma unroll
      for (int k = 0; k < ZB; ++k) {
        const int e = e0 + k * kThreads;
        if (e < nel) {
          if (need_wold) wold[k] = d.w[g0 + e];
          if (need_m) mold[k] = d.m[g0 + e];
          if (need_wst) wst[k] = ub[g0 + e];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < ZB; ++k) {
      const int e = e0 + k * kThreads;
      if (need_wold) wk[r * ZB + k] = wold[k];
      if (grad_only || e >= nel) continue;
      const int rr = e >> LG, iz = e & (N - 1);
      const int64_t g = g0 + e;
      const cplx<T> mw = MW[rr * LS + iz];
      // m^{n+1} = m* + change, or the transform itself in plain form (frozen m: unchanged)
      if (write_m) d.m[g] = change_form<T>() ? mold[k] + mw.x : mw.x;
      if (!freeze_w) {
        const T wn = change_form<T>() ? wst[k] + mw.y : mw.y;
        d.w[g] = wn;
        wk[r * ZB + k] = wn;
      }
      if (change_form<T>()) ub[g] = (T)0;  // cleared for the next step's deposit
    }
  }
  // ---- second phase: the gradient of v ----
  const T cz = d.gz_scale;  // 2 pi / L over the transforms SV went through (N or N^2)
  if (!grad_only) __syncthreads();  // the m and w lines are read
  for (int e0 = threadIdx.x; e0 < n1; e0 += IB * kThreads) {
    cplx<T> sv[IB][2][3];  // (Gx, Gy, V) of rows 2q and 2q + 1
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) {
      const int e = e0 + ib * kThreads;
      if (e < n1) {
        const int kz = e >> lgBh, q = e & (Bh - 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t o = (int64_t)kz * N2 + r0 + 2 * q + h;
          sv[ib][h][0] = d.SGx[o];
          sv[ib][h][1] = d.SGy[o];
          sv[ib][h][2] = d.SVg[o];
        }
      }
    }
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) {
      const int e = e0 + ib * kThreads;
      if (e < n1) {
        const int kz = e >> lgBh, q = e & (Bh - 1);
        const bool mirror = kz > 0 && kz < (N >> 1);
        const int pk = fpos<LG>(kz), pc = fpos<LG>((N - kz) & (N - 1));
        const T kk = cz * (T)deriv_freq(kz, N);
        cplx<T> gz[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          put_pair<T, LG>(GG, 2 * q + h, pk, pc, mirror, sv[ib][h][0], sv[ib][h][1]);
          gz[h] = cplx<T>{-kk * sv[ib][h][2].y, kk * sv[ib][h][2].x};
        }
        put_pair<T, LG>(GZ, q, pk, pc, mirror, gz[0], gz[1]);
      }
    }
  }
  __syncthreads();
  line_inv<T, LG, true>(GG, B + Bh, LS, 1, tw);
#pragma unroll
  for (int r = 0; r < ZR; ++r) {
#pragma unroll
    for (int k = 0; k < ZB; ++k) {
      const int e = threadIdx.x + (r * ZB + k) * kThreads;
      if (e >= nel) continue;
      const int rr = e >> LG, iz = e & (N - 1);
      const cplx<T> gg = GG[rr * LS + iz];
      const cplx<T> gzp = GZ[(rr >> 1) * LS + iz];
      const T gzv = (rr & 1) ? gzp.y : gzp.x;
      // (grad v^{n+1}, w^{n+1}), or with grad_only (grad v^n, w^n)
      gout[g0 + e] = vec4<T>{gg.x, gg.y, gzv, wk[r * ZB + k]};
    }
  }
}

template <typename T, int LG>
__global__ void __launch_bounds__(kThreads) k_zinv(Batch<T> bt, int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int lb;
  const int s = find_sim<kFieldRun>(bt, K_ZINV, lb);
  zinv_body<T, LG>(sim_view(bt, s), lb, smem_raw, mode);
}

// ---- LDS sizes and launchers ----------------------------------------------------------------
// LDS bytes of a kernel kind at log2 N = lg (lines of the padded row stride + twiddles)
template <typename T>
size_t fft_lds_bytes(int kind, int lg) {
  const int E = elems_per_block<T>();
  const int N = 1 << lg;
  const size_t LK = (size_t)skew_stride_rt(lg);   // x pass, 2D column pass
  const size_t LZ = (size_t)zy_stride_rt(lg);     // z and y passes
  const size_t c = sizeof(cplx<T>);
  const size_t tw = (size_t)tw_len_rt(lg) * c;
  const size_t B = (size_t)std::min(N * N, std::max(zfwd_min_rows<T>(lg), E / N));  // z forward
  const size_t Bz = (size_t)std::min(N * N, std::max(2, zinv_elems<T>(N) / N));  // z inverse
  const size_t Bl = (size_t)(E / N);                // lines per block (y passes)
  const size_t Bx = (size_t)std::min(N, xpass_elems(lg) / N);  // columns per block (x pass)
  switch (kind) {
    case K_ZFWD: return (B + B / 2) * LZ * c + tw;
    case K_YFWD: return Bl * LZ * c + tw;
    case K_YINV: return Bl * LZ * c + tw;
    case K_XPASS: return Bx * LK * c + tw;
    case K_ZINV: return (Bz + Bz / 2) * LZ * c + tw;
    case K_PLANE: return (size_t)N * (N + 2) * c + tw;  // plane_stride
    default: return 0;
  }
}
template size_t fft_lds_bytes<double>(int, int);
template size_t fft_lds_bytes<float>(int, int);

// Raise the dynamic LDS limit of the passes that can need more than the default 64 KiB at
// N = 1024 (float64 rows of 1024 nodes, two per block; column blocks of several 1024-point
// lines).  Call once, outside capture.
template <typename T>
void configure_fft(int lg) {
  if (lg != 10) return;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_zfwd<T, 10>),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fft_lds_bytes<T>(K_ZFWD, 10));
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_zinv<T, 10>),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fft_lds_bytes<T>(K_ZINV, 10));
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_xpass<T, 10>),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fft_lds_bytes<T>(K_XPASS, 10));
}
template void configure_fft<double>(int);
template void configure_fft<float>(int);

// Host-side dispatch: one kernel instantiation per log2 N, so each carries only the
// registers its own transform length needs.
#define SIPF_LG_CASE(KER, KIND, L)                                                          \
  case L:                                                                                   \
    hipLaunchKernelGGL((k_##KER<T, L>), dim3(nblk), dim3(kThreads),                        \
                       fft_lds_bytes<T>(KIND, L), st, b, mode);                             \
    break;
#define SIPF_LAUNCH(KER, KIND)                                                     \
  template <typename T>                                                            \
  void launch_##KER(const Batch<T>& b, int nblk, int lg, hipStream_t st, int mode) { \
    if (nblk <= 0) return;                                                         \
    switch (lg) {                                                                  \
      SIPF_LG_CASE(KER, KIND, 2)                                                   \
      SIPF_LG_CASE(KER, KIND, 3)                                                   \
      SIPF_LG_CASE(KER, KIND, 4)                                                   \
      SIPF_LG_CASE(KER, KIND, 5)                                                   \
      SIPF_LG_CASE(KER, KIND, 6)                                                   \
      SIPF_LG_CASE(KER, KIND, 7)                                                   \
      SIPF_LG_CASE(KER, KIND, 8)                                                   \
      SIPF_LG_CASE(KER, KIND, 9)                                                   \
      SIPF_LG_CASE(KER, KIND, 10)                                                  \
      default: break;                                                              \
    }                                                                              \
  }                                                                                \
  template void launch_##KER<double>(const Batch<double>&, int, int, hipStream_t, int); \
  template void launch_##KER<float>(const Batch<float>&, int, int, hipStream_t, int);

SIPF_LAUNCH(zfwd, K_ZFWD)
SIPF_LAUNCH(yfwd, K_YFWD)
SIPF_LAUNCH(xpass, K_XPASS)
SIPF_LAUNCH(yinv, K_YINV)
SIPF_LAUNCH(zinv, K_ZINV)

template <typename T>
size_t plane_lds_bytes(int lg) {
  return fft_lds_bytes<T>(K_PLANE, lg);
}

template <typename T>
bool plane_fits(int lg) {
  return plane_lds_bytes<T>(lg) <= kPlaneLdsMax;
}
template bool plane_fits<double>(int);
template bool plane_fits<float>(int);

#define SIPF_PLANE_CASE(L)                                                                \
  case L:                                                                                 \
    if (configure) {                                                                      \
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_plane<T, L>),            \
                                hipFuncAttributeMaxDynamicSharedMemorySize,               \
                                (int)plane_lds_bytes<T>(L));                              \
    } else {                                                                              \
      hipLaunchKernelGGL((k_plane<T, L>), dim3(nblk), dim3(kPlaneThreads),                \
                         plane_lds_bytes<T>(L), st, b);                                   \
    }                                                                                     \
    break;

// configure != 0: only raise the kernel's dynamic LDS limit (call once, outside capture)
template <typename T>
void launch_plane(const Batch<T>& b, int nblk, int lg, hipStream_t st, int configure) {
  if (!configure && nblk <= 0) return;
  if (!plane_fits<T>(lg)) return;
  switch (lg) {
    SIPF_PLANE_CASE(2)
    SIPF_PLANE_CASE(3)
    SIPF_PLANE_CASE(4)
    SIPF_PLANE_CASE(5)
    SIPF_PLANE_CASE(6)
    SIPF_PLANE_CASE(7)
    default: break;
  }
}
template void launch_plane<double>(const Batch<double>&, int, int, hipStream_t, int);
template void launch_plane<float>(const Batch<float>&, int, int, hipStream_t, int);

}  // namespace sipf
