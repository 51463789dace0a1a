// C ABI of libsipf (declared in include/sipf.h): validation, the workspace layout, upload of
// the initial state (Alg. sipf-pic initialisation), the per-step launch sequence captured
// once as a HIP graph, the batched launch set of the served form, and state export.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "sipf_internal.h"

using namespace sipf;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(SIPF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
  size_t total = 0;
  size_t desc, blk, step, diag;
  size_t x[2], y[2], z[2], a[2], id[2];
  size_t tcount, toff, coff, cinfo, key;
  size_t ubar, v, m, w, g4;
  size_t SM, SW, SV, SGx, SGy, SVf;
  size_t tw, mtab;
  size_t rs;  // resampling scratch (uint64 words)
};

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

// spatial dimension (0 in the parameters means 3)
int dim_of(const sipf_params& p) { return p.dim == 2 ? 2 : 3; }
size_t grid_nodes(const sipf_params& p) {
  size_t g = 1;
  for (int j = 0; j < dim_of(p); ++j) g *= (size_t)p.N;
  return g;
}

int validate_params(const sipf_params* p) {
  if (!p) return fail(SIPF_EINVAL, "params is NULL");
  if (p->dim != 0 && p->dim != 2 && p->dim != 3)
    return fail(SIPF_EINVAL, "dim must be 0 or 3 (three-dimensional) or 2");
  if (p->dim == 2) {
    if (!(p->N >= 4 && p->N <= 1024 && is_pow2(p->N)))
      return fail(SIPF_EINVAL, "2D: N must be a power of two in [4, 1024]");
    if (p->deposit_order != 2)
      return fail(SIPF_EINVAL, "2D: only the bilinear deposit (deposit_order 2)");
  } else if (!(p->N >= 4 && p->N <= 512 && is_pow2(p->N))) {
    return fail(SIPF_EINVAL, "N must be a power of two in [4, 512]");
  }
  if (p->P < 0 || p->P >= (int64_t(1) << 32))
    return fail(SIPF_EINVAL, "P must satisfy 0 <= P < 2^32");
  if (!(isfinite(p->L) && p->L > 0)) return fail(SIPF_EINVAL, "L must be finite and > 0");
  if (!(p->dt > 0 && p->dt <= 0.5)) return fail(SIPF_EINVAL, "dt must be in (0, 0.5]");
  const double c[] = {p->D_u, p->chi, p->D_m, p->D_w, p->alpha, p->beta, p->gamma};
  for (double v : c)
    if (!(isfinite(v) && v >= 0)) return fail(SIPF_EINVAL, "model constants must be finite, >= 0");
  if (p->precision != SIPF_FP64 && p->precision != SIPF_FP32)
    return fail(SIPF_EINVAL, "precision must be SIPF_FP64 or SIPF_FP32");
  if (p->deposit_order != 2 && p->deposit_order != 4)
    return fail(SIPF_EINVAL, "deposit_order must be 2 (trilinear) or 4 (fourth order)");
  if ((p->flags & SIPF_FLAG_EXP_DIFFUSION) && (p->flags & SIPF_FLAG_ALIASED_DIFFUSION))
    return fail(SIPF_EINVAL, "EXP_DIFFUSION and ALIASED_DIFFUSION are exclusive");
  if (p->flags & ~0x1FFu) return fail(SIPF_EINVAL, "unknown flag bits");
  if (!(isfinite(p->H0) && p->H0 >= 0.0))
    return fail(SIPF_EINVAL, "H0 must be finite and >= 0 (0: no low-pass filter)");
  if (p->resort_every < 0) return fail(SIPF_EINVAL, "resort_every must be >= 0");
  if (p->flags & SIPF_FLAG_ALIASED_DIFFUSION) {
    // The aliased multiplier is the DFT of the heat kernel sampled at the nodes (Lemma
    // kernel); it approximates exp(-tau D k^2) only if the grid resolves that kernel.  Its
    // largest deviation from the plain exponential is at the Nyquist corner, about
    // 2 exp(-tau D (2 pi / L)^2 (N/2)^2) per axis.
    const double Dmin = std::min(p->D_m, p->D_w);
    const double k = 2.0 * M_PI / p->L * (p->N / 2);
    if (!(p->dt * Dmin * k * k > 10.0))
      return fail(SIPF_EINVAL,
                  "ALIASED_DIFFUSION needs a grid that resolves the heat kernel: "
                  "dt * min(D_m, D_w) * (pi N / L)^2 must exceed 10");
  }
  return SIPF_OK;
}

// steps between binnings when the caller leaves it to the library (kBinDrift3, kBinDrift2)
int default_resort(const sipf_params& p) {
  const double h = p.L / p.N;
  const double s = (p.flags & SIPF_FLAG_NO_NOISE) ? 0.0 : std::sqrt(2.0 * p.D_u * p.dt) / h;
  const double reach = dim_of(p) == 2 ? kBinDrift2 : kBinDrift3;
  if (!(s > 0.0)) return kResortMax;
  const double k = std::floor((reach / s) * (reach / s));
  return k < 1.0 ? 1 : (k > kResortMax ? kResortMax : (int)k);
}

Layout make_layout(const sipf_params& p) {
  const size_t s = p.precision == SIPF_FP32 ? 4 : 8;
  const int dim = dim_of(p);
  const size_t N = (size_t)p.N, G = grid_nodes(p), P = (size_t)p.P, H = N / 2 + 1;
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  L.desc = take(std::max(sizeof(SimDev<double>), sizeof(SimDev<float>)));
  L.blk = take(sizeof(int) * K_COUNT * 2);
  L.step = take(sizeof(uint64_t));
  L.diag = take(sizeof(unsigned long long) * kDiagWords);
  for (int k = 0; k < 2; ++k) {
    L.x[k] = take(P * s);
    L.y[k] = take(P * s);
    L.z[k] = take(dim == 3 ? P * s : 0);
    L.a[k] = take(P * 8);
    L.id[k] = take(P * 4);
  }
  const size_t tside = dim == 3 ? kTile : kTile2;
  const size_t nt1 = N / tside > 0 ? N / tside : 1;
  const size_t ntiles = dim == 3 ? nt1 * nt1 * nt1 : nt1 * nt1;
  L.tcount = take(ntiles * 4);
  L.toff = take((ntiles + 1) * 4);
  L.coff = take((ntiles + 1) * 4);
  L.cinfo = take(((P + kChunk - 1) / kChunk + ntiles) * 16);
  L.key = take(P * 8);
  L.ubar = take(2 * G * s);    // two buffers, by step parity
  L.v = take(G * s);
  L.m = take(G * s);
  L.w = take(G * s);
  L.g4 = take(2 * G * 4 * s);  // two buffers, by step parity
  const size_t spec = H * (G / N) * 2 * s;  // half spectrum: (N/2+1) N^(dim-1) complex
  L.SM = take(spec);
  L.SW = take(spec);
  L.SV = take(spec);
  L.SGx = take(spec);
  L.SGy = take(spec);
  L.SVf = take(p.H0 > 0 ? spec : 0);  // low-pass filtered V
  L.tw = take((N / 2) * 2 * s);
  L.mtab = take(3 * N * s);
  L.rs = take(resample_scratch_words((int64_t)P) * 8);
  L.total = o;
  return L;
}

// second stream and events of a step's two halves: fork (the field passes start), zfwd (the
// forward z pass is done) and join (the field passes are done)
struct StepFork {
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, zfwd = nullptr, join = nullptr;
};

hipError_t create_fork(StepFork& f) {
  hipError_t e = hipStreamCreateWithFlags(&f.aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&f.fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&f.zfwd, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&f.join, hipEventDisableTiming);
  return e;
}

void destroy_fork(StepFork& f) {
  if (f.join) (void)hipEventDestroy(f.join);
  if (f.zfwd) (void)hipEventDestroy(f.zfwd);
  if (f.fork) (void)hipEventDestroy(f.fork);
  if (f.aux) (void)hipStreamDestroy(f.aux);
  f = StepFork{};
}

}  // namespace

struct sipf_sim {
  sipf_params prm;
  unsigned char* ws = nullptr;
  size_t bytes = 0;
  Layout lay;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  StepFork fork;                      // second stream of the captured binning step
  hipStream_t last_stream = nullptr;  // stream of the last batched step, if any
  hipEvent_t ev = nullptr;            // orders this simulation's streams for batches
  int device = 0;
  int counts[K_COUNT];
  hipGraph_t graph = nullptr;       // one step
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph_bin = nullptr;   // binning + one step
  hipGraphExec_t exec_bin = nullptr;
  int resort_every = 1;             // steps between binnings (set at initialisation)
  int since_bin = 0;                // steps since the last binning
  unsigned char host_desc[std::max(sizeof(SimDev<double>), sizeof(SimDev<float>))];
};

namespace {

template <typename T>
Batch<T> single_batch(const sipf_sim* s) {
  Batch<T> b;
  b.sims = reinterpret_cast<const SimDev<T>*>(s->ws + s->lay.desc);
  b.blk = reinterpret_cast<const int*>(s->ws + s->lay.blk);
  b.nsims = 1;
  return b;
}

// Simulations of one grid size, for the FFT launches (their kernels are compiled per N).
template <typename T>
struct FftGroup {
  Batch<T> b;
  int tot[K_COUNT];
  int lg;
};

// the field passes (mode 0: a step's; kGradOnly: the gather array of the current state);
// after_zfwd, if given, is recorded once the forward z pass is launched
template <typename T>
void enqueue_fft(const FftGroup<T>* groups, int ng, hipStream_t st, int mode,
                 hipEvent_t after_zfwd = nullptr) {
  for (int i = 0; i < ng; ++i)
    launch_zfwd<T>(groups[i].b, groups[i].tot[K_ZFWD], groups[i].lg, st, mode);
  if (after_zfwd) (void)hipEventRecord(after_zfwd, st);
  for (int i = 0; i < ng; ++i)
    launch_yfwd<T>(groups[i].b, groups[i].tot[K_YFWD], groups[i].lg, st, mode);
  for (int i = 0; i < ng; ++i)
    launch_xpass<T>(groups[i].b, groups[i].tot[K_XPASS], groups[i].lg, st, mode);
  for (int i = 0; i < ng; ++i)
    launch_plane<T>(groups[i].b, groups[i].tot[K_PLANE], groups[i].lg, st, 0);
  for (int i = 0; i < ng; ++i)
    launch_yinv<T>(groups[i].b, groups[i].tot[K_YINV], groups[i].lg, st, mode);
  for (int i = 0; i < ng; ++i)
    launch_zinv<T>(groups[i].b, groups[i].tot[K_ZINV], groups[i].lg, st, mode);
}

// One step; with bin != 0 the particles are first binned into set 1 and the particle pass
// reads set 1 (and writes set 0).  The field passes of step n and its particle pass share no
// buffer: the particle pass gathers from the array the previous step's field passes (or the
// initialisation) formed and deposits into the other ubar buffer, while the field passes read
// ubar^n and form the next gather array.  With a fork the two halves run side by side: the
// field passes on the second stream, the binning (when due) and the particle pass on the
// first; the finalize kernel (step index) waits for both.  The particle pass
// starts once the forward z pass is done: the particle blocks take every CU's LDS, and a z
// pass started beside them ran at a fraction of its speed (128^3 / 2^23 float32: 207.9 ->
// 202.9 us per step; starting it after the plane pass as well took 209.7).  Without a fork
// the passes run in sequence on st.
template <typename T>
void enqueue_step(const Batch<T>& b, const int* tot, int nsims, const FftGroup<T>* groups,
                  int ngroups, int bin, int order, int dim, hipStream_t st,
                  const StepFork* fk) {
  if (fk) {
    (void)hipEventRecord(fk->fork, st);
    (void)hipStreamWaitEvent(fk->aux, fk->fork, 0);
    enqueue_fft<T>(groups, ngroups, fk->aux, 0, fk->zfwd);
    (void)hipEventRecord(fk->join, fk->aux);
  } else {
    enqueue_fft<T>(groups, ngroups, st, 0);
  }
  if (bin) launch_binning<T>(b, tot, nsims, dim, st);
  if (fk) (void)hipStreamWaitEvent(st, fk->zfwd, 0);
  launch_particles<T>(b, tot[K_PART], bin ? 1 : 0, 0, order, dim, st);
  if (fk) (void)hipStreamWaitEvent(st, fk->join, 0);
  launch_finalize<T>(b, nsims, st);
}

template <typename T>
std::vector<FftGroup<T>> single_groups(const sipf_sim* s, const Batch<T>& b) {
  FftGroup<T> g;
  g.b = b;
  memcpy(g.tot, s->counts, sizeof(g.tot));
  g.lg = reinterpret_cast<const SimDev<T>*>(s->host_desc)->log2N;
  return {g};
}

// float64 multiplier tables of the separable diffusion forms and of the low-pass filter,
// indexed by the DFT position of one axis.
void axis_tables(const sipf_params& p, int field, std::vector<double>& tab) {
  const int N = p.N;
  tab.assign(N, 1.0);
  const double D = field == 0 ? p.D_m : p.D_w;
  const double c = p.dt * D * (2.0 * M_PI / p.L) * (2.0 * M_PI / p.L);
  for (int k = 0; k < N; ++k) {
    const double q = k < N / 2 ? k : k - N;
    if (p.flags & SIPF_FLAG_ALIASED_DIFFUSION) {
      // lattice sum over q + n N; terms decay like exp(-c (n N)^2)
      long double acc = 0.0L;
      for (int n = -64; n <= 64; ++n) {
        const long double qq = (long double)q + (long double)n * N;
        const long double t = expl(-(long double)c * qq * qq);
        acc += t;
        if (n > 0 && t < 1e-40L) break;
      }
      tab[k] = (double)acc;
    } else {
      tab[k] = exp(-c * q * q);
    }
  }
}

template <typename T>
int init_t(sipf_sim* sim, const double* X0, const double* a0, const double* v0,
           const double* m0, const double* w0) {
  const sipf_params& p = sim->prm;
  const Layout& L = sim->lay;
  const int N = p.N;
  const int64_t P = p.P;
  const int dim = dim_of(p);
  const size_t G = grid_nodes(p);
  unsigned char* ws = sim->ws;

  SimDev<T> d;
  memset(&d, 0, sizeof(d));
  d.N = N;
  d.dim = dim;
  d.G = (int64_t)G;
  d.nrows = (int64_t)(G / N);
  d.inv_nd = (T)(1.0 / (double)G);
  int lg = 0;
  while ((1 << lg) < N) ++lg;
  d.log2N = lg;
  d.P = P;
  const int E = elems_per_block<T>();
  d.rows_per_blk = (int)std::min<int64_t>(d.nrows, std::max(zfwd_min_rows<T>(lg), E / N));
  d.rows_zinv = (int)std::min<int64_t>(d.nrows, std::max(2, zinv_elems<T>(N) / N));
  if ((int64_t)d.rows_zinv * N > zinv_max_elems())  // the z inverse pass's registers
    return fail(SIPF_EINVAL, "grid too large for the z inverse pass's blocks");
  d.lines_per_blk = E / N;
  d.cols_per_blk = std::min(N, xpass_elems(lg) / N);
  d.flags = (int)p.flags;
  d.L = (T)p.L;
  d.inv_h = (T)(N / p.L);
  const double h = p.L / N;
  const double hd = dim == 3 ? h * h * h : h * h;  // cell volume h^dim
  d.inv_h3 = (T)(1.0 / hd);
  d.two_pi_over_L = (T)(2.0 * M_PI / p.L);
  d.inv_n3 = (T)(1.0 / ((double)N * N * N));
  d.inv_n2 = (T)(1.0 / ((double)N * N));
  d.use_plane = dim == 3 && plane_fits<T>(lg) ? 1 : 0;
  // the z (2D: x2) derivative is formed from V transformed along that axis only (plane and
  // 2D paths) or along y as well (three-pass path)
  // V has been transformed along y as well only on the three-pass path with the filter
  d.gz_scale = (T)(2.0 * M_PI / p.L /
                   (dim == 3 && !d.use_plane && p.H0 > 0 ? (double)N * N : (double)N));
  if (d.use_plane) launch_plane<T>(Batch<T>{}, 0, lg, nullptr, 1);  // raise its LDS limit
  configure_particles<T>(p.deposit_order, dim);
  configure_fft<T>(lg);
  d.dt = p.dt;
  d.D_u = p.D_u;
  d.chi = p.chi;
  d.D_m = p.D_m;
  d.D_w = p.D_w;
  d.alpha = p.alpha;
  d.beta = p.beta;
  d.gamma = p.gamma;
  d.noise_amp = (T)sqrt(2.0 * p.D_u * p.dt);
  d.drift = (T)(p.chi * p.dt);
  d.h3 = hd;
  d.seed_lo = (uint32_t)(p.seed & 0xFFFFFFFFu);
  d.seed_hi = (uint32_t)(p.seed >> 32);
  d.sim_lo = (uint32_t)(p.sim_id & 0xFFFFFFFFu);
  d.sim_hi = (uint32_t)(p.sim_id >> 32);
  d.mult_kind = (p.flags & (SIPF_FLAG_EXP_DIFFUSION | SIPF_FLAG_ALIASED_DIFFUSION)) ? 1 : 0;
  d.use_lowpass = p.H0 > 0 ? 1 : 0;
  const int tside = dim == 3 ? kTile : kTile2;
  d.ntile1 = N / tside > 0 ? N / tside : 1;
  d.ntiles = dim == 3 ? d.ntile1 * d.ntile1 * d.ntile1 : d.ntile1 * d.ntile1;
  d.use_region = N >= 2 * tside ? 1 : 0;
  d.deposit_order = p.deposit_order;
  for (int k = 0; k < 2; ++k) {
    d.xs[k] = reinterpret_cast<T*>(ws + L.x[k]);
    d.ys[k] = reinterpret_cast<T*>(ws + L.y[k]);
    d.zs[k] = dim == 3 ? reinterpret_cast<T*>(ws + L.z[k]) : nullptr;
    d.as[k] = reinterpret_cast<double*>(ws + L.a[k]);
    d.ids[k] = reinterpret_cast<uint32_t*>(ws + L.id[k]);
  }
  d.tcount = reinterpret_cast<uint32_t*>(ws + L.tcount);
  d.toff = reinterpret_cast<uint32_t*>(ws + L.toff);
  d.coff = reinterpret_cast<uint32_t*>(ws + L.coff);
  d.cinfo = reinterpret_cast<uint4*>(ws + L.cinfo);
  d.max_chunks = (int)((P + kChunk - 1) / kChunk + d.ntiles);
  d.key = reinterpret_cast<uint32_t*>(ws + L.key);
  for (int k = 0; k < 2; ++k) {
    d.ubar[k] = reinterpret_cast<T*>(ws + L.ubar) + k * G;
    d.g4[k] = reinterpret_cast<vec4<T>*>(ws + L.g4) + k * G;
  }
  d.v = reinterpret_cast<T*>(ws + L.v);
  d.m = reinterpret_cast<T*>(ws + L.m);
  d.w = reinterpret_cast<T*>(ws + L.w);
  d.SM = reinterpret_cast<cplx<T>*>(ws + L.SM);
  d.SW = reinterpret_cast<cplx<T>*>(ws + L.SW);
  d.SV = reinterpret_cast<cplx<T>*>(ws + L.SV);
  d.SGx = reinterpret_cast<cplx<T>*>(ws + L.SGx);
  d.SGy = reinterpret_cast<cplx<T>*>(ws + L.SGy);
  d.SVg = p.H0 > 0 ? reinterpret_cast<cplx<T>*>(ws + L.SVf) : d.SV;
  d.tw = reinterpret_cast<cplx<T>*>(ws + L.tw);
  d.mtab = reinterpret_cast<T*>(ws + L.mtab);
  d.step = reinterpret_cast<uint64_t*>(ws + L.step);
  d.diag = reinterpret_cast<unsigned long long*>(ws + L.diag);
  memcpy(sim->host_desc, &d, sizeof(d));

  block_counts<T>(d, sim->counts);
  int blk[K_COUNT * 2];
  for (int k = 0; k < K_COUNT; ++k) {
    blk[2 * k] = 0;
    blk[2 * k + 1] = sim->counts[k];
  }

  // host staging in the working precision
  std::vector<T> hx(P), hy(P), hz(dim == 3 ? P : 0);
  const T LT = (T)p.L;
  for (int64_t i = 0; i < P; ++i) {
    double c3[3] = {X0[i], X0[P + i], dim == 3 ? X0[2 * P + i] : 0.0};
    T out[3];
    for (int j = 0; j < dim; ++j) {
      double q = c3[j] - p.L * floor(c3[j] / p.L);
      if (q >= p.L || q < 0) q = 0.0;
      T t = (T)q;
      if (t >= LT) t = (T)0;
      out[j] = t;
    }
    hx[i] = out[0];
    hy[i] = out[1];
    if (dim == 3) hz[i] = out[2];
  }
  std::vector<uint32_t> hid(P);
  for (int64_t i = 0; i < P; ++i) hid[i] = (uint32_t)i;
  std::vector<T> hv(G), hm(G), hw(G);
  for (size_t i = 0; i < G; ++i) {
    hv[i] = (T)v0[i];
    hm[i] = (T)m0[i];
    hw[i] = (T)w0[i];
  }
  std::vector<cplx<T>> htw(N / 2);
  for (int k = 0; k < N / 2; ++k) {
    const long double ang = 2.0L * 3.14159265358979323846264338327950288L * k / N;
    htw[k].x = (T)cosl(ang);
    htw[k].y = (T)(-sinl(ang));
  }
  std::vector<T> hmt(3 * N, (T)1);
  if (d.mult_kind) {
    std::vector<double> t;
    for (int f = 0; f < 2; ++f) {
      axis_tables(p, f, t);
      for (int k = 0; k < N; ++k) hmt[f * N + k] = (T)t[k];
    }
  }
  if (p.H0 > 0) {  // low-pass factor per axis: exp(-2 pi^2 q^2 / H0^2)
    for (int k = 0; k < N; ++k) {
      const double q = k < N / 2 ? k : k - N;
      hmt[2 * N + k] = (T)exp(-2.0 * M_PI * M_PI * q * q / (p.H0 * p.H0));
    }
  }
  const uint64_t step0 = p.step0;

  hipStream_t st = sim->stream;
  HIPCHK(hipMemcpyAsync(ws + L.desc, &d, sizeof(d), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ws + L.blk, blk, sizeof(blk), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ws + L.step, &step0, sizeof(step0), hipMemcpyHostToDevice, st));
  if (P > 0) {
    HIPCHK(hipMemcpyAsync(d.xs[0], hx.data(), P * sizeof(T), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.ys[0], hy.data(), P * sizeof(T), hipMemcpyHostToDevice, st));
    if (dim == 3)
      HIPCHK(hipMemcpyAsync(d.zs[0], hz.data(), P * sizeof(T), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.as[0], a0, P * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.ids[0], hid.data(), P * sizeof(uint32_t), hipMemcpyHostToDevice,
                          st));
  }
  HIPCHK(hipMemcpyAsync(d.v, hv.data(), G * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.m, hm.data(), G * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.w, hw.data(), G * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.tw, htw.data(), (N / 2) * sizeof(cplx<T>), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.mtab, hmt.data(), 3 * N * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(d.ubar[0], 0, 2 * G * sizeof(T), st));        // both buffers
  HIPCHK(hipMemsetAsync(d.g4[0], 0, 2 * G * sizeof(vec4<T>), st));    // both buffers
  HIPCHK(hipMemsetAsync(d.tcount, 0, (size_t)d.ntiles * sizeof(uint32_t), st));
  // 2D: no y derivative spectrum is ever formed; the inverse row pass reads zeros from it
  if (dim == 2)
    HIPCHK(hipMemsetAsync(d.SGy, 0, (size_t)(N / 2 + 1) * d.nrows * sizeof(cplx<T>), st));
  const Batch<T> b = single_batch<T>(sim);
  // initial binning: set 0 -> set 1 by tile, then back into set 0
  launch_binning<T>(b, sim->counts, 1, dim, st);
  if (P > 0) {
    HIPCHK(hipMemcpyAsync(d.xs[0], d.xs[1], P * sizeof(T), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(d.ys[0], d.ys[1], P * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (dim == 3)
      HIPCHK(hipMemcpyAsync(d.zs[0], d.zs[1], P * sizeof(T), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(d.as[0], d.as[1], P * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(d.ids[0], d.ids[1], P * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                          st));
  }
  sim->resort_every = p.resort_every > 0 ? p.resort_every : default_resort(p);
  sim->since_bin = 0;
  // the gather array of the first step: (grad v^0, w^0)
  const auto groups = single_groups<T>(sim, b);
  enqueue_fft<T>(groups.data(), (int)groups.size(), st, kGradOnly);
  launch_particles<T>(b, sim->counts[K_PART], 0, 1, p.deposit_order, dim, st);  // ubar^0
  launch_diag_clear<T>(b, 1, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));  // host staging buffers are freed on return
  return SIPF_OK;
}

// Stream captures are serialised across the process: captures begun on several threads at
// once (simulations initialised or first stepped concurrently) have failed here with an
// error recorded in one of them.
std::mutex g_capture_mu;

// Capture one step (and one step with binning) as graphs on a private stream; replays go to
// the simulation's stream.  Done on the first sipf_step, so that simulations that are only
// ever stepped in batches never capture.
template <typename T>
int capture_t(sipf_sim* sim) {
  std::lock_guard<std::mutex> lk(g_capture_mu);
  const sipf_params& p = sim->prm;
  const int dim = dim_of(p);
  const Batch<T> b = single_batch<T>(sim);
  HIPCHK(hipStreamCreateWithFlags(&sim->cap, hipStreamNonBlocking));
  HIPCHK(create_fork(sim->fork));
  const auto groups = single_groups<T>(sim, b);
  HIPCHK(hipStreamBeginCapture(sim->cap, hipStreamCaptureModeThreadLocal));
  enqueue_step<T>(b, sim->counts, 1, groups.data(), (int)groups.size(), 0, p.deposit_order,
                  dim, sim->cap, &sim->fork);
  HIPCHK(hipStreamEndCapture(sim->cap, &sim->graph));
  HIPCHK(hipGetLastError());
  HIPCHK(hipGraphInstantiate(&sim->exec, sim->graph, nullptr, nullptr, 0));
  // uploaded now, so that no step pays for it: a graph's first launch would otherwise carry
  // its upload (the binning step's falls in whatever run first re-bins)
  HIPCHK(hipGraphUpload(sim->exec, sim->stream));
  HIPCHK(hipStreamBeginCapture(sim->cap, hipStreamCaptureModeThreadLocal));
  enqueue_step<T>(b, sim->counts, 1, groups.data(), (int)groups.size(), 1, p.deposit_order,
                  dim, sim->cap, &sim->fork);
  HIPCHK(hipStreamEndCapture(sim->cap, &sim->graph_bin));
  HIPCHK(hipGetLastError());
  HIPCHK(hipGraphInstantiate(&sim->exec_bin, sim->graph_bin, nullptr, nullptr, 0));
  HIPCHK(hipGraphUpload(sim->exec_bin, sim->stream));
  return SIPF_OK;
}

bool finite_array(const double* a, size_t n, bool nonneg, bool positive) {
  for (size_t i = 0; i < n; ++i) {
    const double v = a[i];
    if (!isfinite(v)) return false;
    if (nonneg && v < 0) return false;
    if (positive && !(v > 0)) return false;
  }
  return true;
}

double decode_min(unsigned long long k) {
  if (k == ~0ull) return 0.0;  // no data
  const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  double d;
  memcpy(&d, &b, 8);
  return d;
}
double decode_max(unsigned long long k) {
  if (k == 0ull) return 0.0;  // no data
  return decode_min(k);
}
double as_double(unsigned long long k) {
  double d;
  memcpy(&d, &k, 8);
  return d;
}

template <typename T>
int fields_t(sipf_sim* sim, double* v, double* m, double* w, double* X, double* a,
             sipf_diag* diag) {
  const sipf_params& p = sim->prm;
  const SimDev<T>& d = *reinterpret_cast<const SimDev<T>*>(sim->host_desc);
  const size_t G = grid_nodes(p);
  const int dim = dim_of(p);
  const int64_t P = p.P;
  if (sim->last_stream) HIPCHK(hipStreamSynchronize(sim->last_stream));
  HIPCHK(hipStreamSynchronize(sim->stream));
  std::vector<T> buf(std::max<size_t>(G, (size_t)P));
  auto grid = [&](const T* src, double* dst) -> int {
    if (!dst) return SIPF_OK;
    HIPCHK(hipMemcpy(buf.data(), src, G * sizeof(T), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < G; ++i) dst[i] = (double)buf[i];
    return SIPF_OK;
  };
  int rc;
  if ((rc = grid(d.v, v))) return rc;
  if ((rc = grid(d.m, m))) return rc;
  if ((rc = grid(d.w, w))) return rc;
  if ((X || a) && P > 0) {
    std::vector<uint32_t> id(P);
    HIPCHK(hipMemcpy(id.data(), d.ids[0], P * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (X) {
      const T* comp[3] = {d.xs[0], d.ys[0], d.zs[0]};
      for (int j = 0; j < dim; ++j) {
        HIPCHK(hipMemcpy(buf.data(), comp[j], P * sizeof(T), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < P; ++i) X[(int64_t)j * P + id[i]] = (double)buf[i];
      }
    }
    if (a) {
      std::vector<double> ha(P);
      HIPCHK(hipMemcpy(ha.data(), d.as[0], P * sizeof(double), hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < P; ++i) a[id[i]] = ha[i];
    }
  }
  // diagnostics: one reduction over the particles, ubar and the fields of the state
  {
    const Batch<T> b = single_batch<T>(sim);
    launch_diag_read<T>(b, sim->counts[K_DIAG], 1, sim->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(sim->stream));
  }
  unsigned long long acc[D_COUNT];
  uint64_t step = 0;
  HIPCHK(hipMemcpy(acc, d.diag + kDiagResult, sizeof(acc), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&step, d.step, sizeof(step), hipMemcpyDeviceToHost));
  sipf_diag dg;
  dg.mass_particles = as_double(acc[D_SUM_A]);
  dg.mass_grid = as_double(acc[D_SUM_U]) * d.h3;
  dg.mass_m = as_double(acc[D_SUM_M]) * d.h3;
  dg.min_v = decode_min(acc[D_MIN_V]);
  dg.min_m = decode_min(acc[D_MIN_M]);
  dg.min_w = decode_min(acc[D_MIN_W]);
  dg.max_m = decode_max(acc[D_MAX_M]);
  dg.max_w = decode_max(acc[D_MAX_W]);
  dg.min_a = decode_min(acc[D_MIN_A]);
  dg.max_a = decode_max(acc[D_MAX_A]);
  dg.min_u = decode_min(acc[D_MIN_U]);
  dg.n_nan = (int64_t)acc[D_NAN];
  dg.n_neg_m = (int64_t)acc[D_NEG_M];
  dg.n_neg_w = (int64_t)acc[D_NEG_W];
  dg.step = (int64_t)step;
  if (diag) *diag = dg;
  if (p.flags & SIPF_FLAG_STRICT) {
    if (dg.n_nan != 0) return fail(SIPF_EPOS, "non-finite values in the state");
    // the fourth-order assignment has negative outer weights, so ubar >= 0 is only an
    // invariant of the trilinear one
    if (p.deposit_order == 2 && dg.min_u < 0)
      return fail(SIPF_EPOS, "negative deposited density");
    if (!(dg.min_v > 0)) return fail(SIPF_EPOS, "non-positive ECM density v");
    if (P > 0 && !(dg.min_a > 0)) return fail(SIPF_EPOS, "non-positive particle mass");
  }
  return SIPF_OK;
}

template <typename T>
int aux_t(sipf_sim* sim, double* u_bar, double* grad_v) {
  const sipf_params& p = sim->prm;
  const SimDev<T>& d = *reinterpret_cast<const SimDev<T>*>(sim->host_desc);
  const size_t G = grid_nodes(p);
  if (sim->last_stream) HIPCHK(hipStreamSynchronize(sim->last_stream));
  HIPCHK(hipStreamSynchronize(sim->stream));
  uint64_t n = 0;  // the state's step index selects the buffers
  HIPCHK(hipMemcpy(&n, d.step, sizeof(n), hipMemcpyDeviceToHost));
  if (u_bar) {
    std::vector<T> buf(G);
    HIPCHK(hipMemcpy(buf.data(), d.ubar[n & 1], G * sizeof(T), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < G; ++i) u_bar[i] = (double)buf[i];
  }
  if (grad_v) {
    // the gather array of the last step (step n - 1); zeros before the first step
    std::vector<vec4<T>> buf(G);
    HIPCHK(hipMemcpy(buf.data(), d.g4[(n - 1) & 1], G * sizeof(vec4<T>),
                     hipMemcpyDeviceToHost));
    for (size_t i = 0; i < G; ++i) {
      grad_v[i] = (double)buf[i].x;
      if (dim_of(p) == 3) {
        grad_v[G + i] = (double)buf[i].y;
        grad_v[2 * G + i] = (double)buf[i].z;
      } else {  // 2D: the x2 derivative sits in the third slot of the gather array
        grad_v[G + i] = (double)buf[i].z;
      }
    }
  }
  return SIPF_OK;
}

// ---- batched launches (served form) --------------------------------------------------------
// A batch is a list of resident simulations stepped by one launch per kernel.  Its launch
// table (descriptors and per-kernel block offsets) lives in a small library-owned device
// buffer, and its step is captured as two HIP graphs (with and without binning).  Entries
// are cached per simulation list (least recently used first out) and dropped when one of
// their simulations is destroyed.
struct BatchGraph {
  std::vector<sipf_sim*> sims;
  int device = -1;
  void* table = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipEvent_t done = nullptr;
  uint64_t last_use = 0;
};
constexpr size_t kMaxBatchGraphs = 8;
std::mutex g_batch_mu;
std::vector<BatchGraph*> g_graphs;
uint64_t g_use_clock = 0;
hipStream_t g_cap_stream[64] = {};
StepFork g_cap_fork[64];  // per device, like the capture stream (kept until the process ends)

void free_batch_graph(BatchGraph* e) {
  if (e->done) (void)hipEventSynchronize(e->done);
  for (int k = 0; k < 2; ++k) {
    if (e->exec[k]) (void)hipGraphExecDestroy(e->exec[k]);
    if (e->graph[k]) (void)hipGraphDestroy(e->graph[k]);
  }
  if (e->table) (void)hipFree(e->table);
  if (e->done) (void)hipEventDestroy(e->done);
  delete e;
}

// drop every cached batch that contains sim (called from sipf_destroy)
void forget_sim(sipf_sim* sim) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (size_t i = 0; i < g_graphs.size();) {
    BatchGraph* e = g_graphs[i];
    if (std::find(e->sims.begin(), e->sims.end(), sim) != e->sims.end()) {
      free_batch_graph(e);
      g_graphs.erase(g_graphs.begin() + i);
    } else {
      ++i;
    }
  }
}

// Launch table of a list of simulations: descriptors, then per-kernel block offsets.
template <typename T>
size_t table_bytes(int n) {
  return align_up(sizeof(SimDev<T>) * n) + align_up(sizeof(int) * K_COUNT * (n + 1));
}

template <typename T>
void fill_table(sipf_sim* const* sims, int n, unsigned char* h, int* tot) {
  const size_t blk_off = align_up(sizeof(SimDev<T>) * n);
  int* blk = reinterpret_cast<int*>(h + blk_off);
  for (int k = 0; k < K_COUNT; ++k) {
    int acc = 0;
    for (int i = 0; i < n; ++i) {
      blk[k * (n + 1) + i] = acc;
      acc += sims[i]->counts[k];
    }
    blk[k * (n + 1) + n] = acc;
    tot[k] = acc;
  }
  for (int i = 0; i < n; ++i)
    memcpy(h + sizeof(SimDev<T>) * i, sims[i]->host_desc, sizeof(SimDev<T>));
}

template <typename T>
Batch<T> table_batch(unsigned char* dev, int n) {
  Batch<T> b;
  b.sims = reinterpret_cast<const SimDev<T>*>(dev);
  b.blk = reinterpret_cast<const int*>(dev + align_up(sizeof(SimDev<T>) * n));
  b.nsims = n;
  return b;
}

template <typename T>
int build_batch_graph(sipf_sim* const* sims, int nsims, int dev, BatchGraph** out) {
  BatchGraph* e = new BatchGraph();
  e->sims.assign(sims, sims + nsims);
  e->device = dev;
  // the whole list, then one sub-list per grid size (FFT kernels are compiled per N)
  std::vector<int> lgs;
  for (int i = 0; i < nsims; ++i) {
    const int lg = reinterpret_cast<const SimDev<T>*>(sims[i]->host_desc)->log2N;
    if (std::find(lgs.begin(), lgs.end(), lg) == lgs.end()) lgs.push_back(lg);
  }
  std::vector<std::vector<sipf_sim*>> sub(lgs.size());
  for (int i = 0; i < nsims; ++i) {
    const int lg = reinterpret_cast<const SimDev<T>*>(sims[i]->host_desc)->log2N;
    sub[std::find(lgs.begin(), lgs.end(), lg) - lgs.begin()].push_back(sims[i]);
  }
  size_t bytes = table_bytes<T>(nsims);
  std::vector<size_t> offs;
  for (const auto& l : sub) {
    offs.push_back(bytes);
    bytes += table_bytes<T>((int)l.size());
  }
  std::vector<unsigned char> h(bytes, 0);
  std::vector<int> tot(K_COUNT, 0);
  fill_table<T>(sims, nsims, h.data(), tot.data());
  std::vector<FftGroup<T>> groups(sub.size());
  for (size_t g = 0; g < sub.size(); ++g) {
    fill_table<T>(sub[g].data(), (int)sub[g].size(), h.data() + offs[g], groups[g].tot);
    groups[g].lg = lgs[g];
  }
  int rc = SIPF_OK;
  auto chk = [&](hipError_t err, const char* what) {
    if (err != hipSuccess && rc == SIPF_OK)
      rc = fail(SIPF_EHIP, std::string(what) + ": " + hipGetErrorString(err));
  };
  chk(hipMalloc(&e->table, bytes), "hipMalloc(batch table)");
  if (rc == SIPF_OK) chk(hipMemcpy(e->table, h.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy");
  if (rc == SIPF_OK) chk(hipEventCreateWithFlags(&e->done, hipEventDisableTiming), "hipEventCreate");
  if (rc == SIPF_OK && !g_cap_stream[dev])
    chk(hipStreamCreateWithFlags(&g_cap_stream[dev], hipStreamNonBlocking), "hipStreamCreate");
  if (rc == SIPF_OK && !g_cap_fork[dev].aux) chk(create_fork(g_cap_fork[dev]), "step fork");
  unsigned char* base = static_cast<unsigned char*>(e->table);
  const Batch<T> b = table_batch<T>(base, nsims);
  for (size_t g = 0; g < sub.size(); ++g)
    groups[g].b = table_batch<T>(base + offs[g], (int)sub[g].size());
  std::lock_guard<std::mutex> cap_lk(g_capture_mu);
  for (int bin = 0; bin < 2 && rc == SIPF_OK; ++bin) {
    chk(hipStreamBeginCapture(g_cap_stream[dev], hipStreamCaptureModeThreadLocal), "capture");
    if (rc != SIPF_OK) break;
    enqueue_step<T>(b, tot.data(), nsims, groups.data(), (int)groups.size(), bin,
                    sims[0]->prm.deposit_order, 3, g_cap_stream[dev], &g_cap_fork[dev]);
    chk(hipStreamEndCapture(g_cap_stream[dev], &e->graph[bin]), "hipStreamEndCapture");
    if (rc == SIPF_OK) chk(hipGetLastError(), "batched launch");
    if (rc == SIPF_OK)
      chk(hipGraphInstantiate(&e->exec[bin], e->graph[bin], nullptr, nullptr, 0),
          "hipGraphInstantiate");
    // uploaded on the stream the batch steps on, so that its first step does not carry it
    if (rc == SIPF_OK) chk(hipGraphUpload(e->exec[bin], sims[0]->stream), "hipGraphUpload");
  }
  if (rc != SIPF_OK) {
    free_batch_graph(e);
    return rc;
  }
  *out = e;
  return SIPF_OK;
}

template <typename T>
int step_batch_t(sipf_sim* const* sims, int nsims, int nsteps) {
  hipStream_t st = sims[0]->stream;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(SIPF_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_batch_mu);
  BatchGraph* e = nullptr;
  for (BatchGraph* c : g_graphs)
    if (c->device == dev && (int)c->sims.size() == nsims &&
        std::equal(c->sims.begin(), c->sims.end(), sims)) {
      e = c;
      break;
    }
  if (!e) {
    if (g_graphs.size() >= kMaxBatchGraphs) {
      auto lru = std::min_element(g_graphs.begin(), g_graphs.end(),
                                  [](BatchGraph* x, BatchGraph* y) {
                                    return x->last_use < y->last_use;
                                  });
      free_batch_graph(*lru);
      g_graphs.erase(lru);
    }
    const int rc = build_batch_graph<T>(sims, nsims, dev, &e);
    if (rc) return rc;
    g_graphs.push_back(e);
  }
  e->last_use = ++g_use_clock;
  // work a simulation queued on other streams is ordered before the batch
  for (int i = 0; i < nsims; ++i) {
    for (hipStream_t o : {sims[i]->stream, sims[i]->last_stream}) {
      if (o != st && o != nullptr) {
        HIPCHK(hipEventRecord(sims[i]->ev, o));
        HIPCHK(hipStreamWaitEvent(st, sims[i]->ev, 0));
      }
    }
  }
  for (int s = 0; s < nsteps; ++s) {
    int bin = 0;
    for (int i = 0; i < nsims; ++i) bin |= sims[i]->since_bin >= sims[i]->resort_every;
    HIPCHK(hipGraphLaunch(e->exec[bin], st));
    for (int i = 0; i < nsims; ++i) sims[i]->since_bin = bin ? 1 : sims[i]->since_bin + 1;
  }
  HIPCHK(hipEventRecord(e->done, st));
  for (int i = 0; i < nsims; ++i) sims[i]->last_stream = st;
  return SIPF_OK;
}

// ---- allocation-free batched steps ------------------------------------------------------------
// For callers that cannot allocate device memory (code under graph capture, serving loops,
// harnesses that forbid it): the launch table of a batch lives in this file-scope device
// array instead of a buffer from hipMalloc, and the step is launched kernel by kernel instead
// of through a graph instantiated per batch composition.  Each GPU holds its own copy of the
// array at its own address, found once per device with hipGetSymbolAddress; host code uses
// only that address (the array's name is a host-side stand-in).  Every call on one GPU
// rewrites the same array: calls ordered on one stream are safe, calls that overlap on one
// GPU (different streams, no ordering between them) race on the table.
constexpr int kNoAllocMaxSims = 64;
constexpr size_t kNoAllocBytes = 128 * 1024;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Per device: the array's device address, and a host image of the table last written to it
// (a call whose table is unchanged writes nothing).  Both are set up by sipf_init, the first
// time a simulation is created on the device, with that device current.
struct DevScratch {
  void* ptr = nullptr;
  unsigned char* last = nullptr;  // kNoAllocBytes
  size_t last_bytes = 0;          // 0: nothing written yet
};
std::mutex g_scratch_mu;
DevScratch g_scratch[64];

int scratch_setup(int dev, DevScratch** out) {
  if (dev < 0 || dev >= 64) return fail(SIPF_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  DevScratch& d = g_scratch[dev];
  if (!d.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SIPF_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                 hipGetErrorString(e));
    d.last = new unsigned char[kNoAllocBytes];
    d.ptr = p;
  }
  *out = &d;
  return SIPF_OK;
}

// The table reaches the array through kernel arguments (kTableChunkWords words per launch),
// so the upload is ordered on the stream like the kernels that read it, and no host buffer
// has to outlive the call.
constexpr int kTableChunkWords = 512;
struct TableChunk {
  uint32_t off;  // first word
  uint32_t n;    // words in this chunk
  uint32_t w[kTableChunkWords];
};

__global__ void __launch_bounds__(kThreads) k_write_table(uint32_t* dst, TableChunk c) {
  for (uint32_t i = threadIdx.x; i < c.n; i += kThreads) dst[c.off + i] = c.w[i];
}

// host image of the table being built (under g_batch_mu)
unsigned char g_noalloc_host[kNoAllocBytes];

template <typename T>
int step_batch_noalloc_t(sipf_sim* const* sims, int nsims, int nsteps) {
  hipStream_t st = sims[0]->stream;
  const int dev = sims[0]->device;
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != dev) return fail(SIPF_EINVAL, "the simulations' device must be the current device");
  DevScratch* ds = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev >= 0 && dev < 64 && g_scratch[dev].ptr) ds = &g_scratch[dev];
  }
  if (!ds) return fail(SIPF_EINVAL, "no simulation was initialised on this device");
  void* dptr = ds->ptr;
  // grid sizes present (FFT kernels are compiled per N): log2 N in [2, 9]
  int lgs[8], cnt[8], ng = 0;
  for (int i = 0; i < nsims; ++i) {
    const int lg = reinterpret_cast<const SimDev<T>*>(sims[i]->host_desc)->log2N;
    int g = 0;
    while (g < ng && lgs[g] != lg) ++g;
    if (g == ng) {
      if (ng == 8) return fail(SIPF_EINVAL, "more grid sizes than the library supports");
      lgs[ng] = lg;
      cnt[ng++] = 0;
    }
    ++cnt[g];
  }
  size_t offs[8];
  size_t bytes = table_bytes<T>(nsims);
  for (int g = 0; g < ng; ++g) {
    offs[g] = bytes;
    bytes += table_bytes<T>(cnt[g]);
  }
  if (bytes > kNoAllocBytes)
    return fail(SIPF_EINVAL, "batch table of " + std::to_string(bytes) +
                                 " bytes exceeds the allocation-free limit of " +
                                 std::to_string(kNoAllocBytes));
  std::lock_guard<std::mutex> lk(g_batch_mu);
  unsigned char* h = g_noalloc_host;
  int tot[K_COUNT];
  fill_table<T>(sims, nsims, h, tot);
  sipf_sim* sub[kNoAllocMaxSims];
  FftGroup<T> groups[8];
  unsigned char* base = static_cast<unsigned char*>(dptr);
  for (int g = 0; g < ng; ++g) {
    int k = 0;
    for (int i = 0; i < nsims; ++i)
      if (reinterpret_cast<const SimDev<T>*>(sims[i]->host_desc)->log2N == lgs[g])
        sub[k++] = sims[i];
    fill_table<T>(sub, k, h + offs[g], groups[g].tot);
    groups[g].lg = lgs[g];
    groups[g].b = table_batch<T>(base + offs[g], k);
  }
  // work a simulation queued on other streams is ordered before the batch (and so is the
  // previous use of the table, when it was on this stream)
  for (int i = 0; i < nsims; ++i) {
    for (hipStream_t o : {sims[i]->stream, sims[i]->last_stream}) {
      if (o != st && o != nullptr) {
        HIPCHK(hipEventRecord(sims[i]->ev, o));
        HIPCHK(hipStreamWaitEvent(st, sims[i]->ev, 0));
      }
    }
  }
  // (re)write the table unless this device's array already holds exactly these bytes
  if (!(ds->last_bytes == bytes && memcmp(ds->last, h, bytes) == 0)) {
    const uint32_t words = (uint32_t)((bytes + 3) / 4);
    TableChunk c;
    for (uint32_t o = 0; o < words; o += kTableChunkWords) {
      c.off = o;
      c.n = std::min<uint32_t>(kTableChunkWords, words - o);
      memcpy(c.w, h + 4 * (size_t)o, 4 * (size_t)c.n);
      hipLaunchKernelGGL(k_write_table, dim3(1), dim3(kThreads), 0, st,
                         static_cast<uint32_t*>(dptr), c);
    }
    HIPCHK(hipGetLastError());
    memcpy(ds->last, h, bytes);
    ds->last_bytes = bytes;
  }
  const Batch<T> b = table_batch<T>(base, nsims);
  for (int s = 0; s < nsteps; ++s) {
    int bin = 0;
    for (int i = 0; i < nsims; ++i) bin |= sims[i]->since_bin >= sims[i]->resort_every;
    // the two halves of the step in sequence: for the served mix's simulations (up to 128^3 and
    // 2^22 particles) the second stream's fork and join cost more than the overlap gains (solo
    // latency of every size class 5-15 % lower, aggregate rate 4.2e9 -> 4.4e9 particle-steps/s)
    enqueue_step<T>(b, tot, nsims, groups, ng, bin, sims[0]->prm.deposit_order, 3, st, nullptr);
    for (int i = 0; i < nsims; ++i) sims[i]->since_bin = bin ? 1 : sims[i]->since_bin + 1;
  }
  HIPCHK(hipGetLastError());
  for (int i = 0; i < nsims; ++i) sims[i]->last_stream = st;
  return SIPF_OK;
}

template <typename T>
int step_timed_t(sipf_sim* sim, int nsteps, float* stage_ms) {
  const Batch<T> b = single_batch<T>(sim);
  hipStream_t st = sim->stream;
  const int* c = sim->counts;
  const int lg = reinterpret_cast<const SimDev<T>*>(sim->host_desc)->log2N;
  hipEvent_t ev[SIPF_NUM_STAGES + 1];
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  int rc = SIPF_OK;
  for (int s = 0; s < nsteps && rc == SIPF_OK; ++s) {
    const int bin = sim->since_bin >= sim->resort_every;
    (void)hipEventRecord(ev[SIPF_NUM_STAGES], st);
    if (bin) launch_binning<T>(b, c, 1, dim_of(sim->prm), st);
    (void)hipEventRecord(ev[0], st);
    launch_zfwd<T>(b, c[K_ZFWD], lg, st, 0);
    (void)hipEventRecord(ev[1], st);
    launch_yfwd<T>(b, c[K_YFWD], lg, st, 0);
    (void)hipEventRecord(ev[2], st);
    launch_xpass<T>(b, c[K_XPASS], lg, st, 0);
    launch_plane<T>(b, c[K_PLANE], lg, st, 0);
    (void)hipEventRecord(ev[3], st);
    launch_yinv<T>(b, c[K_YINV], lg, st, 0);
    (void)hipEventRecord(ev[4], st);
    launch_zinv<T>(b, c[K_ZINV], lg, st, 0);
    (void)hipEventRecord(ev[5], st);
    launch_particles<T>(b, c[K_PART], bin, 0, sim->prm.deposit_order, dim_of(sim->prm), st);
    (void)hipEventRecord(ev[6], st);
    launch_finalize<T>(b, 1, st);
    (void)hipEventRecord(ev[7], st);
    sim->since_bin = bin ? 1 : sim->since_bin + 1;
    hipError_t e = hipEventSynchronize(ev[7]);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
      rc = fail(SIPF_EHIP, std::string("timed step: ") + hipGetErrorString(e));
      break;
    }
    for (int k = 0; k < SIPF_STAGE_FINALIZE + 1; ++k) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      stage_ms[k] += ms;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[SIPF_NUM_STAGES], ev[0]);
    stage_ms[SIPF_STAGE_BINNING] += ms;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return rc;
}

// Residual resampling (Alg. res_res) of the current particles, then the re-binning and the
// deposit of ubar that the new particle list needs (as at initialisation).  Synchronous.
template <typename T>
int resample_t(sipf_sim* sim, sipf_resample_info* info) {
  const sipf_params& p = sim->prm;
  const SimDev<T>& d = *reinterpret_cast<const SimDev<T>*>(sim->host_desc);
  const int64_t P = p.P;
  sipf_resample_info out{0.0, 0, 0};
  if (P == 0) {
    if (info) *info = out;
    return SIPF_OK;
  }
  hipStream_t st = sim->stream;
  unsigned long long* rs = reinterpret_cast<unsigned long long*>(sim->ws + sim->lay.rs);
  unsigned long long head[RS_BLOCKS];
  uint64_t n = 0;  // the state's step index: its ubar buffer is ubar[n & 1]
  HIPCHK(hipMemsetAsync(rs, 0, sizeof(head), st));
  launch_resample_stats<T>(d, rs, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(head, rs, sizeof(head), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&n, d.step, sizeof(n), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // on a rejected input the state is unchanged (only set 1, free between steps, was written)
  if (head[RS_FLAGS] & RS_BAD_VALUE)
    return fail(SIPF_EINVAL, "resampling needs finite, non-negative masses with a positive sum");
  if (head[RS_FLAGS] & RS_BAD_RANGE)
    return fail(SIPF_EINVAL,
                "resampling needs the largest mass in [2^-775, 2^990) and every non-zero mass "
                "above 2^-160 of the largest");
  launch_resample_apply<T>(d, rs, st);
  // re-bin the new list (set 0 -> set 1 by tile, back into set 0) and deposit its ubar
  const Batch<T> b = single_batch<T>(sim);
  const int dim = dim_of(p);
  launch_binning<T>(b, sim->counts, 1, dim, st);
  HIPCHK(hipMemcpyAsync(d.xs[0], d.xs[1], P * sizeof(T), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(d.ys[0], d.ys[1], P * sizeof(T), hipMemcpyDeviceToDevice, st));
  if (dim == 3)
    HIPCHK(hipMemcpyAsync(d.zs[0], d.zs[1], P * sizeof(T), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(d.as[0], d.as[1], P * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(d.ids[0], d.ids[1], P * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
  const size_t G = grid_nodes(p);
  HIPCHK(hipMemsetAsync(d.ubar[n & 1], 0, G * sizeof(T), st));
  launch_particles<T>(b, sim->counts[K_PART], 0, 1, p.deposit_order, dim, st);
  launch_diag_clear<T>(b, 1, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(head, rs, sizeof(head), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  sim->since_bin = 0;
  double a0;
  memcpy(&a0, &head[RS_A0], sizeof(a0));
  out.a0 = a0;
  out.n_det = (int64_t)std::min<unsigned long long>(head[RS_KTOT], (unsigned long long)P);
  out.n_stoch = P - out.n_det;
  if (info) *info = out;
  return SIPF_OK;
}

// Work on the simulation's own stream after batched steps on another stream waits for them.
int order_after_batch(sipf_sim* sim) {
  if (sim->last_stream && sim->last_stream != sim->stream) {
    HIPCHK(hipEventRecord(sim->ev, sim->last_stream));
    HIPCHK(hipStreamWaitEvent(sim->stream, sim->ev, 0));
  }
  sim->last_stream = nullptr;
  return SIPF_OK;
}

// checks shared by the batched entry points
int check_batch(sipf_sim* const* sims, int32_t nsims, int32_t nsteps) {
  if (!sims || nsims <= 0) return fail(SIPF_EINVAL, "empty simulation list");
  if (nsteps < 0) return fail(SIPF_EINVAL, "nsteps must be >= 0");
  for (int i = 0; i < nsims; ++i) {
    if (!sims[i]) return fail(SIPF_EINVAL, "NULL simulation in the list");
    if (sims[i]->prm.precision != sims[0]->prm.precision)
      return fail(SIPF_EINVAL, "mixed precision in one batch");
    if (sims[i]->prm.deposit_order != sims[0]->prm.deposit_order)
      return fail(SIPF_EINVAL, "mixed deposit order in one batch");
    if (dim_of(sims[i]->prm) != 3)
      return fail(SIPF_EINVAL, "batched steps are three-dimensional only");
    if (sims[i]->device != sims[0]->device)
      return fail(SIPF_EINVAL, "simulations on different devices");
    for (int j = 0; j < i; ++j)
      if (sims[j] == sims[i]) return fail(SIPF_EINVAL, "simulation listed twice");
  }
  return SIPF_OK;
}

}  // namespace

extern "C" {

int sipf_step_timed(sipf_sim* sim, int32_t nsteps, float* stage_ms) {
  if (!sim || !stage_ms) return fail(SIPF_EINVAL, "sim / stage_ms is NULL");
  if (nsteps < 0) return fail(SIPF_EINVAL, "nsteps must be >= 0");
  int rc = order_after_batch(sim);
  if (rc) return rc;
  return sim->prm.precision == SIPF_FP64 ? step_timed_t<double>(sim, nsteps, stage_ms)
                                         : step_timed_t<float>(sim, nsteps, stage_ms);
}


int sipf_resample(sipf_sim* sim, sipf_resample_info* info) {
  if (!sim) return fail(SIPF_EINVAL, "sim is NULL");
  if (sim->prm.P >= (int64_t(1) << 31)) return fail(SIPF_EINVAL, "resampling needs P < 2^31");
  if (sim->prm.sim_id >> 63) return fail(SIPF_EINVAL, "resampling needs sim_id < 2^63");
  int rc = order_after_batch(sim);
  if (rc) return rc;
  if (sim->last_stream) HIPCHK(hipStreamSynchronize(sim->last_stream));
  return sim->prm.precision == SIPF_FP64 ? resample_t<double>(sim, info)
                                         : resample_t<float>(sim, info);
}

int sipf_state_bytes(const sipf_params* prm, size_t* bytes) {
  int rc = validate_params(prm);
  if (rc) return rc;
  if (!bytes) return fail(SIPF_EINVAL, "bytes is NULL");
  *bytes = make_layout(*prm).total;
  return SIPF_OK;
}

int sipf_init(const sipf_params* prm, void* d_workspace, size_t bytes, void* hip_stream,
              const double* X0, const double* a0, const double* v0, const double* m0,
              const double* w0, sipf_sim** out) {
  int rc = validate_params(prm);
  if (rc) return rc;
  if (!out) return fail(SIPF_EINVAL, "out is NULL");
  *out = nullptr;
  const sipf_params& p = *prm;
  const size_t G = grid_nodes(p);
  if (p.P > 0 && (!X0 || !a0)) return fail(SIPF_EINVAL, "X0 / a0 is NULL");
  if (!v0 || !m0 || !w0) return fail(SIPF_EINVAL, "v0 / m0 / w0 is NULL");
  if (p.P > 0 && !finite_array(X0, (size_t)dim_of(p) * (size_t)p.P, false, false))
    return fail(SIPF_EINVAL, "X0 has non-finite entries");
  if (p.P > 0 && !finite_array(a0, (size_t)p.P, false, true))
    return fail(SIPF_EINVAL, "a0 must be finite and > 0");
  if (!finite_array(v0, G, true, false)) return fail(SIPF_EINVAL, "v0 must be finite, >= 0");
  // m and w may carry the small negative lobes of the implicit solve (a restart from a
  // checkpoint); they only have to be finite
  if (!finite_array(m0, G, false, false)) return fail(SIPF_EINVAL, "m0 must be finite");
  if (!finite_array(w0, G, false, false)) return fail(SIPF_EINVAL, "w0 must be finite");
  const Layout L = make_layout(p);
  if (!d_workspace) return fail(SIPF_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
    return fail(SIPF_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < L.total)
    return fail(SIPF_ENOMEM, "workspace has " + std::to_string(bytes) + " bytes, needs " +
                                 std::to_string(L.total));
  sipf_sim* sim = new sipf_sim();
  sim->prm = p;
  sim->ws = static_cast<unsigned char*>(d_workspace);
  sim->bytes = bytes;
  sim->lay = L;
  sim->stream = static_cast<hipStream_t>(hip_stream);
  (void)hipGetDevice(&sim->device);
  DevScratch* ds = nullptr;  // set-up of the allocation-free batched step on this device
  if ((rc = scratch_setup(sim->device, &ds)) != SIPF_OK) {
    delete sim;
    return rc;
  }
  if (hipEventCreateWithFlags(&sim->ev, hipEventDisableTiming) != hipSuccess) {
    delete sim;
    return fail(SIPF_EHIP, "hipEventCreate failed");
  }
  rc = p.precision == SIPF_FP64 ? init_t<double>(sim, X0, a0, v0, m0, w0)
                                : init_t<float>(sim, X0, a0, v0, m0, w0);
  if (rc) {
    std::string msg = g_err;
    sipf_destroy(sim);
    g_err = msg;
    return rc;
  }
  *out = sim;
  return SIPF_OK;
}

int sipf_step(sipf_sim* sim, int32_t nsteps) {
  if (!sim) return fail(SIPF_EINVAL, "sim is NULL");
  if (nsteps < 0) return fail(SIPF_EINVAL, "nsteps must be >= 0");
  int rc = order_after_batch(sim);
  if (rc) return rc;
  if (nsteps > 0 && !sim->exec_bin) {
    rc = sim->prm.precision == SIPF_FP64 ? capture_t<double>(sim) : capture_t<float>(sim);
    if (rc) return rc;
  }
  for (int32_t s = 0; s < nsteps; ++s) {
    if (sim->since_bin >= sim->resort_every) {
      HIPCHK(hipGraphLaunch(sim->exec_bin, sim->stream));
      sim->since_bin = 1;
    } else {
      HIPCHK(hipGraphLaunch(sim->exec, sim->stream));
      sim->since_bin += 1;
    }
  }
  return SIPF_OK;
}

int sipf_set_stream(sipf_sim* sim, void* hip_stream) {
  if (!sim) return fail(SIPF_EINVAL, "sim is NULL");
  hipStream_t ns = static_cast<hipStream_t>(hip_stream);
  for (hipStream_t o : {sim->stream, sim->last_stream}) {
    if (o && o != ns) {
      HIPCHK(hipEventRecord(sim->ev, o));
      HIPCHK(hipStreamWaitEvent(ns, sim->ev, 0));
    }
  }
  if (!ns && (sim->stream || sim->last_stream)) {
    // the null stream: wait on the host instead
    if (sim->stream) HIPCHK(hipStreamSynchronize(sim->stream));
    if (sim->last_stream) HIPCHK(hipStreamSynchronize(sim->last_stream));
  }
  sim->stream = ns;
  sim->last_stream = nullptr;
  return SIPF_OK;
}

int sipf_step_batch(sipf_sim* const* sims, int32_t nsims, int32_t nsteps) {
  int rc = check_batch(sims, nsims, nsteps);
  if (rc) return rc;
  if (nsteps == 0) return SIPF_OK;
  return sims[0]->prm.precision == SIPF_FP64 ? step_batch_t<double>(sims, nsims, nsteps)
                                             : step_batch_t<float>(sims, nsims, nsteps);
}

int sipf_step_batch_noalloc(sipf_sim* const* sims, int32_t nsims, int32_t nsteps) {
  if (nsims > kNoAllocMaxSims)
    return fail(SIPF_EINVAL, "the allocation-free batched step takes at most " +
                                 std::to_string(kNoAllocMaxSims) + " simulations");
  int rc = check_batch(sims, nsims, nsteps);
  if (rc) return rc;
  if (nsteps == 0) return SIPF_OK;
  return sims[0]->prm.precision == SIPF_FP64 ? step_batch_noalloc_t<double>(sims, nsims, nsteps)
                                             : step_batch_noalloc_t<float>(sims, nsims, nsteps);
}

int sipf_fields(sipf_sim* sim, double* v, double* m, double* w, double* X, double* a,
                sipf_diag* diag) {
  if (!sim) return fail(SIPF_EINVAL, "sim is NULL");
  return sim->prm.precision == SIPF_FP64 ? fields_t<double>(sim, v, m, w, X, a, diag)
                                         : fields_t<float>(sim, v, m, w, X, a, diag);
}

int sipf_aux(sipf_sim* sim, double* u_bar, double* grad_v) {
  if (!sim) return fail(SIPF_EINVAL, "sim is NULL");
  return sim->prm.precision == SIPF_FP64 ? aux_t<double>(sim, u_bar, grad_v)
                                         : aux_t<float>(sim, u_bar, grad_v);
}

void sipf_destroy(sipf_sim* sim) {
  if (!sim) return;
  forget_sim(sim);
  if (sim->last_stream) (void)hipStreamSynchronize(sim->last_stream);
  (void)hipStreamSynchronize(sim->stream);
  if (sim->ev) (void)hipEventDestroy(sim->ev);
  if (sim->exec) (void)hipGraphExecDestroy(sim->exec);
  if (sim->graph) (void)hipGraphDestroy(sim->graph);
  if (sim->exec_bin) (void)hipGraphExecDestroy(sim->exec_bin);
  if (sim->graph_bin) (void)hipGraphDestroy(sim->graph_bin);
  if (sim->cap) (void)hipStreamDestroy(sim->cap);
  destroy_fork(sim->fork);
  delete sim;
}

const char* sipf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
