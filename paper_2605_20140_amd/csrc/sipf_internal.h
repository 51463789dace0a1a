// Internal declarations of libsipf: device-side simulation descriptor, batch tables, device
// helpers (complex arithmetic, Philox4x32-10, ordered atomics) and the kernel launchers.
//
// Every kernel takes a Batch: an array of simulation descriptors in device memory plus, per
// kernel kind, the prefix sums of the blocks each simulation needs.  A block finds its
// simulation from blockIdx.x, so one launch can carry the work of many resident simulations
// (the served form) and a single simulation is the one-entry case.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sipf.h"

namespace sipf {

constexpr int kThreads = 256;  // threads per block of every kernel (4 wavefronts of 64)

// Particle binning: cubic tiles of kTile^3 cells; a particle kernel block handles up to
// kChunk particles of one tile and keeps the tile's nodes, plus the nodes its stencils reach
// and a drift margin, in LDS.
constexpr int kTile = 8;
constexpr int kTile2 = 16;  // square tiles of the two-dimensional form
constexpr int kChunk = 4096;
constexpr int kBinBlock = 2048;  // particles per block of the binning count kernel
// Drift margin of a tile's LDS region, in cells on each side: 3D one cell (11^3 nodes for
// the trilinear stencil; more would cost blocks per CU), 2D four cells (25^2 nodes).
constexpr int kM2 = 4;
// Steps between binnings when the caller leaves it to the library: the largest k for which
// the expected diffusive displacement since the last binning, sqrt(k) s cells with
// s = sqrt(2 D_u dt) / h per step, stays within kBinDrift cells (at most kResortMax).
// Calibrated on the bench workloads.  128^3 / 2^23, s = 0.128: every 8, 12, 16, 24 steps
// 284, 277.5, 277, 283 us per step (binning cost against particles past the margin).  The
// 2D example at 1024^2 / 2^22, s = 0.76: with a one-cell margin 228 us at best (every 2 to 4
// steps), with four cells every 6, 8, 12, 16 steps 191, 188, 187, 192 us.
constexpr double kBinDrift3 = 0.45;
constexpr double kBinDrift2 = 2.4;
constexpr int kResortMax = 64;

// Plane pass: one block of kPlaneThreads per k3 plane and job when a plane fits in LDS.
constexpr int kPlaneThreads = 1024;
constexpr size_t kPlaneLdsMax = 150 * 1024;

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

template <typename T>
struct alignas(4 * sizeof(T)) vec4 {
  T x, y, z, w;
};

// Kernel kinds that need a block table.
enum KernelKind {
  K_ZFWD = 0,   // reaction + forward z transform (real -> half spectrum, transposed)
  K_YFWD,       // forward y transforms of M*, W*, V
  K_XPASS,      // x transform, spectral solves / gradient multiplier, inverse x transform
  K_PLANE,      // y + x transforms, multipliers, inverses on whole k3 planes (small N)
  K_YINV,       // inverse y transforms (forms the y-derivative spectrum)
  K_ZINV,       // inverse z transform (half spectrum -> real), forms d3 v, writes fields
  K_PART,       // gather + Euler-Maruyama push + mass update + deposit
  K_DIAG,       // full reductions for the diagnostics (initialisation, read time)
  K_SCOUNT,     // binning: tile of every particle and its rank within the tile
  K_SSCAN,      // binning: tile and chunk offsets (one block per simulation)
  K_SSCATTER,   // binning: scatter particles into the sorted set
  K_COUNT
};

// Diagnostic accumulator slots (uint64 words; sums stored as float64 bit patterns).
// Layout of SimDesc::diag: kStripes accumulator copies of kStripeWords words, then the
// diagnostics of the latest read (D_COUNT words).
enum DiagSlot {
  D_SUM_A = 0, D_SUM_U, D_SUM_M,
  D_MIN_V, D_MIN_M, D_MIN_W, D_MAX_M, D_MAX_W, D_MIN_A, D_MAX_A, D_MIN_U,
  D_NAN, D_NEG_M, D_NEG_W,
  D_COUNT
};
constexpr int kStripes = 64;
constexpr int kStripeWords = 16;  // >= D_COUNT, 128 bytes
constexpr int kDiagResult = kStripes * kStripeWords;  // offset of the reduced diagnostics
constexpr int kDiagWords = kDiagResult + kStripeWords;

// Pointer kinds of a descriptor.  The host writes plain pointers.  Kernels read the same
// bytes as pointers into the global address space: a pointer loaded from memory is generic to
// the compiler, and generic accesses become flat instructions, which count on the LDS counter
// as well as the vector-memory one, so every wait for an LDS result would also wait for all
// global loads in flight.  (The host compilation pass only type-checks kernels; there both
// kinds are plain pointers.)
template <typename U> using HostPtr = U*;
#if defined(__HIP_DEVICE_COMPILE__)
template <typename U> using GlobalPtr = __attribute__((address_space(1))) U*;
#else
template <typename U> using GlobalPtr = U*;
#endif

// Device-visible description of one simulation.  All pointers point into its workspace.
template <typename T, template <typename> class Ptr>
struct SimDesc {
  int N, log2N;       // grid nodes per axis
  int64_t P;          // particles
  int rows_per_blk;   // z forward pass: rows (i1, i2) per block
  int rows_zinv;      // z inverse pass: rows per block (zinv_elems)
  int lines_per_blk;  // y passes: lines per block
  int cols_per_blk;   // x pass: i2 columns per block
  int flags;
  T L, inv_h;         // period, 1/h
  T inv_h3;           // 1/h^3
  T two_pi_over_L;
  T inv_n3;           // 1/N^3 (normalisation of a 3D transform round trip)
  T inv_n2;           // 1/N^2 (round trip of the y and z transforms only)
  T gz_scale;         // (2 pi / L) / N (plane path) or / N^2 (three-pass path): d3 v from SV
  int use_plane;      // y/x passes fused into the plane pass
  double dt, D_u, chi, D_m, D_w, alpha, beta, gamma;
  T noise_amp;        // sqrt(2 D_u dt)
  T drift;            // chi dt
  double h3;          // h^3 (mass sums)
  uint32_t seed_lo, seed_hi, sim_lo, sim_hi;
  int mult_kind;      // 0 implicit, 1 separable tables (exp / aliased)
  int use_lowpass;
  int ntile1;         // tiles per axis, max(1, N / kTile)
  int ntiles;         // ntile1^3
  int use_region;     // LDS tile regions (N >= 2 tile sides, so a region never aliases itself)
  int dim;            // 3, or 2 for the two-dimensional form (z arrays unused)
  int64_t nrows;      // rows of N nodes along the last axis: N^(dim-1)
  int64_t G;          // grid nodes N^dim
  T inv_nd;           // 1 / N^dim
  int deposit_order;  // 2: trilinear assignment; 4: fourth-order assignment
  // particles, structure of arrays; set 0 is the state, set 1 receives the binned copy
  Ptr<T> xs[2], ys[2], zs[2];
  Ptr<double> as[2];
  Ptr<uint32_t> ids[2];  // particle index: keys the noise stream, restores the input order
  // binning
  Ptr<uint32_t> tcount;  // ntiles: particles per tile (zero between binnings)
  Ptr<uint32_t> toff;    // ntiles + 1: first sorted index of each tile
  Ptr<uint32_t> coff;    // ntiles + 1: first chunk of each tile
  Ptr<uint4> cinfo;      // max_chunks: (first particle, end, tile, -) of each chunk (set at
                         // binning, so a particle-pass block needs one lookup)
  int max_chunks;     // bound on the number of chunks: ceil(P / kChunk) + ntiles
  Ptr<uint32_t> key;     // 2P words: the binning's rank within the tile of each particle
                         // (first P), resampling's 64-bit prefix sums (all 2P)
  // grid (real, N^3 row-major)
  Ptr<T> v, m, w;
  // Deposited density and gather array, two buffers each, chosen by the parity of the step
  // index n: the particle pass of step n gathers from g4[n & 1] = (d1 v^n, d2 v^n, d3 v^n,
  // w^n) and deposits ubar^{n+1} into ubar[(n + 1) & 1], while the field passes of the same
  // step read ubar^n from ubar[n & 1] and write the next gather array into g4[(n + 1) & 1].
  // The two halves of a step share no buffer and run side by side.
  Ptr<T> ubar[2];
  Ptr<vec4<T>> g4[2];
  // spectra, half-spectrum layout S[k3][i1][i2], k3 in [0, N/2]
  Ptr<cplx<T>> SM, SW, SV, SGx, SGy;
  Ptr<cplx<T>> SVg;      // V spectrum the y and z derivatives are formed from: SV, or with the
                         // low-pass filter its filtered copy (a sixth spectrum buffer)
  Ptr<cplx<T>> tw;       // exp(-2 pi i k / N), k < N/2
  Ptr<T> mtab;           // separable multiplier tables: [field m | field w | lowpass] x N each
  Ptr<uint64_t> step;    // absolute step index n (device-resident, advanced once per step)
  Ptr<unsigned long long> diag;  // kDiagWords words, see DiagSlot
};

template <typename T> using SimDev = SimDesc<T, HostPtr>;    // host side
template <typename T> using SimK = SimDesc<T, GlobalPtr>;     // kernel side

template <typename T>
struct Batch {
  const SimDev<T>* sims;  // device array of nsims descriptors
  const int* blk;         // device array: K_COUNT tables of (nsims + 1) block offsets
  int nsims;
};

// Workgroups are handed to the eight XCDs round-robin by id (id mod 8), and each XCD has an
// L2 of its own.  xcd_block<RUN> permutes the ids of every full group of 8 RUN workgroups so
// that RUN consecutive logical blocks run on one XCD, one after another: passes whose
// neighbouring blocks touch the same cache lines (at N >= 256 the z and x passes read and
// write runs of half a line per block) then meet those lines in one L2.  The ids past the
// last full group are kept.
// Measured (float32 unless noted; 1 = ids as dispatched): the field passes and the binning
// with runs of 16 took 256^3 / 2^25 from 1553 to 1487 us per step and the 2D example at
// 1024^2 from 165 to 147 us (row passes at N = 1024), 128^3 unchanged; runs of 8 chunks of
// the particle pass (chunks of one tile stage the same region) a further 680 -> 647 us at
// 256^3 and 145 -> 143 us (float32), 267 -> 263 us (float64) at 128^3.  Contiguous ranges
// per XCD instead of runs unbalanced the particle pass (145 -> 237 us).
constexpr int kFieldRun = 16;  // field passes and binning
constexpr int kPartRun = 8;    // particle passes

template <int RUN>
__device__ __forceinline__ int xcd_block() {
  static_assert(RUN >= 1 && (RUN & (RUN - 1)) == 0, "RUN must be a power of two");
  const int b = (int)blockIdx.x;
  if (RUN == 1) return b;
  constexpr int G = 8 * RUN;
  if (b >= (int)(gridDim.x & ~(unsigned)(G - 1))) return b;
  return (b & ~(G - 1)) | ((b & 7) * RUN) | ((b >> 3) & (RUN - 1));
}

template <int RUN = 1, typename T>
__device__ __forceinline__ int find_sim(const Batch<T>& b, int kind, int& local_block) {
  const int* off = b.blk + kind * (b.nsims + 1);
  int lo = 0, hi = b.nsims;  // invariant: off[lo] <= bid < off[hi]
  const int bid = xcd_block<RUN>();
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= bid) lo = mid; else hi = mid;
  }
  local_block = bid - (lo ? off[lo] : 0);  // off[0] is always 0
  return lo;
}

// Descriptor of simulation s as kernels read it: through the constant address space.  The
// descriptor is never written while a kernel runs.  Read through a plain reference, its
// fields would be reloaded after every float or double store of the kernel (type-based alias
// analysis cannot separate those stores from the descriptor's own fields), and each reload
// would be followed by a wait for all outstanding memory accesses.  Constant-space loads are
// invariant: each field is loaded once, into scalar registers.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> using SimC = __attribute__((address_space(4))) const SimK<T>;
#else
template <typename T> using SimC = const SimK<T>;
#endif

template <typename T>
__device__ __forceinline__ SimC<T>& sim_view(const Batch<T>& b, int s) {
  return *(SimC<T>*)(b.sims + s);
}

// ---- complex arithmetic -------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }

__device__ __forceinline__ int bitrev(int j, int log2n) {
  return (int)(__brev((unsigned)j) >> (32 - log2n));
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ----------------------------------------
// Round: multiply words 0 and 2 by the Philox multipliers into 64-bit products, new counter
// (hi(c2 M1) ^ c1 ^ k0, lo(c2 M1), hi(c0 M0) ^ c3 ^ k1, lo(c0 M0)); the key advances by the
// Weyl increments between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
}

// ---- ordered 64-bit keys for float64 min / max via integer atomics ------------------------
__device__ __forceinline__ unsigned long long order_key(double d) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(d);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// ---- launchers (defined in fft.hip, particles.hip, diag.hip) ------------------------------
template <typename T> int elems_per_block();
// Elements per block of the z inverse pass: at N <= 128 float32 blocks of 1024 elements (half
// the forward pass's; more blocks share a CU), which pays while a block's runs along a
// spectrum row stay a full 64 bytes (8 rows); at N >= 256 they would be shorter, so the pass
// keeps 2048.
// Most elements a z inverse block holds: its threads keep every element's w (and, for the
// float32 solves in change form, m* and w* before the transforms) in registers, 8 per thread
// (ZBatch x ZBatches in fft.hip).
constexpr int zinv_max_elems() { return 8 * kThreads; }
template <typename T> inline int zinv_elems(int N) {
  return sizeof(T) == 4 && N <= 128 ? 1024 : elems_per_block<T>();
}
// Fewest rows per block of the z forward pass (rows come in pairs): two; four for float64
// rows of 1024 nodes (the 2D form's largest grid), where two rows left most of a block's
// threads without a sub-transform (row pass 36.7 -> 27.7 us at 1024^2); and at N = 256 the
// rows of 128 bytes of spectrum row per plane, so that a block writes whole cache lines
// instead of halves (float64, eight rows: z forward pass 285 -> 265 us at 256^3; float32,
// sixteen rows: the pass itself 139.5 -> 144.3 us, but the z inverse pass of the same step
// 230.3 -> 224.6 us and the step 1317.5 -> 1308.8 us, two runs each).
template <typename T> inline int zfwd_min_rows(int lg) {
  if (lg == 8) return 128 / (int)(2 * sizeof(T));
  return lg == 10 && sizeof(T) == 8 ? 4 : 2;
}
// Elements per block of the x pass (columns of N points): 2048 in both precisions, so that a
// float64 block still moves runs of 16 consecutive columns (256 bytes) at N = 128.  The 2D
// column pass at N = 1024 (log2 N = 10, two-dimensional only) takes kXpassElems1024: with
// two 1024-point lines per block only 64 threads have a sub-transform to run.
constexpr int kXpassElems = 2048;
constexpr int kXpassElems1024 = 4096;
inline int xpass_elems(int lg) { return lg == 10 ? kXpassElems1024 : kXpassElems; }
template <typename T> void block_counts(const SimDev<T>& d, int counts[K_COUNT]);

// Field passes.  mode 0: the field half of a step; mode kGradOnly: only the gather array of
// the current state (the gradient of v^n and w^n into g4[n & 1]; m, v, w, ubar and the
// diagnostics untouched), for initialisation.  The y and x passes do the same in both modes.
constexpr int kGradOnly = 1;
template <typename T> void launch_zfwd(const Batch<T>& b, int nblk, int lg, hipStream_t s,
                                       int mode);
template <typename T> void launch_yfwd(const Batch<T>& b, int nblk, int lg, hipStream_t s,
                                       int mode);
template <typename T> void launch_xpass(const Batch<T>& b, int nblk, int lg, hipStream_t s,
                                        int mode);
template <typename T> void launch_yinv(const Batch<T>& b, int nblk, int lg, hipStream_t s,
                                       int mode);
template <typename T> void launch_zinv(const Batch<T>& b, int nblk, int lg, hipStream_t s,
                                       int mode);
template <typename T>
void launch_plane(const Batch<T>& b, int nblk, int lg, hipStream_t s, int configure);
template <typename T> bool plane_fits(int lg);
template <typename T> void configure_fft(int lg);
template <typename T>
void launch_particles(const Batch<T>& b, int nblk, int src_set, int deposit_only, int order,
                      int dim, hipStream_t s);
template <typename T>
void configure_particles(int order, int dim);

// ---- residual resampling (resample.hip) ---------------------------------------------------
// words (uint64) at the start of the resampling scratch area
enum RsWord {
  RS_MAXBITS = 0,  // bit pattern of the largest mass (non-negative doubles order as integers)
  RS_FLAGS = 1,    // RS_BAD_* bits
  RS_DIGITS = 2,   // 8 words: fixed-point sum of the masses
  RS_A0 = 10,      // bit pattern of a0
  RS_KTOT = 11,    // sum_p k_p
  RS_RTOT = 12,    // sum_p R_p
  RS_BLOCKS = 16,  // (sum k, sum R) per scan block, then their exclusive prefix
};
constexpr unsigned long long RS_BAD_VALUE = 1;  // a mass that is negative or not finite
constexpr unsigned long long RS_BAD_RANGE = 2;  // masses beyond the exact sum's range
size_t resample_scratch_words(int64_t P);
// largest mass, exact sum and a0 (reads set 0, leaves set 0 untouched; set 1 := set 0 in
// particle order); scratch words 0 .. RS_BLOCKS - 1 must be zero on entry
template <typename T>
void launch_resample_stats(const SimDev<T>& d, unsigned long long* rs, hipStream_t s);
// copy counts, prefix sums and the resampled list into set 0 (particle order)
template <typename T>
void launch_resample_apply(const SimDev<T>& d, unsigned long long* rs, hipStream_t s);
template <typename T>
void launch_binning(const Batch<T>& b, const int* tot, int nsims, int dim, hipStream_t s);
// diagnostics of the current state: full reduction into the result words (read time)
template <typename T> void launch_diag_read(const Batch<T>& b, int nblk, int nsims, hipStream_t s);
// end of a step: advance the step index
template <typename T> void launch_finalize(const Batch<T>& b, int nsims, hipStream_t s);
template <typename T> void launch_diag_clear(const Batch<T>& b, int nsims, hipStream_t s);

// LDS bytes the FFT kernels need (host side, for launch configuration).
template <typename T> size_t fft_lds_bytes(int kind, int lg);

}  // namespace sipf
