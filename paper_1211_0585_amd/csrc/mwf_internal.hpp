// Internal definitions shared by the host runtime and the HIP kernels of libmwf.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mwf.h"

namespace mwf {

// ---------------------------------------------------------------- error handling
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define MWF_HIP(expr)                                                         \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return ::mwf::fail(WF_EDEVICE, std::string(#expr) + ": " +             \
                                         hipGetErrorString(e_));              \
  } while (0)

// ---------------------------------------------------------------- geometry
// One iso-latitude ring pair: north ring i (1-based, i <= 2 nside) and its
// mirror 4 nside - i in the south. Pair index q counts from the equator
// (q = 0 is the equator ring, which has no partner) towards the north pole
// (q = 2 nside - 1 is ring 1), so that rings near the poles, where the
// Legendre functions of high m vanish, form a contiguous tail.
struct RingPair {
  double z;          // cos(theta) of the north ring
  double sin_t;      // sin(theta)
  int64_t start_n;   // first pixel of the north ring (RING order)
  int64_t start_s;   // first pixel of the south ring, -1 for the equator
  int32_t nphi;      // pixels per ring (same for both rings)
  int32_t log2n;     // log2(nphi) if nphi is a power of two, else -1
  int32_t ph_num;    // longitude of pixel 0 = pi * ph_num / ph_den
  int32_t ph_den;
  int32_t bl_M;      // Bluestein convolution length (0 for power-of-two and mixed-radix rings)
  int32_t mix;       // mixed-radix rings (nphi = 2^a 3^b 5^c 7^d, not a power of two):
                     // b | c << 4 | d << 8, the odd passes after the radix-2/4/8 ones; else 0
  int64_t bl_off;    // Bluestein rings: offset (complex entries) of this length's filter in the
                     // Bluestein table; mixed-radix rings: of exp(-2 pi i t / nphi), t < nphi,
                     // in the mixed-radix table
  int64_t chirp_off; // offset (complex entries) of this length's chirp exp(-i pi j^2 / n)
};

// Odd radix passes of an n-point mixed-radix ring transform: n = 2^a o with o > 1 a product
// of 3, 5 and 7 only (returns the packed counts b | c << 4 | d << 8), else 0 (a power of two,
// or a prime factor above 7: Bluestein).
__host__ __device__ inline int32_t mixed_radix_passes(int n) {
  int o = n;
  while (o > 1 && (o & 1) == 0) o >>= 1;
  if (o == 1) return 0;
  int c[3] = {0, 0, 0};
  const int r[3] = {3, 5, 7};
  for (int k = 0; k < 3; ++k)
    while (o % r[k] == 0) {
      o /= r[k];
      c[k] += 1;
    }
  return o == 1 ? (c[0] | c[1] << 4 | c[2] << 8) : 0;
}

// Scaling of the Legendre recurrence: a value is carried as v * 2^(-SCALE_BITS * s)
// with an integer s >= 0. While s > 0 the value is below 2^(64 - SCALE_BITS)
// and contributes nothing; it is rescaled (s -= 1) when |v| exceeds 2^64.
constexpr int SCALE_BITS = 512;
constexpr int CHUNK = 16;            // l-steps per reduction chunk in phase A (FP64 path)
constexpr int MCH = 32;              // l-steps per staged chunk on the matrix-core path
constexpr int ROW_PAD = 64;          // zero padding after each per-m row of A / C / coefficients
constexpr int LANES = 64;            // wavefront width on CDNA
// FP64 Legendre launches: work items packed at plan time into FP64_WAVES_PER_SIMD
// bins per SIMD, one wave per bin, by estimated cost in steps of l: a step costs 1,
// or FP64_SCALED_COST_{ANA,SYN} / 4 while a ring of the item is still scaled (the
// rescale path runs once per chunk: 16 steps in the analysis, 8 in the synthesis),
// and an item FP64_ITEM_COST_L more for its set-up. (Weights from timing the kernels.)
constexpr int FP64_WAVES_PER_SIMD = 3;
constexpr int FP64_SCALED_COST_ANA = 5;
constexpr int FP64_SCALED_COST_SYN = 6;
constexpr int FP64_ITEM_COST_L = 32;
constexpr uint16_t WAKE_NEVER = 0xffff;

// lambda_mm(z) = norm_m sin^m(theta) as v * 2^(-512 s) with |v| >= 2^-449 when s = 0.
__device__ __forceinline__ void sectoral_seed(int m, double sin_t, double norm, double* v, int* s) {
  int eb;
  double b = frexp(sin_t, &eb);
  double r = 1.0;
  int er = 0;
  int k = m;
  while (k) {
    if (k & 1) {
      int t;
      r = frexp(r * b, &t);
      er += eb + t;
    }
    k >>= 1;
    if (k) {
      int t;
      b = frexp(b * b, &t);
      eb = 2 * eb + t;
    }
  }
  int t;
  double x = frexp(norm * r, &t);
  const int e = er + t;                 // value = x * 2^e, 0.5 <= |x| < 1
  int sc = 0;
  if (e < 64 - SCALE_BITS) sc = (64 - SCALE_BITS - e + SCALE_BITS - 1) / SCALE_BITS;
  *v = ldexp(x, e + SCALE_BITS * sc);
  *s = sc;
}

// Work item of the m-parallel phase: one m and one block of ring pairs.
struct WorkItem {
  int32_t m;
  int32_t blk;
};

// Everything the kernels need, passed by value.
struct PlanDev {
  int32_t nside, lmax, npairs, nrings;
  int64_t npix, nalm;
  double tau, omega;
  int32_t ring_block_ana;    // ring pairs per Legendre-analysis work item (64 * R)
  int32_t ring_block_syn;    // ring pairs per Legendre-synthesis work item (64 * R)
  int32_t nblk_max;          // max analysis blocks per m (partial sums per m)
  int32_t pad0_;
  const RingPair* pairs;     // [npairs]
  const void* q;             // [npix] tau * ninv (observed) or 0, in the storage type
  const double* cl;          // [lmax+1]
  const double* A;           // recurrence coefficients, padded rows (see row_off)
  const double* C;           // lambda = C * mu
  const int64_t* row_off;    // [lmax+1] start of row m in A / C (row length lmax-m+1+ROW_PAD)
  const double* norm_m;      // [lmax+1] signed sectoral normalisation
  const int32_t* n_active;   // [lmax+1] ring pairs with non-negligible lambda_lm
  const int32_t* nblk;       // [lmax+1] analysis blocks of m
  const double2* twiddle;    // exp(-2 pi i k / tw_len), k < tw_len / 2
  int32_t tw_len;
  int32_t pad_;
  const double2* bluestein;  // FFT_M of the Bluestein chirp filter per distinct length
  const double2* chirp;      // exp(-i pi j^2 / n) per distinct Bluestein length
  const float2* twiddle32;   // the same three tables rounded to float (FP32 plans)
  const float2* chirp32;
  const float2* bluestein32;
  const double2* mixtw;      // exp(-2 pi i t / n), t < n, per distinct mixed-radix ring length n
  const float2* mixtw32;
  int64_t rows_total;        // length of the padded per-m row layout of A / C / bcoef
  const int32_t* row_m;      // [rows_total] m of each padded row
};

// Elements per ring pair in the G and F buffers ([map][pair][m][E re, E im, O re, O im]):
// 4 per m <= lmax, unpadded. (Rows padded to whole 128-byte lines made the per-map stride a
// multiple of 2^17 bytes at Nside 512, and the matrix-core Legendre kernels ran 12-18 %
// slower on it despite fetching fewer lines.)
__host__ __device__ inline size_t gf_stride(int lmax) { return (size_t)(lmax + 1) * 4; }

__host__ __device__ inline int64_t alm_index(int lmax, int l, int m) {
  return (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
}

// ---------------------------------------------------------------- kernel launchers
// Phase B (ring-parallel): synthesis ring FFTs, messenger update (Eq. 3), analysis FFTs.
enum PhaseBMode : int32_t {
  PB_SYNTH = 1,       // read F (E/O per m), inverse ring DFT
  PB_UPDATE = 2,      // t = s + w (d - s)
  PB_ANALYSIS = 4,    // forward ring DFT, write G (S/D per m)
  PB_WRITE_MAP = 8,   // write the synthesised map (before the update)
  PB_READ_MAP = 16,   // take the ring values from `map_in` instead of a synthesis
  PB_CHI2 = 32        // with PB_SYNTH and a chi2 pointer: read d and tau N^-1 for the data term
};

// Pointers are in the plan's storage type (double, or float for the FP32 / BF16x3 paths).
// Per-map parameters of a batch whose maps are independent requests (serving):
// each map has its own lambda, lambda tau Omega (filter denominator term), phase-B
// mode (0 = slot idle) and its own rows of tau N^-1 and C_l.
struct SlotParam {
  double lambda;
  double lam_t_o;
  int32_t pb_mode;
  int32_t pad_;
};

struct PhaseBArgs {
  int32_t mode;
  int32_t nmaps;
  double lambda;
  const void* F;          // [map][pair][m][4]
  void* G;                // [map][pair][m][4]
  const void* d;          // [map][npix]
  const void* map_in;     // [map][npix]
  void* map_out;          // [map][npix]
  const SlotParam* slots; // null: mode, lambda and P.q shared by all maps
  int64_t q_stride;       // with slots: elements between the tau N^-1 rows of two maps
  double* chi2;           // null, or where map 0 adds sum tau N^-1 (d - s)^2 of the synthesised s
  int64_t chi2_stride;    // doubles between the chi2 entries of two maps
};

// Sum of v over each wave, added to *dst by one FP64 atomic per wave (no LDS: the
// ring phase of the longest FP64 transforms uses all of it). Every lane of the wave
// must call it.
// A chi^2 term is accumulated in CHI_SLOTS partial sums, each on its own 128-byte
// line, so that the atomics of many workgroups do not all queue on one address;
// readers add the slots in order. A record holds the prior term's slots, then the
// data term's.
constexpr int CHI_SLOTS = 16;
constexpr int CHI_SLOT_STRIDE = 16;                   // doubles between slots
constexpr int CHI_TERM = CHI_SLOTS * CHI_SLOT_STRIDE;  // doubles per term
constexpr int CHI_REC = 2 * CHI_TERM;                  // doubles per iterate

// Sum of v over the workgroup (blockDim.x a multiple of 64, at most 1024, every
// thread present, at most one call per kernel), added to slot blockIdx.x % CHI_SLOTS
// of the term at dst by one atomic.
__device__ __forceinline__ void block_sum_add(double v, double* dst) {
  __shared__ double wsum[16];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wsum[w];
    if (t != 0.0) atomicAdd(dst + (blockIdx.x % CHI_SLOTS) * CHI_SLOT_STRIDE, t);
  }
}

// Ring pairs launched together: a device list of pair indices and the largest
// transform length among them (power-of-two n, the Bluestein M, or a mixed-radix n, which
// counts twice in the class lists and once in the split launches of a plan).
struct RingClass {
  const int32_t* q;
  int32_t count;
  int32_t fft_len;
};

// Ring launches: class 0 rings that are not a power of two (Bluestein and mixed radix,
// 512 threads) and class 1 power-of-two rings (256 threads), class 2 transforms of at
// most 1024 points (one wave per ring pair; used from RING_SPLIT_MAPS maps on, when
// classes 0 and 1 hold only the longer transforms).
constexpr int NRING_CLASSES = 3;
constexpr int RING_SPLIT_MAPS = 4;

// Pass schedule of the in-place Stockham FFT of 2^lg points (lg >= 1): n2 radix-2,
// n4 radix-4 and n8 radix-8 passes in that order (radix 8 as far as lg allows).
__host__ __device__ inline void fft_schedule(int lg, int* n2, int* n4, int* n8) {
  *n8 = lg / 3;
  *n4 = 0;
  *n2 = 0;
  if (lg % 3 == 2) {
    *n4 = 1;
  } else if (lg % 3 == 1) {
    if (*n8 > 0) {
      *n8 -= 1;
      *n4 = 2;
    } else {
      *n2 = 1;
    }
  }
}

// Entries of one per-pass twiddle table set of a 2^lg-point FFT: the sum of Ns over
// the passes that multiply by twiddles (Ns > 1), Ns the points combined before the pass.
__host__ __device__ inline int fft_twiddle_entries(int lg) {
  int n2, n4, n8;
  fft_schedule(lg, &n2, &n4, &n8);
  int ns = 1, e = 0;
  for (int p = 0; p < n2; ++p, ns *= 2) e += ns > 1 ? ns : 0;
  for (int p = 0; p < n4; ++p, ns *= 4) e += ns > 1 ? ns : 0;
  for (int p = 0; p < n8; ++p, ns *= 8) e += ns > 1 ? ns : 0;
  return e;
}

// Points of the FFT buffer in LDS including the padding of the layout between
// passes (one element after every 16).
__host__ __device__ inline int fft_padded(int len) { return len + (len >> 4); }

// Dynamic LDS of a ring launch: the padded data of fft_len points plus the twiddle
// table of its passes (w per pass; the powers of w are formed by products). (At
// least 8 KiB: short rings stage 512 partial sums of two complex doubles.)
inline size_t ring_lds_bytes(int fft_len, size_t elem) {
  int lg = 0;
  while ((1 << lg) < fft_len) ++lg;
  const size_t b = ((size_t)fft_padded(fft_len) + (size_t)fft_twiddle_entries(lg)) * elem;
  return b < 8192 ? 8192 : b;
}

// cls: NRING_CLASSES classes, launched in order (empty ones skipped).
// Zero `bytes` (a multiple of 16, 16-byte aligned) at p on s with a kernel.
hipError_t launch_zero_fill(void* p, size_t bytes, hipStream_t s);
hipError_t launch_phase_b(const PlanDev& P, const PhaseBArgs& a, const RingClass* cls, bool fp32, hipStream_t s);
// One class alone (cls: its index, which fixes the workgroup size).
hipError_t launch_phase_b_class(const PlanDev& P, const PhaseBArgs& a, const RingClass& rc, int cls, bool fp32,
                                hipStream_t s);

// Phase A (m-parallel): Legendre analysis into per-block partial sums. One wave per
// bin: wave w runs items[bins[w] .. bins[w + 1]) (nbins bins).
hipError_t launch_legendre_analysis_f64(const PlanDev& P, const WorkItem* items, const int32_t* bins,
                                        int nbins, int nmaps, const double* G, double2* partial,
                                        hipStream_t s);

enum SynthMode : int32_t {
  SY_FROM_PARTIAL = 0,   // a = C sum(partials); s = f(lambda) a; synthesise s
  SY_FROM_ALM = 1,       // synthesise the caller's alm
  SY_ALM_ONLY = 2        // a = C sum(partials) -> alm output, no synthesis
};

struct SynthArgs {
  int32_t mode;
  int32_t nmaps;
  double lambda;
  const double2* partial;   // [map][blk][nalm]
  const double2* alm_in;    // [map][nalm]
  double2* alm_out;         // [map][nalm] or null
  double2* bcoef;           // [map][rows_total] C_l s_lm in the padded row layout
  double* F;                // [map][pair][m][4]
  double* chi2;             // null, or where map 0 adds sum_lm w_m |s_lm|^2 / C_l (SY_FROM_PARTIAL)
  int64_t chi2_stride;
};

// Sum of partials, filter and C scaling (one launch over all (l, m, map)).
hipError_t launch_legendre_coeff(const PlanDev& P, const SynthArgs& a, hipStream_t s);
hipError_t launch_legendre_synthesis_f64(const PlanDev& P, const WorkItem* items, const int32_t* bins,
                                         int nbins, const SynthArgs& a, hipStream_t s);

// Matrix-core (FP32 / BF16x3) Legendre phase for batches stored in float.
// Threads per workgroup of the matrix-core coefficient kernel (one element each).
constexpr int COEFF_THREADS = 256;

// Ring pairs per block of the matrix-core analysis with ct column tiles per
// workgroup (2 ct waves): 128 for one tile, 256 from two on (from four tiles on,
// the first four waves generate the Legendre values that all waves contract).
constexpr int ana_block(int ct) { return ct == 1 ? 128 : 256; }
// Column tiles a matrix-core analysis workgroup may take: 1, 2, 4, 8 (8: FP32 only).
constexpr bool ana_ct_valid(int ct, bool fp32) { return ct == 1 || ct == 2 || ct == 4 || (ct == 8 && fp32); }

struct MfmaArgs {
  int32_t mode;             // SynthMode of the coefficient step
  int32_t nmaps;
  double lambda;
  int32_t ana_rb;           // ring pairs per analysis block (128 or 256): partial blocks per m
  int32_t pad_;
  const float* G;           // [map][pair][m][4]
  float* F;                 // [map][pair][m][4]
  float* partial;           // [blk of 256 pairs][nalm][nmaps][2]
  float* bcoef;             // [rows_total][nmaps][2]
  const float2* alm_in;     // [map][nalm]
  float2* alm_out;          // [map][nalm] or null
  const SlotParam* slots;   // null: lambda and P.cl, P.tau shared by all maps
  int64_t cl_stride;        // with slots: entries between the C_l rows of two maps
  double* chi2;             // as SynthArgs::chi2
  int64_t chi2_stride;
};

// ct: column tiles (16 columns) per analysis workgroup, 1 or 2 (ring block 128 ct);
// nct: column tiles per synthesis wave, 1, 2 or 4.
hipError_t launch_mfma_analysis(const PlanDev& P, const WorkItem* items, int nitems, int mode, int ct,
                                const MfmaArgs& a, hipStream_t s);
hipError_t launch_mfma_coeff(const PlanDev& P, const MfmaArgs& a, hipStream_t s);
hipError_t launch_mfma_synthesis(const PlanDev& P, const WorkItem* items, int nitems, int mode, int nct,
                                 const MfmaArgs& a, hipStream_t s);
// Wide synthesis: items of 256 ring pairs, 32 nt columns per workgroup (nt = 1 or 2; see
// phase_a_mfma.hip).
hipError_t launch_mfma_wide_synthesis(const PlanDev& P, const WorkItem* items256, int nitems, int mode, int nt,
                                      const MfmaArgs& a, hipStream_t s);

// One entry of a task group: a plan's tables and buffers, its maps and its lambda for
// this step. Groups run every task of a step in one launch per phase.
struct TaskDev {
  PlanDev P;
  int32_t nmaps;
  int32_t pb_mode;          // PhaseBMode bits
  int32_t sy_mode;          // SynthMode
  int32_t pad_;
  double lambda;
  void* G;
  void* F;
  const void* d;
  const void* map_in;
  void* map_out;
  float* partial;
  float* bcoef;
  const float2* alm_in;
  float2* alm_out;
  const WorkItem* items_a128;   // analysis items for 128- and 256-pair blocks
  const WorkItem* items_a256;
  const WorkItem* items_s64;    // synthesis items (64 pairs)
  const SlotParam* slots;       // per-map parameters (serving lanes) or null
  int64_t q_stride;
  int64_t cl_stride;
  const int32_t* ring_q[NRING_CLASSES];   // ring pairs of each ring launch class
  int32_t ring_n[NRING_CLASSES];
};

// One phase of a task group, described on the host: the tasks and, per task, the
// first block of the launch (offs[t] <= block < offs[t + 1], offs[ntasks] blocks).
struct GroupLaunch {
  const TaskDev* tasks;     // host
  const int64_t* offs;      // host, ntasks + 1 block offsets
  int32_t ntasks;
  int32_t pad_;
  int64_t nblocks;
};

// What a group kernel receives, by value: up to GROUP_MAX_TASKS tasks and their block
// offsets (relative to the launch). Passing the task entries as kernel arguments,
// not through a device table, lets the compiler treat their pointers as global and
// emit global rather than flat memory instructions; it also needs no upload. A
// group with more tasks is launched in several parts.
constexpr int GROUP_MAX_TASKS = 8;
struct GroupArgs {
  TaskDev t[GROUP_MAX_TASKS];
  int64_t offs[GROUP_MAX_TASKS + 1];
  int32_t ntasks;
  int32_t pad_;
};
static_assert(sizeof(GroupArgs) <= 3584, "group kernel arguments must stay well under 4 KiB");

// The task of block b: offs[t] <= b < offs[t + 1].
__device__ __forceinline__ int group_task_of(const GroupArgs& g, int64_t b) {
  int lo = 0, hi = g.ntasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.offs[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Launches a phase of a group in parts of at most GROUP_MAX_TASKS tasks:
// launch(args, nblocks) for each part with blocks.
template <class F>
hipError_t for_each_group_part(const GroupLaunch& g, F launch) {
  for (int t0 = 0; t0 < g.ntasks; t0 += GROUP_MAX_TASKS) {
    const int n = g.ntasks - t0 < GROUP_MAX_TASKS ? g.ntasks - t0 : GROUP_MAX_TASKS;
    GroupArgs a{};
    a.ntasks = n;
    for (int i = 0; i < n; ++i) a.t[i] = g.tasks[t0 + i];
    for (int i = 0; i <= n; ++i) a.offs[i] = g.offs[t0 + i] - g.offs[t0];
    if (a.offs[n] == 0) continue;
    if (hipError_t e = launch(a, a.offs[n])) return e;
  }
  return hipSuccess;
}

hipError_t launch_group_analysis(const GroupLaunch& g, int mode, int ct, hipStream_t s);
hipError_t launch_group_coeff(const GroupLaunch& g, int ana_rb, hipStream_t s);
hipError_t launch_group_synthesis(const GroupLaunch& g, int mode, int nct, int ana_rb, hipStream_t s);
// Ring phase over (task, ring pair, map) blocks, float storage and arithmetic.
// Ring launch of class cls over TaskDev::ring_q[cls]; fft_len: the longest transform of the class.
hipError_t launch_group_phase_b(const GroupLaunch& g, int cls, int fft_len, hipStream_t s);

// ---------------------------------------------------------------- polarisation (T, Q, U)
// A polarised problem runs three fields per map. Ring coefficients are stored field
// by field, [field][map][pair][m][4] with field_maps maps per field block (the plan's
// max_batch), so the T block is an ordinary spin-0 buffer; maps and d are
// [map][field][npix]; tau N^-1 is [6][npix] (TT, QQ, UU, TQ, TU, QU).
struct PolRingArgs {
  int32_t mode;          // PhaseBMode bits (PB_SYNTH, PB_UPDATE, PB_ANALYSIS, PB_WRITE_MAP, PB_READ_MAP)
  int32_t nmaps;
  int32_t field_maps;    // maps per field block of F and G
  int32_t pad_;
  double lambda;
  const double* F;
  double* G;
  const double* d;
  const double* map_in;
  double* map_out;
  const double* q6;
};
// The ring launch classes 0 and 1 of a polarised plan (512 threads).
hipError_t launch_pol_ring(const PlanDev& P, const PolRingArgs& a, const RingClass* cls, hipStream_t s);

// Spin-2 Legendre tables and work of a polarised plan (FP64). The functions
// u = s_lambda / K obey u_l = (A_l z + B_l s/2) u_{l-1} - u_{l-2} for s = +2 and -2
// (rows per m in the padded layout of the spin-0 tables; A = B = 0 at l <= l0 =
// max(m, 2), K = 0 below l0).
struct Spin2Dev {
  const double* A;       // [rows_total]
  const double* B;
  const double* K;
  const double* norm;    // [lmax+1] sqrt(m (m-1) / ((m+1)(m+2))) for m >= 2; m = 0, 1: sqrt(15/(32 pi)), sqrt(5/pi)
  const WorkItem* items; // (m, block of 64 ring pairs), longest first
  int32_t nitems;
  int32_t field_maps;    // maps per field block of F and G
};

// Polarised coefficient step: sums the T partials (spin-0 layout) and the E/B partials
// ([map][blk][nalm][4]: E re, E im, B re, B im), applies the TE-coupled 3x3 filter of
// Eq. (4) (SY_FROM_PARTIAL), or passes the transform (SY_ALM_ONLY) or the caller's alm
// (SY_FROM_ALM) through; writes alm_out [map][3][nalm] and the synthesis coefficients.
struct PolCoeffArgs {
  int32_t mode;
  int32_t nmaps;
  double lambda;
  const double2* partial_t;   // [map][nblk_max][nalm]
  const double* partial_eb;   // [map][nblk2][nalm][4]
  int32_t nblk2;              // blocks of 64 ring pairs (partials per (l, m) of E/B)
  int32_t pad_;
  const int32_t* nblk2_m;     // [lmax+1] E/B blocks written for m
  const double2* alm_in;      // [map][3][nalm]
  double2* alm_out;           // [map][3][nalm] or null
  double2* bcoef_t;           // [map][rows_total]: C_l s_T (spin-0 synthesis input)
  double2* bcoef_eb;          // [map][rows_total][2]: -K s_E / 2, -K s_B / 2
  const double* cl4;          // [4][lmax+1] TT, EE, BB, TE
};
hipError_t launch_pol_coeff(const PlanDev& P, const Spin2Dev& S2, const PolCoeffArgs& a, hipStream_t s);
hipError_t launch_spin2_analysis(const PlanDev& P, const Spin2Dev& S2, int nmaps, const double* G, double* partial_eb,
                                 int nblk2, hipStream_t s);
hipError_t launch_spin2_synthesis(const PlanDev& P, const Spin2Dev& S2, int nmaps, const double2* bcoef_eb, double* F,
                                  hipStream_t s);

// Plan-time, per (m, ring pair): where lambda_lm leaves the scaled range, or WAKE_NEVER
// (polar skip and the cost of the FP64 work items).
hipError_t launch_reach(const PlanDev& P, uint16_t* wake, hipStream_t s);

}  // namespace mwf
