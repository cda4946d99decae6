// Phase A of a messenger sweep: m-parallel work in harmonic space (FP64 VALU path).
//
// For each m the Legendre functions lambda_lm(z) of every ring pair are generated
// on the fly, l = m..lmax, by the three-term recurrence in FP64 and contracted
// against the ring Fourier coefficients:
//
//   analysis   a_lm = sum_pairs lambda_lm(z) (S if l-m even else D),  S/D = G_N +/- G_S
//   filter     s_lm = f_l(lambda) a_lm, f_l = C_l / (C_l + lambda tau Omega)     (Eq. 4)
//   synthesis  E = sum_{l-m even} lambda_lm s_lm, O = sum_{l-m odd} lambda_lm s_lm,
//              F_N = E + O, F_S = E - O
//
// using lambda_lm(-z) = (-1)^(l+m) lambda_lm(z) for the mirror rings.
//
// The recurrence runs on rescaled values mu_l = lambda_lm / C_lm that obey
//   mu_l = (A_lm z) mu_{l-1} - mu_{l-2}
// (A and C are plan-time FP64 tables derived from
//  a_lm = sqrt((4 l^2 - 1)/(l^2 - m^2)) with C_l = C_{l-2} a_l / a_{l-1}, A_l = a_l C_{l-1} / C_l),
// i.e. one multiply and one FMA per value; C is applied once per (l, m) after the
// ring sum (analysis) or folded into s_lm (synthesis).
//
// The sectoral seed lambda_mm = norm_m sin^m(theta) underflows FP64 near the
// poles: every value carries an integer scale s (value = v 2^(-512 s)). The scale
// is checked once per chunk of l (|v| > 2^64 with s > 0: v *= 2^-512, s -= 1);
// a ring whose scale is still positive at the start of a chunk contributes
// nothing in that chunk (its values are below 2^-448 times the growth of one
// chunk, far under FP64 resolution of the sums). The recurrence alternates
// between two registers, so a step is one multiply and one FMA and no moves.
//
// Each work item is (m, block of 64 R ring pairs) handled by one wavefront; a
// lane owns R ring pairs. The recurrence coefficients (and, in the synthesis, the
// filtered a_lm) are fetched 64 values of l ahead with one vector load and read
// from LDS. The analysis reduces over lanes through LDS once per chunk of 16
// values of l and writes one partial sum per block; a small kernel sums the
// partials of each (l, m), applies the filter and scales by C for the synthesis.
#include "mwf_internal.hpp"

namespace mwf {
namespace {

constexpr double BIG_THRESH = 0x1p64;
constexpr double RESCALE = 0x1p-512;

__device__ __forceinline__ int wave_any(int pred) { return __any(pred); }

// a + b over lanes l and l + 32 with the halves exchanged (v_permlane32_swap): lanes
// 0..31 return a[l] + a[l + 32], lanes 32..63 return b[l - 32] + b[l].
__device__ __forceinline__ double fold_halves(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

template <int R>
struct RingState {
  double z[R], mu1[R], mu2[R];
  int sc[R];
};

template <int R>
__device__ __forceinline__ void init_rings(const PlanDev& P, int m, int blk, int lane, int nact,
                                           RingState<R>& st) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = blk * (LANES * R) + r * LANES + lane;
    if (q < nact) {
      const RingPair rp = P.pairs[q];
      double v;
      int s;
      sectoral_seed(m, rp.sin_t, P.norm_m[m], &v, &s);
      st.z[r] = rp.z;
      st.mu1[r] = 0.0;    // mu_{m-1}
      st.mu2[r] = -v;     // with A_mm = 0 the first step yields mu_m = v
      st.sc[r] = s;
    } else {
      st.z[r] = 0.0;
      st.mu1[r] = 0.0;
      st.mu2[r] = 0.0;
      st.sc[r] = 0;
    }
  }
}

// Once per chunk: bring large scaled values back by 2^-512. Returns a bit mask of
// the rings whose scale reached zero in this call.
template <int R>
__device__ __forceinline__ int rescale_chunk(RingState<R>& st) {
  int woke = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (st.sc[r] > 0 && fmax(fabs(st.mu1[r]), fabs(st.mu2[r])) > BIG_THRESH) {
      st.mu1[r] *= RESCALE;
      st.mu2[r] *= RESCALE;
      st.sc[r] -= 1;
      if (st.sc[r] == 0) woke |= 1 << r;
    }
  }
  return woke;
}

constexpr int LTILE = 64;  // values of l per prefetched coefficient tile (one per lane)

// FP64 Legendre launches: workgroups of FP64_WG_WAVES waves, one bin each, so that
// every SIMD of a CU gets the same number of waves (with single-wave workgroups
// the spread over a CU's SIMDs depends on what ran before: after a ring phase of
// three concurrent launches, some SIMDs got four waves and some two, and the
// launch took a third longer).
constexpr int FP64_WG_WAVES = 4;

// Orders a wave's LDS accesses around it (one wave's LDS operations execute in
// order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }
constexpr int ACH = 16;    // analysis: values of l per cross-lane reduction (and scale check)
static_assert(LTILE % ACH == 0 && (2 * ACH) <= LANES, "analysis chunking");

template <int R>
__global__ void __launch_bounds__(FP64_WG_WAVES * LANES) legendre_analysis_f64_kernel(
    PlanDev P, const WorkItem* __restrict__ items, const int32_t* __restrict__ bins, int nbins,
    const double* __restrict__ G, double2* __restrict__ partial) {
  // per-wave LDS: the waves of a workgroup run unrelated bins and never synchronise
  __shared__ double red_w[FP64_WG_WAVES][2 * ACH][LANES / 2 + 1];
  __shared__ double sA_w[FP64_WG_WAVES][LTILE];
  const int wave = threadIdx.x / LANES;
  const int bin = blockIdx.x * FP64_WG_WAVES + wave;
  if (bin >= nbins) return;
  double(*red)[LANES / 2 + 1] = red_w[wave];
  double* sA = sA_w[wave];
  const int map = blockIdx.y;
  // this wave's bin of work items (packed at plan time)
  const int k_end = bins[bin + 1];
  for (int k = bins[bin]; k < k_end; ++k) {
    const WorkItem it = items[k];
    const int m = it.m, blk = it.blk;
    const int lane = threadIdx.x % LANES;
    const int lmax = P.lmax;
    const int nact = P.n_active[m];
    const double* __restrict__ Arow = P.A + P.row_off[m];
    const size_t pstride = gf_stride(lmax);
    const double* Gm = G + (size_t)map * P.npairs * pstride + (size_t)m * 4;

    RingState<R> st;
    init_rings<R>(P, m, blk, lane, nact, st);
    // S/D of each ring, zero while the ring's values are still scaled
    double Sre[R], Sim[R], Dre[R], Dim[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = blk * (LANES * R) + r * LANES + lane;
      if (q < nact && st.sc[r] == 0) {
        const double4 sd = *reinterpret_cast<const double4*>(Gm + (size_t)q * pstride);
        Sre[r] = sd.x;
        Sim[r] = sd.y;
        Dre[r] = sd.z;
        Dim[r] = sd.w;
      } else {
        Sre[r] = Sim[r] = Dre[r] = Dim[r] = 0.0;
      }
    }

    double* out = reinterpret_cast<double*>(partial + ((size_t)map * P.nblk_max + blk) * P.nalm);
    const int64_t row = alm_index(lmax, m, m);

    // recurrence coefficients of LTILE values of l: lane i loads l = base + i one
    // tile ahead, the tile in use is read from LDS (the same address in every lane).
    // The loads are unconditional, with the index clamped to nl (the first entry of
    // the row's zero padding), so that no wait for them lands inside the loop.
    const int nl = lmax - m + 1;
    auto tile_a = [&](int i) { return Arow[min(i, nl)]; };
    sA[lane] = tile_a(lane);
    // every load issued so far (ring seeds, S/D, tile 0) completes here, so the loop
    // body waits on nothing but its own LDS reads
    __builtin_amdgcn_s_waitcnt(0);
    wave_sync();
    double An = tile_a(LTILE + lane);

    for (int l0 = m; l0 <= lmax; l0 += ACH) {
      const int t0 = (l0 - m) & (LTILE - 1);
      if (t0 == 0 && l0 > m) {
        sA[lane] = An;      // the previous tile's last readers passed the barrier below
        wave_sync();
        An = tile_a(l0 - m + LTILE + lane);
      }
      double are[ACH], aim[ACH];
#pragma unroll
      for (int j = 0; j < ACH; ++j) are[j] = aim[j] = 0.0;
      const double* Ac = sA + t0;
#pragma unroll
      for (int j = 0; j < ACH; j += 2) {
        const double A0 = Ac[j], A1 = Ac[j + 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // mu2 <- mu_l (l - m even), then mu1 <- mu_{l+1} (odd)
          st.mu2[r] = fma(A0 * st.z[r], st.mu1[r], -st.mu2[r]);
          are[j] = fma(st.mu2[r], Sre[r], are[j]);
          aim[j] = fma(st.mu2[r], Sim[r], aim[j]);
          st.mu1[r] = fma(A1 * st.z[r], st.mu2[r], -st.mu1[r]);
          are[j + 1] = fma(st.mu1[r], Dre[r], are[j + 1]);
          aim[j + 1] = fma(st.mu1[r], Dim[r], aim[j + 1]);
        }
      }
      // reduce the NV = 2 ACH values (v = 2 j + re/im) over the 64 lanes: first lanes
      // l and l + 32 in registers, the lower half keeping values 0..NV/2-1 and the
      // upper half the rest, then the remaining 32 lanes through LDS, LPV lanes per
      // value each adding 32 / LPV entries, and LPV - 1 shuffles
      constexpr int NV = 2 * ACH, LPV = LANES / NV;
#pragma unroll
      for (int i = 0; i < ACH; ++i) {
        const int ja = i >> 1, jb = ACH / 2 + (i >> 1);
        const double va = (i & 1) ? aim[ja] : are[ja];
        const double vb = (i & 1) ? aim[jb] : are[jb];
        red[i + (lane >> 5) * ACH][lane & 31] = fold_halves(va, vb);
      }
      wave_sync();
      const int v = lane / LPV;
      const int h = (lane % LPV) * (32 / LPV);
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < 32 / LPV; ++k) sum += red[v][h + k];
#pragma unroll
      for (int x = 1; x < LPV; x <<= 1) sum += __shfl_xor(sum, x);
      if (lane % LPV == 0) {
        const int l = l0 + (v >> 1);
        if (l <= lmax) out[2 * (row + (l - m)) + (v & 1)] = sum;
      }
      wave_sync();
      int anysc = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) anysc |= st.sc[r];
      const int woke = wave_any(anysc) ? rescale_chunk<R>(st) : 0;
      if (woke) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (woke & (1 << r)) {
            const int q = blk * (LANES * R) + r * LANES + lane;
            const double4 sd = *reinterpret_cast<const double4*>(Gm + (size_t)q * pstride);
            Sre[r] = sd.x;
            Sim[r] = sd.y;
            Dre[r] = sd.z;
            Dim[r] = sd.w;
          }
        // (rare) complete these loads here rather than at their first use, where the
        // wait would also cover the tile prefetch
        __builtin_amdgcn_s_waitcnt(0);
      }
    }
  }
}

// Filtered coefficients for the synthesis, one thread per (l, m, map):
//   SY_FROM_PARTIAL  a = C_l sum_blk partial, s = f_l(lambda) a
//   SY_ALM_ONLY      a = C_l sum_blk partial (the forward transform), s = a
//   SY_FROM_ALM      s = caller's alm (imaginary part of m = 0 dropped)
// s goes to alm_out when requested; bcoef = C_l s, in the padded row layout of
// the recurrence tables (zeros beyond lmax) so the synthesis can read whole chunks.
// A flat grid over the padded rows r of every m (m = row_m[r], l = m + r - row_off[m];
// padding rows get zeros) and the maps: with one workgroup per m instead, the long rows
// of small m went to a few waves in turn, each waiting on its loads.
__global__ void legendre_coeff_kernel(PlanDev P, SynthArgs a) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int map = blockIdx.y;
  const bool chi = a.chi2 != nullptr && a.mode == SY_FROM_PARTIAL;
  double chi_acc = 0.0;
  if (r < P.rows_total) {
    const int lmax = P.lmax;
    const int m = P.row_m[r];
    const int i = (int)(r - P.row_off[m]);
    const int nl = lmax - m + 1;
    double2 b = make_double2(0.0, 0.0);
    if (i < nl) {
      const int64_t row = alm_index(lmax, m, m);
      const double c = P.C[r];
      double2 alm;
      if (a.mode == SY_FROM_ALM) {
        alm = a.alm_in[(size_t)map * P.nalm + row + i];
        if (m == 0) alm.y = 0.0;
      } else {
        // the blocks' partial sums, KB at a time with their loads issued together
        constexpr int KB = 4;
        const int nb = P.nblk[m];
        const double2* pb = a.partial + (size_t)map * P.nblk_max * P.nalm + row + i;
        double sr = 0.0, si = 0.0;
        for (int k0 = 0; k0 < nb; k0 += KB) {
          double2 p[KB];
#pragma unroll
          for (int u = 0; u < KB; ++u) p[u] = k0 + u < nb ? pb[(size_t)(k0 + u) * P.nalm] : make_double2(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < KB; ++u) {
            sr += p[u].x;
            si += p[u].y;
          }
        }
        // the ring phase already applied Omega to G
        alm = make_double2(sr * c, si * c);
        if (a.mode == SY_FROM_PARTIAL) {
          const double cl = P.cl[m + i];
          const double f = cl > 0.0 ? cl / (cl + a.lambda * P.tau * P.omega) : 0.0;
          alm.x *= f;
          alm.y *= f;
          // chi^2 prior term of the new iterate: w_m |s_lm|^2 / C_l (w = 1 at m = 0, else 2)
          if (chi && cl > 0.0) chi_acc = (m == 0 ? 1.0 : 2.0) * (alm.x * alm.x + alm.y * alm.y) / cl;
        }
      }
      if (a.alm_out) a.alm_out[(size_t)map * P.nalm + row + i] = alm;
      b = make_double2(alm.x * c, alm.y * c);
    }
    if (a.mode != SY_ALM_ONLY) a.bcoef[(size_t)map * P.rows_total + r] = b;
  }
  if (chi) block_sum_add(chi_acc, a.chi2 + map * a.chi2_stride);
}

constexpr int SCH = 8;   // synthesis steps per coefficient chunk

template <int R>
__global__ void __launch_bounds__(FP64_WG_WAVES * LANES) legendre_synthesis_f64_kernel(
    PlanDev P, const WorkItem* __restrict__ items, const int32_t* __restrict__ bins, int nbins, SynthArgs a) {
  // per-wave LDS: the waves of a workgroup run unrelated bins and never synchronise
  __shared__ double sA_w[FP64_WG_WAVES][LTILE];
  __shared__ double2 sb_w[FP64_WG_WAVES][LTILE];
  const int wave = threadIdx.x / LANES;
  const int bin = blockIdx.x * FP64_WG_WAVES + wave;
  if (bin >= nbins) return;
  double* sA = sA_w[wave];
  double2* sb = sb_w[wave];
  const int map = blockIdx.y;
  // this wave's bin of work items (packed at plan time)
  const int k_end = bins[bin + 1];
  for (int k = bins[bin]; k < k_end; ++k) {
    const WorkItem it = items[k];
    const int m = it.m, blk = it.blk;
    const int lane = threadIdx.x % LANES;
    const int lmax = P.lmax;
    const int64_t roff = P.row_off[m];
    const double* __restrict__ Arow = P.A + roff;
    const double2* __restrict__ brow = a.bcoef + (size_t)map * P.rows_total + roff;

    const int nact = P.n_active[m];
    const int nl = lmax - m + 1;
    // coefficients of LTILE values of l: lane i loads l = base + i one tile ahead,
    // the tile in use is read from LDS (the same address in every lane). The loads
    // are unconditional, with the index clamped to nl (the first entry of the row's
    // zero padding: A is zero there and the coefficient kernel writes zeros past
    // lmax), so that no wait for them lands inside the loop.
    auto tile_a = [&](int i) { return Arow[min(i, nl)]; };
    auto tile_b = [&](int i) { return brow[min(i, nl)]; };
    RingState<R> st;
    init_rings<R>(P, m, blk, lane, nact, st);
    sA[lane] = tile_a(lane);
    sb[lane] = tile_b(lane);
    // every load issued so far (ring seeds, tile 0) completes here, so the loop body
    // waits on nothing but its own LDS reads
    __builtin_amdgcn_s_waitcnt(0);
    wave_sync();
    double An = tile_a(LTILE + lane);
    double2 bn = tile_b(LTILE + lane);
    double Ere[R], Eim[R], Ore[R], Oim[R];
#pragma unroll
    for (int r = 0; r < R; ++r) Ere[r] = Eim[r] = Ore[r] = Oim[r] = 0.0;

    for (int l0 = m; l0 <= lmax; l0 += SCH) {
      const int t0 = (l0 - m) & (LTILE - 1);
      if (t0 == 0 && l0 > m) {
        wave_sync();
        sA[lane] = An;
        sb[lane] = bn;
        wave_sync();
        An = tile_a(l0 - m + LTILE + lane);
        bn = tile_b(l0 - m + LTILE + lane);
      }
      double A[SCH];
      double2 b[SCH];
#pragma unroll
      for (int j = 0; j < SCH; ++j) {
        A[j] = sA[t0 + j];
        b[j] = sb[t0 + j];
      }
      int scaled = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) scaled |= (st.sc[r] != 0) << r;
#pragma unroll
      for (int j = 0; j < SCH; j += 2) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          st.mu2[r] = fma(A[j] * st.z[r], st.mu1[r], -st.mu2[r]);          // l - m even
          Ere[r] = fma(st.mu2[r], b[j].x, Ere[r]);
          Eim[r] = fma(st.mu2[r], b[j].y, Eim[r]);
          st.mu1[r] = fma(A[j + 1] * st.z[r], st.mu2[r], -st.mu1[r]);      // odd
          Ore[r] = fma(st.mu1[r], b[j + 1].x, Ore[r]);
          Oim[r] = fma(st.mu1[r], b[j + 1].y, Oim[r]);
        }
      }
      // a ring still scaled at the chunk start has contributed nothing so far: clear it
      if (wave_any(scaled)) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (scaled & (1 << r)) Ere[r] = Eim[r] = Ore[r] = Oim[r] = 0.0;
        rescale_chunk<R>(st);
      }
    }

    const size_t pstride = gf_stride(lmax);
    double* Fm = a.F + (size_t)map * P.npairs * pstride + (size_t)m * 4;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = blk * (LANES * R) + r * LANES + lane;
      if (q < nact)
        *reinterpret_cast<double4*>(Fm + (size_t)q * pstride) =
            make_double4(Ere[r], Eim[r], Ore[r], Oim[r]);
    }
  }
}

// Plan time, per (m, ring pair): the first l - m + 1 at which lambda_lm(z_q) has
// risen above the scaled range (its scale reached 0; 0 if it starts there), or
// WAKE_NEVER if that does not happen for l <= lmax (the pair is skipped for m).
__global__ void reach_kernel(PlanDev P, uint16_t* __restrict__ wake) {
  const int m = blockIdx.y;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.npairs) return;
  const RingPair rp = P.pairs[q];
  double v;
  int s;
  sectoral_seed(m, rp.sin_t, P.norm_m[m], &v, &s);
  uint16_t w = s == 0 ? 0 : WAKE_NEVER;
  if (s != 0) {
    const double* Arow = P.A + P.row_off[m];
    double mu1 = 0.0, mu2 = -v;
    for (int l = m; l <= P.lmax; ++l) {
      const double mu = fma(Arow[l - m] * rp.z, mu1, -mu2);
      mu2 = mu1;
      mu1 = mu;
      if (fabs(mu1) > BIG_THRESH) {
        mu1 *= RESCALE;
        mu2 *= RESCALE;
        if (--s == 0) {
          w = (uint16_t)(l - m + 1);
          break;
        }
      }
    }
  }
  wake[(size_t)m * P.npairs + q] = w;
}

template <int R>
hipError_t launch_ana_r(const PlanDev& P, const WorkItem* items, const int32_t* bins, int nbins, int nmaps,
                        const double* G, double2* partial, hipStream_t s) {
  hipLaunchKernelGGL(legendre_analysis_f64_kernel<R>, dim3((nbins + FP64_WG_WAVES - 1) / FP64_WG_WAVES, nmaps),
                     dim3(FP64_WG_WAVES * LANES), 0, s, P, items, bins, nbins, G, partial);
  return hipGetLastError();
}

template <int R>
hipError_t launch_syn_r(const PlanDev& P, const WorkItem* items, const int32_t* bins, int nbins,
                        const SynthArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(legendre_synthesis_f64_kernel<R>, dim3((nbins + FP64_WG_WAVES - 1) / FP64_WG_WAVES, a.nmaps),
                     dim3(FP64_WG_WAVES * LANES), 0, s, P, items, bins, nbins, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_legendre_analysis_f64(const PlanDev& P, const WorkItem* items, const int32_t* bins,
                                        int nbins, int nmaps, const double* G, double2* partial,
                                        hipStream_t s) {
  switch (P.ring_block_ana / LANES) {
    case 1: return launch_ana_r<1>(P, items, bins, nbins, nmaps, G, partial, s);
    case 2: return launch_ana_r<2>(P, items, bins, nbins, nmaps, G, partial, s);
    case 4: return launch_ana_r<4>(P, items, bins, nbins, nmaps, G, partial, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_legendre_coeff(const PlanDev& P, const SynthArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(legendre_coeff_kernel, dim3((unsigned)((P.rows_total + 255) / 256), a.nmaps), dim3(256), 0, s,
                     P, a);
  return hipGetLastError();
}

hipError_t launch_legendre_synthesis_f64(const PlanDev& P, const WorkItem* items, const int32_t* bins,
                                         int nbins, const SynthArgs& a, hipStream_t s) {
  switch (P.ring_block_syn / LANES) {
    case 1: return launch_syn_r<1>(P, items, bins, nbins, a, s);
    case 2: return launch_syn_r<2>(P, items, bins, nbins, a, s);
    case 4: return launch_syn_r<4>(P, items, bins, nbins, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reach(const PlanDev& P, uint16_t* wake, hipStream_t s) {
  dim3 grid((P.npairs + 127) / 128, P.lmax + 1);
  hipLaunchKernelGGL(reach_kernel, grid, dim3(128), 0, s, P, wake);
  return hipGetLastError();
}

}  // namespace mwf
