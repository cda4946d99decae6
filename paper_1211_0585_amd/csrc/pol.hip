// Spin-2 Legendre phase of a polarised messenger sweep (FP64), and the coefficient
// step that couples T and E through the 3x3 signal covariance (Eq. 4).
//
// The polarisation fields Q, U of a ring carry ring Fourier coefficients G_Q, G_U
// (from the ring phase, S = G_N + G_S and D = G_N - G_S per m as for T). With
// lambda+ = ((2)lambda + (-2)lambda)/2 and lambda- = ((2)lambda - (-2)lambda)/2 the
// analysis is
//   E_lm = -sum_rings [lambda+ G_Q + i lambda- G_U],  B_lm = sum_rings [-lambda+ G_U + i lambda- G_Q]
// and the synthesis
//   F_Q = sum_l [-E lambda+ - i B lambda-],  F_U = sum_l [-B lambda+ + i E lambda-].
// Mirror rings follow from (s)lambda_lm(-z) = (-1)^(l+m) (-s)lambda_lm(z): lambda+ has the
// parity (-1)^(l+m) of a spin-0 function and lambda- the opposite one, so each l pairs
// the S of one field with the D of the other.
//
// The spin-2 functions come from the three-term recurrence of the Wigner d-functions,
// run on u = (s)lambda / K_l (plan tables A, B, K):
//   u_l = (A_l z + (s/2) B_l) u_{l-1} - u_{l-2},   s = +2 and -2,
// two multiply-adds per value and spin. The seeds at l0 = max(m, 2) are
//   m >= 2: (+-2)lambda_mm = lambda_mm sqrt(m (m-1) / ((m+1)(m+2))) tan^(+-2)(theta/2)
//           (the spin-0 sectoral value times a ratio, sharing its exponent scale),
//   m = 0:  (+-2)lambda_20 = sqrt(15 / (32 pi)) sin^2 theta,
//   m = 1:  (+-2)lambda_21 = -+ sqrt(5 / pi) sin(theta)/2 (1 -+ z)/2.
// Both spins of a ring share one scale: they are rescaled together once per chunk, and
// while the scale is positive the ring contributes nothing (as for spin 0).
//
// Work: one workgroup of four waves per (m, block of 256 ring pairs); each wave owns 64
// ring pairs, one per lane. The analysis reduces each chunk of 8 values of l over the
// lanes (halves folded in registers, then LDS) and over the four waves (LDS), and
// writes one partial sum of (E, B) per (l, m, block). The synthesis needs no
// reduction and writes F_Q, F_U of its ring pairs.
#include "mwf_internal.hpp"

namespace mwf {
namespace {

constexpr double BIG_THRESH = 0x1p64;
constexpr double RESCALE = 0x1p-512;
constexpr int S2_WAVES = 4;
constexpr int S2_TILE = 64;   // values of l per prefetched coefficient tile
constexpr int S2_ACH = 8;     // values of l per reduction and scale check
constexpr int S2_NV = 4 * S2_ACH;   // reduced values per chunk: (E re, E im, B re, B im) per l
static_assert(S2_NV == 32, "the lane reduction assumes 32 values per chunk");

__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// a + b over lanes l and l + 32 with the halves exchanged (v_permlane32_swap).
__device__ __forceinline__ double fold_halves(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// Spin-2 state of one ring pair: z, the even / odd (l - m) registers of u for s = +2
// and s = -2, and the shared scale.
struct S2Ring {
  double z, ep, op, em, om;
  int sc;
};

__device__ __forceinline__ void s2_init(const PlanDev& P, const Spin2Dev& S2, int m, int q, bool valid, S2Ring& r) {
  r.ep = r.op = r.em = r.om = 0.0;
  r.sc = 0;
  r.z = 0.0;
  if (!valid) return;
  const RingPair rp = P.pairs[q];
  const double z = rp.z, st = rp.sin_t;
  r.z = z;
  if (m >= 2) {
    double v;
    int sc;
    sectoral_seed(m, st, P.norm_m[m], &v, &sc);
    const double t2 = (1.0 - z) / (1.0 + z);        // tan^2(theta / 2)
    const double base = v * S2.norm[m];
    r.ep = -(base * t2);                             // first step (A = B = 0) gives u_m = seed
    r.em = -(base / t2);
    r.sc = sc;
  } else if (m == 0) {
    const double v = S2.norm[0] * (1.0 - z) * (1.0 + z);   // norm[0] = sqrt(15 / (32 pi)); times sin^2
    r.ep = v;                                        // u at l = 0, 1 is not used; l = 2 gets v
    r.em = v;
  } else {
    const double c = S2.norm[1] * 0.5 * st;                  // norm[1] = sqrt(5 / pi); times sin / 2
    r.op = c * 0.5 * (1.0 - z);                      // l = 2 is the odd register for m = 1
    r.om = -(c * 0.5 * (1.0 + z));
  }
}

// Once per chunk: bring large scaled values back by 2^-512 (both spins). Returns 1 if
// the scale reached zero in this call.
__device__ __forceinline__ int s2_rescale(S2Ring& r) {
  if (r.sc > 0 && fmax(fmax(fabs(r.ep), fabs(r.op)), fmax(fabs(r.em), fabs(r.om))) > BIG_THRESH) {
    r.ep *= RESCALE;
    r.op *= RESCALE;
    r.em *= RESCALE;
    r.om *= RESCALE;
    r.sc -= 1;
    return r.sc == 0;
  }
  return 0;
}

// Analysis inputs of one ring pair for l - m even (e) and odd (o):
//   even: P1 = SQ + i DU, P2 = SQ - i DU, P3 = -SU + i DQ, P4 = -SU - i DQ
//   odd:  the same with S and D exchanged,
// so that per l:  sum_E += u+ P1 + u- P2,  sum_B += u+ P3 + u- P4.
struct S2In {
  double e[8], o[8];   // re, im of P1..P4
};

__device__ __forceinline__ void s2_inputs(const double4& gq, const double4& gu, bool on, S2In& in) {
  if (!on) {
#pragma unroll
    for (int i = 0; i < 8; ++i) in.e[i] = in.o[i] = 0.0;
    return;
  }
  const double SQr = gq.x, SQi = gq.y, DQr = gq.z, DQi = gq.w;
  const double SUr = gu.x, SUi = gu.y, DUr = gu.z, DUi = gu.w;
  in.e[0] = SQr - DUi; in.e[1] = SQi + DUr;       // SQ + i DU
  in.e[2] = SQr + DUi; in.e[3] = SQi - DUr;       // SQ - i DU
  in.e[4] = -SUr - DQi; in.e[5] = -SUi + DQr;     // -SU + i DQ
  in.e[6] = -SUr + DQi; in.e[7] = -SUi - DQr;     // -SU - i DQ
  in.o[0] = DQr - SUi; in.o[1] = DQi + SUr;
  in.o[2] = DQr + SUi; in.o[3] = DQi - SUr;
  in.o[4] = -DUr - SQi; in.o[5] = -DUi + SQr;
  in.o[6] = -DUr + SQi; in.o[7] = -DUi - SQr;
}

__global__ void __launch_bounds__(S2_WAVES * LANES) spin2_analysis_kernel(PlanDev P, Spin2Dev S2,
                                                                          const double* __restrict__ G,
                                                                          double* __restrict__ partial, int nblk2) {
  __shared__ double red_w[S2_WAVES][S2_NV][LANES / 2 + 1];
  __shared__ double sA_w[S2_WAVES][S2_TILE], sB_w[S2_WAVES][S2_TILE];
  __shared__ double wsum[2][S2_WAVES][S2_NV];
  const int wave = threadIdx.x / LANES, lane = threadIdx.x % LANES;
  const WorkItem it = S2.items[blockIdx.x];
  const int map = blockIdx.y;
  const int m = it.m, blk = it.blk;
  const int lmax = P.lmax;
  const int nact = P.n_active[m];
  const int q = blk * (S2_WAVES * LANES) + wave * LANES + lane;
  const bool valid = q < nact;
  double(*red)[LANES / 2 + 1] = red_w[wave];
  double* sA = sA_w[wave];
  double* sB = sB_w[wave];
  const size_t pstride = gf_stride(lmax);
  const double* Gq = G + (((size_t)1 * S2.field_maps + map) * P.npairs) * pstride + (size_t)m * 4;
  const double* Gu = G + (((size_t)2 * S2.field_maps + map) * P.npairs) * pstride + (size_t)m * 4;

  S2Ring r;
  s2_init(P, S2, m, q, valid, r);
  S2In in;
  {
    double4 gq = make_double4(0, 0, 0, 0), gu = gq;
    if (valid) {
      gq = *reinterpret_cast<const double4*>(Gq + (size_t)q * pstride);
      gu = *reinterpret_cast<const double4*>(Gu + (size_t)q * pstride);
    }
    s2_inputs(gq, gu, valid && r.sc == 0, in);
  }
  const int64_t roff = P.row_off[m];
  const double* __restrict__ Arow = S2.A + roff;
  const double* __restrict__ Brow = S2.B + roff;
  const int nl = lmax - m + 1;
  auto tile_a = [&](int i) { return Arow[min(i, nl)]; };
  auto tile_b = [&](int i) { return Brow[min(i, nl)]; };
  sA[lane] = tile_a(lane);
  sB[lane] = tile_b(lane);
  __builtin_amdgcn_s_waitcnt(0);
  wave_sync();
  double An = tile_a(S2_TILE + lane), Bn = tile_b(S2_TILE + lane);
  double* out = partial + (((size_t)map * nblk2 + blk) * P.nalm) * 4;
  const int64_t row = alm_index(lmax, m, m);
  int par = 0;

  for (int l0 = m; l0 <= lmax; l0 += S2_ACH) {
    const int t0 = (l0 - m) & (S2_TILE - 1);
    if (t0 == 0 && l0 > m) {
      sA[lane] = An;
      sB[lane] = Bn;
      wave_sync();
      An = tile_a(l0 - m + S2_TILE + lane);
      Bn = tile_b(l0 - m + S2_TILE + lane);
    }
    double acc[S2_NV];
#pragma unroll
    for (int i = 0; i < S2_NV; ++i) acc[i] = 0.0;
#pragma unroll
    for (int j = 0; j < S2_ACH; j += 2) {
      {
        const double A = sA[t0 + j], B = sB[t0 + j];
        const double tp = fma(A, r.z, B), tm = fma(A, r.z, -B);
        r.ep = fma(tp, r.op, -r.ep);
        r.em = fma(tm, r.om, -r.em);
        acc[4 * j + 0] = fma(r.ep, in.e[0], r.em * in.e[2]);
        acc[4 * j + 1] = fma(r.ep, in.e[1], r.em * in.e[3]);
        acc[4 * j + 2] = fma(r.ep, in.e[4], r.em * in.e[6]);
        acc[4 * j + 3] = fma(r.ep, in.e[5], r.em * in.e[7]);
      }
      {
        const double A = sA[t0 + j + 1], B = sB[t0 + j + 1];
        const double tp = fma(A, r.z, B), tm = fma(A, r.z, -B);
        r.op = fma(tp, r.ep, -r.op);
        r.om = fma(tm, r.em, -r.om);
        acc[4 * j + 4] = fma(r.op, in.o[0], r.om * in.o[2]);
        acc[4 * j + 5] = fma(r.op, in.o[1], r.om * in.o[3]);
        acc[4 * j + 6] = fma(r.op, in.o[4], r.om * in.o[6]);
        acc[4 * j + 7] = fma(r.op, in.o[5], r.om * in.o[7]);
      }
    }
    // over the lanes: values 0..15 folded into lanes 0..31, 16..31 into lanes 32..63,
    // then two lanes per value add 16 entries each
#pragma unroll
    for (int i = 0; i < S2_NV / 2; ++i) red[i + (lane >> 5) * (S2_NV / 2)][lane & 31] = fold_halves(acc[i], acc[S2_NV / 2 + i]);
    wave_sync();
    const int v = lane >> 1;
    const int h = (lane & 1) * 16;
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) sum += red[v][h + k];
    sum += __shfl_xor(sum, 1);
    // over the waves of the workgroup (two slots alternate, one barrier per chunk)
    if ((lane & 1) == 0) wsum[par][wave][v] = sum;
    __syncthreads();
    if (wave == 0 && lane < S2_NV) {
      const double t = wsum[par][0][lane] + wsum[par][1][lane] + wsum[par][2][lane] + wsum[par][3][lane];
      const int l = l0 + (lane >> 2);
      if (l <= lmax) out[(row + (l - m)) * 4 + (lane & 3)] = t;
    }
    par ^= 1;
    wave_sync();
    if (__any(r.sc) && s2_rescale(r)) {
      const double4 gq = *reinterpret_cast<const double4*>(Gq + (size_t)q * pstride);
      const double4 gu = *reinterpret_cast<const double4*>(Gu + (size_t)q * pstride);
      s2_inputs(gq, gu, true, in);
      __builtin_amdgcn_s_waitcnt(0);
    }
  }
}

// Synthesis: per l the coefficients e = -K s_E / 2 and b = -K s_B / 2 (plan layout,
// bcoef_eb[map][row][2]); with sigma = u+ + u- and delta = u+ - u-:
//   l - m even: E_Q += e sigma, O_Q += i b delta, E_U += b sigma, O_U -= i e delta
//   l - m odd:  O_Q += e sigma, E_Q += i b delta, O_U += b sigma, E_U -= i e delta
// and F_N = E + O, F_S = E - O in the ring phase.
__global__ void __launch_bounds__(S2_WAVES * LANES) spin2_synthesis_kernel(PlanDev P, Spin2Dev S2,
                                                                           const double2* __restrict__ bcoef,
                                                                           double* __restrict__ F) {
  __shared__ double sA_w[S2_WAVES][S2_TILE], sB_w[S2_WAVES][S2_TILE];
  __shared__ double2 se_w[S2_WAVES][S2_TILE], sb_w[S2_WAVES][S2_TILE];
  const int wave = threadIdx.x / LANES, lane = threadIdx.x % LANES;
  const WorkItem it = S2.items[blockIdx.x];
  const int map = blockIdx.y;
  const int m = it.m, blk = it.blk;
  const int lmax = P.lmax;
  const int nact = P.n_active[m];
  const int q = blk * (S2_WAVES * LANES) + wave * LANES + lane;
  if (blk * (S2_WAVES * LANES) + wave * LANES >= nact) return;   // the whole wave is past the active pairs
  const bool valid = q < nact;
  double* sA = sA_w[wave];
  double* sB = sB_w[wave];
  double2* se = se_w[wave];
  double2* sb = sb_w[wave];
  const int64_t roff = P.row_off[m];
  const double* __restrict__ Arow = S2.A + roff;
  const double* __restrict__ Brow = S2.B + roff;
  const double2* __restrict__ crow = bcoef + ((size_t)map * P.rows_total + roff) * 2;
  const int nl = lmax - m + 1;
  auto tile_a = [&](int i) { return Arow[min(i, nl)]; };
  auto tile_b = [&](int i) { return Brow[min(i, nl)]; };
  auto tile_e = [&](int i) { return crow[2 * min(i, nl)]; };
  auto tile_f = [&](int i) { return crow[2 * min(i, nl) + 1]; };
  S2Ring r;
  s2_init(P, S2, m, q, valid, r);
  sA[lane] = tile_a(lane);
  sB[lane] = tile_b(lane);
  se[lane] = tile_e(lane);
  sb[lane] = tile_f(lane);
  __builtin_amdgcn_s_waitcnt(0);
  wave_sync();
  double An = tile_a(S2_TILE + lane), Bn = tile_b(S2_TILE + lane);
  double2 en = tile_e(S2_TILE + lane), bn = tile_f(S2_TILE + lane);
  double EQr = 0, EQi = 0, OQr = 0, OQi = 0, EUr = 0, EUi = 0, OUr = 0, OUi = 0;

  for (int l0 = m; l0 <= lmax; l0 += S2_ACH) {
    const int t0 = (l0 - m) & (S2_TILE - 1);
    if (t0 == 0 && l0 > m) {
      wave_sync();
      sA[lane] = An;
      sB[lane] = Bn;
      se[lane] = en;
      sb[lane] = bn;
      wave_sync();
      An = tile_a(l0 - m + S2_TILE + lane);
      Bn = tile_b(l0 - m + S2_TILE + lane);
      en = tile_e(l0 - m + S2_TILE + lane);
      bn = tile_f(l0 - m + S2_TILE + lane);
    }
    const int scaled = r.sc != 0;
#pragma unroll
    for (int j = 0; j < S2_ACH; j += 2) {
      {
        const double A = sA[t0 + j], B = sB[t0 + j];
        const double2 e = se[t0 + j], b = sb[t0 + j];
        const double tp = fma(A, r.z, B), tm = fma(A, r.z, -B);
        r.ep = fma(tp, r.op, -r.ep);
        r.em = fma(tm, r.om, -r.em);
        const double sg = r.ep + r.em, dl = r.ep - r.em;
        EQr = fma(e.x, sg, EQr);
        EQi = fma(e.y, sg, EQi);
        OQr = fma(-b.y, dl, OQr);
        OQi = fma(b.x, dl, OQi);
        EUr = fma(b.x, sg, EUr);
        EUi = fma(b.y, sg, EUi);
        OUr = fma(e.y, dl, OUr);
        OUi = fma(-e.x, dl, OUi);
      }
      {
        const double A = sA[t0 + j + 1], B = sB[t0 + j + 1];
        const double2 e = se[t0 + j + 1], b = sb[t0 + j + 1];
        const double tp = fma(A, r.z, B), tm = fma(A, r.z, -B);
        r.op = fma(tp, r.ep, -r.op);
        r.om = fma(tm, r.em, -r.om);
        const double sg = r.op + r.om, dl = r.op - r.om;
        OQr = fma(e.x, sg, OQr);
        OQi = fma(e.y, sg, OQi);
        EQr = fma(-b.y, dl, EQr);
        EQi = fma(b.x, dl, EQi);
        OUr = fma(b.x, sg, OUr);
        OUi = fma(b.y, sg, OUi);
        EUr = fma(e.y, dl, EUr);
        EUi = fma(-e.x, dl, EUi);
      }
    }
    // a ring still scaled at the chunk start has contributed nothing so far
    if (__any(scaled)) {
      if (scaled) EQr = EQi = OQr = OQi = EUr = EUi = OUr = OUi = 0.0;
      s2_rescale(r);
    }
  }
  if (valid) {
    const size_t pstride = gf_stride(lmax);
    double* Fq = F + (((size_t)1 * S2.field_maps + map) * P.npairs + q) * pstride + (size_t)m * 4;
    double* Fu = F + (((size_t)2 * S2.field_maps + map) * P.npairs + q) * pstride + (size_t)m * 4;
    *reinterpret_cast<double4*>(Fq) = make_double4(EQr, EQi, OQr, OQi);
    *reinterpret_cast<double4*>(Fu) = make_double4(EUr, EUi, OUr, OUi);
  }
}

// One thread per (l, m, map), rows padded as the recurrence tables:
//   a_T = C_l sum partial_T,  a_E = -(K/2) sum partial_E,  a_B = (K/2) sum partial_B
//   SY_FROM_PARTIAL: s = F_l a with F_l = C_l (C_l + lambda tau Omega)^-1 (TE-coupled),
//   SY_ALM_ONLY: s = a,  SY_FROM_ALM: s = the caller's alm (imaginary part dropped at m = 0).
// F_l in closed form for the TE block [[TT, TE], [TE, EE]] (mu = lambda tau Omega,
// det = TT EE - TE^2, D = det + mu (TT + EE) + mu^2):
//   F_TT = (det + TT mu) / D, F_TE = TE mu / D, F_EE = (det + EE mu) / D, F_BB = BB / (BB + mu)
// (no cancellation, and 0 where the spectra vanish).
__global__ void pol_coeff_kernel(PlanDev P, Spin2Dev S2, PolCoeffArgs a) {
  const int m = blockIdx.x;
  const int map = blockIdx.y;
  const int lmax = P.lmax;
  const int nl = lmax - m + 1;
  const int64_t row = alm_index(lmax, m, m);
  const int64_t roff = P.row_off[m];
  const double mu = a.lambda * P.tau * P.omega;
  const int nbt = P.nblk[m];
  const int nbe = a.nblk2_m[m];
  for (int i = threadIdx.x; i < nl + ROW_PAD; i += blockDim.x) {
    double2 sT = make_double2(0, 0), sE = sT, sB = sT;
    double K = 0.0, C0 = 0.0;
    if (i < nl) {
      const int l = m + i;
      K = S2.K[roff + i];
      C0 = P.C[roff + i];
      if (a.mode == SY_FROM_ALM) {
        const double2* al = a.alm_in + (size_t)map * 3 * P.nalm + row + i;
        sT = al[0];
        sE = al[P.nalm];
        sB = al[2 * P.nalm];
        if (m == 0) sT.y = sE.y = sB.y = 0.0;
      } else {
        double tr = 0, ti = 0;
        for (int k = 0; k < nbt; ++k) {
          const double2 p = a.partial_t[((size_t)map * P.nblk_max + k) * P.nalm + row + i];
          tr += p.x;
          ti += p.y;
        }
        double er = 0, ei = 0, br = 0, bi = 0;
        for (int k = 0; k < nbe; ++k) {
          const double4 p = reinterpret_cast<const double4*>(a.partial_eb)[((size_t)map * a.nblk2 + k) * P.nalm + row + i];
          er += p.x;
          ei += p.y;
          br += p.z;
          bi += p.w;
        }
        sT = make_double2(tr * C0, ti * C0);
        sE = make_double2(-0.5 * K * er, -0.5 * K * ei);
        sB = make_double2(0.5 * K * br, 0.5 * K * bi);
        if (a.mode == SY_FROM_PARTIAL) {
          const double tt = a.cl4[l], ee = a.cl4[(lmax + 1) + l], bb = a.cl4[2 * (lmax + 1) + l];
          const double te = a.cl4[3 * (lmax + 1) + l];
          const double det = tt * ee - te * te;
          const double D = det + mu * (tt + ee) + mu * mu;
          const double ftt = (det + tt * mu) / D, fte = te * mu / D, fee = (det + ee * mu) / D;
          const double fbb = bb > 0.0 ? bb / (bb + mu) : 0.0;
          const double2 t2 = make_double2(ftt * sT.x + fte * sE.x, ftt * sT.y + fte * sE.y);
          const double2 e2 = make_double2(fte * sT.x + fee * sE.x, fte * sT.y + fee * sE.y);
          sT = t2;
          sE = e2;
          sB = make_double2(fbb * sB.x, fbb * sB.y);
        }
      }
      if (a.alm_out) {
        double2* ao = a.alm_out + (size_t)map * 3 * P.nalm + row + i;
        ao[0] = sT;
        ao[P.nalm] = sE;
        ao[2 * P.nalm] = sB;
      }
    }
    if (a.mode != SY_ALM_ONLY) {
      a.bcoef_t[(size_t)map * P.rows_total + roff + i] = make_double2(sT.x * C0, sT.y * C0);
      double2* be = a.bcoef_eb + ((size_t)map * P.rows_total + roff + i) * 2;
      be[0] = make_double2(-0.5 * K * sE.x, -0.5 * K * sE.y);
      be[1] = make_double2(-0.5 * K * sB.x, -0.5 * K * sB.y);
    }
  }
}

}  // namespace

hipError_t launch_spin2_analysis(const PlanDev& P, const Spin2Dev& S2, int nmaps, const double* G, double* partial_eb,
                                 int nblk2, hipStream_t s) {
  if (S2.nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(spin2_analysis_kernel, dim3(S2.nitems, nmaps), dim3(S2_WAVES * LANES), 0, s, P, S2, G, partial_eb,
                     nblk2);
  return hipGetLastError();
}

hipError_t launch_spin2_synthesis(const PlanDev& P, const Spin2Dev& S2, int nmaps, const double2* bcoef_eb, double* F,
                                  hipStream_t s) {
  if (S2.nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(spin2_synthesis_kernel, dim3(S2.nitems, nmaps), dim3(S2_WAVES * LANES), 0, s, P, S2, bcoef_eb, F);
  return hipGetLastError();
}

hipError_t launch_pol_coeff(const PlanDev& P, const Spin2Dev& S2, const PolCoeffArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(pol_coeff_kernel, dim3(P.lmax + 1, a.nmaps), dim3(256), 0, s, P, S2, a);
  return hipGetLastError();
}

}  // namespace mwf
