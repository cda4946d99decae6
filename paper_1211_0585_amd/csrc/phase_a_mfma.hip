// Phase A on matrix cores: the Legendre contraction of a batch of maps as GEMMs.
//
// For each m and each parity of l - m, the analysis is the product
//   a[l][c] = sum_q lambda_lm(z_q) P[q][c],  P = S (l-m even) or D (l-m odd),
// with c running over (map, re/im) columns, and the synthesis is
//   E[q][c] = sum_{l-m even} lambda_lm(z_q) b[l][c],  O likewise for odd l - m,
// b = C_l s_lm (the filtered alm scaled by the recurrence normalisation).
// Here M = l, K = ring pairs, N = columns (analysis) and M = ring pairs,
// K = l, N = columns (synthesis). The Legendre values are generated on the fly
// in FP64 by the same rescaled recurrence as the VALU path (one ring pair per
// lane), rounded to the matrix type and staged through LDS in chunks of 32 l.
//
// Matrix paths:
//   FP32    v_mfma_f32_16x16x4_f32: A 16x4 (lane i + 16 k), B 4x16 (lane j + 16 k),
//           D 16x16 (lane j + 16 (i / 4), register i % 4).
//   BF16x3  v_mfma_f32_16x16x32_bf16 with operands split as x = hi + lo
//           (hi = bf16(x), lo = bf16(x - hi)) and three products
//           hi*hi + hi*lo + lo*hi accumulated in FP32; A 16x32 (lane i + 16 (k / 8),
//           element k % 8), B 32x16 (lane j + 16 (k / 8), element k % 8).
//   BF16x6  the same with three pieces x = hi + mid + lo and six products (terms
//           below 2^-24 relative dropped), reaching FP32-level accuracy.
// Both accumulate in FP32 within a block of ring pairs; blocks are summed in FP64.
#include "mwf_internal.hpp"

namespace mwf {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr double BIG_THRESH = 0x1p64;
constexpr double RESCALE = 0x1p-512;

// lambda_mm(z) = norm_m sin^m(theta) as v * 2^(-512 s) (same construction as the VALU path).
__device__ __forceinline__ void seed(int m, double sin_t, double norm, double* v, int* s) {
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
  const int e = er + t;
  int sc = 0;
  if (e < 64 - SCALE_BITS) sc = (64 - SCALE_BITS - e + SCALE_BITS - 1) / SCALE_BITS;
  *v = ldexp(x, e + SCALE_BITS * sc);
  *s = sc;
}

// One ring pair per thread: recurrence state.
struct Ring {
  double z, mu1, mu2;
  int sc;
};

__device__ __forceinline__ Ring ring_init(const PlanDev& P, int m, int q, int nact) {
  Ring r{0.0, 0.0, 0.0, 0};
  if (q < nact) {
    const RingPair rp = P.pairs[q];
    double v;
    int s;
    seed(m, rp.sin_t, P.norm_m[m], &v, &s);
    r.z = rp.z;
    r.mu2 = -v;     // with A_mm = 0 the first step yields mu_m = v
    r.sc = s;
  }
  return r;
}

// Advance MCH steps from l0 and hand each value to emit(j, value). A ring still
// scaled at the start of the chunk emits zeros for the whole chunk; the scale is
// checked once at its end. The recurrence alternates between mu2 and mu1, so a
// step is one multiply and one FMA.
template <class Emit>
__device__ __forceinline__ void ring_steps(Ring& r, const double* __restrict__ Ac, Emit emit) {
  const bool scaled = r.sc != 0;
  if (__any(scaled)) {
#pragma unroll
    for (int j = 0; j < MCH; j += 2) {
      r.mu2 = fma(Ac[j] * r.z, r.mu1, -r.mu2);
      emit(j, scaled ? 0.0 : r.mu2);
      r.mu1 = fma(Ac[j + 1] * r.z, r.mu2, -r.mu1);
      emit(j + 1, scaled ? 0.0 : r.mu1);
    }
    if (scaled && fmax(fabs(r.mu1), fabs(r.mu2)) > BIG_THRESH) {
      r.mu1 *= RESCALE;
      r.mu2 *= RESCALE;
      r.sc -= 1;
    }
  } else {
#pragma unroll
    for (int j = 0; j < MCH; j += 2) {
      r.mu2 = fma(Ac[j] * r.z, r.mu1, -r.mu2);
      emit(j, r.mu2);
      r.mu1 = fma(Ac[j + 1] * r.z, r.mu2, -r.mu1);
      emit(j + 1, r.mu1);
    }
  }
}

// x of lane l ^ 1 (DPP quad permutation 1, 0, 3, 2).
__device__ __forceinline__ float swap_lane_pair(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}

// x = p[0] + p[1] (+ p[2]): successive bf16 roundings of the remainder.
template <int NP>
__device__ __forceinline__ void split_pieces(float x, __bf16 (&p)[NP]) {
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    p[i] = (__bf16)x;
    x = x - (float)p[i];
  }
}

// The same split for two values at once, each piece a packed dword (a in the low half):
// one v_cvt_pk_bf16_f32 per piece for both values, and the dword is already laid out as
// two consecutive elements of a bf16 operand.
template <int NP>
__device__ __forceinline__ void split_pieces2(float a, float b, unsigned (&p)[NP]) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  f2 x = {a, b};
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const b2 h = __builtin_convertvector(x, b2);
    p[i] = __builtin_bit_cast(unsigned, h);
    if (i + 1 < NP) x = x - __builtin_convertvector(h, f2);
  }
}

// Piece products kept for an NP-piece split (smallest first): NP = 2 -> hi*lo,
// lo*hi, hi*hi; NP = 3 -> mid*mid, hi*lo, lo*hi, hi*mid, mid*hi, hi*hi.
template <int NP>
struct Products;
template <>
struct Products<1> {
  static constexpr int n = 1;
  static constexpr int a[1] = {0};
  static constexpr int b[1] = {0};
};
template <>
struct Products<2> {
  static constexpr int n = 3;
  static constexpr int a[3] = {0, 1, 0};
  static constexpr int b[3] = {1, 0, 0};
};
template <>
struct Products<3> {
  static constexpr int n = 6;
  static constexpr int a[6] = {1, 0, 2, 0, 1, 0};
  static constexpr int b[6] = {1, 2, 0, 1, 0, 0};
};

// ------------------------------------------------------------------ analysis
// Work item (m, block of RB = ana_block(CT) ring pairs) and column group cg of 16 CT
// columns (8 CT maps); 2 CT waves. The first RB threads run the recurrence, one ring
// pair each, and stage the values in LDS once per chunk of l for every wave of the
// workgroup (from CT = 4 on, half or more of the waves only contract, so the values
// are generated once per 64 or 128 columns rather than once per 32).
// Wave w owns the output tile (parity w & 1, column tile w >> 1).
// NP = 1: FP32 matrix cores; NP = 2 or 3: bf16 pieces.
template <int NP, int CT>
__device__ __forceinline__ void analysis_body(const PlanDev& P, const MfmaArgs& a, const WorkItem it,
                                              const int cg) {
  constexpr int RB = ana_block(CT);
  static_assert(RB <= 128 * CT && RB % LANES == 0, "generating threads are whole waves of the workgroup");
  constexpr bool F32 = (NP == 1);
  constexpr int NB = F32 ? 1 : NP;
  // staged Legendre values [parity][row][ring]; FP32 or bf16 pieces (rows 16 B aligned)
  __shared__ float lam_f[F32 ? 2 : 1][16][RB + 4];
  __shared__ __attribute__((aligned(16))) __bf16 lam_b[NB][F32 ? 1 : 2][16][RB + 8];
  const int m = it.m, blk = it.blk;
  if (m < 0) return;   // empty item of the XCD-ordered list
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lmax = P.lmax;
  const int nact = P.n_active[m];
  const int q0 = blk * RB;
  const double* __restrict__ Arow = P.A + P.row_off[m];
  const size_t pstride = gf_stride(lmax);
  const float* __restrict__ G = a.G;

  const bool gen = tid < RB;                      // uniform over the wave
  Ring ring = ring_init(P, m, gen ? q0 + tid : nact, nact);

  const int par = wave & 1, ct = wave >> 1;
  const int col = cg * (16 * CT) + ct * 16 + (lane & 15);
  const int map = col >> 1, comp = col & 1;
  const bool colok = map < a.nmaps;
  const float* Gc = G + (size_t)map * P.npairs * pstride + (size_t)m * 4 + 2 * par + comp;

  // B fragments: the S (even) or D (odd) column of this wave for all 256 ring pairs
  constexpr int KF = RB / 4;    // FP32 k-steps (K = 4)
  constexpr int KB = RB / 32;   // bf16 k-steps (K = 32)
  float bf[F32 ? KF : 1];
  bf8 bb[NB][F32 ? 1 : KB];
  if constexpr (F32) {
#pragma unroll
    for (int t = 0; t < KF; ++t) {
      const int q = q0 + 4 * t + (lane >> 4);
      bf[t] = (colok && q < nact) ? Gc[(size_t)q * pstride] : 0.0f;
    }
  } else {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int t = 0; t < KB; ++t) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int q = q0 + 32 * t + 8 * (lane >> 4) + e;
        v[e] = (colok && q < nact) ? Gc[(size_t)q * pstride] : 0.0f;
      }
      u4 bw[NB];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        unsigned pk[NB];
        split_pieces2<NB>(v[2 * w], v[2 * w + 1], pk);
#pragma unroll
        for (int i = 0; i < NB; ++i) bw[i][w] = pk[i];
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) bb[i][t] = __builtin_bit_cast(bf8, bw[i]);
    }
  }

  float* out = a.partial + (size_t)blk * P.nalm * 2 * a.nmaps;
  (void)KF;
  (void)KB;
  const int64_t row = alm_index(lmax, m, m);

  for (int l0 = m; l0 <= lmax; l0 += MCH) {
    const double* Ac = Arow + (l0 - m);
    if (gen) {
      if constexpr (F32) {
        ring_steps(ring, Ac, [&](int j, double v) { lam_f[j & 1][j >> 1][tid] = (float)v; });
      } else {
        float ev[2][16];   // [parity][row]
        ring_steps(ring, Ac, [&](int j, double v) { ev[j & 1][j >> 1] = (float)v; });
        // lanes 2k and 2k + 1 (adjacent rings) swap values so that each writes dwords holding
        // the pieces of both rings: the even lane those of rows 2r, the odd lane rows 2r + 1
        const int odd = tid & 1;
#pragma unroll
        for (int pp = 0; pp < 2; ++pp)
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const float a0 = ev[pp][2 * r], a1 = ev[pp][2 * r + 1];
            const float s0 = swap_lane_pair(a0), s1 = swap_lane_pair(a1);
            unsigned pk[NB];
            split_pieces2<NB>(odd ? s1 : a0, odd ? a1 : s0, pk);
#pragma unroll
            for (int i = 0; i < NB; ++i)
              *reinterpret_cast<unsigned*>(&lam_b[i][pp][2 * r + odd][tid & ~1]) = pk[i];
          }
      }
    }
    __syncthreads();
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (F32) {
#pragma unroll
      for (int t = 0; t < KF; ++t) {
        const float av = lam_f[par][lane & 15][4 * t + (lane >> 4)];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bf[t], acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int t = 0; t < KB; ++t) {
        bf8 av[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i)
          av[i] = *reinterpret_cast<const bf8*>(&lam_b[i][par][lane & 15][32 * t + 8 * (lane >> 4)]);
#pragma unroll
        for (int k = 0; k < Products<NB>::n; ++k)
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[Products<NB>::a[k]], bb[Products<NB>::b[k]][t],
                                                        acc, 0, 0, 0);
      }
    }
    if (colok) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * (lane >> 4) + r;
        const int l = l0 + 2 * i + par;
        if (l <= lmax) out[((size_t)(row + (l - m)) * a.nmaps + map) * 2 + comp] = acc[r];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ synthesis
// Work item (m, block of 64 ring pairs) and column group cg of 16 NCT columns, one wave.
// The wave's own Legendre values are staged through its LDS: FP32 in chunks of
// 32 l (16 per parity, K = 4 per product), bf16 pieces in chunks of 64 l
// (32 per parity, K = 32 per product).
template <int NP, int NCT>
__device__ __forceinline__ void synthesis_body(const PlanDev& P, const MfmaArgs& a, const WorkItem it,
                                               const int cg) {
  constexpr bool F32 = (NP == 1);
  constexpr int NB = F32 ? 1 : NP;
  constexpr int CHL = F32 ? MCH : 2 * MCH;       // l per chunk
  constexpr int ROWS = CHL / 2;                  // rows per parity
  // FP32: [parity][row][ring]; bf16 pieces: [piece][parity][ring][row] (row = k contiguous)
  __shared__ float lam_f[F32 ? 2 : 1][16][64 + 4];
  __shared__ __attribute__((aligned(16))) __bf16 lam_b[NB][F32 ? 1 : 2][64][ROWS + 8];
  const int m = it.m, blk = it.blk;
  if (m < 0) return;   // empty item of the XCD-ordered list
  const int lane = threadIdx.x;
  constexpr int CW = 16 * NCT;   // columns of this wave
  const int lmax = P.lmax;
  const int nact = P.n_active[m];
  const int q0 = blk * 64;
  const int64_t roff = P.row_off[m];
  const double* __restrict__ Arow = P.A + roff;
  const int ncols = 2 * a.nmaps;
  const float* __restrict__ brow = a.bcoef + (size_t)roff * ncols;

  Ring ring = ring_init(P, m, q0 + lane, nact);
  f4 acc[4][NCT][2];   // [ring tile][column tile][E / O]
#pragma unroll
  for (int qt = 0; qt < 4; ++qt)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int eo = 0; eo < 2; ++eo) acc[qt][ct][eo] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  // FP32: B fragments of a chunk are loaded one chunk ahead (a chunk's MFMAs give
  // them time to arrive). The loads are unconditional: columns past the last map are
  // clamped to it (their results are never stored) and rows past lmax read the zero
  // padding of the row (the next chunk of the last one ends at most 63 rows past it).
  float bv[F32 ? 2 : 1][4][F32 ? NCT : 1];
  auto load_b = [&](int l0, float (&dst)[F32 ? 2 : 1][4][F32 ? NCT : 1]) {
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const int rr = 4 * kk + (lane >> 4);
          const int colg = min(cg * CW + ct * 16 + (lane & 15), ncols - 1);
          dst[pp][kk][ct] = brow[(size_t)(l0 - m + 2 * rr + pp) * ncols + colg];
        }
  };
  if constexpr (F32) load_b(m, bv);

  for (int l0 = m; l0 <= lmax; l0 += CHL) {
    const double* Ac = Arow + (l0 - m);
    if constexpr (F32) {
      float bn[2][4][NCT];
      load_b(l0 + CHL, bn);
      ring_steps(ring, Ac, [&](int j, double v) { lam_f[j & 1][j >> 1][lane] = (float)v; });
      __syncthreads();
#pragma unroll
      for (int pp = 0; pp < 2; ++pp)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int rr = 4 * kk + (lane >> 4);
#pragma unroll
          for (int qt = 0; qt < 4; ++qt) {
            const float av = lam_f[pp][rr][qt * 16 + (lane & 15)];
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
              acc[qt][ct][pp] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[pp][kk][ct], acc[qt][ct][pp], 0, 0, 0);
          }
        }
#pragma unroll
      for (int pp = 0; pp < 2; ++pp)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) bv[pp][kk][ct] = bn[pp][kk][ct];
    } else {
      // B fragments straight from global: lane holds rows k8..k8+7 of one column
      const int k8 = 8 * (lane >> 4);
      float bvf[2][NCT][8];
#pragma unroll
      for (int pp = 0; pp < 2; ++pp)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const int colg = cg * CW + ct * 16 + (lane & 15);
#pragma unroll
          for (int e = 0; e < 8; ++e)
            bvf[pp][ct][e] = colg < ncols ? brow[(size_t)(l0 - m + 2 * (k8 + e) + pp) * ncols + colg] : 0.0f;
        }
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        float ev[2][MCH / 2];   // [parity][row]
        ring_steps(ring, Ac + half * MCH, [&](int j, double v) { ev[j & 1][j >> 1] = (float)v; });
        // the pieces of rows 2w and 2w + 1 (adjacent in the row-contiguous layout) as dwords
#pragma unroll
        for (int pp = 0; pp < 2; ++pp)
#pragma unroll
          for (int w = 0; w < MCH / 4; ++w) {
            unsigned pk[NB];
            split_pieces2<NB>(ev[pp][2 * w], ev[pp][2 * w + 1], pk);
#pragma unroll
            for (int i = 0; i < NB; ++i)
              *reinterpret_cast<unsigned*>(&lam_b[i][pp][lane][half * (MCH / 2) + 2 * w]) = pk[i];
          }
      }
      __syncthreads();
#pragma unroll
      for (int pp = 0; pp < 2; ++pp) {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        bf8 bv[NB][NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          u4 bw[NB];
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            unsigned pk[NB];
            split_pieces2<NB>(bvf[pp][ct][2 * w], bvf[pp][ct][2 * w + 1], pk);
#pragma unroll
            for (int i = 0; i < NB; ++i) bw[i][w] = pk[i];
          }
#pragma unroll
          for (int i = 0; i < NB; ++i) bv[i][ct] = __builtin_bit_cast(bf8, bw[i]);
        }
#pragma unroll
        for (int qt = 0; qt < 4; ++qt) {
          bf8 av[NB];
#pragma unroll
          for (int i = 0; i < NB; ++i)
            av[i] = *reinterpret_cast<const bf8*>(&lam_b[i][pp][qt * 16 + (lane & 15)][k8]);
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            f4 c = acc[qt][ct][pp];
#pragma unroll
            for (int k = 0; k < Products<NB>::n; ++k)
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[Products<NB>::a[k]], bv[Products<NB>::b[k]][ct],
                                                          c, 0, 0, 0);
            acc[qt][ct][pp] = c;
          }
        }
      }
    }
    __syncthreads();
  }

  // lanes 2j and 2j + 1 (real and imaginary column of one map) swap values so that each
  // writes whole 16-byte entries: the even lane rows r = 0, 2, the odd lane rows r = 1, 3
  const int odd = lane & 1;
  const size_t pstride = gf_stride(lmax);
  float* const Fm = a.F + (size_t)m * 4;
#pragma unroll
  for (int qt = 0; qt < 4; ++qt)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int map = (cg * CW + ct * 16 + (lane & 15)) >> 1;
      const bool map_ok = map < a.nmaps;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float eA = acc[qt][ct][0][2 * i], eB = acc[qt][ct][0][2 * i + 1];
        const float oA = acc[qt][ct][1][2 * i], oB = acc[qt][ct][1][2 * i + 1];
        const float seA = swap_lane_pair(eA), seB = swap_lane_pair(eB);
        const float soA = swap_lane_pair(oA), soB = swap_lane_pair(oB);
        const float4 v = make_float4(odd ? seB : eA, odd ? eB : seA, odd ? soB : oA, odd ? oB : soA);
        const int q = q0 + qt * 16 + 4 * (lane >> 4) + 2 * i + odd;
        if (map_ok && q < nact) *reinterpret_cast<float4*>(Fm + ((size_t)map * P.npairs + q) * pstride) = v;
      }
    }
}

// ------------------------------------------------------------------ wide synthesis
// Work item (m, block of 256 ring pairs) and column group cg of 32 NT columns
// (16 NT maps, NT = 1 or 2 column tiles per wave): four waves, one per 64 ring pairs, each lane running the recurrence of its
// ring pair. 32 x 32 matrix tiles, M = 32 ring pairs, N = 32 columns, K = values of l
// of one parity. The A operand comes straight from the registers of the lanes that
// generated the values: lane l (ring l) and lane l + 32 (ring l + 32) exchange halves
// with v_permlane32_swap, which turns "my ring, all my values" into the fragments of
// both ring tiles. The B operand (the coefficients of a chunk of 32 l for the
// group's columns) is loaded once per chunk by the whole workgroup into LDS, split
// into bf16 pieces there for the bf16 modes, double buffered, and read by all four
// waves. The accumulators (2 ring tiles x NT column tiles x 2 parities, 64 NT
// registers) stay in matrix registers across the loop: the loop body is the same for
// every iteration (waves past the active ring pairs run a separate loop with the same
// barriers), so no copies between register files are needed.
//   FP32  v_mfma_f32_32x32x2f32     A: lane i + 32 k;  B: lane j + 32 k            (K = 2)
//   bf16  v_mfma_f32_32x32x16_bf16  A: lane i + 32 (k / 8), element k % 8; B likewise (K = 16)
//   D     lane j + 32 h, register r: row 8 (r / 4) + 4 h + r % 4, column j.
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void swap_halves(unsigned a, unsigned b, unsigned& lo, unsigned& hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  lo = r[0];   // lanes 0..31: a[l]; lanes 32..63: b[l - 32]
  hi = r[1];   // lanes 0..31: a[l + 32]; lanes 32..63: b[l]
}

template <int NP, int NT>
__global__ void __launch_bounds__(256) mfma_wide_synthesis_kernel(PlanDev P, const WorkItem* __restrict__ items,
                                                                  MfmaArgs a) {
  constexpr int WS_COLS = 32 * NT;
  constexpr bool F32 = (NP == 1);
  constexpr int NB = F32 ? 1 : NP;
  constexpr int HF = 17, HB = 24;     // padded stride of h (floats / bf16) per column
  __shared__ float lds_f[F32 ? 2 : 1][2][WS_COLS][F32 ? HF : 1];
  __shared__ __attribute__((aligned(16))) __bf16 lds_b[F32 ? 1 : 2][NB][2][WS_COLS][F32 ? 8 : HB];
  const WorkItem it = items[blockIdx.x];
  const int cg = blockIdx.y;
  const int m = it.m;
  if (m < 0) return;   // empty item of the XCD-ordered list
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lmax = P.lmax;
  const int nact = P.n_active[m];
  const int q0 = it.blk * 256 + wave * 64;
  const bool wave_on = q0 < nact;                 // uniform over the wave
  const int64_t roff = P.row_off[m];
  const double* __restrict__ Arow = P.A + roff;
  const int ncols = 2 * a.nmaps;
  const float* __restrict__ brow = a.bcoef + (size_t)roff * ncols;
  const int nl = lmax - m + 1;

  // cooperative B load: thread tid takes row lr of the chunk, columns lc .. lc + CPT - 1 of
  // the group (rows past lmax read the row's zero padding: a prefetch ends < 64 rows past it)
  constexpr int CPT = 4 * NT;
  const int lr = tid >> 3, lc = (tid & 7) * CPT;
  const int colg0 = cg * WS_COLS + lc;
  auto gload = [&](int i0, float (&v)[CPT]) {
    const float* src = brow + (size_t)(i0 + lr) * ncols + colg0;
#pragma unroll
    for (int e = 0; e < CPT; ++e) v[e] = (colg0 + e < ncols) ? src[e] : 0.0f;
  };
  auto lstore = [&](int buf, const float (&v)[CPT]) {
    const int pp = lr & 1, h = lr >> 1;
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
      if constexpr (F32) {
        lds_f[buf][pp][lc + e][h] = v[e];
      } else {
        __bf16 pc[NB];
        split_pieces<NB>(v[e], pc);
#pragma unroll
        for (int i = 0; i < NB; ++i) lds_b[buf][i][pp][lc + e][h] = pc[i];
      }
    }
  };

  Ring ring = ring_init(P, m, q0 + lane, nact);
  f16v acc[2][NT][2];   // [ring tile][column tile][parity]
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int pp = 0; pp < 2; ++pp) acc[t][n][pp] = f16v{};

  {
    float v[CPT];
    gload(0, v);
    lstore(0, v);
  }
  __syncthreads();
  if (!wave_on) {
    // a wave past the active ring pairs only helps stage the coefficients (same barriers)
    int buf = 0;
    for (int i0 = 0; i0 < nl; i0 += MCH) {
      float vn[CPT];
      const bool more = i0 + MCH < nl;
      if (more) {
        gload(i0 + MCH, vn);
        lstore(buf ^ 1, vn);
      }
      __syncthreads();
      buf ^= 1;
    }
    return;
  }
  int buf = 0;
  for (int i0 = 0; i0 < nl; i0 += MCH) {
    // prefetch the next chunk's coefficients (stored to the other buffer after the MFMAs)
    float vn[CPT];
    const bool more = i0 + MCH < nl;
    if (more) gload(i0 + MCH, vn);
    if constexpr (F32) {
      float ev[2][16];
      ring_steps(ring, Arow + i0, [&](int j, double v) { ev[j & 1][j >> 1] = (float)v; });
#pragma unroll
      for (int pp = 0; pp < 2; ++pp) {
        float bv[NT][8];
#pragma unroll
        for (int n = 0; n < NT; ++n)
#pragma unroll
          for (int s2 = 0; s2 < 8; ++s2) bv[n][s2] = lds_f[buf][pp][32 * n + (lane & 31)][2 * s2 + (lane >> 5)];
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) {
          unsigned t0, t1;
          swap_halves(__float_as_uint(ev[pp][2 * s2]), __float_as_uint(ev[pp][2 * s2 + 1]), t0, t1);
#pragma unroll
          for (int n = 0; n < NT; ++n) {
            acc[0][n][pp] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(t0), bv[n][s2], acc[0][n][pp], 0, 0, 0);
            acc[1][n][pp] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(t1), bv[n][s2], acc[1][n][pp], 0, 0, 0);
          }
        }
      }
    } else {
      float ev[2][16];   // [parity][value]
      ring_steps(ring, Arow + i0, [&](int j, double v) { ev[j & 1][j >> 1] = (float)v; });
#pragma unroll
      for (int pp = 0; pp < 2; ++pp) {
        // pieces of this parity's 16 values, two values per dword: dwords 0..3 hold values
        // 0..7, dwords 4..7 values 8..15
        unsigned pk[8][NB];
#pragma unroll
        for (int w = 0; w < 8; ++w) split_pieces2<NB>(ev[pp][2 * w], ev[pp][2 * w + 1], pk[w]);
        bf8 A0[NB], A1[NB], B[NT][NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
#pragma unroll
          for (int n = 0; n < NT; ++n)
            B[n][i] = *reinterpret_cast<const bf8*>(&lds_b[buf][i][pp][32 * n + (lane & 31)][8 * (lane >> 5)]);
          typedef unsigned u4 __attribute__((ext_vector_type(4)));
          u4 lo, hi;
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            unsigned l_, h_;
            swap_halves(pk[w][i], pk[4 + w][i], l_, h_);
            lo[w] = l_;
            hi[w] = h_;
          }
          A0[i] = __builtin_bit_cast(bf8, lo);
          A1[i] = __builtin_bit_cast(bf8, hi);
        }
#pragma unroll
        for (int k = 0; k < Products<NB>::n; ++k)
#pragma unroll
          for (int n = 0; n < NT; ++n) {
            acc[0][n][pp] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0[Products<NB>::a[k]], B[n][Products<NB>::b[k]],
                                                                    acc[0][n][pp], 0, 0, 0);
            acc[1][n][pp] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1[Products<NB>::a[k]], B[n][Products<NB>::b[k]],
                                                                    acc[1][n][pp], 0, 0, 0);
          }
      }
    }
    if (more) lstore(buf ^ 1, vn);
    __syncthreads();
    buf ^= 1;
  }

  // Lanes 2j and 2j + 1 hold the real and the imaginary column of one map for the same ring
  // pairs. They swap values (lane ^ 1) so that each writes whole 16-byte entries (E re, E im,
  // O re, O im): the even lane those of rows r = 0, 2, ..., 14, the odd lane those of rows
  // r = 1, 3, ..., 15 — a quarter of the stores, each of one entry.
  const int odd = lane & 1;
  const size_t pstride = gf_stride(lmax);
  float* const Fm = a.F + (size_t)m * 4;
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int map = (cg * WS_COLS + 32 * n + (lane & 31)) >> 1;
    const bool map_ok = map < a.nmaps;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const float eA = acc[t][n][0][2 * i], eB = acc[t][n][0][2 * i + 1];
        const float oA = acc[t][n][1][2 * i], oB = acc[t][n][1][2 * i + 1];
        const float seA = swap_lane_pair(eA), seB = swap_lane_pair(eB);
        const float soA = swap_lane_pair(oA), soB = swap_lane_pair(oB);
        const float4 v = make_float4(odd ? seB : eA, odd ? eB : seA, odd ? soB : oA, odd ? oB : soA);
        const int q = q0 + 32 * t + 8 * (i >> 1) + 4 * (lane >> 5) + 2 * (i & 1) + odd;
        if (map_ok && q < nact)
          *reinterpret_cast<float4*>(Fm + ((size_t)map * P.npairs + q) * pstride) = v;
      }
  }
}

// ------------------------------------------------------------------ coefficients
// Sum the analysis blocks (FP64), scale by C_l, apply the filter, emit the alm and
// the synthesis coefficients b = C_l s_lm in the layout [padded row][map][re/im].
// One thread per element e = r nmaps + map over the padded rows r of every m
// (rows r = row_off[m] + i, i < lmax - m + 1 + ROW_PAD; padding rows get zeros).
__device__ __forceinline__ void coeff_elem(const PlanDev& P, const MfmaArgs& a, const int64_t e, double* chi_acc) {
  const int nm = a.nmaps;
  const int64_t r = e / nm;
  const int map = (int)(e - r * nm);
  const int lmax = P.lmax;
  const int m = P.row_m[r];
  const int64_t roff = P.row_off[m];
  const int i = (int)(r - roff);
  const int nl = lmax - m + 1;
  double br = 0.0, bi = 0.0;
  if (i < nl) {
    const int64_t row = alm_index(lmax, m, m);
    const double c = P.C[roff + i];
    double sr, si;
    if (a.mode == SY_FROM_ALM) {
      const float2 v = a.alm_in[(size_t)map * P.nalm + row + i];
      sr = v.x;
      si = (m == 0) ? 0.0 : v.y;
    } else {
      const int nb = (P.n_active[m] + a.ana_rb - 1) / a.ana_rb;
      sr = si = 0.0;
      // the blocks' partial sums, KB at a time with their loads issued together
      constexpr int KB = 4;
      const float* pbase = a.partial + ((size_t)(row + i) * nm + map) * 2;
      const size_t kstride = (size_t)P.nalm * nm * 2;
      for (int k0 = 0; k0 < nb; k0 += KB) {
        float2 pk[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u)
          pk[u] = k0 + u < nb ? *reinterpret_cast<const float2*>(pbase + (size_t)(k0 + u) * kstride)
                              : make_float2(0.0f, 0.0f);
#pragma unroll
        for (int u = 0; u < KB; ++u) {
          sr += pk[u].x;
          si += pk[u].y;
        }
      }
      sr *= c;
      si *= c;
      if (a.mode == SY_FROM_PARTIAL) {
        const double lam_t_o = a.slots ? a.slots[map].lam_t_o : a.lambda * P.tau * P.omega;
        const double cl = (P.cl + (a.slots ? map * a.cl_stride : 0))[m + i];
        const double f = cl > 0.0 ? cl / (cl + lam_t_o) : 0.0;
        sr *= f;
        si *= f;
        if (cl > 0.0) *chi_acc = (m == 0 ? 1.0 : 2.0) * (sr * sr + si * si) / cl;
      }
    }
    if (a.alm_out) a.alm_out[(size_t)map * P.nalm + row + i] = make_float2((float)sr, (float)si);
    br = sr * c;
    bi = si * c;
  }
  if (a.mode != SY_ALM_ONLY)
    *reinterpret_cast<float2*>(a.bcoef + ((size_t)r * nm + map) * 2) = make_float2((float)br, (float)bi);
}

// ------------------------------------------------------------------ kernels
template <int NP, int CT>
__global__ void __launch_bounds__(128 * CT) mfma_analysis_kernel(PlanDev P, const WorkItem* __restrict__ items,
                                                                 MfmaArgs a) {
  analysis_body<NP, CT>(P, a, items[blockIdx.x], blockIdx.y);
}

template <int NP, int NCT>
__global__ void __launch_bounds__(64) mfma_synthesis_kernel(PlanDev P, const WorkItem* __restrict__ items,
                                                            MfmaArgs a) {
  synthesis_body<NP, NCT>(P, a, items[blockIdx.x], blockIdx.y);
}

// chi^2 prior term of the elements of one workgroup, added per map into the
// workgroup's slot of the term: through an LDS entry per map when the maps fit in
// one workgroup, else one global atomic per element.
__device__ __forceinline__ void coeff_chi2(const MfmaArgs& a, int64_t e, bool valid, double v) {
  __shared__ double macc[COEFF_THREADS];
  const int nm = a.nmaps;
  const int map = (int)(e % nm);
  const int slot = (blockIdx.x % CHI_SLOTS) * CHI_SLOT_STRIDE;
  if (nm <= COEFF_THREADS) {
    if (threadIdx.x < nm) macc[threadIdx.x] = 0.0;
    __syncthreads();
    if (valid && v != 0.0) atomicAdd(&macc[map], v);
    __syncthreads();
    if ((int)threadIdx.x < nm && macc[threadIdx.x] != 0.0)
      atomicAdd(a.chi2 + threadIdx.x * a.chi2_stride + slot, macc[threadIdx.x]);
  } else if (valid && v != 0.0) {
    atomicAdd(a.chi2 + map * a.chi2_stride + slot, v);
  }
}

__global__ void __launch_bounds__(COEFF_THREADS) mfma_coeff_kernel(PlanDev P, MfmaArgs a) {
  const int64_t e = (int64_t)blockIdx.x * COEFF_THREADS + threadIdx.x;
  const bool valid = e < P.rows_total * a.nmaps;
  double v = 0.0;
  if (valid) coeff_elem(P, a, e, &v);
  if (a.chi2 != nullptr && a.mode == SY_FROM_PARTIAL) coeff_chi2(a, e, valid, v);
}

__device__ __forceinline__ MfmaArgs task_args(const TaskDev& t, int ana_rb) {
  MfmaArgs a{};
  a.mode = t.sy_mode;
  a.nmaps = t.nmaps;
  a.lambda = t.lambda;
  a.ana_rb = ana_rb;
  a.G = static_cast<const float*>(t.G);
  a.F = static_cast<float*>(t.F);
  a.partial = t.partial;
  a.bcoef = t.bcoef;
  a.alm_in = t.alm_in;
  a.alm_out = t.alm_out;
  a.slots = t.slots;
  a.cl_stride = t.cl_stride;
  return a;
}

template <int NP, int CT>
__global__ void __launch_bounds__(128 * CT) group_analysis_kernel(GroupArgs g) {
  const int t = group_task_of(g, blockIdx.x);
  const TaskDev& T = g.t[t];
  const int64_t local = blockIdx.x - g.offs[t];
  const int ncg = (2 * T.nmaps + 16 * CT - 1) / (16 * CT);
  const WorkItem* items = CT == 1 ? T.items_a128 : T.items_a256;
  analysis_body<NP, CT>(T.P, task_args(T, ana_block(CT)), items[local / ncg], (int)(local % ncg));
}

template <int NP, int NCT>
__global__ void __launch_bounds__(64) group_synthesis_kernel(GroupArgs g, int ana_rb) {
  const int t = group_task_of(g, blockIdx.x);
  const TaskDev& T = g.t[t];
  const int64_t local = blockIdx.x - g.offs[t];
  const int ncg = (2 * T.nmaps + 16 * NCT - 1) / (16 * NCT);
  synthesis_body<NP, NCT>(T.P, task_args(T, ana_rb), T.items_s64[local / ncg], (int)(local % ncg));
}

__global__ void __launch_bounds__(COEFF_THREADS) group_coeff_kernel(GroupArgs g, int ana_rb) {
  const int t = group_task_of(g, blockIdx.x);
  const TaskDev& T = g.t[t];
  const int64_t e = (blockIdx.x - g.offs[t]) * COEFF_THREADS + threadIdx.x;
  double v = 0.0;
  if (e < T.P.rows_total * T.nmaps) coeff_elem(T.P, task_args(T, ana_rb), e, &v);
}

template <int NP>
hipError_t ana_np(const PlanDev& P, const WorkItem* items, int nitems, int ct, const MfmaArgs& a,
                  hipStream_t s) {
  const dim3 grid(nitems, (2 * a.nmaps + 16 * ct - 1) / (16 * ct));
  switch (ct) {
    case 1: hipLaunchKernelGGL((mfma_analysis_kernel<NP, 1>), grid, dim3(128), 0, s, P, items, a); break;
    case 2: hipLaunchKernelGGL((mfma_analysis_kernel<NP, 2>), grid, dim3(256), 0, s, P, items, a); break;
    case 4: hipLaunchKernelGGL((mfma_analysis_kernel<NP, 4>), grid, dim3(512), 0, s, P, items, a); break;
    case 8:
      if constexpr (NP == 1) {
        hipLaunchKernelGGL((mfma_analysis_kernel<NP, 8>), grid, dim3(1024), 0, s, P, items, a);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int NP>
hipError_t syn_np(const PlanDev& P, const WorkItem* items, int nitems, int nct, const MfmaArgs& a,
                  hipStream_t s) {
  const int cw = 16 * nct;
  const dim3 grid(nitems, (2 * a.nmaps + cw - 1) / cw);
  if (nct == 1)
    hipLaunchKernelGGL((mfma_synthesis_kernel<NP, 1>), grid, dim3(64), 0, s, P, items, a);
  else if (nct == 2)
    hipLaunchKernelGGL((mfma_synthesis_kernel<NP, 2>), grid, dim3(64), 0, s, P, items, a);
  else if (nct == 4)
    hipLaunchKernelGGL((mfma_synthesis_kernel<NP, 4>), grid, dim3(64), 0, s, P, items, a);
  else if constexpr (NP == 1) {
    if (nct != 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL((mfma_synthesis_kernel<NP, 8>), grid, dim3(64), 0, s, P, items, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int NP>
hipError_t gana_np(const GroupLaunch& g, int ct, hipStream_t s) {
  return for_each_group_part(g, [&](const GroupArgs& a, int64_t nb) {
    switch (ct) {
      case 1: hipLaunchKernelGGL((group_analysis_kernel<NP, 1>), dim3(nb), dim3(128), 0, s, a); break;
      case 2: hipLaunchKernelGGL((group_analysis_kernel<NP, 2>), dim3(nb), dim3(256), 0, s, a); break;
      case 4: hipLaunchKernelGGL((group_analysis_kernel<NP, 4>), dim3(nb), dim3(512), 0, s, a); break;
      case 8:
        if constexpr (NP == 1) {
          hipLaunchKernelGGL((group_analysis_kernel<NP, 8>), dim3(nb), dim3(1024), 0, s, a);
          break;
        }
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

template <int NP>
hipError_t gsyn_np(const GroupLaunch& g, int nct, int ana_rb, hipStream_t s) {
  if (nct != 1 && nct != 2 && nct != 4 && !(NP == 1 && nct == 8)) return hipErrorInvalidValue;
  return for_each_group_part(g, [&](const GroupArgs& a, int64_t nb) {
    if (nct == 1)
      hipLaunchKernelGGL((group_synthesis_kernel<NP, 1>), dim3(nb), dim3(64), 0, s, a, ana_rb);
    else if (nct == 2)
      hipLaunchKernelGGL((group_synthesis_kernel<NP, 2>), dim3(nb), dim3(64), 0, s, a, ana_rb);
    else if (nct == 4)
      hipLaunchKernelGGL((group_synthesis_kernel<NP, 4>), dim3(nb), dim3(64), 0, s, a, ana_rb);
    else if constexpr (NP == 1)
      hipLaunchKernelGGL((group_synthesis_kernel<NP, 8>), dim3(nb), dim3(64), 0, s, a, ana_rb);
    return hipGetLastError();
  });
}

}  // namespace

hipError_t launch_mfma_analysis(const PlanDev& P, const WorkItem* items, int nitems, int mode, int ct,
                                const MfmaArgs& a, hipStream_t s) {
  if (mode == WF_BF16X3) return ana_np<2>(P, items, nitems, ct, a, s);
  if (mode == WF_BF16X6) return ana_np<3>(P, items, nitems, ct, a, s);
  return ana_np<1>(P, items, nitems, ct, a, s);
}

hipError_t launch_mfma_coeff(const PlanDev& P, const MfmaArgs& a, hipStream_t s) {
  const int64_t n = P.rows_total * a.nmaps;
  hipLaunchKernelGGL(mfma_coeff_kernel, dim3((unsigned)((n + COEFF_THREADS - 1) / COEFF_THREADS)),
                     dim3(COEFF_THREADS), 0, s, P, a);
  return hipGetLastError();
}

template <int NT>
hipError_t wide_nt(const PlanDev& P, const WorkItem* items256, int nitems, int mode, const MfmaArgs& a,
                   hipStream_t s) {
  const dim3 grid(nitems, (2 * a.nmaps + 32 * NT - 1) / (32 * NT));
  if (mode == WF_BF16X3)
    hipLaunchKernelGGL((mfma_wide_synthesis_kernel<2, NT>), grid, dim3(256), 0, s, P, items256, a);
  else if (mode == WF_BF16X6)
    hipLaunchKernelGGL((mfma_wide_synthesis_kernel<3, NT>), grid, dim3(256), 0, s, P, items256, a);
  else
    hipLaunchKernelGGL((mfma_wide_synthesis_kernel<1, NT>), grid, dim3(256), 0, s, P, items256, a);
  return hipGetLastError();
}

hipError_t launch_mfma_wide_synthesis(const PlanDev& P, const WorkItem* items256, int nitems, int mode, int nt,
                                      const MfmaArgs& a, hipStream_t s) {
  if (nt == 1) return wide_nt<1>(P, items256, nitems, mode, a, s);
  if (nt == 2) return wide_nt<2>(P, items256, nitems, mode, a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_mfma_synthesis(const PlanDev& P, const WorkItem* items, int nitems, int mode, int nct,
                                 const MfmaArgs& a, hipStream_t s) {
  if (mode == WF_BF16X3) return syn_np<2>(P, items, nitems, nct, a, s);
  if (mode == WF_BF16X6) return syn_np<3>(P, items, nitems, nct, a, s);
  return syn_np<1>(P, items, nitems, nct, a, s);
}

hipError_t launch_group_analysis(const GroupLaunch& g, int mode, int ct, hipStream_t s) {
  if (g.nblocks == 0) return hipSuccess;
  if (mode == WF_BF16X3) return gana_np<2>(g, ct, s);
  if (mode == WF_BF16X6) return gana_np<3>(g, ct, s);
  return gana_np<1>(g, ct, s);
}

hipError_t launch_group_coeff(const GroupLaunch& g, int ana_rb, hipStream_t s) {
  if (g.nblocks == 0) return hipSuccess;
  return for_each_group_part(g, [&](const GroupArgs& a, int64_t nb) {
    hipLaunchKernelGGL(group_coeff_kernel, dim3(nb), dim3(COEFF_THREADS), 0, s, a, ana_rb);
    return hipGetLastError();
  });
}

hipError_t launch_group_synthesis(const GroupLaunch& g, int mode, int nct, int ana_rb, hipStream_t s) {
  if (g.nblocks == 0) return hipSuccess;
  if (mode == WF_BF16X3) return gsyn_np<2>(g, nct, ana_rb, s);
  if (mode == WF_BF16X6) return gsyn_np<3>(g, nct, ana_rb, s);
  return gsyn_np<1>(g, nct, ana_rb, s);
}

}  // namespace mwf
