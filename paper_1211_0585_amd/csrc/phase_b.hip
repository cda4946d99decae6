// Phase B of a messenger sweep: ring-parallel work in pixel space.
//
// One workgroup handles one pair of mirror rings (north ring i, south ring
// 4 nside - i), which share n_phi and the longitude phi0 of pixel 0, for one map.
// The two real rings are packed into one complex sequence z_j = x_N[j] + i x_S[j],
// so each direction costs a single complex FFT of length n_phi, staged in LDS:
//
//   synthesis  F_N(m) = E(m) + O(m), F_S(m) = E(m) - O(m) from the Legendre phase;
//              bins B[k] = sum over m = -lmax..lmax with m = k (mod n_phi) of
//              F(m) exp(i m phi0), F(-m) = conj F(m)  (aliasing on short rings);
//              x_j = sum_k B[k] exp(+2 pi i j k / n_phi)
//   update     Eq. (3) per pixel: t = s + w (d - s),
//              w = lambda tau ninv / (1 + (lambda - 1) tau ninv)
//   analysis   X[k] = sum_j t_j exp(-2 pi i j k / n_phi);
//              G(m) = Omega exp(-i m phi0) X[m mod n_phi], m = 0..lmax, written as
//              S = G_N + G_S and D = G_N - G_S for the Legendre phase.
//
// HEALPix rings have phi0 = pi ph_num / n_phi with ph_num in {0, 1}, so
// exp(i n_phi phi0) = (-1)^ph_num: the phases of all aliases of a bin follow from
// one exp(i k phi0).
//
// Ring lengths are 4 i (polar caps) or 4 nside (belt). Powers of two use an
// in-place Stockham FFT (radix 8, with radix-4 passes for log2 n not a multiple
// of 3) whose butterflies are staged in registers between two barriers per pass.
// Lengths 2^a 3^b 5^c 7^d use the same Stockham FFT with mixed radices: the radix-2/4/8
// passes over the whole length, then radix-3, 5 and 7 passes. Lengths with a larger
// prime factor use Bluestein's chirp-z method: chirp, power-of-two FFT of length
// M >= 2 n - 1, multiply by the plan-time filter spectrum, inverse FFT, chirp.
// The FFT arithmetic type C is double for FP64 plans and float for plans that
// store maps and ring coefficients in float. Ring pairs are launched in classes:
// rings that are not a power of two (mixed radix and Bluestein) and power-of-two rings
// separately (512 and 256 threads, LDS sized to the class: the Bluestein length is about
// twice the ring's, and a mixed-radix ring counts twice its length), and, from 4 maps
// on, transforms of at most 1024 points one wave per ring pair, so short polar
// rings do not leave most of a large workgroup idle. Each workgroup stages the
// twiddles of its ring's transform in LDS next to the data, one table per pass
// read by consecutive lanes at consecutive entries, and the data sit in a padded
// layout between passes: both keep the passes' LDS accesses off shared banks.
#include <map>
#include <mutex>
#include <utility>

#include "mwf_internal.hpp"

namespace mwf {
namespace {

// Rings of at most FOLD_PARTS points fold their aliases with FOLD_PARTS / n partial
// sums per bin (see the loading step of phase_b_body).
constexpr int FOLD_PARTS = 256;


template <class C>
struct CT;
template <>
struct CT<double> {
  using V = double2;
  __device__ static V make(double x, double y) { return make_double2(x, y); }
};
template <>
struct CT<float> {
  using V = float2;
  __device__ static V make(float x, float y) { return make_float2(x, y); }
};

template <class V>
__device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <class V>
__device__ __forceinline__ V cadd(V a, V b) {
  V r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <class V>
__device__ __forceinline__ V csub(V a, V b) {
  V r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
template <class V>
__device__ __forceinline__ V cconj(V a) {
  a.y = -a.y;
  return a;
}
// multiply by i * s (s = +1 or -1)
template <class V, class S>
__device__ __forceinline__ V cmul_is(V a, S s) {
  V r;
  r.x = -s * a.y;
  r.y = s * a.x;
  return r;
}

// exp(i pi num / den) with the argument reduced exactly (in FP64, then rounded to C).
template <class C>
__device__ __forceinline__ typename CT<C>::V expipi(int64_t num, int64_t den) {
  int64_t r = num % (2 * den);
  if (r < 0) r += 2 * den;
  double s, c;
  sincospi((double)r / (double)den, &s, &c);
  return CT<C>::make((C)c, (C)s);
}

// Radix-4 DFT of v[0..3] in registers (sd = -1 forward, +1 inverse).
template <class V, class S>
__device__ __forceinline__ void dft4(V& v0, V& v1, V& v2, V& v3, S sd) {
  const V t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = cmul_is(csub(v1, v3), sd);
  v0 = cadd(t0, t2);
  v1 = cadd(t1, t3);
  v2 = csub(t0, t2);
  v3 = csub(t1, t3);
}

// Radix-8 DFT of v[0..7] in registers (sd = -1 forward, +1 inverse): two radix-4
// DFTs of the even and odd inputs, joined with the eighth roots of unity.
template <class V, class S>
__device__ __forceinline__ void dft8(V* v, S sd) {
  V e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  V o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3, sd);
  dft4(o0, o1, o2, o3, sd);
  const S c = (S)0.70710678118654752440;
  // o1 *= exp(sd i pi/4) = c (1 + i sd), o2 *= i sd, o3 *= exp(3 sd i pi/4) = c (-1 + i sd)
  V t1, t3;
  t1.x = c * (o1.x - sd * o1.y);
  t1.y = c * (o1.y + sd * o1.x);
  t3.x = c * (-o3.x - sd * o3.y);
  t3.y = c * (sd * o3.x - o3.y);
  const V t2 = cmul_is(o2, sd);
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

// cos and sin of 2 pi s / R, s = 1 .. (R - 1) / 2, for the odd radices.
template <int R>
struct OddRoots;
template <>
struct OddRoots<3> {
  static constexpr double c[1] = {-0.5};
  static constexpr double s[1] = {0.866025403784438646764};
};
template <>
struct OddRoots<5> {
  static constexpr double c[2] = {0.309016994374947424102, -0.809016994374947424102};
  static constexpr double s[2] = {0.951056516295153572116, 0.587785252292473129169};
};
template <>
struct OddRoots<7> {
  static constexpr double c[3] = {0.623489801858733530525, -0.222520933956314404289, -0.900968867902419126236};
  static constexpr double s[3] = {0.781831482468029808708, 0.974927912181823607018, 0.433883739117558120476};
};

// Radix-R DFT of u[0..R-1] in registers for odd R (sd = -1 forward, +1 inverse), by the
// symmetric pairs a_r = u_r + u_{R-r}, b_r = u_r - u_{R-r}, r = 1 .. H = (R - 1) / 2:
//   y_0 = u_0 + sum_r a_r,  y_s, y_{R-s} = u_0 + sum_r a_r cos(2 pi r s / R)
//                                         +- i sd sum_r b_r sin(2 pi r s / R).
template <int R, class V, class S>
__device__ __forceinline__ void dft_odd(V* u, S sd) {
  constexpr int H = (R - 1) / 2;
  V a[H], b[H];
#pragma unroll
  for (int r = 1; r <= H; ++r) {
    a[r - 1] = cadd(u[r], u[R - r]);
    b[r - 1] = csub(u[r], u[R - r]);
  }
  V y[R];
  y[0] = u[0];
#pragma unroll
  for (int r = 1; r <= H; ++r) y[0] = cadd(y[0], a[r - 1]);
#pragma unroll
  for (int t = 1; t <= H; ++t) {
    V A = u[0], B = {0, 0};
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      const int m = (r * t) % R;                       // cos / sin of 2 pi m / R
      const S c = (S)OddRoots<R>::c[(m <= H ? m : R - m) - 1];
      const S sn = (S)(m <= H ? OddRoots<R>::s[m - 1] : -OddRoots<R>::s[R - m - 1]);
      A.x += c * a[r - 1].x;
      A.y += c * a[r - 1].y;
      B.x += sn * b[r - 1].x;
      B.y += sn * b[r - 1].y;
    }
    const V iB = cmul_is(B, sd);
    y[t] = cadd(A, iB);
    y[R - t] = csub(A, iB);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) u[r] = y[r];
}

// One radix-R pass (R = 2, 4 or 8) of an in-place Stockham FFT of length L in LDS,
// after Ns points have been combined: butterfly j (j < L / R, k = j mod Ns) takes
// input r < R from element j + r L / R, multiplies it by w^r with w = exp(dir 2 pi i
// k / (R Ns)), takes its radix-R DFT and writes output r to element (j - k) R + k +
// r Ns. NBF butterflies per thread; all inputs are read into registers before the
// barrier that precedes the writes, so one buffer suffices and the layout may change
// from pass to pass: element e sits at e (plain) or at fft_padded-style e + e / 16
// (pad_in / pad_out), the padding that spreads the strided writes of the early
// passes over the LDS banks. wk[k] = exp(-2 pi i k / (R Ns)), k < Ns: this pass's
// twiddles, read by consecutive lanes at consecutive entries; the other powers are
// products of it (at most three deep).
template <class C, int NT, int R, int NBF>
__device__ __forceinline__ void stockham_pass(typename CT<C>::V* x, int L, int Ns, int dir, bool pad_in,
                                              bool pad_out, const typename CT<C>::V* __restrict__ wk) {
  using V = typename CT<C>::V;
  const int tid = threadIdx.x;
  const C sd = (C)dir;
  const int nb = L / R;
  auto at = [](int e, bool pad) { return pad ? e + (e >> 4) : e; };
  V v[R * NBF];
#pragma unroll
  for (int b = 0; b < NBF; ++b) {
    const int j = tid + b * NT;
    if (j < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[R * b + r] = x[at(j + r * nb, pad_in)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NBF; ++b) {
    const int j = tid + b * NT;
    if (j < nb) {
      const int k = j & (Ns - 1);
      V* u = v + R * b;
      if (Ns > 1) {
        V w = wk[k];
        if (dir > 0) w.y = -w.y;
        u[1] = cmul(u[1], w);
        if (R >= 4) {
          const V w2 = cmul(w, w), w3 = cmul(w, w2);
          u[2] = cmul(u[2], w2);
          u[3] = cmul(u[3], w3);
          if (R == 8) {
            const V w4 = cmul(w2, w2);
            u[4] = cmul(u[4], w4);
            u[5] = cmul(u[5], cmul(w, w4));
            u[6] = cmul(u[6], cmul(w2, w4));
            u[7] = cmul(u[7], cmul(w3, w4));
          }
        }
      }
      if (R == 2) {
        const V a0 = u[0];
        u[0] = cadd(a0, u[1]);
        u[1] = csub(a0, u[1]);
      } else if (R == 4) {
        dft4(u[0], u[1], u[2], u[3], sd);
      } else {
        dft8(u, sd);
      }
      const int idx = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) x[at(idx + r * Ns, pad_out)] = u[r];
    }
  }
  __syncthreads();
}

// In-place Stockham FFT of length L = 2^lg (2 <= L <= 4 MAXB NT) in LDS, run by
// all NT threads of the workgroup; dir = -1: exp(-2 pi i jk/L), +1: exp(+...).
// Unnormalised. Passes as fft_schedule gives them (radix 8 as far as lg allows, the
// smaller radices first). Input and output are in the plain layout; between passes
// the data sit in the padded one, so the buffer holds fft_padded(L) elements. wt:
// the per-pass twiddle tables in pass order (fft_twiddle_entries(lg) entries, see
// twiddle_glob_index). The caller synchronises before the call; the last pass ends
// with a barrier.
template <class C, int NT, int MAXB>
__device__ __forceinline__ void fft_pow2(typename CT<C>::V* x, int lg, int dir,
                                         const typename CT<C>::V* __restrict__ wt) {
  constexpr int NB8 = (MAXB + 1) / 2;   // radix-8 butterflies per thread: L / 8 <= NB8 NT
  const int L = 1 << lg;
  int n2, n4, n8;
  fft_schedule(lg, &n2, &n4, &n8);
  const int last = n2 + n4 + n8 - 1;
  int Ns = 1, p = 0, off = 0;
  auto next = [&](int R) {
    off += Ns > 1 ? Ns : 0;
    Ns *= R;
    ++p;
  };
  if (n2) {
    stockham_pass<C, NT, 2, 2 * MAXB>(x, L, Ns, dir, p > 0, p < last, wt + off);
    next(2);
  }
  for (int q = 0; q < n4; ++q) {
    stockham_pass<C, NT, 4, MAXB>(x, L, Ns, dir, p > 0, p < last, wt + off);
    next(4);
  }
  for (int q = 0; q < n8; ++q) {
    stockham_pass<C, NT, 8, NB8>(x, L, Ns, dir, p > 0, p < last, wt + off);
    next(8);
  }
}

// One odd radix-R pass (R = 3, 5 or 7) of a mixed-radix Stockham FFT of length L, the
// same butterflies, index map and layouts as stockham_pass with k = j mod Ns for any Ns;
// the powers w^r = exp(dir 2 pi i r k / (R Ns)) are read from T[t] = exp(-2 pi i t / L)
// at t = r k L / (R Ns) (tstride = L / (R Ns); conjugated for dir = +1).
template <class C, int NT, int R, int NBF>
__device__ __forceinline__ void stockham_pass_odd(typename CT<C>::V* x, int L, int Ns, int dir, bool pad_in,
                                                  bool pad_out, const typename CT<C>::V* __restrict__ T,
                                                  int tstride) {
  using V = typename CT<C>::V;
  const int tid = threadIdx.x;
  const C sd = (C)dir;
  const int nb = L / R;
  auto at = [](int e, bool pad) { return pad ? e + (e >> 4) : e; };
  V v[R * NBF];
#pragma unroll
  for (int b = 0; b < NBF; ++b) {
    const int j = tid + b * NT;
    if (j < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[R * b + r] = x[at(j + r * nb, pad_in)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NBF; ++b) {
    const int j = tid + b * NT;
    if (j < nb) {
      const int k = j % Ns;
      V* u = v + R * b;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        V w = T[r * k * tstride];
        if (dir > 0) w.y = -w.y;
        u[r] = cmul(u[r], w);
      }
      dft_odd<R>(u, sd);
      const int idx = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) x[at(idx + r * Ns, pad_out)] = u[r];
    }
  }
  __syncthreads();
}

// In-place mixed-radix Stockham FFT of n = 2^a 3^b 5^c 7^d points (mix = b | c << 4 |
// d << 8) in LDS: the radix-2/4/8 passes of a 2^a-point transform over the whole length
// (their twiddles, which depend only on R Ns, are wt as for fft_pow2 of a), then b radix-3,
// c radix-5 and d radix-7 passes (twiddles from T[t] = exp(-2 pi i t / n)). Layouts,
// direction and synchronisation as fft_pow2; n <= 4 MAXB NT.
template <class C, int NT, int MAXB>
__device__ __forceinline__ void fft_mixed(typename CT<C>::V* x, int n, int mix, int dir,
                                          const typename CT<C>::V* __restrict__ wt,
                                          const typename CT<C>::V* __restrict__ T) {
  constexpr int NB8 = (MAXB + 1) / 2;
  const int lg = __ffs(n) - 1;
  int n2, n4, n8;
  fft_schedule(lg, &n2, &n4, &n8);
  const int n3 = mix & 15, n5 = (mix >> 4) & 15, n7 = (mix >> 8) & 15;
  const int last = n2 + n4 + n8 + n3 + n5 + n7 - 1;
  int Ns = 1, p = 0, off = 0;
  auto next = [&](int R) {
    off += Ns > 1 ? Ns : 0;
    Ns *= R;
    ++p;
  };
  if (n2) {
    stockham_pass<C, NT, 2, 2 * MAXB>(x, n, Ns, dir, p > 0, p < last, wt + off);
    next(2);
  }
  for (int q = 0; q < n4; ++q) {
    stockham_pass<C, NT, 4, MAXB>(x, n, Ns, dir, p > 0, p < last, wt + off);
    next(4);
  }
  for (int q = 0; q < n8; ++q) {
    stockham_pass<C, NT, 8, NB8>(x, n, Ns, dir, p > 0, p < last, wt + off);
    next(8);
  }
  for (int q = 0; q < n3; ++q) {
    stockham_pass_odd<C, NT, 3, (4 * MAXB + 2) / 3>(x, n, Ns, dir, p > 0, p < last, T, n / (3 * Ns));
    Ns *= 3;
    ++p;
  }
  for (int q = 0; q < n5; ++q) {
    stockham_pass_odd<C, NT, 5, (4 * MAXB + 4) / 5>(x, n, Ns, dir, p > 0, p < last, T, n / (5 * Ns));
    Ns *= 5;
    ++p;
  }
  for (int q = 0; q < n7; ++q) {
    stockham_pass_odd<C, NT, 7, (4 * MAXB + 6) / 7>(x, n, Ns, dir, p > 0, p < last, T, n / (7 * Ns));
    Ns *= 7;
    ++p;
  }
}

// Plan-table index of entry e of the per-pass twiddle tables of a 2^lg-point
// transform: for each pass with Ns > 1 (in pass order), entries off + k, k < Ns, hold
// exp(-2 pi i k / (R Ns)) = glob[k glob_len / (R Ns)] of the plan's table glob[t] =
// exp(-2 pi i t / glob_len), t < glob_len / 2.
__device__ __forceinline__ int twiddle_glob_index(int lg, int e, int glob_len) {
  int n2, n4, n8;
  fft_schedule(lg, &n2, &n4, &n8);
  int Ns = 1, off = 0;
  for (int p = 0; p < n2 + n4 + n8; ++p) {
    const int R = p < n2 ? 2 : (p < n2 + n4 ? 4 : 8);
    if (Ns > 1) {
      if (e < off + Ns) return (e - off) * (glob_len / (R * Ns));
      off += Ns;
    }
    Ns *= R;
  }
  return 0;
}

// This thread's share of a ring's Bluestein chirp (cj[u] = chirp[tid + u NT], j < n)
// and filter spectrum (hk[u] = H[tid + u NT], k < M), in registers.
template <class C, int NT, int MAXB>
struct BlueRegs {
  static constexpr int NK = 4 * MAXB;     // M <= 4 MAXB NT
  static constexpr int NJ = 2 * MAXB;     // n <= M / 2
  typename CT<C>::V cj[NJ], hk[NK];
  __device__ __forceinline__ void load(int n, int M, const typename CT<C>::V* __restrict__ chirp,
                                       const typename CT<C>::V* __restrict__ H) {
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
      const int j = threadIdx.x + u * NT;
      if (j < n) cj[u] = chirp[j];
    }
#pragma unroll
    for (int u = 0; u < NK; ++u) {
      const int k = threadIdx.x + u * NT;
      if (k < M) hk[u] = H[k];
    }
  }
};

template <class C, int NT, int MAXB>
__device__ void dft_bluestein(typename CT<C>::V* x, int n, int M, int lgM, int dir,
                              const BlueRegs<C, NT, MAXB>& br,
                              const typename CT<C>::V* __restrict__ wt) {
  using V = typename CT<C>::V;
  constexpr int NK = BlueRegs<C, NT, MAXB>::NK;
  constexpr int NJ = BlueRegs<C, NT, MAXB>::NJ;
  const int tid = threadIdx.x;
  const V(&cj)[NJ] = br.cj;
  const V(&hk)[NK] = br.hk;
#pragma unroll
  for (int u = 0; u < NK; ++u) {
    const int j = tid + u * NT;
    if (j < M) {
      if (u < NJ && j < n) {
        V v = x[j];
        if (dir > 0) v = cconj(v);     // inverse DFT = conj(DFT(conj(x)))
        x[j] = cmul(v, cj[u < NJ ? u : 0]);
      } else {
        x[j] = CT<C>::make(0, 0);
      }
    }
  }
  __syncthreads();
  fft_pow2<C, NT, MAXB>(x, lgM, -1, wt);
#pragma unroll
  for (int u = 0; u < NK; ++u) {
    const int k = tid + u * NT;
    if (k < M) x[k] = cmul(x[k], hk[u]);
  }
  __syncthreads();
  fft_pow2<C, NT, MAXB>(x, lgM, +1, wt);
  const C invM = (C)1 / (C)M;
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int k = tid + u * NT;
    if (k < n) {
      V v = cmul(x[k], cj[u]);
      v.x *= invM;
      v.y *= invM;
      if (dir > 0) v = cconj(v);
      x[k] = v;
    }
  }
  __syncthreads();
}

// Plan tables in the FFT arithmetic type.
template <class C>
struct Tabs;
template <>
struct Tabs<double> {
  __device__ static const double2* tw(const PlanDev& P) { return P.twiddle; }
  __device__ static const double2* chirp(const PlanDev& P) { return P.chirp; }
  __device__ static const double2* blue(const PlanDev& P) { return P.bluestein; }
  __device__ static const double2* mix(const PlanDev& P) { return P.mixtw; }
};
template <>
struct Tabs<float> {
  __device__ static const float2* tw(const PlanDev& P) { return P.twiddle32; }
  __device__ static const float2* chirp(const PlanDev& P) { return P.chirp32; }
  __device__ static const float2* blue(const PlanDev& P) { return P.bluestein32; }
  __device__ static const float2* mix(const PlanDev& P) { return P.mixtw32; }
};

// The ring's transform (n points, mixed radix over n, or Bluestein over M), with the
// per-pass twiddles of its power-of-two length (n, the 2^a of a mixed-radix length, or M)
// staged in LDS (twl). KIND 0: the launch holds only power-of-two rings, 1: only rings
// that are not (mixed radix and Bluestein, n at most half the class length), 2: any.
// The Bluestein chirp and filter spectrum are loaded per transform (held across the
// workgroup they cost occupancy).
template <class C, int NT, int MAXB, int KIND>
__device__ __forceinline__ void ring_dft(typename CT<C>::V* buf, const typename CT<C>::V* twl,
                                         const RingPair& rp, int dir, const PlanDev& P) {
  if (KIND != 1 && rp.log2n >= 0) {
    fft_pow2<C, NT, MAXB>(buf, rp.log2n, dir, twl);
  } else if (KIND != 0 && rp.mix != 0) {
    fft_mixed<C, NT, MAXB>(buf, rp.nphi, rp.mix, dir, twl, Tabs<C>::mix(P) + rp.bl_off);
  } else {
    if constexpr (KIND != 0) {
      BlueRegs<C, NT, MAXB> br;
      br.load(rp.nphi, rp.bl_M, Tabs<C>::chirp(P) + rp.chirp_off, Tabs<C>::blue(P) + rp.bl_off);
      dft_bluestein<C, NT, MAXB>(buf, rp.nphi, rp.bl_M, __ffs(rp.bl_M) - 1, dir, br, twl);
    }
  }
}

// log2 of the power-of-two transform whose per-pass twiddles a ring stages: n, the 2^a
// of a mixed-radix n, or the Bluestein length M.
__device__ __forceinline__ int ring_twiddle_lg(const RingPair& rp) {
  return rp.log2n >= 0 ? rp.log2n : (rp.bl_M > 0 ? __ffs(rp.bl_M) - 1 : __ffs(rp.nphi) - 1);
}

// Kind of transforms in a ring launch class (see ring_dft).
constexpr int class_kind(int cls) { return cls == 0 ? 1 : (cls == 1 ? 0 : 2); }

template <class T>
struct Vec4;
template <>
struct Vec4<double> {
  using type = double4;
};
template <>
struct Vec4<float> {
  using type = float4;
};

// exp(i k phi0) at k = tid and exp(i NT phi0), the factor that advances k by NT: the
// phases of the synthesis bins and (conjugated) of the analysis coefficients, which
// share them (bin k and coefficient m = k). Both 1 on rings with phi0 = 0.
struct RingPhase {
  double2 ph0, step;
};
template <int NT>
__device__ __forceinline__ RingPhase ring_phase(const RingPair& rp) {
  RingPhase r;
  if (rp.ph_num == 0) {
    r.ph0 = make_double2(1.0, 0.0);
    r.step = r.ph0;
  } else {
    r.ph0 = expipi<double>((int64_t)threadIdx.x * rp.ph_num, rp.nphi);
    r.step = expipi<double>((int64_t)NT * rp.ph_num, rp.nphi);
  }
  return r;
}

// Bins (and pixel pairs) of a ring pair a thread handles with their loads issued
// together: the largest number k = tid + u NT a launch class has, at most four.
constexpr int fold_depth(int kind, int maxb) {
  const int u = (kind == 1 ? 2 : 4) * maxb;
  return u < 4 ? u : 4;
}

// Synthesis loading step of one ring pair: the bins B[k] = sum over m = k (mod n) of
// F(m) exp(i m phi0) (F(-m) = conj F(m)) of the north and south rings, from the E/O
// coefficients Fp[m][4] of this map and pair, into buf as B_N + i B_S (k < n), in the
// transform's arithmetic type C. Long rings: thread tid folds bins tid + u NT, KU at a
// time, the first alias of each of the KU loaded before any of them is folded. Short rings use
// lds_raw for partial sums (consumed before the function returns). Every thread of
// the workgroup calls it.
template <class T, class C, int NT, int KU>
__device__ __forceinline__ void fold_synthesis(const PlanDev& P, const T* __restrict__ Fp, const RingPair& rp,
                                               typename CT<C>::V* buf, unsigned char* lds_raw,
                                               const RingPhase& rph) {
  using V4 = typename Vec4<T>::type;
  using V = typename CT<C>::V;
  const int n = rp.nphi;
  const int lmax = P.lmax;
  const int tid = threadIdx.x;
  const C sig = rp.ph_num ? (C)-1 : (C)1;          // exp(i n phi0)
  auto eo_load = [&](int m) { return *reinterpret_cast<const V4*>(Fp + (size_t)m * 4); };
  if (n > FOLD_PARTS) {
    // bin k: positive aliases m = k + t n, negative ones |m| = t n - k (t >= 1); its
    // first alias is m = k if k <= lmax, else n - k (there is then no positive one)
    auto fold_bin = [&](const int k, const V4 f1, const double2 phd) {
      const V ph = CT<C>::make((C)phd.x, (C)phd.y);
      V bn = CT<C>::make(0, 0), bs = CT<C>::make(0, 0);
      C sg = (C)1;                                  // sig^t
      for (int m = k; m <= lmax; m += n) {
        const V4 eo = (m == k) ? f1 : eo_load(m);
        V fn = CT<C>::make((C)eo.x + (C)eo.z, (C)eo.y + (C)eo.w);
        V fs = CT<C>::make((C)eo.x - (C)eo.z, (C)eo.y - (C)eo.w);
        if (m == 0) {
          fn.y = (C)0;
          fs.y = (C)0;
        } else {
          const V phm = CT<C>::make(sg * ph.x, sg * ph.y);
          fn = cmul(fn, phm);
          fs = cmul(fs, phm);
        }
        bn = cadd(bn, fn);
        bs = cadd(bs, fs);
        sg *= sig;
      }
      // exp(i |m| phi0) = sig^t conj(exp(i k phi0))
      sg = sig;
      const int mn = (k == 0) ? n : n - k;
      for (int m = mn; m <= lmax; m += n) {
        const V4 eo = (m == mn && k > lmax) ? f1 : eo_load(m);
        const V phm = CT<C>::make(sg * ph.x, -sg * ph.y);
        const V fn = cmul(CT<C>::make((C)eo.x + (C)eo.z, (C)eo.y + (C)eo.w), phm);
        const V fs = cmul(CT<C>::make((C)eo.x - (C)eo.z, (C)eo.y - (C)eo.w), phm);
        bn = cadd(bn, cconj(fn));
        bs = cadd(bs, cconj(fs));
        sg *= sig;
      }
      return CT<C>::make(bn.x - bs.y, bn.y + bs.x);   // B_N + i B_S
    };
    double2 ph = rph.ph0;
    for (int k0 = tid; k0 < n; k0 += KU * NT) {
      V4 first[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + u * NT;
        const int m1 = k <= lmax ? k : n - k;
        if (k < n && m1 <= lmax) first[u] = eo_load(m1);
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + u * NT;
        if (k < n) buf[k] = fold_bin(k, first[u], ph);
        ph = cmul(ph, rph.step);
      }
    }
  } else {
    // short rings carry many aliases per bin: G partial sums per bin, each over
    // every G-th alias, spread over the whole workgroup, then added in a fixed order
    const int G = FOLD_PARTS / n, np = G * n;
    const C sigG = (G & 1) ? sig : (C)1;
    V* part = reinterpret_cast<V*>(lds_raw);    // [np][N, S]
    for (int p = tid; p < np; p += NT) {
      const int k = p % n, g = p / n;
      const double2 phd = rp.ph_num ? expipi<double>((int64_t)k, n) : make_double2(1.0, 0.0);   // exp(i k phi0)
      const V phk = CT<C>::make((C)phd.x, (C)phd.y);
      V bn = CT<C>::make(0, 0), bs = CT<C>::make(0, 0);
      C sg = (g & 1) ? sig : (C)1;                  // sig^t, t = g + u G
      for (int m = k + g * n; m <= lmax; m += G * n) {
        const V4 eo = eo_load(m);
        V fn = CT<C>::make((C)eo.x + (C)eo.z, (C)eo.y + (C)eo.w);
        V fs = CT<C>::make((C)eo.x - (C)eo.z, (C)eo.y - (C)eo.w);
        if (m == 0) {
          fn.y = (C)0;
          fs.y = (C)0;
        } else {
          const V phm = CT<C>::make(sg * phk.x, sg * phk.y);
          fn = cmul(fn, phm);
          fs = cmul(fs, phm);
        }
        bn = cadd(bn, fn);
        bs = cadd(bs, fs);
        sg *= sigG;
      }
      sg = ((g + 1) & 1) ? sig : (C)1;             // negative aliases |m| = t n - k, t = 1 + g + u G
      for (int m = (g + 1) * n - k; m <= lmax; m += G * n) {
        const V4 eo = eo_load(m);
        const V phm = CT<C>::make(sg * phk.x, -sg * phk.y);
        const V fn = cmul(CT<C>::make((C)eo.x + (C)eo.z, (C)eo.y + (C)eo.w), phm);
        const V fs = cmul(CT<C>::make((C)eo.x - (C)eo.z, (C)eo.y - (C)eo.w), phm);
        bn = cadd(bn, cconj(fn));
        bs = cadd(bs, cconj(fs));
        sg *= sigG;
      }
      part[2 * p] = bn;
      part[2 * p + 1] = bs;
    }
    __syncthreads();
    constexpr int KB = (FOLD_PARTS + NT - 1) / NT;   // bins per thread
    V bk[KB];
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int k = tid + b * NT;
      if (k < n) {
        V bn = CT<C>::make(0, 0), bs = CT<C>::make(0, 0);
        for (int g = 0; g < G; ++g) {
          bn = cadd(bn, part[2 * (g * n + k)]);
          bs = cadd(bs, part[2 * (g * n + k) + 1]);
        }
        bk[b] = CT<C>::make(bn.x - bs.y, bn.y + bs.x);   // B_N + i B_S
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int k = tid + b * NT;
      if (k < n) buf[k] = bk[b];
    }
  }
}

// Analysis unfolding step of one ring pair, after the forward DFT of x_N + i x_S in
// buf: G(m) = Omega exp(-i m phi0) X[m mod n] of each ring (Hermitian unfold), written
// as S = G_N + G_S and D = G_N - G_S to Gp[m][4], m = 0..lmax, in the transform's
// arithmetic type C.
template <class T, class C, int NT>
__device__ __forceinline__ void unfold_analysis(const PlanDev& P, T* __restrict__ Gp, const RingPair& rp,
                                                const typename CT<C>::V* buf, const RingPhase& rph) {
  using V4 = typename Vec4<T>::type;
  using V = typename CT<C>::V;
  const int n = rp.nphi;
  const int lmax = P.lmax;
  const int tid = threadIdx.x;
  const C half_omega = (C)(0.5 * P.omega);
  double2 ph = cconj(rph.ph0);                      // exp(-i m phi0)
  const double2 step = cconj(rph.step);
  int k = tid % n;                                  // m mod n
  const int kstep = NT % n;
  for (int m = tid; m <= lmax; m += NT) {
    const int nk = (k == 0) ? 0 : n - k;
    const V zk = buf[k], znk = buf[nk];
    // X_N = (Z_k + conj Z_nk) / 2, X_S = (Z_k - conj Z_nk) / (2 i); Omega folded in
    const V xn = CT<C>::make((zk.x + znk.x) * half_omega, (zk.y - znk.y) * half_omega);
    const V xs = CT<C>::make((zk.y + znk.y) * half_omega, -(zk.x - znk.x) * half_omega);
    const V phc = CT<C>::make((C)ph.x, (C)ph.y);
    const V gn = cmul(xn, phc), gs = cmul(xs, phc);
    V4 o;
    o.x = (T)(gn.x + gs.x);
    o.y = (T)(gn.y + gs.y);
    o.z = (T)(gn.x - gs.x);
    o.w = (T)(gn.y - gs.y);
    *reinterpret_cast<V4*>(Gp + (size_t)m * 4) = o;
    ph = cmul(ph, step);
    k += kstep;
    if (k >= n) k -= n;
  }
}

// The messenger weight of Eq. (3), w = lambda q / (1 + (lambda - 1) q) with
// q = tau N^-1 in [0, 1]: an IEEE division in FP64, the hardware reciprocal (1 ulp)
// in FP32.
__device__ __forceinline__ double messenger_weight(double lam, double q) {
  return lam * q / (1.0 + (lam - 1.0) * q);
}
__device__ __forceinline__ float messenger_weight(float lam, float q) {
  return lam * q * __builtin_amdgcn_rcpf(1.0f + (lam - 1.0f) * q);
}

template <class T, class C, int NT, int MAXB, int KIND>
__device__ __forceinline__ void phase_b_body(const PlanDev& P, const PhaseBArgs& a, const int q,
                                             const int map, const int buf_elems) {
  using V = typename CT<C>::V;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  V* buf = reinterpret_cast<V*>(lds_raw);
  const RingPair rp = P.pairs[q];
  const int n = rp.nphi;
  const int lmax = P.lmax;
  const bool equator = rp.start_s < 0;
  const int tid = threadIdx.x;
  const size_t pstride = gf_stride(lmax);
  const size_t pbase = ((size_t)map * P.npairs + q) * pstride;
  const int64_t mbase = (int64_t)map * P.npix;
  const int mode = a.slots ? a.slots[map].pb_mode : a.mode;
  if (mode == 0) return;                          // idle slot (uniform over the block)
  const T* __restrict__ q_tab = static_cast<const T*>(P.q) + (a.slots ? map * a.q_stride : 0);

  // per-pass twiddles of this ring's transform length: loaded now, written to LDS
  // (after the padded data buffer) at the end of the loading step (after any partial
  // sums there are consumed) and ordered before their first use by the barrier that
  // closes that step
  // (thread tid holds entries tid + u NT, u < TWP; any beyond TWP NT, none for the
  // lengths a launch admits, are read at the store)
  // (three scalars rather than an array, which the compiler kept in scratch memory)
  V* twl = buf + fft_padded(buf_elems);
  constexpr int TWP = (2 * MAXB + 2) / 3;
  static_assert(TWP <= 3, "twiddle prefetch holds at most three entries per thread");
  const int tw_lg = ring_twiddle_lg(rp);
  const int tw_n = fft_twiddle_entries(tw_lg);
  const V* __restrict__ twg = Tabs<C>::tw(P);
  auto tw_load = [&](int e) { return e < tw_n ? twg[twiddle_glob_index(tw_lg, e, P.tw_len)] : CT<C>::make(0, 0); };
  const V tw0 = tw_load(tid);
  const V tw1 = TWP > 1 ? tw_load(tid + NT) : CT<C>::make(0, 0);
  const V tw2 = TWP > 2 ? tw_load(tid + 2 * NT) : CT<C>::make(0, 0);
  auto stage_twiddles = [&]() {
    if (tid < tw_n) twl[tid] = tw0;
    if (TWP > 1 && tid + NT < tw_n) twl[tid + NT] = tw1;
    if (TWP > 2 && tid + 2 * NT < tw_n) twl[tid + 2 * NT] = tw2;
    for (int e = tid + TWP * NT; e < tw_n; e += NT) twl[e] = twg[twiddle_glob_index(tw_lg, e, P.tw_len)];
  };

  // ---- d and tau N^-1 of the pixels of the update (Eq. 3): thread tid updates
  // pixel pairs j = tid + u NT, KU at a time, their loads issued together right
  // after the synthesis (so they hold no registers across the transform)
  constexpr int KU = fold_depth(KIND, MAXB);
  const bool chi = a.chi2 != nullptr && (mode & PB_SYNTH) && (mode & (PB_UPDATE | PB_CHI2));
  const bool pix_pass = (mode & (PB_WRITE_MAP | PB_UPDATE)) != 0;
  const bool upd = pix_pass && ((mode & PB_UPDATE) != 0 || chi);
  const T* __restrict__ d = static_cast<const T*>(a.d) + mbase;
  const RingPhase rph = ring_phase<NT>(rp);

  // ---- ring values into buf (x = north + i south)
  if (mode & PB_SYNTH) {
    fold_synthesis<T, C, NT, KU>(P, static_cast<const T*>(a.F) + pbase, rp, buf, lds_raw, rph);
    stage_twiddles();
    __syncthreads();
    ring_dft<C, NT, MAXB, KIND>(buf, twl, rp, +1, P);
  } else if (mode & PB_READ_MAP) {
    const T* src = static_cast<const T*>(a.map_in) + mbase;
    for (int j = tid; j < n; j += NT)
      buf[j] = CT<C>::make((C)src[rp.start_n + j], equator ? (C)0 : (C)src[rp.start_s + j]);
    stage_twiddles();
    __syncthreads();
  } else {
    for (int j = tid; j < n; j += NT) buf[j] = CT<C>::make(0, 0);
    stage_twiddles();
    __syncthreads();
  }

  // ---- map output and the messenger update (Eq. 3), in the transform's type C;
  // the chi^2 data term of the synthesised iterate in FP64
  double chi_acc = 0.0;
  if (pix_pass) {
    const C lam = (C)(a.slots ? a.slots[map].lambda : a.lambda);
    T* out = static_cast<T*>(a.map_out) + mbase;
    auto pixel_pair = [&](const int j, const T qn_, const T dn_, const T qs_, const T ds_) {
      const V xv = buf[j];
      C xn = xv.x, xs = xv.y;
      if (mode & PB_WRITE_MAP) {
        out[rp.start_n + j] = (T)xn;
        if (!equator) out[rp.start_s + j] = (T)xs;
      }
      if (chi) {
        const double rn = (double)dn_ - (double)xn;
        chi_acc += (double)qn_ * rn * rn;
        if (!equator) {
          const double rs = (double)ds_ - (double)xs;
          chi_acc += (double)qs_ * rs * rs;
        }
      }
      if (mode & PB_UPDATE) {
        xn = xn + messenger_weight(lam, (C)qn_) * ((C)dn_ - xn);
        if (!equator) xs = xs + messenger_weight(lam, (C)qs_) * ((C)ds_ - xs);
      }
      if (equator) xs = (C)0;
      buf[j] = CT<C>::make(xn, xs);
    };
    for (int j0 = tid; j0 < n; j0 += KU * NT) {
      T qn[KU] = {}, dn[KU] = {}, qs[KU] = {}, ds[KU] = {};
      if (upd) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          const int j = j0 + u * NT;
          if (j < n) {
            qn[u] = q_tab[rp.start_n + j];
            dn[u] = d[rp.start_n + j];
            if (!equator) {
              qs[u] = q_tab[rp.start_s + j];
              ds[u] = d[rp.start_s + j];
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int j = j0 + u * NT;
        if (j < n) pixel_pair(j, qn[u], dn[u], qs[u], ds[u]);
      }
    }
    __syncthreads();
  }
  if (chi) block_sum_add(chi_acc, a.chi2 + map * a.chi2_stride);

  // ---- analysis: forward DFT and unfold into S/D per m
  if (mode & PB_ANALYSIS) {
    ring_dft<C, NT, MAXB, KIND>(buf, twl, rp, -1, P);
    unfold_analysis<T, C, NT>(P, static_cast<T*>(a.G) + pbase, rp, buf, rph);
  }
}

// Eq. (3) for the polarised fields at one pixel: t = s + lambda (1 + (lambda - 1) M)^-1 M (d - s)
// with M = tau N^-1 (q: TT, QQ, UU, TQ, TU, QU). 1 + (lambda - 1) M is symmetric with
// eigenvalues 1 + (lambda - 1) mu, mu in [0, 1] (tau bounds every eigenvalue of N^-1),
// so it is inverted through its adjugate; at lambda = 1 it is the identity.
__device__ __forceinline__ void pol_update(double& s0, double& s1, double& s2, double d0, double d1, double d2,
                                           const double* q, double lam) {
  const double r0 = d0 - s0, r1 = d1 - s1, r2 = d2 - s2;
  const double v0 = q[0] * r0 + q[3] * r1 + q[4] * r2;
  const double v1 = q[3] * r0 + q[1] * r1 + q[5] * r2;
  const double v2 = q[4] * r0 + q[5] * r1 + q[2] * r2;
  const double c = lam - 1.0;
  const double a00 = 1.0 + c * q[0], a11 = 1.0 + c * q[1], a22 = 1.0 + c * q[2];
  const double a01 = c * q[3], a02 = c * q[4], a12 = c * q[5];
  const double i00 = a11 * a22 - a12 * a12, i01 = a02 * a12 - a01 * a22, i02 = a01 * a12 - a02 * a11;
  const double i11 = a00 * a22 - a02 * a02, i12 = a01 * a02 - a00 * a12, i22 = a00 * a11 - a01 * a01;
  const double f = lam / (a00 * i00 + a01 * i01 + a02 * i02);
  s0 += f * (i00 * v0 + i01 * v1 + i02 * v2);
  s1 += f * (i01 * v0 + i11 * v1 + i12 * v2);
  s2 += f * (i02 * v0 + i12 * v1 + i22 * v2);
}

// Polarised ring phase of one (ring pair, map): the three fields T, Q, U of the map,
// each a real field packed north + i south as in phase_b_body. The fields pass one
// after another through the one LDS buffer: the synthesised values of the pixels a
// thread updates are kept in its registers (at most PPT per field: n <= PPT NT), the
// 3x3 update couples them, and the forward transforms follow field by field.
template <class C, int NT, int MAXB, int KIND>
__device__ __forceinline__ void phase_b_pol_body(const PlanDev& P, const PolRingArgs& a, const int q, const int map,
                                                 const int buf_elems) {
  using V = typename CT<C>::V;
  constexpr int PPT = (KIND == 0 ? 4 : 2) * MAXB;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  V* buf = reinterpret_cast<V*>(lds_raw);
  const RingPair rp = P.pairs[q];
  const int n = rp.nphi;
  const int lmax = P.lmax;
  const bool equator = rp.start_s < 0;
  const int tid = threadIdx.x;
  const int mode = a.mode;
  const size_t pstride = gf_stride(lmax);
  auto pbase = [&](int f) { return (((size_t)f * a.field_maps + map) * P.npairs + q) * pstride; };
  const int64_t mbase = (int64_t)map * 3 * P.npix;

  V* twl = buf + fft_padded(buf_elems);
  const int tw_lg = ring_twiddle_lg(rp);
  const int tw_n = fft_twiddle_entries(tw_lg);
  const V* __restrict__ twg = Tabs<C>::tw(P);
  auto stage_twiddles = [&]() {
    for (int e = tid; e < tw_n; e += NT) twl[e] = twg[twiddle_glob_index(tw_lg, e, P.tw_len)];
  };

  const RingPhase rph = ring_phase<NT>(rp);
  V sx[3][PPT];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    if (mode & PB_SYNTH) {
      fold_synthesis<double, C, NT, fold_depth(KIND, MAXB)>(P, a.F + pbase(f), rp, buf, lds_raw, rph);
      stage_twiddles();
      __syncthreads();
      ring_dft<C, NT, MAXB, KIND>(buf, twl, rp, +1, P);
    } else if (mode & PB_READ_MAP) {
      const double* src = a.map_in + mbase + (int64_t)f * P.npix;
      for (int j = tid; j < n; j += NT)
        buf[j] = CT<C>::make((C)src[rp.start_n + j], equator ? (C)0 : (C)src[rp.start_s + j]);
      if (f == 0) stage_twiddles();
      __syncthreads();
    } else {
      for (int j = tid; j < n; j += NT) buf[j] = CT<C>::make(0, 0);
      if (f == 0) stage_twiddles();
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int j = tid + u * NT;
      sx[f][u] = j < n ? buf[j] : CT<C>::make(0, 0);
    }
    __syncthreads();
  }

  if (mode & (PB_WRITE_MAP | PB_UPDATE)) {
    const double lam = a.lambda;
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int j = tid + u * NT;
      if (j >= n) continue;
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        if (side == 1 && equator) continue;
        const int64_t pix = (side == 0 ? rp.start_n : rp.start_s) + j;
        double s0 = side == 0 ? (double)sx[0][u].x : (double)sx[0][u].y;
        double s1 = side == 0 ? (double)sx[1][u].x : (double)sx[1][u].y;
        double s2 = side == 0 ? (double)sx[2][u].x : (double)sx[2][u].y;
        if (mode & PB_WRITE_MAP) {
          a.map_out[mbase + pix] = s0;
          a.map_out[mbase + P.npix + pix] = s1;
          a.map_out[mbase + 2 * P.npix + pix] = s2;
        }
        if (mode & PB_UPDATE) {
          double qv[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) qv[c] = a.q6[(int64_t)c * P.npix + pix];
          const double* dd = a.d + mbase;
          pol_update(s0, s1, s2, dd[pix], dd[P.npix + pix], dd[2 * P.npix + pix], qv, lam);
          if (side == 0) {
            sx[0][u].x = (C)s0;
            sx[1][u].x = (C)s1;
            sx[2][u].x = (C)s2;
          } else {
            sx[0][u].y = (C)s0;
            sx[1][u].y = (C)s1;
            sx[2][u].y = (C)s2;
          }
        }
      }
      if (equator) {
        sx[0][u].y = sx[1][u].y = sx[2][u].y = (C)0;
      }
    }
  }

  if (mode & PB_ANALYSIS) {
#pragma unroll
    for (int f = 0; f < 3; ++f) {
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int j = tid + u * NT;
        if (j < n) buf[j] = sx[f][u];
      }
      __syncthreads();
      ring_dft<C, NT, MAXB, KIND>(buf, twl, rp, -1, P);
      unfold_analysis<double, C, NT>(P, a.G + pbase(f), rp, buf, rph);
      __syncthreads();
    }
  }
}

template <int NT, int MAXB, int CLS>
__global__ void __launch_bounds__(NT) phase_b_pol_kernel(PlanDev P, PolRingArgs a, const int32_t* __restrict__ qlist,
                                                          int buf_elems) {
  phase_b_pol_body<double, NT, MAXB, class_kind(CLS)>(P, a, qlist[blockIdx.x], blockIdx.y, buf_elems);
}

template <class T, class C, int NT, int MAXB, int CLS>
__global__ void __launch_bounds__(NT) phase_b_kernel(PlanDev P, PhaseBArgs a, const int32_t* __restrict__ qlist,
                                                     int buf_elems) {
  phase_b_body<T, C, NT, MAXB, class_kind(CLS)>(P, a, qlist[blockIdx.x], blockIdx.y, buf_elems);
}

// Task groups (float storage and arithmetic): block b of task t covers entry
// (b - offs[t]) / nmaps of the task's ring-pair list of class CLS and map
// (b - offs[t]) % nmaps.
template <int NT, int CLS, int MAXB>
__global__ void __launch_bounds__(NT) group_phase_b_kernel(GroupArgs g, int buf_elems) {
  const int lo = group_task_of(g, blockIdx.x);
  const TaskDev& t = g.t[lo];
  const int64_t local = blockIdx.x - g.offs[lo];
  PhaseBArgs a{};
  a.mode = t.pb_mode;
  a.nmaps = t.nmaps;
  a.lambda = t.lambda;
  a.F = t.F;
  a.G = t.G;
  a.d = t.d;
  a.map_in = t.map_in;
  a.map_out = t.map_out;
  a.slots = t.slots;
  a.q_stride = t.q_stride;
  phase_b_body<float, float, NT, MAXB, class_kind(CLS)>(t.P, a, t.ring_q[CLS][local / t.nmaps],
                                                        (int)(local % t.nmaps), buf_elems);
}

// Threads of a ring workgroup per launch class: Bluestein rings 512, power-of-two
// rings 256 (the longest, 4 nside points, then take eight points a thread, which
// keeps every lane busy in the radix-8 passes and lets four workgroups share a CU),
// the one-wave class 64.
constexpr int ring_threads(int cls) { return cls == 0 ? 512 : (cls == 1 ? 256 : 64); }

// Radix-4 butterflies per thread and pass for a transform of fft_len points.
int maxb_for(int fft_len, int nt) {
  const int b = (fft_len + 4 * nt - 1) / (4 * nt);
  return b <= 1 ? 1 : (b <= 2 ? 2 : (b <= 4 ? 4 : 0));
}

// Raise the dynamic-LDS limit of `kernel` on the current device to at least `lds`
// (never lower it). One lock for every kernel and device: launches of one kernel
// from several host threads (plans, the server's stepping thread) must not undo
// each other's limit.
hipError_t ensure_dynamic_lds(const void* kernel, size_t lds) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, size_t> limit;
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev)) return e;
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = limit[{kernel, dev}];
  if (lds <= cur) return hipSuccess;
  if (hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) return e;
  cur = lds;
  return hipSuccess;
}

template <class T, class C, int NT, int MAXB, int CLS>
hipError_t launch_class_b(const PlanDev& P, const PhaseBArgs& a, const RingClass& rc, hipStream_t s) {
  const size_t lds = ring_lds_bytes(rc.fft_len, sizeof(typename CT<C>::V));
  if (hipError_t e = ensure_dynamic_lds((const void*)phase_b_kernel<T, C, NT, MAXB, CLS>, lds)) return e;
  hipLaunchKernelGGL((phase_b_kernel<T, C, NT, MAXB, CLS>), dim3(rc.count, a.nmaps), dim3(NT), lds, s, P, a, rc.q,
                     rc.fft_len);
  return hipGetLastError();
}

template <class T, class C, int CLS>
hipError_t launch_class(const PlanDev& P, const PhaseBArgs& a, const RingClass& rc, hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  constexpr int NT = ring_threads(CLS);
  switch (maxb_for(rc.fft_len, NT)) {
    case 1: return launch_class_b<T, C, NT, 1, CLS>(P, a, rc, s);
    case 2: return launch_class_b<T, C, NT, 2, CLS>(P, a, rc, s);
    case 4: return launch_class_b<T, C, NT, 4, CLS>(P, a, rc, s);
    default: return hipErrorInvalidValue;
  }
}

template <class T, class C>
hipError_t launch_t(const PlanDev& P, const PhaseBArgs& a, const RingClass* cls, hipStream_t s) {
  hipError_t e = launch_class<T, C, 0>(P, a, cls[0], s);
  if (e == hipSuccess) e = launch_class<T, C, 1>(P, a, cls[1], s);
  if (e == hipSuccess) e = launch_class<T, C, 2>(P, a, cls[2], s);
  return e;
}

template <int NT, int CLS, int MAXB>
hipError_t group_class_b(const GroupLaunch& g, int fft_len, hipStream_t s) {
  const size_t lds = ring_lds_bytes(fft_len, sizeof(float2));
  if (hipError_t e = ensure_dynamic_lds((const void*)group_phase_b_kernel<NT, CLS, MAXB>, lds)) return e;
  return for_each_group_part(g, [&](const GroupArgs& a, int64_t nb) {
    hipLaunchKernelGGL((group_phase_b_kernel<NT, CLS, MAXB>), dim3(nb), dim3(NT), lds, s, a, fft_len);
    return hipGetLastError();
  });
}

template <int NT, int CLS>
hipError_t group_class(const GroupLaunch& g, int fft_len, hipStream_t s) {
  switch (maxb_for(fft_len, NT)) {
    case 1: return group_class_b<NT, CLS, 1>(g, fft_len, s);
    case 2: return group_class_b<NT, CLS, 2>(g, fft_len, s);
    case 4: return group_class_b<NT, CLS, 4>(g, fft_len, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NT, int MAXB, int CLS>
hipError_t launch_pol_class_b(const PlanDev& P, const PolRingArgs& a, const RingClass& rc, hipStream_t s) {
  const size_t lds = ring_lds_bytes(rc.fft_len, sizeof(double2));
  if (hipError_t e = ensure_dynamic_lds((const void*)phase_b_pol_kernel<NT, MAXB, CLS>, lds)) return e;
  hipLaunchKernelGGL((phase_b_pol_kernel<NT, MAXB, CLS>), dim3(rc.count, a.nmaps), dim3(NT), lds, s, P, a, rc.q,
                     rc.fft_len);
  return hipGetLastError();
}

template <int CLS>
hipError_t launch_pol_class(const PlanDev& P, const PolRingArgs& a, const RingClass& rc, hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  switch (maxb_for(rc.fft_len, 512)) {
    case 1: return launch_pol_class_b<512, 1, CLS>(P, a, rc, s);
    case 2: return launch_pol_class_b<512, 2, CLS>(P, a, rc, s);
    case 4: return launch_pol_class_b<512, 4, CLS>(P, a, rc, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_group_phase_b(const GroupLaunch& g, int cls, int fft_len, hipStream_t s) {
  if (g.nblocks == 0) return hipSuccess;
  switch (cls) {
    case 0: return group_class<ring_threads(0), 0>(g, fft_len, s);
    case 1: return group_class<ring_threads(1), 1>(g, fft_len, s);
    default: return group_class<ring_threads(2), 2>(g, fft_len, s);
  }
}

hipError_t launch_phase_b(const PlanDev& P, const PhaseBArgs& a, const RingClass* cls, bool fp32, hipStream_t s) {
  return fp32 ? launch_t<float, float>(P, a, cls, s) : launch_t<double, double>(P, a, cls, s);
}

hipError_t launch_phase_b_class(const PlanDev& P, const PhaseBArgs& a, const RingClass& rc, int cls, bool fp32,
                                hipStream_t s) {
  switch (cls) {
    case 0: return fp32 ? launch_class<float, float, 0>(P, a, rc, s) : launch_class<double, double, 0>(P, a, rc, s);
    case 1: return fp32 ? launch_class<float, float, 1>(P, a, rc, s) : launch_class<double, double, 1>(P, a, rc, s);
    default: return fp32 ? launch_class<float, float, 2>(P, a, rc, s) : launch_class<double, double, 2>(P, a, rc, s);
  }
}

hipError_t launch_pol_ring(const PlanDev& P, const PolRingArgs& a, const RingClass* cls, hipStream_t s) {
  hipError_t e = launch_pol_class<0>(P, a, cls[0], s);
  if (e == hipSuccess) e = launch_pol_class<1>(P, a, cls[1], s);
  return e;
}

}  // namespace mwf
