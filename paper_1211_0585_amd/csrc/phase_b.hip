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
// in-place Stockham FFT (radix 4, plus one radix-2 pass for odd log2 n) whose
// butterflies are staged in registers between two barriers per pass; other
// lengths use Bluestein's chirp-z method: chirp, power-of-two FFT of length
// M >= 2 n - 1, multiply by the plan-time filter spectrum, inverse FFT, chirp.
// The FFT arithmetic type C is double for FP64 plans and float for plans that
// store maps and ring coefficients in float. Rings are launched in two classes:
// transforms of at most 1024 points run one wave per ring pair, longer ones 512
// threads, so short polar rings do not leave most of a large workgroup idle.
#include "mwf_internal.hpp"

namespace mwf {
namespace {

constexpr int PB_MAXB = 4;   // max radix-4 butterflies per thread (L <= 4 * PB_MAXB * threads)

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

// In-place Stockham FFT of length L = 2^lg (4 <= L <= 4 PB_MAXB NT) in LDS, run by
// all NT threads of the workgroup; dir = -1: exp(-2 pi i jk/L), +1: exp(+...). Unnormalised. Radix-4 passes,
// with one radix-2 pass first when lg is odd. tw[t] = exp(-2 pi i t / tw_len),
// t < tw_len / 2. Every pass loads all butterfly inputs into registers,
// synchronises, then writes the outputs, so a single LDS buffer suffices.
template <class C, int NT>
__device__ __forceinline__ void fft_pow2(typename CT<C>::V* x, int lg, int dir,
                                         const typename CT<C>::V* __restrict__ tw, int tw_len) {
  using V = typename CT<C>::V;
  const int L = 1 << lg;
  const int tid = threadIdx.x;
  const C sd = (C)dir;
  int Ns = 1;
  int rem = lg;
  while (Ns < L) {
    const bool r2 = (rem & 1) != 0;
    V v[4 * PB_MAXB];
    if (!r2) {
      const int nb = L / 4;
#pragma unroll
      for (int b = 0; b < PB_MAXB; ++b) {
        const int j = tid + b * NT;
        if (j < nb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) v[4 * b + r] = x[j + r * nb];
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < PB_MAXB; ++b) {
        const int j = tid + b * NT;
        if (j < nb) {
          const int k = j & (Ns - 1);
          V w = tw[k * (tw_len / (Ns * 4))];
          if (dir > 0) w.y = -w.y;
          const V w2 = cmul(w, w), w3 = cmul(w2, w);
          V a0 = v[4 * b], a1 = cmul(v[4 * b + 1], w), a2 = cmul(v[4 * b + 2], w2), a3 = cmul(v[4 * b + 3], w3);
          dft4(a0, a1, a2, a3, sd);
          const int idx = (j - k) * 4 + k;
          x[idx] = a0;
          x[idx + Ns] = a1;
          x[idx + 2 * Ns] = a2;
          x[idx + 3 * Ns] = a3;
        }
      }
      Ns *= 4;
      rem -= 2;
    } else {
      const int nb = L / 2;
#pragma unroll
      for (int b = 0; b < 2 * PB_MAXB; ++b) {
        const int j = tid + b * NT;
        if (j < nb) {
          v[2 * b] = x[j];
          v[2 * b + 1] = x[j + nb];
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 2 * PB_MAXB; ++b) {
        const int j = tid + b * NT;
        if (j < nb) {
          const int k = j & (Ns - 1);
          V w = tw[k * (tw_len / (Ns * 2))];
          if (dir > 0) w.y = -w.y;
          const V a0 = v[2 * b], a1 = cmul(v[2 * b + 1], w);
          const int idx = (j - k) * 2 + k;
          x[idx] = cadd(a0, a1);
          x[idx + Ns] = csub(a0, a1);
        }
      }
      Ns *= 2;
      rem -= 1;
    }
    __syncthreads();
  }
}

// DFT of any length n of x[0..n) in place (dir = -1 forward, +1 inverse) by
// Bluestein's method, using the LDS buffer x[0..M), the chirp exp(-i pi j^2/n)
// (length n) and the filter spectrum H (length M).
template <class C, int NT>
__device__ void dft_bluestein(typename CT<C>::V* x, int n, int M, int lgM, int dir,
                              const typename CT<C>::V* __restrict__ chirp,
                              const typename CT<C>::V* __restrict__ H,
                              const typename CT<C>::V* __restrict__ tw, int tw_len) {
  using V = typename CT<C>::V;
  const int tid = threadIdx.x;
  for (int j = tid; j < M; j += NT) {
    if (j < n) {
      V v = x[j];
      if (dir > 0) v = cconj(v);     // inverse DFT = conj(DFT(conj(x)))
      x[j] = cmul(v, chirp[j]);
    } else {
      x[j] = CT<C>::make(0, 0);
    }
  }
  __syncthreads();
  fft_pow2<C, NT>(x, lgM, -1, tw, tw_len);
  for (int k = tid; k < M; k += NT) x[k] = cmul(x[k], H[k]);
  __syncthreads();
  fft_pow2<C, NT>(x, lgM, +1, tw, tw_len);
  const C invM = (C)1 / (C)M;
  for (int k = tid; k < n; k += NT) {
    V v = cmul(x[k], chirp[k]);
    v.x *= invM;
    v.y *= invM;
    if (dir > 0) v = cconj(v);
    x[k] = v;
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
};
template <>
struct Tabs<float> {
  __device__ static const float2* tw(const PlanDev& P) { return P.twiddle32; }
  __device__ static const float2* chirp(const PlanDev& P) { return P.chirp32; }
  __device__ static const float2* blue(const PlanDev& P) { return P.bluestein32; }
};

template <class C, int NT>
__device__ __forceinline__ void ring_dft(typename CT<C>::V* buf, const RingPair& rp, int dir,
                                         const PlanDev& P) {
  if (rp.log2n >= 0) {
    fft_pow2<C, NT>(buf, rp.log2n, dir, Tabs<C>::tw(P), P.tw_len);
  } else {
    dft_bluestein<C, NT>(buf, rp.nphi, rp.bl_M, __ffs(rp.bl_M) - 1, dir, Tabs<C>::chirp(P) + rp.chirp_off,
                         Tabs<C>::blue(P) + rp.bl_off, Tabs<C>::tw(P), P.tw_len);
  }
}

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

template <class T, class C, int NT>
__device__ __forceinline__ void phase_b_body(const PlanDev& P, const PhaseBArgs& a, const int q,
                                             const int map) {
  using V4 = typename Vec4<T>::type;
  using V = typename CT<C>::V;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  V* buf = reinterpret_cast<V*>(lds_raw);
  const RingPair rp = P.pairs[q];
  const int n = rp.nphi;
  const int lmax = P.lmax;
  const bool equator = rp.start_s < 0;
  const int tid = threadIdx.x;
  const size_t pstride = (size_t)(lmax + 1) * 4;
  const size_t pbase = ((size_t)map * P.npairs + q) * pstride;
  const int64_t mbase = (int64_t)map * P.npix;
  const int mode = a.slots ? a.slots[map].pb_mode : a.mode;
  if (mode == 0) return;                          // idle slot (uniform over the block)
  const double sig = rp.ph_num ? -1.0 : 1.0;      // exp(i n phi0)
  const T* __restrict__ q_tab = static_cast<const T*>(P.q) + (a.slots ? map * a.q_stride : 0);

  // ---- ring values into buf (x = north + i south)
  if (mode & PB_SYNTH) {
    const T* __restrict__ Fp = static_cast<const T*>(a.F) + pbase;
    // exp(i k phi0) for k = tid + s * NT, advanced by one complex multiply
    double2 ph = expipi<double>((int64_t)tid * rp.ph_num, n);
    const double2 step = expipi<double>((int64_t)NT * rp.ph_num, n);
    for (int k = tid; k < n; k += NT) {
      double2 bn = make_double2(0.0, 0.0), bs = make_double2(0.0, 0.0);
      double s = 1.0;                               // sig^t for m = k + t n
      for (int m = k; m <= lmax; m += n) {          // m >= 0 with m = k (mod n)
        const V4 eo = *reinterpret_cast<const V4*>(Fp + (size_t)m * 4);
        double2 fn = make_double2((double)eo.x + (double)eo.z, (double)eo.y + (double)eo.w);
        double2 fs = make_double2((double)eo.x - (double)eo.z, (double)eo.y - (double)eo.w);
        if (m == 0) {
          fn.y = 0.0;
          fs.y = 0.0;
        } else {
          const double2 phm = make_double2(s * ph.x, s * ph.y);
          fn = cmul(fn, phm);
          fs = cmul(fs, phm);
        }
        bn = cadd(bn, fn);
        bs = cadd(bs, fs);
        s *= sig;
      }
      // m < 0 terms: |m| = t n - k (t >= 1), exp(i |m| phi0) = sig^t conj(exp(i k phi0))
      s = sig;
      for (int m = (k == 0 ? n : n - k); m <= lmax; m += n) {
        const V4 eo = *reinterpret_cast<const V4*>(Fp + (size_t)m * 4);
        const double2 phm = make_double2(s * ph.x, -s * ph.y);
        const double2 fn = cmul(make_double2((double)eo.x + (double)eo.z, (double)eo.y + (double)eo.w), phm);
        const double2 fs = cmul(make_double2((double)eo.x - (double)eo.z, (double)eo.y - (double)eo.w), phm);
        bn = cadd(bn, cconj(fn));
        bs = cadd(bs, cconj(fs));
        s *= sig;
      }
      buf[k] = CT<C>::make((C)(bn.x - bs.y), (C)(bn.y + bs.x));   // B_N + i B_S
      ph = cmul(ph, step);
    }
    __syncthreads();
    ring_dft<C, NT>(buf, rp, +1, P);
  } else if (mode & PB_READ_MAP) {
    const T* src = static_cast<const T*>(a.map_in) + mbase;
    for (int j = tid; j < n; j += NT)
      buf[j] = CT<C>::make((C)src[rp.start_n + j], equator ? (C)0 : (C)src[rp.start_s + j]);
    __syncthreads();
  } else {
    for (int j = tid; j < n; j += NT) buf[j] = CT<C>::make(0, 0);
    __syncthreads();
  }

  // ---- map output and the messenger update (Eq. 3)
  if (mode & (PB_WRITE_MAP | PB_UPDATE)) {
    const double lam = a.slots ? a.slots[map].lambda : a.lambda;
    const T* __restrict__ d = static_cast<const T*>(a.d) + mbase;
    T* out = static_cast<T*>(a.map_out) + mbase;
    for (int j = tid; j < n; j += NT) {
      const V xv = buf[j];
      double2 x = make_double2((double)xv.x, (double)xv.y);
      if (mode & PB_WRITE_MAP) {
        out[rp.start_n + j] = (T)x.x;
        if (!equator) out[rp.start_s + j] = (T)x.y;
      }
      if (mode & PB_UPDATE) {
        const double qn = (double)q_tab[rp.start_n + j];
        const double wn = lam * qn / (1.0 + (lam - 1.0) * qn);
        x.x = x.x + wn * ((double)d[rp.start_n + j] - x.x);
        if (!equator) {
          const double qs = (double)q_tab[rp.start_s + j];
          const double ws = lam * qs / (1.0 + (lam - 1.0) * qs);
          x.y = x.y + ws * ((double)d[rp.start_s + j] - x.y);
        }
      }
      if (equator) x.y = 0.0;
      buf[j] = CT<C>::make((C)x.x, (C)x.y);
    }
    __syncthreads();
  }

  // ---- analysis: forward DFT and unfold into S/D per m
  if (mode & PB_ANALYSIS) {
    ring_dft<C, NT>(buf, rp, -1, P);
    T* Gp = static_cast<T*>(a.G) + pbase;
    const double half_omega = 0.5 * P.omega;
    double2 ph = expipi<double>(-(int64_t)tid * rp.ph_num, n);          // exp(-i m phi0)
    const double2 step = expipi<double>(-(int64_t)NT * rp.ph_num, n);
    for (int m = tid; m <= lmax; m += NT) {
      const int k = m % n;
      const int nk = (k == 0) ? 0 : n - k;
      const V zkv = buf[k], znkv = buf[nk];
      const double2 zk = make_double2((double)zkv.x, (double)zkv.y);
      const double2 znk = make_double2((double)znkv.x, (double)znkv.y);
      // X_N = (Z_k + conj Z_nk) / 2, X_S = (Z_k - conj Z_nk) / (2 i); Omega folded in
      const double2 xn = make_double2((zk.x + znk.x) * half_omega, (zk.y - znk.y) * half_omega);
      const double2 xs = make_double2((zk.y + znk.y) * half_omega, -(zk.x - znk.x) * half_omega);
      const double2 gn = cmul(xn, ph), gs = cmul(xs, ph);
      V4 o;
      o.x = (T)(gn.x + gs.x);
      o.y = (T)(gn.y + gs.y);
      o.z = (T)(gn.x - gs.x);
      o.w = (T)(gn.y - gs.y);
      *reinterpret_cast<V4*>(Gp + (size_t)m * 4) = o;
      ph = cmul(ph, step);
    }
  }
}

template <class T, class C, int NT>
__global__ void __launch_bounds__(NT, 4) phase_b_kernel(PlanDev P, PhaseBArgs a,
                                                        const int32_t* __restrict__ qlist) {
  phase_b_body<T, C, NT>(P, a, qlist[blockIdx.x], blockIdx.y);
}

// Task groups (float storage and arithmetic): block b of task t covers entry
// (b - offs[t]) / nmaps of the task's ring-pair list of this class and map
// (b - offs[t]) % nmaps.
template <int NT, int CLS>
__global__ void __launch_bounds__(NT, 4) group_phase_b_kernel(const TaskDev* __restrict__ tasks,
                                                              const int64_t* __restrict__ offs, int ntasks) {
  int lo = 0, hi = ntasks - 1;
  const int64_t b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const TaskDev& t = tasks[lo];
  const int64_t local = b - offs[lo];
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
  phase_b_body<float, float, NT>(t.P, a, t.ring_q[CLS][local / t.nmaps], (int)(local % t.nmaps));
}

template <class T, class C, int NT>
hipError_t launch_class(const PlanDev& P, const PhaseBArgs& a, const RingClass& rc, hipStream_t s) {
  if (rc.count == 0) return hipSuccess;
  static size_t attr_bytes = 0;
  const size_t lds = rc.fft_len * sizeof(typename CT<C>::V);
  if (lds > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)phase_b_kernel<T, C, NT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_bytes = lds;
  }
  hipLaunchKernelGGL((phase_b_kernel<T, C, NT>), dim3(rc.count, a.nmaps), dim3(NT), lds, s, P, a, rc.q);
  return hipGetLastError();
}

template <class T, class C>
hipError_t launch_t(const PlanDev& P, const PhaseBArgs& a, const RingClass& small,
                    const RingClass& large, hipStream_t s) {
  hipError_t e = launch_class<T, C, 512>(P, a, large, s);
  if (e != hipSuccess) return e;
  return launch_class<T, C, 64>(P, a, small, s);
}

}  // namespace

template <int NT, int CLS>
hipError_t group_class(const GroupLaunch& g, size_t lds_bytes, hipStream_t s) {
  static size_t attr_bytes = 0;
  if (lds_bytes > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)group_phase_b_kernel<NT, CLS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    attr_bytes = lds_bytes;
  }
  hipLaunchKernelGGL((group_phase_b_kernel<NT, CLS>), dim3(g.nblocks), dim3(NT), lds_bytes, s, g.tasks, g.offs,
                     g.ntasks);
  return hipGetLastError();
}

hipError_t launch_group_phase_b(const GroupLaunch& g, int cls, size_t lds_bytes, hipStream_t s) {
  if (g.nblocks == 0) return hipSuccess;
  return cls == 0 ? group_class<512, 0>(g, lds_bytes, s) : group_class<64, 1>(g, lds_bytes, s);
}

hipError_t launch_phase_b(const PlanDev& P, const PhaseBArgs& a, const RingClass& small,
                          const RingClass& large, bool fp32, hipStream_t s) {
  return fp32 ? launch_t<float, float>(P, a, small, large, s)
              : launch_t<double, double>(P, a, small, large, s);
}

}  // namespace mwf
