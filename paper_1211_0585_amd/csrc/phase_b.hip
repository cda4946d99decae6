// Phase B of a messenger sweep: ring-parallel work in pixel space.
//
// One workgroup handles one pair of mirror rings (north ring i, south ring
// 4 nside - i), which share n_phi and the longitude of pixel 0, for one map.
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
// Ring lengths are 4 i (polar caps) or 4 nside (belt): powers of two use an
// in-place radix-2 FFT; other lengths use Bluestein's chirp-z method with a
// power-of-two convolution of length M >= 2 n - 1 whose filter spectrum is a
// plan-time table.
#include "mwf_internal.hpp"

namespace mwf {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// exp(i pi num / den) for integers, with the argument reduced exactly.
__device__ __forceinline__ double2 expipi(int64_t num, int64_t den) {
  int64_t r = num % (2 * den);
  if (r < 0) r += 2 * den;
  double s, c;
  sincospi((double)r / (double)den, &s, &c);
  return make_double2(c, s);
}

// In-place radix-2 DIT FFT of length 2^lg held in LDS; dir = -1 for
// exp(-2 pi i jk / L), +1 for exp(+...). Unnormalised. All threads of the block
// must call it.
__device__ void fft_pow2(double2* x, int lg, int dir, const double2* __restrict__ tw, int tw_len) {
  const int L = 1 << lg;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < L; i += nt) {
    int j = (int)(__brev((unsigned)i) >> (32 - lg));
    if (j > i) {
      double2 t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
  __syncthreads();
  for (int s = 1; s <= lg; ++s) {
    const int half = 1 << (s - 1);
    const int tstep = tw_len >> s;
    for (int b = tid; b < (L >> 1); b += nt) {
      const int pos = b & (half - 1);
      const int i0 = ((b >> (s - 1)) << s) + pos;
      const int i1 = i0 + half;
      double2 w = tw[pos * tstep];
      if (dir > 0) w.y = -w.y;
      const double2 u = x[i0];
      const double2 v = cmul(w, x[i1]);
      x[i0] = cadd(u, v);
      x[i1] = csub(u, v);
    }
    __syncthreads();
  }
}

// Bluestein chirp exp(-i pi j^2 / n) with exact argument reduction.
__device__ __forceinline__ double2 chirp(int j, int n) {
  const int64_t jj = ((int64_t)j * j) % (2 * (int64_t)n);
  return expipi(-jj, n);
}

// DFT of length n (any n) of x[0..n) in place, dir = -1 forward / +1 inverse,
// using the LDS buffer x[0..M) and the filter spectrum H (length M).
__device__ void dft_bluestein(double2* x, int n, int M, int lgM, int dir,
                              const double2* __restrict__ H, const double2* __restrict__ tw,
                              int tw_len) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = tid; j < M; j += nt) {
    if (j < n) {
      double2 v = x[j];
      if (dir > 0) v = cconj(v);     // inverse DFT = conj(DFT(conj(x)))
      x[j] = cmul(v, chirp(j, n));
    } else {
      x[j] = make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  fft_pow2(x, lgM, -1, tw, tw_len);
  for (int k = tid; k < M; k += nt) x[k] = cmul(x[k], H[k]);
  __syncthreads();
  fft_pow2(x, lgM, +1, tw, tw_len);
  const double invM = 1.0 / (double)M;
  for (int k = tid; k < n; k += nt) {
    double2 v = cmul(x[k], chirp(k, n));
    v.x *= invM;
    v.y *= invM;
    if (dir > 0) v = cconj(v);
    x[k] = v;
  }
  __syncthreads();
}

__device__ __forceinline__ void ring_dft(double2* buf, const RingPair& rp, int dir, const PlanDev& P) {
  if (rp.log2n >= 0) {
    fft_pow2(buf, rp.log2n, dir, P.twiddle, P.tw_len);
  } else {
    dft_bluestein(buf, rp.nphi, rp.bl_M, __ffs(rp.bl_M) - 1, dir, P.bluestein + rp.bl_off,
                  P.twiddle, P.tw_len);
  }
}

__global__ void __launch_bounds__(256) phase_b_f64_kernel(PlanDev P, PhaseBArgs a) {
  extern __shared__ double2 buf[];
  const int q = blockIdx.x;
  const int map = blockIdx.y;
  const RingPair rp = P.pairs[q];
  const int n = rp.nphi;
  const int lmax = P.lmax;
  const bool equator = rp.start_s < 0;
  const int tid = threadIdx.x, nt = blockDim.x;
  const size_t pstride = (size_t)(lmax + 1) * 4;
  const size_t pbase = ((size_t)map * P.npairs + q) * pstride;
  const int64_t mbase = (int64_t)map * P.npix;
  const int mode = a.mode;

  // ---- ring values into buf (x = north + i south)
  if (mode & PB_SYNTH) {
    const double* Fp = a.F + pbase;
    for (int k = tid; k < n; k += nt) {
      double2 bn = make_double2(0.0, 0.0), bs = make_double2(0.0, 0.0);
      for (int m = k; m <= lmax; m += n) {          // m >= 0 with m = k (mod n)
        const double4 eo = *reinterpret_cast<const double4*>(Fp + (size_t)m * 4);
        double2 fn = make_double2(eo.x + eo.z, eo.y + eo.w);
        double2 fs = make_double2(eo.x - eo.z, eo.y - eo.w);
        if (m == 0) {
          fn.y = 0.0;
          fs.y = 0.0;
        } else {
          const double2 ph = expipi((int64_t)m * rp.ph_num, rp.ph_den);
          fn = cmul(fn, ph);
          fs = cmul(fs, ph);
        }
        bn = cadd(bn, fn);
        bs = cadd(bs, fs);
      }
      for (int m = (k == 0 ? n : n - k); m <= lmax; m += n) {   // m < 0: -m = k (mod n)
        const double4 eo = *reinterpret_cast<const double4*>(Fp + (size_t)m * 4);
        const double2 ph = expipi((int64_t)m * rp.ph_num, rp.ph_den);
        const double2 fn = cmul(make_double2(eo.x + eo.z, eo.y + eo.w), ph);
        const double2 fs = cmul(make_double2(eo.x - eo.z, eo.y - eo.w), ph);
        bn = cadd(bn, cconj(fn));
        bs = cadd(bs, cconj(fs));
      }
      buf[k] = make_double2(bn.x - bs.y, bn.y + bs.x);   // B_N + i B_S
    }
    __syncthreads();
    ring_dft(buf, rp, +1, P);
  } else if (mode & PB_READ_MAP) {
    const double* src = a.map_in + mbase;
    for (int j = tid; j < n; j += nt)
      buf[j] = make_double2(src[rp.start_n + j], equator ? 0.0 : src[rp.start_s + j]);
    __syncthreads();
  } else {
    for (int j = tid; j < n; j += nt) buf[j] = make_double2(0.0, 0.0);
    __syncthreads();
  }

  // ---- map output and the messenger update (Eq. 3)
  if (mode & (PB_WRITE_MAP | PB_UPDATE)) {
    const double lam = a.lambda;
    for (int j = tid; j < n; j += nt) {
      double2 x = buf[j];
      if (mode & PB_WRITE_MAP) {
        a.map_out[mbase + rp.start_n + j] = x.x;
        if (!equator) a.map_out[mbase + rp.start_s + j] = x.y;
      }
      if (mode & PB_UPDATE) {
        const double* d = a.d + mbase;
        const double qn = P.q[rp.start_n + j];
        const double wn = lam * qn / (1.0 + (lam - 1.0) * qn);
        x.x = x.x + wn * (d[rp.start_n + j] - x.x);
        if (!equator) {
          const double qs = P.q[rp.start_s + j];
          const double ws = lam * qs / (1.0 + (lam - 1.0) * qs);
          x.y = x.y + ws * (d[rp.start_s + j] - x.y);
        }
      }
      if (equator) x.y = 0.0;
      buf[j] = x;
    }
    __syncthreads();
  }

  // ---- analysis: forward DFT and unfold into S/D per m
  if (mode & PB_ANALYSIS) {
    ring_dft(buf, rp, -1, P);
    double* Gp = a.G + pbase;
    const double half_omega = 0.5 * P.omega;
    for (int m = tid; m <= lmax; m += nt) {
      const int k = m % n;
      const int nk = (k == 0) ? 0 : n - k;
      const double2 zk = buf[k], znk = buf[nk];
      // X_N = (Z_k + conj Z_nk) / 2, X_S = (Z_k - conj Z_nk) / (2 i); Omega folded in
      const double2 xn = make_double2((zk.x + znk.x) * half_omega, (zk.y - znk.y) * half_omega);
      const double2 xs = make_double2((zk.y + znk.y) * half_omega, -(zk.x - znk.x) * half_omega);
      const double2 ph = expipi(-(int64_t)m * rp.ph_num, rp.ph_den);
      const double2 gn = cmul(xn, ph), gs = cmul(xs, ph);
      *reinterpret_cast<double4*>(Gp + (size_t)m * 4) =
          make_double4(gn.x + gs.x, gn.y + gs.y, gn.x - gs.x, gn.y - gs.y);
    }
  }
}

}  // namespace

hipError_t launch_phase_b_f64(const PlanDev& P, const PhaseBArgs& a, size_t lds_bytes,
                              hipStream_t s) {
  static size_t attr_bytes = 0;
  if (lds_bytes > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)phase_b_f64_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    attr_bytes = lds_bytes;
  }
  dim3 grid(P.npairs, a.nmaps);
  hipLaunchKernelGGL(phase_b_f64_kernel, grid, dim3(256), lds_bytes, s, P, a);
  return hipGetLastError();
}

}  // namespace mwf
