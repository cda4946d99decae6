// Host runtime and C ABI of libmwf: plan construction (geometry, coefficient
// tables, polar-skip work lists, device buffers) and the sweep driver of the
// messenger iteration (Elsner & Wandelt, Sect. 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "mwf_internal.hpp"

namespace mwf {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace mwf

using namespace mwf;

struct wf_plan_s {
  int nside = 0, lmax = 0, dtype = WF_F64, max_batch = 1;
  int64_t npix = 0, nalm = 0;
  int nrings = 0, npairs = 0;
  double tau = 0.0, omega = 0.0;
  hipStream_t stream = nullptr;       // plan-time uploads
  hipStream_t last_stream = nullptr;  // stream of the last enqueued call
  size_t lds_phase_b = 0;
  int nitems_ana = 0, nitems_syn = 0, nitems_m = 0;
  int flags = 0;
  int64_t units_active = 0;
  std::vector<int32_t> n_active;
  // device allocations
  std::vector<void*> allocs;
  RingPair* d_pairs = nullptr;
  void* d_q = nullptr;
  double* d_cl = nullptr;
  double* d_A = nullptr;
  double* d_C = nullptr;
  int64_t* d_row_off = nullptr;
  double* d_norm = nullptr;
  int32_t* d_nact = nullptr;
  int32_t* d_nblk = nullptr;
  double2* d_tw = nullptr;
  double2* d_blue = nullptr;
  double2* d_chirp = nullptr;
  float2* d_tw32 = nullptr;
  float2* d_chirp32 = nullptr;
  float2* d_blue32 = nullptr;
  int32_t* d_ring_small = nullptr;  // ring pairs whose FFT has at most SMALL_FFT points
  int32_t* d_ring_large = nullptr;
  int32_t* d_ring_all = nullptr;
  RingClass ring_small{}, ring_large{}, ring_all{};
  WorkItem* d_items_ana = nullptr; // (m, analysis block), longest first
  WorkItem* d_items_syn = nullptr; // (m, synthesis block), longest first
  WorkItem* d_items_m = nullptr;   // (m, 0), one per m
  WorkItem* d_items_mfa = nullptr; // matrix-core analysis items (256 ring pairs)
  WorkItem* d_items_mfs = nullptr; // matrix-core synthesis items (64 ring pairs)
  int nitems_mfa = 0, nitems_mfs = 0;
  float* d_partial32 = nullptr;    // [blk256][nalm][batch][2]
  float* d_bcoef32 = nullptr;      // [rows_total][batch][2]
  void* d_G = nullptr;             // [batch][pair][m][4] in the storage type
  void* d_F = nullptr;
  size_t elem = 8;                 // bytes per stored real (8 for WF_F64, 4 otherwise)
  double2* d_partial = nullptr;    // [batch][blk][nalm]
  double2* d_bcoef = nullptr;      // [batch][rows_total]
  PlanDev dev{};
};

namespace {

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

// In-place iterative radix-2 FFT in long double (host, plan time only).
void host_fft(std::vector<std::complex<long double>>& a, int sign) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  const long double pi = 3.141592653589793238462643383279502884L;
  for (size_t len = 2; len <= n; len <<= 1) {
    for (size_t k = 0; k < len / 2; ++k) {
      const long double ang = sign * 2.0L * pi * (long double)k / (long double)len;
      const std::complex<long double> w(cosl(ang), sinl(ang));
      for (size_t i = k; i < n; i += len) {
        const auto u = a[i], v = a[i + len / 2] * w;
        a[i] = u + v;
        a[i + len / 2] = u - v;
      }
    }
  }
}

// Ring geometry of the HEALPix RING scheme (Gorski et al. 2005), ring i = 1..4n-1.
struct RingGeo {
  double z;
  int64_t start;
  int32_t nphi, ph_num, ph_den;
};

RingGeo ring_geo(int n, int i) {
  RingGeo g{};
  const int64_t npix = 12LL * n * n;
  if (i < n) {
    g.z = 1.0 - (double)((int64_t)i * i) / (3.0 * n * n);
    g.nphi = 4 * i;
    g.ph_num = 1;
    g.ph_den = 4 * i;
    g.start = 2LL * i * (i - 1);
  } else if (i <= 3 * n) {
    g.z = 2.0 * (2 * n - i) / (3.0 * n);
    g.nphi = 4 * n;
    g.ph_num = (i - n + 1) % 2;
    g.ph_den = 4 * n;
    g.start = 2LL * n * (n - 1) + 4LL * n * (i - n);
  } else {
    const int ip = 4 * n - i;
    g.z = -(1.0 - (double)((int64_t)ip * ip) / (3.0 * n * n));
    g.nphi = 4 * ip;
    g.ph_num = 1;
    g.ph_den = 4 * ip;
    g.start = npix - 2LL * ip * (ip + 1);
  }
  return g;
}

template <class T>
int dev_alloc(wf_plan_s* p, T** ptr, size_t count) {
  void* v = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&v, count * sizeof(T));
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? WF_ENOMEM : WF_EDEVICE,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  p->allocs.push_back(v);
  *ptr = static_cast<T*>(v);
  return WF_OK;
}

template <class T>
int upload(wf_plan_s* p, T** ptr, const std::vector<T>& host) {
  int rc = dev_alloc(p, ptr, host.size());
  if (rc) return rc;
  MWF_HIP(hipMemcpyAsync(*ptr, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice,
                         p->stream));
  return WF_OK;
}

// Ring pairs per analysis work item: two per lane once there are enough rings
// (the cross-lane reduction is then shared by two rings); synthesis uses one per
// lane so that long recurrences are spread over as many waves as possible.
// Ring pairs whose transform (n, or the Bluestein length M) has at most this many
// points run one wave per pair; longer ones a 512-thread workgroup.
constexpr int SMALL_FFT = 1024;
constexpr int SPLIT_MIN_MAPS = 4;

int ana_ring_block(int npairs) { return npairs <= 64 ? 64 : (npairs <= 128 ? 128 : 256); }
int syn_ring_block(int npairs) { return npairs <= 64 ? 64 : (npairs <= 128 ? 128 : 256); }

size_t buffer_bytes(int nside, int lmax, int nmaps, int* ring_block_out, int* nblk_out) {
  const int npairs = 2 * nside;
  const int rb = ana_ring_block(npairs);
  const int nblk = (npairs + rb - 1) / rb;
  if (ring_block_out) *ring_block_out = rb;
  if (nblk_out) *nblk_out = nblk;
  const size_t nalm = (size_t)(lmax + 1) * (lmax + 2) / 2;
  const size_t gf = (size_t)nmaps * npairs * (lmax + 1) * 4 * sizeof(double);
  const size_t part = (size_t)nmaps * nblk * nalm * sizeof(double2);
  return 2 * gf + part;
}

size_t table_bytes(int nside, int lmax) {
  const size_t npix = 12ULL * nside * nside;
  const size_t nalm = (size_t)(lmax + 1) * (lmax + 2) / 2;
  const size_t rows = nalm + (size_t)(lmax + 1) * CHUNK;
  // q, A, C, Bluestein (upper bound 16 n per cap ring pair), reach scratch
  size_t blue = 0;
  for (int i = 1; i < nside; ++i)
    if (!is_pow2(4 * i)) blue += (size_t)1 << ilog2(8 * i - 1);
  return npix * 8 + 2 * rows * 8 + blue * 16 + (size_t)(lmax + 1) * 2 * nside +
         (size_t)(8 * nside + 64) * 16 + 64 * 1024;
}

int validate_plan_args(int nside, int lmax, const double* cl, const double* ninv, const wf_plan_opts* o) {
  if (nside < 1 || nside > 1024 || !is_pow2(nside))
    return fail(WF_EINVAL, "nside must be a power of two in [1, 1024]");
  if (lmax < 0 || lmax > 4 * nside - 1 || lmax > 2048)
    return fail(WF_EINVAL, "lmax must satisfy 0 <= lmax <= min(4 nside - 1, 2048)");
  if (!cl || !ninv) return fail(WF_EINVAL, "cl and ninv must not be NULL");
  if (o) {
    if (o->dtype != WF_F64 && o->dtype != WF_F32 && o->dtype != WF_BF16X3 && o->dtype != WF_BF16X6)
      return fail(WF_EINVAL, "unknown dtype");
    if (o->max_batch < 0) return fail(WF_EINVAL, "max_batch must be >= 0");
    if (o->flags & ~WF_FLAG_TIMING) return fail(WF_EINVAL, "unknown flags");
  }
  return WF_OK;
}

}  // namespace

extern "C" {

const char* wf_strerror(int status) {
  switch (status) {
    case WF_OK: return "ok";
    case WF_EINVAL: return "invalid argument";
    case WF_ENOMEM: return "out of memory";
    case WF_EDEVICE: return "device error";
    case WF_EUNSUPPORTED: return "unsupported";
    case WF_EBUSY: return "busy";
    case WF_ENOTREADY: return "not ready";
    default: return "unknown status";
  }
}

const char* wf_last_error(void) { return g_last_error.c_str(); }

int wf_footprint(int32_t nside, int32_t lmax, int32_t dtype, int32_t nmaps, size_t* bytes) {
  if (!bytes) return fail(WF_EINVAL, "bytes must not be NULL");
  if (nmaps < 1) return fail(WF_EINVAL, "nmaps must be >= 1");
  if (dtype != WF_F64 && dtype != WF_F32 && dtype != WF_BF16X3 && dtype != WF_BF16X6)
    return fail(WF_EINVAL, "unknown dtype");
  if (nside < 1 || nside > 1024 || !is_pow2(nside) || lmax < 0 || lmax > 4 * nside - 1 || lmax > 2048)
    return fail(WF_EINVAL, "bad nside / lmax");
  *bytes = table_bytes(nside, lmax) + buffer_bytes(nside, lmax, nmaps, nullptr, nullptr);
  return WF_OK;
}

int wf_pixel_angles(int32_t nside, double* theta, double* phi) {
  if (nside < 1 || nside > 8192 || !is_pow2(nside)) return fail(WF_EINVAL, "nside must be a power of two in [1, 8192]");
  if (!theta || !phi) return fail(WF_EINVAL, "theta and phi must not be NULL");
  const double pi = 3.141592653589793238462643383279502884;
  for (int i = 1; i <= 4 * nside - 1; ++i) {
    const RingGeo g = ring_geo(nside, i);
    const double th = std::acos(g.z);
    const double ph0 = pi * g.ph_num / g.ph_den;
    for (int j = 0; j < g.nphi; ++j) {
      theta[g.start + j] = th;
      phi[g.start + j] = ph0 + 2.0 * pi * j / g.nphi;
    }
  }
  return WF_OK;
}

void wf_destroy(wf_plan_t p) {
  if (!p) return;
  hipStreamSynchronize(p->stream);
  if (p->last_stream != p->stream) hipStreamSynchronize(p->last_stream);
  for (void* v : p->allocs) hipFree(v);
  delete p;
}

int wf_plan(wf_plan_t* out, int32_t nside, int32_t lmax, const double* cl, const double* ninv,
            const uint8_t* mask, const wf_plan_opts* opts, void* hip_stream) {
  if (!out) return fail(WF_EINVAL, "out must not be NULL");
  *out = nullptr;
  int rc = validate_plan_args(nside, lmax, cl, ninv, opts);
  if (rc) return rc;
  const int dtype = opts ? opts->dtype : WF_F64;
  const int64_t npix = 12LL * nside * nside;
  for (int l = 0; l <= lmax; ++l)
    if (!std::isfinite(cl[l]) || cl[l] < 0) return fail(WF_EINVAL, "cl must be finite and >= 0");
  double nmax = 0.0;
  for (int64_t p = 0; p < npix; ++p) {
    if (!std::isfinite(ninv[p]) || ninv[p] < 0) return fail(WF_EINVAL, "ninv must be finite and >= 0");
    if ((!mask || mask[p]) && ninv[p] > nmax) nmax = ninv[p];
  }
  if (!(nmax > 0)) return fail(WF_EINVAL, "no observed pixel (all ninv == 0 or masked)");

  wf_plan_s* p = new wf_plan_s();
  p->nside = nside;
  p->lmax = lmax;
  p->dtype = dtype;
  p->max_batch = (opts && opts->max_batch > 0) ? opts->max_batch : 1;
  p->flags = opts ? opts->flags : 0;
  p->npix = npix;
  p->nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
  p->nrings = 4 * nside - 1;
  p->npairs = 2 * nside;
  p->tau = 1.0 / nmax;
  p->omega = 4.0 * 3.141592653589793238462643383279502884 / (double)npix;
  p->stream = static_cast<hipStream_t>(hip_stream);
  auto bail = [&](int code) {
    wf_destroy(p);
    return code;
  };

  // ---- ring pairs, equator first
  std::vector<RingPair> pairs(p->npairs);
  std::vector<int> blue_len;        // distinct non-power-of-two ring lengths
  int tw_len = 4;
  size_t lds = 0;
  for (int q = 0; q < p->npairs; ++q) {
    const int i = 2 * nside - q;
    const RingGeo gn = ring_geo(nside, i);
    RingPair rp{};
    rp.z = gn.z;
    rp.sin_t = std::sqrt((1.0 - gn.z) * (1.0 + gn.z));
    rp.start_n = gn.start;
    rp.start_s = (q == 0) ? -1 : ring_geo(nside, 4 * nside - i).start;
    rp.nphi = gn.nphi;
    rp.ph_num = gn.ph_num;
    rp.ph_den = gn.ph_den;
    if (is_pow2(gn.nphi)) {
      rp.log2n = ilog2(gn.nphi);
      rp.bl_M = 0;
      tw_len = std::max(tw_len, gn.nphi);
      lds = std::max(lds, (size_t)gn.nphi * 16);
    } else {
      rp.log2n = -1;
      rp.bl_M = 1 << ilog2(2 * gn.nphi - 1);
      tw_len = std::max(tw_len, rp.bl_M);
      lds = std::max(lds, (size_t)rp.bl_M * 16);
      blue_len.push_back(gn.nphi);
    }
    pairs[q] = rp;
  }
  p->lds_phase_b = lds;

  // Bluestein filter spectra: H = FFT_M(h), h_j = exp(+i pi j^2 / n) for |j| < n
  const long double pi = 3.141592653589793238462643383279502884L;
  std::vector<double2> blue, chirp;
  {
    std::vector<int64_t> off_of(4 * nside + 1, -1), coff_of(4 * nside + 1, -1);
    for (int n : blue_len) {
      if (off_of[n] >= 0) continue;
      coff_of[n] = (int64_t)chirp.size();
      for (int j = 0; j < n; ++j) {
        const long double ang = -pi * (long double)(((int64_t)j * j) % (2LL * n)) / (long double)n;
        chirp.push_back(make_double2((double)cosl(ang), (double)sinl(ang)));
      }
      const int M = 1 << ilog2(2 * n - 1);
      std::vector<std::complex<long double>> h(M, 0.0L);
      for (int j = 0; j < n; ++j) {
        const long double ang = pi * (long double)(((int64_t)j * j) % (2LL * n)) / (long double)n;
        const std::complex<long double> w(cosl(ang), sinl(ang));
        h[j] = w;
        if (j) h[M - j] = w;
      }
      host_fft(h, -1);
      off_of[n] = (int64_t)blue.size();
      for (int k = 0; k < M; ++k) blue.push_back(make_double2((double)h[k].real(), (double)h[k].imag()));
    }
    for (auto& rp : pairs)
      if (rp.log2n < 0) {
        rp.bl_off = off_of[rp.nphi];
        rp.chirp_off = coff_of[rp.nphi];
      }
    if (blue.empty()) blue.push_back(make_double2(0.0, 0.0));
    if (chirp.empty()) chirp.push_back(make_double2(0.0, 0.0));
  }
  std::vector<double2> tw(tw_len / 2);
  for (int k = 0; k < tw_len / 2; ++k) {
    const long double ang = -2.0L * pi * (long double)k / (long double)tw_len;
    tw[k] = make_double2((double)cosl(ang), (double)sinl(ang));
  }

  // ---- per-pixel tau * ninv (0 where unobserved)
  std::vector<float> q32;
  std::vector<double> q(npix);
  for (int64_t i = 0; i < npix; ++i) q[i] = (mask && !mask[i]) ? 0.0 : p->tau * ninv[i];

  // ---- recurrence tables: rows per m, padded with CHUNK zeros
  std::vector<int64_t> row_off(lmax + 1);
  std::vector<double> A, C, norm(lmax + 1);
  {
    int64_t off = 0;
    for (int m = 0; m <= lmax; ++m) {
      row_off[m] = off;
      off += (lmax - m + 1) + ROW_PAD;
    }
    A.assign(off, 0.0);
    C.assign(off, 0.0);
    long double nm = 1.0L / sqrtl(4.0L * pi);
    for (int m = 0; m <= lmax; ++m) {
      if (m > 0) nm *= -sqrtl((2.0L * m + 1.0L) / (2.0L * m));
      norm[m] = (double)nm;
      auto alpha = [&](int l) {
        return sqrtl((4.0L * l * l - 1.0L) / ((long double)(l - m) * (long double)(l + m)));
      };
      const int64_t r = row_off[m];
      long double c_lm2 = 1.0L, c_lm1 = 1.0L;   // C_{l-2}, C_{l-1}
      A[r] = 0.0;
      C[r] = 1.0;
      if (m + 1 <= lmax) {
        A[r + 1] = (double)alpha(m + 1);
        C[r + 1] = 1.0;
      }
      for (int l = m + 2; l <= lmax; ++l) {
        const long double al = alpha(l), alm1 = alpha(l - 1);
        const long double cl_ = c_lm2 * al / alm1;
        A[r + (l - m)] = (double)(al * c_lm1 / cl_);
        C[r + (l - m)] = (double)cl_;
        c_lm2 = c_lm1;
        c_lm1 = cl_;
      }
    }
  }

  // ---- uploads
  if ((rc = upload(p, &p->d_pairs, pairs))) return bail(rc);
  if (dtype == WF_F64) {
    double* dq = nullptr;
    if ((rc = upload(p, &dq, q))) return bail(rc);
    p->d_q = dq;
  } else {
    q32.assign(q.begin(), q.end());
    float* dq = nullptr;
    if ((rc = upload(p, &dq, q32))) return bail(rc);
    p->d_q = dq;
  }
  const std::vector<double> cl_host(cl, cl + lmax + 1);
  if ((rc = upload(p, &p->d_cl, cl_host))) return bail(rc);
  if ((rc = upload(p, &p->d_A, A))) return bail(rc);
  if ((rc = upload(p, &p->d_C, C))) return bail(rc);
  if ((rc = upload(p, &p->d_row_off, row_off))) return bail(rc);
  if ((rc = upload(p, &p->d_norm, norm))) return bail(rc);
  if ((rc = upload(p, &p->d_tw, tw))) return bail(rc);
  if ((rc = upload(p, &p->d_blue, blue))) return bail(rc);
  if ((rc = upload(p, &p->d_chirp, chirp))) return bail(rc);
  auto to32 = [](const std::vector<double2>& v) {
    std::vector<float2> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = make_float2((float)v[i].x, (float)v[i].y);
    return o;
  };
  const std::vector<float2> tw32 = to32(tw), chirp32 = to32(chirp), blue32 = to32(blue);
  if ((rc = upload(p, &p->d_tw32, tw32))) return bail(rc);
  if ((rc = upload(p, &p->d_chirp32, chirp32))) return bail(rc);
  if ((rc = upload(p, &p->d_blue32, blue32))) return bail(rc);
  // ring classes by transform length
  std::vector<int32_t> qs_small, qs_large;
  int len_small = 4, len_large = 4;
  for (int qq = 0; qq < p->npairs; ++qq) {
    const int L = pairs[qq].log2n >= 0 ? pairs[qq].nphi : pairs[qq].bl_M;
    if (L <= SMALL_FFT) {
      qs_small.push_back(qq);
      len_small = std::max(len_small, L);
    } else {
      qs_large.push_back(qq);
      len_large = std::max(len_large, L);
    }
  }
  std::vector<int32_t> qs_all(p->npairs);
  for (int qq = 0; qq < p->npairs; ++qq) qs_all[qq] = qq;
  if ((rc = upload(p, &p->d_ring_small, qs_small))) return bail(rc);
  if ((rc = upload(p, &p->d_ring_large, qs_large))) return bail(rc);
  if ((rc = upload(p, &p->d_ring_all, qs_all))) return bail(rc);
  p->ring_small = RingClass{p->d_ring_small, (int32_t)qs_small.size(), len_small};
  p->ring_large = RingClass{p->d_ring_large, (int32_t)qs_large.size(), len_large};
  p->ring_all = RingClass{p->d_ring_all, p->npairs, std::max(len_small, len_large)};

  int ring_block = 0, nblk_max = 0;
  buffer_bytes(nside, lmax, p->max_batch, &ring_block, &nblk_max);

  PlanDev& D = p->dev;
  D.nside = nside;
  D.lmax = lmax;
  D.npairs = p->npairs;
  D.nrings = p->nrings;
  D.npix = npix;
  D.nalm = p->nalm;
  D.tau = p->tau;
  D.omega = p->omega;
  D.ring_block_ana = ring_block;
  D.ring_block_syn = syn_ring_block(p->npairs);
  D.nblk_max = nblk_max;
  D.pairs = p->d_pairs;
  D.q = p->d_q;
  D.cl = p->d_cl;
  D.A = p->d_A;
  D.C = p->d_C;
  D.row_off = p->d_row_off;
  D.norm_m = p->d_norm;
  D.twiddle = p->d_tw;
  D.tw_len = tw_len;
  D.bluestein = p->d_blue;
  D.chirp = p->d_chirp;
  D.twiddle32 = p->d_tw32;
  D.chirp32 = p->d_chirp32;
  D.bluestein32 = p->d_blue32;
  D.rows_total = (int64_t)A.size();

  // ---- polar skip: ring pairs whose lambda_lm never leaves the negligible range
  {
    uint8_t* d_reach = nullptr;
    void* raw = nullptr;
    MWF_HIP(hipMalloc(&raw, (size_t)(lmax + 1) * p->npairs));
    d_reach = static_cast<uint8_t*>(raw);
    hipError_t e = launch_reach(D, d_reach, p->stream);
    std::vector<uint8_t> reach((size_t)(lmax + 1) * p->npairs);
    if (e == hipSuccess)
      e = hipMemcpyAsync(reach.data(), d_reach, reach.size(), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    hipFree(raw);
    if (e != hipSuccess) {
      set_error(std::string("plan reach kernel: ") + hipGetErrorString(e));
      return bail(WF_EDEVICE);
    }
    p->n_active.assign(lmax + 1, 0);
    p->units_active = 0;
    for (int m = 0; m <= lmax; ++m) {
      int na = 0;
      for (int qq = 0; qq < p->npairs; ++qq)
        if (reach[(size_t)m * p->npairs + qq]) na = qq + 1;
      p->n_active[m] = na;
      p->units_active += (int64_t)na * (lmax - m + 1);
    }
  }
  std::vector<int32_t> nblk(lmax + 1);
  std::vector<WorkItem> items_m;
  // (m, ring block) items, longest first so that the hardware dispatcher balances the tail
  auto make_items = [&](int rb) {
    std::vector<WorkItem> items;
    for (int m = 0; m <= lmax; ++m) {
      const int nb = (p->n_active[m] + rb - 1) / rb;
      for (int b = 0; b < nb; ++b) items.push_back({m, b});
    }
    std::stable_sort(items.begin(), items.end(), [&](const WorkItem& a, const WorkItem& b) {
      auto c = [&](const WorkItem& w) {
        const int rings = std::min(rb, p->n_active[w.m] - w.blk * rb);
        return (double)(lmax - w.m + 1) * (double)std::max(rings, 1);
      };
      return c(a) > c(b);
    });
    if (items.empty()) items.push_back({0, 0});
    return items;
  };
  for (int m = 0; m <= lmax; ++m) {
    nblk[m] = (p->n_active[m] + ring_block - 1) / ring_block;
    items_m.push_back({m, 0});
  }
  const std::vector<WorkItem> items_ana = make_items(ring_block);
  const std::vector<WorkItem> items_syn = make_items(syn_ring_block(p->npairs));
  const std::vector<WorkItem> items_mfa = make_items(256);
  const std::vector<WorkItem> items_mfs = make_items(64);
  p->nitems_mfa = (int)items_mfa.size();
  p->nitems_mfs = (int)items_mfs.size();
  p->nitems_ana = (int)items_ana.size();
  p->nitems_syn = (int)items_syn.size();
  p->nitems_m = (int)items_m.size();
  if ((rc = upload(p, &p->d_nact, p->n_active))) return bail(rc);
  if ((rc = upload(p, &p->d_nblk, nblk))) return bail(rc);
  if ((rc = upload(p, &p->d_items_ana, items_ana))) return bail(rc);
  if ((rc = upload(p, &p->d_items_syn, items_syn))) return bail(rc);
  if ((rc = upload(p, &p->d_items_mfa, items_mfa))) return bail(rc);
  if ((rc = upload(p, &p->d_items_mfs, items_mfs))) return bail(rc);
  if ((rc = upload(p, &p->d_items_m, items_m))) return bail(rc);
  D.n_active = p->d_nact;
  D.nblk = p->d_nblk;

  // ---- work buffers
  p->elem = (dtype == WF_F64) ? 8 : 4;
  const size_t gf = (size_t)p->max_batch * p->npairs * (lmax + 1) * 4 * p->elem;
  {
    uint8_t* g = nullptr;
    uint8_t* f = nullptr;
    if ((rc = dev_alloc(p, &g, gf))) return bail(rc);
    if ((rc = dev_alloc(p, &f, gf))) return bail(rc);
    p->d_G = g;
    p->d_F = f;
  }
  if (dtype == WF_F64) {
    if ((rc = dev_alloc(p, &p->d_partial, (size_t)p->max_batch * nblk_max * p->nalm))) return bail(rc);
    if ((rc = dev_alloc(p, &p->d_bcoef, (size_t)p->max_batch * D.rows_total))) return bail(rc);
  } else {
    const size_t nb256 = (size_t)(p->npairs + 255) / 256;
    if ((rc = dev_alloc(p, &p->d_partial32, nb256 * p->nalm * p->max_batch * 2))) return bail(rc);
    if ((rc = dev_alloc(p, &p->d_bcoef32, (size_t)D.rows_total * p->max_batch * 2))) return bail(rc);
  }
  // F entries of skipped (m, ring pair) combinations are never written: keep them zero
  if (hipMemsetAsync(p->d_F, 0, gf, p->stream) != hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess) {
    set_error("initialising work buffers failed");
    return bail(WF_EDEVICE);
  }
  *out = p;
  return WF_OK;
}

int wf_plan_info(wf_plan_t p, int64_t* npix, int64_t* nalm, double* tau, int64_t* units_all,
                 int64_t* units_active) {
  if (!p) return fail(WF_EINVAL, "plan must not be NULL");
  if (npix) *npix = p->npix;
  if (nalm) *nalm = p->nalm;
  if (tau) *tau = p->tau;
  if (units_all) *units_all = (int64_t)p->npairs * p->nalm;
  if (units_active) *units_active = p->units_active;
  return WF_OK;
}

int wf_sync(wf_plan_t p) {
  if (!p) return fail(WF_EINVAL, "plan must not be NULL");
  MWF_HIP(hipStreamSynchronize(p->stream));
  if (p->last_stream != p->stream) MWF_HIP(hipStreamSynchronize(p->last_stream));
  MWF_HIP(hipGetLastError());
  return WF_OK;
}

}  // extern "C"

namespace {

// Per-solve kernel timing (WF_FLAG_TIMING): an event before and after every launch.
struct Timer {
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;   // 0 ring, 1 analysis, 2 synthesis
  hipStream_t s = nullptr;
  ~Timer() {
    for (auto e : ev) hipEventDestroy(e);
  }
  int begin() {
    if (!on) return WF_OK;
    hipEvent_t e;
    MWF_HIP(hipEventCreate(&e));
    MWF_HIP(hipEventRecord(e, s));
    ev.push_back(e);
    return WF_OK;
  }
  int end(int k) {
    if (!on) return WF_OK;
    hipEvent_t e;
    MWF_HIP(hipEventCreate(&e));
    MWF_HIP(hipEventRecord(e, s));
    ev.push_back(e);
    kind.push_back(k);
    return WF_OK;
  }
  int collect(wf_stats* st) {
    if (!on || !st) return WF_OK;
    MWF_HIP(hipEventSynchronize(ev.back()));
    double ms[3] = {0, 0, 0};
    int cnt[3] = {0, 0, 0};
    for (size_t i = 0; i < kind.size(); ++i) {
      float t = 0.f;
      MWF_HIP(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
      ms[kind[i]] += t;
      cnt[kind[i]] += 1;
    }
    st->timed = 1;
    st->ms_ring = ms[0];
    st->ms_analysis = ms[1];
    st->ms_synthesis = ms[2];
    st->n_ring = cnt[0];
    st->n_analysis = cnt[1];
    st->n_synthesis = cnt[2];
    return WF_OK;
  }
};

thread_local Timer* g_timer = nullptr;

int run_phase_b(wf_plan_s* p, hipStream_t s, int mode, int nmaps, double lam, const void* d,
                const void* map_in, void* map_out) {
  PhaseBArgs a{};
  a.mode = mode;
  a.nmaps = nmaps;
  a.lambda = lam;
  a.F = p->d_F;
  a.G = p->d_G;
  a.d = d;
  a.map_in = map_in;
  a.map_out = map_out;
  if (g_timer && g_timer->begin()) return WF_EDEVICE;
  // With few maps one launch over all ring pairs fills the GPU better than two
  // back-to-back launches split by transform length.
  const RingClass none{nullptr, 0, 4};
  if (nmaps < SPLIT_MIN_MAPS)
    MWF_HIP(launch_phase_b(p->dev, a, none, p->ring_all, p->dtype != WF_F64, s));
  else
    MWF_HIP(launch_phase_b(p->dev, a, p->ring_small, p->ring_large, p->dtype != WF_F64, s));
  if (g_timer && g_timer->end(0)) return WF_EDEVICE;
  return WF_OK;
}

MfmaArgs mfma_args(wf_plan_s* p, int mode, int nmaps, double lam, const void* alm_in, void* alm_out) {
  MfmaArgs a{};
  a.mode = mode;
  a.nmaps = nmaps;
  a.lambda = lam;
  a.G = static_cast<const float*>(p->d_G);
  a.F = static_cast<float*>(p->d_F);
  a.partial = p->d_partial32;
  a.bcoef = p->d_bcoef32;
  a.alm_in = static_cast<const float2*>(alm_in);
  a.alm_out = static_cast<float2*>(alm_out);
  return a;
}

int run_analysis(wf_plan_s* p, hipStream_t s, int nmaps) {
  if (g_timer && g_timer->begin()) return WF_EDEVICE;
  if (p->dtype != WF_F64) {
    MWF_HIP(launch_mfma_analysis(p->dev, p->d_items_mfa, p->nitems_mfa, p->dtype,
                                 mfma_args(p, 0, nmaps, 1.0, nullptr, nullptr), s));
  } else {
    MWF_HIP(launch_legendre_analysis_f64(p->dev, p->d_items_ana, p->nitems_ana, nmaps,
                                         static_cast<const double*>(p->d_G), p->d_partial, s));
  }
  if (g_timer && g_timer->end(1)) return WF_EDEVICE;
  return WF_OK;
}

int run_synthesis(wf_plan_s* p, hipStream_t s, int mode, int nmaps, double lam,
                  const void* alm_in, void* alm_out) {
  if (p->dtype != WF_F64) {
    const MfmaArgs ma = mfma_args(p, mode, nmaps, lam, alm_in, alm_out);
    if (g_timer && g_timer->begin()) return WF_EDEVICE;
    MWF_HIP(launch_mfma_coeff(p->dev, ma, s));
    if (mode != SY_ALM_ONLY)
      MWF_HIP(launch_mfma_synthesis(p->dev, p->d_items_mfs, p->nitems_mfs, p->dtype, ma, s));
    if (g_timer && g_timer->end(2)) return WF_EDEVICE;
    return WF_OK;
  }
  SynthArgs a{};
  a.mode = mode;
  a.nmaps = nmaps;
  a.lambda = lam;
  a.partial = p->d_partial;
  a.alm_in = static_cast<const double2*>(alm_in);
  a.alm_out = static_cast<double2*>(alm_out);
  a.F = static_cast<double*>(p->d_F);
  a.bcoef = p->d_bcoef;
  if (g_timer && g_timer->begin()) return WF_EDEVICE;
  MWF_HIP(launch_legendre_coeff(p->dev, a, s));
  if (mode != SY_ALM_ONLY)
    MWF_HIP(launch_legendre_synthesis_f64(p->dev, p->d_items_syn, p->nitems_syn, a, s));
  if (g_timer && g_timer->end(2)) return WF_EDEVICE;
  return WF_OK;
}

int check_batch(wf_plan_s* p, int nmaps) {
  if (!p) return fail(WF_EINVAL, "plan must not be NULL");
  if (nmaps < 1 || nmaps > p->max_batch)
    return fail(WF_EINVAL, "nmaps must be in [1, max_batch] (max_batch = " +
                               std::to_string(p->max_batch) + ")");
  return WF_OK;
}

}  // namespace

extern "C" {

int wf_solve_batch(wf_plan_t p, int32_t nmaps, const void* d, void* s_wf, void* s_alm,
                   const double* lambda, int32_t nsweeps, void* hip_stream, wf_stats* stats) {
  int rc = check_batch(p, nmaps);
  if (rc) return rc;
  if (!d || !s_wf) return fail(WF_EINVAL, "d and s_wf must not be NULL");
  if (!lambda || nsweeps < 1) return fail(WF_EINVAL, "need a schedule of at least one lambda");
  for (int k = 0; k < nsweeps; ++k)
    if (!std::isfinite(lambda[k]) || !(lambda[k] > 0))
      return fail(WF_EINVAL, "every lambda must be finite and > 0");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  const void* dd = d;
  Timer timer;
  timer.on = (p->flags & WF_FLAG_TIMING) != 0;
  timer.s = s;
  struct Guard {
    Timer* t;
    Guard(Timer* x) : t(x) { g_timer = x->on ? x : nullptr; }
    ~Guard() { g_timer = nullptr; }
  } guard(&timer);
  for (int k = 0; k < nsweeps; ++k) {
    const int mode = (k == 0 ? 0 : PB_SYNTH) | PB_UPDATE | PB_ANALYSIS;
    if ((rc = run_phase_b(p, s, mode, nmaps, lambda[k], dd, nullptr, nullptr))) return rc;
    if ((rc = run_analysis(p, s, nmaps))) return rc;
    void* alm_out = (k == nsweeps - 1) ? s_alm : nullptr;
    if ((rc = run_synthesis(p, s, SY_FROM_PARTIAL, nmaps, lambda[k], nullptr, alm_out))) return rc;
  }
  if ((rc = run_phase_b(p, s, PB_SYNTH | PB_WRITE_MAP, nmaps, 1.0, nullptr, nullptr, s_wf)))
    return rc;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->sweeps_done = nsweeps;
    if ((rc = timer.collect(stats))) return rc;
  }
  return WF_OK;
}

int wf_solve(wf_plan_t p, const void* d, void* s_wf, void* s_alm, const double* lambda,
             int32_t nsweeps, void* hip_stream, wf_stats* stats) {
  return wf_solve_batch(p, 1, d, s_wf, s_alm, lambda, nsweeps, hip_stream, stats);
}

int sht_map2alm(wf_plan_t p, int32_t nmaps, const void* map, void* alm, void* hip_stream) {
  int rc = check_batch(p, nmaps);
  if (rc) return rc;
  if (!map || !alm) return fail(WF_EINVAL, "map and alm must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  if ((rc = run_phase_b(p, s, PB_READ_MAP | PB_ANALYSIS, nmaps, 1.0, nullptr, map, nullptr)))
    return rc;
  if ((rc = run_analysis(p, s, nmaps))) return rc;
  return run_synthesis(p, s, SY_ALM_ONLY, nmaps, 1.0, nullptr, alm);
}

int sht_alm2map(wf_plan_t p, int32_t nmaps, const void* alm, void* map, void* hip_stream) {
  int rc = check_batch(p, nmaps);
  if (rc) return rc;
  if (!map || !alm) return fail(WF_EINVAL, "map and alm must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  if ((rc = run_synthesis(p, s, SY_FROM_ALM, nmaps, 1.0, alm, nullptr)))
    return rc;
  return run_phase_b(p, s, PB_SYNTH | PB_WRITE_MAP, nmaps, 1.0, nullptr, nullptr, map);
}

}  // extern "C"
