// Polarised plans (T, Q, U): host side of the polarised messenger solve and transforms.
//
// Sect. 3 filters temperature and polarisation maps together, with separate
// temperature and polarisation masks. Per pixel the noise is a 3x3 covariance N_p
// (given as its inverse, six entries), per harmonic mode the signal covariance is
// the 3x3 C_l of TT, EE, BB, TE. The messenger covariance is T = tau 1 with tau the
// smallest eigenvalue of N over all pixels (the largest tau with N - T positive
// semi-definite; for a diagonal N it is min(diag N) as in Sect. 2).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.hpp"

namespace mwf {
namespace {

constexpr long double PI_L = 3.141592653589793238462643383279502884L;

// Largest eigenvalue of the symmetric 3x3 [[a, d, e], [d, b, f], [e, f, c]] and whether
// the smallest is >= -tol * the largest (positive semi-definite up to rounding).
// Trigonometric solution of the characteristic cubic (Smith 1961), in long double.
void eig3(double a, double b, double c, double d, double e, double f, double* lmax, bool* psd) {
  const long double p1 = (long double)d * d + (long double)e * e + (long double)f * f;
  long double l1, l3;
  if (p1 == 0.0L) {
    l1 = std::max({(long double)a, (long double)b, (long double)c});
    l3 = std::min({(long double)a, (long double)b, (long double)c});
  } else {
    const long double q = ((long double)a + b + c) / 3.0L;
    const long double aq = a - q, bq = b - q, cq = c - q;
    const long double p2 = aq * aq + bq * bq + cq * cq + 2.0L * p1;
    const long double p = sqrtl(p2 / 6.0L);
    // det((M - q I) / p) / 2
    const long double B00 = aq / p, B11 = bq / p, B22 = cq / p, B01 = d / p, B02 = e / p, B12 = f / p;
    long double r = (B00 * (B11 * B22 - B12 * B12) - B01 * (B01 * B22 - B12 * B02) + B02 * (B01 * B12 - B11 * B02)) / 2.0L;
    r = std::min(1.0L, std::max(-1.0L, r));
    const long double phi = acosl(r) / 3.0L;
    l1 = q + 2.0L * p * cosl(phi);
    l3 = q + 2.0L * p * cosl(phi + 2.0L * PI_L / 3.0L);
  }
  *lmax = (double)l1;
  *psd = l3 >= -1e-12L * std::max(fabsl(l1), 1e-300L);
}

int validate_pol_shape(int nside, int lmax) {
  if (nside < 1 || nside > 512 || (nside & (nside - 1)))
    return fail(WF_EINVAL, "polarised plans: nside must be a power of two in [1, 512]");
  if (lmax < 0 || lmax > 4 * nside - 1) return fail(WF_EINVAL, "lmax must satisfy 0 <= lmax <= 4 nside - 1");
  return WF_OK;
}

}  // namespace
}  // namespace mwf

using namespace mwf;

struct wf_pol_plan_s {
  std::shared_ptr<Geometry> geo;
  int max_batch = 1, flags = 0;
  double tau = 0.0;
  int64_t n_obs_t = 0, n_obs_p = 0;
  hipStream_t stream = nullptr, last_stream = nullptr;
  PlanDev dev{};
  Spin2Dev s2{};
  double* q6 = nullptr;
  double* cl4 = nullptr;
  double* G = nullptr;
  double* F = nullptr;
  double2* partial_t = nullptr;
  double* partial_eb = nullptr;
  double2* bcoef_t = nullptr;
  double2* bcoef_eb = nullptr;
  int32_t* nblk2_m = nullptr;
  int nblk2 = 1;
  DevMem mem;
};

namespace {

// Per-kind launch timing (WF_FLAG_TIMING): events recorded around every phase.
struct PolTimer {
  bool on = false;
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;
  ~PolTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  int mark() {
    if (!on) return WF_OK;
    hipEvent_t e;
    // Timing only: no system-scope fence (no cache write-back and invalidation per event).
    MWF_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    MWF_HIP(hipEventRecord(e, s));
    ev.push_back(e);
    return WF_OK;
  }
  int collect(wf_stats* st) {
    if (!on || !st || ev.empty()) return WF_OK;
    MWF_HIP(hipStreamSynchronize(s));
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

#define POL_TIMED(tm, k, ...)                     \
  do {                                            \
    if (int rc_ = (tm).mark()) return rc_;        \
    { __VA_ARGS__; }                              \
    if (int rc_ = (tm).mark()) return rc_;        \
    if ((tm).on) (tm).kind.push_back(k);          \
  } while (0)

int pol_ring(wf_pol_plan_s* p, hipStream_t s, int mode, int nmaps, double lam, const double* d, const double* map_in,
             double* map_out, PolTimer& tm) {
  PolRingArgs a{};
  a.mode = mode;
  a.nmaps = nmaps;
  a.field_maps = p->max_batch;
  a.lambda = lam;
  a.F = p->F;
  a.G = p->G;
  a.d = d;
  a.map_in = map_in;
  a.map_out = map_out;
  a.q6 = p->q6;
  POL_TIMED(tm, 0, MWF_HIP(launch_pol_ring(p->dev, a, p->geo->ring_cls[0], s)));
  return WF_OK;
}

int pol_analysis(wf_pol_plan_s* p, hipStream_t s, int nmaps, PolTimer& tm) {
  const Geometry& g = *p->geo;
  POL_TIMED(tm, 1, {
    MWF_HIP(launch_legendre_analysis_f64(p->dev, g.items_ana, g.bins_ana, g.nbins_ana, nmaps, p->G, p->partial_t, s));
    MWF_HIP(launch_spin2_analysis(p->dev, p->s2, nmaps, p->G, p->partial_eb, p->nblk2, s));
  });
  return WF_OK;
}

int pol_synthesis(wf_pol_plan_s* p, hipStream_t s, int mode, int nmaps, double lam, const void* alm_in, void* alm_out,
                  PolTimer& tm) {
  const Geometry& g = *p->geo;
  PolCoeffArgs c{};
  c.mode = mode;
  c.nmaps = nmaps;
  c.lambda = lam;
  c.partial_t = p->partial_t;
  c.partial_eb = p->partial_eb;
  c.nblk2 = p->nblk2;
  c.nblk2_m = p->nblk2_m;
  c.alm_in = static_cast<const double2*>(alm_in);
  c.alm_out = static_cast<double2*>(alm_out);
  c.bcoef_t = p->bcoef_t;
  c.bcoef_eb = p->bcoef_eb;
  c.cl4 = p->cl4;
  SynthArgs a{};
  a.mode = SY_FROM_ALM;
  a.nmaps = nmaps;
  a.bcoef = p->bcoef_t;
  a.F = p->F;
  POL_TIMED(tm, 2, {
    MWF_HIP(launch_pol_coeff(p->dev, p->s2, c, s));
    if (mode != SY_ALM_ONLY) {
      MWF_HIP(launch_legendre_synthesis_f64(p->dev, g.items_syn, g.bins_syn, g.nbins_syn, a, s));
      MWF_HIP(launch_spin2_synthesis(p->dev, p->s2, nmaps, p->bcoef_eb, p->F, s));
    }
  });
  return WF_OK;
}

int check_pol_batch(wf_pol_plan_s* p, int nmaps) {
  if (!p) return fail(WF_EINVAL, "plan must not be NULL");
  if (nmaps < 1 || nmaps > p->max_batch)
    return fail(WF_EINVAL, "nmaps must be in [1, max_batch] (max_batch = " + std::to_string(p->max_batch) + ")");
  return WF_OK;
}

// Spin-2 recurrence tables in the padded per-m row layout of the spin-0 tables:
// u_l = (A_l z + (s/2) B_l) u_{l-1} - u_{l-2}, (s)lambda_lm = K_l u_l (see pol.hip), from
// the Wigner-d recurrence y_{l+1} = (a_l z + b_l) y_l - c_l y_{l-1} with, for s = 2,
//   a_l = sqrt((2l+3)(2l+1)) (l+1) / W_l,  b_l = sqrt((2l+3)(2l+1)) 2 m / (l W_l),
//   c_l = (l+1)/l sqrt((2l+3)/(2l-1)) sqrt((l^2-m^2)(l^2-4)) / W_l,
//   W_l = sqrt(((l+1)^2 - m^2)((l+1)^2 - 4)),
// K_l0 = K_l0+1 = 1, K_l = c_{l-1} K_{l-2}, A_l = a_{l-1} K_{l-1} / K_l, B_l = b_{l-1} K_{l-1} / K_l
// above l0 = max(m, 2); A = B = 0 at l <= l0 and K = 0 below l0.
void spin2_tables(int lmax, const std::vector<int64_t>& row_off, int64_t rows_total, std::vector<double>& A,
                  std::vector<double>& B, std::vector<double>& K, std::vector<double>& norm) {
  A.assign(rows_total, 0.0);
  B.assign(rows_total, 0.0);
  K.assign(rows_total, 0.0);
  norm.assign(lmax + 1, 0.0);
  for (int m = 0; m <= lmax; ++m) {
    const long double mm = m;
    if (m >= 2) norm[m] = (double)sqrtl(mm * (mm - 1.0L) / ((mm + 1.0L) * (mm + 2.0L)));
    else if (m == 0) norm[m] = (double)sqrtl(15.0L / (32.0L * PI_L));   // (+-2)lambda_20 / sin^2 theta
    else norm[m] = (double)sqrtl(5.0L / PI_L);                           // (+-2)lambda_21 / (sin theta (1 -+ z) / 4)
    const int l0 = std::max(m, 2);
    if (l0 > lmax) continue;
    const int64_t r = row_off[m];
    std::vector<long double> Kl(lmax + 2, 0.0L);
    Kl[l0] = 1.0L;
    if (l0 + 1 <= lmax) Kl[l0 + 1] = 1.0L;
    auto W = [&](long double l) { return sqrtl(((l + 1) * (l + 1) - mm * mm) * ((l + 1) * (l + 1) - 4.0L)); };
    for (int l = l0 + 2; l <= lmax; ++l) {
      const long double j = l - 1;
      const long double c = (j + 1) / j * sqrtl((2 * j + 3) / (2 * j - 1)) * sqrtl((j * j - mm * mm) * (j * j - 4.0L)) / W(j);
      Kl[l] = c * Kl[l - 2];
    }
    for (int l = l0; l <= lmax; ++l) K[r + (l - m)] = (double)Kl[l];
    for (int l = l0 + 1; l <= lmax; ++l) {
      const long double j = l - 1;
      const long double a = sqrtl((2 * j + 3) * (2 * j + 1)) * (j + 1) / W(j);
      const long double b = sqrtl((2 * j + 3) * (2 * j + 1)) * 2.0L * mm / (j * W(j));
      A[r + (l - m)] = (double)(a * Kl[l - 1] / Kl[l]);
      B[r + (l - m)] = (double)(b * Kl[l - 1] / Kl[l]);
    }
  }
}

}  // namespace

extern "C" {

int wf_pol_plan(wf_pol_plan_t* out, int32_t nside, int32_t lmax, const double* cl, const double* ninv,
                const uint8_t* mask, const wf_plan_opts* opts, void* hip_stream) {
  if (!out) return fail(WF_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (int rc = validate_pol_shape(nside, lmax)) return rc;
  if (!cl || !ninv) return fail(WF_EINVAL, "cl and ninv must not be NULL");
  if (opts) {
    if (opts->dtype != WF_F64) return fail(WF_EUNSUPPORTED, "polarised plans run in FP64 only (WF_F64)");
    if (opts->max_batch < 0) return fail(WF_EINVAL, "max_batch must be >= 0");
    if (opts->flags & ~WF_FLAG_TIMING) return fail(WF_EINVAL, "polarised plans accept WF_FLAG_TIMING only");
  }
  const int L1 = lmax + 1;
  for (int i = 0; i < 4 * L1; ++i)
    if (!std::isfinite(cl[i])) return fail(WF_EINVAL, "cl must be finite");
  for (int l = 0; l <= lmax; ++l) {
    const double tt = cl[l], ee = cl[L1 + l], bb = cl[2 * L1 + l], te = cl[3 * L1 + l];
    if (tt < 0 || ee < 0 || bb < 0) return fail(WF_EINVAL, "TT, EE and BB must be >= 0");
    if (te * te > tt * ee * (1.0 + 1e-12)) return fail(WF_EINVAL, "each C_l block must be positive semi-definite (TE^2 <= TT EE)");
    if (l < 2 && (ee != 0 || bb != 0 || te != 0)) return fail(WF_EINVAL, "E and B have no modes below l = 2: EE, BB, TE must be 0 there");
  }
  const int64_t npix = 12LL * nside * nside;
  std::vector<double> m6(6 * npix);
  double nmax = 0.0;
  int64_t nobs_t = 0, nobs_p = 0;
  for (int64_t p = 0; p < npix; ++p) {
    double v[6];
    for (int c = 0; c < 6; ++c) {
      v[c] = ninv[c * npix + p];
      if (!std::isfinite(v[c])) return fail(WF_EINVAL, "ninv must be finite");
    }
    const bool ot = !mask || (mask[p] & 1), op = !mask || (mask[p] & 2);
    if (!ot) v[0] = v[3] = v[4] = 0.0;           // T row and column
    if (!op) v[1] = v[2] = v[3] = v[4] = v[5] = 0.0;   // Q, U rows and columns
    double lm;
    bool psd;
    eig3(v[0], v[1], v[2], v[3], v[4], v[5], &lm, &psd);
    if (!psd || v[0] < 0 || v[1] < 0 || v[2] < 0) return fail(WF_EINVAL, "every N^-1_p must be positive semi-definite");
    nmax = std::max(nmax, lm);
    nobs_t += v[0] > 0;
    nobs_p += (v[1] > 0 || v[2] > 0);
    for (int c = 0; c < 6; ++c) m6[c * npix + p] = v[c];
  }
  if (!(nmax > 0)) return fail(WF_EINVAL, "no observed pixel (N^-1 zero everywhere after masking)");

  std::shared_ptr<Geometry> geo;
  if (int rc = get_geometry(nside, lmax, &geo)) return rc;
  auto* p = new wf_pol_plan_s();
  auto bail = [&](int code) {
    wf_pol_destroy(p);
    return code;
  };
  const Geometry& g = *geo;
  p->geo = geo;
  p->max_batch = (opts && opts->max_batch > 0) ? opts->max_batch : 1;
  p->flags = opts ? opts->flags : 0;
  p->tau = 1.0 / nmax;
  p->n_obs_t = nobs_t;
  p->n_obs_p = nobs_p;
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->last_stream = p->stream;
  int rc;
  for (double& v : m6) v *= p->tau;
  if ((rc = p->mem.upload(&p->q6, m6))) return bail(rc);
  std::vector<double> c4(cl, cl + 4 * L1);
  if ((rc = p->mem.upload(&p->cl4, c4))) return bail(rc);

  // spin-2 tables and work items: (m, block of 256 ring pairs) over the active pairs of m
  std::vector<int64_t> row_off(lmax + 1);
  MWF_HIP(hipMemcpy(row_off.data(), g.row_off, row_off.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  std::vector<double> A2, B2, K2, n2;
  spin2_tables(lmax, row_off, g.rows_total, A2, B2, K2, n2);
  double *dA = nullptr, *dB = nullptr, *dK = nullptr, *dn = nullptr;
  if ((rc = p->mem.upload(&dA, A2)) || (rc = p->mem.upload(&dB, B2)) || (rc = p->mem.upload(&dK, K2)) ||
      (rc = p->mem.upload(&dn, n2)))
    return bail(rc);
  std::vector<WorkItem> items;
  std::vector<int32_t> nb2(lmax + 1, 0);
  for (int m = 0; m <= lmax; ++m) {
    nb2[m] = (g.n_active[m] + 255) / 256;
    for (int b = 0; b < nb2[m]; ++b) items.push_back(WorkItem{m, b});
  }
  p->nblk2 = std::max(1, (g.npairs + 255) / 256);
  WorkItem* ditems = nullptr;
  if ((rc = p->mem.upload(&ditems, items.empty() ? std::vector<WorkItem>{WorkItem{0, 0}} : items)) ||
      (rc = p->mem.upload(&p->nblk2_m, nb2)))
    return bail(rc);
  p->s2.A = dA;
  p->s2.B = dB;
  p->s2.K = dK;
  p->s2.norm = dn;
  p->s2.items = ditems;
  p->s2.nitems = (int32_t)items.size();
  p->s2.field_maps = p->max_batch;

  // work buffers: G, F [3][max_batch][pair][m][4]; partial sums; synthesis coefficients
  const size_t gf = (size_t)3 * p->max_batch * g.npairs * gf_stride(lmax);
  if ((rc = p->mem.alloc(&p->G, gf)) || (rc = p->mem.alloc(&p->F, gf)) ||
      (rc = p->mem.alloc(&p->partial_t, (size_t)p->max_batch * g.nblk_max_ana * g.nalm)) ||
      (rc = p->mem.alloc(&p->partial_eb, (size_t)p->max_batch * p->nblk2 * g.nalm * 4)) ||
      (rc = p->mem.alloc(&p->bcoef_t, (size_t)p->max_batch * g.rows_total)) ||
      (rc = p->mem.alloc(&p->bcoef_eb, (size_t)p->max_batch * g.rows_total * 2)))
    return bail(rc);
  // F entries of skipped (m, ring pair) combinations are never written: keep them zero
  MWF_HIP(hipMemset(p->F, 0, gf * sizeof(double)));
  MWF_HIP(hipMemset(p->G, 0, gf * sizeof(double)));

  PlanDev& D = p->dev;
  D.nside = nside;
  D.lmax = lmax;
  D.npairs = g.npairs;
  D.nrings = g.nrings;
  D.npix = g.npix;
  D.nalm = g.nalm;
  D.tau = p->tau;
  D.omega = g.omega;
  D.ring_block_ana = g.ring_block_ana;
  D.ring_block_syn = g.ring_block_syn;
  D.nblk_max = g.nblk_max_ana;
  D.pairs = g.pairs;
  D.q = p->q6;
  D.cl = p->cl4;
  D.A = g.A;
  D.C = g.C;
  D.row_off = g.row_off;
  D.row_m = g.row_m;
  D.norm_m = g.norm;
  D.n_active = g.nact;
  D.nblk = g.nblk_ana;
  D.twiddle = g.tw;
  D.tw_len = g.tw_len;
  D.bluestein = g.blue;
  D.chirp = g.chirp;
  D.twiddle32 = g.tw32;
  D.chirp32 = g.chirp32;
  D.bluestein32 = g.blue32;
  D.mixtw = g.mixtw;
  D.mixtw32 = g.mixtw32;
  D.rows_total = g.rows_total;
  *out = p;
  return WF_OK;
}

int wf_pol_plan_info(wf_pol_plan_t p, int64_t* npix, int64_t* nalm, double* tau, int64_t* units_active) {
  if (!p) return fail(WF_EINVAL, "plan must not be NULL");
  if (npix) *npix = p->geo->npix;
  if (nalm) *nalm = p->geo->nalm;
  if (tau) *tau = p->tau;
  if (units_active) *units_active = p->geo->units_active;
  return WF_OK;
}

int wf_pol_solve_batch(wf_pol_plan_t p, int32_t nmaps, const void* d, void* s_wf, void* s_alm, const double* lambda,
                       int32_t nsweeps, void* hip_stream, wf_stats* stats) {
  int rc = check_pol_batch(p, nmaps);
  if (rc) return rc;
  if (!d || !s_wf) return fail(WF_EINVAL, "d and s_wf must not be NULL");
  if (!lambda || nsweeps < 1) return fail(WF_EINVAL, "need a schedule of at least one lambda");
  for (int k = 0; k < nsweeps; ++k)
    if (!std::isfinite(lambda[k]) || !(lambda[k] > 0)) return fail(WF_EINVAL, "every lambda must be finite and > 0");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  PolTimer tm;
  tm.on = (p->flags & WF_FLAG_TIMING) != 0;
  tm.s = s;
  const double* dd = static_cast<const double*>(d);
  for (int k = 0; k < nsweeps; ++k) {
    const int mode = (k == 0 ? 0 : PB_SYNTH) | PB_UPDATE | PB_ANALYSIS;
    if ((rc = pol_ring(p, s, mode, nmaps, lambda[k], dd, nullptr, nullptr, tm))) return rc;
    if ((rc = pol_analysis(p, s, nmaps, tm))) return rc;
    if ((rc = pol_synthesis(p, s, SY_FROM_PARTIAL, nmaps, lambda[k], nullptr, k == nsweeps - 1 ? s_alm : nullptr, tm)))
      return rc;
  }
  if ((rc = pol_ring(p, s, PB_SYNTH | PB_WRITE_MAP, nmaps, 1.0, nullptr, nullptr, static_cast<double*>(s_wf), tm)))
    return rc;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->sweeps_done = nsweeps;
    if ((rc = tm.collect(stats))) return rc;
  }
  return WF_OK;
}

int sht_pol_map2alm(wf_pol_plan_t p, int32_t nmaps, const void* map, void* alm, void* hip_stream) {
  int rc = check_pol_batch(p, nmaps);
  if (rc) return rc;
  if (!map || !alm) return fail(WF_EINVAL, "map and alm must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  PolTimer tm;
  if ((rc = pol_ring(p, s, PB_READ_MAP | PB_ANALYSIS, nmaps, 1.0, nullptr, static_cast<const double*>(map), nullptr, tm)))
    return rc;
  if ((rc = pol_analysis(p, s, nmaps, tm))) return rc;
  return pol_synthesis(p, s, SY_ALM_ONLY, nmaps, 1.0, nullptr, alm, tm);
}

int sht_pol_alm2map(wf_pol_plan_t p, int32_t nmaps, const void* alm, void* map, void* hip_stream) {
  int rc = check_pol_batch(p, nmaps);
  if (rc) return rc;
  if (!map || !alm) return fail(WF_EINVAL, "map and alm must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  PolTimer tm;
  if ((rc = pol_synthesis(p, s, SY_FROM_ALM, nmaps, 1.0, alm, nullptr, tm))) return rc;
  return pol_ring(p, s, PB_SYNTH | PB_WRITE_MAP, nmaps, 1.0, nullptr, nullptr, static_cast<double*>(map), tm);
}

int wf_pol_sync(wf_pol_plan_t p) {
  if (!p) return fail(WF_EINVAL, "plan must not be NULL");
  MWF_HIP(hipStreamSynchronize(p->stream));
  if (p->last_stream != p->stream) MWF_HIP(hipStreamSynchronize(p->last_stream));
  MWF_HIP(hipGetLastError());
  return WF_OK;
}

void wf_pol_destroy(wf_pol_plan_t p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  if (p->last_stream != p->stream) (void)hipStreamSynchronize(p->last_stream);
  delete p;
}

}  // extern "C"
