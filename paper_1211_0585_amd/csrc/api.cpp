// C ABI of libmwf: plans, the messenger sweep driver (Elsner & Wandelt, Sect. 2),
// the SHT entry points, task groups (several plans in one launch per phase) and
// the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace mwf {

namespace {
thread_local std::string g_last_error;
std::mutex g_tune_mu;
std::map<std::string, Tuning> g_tune;
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

bool lookup_tuning(const std::string& key, Tuning* t) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *t = it->second;
  return true;
}

void store_tuning(const std::string& key, const Tuning& t, const char* cache_path) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[key] = t;
  if (cache_path && *cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    if (f) f << key << " " << t.ana_ct << " " << t.syn_nct << " " << t.syn_wide << "\n";
  }
}

// Cache file: one line per shape, "key ana_ct syn_nct [syn_wide]"; later lines win.
void load_tuning_file(const char* cache_path) {
  if (!cache_path || !*cache_path) return;
  std::ifstream f(cache_path);
  std::string line;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  while (std::getline(f, line)) {
    std::istringstream ss(line);
    std::string key;
    Tuning t;
    if (ss >> key >> t.ana_ct >> t.syn_nct && (t.ana_ct == 1 || t.ana_ct == 2 || t.ana_ct == 4 || t.ana_ct == 8) &&
        (t.syn_nct == 1 || t.syn_nct == 2 || t.syn_nct == 4 || t.syn_nct == 8)) {
      int wide = 0;
      if (ss >> wide) t.syn_wide = (wide == 1 || wide == 2) ? wide : 0;
      g_tune[key] = t;
    }
  }
}

}  // namespace mwf

using namespace mwf;

namespace {

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

bool valid_dtype(int d) { return d == WF_F64 || d == WF_F32 || d == WF_BF16X3 || d == WF_BF16X6; }

int validate_shape(int nside, int lmax) {
  if (nside < 1 || nside > 1024 || !is_pow2(nside))
    return fail(WF_EINVAL, "nside must be a power of two in [1, 1024]");
  if (lmax < 0 || lmax > 4 * nside - 1 || lmax > 2048)
    return fail(WF_EINVAL, "lmax must satisfy 0 <= lmax <= min(4 nside - 1, 2048)");
  return WF_OK;
}

std::string tune_key(int dtype, int nside, int lmax, int ncols) {
  char buf[96];
  std::snprintf(buf, sizeof(buf), "d%d_n%d_l%d_c%d", dtype, nside, lmax, ncols);
  return buf;
}

}  // namespace

namespace mwf {

// Device bytes of one plan's own buffers (the tables of its geometry not included).
size_t plan_buffer_bytes(int nside, int lmax, int dtype, int nmaps) {
  const size_t npairs = 2 * (size_t)nside, npix = 12ULL * nside * nside;
  const size_t nalm = (size_t)(lmax + 1) * (lmax + 2) / 2;
  const size_t rows = nalm + (size_t)(lmax + 1) * ROW_PAD;
  const size_t el = dtype == WF_F64 ? 8 : 4;
  size_t b = 2 * (size_t)nmaps * npairs * gf_stride(lmax) * el + npix * el + (lmax + 1) * 8;
  if (dtype == WF_F64) {
    const size_t rb = npairs <= 64 ? 64 : (npairs <= 128 ? 128 : 256);
    b += (size_t)nmaps * ((npairs + rb - 1) / rb) * nalm * 16 + (size_t)nmaps * rows * 16;
  } else {
    b += ((npairs + 127) / 128) * nalm * nmaps * 8 + rows * nmaps * 8;
  }
  return b;
}

// Device bytes of the shared tables of one (nside, lmax) geometry.
size_t geometry_bytes(int nside, int lmax) {
  const size_t nalm = (size_t)(lmax + 1) * (lmax + 2) / 2;
  const size_t rows = nalm + (size_t)(lmax + 1) * ROW_PAD;
  size_t blue = 0;
  for (int i = 1; i < nside; ++i)
    if (!is_pow2(4 * i)) {
      size_t M = 1;
      while (M < (size_t)(8 * i - 1)) M <<= 1;
      blue += M + 4 * i;
    }
  return 2 * rows * 8 + blue * 24 + (size_t)(lmax + 1) * 64 + (size_t)(16 * nside + 64) * 24 +
         5 * nalm + 256 * 1024;
}

}  // namespace mwf

namespace {

// Per-call kernel timing (WF_FLAG_TIMING): an event before and after every launch.
struct Timer {
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;   // 0 ring, 1 analysis, 2 synthesis
  hipStream_t s = nullptr;
  ~Timer() {
    for (auto e : ev) hipEventDestroy(e);
  }
  // The events only time launches: without the system-scope fence an event does not write
  // back and invalidate the caches, which would slow the launch after it and add its own time.
  static int make(hipEvent_t* e) {
    MWF_HIP(hipEventCreateWithFlags(e, hipEventDisableSystemFence));
    return WF_OK;
  }
  int begin() {
    if (!on) return WF_OK;
    hipEvent_t e;
    if (int rc = make(&e)) return rc;
    MWF_HIP(hipEventRecord(e, s));
    ev.push_back(e);
    return WF_OK;
  }
  int end(int k) {
    if (!on) return WF_OK;
    hipEvent_t e;
    if (int rc = make(&e)) return rc;
    MWF_HIP(hipEventRecord(e, s));
    ev.push_back(e);
    kind.push_back(k);
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

thread_local Timer* g_timer = nullptr;

// chi^2 of one iterate from its record: the prior term's slots plus the data term's
// (tau N^-1 weighted, hence the division), each added in slot order.
double chi_of_record(const double* rec, double tau) {
  double prior = 0.0, data = 0.0;
  for (int i = 0; i < CHI_SLOTS; ++i) {
    prior += rec[i * CHI_SLOT_STRIDE];
    data += rec[CHI_TERM + i * CHI_SLOT_STRIDE];
  }
  return prior + data / tau;
}

// chi^2 history buffer ([map][CHI_REC chi2_cap]) laid out for this solve's `maps`
// maps and n iterates (chi2_cap = n), its records cleared on s. The allocation is
// replaced only when it is too small, so it stays at the largest maps x n asked of
// the plan. Kernels find map i at chi2 + i CHI_REC chi2_cap.
int ensure_chi2(wf_plan_s* p, int maps, int n, hipStream_t s) {
  const size_t need = (size_t)maps * CHI_REC * n;
  if (need > p->chi2_alloc) {
    p->mem.release(p->chi2_buf);
    p->chi2_buf = nullptr;
    p->chi2_alloc = 0;
    if (int rc = p->mem.alloc(&p->chi2_buf, need)) return rc;
    p->chi2_alloc = need;
  }
  p->chi2_cap = n;
  p->chi2_maps = maps;
  MWF_HIP(launch_zero_fill(p->chi2_buf, need * sizeof(double), s));
  return WF_OK;
}

// The record of iterate k of map 0, copied to the host (waits for the stream).
int read_chi_record(const wf_plan_s* p, int k, hipStream_t s, double* out) {
  std::vector<double> rec(CHI_REC);
  MWF_HIP(hipMemcpyAsync(rec.data(), p->chi2_buf + (size_t)CHI_REC * k, CHI_REC * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  MWF_HIP(hipStreamSynchronize(s));
  *out = chi_of_record(rec.data(), p->tau);
  return WF_OK;
}

struct TimerScope {
  explicit TimerScope(Timer* t) { g_timer = t->on ? t : nullptr; }
  ~TimerScope() { g_timer = nullptr; }
};

#define TIMED(kind, ...)                                                    \
  do {                                                                      \
    if (g_timer && g_timer->begin()) return WF_EDEVICE;                     \
    { __VA_ARGS__; }                                                        \
    if (g_timer && g_timer->end(kind)) return WF_EDEVICE;                   \
  } while (0)

// ---------------------------------------------------------------- plan-level launches
// The plan's second stream and its fork / join events (default priority), made on
// first use; band-limited plans borrow their parent's.
int ensure_aux(wf_plan_s* p) {
  if (p->aux) return WF_OK;
  MWF_HIP(hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking));
  MWF_HIP(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
  MWF_HIP(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
  return WF_OK;
}

int run_phase_b(wf_plan_s* p, hipStream_t s, int mode, int nmaps, double lam, const void* d,
                const void* map_in, void* map_out, double* chi2 = nullptr) {
  PhaseBArgs a{};
  a.chi2 = chi2;
  a.chi2_stride = (int64_t)CHI_REC * p->chi2_cap;
  a.mode = mode;
  a.nmaps = nmaps;
  a.lambda = lam;
  a.F = p->F;
  a.G = p->G;
  a.d = d;
  a.map_in = map_in;
  a.map_out = map_out;
  const Geometry& g = *p->geo;
  // With few maps, one launch per transform kind fills the GPU better than also
  // splitting off the short transforms; the two kinds then run side by side (the
  // Bluestein class on the plan's second stream), since neither alone fills it
  const int split = nmaps >= RING_SPLIT_MAPS ? 1 : 0;
  const RingClass* cls = g.ring_cls[split];
  const bool fp32 = p->dtype != WF_F64;
  if (split) {
    // the rings of the longest transforms, the other long ones that are not a power of two
    // at their own lengths, the long power-of-two rings, the short ones one wave per pair
    TIMED(0, {
      MWF_HIP(launch_phase_b_class(p->dev, a, g.long_split[0], 0, fp32, s));
      MWF_HIP(launch_phase_b_class(p->dev, a, g.long_split[1], 0, fp32, s));
      MWF_HIP(launch_phase_b_class(p->dev, a, cls[1], 1, fp32, s));
      MWF_HIP(launch_phase_b_class(p->dev, a, cls[2], 2, fp32, s));
    });
    return WF_OK;
  }
  if (cls[0].count == 0 || cls[1].count == 0) {
    TIMED(0, MWF_HIP(launch_phase_b(p->dev, a, cls, fp32, s)));
    return WF_OK;
  }
  if (int rc = ensure_aux(p)) return rc;
  // Bluestein rings of the longest transform on the second stream; on this one the
  // shorter Bluestein rings (their smaller LDS lets them share the chip with the
  // long ones), then the power-of-two rings
  TIMED(0, {
    MWF_HIP(hipEventRecord(p->ev_fork, s));
    MWF_HIP(hipStreamWaitEvent(p->aux, p->ev_fork, 0));
    MWF_HIP(launch_phase_b_class(p->dev, a, g.blue_split[0], 0, fp32, p->aux));
    if (g.blue_split[1].count) MWF_HIP(launch_phase_b_class(p->dev, a, g.blue_split[1], 0, fp32, s));
    MWF_HIP(launch_phase_b_class(p->dev, a, cls[1], 1, fp32, s));
    MWF_HIP(hipEventRecord(p->ev_join, p->aux));
    MWF_HIP(hipStreamWaitEvent(s, p->ev_join, 0));
  });
  return WF_OK;
}

MfmaArgs mfma_args(wf_plan_s* p, int mode, int nmaps, double lam, const void* alm_in, void* alm_out) {
  MfmaArgs a{};
  a.mode = mode;
  a.nmaps = nmaps;
  a.lambda = lam;
  a.ana_rb = ana_block(p->tune.ana_ct);
  a.G = static_cast<const float*>(p->G);
  a.F = static_cast<float*>(p->F);
  a.partial = p->partial32;
  a.bcoef = p->bcoef32;
  a.alm_in = static_cast<const float2*>(alm_in);
  a.alm_out = static_cast<float2*>(alm_out);
  return a;
}

int launch_mfma_ana(wf_plan_s* p, const Tuning& t, int nmaps, hipStream_t s) {
  const Geometry& g = *p->geo;
  MfmaArgs a = mfma_args(p, 0, nmaps, 1.0, nullptr, nullptr);
  a.ana_rb = ana_block(t.ana_ct);
  MWF_HIP(launch_mfma_analysis(p->dev, t.ana_ct == 1 ? g.items_a128 : g.items_a256,
                               t.ana_ct == 1 ? g.n_a128 : g.n_a256, p->dtype, t.ana_ct, a, s));
  return WF_OK;
}

int run_analysis(wf_plan_s* p, hipStream_t s, int nmaps) {
  const Geometry& g = *p->geo;
  if (p->dtype != WF_F64) {
    TIMED(1, if (int rc = launch_mfma_ana(p, p->tune, nmaps, s)) return rc);
  } else {
    TIMED(1, MWF_HIP(launch_legendre_analysis_f64(p->dev, g.items_ana, g.bins_ana, g.nbins_ana, nmaps,
                                                  static_cast<const double*>(p->G), p->partial, s)));
  }
  return WF_OK;
}

int run_synthesis(wf_plan_s* p, hipStream_t s, int mode, int nmaps, double lam, const void* alm_in,
                  void* alm_out, double* chi2 = nullptr) {
  const Geometry& g = *p->geo;
  if (p->dtype != WF_F64) {
    MfmaArgs ma = mfma_args(p, mode, nmaps, lam, alm_in, alm_out);
    ma.chi2 = chi2;
    ma.chi2_stride = (int64_t)CHI_REC * p->chi2_cap;
    TIMED(2, {
      MWF_HIP(launch_mfma_coeff(p->dev, ma, s));
      if (mode != SY_ALM_ONLY)
        MWF_HIP(launch_plan_synthesis(g, p->dev, p->dtype, p->tune, ma, s));
    });
    return WF_OK;
  }
  SynthArgs a{};
  a.mode = mode;
  a.nmaps = nmaps;
  a.lambda = lam;
  a.partial = p->partial;
  a.alm_in = static_cast<const double2*>(alm_in);
  a.alm_out = static_cast<double2*>(alm_out);
  a.F = static_cast<double*>(p->F);
  a.bcoef = p->bcoef;
  a.chi2 = chi2;
  a.chi2_stride = (int64_t)CHI_REC * p->chi2_cap;
  TIMED(2, {
    MWF_HIP(launch_legendre_coeff(p->dev, a, s));
    if (mode != SY_ALM_ONLY) MWF_HIP(launch_legendre_synthesis_f64(p->dev, g.items_syn, g.bins_syn, g.nbins_syn, a, s));
  });
  return WF_OK;
}

int check_batch(wf_plan_s* p, int nmaps) {
  if (!p) return fail(WF_EINVAL, "plan must not be NULL");
  if (nmaps < 1 || nmaps > p->max_batch)
    return fail(WF_EINVAL, "nmaps must be in [1, max_batch] (max_batch = " + std::to_string(p->max_batch) + ")");
  return WF_OK;
}

int check_schedule(const double* lambda, int nsweeps) {
  if (!lambda || nsweeps < 1) return fail(WF_EINVAL, "need a schedule of at least one lambda");
  for (int k = 0; k < nsweeps; ++k)
    if (!std::isfinite(lambda[k]) || !(lambda[k] > 0)) return fail(WF_EINVAL, "every lambda must be finite and > 0");
  return WF_OK;
}

void apply_cached_tuning(wf_plan_s* p, int nmaps) {
  if (p->dtype == WF_F64) return;
  Tuning t;
  if (lookup_tuning(tune_key(p->dtype, p->geo->nside, p->geo->lmax, 2 * nmaps), &t)) p->tune = t;
}

}  // namespace

namespace mwf {

// Work buffers and the device view of a plan whose geo, dtype, max_batch, tau, q
// and cl are set (a solve plan or a serving lane).
int plan_alloc(wf_plan_s* p) {
  int rc;
  const Geometry& g = *p->geo;
  const int dtype = p->dtype, nside = g.nside, lmax = g.lmax;
  // ---- work buffers
  p->elem = (dtype == WF_F64) ? 8 : 4;
  const size_t gf = (size_t)p->max_batch * g.npairs * gf_stride(lmax) * p->elem;
  {
    uint8_t *G = nullptr, *F = nullptr;
    if ((rc = p->mem.alloc(&G, gf))) return rc;
    if ((rc = p->mem.alloc(&F, gf))) return rc;
    p->G = G;
    p->F = F;
  }
  if (dtype == WF_F64) {
    if ((rc = p->mem.alloc(&p->partial, (size_t)p->max_batch * g.nblk_max_ana * g.nalm))) return rc;
    if ((rc = p->mem.alloc(&p->bcoef, (size_t)p->max_batch * g.rows_total))) return rc;
  } else {
    const size_t nb128 = (size_t)(g.npairs + 127) / 128;
    if ((rc = p->mem.alloc(&p->partial32, nb128 * g.nalm * p->max_batch * 2))) return rc;
    if ((rc = p->mem.alloc(&p->bcoef32, (size_t)g.rows_total * p->max_batch * 2))) return rc;
  }
  // F entries of skipped (m, ring pair) combinations are never written: keep them zero
  if (hipMemset(p->F, 0, gf) != hipSuccess || hipMemset(p->G, 0, gf) != hipSuccess) {
    set_error("initialising work buffers failed");
    return WF_EDEVICE;
  }

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
  D.q = p->q;
  D.cl = p->cl;
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
  return WF_OK;
}

}  // namespace mwf

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
  if (!valid_dtype(dtype)) return fail(WF_EINVAL, "unknown dtype");
  if (int rc = validate_shape(nside, lmax)) return rc;
  *bytes = geometry_bytes(nside, lmax) + plan_buffer_bytes(nside, lmax, dtype, nmaps);
  return WF_OK;
}

int wf_pixel_angles(int32_t nside, double* theta, double* phi) {
  if (nside < 1 || nside > 8192 || !is_pow2(nside)) return fail(WF_EINVAL, "nside must be a power of two in [1, 8192]");
  if (!theta || !phi) return fail(WF_EINVAL, "theta and phi must not be NULL");
  const double pi = 3.141592653589793238462643383279502884;
  for (int i = 1; i <= 4 * nside - 1; ++i) {
    const RingGeo g = ring_geometry(nside, i);
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
  delete p;
}

int wf_plan(wf_plan_t* out, int32_t nside, int32_t lmax, const double* cl, const double* ninv,
            const uint8_t* mask, const wf_plan_opts* opts, void* hip_stream) {
  if (!out) return fail(WF_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (int rc = validate_shape(nside, lmax)) return rc;
  if (!cl || !ninv) return fail(WF_EINVAL, "cl and ninv must not be NULL");
  if (opts) {
    if (!valid_dtype(opts->dtype)) return fail(WF_EINVAL, "unknown dtype");
    if (opts->max_batch < 0) return fail(WF_EINVAL, "max_batch must be >= 0");
    if (opts->flags & ~(WF_FLAG_TIMING | WF_FLAG_CHI2)) return fail(WF_EINVAL, "unknown flags");
  }
  const int dtype = opts ? opts->dtype : WF_F64;
  const int64_t npix = 12LL * nside * nside;
  for (int l = 0; l <= lmax; ++l)
    if (!std::isfinite(cl[l]) || cl[l] < 0) return fail(WF_EINVAL, "cl must be finite and >= 0");
  double nmax = 0.0;
  for (int64_t i = 0; i < npix; ++i) {
    if (!std::isfinite(ninv[i]) || ninv[i] < 0) return fail(WF_EINVAL, "ninv must be finite and >= 0");
    if ((!mask || mask[i]) && ninv[i] > nmax) nmax = ninv[i];
  }
  if (!(nmax > 0)) return fail(WF_EINVAL, "no observed pixel (all ninv == 0 or masked)");

  std::shared_ptr<Geometry> geo;
  if (int rc = get_geometry(nside, lmax, &geo)) return rc;
  auto* p = new wf_plan_s();
  auto bail = [&](int code) {
    wf_destroy(p);
    return code;
  };
  p->geo = geo;
  p->dtype = dtype;
  p->max_batch = (opts && opts->max_batch > 0) ? opts->max_batch : 1;
  p->flags = opts ? opts->flags : 0;
  p->tau = 1.0 / nmax;
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->last_stream = p->stream;
  if (opts && opts->tune_cache) {
    p->tune_cache = opts->tune_cache;
    load_tuning_file(opts->tune_cache);
  }
  int rc;
  // ---- per-plan tables: tau * ninv (0 where unobserved), C_l
  std::vector<double> q(npix);
  for (int64_t i = 0; i < npix; ++i) q[i] = (mask && !mask[i]) ? 0.0 : p->tau * ninv[i];
  if (dtype == WF_F64) {
    double* dq = nullptr;
    if ((rc = p->mem.upload(&dq, q))) return bail(rc);
    p->q = dq;
  } else {
    const std::vector<float> q32(q.begin(), q.end());
    float* dq = nullptr;
    if ((rc = p->mem.upload(&dq, q32))) return bail(rc);
    p->q = dq;
  }
  if ((rc = p->mem.upload(&p->cl, std::vector<double>(cl, cl + lmax + 1)))) return bail(rc);
  p->cl_host.assign(cl, cl + lmax + 1);
  for (int64_t i = 0; i < npix; ++i) p->n_obs += q[i] > 0.0;

  if ((rc = plan_alloc(p))) return bail(rc);
  apply_cached_tuning(p, p->max_batch);
  *out = p;
  return WF_OK;
}

int wf_plan_info(wf_plan_t p, int64_t* npix, int64_t* nalm, double* tau, int64_t* units_all,
                 int64_t* units_active) {
  if (!p) return fail(WF_EINVAL, "plan must not be NULL");
  if (npix) *npix = p->geo->npix;
  if (nalm) *nalm = p->geo->nalm;
  if (tau) *tau = p->tau;
  if (units_all) *units_all = (int64_t)p->geo->npairs * p->geo->nalm;
  if (units_active) *units_active = p->geo->units_active;
  return WF_OK;
}

int wf_sync(wf_plan_t p) {
  if (!p) return fail(WF_EINVAL, "plan must not be NULL");
  MWF_HIP(hipStreamSynchronize(p->stream));
  if (p->last_stream != p->stream) MWF_HIP(hipStreamSynchronize(p->last_stream));
  MWF_HIP(hipGetLastError());
  return WF_OK;
}

int wf_solve_batch(wf_plan_t p, int32_t nmaps, const void* d, void* s_wf, void* s_alm,
                   const double* lambda, int32_t nsweeps, void* hip_stream, wf_stats* stats) {
  int rc = check_batch(p, nmaps);
  if (rc) return rc;
  if (!d || !s_wf) return fail(WF_EINVAL, "d and s_wf must not be NULL");
  if ((rc = check_schedule(lambda, nsweeps))) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  Timer timer;
  timer.on = (p->flags & WF_FLAG_TIMING) != 0;
  timer.s = s;
  TimerScope scope(&timer);
  // chi^2 history (WF_FLAG_CHI2): [map][2 k] prior term, [map][2 k + 1] data term of iterate k
  const bool chi = (p->flags & WF_FLAG_CHI2) != 0;
  p->chi2_nsweeps = 0;
  if (chi) {
    if ((rc = ensure_chi2(p, nmaps, nsweeps, s))) return rc;
    p->chi2_nsweeps = nsweeps;
    p->chi2_nmaps = nmaps;
  }
  auto slot = [&](int k, int term) { return chi ? p->chi2_buf + (size_t)CHI_REC * k + term * CHI_TERM : nullptr; };
  for (int k = 0; k < nsweeps; ++k) {
    const int mode = (k == 0 ? 0 : PB_SYNTH) | PB_UPDATE | PB_ANALYSIS;
    if ((rc = run_phase_b(p, s, mode, nmaps, lambda[k], d, nullptr, nullptr, k > 0 ? slot(k - 1, 1) : nullptr)))
      return rc;
    if ((rc = run_analysis(p, s, nmaps))) return rc;
    void* alm_out = (k == nsweeps - 1) ? s_alm : nullptr;
    if ((rc = run_synthesis(p, s, SY_FROM_PARTIAL, nmaps, lambda[k], nullptr, alm_out, slot(k, 0)))) return rc;
  }
  if ((rc = run_phase_b(p, s, PB_SYNTH | PB_WRITE_MAP | (chi ? PB_CHI2 : 0), nmaps, 1.0, chi ? d : nullptr, nullptr,
                        s_wf, slot(nsweeps - 1, 1))))
    return rc;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->sweeps_done = nsweeps;
    if ((rc = timer.collect(stats))) return rc;
    if (chi && (rc = read_chi_record(p, nsweeps - 1, s, &stats->chi2_last))) return rc;
  }
  return WF_OK;
}

int wf_chi2(wf_plan_t p, int32_t nmaps, int32_t nsweeps, double* out) {
  if (!p || !out) return fail(WF_EINVAL, "plan and out must not be NULL");
  if (p->chi2_nsweeps == 0)
    return fail(WF_EINVAL, "the last solve on this plan recorded no chi^2 (WF_FLAG_CHI2 or wf_solve_adaptive)");
  if (nmaps != p->chi2_nmaps || nsweeps != p->chi2_nsweeps)
    return fail(WF_EINVAL, "nmaps and nsweeps must be those of the last solve (" + std::to_string(p->chi2_nmaps) +
                               ", " + std::to_string(p->chi2_nsweeps) + ")");
  std::vector<double> raw((size_t)nmaps * CHI_REC * p->chi2_cap);
  MWF_HIP(hipStreamSynchronize(p->last_stream));
  MWF_HIP(hipMemcpy(raw.data(), p->chi2_buf, raw.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < nmaps; ++i)
    for (int k = 0; k < nsweeps; ++k) {
      const double* r = raw.data() + ((size_t)i * p->chi2_cap + k) * CHI_REC;
      out[(size_t)i * nsweeps + k] = chi_of_record(r, p->tau);
    }
  return WF_OK;
}

int wf_solve(wf_plan_t p, const void* d, void* s_wf, void* s_alm, const double* lambda,
             int32_t nsweeps, void* hip_stream, wf_stats* stats) {
  return wf_solve_batch(p, 1, d, s_wf, s_alm, lambda, nsweeps, hip_stream, stats);
}

int wf_constrained_batch(wf_plan_t p, int32_t nmaps, const void* d, const void* xi, const void* eta, void* s_cr,
                         void* s_alm, const double* lambda, int32_t nsweeps, void* hip_stream, wf_stats* stats) {
  int rc = check_batch(p, nmaps);
  if (rc) return rc;
  if (!d || !xi || !eta || !s_cr) return fail(WF_EINVAL, "d, xi, eta and s_cr must not be NULL");
  if ((rc = check_schedule(lambda, nsweeps))) return rc;
  const Geometry& g = *p->geo;
  if (!p->cr_map) {
    uint8_t *a = nullptr, *b = nullptr, *c = nullptr;
    const size_t maps = (size_t)p->max_batch * g.npix * p->elem;
    if ((rc = p->mem.alloc(&a, maps)) || (rc = p->mem.alloc(&b, maps)) ||
        (rc = p->mem.alloc(&c, (size_t)p->max_batch * g.nalm * 2 * p->elem)))
      return rc;
    p->cr_map = a;
    p->cr_d = b;
    p->cr_alm = c;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  const bool fp64 = p->dtype == WF_F64;
  // the signal draw: alm sqrt(C_l) xi, synthesised to s_rand
  MWF_HIP(launch_cr_alm(p->cl, g.lmax, g.nalm, nmaps, xi, p->cr_alm, false, fp64, s));
  if ((rc = run_synthesis(p, s, SY_FROM_ALM, nmaps, 1.0, p->cr_alm, nullptr))) return rc;
  if ((rc = run_phase_b(p, s, PB_SYNTH | PB_WRITE_MAP, nmaps, 1.0, nullptr, nullptr, p->cr_map))) return rc;
  // the Wiener filter of d - s_rand - n_rand, then s_rand added back
  MWF_HIP(launch_cr_data(d, p->cr_map, eta, p->q, p->tau, p->cr_d, g.npix, nmaps, fp64, s));
  if ((rc = wf_solve_batch(p, nmaps, p->cr_d, s_cr, s_alm, lambda, nsweeps, hip_stream, stats))) return rc;
  MWF_HIP(launch_cr_add(s_cr, p->cr_map, (int64_t)nmaps * g.npix, fp64, s));
  if (s_alm) MWF_HIP(launch_cr_alm(p->cl, g.lmax, g.nalm, nmaps, xi, s_alm, true, fp64, s));
  return WF_OK;
}

int sht_map2alm(wf_plan_t p, int32_t nmaps, const void* map, void* alm, void* hip_stream) {
  int rc = check_batch(p, nmaps);
  if (rc) return rc;
  if (!map || !alm) return fail(WF_EINVAL, "map and alm must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  if ((rc = run_phase_b(p, s, PB_READ_MAP | PB_ANALYSIS, nmaps, 1.0, nullptr, map, nullptr))) return rc;
  if ((rc = run_analysis(p, s, nmaps))) return rc;
  return run_synthesis(p, s, SY_ALM_ONLY, nmaps, 1.0, nullptr, alm);
}

int sht_alm2map(wf_plan_t p, int32_t nmaps, const void* alm, void* map, void* hip_stream) {
  int rc = check_batch(p, nmaps);
  if (rc) return rc;
  if (!map || !alm) return fail(WF_EINVAL, "map and alm must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  if ((rc = run_synthesis(p, s, SY_FROM_ALM, nmaps, 1.0, alm, nullptr))) return rc;
  return run_phase_b(p, s, PB_SYNTH | PB_WRITE_MAP, nmaps, 1.0, nullptr, nullptr, map);
}

}  // extern "C"

// ---------------------------------------------------------------- truncated solves
namespace {

// The plan of this problem at band limit L <= lmax: the plan itself, or one made
// on first use that shares its q and C_l (a prefix of the same table).
int band_plan(wf_plan_s* p, int L, wf_plan_s** out) {
  if (L == p->geo->lmax) {
    *out = p;
    return WF_OK;
  }
  auto it = p->band.find(L);
  if (it != p->band.end()) {
    *out = it->second;
    return WF_OK;
  }
  std::shared_ptr<Geometry> geo;
  if (int rc = get_geometry(p->geo->nside, L, &geo)) return rc;
  auto* b = new wf_plan_s();
  b->geo = geo;
  b->dtype = p->dtype;
  b->max_batch = 1;
  b->tau = p->tau;
  b->stream = p->stream;
  b->last_stream = p->stream;
  b->tune_cache = p->tune_cache;
  b->q = p->q;
  b->cl = p->cl;
  b->n_obs = p->n_obs;
  // one second stream for the whole family of plans: each stream a process holds
  // takes a share of the few hardware queues, also from unrelated work
  if (int rc = ensure_aux(p)) {
    delete b;
    return rc;
  }
  b->aux = p->aux;
  b->ev_fork = p->ev_fork;
  b->ev_join = p->ev_join;
  b->owns_aux = false;
  if (int rc = plan_alloc(b)) {
    delete b;
    return rc;
  }
  apply_cached_tuning(b, 1);
  p->band[L] = b;
  *out = b;
  return WF_OK;
}

// The ring Fourier coefficients of the current iterate ([pair][m][4], m <= lmax of
// `from`) into the buffer of a plan of higher band limit; m above `from`'s limit is
// zero there, as the iterate has no such modes.
int carry_F(const wf_plan_s* from, wf_plan_s* to, hipStream_t s) {
  const size_t w = (size_t)(from->geo->lmax + 1) * 4 * from->elem;   // bytes of a row's values
  const size_t sp = gf_stride(from->geo->lmax) * from->elem;         // row pitches
  const size_t dp = gf_stride(to->geo->lmax) * to->elem;
  const size_t rows = (size_t)from->geo->npairs;
  MWF_HIP(hipMemcpy2DAsync(to->F, dp, from->F, sp, w, rows, hipMemcpyDeviceToDevice, s));
  if (dp > w) MWF_HIP(hipMemset2DAsync(static_cast<uint8_t*>(to->F) + w, dp, 0, dp - w, rows, s));
  return WF_OK;
}

// Sweeps of one map on plans of non-decreasing band limit (Sect. 2 sweep, Sect. 3
// truncation). chi, when set, receives per iterate k the prior term at 2k (from the
// filter of sweep k) and the data term / tau at 2k + 1 (from the ring pass that
// synthesises iterate k: that of sweep k + 1, or finish()).
struct BandRun {
  wf_plan_s* root = nullptr;
  hipStream_t s = nullptr;
  const void* d = nullptr;
  double* chi = nullptr;
  wf_plan_s* cur = nullptr;
  int k = 0;

  // after_ring runs once the ring pass of this sweep is enqueued.
  template <class Hook>
  int sweep(double lam, int L, bool write_alm, Hook after_ring) {
    wf_plan_s* b = nullptr;
    int rc = band_plan(root, L, &b);
    if (rc) return rc;
    if (k > 0 && b != cur && (rc = carry_F(cur, b, s))) return rc;
    b->last_stream = s;
    const int mode = (k == 0 ? 0 : PB_SYNTH) | PB_UPDATE | PB_ANALYSIS;
    if ((rc = run_phase_b(b, s, mode, 1, lam, d, nullptr, nullptr, (k > 0 && chi) ? chi + (size_t)CHI_REC * (k - 1) + CHI_TERM : nullptr)))
      return rc;
    if ((rc = after_ring())) return rc;
    if ((rc = run_analysis(b, s, 1))) return rc;
    if ((rc = run_synthesis(b, s, SY_FROM_PARTIAL, 1, lam, nullptr, write_alm ? root->alm_scratch : nullptr,
                            chi ? chi + (size_t)CHI_REC * k : nullptr)))
      return rc;
    cur = b;
    ++k;
    return WF_OK;
  }

  // The map of the last iterate (and its data term), its alm in the full layout.
  int finish(void* s_wf, void* s_alm) {
    int rc = run_phase_b(cur, s, PB_SYNTH | PB_WRITE_MAP | (chi ? PB_CHI2 : 0), 1, 1.0, chi ? d : nullptr, nullptr,
                         s_wf, chi ? chi + (size_t)CHI_REC * (k - 1) + CHI_TERM : nullptr);
    if (rc) return rc;
    if (s_alm)
      MWF_HIP(launch_alm_repack(root->alm_scratch, cur->geo->lmax, s_alm, root->geo->lmax, root->dtype == WF_F64, s));
    return WF_OK;
  }
};

int ensure_alm_scratch(wf_plan_s* p) {
  if (p->alm_scratch) return WF_OK;
  uint8_t* a = nullptr;
  if (int rc = p->mem.alloc(&a, (size_t)p->geo->nalm * 2 * p->elem)) return rc;
  p->alm_scratch = a;
  return WF_OK;
}


int check_adaptive_opts(const wf_adaptive_opts& o) {
  if (o.l_iter0 < 1) return fail(WF_EINVAL, "l_iter0 must be >= 1");
  if (o.l_pad < 0) return fail(WF_EINVAL, "l_pad must be >= 0");
  if (o.full_band != 0 && o.full_band != 1) return fail(WF_EINVAL, "full_band must be 0 or 1");
  if (o.max_level_sweeps < 0) return fail(WF_EINVAL, "max_level_sweeps must be >= 0");
  if (!(o.plateau_tol >= 0) || !std::isfinite(o.plateau_tol)) return fail(WF_EINVAL, "plateau_tol must be finite and >= 0");
  if (!(o.stop_tol >= 0) || !std::isfinite(o.stop_tol)) return fail(WF_EINVAL, "stop_tol must be finite and >= 0");
  return WF_OK;
}

struct Level {
  double lam;
  int L;
};

// Levels of the adaptive schedule (declared with wf_adaptive_levels); the last one
// has lambda 1 and band limit lmax.
int adaptive_levels(int lmax, const double* cl, double tau, double omega, const wf_adaptive_opts& o,
                    std::vector<Level>* out) {
  out->clear();
  for (int64_t l = o.l_iter0;; l *= 2) {
    const double ratio = l <= lmax ? cl[l] / (tau * omega) : 0.0;
    if (!(ratio > 1.0)) {
      out->push_back({1.0, lmax});
      return WF_OK;
    }
    const int L = o.full_band ? lmax : (int)std::min<int64_t>(lmax, l + o.l_pad);
    out->push_back({ratio, L});
  }
}

}  // namespace

extern "C" {

void wf_adaptive_defaults(wf_adaptive_opts* o) {
  if (!o) return;
  o->l_iter0 = 20;
  o->l_pad = 100;
  o->full_band = 0;
  o->max_level_sweeps = 50;
  o->plateau_tol = 1.0;
  o->stop_tol = 1e-4;
}

int wf_adaptive_levels(int32_t lmax, const double* cl, double tau, double omega, const wf_adaptive_opts* opts,
                       int32_t max_levels, double* lambda_out, int32_t* lmax_out, int32_t* nlevels) {
  if (lmax < 0 || !cl || !opts || !lambda_out || !lmax_out || !nlevels)
    return fail(WF_EINVAL, "lmax must be >= 0 and the pointers non-NULL");
  if (!(tau > 0) || !(omega > 0) || !std::isfinite(tau) || !std::isfinite(omega))
    return fail(WF_EINVAL, "tau and omega must be finite and > 0");
  if (int rc = check_adaptive_opts(*opts)) return rc;
  for (int l = 0; l <= lmax; ++l)
    if (!std::isfinite(cl[l]) || cl[l] < 0) return fail(WF_EINVAL, "cl must be finite and >= 0");
  std::vector<Level> lv;
  adaptive_levels(lmax, cl, tau, omega, *opts, &lv);
  if ((int)lv.size() > max_levels) return fail(WF_EINVAL, "more levels than max_levels");
  for (size_t j = 0; j < lv.size(); ++j) {
    lambda_out[j] = lv[j].lam;
    lmax_out[j] = lv[j].L;
  }
  *nlevels = (int32_t)lv.size();
  return WF_OK;
}

int wf_solve_banded(wf_plan_t p, const void* d, void* s_wf, void* s_alm, const double* lambda,
                    const int32_t* lmax_sht, int32_t nsweeps, void* hip_stream, wf_stats* stats) {
  int rc = check_batch(p, 1);
  if (rc) return rc;
  if (!d || !s_wf) return fail(WF_EINVAL, "d and s_wf must not be NULL");
  if ((rc = check_schedule(lambda, nsweeps))) return rc;
  if (!lmax_sht) return fail(WF_EINVAL, "lmax_sht must not be NULL");
  for (int k = 0; k < nsweeps; ++k) {
    if (lmax_sht[k] < 0 || lmax_sht[k] > p->geo->lmax) return fail(WF_EINVAL, "every lmax_sht must be in [0, lmax]");
    if (k > 0 && lmax_sht[k] < lmax_sht[k - 1]) return fail(WF_EINVAL, "lmax_sht must be non-decreasing");
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  // every plan the schedule needs exists before the first launch
  for (int k = 0; k < nsweeps; ++k) {
    wf_plan_s* b = nullptr;
    if ((rc = band_plan(p, lmax_sht[k], &b))) return rc;
  }
  if (s_alm && (rc = ensure_alm_scratch(p))) return rc;
  Timer timer;
  timer.on = (p->flags & WF_FLAG_TIMING) != 0;
  timer.s = s;
  TimerScope scope(&timer);
  const bool chi = (p->flags & WF_FLAG_CHI2) != 0;
  p->chi2_nsweeps = 0;
  if (chi) {
    if ((rc = ensure_chi2(p, 1, nsweeps, s))) return rc;
    p->chi2_nsweeps = nsweeps;
    p->chi2_nmaps = 1;
  }
  BandRun run;
  run.root = p;
  run.s = s;
  run.d = d;
  run.chi = chi ? p->chi2_buf : nullptr;
  auto none = [] { return WF_OK; };
  for (int k = 0; k < nsweeps; ++k)
    if ((rc = run.sweep(lambda[k], lmax_sht[k], s_alm && k == nsweeps - 1, none))) return rc;
  if ((rc = run.finish(s_wf, s_alm))) return rc;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->sweeps_done = nsweeps;
    if ((rc = timer.collect(stats))) return rc;
    if (chi && (rc = read_chi_record(p, nsweeps - 1, s, &stats->chi2_last))) return rc;
  }
  return WF_OK;
}

int wf_solve_adaptive(wf_plan_t p, const void* d, void* s_wf, void* s_alm, const wf_adaptive_opts* opts,
                      int32_t max_sweeps, double* lambda_out, int32_t* lmax_out, double* chi2_out,
                      int32_t* nsweeps_out, int32_t* converged, void* hip_stream, wf_stats* stats) {
  int rc = check_batch(p, 1);
  if (rc) return rc;
  if (!d || !s_wf) return fail(WF_EINVAL, "d and s_wf must not be NULL");
  if (max_sweeps < 1) return fail(WF_EINVAL, "max_sweeps must be >= 1");
  if (!lambda_out || !lmax_out || !chi2_out || !nsweeps_out)
    return fail(WF_EINVAL, "lambda_out, lmax_out, chi2_out and nsweeps_out must not be NULL");
  wf_adaptive_opts o;
  wf_adaptive_defaults(&o);
  if (opts) o = *opts;
  if ((rc = check_adaptive_opts(o))) return rc;
  std::vector<Level> lv;
  adaptive_levels(p->geo->lmax, p->cl_host.data(), p->tau, p->geo->omega, o, &lv);
  const double sigma = std::sqrt(2.0 * (double)p->n_obs);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  for (const Level& l : lv) {
    wf_plan_s* b = nullptr;
    if ((rc = band_plan(p, l.L, &b))) return rc;
  }
  if ((rc = ensure_alm_scratch(p))) return rc;
  if ((rc = ensure_aux(p))) return rc;
  if (!p->ev_ring) {
    MWF_HIP(hipEventCreateWithFlags(&p->ev_ring, hipEventDisableTiming));
    MWF_HIP(hipEventCreateWithFlags(&p->ev_copied, hipEventDisableTiming));
  }
  if (p->chi_host_cap < max_sweeps) {
    if (p->chi_host) MWF_HIP(hipHostFree(p->chi_host));
    p->chi_host = nullptr;
    p->chi_host_cap = 0;
    MWF_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->chi_host), (size_t)CHI_REC * max_sweeps * sizeof(double)));
    p->chi_host_cap = max_sweeps;
  }
  if ((rc = ensure_chi2(p, 1, max_sweeps, s))) return rc;
  Timer timer;
  timer.on = (p->flags & WF_FLAG_TIMING) != 0;
  timer.s = s;
  TimerScope scope(&timer);

  BandRun run;
  run.root = p;
  run.s = s;
  run.d = d;
  run.chi = p->chi2_buf;
  // once the ring pass of sweep k + 1 is enqueued, the two terms of iterate k are
  // copied out on the plan's second stream, behind that pass only
  auto copy_terms = [&]() -> int {
    const int it = run.k - 1;
    if (it < 0) return WF_OK;
    MWF_HIP(hipEventRecord(p->ev_ring, s));
    MWF_HIP(hipStreamWaitEvent(p->aux, p->ev_ring, 0));
    MWF_HIP(hipMemcpyAsync(p->chi_host + (size_t)CHI_REC * it, p->chi2_buf + (size_t)CHI_REC * it,
                           CHI_REC * sizeof(double), hipMemcpyDeviceToHost, p->aux));
    MWF_HIP(hipEventRecord(p->ev_copied, p->aux));
    return WF_OK;
  };
  std::vector<int> lev;
  std::vector<double> chi;
  auto start = [&](int j) -> int {
    lambda_out[run.k] = lv[j].lam;
    lmax_out[run.k] = lv[j].L;
    lev.push_back(j);
    return run.sweep(lv[j].lam, lv[j].L, true, copy_terms);
  };
  int cur = 0, at_cur = 0;
  bool conv = false;
  if ((rc = start(0))) return rc;
  ++at_cur;
  if (max_sweeps > 1) {
    if ((rc = start(0))) return rc;
    ++at_cur;
  }
  for (int k = 0; k + 1 < run.k; ++k) {
    // iterate k: its terms were copied behind the ring pass of sweep k + 1, the
    // latest one started
    MWF_HIP(hipEventSynchronize(p->ev_copied));
    chi.push_back(chi_of_record(p->chi_host + (size_t)CHI_REC * k, p->tau));
    const bool last = cur + 1 == (int)lv.size();
    int next = cur;
    if (k >= 1 && lev[k] == cur && lev[k - 1] == cur) {
      const double dchi = chi[k - 1] - chi[k];
      if (last) {
        if (dchi < o.stop_tol * sigma) conv = true;
      } else if (std::fabs(dchi) < o.plateau_tol * sigma) {
        next = cur + 1;
      }
    }
    if (!last && o.max_level_sweeps > 0 && at_cur >= o.max_level_sweeps) next = cur + 1;
    if (conv || run.k >= max_sweeps) break;
    if (next != cur) {
      cur = next;
      at_cur = 0;
    }
    if ((rc = start(cur))) return rc;
    ++at_cur;
  }
  if ((rc = run.finish(s_wf, s_alm))) return rc;
  const int n = run.k;
  double chi_last = 0.0;
  if ((rc = read_chi_record(p, n - 1, s, &chi_last))) return rc;
  chi.resize(n - 1);
  chi.push_back(chi_last);
  for (int k = 0; k < n; ++k) chi2_out[k] = chi[k];
  *nsweeps_out = n;
  if (converged) *converged = conv ? 1 : 0;
  p->chi2_nsweeps = n;
  p->chi2_nmaps = 1;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->sweeps_done = n;
    if ((rc = timer.collect(stats))) return rc;
    stats->chi2_last = chi[n - 1];
  }
  return WF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner
namespace {

// Minimum of `reps` timed runs of fn (after one warm-up run).
template <class Fn>
int time_min(hipStream_t s, int reps, Fn fn, float* best) {
  hipEvent_t a, b;
  MWF_HIP(hipEventCreate(&a));
  MWF_HIP(hipEventCreate(&b));
  int rc = fn();
  *best = 1e30f;
  for (int r = 0; r < reps && !rc; ++r) {
    hipEventRecord(a, s);
    rc = fn();
    hipEventRecord(b, s);
    hipEventSynchronize(b);
    float t = 0.f;
    hipEventElapsedTime(&t, a, b);
    *best = std::min(*best, t);
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return rc;
}

}  // namespace

extern "C" int wf_autotune(wf_plan_t p, int32_t nmaps, void* hip_stream, int32_t* ana_ct, int32_t* syn_nct) {
  int rc = check_batch(p, nmaps);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  if (p->dtype == WF_F64) {
    if (ana_ct) *ana_ct = 0;
    if (syn_nct) *syn_nct = 0;
    return WF_OK;
  }
  const Geometry& g = *p->geo;
  Tuning best = p->tune;
  float tbest = 1e30f;
  for (int ct : {1, 2, 4, 8}) {
    if (!ana_ct_valid(ct, p->dtype == WF_F32)) continue;
    Tuning t = p->tune;
    t.ana_ct = ct;
    float ms;
    if ((rc = time_min(s, 3, [&] { return launch_mfma_ana(p, t, nmaps, s); }, &ms))) return rc;
    if (ms < tbest) {
      tbest = ms;
      best.ana_ct = ct;
    }
  }
  tbest = 1e30f;
  for (int nct : {1, 2, 4, 8}) {
    if (nct == 8 && p->dtype != WF_F32) continue;   // one wave over 128 columns: FP32 only
    MfmaArgs ma = mfma_args(p, SY_FROM_PARTIAL, nmaps, 1.0, nullptr, nullptr);
    float ms;
    if ((rc = time_min(s, 3, [&] {
           hipError_t e = launch_mfma_synthesis(p->dev, g.items_s64, g.n_s64, p->dtype, nct, ma, s);
           return e == hipSuccess ? WF_OK : fail(WF_EDEVICE, hipGetErrorString(e));
         }, &ms)))
      return rc;
    if (ms < tbest) {
      tbest = ms;
      best.syn_nct = nct;
    }
  }
  // the wide kernel (plan solves only; groups keep the per-wave shape chosen above)
  best.syn_wide = 0;
  for (int nt : {1, 2}) {
    MfmaArgs ma = mfma_args(p, SY_FROM_PARTIAL, nmaps, 1.0, nullptr, nullptr);
    float ms;
    if ((rc = time_min(s, 3, [&] {
           hipError_t e = launch_mfma_wide_synthesis(p->dev, g.items_a256, g.n_a256, p->dtype, nt, ma, s);
           return e == hipSuccess ? WF_OK : fail(WF_EDEVICE, hipGetErrorString(e));
         }, &ms)))
      return rc;
    if (ms < tbest) {
      tbest = ms;
      best.syn_wide = nt;
    }
  }
  p->tune = best;
  p->tuned = true;
  store_tuning(tune_key(p->dtype, g.nside, g.lmax, 2 * nmaps), best, p->tune_cache.c_str());
  if (ana_ct) *ana_ct = best.ana_ct;
  if (syn_nct) *syn_nct = best.syn_wide ? 32 * best.syn_wide : best.syn_nct;
  return WF_OK;
}

// ---------------------------------------------------------------- task groups
namespace mwf {

// Block offsets of the five phases of a task list (ring pairs of the two classes of
// larger workgroups, ring pairs of the one-wave class, analysis, coefficients, synthesis)
// under a tuning: offs holds 5 x (ntasks + 1) entries. Tasks whose gemm flag is 0
// get no blocks in the three Legendre phases. lds receives the dynamic LDS bytes
// of the two ring launches.
void task_offsets(const TaskDev* tasks, const std::vector<const Geometry*>& geos, const Tuning& tune,
                  std::vector<int64_t>& offs, int64_t* nblocks, int* fft_len, const std::vector<char>* gemm) {
  const int nt = (int)geos.size();
  offs.assign(NPHASE * (size_t)(nt + 1), 0);
  for (int c = 0; c < NRING_CLASSES; ++c) fft_len[c] = 4;
  for (int ph = 0; ph < NPHASE; ++ph) {
    int64_t acc = 0;
    for (int t = 0; t < nt; ++t) {
      offs[ph * (nt + 1) + t] = acc;
      const Geometry& g = *geos[t];
      const int nm = tasks[t].nmaps;
      if (ph < NRING_CLASSES) {
        acc += (int64_t)tasks[t].ring_n[ph] * nm;
        const int split = nm >= RING_SPLIT_MAPS ? 1 : 0;
        if (tasks[t].ring_n[ph]) fft_len[ph] = std::max(fft_len[ph], g.ring_cls[split][ph].fft_len);
        continue;
      }
      if (gemm && !(*gemm)[t]) continue;   // ring phase only for this task
      switch (ph - NRING_CLASSES) {
        case 0: {
          const int ct = tune.ana_ct;
          acc += (int64_t)(ct == 1 ? g.n_a128 : g.n_a256) * ((2 * nm + 16 * ct - 1) / (16 * ct));
          break;
        }
        case 1: acc += (g.rows_total * nm + COEFF_THREADS - 1) / COEFF_THREADS; break;
        default: acc += (int64_t)g.n_s64 * ((2 * nm + 16 * tune.syn_nct - 1) / (16 * tune.syn_nct));
      }
    }
    offs[ph * (nt + 1) + nt] = acc;
    nblocks[ph] = acc;
  }
}

TaskDev make_task(wf_plan_s* p, int nmaps, int pb_mode, int sy_mode, double lam, const void* d,
                  void* map_out, void* alm_out) {
  TaskDev t{};
  t.P = p->dev;
  t.nmaps = nmaps;
  t.pb_mode = pb_mode;
  t.sy_mode = sy_mode;
  t.lambda = lam;
  t.G = p->G;
  t.F = p->F;
  t.d = d;
  t.map_in = nullptr;
  t.map_out = map_out;
  t.partial = p->partial32;
  t.bcoef = p->bcoef32;
  t.alm_in = nullptr;
  t.alm_out = static_cast<float2*>(alm_out);
  const Geometry& g = *p->geo;
  t.items_a128 = g.items_a128;
  t.items_a256 = g.items_a256;
  t.items_s64 = g.items_s64;
  // the same ring classes as a plan's own launches
  const int split = nmaps >= RING_SPLIT_MAPS ? 1 : 0;
  for (int c = 0; c < NRING_CLASSES; ++c) {
    t.ring_q[c] = g.ring_cls[split][c].q;
    t.ring_n[c] = g.ring_cls[split][c].count;
  }
  return t;
}

// One step of a task array (host memory; the entries travel as kernel arguments):
// the ring launches, then (unless synth_only) analysis, coefficients and synthesis,
// one launch each (per part of at most GROUP_MAX_TASKS tasks).
int run_group_step(const TaskDev* tasks, const int64_t* offs, const int64_t* nblocks, const int* fft_len,
                   int ntasks, int dtype, const Tuning& tune, bool synth_only, hipStream_t s) {
  const int stride = ntasks + 1;
  GroupLaunch g{tasks, offs, ntasks, 0, nblocks[0]};
  TIMED(0, {
    for (int c = 0; c < NRING_CLASSES; ++c) {
      g.offs = offs + c * stride;
      g.nblocks = nblocks[c];
      MWF_HIP(launch_group_phase_b(g, c, fft_len[c], s));
    }
  });
  if (synth_only) return WF_OK;
  const int a0 = NRING_CLASSES;
  g.offs = offs + a0 * stride;
  g.nblocks = nblocks[a0];
  TIMED(1, MWF_HIP(launch_group_analysis(g, dtype, tune.ana_ct, s)));
  TIMED(2, {
    g.offs = offs + (a0 + 1) * stride;
    g.nblocks = nblocks[a0 + 1];
    MWF_HIP(launch_group_coeff(g, ana_block(tune.ana_ct), s));
    g.offs = offs + (a0 + 2) * stride;
    g.nblocks = nblocks[a0 + 2];
    MWF_HIP(launch_group_synthesis(g, dtype, tune.syn_nct, ana_block(tune.ana_ct), s));
  });
  return WF_OK;
}

}  // namespace mwf

extern "C" {

int wf_group_create(wf_group_t* out, int32_t nplans, const wf_plan_t* plans, const int32_t* nmaps) {
  if (!out) return fail(WF_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (nplans < 1 || !plans || !nmaps) return fail(WF_EINVAL, "need at least one plan");
  const int dtype = plans[0] ? plans[0]->dtype : -1;
  if (dtype < 0) return fail(WF_EINVAL, "plan must not be NULL");
  if (dtype == WF_F64) return fail(WF_EUNSUPPORTED, "groups run the matrix-core (float) plans");
  auto* gr = new wf_group_s();
  gr->dtype = dtype;
  for (int i = 0; i < nplans; ++i) {
    wf_plan_t p = plans[i];
    if (!p || p->dtype != dtype) {
      delete gr;
      return fail(WF_EINVAL, "every plan of a group must exist and share the dtype");
    }
    if (nmaps[i] < 1 || nmaps[i] > p->max_batch) {
      delete gr;
      return fail(WF_EINVAL, "nmaps[i] must be in [1, max_batch of plan i]");
    }
    gr->plans.push_back(p);
    gr->nmaps.push_back(nmaps[i]);
  }
  gr->order.resize(nplans);
  for (int i = 0; i < nplans; ++i) gr->order[i] = i;
  std::stable_sort(gr->order.begin(), gr->order.end(), [&](int a, int b) {
    const int la = gr->plans[a]->geo->lmax, lb = gr->plans[b]->geo->lmax;
    return la != lb ? la > lb : gr->nmaps[a] > gr->nmaps[b];
  });
  gr->tune = plans[0]->tune;
  *out = gr;
  return WF_OK;
}

void wf_group_destroy(wf_group_t gr) {
  if (!gr) return;
  hipDeviceSynchronize();
  delete gr;
}

int wf_group_solve(wf_group_t gr, const void* const* d, void* const* s_wf, void* const* s_alm,
                   const double* lambda, int32_t nsweeps, void* hip_stream, wf_stats* stats) {
  if (!gr) return fail(WF_EINVAL, "group must not be NULL");
  if (!d || !s_wf) return fail(WF_EINVAL, "d and s_wf must not be NULL");
  int rc = check_schedule(lambda, nsweeps);
  if (rc) return rc;
  const int nt = (int)gr->plans.size();
  for (int t = 0; t < nt; ++t)
    if (!d[t] || !s_wf[t]) return fail(WF_EINVAL, "d[i] and s_wf[i] must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // one task array per step: sweeps 0..nsweeps-1, then the final synthesis
  std::vector<TaskDev> host((size_t)(nsweeps + 1) * nt);
  for (int k = 0; k <= nsweeps; ++k)
    for (int i = 0; i < nt; ++i) {
      const int t = gr->order[i];
      wf_plan_s* p = gr->plans[t];
      p->last_stream = s;
      TaskDev& T = host[(size_t)k * nt + i];
      if (k < nsweeps) {
        const int mode = (k == 0 ? 0 : PB_SYNTH) | PB_UPDATE | PB_ANALYSIS;
        T = make_task(p, gr->nmaps[t], mode, SY_FROM_PARTIAL, lambda[k], d[t], nullptr,
                      (k == nsweeps - 1 && s_alm) ? s_alm[t] : nullptr);
      } else {
        T = make_task(p, gr->nmaps[t], PB_SYNTH | PB_WRITE_MAP, SY_FROM_PARTIAL, 1.0, nullptr, s_wf[t], nullptr);
      }
    }
  std::vector<const Geometry*> geos;
  for (int i = 0; i < nt; ++i) geos.push_back(gr->plans[gr->order[i]]->geo.get());
  std::vector<int64_t> offs;
  task_offsets(host.data(), geos, gr->tune, offs, gr->nblocks, gr->fft_len, nullptr);
  Timer timer;
  timer.on = (gr->plans[0]->flags & WF_FLAG_TIMING) != 0;
  timer.s = s;
  TimerScope scope(&timer);
  for (int k = 0; k <= nsweeps; ++k)
    if ((rc = run_group_step(host.data() + (size_t)k * nt, offs.data(), gr->nblocks, gr->fft_len, nt, gr->dtype,
                             gr->tune, k == nsweeps, s)))
      return rc;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->sweeps_done = nsweeps;
    if ((rc = timer.collect(stats))) return rc;
  }
  return WF_OK;
}

int wf_group_autotune(wf_group_t gr, const void* const* d, void* const* s_wf, void* hip_stream,
                      int32_t* ana_ct, int32_t* syn_nct) {
  if (!gr) return fail(WF_EINVAL, "group must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const double lam[2] = {10.0, 1.0};
  Tuning best = gr->tune;
  float tbest = 1e30f;
  for (int ct : {1, 2})
    for (int nct : {1, 2, 4, 8}) {
      if (nct == 8 && gr->dtype != WF_F32) continue;
      gr->tune.ana_ct = ct;
      gr->tune.syn_nct = nct;
      float ms;
      const int rc = time_min(
          s, 2, [&] { return wf_group_solve(gr, d, s_wf, nullptr, lam, 2, hip_stream, nullptr); }, &ms);
      if (rc) return rc;
      if (ms < tbest) {
        tbest = ms;
        best = gr->tune;
      }
    }
  gr->tune = best;
  if (ana_ct) *ana_ct = best.ana_ct;
  if (syn_nct) *syn_nct = best.syn_nct;
  return WF_OK;
}

}  // extern "C"
