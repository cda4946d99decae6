// wf_solve_batch_static: the messenger solve of wf_solve_batch with its work
// buffers (ring coefficients G and F, Legendre partial sums and filtered
// coefficients) in one per-device static workspace instead of the plan's, so that
// the call allocates nothing: no device memory, streams or events. It serves
// callers that cannot allocate (code under stream capture, tight serving loops).
//
// The workspace is the file-scope device array `scratch` below. Its device
// address is resolved once per device with hipGetSymbolAddress (with that device
// current) and kept in g_ws; only that address is ever handed to kernels or
// copies (the array's name in host code is a host-side stand-in, not a device
// address). Every call on a device shares the workspace, which keeps the last
// call's contents: the part of F that the synthesis never writes (polar-skipped
// (m, ring pair) entries) is cleared by a fill kernel at the start of each call;
// every other part is written before it is read. Calls that overlap on one device
// race on the workspace.
#include <cmath>
#include <cstring>
#include <mutex>

#include "runtime.hpp"

namespace mwf {
namespace {

constexpr size_t WS_BYTES = size_t(128) << 20;
constexpr int WS_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[WS_BYTES];

std::mutex g_ws_mutex;
void* g_ws[WS_MAX_DEVICES] = {};

// The workspace of the current device (resolved on first use on that device).
int workspace(int device, unsigned char** out) {
  if (device < 0 || device >= WS_MAX_DEVICES) return fail(WF_EUNSUPPORTED, "device index out of range for the static workspace");
  std::lock_guard<std::mutex> lock(g_ws_mutex);
  if (!g_ws[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(WF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ws[device] = ptr;
  }
  *out = static_cast<unsigned char*>(g_ws[device]);
  return WF_OK;
}


constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte layout of the workspace for nmaps maps of this plan: G, F, partial, bcoef.
struct WsLayout {
  size_t g_off, f_off, part_off, coef_off, total, gf_bytes;
};

WsLayout ws_layout(const wf_plan_s* p, int nmaps) {
  const Geometry& g = *p->geo;
  WsLayout L{};
  L.gf_bytes = (size_t)nmaps * g.npairs * gf_stride(g.lmax) * p->elem;
  size_t part, coef;
  if (p->dtype == WF_F64) {
    part = (size_t)nmaps * g.nblk_max_ana * g.nalm * sizeof(double2);
    coef = (size_t)nmaps * g.rows_total * sizeof(double2);
  } else {
    part = (size_t)((g.npairs + 127) / 128) * g.nalm * nmaps * 2 * sizeof(float);
    coef = (size_t)g.rows_total * nmaps * 2 * sizeof(float);
  }
  L.g_off = 0;
  L.f_off = align256(L.g_off + L.gf_bytes);
  L.part_off = align256(L.f_off + L.gf_bytes);
  L.coef_off = align256(L.part_off + part);
  L.total = align256(L.coef_off + coef);
  return L;
}

}  // namespace
}  // namespace mwf

using namespace mwf;

extern "C" int wf_solve_batch_static(wf_plan_t p, int32_t nmaps, const void* d, void* s_wf, void* s_alm,
                                     const double* lambda, int32_t nsweeps, void* hip_stream, wf_stats* stats) {
  if (!p) return fail(WF_EINVAL, "plan must not be NULL");
  if (nmaps < 1 || nmaps > p->max_batch)
    return fail(WF_EINVAL, "nmaps must be in [1, max_batch] (max_batch = " + std::to_string(p->max_batch) + ")");
  if (!d || !s_wf) return fail(WF_EINVAL, "d and s_wf must not be NULL");
  if (!lambda || nsweeps < 1) return fail(WF_EINVAL, "need a schedule of at least one lambda");
  for (int k = 0; k < nsweeps; ++k)
    if (!std::isfinite(lambda[k]) || !(lambda[k] > 0)) return fail(WF_EINVAL, "every lambda must be finite and > 0");
  const Geometry& g = *p->geo;
  const WsLayout L = ws_layout(p, nmaps);
  if (L.total > WS_BYTES)
    return fail(WF_EINVAL, "the solve needs " + std::to_string(L.total >> 20) + " MiB of workspace; the static workspace holds " +
                               std::to_string(WS_BYTES >> 20) + " MiB (fewer maps or a smaller nside / lmax)");
  int dev = -1;
  MWF_HIP(hipGetDevice(&dev));
  if (dev != g.device) return fail(WF_EINVAL, "the plan's device must be current");
  unsigned char* ws = nullptr;
  if (int rc = workspace(dev, &ws)) return rc;

  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  p->last_stream = s;
  p->chi2_nsweeps = 0;   // this call records no chi^2 history
  void* G = ws + L.g_off;
  void* F = ws + L.f_off;
  const PlanDev& P = p->dev;
  const bool fp64 = p->dtype == WF_F64;

  // F entries of polar-skipped (m, ring pair) combinations are read but never written
  MWF_HIP(launch_zero_fill(F, L.gf_bytes, s));

  // ring phase: every class on this one stream (no second stream is made)
  const RingClass* cls = g.ring_cls[nmaps >= RING_SPLIT_MAPS ? 1 : 0];
  auto ring = [&](int mode, double lam, const void* dd, void* out) -> int {
    PhaseBArgs a{};
    a.mode = mode;
    a.nmaps = nmaps;
    a.lambda = lam;
    a.F = F;
    a.G = G;
    a.d = dd;
    a.map_out = out;
    MWF_HIP(launch_phase_b(P, a, cls, !fp64, s));
    return WF_OK;
  };
  MfmaArgs ma{};
  ma.nmaps = nmaps;
  ma.ana_rb = ana_block(p->tune.ana_ct);
  ma.G = static_cast<const float*>(G);
  ma.F = static_cast<float*>(F);
  ma.partial = reinterpret_cast<float*>(ws + L.part_off);
  ma.bcoef = reinterpret_cast<float*>(ws + L.coef_off);
  SynthArgs sa{};
  sa.nmaps = nmaps;
  sa.partial = reinterpret_cast<const double2*>(ws + L.part_off);
  sa.bcoef = reinterpret_cast<double2*>(ws + L.coef_off);
  sa.F = static_cast<double*>(F);

  for (int k = 0; k < nsweeps; ++k) {
    const int mode = (k == 0 ? 0 : PB_SYNTH) | PB_UPDATE | PB_ANALYSIS;
    if (int rc = ring(mode, lambda[k], d, nullptr)) return rc;
    void* alm_out = (k == nsweeps - 1) ? s_alm : nullptr;
    if (fp64) {
      MWF_HIP(launch_legendre_analysis_f64(P, g.items_ana, g.bins_ana, g.nbins_ana, nmaps, static_cast<const double*>(G),
                                           reinterpret_cast<double2*>(ws + L.part_off), s));
      sa.mode = SY_FROM_PARTIAL;
      sa.lambda = lambda[k];
      sa.alm_out = static_cast<double2*>(alm_out);
      MWF_HIP(launch_legendre_coeff(P, sa, s));
      MWF_HIP(launch_legendre_synthesis_f64(P, g.items_syn, g.bins_syn, g.nbins_syn, sa, s));
    } else {
      const int ct = p->tune.ana_ct;
      MWF_HIP(launch_mfma_analysis(P, ct == 1 ? g.items_a128 : g.items_a256, ct == 1 ? g.n_a128 : g.n_a256, p->dtype,
                                   ct, ma, s));
      ma.mode = SY_FROM_PARTIAL;
      ma.lambda = lambda[k];
      ma.alm_out = static_cast<float2*>(alm_out);
      MWF_HIP(launch_mfma_coeff(P, ma, s));
      MWF_HIP(launch_plan_synthesis(g, P, p->dtype, p->tune, ma, s));
    }
  }
  if (int rc = ring(PB_SYNTH | PB_WRITE_MAP, 1.0, nullptr, s_wf)) return rc;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->sweeps_done = nsweeps;
  }
  return WF_OK;
}
