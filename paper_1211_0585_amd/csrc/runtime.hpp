// Host runtime structures of libmwf: cached geometry, plans, task groups.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "mwf_internal.hpp"

namespace mwf {

// Device allocations owned by one object, released with it.
struct DevMem {
  std::vector<void*> ptrs;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() {
    for (void* p : ptrs) hipFree(p);
  }
  // Free one allocation made by alloc (no-op for nullptr). hipFree waits for the
  // device, so work already enqueued on it has finished.
  void release(void* p) {
    if (!p) return;
    for (size_t i = 0; i < ptrs.size(); ++i)
      if (ptrs[i] == p) {
        hipFree(p);
        ptrs.erase(ptrs.begin() + i);
        return;
      }
  }
  template <class T>
  int alloc(T** out, size_t count) {
    void* v = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&v, count * sizeof(T));
    if (e != hipSuccess)
      return fail(e == hipErrorOutOfMemory ? WF_ENOMEM : WF_EDEVICE,
                  std::string("hipMalloc: ") + hipGetErrorString(e));
    ptrs.push_back(v);
    *out = static_cast<T*>(v);
    return WF_OK;
  }
  // Synchronous upload (the host vector may be released right after).
  template <class T>
  int upload(T** out, const std::vector<T>& host) {
    int rc = alloc(out, host.size());
    if (rc) return rc;
    MWF_HIP(hipMemcpy(*out, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
    return WF_OK;
  }
};

// Everything that depends only on (device, nside, lmax): ring geometry, Legendre
// recurrence tables, FFT tables, polar-skip work lists. Shared by every plan of
// that shape through a process-wide cache.
struct Geometry {
  int device = 0, nside = 0, lmax = 0;
  int64_t npix = 0, nalm = 0;
  int npairs = 0, nrings = 0;
  double omega = 0.0;
  int tw_len = 4;
  int64_t rows_total = 0;
  int64_t units_active = 0;
  std::vector<int32_t> n_active;       // per m
  // FP64 VALU path
  int ring_block_ana = 64, ring_block_syn = 64, nblk_max_ana = 1;
  // device tables
  RingPair* pairs = nullptr;
  double* A = nullptr;
  double* C = nullptr;
  int64_t* row_off = nullptr;
  int32_t* row_m = nullptr;
  double* norm = nullptr;
  int32_t* nact = nullptr;
  int32_t* nblk_ana = nullptr;
  double2* tw = nullptr;
  double2* chirp = nullptr;
  double2* blue = nullptr;
  float2* tw32 = nullptr;
  float2* chirp32 = nullptr;
  float2* blue32 = nullptr;
  double2* mixtw = nullptr;            // mixed-radix ring tables exp(-2 pi i t / n)
  float2* mixtw32 = nullptr;
  // work lists, longest first
  WorkItem* items_ana = nullptr;       // FP64 analysis (ring_block_ana), packed into bins
  WorkItem* items_syn = nullptr;       // FP64 synthesis (ring_block_syn), packed into bins
  int32_t* bins_ana = nullptr;         // [nbins + 1] item range of each wave of an FP64 launch
  int32_t* bins_syn = nullptr;
  int nbins_ana = 0, nbins_syn = 0;
  int n_cu = 0;                        // compute units of the device
  WorkItem* items_a128 = nullptr;      // matrix-core analysis, 128 / 256 ring pairs
  WorkItem* items_a256 = nullptr;
  WorkItem* items_s64 = nullptr;       // matrix-core synthesis, 64 ring pairs
  int n_ana = 0, n_syn = 0, n_a128 = 0, n_a256 = 0, n_s64 = 0;
  // ring launch classes: [0] one or few maps (Bluestein, power of two), [1] from
  // RING_SPLIT_MAPS maps on (long Bluestein, long power of two, short)
  RingClass ring_cls[2][NRING_CLASSES]{};
  // few-maps plan launches: the Bluestein rings split by transform length, [0] those
  // of the longest M, [1] the rest (each launch's LDS sized to its own length)
  RingClass blue_split[2]{};
  // the batched class 0 (rings that are not a power of two, longer than SMALL_FFT) split the
  // same way for a plan's own launches: [0] the longest transforms, [1] the others at their
  // own lengths (mixed radix at n, not 2 n)
  RingClass long_split[2]{};
  DevMem mem;
};

int get_geometry(int nside, int lmax, std::shared_ptr<Geometry>* out);

// One HEALPix ring (RING order, 1 <= i <= 4 nside - 1): z = cos(theta), first
// pixel index, pixel count and the longitude of its first pixel, pi ph_num / ph_den.
struct RingGeo {
  double z;
  int64_t start;
  int32_t nphi, ph_num, ph_den;
};
RingGeo ring_geometry(int n, int i);

// Launch-shape choices of the matrix-core kernels (see the autotuner).
struct Tuning {
  int ana_ct = 2;    // column tiles per analysis workgroup (ring block ana_block(ana_ct))
  int syn_nct = 2;   // column tiles per synthesis wave (8 for FP32 only)
  int syn_wide = 0;  // 1 or 2: a plan's own solves use the wide synthesis kernel with that many column
                     // tiles per wave (task groups keep syn_nct)
};

// The matrix-core synthesis of a plan with its tuning: the wide kernel (256 ring pairs,
// 32 syn_wide columns per workgroup) or the per-wave kernel with syn_nct column tiles.
inline hipError_t launch_plan_synthesis(const Geometry& g, const PlanDev& P, int dtype, const Tuning& t,
                                        const MfmaArgs& a, hipStream_t s) {
  if (t.syn_wide) return launch_mfma_wide_synthesis(P, g.items_a256, g.n_a256, dtype, t.syn_wide, a, s);
  return launch_mfma_synthesis(P, g.items_s64, g.n_s64, dtype, t.syn_nct, a, s);
}

bool lookup_tuning(const std::string& key, Tuning* t);
void store_tuning(const std::string& key, const Tuning& t, const char* cache_path);
void load_tuning_file(const char* cache_path);

}  // namespace mwf

struct wf_plan_s;

namespace mwf {

int plan_alloc(wf_plan_s* p);
// Phases of a group step: the ring launch classes, then analysis, coefficients
// and synthesis.
constexpr int NPHASE = NRING_CLASSES + 3;

void task_offsets(const TaskDev* tasks, const std::vector<const Geometry*>& geos, const Tuning& tune,
                  std::vector<int64_t>& offs, int64_t* nblocks, int* fft_len, const std::vector<char>* gemm);
TaskDev make_task(wf_plan_s* p, int nmaps, int pb_mode, int sy_mode, double lam, const void* d,
                  void* map_out, void* alm_out);
// tasks and offs ([NPHASE][ntasks + 1]) in host memory; see GroupLaunch.
int run_group_step(const TaskDev* tasks, const int64_t* offs, const int64_t* nblocks, const int* fft_len,
                   int ntasks, int dtype, const Tuning& tune, bool synth_only, hipStream_t s);
size_t plan_buffer_bytes(int nside, int lmax, int dtype, int nmaps);
size_t geometry_bytes(int nside, int lmax);
// Constrained realisations: out (+)= sqrt(C_l) xi over nmaps packed alm sets; the data
// map d - s_rand - eta sqrt(tau / q); out += s_rand.
hipError_t launch_cr_alm(const double* cl, int lmax, int64_t nalm, int nmaps, const void* xi, void* out,
                         bool accumulate, bool fp64, hipStream_t s);
hipError_t launch_cr_data(const void* d, const void* srand, const void* eta, const void* q, double tau, void* out,
                          int64_t npix, int nmaps, bool fp64, hipStream_t s);
hipError_t launch_cr_add(void* out, const void* srand, int64_t total, bool fp64, hipStream_t s);
// Packed alm of band limit ls into the packed layout of band limit ld >= ls (zero above ls).
hipError_t launch_alm_repack(const void* src, int ls, void* dst, int ld, bool fp64, hipStream_t s);

}  // namespace mwf

struct wf_plan_s {
  std::shared_ptr<mwf::Geometry> geo;
  int dtype = WF_F64, max_batch = 1, flags = 0;
  double tau = 0.0;
  hipStream_t stream = nullptr;        // plan-time uploads
  hipStream_t last_stream = nullptr;   // stream of the last enqueued call
  std::string tune_cache;
  mwf::Tuning tune;
  bool tuned = false;
  void* q = nullptr;                   // tau * ninv in the storage type
  double* cl = nullptr;
  void* G = nullptr;                   // [batch][pair][m][4]
  void* F = nullptr;
  size_t elem = 8;
  double2* partial = nullptr;          // FP64: [batch][blk][nalm]
  double2* bcoef = nullptr;            // FP64: [batch][rows_total]
  float* partial32 = nullptr;          // matrix cores: [blk128][nalm][batch][2]
  float* bcoef32 = nullptr;            // matrix cores: [rows_total][batch][2]
  double* chi2_buf = nullptr;          // chi^2 history: [chi2_maps][CHI_REC chi2_cap], one record per iterate
  int chi2_cap = 0, chi2_maps = 0, chi2_nsweeps = 0, chi2_nmaps = 0;
  size_t chi2_alloc = 0;               // doubles allocated at chi2_buf
  mwf::PlanDev dev{};
  mwf::DevMem mem;
  // second stream for ring classes that run side by side (default priority),
  // with the fork / join events; created on first use
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool owns_aux = true;                // false for band-limited plans (the parent's)
  // host copies kept for the truncated solves
  std::vector<double> cl_host;         // C_l, l = 0..lmax
  int64_t n_obs = 0;                   // observed pixels (ninv > 0, not masked)
  // truncated solves: plans of this problem at lower band limits, by lmax. They
  // share q and cl with this plan (which owns both) and hold their own work buffers.
  std::map<int, wf_plan_s*> band;
  void* alm_scratch = nullptr;         // packed alm of the latest sweep (any band limit)
  // constrained realisations: signal draw (map, alm) and the modified data, max_batch maps
  void* cr_map = nullptr;
  void* cr_alm = nullptr;
  void* cr_d = nullptr;
  // adaptive solve: chi^2 terms copied to pinned host memory on the second stream
  double* chi_host = nullptr;
  int chi_host_cap = 0;
  hipEvent_t ev_ring = nullptr, ev_copied = nullptr;
  ~wf_plan_s() {
    for (auto& kv : band) {
      hipStreamSynchronize(kv.second->last_stream);
      delete kv.second;
    }
    if (aux && owns_aux) {
      hipStreamSynchronize(aux);
      hipStreamDestroy(aux);
      if (ev_fork) hipEventDestroy(ev_fork);
      if (ev_join) hipEventDestroy(ev_join);
    }
    if (ev_ring) hipEventDestroy(ev_ring);
    if (ev_copied) hipEventDestroy(ev_copied);
    if (chi_host) hipHostFree(chi_host);
  }
};

struct wf_group_s {
  std::vector<wf_plan_t> plans;
  std::vector<int32_t> nmaps;
  // launch order of the tasks: descending lmax, then descending map count, so the
  // longest Legendre work items of the group are dispatched first
  std::vector<int> order;
  int dtype = WF_F32;
  mwf::Tuning tune;
  int fft_len[mwf::NRING_CLASSES] = {};  // longest transform of each ring launch class
  int64_t nblocks[mwf::NPHASE] = {};
};
