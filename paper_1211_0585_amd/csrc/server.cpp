// Serving: a request loop over the messenger iteration (Sect. 2) with continuous
// batching. Requests of one (nside, lmax, dtype) share a lane: one plan whose maps
// are request slots, each slot with its own tau N^-1, C_l, lambda schedule and
// sweep position. Every step advances every active slot of every lane by one
// sweep, one kernel launch per phase for all lanes together (task groups), so
// requests that arrive while others run join at the next step boundary and
// requests of equal shape share the FP64 Legendre recurrence inside one GEMM.
//
// Threads: submit() only queues a copy of the request. An admission thread takes
// requests in arrival order, admits one when a slot is free and its lane fits the
// HBM budget (creating lanes, evicting idle ones), computes tau N^-1 and uploads
// the slot's inputs. A stepping thread launches the steps on the server's own
// non-blocking stream, keeps at most two steps in flight and copies finished maps
// back to pinned host memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "runtime.hpp"

using namespace mwf;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int LANE_MAX_SLOTS = 16;
constexpr int STAGE_RING = 4;
constexpr size_t STAGE_BYTES = 1 << 20;

struct Request {
  uint64_t ticket = 0;
  int nside = 0, lmax = 0, dtype = WF_F32;
  std::vector<double> cl, ninv, d, lambda;
  std::vector<uint8_t> mask;
  double t_submit = 0.0;
};

struct Lane;

struct Job {
  Request req;
  Lane* lane = nullptr;
  int slot = -1;
  int k = 0;                 // next step: 0..nsweeps-1 sweeps, nsweeps the final synthesis
  double tau = 0.0;
  hipEvent_t done = nullptr;
};

struct Lane {
  int nside = 0, lmax = 0, dtype = WF_F32, cap = 0;
  size_t bytes = 0;
  wf_plan_s* plan = nullptr;
  float* d_all = nullptr;    // [cap][npix]
  float* s_all = nullptr;    // [cap][npix]
  float* host_out = nullptr; // pinned [cap][npix]
  std::vector<int> busy;     // per slot: 0 free, 1 reserved, 2 in steps, 3 draining
  int in_use = 0;
  ~Lane() {
    delete plan;
    if (host_out) hipHostFree(host_out);
  }
};

struct Result {
  int status = WF_ENOTREADY;
  std::string error;
  std::vector<double> s_wf;
  double latency = 0.0;
};

size_t lane_bytes(int nside, int lmax, int dtype, int cap) {
  const size_t npix = 12ULL * nside * nside;
  return plan_buffer_bytes(nside, lmax, dtype, cap) + (size_t)(cap - 1) * (npix * 4 + (lmax + 1) * 8) +
         2 * (size_t)cap * npix * 4;
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

}  // namespace

struct wf_server_s {
  int device = 0;
  size_t budget = 0;
  int max_slots = 1;
  hipStream_t stream = nullptr;

  std::mutex mu;
  std::condition_variable cv_admit, cv_step;
  bool stop = false;
  int fatal = WF_OK;
  std::string fatal_msg;

  std::deque<Request> pending;
  std::vector<Job*> ready;
  std::list<std::unique_ptr<Lane>> lanes;
  std::set<std::pair<int, int>> geometries;   // shapes with a lane: their tables are charged
  size_t used = 0;
  int slots_in_use = 0;
  uint64_t next_ticket = 1;
  std::map<uint64_t, Result> results;
  wf_server_stats st{};

  // stepping thread only
  std::vector<Job*> active, draining;
  std::deque<hipEvent_t> inflight;
  uint8_t* stage_host[STAGE_RING] = {};
  uint8_t* stage_dev[STAGE_RING] = {};
  hipEvent_t stage_ev[STAGE_RING] = {};
  int64_t step_no = 0;

  std::thread admit_thread, step_thread;

  void set_fatal(int code, const std::string& msg) {
    std::lock_guard<std::mutex> lock(mu);
    if (fatal == WF_OK) {
      fatal = code;
      fatal_msg = msg;
    }
    stop = true;
    cv_admit.notify_all();
    cv_step.notify_all();
  }

  // ------------------------------------------------------------ admission
  Lane* find_lane(const Request& r) {
    for (auto& l : lanes)
      if (l->nside == r.nside && l->lmax == r.lmax && l->dtype == r.dtype) return l.get();
    return nullptr;
  }

  int lane_cap(int nside, int lmax, int dtype) const {
    int cap = std::min(max_slots, LANE_MAX_SLOTS);
    while (cap > 1 && lane_bytes(nside, lmax, dtype, cap) > budget / 2) --cap;
    return cap;
  }

  size_t new_lane_cost(const Request& r) const {
    size_t c = lane_bytes(r.nside, r.lmax, r.dtype, lane_cap(r.nside, r.lmax, r.dtype));
    if (!geometries.count({r.nside, r.lmax})) c += geometry_bytes(r.nside, r.lmax);
    return c;
  }

  // Called with mu held. Frees idle lanes (oldest first) until `need` bytes fit.
  // The stepping thread references a lane only while one of its slots is in use,
  // and the lane's last use ended with a completed event, so freeing is safe.
  bool make_room(size_t need) {
    for (auto it = lanes.begin(); it != lanes.end() && used + need > budget;) {
      if ((*it)->in_use == 0) {
        const std::pair<int, int> shape{(*it)->nside, (*it)->lmax};
        used -= (*it)->bytes;
        it = lanes.erase(it);
        st.lanes_evicted++;
        // the shape's tables go with its last lane
        if (std::none_of(lanes.begin(), lanes.end(), [&](const std::unique_ptr<Lane>& l) {
              return l->nside == shape.first && l->lmax == shape.second;
            })) {
          geometries.erase(shape);
          used -= geometry_bytes(shape.first, shape.second);
        }
      } else {
        ++it;
      }
    }
    return used + need <= budget;
  }

  int create_lane(const Request& r, Lane** out) {
    std::shared_ptr<Geometry> geo;
    if (int rc = get_geometry(r.nside, r.lmax, &geo)) return rc;
    auto lane = std::make_unique<Lane>();
    lane->nside = r.nside;
    lane->lmax = r.lmax;
    lane->dtype = r.dtype;
    lane->cap = lane_cap(r.nside, r.lmax, r.dtype);
    lane->bytes = lane_bytes(r.nside, r.lmax, r.dtype, lane->cap);
    lane->busy.assign(lane->cap, 0);
    auto* p = new wf_plan_s();
    lane->plan = p;
    p->geo = geo;
    p->dtype = r.dtype;
    p->max_batch = lane->cap;
    p->stream = stream;
    p->last_stream = stream;
    Tuning t;
    char key[96];
    std::snprintf(key, sizeof(key), "d%d_n%d_l%d_c%d", r.dtype, r.nside, r.lmax, 2 * lane->cap);
    if (lookup_tuning(key, &t)) p->tune = t;
    const size_t npix = (size_t)geo->npix;
    float* q = nullptr;
    int rc;
    if ((rc = p->mem.alloc(&q, (size_t)lane->cap * npix))) return rc;
    p->q = q;
    if ((rc = p->mem.alloc(&p->cl, (size_t)lane->cap * (r.lmax + 1)))) return rc;
    if ((rc = plan_alloc(p))) return rc;
    if ((rc = p->mem.alloc(&lane->d_all, (size_t)lane->cap * npix))) return rc;
    if ((rc = p->mem.alloc(&lane->s_all, (size_t)lane->cap * npix))) return rc;
    if (hipHostMalloc((void**)&lane->host_out, (size_t)lane->cap * npix * sizeof(float), hipHostMallocDefault) !=
        hipSuccess)
      return fail(WF_ENOMEM, "pinned host buffer for a lane");
    *out = lane.release();
    return WF_OK;
  }

  // Uploads one admitted request into its slot (no stream work of the server is
  // touched: the slot is idle in every step in flight).
  int upload_slot(Job* j) {
    Lane& L = *j->lane;
    const Request& r = j->req;
    const size_t npix = 12ULL * r.nside * r.nside;
    double nmax = 0.0;
    for (size_t i = 0; i < npix; ++i)
      if ((r.mask.empty() || r.mask[i]) && r.ninv[i] > nmax) nmax = r.ninv[i];
    j->tau = 1.0 / nmax;
    std::vector<float> q(npix), d(npix);
    for (size_t i = 0; i < npix; ++i) {
      q[i] = (!r.mask.empty() && !r.mask[i]) ? 0.f : (float)(j->tau * r.ninv[i]);
      d[i] = (float)r.d[i];
    }
    float* qdst = static_cast<float*>(L.plan->q) + (size_t)j->slot * npix;
    MWF_HIP(hipMemcpy(qdst, q.data(), npix * sizeof(float), hipMemcpyHostToDevice));
    MWF_HIP(hipMemcpy(L.d_all + (size_t)j->slot * npix, d.data(), npix * sizeof(float), hipMemcpyHostToDevice));
    MWF_HIP(hipMemcpy(L.plan->cl + (size_t)j->slot * (r.lmax + 1), r.cl.data(), (r.lmax + 1) * sizeof(double),
                      hipMemcpyHostToDevice));
    return WF_OK;
  }

  void admit_loop() {
    if (hipSetDevice(device) != hipSuccess) return set_fatal(WF_EDEVICE, "hipSetDevice in admission thread");
    std::unique_lock<std::mutex> lock(mu);
    while (true) {
      if (stop) return;
      Job* job = nullptr;
      bool create = false, dropped = false;
      if (!pending.empty() && slots_in_use < max_slots) {
        // the oldest request first; a later one is admitted when the oldest waits
        // for a free slot of its lane, never past an oldest request waiting for
        // memory (so lanes drain and become evictable)
        bool oldest_waits_memory = false;
        for (auto it = pending.begin(); it != pending.end(); ++it) {
          if (oldest_waits_memory) break;
          Lane* l = find_lane(*it);
          if (l) {
            const auto f = std::find(l->busy.begin(), l->busy.end(), 0);
            if (f == l->busy.end()) continue;
            job = new Job();
            job->lane = l;
            job->slot = (int)(f - l->busy.begin());
          } else {
            if (!make_room(new_lane_cost(*it))) {
              const bool any_busy =
                  std::any_of(lanes.begin(), lanes.end(), [](const std::unique_ptr<Lane>& l) { return l->in_use > 0; });
              if (!any_busy) {
                // nothing left to evict and still too little room
                Result& res = results[it->ticket];
                res.status = WF_ENOMEM;
                res.error = "request does not fit the HBM budget";
                pending.erase(it);
                dropped = true;
                break;
              }
              if (it == pending.begin()) oldest_waits_memory = true;
              continue;
            }
            job = new Job();
            create = true;
          }
          job->req = std::move(*it);
          pending.erase(it);
          break;
        }
      }
      if (dropped) continue;
      if (!job) {
        cv_admit.wait(lock);
        continue;
      }
      slots_in_use++;
      st.peak_slots = std::max<int64_t>(st.peak_slots, slots_in_use);
      if (create) {
        // charge the lane (and the shape's tables, once) before allocating
        const bool new_geo = !geometries.count({job->req.nside, job->req.lmax});
        const size_t cost = new_lane_cost(job->req);
        used += cost;
        if (new_geo) geometries.insert({job->req.nside, job->req.lmax});
        lock.unlock();
        Lane* l = nullptr;
        const int rc = create_lane(job->req, &l);
        lock.lock();
        if (rc) {
          used -= cost;
          if (new_geo) geometries.erase({job->req.nside, job->req.lmax});
          Result& res = results[job->req.ticket];
          res.status = rc;
          res.error = wf_last_error();
          slots_in_use--;
          delete job;
          continue;
        }
        st.peak_bytes = std::max<int64_t>(st.peak_bytes, (int64_t)used);
        lanes.emplace_back(l);
        st.lanes_created++;
        job->lane = l;
        job->slot = 0;
      }
      job->lane->busy[job->slot] = 1;
      job->lane->in_use++;
      lock.unlock();
      const int rc = upload_slot(job);
      lock.lock();
      if (rc) {
        const std::string msg = wf_last_error();
        lock.unlock();
        return set_fatal(rc, msg);
      }
      ready.push_back(job);
      cv_step.notify_all();
    }
  }

  // ------------------------------------------------------------ stepping
  void finish(Job* j) {
    Lane& L = *j->lane;
    const size_t npix = 12ULL * L.nside * L.nside;
    Result res;
    res.status = WF_OK;
    res.s_wf.resize(npix);
    const float* src = L.host_out + (size_t)j->slot * npix;
    for (size_t i = 0; i < npix; ++i) res.s_wf[i] = src[i];
    res.latency = now_s() - j->req.t_submit;
    hipEventDestroy(j->done);
    std::lock_guard<std::mutex> lock(mu);
    results[j->req.ticket] = std::move(res);
    L.busy[j->slot] = 0;
    L.in_use--;
    slots_in_use--;
    st.completed++;
    st.map_sweeps += (int64_t)j->req.lambda.size();
    delete j;
    cv_admit.notify_all();
  }

  // Enqueues one step for every active job. Returns a status.
  int enqueue_step() {
    // staging block layout: per dtype group [offs][tasks][slot params]
    const int r = (int)(step_no % STAGE_RING);
    MWF_HIP(hipEventSynchronize(stage_ev[r]));
    uint8_t* hb = stage_host[r];
    uint8_t* db = stage_dev[r];
    size_t off = 0;
    auto carve = [&](size_t bytes) {
      const size_t o = off;
      off = (off + bytes + 255) & ~(size_t)255;
      return o;
    };
    struct Launch {
      int dtype;
      size_t tasks_off, offs_off;
      int ntasks;
      int64_t nblocks[NPHASE];
      int fft_len[NRING_CLASSES];
      Tuning tune;
    };
    std::vector<Launch> launches;
    std::vector<Job*> finals;
    for (int dtype : {WF_F32, WF_BF16X6, WF_BF16X3}) {
      std::vector<Lane*> ls;
      for (Job* j : active)
        if (j->lane->dtype == dtype && std::find(ls.begin(), ls.end(), j->lane) == ls.end()) ls.push_back(j->lane);
      if (ls.empty()) continue;
      const int nt = (int)ls.size();
      Launch ln{};
      ln.dtype = dtype;
      ln.ntasks = nt;
      ln.offs_off = carve(NPHASE * (size_t)(nt + 1) * sizeof(int64_t));
      ln.tasks_off = carve((size_t)nt * sizeof(TaskDev));
      std::vector<const Geometry*> geos;
      std::vector<char> gemm;
      for (int t = 0; t < nt; ++t) {
        Lane* L = ls[t];
        int extent = 0;
        bool sweeps = false;
        for (Job* j : active)
          if (j->lane == L) {
            extent = std::max(extent, j->slot + 1);
            if (j->k < (int)j->req.lambda.size()) sweeps = true;
          }
        const size_t sp_off = carve((size_t)extent * sizeof(SlotParam));
        if (off > STAGE_BYTES) return fail(WF_ENOMEM, "server step table exceeds its staging block");
        auto* sp = reinterpret_cast<SlotParam*>(hb + sp_off);
        for (int i = 0; i < extent; ++i) sp[i] = SlotParam{1.0, 0.0, 0, 0};
        for (Job* j : active)
          if (j->lane == L) {
            const int ns = (int)j->req.lambda.size();
            SlotParam& P = sp[j->slot];
            if (j->k < ns) {
              P.lambda = j->req.lambda[j->k];
              P.lam_t_o = P.lambda * j->tau * L->plan->geo->omega;
              P.pb_mode = (j->k == 0 ? 0 : PB_SYNTH) | PB_UPDATE | PB_ANALYSIS;
            } else {
              P.pb_mode = PB_SYNTH | PB_WRITE_MAP;
              finals.push_back(j);
            }
          }
        TaskDev T = make_task(L->plan, extent, 0, SY_FROM_PARTIAL, 1.0, L->d_all, L->s_all, nullptr);
        T.slots = reinterpret_cast<const SlotParam*>(db + sp_off);
        T.q_stride = L->plan->geo->npix;
        T.cl_stride = L->lmax + 1;
        reinterpret_cast<TaskDev*>(hb + ln.tasks_off)[t] = T;
        geos.push_back(L->plan->geo.get());
        gemm.push_back(sweeps ? 1 : 0);
      }
      ln.tune = ls[0]->plan->tune;
      std::vector<int64_t> offs;
      task_offsets(reinterpret_cast<const TaskDev*>(hb + ln.tasks_off), geos, ln.tune, offs, ln.nblocks,
                   ln.fft_len, &gemm);
      std::memcpy(hb + ln.offs_off, offs.data(), offs.size() * sizeof(int64_t));
      launches.push_back(ln);
    }
    if (off > STAGE_BYTES) return fail(WF_ENOMEM, "server step table exceeds its staging block");
    MWF_HIP(hipMemcpyAsync(db, hb, off, hipMemcpyHostToDevice, stream));
    MWF_HIP(hipEventRecord(stage_ev[r], stream));
    for (const Launch& ln : launches) {
      // the task entries travel as kernel arguments (copied at launch); the slot
      // parameters they point to are read from the device copy of the block
      const auto* tasks = reinterpret_cast<const TaskDev*>(hb + ln.tasks_off);
      const auto* offs = reinterpret_cast<const int64_t*>(hb + ln.offs_off);
      if (int rc = run_group_step(tasks, offs, ln.nblocks, ln.fft_len, ln.ntasks, ln.dtype, ln.tune, false, stream))
        return rc;
    }
    for (Job* j : finals) {
      Lane& L = *j->lane;
      const size_t npix = (size_t)L.plan->geo->npix;
      MWF_HIP(hipMemcpyAsync(L.host_out + (size_t)j->slot * npix, L.s_all + (size_t)j->slot * npix,
                             npix * sizeof(float), hipMemcpyDeviceToHost, stream));
      MWF_HIP(hipEventCreateWithFlags(&j->done, hipEventDisableTiming));
      MWF_HIP(hipEventRecord(j->done, stream));
    }
    for (Job* j : active) j->k++;
    for (Job* j : finals) {
      j->lane->busy[j->slot] = 3;
      active.erase(std::find(active.begin(), active.end(), j));
      draining.push_back(j);
    }
    hipEvent_t ev;
    MWF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    MWF_HIP(hipEventRecord(ev, stream));
    inflight.push_back(ev);
    step_no++;
    {
      std::lock_guard<std::mutex> lock(mu);
      st.steps++;
    }
    return WF_OK;
  }

  int reap(bool block) {
    while (!draining.empty()) {
      Job* j = draining.front();
      hipError_t e = block ? hipEventSynchronize(j->done) : hipEventQuery(j->done);
      if (e == hipErrorNotReady) return WF_OK;
      if (e != hipSuccess) return fail(WF_EDEVICE, std::string("server step: ") + hipGetErrorString(e));
      draining.erase(draining.begin());
      finish(j);
      block = false;
    }
    return WF_OK;
  }

  void step_loop() {
    if (hipSetDevice(device) != hipSuccess) return set_fatal(WF_EDEVICE, "hipSetDevice in stepping thread");
    while (true) {
      {
        std::unique_lock<std::mutex> lock(mu);
        if (stop) return;
        for (Job* j : ready) {
          j->lane->busy[j->slot] = 2;
          active.push_back(j);
        }
        ready.clear();
        if (active.empty() && draining.empty()) {
          cv_step.wait(lock);
          continue;
        }
      }
      int rc = reap(false);
      if (!rc && active.empty()) rc = reap(true);
      if (!rc && !active.empty()) {
        while (!rc && inflight.size() >= 2) {
          if (hipEventSynchronize(inflight.front()) != hipSuccess) rc = fail(WF_EDEVICE, "server step failed");
          hipEventDestroy(inflight.front());
          inflight.pop_front();
        }
        if (!rc) rc = enqueue_step();
      }
      if (rc) {
        const std::string msg = wf_last_error();
        return set_fatal(rc, msg);
      }
    }
  }
};

extern "C" {

int wf_server_create(wf_server_t* out, size_t hbm_budget_bytes, int32_t max_slots) {
  if (!out) return fail(WF_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (max_slots < 1) return fail(WF_EINVAL, "max_slots must be >= 1");
  if (hbm_budget_bytes < (16u << 20)) return fail(WF_EINVAL, "hbm_budget_bytes must be at least 16 MiB");
  auto* s = new wf_server_s();
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  auto bail = [&](int rc) {
    wf_server_destroy(s);
    return rc;
  };
  if (hipGetDevice(&s->device) != hipSuccess) return bail(fail(WF_EDEVICE, "hipGetDevice"));
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(WF_EDEVICE, "hipStreamCreateWithFlags"));
  for (int r = 0; r < STAGE_RING; ++r) {
    if (hipHostMalloc((void**)&s->stage_host[r], STAGE_BYTES, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&s->stage_dev[r], STAGE_BYTES) != hipSuccess ||
        hipEventCreateWithFlags(&s->stage_ev[r], hipEventDisableTiming) != hipSuccess)
      return bail(fail(WF_ENOMEM, "server staging buffers"));
    if (hipEventRecord(s->stage_ev[r], s->stream) != hipSuccess) return bail(fail(WF_EDEVICE, "hipEventRecord"));
  }
  s->admit_thread = std::thread([s] { s->admit_loop(); });
  s->step_thread = std::thread([s] { s->step_loop(); });
  *out = s;
  return WF_OK;
}

void wf_server_destroy(wf_server_t s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
  }
  s->cv_admit.notify_all();
  s->cv_step.notify_all();
  if (s->admit_thread.joinable()) s->admit_thread.join();
  if (s->step_thread.joinable()) s->step_thread.join();
  if (s->stream) hipStreamSynchronize(s->stream);
  for (hipEvent_t e : s->inflight) hipEventDestroy(e);
  for (Job* j : s->draining) {
    if (j->done) hipEventDestroy(j->done);
    delete j;
  }
  for (Job* j : s->active) delete j;
  for (Job* j : s->ready) delete j;
  s->lanes.clear();
  for (int r = 0; r < STAGE_RING; ++r) {
    if (s->stage_host[r]) hipHostFree(s->stage_host[r]);
    if (s->stage_dev[r]) hipFree(s->stage_dev[r]);
    if (s->stage_ev[r]) hipEventDestroy(s->stage_ev[r]);
  }
  if (s->stream) hipStreamDestroy(s->stream);
  delete s;
}

int wf_server_submit(wf_server_t s, int32_t nside, int32_t lmax, const double* cl, const double* ninv,
                     const uint8_t* mask, const double* d, const double* lambda, int32_t nsweeps, int32_t dtype,
                     uint64_t* ticket) {
  if (!s || !ticket) return fail(WF_EINVAL, "server and ticket must not be NULL");
  if (nside < 1 || nside > 1024 || !is_pow2(nside)) return fail(WF_EINVAL, "nside must be a power of two in [1, 1024]");
  if (lmax < 0 || lmax > 4 * nside - 1 || lmax > 2048)
    return fail(WF_EINVAL, "lmax must satisfy 0 <= lmax <= min(4 nside - 1, 2048)");
  if (dtype == WF_F64) return fail(WF_EUNSUPPORTED, "serving runs WF_F32, WF_BF16X3 or WF_BF16X6 (use wf_solve for FP64)");
  if (dtype != WF_F32 && dtype != WF_BF16X3 && dtype != WF_BF16X6) return fail(WF_EINVAL, "unknown dtype");
  if (!cl || !ninv || !d || !lambda) return fail(WF_EINVAL, "cl, ninv, d and lambda must not be NULL");
  if (nsweeps < 1) return fail(WF_EINVAL, "nsweeps must be >= 1");
  const size_t npix = 12ULL * nside * nside;
  Request r;
  r.nside = nside;
  r.lmax = lmax;
  r.dtype = dtype;
  r.cl.assign(cl, cl + lmax + 1);
  r.ninv.assign(ninv, ninv + npix);
  r.d.assign(d, d + npix);
  r.lambda.assign(lambda, lambda + nsweeps);
  if (mask) r.mask.assign(mask, mask + npix);
  for (double v : r.cl)
    if (!std::isfinite(v) || v < 0) return fail(WF_EINVAL, "cl must be finite and >= 0");
  for (double v : r.lambda)
    if (!std::isfinite(v) || !(v > 0)) return fail(WF_EINVAL, "every lambda must be finite and > 0");
  bool observed = false;
  for (size_t i = 0; i < npix; ++i) {
    if (!std::isfinite(r.ninv[i]) || r.ninv[i] < 0) return fail(WF_EINVAL, "ninv must be finite and >= 0");
    if (!std::isfinite(r.d[i])) return fail(WF_EINVAL, "d must be finite");
    if ((!mask || mask[i]) && r.ninv[i] > 0) observed = true;
  }
  if (!observed) return fail(WF_EINVAL, "no observed pixel (all ninv == 0 or masked)");
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->fatal) return fail(s->fatal, "server stopped: " + s->fatal_msg);
  {
    const int cap1 = 1;
    size_t need = lane_bytes(nside, lmax, dtype, cap1) + geometry_bytes(nside, lmax);
    if (need > s->budget) return fail(WF_ENOMEM, "request does not fit the server's HBM budget");
  }
  r.ticket = s->next_ticket++;
  r.t_submit = now_s();
  *ticket = r.ticket;
  s->results[r.ticket] = Result{};
  s->pending.push_back(std::move(r));
  s->st.submitted++;
  s->cv_admit.notify_all();
  return WF_OK;
}

int wf_server_poll(wf_server_t s, uint64_t ticket, double* s_wf_host, double* latency_s) {
  if (!s) return fail(WF_EINVAL, "server must not be NULL");
  std::lock_guard<std::mutex> lock(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return fail(WF_EINVAL, "unknown ticket (never issued or already collected)");
  Result& r = it->second;
  if (r.status == WF_ENOTREADY) {
    if (s->fatal) return fail(s->fatal, "server stopped: " + s->fatal_msg);
    return WF_ENOTREADY;
  }
  const int status = r.status;
  if (status == WF_OK) {
    if (s_wf_host) std::memcpy(s_wf_host, r.s_wf.data(), r.s_wf.size() * sizeof(double));
    if (latency_s) *latency_s = r.latency;
  } else {
    set_error(r.error);
  }
  s->results.erase(it);
  return status;
}

int wf_server_query(wf_server_t s, wf_server_stats* out) {
  if (!s || !out) return fail(WF_EINVAL, "server and out must not be NULL");
  std::lock_guard<std::mutex> lock(s->mu);
  *out = s->st;
  out->bytes_in_use = (int64_t)s->used;
  out->slots_in_use = s->slots_in_use;
  out->pending = (int64_t)s->pending.size();
  out->lanes = (int64_t)s->lanes.size();
  if (s->fatal) set_error("server stopped: " + s->fatal_msg);
  return s->fatal;
}

}  // extern "C"
