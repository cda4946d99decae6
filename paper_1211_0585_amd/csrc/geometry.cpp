// Plan-time tables shared by every plan of a given (device, nside, lmax):
// HEALPix ring geometry (Gorski et al. 2005), the rescaled Legendre recurrence
// coefficients, FFT twiddles, mixed-radix and Bluestein tables, and the polar-skip work
// lists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <queue>
#include <tuple>

#include "runtime.hpp"

namespace mwf {

namespace {

constexpr long double PI_L = 3.141592653589793238462643383279502884L;
// Ring pairs whose class length (n; twice n for mixed radix; the Bluestein length M) is at
// most this many points run one wave per pair when batched; longer ones a larger workgroup
// (512 threads for rings that are not a power of two, 256 for power-of-two rings).
constexpr int SMALL_FFT = 1024;

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2_ceil(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

// In-place iterative radix-2 FFT in long double (plan time only).
void host_fft(std::vector<std::complex<long double>>& a, int sign) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    for (size_t k = 0; k < len / 2; ++k) {
      const long double ang = sign * 2.0L * PI_L * (long double)k / (long double)len;
      const std::complex<long double> w(cosl(ang), sinl(ang));
      for (size_t i = k; i < n; i += len) {
        const auto u = a[i], v = a[i + len / 2] * w;
        a[i] = u + v;
        a[i + len / 2] = u - v;
      }
    }
  }
}

int ana_ring_block(int npairs) { return npairs <= 64 ? 64 : (npairs <= 128 ? 128 : 256); }

std::mutex g_geo_mu;
// Weak entries: the tables of a shape live while a plan or serving lane holds them.
std::map<std::tuple<int, int, int>, std::weak_ptr<Geometry>> g_geo;

int build_geometry(Geometry& g) {
  const int nside = g.nside, lmax = g.lmax;
  g.npix = 12LL * nside * nside;
  g.nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
  g.nrings = 4 * nside - 1;
  g.npairs = 2 * nside;
  g.omega = 4.0 * 3.141592653589793238462643383279502884 / (double)g.npix;
  int rc;

  // ---- ring pairs, equator first
  std::vector<RingPair> pairs(g.npairs);
  std::vector<int> blue_len;
  for (int q = 0; q < g.npairs; ++q) {
    const int i = 2 * nside - q;
    const RingGeo gn = ring_geometry(nside, i);
    RingPair rp{};
    rp.z = gn.z;
    rp.sin_t = std::sqrt((1.0 - gn.z) * (1.0 + gn.z));
    rp.start_n = gn.start;
    rp.start_s = (q == 0) ? -1 : ring_geometry(nside, 4 * nside - i).start;
    rp.nphi = gn.nphi;
    rp.ph_num = gn.ph_num;
    rp.ph_den = gn.ph_den;
    if (is_pow2(gn.nphi)) {
      rp.log2n = ilog2_ceil(gn.nphi);
      rp.bl_M = 0;
      g.tw_len = std::max(g.tw_len, gn.nphi);
    } else if ((rp.mix = mixed_radix_passes(gn.nphi)) != 0) {
      // 2^a 3^b 5^c 7^d points: radix-2/4/8 passes (their twiddles from the power-of-two
      // table, as for a 2^a-point transform), then the odd passes
      rp.log2n = -1;
      rp.bl_M = 0;
      g.tw_len = std::max(g.tw_len, gn.nphi & -gn.nphi);
    } else {
      rp.log2n = -1;
      rp.bl_M = 1 << ilog2_ceil(2 * gn.nphi - 1);
      g.tw_len = std::max(g.tw_len, rp.bl_M);
      blue_len.push_back(gn.nphi);
    }
    pairs[q] = rp;
  }

  // ---- Bluestein chirps exp(-i pi j^2 / n) and filter spectra H = FFT_M(h),
  //      h_j = exp(+i pi j^2 / n) for |j| < n
  std::vector<double2> blue, chirp;
  {
    std::vector<int64_t> off_of(4 * nside + 1, -1), coff_of(4 * nside + 1, -1);
    for (int n : blue_len) {
      if (off_of[n] >= 0) continue;
      coff_of[n] = (int64_t)chirp.size();
      for (int j = 0; j < n; ++j) {
        const long double ang = -PI_L * (long double)(((int64_t)j * j) % (2LL * n)) / (long double)n;
        chirp.push_back(make_double2((double)cosl(ang), (double)sinl(ang)));
      }
      const int M = 1 << ilog2_ceil(2 * n - 1);
      std::vector<std::complex<long double>> h(M, 0.0L);
      for (int j = 0; j < n; ++j) {
        const long double ang = PI_L * (long double)(((int64_t)j * j) % (2LL * n)) / (long double)n;
        const std::complex<long double> w(cosl(ang), sinl(ang));
        h[j] = w;
        if (j) h[M - j] = w;
      }
      host_fft(h, -1);
      off_of[n] = (int64_t)blue.size();
      for (int k = 0; k < M; ++k) blue.push_back(make_double2((double)h[k].real(), (double)h[k].imag()));
    }
    for (auto& rp : pairs)
      if (rp.bl_M > 0) {
        rp.bl_off = off_of[rp.nphi];
        rp.chirp_off = coff_of[rp.nphi];
      }
    if (blue.empty()) blue.push_back(make_double2(0.0, 0.0));
    if (chirp.empty()) chirp.push_back(make_double2(0.0, 0.0));
  }
  // ---- mixed-radix rings: exp(-2 pi i t / n), t < n, per distinct length
  std::vector<double2> mixtw;
  {
    std::vector<int64_t> off_of(4 * nside + 1, -1);
    for (auto& rp : pairs) {
      if (!rp.mix) continue;
      const int n = rp.nphi;
      if (off_of[n] < 0) {
        off_of[n] = (int64_t)mixtw.size();
        for (int t = 0; t < n; ++t) {
          const long double ang = -2.0L * PI_L * (long double)t / (long double)n;
          mixtw.push_back(make_double2((double)cosl(ang), (double)sinl(ang)));
        }
      }
      rp.bl_off = off_of[n];
    }
    if (mixtw.empty()) mixtw.push_back(make_double2(0.0, 0.0));
  }
  std::vector<double2> tw(g.tw_len / 2);
  for (int k = 0; k < g.tw_len / 2; ++k) {
    const long double ang = -2.0L * PI_L * (long double)k / (long double)g.tw_len;
    tw[k] = make_double2((double)cosl(ang), (double)sinl(ang));
  }
  auto to32 = [](const std::vector<double2>& v) {
    std::vector<float2> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = make_float2((float)v[i].x, (float)v[i].y);
    return o;
  };

  // ---- recurrence tables mu_l = (A z) mu_{l-1} - mu_{l-2}, lambda = C mu; padded rows
  std::vector<int64_t> row_off(lmax + 1);
  std::vector<int32_t> row_m;             // m of every padded row
  std::vector<double> A, C, norm(lmax + 1);
  {
    int64_t off = 0;
    for (int m = 0; m <= lmax; ++m) {
      row_off[m] = off;
      off += (lmax - m + 1) + ROW_PAD;
    }
    g.rows_total = off;
    row_m.resize(off);
    for (int m = 0; m <= lmax; ++m)
      for (int64_t r = row_off[m]; r < (m < lmax ? row_off[m + 1] : off); ++r) row_m[r] = m;
    A.assign(off, 0.0);
    C.assign(off, 0.0);
    long double nm = 1.0L / sqrtl(4.0L * PI_L);
    for (int m = 0; m <= lmax; ++m) {
      if (m > 0) nm *= -sqrtl((2.0L * m + 1.0L) / (2.0L * m));
      norm[m] = (double)nm;
      auto alpha = [&](int l) {
        return sqrtl((4.0L * l * l - 1.0L) / ((long double)(l - m) * (long double)(l + m)));
      };
      const int64_t r = row_off[m];
      long double c_lm2 = 1.0L, c_lm1 = 1.0L;
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

  DevMem& M = g.mem;
  if ((rc = M.upload(&g.pairs, pairs))) return rc;
  if ((rc = M.upload(&g.A, A))) return rc;
  if ((rc = M.upload(&g.C, C))) return rc;
  if ((rc = M.upload(&g.row_off, row_off))) return rc;
  if ((rc = M.upload(&g.row_m, row_m))) return rc;
  if ((rc = M.upload(&g.norm, norm))) return rc;
  if ((rc = M.upload(&g.tw, tw))) return rc;
  if ((rc = M.upload(&g.chirp, chirp))) return rc;
  if ((rc = M.upload(&g.blue, blue))) return rc;
  if ((rc = M.upload(&g.tw32, to32(tw)))) return rc;
  if ((rc = M.upload(&g.chirp32, to32(chirp)))) return rc;
  if ((rc = M.upload(&g.blue32, to32(blue)))) return rc;
  if ((rc = M.upload(&g.mixtw, mixtw))) return rc;
  if ((rc = M.upload(&g.mixtw32, to32(mixtw)))) return rc;

  // ---- ring launch classes by transform kind and length
  {
    std::vector<int32_t> lists[2][NRING_CLASSES];
    int lens[2][NRING_CLASSES];
    for (auto& row : lens)
      for (int& l : row) l = 4;
    // a ring that is not a power of two (mixed radix or Bluestein) goes with the Bluestein
    // rings, its class length at least twice its own (the kernels of that kind assume it)
    auto class_len = [&](const RingPair& rp) {
      return rp.bl_M > 0 ? rp.bl_M : (rp.mix ? 2 * rp.nphi : rp.nphi);
    };
    for (int q = 0; q < g.npairs; ++q) {
      const bool npot = pairs[q].log2n < 0;
      const int L = class_len(pairs[q]);
      const int c0 = npot ? 0 : 1;                    // few maps: by kind only
      const int c1 = L <= SMALL_FFT ? 2 : c0;          // batched: short ones apart
      lists[0][c0].push_back(q);
      lens[0][c0] = std::max(lens[0][c0], L);
      lists[1][c1].push_back(q);
      lens[1][c1] = std::max(lens[1][c1], L);
    }
    for (int k = 0; k < 2; ++k)
      for (int c = 0; c < NRING_CLASSES; ++c) {
        int32_t* d = nullptr;
        if ((rc = M.upload(&d, lists[k][c]))) return rc;
        g.ring_cls[k][c] = RingClass{d, (int32_t)lists[k][c].size(), lens[k][c]};
      }
    // Bluestein rings of the longest transform apart from the shorter ones: at the
    // longest length alone they can hold all of the chip's LDS. The mixed-radix rings go
    // with the shorter ones at their own length: these two launches run only the plain
    // ring kernel, whose transforms need n <= 4 MAXB NT, not the half-length bound of
    // the class lists (with the longest ones, or at twice their length, they made the
    // one-map ring phase 5 and 16 us slower).
    std::vector<int32_t> bl[2];
    int bl_len[2] = {4, 4};
    for (int q : lists[0][0]) {
      const int k = pairs[q].bl_M == lens[0][0] ? 0 : 1;
      bl[k].push_back(q);
      bl_len[k] = std::max(bl_len[k], pairs[q].mix ? pairs[q].nphi : class_len(pairs[q]));
    }
    for (int k = 0; k < 2; ++k) {
      int32_t* d = nullptr;
      if ((rc = M.upload(&d, bl[k]))) return rc;
      g.blue_split[k] = RingClass{d, (int32_t)bl[k].size(), bl_len[k]};
    }
    // the same split of the batched class 0: at 64 maps the 2048-point Bluestein rings and
    // the long mixed-radix rings ran in the launch sized for the 4096-point ones
    std::vector<int32_t> ls[2];
    int ls_len[2] = {4, 4};
    for (int q : lists[1][0]) {
      const int k = pairs[q].bl_M == lens[1][0] ? 0 : 1;
      ls[k].push_back(q);
      ls_len[k] = std::max(ls_len[k], pairs[q].mix ? pairs[q].nphi : class_len(pairs[q]));
    }
    for (int k = 0; k < 2; ++k) {
      int32_t* d = nullptr;
      if ((rc = M.upload(&d, ls[k]))) return rc;
      g.long_split[k] = RingClass{d, (int32_t)ls[k].size(), ls_len[k]};
    }
  }

  // ---- polar skip: ring pairs whose lambda_lm never leaves the negligible range
  PlanDev D{};
  D.nside = nside;
  D.lmax = lmax;
  D.npairs = g.npairs;
  D.pairs = g.pairs;
  D.A = g.A;
  D.C = g.C;
  D.row_off = g.row_off;
  D.row_m = g.row_m;
  D.norm_m = g.norm;
  std::vector<uint16_t> wake((size_t)(lmax + 1) * g.npairs);
  {
    uint16_t* d_wake = nullptr;
    DevMem tmp;
    if ((rc = tmp.alloc(&d_wake, wake.size()))) return rc;
    MWF_HIP(launch_reach(D, d_wake, nullptr));
    MWF_HIP(hipMemcpy(wake.data(), d_wake, wake.size() * sizeof(uint16_t), hipMemcpyDeviceToHost));
    g.n_active.assign(lmax + 1, 0);
    g.units_active = 0;
    for (int m = 0; m <= lmax; ++m) {
      int na = 0;
      for (int q = 0; q < g.npairs; ++q)
        if (wake[(size_t)m * g.npairs + q] != WAKE_NEVER) na = q + 1;
      g.n_active[m] = na;
      g.units_active += (int64_t)na * (lmax - m + 1);
    }
  }
  // estimated cost of an FP64 work item of rb ring pairs, in steps of l: steps with a
  // still-scaled ring in the block take the rescale path of every chunk
  auto item_cost = [&](const WorkItem& w, int rb, int scaled_cost) {
    const int nl = lmax - w.m + 1;
    int scaled = 0;
    const int q1 = std::min(g.n_active[w.m], (w.blk + 1) * rb);
    for (int q = w.blk * rb; q < q1; ++q) {
      const uint16_t wk = wake[(size_t)w.m * g.npairs + q];
      if (wk != WAKE_NEVER) scaled = std::max(scaled, std::min((int)wk, nl));
    }
    return (int64_t)4 * (nl - scaled) + (int64_t)scaled_cost * scaled + 4 * FP64_ITEM_COST_L;
  };
  auto make_items = [&](int rb) {
    std::vector<WorkItem> items;
    for (int m = 0; m <= lmax; ++m) {
      const int nb = (g.n_active[m] + rb - 1) / rb;
      for (int b = 0; b < nb; ++b) items.push_back({m, b});
    }
    std::stable_sort(items.begin(), items.end(), [&](const WorkItem& a, const WorkItem& b) {
      auto c = [&](const WorkItem& w) {
        const int rings = std::min(rb, g.n_active[w.m] - w.blk * rb);
        return (double)(lmax - w.m + 1) * (double)std::max(rings, 1);
      };
      return c(a) > c(b);
    });
    if (items.empty()) items.push_back({0, 0});
    return items;
  };
  // Matrix-core lists, ordered for the L2 caches of the XCDs. A row of G or F holds the
  // entries of consecutive m side by side (16 bytes each in FP32), so the items of one ring
  // block and eight consecutive m read or write the same one or two 128-byte lines of every
  // row. Such a group, taken in the
  // order of its most costly item, is dealt with seven others so that group g of the eight
  // holds positions g, g + 8, ..., g + 56: a dispatch that deals workgroups to the XCDs in
  // turn runs each group on one XCD, its members one after another. Missing members are
  // empty items (m = -1, the kernels return at once).
  auto xcd_order = [&](const std::vector<WorkItem>& items) {
    std::vector<std::vector<WorkItem>> groups;
    std::map<std::pair<int, int>, int> index;
    for (const WorkItem& w : items) {
      const auto key = std::make_pair(w.blk, w.m >> 3);
      auto f = index.find(key);
      if (f == index.end()) {
        f = index.emplace(key, (int)groups.size()).first;
        groups.emplace_back();
      }
      groups[f->second].push_back(w);
    }
    for (auto& g : groups)
      std::sort(g.begin(), g.end(), [](const WorkItem& a, const WorkItem& b) { return a.m < b.m; });
    std::vector<WorkItem> out;
    for (size_t s0 = 0; s0 < groups.size(); s0 += 8)
      for (size_t k = 0; k < 8; ++k)
        for (size_t g = s0; g < s0 + 8; ++g)
          out.push_back(g < groups.size() && k < groups[g].size() ? groups[g][k] : WorkItem{-1, 0});
    return out;
  };
  // FP64 lists: one bin per wave of a launch (FP64_WAVES_PER_SIMD per SIMD, at most one
  // per item); items, most costly first, each go to the least-loaded bin; bins are
  // stored in turn, with off[b] .. off[b + 1] the items of bin b
  auto pack_bins = [&](int rb, int scaled_cost, std::vector<int32_t>* off) {
    std::vector<WorkItem> items = make_items(rb);
    std::vector<int64_t> cost(items.size());
    for (size_t i = 0; i < items.size(); ++i) cost[i] = item_cost(items[i], rb, scaled_cost);
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    const int nb = std::max(1, std::min((int)items.size(), FP64_WAVES_PER_SIMD * 4 * g.n_cu));
    std::vector<std::vector<int>> bins(nb);
    using Load = std::pair<int64_t, int>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> least;
    for (int b = 0; b < nb; ++b) least.push({0, b});
    for (int i : order) {
      const Load l = least.top();
      least.pop();
      bins[l.second].push_back(i);
      least.push({l.first + cost[i], l.second});
    }
    std::vector<WorkItem> packed;
    off->assign(1, 0);
    for (const auto& b : bins) {
      for (int i : b) packed.push_back(items[i]);
      off->push_back((int32_t)packed.size());
    }
    return packed;
  };
  g.ring_block_ana = ana_ring_block(g.npairs);
  g.ring_block_syn = ana_ring_block(g.npairs);
  g.nblk_max_ana = (g.npairs + g.ring_block_ana - 1) / g.ring_block_ana;
  std::vector<int32_t> nblk(lmax + 1);
  for (int m = 0; m <= lmax; ++m) nblk[m] = (g.n_active[m] + g.ring_block_ana - 1) / g.ring_block_ana;
  std::vector<int32_t> bins_ana, bins_syn;
  const auto ia = pack_bins(g.ring_block_ana, FP64_SCALED_COST_ANA, &bins_ana);
  const auto is = pack_bins(g.ring_block_syn, FP64_SCALED_COST_SYN, &bins_syn);
  const auto i128 = xcd_order(make_items(128)), i256 = xcd_order(make_items(256)), i64 = xcd_order(make_items(64));
  g.n_ana = (int)ia.size();
  g.n_syn = (int)is.size();
  g.nbins_ana = (int)bins_ana.size() - 1;
  g.nbins_syn = (int)bins_syn.size() - 1;
  g.n_a128 = (int)i128.size();
  g.n_a256 = (int)i256.size();
  g.n_s64 = (int)i64.size();
  if ((rc = M.upload(&g.nact, g.n_active))) return rc;
  if ((rc = M.upload(&g.nblk_ana, nblk))) return rc;
  if ((rc = M.upload(&g.items_ana, ia))) return rc;
  if ((rc = M.upload(&g.items_syn, is))) return rc;
  if ((rc = M.upload(&g.bins_ana, bins_ana))) return rc;
  if ((rc = M.upload(&g.bins_syn, bins_syn))) return rc;
  if ((rc = M.upload(&g.items_a128, i128))) return rc;
  if ((rc = M.upload(&g.items_a256, i256))) return rc;
  if ((rc = M.upload(&g.items_s64, i64))) return rc;
  return WF_OK;
}

}  // namespace

RingGeo ring_geometry(int n, int i) {
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

int get_geometry(int nside, int lmax, std::shared_ptr<Geometry>* out) {
  int dev = 0;
  MWF_HIP(hipGetDevice(&dev));
  const auto key = std::make_tuple(dev, nside, lmax);
  std::lock_guard<std::mutex> lock(g_geo_mu);
  auto it = g_geo.find(key);
  if (it != g_geo.end()) {
    if (auto live = it->second.lock()) {
      *out = live;
      return WF_OK;
    }
  }
  auto g = std::make_shared<Geometry>();
  g->device = dev;
  MWF_HIP(hipDeviceGetAttribute(&g->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  if (g->n_cu <= 0) g->n_cu = 1;
  g->nside = nside;
  g->lmax = lmax;
  const int rc = build_geometry(*g);
  if (rc) return rc;
  g_geo[key] = g;
  *out = g;
  return WF_OK;
}

}  // namespace mwf
