// dsp_runtime.hip -- host side of libdsp.so: argument checks, patch geometry
// on an exact integer lattice, neighbour and guard-box tables, device memory,
// the round driver of the dispatcher, and the C ABI declared in dsp.h.
//
// Dispatcher (Sec. 3B): a round scans every patch for readiness (Eq. (1):
// no neighbour lags behind it by more than the grace, and the slot the update
// overwrites is no longer needed), then updates the whole ready set in one
// launch sequence and publishes it.  The updates of one round never read a
// slot that another update of the round writes, so the result does not
// depend on how the ready set is split or ordered.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <memory>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/dsp.h"
#include "dsp_dev.h"
#include "dsp_guard.h"

using namespace dsp;

namespace {

thread_local std::string g_err;
int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

int64_t gcd_i64(int64_t a, int64_t b) {
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a < 0 ? -a : a;
}
int64_t floordiv(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  if ((a % b) != 0 && (a < 0)) --q;
  return q;
}
int64_t ceildiv(int64_t a, int64_t b) { return -floordiv(-a, b); }

struct HPatch {
  int n, level;
  bool frozen;
  double dx;
  int64_t lo[3], len, dxl;
  int64_t V, slot_off;
};

}  // namespace

struct dsp_set {
  dsp_config cfg;
  int np = 0;
  std::vector<HPatch> P;
  int64_t box_lo[3], box_len[3];
  int64_t bsize = 1;
  int nb[3] = {1, 1, 1};
  std::vector<std::vector<int>> bucket;
  std::vector<std::vector<int>> nbors;  // host copy (plain path)
  hipStream_t stream = nullptr;
  bool use_alloc = false;
  dsp_allocator alloc{};
  std::vector<void*> allocs;
  bool f32 = false;
  int nmax = 0;
  int nmin = 1 << 30;
  int B = 0;  // batch capacity (patch slots of work memory)
  int klog_cap = 256;
  int64_t total_values = 0;
  std::vector<int64_t> host_off;
  // device memory
  void* slots = nullptr;
  DevSet D{};
  void* work_pad = nullptr;
  void *work_w = nullptr, *work_h = nullptr, *work_s = nullptr, *work_f = nullptr, *work_e = nullptr;
  int64_t pad_stride = 0, w_stride = 0, s_stride = 0, f_stride = 0, e_stride = 0, fm3 = 0;
  double* smax = nullptr;
  int* d_list = nullptr;
  int* d_counters = nullptr;
  int* d_single = nullptr;
  StepPtr st{};
  double* d_hostbuf = nullptr;
  int64_t* d_host_off = nullptr;
  double* d_stats = nullptr;
  // device-side mutable pointers (same memory as in D, non-const views)
  int* d_err = nullptr;
  unsigned long long* d_cnt = nullptr;  // floor, fallback, updates
  bool initialised = false;
  double last_ms = 0.0;
  int64_t rounds = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t ev_used = 0;
  double kern_ms = 0.0;
  int64_t kern_launches = 0;

  ~dsp_set() { release(); }

  bool alloc_failed = false;
  std::string alloc_msg;
  void* dalloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* p = nullptr;
    if (use_alloc) {
      p = alloc.alloc(alloc.ctx, bytes);
    } else {
      const hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        p = nullptr;
        if (alloc_msg.empty())
          alloc_msg = std::string(hipGetErrorString(e)) + " (" + std::to_string(bytes) + " bytes)";
      }
    }
    if (p)
      allocs.push_back(p);
    else
      alloc_failed = true;
    return p;
  }
  void release() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    if (gstream) (void)hipStreamDestroy(gstream);
    gstream = nullptr;
    if (tend_host) (void)hipHostFree(tend_host);
    tend_host = nullptr;
    for (hipEvent_t& e : qev)
      if (e) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
    for (void* p : allocs) {
      if (use_alloc)
        alloc.free(alloc.ctx, p);
      else
        (void)hipFree(p);
    }
    allocs.clear();
    for (auto& e : ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    ev.clear();
  }

  // ---- geometry -------------------------------------------------------------
  int locate(int64_t X[3], const int mode[3]) const {
    for (int d = 0; d < 3; ++d) {
      const int64_t L = box_len[d];
      if (mode[d] == 0)
        X[d] = box_lo[d] + ((X[d] - box_lo[d]) % L + L) % L;
      else
        X[d] = box_lo[d] + L - ((box_lo[d] + L - X[d]) % L + L) % L;
    }
    int bi[3];
    for (int d = 0; d < 3; ++d) {
      int64_t x = X[d] - box_lo[d] - (mode[d] ? 1 : 0);
      if (x < 0) x += box_len[d];
      bi[d] = (int)std::min<int64_t>(x / bsize, nb[d] - 1);
    }
    int best = -1;
    for (int q : bucket[((size_t)bi[2] * nb[1] + bi[1]) * nb[0] + bi[0]]) {
      bool in = true;
      for (int d = 0; d < 3 && in; ++d) {
        const int64_t a = P[q].lo[d], b = P[q].lo[d] + P[q].len;
        in = mode[d] == 0 ? (X[d] >= a && X[d] < b) : (X[d] > a && X[d] <= b);
      }
      if (in && (best < 0 || P[q].dxl < P[best].dxl)) best = q;
    }
    return best;
  }

  // Guard boxes of patch p for guard depth `depth`: per (component, region)
  // the element boxes and their source patches.
  int build_boxes(int p, int depth, std::vector<std::vector<GBox>>& per_key, std::set<int>* sources) {
    const HPatch& H = P[p];
    const int n = H.n;
    per_key.assign(108, std::vector<GBox>());
    int64_t minlen = bsize;
    for (int comp = -1; comp < 3; ++comp) {
      for (int rz = 0; rz < 3; ++rz)
        for (int ry = 0; ry < 3; ++ry)
          for (int rx = 0; rx < 3; ++rx) {
            if (rx == 1 && ry == 1 && rz == 1) continue;
            const int rg[3] = {rx, ry, rz};
            const int key = (comp + 1) * 27 + (rz * 3 + ry) * 3 + rx;
            // index ranges, split at the patch centre along a face's own axis
            std::vector<std::pair<std::array<int, 6>, std::array<int, 3>>> subs;
            int lo3[3], hi3[3], md[3];
            for (int d = 0; d < 3; ++d) {
              const bool fa = (d == comp);
              if (rg[d] == 0) { lo3[d] = -depth; hi3[d] = -1; }
              else if (rg[d] == 1) { lo3[d] = 0; hi3[d] = fa ? n : n - 1; }
              else { lo3[d] = fa ? n + 1 : n; hi3[d] = fa ? n + depth : n + depth - 1; }
              md[d] = (fa && rg[d] == 2) ? 1 : 0;
            }
            if (comp >= 0 && rg[comp] == 1) {
              std::array<int, 6> a{lo3[0], lo3[1], lo3[2], hi3[0], hi3[1], hi3[2]};
              std::array<int, 6> b = a;
              a[3 + comp] = n / 2;
              b[comp] = n / 2 + 1;
              std::array<int, 3> ma{md[0], md[1], md[2]}, mb = ma;
              ma[comp] = 0;
              mb[comp] = 1;
              subs.push_back({a, ma});
              subs.push_back({b, mb});
            } else {
              subs.push_back({{lo3[0], lo3[1], lo3[2], hi3[0], hi3[1], hi3[2]}, {md[0], md[1], md[2]}});
            }
            for (auto& sb : subs) {
              const int* blo = sb.first.data();
              const int* bhi = sb.first.data() + 3;
              const int* mode = sb.second.data();
              int64_t base[3];
              for (int d = 0; d < 3; ++d) base[d] = H.lo[d] + (d == comp ? 0 : H.dxl / 2);
              // periodic image shift of the whole box
              int64_t W[3];
              for (int d = 0; d < 3; ++d) {
                int64_t x0 = base[d] + (int64_t)blo[d] * H.dxl, x1 = base[d] + (int64_t)bhi[d] * H.dxl;
                int64_t X0[3] = {0, 0, 0}, X1[3] = {0, 0, 0};
                X0[d] = x0;
                X1[d] = x1;
                const int64_t L = box_len[d];
                auto wrap = [&](int64_t x) {
                  return mode[d] == 0 ? box_lo[d] + ((x - box_lo[d]) % L + L) % L
                                      : box_lo[d] + L - ((box_lo[d] + L - x) % L + L) % L;
                };
                W[d] = wrap(x0) - x0;
                if (wrap(x1) - x1 != W[d]) return fail(DSP_EINVAL, "guard region straddles the periodic boundary");
              }
              // discover the source patches by sampling the box
              std::set<int> qs;
              int stride[3];
              for (int d = 0; d < 3; ++d) stride[d] = (int)std::max<int64_t>(1, (minlen / 2) / H.dxl);
              for (int k = blo[2];; k = std::min(k + stride[2], bhi[2])) {
                for (int j = blo[1];; j = std::min(j + stride[1], bhi[1])) {
                  for (int i = blo[0];; i = std::min(i + stride[0], bhi[0])) {
                    const int id[3] = {i, j, k};
                    int64_t X[3];
                    for (int d = 0; d < 3; ++d) X[d] = base[d] + (int64_t)id[d] * H.dxl;
                    const int q = locate(X, mode);
                    if (q < 0) return fail(DSP_EINVAL, "a guard zone lies outside every patch");
                    qs.insert(q);
                    if (i == bhi[0]) break;
                  }
                  if (j == bhi[1]) break;
                }
                if (k == bhi[2]) break;
              }
              int64_t covered = 0;
              for (int q : qs) {
                const HPatch& Q = P[q];
                GBox g{};
                g.q = q;
                bool empty = false;
                for (int d = 0; d < 3; ++d) {
                  const int64_t off = base[d] + W[d];
                  int64_t a, b;
                  if (mode[d] == 0) {
                    a = ceildiv(Q.lo[d] - off, H.dxl);
                    b = floordiv(Q.lo[d] + Q.len - 1 - off, H.dxl);
                  } else {
                    a = floordiv(Q.lo[d] - off, H.dxl) + 1;
                    b = floordiv(Q.lo[d] + Q.len - off, H.dxl);
                  }
                  g.lo[d] = (int)std::max<int64_t>(a, blo[d]);
                  g.hi[d] = (int)std::min<int64_t>(b, bhi[d]);
                  if (g.lo[d] > g.hi[d]) empty = true;
                  g.wrap[d] = W[d];
                }
                if (empty) continue;
                bool same = (Q.dxl == H.dxl);
                for (int d = 0; d < 3 && same; ++d) {
                  const int64_t rel = base[d] + W[d] + (int64_t)g.lo[d] * H.dxl - Q.lo[d] - (d == comp ? 0 : Q.dxl / 2);
                  if (rel % Q.dxl != 0) same = false;
                  else g.shift[d] = (int)(rel / Q.dxl) - g.lo[d];
                }
                g.same = same ? 1 : 0;
                if (same) {  // the shifted box must lie inside the source slice
                  for (int d = 0; d < 3; ++d) {
                    const int qhi = Q.n - 1 + (d == comp ? 1 : 0);
                    if (g.lo[d] + g.shift[d] < 0 || g.hi[d] + g.shift[d] > qhi)
                      return fail(DSP_EINVAL, "guard box maps outside its source patch");
                  }
                }
                covered += (int64_t)(g.hi[0] - g.lo[0] + 1) * (g.hi[1] - g.lo[1] + 1) * (g.hi[2] - g.lo[2] + 1);
                per_key[key].push_back(g);
                if (sources && q != p) sources->insert(q);
              }
              const int64_t vol = (int64_t)(bhi[0] - blo[0] + 1) * (bhi[1] - blo[1] + 1) * (bhi[2] - blo[2] + 1);
              if (covered != vol) return fail(DSP_EINVAL, "guard zone not covered by exactly one patch (overlap?)");
            }
            merge_boxes(per_key[key]);
          }
    }
    return 0;
  }

  // Join boxes of one region that read the same source the same way and
  // tile a larger box (the split at the patch centre usually leaves two such
  // halves), so most regions end up as one box.
  static void merge_boxes(std::vector<GBox>& v) {
    auto alike = [](const GBox& a, const GBox& b) {
      if (a.q != b.q || a.same != b.same) return false;
      for (int d = 0; d < 3; ++d)
        if (a.shift[d] != b.shift[d] || a.wrap[d] != b.wrap[d]) return false;
      return true;
    };
    for (bool changed = true; changed;) {
      changed = false;
      for (size_t x = 0; x < v.size() && !changed; ++x)
        for (size_t y = 0; y < v.size() && !changed; ++y) {
          if (x == y || !alike(v[x], v[y])) continue;
          for (int d = 0; d < 3; ++d) {
            const int e = (d + 1) % 3, f = (d + 2) % 3;
            if (v[x].hi[d] + 1 == v[y].lo[d] && v[x].lo[e] == v[y].lo[e] && v[x].hi[e] == v[y].hi[e] &&
                v[x].lo[f] == v[y].lo[f] && v[x].hi[f] == v[y].hi[f]) {
              v[x].hi[d] = v[y].hi[d];
              v.erase(v.begin() + (long)y);
              changed = true;
              break;
            }
          }
        }
    }
  }

  template <class T> WorkPtr<T> work() const {
    WorkPtr<T> W;
    W.pad = (T*)work_pad;
    W.pad_stride = pad_stride;
    W.w = (T*)work_w;
    W.h = (T*)work_h;
    W.w_stride = w_stride;
    W.s = (T*)work_s;
    W.s_stride = s_stride;
    W.f = (T*)work_f;
    W.f_stride = f_stride;
    W.fm3 = fm3;
    W.e = (T*)work_e;
    W.e_stride = e_stride;
    W.smax = smax;
    return W;
  }

  hipEvent_t next_event(bool first) {
    if (ev_used >= ev.size()) {
      hipEvent_t a, b;
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      ev.push_back({a, b});
    }
    return first ? ev[ev_used].first : ev[ev_used].second;
  }

  // one launch sequence for list[off .. off+count)
  bool fused = true;  // fused marching kernel (false: staged kernels)
  bool any_generic = false;  // some guard region is not one same-resolution box
  // adjoint: staged work buffers of the recomputed forward steps (one set
  // per step of a checkpoint segment when they fit in kAdjKeepBytes, else
  // one set, refilled by a second recompute), their cotangents, the states
  // of one segment and two cotangent vectors (allocated on first use)
  static constexpr size_t kAdjKeepBytes = (size_t)16 << 30;
  bool adj_ready = false;
  int adj_copies = 1;
  void* adj_w[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  void* adj_l[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  void *adj_states = nullptr, *adj_la = nullptr, *adj_lb = nullptr;
  int adj_prepare() {
    if (adj_ready) return 0;
    const size_t tsz = f32 ? 4 : 8;
    const int64_t sizes[6] = {pad_stride, w_stride, w_stride, s_stride, f_stride, e_stride};
    size_t one = 0;
    for (int q = 0; q < 6; ++q) one += tsz * (size_t)sizes[q] * np;
    adj_copies = 8 * one <= kAdjKeepBytes ? 8 : 1;
    const char* rc = getenv("DSP_ADJ_RECOMPUTE");  // "1": one set, each step recomputed twice
    if (rc && std::string(rc) == "1") adj_copies = 1;
    for (int q = 0; q < 6; ++q) {
      adj_w[q] = dalloc(tsz * (size_t)sizes[q] * np * adj_copies);
      adj_l[q] = dalloc(tsz * (size_t)sizes[q] * np);
    }
    adj_states = dalloc(tsz * (size_t)total_values * 8);
    adj_la = dalloc(tsz * (size_t)total_values);
    adj_lb = dalloc(tsz * (size_t)total_values);
    if (alloc_failed) return DSP_ENOMEM;
    adj_ready = true;
    return 0;
  }
  // copy: which step's set of the forward work buffers (0 for cot)
  template <class T> WorkPtr<T> adj_work(bool cot, int copy = 0) const {
    void* const* b = cot ? adj_l : adj_w;
    WorkPtr<T> W;
    W.pad = (T*)b[0] + (int64_t)copy * pad_stride * np;
    W.pad_stride = pad_stride;
    W.w = (T*)b[1] + (int64_t)copy * w_stride * np;
    W.h = (T*)b[2] + (int64_t)copy * w_stride * np;
    W.w_stride = w_stride;
    W.s = (T*)b[3] + (int64_t)copy * s_stride * np;
    W.s_stride = s_stride;
    W.f = (T*)b[4] + (int64_t)copy * f_stride * np;
    W.f_stride = f_stride;
    W.fm3 = fm3;
    W.e = (T*)b[5] + (int64_t)copy * e_stride * np;
    W.e_stride = e_stride;
    W.smax = smax;
    return W;
  }
  int dt_fused = 0;          // the last step launch also computed the Courant rate and level
  // persistent dispatcher (work queue): eligible sets, its queue, workers,
  // and the captured graph of its launches (seed + persistent kernel)
  bool poison = false;  // DSP_POISON=1: unwritten ring slots hold NaN (a check for wrong-slot guard reads)
  bool queue_ok = false;
  int dispatch = DSP_DISPATCH_ROUNDS;  // how dsp_advance_to runs LOCAL steps
  int workers = 0;
  int queue_fn = 0;
  QueueState Q{};
  int64_t* tend_host = nullptr;  // pinned: the end time copied into Q.tend before a launch
  hipStream_t gstream = nullptr;  // stream of the graph launches
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t qev[2] = {nullptr, nullptr};
  void update_batch(int off, int count, int dt_kind, double t_end, int clip, const int* list) {
    hipEvent_t e0 = next_event(true), e1 = next_event(false);
    ev_used++;
    StepPtr s2{st.k + off, st.dtk + off, st.dt + off};
    if (fused) {
      if (f32)
        dt_fused = launch_fused<float>(D, list + off, count, nmin, nmax, (float*)slots, (float*)work_pad,
                                       pad_stride, any_generic, smax, s2, stream, dt_kind, t_end, clip, e0, e1);
      else
        dt_fused = launch_fused<double>(D, list + off, count, nmin, nmax, (double*)slots, (double*)work_pad,
                                        pad_stride, any_generic, smax, s2, stream, dt_kind, t_end, clip, e0, e1);
      return;
    }
    if (f32)
      launch_update<float>(D, list + off, count, nmax, (float*)slots, work<float>(), s2, stream, dt_kind, t_end,
                           clip, e0, e1);
    else
      launch_update<double>(D, list + off, count, nmax, (double*)slots, work<double>(), s2, stream, dt_kind, t_end,
                            clip, e0, e1);
  }

  int check_err(int bits) {
    if (bits & ERR_NONFINITE) return fail(DSP_ENONFINITE, "non-finite state or signal speed");
    if (bits & ERR_NEGATIVE) return fail(DSP_ENEGATIVE, "non-positive density or pressure");
    if (bits & ERR_KMAX) return fail(DSP_EKMAX, "time-step level exceeds kmax");
    if (bits & ERR_STATE) return fail(DSP_ESTATE, "guard data not available (internal)");
    if (bits & ERR_TIMEOUT) return fail(DSP_ESTATE, "the persistent dispatcher timed out waiting for work");
    return 0;
  }

  void begin_timing() {
    (void)hipMemsetAsync(d_cnt + 3, 0, sizeof(unsigned long long), stream);
    ev_used = 0;
    kern_ms = 0.0;
    kern_launches = 0;
  }
  // real: how many of the recorded launches did work (rounds counted on the
  // device also enqueue a few empty rounds at the end); -1 = all
  void end_timing(int64_t real = -1) {
    (void)hipStreamSynchronize(stream);
    const size_t m_end = (real >= 0 && (size_t)real < ev_used) ? (size_t)real : ev_used;
    for (size_t m = 0; m < m_end; ++m) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[m].first, ev[m].second) == hipSuccess) kern_ms += ms;
    }
    kern_launches = (int64_t)m_end;
  }
};

namespace {

// Static plan of the staged guard resampling (k_gfill), built once at
// create: the per-axis overlap tables of every resampled box (one copy per
// distinct geometry) and the work items of every patch.  The tables follow
// cross_value's reading of the overlap (exact integer lattice lengths, the
// weights and centre offsets in double); the chunks cut a box along its
// longest axis into runs of target indices whose time-interpolated source
// block, with its slope neighbours, fits the LDS stage: every variable over
// as many indices as fit, else one index with as many variables as fit.
struct GTabH {
  int i0, cnt;
  double w[GMAXC], off[GMAXC];
};

struct GfillPlan {
  std::vector<GTabH> pool;
  std::map<std::array<int64_t, 7>, int> seen;  // geometry -> pool offset (-1: over the table limits)

  // Axis-d table of box g (target patch H, source patch Q): the pool entry
  // of target index 0, or -1 when a target index overlaps more than GMAXC
  // source indices.
  int table(const HPatch& H, const HPatch& Q, int comp, const GBox& g, int d) {
    const int ext = g.hi[d] - g.lo[d] + 1;
    const int64_t sdx = Q.dxl, len = Q.len, tdx = H.dxl;
    const int64_t X0 = H.lo[d] + (int64_t)g.lo[d] * tdx + (d == comp ? 0 : tdx / 2) + g.wrap[d] - Q.lo[d];
    const std::array<int64_t, 7> key{d == comp ? 1 : 0, Q.n, sdx, len, tdx, ext, X0};
    const auto f = seen.find(key);
    if (f != seen.end()) return f->second;
    const int at = (int)pool.size(), nq = Q.n;
    auto clamp = [&](int64_t v) { return v < 0 ? (int64_t)0 : (v > len ? len : v); };
    for (int t = 0; t < ext; ++t) {
      const int64_t X = X0 + (int64_t)t * tdx;
      GTabH e{};
      if (d == comp) {  // the two source faces bracketing the target face
        const int64_t A = clamp(X);
        int f0 = (int)(A / sdx);
        int64_t rem = A - (int64_t)f0 * sdx;
        if (f0 >= nq) {
          f0 = nq;
          rem = 0;
        }
        const double wn = (double)rem / (double)sdx;
        e.i0 = f0;
        e.cnt = wn == 0.0 ? 1 : 2;
        e.w[0] = 1.0 - wn;
        e.w[1] = wn;
      } else {
        const int64_t A = clamp(X - tdx / 2), B = clamp(X + tdx / 2);
        const int c0 = std::min(std::max((int)(A / sdx), 0), nq - 1);
        const int c1 = std::min(std::max((int)((B - 1) / sdx), 0), nq - 1);
        double tot = 0.0;
        int k = 0, first = -1;
        for (int c = c0; c <= c1; ++c) {
          const int64_t a = std::max(A, (int64_t)c * sdx), b = std::min(B, (int64_t)(c + 1) * sdx);
          if (b - a <= 0) continue;
          if (first < 0) first = c;
          tot += (double)(b - a);
          ++k;
        }
        if (k > GMAXC || k == 0) {
          pool.resize(at);
          seen[key] = -1;
          return -1;
        }
        e.i0 = first;
        e.cnt = k;
        for (int m = 0; m < k; ++m) {
          const int c = first + m;
          const int64_t a = std::max(A, (int64_t)c * sdx), b = std::min(B, (int64_t)(c + 1) * sdx);
          e.w[m] = (double)(b - a) / tot;
          e.off[m] = (0.5 * (double)(a + b) - ((double)c + 0.5) * (double)sdx) / (double)sdx;
        }
      }
      pool.push_back(e);
    }
    seen[key] = at;
    return at;
  }

  // Work items of resampled box m (g, from Q into H) appended to out;
  // false (nothing appended) if the box exceeds the tables or the stage.
  bool box(const HPatch& H, const HPatch& Q, int comp, const GBox& g, int m, int prec, std::vector<GItem>& out) {
    const int64_t stage = GSTAGE_BYTES / (prec == DSP_F32 ? 4 : 8);
    int ext[3], tab[3];
    for (int d = 0; d < 3; ++d) {
      ext[d] = g.hi[d] - g.lo[d] + 1;
      if (ext[d] > GMAXT) return false;
    }
    for (int d = 0; d < 3; ++d)
      if ((tab[d] = table(H, Q, comp, g, d)) < 0) return false;
    const int nq = Q.n, nvar = comp < 0 ? 5 : 1;
    int ca = 0;
    if (ext[1] > ext[ca]) ca = 1;
    if (ext[2] > ext[ca]) ca = 2;
    const int cb = (ca + 1) % 3, cc = (ca + 2) % 3;
    // source range of target indices [a, b] along axis d: the overlapped
    // indices, plus the slope neighbours across (not along a face's own axis)
    auto range = [&](int d, int a, int b, int& r0, int& r1) {
      r0 = pool[tab[d] + a].i0;
      r1 = pool[tab[d] + b].i0 + pool[tab[d] + b].cnt - 1;
      if (d != comp) {
        r0 = std::max(r0 - 1, 0);
        r1 = std::min(r1 + 1, nq - 1);
      }
    };
    int rb0, rb1, rc0, rc1;
    range(cb, 0, ext[cb] - 1, rb0, rb1);
    range(cc, 0, ext[cc] - 1, rc0, rc1);
    const int64_t across = (int64_t)(rb1 - rb0 + 1) * (rc1 - rc0 + 1);
    auto size = [&](int a, int b) {
      int x0, x1;
      range(ca, a, b, x0, x1);
      return across * (x1 - x0 + 1);
    };
    std::vector<GItem> its;
    int ta = 0, v0 = 0;
    while (ta < ext[ca]) {
      int tb = ta, nv;
      if (v0 == 0 && size(ta, ta) * nvar <= stage) {
        nv = nvar;
        while (tb + 1 < ext[ca] && size(ta, tb + 1) * nvar <= stage) ++tb;
      } else {
        nv = (int)std::min<int64_t>(stage / size(ta, ta), nvar - v0);
        if (nv < 1) return false;
      }
      GItem it{};
      it.m = m;
      it.comp = comp;
      it.ca = ca;
      it.ta = ta;
      it.tb = tb;
      it.v0 = v0;
      it.nv = nv;
      range(ca, ta, tb, it.r0[ca], it.r1[ca]);
      it.r0[cb] = rb0;
      it.r1[cb] = rb1;
      it.r0[cc] = rc0;
      it.r1[cc] = rc1;
      for (int d = 0; d < 3; ++d) it.tab[d] = tab[d];
      it.nq = nq;
      its.push_back(it);
      v0 += nv;
      if (v0 >= nvar) {
        v0 = 0;
        ta = tb + 1;
      }
    }
    out.insert(out.end(), its.begin(), its.end());
    return true;
  }
};

bool tolat(double x, int64_t scale, int64_t& out) {
  const double y = x * (double)scale;
  const double r = std::nearbyint(y);
  if (std::fabs(y - r) > 1e-6) return false;
  out = (int64_t)r;
  return true;
}

int hipck(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(DSP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return 0;
}

}  // namespace

extern "C" {

const char* dsp_last_error(void) { return g_err.c_str(); }

int dsp_create(const dsp_config* cfg, const dsp_patch_desc* pd, int32_t npatch, void* hip_stream,
               const dsp_allocator* alloc, dsp_set** out) {
  if (!out) return fail(DSP_EINVAL, "null output handle");
  *out = nullptr;
  if (!cfg || !pd || npatch <= 0) return fail(DSP_EINVAL, "null argument or no patches");
  {
    int nactive = 0;
    for (int p = 0; p < npatch; ++p) nactive += (pd[p].flags & DSP_PATCH_FROZEN) ? 0 : 1;
    if (nactive == 0) return fail(DSP_EINVAL, "every patch is a boundary patch");
    if (nactive < npatch && cfg->dt_mode != DSP_DT_LOCAL)
      return fail(DSP_EINVAL, "boundary patches need LOCAL time steps");
  }
  const dsp_config c = *cfg;
  if (!(c.gamma > 1.0) || !(c.courant > 0.0) || c.nguard < 2 || c.nguard > 3 || c.nslots < 2 ||
      c.nslots > 8 || c.kmax < 0 || c.kmax > 40 || c.limiter != 0 || !(c.grace >= 0.0 && c.grace < 1.0) ||
      (c.prec != DSP_F32 && c.prec != DSP_F64) || c.dt_mode < 0 || c.dt_mode > 3 || c.p_floor < 0.0)
    return fail(DSP_EINVAL, "invalid configuration");
  if ((c.dt_mode == DSP_DT_LOCAL || c.dt_mode == DSP_DT_GLOBAL_QUANT) && !(c.dt_base > 0.0))
    return fail(DSP_EINVAL, "dt_base must be positive");
  if (c.grace > 0.0 && (c.dt_mode != DSP_DT_LOCAL || c.nslots < 3))
    return fail(DSP_EINVAL, "a grace needs LOCAL time steps and at least 3 slots");
  if (!(c.eta >= 0.0) || !(c.gamma_ad >= 0.0) || (c.gamma_ad > 0.0 && !(c.rho_ion > 0.0)))
    return fail(DSP_EINVAL, "invalid non-ideal parameters");
  if (c.torder < 0 || c.torder > 2 || (c.torder == 2 && c.nslots < 3))
    return fail(DSP_EINVAL, "time order must be 1 or 2 (2 needs at least 3 slots)");
  if (c.dt_mode == DSP_DT_FIXED && !(c.dt_fixed > 0.0)) return fail(DSP_EINVAL, "dt_fixed must be positive");
  for (int d = 0; d < 3; ++d)
    if (c.periodic[d] != 1) return fail(DSP_EINVAL, "only periodic boxes are supported");

  std::unique_ptr<dsp_set> S(new dsp_set());
  S->cfg = c;
  S->np = npatch;
  S->stream = (hipStream_t)hip_stream;
  S->f32 = (c.prec == DSP_F32);
  {
    const char* pz = getenv("DSP_POISON");
    S->poison = pz && std::string(pz) == "1";
  }
  if (alloc) {
    if (!alloc->alloc || !alloc->free) return fail(DSP_EINVAL, "allocator without alloc/free");
    S->use_alloc = true;
    S->alloc = *alloc;
  }
  // lattice: 2 lcm(n/size) points per unit length
  int64_t F = 1;
  for (int p = 0; p < npatch; ++p) {
    const dsp_patch_desc& q = pd[p];
    if (q.n < 4 || q.n > 64 || !(q.size[0] > 0.0) || q.size[0] != q.size[1] || q.size[0] != q.size[2])
      return fail(DSP_EINVAL, "patches must be cubic with 4 <= n <= 64");
    const double cpl = q.n / q.size[0];
    const int64_t ic = (int64_t)std::llround(cpl);
    if (ic <= 0 || std::fabs(cpl - (double)ic) > 1e-9 * cpl) return fail(DSP_EINVAL, "n/size must be an integer");
    F = F / gcd_i64(F, ic) * ic;
    if (F > ((int64_t)1 << 40)) return fail(DSP_EINVAL, "lattice too fine");
  }
  const int64_t scale = 2 * F;
  for (int d = 0; d < 3; ++d) {
    int64_t a, b;
    if (!tolat(c.box_lo[d], scale, a) || !tolat(c.box_hi[d], scale, b) || b <= a)
      return fail(DSP_EINVAL, "box not on the patch lattice");
    S->box_lo[d] = a;
    S->box_len[d] = b - a;
  }
  S->P.resize(npatch);
  int64_t minlen = INT64_MAX, off = 0;
  S->host_off.assign(npatch + 1, 0);
  for (int p = 0; p < npatch; ++p) {
    HPatch& H = S->P[p];
    H.n = pd[p].n;
    H.level = pd[p].level;
    H.frozen = (pd[p].flags & DSP_PATCH_FROZEN) != 0;
    H.dx = pd[p].size[0] / pd[p].n;
    if (!tolat(pd[p].size[0], scale, H.len)) return fail(DSP_EINVAL, "patch size not on the lattice");
    H.dxl = H.len / H.n;
    for (int d = 0; d < 3; ++d) {
      if (!tolat(pd[p].origin[d], scale, H.lo[d])) return fail(DSP_EINVAL, "origin not on the lattice");
      if (H.lo[d] < S->box_lo[d] || H.lo[d] + H.len > S->box_lo[d] + S->box_len[d])
        return fail(DSP_EINVAL, "patch outside the box");
    }
    if (c.nguard > H.n) return fail(DSP_EINVAL, "patch smaller than its guard zones");
    H.V = 5LL * H.n * H.n * H.n + 3LL * H.n * H.n * (H.n + 1);
    H.slot_off = off;
    off += H.V * c.nslots;
    S->host_off[p + 1] = S->host_off[p] + H.V;
    minlen = std::min(minlen, H.len);
    S->nmax = std::max(S->nmax, H.n);
    S->nmin = std::min(S->nmin, H.n);
  }
  S->total_values = S->host_off[npatch];
  S->bsize = minlen;
  for (int d = 0; d < 3; ++d) S->nb[d] = (int)((S->box_len[d] + minlen - 1) / minlen);
  S->bucket.assign((size_t)S->nb[0] * S->nb[1] * S->nb[2], std::vector<int>());
  for (int p = 0; p < npatch; ++p) {
    int a[3], b[3];
    for (int d = 0; d < 3; ++d) {
      a[d] = (int)((S->P[p].lo[d] - S->box_lo[d]) / minlen);
      b[d] = (int)((S->P[p].lo[d] + S->P[p].len - 1 - S->box_lo[d]) / minlen);
    }
    for (int z = a[2]; z <= b[2]; ++z)
      for (int y = a[1]; y <= b[1]; ++y)
        for (int x = a[0]; x <= b[0]; ++x) {
          auto& bk = S->bucket[((size_t)z * S->nb[1] + y) * S->nb[0] + x];
          for (int q : bk) {  // patches may not overlap
            bool ov = true;
            for (int d = 0; d < 3; ++d)
              ov = ov && S->P[q].lo[d] < S->P[p].lo[d] + S->P[p].len && S->P[p].lo[d] < S->P[q].lo[d] + S->P[q].len;
            if (ov) return fail(DSP_EINVAL, "patches overlap");
          }
          bk.push_back(p);
        }
  }
  // neighbour relation over the configured guard depth; guard boxes of the
  // two layers the stencil reads
  std::vector<std::set<int>> reads(npatch);
  std::vector<int> rbox_off(1, 0);
  std::vector<GBox> boxes;
  std::vector<std::vector<GBox>> keys;
  // the resampling plan: per patch its work items (the boxes of the regions
  // read through the padded buffer; a resampled box that exceeds the tables
  // or the stage is flagged direct instead)
  GfillPlan plan;
  std::vector<GItem> gitems;
  std::vector<int> gitem_off(1, 0);
  for (int p = 0; p < npatch; ++p) {
    int e = S->build_boxes(p, c.nguard, keys, &reads[p]);
    if (e) return e;
    e = S->build_boxes(p, 2, keys, nullptr);
    if (e) return e;
    for (int k = 0; k < 108; ++k) {
      const int comp = k / 27 - 1;
      const bool padded = k % 27 != 13 && !(keys[k].size() == 1 && keys[k][0].same && c.torder < 2);
      for (GBox g : keys[k]) {
        const int m = (int)boxes.size();
        g.direct = 0;
        if (!g.same) {
          const size_t before = gitems.size();
          if (!plan.box(S->P[p], S->P[g.q], comp, g, m, c.prec, gitems)) g.direct = 1;
          if (!padded) gitems.resize(before);
        } else if (padded) {
          GItem it{};
          it.m = m;
          it.comp = comp;
          it.nv = comp < 0 ? 5 : 1;
          it.tab[0] = it.tab[1] = it.tab[2] = -1;
          it.nq = S->P[g.q].n;
          gitems.push_back(it);
        }
        boxes.push_back(g);
      }
      rbox_off.push_back((int)boxes.size());
    }
    gitem_off.push_back((int)gitems.size());
  }
  {
    // the fused kernel keeps the time brackets of a patch's guard boxes in LDS
    int maxbox = 0;
    for (int p = 0; p < npatch; ++p) maxbox = std::max(maxbox, rbox_off[(p + 1) * 108] - rbox_off[p * 108]);
    const char* path = getenv("DSP_PATH");
    // the non-ideal terms run on the staged kernels only
    S->fused = !(path && std::string(path) == "staged") && maxbox <= 256 && !(cfg->eta > 0.0 || cfg->gamma_ad > 0.0);
    int ngen = 0;
    for (int p = 0; p < npatch; ++p)
      for (int k = 0; k < 108; ++k) {
        if (k % 27 == 13) continue;
        const int m0 = rbox_off[p * 108 + k], m1 = rbox_off[p * 108 + k + 1];
        if (!(m1 - m0 == 1 && boxes[m0].same) || cfg->torder >= 2) ++ngen;
      }
    S->any_generic = ngen > 0;
    if (getenv("DSP_DEBUG")) fprintf(stderr, "dsp_create: %d guard regions need the padded buffer\n", ngen);
    if (getenv("DSP_DEBUG"))
      fprintf(stderr, "dsp_create: %d patches, nmax %d, max guard boxes per patch %d, %s path\n", npatch,
              S->nmax, maxbox, S->fused ? "fused" : "staged");
  }
  S->nbors.assign(npatch, std::vector<int>());
  for (int p = 0; p < npatch; ++p)
    for (int q : reads[p]) {
      S->nbors[p].push_back(q);
      S->nbors[q].push_back(p);
    }
  std::vector<int> nb_off(1, 0), nb_idx;
  for (int p = 0; p < npatch; ++p) {
    auto& v = S->nbors[p];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    for (int q : v) nb_idx.push_back(q);
    nb_off.push_back((int)nb_idx.size());
  }

  // ---- device memory ----------------------------------------------------------
  dsp_set* s = S.get();
  const size_t tsz = s->f32 ? 4 : 8;
  const int ns = c.nslots;
  auto A = [&](size_t bytes) { return s->dalloc(bytes); };
  s->slots = A(tsz * (size_t)off);
  const int N = s->nmax + 4;
  s->pad_stride = 5LL * N * N * N + 3LL * N * N * (N + 1);
  s->w_stride = 8LL * N * N * N;
  s->s_stride = 24LL * N * N * N;
  s->fm3 = (int64_t)(N + 1) * (N + 1) * (N + 1);
  s->f_stride = 24LL * s->fm3;
  s->e_stride = 3LL * s->fm3;
  // work memory per batch entry: the staged kernels need every buffer; the
  // fused kernels only a padded buffer, and only if some guard region is
  // resampled or has several sources
  const int64_t pad_vals = (!s->fused || s->any_generic) ? s->pad_stride : 0;
  const int64_t per_slot =
      s->fused ? tsz * (pad_vals + 1)
               : tsz * (s->pad_stride + 2 * s->w_stride + s->s_stride + s->f_stride + s->e_stride);
  const int64_t budget = (int64_t)16 << 30;  // work memory cap
  s->B = (int)std::max<int64_t>(1, std::min<int64_t>(npatch, budget / per_slot));
  if ((c.dt_mode != DSP_DT_LOCAL) && s->B < npatch)
    return fail(DSP_EINVAL, "global time-step modes need work memory for every patch");
  s->work_pad = A(tsz * pad_vals * s->B);
  if (!s->fused) {
    s->work_w = A(tsz * s->w_stride * s->B);
    s->work_h = A(tsz * s->w_stride * s->B);
    s->work_s = A(tsz * s->s_stride * s->B);
    s->work_f = A(tsz * s->f_stride * s->B);
    s->work_e = A(tsz * s->e_stride * s->B);
  }
  s->smax = (double*)A(sizeof(double) * s->B);
  s->d_list = (int*)A(sizeof(int) * npatch);
  s->d_single = (int*)A(sizeof(int) * 4);
  s->d_counters = (int*)A(sizeof(int) * 8);
  s->st.k = (int*)A(sizeof(int) * npatch);
  s->st.dtk = (int64_t*)A(sizeof(int64_t) * npatch);
  s->st.dt = (double*)A(sizeof(double) * npatch);
  s->d_hostbuf = (double*)A(sizeof(double) * (size_t)s->total_values);
  s->d_host_off = (int64_t*)A(sizeof(int64_t) * (npatch + 1));
  s->D.host_off = s->d_host_off;
  s->D.out_words = (int)(tsz / 4);
  s->d_stats = (double*)A(sizeof(double) * 9 * npatch);
  if (s->alloc_failed) return fail(DSP_ENOMEM, "device allocation failed: " + s->alloc_msg);

  // metadata arrays
  std::vector<int> hn(npatch);
  std::vector<int8_t> hfz(npatch);
  std::vector<double> hdx(npatch);
  std::vector<int64_t> hlo(3 * npatch), hlen(npatch), hdxl(npatch), hoff(npatch), hV(npatch);
  for (int p = 0; p < npatch; ++p) {
    hn[p] = s->P[p].n;
    hfz[p] = s->P[p].frozen ? 1 : 0;
    hdx[p] = s->P[p].dx;
    for (int d = 0; d < 3; ++d) hlo[3 * p + d] = s->P[p].lo[d];
    hlen[p] = s->P[p].len;
    hdxl[p] = s->P[p].dxl;
    hoff[p] = s->P[p].slot_off;
    hV[p] = s->P[p].V;
  }
  DevSet& D = s->D;
  D.npatch = npatch;
  D.nslots = ns;
  D.kmax = c.kmax;
  D.dt_mode = c.dt_mode;
  D.exact_time = (c.dt_mode == DSP_DT_GLOBAL_EXACT || c.dt_mode == DSP_DT_FIXED) ? 1 : 0;
  D.klog_cap = s->klog_cap;
  D.gamma = c.gamma;
  D.courant = c.courant;
  D.dt_base = c.dt_base;
  D.dt_fixed = c.dt_fixed;
  D.p_floor = c.p_floor;
  D.grace = c.grace;
  D.eta = c.eta;
  D.gamma_ad = c.gamma_ad;
  D.rho_i = c.rho_ion;
  D.nonideal = (c.eta > 0.0 || c.gamma_ad > 0.0) ? 1 : 0;
  D.torder = c.torder;
  auto up = [&](const void* h, size_t bytes) -> void* {
    void* d = A(bytes);
    if (d && bytes && h) (void)hipMemcpy(d, h, bytes, hipMemcpyHostToDevice);  // empty tables: nothing to copy
    return d;
  };
  D.n = (const int*)up(hn.data(), sizeof(int) * npatch);
  D.frozen = (const int8_t*)up(hfz.data(), (size_t)npatch);
  D.dx = (const double*)up(hdx.data(), sizeof(double) * npatch);
  D.lo = (const int64_t*)up(hlo.data(), sizeof(int64_t) * 3 * npatch);
  D.len = (const int64_t*)up(hlen.data(), sizeof(int64_t) * npatch);
  D.dxl = (const int64_t*)up(hdxl.data(), sizeof(int64_t) * npatch);
  D.slot_off = (const int64_t*)up(hoff.data(), sizeof(int64_t) * npatch);
  D.slice_len = (const int64_t*)up(hV.data(), sizeof(int64_t) * npatch);
  D.cur = (int*)A(sizeof(int) * npatch);
  D.ticks = (int64_t*)A(sizeof(int64_t) * npatch);
  D.tcur = (double*)A(sizeof(double) * npatch);
  D.sticks = (int64_t*)A(sizeof(int64_t) * npatch * ns);
  D.stime = (double*)A(sizeof(double) * npatch * ns);
  D.svalid = (int8_t*)A((size_t)npatch * ns);
  D.steps = (int64_t*)A(sizeof(int64_t) * npatch);
  D.khash = (uint64_t*)A(sizeof(uint64_t) * npatch);
  D.klog = (int8_t*)A((size_t)npatch * s->klog_cap);
  {
    std::vector<int> order(npatch);
    for (int p = 0; p < npatch; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return s->P[a].n > s->P[b].n; });
    D.scan_order = (const int*)up(order.data(), sizeof(int) * npatch);
  }
  D.nb_off = (const int*)up(nb_off.data(), sizeof(int) * nb_off.size());
  D.nb_idx = (const int*)up(nb_idx.data(), sizeof(int) * std::max<size_t>(1, nb_idx.size()));
  D.rbox_off = (const int*)up(rbox_off.data(), sizeof(int) * rbox_off.size());
  D.gitem_off = (const int*)up(gitem_off.data(), sizeof(int) * gitem_off.size());
  if (gitems.empty()) gitems.resize(1);  // a placeholder: no patch lists an item
  D.gitems = (const GItem*)up(gitems.data(), sizeof(GItem) * gitems.size());
  {
    // the table pool in the set's precision
    const size_t ne = std::max<size_t>(1, plan.pool.size());
    if (s->f32) {
      std::vector<GTab<float>> t(ne);
      for (size_t i = 0; i < plan.pool.size(); ++i) {
        t[i].i0 = plan.pool[i].i0;
        t[i].cnt = plan.pool[i].cnt;
        for (int m = 0; m < GMAXC; ++m) {
          t[i].w[m] = (float)plan.pool[i].w[m];
          t[i].off[m] = (float)plan.pool[i].off[m];
        }
      }
      D.gtab = up(t.data(), sizeof(GTab<float>) * ne);
    } else {
      std::vector<GTab<double>> t(ne);
      for (size_t i = 0; i < plan.pool.size(); ++i) {
        t[i].i0 = plan.pool[i].i0;
        t[i].cnt = plan.pool[i].cnt;
        for (int m = 0; m < GMAXC; ++m) {
          t[i].w[m] = plan.pool[i].w[m];
          t[i].off[m] = plan.pool[i].off[m];
        }
      }
      D.gtab = up(t.data(), sizeof(GTab<double>) * ne);
    }
  }
  if (getenv("DSP_DEBUG"))
    fprintf(stderr, "dsp_create: %zu guard resampling items, %zu table entries\n", gitems.size(), plan.pool.size());
  D.boxes = (const GBox*)up(boxes.data(), sizeof(GBox) * std::max<size_t>(1, boxes.size()));
  D.brk = (Bracket*)A(sizeof(Bracket) * std::max<size_t>(1, boxes.size()));
  {
    // boxes grouped by (source patch, component) for the adjoint's gathered
    // guard fill; within a group in box order, which fixes the order of its sums
    std::vector<int> roff((size_t)npatch * 4 + 1, 0);
    for (int p = 0; p < npatch; ++p)
      for (int k = 0; k < 108; ++k)
        for (int m = rbox_off[p * 108 + k]; m < rbox_off[p * 108 + k + 1]; ++m)
          if (boxes[m].same) ++roff[(size_t)boxes[m].q * 4 + k / 27 + 1];
    for (size_t g = 0; g + 1 < roff.size(); ++g) roff[g + 1] += roff[g];
    std::vector<int2> rev(std::max(1, roff.back()));
    std::vector<int> fillp(roff.begin(), roff.end() - 1);
    for (int p = 0; p < npatch; ++p)
      for (int k = 0; k < 108; ++k)
        for (int m = rbox_off[p * 108 + k]; m < rbox_off[p * 108 + k + 1]; ++m)
          if (boxes[m].same) rev[fillp[(size_t)boxes[m].q * 4 + k / 27]++] = make_int2(m, p);
    D.rev_off = (const int*)up(roff.data(), sizeof(int) * roff.size());
    D.rev = (const int2*)up(rev.data(), sizeof(int2) * rev.size());
  }
  for (int p = 0; p < npatch; ++p) D.maxbox = std::max(D.maxbox, rbox_off[(p + 1) * 108] - rbox_off[p * 108]);
  D.any_direct = 0;
  for (const GBox& g : boxes) D.any_direct |= g.direct;
  if (getenv("DSP_DEBUG")) {
    int nd = 0, nx = 0;
    for (const GBox& g : boxes) {
      nd += g.direct;
      nx += g.same ? 0 : 1;
    }
    fprintf(stderr, "dsp_create: %d of %d resampled guard boxes resample without staging\n", nd, nx);
  }
  s->d_err = (int*)A(sizeof(int) * 2);
  s->d_cnt = (unsigned long long*)A(sizeof(unsigned long long) * 4);  // floor, fallback, updates, bytes
  D.err = s->d_err;
  D.floor_hits = s->d_cnt;
  D.fallback = s->d_cnt + 1;
  D.updates = s->d_cnt + 2;
  D.algo_bytes = s->d_cnt + 3;
  if (s->alloc_failed) return fail(DSP_ENOMEM, "device allocation failed: " + s->alloc_msg);
  {
    // persistent dispatcher: single-precision sets in LOCAL mode without a
    // grace, whose resampled boxes all stage (the worker has no separate
    // direct pass), on the fused path.  A worker runs the tiles of a patch in
    // turn, so sets of one-tile patches start in the queue and sets with
    // larger patches in the rounds (which run a patch's tiles side by side).
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    s->queue_ok = s->fused && s->f32 && c.dt_mode == DSP_DT_LOCAL && c.grace == 0.0 &&
                  !D.any_direct && cus > 0;
    if (s->queue_ok) {
      s->workers = std::min(cus, std::min(npatch, s->B));  // one workgroup per CU: the step takes the LDS
      s->queue_fn = (s->nmin == 16 && s->nmax == 16 && !s->any_generic) ? 16 : 0;
      QueueState& Q = s->Q;
      Q.cap = 4 * npatch;
      Q.buf = (int*)A(sizeof(int) * Q.cap);
      Q.state = (int*)A(sizeof(int) * npatch);
      int* ctr = (int*)A(sizeof(int) * 8);
      Q.head = (unsigned*)ctr;
      Q.tail = (unsigned*)(ctr + 1);
      Q.done = ctr + 2;
      Q.remaining = ctr + 3;
      Q.finished = ctr + 4;
      int64_t* tend = (int64_t*)A(sizeof(int64_t));
      Q.tend = tend;
      double tmo = 30.0;
      if (const char* e = getenv("DSP_QUEUE_TIMEOUT_S")) tmo = std::max(0.1, atof(e));
      Q.timeout = (uint64_t)(tmo * 1e8);  // s_memrealtime runs at 100 MHz
      if (s->alloc_failed) return fail(DSP_ENOMEM, "device allocation failed: " + s->alloc_msg);
      if (hipHostMalloc((void**)&s->tend_host, sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
        return fail(DSP_ENOMEM, "pinned host allocation failed");
      const char* dm = getenv("DSP_DISPATCH");
      s->dispatch =
          ((dm && std::string(dm) == "rounds") || s->nmax > MT) ? DSP_DISPATCH_ROUNDS : DSP_DISPATCH_QUEUE;
    }
  }
  int e = hipck(hipMemcpy(s->d_host_off, s->host_off.data(), sizeof(int64_t) * (npatch + 1), hipMemcpyHostToDevice),
                "hipMemcpy");
  if (e) return e;
  e = hipck(hipDeviceSynchronize(), "create");
  if (e) return e;
  *out = S.release();
  return 0;
}

static int init_common(dsp_set* s, const double* U, const void* U_dev, double t0);

int dsp_init(dsp_set* s, const double* U, size_t n_values, double t0) {
  if (!s || !U) return fail(DSP_EINVAL, "null argument");
  if ((int64_t)n_values != s->total_values) return fail(DSP_EINVAL, "wrong number of values");
  for (size_t m = 0; m < n_values; ++m)
    if (!std::isfinite(U[m])) return fail(DSP_ENONFINITE, "non-finite initial state");
  return init_common(s, U, nullptr, t0);
}

int dsp_init_device(dsp_set* s, const void* U_dev, double t0) {
  if (!s || !U_dev) return fail(DSP_EINVAL, "null argument");
  return init_common(s, nullptr, U_dev, t0);
}

static int init_common(dsp_set* s, const double* U, const void* U_dev, double t0) {
  const size_t n_values = (size_t)s->total_values;
  const dsp_config& c = s->cfg;
  int64_t tk0 = 0;
  const bool exact = (c.dt_mode == DSP_DT_GLOBAL_EXACT || c.dt_mode == DSP_DT_FIXED);
  if (!exact) {
    const double m = t0 / c.dt_base, mr = std::nearbyint(m);
    if (std::fabs(m - mr) > 1e-9 * std::max(1.0, std::fabs(m))) return fail(DSP_EALIGN, "t0 is not a multiple of dt_base");
    tk0 = (int64_t)mr << c.kmax;
  }
  const int np = s->np, ns = c.nslots;
  std::vector<int> cur(np, 0);
  std::vector<int64_t> ticks(np, tk0), sticks((size_t)np * ns, 0), zero64(np, 0);
  std::vector<double> tc(np, t0), stime((size_t)np * ns, 0.0);
  std::vector<int8_t> valid((size_t)np * ns, 0), klog((size_t)np * s->klog_cap, -2);
  std::vector<uint64_t> kh(np, 1469598103934665603ull);
  for (int p = 0; p < np; ++p) {
    valid[(size_t)p * ns] = 1;
    sticks[(size_t)p * ns] = tk0;
    stime[(size_t)p * ns] = t0;
  }
  int e = 0;
  auto cp = [&](void* d, const void* h, size_t b) {
    if (!e) e = hipck(hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, s->stream), "upload");
  };
  DevSet& D = s->D;
  cp(D.cur, cur.data(), sizeof(int) * np);
  cp(D.ticks, ticks.data(), sizeof(int64_t) * np);
  cp(D.tcur, tc.data(), sizeof(double) * np);
  cp(D.sticks, sticks.data(), sizeof(int64_t) * np * ns);
  cp(D.stime, stime.data(), sizeof(double) * np * ns);
  cp(D.svalid, valid.data(), (size_t)np * ns);
  cp(D.steps, zero64.data(), sizeof(int64_t) * np);
  cp(D.khash, kh.data(), sizeof(uint64_t) * np);
  cp(D.klog, klog.data(), (size_t)np * s->klog_cap);
  if (U) cp(s->d_hostbuf, U, sizeof(double) * n_values);
  if (e) return e;
  (void)hipMemsetAsync(s->d_err, 0, sizeof(int) * 2, s->stream);
  (void)hipMemsetAsync(s->d_cnt, 0, sizeof(unsigned long long) * 4, s->stream);
  if (s->poison) {  // checking switch: slots not yet written hold NaN
    if (s->f32)
      launch_poison<float>(D, (float*)s->slots, s->stream);
    else
      launch_poison<double>(D, (double*)s->slots, s->stream);
  }
  if (U) {
    if (s->f32)
      launch_scatter<float>(D, (float*)s->slots, s->d_hostbuf, s->d_host_off, s->stream);
    else
      launch_scatter<double>(D, (double*)s->slots, s->d_hostbuf, s->d_host_off, s->stream);
  } else {
    if (s->f32)
      launch_unpack<float>(D, (float*)s->slots, (const float*)U_dev, s->d_host_off, s->stream);
    else
      launch_unpack<double>(D, (double*)s->slots, (const double*)U_dev, s->d_host_off, s->stream);
  }
  e = hipck(hipStreamSynchronize(s->stream), "init");
  if (e) return e;
  s->initialised = true;
  s->rounds = 0;
  return 0;
}

static int read_err(dsp_set* s, int* counters_out, const int* counters = nullptr) {
  int hbuf[4] = {0, 0, 0, 0};
  int e = hipck(hipMemcpyAsync(hbuf, counters ? counters : s->d_counters, sizeof(int) * 2, hipMemcpyDeviceToHost,
                               s->stream),
                "readback");
  if (!e) e = hipck(hipMemcpyAsync(hbuf + 2, s->d_err, sizeof(int), hipMemcpyDeviceToHost, s->stream), "readback");
  if (!e) e = hipck(hipStreamSynchronize(s->stream), "round");
  if (e) return e;
  if (counters_out) {
    counters_out[0] = hbuf[0];
    counters_out[1] = hbuf[1];
  }
  return s->check_err(hbuf[2]);
}

static int end_time_ticks(dsp_set* s, double t_end, int64_t& T) {
  const double m = t_end / s->cfg.dt_base, mr = std::nearbyint(m);
  if (std::fabs(m - mr) > 1e-9 * std::max(1.0, std::fabs(m))) return fail(DSP_EALIGN, "end time is not a multiple of dt_base");
  if (mr < 0 || mr * std::ldexp(1.0, s->cfg.kmax) > 9.0e18) return fail(DSP_EINVAL, "end time out of range");
  T = (int64_t)mr << s->cfg.kmax;
  return 0;
}

// GLOBAL modes: every patch steps together; all patches form one batch.
static int run_global(dsp_set* s, double t_end, int64_t T, int max_steps) {
  std::vector<int> all(s->np);
  for (int p = 0; p < s->np; ++p) all[p] = p;
  int e = hipck(hipMemcpyAsync(s->d_list, all.data(), sizeof(int) * s->np, hipMemcpyHostToDevice, s->stream), "list");
  if (e) return e;
  int nstep = 0;
  while (true) {
    if (max_steps >= 0 && nstep >= max_steps) return 0;
    if (max_steps < 0) {
      if (s->D.exact_time) {
        double t0;
        e = hipck(hipMemcpy(&t0, s->D.tcur, sizeof(double), hipMemcpyDeviceToHost), "time");
        if (e) return e;
        if (!(t0 < t_end)) return 0;
      } else {
        int64_t tk;
        e = hipck(hipMemcpy(&tk, s->D.ticks, sizeof(int64_t), hipMemcpyDeviceToHost), "time");
        if (e) return e;
        if (tk >= T) return 0;
      }
    }
    s->update_batch(0, s->np, 1, t_end, max_steps < 0 ? 1 : 0, s->d_list);
    launch_publish(s->D, s->d_list, s->np, s->st, s->stream, s->slots);
    s->rounds++;
    nstep++;
    (void)hipMemsetAsync(s->d_counters, 0, sizeof(int) * 2, s->stream);
    // a fixed number of steps is queued whole; the error flags stay set, so
    // one check after the last step sees an error of any of them
    if (max_steps < 0 || nstep >= max_steps) {
      e = read_err(s, nullptr);
      if (e) return e;
    }
  }
}

// LOCAL rounds without a host round trip per round: chunks of rounds (scan,
// step, publish) are queued on the stream, every round kernel bounded by the
// ready-list length that the scan writes on the device; the host reads the
// counters and the error flags once per chunk.  Rounds queued after the last
// patch reached t_end find an empty ready list and do nothing.
constexpr int kRoundCap = 1024;

static int run_local_device(dsp_set* s, double t_end, int64_t T, int64_t& rounds_done) {
  const int K = 16;
  // two counter pairs, used by alternate rounds: each scan clears the pair
  // of the round after it, so no clearing operation runs between rounds
  int* const pair[2] = {s->d_counters + 4, s->d_counters + 6};
  int e = hipck(hipMemsetAsync(s->d_counters + 2, 0, sizeof(int) * 6, s->stream), "rounds");
  if (e) return e;
  s->D.rounds = s->d_counters + 2;
  // Without a grace, a round takes at most kRoundCap ready patches: its
  // kernels are then launched for that many entries, not for every patch of
  // a large set (whose surplus workgroups would only exit).  With a grace
  // the result depends on which patches share a round, so rounds stay whole.
  const char* cap_env = getenv("DSP_ROUND_CAP");  // a smaller cap (tests of the deferral)
  const int cap_max = cap_env ? std::max(1, atoi(cap_env)) : kRoundCap;
  const int cap = (s->cfg.grace == 0.0 && s->np > cap_max) ? cap_max : 0;
  const int count = cap ? cap : s->np;
  s->D.scan_cap = cap;
  while (!e) {
    for (int r = 0; r < K; ++r) {  // K is even: every chunk starts on pair 0
      int* const cur = pair[r & 1];
      s->D.live = cur;
      launch_scan(s->D, T, s->d_list, cur, s->stream, pair[(r + 1) & 1]);
      s->update_batch(0, count, 0, t_end, 0, s->d_list);
      launch_publish(s->D, s->d_list, count, s->st, s->stream, s->slots);
    }
    int cnt[2];
    e = read_err(s, cnt, pair[(K - 1) & 1]);
    if (e) break;
    if (cnt[1] == 0) break;
    if (cnt[0] == 0) e = fail(DSP_ESTATE, "no ready patch but not done");
  }
  s->D.live = nullptr;
  s->D.rounds = nullptr;
  s->D.scan_cap = 0;
  int r = 0;
  const int e2 = hipck(hipMemcpy(&r, s->d_counters + 2, sizeof(int), hipMemcpyDeviceToHost), "rounds");
  rounds_done = r;
  s->rounds += r;
  return e ? e : e2;
}

// LOCAL steps with the persistent dispatcher: one replay of the captured
// graph (queue reset and seed, the persistent kernel) on the set's graph
// stream, ordered after the set's stream.
static int run_queue(dsp_set* s, int64_t T) {
  int e = 0;
  if (!s->gstream) {
    // a stream of default priority of its own (capturable; ordered with the
    // set's stream by the synchronisations around each launch)
    e = hipck(hipStreamCreateWithFlags(&s->gstream, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    if (!e) e = hipck(hipEventCreate(&s->qev[0]), "hipEventCreate");
    if (!e) e = hipck(hipEventCreate(&s->qev[1]), "hipEventCreate");
    if (e) return e;
  }
  if (!s->gexec) {
    e = hipck(hipStreamBeginCapture(s->gstream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (e) return e;
    launch_queue_seed(s->D, s->Q, s->gstream);
    launch_persist(s->D, s->Q, (float*)s->slots, (float*)s->work_pad, s->pad_stride, s->st, s->workers, s->queue_fn,
                   s->nmax > MT, s->any_generic, s->gstream);
    e = hipck(hipStreamEndCapture(s->gstream, &s->graph), "hipStreamEndCapture");
    if (!e) e = hipck(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (e) return e;
  }
  e = hipck(hipStreamSynchronize(s->stream), "stream");  // the set's earlier work (init, counters)
  if (e) return e;
  *s->tend_host = T;
  e = hipck(hipMemcpyAsync((void*)s->Q.tend, s->tend_host, sizeof(int64_t), hipMemcpyHostToDevice, s->gstream),
            "end time");
  if (!e) e = hipck(hipEventRecord(s->qev[0], s->gstream), "event");
  if (!e) e = hipck(hipGraphLaunch(s->gexec, s->gstream), "hipGraphLaunch");
  if (!e) e = hipck(hipEventRecord(s->qev[1], s->gstream), "event");
  if (!e) e = hipck(hipStreamSynchronize(s->gstream), "persistent dispatcher");
  if (e) return e;
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, s->qev[0], s->qev[1]);
  s->kern_ms = ms;
  s->kern_launches = 1;
  s->dt_fused = 1;
  s->rounds += 1;
  return read_err(s, nullptr);
}

int dsp_advance_to(dsp_set* s, double t_end) {
  if (!s || !s->initialised) return fail(DSP_ESTATE, "set not initialised");
  auto w0 = std::chrono::steady_clock::now();
  s->begin_timing();
  int e;
  int64_t real_launches = -1;
  if (s->D.exact_time) {
    e = run_global(s, t_end, 0, -1);
  } else {
    int64_t T;
    e = end_time_ticks(s, t_end, T);
    if (e) return e;
    if (s->cfg.dt_mode == DSP_DT_GLOBAL_QUANT) {
      e = run_global(s, t_end, T, -1);
    } else if (s->queue_ok && s->dispatch == DSP_DISPATCH_QUEUE) {
      e = run_queue(s, T);
      s->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
      return e;
    } else if (s->fused && s->B >= s->np && !getenv("DSP_HOST_ROUNDS")) {
      int64_t done = 0;
      e = run_local_device(s, t_end, T, done);
      real_launches = done;
    } else {
      while (true) {
        launch_scan(s->D, T, s->d_list, s->d_counters, s->stream);
        int cnt[2];
        e = read_err(s, cnt);
        if (e) break;
        if (cnt[1] == 0) break;
        if (cnt[0] == 0) {
          e = fail(DSP_ESTATE, "no ready patch but not done");
          break;
        }
        for (int off = 0; off < cnt[0]; off += s->B)
          s->update_batch(off, std::min(s->B, cnt[0] - off), 0, t_end, 0, s->d_list);
        launch_publish(s->D, s->d_list, cnt[0], s->st, s->stream, s->slots);
        s->rounds++;
      }
    }
  }
  s->end_timing(real_launches);
  s->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
  return e;
}

int dsp_set_dispatch(dsp_set* s, int32_t mode, int32_t workers) {
  if (!s) return fail(DSP_EINVAL, "null handle");
  if (mode != DSP_DISPATCH_ROUNDS && mode != DSP_DISPATCH_QUEUE) return fail(DSP_EINVAL, "unknown dispatch mode");
  if (mode == DSP_DISPATCH_QUEUE && !s->queue_ok)
    return fail(DSP_EINVAL, "the queue dispatch needs a single-precision LOCAL set of patches of at most 16^3 "
                            "cells without a grace");
  if (workers < 0) return fail(DSP_EINVAL, "negative worker count");
  if (mode == DSP_DISPATCH_QUEUE) {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int cap = std::min(cus, std::min(s->np, s->B));
    const int w = workers == 0 ? cap : std::min(workers, cap);
    if (w != s->workers) {  // the captured graph holds the launch shape
      if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
      if (s->graph) (void)hipGraphDestroy(s->graph);
      s->gexec = nullptr;
      s->graph = nullptr;
      s->workers = w;
    }
  }
  s->dispatch = mode;
  return 0;
}

// The captured graph of the persistent dispatcher holds the set's description
// (kernel arguments): dropped when that changes, captured again on use.
static void drop_graph(dsp_set* s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->gexec = nullptr;
  s->graph = nullptr;
}

int dsp_set_output(dsp_set* s, double out_dt, void* frames_dev, int32_t nframes) {
  if (!s) return fail(DSP_EINVAL, "null handle");
  DevSet& D = s->D;
  if (!frames_dev || nframes <= 0) {
    D.out_frames = nullptr;
  } else {
    if (s->cfg.dt_mode != DSP_DT_LOCAL && s->cfg.dt_mode != DSP_DT_GLOBAL_QUANT)
      return fail(DSP_EINVAL, "an output cadence needs the quantised time steps (LOCAL or GLOBAL_QUANT)");
    // every patch lands on each multiple of dt_base (its step never crosses
    // a multiple of its own alignment), so a multiple of dt_base is met exactly
    int64_t m = 0;
    if (!(out_dt > 0.0) || !tolat(out_dt / s->cfg.dt_base, 1, m) || m < 1)
      return fail(DSP_EINVAL, "the output interval must be a positive multiple of dt_base");
    D.out_frames = frames_dev;
    D.out_ticks = m << s->cfg.kmax;
    D.out_nframes = nframes;
    D.out_frame_values = s->total_values;
  }
  drop_graph(s);
  return 0;
}

int dsp_get_dispatch(const dsp_set* s, int32_t* mode, int32_t* queue_available, int32_t* workers) {
  if (!s) return fail(DSP_EINVAL, "null handle");
  if (mode) *mode = s->dispatch;
  if (queue_available) *queue_available = s->queue_ok ? 1 : 0;
  if (workers) *workers = s->workers;
  return 0;
}

extern "C++" {
namespace {
// every device array that an advance changes, for the autotuner's save and restore
std::vector<std::pair<void*, size_t>> mutable_state(dsp_set* s) {
  const size_t np = (size_t)s->np, ns = (size_t)s->cfg.nslots, tsz = s->f32 ? 4 : 8;
  const DevSet& D = s->D;
  return {{s->slots, (size_t)s->total_values * ns * tsz},
          {D.cur, sizeof(int) * np},
          {D.ticks, sizeof(int64_t) * np},
          {D.tcur, sizeof(double) * np},
          {D.sticks, sizeof(int64_t) * np * ns},
          {D.stime, sizeof(double) * np * ns},
          {D.svalid, np * ns},
          {D.steps, sizeof(int64_t) * np},
          {D.khash, sizeof(uint64_t) * np},
          {D.klog, np * (size_t)s->klog_cap},
          {s->d_cnt, sizeof(unsigned long long) * 4},
          {s->d_err, sizeof(int) * 2}};
}

std::string tune_key(const dsp_set* s) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  std::string name = "gpu";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) name = prop.gcnArchName;
  char buf[256];
  snprintf(buf, sizeof(buf), "%s np=%d n=%d..%d prec=%d resampled=%d", name.c_str(), s->np, s->nmin, s->nmax,
           (int)s->cfg.prec, s->any_generic ? 1 : 0);
  return buf;
}
}  // namespace
}  // extern "C++"

int dsp_autotune(dsp_set* s, double t_probe, const char* cache_path, double* ms_out) {
  if (!s || !s->initialised) return fail(DSP_ESTATE, "set not initialised");
  if (s->cfg.dt_mode != DSP_DT_LOCAL) return fail(DSP_EINVAL, "the autotuner covers LOCAL steps");
  if (ms_out)
    for (int m = 0; m < 4; ++m) ms_out[m] = -1.0;
  const std::string key = tune_key(s);
  // candidates: rounds, then the queue with 1, 3/4 and 1/2 of its workgroups
  int cus = 0, dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int wmax = std::min(cus, std::min(s->np, s->B));
  const int cand_mode[4] = {DSP_DISPATCH_ROUNDS, DSP_DISPATCH_QUEUE, DSP_DISPATCH_QUEUE, DSP_DISPATCH_QUEUE};
  const int cand_w[4] = {0, wmax, std::max(1, wmax * 3 / 4), std::max(1, wmax / 2)};
  const int ncand = s->queue_ok ? 4 : 1;
  // a cached choice for this key
  if (cache_path) {
    FILE* f = fopen(cache_path, "r");
    if (f) {
      char line[1024];
      int mode = -1, workers = 0;
      while (fgets(line, sizeof(line), f)) {
        const std::string l(line);
        if (l.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
        const size_t a = l.find("\"dispatch\": "), b = l.find("\"workers\": ");
        if (a != std::string::npos && b != std::string::npos) {
          mode = atoi(line + a + 12);
          workers = atoi(line + b + 11);
        }
      }
      fclose(f);
      if (mode == DSP_DISPATCH_ROUNDS || (mode == DSP_DISPATCH_QUEUE && s->queue_ok))
        return dsp_set_dispatch(s, mode, workers);
    }
  }
  // the probe window from the set's current time
  std::vector<double> tc(s->np);
  int e = hipck(hipMemcpy(tc.data(), s->D.tcur, sizeof(double) * s->np, hipMemcpyDeviceToHost), "time");
  if (e) return e;
  const double t0 = *std::min_element(tc.begin(), tc.end());
  // no output from the probe runs
  void* const out0 = s->D.out_frames;
  if (out0) {
    s->D.out_frames = nullptr;
    drop_graph(s);
  }
  // save the state
  std::vector<std::pair<void*, size_t>> items = mutable_state(s);
  std::vector<void*> saved(items.size(), nullptr);
  for (size_t m = 0; m < items.size() && !e; ++m) {
    e = hipck(hipMalloc(&saved[m], items[m].second), "hipMalloc");
    if (!e) e = hipck(hipMemcpy(saved[m], items[m].first, items[m].second, hipMemcpyDeviceToDevice), "save");
  }
  const int64_t rounds0 = s->rounds;
  const int mode0 = s->dispatch, workers0 = s->workers;
  double best = 1e300;
  int bi = 0;
  for (int c = 0; c < ncand && !e; ++c) {
    e = dsp_set_dispatch(s, cand_mode[c], cand_w[c]);
    if (e) break;
    double ms = 0.0;
    for (int rep = 0; rep < 2 && !e; ++rep) {  // the first run also captures the graph
      for (size_t m = 0; m < items.size() && !e; ++m)
        e = hipck(hipMemcpy(items[m].first, saved[m], items[m].second, hipMemcpyDeviceToDevice), "restore");
      if (e) break;
      e = hipck(hipDeviceSynchronize(), "restore");
      const auto w0 = std::chrono::steady_clock::now();
      if (!e) e = dsp_advance_to(s, t0 + t_probe);
      ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
    }
    if (e) break;
    if (ms_out) ms_out[c] = ms;
    if (ms < best) {
      best = ms;
      bi = c;
    }
  }
  // restore the state and choose
  for (size_t m = 0; m < items.size(); ++m) {
    if (saved[m] && !e) e = hipck(hipMemcpy(items[m].first, saved[m], items[m].second, hipMemcpyDeviceToDevice), "restore");
    if (saved[m]) (void)hipFree(saved[m]);
  }
  s->rounds = rounds0;
  if (out0) {
    s->D.out_frames = out0;
    drop_graph(s);
  }
  if (e) {
    (void)dsp_set_dispatch(s, mode0, workers0);
    return e;
  }
  e = dsp_set_dispatch(s, cand_mode[bi], cand_w[bi]);
  if (e) return e;
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "{\"key\": \"%s\", \"dispatch\": %d, \"workers\": %d, \"ms\": %.4f}\n", key.c_str(), cand_mode[bi],
              cand_mode[bi] == DSP_DISPATCH_QUEUE ? s->workers : 0, best);
      fclose(f);
    }
  }
  return 0;
}

int dsp_advance_to_plain(dsp_set* s, double t_end) {
  if (!s || !s->initialised) return fail(DSP_ESTATE, "set not initialised");
  if (s->cfg.dt_mode != DSP_DT_LOCAL) return dsp_advance_to(s, t_end);
  int64_t T;
  int e = end_time_ticks(s, t_end, T);
  if (e) return e;
  auto w0 = std::chrono::steady_clock::now();
  s->begin_timing();
  const int np = s->np, ns = s->cfg.nslots;
  // host copy of the time bookkeeping, kept in step with the publish kernel
  std::vector<int64_t> ticks(np), sticks((size_t)np * ns), steps(np);
  std::vector<int> cur(np);
  std::vector<int8_t> valid((size_t)np * ns);
  auto get = [&](void* h, const void* d, size_t b) {
    if (!e) e = hipck(hipMemcpy(h, d, b, hipMemcpyDeviceToHost), "ticks");
  };
  get(ticks.data(), s->D.ticks, sizeof(int64_t) * np);
  get(sticks.data(), s->D.sticks, sizeof(int64_t) * np * ns);
  get(steps.data(), s->D.steps, sizeof(int64_t) * np);
  get(cur.data(), s->D.cur, sizeof(int) * np);
  get(valid.data(), s->D.svalid, (size_t)np * ns);
  // readiness as in the scan kernel: Eq. (1) with the grace, and a free slot
  auto ready = [&](int p) {
    if (s->P[p].frozen) return false;
    const size_t ob = (size_t)p * ns;
    const int oldest = (cur[p] + 1) % ns, after = (cur[p] + 1 + (s->cfg.torder > 1 ? 2 : 1)) % ns;
    const int64_t t_after = valid[ob + oldest] ? sticks[ob + after] : INT64_MIN;
    for (int q : s->nbors[p]) {
      if (s->P[q].frozen) continue;
      int64_t g = 0;
      if (s->cfg.grace > 0.0 && steps[q] > 0) {
        const int prev = (cur[q] + ns - 1) % ns;
        if (valid[(size_t)q * ns + prev])
          g = (int64_t)std::floor(s->cfg.grace * (double)(ticks[q] - sticks[(size_t)q * ns + prev]));
      }
      if (ticks[p] > ticks[q] + g || t_after > ticks[q]) return false;
    }
    return true;
  };
  while (!e) {
    // oldest ready patch, ties by id (Sec. 3B mode (i))
    int best = -1;
    bool done = true;
    for (int p = 0; p < np; ++p) {
      if (s->P[p].frozen || ticks[p] >= T) continue;
      done = false;
      if (ready(p) && (best < 0 || ticks[p] < ticks[best])) best = p;
    }
    if (done) break;
    if (best < 0) { e = fail(DSP_ESTATE, "no ready patch but not done"); break; }
    e = hipck(hipMemcpyAsync(s->d_single, &best, sizeof(int), hipMemcpyHostToDevice, s->stream), "list");
    if (e) break;
    s->update_batch(0, 1, 0, t_end, 0, s->d_single);
    launch_publish(s->D, s->d_single, 1, s->st, s->stream, s->slots);
    s->rounds++;
    int64_t dtk = 0;
    e = hipck(hipMemcpyAsync(&dtk, s->st.dtk, sizeof(int64_t), hipMemcpyDeviceToHost, s->stream), "dt");
    if (e) break;
    e = read_err(s, nullptr);
    if (e) break;
    ticks[best] += dtk;
    cur[best] = (cur[best] + 1) % ns;
    sticks[(size_t)best * ns + cur[best]] = ticks[best];
    valid[(size_t)best * ns + cur[best]] = 1;
    steps[best]++;
  }
  s->end_timing();
  s->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
  return e;
}

int dsp_read_state(const dsp_set* cs, double* U, size_t n_values, double* t_out) {
  dsp_set* s = const_cast<dsp_set*>(cs);
  if (!s || !U || !s->initialised) return fail(DSP_EINVAL, "bad argument");
  if ((int64_t)n_values < s->total_values) return fail(DSP_EINVAL, "output buffer too small");
  if (s->f32)
    launch_gather<float>(s->D, (const float*)s->slots, s->d_hostbuf, s->d_host_off, s->stream);
  else
    launch_gather<double>(s->D, (const double*)s->slots, s->d_hostbuf, s->d_host_off, s->stream);
  int e = hipck(hipMemcpyAsync(U, s->d_hostbuf, sizeof(double) * s->total_values, hipMemcpyDeviceToHost, s->stream),
                "download");
  if (!e) e = hipck(hipStreamSynchronize(s->stream), "download");
  if (e) return e;
  if (t_out) {
    std::vector<double> tc(s->np);
    e = hipck(hipMemcpy(tc.data(), s->D.tcur, sizeof(double) * s->np, hipMemcpyDeviceToHost), "time");
    if (e) return e;
    *t_out = *std::min_element(tc.begin(), tc.end());
  }
  return 0;
}

int dsp_read_schedule(const dsp_set* s, int64_t* steps, uint64_t* khash, int32_t* klog, size_t klog_cap) {
  if (!s) return fail(DSP_EINVAL, "null handle");
  const int np = s->np;
  int e = 0;
  if (steps) e = hipck(hipMemcpy(steps, s->D.steps, sizeof(int64_t) * np, hipMemcpyDeviceToHost), "steps");
  if (!e && khash) e = hipck(hipMemcpy(khash, s->D.khash, sizeof(uint64_t) * np, hipMemcpyDeviceToHost), "khash");
  if (!e && klog) {
    std::vector<int8_t> kl((size_t)np * s->klog_cap);
    e = hipck(hipMemcpy(kl.data(), s->D.klog, kl.size(), hipMemcpyDeviceToHost), "klog");
    for (int p = 0; p < np && !e; ++p)
      for (size_t m = 0; m < klog_cap; ++m)
        klog[(size_t)p * klog_cap + m] = m < (size_t)s->klog_cap ? kl[(size_t)p * s->klog_cap + m] : -2;
  }
  return e;
}

int dsp_stats(const dsp_set* cs, double out[16]) {
  dsp_set* s = const_cast<dsp_set*>(cs);
  if (!s || !out) return fail(DSP_EINVAL, "null argument");
  for (int m = 0; m < 16; ++m) out[m] = 0.0;
  if (!s->initialised) return fail(DSP_ESTATE, "set not initialised");
  if (s->f32)
    launch_stats<float>(s->D, (const float*)s->slots, s->d_stats, s->stream);
  else
    launch_stats<double>(s->D, (const double*)s->slots, s->d_stats, s->stream);
  std::vector<double> ps((size_t)9 * s->np), tc(s->np);
  unsigned long long cnt[3];
  int e = hipck(hipMemcpyAsync(ps.data(), s->d_stats, sizeof(double) * ps.size(), hipMemcpyDeviceToHost, s->stream), "stats");
  if (!e) e = hipck(hipMemcpyAsync(cnt, s->d_cnt, sizeof(cnt), hipMemcpyDeviceToHost, s->stream), "stats");
  if (!e) e = hipck(hipMemcpyAsync(tc.data(), s->D.tcur, sizeof(double) * s->np, hipMemcpyDeviceToHost, s->stream), "stats");
  if (!e) e = hipck(hipStreamSynchronize(s->stream), "stats");
  if (e) return e;
  double dmax = 0.0;
  for (int p = 0; p < s->np; ++p) {
    for (int q = 0; q < 8; ++q) out[1 + q] += ps[(size_t)p * 9 + q];
    dmax = std::max(dmax, ps[(size_t)p * 9 + 8]);
  }
  out[0] = (double)cnt[2];
  out[9] = dmax;
  out[10] = (double)cnt[0];
  out[11] = (double)cnt[1];
  out[12] = s->last_ms;
  out[13] = (double)s->rounds;
  // times of the updated patches (boundary patches stay at t0)
  double tmin = INFINITY, tmax = -INFINITY;
  for (int p = 0; p < s->np; ++p)
    if (!s->P[p].frozen) {
      tmin = std::min(tmin, tc[p]);
      tmax = std::max(tmax, tc[p]);
    }
  out[14] = tmin;
  out[15] = tmax;
  return 0;
}

int dsp_kernel_stats(const dsp_set* cs, double out[4]) {
  dsp_set* s = const_cast<dsp_set*>(cs);
  if (!s || !out) return fail(DSP_EINVAL, "null argument");
  unsigned long long cnt[4];
  int e = hipck(hipMemcpy(cnt, s->d_cnt, sizeof(cnt), hipMemcpyDeviceToHost), "stats");
  if (e) return e;
  out[0] = s->kern_ms;
  out[1] = (double)s->kern_launches;
  out[2] = s->fused ? (double)cnt[3] : 0.0;
  out[3] = s->fused ? (s->dt_fused ? 2.0 : 1.0) : 0.0;
  return 0;
}

int dsp_kernel_time(const dsp_set* s, double* ms, int64_t* launches) {
  if (!s) return fail(DSP_EINVAL, "null handle");
  if (ms) *ms = s->kern_ms;
  if (launches) *launches = s->kern_launches;
  return 0;
}

// Fixed steps: every patch at t = 0 with the given state (device, host
// layout) in slot 0, schedule record, counters and error flags cleared.
static int reset_fixed(dsp_set* s, const void* U_dev) { return init_common(s, nullptr, U_dev, 0.0); }

extern "C++" {
// One fixed step with the staged kernels from state U_in, leaving every
// intermediate in the adjoint's work buffers; U_out (nullable) receives the
// new state.
template <class T> static int staged_fixed_step(dsp_set* s, const T* U_in, T* U_out, int copy) {
  // queued on the stream without a host round trip: time records reset on
  // the device, the state unpacked from U_in; errors stay flagged until the
  // caller reads them
  launch_reset_times(s->D, s->d_cnt, s->stream);
  launch_unpack<T>(s->D, (T*)s->slots, U_in, s->d_host_off, s->stream);
  launch_update<T>(s->D, s->d_list, s->np, s->nmax, (T*)s->slots, s->adj_work<T>(false, copy), s->st, s->stream, 1,
                   0.0, 0, nullptr, nullptr);
  if (U_out) {
    launch_publish(s->D, s->d_list, s->np, s->st, s->stream);
    launch_pack<T>(s->D, (const T*)s->slots, U_out, s->d_host_off, s->stream);
  }
  return 0;
}

template <class T>
static int adjoint_run(dsp_set* s, const T* ckpt, const T* lamT, T* lam0, int nsteps) {
  const size_t V = (size_t)s->total_values;
  std::vector<int> all(s->np);
  for (int p = 0; p < s->np; ++p) all[p] = p;
  int e = hipck(hipMemcpyAsync(s->d_list, all.data(), sizeof(int) * s->np, hipMemcpyHostToDevice, s->stream), "list");
  if (e) return e;
  T* states = (T*)s->adj_states;
  T* la = (T*)s->adj_la;
  T* lb = (T*)s->adj_lb;
  e = hipck(hipMemcpyAsync(la, lamT, sizeof(T) * V, hipMemcpyDeviceToDevice, s->stream), "adjoint");
  if (!e) e = hipck(hipMemsetAsync(s->d_err, 0, sizeof(int) * 2, s->stream), "adjoint");
  const WorkPtr<T> L = s->adj_work<T>(true);
  // with a set of work buffers per step, the segment's forward pass keeps
  // every step's intermediates and the reverse pass uses them directly
  const bool keep = s->adj_copies >= 8;
  const int nseg = (nsteps + 7) / 8;
  for (int seg = nseg - 1; seg >= 0 && !e; --seg) {
    const int len = std::min(8, nsteps - 8 * seg);
    e = hipck(hipMemcpyAsync(states, ckpt + (size_t)seg * V, sizeof(T) * V, hipMemcpyDeviceToDevice, s->stream),
              "adjoint");
    const int nfwd = keep ? len : len - 1;  // steps j < nfwd run forward here (into set j when kept)
    for (int j = 0; j < nfwd && !e; ++j)
      e = staged_fixed_step<T>(s, states + (size_t)j * V, j + 1 < len ? states + (size_t)(j + 1) * V : (T*)nullptr,
                               keep ? j : 0);
    for (int j = len - 1; j >= 0 && !e; --j) {
      if (!keep) e = staged_fixed_step<T>(s, states + (size_t)j * V, (T*)nullptr, 0);
      if (e) break;
      const WorkPtr<T> W = s->adj_work<T>(false, keep ? j : 0);
      // padded state, primitives and half-step state take accumulated
      // cotangents; the slope, flux and edge buffers are written whole by
      // their first writer in the step (k_adj_flux_sum, k_adj_update), and
      // lam^k whole by the gathered guard fill
      for (int q = 0; q < 3; ++q) {
        const int64_t sizes[3] = {s->pad_stride, s->w_stride, s->w_stride};
        (void)hipMemsetAsync(s->adj_l[q], 0, sizeof(T) * (size_t)sizes[q] * s->np, s->stream);
      }
      launch_adjoint_step<T>(s->D, s->d_list, s->np, s->nmax, W, L, s->st, la, lb, s->d_host_off, s->stream);
      std::swap(la, lb);
    }
    if (!e) e = read_err(s, nullptr);  // once per segment: the error flags stick
  }
  if (!e) e = hipck(hipMemcpyAsync(lam0, la, sizeof(T) * V, hipMemcpyDeviceToDevice, s->stream), "adjoint");
  if (!e) e = hipck(hipStreamSynchronize(s->stream), "adjoint");
  return e;
}
}  // extern "C++"

int dsp_fixed_steps_fwd(dsp_set* s, const void* U0_dev, void* UT_dev, int32_t nsteps, void* ckpt_dev) {
  if (!s || !U0_dev || !UT_dev || nsteps < 0) return fail(DSP_EINVAL, "bad argument");
  if (s->cfg.dt_mode != DSP_DT_FIXED) return fail(DSP_EINVAL, "fixed steps need the FIXED dt mode");
  int e = reset_fixed(s, U0_dev);
  if (e) return e;
  const size_t tsz = s->f32 ? 4 : 8;
  s->begin_timing();
  for (int m = 0; m < nsteps && !e; m += 8) {
    if (ckpt_dev) {
      char* dst = (char*)ckpt_dev + (size_t)(m / 8) * s->total_values * tsz;
      if (s->f32)
        launch_pack<float>(s->D, (const float*)s->slots, (float*)dst, s->d_host_off, s->stream);
      else
        launch_pack<double>(s->D, (const double*)s->slots, (double*)dst, s->d_host_off, s->stream);
    }
    e = run_global(s, 0.0, 0, std::min(8, nsteps - m));
  }
  if (e) return e;
  if (ckpt_dev && nsteps % 8 == 0) {
    char* dst = (char*)ckpt_dev + (size_t)(nsteps / 8) * s->total_values * tsz;
    if (s->f32)
      launch_pack<float>(s->D, (const float*)s->slots, (float*)dst, s->d_host_off, s->stream);
    else
      launch_pack<double>(s->D, (const double*)s->slots, (double*)dst, s->d_host_off, s->stream);
  }
  if (s->f32)
    launch_pack<float>(s->D, (const float*)s->slots, (float*)UT_dev, s->d_host_off, s->stream);
  else
    launch_pack<double>(s->D, (const double*)s->slots, (double*)UT_dev, s->d_host_off, s->stream);
  s->end_timing();
  return hipck(hipStreamSynchronize(s->stream), "fixed steps");
}

int dsp_fixed_steps_adj(dsp_set* s, const void* ckpt_dev, const void* lamT_dev, void* lam0_dev, int32_t nsteps,
                        int32_t seg) {
  if (!s || !ckpt_dev || !lamT_dev || !lam0_dev || nsteps < 0) return fail(DSP_EINVAL, "bad argument");
  if (s->cfg.dt_mode != DSP_DT_FIXED) return fail(DSP_EINVAL, "the adjoint needs the FIXED dt mode");
  if (s->D.nonideal) return fail(DSP_EINVAL, "the adjoint covers ideal MHD only");
  if (seg != 8) return fail(DSP_EINVAL, "checkpoint segments are 8 steps");
  if (s->any_generic)
    return fail(DSP_EINVAL, "the adjoint covers sets whose guard regions are same-resolution copies");
  int e = s->adj_prepare();
  if (e) return fail(DSP_ENOMEM, "device allocation failed: " + s->alloc_msg);
  if (s->f32)
    e = adjoint_run<float>(s, (const float*)ckpt_dev, (const float*)lamT_dev, (float*)lam0_dev, nsteps);
  else
    e = adjoint_run<double>(s, (const double*)ckpt_dev, (const double*)lamT_dev, (double*)lam0_dev, nsteps);
  return e;
}

// ---------------------------------------------------------------------------
// Snapshot files (restart).  The whole device state of the set: every ring
// slot with its time, the patch times and the schedule record, so that a run
// restarted from the file continues exactly as the uninterrupted run.

static const char kSnapMagic[8] = {'D', 'S', 'P', 'S', 'N', 'A', 'P', '1'};

struct SnapHost {
  std::vector<int> cur;
  std::vector<int64_t> ticks, sticks, steps;
  std::vector<double> tcur, stime;
  std::vector<int8_t> svalid, klog;
  std::vector<uint64_t> khash;
  std::vector<char> slots;
  void size_for(const dsp_set* s) {
    const size_t np = (size_t)s->np, ns = (size_t)s->cfg.nslots;
    cur.resize(np);
    ticks.resize(np);
    steps.resize(np);
    tcur.resize(np);
    khash.resize(np);
    sticks.resize(np * ns);
    stime.resize(np * ns);
    svalid.resize(np * ns);
    klog.resize(np * (size_t)s->klog_cap);
    slots.resize((size_t)s->total_values * ns * (s->f32 ? 4 : 8));
  }
};

int dsp_save_snapshot(const dsp_set* s, const char* path) {
  if (!s || !path) return fail(DSP_EINVAL, "null argument");
  if (!s->initialised) return fail(DSP_ESTATE, "set not initialised");
  SnapHost h;
  h.size_for(s);
  const size_t np = (size_t)s->np, ns = (size_t)s->cfg.nslots;
  const DevSet& D = s->D;
  int e = 0;
  auto get = [&](void* dst, const void* src, size_t b) {
    if (!e) e = hipck(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToHost, s->stream), "snapshot");
  };
  get(h.cur.data(), D.cur, sizeof(int) * np);
  get(h.ticks.data(), D.ticks, sizeof(int64_t) * np);
  get(h.tcur.data(), D.tcur, sizeof(double) * np);
  get(h.sticks.data(), D.sticks, sizeof(int64_t) * np * ns);
  get(h.stime.data(), D.stime, sizeof(double) * np * ns);
  get(h.svalid.data(), D.svalid, np * ns);
  get(h.steps.data(), D.steps, sizeof(int64_t) * np);
  get(h.khash.data(), D.khash, sizeof(uint64_t) * np);
  get(h.klog.data(), D.klog, h.klog.size());
  get(h.slots.data(), s->slots, h.slots.size());
  if (!e) e = hipck(hipStreamSynchronize(s->stream), "snapshot");
  if (e) return e;
  FILE* f = fopen(path, "wb");
  if (!f) return fail(DSP_EINVAL, std::string("cannot write ") + path);
  bool ok = true;
  auto put = [&](const void* p, size_t b) { ok = ok && fwrite(p, 1, b, f) == b; };
  const int32_t hdr[5] = {(int32_t)np, (int32_t)ns, (int32_t)s->cfg.prec, s->cfg.kmax, s->klog_cap};
  put(kSnapMagic, 8);
  put(hdr, sizeof(hdr));
  put(&s->cfg.dt_base, sizeof(double));
  const size_t tsz = s->f32 ? 4 : 8;
  for (size_t p = 0; p < np && ok; ++p) {
    const int32_t nl[2] = {s->P[p].n, s->P[p].level};
    put(nl, sizeof(nl));
    put(&h.ticks[p], 8);
    put(&h.tcur[p], 8);
    put(&h.cur[p], 4);
    put(&h.steps[p], 8);
    put(&h.khash[p], 8);
    for (size_t q = 0; q < ns; ++q) {
      put(&h.sticks[p * ns + q], 8);
      put(&h.stime[p * ns + q], 8);
      put(&h.svalid[p * ns + q], 1);
    }
    put(&h.klog[p * (size_t)s->klog_cap], (size_t)s->klog_cap);
    put(h.slots.data() + (size_t)s->P[p].slot_off * tsz, (size_t)s->P[p].V * ns * tsz);
  }
  ok = (fclose(f) == 0) && ok;
  return ok ? 0 : fail(DSP_EINVAL, std::string("write failed: ") + path);
}

int dsp_load_snapshot(dsp_set* s, const char* path) {
  if (!s || !path) return fail(DSP_EINVAL, "null argument");
  FILE* f = fopen(path, "rb");
  if (!f) return fail(DSP_EINVAL, std::string("cannot read ") + path);
  bool ok = true;
  auto take = [&](void* p, size_t b) { ok = ok && fread(p, 1, b, f) == b; };
  char magic[8];
  int32_t hdr[5];
  double dtb = 0.0;
  take(magic, 8);
  take(hdr, sizeof(hdr));
  take(&dtb, sizeof(double));
  const size_t np = (size_t)s->np, ns = (size_t)s->cfg.nslots;
  if (!ok || memcmp(magic, kSnapMagic, 8) != 0) {
    fclose(f);
    return fail(DSP_EINVAL, "not a snapshot file");
  }
  if (hdr[0] != (int32_t)np || hdr[1] != (int32_t)ns || hdr[2] != (int32_t)s->cfg.prec || hdr[3] != s->cfg.kmax ||
      hdr[4] != s->klog_cap || dtb != s->cfg.dt_base) {
    fclose(f);
    return fail(DSP_EINVAL, "snapshot does not match the set (patches, slots, precision, kmax or dt_base)");
  }
  SnapHost h;
  h.size_for(s);
  const size_t tsz = s->f32 ? 4 : 8;
  for (size_t p = 0; p < np && ok; ++p) {
    int32_t nl[2];
    take(nl, sizeof(nl));
    if (ok && (nl[0] != s->P[p].n || nl[1] != s->P[p].level)) {
      fclose(f);
      return fail(DSP_EINVAL, "snapshot does not match the set's patches");
    }
    take(&h.ticks[p], 8);
    take(&h.tcur[p], 8);
    take(&h.cur[p], 4);
    take(&h.steps[p], 8);
    take(&h.khash[p], 8);
    for (size_t q = 0; q < ns; ++q) {
      take(&h.sticks[p * ns + q], 8);
      take(&h.stime[p * ns + q], 8);
      take(&h.svalid[p * ns + q], 1);
    }
    take(&h.klog[p * (size_t)s->klog_cap], (size_t)s->klog_cap);
    take(h.slots.data() + (size_t)s->P[p].slot_off * tsz, (size_t)s->P[p].V * ns * tsz);
    if (ok && (h.cur[p] < 0 || h.cur[p] >= (int)ns)) ok = false;
  }
  fclose(f);
  if (!ok) return fail(DSP_EINVAL, "truncated or corrupt snapshot");
  DevSet& D = s->D;
  int e = 0;
  auto cp = [&](void* dst, const void* src, size_t b) {
    if (!e) e = hipck(hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, s->stream), "snapshot");
  };
  cp(D.cur, h.cur.data(), sizeof(int) * np);
  cp(D.ticks, h.ticks.data(), sizeof(int64_t) * np);
  cp(D.tcur, h.tcur.data(), sizeof(double) * np);
  cp(D.sticks, h.sticks.data(), sizeof(int64_t) * np * ns);
  cp(D.stime, h.stime.data(), sizeof(double) * np * ns);
  cp(D.svalid, h.svalid.data(), np * ns);
  cp(D.steps, h.steps.data(), sizeof(int64_t) * np);
  cp(D.khash, h.khash.data(), sizeof(uint64_t) * np);
  cp(D.klog, h.klog.data(), h.klog.size());
  cp(s->slots, h.slots.data(), h.slots.size());
  if (!e) e = hipck(hipMemsetAsync(s->d_err, 0, sizeof(int) * 2, s->stream), "snapshot");
  if (!e) e = hipck(hipMemsetAsync(s->d_cnt, 0, sizeof(unsigned long long) * 4, s->stream), "snapshot");
  if (!e) e = hipck(hipStreamSynchronize(s->stream), "snapshot");
  if (e) return e;
  s->initialised = true;
  s->rounds = 0;
  return 0;
}

// HLLD flux of a batch of independent faces, with the step kernels' own
// arithmetic in the requested precision (a check of the flux on its own).
int dsp_hlld_faces(int32_t prec, const double* wl, const double* wr, const double* bn, int64_t nface, double gamma,
                   double* flux8) {
  if (prec != DSP_F32 && prec != DSP_F64) return fail(DSP_EINVAL, "invalid precision");
  if (nface < 0 || (nface > 0 && (!wl || !wr || !bn || !flux8))) return fail(DSP_EINVAL, "bad argument");
  if (!(gamma > 1.0)) return fail(DSP_EINVAL, "gamma must exceed 1");
  if (nface == 0) return 0;
  const size_t nw = sizeof(double) * 7 * (size_t)nface, nb = sizeof(double) * (size_t)nface,
               nf = sizeof(double) * 8 * (size_t)nface;
  double *dl = nullptr, *dr = nullptr, *db = nullptr, *df = nullptr;
  int e = hipck(hipMalloc(&dl, nw), "hipMalloc");
  if (!e) e = hipck(hipMalloc(&dr, nw), "hipMalloc");
  if (!e) e = hipck(hipMalloc(&db, nb), "hipMalloc");
  if (!e) e = hipck(hipMalloc(&df, nf), "hipMalloc");
  if (!e) e = hipck(hipMemcpy(dl, wl, nw, hipMemcpyHostToDevice), "upload");
  if (!e) e = hipck(hipMemcpy(dr, wr, nw, hipMemcpyHostToDevice), "upload");
  if (!e) e = hipck(hipMemcpy(db, bn, nb, hipMemcpyHostToDevice), "upload");
  if (!e) {
    (void)hipGetLastError();  // clear an error left by an earlier call, so the check below is this launch's
    if (prec == DSP_F32)
      launch_hlld_faces<float>(dl, dr, db, nface, gamma, df, nullptr);
    else
      launch_hlld_faces<double>(dl, dr, db, nface, gamma, df, nullptr);
    e = hipck(hipGetLastError(), "launch");
  }
  if (!e) e = hipck(hipMemcpy(flux8, df, nf, hipMemcpyDeviceToHost), "download");
  for (double* q : {dl, dr, db, df})
    if (q) (void)hipFree(q);
  return e;
}

// ---------------------------------------------------------------------------
// The face-flux check without allocation: the staging of the inputs and
// outputs lives in a file-scope device array (each GPU holds its own copy
// until the process ends).  Host code never passes the array's name to a
// kernel or a copy: its device address is taken once per device with
// hipGetSymbolAddress and kept.

namespace {
constexpr int64_t kScratchFaces = 65536;   // largest batch of dsp_hlld_faces_noalloc
constexpr int64_t kScratchPerFace = 7 + 7 + 1 + 8;  // wl, wr, bn, flux8
__device__ __align__(256) double scratch[kScratchFaces * kScratchPerFace];  // 12 MiB per GPU
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;  // device ordinal -> device address of that GPU's scratch

int scratch_address(double** out) {
  int dev = -1;
  int e = hipck(hipGetDevice(&dev), "hipGetDevice");
  if (e) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    e = hipck(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (e) return e;
    if (!p) return fail(DSP_EHIP, "hipGetSymbolAddress returned no address");
    it = g_scratch_ptr.emplace(dev, (double*)p).first;
  }
  *out = it->second;
  return 0;
}
}  // namespace

int dsp_hlld_faces_noalloc(int32_t prec, const double* wl, const double* wr, const double* bn, int64_t nface,
                           double gamma, double* flux8) {
  if (prec != DSP_F32 && prec != DSP_F64) return fail(DSP_EINVAL, "invalid precision");
  if (nface < 0 || (nface > 0 && (!wl || !wr || !bn || !flux8))) return fail(DSP_EINVAL, "bad argument");
  if (nface > kScratchFaces)
    return fail(DSP_EINVAL, "at most " + std::to_string(kScratchFaces) + " faces per call without allocation");
  if (!(gamma > 1.0)) return fail(DSP_EINVAL, "gamma must exceed 1");
  double* base = nullptr;
  int e = scratch_address(&base);
  if (e || nface == 0) return e;
  // the batch is packed at the start of the array; nothing in it needs to
  // start at zero (every value the kernel reads is copied in first)
  double* dl = base;
  double* dr = dl + 7 * nface;
  double* db = dr + 7 * nface;
  double* df = db + nface;
  const size_t nw = sizeof(double) * 7 * (size_t)nface, nb = sizeof(double) * (size_t)nface,
               nf = sizeof(double) * 8 * (size_t)nface;
  e = hipck(hipMemcpy(dl, wl, nw, hipMemcpyHostToDevice), "upload");
  if (!e) e = hipck(hipMemcpy(dr, wr, nw, hipMemcpyHostToDevice), "upload");
  if (!e) e = hipck(hipMemcpy(db, bn, nb, hipMemcpyHostToDevice), "upload");
  if (!e) {
    (void)hipGetLastError();  // clear an error left by an earlier call, so the check below is this launch's
    if (prec == DSP_F32)
      launch_hlld_faces<float>(dl, dr, db, nface, gamma, df, nullptr);
    else
      launch_hlld_faces<double>(dl, dr, db, nface, gamma, df, nullptr);
    e = hipck(hipGetLastError(), "launch");
  }
  if (!e) e = hipck(hipMemcpy(flux8, df, nf, hipMemcpyDeviceToHost), "download");
  return e;
}

void dsp_destroy(dsp_set* s) { delete s; }

}  // extern "C"
