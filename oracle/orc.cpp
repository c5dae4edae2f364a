// orc.cpp -- patch set, guard fill, time stepping and dispatcher of the CPU
// oracle.  TEST INFRASTRUCTURE ONLY (see orc.h): used by the tests, the smoke
// check and the CPU-baseline leg of the benchmark, never by the GPU library.
//
// The framework method follows the paper:
//  * a patch task keeps its state in a ring of time slices (Sec. 3A);
//  * before an update its guard zones are filled from the neighbouring
//    patches, interpolating linearly in time between the two slices that
//    bracket the patch time (Sec. 3A, Sec. 3B "Defining task readiness"),
//    or extrapolating linearly from a neighbour's two newest slices when
//    the grace of Eq. (1) lets the task run ahead of it;
//  * a task is ready when no neighbour lags behind it by more than the
//    grace g times the neighbour's step, Eq. (1) (Sec. 3B), and its ring has
//    a slice that no neighbour still needs;
//  * the task list executes ready tasks, oldest first, until every task
//    reaches the final time (Sec. 2.2, Sec. 3B mode (i));
//  * the new slice overwrites the oldest one and the task waits again.
// Each patch takes its own Courant step, quantised to dt_base * 2^-k (local
// time steps, Sec. 1 and Sec. 5.2), with every patch time an exact integer
// number of ticks dt_base * 2^-kmax.
#include "orc.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "orc_mhd.hpp"

namespace orc {

static thread_local std::string g_err;
static int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

static int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a < 0 ? -a : a;
}

// Time-step hash: FNV-1a over the sequence of per-step levels k.
static inline uint64_t khash_step(uint64_t h, int k) {
  h ^= (uint64_t)(uint8_t)(k & 0xff);
  h *= 1099511628211ull;
  return h;
}
static const uint64_t KHASH0 = 1469598103934665603ull;

template <class R> struct PatchT {
  int n = 0, level = 0;
  double dx = 0.0;
  int64_t lo[3] = {0, 0, 0}, len = 0, dxl = 0;  // exact lattice coordinates
  std::vector<std::vector<R>> slot;
  std::vector<int64_t> sticks;  // slot time in ticks (LOCAL, GLOBAL_QUANT)
  std::vector<double> stime;    // slot time (GLOBAL_EXACT, FIXED)
  std::vector<char> svalid;
  int cur = 0;
  int64_t ticks = 0;
  double t = 0.0;
  int64_t steps = 0;
  uint64_t khash = KHASH0;
  std::vector<int8_t> klog;
  std::vector<int> nbors;
  bool frozen = false;  // boundary patch: never updated, its slice holds at every time
};

template <class R> struct SetT {
  orc_config cfg;
  std::vector<PatchT<R>> p;
  int64_t box_lo[3], box_len[3];
  int64_t scale2 = 0;  // lattice units per unit length
  // bucket grid for point location
  int64_t bsize = 0;
  int nb[3] = {1, 1, 1};
  std::vector<std::vector<int>> bucket;
  Phys ph;
  int order = 0;
  uint64_t seed = 1;
  int nthreads = 1;
  bool initialised = false;
  bool exact_time = false;  // GLOBAL_EXACT / FIXED keep double times
  StepCounters cnt;
  int64_t updates = 0;
  int64_t rounds = 0;
  int64_t extrapolated = 0;  // updates whose guard fill extrapolated in time
  double last_ms = 0.0;

  size_t slice_size(int q) const { return Layout(p[q].n, 0).size(); }

  // ---- point location ----------------------------------------------------
  // mode[d] = 0: half-open [lo, hi); 1: (lo, hi].  Returns the finest patch
  // containing X (periodic), or -1.
  int locate(int64_t X[3], const int mode[3]) const {
    for (int d = 0; d < 3; ++d) {
      int64_t L = box_len[d];
      if (mode[d] == 0) {
        int64_t r = ((X[d] - box_lo[d]) % L + L) % L;
        X[d] = box_lo[d] + r;
      } else {
        int64_t r = ((box_lo[d] + L - X[d]) % L + L) % L;
        X[d] = box_lo[d] + L - r;
      }
    }
    int bi[3];
    for (int d = 0; d < 3; ++d) {
      int64_t x = X[d] - box_lo[d] - (mode[d] == 1 ? 1 : 0);
      if (x < 0) x += box_len[d];
      bi[d] = (int)std::min<int64_t>(x / bsize, nb[d] - 1);
    }
    const std::vector<int>& cand = bucket[((size_t)bi[2] * nb[1] + bi[1]) * nb[0] + bi[0]];
    int best = -1;
    for (int q : cand) {
      bool in = true;
      for (int d = 0; d < 3 && in; ++d) {
        int64_t a = p[q].lo[d], b = p[q].lo[d] + p[q].len;
        in = (mode[d] == 0) ? (X[d] >= a && X[d] < b) : (X[d] > a && X[d] <= b);
      }
      if (!in) continue;
      if (best < 0 || p[q].dxl < p[best].dxl) best = q;
    }
    return best;
  }

  // Position of a padded-array entry of patch q: component c = -1 for a cell
  // variable, 0..2 for a face field (index along c is a face index).
  void position(int q, int c, int i, int j, int k, int64_t X[3], int mode[3]) const {
    const PatchT<R>& P = p[q];
    int idx[3] = {i, j, k};
    for (int d = 0; d < 3; ++d) {
      if (d == c) {
        X[d] = P.lo[d] + (int64_t)idx[d] * P.dxl;
        // a face on a patch boundary is taken from the side of q's centre
        mode[d] = (2 * X[d] <= 2 * P.lo[d] + P.len) ? 0 : 1;
      } else {
        X[d] = P.lo[d] + (int64_t)idx[d] * P.dxl + P.dxl / 2;
        mode[d] = 0;
      }
    }
  }

  // ---- time interpolation ---------------------------------------------------
  // Pick the slice(s) of patch q for time (ticks or t): an exact copy when a
  // slice has that time, else the adjacent pair a < t < b with weight w.  With
  // a grace g > 0 (LOCAL mode) a time past q's newest slice is extrapolated
  // from the two newest slices a < b < t (w > 1; Sec. 3B).  With time order 2
  // (ticks modes) a third slice c joins (the next older than a, else the next
  // newer than b) and the value is the quadratic through the three:
  // s_a + L_b (s_b - s_a) + L_c (s_c - s_a), L the Lagrange weights.
  struct TB {
    int sa = -1, sb = -1, sc = -1;  // sc < 0: linear (or a copy when sa == sb)
    double w = 0.0, wc = 0.0;       // weights of b and c
  };
  int bracket(int q, int64_t tk, double tt, TB& tb) const {
    int e = bracket2(q, tk, tt, tb.sa, tb.sb, tb.w);
    tb.sc = -1;
    tb.wc = 0.0;
    if (e || tb.sa == tb.sb || cfg.torder < 2 || exact_time) return e;
    const PatchT<R>& Q = p[q];
    const int ns = (int)Q.slot.size();
    const int64_t ta = Q.sticks[tb.sa], tbk = Q.sticks[tb.sb];
    int c = -1;
    for (int s = 0; s < ns; ++s)  // the next older than a
      if (Q.svalid[s] && Q.sticks[s] < ta && (c < 0 || Q.sticks[s] > Q.sticks[c])) c = s;
    if (c < 0)
      for (int s = 0; s < ns; ++s)  // else the next newer than b
        if (Q.svalid[s] && Q.sticks[s] > tbk && (c < 0 || Q.sticks[s] < Q.sticks[c])) c = s;
    if (c < 0) return 0;
    const double x = (double)(tk - ta), xb = (double)(tbk - ta), xc = (double)(Q.sticks[c] - ta);
    tb.sc = c;
    tb.w = x * (x - xc) / (xb * (xb - xc));
    tb.wc = x * (x - xb) / (xc * (xc - xb));
    return 0;
  }
  int bracket2(int q, int64_t tk, double tt, int& sa, int& sb, double& w) const {
    const PatchT<R>& Q = p[q];
    int ns = (int)Q.slot.size();
    if (Q.frozen) {  // a boundary value: the same at every time
      sa = sb = Q.cur;
      w = 0.0;
      return 0;
    }
    sa = sb = -1;
    for (int s = 0; s < ns; ++s) {
      if (!Q.svalid[s]) continue;
      bool eq = exact_time ? (Q.stime[s] == tt) : (Q.sticks[s] == tk);
      if (eq) {
        sa = sb = s;
        w = 0.0;
        return 0;
      }
    }
    int ia = -1, ib = -1;
    for (int s = 0; s < ns; ++s) {
      if (!Q.svalid[s]) continue;
      if (exact_time) {
        if (Q.stime[s] < tt && (ia < 0 || Q.stime[s] > Q.stime[ia])) ia = s;
        if (Q.stime[s] > tt && (ib < 0 || Q.stime[s] < Q.stime[ib])) ib = s;
      } else {
        if (Q.sticks[s] < tk && (ia < 0 || Q.sticks[s] > Q.sticks[ia])) ia = s;
        if (Q.sticks[s] > tk && (ib < 0 || Q.sticks[s] < Q.sticks[ib])) ib = s;
      }
    }
    if (ia >= 0 && ib < 0 && cfg.grace > 0.0 && !exact_time) {
      // every slice is older than tk: ia is the newest; a = the next older one
      int i2 = -1;
      for (int s = 0; s < ns; ++s)
        if (Q.svalid[s] && Q.sticks[s] < Q.sticks[ia] && (i2 < 0 || Q.sticks[s] > Q.sticks[i2])) i2 = s;
      if (i2 < 0) return -1;
      ib = ia;
      ia = i2;
    }
    if (ia < 0 || ib < 0) return -1;
    sa = ia;
    sb = ib;
    if (exact_time)
      w = (tt - Q.stime[ia]) / (Q.stime[ib] - Q.stime[ia]);
    else
      w = (double)(tk - Q.sticks[ia]) / (double)(Q.sticks[ib] - Q.sticks[ia]);
    return 0;
  }

  // value of slice entry e of patch q at the bracket: s_a + w (s_b - s_a)
  // [+ w_c (s_c - s_a)]
  R tval(int q, size_t e, const TB& tb) const {
    const R& a = p[q].slot[tb.sa][e];
    if (tb.sa == tb.sb) return a;
    const R& b = p[q].slot[tb.sb][e];
    if (tb.sc < 0) return a + tb.w * (b - a);
    const R& c = p[q].slot[tb.sc][e];
    return a + tb.w * (b - a) + tb.wc * (c - a);
  }

  // ---- cross-resolution guard value --------------------------------------
  // Integral over the target box of the source patch's piecewise-linear,
  // minmod-limited reconstruction (slopes from the source interior only,
  // one-sided in the source's edge cells), divided by the box size.  For a
  // cell variable the box is the target cell; for a face field it is the
  // face area (and the source field is linear in the normal direction
  // between the two bracketing source faces).
  R cross_value(int q, int c, int var, const int64_t X[3], int64_t tdx, const TB& tb) const {
    const PatchT<R>& Q = p[q];
    const int n = Q.n;
    Layout SL(n, 0);
    auto get = [&](int v, int cc, int i, int j, int k) -> R {
      size_t e = (cc < 0) ? SL.cell(v, i, j, k) : SL.face(cc, i, j, k);
      return tval(q, e, tb);
    };
    auto minmod = [](R a, R b) -> R {
      if (val(a) * val(b) <= 0.0) return R(0.0);
      return (fabs(a) < fabs(b)) ? a : b;
    };
    // target box in lattice units, per axis [a, b]
    int64_t A[3], B[3];
    for (int d = 0; d < 3; ++d) {
      if (d == c) {
        A[d] = B[d] = X[d];
      } else {
        A[d] = X[d] - tdx / 2;
        B[d] = X[d] + tdx / 2;
      }
    }
    // Relative to the source origin (X was already wrapped into the source by
    // locate()); the target box lies inside the source when patch boundaries
    // coincide with cell faces of both patches, clamping only guards rounding.
    int64_t rel[3][2];
    for (int d = 0; d < 3; ++d) {
      rel[d][0] = std::max<int64_t>(0, std::min<int64_t>(Q.len, A[d] - Q.lo[d]));
      rel[d][1] = std::max<int64_t>(0, std::min<int64_t>(Q.len, B[d] - Q.lo[d]));
    }
    const double sdx = (double)Q.dxl;
    if (c < 0) {
      // source cells overlapping the target cell
      int i0[3], i1[3];
      for (int d = 0; d < 3; ++d) {
        i0[d] = (int)(rel[d][0] / Q.dxl);
        i1[d] = (int)((rel[d][1] - 1) / Q.dxl);
        i0[d] = std::max(0, std::min(n - 1, i0[d]));
        i1[d] = std::max(0, std::min(n - 1, i1[d]));
      }
      R acc = 0.0;
      double vol = 0.0;
      for (int k = i0[2]; k <= i1[2]; ++k)
        for (int j = i0[1]; j <= i1[1]; ++j)
          for (int i = i0[0]; i <= i1[0]; ++i) {
            int ci[3] = {i, j, k};
            double ov = 1.0, ctr[3];
            for (int d = 0; d < 3; ++d) {
              int64_t a = std::max(rel[d][0], (int64_t)ci[d] * Q.dxl);
              int64_t b = std::min(rel[d][1], (int64_t)(ci[d] + 1) * Q.dxl);
              ov *= (double)(b - a);
              // offset of the overlap centre from the source cell centre, in cells
              ctr[d] = (0.5 * (double)(a + b) - ((double)ci[d] + 0.5) * sdx) / sdx;
            }
            if (ov <= 0.0) continue;
            R v0 = get(var, -1, i, j, k);
            R vv = v0;
            for (int d = 0; d < 3; ++d) {
              int cm[3] = {i, j, k}, cp[3] = {i, j, k};
              cm[d] -= 1;
              cp[d] += 1;
              R s = 0.0;
              if (cm[d] >= 0 && cp[d] <= n - 1) {
                R vm = get(var, -1, cm[0], cm[1], cm[2]);
                R vp = get(var, -1, cp[0], cp[1], cp[2]);
                s = minmod(v0 - vm, vp - v0);
              } else if (cp[d] <= n - 1) {
                s = get(var, -1, cp[0], cp[1], cp[2]) - v0;  // one-sided at the edge
              } else if (cm[d] >= 0) {
                s = v0 - get(var, -1, cm[0], cm[1], cm[2]);
              }
              vv = vv + ctr[d] * s;
            }
            acc = acc + ov * vv;
            vol += ov;
          }
      return acc / vol;
    }
    // face field component c: faces of the source along c bracketing the plane
    int64_t xn = rel[c][0];
    int f0 = (int)(xn / Q.dxl);
    int64_t rem = xn - (int64_t)f0 * Q.dxl;
    if (f0 >= n) { f0 = n; rem = 0; }
    double wn = (double)rem / sdx;  // weight of face f0+1
    int t[2] = {(c + 1) % 3, (c + 2) % 3};
    int i0[2], i1[2];
    for (int m = 0; m < 2; ++m) {
      int d = t[m];
      i0[m] = std::max(0, std::min(n - 1, (int)(rel[d][0] / Q.dxl)));
      i1[m] = std::max(0, std::min(n - 1, (int)((rel[d][1] - 1) / Q.dxl)));
    }
    R acc = 0.0;
    double area = 0.0;
    for (int u = i0[0]; u <= i1[0]; ++u)
      for (int v = i0[1]; v <= i1[1]; ++v) {
        int ti[2] = {u, v};
        double ov = 1.0, ctr[2];
        for (int m = 0; m < 2; ++m) {
          int d = t[m];
          int64_t a = std::max(rel[d][0], (int64_t)ti[m] * Q.dxl);
          int64_t b = std::min(rel[d][1], (int64_t)(ti[m] + 1) * Q.dxl);
          ov *= (double)(b - a);
          ctr[m] = (0.5 * (double)(a + b) - ((double)ti[m] + 0.5) * sdx) / sdx;
        }
        if (ov <= 0.0) continue;
        R vv = 0.0;
        for (int side = 0; side < 2; ++side) {
          int f = f0 + side;
          double ws = side == 0 ? 1.0 - wn : wn;
          if (ws == 0.0) continue;
          int idx[3];
          idx[c] = f;
          idx[t[0]] = u;
          idx[t[1]] = v;
          R v0 = get(0, c, idx[0], idx[1], idx[2]);
          R lin = v0;
          for (int m = 0; m < 2; ++m) {
            int d = t[m];
            int im[3] = {idx[0], idx[1], idx[2]}, ip[3] = {idx[0], idx[1], idx[2]};
            im[d] -= 1;
            ip[d] += 1;
            R s = 0.0;
            if (im[d] >= 0 && ip[d] <= n - 1) {
              R vm = get(0, c, im[0], im[1], im[2]);
              R vp = get(0, c, ip[0], ip[1], ip[2]);
              s = minmod(v0 - vm, vp - v0);
            } else if (ip[d] <= n - 1) {
              s = get(0, c, ip[0], ip[1], ip[2]) - v0;  // one-sided at the edge
            } else if (im[d] >= 0) {
              s = v0 - get(0, c, im[0], im[1], im[2]);
            }
            lin = lin + ctr[m] * s;
          }
          vv = vv + ws * lin;
        }
        acc = acc + ov * vv;
        area += ov;
      }
    return acc / area;
  }

  // ---- guard fill (Sec. 3A) -------------------------------------------------
  // Fill the padded array of patch q at its own time: interior from its
  // latest slice, every guard entry of the nguard-deep shell from the patch
  // that holds that point (the finest one), interpolated in time.
  int fill(int q, std::vector<R>& Pd, bool& extrap) const {
    extrap = false;
    const PatchT<R>& P = p[q];
    const int n = P.n, ng = cfg.nguard;
    Layout L(n, ng), S(n, 0);
    Pd.assign(L.size(), R(0.0));
    const std::vector<R>& own = P.slot[P.cur];
    for (int c = -1; c < 3; ++c) {
      int nv = (c < 0) ? 5 : 1;
      int hi[3] = {n + ng - 1, n + ng - 1, n + ng - 1};
      int ihi[3] = {n - 1, n - 1, n - 1};
      if (c >= 0) { hi[c] += 1; ihi[c] += 1; }
      for (int k = -ng; k <= hi[2]; ++k)
        for (int j = -ng; j <= hi[1]; ++j)
          for (int i = -ng; i <= hi[0]; ++i) {
            bool interior = i >= 0 && j >= 0 && k >= 0 && i <= ihi[0] && j <= ihi[1] && k <= ihi[2];
            if (interior) {
              for (int v = 0; v < nv; ++v) {
                if (c < 0)
                  Pd[L.cell(v, i, j, k)] = own[S.cell(v, i, j, k)];
                else
                  Pd[L.face(c, i, j, k)] = own[S.face(c, i, j, k)];
              }
              continue;
            }
            int64_t X[3];
            int mode[3];
            position(q, c, i, j, k, X, mode);
            int64_t Xw[3] = {X[0], X[1], X[2]};
            int s = locate(Xw, mode);
            if (s < 0) return fail(ORC_ESTATE, "guard point outside every patch");
            TB tb;
            if (bracket(s, P.ticks, P.t, tb) != 0)
              return fail(ORC_ESTATE, "no time slices bracket the guard time");
            if (tb.sa != tb.sb && !exact_time && P.ticks > p[s].sticks[tb.sb]) extrap = true;
            const PatchT<R>& Q = p[s];
            bool same = (Q.dxl == P.dxl);
            int li[3];
            if (same) {
              for (int d = 0; d < 3; ++d) {
                int64_t off = Xw[d] - Q.lo[d];
                if (d != c) off -= Q.dxl / 2;
                if (off % Q.dxl != 0) same = false;
                li[d] = (int)(off / Q.dxl);
              }
            }
            for (int v = 0; v < nv; ++v) {
              R val_;
              if (same) {
                Layout QS(Q.n, 0);
                size_t eq = (c < 0) ? QS.cell(v, li[0], li[1], li[2]) : QS.face(c, li[0], li[1], li[2]);
                val_ = tval(s, eq, tb);
              } else {
                val_ = cross_value(s, c, v, Xw, P.dxl, tb);
              }
              if (c < 0)
                Pd[L.cell(v, i, j, k)] = val_;
              else
                Pd[L.face(c, i, j, k)] = val_;
            }
          }
    }
    return 0;
  }

  // ---- neighbour relation ---------------------------------------------------
  // q reads guard data from s  =>  s and q are neighbours (symmetric closure).
  void build_nbors() {
    const int np_ = (int)p.size();
    std::vector<std::vector<int>> reads(np_);
    for (int q = 0; q < np_; ++q) {
      const int n = p[q].n, ng = cfg.nguard;
      std::vector<char> seen(np_, 0);
      for (int c = -1; c < 3; ++c) {
        int hi[3] = {n + ng - 1, n + ng - 1, n + ng - 1};
        int ihi[3] = {n - 1, n - 1, n - 1};
        if (c >= 0) { hi[c] += 1; ihi[c] += 1; }
        for (int k = -ng; k <= hi[2]; ++k)
          for (int j = -ng; j <= hi[1]; ++j)
            for (int i = -ng; i <= hi[0]; ++i) {
              bool interior =
                  i >= 0 && j >= 0 && k >= 0 && i <= ihi[0] && j <= ihi[1] && k <= ihi[2];
              if (interior) continue;
              int64_t X[3];
              int mode[3];
              position(q, c, i, j, k, X, mode);
              int s = locate(X, mode);
              if (s >= 0 && s != q && !seen[s]) {
                seen[s] = 1;
                reads[q].push_back(s);
              }
            }
      }
    }
    std::vector<std::vector<char>> adj(np_);
    for (int q = 0; q < np_; ++q) adj[q].assign(np_, 0);
    for (int q = 0; q < np_; ++q)
      for (int s : reads[q]) {
        adj[q][s] = 1;
        adj[s][q] = 1;
      }
    for (int q = 0; q < np_; ++q) {
      p[q].nbors.clear();
      for (int s = 0; s < np_; ++s)
        if (adj[q][s]) p[q].nbors.push_back(s);
    }
  }

  // ---- per-patch update pieces ------------------------------------------------
  // Level k of a LOCAL step: k_c from the Courant rate (exact ceil(log2 r) via
  // frexp), raised so that the step keeps the patch time a multiple of its step.
  int level_for(double smax, int64_t ticks, int& k) const {
    if (!std::isfinite(smax)) return fail(ORC_ENONFINITE, "non-finite signal speed");
    double r = cfg.dt_base * smax / cfg.courant;
    int kc = 0;
    if (r > 1.0) {
      int e;
      double m = std::frexp(r, &e);
      kc = (m == 0.5) ? e - 1 : e;
    }
    int align = INT_MIN;
    if (ticks != 0) {
      int tz = 0;
      while (((ticks >> tz) & 1) == 0) ++tz;
      align = cfg.kmax - tz;
    }
    k = std::max(kc, align);
    if (k > cfg.kmax) return fail(ORC_EKMAX, "time-step level exceeds kmax");
    return 0;
  }

  struct Work {
    std::vector<R> P;
    Box3<Prim<R>> W;
    std::vector<R> out;
    double smax = 0.0;
    int k = 0;
    int64_t dtk = 0;
    StepCounters c;
    int err = 0;
    bool extrap = false;
  };

  int prepare(int q, Work& wk) const {
    int e = fill(q, wk.P, wk.extrap);
    if (e) return e;
    Layout L(p[q].n, cfg.nguard);
    e = prims(L, wk.P, ph, wk.W, wk.c);
    if (e == S_ENONFINITE) return fail(ORC_ENONFINITE, "non-finite state");
    if (e == S_ENEGATIVE) return fail(ORC_ENEGATIVE, "non-positive density or pressure");
    wk.smax = courant_rate(wk.W, p[q].n, p[q].dx, ph);
    if (!std::isfinite(wk.smax)) return fail(ORC_ENONFINITE, "non-finite signal speed");
    return 0;
  }

  void advance_patch(int q, Work& wk, R dt) const {
    Layout L(p[q].n, cfg.nguard);
    step(L, wk.P, wk.W, dt, p[q].dx, ph, wk.out, wk.c);
  }

  // publish: the new slice overwrites the oldest slot (Sec. 3A)
  void commit(int q, Work& wk, int64_t dtk, double dtd, int k) {
    PatchT<R>& P = p[q];
    int ns = (int)P.slot.size();
    int nxt = (P.cur + 1) % ns;
    P.slot[nxt].swap(wk.out);
    P.svalid[nxt] = 1;
    if (exact_time) {
      P.t = P.t + dtd;
      P.stime[nxt] = P.t;
    } else {
      P.ticks += dtk;
      P.sticks[nxt] = P.ticks;
      P.t = std::ldexp((double)P.ticks, -cfg.kmax) * cfg.dt_base;
    }
    P.cur = nxt;
    P.steps++;
    if (wk.extrap) extrapolated++;
    P.khash = khash_step(P.khash, k);
    if (P.klog.size() < 4096) P.klog.push_back((int8_t)k);
    cnt.floor_hits += wk.c.floor_hits;
    cnt.fallback_faces += wk.c.fallback_faces;
    updates += (int64_t)P.n * P.n * P.n;
  }

  // Eq. (1): t_q <= t_s + g dt_s for every neighbour s, with dt_s the step s
  // took last (0 before its first update, so no grace then), in ticks
  // floor(g dt_s).  The new slice overwrites q's oldest slot, so q also waits
  // until no neighbour can still need that slice: the slice after it must not
  // be newer than any neighbour's time (implied when g = 0).
  int64_t last_step(int s) const {
    const PatchT<R>& S = p[s];
    const int ns = (int)S.slot.size();
    const int prev = (S.cur + ns - 1) % ns;
    if (S.steps == 0 || !S.svalid[prev] || prev == S.cur) return 0;
    return S.ticks - S.sticks[prev];
  }
  bool ready(int q, int64_t T) const {
    const PatchT<R>& P = p[q];
    if (P.frozen || P.ticks >= T) return false;
    const int ns = (int)P.slot.size();
    // with time order 2 the slice before a bracket is read too: keep two
    const int oldest = (P.cur + 1) % ns, after = (P.cur + 1 + std::max(1, cfg.torder)) % ns;
    for (int s : P.nbors) {
      if (p[s].frozen) continue;  // boundary patches never lag
      const int64_t g = (int64_t)std::floor(cfg.grace * (double)last_step(s));
      if (P.ticks > p[s].ticks + g) return false;
      if (P.svalid[oldest] && P.sticks[after] > p[s].ticks) return false;
    }
    return true;
  }

  // ---- LOCAL time steps: the dispatcher (Sec. 3B) ------------------------
  int run_local(int64_t T, int64_t max_updates = -1) {
    const int np_ = (int)p.size();
    std::mt19937_64 rng(seed);
    std::vector<int> R_;
    int64_t nupd = 0;
    while (true) {
      if (max_updates >= 0 && nupd >= max_updates) return 0;
      nupd++;
      R_.clear();
      bool done = true;
      for (int q = 0; q < np_; ++q) {
        if (!p[q].frozen && p[q].ticks < T) done = false;
        if (ready(q, T)) R_.push_back(q);
      }
      if (done) return 0;
      if (R_.empty()) return fail(ORC_ESTATE, "no ready patch but not done");
      rounds++;
      if (order == 2) {
        // the whole ready set at once: compute from the pre-round state, then publish
        std::vector<Work> wk(R_.size());
        std::vector<int> err(R_.size(), 0);
        std::vector<std::string> msg(R_.size());
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
        for (long m = 0; m < (long)R_.size(); ++m) {
          int q = R_[m];
          int e = prepare(q, wk[m]);
          if (!e) e = level_for(wk[m].smax, p[q].ticks, wk[m].k);
          if (e) {
            err[m] = e;
            msg[m] = g_err;
            continue;
          }
          R dt = R(cfg.dt_base * std::ldexp(1.0, -wk[m].k));
          advance_patch(q, wk[m], dt);
        }
        for (size_t m = 0; m < R_.size(); ++m)
          if (err[m]) return fail(err[m], msg[m]);
        for (size_t m = 0; m < R_.size(); ++m) {
          int q = R_[m];
          int64_t dtk = (int64_t)1 << (cfg.kmax - wk[m].k);
          commit(q, wk[m], dtk, 0.0, wk[m].k);
        }
        continue;
      }
      int q;
      if (order == 1) {
        q = R_[(size_t)(rng() % R_.size())];
      } else {
        q = R_[0];
        for (int s : R_)
          if (p[s].ticks < p[q].ticks) q = s;  // oldest first, ties by id
      }
      Work wk;
      int e = prepare(q, wk);
      if (!e) e = level_for(wk.smax, p[q].ticks, wk.k);
      if (e) return e;
      R dt = R(cfg.dt_base * std::ldexp(1.0, -wk.k));
      advance_patch(q, wk, dt);
      int64_t dtk = (int64_t)1 << (cfg.kmax - wk.k);
      commit(q, wk, dtk, 0.0, wk.k);
    }
  }

  // ---- GLOBAL modes: every patch takes the same step ------------------------
  // mode 1: k = max over patches; mode 2: dt = courant / max smax, last step
  // clipped to the end time; mode 3: the fixed dt (also clipped).
  int run_global(int64_t T, double Td, int max_steps) {
    const int np_ = (int)p.size();
    int nstep = 0;
    while (true) {
      if (exact_time) {
        if (!(p[0].t < Td)) return 0;
      } else if (p[0].ticks >= T) {
        return 0;
      }
      if (max_steps >= 0 && nstep >= max_steps) return 0;
      std::vector<Work> wk(np_);
      std::vector<int> err(np_, 0);
      std::vector<std::string> msg(np_);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
      for (int q = 0; q < np_; ++q) {
        err[q] = prepare(q, wk[q]);
        if (err[q]) msg[q] = g_err;
      }
      for (int q = 0; q < np_; ++q)
        if (err[q]) return fail(err[q], msg[q]);
      double S = 0.0;
      int kq = 0;
      for (int q = 0; q < np_; ++q) {
        if (!(wk[q].smax <= S)) S = wk[q].smax;
        if (cfg.dt_mode == 1) {
          int k;
          int e = level_for(wk[q].smax, p[q].ticks, k);
          if (e) return e;
          kq = std::max(kq, k);
        }
      }
      double dtd = 0.0;
      int64_t dtk = 0;
      int klog = -1;
      if (cfg.dt_mode == 1) {
        dtk = (int64_t)1 << (cfg.kmax - kq);
        dtd = cfg.dt_base * std::ldexp(1.0, -kq);
        klog = kq;
      } else {
        dtd = (cfg.dt_mode == 2) ? cfg.courant / S : cfg.dt_fixed;
        if (max_steps < 0 && p[0].t + dtd > Td) dtd = Td - p[0].t;
      }
      rounds++;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
      for (int q = 0; q < np_; ++q) advance_patch(q, wk[q], R(dtd));
      for (int q = 0; q < np_; ++q) commit(q, wk[q], dtk, dtd, klog);
      nstep++;
    }
  }
};

static int build_set_common(const orc_config* cfg, const orc_patch_desc* pd, int32_t npatch,
                            orc_config& c, std::vector<orc_patch_desc>& d) {
  if (!cfg || !pd || npatch <= 0) return fail(ORC_EINVAL, "null argument or no patches");
  c = *cfg;
  if (!(c.gamma > 1.0) || !(c.courant > 0.0) || c.nguard < 2 || c.nslots < 2 || c.kmax < 0 ||
      c.kmax > 40 || c.limiter != 0 || !(c.grace >= 0.0 && c.grace < 1.0) || c.dt_mode < 0 || c.dt_mode > 3)
    return fail(ORC_EINVAL, "invalid configuration");
  if (c.grace > 0.0 && (c.dt_mode != 0 || c.nslots < 3))
    return fail(ORC_EINVAL, "a grace needs LOCAL time steps and at least 3 slots");
  if (!(c.eta >= 0.0) || !(c.gamma_ad >= 0.0) || (c.gamma_ad > 0.0 && !(c.rho_ion > 0.0)))
    return fail(ORC_EINVAL, "invalid non-ideal parameters");
  if (c.torder < 0 || c.torder > 2 || (c.torder == 2 && c.nslots < 3))
    return fail(ORC_EINVAL, "time order must be 1 or 2 (2 needs at least 3 slots)");
  if ((c.dt_mode == 0 || c.dt_mode == 1) && !(c.dt_base > 0.0))
    return fail(ORC_EINVAL, "dt_base must be positive");
  if (c.dt_mode == 3 && !(c.dt_fixed > 0.0)) return fail(ORC_EINVAL, "dt_fixed must be positive");
  for (int dd = 0; dd < 3; ++dd)
    if (!c.periodic[dd]) return fail(ORC_EINVAL, "only periodic boxes are supported");
  d.assign(pd, pd + npatch);
  int nactive = 0;
  for (auto& q : d) nactive += (q.flags & 1) ? 0 : 1;
  if (nactive == 0) return fail(ORC_EINVAL, "every patch is a boundary patch");
  if (nactive < npatch && c.dt_mode != 0) return fail(ORC_EINVAL, "boundary patches need LOCAL time steps");
  for (auto& q : d)
    if (q.n < 4 || !(q.size[0] > 0.0) || q.size[0] != q.size[1] || q.size[0] != q.size[2])
      return fail(ORC_EINVAL, "patches must be cubic with n >= 4");
  return 0;
}

template <class R> static int make_set(const orc_config& c, const std::vector<orc_patch_desc>& d,
                                       SetT<R>& s) {
  s.cfg = c;
  s.ph.gamma = c.gamma;
  s.ph.eps_deg = 1e-12;
  s.ph.p_floor = c.p_floor;
  s.ph.eta = c.eta;
  s.ph.gamma_ad = c.gamma_ad;
  s.ph.rho_i = c.rho_ion;
  s.ph.courant = c.courant;
  s.exact_time = (c.dt_mode == 2 || c.dt_mode == 3);
  // lattice: 2 * lcm(cells per unit length) units per unit length, so every
  // cell centre and face lies on an integer point
  int64_t F = 1;
  for (auto& q : d) {
    double cpl = q.n / q.size[0];
    int64_t ic = (int64_t)std::llround(cpl);
    if (ic <= 0 || std::fabs(cpl - (double)ic) > 1e-9 * cpl)
      return fail(ORC_EINVAL, "n/size must be an integer");
    F = F / gcd64(F, ic) * ic;
    if (F > ((int64_t)1 << 40)) return fail(ORC_EINVAL, "lattice too fine");
  }
  s.scale2 = 2 * F;
  auto tolat = [&](double x, int64_t& out) {
    double y = x * (double)s.scale2;
    int64_t iy = (int64_t)std::llround(y);
    if (std::fabs(y - (double)iy) > 1e-6) return false;
    out = iy;
    return true;
  };
  for (int dd = 0; dd < 3; ++dd) {
    int64_t a, b;
    if (!tolat(c.box_lo[dd], a) || !tolat(c.box_hi[dd], b) || b <= a)
      return fail(ORC_EINVAL, "box not on the patch lattice");
    s.box_lo[dd] = a;
    s.box_len[dd] = b - a;
  }
  s.p.resize(d.size());
  int64_t minlen = INT64_MAX;
  for (size_t q = 0; q < d.size(); ++q) {
    PatchT<R>& P = s.p[q];
    P.n = d[q].n;
    P.level = d[q].level;
    P.frozen = (d[q].flags & 1) != 0;
    P.dx = d[q].size[0] / d[q].n;
    if (!tolat(d[q].size[0], P.len)) return fail(ORC_EINVAL, "patch size not on the lattice");
    P.dxl = P.len / P.n;
    for (int dd = 0; dd < 3; ++dd) {
      if (!tolat(d[q].origin[dd], P.lo[dd])) return fail(ORC_EINVAL, "origin not on the lattice");
      if (P.lo[dd] < s.box_lo[dd] || P.lo[dd] + P.len > s.box_lo[dd] + s.box_len[dd])
        return fail(ORC_EINVAL, "patch outside the box");
    }
    if (c.nguard > P.n) return fail(ORC_EINVAL, "patch too small for its guard zones");
    minlen = std::min(minlen, P.len);
    int ns = c.nslots;
    P.slot.assign(ns, std::vector<R>());
    P.sticks.assign(ns, 0);
    P.stime.assign(ns, 0.0);
    P.svalid.assign(ns, 0);
  }
  s.bsize = minlen;
  for (int dd = 0; dd < 3; ++dd) s.nb[dd] = (int)((s.box_len[dd] + minlen - 1) / minlen);
  s.bucket.assign((size_t)s.nb[0] * s.nb[1] * s.nb[2], std::vector<int>());
  for (size_t q = 0; q < d.size(); ++q) {
    int a[3], b[3];
    for (int dd = 0; dd < 3; ++dd) {
      a[dd] = (int)((s.p[q].lo[dd] - s.box_lo[dd]) / minlen);
      b[dd] = (int)((s.p[q].lo[dd] + s.p[q].len - 1 - s.box_lo[dd]) / minlen);
    }
    for (int z = a[2]; z <= b[2]; ++z)
      for (int y = a[1]; y <= b[1]; ++y)
        for (int x = a[0]; x <= b[0]; ++x)
          s.bucket[((size_t)z * s.nb[1] + y) * s.nb[0] + x].push_back((int)q);
  }
  s.build_nbors();
  return 0;
}

template <class R> static int init_set(SetT<R>& s, const R* U, size_t nvals, double t0) {
  size_t need = 0;
  for (size_t q = 0; q < s.p.size(); ++q) need += s.slice_size((int)q);
  if (nvals != need) return fail(ORC_EINVAL, "wrong number of values");
  int64_t tk0 = 0;
  if (!s.exact_time) {
    double m = t0 / s.cfg.dt_base;
    double mr = std::nearbyint(m);
    if (std::fabs(m - mr) > 1e-9 * std::max(1.0, std::fabs(m)))
      return fail(ORC_EALIGN, "t0 is not a multiple of dt_base");
    tk0 = (int64_t)mr << s.cfg.kmax;
  }
  size_t off = 0;
  for (size_t q = 0; q < s.p.size(); ++q) {
    PatchT<R>& P = s.p[q];
    size_t m = s.slice_size((int)q);
    for (size_t e = 0; e < m; ++e)
      if (!std::isfinite(val(U[off + e]))) return fail(ORC_ENONFINITE, "non-finite initial state");
    for (size_t sl = 0; sl < P.slot.size(); ++sl) {
      P.slot[sl].assign(m, R(0.0));
      P.svalid[sl] = 0;
    }
    std::copy(U + off, U + off + m, P.slot[0].begin());
    P.svalid[0] = 1;
    P.cur = 0;
    P.ticks = tk0;
    P.sticks[0] = tk0;
    P.t = t0;
    P.stime[0] = t0;
    P.steps = 0;
    P.khash = KHASH0;
    P.klog.clear();
    off += m;
  }
  s.cnt = StepCounters();
  s.updates = 0;
  s.rounds = 0;
  s.extrapolated = 0;
  s.initialised = true;
  return 0;
}

}  // namespace orc

using namespace orc;

struct orc_set {
  SetT<double> s;
  std::vector<orc_patch_desc> desc;
};

extern "C" {

const char* orc_last_error(void) { return g_err.c_str(); }

int orc_create(const orc_config* cfg, const orc_patch_desc* pd, int32_t npatch, orc_set** out) {
  if (!out) return fail(ORC_EINVAL, "null output handle");
  *out = nullptr;
  orc_config c;
  std::vector<orc_patch_desc> d;
  int e = build_set_common(cfg, pd, npatch, c, d);
  if (e) return e;
  orc_set* h = new orc_set();
  h->desc = d;
  e = make_set(c, d, h->s);
  if (e) {
    delete h;
    return e;
  }
  *out = h;
  return 0;
}

int orc_init(orc_set* h, const double* U, size_t n_values, double t0) {
  if (!h || !U) return fail(ORC_EINVAL, "null argument");
  return init_set(h->s, U, n_values, t0);
}

int orc_advance_to(orc_set* h, double t_end) {
  if (!h || !h->s.initialised) return fail(ORC_ESTATE, "set not initialised");
  SetT<double>& s = h->s;
  auto t0 = std::chrono::steady_clock::now();
  int e;
  if (s.exact_time) {
    e = s.run_global(0, t_end, -1);
  } else {
    double m = t_end / s.cfg.dt_base;
    double mr = std::nearbyint(m);
    if (std::fabs(m - mr) > 1e-9 * std::max(1.0, std::fabs(m)))
      return fail(ORC_EALIGN, "end time is not a multiple of dt_base");
    if (mr * std::ldexp(1.0, s.cfg.kmax) > 9.0e18) return fail(ORC_EINVAL, "end time too large");
    int64_t T = (int64_t)mr << s.cfg.kmax;
    for (auto& P : s.p)
      if (P.ticks > T) return fail(ORC_EINVAL, "end time is before the current time");
    e = (s.cfg.dt_mode == 0) ? s.run_local(T) : s.run_global(T, 0.0, -1);
  }
  s.last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return e;
}

int orc_advance_limited(orc_set* h, double t_end, int64_t max_updates) {
  if (!h || !h->s.initialised || h->s.cfg.dt_mode != 0)
    return fail(ORC_ESTATE, "limited advance needs LOCAL mode");
  SetT<double>& s = h->s;
  double m = t_end / s.cfg.dt_base;
  double mr = std::nearbyint(m);
  if (std::fabs(m - mr) > 1e-9 * std::max(1.0, std::fabs(m)))
    return fail(ORC_EALIGN, "end time is not a multiple of dt_base");
  return s.run_local((int64_t)mr << s.cfg.kmax, max_updates);
}

int orc_read_state(const orc_set* h, double* U, size_t n_values, double* t_out) {
  if (!h || !U || !h->s.initialised) return fail(ORC_EINVAL, "bad argument");
  const SetT<double>& s = h->s;
  size_t off = 0;
  double tmin = INFINITY;
  for (size_t q = 0; q < s.p.size(); ++q) {
    size_t m = s.slice_size((int)q);
    if (off + m > n_values) return fail(ORC_EINVAL, "output buffer too small");
    std::copy(s.p[q].slot[s.p[q].cur].begin(), s.p[q].slot[s.p[q].cur].end(), U + off);
    off += m;
    tmin = std::min(tmin, s.p[q].t);
  }
  if (t_out) *t_out = tmin;
  return 0;
}

int orc_read_schedule(const orc_set* h, int64_t* steps, uint64_t* khash, int32_t* klog,
                      size_t klog_cap) {
  if (!h) return fail(ORC_EINVAL, "null handle");
  const SetT<double>& s = h->s;
  for (size_t q = 0; q < s.p.size(); ++q) {
    if (steps) steps[q] = s.p[q].steps;
    if (khash) khash[q] = s.p[q].khash;
    if (klog)
      for (size_t m = 0; m < klog_cap; ++m)
        klog[q * klog_cap + m] = m < s.p[q].klog.size() ? s.p[q].klog[m] : -2;
  }
  return 0;
}

int orc_stats(const orc_set* h, double out[16]) {
  if (!h || !out) return fail(ORC_EINVAL, "null argument");
  const SetT<double>& s = h->s;
  for (int m = 0; m < 16; ++m) out[m] = 0.0;
  out[0] = (double)s.updates;
  double divmax = 0.0, tmin = INFINITY, tmax = -INFINITY;
  for (size_t q = 0; q < s.p.size(); ++q) {
    const PatchT<double>& P = s.p[q];
    Layout S(P.n, 0);
    const std::vector<double>& u = P.slot[P.cur];
    double dv = P.dx * P.dx * P.dx;
    for (int k = 0; k < P.n; ++k)
      for (int j = 0; j < P.n; ++j)
        for (int i = 0; i < P.n; ++i) {
          for (int v = 0; v < 5; ++v) out[1 + v] += u[S.cell(v, i, j, k)] * dv;
          out[6] += 0.5 * (u[S.face(0, i, j, k)] + u[S.face(0, i + 1, j, k)]) * dv;
          out[7] += 0.5 * (u[S.face(1, i, j, k)] + u[S.face(1, i, j + 1, k)]) * dv;
          out[8] += 0.5 * (u[S.face(2, i, j, k)] + u[S.face(2, i, j, k + 1)]) * dv;
          double div = (u[S.face(0, i + 1, j, k)] - u[S.face(0, i, j, k)]) +
                       (u[S.face(1, i, j + 1, k)] - u[S.face(1, i, j, k)]) +
                       (u[S.face(2, i, j, k + 1)] - u[S.face(2, i, j, k)]);
          divmax = std::max(divmax, std::fabs(div) / P.dx);
        }
    if (!P.frozen) {
      tmin = std::min(tmin, P.t);
      tmax = std::max(tmax, P.t);
    }
  }
  out[9] = divmax;
  out[10] = (double)s.cnt.floor_hits;
  out[11] = (double)s.cnt.fallback_faces;
  out[12] = s.last_ms;
  out[13] = (double)s.rounds;
  out[14] = tmin;
  out[15] = tmax;
  return 0;
}

void orc_destroy(orc_set* h) { delete h; }

int orc_set_order(orc_set* h, int32_t order, uint64_t seed, int32_t nthreads) {
  if (!h || order < 0 || order > 2 || nthreads < 1) return fail(ORC_EINVAL, "bad argument");
  h->s.order = order;
  h->s.seed = seed;
  h->s.nthreads = nthreads;
  return 0;
}

int orc_times(const orc_set* h, int64_t* ticks, double* t) {
  if (!h) return fail(ORC_EINVAL, "null handle");
  for (size_t q = 0; q < h->s.p.size(); ++q) {
    if (ticks) ticks[q] = h->s.p[q].ticks;
    if (t) t[q] = h->s.p[q].t;
  }
  return 0;
}

int orc_layout(const orc_set* h, int64_t* offsets) {
  if (!h || !offsets) return fail(ORC_EINVAL, "null argument");
  int64_t off = 0;
  for (size_t q = 0; q < h->s.p.size(); ++q) {
    offsets[q] = off;
    off += (int64_t)h->s.slice_size((int)q);
  }
  offsets[h->s.p.size()] = off;
  return 0;
}

int orc_nbors(const orc_set* h, int32_t* counts, int32_t* ids, size_t cap) {
  if (!h || !counts) return fail(ORC_EINVAL, "null argument");
  size_t m = 0;
  for (size_t q = 0; q < h->s.p.size(); ++q) {
    counts[q] = (int32_t)h->s.p[q].nbors.size();
    for (int s : h->s.p[q].nbors) {
      if (ids && m < cap) ids[m] = s;
      m++;
    }
  }
  return (ids && m > cap) ? fail(ORC_EINVAL, "capacity too small") : 0;
}

int orc_extrapolated(const orc_set* h, int64_t* count) {
  if (!h || !count) return fail(ORC_EINVAL, "null argument");
  *count = h->s.extrapolated;
  return 0;
}

int orc_padded(const orc_set* h, int32_t q, double* out, size_t n_values) {
  if (!h || !out || q < 0 || q >= (int32_t)h->s.p.size()) return fail(ORC_EINVAL, "bad argument");
  std::vector<double> P;
  bool extrap;
  int e = h->s.fill(q, P, extrap);
  if (e) return e;
  if (n_values != P.size()) return fail(ORC_EINVAL, "wrong size");
  std::copy(P.begin(), P.end(), out);
  return 0;
}

int orc_slot(const orc_set* h, int32_t q, int32_t rel, double* out, size_t n_values,
             int64_t* ticks, double* t) {
  if (!h || q < 0 || q >= (int32_t)h->s.p.size() || rel < 0) return fail(ORC_EINVAL, "bad argument");
  const PatchT<double>& P = h->s.p[q];
  int ns = (int)P.slot.size();
  if (rel >= ns) return fail(ORC_EINVAL, "bad slot");
  int sl = ((P.cur - rel) % ns + ns) % ns;
  if (!P.svalid[sl]) return fail(ORC_ESTATE, "slot not valid");
  if (out) {
    if (n_values != P.slot[sl].size()) return fail(ORC_EINVAL, "wrong size");
    std::copy(P.slot[sl].begin(), P.slot[sl].end(), out);
  }
  if (ticks) *ticks = P.sticks[sl];
  if (t) *t = P.stime[sl];
  return 0;
}

int orc_hlld_flux(const double* wl, const double* wr, double bn, double gamma, double eps,
                  double* flux8) {
  if (!wl || !wr || !flux8) return fail(ORC_EINVAL, "null argument");
  Phys ph{gamma, eps, 0.0};
  hlld(wl, wr, bn, ph, flux8);
  return 0;
}

int orc_jvp_fixed(orc_set* h, const double* U0, const double* dU0, int32_t nsteps, double dt,
                  double* UT, double* dUT) {
  if (!h || !U0 || !dU0 || !UT || !dUT || nsteps < 0 || !(dt > 0.0))
    return fail(ORC_EINVAL, "bad argument");
  orc_config c = h->s.cfg;
  c.dt_mode = 3;
  c.dt_fixed = dt;
  SetT<Dual> s;
  int e = make_set(c, h->desc, s);
  if (e) return e;
  size_t need = 0;
  for (size_t q = 0; q < s.p.size(); ++q) need += s.slice_size((int)q);
  std::vector<Dual> u(need);
  for (size_t m = 0; m < need; ++m) u[m] = Dual(U0[m], dU0[m]);
  e = init_set(s, u.data(), need, 0.0);
  if (e) return e;
  e = s.run_global(0, INFINITY, nsteps);
  if (e) return e;
  size_t off = 0;
  for (size_t q = 0; q < s.p.size(); ++q) {
    const std::vector<Dual>& v = s.p[q].slot[s.p[q].cur];
    for (size_t m = 0; m < v.size(); ++m) {
      UT[off + m] = v[m].v;
      dUT[off + m] = v[m].d;
    }
    off += v.size();
  }
  return 0;
}

// Floating-point operations of the method from the given state up to t_end
// (same configuration and dispatch as the handle, one thread): out[0] =
// operations (see Flop), out[1] = cell updates, out[2] = the part of out[0]
// spent in the Courant rate.
int orc_count_flops(orc_set* h, const double* U0, double t_end, double* out) {
  if (!h || !U0 || !out) return fail(ORC_EINVAL, "null argument");
  SetT<Flop> s;
  int e = make_set(h->s.cfg, h->desc, s);
  if (e) return e;
  size_t need = 0;
  for (size_t q = 0; q < s.p.size(); ++q) need += s.slice_size((int)q);
  std::vector<Flop> u(need);
  for (size_t m = 0; m < need; ++m) u[m] = Flop(U0[m]);
  e = init_set(s, u.data(), need, 0.0);
  if (e) return e;
  s.nthreads = 1;
  flop_tally()[0].store(0);
  flop_tally()[1].store(0);
  if (s.exact_time) {
    e = s.run_global(0, t_end, -1);
  } else {
    double m = t_end / s.cfg.dt_base;
    double mr = std::nearbyint(m);
    if (std::fabs(m - mr) > 1e-9 * std::max(1.0, std::fabs(m)))
      return fail(ORC_EALIGN, "end time is not a multiple of dt_base");
    const int64_t T = (int64_t)mr << s.cfg.kmax;
    e = (s.cfg.dt_mode == 0) ? s.run_local(T) : s.run_global(T, 0.0, -1);
  }
  if (e) return e;
  out[0] = (double)(flop_tally()[0].load() + flop_tally()[1].load());
  out[1] = (double)s.updates;
  out[2] = (double)flop_tally()[1].load();
  return 0;
}

}  // extern "C"
