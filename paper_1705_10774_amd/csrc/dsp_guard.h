// dsp_guard.h -- index helpers of the slice / padded layouts and the guard
// value of one element: an exact copy or a linear time interpolation
// s_a + w (s_b - s_a) between the two slices of the source patch that bracket
// the reader's time (Sec. 3A), resampled conservatively when the source has
// another resolution.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsp_dev.h"

namespace dsp {

// ---------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ int64_t pcell(int N, int v, int i, int j, int k) {
  return (int64_t)v * N * N * N + ((int64_t)(k + 2) * N + (j + 2)) * N + (i + 2);
}
// padded face array of component d inside the padded patch buffer
__device__ __forceinline__ int64_t pface(int N, int d, int i, int j, int k) {
  const int sx = N + (d == 0), sy = N + (d == 1);
  return 5LL * N * N * N + (int64_t)d * N * N * (N + 1) + ((int64_t)(k + 2) * sy + (j + 2)) * sx + (i + 2);
}
// slice (interior) layout
__device__ __forceinline__ int64_t scell(int n, int v, int i, int j, int k) {
  return (int64_t)v * n * n * n + ((int64_t)k * n + j) * n + i;
}
__device__ __forceinline__ int64_t sface(int n, int d, int i, int j, int k) {
  const int sx = n + (d == 0), sy = n + (d == 1);
  return 5LL * n * n * n + (int64_t)d * n * n * (n + 1) + ((int64_t)k * sy + j) * sx + i;
}
// work arrays indexed by padded cell coordinates [-2, n+1]^3 (stride N^3 per
// component) and face/edge arrays over [-2, n+2]^3 (stride (N+1)^3)
__device__ __forceinline__ int64_t wcell(int N, int v, int i, int j, int k) {
  return (int64_t)v * N * N * N + ((int64_t)(k + 2) * N + (j + 2)) * N + (i + 2);
}
__device__ __forceinline__ int64_t wface(int N, int v, int i, int j, int k) {
  const int M = N + 1;
  return (int64_t)v * M * M * M + ((int64_t)(k + 2) * M + (j + 2)) * M + (i + 2);
}

// ordered bit patterns of non-negative floating-point numbers
__device__ __forceinline__ void atomic_max_pos(double* a, double v) {
  atomicMax((unsigned long long*)a, (unsigned long long)__double_as_longlong(v));
}

// time-slice bracket of patch q for time (tk, tt): exact slice or a < t < b;
// with a grace (LOCAL mode) a time past q's newest slice is extrapolated from
// the two newest slices a < b < t (w > 1).  With time order 2 (ticks modes)
// a third slice c joins, the next older than a, else the next newer than b,
// and the value is the quadratic s_a + w (s_b - s_a) + wc (s_c - s_a) with
// the Lagrange weights.
struct Bracket {
  int64_t oa, ob, oc;  // element offsets of the slices (oc < 0: no third)
  double w, wc;        // weights of b and c (0 for an exact copy)
};
__device__ inline Bracket bracket(const DevSet& S, int q, int64_t tk, double tt) {
  Bracket br;
  const int ns = S.nslots;
  if (S.frozen[q]) {  // a boundary value: the same at every time
    br.oa = br.ob = S.slot_off[q] + (int64_t)S.cur[q] * S.slice_len[q];
    br.oc = -1;
    br.w = br.wc = 0.0;
    return br;
  }
  int ia = -1, ib = -1, ie = -1;
  for (int s = 0; s < ns; ++s) {
    const int64_t e = (int64_t)q * ns + s;
    if (!S.svalid[e]) continue;
    const bool eq = S.exact_time ? (S.stime[e] == tt) : (S.sticks[e] == tk);
    if (eq) ie = s;
    if (S.exact_time) {
      if (S.stime[e] < tt && (ia < 0 || S.stime[e] > S.stime[(int64_t)q * ns + ia])) ia = s;
      if (S.stime[e] > tt && (ib < 0 || S.stime[e] < S.stime[(int64_t)q * ns + ib])) ib = s;
    } else {
      if (S.sticks[e] < tk && (ia < 0 || S.sticks[e] > S.sticks[(int64_t)q * ns + ia])) ia = s;
      if (S.sticks[e] > tk && (ib < 0 || S.sticks[e] < S.sticks[(int64_t)q * ns + ib])) ib = s;
    }
  }
  const int64_t base = S.slot_off[q];
  const int64_t V = S.slice_len[q];
  br.oc = -1;
  br.wc = 0.0;
  if (ie >= 0) {
    br.oa = br.ob = base + ie * V;
    br.w = 0.0;
    return br;
  }
  if (ia >= 0 && ib < 0 && S.grace > 0.0 && !S.exact_time) {
    int i2 = -1;
    for (int s = 0; s < ns; ++s) {
      const int64_t e = (int64_t)q * ns + s;
      if (S.svalid[e] && S.sticks[e] < S.sticks[(int64_t)q * ns + ia] &&
          (i2 < 0 || S.sticks[e] > S.sticks[(int64_t)q * ns + i2]))
        i2 = s;
    }
    ib = ia;
    ia = i2;
  }
  if (ia < 0 || ib < 0) {
    atomicOr(S.err, ERR_STATE);
    br.oa = br.ob = base;
    br.w = 0.0;
    return br;
  }
  br.oa = base + ia * V;
  br.ob = base + ib * V;
  const int64_t e_a = (int64_t)q * ns + ia, e_b = (int64_t)q * ns + ib;
  if (S.exact_time)
    br.w = (tt - S.stime[e_a]) / (S.stime[e_b] - S.stime[e_a]);
  else
    br.w = (double)(tk - S.sticks[e_a]) / (double)(S.sticks[e_b] - S.sticks[e_a]);
  if (S.torder >= 2 && !S.exact_time) {
    const int64_t ta = S.sticks[e_a], tb = S.sticks[e_b];
    int ic = -1;
    for (int s = 0; s < ns; ++s) {  // the next older than a
      const int64_t e = (int64_t)q * ns + s;
      if (S.svalid[e] && S.sticks[e] < ta && (ic < 0 || S.sticks[e] > S.sticks[(int64_t)q * ns + ic])) ic = s;
    }
    if (ic < 0)
      for (int s = 0; s < ns; ++s) {  // else the next newer than b
        const int64_t e = (int64_t)q * ns + s;
        if (S.svalid[e] && S.sticks[e] > tb && (ic < 0 || S.sticks[e] < S.sticks[(int64_t)q * ns + ic])) ic = s;
      }
    if (ic >= 0) {
      const double x = (double)(tk - ta), xb = (double)(tb - ta), xc = (double)(S.sticks[(int64_t)q * ns + ic] - ta);
      br.oc = base + ic * V;
      br.w = x * (x - xc) / (xb * (xb - xc));
      br.wc = x * (x - xb) / (xc * (xc - xb));
    }
  }
  return br;
}

// Publish the update of patch p whose step record is entry b of st (Sec. 3A):
// the new slot becomes current, the time advances, the step count, level log
// and level hash record the level.
__device__ inline void publish_patch(const DevSet& S, int p, const StepPtr& st, int b) {
  const int ns = S.nslots;
  const int nxt = (S.cur[p] + 1) % ns;
  const int64_t e = (int64_t)p * ns + nxt;
  if (S.exact_time) {
    S.tcur[p] = S.tcur[p] + st.dt[b];
    S.stime[e] = S.tcur[p];
  } else {
    S.ticks[p] += st.dtk[b];
    S.sticks[e] = S.ticks[p];
    S.tcur[p] = ldexp((double)S.ticks[p], -S.kmax) * S.dt_base;
  }
  S.svalid[e] = 1;
  S.cur[p] = nxt;
  const int k = st.k[b];
  const int64_t m = S.steps[p];
  if (m < S.klog_cap) S.klog[(int64_t)p * S.klog_cap + m] = (int8_t)k;
  S.steps[p] = m + 1;
  uint64_t h = S.khash[p];
  h ^= (uint64_t)(uint8_t)(k & 0xff);
  h *= 1099511628211ULL;
  S.khash[p] = h;
  const int n = S.n[p];
  atomicAdd(S.updates, (unsigned long long)n * n * n);
}

template <class T>
__device__ __forceinline__ T tlerp(const T* slots, const Bracket& br, int64_t e) {
  const T a = slots[br.oa + e];
  if (br.oa == br.ob) return a;
  const T b = slots[br.ob + e];
  if (br.oc < 0) return a + (T)br.w * (b - a);
  const T c = slots[br.oc + e];
  return a + (T)br.w * (b - a) + (T)br.wc * (c - a);
}

// Cross-resolution guard value: mean over the target box of the source's
// piecewise-linear, minmod-limited reconstruction (source-interior slopes,
// one-sided in the source's edge cells).  comp < 0: cell variable var over
// the target cell [X - h, X + h] per axis; comp = d: face field d over the
// target face (the source field is linear along d between its faces).
// The source values come from get(i, j, k) (time-interpolated value of the
// source element at source index (i, j, k) of component comp / variable var).
template <class T, class G>
__device__ T cross_value_from(const DevSet& S, int q, int comp, const int64_t* X, int64_t tdx, G&& get);

template <class T>
__device__ T cross_value(const DevSet& S, const T* slots, const Bracket& br, int q, int comp,
                         int var, const int64_t* X, int64_t tdx) {
  const int n = S.n[q];
  return cross_value_from<T>(S, q, comp, X, tdx, [&](int i, int j, int k) -> T {
    const int64_t e = (comp < 0) ? scell(n, var, i, j, k) : sface(n, comp, i, j, k);
    return tlerp(slots, br, e);
  });
}

template <class T, class G>
__device__ T cross_value_from(const DevSet& S, int q, int comp, const int64_t* X, int64_t tdx, G&& get) {
  const int n = S.n[q];
  const int64_t sdx = S.dxl[q];
  const int64_t* lo = S.lo + 3 * q;
  const int64_t len = S.len[q];
  int64_t a[3], b[3];
  for (int d = 0; d < 3; ++d) {
    int64_t A = (d == comp) ? X[d] : X[d] - tdx / 2;
    int64_t B = (d == comp) ? X[d] : X[d] + tdx / 2;
    A -= lo[d];
    B -= lo[d];
    a[d] = A < 0 ? 0 : (A > len ? len : A);
    b[d] = B < 0 ? 0 : (B > len ? len : B);
  }
  // offsets in source cells: numerators are exact integers in double, so
  // scaling by 1/sdx is within an ulp of the quotient
  const double isdx = 1.0 / (double)sdx;
  auto minmod = [](T x, T y) -> T {
    if (x * y <= T(0)) return T(0);
    return (fabs(x) < fabs(y)) ? x : y;
  };
  // slope of the (cell or face) sample at idx along axis d, in source cells
  auto slope = [&](int* idx, int d, int hi, T v0) -> T {
    const int c = idx[d];
    T s = T(0);
    if (c - 1 >= 0 && c + 1 <= hi) {
      idx[d] = c - 1; T vm = get(idx[0], idx[1], idx[2]);
      idx[d] = c + 1; T vp = get(idx[0], idx[1], idx[2]);
      s = minmod(v0 - vm, vp - v0);
    } else if (c + 1 <= hi) {
      idx[d] = c + 1; s = get(idx[0], idx[1], idx[2]) - v0;
    } else if (c - 1 >= 0) {
      idx[d] = c - 1; s = v0 - get(idx[0], idx[1], idx[2]);
    }
    idx[d] = c;
    return s;
  };
  if (comp < 0) {
    int i0[3], i1[3];
    for (int d = 0; d < 3; ++d) {
      i0[d] = (int)(a[d] / sdx);
      i1[d] = (int)((b[d] - 1) / sdx);
      i0[d] = i0[d] < 0 ? 0 : (i0[d] > n - 1 ? n - 1 : i0[d]);
      i1[d] = i1[d] < 0 ? 0 : (i1[d] > n - 1 ? n - 1 : i1[d]);
    }
    T acc = T(0);
    double vol = 0.0;
    for (int k = i0[2]; k <= i1[2]; ++k)
      for (int j = i0[1]; j <= i1[1]; ++j)
        for (int i = i0[0]; i <= i1[0]; ++i) {
          int ci[3] = {i, j, k};
          double ov = 1.0, off[3];
          for (int d = 0; d < 3; ++d) {
            int64_t x0 = a[d] > (int64_t)ci[d] * sdx ? a[d] : (int64_t)ci[d] * sdx;
            int64_t x1 = b[d] < (int64_t)(ci[d] + 1) * sdx ? b[d] : (int64_t)(ci[d] + 1) * sdx;
            ov *= (double)(x1 - x0);
            off[d] = (0.5 * (double)(x0 + x1) - ((double)ci[d] + 0.5) * (double)sdx) * isdx;
          }
          if (ov <= 0.0) continue;
          const T v0 = get(i, j, k);
          T vv = v0;
          for (int d = 0; d < 3; ++d) vv = vv + (T)off[d] * slope(ci, d, n - 1, v0);
          acc = acc + (T)ov * vv;
          vol += ov;
        }
    return acc / (T)vol;
  }
  // face field
  const int d = comp, t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  int f0 = (int)(a[d] / sdx);
  int64_t rem = a[d] - (int64_t)f0 * sdx;
  if (f0 >= n) { f0 = n; rem = 0; }
  const double wn = (double)rem / (double)sdx;
  int u0 = (int)(a[t1] / sdx), u1 = (int)((b[t1] - 1) / sdx);
  int v0_ = (int)(a[t2] / sdx), v1 = (int)((b[t2] - 1) / sdx);
  u0 = u0 < 0 ? 0 : (u0 > n - 1 ? n - 1 : u0);
  u1 = u1 < 0 ? 0 : (u1 > n - 1 ? n - 1 : u1);
  v0_ = v0_ < 0 ? 0 : (v0_ > n - 1 ? n - 1 : v0_);
  v1 = v1 < 0 ? 0 : (v1 > n - 1 ? n - 1 : v1);
  T acc = T(0);
  double area = 0.0;
  for (int u = u0; u <= u1; ++u)
    for (int v = v0_; v <= v1; ++v) {
      const int ti[2] = {u, v};
      const int ax[2] = {t1, t2};
      double ov = 1.0, off[2];
      for (int m = 0; m < 2; ++m) {
        const int dd = ax[m];
        int64_t x0 = a[dd] > (int64_t)ti[m] * sdx ? a[dd] : (int64_t)ti[m] * sdx;
        int64_t x1 = b[dd] < (int64_t)(ti[m] + 1) * sdx ? b[dd] : (int64_t)(ti[m] + 1) * sdx;
        ov *= (double)(x1 - x0);
        off[m] = (0.5 * (double)(x0 + x1) - ((double)ti[m] + 0.5) * (double)sdx) * isdx;
      }
      if (ov <= 0.0) continue;
      T vv = T(0);
      for (int side = 0; side < 2; ++side) {
        const double ws = side == 0 ? 1.0 - wn : wn;
        if (ws == 0.0) continue;
        int idx[3];
        idx[d] = f0 + side;
        idx[t1] = u;
        idx[t2] = v;
        const T c0 = get(idx[0], idx[1], idx[2]);
        T lin = c0;
        for (int m = 0; m < 2; ++m) lin = lin + (T)off[m] * slope(idx, ax[m], n - 1, c0);
        vv = vv + (T)ws * lin;
      }
      acc = acc + (T)ov * vv;
      area += ov;
    }
  return acc / (T)area;
}


// Value of element (comp, var, i, j, k) of patch p's padded view: the
// interior from the patch's own current slice, guard elements from the box
// table (source patch, shift or resampling) with brackets br[m - box0].
template <class T>
__device__ T fetch_elem(const DevSet& S, const T* slots, int p, int n, int64_t own, int box0,
                        const Bracket* br, int comp, int var, int i, int j, int k) {
  const int idx[3] = {i, j, k};
  int rg[3];
  bool interior = true;
  for (int d = 0; d < 3; ++d) {
    const int hi = n + (d == comp ? 1 : 0);
    rg[d] = idx[d] < 0 ? 0 : (idx[d] < hi ? 1 : 2);
    interior = interior && rg[d] == 1;
  }
  if (interior) {
    const int64_t se = (comp < 0) ? scell(n, var, i, j, k) : sface(n, comp, i, j, k);
    return slots[own + se];
  }
  const int key = p * 108 + (comp + 1) * 27 + (rg[2] * 3 + rg[1]) * 3 + rg[0];
  const int b0 = S.rbox_off[key], b1 = S.rbox_off[key + 1];
  for (int m = b0; m < b1; ++m) {
    const GBox& G = S.boxes[m];
    if (i < G.lo[0] || i > G.hi[0] || j < G.lo[1] || j > G.hi[1] || k < G.lo[2] || k > G.hi[2]) continue;
    const Bracket b = br[m - box0];
    if (G.same) {
      const int nq = S.n[G.q];
      const int qi = i + G.shift[0], qj = j + G.shift[1], qk = k + G.shift[2];
      const int64_t se = (comp < 0) ? scell(nq, var, qi, qj, qk) : sface(nq, comp, qi, qj, qk);
      return tlerp(slots, b, se);
    }
    const int64_t dxl = S.dxl[p];
    int64_t X[3];
    for (int d = 0; d < 3; ++d)
      X[d] = S.lo[3 * p + d] + (int64_t)idx[d] * dxl + (d == comp ? 0 : dxl / 2) + G.wrap[d];
    return cross_value(S, slots, b, G.q, comp, var, X, dxl);
  }
  atomicOr(S.err, ERR_STATE);
  return T(0);
}

// A guard region (key = (component + 1) * 27 + region, region = (rz * 3 + ry)
// * 3 + rx, r = 0 / 1 / 2 below / inside / above the interior along an axis)
// is "direct" when one same-resolution box covers it: its values are then
// read straight from the source's two bracketing slices.  Every other region
// is first written into a padded per-entry buffer (k_gfill) and read there.
__device__ __forceinline__ bool region_direct(const DevSet& S, int p, int key) {
  const int m0 = S.rbox_off[p * 108 + key], m1 = S.rbox_off[p * 108 + key + 1];
  return m1 - m0 == 1 && S.boxes[m0].same && S.torder < 2;  // the table blends two slices
}

// Per-workgroup table of the 108 regions of one patch (the four interior
// regions included): element (var, i, j, k) of region `key` is
// pa[e] + w (pb[e] - pa[e]), e the slice-layout offset of (var, i, j, k) for a
// patch of nq cells per edge.  Exact copies and the interior have pa == pb
// and w = 0, which gives pa[e] exactly.
template <class T> struct RegionEnt {
  const T* pa;
  const T* pb;
  T w;
  int nq;
};
template <class T> struct RegionTab {
  RegionEnt<T> r[108];
};

// Fill entry `key`.  ownp: the patch's current slice; pad: this entry's
// padded buffer (layout pcell / pface, N cells per edge including the guard
// layers).
template <class T>
__device__ inline void region_tab_init(const DevSet& S, const T* slots, const T* ownp, const T* pad, int N, int p,
                                       RegionTab<T>& R, int key) {
  const int comp = key / 27 - 1;
  RegionEnt<T> E;
  if (key % 27 == 13) {  // interior
    const int n = S.n[p];
    E.pa = E.pb = ownp + ((comp < 0) ? 0 : sface(n, comp, 0, 0, 0));
    E.w = T(0);
    E.nq = n;
  } else if (region_direct(S, p, key)) {
    const int m = S.rbox_off[p * 108 + key];
    const GBox& G = S.boxes[m];
    const Bracket b = S.brk_ready ? S.brk[m] : bracket(S, G.q, S.ticks[p], S.tcur[p]);
    const int nq = S.n[G.q];
    const int64_t e0 = (comp < 0) ? scell(nq, 0, G.shift[0], G.shift[1], G.shift[2])
                                  : sface(nq, comp, G.shift[0], G.shift[1], G.shift[2]);
    E.pa = slots + b.oa + e0;
    E.pb = slots + b.ob + e0;
    E.w = (T)b.w;
    E.nq = nq;
  } else {
    E.pa = E.pb = pad + ((comp < 0) ? pcell(N, 0, 0, 0, 0) : pface(N, comp, 0, 0, 0));
    E.w = T(0);
    E.nq = N;
  }
  R.r[key] = E;
}

// Same value as fetch_elem, through the region table, without branches: the
// region is selected arithmetically, both slices are read (the same address
// twice for an exact copy) and blended.  Offsets inside one slice fit in 32
// bits.  comp is a constant at every call site.
// The two reads of fetch_fast without the blend (issued early, blended later
// with blend_weight): same region, same offsets.
template <class T, int FNQ>
__device__ __forceinline__ void fetch_pair(int n, const RegionTab<T>& R, int comp, int var, int i, int j, int k,
                                           T& a, T& b) {
  const int hx = n + (comp == 0 ? 1 : 0), hy = n + (comp == 1 ? 1 : 0), hz = n + (comp == 2 ? 1 : 0);
  const int rx = (i >= 0) + (i >= hx);
  const int ry = (j >= 0) + (j >= hy);
  const int rz = (k >= 0) + (k >= hz);
  const RegionEnt<T>& E = R.r[(comp + 1) * 27 + (rz * 3 + ry) * 3 + rx];
  const int nq = FNQ ? FNQ : E.nq;
  int e;
  if (comp < 0) {
    e = ((var * nq + k) * nq + j) * nq + i;
  } else {
    const int sx = nq + (comp == 0), sy = nq + (comp == 1);
    e = (k * sy + j) * sx + i;
  }
  using gptr = const T __attribute__((address_space(1)))*;
  a = ((gptr)E.pa)[e];
  b = ((gptr)E.pb)[e];
}
template <class T>
__device__ __forceinline__ T blend_weight(int n, const RegionTab<T>& R, int comp, int i, int j, int k) {
  const int hx = n + (comp == 0 ? 1 : 0), hy = n + (comp == 1 ? 1 : 0), hz = n + (comp == 2 ? 1 : 0);
  const int rx = (i >= 0) + (i >= hx);
  const int ry = (j >= 0) + (j >= hy);
  const int rz = (k >= 0) + (k >= hz);
  return R.r[(comp + 1) * 27 + (rz * 3 + ry) * 3 + rx].w;
}

// FNQ > 0: every region's source patch has FNQ cells per edge (a set of
// equal patches whose guard regions are all single same-resolution boxes),
// so the offsets are compile-time strides.
template <class T, int FNQ = 0>
__device__ __forceinline__ T fetch_fast(int n, const RegionTab<T>& R, int comp, int var, int i, int j, int k) {
  const int hx = n + (comp == 0 ? 1 : 0), hy = n + (comp == 1 ? 1 : 0), hz = n + (comp == 2 ? 1 : 0);
  const int rx = (i >= 0) + (i >= hx);
  const int ry = (j >= 0) + (j >= hy);
  const int rz = (k >= 0) + (k >= hz);
  const RegionEnt<T> E = R.r[(comp + 1) * 27 + (rz * 3 + ry) * 3 + rx];
  const int nq = FNQ ? FNQ : E.nq;
  int e;
  if (comp < 0) {
    e = ((var * nq + k) * nq + j) * nq + i;
  } else {
    const int sx = nq + (comp == 0), sy = nq + (comp == 1);
    e = (k * sy + j) * sx + i;
  }
  // the table's pointers are global memory: say so, so the reads are global
  // (not flat) loads and do not hold up the workgroup's LDS traffic
  using gptr = const T __attribute__((address_space(1)))*;
  const T a = ((gptr)E.pa)[e];
  const T b = ((gptr)E.pb)[e];
  return a + E.w * (b - a);
}


}  // namespace dsp
