// dsp_fused.hip -- fused patch update for gfx950.
//
// One round of the dispatcher (Sec. 3B) updates every ready patch with two
// kernels:
//   k_courant   the Courant rate of each patch over its interior and the two
//               guard layers the stencil reads, guard values fetched on the
//               fly (time interpolation, resampling), wavefront + workgroup
//               maxima; pressure-floor and error accounting;
//   k_step      the whole MUSCL-Hancock + HLLD + constrained-transport step of
//               one patch tile, fused: the workgroup owns a tile of at most
//               16 x 16 columns (plus a 2-cell halo) and marches through the
//               patch along z.  Each (x, y) column is one thread; a plane of
//               primitives, half-step states, interface fluxes and edge EMFs
//               lives in LDS, the three planes of primitives the z-slopes need
//               and the carried z-face state live in registers.  Guard values
//               are read straight from the neighbours' ring slots, so nothing
//               but the new slice is written to HBM.
// Tiles of one patch are given workgroup ids that are equal modulo 8, so they
// run on the same XCD and share its L2 for the halo and guard reads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsp_dev.h"
#include "dsp_guard.h"
#include "mhd_dev.h"

namespace dsp {

constexpr int MCX = MT + 4;              // columns per edge incl. 2-cell halo
constexpr int MCOL = MCX * MCX;          // 400 column threads at most
constexpr int MPX = MT + 2;              // predictor cells per edge
constexpr int MPRED = MPX * MPX;         // 324
constexpr int MXF = (MT + 1) * (MT + 2); // x-faces (or y-faces) per plane: 306
constexpr int NTHR = 512;

template <class T> struct StepSmem {
  // region A: primitives of plane z (load -> predictor), then the plane's
  // x- and y-face fluxes (fluxes -> edges -> updates)
  union A {
    T w[8][MCOL];
    struct {
      T fx[8][MXF];
      T fy[8][MXF];
    } f;
  } a;
  // region B: half-step state, slopes and normal-field increments
  // (predictor -> fluxes), then the edge EMFs (edges -> updates)
  union B {
    struct {
      T h[8][MPRED];
      T sx[8][MPRED];
      T sy[8][MPRED];
      T db[2][MPRED];
    } p;
    struct {
      T ez[(MT + 1) * (MT + 1)];
      T ex[MT * (MT + 1)];
      T ey[(MT + 1) * MT];
    } e;
  } b;
  T bf[2][MCOL];        // Bx on the low x-face and By on the low y-face of each column (t^n)
  T px[2][MXF];         // previous plane: x-face upwind speed and Bz induction flux
  T py[2][MXF];         // previous plane: y-face upwind speed and Bz induction flux
  T fz[3][MPRED];       // current z-face: upwind speed, Bx and By induction fluxes
  T ecc[2][3][MPRED];   // cell-centred EMF -v x B of the half-step state, two planes
  RegionTab<T> rt;      // addressing of the guard regions
};

// primitives of one cell from guard-filled values
template <class T, class M = Exact<T>>
__device__ __forceinline__ void prim_of(T rho, T m0, T m1, T m2, T en, T bx, T by, T bz, T gamma,
                                        T pfloor, T* w) {
  const T ir = M::rcp(rho);
  w[0] = rho;
  w[1] = m0 * ir;
  w[2] = m1 * ir;
  w[3] = m2 * ir;
  T p = (gamma - T(1)) * (en - T(0.5) * (m0 * m0 + m1 * m1 + m2 * m2) * ir - T(0.5) * (bx * bx + by * by + bz * bz));
  if (pfloor > T(0) && p < pfloor) p = pfloor;
  w[4] = p;
  w[5] = bx;
  w[6] = by;
  w[7] = bz;
}

template <class T> struct PatchCtx {
  int p, n;
  const T* ownp;  // current slice of the patch
};

// guard-filled primitives of cell (i, j, k); the fields on its three low
// faces are returned too (outputs are written last, so they may alias)
template <class T, class M = Exact<T>, int FN = 0>
__device__ __forceinline__ void load_cell(const PatchCtx<T>& c, const RegionTab<T>& rt, int i, int j, int k,
                                          T gamma, T pfloor, T* w, T& bxl, T& byl, T& bzl) {
  const T rho = fetch_fast<T, FN>(FN ? FN : c.n, rt, -1, 0, i, j, k);
  const T m0 = fetch_fast<T, FN>(FN ? FN : c.n, rt, -1, 1, i, j, k);
  const T m1 = fetch_fast<T, FN>(FN ? FN : c.n, rt, -1, 2, i, j, k);
  const T m2 = fetch_fast<T, FN>(FN ? FN : c.n, rt, -1, 3, i, j, k);
  const T en = fetch_fast<T, FN>(FN ? FN : c.n, rt, -1, 4, i, j, k);
  const T xl = fetch_fast<T, FN>(FN ? FN : c.n, rt, 0, 0, i, j, k);
  const T xr = fetch_fast<T, FN>(FN ? FN : c.n, rt, 0, 0, i + 1, j, k);
  const T yl = fetch_fast<T, FN>(FN ? FN : c.n, rt, 1, 0, i, j, k);
  const T yr = fetch_fast<T, FN>(FN ? FN : c.n, rt, 1, 0, i, j + 1, k);
  const T zl = fetch_fast<T, FN>(FN ? FN : c.n, rt, 2, 0, i, j, k);
  const T zr = fetch_fast<T, FN>(FN ? FN : c.n, rt, 2, 0, i, j, k + 1);
  prim_of<T, M>(rho, m0, m1, m2, en, T(0.5) * (xl + xr), T(0.5) * (yl + yr), T(0.5) * (zl + zr), gamma, pfloor,
                w);
  bxl = xl;
  byl = yl;
  bzl = zl;
}

// load_cell in two halves: raw_issue starts the reads of one cell (both time
// slices of each value), raw_finish blends and converts them exactly as
// load_cell does, so independent work can run while the reads are in flight.
// n: cells per edge of the patch (FN when FN > 0).
template <class T> struct RawCell {
  T a[11], b[11];
};
template <class T, int FN>
__device__ __forceinline__ void raw_issue(int n, const RegionTab<T>& rt, int i, int j, int k, RawCell<T>& r) {
  if (FN) n = FN;
#pragma unroll
  for (int v = 0; v < 5; ++v) fetch_pair<T, FN>(n, rt, -1, v, i, j, k, r.a[v], r.b[v]);
  fetch_pair<T, FN>(n, rt, 0, 0, i, j, k, r.a[5], r.b[5]);
  fetch_pair<T, FN>(n, rt, 0, 0, i + 1, j, k, r.a[6], r.b[6]);
  fetch_pair<T, FN>(n, rt, 1, 0, i, j, k, r.a[7], r.b[7]);
  fetch_pair<T, FN>(n, rt, 1, 0, i, j + 1, k, r.a[8], r.b[8]);
  fetch_pair<T, FN>(n, rt, 2, 0, i, j, k, r.a[9], r.b[9]);
  fetch_pair<T, FN>(n, rt, 2, 0, i, j, k + 1, r.a[10], r.b[10]);
}
template <class T, class M, int FN>
__device__ __forceinline__ void raw_finish(int n, const RegionTab<T>& rt, int i, int j, int k, const RawCell<T>& r,
                                           T gamma, T pfloor, T* w, T& bxl, T& byl, T& bzl) {
  if (FN) n = FN;
  T v[11];
  const T wc = blend_weight(n, rt, -1, i, j, k);
#pragma unroll
  for (int q = 0; q < 5; ++q) v[q] = r.a[q] + wc * (r.b[q] - r.a[q]);
  const T wf[6] = {blend_weight(n, rt, 0, i, j, k),     blend_weight(n, rt, 0, i + 1, j, k),
                   blend_weight(n, rt, 1, i, j, k),     blend_weight(n, rt, 1, i, j + 1, k),
                   blend_weight(n, rt, 2, i, j, k),     blend_weight(n, rt, 2, i, j, k + 1)};
#pragma unroll
  for (int q = 0; q < 6; ++q) v[5 + q] = r.a[5 + q] + wf[q] * (r.b[5 + q] - r.a[5 + q]);
  prim_of<T, M>(v[0], v[1], v[2], v[3], v[4], T(0.5) * (v[5] + v[6]), T(0.5) * (v[7] + v[8]),
                T(0.5) * (v[9] + v[10]), gamma, pfloor, w);
  bxl = v[5];
  byl = v[7];
  bzl = v[9];
}

// first-order fallback states of a face along d: the primitives at t^n of
// the two cells beside it (cell (i, j, z) on its upper side), rotated to the
// face normal.  Rare; kept out of line, and returned by value so that the
// caller's face states never need to live in memory.
template <class T> struct FaceStates {
  T l[7], r[7];
};
template <class T, class M = Exact<T>>
__device__ __attribute__((noinline)) FaceStates<T> fallback_states(const PatchCtx<T>& c, const RegionTab<T>& rt,
                                                                   int d, int i, int j, int z, T gamma, T pfloor) {
  T wa[8], wb[8], dmy;
  load_cell<T, M>(c, rt, i - (d == 0), j - (d == 1), z - (d == 2), gamma, pfloor, wa, dmy, dmy, dmy);
  load_cell<T, M>(c, rt, i, j, z, gamma, pfloor, wb, dmy, dmy, dmy);
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  const int ord[7] = {0, 1 + d, 1 + t1, 1 + t2, 4, 5 + t1, 5 + t2};
  FaceStates<T> fs;
  for (int q = 0; q < 7; ++q) {
    fs.l[q] = wa[ord[q]];
    fs.r[q] = wb[ord[q]];
  }
  return fs;
}

// ---------------------------------------------------------------------------
// Guard regions that are not a single same-resolution box (several sources,
// or another resolution): values written into the entry's padded buffer, so
// the marching kernel reads every guard region with one addressing rule.
//
// A box from a patch of another resolution is resampled as cross_value
// defines it: the mean over the target cell (or face) of the source's
// piecewise-linear, minmod-limited reconstruction of its time-interpolated
// data.  The source cells a target cell overlaps form a tensor product of
// per-axis ranges, and the overlap volume is the product of per-axis
// lengths, so per axis and target index a table (GTab) holds the overlapped
// source indices with their weights (overlap length over the sum of the
// axis's overlaps) and the offsets of the overlap centres from the source
// cell centres (along a face field's own axis: the two bracketing source
// faces and their linear weights).  The geometry is static, so the host
// builds the tables once at create, shared between boxes of equal geometry,
// and cuts every box into work items (GItem) whose time-interpolated source
// block (all variables when they fit, slope neighbours included) fits the
// LDS stage.  A work item stages its tables and its source block, waits at
// one barrier, and every target value of the item sums over its overlapped
// cells from there.  Boxes whose overlaps exceed the tables (resolution
// ratios above three) or whose smallest chunk does not fit the stage are
// flagged by the host (GBox::direct) and resampled straight from the slices
// by k_gfill_direct.

template <class T> struct GfillSmem {
  T stage[GSTAGE_BYTES / sizeof(T)];
  GTab<T> tab[3][GMAXT];  // the item's box tables, indexed by target index
};

// Boxes flagged direct, resampled straight from the source slices: one
// workgroup per (region, patch) as k_gfill, one thread per element.
template <class T>
__global__ __launch_bounds__(256) void k_gfill_direct(DevSet S, const int* __restrict__ list, int count,
                                                      const T* __restrict__ slots, T* __restrict__ pad,
                                                      int64_t pad_stride) {
  const int key = blockIdx.x;
  const int b = blockIdx.y;
  if (b >= live_count(S, count)) return;
  const int p = list[b];
  const int comp = key / 27 - 1;
  const int n = S.n[p], N = n + 4;
  const int nvar = comp < 0 ? 5 : 1;
  const int m0 = S.rbox_off[p * 108 + key], m1 = S.rbox_off[p * 108 + key + 1];
  const int64_t dxl = S.dxl[p];
  T* dst = pad + (int64_t)b * pad_stride;
  for (int m = m0; m < m1; ++m) {
    const GBox G = S.boxes[m];
    if (!G.direct) continue;
    const Bracket br = S.brk[m];
    const int ex = G.hi[0] - G.lo[0] + 1, ey = G.hi[1] - G.lo[1] + 1, ez = G.hi[2] - G.lo[2] + 1;
    for (int e = threadIdx.x; e < ex * ey * ez * nvar; e += blockDim.x) {
      int r = e;
      const int i = G.lo[0] + r % ex;
      r /= ex;
      const int j = G.lo[1] + r % ey;
      r /= ey;
      const int k = G.lo[2] + r % ez;
      const int var = r / ez;
      const int idx[3] = {i, j, k};
      int64_t X[3];
      for (int d = 0; d < 3; ++d) X[d] = S.lo[3 * p + d] + (int64_t)idx[d] * dxl + (d == comp ? 0 : dxl / 2) + G.wrap[d];
      dst[(comp < 0) ? pcell(N, var, i, j, k) : pface(N, comp, i, j, k)] =
          cross_value(S, slots, br, G.q, comp, var, X, dxl);
    }
  }
}

// Time-interpolated values (tlerp) of count elements, U per thread at a
// time: every read of a batch is issued before the first value is used, so
// the read latencies overlap instead of adding up along the loop.  off(e):
// the element's offset within a slice; put(e, v) stores the value.
template <class T, int U, class Off, class Put>
__device__ __forceinline__ void tlerp_batched(const T* slots, const Bracket& br, int count, int tid, int nthr,
                                              Off&& off, Put&& put) {
  using gptr = const T __attribute__((address_space(1)))*;
  const gptr g = (gptr)slots;
  const bool two = br.oa != br.ob, three = br.oc >= 0;
  const T w = (T)br.w, wc = (T)br.wc;
  for (int e0 = tid; e0 < count; e0 += nthr * U) {
    T a[U], b[U], c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * nthr;
      if (e < count) {
        const int64_t se = off(e);
        a[u] = g[br.oa + se];
        b[u] = two ? g[br.ob + se] : a[u];
        c[u] = three ? g[br.oc + se] : a[u];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * nthr;
      if (e < count) {
        T v = a[u];
        if (two) v = three ? a[u] + w * (b[u] - a[u]) + wc * (c[u] - a[u]) : a[u] + w * (b[u] - a[u]);
        put(e, v);
      }
    }
  }
}

// Limited slope of a staged source cell along one axis: the minmod of the
// two one-sided differences when both neighbours exist, the one-sided
// difference at the source's edge, 0 for a single cell.  Branch-free: a
// missing neighbour is read as the cell itself (vm or vp = v0), so its
// difference is exactly 0 and a + b is the other one.
template <class T>
__device__ __forceinline__ T limited_slope(T vm, T v0, T vp, bool both) {
  const T a = v0 - vm, b = vp - v0;
  const T mm = (a * b <= T(0)) ? T(0) : ((fabs(a) < fabs(b)) ? a : b);
  return both ? mm : a + b;
}

// q = r / d for 0 <= r < 2^22 and 1 <= d < 2^11 without an integer division:
// the single-precision estimate r * (1/d) is within one of the quotient,
// and one correction step makes it exact.
__device__ __forceinline__ int small_div(int r, int d, float inv) {
  int q = (int)((float)r * inv);
  const int rem = r - q * d;
  q += rem >= d ? 1 : 0;
  q -= rem < 0 ? 1 : 0;
  return q;
}

// Quotient r / d of the index decoding: a compile-time patch size (FN > 0)
// divides by constants, a run-time one through the reciprocal (small_div).
template <int FN>
__device__ __forceinline__ int qdiv(int r, int d, float inv) {
  if constexpr (FN > 0)
    return r / d;
  else
    return small_div(r, d, inv);
}

constexpr int GFILL_ROWS = 512;  // patch rows of the resampling grid (a row strides over the ready list)
constexpr int GFILL_COLS = 24;   // workgroups per patch row (a column strides over the patch's items)

// Metadata of a work item prefetched into registers, one 32-bit word per
// lane: the item (lanes from 0) in one register; its box (lanes from 0) and
// the round's time bracket of the box (lanes from 32) in another, loaded once
// the item's box index has arrived.  The words come back as scalars
// (readlane) when the item starts.  A workgroup so fetches the next item's
// metadata while it works on the current one, instead of waiting at the start
// of every item on the chain item -> box and bracket -> staged values.
constexpr int GI_WORDS = (int)(sizeof(GItem) / 4), GB_WORDS = (int)(sizeof(GBox) / 4);
constexpr int BR_WORDS = (int)(sizeof(Bracket) / 4);
static_assert(GI_WORDS <= 64 && GB_WORDS <= 32 && BR_WORDS <= 32, "one word per lane of a wavefront");
__device__ __forceinline__ int gmeta_item(const DevSet& S, int i, int lane) {
  return lane < GI_WORDS ? ((const int*)(S.gitems + i))[lane] : 0;
}
__device__ __forceinline__ int gmeta_box(const DevSet& S, int m, int lane) {
  if (lane < GB_WORDS) return ((const int*)(S.boxes + m))[lane];
  if (lane >= 32 && lane < 32 + BR_WORDS) return ((const int*)(S.brk + m))[lane - 32];
  return 0;
}
__device__ __forceinline__ GItem gmeta_unpack_item(int reg) {
  int w[GI_WORDS];
#pragma unroll
  for (int k = 0; k < GI_WORDS; ++k) w[k] = __builtin_amdgcn_readlane(reg, k);
  GItem r;
  __builtin_memcpy(&r, w, sizeof(GItem));
  return r;
}
// the parts of the box that the resampling reads
struct GBoxLo {
  int lo[3], hi[3], shift[3];
};
__device__ __forceinline__ GBoxLo gmeta_unpack_box(int reg) {
  GBoxLo r;
  constexpr int lo = offsetof(GBox, lo) / 4, hi = offsetof(GBox, hi) / 4, sh = offsetof(GBox, shift) / 4;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    r.lo[d] = __builtin_amdgcn_readlane(reg, lo + d);
    r.hi[d] = __builtin_amdgcn_readlane(reg, hi + d);
    r.shift[d] = __builtin_amdgcn_readlane(reg, sh + d);
  }
  return r;
}
__device__ __forceinline__ Bracket gmeta_unpack_bracket(int reg) {
  auto i64 = [&](int o) {
    const int w = 32 + o / 4;
    return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(reg, w + 1) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane(reg, w));
  };
  auto f64 = [&](int o) {
    const int w = 32 + o / 4;
    return __hiloint2double(__builtin_amdgcn_readlane(reg, w + 1), __builtin_amdgcn_readlane(reg, w));
  };
  Bracket r;
  r.oa = i64(offsetof(Bracket, oa));
  r.ob = i64(offsetof(Bracket, ob));
  r.oc = i64(offsetof(Bracket, oc));
  r.w = f64(offsetof(Bracket, w));
  r.wc = f64(offsetof(Bracket, wc));
  return r;
}

// Work item it of patch p (box G, time bracket br) into its padded buffer
// dst, by the whole workgroup (every thread calls it).  mid() runs once the
// item's source values are staged (a copy item: at its start), to start
// loads for the next item.  A resampling item ends with a barrier (the next
// item reuses the stage); a copy item uses no LDS and has none.
template <class T, class Mid>
__device__ __forceinline__ void gfill_item(const DevSet& S, GfillSmem<T>& sm, const T* __restrict__ slots,
                                           T* __restrict__ dst, int p, const GItem& it, const GBoxLo& G,
                                           const Bracket& br, int tid, Mid&& mid) {
  constexpr int GSTAGE = GSTAGE_BYTES / (int)sizeof(T);
  const int comp = it.comp;
  const int nthr = blockDim.x;
  const int n = S.n[p], N = n + 4;
  // padded-buffer offset (32 bits: a padded patch holds fewer than 2^31 values)
  const int N2 = N * N;
  auto dst_off = [&](int var, int i, int j, int k) -> int {
    if (comp < 0) return var * N2 * N + ((k + 2) * N + (j + 2)) * N + (i + 2);
    const int sx = N + (comp == 0), sy = N + (comp == 1);
    return 5 * N2 * N + comp * N2 * (N + 1) + ((k + 2) * sy + (j + 2)) * sx + (i + 2);
  };
  const int ext[3] = {G.hi[0] - G.lo[0] + 1, G.hi[1] - G.lo[1] + 1, G.hi[2] - G.lo[2] + 1};
  const int nq = it.nq;
  if (it.tab[0] < 0) {  // a same-resolution box of a padded region: a time-interpolated copy
    mid();
    const int cnt = ext[0] * ext[1] * ext[2];
    const float ie0 = 1.0f / (float)ext[0], ie1 = 1.0f / (float)ext[1], ie2 = 1.0f / (float)ext[2];
    auto decode = [&](int e, int& var, int& i, int& j, int& k) {
      int r = e;
      int qq = small_div(r, ext[0], ie0);
      i = G.lo[0] + (r - qq * ext[0]);
      r = qq;
      qq = small_div(r, ext[1], ie1);
      j = G.lo[1] + (r - qq * ext[1]);
      r = qq;
      qq = small_div(r, ext[2], ie2);
      k = G.lo[2] + (r - qq * ext[2]);
      var = qq;
    };
    tlerp_batched<T, 8>(
        slots, br, cnt * it.nv, tid, nthr,
        [&](int e) -> int64_t {
          int var, i, j, k;
          decode(e, var, i, j, k);
          const int qi = i + G.shift[0], qj = j + G.shift[1], qk = k + G.shift[2];
          return (comp < 0) ? scell(nq, var, qi, qj, qk) : sface(nq, comp, qi, qj, qk);
        },
        [&](int e, T v) {
          int var, i, j, k;
          decode(e, var, i, j, k);
          dst[dst_off(var, i, j, k)] = v;
        });
    return;
  }
  // the box's tables (the chunk axis only over the chunk) and the staged block
  const GTab<T>* pool = (const GTab<T>*)S.gtab;
  const int ca = it.ca, ta = it.ta, tb = it.tb;
  {
    const int l0 = ca == 0 ? tb - ta + 1 : ext[0], l1 = ca == 1 ? tb - ta + 1 : ext[1];
    const int l2 = ca == 2 ? tb - ta + 1 : ext[2];
    for (int e = tid; e < l0 + l1 + l2; e += nthr) {
      const int d = e < l0 ? 0 : (e < l0 + l1 ? 1 : 2);
      const int t = e - (d > 0 ? l0 : 0) - (d > 1 ? l1 : 0) + (d == ca ? ta : 0);
      sm.tab[d][t] = pool[(d == 0 ? it.tab[0] : (d == 1 ? it.tab[1] : it.tab[2])) + t];
    }
  }
  const int r00 = it.r0[0], r01 = it.r0[1], r02 = it.r0[2];
  const int sx = it.r1[0] - r00 + 1, sy = it.r1[1] - r01 + 1, sz = it.r1[2] - r02 + 1;
  const int sxy = sx * sy, sblk = sxy * sz;
  const int v0 = it.v0, nv = it.nv;
  if (nv * sblk > GSTAGE) {  // the host plans every item to fit
    if (tid == 0) atomicOr(S.err, ERR_STATE);
    mid();
    return;
  }
  {
    const float isx = 1.0f / (float)sx, isxy = 1.0f / (float)sxy, isblk = 1.0f / (float)sblk;
    tlerp_batched<T, 8>(
        slots, br, nv * sblk, tid, nthr,
        [&](int e) -> int64_t {
          const int v = small_div(e, sblk, isblk), r = e - v * sblk;
          const int kq = small_div(r, sxy, isxy), rr = r - kq * sxy;
          const int jq = small_div(rr, sx, isx);
          const int ii = r00 + (rr - jq * sx), jj = r01 + jq, kk = r02 + kq;
          return (comp < 0) ? scell(nq, v0 + v, ii, jj, kk) : sface(nq, comp, ii, jj, kk);
        },
        [&](int e, T v) { sm.stage[e] = v; });
  }
  __syncthreads();
  mid();
  // target elements of the chunk: ta..tb along the chunk axis, all of the
  // others (per-axis indices kept in scalars: no private arrays indexed at
  // run time in the hot loop)
  const int ce0 = ca == 0 ? tb - ta + 1 : ext[0], ce1 = ca == 1 ? tb - ta + 1 : ext[1];
  const int ce2 = ca == 2 ? tb - ta + 1 : ext[2];
  const int ce01 = ce0 * ce1, ccnt = ce01 * ce2;
  const float ice0 = 1.0f / (float)ce0, ice01 = 1.0f / (float)ce01, iccnt = 1.0f / (float)ccnt;
  for (int e = tid; e < nv * ccnt; e += nthr) {
    const int v = small_div(e, ccnt, iccnt), r = e - v * ccnt;
    int t2 = small_div(r, ce01, ice01);
    const int r2 = r - t2 * ce01;
    int t1 = small_div(r2, ce0, ice0);
    int t0 = r2 - t1 * ce0;
    t0 += ca == 0 ? ta : 0;
    t1 += ca == 1 ? ta : 0;
    t2 += ca == 2 ? ta : 0;
    const T* st = sm.stage + v * sblk;
    T acc = T(0);
    if (comp < 0) {
      const GTab<T>& Z = sm.tab[2][t2];
      const GTab<T>& Y = sm.tab[1][t1];
      const GTab<T>& X = sm.tab[0][t0];
      for (int c = 0; c < Z.cnt; ++c) {
        const int kk = Z.i0 + c;
        const T wz = Z.w[c], oz = Z.off[c];
        const bool zm = kk - 1 >= 0, zp = kk + 1 <= nq - 1;
        for (int bq = 0; bq < Y.cnt; ++bq) {
          const int jj = Y.i0 + bq;
          const T wy = Y.w[bq], oy = Y.off[bq];
          const bool ym = jj - 1 >= 0, yp = jj + 1 <= nq - 1;
          const T wyz = wy * wz;
          const int rowb = (kk - r02) * sxy + (jj - r01) * sx - r00;
          for (int a = 0; a < X.cnt; ++a) {
            const int ii = X.i0 + a;
            const T wx = X.w[a], ox = X.off[a];
            const int o = rowb + ii;
            const bool xm = ii - 1 >= 0, xp = ii + 1 <= nq - 1;
            const T c0 = st[o];
            const T xl = st[o - (xm ? 1 : 0)], xr = st[o + (xp ? 1 : 0)];
            const T yl = st[o - (ym ? sx : 0)], yr = st[o + (yp ? sx : 0)];
            const T zl = st[o - (zm ? sxy : 0)], zr = st[o + (zp ? sxy : 0)];
            const T gx = limited_slope(xl, c0, xr, xm && xp);
            const T gy = limited_slope(yl, c0, yr, ym && yp);
            const T gz = limited_slope(zl, c0, zr, zm && zp);
            acc = acc + (wx * wyz) * (((c0 + ox * gx) + oy * gy) + oz * gz);
          }
        }
      }
    } else {
      // face field of component d = comp: index f along d, u along
      // t1 = d + 1, w along t2 = d + 2 (cyclic); stage strides of the three
      const int d = comp;
      const int tn = d == 0 ? t0 : (d == 1 ? t1 : t2);
      const int tu = d == 0 ? t1 : (d == 1 ? t2 : t0);
      const int tw = d == 0 ? t2 : (d == 1 ? t0 : t1);
      const int au = d == 2 ? 0 : d + 1, aw = d == 0 ? 2 : d - 1;  // the axes t1, t2
      const int su = au == 0 ? 1 : (au == 1 ? sx : sxy), sw = aw == 0 ? 1 : (aw == 1 ? sx : sxy);
      const int sn = d == 0 ? 1 : (d == 1 ? sx : sxy);
      const int rn = d == 0 ? r00 : (d == 1 ? r01 : r02);
      const int ru = au == 0 ? r00 : (au == 1 ? r01 : r02);
      const int rw = aw == 0 ? r00 : (aw == 1 ? r01 : r02);
      const GTab<T>& U = sm.tab[au][tu];
      const GTab<T>& W = sm.tab[aw][tw];
      const GTab<T>& F = sm.tab[d][tn];
      for (int cu = 0; cu < U.cnt; ++cu) {
        const int u = U.i0 + cu;
        const T wu = U.w[cu], ou = U.off[cu];
        const bool um = u - 1 >= 0, up = u + 1 <= nq - 1;
        for (int cw = 0; cw < W.cnt; ++cw) {
          const int w = W.i0 + cw;
          const T ww = W.w[cw], ow = W.off[cw];
          const bool wm = w - 1 >= 0, wp = w + 1 <= nq - 1;
          T lin2 = T(0);
          for (int side = 0; side < F.cnt; ++side) {
            const int f = F.i0 + side;
            const int o = (f - rn) * sn + (u - ru) * su + (w - rw) * sw;
            const T c0 = st[o];
            const T ul = st[o - (um ? su : 0)], ur = st[o + (up ? su : 0)];
            const T wl = st[o - (wm ? sw : 0)], wr = st[o + (wp ? sw : 0)];
            const T gu = limited_slope(ul, c0, ur, um && up);
            const T gw = limited_slope(wl, c0, wr, wm && wp);
            lin2 = lin2 + F.w[side] * ((c0 + ou * gu) + ow * gw);
          }
          acc = acc + (wu * ww) * lin2;
        }
      }
    }
    dst[dst_off(v0 + v, G.lo[0] + t0, G.lo[1] + t1, G.lo[2] + t2)] = acc;
  }
  __syncthreads();  // the next item reuses the tables and the stage
}

// Work items i0, i0 + step, ... below i1 of patch p into its padded buffer
// dst, by the whole workgroup: each item's metadata is prefetched during the
// item before it (the item word at its start, box and bracket once its
// source values are staged).  The brackets of the patch's boxes are in S.brk.
template <class T>
__device__ void gfill_items(const DevSet& S, GfillSmem<T>& sm, const T* __restrict__ slots, T* __restrict__ dst,
                            int p, int i0, int i1, int step, int tid) {
  if (i0 >= i1) return;
  const int lane = tid & 63;
  int ra = gmeta_item(S, i0, lane);
  int rb = gmeta_box(S, __builtin_amdgcn_readlane(ra, 0), lane);
  for (int i = i0; i < i1; i += step) {
    const GItem it = gmeta_unpack_item(ra);
    const GBoxLo G = gmeta_unpack_box(rb);
    const Bracket br = gmeta_unpack_bracket(rb);
    const bool more = i + step < i1;
    if (more) ra = gmeta_item(S, i + step, lane);
    gfill_item<T>(S, sm, slots, dst, p, it, G, br, tid, [&]() {
      if (more) rb = gmeta_box(S, __builtin_amdgcn_readlane(ra, 0), lane);
    });
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_gfill(DevSet S, const int* __restrict__ list, int count,
                                               const T* __restrict__ slots, T* __restrict__ pad,
                                               int64_t pad_stride) {
  __shared__ GfillSmem<T> sm;
  const int live = live_count(S, count);
  for (int b = blockIdx.y; b < live; b += gridDim.y) {
    const int p = list[b];
    gfill_items<T>(S, sm, slots, pad + (int64_t)b * pad_stride, p, S.gitem_off[p] + blockIdx.x,
                   S.gitem_off[p + 1], gridDim.x, threadIdx.x);
  }
}

// ---------------------------------------------------------------------------
// Courant rate and pressure accounting over the padded cells [-2, n+1]^3

// Signal-speed sum over the three directions, sum_d (|v_d| + c_f,d), of a
// cell with primitives w (0 for a cell that fails the checks); sets the error
// bits and counts floor hits.  Always IEEE arithmetic: the level of the step
// follows from it.  The Courant rate is the sum divided by dx.
template <class T>
__device__ __forceinline__ T cell_sum(const DevSet& S, const T* w) {
  T pr = w[4];
  T sum = T(0);
  if (!isfinite(w[0]) || !isfinite(pr)) {
    atomicOr(S.err, ERR_NONFINITE);
  } else if (!(w[0] > T(0))) {
    atomicOr(S.err, ERR_NEGATIVE);
  } else {
    if (S.p_floor > 0.0) {
      if (pr < T(S.p_floor)) {
        pr = T(S.p_floor);
        atomicAdd(S.floor_hits, 1ULL);
      }
    } else if (!(pr > T(0))) {
      atomicOr(S.err, ERR_NEGATIVE);
    }
    if (pr > T(0)) {
      const T ir = T(1) / w[0];
      const T a2 = T(S.gamma) * pr * ir;
      const T bb = (w[5] * w[5] + w[6] * w[6] + w[7] * w[7]) * ir;
      sum = fabs(w[1]) + fast_speed(a2, bb, (w[6] * w[6] + w[7] * w[7]) * ir);
      sum = sum + (fabs(w[2]) + fast_speed(a2, bb, (w[7] * w[7] + w[5] * w[5]) * ir));
      sum = sum + (fabs(w[3]) + fast_speed(a2, bb, (w[5] * w[5] + w[6] * w[6]) * ir));
      if (!isfinite(sum)) atomicOr(S.err, ERR_NONFINITE);
    }
  }
  return sum;
}

// Courant rate of padded cell (i, j, k) through the region table
template <class T>
__device__ __forceinline__ double cell_rate(const DevSet& S, const PatchCtx<T>& c, const RegionTab<T>& rt, int i,
                                            int j, int k) {
  T w[8], bxl, byl, bzl;
  load_cell(c, rt, i, j, k, T(S.gamma), T(0), w, bxl, byl, bzl);
  const double s = (double)cell_sum(S, w) / S.dx[c.p];
  if (!isfinite(s)) atomicOr(S.err, ERR_NONFINITE);
  return s;
}

// Signal-speed sum of interior cell (i, j, k), read straight from the patch's
// own slice
template <class T>
__device__ __forceinline__ T interior_sum(const DevSet& S, const PatchCtx<T>& c, int i, int j, int k) {
  using gptr = const T __attribute__((address_space(1)))*;
  const gptr u = (gptr)c.ownp;
  const int n = c.n;
  const int64_t e = ((int64_t)k * n + j) * n + i, n3 = (int64_t)n * n * n, nf = (int64_t)n * n * (n + 1);
  const int64_t fx = 5 * n3 + ((int64_t)k * n + j) * (n + 1) + i;
  const int64_t fy = 5 * n3 + nf + ((int64_t)k * (n + 1) + j) * n + i;
  const int64_t fz = 5 * n3 + 2 * nf + ((int64_t)k * n + j) * n + i;
  T w[8];
  prim_of<T>(u[e], u[n3 + e], u[2 * n3 + e], u[3 * n3 + e], u[4 * n3 + e], T(0.5) * (u[fx] + u[fx + 1]),
             T(0.5) * (u[fy] + u[fy + n]), T(0.5) * (u[fz] + u[fz + (int64_t)n * n]), T(S.gamma), T(0), w);
  return cell_sum(S, w);
}

// Padded coordinates of entry r of the two-layer guard shell around an n^3
// interior (N = n + 4): the two full planes below, the rings of the n
// interior planes, the two full planes above.
// Reciprocals of the shell's divisors (N = n + 4, N^2, the ring N^2 - n^2)
struct ShellRcp {
  float iN, iN2, iring;
};
__device__ __forceinline__ ShellRcp shell_rcp(int n) {
  const int N = n + 4;
  return {1.0f / (float)N, 1.0f / (float)(N * N), 1.0f / (float)(N * N - n * n)};
}
template <int FN>
__device__ __forceinline__ void shell_cell(int r, int n, const ShellRcp& rc, int& i, int& j, int& k) {
  const int N = n + 4, N2 = N * N, ring = N2 - n * n;
  if (r < 2 * N2 || r >= 2 * N2 + n * ring) {
    const int q = r < 2 * N2 ? r : r - n * ring;  // planes -2, -1 | n, n + 1
    const int kq = qdiv<FN>(q, N2, rc.iN2);
    k = kq - 2 + (r < 2 * N2 ? 0 : n);
    const int m = q - kq * N2;
    const int jq = qdiv<FN>(m, N, rc.iN);
    j = jq - 2;
    i = m - jq * N - 2;
    return;
  }
  const int q = r - 2 * N2;
  k = qdiv<FN>(q, ring, rc.iring);
  int m = q - k * ring;
  if (m < 2 * N) {  // rows -2, -1
    const int jq = qdiv<FN>(m, N, rc.iN);
    j = jq - 2;
    i = m - jq * N - 2;
  } else if (m < 2 * N + 4 * n) {  // rows 0 .. n-1: two cells on each side
    m -= 2 * N;
    j = m >> 2;
    const int s = m & 3;
    i = s < 2 ? s - 2 : n + s - 2;
  } else {  // rows n, n + 1
    m -= 2 * N + 4 * n;
    const int jq = qdiv<FN>(m, N, rc.iN);
    j = n + jq;
    i = m - jq * N - 2;
  }
}

// Interior cell cid of an n^3 patch (x fastest), rn = 1 / n
template <int FN>
__device__ __forceinline__ void interior_cell(int cid, int n, float rn, int& i, int& j, int& k) {
  const int jk = qdiv<FN>(cid, n, rn);
  i = cid - jk * n;
  k = qdiv<FN>(jk, n, rn);
  j = jk - k * n;
}

// largest value over the workgroup (red: one slot per wavefront)
__device__ inline double wg_max(double s, double* red, int tid, int nthr) {
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(s, off, 64);
    s = o > s ? o : s;
  }
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  double m = 0.0;
  for (int q = 0; q < nthr / 64; ++q) m = red[q] > m ? red[q] : m;
  return m;
}

template <class T>
__global__ __launch_bounds__(256) void k_courant(DevSet S, const int* __restrict__ list, int count,
                                                 const T* __restrict__ slots, const T* __restrict__ pad,
                                                 int64_t pad_stride, double* __restrict__ smax) {
  __shared__ RegionTab<T> rt;
  __shared__ double red[4];
  const int b = blockIdx.y;
  if (b >= live_count(S, count)) return;
  PatchCtx<T> c;
  c.p = list[b];
  c.n = S.n[c.p];
  c.ownp = slots + S.slot_off[c.p] + (int64_t)S.cur[c.p] * S.slice_len[c.p];
  for (int m = threadIdx.x; m < 108; m += blockDim.x)
    region_tab_init(S, slots, c.ownp, pad + (int64_t)b * pad_stride, c.n + 4, c.p, rt, m);
  __syncthreads();
  // several cells per thread (one table per workgroup): interior cells from
  // the own slice, the guard shell through the table; the largest signal-speed
  // sum, divided by dx once (monotonic: the largest per-cell rate)
  const int n = c.n, N = n + 4;
  const int first = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  T ms = T(0);
  const float rn = 1.0f / (float)n;
  const ShellRcp rc = shell_rcp(n);
  for (int cid = first; cid < n * n * n; cid += stride) {
    int i, j, k;
    interior_cell<0>(cid, n, rn, i, j, k);
    const T v = interior_sum(S, c, i, j, k);
    ms = v > ms ? v : ms;
  }
  for (int r = first; r < N * N * N - n * n * n; r += stride) {
    int i, j, k;
    shell_cell<0>(r, n, rc, i, j, k);
    T w[8], bxl, byl, bzl;
    load_cell(c, rt, i, j, k, T(S.gamma), T(0), w, bxl, byl, bzl);
    const T v = cell_sum(S, w);
    ms = v > ms ? v : ms;
  }
  const double m = wg_max((double)ms, red, threadIdx.x, blockDim.x) / S.dx[c.p];
  if (threadIdx.x == 0) {
    if (!isfinite(m)) atomicOr(S.err, ERR_NONFINITE);
    if (m > 0.0) atomicMax((unsigned long long*)(smax + b), (unsigned long long)__double_as_longlong(m));
  }
}

// Local time step of a patch whose whole update is one workgroup (LOCAL
// mode, one tile per patch): the Courant rate over the padded patch, its
// level, and the step record the publish kernel reads.  Returns dt to every
// thread of the workgroup.
template <class T, int FN = 0>
__device__ __forceinline__ double fused_local_dt(const DevSet& S, const PatchCtx<T>& c, const RegionTab<T>& rt,
                                                 const StepPtr& st, int bidx, int tid, int nthr, double* red) {
  // The largest signal-speed sum, divided by dx once: division by a positive
  // number is monotonic, so this is the largest of the per-cell rates.
  const int n = FN ? FN : c.n, N = n + 4;
  T ms = T(0);
  const float rn = 1.0f / (float)n;
  const ShellRcp rc = shell_rcp(n);
#pragma unroll 4
  for (int cid = tid; cid < n * n * n; cid += nthr) {
    int i, j, k;
    interior_cell<FN>(cid, n, rn, i, j, k);
    const T v = interior_sum(S, c, i, j, k);
    ms = v > ms ? v : ms;
  }
  const int nshell = N * N * N - n * n * n;
#pragma unroll 2
  for (int r = tid; r < nshell; r += nthr) {
    int i, j, k;
    shell_cell<FN>(r, n, rc, i, j, k);
    T w[8], bxl, byl, bzl;
    load_cell<T, Exact<T>, FN>(c, rt, i, j, k, T(S.gamma), T(0), w, bxl, byl, bzl);
    const T v = cell_sum(S, w);
    ms = v > ms ? v : ms;
  }
  const double m = wg_max((double)ms, red, tid, nthr) / S.dx[c.p];
  if (tid == 0 && !isfinite(m)) atomicOr(S.err, ERR_NONFINITE);
  int k = level_for(S, m, S.ticks[c.p]);
  if (k > S.kmax) {
    if (tid == 0) atomicOr(S.err, ERR_KMAX);
    k = S.kmax;
  }
  if (tid == 0) {
    st.k[bidx] = k;
    st.dtk[bidx] = (int64_t)1 << (S.kmax - k);
    st.dt[bidx] = S.dt_base * ldexp(1.0, -k);
  }
  return S.dt_base * ldexp(1.0, -k);
}

// ---------------------------------------------------------------------------
// the fused step

// Algorithmic HBM traffic of one patch update, added to S.algo_bytes: the own
// slice read and written once, every guard value of the two stencil layers
// read from one slice (exact time) or two (interpolated).  The boxes of the
// cell-centred regions (the first 27 keys of the patch) carry all five cell
// variables, the face boxes one field component.  Called by every thread of
// the first tile's workgroup (one box per thread, summed in LDS); the caller
// synchronises the workgroup before thread 0 publishes the sum.
__device__ inline void count_traffic(const DevSet& S, int p, int box0, int nbox, int64_t V, int tsz, int tid,
                                     int nthr, unsigned long long* acc) {
  if (tid == 0) atomicAdd(acc, 2ULL * (unsigned long long)V * (unsigned long long)tsz);
  const int ncellbox = S.rbox_off[p * 108 + 27] - box0;
  for (int m = tid; m < nbox; m += nthr) {
    const GBox& G = S.boxes[box0 + m];
    const Bracket b = bracket(S, G.q, S.ticks[p], S.tcur[p]);
    const unsigned long long cnt =
        (unsigned long long)(G.hi[0] - G.lo[0] + 1) * (G.hi[1] - G.lo[1] + 1) * (G.hi[2] - G.lo[2] + 1) *
        (m < ncellbox ? 5ULL : 1ULL);
    atomicAdd(acc, cnt * (b.oa == b.ob ? 1ULL : (b.oc < 0 ? 2ULL : 3ULL)) * (unsigned long long)tsz);
  }
}

// x-face flux of plane z with face index f (left cell f-1) and row j, from the
// predictor buffers; rotated order (rho, un, ut1, ut2, p, bt1, bt2)
template <class T>
__device__ __forceinline__ void face_states(const StepSmem<T>& sm, int d, int pa, int pb, T* l, T* r) {
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  const T(*sl)[MPRED] = (d == 0) ? sm.b.p.sx : sm.b.p.sy;
  const int ord[7] = {0, 1 + d, 1 + t1, 1 + t2, 4, 5 + t1, 5 + t2};
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    const int v = ord[m];
    l[m] = sm.b.p.h[v][pa] + T(0.5) * sl[v][pa];
    r[m] = sm.b.p.h[v][pb] - T(0.5) * sl[v][pb];
  }
}

// FN as for k_step2: a compile-time patch size for sets of equal one-tile
// patches whose guard regions are single same-resolution boxes.
template <class T, int FN>
__global__ __launch_bounds__(NTHR) void k_step(DevSet S, const int* __restrict__ list, int count,
                                               T* __restrict__ slots, const T* __restrict__ pad,
                                               int64_t pad_stride, StepPtr st, int tpa, int fuse_dt) {
  static_assert(FN >= 0 && FN <= MT, "a fixed patch size is one tile");
  __shared__ StepSmem<T> sm;
  const int tid = threadIdx.x;
  if (FN) tpa = 1;
  const int T2 = tpa * tpa;  // tile slots per patch
  const int w = blockIdx.x;
  const int bidx = (w / (8 * T2)) * 8 + (w % 8);
  const int tile = (w / 8) % T2;
  if (bidx >= live_count(S, count)) return;
  PatchCtx<T> c;
  c.p = list[bidx];
  const int n = c.n = FN ? FN : S.n[c.p];
  const int nt = (n + MT - 1) / MT;
  const int tx = tile % tpa, ty = tile / tpa;
  if (tx >= nt || ty >= nt) return;
  const int x0 = tx * n / nt, x1 = (tx + 1) * n / nt;
  const int y0 = ty * n / nt, y1 = (ty + 1) * n / nt;
  const int TX = x1 - x0, TY = y1 - y0;
  const int CX = TX + 4, CY = TY + 4, PX = TX + 2;
  const bool lastx = (x1 == n), lasty = (y1 == n), firstx = (x0 == 0), firsty = (y0 == 0);
  // index decoding of the face and edge phases: with a compile-time patch
  // size the divisors are constants; otherwise quotients through their
  // single-precision reciprocals (small_div), uniform over the workgroup
  auto uniform_rcp = [](int d) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(1.0f / (float)d)));
  };
  const float iTX = uniform_rcp(TX), iTX1 = uniform_rcp(TX + 1), iTX2 = uniform_rcp(TX + 2);
  auto qd = [&](int r, int d, float inv) -> int { return qdiv<FN>(r, d, inv); };
  const int box0 = S.rbox_off[c.p * 108];
  const int nbox = S.rbox_off[c.p * 108 + 108] - box0;
  const int64_t V = S.slice_len[c.p];
  const int64_t own = S.slot_off[c.p] + (int64_t)S.cur[c.p] * V;
  T* const outp = slots + S.slot_off[c.p] + (int64_t)((S.cur[c.p] + 1) % S.nslots) * V;
  c.ownp = slots + own;
  for (int m = tid; m < 108; m += NTHR)
    region_tab_init(S, (const T*)slots, (const T*)c.ownp, pad + (int64_t)bidx * pad_stride, n + 4, c.p, sm.rt, m);
  const T gamma = T(S.gamma), pfloor = T(S.p_floor);
  __shared__ unsigned long long traffic;
  __shared__ double red[NTHR / 64];
  if (tid == 0) traffic = 0;
  __syncthreads();
  if (tile == 0) count_traffic(S, c.p, box0, nbox, V, (int)sizeof(T), tid, NTHR, &traffic);
  const double dt = fuse_dt ? fused_local_dt<T, FN>(S, c, sm.rt, st, bidx, tid, NTHR, red) : st.dt[bidx];
  const T dtdx = T(dt / S.dx[c.p]);
  const T hdtdx = T(0.5) * dtdx;
  __syncthreads();
  if (tile == 0 && tid == 0) atomicAdd(S.algo_bytes, traffic);

  // column of this thread
  const bool col = tid < CX * CY;
  const int ca = tid % CX, cb = tid / CX;
  const int ci = x0 - 2 + ca, cj = y0 - 2 + cb;
  const bool pred = col && ca >= 1 && ca <= CX - 2 && cb >= 1 && cb <= CY - 2;
  const int pc = (ca - 1) + (cb - 1) * PX;  // predictor index (valid if pred)
  const bool own_cell = col && ci >= x0 && ci < x1 && cj >= y0 && cj < y1;
  const bool own_bx = col && cj >= y0 && cj < y1 && ((ci >= x0 && ci < x1) || (lastx && ci == n));
  const bool own_by = col && ci >= x0 && ci < x1 && ((cj >= y0 && cj < y1) || (lasty && cj == n));
  // halo faces are computed by several tiles; each counts only its own
  auto own_c = [&](int v, int lo, int hi, bool first, bool last) {
    return (v >= lo && v < hi) || (first && v < 0) || (last && v >= n);
  };

  T Wm[8], W0[8], Wp[8];
  T bx0 = 0, by0 = 0, bz0 = 0, bxp = 0, byp = 0, bzp = 0, dummy;
  if (col) {
    load_cell<T, Exact<T>, FN>(c, sm.rt, ci, cj, -2, gamma, pfloor, Wm, dummy, dummy, dummy);
    load_cell<T, Exact<T>, FN>(c, sm.rt, ci, cj, -1, gamma, pfloor, W0, bx0, by0, bz0);
  }
  T tl[7];     // top state of the previous plane's z-face (rotated z, x, y)
  T dzl = 0;   // normal-field increment of the previous plane
  T fzl[5], fzc[5], duxy[5], dnew[5];
  T pbx = 0, pby = 0;
#pragma unroll
  for (int q = 0; q < 5; ++q) fzl[q] = fzc[q] = duxy[q] = dnew[q] = T(0);
#pragma unroll
  for (int q = 0; q < 7; ++q) tl[q] = T(0);
  const int nxf = (TX + 1) * (TY + 2), nyf = (TX + 2) * (TY + 1);

  for (int z = -1; z <= n; ++z) {
    // ---- P1: load plane z+1; publish plane z primitives and lo-face fields
    if (col) {
      load_cell<T, Exact<T>, FN>(c, sm.rt, ci, cj, z + 1, gamma, pfloor, Wp, bxp, byp, bzp);
#pragma unroll
      for (int v = 0; v < 8; ++v) sm.a.w[v][tid] = W0[v];
      sm.bf[0][tid] = bx0;
      sm.bf[1][tid] = by0;
    }
    __syncthreads();
    // ---- P2: slopes, Hancock predictor, z-face flux at face z, cell EMF
    if (pred) {
      T sl[3][8];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const T c0 = W0[v];
        sl[0][v] = van_leer(c0 - sm.a.w[v][tid - 1], sm.a.w[v][tid + 1] - c0);
        sl[1][v] = van_leer(c0 - sm.a.w[v][tid - CX], sm.a.w[v][tid + CX] - c0);
        sl[2][v] = van_leer(c0 - Wm[v], Wp[v] - c0);
      }
      sl[0][5] = T(0);
      sl[1][6] = T(0);
      sl[2][7] = T(0);
      const T ir = T(1) / W0[0];
      T sum[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) sum[v] = T(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        const T un = W0[1 + d], bn = W0[5 + d], b1 = W0[5 + t1], b2 = W0[5 + t2];
        const T* s = sl[d];
        sum[0] = sum[0] + (un * s[0] + W0[0] * s[1 + d]);
        sum[1 + d] = sum[1 + d] + (un * s[1 + d] + (s[4] + b1 * s[5 + t1] + b2 * s[5 + t2]) * ir);
        sum[1 + t1] = sum[1 + t1] + (un * s[1 + t1] - bn * s[5 + t1] * ir);
        sum[1 + t2] = sum[1 + t2] + (un * s[1 + t2] - bn * s[5 + t2] * ir);
        sum[4] = sum[4] + (un * s[4] + gamma * W0[4] * s[1 + d]);
        sum[5 + t1] = sum[5 + t1] + (un * s[5 + t1] + b1 * s[1 + d] - bn * s[1 + t1]);
        sum[5 + t2] = sum[5 + t2] + (un * s[5 + t2] + b2 * s[1 + d] - bn * s[1 + t2]);
      }
      T H[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        H[v] = W0[v] - hdtdx * sum[v];
        sm.b.p.h[v][pc] = H[v];
        sm.b.p.sx[v][pc] = sl[0][v];
        sm.b.p.sy[v][pc] = sl[1][v];
      }
      sm.b.p.db[0][pc] = H[5] - W0[5];
      sm.b.p.db[1][pc] = H[6] - W0[6];
      const T dz = H[7] - W0[7];
      // rotated (z, x, y): rho, vz, vx, vy, p, bx, by
      const int ord[7] = {0, 3, 1, 2, 4, 5, 6};
      T rb[7];
#pragma unroll
      for (int m = 0; m < 7; ++m) rb[m] = H[ord[m]] - T(0.5) * sl[2][ord[m]];
      if (z >= 0) {
        T l[7], r[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) {
          l[m] = tl[m];
          r[m] = rb[m];
        }
        T bn = bz0 + T(0.5) * (dzl + dz);
        if (!(l[0] > T(0)) || !(l[4] > T(0)) || !(r[0] > T(0)) || !(r[4] > T(0))) {
#pragma unroll
          for (int m = 0; m < 7; ++m) {
            l[m] = Wm[ord[m]];
            r[m] = W0[ord[m]];
          }
          bn = bz0;
          if (own_c(ci, x0, x1, firstx, lastx) && own_c(cj, y0, y1, firsty, lasty))
            atomicAdd(S.fallback, 1ULL);
        }
        T f[8];
        hlld_flux(l, r, bn, gamma, f);
        // unrotated: mass, mx, my, mz, energy; induction fluxes of Bx, By
        fzc[0] = f[0];
        fzc[1] = f[2];
        fzc[2] = f[3];
        fzc[3] = f[1];
        fzc[4] = f[4];
        sm.fz[0][pc] = f[7];  // upwind speed (orientation of the edge EMFs)
        sm.fz[1][pc] = f[5];
        sm.fz[2][pc] = f[6];
      }
#pragma unroll
      for (int m = 0; m < 7; ++m) tl[m] = H[ord[m]] + T(0.5) * sl[2][ord[m]];
      dzl = dz;
      // E = -v x B of the half-step state
      sm.ecc[z & 1][0][pc] = H[3] * H[6] - H[2] * H[7];
      sm.ecc[z & 1][1][pc] = H[1] * H[7] - H[3] * H[5];
      sm.ecc[z & 1][2][pc] = H[2] * H[5] - H[1] * H[6];
    }
    __syncthreads();
    // ---- P3: x- and y-face fluxes of plane z
    for (int m = tid; m < nxf + nyf; m += NTHR) {
      const int d = (m < nxf) ? 0 : 1;
      int pa, pb, fa, fb, e;
      T bface;
      int cix, cjx;  // cell (i, j) right/upper of the face
      if (d == 0) {
        e = m;
        const int jr = qd(e, TX + 1, iTX1), fl = e - jr * (TX + 1);
        pa = fl + jr * PX;
        pb = pa + 1;
        cix = x0 + fl;
        cjx = y0 - 1 + jr;
        fa = (cix - (x0 - 2)) + (cjx - (y0 - 2)) * CX;
        fb = fa;
        bface = sm.bf[0][fa];
      } else {
        e = m - nxf;
        const int gl = qd(e, TX + 2, iTX2), ir = e - gl * (TX + 2);
        pa = ir + gl * PX;
        pb = pa + PX;
        cix = x0 - 1 + ir;
        cjx = y0 + gl;
        fa = (cix - (x0 - 2)) + (cjx - (y0 - 2)) * CX;
        fb = fa;
        bface = sm.bf[1][fa];
      }
      (void)fb;
      T l[7], r[7];
      face_states(sm, d, pa, pb, l, r);
      T bn = bface + T(0.5) * (sm.b.p.db[d][pa] + sm.b.p.db[d][pb]);
      if (!(l[0] > T(0)) || !(l[4] > T(0)) || !(r[0] > T(0)) || !(r[4] > T(0))) {
        // first-order fallback: primitives of the two cells at t^n
        {
          const FaceStates<T> fs = fallback_states(c, sm.rt, d, cix, cjx, z, gamma, pfloor);
#pragma unroll
          for (int q = 0; q < 7; ++q) {
            l[q] = fs.l[q];
            r[q] = fs.r[q];
          }
        }
        bn = bface;
        const bool owned = (d == 0) ? (own_c(cix, x0, x1, firstx, false) || (lastx && cix == n)) &&
                                          own_c(cjx, y0, y1, firsty, lasty)
                                    : own_c(cix, x0, x1, firstx, lastx) &&
                                          (own_c(cjx, y0, y1, firsty, false) || (lasty && cjx == n));
        if (owned) atomicAdd(S.fallback, 1ULL);
      }
      T f[8];
      hlld_flux(l, r, bn, gamma, f);
      T(*F)[MXF] = (d == 0) ? sm.a.f.fx : sm.a.f.fy;
      const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
      F[0][e] = f[0];
      F[1 + d][e] = f[1];
      F[1 + t1][e] = f[2];
      F[1 + t2][e] = f[3];
      F[4][e] = f[4];
      F[5 + d][e] = f[7];  // the normal field has no flux: the slot holds the upwind speed
      F[5 + t1][e] = f[5];
      F[5 + t2][e] = f[6];
    }
    __syncthreads();
    // ---- P4: edge EMFs (upwinded by the sign of the face upwind speed) and x/y flux sums
    {
      auto up = [](T mflux, T a, T b) -> T {
        if (mflux > T(0)) return a;
        if (mflux < T(0)) return b;
        return T(0.5) * (a + b);
      };
      auto edge = [&](T A, T B, T C, T D, T mA, T mB, T mC, T mD, T c00, T c10, T c01, T c11) -> T {
        const T dc14 = up(mA, c01 - D, c11 - C);
        const T dc34 = up(mB, D - c00, C - c10);
        const T db14 = up(mC, c10 - B, c11 - A);
        const T db34 = up(mD, B - c00, A - c01);
        return T(0.25) * (A + B + C + D) + T(0.25) * ((dc34 - dc14) + (db34 - db14));
      };
      const int pz = z & 1, pzm = (z - 1) & 1;
      auto P = [&](int i, int j) { return (i - (x0 - 1)) + (j - (y0 - 1)) * PX; };
      auto XF = [&](int f, int j) { return (f - x0) + (j - (y0 - 1)) * (TX + 1); };
      auto YF = [&](int i, int g) { return (i - (x0 - 1)) + (g - y0) * (TX + 2); };
      const int nez = (z >= 0 && z < n) ? (TX + 1) * (TY + 1) : 0;
      const int nex = (z >= 0) ? TX * (TY + 1) : 0;
      const int ney = (z >= 0) ? (TX + 1) * TY : 0;
      // each kind of edge starts on a wavefront boundary (no wavefront runs
      // two of the branches)
      const int ex0 = (nez + 63) & ~63, ey0 = ex0 + ((nex + 63) & ~63);
      for (int m = tid; m < ey0 + ney; m += NTHR) {
        if (m < nez) {  // E_z in plane z at (x-face f, y-face g)
          const int mq = qd(m, TX + 1, iTX1);
          const int f = x0 + (m - mq * (TX + 1)), g = y0 + mq;
          const T A = -sm.a.f.fx[6][XF(f, g)], B = -sm.a.f.fx[6][XF(f, g - 1)];
          const T C = sm.a.f.fy[5][YF(f, g)], D = sm.a.f.fy[5][YF(f - 1, g)];
          const T v = edge(A, B, C, D, sm.a.f.fx[5][XF(f, g)], sm.a.f.fx[5][XF(f, g - 1)],
                           sm.a.f.fy[6][YF(f, g)], sm.a.f.fy[6][YF(f - 1, g)], sm.ecc[pz][2][P(f - 1, g - 1)],
                           sm.ecc[pz][2][P(f, g - 1)], sm.ecc[pz][2][P(f - 1, g)], sm.ecc[pz][2][P(f, g)]);
          sm.b.e.ez[m] = v;
        } else if (m >= ex0 && m < ex0 + nex) {  // E_x at z-face z, (x-cell i, y-face g)
          const int e = m - ex0;
          const int eq = qd(e, TX, iTX);
          const int i = x0 + (e - eq * TX), g = y0 + eq;
          const T A = -sm.a.f.fy[7][YF(i, g)], B = -sm.py[1][YF(i, g)];
          const T C = sm.fz[2][P(i, g)], D = sm.fz[2][P(i, g - 1)];
          const T v = edge(A, B, C, D, sm.a.f.fy[6][YF(i, g)], sm.py[0][YF(i, g)], sm.fz[0][P(i, g)],
                           sm.fz[0][P(i, g - 1)], sm.ecc[pzm][0][P(i, g - 1)], sm.ecc[pzm][0][P(i, g)],
                           sm.ecc[pz][0][P(i, g - 1)], sm.ecc[pz][0][P(i, g)]);
          sm.b.e.ex[e] = v;
        } else if (m >= ey0) {  // E_y at z-face z, (x-face f, y-cell j)
          const int e = m - ey0;
          const int eq = qd(e, TX + 1, iTX1);
          const int f = x0 + (e - eq * (TX + 1)), j = y0 + eq;
          const T A = -sm.fz[1][P(f, j)], B = -sm.fz[1][P(f - 1, j)];
          const T C = sm.a.f.fx[7][XF(f, j)], D = sm.px[1][XF(f, j)];
          const T v = edge(A, B, C, D, sm.fz[0][P(f, j)], sm.fz[0][P(f - 1, j)], sm.a.f.fx[5][XF(f, j)],
                           sm.px[0][XF(f, j)], sm.ecc[pzm][1][P(f - 1, j)], sm.ecc[pz][1][P(f - 1, j)],
                           sm.ecc[pzm][1][P(f, j)], sm.ecc[pz][1][P(f, j)]);
          sm.b.e.ey[e] = v;
        }
      }
      if (own_cell && z >= 0 && z < n) {
#pragma unroll
        for (int q = 0; q < 5; ++q)
          dnew[q] = (sm.a.f.fx[q][XF(ci + 1, cj)] - sm.a.f.fx[q][XF(ci, cj)]) +
                    (sm.a.f.fy[q][YF(ci, cj + 1)] - sm.a.f.fy[q][YF(ci, cj)]);
      }
    }
    __syncthreads();
    // ---- P5: write plane z-1 (cells, Bx, By) and face z (Bz); carry partials
    {
      const int n3 = n * n * n;
      (void)n3;
      auto EZ = [&](int f, int g) { return sm.b.e.ez[(f - x0) + (g - y0) * (TX + 1)]; };
      auto EX = [&](int i, int g) { return sm.b.e.ex[(i - x0) + (g - y0) * TX]; };
      auto EY = [&](int f, int j) { return sm.b.e.ey[(f - x0) + (j - y0) * (TX + 1)]; };
      if (z >= 1) {
        const int zc = z - 1;
        if (own_cell) {
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            const T du = duxy[q] + (fzc[q] - fzl[q]);
            const int64_t e = scell(n, q, ci, cj, zc);
            outp[e] = c.ownp[e] - dtdx * du;
          }
        }
        if (own_bx) {
          const int64_t e = sface(n, 0, ci, cj, zc);
          outp[e] = c.ownp[e] - dtdx * (pbx - EY(ci, cj));
        }
        if (own_by) {
          const int64_t e = sface(n, 1, ci, cj, zc);
          outp[e] = c.ownp[e] - dtdx * (pby + EX(ci, cj));
        }
      }
      if (z >= 0 && z < n) {
        if (own_bx) pbx = (EZ(ci, cj + 1) - EZ(ci, cj)) + EY(ci, cj);
        if (own_by) pby = -EX(ci, cj) - (EZ(ci + 1, cj) - EZ(ci, cj));
      }
      if (z >= 0 && own_cell) {
        const T curl = (EY(ci + 1, cj) - EY(ci, cj)) - (EX(ci, cj + 1) - EX(ci, cj));
        const int64_t e = sface(n, 2, ci, cj, z);
        outp[e] = c.ownp[e] - dtdx * curl;
      }
      for (int m = tid; m < nxf; m += NTHR) {
        sm.px[0][m] = sm.a.f.fx[5][m];
        sm.px[1][m] = sm.a.f.fx[7][m];
      }
      for (int m = tid; m < nyf; m += NTHR) {
        sm.py[0][m] = sm.a.f.fy[6][m];
        sm.py[1][m] = sm.a.f.fy[7][m];
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        duxy[q] = dnew[q];
        fzl[q] = fzc[q];
      }
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        Wm[v] = W0[v];
        W0[v] = Wp[v];
      }
      bx0 = bxp;
      by0 = byp;
      bz0 = bzp;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The fused step, wide variant (single precision): 1024 threads per tile.
// The three planes of primitives the z-slopes need live in an LDS ring instead
// of registers, and the x-, y- and z-face Riemann problems of a plane are
// solved in one phase (about one face per thread), so the per-thread state
// carried through the march is a handful of registers and four waves share
// each SIMD.

constexpr int NTHR2 = 1024;

template <class T> struct Step2Smem {
  T w[3][8][MCOL];      // primitives of planes z-1, z, z+1 (slot = plane mod 3)
  T bfc[3][3][MCOL];    // t^n field on the low x-, y- and z-face of each column (slot = plane mod 3)
  union B {
    struct {
      T h[8][MPRED];    // half-step primitives
      T sx[8][MPRED];   // x-slopes
      T sy[8][MPRED];   // y-slopes
      T db[2][MPRED];   // predictor increments of the cell-centred Bx, By
    } p;
    struct {
      T ez[(MT + 1) * (MT + 1)];
      T ex[MT * (MT + 1)];
      T ey[(MT + 1) * MT];
    } e;
  } b;
  T fx[8][MXF];         // x-face fluxes of plane z (slot 5: upwind speed)
  T fy[8][MXF];         // y-face fluxes of plane z (slot 6: upwind speed)
  T fz[8][MPRED];       // face z: mass, mx, my, mz, energy, Bx and By induction, upwind speed
  T zt[2][7][MPRED];    // top face state (z-rotated order) of each cell (slot = plane mod 2)
  T zb[7][MPRED];       // bottom face state of plane z
  T dz[2][MPRED];       // predictor increment of the cell-centred Bz (slot = plane mod 2)
  T px[2][MXF];         // previous plane: x-face upwind speed and Bz induction flux
  T py[2][MXF];         // previous plane: y-face upwind speed and Bz induction flux
  T ecc[2][3][MPRED];   // cell-centred EMF -v x B of the half-step state (slot = plane mod 2)
  RegionTab<T> rt;
  unsigned long long traffic;  // algorithmic bytes of the update (tile 0)
  double red[NTHR2 / 64];      // one slot per wavefront: the Courant-rate maximum
};

__device__ __forceinline__ int mod3(int z) { return (z + 3) % 3; }

// FN > 0: every patch has FN <= MT cells per edge (one tile each) and every
// guard region is a single same-resolution box, so the patch and region
// strides are compile-time constants; FN = 0 takes them at run time.
// One tile of one patch update by one workgroup of NTHR2 threads: bidx is the
// entry of the step record (st) and of the padded buffer, p the patch.
template <class T, int FN>
__device__ __forceinline__ void step2_tile(const DevSet& S, Step2Smem<T>& sm, T* __restrict__ slots,
                                           const T* __restrict__ pad, int64_t pad_stride, const StepPtr& st,
                                           int bidx, int p, int tile, int tpa, int fuse_dt, int tid) {
  static_assert(sizeof(T) == 4, "the wide step kernel is the single-precision variant");
  static_assert(FN >= 0 && FN <= MT, "a fixed patch size is one tile");
  using M = FastF32;
  PatchCtx<T> c;
  c.p = p;
  const int n = c.n = FN ? FN : S.n[c.p];
  const int nt = (n + MT - 1) / MT;
  const int tx = tile % tpa, ty = tile / tpa;
  if (tx >= nt || ty >= nt) return;
  const int x0 = tx * n / nt, x1 = (tx + 1) * n / nt;
  const int y0 = ty * n / nt, y1 = (ty + 1) * n / nt;
  const int TX = x1 - x0, TY = y1 - y0;
  const int CX = TX + 4, CY = TY + 4, PX = TX + 2, PY = TY + 2;
  const bool lastx = (x1 == n), lasty = (y1 == n), firstx = (x0 == 0), firsty = (y0 == 0);
  // index decoding of the face and edge phases: with a compile-time patch
  // size the divisors are constants; otherwise quotients through their
  // single-precision reciprocals (small_div), uniform over the workgroup
  auto uniform_rcp = [](int d) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(1.0f / (float)d)));
  };
  const float iTX = uniform_rcp(TX), iTX1 = uniform_rcp(TX + 1), iTX2 = uniform_rcp(TX + 2), iPX = uniform_rcp(PX);
  auto qd = [&](int r, int d, float inv) -> int { return qdiv<FN>(r, d, inv); };
  const int box0 = S.rbox_off[c.p * 108];
  const int nbox = S.rbox_off[c.p * 108 + 108] - box0;
  const int64_t V = S.slice_len[c.p];
  const int64_t own = S.slot_off[c.p] + (int64_t)S.cur[c.p] * V;
  T* const outp = slots + S.slot_off[c.p] + (int64_t)((S.cur[c.p] + 1) % S.nslots) * V;
  c.ownp = slots + own;
  for (int m = tid; m < 108; m += NTHR2)
    region_tab_init(S, (const T*)slots, (const T*)c.ownp, pad + (int64_t)bidx * pad_stride, n + 4, c.p, sm.rt, m);
  const T gamma = T(S.gamma), pfloor = T(S.p_floor);
  if (tid == 0) sm.traffic = 0;
  __syncthreads();
  if (tile == 0) count_traffic(S, c.p, box0, nbox, V, (int)sizeof(T), tid, NTHR2, &sm.traffic);
  const double dt = fuse_dt ? fused_local_dt<T, FN>(S, c, sm.rt, st, bidx, tid, NTHR2, sm.red) : st.dt[bidx];
  const T dtdx = T(dt / S.dx[c.p]);
  const T hdtdx = T(0.5) * dtdx;
  __syncthreads();
  if (tile == 0 && tid == 0) atomicAdd(S.algo_bytes, sm.traffic);

  // column of this thread (load phase) and its predictor cell.  The lane
  // indices are re-declared opaque at the start of every phase (reopen), so
  // the addresses derived from them are recomputed there instead of being
  // hoisted out of the march and held (or spilled) through the face phase.
  const bool col = tid < CX * CY;
  const int ca = tid % CX, cb = tid / CX;
  int ci = x0 - 2 + ca, cj = y0 - 2 + cb;
  const bool pred = col && ca >= 1 && ca <= CX - 2 && cb >= 1 && cb <= CY - 2;
  int pc = (ca - 1) + (cb - 1) * PX;
  int lane = tid;
  auto reopen = [&]() {
    DSP_OPAQUE(lane);
    DSP_OPAQUE(ci);
    DSP_OPAQUE(cj);
    DSP_OPAQUE(pc);
  };
  const bool own_cell = col && ci >= x0 && ci < x1 && cj >= y0 && cj < y1;
  const bool own_bx = col && cj >= y0 && cj < y1 && ((ci >= x0 && ci < x1) || (lastx && ci == n));
  const bool own_by = col && ci >= x0 && ci < x1 && ((cj >= y0 && cj < y1) || (lasty && cj == n));
  auto own_c = [&](int v, int lo, int hi, bool first, bool last) {
    return (v >= lo && v < hi) || (first && v < 0) || (last && v >= n);
  };
  // Plane z + 2 is read during the face phase of plane z (its ring slot,
  // that of plane z - 1, is free by then), which saves a load phase and its
  // barrier.  PIPE = false keeps the load of plane z + 1 in a phase of its own.
  constexpr bool PIPE = true;
  auto store_plane = [&](int z, const T* wv, T bx, T by, T bz) {
    const int s3 = mod3(z);
#pragma unroll
    for (int v = 0; v < 8; ++v) sm.w[s3][v][lane] = wv[v];
    sm.bfc[s3][0][lane] = bx;
    sm.bfc[s3][1][lane] = by;
    sm.bfc[s3][2][lane] = bz;
  };
  auto load_plane = [&](int z) {  // primitives and low-face fields of plane z into the rings
    T wv[8], bx, by, bz;
    load_cell<T, M, FN>(c, sm.rt, ci, cj, z, gamma, pfloor, wv, bx, by, bz);
    store_plane(z, wv, bx, by, bz);
  };
  if (col) {
    load_plane(-2);
    load_plane(-1);
    if (PIPE) load_plane(0);
  }
  // without a load phase, the first predictor phase reads these planes next
  if (PIPE) __syncthreads();
  T acc[5];  // x/y flux differences of the pending cell minus its bottom z-flux
  T dnew[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) acc[q] = dnew[q] = T(0);
  T pbx = 0, pby = 0;
  const int nxf = (TX + 1) * (TY + 2), nyf = (TX + 2) * (TY + 1), nzf = PX * PY;

  for (int z = -1; z <= n; ++z) {
    // ---- P1: load plane z+1
    if (!PIPE) {
      reopen();
      if (col) load_plane(z + 1);
      __syncthreads();
    }
    // ---- P2: slopes, Hancock predictor, z-face states and cell EMF of plane z
    reopen();
    if (pred) {
      const int sm3 = mod3(z - 1), s0 = mod3(z), sp3 = mod3(z + 1);
      T W0[8], sl[3][8];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const T c0 = sm.w[s0][v][lane];
        W0[v] = c0;
        sl[0][v] = van_leer<T, M>(c0 - sm.w[s0][v][lane - 1], sm.w[s0][v][lane + 1] - c0);
        sl[1][v] = van_leer<T, M>(c0 - sm.w[s0][v][lane - CX], sm.w[s0][v][lane + CX] - c0);
        sl[2][v] = van_leer<T, M>(c0 - sm.w[sm3][v][lane], sm.w[sp3][v][lane] - c0);
      }
      sl[0][5] = T(0);
      sl[1][6] = T(0);
      sl[2][7] = T(0);
      const T ir = M::rcp(W0[0]);
      T sum[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) sum[v] = T(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        const T un = W0[1 + d], bn = W0[5 + d], b1 = W0[5 + t1], b2 = W0[5 + t2];
        const T* s = sl[d];
        sum[0] = sum[0] + (un * s[0] + W0[0] * s[1 + d]);
        sum[1 + d] = sum[1 + d] + (un * s[1 + d] + (s[4] + b1 * s[5 + t1] + b2 * s[5 + t2]) * ir);
        sum[1 + t1] = sum[1 + t1] + (un * s[1 + t1] - bn * s[5 + t1] * ir);
        sum[1 + t2] = sum[1 + t2] + (un * s[1 + t2] - bn * s[5 + t2] * ir);
        sum[4] = sum[4] + (un * s[4] + gamma * W0[4] * s[1 + d]);
        sum[5 + t1] = sum[5 + t1] + (un * s[5 + t1] + b1 * s[1 + d] - bn * s[1 + t1]);
        sum[5 + t2] = sum[5 + t2] + (un * s[5 + t2] + b2 * s[1 + d] - bn * s[1 + t2]);
      }
      T H[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        H[v] = W0[v] - hdtdx * sum[v];
        sm.b.p.h[v][pc] = H[v];
        sm.b.p.sx[v][pc] = sl[0][v];
        sm.b.p.sy[v][pc] = sl[1][v];
      }
      sm.b.p.db[0][pc] = H[5] - W0[5];
      sm.b.p.db[1][pc] = H[6] - W0[6];
      sm.dz[z & 1][pc] = H[7] - W0[7];
      const int ord[7] = {0, 3, 1, 2, 4, 5, 6};  // z-rotated: rho, vz, vx, vy, p, bx, by
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        sm.zt[z & 1][m][pc] = H[ord[m]] + T(0.5) * sl[2][ord[m]];
        sm.zb[m][pc] = H[ord[m]] - T(0.5) * sl[2][ord[m]];
      }
      sm.ecc[z & 1][0][pc] = H[3] * H[6] - H[2] * H[7];
      sm.ecc[z & 1][1][pc] = H[1] * H[7] - H[3] * H[5];
      sm.ecc[z & 1][2][pc] = H[2] * H[5] - H[1] * H[6];
    }
    __syncthreads();
    // ---- P3: x- and y-face fluxes of plane z, z-face fluxes at face z
    reopen();
    const bool ld = PIPE && col && z + 2 <= n + 1;
    RawCell<T> raw;
    if constexpr (PIPE) {
      if (ld) raw_issue<T, FN>(n, sm.rt, ci, cj, z + 2, raw);
    }
    // the z-faces start on a wavefront boundary, so that no wavefront
    // evaluates both kinds of face (the HLLD flux twice)
    const int zf0 = (nxf + nyf + 63) & ~63;
    const int nface = z >= 0 ? zf0 + nzf : nxf + nyf;
    for (int m = lane; m < nface; m += NTHR2) {
      T l[7], r[7], bn, f[8];
      if (m < nxf + nyf) {
        const int d = (m < nxf) ? 0 : 1;
        int e, pa, pb, cix, cjx;
        T bface;
        if (d == 0) {
          e = m;
          const int jr = qd(e, TX + 1, iTX1), fl = e - jr * (TX + 1);
          pa = fl + jr * PX;
          pb = pa + 1;
          cix = x0 + fl;
          cjx = y0 - 1 + jr;
        } else {
          e = m - nxf;
          const int gl = qd(e, TX + 2, iTX2), ir = e - gl * (TX + 2);
          pa = ir + gl * PX;
          pb = pa + PX;
          cix = x0 - 1 + ir;
          cjx = y0 + gl;
        }
        bface = sm.bfc[mod3(z)][d][(cix - (x0 - 2)) + (cjx - (y0 - 2)) * CX];
        const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        const T(*slp)[MPRED] = (d == 0) ? sm.b.p.sx : sm.b.p.sy;
        const int ord[7] = {0, 1 + d, 1 + t1, 1 + t2, 4, 5 + t1, 5 + t2};
#pragma unroll
        for (int q = 0; q < 7; ++q) {
          const int v = ord[q];
          l[q] = sm.b.p.h[v][pa] + T(0.5) * slp[v][pa];
          r[q] = sm.b.p.h[v][pb] - T(0.5) * slp[v][pb];
        }
        bn = bface + T(0.5) * (sm.b.p.db[d][pa] + sm.b.p.db[d][pb]);
        if (!(l[0] > T(0)) || !(l[4] > T(0)) || !(r[0] > T(0)) || !(r[4] > T(0))) {
          {
          const FaceStates<T> fs = fallback_states<T, M>(c, sm.rt, d, cix, cjx, z, gamma, pfloor);
#pragma unroll
          for (int q = 0; q < 7; ++q) {
            l[q] = fs.l[q];
            r[q] = fs.r[q];
          }
        }
          bn = bface;
          const bool owned = (d == 0) ? (own_c(cix, x0, x1, firstx, false) || (lastx && cix == n)) &&
                                            own_c(cjx, y0, y1, firsty, lasty)
                                      : own_c(cix, x0, x1, firstx, lastx) &&
                                            (own_c(cjx, y0, y1, firsty, false) || (lasty && cjx == n));
          if (owned) atomicAdd(S.fallback, 1ULL);
        }
        hlld_flux<T, M>(l, r, bn, gamma, f);
        T(*F)[MXF] = (d == 0) ? sm.fx : sm.fy;
        F[0][e] = f[0];
        F[1 + d][e] = f[1];
        F[1 + t1][e] = f[2];
        F[1 + t2][e] = f[3];
        F[4][e] = f[4];
        F[5 + d][e] = f[7];  // the normal field has no flux: the slot holds the upwind speed
        F[5 + t1][e] = f[5];
        F[5 + t2][e] = f[6];
      } else if (m >= zf0) {
        const int q = m - zf0;  // predictor cell of the face's upper cell
        const int qb = qd(q, PX, iPX), qa = q - qb * PX;
        const int cix = x0 - 1 + qa, cjx = y0 - 1 + qb;
        const int cq = (qa + 1) + (qb + 1) * CX;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
          l[k] = sm.zt[(z - 1) & 1][k][q];
          r[k] = sm.zb[k][q];
        }
        const T bface = sm.bfc[mod3(z)][2][cq];
        bn = bface + T(0.5) * (sm.dz[(z - 1) & 1][q] + sm.dz[z & 1][q]);
        if (!(l[0] > T(0)) || !(l[4] > T(0)) || !(r[0] > T(0)) || !(r[4] > T(0))) {
          {
          const FaceStates<T> fs = fallback_states<T, M>(c, sm.rt, 2, cix, cjx, z, gamma, pfloor);
#pragma unroll
          for (int q = 0; q < 7; ++q) {
            l[q] = fs.l[q];
            r[q] = fs.r[q];
          }
        }
          bn = bface;
          if (own_c(cix, x0, x1, firstx, lastx) && own_c(cjx, y0, y1, firsty, lasty)) atomicAdd(S.fallback, 1ULL);
        }
        hlld_flux<T, M>(l, r, bn, gamma, f);
        sm.fz[0][q] = f[0];
        sm.fz[1][q] = f[2];
        sm.fz[2][q] = f[3];
        sm.fz[3][q] = f[1];
        sm.fz[4][q] = f[4];
        sm.fz[5][q] = f[5];
        sm.fz[6][q] = f[6];
        sm.fz[7][q] = f[7];
      }
    }
    if constexpr (PIPE) {
      if (ld) {
        T wv[8], bx, by, bz;
        raw_finish<T, M, FN>(n, sm.rt, ci, cj, z + 2, raw, gamma, pfloor, wv, bx, by, bz);
        store_plane(z + 2, wv, bx, by, bz);
      }
    }
    __syncthreads();
    // ---- P4: edge EMFs (upwinded by the sign of the face upwind speed) and x/y flux sums
    reopen();
    // The t^n values that P5 updates are requested first, so their latency
    // overlaps the edge work.
    T old[8];
    {
      const int zc = z - 1;
      if (own_cell && z >= 1) {
#pragma unroll
        for (int q = 0; q < 5; ++q) old[q] = c.ownp[scell(n, q, ci, cj, zc)];
      }
      if (own_bx && z >= 1) old[5] = c.ownp[sface(n, 0, ci, cj, zc)];
      if (own_by && z >= 1) old[6] = c.ownp[sface(n, 1, ci, cj, zc)];
      if (own_cell && z >= 0) old[7] = c.ownp[sface(n, 2, ci, cj, z)];
    }
    {
      auto up = [](T u, T a, T b) -> T {
        if (u > T(0)) return a;
        if (u < T(0)) return b;
        return T(0.5) * (a + b);
      };
      auto edge = [&](T A, T B, T C, T D, T uA, T uB, T uC, T uD, T c00, T c10, T c01, T c11) -> T {
        const T dc14 = up(uA, c01 - D, c11 - C);
        const T dc34 = up(uB, D - c00, C - c10);
        const T db14 = up(uC, c10 - B, c11 - A);
        const T db34 = up(uD, B - c00, A - c01);
        return T(0.25) * (A + B + C + D) + T(0.25) * ((dc34 - dc14) + (db34 - db14));
      };
      const int pz = z & 1, pzm = (z - 1) & 1;
      auto P = [&](int i, int j) { return (i - (x0 - 1)) + (j - (y0 - 1)) * PX; };
      auto XF = [&](int f, int j) { return (f - x0) + (j - (y0 - 1)) * (TX + 1); };
      auto YF = [&](int i, int g) { return (i - (x0 - 1)) + (g - y0) * (TX + 2); };
      const int nez = (z >= 0 && z < n) ? (TX + 1) * (TY + 1) : 0;
      const int nex = (z >= 0) ? TX * (TY + 1) : 0;
      const int ney = (z >= 0) ? (TX + 1) * TY : 0;
      // each kind of edge starts on a wavefront boundary (no wavefront runs
      // two of the branches)
      const int ex0 = (nez + 63) & ~63, ey0 = ex0 + ((nex + 63) & ~63);
      for (int m = lane; m < ey0 + ney; m += NTHR2) {
        if (m < nez) {  // E_z in plane z at (x-face f, y-face g)
          const int mq = qd(m, TX + 1, iTX1);
          const int f = x0 + (m - mq * (TX + 1)), g = y0 + mq;
          const T A = -sm.fx[6][XF(f, g)], B = -sm.fx[6][XF(f, g - 1)];
          const T C = sm.fy[5][YF(f, g)], D = sm.fy[5][YF(f - 1, g)];
          sm.b.e.ez[m] = edge(A, B, C, D, sm.fx[5][XF(f, g)], sm.fx[5][XF(f, g - 1)], sm.fy[6][YF(f, g)],
                              sm.fy[6][YF(f - 1, g)], sm.ecc[pz][2][P(f - 1, g - 1)], sm.ecc[pz][2][P(f, g - 1)],
                              sm.ecc[pz][2][P(f - 1, g)], sm.ecc[pz][2][P(f, g)]);
        } else if (m >= ex0 && m < ex0 + nex) {  // E_x at z-face z, (x-cell i, y-face g)
          const int e = m - ex0;
          const int eq = qd(e, TX, iTX);
          const int i = x0 + (e - eq * TX), g = y0 + eq;
          const T A = -sm.fy[7][YF(i, g)], B = -sm.py[1][YF(i, g)];
          const T C = sm.fz[6][P(i, g)], D = sm.fz[6][P(i, g - 1)];
          sm.b.e.ex[e] = edge(A, B, C, D, sm.fy[6][YF(i, g)], sm.py[0][YF(i, g)], sm.fz[7][P(i, g)],
                              sm.fz[7][P(i, g - 1)], sm.ecc[pzm][0][P(i, g - 1)], sm.ecc[pzm][0][P(i, g)],
                              sm.ecc[pz][0][P(i, g - 1)], sm.ecc[pz][0][P(i, g)]);
        } else if (m >= ey0) {  // E_y at z-face z, (x-face f, y-cell j)
          const int e = m - ey0;
          const int eq = qd(e, TX + 1, iTX1);
          const int f = x0 + (e - eq * (TX + 1)), j = y0 + eq;
          const T A = -sm.fz[5][P(f, j)], B = -sm.fz[5][P(f - 1, j)];
          const T C = sm.fx[7][XF(f, j)], D = sm.px[1][XF(f, j)];
          sm.b.e.ey[e] = edge(A, B, C, D, sm.fz[7][P(f, j)], sm.fz[7][P(f - 1, j)], sm.fx[5][XF(f, j)],
                              sm.px[0][XF(f, j)], sm.ecc[pzm][1][P(f - 1, j)], sm.ecc[pz][1][P(f - 1, j)],
                              sm.ecc[pzm][1][P(f, j)], sm.ecc[pz][1][P(f, j)]);
        }
      }
      if (own_cell && z >= 0 && z < n) {
#pragma unroll
        for (int q = 0; q < 5; ++q)
          dnew[q] = (sm.fx[q][XF(ci + 1, cj)] - sm.fx[q][XF(ci, cj)]) +
                    (sm.fy[q][YF(ci, cj + 1)] - sm.fy[q][YF(ci, cj)]);
      }
    }
    __syncthreads();
    // ---- P5: write plane z-1 (cells, Bx, By) and face z (Bz); carry partials
    reopen();
    {
      auto EZ = [&](int f, int g) { return sm.b.e.ez[(f - x0) + (g - y0) * (TX + 1)]; };
      auto EX = [&](int i, int g) { return sm.b.e.ex[(i - x0) + (g - y0) * TX]; };
      auto EY = [&](int f, int j) { return sm.b.e.ey[(f - x0) + (j - y0) * (TX + 1)]; };
      if (own_cell && z >= 0) {
        T fzc[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) fzc[q] = sm.fz[q][pc];
        if (z >= 1) {
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            outp[scell(n, q, ci, cj, z - 1)] = old[q] - dtdx * (acc[q] + fzc[q]);
          }
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[q] = dnew[q] - fzc[q];
      }
      if (z >= 1) {
        const int zc = z - 1;
        if (own_bx) outp[sface(n, 0, ci, cj, zc)] = old[5] - dtdx * (pbx - EY(ci, cj));
        if (own_by) outp[sface(n, 1, ci, cj, zc)] = old[6] - dtdx * (pby + EX(ci, cj));
      }
      if (z >= 0 && z < n) {
        if (own_bx) pbx = (EZ(ci, cj + 1) - EZ(ci, cj)) + EY(ci, cj);
        if (own_by) pby = -EX(ci, cj) - (EZ(ci + 1, cj) - EZ(ci, cj));
      }
      if (z >= 0 && own_cell) {
        const T curl = (EY(ci + 1, cj) - EY(ci, cj)) - (EX(ci, cj + 1) - EX(ci, cj));
        outp[sface(n, 2, ci, cj, z)] = old[7] - dtdx * curl;
      }
      // copied by the threads past the columns, which have no update here
      static_assert(MCOL + 2 * MXF <= NTHR2, "one copy per thread past the columns");
      const int mx = lane - MCOL, my = lane - MCOL - MXF;
      if (mx >= 0 && mx < nxf) {
        sm.px[0][mx] = sm.fx[5][mx];
        sm.px[1][mx] = sm.fx[7][mx];
      }
      if (my >= 0 && my < nyf) {
        sm.py[0][my] = sm.fy[6][my];
        sm.py[1][my] = sm.fy[7][my];
      }
    }
    __syncthreads();
  }
}

template <class T, int FN>
__global__ __launch_bounds__(NTHR2) void k_step2(DevSet S, const int* __restrict__ list, int count,
                                                 T* __restrict__ slots, const T* __restrict__ pad,
                                                 int64_t pad_stride, StepPtr st, int tpa, int fuse_dt) {
  __shared__ Step2Smem<T> sm;
  if (FN) tpa = 1;
  const int T2 = tpa * tpa;
  const int wg = blockIdx.x;
  const int bidx = (wg / (8 * T2)) * 8 + (wg % 8);
  const int tile = (wg / 8) % T2;
  if (bidx >= live_count(S, count)) return;
  step2_tile<T, FN>(S, sm, slots, pad, pad_stride, st, bidx, list[bidx], tile, tpa, fuse_dt, threadIdx.x);
}

#ifdef DSP_TU_F32
// ---------------------------------------------------------------------------
// Persistent dispatcher: the paper's mode (i) of the dispatcher (Sec. 3B), in
// which workers take the head of a ready queue, on the device.  One
// persistent launch of `workers` workgroups (one per CU: the step needs the
// whole LDS) replaces the rounds.  A worker takes a ticket, waits until the
// ticket's ring slot holds a patch, updates it (guard brackets, resampled
// guard regions, Courant level, the fused step of each of its tiles in
// turn), publishes it, and tests the patch and its neighbours for readiness
// (Eq. (1) with g = 0), pushing each that became ready.
//
// Exactly-once push: a patch is pushed only by the thread that owns it, and
// ownership moves from idle to queued with a compare-and-swap.  The owner
// re-tests readiness after taking ownership (its first test may have read a
// patch that was being published) and gives ownership back when the patch
// is not ready.  With g = 0 readiness is monotone while a patch is idle (its
// time is fixed and its neighbours' times only grow), so a patch that
// passes both tests stays ready.  No wake-up is lost: every publish is
// followed by a sequentially consistent fence before the publisher tests its
// neighbours, so of two concurrent publishers at least one sees the other's
// time.  With g = 0 the result does not depend on the order of the updates
// (the rounds give the same bits).
//
// Visibility across XCDs (each has its own L2): a worker's new slice and
// metadata are released at agent scope before its patch becomes idle, and a
// worker acquires at agent scope before it reads guard data; the queue words
// are agent-scope atomics.  Every wait is bounded by Q.timeout and also ends
// when the queue is finished or an error is flagged, so the grid always
// drains.

__device__ __forceinline__ int q_load(const int* a) {
  return __hip_atomic_load(a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void q_store(int* a, int v) {
  __hip_atomic_store(a, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t q_load64(const int64_t* a) {
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Eq. (1) with g = 0 and the free-slot rule (as the readiness scan).  The
// neighbours' times are read eight at a time before any is tested, so the
// reads overlap instead of following each other.
__device__ inline bool queue_ready(const DevSet& S, int q, int64_t Tend) {
  if (S.frozen[q]) return false;
  const int64_t t = q_load64(S.ticks + q);
  if (t >= Tend) return false;
  const int ns = S.nslots;
  const int64_t ob = (int64_t)q * ns;
  const int cur = S.cur[q];
  const int oldest = (cur + 1) % ns, after = (cur + 1 + (S.torder > 1 ? 2 : 1)) % ns;
  const int64_t t_after = S.svalid[ob + oldest] ? S.sticks[ob + after] : INT64_MIN;
  const int m0 = S.nb_off[q], m1 = S.nb_off[q + 1];
  for (int mb = m0; mb < m1; mb += 8) {
    int rs[8];
    int64_t tr[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) rs[u] = mb + u < m1 ? S.nb_idx[mb + u] : -1;
#pragma unroll
    for (int u = 0; u < 8; ++u) tr[u] = (rs[u] >= 0 && !S.frozen[rs[u]]) ? q_load64(S.ticks + rs[u]) : INT64_MAX;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (t > tr[u] || t_after > tr[u]) return false;
  }
  return true;
}

__device__ inline bool q_expired(const QueueState& Q, uint64_t t0) {
  return __builtin_amdgcn_s_memrealtime() - t0 > Q.timeout;
}

__device__ inline void q_push(const DevSet& S, const QueueState& Q, int q, uint64_t t0) {
  const unsigned t = __hip_atomic_fetch_add(Q.tail, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  int* slot = Q.buf + (t % (unsigned)Q.cap);
  // the ring holds four times as many entries as patches (each queued at
  // most once), so the slot is free but for a worker that has not yet
  // cleared it
  while (q_load(slot) != 0) {
    if (q_expired(Q, t0)) {
      atomicOr(S.err, ERR_TIMEOUT);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  q_store(slot, q + 1);
}

// push q if it is ready and idle (see the protocol above)
__device__ inline void q_try_push(const DevSet& S, const QueueState& Q, int q, int64_t Tend, uint64_t t0) {
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (!queue_ready(S, q, Tend)) return;
    int idle = 0;
    if (!__hip_atomic_compare_exchange_strong(Q.state + q, &idle, 1, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                              __HIP_MEMORY_SCOPE_AGENT))
      return;  // queued or being updated: its owner tests it again
    if (queue_ready(S, q, Tend)) {
      q_push(S, Q, q, t0);
      return;
    }
    q_store(Q.state + q, 0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
  }
}

__global__ void k_queue_reset(DevSet S, QueueState Q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < Q.cap) Q.buf[i] = 0;
  if (i < S.npatch) Q.state[i] = 0;
  if (i == 0) {
    *Q.head = 0u;
    *Q.tail = 0u;
    *Q.done = 0;
    *Q.remaining = 0;
    *Q.finished = 0;
  }
}

// the patches to advance, and the queue seeded with those ready now
__global__ void k_queue_seed(DevSet S, QueueState Q) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= S.npatch) return;
  const int64_t Tend = *Q.tend;
  if (S.frozen[p] || S.ticks[p] >= Tend) return;
  atomicAdd(Q.remaining, 1);
  if (!queue_ready(S, p, Tend)) return;
  Q.state[p] = 1;
  q_push(S, Q, p, __builtin_amdgcn_s_memrealtime());
}

// S.brk_ready = 1 (each worker computes its patch's brackets first) and
// S.live = nullptr, as set by launch_persist.
template <int FN, bool MULTI>
__global__ __launch_bounds__(NTHR2) void k_persist(DevSet S, QueueState Q, float* __restrict__ slots,
                                                   float* __restrict__ pad, int64_t pad_stride, StepPtr st,
                                                   int gfill) {
  union PersistSmem {
    Step2Smem<float> step;
    GfillSmem<float> gf;
  };
  __shared__ PersistSmem sm;
  __shared__ int s_p;
  const int w = blockIdx.x, tid = threadIdx.x;
  const int64_t Tend = *Q.tend;
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  while (true) {
    // ---- take the next ticket and wait for its patch
    if (tid == 0) {
      int p = -1;
      if (q_load(Q.remaining) > 0) {
        const unsigned t = __hip_atomic_fetch_add(Q.head, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        int* slot = Q.buf + (t % (unsigned)Q.cap);
        while (true) {
          const int v = q_load(slot);
          if (v != 0) {
            q_store(slot, 0);
            p = v - 1;
            break;
          }
          if (q_load(Q.finished) || q_load(S.err)) break;
          if (q_expired(Q, t0)) {
            atomicOr(S.err, ERR_TIMEOUT);
            break;
          }
          __builtin_amdgcn_s_sleep(20);
        }
      }
      // guard data and metadata published by other workers (other XCDs):
      // one acquire invalidates the CU's and the XCD's caches for every
      // wavefront of the workgroup, which reads only after the barrier
      if (p >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_p = p;
    }
    __syncthreads();
    const int p = s_p;
    if (p < 0) break;
    // the thread index made opaque for each patch: what the guard fill and
    // the step derive from it is recomputed per patch, not hoisted out of the
    // worker loop and held (spilled) across it
    int ltid = tid;
    DSP_OPAQUE(ltid);
    // ---- brackets of the patch's guard boxes at its time
    const int box0 = S.rbox_off[p * 108], nbox = S.rbox_off[p * 108 + 108] - box0;
    for (int m = tid; m < nbox; m += NTHR2) S.brk[box0 + m] = bracket(S, S.boxes[box0 + m].q, S.ticks[p], S.tcur[p]);
    __syncthreads();
    // ---- guard regions resampled across resolutions, into this worker's padded buffer
    if constexpr (FN == 0) {  // a fixed size (FN > 0) means no resampled region
      if (gfill) {
        gfill_items<float>(S, sm.gf, slots, pad + (int64_t)w * pad_stride, p, S.gitem_off[p], S.gitem_off[p + 1], 1,
                           ltid);
        __syncthreads();
      }
    }
    // ---- Courant level and the fused step (record entry w), tile by tile:
    // the first tile takes the Courant rate over the whole padded patch and
    // writes the step record, which the other tiles read
    // (MULTI: the set has patches of more than one tile; otherwise the one
    // tile runs without the loop around it)
    if constexpr (MULTI) {
      const int nt = (S.n[p] + MT - 1) / MT;
      for (int tile = 0; tile < nt * nt; ++tile) {
        int ttid = ltid;  // opaque per tile as well (nothing held across the tile loop)
        DSP_OPAQUE(ttid);
        step2_tile<float, FN>(S, sm.step, slots, pad, pad_stride, st, w, p, tile, nt, tile == 0 ? 1 : 0, ttid);
        __syncthreads();
      }
    } else {
      step2_tile<float, FN>(S, sm.step, slots, pad, pad_stride, st, w, p, 0, 1, 1, ltid);
      __syncthreads();
    }
    // ---- output cadence: the new slice into its frame before it is published
    if (S.out_frames) {
      const int f = output_frame(S, S.ticks[p] + st.dtk[w]);
      if (f >= 0) {
        const int64_t V = S.slice_len[p];
        const int64_t w4 = S.out_words;
        const uint32_t* src = (const uint32_t*)slots + (S.slot_off[p] + (int64_t)((S.cur[p] + 1) % S.nslots) * V) * w4;
        uint32_t* dst = (uint32_t*)S.out_frames + ((int64_t)f * S.out_frame_values + S.host_off[p]) * w4;
        for (int64_t e = tid; e < V * w4; e += NTHR2) dst[e] = src[e];
      }
      __syncthreads();  // every wave has read cur before thread 0 advances it
    }
    // ---- publish, give the patch back, count it when it has arrived
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the new slice and the step record
      publish_patch(S, p, st, w);
      q_store(Q.state + p, 0);  // a release store: after the metadata
      if (S.ticks[p] >= Tend) {
        const int d = __hip_atomic_fetch_add(Q.done, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (d == q_load(Q.remaining)) q_store(Q.finished, 1);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    }
    __syncthreads();
    // ---- readiness of the patch and of its neighbours, one thread each
    // (after thread 0's sequentially consistent fence and the barrier)
    const int nb0 = S.nb_off[p], nnb = S.nb_off[p + 1] - nb0;
    for (int c = tid; c <= nnb; c += NTHR2) q_try_push(S, Q, c == 0 ? p : S.nb_idx[nb0 + c - 1], Tend, t0);
    __syncthreads();
  }
}

void launch_queue_seed(const DevSet& S, const QueueState& Q, hipStream_t s) {
  const int n = std::max(Q.cap, S.npatch);
  hipLaunchKernelGGL(k_queue_reset, dim3((n + 255) / 256), dim3(256), 0, s, S, Q);
  hipLaunchKernelGGL(k_queue_seed, dim3((S.npatch + 255) / 256), dim3(256), 0, s, S, Q);
}

void launch_persist(const DevSet& S0, const QueueState& Q, float* slots, float* pad, int64_t pad_stride,
                    const StepPtr& st, int workers, int fn, bool multi, bool gfill, hipStream_t s) {
  DevSet S = S0;
  S.brk_ready = 1;
  S.live = nullptr;
  if (fn == 16)
    hipLaunchKernelGGL((k_persist<16, false>), dim3(workers), dim3(NTHR2), 0, s, S, Q, slots, pad, pad_stride, st,
                       gfill ? 1 : 0);
  else if (multi)
    hipLaunchKernelGGL((k_persist<0, true>), dim3(workers), dim3(NTHR2), 0, s, S, Q, slots, pad, pad_stride, st,
                       gfill ? 1 : 0);
  else
    hipLaunchKernelGGL((k_persist<0, false>), dim3(workers), dim3(NTHR2), 0, s, S, Q, slots, pad, pad_stride, st,
                       gfill ? 1 : 0);
}

#endif  // DSP_TU_F32

// ---------------------------------------------------------------------------

template <class T>
int launch_fused(const DevSet& S0, const int* list, int count, int nmin, int nmax, T* slots, T* pad,
                  int64_t pad_stride, bool gfill, double* smax, const StepPtr& st, hipStream_t s, int dt_kind,
                  double t_end, int clip, hipEvent_t ev0, hipEvent_t ev1) {
  const int N = nmax + 4;
  // with the resampling, the round's brackets are computed first and every
  // kernel of the round reads them
  DevSet S = S0;
  S.brk_ready = gfill ? 1 : 0;
  // the events bracket the round's whole update sequence: guard resampling,
  // separate Courant pass (if any) and the step
  if (ev0) (void)hipEventRecord(ev0, s);
  if (gfill) {
    // the time bracket of every guard box of the listed patches, once (a
    // chain of dependent reads that every resampling workgroup would repeat)
    launch_brackets(S, list, count, s);
    hipLaunchKernelGGL(k_gfill<T>, dim3(GFILL_COLS, std::min(count, GFILL_ROWS)), dim3(256), 0, s, S, list, count,
                       (const T*)slots, pad, pad_stride);
    if (S.any_direct)
      hipLaunchKernelGGL(k_gfill_direct<T>, dim3(108, count), dim3(256), 0, s, S, list, count, (const T*)slots,
                         pad, pad_stride);
  }
  const int tpa = (nmax + MT - 1) / MT;
  // a local step of single-tile patches takes its Courant rate and level
  // inside the step kernel; otherwise a separate pass (the global modes
  // need the rate of every patch first)
  const int fuse_dt = (dt_kind == 0 && tpa == 1) ? 1 : 0;
  if (!fuse_dt) {
    (void)hipMemsetAsync(smax, 0, sizeof(double) * count, s);
    const unsigned gx = (unsigned)std::max<int64_t>(1, ((int64_t)N * N * N + 2047) / 2048);  // ~8 cells per thread
    hipLaunchKernelGGL(k_courant<T>, dim3(gx, count), dim3(256), 0, s, S,
                       list, count, (const T*)slots, (const T*)pad, pad_stride, smax);
    launch_dt(S, list, count, st, smax, s, dt_kind, t_end, clip);
  }
  const int T2 = tpa * tpa;
  const int groups = ((count + 7) / 8) * 8 * T2;
  if constexpr (sizeof(T) == 4) {
    // equal 16^3 patches without padded guard regions: the fixed-size variant
    if (nmin == 16 && nmax == 16 && !gfill)
      hipLaunchKernelGGL((k_step2<T, 16>), dim3(groups), dim3(NTHR2), 0, s, S, list, count, slots, (const T*)pad,
                         pad_stride, st, tpa, fuse_dt);
    else
      hipLaunchKernelGGL((k_step2<T, 0>), dim3(groups), dim3(NTHR2), 0, s, S, list, count, slots, (const T*)pad,
                         pad_stride, st, tpa, fuse_dt);
  } else {
    if (nmin == 16 && nmax == 16 && !gfill)
      hipLaunchKernelGGL((k_step<T, 16>), dim3(groups), dim3(NTHR), 0, s, S, list, count, slots, (const T*)pad,
                         pad_stride, st, tpa, fuse_dt);
    else
      hipLaunchKernelGGL((k_step<T, 0>), dim3(groups), dim3(NTHR), 0, s, S, list, count, slots, (const T*)pad,
                         pad_stride, st, tpa, fuse_dt);
  }
  if (ev1) (void)hipEventRecord(ev1, s);
  return fuse_dt;
}

#ifdef DSP_TU_F32
template int launch_fused<float>(const DevSet&, const int*, int, int, int, float*, float*, int64_t, bool, double*,
                                  const StepPtr&, hipStream_t, int, double, int, hipEvent_t, hipEvent_t);
#endif
#ifdef DSP_TU_F64
template int launch_fused<double>(const DevSet&, const int*, int, int, int, double*, double*, int64_t, bool,
                                   double*, const StepPtr&, hipStream_t, int, double, int, hipEvent_t, hipEvent_t);
#endif

}  // namespace dsp
