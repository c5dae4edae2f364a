// dsp_kernels.hip -- HIP kernels of the patch engine (gfx950).
//
// One update of a set of ready patches (Sec. 3A/3B of the paper) is a short
// sequence of kernels over a batch of patch slots b = 0..count-1, patch
// p = list[b]:
//   k_fill     guard-filled padded copy of the patch (2 guard layers), guard
//              values interpolated linearly in time between the neighbour's
//              two bracketing slices (or copied at an exact slice time), and
//              conservatively prolonged / restricted across resolutions;
//   k_prim     primitive variables and the Courant rate of every padded cell,
//              reduced per patch with wavefront + workgroup maxima;
//   k_dt_*     the quantised step (FP64 + integer ticks);
//   k_pred     van Leer slopes and the Hancock half-step predictor;
//   k_flux     HLLD fluxes on every face the update and the edge EMFs need;
//   k_emf      upwinded edge EMFs (constrained transport);
//   k_ni_emf   with non-ideal MHD: Ohmic and ambipolar fields added to the
//              edge EMFs, and k_ni_flux their Poynting flux to the energy flux;
//   k_update   conservative update of the cell variables and CT update of B,
//              written into the patch's next ring slot;
//   k_publish  new slot, ticks, step count and level hash (after the whole
//              round, so every read of the round saw the old metadata).
// Kernels that read per-patch data take a list of patch ids; a patch's
// interior size n may differ between patches (uneven sets).
//
// The source is compiled three times: with DSP_TU_COMMON for the kernels that
// do not depend on the precision (readiness scan, levels, publish, time
// records, guard-box brackets), with DSP_TU_F32 for the single-precision
// instantiations and with DSP_TU_F64 for the double-precision ones, which are
// built without floating-point contraction (IEEE operations one at a time,
// as the FP64 oracle computes them).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsp_dev.h"
#include "dsp_guard.h"
#include "mhd_dev.h"

namespace dsp {

// ---------------------------------------------------------------------------
// k_brackets: the time bracket of every guard box of the listed patches at
// the patch's current time (one thread per box), so that k_fill reads it
// instead of searching the source's slices for every element.

#ifdef DSP_TU_COMMON
__global__ void k_brackets(DevSet S, const int* __restrict__ list, int count) {
  const int b = blockIdx.y;
  if (b >= live_count(S, count)) return;
  const int p = list[b];
  const int m = S.rbox_off[p * 108] + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (m >= S.rbox_off[p * 108 + 108]) return;
  S.brk[m] = bracket(S, S.boxes[m].q, S.ticks[p], S.tcur[p]);
}
#endif  // DSP_TU_COMMON

// ---------------------------------------------------------------------------
// k_fill: one thread per padded element (5 N^3 cell values, then 3 face
// arrays) of patch list[b].

template <class T>
__global__ void k_fill(DevSet S, const int* __restrict__ list, int count, T* __restrict__ slots,
                       WorkPtr<T> W) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const int p = list[b];
  const int n = S.n[p], N = n + 4;
  const int64_t ncell = (int64_t)N * N * N, nface = (int64_t)N * N * (N + 1);
  const int64_t total = 5 * ncell + 3 * nface;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int comp, var, i, j, k;
  if (e < 5 * ncell) {
    comp = -1;
    var = (int)(e / ncell);
    int64_t r = e - var * ncell;
    i = (int)(r % N) - 2;
    r /= N;
    j = (int)(r % N) - 2;
    k = (int)(r / N) - 2;
  } else {
    int64_t r = e - 5 * ncell;
    comp = (int)(r / nface);
    var = 0;
    r -= comp * nface;
    const int sx = N + (comp == 0), sy = N + (comp == 1);
    i = (int)(r % sx) - 2;
    r /= sx;
    j = (int)(r % sy) - 2;
    k = (int)(r / sy) - 2;
  }
  T* Pd = W.pad + (int64_t)b * W.pad_stride;
  const int idx[3] = {i, j, k};
  int rg[3];
  bool interior = true;
  for (int d = 0; d < 3; ++d) {
    const int hi = n + (d == comp ? 1 : 0);
    rg[d] = idx[d] < 0 ? 0 : (idx[d] < hi ? 1 : 2);
    interior = interior && rg[d] == 1;
  }
  if (interior) {
    const int64_t own = S.slot_off[p] + (int64_t)S.cur[p] * S.slice_len[p];
    const int64_t se = (comp < 0) ? scell(n, var, i, j, k) : sface(n, comp, i, j, k);
    Pd[e] = slots[own + se];
    return;
  }
  // guard element: find its box among the boxes of (patch, component, region)
  const int region = (rg[2] * 3 + rg[1]) * 3 + rg[0];
  const int key = p * 108 + (comp + 1) * 27 + region;
  const int b0 = S.rbox_off[key], b1 = S.rbox_off[key + 1];
  for (int m = b0; m < b1; ++m) {
    const GBox& G = S.boxes[m];
    if (i < G.lo[0] || i > G.hi[0] || j < G.lo[1] || j > G.hi[1] || k < G.lo[2] || k > G.hi[2])
      continue;
    const int q = G.q;
    const Bracket br = S.brk[m];
    T val;
    if (G.same) {
      const int qi = i + G.shift[0], qj = j + G.shift[1], qk = k + G.shift[2];
      const int64_t se = (comp < 0) ? scell(S.n[q], var, qi, qj, qk) : sface(S.n[q], comp, qi, qj, qk);
      val = tlerp(slots, br, se);
    } else {
      // lattice position of the element, shifted into the source's periodic image
      const int64_t dxl = S.dxl[p];
      int64_t X[3];
      for (int d = 0; d < 3; ++d) {
        X[d] = S.lo[3 * p + d] + (int64_t)idx[d] * dxl + (d == comp ? 0 : dxl / 2) + G.wrap[d];
      }
      val = cross_value(S, slots, br, q, comp, var, X, dxl);
    }
    Pd[e] = val;
    return;
  }
  atomicOr(S.err, ERR_STATE);  // no source: the plan is inconsistent
}

// ---------------------------------------------------------------------------
// k_prim: primitives and Courant rate over the padded cells [-2, n+1]^3.

template <class T>
__global__ void k_prim(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const int p = list[b];
  const int n = S.n[p], N = n + 4;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ncell = (int64_t)N * N * N;
  double s = 0.0;
  if (c < ncell) {
    const int i = (int)(c % N) - 2, j = (int)((c / N) % N) - 2, k = (int)(c / ((int64_t)N * N)) - 2;
    const T* Pd = W.pad + (int64_t)b * W.pad_stride;
    T* Wp = W.w + (int64_t)b * W.w_stride;
    const T rho = Pd[pcell(N, 0, i, j, k)];
    const T mx = Pd[pcell(N, 1, i, j, k)], my = Pd[pcell(N, 2, i, j, k)], mz = Pd[pcell(N, 3, i, j, k)];
    const T en = Pd[pcell(N, 4, i, j, k)];
    const T bx = T(0.5) * (Pd[pface(N, 0, i, j, k)] + Pd[pface(N, 0, i + 1, j, k)]);
    const T by = T(0.5) * (Pd[pface(N, 1, i, j, k)] + Pd[pface(N, 1, i, j + 1, k)]);
    const T bz = T(0.5) * (Pd[pface(N, 2, i, j, k)] + Pd[pface(N, 2, i, j, k + 1)]);
    const T ir = T(1) / rho;
    const T vx = mx * ir, vy = my * ir, vz = mz * ir;
    const T ke = T(0.5) * (mx * mx + my * my + mz * mz) * ir;
    const T bb = bx * bx + by * by + bz * bz;
    T pr = (T(S.gamma) - T(1)) * (en - ke - T(0.5) * bb);
    if (!isfinite(rho) || !isfinite(pr)) {
      atomicOr(S.err, ERR_NONFINITE);
      pr = T(1);
    }
    if (!(rho > T(0))) {
      atomicOr(S.err, ERR_NEGATIVE);
    } else if (S.p_floor > 0.0) {
      if (pr < T(S.p_floor)) {
        pr = T(S.p_floor);
        atomicAdd(S.floor_hits, 1ULL);
      }
    } else if (!(pr > T(0))) {
      atomicOr(S.err, ERR_NEGATIVE);
    }
    const int64_t o = wcell(N, 0, i, j, k), st = ncell;
    Wp[o] = rho;
    Wp[o + st] = vx;
    Wp[o + 2 * st] = vy;
    Wp[o + 3 * st] = vz;
    Wp[o + 4 * st] = pr;
    Wp[o + 5 * st] = bx;
    Wp[o + 6 * st] = by;
    Wp[o + 7 * st] = bz;
    // Courant rate sum_d (|v_d| + c_f,d) / dx in stencil precision
    if (rho > T(0) && pr > T(0)) {
      const T a2 = T(S.gamma) * pr * ir, b2 = bb * ir;
      T sum = fabs(vx) + fast_speed(a2, b2, (by * by + bz * bz) * ir);
      sum = sum + (fabs(vy) + fast_speed(a2, b2, (bz * bz + bx * bx) * ir));
      sum = sum + (fabs(vz) + fast_speed(a2, b2, (bx * bx + by * by) * ir));
      s = (double)sum / S.dx[p];
      if (S.nonideal) {
        // Ohmic and ambipolar limits as rates (Eqs. dtOhm, dtAD, C = 0.1)
        const double f = S.courant / kCourantNonideal / (S.dx[p] * S.dx[p]);
        if (S.eta > 0.0) {
          const double so = S.eta * f;
          if (so > s) s = so;
        }
        if (S.gamma_ad > 0.0) {
          const double sa = (double)bb / (S.gamma_ad * S.rho_i * (double)rho) * f;
          if (sa > s) s = sa;
        }
      }
      if (!isfinite(s)) atomicOr(S.err, ERR_NONFINITE);
    }
  }
  // wavefront maximum, then one atomic per wavefront
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(s, off, 64);
    s = o > s ? o : s;
  }
  if ((threadIdx.x & 63) == 0 && s > 0.0) atomic_max_pos(W.smax + b, s);
}

// ---------------------------------------------------------------------------
// time-step choice

#ifdef DSP_TU_COMMON
__global__ void k_dt_local(DevSet S, const int* __restrict__ list, int count, StepPtr st,
                           const double* smax) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= live_count(S, count)) return;
  const int p = list[b];
  const int k = level_for(S, smax[b], S.ticks[p]);
  if (k > S.kmax) {
    atomicOr(S.err, ERR_KMAX);
    st.k[b] = S.kmax;
  } else {
    st.k[b] = k;
  }
  st.dtk[b] = (int64_t)1 << (S.kmax - st.k[b]);
  st.dt[b] = S.dt_base * ldexp(1.0, -st.k[b]);
}

// GLOBAL modes: one step for the whole set (single workgroup reduction).
// mode 1: k = max of the per-patch levels; mode 2: courant / max rate,
// clipped to t_end; mode 3: dt_fixed, clipped to t_end unless nsteps mode.
__global__ void k_dt_global(DevSet S, const int* __restrict__ list, int count, StepPtr st,
                            const double* smax, double t_end, int clip) {
  __shared__ double red[256];
  __shared__ int redk[256];
  double m = 0.0;
  int km = 0;
  for (int b = threadIdx.x; b < count; b += blockDim.x) {
    m = smax[b] > m ? smax[b] : m;
    if (S.dt_mode == 1) {
      const int k = level_for(S, smax[b], S.ticks[list[b]]);
      km = k > km ? k : km;
    }
  }
  red[threadIdx.x] = m;
  redk[threadIdx.x] = km;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x] = red[threadIdx.x + s] > red[threadIdx.x] ? red[threadIdx.x + s] : red[threadIdx.x];
      redk[threadIdx.x] = redk[threadIdx.x + s] > redk[threadIdx.x] ? redk[threadIdx.x + s] : redk[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double dt;
  int64_t dtk = 0;
  int k = -1;
  const double t0 = S.tcur[list[0]];
  if (S.dt_mode == 1) {
    k = redk[0];
    if (k > S.kmax) {
      atomicOr(S.err, ERR_KMAX);
      k = S.kmax;
    }
    dtk = (int64_t)1 << (S.kmax - k);
    dt = S.dt_base * ldexp(1.0, -k);
  } else {
    dt = (S.dt_mode == 2) ? S.courant / red[0] : S.dt_fixed;
    if (clip && t0 + dt > t_end) dt = t_end - t0;
  }
  for (int b = 0; b < count; ++b) {
    st.k[b] = k;
    st.dtk[b] = dtk;
    st.dt[b] = dt;
  }
}
#endif  // DSP_TU_COMMON

// ---------------------------------------------------------------------------
// k_pred: slopes (per direction) and half-step predictor on [-1, n]^3.

template <class T>
__global__ void k_pred(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W, StepPtr st) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const int p = list[b];
  const int n = S.n[p], N = n + 4, M = n + 2;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)M * M * M) return;
  const int i = (int)(c % M) - 1, j = (int)((c / M) % M) - 1, k = (int)(c / ((int64_t)M * M)) - 1;
  const T* Wp = W.w + (int64_t)b * W.w_stride;
  T* Sp = W.s + (int64_t)b * W.s_stride;
  T* Hp = W.h + (int64_t)b * W.w_stride;
  const int64_t NC = (int64_t)N * N * N;
  T w[8], sl[3][8], H[8];
  for (int v = 0; v < 8; ++v) w[v] = Wp[wcell(N, v, i, j, k)];
  for (int d = 0; d < 3; ++d) {
    int im = i, jm = j, km = k, ip = i, jp = j, kp = k;
    if (d == 0) { im--; ip++; } else if (d == 1) { jm--; jp++; } else { km--; kp++; }
    for (int v = 0; v < 8; ++v) {
      if (v == 5 + d) {
        sl[d][v] = T(0);
        continue;
      }
      const T a = Wp[wcell(N, v, im, jm, km)], cc = Wp[wcell(N, v, ip, jp, kp)];
      sl[d][v] = van_leer(w[v] - a, cc - w[v]);
    }
    for (int v = 0; v < 8; ++v) Sp[(int64_t)(d * 8 + v) * NC + wcell(N, 0, i, j, k)] = sl[d][v];
  }
  const T hdtdx = (T)(0.5 * st.dt[b] / S.dx[p]);
  hancock(w, sl, hdtdx, T(S.gamma), H);
  for (int v = 0; v < 8; ++v) Hp[wcell(N, v, i, j, k)] = H[v];
}

// ---------------------------------------------------------------------------
// k_flux: HLLD on faces along d (face index [0, n]) with the other indices in
// [-1, n].  Thread layout: the three directions concatenated.

template <class T>
__global__ void k_flux(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const int p = list[b];
  const int n = S.n[p], N = n + 4, M = n + 2;
  const int64_t per = (int64_t)(n + 1) * M * M;
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 3 * per) return;
  const int d = (int)(c / per);
  c -= d * per;
  // faces idx[d] in [0, n], the other two indices in [-1, n]; x fastest, so
  // that neighbouring threads read neighbouring cells in every direction
  int idx[3];
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  const int e0 = d == 0 ? n + 1 : M, e1 = d == 1 ? n + 1 : M;
  idx[0] = (int)(c % e0) - (d == 0 ? 0 : 1);
  idx[1] = (int)((c / e0) % e1) - (d == 1 ? 0 : 1);
  idx[2] = (int)(c / ((int64_t)e0 * e1)) - (d == 2 ? 0 : 1);
  int ia[3] = {idx[0], idx[1], idx[2]};
  ia[d] -= 1;
  const T* Wp = W.w + (int64_t)b * W.w_stride;
  const T* Hp = W.h + (int64_t)b * W.w_stride;
  const T* Sp = W.s + (int64_t)b * W.s_stride;
  const T* Pd = W.pad + (int64_t)b * W.pad_stride;
  const int64_t NC = (int64_t)N * N * N;
  const int64_t ca = wcell(N, 0, ia[0], ia[1], ia[2]), cb = wcell(N, 0, idx[0], idx[1], idx[2]);
  const int order[7] = {0, 1 + d, 1 + t1, 1 + t2, 4, 5 + t1, 5 + t2};
  T l[7], r[7];
  for (int m = 0; m < 7; ++m) {
    const int v = order[m];
    l[m] = Hp[v * NC + ca] + T(0.5) * Sp[(int64_t)(d * 8 + v) * NC + ca];
    r[m] = Hp[v * NC + cb] - T(0.5) * Sp[(int64_t)(d * 8 + v) * NC + cb];
  }
  const T bface = Pd[pface(N, d, idx[0], idx[1], idx[2])];
  T bn = bface + T(0.5) * ((Hp[(5 + d) * NC + ca] - Wp[(5 + d) * NC + ca]) +
                           (Hp[(5 + d) * NC + cb] - Wp[(5 + d) * NC + cb]));
  if (!(l[0] > T(0)) || !(l[4] > T(0)) || !(r[0] > T(0)) || !(r[4] > T(0))) {
    for (int m = 0; m < 7; ++m) {
      l[m] = Wp[order[m] * NC + ca];
      r[m] = Wp[order[m] * NC + cb];
    }
    bn = bface;
    atomicAdd(S.fallback, 1ULL);
  }
  T f[8];
  hlld_flux(l, r, bn, T(S.gamma), f);
  T* Fp = W.f + (int64_t)b * W.f_stride + (int64_t)d * 8 * W.fm3;
  const int64_t o = wface(N, 0, idx[0], idx[1], idx[2]);
  const int64_t fs = W.fm3;
  Fp[o] = f[0];
  Fp[(1 + d) * fs + o] = f[1];
  Fp[(1 + t1) * fs + o] = f[2];
  Fp[(1 + t2) * fs + o] = f[3];
  Fp[4 * fs + o] = f[4];
  Fp[(5 + d) * fs + o] = f[7];  // the normal field has no flux: the slot holds the upwind speed
  Fp[(5 + t1) * fs + o] = f[5];
  Fp[(5 + t2) * fs + o] = f[6];
}

// ---------------------------------------------------------------------------
// k_emf: edge EMF E_a on edges along a (a-index a cell index in [0, n-1], the
// other two face indices in [0, n]), (a, b, c) cyclic.  Face EMFs come from
// the induction fluxes: on b-faces E_a = -F_b[B_c], on c-faces E_a = +F_c[B_b];
// the cell reference value is E = -v x B of the half-step state; corrections
// are upwinded by the direction of the mass flux (Gardiner & Stone 2005),
// taken as the sign of the face's upwind speed (HLLD f[7]).

template <class T>
__global__ void k_emf(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W) {
  const int blk = blockIdx.y;
  if (blk >= count) return;
  const int p = list[blk];
  const int n = S.n[p], N = n + 4;
  const int64_t per = (int64_t)n * (n + 1) * (n + 1);
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 3 * per) return;
  const int a = (int)(c / per);
  c -= a * per;
  const int bax = (a + 1) % 3, cax = (a + 2) % 3;
  // edges e[a] in [0, n), the other two indices in [0, n]; x fastest
  int e[3];
  const int x0 = a == 0 ? n : n + 1, x1 = a == 1 ? n : n + 1;
  e[0] = (int)(c % x0);
  e[1] = (int)((c / x0) % x1);
  e[2] = (int)(c / ((int64_t)x0 * x1));
  const T* Hp = W.h + (int64_t)blk * W.w_stride;
  const T* Fb = W.f + (int64_t)blk * W.f_stride + (int64_t)bax * 8 * W.fm3;
  const T* Fc = W.f + (int64_t)blk * W.f_stride + (int64_t)cax * 8 * W.fm3;
  const int64_t fs = W.fm3;
  const int64_t NC = (int64_t)N * N * N;
  int pA[3] = {e[0], e[1], e[2]}, pB[3] = {e[0], e[1], e[2]};
  pB[cax] -= 1;
  int pC[3] = {e[0], e[1], e[2]}, pD[3] = {e[0], e[1], e[2]};
  pD[bax] -= 1;
  const int64_t oA = wface(N, 0, pA[0], pA[1], pA[2]), oB = wface(N, 0, pB[0], pB[1], pB[2]);
  const int64_t oC = wface(N, 0, pC[0], pC[1], pC[2]), oD = wface(N, 0, pD[0], pD[1], pD[2]);
  const T A = -Fb[(5 + cax) * fs + oA], B = -Fb[(5 + cax) * fs + oB];
  const T C = Fc[(5 + bax) * fs + oC], D = Fc[(5 + bax) * fs + oD];
  const T mA = Fb[(5 + bax) * fs + oA], mB = Fb[(5 + bax) * fs + oB];
  const T mC = Fc[(5 + cax) * fs + oC], mD = Fc[(5 + cax) * fs + oD];
  auto ecc = [&](int db, int dc) -> T {
    int q[3] = {e[0], e[1], e[2]};
    q[bax] += db;
    q[cax] += dc;
    const int64_t o = wcell(N, 0, q[0], q[1], q[2]);
    // E_a = v_c B_b - v_b B_c
    return Hp[(1 + cax) * NC + o] * Hp[(5 + bax) * NC + o] - Hp[(1 + bax) * NC + o] * Hp[(5 + cax) * NC + o];
  };
  const T c00 = ecc(-1, -1), c10 = ecc(0, -1), c01 = ecc(-1, 0), c11 = ecc(0, 0);
  auto up = [](T m, T x, T y) -> T {
    if (m > T(0)) return x;
    if (m < T(0)) return y;
    return T(0.5) * (x + y);
  };
  const T dc14 = up(mA, c01 - D, c11 - C);
  const T dc34 = up(mB, D - c00, C - c10);
  const T db14 = up(mC, c10 - B, c11 - A);
  const T db34 = up(mD, B - c00, A - c01);
  T* Ep = W.e + (int64_t)blk * W.e_stride + (int64_t)a * W.fm3;
  Ep[wface(N, 0, e[0], e[1], e[2])] =
      T(0.25) * (A + B + C + D) + T(0.25) * ((dc34 - dc14) + (db34 - db14));
}

// ---------------------------------------------------------------------------
// Non-ideal electric field (Sec. 4.3) from the padded state at t^n, on the
// edges of k_emf: Ohmic E = eta J (Eq. Ohm) plus ambipolar
// E = -v_D x B = (B^2 J - (J.B) B) / (gamma_AD rho rho_i) (Eq. AD).  J_a is the
// discrete curl of the face field on the a-edge; on an a-edge the b and c
// components of J are the means of the four nearest b- (c-) edges, B_a the
// mean of the eight nearest a-faces, B_b and B_c the means of the two faces
// through the edge, rho the mean of the four cells around it.  The field is
// added to the edge EMFs and kept (in the slope buffer, dead after k_flux)
// for k_ni_flux.

// J_a on the a-edge (a-index a cell index, the others face indices) of the
// padded patch Pd
template <class T>
__device__ __forceinline__ T edge_current(const T* Pd, int N, T dx, int a, int i0, int i1, int i2) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  int e[3] = {i0, i1, i2}, eb[3] = {i0, i1, i2}, ec[3] = {i0, i1, i2};
  eb[b] -= 1;
  ec[c] -= 1;
  const T dcb = Pd[pface(N, c, e[0], e[1], e[2])] - Pd[pface(N, c, eb[0], eb[1], eb[2])];
  const T dbc = Pd[pface(N, b, e[0], e[1], e[2])] - Pd[pface(N, b, ec[0], ec[1], ec[2])];
  return (dcb - dbc) / dx;
}

template <class T>
__global__ void k_ni_emf(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W) {
  const int blk = blockIdx.y;
  if (blk >= count) return;
  const int p = list[blk];
  const int n = S.n[p], N = n + 4;
  const int64_t per = (int64_t)n * (n + 1) * (n + 1);
  int64_t c0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c0 >= 3 * per) return;
  const int a = (int)(c0 / per);
  c0 -= a * per;
  const int bax = (a + 1) % 3, cax = (a + 2) % 3;
  // edges e[a] in [0, n), the other two indices in [0, n]; x fastest
  int e[3];
  const int x0 = a == 0 ? n : n + 1, x1 = a == 1 ? n : n + 1;
  e[0] = (int)(c0 % x0);
  e[1] = (int)((c0 / x0) % x1);
  e[2] = (int)(c0 / ((int64_t)x0 * x1));
  const T* Pd = W.pad + (int64_t)blk * W.pad_stride;
  const T* Wp = W.w + (int64_t)blk * W.w_stride;
  const T dx = (T)S.dx[p];
  const T ja = edge_current(Pd, N, dx, a, e[0], e[1], e[2]);
  T en = T(S.eta) * ja;
  if (S.gamma_ad > 0.0) {
    T jb = T(0), jc = T(0), ba = T(0), bb = T(0), bc = T(0), rho = T(0);
    for (int s = -1; s <= 0; ++s)
      for (int t = 0; t <= 1; ++t) {
        int q[3] = {e[0], e[1], e[2]}, r[3] = {e[0], e[1], e[2]};
        q[bax] += s;
        q[a] += t;
        jb = jb + edge_current(Pd, N, dx, bax, q[0], q[1], q[2]);
        r[cax] += s;
        r[a] += t;
        jc = jc + edge_current(Pd, N, dx, cax, r[0], r[1], r[2]);
      }
    for (int t = 0; t <= 1; ++t)
      for (int s = -1; s <= 0; ++s)
        for (int u = -1; u <= 0; ++u) {
          int q[3] = {e[0], e[1], e[2]};
          q[a] += t;
          q[bax] += s;
          q[cax] += u;
          ba = ba + Pd[pface(N, a, q[0], q[1], q[2])];
        }
    for (int s = -1; s <= 0; ++s) {
      int q[3] = {e[0], e[1], e[2]}, r[3] = {e[0], e[1], e[2]}, w[3] = {e[0], e[1], e[2]};
      q[cax] += s;
      bb = bb + Pd[pface(N, bax, q[0], q[1], q[2])];
      r[bax] += s;
      bc = bc + Pd[pface(N, cax, r[0], r[1], r[2])];
      for (int u = -1; u <= 0; ++u) {
        w[bax] = e[bax] + s;
        w[cax] = e[cax] + u;
        rho = rho + Wp[wcell(N, 0, w[0], w[1], w[2])];
      }
    }
    jb = T(0.25) * jb;
    jc = T(0.25) * jc;
    ba = T(0.125) * ba;
    bb = T(0.5) * bb;
    bc = T(0.5) * bc;
    rho = T(0.25) * rho;
    const T b2 = ba * ba + bb * bb + bc * bc;
    const T jdotb = ja * ba + jb * bb + jc * bc;
    en = en + (b2 * ja - jdotb * ba) / (T(S.gamma_ad * S.rho_i) * rho);
  }
  const int64_t o = (int64_t)a * W.fm3 + wface(N, 0, e[0], e[1], e[2]);
  W.s[(int64_t)blk * W.s_stride + o] = en;
  W.e[(int64_t)blk * W.e_stride + o] += en;
}

// Poynting flux (E x B)_d of the non-ideal field through the d-faces of the
// update (face index [0, n] along d, cells [0, n-1] across): the means of E_t1
// and E_t2 over the two edges of each kind on the face, and of B_t1 and B_t2
// over the four faces around it, added to the energy flux.  Total energy
// stays conserved; the magnetic energy removed becomes the heat J.E (Eqs.
// Ohm_heat and Q_AD).
template <class T>
__global__ void k_ni_flux(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W) {
  const int blk = blockIdx.y;
  if (blk >= count) return;
  const int p = list[blk];
  const int n = S.n[p], N = n + 4;
  const int64_t per = (int64_t)(n + 1) * n * n;
  int64_t c0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c0 >= 3 * per) return;
  const int d = (int)(c0 / per);
  c0 -= d * per;
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  // faces f[d] in [0, n], the other two indices in [0, n); x fastest
  int f[3];
  const int x0 = d == 0 ? n + 1 : n, x1 = d == 1 ? n + 1 : n;
  f[0] = (int)(c0 % x0);
  f[1] = (int)((c0 / x0) % x1);
  f[2] = (int)(c0 / ((int64_t)x0 * x1));
  const T* Pd = W.pad + (int64_t)blk * W.pad_stride;
  const T* En = W.s + (int64_t)blk * W.s_stride;
  T e1 = T(0), e2 = T(0), b1 = T(0), b2 = T(0);
  for (int s = 0; s <= 1; ++s) {
    int q[3] = {f[0], f[1], f[2]}, r[3] = {f[0], f[1], f[2]};
    q[t2] += s;
    e1 = e1 + En[(int64_t)t1 * W.fm3 + wface(N, 0, q[0], q[1], q[2])];
    r[t1] += s;
    e2 = e2 + En[(int64_t)t2 * W.fm3 + wface(N, 0, r[0], r[1], r[2])];
    for (int u = -1; u <= 0; ++u) {
      int x[3] = {f[0], f[1], f[2]}, y[3] = {f[0], f[1], f[2]};
      x[t2] += s;
      x[d] += u;
      b2 = b2 + Pd[pface(N, t2, x[0], x[1], x[2])];
      y[t1] += s;
      y[d] += u;
      b1 = b1 + Pd[pface(N, t1, y[0], y[1], y[2])];
    }
  }
  e1 = T(0.5) * e1;
  e2 = T(0.5) * e2;
  b1 = T(0.25) * b1;
  b2 = T(0.25) * b2;
  T* Fd = W.f + (int64_t)blk * W.f_stride + (int64_t)d * 8 * W.fm3;
  Fd[4 * W.fm3 + wface(N, 0, f[0], f[1], f[2])] += e1 * b2 - e2 * b1;
}

// ---------------------------------------------------------------------------
// k_update: new slice = conservative update of the cells + CT update of the
// faces, written into the patch's next ring slot.

template <class T>
__global__ void k_update(DevSet S, const int* __restrict__ list, int count, T* __restrict__ slots,
                         WorkPtr<T> W, StepPtr st) {
  const int blk = blockIdx.y;
  if (blk >= count) return;
  const int p = list[blk];
  const int n = S.n[p], N = n + 4;
  const int64_t n3 = (int64_t)n * n * n, nf = (int64_t)n * n * (n + 1);
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n3 + 3 * nf) return;
  const T* Pd = W.pad + (int64_t)blk * W.pad_stride;
  const int nxt = (S.cur[p] + 1) % S.nslots;
  T* out = slots + S.slot_off[p] + (int64_t)nxt * S.slice_len[p];
  const T dtdx = (T)(st.dt[blk] / S.dx[p]);
  const int64_t fs = W.fm3;
  if (c < n3) {
    const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / ((int64_t)n * n));
    T du[5] = {T(0), T(0), T(0), T(0), T(0)};
    for (int d = 0; d < 3; ++d) {
      const T* Fd = W.f + (int64_t)blk * W.f_stride + (int64_t)d * 8 * fs;
      int r[3] = {i, j, k};
      r[d] += 1;
      const int64_t ol = wface(N, 0, i, j, k), orr = wface(N, 0, r[0], r[1], r[2]);
      for (int v = 0; v < 5; ++v) du[v] = du[v] + (Fd[v * fs + orr] - Fd[v * fs + ol]);
    }
    for (int v = 0; v < 5; ++v)
      out[scell(n, v, i, j, k)] = Pd[pcell(N, v, i, j, k)] - dtdx * du[v];
    return;
  }
  c -= n3;
  const int d = (int)(c / nf);
  c -= d * nf;
  const int sx = n + (d == 0), sy = n + (d == 1);
  const int i = (int)(c % sx), j = (int)((c / sx) % sy), k = (int)(c / ((int64_t)sx * sy));
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  const T* E1 = W.e + (int64_t)blk * W.e_stride + (int64_t)t1 * fs;
  const T* E2 = W.e + (int64_t)blk * W.e_stride + (int64_t)t2 * fs;
  int p1[3] = {i, j, k}, p2[3] = {i, j, k};
  p1[t1] += 1;
  p2[t2] += 1;
  const int64_t o0 = wface(N, 0, i, j, k);
  const T curl = (E2[wface(N, 0, p1[0], p1[1], p1[2])] - E2[o0]) - (E1[wface(N, 0, p2[0], p2[1], p2[2])] - E1[o0]);
  out[sface(n, d, i, j, k)] = Pd[pface(N, d, i, j, k)] - dtdx * curl;
}

// ---------------------------------------------------------------------------
// k_publish: the new slice becomes current (Sec. 3A), ticks advance.

#ifdef DSP_TU_COMMON
__global__ void k_publish(DevSet S, const int* __restrict__ list, int count, StepPtr st) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= live_count(S, count)) return;
  if (b == 0 && S.rounds) atomicAdd(S.rounds, 1);
  publish_patch(S, list[b], st, b);
}

// k_output: the output cadence (Sec. 3E).  A listed patch whose new time is
// a multiple of the output interval copies its new slice into the frame of
// that time (after k_publish, so the slice is current).

__global__ void k_output(DevSet S, const int* __restrict__ list, int count, const void* __restrict__ slots) {
  const int b = blockIdx.y;
  if (b >= live_count(S, count)) return;
  const int p = list[b];
  const int f = output_frame(S, S.ticks[p]);
  if (f < 0) return;
  output_copy(S, p, f, slots, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// ---------------------------------------------------------------------------
// k_scan: readiness of every patch (Eq. (1), with the grace) and the ready list.

__global__ void k_scan(DevSet S, int64_t T_end, int* __restrict__ list, int* __restrict__ counters,
                       int* __restrict__ clear) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // the other counter pair, which the next round's scan uses (the round
  // before this one has finished reading it)
  if (clear && i == 0) {
    clear[0] = 0;
    clear[1] = 0;
  }
  if (i >= S.npatch) return;
  // patches in decreasing size: the ready list then starts with the longest
  // updates, whose workgroups are dispatched first (the order of a round
  // does not change its result)
  const int p = S.scan_order[i];
  if (*S.err) return;  // an error stops the scheduling: later rounds find nothing to do
  if (S.frozen[p]) return;  // boundary patches never update
  const int64_t t = S.ticks[p];
  if (t >= T_end) return;
  atomicAdd(counters + 1, 1);  // not yet done
  // Eq. (1): t_p <= t_q + floor(g dt_q) for every neighbour q (dt_q: the step
  // q took last, 0 before its first); and p's oldest slot, which the update
  // overwrites, must not be needed by any neighbour any more: the slice after
  // it is not newer than the neighbour (implied when g = 0)
  const int ns = S.nslots;
  const int64_t ob = (int64_t)p * ns;
  // (with time order 2 the slice before a bracket is read too: two are kept)
  const int oldest = (S.cur[p] + 1) % ns, after = (S.cur[p] + 1 + (S.torder > 1 ? 2 : 1)) % ns;
  const int64_t t_after = S.svalid[ob + oldest] ? S.sticks[ob + after] : INT64_MIN;
  // the neighbours' times are fetched eight at a time before any is tested,
  // so their loads overlap instead of waiting on each other
  const int m0 = S.nb_off[p], m1 = S.nb_off[p + 1];
  for (int mb = m0; mb < m1; mb += 8) {
    int qs[8];
    int64_t tqs[8];
    bool fz[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) qs[u] = mb + u < m1 ? S.nb_idx[mb + u] : -1;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      tqs[u] = qs[u] >= 0 ? S.ticks[qs[u]] : INT64_MAX;
      fz[u] = qs[u] < 0 || S.frozen[qs[u]];  // boundary patches never lag
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (fz[u]) continue;
      const int q = qs[u];
      const int64_t tq = tqs[u];
      int64_t g = 0;
      if (S.grace > 0.0 && S.steps[q] > 0) {
        const int prev = (S.cur[q] + ns - 1) % ns;
        if (S.svalid[(int64_t)q * ns + prev]) g = (int64_t)floor(S.grace * (double)(tq - S.sticks[(int64_t)q * ns + prev]));
      }
      if (t > tq + g || t_after > tq) return;
    }
  }
  const int slot = atomicAdd(counters, 1);
  // a capped round takes the first scan_cap ready patches; the others stay
  // ready for the next round (with g = 0 the order of the updates does not
  // change the result)
  if (S.scan_cap > 0 && slot >= S.scan_cap) return;
  list[slot] = p;
}
#endif  // DSP_TU_COMMON

// ---------------------------------------------------------------------------
// diagnostics: per-patch FP64 sums (one workgroup per patch, fixed-order tree
// reduction, so the result does not depend on scheduling)

template <class T>
__global__ void k_stats(DevSet S, const T* __restrict__ slots, double* __restrict__ out) {
  const int p = blockIdx.x;
  const int n = S.n[p];
  const int64_t n3 = (int64_t)n * n * n;
  const T* u = slots + S.slot_off[p] + (int64_t)S.cur[p] * S.slice_len[p];
  const double dv = S.dx[p] * S.dx[p] * S.dx[p];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double dmax = 0.0;
  for (int64_t c = threadIdx.x; c < n3; c += blockDim.x) {
    const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / ((int64_t)n * n));
    for (int v = 0; v < 5; ++v) acc[v] += (double)u[scell(n, v, i, j, k)] * dv;
    const double bl[3] = {(double)u[sface(n, 0, i, j, k)], (double)u[sface(n, 1, i, j, k)],
                          (double)u[sface(n, 2, i, j, k)]};
    const double br[3] = {(double)u[sface(n, 0, i + 1, j, k)], (double)u[sface(n, 1, i, j + 1, k)],
                          (double)u[sface(n, 2, i, j, k + 1)]};
    for (int d = 0; d < 3; ++d) acc[5 + d] += 0.5 * (bl[d] + br[d]) * dv;
    const double dvg = fabs((br[0] - bl[0]) + (br[1] - bl[1]) + (br[2] - bl[2])) / S.dx[p];
    dmax = dvg > dmax ? dvg : dmax;
  }
  __shared__ double red[256];
  for (int q = 0; q < 9; ++q) {
    red[threadIdx.x] = (q < 8) ? acc[q] : dmax;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s)
        red[threadIdx.x] = (q < 8) ? red[threadIdx.x] + red[threadIdx.x + s]
                                   : (red[threadIdx.x + s] > red[threadIdx.x] ? red[threadIdx.x + s] : red[threadIdx.x]);
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)p * 9 + q] = red[0];
    __syncthreads();
  }
}

// host layout <-> ring slot (the host layout is the concatenation of slices)
template <class T>
__global__ void k_gather(DevSet S, const T* __restrict__ slots, double* __restrict__ dst,
                         const int64_t* __restrict__ host_off) {
  const int p = blockIdx.y;
  const int64_t V = S.slice_len[p];
  const T* src = slots + S.slot_off[p] + (int64_t)S.cur[p] * V;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < V; e += (int64_t)gridDim.x * blockDim.x)
    dst[host_off[p] + e] = (double)src[e];
}

template <class T>
__global__ void k_scatter(DevSet S, T* __restrict__ slots, const double* __restrict__ src,
                          const int64_t* __restrict__ host_off) {
  const int p = blockIdx.y;
  const int64_t V = S.slice_len[p];
  T* dst = slots + S.slot_off[p];  // slot 0
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < V; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (T)src[host_off[p] + e];
}

// copy between the host-layout (contiguous) representation and slot 0 / the
// current slot in the set's precision, device to device (fixed-step entry)
template <class T>
__global__ void k_pack(DevSet S, const T* __restrict__ slots, T* __restrict__ dst,
                       const int64_t* __restrict__ host_off) {
  const int p = blockIdx.y;
  const int64_t V = S.slice_len[p];
  const T* src = slots + S.slot_off[p] + (int64_t)S.cur[p] * V;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < V; e += (int64_t)gridDim.x * blockDim.x)
    dst[host_off[p] + e] = src[e];
}
template <class T>
__global__ void k_unpack(DevSet S, T* __restrict__ slots, const T* __restrict__ src,
                         const int64_t* __restrict__ host_off) {
  const int p = blockIdx.y;
  const int64_t V = S.slice_len[p];
  T* dst = slots + S.slot_off[p];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < V; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[host_off[p] + e];
}

// ---------------------------------------------------------------------------
// k_hlld_faces: the HLLD flux of a batch of independent faces with the step
// kernels' own arithmetic (single precision: hardware reciprocal and square
// root, as the fused single-precision step; double: IEEE), for element-wise
// checks of the flux on its own.  One thread per face; FP64 in and out.

template <class T, class M>
__global__ void k_hlld_faces(const double* __restrict__ wl, const double* __restrict__ wr,
                             const double* __restrict__ bn, int64_t nface, double gamma, double* __restrict__ out) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nface) return;
  T l[7], r[7], F[8];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    l[q] = (T)wl[7 * f + q];
    r[q] = (T)wr[7 * f + q];
  }
  hlld_flux<T, M>(l, r, (T)bn[f], (T)gamma, F);
#pragma unroll
  for (int q = 0; q < 8; ++q) out[8 * f + q] = (double)F[q];
}

// ---------------------------------------------------------------------------
// launchers (explicit instantiation for float and double)

template <class T>
void launch_update(const DevSet& S, const int* list, int count, int nmax, T* slots, const WorkPtr<T>& W,
                   const StepPtr& st, hipStream_t s, int dt_kind, double t_end, int clip,
                   hipEvent_t ev0, hipEvent_t ev1) {
  const int N = nmax + 4, M = nmax + 2;
  const int TPB = 256;
  auto blocks = [&](int64_t elems) { return (unsigned)((elems + TPB - 1) / TPB); };
  (void)hipMemsetAsync(W.smax, 0, sizeof(double) * count, s);
  const int64_t fill_elems = 5LL * N * N * N + 3LL * N * N * (N + 1);
  launch_brackets(S, list, count, s);
  hipLaunchKernelGGL(k_fill<T>, dim3(blocks(fill_elems), count), dim3(TPB), 0, s, S, list, count, slots, W);
  hipLaunchKernelGGL(k_prim<T>, dim3(blocks((int64_t)N * N * N), count), dim3(TPB), 0, s, S, list, count, W);
  launch_dt(S, list, count, st, W.smax, s, dt_kind, t_end, clip);
  hipLaunchKernelGGL(k_pred<T>, dim3(blocks((int64_t)M * M * M), count), dim3(TPB), 0, s, S, list, count, W, st);
  if (ev0) (void)hipEventRecord(ev0, s);
  hipLaunchKernelGGL(k_flux<T>, dim3(blocks(3LL * (nmax + 1) * M * M), count), dim3(TPB), 0, s, S, list, count, W);
  if (ev1) (void)hipEventRecord(ev1, s);
  hipLaunchKernelGGL(k_emf<T>, dim3(blocks(3LL * nmax * (nmax + 1) * (nmax + 1)), count), dim3(TPB), 0, s, S, list,
                     count, W);
  if (S.nonideal) {
    hipLaunchKernelGGL(k_ni_emf<T>, dim3(blocks(3LL * nmax * (nmax + 1) * (nmax + 1)), count), dim3(TPB), 0, s, S,
                       list, count, W);
    hipLaunchKernelGGL(k_ni_flux<T>, dim3(blocks(3LL * (nmax + 1) * nmax * nmax), count), dim3(TPB), 0, s, S, list,
                       count, W);
  }
  hipLaunchKernelGGL(k_update<T>, dim3(blocks((int64_t)nmax * nmax * nmax + 3LL * nmax * nmax * (nmax + 1)), count),
                     dim3(TPB), 0, s, S, list, count, slots, W, st);
}

#ifdef DSP_TU_COMMON
void launch_brackets(const DevSet& S, const int* list, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_brackets, dim3((unsigned)((S.maxbox > 0 ? S.maxbox : 1) + 255) / 256, count), dim3(256), 0, s,
                     S, list, count);
}

void launch_dt(const DevSet& S, const int* list, int count, const StepPtr& st, const double* smax, hipStream_t s,
               int dt_kind, double t_end, int clip) {
  if (dt_kind == 0)
    hipLaunchKernelGGL(k_dt_local, dim3((count + 255) / 256), dim3(256), 0, s, S, list, count, st, smax);
  else
    hipLaunchKernelGGL(k_dt_global, dim3(1), dim3(256), 0, s, S, list, count, st, smax, t_end, clip);
}

// Time records of every patch back to t = 0 with one valid slice (slot 0),
// as a fresh initialisation at t0 = 0 in the exact-time modes, on the device;
// the statistics counters are cleared, the error flags are kept.
__global__ void k_reset_times(DevSet S, unsigned long long* cnt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0)
    for (int q = 0; q < 4; ++q) cnt[q] = 0ULL;
  if (p >= S.npatch) return;
  const int ns = S.nslots;
  S.cur[p] = 0;
  S.ticks[p] = 0;
  S.tcur[p] = 0.0;
  for (int q = 0; q < ns; ++q) {
    S.sticks[(int64_t)p * ns + q] = 0;
    S.stime[(int64_t)p * ns + q] = 0.0;
    S.svalid[(int64_t)p * ns + q] = q == 0 ? 1 : 0;
  }
  S.steps[p] = 0;
  S.khash[p] = 1469598103934665603ull;
  for (int m = 0; m < S.klog_cap; ++m) S.klog[(int64_t)p * S.klog_cap + m] = -2;
}

void launch_reset_times(const DevSet& S, unsigned long long* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_times, dim3((S.npatch + 255) / 256), dim3(256), 0, s, S, cnt);
}

void launch_publish(const DevSet& S, const int* list, int count, const StepPtr& st, hipStream_t s,
                    const void* slots) {
  hipLaunchKernelGGL(k_publish, dim3((count + 255) / 256), dim3(256), 0, s, S, list, count, st);
  if (S.out_frames && slots)
    hipLaunchKernelGGL(k_output, dim3(64, count), dim3(256), 0, s, S, list, count, slots);
}

void launch_scan(const DevSet& S, int64_t T_end, int* list, int* counters, hipStream_t s, int* clear) {
  // counters must be zero: cleared here, or by the previous scan (clear)
  if (!clear) (void)hipMemsetAsync(counters, 0, 2 * sizeof(int), s);
  hipLaunchKernelGGL(k_scan, dim3((S.npatch + 255) / 256), dim3(256), 0, s, S, T_end, list, counters, clear);
}
#endif  // DSP_TU_COMMON

template <class T>
void launch_stats(const DevSet& S, const T* slots, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_stats<T>, dim3(S.npatch), dim3(256), 0, s, S, slots, out);
}

template <class T>
void launch_gather(const DevSet& S, const T* slots, double* dst, const int64_t* host_off, hipStream_t s) {
  hipLaunchKernelGGL(k_gather<T>, dim3(64, S.npatch), dim3(256), 0, s, S, slots, dst, host_off);
}
template <class T>
void launch_scatter(const DevSet& S, T* slots, const double* src, const int64_t* host_off, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter<T>, dim3(64, S.npatch), dim3(256), 0, s, S, slots, src, host_off);
}
template <class T>
void launch_pack(const DevSet& S, const T* slots, T* dst, const int64_t* host_off, hipStream_t s) {
  hipLaunchKernelGGL(k_pack<T>, dim3(64, S.npatch), dim3(256), 0, s, S, slots, dst, host_off);
}
template <class T>
void launch_unpack(const DevSet& S, T* slots, const T* src, const int64_t* host_off, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack<T>, dim3(64, S.npatch), dim3(256), 0, s, S, slots, src, host_off);
}

// Every ring slot but slot 0 of every patch set to NaN (a checking switch:
// a guard value read from a slot that was never written then shows up as a
// non-finite state at once).
template <class T>
__global__ void k_poison(DevSet S, T* __restrict__ slots) {
  const int p = blockIdx.y;
  const int64_t V = S.slice_len[p];
  T* base = slots + S.slot_off[p] + V;
  const int64_t n = V * (S.nslots - 1);
  const T nan = __builtin_nan("");
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    base[e] = nan;
}

template <class T>
void launch_poison(const DevSet& S, T* slots, hipStream_t s) {
  if (S.nslots > 1) hipLaunchKernelGGL(k_poison<T>, dim3(64, S.npatch), dim3(256), 0, s, S, slots);
}

template <class T>
void launch_hlld_faces(const double* wl, const double* wr, const double* bn, int64_t nface, double gamma, double* out,
                       hipStream_t s) {
  if (nface <= 0) return;
  const unsigned blocks = (unsigned)((nface + 255) / 256);
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL((k_hlld_faces<float, FastF32>), dim3(blocks), dim3(256), 0, s, wl, wr, bn, nface, gamma, out);
  else
    hipLaunchKernelGGL((k_hlld_faces<double, Exact<double>>), dim3(blocks), dim3(256), 0, s, wl, wr, bn, nface, gamma,
                       out);
}

#define DSP_INST(T)                                                                                    \
  template void launch_poison<T>(const DevSet&, T*, hipStream_t);                                      \
  template void launch_hlld_faces<T>(const double*, const double*, const double*, int64_t, double, double*, \
                                     hipStream_t);                                                     \
  template void launch_update<T>(const DevSet&, const int*, int, int, T*, const WorkPtr<T>&,          \
                                 const StepPtr&, hipStream_t, int, double, int, hipEvent_t, hipEvent_t); \
  template void launch_stats<T>(const DevSet&, const T*, double*, hipStream_t);                        \
  template void launch_gather<T>(const DevSet&, const T*, double*, const int64_t*, hipStream_t);       \
  template void launch_scatter<T>(const DevSet&, T*, const double*, const int64_t*, hipStream_t);      \
  template void launch_pack<T>(const DevSet&, const T*, T*, const int64_t*, hipStream_t);              \
  template void launch_unpack<T>(const DevSet&, T*, const T*, const int64_t*, hipStream_t);
#ifdef DSP_TU_F32
DSP_INST(float)
#endif
#ifdef DSP_TU_F64
DSP_INST(double)
#endif

}  // namespace dsp
