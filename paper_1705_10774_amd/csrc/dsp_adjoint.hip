// dsp_adjoint.hip -- reverse (adjoint) of one fixed-dt step of the whole set.
//
// The forward step is the staged one (k_fill, k_prim, k_pred, k_flux, k_emf,
// k_update), run on the state U^k so that its intermediates sit in the work
// buffers.  Given lam^{k+1} = dJ/dU^{k+1} (host layout), the kernels below
// accumulate lam^k = (dU^{k+1}/dU^k)^T lam^{k+1}, walking the stages backwards:
//
//   update  -> fluxes, edge EMFs, padded state (identity part)
//   EMFs    -> induction fluxes, half-step state (cell EMF -v x B)
//   fluxes  -> half-step state, slopes, primitives, padded face field
//   Hancock -> primitives, slopes
//   slopes  -> primitives
//   prims   -> padded state
//   fill    -> lam^k of the owning patch (interior) or of the source patch
//              (guard copy; all patches share the time of a fixed step)
//
// The upwind choices of the EMFs, the first-order fallback and the Riemann
// solver's wave pattern are those of the forward state: the result is the
// derivative along the branches the forward step takes.  The Riemann solver
// and the predictor have hand-written reverse passes (hlld_vjp.h, k_adj_pred).
// Every kernel gathers (one writer per entry, a fixed order of every sum), so
// the reverse run is deterministic: two runs give the same bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsp_dev.h"
#include "dsp_guard.h"
#include "hlld_vjp.h"
#include "mhd_dev.h"

namespace dsp {

// ---------------------------------------------------------------------------
// update: out = P - dtdx * sum_d (F_d(+) - F_d(-)) for the cells,
//         out = P - dtdx * curl(E) for the faces.

template <class T>
__global__ __launch_bounds__(256) void k_adj_update(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> L, StepPtr st,
                             const T* __restrict__ lam, const int64_t* __restrict__ host_off) {
  // Gathered, one writer per entry: the cells (lam to the padded state), the
  // faces (lam of the face field to the padded state; the flux cotangents
  // +dtdx lam of the cell above and -dtdx lam of the cell below) and the
  // edges (the four faces whose curl the edge EMF enters).  L.f and L.e are
  // first written here, every entry that later kernels read: all eight
  // slots of the faces of [-1, n] in the transverse directions (zero where
  // no cell updates), and every edge; so they need no clearing.
  const int blk = blockIdx.y;
  if (blk >= count) return;
  const int p = list[blk];
  const int n = S.n[p], N = n + 4, M = n + 2;
  const int64_t n3 = (int64_t)n * n * n, nf = (int64_t)(n + 1) * M * M, ne = (int64_t)n * (n + 1) * (n + 1);
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n3 + 3 * nf + 3 * ne) return;
  const T* lo = lam + host_off[p];
  T* LP = L.pad + (int64_t)blk * L.pad_stride;
  const T dtdx = (T)(st.dt[blk] / S.dx[p]);
  const int64_t fs = L.fm3;
  if (c < n3) {
    const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / ((int64_t)n * n));
    for (int v = 0; v < 5; ++v) LP[pcell(N, v, i, j, k)] += lo[scell(n, v, i, j, k)];
    return;
  }
  c -= n3;
  if (c < 3 * nf) {
    // faces f[d] in [0, n], the other two indices in [-1, n]; x fastest
    const int d = (int)(c / nf);
    c -= d * nf;
    const int e0 = d == 0 ? n + 1 : M, e1 = d == 1 ? n + 1 : M;
    int f[3] = {(int)(c % e0) - (d == 0 ? 0 : 1), (int)((c / e0) % e1) - (d == 1 ? 0 : 1),
                (int)(c / ((int64_t)e0 * e1)) - (d == 2 ? 0 : 1)};
    bool inner = true;  // a face of the patch (its face field and its two cells)
    for (int e = 0; e < 3; ++e)
      if (e != d) inner = inner && f[e] >= 0 && f[e] < n;
    if (inner) LP[pface(N, d, f[0], f[1], f[2])] += lo[sface(n, d, f[0], f[1], f[2])];
    const int64_t of = wface(N, 0, f[0], f[1], f[2]);
    T* LF = L.f + (int64_t)blk * L.f_stride + (int64_t)d * 8 * fs;
    const bool above = inner && f[d] < n, below = inner && f[d] > 0;
    int g[3] = {f[0], f[1], f[2]};
    g[d] -= 1;
    for (int v = 0; v < 5; ++v) {
      const T a = above ? dtdx * lo[scell(n, v, f[0], f[1], f[2])] : T(0);
      const T b = below ? -dtdx * lo[scell(n, v, g[0], g[1], g[2])] : T(0);
      LF[v * fs + of] = a + b;
    }
    for (int v = 5; v < 8; ++v) LF[v * fs + of] = T(0);
    return;
  }
  c -= 3 * nf;
  const int ax = (int)(c / ne);
  c -= ax * ne;
  const int x0 = ax == 0 ? n : n + 1, x1 = ax == 1 ? n : n + 1;
  const int x[3] = {(int)(c % x0), (int)((c / x0) % x1), (int)(c / ((int64_t)x0 * x1))};
  // lam of face (d, q) of the face field, 0 off the patch's faces
  auto lamf = [&](int d, const int* q) -> T {
    for (int e = 0; e < 3; ++e)
      if (q[e] < 0 || q[e] > (e == d ? n : n - 1)) return T(0);
    return lo[sface(n, d, q[0], q[1], q[2])];
  };
  // faces of direction d1 = ax + 1 see this edge as their E_t2 (at q and at
  // q + e_t1), faces of direction d2 = ax + 2 as their E_t1 (at q and q + e_t2)
  const int d1 = (ax + 1) % 3, d2 = (ax + 2) % 3;
  const int t1 = (d1 + 1) % 3, t2 = (d2 + 2) % 3;
  int q1[3] = {x[0], x[1], x[2]}, q2[3] = {x[0], x[1], x[2]};
  q1[t1] -= 1;
  q2[t2] -= 1;
  const T e = (dtdx * lamf(d1, x) - dtdx * lamf(d1, q1)) + (dtdx * lamf(d2, q2) - dtdx * lamf(d2, x));
  L.e[(int64_t)blk * L.e_stride + (int64_t)ax * fs + wface(N, 0, x[0], x[1], x[2])] = e;
}

// ---------------------------------------------------------------------------
// edge EMFs (Gardiner & Stone E^c, upwinded by the face upwind speed)

template <class T> __device__ __forceinline__ void up_adj(T u, T lam, T& la, T& lb) {
  if (u > T(0)) {
    la += lam;
  } else if (u < T(0)) {
    lb += lam;
  } else {
    la += T(0.5) * lam;
    lb += T(0.5) * lam;
  }
}

// Cotangent weights of edge (a, e), e[a] in [0, n), the others in [0, n]:
// E = (A + B + C + D)/4 + ((dc34 - dc14) + (db34 - db14))/4 with
//   dc14 = up(uA, c01 - D, c11 - C), dc34 = up(uB, D - c00, C - c10),
//   db14 = up(uC, c10 - B, c11 - A), db34 = up(uD, B - c00, A - c01),
// A, B the b-face and C, D the c-face EMFs and c.. the cell EMFs around the
// edge; l[0..3] = lam of A, B, C, D, l[4..7] = lam of c00, c10, c01, c11.
template <class T>
__device__ __forceinline__ void emf_weights(const WorkPtr<T>& W, int blk, int N, int a, const int* e, T lamE, T* l) {
  const int bax = (a + 1) % 3, cax = (a + 2) % 3;
  const int64_t fs = W.fm3;
  const T* Fb = W.f + (int64_t)blk * W.f_stride + (int64_t)bax * 8 * fs;
  const T* Fc = W.f + (int64_t)blk * W.f_stride + (int64_t)cax * 8 * fs;
  int pB[3] = {e[0], e[1], e[2]}, pD[3] = {e[0], e[1], e[2]};
  pB[cax] -= 1;
  pD[bax] -= 1;
  const int64_t oA = wface(N, 0, e[0], e[1], e[2]), oB = wface(N, 0, pB[0], pB[1], pB[2]);
  const int64_t oD = wface(N, 0, pD[0], pD[1], pD[2]);
  // upwind speeds (the slot of the normal component holds them)
  const T uA = Fb[(5 + bax) * fs + oA], uB = Fb[(5 + bax) * fs + oB];
  const T uC = Fc[(5 + cax) * fs + oA], uD = Fc[(5 + cax) * fs + oD];
  const T q = T(0.25) * lamE;
  T lA = q, lB = q, lC = q, lD = q, l00 = 0, l10 = 0, l01 = 0, l11 = 0;
  T x, y;
  x = y = T(0);  // dc14: weight -q
  up_adj(uA, -q, x, y);
  l01 += x; lD -= x; l11 += y; lC -= y;
  x = y = T(0);  // dc34: weight +q
  up_adj(uB, q, x, y);
  lD += x; l00 -= x; lC += y; l10 -= y;
  x = y = T(0);  // db14: weight -q
  up_adj(uC, -q, x, y);
  l10 += x; lB -= x; l11 += y; lA -= y;
  x = y = T(0);  // db34: weight +q
  up_adj(uD, q, x, y);
  lB += x; l00 -= x; lA += y; l01 -= y;
  l[0] = lA; l[1] = lB; l[2] = lC; l[3] = lD;
  l[4] = l00; l[5] = l10; l[6] = l01; l[7] = l11;
}

// Pass 1: the weights of every edge, stored in the slope-cotangent buffer
// (free until k_adj_flux_sum writes it): 8 per edge and direction, edges
// x-fastest in the box [0, n)_a x [0, n]^2.
template <class T>
__global__ __launch_bounds__(256) void k_adj_emf(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W, WorkPtr<T> L) {
  const int blk = blockIdx.y;
  if (blk >= count) return;
  const int p = list[blk];
  const int n = S.n[p], N = n + 4;
  const int64_t ne = (int64_t)n * (n + 1) * (n + 1);
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 3 * ne) return;
  const int a = (int)(c / ne);
  c -= a * ne;
  const int x0 = a == 0 ? n : n + 1, x1 = a == 1 ? n : n + 1;
  const int e[3] = {(int)(c % x0), (int)((c / x0) % x1), (int)(c / ((int64_t)x0 * x1))};
  const T lamE = L.e[(int64_t)blk * L.e_stride + (int64_t)a * W.fm3 + wface(N, 0, e[0], e[1], e[2])];
  T l[8];
  if (lamE == T(0)) {
    for (int k = 0; k < 8; ++k) l[k] = T(0);
  } else {
    emf_weights(W, blk, N, a, e, lamE, l);
  }
  T* G = L.s + (int64_t)blk * L.s_stride + (int64_t)a * 8 * ne;
  for (int k = 0; k < 8; ++k) G[k * ne + c] = l[k];
}

// Pass 2, one writer per entry: the face EMFs' weights to the induction
// fluxes of the faces (A = -F_b[B_c], B likewise one c-cell lower, C = F_c[B_b],
// D likewise one b-cell lower), the cell-EMF weights (E_a = v_c B_b - v_b B_c
// of the half-step state) to the cells.  Faces of [-1, n] across, cells of
// [-1, n]^3.
template <class T>
__global__ __launch_bounds__(256) void k_adj_emf_sum(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W,
                                                     WorkPtr<T> L) {
  const int blk = blockIdx.y;
  if (blk >= count) return;
  const int p = list[blk];
  const int n = S.n[p], N = n + 4, M = n + 2;
  const int64_t ne = (int64_t)n * (n + 1) * (n + 1), nfm = (int64_t)(n + 1) * M * M;
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 3 * nfm + (int64_t)M * M * M) return;
  const T* G = L.s + (int64_t)blk * L.s_stride;
  // weight k of a-edge q (0 off the edge box)
  auto wt = [&](int a, const int* q, int k) -> T {
    const int x0 = a == 0 ? n : n + 1, x1 = a == 1 ? n : n + 1, x2 = a == 2 ? n : n + 1;
    if (q[0] < 0 || q[0] >= x0 || q[1] < 0 || q[1] >= x1 || q[2] < 0 || q[2] >= x2) return T(0);
    return G[((int64_t)a * 8 + k) * ne + ((int64_t)q[2] * x1 + q[1]) * x0 + q[0]];
  };
  const int64_t fs = W.fm3;
  if (c < 3 * nfm) {
    const int d = (int)(c / nfm);
    c -= d * nfm;
    const int e0 = d == 0 ? n + 1 : M, e1 = d == 1 ? n + 1 : M;
    const int f[3] = {(int)(c % e0) - (d == 0 ? 0 : 1), (int)((c / e0) % e1) - (d == 1 ? 0 : 1),
                      (int)(c / ((int64_t)e0 * e1)) - (d == 2 ? 0 : 1)};
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    // edges a1 = d + 2 (b-axis d, c-axis t1): A at the edge, B one t1-cell up
    const int a1 = (d + 2) % 3, a2 = (d + 1) % 3;
    int g1[3] = {f[0], f[1], f[2]}, g2[3] = {f[0], f[1], f[2]};
    g1[t1] += 1;
    g2[t2] += 1;
    const T s1 = -wt(a1, f, 0) - wt(a1, g1, 1);
    // edges a2 = d + 1 (c-axis d, b-axis t2): C at the edge, D one t2-cell up
    const T s2 = wt(a2, f, 2) + wt(a2, g2, 3);
    T* LF = L.f + (int64_t)blk * L.f_stride + (int64_t)d * 8 * fs;
    const int64_t of = wface(N, 0, f[0], f[1], f[2]);
    LF[(5 + t1) * fs + of] += s1;
    LF[(5 + t2) * fs + of] += s2;
    return;
  }
  c -= 3 * nfm;
  const int qq[3] = {(int)(c % M) - 1, (int)((c / M) % M) - 1, (int)(c / ((int64_t)M * M)) - 1};
  const int64_t NC = (int64_t)N * N * N;
  const int64_t o = wcell(N, 0, qq[0], qq[1], qq[2]);
  const T* Hp = W.h + (int64_t)blk * W.w_stride;
  T* LH = L.h + (int64_t)blk * L.w_stride;
  T acc[8];
  for (int v = 0; v < 8; ++v) acc[v] = T(0);
  for (int a = 0; a < 3; ++a) {
    const int bax = (a + 1) % 3, cax = (a + 2) % 3;
    // the cell is c00 of edge qq + e_b + e_c, c10 of qq + e_c, c01 of qq + e_b, c11 of qq
    int e00[3] = {qq[0], qq[1], qq[2]}, e10[3] = {qq[0], qq[1], qq[2]}, e01[3] = {qq[0], qq[1], qq[2]};
    e00[bax] += 1;
    e00[cax] += 1;
    e10[cax] += 1;
    e01[bax] += 1;
    const T lc = wt(a, e00, 4) + wt(a, e10, 5) + wt(a, e01, 6) + wt(a, qq, 7);
    if (lc == T(0)) continue;
    const T vc = Hp[(1 + cax) * NC + o], bb = Hp[(5 + bax) * NC + o];
    const T vb = Hp[(1 + bax) * NC + o], bc = Hp[(5 + cax) * NC + o];
    acc[1 + cax] += lc * bb;
    acc[5 + bax] += lc * vc;
    acc[1 + bax] -= lc * bc;
    acc[5 + cax] -= lc * vb;
  }
  for (int v = 0; v < 8; ++v)
    if (acc[v] != T(0)) LH[v * NC + o] += acc[v];
}

// ---------------------------------------------------------------------------
// interface fluxes

template <class T>
__global__ __launch_bounds__(256, 2) void k_adj_flux(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W, WorkPtr<T> L) {
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
  const int64_t fs = W.fm3;
  const int64_t of = wface(N, 0, idx[0], idx[1], idx[2]);
  const T* LF = L.f + (int64_t)b * L.f_stride + (int64_t)d * 8 * fs;
  T lf[7];
  lf[0] = LF[of];
  lf[1] = LF[(1 + d) * fs + of];
  lf[2] = LF[(1 + t1) * fs + of];
  lf[3] = LF[(1 + t2) * fs + of];
  lf[4] = LF[4 * fs + of];
  lf[5] = LF[(5 + t1) * fs + of];
  lf[6] = LF[(5 + t2) * fs + of];
  // The face's 15 cotangents go to the flux buffers, which no later kernel
  // of this step reads: the left-state ones (and the fallback flag, in the
  // slot of the normal field, which has no flux) over lf in L.f, the
  // right-state ones and that of bn over the forward fluxes in W.f.
  // k_adj_flux_sum adds them into the cells without atomics.
  T* GL = L.f + (int64_t)b * L.f_stride + (int64_t)d * 8 * fs;
  T* GR = W.f + (int64_t)b * W.f_stride + (int64_t)d * 8 * fs;
  bool any = false;
  for (int q = 0; q < 7; ++q) any = any || lf[q] != T(0);
  if (!any) {  // L.f already holds zeros here
    for (int v = 0; v < 8; ++v) GR[v * fs + of] = T(0);
    return;
  }
  const T* Wp = W.w + (int64_t)b * W.w_stride;
  const T* Hp = W.h + (int64_t)b * W.w_stride;
  const T* Sp = W.s + (int64_t)b * W.s_stride;
  const T* Pd = W.pad + (int64_t)b * W.pad_stride;
  T* LP = L.pad + (int64_t)b * L.pad_stride;
  const int64_t NC = (int64_t)N * N * N;
  const int64_t ca = wcell(N, 0, ia[0], ia[1], ia[2]), cb = wcell(N, 0, idx[0], idx[1], idx[2]);
  const int order[7] = {0, 1 + d, 1 + t1, 1 + t2, 4, 5 + t1, 5 + t2};
  T l[7], r[7];
  for (int m = 0; m < 7; ++m) {
    const int v = order[m];
    l[m] = Hp[v * NC + ca] + T(0.5) * Sp[(int64_t)(d * 8 + v) * NC + ca];
    r[m] = Hp[v * NC + cb] - T(0.5) * Sp[(int64_t)(d * 8 + v) * NC + cb];
  }
  const int64_t opf = pface(N, d, idx[0], idx[1], idx[2]);
  const T bface = Pd[opf];
  T bn = bface + T(0.5) * ((Hp[(5 + d) * NC + ca] - Wp[(5 + d) * NC + ca]) +
                           (Hp[(5 + d) * NC + cb] - Wp[(5 + d) * NC + cb]));
  const bool fallback = !(l[0] > T(0)) || !(l[4] > T(0)) || !(r[0] > T(0)) || !(r[4] > T(0));
  if (fallback) {
    for (int m = 0; m < 7; ++m) {
      l[m] = Wp[order[m] * NC + ca];
      r[m] = Wp[order[m] * NC + cb];
    }
    bn = bface;
  }
  // lam of the 15 inputs (l, r, bn): one reverse pass through the HLLD flux
  T g[15];
  hlld_vjp<T>(l, r, bn, T(S.gamma), lf, g, g + 7, g[14]);
  for (int m = 0; m < 7; ++m) {
    GL[order[m] * fs + of] = g[m];
    GR[order[m] * fs + of] = g[7 + m];
  }
  GL[(5 + d) * fs + of] = fallback ? T(1) : T(0);
  GR[(5 + d) * fs + of] = g[14];
  LP[opf] += g[14];  // the face's own entry: one writer
}

// Sum of the face cotangents of k_adj_flux into cell c of [-1, n]^3: for each
// direction, the face above c (c its left cell) and the face below (c its
// right cell).  Face states l = H + S/2 and r = H - S/2 along the face
// normal; a fallback face took the t^n primitives W instead.  The normal
// field of the face, bn = B_face + (H_a - W_a + H_b - W_b)/2, gives each of
// its two cells lam_bn/2 on H and -lam_bn/2 on W (not for a fallback face).
template <class T>
__global__ __launch_bounds__(256) void k_adj_flux_sum(DevSet S, const int* __restrict__ list, int count,
                                                      WorkPtr<T> W, WorkPtr<T> L) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const int p = list[b];
  const int n = S.n[p], N = n + 4, M = n + 2;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)M * M * M) return;
  const int cc[3] = {(int)(c % M) - 1, (int)((c / M) % M) - 1, (int)(c / ((int64_t)M * M)) - 1};
  const int64_t fs = W.fm3, NC = (int64_t)N * N * N;
  const int64_t oc = wcell(N, 0, cc[0], cc[1], cc[2]);
  T aH[8], aW[8];
  for (int v = 0; v < 8; ++v) aH[v] = aW[v] = T(0);
  T* LS = L.s + (int64_t)b * L.s_stride;
  for (int d = 0; d < 3; ++d) {
    const T* GL = L.f + (int64_t)b * L.f_stride + (int64_t)d * 8 * fs;
    const T* GR = W.f + (int64_t)b * W.f_stride + (int64_t)d * 8 * fs;
    T aS[8];
    for (int v = 0; v < 8; ++v) aS[v] = T(0);
    for (int side = 0; side < 2; ++side) {
      // side 0: the face above (c is its left cell); side 1: the face below
      int f[3] = {cc[0], cc[1], cc[2]};
      if (side == 0) f[d] += 1;
      if (f[d] < 0 || f[d] > n) continue;
      const int64_t of = wface(N, 0, f[0], f[1], f[2]);
      const T* G = side == 0 ? GL : GR;
      const bool fb = GL[(5 + d) * fs + of] != T(0);
      const T sg = side == 0 ? T(0.5) : T(-0.5);
      for (int v = 0; v < 8; ++v) {
        if (v == 5 + d) continue;
        const T g = G[v * fs + of];
        if (fb) {
          aW[v] += g;
        } else {
          aH[v] += g;
          aS[v] += sg * g;
        }
      }
      if (!fb) {
        const T hb = T(0.5) * GR[(5 + d) * fs + of];
        aH[5 + d] += hb;
        aW[5 + d] -= hb;
      }
    }
    // the first writer of the slope cotangents of [-1, n]^3 (no clearing)
    for (int v = 0; v < 8; ++v)
      if (v != 5 + d) LS[(int64_t)(d * 8 + v) * NC + oc] = aS[v];
  }
  T* LW = L.w + (int64_t)b * L.w_stride;
  T* LH = L.h + (int64_t)b * L.w_stride;
  for (int v = 0; v < 8; ++v) {
    if (aH[v] != T(0)) LH[v * NC + oc] += aH[v];
    if (aW[v] != T(0)) LW[v * NC + oc] += aW[v];
  }
}

// ---------------------------------------------------------------------------
// Hancock predictor on [-1, n]^3 (one thread per cell; no other writer of the
// cell's entries in this kernel)

template <class T>
__global__ __launch_bounds__(256) void k_adj_pred(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W, WorkPtr<T> L,
                           StepPtr st) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const int p = list[b];
  const int n = S.n[p], N = n + 4, M = n + 2;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)M * M * M) return;
  const int i = (int)(c % M) - 1, j = (int)((c / M) % M) - 1, k = (int)(c / ((int64_t)M * M)) - 1;
  const int64_t NC = (int64_t)N * N * N;
  const int64_t o = wcell(N, 0, i, j, k);
  T* LH = L.h + (int64_t)b * L.w_stride;
  T lh[8];
  bool any = false;
  for (int v = 0; v < 8; ++v) {
    lh[v] = LH[v * NC + o];
    any = any || lh[v] != T(0);
  }
  if (!any) return;
  const T* Wp = W.w + (int64_t)b * W.w_stride;
  const T* Sp = W.s + (int64_t)b * W.s_stride;
  T* LW = L.w + (int64_t)b * L.w_stride;
  T* LS = L.s + (int64_t)b * L.s_stride;
  T w[8], sl[3][8];
  for (int v = 0; v < 8; ++v) w[v] = Wp[v * NC + o];
  for (int d = 0; d < 3; ++d)
    for (int v = 0; v < 8; ++v) sl[d][v] = Sp[(int64_t)(d * 8 + v) * NC + o];
  const T hdtdx = (T)(0.5 * st.dt[b] / S.dx[p]);
  const T gamma = T(S.gamma);
  // H = w - hdtdx sum(w, sl), with sum the Hancock terms of each direction
  // (mhd_dev.h, hancock): reverse mode by hand.  a = -hdtdx lam_H is the
  // cotangent of sum; sl[d][5 + d] is not an input.
  const T ir = T(1) / w[0];
  T a[8], gw[8];
  for (int v = 0; v < 8; ++v) {
    a[v] = -hdtdx * lh[v];
    gw[v] = lh[v];
  }
  T gir = T(0);  // cotangent of 1/rho
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    const T un = w[1 + d], bn = w[5 + d], b1 = w[5 + t1], b2 = w[5 + t2];
    const T* sd = sl[d];
    const T A0 = a[0], A1 = a[1 + d], A2 = a[1 + t1], A3 = a[1 + t2], A4 = a[4], A5 = a[5 + t1], A6 = a[5 + t2];
    // slopes of direction d
    T gs[8];
    gs[0] = A0 * un;
    gs[1 + d] = A0 * w[0] + A1 * un + A4 * gamma * w[4] + A5 * b1 + A6 * b2;
    gs[1 + t1] = A2 * un - A5 * bn;
    gs[1 + t2] = A3 * un - A6 * bn;
    gs[4] = A1 * ir + A4 * un;
    gs[5 + t1] = A1 * b1 * ir - A2 * bn * ir + A5 * un;
    gs[5 + t2] = A1 * b2 * ir - A3 * bn * ir + A6 * un;
    gs[5 + d] = T(0);
    for (int v = 0; v < 8; ++v)
      if (v != 5 + d) LS[(int64_t)(d * 8 + v) * NC + o] += gs[v];
    // primitives
    gw[1 + d] += A0 * sd[0] + A1 * sd[1 + d] + A2 * sd[1 + t1] + A3 * sd[1 + t2] + A4 * sd[4] +
                 A5 * sd[5 + t1] + A6 * sd[5 + t2];
    gw[0] += A0 * sd[1 + d];
    gir += A1 * (sd[4] + b1 * sd[5 + t1] + b2 * sd[5 + t2]) - A2 * bn * sd[5 + t1] - A3 * bn * sd[5 + t2];
    gw[4] += A4 * gamma * sd[1 + d];
    gw[5 + t1] += A1 * sd[5 + t1] * ir + A5 * sd[1 + d];
    gw[5 + t2] += A1 * sd[5 + t2] * ir + A6 * sd[1 + d];
    gw[5 + d] += -(A2 * sd[5 + t1] + A3 * sd[5 + t2]) * ir - A5 * sd[1 + t1] - A6 * sd[1 + t2];
  }
  gw[0] -= gir * ir * ir;
  for (int v = 0; v < 8; ++v) LW[v * NC + o] += gw[v];
}

// ---------------------------------------------------------------------------
// van Leer slopes S_d(c) = vl(W(c) - W(c - e_d), W(c + e_d) - W(c)), c in [-1, n]^3

template <class T>
__global__ __launch_bounds__(256) void k_adj_slope(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W, WorkPtr<T> L) {
  // Gathered per padded cell c: the slope of cell x = c + s e_d (x in
  // [-1, n]^3) is van Leer of dl = w(x) - w(x - e_d), dr = w(x + e_d) - w(x),
  // with partials 2 dr^2 / (dl + dr)^2 on dl and 2 dl^2 / (dl + dr)^2 on dr,
  // so c receives lam_s(x) times -gl (s = 1), gl - gr (s = 0) or gr (s = -1).
  const int b = blockIdx.y;
  if (b >= count) return;
  const int p = list[b];
  const int n = S.n[p], N = n + 4;
  const int64_t NC = (int64_t)N * N * N;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= NC) return;
  const int cc[3] = {(int)(c % N) - 2, (int)((c / N) % N) - 2, (int)(c / ((int64_t)N * N)) - 2};
  const T* Wp = W.w + (int64_t)b * W.w_stride;
  const T* LS = L.s + (int64_t)b * L.s_stride;
  T* LW = L.w + (int64_t)b * L.w_stride;
  auto inside = [&](const int* x) {
    return x[0] >= -1 && x[0] <= n && x[1] >= -1 && x[1] <= n && x[2] >= -1 && x[2] <= n;
  };
  T acc[8];
  for (int v = 0; v < 8; ++v) acc[v] = T(0);
  for (int d = 0; d < 3; ++d) {
    for (int s = -1; s <= 1; ++s) {
      int x[3] = {cc[0], cc[1], cc[2]};
      x[d] += s;
      if (!inside(x)) continue;
      int xm[3] = {x[0], x[1], x[2]}, xp[3] = {x[0], x[1], x[2]};
      xm[d] -= 1;
      xp[d] += 1;
      const int64_t o = wcell(N, 0, x[0], x[1], x[2]);
      const int64_t om = wcell(N, 0, xm[0], xm[1], xm[2]), op = wcell(N, 0, xp[0], xp[1], xp[2]);
      for (int v = 0; v < 8; ++v) {
        if (v == 5 + d) continue;
        const T ls = LS[(int64_t)(d * 8 + v) * NC + o];
        if (ls == T(0)) continue;
        const T w0 = Wp[v * NC + o];
        const T dl = w0 - Wp[v * NC + om], dr = Wp[v * NC + op] - w0;
        if (!(dl * dr > T(0))) continue;  // limited to zero: no dependence
        const T sum = dl + dr;
        const T gl = T(2) * dr * dr / (sum * sum), gr = T(2) * dl * dl / (sum * sum);
        acc[v] += s == 0 ? ls * (gl - gr) : (s > 0 ? -ls * gl : ls * gr);
      }
    }
  }
  const int64_t oc = wcell(N, 0, cc[0], cc[1], cc[2]);
  for (int v = 0; v < 8; ++v)
    if (acc[v] != T(0)) LW[v * NC + oc] += acc[v];
}

// ---------------------------------------------------------------------------
// primitives over the padded cells [-2, n+1]^3

template <class T>
__global__ __launch_bounds__(256) void k_adj_prim(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> W, WorkPtr<T> L) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const int p = list[b];
  const int n = S.n[p], N = n + 4;
  const int64_t NC = (int64_t)N * N * N;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= NC) return;
  const int i = (int)(c % N) - 2, j = (int)((c / N) % N) - 2, k = (int)(c / ((int64_t)N * N)) - 2;
  const int64_t o = wcell(N, 0, i, j, k);
  T* LW = L.w + (int64_t)b * L.w_stride;
  T lw[8];
  bool any = false;
  for (int v = 0; v < 8; ++v) {
    lw[v] = LW[v * NC + o];
    any = any || lw[v] != T(0);
  }
  if (!any) return;
  const T* Pd = W.pad + (int64_t)b * W.pad_stride;
  T* LP = L.pad + (int64_t)b * L.pad_stride;
  const T rho = Pd[pcell(N, 0, i, j, k)];
  const T m[3] = {Pd[pcell(N, 1, i, j, k)], Pd[pcell(N, 2, i, j, k)], Pd[pcell(N, 3, i, j, k)]};
  const T en = Pd[pcell(N, 4, i, j, k)];
  const int64_t fl[3] = {pface(N, 0, i, j, k), pface(N, 1, i, j, k), pface(N, 2, i, j, k)};
  const int64_t fr[3] = {pface(N, 0, i + 1, j, k), pface(N, 1, i, j + 1, k), pface(N, 2, i, j, k + 1)};
  T bc[3];
  for (int d = 0; d < 3; ++d) bc[d] = T(0.5) * (Pd[fl[d]] + Pd[fr[d]]);
  const T ir = T(1) / rho;
  const T ke = T(0.5) * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * ir;
  const T gm1 = T(S.gamma) - T(1);
  const T pr = gm1 * (en - ke - T(0.5) * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]));
  // a pressure raised to the floor does not depend on the state
  const T lp = (S.p_floor > 0.0 && pr < T(S.p_floor)) ? T(0) : lw[4];
  T lrho = lw[0] + lp * gm1 * ke * ir;
  T lm[3], lb[3];
  for (int d = 0; d < 3; ++d) {
    const T vd = m[d] * ir;
    lrho -= lw[1 + d] * vd * ir;
    lm[d] = lw[1 + d] * ir - lp * gm1 * vd;
    lb[d] = lw[5 + d] - lp * gm1 * bc[d];
  }
  LP[pcell(N, 0, i, j, k)] += lrho;
  for (int d = 0; d < 3; ++d) LP[pcell(N, 1 + d, i, j, k)] += lm[d];
  LP[pcell(N, 4, i, j, k)] += lp * gm1;
  // the cell-centred field's cotangent goes to the two faces it averages
  // (k_adj_prim_faces): kept in place of the cell's own B cotangent, which
  // nothing reads after this kernel (a cell with no cotangent keeps its
  // zeros, which equal its lb)
  for (int d = 0; d < 3; ++d) LW[(5 + d) * NC + o] = lb[d];
}

// faces of the padded patch: half the B cotangent of each of the (at most
// two) padded cells a face bounds
template <class T>
__global__ __launch_bounds__(256) void k_adj_prim_faces(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> L) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const int p = list[b];
  const int n = S.n[p], N = n + 4;
  const int64_t NC = (int64_t)N * N * N, NF = (int64_t)N * N * (N + 1);
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 3 * NF) return;
  const int d = (int)(c / NF);
  c -= d * NF;
  const int sx = N + (d == 0), sy = N + (d == 1);
  int f[3] = {(int)(c % sx) - 2, (int)((c / sx) % sy) - 2, (int)(c / ((int64_t)sx * sy)) - 2};
  const T* LB = L.w + (int64_t)b * L.w_stride + (5 + d) * NC;
  const T right = (f[d] <= n + 1) ? LB[wcell(N, 0, f[0], f[1], f[2])] : T(0);
  f[d] -= 1;
  const T left = (f[d] >= -2) ? LB[wcell(N, 0, f[0], f[1], f[2])] : T(0);
  f[d] += 1;
  L.pad[(int64_t)b * L.pad_stride + pface(N, d, f[0], f[1], f[2])] += T(0.5) * left + T(0.5) * right;
}

// ---------------------------------------------------------------------------
// guard fill: every padded element is the patch's own value (interior) or a
// copy of one source element (same resolution, same time in a fixed step).
// Gathered: each state element of patch q takes the cotangent of its own
// padded element plus those of the guard elements that copy it, found
// through the boxes that read from q (rev).  The list holds every patch in
// id order, so the padded buffers of patch p sit in block p.

template <class T>
__global__ __launch_bounds__(256) void k_adj_fill(DevSet S, const int* __restrict__ list, int count, WorkPtr<T> L,
                           T* __restrict__ lam, const int64_t* __restrict__ host_off) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const int q = list[b];
  const int n = S.n[q], N = n + 4;
  const int64_t n3 = (int64_t)n * n * n, nf = (int64_t)n * n * (n + 1);
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 5 * n3 + 3 * nf) return;
  int comp, var, i, j, k;
  if (e < 5 * n3) {
    comp = -1;
    var = (int)(e / n3);
    const int64_t r = e - var * n3;
    i = (int)(r % n);
    j = (int)((r / n) % n);
    k = (int)(r / ((int64_t)n * n));
  } else {
    int64_t r = e - 5 * n3;
    comp = (int)(r / nf);
    var = 0;
    r -= comp * nf;
    const int sx = n + (comp == 0), sy = n + (comp == 1);
    i = (int)(r % sx);
    j = (int)((r / sx) % sy);
    k = (int)(r / ((int64_t)sx * sy));
  }
  auto padded = [&](int pp, int a, int bb, int c) -> T {
    const int NP = S.n[pp] + 4;
    const int64_t pe = (comp < 0) ? pcell(NP, var, a, bb, c) : pface(NP, comp, a, bb, c);
    return L.pad[(int64_t)pp * L.pad_stride + pe];
  };
  T acc = L.pad[(int64_t)q * L.pad_stride + ((comp < 0) ? pcell(N, var, i, j, k) : pface(N, comp, i, j, k))];
  const int g = q * 4 + comp + 1;
  for (int r = S.rev_off[g]; r < S.rev_off[g + 1]; ++r) {
    const int2 mp = S.rev[r];
    const GBox& G = S.boxes[mp.x];
    const int a = i - G.shift[0], bb = j - G.shift[1], c = k - G.shift[2];
    if (a < G.lo[0] || a > G.hi[0] || bb < G.lo[1] || bb > G.hi[1] || c < G.lo[2] || c > G.hi[2]) continue;
    acc += padded(mp.y, a, bb, c);
  }
  lam[host_off[q] + e] = acc;
}

// ---------------------------------------------------------------------------

template <class T>
void launch_adjoint_step(const DevSet& S, const int* list, int count, int nmax, const WorkPtr<T>& W,
                         const WorkPtr<T>& L, const StepPtr& st, const T* lam_next, T* lam_prev,
                         const int64_t* host_off, hipStream_t s) {
  const int n = nmax, N = n + 4, M = n + 2;
  auto blocks = [](int64_t items) { return (unsigned)((items + 255) / 256); };
  const int64_t n3 = (int64_t)n * n * n;
  const int64_t ne = (int64_t)n * (n + 1) * (n + 1), nfm = (int64_t)(n + 1) * M * M;
  hipLaunchKernelGGL(k_adj_update<T>, dim3(blocks(n3 + 3 * nfm + 3 * ne), count), dim3(256), 0, s, S, list, count, L,
                     st, lam_next, host_off);
  hipLaunchKernelGGL(k_adj_emf<T>, dim3(blocks(3LL * n * (n + 1) * (n + 1)), count), dim3(256), 0, s, S, list, count,
                     W, L);
  hipLaunchKernelGGL(k_adj_emf_sum<T>, dim3(blocks(3 * nfm + (int64_t)M * M * M), count), dim3(256), 0, s, S, list,
                     count, W, L);
  hipLaunchKernelGGL(k_adj_flux<T>, dim3(blocks(3LL * (n + 1) * M * M), count), dim3(256), 0, s, S, list, count, W,
                     L);
  hipLaunchKernelGGL(k_adj_flux_sum<T>, dim3(blocks((int64_t)M * M * M), count), dim3(256), 0, s, S, list, count, W,
                     L);
  hipLaunchKernelGGL(k_adj_pred<T>, dim3(blocks((int64_t)M * M * M), count), dim3(256), 0, s, S, list, count, W, L,
                     st);
  hipLaunchKernelGGL(k_adj_slope<T>, dim3(blocks((int64_t)N * N * N), count), dim3(256), 0, s, S, list, count, W, L);
  hipLaunchKernelGGL(k_adj_prim<T>, dim3(blocks((int64_t)N * N * N), count), dim3(256), 0, s, S, list, count, W, L);
  hipLaunchKernelGGL(k_adj_prim_faces<T>, dim3(blocks(3LL * N * N * (N + 1)), count), dim3(256), 0, s, S, list, count,
                     L);
  hipLaunchKernelGGL(k_adj_fill<T>, dim3(blocks(5 * n3 + 3LL * n * n * (n + 1)), count), dim3(256), 0, s, S, list,
                     count, L, lam_prev, host_off);
}

#ifdef DSP_TU_F32
template void launch_adjoint_step<float>(const DevSet&, const int*, int, int, const WorkPtr<float>&,
                                         const WorkPtr<float>&, const StepPtr&, const float*, float*,
                                         const int64_t*, hipStream_t);
#endif
#ifdef DSP_TU_F64
template void launch_adjoint_step<double>(const DevSet&, const int*, int, int, const WorkPtr<double>&,
                                          const WorkPtr<double>&, const StepPtr&, const double*, double*,
                                          const int64_t*, hipStream_t);
#endif

}  // namespace dsp
