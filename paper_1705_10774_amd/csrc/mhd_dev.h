// mhd_dev.h -- per-cell and per-face arithmetic of the patch step, as
// device functions templated on the stencil precision (float or double).
//
// Ideal MHD, mu0 = 1, gamma-law gas.  The paper leaves the solver to the code
// plugged into its patch tasks (Sec. 4.1) and keeps B divergence-free with
// edge-centred electric fields (constrained transport, Sec. 4.3).  The solver
// here: primitive-variable MUSCL-Hancock with van Leer slopes, HLLD fluxes
// (Miyoshi & Kusano 2005) and the upwinded edge EMFs of Gardiner & Stone
// (2005).
#pragma once
#include <hip/hip_runtime.h>

namespace dsp {

// Arithmetic policy of the stencil.  Exact: IEEE division and square root.
// FastF32: the hardware reciprocal and square root (about 1 ulp each), for
// the single-precision step kernel, whose results are held to the
// single-precision tolerance anyway.
template <class T> struct Exact {
  static __device__ __forceinline__ T rcp(T x) { return T(1) / x; }
  static __device__ __forceinline__ T div(T a, T b) { return a / b; }
  static __device__ __forceinline__ T root(T x) { return sqrt(x); }
};
struct FastF32 {
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
  static __device__ __forceinline__ float root(float x) { return __builtin_amdgcn_sqrtf(x); }
};

template <class T> struct Eps;
template <> struct Eps<float> { static constexpr float deg = 1e-5f; };
template <> struct Eps<double> { static constexpr double deg = 1e-12; };

// Fast magnetosonic speed from a^2 = gamma p / rho, b^2 = |B|^2 / rho and the
// transverse part bt^2: cf^2 = (a^2 + b^2 + sqrt((a^2 - b^2)^2 + 4 a^2 bt^2)) / 2.
template <class T, class M = Exact<T>>
__device__ __forceinline__ T fast_speed(T a2, T b2, T bt2) {
  T d = a2 - b2;
  return M::root(T(0.5) * (a2 + b2 + M::root(d * d + T(4) * a2 * bt2)));
}

// HLLD interface flux.  Rotated states (rho, un, ut1, ut2, p, bt1, bt2) on the
// left (l) and right (r), common normal field bn.  f receives
// (mass, mn, mt1, mt2, energy, bt1, bt2) and, in f[7], the upwind speed that
// orients the edge EMFs: S_L if S_L > 0, S_R if S_R < 0, else the contact
// speed S_M (the mass flux's sign in exact arithmetic, and exactly zero where
// both normal velocities vanish and the total pressures agree), taken as zero
// when |S_M| <= eps max(-S_L, S_R) with eps the degeneracy threshold of the
// precision: a contact speed at the rounding level of the signal speeds (a
// symmetry plane of the flow) has no direction, and the edge EMFs average
// the two sides there.  Regions are
// chosen outermost first:
// F_L if S_L > 0, F*_L if S*_L >= 0, F**_L if S_M >= 0, F**_R if S*_R >= 0,
// F*_R if S_R >= 0, else F_R.  Degenerate star states (vanishing
// rho (S - u)(S - S_M) - bn^2) keep the transverse velocity and field.
template <class T, class M = Exact<T>>
__device__ __forceinline__ void hlld_flux(const T* l, const T* r, T bn, T gamma, T* f) {
  const T gm1 = gamma - T(1);
  const T bn2 = bn * bn;
  // left
  const T rl = l[0], ul = l[1], vl1 = l[2], vl2 = l[3], pl = l[4], bl1 = l[5], bl2 = l[6];
  const T bbl = bn2 + bl1 * bl1 + bl2 * bl2;
  const T El = M::div(pl, gm1) + T(0.5) * rl * (ul * ul + vl1 * vl1 + vl2 * vl2) + T(0.5) * bbl;
  const T ptl = pl + T(0.5) * bbl;
  const T cfl = fast_speed<T, M>(M::div(gamma * pl, rl), M::div(bbl, rl), M::div(bl1 * bl1 + bl2 * bl2, rl));
  // right
  const T rr = r[0], ur = r[1], vr1 = r[2], vr2 = r[3], pr = r[4], br1 = r[5], br2 = r[6];
  const T bbr = bn2 + br1 * br1 + br2 * br2;
  const T Er = M::div(pr, gm1) + T(0.5) * rr * (ur * ur + vr1 * vr1 + vr2 * vr2) + T(0.5) * bbr;
  const T ptr = pr + T(0.5) * bbr;
  const T cfr = fast_speed<T, M>(M::div(gamma * pr, rr), M::div(bbr, rr), M::div(br1 * br1 + br2 * br2, rr));

  const T cmax = (cfl < cfr) ? cfr : cfl;
  const T SL = ((ur < ul) ? ur : ul) - cmax;
  const T SR = ((ul < ur) ? ur : ul) + cmax;

  // physical fluxes
  auto phys = [&](T rho, T u, T v1, T v2, T pt, T b1, T b2, T E, T* F) {
    T vb = u * bn + v1 * b1 + v2 * b2;
    F[0] = rho * u;
    F[1] = rho * u * u + pt - bn2;
    F[2] = rho * u * v1 - bn * b1;
    F[3] = rho * u * v2 - bn * b2;
    F[4] = (E + pt) * u - bn * vb;
    F[5] = b1 * u - bn * v1;
    F[6] = b2 * u - bn * v2;
  };
  if (SL > T(0)) {
    phys(rl, ul, vl1, vl2, ptl, bl1, bl2, El, f);
    f[7] = SL;
    return;
  }
  if (SR < T(0)) {
    phys(rr, ur, vr1, vr2, ptr, br1, br2, Er, f);
    f[7] = SR;
    return;
  }
  const T dl = (SL - ul) * rl, dr = (SR - ur) * rr;
  const T SM = M::div(dr * ur - dl * ul - ptr + ptl, dr - dl);
  f[7] = (fabs(SM) <= Eps<T>::deg * ((-SL > SR) ? -SL : SR)) ? T(0) : SM;
  const T pts = M::div(dr * ptl - dl * ptr + dr * dl * (ur - ul), dr - dl);

  // single-star state of one side
  struct Star {
    T rho, v1, v2, b1, b2, E, sq;
  };
  auto star = [&](T rho, T u, T v1, T v2, T pt, T b1, T b2, T E, T S, T d) {
    Star s;
    s.rho = M::div(d, S - SM);
    const T den = d * (S - SM) - bn2;
    const T lim = Eps<T>::deg * (d * (S - u) + bn2);
    if (fabs(den) <= lim) {
      s.v1 = v1; s.v2 = v2; s.b1 = b1; s.b2 = b2;
    } else {
      const T cv = M::div(bn * (SM - u), den);
      const T cb = M::div(d * (S - u) - bn2, den);
      s.v1 = v1 - b1 * cv;
      s.v2 = v2 - b2 * cv;
      s.b1 = b1 * cb;
      s.b2 = b2 * cb;
    }
    const T vb = u * bn + v1 * b1 + v2 * b2;
    const T vbs = SM * bn + s.v1 * s.b1 + s.v2 * s.b2;
    s.E = M::div((S - u) * E - pt * u + pts * SM + bn * (vb - vbs), S - SM);
    s.sq = M::root(s.rho);
    return s;
  };
  const Star sl = star(rl, ul, vl1, vl2, ptl, bl1, bl2, El, SL, dl);
  const Star sr = star(rr, ur, vr1, vr2, ptr, br1, br2, Er, SR, dr);
  const T SsL = SM - M::div(fabs(bn), sl.sq);
  const T SsR = SM + M::div(fabs(bn), sr.sq);

  // choose the side, then F = F_a + S_a (U*_a - U_a) [+ S*_a (U**_a - U*_a)]
  const bool left = SM >= T(0);
  const T rho = left ? rl : rr, u = left ? ul : ur, v1 = left ? vl1 : vr1, v2 = left ? vl2 : vr2;
  const T pt = left ? ptl : ptr, b1 = left ? bl1 : br1, b2 = left ? bl2 : br2, E = left ? El : Er;
  const T S = left ? SL : SR;
  const Star& s = left ? sl : sr;
  phys(rho, u, v1, v2, pt, b1, b2, E, f);
  // U* - U
  T du[7];
  du[0] = s.rho - rho;
  du[1] = s.rho * SM - rho * u;
  du[2] = s.rho * s.v1 - rho * v1;
  du[3] = s.rho * s.v2 - rho * v2;
  du[4] = s.E - E;
  du[5] = s.b1 - b1;
  du[6] = s.b2 - b2;
  for (int q = 0; q < 7; ++q) f[q] = f[q] + S * du[q];
  const T Ss = left ? SsL : SsR;
  const bool inner = left ? (SsL < T(0)) : (SsR >= T(0));
  if (!inner) return;  // single-star region
  // double-star region, s = sign(bn) with sign(0) = +1
  const T sg = (bn >= T(0)) ? T(1) : T(-1);
  const T isum = M::rcp(sl.sq + sr.sq);
  const T w1 = (sl.sq * sl.v1 + sr.sq * sr.v1 + sg * (sr.b1 - sl.b1)) * isum;
  const T w2 = (sl.sq * sl.v2 + sr.sq * sr.v2 + sg * (sr.b2 - sl.b2)) * isum;
  const T c1 = (sl.sq * sr.b1 + sr.sq * sl.b1 + sg * sl.sq * sr.sq * (sr.v1 - sl.v1)) * isum;
  const T c2 = (sl.sq * sr.b2 + sr.sq * sl.b2 + sg * sl.sq * sr.sq * (sr.v2 - sl.v2)) * isum;
  const T vbss = SM * bn + w1 * c1 + w2 * c2;
  const T vbs = SM * bn + s.v1 * s.b1 + s.v2 * s.b2;
  const T Ess = left ? (s.E - sg * s.sq * (vbs - vbss)) : (s.E + sg * s.sq * (vbs - vbss));
  f[2] = f[2] + Ss * (s.rho * w1 - s.rho * s.v1);
  f[3] = f[3] + Ss * (s.rho * w2 - s.rho * s.v2);
  f[4] = f[4] + Ss * (Ess - s.E);
  f[5] = f[5] + Ss * (c1 - s.b1);
  f[6] = f[6] + Ss * (c2 - s.b2);
}

// Hancock half-step predictor of one cell: W^{n+1/2} = W - (dt/2dx) sum_d
// A_d(W) sl_d, with A_d the 1-D primitive Jacobian along d (normal field held
// constant), summed in the order x, y, z.  w = (rho, vx, vy, vz, p, Bx, By,
// Bz); sl[d] the limited slopes along d (sl[d][5 + d] = 0).
template <class T, class M = Exact<T>>
__device__ __forceinline__ void hancock(const T* w, const T (*sl)[8], T hdtdx, T gamma, T* H) {
  const T ir = M::rcp(w[0]);
  T sum[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) sum[v] = T(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    const T un = w[1 + d], bn = w[5 + d], b1 = w[5 + t1], b2 = w[5 + t2];
    const T* s = sl[d];
    sum[0] = sum[0] + (un * s[0] + w[0] * s[1 + d]);
    sum[1 + d] = sum[1 + d] + (un * s[1 + d] + (s[4] + b1 * s[5 + t1] + b2 * s[5 + t2]) * ir);
    sum[1 + t1] = sum[1 + t1] + (un * s[1 + t1] - bn * s[5 + t1] * ir);
    sum[1 + t2] = sum[1 + t2] + (un * s[1 + t2] - bn * s[5 + t2] * ir);
    sum[4] = sum[4] + (un * s[4] + gamma * w[4] * s[1 + d]);
    sum[5 + t1] = sum[5 + t1] + (un * s[5 + t1] + b1 * s[1 + d] - bn * s[1 + t1]);
    sum[5 + t2] = sum[5 + t2] + (un * s[5 + t2] + b2 * s[1 + d] - bn * s[1 + t2]);
  }
#pragma unroll
  for (int v = 0; v < 8; ++v) H[v] = w[v] - hdtdx * sum[v];
}

// van Leer limited slope from the two one-sided differences.
template <class T, class M = Exact<T>>
__device__ __forceinline__ T van_leer(T dl, T dr) {
  const T pr = dl * dr;
  return (pr > T(0)) ? M::div(T(2) * pr, dl + dr) : T(0);
}

}  // namespace dsp
