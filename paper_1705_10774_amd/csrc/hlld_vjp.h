// hlld_vjp.h -- reverse mode of the HLLD interface flux (mhd_dev.h,
// hlld_flux with IEEE arithmetic): given the cotangent lam of the seven flux
// components, the cotangents of the fifteen inputs (left and right rotated
// states and the normal field) in one pass.  The branches (wave pattern,
// degenerate star states, the larger fast speed, the outer speed estimates)
// are those of the forward evaluation, so this is the derivative along the
// branches taken, like a forward-mode pass per input; the upwind speed f[7]
// only orients the EMFs and has no cotangent.
#pragma once
#include <hip/hip_runtime.h>

#include "mhd_dev.h"

namespace dsp {

namespace vjp_detail {

// one side of the interface with the intermediates the reverse pass reads
template <class T> struct Side {
  T rho, u, v1, v2, p, b1, b2;
  T bb, E, pt;             // |B|^2 (with bn), total energy, total pressure
  T a2, b2r, bt2, dd, q, c;  // fast speed pieces
  // adjoints of the primitives and of E, pt, c
  T arho, au, av1, av2, ap, ab1, ab2, aE, apt, ac;
};

template <class T> __device__ __forceinline__ void side_fwd(Side<T>& s, const T* w, T bn2, T gamma, T gm1) {
  s.rho = w[0]; s.u = w[1]; s.v1 = w[2]; s.v2 = w[3]; s.p = w[4]; s.b1 = w[5]; s.b2 = w[6];
  s.bb = bn2 + s.b1 * s.b1 + s.b2 * s.b2;
  s.E = s.p / gm1 + T(0.5) * s.rho * (s.u * s.u + s.v1 * s.v1 + s.v2 * s.v2) + T(0.5) * s.bb;
  s.pt = s.p + T(0.5) * s.bb;
  s.a2 = (gamma * s.p) / s.rho;
  s.b2r = s.bb / s.rho;
  s.bt2 = (s.b1 * s.b1 + s.b2 * s.b2) / s.rho;
  s.dd = s.a2 - s.b2r;
  s.q = sqrt(s.dd * s.dd + T(4) * s.a2 * s.bt2);
  s.c = sqrt(T(0.5) * (s.a2 + s.b2r + s.q));
  s.arho = s.au = s.av1 = s.av2 = s.ap = s.ab1 = s.ab2 = s.aE = s.apt = s.ac = T(0);
}

// reverse of E, pt and the fast speed into the primitives (and bn)
template <class T> __device__ __forceinline__ void side_rev(Side<T>& s, T bn, T gamma, T gm1, T& abn) {
  // c = sqrt(C), C = (a2 + b2r + q) / 2, q = sqrt(dd^2 + 4 a2 bt2), dd = a2 - b2r
  const T aC = s.c > T(0) ? s.ac / (T(2) * s.c) : T(0);
  T aa2 = T(0.5) * aC, ab2r = T(0.5) * aC;
  const T aq = T(0.5) * aC;
  const T aQ = s.q > T(0) ? aq / (T(2) * s.q) : T(0);
  const T add = T(2) * s.dd * aQ;
  aa2 = aa2 + T(4) * s.bt2 * aQ + add;
  ab2r = ab2r - add;
  const T abt2 = T(4) * s.a2 * aQ;
  // a2 = gamma p / rho, b2r = bb / rho, bt2 = (b1^2 + b2^2) / rho
  s.ap = s.ap + aa2 * gamma / s.rho;
  s.arho = s.arho - (aa2 * s.a2 + ab2r * s.b2r + abt2 * s.bt2) / s.rho;
  T abb = ab2r / s.rho;
  s.ab1 = s.ab1 + abt2 * T(2) * s.b1 / s.rho;
  s.ab2 = s.ab2 + abt2 * T(2) * s.b2 / s.rho;
  // pt = p + bb / 2
  s.ap = s.ap + s.apt;
  abb = abb + T(0.5) * s.apt;
  // E = p / gm1 + rho |v|^2 / 2 + bb / 2
  s.ap = s.ap + s.aE / gm1;
  s.arho = s.arho + T(0.5) * s.aE * (s.u * s.u + s.v1 * s.v1 + s.v2 * s.v2);
  s.au = s.au + s.aE * s.rho * s.u;
  s.av1 = s.av1 + s.aE * s.rho * s.v1;
  s.av2 = s.av2 + s.aE * s.rho * s.v2;
  abb = abb + T(0.5) * s.aE;
  // bb = bn^2 + b1^2 + b2^2
  abn = abn + T(2) * bn * abb;
  s.ab1 = s.ab1 + T(2) * s.b1 * abb;
  s.ab2 = s.ab2 + T(2) * s.b2 * abb;
}

// reverse of the physical flux of side s with cotangent lam
template <class T> __device__ __forceinline__ void phys_rev(Side<T>& s, T bn, const T* lam, T& abn) {
  const T rho = s.rho, u = s.u, v1 = s.v1, v2 = s.v2, b1 = s.b1, b2 = s.b2;
  const T vb = u * bn + v1 * b1 + v2 * b2;
  s.arho = s.arho + lam[0] * u + lam[1] * u * u + lam[2] * u * v1 + lam[3] * u * v2;
  s.au = s.au + lam[0] * rho + lam[1] * T(2) * rho * u + lam[2] * rho * v1 + lam[3] * rho * v2 +
         lam[4] * (s.E + s.pt) - lam[4] * bn * bn + lam[5] * b1 + lam[6] * b2;
  s.av1 = s.av1 + lam[2] * rho * u - lam[4] * bn * b1 - lam[5] * bn;
  s.av2 = s.av2 + lam[3] * rho * u - lam[4] * bn * b2 - lam[6] * bn;
  s.apt = s.apt + lam[1] + lam[4] * u;
  s.aE = s.aE + lam[4] * u;
  s.ab1 = s.ab1 - lam[2] * bn - lam[4] * bn * v1 + lam[5] * u;
  s.ab2 = s.ab2 - lam[3] * bn - lam[4] * bn * v2 + lam[6] * u;
  abn = abn - lam[1] * T(2) * bn - lam[2] * b1 - lam[3] * b2 - lam[4] * (vb + bn * u) - lam[5] * v1 - lam[6] * v2;
}

// star state of one side and its intermediates
template <class T> struct Star {
  T S, d, SSM, rho, den, cv, cb, v1, v2, b1, b2, vb, vbs, num, E, sq;
  bool degen;
  T aS, ad, arho, av1, av2, ab1, ab2, aE, asq;  // adjoints of S, d and the star values
};

template <class T>
__device__ __forceinline__ void star_fwd(Star<T>& st, const Side<T>& s, T S, T d, T SM, T pts, T bn, T bn2) {
  st.S = S;
  st.d = d;
  st.SSM = S - SM;
  st.rho = d / st.SSM;
  st.den = d * st.SSM - bn2;
  const T lim = Eps<T>::deg * (d * (S - s.u) + bn2);
  st.degen = (st.den < T(0) ? -st.den : st.den) <= lim;
  if (st.degen) {
    st.v1 = s.v1; st.v2 = s.v2; st.b1 = s.b1; st.b2 = s.b2;
    st.cv = st.cb = T(0);
  } else {
    st.cv = (bn * (SM - s.u)) / st.den;
    st.cb = (d * (S - s.u) - bn2) / st.den;
    st.v1 = s.v1 - s.b1 * st.cv;
    st.v2 = s.v2 - s.b2 * st.cv;
    st.b1 = s.b1 * st.cb;
    st.b2 = s.b2 * st.cb;
  }
  st.vb = s.u * bn + s.v1 * s.b1 + s.v2 * s.b2;
  st.vbs = SM * bn + st.v1 * st.b1 + st.v2 * st.b2;
  st.num = (S - s.u) * s.E - s.pt * s.u + pts * SM + bn * (st.vb - st.vbs);
  st.E = st.num / st.SSM;
  st.sq = sqrt(st.rho);
  st.aS = st.ad = st.arho = st.av1 = st.av2 = st.ab1 = st.ab2 = st.aE = st.asq = T(0);
}

template <class T>
__device__ __forceinline__ void star_rev(Star<T>& st, Side<T>& s, T SM, T pts, T bn, T& aSM, T& apts, T& abn) {
  // sq = sqrt(rho*)
  st.arho = st.arho + (st.sq > T(0) ? st.asq / (T(2) * st.sq) : T(0));
  // E* = num / (S - SM)
  const T anum = st.aE / st.SSM;
  T aSSM = -st.aE * st.E / st.SSM;
  // num = (S - u) E - pt u + pts SM + bn (vb - vbs)
  st.aS = st.aS + anum * s.E;
  s.au = s.au - anum * s.E - anum * s.pt;
  s.aE = s.aE + anum * (st.S - s.u);
  s.apt = s.apt - anum * s.u;
  apts = apts + anum * SM;
  aSM = aSM + anum * pts;
  abn = abn + anum * (st.vb - st.vbs);
  const T avb = anum * bn, avbs = -anum * bn;
  // vbs = SM bn + v1* b1* + v2* b2*
  aSM = aSM + avbs * bn;
  abn = abn + avbs * SM;
  st.av1 = st.av1 + avbs * st.b1;
  st.ab1 = st.ab1 + avbs * st.v1;
  st.av2 = st.av2 + avbs * st.b2;
  st.ab2 = st.ab2 + avbs * st.v2;
  // vb = u bn + v1 b1 + v2 b2
  s.au = s.au + avb * bn;
  abn = abn + avb * s.u;
  s.av1 = s.av1 + avb * s.b1;
  s.ab1 = s.ab1 + avb * s.v1;
  s.av2 = s.av2 + avb * s.b2;
  s.ab2 = s.ab2 + avb * s.v2;
  if (st.degen) {
    s.av1 = s.av1 + st.av1;
    s.av2 = s.av2 + st.av2;
    s.ab1 = s.ab1 + st.ab1;
    s.ab2 = s.ab2 + st.ab2;
  } else {
    // v* = v - b cv, b* = b cb
    s.av1 = s.av1 + st.av1;
    s.av2 = s.av2 + st.av2;
    s.ab1 = s.ab1 - st.av1 * st.cv + st.ab1 * st.cb;
    s.ab2 = s.ab2 - st.av2 * st.cv + st.ab2 * st.cb;
    const T acv = -st.av1 * s.b1 - st.av2 * s.b2;
    const T acb = st.ab1 * s.b1 + st.ab2 * s.b2;
    // cv = bn (SM - u) / den, cb = (d (S - u) - bn^2) / den
    abn = abn + acv * (SM - s.u) / st.den - acb * T(2) * bn / st.den;
    aSM = aSM + acv * bn / st.den;
    s.au = s.au - acv * bn / st.den - acb * st.d / st.den;
    st.ad = st.ad + acb * (st.S - s.u) / st.den;
    st.aS = st.aS + acb * st.d / st.den;
    const T aden = -acv * st.cv / st.den - acb * st.cb / st.den;
    // den = d (S - SM) - bn^2
    st.ad = st.ad + aden * st.SSM;
    aSSM = aSSM + aden * st.d;
    abn = abn - aden * T(2) * bn;
  }
  // rho* = d / (S - SM)
  st.ad = st.ad + st.arho / st.SSM;
  aSSM = aSSM - st.arho * st.rho / st.SSM;
  // S - SM
  st.aS = st.aS + aSSM;
  aSM = aSM - aSSM;
}

}  // namespace vjp_detail

// gl, gr: cotangents of l and r (order rho, un, ut1, ut2, p, bt1, bt2); gbn:
// of bn.  Outputs are overwritten.
template <class T>
__device__ void hlld_vjp(const T* l, const T* r, T bn, T gamma, const T* lam, T* gl, T* gr, T& gbn) {
  using namespace vjp_detail;
  const T gm1 = gamma - T(1);
  const T bn2 = bn * bn;
  Side<T> L, R;
  side_fwd(L, l, bn2, gamma, gm1);
  side_fwd(R, r, bn2, gamma, gm1);
  const bool rfast = L.c < R.c;  // cmax = rfast ? cR : cL
  const T cmax = rfast ? R.c : L.c;
  const bool slr = R.u < L.u;  // SL from the smaller normal velocity
  const bool srr = L.u < R.u;  // SR from the larger
  const T SL = (slr ? R.u : L.u) - cmax;
  const T SR = (srr ? R.u : L.u) + cmax;
  T abn = T(0), aSL = T(0), aSR = T(0);
  if (SL > T(0) || SR < T(0)) {
    Side<T>& s = SL > T(0) ? L : R;
    phys_rev(s, bn, lam, abn);
  } else {
    const T dl = (SL - L.u) * L.rho, dr = (SR - R.u) * R.rho;
    const T dm = dr - dl;
    const T nSM = dr * R.u - dl * L.u - R.pt + L.pt;
    const T SM = nSM / dm;
    const T nps = dr * L.pt - dl * R.pt + dr * dl * (R.u - L.u);
    const T pts = nps / dm;
    Star<T> sl, sr;
    star_fwd(sl, L, SL, dl, SM, pts, bn, bn2);
    star_fwd(sr, R, SR, dr, SM, pts, bn, bn2);
    const T abs_bn = bn < T(0) ? -bn : bn, sgn_abs = bn < T(0) ? T(-1) : T(1);
    const T SsL = SM - abs_bn / sl.sq;
    const T SsR = SM + abs_bn / sr.sq;
    const bool left = SM >= T(0);
    Side<T>& a = left ? L : R;
    Star<T>& s = left ? sl : sr;
    const T S = left ? SL : SR;
    const T Ss = left ? SsL : SsR;
    const bool inner = left ? (SsL < T(0)) : (SsR >= T(0));
    T aSM = T(0), apts = T(0), aS = T(0), aSs = T(0);
    if (inner) {
      const T sg = (bn >= T(0)) ? T(1) : T(-1);
      const T sum = sl.sq + sr.sq;
      const T isum = T(1) / sum;
      const T M1 = sl.sq * sl.v1 + sr.sq * sr.v1 + sg * (sr.b1 - sl.b1);
      const T M2 = sl.sq * sl.v2 + sr.sq * sr.v2 + sg * (sr.b2 - sl.b2);
      const T N1 = sl.sq * sr.b1 + sr.sq * sl.b1 + sg * sl.sq * sr.sq * (sr.v1 - sl.v1);
      const T N2 = sl.sq * sr.b2 + sr.sq * sl.b2 + sg * sl.sq * sr.sq * (sr.v2 - sl.v2);
      const T w1 = M1 * isum, w2 = M2 * isum, c1 = N1 * isum, c2 = N2 * isum;
      const T vbss = SM * bn + w1 * c1 + w2 * c2;
      const T vbsa = SM * bn + s.v1 * s.b1 + s.v2 * s.b2;
      const T sig = left ? T(-1) : T(1);
      const T Ess = s.E + sig * sg * s.sq * (vbsa - vbss);
      // f2..f6 += Ss (...)
      aSs = lam[2] * (s.rho * w1 - s.rho * s.v1) + lam[3] * (s.rho * w2 - s.rho * s.v2) + lam[4] * (Ess - s.E) +
            lam[5] * (c1 - s.b1) + lam[6] * (c2 - s.b2);
      s.arho = s.arho + Ss * (lam[2] * (w1 - s.v1) + lam[3] * (w2 - s.v2));
      T aw1 = Ss * lam[2] * s.rho, aw2 = Ss * lam[3] * s.rho;
      s.av1 = s.av1 - Ss * lam[2] * s.rho;
      s.av2 = s.av2 - Ss * lam[3] * s.rho;
      const T aEss = Ss * lam[4];
      s.aE = s.aE - Ss * lam[4];
      T ac1 = Ss * lam[5], ac2 = Ss * lam[6];
      s.ab1 = s.ab1 - Ss * lam[5];
      s.ab2 = s.ab2 - Ss * lam[6];
      // Ess = E* + sig sg sq* (vbsa - vbss)
      s.aE = s.aE + aEss;
      s.asq = s.asq + aEss * sig * sg * (vbsa - vbss);
      const T avbsa = aEss * sig * sg * s.sq, avbss = -aEss * sig * sg * s.sq;
      aSM = aSM + avbsa * bn + avbss * bn;
      abn = abn + avbsa * SM + avbss * SM;
      s.av1 = s.av1 + avbsa * s.b1;
      s.ab1 = s.ab1 + avbsa * s.v1;
      s.av2 = s.av2 + avbsa * s.b2;
      s.ab2 = s.ab2 + avbsa * s.v2;
      aw1 = aw1 + avbss * c1;
      ac1 = ac1 + avbss * w1;
      aw2 = aw2 + avbss * c2;
      ac2 = ac2 + avbss * w2;
      // w = M isum, c = N isum
      const T aM1 = aw1 * isum, aM2 = aw2 * isum, aN1 = ac1 * isum, aN2 = ac2 * isum;
      const T aisum = aw1 * M1 + aw2 * M2 + ac1 * N1 + ac2 * N2;
      // M = sqL vL + sqR vR + sg (bR - bL)
      sl.asq = sl.asq + aM1 * sl.v1 + aM2 * sl.v2;
      sr.asq = sr.asq + aM1 * sr.v1 + aM2 * sr.v2;
      sl.av1 = sl.av1 + aM1 * sl.sq;
      sr.av1 = sr.av1 + aM1 * sr.sq;
      sl.av2 = sl.av2 + aM2 * sl.sq;
      sr.av2 = sr.av2 + aM2 * sr.sq;
      sr.ab1 = sr.ab1 + aM1 * sg;
      sl.ab1 = sl.ab1 - aM1 * sg;
      sr.ab2 = sr.ab2 + aM2 * sg;
      sl.ab2 = sl.ab2 - aM2 * sg;
      // N = sqL bR + sqR bL + sg sqL sqR (vR - vL)
      sl.asq = sl.asq + aN1 * (sr.b1 + sg * sr.sq * (sr.v1 - sl.v1)) + aN2 * (sr.b2 + sg * sr.sq * (sr.v2 - sl.v2));
      sr.asq = sr.asq + aN1 * (sl.b1 + sg * sl.sq * (sr.v1 - sl.v1)) + aN2 * (sl.b2 + sg * sl.sq * (sr.v2 - sl.v2));
      sr.ab1 = sr.ab1 + aN1 * sl.sq;
      sl.ab1 = sl.ab1 + aN1 * sr.sq;
      sr.ab2 = sr.ab2 + aN2 * sl.sq;
      sl.ab2 = sl.ab2 + aN2 * sr.sq;
      sr.av1 = sr.av1 + aN1 * sg * sl.sq * sr.sq;
      sl.av1 = sl.av1 - aN1 * sg * sl.sq * sr.sq;
      sr.av2 = sr.av2 + aN2 * sg * sl.sq * sr.sq;
      sl.av2 = sl.av2 - aN2 * sg * sl.sq * sr.sq;
      // isum = 1 / (sqL + sqR)
      const T asum = -aisum * isum * isum;
      sl.asq = sl.asq + asum;
      sr.asq = sr.asq + asum;
    }
    // single-star part: f = F(a) + S (U* - U)
    phys_rev(a, bn, lam, abn);
    const T du[7] = {s.rho - a.rho,          s.rho * SM - a.rho * a.u, s.rho * s.v1 - a.rho * a.v1,
                     s.rho * s.v2 - a.rho * a.v2, s.E - a.E,              s.b1 - a.b1,
                     s.b2 - a.b2};
    for (int q = 0; q < 7; ++q) aS = aS + lam[q] * du[q];
    s.arho = s.arho + S * (lam[0] + lam[1] * SM + lam[2] * s.v1 + lam[3] * s.v2);
    aSM = aSM + S * lam[1] * s.rho;
    s.av1 = s.av1 + S * lam[2] * s.rho;
    s.av2 = s.av2 + S * lam[3] * s.rho;
    s.aE = s.aE + S * lam[4];
    s.ab1 = s.ab1 + S * lam[5];
    s.ab2 = s.ab2 + S * lam[6];
    a.arho = a.arho - S * (lam[0] + lam[1] * a.u + lam[2] * a.v1 + lam[3] * a.v2);
    a.au = a.au - S * lam[1] * a.rho;
    a.av1 = a.av1 - S * lam[2] * a.rho;
    a.av2 = a.av2 - S * lam[3] * a.rho;
    a.aE = a.aE - S * lam[4];
    a.ab1 = a.ab1 - S * lam[5];
    a.ab2 = a.ab2 - S * lam[6];
    if (left) aSL = aSL + aS; else aSR = aSR + aS;
    // Ss: SsL = SM - |bn| / sqL, SsR = SM + |bn| / sqR
    if (left) {
      aSM = aSM + aSs;
      sl.asq = sl.asq + aSs * abs_bn / (sl.sq * sl.sq);
      abn = abn - aSs * sgn_abs / sl.sq;
    } else {
      aSM = aSM + aSs;
      sr.asq = sr.asq - aSs * abs_bn / (sr.sq * sr.sq);
      abn = abn + aSs * sgn_abs / sr.sq;
    }
    // the two star states
    star_rev(sl, L, SM, pts, bn, aSM, apts, abn);
    star_rev(sr, R, SM, pts, bn, aSM, apts, abn);
    aSL = aSL + sl.aS;
    aSR = aSR + sr.aS;
    T adl = sl.ad, adr = sr.ad;
    // pts = nps / dm, nps = dr ptL - dl ptR + dr dl (uR - uL)
    const T anps = apts / dm;
    T adm = -apts * pts / dm;
    adr = adr + anps * (L.pt + dl * (R.u - L.u));
    adl = adl + anps * (-R.pt + dr * (R.u - L.u));
    L.apt = L.apt + anps * dr;
    R.apt = R.apt - anps * dl;
    R.au = R.au + anps * dr * dl;
    L.au = L.au - anps * dr * dl;
    // SM = nSM / dm, nSM = dr uR - dl uL - ptR + ptL
    const T anSM = aSM / dm;
    adm = adm - aSM * SM / dm;
    adr = adr + anSM * R.u;
    R.au = R.au + anSM * dr;
    adl = adl - anSM * L.u;
    L.au = L.au - anSM * dl;
    R.apt = R.apt - anSM;
    L.apt = L.apt + anSM;
    // dm = dr - dl
    adr = adr + adm;
    adl = adl - adm;
    // dl = (SL - uL) rhoL, dr = (SR - uR) rhoR
    aSL = aSL + adl * L.rho;
    L.au = L.au - adl * L.rho;
    L.arho = L.arho + adl * (SL - L.u);
    aSR = aSR + adr * R.rho;
    R.au = R.au - adr * R.rho;
    R.arho = R.arho + adr * (SR - R.u);
  }
  // SL = min-side u - cmax, SR = max-side u + cmax
  if (slr) R.au = R.au + aSL; else L.au = L.au + aSL;
  if (srr) R.au = R.au + aSR; else L.au = L.au + aSR;
  const T acmax = aSR - aSL;
  if (rfast) R.ac = R.ac + acmax; else L.ac = L.ac + acmax;
  side_rev(L, bn, gamma, gm1, abn);
  side_rev(R, bn, gamma, gm1, abn);
  gl[0] = L.arho; gl[1] = L.au; gl[2] = L.av1; gl[3] = L.av2; gl[4] = L.ap; gl[5] = L.ab1; gl[6] = L.ab2;
  gr[0] = R.arho; gr[1] = R.au; gr[2] = R.av1; gr[3] = R.av2; gr[4] = R.ap; gr[5] = R.ab1; gr[6] = R.ab2;
  gbn = abn;
}

}  // namespace dsp
