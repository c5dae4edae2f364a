// orc_mhd.hpp -- the single-patch step of the CPU oracle (test infrastructure).
//
// Ideal MHD in units with mu0 = 1 (magnetic pressure |B|^2/2), gamma-law gas.
// The paper fixes the framework (tasks, patches, time slices, readiness) but
// leaves the solver to the code plugged into it (Sec. 4.1, "Internal and
// external HD, MHD and PIC solvers"; constrained transport, Sec. 4.3).  The
// solver here is second-order MUSCL-Hancock on primitive variables with van
// Leer slopes, the HLLD approximate Riemann solver of Miyoshi & Kusano
// (2005), and constrained transport of face-centred B (Evans & Hawley 1988,
// cited in Sec. 4.3) with the upwinded edge EMFs of Gardiner & Stone (2005).
// Everything is written out literally, one quantity at a time, so it can be
// checked against those methods by eye.  No blocking, fusion or reordering.
#pragma once
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace orc {

// ---------------------------------------------------------------------------
// Scalars: double, and a forward-mode dual number (value, tangent) that turns
// the same code into an exact Jacobian-vector product along the taken branches.
struct Dual {
  double v, d;
  Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
// At a zero argument the square root has a kink (e.g. sqrt of the square of a
// difference that vanishes); its tangent is taken as 0 there, the symmetric
// (central-difference) derivative.
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  if (s == 0.0) return Dual(0.0, 0.0);
  return Dual(s, a.d / (2.0 * s));
}
inline Dual fabs(Dual a) { return a.v < 0.0 ? -a : a; }
// Counting scalar: a double plus a tally of the floating-point operations
// applied to it (each +, -, *, / and square root counts one; comparisons,
// signs and absolute values count none).  Used to state the arithmetic work
// of the method per cell update.
struct Flop {
  double v;
  Flop(double a = 0.0) : v(a) {}
};
// Two tallies: [0] everything else, [1] the Courant rate (while a
// FlopCourant object is alive).
inline std::atomic<unsigned long long>* flop_tally() {
  static std::atomic<unsigned long long> t[2] = {{0}, {0}};
  return t;
}
inline std::atomic<int>& flop_bucket() {
  static std::atomic<int> b{0};
  return b;
}
struct FlopCourant {
  FlopCourant() { flop_bucket().store(1); }
  ~FlopCourant() { flop_bucket().store(0); }
};
inline Flop flop1(double r) {
  flop_tally()[flop_bucket().load(std::memory_order_relaxed)].fetch_add(1, std::memory_order_relaxed);
  return Flop(r);
}
inline Flop operator+(Flop a, Flop b) { return flop1(a.v + b.v); }
inline Flop operator-(Flop a, Flop b) { return flop1(a.v - b.v); }
inline Flop operator-(Flop a) { return Flop(-a.v); }
inline Flop operator*(Flop a, Flop b) { return flop1(a.v * b.v); }
inline Flop operator/(Flop a, Flop b) { return flop1(a.v / b.v); }
inline Flop& operator+=(Flop& a, Flop b) { a = a + b; return a; }
inline bool operator<(Flop a, Flop b) { return a.v < b.v; }
inline bool operator>(Flop a, Flop b) { return a.v > b.v; }
inline bool operator<=(Flop a, Flop b) { return a.v <= b.v; }
inline bool operator>=(Flop a, Flop b) { return a.v >= b.v; }
inline Flop sqrt(Flop a) { return flop1(std::sqrt(a.v)); }
inline Flop fabs(Flop a) { return Flop(std::fabs(a.v)); }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double val(const Flop& x) { return x.v; }
using std::fabs;
using std::sqrt;

template <class R> inline R rmin(R a, R b) { return (b < a) ? b : a; }
template <class R> inline R rmax(R a, R b) { return (a < b) ? b : a; }

// ---------------------------------------------------------------------------
// Storage of one patch: 5 cell-centred conserved arrays (rho, mx, my, mz, E),
// then face-centred Bx, By, Bz, each C-ordered (z, y, x) with x fastest.
// With ng = 0 this is the stored slice (interior only, both boundary faces);
// with ng > 0 it is the padded work array that carries guard zones.
struct Layout {
  int n, ng, N;
  size_t nc, nf;
  Layout(int n_, int ng_) : n(n_), ng(ng_), N(n_ + 2 * ng_) {
    nc = (size_t)N * N * N;
    nf = (size_t)N * N * (N + 1);
  }
  size_t size() const { return 5 * nc + 3 * nf; }
  // local cell index i, j, k in [-ng, n + ng)
  size_t cell(int v, int i, int j, int k) const {
    return v * nc + ((size_t)(k + ng) * N + (j + ng)) * N + (i + ng);
  }
  // face component d; the d-th index is a face index in [-ng, n + ng]
  size_t face(int d, int i, int j, int k) const {
    size_t sx = N + (d == 0), sy = N + (d == 1);
    return 5 * nc + d * nf + ((size_t)(k + ng) * sy + (j + ng)) * sx + (i + ng);
  }
};

// A 3-D array over an inclusive index box.
template <class T> struct Box3 {
  int lo[3] = {0, 0, 0}, nx = 0, ny = 0, nz = 0;
  std::vector<T> a;
  void init(int l0, int h0, int l1, int h1, int l2, int h2) {
    lo[0] = l0; lo[1] = l1; lo[2] = l2;
    nx = h0 - l0 + 1; ny = h1 - l1 + 1; nz = h2 - l2 + 1;
    a.assign((size_t)nx * ny * nz, T());
  }
  T& operator()(int i, int j, int k) {
    return a[((size_t)(k - lo[2]) * ny + (j - lo[1])) * nx + (i - lo[0])];
  }
  const T& operator()(int i, int j, int k) const {
    return a[((size_t)(k - lo[2]) * ny + (j - lo[1])) * nx + (i - lo[0])];
  }
  T& at(const int c[3]) { return (*this)(c[0], c[1], c[2]); }
  const T& at(const int c[3]) const { return (*this)(c[0], c[1], c[2]); }
};

// Primitive state: density, velocity, gas pressure, cell-centred field.
template <class R> struct Prim {
  R r, v[3], p, b[3];
};
// Unrotated interface flux: mass, momentum, energy, and induction flux of
// each field component (the normal component's own flux is zero); u is the
// upwind speed that orients the edge EMFs (see hlld).
template <class R> struct Flux {
  R r, m[3], e, b[3];
  R u;
};

struct StepCounters {
  int64_t floor_hits = 0;      // cells whose pressure was raised to p_floor
  int64_t fallback_faces = 0;  // faces that fell back to first-order states
};

struct Phys {
  double gamma;
  double eps_deg;  // HLLD degeneracy threshold
  double p_floor;  // 0 = no floor (negative pressure is an error)
  // non-ideal terms (Sec. 4.3): Ohmic resistivity, ambipolar drift
  // coefficient and ion density; eta = gamma_ad = 0 is ideal MHD
  double eta = 0.0, gamma_ad = 0.0, rho_i = 1.0;
  double courant = 0.4;  // MHD Courant number (converts the non-ideal limits to rates)
  bool nonideal() const { return eta > 0.0 || gamma_ad > 0.0; }
};

// Courant-like factor of the Ohmic and ambipolar step limits, C_Ohm = C_AD
// (Eqs. dtOhm and dtAD).
constexpr double kCourantNonideal = 0.1;

// Return codes shared with orc.h.
enum { S_OK = 0, S_ENONFINITE = -6, S_ENEGATIVE = -7 };

// ---------------------------------------------------------------------------
// Primitive variables from conserved cell data and face-centred B.
// The cell-centred field is the mean of the two faces of the cell.
template <class R>
int prims(const Layout& L, const std::vector<R>& P, const Phys& ph, Box3<Prim<R>>& W,
          StepCounters& cnt) {
  const int n = L.n;
  W.init(-2, n + 1, -2, n + 1, -2, n + 1);
  for (int k = -2; k <= n + 1; ++k)
    for (int j = -2; j <= n + 1; ++j)
      for (int i = -2; i <= n + 1; ++i) {
        Prim<R> w;
        R rho = P[L.cell(0, i, j, k)];
        R mx = P[L.cell(1, i, j, k)], my = P[L.cell(2, i, j, k)], mz = P[L.cell(3, i, j, k)];
        R en = P[L.cell(4, i, j, k)];
        w.b[0] = 0.5 * (P[L.face(0, i, j, k)] + P[L.face(0, i + 1, j, k)]);
        w.b[1] = 0.5 * (P[L.face(1, i, j, k)] + P[L.face(1, i, j + 1, k)]);
        w.b[2] = 0.5 * (P[L.face(2, i, j, k)] + P[L.face(2, i, j, k + 1)]);
        w.r = rho;
        w.v[0] = mx / rho;
        w.v[1] = my / rho;
        w.v[2] = mz / rho;
        R ke = 0.5 * (mx * mx + my * my + mz * mz) / rho;
        R me = 0.5 * (w.b[0] * w.b[0] + w.b[1] * w.b[1] + w.b[2] * w.b[2]);
        w.p = (ph.gamma - 1.0) * (en - ke - me);
        if (!std::isfinite(val(rho)) || !std::isfinite(val(w.p))) return S_ENONFINITE;
        if (!(val(rho) > 0.0)) return S_ENEGATIVE;
        if (ph.p_floor > 0.0) {
          if (val(w.p) < ph.p_floor) {
            w.p = R(ph.p_floor);
            cnt.floor_hits++;
          }
        } else if (!(val(w.p) > 0.0)) {
          return S_ENEGATIVE;
        }
        W(i, j, k) = w;
      }
  return S_OK;
}

// Fast magnetosonic speed along direction d for one primitive state:
// cf^2 = (a^2 + b^2 + sqrt((a^2 - b^2)^2 + 4 a^2 bt^2)) / 2 with a^2 = gamma p / rho,
// b^2 = |B|^2 / rho and bt^2 the transverse part; this form has no cancellation.
template <class R> R fast_speed(const Prim<R>& w, int d, double gamma) {
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  R a2 = gamma * w.p / w.r;
  R b2 = (w.b[0] * w.b[0] + w.b[1] * w.b[1] + w.b[2] * w.b[2]) / w.r;
  R bt2 = (w.b[t1] * w.b[t1] + w.b[t2] * w.b[t2]) / w.r;
  R dd = a2 - b2;
  return sqrt(0.5 * (a2 + b2 + sqrt(dd * dd + 4.0 * a2 * bt2)));
}

// Courant rate of a patch: the largest sum over directions of
// (|v_d| + c_f,d) / dx over the interior and the two guard layers the
// stencil reads.  The largest stable step is courant / smax.
// With non-ideal terms the step must also satisfy dt <= C_Ohm dx^2 / eta
// (Eq. dtOhm) and dt <= C_AD gamma_AD rho_i rho dx^2 / B^2 (Eq. dtAD); each
// limit enters as the rate that gives that step with the MHD Courant number,
// (C / C_ni) eta / dx^2 and (C / C_ni) B^2 / (gamma_AD rho_i rho dx^2).
template <class R> double courant_rate(const Box3<Prim<R>>& W, int n, double dx, const Phys& ph) {
  FlopCourant tally_as_courant;
  const double gamma = ph.gamma;
  const double f = ph.courant / kCourantNonideal / (dx * dx);
  double smax = 0.0;
  for (int k = -2; k <= n + 1; ++k)
    for (int j = -2; j <= n + 1; ++j)
      for (int i = -2; i <= n + 1; ++i) {
        const Prim<R>& w = W(i, j, k);
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s = s + (std::fabs(val(w.v[d])) + val(fast_speed(w, d, gamma)));
        s = s / dx;
        if (ph.eta > 0.0) {
          const double so = ph.eta * f;
          if (so > s) s = so;
        }
        if (ph.gamma_ad > 0.0) {
          const double bb = val(w.b[0] * w.b[0] + w.b[1] * w.b[1] + w.b[2] * w.b[2]);
          const double sa = bb / (ph.gamma_ad * ph.rho_i * val(w.r)) * f;
          if (sa > s) s = sa;
        }
        if (!(s <= smax)) smax = s;  // also propagates NaN
      }
  return smax;
}

// ---------------------------------------------------------------------------
// HLLD flux (Miyoshi & Kusano 2005) for one interface in the rotated frame.
// State vectors are (rho, un, ut1, ut2, p, bt1, bt2); bn is the common
// normal field.  Output flux is (mass, mn, mt1, mt2, energy, bt1, bt2),
// followed by F[7], the upwind speed: S_L if S_L > 0, S_R if S_R < 0, else
// the contact speed S_M.  Its sign is the sign of the mass flux in exact
// arithmetic (S_L < S_M < S_R, rho* > 0), and it is exactly zero when both
// normal velocities vanish and the total pressures agree, where the computed
// mass flux is zero only up to rounding.  A contact speed within the
// degeneracy threshold of the outer speeds, |S_M| <= eps_deg max(-S_L, S_R),
// is taken as zero: at that size its sign is rounding noise (on a symmetry
// plane of the flow, say), and the edge EMFs average the two sides there
// instead of following it.
template <class R>
void hlld(const R* wl, const R* wr, R bn, const Phys& ph, R* F) {
  const double g = ph.gamma;
  struct Side {
    R rho, un, v1, v2, p, b1, b2, E, pt, cf;
  };
  auto mk = [&](const R* w) {
    Side s;
    s.rho = w[0]; s.un = w[1]; s.v1 = w[2]; s.v2 = w[3]; s.p = w[4]; s.b1 = w[5]; s.b2 = w[6];
    R bb = bn * bn + s.b1 * s.b1 + s.b2 * s.b2;
    R vv = s.un * s.un + s.v1 * s.v1 + s.v2 * s.v2;
    s.E = s.p / (g - 1.0) + 0.5 * s.rho * vv + 0.5 * bb;
    s.pt = s.p + 0.5 * bb;
    R a2 = g * s.p / s.rho;
    R b2 = bb / s.rho;
    R bt2 = (s.b1 * s.b1 + s.b2 * s.b2) / s.rho;
    R dd = a2 - b2;
    s.cf = sqrt(0.5 * (a2 + b2 + sqrt(dd * dd + 4.0 * a2 * bt2)));
    return s;
  };
  Side L = mk(wl), Rt = mk(wr);

  // physical flux of one side
  auto pflux = [&](const Side& s, R* f) {
    R vb = s.un * bn + s.v1 * s.b1 + s.v2 * s.b2;
    f[0] = s.rho * s.un;
    f[1] = s.rho * s.un * s.un + s.pt - bn * bn;
    f[2] = s.rho * s.un * s.v1 - bn * s.b1;
    f[3] = s.rho * s.un * s.v2 - bn * s.b2;
    f[4] = (s.E + s.pt) * s.un - bn * vb;
    f[5] = s.b1 * s.un - bn * s.v1;
    f[6] = s.b2 * s.un - bn * s.v2;
  };
  auto cons = [&](const Side& s, R* u) {
    u[0] = s.rho; u[1] = s.rho * s.un; u[2] = s.rho * s.v1; u[3] = s.rho * s.v2;
    u[4] = s.E; u[5] = s.b1; u[6] = s.b2;
  };

  // outer wave speeds
  R cmax = rmax(L.cf, Rt.cf);
  R SL = rmin(L.un, Rt.un) - cmax;
  R SR = rmax(L.un, Rt.un) + cmax;
  // entropy (contact) speed and star total pressure
  R dL = (SL - L.un) * L.rho;
  R dR = (SR - Rt.un) * Rt.rho;
  R SM = (dR * Rt.un - dL * L.un - Rt.pt + L.pt) / (dR - dL);
  R pts = (dR * L.pt - dL * Rt.pt + dR * dL * (Rt.un - L.un)) / (dR - dL);

  // single-star states
  struct Star {
    R rho, v1, v2, b1, b2, E, sq;
  };
  auto star = [&](const Side& s, R S, R d) {
    Star st;
    st.rho = d / (S - SM);
    R den = d * (S - SM) - bn * bn;
    R lim = ph.eps_deg * (d * (S - s.un) + bn * bn);
    if (fabs(den) <= lim) {
      st.v1 = s.v1; st.v2 = s.v2; st.b1 = s.b1; st.b2 = s.b2;
    } else {
      st.v1 = s.v1 - bn * s.b1 * (SM - s.un) / den;
      st.v2 = s.v2 - bn * s.b2 * (SM - s.un) / den;
      st.b1 = s.b1 * (d * (S - s.un) - bn * bn) / den;
      st.b2 = s.b2 * (d * (S - s.un) - bn * bn) / den;
    }
    R vb = s.un * bn + s.v1 * s.b1 + s.v2 * s.b2;
    R vbs = SM * bn + st.v1 * st.b1 + st.v2 * st.b2;
    st.E = ((S - s.un) * s.E - s.pt * s.un + pts * SM + bn * (vb - vbs)) / (S - SM);
    st.sq = sqrt(st.rho);
    return st;
  };
  Star sL = star(L, SL, dL), sR = star(Rt, SR, dR);
  R SsL = SM - fabs(bn) / sL.sq;
  R SsR = SM + fabs(bn) / sR.sq;

  auto ucons_star = [&](const Star& st, R* u) {
    u[0] = st.rho; u[1] = st.rho * SM; u[2] = st.rho * st.v1; u[3] = st.rho * st.v2;
    u[4] = st.E; u[5] = st.b1; u[6] = st.b2;
  };

  R FL[7], FR[7], UL[7], UR[7], UsL[7], UsR[7];
  pflux(L, FL); pflux(Rt, FR);
  cons(L, UL); cons(Rt, UR);
  ucons_star(sL, UsL); ucons_star(sR, UsR);

  // double-star states (between the rotational discontinuities), s = sign(bn)
  R s = (bn >= 0.0) ? R(1.0) : R(-1.0);
  R sum = sL.sq + sR.sq;
  R v1 = (sL.sq * sL.v1 + sR.sq * sR.v1 + s * (sR.b1 - sL.b1)) / sum;
  R v2 = (sL.sq * sL.v2 + sR.sq * sR.v2 + s * (sR.b2 - sL.b2)) / sum;
  R b1 = (sL.sq * sR.b1 + sR.sq * sL.b1 + s * sL.sq * sR.sq * (sR.v1 - sL.v1)) / sum;
  R b2 = (sL.sq * sR.b2 + sR.sq * sL.b2 + s * sL.sq * sR.sq * (sR.v2 - sL.v2)) / sum;
  R vbss = SM * bn + v1 * b1 + v2 * b2;
  R vbsL = SM * bn + sL.v1 * sL.b1 + sL.v2 * sL.b2;
  R vbsR = SM * bn + sR.v1 * sR.b1 + sR.v2 * sR.b2;
  R EssL = sL.E - s * sL.sq * (vbsL - vbss);
  R EssR = sR.E + s * sR.sq * (vbsR - vbss);
  R UssL[7] = {sL.rho, sL.rho * SM, sL.rho * v1, sL.rho * v2, EssL, b1, b2};
  R UssR[7] = {sR.rho, sR.rho * SM, sR.rho * v1, sR.rho * v2, EssR, b1, b2};

  // flux of the region that contains the interface, outermost first
  if (SL > 0.0) {
    for (int q = 0; q < 7; ++q) F[q] = FL[q];
  } else if (SsL >= 0.0) {
    for (int q = 0; q < 7; ++q) F[q] = FL[q] + SL * (UsL[q] - UL[q]);
  } else if (SM >= 0.0) {
    for (int q = 0; q < 7; ++q) F[q] = FL[q] + SL * (UsL[q] - UL[q]) + SsL * (UssL[q] - UsL[q]);
  } else if (SsR >= 0.0) {
    for (int q = 0; q < 7; ++q) F[q] = FR[q] + SR * (UsR[q] - UR[q]) + SsR * (UssR[q] - UsR[q]);
  } else if (SR >= 0.0) {
    for (int q = 0; q < 7; ++q) F[q] = FR[q] + SR * (UsR[q] - UR[q]);
  } else {
    for (int q = 0; q < 7; ++q) F[q] = FR[q];
  }
  R up = SM;
  if (std::fabs(val(SM)) <= ph.eps_deg * std::max(-val(SL), val(SR))) up = R(0.0);
  F[7] = (SL > 0.0) ? SL : ((SR < 0.0) ? SR : up);
}

// ---------------------------------------------------------------------------
// Non-ideal electric field (Sec. 4.3) on the edges of constrained transport,
// from the state at t^n: Ohmic E = eta J (Eq. Ohm) and ambipolar
// E = -v_D x B with v_D = J x B / (gamma_AD rho rho_i) (Eq. AD), written as
// (B^2 J - (J.B) B) / (gamma_AD rho rho_i).  J_a = (curl B)_a lives on the
// a-edges (a-index a cell index, b- and c-indices face indices, (a, b, c)
// cyclic); on each a-edge the other two components of J are the means of
// the four nearest b- (c-) edges, B_a the mean of the eight nearest a-faces,
// B_b and B_c the means of the two b- (c-) faces through the edge, and rho
// the mean of the four cells around it.  The field is added to the edge
// EMFs.  The energy flux through each face gains the Poynting flux E x B of
// this field (the face means of the two E components on its edges and of the
// two transverse B components on the four faces around it), so that total
// energy is conserved and the magnetic energy removed appears as heat J.E
// (Eqs. Ohm_heat and Q_AD) in the internal energy.
template <class R>
void nonideal(const Layout& L, const std::vector<R>& P, const Box3<Prim<R>>& W, double dx, const Phys& ph,
              Box3<R>* E, Box3<Flux<R>>* Fx) {
  const int n = L.n;
  auto bf = [&](int d, const int* q) -> R { return P[L.face(d, q[0], q[1], q[2])]; };
  // J_a on a-edges with a-cell index in [-1, n] and face indices in [0, n]
  Box3<R> J[3];
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    int lo[3] = {0, 0, 0}, hi[3] = {n, n, n};
    lo[a] = -1;
    J[a].init(lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]);
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          const int e[3] = {i, j, k};
          int eb[3] = {i, j, k}, ec[3] = {i, j, k};
          eb[b] -= 1;
          ec[c] -= 1;
          // dB_c/dx_b - dB_b/dx_c
          J[a].at(e) = ((bf(c, e) - bf(c, eb)) - (bf(b, e) - bf(b, ec))) / dx;
        }
  }
  // the non-ideal field on the EMF edges: a-cell in [0, n-1], faces in [0, n]
  Box3<R> En[3];
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    int lo[3] = {0, 0, 0}, hi[3] = {n, n, n};
    hi[a] = n - 1;
    En[a].init(lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]);
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          const int e[3] = {i, j, k};
          const R ja = J[a].at(e);
          R en = ph.eta * ja;
          if (ph.gamma_ad > 0.0) {
            R jb = 0.0, jc = 0.0, ba = 0.0, bb = 0.0, bc = 0.0, rho = 0.0;
            for (int s = -1; s <= 0; ++s)
              for (int t = 0; t <= 1; ++t) {
                int q[3] = {i, j, k};
                q[b] += s;
                q[a] += t;
                jb = jb + J[b].at(q);
                int r[3] = {i, j, k};
                r[c] += s;
                r[a] += t;
                jc = jc + J[c].at(r);
              }
            for (int t = 0; t <= 1; ++t)
              for (int s = -1; s <= 0; ++s)
                for (int u = -1; u <= 0; ++u) {
                  int q[3] = {i, j, k};
                  q[a] += t;
                  q[b] += s;
                  q[c] += u;
                  ba = ba + bf(a, q);
                }
            for (int s = -1; s <= 0; ++s) {
              int q[3] = {i, j, k}, r[3] = {i, j, k}, w[3] = {i, j, k};
              q[c] += s;  // b-faces through the edge
              bb = bb + bf(b, q);
              r[b] += s;  // c-faces through the edge
              bc = bc + bf(c, r);
              for (int u = -1; u <= 0; ++u) {
                w[b] = e[b] + s;
                w[c] = e[c] + u;
                rho = rho + W.at(w).r;
              }
            }
            jb = 0.25 * jb;
            jc = 0.25 * jc;
            ba = 0.125 * ba;
            bb = 0.5 * bb;
            bc = 0.5 * bc;
            rho = 0.25 * rho;
            const R b2 = ba * ba + bb * bb + bc * bc;
            const R jdotb = ja * ba + jb * bb + jc * bc;
            en = en + (b2 * ja - jdotb * ba) / (ph.gamma_ad * ph.rho_i * rho);
          }
          En[a].at(e) = en;
          E[a].at(e) = E[a].at(e) + en;
        }
  }
  // Poynting flux (E x B)_d on d-faces with face index in [0, n] and cells in [0, n-1]
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    int hi[3] = {n - 1, n - 1, n - 1};
    hi[d] = n;
    for (int k = 0; k <= hi[2]; ++k)
      for (int j = 0; j <= hi[1]; ++j)
        for (int i = 0; i <= hi[0]; ++i) {
          const int f[3] = {i, j, k};
          R e1 = 0.0, e2 = 0.0, b1 = 0.0, b2 = 0.0;
          for (int s = 0; s <= 1; ++s) {
            int q[3] = {i, j, k}, r[3] = {i, j, k};
            q[t2] += s;  // t1-edges on the face
            e1 = e1 + En[t1].at(q);
            r[t1] += s;  // t2-edges on the face
            e2 = e2 + En[t2].at(r);
            for (int u = -1; u <= 0; ++u) {
              int x[3] = {i, j, k}, y[3] = {i, j, k};
              x[t2] += s;  // t2-faces around the face
              x[d] += u;
              b2 = b2 + bf(t2, x);
              y[t1] += s;  // t1-faces around the face
              y[d] += u;
              b1 = b1 + bf(t1, y);
            }
          }
          e1 = 0.5 * e1;
          e2 = 0.5 * e2;
          b1 = 0.25 * b1;
          b2 = 0.25 * b2;
          Flux<R>& F = Fx[d].at(f);
          F.e = F.e + (e1 * b2 - e2 * b1);
        }
  }
}

// ---------------------------------------------------------------------------
// One MUSCL-Hancock + HLLD + CT step of one patch.
//   P   padded array (ng >= 2 guard layers filled), at time t^n
//   W   primitives of P over [-2, n+1]^3 (from prims())
//   out the new interior slice (layout with ng = 0)
template <class R>
void step(const Layout& L, const std::vector<R>& P, const Box3<Prim<R>>& W, R dt, double dx,
          const Phys& ph, std::vector<R>& out, StepCounters& cnt) {
  const int n = L.n;
  const double g = ph.gamma;

  // van Leer slopes of primitive variables, per direction, on [-1, n]^3.
  // The normal field component is not reconstructed along its own axis.
  Box3<Prim<R>> S[3];
  for (int d = 0; d < 3; ++d) {
    S[d].init(-1, n, -1, n, -1, n);
    for (int k = -1; k <= n; ++k)
      for (int j = -1; j <= n; ++j)
        for (int i = -1; i <= n; ++i) {
          int c[3] = {i, j, k}, cm[3] = {i, j, k}, cp[3] = {i, j, k};
          cm[d] -= 1;
          cp[d] += 1;
          const Prim<R>& w0 = W.at(c);
          const Prim<R>& wm = W.at(cm);
          const Prim<R>& wp = W.at(cp);
          auto vl = [](R a, R b, R c2) {
            R dl = b - a, dr = c2 - b;
            if (dl * dr > 0.0) return R(2.0 * dl * dr / (dl + dr));
            return R(0.0);
          };
          Prim<R> s;
          s.r = vl(wm.r, w0.r, wp.r);
          for (int q = 0; q < 3; ++q) s.v[q] = vl(wm.v[q], w0.v[q], wp.v[q]);
          s.p = vl(wm.p, w0.p, wp.p);
          for (int q = 0; q < 3; ++q) s.b[q] = (q == d) ? R(0.0) : vl(wm.b[q], w0.b[q], wp.b[q]);
          S[d](i, j, k) = s;
        }
  }

  // Hancock half-step predictor with the primitive-variable Jacobians of the
  // three 1-D problems (normal field held constant in each), summed x, y, z.
  Box3<Prim<R>> H;
  H.init(-1, n, -1, n, -1, n);
  const R hdtdx = 0.5 * dt / dx;
  for (int k = -1; k <= n; ++k)
    for (int j = -1; j <= n; ++j)
      for (int i = -1; i <= n; ++i) {
        const Prim<R>& w = W(i, j, k);
        R sr = 0.0, sv[3] = {0.0, 0.0, 0.0}, sp = 0.0, sb[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < 3; ++d) {
          int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
          const Prim<R>& s = S[d](i, j, k);
          R un = w.v[d];
          sr = sr + (un * s.r + w.r * s.v[d]);
          sv[d] = sv[d] + (un * s.v[d] + (s.p + w.b[t1] * s.b[t1] + w.b[t2] * s.b[t2]) / w.r);
          sv[t1] = sv[t1] + (un * s.v[t1] - w.b[d] * s.b[t1] / w.r);
          sv[t2] = sv[t2] + (un * s.v[t2] - w.b[d] * s.b[t2] / w.r);
          sp = sp + (un * s.p + g * w.p * s.v[d]);
          sb[t1] = sb[t1] + (un * s.b[t1] + w.b[t1] * s.v[d] - w.b[d] * s.v[t1]);
          sb[t2] = sb[t2] + (un * s.b[t2] + w.b[t2] * s.v[d] - w.b[d] * s.v[t2]);
        }
        Prim<R> h;
        h.r = w.r - hdtdx * sr;
        for (int q = 0; q < 3; ++q) h.v[q] = w.v[q] - hdtdx * sv[q];
        h.p = w.p - hdtdx * sp;
        for (int q = 0; q < 3; ++q) h.b[q] = w.b[q] - hdtdx * sb[q];
        H(i, j, k) = h;
      }

  // Interface fluxes: faces along d with face index in [0, n] and the other
  // two indices in [-1, n] (the transverse halo is needed by the edge EMFs).
  Box3<Flux<R>> Fx[3];
  for (int d = 0; d < 3; ++d) {
    int lo[3] = {-1, -1, -1}, hi[3] = {n, n, n};
    lo[d] = 0;
    Fx[d].init(lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]);
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          int cb[3] = {i, j, k}, ca[3] = {i, j, k};
          ca[d] -= 1;  // left cell a, right cell b; face index = index of b
          const Prim<R>& ha = H.at(ca);
          const Prim<R>& hb = H.at(cb);
          const Prim<R>& sa = S[d].at(ca);
          const Prim<R>& sb = S[d].at(cb);
          const Prim<R>& wa = W.at(ca);
          const Prim<R>& wb = W.at(cb);
          R bface = P[L.face(d, i, j, k)];
          R wl[7], wr[7], bn;
          wl[0] = ha.r + 0.5 * sa.r;
          wl[1] = ha.v[d] + 0.5 * sa.v[d];
          wl[2] = ha.v[t1] + 0.5 * sa.v[t1];
          wl[3] = ha.v[t2] + 0.5 * sa.v[t2];
          wl[4] = ha.p + 0.5 * sa.p;
          wl[5] = ha.b[t1] + 0.5 * sa.b[t1];
          wl[6] = ha.b[t2] + 0.5 * sa.b[t2];
          wr[0] = hb.r - 0.5 * sb.r;
          wr[1] = hb.v[d] - 0.5 * sb.v[d];
          wr[2] = hb.v[t1] - 0.5 * sb.v[t1];
          wr[3] = hb.v[t2] - 0.5 * sb.v[t2];
          wr[4] = hb.p - 0.5 * sb.p;
          wr[5] = hb.b[t1] - 0.5 * sb.b[t1];
          wr[6] = hb.b[t2] - 0.5 * sb.b[t2];
          // time-centred normal field: face value plus the mean predictor
          // increment of the cell-centred normal component on both sides
          bn = bface + 0.5 * ((ha.b[d] - wa.b[d]) + (hb.b[d] - wb.b[d]));
          if (!(val(wl[0]) > 0.0) || !(val(wl[4]) > 0.0) || !(val(wr[0]) > 0.0) ||
              !(val(wr[4]) > 0.0)) {
            // first-order fallback: the cell states at t^n
            wl[0] = wa.r; wl[1] = wa.v[d]; wl[2] = wa.v[t1]; wl[3] = wa.v[t2];
            wl[4] = wa.p; wl[5] = wa.b[t1]; wl[6] = wa.b[t2];
            wr[0] = wb.r; wr[1] = wb.v[d]; wr[2] = wb.v[t1]; wr[3] = wb.v[t2];
            wr[4] = wb.p; wr[5] = wb.b[t1]; wr[6] = wb.b[t2];
            bn = bface;
            cnt.fallback_faces++;
          }
          R f7[8];
          hlld(wl, wr, bn, ph, f7);
          Flux<R> f;
          f.r = f7[0];
          f.m[d] = f7[1];
          f.m[t1] = f7[2];
          f.m[t2] = f7[3];
          f.e = f7[4];
          f.b[d] = 0.0;
          f.b[t1] = f7[5];
          f.b[t2] = f7[6];
          f.u = f7[7];
          Fx[d](i, j, k) = f;
        }
  }

  // Cell-centred reference EMF, E = -v x B, from the half-step state.
  Box3<Prim<R>> Ecc;  // only .v[] used, as the three EMF components
  Ecc.init(-1, n, -1, n, -1, n);
  for (int k = -1; k <= n; ++k)
    for (int j = -1; j <= n; ++j)
      for (int i = -1; i <= n; ++i) {
        const Prim<R>& h = H(i, j, k);
        Prim<R> e;
        for (int a = 0; a < 3; ++a) {
          int b = (a + 1) % 3, c = (a + 2) % 3;
          e.v[a] = h.v[c] * h.b[b] - h.v[b] * h.b[c];
        }
        Ecc(i, j, k) = e;
      }

  // Edge EMFs (Gardiner & Stone 2005), upwinded by the direction of the mass
  // flux, taken as the sign of the face's upwind speed (Flux::u).
  // E_a lives on edges along a; its a-index is a cell index in [0, n-1] and
  // its b- and c-indices are face indices in [0, n], with (a, b, c) cyclic.
  Box3<R> E[3];
  for (int a = 0; a < 3; ++a) {
    int b = (a + 1) % 3, c = (a + 2) % 3;
    int lo[3] = {0, 0, 0}, hi[3] = {n, n, n};
    hi[a] = n - 1;
    E[a].init(lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]);
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          int e0[3] = {i, j, k};
          // b-faces at the edge's b position, c-cells fc (upper) and fc-1 (lower)
          int pA[3] = {i, j, k}, pB[3] = {i, j, k};
          pB[c] -= 1;
          // c-faces at the edge's c position, b-cells fb (upper) and fb-1 (lower)
          int pC[3] = {i, j, k}, pD[3] = {i, j, k};
          pD[b] -= 1;
          const Flux<R>& FA = Fx[b].at(pA);
          const Flux<R>& FB = Fx[b].at(pB);
          const Flux<R>& FC = Fx[c].at(pC);
          const Flux<R>& FD = Fx[c].at(pD);
          R A = -FA.b[c], B = -FB.b[c];  // face EMF E_a = -F_b[B_c]
          R C = FC.b[b], D = FD.b[b];    // face EMF E_a = +F_c[B_b]
          // cell centres around the edge: (b-cell, c-cell) offsets
          int q00[3] = {i, j, k}, q10[3] = {i, j, k}, q01[3] = {i, j, k}, q11[3] = {i, j, k};
          q00[b] -= 1; q00[c] -= 1;
          q10[c] -= 1;
          q01[b] -= 1;
          R c00 = Ecc.at(q00).v[a], c10 = Ecc.at(q10).v[a];
          R c01 = Ecc.at(q01).v[a], c11 = Ecc.at(q11).v[a];
          auto up = [](R m, R x, R y) {  // x if m > 0, y if m < 0, mean if 0
            if (m > 0.0) return x;
            if (m < 0.0) return y;
            return R(0.5 * (x + y));
          };
          R dc14 = up(FA.u, c01 - D, c11 - C);
          R dc34 = up(FB.u, D - c00, C - c10);
          R db14 = up(FC.u, c10 - B, c11 - A);
          R db34 = up(FD.u, B - c00, A - c01);
          E[a].at(e0) = 0.25 * (A + B + C + D) + 0.25 * ((dc34 - dc14) + (db34 - db14));
        }
  }

  if (ph.nonideal()) nonideal(L, P, W, dx, ph, E, Fx);

  // Conservative update of the cell variables, fluxes summed x, y, z.
  Layout O(n, 0);
  out.assign(O.size(), R(0.0));
  const R dtdx = dt / dx;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        R du[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int d = 0; d < 3; ++d) {
          int cl[3] = {i, j, k}, cr[3] = {i, j, k};
          cr[d] += 1;
          const Flux<R>& fl = Fx[d].at(cl);
          const Flux<R>& fr = Fx[d].at(cr);
          du[0] = du[0] + (fr.r - fl.r);
          du[1] = du[1] + (fr.m[0] - fl.m[0]);
          du[2] = du[2] + (fr.m[1] - fl.m[1]);
          du[3] = du[3] + (fr.m[2] - fl.m[2]);
          du[4] = du[4] + (fr.e - fl.e);
        }
        for (int v = 0; v < 5; ++v) out[O.cell(v, i, j, k)] = P[L.cell(v, i, j, k)] - dtdx * du[v];
      }

  // Constrained transport: each face field changes by minus the circulation
  // of the edge EMF around the face, so the discrete divergence is unchanged.
  for (int d = 0; d < 3; ++d) {
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    int hi[3] = {n - 1, n - 1, n - 1};
    hi[d] = n;
    for (int k = 0; k <= hi[2]; ++k)
      for (int j = 0; j <= hi[1]; ++j)
        for (int i = 0; i <= hi[0]; ++i) {
          int p0[3] = {i, j, k}, p1[3] = {i, j, k}, p2[3] = {i, j, k};
          p1[t1] += 1;
          p2[t2] += 1;
          R curl = (E[t2].at(p1) - E[t2].at(p0)) - (E[t1].at(p2) - E[t1].at(p0));
          out[O.face(d, i, j, k)] = P[L.face(d, i, j, k)] - dtdx * curl;
        }
  }
}

}  // namespace orc
