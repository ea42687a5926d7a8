// VIPER rod-solver ORACLE -- test infrastructure only.
//
// A plain, serial CPU implementation of one VIPER substep (prediction, coloured
// Gauss-Seidel projection of the rod constraints, Jacobi pill-pill contacts,
// velocity update) and of the skinning transform, written from the paper
// "VIPER: Volume Invariant Position-based Elastic Rods" (Angles et al. 2019).
// It exists only to check the GPU library: only tests/, the smoke entry point and
// the benchmark's CPU-baseline leg may load it.  It shares no code, header or
// table with the GPU library.
//
// Everything is templated on the scalar type R:
//   double      -- the reference (FP64),
//   float       -- the FP32 rounding floor of the same algorithm,
//   Dual<K>     -- forward-mode dual numbers, giving exact derivatives of the
//                  discrete algorithm (gradient oracle); Dual<K, float> gives
//                  the FP32 rounding floor of those derivatives.
//
// Every constraint is projected with ONE generic routine: the per-constraint
// dual update of Sec. 6 (eq. app_dual_formulation_update, beta = 1), written
// with explicit Jacobian blocks J_b and inverse-inertia blocks W_b:
//     S   = sum_b J_b W_b J_b^T + alpha~          (alpha~ = compliance / h^2)
//     dl  = S^-1 (-C - alpha~ lambda),   lambda += dl
//     dX_b = W_b J_b^T dl
// (the paper's lambda equals -lambda/h^2 here and K^-1 = compliance).  No closed
// form shortcut is used, so the GPU's closed forms are checked against this.
//
// Readings of the paper that this file commits to (the paper is silent or
// inconsistent there) are listed where used; each is marked "reading:".
//
// Parity pins for every function live in tests/test_oracle_*.py.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <type_traits>
#include <vector>

namespace orc {

// ---------------------------------------------------------------------------
// Forward-mode dual numbers with K directions.
// ---------------------------------------------------------------------------
template <int K, class B = double>
struct Dual {
  B v;
  B d[K];
  Dual() : v(0) { for (int i = 0; i < K; ++i) d[i] = 0; }
  Dual(double a) : v(B(a)) { for (int i = 0; i < K; ++i) d[i] = 0; }
};
#define DT_ template <int K, class B>
#define DD_ Dual<K, B>
DT_ DD_ operator+(const DD_& a, const DD_& b) { DD_ r; r.v = a.v + b.v; for (int i = 0; i < K; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
DT_ DD_ operator-(const DD_& a, const DD_& b) { DD_ r; r.v = a.v - b.v; for (int i = 0; i < K; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
DT_ DD_ operator-(const DD_& a) { DD_ r; r.v = -a.v; for (int i = 0; i < K; ++i) r.d[i] = -a.d[i]; return r; }
DT_ DD_ operator*(const DD_& a, const DD_& b) { DD_ r; r.v = a.v * b.v; for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
DT_ DD_ operator/(const DD_& a, const DD_& b) { DD_ r; r.v = a.v / b.v; for (int i = 0; i < K; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
DT_ DD_& operator+=(DD_& a, const DD_& b) { a = a + b; return a; }
DT_ DD_& operator-=(DD_& a, const DD_& b) { a = a - b; return a; }
DT_ DD_& operator*=(DD_& a, const DD_& b) { a = a * b; return a; }
DT_ DD_& operator/=(DD_& a, const DD_& b) { a = a / b; return a; }
DT_ bool operator<(const DD_& a, const DD_& b) { return a.v < b.v; }
DT_ bool operator>(const DD_& a, const DD_& b) { return a.v > b.v; }
DT_ bool operator<=(const DD_& a, const DD_& b) { return a.v <= b.v; }
DT_ bool operator>=(const DD_& a, const DD_& b) { return a.v >= b.v; }
DT_ DD_ sqrt(const DD_& a) { DD_ r; r.v = std::sqrt(a.v); for (int i = 0; i < K; ++i) r.d[i] = a.d[i] / (B(2) * r.v); return r; }

inline double val(double a) { return a; }
inline double val(float a) { return a; }
DT_ double val(const DD_& a) { return a.v; }
#undef DT_
#undef DD_
inline double sqrt(double a) { return std::sqrt(a); }
inline float sqrt(float a) { return std::sqrt(a); }

template <class R> R rmax(const R& a, const R& b) { return (a < b) ? b : a; }
template <class R> R rmin(const R& a, const R& b) { return (b < a) ? b : a; }

// ---------------------------------------------------------------------------
// 3-vectors, 3x3 matrices and quaternions (x, y, z, w; w is the real part).
// ---------------------------------------------------------------------------
template <class R> struct V3 { R x, y, z; };
template <class R> V3<R> v3(R a, R b, R c) { V3<R> r; r.x = a; r.y = b; r.z = c; return r; }
template <class R> V3<R> operator+(const V3<R>& a, const V3<R>& b) { return v3<R>(a.x + b.x, a.y + b.y, a.z + b.z); }
template <class R> V3<R> operator-(const V3<R>& a, const V3<R>& b) { return v3<R>(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class R> V3<R> operator*(const R& s, const V3<R>& a) { return v3<R>(s * a.x, s * a.y, s * a.z); }
template <class R> R dot(const V3<R>& a, const V3<R>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class R> V3<R> cross(const V3<R>& a, const V3<R>& b) { return v3<R>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
template <class R> R norm(const V3<R>& a) { return sqrt(dot(a, a)); }

template <class R> struct M3 { R m[3][3]; };
template <class R> M3<R> mzero() { M3<R> r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.m[i][j] = R(0.0); return r; }
template <class R> M3<R> mident() { M3<R> r = mzero<R>(); r.m[0][0] = r.m[1][1] = r.m[2][2] = R(1.0); return r; }
template <class R> M3<R> mmul(const M3<R>& a, const M3<R>& b) { M3<R> r = mzero<R>(); for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) for (int k = 0; k < 3; ++k) r.m[i][j] += a.m[i][k] * b.m[k][j]; return r; }
template <class R> M3<R> mtrans(const M3<R>& a) { M3<R> r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[j][i]; return r; }
template <class R> V3<R> mvec(const M3<R>& a, const V3<R>& v) { return v3<R>(a.m[0][0] * v.x + a.m[0][1] * v.y + a.m[0][2] * v.z, a.m[1][0] * v.x + a.m[1][1] * v.y + a.m[1][2] * v.z, a.m[2][0] * v.x + a.m[2][1] * v.y + a.m[2][2] * v.z); }
template <class R> M3<R> skew(const V3<R>& a) { M3<R> r = mzero<R>(); r.m[0][1] = -a.z; r.m[0][2] = a.y; r.m[1][0] = a.z; r.m[1][2] = -a.x; r.m[2][0] = -a.y; r.m[2][1] = a.x; return r; }

template <class R> struct Q4 { R x, y, z, w; };
template <class R> Q4<R> q4(R x, R y, R z, R w) { Q4<R> r; r.x = x; r.y = y; r.z = z; r.w = w; return r; }
// Hamilton product a (x) b.
template <class R> Q4<R> qmul(const Q4<R>& a, const Q4<R>& b) {
  return q4<R>(a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
               a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
               a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w,
               a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z);
}
template <class R> Q4<R> qconj(const Q4<R>& a) { return q4<R>(-a.x, -a.y, -a.z, a.w); }
template <class R> Q4<R> qnormalize(const Q4<R>& a) { R n = sqrt(a.x * a.x + a.y * a.y + a.z * a.z + a.w * a.w); return q4<R>(a.x / n, a.y / n, a.z / n, a.w / n); }
template <class R> V3<R> qim(const Q4<R>& a) { return v3<R>(a.x, a.y, a.z); }
// Rotation matrix of a unit quaternion.
template <class R> M3<R> qmat(const Q4<R>& q) {
  M3<R> r;
  R x = q.x, y = q.y, z = q.z, w = q.w;
  R one(1.0), two(2.0);
  r.m[0][0] = one - two * (y * y + z * z); r.m[0][1] = two * (x * y - w * z); r.m[0][2] = two * (x * z + w * y);
  r.m[1][0] = two * (x * y + w * z); r.m[1][1] = one - two * (x * x + z * z); r.m[1][2] = two * (y * z - w * x);
  r.m[2][0] = two * (x * z - w * y); r.m[2][1] = two * (y * z + w * x); r.m[2][2] = one - two * (x * x + y * y);
  return r;
}
// The rod tangent director d3 = R(q) e_z (the frame axis along the curve, Sec. 3).
template <class R> V3<R> qd3(const Q4<R>& q) { M3<R> m = qmat(q); return v3<R>(m.m[0][2], m.m[1][2], m.m[2][2]); }
// Apply a small world-frame rotation dtheta to q: q <- normalize(q + 1/2 [dtheta, 0] (x) q).
// Reading: the paper's small-angle quaternion [theta/2, 1] (Sec. 7, energy implementation).
template <class R> Q4<R> qrotate(const Q4<R>& q, const V3<R>& dth) {
  R h(0.5);
  Q4<R> p = q4<R>(h * dth.x, h * dth.y, h * dth.z, R(0.0));
  Q4<R> d = qmul(p, q);
  return qnormalize(q4<R>(q.x + d.x, q.y + d.y, q.z + d.z, q.w + d.w));
}

// Shortest-arc rotation taking unit vector a onto unit vector b (double only; rest data).
inline Q4<double> shortest_arc(const V3<double>& a, const V3<double>& b) {
  double c = dot(a, b);
  if (c < -1.0 + 1e-12) {
    // Opposite vectors: rotate by pi about any axis orthogonal to a.
    V3<double> ax = (std::fabs(a.x) < 0.9) ? cross(a, v3<double>(1, 0, 0)) : cross(a, v3<double>(0, 1, 0));
    double n = norm(ax);
    return q4<double>(ax.x / n, ax.y / n, ax.z / n, 0.0);
  }
  V3<double> ax = cross(a, b);
  return qnormalize(q4<double>(ax.x, ax.y, ax.z, 1.0 + c));
}

// ---------------------------------------------------------------------------
// Generic per-constraint dual (XPBD) update of Sec. 6 for a constraint of
// dimension m (1 or 3) acting on blocks of 1 (scale) or 3 (position, rotation)
// degrees of freedom.
// ---------------------------------------------------------------------------
template <class R> struct Block {
  int ndof;        // 1 or 3
  R J[3][3];       // m x ndof Jacobian block
  R W[3][3];       // ndof x ndof inverse inertia block
  R out[3];        // resulting correction W J^T dl
};

// Solve the m x m system S y = b by Cramer's rule (m = 1, 2 or 3).  The system is
// first divided by its largest entry (same solution) so that the cubic
// determinants stay inside the float range when R = float.
template <class R> void solve_small(int m, const R S0[3][3], const R b0[3], R y[3]) {
  if (m == 1) { y[0] = b0[0] / S0[0][0]; return; }
  if (m == 2) {
    R big(0.0);
    for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) { R a = S0[i][j] < R(0.0) ? -S0[i][j] : S0[i][j]; big = rmax(big, a); }
    const R a = S0[0][0] / big, b = S0[0][1] / big, c = S0[1][0] / big, d = S0[1][1] / big;
    const R e = b0[0] / big, f = b0[1] / big;
    const R det = a * d - b * c;
    y[0] = (e * d - b * f) / det;
    y[1] = (a * f - e * c) / det;
    return;
  }
  R big(0.0);
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) { R a = S0[i][j] < R(0.0) ? -S0[i][j] : S0[i][j]; big = rmax(big, a); }
  R S[3][3], b[3];
  for (int i = 0; i < 3; ++i) { b[i] = b0[i] / big; for (int j = 0; j < 3; ++j) S[i][j] = S0[i][j] / big; }
  R det = S[0][0] * (S[1][1] * S[2][2] - S[1][2] * S[2][1]) - S[0][1] * (S[1][0] * S[2][2] - S[1][2] * S[2][0]) +
          S[0][2] * (S[1][0] * S[2][1] - S[1][1] * S[2][0]);
  for (int c = 0; c < 3; ++c) {
    R T[3][3];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) T[i][j] = (j == c) ? b[i] : S[i][j];
    R dc = T[0][0] * (T[1][1] * T[2][2] - T[1][2] * T[2][1]) - T[0][1] * (T[1][0] * T[2][2] - T[1][2] * T[2][0]) +
           T[0][2] * (T[1][0] * T[2][1] - T[1][1] * T[2][0]);
    y[c] = dc / det;
  }
}

// C[m], alpha[m] (diagonal compliance already divided by h^2), lambda[m] in/out.
template <class R> void xpbd_update(int m, const R* C, const R* alpha, R* lambda, Block<R>* blocks, int nb) {
  R S[3][3];
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) S[i][j] = R(0.0);
  for (int b = 0; b < nb; ++b) {
    Block<R>& B = blocks[b];
    // JW = J W   (m x ndof)
    R JW[3][3];
    for (int i = 0; i < m; ++i) for (int k = 0; k < B.ndof; ++k) { JW[i][k] = R(0.0); for (int l = 0; l < B.ndof; ++l) JW[i][k] += B.J[i][l] * B.W[l][k]; }
    for (int i = 0; i < m; ++i) for (int j = 0; j < m; ++j) for (int k = 0; k < B.ndof; ++k) S[i][j] += JW[i][k] * B.J[j][k];
  }
  for (int i = 0; i < m; ++i) S[i][i] += alpha[i];
  R rhs[3], dl[3];
  for (int i = 0; i < m; ++i) rhs[i] = -C[i] - alpha[i] * lambda[i];
  solve_small(m, S, rhs, dl);
  for (int i = 0; i < m; ++i) lambda[i] += dl[i];
  for (int b = 0; b < nb; ++b) {
    Block<R>& B = blocks[b];
    for (int k = 0; k < B.ndof; ++k) {
      R acc(0.0);
      for (int l = 0; l < B.ndof; ++l) for (int i = 0; i < m; ++i) acc += B.W[k][l] * B.J[i][l] * dl[i];
      B.out[k] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Scene description (host arrays; FP64) -- the oracle's own copy of the inputs.
// ---------------------------------------------------------------------------
struct Desc {
  int num_rods;
  const int32_t* rod_offsets;    // [num_rods + 1]
  const double* rest_pos;        // [P*3]
  const double* rest_radius;     // [P]
  const uint8_t* pinned;         // [P]
  const double* activation;      // [num_rods]
  const double* compliance;      // [num_rods*4]: ss, vol, sg, bt (Pa^-1); +inf disables
  const int32_t* group;          // [num_rods]
  double density;
  double gravity[3];
};

enum { SS = 0, VOL = 1, SG = 2, BT = 3, SR = 4, SB = 5, VB = 6 };

template <class R> struct Scene {
  int nrods = 0, P = 0;
  std::vector<int> off, rod_of, group;
  std::vector<uint8_t> pinned;
  V3<R> g;
  double density = 1000.0;
  // parameters (differentiable)
  std::vector<R> rbar;        // rest radius per pill
  std::vector<R> act;         // activation per rod
  // rest data
  std::vector<V3<double>> xrest;
  std::vector<R> l0, lbar;    // per edge slot (slot j of pill j; last slot of a rod unused)
  std::vector<Q4<R>> qrest;
  std::vector<V3<R>> darb_rest;   // rest Darboux vector of the BT constraint at slot j (edges j, j+1)
  std::vector<R> winv, wsinv;     // inverse position / scale mass per pill
  std::vector<R> inert_base;      // rho pi rbar_{j+1/2}^4 l0_j per edge (times s^2 diag(1/4,1/4,1/2))
  std::vector<R> comp[4];         // per-constraint compliance alpha_type / (G * length), per slot
  std::vector<uint8_t> enabled;   // [nrods*4]
  // cross-section stretch (eq. stretch_xy), optional, off by default: per-rod enable,
  // per-slot compliance alpha / (pi r^2 l) and multiplier
  std::vector<uint8_t> sr_on;
  std::vector<R> comp_sr, lam_sr;
  // surface bending (second variation of the scale along the rod), optional, off by default:
  // per-rod enable, per-slot compliance alpha / (pi r^4 / 4 l_v) and multiplier (slot p: the
  // vertex between edges p and p+1)
  std::vector<uint8_t> sb_on;
  std::vector<R> comp_sb, lam_sb;
  // volume-bending coupling (the s^3 Omega^{u,v} terms of the volume energy), optional, off by
  // default, on rods whose volume constraint is on: compliance alpha_vol / (pi r^4 / 2 l_v)
  // per slot (vertex after edge p) and two multipliers
  bool vb_on = false;
  std::vector<double> alpha_vol;   // [nrods] the volume compliance as given
  std::vector<R> comp_vb, lam_vb;
  // state
  std::vector<V3<R>> x, v;
  std::vector<R> s, sd;
  std::vector<Q4<R>> q;
  std::vector<V3<R>> om;
  // per-substep scratch
  std::vector<V3<R>> xprev;
  std::vector<R> sprev, I1inv, I3inv;
  std::vector<Q4<R>> qprev;
  std::vector<R> lam;          // [slot*8]: ss(3) vol(1) sg(1) bt(3)
  // contacts
  // bundling (Sec. 7.3): cross-sections as lists of pills, and each section's rotation of the
  // previous substep (the start of the next rotation extraction)
  std::vector<int> sec_off, sec_pill;
  std::vector<Q4<double>> sec_q;
  // solver for the rod constraints: false = coloured Gauss-Seidel, true = Jacobi with
  // averaging (the paper's engine, Sec. 7)
  bool jacobi = false;
  // kinematic half-plane floor (Sec. 7): pills stay in n . x >= d
  bool floor_on = false;
  V3<double> floor_n;
  double floor_d = 0.0;
  // kinematic bones (Sec. 8.2): each bone's transform of the last frame, [A | b] row-major
  // 3x4 per bone, and two (bone, weight) influences per pill
  int nbones = 0;
  std::vector<double> bone_prev;
  std::vector<int32_t> pill_bone;
  std::vector<double> pill_bone_w;
  std::vector<int32_t> pairs;  // sorted (a, b), a < b, capsule id = first pill of the edge
  std::vector<int> active_count; // number of active contacts in the last contact pass
  int64_t projections = 0;     // count of rod + active contact projections performed

  bool has_edge(int p) const { return p + 1 < off[rod_of[p] + 1]; }
  bool has_bt(int p) const { return p + 2 < off[rod_of[p] + 1]; }
  int local(int p) const { return p - off[rod_of[p]]; }
};

// Build rest data (Sec. 4 discretisation, Sec. 6 inertia weights, App. B).
// Reading: masses lump each element's inertia weight half to each end vertex;
// rotational inertia uses the substep-start midpoint scale (frozen per substep).
template <class R> void build(Scene<R>& S, const Desc& d, const R* rbar, const R* act) {
  const double pi = 3.14159265358979323846;
  S.nrods = d.num_rods;
  S.off.assign(d.rod_offsets, d.rod_offsets + d.num_rods + 1);
  S.P = S.off[S.nrods];
  const int P = S.P;
  S.rod_of.resize(P);
  for (int k = 0; k < S.nrods; ++k) for (int p = S.off[k]; p < S.off[k + 1]; ++p) S.rod_of[p] = k;
  S.group.assign(d.group, d.group + S.nrods);
  S.pinned.assign(d.pinned, d.pinned + P);
  S.g = v3<R>(R(d.gravity[0]), R(d.gravity[1]), R(d.gravity[2]));
  S.density = d.density;
  S.rbar.assign(rbar, rbar + P);
  S.act.assign(act, act + S.nrods);
  S.xrest.resize(P);
  for (int p = 0; p < P; ++p) S.xrest[p] = v3<double>(d.rest_pos[3 * p], d.rest_pos[3 * p + 1], d.rest_pos[3 * p + 2]);
  S.l0.assign(P, R(0.0)); S.lbar.assign(P, R(0.0));
  S.qrest.assign(P, q4<R>(R(0.0), R(0.0), R(0.0), R(1.0)));
  S.darb_rest.assign(P, v3<R>(R(0.0), R(0.0), R(0.0)));
  S.inert_base.assign(P, R(0.0));
  for (int t = 0; t < 4; ++t) S.comp[t].assign(P, R(0.0));
  S.enabled.assign(S.nrods * 4, 1);
  S.alpha_vol.assign(S.nrods, 0.0);
  std::vector<R> M(P, R(0.0)), Ms(P, R(0.0));
  R rho(d.density), PI(pi);
  for (int k = 0; k < S.nrods; ++k) {
    for (int t = 0; t < 4; ++t) S.enabled[4 * k + t] = std::isfinite(d.compliance[4 * k + t]) ? 1 : 0;
    S.alpha_vol[k] = d.compliance[4 * k + VOL];
    const int a = S.off[k], b = S.off[k + 1];
    // rest frames by parallel transport (reading: zero rest twist; q0 takes e_z onto t0)
    std::vector<Q4<double>> qd(b - a);
    V3<double> tprev = v3<double>(0, 0, 1);
    Q4<double> qcur = q4<double>(0, 0, 0, 1);
    for (int p = a; p + 1 < b; ++p) {
      V3<double> e = S.xrest[p + 1] - S.xrest[p];
      double len = norm(e);
      V3<double> t = (1.0 / len) * e;
      qcur = qnormalize(qmul(shortest_arc(tprev, t), qcur));
      qd[p - a] = qcur;
      tprev = t;
      S.l0[p] = R(len);
      S.lbar[p] = S.act[k] * R(len);
      S.qrest[p] = q4<R>(R(qcur.x), R(qcur.y), R(qcur.z), R(qcur.w));
    }
    for (int p = a; p + 1 < b; ++p) {
      R rm = R(0.5) * (S.rbar[p] + S.rbar[p + 1]);
      R r2 = rm * rm, r4 = r2 * r2;
      R Me = rho * PI * r2 * S.l0[p];                 // pi r^2 m l   (position weight)
      R Mse = rho * PI * r4 * S.l0[p] / R(2.0);       // pi r^4 m / 2 l (scale weight)
      M[p] += R(0.5) * Me; M[p + 1] += R(0.5) * Me;
      Ms[p] += R(0.5) * Mse; Ms[p + 1] += R(0.5) * Mse;
      S.inert_base[p] = rho * PI * r4 * S.l0[p];
      // compliance alpha / (G * length) with G = pi r^2 (SS, VOL), pi r^4 / 2 (SG)
      S.comp[SS][p] = R(d.compliance[4 * k + SS]) / (PI * r2 * S.l0[p]);
      S.comp[VOL][p] = R(d.compliance[4 * k + VOL]) / (PI * r2 * S.l0[p]);
      S.comp[SG][p] = R(d.compliance[4 * k + SG]) / (PI * r4 / R(2.0) * S.l0[p]);
    }
    for (int p = a; p + 2 < b; ++p) {
      // BT lives at vertex p+1; G = pi r^4 / 4 (disc second moment, appendix H), length = Voronoi.
      R rv = S.rbar[p + 1];
      R r4 = rv * rv * rv * rv;
      R lv = R(0.5) * (S.l0[p] + S.l0[p + 1]);
      S.comp[BT][p] = R(d.compliance[4 * k + BT]) / (PI * r4 / R(4.0) * lv);
      Q4<double> rr = qmul(qconj(qd[p - a]), qd[p + 1 - a]);
      if (rr.w < 0) rr = q4<double>(-rr.x, -rr.y, -rr.z, -rr.w);
      R c = R(4.0) / (S.l0[p] + S.l0[p + 1]);
      S.darb_rest[p] = v3<R>(c * R(rr.x), c * R(rr.y), c * R(rr.z));
    }
  }
  S.winv.assign(P, R(0.0)); S.wsinv.assign(P, R(0.0));
  for (int p = 0; p < P; ++p) {
    S.winv[p] = S.pinned[p] ? R(0.0) : R(1.0) / M[p];
    S.wsinv[p] = R(1.0) / Ms[p];
  }
  // initial state: at rest
  S.x.resize(P); S.v.assign(P, v3<R>(R(0.0), R(0.0), R(0.0)));
  for (int p = 0; p < P; ++p) S.x[p] = v3<R>(R(S.xrest[p].x), R(S.xrest[p].y), R(S.xrest[p].z));
  S.s.assign(P, R(1.0)); S.sd.assign(P, R(0.0));
  S.q = S.qrest;
  S.om.assign(P, v3<R>(R(0.0), R(0.0), R(0.0)));
  S.xprev.resize(P); S.sprev.resize(P); S.qprev.resize(P);
  S.I1inv.assign(P, R(0.0)); S.I3inv.assign(P, R(0.0));
  S.lam.assign(size_t(P) * 8, R(0.0));
  S.sr_on.assign(S.nrods, 0);
  S.comp_sr.assign(P, R(0.0));
  S.lam_sr.assign(P, R(0.0));
  S.sb_on.assign(S.nrods, 0);
  S.comp_sb.assign(P, R(0.0));
  S.lam_sb.assign(P, R(0.0));
  S.comp_vb.assign(P, R(0.0));
  S.lam_vb.assign(2 * size_t(P), R(0.0));
  S.active_count.assign(P, 0);
}

// ------------------------------ constraints ---------------------------------

// World-frame inverse rotational inertia of edge p: R diag(1/I1, 1/I1, 1/I3) R^T.
template <class R> M3<R> inv_inertia_world(const Scene<R>& S, int p) {
  M3<R> Rm = qmat(S.q[p]);
  M3<R> D = mzero<R>();
  D.m[0][0] = S.I1inv[p]; D.m[1][1] = S.I1inv[p]; D.m[2][2] = S.I3inv[p];
  return mmul(mmul(Rm, D), mtrans(Rm));
}

// Stretch-shear at edge p (eq. stretch_z; finite difference of Sec. 7):
//   C = (x_{p+1} - x_p) / lbar - d3(q_p)
template <class R> int project_ss(Scene<R>& S, int p, R ih2) {
  const int k = S.rod_of[p];
  if (!S.enabled[4 * k + SS]) return 0;
  R lb = S.lbar[p];
  V3<R> d3 = qd3(S.q[p]);
  V3<R> dx = S.x[p + 1] - S.x[p];
  V3<R> Cv = (R(1.0) / lb) * dx - d3;
  R C[3] = {Cv.x, Cv.y, Cv.z};
  R a = S.comp[SS][p] * ih2;
  R alpha[3] = {a, a, a};
  Block<R> B[3];
  // J_{x_p} = -I/lbar, J_{x_p+1} = I/lbar
  for (int bi = 0; bi < 2; ++bi) {
    B[bi].ndof = 3;
    R sg = (bi == 0) ? R(-1.0) / lb : R(1.0) / lb;
    R w = (bi == 0) ? S.winv[p] : S.winv[p + 1];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) { B[bi].J[i][j] = (i == j) ? sg : R(0.0); B[bi].W[i][j] = (i == j) ? w : R(0.0); }
  }
  // J_theta = dC/dtheta = -d(d3)/dtheta = [d3]_x   (d3 <- d3 + dtheta x d3)
  M3<R> Jt = skew(d3);
  M3<R> Wt = inv_inertia_world(S, p);
  B[2].ndof = 3;
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) { B[2].J[i][j] = Jt.m[i][j]; B[2].W[i][j] = Wt.m[i][j]; }
  xpbd_update(3, C, alpha, &S.lam[size_t(p) * 8 + 0], B, 3);
  S.x[p] = S.x[p] + v3<R>(B[0].out[0], B[0].out[1], B[0].out[2]);
  S.x[p + 1] = S.x[p + 1] + v3<R>(B[1].out[0], B[1].out[1], B[1].out[2]);
  S.q[p] = qrotate(S.q[p], v3<R>(B[2].out[0], B[2].out[1], B[2].out[2]));
  return 1;
}

// Volume at edge p (eq. vol, tangential scalar reading):
//   C = s_{p+1/2}^2 |x_{p+1} - x_p| / l0 - 1,  s_{p+1/2} = (s_p + s_{p+1}) / 2
template <class R> int project_vol(Scene<R>& S, int p, R ih2) {
  const int k = S.rod_of[p];
  if (!S.enabled[4 * k + VOL]) return 0;
  R l0 = S.l0[p];
  V3<R> e = S.x[p + 1] - S.x[p];
  R len = norm(e);
  V3<R> n = (R(1.0) / len) * e;
  R sm = R(0.5) * (S.s[p] + S.s[p + 1]);
  R C[1] = {sm * sm * len / l0 - R(1.0)};
  R alpha[1] = {S.comp[VOL][p] * ih2};
  Block<R> B[4];
  R gx = sm * sm / l0;
  for (int bi = 0; bi < 2; ++bi) {
    B[bi].ndof = 3;
    R sg = (bi == 0) ? -gx : gx;
    R w = (bi == 0) ? S.winv[p] : S.winv[p + 1];
    B[bi].J[0][0] = sg * n.x; B[bi].J[0][1] = sg * n.y; B[bi].J[0][2] = sg * n.z;
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) B[bi].W[i][j] = (i == j) ? w : R(0.0);
  }
  R gs = sm * len / l0;   // dC/ds_p = dC/ds_{p+1} = 2 s_m * 1/2 * len / l0
  for (int bi = 2; bi < 4; ++bi) {
    B[bi].ndof = 1;
    B[bi].J[0][0] = gs;
    B[bi].W[0][0] = (bi == 2) ? S.wsinv[p] : S.wsinv[p + 1];
  }
  xpbd_update(1, C, alpha, &S.lam[size_t(p) * 8 + 3], B, 4);
  S.x[p] = S.x[p] + v3<R>(B[0].out[0], B[0].out[1], B[0].out[2]);
  S.x[p + 1] = S.x[p + 1] + v3<R>(B[1].out[0], B[1].out[1], B[1].out[2]);
  S.s[p] += B[2].out[0];
  S.s[p + 1] += B[3].out[0];
  return 1;
}

// Scale gradient at edge p (eq. surface_stretch): C = (s_{p+1} - s_p) / l0
template <class R> int project_sg(Scene<R>& S, int p, R ih2) {
  const int k = S.rod_of[p];
  if (!S.enabled[4 * k + SG]) return 0;
  R l0 = S.l0[p];
  R C[1] = {(S.s[p + 1] - S.s[p]) / l0};
  R alpha[1] = {S.comp[SG][p] * ih2};
  Block<R> B[2];
  B[0].ndof = 1; B[0].J[0][0] = R(-1.0) / l0; B[0].W[0][0] = S.wsinv[p];
  B[1].ndof = 1; B[1].J[0][0] = R(1.0) / l0; B[1].W[0][0] = S.wsinv[p + 1];
  xpbd_update(1, C, alpha, &S.lam[size_t(p) * 8 + 4], B, 2);
  S.s[p] += B[0].out[0];
  S.s[p + 1] += B[1].out[0];
  return 1;
}

// Cross-section stretch at edge p (eq. stretch_xy): the midpoint scale is pulled back to its
// rest value one, C = (s_p + s_{p+1}) / 2 - 1, with the energy weight pi r^2 of SS and VOL.
template <class R> int project_sr(Scene<R>& S, int p, R ih2) {
  if (!S.sr_on[S.rod_of[p]]) return 0;
  R C[1] = {R(0.5) * (S.s[p] + S.s[p + 1]) - R(1.0)};
  R alpha[1] = {S.comp_sr[p] * ih2};
  Block<R> B[2];
  B[0].ndof = 1; B[0].J[0][0] = R(0.5); B[0].W[0][0] = S.wsinv[p];
  B[1].ndof = 1; B[1].J[0][0] = R(0.5); B[1].W[0][0] = S.wsinv[p + 1];
  xpbd_update(1, C, alpha, &S.lam_sr[p], B, 2);
  S.s[p] += B[0].out[0];
  S.s[p + 1] += B[1].out[0];
  return 1;
}

// Surface bending at vertex p+1 (the energy of the Laplacian of the scale, Sec. 5): along the
// rod the Laplacian is the second difference of the pill scales over the vertex's Voronoi
// length l_v = (l0_p + l0_{p+1}) / 2; the rest scale is one everywhere, so its Laplacian is 0:
//   C = [(s_{p+2} - s_{p+1}) / l0_{p+1} - (s_{p+1} - s_p) / l0_p] / l_v
template <class R> int project_sb(Scene<R>& S, int p, R ih2) {
  if (!S.sb_on[S.rod_of[p]]) return 0;
  const R la = S.l0[p], lb = S.l0[p + 1], lv = R(0.5) * (la + lb);
  R C[1] = {((S.s[p + 2] - S.s[p + 1]) / lb - (S.s[p + 1] - S.s[p]) / la) / lv};
  R alpha[1] = {S.comp_sb[p] * ih2};
  Block<R> B[3];
  const R g0 = R(1.0) / (la * lv), g2 = R(1.0) / (lb * lv);
  B[0].ndof = 1; B[0].J[0][0] = g0; B[0].W[0][0] = S.wsinv[p];
  B[1].ndof = 1; B[1].J[0][0] = -(g0 + g2); B[1].W[0][0] = S.wsinv[p + 1];
  B[2].ndof = 1; B[2].J[0][0] = g2; B[2].W[0][0] = S.wsinv[p + 2];
  xpbd_update(1, C, alpha, &S.lam_sb[p], B, 3);
  S.s[p] += B[0].out[0];
  S.s[p + 1] += B[1].out[0];
  S.s[p + 2] += B[2].out[0];
  return 1;
}

// Bend-twist at vertex p+1, between edges p and p+1 (eq. bending_twist, Darboux of Sec. 7):
//   r = conj(q_p) (x) q_{p+1} (shortest arc), c = 4 / (l0_p + l0_{p+1})
//   C = s_{p+1} c Im(r) - Omega_rest
template <class R> int project_bt(Scene<R>& S, int p, R ih2) {
  const int k = S.rod_of[p];
  if (!S.enabled[4 * k + BT]) return 0;
  Q4<R> r = qmul(qconj(S.q[p]), S.q[p + 1]);
  if (r.w < R(0.0)) r = q4<R>(-r.x, -r.y, -r.z, -r.w);
  R c = R(4.0) / (S.l0[p] + S.l0[p + 1]);
  R sv = S.s[p + 1];
  V3<R> im = qim(r);
  V3<R> Om = (sv * c) * im;
  V3<R> Cv = Om - S.darb_rest[p];
  R C[3] = {Cv.x, Cv.y, Cv.z};
  R a = S.comp[BT][p] * ih2;
  R alpha[3] = {a, a, a * R(0.5)};   // compliance diag(1, 1, 1/2) in the material frame of edge p
  // d Im(r) / d theta_{p+1} = 1/2 (r_w I - [r_v]_x) R_p^T ; d/d theta_p = minus that.
  M3<R> Bm = mzero<R>();
  Bm.m[0][0] = Bm.m[1][1] = Bm.m[2][2] = r.w;
  M3<R> sk = skew(im);
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) Bm.m[i][j] -= sk.m[i][j];
  M3<R> Jp1 = mmul(Bm, mtrans(qmat(S.q[p])));
  R fac = R(0.5) * sv * c;
  Block<R> B[3];
  M3<R> W0 = inv_inertia_world(S, p), W1 = inv_inertia_world(S, p + 1);
  B[0].ndof = 3; B[1].ndof = 3;
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
    B[0].J[i][j] = -fac * Jp1.m[i][j]; B[0].W[i][j] = W0.m[i][j];
    B[1].J[i][j] = fac * Jp1.m[i][j];  B[1].W[i][j] = W1.m[i][j];
  }
  B[2].ndof = 1;
  B[2].J[0][0] = c * im.x; B[2].J[1][0] = c * im.y; B[2].J[2][0] = c * im.z;
  B[2].W[0][0] = S.wsinv[p + 1];
  xpbd_update(3, C, alpha, &S.lam[size_t(p) * 8 + 5], B, 3);
  S.q[p] = qrotate(S.q[p], v3<R>(B[0].out[0], B[0].out[1], B[0].out[2]));
  S.q[p + 1] = qrotate(S.q[p + 1], v3<R>(B[1].out[0], B[1].out[1], B[1].out[2]));
  S.s[p + 1] += B[2].out[0];
  return 1;
}

// Volume-bending coupling at vertex p+1 (the s^3 Omega^u, s^3 Omega^v terms of the volume
// energy, Sec. 5): the bending components of the bend-twist Darboux vector with the vertex scale
// cubed, against their rest values (rest scale one),
//   C = s_{p+1}^3 c Im(r)_{u,v} - Omega_rest_{u,v},   r, c as in bend-twist,
// with the volume stiffness k_v and the weight pi r^4 / 2 of the energy.
template <class R> int project_vb(Scene<R>& S, int p, R ih2) {
  const int k = S.rod_of[p];
  if (!S.vb_on || !S.enabled[4 * k + VOL]) return 0;
  Q4<R> r = qmul(qconj(S.q[p]), S.q[p + 1]);
  if (r.w < R(0.0)) r = q4<R>(-r.x, -r.y, -r.z, -r.w);
  const R c = R(4.0) / (S.l0[p] + S.l0[p + 1]);
  const R sv = S.s[p + 1], s3 = sv * sv * sv;
  const V3<R> im = qim(r);
  R C[2] = {s3 * c * im.x - S.darb_rest[p].x, s3 * c * im.y - S.darb_rest[p].y};
  const R a = S.comp_vb[p] * ih2;
  R alpha[2] = {a, a};
  // d Im(r) / d theta_{p+1} = 1/2 (r_w I - [r_v]_x) R_p^T ; d/d theta_p = minus that
  M3<R> Bm = mzero<R>();
  Bm.m[0][0] = Bm.m[1][1] = Bm.m[2][2] = r.w;
  M3<R> sk = skew(im);
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) Bm.m[i][j] -= sk.m[i][j];
  const M3<R> Jp1 = mmul(Bm, mtrans(qmat(S.q[p])));
  const R fac = R(0.5) * s3 * c;
  Block<R> B[3];
  const M3<R> W0 = inv_inertia_world(S, p), W1 = inv_inertia_world(S, p + 1);
  B[0].ndof = 3; B[1].ndof = 3;
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 3; ++j) {
    B[0].J[i][j] = -fac * Jp1.m[i][j];
    B[1].J[i][j] = fac * Jp1.m[i][j];
  }
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) { B[0].W[i][j] = W0.m[i][j]; B[1].W[i][j] = W1.m[i][j]; }
  B[2].ndof = 1;
  B[2].J[0][0] = R(3.0) * sv * sv * c * im.x; B[2].J[1][0] = R(3.0) * sv * sv * c * im.y;
  B[2].W[0][0] = S.wsinv[p + 1];
  xpbd_update(2, C, alpha, &S.lam_vb[2 * size_t(p)], B, 3);
  S.q[p] = qrotate(S.q[p], v3<R>(B[0].out[0], B[0].out[1], B[0].out[2]));
  S.q[p + 1] = qrotate(S.q[p + 1], v3<R>(B[1].out[0], B[1].out[1], B[1].out[2]));
  S.s[p + 1] += B[2].out[0];
  return 1;
}

// ------------------------------ contacts ------------------------------------

// Closed-form projection of a point onto a tapered capsule (App. D, corrected):
// returns the barycentric t of the sphere of the capsule closest (surface distance)
// to x.  Reading: p_s = c1 + e ((x - c1) . e); o = |x - p_s| tan(theta) unsquared;
// when |r1 - r2| >= l the capsule is its larger end sphere.
template <class R> R pill_project(const V3<R>& x, const V3<R>& c1, R r1, const V3<R>& c2, R r2) {
  V3<R> ax = c2 - c1;
  R l = norm(ax);
  if (!(l > R(0.0))) return R(0.0);
  V3<R> e = (R(1.0) / l) * ax;
  R sn = (r1 - r2) / l;
  if (sn >= R(1.0)) return R(0.0);
  if (sn <= R(-1.0)) return R(1.0);
  V3<R> rel = x - c1;
  R u = dot(rel, e);
  V3<R> perp = rel - u * e;
  R dp = norm(perp);
  R tn = sn / sqrt(R(1.0) - sn * sn);
  R t = (u - dp * tn) / l;
  return rmin(rmax(t, R(0.0)), R(1.0));
}

template <class R> V3<R> lerp3(const V3<R>& a, const V3<R>& b, R t) { return (R(1.0) - t) * a + t * b; }

// Objective of the scalar collision search (eq. collsearch).
template <class R> R coll_gap(const V3<R>& a1, R ra1, const V3<R>& a2, R ra2, const V3<R>& b1, R rb1, const V3<R>& b2, R rb2, R al) {
  V3<R> ca = lerp3(a1, a2, al);
  R ra = (R(1.0) - al) * ra1 + al * ra2;
  R be = pill_project(ca, b1, rb1, b2, rb2);
  V3<R> cb = lerp3(b1, b2, be);
  R rb = (R(1.0) - be) * rb1 + be * rb2;
  return norm(ca - cb) - ra - rb;
}

// Dichotomous search (Antoniou & Lu), fixed iteration count (10 in the engine, Sec. 7.2).
// Reading: bracket [0,1], probe offset delta = 1e-4, ties keep the upper part.
template <class R> R dichotomous(const V3<R>& a1, R ra1, const V3<R>& a2, R ra2, const V3<R>& b1, R rb1, const V3<R>& b2, R rb2, int iters, R delta) {
  R lo(0.0), hi(1.0);
  for (int i = 0; i < iters; ++i) {
    R m = R(0.5) * (lo + hi);
    R x1 = m - delta, x2 = m + delta;
    R g1 = coll_gap(a1, ra1, a2, ra2, b1, rb1, b2, rb2, x1);
    R g2 = coll_gap(a1, ra1, a2, ra2, b1, rb1, b2, rb2, x2);
    if (g1 < g2) hi = x2; else lo = x1;
  }
  return R(0.5) * (lo + hi);
}

// Candidate pair predicate on capsule bounding spheres, evaluated in FP64 with a
// fixed operation order and no contraction (this file is built -ffp-contract=off).
// Sphere: centre = edge midpoint, radius = half length + larger end radius.
struct Sphere { double mx, my, mz, R; };
inline Sphere capsule_sphere(const double* x, const double* s, const double* rbar, int p) {
  Sphere o;
  o.mx = 0.5 * (x[3 * p + 0] + x[3 * p + 3]);
  o.my = 0.5 * (x[3 * p + 1] + x[3 * p + 4]);
  o.mz = 0.5 * (x[3 * p + 2] + x[3 * p + 5]);
  double dx = x[3 * p + 3] - x[3 * p + 0];
  double dy = x[3 * p + 4] - x[3 * p + 1];
  double dz = x[3 * p + 5] - x[3 * p + 2];
  double len = std::sqrt((dx * dx + dy * dy) + dz * dz);
  double ra = s[p] * rbar[p];
  double rb = s[p + 1] * rbar[p + 1];
  o.R = 0.5 * len + ((ra < rb) ? rb : ra);
  return o;
}
inline bool spheres_overlap(const Sphere& a, const Sphere& b) {
  double dx = a.mx - b.mx, dy = a.my - b.my, dz = a.mz - b.mz;
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double rr = a.R + b.R;
  return d2 < rr * rr;
}

// Brute-force O(E^2) candidate set, sorted by (a, b), a < b; excludes same rod and same group.
// Reading: a capsule is the swept sphere of radius s r (Sec. 7); one whose end radius is not
// positive (a scale driven through zero) has no surface and takes no contact.
inline void brute_pairs(int nrods, const int* off, const int* group, const double* x, const double* s, const double* rbar, std::vector<int32_t>& out) {
  out.clear();
  int P = off[nrods];
  std::vector<int> rod_of(P);
  for (int k = 0; k < nrods; ++k) for (int p = off[k]; p < off[k + 1]; ++p) rod_of[p] = k;
  std::vector<int> caps;
  std::vector<Sphere> sph;
  for (int p = 0; p < P; ++p)
    if (p + 1 < off[rod_of[p] + 1] && s[p] > 0.0 && s[p + 1] > 0.0) {
      caps.push_back(p);
      sph.push_back(capsule_sphere(x, s, rbar, p));
    }
  for (size_t i = 0; i < caps.size(); ++i)
    for (size_t j = i + 1; j < caps.size(); ++j) {
      int a = caps[i], b = caps[j];
      if (rod_of[a] == rod_of[b] || group[rod_of[a]] == group[rod_of[b]]) continue;
      if (spheres_overlap(sph[i], sph[j])) { out.push_back(a); out.push_back(b); }
    }
}

template <class R> void detect(Scene<R>& S) {
  std::vector<double> xd(size_t(S.P) * 3), sdv(S.P), rd(S.P);
  for (int p = 0; p < S.P; ++p) { xd[3 * p] = val(S.x[p].x); xd[3 * p + 1] = val(S.x[p].y); xd[3 * p + 2] = val(S.x[p].z); sdv[p] = val(S.s[p]); rd[p] = val(S.rbar[p]); }
  brute_pairs(S.nrods, S.off.data(), S.group.data(), xd.data(), sdv.data(), rd.data(), S.pairs);
}

// Contact projection: every candidate pair is evaluated on the same pre-pass
// state (Jacobi, Sec. 7 engine), hard constraint
//   C = |c_a(a*) - c_b(b*)| - r_a(a*) - r_b(b*)   projected only when C < 0,
// corrections summed per DOF in sorted pair order and divided by the number of
// active contacts touching the DOF (averaging reduction).  a*, b* held fixed.
template <class R> void project_contacts(Scene<R>& S, int search_iters, double delta) {
  const int P = S.P;
  std::vector<V3<R>> dx(P, v3<R>(R(0.0), R(0.0), R(0.0)));
  std::vector<R> ds(P, R(0.0));
  std::vector<int> cnt(P, 0);
  const size_t np = S.pairs.size() / 2;
  for (size_t i = 0; i < np; ++i) {
    int a = S.pairs[2 * i], b = S.pairs[2 * i + 1];
    int pid[4] = {a, a + 1, b, b + 1};
    V3<R> c[4];
    R rad[4];
    for (int t = 0; t < 4; ++t) { c[t] = S.x[pid[t]]; rad[t] = S.s[pid[t]] * S.rbar[pid[t]]; }
    R al = dichotomous(c[0], rad[0], c[1], rad[1], c[2], rad[2], c[3], rad[3], search_iters, R(delta));
    V3<R> ca = lerp3(c[0], c[1], al);
    R be = pill_project(ca, c[2], rad[2], c[3], rad[3]);
    V3<R> cb = lerp3(c[2], c[3], be);
    V3<R> dv = ca - cb;
    R dist = norm(dv);
    R C = dist - ((R(1.0) - al) * rad[0] + al * rad[1]) - ((R(1.0) - be) * rad[2] + be * rad[3]);
    if (!(C < R(0.0))) continue;
    if (!(dist > R(0.0))) continue;
    V3<R> n = (R(1.0) / dist) * dv;
    R wts[4] = {R(1.0) - al, al, -(R(1.0) - be), -be};   // dC/dx_t = wts[t] n
    R den(0.0);
    for (int t = 0; t < 4; ++t) {
      R gs = -(wts[t] < R(0.0) ? -wts[t] : wts[t]) * S.rbar[pid[t]];  // dC/ds_t = -|wts| rbar
      den += S.winv[pid[t]] * wts[t] * wts[t] + S.wsinv[pid[t]] * gs * gs;
    }
    if (!(den > R(0.0))) continue;
    R dl = -C / den;
    for (int t = 0; t < 4; ++t) {
      R gs = -(wts[t] < R(0.0) ? -wts[t] : wts[t]) * S.rbar[pid[t]];
      dx[pid[t]] = dx[pid[t]] + (S.winv[pid[t]] * wts[t] * dl) * n;
      ds[pid[t]] += S.wsinv[pid[t]] * gs * dl;
      cnt[pid[t]] += 1;
    }
    S.projections++;
  }
  for (int p = 0; p < P; ++p) {
    S.active_count[p] = cnt[p];
    if (cnt[p] > 0) {
      R inv = R(1.0) / R(double(cnt[p]));
      S.x[p] = S.x[p] + inv * dx[p];
      S.s[p] += inv * ds[p];
    }
  }
}

// ------------------------------ substep -------------------------------------

// Rotational inertia of every edge for one substep (App. B, the m s^2 I term of the frame
// update): the body-frame tensor of edge p is  rho pi rbar^4 l0 * s^2 * diag(1/4, 1/4, 1/2),
// with s the midpoint scale at the START of the substep (held fixed through the substep).
// inert_base = rho pi rbar^4 l0; only the inverses are stored.
template <class R> void substep_inertia(Scene<R>& S, int r0, int r1) {
  for (int k = r0; k < r1; ++k)
    for (int p = S.off[k]; p + 1 < S.off[k + 1]; ++p) {
      R sm = R(0.5) * (S.sprev[p] + S.sprev[p + 1]);
      R I = S.inert_base[p] * sm * sm;
      S.I1inv[p] = R(4.0) / I;   // I1 = I/4
      S.I3inv[p] = R(2.0) / I;   // I3 = I/2
    }
}

// Prediction (Sec. 6 prediction step, App. B): under gravity the external
// torque and the scale counterpart vanish, so
//   c^ = c + h v + h^2 g,  s^ = s + h sdot,  theta^ = theta + h omega.
// Pinned vertices keep their position.
template <class R> void predict_rods(Scene<R>& S, R h, int r0, int r1) {
  for (int k = r0; k < r1; ++k)
    for (int p = S.off[k]; p < S.off[k + 1]; ++p) {
      S.xprev[p] = S.x[p];
      S.sprev[p] = S.s[p];
      if (S.winv[p] > R(0.0)) S.x[p] = S.x[p] + h * S.v[p] + (h * h) * S.g;
      S.s[p] = S.s[p] + h * S.sd[p];
      if (S.has_edge(p)) {
        S.qprev[p] = S.q[p];
        S.q[p] = qrotate(S.q[p], h * S.om[p]);
      }
      for (int t = 0; t < 8; ++t) S.lam[size_t(p) * 8 + t] = R(0.0);
      S.lam_sr[p] = R(0.0);
      S.lam_sb[p] = R(0.0);
      S.lam_vb[2 * size_t(p)] = S.lam_vb[2 * size_t(p) + 1] = R(0.0);
    }
  substep_inertia(S, r0, r1);
}

// One iteration of the four colour passes (reading: colours 0/1 = even/odd edges
// for stretch-shear, volume, scale gradient in that order; colours 2/3 = even/odd
// bend-twist).  Returns the number of projections.
template <class R> int64_t solve_colours(Scene<R>& S, R ih2, int r0, int r1) {
  int64_t n = 0;
  for (int colour = 0; colour < 2; ++colour)
    for (int k = r0; k < r1; ++k)
      for (int p = S.off[k] + colour; p + 1 < S.off[k + 1]; p += 2) {
        n += project_ss(S, p, ih2);
        n += project_vol(S, p, ih2);
        n += project_sg(S, p, ih2);
        n += project_sr(S, p, ih2);
      }
  for (int colour = 0; colour < 2; ++colour)
    for (int k = r0; k < r1; ++k)
      for (int p = S.off[k] + colour; p + 2 < S.off[k + 1]; p += 2) n += project_bt(S, p, ih2);
  // the volume-bending coupling at the same vertices, after every bend-twist projection
  for (int colour = 0; colour < 2; ++colour)
    for (int k = r0; k < r1; ++k)
      for (int p = S.off[k] + colour; p + 2 < S.off[k + 1]; p += 2) n += project_vb(S, p, ih2);
  // surface bending touches three consecutive scales: three colours
  for (int colour = 0; colour < 3; ++colour)
    for (int k = r0; k < r1; ++k)
      for (int p = S.off[k] + colour; p + 2 < S.off[k + 1]; p += 3) n += project_sb(S, p, ih2);
  return n;
}

// One all-Jacobi iteration with averaging (Sec. 7: constraints computed in parallel, their
// displacements averaged by a reduction).  Every rod constraint is projected from the state
// at the start of the iteration; each degree of freedom then moves by the mean of the
// corrections of the active constraints acting on it.  Readings: the count is the number of
// active constraints on the DOF; a rotation moves by the mean quaternion increment,
// q <- normalize(q + mean(q_c - q)); each constraint keeps its own multiplier update.
template <class R> int64_t solve_jacobi(Scene<R>& S, R ih2) {
  const int P = S.P;
  std::vector<V3<R>> dx(P, v3<R>(R(0.0), R(0.0), R(0.0)));
  std::vector<R> ds(P, R(0.0));
  std::vector<Q4<R>> dq(P, q4<R>(R(0.0), R(0.0), R(0.0), R(0.0)));
  std::vector<int> nx(P, 0), ns(P, 0), nq(P, 0);
  int64_t n = 0;
  // project constraint `kind` at p in place, record what it moved, restore the state
  auto eval = [&](int kind, int p) {
    const int q1 = p + 1;
    const V3<R> x0 = S.x[p], x1 = S.x[q1];
    const R s0 = S.s[p], s1 = S.s[q1];
    const R s2 = (kind == SB) ? S.s[p + 2] : R(0.0);
    const Q4<R> r0 = S.q[p], r1 = S.q[q1];
    int a = 0;
    if (kind == SS) a = project_ss(S, p, ih2);
    else if (kind == VOL) a = project_vol(S, p, ih2);
    else if (kind == SG) a = project_sg(S, p, ih2);
    else if (kind == SR) a = project_sr(S, p, ih2);
    else if (kind == SB) a = project_sb(S, p, ih2);
    else if (kind == VB) a = project_vb(S, p, ih2);
    else a = project_bt(S, p, ih2);
    if (!a) return;
    n += a;
    if (kind == SS || kind == VOL) {
      dx[p] = dx[p] + (S.x[p] - x0); dx[q1] = dx[q1] + (S.x[q1] - x1); ++nx[p]; ++nx[q1];
    }
    if (kind == VOL || kind == SG || kind == SR) {
      ds[p] = ds[p] + (S.s[p] - s0); ds[q1] = ds[q1] + (S.s[q1] - s1); ++ns[p]; ++ns[q1];
    }
    if (kind == BT || kind == VB) { ds[q1] = ds[q1] + (S.s[q1] - s1); ++ns[q1]; }
    if (kind == SB) {
      ds[p] = ds[p] + (S.s[p] - s0); ds[q1] = ds[q1] + (S.s[q1] - s1); ds[p + 2] = ds[p + 2] + (S.s[p + 2] - s2);
      ++ns[p]; ++ns[q1]; ++ns[p + 2];
      S.s[p + 2] = s2;
    }
    auto addq = [&](int i, const Q4<R>& before) {
      dq[i] = q4<R>(dq[i].x + (S.q[i].x - before.x), dq[i].y + (S.q[i].y - before.y), dq[i].z + (S.q[i].z - before.z),
                    dq[i].w + (S.q[i].w - before.w));
      ++nq[i];
    };
    if (kind == SS) addq(p, r0);
    if (kind == BT || kind == VB) { addq(p, r0); addq(q1, r1); }
    S.x[p] = x0; S.x[q1] = x1; S.s[p] = s0; S.s[q1] = s1; S.q[p] = r0; S.q[q1] = r1;
  };
  for (int k = 0; k < S.nrods; ++k)
    for (int p = S.off[k]; p + 1 < S.off[k + 1]; ++p) {
      eval(SS, p);
      eval(VOL, p);
      eval(SG, p);
      eval(SR, p);
      if (p + 2 < S.off[k + 1]) eval(BT, p);
      if (p + 2 < S.off[k + 1]) eval(SB, p);
      if (p + 2 < S.off[k + 1]) eval(VB, p);
    }
  for (int p = 0; p < P; ++p) {
    if (nx[p]) S.x[p] = S.x[p] + (R(1.0) / R(double(nx[p]))) * dx[p];
    if (ns[p]) S.s[p] = S.s[p] + ds[p] / R(double(ns[p]));
    if (nq[p]) {
      const R f = R(1.0) / R(double(nq[p]));
      S.q[p] = qnormalize(q4<R>(S.q[p].x + f * dq[p].x, S.q[p].y + f * dq[p].y, S.q[p].z + f * dq[p].z,
                                S.q[p].w + f * dq[p].w));
    }
  }
  return n;
}

// Velocity update (reading: first-order finite difference over the substep).
template <class R> void velocity_rods(Scene<R>& S, R h, int r0, int r1) {
  for (int k = r0; k < r1; ++k)
    for (int p = S.off[k]; p < S.off[k + 1]; ++p) {
      S.v[p] = (S.winv[p] > R(0.0)) ? (R(1.0) / h) * (S.x[p] - S.xprev[p]) : v3<R>(R(0.0), R(0.0), R(0.0));
      S.sd[p] = (S.s[p] - S.sprev[p]) / h;
      if (S.has_edge(p)) {
        Q4<R> r = qmul(S.q[p], qconj(S.qprev[p]));
        if (r.w < R(0.0)) r = q4<R>(-r.x, -r.y, -r.z, -r.w);
        S.om[p] = (R(2.0) / h) * qim(r);
      }
    }
}

// ---------------------------------------------------------------------------
// Half-plane floor (Sec. 7: the floor is a kinematic half-plane collision proxy).  For every
// pill the hard constraint C = n . x - d - s rbar >= 0 (its sphere above the plane) is
// projected on the position only: x += -C n (S = w |n|^2, dl = -C / S, dx = w n dl).
// Readings: the paper couples radii and positions for pill-pill contacts but calls the floor a
// simple half-plane constraint; with the scale DOF in the update its very small mass would
// take nearly the whole correction and shrink penetrating pills (to negative radii) instead of
// lifting them.  A pill's sphere suffices (the distance of a capsule to a plane minus its
// radius is linear along it, so its minimum is at a pill); pinned pills are not moved; the
// projection runs at the start of every iteration, after the previous contact pass.
// ---------------------------------------------------------------------------
template <class R> int64_t project_floor(Scene<R>& S) {
  int64_t n = 0;
  const R nx = R(S.floor_n.x), ny = R(S.floor_n.y), nz = R(S.floor_n.z), d = R(S.floor_d);
  for (int p = 0; p < S.P; ++p) {
    const R C = (nx * S.x[p].x + ny * S.x[p].y + nz * S.x[p].z) - d - S.s[p] * S.rbar[p];
    if (!(C < R(0.0)) || !(S.winv[p] > R(0.0))) continue;
    S.x[p] = S.x[p] + (-C) * v3<R>(nx, ny, nz);
    ++n;
  }
  return n;
}

// ---------------------------------------------------------------------------
// Scale-invariant shape matching of a muscle cross-section ("bundling", Sec. 7.3).
// Each pill i of a section carries a similarity transform T_i = [s_i R_i | x_i]; the
// section is fitted with one global similarity T* of its rest transforms (Umeyama),
// and then every T_i is set to T* Tbar_i.  Readings (the paper gives the energy and the
// fit, not where the step sits or what a rod's last pill contributes):
//   - the projection runs once per substep, after the constraint iterations and before
//     the velocity update; every section is fitted from the same state, then applied;
//   - R_i is the rotation of the edge that starts at pill i; the last pill of a rod
//     (no edge of its own) contributes the rotation of its incoming edge, and only its
//     position and scale are set;
//   - rest transforms: scale 1, rest frames qrest, rest positions;
//   - pinned pills keep their position (pins fix position only); scale and rotation
//     are set as for any pill;
//   - the optimal rotation is extracted with the iteration of Mueller et al. 2016,
//     started from the section's rotation of the previous substep (identity at first),
//     at most 20 steps, stopping when the update angle falls below 1e-9.
// ---------------------------------------------------------------------------
struct SectionFit { M3<double> R; Q4<double> q; double s; V3<double> c; };

inline M3<double> qmat_d(const Q4<double>& q) { return qmat(q); }

// Rotation that maximises trace(R^T A) (= argmin_R |R - A|_F over SO(3)), by the
// iteration of Mueller et al. 2016: rotate by the axis-angle vector
// sum_k r_k x a_k / (|sum_k r_k . a_k| + 1e-9) (r_k, a_k the columns of R and A).
inline Q4<double> extract_rotation(const M3<double>& A, Q4<double> q) {
  for (int it = 0; it < 20; ++it) {
    M3<double> Rm = qmat(q);
    V3<double> num = v3<double>(0, 0, 0);
    double den = 0;
    for (int k = 0; k < 3; ++k) {
      V3<double> r = v3<double>(Rm.m[0][k], Rm.m[1][k], Rm.m[2][k]);
      V3<double> a = v3<double>(A.m[0][k], A.m[1][k], A.m[2][k]);
      num = num + cross(r, a);
      den += dot(r, a);
    }
    V3<double> om = (1.0 / (std::fabs(den) + 1e-9)) * num;
    double w = norm(om);
    if (w < 1e-9) break;
    double sh = std::sin(0.5 * w) / w;
    q = qnormalize(qmul(q4<double>(sh * om.x, sh * om.y, sh * om.z, std::cos(0.5 * w)), q));
  }
  return q;
}

// The pill's transform: rotation of its edge, or of its incoming edge for a rod's last pill.
template <class R> int section_edge(const Scene<R>& S, int p) { return S.has_edge(p) ? p : p - 1; }

template <class R> SectionFit fit_section(const Scene<R>& S, int k) {
  const int i0 = S.sec_off[k], i1 = S.sec_off[k + 1];
  const double n = double(i1 - i0);
  V3<double> mu = v3<double>(0, 0, 0), mub = v3<double>(0, 0, 0);
  for (int i = i0; i < i1; ++i) {
    const int p = S.sec_pill[i];
    mu = mu + v3<double>(val(S.x[p].x), val(S.x[p].y), val(S.x[p].z));
    mub = mub + S.xrest[p];
  }
  mu = (1.0 / n) * mu;
  mub = (1.0 / n) * mub;
  // A = sum_i [s_i R_i | x_i - mu] [sbar_i Rbar_i | xbar_i - mubar]^T,
  // D = sum_i |[sbar_i Rbar_i | xbar_i - mubar]|_F^2
  M3<double> A = mzero<double>();
  double D = 0;
  for (int i = i0; i < i1; ++i) {
    const int p = S.sec_pill[i], e = section_edge(S, p);
    const Q4<double> qe = q4<double>(val(S.q[e].x), val(S.q[e].y), val(S.q[e].z), val(S.q[e].w));
    const Q4<double> qb = q4<double>(val(S.qrest[e].x), val(S.qrest[e].y), val(S.qrest[e].z), val(S.qrest[e].w));
    const M3<double> Ri = qmat(qe), Rb = qmat(qb);
    const double si = val(S.s[p]), sb = 1.0;
    const V3<double> d = v3<double>(val(S.x[p].x), val(S.x[p].y), val(S.x[p].z)) - mu;
    const V3<double> db = S.xrest[p] - mub;
    const double dv[3] = {d.x, d.y, d.z}, dbv[3] = {db.x, db.y, db.z};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = dv[r] * dbv[c];
        for (int t = 0; t < 3; ++t) acc += (si * Ri.m[r][t]) * (sb * Rb.m[c][t]);
        A.m[r][c] += acc;
      }
    D += 3.0 * sb * sb + dot(db, db);
  }
  SectionFit F;
  F.q = extract_rotation(A, S.sec_q[k]);
  F.R = qmat(F.q);
  // s* = sum_i <R* Bbar_i, B_i>_F / D  =  trace(R*^T A) / D
  double num = 0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) num += F.R.m[r][c] * A.m[r][c];
  F.s = num / D;
  F.c = mu - F.s * mvec(F.R, mub);
  return F;
}

template <class R> void bundle(Scene<R>& S) {
  const int ns = int(S.sec_off.size()) - 1;
  if (ns <= 0) return;
  std::vector<SectionFit> fits(ns);
  for (int k = 0; k < ns; ++k) fits[k] = fit_section(S, k);
  for (int k = 0; k < ns; ++k) {
    const SectionFit& F = fits[k];
    S.sec_q[k] = F.q;
    for (int i = S.sec_off[k]; i < S.sec_off[k + 1]; ++i) {
      const int p = S.sec_pill[i];
      if (S.winv[p] > R(0.0)) {
        const V3<double> y = F.s * mvec(F.R, S.xrest[p]) + F.c;
        S.x[p] = v3<R>(R(y.x), R(y.y), R(y.z));
      }
      S.s[p] = R(F.s * 1.0);
      if (S.has_edge(p)) {
        const Q4<double> qb = q4<double>(val(S.qrest[p].x), val(S.qrest[p].y), val(S.qrest[p].z), val(S.qrest[p].w));
        const Q4<double> qn = qnormalize(qmul(F.q, qb));
        S.q[p] = q4<R>(R(qn.x), R(qn.y), R(qn.z), R(qn.w));
      }
    }
  }
}

template <class R> void substep(Scene<R>& S, R h, int iters, bool collide, int search_iters, double delta, int threads) {
  R ih2 = R(1.0) / (h * h);
  if (!collide && threads > 1 && S.nrods > 1 && S.sec_off.size() < 2 && !S.floor_on && !S.jacobi) {
    int nt = std::min(threads, S.nrods);
    std::vector<std::thread> pool;
    std::vector<int64_t> proj(nt, 0);
    for (int t = 0; t < nt; ++t) {
      int r0 = int(int64_t(S.nrods) * t / nt), r1 = int(int64_t(S.nrods) * (t + 1) / nt);
      pool.emplace_back([&, r0, r1, t]() {
        predict_rods(S, h, r0, r1);
        for (int it = 0; it < iters; ++it) proj[t] += solve_colours(S, ih2, r0, r1);   // (Gauss-Seidel only)
        velocity_rods(S, h, r0, r1);
      });
    }
    for (auto& th : pool) th.join();
    for (int t = 0; t < nt; ++t) S.projections += proj[t];
    return;
  }
  predict_rods(S, h, 0, S.nrods);
  if (collide) detect(S);
  else S.pairs.clear();
  for (int it = 0; it < iters; ++it) {
    if (S.floor_on) S.projections += project_floor(S);
    S.projections += S.jacobi ? solve_jacobi(S, ih2) : solve_colours(S, ih2, 0, S.nrods);
    if (collide) project_contacts(S, search_iters, delta);
  }
  if constexpr (std::is_floating_point<R>::value) bundle(S);
  velocity_rods(S, h, 0, S.nrods);
}

// Sum of squared XPBD residuals |C + alpha~ lambda|^2 over all rod constraints,
// evaluated at the current state (used by the convergence property test).
template <class R> double rod_residual(const Scene<R>& S0, R ih2) {
  Scene<R> S = S0;   // evaluate without touching the state
  double acc = 0;
  for (int k = 0; k < S.nrods; ++k)
    for (int p = S.off[k]; p + 1 < S.off[k + 1]; ++p) {
      const R* L = &S.lam[size_t(p) * 8];
      if (S.enabled[4 * k + SS]) {
        V3<R> Cv = (R(1.0) / S.lbar[p]) * (S.x[p + 1] - S.x[p]) - qd3(S.q[p]);
        R a = S.comp[SS][p] * ih2;
        R c0 = Cv.x + a * L[0], c1 = Cv.y + a * L[1], c2 = Cv.z + a * L[2];
        acc += val(c0 * c0 + c1 * c1 + c2 * c2);
      }
      if (S.enabled[4 * k + VOL]) {
        R sm = R(0.5) * (S.s[p] + S.s[p + 1]);
        R C = sm * sm * norm(S.x[p + 1] - S.x[p]) / S.l0[p] - R(1.0) + S.comp[VOL][p] * ih2 * L[3];
        acc += val(C * C);
      }
      if (S.enabled[4 * k + SG]) {
        R C = (S.s[p + 1] - S.s[p]) / S.l0[p] + S.comp[SG][p] * ih2 * L[4];
        acc += val(C * C);
      }
      if (S.sr_on[k]) {
        R C = R(0.5) * (S.s[p] + S.s[p + 1]) - R(1.0) + S.comp_sr[p] * ih2 * S.lam_sr[p];
        acc += val(C * C);
      }
      if (p + 2 < S.off[k + 1] && S.vb_on && S.enabled[4 * k + VOL]) {
        Q4<R> r = qmul(qconj(S.q[p]), S.q[p + 1]);
        if (r.w < R(0.0)) r = q4<R>(-r.x, -r.y, -r.z, -r.w);
        const R c = R(4.0) / (S.l0[p] + S.l0[p + 1]), s3 = S.s[p + 1] * S.s[p + 1] * S.s[p + 1];
        const R a = S.comp_vb[p] * ih2;
        R c0 = s3 * c * r.x - S.darb_rest[p].x + a * S.lam_vb[2 * size_t(p)];
        R c1 = s3 * c * r.y - S.darb_rest[p].y + a * S.lam_vb[2 * size_t(p) + 1];
        acc += val(c0 * c0 + c1 * c1);
      }
      if (p + 2 < S.off[k + 1] && S.sb_on[k]) {
        const R la = S.l0[p], lb = S.l0[p + 1], lv = R(0.5) * (la + lb);
        R C = ((S.s[p + 2] - S.s[p + 1]) / lb - (S.s[p + 1] - S.s[p]) / la) / lv + S.comp_sb[p] * ih2 * S.lam_sb[p];
        acc += val(C * C);
      }
      if (p + 2 < S.off[k + 1] && S.enabled[4 * k + BT]) {
        Q4<R> r = qmul(qconj(S.q[p]), S.q[p + 1]);
        if (r.w < R(0.0)) r = q4<R>(-r.x, -r.y, -r.z, -r.w);
        R c = R(4.0) / (S.l0[p] + S.l0[p + 1]);
        V3<R> Cv = (S.s[p + 1] * c) * qim(r) - S.darb_rest[p];
        R a = S.comp[BT][p] * ih2;
        R c0 = Cv.x + a * L[5], c1 = Cv.y + a * L[6], c2 = Cv.z + R(0.5) * a * L[7];
        acc += val(c0 * c0 + c1 * c1 + c2 * c2);
      }
    }
  return acc;
}

// ------------------------------ skinning ------------------------------------

// Per-capsule similarity transform (Sec. 7.4, transform of eq. shapematch):
//   M = [ s R(q) R(q_rest)^T | m - s R(q) R(q_rest)^T m_rest ],  s, m = midpoint scale, centre.
template <class R> void capsule_transform(const Scene<R>& S, int p, double out[12]) {
  R sm = R(0.5) * (S.s[p] + S.s[p + 1]);
  V3<R> m = R(0.5) * (S.x[p] + S.x[p + 1]);
  V3<double> mr = 0.5 * (S.xrest[p] + S.xrest[p + 1]);
  M3<R> Rr = mmul(qmat(S.q[p]), mtrans(qmat(S.qrest[p])));
  for (int i = 0; i < 3; ++i) {
    R t = m.x; if (i == 1) t = m.y; if (i == 2) t = m.z;
    for (int j = 0; j < 3; ++j) {
      out[4 * i + j] = val(sm * Rr.m[i][j]);
    }
    R acc = t - sm * (Rr.m[i][0] * R(mr.x) + Rr.m[i][1] * R(mr.y) + Rr.m[i][2] * R(mr.z));
    out[4 * i + 3] = val(acc);
  }
}

}  // namespace orc

// =============================================================================
// C API (ctypes).  Opaque handles; precision 0 = float, 1 = double.
// =============================================================================
using namespace orc;

struct Handle {
  int prec;
  Scene<double>* d = nullptr;
  Scene<float>* f = nullptr;
};

template <class R> static void set_state_t(Scene<R>& S, const double* x, const double* v, const double* s, const double* sd, const double* q, const double* om) {
  for (int p = 0; p < S.P; ++p) {
    if (x) S.x[p] = v3<R>(R(x[3 * p]), R(x[3 * p + 1]), R(x[3 * p + 2]));
    if (v) S.v[p] = v3<R>(R(v[3 * p]), R(v[3 * p + 1]), R(v[3 * p + 2]));
    if (s) S.s[p] = R(s[p]);
    if (sd) S.sd[p] = R(sd[p]);
    if (q) S.q[p] = q4<R>(R(q[4 * p]), R(q[4 * p + 1]), R(q[4 * p + 2]), R(q[4 * p + 3]));
    if (om) S.om[p] = v3<R>(R(om[3 * p]), R(om[3 * p + 1]), R(om[3 * p + 2]));
  }
}
template <class R> static void get_state_t(const Scene<R>& S, double* x, double* v, double* s, double* sd, double* q, double* om) {
  for (int p = 0; p < S.P; ++p) {
    if (x) { x[3 * p] = val(S.x[p].x); x[3 * p + 1] = val(S.x[p].y); x[3 * p + 2] = val(S.x[p].z); }
    if (v) { v[3 * p] = val(S.v[p].x); v[3 * p + 1] = val(S.v[p].y); v[3 * p + 2] = val(S.v[p].z); }
    if (s) s[p] = val(S.s[p]);
    if (sd) sd[p] = val(S.sd[p]);
    if (q) { q[4 * p] = val(S.q[p].x); q[4 * p + 1] = val(S.q[p].y); q[4 * p + 2] = val(S.q[p].z); q[4 * p + 3] = val(S.q[p].w); }
    if (om) { om[3 * p] = val(S.om[p].x); om[3 * p + 1] = val(S.om[p].y); om[3 * p + 2] = val(S.om[p].z); }
  }
}

template <class R> static void set_sections_t(Scene<R>& S, int nsec, const int32_t* off, const int32_t* pill) {
  S.sec_off.assign(off, off + nsec + 1);
  S.sec_pill.assign(pill, pill + off[nsec]);
  S.sec_q.assign(nsec, q4<double>(0, 0, 0, 1));
}

// x -> A x + b for a bone transform T = [A | b] (3x4, row-major).
inline V3<double> affine_apply(const double* T, const V3<double>& x) {
  return v3<double>(T[0] * x.x + T[1] * x.y + T[2] * x.z + T[3], T[4] * x.x + T[5] * x.y + T[6] * x.z + T[7],
                    T[8] * x.x + T[9] * x.y + T[10] * x.z + T[11]);
}

// Inverse of T = [A | b]: [A^-1 | -A^-1 b], A^-1 by the adjugate over the determinant.
inline void affine_inverse(const double* T, double* out) {
  const double a = T[0], b = T[1], c = T[2], d = T[4], e = T[5], f = T[6], g = T[8], h = T[9], i = T[10];
  const double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
  const double adj[9] = {e * i - f * h, c * h - b * i, b * f - c * e,
                         f * g - d * i, a * i - c * g, c * d - a * f,
                         d * h - e * g, b * g - a * h, a * e - b * d};
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) out[4 * r + k] = adj[3 * r + k] / det;
    out[4 * r + 3] = -(out[4 * r] * T[3] + out[4 * r + 1] * T[7] + out[4 * r + 2] * T[11]);
  }
}

// Bone-driven warm start (Sec. 8.2): the bones moved from their last transforms T_prev to
// T_cur; every pill with influences moves to the weighted blend of its bones' motions,
//     x <- sum_k w_k T_cur,k T_prev,k^-1 x / sum_k w_k      (linear blend skinning)
// (pinned pills too: that is their kinematic attachment); pills without weight stay.
// Velocities, scales and rotations are not changed.  T_prev <- T_cur afterwards.
template <class R> void bone_warm_start(Scene<R>& S, const double* cur) {
  std::vector<double> inv(12 * (size_t)S.nbones);
  for (int b = 0; b < S.nbones; ++b) affine_inverse(&S.bone_prev[12 * (size_t)b], &inv[12 * (size_t)b]);
  for (int p = 0; p < S.P; ++p) {
    const V3<double> x = v3<double>(val(S.x[p].x), val(S.x[p].y), val(S.x[p].z));
    V3<double> acc = v3<double>(0, 0, 0);
    double wsum = 0.0;
    for (int k = 0; k < 2; ++k) {
      const double w = S.pill_bone_w[2 * (size_t)p + k];
      if (w <= 0.0) continue;
      const int b = S.pill_bone[2 * (size_t)p + k];
      const V3<double> y = affine_apply(&cur[12 * (size_t)b], affine_apply(&inv[12 * (size_t)b], x));
      acc = acc + w * y;
      wsum += w;
    }
    if (wsum > 0.0) {
      const V3<double> y = (1.0 / wsum) * acc;
      S.x[p] = v3<R>(R(y.x), R(y.y), R(y.z));
    }
  }
  S.bone_prev.assign(cur, cur + 12 * (size_t)S.nbones);
}

// Cross-section stretch compliance per rod (+inf: off); G = pi r^2 over the edge length, with
// r the edge's mean rest radius, as for SS and VOL.
template <class R> static void set_cross_stretch_t(Scene<R>& S, const double* comp) {
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < S.nrods; ++k) {
    S.sr_on[k] = std::isfinite(comp[k]) ? 1 : 0;
    for (int p = S.off[k]; p + 1 < S.off[k + 1]; ++p) {
      const R rm = R(0.5) * (S.rbar[p] + S.rbar[p + 1]);
      S.comp_sr[p] = S.sr_on[k] ? R(comp[k]) / (R(pi) * rm * rm * S.l0[p]) : R(0.0);
    }
  }
}

// Surface-bending compliance per rod (+inf: off); G = pi r^4 / 4 over the Voronoi length,
// r the vertex's rest radius, as for bend-twist.
template <class R> static void set_surface_bending_t(Scene<R>& S, const double* comp) {
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < S.nrods; ++k) {
    S.sb_on[k] = std::isfinite(comp[k]) ? 1 : 0;
    for (int p = S.off[k]; p + 2 < S.off[k + 1]; ++p) {
      const R rv = S.rbar[p + 1], lv = R(0.5) * (S.l0[p] + S.l0[p + 1]);
      S.comp_sb[p] = S.sb_on[k] ? R(comp[k]) / (R(pi) * rv * rv * rv * rv / R(4.0) * lv) : R(0.0);
    }
  }
}

// Volume-bending coupling on (on rods with the volume constraint): compliance = the rod's volume
// compliance over G l_v with G = pi r^4 / 2 and r the vertex's rest radius.
template <class R> static void set_volume_bending_t(Scene<R>& S, int on) {
  const double pi = 3.14159265358979323846;
  S.vb_on = on != 0;
  for (int k = 0; k < S.nrods; ++k)
    for (int p = S.off[k]; p + 2 < S.off[k + 1]; ++p) {
      const R rv = S.rbar[p + 1], lv = R(0.5) * (S.l0[p] + S.l0[p + 1]);
      S.comp_vb[p] = S.enabled[4 * k + VOL] ? R(S.alpha_vol[k]) / (R(pi) * rv * rv * rv * rv / R(2.0) * lv) : R(0.0);
    }
}

template <class R> static void set_floor_t(Scene<R>& S, const double* n, double d) {
  const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  S.floor_on = true;
  S.floor_n = v3<double>(n[0] / l, n[1] / l, n[2] / l);
  S.floor_d = d / l;
}

// `iters` rod-constraint iterations (no prediction, no contacts) at the current state, from
// zero multipliers and the inertias of the current scales (as orc_project_one).
template <class R> static int64_t rod_iterations_t(Scene<R>& S, double h_sub, int iters) {
  for (int i = 0; i < S.P; ++i) S.sprev[i] = S.s[i];
  substep_inertia(S, 0, S.nrods);
  for (int i = 0; i < S.P; ++i) {
    for (int t = 0; t < 8; ++t) S.lam[size_t(i) * 8 + t] = R(0.0);
    S.lam_sr[i] = R(0.0);
    S.lam_sb[i] = R(0.0);
    S.lam_vb[2 * size_t(i)] = S.lam_vb[2 * size_t(i) + 1] = R(0.0);
  }
  const R ih2 = R(1.0 / (h_sub * h_sub));
  int64_t n = 0;
  for (int it = 0; it < iters; ++it) n += S.jacobi ? solve_jacobi(S, ih2) : solve_colours(S, ih2, 0, S.nrods);
  return n;
}
static Desc make_desc(int num_rods, const int32_t* off, const double* rest_pos, const double* rest_radius, const uint8_t* pinned,
                      const double* activation, const double* compliance, const int32_t* group, double density, const double* gravity) {
  Desc d;
  d.num_rods = num_rods; d.rod_offsets = off; d.rest_pos = rest_pos; d.rest_radius = rest_radius; d.pinned = pinned;
  d.activation = activation; d.compliance = compliance; d.group = group; d.density = density;
  d.gravity[0] = gravity[0]; d.gravity[1] = gravity[1]; d.gravity[2] = gravity[2];
  return d;
}

extern "C" {

void* orc_create(int precision, int num_rods, const int32_t* off, const double* rest_pos, const double* rest_radius,
                 const uint8_t* pinned, const double* activation, const double* compliance, const int32_t* group,
                 double density, const double* gravity) {
  Desc d = make_desc(num_rods, off, rest_pos, rest_radius, pinned, activation, compliance, group, density, gravity);
  Handle* h = new Handle();
  h->prec = precision;
  int P = off[num_rods];
  if (precision == 1) {
    h->d = new Scene<double>();
    build(*h->d, d, rest_radius, activation);
  } else {
    h->f = new Scene<float>();
    std::vector<float> rb(rest_radius, rest_radius + P), ac(activation, activation + num_rods);
    build(*h->f, d, rb.data(), ac.data());
  }
  return h;
}

void orc_destroy(void* hp) {
  Handle* h = (Handle*)hp;
  delete h->d; delete h->f; delete h;
}

void orc_set_state(void* hp, const double* x, const double* v, const double* s, const double* sd, const double* q, const double* om) {
  Handle* h = (Handle*)hp;
  if (h->d) set_state_t(*h->d, x, v, s, sd, q, om); else set_state_t(*h->f, x, v, s, sd, q, om);
}

void orc_get_state(void* hp, double* x, double* v, double* s, double* sd, double* q, double* om) {
  Handle* h = (Handle*)hp;
  if (h->d) get_state_t(*h->d, x, v, s, sd, q, om); else get_state_t(*h->f, x, v, s, sd, q, om);
}

// Bundling cross-sections (Sec. 7.3): nsec sections, section k = pills sec_pill[sec_off[k]..sec_off[k+1]).
void orc_set_sections(void* hp, int nsec, const int32_t* off, const int32_t* pill) {
  Handle* h = (Handle*)hp;
  if (h->d) set_sections_t(*h->d, nsec, off, pill); else set_sections_t(*h->f, nsec, off, pill);
}
// The fit of section k at the current state: R* (row-major 9), s*, c* (3), q* (4).
void orc_section_fit(void* hp, int k, double* out) {
  Handle* h = (Handle*)hp;
  SectionFit F = h->d ? fit_section(*h->d, k) : fit_section(*h->f, k);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) out[3 * r + c] = F.R.m[r][c];
  out[9] = F.s; out[10] = F.c.x; out[11] = F.c.y; out[12] = F.c.z;
  out[13] = F.q.x; out[14] = F.q.y; out[15] = F.q.z; out[16] = F.q.w;
}
// Half-plane floor n . x >= d (n normalised here); one projection pass at the current state.
void orc_set_floor(void* hp, const double* n, double d) {
  Handle* h = (Handle*)hp;
  if (h->d) set_floor_t(*h->d, n, d); else set_floor_t(*h->f, n, d);
}
// Bones (Sec. 8.2): nb rest transforms [nb*12] (3x4 row-major, the bones' pose at the rest
// positions) and two (bone, weight) influences per pill, [P*2] each.
void orc_set_bones(void* hp, int nb, const double* rest, const int32_t* pb, const double* pw) {
  Handle* h = (Handle*)hp;
  auto set = [&](auto& S) {
    S.nbones = nb;
    S.bone_prev.assign(rest, rest + 12 * (size_t)nb);
    S.pill_bone.assign(pb, pb + 2 * (size_t)S.P);
    S.pill_bone_w.assign(pw, pw + 2 * (size_t)S.P);
  };
  if (h->d) set(*h->d); else set(*h->f);
}
// The bones' transforms of the new frame, [nb*12]: warm start of every influenced pill.
void orc_bone_frame(void* hp, const double* cur) {
  Handle* h = (Handle*)hp;
  if (h->d) bone_warm_start(*h->d, cur); else bone_warm_start(*h->f, cur);
}
// Cross-section stretch (eq. stretch_xy) compliance per rod, [nrods]; +inf leaves it off.
void orc_set_cross_stretch(void* hp, const double* comp) {
  Handle* h = (Handle*)hp;
  if (h->d) set_cross_stretch_t(*h->d, comp); else set_cross_stretch_t(*h->f, comp);
}
// Surface-bending compliance per rod, [nrods]; +inf leaves it off.
void orc_set_surface_bending(void* hp, const double* comp) {
  Handle* h = (Handle*)hp;
  if (h->d) set_surface_bending_t(*h->d, comp); else set_surface_bending_t(*h->f, comp);
}
// Volume-bending coupling: nonzero turns it on for every rod with the volume constraint.
void orc_set_volume_bending(void* hp, int on) {
  Handle* h = (Handle*)hp;
  if (h->d) set_volume_bending_t(*h->d, on); else set_volume_bending_t(*h->f, on);
}
// Solver of the rod constraints: 0 = coloured Gauss-Seidel, 1 = Jacobi with averaging.
void orc_set_solver(void* hp, int jacobi) {
  Handle* h = (Handle*)hp;
  if (h->d) h->d->jacobi = jacobi != 0; else h->f->jacobi = jacobi != 0;
}
int64_t orc_rod_iteration(void* hp, double h_sub, int iters) {
  Handle* h = (Handle*)hp;
  return h->d ? rod_iterations_t(*h->d, h_sub, iters) : rod_iterations_t(*h->f, h_sub, iters);
}
void orc_floor_pass(void* hp) {
  Handle* h = (Handle*)hp;
  if (h->d) project_floor(*h->d); else project_floor(*h->f);
}
// One bundling projection of every section at the current state.
void orc_bundle(void* hp) {
  Handle* h = (Handle*)hp;
  if (h->d) bundle(*h->d); else bundle(*h->f);
}
// Rotation extraction alone (A row-major, q0 = start quaternion x y z w): q out.
void orc_extract_rotation(const double* A, const double* q0, double* q) {
  M3<double> M;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M.m[r][c] = A[3 * r + c];
  Q4<double> o = extract_rotation(M, q4<double>(q0[0], q0[1], q0[2], q0[3]));
  q[0] = o.x; q[1] = o.y; q[2] = o.z; q[3] = o.w;
}

// One frame = `substeps` substeps of h = dt / substeps.  Returns projections performed.
int64_t orc_step(void* hp, double dt, int substeps, int iters, int collide, int search_iters, double delta, int threads) {
  Handle* h = (Handle*)hp;
  if (h->d) {
    Scene<double>& S = *h->d;
    int64_t p0 = S.projections;
    double hh = dt / substeps;
    for (int i = 0; i < substeps; ++i) substep(S, hh, iters, collide != 0, search_iters, delta, threads);
    return S.projections - p0;
  }
  Scene<float>& S = *h->f;
  int64_t p0 = S.projections;
  float hh = float(dt / substeps);
  for (int i = 0; i < substeps; ++i) substep(S, hh, iters, collide != 0, search_iters, delta, threads);
  return S.projections - p0;
}

// Rest data export (for pins): l0, lbar, qrest[4], darboux_rest[3], winv, wsinv, inert_base, comp[4] per slot.
void orc_get_rest(void* hp, double* l0, double* lbar, double* qrest, double* darb, double* winv, double* wsinv, double* inert, double* comp) {
  Handle* h = (Handle*)hp;
  Scene<double>& S = *h->d;
  for (int p = 0; p < S.P; ++p) {
    l0[p] = S.l0[p]; lbar[p] = S.lbar[p];
    qrest[4 * p] = S.qrest[p].x; qrest[4 * p + 1] = S.qrest[p].y; qrest[4 * p + 2] = S.qrest[p].z; qrest[4 * p + 3] = S.qrest[p].w;
    darb[3 * p] = S.darb_rest[p].x; darb[3 * p + 1] = S.darb_rest[p].y; darb[3 * p + 2] = S.darb_rest[p].z;
    winv[p] = S.winv[p]; wsinv[p] = S.wsinv[p]; inert[p] = S.inert_base[p];
    for (int t = 0; t < 4; ++t) comp[4 * p + t] = S.comp[t][p];
  }
}

// Single-constraint primitives for closed-form pins (double scene only).
// kind: 0 SS, 1 VOL, 2 SG, 3 BT, 4 SR, 5 SB, 6 VB at slot p, with the substep inertia computed from
// the current scale.  lambda is zeroed first.
void orc_project_one(void* hp, int kind, int p, double h) {
  Handle* hd = (Handle*)hp;
  Scene<double>& S = *hd->d;
  for (int i = 0; i < S.P; ++i) S.sprev[i] = S.s[i];
  substep_inertia(S, 0, S.nrods);     // the routine every substep's prediction uses
  for (int i = 0; i < S.P; ++i) {
    for (int t = 0; t < 8; ++t) S.lam[size_t(i) * 8 + t] = 0.0;
    S.lam_sr[i] = 0.0;
    S.lam_sb[i] = 0.0;
    S.lam_vb[2 * size_t(i)] = S.lam_vb[2 * size_t(i) + 1] = 0.0;
  }
  double ih2 = 1.0 / (h * h);
  if (kind == 0) project_ss(S, p, ih2);
  if (kind == 1) project_vol(S, p, ih2);
  if (kind == 4) project_sr(S, p, ih2);
  if (kind == 5) project_sb(S, p, ih2);
  if (kind == 6) project_vb(S, p, ih2);
  if (kind == 2) project_sg(S, p, ih2);
  if (kind == 3) project_bt(S, p, ih2);
}

// Pin hooks (double scene): override inverse masses / inertia bases (nullptr keeps).
void orc_set_masses(void* hp, const double* winv, const double* wsinv, const double* inert) {
  Handle* hd = (Handle*)hp;
  Scene<double>& S = *hd->d;
  for (int p = 0; p < S.P; ++p) {
    if (winv) S.winv[p] = winv[p];
    if (wsinv) S.wsinv[p] = wsinv[p];
    if (inert) S.inert_base[p] = inert[p];
  }
}

// Pin hook: detection on the current state followed by one contact pass.
void orc_contact_pass(void* hp, int search_iters, double delta) {
  Handle* hd = (Handle*)hp;
  Scene<double>& S = *hd->d;
  detect(S);
  project_contacts(S, search_iters, delta);
}

// One substep reporting the rod residual after every iteration (double scene).
void orc_substep_residuals(void* hp, double h, int iters, double* out) {
  Handle* hd = (Handle*)hp;
  Scene<double>& S = *hd->d;
  double ih2 = 1.0 / (h * h);
  predict_rods(S, h, 0, S.nrods);
  for (int it = 0; it < iters; ++it) {
    if (S.jacobi) solve_jacobi(S, ih2); else solve_colours(S, ih2, 0, S.nrods);
    out[it] = rod_residual(S, ih2);
  }
  velocity_rods(S, h, 0, S.nrods);
}

int orc_num_pairs(void* hp) { Handle* h = (Handle*)hp; return h->d ? int(h->d->pairs.size() / 2) : int(h->f->pairs.size() / 2); }
void orc_get_pairs(void* hp, int32_t* out) {
  Handle* h = (Handle*)hp;
  const std::vector<int32_t>& v = h->d ? h->d->pairs : h->f->pairs;
  std::memcpy(out, v.data(), v.size() * sizeof(int32_t));
}
void orc_get_active_count(void* hp, int32_t* out) {
  Handle* h = (Handle*)hp;
  const std::vector<int>& v = h->d ? h->d->active_count : h->f->active_count;
  for (size_t i = 0; i < v.size(); ++i) out[i] = v[i];
}

// Brute-force candidate pairs from explicit FP64 values; returns the count and
// writes up to cap pairs.
int orc_brute_pairs(int num_rods, const int32_t* off, const int32_t* group, const double* x, const double* s, const double* rbar, int32_t* out, int cap) {
  std::vector<int32_t> v;
  brute_pairs(num_rods, off, group, x, s, rbar, v);
  int n = int(v.size() / 2);
  for (int i = 0; i < std::min(n, cap) * 2; ++i) out[i] = v[i];
  return n;
}

// Skinning weights (Sec. 7.4): each vertex's initial weights are proportional to the inverse
// square distance from the vertex to the surface of each capsule (rest pose).  Readings: the
// distance is |v - c(t)| - r(t) at the capsule's closest sphere t (App. D projection), clamped
// below at 1e-9 m (a vertex inside a capsule); the four largest weights are kept and
// normalised to sum 1 (4-influence LBS); the paper's fairing over the mesh is not applied
// (it needs the mesh connectivity).  Ties keep the lower capsule id.  Outputs the capsule
// ids (first pill of each capsule) and weights, 4 per vertex, strongest first.
void orc_skin_weights(void* hp, int V, const double* v, int32_t* caps, double* w) {
  Handle* h = (Handle*)hp;
  Scene<double>& S = *h->d;
  std::vector<int> cap;
  for (int k = 0; k < S.nrods; ++k)
    for (int p = S.off[k]; p + 1 < S.off[k + 1]; ++p) cap.push_back(p);
  for (int i = 0; i < V; ++i) {
    const V3<double> x = v3(v[3 * i], v[3 * i + 1], v[3 * i + 2]);
    int best[4] = {-1, -1, -1, -1};
    double bw[4] = {-1.0, -1.0, -1.0, -1.0};
    for (int e : cap) {
      const V3<double> c1 = S.xrest[e], c2 = S.xrest[e + 1];
      const double r1 = S.rbar[e], r2 = S.rbar[e + 1];
      const double t = pill_project(x, c1, r1, c2, r2);
      const V3<double> c = c1 + t * (c2 - c1);
      const double r = r1 + t * (r2 - r1);
      const double d = std::max(norm(x - c) - r, 1e-9);
      const double wt = 1.0 / (d * d);
      // insert into the strongest four (strictly greater moves ahead: ties keep the lower id)
      for (int k = 0; k < 4; ++k)
        if (wt > bw[k]) {
          for (int m = 3; m > k; --m) { bw[m] = bw[m - 1]; best[m] = best[m - 1]; }
          bw[k] = wt; best[k] = e;
          break;
        }
    }
    double sum = 0.0;
    for (int k = 0; k < 4; ++k) if (best[k] >= 0) sum += bw[k];
    for (int k = 0; k < 4; ++k) {
      caps[4 * i + k] = best[k] >= 0 ? best[k] : best[0];
      w[4 * i + k] = best[k] >= 0 ? bw[k] / sum : 0.0;
    }
  }
}

// Fairing of the initial skinning weights over the mesh (Sec. 7.4: the weights start from the
// inverse-square assignment and are then faired over the surface, following the
// Sphere-Meshes skinning the paper builds on; the paper gives no steps).  Readings:
//  - every vertex keeps a list of at most kFairK = 8 (capsule, weight) entries: initially its
//    8 strongest inverse-square weights (as above, ties keep the lower id), normalised to sum 1;
//  - the mesh graph: the undirected edges of the triangles, each vertex's neighbours in
//    ascending index, no repeats;
//  - one fairing iteration (Jacobi, every vertex from the previous lists) is the Laplacian
//    smoothing step w <- (1 - lambda) w(v) + lambda * mean over neighbours u of w(u), on the
//    sparse lists: a vertex's own entries (scaled by 1 - lambda) in list order, then each
//    neighbour's entries (scaled by lambda / degree) in neighbour order, each added into the
//    entry of its capsule (a new capsule is appended); the 8 largest are kept (ties keep the
//    lower id), ordered largest first, and divided by their sum (summed in that order);
//  - after the iterations the 4 largest are kept and normalised the same way (fewer than 4
//    capsules: the remaining slots repeat the first capsule with weight 0).
// With at most 8 capsules in reach nothing is truncated and this is exactly linear Laplacian
// smoothing of the weight field.
constexpr int kFairK = 8;
struct FairList {
  int n = 0;
  int id[kFairK];
  double w[kFairK];
};

// Keep the `keep` largest of (id, w) (ties: lower id first), ordered, normalised in that order.
inline void fair_select(const std::vector<std::pair<int, double>>& acc, int keep, FairList& out) {
  std::vector<std::pair<int, double>> e(acc);
  std::sort(e.begin(), e.end(), [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
    return a.second > b.second || (a.second == b.second && a.first < b.first);
  });
  out.n = std::min<int>(keep, int(e.size()));
  double sum = 0.0;
  for (int k = 0; k < out.n; ++k) sum += e[k].second;
  for (int k = 0; k < out.n; ++k) { out.id[k] = e[k].first; out.w[k] = e[k].second / sum; }
}

void orc_skin_weights_faired(void* hp, int V, const double* v, int nf, const int32_t* tris, int iters, double lam,
                             int32_t* caps, double* w) {
  Handle* h = (Handle*)hp;
  Scene<double>& S = *h->d;
  std::vector<int> cap;
  for (int k = 0; k < S.nrods; ++k)
    for (int p = S.off[k]; p + 1 < S.off[k + 1]; ++p) cap.push_back(p);
  // initial lists: inverse-square distance to each capsule surface (as orc_skin_weights)
  std::vector<FairList> cur(V), nxt(V);
  for (int i = 0; i < V; ++i) {
    const V3<double> x = v3(v[3 * i], v[3 * i + 1], v[3 * i + 2]);
    std::vector<std::pair<int, double>> all;
    for (int e : cap) {
      const V3<double> c1 = S.xrest[e], c2 = S.xrest[e + 1];
      const double r1 = S.rbar[e], r2 = S.rbar[e + 1];
      const double t = pill_project(x, c1, r1, c2, r2);
      const V3<double> c = c1 + t * (c2 - c1);
      const double r = r1 + t * (r2 - r1);
      const double d = std::max(norm(x - c) - r, 1e-9);
      all.push_back({e, 1.0 / (d * d)});
    }
    fair_select(all, kFairK, cur[i]);
  }
  // mesh graph
  std::vector<std::vector<int>> nb(V);
  for (int f = 0; f < nf; ++f)
    for (int a = 0; a < 3; ++a) {
      const int p = tris[3 * f + a], q = tris[3 * f + (a + 1) % 3];
      if (p == q) continue;
      nb[p].push_back(q);
      nb[q].push_back(p);
    }
  for (auto& n : nb) {
    std::sort(n.begin(), n.end());
    n.erase(std::unique(n.begin(), n.end()), n.end());
  }
  for (int it = 0; it < iters; ++it) {
    for (int i = 0; i < V; ++i) {
      std::vector<std::pair<int, double>> acc;
      auto add = [&](int id, double x) {
        for (auto& a : acc)
          if (a.first == id) { a.second += x; return; }
        acc.push_back({id, x});
      };
      const double self = 1.0 - lam;
      for (int k = 0; k < cur[i].n; ++k) add(cur[i].id[k], self * cur[i].w[k]);
      if (!nb[i].empty()) {
        const double c = lam / double(nb[i].size());
        for (int u : nb[i])
          for (int k = 0; k < cur[u].n; ++k) add(cur[u].id[k], c * cur[u].w[k]);
      }
      fair_select(acc, kFairK, nxt[i]);
    }
    std::swap(cur, nxt);
  }
  for (int i = 0; i < V; ++i) {
    std::vector<std::pair<int, double>> acc;
    for (int k = 0; k < cur[i].n; ++k) acc.push_back({cur[i].id[k], cur[i].w[k]});
    FairList out;
    fair_select(acc, 4, out);
    for (int k = 0; k < 4; ++k) {
      caps[4 * i + k] = k < out.n ? out.id[k] : out.id[0];
      w[4 * i + k] = k < out.n ? out.w[k] : 0.0;
    }
  }
}

double orc_pill_project(const double* x, const double* c1, double r1, const double* c2, double r2) {
  return pill_project(v3(x[0], x[1], x[2]), v3(c1[0], c1[1], c1[2]), r1, v3(c2[0], c2[1], c2[2]), r2);
}
double orc_coll_gap(const double* a1, double ra1, const double* a2, double ra2, const double* b1, double rb1, const double* b2, double rb2, double al) {
  return coll_gap(v3(a1[0], a1[1], a1[2]), ra1, v3(a2[0], a2[1], a2[2]), ra2, v3(b1[0], b1[1], b1[2]), rb1, v3(b2[0], b2[1], b2[2]), rb2, al);
}
double orc_dichotomous(const double* a1, double ra1, const double* a2, double ra2, const double* b1, double rb1, const double* b2, double rb2, int iters, double delta) {
  return dichotomous(v3(a1[0], a1[1], a1[2]), ra1, v3(a2[0], a2[1], a2[2]), ra2, v3(b1[0], b1[1], b1[2]), rb1, v3(b2[0], b2[1], b2[2]), rb2, iters, delta);
}

// Skinning: per-capsule transforms of the current state, then linear blend of
// V rest vertices with 4 (capsule, weight) influences each.
void orc_skin(void* hp, int V, const double* rest_v, const int32_t* caps, const double* w, double* out) {
  Handle* h = (Handle*)hp;
  int P = h->d ? h->d->P : h->f->P;
  std::vector<double> T(size_t(P) * 12, 0.0);
  for (int p = 0; p < P; ++p) {
    if (h->d ? h->d->has_edge(p) : h->f->has_edge(p)) {
      if (h->d) capsule_transform(*h->d, p, &T[size_t(p) * 12]);
      else capsule_transform(*h->f, p, &T[size_t(p) * 12]);
    }
  }
  for (int i = 0; i < V; ++i) {
    double o[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k) {
      const double* M = &T[size_t(caps[4 * i + k]) * 12];
      double wk = w[4 * i + k];
      for (int r = 0; r < 3; ++r) o[r] += wk * (M[4 * r] * rest_v[3 * i] + M[4 * r + 1] * rest_v[3 * i + 1] + M[4 * r + 2] * rest_v[3 * i + 2] + M[4 * r + 3]);
    }
    out[3 * i] = o[0]; out[3 * i + 1] = o[1]; out[3 * i + 2] = o[2];
  }
}

void orc_capsule_transforms(void* hp, double* out) {
  Handle* h = (Handle*)hp;
  int P = h->d ? h->d->P : h->f->P;
  for (int p = 0; p < P; ++p) {
    for (int i = 0; i < 12; ++i) out[size_t(p) * 12 + i] = 0.0;
    if (h->d ? h->d->has_edge(p) : h->f->has_edge(p)) {
      if (h->d) capsule_transform(*h->d, p, &out[size_t(p) * 12]);
      else capsule_transform(*h->f, p, &out[size_t(p) * 12]);
    }
  }
}

// ----------------------------------------------------------------------------
// Gradient oracle.  Loss L = sum_k |x_{last pill of rod k} - target_k|^2 after
// `frames` frames from rest, collision-free.  Rods are independent, so each
// rod is simulated alone with dual numbers seeded on chunks of its parameters
// (its rest radii, then its activation).  Exact FP64 derivatives of the
// discrete algorithm.
// ----------------------------------------------------------------------------
static const int KD = 8;

}  // extern "C"

// B = double: exact FP64 derivatives; B = float: the same derivatives in FP32 arithmetic.
template <class B>
static double grad_impl(int num_rods, const int32_t* off, const double* rest_pos, const double* rest_radius,
                        const uint8_t* pinned, const double* activation, const double* compliance, const int32_t* group,
                        double density, const double* gravity, double dt, int substeps, int iters, int frames,
                        const double* targets, double* d_rbar, double* d_act, int threads) {
  typedef Dual<KD, B> DN;
  std::vector<double> loss_k(num_rods, 0.0);
  auto work = [&](int k0, int k1) {
    for (int k = k0; k < k1; ++k) {
      int a = off[k], b = off[k + 1], N = b - a;
      int32_t loff[2] = {0, N};
      Desc d = make_desc(1, loff, rest_pos + 3 * a, rest_radius + a, pinned + a, activation + k, compliance + 4 * k, group + k, density, gravity);
      int nparam = N + 1;
      for (int c0 = 0; c0 < nparam; c0 += KD) {
        std::vector<DN> rb(N), ac(1);
        for (int i = 0; i < N; ++i) { rb[i] = DN(rest_radius[a + i]); if (i >= c0 && i < c0 + KD) rb[i].d[i - c0] = 1; }
        ac[0] = DN(activation[k]);
        if (N >= c0 && N < c0 + KD) ac[0].d[N - c0] = 1;
        Scene<DN> S;
        build(S, d, rb.data(), ac.data());
        DN hh(dt / substeps);
        for (int f = 0; f < frames; ++f)
          for (int i = 0; i < substeps; ++i) substep(S, hh, iters, false, 10, 1e-4, 1);
        V3<DN> e = S.x[N - 1] - v3<DN>(DN(targets[3 * k]), DN(targets[3 * k + 1]), DN(targets[3 * k + 2]));
        DN L = dot(e, e);
        loss_k[k] = L.v;
        for (int j = 0; j < KD; ++j) {
          int pi = c0 + j;
          if (pi < N) d_rbar[a + pi] = L.d[j];
          else if (pi == N) d_act[k] = L.d[j];
        }
      }
    }
  };
  int nt = std::max(1, std::min(threads, num_rods));
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t) pool.emplace_back(work, int(int64_t(num_rods) * t / nt), int(int64_t(num_rods) * (t + 1) / nt));
  for (auto& th : pool) th.join();
  double L = 0;
  for (double v : loss_k) L += v;
  return L;
}

extern "C" {

// precision 1: FP64 (exact derivatives of the discrete algorithm); 0: FP32 (its rounding floor).
double orc_grad(int num_rods, const int32_t* off, const double* rest_pos, const double* rest_radius, const uint8_t* pinned,
                const double* activation, const double* compliance, const int32_t* group, double density, const double* gravity,
                double dt, int substeps, int iters, int frames, const double* targets, double* d_rbar, double* d_act, int threads,
                int precision) {
  return precision ? grad_impl<double>(num_rods, off, rest_pos, rest_radius, pinned, activation, compliance, group, density,
                                       gravity, dt, substeps, iters, frames, targets, d_rbar, d_act, threads)
                   : grad_impl<float>(num_rods, off, rest_pos, rest_radius, pinned, activation, compliance, group, density,
                                      gravity, dt, substeps, iters, frames, targets, d_rbar, d_act, threads);
}

}  // extern "C"
