// Device-side rod solver building blocks shared by the step kernels and the adjoint:
// per-slot state, the closed-form constraint updates, the colour passes and the lane
// layout (two pill slots per lane, DPP neighbour shifts).  See rod_kernels.hip.
#pragma once

#include "viper_dev.h"


namespace viper {

// Hardware reciprocal / reciprocal square root (1 ulp) for FP32; exact for FP64.
template <class T> __device__ __forceinline__ T rsq(T a);
template <> __device__ __forceinline__ float rsq<float>(float a) { return __builtin_amdgcn_rsqf(a); }
template <> __device__ __forceinline__ double rsq<double>(double a) { return rsqrt(a); }
template <class T> __device__ __forceinline__ T rcp(T a);
template <> __device__ __forceinline__ float rcp<float>(float a) { return __builtin_amdgcn_rcpf(a); }
template <> __device__ __forceinline__ double rcp<double>(double a) { return 1.0 / a; }

// Neighbour exchange by DPP wave shifts (a VALU move, no LDS round trip):
// wave_shl:1 delivers lane l+1's value to lane l, wave_shr:1 lane l-1's.  The lane
// without a source (63, resp. 0) reads zero (bound_ctrl), so the move needs no copy of the
// source to preserve; the rod layout never reads that value (rods do not cross wavefronts:
// lane 63 holds no edge that continues into a next lane, lane 0's slot A starts a rod).
__device__ __forceinline__ int dpp_dn(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_up(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true); }
template <class T> __device__ __forceinline__ T dn(T v);
template <class T> __device__ __forceinline__ T up(T v);
template <> __device__ __forceinline__ float dn<float>(float v) { return __int_as_float(dpp_dn(__float_as_int(v))); }
template <> __device__ __forceinline__ float up<float>(float v) { return __int_as_float(dpp_up(__float_as_int(v))); }
template <> __device__ __forceinline__ double dn<double>(double v) {
  return __hiloint2double(dpp_dn(__double2hiint(v)), dpp_dn(__double2loint(v)));
}
template <> __device__ __forceinline__ double up<double>(double v) {
  return __hiloint2double(dpp_up(__double2hiint(v)), dpp_up(__double2loint(v)));
}

// q <- normalize(q + [a, 0] (x) q): rotate by the world-frame vector 2a (a = half the
// rotation vector).
template <class T>
__device__ __forceinline__ void qrot_world_half(T& x, T& y, T& z, T& w, T a0, T a1, T a2) {
  const T nx = x + (w * a0 + (a1 * z - a2 * y));
  const T ny = y + (w * a1 + (a2 * x - a0 * z));
  const T nz = z + (w * a2 + (a0 * y - a1 * x));
  const T nw = w - (a0 * x + a1 * y + a2 * z);
  const T in = rsq(nx * nx + ny * ny + nz * nz + nw * nw);
  x = nx * in; y = ny * in; z = nz * in; w = nw * in;
}

// q <- normalize(q + 1/2 [t, 0] (x) q): rotate by the world-frame vector t.
template <class T>
__device__ __forceinline__ void qrot_world(T& x, T& y, T& z, T& w, T t0, T t1, T t2) {
  const T a0 = T(0.5) * t0, a1 = T(0.5) * t1, a2 = T(0.5) * t2;
  const T nx = x + (w * a0 + (a1 * z - a2 * y));
  const T ny = y + (w * a1 + (a2 * x - a0 * z));
  const T nz = z + (w * a2 + (a0 * y - a1 * x));
  const T nw = w - (a0 * x + a1 * y + a2 * z);
  const T in = rsq(nx * nx + ny * ny + nz * nz + nw * nw);
  x = nx * in; y = ny * in; z = nz * in; w = nw * in;
}

// One pill slot held in registers.
template <class T>
struct Slot {
  T x0, x1, x2, v0, v1, v2, s, sd;
  T q0, q1, q2, q3, o0, o1, o2;
  T xp0, xp1, xp2, sp, qp0, qp1, qp2, qp3;
  T l[12];                     // multipliers of the slot's constraints: ss(3) vol sg bt(3) sr sb vb(2)
  T w, ws;                     // inverse position / scale mass
  T ilb, il0, cbt, inert;      // edge constants
  T db0, db1, db2;             // rest Darboux vector
  T ass, avol, asg, abt, asr;  // compliance / (G l h^2)
  T asb, sg0, sg2;             // surface bending: compliance / (G l_v h^2), dC/ds of the first and third pill
  T avb;                       // volume-bending coupling: compliance / (G l_v h^2)
  T I1;                        // inverse bending inertia of the slot's edge (this substep)
  uint32_t f;
};

template <class T>
struct Lane2 {
  Slot<T> A, B;
  T wN, wsN, I1N;              // next lane's slot A: inverse masses, inverse bending inertia
  bool sb;                     // some rod of the wavefront has surface bending
  bool vb;                     // some rod of the wavefront has the volume-bending coupling
};

// ---------------------------------------------------------------- per-slot stages

template <class T>
__device__ __forceinline__ void predict_slot(Slot<T>& L, T h, T gx, T gy, T gz) {
  L.xp0 = L.x0; L.xp1 = L.x1; L.xp2 = L.x2; L.sp = L.s;
  if (L.w > T(0)) {
    const T h2 = h * h;
    L.x0 = L.x0 + h * L.v0 + h2 * gx;
    L.x1 = L.x1 + h * L.v1 + h2 * gy;
    L.x2 = L.x2 + h * L.v2 + h2 * gz;
  }
  L.s = L.s + h * L.sd;
  L.qp0 = L.q0; L.qp1 = L.q1; L.qp2 = L.q2; L.qp3 = L.q3;
  if (L.f & F_EDGE) qrot_world(L.q0, L.q1, L.q2, L.q3, h * L.o0, h * L.o1, h * L.o2);
#pragma unroll
  for (int i = 0; i < 12; ++i) L.l[i] = T(0);
}

// Inverse bending inertia 4 / (rho pi r^4 l s_m^2) of an edge from the substep-start
// midpoint scale (rotational weight of App. B).
template <class T>
__device__ __forceinline__ T inv_bend_inertia(const Slot<T>& L, T sp_right) {
  if (!(L.f & F_EDGE)) return T(0);
  const T sm = T(0.5) * (L.sp + sp_right);
  return T(4) * rcp(L.inert * sm * sm);
}

template <class T>
__device__ __forceinline__ void inertia_lane(Lane2<T>& P) {
  const T spN = dn(P.A.sp);
  P.A.I1 = inv_bend_inertia(P.A, P.B.sp);
  P.B.I1 = inv_bend_inertia(P.B, spN);
  P.I1N = dn(P.A.I1);
}

// Angular velocity of an edge from its quaternion before (p) and after (q) a substep:
// r = q (x) conj(p), shortest arc; omega = 2 Im(r) / h.
template <class T>
__device__ __forceinline__ void omega_of(T q0, T q1, T q2, T q3, T p0, T p1, T p2, T p3, T ih, T& o0, T& o1, T& o2) {
  const T rx = -q3 * p0 + q0 * p3 - q1 * p2 + q2 * p1;
  const T ry = -q3 * p1 + q0 * p2 + q1 * p3 - q2 * p0;
  const T rz = -q3 * p2 - q0 * p1 + q1 * p0 + q2 * p3;
  const T rw = q3 * p3 + q0 * p0 + q1 * p1 + q2 * p2;
  const T sg = (rw < T(0)) ? T(-2) * ih : T(2) * ih;
  o0 = sg * rx; o1 = sg * ry; o2 = sg * rz;
}

template <class T>
__device__ __forceinline__ void velocity_slot(Slot<T>& L, T ih) {
  if (L.w > T(0)) {
    L.v0 = (L.x0 - L.xp0) * ih; L.v1 = (L.x1 - L.xp1) * ih; L.v2 = (L.x2 - L.xp2) * ih;
  } else {
    L.v0 = T(0); L.v1 = T(0); L.v2 = T(0);
  }
  L.sd = (L.s - L.sp) * ih;
  if (L.f & F_EDGE) omega_of(L.q0, L.q1, L.q2, L.q3, L.qp0, L.qp1, L.qp2, L.qp3, ih, L.o0, L.o1, L.o2);
}

// ---------------------------------------------------------------- constraints

// Stretch-shear, volume and scale gradient of the edge from slot L to the right pill
// (b, sb) with inverse masses (wb, wsb).  Updates L and (b, sb) in place.  X: the optional
// terms (cross-section stretch here) are compiled in; without them the code is the plain
// constraint set.
template <class T, bool X = false>
__device__ __forceinline__ void edge_update(Slot<T>& L, T& b0, T& b1, T& b2, T& sb, T wb, T wsb) {
  T a0 = L.x0, a1 = L.x1, a2 = L.x2, sa = L.s;
  const T wa = L.w;
  if (L.f & F_SS) {
    const T q0 = L.q0, q1 = L.q1, q2 = L.q2, q3 = L.q3;
    // director d3 = q e_z conj(q) / |q|^2: exactly unit whatever rounding left in |q|.  The
    // unit-quaternion form 1 - 2(q0^2 + q1^2) turns a 1e-7 norm error into an edge-length
    // bias that a stiff stretch-shear constraint enforces, and gradients of stiff FP32 rods
    // amplify it by orders of magnitude.
    const T na = q0 * q0 + q1 * q1, nb = q2 * q2 + q3 * q3;
    const T in = rcp(na + nb), tw = in + in;
    const T d0 = (q0 * q2 + q3 * q1) * tw;
    const T d1 = (q1 * q2 - q3 * q0) * tw;
    const T d2 = (nb - na) * in;
    const T ilb = L.ilb, at = L.ass;
    const T c0 = (b0 - a0) * ilb - d0, c1 = (b1 - a1) * ilb - d1, c2 = (b2 - a2) * ilb - d2;
    const T k1 = (wa + wb) * ilb * ilb + at;
    const T ik1 = rcp(k1), ik2 = rcp(k1 + L.I1);
    const T r0 = -c0 - at * L.l[0], r1 = -c1 - at * L.l[1], r2 = -c2 - at * L.l[2];
    const T dr = d0 * r0 + d1 * r1 + d2 * r2;
    const T e = dr * (ik1 - ik2);
    const T g0 = r0 * ik2 + e * d0, g1 = r1 * ik2 + e * d1, g2 = r2 * ik2 + e * d2;
    L.l[0] += g0; L.l[1] += g1; L.l[2] += g2;
    const T fa = wa * ilb, fb = wb * ilb;
    a0 -= fa * g0; a1 -= fa * g1; a2 -= fa * g2;
    b0 += fb * g0; b1 += fb * g1; b2 += fb * g2;
    const T nI = T(-0.5) * L.I1;   // dtheta = -(d3 x dl) / I_bend, halved for the quaternion update
    qrot_world_half(L.q0, L.q1, L.q2, L.q3, nI * (d1 * g2 - d2 * g1), nI * (d2 * g0 - d0 * g2),
                    nI * (d0 * g1 - d1 * g0));
  }
  if (L.f & F_VOL) {
    const T e0 = b0 - a0, e1 = b1 - a1, e2 = b2 - a2;
    const T len2 = e0 * e0 + e1 * e1 + e2 * e2;
    const T ilen = rsq(len2);
    const T len = len2 * ilen;
    const T ss = sa + sb;   // twice the midpoint scale sm
    const T gx = (ss * ss) * (T(0.25) * L.il0), gs = (ss * len) * (T(0.5) * L.il0);   // sm^2 / l0, sm l / l0
    const T C = gx * len - T(1);
    const T at = L.avol;
    const T S = (wa + wb) * gx * gx + (L.ws + wsb) * gs * gs + at;
    const T dl = (-C - at * L.l[3]) * rcp(S);
    L.l[3] += dl;
    const T k = gx * dl * ilen;
    a0 -= wa * k * e0; a1 -= wa * k * e1; a2 -= wa * k * e2;
    b0 += wb * k * e0; b1 += wb * k * e1; b2 += wb * k * e2;
    sa += L.ws * gs * dl;
    sb += wsb * gs * dl;
  }
  if (L.f & F_SG) {
    const T il0 = L.il0, at = L.asg;
    const T C = (sb - sa) * il0;
    const T S = (L.ws + wsb) * il0 * il0 + at;
    const T dl = (-C - at * L.l[4]) * rcp(S);
    L.l[4] += dl;
    sa -= L.ws * il0 * dl;
    sb += wsb * il0 * dl;
  }
  if (X && (L.f & F_SR)) {   // cross-section stretch: midpoint scale back to one, dC/ds = 1/2 each
    const T at = L.asr;
    const T C = T(0.5) * (sa + sb) - T(1);
    const T S = T(0.25) * (L.ws + wsb) + at;
    const T dl = (-C - at * L.l[8]) * rcp(S);
    L.l[8] += dl;
    sa += T(0.5) * L.ws * dl;
    sb += T(0.5) * wsb * dl;
  }
  L.x0 = a0; L.x1 = a1; L.x2 = a2; L.s = sa;
}

// Bend-twist at the vertex between slot L's edge (a) and the next edge (b: quaternion
// b0..b3, vertex scale sb, inverse bending inertia Ib, inverse scale mass wsb).
template <class T>
__device__ __forceinline__ void bt_update(Slot<T>& L, T& b0, T& b1, T& b2, T& b3, T& sb, T Ib, T wsb) {
  const T a0 = L.q0, a1 = L.q1, a2 = L.q2, a3 = L.q3;
  // r = conj(qa) (x) qb
  const T rx = a3 * b0 - a0 * b3 - a1 * b2 + a2 * b1;
  const T ry = a3 * b1 + a0 * b2 - a1 * b3 - a2 * b0;
  const T rz = a3 * b2 - a0 * b1 + a1 * b0 - a2 * b3;
  const T rw = a3 * b3 + a0 * b0 + a1 * b1 + a2 * b2;
  const T sg = (rw < T(0)) ? T(-1) : T(1);
  const T v0 = sg * rx, v1 = sg * ry, v2 = sg * rz, w = sg * rw;
  const T c = L.cbt;
  const T sc = sb * c;
  const T C0 = sc * v0 - L.db0, C1 = sc * v1 - L.db1, C2 = sc * v2 - L.db2;
  // tangent of edge b in frame a: t = R(r) e_z;  u = B e_z, y = B t with B = w I - [v]x.
  // For a unit r, B t = Im(conj(r) (x) r (x) e_z (x) conj(r)) = Im(e_z (x) conj(r)), so
  // y = (v1, -v0, w) and u = (-v1, v0, w): y y^T is u u^T with its (0,2), (1,2) entries negated.
  const T v0s = v0 * v0, v1s = v1 * v1;
  const T th0 = v0 * v2 + w * v1, th1 = v1 * v2 - w * v0, th2 = T(0.5) - (v0s + v1s);   // t / 2
  // S = K[(Ia+Ib)(I - v v^T) - Ia/2 u u^T - Ib/2 y y^T] + wsb c^2 v v^T + diag(a, a, a/2),
  // assembled directly as s = S / (m + a), m = K (Ia + Ib): the entries reach ~1e14 for thin
  // rods and the cubic determinant would leave the FP32 range; scaled they are O(1) (each
  // term of S is at most of the order of m or a).  S^-1 = adj(s) / (det(s) (m + a)).
  //   s = I - diag(0, 0, a/2) sgm + qs v v^T - has u u^T - hbs y y^T
  //     = I - diag(0, 0, a/2) sgm + qs v v^T - hp (u0^2, u1^2, u2^2, u0 u1 off the last
  //       column) - hm (u0 u2, u1 u2),  hp = has + hbs, hm = has - hbs
  //   (K = sc^2 / 4: m = sc^2 (Ia+Ib)/4, hp = sc^2 sgm (Ia+Ib)/8, hm = sc^2 sgm (Ia-Ib)/8)
  const T Ia = L.I1;
  const T sc2 = sc * sc;
  const T m = sc2 * (T(0.25) * (Ia + Ib));
  const T at = L.abt;
  const T sgm = rcp(m + at);
  const T qs = (wsb * c * c - m) * sgm;
  const T ks = sc2 * sgm;
  const T hp = ks * (T(0.125) * (Ia + Ib)), hm = ks * (T(0.125) * (Ia - Ib));
  const T pv0 = qs * v0, pv1 = qs * v1, pv2 = qs * v2;
  const T s00 = T(1) + pv0 * v0 - hp * v1s;
  const T s11 = T(1) + pv1 * v1 - hp * v0s;
  const T s22 = (T(1) - T(0.5) * at * sgm) + pv2 * v2 - hp * (w * w);
  const T s01 = (qs + hp) * (v0 * v1);
  const T s02 = pv0 * v2 + hm * (v1 * w);
  const T s12 = pv1 * v2 - hm * (v0 * w);
  const T r0 = -C0 - at * L.l[5], r1 = -C1 - at * L.l[6], r2 = -C2 - T(0.5) * at * L.l[7];
  const T A00 = s11 * s22 - s12 * s12, A01 = s02 * s12 - s01 * s22, A02 = s01 * s12 - s02 * s11;
  const T A11 = s00 * s22 - s02 * s02, A12 = s01 * s02 - s00 * s12, A22 = s00 * s11 - s01 * s01;
  const T idet = sgm * rcp(s00 * A00 + s01 * A01 + s02 * A02);
  const T g0 = (A00 * r0 + A01 * r1 + A02 * r2) * idet;
  const T g1 = (A01 * r0 + A11 * r1 + A12 * r2) * idet;
  const T g2 = (A02 * r0 + A12 * r1 + A22 * r2) * idet;
  L.l[5] += g0; L.l[6] += g1; L.l[7] += g2;
  // B^T dl = w dl + v x dl   (frame a)
  const T e0 = w * g0 + (v1 * g2 - v2 * g1);
  const T e1 = w * g1 + (v2 * g0 - v0 * g2);
  const T e2 = w * g2 + (v0 * g1 - v1 * g0);
  // body-frame (a) rotation of edge a: da = -hs Ia (e - e_z e_z/2), hs = sc/2; h = da / 2
  const T ka = sc * (T(-0.25) * Ia), ka2 = sc * (T(-0.125) * Ia);
  // frame-a rotation of edge b: dB = hs Ib (e - (t.e) t / 2); h = sg dB / 2
  const T te = th0 * e0 + th1 * e1 + th2 * e2;   // (t.e) / 2
  const T te2 = te + te;
  const T kb = (sg * sc) * (T(0.25) * Ib);
  // q_a <- normalize(q_a + 1/2 q_a (x) [da, 0])
  {
    const T h0 = ka * e0, h1 = ka * e1, h2 = ka2 * e2;
    const T nx = a0 + (a3 * h0 + (a1 * h2 - a2 * h1));
    const T ny = a1 + (a3 * h1 + (a2 * h0 - a0 * h2));
    const T nz = a2 + (a3 * h2 + (a0 * h1 - a1 * h0));
    const T nw = a3 - (a0 * h0 + a1 * h1 + a2 * h2);
    const T in = rsq(nx * nx + ny * ny + nz * nz + nw * nw);
    L.q0 = nx * in; L.q1 = ny * in; L.q2 = nz * in; L.q3 = nw * in;
  }
  // q_b <- normalize(q_b + 1/2 q_a (x) [dB, 0] (x) r_true),  r_true = sg (v, w)
  {
    const T h0 = kb * (e0 - te2 * th0), h1 = kb * (e1 - te2 * th1), h2 = kb * (e2 - te2 * th2);
    const T p0 = w * h0 + (h1 * v2 - h2 * v1);
    const T p1 = w * h1 + (h2 * v0 - h0 * v2);
    const T p2 = w * h2 + (h0 * v1 - h1 * v0);
    const T p3 = -(h0 * v0 + h1 * v1 + h2 * v2);
    const T nx = b0 + (a3 * p0 + a0 * p3 + a1 * p2 - a2 * p1);
    const T ny = b1 + (a3 * p1 - a0 * p2 + a1 * p3 + a2 * p0);
    const T nz = b2 + (a3 * p2 + a0 * p1 - a1 * p0 + a2 * p3);
    const T nw = b3 + (a3 * p3 - a0 * p0 - a1 * p1 - a2 * p2);
    const T in = rsq(nx * nx + ny * ny + nz * nz + nw * nw);
    b0 = nx * in; b1 = ny * in; b2 = nz * in; b3 = nw * in;
  }
  sb += wsb * c * (v0 * g0 + v1 * g1 + v2 * g2);
}

// Volume-bending coupling at the same vertex: the two bending rows of the bend-twist Darboux
// vector with the vertex scale cubed, C = s^3 c v_{u,v} - Omega_rest_{u,v}.  The bend-twist
// system restricted to those rows, with K = (s^3 c)^2 / 4 and the scale column 3 s^2 c v:
//   S = K[(Ia+Ib)(I - v v^T) - Ia/2 u u^T - Ib/2 y y^T] + wsb (3 s^2 c)^2 v v^T + a I   (2 x 2)
// and the rotations of bend-twist driven by B^T (g0, g1, 0).
template <class T>
__device__ __forceinline__ void vb_update(Slot<T>& L, T& b0, T& b1, T& b2, T& b3, T& sb, T Ib, T wsb) {
  const T a0 = L.q0, a1 = L.q1, a2 = L.q2, a3 = L.q3;
  const T rx = a3 * b0 - a0 * b3 - a1 * b2 + a2 * b1;
  const T ry = a3 * b1 + a0 * b2 - a1 * b3 - a2 * b0;
  const T rz = a3 * b2 - a0 * b1 + a1 * b0 - a2 * b3;
  const T rw = a3 * b3 + a0 * b0 + a1 * b1 + a2 * b2;
  const T sg = (rw < T(0)) ? T(-1) : T(1);
  const T v0 = sg * rx, v1 = sg * ry, v2 = sg * rz, w = sg * rw;
  const T c = L.cbt;
  const T s2 = sb * sb;
  const T sc = s2 * sb * c, gs = T(3) * s2 * c;
  const T C0 = sc * v0 - L.db0, C1 = sc * v1 - L.db1;
  const T t0 = T(2) * (v0 * v2 + w * v1);
  const T t1 = T(2) * (v1 * v2 - w * v0);
  const T t2 = T(1) - T(2) * (v0 * v0 + v1 * v1);
  const T u0 = -v1, u1 = v0;
  const T y0 = w * t0 - (v1 * t2 - v2 * t1);
  const T y1 = w * t1 - (v2 * t0 - v0 * t2);
  const T Ia = L.I1;
  const T K = T(0.25) * sc * sc;
  const T m = K * (Ia + Ib);
  const T ha = T(0.5) * K * Ia, hb = T(0.5) * K * Ib;
  const T qv = wsb * gs * gs - m;
  const T at = L.avb;
  const T S00 = m + qv * v0 * v0 - ha * u0 * u0 - hb * y0 * y0 + at;
  const T S11 = m + qv * v1 * v1 - ha * u1 * u1 - hb * y1 * y1 + at;
  const T S01 = qv * v0 * v1 - ha * u0 * u1 - hb * y0 * y1;
  const T r0 = -C0 - at * L.l[10], r1 = -C1 - at * L.l[11];
  // equilibrate by the trace (FP32 range), then 2 x 2 inverse
  const T sgm = rcp(S00 + S11);
  const T s00 = S00 * sgm, s11 = S11 * sgm, s01 = S01 * sgm;
  const T idet = sgm * rcp(s00 * s11 - s01 * s01);
  const T g0 = (s11 * r0 - s01 * r1) * idet;
  const T g1 = (s00 * r1 - s01 * r0) * idet;
  L.l[10] += g0; L.l[11] += g1;
  const T e0 = w * g0 - v2 * g1;
  const T e1 = w * g1 + v2 * g0;
  const T e2 = v0 * g1 - v1 * g0;
  const T hs = T(0.5) * sc;
  const T ka = -hs * Ia;
  const T da0 = ka * e0, da1 = ka * e1, da2 = T(0.5) * ka * e2;
  const T te = T(0.5) * (t0 * e0 + t1 * e1 + t2 * e2);
  const T kb = hs * Ib;
  const T dB0 = kb * (e0 - te * t0), dB1 = kb * (e1 - te * t1), dB2 = kb * (e2 - te * t2);
  {
    const T h0 = T(0.5) * da0, h1 = T(0.5) * da1, h2 = T(0.5) * da2;
    const T nx = a0 + (a3 * h0 + (a1 * h2 - a2 * h1));
    const T ny = a1 + (a3 * h1 + (a2 * h0 - a0 * h2));
    const T nz = a2 + (a3 * h2 + (a0 * h1 - a1 * h0));
    const T nw = a3 - (a0 * h0 + a1 * h1 + a2 * h2);
    const T in = rsq(nx * nx + ny * ny + nz * nz + nw * nw);
    L.q0 = nx * in; L.q1 = ny * in; L.q2 = nz * in; L.q3 = nw * in;
  }
  {
    const T h0 = T(0.5) * sg * dB0, h1 = T(0.5) * sg * dB1, h2 = T(0.5) * sg * dB2;
    const T p0 = w * h0 + (h1 * v2 - h2 * v1);
    const T p1 = w * h1 + (h2 * v0 - h0 * v2);
    const T p2 = w * h2 + (h0 * v1 - h1 * v0);
    const T p3 = -(h0 * v0 + h1 * v1 + h2 * v2);
    const T nx = b0 + (a3 * p0 + a0 * p3 + a1 * p2 - a2 * p1);
    const T ny = b1 + (a3 * p1 - a0 * p2 + a1 * p3 + a2 * p0);
    const T nz = b2 + (a3 * p2 + a0 * p1 - a1 * p0 + a2 * p3);
    const T nw = b3 + (a3 * p3 - a0 * p0 - a1 * p1 - a2 * p2);
    const T in = rsq(nx * nx + ny * ny + nz * nz + nw * nw);
    b0 = nx * in; b1 = ny * in; b2 = nz * in; b3 = nw * in;
  }
  sb += wsb * gs * (v0 * g0 + v1 * g1);
}

__device__ __forceinline__ bool colour_is(uint32_t f, int colour) { return ((f & F_ODD) != 0) == (colour != 0); }

// Stretch-shear, volume and scale gradient of every edge of parity `colour`.  EVEN: every rod
// of the batch starts on an even slot of its wavefront, so slot A holds the even pills: the
// even edges are lane-local (A to B) and the odd ones all join slot B to the next lane's A.
template <class T, bool X = false, bool EVEN = false>
__device__ __forceinline__ void pass_edges(Lane2<T>& P, int colour) {
  if constexpr (EVEN) {
    if (colour == 0) {
      if (P.A.f & F_EDGE) edge_update<T, X>(P.A, P.B.x0, P.B.x1, P.B.x2, P.B.s, P.B.w, P.B.ws);
      return;
    }
    T n0 = dn(P.A.x0), n1 = dn(P.A.x1), n2 = dn(P.A.x2), ns = dn(P.A.s);
    if (P.B.f & F_EDGE) edge_update<T, X>(P.B, n0, n1, n2, ns, P.wN, P.wsN);
    n0 = up(n0); n1 = up(n1); n2 = up(n2); ns = up(ns);
    if ((P.A.f & F_VALID) && !(P.A.f & F_FIRST)) {
      P.A.x0 = n0; P.A.x1 = n1; P.A.x2 = n2; P.A.s = ns;
    }
    return;
  }
  T n0 = dn(P.A.x0), n1 = dn(P.A.x1), n2 = dn(P.A.x2), ns = dn(P.A.s);
  if ((P.A.f & F_EDGE) && colour_is(P.A.f, colour)) {
    edge_update<T, X>(P.A, P.B.x0, P.B.x1, P.B.x2, P.B.s, P.B.w, P.B.ws);
  } else if ((P.B.f & F_EDGE) && colour_is(P.B.f, colour)) {
    edge_update<T, X>(P.B, n0, n1, n2, ns, P.wN, P.wsN);
  }
  // the right end of a B-edge belongs to the next lane's slot A
  n0 = up(n0); n1 = up(n1); n2 = up(n2); ns = up(ns);
  if ((P.A.f & F_VALID) && !(P.A.f & F_FIRST) && !colour_is(P.A.f, colour)) {
    P.A.x0 = n0; P.A.x1 = n1; P.A.x2 = n2; P.A.s = ns;
  }
}

// Bend-twist at every vertex of parity `colour` (between the slot's edge and the next).
// EVEN: as for pass_edges.
template <class T, bool EVEN = false>
__device__ __forceinline__ void pass_bt(Lane2<T>& P, int colour) {
  if constexpr (EVEN) {
    if (colour == 0) {
      if ((P.A.f & F_BT) && (P.A.f & F_BTEN)) bt_update(P.A, P.B.q0, P.B.q1, P.B.q2, P.B.q3, P.B.s, P.B.I1, P.B.ws);
      return;
    }
    T n0 = dn(P.A.q0), n1 = dn(P.A.q1), n2 = dn(P.A.q2), n3 = dn(P.A.q3), ns = dn(P.A.s);
    if ((P.B.f & F_BT) && (P.B.f & F_BTEN)) bt_update(P.B, n0, n1, n2, n3, ns, P.I1N, P.wsN);
    n0 = up(n0); n1 = up(n1); n2 = up(n2); n3 = up(n3); ns = up(ns);
    if ((P.A.f & F_EDGE) && !(P.A.f & F_FIRST) && (P.A.f & F_BTEN)) {
      P.A.q0 = n0; P.A.q1 = n1; P.A.q2 = n2; P.A.q3 = n3; P.A.s = ns;
    }
    return;
  }
  T n0 = dn(P.A.q0), n1 = dn(P.A.q1), n2 = dn(P.A.q2), n3 = dn(P.A.q3), ns = dn(P.A.s);
  if ((P.A.f & F_BT) && (P.A.f & F_BTEN) && colour_is(P.A.f, colour)) {
    bt_update(P.A, P.B.q0, P.B.q1, P.B.q2, P.B.q3, P.B.s, P.B.I1, P.B.ws);
  } else if ((P.B.f & F_BT) && (P.B.f & F_BTEN) && colour_is(P.B.f, colour)) {
    bt_update(P.B, n0, n1, n2, n3, ns, P.I1N, P.wsN);
  }
  n0 = up(n0); n1 = up(n1); n2 = up(n2); n3 = up(n3); ns = up(ns);
  if ((P.A.f & F_EDGE) && !(P.A.f & F_FIRST) && (P.A.f & F_BTEN) && !colour_is(P.A.f, colour)) {
    P.A.q0 = n0; P.A.q1 = n1; P.A.q2 = n2; P.A.q3 = n3; P.A.s = ns;
  }
}

// Volume-bending coupling at every vertex of parity `colour` (after all bend-twist passes;
// the same lane exchange as bend-twist).
template <class T>
__device__ __forceinline__ void pass_vb(Lane2<T>& P, int colour) {
  T n0 = dn(P.A.q0), n1 = dn(P.A.q1), n2 = dn(P.A.q2), n3 = dn(P.A.q3), ns = dn(P.A.s);
  if ((P.A.f & F_BT) && (P.A.f & F_VB) && colour_is(P.A.f, colour)) {
    vb_update(P.A, P.B.q0, P.B.q1, P.B.q2, P.B.q3, P.B.s, P.B.I1, P.B.ws);
  } else if ((P.B.f & F_BT) && (P.B.f & F_VB) && colour_is(P.B.f, colour)) {
    vb_update(P.B, n0, n1, n2, n3, ns, P.I1N, P.wsN);
  }
  n0 = up(n0); n1 = up(n1); n2 = up(n2); n3 = up(n3); ns = up(ns);
  if ((P.A.f & F_EDGE) && !(P.A.f & F_FIRST) && (P.A.f & F_VB) && !colour_is(P.A.f, colour)) {
    P.A.q0 = n0; P.A.q1 = n1; P.A.q2 = n2; P.A.q3 = n3; P.A.s = ns;
  }
}

// Surface bending at the vertex after slot L's edge: scales s0 (the slot's), s1, s2 (the next
// two pills) with inverse scale masses w0..w2,
//   C = g0 s0 - (g0 + g2) s1 + g2 s2,  g0 = 1 / (l_a l_v), g2 = 1 / (l_b l_v).
template <class T>
__device__ __forceinline__ void sb_update(Slot<T>& L, T& s0, T& s1, T& s2, T w0, T w1, T w2) {
  const T g0 = L.sg0, g2 = L.sg2, g1 = -(g0 + g2), at = L.asb;
  const T C = g0 * s0 + g1 * s1 + g2 * s2;
  const T S = w0 * g0 * g0 + w1 * g1 * g1 + w2 * g2 * g2 + at;
  const T dl = (-C - at * L.l[9]) * rcp(S);
  L.l[9] += dl;
  s0 += w0 * g0 * dl;
  s1 += w1 * g1 * dl;
  s2 += w2 * g2 * dl;
}

__device__ __forceinline__ bool mod3_is(uint32_t f, int colour) {
  return (int)((f & F_M3A) ? 1 : (f & F_M3B) ? 2 : 0) == colour;
}

// Surface bending at every vertex whose first pill has local index `colour` mod 3.  Three
// consecutive scales: an owner in slot A reaches the next lane's A, an owner in slot B the
// next lane's A and B; the changed values travel back up one lane.
template <class T>
__device__ __forceinline__ void pass_sb(Lane2<T>& P, int colour) {
  T nA = dn(P.A.s), nB = dn(P.B.s);
  const T wsNB = dn(P.B.ws);
  T sent = T(0);   // 1: the next lane's A changed, 2: its A and B
  if ((P.A.f & F_BT) && (P.A.f & F_SB) && mod3_is(P.A.f, colour)) {
    sb_update(P.A, P.A.s, P.B.s, nA, P.A.ws, P.B.ws, P.wsN);
    sent = T(1);
  } else if ((P.B.f & F_BT) && (P.B.f & F_SB) && mod3_is(P.B.f, colour)) {
    sb_update(P.B, P.B.s, nA, nB, P.B.ws, P.wsN, wsNB);
    sent = T(2);
  }
  nA = up(nA); nB = up(nB); sent = up(sent);
  // a rod's first pill is never reached from the previous lane (this also covers lane 0,
  // whose shifted values are its own)
  if ((P.A.f & F_VALID) && !(P.A.f & F_FIRST) && sent > T(0)) {
    P.A.s = nA;
    if (sent > T(1.5) && (P.B.f & F_VALID)) P.B.s = nB;
  }
}

// One Gauss-Seidel iteration.  X: the optional terms (cross-section stretch, volume-bending
// coupling, surface bending) are compiled in; the plain instantiation runs scenes without them.
template <class T, bool X = false, bool EVEN = false>
__device__ __forceinline__ void iteration_lane(Lane2<T>& P) {
  pass_edges<T, X, EVEN>(P, 0);
  pass_edges<T, X, EVEN>(P, 1);
  pass_bt<T, EVEN>(P, 0);
  pass_bt<T, EVEN>(P, 1);
  if constexpr (X) {
    if (P.vb) {   // the same on every lane of the wavefront
      pass_vb(P, 0);
      pass_vb(P, 1);
    }
    if (P.sb) {   // the same on every lane of the wavefront
      pass_sb(P, 0);
      pass_sb(P, 1);
      pass_sb(P, 2);
    }
  }
}

// ---------------------------------------------------------------- load / store

// Slots of this lane: pA = p0 + 2 lane, pB = pA + 1 of its wavefront's run (clamped to a
// valid index beyond the run; such slots carry no flags and are never stored).  The block
// table maps the block to its scene and first wavefront.
template <class T>
__device__ __forceinline__ const Dev<T>* lane_setup_wave(const Dev<T>* D, const Blk b, int wave, Lane2<T>& P, int& pA,
                                                         int& pB) {
  const Dev<T>* d = D + b.scene;
  const int lane = (int)(threadIdx.x & 63);
  if (wave >= d->W) return nullptr;
  const int p0 = d->wave_start[wave];
  const int n = d->wave_start[wave + 1] - p0;
  const bool vA = 2 * lane < n, vB = 2 * lane + 1 < n;
  pA = p0 + (vA ? 2 * lane : 0);
  pB = p0 + (vB ? 2 * lane + 1 : 0);
  P.A.f = vA ? d->flags[pA] : 0u;
  P.B.f = vB ? d->flags[pB] : 0u;
  P.sb = __any(((P.A.f | P.B.f) & F_SB) != 0u) != 0;
  P.vb = __any(((P.A.f | P.B.f) & F_VB) != 0u) != 0;
  return d;
}

// Blocks of four wavefronts: wavefront w of the block is tab[block].base + w.
template <class T>
__device__ __forceinline__ const Dev<T>* lane_setup(const Dev<T>* D, const Blk* tab, Lane2<T>& P, int& pA, int& pB) {
  const Blk b = tab[blockIdx.x];
  return lane_setup_wave(D, b, b.base + (int)(threadIdx.x >> 6), P, pA, pB);
}

template <class T>
__device__ __forceinline__ void load_state(const Dev<T>& d, Slot<T>& L, int p) {
  L.x0 = d.px[p]; L.x1 = d.py[p]; L.x2 = d.pz[p];
  L.v0 = d.vx[p]; L.v1 = d.vy[p]; L.v2 = d.vz[p];
  L.s = d.s[p]; L.sd = d.sd[p];
  L.q0 = d.qx[p]; L.q1 = d.qy[p]; L.q2 = d.qz[p]; L.q3 = d.qw[p];
  L.o0 = d.ox[p]; L.o1 = d.oy[p]; L.o2 = d.oz[p];
}

template <class T, bool X = false>
__device__ __forceinline__ void load_consts(const Dev<T>& d, Slot<T>& L, int p, T ih2) {
  L.w = d.winv[p]; L.ws = d.wsinv[p];
  L.ilb = d.ilb[p]; L.il0 = d.il0[p]; L.cbt = d.cbt[p]; L.inert = d.inert[p];
  L.db0 = d.dbx[p]; L.db1 = d.dby[p]; L.db2 = d.dbz[p];
  L.ass = d.css[p] * ih2; L.avol = d.cvol[p] * ih2; L.asg = d.csg[p] * ih2; L.abt = d.cbtc[p] * ih2;
  if constexpr (X) {
    L.asr = (L.f & F_SR) ? d.csr[p] * ih2 : T(0);
    const bool sb = (L.f & F_SB) && (L.f & F_BT);
    L.asb = sb ? d.csb[p] * ih2 : T(0);
    L.sg0 = sb ? d.sbg0[p] : T(0);
    L.sg2 = sb ? d.sbg2[p] : T(0);
    L.avb = (L.f & F_VB) ? d.cvb[p] * ih2 : T(0);
  }
}

template <class T, bool X = false>
__device__ __forceinline__ void load_lane_consts(const Dev<T>& d, Lane2<T>& P, int pA, int pB, T ih2) {
  load_consts<T, X>(d, P.A, pA, ih2);
  load_consts<T, X>(d, P.B, pB, ih2);
  P.wN = dn(P.A.w);
  P.wsN = dn(P.A.ws);
}

template <class T>
__device__ __forceinline__ void store_state(const Dev<T>& d, const Slot<T>& L, int p) {
  if (!(L.f & F_VALID)) return;
  d.px[p] = L.x0; d.py[p] = L.x1; d.pz[p] = L.x2;
  d.vx[p] = L.v0; d.vy[p] = L.v1; d.vz[p] = L.v2;
  d.s[p] = L.s; d.sd[p] = L.sd;
  if (L.f & F_EDGE) {
    d.qx[p] = L.q0; d.qy[p] = L.q1; d.qz[p] = L.q2; d.qw[p] = L.q3;
    d.ox[p] = L.o0; d.oy[p] = L.o1; d.oz[p] = L.o2;
  }
}

template <class T>
__device__ __forceinline__ void check_finite(const Dev<T>& d, const Slot<T>& L) {
  if (!(L.f & F_VALID)) return;
  const T acc = L.x0 + L.x1 + L.x2 + L.s + L.q0 + L.q1 + L.q2 + L.q3;
  if (!isfinite(acc)) d.status[ST_NAN] = 1;
}

}  // namespace viper
