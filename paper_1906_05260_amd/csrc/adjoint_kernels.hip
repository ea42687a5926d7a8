// Adjoint (reverse mode) of the collision-free rod frame, for gfx950.
//
// Forward: the frame kernel variant below also writes the state at the start of every
// substep (per-substep checkpoint).  Backward: one launch per substep, in reverse order.
// Each launch reloads its checkpoint, recomputes the substep exactly as the forward does
// (same device code) while storing the state before every colour pass, then sweeps back:
// velocity update, the 4 x iterations passes in reverse, the substep-start inertia, and
// the prediction.  The vector-Jacobian product of each projection is written out in closed
// form: the projection's intermediates are recomputed from its pre-pass inputs, then their
// adjoints are propagated back through the same formulas in reverse order (the derivative
// of the arithmetic the forward performs, with the hardware reciprocal and reciprocal
// square root taken as exact).  Adjoints of the per-slot parameters (inverse masses,
// inverse stretch rest length, inertia base, compliance scalings) are accumulated per slot
// and chained to rest radii and activations on the host.

#include "rod_device.h"
#include "stage_setup.h"

namespace viper {

// ---------------------------------------------------------------- quaternion helpers

template <class T>
struct Q4 {
  T x, y, z, w;
};

// a (x) b
template <class T>
__device__ __forceinline__ Q4<T> qmul(const Q4<T>& a, const Q4<T>& b) {
  return {a.w * b.x + b.w * a.x + (a.y * b.z - a.z * b.y), a.w * b.y + b.w * a.y + (a.z * b.x - a.x * b.z),
          a.w * b.z + b.w * a.z + (a.x * b.y - a.y * b.x), a.w * b.w - (a.x * b.x + a.y * b.y + a.z * b.z)};
}
template <class T>
__device__ __forceinline__ Q4<T> qconj(const Q4<T>& a) { return {-a.x, -a.y, -a.z, a.w}; }

// Adjoint of n through u = n / |n| (u computed with inv = rsq(n.n)): inv u_bar - inv^3 (n.u_bar) n.
template <class T>
__device__ __forceinline__ Q4<T> normalize_vjp(const Q4<T>& n, T inv, const Q4<T>& ub) {
  const T k = inv * inv * inv * (n.x * ub.x + n.y * ub.y + n.z * ub.z + n.w * ub.w);
  return {inv * ub.x - k * n.x, inv * ub.y - k * n.y, inv * ub.z - k * n.z, inv * ub.w - k * n.w};
}

// ---------------------------------------------------------------- local VJPs

// Stretch-shear + volume + scale gradient of slot L's edge (edge_update, the plain
// constraint set).  Inputs (26): x0 x1 x2 s q0 q1 q2 q3 l0..l4 | b0 b1 b2 sb |
// w ws ilb ass avol asg I1 | wb wsb.  Outputs (17): x0 x1 x2 s q0..q3 l0..l4 | b0 b1 b2 sb.
// xb = J^T yb.
template <class T>
__device__ void edge_vjp(const Slot<T>& L, T b0, T b1, T b2, T sb, T wb, T wsb, const T (&yb)[17], T (&xb)[26]) {
  const uint32_t f = L.f;
  const bool ss = (f & F_SS) != 0, vol = (f & F_VOL) != 0, sgr = (f & F_SG) != 0;
  const T wa = L.w, wsa = L.ws, ilb = L.ilb, il0 = L.il0, I1 = L.I1;
  const T ass = L.ass, avol = L.avol, asg = L.asg;
  const Q4<T> q = {L.q0, L.q1, L.q2, L.q3};
  // ---- forward recompute
  // stretch-shear
  T a0 = L.x0, a1 = L.x1, a2 = L.x2, c0 = b0, c1 = b1, c2 = b2;   // pills after it
  T na = 0, nb = 0, in = 0, P0 = 0, P1 = 0, d0 = 0, d1 = 0, d2 = 0, ik1 = 0, ik2 = 0;
  T r0 = 0, r1 = 0, r2 = 0, dr = 0, ee = 0, g0 = 0, g1 = 0, g2 = 0, nI = 0, rho0 = 0, rho1 = 0, rho2 = 0, inn = 0;
  Q4<T> n = q;
  if (ss) {
    na = q.x * q.x + q.y * q.y; nb = q.z * q.z + q.w * q.w;
    in = rcp(na + nb);
    const T tw = in + in;
    P0 = q.x * q.z + q.w * q.y; P1 = q.y * q.z - q.w * q.x;
    d0 = P0 * tw; d1 = P1 * tw; d2 = (nb - na) * in;
    const T k1 = (wa + wb) * ilb * ilb + ass;
    ik1 = rcp(k1); ik2 = rcp(k1 + I1);
    r0 = -((b0 - a0) * ilb - d0) - ass * L.l[0];
    r1 = -((b1 - a1) * ilb - d1) - ass * L.l[1];
    r2 = -((b2 - a2) * ilb - d2) - ass * L.l[2];
    dr = d0 * r0 + d1 * r1 + d2 * r2;
    ee = dr * (ik1 - ik2);
    g0 = r0 * ik2 + ee * d0; g1 = r1 * ik2 + ee * d1; g2 = r2 * ik2 + ee * d2;
    const T fa = wa * ilb, fb = wb * ilb;
    a0 -= fa * g0; a1 -= fa * g1; a2 -= fa * g2;
    c0 += fb * g0; c1 += fb * g1; c2 += fb * g2;
    nI = T(-0.5) * I1;
    rho0 = nI * (d1 * g2 - d2 * g1); rho1 = nI * (d2 * g0 - d0 * g2); rho2 = nI * (d0 * g1 - d1 * g0);
    n = {q.x + (q.w * rho0 + (rho1 * q.z - rho2 * q.y)), q.y + (q.w * rho1 + (rho2 * q.x - rho0 * q.z)),
         q.z + (q.w * rho2 + (rho0 * q.y - rho1 * q.x)), q.w - (rho0 * q.x + rho1 * q.y + rho2 * q.z)};
    inn = rsq(n.x * n.x + n.y * n.y + n.z * n.z + n.w * n.w);
  }
  // volume (on the pills after stretch-shear)
  T e0 = 0, e1 = 0, e2 = 0, len2 = 0, ilen = 0, len = 0, ssum = 0, gx = 0, gs = 0, iSv = 0, dlv = 0, kv = 0;
  T sa1 = L.s, sb1 = sb;
  if (vol) {
    e0 = c0 - a0; e1 = c1 - a1; e2 = c2 - a2;
    len2 = e0 * e0 + e1 * e1 + e2 * e2;
    ilen = rsq(len2);
    len = len2 * ilen;
    ssum = L.s + sb;
    gx = (ssum * ssum) * (T(0.25) * il0); gs = (ssum * len) * (T(0.5) * il0);
    const T C = gx * len - T(1);
    iSv = rcp((wa + wb) * gx * gx + (wsa + wsb) * gs * gs + avol);
    dlv = (-C - avol * L.l[3]) * iSv;
    kv = gx * dlv * ilen;
    sa1 += wsa * gs * dlv; sb1 += wsb * gs * dlv;
  }
  // scale gradient (on the scales after volume)
  T iSg = 0, dlg = 0;
  if (sgr) {
    iSg = rcp((wsa + wsb) * il0 * il0 + asg);
    dlg = (-((sb1 - sa1) * il0) - asg * L.l[4]) * iSg;
  }
  // ---- reverse sweep
  T Ax0 = yb[0], Ax1 = yb[1], Ax2 = yb[2], As = yb[3];
  Q4<T> Aq = {yb[4], yb[5], yb[6], yb[7]};
  T Al0 = yb[8], Al1 = yb[9], Al2 = yb[10], Al3 = yb[11], Al4 = yb[12];
  T Ab0 = yb[13], Ab1 = yb[14], Ab2 = yb[15], Asb = yb[16];
  T Awa = 0, Awsa = 0, Ailb = 0, Aass = 0, Aavol = 0, Aasg = 0, AI1 = 0, Awb = 0, Awsb = 0;
  if (sgr) {
    // sa'' = sa' - wsa il0 dl,  sb'' = sb' + wsb il0 dl,  l4' = l4 + dl
    const T Adl = -wsa * il0 * As + wsb * il0 * Asb + Al4;
    Awsa -= il0 * dlg * As; Awsb += il0 * dlg * Asb;
    // dl = (-C - asg l4) / S,  C = (sb' - sa') il0,  S = (wsa + wsb) il0^2 + asg
    const T AN = Adl * iSg, AS = -Adl * dlg * iSg;
    Aasg += AS - L.l[4] * AN;
    Al4 -= asg * AN;
    Awsa += il0 * il0 * AS; Awsb += il0 * il0 * AS;
    Asb -= il0 * AN; As += il0 * AN;
  }
  if (vol) {
    // a'' = a' - wa k e,  b'' = b' + wb k e,  sa' = sa + wsa gs dl,  sb' = sb + wsb gs dl,  l3' = l3 + dl
    const T Axe = Ax0 * e0 + Ax1 * e1 + Ax2 * e2, Abe = Ab0 * e0 + Ab1 * e1 + Ab2 * e2;
    Awa -= kv * Axe; Awb += kv * Abe;
    const T Ak = wb * Abe - wa * Axe;
    T Ae0 = kv * (wb * Ab0 - wa * Ax0), Ae1 = kv * (wb * Ab1 - wa * Ax1), Ae2 = kv * (wb * Ab2 - wa * Ax2);
    T Ags = dlv * (wsa * As + wsb * Asb);
    T Adl = gs * (wsa * As + wsb * Asb) + Al3;
    Awsa += gs * dlv * As; Awsb += gs * dlv * Asb;
    // k = gx dl ilen
    T Agx = dlv * ilen * Ak;
    Adl += gx * ilen * Ak;
    T Ailen = gx * dlv * Ak;
    // dl = (-C - avol l3) / S
    const T AN = Adl * iSv, AS = -Adl * dlv * iSv;
    Aavol += AS - L.l[3] * AN;
    Al3 -= avol * AN;
    // S = (wa + wb) gx^2 + (wsa + wsb) gs^2 + avol
    Awa += gx * gx * AS; Awb += gx * gx * AS; Awsa += gs * gs * AS; Awsb += gs * gs * AS;
    Agx += T(2) * (wa + wb) * gx * AS;
    Ags += T(2) * (wsa + wsb) * gs * AS;
    // C = gx len - 1 (AC = -AN)
    Agx -= len * AN;
    T Alen = -gx * AN;
    // gs = ssum len il0 / 2,  gx = ssum^2 il0 / 4,  ssum = sa + sb
    const T Assum = (T(0.5) * il0) * (len * Ags + ssum * Agx);
    Alen += ssum * (T(0.5) * il0) * Ags;
    As += Assum; Asb += Assum;
    // len = len2 ilen,  ilen = rsq(len2),  len2 = e.e,  e = b' - a'
    Ailen += len2 * Alen;
    const T Alen2 = ilen * Alen - T(0.5) * ilen * ilen * ilen * Ailen;
    Ae0 += T(2) * e0 * Alen2; Ae1 += T(2) * e1 * Alen2; Ae2 += T(2) * e2 * Alen2;
    Ab0 += Ae0; Ab1 += Ae1; Ab2 += Ae2;
    Ax0 -= Ae0; Ax1 -= Ae1; Ax2 -= Ae2;
  }
  if (ss) {
    // q' = n / |n|,  n = q + [rho, 0] (x) q
    const Q4<T> An = normalize_vjp(n, inn, Aq);
    Aq = {An.x - An.w * rho0 - (rho1 * An.z - rho2 * An.y), An.y - An.w * rho1 - (rho2 * An.x - rho0 * An.z),
          An.z - An.w * rho2 - (rho0 * An.y - rho1 * An.x), An.w + (rho0 * An.x + rho1 * An.y + rho2 * An.z)};
    const T Ar0 = q.w * An.x - q.z * An.y + q.y * An.z - q.x * An.w;
    const T Ar1 = q.z * An.x + q.w * An.y - q.x * An.z - q.y * An.w;
    const T Ar2 = -q.y * An.x + q.x * An.y + q.w * An.z - q.z * An.w;
    // rho = nI (d x g),  nI = -I1 / 2
    AI1 -= T(0.5) * ((d1 * g2 - d2 * g1) * Ar0 + (d2 * g0 - d0 * g2) * Ar1 + (d0 * g1 - d1 * g0) * Ar2);
    T Ad0 = nI * (g1 * Ar2 - g2 * Ar1), Ad1 = nI * (g2 * Ar0 - g0 * Ar2), Ad2 = nI * (g0 * Ar1 - g1 * Ar0);
    T Ag0 = nI * (Ar1 * d2 - Ar2 * d1), Ag1 = nI * (Ar2 * d0 - Ar0 * d2), Ag2 = nI * (Ar0 * d1 - Ar1 * d0);
    // a' = a - wa ilb g,  b' = b + wb ilb g,  l' = l + g
    const T Afa = -(Ax0 * g0 + Ax1 * g1 + Ax2 * g2), Afb = Ab0 * g0 + Ab1 * g1 + Ab2 * g2;
    Awa += ilb * Afa; Awb += ilb * Afb; Ailb += wa * Afa + wb * Afb;
    const T fa = wa * ilb, fb = wb * ilb;
    Ag0 += fb * Ab0 - fa * Ax0 + Al0; Ag1 += fb * Ab1 - fa * Ax1 + Al1; Ag2 += fb * Ab2 - fa * Ax2 + Al2;
    // g = r ik2 + ee d,  ee = dr (ik1 - ik2),  dr = d.r
    T Ar_0 = ik2 * Ag0, Ar_1 = ik2 * Ag1, Ar_2 = ik2 * Ag2;
    T Aik2 = r0 * Ag0 + r1 * Ag1 + r2 * Ag2;
    const T Aee = d0 * Ag0 + d1 * Ag1 + d2 * Ag2;
    Ad0 += ee * Ag0; Ad1 += ee * Ag1; Ad2 += ee * Ag2;
    const T Adr = (ik1 - ik2) * Aee;
    const T Aik1 = dr * Aee;
    Aik2 -= dr * Aee;
    Ad0 += r0 * Adr; Ad1 += r1 * Adr; Ad2 += r2 * Adr;
    Ar_0 += d0 * Adr; Ar_1 += d1 * Adr; Ar_2 += d2 * Adr;
    // r = -C - ass l,  C = (b - a) ilb - d  (AC = -Ar)
    Aass -= L.l[0] * Ar_0 + L.l[1] * Ar_1 + L.l[2] * Ar_2;
    Al0 -= ass * Ar_0; Al1 -= ass * Ar_1; Al2 -= ass * Ar_2;
    Ab0 -= ilb * Ar_0; Ab1 -= ilb * Ar_1; Ab2 -= ilb * Ar_2;
    Ax0 += ilb * Ar_0; Ax1 += ilb * Ar_1; Ax2 += ilb * Ar_2;
    Ailb -= (b0 - L.x0) * Ar_0 + (b1 - L.x1) * Ar_1 + (b2 - L.x2) * Ar_2;
    Ad0 += Ar_0; Ad1 += Ar_1; Ad2 += Ar_2;
    // ik1 = 1 / k1,  ik2 = 1 / (k1 + I1),  k1 = (wa + wb) ilb^2 + ass
    const T Ak1 = -ik1 * ik1 * Aik1 - ik2 * ik2 * Aik2;
    AI1 -= ik2 * ik2 * Aik2;
    Awa += ilb * ilb * Ak1; Awb += ilb * ilb * Ak1; Ailb += T(2) * (wa + wb) * ilb * Ak1; Aass += Ak1;
    // d = (P0 tw, P1 tw, (nb - na) in),  tw = 2 in,  in = 1 / (na + nb)
    const T AP0 = T(2) * in * Ad0, AP1 = T(2) * in * Ad1;
    const T Ain = T(2) * (P0 * Ad0 + P1 * Ad1) + (nb - na) * Ad2;
    const T t = -in * in * Ain;
    const T Ana = t - in * Ad2, Anb = t + in * Ad2;
    Aq.x += q.z * AP0 - q.w * AP1 + T(2) * q.x * Ana;
    Aq.y += q.w * AP0 + q.z * AP1 + T(2) * q.y * Ana;
    Aq.z += q.x * AP0 + q.y * AP1 + T(2) * q.z * Anb;
    Aq.w += q.y * AP0 - q.x * AP1 + T(2) * q.w * Anb;
  }
  xb[0] = Ax0; xb[1] = Ax1; xb[2] = Ax2; xb[3] = As;
  xb[4] = Aq.x; xb[5] = Aq.y; xb[6] = Aq.z; xb[7] = Aq.w;
  xb[8] = Al0; xb[9] = Al1; xb[10] = Al2; xb[11] = Al3; xb[12] = Al4;
  xb[13] = Ab0; xb[14] = Ab1; xb[15] = Ab2; xb[16] = Asb;
  xb[17] = Awa; xb[18] = Awsa; xb[19] = Ailb; xb[20] = Aass; xb[21] = Aavol; xb[22] = Aasg; xb[23] = AI1;
  xb[24] = Awb; xb[25] = Awsb;
}

// Bend-twist between slot L's edge and the next edge (bt_update).
// Inputs (16): q0..q3 l5 l6 l7 | b0..b3 sb | Ia Ib wsb abt      Outputs (12): q0..q3 l5..l7 | b0..b3 sb
template <class T>
__device__ void bt_vjp(const Slot<T>& L, T b0, T b1, T b2, T b3, T sb, T Ib, T wsb, const T (&yb)[12], T (&xb)[16]) {
  const Q4<T> qa = {L.q0, L.q1, L.q2, L.q3}, qb = {b0, b1, b2, b3};
  // ---- forward recompute
  const Q4<T> r = qmul(qconj(qa), qb);
  const T sg = (r.w < T(0)) ? T(-1) : T(1);
  const T v0 = sg * r.x, v1 = sg * r.y, v2 = sg * r.z, w = sg * r.w;
  const T c = L.cbt, sc = sb * c;
  const T v0s = v0 * v0, v1s = v1 * v1;
  const T th0 = v0 * v2 + w * v1, th1 = v1 * v2 - w * v0, th2 = T(0.5) - (v0s + v1s);
  const T Ia = L.I1, at = L.abt;
  const T sc2 = sc * sc;
  const T m = sc2 * (T(0.25) * (Ia + Ib));
  const T sgm = rcp(m + at);
  const T wc2 = wsb * c * c;
  const T qs = (wc2 - m) * sgm;
  const T ks = sc2 * sgm;
  const T hp = ks * (T(0.125) * (Ia + Ib)), hm = ks * (T(0.125) * (Ia - Ib));
  const T pv0 = qs * v0, pv1 = qs * v1, pv2 = qs * v2;
  const T s00 = T(1) + pv0 * v0 - hp * v1s;
  const T s11 = T(1) + pv1 * v1 - hp * v0s;
  const T s22 = (T(1) - T(0.5) * at * sgm) + pv2 * v2 - hp * (w * w);
  const T s01 = (qs + hp) * (v0 * v1);
  const T s02 = pv0 * v2 + hm * (v1 * w);
  const T s12 = pv1 * v2 - hm * (v0 * w);
  const T C0 = sc * v0 - L.db0, C1 = sc * v1 - L.db1, C2 = sc * v2 - L.db2;
  const T r0 = -C0 - at * L.l[5], r1 = -C1 - at * L.l[6], r2 = -C2 - T(0.5) * at * L.l[7];
  const T A00 = s11 * s22 - s12 * s12, A01 = s02 * s12 - s01 * s22, A02 = s01 * s12 - s02 * s11;
  const T A11 = s00 * s22 - s02 * s02, A12 = s01 * s02 - s00 * s12, A22 = s00 * s11 - s01 * s01;
  const T idt = rcp(s00 * A00 + s01 * A01 + s02 * A02);
  const T m0 = (A00 * r0 + A01 * r1 + A02 * r2) * idt;   // s^-1 r
  const T m1 = (A01 * r0 + A11 * r1 + A12 * r2) * idt;
  const T m2 = (A02 * r0 + A12 * r1 + A22 * r2) * idt;
  const T g0 = sgm * m0, g1 = sgm * m1, g2 = sgm * m2;
  const T e0 = w * g0 + (v1 * g2 - v2 * g1);
  const T e1 = w * g1 + (v2 * g0 - v0 * g2);
  const T e2 = w * g2 + (v0 * g1 - v1 * g0);
  const T ka = sc * (T(-0.25) * Ia), ka2 = sc * (T(-0.125) * Ia);
  const T te = th0 * e0 + th1 * e1 + th2 * e2;
  const T te2 = te + te;
  const T kb = (sg * sc) * (T(0.25) * Ib);
  const Q4<T> ha = {ka * e0, ka * e1, ka2 * e2, T(0)};
  const Q4<T> qha = qmul(qa, ha);
  const Q4<T> na = {qa.x + qha.x, qa.y + qha.y, qa.z + qha.z, qa.w + qha.w};
  const T ina = rsq(na.x * na.x + na.y * na.y + na.z * na.z + na.w * na.w);
  const T u0 = e0 - te2 * th0, u1 = e1 - te2 * th1, u2 = e2 - te2 * th2;
  const Q4<T> hb = {kb * u0, kb * u1, kb * u2, T(0)};
  const Q4<T> rt = {v0, v1, v2, w};
  const Q4<T> p = qmul(hb, rt);
  const Q4<T> qp = qmul(qa, p);
  const Q4<T> nb = {qb.x + qp.x, qb.y + qp.y, qb.z + qp.z, qb.w + qp.w};
  const T inb = rsq(nb.x * nb.x + nb.y * nb.y + nb.z * nb.z + nb.w * nb.w);
  // ---- reverse sweep
  Q4<T> Aqa = {0, 0, 0, 0};
  T Al5 = yb[4], Al6 = yb[5], Al7 = yb[6];
  T Asb = yb[11];
  T AIa = 0, AIb = 0, Awsb = 0, Aat = 0;
  // sb' = sb + wsb c (v.g)
  T Av0 = wsb * c * g0 * Asb, Av1 = wsb * c * g1 * Asb, Av2 = wsb * c * g2 * Asb, Aw = 0;
  T Ag0 = wsb * c * v0 * Asb, Ag1 = wsb * c * v1 * Asb, Ag2 = wsb * c * v2 * Asb;
  Awsb += c * (v0 * g0 + v1 * g1 + v2 * g2) * Asb;
  // qb' = nb / |nb|,  nb = qb + qa (x) p,  p = [hb, 0] (x) (v, w)
  const Q4<T> Anb = normalize_vjp(nb, inb, Q4<T>{yb[7], yb[8], yb[9], yb[10]});
  Q4<T> Aqb = Anb;
  {
    const Q4<T> t = qmul(Anb, qconj(p));
    Aqa.x += t.x; Aqa.y += t.y; Aqa.z += t.z; Aqa.w += t.w;
  }
  const Q4<T> Ap = qmul(qconj(qa), Anb);
  const Q4<T> Ahb = qmul(Ap, qconj(rt));
  {
    const Q4<T> t = qmul(Q4<T>{-hb.x, -hb.y, -hb.z, T(0)}, Ap);
    Av0 += t.x; Av1 += t.y; Av2 += t.z; Aw += t.w;
  }
  // hb = kb (e - te2 th)
  const T Akb = Ahb.x * u0 + Ahb.y * u1 + Ahb.z * u2;
  T Ae0 = kb * Ahb.x, Ae1 = kb * Ahb.y, Ae2 = kb * Ahb.z;
  const T Ate2 = -kb * (th0 * Ahb.x + th1 * Ahb.y + th2 * Ahb.z);
  T Ath0 = -kb * te2 * Ahb.x, Ath1 = -kb * te2 * Ahb.y, Ath2 = -kb * te2 * Ahb.z;
  // qa' = na / |na|,  na = qa + qa (x) [ha, 0]
  const Q4<T> Ana = normalize_vjp(na, ina, Q4<T>{yb[0], yb[1], yb[2], yb[3]});
  {
    const Q4<T> t = qmul(Ana, Q4<T>{-ha.x, -ha.y, -ha.z, T(0)});
    Aqa.x += Ana.x + t.x; Aqa.y += Ana.y + t.y; Aqa.z += Ana.z + t.z; Aqa.w += Ana.w + t.w;
  }
  const Q4<T> Aha = qmul(qconj(qa), Ana);
  // ha = (ka e0, ka e1, ka2 e2)
  const T Aka = Aha.x * e0 + Aha.y * e1, Aka2 = Aha.z * e2;
  Ae0 += ka * Aha.x; Ae1 += ka * Aha.y; Ae2 += ka2 * Aha.z;
  // kb = sg sc Ib / 4,  ka = -sc Ia / 4,  ka2 = -sc Ia / 8
  T Asc = sg * T(0.25) * Ib * Akb - T(0.25) * Ia * Aka - T(0.125) * Ia * Aka2;
  AIb += sg * sc * T(0.25) * Akb;
  AIa -= sc * (T(0.25) * Aka + T(0.125) * Aka2);
  // te2 = 2 te,  te = th.e
  const T Ate = T(2) * Ate2;
  Ath0 += e0 * Ate; Ath1 += e1 * Ate; Ath2 += e2 * Ate;
  Ae0 += th0 * Ate; Ae1 += th1 * Ate; Ae2 += th2 * Ate;
  // e = w g + v x g
  Aw += Ae0 * g0 + Ae1 * g1 + Ae2 * g2;
  Ag0 += w * Ae0 + (Ae1 * v2 - Ae2 * v1);
  Ag1 += w * Ae1 + (Ae2 * v0 - Ae0 * v2);
  Ag2 += w * Ae2 + (Ae0 * v1 - Ae1 * v0);
  Av0 += g1 * Ae2 - g2 * Ae1;
  Av1 += g2 * Ae0 - g0 * Ae2;
  Av2 += g0 * Ae1 - g1 * Ae0;
  // l' = l + g
  Ag0 += Al5; Ag1 += Al6; Ag2 += Al7;
  // g = sgm s^-1 r:  r_bar = sgm s^-1 g_bar,  sgm_bar = g_bar . s^-1 r,  s_bar = -(s^-1 g_bar) g^T
  const T z0 = (A00 * Ag0 + A01 * Ag1 + A02 * Ag2) * idt;
  const T z1 = (A01 * Ag0 + A11 * Ag1 + A12 * Ag2) * idt;
  const T z2 = (A02 * Ag0 + A12 * Ag1 + A22 * Ag2) * idt;
  const T Ar0 = sgm * z0, Ar1 = sgm * z1, Ar2 = sgm * z2;
  T Asgm = Ag0 * m0 + Ag1 * m1 + Ag2 * m2;
  const T As00 = -z0 * g0, As11 = -z1 * g1, As22 = -z2 * g2;
  const T As01 = -(z0 * g1 + z1 * g0), As02 = -(z0 * g2 + z2 * g0), As12 = -(z1 * g2 + z2 * g1);
  // r = -C - at (l5, l6, l7 / 2),  C = sc v - db
  Aat -= L.l[5] * Ar0 + L.l[6] * Ar1 + T(0.5) * L.l[7] * Ar2;
  Al5 -= at * Ar0; Al6 -= at * Ar1; Al7 -= T(0.5) * at * Ar2;
  Asc -= v0 * Ar0 + v1 * Ar1 + v2 * Ar2;
  Av0 -= sc * Ar0; Av1 -= sc * Ar1; Av2 -= sc * Ar2;
  // s assembly
  T Aqs = v0s * As00 + v1s * As11 + v2 * v2 * As22 + v0 * v1 * As01 + v0 * v2 * As02 + v1 * v2 * As12;
  T Ahp = -v1s * As00 - v0s * As11 - w * w * As22 + v0 * v1 * As01;
  const T Ahm = v1 * w * As02 - v0 * w * As12;
  Av0 += T(2) * qs * v0 * As00 - T(2) * hp * v0 * As11 + (qs + hp) * v1 * As01 + qs * v2 * As02 - hm * w * As12;
  Av1 += T(2) * qs * v1 * As11 - T(2) * hp * v1 * As00 + (qs + hp) * v0 * As01 + hm * w * As02 + qs * v2 * As12;
  Av2 += T(2) * qs * v2 * As22 + qs * v0 * As02 + qs * v1 * As12;
  Aw += -T(2) * hp * w * As22 + hm * v1 * As02 - hm * v0 * As12;
  Aat -= T(0.5) * sgm * As22;
  Asgm -= T(0.5) * at * As22;
  // hp = ks (Ia + Ib) / 8,  hm = ks (Ia - Ib) / 8
  const T Aks = T(0.125) * ((Ia + Ib) * Ahp + (Ia - Ib) * Ahm);
  AIa += T(0.125) * ks * (Ahp + Ahm);
  AIb += T(0.125) * ks * (Ahp - Ahm);
  // ks = sc2 sgm,  qs = (wc2 - m) sgm
  T Asc2 = sgm * Aks;
  Asgm += sc2 * Aks + (wc2 - m) * Aqs;
  Awsb += c * c * sgm * Aqs;
  T Am = -sgm * Aqs;
  // sgm = 1 / (m + at)
  const T tq = -sgm * sgm * Asgm;
  Am += tq; Aat += tq;
  // m = sc2 (Ia + Ib) / 4,  sc2 = sc^2,  sc = sb c
  Asc2 += T(0.25) * (Ia + Ib) * Am;
  AIa += T(0.25) * sc2 * Am; AIb += T(0.25) * sc2 * Am;
  Asc += T(2) * sc * Asc2;
  Asb += c * Asc;
  // t/2 = (v0 v2 + w v1, v1 v2 - w v0, 1/2 - v0^2 - v1^2)
  Av0 += v2 * Ath0 - w * Ath1 - T(2) * v0 * Ath2;
  Av1 += w * Ath0 + v2 * Ath1 - T(2) * v1 * Ath2;
  Av2 += v0 * Ath0 + v1 * Ath1;
  Aw += v1 * Ath0 - v0 * Ath1;
  // (v, w) = sg r,  r = conj(qa) (x) qb
  const Q4<T> Ar = {sg * Av0, sg * Av1, sg * Av2, sg * Aw};
  {
    const Q4<T> t = qmul(qa, Ar);
    Aqb.x += t.x; Aqb.y += t.y; Aqb.z += t.z; Aqb.w += t.w;
    const Q4<T> u = qmul(qb, qconj(Ar));
    Aqa.x += u.x; Aqa.y += u.y; Aqa.z += u.z; Aqa.w += u.w;
  }
  xb[0] = Aqa.x; xb[1] = Aqa.y; xb[2] = Aqa.z; xb[3] = Aqa.w;
  xb[4] = Al5; xb[5] = Al6; xb[6] = Al7;
  xb[7] = Aqb.x; xb[8] = Aqb.y; xb[9] = Aqb.z; xb[10] = Aqb.w; xb[11] = Asb;
  xb[12] = AIa; xb[13] = AIb; xb[14] = Awsb; xb[15] = Aat;
}

// Angular velocity from the quaternions after / before the substep (omega_of):
// o = sgf Im(q (x) conj(p)), sgf = +-2 / h by the sign of the real part.
// Inputs (8): q0..q3 p0..p3       Outputs (3): o0 o1 o2
template <class T>
__device__ void omega_vjp(const Slot<T>& L, T ih, const T (&yb)[3], T (&xb)[8]) {
  const Q4<T> q = {L.q0, L.q1, L.q2, L.q3}, p = {L.qp0, L.qp1, L.qp2, L.qp3};
  const Q4<T> r = qmul(q, qconj(p));
  const T sgf = (r.w < T(0)) ? T(-2) * ih : T(2) * ih;
  const Q4<T> Ar = {sgf * yb[0], sgf * yb[1], sgf * yb[2], T(0)};
  const Q4<T> Aq = qmul(Ar, p);                 // r = R(conj p) q
  const Q4<T> Ap = qmul(qconj(Ar), q);          // r = L(q) conj(p)
  xb[0] = Aq.x; xb[1] = Aq.y; xb[2] = Aq.z; xb[3] = Aq.w;
  xb[4] = Ap.x; xb[5] = Ap.y; xb[6] = Ap.z; xb[7] = Ap.w;
}

// Predicted quaternion normalize(q + [a, 0] (x) q), a = h w / 2 (qrot_world).
// Inputs (7): q0..q3 w0 w1 w2     Outputs (4): q0..q3
template <class T>
__device__ void qpredict_vjp(T q0, T q1, T q2, T q3, T w0, T w1, T w2, T h, const T (&yb)[4], T (&xb)[7]) {
  const Q4<T> q = {q0, q1, q2, q3};
  const Q4<T> a = {T(0.5) * (h * w0), T(0.5) * (h * w1), T(0.5) * (h * w2), T(0)};
  const Q4<T> aq = qmul(a, q);
  const Q4<T> n = {q.x + aq.x, q.y + aq.y, q.z + aq.z, q.w + aq.w};
  const T inv = rsq(n.x * n.x + n.y * n.y + n.z * n.z + n.w * n.w);
  const Q4<T> An = normalize_vjp(n, inv, Q4<T>{yb[0], yb[1], yb[2], yb[3]});
  const Q4<T> t = qmul(Q4<T>{-a.x, -a.y, -a.z, T(0)}, An);   // n = q + L(a) q
  const Q4<T> Aa = qmul(An, qconj(q));                      // n = q + R(q) a
  xb[0] = An.x + t.x; xb[1] = An.y + t.y; xb[2] = An.z + t.z; xb[3] = An.w + t.w;
  xb[4] = T(0.5) * h * Aa.x; xb[5] = T(0.5) * h * Aa.y; xb[6] = T(0.5) * h * Aa.z;
}

// ---------------------------------------------------------------- adjoint state

template <class T>
struct SAdj {
  T x0, x1, x2, s, q0, q1, q2, q3, l[8];   // adjoint of the current state
  T v0, v1, v2, sd, o0, o1, o2;            // of the substep-end velocities
  T xp0, xp1, xp2, sp, qp0, qp1, qp2, qp3; // of the substep-start copies
  T w, ws, ilb, ass, avol, asg, abt, I1, inert;  // of the slot's parameters
};

template <class T>
__device__ __forceinline__ void zero_adj(SAdj<T>& a) {
  a.x0 = a.x1 = a.x2 = a.s = a.q0 = a.q1 = a.q2 = a.q3 = T(0);
#pragma unroll
  for (int i = 0; i < 8; ++i) a.l[i] = T(0);
  a.v0 = a.v1 = a.v2 = a.sd = a.o0 = a.o1 = a.o2 = T(0);
  a.xp0 = a.xp1 = a.xp2 = a.sp = a.qp0 = a.qp1 = a.qp2 = a.qp3 = T(0);
  a.w = a.ws = a.ilb = a.ass = a.avol = a.asg = a.abt = a.I1 = a.inert = T(0);
}

// Snapshots of the pre-pass state, stored field-major over the scene's lanes for coalesced
// access: before an edge pass the values it reads and changes (x, s, q, the stretch-shear,
// volume and scale-gradient multipliers) of both slots, 26 per lane; before a bend-twist
// pass q, s and the bend-twist multipliers of both slots, 16 per lane.  One iteration's four
// snapshots take kSnapPerIter values per lane.
__host__ __device__ constexpr int snap_offset(int k) { return k < 2 ? k * kSnapEdge : 2 * kSnapEdge + (k - 2) * kSnapBt; }

template <class T>
__device__ __forceinline__ void snap_edge_store(T* base, size_t NL, const Slot<T>& A, const Slot<T>& B) {
  const T v[kSnapEdge] = {A.x0, A.x1, A.x2, A.s, A.q0, A.q1, A.q2, A.q3, A.l[0], A.l[1], A.l[2], A.l[3], A.l[4],
                          B.x0, B.x1, B.x2, B.s, B.q0, B.q1, B.q2, B.q3, B.l[0], B.l[1], B.l[2], B.l[3], B.l[4]};
#pragma unroll
  for (int i = 0; i < kSnapEdge; ++i) base[(size_t)i * NL] = v[i];
}
template <class T>
__device__ __forceinline__ void snap_bt_store(T* base, size_t NL, const Slot<T>& A, const Slot<T>& B) {
  const T v[kSnapBt] = {A.q0, A.q1, A.q2, A.q3, A.s, A.l[5], A.l[6], A.l[7],
                        B.q0, B.q1, B.q2, B.q3, B.s, B.l[5], B.l[6], B.l[7]};
#pragma unroll
  for (int i = 0; i < kSnapBt; ++i) base[(size_t)i * NL] = v[i];
}
template <class T, int N>
__device__ __forceinline__ void snap_load(const T* base, size_t NL, T (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = base[(size_t)i * NL];
}
template <class T>
__device__ __forceinline__ void snap_edge_apply(const T (&v)[kSnapEdge], Slot<T>& A, Slot<T>& B) {
  A.x0 = v[0]; A.x1 = v[1]; A.x2 = v[2]; A.s = v[3]; A.q0 = v[4]; A.q1 = v[5]; A.q2 = v[6]; A.q3 = v[7];
  A.l[0] = v[8]; A.l[1] = v[9]; A.l[2] = v[10]; A.l[3] = v[11]; A.l[4] = v[12];
  B.x0 = v[13]; B.x1 = v[14]; B.x2 = v[15]; B.s = v[16]; B.q0 = v[17]; B.q1 = v[18]; B.q2 = v[19]; B.q3 = v[20];
  B.l[0] = v[21]; B.l[1] = v[22]; B.l[2] = v[23]; B.l[3] = v[24]; B.l[4] = v[25];
}
template <class T>
__device__ __forceinline__ void snap_bt_apply(const T (&v)[kSnapBt], Slot<T>& A, Slot<T>& B) {
  A.q0 = v[0]; A.q1 = v[1]; A.q2 = v[2]; A.q3 = v[3]; A.s = v[4]; A.l[5] = v[5]; A.l[6] = v[6]; A.l[7] = v[7];
  B.q0 = v[8]; B.q1 = v[9]; B.q2 = v[10]; B.q3 = v[11]; B.s = v[12]; B.l[5] = v[13]; B.l[6] = v[14]; B.l[7] = v[15];
}

// ---------------------------------------------------------------- reverse passes

// Each lane forms the local VJP of the projection it owns in this pass (its A edge or its B
// edge; none when neither has the colour).  The right end of a B edge is the next lane's A:
// its pre-pass values come down one lane, its adjoint goes back up.
// The edge VJP of slot L with right end (b, sb; wb, wsb), result written to the adjoints a
// (slot) and its right end (bx, bs, bw, bws).
template <class T>
__device__ __forceinline__ void edge_vjp_apply(const Slot<T>& L, SAdj<T>& a, T b0, T b1, T b2, T sb, T wb, T wsb,
                                               T& bx0, T& bx1, T& bx2, T& bs, T& bw, T& bws) {
  const T yb[17] = {a.x0, a.x1, a.x2, a.s, a.q0, a.q1, a.q2, a.q3, a.l[0], a.l[1], a.l[2], a.l[3], a.l[4],
                    bx0, bx1, bx2, bs};
  T xb[26];
  edge_vjp(L, b0, b1, b2, sb, wb, wsb, yb, xb);
  a.x0 = xb[0]; a.x1 = xb[1]; a.x2 = xb[2]; a.s = xb[3];
  a.q0 = xb[4]; a.q1 = xb[5]; a.q2 = xb[6]; a.q3 = xb[7];
  a.l[0] = xb[8]; a.l[1] = xb[9]; a.l[2] = xb[10]; a.l[3] = xb[11]; a.l[4] = xb[12];
  a.w += xb[17]; a.ws += xb[18]; a.ilb += xb[19]; a.ass += xb[20]; a.avol += xb[21]; a.asg += xb[22];
  a.I1 += xb[23];
  bx0 = xb[13]; bx1 = xb[14]; bx2 = xb[15]; bs = xb[16]; bw += xb[24]; bws += xb[25];
}

// The bend-twist VJP of slot L with the next edge (qb, sb; Ib, wsb), result written to the
// adjoints a (slot) and the next edge's (bq, bs, bI, bws).
template <class T>
__device__ __forceinline__ void bt_vjp_apply(const Slot<T>& L, SAdj<T>& a, T b0, T b1, T b2, T b3, T sb, T Ib, T wsb,
                                             T& bq0, T& bq1, T& bq2, T& bq3, T& bs, T& bI, T& bws) {
  const T yb[12] = {a.q0, a.q1, a.q2, a.q3, a.l[5], a.l[6], a.l[7], bq0, bq1, bq2, bq3, bs};
  T xb[16];
  bt_vjp(L, b0, b1, b2, b3, sb, Ib, wsb, yb, xb);
  a.q0 = xb[0]; a.q1 = xb[1]; a.q2 = xb[2]; a.q3 = xb[3];
  a.l[5] = xb[4]; a.l[6] = xb[5]; a.l[7] = xb[6];
  a.I1 += xb[12]; a.abt += xb[15];
  bq0 = xb[7]; bq1 = xb[8]; bq2 = xb[9]; bq3 = xb[10]; bs = xb[11]; bI += xb[13]; bws += xb[14];
}

template <class T, bool EVEN>
__device__ void pass_edges_vjp(Lane2<T>& P, SAdj<T>& aA, SAdj<T>& aB, int colour) {
  if constexpr (EVEN) {   // slot A holds the even pills (the forward's lane-local passes)
    if (colour == 0) {
      if (P.A.f & F_EDGE)
        edge_vjp_apply(P.A, aA, P.B.x0, P.B.x1, P.B.x2, P.B.s, P.B.w, P.B.ws, aB.x0, aB.x1, aB.x2, aB.s, aB.w, aB.ws);
      return;
    }
    const T n0 = dn(P.A.x0), n1 = dn(P.A.x1), n2 = dn(P.A.x2), ns = dn(P.A.s);
    T r0 = dn(aA.x0), r1 = dn(aA.x1), r2 = dn(aA.x2), rs = dn(aA.s), rw = T(0), rws = T(0);
    if (P.B.f & F_EDGE) edge_vjp_apply(P.B, aB, n0, n1, n2, ns, P.wN, P.wsN, r0, r1, r2, rs, rw, rws);
    r0 = up(r0); r1 = up(r1); r2 = up(r2); rs = up(rs); rw = up(rw); rws = up(rws);
    if ((P.A.f & F_VALID) && !(P.A.f & F_FIRST)) {
      aA.x0 = r0; aA.x1 = r1; aA.x2 = r2; aA.s = rs; aA.w += rw; aA.ws += rws;
    }
    return;
  }
  const T n0 = dn(P.A.x0), n1 = dn(P.A.x1), n2 = dn(P.A.x2), ns = dn(P.A.s);       // pre-pass next slot A
  const T g0 = dn(aA.x0), g1 = dn(aA.x1), g2 = dn(aA.x2), gs = dn(aA.s);            // adjoint of its post-pass value
  const bool useA = (P.A.f & F_EDGE) && colour_is(P.A.f, colour);
  const bool useB = !useA && (P.B.f & F_EDGE) && colour_is(P.B.f, colour);
  T r0 = T(0), r1 = T(0), r2 = T(0), rs = T(0), rw = T(0), rws = T(0);
  if (useA || useB) {
    const Slot<T>& L = useB ? P.B : P.A;
    SAdj<T>& a = useB ? aB : aA;
    const T yb[17] = {a.x0, a.x1, a.x2, a.s, a.q0, a.q1, a.q2, a.q3, a.l[0], a.l[1], a.l[2], a.l[3], a.l[4],
                      useB ? g0 : aB.x0, useB ? g1 : aB.x1, useB ? g2 : aB.x2, useB ? gs : aB.s};
    T xb[26];
    edge_vjp(L, useB ? n0 : P.B.x0, useB ? n1 : P.B.x1, useB ? n2 : P.B.x2, useB ? ns : P.B.s,
             useB ? P.wN : P.B.w, useB ? P.wsN : P.B.ws, yb, xb);
    a.x0 = xb[0]; a.x1 = xb[1]; a.x2 = xb[2]; a.s = xb[3];
    a.q0 = xb[4]; a.q1 = xb[5]; a.q2 = xb[6]; a.q3 = xb[7];
    a.l[0] = xb[8]; a.l[1] = xb[9]; a.l[2] = xb[10]; a.l[3] = xb[11]; a.l[4] = xb[12];
    a.w += xb[17]; a.ws += xb[18]; a.ilb += xb[19]; a.ass += xb[20]; a.avol += xb[21]; a.asg += xb[22];
    a.I1 += xb[23];
    if (useA) {
      aB.x0 = xb[13]; aB.x1 = xb[14]; aB.x2 = xb[15]; aB.s = xb[16];
      aB.w += xb[24]; aB.ws += xb[25];
    } else {
      r0 = xb[13]; r1 = xb[14]; r2 = xb[15]; rs = xb[16]; rw = xb[24]; rws = xb[25];
    }
  }
  r0 = up(r0); r1 = up(r1); r2 = up(r2); rs = up(rs); rw = up(rw); rws = up(rws);
  if ((P.A.f & F_VALID) && !(P.A.f & F_FIRST) && !colour_is(P.A.f, colour)) {
    aA.x0 = r0; aA.x1 = r1; aA.x2 = r2; aA.s = rs; aA.w += rw; aA.ws += rws;
  }
}

template <class T, bool EVEN>
__device__ void pass_bt_vjp(Lane2<T>& P, SAdj<T>& aA, SAdj<T>& aB, int colour) {
  if constexpr (EVEN) {
    if (colour == 0) {
      if ((P.A.f & F_BT) && (P.A.f & F_BTEN))
        bt_vjp_apply(P.A, aA, P.B.q0, P.B.q1, P.B.q2, P.B.q3, P.B.s, P.B.I1, P.B.ws, aB.q0, aB.q1, aB.q2, aB.q3, aB.s,
                     aB.I1, aB.ws);
      return;
    }
    const T n0 = dn(P.A.q0), n1 = dn(P.A.q1), n2 = dn(P.A.q2), n3 = dn(P.A.q3), ns = dn(P.A.s);
    T r0 = dn(aA.q0), r1 = dn(aA.q1), r2 = dn(aA.q2), r3 = dn(aA.q3), rs = dn(aA.s), rI = T(0), rws = T(0);
    if ((P.B.f & F_BT) && (P.B.f & F_BTEN))
      bt_vjp_apply(P.B, aB, n0, n1, n2, n3, ns, P.I1N, P.wsN, r0, r1, r2, r3, rs, rI, rws);
    r0 = up(r0); r1 = up(r1); r2 = up(r2); r3 = up(r3); rs = up(rs); rI = up(rI); rws = up(rws);
    if ((P.A.f & F_EDGE) && !(P.A.f & F_FIRST) && (P.A.f & F_BTEN)) {
      aA.q0 = r0; aA.q1 = r1; aA.q2 = r2; aA.q3 = r3; aA.s = rs; aA.I1 += rI; aA.ws += rws;
    }
    return;
  }
  const T n0 = dn(P.A.q0), n1 = dn(P.A.q1), n2 = dn(P.A.q2), n3 = dn(P.A.q3), ns = dn(P.A.s);
  const T g0 = dn(aA.q0), g1 = dn(aA.q1), g2 = dn(aA.q2), g3 = dn(aA.q3), gs = dn(aA.s);
  const bool useA = (P.A.f & F_BT) && (P.A.f & F_BTEN) && colour_is(P.A.f, colour);
  const bool useB = !useA && (P.B.f & F_BT) && (P.B.f & F_BTEN) && colour_is(P.B.f, colour);
  T r0 = T(0), r1 = T(0), r2 = T(0), r3 = T(0), rs = T(0), rI = T(0), rws = T(0);
  if (useA || useB) {
    const Slot<T>& L = useB ? P.B : P.A;
    SAdj<T>& a = useB ? aB : aA;
    const T yb[12] = {a.q0, a.q1, a.q2, a.q3, a.l[5], a.l[6], a.l[7],
                      useB ? g0 : aB.q0, useB ? g1 : aB.q1, useB ? g2 : aB.q2, useB ? g3 : aB.q3, useB ? gs : aB.s};
    T xb[16];
    bt_vjp(L, useB ? n0 : P.B.q0, useB ? n1 : P.B.q1, useB ? n2 : P.B.q2, useB ? n3 : P.B.q3, useB ? ns : P.B.s,
           useB ? P.I1N : P.B.I1, useB ? P.wsN : P.B.ws, yb, xb);
    a.q0 = xb[0]; a.q1 = xb[1]; a.q2 = xb[2]; a.q3 = xb[3];
    a.l[5] = xb[4]; a.l[6] = xb[5]; a.l[7] = xb[6];
    a.I1 += xb[12]; a.abt += xb[15];
    if (useA) {
      aB.q0 = xb[7]; aB.q1 = xb[8]; aB.q2 = xb[9]; aB.q3 = xb[10]; aB.s = xb[11];
      aB.I1 += xb[13]; aB.ws += xb[14];
    } else {
      r0 = xb[7]; r1 = xb[8]; r2 = xb[9]; r3 = xb[10]; rs = xb[11]; rI = xb[13]; rws = xb[14];
    }
  }
  r0 = up(r0); r1 = up(r1); r2 = up(r2); r3 = up(r3); rs = up(rs); rI = up(rI); rws = up(rws);
  if ((P.A.f & F_EDGE) && !(P.A.f & F_FIRST) && (P.A.f & F_BTEN) && !colour_is(P.A.f, colour)) {
    aA.q0 = r0; aA.q1 = r1; aA.q2 = r2; aA.q3 = r3; aA.s = rs; aA.I1 += rI; aA.ws += rws;
  }
}

template <class T>
__device__ __forceinline__ void velocity_vjp(const Slot<T>& L, SAdj<T>& a, T ih) {
  if (!(L.f & F_VALID)) return;
  if (L.w > T(0)) {
    a.x0 += a.v0 * ih; a.x1 += a.v1 * ih; a.x2 += a.v2 * ih;
    a.xp0 -= a.v0 * ih; a.xp1 -= a.v1 * ih; a.xp2 -= a.v2 * ih;
  }
  a.s += a.sd * ih;
  a.sp -= a.sd * ih;
  if (L.f & F_EDGE) {
    const T yb[3] = {a.o0, a.o1, a.o2};
    T xb[8];
    omega_vjp(L, ih, yb, xb);
    a.q0 += xb[0]; a.q1 += xb[1]; a.q2 += xb[2]; a.q3 += xb[3];
    a.qp0 += xb[4]; a.qp1 += xb[5]; a.qp2 += xb[6]; a.qp3 += xb[7];
  }
}

// I1 = 4 / (inert s_m^2), s_m = (sp + sp_right) / 2: adjoint to inert, sp, sp_right.
template <class T>
__device__ __forceinline__ T inertia_vjp(const Slot<T>& L, T sp_right, SAdj<T>& a) {
  if (!(L.f & F_EDGE)) return T(0);
  const T sm = T(0.5) * (L.sp + sp_right);
  a.inert += a.I1 * (-L.I1 / L.inert);
  const T t = a.I1 * (-L.I1 / sm);        // d I1 / d sp = (-2 I1 / sm) * 1/2 for either end
  a.sp += t;
  return t;
}

// ---------------------------------------------------------------- kernels

// checkpoint fields (kCkptFields): x0 x1 x2 v0 v1 v2 s sd q0 q1 q2 q3 o0 o1 o2

template <class T>
__device__ __forceinline__ void ckpt_io(T* base, size_t P, int p, Slot<T>& L, bool store) {
  T* v[kCkptFields] = {&L.x0, &L.x1, &L.x2, &L.v0, &L.v1, &L.v2, &L.s, &L.sd, &L.q0, &L.q1, &L.q2, &L.q3,
                     &L.o0, &L.o1, &L.o2};
#pragma unroll
  for (int f = 0; f < kCkptFields; ++f) {
    if (store) base[(size_t)f * P + p] = *v[f];
    else *v[f] = base[(size_t)f * P + p];
  }
}

// The frame kernel with the state at the start of every substep written to ckpt
// ([substep][field][pill]).  EVEN as in the frame kernel (the same instantiation of the
// passes, so that both give the same bits).
template <class T, bool EVEN>
__global__ void __launch_bounds__(256) rod_frame_ckpt_kernel(const Dev<T>* __restrict__ D, const Blk* __restrict__ tab,
                                                             int nsub, T h, int iters, T* __restrict__ ckpt) {
  Lane2<T> P;
  int pA, pB;
  const Dev<T>* dp = lane_setup(D, tab, P, pA, pB);
  if (!dp) return;
  const Dev<T>& d = *dp;
  load_state(d, P.A, pA);
  load_state(d, P.B, pB);
  load_lane_consts(d, P, pA, pB, rcp(h * h));
  const T ih = T(1) / h;
  for (int sub = 0; sub < nsub; ++sub) {
    T* base = ckpt + (size_t)sub * kCkptFields * d.P;
    if (P.A.f & F_VALID) ckpt_io(base, d.P, pA, P.A, true);
    if (P.B.f & F_VALID) ckpt_io(base, d.P, pB, P.B, true);
    predict_slot(P.A, h, d.gx, d.gy, d.gz);
    predict_slot(P.B, h, d.gx, d.gy, d.gz);
    inertia_lane(P);
    for (int it = 0; it < iters; ++it) iteration_lane<T, false, EVEN>(P);
    velocity_slot(P.A, ih);
    velocity_slot(P.B, ih);
  }
  store_state(d, P.A, pA);
  store_state(d, P.B, pB);
  check_finite(d, P.A);
  check_finite(d, P.B);
}

// Backward of the substeps, software-pipelined: launch k reverses substep s = n - k while
// other blocks of the same launch replay substep s - 1 (its recompute and snapshots do not
// depend on the reverse sweep), so the replay of one substep hides under the reverse of the
// next.  A substep's snapshots (kSnapPerIter per iteration and lane, then the substep-end
// quaternions of both slots, kSnapEnd) go to one of two buffers by the substep's parity.

// Replay of one substep from its checkpoint, storing the pre-pass snapshots and the
// substep-end quaternions into sb (this lane's column of one snapshot buffer).
template <class T, bool EVEN>
__device__ __forceinline__ void backward_replay(Lane2<T>& P, const Dev<T>& d, int pA, int pB, T h, int iters,
                                                const T* __restrict__ ckpt, T* __restrict__ sb, size_t NL) {
  T* cbase = const_cast<T*>(ckpt);
  ckpt_io(cbase, d.P, pA, P.A, false);
  ckpt_io(cbase, d.P, pB, P.B, false);
  load_lane_consts(d, P, pA, pB, rcp(h * h));
  predict_slot(P.A, h, d.gx, d.gy, d.gz);
  predict_slot(P.B, h, d.gx, d.gy, d.gz);
  inertia_lane(P);
  for (int it = 0; it < iters; ++it) {
    T* const si = sb + (size_t)it * kSnapPerIter * NL;
    snap_edge_store(si + snap_offset(0) * NL, NL, P.A, P.B);
    pass_edges<T, false, EVEN>(P, 0);
    snap_edge_store(si + snap_offset(1) * NL, NL, P.A, P.B);
    pass_edges<T, false, EVEN>(P, 1);
    snap_bt_store(si + snap_offset(2) * NL, NL, P.A, P.B);
    pass_bt<T, EVEN>(P, 0);
    snap_bt_store(si + snap_offset(3) * NL, NL, P.A, P.B);
    pass_bt<T, EVEN>(P, 1);
  }
  T* const se = sb + (size_t)iters * kSnapPerIter * NL;   // the velocity update leaves q as it is
  const T q[kSnapEnd] = {P.A.q0, P.A.q1, P.A.q2, P.A.q3, P.B.q0, P.B.q1, P.B.q2, P.B.q3};
#pragma unroll
  for (int i = 0; i < kSnapEnd; ++i) se[(size_t)i * NL] = q[i];
}

// Reverse of one substep.  adj ([field][pill], kCkptFields) holds the adjoint of the state
// at the end of the substep on entry and at its start on exit; padj ([8][pill]) accumulates
// the parameter adjoints: 1/M, 1/M_s, 1/lbar, rho pi r^4 l0, and the four compliance
// scalings; sb is this lane's column of the substep's snapshot buffer (written by its replay).
template <class T, bool EVEN>
__device__ __forceinline__ void backward_reverse(Lane2<T>& P, const Dev<T>& d, int pA, int pB, T h, int iters,
                                                 const T* __restrict__ ckpt, const T* __restrict__ sb, size_t NL,
                                                 T* __restrict__ adj, T* __restrict__ padj) {
  T* cbase = const_cast<T*>(ckpt);
  ckpt_io(cbase, d.P, pA, P.A, false);
  ckpt_io(cbase, d.P, pB, P.B, false);
  const T ih2 = rcp(h * h);
  load_lane_consts(d, P, pA, pB, ih2);
  const T ih = T(1) / h;
  // the substep-start copies and inertias the reverse sweep needs (the prediction itself is
  // replaced by the snapshots), and the substep-end quaternions from the replay
  predict_slot(P.A, h, d.gx, d.gy, d.gz);
  predict_slot(P.B, h, d.gx, d.gy, d.gz);
  inertia_lane(P);
  {
    T q[kSnapEnd];
    snap_load(sb + (size_t)iters * kSnapPerIter * NL, NL, q);
    P.A.q0 = q[0]; P.A.q1 = q[1]; P.A.q2 = q[2]; P.A.q3 = q[3];
    P.B.q0 = q[4]; P.B.q1 = q[5]; P.B.q2 = q[6]; P.B.q3 = q[7];
  }
  // adjoint of the substep-end state
  SAdj<T> aA, aB;
  zero_adj(aA);
  zero_adj(aB);
  {
    Slot<T> t;   // scratch holder for the adjoint fields in checkpoint order
    ckpt_io(adj, d.P, pA, t, false);
    aA.x0 = t.x0; aA.x1 = t.x1; aA.x2 = t.x2; aA.v0 = t.v0; aA.v1 = t.v1; aA.v2 = t.v2; aA.s = t.s; aA.sd = t.sd;
    aA.q0 = t.q0; aA.q1 = t.q1; aA.q2 = t.q2; aA.q3 = t.q3; aA.o0 = t.o0; aA.o1 = t.o1; aA.o2 = t.o2;
    ckpt_io(adj, d.P, pB, t, false);
    aB.x0 = t.x0; aB.x1 = t.x1; aB.x2 = t.x2; aB.v0 = t.v0; aB.v1 = t.v1; aB.v2 = t.v2; aB.s = t.s; aB.sd = t.sd;
    aB.q0 = t.q0; aB.q1 = t.q1; aB.q2 = t.q2; aB.q3 = t.q3; aB.o0 = t.o0; aB.o1 = t.o1; aB.o2 = t.o2;
    if (!(P.A.f & F_VALID)) zero_adj(aA);
    if (!(P.B.f & F_VALID)) zero_adj(aB);
  }
  velocity_vjp(P.A, aA, ih);
  velocity_vjp(P.B, aB, ih);
  // the passes in reverse order, each from its pre-pass snapshot.  FP32: the loads of the
  // next snapshot are issued before the current pass's VJP (FP64 has no registers to spare
  // for that and loads it after).
  constexpr bool kPre = sizeof(T) == 4;
  if (iters > 0) {
    T v[kSnapBt];
    snap_load(sb + ((size_t)(iters - 1) * kSnapPerIter + snap_offset(3)) * NL, NL, v);
    snap_bt_apply(v, P.A, P.B);
  }
  for (int it = iters - 1; it >= 0; --it) {
    const T* const si = sb + (size_t)it * kSnapPerIter * NL;
    {
      T v[kSnapBt];
      if (kPre) snap_load(si + snap_offset(2) * NL, NL, v);
      pass_bt_vjp<T, EVEN>(P, aA, aB, 1);
      if (!kPre) __builtin_amdgcn_sched_barrier(0);
      if (!kPre) snap_load(si + snap_offset(2) * NL, NL, v);
      snap_bt_apply(v, P.A, P.B);
    }
    {
      T v[kSnapEdge];
      if (kPre) snap_load(si + snap_offset(1) * NL, NL, v);
      pass_bt_vjp<T, EVEN>(P, aA, aB, 0);
      if (!kPre) __builtin_amdgcn_sched_barrier(0);
      if (!kPre) snap_load(si + snap_offset(1) * NL, NL, v);
      snap_edge_apply(v, P.A, P.B);
    }
    {
      T v[kSnapEdge];
      if (kPre) snap_load(si + snap_offset(0) * NL, NL, v);
      pass_edges_vjp<T, EVEN>(P, aA, aB, 1);
      if (!kPre) __builtin_amdgcn_sched_barrier(0);
      if (!kPre) snap_load(si + snap_offset(0) * NL, NL, v);
      snap_edge_apply(v, P.A, P.B);
    }
    if (it > 0) {
      T v[kSnapBt];
      if (kPre) snap_load(si - (size_t)kSnapPerIter * NL + snap_offset(3) * NL, NL, v);
      pass_edges_vjp<T, EVEN>(P, aA, aB, 0);
      if (!kPre) __builtin_amdgcn_sched_barrier(0);
      if (!kPre) snap_load(si - (size_t)kSnapPerIter * NL + snap_offset(3) * NL, NL, v);
      snap_bt_apply(v, P.A, P.B);
    } else {
      pass_edges_vjp<T, EVEN>(P, aA, aB, 0);
    }
  }
  // substep-start inertia of both edges (the B edge's right end is the next lane's A)
  const T spN = dn(P.A.sp);
  aB.sp += inertia_vjp(P.A, P.B.sp, aA);
  T rsp = inertia_vjp(P.B, spN, aB);
  rsp = up(rsp);
  if ((P.A.f & F_VALID) && !(P.A.f & F_FIRST)) aA.sp += rsp;
  // prediction, from the substep-start state
  Slot<T>* S[2] = {&P.A, &P.B};
  SAdj<T>* Aj[2] = {&aA, &aB};
  const int ps[2] = {pA, pB};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    Slot<T>& L = *S[j];
    SAdj<T>& a = *Aj[j];
    if (!(L.f & F_VALID)) continue;
    Slot<T> st;
    ckpt_io(cbase, d.P, ps[j], st, false);
    Slot<T> out;
    out.x0 = a.x0 + a.xp0; out.x1 = a.x1 + a.xp1; out.x2 = a.x2 + a.xp2;
    if (L.w > T(0)) { out.v0 = h * a.x0; out.v1 = h * a.x1; out.v2 = h * a.x2; }
    else { out.v0 = T(0); out.v1 = T(0); out.v2 = T(0); }
    out.s = a.s + a.sp;
    out.sd = h * a.s;
    if (L.f & F_EDGE) {
      const T yb[4] = {a.q0, a.q1, a.q2, a.q3};
      T xb[7];
      qpredict_vjp(st.q0, st.q1, st.q2, st.q3, st.o0, st.o1, st.o2, h, yb, xb);
      out.q0 = xb[0] + a.qp0; out.q1 = xb[1] + a.qp1; out.q2 = xb[2] + a.qp2; out.q3 = xb[3] + a.qp3;
      out.o0 = xb[4]; out.o1 = xb[5]; out.o2 = xb[6];
    } else {
      out.q0 = T(0); out.q1 = T(0); out.q2 = T(0); out.q3 = T(0);
      out.o0 = T(0); out.o1 = T(0); out.o2 = T(0);
    }
    ckpt_io(adj, d.P, ps[j], out, true);
    const int p = ps[j];
    padj[0 * (size_t)d.P + p] += a.w;
    padj[1 * (size_t)d.P + p] += a.ws;
    padj[2 * (size_t)d.P + p] += a.ilb;
    padj[3 * (size_t)d.P + p] += a.inert;
    padj[4 * (size_t)d.P + p] += a.ass * ih2;
    padj[5 * (size_t)d.P + p] += a.avol * ih2;
    padj[6 * (size_t)d.P + p] += a.asg * ih2;
    padj[7 * (size_t)d.P + p] += a.abt * ih2;
  }
}

// Block roles: blocks [0, nb) reverse the substep whose checkpoint is rev_ckpt (none when it
// is null), blocks [nb, 2 nb) replay the substep whose checkpoint is rep_ckpt (none when null);
// within a role the forward's lane layout, one wavefront per block (block b runs wavefront
// tab[b / 4].base + b % 4), so that a small scene's wavefronts spread over every compute unit.
template <class T, bool EVEN>
__global__ void __launch_bounds__(64) rod_backward_kernel(const Dev<T>* __restrict__ D, const Blk* __restrict__ tab,
                                                           T h, int iters, int nb, const T* __restrict__ rev_ckpt,
                                                           int rev_buf, const T* __restrict__ rep_ckpt, int rep_buf,
                                                           T* __restrict__ snap, T* __restrict__ adj,
                                                           T* __restrict__ padj) {
  const bool replay = (int)blockIdx.x >= nb;
  if (replay ? rep_ckpt == nullptr : rev_ckpt == nullptr) return;
  const int bi = replay ? (int)blockIdx.x - nb : (int)blockIdx.x;
  Lane2<T> P;
  int pA, pB;
  const Blk blk = tab[bi >> 2];
  const int wave = blk.base + (bi & 3);
  const Dev<T> d = D[blk.scene];
  asm volatile("" ::"s"(d.gx), "s"(d.gy), "s"(d.gz), "s"(h));
  stage_setup(d, wave, P, pA, pB);
  if (wave >= d.W) return;             // wave-uniform: a block past the scene's last wavefront
  const size_t NL = (size_t)d.W * 64;
  const size_t region = ((size_t)iters * kSnapPerIter + kSnapEnd) * NL;
  const size_t lg = (size_t)wave * 64 + (threadIdx.x & 63);
  if (replay) backward_replay<T, EVEN>(P, d, pA, pB, h, iters, rep_ckpt, snap + (size_t)rep_buf * region + lg, NL);
  else backward_reverse<T, EVEN>(P, d, pA, pB, h, iters, rev_ckpt, snap + (size_t)rev_buf * region + lg, NL, adj, padj);
}

// Seed: adjoint of the end-of-frame state from dL/dx (pill-major [P*3]); other fields 0.
template <class T>
__global__ void adjoint_seed_kernel(int P, const T* __restrict__ dldx, T* __restrict__ adj, T* __restrict__ padj) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= P) return;
#pragma unroll
  for (int f = 0; f < kCkptFields; ++f) adj[(size_t)f * P + p] = (f < 3 && dldx) ? dldx[3 * (size_t)p + f] : T(0);
#pragma unroll
  for (int f = 0; f < 8; ++f) padj[(size_t)f * P + p] = T(0);
}


// Parameter adjoints to rest radii and activations, in FP64 (one thread per pill).
// Lumped masses (App. B): M_p, M_s,p gather half of  rho pi rm^2 l0  and  rho pi rm^4 l0 / 2
// from each adjacent edge, rm the mean of the edge's end radii; inertia base rho pi rm^4 l0;
// compliance scalings  alpha / (pi rm^2 l0)  (stretch-shear, volume),  alpha / (pi rm^4 l0 / 2)
// (scale gradient),  alpha / (pi r^4 lv / 4)  (bend-twist, r the vertex radius);
// inverse stretch rest length  1 / (a l0).
template <class T>
__device__ __forceinline__ double edge_radius_adj(const Dev<T>& d, const T* __restrict__ padj, int e, double rho) {
  const size_t P = (size_t)d.P;
  const double pi = 3.14159265358979323846;
  const double rm = 0.5 * ((double)d.rbar[e] + (double)d.rbar[e + 1]);
  const double len = 1.0 / (double)d.il0[e];
  const double w0 = d.winv[e], w1 = d.winv[e + 1], s0 = d.wsinv[e], s1 = d.wsinv[e + 1];
  const double Mb = 0.5 * (-(double)padj[e] * w0 * w0 - (double)padj[e + 1] * w1 * w1);
  const double Msb = 0.5 * (-(double)padj[P + e] * s0 * s0 - (double)padj[P + e + 1] * s1 * s1);
  double g = Mb * 2.0 * rho * pi * rm * len + Msb * 2.0 * rho * pi * rm * rm * rm * len;
  g += (double)padj[3 * P + e] * 4.0 * (double)d.inert[e] / rm;
  g -= 2.0 * ((double)padj[4 * P + e] * (double)d.css[e] + (double)padj[5 * P + e] * (double)d.cvol[e]) / rm;
  g -= 4.0 * (double)padj[6 * P + e] * (double)d.csg[e] / rm;
  return g;
}

template <class T>
__global__ void adjoint_chain_kernel(const Dev<T>* __restrict__ D, const T* __restrict__ padj, double rho,
                                     double* __restrict__ drbar, double* __restrict__ dact) {
  const Dev<T>& d = *D;
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= d.P) return;
  const size_t P = (size_t)d.P;
  const uint32_t f = d.flags[p];
  double g = 0.0;
  if (f & F_EDGE) g += 0.5 * edge_radius_adj(d, padj, p, rho);
  if (!(f & F_FIRST)) {
    g += 0.5 * edge_radius_adj(d, padj, p - 1, rho);
    if (d.flags[p - 1] & F_BT) g -= 4.0 * (double)padj[7 * P + p - 1] * (double)d.cbtc[p - 1] / (double)d.rbar[p];
  }
  drbar[p] = g;
  if (f & F_FIRST) {
    double a = 0.0;
    for (int q = p; q < d.P && (q == p || !(d.flags[q] & F_FIRST)); ++q) {
      if (!(d.flags[q] & F_EDGE)) continue;
      const double ilb = d.ilb[q];
      a -= (double)padj[2 * P + q] * ilb * ilb / (double)d.il0[q];
    }
    dact[d.rod_of[p]] = a;
  }
}

// ---------------------------------------------------------------- launchers

template <class T>
hipError_t launch_frame_ckpt(const BatchDev& b, int nsub, double h, int iters, T* ckpt, hipStream_t st) {
  if (b.nblk[TB_WAVES] == 0) return hipSuccess;
  if (b.even)
    hipLaunchKernelGGL((rod_frame_ckpt_kernel<T, true>), dim3(b.nblk[TB_WAVES]), dim3(256), 0, st, (const Dev<T>*)b.dev,
                       b.tab[TB_WAVES], nsub, (T)h, iters, ckpt);
  else
    hipLaunchKernelGGL((rod_frame_ckpt_kernel<T, false>), dim3(b.nblk[TB_WAVES]), dim3(256), 0, st, (const Dev<T>*)b.dev,
                       b.tab[TB_WAVES], nsub, (T)h, iters, ckpt);
  return hipGetLastError();
}

template <class T>
hipError_t launch_backward(const BatchDev& b, int P, int nsub, double h, int iters, const T* ckpt, const T* dldx,
                           T* snap, T* adj, T* padj, double rho, double* drbar, double* dact, hipStream_t st) {
  if (P == 0) return hipSuccess;
  hipLaunchKernelGGL(adjoint_seed_kernel<T>, dim3((P + 255) / 256), dim3(256), 0, st, P, dldx, adj, padj);
  const int nb = 4 * b.nblk[TB_WAVES];
  const size_t per = (size_t)kCkptFields * P;
  // launch k reverses substep nsub - k (k >= 1) and replays substep nsub - 1 - k (if any)
  for (int k = 0; k <= nsub; ++k) {
    const int rs = nsub - k, ps = nsub - 1 - k;
    const T* rc = k >= 1 ? ckpt + (size_t)rs * per : nullptr;
    const T* pc = ps >= 0 ? ckpt + (size_t)ps * per : nullptr;
    if (b.even)
      hipLaunchKernelGGL((rod_backward_kernel<T, true>), dim3(2 * nb), dim3(64), 0, st, (const Dev<T>*)b.dev,
                         b.tab[TB_WAVES], (T)h, iters, nb, rc, rs & 1, pc, ps & 1, snap, adj, padj);
    else
      hipLaunchKernelGGL((rod_backward_kernel<T, false>), dim3(2 * nb), dim3(64), 0, st, (const Dev<T>*)b.dev,
                         b.tab[TB_WAVES], (T)h, iters, nb, rc, rs & 1, pc, ps & 1, snap, adj, padj);
  }
  hipLaunchKernelGGL(adjoint_chain_kernel<T>, dim3((P + 255) / 256), dim3(256), 0, st, (const Dev<T>*)b.dev,
                     (const T*)padj, rho, drbar, dact);
  return hipGetLastError();
}

template hipError_t launch_frame_ckpt<float>(const BatchDev&, int, double, int, float*, hipStream_t);
template hipError_t launch_frame_ckpt<double>(const BatchDev&, int, double, int, double*, hipStream_t);
template hipError_t launch_backward<float>(const BatchDev&, int, int, double, int, const float*, const float*, float*,
                                           float*, float*, double, double*, double*, hipStream_t);
template hipError_t launch_backward<double>(const BatchDev&, int, int, double, int, const double*, const double*,
                                            double*, double*, double*, double, double*, double*, hipStream_t);

}  // namespace viper
