// VIPER rod substep kernels for gfx950 (CDNA4, wave64).
//
// One wavefront owns a contiguous run of whole rods of up to 128 pills; lane l
// holds two consecutive pill slots, A = 2l and B = 2l+1 of that run.  A slot
// carries its vertex state (position, velocity, scale and rate) and the edge
// that starts at it (quaternion, angular velocity).  Constraints are projected
// in four colour passes per iteration (even/odd edges for stretch-shear, volume
// and scale gradient; even/odd vertices for bend-twist), so inside a pass every
// constraint touches disjoint state.  For rods that start on an even slot the
// even-colour constraints live entirely inside one lane (edge A-B) and the
// odd-colour ones join slot B to the next lane's slot A, whose values arrive by
// a cross-lane shift and go back the same way: every lane works in every pass.
//
// The closed forms used here (derived from the generic per-constraint update of
// Sec. 6,  S = sum_b J_b W_b J_b^T + alpha~,  dl = S^-1(-C - alpha~ lambda),
// dX_b = W_b J_b^T dl,  relaxation 1) are:
//  stretch-shear (eq. stretch_z):  C = (x1-x0)/lbar - d3(q),
//      S = k1 d3 d3^T + k2 (I - d3 d3^T),  k1 = (w0+w1)/lbar^2 + a~,  k2 = k1 + 1/I_bend
//  volume (eq. vol, tangential):   C = s_m^2 |x1-x0| / l0 - 1   (scalar)
//  scale gradient (eq. surface_stretch): C = (s1-s0)/l0         (scalar)
//  bend-twist (eq. bending_twist, Darboux vector of Sec. 7.5):
//      C = s1 c Im(r) - Omega_rest,  r = conj(q0) q1 (shortest arc), c = 4/(l0_0+l0_1),
//      J_q1 = -J_q0 = (s1 c / 2)(r_w I - [r_v]x) R0^T, solved as a symmetric 3x3 in frame 0.

#include "rod_device.h"
#include "stage_setup.h"
#include "detect_device.h"

namespace viper {

// ---------------------------------------------------------------- kernels

// FRAME / SUBSTEP mode: nsub substeps with the rod state in registers.  X: the optional
// constraint terms are compiled in; EVEN: every rod starts on an even slot of its wavefront
// (both chosen per batch on the host).
template <class T, bool X, bool EVEN>
__global__ void __launch_bounds__(256) rod_frame_kernel(const Dev<T>* __restrict__ D, const Blk* __restrict__ tab,
                                                        int nsub, T h, int iters) {
  Lane2<T> P;
  int pA, pB;
  const Dev<T>* dp = lane_setup(D, tab, P, pA, pB);
  if (!dp) return;
  const Dev<T>& d = *dp;
  load_state(d, P.A, pA);
  load_state(d, P.B, pB);
  load_lane_consts<T, X>(d, P, pA, pB, rcp(h * h));
  const T ih = T(1) / h;
  for (int sub = 0; sub < nsub; ++sub) {
    predict_slot(P.A, h, d.gx, d.gy, d.gz);
    predict_slot(P.B, h, d.gx, d.gy, d.gz);
    inertia_lane(P);
    for (int it = 0; it < iters; ++it) iteration_lane<T, X, EVEN>(P);
    velocity_slot(P.A, ih);
    velocity_slot(P.B, ih);
  }
  store_state(d, P.A, pA);
  store_state(d, P.B, pB);
  check_finite(d, P.A);
  check_finite(d, P.B);
}

// The previous contact pass's averaged corrections for both slots of a lane (the
// single-slot contact_apply, with the reads of both slots issued together and used
// unconditionally: counts and fixed-point sums are read whether or not a slot has contacts).
template <class T>
__device__ __forceinline__ int contact_apply_lane(int32_t* acnt, unsigned long long* acc, Lane2<T>& P, int pA, int pB) {
  const int n[2] = {acnt[pA], acnt[pB]};
  const int p[2] = {pA, pB};
  int moved = 0;
  longlong2 a01[2], a23[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const longlong2* q = (const longlong2*)(acc + 4 * (size_t)p[k]);
    a01[k] = q[0];
    a23[k] = q[1];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    // without contacts the factor is 0 and the slot keeps its values exactly (a finite
    // fixed-point sum times 0 adds a zero)
    Slot<T>& L = k ? P.B : P.A;
    const bool on = (L.f & F_VALID) && n[k] != 0;
    const double inv = on ? 1.0 / (double)n[k] : 0.0;
    L.x0 = (T)((double)L.x0 + inv * ((double)a01[k].x * 0x1p-44));
    L.x1 = (T)((double)L.x1 + inv * ((double)a01[k].y * 0x1p-44));
    L.x2 = (T)((double)L.x2 + inv * ((double)a23[k].x * 0x1p-44));
    L.s = (T)((double)L.s + inv * ((double)a23[k].y * 0x1p-44));
    if (on) {
      longlong2* q = (longlong2*)(acc + 4 * (size_t)p[k]);
      q[0] = make_longlong2(0, 0);
      q[1] = make_longlong2(0, 0);
      acnt[p[k]] = 0;
      moved |= 1 << k;
    }
  }
  return moved;
}

// ITERATION mode, stage 1: prediction of every pill and edge, saving the substep-start
// state and resetting the multipliers.
template <class T>
__device__ __forceinline__ void store_predicted(const Dev<T>& d, const Slot<T>& L, int p) {
  if (!(L.f & F_VALID)) return;
  d.px[p] = L.x0; d.py[p] = L.x1; d.pz[p] = L.x2; d.s[p] = L.s;
  d.qx[p] = L.q0; d.qy[p] = L.q1; d.qz[p] = L.q2; d.qw[p] = L.q3;
  d.xpx[p] = L.xp0; d.xpy[p] = L.xp1; d.xpz[p] = L.xp2; d.spv[p] = L.sp;
  d.qpx[p] = L.qp0; d.qpy[p] = L.qp1; d.qpz[p] = L.qp2; d.qpw[p] = L.qp3;
  d.i1[p] = L.I1;
#pragma unroll
  for (int i = 0; i < 12; ++i) d.lam[(size_t)i * d.P + p] = T(0);
}

// Start of a contact detection, by the wavefront that has just predicted its pills (the
// prediction launch of a contact scene): the detection copy of its state (FP64 world positions
// -- rod anchor + stored position, as the contact pass forms them -- and scales), which the
// detection reads instead of the state (the substep's first constraint iteration may already
// have moved it); the bounding sphere and radius bin of every capsule that starts on one of
// its pills (a capsule's pills lie in one wavefront: slot A's capsule ends on slot B, slot
// B's on the next lane's slot A); the wavefront's radius histogram, added into one of
// kHistCopies copies; and the scene's per-detection resets, shared over its threads.
// s_hist [kRadBins + 1] and s_hmax [kRadBins] are the block's LDS (one wavefront per block).
template <class T>
__device__ __forceinline__ void detect_start_wave(const Dev<T>& d, const ContactDev& c, const Lane2<T>& P, int pA, int pB,
                                                  int rA, int rB, T rbA, T rbB, int wave, int* s_hist,
                                                  unsigned long long* s_hmax) {
  const int lane = (int)(threadIdx.x & 63);
  for (int k = lane; k <= kRadBins; k += 64) {
    s_hist[k] = 0;
    if (k < kRadBins) s_hmax[k] = 0ull;
  }
  detect_reset(c, wave * 64 + lane, d.W * 64);
  double wA[3], wB[3];
  {
    const double* an = d.anchor + 3 * (size_t)rA;
    wA[0] = an[0] + (double)P.A.x0; wA[1] = an[1] + (double)P.A.x1; wA[2] = an[2] + (double)P.A.x2;
    const double* bn = d.anchor + 3 * (size_t)rB;
    wB[0] = bn[0] + (double)P.B.x0; wB[1] = bn[1] + (double)P.B.x1; wB[2] = bn[2] + (double)P.B.x2;
  }
  T* sdet = (T*)c.sdet;
  if (P.A.f & F_VALID) {
    c.xdet[3 * (size_t)pA] = wA[0]; c.xdet[3 * (size_t)pA + 1] = wA[1]; c.xdet[3 * (size_t)pA + 2] = wA[2];
    sdet[pA] = P.A.s;
  }
  if (P.B.f & F_VALID) {
    c.xdet[3 * (size_t)pB] = wB[0]; c.xdet[3 * (size_t)pB + 1] = wB[1]; c.xdet[3 * (size_t)pB + 2] = wB[2];
    sdet[pB] = P.B.s;
  }
  // the next lane's slot A: the far end of slot B's capsule
  const double wN[3] = {dn(wA[0]), dn(wA[1]), dn(wA[2])};
  const T sN = dn(P.A.s), rbN = dn(rbA);
  __syncthreads();   // the block is this wavefront: its histogram is cleared
  double sp[4];
  if (P.A.f & F_EDGE) {
    const int bin = capsule_record(c, pA - rA, wA, wB, P.A.s, P.B.s, rbA, rbB, sp);
    atomicAdd(&s_hist[bin], 1);
    if (bin < kRadBins) atomicMax(&s_hmax[bin], (unsigned long long)__double_as_longlong(fmax(sp[3], 0.0)));
  }
  if (P.B.f & F_EDGE) {
    const int bin = capsule_record(c, pB - rB, wB, wN, P.B.s, sN, rbB, rbN, sp);
    atomicAdd(&s_hist[bin], 1);
    if (bin < kRadBins) atomicMax(&s_hmax[bin], (unsigned long long)__double_as_longlong(fmax(sp[3], 0.0)));
  }
  __syncthreads();
  int32_t* hist = c.hist + (size_t)(wave & (kHistCopies - 1)) * (kRadBins + 1);
  unsigned long long* hmax = c.binmax + (size_t)(wave & (kHistCopies - 1)) * kRadBins;
  for (int k = lane; k <= kRadBins; k += 64)
    if (s_hist[k]) {
      atomicAdd(&hist[k], s_hist[k]);
      if (k < kRadBins) atomicMax(&hmax[k], s_hmax[k]);
    }
}

// C: the scenes have contacts (the prediction starts their detection).
template <class T, bool C>
__global__ void __launch_bounds__(256) predict_kernel(const char* __restrict__ wrec, int stride, T h,
                                                      const ContactDev* __restrict__ CD) {
  Lane2<T> P;
  int pA, pB;
  const char* rec = wrec + (size_t)blockIdx.x * stride;
  const WaveBlk b = ((const WaveRec*)rec)->b;
  const Dev<T> d = *(const Dev<T>*)(rec + sizeof(WaveRec));
  __shared__ int s_hist[kRadBins + 1];
  __shared__ unsigned long long s_hmax[kRadBins];
  asm volatile("" ::"s"(d.gx), "s"(d.gy), "s"(d.gz), "s"(h));
  const int wave = b.wave;
  stage_setup(d, b, P, pA, pB);
  load_state(d, P.A, pA);
  load_state(d, P.B, pB);
  P.A.w = d.winv[pA]; P.A.inert = d.inert[pA];
  P.B.w = d.winv[pB]; P.B.inert = d.inert[pB];
  int rA = 0, rB = 0;
  T rbA = T(0), rbB = T(0);
  if constexpr (C) {
    rA = d.rod_of[pA];
    rB = d.rod_of[pB];
    rbA = d.rbar[pA];
    rbB = d.rbar[pB];
  }
  predict_slot(P.A, h, d.gx, d.gy, d.gz);
  predict_slot(P.B, h, d.gx, d.gy, d.gz);
  inertia_lane(P);
  store_predicted(d, P.A, pA);
  store_predicted(d, P.B, pB);
  if constexpr (C) detect_start_wave(d, CD[b.scene], P, pA, pB, rA, rB, rbA, rbB, wave, s_hist, s_hmax);
}

// Substep start without the multipliers' reset (the first iteration that follows in the same
// launch writes them).
template <class T>
__device__ __forceinline__ void store_substep_start(const Dev<T>& d, const Slot<T>& L, int p) {
  if (!(L.f & F_VALID)) return;
  d.xpx[p] = L.xp0; d.xpy[p] = L.xp1; d.xpz[p] = L.xp2; d.spv[p] = L.sp;
  d.qpx[p] = L.qp0; d.qpy[p] = L.qp1; d.qpz[p] = L.qp2; d.qpw[p] = L.qp3;
  d.i1[p] = L.I1;
}

// ITERATION mode, stage 2: one constraint iteration (four colour passes) with the
// state and multipliers streamed from and back to memory.
// Multipliers streamed per iteration: the plain constraint set's 8, or all 12 with the
// optional terms (cross-section stretch, surface bending, volume-bending coupling).
template <bool X> constexpr int kLam = X ? 12 : 8;

template <class T, bool X>
__device__ __forceinline__ void load_iter(const Dev<T>& d, Slot<T>& L, int p) {
  L.x0 = d.px[p]; L.x1 = d.py[p]; L.x2 = d.pz[p]; L.s = d.s[p];
  L.q0 = d.qx[p]; L.q1 = d.qy[p]; L.q2 = d.qz[p]; L.q3 = d.qw[p];
#pragma unroll
  for (int i = 0; i < kLam<X>; ++i) L.l[i] = d.lam[(size_t)i * d.P + p];
  L.I1 = d.i1[p];
}

template <class T, bool X>
__device__ __forceinline__ void store_iter(const Dev<T>& d, const Slot<T>& L, int p) {
  if (!(L.f & F_VALID)) return;
  d.px[p] = L.x0; d.py[p] = L.x1; d.pz[p] = L.x2; d.s[p] = L.s;
  d.qx[p] = L.q0; d.qy[p] = L.q1; d.qz[p] = L.q2; d.qw[p] = L.q3;
#pragma unroll
  for (int i = 0; i < kLam<X>; ++i) d.lam[(size_t)i * d.P + p] = L.l[i];
}

// ITERATION mode, Jacobi variant of stage 2 (Sec. 7: constraints computed in parallel, their
// displacements averaged by a reduction).  Every rod constraint of the lane's slots is
// projected on register copies of the state at the start of the iteration (one constraint
// type at a time, through the same closed forms as the Gauss-Seidel passes); each slot then
// moves by the mean of the corrections of the active constraints acting on it (positions and
// scales; rotations by the mean quaternion increment, renormalised).  Each constraint keeps
// its own multiplier update.  Corrections of the next lane's slot A (from this lane's B-edge
// and B-vertex bend-twist) travel back by one lane shift.
template <class T>
struct JacobiAcc {
  T dx0 = T(0), dx1 = T(0), dx2 = T(0), ds = T(0), dq0 = T(0), dq1 = T(0), dq2 = T(0), dq3 = T(0);
  T nx = T(0), ns = T(0), nq = T(0);
};

template <class T, bool X>
__device__ __forceinline__ void jacobi_edge(Slot<T>& L, const Slot<T>& L0, T b0, T b1, T b2, T sb, T wb, T wsb,
                                            JacobiAcc<T>& aL, JacobiAcc<T>& aR) {
  const uint32_t types[4] = {F_SS, F_VOL, F_SG, F_SR};
#pragma unroll
  for (int t = 0; t < (X ? 4 : 3); ++t) {
    if (!(L0.f & types[t])) continue;
    Slot<T> a = L0;
    a.f = (L0.f & ~(F_SS | F_VOL | F_SG | F_SR)) | types[t];
    T c0 = b0, c1 = b1, c2 = b2, cs = sb;
    edge_update<T, X>(a, c0, c1, c2, cs, wb, wsb);
    if (t == 0) {
      L.l[0] = a.l[0]; L.l[1] = a.l[1]; L.l[2] = a.l[2];
      aL.dq0 += a.q0 - L0.q0; aL.dq1 += a.q1 - L0.q1; aL.dq2 += a.q2 - L0.q2; aL.dq3 += a.q3 - L0.q3; aL.nq += T(1);
    } else {
      const int li = (t == 3) ? 8 : 2 + t;
      L.l[li] = a.l[li];
      aL.ds += a.s - L0.s; aR.ds += cs - sb; aL.ns += T(1); aR.ns += T(1);
    }
    if (t < 2) {
      aL.dx0 += a.x0 - L0.x0; aL.dx1 += a.x1 - L0.x1; aL.dx2 += a.x2 - L0.x2; aL.nx += T(1);
      aR.dx0 += c0 - b0; aR.dx1 += c1 - b1; aR.dx2 += c2 - b2; aR.nx += T(1);
    }
  }
}

template <class T>
__device__ __forceinline__ void jacobi_bt(Slot<T>& L, const Slot<T>& L0, T b0, T b1, T b2, T b3, T sb, T Ib, T wsb,
                                          JacobiAcc<T>& aL, JacobiAcc<T>& aR) {
  Slot<T> a = L0;
  T c0 = b0, c1 = b1, c2 = b2, c3 = b3, cs = sb;
  bt_update(a, c0, c1, c2, c3, cs, Ib, wsb);
  L.l[5] = a.l[5]; L.l[6] = a.l[6]; L.l[7] = a.l[7];
  aL.dq0 += a.q0 - L0.q0; aL.dq1 += a.q1 - L0.q1; aL.dq2 += a.q2 - L0.q2; aL.dq3 += a.q3 - L0.q3; aL.nq += T(1);
  aR.dq0 += c0 - b0; aR.dq1 += c1 - b1; aR.dq2 += c2 - b2; aR.dq3 += c3 - b3; aR.nq += T(1);
  aR.ds += cs - sb; aR.ns += T(1);
}

template <class T>
__device__ __forceinline__ void jacobi_apply(Slot<T>& L, const JacobiAcc<T>& a) {
  if (a.nx > T(0)) {
    const T f = T(1) / a.nx;
    L.x0 += f * a.dx0; L.x1 += f * a.dx1; L.x2 += f * a.dx2;
  }
  if (a.ns > T(0)) L.s += a.ds / a.ns;
  if (a.nq > T(0)) {
    const T f = T(1) / a.nq;
    const T q0 = L.q0 + f * a.dq0, q1 = L.q1 + f * a.dq1, q2 = L.q2 + f * a.dq2, q3 = L.q3 + f * a.dq3;
    const T in = T(1) / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    L.q0 = q0 * in; L.q1 = q1 * in; L.q2 = q2 * in; L.q3 = q3 * in;
  }
}

template <class T, bool X>
__device__ __forceinline__ void jacobi_lane(Lane2<T>& P) {
  const Slot<T> A0 = P.A, B0 = P.B;
  // the next lane's slot A as it stands at the start of the iteration
  const T n0 = dn(A0.x0), n1 = dn(A0.x1), n2 = dn(A0.x2), ns = dn(A0.s);
  const T nq0 = dn(A0.q0), nq1 = dn(A0.q1), nq2 = dn(A0.q2), nq3 = dn(A0.q3);
  JacobiAcc<T> aA, aB, aN;
  if (A0.f & F_EDGE) jacobi_edge<T, X>(P.A, A0, B0.x0, B0.x1, B0.x2, B0.s, B0.w, B0.ws, aA, aB);
  if (B0.f & F_EDGE) jacobi_edge<T, X>(P.B, B0, n0, n1, n2, ns, P.wN, P.wsN, aB, aN);
  if ((A0.f & F_BT) && (A0.f & F_BTEN)) jacobi_bt(P.A, A0, B0.q0, B0.q1, B0.q2, B0.q3, B0.s, B0.I1, B0.ws, aA, aB);
  if ((B0.f & F_BT) && (B0.f & F_BTEN)) jacobi_bt(P.B, B0, nq0, nq1, nq2, nq3, ns, P.I1N, P.wsN, aB, aN);
  // this lane's contributions to the next lane's A arrive there; add the previous lane's here
  JacobiAcc<T> r;
  r.dx0 = up(aN.dx0); r.dx1 = up(aN.dx1); r.dx2 = up(aN.dx2); r.ds = up(aN.ds);
  r.dq0 = up(aN.dq0); r.dq1 = up(aN.dq1); r.dq2 = up(aN.dq2); r.dq3 = up(aN.dq3);
  r.nx = up(aN.nx); r.ns = up(aN.ns); r.nq = up(aN.nq);
  if ((A0.f & F_VALID) && !(A0.f & F_FIRST)) {
    aA.dx0 += r.dx0; aA.dx1 += r.dx1; aA.dx2 += r.dx2; aA.ds += r.ds;
    aA.dq0 += r.dq0; aA.dq1 += r.dq1; aA.dq2 += r.dq2; aA.dq3 += r.dq3;
    aA.nx += r.nx; aA.ns += r.ns; aA.nq += r.nq;
  }
  jacobi_apply(P.A, aA);
  jacobi_apply(P.B, aB);
}

// C: the scenes have contacts (CD holds their buffers).
template <class T, bool X, bool EVEN, bool C>
__global__ void __launch_bounds__(256) rod_iteration_kernel(const char* __restrict__ wrec, int stride, T h,
                                                            const ContactDev* __restrict__ CD) {
  Lane2<T> P;
  int pA, pB;
  const char* rec = wrec + (size_t)blockIdx.x * stride;
  const WaveRec wr = *(const WaveRec*)rec;
  const WaveBlk b = wr.b;
  const Dev<T> d = *(const Dev<T>*)(rec + sizeof(WaveRec));
  int32_t* acnt = nullptr;
  unsigned long long* acc = nullptr;
  if constexpr (C) {
    acnt = wr.acnt;
    acc = wr.acc;
  }
  // the scalars read after the state are requested with the pointers (an empty statement
  // that takes them as operands), not in a round trip of their own later
  asm volatile("" ::"s"(d.floor_on), "s"(d.jacobi), "s"(h));
  stage_setup(d, b, P, pA, pB);
  load_iter<T, X>(d, P.A, pA);
  load_iter<T, X>(d, P.B, pB);
  load_lane_consts<T, X>(d, P, pA, pB, rcp(h * h));
  // the previous contact pass's corrections come first
  if constexpr (C) contact_apply_lane(acnt, acc, P, pA, pB);
  if (d.floor_on) {   // then the half-plane floor, at the start of the iteration
    if (P.A.f & F_VALID) floor_apply(d, pA, P.A.x0, P.A.x1, P.A.x2, P.A.s);
    if (P.B.f & F_VALID) floor_apply(d, pB, P.B.x0, P.B.x1, P.B.x2, P.B.s);
  }
  P.I1N = dn(P.A.I1);
  if (d.jacobi) jacobi_lane<T, X>(P);       // wave-uniform: one scene per block
  else iteration_lane<T, X, EVEN>(P);
  store_iter<T, X>(d, P.A, pA);
  store_iter<T, X>(d, P.B, pB);
}

// ITERATION mode, stage 3: velocity update.
template <class T>
__device__ __forceinline__ void velocity_load(const Dev<T>& d, Slot<T>& L, int p) {
  L.x0 = d.px[p]; L.x1 = d.py[p]; L.x2 = d.pz[p]; L.s = d.s[p];
  L.q0 = d.qx[p]; L.q1 = d.qy[p]; L.q2 = d.qz[p]; L.q3 = d.qw[p];
  L.xp0 = d.xpx[p]; L.xp1 = d.xpy[p]; L.xp2 = d.xpz[p]; L.sp = d.spv[p];
  L.qp0 = d.qpx[p]; L.qp1 = d.qpy[p]; L.qp2 = d.qpz[p]; L.qp3 = d.qpw[p];
  L.w = d.winv[p];
}

// moved: the last contact pass's corrections changed the slot's position and scale, which
// are stored back with the velocities
template <class T>
__device__ __forceinline__ void velocity_store(const Dev<T>& d, Slot<T>& L, int p, T ih, bool moved) {
  if (!(L.f & F_VALID)) return;
  if (moved) { d.px[p] = L.x0; d.py[p] = L.x1; d.pz[p] = L.x2; d.s[p] = L.s; }
  velocity_slot(L, ih);
  d.vx[p] = L.v0; d.vy[p] = L.v1; d.vz[p] = L.v2; d.sd[p] = L.sd;
  if (L.f & F_EDGE) { d.ox[p] = L.o0; d.oy[p] = L.o1; d.oz[p] = L.o2; }
  check_finite(d, L);
}

// C: the scenes have contacts, whose last pass's corrections are applied first.  NEXT: what
// follows in the same launch, from the state in registers (the values the next stage would
// read back: positions, scales and rotations as stored, the velocities just formed):
// 0 nothing; 1 the next substep's prediction; 2 the prediction and that substep's first
// constraint iteration (X, EVEN as for rod_iteration_kernel), which needs nothing from other
// wavefronts: a rod lies in one wavefront, and no contact correction is pending before the
// first iteration (this launch has just applied and cleared the last ones).
template <class T, bool C, int NEXT, bool X, bool EVEN>
__global__ void __launch_bounds__(256) velocity_kernel(const char* __restrict__ wrec, int stride, T h,
                                                       const ContactDev* __restrict__ CD) {
  Lane2<T> P;
  int pA, pB;
  const char* rec = wrec + (size_t)blockIdx.x * stride;
  const WaveRec wr = *(const WaveRec*)rec;
  const WaveBlk b = wr.b;
  const Dev<T> d = *(const Dev<T>*)(rec + sizeof(WaveRec));
  int32_t* acnt = nullptr;
  unsigned long long* acc = nullptr;
  if constexpr (C) {
    acnt = wr.acnt;
    acc = wr.acc;
  }
  __shared__ int s_hist[kRadBins + 1];
  __shared__ unsigned long long s_hmax[kRadBins];
  if constexpr (NEXT == 2) asm volatile("" ::"s"(h), "s"(d.gx), "s"(d.gy), "s"(d.gz), "s"(d.floor_on), "s"(d.jacobi));
  else if constexpr (NEXT == 1) asm volatile("" ::"s"(h), "s"(d.gx), "s"(d.gy), "s"(d.gz));
  else asm volatile("" ::"s"(h));
  const int wave = b.wave;
  stage_setup(d, b, P, pA, pB);
  velocity_load(d, P.A, pA);
  velocity_load(d, P.B, pB);
  int rA = 0, rB = 0;
  T rbA = T(0), rbB = T(0);
  if constexpr (NEXT > 0) {
    P.A.inert = d.inert[pA];
    P.B.inert = d.inert[pB];
    if constexpr (C) {
      rA = d.rod_of[pA];
      rB = d.rod_of[pB];
      rbA = d.rbar[pA];
      rbB = d.rbar[pB];
    }
  }
  if constexpr (NEXT == 2) load_lane_consts<T, X>(d, P, pA, pB, rcp(h * h));
  int moved = 0;
  if constexpr (C) moved = contact_apply_lane(acnt, acc, P, pA, pB);
  const T ih = T(1) / h;
  velocity_store(d, P.A, pA, ih, (moved & 1) != 0);
  velocity_store(d, P.B, pB, ih, (moved & 2) != 0);
  if constexpr (NEXT > 0) {
    // an empty slot's values are left as they are: it stores nothing, and no valid slot
    // reads it (a slot's inertia takes the next pill only when its own edge exists)
    predict_slot(P.A, h, d.gx, d.gy, d.gz);
    predict_slot(P.B, h, d.gx, d.gy, d.gz);
    inertia_lane(P);
    if constexpr (C) detect_start_wave(d, CD[b.scene], P, pA, pB, rA, rB, rbA, rbB, wave, s_hist, s_hmax);
  }
  if constexpr (NEXT == 1) {
    store_predicted(d, P.A, pA);
    store_predicted(d, P.B, pB);
  }
  if constexpr (NEXT == 2) {
    store_substep_start(d, P.A, pA);
    store_substep_start(d, P.B, pB);
    if (d.floor_on) {   // the half-plane floor, at the start of the iteration
      if (P.A.f & F_VALID) floor_apply(d, pA, P.A.x0, P.A.x1, P.A.x2, P.A.s);
      if (P.B.f & F_VALID) floor_apply(d, pB, P.B.x0, P.B.x1, P.B.x2, P.B.s);
    }
    P.I1N = dn(P.A.I1);
    if (d.jacobi) jacobi_lane<T, X>(P);       // wave-uniform: one scene per block
    else iteration_lane<T, X, EVEN>(P);
    store_iter<T, X>(d, P.A, pA);
    store_iter<T, X>(d, P.B, pB);
  }
}

// Field gather/scatter between the SoA layout and a pill-major array.
template <class T>
__global__ void gather_kernel(Dev<T> d, int which, T* out) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= d.P) return;
  const bool edge = (d.flags[p] & F_EDGE) != 0;
  const double* an = d.anchor + 3 * (size_t)d.rod_of[p];
  switch (which) {
    case 0:
      out[3 * p] = (T)(an[0] + (double)d.px[p]);
      out[3 * p + 1] = (T)(an[1] + (double)d.py[p]);
      out[3 * p + 2] = (T)(an[2] + (double)d.pz[p]);
      break;
    case 1: out[3 * p] = d.vx[p]; out[3 * p + 1] = d.vy[p]; out[3 * p + 2] = d.vz[p]; break;
    case 2: out[p] = d.s[p]; break;
    case 3: out[p] = d.sd[p]; break;
    case 4:
      out[4 * p] = edge ? d.qx[p] : T(0); out[4 * p + 1] = edge ? d.qy[p] : T(0);
      out[4 * p + 2] = edge ? d.qz[p] : T(0); out[4 * p + 3] = edge ? d.qw[p] : T(0);
      break;
    case 5:
      out[3 * p] = edge ? d.ox[p] : T(0); out[3 * p + 1] = edge ? d.oy[p] : T(0); out[3 * p + 2] = edge ? d.oz[p] : T(0);
      break;
    case 6: out[p] = d.s[p] * d.rbar[p]; break;
    case 9: out[3 * p] = d.px[p]; out[3 * p + 1] = d.py[p]; out[3 * p + 2] = d.pz[p]; break;
    default: break;
  }
}

template <class T>
__global__ void scatter_kernel(Dev<T> d, int which, const T* in) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= d.P) return;
  const bool edge = (d.flags[p] & F_EDGE) != 0;
  const double* an = d.anchor + 3 * (size_t)d.rod_of[p];
  switch (which) {
    case 0:
      d.px[p] = (T)((double)in[3 * p] - an[0]);
      d.py[p] = (T)((double)in[3 * p + 1] - an[1]);
      d.pz[p] = (T)((double)in[3 * p + 2] - an[2]);
      break;
    case 1: d.vx[p] = in[3 * p]; d.vy[p] = in[3 * p + 1]; d.vz[p] = in[3 * p + 2]; break;
    case 2: d.s[p] = in[p]; break;
    case 3: d.sd[p] = in[p]; break;
    case 4:
      if (edge) { d.qx[p] = in[4 * p]; d.qy[p] = in[4 * p + 1]; d.qz[p] = in[4 * p + 2]; d.qw[p] = in[4 * p + 3]; }
      break;
    case 5:
      if (edge) { d.ox[p] = in[3 * p]; d.oy[p] = in[3 * p + 1]; d.oz[p] = in[3 * p + 2]; }
      break;
    case 9: d.px[p] = in[3 * p]; d.py[p] = in[3 * p + 1]; d.pz[p] = in[3 * p + 2]; break;
    default: break;
  }
}

// ---------------------------------------------------------------- skinning (Sec. 7.4)

// Per capsule: M = [ s R(q) R(q_rest)^T | m - s R(q) R(q_rest)^T m_rest ] as 12 floats.
template <class T>
__global__ void __launch_bounds__(256) skin_transform_kernel(Dev<T> d, float* xf) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= d.P) return;
  if (!(d.flags[p] & F_EDGE)) return;
  // relative rotation q (x) conj(q_rest)
  const T a0 = d.qx[p], a1 = d.qy[p], a2 = d.qz[p], a3 = d.qw[p];
  const T b0 = -d.qrx[p], b1 = -d.qry[p], b2 = -d.qrz[p], b3 = d.qrw[p];
  const T x = a3 * b0 + a0 * b3 + a1 * b2 - a2 * b1;
  const T y = a3 * b1 - a0 * b2 + a1 * b3 + a2 * b0;
  const T z = a3 * b2 + a0 * b1 - a1 * b0 + a2 * b3;
  const T w = a3 * b3 - a0 * b0 - a1 * b1 - a2 * b2;
  const T sm = T(0.5) * (d.s[p] + d.s[p + 1]);
  const T R00 = T(1) - T(2) * (y * y + z * z), R01 = T(2) * (x * y - w * z), R02 = T(2) * (x * z + w * y);
  const T R10 = T(2) * (x * y + w * z), R11 = T(1) - T(2) * (x * x + z * z), R12 = T(2) * (y * z - w * x);
  const T R20 = T(2) * (x * z - w * y), R21 = T(2) * (y * z + w * x), R22 = T(1) - T(2) * (x * x + y * y);
  // translation m - s R m_rest in world coordinates (FP64): anchor + local midpoints
  const double* an = d.anchor + 3 * (size_t)d.rod_of[p];
  const double m0 = an[0] + 0.5 * ((double)d.px[p] + (double)d.px[p + 1]);
  const double m1 = an[1] + 0.5 * ((double)d.py[p] + (double)d.py[p + 1]);
  const double m2 = an[2] + 0.5 * ((double)d.pz[p] + (double)d.pz[p + 1]);
  const double r0 = an[0] + (double)d.mrx[p], r1 = an[1] + (double)d.mry[p], r2 = an[2] + (double)d.mrz[p];
  const double s0 = (double)sm;
  float* o = xf + (size_t)12 * p;
  o[0] = (float)(sm * R00); o[1] = (float)(sm * R01); o[2] = (float)(sm * R02);
  o[3] = (float)(m0 - s0 * ((double)R00 * r0 + (double)R01 * r1 + (double)R02 * r2));
  o[4] = (float)(sm * R10); o[5] = (float)(sm * R11); o[6] = (float)(sm * R12);
  o[7] = (float)(m1 - s0 * ((double)R10 * r0 + (double)R11 * r1 + (double)R12 * r2));
  o[8] = (float)(sm * R20); o[9] = (float)(sm * R21); o[10] = (float)(sm * R22);
  o[11] = (float)(m2 - s0 * ((double)R20 * r0 + (double)R21 * r1 + (double)R22 * r2));
}

// Per vertex: 4 gathers of the transform table (L2-resident), one blended affine map.
__global__ void __launch_bounds__(256) lbs_kernel(int V, const float* __restrict__ rest_v, const int4* __restrict__ caps,
                                                  const float4* __restrict__ w, const float4* __restrict__ xf,
                                                  float* __restrict__ out) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= V) return;
  const int4 c = caps[i];
  const float4 wt = w[i];
  const float vx = rest_v[3 * i], vy = rest_v[3 * i + 1], vz = rest_v[3 * i + 2];
  // Issue every streamed load before the gathers: left alone, the scheduler sinks the
  // weight load below them and each wave pays a second HBM round trip.
  __builtin_amdgcn_sched_barrier(0);
  const int ci[4] = {c.x, c.y, c.z, c.w};
  const float wk[4] = {wt.x, wt.y, wt.z, wt.w};
  float o0 = 0.f, o1 = 0.f, o2 = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float4 r0 = xf[3 * (size_t)ci[k] + 0];
    const float4 r1 = xf[3 * (size_t)ci[k] + 1];
    const float4 r2 = xf[3 * (size_t)ci[k] + 2];
    o0 += wk[k] * (r0.x * vx + r0.y * vy + r0.z * vz + r0.w);
    o1 += wk[k] * (r1.x * vx + r1.y * vy + r1.z * vz + r1.w);
    o2 += wk[k] * (r2.x * vx + r2.y * vy + r2.z * vz + r2.w);
  }
  out[3 * i] = o0; out[3 * i + 1] = o1; out[3 * i + 2] = o2;
}

// ---------------------------------------------------------------- launchers

template <class T, bool X, bool EVEN>
void launch_rod_frame_as(const BatchDev& b, int nsub, double h, int iters, hipStream_t st) {
  hipLaunchKernelGGL((rod_frame_kernel<T, X, EVEN>), dim3(b.nblk[TB_WAVES]), dim3(256), 0, st, (const Dev<T>*)b.dev,
                     b.tab[TB_WAVES], nsub, (T)h, iters);
}
template <class T> hipError_t launch_rod_frame(const BatchDev& b, int nsub, double h, int iters, hipStream_t st) {
  if (b.nblk[TB_WAVES] == 0) return hipSuccess;
  if (b.extras) {
    if (b.even) launch_rod_frame_as<T, true, true>(b, nsub, h, iters, st);
    else launch_rod_frame_as<T, true, false>(b, nsub, h, iters, st);
  } else {
    if (b.even) launch_rod_frame_as<T, false, true>(b, nsub, h, iters, st);
    else launch_rod_frame_as<T, false, false>(b, nsub, h, iters, st);
  }
  return hipGetLastError();
}
template <class T> hipError_t launch_predict(const BatchDev& b, double h, const ContactDev* cd, hipStream_t st) {
  if (b.nblk[TB_WAVES] == 0) return hipSuccess;
  if (cd)
    hipLaunchKernelGGL((predict_kernel<T, true>), dim3(b.nwaves), dim3(64), 0, st, b.wrec, b.wrec_stride, (T)h,
                       cd);
  else
    hipLaunchKernelGGL((predict_kernel<T, false>), dim3(b.nwaves), dim3(64), 0, st, b.wrec, b.wrec_stride, (T)h,
                       cd);
  return hipGetLastError();
}
template <class T, bool X, bool EVEN>
void launch_rod_iteration_as(const BatchDev& b, double h, const ContactDev* cd, hipStream_t st) {
  if (cd)
    hipLaunchKernelGGL((rod_iteration_kernel<T, X, EVEN, true>), dim3(b.nwaves), dim3(64), 0, st, b.wrec,
                       b.wrec_stride, (T)h, cd);
  else
    hipLaunchKernelGGL((rod_iteration_kernel<T, X, EVEN, false>), dim3(b.nwaves), dim3(64), 0, st, b.wrec,
                       b.wrec_stride, (T)h, cd);
}
template <class T> hipError_t launch_rod_iteration(const BatchDev& b, double h, const ContactDev* cd, hipStream_t st) {
  if (b.nblk[TB_WAVES] == 0) return hipSuccess;
  if (b.extras) {
    if (b.even) launch_rod_iteration_as<T, true, true>(b, h, cd, st);
    else launch_rod_iteration_as<T, true, false>(b, h, cd, st);
  } else {
    if (b.even) launch_rod_iteration_as<T, false, true>(b, h, cd, st);
    else launch_rod_iteration_as<T, false, false>(b, h, cd, st);
  }
  return hipGetLastError();
}
template <class T, bool C, int NEXT, bool X, bool EVEN>
void launch_velocity_as(const BatchDev& b, double h, const ContactDev* cd, hipStream_t st) {
  hipLaunchKernelGGL((velocity_kernel<T, C, NEXT, X, EVEN>), dim3(b.nwaves), dim3(64), 0, st, b.wrec, b.wrec_stride,
                     (T)h, cd);
}
template <class T, bool C>
void launch_velocity_c(const BatchDev& b, double h, const ContactDev* cd, int next, hipStream_t st) {
  if (next == 0) launch_velocity_as<T, C, 0, false, false>(b, h, cd, st);
  else if (next == 1) launch_velocity_as<T, C, 1, false, false>(b, h, cd, st);
  else if (b.extras) {
    if (b.even) launch_velocity_as<T, C, 2, true, true>(b, h, cd, st);
    else launch_velocity_as<T, C, 2, true, false>(b, h, cd, st);
  } else {
    if (b.even) launch_velocity_as<T, C, 2, false, true>(b, h, cd, st);
    else launch_velocity_as<T, C, 2, false, false>(b, h, cd, st);
  }
}
template <class T>
hipError_t launch_velocity(const BatchDev& b, double h, const ContactDev* cd, int next, hipStream_t st) {
  if (b.nblk[TB_WAVES] == 0) return hipSuccess;
  if (next < 0 || next > 2) return hipErrorInvalidValue;
  if (cd) launch_velocity_c<T, true>(b, h, cd, next, st);
  else launch_velocity_c<T, false>(b, h, cd, next, st);
  return hipGetLastError();
}
template <class T> hipError_t launch_gather_field(const Dev<T>& d, int which, T* out, hipStream_t st) {
  if (d.P == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel<T>, dim3((d.P + 255) / 256), dim3(256), 0, st, d, which, out);
  return hipGetLastError();
}
template <class T> hipError_t launch_scatter_field(const Dev<T>& d, int which, const T* in, hipStream_t st) {
  if (d.P == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel<T>, dim3((d.P + 255) / 256), dim3(256), 0, st, d, which, in);
  return hipGetLastError();
}
template <class T> hipError_t launch_skin(const Dev<T>& d, int V, const float* rest_v, const int32_t* caps,
                                          const float* w, float* out, float* xform, hipStream_t st) {
  if (d.P > 0) hipLaunchKernelGGL(skin_transform_kernel<T>, dim3((d.P + 255) / 256), dim3(256), 0, st, d, xform);
  if (V > 0)
    hipLaunchKernelGGL(lbs_kernel, dim3((V + 255) / 256), dim3(256), 0, st, V, rest_v, (const int4*)caps,
                       (const float4*)w, (const float4*)xform, out);
  return hipGetLastError();
}

#define VIPER_INST(T)                                                                                         \
  template hipError_t launch_rod_frame<T>(const BatchDev&, int, double, int, hipStream_t);                   \
  template hipError_t launch_predict<T>(const BatchDev&, double, const ContactDev*, hipStream_t);            \
  template hipError_t launch_rod_iteration<T>(const BatchDev&, double, const ContactDev*, hipStream_t);      \
  template hipError_t launch_velocity<T>(const BatchDev&, double, const ContactDev*, int, hipStream_t);           \
  template hipError_t launch_gather_field<T>(const Dev<T>&, int, T*, hipStream_t);                           \
  template hipError_t launch_scatter_field<T>(const Dev<T>&, int, const T*, hipStream_t);                    \
  template hipError_t launch_skin<T>(const Dev<T>&, int, const float*, const int32_t*, const float*, float*, \
                                     float*, hipStream_t);
VIPER_INST(float)
VIPER_INST(double)

}  // namespace viper
