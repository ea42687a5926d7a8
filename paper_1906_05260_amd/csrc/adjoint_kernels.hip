// Adjoint (reverse mode) of the collision-free rod frame, for gfx950.
//
// Forward: the frame kernel variant below also writes the state at the start of every
// substep (per-substep checkpoint).  Backward: one launch per substep, in reverse order.
// Each launch reloads its checkpoint, recomputes the substep exactly as the forward does
// (same device code) while storing the state before every colour pass, then sweeps back:
// velocity update, the 4 x iterations passes in reverse, the substep-start inertia, and
// the prediction.  The vector-Jacobian product of each projection is formed from forward
// derivatives of that projection taken with dual numbers over the same templated update
// (four input directions per evaluation), so the adjoint differentiates exactly the
// arithmetic the forward performs.  Adjoints of the per-slot parameters (inverse masses,
// inverse stretch rest length, inertia base, compliance scalings) are accumulated per
// slot and chained to rest radii and activations on the host.

#include <type_traits>

#include "rod_device.h"

namespace viper {

// ---------------------------------------------------------------- dual numbers

template <class S, int K>
struct Dual {
  S v;
  S d[K];
  __device__ __forceinline__ Dual() : v(S(0)) {
#pragma unroll
    for (int k = 0; k < K; ++k) d[k] = S(0);
  }
  template <class U, class = typename std::enable_if<std::is_arithmetic<U>::value>::type>
  __device__ __forceinline__ Dual(U a) : v(S(a)) {
#pragma unroll
    for (int k = 0; k < K; ++k) d[k] = S(0);
  }
};

template <class S, int K> __device__ __forceinline__ Dual<S, K> operator+(const Dual<S, K>& a, const Dual<S, K>& b) {
  Dual<S, K> r; r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <class S, int K> __device__ __forceinline__ Dual<S, K> operator-(const Dual<S, K>& a, const Dual<S, K>& b) {
  Dual<S, K> r; r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <class S, int K> __device__ __forceinline__ Dual<S, K> operator-(const Dual<S, K>& a) {
  Dual<S, K> r; r.v = -a.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}
template <class S, int K> __device__ __forceinline__ Dual<S, K> operator*(const Dual<S, K>& a, const Dual<S, K>& b) {
  Dual<S, K> r; r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <class S, int K> __device__ __forceinline__ Dual<S, K>& operator+=(Dual<S, K>& a, const Dual<S, K>& b) { a = a + b; return a; }
template <class S, int K> __device__ __forceinline__ Dual<S, K>& operator-=(Dual<S, K>& a, const Dual<S, K>& b) { a = a - b; return a; }
template <class S, int K> __device__ __forceinline__ bool operator<(const Dual<S, K>& a, const Dual<S, K>& b) { return a.v < b.v; }
template <class S, int K> __device__ __forceinline__ bool operator>(const Dual<S, K>& a, const Dual<S, K>& b) { return a.v > b.v; }
// the same hardware reciprocal / rsqrt as the forward, with their exact derivatives
template <class S, int K> __device__ __forceinline__ Dual<S, K> rcp(const Dual<S, K>& a) {
  Dual<S, K> r; r.v = rcp(a.v);
  const S g = -r.v * r.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = g * a.d[k];
  return r;
}
template <class S, int K> __device__ __forceinline__ Dual<S, K> rsq(const Dual<S, K>& a) {
  Dual<S, K> r; r.v = rsq(a.v);
  const S g = S(-0.5) * r.v * r.v * r.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = g * a.d[k];
  return r;
}

// Input directions per dual evaluation: four in FP32, two in FP64 (register budget).
template <class T> struct KDim { static constexpr int v = 4; };
template <> struct KDim<double> { static constexpr int v = 2; };
template <class T> using DT = Dual<T, KDim<T>::v>;

// Seed in[i] with unit derivative in direction i - c0 when i lies in [c0, c0 + KD).
template <class T, int N>
__device__ __forceinline__ void seed(DT<T> (&in)[N], const T (&v)[N], int c0) {
  constexpr int KD = KDim<T>::v;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    in[i] = DT<T>(v[i]);
#pragma unroll
    for (int k = 0; k < KD; ++k) in[i].d[k] = (i == c0 + k) ? T(1) : T(0);
  }
}

// xb[c0 + k] = sum_o yb[o] d out[o] / d in[c0 + k]
template <class T, int N, int M>
__device__ __forceinline__ void gather_vjp(const DT<T> (&out)[M], const T (&yb)[M], int c0, T (&xb)[N]) {
  constexpr int KD = KDim<T>::v;
  T acc[KD];
#pragma unroll
  for (int k = 0; k < KD; ++k) {
    acc[k] = T(0);
#pragma unroll
    for (int o = 0; o < M; ++o) acc[k] += yb[o] * out[o].d[k];
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < KD; ++k)
      if (i == c0 + k) xb[i] = acc[k];
}

// ---------------------------------------------------------------- local VJPs

// The backward kernel runs every logical lane in kReps replica waves of one block: all
// replicas recompute the same state, and the input-direction chunks of each local VJP are
// split between them (chunk c on replica c % kReps); share_chunks then gives every replica
// the full result through LDS.  Called by all threads of the block (it has barriers).
constexpr int kReps = 4;

template <class T, int N>
__device__ __forceinline__ void share_chunks(T (&xb)[N], int rep, T* X, int lane) {
  constexpr int KD = KDim<T>::v;
#pragma unroll
  for (int i = 0; i < N; ++i)
    if ((i / KD) % kReps == rep) X[i * 64 + lane] = xb[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) xb[i] = X[i * 64 + lane];
  __syncthreads();
}

// Stretch-shear + volume + scale gradient of slot L's edge (edge_update).
// Inputs (26): x0 x1 x2 s q0 q1 q2 q3 l0..l4 | b0 b1 b2 sb | w ws ilb ass avol asg I1 | wb wsb
// Outputs (17): x0 x1 x2 s q0..q3 l0..l4 | b0 b1 b2 sb
template <class T>
__device__ void edge_vjp(const Slot<T>& L, T b0, T b1, T b2, T sb, T wb, T wsb, const T (&yb)[17], T (&xb)[26],
                         int rep, T* X, int lane) {
  constexpr int KD = KDim<T>::v;
  const T v[26] = {L.x0, L.x1, L.x2, L.s, L.q0, L.q1, L.q2, L.q3, L.l[0], L.l[1], L.l[2], L.l[3], L.l[4],
                   b0, b1, b2, sb, L.w, L.ws, L.ilb, L.ass, L.avol, L.asg, L.I1, wb, wsb};
#pragma unroll
  for (int i = 0; i < 26; ++i) xb[i] = T(0);
  for (int c0 = rep * KD; c0 < 26; c0 += kReps * KD) {
    DT<T> in[26];
    seed(in, v, c0);
    Slot<DT<T>> S;
    S.f = L.f;
    S.x0 = in[0]; S.x1 = in[1]; S.x2 = in[2]; S.s = in[3];
    S.q0 = in[4]; S.q1 = in[5]; S.q2 = in[6]; S.q3 = in[7];
    S.l[0] = in[8]; S.l[1] = in[9]; S.l[2] = in[10]; S.l[3] = in[11]; S.l[4] = in[12];
    DT<T> c0_ = in[13], c1_ = in[14], c2_ = in[15], cs_ = in[16];
    S.w = in[17]; S.ws = in[18]; S.ilb = in[19]; S.ass = in[20]; S.avol = in[21]; S.asg = in[22]; S.I1 = in[23];
    S.il0 = DT<T>(L.il0);
    edge_update(S, c0_, c1_, c2_, cs_, in[24], in[25]);
    const DT<T> out[17] = {S.x0, S.x1, S.x2, S.s, S.q0, S.q1, S.q2, S.q3, S.l[0], S.l[1], S.l[2], S.l[3], S.l[4],
                           c0_, c1_, c2_, cs_};
    gather_vjp(out, yb, c0, xb);
  }
  share_chunks(xb, rep, X, lane);
}

// Bend-twist between slot L's edge and the next edge (bt_update).
// Inputs (16): q0..q3 l5 l6 l7 | b0..b3 sb | Ia Ib wsb abt      Outputs (12): q0..q3 l5..l7 | b0..b3 sb
template <class T>
__device__ void bt_vjp(const Slot<T>& L, T b0, T b1, T b2, T b3, T sb, T Ib, T wsb, const T (&yb)[12], T (&xb)[16],
                       int rep, T* X, int lane) {
  constexpr int KD = KDim<T>::v;
  const T v[16] = {L.q0, L.q1, L.q2, L.q3, L.l[5], L.l[6], L.l[7], b0, b1, b2, b3, sb, L.I1, Ib, wsb, L.abt};
#pragma unroll
  for (int i = 0; i < 16; ++i) xb[i] = T(0);
  for (int c0 = rep * KD; c0 < 16; c0 += kReps * KD) {
    DT<T> in[16];
    seed(in, v, c0);
    Slot<DT<T>> S;
    S.f = L.f;
    S.q0 = in[0]; S.q1 = in[1]; S.q2 = in[2]; S.q3 = in[3];
    S.l[5] = in[4]; S.l[6] = in[5]; S.l[7] = in[6];
    DT<T> e0 = in[7], e1 = in[8], e2 = in[9], e3 = in[10], es = in[11];
    S.I1 = in[12]; S.abt = in[15];
    S.cbt = DT<T>(L.cbt); S.db0 = DT<T>(L.db0); S.db1 = DT<T>(L.db1); S.db2 = DT<T>(L.db2);
    bt_update(S, e0, e1, e2, e3, es, in[13], in[14]);
    const DT<T> out[12] = {S.q0, S.q1, S.q2, S.q3, S.l[5], S.l[6], S.l[7], e0, e1, e2, e3, es};
    gather_vjp(out, yb, c0, xb);
  }
  share_chunks(xb, rep, X, lane);
}

// Angular velocity from the quaternions after / before the substep (omega_of).
// Inputs (8): q0..q3 p0..p3       Outputs (3): o0 o1 o2
template <class T>
__device__ void omega_vjp(const Slot<T>& L, T ih, const T (&yb)[3], T (&xb)[8]) {
  const T v[8] = {L.q0, L.q1, L.q2, L.q3, L.qp0, L.qp1, L.qp2, L.qp3};
  for (int c0 = 0; c0 < 8; c0 += KDim<T>::v) {
    DT<T> in[8];
    seed(in, v, c0);
    DT<T> o[3];
    omega_of(in[0], in[1], in[2], in[3], in[4], in[5], in[6], in[7], DT<T>(ih), o[0], o[1], o[2]);
    gather_vjp(o, yb, c0, xb);
  }
}

// Predicted quaternion normalize(q + 1/2 [h w, 0] (x) q).
// Inputs (7): q0..q3 w0 w1 w2     Outputs (4): q0..q3
template <class T>
__device__ void qpredict_vjp(T q0, T q1, T q2, T q3, T w0, T w1, T w2, T h, const T (&yb)[4], T (&xb)[7]) {
  const T v[7] = {q0, q1, q2, q3, w0, w1, w2};
  for (int c0 = 0; c0 < 7; c0 += KDim<T>::v) {
    DT<T> in[7];
    seed(in, v, c0);
    DT<T> a = in[0], b = in[1], c = in[2], e = in[3];
    const DT<T> hh(h);
    qrot_world(a, b, c, e, hh * in[4], hh * in[5], hh * in[6]);
    const DT<T> out[4] = {a, b, c, e};
    gather_vjp(out, yb, c0, xb);
  }
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

// Snapshot of the pre-pass state of both slots (x, s, q, lambda): 32 values per lane,
// stored field-major over the scene's lanes for coalesced access.
template <class T>
__device__ __forceinline__ void snap_io(T* base, size_t NL, Slot<T>& A, Slot<T>& B, bool store) {
#define SNAP_FIELD(i, ref) { T* p = base + (size_t)(i) * NL; if (store) *p = (ref); else (ref) = *p; }
  SNAP_FIELD(0, A.x0) SNAP_FIELD(1, A.x1) SNAP_FIELD(2, A.x2) SNAP_FIELD(3, A.s)
  SNAP_FIELD(4, A.q0) SNAP_FIELD(5, A.q1) SNAP_FIELD(6, A.q2) SNAP_FIELD(7, A.q3)
  SNAP_FIELD(16, B.x0) SNAP_FIELD(17, B.x1) SNAP_FIELD(18, B.x2) SNAP_FIELD(19, B.s)
  SNAP_FIELD(20, B.q0) SNAP_FIELD(21, B.q1) SNAP_FIELD(22, B.q2) SNAP_FIELD(23, B.q3)
#pragma unroll
  for (int i = 0; i < 8; ++i) { SNAP_FIELD(8 + i, A.l[i]) SNAP_FIELD(24 + i, B.l[i]) }
#undef SNAP_FIELD
}

// ---------------------------------------------------------------- reverse passes

// Every lane calls the local VJP once per pass (the call has block barriers): on its A edge,
// its B edge, or on a dummy whose result it discards.
template <class T>
__device__ void pass_edges_vjp(Lane2<T>& P, SAdj<T>& aA, SAdj<T>& aB, int colour, int rep, T* X, int lane) {
  const T n0 = dn(P.A.x0), n1 = dn(P.A.x1), n2 = dn(P.A.x2), ns = dn(P.A.s);       // pre-pass next slot A
  const T g0 = dn(aA.x0), g1 = dn(aA.x1), g2 = dn(aA.x2), gs = dn(aA.s);            // adjoint of its post-pass value
  const bool useA = (P.A.f & F_EDGE) && colour_is(P.A.f, colour);
  const bool useB = !useA && (P.B.f & F_EDGE) && colour_is(P.B.f, colour);
  const Slot<T> L = useB ? P.B : P.A;
  const T yb[17] = {useB ? aB.x0 : aA.x0, useB ? aB.x1 : aA.x1, useB ? aB.x2 : aA.x2, useB ? aB.s : aA.s,
                    useB ? aB.q0 : aA.q0, useB ? aB.q1 : aA.q1, useB ? aB.q2 : aA.q2, useB ? aB.q3 : aA.q3,
                    useB ? aB.l[0] : aA.l[0], useB ? aB.l[1] : aA.l[1], useB ? aB.l[2] : aA.l[2],
                    useB ? aB.l[3] : aA.l[3], useB ? aB.l[4] : aA.l[4],
                    useB ? g0 : aB.x0, useB ? g1 : aB.x1, useB ? g2 : aB.x2, useB ? gs : aB.s};
  T xb[26];
  edge_vjp(L, useB ? n0 : P.B.x0, useB ? n1 : P.B.x1, useB ? n2 : P.B.x2, useB ? ns : P.B.s,
           useB ? P.wN : P.B.w, useB ? P.wsN : P.B.ws, yb, xb, rep, X, lane);
  T r0 = T(0), r1 = T(0), r2 = T(0), rs = T(0), rw = T(0), rws = T(0);
  if (useA) {
    aA.x0 = xb[0]; aA.x1 = xb[1]; aA.x2 = xb[2]; aA.s = xb[3];
    aA.q0 = xb[4]; aA.q1 = xb[5]; aA.q2 = xb[6]; aA.q3 = xb[7];
    aA.l[0] = xb[8]; aA.l[1] = xb[9]; aA.l[2] = xb[10]; aA.l[3] = xb[11]; aA.l[4] = xb[12];
    aB.x0 = xb[13]; aB.x1 = xb[14]; aB.x2 = xb[15]; aB.s = xb[16];
    aA.w += xb[17]; aA.ws += xb[18]; aA.ilb += xb[19]; aA.ass += xb[20]; aA.avol += xb[21]; aA.asg += xb[22];
    aA.I1 += xb[23]; aB.w += xb[24]; aB.ws += xb[25];
  } else if (useB) {
    aB.x0 = xb[0]; aB.x1 = xb[1]; aB.x2 = xb[2]; aB.s = xb[3];
    aB.q0 = xb[4]; aB.q1 = xb[5]; aB.q2 = xb[6]; aB.q3 = xb[7];
    aB.l[0] = xb[8]; aB.l[1] = xb[9]; aB.l[2] = xb[10]; aB.l[3] = xb[11]; aB.l[4] = xb[12];
    r0 = xb[13]; r1 = xb[14]; r2 = xb[15]; rs = xb[16];
    aB.w += xb[17]; aB.ws += xb[18]; aB.ilb += xb[19]; aB.ass += xb[20]; aB.avol += xb[21]; aB.asg += xb[22];
    aB.I1 += xb[23]; rw = xb[24]; rws = xb[25];
  }
  r0 = up(r0); r1 = up(r1); r2 = up(r2); rs = up(rs); rw = up(rw); rws = up(rws);
  if ((P.A.f & F_VALID) && !(P.A.f & F_FIRST) && !colour_is(P.A.f, colour)) {
    aA.x0 = r0; aA.x1 = r1; aA.x2 = r2; aA.s = rs; aA.w += rw; aA.ws += rws;
  }
}

template <class T>
__device__ void pass_bt_vjp(Lane2<T>& P, SAdj<T>& aA, SAdj<T>& aB, int colour, int rep, T* X, int lane) {
  const T n0 = dn(P.A.q0), n1 = dn(P.A.q1), n2 = dn(P.A.q2), n3 = dn(P.A.q3), ns = dn(P.A.s);
  const T g0 = dn(aA.q0), g1 = dn(aA.q1), g2 = dn(aA.q2), g3 = dn(aA.q3), gs = dn(aA.s);
  const bool useA = (P.A.f & F_BT) && (P.A.f & F_BTEN) && colour_is(P.A.f, colour);
  const bool useB = !useA && (P.B.f & F_BT) && (P.B.f & F_BTEN) && colour_is(P.B.f, colour);
  const Slot<T> L = useB ? P.B : P.A;
  const T yb[12] = {useB ? aB.q0 : aA.q0, useB ? aB.q1 : aA.q1, useB ? aB.q2 : aA.q2, useB ? aB.q3 : aA.q3,
                    useB ? aB.l[5] : aA.l[5], useB ? aB.l[6] : aA.l[6], useB ? aB.l[7] : aA.l[7],
                    useB ? g0 : aB.q0, useB ? g1 : aB.q1, useB ? g2 : aB.q2, useB ? g3 : aB.q3, useB ? gs : aB.s};
  T xb[16];
  bt_vjp(L, useB ? n0 : P.B.q0, useB ? n1 : P.B.q1, useB ? n2 : P.B.q2, useB ? n3 : P.B.q3, useB ? ns : P.B.s,
         useB ? P.I1N : P.B.I1, useB ? P.wsN : P.B.ws, yb, xb, rep, X, lane);
  T r0 = T(0), r1 = T(0), r2 = T(0), r3 = T(0), rs = T(0), rI = T(0), rws = T(0);
  if (useA) {
    aA.q0 = xb[0]; aA.q1 = xb[1]; aA.q2 = xb[2]; aA.q3 = xb[3];
    aA.l[5] = xb[4]; aA.l[6] = xb[5]; aA.l[7] = xb[6];
    aB.q0 = xb[7]; aB.q1 = xb[8]; aB.q2 = xb[9]; aB.q3 = xb[10]; aB.s = xb[11];
    aA.I1 += xb[12]; aB.I1 += xb[13]; aB.ws += xb[14]; aA.abt += xb[15];
  } else if (useB) {
    aB.q0 = xb[0]; aB.q1 = xb[1]; aB.q2 = xb[2]; aB.q3 = xb[3];
    aB.l[5] = xb[4]; aB.l[6] = xb[5]; aB.l[7] = xb[6];
    r0 = xb[7]; r1 = xb[8]; r2 = xb[9]; r3 = xb[10]; rs = xb[11];
    aB.I1 += xb[12]; rI = xb[13]; rws = xb[14]; aB.abt += xb[15];
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

// Reverse of one substep.  adj ([field][pill], kCkptFields) holds the adjoint of the state
// at the end of the substep on entry and at its start on exit; padj ([8][pill]) accumulates
// the parameter adjoints: 1/M, 1/M_s, 1/lbar, rho pi r^4 l0, and the four compliance
// scalings; snap is this lane's pass-snapshot scratch.
// Block b works on logical wavefront tab[b / 4].base + b % 4 (the forward's lane layout),
// replicated in its kReps waves: replica r = wave index within the block.  A whole block is
// inactive or active, so the early return never splits a barrier.
template <class T>
__device__ __forceinline__ const Dev<T>* lane_setup_rep(const Dev<T>* D, const Blk* tab, Lane2<T>& P, int& pA,
                                                        int& pB, int& wave) {
  const Blk b = tab[blockIdx.x >> 2];
  const Dev<T>* d = D + b.scene;
  wave = b.base + (int)(blockIdx.x & 3);
  const int lane = (int)(threadIdx.x & 63);
  if (wave >= d->W) return nullptr;
  const int p0 = d->wave_start[wave];
  const int n = d->wave_start[wave + 1] - p0;
  const bool vA = 2 * lane < n, vB = 2 * lane + 1 < n;
  pA = p0 + (vA ? 2 * lane : 0);
  pB = p0 + (vB ? 2 * lane + 1 : 0);
  P.A.f = vA ? d->flags[pA] : 0u;
  P.B.f = vB ? d->flags[pB] : 0u;
  return d;
}

template <class T, bool EVEN>
__global__ void __launch_bounds__(64 * kReps) rod_backward_kernel(const Dev<T>* __restrict__ D, const Blk* __restrict__ tab,
                                                           T h, int iters, const T* __restrict__ ckpt, T* __restrict__ snap,
                                                           T* __restrict__ adj, T* __restrict__ padj) {
  __shared__ T X[26 * 64];                 // chunk exchange between the replicas
  Lane2<T> P;
  int pA, pB, wave;
  const Dev<T>* dp = lane_setup_rep(D, tab, P, pA, pB, wave);
  if (!dp) return;
  const Dev<T>& d = *dp;
  const int lane = (int)(threadIdx.x & 63);
  const int rep = (int)(threadIdx.x >> 6);
  const bool writer = rep == 0;
  const size_t NL = (size_t)d.W * 64;
  const size_t lg = (size_t)wave * 64 + lane;
  T* cbase = const_cast<T*>(ckpt);
  ckpt_io(cbase, d.P, pA, P.A, false);
  ckpt_io(cbase, d.P, pB, P.B, false);
  const T ih2 = rcp(h * h);
  load_lane_consts(d, P, pA, pB, ih2);
  const T ih = T(1) / h;
  // forward recompute with pass snapshots
  predict_slot(P.A, h, d.gx, d.gy, d.gz);
  predict_slot(P.B, h, d.gx, d.gy, d.gz);
  inertia_lane(P);
  for (int it = 0; it < iters; ++it) {
    for (int k = 0; k < 4; ++k) {
      if (writer) snap_io(snap + ((size_t)(it * 4 + k) * 32) * NL + lg, NL, P.A, P.B, true);
      if (k < 2) pass_edges<T, false, EVEN>(P, k); else pass_bt<T, EVEN>(P, k - 2);
    }
  }
  velocity_slot(P.A, ih);
  velocity_slot(P.B, ih);
  __syncthreads();                         // the snapshots of replica 0 are read by all
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
  // the passes in reverse order, each from its pre-pass snapshot
  for (int it = iters - 1; it >= 0; --it) {
    for (int k = 3; k >= 0; --k) {
      snap_io(snap + ((size_t)(it * 4 + k) * 32) * NL + lg, NL, P.A, P.B, false);
      if (k < 2) pass_edges_vjp(P, aA, aB, k, rep, X, lane); else pass_bt_vjp(P, aA, aB, k - 2, rep, X, lane);
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
    if (!writer) continue;
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
  for (int sub = nsub - 1; sub >= 0; --sub) {
    const T* ck = ckpt + (size_t)sub * kCkptFields * P;
    if (b.even)
      hipLaunchKernelGGL((rod_backward_kernel<T, true>), dim3(4 * b.nblk[TB_WAVES]), dim3(64 * kReps), 0, st,
                         (const Dev<T>*)b.dev, b.tab[TB_WAVES], (T)h, iters, ck, snap, adj, padj);
    else
      hipLaunchKernelGGL((rod_backward_kernel<T, false>), dim3(4 * b.nblk[TB_WAVES]), dim3(64 * kReps), 0, st,
                         (const Dev<T>*)b.dev, b.tab[TB_WAVES], (T)h, iters, ck, snap, adj, padj);
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
