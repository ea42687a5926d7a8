// Scale-invariant shape matching of muscle cross-sections ("bundling", Sec. 7.3, eq.
// shapematch) for gfx950.
//
// Every pill i of a cross-section carries the similarity transform T_i = [s_i R_i | x_i]
// (its scale, the rotation of the edge that starts at it -- of its incoming edge for a
// rod's last pill -- and its position).  Once per substep, after the constraint
// iterations, each section is fitted with the global similarity T* = [s* R* | c*] that
// minimises sum_i |T* Tbar_i - T_i|^2 over its rest transforms Tbar_i = [Rbar_i | xbar_i]
// (Umeyama):
//     mu, mubar   = means of x_i, xbar_i
//     A           = sum_i [s_i R_i | x_i - mu] [Rbar_i | xbar_i - mubar]^T     (3x3)
//     R*          = argmax_R trace(R^T A) over SO(3)   (rotation extraction of Mueller
//                   et al. 2016, started from the section's rotation of the previous substep)
//     s*          = trace(R*^T A) / sum_i (3 + |xbar_i - mubar|^2)
//     c*          = mu - s* R* mubar
// and every pill is then set to T* Tbar_i: x_i = s* R* xbar_i + c* (pinned pills keep
// their position), s_i = s*, q_i = q* (x) qbar_i for pills with an edge.
//
// Layout: one wavefront per section for the fit (sums over its entries by butterfly
// reduction, FP64 in world coordinates: the rods of a section have different anchors),
// one thread per section entry for the update.  Every section is fitted from the same
// state before any is updated (two launches).

#include "viper_dev.h"

namespace viper {
namespace {

__device__ __forceinline__ void qmat_d(double x, double y, double z, double w, double* M) {
  M[0] = 1.0 - 2.0 * (y * y + z * z); M[1] = 2.0 * (x * y - w * z);       M[2] = 2.0 * (x * z + w * y);
  M[3] = 2.0 * (x * y + w * z);       M[4] = 1.0 - 2.0 * (x * x + z * z); M[5] = 2.0 * (y * z - w * x);
  M[6] = 2.0 * (x * z - w * y);       M[7] = 2.0 * (y * z + w * x);       M[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Sum over the wavefront, the same value on every lane (lane 0's, broadcast).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return __shfl(v, 0);
}

template <class T>
__global__ void __launch_bounds__(256) bundle_fit_kernel(const Dev<T>* __restrict__ D, const Blk* __restrict__ tab) {
  const Blk blk = tab[blockIdx.x];
  const Dev<T>& d = D[blk.scene];
  const int k = blk.base + (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  if (k >= d.nsec) return;                       // whole wavefronts leave together
  const int i0 = d.sec_off[k], i1 = d.sec_off[k + 1];
  const double inv_n = 1.0 / (double)(i1 - i0);
  // means of the current and rest positions
  double m[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = i0 + lane; i < i1; i += 64) {
    const int p = d.sec_pill[i];
    const double* an = d.anchor + 3 * (size_t)d.rod_of[p];
    m[0] += an[0] + (double)d.px[p];
    m[1] += an[1] + (double)d.py[p];
    m[2] += an[2] + (double)d.pz[p];
    m[3] += d.sec_xr[3 * (size_t)i];
    m[4] += d.sec_xr[3 * (size_t)i + 1];
    m[5] += d.sec_xr[3 * (size_t)i + 2];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) m[j] = inv_n * wave_sum(m[j]);
  // A = sum_i [s_i R_i | x_i - mu] [Rbar_i | xbar_i - mubar]^T,  Dn = sum_i |[Rbar_i | xbar_i - mubar]|^2
  double A[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, Dn = 0.0;
  for (int i = i0 + lane; i < i1; i += 64) {
    const int p = d.sec_pill[i];
    const int e = (d.flags[p] & F_EDGE) ? p : p - 1;
    const double* an = d.anchor + 3 * (size_t)d.rod_of[p];
    const double dv[3] = {an[0] + (double)d.px[p] - m[0], an[1] + (double)d.py[p] - m[1],
                          an[2] + (double)d.pz[p] - m[2]};
    const double db[3] = {d.sec_xr[3 * (size_t)i] - m[3], d.sec_xr[3 * (size_t)i + 1] - m[4],
                          d.sec_xr[3 * (size_t)i + 2] - m[5]};
    double R[9], Rb[9];
    qmat_d((double)d.qx[e], (double)d.qy[e], (double)d.qz[e], (double)d.qw[e], R);
    qmat_d((double)d.qrx[e], (double)d.qry[e], (double)d.qrz[e], (double)d.qrw[e], Rb);
    const double s = (double)d.s[p];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double acc = dv[r] * db[c];
#pragma unroll
        for (int t = 0; t < 3; ++t) acc += (s * R[3 * r + t]) * Rb[3 * c + t];
        A[3 * r + c] += acc;
      }
    Dn += 3.0 + (db[0] * db[0] + db[1] * db[1] + db[2] * db[2]);
  }
#pragma unroll
  for (int j = 0; j < 9; ++j) A[j] = wave_sum(A[j]);
  Dn = wave_sum(Dn);
  // rotation extraction: rotate q by the axis-angle vector sum_c r_c x a_c / (|sum_c r_c . a_c| + 1e-9)
  // (r_c, a_c columns of R(q) and A) until the angle falls below 1e-9, at most 20 times
  double qx = d.sec_q[4 * (size_t)k], qy = d.sec_q[4 * (size_t)k + 1], qz = d.sec_q[4 * (size_t)k + 2],
         qw = d.sec_q[4 * (size_t)k + 3];
  for (int it = 0; it < 20; ++it) {
    double Rm[9];
    qmat_d(qx, qy, qz, qw, Rm);
    double n0 = 0.0, n1 = 0.0, n2 = 0.0, den = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double r0 = Rm[c], r1 = Rm[3 + c], r2 = Rm[6 + c];
      const double a0 = A[c], a1 = A[3 + c], a2 = A[6 + c];
      n0 += r1 * a2 - r2 * a1;
      n1 += r2 * a0 - r0 * a2;
      n2 += r0 * a1 - r1 * a0;
      den += r0 * a0 + r1 * a1 + r2 * a2;
    }
    const double f = 1.0 / (fabs(den) + 1e-9);
    const double o0 = f * n0, o1 = f * n1, o2 = f * n2;
    const double w = sqrt(o0 * o0 + o1 * o1 + o2 * o2);
    if (w < 1e-9) break;
    const double sh = sin(0.5 * w) / w, ch = cos(0.5 * w);
    const double ax = sh * o0, ay = sh * o1, az = sh * o2;
    // (ax ay az ch) (x) q, normalised
    const double nx = ch * qx + ax * qw + ay * qz - az * qy;
    const double ny = ch * qy - ax * qz + ay * qw + az * qx;
    const double nz = ch * qz + ax * qy - ay * qx + az * qw;
    const double nw = ch * qw - ax * qx - ay * qy - az * qz;
    const double in = 1.0 / sqrt(nx * nx + ny * ny + nz * nz + nw * nw);
    qx = nx * in; qy = ny * in; qz = nz * in; qw = nw * in;
  }
  double Rs[9];
  qmat_d(qx, qy, qz, qw, Rs);
  double tr = 0.0;
#pragma unroll
  for (int j = 0; j < 9; ++j) tr += Rs[j] * A[j];
  const double sc = tr / Dn;
  if (lane != 0) return;
  double* F = d.sec_fit + (size_t)kSecFit * k;
#pragma unroll
  for (int j = 0; j < 9; ++j) F[j] = Rs[j];
  F[9] = sc;
#pragma unroll
  for (int r = 0; r < 3; ++r) F[10 + r] = m[r] - sc * (Rs[3 * r] * m[3] + Rs[3 * r + 1] * m[4] + Rs[3 * r + 2] * m[5]);
  F[16] = qx; F[17] = qy; F[18] = qz; F[19] = qw;
  d.sec_q[4 * (size_t)k] = qx; d.sec_q[4 * (size_t)k + 1] = qy;
  d.sec_q[4 * (size_t)k + 2] = qz; d.sec_q[4 * (size_t)k + 3] = qw;
}

template <class T>
__global__ void __launch_bounds__(256) bundle_apply_kernel(const Dev<T>* __restrict__ D, const Blk* __restrict__ tab) {
  const Blk blk = tab[blockIdx.x];
  const Dev<T>& d = D[blk.scene];
  const int i = blk.base + (int)threadIdx.x;
  if (i >= d.nsecp) return;
  const int p = d.sec_pill[i];
  const double* F = d.sec_fit + (size_t)kSecFit * d.sec_of[i];
  const double sc = F[9];
  if (d.winv[p] > T(0)) {                       // pins fix position only
    const double* xr = d.sec_xr + 3 * (size_t)i;
    const double* an = d.anchor + 3 * (size_t)d.rod_of[p];
    T* const out[3] = {d.px, d.py, d.pz};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double y = sc * (F[3 * r] * xr[0] + F[3 * r + 1] * xr[1] + F[3 * r + 2] * xr[2]) + F[10 + r];
      out[r][p] = (T)(y - an[r]);
    }
  }
  d.s[p] = (T)sc;
  if (d.flags[p] & F_EDGE) {
    // q* (x) qbar_p, normalised
    const double ax = F[16], ay = F[17], az = F[18], aw = F[19];
    const double bx = (double)d.qrx[p], by = (double)d.qry[p], bz = (double)d.qrz[p], bw = (double)d.qrw[p];
    const double nx = aw * bx + ax * bw + ay * bz - az * by;
    const double ny = aw * by - ax * bz + ay * bw + az * bx;
    const double nz = aw * bz + ax * by - ay * bx + az * bw;
    const double nw = aw * bw - ax * bx - ay * by - az * bz;
    const double in = 1.0 / sqrt(nx * nx + ny * ny + nz * nz + nw * nw);
    d.qx[p] = (T)(nx * in); d.qy[p] = (T)(ny * in); d.qz[p] = (T)(nz * in); d.qw[p] = (T)(nw * in);
  }
}

}  // namespace

template <class T> hipError_t launch_bundle(const BatchDev& b, hipStream_t st) {
  if (b.nblk[TB_SECT] == 0) return hipSuccess;
  hipLaunchKernelGGL(bundle_fit_kernel<T>, dim3(b.nblk[TB_SECT]), dim3(256), 0, st, (const Dev<T>*)b.dev,
                     b.tab[TB_SECT]);
  hipLaunchKernelGGL(bundle_apply_kernel<T>, dim3(b.nblk[TB_SECP]), dim3(256), 0, st, (const Dev<T>*)b.dev,
                     b.tab[TB_SECP]);
  return hipGetLastError();
}

template hipError_t launch_bundle<float>(const BatchDev&, hipStream_t);
template hipError_t launch_bundle<double>(const BatchDev&, hipStream_t);

}  // namespace viper
