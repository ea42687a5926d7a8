// Kinematic bones: the per-frame warm start of Sec. 8.2 for gfx950.
//
// At the start of a frame the caller hands in every bone's new transform.  Each pill carries
// two (bone, weight) influences; it is moved by the linear blend of its bones' motions since
// the last frame, which starts the solver near the pose the bones imply instead of where the
// muscle was left (the displacement is then refined by the substeps).  One thread per bone
// forms the relative transforms (the new transforms arrive in the launch arguments, 32 bones
// per launch), then one thread per pill applies them in FP64 world coordinates (anchor +
// local position) and writes the local position back.

#include "bones.h"

namespace viper {
namespace {

struct BoneChunk {
  double T[kBoneChunk * 12];   // new transforms of bones base .. base + n - 1
  int base, n;
};

__global__ void __launch_bounds__(64) bone_delta_kernel(const BoneChunk ch, double* __restrict__ prev,
                                                        double* __restrict__ delta) {
  const int j = (int)threadIdx.x;
  if (j >= ch.n) return;
  const int b = ch.base + j;
  const double* C = ch.T + 12 * j;
  double* Pv = prev + 12 * (size_t)b;
  double* D = delta + 12 * (size_t)b;
  double c[12], p[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) { c[i] = C[i]; p[i] = Pv[i]; }
  // inverse of the previous linear part by its adjugate
  const double a0 = p[0], a1 = p[1], a2 = p[2], a3 = p[4], a4 = p[5], a5 = p[6], a6 = p[8], a7 = p[9], a8 = p[10];
  const double m[9] = {a4 * a8 - a5 * a7, a2 * a7 - a1 * a8, a1 * a5 - a2 * a4,
                       a5 * a6 - a3 * a8, a0 * a8 - a2 * a6, a2 * a3 - a0 * a5,
                       a3 * a7 - a4 * a6, a1 * a6 - a0 * a7, a0 * a4 - a1 * a3};
  const double idet = 1.0 / (a0 * m[0] + a1 * m[3] + a2 * m[6]);
  double inv[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) inv[i] = m[i] * idet;
  // delta = [C_A inv | C_b - C_A inv p_b]
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double row[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) row[k] = c[4 * r] * inv[k] + c[4 * r + 1] * inv[3 + k] + c[4 * r + 2] * inv[6 + k];
    D[4 * r] = row[0]; D[4 * r + 1] = row[1]; D[4 * r + 2] = row[2];
    D[4 * r + 3] = c[4 * r + 3] - (row[0] * p[3] + row[1] * p[7] + row[2] * p[11]);
  }
#pragma unroll
  for (int i = 0; i < 12; ++i) Pv[i] = c[i];
}

template <class T>
__global__ void __launch_bounds__(256) bone_warm_kernel(const Dev<T> d, const int32_t* __restrict__ pb,
                                                        const double* __restrict__ pw, const double* __restrict__ delta) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= d.P) return;
  const double w[2] = {pw[2 * (size_t)p], pw[2 * (size_t)p + 1]};
  if (!(w[0] > 0.0) && !(w[1] > 0.0)) return;
  const double* an = d.anchor + 3 * (size_t)d.rod_of[p];
  const double x0 = an[0] + (double)d.px[p], x1 = an[1] + (double)d.py[p], x2 = an[2] + (double)d.pz[p];
  double y0 = 0.0, y1 = 0.0, y2 = 0.0, ws = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (!(w[k] > 0.0)) continue;
    const double* D = delta + 12 * (size_t)pb[2 * (size_t)p + k];
    y0 += w[k] * (D[0] * x0 + D[1] * x1 + D[2] * x2 + D[3]);
    y1 += w[k] * (D[4] * x0 + D[5] * x1 + D[6] * x2 + D[7]);
    y2 += w[k] * (D[8] * x0 + D[9] * x1 + D[10] * x2 + D[11]);
    ws += w[k];
  }
  const double iw = 1.0 / ws;
  d.px[p] = (T)(y0 * iw - an[0]);
  d.py[p] = (T)(y1 * iw - an[1]);
  d.pz[p] = (T)(y2 * iw - an[2]);
}

}  // namespace

template <class T>
hipError_t launch_bone_warm(const Dev<T>& d, int nb, const double* cur, double* prev, double* delta,
                            const int32_t* pb, const double* pw, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  for (int base = 0; base < nb; base += kBoneChunk) {
    BoneChunk ch;
    ch.base = base;
    ch.n = nb - base < kBoneChunk ? nb - base : kBoneChunk;
    for (int i = 0; i < 12 * ch.n; ++i) ch.T[i] = cur[12 * (size_t)base + i];
    hipLaunchKernelGGL(bone_delta_kernel, dim3(1), dim3(64), 0, st, ch, prev, delta);
  }
  if (d.P > 0)
    hipLaunchKernelGGL(bone_warm_kernel<T>, dim3((d.P + 255) / 256), dim3(256), 0, st, d, pb, pw, (const double*)delta);
  return hipGetLastError();
}

template hipError_t launch_bone_warm<float>(const Dev<float>&, int, const double*, double*, double*, const int32_t*,
                                            const double*, hipStream_t);
template hipError_t launch_bone_warm<double>(const Dev<double>&, int, const double*, double*, double*, const int32_t*,
                                             const double*, hipStream_t);

}  // namespace viper
