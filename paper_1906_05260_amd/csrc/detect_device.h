// Start of a contact detection (Sec. 7.1), shared by the launch that predicts a substep (it
// forms the detection record of its own pills) and by the detection kernels, for gfx950.
#pragma once

#include "viper_dev.h"

namespace viper {

// Neighbour search: 9 threads per capsule, one per (dz, dy) column of its neighbour cells.
constexpr int kSearchSub = 9;

// The radius histogram is added into kHistCopies copies (wavefront index mod kHistCopies),
// so that the adds of a scene's wavefronts into its few occupied bins spread over more
// addresses; its readers sum the copies.
constexpr int kHistCopies = 8;

// Neighbour search blocks: 28 capsules (252 threads of 256) each.
constexpr int kSearchCaps = 28;
__host__ __device__ __forceinline__ int search_blocks(int E) { return (E + kSearchCaps - 1) / kSearchCaps; }

// Chunk totals of the cell scan, in kCellTotalCopies copies (every capsule adds one to its
// bucket's chunk; the copies spread those adds over more addresses, since adds to one address
// from the whole chip queue behind each other; a chunk is the 1024 items of one scan block).
constexpr int kCellTotalCopies = 32;
__host__ __device__ __forceinline__ int cell_chunks(int T) { return (T + 1023) / 1024; }
__host__ __device__ __forceinline__ int chunk_total_words(int T) { return kCellTotalCopies * cell_chunks(T); }

// Histogram bin of a bounding radius R (finite, m): 4 bins per octave, bin 96 starts at 1 m,
// clamped to [0, kRadBins - 1]; bin b holds [2^((b-96)/4), 2^((b-95)/4)).
__device__ __forceinline__ int radius_bin(double R) {
  if (!(R > 0x1p-24)) return 0;
  const double f = floor(4.0 * log2(R)) + 96.0;
  return f < 0.0 ? 0 : (f > kRadBins - 1 ? kRadBins - 1 : (int)f);
}

// Bounding sphere of a capsule in FP64 from its end points' world positions w0, w1 and end
// radii ra, rb (s r): centre = midpoint, radius = half length + larger end radius.
__device__ __forceinline__ void capsule_sphere_of(const double* w0, const double* w1, double ra, double rb, double* out) {
#pragma clang fp contract(off)
  const double x0 = w0[0], y0 = w0[1], z0 = w0[2];
  const double x1 = w1[0], y1 = w1[1], z1 = w1[2];
  out[0] = 0.5 * (x0 + x1);
  out[1] = 0.5 * (y0 + y1);
  out[2] = 0.5 * (z0 + z1);
  const double dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
  const double len = __builtin_sqrt((dx * dx + dy * dy) + dz * dz);
  out[3] = 0.5 * len + ((ra < rb) ? rb : ra);
}

// The detection record of capsule i (sphere and radius bin) from its end points (world
// positions, scales in the scene's precision, rest radii); a sphere that is not finite raises
// the scene's non-finite status, and such a capsule or one with an end radius s r <= 0 (no
// surface while a scale passes through zero) gets no bin (kRadBins: left out of the
// detection).  Returns the bin.
template <class T>
__device__ __forceinline__ int capsule_record(const ContactDev& c, int i, const double* w0, const double* w1, T s0, T s1,
                                              T rb0, T rb1, double* sp) {
  capsule_sphere_of(w0, w1, (double)s0 * (double)rb0, (double)s1 * (double)rb1, sp);
  c.sph[4 * (size_t)i + 0] = sp[0];
  c.sph[4 * (size_t)i + 1] = sp[1];
  c.sph[4 * (size_t)i + 2] = sp[2];
  c.sph[4 * (size_t)i + 3] = sp[3];
  int bin = kRadBins;
  if (!(isfinite(sp[0]) && isfinite(sp[1]) && isfinite(sp[2]) && isfinite(sp[3]))) c.status[ST_NAN] = 1;
  else if (s0 > T(0) && s1 > T(0)) bin = radius_bin(sp[3]);
  c.key[i] = bin;
  return bin;
}

// The per-detection resets a scene's threads share (thread tid of nth): hash-bucket counts,
// cursors and group ranges, the cell scan's chunk totals, the walk record, the oversized count and
// the pair count.
__device__ __forceinline__ void detect_reset(const ContactDev& c, int tid, int nth) {
  for (int k = tid; k < c.T; k += nth) {
    c.cell_cnt[k] = 0;
    c.cell_cur[k] = 0;
    c.cgmin[k] = 0x7fffffff;
    c.cgmax[k] = -0x7fffffff - 1;
  }
  const int nw = chunk_total_words(c.T);
  for (int k = tid; k < nw; k += nth) c.bsum[k] = 0;
  for (int k = tid; k < kWalkCounters; k += nth) c.walk[k] = 0ull;
  if (tid == 0) {
    c.dcnt[0] = 0;
    c.npairs[0] = 0;
  }
}

}  // namespace viper
