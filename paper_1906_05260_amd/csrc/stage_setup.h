// Start of a kernel that runs one wavefront of a scene per block, for gfx950.
#pragma once

#include "rod_device.h"

namespace viper {

// The per-stage kernels run one wavefront per block, so that a scene of a few hundred
// wavefronts spreads over every compute unit.  Such a launch is mostly the chain of dependent
// reads a wavefront waits for before its work, so its start is laid out for few round trips to
// memory: the caller copies the scene's fields into registers in one go (a copy of them sits in
// the wavefront's launch record, or behind the block's table entry) and names the scalars it
// reads later in an empty statement, so that they come with them; the start has no branch; the slot flags are read unconditionally (an empty
// slot reads its wave's first pill, which exists), and the per-pill reads that follow depend on
// the wave's range only.  This form takes the wave index of a 4-wavefront block table entry
// (block b: wavefront tab[b / 4].base + b % 4; a wavefront past the scene's last reads that
// wave's range and gets no valid slot).
template <class T>
__device__ __forceinline__ void stage_setup(const Dev<T>& d, int wave, Lane2<T>& P, int& pA, int& pB) {
  const bool live = wave < d.W;        // a dead wavefront (last block of a scene) gets no valid slot
  const int w = live ? wave : d.W - 1;
  const int lane = (int)(threadIdx.x & 63);
  const int p0 = d.wave_start[w];
  const int n = live ? d.wave_start[w + 1] - p0 : 0;
  const bool vA = 2 * lane < n, vB = 2 * lane + 1 < n;
  pA = p0 + (vA ? 2 * lane : 0);
  pB = p0 + (vB ? 2 * lane + 1 : 0);
  const uint32_t fA = d.flags[pA], fB = d.flags[pB];
  P.A.f = vA ? fA : 0u;
  P.B.f = vB ? fB : 0u;
  P.sb = __any(((P.A.f | P.B.f) & F_SB) != 0u) != 0;
  P.vb = __any(((P.A.f | P.B.f) & F_VB) != 0u) != 0;
}

// The same start from the wavefront's launch record (its pill range comes with it: no read of
// the scene's wave table before the per-pill reads).
template <class T>
__device__ __forceinline__ void stage_setup(const Dev<T>& d, const WaveBlk& wb, Lane2<T>& P, int& pA, int& pB) {
  const int lane = (int)(threadIdx.x & 63);
  const int p0 = wb.p0, n = wb.n;
  const bool vA = 2 * lane < n, vB = 2 * lane + 1 < n;
  pA = p0 + (vA ? 2 * lane : 0);
  pB = p0 + (vB ? 2 * lane + 1 : 0);
  const uint32_t fA = d.flags[pA], fB = d.flags[pB];
  P.A.f = vA ? fA : 0u;
  P.B.f = vB ? fB : 0u;
  P.sb = __any(((P.A.f | P.B.f) & F_SB) != 0u) != 0;
  P.vb = __any(((P.A.f | P.B.f) & F_VB) != 0u) != 0;
}

}  // namespace viper
