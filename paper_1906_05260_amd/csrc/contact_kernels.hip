// Pill-pill contacts for gfx950.
//
// Detection (Sec. 7.1, after Green 2010): each capsule (tapered pill primitive)
// gets a bounding sphere; a uniform grid with cell width equal to the largest
// sphere diameter guarantees that overlapping spheres sit in neighbouring cells.
// The grid here has two levels and a list.  A histogram of the radii finds the bin that
// holds the (kOversized+1)-th largest; the at most kOversized larger capsules are kept in a
// short list that every capsule walks (one stretched capsule would otherwise widen every
// cell of its scene and make the walk quadratic).  The capsules up to that bin are split at
// a lower bin into a fine grid (cell diameter the largest fine radius) and a coarse grid of
// the larger ones (cell diameter the sum of the largest coarse and fine radii), where that
// split shortens the walk: a scene whose few percent of stretched capsules would otherwise
// set the cell width of all.  A capsule walks half of the 27 cells around its own in its
// level (the home cell for partners above it, the cells after it in (dz, dy, dx) order for
// every partner: each pair is found once), a fine capsule also the 2 x 2 x 2 coarse cells
// nearest its centre (the coarse capsules walk no fine cell), and the list.
// A capsule whose bounding sphere is not
// finite is left out and raises the scene's non-finite status; one with an end radius s r
// <= 0 (no surface) is left out too; a scene whose cell radius would exceed kRadLimit times
// its largest bounding radius at rest has diverged: its detection is skipped (no
// candidates) and its status says so.
// Cells are hashed into a table and filled by a counting sort; every capsule then
// counts its candidates in its cells, an exclusive scan turns the counts into offsets
// (in each search block, whose range of the list comes from one add), and the candidates
// are listed in parallel (the parallel count-then-list construction of Sec. 7.1).  The set of pairs is exact; their
// order inside a capsule's segment follows the order of the atomics and is not kept: the
// handling sums its corrections in fixed point, so its result does not depend on it, and the
// host sorts a list it hands out.  The overlap predicate runs in FP64 with no contraction, so it
// decides exactly as a serial FP64 evaluation of the same stored values.
//
// Handling (Sec. 7.2, App. D): per candidate pair, a 10-step dichotomous search of
// the largest inter-penetration over the first capsule's barycentric coordinate,
// with the closed-form projection onto the second capsule; a violated pair gets a
// hard (zero-compliance) correction of the four end positions and scales.  All
// pairs read the same state and the corrections are averaged per pill (the Jacobi
// reduction of Sec. 7).  The per-pill sums are accumulated with 64-bit integer atomics
// in fixed point (2^-44 m resolution): integer addition is associative, so the sum does
// not depend on the order in which pairs arrive and the result is deterministic.

#include "contact.h"
#include "detect_device.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>

namespace viper {

namespace {

// Neighbour search: kSearchSub = 9 threads per capsule, one per (dz, dy) column of its
// neighbour cells; 28 capsules (252 threads) per block.
constexpr int kStage = 8;       // candidates per (capsule, column) kept by the count pass
constexpr int kWalkItems = 3;   // bucket entries per lane whose loads are issued together
constexpr int kWaves = 4;       // wavefronts per search block
constexpr int kCapsPerWave = 7; // capsules per wavefront (7 x 9 columns = 63 lanes)
static_assert(kWaves * kCapsPerWave == kSearchCaps, "search block layout");

// Key of a grid cell: integer cell coordinates wrapped to 21 / 21 / 20 bits and the grid
// level (0 fine, 1 coarse) in bit 62, so every key is >= 0 (an oversized capsule's key is
// -1).  Two cells of one level share a key only if they are >= 2^20 cells apart, too far
// for any sphere of one to overlap a sphere of the other: the walk's key filter may admit
// such an entry, the exact overlap test then rejects it.  Neighbour keys are formed from
// the wrapped coordinates, so the wrap commutes with the +-1 steps.
constexpr long long kM21 = (1ll << 21) - 1, kM20 = (1ll << 20) - 1;
__device__ __forceinline__ long long pack_key(int x, int y, int z, int level) {
  return ((long long)x & kM21) | (((long long)y & kM21) << 21) | (((long long)z & kM20) << 42) |
         ((long long)level << 62);
}

// Hash-table bucket of a cell key: the two 32-bit halves multiplied by odd constants and
// combined, then the 32-bit finalizer of MurmurHash3 (Appleby), masked to the table size T
// (a power of two).  Neighbouring cells land in unrelated buckets, so an empty neighbour
// rarely meets an occupied bucket.
__device__ __forceinline__ uint32_t bucket_of(long long K, int T) {
  uint32_t h = (uint32_t)K * 0x8DA6B343u ^ (uint32_t)((unsigned long long)K >> 32) * 0xD8163841u;
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h & (uint32_t)(T - 1);
}

__device__ __forceinline__ int cell_of(double m, double cw) {
  double f = floor(m / cw);
  f = fmin(fmax(f, -1073741824.0), 1073741823.0);
  return (int)f;
}

// World position of pill p in FP64: anchor of its rod + stored local offset.
template <class T>
__device__ __forceinline__ void world_pos(const Dev<T>& d, int p, double* w) {
#pragma clang fp contract(off)
  const double* an = d.anchor + 3 * (size_t)d.rod_of[p];
  w[0] = an[0] + (double)d.px[p];
  w[1] = an[1] + (double)d.py[p];
  w[2] = an[2] + (double)d.pz[p];
}

__device__ bool spheres_overlap(const double* a, const double* b) {
#pragma clang fp contract(off)
  const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  const double d2 = (dx * dx + dy * dy) + dz * dz;
  const double rr = a[3] + b[3];
  return d2 < rr * rr;
}

// Fixed-point accumulation (2^-44 m per unit; a single term is clamped to +-2^12 m so
// that no sum of a pass can wrap): deterministic whatever the order of the atomics.
__device__ __forceinline__ void acc_add(unsigned long long* a, double v) {
  const double s = fmin(fmax(v * 0x1p44, -0x1p56), 0x1p56);
  atomicAdd(a, (unsigned long long)(long long)rint(s));
}

// ---- block-table helpers

#define BLOCK_SCENE(tab, D, CD)                 \
  const Blk blk_ = (tab)[blockIdx.x];           \
  const Dev<T>& d = (D)[blk_.scene];            \
  const ContactDev& c = (CD)[blk_.scene];       \
  (void)d; (void)c;

// ---- exclusive scan of the hash-cell counts (cell_start[T] = total), 1024 cells per block.
// The key kernel that produces the counts also adds them into per-chunk totals (a chunk is the
// 1024 cells of one scan block; the totals are cleared by the prediction launch), so the scan
// is one launch with no wait between blocks: block b scans its chunk and adds the totals of
// the chunks before it.
__global__ void __launch_bounds__(256) scan_kernel(const ContactDev* __restrict__ CD, const Blk* __restrict__ tab) {
  __shared__ int32_t s_sum[4], s_pre[4];
  const Blk b = tab[blockIdx.x];
  const ContactDev& c = CD[b.scene];
  const int32_t* in = c.cell_cnt;
  int32_t* out = c.cell_start;
  const int n = c.T;
  const int32_t* tot = c.bsum;
  const int t = (int)threadIdx.x, lane = t & 63, wv = t >> 6;
  int pre = 0;                          // totals of the chunks before this block's
  const int nch = cell_chunks(c.T), m = kCellTotalCopies * (b.base >> 10);
  for (int k = t; k < m; k += 256) pre += tot[(k % kCellTotalCopies) * nch + k / kCellTotalCopies];
  const int base = b.base + 4 * t;
  int v[4];
  int sv = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    sv += v[k];
  }
  int incl = sv;                        // wavefront inclusive scan of the thread sums
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int x = __shfl_up(incl, o);
    if (lane >= o) incl += x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o);
  if (lane == 63) s_sum[wv] = incl;
  if (lane == 0) s_pre[wv] = pre;
  __syncthreads();
  int run = s_pre[0] + s_pre[1] + s_pre[2] + s_pre[3] + incl - sv;
  for (int k = 0; k < wv; ++k) run += s_sum[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (base < n && n <= base + 4) out[n] = run;   // the thread holding the last item: the total
}

// ---- detection

// Cell width for cell radius rc (> every grid capsule's bounding radius; a zero radius, an
// empty scene, gets a unit cell).
__device__ __forceinline__ double cell_width_of(double rc) { return rc > 0.0 ? 2.0 * rc * (1.0 + 1e-6) : 1.0; }

// Grid levels from the histogram, by the first wavefront (64 lanes, two bins each).
// The cell bin cb holds the (kOversized+1)-th largest radius: the highest bin whose suffix
// count (capsules in bins >= it) exceeds kOversized, or bin 0; bins above it hold at most
// kOversized capsules, searched from a list.  The fine bin bf <= cb splits the rest: bins up
// to bf form the fine grid (cell radius rf = the largest radius of bin bf), bins in (bf, cb]
// a coarse grid of cell radius rc + rf (rc = the largest radius of bin cb), so that a fine
// capsule finds every coarse partner in the 2 x 2 x 2 coarse cells nearest its centre.  bf
// is the non-empty bin that minimises the entries walked for capsules spread uniformly:
// E_f fine capsules walk half of 27 fine cells holding E_f capsules and 8 coarse cells
// holding E_c, the coarse ones half of 27 coarse cells (cell volumes (2 rf)^3 and
// (2 (rc + rf))^3); bf = cb, one level, when that is cheapest or no bin qualifies.
struct GridLevels {
  int cb, bf, ncoarse;
  double rc, rf;
};
__device__ GridLevels grid_levels_wave(const int32_t* h, const unsigned long long* bm, int lane) {
  static_assert(kRadBins == 128, "two bins per lane");
  int h0 = 0, h1 = 0;                   // the histogram's copies summed
  unsigned long long b0 = 0ull, b1 = 0ull;
#pragma unroll
  for (int k = 0; k < kHistCopies; ++k) {
    h0 += h[k * (kRadBins + 1) + 2 * lane];
    h1 += h[k * (kRadBins + 1) + 2 * lane + 1];
    b0 = max(b0, bm[k * kRadBins + 2 * lane]);
    b1 = max(b1, bm[k * kRadBins + 2 * lane + 1]);
  }
  const double m0 = __longlong_as_double((long long)b0), m1 = __longlong_as_double((long long)b1);
  int t = h0 + h1;                      // suffix sum over lanes >= this one
  int p = h0 + h1;                      // prefix sum over lanes <= this one
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_down(t, o);
    if (lane + o < 64) t += u;
    const int v = __shfl_up(p, o);
    if (lane >= o) p += v;
  }
  const int s0 = t, s1 = t - h0;        // capsules in bins >= 2 lane, >= 2 lane + 1
  const int n = __popcll(__ballot(s0 > kOversized)) + __popcll(__ballot(s1 > kOversized));
  GridLevels g;
  g.cb = n > 0 ? n - 1 : 0;
  const int p1 = p, p0 = p - h1;        // capsules in bins <= 2 lane, <= 2 lane + 1
  const int pc = __shfl((g.cb & 1) ? p1 : p0, g.cb >> 1);
  const double rc = __shfl((g.cb & 1) ? m1 : m0, g.cb >> 1);
  double best = INFINITY;
  int bb = g.cb;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int bin = 2 * lane + k, cnt = k ? h1 : h0;
    if (bin > g.cb || cnt == 0) continue;
    const double ef = (double)(k ? p1 : p0), ec = (double)pc - ef;
    const double rf = k ? m1 : m0;
    const double vf = 8.0 * rf * rf * rf, vc = 8.0 * (rc + rf) * (rc + rf) * (rc + rf);
    const double cost = 27.0 * ef * ef * vf + (16.0 * ef * ec + 27.0 * ec * ec) * vc;
    if (cost <= best) { best = cost; bb = bin; }   // ties: the higher bin
  }
  // wave argmin (ties: the higher bin)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o);
    const int obb = __shfl_xor(bb, o);
    if (ob < best || (ob == best && obb > bb)) { best = ob; bb = obb; }
  }
  g.bf = bb;
  g.ncoarse = pc - __shfl((bb & 1) ? p1 : p0, bb >> 1);
  g.rc = rc;
  g.rf = __shfl((bb & 1) ? m1 : m0, bb >> 1);
  return g;
}

// The cell-key and bucket-scatter kernels take kCapsBlock capsules per block (one thread each).
constexpr int kCapsBlock = 256;
// A block's distinct hash buckets, so that the block adds into each bucket once (capsules of
// consecutive indices share cells: one muscle's neighbouring rods): open addressing over
// kBlockSlots slots (at most kCapsBlock keys, so every probe sequence ends), cleared by the caller.
constexpr int kBlockSlots = 2 * kCapsBlock;
__device__ __forceinline__ int block_slot(int* keys, int h) {
  int s = h & (kBlockSlots - 1);
  for (int n = 0; n < kBlockSlots; ++n) {
    const int prev = atomicCAS(&keys[s], -1, h);
    if (prev == -1 || prev == h) return s;
    s = (s + 1) & (kBlockSlots - 1);
  }
  return -1;   // not reached: fewer keys than slots
}

// Cell keys: a capsule in a bin up to the fine bin goes to its fine-grid cell, one up to the
// cell bin to its coarse-grid cell, a larger one to the oversized list, a non-finite one (or
// every capsule of a skipped scene) nowhere.
__global__ void __launch_bounds__(kCapsBlock) key_kernel(const ContactDev* __restrict__ CD, const Blk* __restrict__ tab) {
  __shared__ int s_cb, s_bf;
  __shared__ double s_rc, s_rf;
  __shared__ int s_key[kBlockSlots], s_cnt[kBlockSlots], s_gmin[kBlockSlots], s_gmax[kBlockSlots];
  const Blk b = tab[blockIdx.x];
  const ContactDev& c = CD[b.scene];
  for (int k = (int)threadIdx.x; k < kBlockSlots; k += kCapsBlock) {
    s_key[k] = -1;
    s_cnt[k] = 0;
    s_gmin[k] = 0x7fffffff;
    s_gmax[k] = -0x7fffffff - 1;
  }
  // the capsule's bin and sphere are read before the block waits for its grid levels
  const int i = b.base + (int)threadIdx.x;
  const bool mine = i < c.E;
  const int bin = mine ? c.key[i] : kRadBins;
  const int grp = mine ? c.cap_grp[i] : 0;
  double m[3] = {0.0, 0.0, 0.0};
  if (mine) {
#pragma unroll
    for (int k = 0; k < 3; ++k) m[k] = c.sph[4 * (size_t)i + k];
  }
  if (threadIdx.x < 64) {
    const int lane = (int)threadIdx.x;
    const GridLevels g = grid_levels_wave(c.hist, c.binmax, lane);
    if (lane == 0) {
      const double rc = g.rc, rf = g.rf;
      s_cb = g.cb;
      s_bf = g.bf;
      s_rc = rc;
      s_rf = rf;
      if (b.base == 0) {               // the detection's record, read back by viper_contact_stats
        const bool skip = !(rc <= c.rlim);
        const bool two = !skip && g.bf < g.cb;
        c.dcnt[1] = skip;
        int excl = 0;
#pragma unroll
        for (int k = 0; k < kHistCopies; ++k) excl += c.hist[k * (kRadBins + 1) + kRadBins];
        c.dcnt[2] = excl;
        c.dcnt[3] = g.bf;
        c.dcnt[4] = two ? g.cb : -1;
        c.dcnt[5] = two ? g.ncoarse : 0;
        c.cw[0] = skip ? 0.0 : cell_width_of(rf);
        c.cw[1] = two ? cell_width_of(rc + rf) : 0.0;
        if (skip) c.status[ST_DIVERGED] = 1;
      }
    }
  }
  __syncthreads();
  const int cb = s_cb, bf = s_bf;
  const double rc = s_rc, rf = s_rf;
  if (mine) {
    if (!(rc <= c.rlim) || bin == kRadBins) {
      c.key[i] = -1;
    } else if (bin > cb) {             // oversized: position in the list after the grid's entries
      c.key[i] = -2 - atomicAdd(&c.dcnt[0], 1);
    } else {
      const int level = bin > bf;
      const double cw = level ? cell_width_of(rc + rf) : cell_width_of(rf);
      const long long K = pack_key(cell_of(m[0], cw), cell_of(m[1], cw), cell_of(m[2], cw), level);
      c.pkey[i] = K;
      const int h = (int)bucket_of(K, c.T);
      c.key[i] = h;
      const int sl = block_slot(s_key, h);
      atomicAdd(&s_cnt[sl], 1);
      atomicMin(&s_gmin[sl], grp);
      atomicMax(&s_gmax[sl], grp);
    }
  }
  __syncthreads();
  // one add per distinct bucket of the block: its count, its group range, and the cell scan's
  // chunk total (in the copy of this block)
  for (int k = (int)threadIdx.x; k < kBlockSlots; k += kCapsBlock) {
    const int h = s_key[k];
    if (h < 0) continue;
    atomicAdd(&c.cell_cnt[h], s_cnt[k]);
    atomicAdd(&c.bsum[(blockIdx.x % kCellTotalCopies) * cell_chunks(c.T) + (h >> 10)], s_cnt[k]);
    atomicMin(&c.cgmin[h], s_gmin[k]);
    atomicMax(&c.cgmax[h], s_gmax[k]);
  }
}

__global__ void __launch_bounds__(kCapsBlock) bucket_scatter_kernel(const ContactDev* __restrict__ CD, const Blk* __restrict__ tab) {
  __shared__ int s_key[kBlockSlots], s_cnt[kBlockSlots], s_base[kBlockSlots];
  const Blk b = tab[blockIdx.x];
  const ContactDev& c = CD[b.scene];
  for (int k = (int)threadIdx.x; k < kBlockSlots; k += kCapsBlock) {
    s_key[k] = -1;
    s_cnt[k] = 0;
  }
  const int i = b.base + (int)threadIdx.x;
  const bool mine = i < c.E;
  const int h = mine ? c.key[i] : -1;
  // the capsule's search data (sphere, cell key, rod, group) is read while its slot is taken
  double sp[4] = {0.0, 0.0, 0.0, 0.0};
  long long K = -1;
  int rod = 0, grp = 0, id = 0;
  if (mine) {
#pragma unroll
    for (int k = 0; k < 4; ++k) sp[k] = c.sph[4 * (size_t)i + k];
    K = c.pkey[i];
    rod = c.cap_rod[i];
    grp = c.cap_grp[i];
    id = c.cap_ids[i];
  }
  __syncthreads();
  // grid capsules go to their bucket: the block takes one range of each of its buckets (one
  // global add per distinct bucket) and its capsules are ranked inside it
  int sl = -1, rank = 0;
  if (h >= 0) {
    sl = block_slot(s_key, h);
    rank = atomicAdd(&s_cnt[sl], 1);
  }
  __syncthreads();
  for (int k = (int)threadIdx.x; k < kBlockSlots; k += kCapsBlock)
    if (s_key[k] >= 0) s_base[k] = c.cell_start[s_key[k]] + atomicAdd(&c.cell_cur[s_key[k]], s_cnt[k]);
  __syncthreads();
  if (h == -1) return;                 // not placed in this detection (or past the scene's capsules)
  // oversized capsules go after every bucket (cell_start[T] is the number of grid capsules)
  const int pos = h >= 0 ? s_base[sl] + rank : c.cell_start[c.T] + (-2 - h);
  c.sorted[pos] = id;
#pragma unroll
  for (int k = 0; k < 4; ++k) c.ssph[4 * (size_t)pos + k] = sp[k];
  c.skey[pos] = h >= 0 ? K : -1ll;
  c.srg[2 * (size_t)pos] = rod;
  c.srg[2 * (size_t)pos + 1] = grp;
}

// Find and list the candidates of capsule a's walk (see the slots below).  Threads follow
// bucket order, so the lanes of a wave mostly share a home cell and walk the same neighbour
// entries (their loads coalesce); each of a capsule's 9 threads covers one (dz, dy) column.
// The first walk counts every column's candidates and keeps its first kStage in the thread's
// staging slot; the block then takes the range of its candidates in the scene's list with one
// add to the scene's pair count (every thread's offset follows from an exclusive scan of the
// block's counts), copies the staged candidates and walks again the columns that had more,
// listing them.  A bucket whose entries all share the capsule's collision group (the interior
// of a muscle) is skipped unread.  Bucket entries carry capsule ids (the first pill of a
// capsule, which grows with the capsule index, so comparisons of ids order capsules as their
// indices do); a pair is stored as (lower, higher) capsule id.  The blocks' ranges follow the
// order of their adds, which is not kept (see the handling below).
__global__ void __launch_bounds__(256) pair_kernel(const ContactDev* __restrict__ CD, const Blk* __restrict__ tab) {
  const Blk blk = tab[blockIdx.x];
  const ContactDev& c = CD[blk.scene];
  const int lb = blk.base / kSearchCaps;                  // the block's index in its scene
  const int slot = 256 * lb + (int)threadIdx.x;           // the thread's staging slot
  if (blk.base == 0) {
    // the radius histogram has had its last reader
    for (int k = (int)threadIdx.x; k < kHistCopies * (kRadBins + 1); k += 256) {
      c.hist[k] = 0;
      if (k < kHistCopies * kRadBins) c.binmax[k] = 0ull;
    }
  }
  // Each wavefront holds 7 whole capsules x 9 columns (lane 63 idles): a capsule's columns
  // and the balanced walk below stay inside one wavefront.  Wavefront w of the scene takes
  // bucket positions w, w + n, ..., w + 6n (n = the scene's wavefronts): capsules of one
  // crowded cell, adjacent in bucket order, land in different wavefronts.
  const int wv = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int sub = lane % kSearchSub;
  const int nwave = kWaves * search_blocks(c.E);
  const int jh = blk.base / kCapsPerWave + wv + nwave * (lane / kSearchSub);   // home capsule's bucket position
  // the home capsule's bucket entry is read before the number of placed capsules is known
  // (the position clamped into the scene: an unplaced position reads a stale entry, unused)
  const int jc = min(jh, c.E - 1);
  const int a0 = c.sorted[jc];
  const long long K0 = c.skey[jc];
  const double2 sa01 = ((const double2*)c.ssph)[2 * (size_t)jc], sa23 = ((const double2*)c.ssph)[2 * (size_t)jc + 1];
  const int2 rg0 = ((const int2*)c.srg)[jc];
  const int ngrid = c.cell_start[c.T];                 // grid capsules; the oversized list follows
  const int nplaced = ngrid + c.dcnt[0];
  asm volatile("" ::"v"(a0), "v"(K0), "v"(sa01.x), "v"(sa01.y), "v"(sa23.x), "v"(sa23.y), "v"(rg0.x), "v"(rg0.y));
  const bool live = lane < kCapsPerWave * kSearchSub && jh < nplaced;
  const int a = live ? a0 : 0;
  // A lane lists up to 4 slots (a run of bucket entries, the key they must carry, whether
  // b > a is required) ...
  //  - slots 0..2, the cells dx = -1, 0, +1 of its (dz, dy) column in its capsule's own
  //    level, half shell: a cell after the home cell in (dz, dy, dx) order gives every
  //    partner, the home cell those above a, a cell before it none (the partner's own walk
  //    finds that pair), so the columns with dz < 0 or (dz = 0, dy < 0) list no cell and
  //    the centre column its home cell and dx = +1;
  //  - slot 3 of a fine capsule's lanes 0..7: one of the 2 x 2 x 2 coarse cells nearest its
  //    centre, every partner (a coarse capsule walks no fine cell);
  //  - slot 3 of lane 8: the oversized list, every entry for a grid capsule, those above a
  //    for an oversized capsule (which walks nothing else).
  // A bucket whose entries all share the capsule's group is left out.
  __shared__ int s_off[kWaves][65];
  __shared__ int s_cnt[kWaves][64];
  __shared__ int s_col[kWaves][64][12];   // js0..js3, cum1 cum2 cum3, b > a mask, a ra ga, out
  __shared__ long long s_key[kWaves][64][2];   // key of the column's dx = -1 cell, key of slot 3
  __shared__ double s_sph[kWaves][64][4];
  __shared__ int s_tot[kWaves], s_base;
  int w = 0;
  {
    int js[4] = {0, 0, 0, 0}, ln[4] = {0, 0, 0, 0}, ra = 0, ga = 0, gt = 0;
    long long k0 = -1, k3 = -1;
    const bool over = jh >= ngrid;
    double sa[4] = {0.0, 0.0, 0.0, 0.0};
    if (live) {
      const long long K = K0;
      sa[0] = sa01.x; sa[1] = sa01.y; sa[2] = sa23.x; sa[3] = sa23.y;
      ra = rg0.x; ga = rg0.y;
      if (!over) {
        const int level = (int)(K >> 62);
        const int x = (int)(K & kM21), y = (int)((K >> 21) & kM21), z = (int)((K >> 42) & kM20);
        k0 = pack_key(x - 1, y + sub % 3 - 1, z + sub / 3 - 1, level);
        const int dfirst = sub < kSearchSub / 2 ? 3 : (sub == kSearchSub / 2 ? 1 : 0);
        if (sub == kSearchSub / 2) gt = 1 << 1;
        const double cwc = c.cw[1];
        bool coarse = false;
        if (level == 0 && sub < 8 && cwc > 0.0) {
          // coarse cell (bits of sub: step towards the nearer neighbour along x, y, z)
          int kc[3];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const double q = sa[j] / cwc;
            const double f = floor(q);
            const int side = (q - f < 0.5) ? -1 : 1;
            kc[j] = (int)fmin(fmax(f, -1073741824.0), 1073741823.0) + (((sub >> j) & 1) ? side : 0);
          }
          k3 = pack_key(kc[0], kc[1], kc[2], 1);
          coarse = true;
        }
        uint32_t hc[4];
        int gmn[4], gmx[4], je[4];
#pragma unroll
        for (int d = 0; d < 3; ++d) hc[d] = bucket_of((k0 & ~kM21) | ((k0 + d) & kM21), c.T);
        hc[3] = coarse ? bucket_of(k3, c.T) : 0u;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          if (d < 3 ? d < dfirst : !coarse) continue;
          gmn[d] = c.cgmin[hc[d]]; gmx[d] = c.cgmax[hc[d]];
          js[d] = c.cell_start[hc[d]]; je[d] = c.cell_start[hc[d] + 1];
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          if (d < 3 ? d < dfirst : !coarse) continue;
          ln[d] = (gmn[d] == ga && gmx[d] == ga) ? 0 : je[d] - js[d];
        }
      } else if (sub == kSearchSub - 1) {
        gt = 1 << 3;
      }
      if (sub == kSearchSub - 1) { js[3] = ngrid; ln[3] = nplaced - ngrid; k3 = -1; }
    }
    w = ln[0] + ln[1] + ln[2] + ln[3];
    int* sc = s_col[wv][lane];
    sc[0] = js[0]; sc[1] = js[1]; sc[2] = js[2]; sc[3] = js[3];
    sc[4] = ln[0]; sc[5] = ln[0] + ln[1]; sc[6] = ln[0] + ln[1] + ln[2];
    sc[7] = gt; sc[8] = a; sc[9] = ra; sc[10] = ga;
    sc[11] = slot;
    s_key[wv][lane][0] = k0;
    s_key[wv][lane][1] = k3;
#pragma unroll
    for (int k = 0; k < 4; ++k) s_sph[wv][lane][k] = sa[k];
    s_cnt[wv][lane] = 0;
  }
  // ... and the wavefront walks the concatenation of its lanes' lists (w entries on this lane)
  // 64 entries at a time (a lane finds the column of its entry by binary search over the
  // exclusive prefix sums), so that lanes stay busy however unevenly the entries fall on
  // columns.  A found candidate is counted in its column; the first walk stages it (up to
  // kStage per column), the second lists it at its column's offset (s_col out).
  auto walk = [&](auto listing) {
    constexpr bool kList = decltype(listing)::value;
    int incl = w;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    s_off[wv][lane] = incl - w;
    if (lane == 63) s_off[wv][64] = incl;
    __syncthreads();
    const int W = s_off[wv][64];
    // walk length for the detection record: one add per block, spread over kWalkCounters
    // addresses so that the adds of a scene's blocks do not queue on one
    if (!kList && threadIdx.x == 0) {
      unsigned long long wb = 0;
#pragma unroll
      for (int k = 0; k < kWaves; ++k) wb += (unsigned long long)s_off[k][64];
      if (wb) atomicAdd(c.walk + (blockIdx.x & (kWalkCounters - 1)), wb);
    }
    for (int g0 = 0; g0 < W; g0 += 64 * kWalkItems) {
      int own[kWalkItems], jj[kWalkItems], dd[kWalkItems], bb[kWalkItems], rr[kWalkItems], gg[kWalkItems];
      long long kk[kWalkItems];
      double2 s01[kWalkItems], s23[kWalkItems];
#pragma unroll
      for (int u = 0; u < kWalkItems; ++u) {
        const int g = g0 + 64 * u + lane;
        int lo = 0, hi = 64;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_off[wv][mid] <= g) lo = mid; else hi = mid;
        }
        const int* sc = s_col[wv][lo];
        const int k = g - s_off[wv][lo];
        own[u] = g < W ? lo : -1;
        dd[u] = k < sc[4] ? 0 : (k < sc[5] ? 1 : (k < sc[6] ? 2 : 3));
        jj[u] = sc[dd[u]] + k - (dd[u] == 0 ? 0 : sc[3 + dd[u]]);
        if (g >= W) jj[u] = 0;          // past the end: a harmless in-bounds read, masked below
      }
#pragma unroll
      for (int u = 0; u < kWalkItems; ++u) {
        const size_t j = (size_t)jj[u];
        bb[u] = c.sorted[j];
        kk[u] = c.skey[j];
        const int2 rg = ((const int2*)c.srg)[j];
        rr[u] = rg.x; gg[u] = rg.y;
        s01[u] = ((const double2*)c.ssph)[2 * j];
        s23[u] = ((const double2*)c.ssph)[2 * j + 1];
      }
#pragma unroll
      for (int u = 0; u < kWalkItems; ++u) {
        const int o = own[u];
        if (o < 0) continue;
        const int* sc = s_col[wv][o];
        const int b = bb[u];
        const int d = dd[u];
        const long long k0 = s_key[wv][o][0];
        const long long want = d < 3 ? ((k0 & ~kM21) | ((k0 + d) & kM21)) : s_key[wv][o][1];
        if (kk[u] != want) continue;                         // another cell or level (hash collision)
        if (((sc[7] >> d) & 1) && b <= sc[8]) continue;      // the home cell / an oversized capsule's list
        if (rr[u] == sc[9] || gg[u] == sc[10]) continue;
        const double sb[4] = {s01[u].x, s01[u].y, s23[u].x, s23[u].y};
        if (!spheres_overlap(s_sph[wv][o], sb)) continue;
        const int pos = atomicAdd(&s_cnt[wv][o], 1);
        if (kList) {
          const int idx = sc[11] + pos;
          if (idx < c.cap) ((int2*)c.pairs)[idx] = make_int2(min(sc[8], b), max(sc[8], b));
        } else if (pos < kStage) {
          c.stage[(size_t)kStage * sc[11] + pos] = b;
        }
      }
    }
  };
  walk(std::false_type{});
  // the block's range: its columns' counts scanned in thread order, one add for the block
  __syncthreads();                        // every count is final and every staged entry written
  const int cnt = s_cnt[wv][lane];
  const int w1 = s_off[wv][lane + 1] - s_off[wv][lane];   // the lane's entries (kept in LDS over the walk)
  const int ida = s_col[wv][lane][8];
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) s_tot[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int total = s_tot[0] + s_tot[1] + s_tot[2] + s_tot[3];
    const int base = total > 0 ? atomicAdd(c.npairs, total) : 0;
    if (total > c.cap - base) c.status[ST_OVERFLOW] = 1;   // the list keeps its first cap pairs
    s_base = base;
  }
  __syncthreads();
  int out = s_base + incl - cnt;
  for (int k = 0; k < wv; ++k) out += s_tot[k];
  if (cnt <= kStage) {
    // the first walk kept every candidate of this column: copy them
    const int32_t* stg = c.stage + (size_t)kStage * (256 * lb + (int)threadIdx.x);
    for (int k = 0; k < cnt; ++k)
      if (out + k < c.cap) ((int2*)c.pairs)[out + k] = make_int2(min(ida, stg[k]), max(ida, stg[k]));
  }
  // the columns with more are walked again, listing
  w = cnt > kStage ? w1 : 0;
  s_cnt[wv][lane] = 0;
  s_col[wv][lane][11] = out;
  walk(std::true_type{});
}

// ---- handling (FP64 arithmetic)

struct D3 { double x, y, z; };
__device__ __forceinline__ D3 d3(double x, double y, double z) { D3 r; r.x = x; r.y = y; r.z = z; return r; }
__device__ __forceinline__ D3 sub(D3 a, D3 b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ double dotp(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 lerp(D3 a, D3 b, double t) { return d3(a.x + t * (b.x - a.x), a.y + t * (b.y - a.y), a.z + t * (b.z - a.z)); }

// Barycentric coordinate on capsule (c1,r1)-(c2,r2) of the sphere nearest (in surface
// distance) to point x: stationary point of |x - c(t)| - r(t) along the axis, clamped
// (App. D with its sign and square corrected; a capsule whose radii differ by more than
// its length is its larger end sphere).
__device__ double pill_param(D3 x, D3 c1, double r1, D3 c2, double r2) {
  const D3 ax = sub(c2, c1);
  const double l = sqrt(dotp(ax, ax));
  if (!(l > 0.0)) return 0.0;
  const double sn = (r1 - r2) / l;
  if (sn >= 1.0) return 0.0;
  if (sn <= -1.0) return 1.0;
  const D3 e = d3(ax.x / l, ax.y / l, ax.z / l);
  const D3 rel = sub(x, c1);
  const double u = dotp(rel, e);
  const D3 perp = d3(rel.x - u * e.x, rel.y - u * e.y, rel.z - u * e.z);
  const double dp = sqrt(dotp(perp, perp));
  const double t = (u - dp * sn / sqrt(1.0 - sn * sn)) / l;
  return fmin(fmax(t, 0.0), 1.0);
}

// The terms of pill_param that depend on the capsule only (its start and unit axis, 1 / its
// length and the slope sn / sqrt(1 - sn^2) of the nearest-sphere line), formed once for the
// many points of a search; `fixed` >= 0 is the parameter of every point (a capsule without
// length, or one that is its larger end sphere).
struct PillAxis {
  D3 c1, e;
  double il, cot, fixed;
};
__device__ PillAxis pill_axis(D3 c1, double r1, D3 c2, double r2) {
  PillAxis A;
  A.c1 = c1;
  A.e = d3(0.0, 0.0, 0.0);
  A.il = 0.0;
  A.cot = 0.0;
  A.fixed = 0.0;
  const D3 ax = sub(c2, c1);
  const double l = sqrt(dotp(ax, ax));
  if (!(l > 0.0)) return A;
  const double sn = (r1 - r2) / l;
  if (sn >= 1.0) return A;
  if (sn <= -1.0) {
    A.fixed = 1.0;
    return A;
  }
  A.e = d3(ax.x / l, ax.y / l, ax.z / l);
  A.il = 1.0 / l;
  A.cot = sn / sqrt(1.0 - sn * sn);
  A.fixed = -1.0;
  return A;
}

// pill_param of point x on a capsule given by its axis terms.
__device__ __forceinline__ double pill_param_at(const PillAxis& A, D3 x) {
  const D3 rel = sub(x, A.c1);
  const double u = dotp(rel, A.e);
  const D3 perp = d3(rel.x - u * A.e.x, rel.y - u * A.e.y, rel.z - u * A.e.z);
  const double dp = sqrt(dotp(perp, perp));
  const double t = (u - dp * A.cot) * A.il;
  return A.fixed >= 0.0 ? A.fixed : fmin(fmax(t, 0.0), 1.0);
}

// Signed surface gap between the first capsule's sphere at parameter al and its nearest
// sphere on the second capsule (axis terms B).
__device__ __forceinline__ double gap_at(const D3* c, const double* r, const PillAxis& B, double al) {
  const D3 ca = lerp(c[0], c[1], al);
  const double ra = r[0] + al * (r[1] - r[0]);
  const double be = pill_param_at(B, ca);
  const D3 cb = lerp(c[2], c[3], be);
  const D3 dv = sub(ca, cb);
  return sqrt(dotp(dv, dv)) - ra - (r[2] + be * (r[3] - r[2]));
}

// Exchange of a double between the two lanes of a lane pair (2k, 2k + 1).
__device__ __forceinline__ double pair_swap(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// One candidate pair per lane pair: the two gap evaluations of each step of the dichotomous
// search run on the two lanes (the lower at m - delta, the upper at m + delta) and are
// exchanged, so both lanes take the same decision; both then form the projection, and the
// lower lane accumulates the corrections of the first capsule's pills, the upper lane those
// of the second's.  A scene's blocks cover pair_span(cap) pairs per round.
template <class T>
__global__ void __launch_bounds__(64) contact_pair_kernel(const Dev<T>* __restrict__ D, const ContactDev* __restrict__ CD,
                                                           const Blk* __restrict__ tab) {
  BLOCK_SCENE(tab, D, CD)
  const int lane2 = blk_.base + (int)threadIdx.x;
  const bool upper = (lane2 & 1) != 0;
  const int span = pair_span(c.cap);
  // the first pair is read before the count is known (clamped into the list: the last
  // block's padding lanes read the last slot), everything per pill right after it
  int i = lane2 >> 1;
  // the scene's pointers and scalars are requested together (an empty statement that takes
  // them as operands), not in round trips of their own after the count
  asm volatile("" ::"s"(d.px), "s"(d.py), "s"(d.pz), "s"(d.s), "s"(d.rbar), "s"(d.winv), "s"(d.wsinv), "s"(d.rod_of),
               "s"(d.anchor), "s"(c.acc), "s"(c.acnt), "s"(c.search_iters), "s"(c.delta), "s"(c.pairs), "s"(c.npairs));
  int2 ab = ((const int2*)c.pairs)[min(i, c.cap - 1)];
  const int np = min(c.npairs[0], c.cap);
  asm volatile("" ::"v"(ab.x), "v"(ab.y));
  while (i < np) {   // the same trip count on both lanes of a pair
    const int pid[4] = {ab.x, ab.x + 1, ab.y, ab.y + 1};
    D3 cp[4];
    double r[4], rb[4], w[4], ws[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int p = pid[t];
      double x[3];
      world_pos(d, p, x);
      cp[t] = d3(x[0], x[1], x[2]);
      rb[t] = (double)d.rbar[p];
      r[t] = (double)d.s[p] * rb[t];
      w[t] = (double)d.winv[p];
      ws[t] = (double)d.wsinv[p];
    }
    // dichotomous search over the first capsule's parameter (fixed iteration count)
    const PillAxis B = pill_axis(cp[2], r[2], cp[3], r[3]);
    double lo = 0.0, hi = 1.0;
    for (int k = 0; k < c.search_iters; ++k) {
      const double m = 0.5 * (lo + hi);
      const double x1 = m - c.delta, x2 = m + c.delta;
      const double g = gap_at(cp, r, B, upper ? x2 : x1);
      const double go = pair_swap(g);
      const double g1 = upper ? go : g, g2 = upper ? g : go;
      if (g1 < g2) hi = x2; else lo = x1;
    }
    const double al = 0.5 * (lo + hi);
    const D3 ca = lerp(cp[0], cp[1], al);
    const double be = pill_param_at(B, ca);
    const D3 cb = lerp(cp[2], cp[3], be);
    const D3 dv = sub(ca, cb);
    const double dist = sqrt(dotp(dv, dv));
    const double C = dist - (r[0] + al * (r[1] - r[0])) - (r[2] + be * (r[3] - r[2]));
    if (C < 0.0 && dist > 0.0) {
      const D3 n = d3(dv.x / dist, dv.y / dist, dv.z / dist);
      const double wt[4] = {1.0 - al, al, -(1.0 - be), -be};   // dC/dx_t = wt n, dC/ds_t = -|wt| rbar
      double den = 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double gs = fabs(wt[t]) * rb[t];
        den += w[t] * wt[t] * wt[t] + ws[t] * gs * gs;
      }
      if (den > 0.0) {
        const double dl = -C / den;
        const int t0 = upper ? 2 : 0;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int t = t0 + u;
          const double k = w[t] * wt[t] * dl;
          unsigned long long* o = c.acc + 4 * (size_t)pid[t];
          acc_add(o + 0, k * n.x);
          acc_add(o + 1, k * n.y);
          acc_add(o + 2, k * n.z);
          acc_add(o + 3, -ws[t] * fabs(wt[t]) * rb[t] * dl);
          atomicAdd(&c.acnt[pid[t]], 1);
        }
      }
    }
    i += span;
    if (i < np) ab = ((const int2*)c.pairs)[i];
  }
}

// Initial skinning weights (Sec. 7.4): a vertex's weight for each capsule is proportional to
// the inverse square distance from the vertex to the capsule's surface, |v - c(t)| - r(t) at the
// capsule's closest sphere t (App. D projection, FP64), clamped below at 1e-9 m; the K
// strongest are kept (ties keep the lower capsule id) and normalised.  One thread per vertex
// over every capsule of the scene, at the scene's current pose; the block stages the capsules
// in tiles of kSkinTile (world endpoints and radii in FP64, 17 KB of LDS) and every thread
// scans the tile in capsule order.  K = 4: the final influences (float weights); K = kFairK:
// the start of the fairing (FP64 lists, largest first).
constexpr int kSkinTile = 256;
constexpr int kFairK = 8;       // entries kept per vertex while fairing
constexpr int kFairAcc = 256;   // distinct capsules a fairing step can gather around one vertex

struct FairLists {
  int32_t* id;    // [V*kFairK]
  double* w;      // [V*kFairK]
  int32_t* n;     // [V] entries in use
};

template <class T, int K>
__global__ void __launch_bounds__(kSkinTile) skin_weights_kernel(const Dev<T> d, int V, const float* __restrict__ rest_v,
                                                                 int32_t* __restrict__ caps, float* __restrict__ w,
                                                                 FairLists fl) {
  __shared__ double s_geo[kSkinTile][8];   // c1 (3), c2 (3), r1, r2
  __shared__ int s_id[kSkinTile];          // capsule id, -1 for a slot without an edge
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const bool live = i < V;                 // every thread takes part in the staging
  const D3 x = live ? d3((double)rest_v[3 * (size_t)i], (double)rest_v[3 * (size_t)i + 1], (double)rest_v[3 * (size_t)i + 2])
                    : d3(0.0, 0.0, 0.0);
  int best[K];
  double bw[K];
#pragma unroll
  for (int k = 0; k < K; ++k) { best[k] = -1; bw[k] = -1.0; }
  for (int base = 0; base + 1 < d.P; base += kSkinTile) {
    const int p = base + (int)threadIdx.x;
    int id = -1;
    if (p + 1 < d.P && (d.flags[p] & F_EDGE)) {
      const double* an = d.anchor + 3 * (size_t)d.rod_of[p];
      double* g = s_geo[threadIdx.x];
      g[0] = an[0] + (double)d.px[p]; g[1] = an[1] + (double)d.py[p]; g[2] = an[2] + (double)d.pz[p];
      g[3] = an[0] + (double)d.px[p + 1]; g[4] = an[1] + (double)d.py[p + 1]; g[5] = an[2] + (double)d.pz[p + 1];
      g[6] = (double)d.s[p] * (double)d.rbar[p];
      g[7] = (double)d.s[p + 1] * (double)d.rbar[p + 1];
      id = p;
    }
    s_id[threadIdx.x] = id;
    __syncthreads();
    if (live) {
      const int n = min(kSkinTile, d.P - 1 - base);
      for (int j = 0; j < n; ++j) {
        const int pid = s_id[j];
        if (pid < 0) continue;
        const double* g = s_geo[j];
        const D3 c1 = d3(g[0], g[1], g[2]), c2 = d3(g[3], g[4], g[5]);
        const double r1 = g[6], r2 = g[7];
        const double t = pill_param(x, c1, r1, c2, r2);
        const D3 rel = sub(x, lerp(c1, c2, t));
        const double dist = fmax(sqrt(dotp(rel, rel)) - (r1 + t * (r2 - r1)), 1e-9);
        const double wt = 1.0 / (dist * dist);
        if (wt > bw[K - 1]) {
          int k = K - 1;
          while (k > 0 && wt > bw[k - 1]) {
            bw[k] = bw[k - 1]; best[k] = best[k - 1];
            --k;
          }
          bw[k] = wt; best[k] = pid;
        }
      }
    }
    __syncthreads();                       // the tile is overwritten next
  }
  if (!live) return;
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) if (best[k] >= 0) sum += bw[k];
  if constexpr (K == 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      caps[4 * (size_t)i + k] = best[k] >= 0 ? best[k] : best[0];
      w[4 * (size_t)i + k] = best[k] >= 0 ? (float)(bw[k] / sum) : 0.0f;
    }
  } else {
    int n = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (best[k] >= 0) n = k + 1;
      fl.id[(size_t)K * i + k] = best[k];
      fl.w[(size_t)K * i + k] = best[k] >= 0 ? bw[k] / sum : 0.0;
    }
    fl.n[i] = n;
  }
}

// One fairing iteration (Jacobi; the readings are those of the oracle's fairing): vertex i's
// new list is (1 - lambda) times its own entries, then lambda / degree times each neighbour's
// entries (neighbours in ascending index, each list largest first), summed per capsule in
// that order (FP64, no contraction); the kFairK largest are kept (ties: lower id first), in
// that order, divided by their sum (summed in that order).  More than kFairAcc distinct
// capsules around a vertex set *overflow.
__global__ void __launch_bounds__(256) skin_fair_step_kernel(int V, const int32_t* __restrict__ off,
                                                             const int32_t* __restrict__ nbr, FairLists in,
                                                             FairLists out, double lam, int32_t* __restrict__ overflow) {
#pragma clang fp contract(off)
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= V) return;
  int aid[kFairAcc];
  double aw[kFairAcc];
  int na = 0;
  bool full = false;
  auto add = [&](int id, double x) {
    for (int a = 0; a < na; ++a)
      if (aid[a] == id) { aw[a] += x; return; }
    if (na == kFairAcc) { full = true; return; }
    aid[na] = id; aw[na] = x; ++na;
  };
  const double self = 1.0 - lam;
  const int n0 = in.n[i];
  for (int k = 0; k < n0; ++k) add(in.id[(size_t)kFairK * i + k], self * in.w[(size_t)kFairK * i + k]);
  const int b = off[i], e = off[i + 1];
  if (e > b) {
    const double c = lam / (double)(e - b);
    for (int j = b; j < e; ++j) {
      const int u = nbr[j];
      const int nu = in.n[u];
      for (int k = 0; k < nu; ++k) add(in.id[(size_t)kFairK * u + k], c * in.w[(size_t)kFairK * u + k]);
    }
  }
  if (full) atomicExch(overflow, 1);
  // the kFairK largest, largest first (ties: lower id)
  int sid[kFairK];
  double sw[kFairK];
  const int n = min(kFairK, na);
  for (int k = 0; k < n; ++k) {
    int bi = -1;
    for (int a = 0; a < na; ++a) {
      if (aid[a] < 0) continue;
      if (bi < 0 || aw[a] > aw[bi] || (aw[a] == aw[bi] && aid[a] < aid[bi])) bi = a;
    }
    sid[k] = aid[bi];
    sw[k] = aw[bi];
    aid[bi] = -1;                        // taken
  }
  double sum = 0.0;
  for (int k = 0; k < n; ++k) sum += sw[k];
  for (int k = 0; k < kFairK; ++k) {
    out.id[(size_t)kFairK * i + k] = k < n ? sid[k] : -1;
    out.w[(size_t)kFairK * i + k] = k < n ? sw[k] / sum : 0.0;
  }
  out.n[i] = n;
}

// The four largest entries of each faired list (the lists are ordered largest first),
// normalised (summed in that order); fewer than four: the first capsule repeated, weight 0.
__global__ void __launch_bounds__(256) skin_fair_final_kernel(int V, FairLists in, int32_t* __restrict__ caps,
                                                              float* __restrict__ w) {
#pragma clang fp contract(off)
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= V) return;
  const int n = min(4, in.n[i]);
  double sum = 0.0;
  for (int k = 0; k < n; ++k) sum += in.w[(size_t)kFairK * i + k];
  const int first = in.id[(size_t)kFairK * i];
  for (int k = 0; k < 4; ++k) {
    caps[4 * (size_t)i + k] = k < n ? in.id[(size_t)kFairK * i + k] : first;
    w[4 * (size_t)i + k] = k < n ? (float)(in.w[(size_t)kFairK * i + k] / sum) : 0.0f;
  }
}

// Apply the last pass's averaged corrections now (before a bundling projection, which
// reads and overwrites the state of its section pills); the velocity update then finds
// nothing left to apply.
template <class T>
__global__ void __launch_bounds__(256) contact_flush_kernel(const Dev<T>* __restrict__ D, const ContactDev* __restrict__ CD,
                                                            const Blk* __restrict__ tab) {
  BLOCK_SCENE(tab, D, CD)
  const int p = blk_.base + (int)threadIdx.x;
  if (p >= c.P) return;
  T x0 = d.px[p], x1 = d.py[p], x2 = d.pz[p], s = d.s[p];
  if (contact_apply(c, p, x0, x1, x2, s)) {
    d.px[p] = x0; d.py[p] = x1; d.pz[p] = x2; d.s[p] = s;
  }
}

}  // namespace

// ----------------------------------------------------------------------------- host side

ContactOffsets contact_layout(size_t start, bool on, int P, int E, int cpc, bool f64) {
  ContactOffsets o;
  o.on = on;
  size_t off = start;
  auto take = [&](size_t bytes) {
    size_t r = off;
    off += (bytes + 255) & ~size_t(255);
    return r;
  };
  if (!on) {
    o.end = start;
    return o;
  }
  const int T = contact_table_size(E);
  const size_t cap = (size_t)cpc * (size_t)E;
  const size_t ts = f64 ? 8 : 4;
  const int nb = chunk_total_words(T);      // cell scan chunk totals
  o.cap_ids = take(4 * (size_t)E);
  o.cap_rod = take(4 * (size_t)E);
  o.cap_grp = take(4 * (size_t)E);
  o.sph = take(8 * 4 * (size_t)E);
  o.hist = take(4 * (size_t)kHistCopies * (kRadBins + 1));
  o.binmax = take(8 * (size_t)kHistCopies * kRadBins);
  o.dcnt = take(4 * 8);
  o.walk = take(8 * kWalkCounters);
  o.cw = take(8 * 2);
  o.key = take(4 * (size_t)E);
  o.pkey = take(8 * (size_t)E);
  o.cell_cnt = take(4 * (size_t)T);
  o.cell_start = take(4 * (size_t)(T + 1));
  o.cell_cur = take(4 * (size_t)T);
  o.sorted = take(4 * (size_t)E);
  o.cgmin = take(4 * (size_t)T);
  o.cgmax = take(4 * (size_t)T);
  o.stage = take(4 * (size_t)kStage * 256 * search_blocks(E));
  o.pairs = take(8 * cap);
  o.npairs = take(4);
  o.ssph = take(8 * 4 * (size_t)E);
  o.skey = take(8 * (size_t)E);
  o.srg = take(8 * (size_t)E);
  o.acc = take(8 * 4 * (size_t)P);
  o.acnt = take(4 * (size_t)P);
  o.xdet = take(8 * 3 * (size_t)P);   // FP64 world positions
  o.sdet = take(ts * (size_t)P);
  o.bsum = take(4 * (size_t)nb);
  o.end = off;
  return o;
}

int contact_table_size(int E) {
  int T = 64;
  while (T < 2 * E) T <<= 1;
  return T;
}

viper_status contact_init(ContactDev& c, char* ws, const ContactOffsets& o, const viper_scene_desc* d,
                          const std::vector<int32_t>& off, const std::vector<int32_t>& group, int32_t* status,
                          hipStream_t st) {
  c = ContactDev();
  if (!o.on) return VIPER_OK;
  const int R = (int)off.size() - 1;
  c.P = off[R];
  std::vector<int32_t> ids, rod, grp;
  double rmax = 0.0;                   // largest bounding radius at rest
  for (int k = 0; k < R; ++k)
    for (int p = off[k]; p + 1 < off[k + 1]; ++p) {
      ids.push_back(p); rod.push_back(k); grp.push_back(group[k]);
      const double* x0 = d->rest_pos + 3 * (size_t)p;
      const double dx = x0[3] - x0[0], dy = x0[4] - x0[1], dz = x0[5] - x0[2];
      const double R0 = 0.5 * std::sqrt(dx * dx + dy * dy + dz * dz) + std::max(d->rest_radius[p], d->rest_radius[p + 1]);
      rmax = std::max(rmax, R0);
    }
  c.rlim = kRadLimit * rmax;
  c.E = (int)ids.size();
  c.T = contact_table_size(c.E);
  const int cpc = d->contact_capacity_per_capsule > 0 ? d->contact_capacity_per_capsule : 16;
  c.cap = cpc * c.E;
  c.cap_ids = (int32_t*)(ws + o.cap_ids);
  c.cap_rod = (int32_t*)(ws + o.cap_rod);
  c.cap_grp = (int32_t*)(ws + o.cap_grp);
  c.sph = (double*)(ws + o.sph);
  c.hist = (int32_t*)(ws + o.hist);
  c.binmax = (unsigned long long*)(ws + o.binmax);
  c.dcnt = (int32_t*)(ws + o.dcnt);
  c.walk = (unsigned long long*)(ws + o.walk);
  c.cw = (double*)(ws + o.cw);
  c.key = (int32_t*)(ws + o.key);
  c.pkey = (long long*)(ws + o.pkey);
  c.cell_cnt = (int32_t*)(ws + o.cell_cnt);
  c.cell_start = (int32_t*)(ws + o.cell_start);
  c.cell_cur = (int32_t*)(ws + o.cell_cur);
  c.sorted = (int32_t*)(ws + o.sorted);
  c.cgmin = (int32_t*)(ws + o.cgmin);
  c.cgmax = (int32_t*)(ws + o.cgmax);
  c.stage = (int32_t*)(ws + o.stage);
  c.pairs = (int32_t*)(ws + o.pairs);
  c.npairs = (int32_t*)(ws + o.npairs);
  c.ssph = (double*)(ws + o.ssph);
  c.skey = (long long*)(ws + o.skey);
  c.srg = (int32_t*)(ws + o.srg);
  c.acc = (unsigned long long*)(ws + o.acc);
  c.acnt = (int32_t*)(ws + o.acnt);
  c.xdet = (double*)(ws + o.xdet);
  c.sdet = ws + o.sdet;
  c.bsum = (int32_t*)(ws + o.bsum);
  c.status = status;
  if (hipMemcpyAsync(c.cap_ids, ids.data(), 4 * ids.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c.cap_rod, rod.data(), 4 * rod.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c.cap_grp, grp.data(), 4 * grp.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemsetAsync(c.npairs, 0, 4, st) != hipSuccess ||
      hipMemsetAsync(c.hist, 0, 4 * (size_t)kHistCopies * (kRadBins + 1), st) != hipSuccess ||
      hipMemsetAsync(c.binmax, 0, 8 * (size_t)kHistCopies * kRadBins, st) != hipSuccess ||
      hipMemsetAsync(c.dcnt, 0, 4 * 8, st) != hipSuccess || hipMemsetAsync(c.walk, 0, 8 * kWalkCounters, st) != hipSuccess ||
      hipMemsetAsync(c.cw, 0, 8 * 2, st) != hipSuccess ||
      hipMemsetAsync(c.acc, 0, 8 * 4 * (size_t)c.P, st) != hipSuccess ||
      hipMemsetAsync(c.acnt, 0, 4 * (size_t)c.P, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return VIPER_ERR_DEVICE;
  return VIPER_OK;
}

template <class T>
hipError_t launch_contact_detect(const BatchDev& b, hipStream_t st) {
  if (b.nscenes == 0) return hipSuccess;
  const Dev<T>* D = (const Dev<T>*)b.dev;
  const ContactDev* CD = b.cd;
  const dim3 blk(256);
  // the detection record of every capsule (sphere, radius bin, histogram) and the resets were
  // formed by the prediction launch (launch_predict / launch_velocity with a next substep)
  (void)D;
  hipLaunchKernelGGL(key_kernel, dim3(b.nblk[TB_CAPS]), dim3(kCapsBlock), 0, st, CD, b.tab[TB_CAPS]);
  hipLaunchKernelGGL(scan_kernel, dim3(b.nblk[TB_SCAN_T]), blk, 0, st, CD, b.tab[TB_SCAN_T]);
  hipLaunchKernelGGL(bucket_scatter_kernel, dim3(b.nblk[TB_CAPS]), dim3(kCapsBlock), 0, st, CD, b.tab[TB_CAPS]);
  hipLaunchKernelGGL(pair_kernel, dim3(b.nblk[TB_SEARCH]), blk, 0, st, CD, b.tab[TB_SEARCH]);
  return hipGetLastError();
}

template <class T>
hipError_t launch_contact_project(const BatchDev& b, hipStream_t st) {
  if (b.nscenes == 0) return hipSuccess;
  const Dev<T>* D = (const Dev<T>*)b.dev;
  hipLaunchKernelGGL(contact_pair_kernel<T>, dim3(b.nblk[TB_PAIRS]), dim3(64), 0, st, D, b.cd, b.tab[TB_PAIRS]);
  return hipGetLastError();
}

template <class T>
hipError_t launch_contact_flush(const BatchDev& b, hipStream_t st) {
  if (b.nscenes == 0 || b.nblk[TB_DET] == 0) return hipSuccess;
  hipLaunchKernelGGL(contact_flush_kernel<T>, dim3(b.nblk[TB_DET]), dim3(256), 0, st, (const Dev<T>*)b.dev, b.cd,
                     b.tab[TB_DET]);
  return hipGetLastError();
}

template <class T>
hipError_t launch_skin_weights(const Dev<T>& d, int V, const float* rest_v, int32_t* caps, float* w, hipStream_t st) {
  if (V <= 0) return hipSuccess;
  hipLaunchKernelGGL((skin_weights_kernel<T, 4>), dim3((V + kSkinTile - 1) / kSkinTile), dim3(kSkinTile), 0, st, d, V,
                     rest_v, caps, w, FairLists{nullptr, nullptr, nullptr});
  return hipGetLastError();
}
template hipError_t launch_skin_weights<float>(const Dev<float>&, int, const float*, int32_t*, float*, hipStream_t);
template hipError_t launch_skin_weights<double>(const Dev<double>&, int, const float*, int32_t*, float*, hipStream_t);

size_t skin_fair_work_bytes(int V, int64_t nbr_entries) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t lists = al(4 * (size_t)kFairK * V) + al(8 * (size_t)kFairK * V) + al(4 * (size_t)V);
  return al(4 * ((size_t)V + 1)) + al(4 * (size_t)nbr_entries) + 2 * lists + 256;
}

template <class T>
hipError_t launch_skin_weights_faired(const Dev<T>& d, int V, const float* rest_v, const int32_t* off,
                                      const int32_t* nbr, int64_t nbr_entries, int iters, double lam, char* work,
                                      int32_t* overflow, int32_t* caps, float* w, hipStream_t st) {
  if (V <= 0) return hipSuccess;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* at = work + al(4 * ((size_t)V + 1)) + al(4 * (size_t)nbr_entries);
  FairLists L[2];
  for (int b = 0; b < 2; ++b) {
    L[b].id = (int32_t*)at; at += al(4 * (size_t)kFairK * V);
    L[b].w = (double*)at; at += al(8 * (size_t)kFairK * V);
    L[b].n = (int32_t*)at; at += al(4 * (size_t)V);
  }
  hipLaunchKernelGGL((skin_weights_kernel<T, kFairK>), dim3((V + kSkinTile - 1) / kSkinTile), dim3(kSkinTile), 0, st, d,
                     V, rest_v, (int32_t*)nullptr, (float*)nullptr, L[0]);
  const dim3 g((V + 255) / 256), blk(256);
  for (int it = 0; it < iters; ++it)
    hipLaunchKernelGGL(skin_fair_step_kernel, g, blk, 0, st, V, off, nbr, L[it & 1], L[(it + 1) & 1], lam, overflow);
  hipLaunchKernelGGL(skin_fair_final_kernel, g, blk, 0, st, V, L[iters & 1], caps, w);
  return hipGetLastError();
}
template hipError_t launch_skin_weights_faired<float>(const Dev<float>&, int, const float*, const int32_t*, const int32_t*,
                                                      int64_t, int, double, char*, int32_t*, int32_t*, float*, hipStream_t);
template hipError_t launch_skin_weights_faired<double>(const Dev<double>&, int, const float*, const int32_t*,
                                                       const int32_t*, int64_t, int, double, char*, int32_t*, int32_t*,
                                                       float*, hipStream_t);

hipError_t contact_copy_det(const ContactDev& c, bool x, void* dst, int P, size_t ts, hipStream_t st) {
  return hipMemcpyAsync(dst, x ? (void*)c.xdet : c.sdet, (x ? 3 * 8 : ts) * (size_t)P, hipMemcpyDefault, st);
}

viper_status contact_get_pairs(const ContactDev& c, int32_t* pairs, int32_t cap, int32_t* n, hipStream_t st) {
  int32_t h = 0;
  if (hipMemcpyAsync(&h, c.npairs, 4, hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return VIPER_ERR_DEVICE;
  h = std::min(h, c.cap);               // an overflowing detection keeps its first cap pairs
  *n = h;
  if (h > cap) return VIPER_ERR_NO_CAPACITY;
  if (h > 0) {
    if (!pairs) return VIPER_ERR_INVALID;
    // the device list holds each pair once as (lower, higher) capsule id, grouped by the
    // capsule whose walk found it and in the order of the atomics: sorted here
    std::vector<int64_t> v((size_t)h);
    if (hipMemcpyAsync(v.data(), c.pairs, 8 * (size_t)h, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return VIPER_ERR_DEVICE;
    std::vector<std::pair<int32_t, int32_t>> pr((size_t)h);
    std::memcpy(pr.data(), v.data(), 8 * (size_t)h);
    std::sort(pr.begin(), pr.end());
    std::memcpy(v.data(), pr.data(), 8 * (size_t)h);
    if (hipMemcpyAsync(pairs, v.data(), 8 * (size_t)h, hipMemcpyDefault, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return VIPER_ERR_DEVICE;
  }
  return VIPER_OK;
}

viper_status contact_get_info(const ContactDev& c, viper_contact_info* out, hipStream_t st) {
  int32_t cnt[8];
  unsigned long long walk[kWalkCounters];
  double cw[2] = {0.0, 0.0};
  if (hipMemcpyAsync(cnt, c.dcnt, sizeof(cnt), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(walk, c.walk, sizeof(walk), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(cw, c.cw, sizeof(cw), hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return VIPER_ERR_DEVICE;
  unsigned long long total = 0;
  for (int k = 0; k < kWalkCounters; ++k) total += walk[k];
  out->walk_entries = (int64_t)total;
  out->oversized = cnt[0];
  out->skipped = cnt[1];
  out->excluded = cnt[2];
  out->cell_bin = cnt[3];
  out->cell_width = cw[0];
  out->cell_radius_limit = c.rlim;
  out->coarse_bin = cnt[4];
  out->coarse_capsules = cnt[5];
  out->coarse_width = cw[1];
  return VIPER_OK;
}

template hipError_t launch_contact_detect<float>(const BatchDev&, hipStream_t);
template hipError_t launch_contact_detect<double>(const BatchDev&, hipStream_t);
template hipError_t launch_contact_project<float>(const BatchDev&, hipStream_t);
template hipError_t launch_contact_project<double>(const BatchDev&, hipStream_t);
template hipError_t launch_contact_flush<float>(const BatchDev&, hipStream_t);
template hipError_t launch_contact_flush<double>(const BatchDev&, hipStream_t);

}  // namespace viper
