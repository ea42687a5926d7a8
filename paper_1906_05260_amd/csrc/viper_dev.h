// Private device-side layout of a VIPER scene and the kernel launchers.
//
// Structure-of-arrays in one caller-owned workspace, rod-major and contiguous:
// pill slot p holds vertex p of its rod and, when it is not the rod's last
// vertex, the edge (p, p+1) and the bend-twist constraint between edges p and
// p+1 (staggered storage: scales at vertices, frames at edge midpoints, Sec. 4).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace viper {

// Per-pill flags (rod structure and per-rod constraint enables).
enum : uint32_t {
  F_VALID = 1u,   // slot holds a pill
  F_EDGE = 2u,    // pill is not the last of its rod: edge (p, p+1) exists
  F_BT = 4u,      // edges (p, p+1) and (p+1, p+2) exist: bend-twist at vertex p+1
  F_ODD = 8u,     // local vertex index within the rod is odd (colour parity)
  F_FIRST = 16u,  // first pill of its rod
  F_SS = 32u, F_VOL = 64u, F_SG = 128u, F_BTEN = 256u,  // constraint types enabled for the rod
  F_SR = 512u,    // cross-section stretch enabled for the rod (optional, eq. stretch_xy)
  F_SB = 1024u,   // surface bending enabled for the rod (optional, Laplacian of the scale)
  F_M3A = 2048u, F_M3B = 4096u,  // local pill index mod 3 is 1 / is 2 (surface-bending colour)
  F_VB = 8192u    // volume-bending coupling at the vertex after the slot's edge (optional)
};

// Status words of a scene, set by kernels and read by viper_sync: a non-finite state, a full
// contact-pair buffer, and a contact detection skipped because the scene's capsules outgrew
// the grid's limit (a diverged scene).
enum { ST_NAN = 0, ST_OVERFLOW = 1, ST_DIVERGED = 2, ST_WORDS = 4 };

template <class T>
struct Dev {
  int P;                     // pills
  int W;                     // waves (each holds whole rods, <= 128 pills)
  const int32_t* wave_start; // [W+1] first pill of each wave
  const uint32_t* flags;     // [P]
  // state
  T *px, *py, *pz, *vx, *vy, *vz, *s, *sd;      // per pill
  T *qx, *qy, *qz, *qw, *ox, *oy, *oz;          // per edge slot
  // rest data per pill
  const T *winv, *wsinv, *rbar;
  // rest data per edge slot
  const T *ilb, *il0, *cbt, *inert;             // 1/lbar, 1/l0, 4/(l0_j + l0_{j+1}), rho pi r^4 l0
  const T *dbx, *dby, *dbz;                     // rest Darboux vector of the bend-twist at this slot
  const T *css, *cvol, *csg, *cbtc, *csr;
  const T *csb, *sbg0, *sbg2;                   // surface bending at the vertex after the slot's edge
  const T *cvb;                                 // volume-bending coupling, compliance / (G l_v)             // compliance / (G * length)
  const T *qrx, *qry, *qrz, *qrw;               // rest quaternion
  const T *mrx, *mry, *mrz;                     // rest capsule midpoint
  // substep scratch (ITERATION mode)
  T *xpx, *xpy, *xpz, *spv, *qpx, *qpy, *qpz, *qpw;  // state at substep start
  T *lam;                    // [12*P] accumulated multipliers: ss(3) vol sg bt(3) sr sb vb(2)
  T *i1;                     // [P] inverse bending inertia of the edge for this substep
  int32_t* status;           // [ST_WORDS]
  // Positions are stored relative to a per-rod anchor (the rest position of the rod's
  // first pill), so that FP32 resolves edge vectors independently of where the rod
  // sits in the world; world = anchor[rod] + local, formed in FP64 where needed.
  const double* anchor;      // [3*R]
  const int32_t* rod_of;     // [P]
  T gx, gy, gz;
  // bundling cross-sections (Sec. 7.3): nsec sections over nsecp entries
  int nsec, nsecp;
  const int32_t *sec_off, *sec_pill, *sec_of;  // [nsec+1], [nsecp] pill, [nsecp] section of the entry
  const double* sec_xr;      // [3*nsecp] world rest position of each entry
  double* sec_q;             // [4*nsec] rotation of the last fit (start of the next extraction)
  double* sec_fit;           // [kSecFit*nsec] R* (row-major), s*, c*, q*
  // half-plane floor (Sec. 7): n . x >= fd + s rbar, unit n
  int floor_on;
  double fnx, fny, fnz, fd;
  // rod-constraint solver in ITERATION mode: 0 = coloured Gauss-Seidel, 1 = Jacobi with averaging
  int jacobi;
};
constexpr int kSecFit = 20;

constexpr int kRadBins = 128;     // bounding-radius histogram: 4 bins per octave, bin 96 starts at 1 m
constexpr int kOversized = 32;    // at most this many capsules are larger than the cell radius
constexpr int kWalkCounters = 64; // partial sums of the candidate walk length (a power of two)
constexpr double kRadLimit = 4.0; // cell radius limit, in units of the largest bounding radius at rest

// Contact buffers of one scene (device pointers into its workspace).
struct ContactDev {
  int P = 0, E = 0, T = 0, cap = 0;   // pills, capsules, hash-table size, pair capacity
  int search_iters = 10;
  double delta = 1e-4;
  int32_t *cap_ids = nullptr, *cap_rod = nullptr, *cap_grp = nullptr;
  double* sph = nullptr;              // [E*4] mx my mz R
  // Grid sizing: a histogram of the bounding radii (kRadBins log-spaced bins, then one count of
  // capsules left out) finds the bin holding the (kOversized+1)-th largest radius (larger
  // capsules are walked from a list instead) and the split between a fine and a coarse grid
  // level below it.
  int32_t* hist = nullptr;            // [kRadBins + 1]
  unsigned long long* binmax = nullptr;  // [kRadBins] bits of the largest radius in each bin
  // Last detection: [0] oversized, [1] skipped, [2] non-finite, [3] fine bin, [4] cell bin
  // when a coarse level is used (else -1), [5] coarse-level capsules
  int32_t* dcnt = nullptr;            // [8]
  unsigned long long* walk = nullptr; // [kWalkCounters] partial sums of the entries the last count pass examined
  double* cw = nullptr;               // [2] fine and coarse cell widths of the last detection (0: skipped / one level)
  double rlim = 0.0;                  // largest admitted cell radius (4x the largest at rest)
  int32_t* key = nullptr;             // [E] radius bin, then hash bucket
  long long* pkey = nullptr;          // [E] cell key (wrapped cell coordinates and grid level)
  int32_t *cell_cnt = nullptr, *cell_start = nullptr, *cell_cur = nullptr;
  int32_t* sorted = nullptr;          // [E] capsule ids (first pill) in bucket order
  int32_t *cgmin = nullptr, *cgmax = nullptr;  // [T] smallest / largest group id in each bucket
  int32_t* stage = nullptr;           // [8 * 256 search_blocks(E)] first candidates of each search thread
  int32_t* pairs = nullptr;           // [cap] candidate pairs (lower, higher capsule id)
  int32_t* npairs = nullptr;          // pairs found (the list keeps the first cap of them)
  double* ssph = nullptr;             // [E*4] spheres in bucket (cell) order
  long long* skey = nullptr;          // [E] cell keys in bucket order (-1: oversized list)
  int32_t* srg = nullptr;             // [E*2] rod, group in bucket order
  unsigned long long* acc = nullptr;  // [P*4] fixed-point sums of contact corrections (dx dy dz ds)
  int32_t* acnt = nullptr;            // [P] active contacts per pill this pass
  double* xdet = nullptr;             // [3P] FP64 world positions at detection
  void* sdet = nullptr;               // [P] scales at detection (scene precision)
  int32_t* bsum = nullptr;            // cell scan chunk totals
  int32_t* status = nullptr;          // the scene's status words
};

// End of a Jacobi contact pass, for pill p: add the average of the fixed-point sums of its
// contact corrections (position and scale, 2^-44 per unit) and clear the sums.  Returns
// whether the pill had an active contact.
template <class T>
__device__ __forceinline__ bool contact_apply(const ContactDev& c, int p, T& x0, T& x1, T& x2, T& s) {
  const int n = c.acnt[p];
  if (n == 0) return false;
  unsigned long long* a = c.acc + 4 * (size_t)p;
  const double inv = 1.0 / (double)n;
  const double ax = (double)(long long)a[0] * 0x1p-44, ay = (double)(long long)a[1] * 0x1p-44;
  const double az = (double)(long long)a[2] * 0x1p-44, as = (double)(long long)a[3] * 0x1p-44;
  x0 = (T)((double)x0 + inv * ax);
  x1 = (T)((double)x1 + inv * ay);
  x2 = (T)((double)x2 + inv * az);
  s = (T)((double)s + inv * as);
  a[0] = 0ull; a[1] = 0ull; a[2] = 0ull; a[3] = 0ull;
  c.acnt[p] = 0;
  return true;
}

// Half-plane floor, for pill p at (x0, x1, x2) with scale s: lift the pill along the normal
// until its sphere touches the plane (positions only; pinned pills stay).
template <class T>
__device__ __forceinline__ void floor_apply(const Dev<T>& d, int p, T& x0, T& x1, T& x2, T s) {
  if (!(d.winv[p] > T(0))) return;
  const double* an = d.anchor + 3 * (size_t)d.rod_of[p];
  const double C = (d.fnx * (an[0] + (double)x0) + d.fny * (an[1] + (double)x1) + d.fnz * (an[2] + (double)x2)) -
                   d.fd - (double)s * (double)d.rbar[p];
  if (!(C < 0.0)) return;
  x0 = (T)((double)x0 - C * d.fnx);
  x1 = (T)((double)x1 - C * d.fny);
  x2 = (T)((double)x2 - C * d.fnz);
}

// A batch of scenes advanced by the same launches.  Each launch's grid is described by a
// block table: block b works on scene tab[b].scene, items tab[b].base + [0, block size).
// Every scene's item range is padded to whole blocks, so a block never spans two scenes.
struct Blk {
  int32_t scene, base;
};

// One wavefront of a scene, for the kernels that run one wavefront per block: its scene, its
// index in the scene, its first pill and its pill count (the wave's range, so that a launch
// starts without reading it from the scene's wave table).
struct WaveBlk {
  int32_t scene, wave, p0, n;
};

// The launch record of such a wavefront: its WaveBlk and its scene's contact sums (null without
// contacts), followed in memory by a copy of its scene's Dev (in the batch's precision), so that
// a block starts with reads that depend on nothing but its index.
struct WaveRec {
  WaveBlk b;
  unsigned long long* acc;
  int32_t* acnt;
};

enum Stage {
  TB_WAVES = 0,   // 4 wavefronts (<= 512 pill slots) per block: rod kernels
  TB_CAPS,        // 256 capsules per block
  TB_SEARCH,      // 28 capsules per block, 9 threads each: neighbour search
  TB_PAIRS,       // 64 lanes per block, two per candidate pair, 2 pair_span(cap) lanes per scene
  TB_SCAN_T,      // 1024 cells per block (cell scan)
  TB_DET,         // 256 of max(pills, cells, capsules) per block: contact flush
  TB_SECT,        // 4 bundling sections per block (one wavefront each)
  TB_SECP,        // 256 bundling section entries per block
  TB_COUNT
};

// Candidate pairs the contact pass covers per round and scene (its blocks stride over the
// pair list in rounds of this many pairs).
constexpr int kPairSpan = 32768;
__host__ __device__ inline int pair_span(int cap) { return cap < kPairSpan ? cap : kPairSpan; }


struct BatchDev {
  int nscenes = 0;
  const void* dev = nullptr;          // Dev<T>[nscenes] in device memory
  const ContactDev* cd = nullptr;     // ContactDev[nscenes] in device memory (contact batches)
  const Blk* tab[TB_COUNT] = {};
  int nblk[TB_COUNT] = {};
  const char* wrec = nullptr;         // WaveRec + Dev of every wavefront of every scene, in scene order
  int wrec_stride = 0;                // bytes per record
  int nwaves = 0;
  bool extras = false;                // some scene uses an optional constraint term (the rod
                                      // kernels' instantiation with them compiled in)
  bool even = false;                  // every rod of every scene starts on an even slot of its
                                      // wavefront (the rod kernels' lane-local colour passes)
};

// Launchers over a batch (enqueue on `stream`, return hipError_t of the launches).
template <class T> hipError_t launch_rod_frame(const BatchDev& b, int nsub, double h, int iters, hipStream_t st);
// With contacts (cd non-null) the prediction also writes the detection copy of the state.
template <class T> hipError_t launch_predict(const BatchDev& b, double h, const ContactDev* cd, hipStream_t st);
// With contacts (cd non-null) the rod iteration and the velocity update first apply each
// pill's averaged corrections of the preceding contact pass (contact_apply).
template <class T> hipError_t launch_rod_iteration(const BatchDev& b, double h, const ContactDev* cd, hipStream_t st);
// `next`: what the same launch does after the velocity update, from the state it has just
// formed: 0 nothing, 1 the next substep's prediction (of the same step h, in place of a
// separate launch_predict), 2 that prediction and the next substep's first iteration (in
// place of its first launch_rod_iteration).
template <class T>
hipError_t launch_velocity(const BatchDev& b, double h, const ContactDev* cd, int next, hipStream_t st);
template <class T> hipError_t launch_contact_detect(const BatchDev& b, hipStream_t st);
template <class T> hipError_t launch_contact_project(const BatchDev& b, hipStream_t st);
// Apply the last contact pass's averaged corrections now (before a bundling projection).
template <class T> hipError_t launch_contact_flush(const BatchDev& b, hipStream_t st);
// Bundling projection of every section (fit, then apply).
template <class T> hipError_t launch_bundle(const BatchDev& b, hipStream_t st);
template <class T> hipError_t launch_gather_field(const Dev<T>& d, int which, T* out, hipStream_t st);
template <class T> hipError_t launch_scatter_field(const Dev<T>& d, int which, const T* in, hipStream_t st);
// Adjoint of the collision-free frame (single scene): checkpoint layout [substep][15][P].
constexpr int kCkptFields = 15;
// Backward scratch: per iteration, the pre-pass snapshots of the two edge passes (26 values
// per lane) and of the two bend-twist passes (16 values per lane).
constexpr int kSnapEdge = 26, kSnapBt = 16;
constexpr int kSnapPerIter = 2 * kSnapEdge + 2 * kSnapBt;
// ... after the last iteration the substep-end quaternions of both slots; two such buffers
// (the replay of one substep runs beside the reverse of the next).
constexpr int kSnapEnd = 8;
template <class T> hipError_t launch_frame_ckpt(const BatchDev& b, int nsub, double h, int iters, T* ckpt, hipStream_t st);
template <class T> hipError_t launch_backward(const BatchDev& b, int P, int nsub, double h, int iters, const T* ckpt,
                                              const T* dldx, T* snap, T* adj, T* padj, double rho, double* drbar,
                                              double* dact, hipStream_t st);
template <class T> hipError_t launch_skin(const Dev<T>& d, int V, const float* rest_v, const int32_t* caps,
                                          const float* w, float* out, float* xform, hipStream_t st);

}  // namespace viper
