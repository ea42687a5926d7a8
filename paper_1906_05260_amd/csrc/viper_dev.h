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
  F_SS = 32u, F_VOL = 64u, F_SG = 128u, F_BTEN = 256u  // constraint types enabled for the rod
};

enum { ST_NAN = 0, ST_OVERFLOW = 1, ST_WORDS = 4 };

template <class T>
struct Dev {
  int P;                     // pills
  int W;                     // waves (each holds whole rods, <= 64 pills)
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
  const T *css, *cvol, *csg, *cbtc;             // compliance / (G * length)
  const T *qrx, *qry, *qrz, *qrw;               // rest quaternion
  const T *mrx, *mry, *mrz;                     // rest capsule midpoint
  // substep scratch (ITERATION mode)
  T *xpx, *xpy, *xpz, *spv, *qpx, *qpy, *qpz, *qpw;  // state at substep start
  T *lam;                    // [8*P] accumulated multipliers: ss(3) vol sg bt(3)
  T *i1;                     // [P] inverse bending inertia of the edge for this substep
  int32_t* status;           // [ST_WORDS]
  // Positions are stored relative to a per-rod anchor (the rest position of the rod's
  // first pill), so that FP32 resolves edge vectors independently of where the rod
  // sits in the world; world = anchor[rod] + local, formed in FP64 where needed.
  const double* anchor;      // [3*R]
  const int32_t* rod_of;     // [P]
  T gx, gy, gz;
};

// Launchers (enqueue on `stream`, return hipError_t of the launch).
template <class T> hipError_t launch_rod_frame(const Dev<T>& d, int nsub, double h, int iters, hipStream_t st);
template <class T> hipError_t launch_predict(const Dev<T>& d, double h, hipStream_t st);
template <class T> hipError_t launch_rod_iteration(const Dev<T>& d, double h, hipStream_t st);
template <class T> hipError_t launch_velocity(const Dev<T>& d, double h, hipStream_t st);
template <class T> hipError_t launch_gather_field(const Dev<T>& d, int which, T* out, hipStream_t st);
template <class T> hipError_t launch_scatter_field(const Dev<T>& d, int which, const T* in, hipStream_t st);
template <class T> hipError_t launch_skin(const Dev<T>& d, int V, const float* rest_v, const int32_t* caps,
                                          const float* w, float* out, float* xform, hipStream_t st);

}  // namespace viper
