// Pill-pill contacts (Sec. 7.1 detection, Sec. 7.2 handling): private host interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "../../include/viper.h"
#include "viper_dev.h"

namespace viper {

// Offsets of the contact buffers inside a scene workspace.
struct ContactOffsets {
  bool on = false;
  size_t cap_ids, cap_rod, cap_grp, sph, hist, binmax, dcnt, walk, cw, key, pkey, cell_cnt, cell_start, cell_cur, sorted, cgmin, cgmax;
  size_t stage, pairs, npairs, ssph, skey, srg, acc, acnt;
  size_t xdet, sdet, bsum;
  size_t end;
};

int contact_table_size(int E);
ContactOffsets contact_layout(size_t start, bool on, int P, int E, int cap_per_capsule, bool f64);
// Fill `c` with the scene's contact buffers and upload the capsule tables.
viper_status contact_init(ContactDev& c, char* ws, const ContactOffsets& o, const viper_scene_desc* d,
                          const std::vector<int32_t>& off, const std::vector<int32_t>& group, int32_t* status,
                          hipStream_t st);
hipError_t contact_copy_det(const ContactDev& c, bool x, void* dst, int P, size_t ts, hipStream_t st);
viper_status contact_get_pairs(const ContactDev& c, int32_t* pairs, int32_t cap, int32_t* n, hipStream_t st);
// Record of the last detection (walk length, oversized and non-finite capsules, cell width).
viper_status contact_get_info(const ContactDev& c, viper_contact_info* out, hipStream_t st);
// Initial skinning weights of V rest vertices at the scene's current pose (Sec. 7.4).
template <class T>
hipError_t launch_skin_weights(const Dev<T>& d, int V, const float* rest_v, int32_t* caps, float* w, hipStream_t st);
// Scratch of the faired weights: the mesh graph (CSR offsets [V+1], neighbours) at the start,
// then two sets of per-vertex candidate lists.
size_t skin_fair_work_bytes(int V, int64_t nbr_entries);
// Initial weights faired over the mesh graph (off, nbr: CSR inside `work`, already uploaded),
// `iters` Jacobi Laplacian-smoothing iterations with weight `lam`; the four largest written to
// caps / w.  *overflow (device) is set if a vertex gathers more capsules than a step holds.
template <class T>
hipError_t launch_skin_weights_faired(const Dev<T>& d, int V, const float* rest_v, const int32_t* off,
                                      const int32_t* nbr, int64_t nbr_entries, int iters, double lam, char* work,
                                      int32_t* overflow, int32_t* caps, float* w, hipStream_t st);

}  // namespace viper
