// Pill-pill contacts (Sec. 7.1 detection, Sec. 7.2 handling): private interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "../../include/viper.h"
#include "viper_dev.h"

namespace viper {

struct ContactOffsets {
  bool on = false;
  size_t cap_ids, cap_rod, cap_grp, sph, maxr, key, cell_cnt, cell_start, cell_cur, sorted;
  size_t pcount, poff, pairs, npairs, pill_cnt, pill_start, pill_cur, entries, delta, active;
  size_t xdet, sdet, bsum;
  size_t end;
};

struct ContactDev {
  bool on = false;
  int P = 0, E = 0, T = 0, cap = 0, nbsum = 0;   // pills, capsules, hash-table size, pair capacity
  int search_iters = 10;
  double delta = 1e-4;
  int32_t *cap_ids = nullptr, *cap_rod = nullptr, *cap_grp = nullptr;
  double* sph = nullptr;              // [E*4] mx my mz R
  unsigned long long* maxr = nullptr; // bits of the largest sphere radius
  int32_t *key = nullptr, *cell_cnt = nullptr, *cell_start = nullptr, *cell_cur = nullptr, *sorted = nullptr;
  int32_t *pcount = nullptr, *poff = nullptr, *pairs = nullptr, *npairs = nullptr;
  int32_t *pill_cnt = nullptr, *pill_start = nullptr, *pill_cur = nullptr, *entries = nullptr;
  double* delta_buf = nullptr;        // [cap*16] per-pair corrections of the 4 end pills (dx dy dz ds)
  int32_t* active = nullptr;          // [cap]
  void *xdet = nullptr, *sdet = nullptr;
  int32_t* bsum = nullptr;            // scan scratch
  int32_t* status = nullptr;
};

ContactOffsets contact_layout(size_t start, bool on, int P, int E, int cap_per_capsule, bool f64);
viper_status contact_init(ContactDev& c, char* ws, const ContactOffsets& o, const viper_scene_desc* d,
                          const std::vector<int32_t>& off, const std::vector<int32_t>& group, hipStream_t st);
template <class T> hipError_t contact_detect(const Dev<T>& d, ContactDev& c, hipStream_t st);
template <class T> hipError_t contact_project(const Dev<T>& d, ContactDev& c, hipStream_t st);
hipError_t contact_copy_det(ContactDev& c, bool x, void* dst, int P, size_t ts, hipStream_t st);
viper_status contact_get_pairs(ContactDev& c, int32_t* pairs, int32_t cap, int32_t* n, hipStream_t st);

}  // namespace viper
