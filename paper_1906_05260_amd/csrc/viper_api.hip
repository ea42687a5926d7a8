// Host runtime of libviper.so: the C ABI declared in include/viper.h.
//
// Scene creation validates the description, computes the rest quantities on
// the host in FP64 (rest lengths, parallel-transported rest frames, rest
// Darboux vectors, lumped inverse masses, inertias and compliance scalings),
// and packs them with the initial state into the caller's workspace as
// structure-of-arrays.  Steps only enqueue kernels on the caller's stream.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/viper.h"
#include "viper_dev.h"
#include "bones.h"
#include "contact.h"

using namespace viper;

namespace {

thread_local std::string g_err;

viper_status fail(viper_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(VIPER_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

const double kPi = 3.14159265358979323846;
const int kMaxPills = 128;    // pills per rod: a rod lives in one wavefront (two slots per lane)
const int kWaveSpan = 128;    // pill slots per wavefront (two per lane)

// ----------------------------------------------------------------------------- layout

struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};

// Offsets of every array inside the workspace.
struct Offsets {
  size_t state[15];        // px py pz vx vy vz s sd qx qy qz qw ox oy oz
  size_t pill_rest[3];     // winv wsinv rbar
  size_t edge_rest[23];    // ilb il0 cbt inert dbx dby dbz css cvol csg cbtc qrx qry qrz qrw mrx mry mrz csr
                           // csb sbg0 sbg2 cvb
  size_t scratch[10];      // xpx xpy xpz spv qpx qpy qpz qpw i1 lam(12P)
  size_t flags, wave_start, status, stage, xform, anchor, rod_of, header;
  size_t sec_off = 0, sec_pill = 0, sec_of = 0, sec_xr = 0, sec_q = 0, sec_fit = 0;   // bundling
  size_t bone_prev = 0, bone_delta = 0, pill_bone = 0, pill_bone_w = 0;  // bones
  ContactOffsets contact;
  size_t total;
};

struct Host {
  int R = 0, P = 0, W = 0, E = 0;
  int64_t proj_per_iter = 0;
  std::vector<int32_t> off, wave_start, group;
  std::vector<uint32_t> flags;
  // rest data (FP64)
  std::vector<double> x, rbar, winv, wsinv, anchor, xloc;
  std::vector<int32_t> rod_of;
  std::vector<double> ilb, il0, cbt, inert, db[3], cs[5], qr[4], mr[3];
  std::vector<double> sbc, sbg0, sbg2;   // surface bending: compliance scaling, dC/ds_j-1, dC/ds_j+1
  std::vector<double> vbc;               // volume-bending coupling: compliance scaling
  bool any_sr = false, any_sb = false;
  bool even = true;                      // every rod starts on an even slot of its wavefront
  std::vector<double> bone_rest, pill_bone_w;   // bones: rest transforms, two weights per pill
  std::vector<int32_t> pill_bone;
  // bundling sections: offsets, pills, section of each entry, world rest position of each entry
  std::vector<int32_t> sec_off, sec_pill, sec_of;
  std::vector<double> sec_xr;
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

// A bone transform [A | b] (3x4 row-major): finite, and A far from singular.
bool affine_ok(const double* T) {
  double m = 0.0;
  for (int i = 0; i < 12; ++i) {
    if (!std::isfinite(T[i])) return false;
    if (i % 4 != 3) m = std::max(m, std::fabs(T[i]));
  }
  const double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                     T[2] * (T[4] * T[9] - T[5] * T[8]);
  return m > 0 && std::fabs(det) > 1e-12 * m * m * m;
}

viper_status validate(const viper_scene_desc* d) {
  if (!d) return fail(VIPER_ERR_INVALID, "desc is NULL");
  if (d->num_rods < 0) return fail(VIPER_ERR_INVALID, "num_rods < 0");
  if (d->num_rods > 0 && (!d->rod_offsets || !d->rest_pos || !d->rest_radius || !d->compliance))
    return fail(VIPER_ERR_INVALID, "rod_offsets, rest_pos, rest_radius and compliance are required");
  if (d->precision != VIPER_F32 && d->precision != VIPER_F64) return fail(VIPER_ERR_INVALID, "unknown precision");
  if (!finite_pos(d->density)) return fail(VIPER_ERR_INVALID, "density must be finite and > 0");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(d->gravity[i])) return fail(VIPER_ERR_INVALID, "gravity must be finite");
  if (d->floor_on) {
    const double* n = d->floor_normal;
    if (!std::isfinite(n[0]) || !std::isfinite(n[1]) || !std::isfinite(n[2]) || !std::isfinite(d->floor_offset) ||
        !(n[0] * n[0] + n[1] * n[1] + n[2] * n[2] > 0))
      return fail(VIPER_ERR_INVALID, "floor_normal must be finite and nonzero, floor_offset finite");
  }
  if (d->solver != 0 && d->solver != 1) return fail(VIPER_ERR_INVALID, "solver must be 0 (Gauss-Seidel) or 1 (Jacobi)");
  if (d->volume_bending && d->solver == 1)
    return fail(VIPER_ERR_INVALID, "the volume-bending coupling (volume_bending) needs the Gauss-Seidel solver");
  if (d->num_bones < 0) return fail(VIPER_ERR_INVALID, "num_bones < 0");
  if (d->num_bones > 0) {
    if (!d->bone_rest || !d->pill_bones || !d->pill_bone_weights)
      return fail(VIPER_ERR_INVALID, "bone_rest, pill_bones and pill_bone_weights are required");
    for (int b = 0; b < d->num_bones; ++b)
      if (!affine_ok(d->bone_rest + 12 * (size_t)b))
        return fail(VIPER_ERR_INVALID, "bone_rest must be finite with an invertible linear part");
  }
  if (d->num_sections < 0) return fail(VIPER_ERR_INVALID, "num_sections < 0");
  if (d->num_rods == 0) {
    if (d->num_sections > 0) return fail(VIPER_ERR_INVALID, "bundling sections need pills");
    return VIPER_OK;
  }
  if (d->rod_offsets[0] != 0) return fail(VIPER_ERR_INVALID, "rod_offsets[0] must be 0");
  for (int k = 0; k < d->num_rods; ++k) {
    int n = d->rod_offsets[k + 1] - d->rod_offsets[k];
    if (n < 2 || n > kMaxPills)
      return fail(VIPER_ERR_INVALID, "rod " + std::to_string(k) + " has " + std::to_string(n) +
                                         " pills; each rod needs 2..128 pills");
    if (d->activation && !finite_pos(d->activation[k])) return fail(VIPER_ERR_INVALID, "activation must be > 0");
    for (int t = 0; t < 4; ++t) {
      double c = d->compliance[4 * k + t];
      if (std::isnan(c) || c < 0) return fail(VIPER_ERR_INVALID, "compliance must be >= 0 or +inf");
    }
    if (d->cross_compliance && (std::isnan(d->cross_compliance[k]) || d->cross_compliance[k] < 0))
      return fail(VIPER_ERR_INVALID, "cross_compliance must be >= 0 or +inf");
    if (d->bending_compliance) {
      const double c = d->bending_compliance[k];
      if (std::isnan(c) || c < 0) return fail(VIPER_ERR_INVALID, "bending_compliance must be >= 0 or +inf");
      if (d->solver == 1 && std::isfinite(c))
        return fail(VIPER_ERR_INVALID, "surface bending (bending_compliance) needs the Gauss-Seidel solver");
    }
  }
  const int P = d->rod_offsets[d->num_rods];
  if (P > (1 << 27)) return fail(VIPER_ERR_INVALID, "too many pills");
  for (int p = 0; p < P; ++p) {
    if (!finite_pos(d->rest_radius[p])) return fail(VIPER_ERR_INVALID, "rest_radius must be finite and > 0");
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(d->rest_pos[3 * p + i])) return fail(VIPER_ERR_INVALID, "rest_pos must be finite");
  }
  for (int k = 0; k < d->num_rods; ++k)
    for (int p = d->rod_offsets[k]; p + 1 < d->rod_offsets[k + 1]; ++p) {
      double dx = d->rest_pos[3 * p + 3] - d->rest_pos[3 * p], dy = d->rest_pos[3 * p + 4] - d->rest_pos[3 * p + 1],
             dz = d->rest_pos[3 * p + 5] - d->rest_pos[3 * p + 2];
      if (!(dx * dx + dy * dy + dz * dz > 0)) return fail(VIPER_ERR_INVALID, "consecutive rest pills coincide");
    }
  if (d->num_bones > 0)
    for (int p = 0; p < P; ++p)
      for (int k = 0; k < 2; ++k) {
        const double w = d->pill_bone_weights[2 * (size_t)p + k];
        if (!std::isfinite(w) || w < 0) return fail(VIPER_ERR_INVALID, "pill_bone_weights must be finite and >= 0");
        const int b = d->pill_bones[2 * (size_t)p + k];
        if (w > 0 && (b < 0 || b >= d->num_bones)) return fail(VIPER_ERR_INVALID, "pill_bones out of range");
      }
  if (d->num_sections > 0) {
    if (!d->section_offsets || !d->section_pills)
      return fail(VIPER_ERR_INVALID, "section_offsets and section_pills are required");
    if (d->section_offsets[0] != 0) return fail(VIPER_ERR_INVALID, "section_offsets[0] must be 0");
    std::vector<uint8_t> used(P, 0);
    for (int k = 0; k < d->num_sections; ++k) {
      if (d->section_offsets[k + 1] <= d->section_offsets[k])
        return fail(VIPER_ERR_INVALID, "section " + std::to_string(k) + " is empty");
      for (int i = d->section_offsets[k]; i < d->section_offsets[k + 1]; ++i) {
        const int p = d->section_pills[i];
        if (p < 0 || p >= P) return fail(VIPER_ERR_INVALID, "section pill out of range");
        if (used[p]) return fail(VIPER_ERR_INVALID, "pill " + std::to_string(p) + " is in two sections");
        used[p] = 1;
      }
    }
  }
  return VIPER_OK;
}

int pack_waves(const viper_scene_desc* d, std::vector<int32_t>& ws, bool& even) {
  ws.clear();
  even = true;
  int start = 0, n = 0;
  for (int k = 0; k < d->num_rods; ++k) {
    int len = d->rod_offsets[k + 1] - d->rod_offsets[k];
    if (n + len > kWaveSpan) {
      ws.push_back(start);
      start = d->rod_offsets[k];
      n = 0;
    }
    if (n & 1) even = false;   // this rod starts on an odd slot of its wavefront
    n += len;
  }
  if (d->num_rods > 0) ws.push_back(start);
  ws.push_back(d->num_rods > 0 ? d->rod_offsets[d->num_rods] : 0);
  return (int)ws.size() - 1;
}

// ----------------------------------------------------------------------------- batch tables

// Per-scene item counts of every stage.
struct Counts {
  int W = 0, P = 0, E = 0, T = 0, cap = 0, S = 0, N = 0;   // ... bundling sections and entries
  bool contacts = false;
  const std::vector<int32_t>* wave_start = nullptr;      // [W+1] first pill of each wave (host)
};

const int kStageItems[TB_COUNT] = {4, 256, 28, 64, 1024, 256, 4, 256};

int stage_items(const Counts& c, int stage) {
  switch (stage) {
    case TB_WAVES: return c.W;
    case TB_CAPS: return c.contacts ? c.E : 0;
    case TB_SEARCH: return c.contacts ? c.E : 0;
    case TB_PAIRS: return c.contacts ? 2 * pair_span(c.cap) : 0;
    case TB_SCAN_T: return c.contacts ? c.T : 0;
    case TB_DET: return c.contacts ? std::max(c.P, std::max(c.T, c.E)) : 0;
    case TB_SECT: return c.S;
    case TB_SECP: return c.N;
    default: return 0;
  }
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
// Bytes of one wavefront launch record: WaveRec, then the scene's Dev, in whole cache lines.
size_t wave_rec_bytes(size_t dev_size) { return (sizeof(WaveRec) + dev_size + 63) & ~size_t(63); }

// Bytes of the device header of a batch: Dev structs, ContactDev structs, block tables.
size_t header_bytes(const std::vector<Counts>& v, size_t dev_size) {
  size_t n = align256(v.size() * dev_size) + align256(v.size() * sizeof(ContactDev));
  for (int t = 0; t < TB_COUNT; ++t) {
    size_t e = 0;
    for (const Counts& c : v) e += (size_t)((stage_items(c, t) + kStageItems[t] - 1) / kStageItems[t]);
    n += align256(e * sizeof(Blk));
  }
  size_t w = 0;
  for (const Counts& c : v) w += (size_t)c.W;
  n += align256(w * wave_rec_bytes(dev_size));
  return n;
}

// Lay the batch header out in `buf` (host image of the device bytes at `dev_base`) and
// point `b` at the device copy.
void build_header(std::vector<char>& buf, const std::vector<const void*>& devs, size_t dev_size,
                  const std::vector<ContactDev>& cds, const std::vector<Counts>& v, char* dev_base, BatchDev& b) {
  buf.assign(header_bytes(v, dev_size), 0);
  size_t off = 0;
  for (size_t i = 0; i < devs.size(); ++i) std::memcpy(buf.data() + off + i * dev_size, devs[i], dev_size);
  b.dev = dev_base + off;
  off += align256(v.size() * dev_size);
  for (size_t i = 0; i < cds.size(); ++i) std::memcpy(buf.data() + off + i * sizeof(ContactDev), &cds[i], sizeof(ContactDev));
  b.cd = (const ContactDev*)(dev_base + off);
  off += align256(v.size() * sizeof(ContactDev));
  for (int t = 0; t < TB_COUNT; ++t) {
    std::vector<Blk> tab;
    for (size_t s = 0; s < v.size(); ++s)
      for (int base = 0; base < stage_items(v[s], t); base += kStageItems[t]) tab.push_back(Blk{(int32_t)s, base});
    std::memcpy(buf.data() + off, tab.data(), tab.size() * sizeof(Blk));
    b.tab[t] = (const Blk*)(dev_base + off);
    b.nblk[t] = (int)tab.size();
    off += align256(tab.size() * sizeof(Blk));
  }
  const size_t rs = wave_rec_bytes(dev_size);
  size_t k = 0;
  for (size_t s = 0; s < v.size(); ++s) {
    const std::vector<int32_t>& ws = *v[s].wave_start;
    for (int w = 0; w < v[s].W; ++w, ++k) {
      WaveRec r{};
      r.b = WaveBlk{(int32_t)s, w, ws[w], ws[w + 1] - ws[w]};
      r.acc = s < cds.size() ? cds[s].acc : nullptr;
      r.acnt = s < cds.size() ? cds[s].acnt : nullptr;
      std::memcpy(buf.data() + off + k * rs, &r, sizeof(WaveRec));
      std::memcpy(buf.data() + off + k * rs + sizeof(WaveRec), devs[s], dev_size);
    }
  }
  b.wrec = dev_base + off;
  b.wrec_stride = (int)rs;
  b.nwaves = (int)k;
  off += align256(k * rs);
  b.nscenes = (int)v.size();
}

Offsets make_layout(const viper_scene_desc* d, int P, int W, int E, int cap) {
  const size_t ts = d->precision == VIPER_F64 ? 8 : 4;
  Layout L;
  Offsets o;
  for (auto& v : o.state) v = L.take(ts * P);
  for (auto& v : o.pill_rest) v = L.take(ts * P);
  for (auto& v : o.edge_rest) v = L.take(ts * P);
  for (int i = 0; i < 9; ++i) o.scratch[i] = L.take(ts * P);
  o.scratch[9] = L.take(ts * 12 * (size_t)P);
  o.flags = L.take(4 * (size_t)P);
  o.wave_start = L.take(4 * (size_t)(W + 1));
  o.status = L.take(4 * ST_WORDS);
  o.stage = L.take(std::max(ts * 4, (size_t)24) * (size_t)P);   // gather/scatter staging (FP64 XDET: 24 B/pill)
  o.xform = L.take(4 * 12 * (size_t)P);      // skinning transforms
  o.anchor = L.take(8 * 3 * (size_t)std::max(d->num_rods, 1));
  o.rod_of = L.take(4 * (size_t)P);
  const int NS = d->num_sections > 0 ? d->num_sections : 0, NP = NS ? d->section_offsets[NS] : 0;
  if (NS) {
    o.sec_off = L.take(4 * (size_t)(NS + 1));
    o.sec_pill = L.take(4 * (size_t)NP);
    o.sec_of = L.take(4 * (size_t)NP);
    o.sec_xr = L.take(8 * 3 * (size_t)NP);
    o.sec_q = L.take(8 * 4 * (size_t)NS);
    o.sec_fit = L.take(8 * (size_t)kSecFit * NS);
  }
  if (d->num_bones > 0) {
    o.bone_prev = L.take(8 * 12 * (size_t)d->num_bones);
    o.bone_delta = L.take(8 * 12 * (size_t)d->num_bones);
    o.pill_bone = L.take(4 * 2 * (size_t)P);
    o.pill_bone_w = L.take(8 * 2 * (size_t)P);
  }
  Counts c;
  c.W = W; c.P = P; c.E = E; c.T = contact_table_size(E); c.cap = cap * E; c.contacts = d->collisions != 0;
  c.S = NS; c.N = NP;
  o.header = L.take(header_bytes(std::vector<Counts>{c}, d->precision == VIPER_F64 ? sizeof(Dev<double>) : sizeof(Dev<float>)));
  o.contact = contact_layout(L.off, d->collisions != 0, P, E, cap, d->precision == VIPER_F64);
  L.off = o.contact.end;
  o.total = L.off;
  return o;
}

// Shortest-arc rotation taking unit a onto unit b (x, y, z, w).
void shortest_arc(const double a[3], const double b[3], double q[4]) {
  double c = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
  if (c < -1.0 + 1e-12) {
    double ax[3];
    if (std::fabs(a[0]) < 0.9) { ax[0] = 0; ax[1] = a[2]; ax[2] = -a[1]; }   // a x e_x
    else { ax[0] = -a[2]; ax[1] = 0; ax[2] = a[0]; }                          // a x e_y
    double n = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    q[0] = ax[0] / n; q[1] = ax[1] / n; q[2] = ax[2] / n; q[3] = 0;
    return;
  }
  double x = a[1] * b[2] - a[2] * b[1], y = a[2] * b[0] - a[0] * b[2], z = a[0] * b[1] - a[1] * b[0], w = 1.0 + c;
  double n = std::sqrt(x * x + y * y + z * z + w * w);
  q[0] = x / n; q[1] = y / n; q[2] = z / n; q[3] = w / n;
}

void qmul(const double a[4], const double b[4], double r[4]) {
  r[0] = a[3] * b[0] + a[0] * b[3] + a[1] * b[2] - a[2] * b[1];
  r[1] = a[3] * b[1] - a[0] * b[2] + a[1] * b[3] + a[2] * b[0];
  r[2] = a[3] * b[2] + a[0] * b[1] - a[1] * b[0] + a[2] * b[3];
  r[3] = a[3] * b[3] - a[0] * b[0] - a[1] * b[1] - a[2] * b[2];
}

void build_host(const viper_scene_desc* d, Host& H) {
  H.R = d->num_rods;
  H.off.assign(d->rod_offsets, d->rod_offsets + H.R + 1);
  H.P = H.off[H.R];
  const int P = H.P;
  if (d->num_bones > 0) {
    H.bone_rest.assign(d->bone_rest, d->bone_rest + 12 * (size_t)d->num_bones);
    H.pill_bone.assign(d->pill_bones, d->pill_bones + 2 * (size_t)P);
    H.pill_bone_w.assign(d->pill_bone_weights, d->pill_bone_weights + 2 * (size_t)P);
  }
  H.group.resize(H.R);
  for (int k = 0; k < H.R; ++k) H.group[k] = d->group ? d->group[k] : k;
  H.W = pack_waves(d, H.wave_start, H.even);
  H.x.assign(d->rest_pos, d->rest_pos + 3 * (size_t)P);
  if (d->num_sections > 0) {
    const int NS = d->num_sections, NP = d->section_offsets[NS];
    H.sec_off.assign(d->section_offsets, d->section_offsets + NS + 1);
    H.sec_pill.assign(d->section_pills, d->section_pills + NP);
    H.sec_of.resize(NP);
    H.sec_xr.resize(3 * (size_t)NP);
    for (int k = 0; k < NS; ++k)
      for (int i = H.sec_off[k]; i < H.sec_off[k + 1]; ++i) {
        H.sec_of[i] = k;
        for (int t = 0; t < 3; ++t) H.sec_xr[3 * (size_t)i + t] = H.x[3 * (size_t)H.sec_pill[i] + t];
      }
  }
  H.anchor.assign(3 * (size_t)H.R, 0.0);
  H.xloc.assign(3 * (size_t)P, 0.0);
  H.rod_of.assign(P, 0);
  for (int k = 0; k < H.R; ++k) {
    const int a = H.off[k];
    for (int i = 0; i < 3; ++i) H.anchor[3 * k + i] = H.x[3 * (size_t)a + i];
    for (int p = a; p < H.off[k + 1]; ++p) {
      H.rod_of[p] = k;
      for (int i = 0; i < 3; ++i) H.xloc[3 * (size_t)p + i] = H.x[3 * (size_t)p + i] - H.anchor[3 * k + i];
    }
  }
  H.rbar.assign(d->rest_radius, d->rest_radius + P);
  H.flags.assign(P, 0);
  std::vector<double> M(P, 0.0), Ms(P, 0.0);
  H.ilb.assign(P, 0); H.il0.assign(P, 0); H.cbt.assign(P, 0); H.inert.assign(P, 0);
  for (int i = 0; i < 3; ++i) { H.db[i].assign(P, 0); H.mr[i].assign(P, 0); }
  for (int i = 0; i < 4; ++i) { H.cs[i].assign(P, 0); H.qr[i].assign(P, 0); }
  H.cs[4].assign(P, 0);
  H.sbc.assign(P, 0); H.sbg0.assign(P, 0); H.sbg2.assign(P, 0);
  H.vbc.assign(P, 0);
  H.any_sr = false;
  H.any_sb = false;
  for (int p = 0; p < P; ++p) H.qr[3][p] = 1.0;
  const double rho = d->density;
  H.E = 0;
  H.proj_per_iter = 0;
  std::vector<double> l0(P, 0.0);
  for (int k = 0; k < H.R; ++k) {
    const int a = H.off[k], b = H.off[k + 1];
    const double act = d->activation ? d->activation[k] : 1.0;
    bool en[4];
    for (int t = 0; t < 4; ++t) en[t] = std::isfinite(d->compliance[4 * k + t]);
    const bool sr = d->cross_compliance && std::isfinite(d->cross_compliance[k]);
    const bool sb = d->bending_compliance && std::isfinite(d->bending_compliance[k]);
    H.any_sr = H.any_sr || sr;
    H.any_sb = H.any_sb || sb;
    const bool vb = d->volume_bending != 0 && en[1];
    uint32_t ef = (en[0] ? F_SS : 0u) | (en[1] ? F_VOL : 0u) | (en[2] ? F_SG : 0u) | (en[3] ? F_BTEN : 0u) |
                  (sr ? F_SR : 0u) | (sb ? F_SB : 0u) | (vb ? F_VB : 0u);
    double tprev[3] = {0, 0, 1}, qcur[4] = {0, 0, 0, 1};
    for (int p = a; p < b; ++p) {
      uint32_t f = F_VALID | ef;
      if (p == a) f |= F_FIRST;
      if ((p - a) & 1) f |= F_ODD;
      if ((p - a) % 3 == 1) f |= F_M3A;
      if ((p - a) % 3 == 2) f |= F_M3B;
      if (p + 1 < b) f |= F_EDGE;
      if (p + 2 < b) f |= F_BT;
      H.flags[p] = f;
    }
    for (int p = a; p + 1 < b; ++p) {
      double e[3] = {H.x[3 * p + 3] - H.x[3 * p], H.x[3 * p + 4] - H.x[3 * p + 1], H.x[3 * p + 5] - H.x[3 * p + 2]};
      double len = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
      double t[3] = {e[0] / len, e[1] / len, e[2] / len};
      double sa[4], qn[4];
      shortest_arc(tprev, t, sa);
      qmul(sa, qcur, qn);
      double n = std::sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
      for (int i = 0; i < 4; ++i) { qcur[i] = qn[i] / n; H.qr[i][p] = qcur[i]; }
      for (int i = 0; i < 3; ++i) { tprev[i] = t[i]; H.mr[i][p] = 0.5 * (H.xloc[3 * p + i] + H.xloc[3 * p + 3 + i]); }
      l0[p] = len;
      H.il0[p] = 1.0 / len;
      H.ilb[p] = 1.0 / (act * len);
      const double rm = 0.5 * (H.rbar[p] + H.rbar[p + 1]);
      const double r2 = rm * rm, r4 = r2 * r2;
      const double Me = rho * kPi * r2 * len, Mse = rho * kPi * r4 * len / 2.0;
      M[p] += 0.5 * Me; M[p + 1] += 0.5 * Me;
      Ms[p] += 0.5 * Mse; Ms[p + 1] += 0.5 * Mse;
      H.inert[p] = rho * kPi * r4 * len;
      if (en[0]) H.cs[0][p] = d->compliance[4 * k + 0] / (kPi * r2 * len);
      if (en[1]) H.cs[1][p] = d->compliance[4 * k + 1] / (kPi * r2 * len);
      if (en[2]) H.cs[2][p] = d->compliance[4 * k + 2] / (kPi * r4 / 2.0 * len);
      if (sr) H.cs[4][p] = d->cross_compliance[k] / (kPi * r2 * len);
      H.E += 1;
      H.proj_per_iter += (int64_t)en[0] + en[1] + en[2] + sr;
    }
    for (int p = a; p + 2 < b; ++p) {
      const double rv = H.rbar[p + 1], r4 = rv * rv * rv * rv;
      const double lv = 0.5 * (l0[p] + l0[p + 1]);
      if (en[3]) H.cs[3][p] = d->compliance[4 * k + 3] / (kPi * r4 / 4.0 * lv);
      if (vb) {
        H.vbc[p] = d->compliance[4 * k + 1] / (kPi * r4 / 2.0 * lv);
        H.proj_per_iter += 1;
      }
      if (sb) {
        H.sbc[p] = d->bending_compliance[k] / (kPi * r4 / 4.0 * lv);
        H.sbg0[p] = 1.0 / (l0[p] * lv);
        H.sbg2[p] = 1.0 / (l0[p + 1] * lv);
        H.proj_per_iter += 1;
      }
      const double c = 4.0 / (l0[p] + l0[p + 1]);
      H.cbt[p] = c;
      const double qa[4] = {-H.qr[0][p], -H.qr[1][p], -H.qr[2][p], H.qr[3][p]};
      const double qb[4] = {H.qr[0][p + 1], H.qr[1][p + 1], H.qr[2][p + 1], H.qr[3][p + 1]};
      double r[4];
      qmul(qa, qb, r);
      const double sg = r[3] < 0 ? -1.0 : 1.0;
      for (int i = 0; i < 3; ++i) H.db[i][p] = c * sg * r[i];
      H.proj_per_iter += (int64_t)en[3];
    }
  }
  H.winv.assign(P, 0); H.wsinv.assign(P, 0);
  for (int p = 0; p < P; ++p) {
    bool pin = d->pinned && d->pinned[p];
    H.winv[p] = pin ? 0.0 : 1.0 / M[p];
    H.wsinv[p] = 1.0 / Ms[p];
  }
}

template <class T>
std::vector<T> cvt(const std::vector<double>& v) {
  std::vector<T> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (T)v[i];
  return o;
}

}  // namespace

// ----------------------------------------------------------------------------- scene

struct Skin {
  int V;
  const float* rest_v;
  const int32_t* caps;
  const float* w;
};

struct viper_scene_s {
  int precision = 0;
  int collisions = 0;
  int nsec = 0, nsecp = 0;    // bundling sections and their entries
  int floor_on = 0;           // half-plane floor (unit normal, offset)
  int jacobi = 0;             // rod constraints by Jacobi with averaging
  int cross_stretch = 0;      // some rod has the cross-section stretch constraint
  int nbones = 0;             // kinematic bones
  int surface_bending = 0;    // some rod has the surface-bending constraint
  int volume_bending = 0;     // the volume-bending coupling is on
  int even = 0;               // every rod starts on an even slot of its wavefront
  double floor_n[3] = {0.0, 0.0, 0.0}, floor_d = 0.0;
  int cap = 16;
  int R = 0, P = 0, W = 0, E = 0;
  int64_t proj_per_iter = 0;
  char* ws = nullptr;
  size_t bytes = 0;
  Offsets o;
  Dev<float> df;
  Dev<double> dd;
  ContactDev cd;
  BatchDev batch;             // this scene as a batch of one
  std::vector<char> header;   // host image of the batch header
  std::vector<Skin> skins;
  std::vector<int32_t> off;  // rod offsets (host copy)
  std::vector<int32_t> wave_start;   // first pill of each wave (host copy)
  double density = 1000.0;
  // GRAPH mode: one captured frame, valid for (h, substeps, iterations) of its capture
  hipStream_t capture = nullptr;
  hipGraphExec_t graph = nullptr;
  double graph_h = 0.0;
  int graph_sub = 0, graph_iters = 0;
  ~viper_scene_s() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (capture) (void)hipStreamDestroy(capture);
  }
};

namespace {

template <class T>
void fill_dev(viper_scene_s* S, Dev<T>& d) {
  char* b = S->ws;
  auto P_ = [&](size_t off) { return (T*)(b + off); };
  d.P = S->P;
  d.W = S->W;
  d.wave_start = (const int32_t*)(b + S->o.wave_start);
  d.flags = (const uint32_t*)(b + S->o.flags);
  T** st[15] = {&d.px, &d.py, &d.pz, &d.vx, &d.vy, &d.vz, &d.s, &d.sd, &d.qx, &d.qy, &d.qz, &d.qw, &d.ox, &d.oy, &d.oz};
  for (int i = 0; i < 15; ++i) *st[i] = P_(S->o.state[i]);
  const T** pr[3] = {&d.winv, &d.wsinv, &d.rbar};
  for (int i = 0; i < 3; ++i) *pr[i] = P_(S->o.pill_rest[i]);
  const T** er[23] = {&d.ilb, &d.il0, &d.cbt, &d.inert, &d.dbx, &d.dby, &d.dbz, &d.css, &d.cvol,
                      &d.csg, &d.cbtc, &d.qrx, &d.qry, &d.qrz, &d.qrw, &d.mrx, &d.mry, &d.mrz, &d.csr,
                      &d.csb, &d.sbg0, &d.sbg2, &d.cvb};
  for (int i = 0; i < 23; ++i) *er[i] = P_(S->o.edge_rest[i]);
  T** sc[9] = {&d.xpx, &d.xpy, &d.xpz, &d.spv, &d.qpx, &d.qpy, &d.qpz, &d.qpw, &d.i1};
  for (int i = 0; i < 9; ++i) *sc[i] = P_(S->o.scratch[i]);
  d.lam = P_(S->o.scratch[9]);
  d.status = (int32_t*)(b + S->o.status);
  d.anchor = (const double*)(b + S->o.anchor);
  d.rod_of = (const int32_t*)(b + S->o.rod_of);
  d.nsec = S->nsec;
  d.nsecp = S->nsecp;
  d.sec_off = S->nsec ? (const int32_t*)(b + S->o.sec_off) : nullptr;
  d.sec_pill = S->nsec ? (const int32_t*)(b + S->o.sec_pill) : nullptr;
  d.sec_of = S->nsec ? (const int32_t*)(b + S->o.sec_of) : nullptr;
  d.sec_xr = S->nsec ? (const double*)(b + S->o.sec_xr) : nullptr;
  d.sec_q = S->nsec ? (double*)(b + S->o.sec_q) : nullptr;
  d.sec_fit = S->nsec ? (double*)(b + S->o.sec_fit) : nullptr;
  d.floor_on = S->floor_on;
  d.fnx = S->floor_n[0]; d.fny = S->floor_n[1]; d.fnz = S->floor_n[2]; d.fd = S->floor_d;
  d.jacobi = S->jacobi;
}

template <class T>
viper_status upload(viper_scene_s* S, const Host& H, hipStream_t st) {
  char* b = S->ws;
  const int P = H.P;
  // converted host copies stay alive until the stream has drained (end of this function)
  std::vector<std::vector<T>> keep;
  keep.reserve(64);
  auto put = [&](size_t off, const std::vector<double>& v) -> hipError_t {
    keep.push_back(cvt<T>(v));
    const std::vector<T>& t = keep.back();
    return hipMemcpyAsync(b + off, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice, st);
  };
  std::vector<double> comp[3];
  for (int i = 0; i < 3; ++i) {
    comp[i].resize(P);
    for (int p = 0; p < P; ++p) comp[i][p] = H.xloc[3 * (size_t)p + i];
  }
  std::vector<double> zero(P, 0.0), one(P, 1.0);
  for (int i = 0; i < 3; ++i) HIP_TRY(put(S->o.state[i], comp[i]));
  for (int i = 3; i < 6; ++i) HIP_TRY(put(S->o.state[i], zero));
  HIP_TRY(put(S->o.state[6], one));
  HIP_TRY(put(S->o.state[7], zero));
  for (int i = 0; i < 4; ++i) HIP_TRY(put(S->o.state[8 + i], H.qr[i]));
  for (int i = 12; i < 15; ++i) HIP_TRY(put(S->o.state[i], zero));
  HIP_TRY(put(S->o.pill_rest[0], H.winv));
  HIP_TRY(put(S->o.pill_rest[1], H.wsinv));
  HIP_TRY(put(S->o.pill_rest[2], H.rbar));
  const std::vector<double>* er[23] = {&H.ilb, &H.il0, &H.cbt, &H.inert, &H.db[0], &H.db[1], &H.db[2], &H.cs[0],
                                       &H.cs[1], &H.cs[2], &H.cs[3], &H.qr[0], &H.qr[1], &H.qr[2], &H.qr[3],
                                       &H.mr[0], &H.mr[1], &H.mr[2], &H.cs[4], &H.sbc, &H.sbg0, &H.sbg2, &H.vbc};
  for (int i = 0; i < 23; ++i) HIP_TRY(put(S->o.edge_rest[i], *er[i]));
  HIP_TRY(hipMemcpyAsync(b + S->o.flags, H.flags.data(), 4 * (size_t)P, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(b + S->o.anchor, H.anchor.data(), 8 * H.anchor.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(b + S->o.rod_of, H.rod_of.data(), 4 * (size_t)P, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(b + S->o.wave_start, H.wave_start.data(), 4 * H.wave_start.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(b + S->o.status, 0, 4 * ST_WORDS, st));
  if (S->nsec) {
    std::vector<double> q0(4 * (size_t)S->nsec, 0.0);
    for (int k = 0; k < S->nsec; ++k) q0[4 * (size_t)k + 3] = 1.0;     // first extraction starts at the identity
    HIP_TRY(hipMemcpyAsync(b + S->o.sec_off, H.sec_off.data(), 4 * H.sec_off.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b + S->o.sec_pill, H.sec_pill.data(), 4 * H.sec_pill.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b + S->o.sec_of, H.sec_of.data(), 4 * H.sec_of.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b + S->o.sec_xr, H.sec_xr.data(), 8 * H.sec_xr.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b + S->o.sec_q, q0.data(), 8 * q0.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // q0 dies with this block
  }
  if (S->nbones) {
    HIP_TRY(hipMemcpyAsync(b + S->o.bone_prev, H.bone_rest.data(), 8 * H.bone_rest.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b + S->o.pill_bone, H.pill_bone.data(), 4 * H.pill_bone.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b + S->o.pill_bone_w, H.pill_bone_w.data(), 8 * H.pill_bone_w.size(), hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipStreamSynchronize(st));   // the host staging vectors die with this frame
  return VIPER_OK;
}

template <class T> Dev<T>& dev(viper_scene_s* S);
template <> Dev<float>& dev<float>(viper_scene_s* S) { return S->df; }
template <> Dev<double>& dev<double>(viper_scene_s* S) { return S->dd; }

// One frame of a batch (all scenes share precision, dt, substeps and iterations).
template <class T>
// `iteration_only`: the batch has collisions, bundling sections or a floor, whose projections
// need a grid-wide step between iterations (the single-launch modes cannot run them).
viper_status batch_step(const BatchDev& b, bool collisions, bool iteration_only, double dt, int sub, int iters, int mode,
                        hipStream_t st) {
  const double h = dt / sub;
  const bool bundled = b.nblk[TB_SECT] > 0;
  iteration_only = iteration_only || collisions || bundled;
  if (mode == VIPER_MODE_AUTO) mode = iteration_only ? VIPER_MODE_ITERATION : VIPER_MODE_FRAME;
  if (iteration_only && mode != VIPER_MODE_ITERATION)
    return fail(VIPER_ERR_INVALID,
                "scenes with collisions, bundling sections, a floor or the Jacobi solver step in VIPER_MODE_ITERATION");
  if (mode == VIPER_MODE_FRAME) {
    HIP_TRY(launch_rod_frame<T>(b, sub, h, iters, st));
  } else if (mode == VIPER_MODE_SUBSTEP) {
    for (int i = 0; i < sub; ++i) HIP_TRY(launch_rod_frame<T>(b, 1, h, iters, st));
  } else if (mode == VIPER_MODE_ITERATION) {
    const ContactDev* cd = collisions ? b.cd : nullptr;
    for (int i = 0; i < sub; ++i) {
      // the first substep's prediction; a later substep's prediction and first iteration come
      // with the previous substep's velocity update
      if (i == 0) HIP_TRY(launch_predict<T>(b, h, cd, st));
      if (collisions) HIP_TRY(launch_contact_detect<T>(b, st));
      for (int it = 0; it < iters; ++it) {
        if (i == 0 || it > 0) HIP_TRY(launch_rod_iteration<T>(b, h, cd, st));
        if (collisions) HIP_TRY(launch_contact_project<T>(b, st));
      }
      if (bundled) {      // shape matching of the cross-sections (Sec. 7.3) after the iterations
        if (collisions) HIP_TRY(launch_contact_flush<T>(b, st));
        HIP_TRY(launch_bundle<T>(b, st));
      }
      HIP_TRY(launch_velocity<T>(b, h, cd, i + 1 < sub ? (iters > 0 ? 2 : 1) : 0, st));
    }
  } else {
    return fail(VIPER_ERR_INVALID, "unknown mode");
  }
  return VIPER_OK;
}

// Capture one ITERATION-mode frame of the scene into a graph (on a private stream, so
// that any caller stream, the legacy default stream included, can replay it).
template <class T>
viper_status capture_frame(viper_scene_s* S, double dt, int sub, int iters) {
  if (S->graph) {
    HIP_TRY(hipGraphExecDestroy(S->graph));
    S->graph = nullptr;
  }
  if (!S->capture) HIP_TRY(hipStreamCreateWithFlags(&S->capture, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(S->capture, hipStreamCaptureModeThreadLocal));
  viper_status r = batch_step<T>(S->batch, S->collisions != 0, S->floor_on || S->jacobi, dt, sub, iters,
                                 VIPER_MODE_ITERATION, S->capture);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(S->capture, &g);
  if (r != VIPER_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) return fail(VIPER_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&S->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    S->graph = nullptr;
    return fail(VIPER_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  S->graph_h = dt / sub;
  S->graph_sub = sub;
  S->graph_iters = iters;
  return VIPER_OK;
}

template <class T>
viper_status step_t(viper_scene_s* S, double dt, int sub, int iters, int mode, hipStream_t st) {
  if (mode == VIPER_MODE_AUTO && (S->collisions || S->nsec || S->floor_on || S->jacobi)) mode = VIPER_MODE_GRAPH;
  if (mode != VIPER_MODE_GRAPH)
    return batch_step<T>(S->batch, S->collisions != 0, S->floor_on || S->jacobi, dt, sub, iters, mode, st);
  if (!S->graph || S->graph_h != dt / sub || S->graph_sub != sub || S->graph_iters != iters) {
    viper_status r = capture_frame<T>(S, dt, sub, iters);
    if (r != VIPER_OK) return r;
  }
  HIP_TRY(hipGraphLaunch(S->graph, st));
  return VIPER_OK;
}

// Some optional constraint term is on (the rod kernels' instantiation with them compiled in).
bool scene_extras(const viper_scene_s* S) { return S->cross_stretch || S->surface_bending || S->volume_bending; }

Counts scene_counts(const viper_scene_s* S) {
  Counts c;
  c.W = S->W; c.P = S->P; c.E = S->E; c.T = S->collisions ? S->cd.T : contact_table_size(S->E);
  c.cap = S->collisions ? S->cd.cap : S->cap * S->E;
  c.contacts = S->collisions != 0;
  c.S = S->nsec; c.N = S->nsecp;
  c.wave_start = &S->wave_start;
  return c;
}

}  // namespace

// ============================================================================= C ABI

extern "C" {

const char* viper_last_error(void) { return g_err.c_str(); }

viper_status viper_scene_footprint(const viper_scene_desc* desc, size_t* bytes) {
  viper_status s = validate(desc);
  if (s != VIPER_OK) return s;
  if (!bytes) return fail(VIPER_ERR_INVALID, "bytes is NULL");
  std::vector<int32_t> ws;
  bool even;
  int W = pack_waves(desc, ws, even);
  int P = desc->num_rods ? desc->rod_offsets[desc->num_rods] : 0;
  int E = P - desc->num_rods;
  int cap = desc->contact_capacity_per_capsule > 0 ? desc->contact_capacity_per_capsule : 16;
  *bytes = make_layout(desc, P, W, E, cap).total;
  return VIPER_OK;
}

viper_status viper_create_scene(const viper_scene_desc* desc, void* workspace, size_t bytes, void* stream,
                                viper_scene* out) {
  viper_status s = validate(desc);
  if (s != VIPER_OK) return s;
  if (!out) return fail(VIPER_ERR_INVALID, "out is NULL");
  if (!workspace) return fail(VIPER_ERR_INVALID, "workspace is NULL");
  if (((uintptr_t)workspace) & 255) return fail(VIPER_ERR_INVALID, "workspace must be 256-byte aligned");
  Host H;
  build_host(desc, H);
  int cap = desc->contact_capacity_per_capsule > 0 ? desc->contact_capacity_per_capsule : 16;
  Offsets o = make_layout(desc, H.P, H.W, H.E, cap);
  if (bytes < o.total)
    return fail(VIPER_ERR_NO_CAPACITY, "workspace too small: need " + std::to_string(o.total) + " bytes");
  viper_scene_s* S = new viper_scene_s();
  S->precision = desc->precision;
  S->collisions = desc->collisions != 0;
  S->nsec = desc->num_sections > 0 ? desc->num_sections : 0;
  S->nsecp = S->nsec ? desc->section_offsets[S->nsec] : 0;
  S->jacobi = desc->solver == 1;
  S->cross_stretch = H.any_sr ? 1 : 0;
  S->surface_bending = H.any_sb ? 1 : 0;
  S->volume_bending = desc->volume_bending != 0;
  S->even = H.even ? 1 : 0;
  S->nbones = desc->num_bones > 0 ? desc->num_bones : 0;
  if (desc->floor_on) {
    const double* n = desc->floor_normal;
    const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    S->floor_on = 1;
    for (int i = 0; i < 3; ++i) S->floor_n[i] = n[i] / l;
    S->floor_d = desc->floor_offset / l;
  }
  S->cap = cap;
  S->R = H.R; S->P = H.P; S->W = H.W; S->E = H.E;
  S->proj_per_iter = H.proj_per_iter;
  S->ws = (char*)workspace;
  S->bytes = bytes;
  S->o = o;
  S->off = H.off;
  S->wave_start = H.wave_start;
  S->density = desc->density;
  hipStream_t st = (hipStream_t)stream;
  viper_status r;
  if (S->precision == VIPER_F64) {
    fill_dev(S, S->dd);
    S->dd.gx = desc->gravity[0]; S->dd.gy = desc->gravity[1]; S->dd.gz = desc->gravity[2];
    r = upload<double>(S, H, st);
  } else {
    fill_dev(S, S->df);
    S->df.gx = (float)desc->gravity[0]; S->df.gy = (float)desc->gravity[1]; S->df.gz = (float)desc->gravity[2];
    r = upload<float>(S, H, st);
  }
  if (r == VIPER_OK) r = contact_init(S->cd, S->ws, o.contact, desc, H.off, H.group, (int32_t*)(S->ws + o.status), st);
  if (r == VIPER_OK) {
    const void* dv = S->precision == VIPER_F64 ? (const void*)&S->dd : (const void*)&S->df;
    const size_t dsz = S->precision == VIPER_F64 ? sizeof(Dev<double>) : sizeof(Dev<float>);
    build_header(S->header, std::vector<const void*>{dv}, dsz, std::vector<ContactDev>{S->cd},
                 std::vector<Counts>{scene_counts(S)}, S->ws + o.header, S->batch);
    S->batch.extras = scene_extras(S);
    S->batch.even = S->even != 0;
    if (hipMemcpyAsync(S->ws + o.header, S->header.data(), S->header.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      r = fail(VIPER_ERR_DEVICE, "header upload failed");
  }
  if (r != VIPER_OK) {
    delete S;
    return r;
  }
  *out = S;
  return VIPER_OK;
}

viper_status viper_step_ex(viper_scene S, double dt, int32_t substeps, int32_t iterations, int32_t mode, void* stream) {
  if (!S) return fail(VIPER_ERR_INVALID, "scene is NULL");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(VIPER_ERR_INVALID, "dt must be finite and > 0");
  if (substeps < 1 || iterations < 0) return fail(VIPER_ERR_INVALID, "substeps >= 1 and iterations >= 0 required");
  hipStream_t st = (hipStream_t)stream;
  return S->precision == VIPER_F64 ? step_t<double>(S, dt, substeps, iterations, mode, st)
                                   : step_t<float>(S, dt, substeps, iterations, mode, st);
}

viper_status viper_step(viper_scene S, double dt, int32_t substeps, int32_t iterations, void* stream) {
  return viper_step_ex(S, dt, substeps, iterations, VIPER_MODE_AUTO, stream);
}

static int field_width(int which) {
  switch (which) {
    case VIPER_X: case VIPER_V: case VIPER_OMEGA: case VIPER_XDET: case VIPER_XLOCAL: return 3;
    case VIPER_Q: return 4;
    case VIPER_S: case VIPER_SDOT: case VIPER_RADIUS: case VIPER_SDET: return 1;
    default: return 0;
  }
}

viper_status viper_get_state(viper_scene S, int32_t which, void* dst, void* stream) {
  if (!S || !dst) return fail(VIPER_ERR_INVALID, "scene and dst are required");
  int wdt = field_width(which);
  if (!wdt) return fail(VIPER_ERR_INVALID, "unknown field");
  hipStream_t st = (hipStream_t)stream;
  const size_t ts = S->precision == VIPER_F64 ? 8 : 4;
  void* stage = S->ws + S->o.stage;
  if (which == VIPER_XDET || which == VIPER_SDET) {
    if (!S->collisions) return fail(VIPER_ERR_INVALID, "XDET/SDET exist only for scenes with collisions");
    HIP_TRY(contact_copy_det(S->cd, which == VIPER_XDET, stage, S->P, ts, st));
  } else if (S->precision == VIPER_F64) {
    HIP_TRY(launch_gather_field<double>(S->dd, which, (double*)stage, st));
  } else {
    HIP_TRY(launch_gather_field<float>(S->df, which, (float*)stage, st));
  }
  const size_t es = (which == VIPER_XDET) ? 8 : ts;   // XDET is FP64 in both precisions
  HIP_TRY(hipMemcpyAsync(dst, stage, es * wdt * (size_t)S->P, hipMemcpyDefault, st));
  return VIPER_OK;
}

viper_status viper_set_state(viper_scene S, int32_t which, const void* src, void* stream) {
  if (!S || !src) return fail(VIPER_ERR_INVALID, "scene and src are required");
  int wdt = field_width(which);
  if (!wdt || which == VIPER_RADIUS || which == VIPER_XDET || which == VIPER_SDET)
    return fail(VIPER_ERR_INVALID, "field is not writable");
  hipStream_t st = (hipStream_t)stream;
  const size_t ts = S->precision == VIPER_F64 ? 8 : 4;
  void* stage = S->ws + S->o.stage;
  HIP_TRY(hipMemcpyAsync(stage, src, ts * wdt * (size_t)S->P, hipMemcpyDefault, st));
  if (S->precision == VIPER_F64) HIP_TRY(launch_scatter_field<double>(S->dd, which, (const double*)stage, st));
  else HIP_TRY(launch_scatter_field<float>(S->df, which, (const float*)stage, st));
  return VIPER_OK;
}

viper_status viper_get_contacts(viper_scene S, int32_t* pairs, int32_t cap, int32_t* n, void* stream) {
  if (!S || !n) return fail(VIPER_ERR_INVALID, "scene and n are required");
  if (!S->collisions) { *n = 0; return VIPER_OK; }
  return contact_get_pairs(S->cd, pairs, cap, n, (hipStream_t)stream);
}

viper_status viper_create_skin(viper_scene S, int32_t V, const float* rest_v, const int32_t* caps, const float* w,
                               void* stream, int32_t* skin_id) {
  if (!S || !skin_id || V < 0) return fail(VIPER_ERR_INVALID, "scene, skin_id and V >= 0 are required");
  if (V > 0 && (!rest_v || !caps || !w)) return fail(VIPER_ERR_INVALID, "rest_v, caps and w are required");
  if ((((uintptr_t)caps) & 15) || (((uintptr_t)w) & 15)) return fail(VIPER_ERR_INVALID, "caps and w must be 16-byte aligned");
  if (V > 0) {
    std::vector<int32_t> hc(4 * (size_t)V);
    HIP_TRY(hipMemcpyAsync(hc.data(), caps, hc.size() * 4, hipMemcpyDefault, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    std::vector<uint8_t> is_cap(S->P, 0);
    for (int k = 0; k < S->R; ++k)
      for (int p = S->off[k]; p + 1 < S->off[k + 1]; ++p) is_cap[p] = 1;
    for (size_t i = 0; i < hc.size(); ++i)
      if (hc[i] < 0 || hc[i] >= S->P || !is_cap[hc[i]])
        return fail(VIPER_ERR_INVALID, "skin influence " + std::to_string(i) + " is not a capsule id");
  }
  S->skins.push_back(Skin{V, rest_v, caps, w});
  *skin_id = (int32_t)S->skins.size() - 1;
  return VIPER_OK;
}

viper_status viper_skin(viper_scene S, int32_t skin_id, float* out, void* stream) {
  if (!S || skin_id < 0 || skin_id >= (int32_t)S->skins.size()) return fail(VIPER_ERR_INVALID, "bad skin id");
  const Skin& k = S->skins[skin_id];
  if (k.V > 0 && !out) return fail(VIPER_ERR_INVALID, "out is NULL");
  float* xf = (float*)(S->ws + S->o.xform);
  hipStream_t st = (hipStream_t)stream;
  if (S->precision == VIPER_F64) HIP_TRY(launch_skin<double>(S->dd, k.V, k.rest_v, k.caps, k.w, out, xf, st));
  else HIP_TRY(launch_skin<float>(S->df, k.V, k.rest_v, k.caps, k.w, out, xf, st));
  return VIPER_OK;
}

viper_status viper_skin_weights(viper_scene S, int32_t V, const float* rest_v, int32_t* caps, float* w, void* stream) {
  if (!S || V < 0) return fail(VIPER_ERR_INVALID, "scene and V >= 0 are required");
  if (V > 0 && (!rest_v || !caps || !w)) return fail(VIPER_ERR_INVALID, "rest_v, caps and w are required");
  if (S->E == 0 && V > 0) return fail(VIPER_ERR_INVALID, "the scene has no capsules");
  hipStream_t st = (hipStream_t)stream;
  if (S->precision == VIPER_F64) HIP_TRY(launch_skin_weights<double>(S->dd, V, rest_v, caps, w, st));
  else HIP_TRY(launch_skin_weights<float>(S->df, V, rest_v, caps, w, st));
  return VIPER_OK;
}

}  // extern "C"

namespace {

// Undirected edges of the triangles as a CSR graph: neighbours of each vertex ascending, no
// repeats, no self loops.  False if a vertex index is out of range.
bool mesh_graph(int V, int nf, const int32_t* tris, std::vector<int32_t>& off, std::vector<int32_t>& nbr) {
  std::vector<std::pair<int32_t, int32_t>> e;
  e.reserve(6 * (size_t)nf);
  for (int f = 0; f < nf; ++f)
    for (int a = 0; a < 3; ++a) {
      const int32_t p = tris[3 * (size_t)f + a], q = tris[3 * (size_t)f + (a + 1) % 3];
      if (p < 0 || p >= V || q < 0 || q >= V) return false;
      if (p == q) continue;
      e.push_back({p, q});
      e.push_back({q, p});
    }
  std::sort(e.begin(), e.end());
  e.erase(std::unique(e.begin(), e.end()), e.end());
  off.assign((size_t)V + 1, 0);
  nbr.resize(e.size());
  for (size_t k = 0; k < e.size(); ++k) {
    ++off[(size_t)e[k].first + 1];
    nbr[k] = e[k].second;
  }
  for (int i = 0; i < V; ++i) off[i + 1] += off[i];
  return true;
}

}  // namespace

extern "C" {

viper_status viper_skin_fair_work_bytes(int32_t V, int32_t nf, const int32_t* tris, size_t* bytes) {
  if (V < 0 || nf < 0 || !bytes || (nf > 0 && !tris)) return fail(VIPER_ERR_INVALID, "V, nf >= 0, tris and bytes required");
  std::vector<int32_t> off, nbr;
  if (!mesh_graph(V, nf, tris, off, nbr)) return fail(VIPER_ERR_INVALID, "a triangle references a vertex outside [0, V)");
  *bytes = skin_fair_work_bytes(V, (int64_t)nbr.size());
  return VIPER_OK;
}

viper_status viper_skin_weights_faired(viper_scene S, int32_t V, const float* rest_v, int32_t nf, const int32_t* tris,
                                       int32_t iterations, double lambda, void* work, size_t work_bytes, int32_t* caps,
                                       float* w, void* stream) {
  if (!S || V < 0 || nf < 0) return fail(VIPER_ERR_INVALID, "scene, V >= 0 and nf >= 0 are required");
  if (V > 0 && (!rest_v || !caps || !w || !work)) return fail(VIPER_ERR_INVALID, "rest_v, caps, w and work are required");
  if (nf > 0 && !tris) return fail(VIPER_ERR_INVALID, "tris is NULL");
  if (S->E == 0 && V > 0) return fail(VIPER_ERR_INVALID, "the scene has no capsules");
  if (iterations < 0 || !(lambda > 0.0 && lambda <= 1.0))
    return fail(VIPER_ERR_INVALID, "iterations >= 0 and 0 < lambda <= 1 required");
  if (V == 0) return VIPER_OK;
  std::vector<int32_t> off, nbr;
  if (!mesh_graph(V, nf, tris, off, nbr)) return fail(VIPER_ERR_INVALID, "a triangle references a vertex outside [0, V)");
  const size_t need = skin_fair_work_bytes(V, (int64_t)nbr.size());
  if (work_bytes < need) return fail(VIPER_ERR_INVALID, "work buffer too small: need " + std::to_string(need) + " bytes");
  hipStream_t st = (hipStream_t)stream;
  char* wk = (char*)work;
  const size_t noff = align256(4 * off.size());
  int32_t* overflow = (int32_t*)(wk + need - 256);
  const int32_t zero = 0;
  HIP_TRY(hipMemcpyAsync(wk, off.data(), 4 * off.size(), hipMemcpyHostToDevice, st));
  if (!nbr.empty()) HIP_TRY(hipMemcpyAsync(wk + noff, nbr.data(), 4 * nbr.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(overflow, &zero, 4, hipMemcpyHostToDevice, st));
  const int32_t* doff = (const int32_t*)wk;
  const int32_t* dnbr = (const int32_t*)(wk + noff);
  if (S->precision == VIPER_F64)
    HIP_TRY(launch_skin_weights_faired<double>(S->dd, V, rest_v, doff, dnbr, (int64_t)nbr.size(), iterations, lambda, wk,
                                               overflow, caps, w, st));
  else
    HIP_TRY(launch_skin_weights_faired<float>(S->df, V, rest_v, doff, dnbr, (int64_t)nbr.size(), iterations, lambda, wk,
                                              overflow, caps, w, st));
  int32_t flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, overflow, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));   // the host graph and flag die with this frame
  if (flag) return fail(VIPER_ERR_CAPACITY, "a vertex gathered more than 256 distinct capsules in one fairing step");
  return VIPER_OK;
}

viper_status viper_set_floor(viper_scene S, const double* normal, double offset, void* stream) {
  if (!S || !normal) return fail(VIPER_ERR_INVALID, "scene and normal are required");
  if (!S->floor_on) return fail(VIPER_ERR_INVALID, "the scene was created without a floor");
  if (!std::isfinite(normal[0]) || !std::isfinite(normal[1]) || !std::isfinite(normal[2]) || !std::isfinite(offset) ||
      !(normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2] > 0))
    return fail(VIPER_ERR_INVALID, "floor normal must be finite and nonzero, offset finite");
  const double l = std::sqrt(normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2]);
  for (int i = 0; i < 3; ++i) S->floor_n[i] = normal[i] / l;
  S->floor_d = offset / l;
  // the scene record lives at the start of the device header: update it there, in stream order ...
  size_t dsz;
  if (S->precision == VIPER_F64) {
    S->dd.fnx = S->floor_n[0]; S->dd.fny = S->floor_n[1]; S->dd.fnz = S->floor_n[2]; S->dd.fd = S->floor_d;
    dsz = sizeof(Dev<double>);
    std::memcpy(S->header.data(), &S->dd, dsz);
  } else {
    S->df.fnx = S->floor_n[0]; S->df.fny = S->floor_n[1]; S->df.fnz = S->floor_n[2]; S->df.fd = S->floor_d;
    dsz = sizeof(Dev<float>);
    std::memcpy(S->header.data(), &S->df, dsz);
  }
  // ... and in every wavefront's launch record, which carries a copy of it
  const size_t rec0 = (size_t)(S->batch.wrec - (S->ws + S->o.header));
  for (int k = 0; k < S->batch.nwaves; ++k)
    std::memcpy(S->header.data() + rec0 + (size_t)k * S->batch.wrec_stride + sizeof(WaveRec), S->header.data(), dsz);
  HIP_TRY(hipMemcpyAsync(S->ws + S->o.header, S->header.data(), S->header.size(), hipMemcpyHostToDevice,
                         (hipStream_t)stream));
  return VIPER_OK;
}

viper_status viper_set_bones(viper_scene S, const double* transforms, void* stream) {
  if (!S || !transforms) return fail(VIPER_ERR_INVALID, "scene and transforms are required");
  if (S->nbones == 0) return fail(VIPER_ERR_INVALID, "the scene has no bones");
  for (int b = 0; b < S->nbones; ++b)
    if (!affine_ok(transforms + 12 * (size_t)b))
      return fail(VIPER_ERR_INVALID, "bone transforms must be finite with an invertible linear part");
  hipStream_t st = (hipStream_t)stream;
  char* w = S->ws;
  double* prev = (double*)(w + S->o.bone_prev);
  double* delta = (double*)(w + S->o.bone_delta);
  const int32_t* pb = (const int32_t*)(w + S->o.pill_bone);
  const double* pw = (const double*)(w + S->o.pill_bone_w);
  if (S->precision == VIPER_F64) HIP_TRY(launch_bone_warm<double>(S->dd, S->nbones, transforms, prev, delta, pb, pw, st));
  else HIP_TRY(launch_bone_warm<float>(S->df, S->nbones, transforms, prev, delta, pb, pw, st));
  return VIPER_OK;
}

viper_status viper_sync(viper_scene S, void* stream) {
  if (!S) return fail(VIPER_ERR_INVALID, "scene is NULL");
  hipStream_t st = (hipStream_t)stream;
  int32_t h[ST_WORDS];
  HIP_TRY(hipMemcpyAsync(h, S->ws + S->o.status, sizeof(h), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipGetLastError());
  if (h[ST_NAN] || h[ST_OVERFLOW] || h[ST_DIVERGED]) {
    HIP_TRY(hipMemsetAsync(S->ws + S->o.status, 0, sizeof(h), st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h[ST_NAN]) return fail(VIPER_ERR_NAN, "non-finite state detected");
    if (h[ST_DIVERGED])
      return fail(VIPER_ERR_NAN, "the scene diverged: capsules outgrew 4x their rest bounding radius "
                                 "(contact detection skipped)");
    return fail(VIPER_ERR_CAPACITY, "contact buffer overflow: raise contact_capacity_per_capsule");
  }
  return VIPER_OK;
}

viper_status viper_contact_stats(viper_scene S, viper_contact_info* info, void* stream) {
  if (!S || !info) return fail(VIPER_ERR_INVALID, "scene and info are required");
  if (!S->collisions) return fail(VIPER_ERR_INVALID, "the scene has no contacts");
  viper_status r = contact_get_info(S->cd, info, (hipStream_t)stream);
  if (r != VIPER_OK) return fail(r, "could not read the detection record");
  return VIPER_OK;
}

viper_status viper_destroy_scene(viper_scene S) {
  delete S;
  return VIPER_OK;
}

viper_status viper_scene_info(viper_scene S, int64_t* pills, int64_t* rods, int64_t* capsules, int64_t* ppi) {
  if (!S) return fail(VIPER_ERR_INVALID, "scene is NULL");
  if (pills) *pills = S->P;
  if (rods) *rods = S->R;
  if (capsules) *capsules = S->E;
  if (ppi) *ppi = S->proj_per_iter;
  return VIPER_OK;
}


}  // extern "C"

// ----------------------------------------------------------------------------- adjoint

namespace {

viper_status adjoint_check(viper_scene S, int32_t frames, int32_t substeps, int32_t iterations) {
  if (!S) return fail(VIPER_ERR_INVALID, "scene is NULL");
  if (S->collisions) return fail(VIPER_ERR_INVALID, "the adjoint covers collision-free scenes");
  if (S->nsec) return fail(VIPER_ERR_INVALID, "the adjoint does not cover bundling sections");
  if (S->floor_on) return fail(VIPER_ERR_INVALID, "the adjoint does not cover the floor");
  if (S->jacobi) return fail(VIPER_ERR_INVALID, "the adjoint covers the Gauss-Seidel solver");
  if (S->cross_stretch) return fail(VIPER_ERR_INVALID, "the adjoint does not cover the cross-section stretch");
  if (S->nbones) return fail(VIPER_ERR_INVALID, "the adjoint does not cover bones");
  if (S->surface_bending) return fail(VIPER_ERR_INVALID, "the adjoint does not cover surface bending");
  if (S->volume_bending) return fail(VIPER_ERR_INVALID, "the adjoint does not cover the volume-bending coupling");
  if (frames < 1 || substeps < 1 || iterations < 0)
    return fail(VIPER_ERR_INVALID, "frames >= 1, substeps >= 1 and iterations >= 0 required");
  return VIPER_OK;
}

void adjoint_bytes(viper_scene S, int32_t frames, int32_t substeps, int32_t iterations, size_t* ckpt,
                   size_t* snap, size_t* adj, size_t* padj) {
  const size_t ts = S->precision == VIPER_F64 ? 8 : 4;
  const size_t P = (size_t)S->P, NL = (size_t)S->W * 64;
  *ckpt = (size_t)frames * substeps * kCkptFields * P * ts;
  *snap = align256(2 * ((size_t)iterations * kSnapPerIter + kSnapEnd) * NL * ts);
  *adj = align256((size_t)kCkptFields * P * ts);
  *padj = align256(8 * P * ts);
}

viper_status backward_launch(viper_scene S, double dt, int32_t frames, int32_t substeps, int32_t iterations,
                             const void* ckpt, const void* dl_dx, char* w, double* dl_drbar, double* dl_dact,
                             void* stream);

// Scratch of viper_step_backward_static, for callers that cannot allocate device memory: one
// copy per GPU (each device holds it from the library's load until the process ends), shared
// by every call on that GPU.  Host code never uses the array's name as an address: its device
// address is looked up once per device (static_scratch) and kept.
constexpr size_t kStaticScratchBytes = size_t(160) << 20;
__device__ __align__(256) static char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::vector<char*> g_scratch_ptr;      // device address of `scratch`, per device id

// Device address of the current device's `scratch` (looked up at the first call on a device,
// with that device current).
viper_status static_scratch(char** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(VIPER_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return VIPER_OK;
}

template <class T>
viper_status ckpt_t(viper_scene S, double h, int32_t frames, int32_t sub, int32_t iters, T* ckpt,
                           hipStream_t st) {
  const size_t per_frame = (size_t)sub * kCkptFields * S->P;
  for (int f = 0; f < frames; ++f) HIP_TRY(launch_frame_ckpt<T>(S->batch, sub, h, iters, ckpt + f * per_frame, st));
  return VIPER_OK;
}

}  // namespace

extern "C" {

viper_status viper_adjoint_sizes(viper_scene S, int32_t frames, int32_t substeps, int32_t iterations,
                                 size_t* ckpt_bytes, size_t* work_bytes) {
  viper_status r = adjoint_check(S, frames, substeps, iterations);
  if (r != VIPER_OK) return r;
  size_t c, sn, a, pa;
  adjoint_bytes(S, frames, substeps, iterations, &c, &sn, &a, &pa);
  if (ckpt_bytes) *ckpt_bytes = c;
  if (work_bytes) *work_bytes = sn + a + pa;
  return VIPER_OK;
}

viper_status viper_step_checkpointed(viper_scene S, double dt, int32_t frames, int32_t substeps, int32_t iterations,
                                     void* ckpt, size_t ckpt_bytes, void* stream) {
  viper_status r = adjoint_check(S, frames, substeps, iterations);
  if (r != VIPER_OK) return r;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(VIPER_ERR_INVALID, "dt must be finite and > 0");
  size_t c, sn, a, pa;
  adjoint_bytes(S, frames, substeps, iterations, &c, &sn, &a, &pa);
  if (!ckpt || ckpt_bytes < c) return fail(VIPER_ERR_INVALID, "checkpoint buffer missing or too small");
  const double h = dt / substeps;
  hipStream_t st = (hipStream_t)stream;
  return S->precision == VIPER_F64 ? ckpt_t<double>(S, h, frames, substeps, iterations, (double*)ckpt, st)
                                   : ckpt_t<float>(S, h, frames, substeps, iterations, (float*)ckpt, st);
}

viper_status viper_step_backward(viper_scene S, double dt, int32_t frames, int32_t substeps, int32_t iterations,
                                 const void* ckpt, const void* dl_dx, void* work, size_t work_bytes,
                                 double* dl_drbar, double* dl_dact, void* stream) {
  viper_status r = adjoint_check(S, frames, substeps, iterations);
  if (r != VIPER_OK) return r;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(VIPER_ERR_INVALID, "dt must be finite and > 0");
  if (!ckpt || !dl_dx || !dl_drbar || !dl_dact) return fail(VIPER_ERR_INVALID, "ckpt, dl_dx and outputs are required");
  size_t c, sn, a, pa;
  adjoint_bytes(S, frames, substeps, iterations, &c, &sn, &a, &pa);
  if (!work || work_bytes < sn + a + pa) return fail(VIPER_ERR_INVALID, "work buffer missing or too small");
  return backward_launch(S, dt, frames, substeps, iterations, ckpt, dl_dx, (char*)work, dl_drbar, dl_dact, stream);
}

viper_status viper_step_backward_static(viper_scene S, double dt, int32_t frames, int32_t substeps, int32_t iterations,
                                        const void* ckpt, const void* dl_dx, double* dl_drbar, double* dl_dact,
                                        void* stream) {
  viper_status r = adjoint_check(S, frames, substeps, iterations);
  if (r != VIPER_OK) return r;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(VIPER_ERR_INVALID, "dt must be finite and > 0");
  if (!ckpt || !dl_dx || !dl_drbar || !dl_dact) return fail(VIPER_ERR_INVALID, "ckpt, dl_dx and outputs are required");
  size_t c, sn, a, pa;
  adjoint_bytes(S, frames, substeps, iterations, &c, &sn, &a, &pa);
  if (sn + a + pa > kStaticScratchBytes)
    return fail(VIPER_ERR_NO_CAPACITY, "the backward needs " + std::to_string(sn + a + pa) +
                                           " bytes of scratch, more than the static " +
                                           std::to_string(kStaticScratchBytes) + "; use viper_step_backward");
  char* w = nullptr;
  r = static_scratch(&w);
  if (r != VIPER_OK) return r;
  return backward_launch(S, dt, frames, substeps, iterations, ckpt, dl_dx, w, dl_drbar, dl_dact, stream);
}

}  // extern "C"

namespace {

viper_status backward_launch(viper_scene S, double dt, int32_t frames, int32_t substeps, int32_t iterations,
                             const void* ckpt, const void* dl_dx, char* w, double* dl_drbar, double* dl_dact,
                             void* stream) {
  size_t c, sn, a, pa;
  adjoint_bytes(S, frames, substeps, iterations, &c, &sn, &a, &pa);
  const double h = dt / substeps;
  const int nsub = frames * substeps;
  hipStream_t st = (hipStream_t)stream;
  if (S->precision == VIPER_F64) {
    HIP_TRY(launch_backward<double>(S->batch, S->P, nsub, h, iterations, (const double*)ckpt, (const double*)dl_dx,
                                    (double*)w, (double*)(w + sn), (double*)(w + sn + a), S->density, dl_drbar,
                                    dl_dact, st));
  } else {
    HIP_TRY(launch_backward<float>(S->batch, S->P, nsub, h, iterations, (const float*)ckpt, (const float*)dl_dx,
                                   (float*)w, (float*)(w + sn), (float*)(w + sn + a), S->density, dl_drbar, dl_dact,
                                   st));
  }
  return VIPER_OK;
}

}  // namespace

// ============================================================================= serving pool

namespace {
struct PoolSlot {
  viper_scene_s* scene = nullptr;
  size_t off = 0, size = 0;
};
}  // namespace

struct viper_pool_s {
  char* ws = nullptr;
  size_t bytes = 0;
  int precision = 0;
  int max_scenes = 0;
  size_t header_cap = 0;                 // [0, header_cap): two batch headers
  std::map<size_t, size_t> free_;        // offset -> size of free ranges
  std::vector<PoolSlot> slots;
  bool dirty_f = true, dirty_c = true;   // membership of a class changed since its header was built
  BatchDev fb, cb;                       // collision-free batch, contact batch
  std::vector<char> hf, hc;              // host images of the headers
  hipStream_t aux = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t done[2] = {nullptr, nullptr};   // end of the last step of each class (any stream)
  bool stepped[2] = {false, false};
  // status words of each class's last step: device [2][max_scenes] (after the headers), the
  // slot of every batch member [2][max_scenes], and the pinned host copy [2][max_scenes]
  int32_t* dstat = nullptr;
  int32_t* dslot = nullptr;
  int32_t* hstat = nullptr;
};

namespace {

void pool_free_range(viper_pool_s* P, size_t off, size_t size) {
  auto it = P->free_.emplace(off, size).first;
  auto nx = std::next(it);
  if (nx != P->free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    P->free_.erase(nx);
  }
  if (it != P->free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      P->free_.erase(it);
    }
  }
}

// Rebuild the header of one class (collision-free or with contacts) in its own half of
// the header region.  `st` is the stream that stepped that class last: it is synchronised
// first, so that no step still reads the header being replaced.
template <class T>
viper_status pool_rebuild(viper_pool_s* P, bool contact, hipStream_t st) {
  const int cls = contact ? 1 : 0;
  if (P->stepped[cls]) HIP_TRY(hipEventSynchronize(P->done[cls]));   // its last step, on any stream
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<const void*> dv;
  std::vector<ContactDev> cc;
  std::vector<Counts> vc;
  std::vector<int32_t> slot_of;
  bool extras = false, even = true;
  for (int i = 0; i < (int)P->slots.size(); ++i) {
    const PoolSlot& sl = P->slots[i];
    if (!sl.scene || (sl.scene->collisions != 0) != contact) continue;
    viper_scene_s* S = sl.scene;
    extras = extras || scene_extras(S);
    even = even && S->even != 0;
    dv.push_back((const void*)&dev<T>(S));
    if (contact) cc.push_back(S->cd);
    vc.push_back(scene_counts(S));
    slot_of.push_back(i);
  }
  if (!slot_of.empty())
    HIP_TRY(hipMemcpyAsync(P->dslot + (size_t)cls * P->max_scenes, slot_of.data(), 4 * slot_of.size(),
                           hipMemcpyHostToDevice, st));
  const size_t half = P->header_cap / 2;
  if (header_bytes(vc, sizeof(Dev<T>)) > half)
    return fail(VIPER_ERR_NO_CAPACITY, "pool header region too small for the resident set");
  std::vector<char>& img = contact ? P->hc : P->hf;
  char* at = P->ws + (contact ? half : 0);
  BatchDev& b = contact ? P->cb : P->fb;
  build_header(img, dv, sizeof(Dev<T>), cc, vc, at, b);
  b.extras = extras;
  b.even = even;
  if (!img.empty()) {
    HIP_TRY(hipMemcpyAsync(at, img.data(), img.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // the host image may change before the next rebuild
  }
  (contact ? P->dirty_c : P->dirty_f) = false;
  return VIPER_OK;
}

// Status words of every scene of a batch into the class's status array, by slot.
template <class T>
__global__ void __launch_bounds__(256) pool_status_kernel(const Dev<T>* __restrict__ D, int n, const int32_t* __restrict__ slot,
                                                          int32_t* __restrict__ out) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  const int32_t* w = D[i].status;
  out[slot[i]] = w[ST_NAN] || w[ST_DIVERGED] ? VIPER_ERR_NAN : (w[ST_OVERFLOW] ? VIPER_ERR_CAPACITY : VIPER_OK);
}

template <class T>
viper_status pool_step_class(viper_pool_s* P, bool contact, double dt, int sub, int iters, hipStream_t st) {
  if (contact ? P->dirty_c : P->dirty_f) {
    viper_status r = pool_rebuild<T>(P, contact, st);
    if (r != VIPER_OK) return r;
  }
  const BatchDev& b = contact ? P->cb : P->fb;
  if (b.nscenes == 0) return VIPER_OK;
  viper_status r =
      batch_step<T>(b, contact, false, dt, sub, iters, contact ? VIPER_MODE_ITERATION : VIPER_MODE_FRAME, st);
  if (r != VIPER_OK) return r;
  // the members' conditions, to pinned host memory in stream order (read by viper_pool_status
  // once the caller has seen this step complete)
  const int cls = contact ? 1 : 0;
  int32_t* ds = P->dstat + (size_t)cls * P->max_scenes;
  hipLaunchKernelGGL(pool_status_kernel<T>, dim3((b.nscenes + 255) / 256), dim3(256), 0, st, (const Dev<T>*)b.dev,
                     b.nscenes, P->dslot + (size_t)cls * P->max_scenes, ds);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(P->hstat + (size_t)cls * P->max_scenes, ds, 4 * (size_t)P->max_scenes, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(P->done[cls], st));
  P->stepped[cls] = true;
  return VIPER_OK;
}

// Both classes: collision-free on `st`, contacts on the pool's second stream; both start
// after the work already on `st`, and `st` waits for both.
template <class T>
viper_status pool_step_t(viper_pool_s* P, double dt, int sub, int iters, hipStream_t st) {
  const bool contacts = P->dirty_c || P->cb.nscenes > 0;
  if (contacts) {
    if (!P->aux) HIP_TRY(hipStreamCreateWithFlags(&P->aux, hipStreamNonBlocking));
    HIP_TRY(hipEventRecord(P->ev0, st));
    HIP_TRY(hipStreamWaitEvent(P->aux, P->ev0, 0));
  }
  viper_status r = pool_step_class<T>(P, false, dt, sub, iters, st);
  if (r != VIPER_OK) return r;
  if (contacts) {
    r = pool_step_class<T>(P, true, dt, sub, iters, P->aux);
    if (r != VIPER_OK) return r;
    HIP_TRY(hipEventRecord(P->ev1, P->aux));
    HIP_TRY(hipStreamWaitEvent(st, P->ev1, 0));
  }
  return VIPER_OK;
}

}  // namespace

extern "C" {

viper_status viper_pool_create(void* workspace, size_t bytes, int32_t max_scenes, int32_t precision, void* stream,
                               viper_pool* out) {
  (void)stream;
  if (!workspace || !out || max_scenes < 1) return fail(VIPER_ERR_INVALID, "workspace, out and max_scenes >= 1 are required");
  if (((uintptr_t)workspace) & 255) return fail(VIPER_ERR_INVALID, "workspace must be 256-byte aligned");
  if (precision != VIPER_F32 && precision != VIPER_F64) return fail(VIPER_ERR_INVALID, "unknown precision");
  const size_t header = align256(std::max<size_t>(bytes / 64, 1u << 20) + (size_t)max_scenes * 8192);
  const size_t stat = align256(4 * 4 * (size_t)max_scenes);   // status words and member slots of both classes
  if (bytes < 2 * (header + stat)) return fail(VIPER_ERR_NO_CAPACITY, "pool workspace too small");
  viper_pool_s* P = new viper_pool_s();
  P->ws = (char*)workspace;
  P->bytes = bytes;
  P->precision = precision;
  P->max_scenes = max_scenes;
  P->header_cap = header;
  P->dstat = (int32_t*)(P->ws + header);
  P->dslot = P->dstat + 2 * (size_t)max_scenes;
  P->free_[header + stat] = bytes - header - stat;
  P->slots.resize(max_scenes);
  // the second stream of the joint step is created at its first use (callers that step the
  // classes on their own streams never need it, and every stream takes a hardware queue)
  if (hipEventCreateWithFlags(&P->ev0, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P->ev1, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P->done[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P->done[1], hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void**)&P->hstat, 4 * 2 * (size_t)max_scenes, hipHostMallocDefault) != hipSuccess) {
    viper_pool_destroy(P);
    return fail(VIPER_ERR_DEVICE, "could not create the pool's events and status buffer");
  }
  std::memset(P->hstat, 0, 4 * 2 * (size_t)max_scenes);
  *out = P;
  return VIPER_OK;
}

viper_status viper_pool_admit(viper_pool P, const viper_scene_desc* desc, void* stream, int32_t* slot) {
  if (!P || !desc || !slot) return fail(VIPER_ERR_INVALID, "pool, desc and slot are required");
  if (desc->precision != P->precision) return fail(VIPER_ERR_INVALID, "scene precision differs from the pool's");
  if (desc->num_sections > 0 || desc->floor_on || desc->solver == 1)
    return fail(VIPER_ERR_INVALID, "scenes with bundling sections, a floor or the Jacobi solver are stepped with viper_step");
  if (desc->cross_compliance)
    for (int k = 0; k < desc->num_rods; ++k)
      if (std::isfinite(desc->cross_compliance[k]))
        return fail(VIPER_ERR_INVALID, "scenes with the cross-section stretch are stepped with viper_step");
  if (desc->num_bones > 0) return fail(VIPER_ERR_INVALID, "scenes with bones are stepped with viper_step");
  if (desc->volume_bending)
    return fail(VIPER_ERR_INVALID, "scenes with the volume-bending coupling are stepped with viper_step");
  if (desc->bending_compliance)
    for (int k = 0; k < desc->num_rods; ++k)
      if (std::isfinite(desc->bending_compliance[k]))
        return fail(VIPER_ERR_INVALID, "scenes with surface bending are stepped with viper_step");
  size_t fp = 0;
  viper_status r = viper_scene_footprint(desc, &fp);
  if (r != VIPER_OK) return r;
  fp = align256(fp);
  int sid = -1;
  for (int i = 0; i < P->max_scenes; ++i)
    if (!P->slots[i].scene) { sid = i; break; }
  if (sid < 0) return fail(VIPER_ERR_NO_CAPACITY, "all pool slots are in use");
  auto it = P->free_.begin();
  for (; it != P->free_.end(); ++it)
    if (it->second >= fp) break;
  if (it == P->free_.end()) return fail(VIPER_ERR_NO_CAPACITY, "no free range of " + std::to_string(fp) + " bytes");
  const size_t off = it->first, size = it->second;
  P->free_.erase(it);
  if (size > fp) P->free_[off + fp] = size - fp;
  viper_scene S = nullptr;
  r = viper_create_scene(desc, P->ws + off, fp, stream, &S);
  if (r != VIPER_OK) {
    pool_free_range(P, off, fp);
    return r;
  }
  P->slots[sid] = PoolSlot{S, off, fp};
  (S->collisions ? P->dirty_c : P->dirty_f) = true;
  *slot = sid;
  return VIPER_OK;
}

viper_status viper_pool_step(viper_pool P, double dt, int32_t substeps, int32_t iterations, void* stream) {
  if (!P) return fail(VIPER_ERR_INVALID, "pool is NULL");
  if (!(dt > 0) || !std::isfinite(dt) || substeps < 1 || iterations < 0)
    return fail(VIPER_ERR_INVALID, "dt > 0, substeps >= 1, iterations >= 0 required");
  hipStream_t st = (hipStream_t)stream;
  return P->precision == VIPER_F64 ? pool_step_t<double>(P, dt, substeps, iterations, st)
                                   : pool_step_t<float>(P, dt, substeps, iterations, st);
}

viper_status viper_pool_step_ex(viper_pool P, double dt, int32_t substeps, int32_t iterations, int32_t classes,
                                void* stream) {
  if (!P) return fail(VIPER_ERR_INVALID, "pool is NULL");
  if (!(dt > 0) || !std::isfinite(dt) || substeps < 1 || iterations < 0)
    return fail(VIPER_ERR_INVALID, "dt > 0, substeps >= 1, iterations >= 0 required");
  if (classes < 1 || classes > 3) return fail(VIPER_ERR_INVALID, "classes must be 1, 2 or 3");
  hipStream_t st = (hipStream_t)stream;
  viper_status r = VIPER_OK;
  for (int c = 0; c < 2 && r == VIPER_OK; ++c)
    if (classes & (1 << c))
      r = P->precision == VIPER_F64 ? pool_step_class<double>(P, c == 1, dt, substeps, iterations, st)
                                    : pool_step_class<float>(P, c == 1, dt, substeps, iterations, st);
  return r;
}

viper_status viper_pool_retire(viper_pool P, int32_t slot, void* stream) {
  (void)stream;
  if (!P || slot < 0 || slot >= P->max_scenes || !P->slots[slot].scene) return fail(VIPER_ERR_INVALID, "bad slot");
  // the range may be reused by the next admission: let the device finish with it first (the
  // scene's class's last step, on whichever stream it ran)
  const int cls = P->slots[slot].scene->collisions ? 1 : 0;
  if (P->stepped[cls]) HIP_TRY(hipEventSynchronize(P->done[cls]));
  PoolSlot& sl = P->slots[slot];
  (sl.scene->collisions ? P->dirty_c : P->dirty_f) = true;
  delete sl.scene;
  pool_free_range(P, sl.off, sl.size);
  sl = PoolSlot();
  return VIPER_OK;
}

viper_status viper_pool_status(viper_pool P, int32_t slot, int32_t* scene_status) {
  if (!P || !scene_status || slot < 0 || slot >= P->max_scenes || !P->slots[slot].scene)
    return fail(VIPER_ERR_INVALID, "bad slot");
  const int cls = P->slots[slot].scene->collisions ? 1 : 0;
  *scene_status = ((volatile int32_t*)P->hstat)[(size_t)cls * P->max_scenes + slot];
  return VIPER_OK;
}

viper_status viper_pool_scene(viper_pool P, int32_t slot, viper_scene* scene) {
  if (!P || !scene || slot < 0 || slot >= P->max_scenes || !P->slots[slot].scene) return fail(VIPER_ERR_INVALID, "bad slot");
  *scene = P->slots[slot].scene;
  return VIPER_OK;
}

viper_status viper_pool_info(viper_pool P, size_t* free_bytes, size_t* largest_free, int32_t* resident,
                             int64_t* resident_pills) {
  if (!P) return fail(VIPER_ERR_INVALID, "pool is NULL");
  size_t fb = 0, lf = 0;
  for (auto& kv : P->free_) { fb += kv.second; lf = std::max(lf, kv.second); }
  int n = 0;
  int64_t pills = 0;
  for (auto& sl : P->slots)
    if (sl.scene) { ++n; pills += sl.scene->P; }
  if (free_bytes) *free_bytes = fb;
  if (largest_free) *largest_free = lf;
  if (resident) *resident = n;
  if (resident_pills) *resident_pills = pills;
  return VIPER_OK;
}

viper_status viper_pool_destroy(viper_pool P) {
  if (!P) return VIPER_OK;
  if (P->aux) (void)hipStreamSynchronize(P->aux);
  for (int c = 0; c < 2; ++c)     // the classes' last steps (and their status copies) first
    if (P->done[c]) {
      if (P->stepped[c]) (void)hipEventSynchronize(P->done[c]);
      (void)hipEventDestroy(P->done[c]);
    }
  for (auto& sl : P->slots) delete sl.scene;
  if (P->hstat) (void)hipHostFree(P->hstat);
  if (P->ev0) (void)hipEventDestroy(P->ev0);
  if (P->ev1) (void)hipEventDestroy(P->ev1);
  if (P->aux) (void)hipStreamDestroy(P->aux);
  delete P;
  return VIPER_OK;
}

}  // extern "C"
