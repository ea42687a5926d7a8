/*
 * viper.h -- C ABI of the MI355X VIPER rod-solver library (libviper.so).
 *
 * The library advances many volume-invariant elastic rods ("VIPER" rods,
 * Angles et al. 2019) with the position-based substep of Sec. 6: inertial
 * prediction, coloured Gauss-Seidel projection of the stretch-shear,
 * volume, scale-gradient and bend-twist constraints (Sec. 5, Sec. 7.5),
 * pill-pill contacts (Sec. 7.1-7.2) and a velocity update; plus linear-blend
 * skinning of a mesh onto the rods (Sec. 7.4).
 *
 * Conventions (all entry points):
 *   - Every call returns a viper_status; no C++ exception crosses the ABI.
 *     On failure viper_last_error() returns a thread-local message.
 *   - The library never allocates device memory.  The caller allocates one
 *     device workspace of viper_scene_footprint() bytes (any allocator; the
 *     Python binding uses a torch uint8 tensor), keeps it alive and
 *     unmodified until viper_destroy_scene(), and owns it afterwards.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Kernels and
 *     copies are enqueued asynchronously on it; device-side conditions
 *     (non-finite state, contact-buffer overflow) surface at viper_sync().
 *   - Host description arrays are read only during the call that takes them.
 *   - Indices: pills (vertices) are numbered globally in rod order; rod k owns
 *     pills [rod_offsets[k], rod_offsets[k+1]).  Edge j of a rod joins its pills
 *     j and j+1 and is stored in the slot of pill j (the last slot of a rod has
 *     no edge).  A capsule (the paper's tapered "pill" primitive, Sec. 7) is an
 *     edge; its id is the global index of its first pill.
 */
#ifndef VIPER_H
#define VIPER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct viper_scene_s* viper_scene;

typedef enum {
  VIPER_OK = 0,
  VIPER_ERR_INVALID = 1,      /* bad argument or scene description (nothing enqueued) */
  VIPER_ERR_NO_CAPACITY = 2,  /* workspace / pool too small */
  VIPER_ERR_CAPACITY = 3,     /* contact buffer overflowed during a step (reported by viper_sync) */
  VIPER_ERR_NAN = 4,          /* non-finite state detected (reported by viper_sync) */
  VIPER_ERR_DEVICE = 5        /* a HIP runtime call failed */
} viper_status;

typedef enum { VIPER_F32 = 0, VIPER_F64 = 1 } viper_precision;

/* Scene description.  Physical inputs of the problem as the paper states it:
 * rest centre line and rest radius r (Sec. 3, eq. rest_parametrization), mass
 * density m (Sec. 4), per-type material compliances = inverse stiffnesses K^-1
 * (Sec. 5/6), external gravity (Sec. 4, prediction), kinematic pins (Sec. 7),
 * fibre activation as a rest-length scale (Sec. 8, muscle simulation) and
 * collision groups (intra-muscle collisions disabled, Sec. 8). */
typedef struct {
  int32_t num_rods;
  const int32_t* rod_offsets;   /* [num_rods+1], increasing, 2 <= pills per rod <= 128 */
  const double* rest_pos;       /* [P*3] rest vertex positions, m; consecutive pills distinct */
  const double* rest_radius;    /* [P] rest radius r, m, > 0 */
  const uint8_t* pinned;        /* [P] nonzero = position fixed (scale, rotation stay free); may be NULL */
  const double* activation;     /* [num_rods] > 0, scales the stretch rest length; may be NULL (= 1) */
  const double* compliance;     /* [num_rods*4] Pa^-1 for stretch-shear, volume, scale-gradient,
                                   bend-twist; >= 0; +inf disables that constraint type for the rod */
  const int32_t* group;         /* [num_rods] collision group; equal groups never collide; may be NULL */
  double density;               /* kg/m^3, > 0 */
  double gravity[3];            /* m/s^2 */
  int32_t precision;            /* viper_precision: storage and arithmetic type on the device */
  int32_t collisions;           /* nonzero = pill-pill contacts on */
  int32_t contact_capacity_per_capsule; /* candidate pairs per capsule reserved (<= 0: 16) */
  /* Bundling (Sec. 7.3, scale-invariant shape matching of muscle cross-sections): section k
   * is the pills section_pills[section_offsets[k] .. section_offsets[k+1]) (host arrays, read
   * during create only; section_offsets[0] = 0, every section non-empty, no pill in two
   * sections).  Once per substep, after the constraint iterations, each section is fitted
   * with one similarity transform of its rest frames (current and rest frames [s R | x] of
   * its pills; a rod's last pill takes the rotation of its incoming edge) and every pill is
   * set to that transform of its rest frame; pinned pills keep their position.
   * num_sections = 0 turns bundling off.  A scene with sections steps in
   * VIPER_MODE_ITERATION or VIPER_MODE_GRAPH; the pool and the adjoint reject it. */
  int32_t num_sections;
  const int32_t* section_offsets;
  const int32_t* section_pills;
  /* Kinematic half-plane floor (Sec. 7): nonzero floor_on keeps every pill's sphere in
   * floor_normal . x >= floor_offset + s rbar (normal need not be unit; it is normalised).
   * Projected on positions only, at the start of every constraint iteration; pinned pills
   * are not moved.  A scene with a floor steps in VIPER_MODE_ITERATION or VIPER_MODE_GRAPH;
   * the pool and the adjoint reject it. */
  int32_t floor_on;
  double floor_normal[3];
  double floor_offset;
  /* Rod-constraint solver: 0 = coloured Gauss-Seidel (default), 1 = Jacobi with averaging
   * (Sec. 7: every constraint projected from the state at the start of the iteration, each
   * degree of freedom moved by the mean correction of the constraints acting on it).  A
   * Jacobi scene steps in VIPER_MODE_ITERATION or VIPER_MODE_GRAPH; the pool and the adjoint
   * reject it. */
  int32_t solver;
  /* Cross-section stretch (eq. stretch_xy), optional: compliance per rod [num_rods] of the
   * constraint C = (s_j + s_{j+1}) / 2 - 1 on every edge (the midpoint scale pulled back to
   * its rest value), scaled by 1 / (pi r^2 l) as stretch-shear and volume; >= 0, +inf = off
   * for that rod; NULL = off everywhere.  Solved after the scale gradient in the same edge
   * pass (both solvers); the pool and the adjoint reject a scene that turns it on. */
  const double* cross_compliance;
  /* Kinematic bones (Sec. 8.2), optional: num_bones rest transforms bone_rest [num_bones*12]
   * (each [A | b], 3x4 row-major: the bone's pose when the pills are at rest_pos; A
   * invertible), and two influences per pill, pill_bones [P*2] bone ids and
   * pill_bone_weights [P*2] weights >= 0 (an id is read only where its weight is > 0; a pill
   * whose weights are both 0 has no bone).  viper_set_bones then moves the pills with the
   * bones.  num_bones = 0 turns them off; the pool and the adjoint reject a scene with bones. */
  int32_t num_bones;
  const double* bone_rest;
  const int32_t* pill_bones;
  const double* pill_bone_weights;
  /* Surface bending (Sec. 5: the energy of the Laplacian of the scale), optional: compliance
   * per rod [num_rods] of the constraint at every interior vertex j (between edges j-1, j)
   * C = [(s_{j+1} - s_j) / l_j - (s_j - s_{j-1}) / l_{j-1}] / l_v, l_v = (l_{j-1} + l_j) / 2
   * (the rest scale is one, its Laplacian zero), scaled by 1 / (pi r^4 / 4 l_v) as bend-twist;
   * >= 0, +inf = off for that rod; NULL = off everywhere.  Solved in three colour passes after
   * bend-twist (Gauss-Seidel only: a Jacobi scene that turns it on is VIPER_ERR_INVALID); the
   * pool and the adjoint reject a scene that turns it on. */
  const double* bending_compliance;
  /* Volume-bending coupling (Sec. 5: the s^3 Omega^u, s^3 Omega^v terms of the volume
   * energy), optional: nonzero turns it on for every rod whose volume constraint is on, at
   * every interior vertex, C = s^3 c Im(r)_{u,v} - Omega_rest_{u,v} (r, c as bend-twist, s the
   * vertex scale; rest scale one), with the rod's volume compliance scaled by
   * 1 / (pi r^4 / 2 l_v).  Solved right after bend-twist at the same vertex (Gauss-Seidel only:
   * a Jacobi scene that turns it on is VIPER_ERR_INVALID); the pool and the adjoint reject a
   * scene that turns it on. */
  int32_t volume_bending;
} viper_scene_desc;

/* Bytes of device workspace the scene needs (host-only computation; validates the
 * description).  The workspace must be 256-byte aligned. */
viper_status viper_scene_footprint(const viper_scene_desc* desc, size_t* bytes);

/* Validate the description, compute rest quantities on the host (rest lengths,
 * parallel-transported rest frames, rest Darboux vectors, lumped inverse masses and
 * inertias, compliance scalings) and upload them with the initial state (at rest) into
 * `workspace` on `stream`.  The returned handle is owned by the caller and released
 * with viper_destroy_scene(). */
viper_status viper_create_scene(const viper_scene_desc* desc, void* workspace, size_t bytes, void* stream,
                                viper_scene* out);

/* Execution strategy for viper_step_ex. */
typedef enum {
  VIPER_MODE_AUTO = 0,      /* FRAME for plain rod scenes; GRAPH with collisions, bundling sections,
                               a floor or the Jacobi solver (these need the ITERATION launches) */
  VIPER_MODE_FRAME = 1,     /* one launch per call: all substeps with the rod state in registers */
  VIPER_MODE_SUBSTEP = 2,   /* one launch per substep: state streamed through HBM every substep */
  VIPER_MODE_ITERATION = 3, /* separate launches per stage and iteration (the contact path) */
  VIPER_MODE_GRAPH = 4      /* the ITERATION launches of one frame captured once into a HIP graph
                               (per scene and dt, substeps, iterations) and replayed: same kernels,
                               same results, one submission per frame */
} viper_mode;

/* Advance one frame of length dt (s) in `substeps` substeps of h = dt/substeps, each with
 * `iterations` constraint iterations (Sec. 6: prediction, then per-constraint dual
 * updates with lambda reset to 0 each substep, relaxation 1).  dt > 0, substeps >= 1,
 * iterations >= 0.  Per substep: prediction; contact detection (collisions); per iteration
 * the floor projection, the rod constraints (coloured Gauss-Seidel or Jacobi) and the
 * contact pass; after the iterations the bundling projection; the velocity update.
 * viper_step = viper_step_ex with VIPER_MODE_AUTO.  A mode the scene cannot run in (FRAME or
 * SUBSTEP with collisions, sections, a floor or the Jacobi solver) is VIPER_ERR_INVALID. */
viper_status viper_step(viper_scene scene, double dt, int32_t substeps, int32_t iterations, void* stream);
viper_status viper_step_ex(viper_scene scene, double dt, int32_t substeps, int32_t iterations, int32_t mode,
                           void* stream);

/* State fields for get/set.  Arrays are in the scene's precision (float or double),
 * pill-major: X, V: [P*3]; S (scale), SDOT: [P]; Q (edge quaternion x,y,z,w), [P*4];
 * OMEGA (edge angular velocity, world frame) [P*3]; RADIUS (physical radius s*r) [P];
 * XDET, SDET: positions/scales the last contact detection ran on (read only; XDET is
 * always FP64 world coordinates, exactly the values the FP64 candidate test used).
 * Positions are stored on the device relative to a per-rod anchor (the rest position
 * of the rod's first pill) and converted to world coordinates in FP64 at this boundary. */
typedef enum {
  VIPER_X = 0, VIPER_V = 1, VIPER_S = 2, VIPER_SDOT = 3, VIPER_Q = 4, VIPER_OMEGA = 5, VIPER_RADIUS = 6,
  VIPER_XDET = 7, VIPER_SDET = 8,
  VIPER_XLOCAL = 9   /* [P*3] positions relative to the rod anchor, exactly as stored (bit-exact
                        checkpoint / resume together with V, S, SDOT, Q, OMEGA) */
} viper_field;

/* Copy a state field to `dst` (device or host memory) / from `src` (device or host),
 * ordered on `stream`.  Slots without an edge read as zero and are ignored on write. */
viper_status viper_get_state(viper_scene scene, int32_t which, void* dst, void* stream);
viper_status viper_set_state(viper_scene scene, int32_t which, const void* src, void* stream);

/* Candidate contact pairs of the last substep's detection (Sec. 7.1): sorted (a, b),
 * a < b, capsule ids; written to device or host `pairs` [cap*2]; *n receives the count
 * (synchronises `stream`).  VIPER_ERR_NO_CAPACITY if n > cap (nothing written).  After a
 * detection that overflowed the scene's pair capacity (reported by viper_sync) the list
 * holds capacity-many of the candidates, which ones depending on the order of the search. */
viper_status viper_get_contacts(viper_scene scene, int32_t* pairs, int32_t cap, int32_t* n, void* stream);

/* Record of the last contact detection of a scene (Sec. 7.1 uniform grid, in two levels).
 * The capsule bounding radii are histogrammed (4 bins per octave).  The cell bin holds the
 * 33rd-largest radius: the at most 32 larger capsules are kept in a list that every capsule
 * searches.  Below it, a fine bin splits the capsules into a fine grid (cell width twice the
 * largest radius of the fine bin; the radii up to it) and a coarse grid (cell width twice
 * the sum of the cell bin's and the fine bin's largest radii; the radii above it), chosen to
 * minimise the entries examined for capsules spread uniformly; with one level the fine bin
 * is the cell bin.  A capsule examines half of the 27 cells around its own in its level
 * (the other half find the same pairs), a fine capsule also the 8 coarse cells nearest its
 * centre, and the list.
 * Capsules whose bounding sphere is not finite are left out and raise VIPER_ERR_NAN at
 * viper_sync; capsules with an end radius s r <= 0 (no surface while a scale passes through
 * zero) are left out too (no contact).  If the cell bin's radius would exceed 4 times the
 * largest bounding radius of the rest pose, the scene has diverged: its detection is skipped
 * (no candidates that substep) and viper_sync reports VIPER_ERR_NAN.  So every cell is at
 * most 16 rest radii wide. */
typedef struct {
  int64_t walk_entries;       /* bucket and list entries the candidate count pass examined */
  int32_t oversized;          /* capsules in the oversized list */
  int32_t excluded;           /* capsules left out: sphere not finite or an end radius <= 0 */
  int32_t skipped;            /* 1 if the detection was skipped (diverged scene) */
  int32_t cell_bin;           /* histogram bin of the fine grid's cell radius */
  double cell_width;          /* m, fine grid; 0 when skipped */
  double cell_radius_limit;   /* m: 4 x the largest bounding radius at rest */
  int32_t coarse_bin;         /* histogram bin of the coarse grid's largest radius; -1: one level */
  int32_t coarse_capsules;    /* capsules in the coarse grid */
  double coarse_width;        /* m, coarse grid; 0 with one level or when skipped */
} viper_contact_info;
/* Fills *info for a scene with collisions (synchronises `stream`); VIPER_ERR_INVALID
 * otherwise. */
viper_status viper_contact_stats(viper_scene scene, viper_contact_info* info, void* stream);

/* Linear-blend skinning (Sec. 7.4): register a mesh of V rest vertices, each with 4
 * (capsule id, weight) influences.  Device arrays, owned by the caller, read at every
 * viper_skin call: rest_v [V*3] float, caps [V*4] int32, w [V*4] float. */
viper_status viper_create_skin(viper_scene scene, int32_t V, const float* rest_v_dev, const int32_t* caps_dev,
                               const float* w_dev, void* stream, int32_t* skin_id);
/* out [V*3] float (device): v = sum_k w_k [s R(q) R(q_rest)^T | m - s R(q) R(q_rest)^T m_rest] [v_rest; 1]
 * per capsule (similarity transform of eq. shapematch, blended as in Sec. 7.4). */
viper_status viper_skin(viper_scene scene, int32_t skin_id, float* out_dev, void* stream);
/* Initial skinning weights (Sec. 7.4): for each of V vertices rest_v_dev [V*3] float (device),
 * weights proportional to the inverse square distance from the vertex to the surface of each
 * capsule at the scene's current pose (call it right after creation for the rest pose),
 * the four strongest kept and normalised: caps_dev [V*4] int32 capsule ids (first pill of the
 * capsule), w_dev [V*4] float, strongest first (device; caller-owned).  Without fairing (see
 * viper_skin_weights_faired, which needs the mesh connectivity).  Brute force over all
 * capsules: O(V * capsules). */
viper_status viper_skin_weights(viper_scene scene, int32_t V, const float* rest_v_dev, int32_t* caps_dev, float* w_dev,
                                void* stream);

/* Skinning weights faired over the mesh (Sec. 7.4: the paper starts from the inverse-square
 * assignment above and fairs it over the surface, after the Sphere-Meshes skinning it cites;
 * the steps are this library's reading).  Every vertex keeps its 8 strongest initial weights
 * (ties: lower capsule id), normalised; then `iterations` Jacobi Laplacian-smoothing steps on
 * the mesh graph (the undirected edges of the nf triangles tris_host [nf*3], host memory):
 * w(v) <- (1 - lambda) w(v) + lambda * mean of w over v's neighbours, summed per capsule in a
 * fixed order (own entries, then neighbours in ascending index) in FP64, the 8 largest kept
 * and renormalised after each step; finally the 4 largest, renormalised, are written to
 * caps_dev [V*4] / w_dev [V*4] (device; as viper_skin_weights).  With at most 8 capsules in
 * reach this is exactly linear Laplacian smoothing, which keeps a partition of unity.
 * work: device scratch of viper_skin_fair_work_bytes (the mesh graph and two sets of
 * per-vertex lists).  Synchronises `stream`.  VIPER_ERR_INVALID for 0 < lambda <= 1 violated,
 * iterations < 0, a triangle index outside [0, V) or a short work buffer; VIPER_ERR_CAPACITY
 * if a fairing step gathers more than 256 distinct capsules around one vertex (the result is
 * then incomplete). */
viper_status viper_skin_fair_work_bytes(int32_t V, int32_t nf, const int32_t* tris_host, size_t* work_bytes);
viper_status viper_skin_weights_faired(viper_scene scene, int32_t V, const float* rest_v_dev, int32_t nf,
                                       const int32_t* tris_host, int32_t iterations, double lambda, void* work,
                                       size_t work_bytes, int32_t* caps_dev, float* w_dev, void* stream);

/* Kinematic half-plane (Sec. 7 collision proxies): move the floor of a scene created with
 * floor_on to floor_normal . x >= floor_offset + s rbar (host values; the normal need not be
 * unit, it is normalised).  Ordered on `stream`: frames enqueued after it (captured graph
 * replays included) project onto the new plane; frames already enqueued keep the old one.
 * VIPER_ERR_INVALID for a scene without a floor or a non-finite or zero normal (nothing
 * changed). */
viper_status viper_set_floor(viper_scene scene, const double* floor_normal, double floor_offset, void* stream);

/* Kinematic bones (Sec. 8.2): the bones' transforms of a new frame, transforms [num_bones*12]
 * host memory (read before the call returns), each [A | b] 3x4 row-major with A invertible.
 * Every pill with bone weight moves by the blend of its bones' motions since the previous
 * call (or since the rest transforms), x <- sum_k w_k T_k T_prev,k^-1 x / sum_k w_k, in world
 * coordinates; pinned pills too (that is their kinematic attachment); velocities, scales and
 * rotations are kept.  Call it at the start of a frame, before viper_step; ordered on
 * `stream`.  VIPER_ERR_INVALID for a scene without bones or a non-finite or singular
 * transform (nothing moved). */
viper_status viper_set_bones(viper_scene scene, const double* transforms, void* stream);

/* Wait for `stream` and report device-side conditions raised since the last sync:
 * VIPER_ERR_NAN (a non-finite state, or a contact detection skipped because the scene
 * diverged), VIPER_ERR_CAPACITY, or VIPER_ERR_DEVICE. Clears them. */
viper_status viper_sync(viper_scene scene, void* stream);

/* Release the host handle (the workspace stays the caller's). */
viper_status viper_destroy_scene(viper_scene scene);

/* Numbers of pills, rods, capsules, and rod constraint projections per iteration. */
viper_status viper_scene_info(viper_scene scene, int64_t* pills, int64_t* rods, int64_t* capsules,
                              int64_t* projections_per_iteration);

const char* viper_last_error(void);

/* ---- Adjoint of the frame ---------------------------------------------------------------
 * Reverse mode through the collision-free frame of viper_step (Sec. 6: prediction, the
 * stretch-shear / volume / scale-gradient / bend-twist dual updates in their colour order,
 * velocity update), giving the gradient of a scalar loss of the final positions with
 * respect to the rest radii r (Sec. 3, through the lumped masses and inertias of App. B and
 * the compliance scalings of Sec. 5/6) and the per-rod activation a (Sec. 8: rest length
 * a l0).  The forward writes the state at the start of every substep (checkpoint); the
 * backward replays each substep from it in reverse order.  Scenes with collisions are
 * rejected with VIPER_ERR_INVALID.
 *
 * Device bytes needed: the checkpoint holds frames*substeps*15*P values in the scene's
 * precision; the backward scratch holds two substeps' per-pass state snapshots (the replay
 * of one substep runs beside the reverse sweep of the next) plus the state and parameter
 * adjoints. */
viper_status viper_adjoint_sizes(viper_scene scene, int32_t frames, int32_t substeps, int32_t iterations,
                                 size_t* ckpt_bytes, size_t* work_bytes);

/* Advance `frames` frames exactly as viper_step_ex(..., VIPER_MODE_FRAME) does (bitwise
 * the same state) and write the checkpoint to ckpt (device memory of ckpt_bytes). */
viper_status viper_step_checkpointed(viper_scene scene, double dt, int32_t frames, int32_t substeps,
                                     int32_t iterations, void* ckpt, size_t ckpt_bytes, void* stream);

/* Reverse of the viper_step_checkpointed call that wrote ckpt (same dt, frames, substeps,
 * iterations; the scene's parameters unchanged since).  dl_dx: device [P*3] in the scene's
 * precision, dL/dx of the positions after the last frame (world and stored rod-local
 * positions differ by a constant, so either gradient).  work: device scratch of work_bytes.
 * Outputs, device FP64, overwritten: dl_drbar [P], dl_dact [R].  The scene state is not
 * changed. */
viper_status viper_step_backward(viper_scene scene, double dt, int32_t frames, int32_t substeps, int32_t iterations,
                                 const void* ckpt, const void* dl_dx, void* work, size_t work_bytes,
                                 double* dl_drbar, double* dl_dact, void* stream);

/* viper_step_backward without a work buffer, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid allocation): the
 * scratch is a library-owned static device array of 160 MiB per GPU (held from the library's
 * load until the process ends), so the call allocates nothing.  Same arguments, semantics
 * and results as viper_step_backward otherwise.  VIPER_ERR_NO_CAPACITY (nothing enqueued)
 * when the work bytes of viper_adjoint_sizes exceed 160 MiB (the 1024 x 32 FP32 workload at
 * 8 iterations needs 90 MiB).  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams or threads) race and must be serialised by the caller. */
viper_status viper_step_backward_static(viper_scene scene, double dt, int32_t frames, int32_t substeps,
                                        int32_t iterations, const void* ckpt, const void* dl_dx, double* dl_drbar,
                                        double* dl_dact, void* stream);

/* ---- Serving pool: continuous batching of many scenes in one workspace ----------------
 * The pool owns no device memory either: the caller hands in one workspace.  Scenes are
 * admitted by footprint (first-fit inside the workspace; VIPER_ERR_NO_CAPACITY when no
 * free range or slot fits, nothing changed), stay resident on the device, and every
 * viper_pool_step advances every resident scene by one frame: all collision-free scenes
 * in one launch over a shared block table, all scenes with contacts through one shared
 * sequence of launches on a second stream that overlaps the first (both start after the
 * work already on `stream`; `stream` then waits for both).  A scene admitted
 * while a step runs joins at the next step; uploads of new scenes do not touch resident
 * state.  All scenes of a pool share `precision`.  The scene handles of a pool
 * (viper_pool_scene) serve viper_get_state / viper_set_state / viper_get_contacts /
 * viper_sync and must not be destroyed by the caller. */
typedef struct viper_pool_s* viper_pool;
viper_status viper_pool_create(void* workspace, size_t bytes, int32_t max_scenes, int32_t precision, void* stream,
                               viper_pool* out);
viper_status viper_pool_admit(viper_pool pool, const viper_scene_desc* desc, void* stream, int32_t* slot);
viper_status viper_pool_step(viper_pool pool, double dt, int32_t substeps, int32_t iterations, void* stream);
/* One frame of one class of resident scenes, enqueued on `stream`: classes = 1 the
 * collision-free scenes (one launch), 2 the scenes with contacts (their shared launch
 * sequence), 3 both on the same stream.  The classes are independent: a caller may keep a
 * step of each in flight on its own stream (a collision-free frame then does not wait for
 * the contact scenes' much longer one).  A class whose membership changed since its last
 * step first waits for `stream` and rebuilds its header.  Retire a scene only after its
 * class's last step has completed. */
viper_status viper_pool_step_ex(viper_pool pool, double dt, int32_t substeps, int32_t iterations, int32_t classes,
                                void* stream);
/* Free a scene's slot and range.  Waits for the last step of the scene's class (on
 * whichever stream it ran) before the range can be reused; `stream` is not used. */
viper_status viper_pool_retire(viper_pool pool, int32_t slot, void* stream);
/* Device-side condition of a resident scene as of the last step of its class: every class
 * step ends by copying its scenes' status words to pinned host memory in stream order, so
 * once the caller has seen that step complete (an event recorded after it, or a stream
 * synchronisation) *scene_status holds VIPER_OK, VIPER_ERR_NAN (non-finite state or a
 * diverged contact detection) or VIPER_ERR_CAPACITY (contact buffer overflow) for it,
 * without a further synchronisation.  Before the scene's first completed step the value
 * is meaningless.  The conditions stay set (viper_sync on the scene clears them). */
viper_status viper_pool_status(viper_pool pool, int32_t slot, int32_t* scene_status);
viper_status viper_pool_scene(viper_pool pool, int32_t slot, viper_scene* scene);
viper_status viper_pool_info(viper_pool pool, size_t* free_bytes, size_t* largest_free, int32_t* resident,
                             int64_t* resident_pills);
viper_status viper_pool_destroy(viper_pool pool);

#ifdef __cplusplus
}
#endif
#endif /* VIPER_H */
