/*
 * grasp.h - C ABI of the MI355X (gfx950) grid-SDF grasp-step library.
 *
 * The library computes the data-parallel hot path of Fast-Grasp'D's
 * gradient-based grasp synthesis (Sec. III-C "Position-based dynamics",
 * Sec. IV-A "Gradient-based grasp optimization"): for a batch of candidate
 * hand configurations q_h (a base pose plus joint angles, Sec. III), it runs
 * forward kinematics of the hand's contact points, samples the object's
 * signed-distance grid at every point in each of M = 7 velocity-test
 * simulations, turns penetration into position-based-dynamics corrections of
 * the object pose (Eq. (1)), forms the stability loss from the resulting
 * object velocities plus penetration and joint range/limit losses, and
 * back-propagates that loss to q_h with the leaky contact gradient, followed
 * by an Adam step.
 *
 * Object representation: a dense vertex-centred FP32 SDF grid sampled
 * trilinearly (the representation the paper describes for its predecessor,
 * Sec. III-A), with the analytic gradient of the trilinear blend.
 *
 * Conventions
 *  - Every call returns grasp_status (0 = GRASP_OK, negative = error) and
 *    never throws. grasp_last_error() describes the last failure of the
 *    calling thread.
 *  - "dev" pointers are device memory of the context's GPU, owned by the
 *    caller, and must stay valid until the work queued on the given stream
 *    has run. "host" pointers are read (or written) before the call returns.
 *  - hip_stream is a hipStream_t (NULL = the default stream). Step calls are
 *    asynchronous in stream order; argument errors are reported at once.
 *  - Units are SI: metres, seconds, radians.
 *  - A HIP runtime failure returns GRASP_EDEVICE and poisons the context:
 *    every later call on it returns GRASP_EDEVICE.
 */
#ifndef GRASP_H
#define GRASP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif
#pragma GCC visibility push(default)

typedef int32_t grasp_status;
enum {
  GRASP_OK = 0,
  GRASP_EINVAL = -1,     /* bad argument: NULL, shape, id, value */
  GRASP_ENOMEM = -2,     /* arena or workspace too small */
  GRASP_EDEVICE = -3,    /* HIP runtime failure; the context is poisoned */
  GRASP_EBUSY = -4,      /* object still used by a live job */
  GRASP_EAGAIN = -5,     /* job not finished yet */
  GRASP_ENONFINITE = -6, /* a loss or configuration became NaN/Inf */
  GRASP_ECANCELED = -7   /* job was cancelled */
};

typedef struct grasp_ctx grasp_ctx; /* opaque */
typedef uint64_t grasp_hand_id;
typedef uint64_t grasp_sdf_id;
typedef uint64_t grasp_job_id;

/* ---------------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------------- */

/* Creates a context on HIP device `device`. Hands, SDF grids and serving
 * state are sub-allocated from an arena of arena_bytes: arena_dev (dev,
 * caller-owned, 256-byte aligned) or, when arena_dev is NULL, device memory
 * the library allocates and frees itself. arena_bytes is also the HBM budget
 * that job admission respects. */
grasp_status grasp_init(int device, void* arena_dev, size_t arena_bytes, grasp_ctx** out);

/* Waits for the context's work, stops its scheduler and frees what it owns.
 * NULL is ignored. */
void grasp_shutdown(grasp_ctx* ctx);

/* Thread-local description of the calling thread's last error; valid until
 * that thread's next grasp_* call. Never NULL. */
const char* grasp_last_error(void);

/* ---------------------------------------------------------------------------
 * Hands: an articulation chain with contact points on its links (Sec. III:
 * "a mesh and an articulation chain"; every hand vertex is a constraint,
 * Sec. III-C).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t n_links;             /* 1..32; link 0 = palm; n_dof = 6 + (n_links - 1) */
  const int32_t* parent;       /* host [n_links]; parent[0] = -1, 0 <= parent[l] < l;
                                  at most 8 links on any root-to-leaf path below the palm */
  const float* joint_origin;   /* host [n_links][12], row-major 3x4 rigid transform from the
                                  parent link frame to joint l at q = 0 (entry 0 ignored) */
  const float* joint_axis;     /* host [n_links][3], unit revolute axis in the joint frame;
                                  link l turns by q[5 + l] (entry 0 ignored) */
  const float* q_low;          /* host [n_dof] joint limits; entries 0..5 (wrist) unused */
  const float* q_up;           /* host [n_dof] */
  int32_t n_contacts;          /* >= 1 */
  const float* contact_local;  /* host [n_contacts][3], in the frame of contact_link[i] */
  const int32_t* contact_link; /* host [n_contacts], 0 <= link < n_links */
} grasp_hand_desc;

/* The wrist is Trans(q0, q1, q2) Rz(q3) Ry(q4) Rx(q5); link l >= 1 has pose
 * T_parent * joint_origin[l] * Rot(joint_axis[l], q[5 + l]). The library
 * copies the description and re-lays the contacts out sorted by link, within
 * a link along a Morton curve of their link-frame coordinates (sums over
 * contacts run in that order); the Gauss-Seidel sweep takes the contacts of
 * a link in the caller's order. Results indexed by contact come back in the
 * caller's order.
 * EINVAL on a malformed description (e.g. a non-unit axis, |1 - |a|| > 1e-3). */
grasp_status grasp_create_hand(grasp_ctx* ctx, const grasp_hand_desc* desc, grasp_hand_id* out);
/* EBUSY while a live job uses the hand. */
grasp_status grasp_destroy_hand(grasp_ctx* ctx, grasp_hand_id hand);

/* Writes host out[n_contacts]: the link of each contact in caller order, as
 * the device holds it (exact copy of the description's contact_link). */
grasp_status grasp_hand_contact_links(grasp_ctx* ctx, grasp_hand_id hand, int32_t* out);

/* ---------------------------------------------------------------------------
 * Objects: a signed-distance grid (Sec. III-A/B)
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t n;                 /* vertices per axis, 2..512 (cubic grid) */
  float lo[3];               /* position of vertex (0,0,0) */
  float h;                   /* vertex spacing, > 0: vertex (i,j,k) at lo + (i,j,k) h */
  const float* values;       /* host [n][n][n], x fastest: index (k n + j) n + i; negative inside */
  float inertia_over_mass;   /* I/m of the isotropic object; <= 0 selects 2/5 R_eq^2 with
                                R_eq^3 = 3 V / (4 pi), V = h^3 #{vertices with value < 0} */
  int32_t layout;            /* GRASP_LAYOUT_*: the device gather copy of the grid */
} grasp_sdf_desc;

enum {
  GRASP_LAYOUT_AUTO = 0,     /* yz-quads */
  GRASP_LAYOUT_YZQUADS = 1,  /* (phi(i,j,k), phi(i,j+1,k), phi(i,j,k+1), phi(i,j+1,k+1)) per vertex, 16
                                bytes: a cell's 8 corners are 32 contiguous bytes of one row, so the seven
                                tests of a contact touch few cache lines; 4x the grid */
  GRASP_LAYOUT_ZPAIRS = 2    /* (phi(i,j,k), phi(i,j,k+1)) per vertex: two rows per sample, 2x the grid */
};

/* Copies the grid to the device with a gather copy in the chosen layout.
 * Samples are identical in every layout; only speed differs.
 * EINVAL when the object has no interior and inertia_over_mass <= 0, or for
 * an unknown layout. */
grasp_status grasp_load_sdf(grasp_ctx* ctx, const grasp_sdf_desc* desc, grasp_sdf_id* out);
/* EBUSY while a live job uses the grid. */
grasp_status grasp_unload_sdf(grasp_ctx* ctx, grasp_sdf_id sdf);
/* Host out: the I/m the library uses for this grid. */
grasp_status grasp_sdf_inertia(grasp_ctx* ctx, grasp_sdf_id sdf, float* out);

/* ---------------------------------------------------------------------------
 * Mesh objects (Sec. III-B): the Phong signed distance of a closed triangle
 * mesh, rho(r) = s(r) |r - p| with p the closest point r* of the mesh moved
 * towards the curved (Phong) triangle, p = (1 - alpha) r* + alpha sum_b w_b
 * psi_b(r*) (w_b the barycentric weights of r*, psi_b the projection onto the
 * tangent plane of vertex b), s = -1 inside; grad rho = (r - p) / rho.
 * ------------------------------------------------------------------------- */
typedef uint64_t grasp_mesh_id;

typedef struct {
  int32_t n_vertices;       /* 3 .. 2^24 */
  const float* vertices;    /* host [n_vertices][3], object frame */
  const float* normals;     /* host [n_vertices][3] unit vertex normals of the Phong surface, or NULL for
                               the angle-weighted normals of the incident faces */
  int32_t n_faces;          /* 4 .. 2^22 */
  const int32_t* faces;     /* host [n_faces][3] vertex indices, counter-clockwise seen from outside; the
                               mesh must be closed: every edge shared by exactly two faces, traversed in
                               opposite directions; no face of zero area */
  float alpha;              /* Phong blend in [0, 1]; 0 is the flat mesh */
} grasp_mesh_desc;

/* Builds a bounding-volume hierarchy on the host and copies it to the device.
 * EINVAL for a mesh that is not closed and consistently oriented outward (its
 * enclosed volume must be positive), a degenerate face, an index out of range,
 * a non-finite coordinate or alpha outside [0, 1]; ENOMEM when the arena is
 * full. */
grasp_status grasp_load_mesh(grasp_ctx* ctx, const grasp_mesh_desc* desc, grasp_mesh_id* out);
grasp_status grasp_unload_mesh(grasp_ctx* ctx, grasp_mesh_id mesh);

/* Phong signed distance at n points r (dev [n][3], object frame): out (dev
 * [n][4]) = rho, grad rho. A non-finite point gives NaN. Asynchronous on
 * hip_stream. */
grasp_status grasp_mesh_sample(grasp_ctx* ctx, grasp_mesh_id mesh, int32_t n, const float* r, float* out,
                               void* hip_stream);

/* Debugging and tests: the sample the mesh step (grasp_step_fused_mesh) takes
 * at n points r (dev [n][3]): out (dev [n][8]) = rho, the stated normal
 * (r - p) / rho, the exact gradient of rho through the closest point and the
 * Phong point, and the closest feature's region (0 face interior, 1 edge,
 * 2 vertex). Asynchronous on hip_stream. */
grasp_status grasp_debug_mesh_step_sample(grasp_ctx* ctx, grasp_mesh_id mesh, int32_t n, const float* r,
                                          float* out, void* hip_stream);

typedef struct {
  int32_t n;                /* vertices per axis, 2..512 */
  float lo[3];              /* position of vertex (0,0,0) */
  float h;                  /* vertex spacing, > 0 */
  float inertia_over_mass;  /* <= 0: 2/5 R_eq^2 with R_eq^3 = 3 V / (4 pi), V the mesh's volume */
  int32_t layout;           /* GRASP_LAYOUT_* of the gather copy */
} grasp_mesh_grid_desc;

/* Samples the mesh's Phong signed distance at the n^3 grid vertices on the
 * device and loads the result as an SDF grid (the same object as
 * grasp_load_sdf with those values), usable by every step form. */
grasp_status grasp_load_sdf_from_mesh(grasp_ctx* ctx, grasp_mesh_id mesh, const grasp_mesh_grid_desc* desc,
                                      grasp_sdf_id* out);

/* ---------------------------------------------------------------------------
 * Post-synthesis evaluation (Sec. V-A metrics). The paper reports contact area
 * (CA) at a distance threshold (2, 5 and 9 mm in its figures) and
 * intersection volume (IV) of the top-10 grasps. Read as integrals over the
 * hand estimated from weighted samples: CA(tau) = total area of the surface
 * samples whose signed distance to the object (at rest) is below tau,
 * penetrating ones included; IV = total volume of the volume samples whose
 * signed distance is below 0. Samples are placed by the hand's forward
 * kinematics and read through the grid's trilinear value, as in the step.
 * ------------------------------------------------------------------------- */
typedef uint64_t grasp_eval_id;

#define GRASP_MAX_THRESHOLDS 8
#define GRASP_MAX_TOP 64

typedef struct {
  int32_t n_surface;            /* surface samples, 0 .. 2^24 */
  const int32_t* surface_link;  /* host [n_surface], each in [0, n_links) */
  const float* surface_local;   /* host [n_surface][3] in the frame of the link */
  const float* surface_area;    /* host [n_surface] area each stands for (m^2), finite, >= 0 */
  int32_t n_volume;             /* volume samples, 0 .. 2^24; n_surface + n_volume >= 1 */
  const int32_t* volume_link;   /* host [n_volume] */
  const float* volume_local;    /* host [n_volume][3] */
  const float* volume_weight;   /* host [n_volume] volume each stands for (m^3), finite, >= 0 */
} grasp_eval_desc;

/* Copies a hand's weighted samples to the device (each set sorted by link;
 * the sums do not depend on the order). The set belongs to the hand: it is
 * usable while the hand exists. EINVAL on a bad count, link, coordinate or
 * weight; ENOMEM when the arena is full. */
grasp_status grasp_load_eval_points(grasp_ctx* ctx, grasp_hand_id hand, const grasp_eval_desc* desc,
                                    grasp_eval_id* out);
/* EBUSY while a served job that names the set has not ended. */
grasp_status grasp_unload_eval_points(grasp_ctx* ctx, grasp_eval_id ev);

/* Metrics of B candidates q (dev [B][n_dof]) against the grid: out (dev
 * [B][n_thr + 1]) = CA at thresholds[0 .. n_thr) (host, metres, finite,
 * 1 <= n_thr <= GRASP_MAX_THRESHOLDS), then IV. A candidate with a
 * non-finite coordinate gets NaN in every column. Asynchronous on hip_stream. */
grasp_status grasp_evaluate(grasp_ctx* ctx, grasp_eval_id ev, grasp_sdf_id sdf, int32_t B, const float* q,
                            int32_t n_thr, const float* thresholds, float* out, void* hip_stream);

/* The same metrics against a mesh object's Phong signed distance (Sec. III-B;
 * the mesh as loaded by grasp_load_mesh, at rest) instead of a grid: each
 * sample through the hierarchy query, walked once per wave for 64 samples of
 * one candidate. Errors and layouts as grasp_evaluate. */
grasp_status grasp_evaluate_mesh(grasp_ctx* ctx, grasp_eval_id ev, grasp_mesh_id mesh, int32_t B, const float* q,
                                 int32_t n_thr, const float* thresholds, float* out, void* hip_stream);

/* The k best of B candidates by key (dev [B]): ascending, or descending when
 * higher_is_better; NaN keys after every other; equal keys (-0 equal to +0) in
 * index order. top (dev [k]) gets their indices, best first; mean (dev [M], or
 * NULL when M = 0) the average of metrics (dev [B][M]) over them, summed in
 * FP64 in rank order. 1 <= k <= min(B, GRASP_MAX_TOP), B <= 2^24, M >= 0. The
 * paper ranks by the epsilon metric, which is not computed here: any key can
 * be given, for instance the final loss. Asynchronous on hip_stream; one
 * workgroup, k passes over the keys. */
grasp_status grasp_select_top(grasp_ctx* ctx, int32_t B, const float* key, int32_t higher_is_better, int32_t k,
                              int32_t M, const float* metrics, int32_t* top, float* mean, void* hip_stream);

/* ---------------------------------------------------------------------------
 * The step (Sec. III-C, Sec. IV-A)
 * ------------------------------------------------------------------------- */
typedef struct {
  float dt;          /* PBD time step, 1e-3 s in the paper */
  float v0;          /* test speed (m/s): initial object velocities +x,-x,+y,-y,+z,-z,0 times v0 */
  int32_t K;         /* projection iterations inside the one step, >= 1 */
  int32_t ckpt_every;/* pose checkpoint interval for the backward, divides K (1 = keep all) */
  float omega;       /* relaxation of the summed (Jacobi) corrections, default 1 */
  float r_dil;       /* SDF dilation radius of this step (Sec. III-B), >= 0 */
  float alpha_leak;  /* leaky-gradient factor (Sec. III-C), 0.1 in the paper; 0 = exact */
  float w_stable, w_pen, w_range, w_limit; /* loss weights */
  float w_min;       /* constraints with J M^-1 J^T <= w_min are skipped (1e-8: below it the trilinear
                        gradient is single-precision rounding noise) */
  int32_t mode;      /* GRASP_MODE_*: how grasp_step_fwd/bwd share state */
  int32_t projection;/* GRASP_PROJECTION_*: how the constraint corrections combine */
  float mu;          /* Coulomb friction coefficient, >= 0 (0: frictionless). The paper's projection
                        includes friction (Sec. III-C) by a cited model; read as positional friction:
                        each active contact's tangential displacement over the step (of the object's
                        point at the contact, dp_t = dp - (dp . n) n, n = g / |g|) is removed up to
                        mu C, wholly while |dp_t| <= mu C (static), by mu C beyond (kinetic), as the
                        Eq. (1) correction of a positional constraint along dp_t / |dp_t|, averaged
                        with the normal corrections; dp = p - r, the hand point minus its
                        object-frame coordinates at the iteration's pose. mu > 0 needs the averaged
                        projection (EINVAL otherwise); the plain form and the mesh step refuse it. */
} grasp_step_params;

/* Projection of the contact constraints (Sec. III-C). AVERAGED (default): every
 * Eq. (1) correction at the same pose, their sum divided by the number of
 * active constraints of the test; every step form. GAUSS_SEIDEL: the paper's
 * serial form, each constraint at the pose the previous ones left, in
 * link-major order (contacts stable-sorted by link); grasp_step_fwd, _bwd and
 * _fused, and served jobs (each stepped by a fused launch of its own; the
 * batched launch refuses it); K iterations are K sweeps. No workspace: the
 * backward replays the sweeps from their start poses, 168 K bytes per
 * candidate and 64-contact chunk, which the context keeps in its arena
 * (ENOMEM when they do not fit); a served job keeps its own table in its
 * arena block, counted in its footprint at admission. */
#define GRASP_PROJECTION_AVERAGED 0
#define GRASP_PROJECTION_GAUSS_SEIDEL 1

enum {
  GRASP_MODE_AUTO = 0,      /* SAVE when a workspace is given, else RECOMPUTE */
  GRASP_MODE_SAVE = 1,      /* fwd stores pose checkpoints in the workspace, bwd reads them */
  GRASP_MODE_RECOMPUTE = 2  /* bwd recomputes the forward (FK, samples, corrections) */
};

/* Fills p with the defaults above (dt 1e-3, v0 1, K 1, ckpt 1, omega 1, r_dil 0,
 * alpha 0.1, weights 1 / 1e4 / 1e-2 / 1, w_min 1e-8, AUTO, averaged, mu 0). */
void grasp_default_params(grasp_step_params* p);

/* Host out: workspace bytes grasp_step_fwd/bwd need for B candidates in SAVE
 * mode (pose checkpoints and per-iteration active-constraint counts,
 * 168 (K/ckpt + 1) + 28 K bytes per candidate). */
grasp_status grasp_step_workspace_bytes(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                                        const grasp_step_params* p, int32_t B, size_t* out);

/* Forward: loss (dev [B]) and terms (dev [B][4] = L_stable, L_pen, L_range,
 * L_limit, or NULL) for configurations q (dev [B][n_dof]). In SAVE mode ws
 * (dev, ws_bytes from grasp_step_workspace_bytes) receives the pose
 * checkpoints the backward reads; otherwise ws may be NULL. A candidate
 * whose q has a NaN or Inf entry gets a NaN loss (every form).
 * ENOMEM if ws_bytes is too small for SAVE. */
grasp_status grasp_step_fwd(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                            const grasp_step_params* p, int32_t B, const float* q, float* loss,
                            float* terms, void* ws, size_t ws_bytes, void* hip_stream);

/* Backward: dq (dev [B][n_dof]) = dloss[b] * dL_b/dq_b with the leaky rule,
 * for dloss dev [B] (NULL = all ones). Same q, p, ws as the forward. */
grasp_status grasp_step_bwd(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                            const grasp_step_params* p, int32_t B, const float* q, const float* dloss,
                            float* dq, void* ws, size_t ws_bytes, void* hip_stream);

/* Bias-corrected Adam on n values in place (dev q, m, v; dev g), step t >= 1. */
grasp_status grasp_adam_step(grasp_ctx* ctx, int32_t n, float* q, float* m, float* v, const float* g,
                             int32_t t, float lr, float b1, float b2, float eps, void* hip_stream);

/* One fused optimizer step in a single launch: forward, backward and Adam
 * for B candidates. q, m, v (dev [B][n_dof]) are updated in place; loss,
 * terms, dq (dev) are written when not NULL (loss/terms before the update).
 * t >= 1 is the Adam step number. */
grasp_status grasp_step_fused(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                              const grasp_step_params* p, int32_t B, float* q, float* m, float* v,
                              int32_t t, float lr, float b1, float b2, float eps, float* loss,
                              float* terms, float* dq, void* hip_stream);

/* The fused step on a mesh object (Sec. III-B's Phong signed distance as the
 * constraint's rho, Sec. III-C): the samples query the mesh through its
 * hierarchy instead of a grid. With one iteration the forward records every
 * sample's nearest face in a context buffer (B x 7 x n_contacts ints from the
 * arena, kept and reused, shared by streams in launch order) and the adjoint
 * reuses it; under stream capture or without room in the arena both passes
 * walk, and the forward skips a sample whose distance to the mesh's box, less
 * alpha times the longest edge, clears r_dil (it adds exactly nothing there).
 * The results are the same bits either way. Each wave walks the hierarchy
 * once for its 63 samples, all of one candidate, so a candidate's result
 * depends on its own inputs only. The constraint normal is
 * (r - p) / rho the paper states and, in the adjoint, the exact derivative of
 * rho and of that normal through the closest point (face interior, edge or
 * vertex) and the Phong point. Arguments as grasp_step_fused, with the mesh
 * of grasp_load_mesh and the object's I/m (<= 0: 2/5 R_eq^2 from the mesh's
 * volume). The averaged projection only (EINVAL for Gauss-Seidel), mu = 0
 * (EINVAL otherwise); no locality order or tile choice: two candidates per
 * workgroup. Asynchronous on hip_stream. */
grasp_status grasp_step_fused_mesh(grasp_ctx* ctx, grasp_hand_id hand, grasp_mesh_id mesh,
                                   const grasp_step_params* p, float inertia_over_mass, int32_t B, float* q,
                                   float* m, float* v, int32_t t, float lr, float b1, float b2, float eps,
                                   float* loss, float* terms, float* dq, void* hip_stream);

/* Debugging and tests: the forward pass of grasp_step_fused_mesh with the
 * trace of grasp_debug_trace (contact points, poses, per-sample d, g, w,
 * lambda), in the same layouts. */
grasp_status grasp_debug_trace_mesh(grasp_ctx* ctx, grasp_hand_id hand, grasp_mesh_id mesh,
                                    const grasp_step_params* p, float inertia_over_mass, int32_t B, const float* q,
                                    float* p_world, float* poses, float* samples, void* hip_stream);

/* grasp_step_fused for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same step, bit for bit, with the candidate locality order kept in a
 * fixed device array of the library (1 MiB per GPU, held until the process
 * ends) instead of the context's arena. It calls no hipMalloc, hipFree or
 * allocating routine, and can be captured into a graph (the order is computed
 * inside the captured work). Limits: B <= 262144 (EINVAL above), averaged
 * projection only (EINVAL for Gauss-Seidel, whose start-pose table needs
 * memory). Every call on one GPU shares that array: calls that overlap on one
 * GPU (different streams, or concurrent graph replays) race and must be
 * serialized by the caller. */
grasp_status grasp_step_fused_static(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                                     const grasp_step_params* p, int32_t B, float* q, float* m, float* v, int32_t t,
                                     float lr, float b1, float b2, float eps, float* loss, float* terms, float* dq,
                                     void* hip_stream);

/* ---------------------------------------------------------------------------
 * The plain per-job form: the same step (K = 1) as one unfused kernel per
 * stage (link transforms, contact points, SDF samples, summed corrections,
 * losses, contact adjoints, link sums, tree sweep, Adam) with every
 * intermediate in the workspace. It is the baseline the fused and batched
 * forms are measured against.
 * ------------------------------------------------------------------------- */

/* Host out: workspace bytes of grasp_plain_step for B candidates (EINVAL unless K = 1). */
grasp_status grasp_plain_workspace_bytes(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                                         const grasp_step_params* p, int32_t B, size_t* out);

/* One optimizer step of B candidates: loss (dev [B]) and terms (dev [B][4]
 * or NULL) at q, then Adam on q, m, v (dev [B][n_dof], in place) with step
 * number t. ws: dev, 64-byte aligned, ws_bytes from grasp_plain_workspace_bytes
 * (ENOMEM if smaller). */
grasp_status grasp_plain_step(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                              int32_t B, float* q, float* m, float* v, int32_t t, float lr, float b1, float b2,
                              float eps, float* loss, float* terms, void* ws, size_t ws_bytes, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Launch-shape tuning. A tile is the step kernel's launch shape; every tile
 * computes bit-identical results, only speed differs.
 * ------------------------------------------------------------------------- */
/* Launch shape of the step kernels. Where none is tuned or set: two
 * candidates per workgroup at four waves per SIMD for one projection
 * iteration, one at four for several. Every shape gives the same bits. */
typedef struct {
  int32_t waves_per_block;     /* candidates per workgroup: 1, 2 or 4 */
  int32_t min_waves_per_simd;  /* register budget: 1 (compiler's choice) .. 6 */
} grasp_tile;

/* Times every tile on a private copy of q (dev [B][n_dof]) with reps fused
 * steps each, keeps the fastest for this shape (hand, grid, K, B) in the
 * context, and returns it (host best, best_ms = ms per fused step). q is not
 * modified. Tiles are also persisted to the file named by the environment
 * variable GRASP_TUNE_CACHE when it is set. */
grasp_status grasp_tune(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                        int32_t B, const float* q, int32_t reps, grasp_tile* best, float* best_ms);

/* Pins a tile for this shape (overrides the tuner). EINVAL on a bad tile. */
grasp_status grasp_set_tile(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                            int32_t B, const grasp_tile* tile);

/* ---------------------------------------------------------------------------
 * The batched form: many jobs, each its own hand, grid, candidate count and
 * schedule position, advance one optimizer step in a single launch over a
 * device job table (batching amortizes launch and tail cost, Sec. V-C reports
 * the amortized time per grasp). On a non-default stream the launch is
 * captured once per launch shape in a hipGraph and replayed every step.
 * Each candidate is computed exactly as grasp_step_fused computes it, so a
 * job's results do not depend on the other jobs in the step.
 * ------------------------------------------------------------------------- */
typedef struct {
  grasp_hand_id hand;
  grasp_sdf_id sdf;
  grasp_step_params p;   /* p.r_dil is replaced by the schedule r0 (1 - t/(T-1)) */
  int32_t B;             /* candidates, >= 1 */
  float* q;              /* dev [B][n_dof], updated in place */
  float* m;              /* dev [B][n_dof] Adam moments, updated in place */
  float* v;
  float* loss;           /* dev [B] or NULL: loss at the start of the step */
  float* terms;          /* dev [B][4] or NULL */
  float* dq;             /* dev [B][n_dof] or NULL: the gradient the step's Adam update used */
  int32_t t;             /* optimizer steps already taken; the call runs Adam step t + 1
                            and increments t */
  int32_t T;             /* schedule length (dilation reaches 0 at t = T - 1) */
  float r0;              /* initial dilation radius */
  float lr, b1, b2, eps; /* Adam */
} grasp_batch_job;

typedef struct grasp_batch grasp_batch; /* opaque */

/* A batch able to hold up to capacity candidates in max_jobs jobs per step.
 * use_graph = 0 launches eagerly. Allocates its job table in the arena. */
grasp_status grasp_batch_create(grasp_ctx* ctx, int32_t capacity, int32_t max_jobs, int32_t use_graph,
                                grasp_batch** out);
grasp_status grasp_batch_destroy(grasp_batch* batch);
/* Launch shape of the batched kernel (see grasp_tile). */
grasp_status grasp_batch_set_tile(grasp_batch* batch, const grasp_tile* tile);
/* One optimizer step for every job (host array jobs[n]; each job's t is
 * incremented). The call waits for the previous step of this batch before
 * rewriting the table, then queues the step on hip_stream. */
grasp_status grasp_batch_step(grasp_batch* batch, grasp_batch_job* jobs, int32_t n, void* hip_stream);
/* Host out[n]: per job (in the order of the last step's array) whether a loss
 * was not finite since the previous call; clears the flags. Synchronous. */
grasp_status grasp_batch_flags(grasp_batch* batch, int32_t n, int32_t* out);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of grasp jobs (Sec. V-C contrasts the online
 * and the amortized time per grasp). A scheduler thread owned by the context
 * admits queued jobs at step boundaries, first come first served, when their
 * device footprint (q, m, v, loss, terms: 12 B n_dof + 20 B per candidate)
 * fits the arena and the candidate capacity; advances every resident job by
 * one optimizer step per batched launch; and retires a job after its T steps
 * with one forward at r_dil = 0 (final loss, terms) and the ranking, freeing
 * its memory. Hands and grids stay resident and are shared between jobs. A
 * job may also name an evaluation set of its hand: it then retires with the
 * post-synthesis metrics of every candidate at its final configuration and,
 * with top_k > 0, the top_k best by final loss and their mean metrics (the
 * paper's top-10 figures); the set cannot be unloaded while such a job lives
 * (EBUSY, as for its hand and grid), and the job's footprint grows by
 * 4 (n_thr + 1) bytes per candidate.
 * ------------------------------------------------------------------------- */
typedef struct {
  grasp_hand_id hand;
  grasp_sdf_id sdf;
  int32_t B;             /* candidates, >= 1 */
  const float* q0;       /* host [B][n_dof] initial configurations, copied by grasp_submit */
  int32_t T;             /* optimizer steps, >= 1 */
  float r0;              /* initial dilation; r(t) = r0 (1 - t/(T-1)) */
  grasp_step_params p;   /* p.r_dil is ignored */
  float lr, b1, b2, eps; /* Adam */
  grasp_eval_id eval;    /* evaluation set of the job's hand (grasp_load_eval_points), or 0 for none */
  int32_t n_thr;         /* with eval: contact-area thresholds in thresholds[], 1..GRASP_MAX_THRESHOLDS */
  float thresholds[GRASP_MAX_THRESHOLDS]; /* metres, finite */
  int32_t top_k;         /* with eval: 0..min(B, GRASP_MAX_TOP); without: 0 */
  int32_t record_history;/* 1: keep q before and the loss at every step (host memory, 4 B (n_dof + 1)
                            per candidate and step), returned through hist_q / hist_loss */
} grasp_job_desc;

typedef struct {
  grasp_status status;   /* GRASP_OK, GRASP_ENONFINITE or GRASP_ECANCELED */
  float* q;              /* host [B][n_dof] final configurations, caller-owned, or NULL */
  float* loss;           /* host [B] final loss at r_dil = 0, or NULL */
  float* terms;          /* host [B][4], or NULL */
  int32_t* rank;         /* host [B]: candidate indices by ascending final loss (ties by index), or NULL */
  double t_submit, t_admit, t_done; /* seconds since grasp_init */
  int32_t steps;         /* optimizer steps the job took */
  float* metrics;        /* host [B][n_thr + 1]: contact areas and intersection volume at the final q (jobs
                            with an evaluation set), or NULL */
  int32_t* top;          /* host [top_k]: the best candidates by final loss, best first, or NULL */
  float* top_mean;       /* host [n_thr + 1]: their mean metrics, or NULL */
  float* hist_q;         /* host [T][B][n_dof] or NULL: with record_history, q before each step taken (rows
                            past `steps` untouched) */
  float* hist_loss;      /* host [T][B] or NULL: with record_history, the loss at the start of each step
                            (at that step's dilation) */
} grasp_job_result;

/* Sets the scheduler's candidate capacity per step (default 65536) and job
 * limit (default 256); only before the first grasp_submit. */
grasp_status grasp_serve_config(grasp_ctx* ctx, int32_t capacity, int32_t max_jobs);
/* Queues a job (thread-safe, non-blocking). ENOMEM if the job can never fit
 * (footprint > arena or B > capacity); EINVAL on bad ids or parameters. */
grasp_status grasp_submit(grasp_ctx* ctx, const grasp_job_desc* job, grasp_job_id* out);
/* GRASP_EAGAIN while the job is queued or running. Once it has ended, copies
 * its results into the caller's buffers in *inout, returns its final status
 * and forgets the job (a second poll returns EINVAL). Thread-safe. */
grasp_status grasp_poll(grasp_ctx* ctx, grasp_job_id job, grasp_job_result* inout);
/* Asks the scheduler to stop a job at the next step boundary (it then ends
 * with GRASP_ECANCELED). EINVAL for an unknown or already polled job. */
grasp_status grasp_cancel(grasp_ctx* ctx, grasp_job_id job);

typedef struct {
  int64_t steps;          /* batched launches so far */
  int64_t contact_evals;  /* sum over steps of resident candidates x contacts x 7 x K */
  int32_t queued, resident, finished;
} grasp_serve_stats;
grasp_status grasp_serve_stats_get(grasp_ctx* ctx, grasp_serve_stats* out);

/* ---------------------------------------------------------------------------
 * Parity introspection (tests)
 * ------------------------------------------------------------------------- */

/* Samples the grid at n points r (dev [n][3], object frame): out (dev [n][4] =
 * phi, grad phi) and hess (dev [n][9] row-major d grad/dr, or NULL). */
grasp_status grasp_debug_sdf_sample(grasp_ctx* ctx, grasp_sdf_id sdf, int32_t n, const float* r,
                                    float* out, float* hess, void* hip_stream);

/* Forward trace of the step, caller contact order: p_world (dev [B][Nc][3]
 * or NULL), poses (dev [B][7][K+1][6] = x, theta before each iteration and
 * after the last, or NULL), samples (dev [B][7][K][Nc][6] = d, g, w, lambda,
 * or NULL). */
grasp_status grasp_debug_trace(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                               const grasp_step_params* p, int32_t B, const float* q, float* p_world,
                               float* poses, float* samples, void* hip_stream);

/* Runs one fused step without Adam (q, m, v untouched; no loss or dq written)
 * and adds to groups (dev [2], uint64) the number of sample groups (9 contacts
 * x 7 tests) its forward passes gathered, and the number of groups those
 * passes hold. The rest were skipped as provably clear of the dilated surface
 * (Eq. (1): they contribute no correction). Counts are exact and independent
 * of the launch shape. Errors as grasp_step_fused. */
grasp_status grasp_debug_forward_groups(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf,
                                        const grasp_step_params* p, int32_t B, const float* q,
                                        uint64_t* groups, void* hip_stream);

#pragma GCC visibility pop
#ifdef __cplusplus
}
#endif
#endif /* GRASP_H */
