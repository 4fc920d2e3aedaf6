/*
 * tacsl.h -- C-ABI of libtacsl, the MI355X (gfx950) tactile force field.
 *
 * The library evaluates the penalty-based tactile force field of the TacSL
 * paper, Section III-C ("Normal/Shear Force-Field Computation"): for every
 * tactile point ("taxel") of every elastomer pad, in every simulated
 * environment at once, it
 *   1. moves the taxel into the object frame,
 *   2. queries the object's voxelized signed-distance field (SDF) with
 *      trilinear interpolation to get the interpenetration distance d,
 *   3. takes the contact normal n from finite-difference gradients of the SDF,
 *   4. applies  f_n = (-k_n + k_d d_dot) d n  and
 *      f_t = -(v_t/|v_t|) min(k_t |v_t|, mu |f_n|),  d_dot = n . x_dot,
 *   5. writes per-taxel depth, normal and forces and each pad's net force and
 *      torque.
 * The SDFs are computed before simulation and queried every step (Section
 * III-C); the force field is a post-processing step after each dynamics step
 * (notation appendix); contact parameters are randomized per environment
 * (Section V-A, Appendix C); each environment may hold several pads (two
 * fingers, Section V-B).
 *
 * Conventions (all entry points)
 *  - Units: metres, seconds, newtons.  FP32 inputs and outputs.
 *  - Poses: [qw qx qy qz tx ty tz], world frame; quaternions need not be
 *    normalized (they are normalized internally in FP64).
 *  - Twists: [vx vy vz wx wy wz], world frame; v is the velocity of the body
 *    origin.
 *  - Signed distance: negative inside the object.  d = phi; contact where
 *    phi < 0 inside the grid's node box; the reported depth is -phi >= 0.
 *    n = normalized finite-difference gradient, pointing out of the object.
 *    x_dot = velocity of the taxel minus velocity of the coincident object
 *    point.  v_t = x_dot - (n . x_dot) n.  When |grad| < 1e-6 the normal and
 *    both forces are zero.
 *  - Outputs are in the pad frame; torque is about the pad origin.
 *  - Global taxel index = inst_offset[i] + k (instance-major; k indexes the
 *    instance's template).  tacsl_plan_offsets returns inst_offset.
 *  - Pointers marked "host" are read during the call; pointers marked
 *    "device" must stay valid while the plan (or graph) uses them.  The
 *    library never frees caller memory.
 *  - A plan's per-step buffers (prologue records, work-list order, queue,
 *    partial sums) are shared by its calls: calls on one plan must be ordered
 *    (one stream, or streams joined by events); overlapping calls race.
 *  - Every function returns an int status: TACSL_OK (0) or a negative
 *    tacsl_status code.  Host-side validation happens before any launch; on
 *    error nothing is launched and no output is touched.  Device-side
 *    anomalies are reported as bits in the optional device status word.
 *    No exception crosses the ABI and nothing aborts.
 */
#ifndef TACSL_H_
#define TACSL_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TACSL_ABI_VERSION 1

typedef enum {
  TACSL_OK = 0,
  TACSL_ERR_NULL_ARG = -1,     /* a required pointer is NULL */
  TACSL_ERR_SHAPE = -2,        /* counts/offsets inconsistent (non-monotone, negative, empty grid) */
  TACSL_ERR_RANGE = -3,        /* an id or value out of range (bad index, spacing <= 0, non-finite) */
  TACSL_ERR_HIP = -4,          /* a HIP runtime call failed */
  TACSL_ERR_ALLOC = -5,        /* device or host allocation failed (plan creation only) */
  TACSL_ERR_UNSUPPORTED = -6,  /* valid but beyond this build's limits (grid copy >= 4 GiB, ...) */
  TACSL_ERR_STATE = -7         /* call not valid for this object (e.g. graph of a destroyed plan) */
} tacsl_status;

/* Bits OR-ed into tacsl_outputs.status / tacsl_grads.status by the kernels. */
#define TACSL_DEV_NONFINITE_POSE 0x1u /* a pose, twist or parameter is NaN/Inf: that pad outputs zeros */
#define TACSL_DEV_ZERO_QUAT 0x2u      /* a quaternion has zero norm: that pad outputs zeros */
#define TACSL_DEV_BAD_CONTACT 0x4u    /* tacsl_contact_impulse: an invalid contact (see there) got lambda = 0 */
#define TACSL_DEV_DEPTH_CAPPED 0x8u   /* tacsl_depth_image: a ray hit the iteration limit; it reads the gel surface */

/* Scene: everything that stays fixed across steps.  Read at plan creation.
 *   n_env   environments (>= 0); n_inst pads (instances, >= 0);
 *   n_tmpl  pad templates; n_sdf object grids.
 *   inst_env  host [n_inst]    environment of each pad, in [0, n_env)
 *   inst_tmpl host [n_inst]    template of each pad, in [0, n_tmpl)
 *   env_sdf   host [n_env]     object grid of each environment, in [0, n_sdf)
 *   tmpl_offset host [n_tmpl+1] prefix sums of template sizes; [0] = 0, non-decreasing
 *   tmpl_xyz  device [3][T_tmpl] FP32 SoA taxel positions in the pad frame
 *             (T_tmpl = tmpl_offset[n_tmpl]); the pad plane faces +z towards the object
 *   sdf_dims  host [n_sdf][3]  nodes per axis (nx, ny, nz), each >= 2; the plan's copy
 *             (16 bytes per node, x and y rounded up to even, plus a ~0.1% bit mask) must stay
 *             below 4 GiB, i.e. up to 644^3, and 64 ceil(ny/2) nz below 2^24 (ceil(ny/2) nz < 262144,
 *             e.g. 724 x 723); else TACSL_ERR_UNSUPPORTED
 *   sdf_origin host [n_sdf][3] position of node (0,0,0) in the object frame
 *   sdf_spacing host [n_sdf]   isotropic node spacing h > 0
 *   sdf_offset host [n_sdf]    element offset of each grid in sdf_data
 *   sdf_data  device           node values (FP32 metres), x fastest: (k*ny + j)*nx + i
 * The plan copies what it needs: tmpl_xyz and sdf_data are only read at plan
 * creation.  Taxels are visited in template order, 64 consecutive ones per
 * wavefront: numbering a template in compact blocks (e.g. 8 x 8 tiles of a
 * grid) keeps each wavefront's SDF gathers on few cache lines. */
typedef struct {
  int32_t n_env, n_inst, n_tmpl, n_sdf;
  const int32_t* inst_env;
  const int32_t* inst_tmpl;
  const int32_t* env_sdf;
  const int64_t* tmpl_offset;
  const float* tmpl_xyz;
  const int32_t* sdf_dims;
  const float* sdf_origin;
  const float* sdf_spacing;
  const int64_t* sdf_offset;
  const float* sdf_data;
} tacsl_scene_desc;

/* Launch shape and work-list choices (chosen by the autotuner).
 *   block        threads per workgroup: 64, 128, 256 or 512 (0 -> 256)
 *   tile_taxels  taxels per tile; 0 -> one tile per pad; else >= 64
 *   schedule     0: one workgroup per tile; 1: persistent workgroups, static
 *                stride over the tile list; 2: persistent, dynamic queue
 *   grid         persistent workgroups for schedules 1-2 (0 -> 8 per CU)
 *   order        0: instance-major; 1: XCD-aware (tiles of one object grid
 *                kept on one XCD's L2); 2: longest tiles first; 3: object-major
 *                (the whole GPU on one object grid at a time); 4: object-major
 *                with each XCD on a contiguous run of the object's tiles;
 *                5: as 4 with the pads in a spatial order rebuilt on the device
 *                every call (pads binned by object grid and by the 8 x 8 x 8
 *                coarse cell of their origin in the grid, Morton order); any
 *                other value is TACSL_ERR_RANGE.  The order changes no output
 *                (per-taxel outputs are bitwise independent of the tuning). */
typedef struct {
  int32_t block, tile_taxels, schedule, grid, order;
} tacsl_tuning;

/* Per-step state (device, FP32).  obj_pose_delta may be NULL; when given the
 * object pose used is R_o <- Exp(dtheta) R_o, t_o <- t_o + dt (world frame),
 * the perturbation the pose gradient is taken against.
 *   pad_pose [n_inst][7], obj_pose [n_env][7], pad_twist [n_inst][6],
 *   obj_twist [n_env][6], params [n_env][4] = (k_n, k_d, k_t, mu),
 *   obj_pose_delta [n_env][6] = (dt, dtheta). */
typedef struct {
  const float* pad_pose;
  const float* obj_pose;
  const float* pad_twist;
  const float* obj_twist;
  const float* params;
  const float* obj_pose_delta;
} tacsl_state;

/* Outputs (device, FP32, caller-owned; T = total taxels):
 *   depth [T] (>= 0), normal [3][T], fn [3][T], ft [3][T] (pad frame),
 *   wrench [n_inst][6] = (F, torque about the pad origin), pad frame,
 *   status: optional device uint32 word; bits are OR-ed in, never cleared. */
typedef struct {
  float* depth;
  float* normal;
  float* fn;
  float* ft;
  float* wrench;
  uint32_t* status;
} tacsl_outputs;

/* Reverse mode of L = sum_k (w_fn[:,k] . f_n,k + w_ft[:,k] . f_t,k).
 *   w_fn, w_ft  device [3][T] upstream weights (dL/df_n, dL/df_t)
 *   g_obj_pose  device [n_env][6]: dL/d(dt, dtheta) of the object pose
 *               perturbation t_o <- t_o + dt, R_o <- Exp(dtheta) R_o (world),
 *               evaluated at the state's obj_pose_delta (0 when NULL)
 *   g_obj_twist device [n_env][6]: dL/d(v_o, w_o); the gradient w.r.t. the
 *               relative velocity of the pads is its negative
 *   g_params    device [n_env][4]: dL/d(k_n, k_d, k_t, mu)
 * Outputs are overwritten (not accumulated). */
typedef struct {
  const float* w_fn;
  const float* w_ft;
  float* g_obj_pose;
  float* g_obj_twist;
  float* g_params;
  uint32_t* status;
} tacsl_grads;

typedef struct {
  int64_t n_taxels;          /* T */
  int64_t n_tiles;
  int32_t n_env, n_inst;
  int32_t cu_count;          /* compute units of the plan's device */
  int32_t xcd_count;         /* XCDs assumed by the XCD-aware order */
  int64_t prepared_bytes;    /* device bytes of the prepared SDF pool */
  int64_t workspace_bytes;   /* device bytes of the plan's other buffers, as allocated at the call */
  tacsl_tuning tuning;       /* resolved tuning (defaults filled in) */
} tacsl_plan_info;

typedef struct tacsl_plan_s* tacsl_plan;
typedef struct tacsl_graph_s* tacsl_graph;

/* Version of this ABI (TACSL_ABI_VERSION). */
int tacsl_abi_version(void);

/* Human-readable name of a status code; never NULL. */
const char* tacsl_status_string(int status);

/* Host-only check of a scene description (no GPU needed).  Checks counts,
 * ids, offsets, grid sizes and spacings; does not dereference the device
 * pointers (only checks that they are non-NULL when needed). */
int tacsl_validate_scene(const tacsl_scene_desc* desc);

/* Host-only construction of the tile work list the plan would use (no GPU
 * needed), for inspection and tests.  Tiles are numbered instance-major:
 * tile t covers taxels [tile_k0[t], tile_k0[t] + tile_count[t]) of pad
 * tile_inst[t]; every pad has at least one tile (an empty pad has one tile of
 * 0 taxels).  exec_order[s] is the tile run in execution slot s (a
 * permutation).  Pass NULL arrays to query *n_tiles only; otherwise each
 * array holds max_tiles entries and TACSL_ERR_SHAPE is returned if the list
 * is longer.  xcd_count is the number of XCDs the order assumes (8 on MI355X). */
int tacsl_build_worklist(const tacsl_scene_desc* desc, const tacsl_tuning* tuning, int32_t xcd_count,
                         int64_t max_tiles, int64_t* n_tiles, int32_t* tile_inst, int32_t* tile_k0,
                         int32_t* tile_count, int32_t* exec_order);

/* Create a plan on the current HIP device: validates the scene, builds the
 * instance offsets and work list, and prepares the SDF pool (node values plus
 * central-difference gradients, one-sided on grid faces, re-laid out for the
 * gathers).  Allocates device memory and synchronizes; not for use inside
 * graph capture.
 * tuning may be NULL (defaults).  On error *out is NULL. */
int tacsl_plan_create(const tacsl_scene_desc* desc, const tacsl_tuning* tuning, tacsl_plan* out);

/* Replace the plan's tuning (rebuilds the work list; allocates; synchronizes). */
int tacsl_plan_set_tuning(tacsl_plan plan, const tacsl_tuning* tuning);

int tacsl_plan_get_info(tacsl_plan plan, tacsl_plan_info* info);

/* Copy the instance offsets (host int64 [n_inst+1]). */
int tacsl_plan_offsets(tacsl_plan plan, int64_t* host_inst_offset);

/* Forward force field (Section III-C, "Normal/Shear Force-Field
 * Computation": the SDF queried at every tactile point for the
 * interpenetration distance, the normal from finite-difference SDF
 * gradients, the penalty law for f_n and the Coulomb-capped f_t; run once
 * per simulation step as post-processing, notation appendix), enqueued on
 * `stream` (asynchronous; no allocation, no host synchronization, capturable
 * in a HIP graph).  All state and output pointers except obj_pose_delta and
 * status are required when n_inst > 0; outputs are overwritten.  Errors:
 * TACSL_ERR_NULL_ARG (plan, state, out or a required pointer NULL),
 * TACSL_ERR_HIP (a launch failed). */
int tacsl_force_field(tacsl_plan plan, const tacsl_state* state, const tacsl_outputs* out, hipStream_t stream);

/* Allocation-free forward, for callers that cannot allocate device memory
 * at call time (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same outputs as tacsl_force_field, bit for bit,
 * but the buffers a call writes and reads back (per-pad prologue records,
 * per-tile wrench partials, the dynamic-queue counter and, for order 5, the
 * spatial-order tables) come from one static device array of the library,
 * 16 MiB per GPU, held until the process ends, instead of the plan.  The call
 * allocates and frees nothing.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (any plans, any streams) race; order them.
 * The plan's device must be current.  Needs about
 * 100 n_pads + 24 n_tiles bytes (+ 4 kB per object grid, 4 bytes per pad and
 * 4 per tile for order 5).  Errors: as tacsl_force_field, plus
 * TACSL_ERR_UNSUPPORTED when the plan needs more scratch than that or its
 * device index is 64 or above, and TACSL_ERR_STATE when the plan's device is
 * not current. */
int tacsl_force_field_noalloc(tacsl_plan plan, const tacsl_state* state, const tacsl_outputs* out,
                              hipStream_t stream);

/* Force-field observation (the policy input of Section V-B: per finger a
 * small grid of bins with three channels).  For every pad and bin the
 * channels (|f_n|, f_t,x, f_t,y), pad frame, are averaged over the pad's
 * taxels in that bin, divided by scale[c] and clipped to [-clip, clip]
 * (clip <= 0: no clipping); a bin without taxels reads 0.
 *   n_bins    bins per pad, 1..TACSL_MAX_OBS_BINS (e.g. 14 x 10 = 140); 0 removes the observation
 *   tmpl_bin  host int32 [T_tmpl]: bin of each template taxel, -1 = in no bin
 *   scale     host float [3], finite and > 0
 * Allocates and synchronizes (not inside capture); TACSL_ERR_STATE while a
 * graph of the plan exists. */
#define TACSL_MAX_OBS_BINS 256
int tacsl_plan_set_observation(tacsl_plan plan, int32_t n_bins, const int32_t* tmpl_bin, const float* scale,
                               float clip);

/* Forward force field with the observation epilogue fused into the per-taxel
 * pass: writes obs (device float [n_inst][n_bins][3]) and the wrench, and the
 * per-taxel fields when out->depth, normal, fn and ft are all given; when all
 * four are NULL they are not written at all (observation only: no per-taxel
 * HBM traffic).  A mix of NULL and non-NULL fields is TACSL_ERR_NULL_ARG;
 * TACSL_ERR_STATE when no observation is set.  Same asynchrony rules as
 * tacsl_force_field; the observation is deterministic (fixed summation order). */
int tacsl_force_field_observe(tacsl_plan plan, const tacsl_state* state, const tacsl_outputs* out, float* obs,
                              hipStream_t stream);

/* Normal law of the plan: the penetration -phi enters the normal force as
 * (-phi)^p, f_n = (k_n - k_d d_dot) (-phi)^p n (damping scaled by the same
 * power), the nonlinear (Hunt-Crossley) variant named in Section VII; p = 1
 * (the default) is the law of Section III-C.  k_n is then in N/m^p and k_d in
 * N s/m^(p+1).  Applies to the forward, observation and adjoint passes (the
 * adjoint does not differentiate with respect to p).  exponent in [1, 4],
 * else TACSL_ERR_RANGE; TACSL_ERR_STATE while a graph of the plan exists
 * (graphs keep the exponent they were captured with).  Host only. */
int tacsl_plan_set_normal_law(tacsl_plan plan, float exponent);

/* Tactile camera for the depth image (Section III-B: a camera inside the
 * sensor renders the depth of the indenting object).  Pad frame, +z towards
 * the object; the gel fills z in [-gel, 0] and the camera sits behind it.
 *   rows, cols  image size, 1..4096 each; row r, column c looks through the
 *               pad-plane point (x0 + (c + 1/2) dx, y0 + (r + 1/2) dy, 0)
 *   ortho       1: rays parallel to +z; 0: pinhole at (0, 0, -cam_dist)
 *   dx, dy      pixel pitch on the pad plane (> 0), metres
 *   cam_dist    distance of the camera plane behind the pad plane, >= gel
 *   gel         gel thickness (> 0) */
typedef struct {
  int32_t rows, cols, ortho;
  float x0, y0, dx, dy;
  float cam_dist, gel;
} tacsl_camera;

/* Install (or with cam = NULL remove) the plan's tactile camera.  The first
 * call builds a copy of the object grids' node values laid out for the ray
 * march (4 bytes per node; allocates and synchronizes, not inside capture).
 * TACSL_ERR_RANGE for invalid values. */
int tacsl_plan_set_camera(tacsl_plan plan, const tacsl_camera* cam);

/* Tactile depth image of every pad: image (device float [n_inst][rows][cols])
 * receives, per pixel, the distance along +z from the camera plane to the
 * first point of the pixel's ray inside the gel where the object's trilinear
 * SDF is <= 0, or cam_dist (the undeformed gel surface) when the ray meets no
 * object inside the gel and the object's grid box.  An object reaching
 * below the gel reads cam_dist - gel.  The ray advances cell by cell:
 * sphere-tracing steps (with bounds on the field's slopes near the current
 * block of 8 x 8 x 8 cells) where they leave the current cell, else an exact search of the rest of the cell (the
 * field is a cubic along the ray, split at the roots of its derivative, the
 * first sign change refined by safeguarded Newton steps).  A ray that needs more than 4096 iterations
 * (more grid planes than that inside the gel) reads the gel surface and sets
 * TACSL_DEV_DEPTH_CAPPED in *status (optional device word).  TACSL_ERR_STATE
 * without a camera.  Asynchronous on
 * `stream`, no allocation, capturable. */
int tacsl_depth_image(tacsl_plan plan, const tacsl_state* state, float* image, uint32_t* status,
                      hipStream_t stream);

/* Reverse mode of the force field of Section III-C (the paper does not
 * differentiate it; this is the exact derivative of the same FP32 forward
 * path: the trilinear SDF value and nodal-gradient field, the normalized
 * normal, the penalty law and the Coulomb cap, with the kinks at phi = 0, at
 * the stick/slip switch and at cell faces taken one-sided as the forward
 * branches decide).  A hand-written adjoint that recomputes the forward per
 * taxel (nothing is stored between the passes), reduces per pad in FP64 in a
 * fixed order, and maps the sums to world-frame gradients per environment.
 * Enqueued on `stream`; same asynchrony rules as tacsl_force_field.  Errors:
 * TACSL_ERR_NULL_ARG (plan, state, grads or a required pointer NULL),
 * TACSL_ERR_HIP (a launch failed). */
int tacsl_force_field_backward(tacsl_plan plan, const tacsl_state* state, const tacsl_grads* grads,
                               hipStream_t stream);

/* Capture n_steps forward evaluations of n_plans plans into one HIP graph,
 * substep-major: for s in [0, n_steps), for p in [0, n_plans), plan p runs
 * with states[s*n_plans + p] and outs[s*n_plans + p] (host arrays of structs
 * whose device pointers are baked into the graph).  Plans must be distinct.
 * The graph holds a reference to the plans' buffers: destroy it before any of
 * its plans. */
int tacsl_graph_create(int32_t n_plans, const tacsl_plan* plans, int32_t n_steps, const tacsl_state* states,
                       const tacsl_outputs* outs, tacsl_graph* out);

/* Closed-form object poses along a constant twist (the seeded per-substep
 * pose update of a substep loop; the paper's tactile step reads the state the
 * dynamics step left, notation appendix): for every environment e,
 *   t_o(t) = t_o + v t,   R_o(t) = Exp(w t) R_o   (w the world-frame angular
 *   velocity), i.e. q(t) = (cos(|w| t/2), sin(|w| t/2) w/|w|) * q_0,
 * computed in FP64 and stored as FP32.
 *   pose0  device float [n_env][7] (qw qx qy qz tx ty tz), twist device float
 *          [n_env][6] (v, w), pose device float [n_env][7] out (may not
 *          alias pose0); t the elapsed time (finite).
 * Errors: TACSL_ERR_SHAPE (n_env < 0), TACSL_ERR_NULL_ARG, TACSL_ERR_RANGE (t
 * not finite), TACSL_ERR_HIP.  Asynchronous on `stream`, no allocation,
 * capturable. */
int tacsl_pose_step(int32_t n_env, const float* pose0, const float* twist, double t, float* pose,
                    hipStream_t stream);

/* A plan's substep pose path for tacsl_graph_create_path: before substep s
 * the graph writes the object poses at time s dt from (pose0, twist) into row
 * s of poses (device float [n_steps][n_env][7], the recorded path), and the
 * plan's forward of that substep reads them (the state's obj_pose is then
 * ignored).  poses = NULL: no path for this plan. */
typedef struct {
  const float* pose0;
  const float* twist;
  double dt;
  float* poses;
} tacsl_pose_path;

/* As tacsl_graph_create, with a pose path per plan (paths may be NULL, or
 * hold a NULL poses entry for plans without one): each captured substep runs
 * the path's pose step, then the forward (prologue, per-taxel pass, wrench
 * reduction) on those poses. */
int tacsl_graph_create_path(int32_t n_plans, const tacsl_plan* plans, int32_t n_steps, const tacsl_pose_path* paths,
                            const tacsl_state* states, const tacsl_outputs* outs, tacsl_graph* out);

/* Replay the captured steps on `stream`. */
int tacsl_graph_launch(tacsl_graph graph, hipStream_t stream);

int tacsl_graph_destroy(tacsl_graph graph);

/* Instrumentation: record a HIP event pair around the main kernel (forward
 * k_force_fwd or adjoint k_force_bwd) of each of the next `capacity` calls on
 * this plan, on the stream of the call.  capacity = 0 stops recording and
 * releases the events.  Recording is skipped inside graph capture.  Creates
 * events (allocates): call outside capture and timed regions. */
int tacsl_plan_timer_start(tacsl_plan plan, int32_t capacity);

/* Wait for the recorded events and copy the kernel durations in milliseconds
 * of the calls recorded since tacsl_plan_timer_start (host float [max]);
 * *n receives the number recorded (<= max). */
int tacsl_plan_timer_read(tacsl_plan plan, int32_t max, int32_t* n, float* ms);

/* Release the plan's device memory (synchronizes its device).  NULL is a no-op. */
int tacsl_plan_destroy(tacsl_plan plan);

/* Implicit soft-contact impulse, batched over contacts (Section III-A,
 * "Constraint Solution": the Kelvin-Voigt law imposed at the end of the step,
 * solved in closed form with the semi-implicit Euler update).  For contact k
 * with contact distance eps (negative when interpenetrating), separation
 * velocity eps_dot, inverse effective inertia inv_mass = 1/m (0 for an
 * immovable body) and the stiffness and damping (kappa, c) of its
 * environment:
 *   alpha     = dt (dt kappa + c)
 *   lambda[k] = max(0, (-dt kappa eps - alpha eps_dot) / (1 + alpha inv_mass))
 *   dv[k]     = lambda[k] inv_mass       (the change of eps_dot over the step)
 * Arguments (FP32 unless noted; all arrays device memory, caller-owned):
 *   n         contacts (>= 0)
 *   eps, eps_dot, inv_mass  [n]
 *   env       int32 [n] environment of each contact, or NULL (all use row 0)
 *   n_env     rows of kc (>= 1)
 *   kc        [n_env][2] = (kappa, c), 8-byte aligned
 *   dt        step length, finite and > 0
 *   lambda    [n] out: impulse (N s); dv [n] out or NULL
 *   status    optional device word: TACSL_DEV_BAD_CONTACT is OR-ed in when a
 *             contact is invalid (env outside [0, n_env), a non-finite input or
 *             result, or 1 + alpha inv_mass <= 0); such a contact gets
 *             lambda = dv = 0
 * Errors: TACSL_ERR_SHAPE (n < 0 or n_env < 1), TACSL_ERR_RANGE (dt, kc
 * alignment), TACSL_ERR_NULL_ARG (a required array NULL while n > 0),
 * TACSL_ERR_HIP (launch failed).  Asynchronous on `stream`; no allocation,
 * no host synchronization, capturable in a HIP graph.  16-byte aligned
 * arrays take the four-contacts-per-lane path. */
int tacsl_contact_impulse(int64_t n, const float* eps, const float* eps_dot, const float* inv_mass,
                          const int32_t* env, int32_t n_env, const float* kc, float dt, float* lambda, float* dv,
                          uint32_t* status, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TACSL_H_ */
