/*
 * scn.h -- C ABI of libscn.so: batched candidate-pose sampling, exact
 * collision checking and first-valid placement for procedural scene
 * generation on one MI355X (gfx950).
 *
 * The method is the batched rejection-sampling placement of Sceniris
 * (arXiv 2512.16896): for every object of every scene, sample candidate poses
 * on the object's support surface (Sec. III "Position sampling"; Sec. IV-C),
 * check them for collision against the static scene and the objects already
 * placed (Sec. IV-D), keep one collision-free pose, retry the scenes that found
 * none (Sec. IV-D), and mark a scene invalid once an object has used up its
 * retries (Sec. V-A: 10 retries).  Objects are sphere sets; static furniture is
 * oriented boxes and, optionally, voxel signed-distance grids.
 *
 * Conventions for every call
 *   - C linkage, returns an int status: SCN_OK (0) or a negative SCN_E_* code.
 *     Nothing throws across the ABI.  scn_last_error() gives a detail string
 *     (thread-local) for the last failing call on this thread.
 *   - Pointers named in scn_batch, scn_poses and the array arguments are
 *     DEVICE pointers to caller-owned memory (e.g. torch tensors).  The library
 *     never frees or reallocates them.  Host pointers are marked "host".
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*;
 *     NULL = the null stream) unless the description says they synchronize.
 *   - Argument and shape errors are found on the host before any launch
 *     (SCN_E_INVALID_ARG).  Errors only the device can see (a scene larger than
 *     the capacity the call was planned for, non-finite input) are recorded in
 *     a device error word and returned by the next synchronizing call
 *     (scn_read_counters) as SCN_E_CAPACITY / SCN_E_NONFINITE.
 *   - Non-finite input (NaN or an infinity; the paper is silent on it): a
 *     candidate whose own spheres or pose, or any box row, grid instance row,
 *     placed sphere or sampled grid node it is tested against, is not finite
 *     collides; its clearance is NaN.  In the place calls every candidate of
 *     the object then collides, so the object fails and its scene becomes
 *     INVALID.  Each such decision is counted (scn_counters.nonfinite).
 *   - Device scratch memory comes from a caller-owned workspace attached to
 *     the context (scn_set_workspace; size from scn_workspace_bytes).  The
 *     library allocates device memory only in scn_ctx_create (counters).
 *     A call whose workspace is too small fails with SCN_E_INVALID_ARG
 *     before any launch.
 *   - A context is used by one host thread at a time.
 *   - FP32 data; metres and radians.  All arrays are row-major.
 */
#ifndef SCN_H
#define SCN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SCN_OK = 0,
    SCN_E_INVALID_ARG = -1, /* bad pointer, size or shape; nothing was launched */
    SCN_E_HIP = -2,         /* a HIP runtime call failed; see scn_last_error()  */
    SCN_E_CAPACITY = -3,    /* a scene exceeded the planned on-chip capacity    */
    SCN_E_NO_DEVICE = -4,   /* no usable gfx950 device                          */
    SCN_E_UNSUPPORTED = -5, /* a size or batch kind the call does not support   */
    SCN_E_NONFINITE = -6    /* non-finite input was met (and treated as a collision) */
};

/* Scene status values (scn_batch.status). */
enum { SCN_SCENE_ACTIVE = 0, SCN_SCENE_VALID = 1, SCN_SCENE_INVALID = 2 };

typedef struct scn_ctx scn_ctx;
typedef void *scn_stream; /* hipStream_t */

/* Record of a placed object: pose in its support frame and which candidate
 * won.  attempt = idx = -1 when the object was not placed. 24 bytes.        */
typedef struct {
    float x, y, z, yaw;
    int32_t attempt, idx;
} scn_pose_rec;

/*
 * A batch of scenes (Sec. IV-B: one pose per object per scene instance).
 *
 * Read-only inputs (device):
 *   obj_off   [n_scenes+1]   objects of scene s are obj_off[s]..obj_off[s+1]-1,
 *                            in placement order (Sec. IV-A)
 *   sph_off   [n_objects+1]  template spheres of object o
 *   tmpl      [n_spheres][4] sphere (x,y,z,r) in the object frame
 *   obj_sup   [n_objects]    support surface of object o (index into sup)
 *   obj_ncand [n_objects]    candidates per attempt for object o; NULL = use
 *                            scn_gen_args.default_ncand
 *   sup       [n_supports][16]  R[9] (support->world, row-major), t[3],
 *                            half-x, half-y, inset, lift.  Candidates are drawn
 *                            uniformly on the rectangle [-(hx-inset), hx-inset] x
 *                            [-(hy-inset), hy-inset] of the support plane (the
 *                            canonical polygon moved by the support's world pose,
 *                            Sec. IV-C; inset = the ratio_on_support erosion of
 *                            Sec. IV-F expressed in metres), yaw ~ U[0, 2pi),
 *                            z = lift + the height that rests the lowest sphere
 *                            on the plane (Sec. III "Position sampling").
 *   box_off   [n_scenes+1]   static boxes of scene s
 *   box       [n_boxes][16]  R[9] (box->world), centre[3], half extents[3], pad
 *   grid_off  [n_scenes+1]   voxel-grid instances of scene s (NULL: no grids)
 *   grid      [n_grids][24]  world->grid rotation W[9], translation tw[3],
 *                            origin[3], spacing h, nodes nx,ny,nz (as floats), pad[2]
 *   grid_src  [n_grids]      asset index of the instance
 *   grid_val_off [n_assets+1] (int64) offsets of each asset's node values in grid_val
 *   grid_val  node values, x fastest (value at origin + h*(i,j,k))
 * Mutable state (device):
 *   placed    [n_spheres][4] world spheres of placed objects, parallel to tmpl
 *   n_placed  [n_scenes]     objects placed so far (always a prefix)
 *   status    [n_scenes]     SCN_SCENE_*
 *   rec       [n_objects]    pose records
 * Host-side planning sizes (maxima over the batch; a scene beyond them is
 * reported as SCN_E_CAPACITY and left untouched):
 *   max_objects_per_scene, max_spheres_per_object, max_spheres_per_scene,
 *   max_boxes_per_scene, max_grids_per_scene, max_cand_per_object
 * Declared geometry class (`geometry`):
 *   SCN_GEOM_GENERAL  any rotations.
 *   SCN_GEOM_YAW      every support rotation is a turn about z, exactly
 *                     [[a, -b, 0], [b, a, 0], [0, 0, 1]], and every box rotation
 *                     keeps the z axis (R[2] = R[5] = R[6] = R[7] = 0, R[8] = 1).
 *                     The place kernel then composes transforms in the plane.
 *                     A scene that breaks the declaration is not placed: it is
 *                     marked SCN_SCENE_INVALID and bit 1 of the counters' error
 *                     word is set.  Grids may have any rotation either way.
 */
#define SCN_GEOM_GENERAL 0
#define SCN_GEOM_YAW 1

/* Reachability map (Sec. IV-E): a 4-D map over (z*, theta, x*, y*), the
 * base-symmetric single-structure parametrization of the reachability map
 * the paper uses.  For an object frame at world position p with x axis d and
 * a robot base at (R_b, t_b): q = R_b^T (p - t_b), e = R_b^T d, psi = the
 * angle of (e_x, e_y); (x*, y*) = (q_x, q_y) turned by -psi about z, z* = q_z;
 * theta = the object's approach angle.  Cell i_a = floor((v_a - lo[a]) /
 * h[a]) on each axis (z*, theta, x*, y*, with y* fastest in `map`); a query
 * outside the map or on a zero cell is not reachable.                       */
typedef struct {
    const uint8_t *map;    /* device, dims[0] * dims[1] * dims[2] * dims[3] bytes */
    float lo[4], h[4];     /* host values                                         */
    int32_t dims[4];
} scn_reach_map;

typedef struct scn_batch {
    int32_t n_scenes, n_objects, n_spheres, n_supports, n_boxes, n_grids, n_grid_assets;
    int32_t max_objects_per_scene, max_spheres_per_object, max_spheres_per_scene;
    int32_t max_boxes_per_scene, max_grids_per_scene, max_cand_per_object;
    int32_t geometry;      /* SCN_GEOM_GENERAL or SCN_GEOM_YAW (see above)      */
    const int32_t *obj_off;
    const int32_t *sph_off;
    const float *tmpl;
    const int32_t *obj_sup;
    const int32_t *obj_ncand;
    const float *sup;
    const int32_t *box_off;
    const float *box;
    const int32_t *grid_off;
    const float *grid;
    const int32_t *grid_src;
    const int64_t *grid_val_off;
    const float *grid_val;
    float *placed;
    int32_t *n_placed;
    int8_t *status;
    scn_pose_rec *rec;
    /* Object-object spatial relations and support erosion (Sec. IV-F),
     * optional (NULL: none), read by the place calls:
     *   obj_rel   [n_objects] relation row of object o, -1 none
     *   rel       [n_rel][16] kind (1 = one anchor, partial annulus; 2 =
     *             'middle' of several anchors), anchor count, anchors[8]
     *             (positions of earlier objects of the same scene on the same
     *             support), direction v[2] in the support frame ((0,0): any),
     *             min_r, max_r (may be +inf), direction angle threshold theta,
     *             flags (bit 0: face_to, the object's x axis points at the
     *             first anchor).  One anchor: the candidate's (x, y) is drawn
     *             area-uniformly in the sector min_r <= |p - a| <= R, angle of
     *             p - a within theta of v (R = max_r clipped to the farthest
     *             corner of the support); 'middle': uniformly in the anchors'
     *             bounding box.  A point outside the region (the support
     *             rectangle, and for 'middle' the anchors' convex hull) is not
     *             a valid candidate.  Anchors that are not earlier objects on
     *             the same support, or fewer than 3 'middle' anchors, leave no
     *             valid candidate.  Counter and words as for uniform
     *             candidates (u0, u1: position; u2: yaw unless face_to).
     *   obj_ratio [n_objects] ratio_on_support: the support rectangle is
     *             eroded by ratio * half the shorter x / y extent of the
     *             object's sphere set (also in scn_sample_poses).
     * The learned-proposal calls refuse batches that have them.             */
    const int32_t *obj_rel;
    const float *rel;
    const float *obj_ratio;
    /* Reachability (Sec. IV-E), optional (robot NULL: none), read by the
     * place calls: a candidate of an object with obj_reach[o] >= 0 (its
     * approach angle) that the robot of its scene (robot [n_scenes][12]:
     * base pose R[9], t[3]) cannot reach, by `reach`, is not valid.         */
    const float *robot;
    const float *obj_reach;
    scn_reach_map reach;
    /* Stable poses (Sec. III "Main algorithm": an orientation from an
     * object's stable poses), optional (obj_pose_off NULL: none), read by the
     * place calls and scn_sample_poses:
     *   obj_pose_off [n_objects+1] rows of object o in `stable` (at most
     *                SCN_MAX_STABLE per object; an object without rows turns
     *                about z only)
     *   stable    [n_rows][12] R[9] (row-major, object frame -> resting
     *             frame), cumulative weight (increasing; the object's last row
     *             1), 2 unused.
     * A candidate of an object with rows takes row r0 + m, the first whose
     * cumulative weight reaches u3 (the candidate's fourth Philox word as a
     * unit value); its spheres are R_m c before the turn about z, and z rests
     * the turned set's lowest point on the support: z = dz + max_k (r_k -
     * (R_m c_k)_z).  ratio_on_support erodes by the unturned set's extents.
     *   rec_stable [n_objects] (output, nullable) the row each placed object
     *             took (-1: none).
     * The learned-proposal calls refuse batches that have them, and grid
     * batches do not take them (SCN_E_UNSUPPORTED).                          */
    const int32_t *obj_pose_off;
    const float *stable;
    int32_t *rec_stable;
} scn_batch;

/* Largest number of stable-pose rows of one object. */
#define SCN_MAX_STABLE 16

/* Candidate poses in the support frame, structure of arrays (device).
 * stable (nullable): the stable-pose row of each candidate (-1: none);
 * written by scn_sample_poses for batches with stable poses.             */
typedef struct {
    float *x, *y, *z, *yaw;
    int32_t *stable;
} scn_poses;

typedef struct {
    uint64_t seed;         /* key of the counter-based generator                  */
    float margin;          /* a candidate collides iff its clearance < margin      */
    int32_t retries;       /* attempts per object = retries + 1 (paper: 10)        */
    int32_t default_ncand; /* candidates per attempt when obj_ncand is NULL        */
    int32_t max_steps;     /* scn_generate_scenes: objects per scene (<= 0: all)    */
    int32_t schedule;      /* 0: autotuned / default; >0: explicit schedule id      */
    int32_t use_graph;     /* replay the launches as a hipGraph: scn_generate_scenes
                            * keeps one executable graph per batch and plan and
                            * refreshes its arguments each call; the learned
                            * generation captures its step launch once per call */
    int32_t fallback_chunk;/* scn_generate_scenes_learned: uniform fallback entries
                            * a pending object tries per tick (<= 0: all that
                            * remain, in one launch)                                */
    int32_t wide_schedule; /* scn_generate_scenes_learned: schedule of its
                            * latency-bound launches (0: 4 waves, placed spheres
                            * from global memory)                                   */
    int32_t reserved[2];   /* zero                                                  */
} scn_gen_args;

/* Work counters accumulated on the device since the last scn_reset_counters. */
typedef struct {
    int64_t candidates;    /* candidate poses brought to a decision               */
    int64_t sphere_pairs;  /* sphere-sphere tests evaluated                        */
    int64_t box_pairs;     /* sphere-box tests evaluated                           */
    int64_t grid_samples;  /* sphere-grid trilinear samples evaluated             */
    int64_t attempts;      /* (scene, object, attempt) triples started            */
    int64_t placed;        /* objects placed                                       */
    int64_t error_word;    /* device-detected errors (bit 0: capacity, bit 1:
                            * a scene breaks the declared SCN_GEOM_YAW geometry) */
    int64_t transforms;    /* candidate spheres moved to the world frame          */
    int64_t box_culls;     /* bounding-sphere vs box pretests                      */
    int64_t object_culls;  /* bounding-sphere vs placed-object pretests            */
    int64_t valid_scenes;  /* scenes that became VALID                             */
    int64_t invalid_scenes;/* scenes that became INVALID                           */
    int64_t sphere_culls;  /* bounding-sphere vs placed-sphere pretests            */
    int64_t nonfinite;     /* decisions forced by non-finite input: objects failed
                            * by the place kernel, candidates by the dense check */
    int64_t check_refined; /* dense-check candidates with a sphere pair so close
                            * that their pairs were evaluated again in the direct
                            * form |p - q| (see scn_check_batch)                 */
    int64_t reserved[1];
} scn_counters;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device` (must be gfx950).  Allocates a few
 * KB of device memory for counters.  *out owned by the caller; free with
 * scn_ctx_destroy.                                                          */
int scn_ctx_create(scn_ctx **out, int device);
int scn_ctx_destroy(scn_ctx *ctx);
const char *scn_status_string(int status);
const char *scn_last_error(void);

/* ---- workspace --------------------------------------------------------- */

/* What a workspace is sized for (scn_workspace_bytes `kind`):
 *   SCN_WS_GENERATE          scn_generate_scenes / scn_place_step / scn_autotune:
 *                            the longest-first scene order of batch b (0 bytes
 *                            for schedules without SCN_SCHED_LONGEST_FIRST;
 *                            the value returned covers them all)
 *   SCN_WS_MLP_FORWARD       scn_mlp_forward of `rows` feature rows through net
 *   SCN_WS_MLP_BACKWARD      scn_mlp_backward of `rows` rows
 *   SCN_WS_MLP_TRAIN         scn_mlp_train_step of `rows` rows (backward plus the
 *                            gradient buffers)
 *   SCN_WS_GENERATE_LEARNED  scn_generate_scenes_learned of batch b with net and
 *                            top_k proposals                                  */
enum {
    SCN_WS_GENERATE = 0,
    SCN_WS_MLP_FORWARD = 1,
    SCN_WS_MLP_BACKWARD = 2,
    SCN_WS_MLP_TRAIN = 3,
    SCN_WS_GENERATE_LEARNED = 4
};
typedef struct scn_mlp scn_mlp;

/* *bytes (host) = device workspace bytes the call of `kind` needs; b, net,
 * rows and top_k are read as the kind needs them (others may be NULL / 0).  */
int scn_workspace_bytes(int kind, const struct scn_batch *b, const scn_mlp *net, int32_t rows,
                        int32_t top_k, size_t *bytes);

/* Attach a caller-owned device buffer of `bytes` bytes (256-byte aligned) as
 * the context's workspace; NULL detaches.  The buffer must stay allocated
 * while calls that use it are in flight; calls on one context share it, so
 * they must not overlap.                                                   */
int scn_set_workspace(scn_ctx *ctx, void *ptr, size_t bytes);

/* Zero the device counters (asynchronous, graph-safe fill kernel).          */
int scn_reset_counters(scn_ctx *ctx, scn_stream stream);
/* Synchronize `stream` and copy the counters to *out (host).  Returns
 * SCN_E_CAPACITY if bit 0 of the device error word is set, SCN_E_INVALID_ARG
 * if bit 1 is (a scene broke the declared SCN_GEOM_YAW geometry), bit 3 (a
 * joint or link index out of range in scn_forward_kinematics) or bit 4 (the
 * learned generation found a support shared by two scenes),
 * SCN_E_NONFINITE if bit 2 is (non-finite input); *out is filled either way. */
int scn_read_counters(scn_ctx *ctx, scn_counters *out, scn_stream stream);

/* ---- the hot path ------------------------------------------------------ */

/* Sample the candidate poses of one attempt (Sec. III "Position sampling",
 * Sec. IV-C).  obj_idx[s] (device, int32) is the object of scene s to sample
 * for (-1: none); cand_off[n_scenes+1] (device) gives where scene s's
 * candidates go in `out`; total = cand_off[n_scenes] (host).  Candidate i of
 * attempt `attempt` for the object at position j = obj_idx[s] - obj_off[s] of
 * scene s uses Philox4x32-10(key = seed, counter = (i, attempt, j, s)). */
int scn_sample_poses(scn_ctx *ctx, const scn_batch *b, const int32_t *obj_idx,
                     const int32_t *cand_off, int32_t total, int32_t max_cand_per_scene,
                     uint64_t seed, int32_t attempt, scn_poses out, scn_stream stream);

/* Dense exact check (Sec. IV-D) of given candidate poses of object obj_idx[s]
 * against scene s's boxes, grids and its first n_placed[s] objects (their
 * world spheres in b->placed).  clearance[t] (nullable) = min over the
 * candidate's spheres and all obstacles of (signed distance - radii);
 * +inf without obstacles.  collide[t] (nullable, uint8) = clearance < margin.
 * Every pair is evaluated (no culling, no early exit).  Candidates turn
 * about z only: poses.stable must be NULL (SCN_E_UNSUPPORTED otherwise).    */
int scn_check_batch(scn_ctx *ctx, const scn_batch *b, const int32_t *obj_idx,
                    const int32_t *cand_off, int32_t total, int32_t max_cand_per_scene,
                    scn_poses poses, float margin, float *clearance, uint8_t *collide,
                    scn_stream stream);

/* Set every scene to ACTIVE with nothing placed (graph-safe fill kernel).   */
int scn_reset_scenes(scn_ctx *ctx, scn_batch *b, scn_stream stream);

/* One placement step (Sec. IV-A): every ACTIVE scene places its next object
 * n_placed[s]: attempts 0..retries, each with fresh candidates; the winner is
 * the lowest-index collision-free candidate of the first attempt that has
 * one; its world spheres are appended to b->placed and its record to b->rec.
 * A scene whose object finds none becomes INVALID; a scene whose last object
 * is placed becomes VALID.  chosen[s] (device, nullable) = winning index, -1
 * if the object failed, -2 if the scene was not active.                     */
int scn_place_step(scn_ctx *ctx, scn_batch *b, const scn_gen_args *args, int32_t *chosen,
                   scn_stream stream);

/* The whole batch (Sec. IV-A, Fig. 2 "generates a batch of scenes"): resets
 * the scenes and places every object of every scene in one persistent fused
 * launch (sampling, checking, selection, commit and retries on the device,
 * no host round trip).  Equivalent to scn_reset_scenes followed by
 * scn_place_step until no scene is ACTIVE.                                 */
int scn_generate_scenes(scn_ctx *ctx, scn_batch *b, const scn_gen_args *args,
                        scn_stream stream);

/* ---- allocation-free generation ---------------------------------------- */

/* For callers that cannot allocate device memory or attach a workspace (code
 * under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): scn_generate_scenes with its scratch memory (the longest-first
 * scene order of schedules with SCN_SCHED_LONGEST_FIRST) taken from a fixed
 * array inside the library instead of the context's workspace.
 *   - Limit: SCN_NOALLOC_MAX_SCENES scenes (the array is 4 MiB + 1.25 KiB per
 *     device, held until the process ends; scn_ctx_create looks up its address
 *     on the context's device).  A larger batch fails with SCN_E_INVALID_ARG
 *     before any launch.
 *   - Calls no hipMalloc / hipFree and no allocating runtime routine; launches
 *     eagerly on `stream` (args->use_graph must be 0, else SCN_E_UNSUPPORTED).
 *   - Every call on one device shares that device's array and leaves its
 *     contents behind (the order is rebuilt and its histogram cleared by a fill
 *     kernel in each call): calls that overlap on one device, from any stream,
 *     context or thread, race; the caller serializes them.
 *   - Results are identical to scn_generate_scenes with the same arguments. */
#define SCN_NOALLOC_MAX_SCENES (1 << 20)
int scn_generate_scenes_noalloc(scn_ctx *ctx, scn_batch *b, const scn_gen_args *args,
                                scn_stream stream);

/* ---- reachability queries --------------------------------------------- */

/* Batched reachability (Sec. IV-E: the map on the GPU, queries batched):
 * pose [n][12] world pose (R[9], t[3]) of each object frame, robot [n][12]
 * the robot base pose of each query, theta [n] approach angles (device);
 * out [n] (device, uint8) = 1 if reachable by `map`.  Asynchronous.        */
int scn_reach_query(scn_ctx *ctx, const scn_reach_map *map, int32_t n, const float *robot,
                    const float *pose, const float *theta, uint8_t *out, scn_stream stream);

/* ---- articulated parts: batched forward kinematics --------------------- */

/* Articulated furniture of a batch (Sec. IV-B: one transform per scene
 * instance on every scene-graph edge, moved by a batched forward-kinematics
 * function; Sec. V-A: drawer joint states randomized per scene).  Device
 * arrays, caller-owned:
 *   joint_off [n_scenes+1]   joints of scene s, in topological order
 *   joint     [n_joints][24] type (0 prismatic, 1 revolute), parent (index of
 *                            an earlier joint of the same scene, -1 = the
 *                            scene's base), lower, upper, axis[3] (in the joint
 *                            frame; unit length for revolute joints, the step
 *                            per unit of q for prismatic ones), pad,
 *                            R_j[9], t_j[3] (joint frame in the parent link
 *                            frame), pad[4]
 *   base      [n_scenes][12] R[9], t[3]: world pose of each scene's base link */
typedef struct {
    int32_t n_scenes, n_joints;
    const int32_t *joint_off;
    const float *joint;
    const float *base;
} scn_joints;

/* Joint values and link poses of every scene, then the rows carried by links:
 *   q     [n_joints] (device) joint values: drawn when sample_q != 0 as
 *         lower + u (upper - lower), u from Philox4x32-10 (key = seed, counter
 *         = (joint index within its scene, 0x30000, 0, scene)); read otherwise
 *   link  [n_joints][12] (device, out) world pose of each joint's child link:
 *         link_i = link_parent * [R_j | t_j] * M(q_i), M = translation by q a
 *         (prismatic) or rotation by q about a (revolute, Rodrigues)
 *   box rows b with box_link[b] >= 0 (global joint index) get R and centre of
 *         link[box_link[b]] * box_local[b] (box_local [n_box][12]: R[9], t[3]);
 *         half extents are kept.  support rows likewise (R and t; sizes kept).
 *         box_link / sup_link NULL: no rows of that kind move.
 * A parent that is not an earlier joint of its scene, or a link index >=
 * n_joints, leaves that link (NaN) / row untouched and is reported as
 * SCN_E_INVALID_ARG by the next scn_read_counters.  Asynchronous.          */
int scn_forward_kinematics(scn_ctx *ctx, const scn_joints *joints, uint64_t seed, int32_t sample_q,
                           float *q, float *link, int32_t n_box, const int32_t *box_link,
                           const float *box_local, float *box, int32_t n_sup,
                           const int32_t *sup_link, const float *sup_local, float *sup,
                           scn_stream stream);

/* ---- uneven batching: autotuned schedules ------------------------------ */

/* Schedule ids for scn_gen_args.schedule (0 = the context's tuned choice for
 * this batch shape, or the default 0xF04: 4 waves, batch order, placed
 * spheres from global memory):
 *   bits 0-4  waves per workgroup: candidates of one scene in flight
 *             (1..16)
 *   bit  5    longest-first scene order: scenes with more work start
 *             first, the work estimated as objects x (spheres + 16 boxes)
 *             scaled by how crowded the support is with boxes (crowded
 *             supports are where objects exhaust their attempts)
 *   bits 8-11 LDS budget for a scene's placed spheres: 0 = sized for the
 *             largest scene (every scene LDS-resident); 1..5 = 32, 48, 64,
 *             80, 96 KB (larger scenes read their placed spheres from global
 *             memory in a second launch); 15 = every scene from global memory */
enum {
    SCN_SCHED_WAVES_MASK = 0x1F,
    SCN_SCHED_LONGEST_FIRST = 0x20,
    SCN_SCHED_LDS_SHIFT = 8,
    SCN_SCHED_LDS_MASK = 0xF00,
    SCN_SCHED_LDS_NONE = 0xF
};

/* Time the schedules of the fused place kernel on this batch (coordinate
 * descent over LDS budget, waves and scene order; per schedule the best of
 * three full generations after one warm-up run) and remember the fastest
 * for batches of the same shape bucket (largest object, largest scene,
 * objects per scene, number of scenes) in the context.  Synchronizes
 * `stream`; leaves the batch state of the last run.  *best_schedule and
 * *best_ms (host, nullable) receive the choice and its time.  This is the
 * project's autotuner for the uneven-batch launch (one persistent fused
 * launch whose best shape depends on the batch).                         */
int scn_autotune(scn_ctx *ctx, scn_batch *b, const scn_gen_args *args, int32_t *best_schedule,
                 float *best_ms, scn_stream stream);

/* Persist / restore the context's tuned choices as a small JSON file
 * (host path).                                                            */
int scn_autotune_save(scn_ctx *ctx, const char *path);
int scn_autotune_load(scn_ctx *ctx, const char *path);

/* ---- learned pose proposal: the network ------------------------------- */

/* A 4-layer perceptron over a state's features (a 64 x 64 height map of the
 * support plus a 32-d object descriptor, dims[0] = 4128 values) to 4096 pose-
 * bin logits (32 x-cells x 16 y-cells x 8 yaw cells), ReLU between layers,
 * BF16 weights and activations with FP32 accumulation.  All pointers are
 * device pointers to caller-owned buffers:
 *   w[l]  FP32 master weights [dims[l+1]][dims[l]]      b[l]  FP32 biases [dims[l+1]]
 *   wb[l] BF16 copy of w[l] (same layout)               wt[l] BF16 transpose [dims[l]][dims[l+1]]
 *   m_w, v_w, m_b, v_b  AdamW moments like w / b (only needed for training).
 * dims[0..3] must be multiples of 32 (K of the matrix-core GEMMs).          */
#define SCN_MLP_LAYERS 4
struct scn_mlp {
    int32_t dims[SCN_MLP_LAYERS + 1];
    float *w[SCN_MLP_LAYERS], *b[SCN_MLP_LAYERS];
    uint16_t *wb[SCN_MLP_LAYERS], *wt[SCN_MLP_LAYERS];
    float *m_w[SCN_MLP_LAYERS], *v_w[SCN_MLP_LAYERS], *m_b[SCN_MLP_LAYERS], *v_b[SCN_MLP_LAYERS];
    int64_t step; /* AdamW steps taken; advanced by scn_mlp_train_step (host field) */
};

typedef struct {
    float lr, beta1, beta2, eps, weight_decay;
} scn_adamw;

/* Kaiming-uniform weights from Philox4x32-10 (bound sqrt(6 / fan_in)), zero
 * biases and moments, step = 0.                                              */
int scn_mlp_init(scn_ctx *ctx, scn_mlp *net, uint64_t seed, scn_stream stream);

/* logits[M][dims[4]] (FP32) of the BF16 feature rows x[M][dims[0]].  The
 * hidden activations live in the context's workspace
 * (SCN_WS_MLP_FORWARD).                                                      */
int scn_mlp_forward(scn_ctx *ctx, const scn_mlp *net, const uint16_t *x, int32_t M,
                    float *logits, scn_stream stream);

/* Gradients of the mean binary cross-entropy over the labelled bins
 * (workspace SCN_WS_MLP_BACKWARD):
 * label_bins[M][L] (int32, -1 = no label), label_tgt[M][L] (1 accepted, 0
 * rejected); loss = mean over labels of softplus(z) - t z with z the logit of
 * the labelled bin.  gw[l] [dims[l+1]][dims[l]], gb[l] [dims[l+1]] (FP32,
 * caller-owned) receive dLoss/dW and dLoss/db; *loss (device) the loss.      */
int scn_mlp_backward(scn_ctx *ctx, const scn_mlp *net, const uint16_t *x, int32_t M,
                     const int32_t *label_bins, const float *label_tgt, int32_t L,
                     float *const *gw, float *const *gb, float *loss, scn_stream stream);

/* One AdamW step (decoupled weight decay, bias-corrected moments) on the
 * gradients of scn_mlp_backward; refreshes the BF16 copies; ++net->step.
 * Weight decay applies to the weight matrices only, not to the biases.
 * Workspace SCN_WS_MLP_TRAIN.                                               */
int scn_mlp_train_step(scn_ctx *ctx, scn_mlp *net, const uint16_t *x, int32_t M,
                       const int32_t *label_bins, const float *label_tgt, int32_t L,
                       const scn_adamw *opt, float *loss, scn_stream stream);

/* ---- learned pose proposal: state features, ranking, labels ----------- */

#define SCN_HMAP_CELLS 4096 /* 64 x 64 height map of the support                */
#define SCN_DESC 32         /* object descriptor length                          */
#define SCN_FEATURES 4128   /* network input: height map + descriptor            */
#define SCN_BINS 4096       /* pose bins: 32 x-cells x 16 y-cells x 8 yaw cells  */

/* desc[o][32] (FP32) for every object: sphere-set moments of its template
 * (count/256; mean, min, max, std radius; sum r^3; r^3-weighted centroid;
 * centre covariance; AABB half extents; rest lift; resting top height;
 * footprint radius; zeros), lengths in decimetres.                          */
int scn_descriptors(scn_ctx *ctx, const scn_batch *b, float *desc, scn_stream stream);

/* hmap[u][64][64] (FP32, metres above support u's plane), one per support
 * of the batch, for the state where each scene s has its first n_state[s]
 * objects placed (n_state NULL: b->n_placed).  Cell (ix, iy) is centred at
 * (-hx + (ix+1/2) 2hx/64, -hy + (iy+1/2) 2hy/64) in the support frame; the value
 * is the highest top above that point of the boxes of the support's scene and
 * of the placed spheres of the objects resting on u, or 0.  Each support
 * belongs to one scene (the objects on it are that scene's); supports no
 * object rests on are left untouched.                                      */
int scn_heightmaps(scn_ctx *ctx, const scn_batch *b, const int32_t *n_state, float *hmap,
                   scn_stream stream);

/* x[r][SCN_FEATURES] (BF16) = [10 * hmap[b->obj_sup[o]], desc[o]] for object
 * o = obj_idx[r] (the map of its own support); zeros for obj_idx[r] < 0.    */
int scn_features(scn_ctx *ctx, const scn_batch *b, int32_t n, const float *hmap,
                 const float *desc, const int32_t *obj_idx, uint16_t *x, scn_stream stream);

/* bins[m][k]: the k best pose bins of logits[m][SCN_BINS] in rank order
 * (logit descending, ties to the lower bin); rows with active[m] < 0 are left
 * untouched (active nullable).  1 <= k <= SCN_BINS.                          */
int scn_proposal_topk(scn_ctx *ctx, const float *logits, int32_t M, int32_t k,
                      const int32_t *active, int32_t *bins, scn_stream stream);

/* Accept / reject labels for the learned proposal (from the exact checker):
 * for each scene s in the state with its first n_state[s] objects placed
 * (n_state NULL: b->n_placed), L uniform candidates of the next object
 * (counter (i, 0x20000 | round, n_state[s], s)); bins[s][i] = the candidate's
 * pose bin, accept[s][i] = 1 if its clearance (boxes, voxel grids and the
 * state's placed spheres) >= margin else 0.  Scenes with no next object get
 * bins -1.                                                                   */
int scn_harvest_labels(scn_ctx *ctx, const scn_batch *b, const int32_t *n_state, int32_t L,
                       uint64_t seed, int32_t round, float margin, int32_t *bins,
                       float *accept, scn_stream stream);

/* The whole batch with the learned proposal (Sec. IV-A loop; proposal, then
 * uniform fallback): for each object position j, every active scene ranks the
 * pose bins of its state with the network, its top_k bins (one pose drawn in
 * each) are checked in rank order before the uniform attempts, and the exact
 * check alone decides validity.  Records of proposal picks have attempt = -2
 * and idx = rank.  Runs as ticks on `stream` and a second stream of the
 * context (default priority): each tick splits the scenes with work into
 * those starting an object and those with a pending one; the first run the
 * network over their compacted rows and try their proposals, while the
 * others try args->fallback_chunk more uniform entries (<= 0: all) on the
 * second stream.  Scenes progress independently and every scene's list is
 * tried in order, which gives the placements of one pass over the whole
 * list.  Launch sizes are fixed; kernels read the list sizes on the device.
 * The host reads the two list sizes (8 bytes) after a first batch of ticks
 * as long as a scene's object count, then every 8 ticks, so the call
 * returns with the stream drained.  args->schedule (0: one wave per scene)
 * shapes the first ticks' new-object launches, args->wide_schedule (0: 4
 * waves) the rest; neither is the context's tuned plain schedule, and of
 * either only the waves count (placed spheres stay in global memory and the
 * scenes run in list order, whatever the LDS and order bits say).  The
 * workspace also keeps each scene's depth map, each placed object's bounding
 * sphere and each object's constants across the ticks.  A state's height map
 * is that of its next object's support (multi-support and voxel-grid batches
 * are taken; a support shared by two scenes sets an error that the next
 * scn_read_counters reports as SCN_E_INVALID_ARG).                          */
int scn_generate_scenes_learned(scn_ctx *ctx, scn_batch *b, const scn_gen_args *args,
                                const scn_mlp *net, int32_t top_k, scn_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* SCN_H */
