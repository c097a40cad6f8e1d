/*
 * oracle.c -- plain FP64 CPU oracle for batched rejection-sampling placement.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) links, imports or calls this file.  Only tests/,
 * __graft_entry__.smoke() and the cpu_baseline leg of bench.py use it.
 * It shares no code, header, table or helper with the GPU path.
 *
 * What it computes, and where the paper defines it (Sceniris, arXiv 2512.16896):
 *   - Rejection sampling per object: sample a pose, check it for collision,
 *     retry on collision (Sec. III "Main algorithm"; Sec. IV-A overview).
 *   - Candidate positions are 2-D points sampled on the support polygon plus a
 *     z offset (Sec. III "Position sampling"), sampled in the canonical support
 *     frame and moved by the support's world pose (Sec. IV-C, last paragraph).
 *   - Orientation: random rotation about z, or a stable pose of the object
 *     drawn from its table (weights) followed by the random rotation about z
 *     (Sec. III "Main algorithm": pre-defined rules or stable poses).
 *   - Batched form: N independent scenes, one pose per (scene, object)
 *     (Sec. IV-B); retries only for the scenes that failed (Sec. IV-D).
 *   - 10 retries per object; a scene whose object exhausts them is invalid
 *     (Sec. V-A).
 * Readings where the paper is silent (collision geometry = sphere sets vs.
 * oriented boxes / placed spheres; strict margin test; first-valid selection;
 * Philox counter layout) are the project's and are listed in the design notes.
 *
 * Everything is FP64 except the random bits, which are exact integers.
 * There is no culling and no blocking: every candidate's clearance is the
 * plain minimum over all sphere/obstacle pairs.  (orc_generate's optional
 * early_exit mode, used by tests that replay large scenes, stops a candidate
 * at its first term below margin - band: such a candidate collides and is not
 * banded whatever its exact minimum, so every output is the same.)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, J. Salmon et al., "Parallel random numbers: as easy as     */
/* 1, 2, 3", SC'11.  Ten rounds of the 4x32 Philox S-box with the published  */
/* multipliers and Weyl key increments.                                      */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 32 random bits -> a uniform in (0,1): the top 23 bits plus one half, times
 * 2^-23.  Exactly representable in binary32 and binary64.                   */
double orc_u01(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* ------------------------------------------------------------------------ */
/* Scene batch (all arrays row-major, FP64 copies of the FP32 inputs).       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n_scenes;
    const int32_t *obj_off;   /* [n_scenes+1] objects of a scene, in placement order */
    const int32_t *sph_off;   /* [n_obj+1] template spheres of an object            */
    const double  *tmpl;      /* [n_sph][4] sphere (x,y,z,r) in the object frame      */
    const int32_t *obj_sup;   /* [n_obj] support surface of the object                */
    const int32_t *obj_ncand; /* [n_obj] candidates per attempt (NULL: default)       */
    const double  *sup;       /* [n_sup][16] R[9] t[3] half-x half-y inset dz         */
    const int32_t *box_off;   /* [n_scenes+1] static boxes of a scene                 */
    const double  *box;       /* [n_box][16] R[9] c[3] h[3] pad                        */
    const int32_t *grid_off;  /* [n_scenes+1] voxel grid instances of a scene (NULL)  */
    const double  *grid;      /* [n_grid][24] inst. pose W[9] tw[3], origin[3], h, dims[3], pad */
    const int32_t *grid_src;  /* [n_grid] which voxel asset the instance samples       */
    const float  **grid_val;  /* [n_asset] node values, x fastest                     */
    const int32_t *scene_id;  /* [n_scenes] scene number used in the random counter
                                 (NULL: the position in the batch)                   */
    const int32_t *obj_rel;   /* [n_obj] spatial relation row of the object, -1 none (NULL: none) */
    const double  *rel;       /* [n_rel][16] relation rows (see sample_relation)      */
    const double  *obj_ratio; /* [n_obj] ratio_on_support (NULL: 0)                   */
    const double  *robot;     /* [n_scenes][12] robot base pose R[9] t[3] (NULL: no reachability) */
    const double  *obj_reach; /* [n_obj] approach angle of the reachability check, < 0 none */
    const uint8_t *reach_map; /* 4-D map, 1 = reachable (see reachable())             */
    const double  *reach_geom;/* lo[4], h[4], dims[4] of the map axes (z*, theta, x*, y*) */
    const int32_t *obj_pose_off; /* [n_obj+1] stable-pose rows of an object (NULL: none) */
    const double  *stable;    /* [n_rows][12] R[9] (object frame -> resting frame),
                                 cumulative weight (last row of an object 1), 2 unused */
} orc_batch;

typedef struct {
    uint64_t seed;
    double   margin;
    int      retries;       /* attempts per object = retries + 1 */
    int      default_ncand;
    double   band;          /* |clearance - margin| < band marks a candidate as banded */
    int      max_steps;     /* place at most this many objects per scene (<=0: all) */
    int      early_exit;    /* nonzero: a candidate's clearance stops at its first term
                               below margin - band (the candidate collides and is not
                               banded either way; results are identical, only faster) */
    double   band_region;   /* a relation sample within this of its region's boundary
                               marks the decision as banded (FP32 may decide it either way) */
} orc_gen_args;

/* Pose of a candidate in its support frame: position (x,y,z), yaw about z,
 * and the stable-pose row k applied before the yaw (-1: none).              */
typedef struct { double x, y, z, yaw; int k; } orc_pose;

/* Template sphere c (object frame) turned into the resting frame of stable
 * pose row k (unchanged for k < 0): R_k c.                                   */
static void rest_point(const orc_batch *b, int k, const double *c, double out[3])
{
    if (k < 0) { out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; return; }
    const double *R = b->stable + 12 * k;
    for (int r = 0; r < 3; ++r) out[r] = R[3 * r] * c[0] + R[3 * r + 1] * c[1] + R[3 * r + 2] * c[2];
}

/* Lift that rests the lowest point of the sphere set on the support plane:
 * max over spheres of (r - z), z in the resting frame of row k.             */
static double zrest_of(const orc_batch *b, int o, int k)
{
    double lift = -INFINITY;
    for (int m = b->sph_off[o]; m < b->sph_off[o + 1]; ++m) {
        double q[3];
        rest_point(b, k, b->tmpl + 4 * m, q);
        double v = b->tmpl[4 * m + 3] - q[2];
        if (v > lift) lift = v;
    }
    return lift;
}

/* Stable pose of a candidate from its fourth Philox word: the first row of
 * the object's table whose cumulative weight reaches u = u01(w3), i.e. row
 * r0 + m with probability cum_m - cum_{m-1}; -1 when the object has none. */
static int stable_row(const orc_batch *b, int o, uint32_t w3)
{
    if (!b->obj_pose_off) return -1;
    int r0 = b->obj_pose_off[o], r1 = b->obj_pose_off[o + 1];
    if (r1 <= r0) return -1;
    double u = orc_u01(w3);
    for (int r = r0; r < r1 - 1; ++r)
        if (u <= b->stable[12 * r + 9]) return r;
    return r1 - 1;
}

/* ratio_on_support (Sec. IV-F): the support is eroded by ratio x half the
 * shorter edge of the object's projection, taken as the x / y extent of its
 * sphere set in the object frame (centres +- radii).                         */
static double erosion_of(const orc_batch *b, int o)
{
    if (!b->obj_ratio || !(b->obj_ratio[o] > 0.0)) return 0.0;
    double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
    for (int k = b->sph_off[o]; k < b->sph_off[o + 1]; ++k)
        for (int d = 0; d < 2; ++d) {
            double c = b->tmpl[4 * k + d], r = b->tmpl[4 * k + 3];
            if (c - r < lo[d]) lo[d] = c - r;
            if (c + r > hi[d]) hi[d] = c + r;
        }
    double ex = hi[0] - lo[0], ey = hi[1] - lo[1];
    return b->obj_ratio[o] * 0.5 * (ex < ey ? ex : ey);
}

/* Candidate i of attempt a for the object at position `step` of scene s:
 * the four Philox words of counter (i, a, step, scene).                      */
static void candidate_words(const orc_batch *b, uint64_t seed, int s, int step, int attempt, int i,
                            uint32_t w[4])
{
    uint32_t sid = b->scene_id ? (uint32_t)b->scene_id[s] : (uint32_t)s;
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)attempt, (uint32_t)step, sid};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, w);
}

static orc_pose sample_pose(const orc_batch *b, uint64_t seed, int s, int step, int o,
                            int attempt, int i)
{
    const double *u = b->sup + 16 * b->obj_sup[o];
    uint32_t w[4];
    candidate_words(b, seed, s, step, attempt, i, w);
    double e = erosion_of(b, o);
    double ax = u[12] - u[14] - e, ay = u[13] - u[14] - e;
    orc_pose p;
    p.x = ax * (2.0 * orc_u01(w[0]) - 1.0);
    p.y = ay * (2.0 * orc_u01(w[1]) - 1.0);
    p.yaw = 2.0 * M_PI * orc_u01(w[2]);
    p.k = stable_row(b, o, w[3]);
    p.z = u[15] + zrest_of(b, o, p.k);
    return p;
}

/* ------------------------------------------------------------------------ */
/* Object-object spatial relations (Sec. IV-F).  A relation row (16 values): */
/*   [0] kind: 1 = one anchor (partial annulus), 2 = several anchors         */
/*       ('middle'); [1] number of anchors; [2..9] anchors (positions of     */
/*       earlier objects of the scene); [10..11] direction v in the support  */
/*       frame ((0,0): every direction); [12] min_r, [13] max_r (may be      */
/*       +inf); [14] direction_angle_threshold theta; [15] flags, bit 0 =    */
/*       face_to (the object's x axis points at the first anchor).           */
/* Single anchor: the region S' = S_r cap S, S_r the points p with           */
/*   min_r <= |p - a| <= max_r and the direction of p - a within theta of v, */
/* S the (eroded) support rectangle.  Sampled uniformly by area in the       */
/* annulus sector: r = sqrt(min_r^2 + u0 (R^2 - min_r^2)), angle = angle(v) +  */
/* theta (2 u1 - 1), with R = min(max_r, the farthest corner of S from a);   */
/* a point outside S is rejected (the candidate is not valid).               */
/* Several anchors: the region is the anchors' convex hull cap S, sampled    */
/* uniformly in the anchors' bounding box (u0, u1) and rejected outside the  */
/* hull or outside S.  Fewer than 3 anchors enclose no area: no candidate is */
/* valid.  Yaw: face_to, else 2 pi u2.                                        */
/* ------------------------------------------------------------------------ */
typedef struct { double x, y, yaw; int inside; int banded; } orc_rel_sample;

static double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

static orc_rel_sample sample_relation(const double *rel, const double anc[][2], double ax,
                                      double ay, const uint32_t w[4], double band)
{
    orc_rel_sample r = {0.0, 0.0, 0.0, 0, 0};
    double u0 = orc_u01(w[0]), u1 = orc_u01(w[1]), u2 = orc_u01(w[2]);
    int n = (int)rel[1];
    if ((int)rel[0] == 1) {
        double a0 = anc[0][0], a1 = anc[0][1];
        double far = 0.0;
        for (int c = 0; c < 4; ++c) {
            double cx = (c & 1 ? ax : -ax) - a0, cy = (c & 2 ? ay : -ay) - a1;
            double d = sqrt(cx * cx + cy * cy);
            if (d > far) far = d;
        }
        double rmin = rel[12], rmax = rel[13] < far ? rel[13] : far;
        if (!(rmin < rmax)) return r;
        int dir = rel[10] != 0.0 || rel[11] != 0.0;
        double th = dir ? (rel[14] < M_PI ? rel[14] : M_PI) : M_PI;
        double phi0 = dir ? atan2(rel[11], rel[10]) : 0.0;
        double rr = sqrt(rmin * rmin + u0 * (rmax * rmax - rmin * rmin));
        double phi = phi0 + th * (2.0 * u1 - 1.0);
        r.x = a0 + rr * cos(phi);
        r.y = a1 + rr * sin(phi);
    } else {
        if (n < 3) return r;
        double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
        for (int k = 0; k < n; ++k)
            for (int d = 0; d < 2; ++d) {
                if (anc[k][d] < lo[d]) lo[d] = anc[k][d];
                if (anc[k][d] > hi[d]) hi[d] = anc[k][d];
            }
        r.x = lo[0] + u0 * (hi[0] - lo[0]);
        r.y = lo[1] + u1 * (hi[1] - lo[1]);
        /* hull edges: (i, k) with every other anchor strictly to its left */
        int inside = 1, nedge = 0;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                if (i == k) continue;
                double ex = anc[k][0] - anc[i][0], ey = anc[k][1] - anc[i][1];
                int edge = 1;
                for (int m = 0; m < n && edge; ++m)
                    if (m != i && m != k && !(cross2(ex, ey, anc[m][0] - anc[i][0], anc[m][1] - anc[i][1]) > 0.0))
                        edge = 0;
                if (!edge) continue;
                ++nedge;
                double c = cross2(ex, ey, r.x - anc[i][0], r.y - anc[i][1]);
                double len = sqrt(ex * ex + ey * ey);
                if (fabs(c) < band * len) r.banded = 1;
                if (c < 0.0) inside = 0;
            }
        if (nedge < 3) return r;
        if (!inside) { r.inside = 0; goto yaw; }
    }
    r.inside = fabs(r.x) <= ax && fabs(r.y) <= ay;
    if (fabs(fabs(r.x) - ax) < band || fabs(fabs(r.y) - ay) < band) r.banded = 1;
yaw:
    if (((int)rel[15]) & 1) r.yaw = atan2(anc[0][1] - r.y, anc[0][0] - r.x);
    else r.yaw = 2.0 * M_PI * u2;
    return r;
}

/* World position of an object-frame point c under pose p on support u:
 *   world = R_u * (Rz(yaw) * R_k * c + (x,y,z)) + t_u   (R_k = I without a
 * stable pose)                                                              */
static void world_point(const orc_batch *b, int o, const double c[4], orc_pose p, double out[4])
{
    const double *u = b->sup + 16 * b->obj_sup[o];
    double q[3];
    rest_point(b, p.k, c, q);
    double cs = cos(p.yaw), sn = sin(p.yaw);
    double l[3] = {cs * q[0] - sn * q[1] + p.x, sn * q[0] + cs * q[1] + p.y, q[2] + p.z};
    for (int r = 0; r < 3; ++r)
        out[r] = u[3 * r + 0] * l[0] + u[3 * r + 1] * l[1] + u[3 * r + 2] * l[2] + u[9 + r];
    out[3] = 0.0;
}

/* World sphere k of object o at pose p (the same transform; radius kept).  */
static void world_sphere(const orc_batch *b, int o, int k, orc_pose p, double out[4])
{
    world_point(b, o, b->tmpl + 4 * k, p, out);
    out[3] = b->tmpl[4 * k + 3];
}

/* Exact signed distance from point p to an oriented box (R: box->world
 * rotation, c: centre, h: half extents).  Standard box SDF:
 *   q = |R^T (p - c)| - h,  sdf = || max(q,0) || + min(max(qx,qy,qz), 0).    */
double orc_box_sdf(const double R[9], const double c[3], const double h[3], const double p[3])
{
    double d[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
    double q[3];
    for (int a = 0; a < 3; ++a) {
        double loc = R[0 * 3 + a] * d[0] + R[1 * 3 + a] * d[1] + R[2 * 3 + a] * d[2];
        q[a] = fabs(loc) - h[a];
    }
    double ox = q[0] > 0 ? q[0] : 0, oy = q[1] > 0 ? q[1] : 0, oz = q[2] > 0 ? q[2] : 0;
    double outside = sqrt(ox * ox + oy * oy + oz * oz);
    double m = q[0];
    if (q[1] > m) m = q[1];
    if (q[2] > m) m = q[2];
    double inside = m < 0 ? m : 0;
    return outside + inside;
}

/* Trilinear interpolation of a node-centred voxel grid (value v[i,j,k] at
 * origin + h*(i,j,k)), queried at a point already in the grid frame.  Outside
 * the node box the grid returns +inf (nothing there).  Inside it, a sample
 * that reads a non-finite node value is NaN (see clearance() below).        */
double orc_grid_sample(const float *val, const int dims[3], const double origin[3], double h,
                       const double pg[3])
{
    double f[3];
    int i0[3];
    for (int a = 0; a < 3; ++a) {
        double g = (pg[a] - origin[a]) / h;
        if (!(g >= 0.0) || g > (double)(dims[a] - 1)) return INFINITY;
        int i = (int)floor(g);
        if (i > dims[a] - 2) i = dims[a] - 2;
        i0[a] = i;
        f[a] = g - (double)i;
    }
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? f[0] : 1 - f[0]) * (dy ? f[1] : 1 - f[1]) * (dz ? f[2] : 1 - f[2]);
                size_t idx = ((size_t)(i0[2] + dz) * dims[1] + (size_t)(i0[1] + dy)) * dims[0]
                             + (size_t)(i0[0] + dx);
                if (!isfinite((double)val[idx])) return NAN;
                acc += w * (double)val[idx];
            }
    return acc;
}

static int finite_n(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Clearance of one placed sphere set against the obstacles of scene s:
 * min over its spheres of (signed distance to every box, grid and already
 * placed sphere) minus the sphere radius.  +inf with no obstacles.
 * stop_below (-inf: never): return the first term found below it instead of
 * the minimum.  The minimum is then below stop_below too, which is all a
 * caller that only compares the minimum with stop_below needs to know.
 *
 * Non-finite input (the paper is silent; the project's reading): a candidate
 * whose world spheres, or any box row, grid instance row, placed sphere or
 * sampled grid node it is tested against, hold a NaN or an infinity has no
 * clearance: the result is NaN, which no margin test accepts, so the
 * candidate collides.                                                        */
static double clearance(const orc_batch *b, int s, const double *sph, int n_sph,
                        const double *placed, int n_placed_sph, double stop_below)
{
    double best = INFINITY;
    if (!finite_n(sph, 4 * n_sph)) return NAN;
    for (int bx = b->box_off[s]; bx < b->box_off[s + 1]; ++bx)
        if (!finite_n(b->box + 16 * bx, 15)) return NAN;
    if (b->grid_off)
        for (int g = b->grid_off[s]; g < b->grid_off[s + 1]; ++g)
            if (!finite_n(b->grid + 24 * g, 19)) return NAN;
    if (!finite_n(placed, 4 * n_placed_sph)) return NAN;
    for (int k = 0; k < n_sph; ++k) {
        const double *p = sph + 4 * k;
        for (int bx = b->box_off[s]; bx < b->box_off[s + 1]; ++bx) {
            const double *B = b->box + 16 * bx;
            double v = orc_box_sdf(B, B + 9, B + 12, p) - p[3];
            if (v < best) best = v;
            if (v < stop_below) return v;
        }
        if (b->grid_off) {
            for (int g = b->grid_off[s]; g < b->grid_off[s + 1]; ++g) {
                const double *G = b->grid + 24 * g;
                /* world -> grid frame: pg = W p + tw */
                double pg[3];
                for (int r = 0; r < 3; ++r)
                    pg[r] = G[3 * r] * p[0] + G[3 * r + 1] * p[1] + G[3 * r + 2] * p[2] + G[9 + r];
                int dims[3] = {(int)G[16], (int)G[17], (int)G[18]};
                double v = orc_grid_sample(b->grid_val[b->grid_src[g]], dims, G + 12, G[15], pg) - p[3];
                if (isnan(v)) return NAN;
                if (v < best) best = v;
                if (v < stop_below) return v;
            }
        }
        for (int j = 0; j < n_placed_sph; ++j) {
            const double *q = placed + 4 * j;
            double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
            double v = sqrt(dx * dx + dy * dy + dz * dz) - q[3] - p[3];
            if (v < best) best = v;
            if (v < stop_below) return v;
        }
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Reachability (Sec. IV-E): a 4-D map over (z*, theta, x*, y*), the         */
/* single-structure parametrization of RM4D (Rudorfer et al. 2024) that     */
/* uses the robot's symmetry about its base z axis.  For an object frame at  */
/* world position p with x axis d, in the base frame (R_b, t_b):             */
/*   q = R_b^T (p - t_b),  e = R_b^T d,  psi = angle of (e_x, e_y),          */
/*   (x*, y*) = (q_x, q_y) turned by -psi about z,  z* = q_z,                */
/* theta = the object's approach angle.  Cell index i_d = floor((v_d - lo_d) */
/* / h_d); outside the map, or a zero cell, is not reachable.  A coordinate  */
/* within `band` of a cell boundary marks the decision as banded.            */
/* ------------------------------------------------------------------------ */
static int reachable(const uint8_t *map, const double *geom, const double *robot,
                     const double p[3], const double d[3], double theta, double band,
                     int *banded)
{
    const double *R = robot, *t = robot + 9;
    double v[3] = {p[0] - t[0], p[1] - t[1], p[2] - t[2]};
    double q[3], e[2];
    for (int c = 0; c < 3; ++c) q[c] = R[c] * v[0] + R[3 + c] * v[1] + R[6 + c] * v[2];
    for (int c = 0; c < 2; ++c) e[c] = R[c] * d[0] + R[3 + c] * d[1] + R[6 + c] * d[2];
    double n = sqrt(e[0] * e[0] + e[1] * e[1]);
    double cs = n > 0.0 ? e[0] / n : 1.0, sn = n > 0.0 ? e[1] / n : 0.0;
    double coord[4] = {q[2], theta, cs * q[0] + sn * q[1], -sn * q[0] + cs * q[1]};
    int idx[4];
    for (int a = 0; a < 4; ++a) {
        double f = (coord[a] - geom[a]) / geom[4 + a];
        double fl = floor(f);
        if (fabs(f - fl) * geom[4 + a] < band || fabs(fl + 1.0 - f) * geom[4 + a] < band) *banded = 1;
        if (!(f >= 0.0) || !(f < geom[8 + a])) return 0;
        idx[a] = (int)fl;
    }
    long cell = (((long)idx[0] * (long)geom[9] + idx[1]) * (long)geom[10] + idx[2]) * (long)geom[11] + idx[3];
    return map[cell] != 0;
}

/* Batched reachability queries (tests): pose[n][12] (world R[9] t[3] of the
 * object frame), robot[n][12], theta[n] -> out[n] (1 reachable), banded[n]. */
void orc_reach_query(int n, const uint8_t *map, const double *geom, const double *robot,
                     const double *pose, const double *theta, double band, int8_t *out,
                     int8_t *banded)
{
    for (int i = 0; i < n; ++i) {
        const double *P = pose + 12 * i;
        double p[3] = {P[9], P[10], P[11]}, d[3] = {P[0], P[3], P[6]};
        int bd = 0;
        out[i] = (int8_t)reachable(map, geom, robot + 12 * i, p, d, theta[i], band, &bd);
        banded[i] = (int8_t)bd;
    }
}

/* One relation sample (tests): out = x, y, yaw, inside, banded.            */
void orc_sample_relation(const double rel[16], const double *anchors, double ax, double ay,
                         const uint32_t w[4], double band, double out[5])
{
    double anc[8][2];
    int n = (int)rel[1];
    for (int k = 0; k < n && k < 8; ++k) { anc[k][0] = anchors[2 * k]; anc[k][1] = anchors[2 * k + 1]; }
    orc_rel_sample r = sample_relation(rel, (const double (*)[2])anc, ax, ay, w, band);
    out[0] = r.x; out[1] = r.y; out[2] = r.yaw; out[3] = r.inside; out[4] = r.banded;
}

/* ------------------------------------------------------------------------ */
/* Exported: sample poses for one attempt, dense clearance of given poses,   */
/* and the whole batched rejection-sampling generation.                      */
/* ------------------------------------------------------------------------ */

/* obj_idx[s]: object to sample for scene s (-1: none); cand_off: CSR of the
 * candidates of each scene in the output arrays.                            */
void orc_sample_poses(const orc_batch *b, const int32_t *obj_idx, const int32_t *cand_off,
                      uint64_t seed, int attempt, double *x, double *y, double *z, double *yaw,
                      int32_t *kk)
{
    for (int s = 0; s < b->n_scenes; ++s) {
        int o = obj_idx[s];
        if (o < 0) continue;
        int step = o - b->obj_off[s];
        for (int i = 0; i < cand_off[s + 1] - cand_off[s]; ++i) {
            orc_pose p = sample_pose(b, seed, s, step, o, attempt, i);
            int t = cand_off[s] + i;
            x[t] = p.x; y[t] = p.y; z[t] = p.z; yaw[t] = p.yaw;
            if (kk) kk[t] = p.k;
        }
    }
}

/* Clearance of the given candidate poses of object obj_idx[s] against the
 * boxes and grids of scene s and the first n_placed[s] objects of scene s,
 * whose world spheres are in `placed` (parallel to the template table).     */
void orc_check(const orc_batch *b, const int32_t *obj_idx, const int32_t *cand_off,
               const int32_t *n_placed, const double *placed, const double *x, const double *y,
               const double *z, const double *yaw, const int32_t *kk, double *clr)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < b->n_scenes; ++s) {
        int o = obj_idx[s];
        if (o < 0) continue;
        int ns = b->sph_off[o + 1] - b->sph_off[o];
        double *sph = (double *)malloc(sizeof(double) * 4 * (ns > 0 ? ns : 1));
        int first = b->sph_off[b->obj_off[s]];
        int n_pl = b->sph_off[b->obj_off[s] + n_placed[s]] - first;
        for (int t = cand_off[s]; t < cand_off[s + 1]; ++t) {
            orc_pose p = {x[t], y[t], z[t], yaw[t], kk ? kk[t] : -1};
            for (int k = 0; k < ns; ++k) world_sphere(b, o, b->sph_off[o] + k, p, sph + 4 * k);
            clr[t] = clearance(b, s, sph, ns, placed + 4 * first, n_pl, -INFINITY);
        }
        free(sph);
    }
}

typedef struct {
    int8_t  *status;     /* [n_scenes] 0 in progress, 1 valid, 2 invalid       */
    int32_t *n_placed;   /* [n_scenes]                                          */
    int32_t *rec_attempt;/* [n_obj] attempt that placed the object (-1 none)    */
    int32_t *rec_idx;    /* [n_obj] chosen candidate index (-1 none)            */
    double  *rec_pose;   /* [n_obj][4] x y z yaw in the support frame           */
    int32_t *rec_stable; /* [n_obj] stable-pose row of the placement (-1 none)  */
    int8_t  *rec_banded; /* [n_obj] a candidate the decision depended on was banded */
    double  *rec_clear;  /* [n_obj] clearance of the chosen candidate           */
    double  *placed;     /* [n_sph][4] world spheres of placed objects          */
    int64_t *n_cand;     /* [n_scenes] candidates evaluated                     */
} orc_gen_out;

void orc_generate(const orc_batch *b, const orc_gen_args *g, orc_gen_out *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < b->n_scenes; ++s) {
        int o0 = b->obj_off[s], o1 = b->obj_off[s + 1];
        int first = b->sph_off[o0];
        int maxsph = 1;
        for (int o = o0; o < o1; ++o)
            if (b->sph_off[o + 1] - b->sph_off[o] > maxsph) maxsph = b->sph_off[o + 1] - b->sph_off[o];
        double *sph = (double *)malloc(sizeof(double) * 4 * maxsph);
        int8_t status = 0;
        int placed_obj = 0;
        int64_t ncand = 0;
        for (int o = o0; o < o1; ++o) {
            out->rec_attempt[o] = -1; out->rec_idx[o] = -1; out->rec_banded[o] = 0;
            out->rec_clear[o] = NAN;
            out->rec_stable[o] = -1;
            for (int c = 0; c < 4; ++c) out->rec_pose[4 * o + c] = NAN;
        }
        for (int o = o0; o < o1 && status == 0; ++o) {
            int step = o - o0;
            if (g->max_steps > 0 && step >= g->max_steps) break;
            int ns = b->sph_off[o + 1] - b->sph_off[o];
            int nc = b->obj_ncand ? b->obj_ncand[o] : g->default_ncand;
            int n_pl = b->sph_off[o] - first;
            int chosen = -1, chosen_att = -1;
            double chosen_clr = NAN;
            orc_pose chosen_pose = {0, 0, 0, 0, -1};
            int8_t banded = 0;
            /* the object's relation: its anchors' recorded positions (earlier
             * objects of the scene, on the same support) */
            const double *rel = (b->obj_rel && b->obj_rel[o] >= 0) ? b->rel + 16 * b->obj_rel[o] : NULL;
            double anc[8][2];
            int rel_ok = 1;
            if (rel) {
                int na = (int)rel[1];
                if (na < 1 || na > 8) rel_ok = 0;
                for (int k = 0; k < na && k < 8 && rel_ok; ++k) {
                    int ja = (int)rel[2 + k];
                    if (ja < 0 || ja >= step || b->obj_sup[o0 + ja] != b->obj_sup[o]) { rel_ok = 0; break; }
                    anc[k][0] = out->rec_pose[4 * (o0 + ja) + 0];
                    anc[k][1] = out->rec_pose[4 * (o0 + ja) + 1];
                }
            }
            const double *uu = b->sup + 16 * b->obj_sup[o];
            const double ero = erosion_of(b, o);
            const double rax = uu[12] - uu[14] - ero, ray = uu[13] - uu[14] - ero;
            for (int a = 0; a <= g->retries && chosen < 0; ++a) {
                for (int i = 0; i < nc; ++i) {
                    orc_pose p = sample_pose(b, g->seed, s, step, o, a, i);
                    if (rel) {
                        uint32_t w[4];
                        candidate_words(b, g->seed, s, step, a, i, w);
                        orc_rel_sample q = sample_relation(rel, (const double (*)[2])anc, rax, ray, w,
                                                           g->band_region);
                        ++ncand;
                        if (q.banded) banded = 1;
                        if (!rel_ok || !q.inside) continue;   /* outside the region: not valid */
                        --ncand;
                        p.x = q.x; p.y = q.y; p.yaw = q.yaw;
                    }
                    if (b->robot && b->obj_reach && b->obj_reach[o] >= 0.0) {
                        /* the object frame's world origin and x axis */
                        double org[4], ex[4];
                        double c0[4] = {0, 0, 0, 0}, c1[4] = {1, 0, 0, 0};
                        world_point(b, o, c0, p, org);
                        world_point(b, o, c1, p, ex);
                        double d[3] = {ex[0] - org[0], ex[1] - org[1], ex[2] - org[2]};
                        int bd = 0;
                        int ok = reachable(b->reach_map, b->reach_geom, b->robot + 12 * s, org, d,
                                           b->obj_reach[o], g->band_region, &bd);
                        if (bd) banded = 1;
                        if (!ok) { ++ncand; continue; }   /* not reachable: not valid */
                    }
                    for (int k = 0; k < ns; ++k) world_sphere(b, o, b->sph_off[o] + k, p, sph + 4 * k);
                    double cl = clearance(b, s, sph, ns, out->placed + 4 * first, n_pl,
                                          g->early_exit ? g->margin - g->band : -INFINITY);
                    ++ncand;
                    if (fabs(cl - g->margin) < g->band) banded = 1;
                    if (cl >= g->margin) {   /* collision-free: clearance not below the margin */
                        chosen = i; chosen_att = a; chosen_pose = p; chosen_clr = cl;
                        break;
                    }
                }
            }
            out->rec_banded[o] = banded;
            if (chosen < 0) { status = 2; break; }
            out->rec_attempt[o] = chosen_att;
            out->rec_idx[o] = chosen;
            out->rec_clear[o] = chosen_clr;
            out->rec_pose[4 * o + 0] = chosen_pose.x;
            out->rec_pose[4 * o + 1] = chosen_pose.y;
            out->rec_pose[4 * o + 2] = chosen_pose.z;
            out->rec_pose[4 * o + 3] = chosen_pose.yaw;
            out->rec_stable[o] = chosen_pose.k;
            for (int k = 0; k < ns; ++k)
                world_sphere(b, o, b->sph_off[o] + k, chosen_pose, out->placed + 4 * (b->sph_off[o] + k));
            ++placed_obj;
        }
        if (status == 0 && placed_obj == o1 - o0) status = 1;
        out->status[s] = status;
        out->n_placed[s] = placed_obj;
        out->n_cand[s] = ncand;
        free(sph);
    }
}

/* Thread control for timing runs (OpenMP over scenes). */
#ifdef _OPENMP
#include <omp.h>
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int orc_max_threads(void) { return omp_get_max_threads(); }
#else
void orc_set_threads(int n) { (void)n; }
int orc_max_threads(void) { return 1; }
#endif
