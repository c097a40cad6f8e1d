/*
 * fk.c -- plain FP64 CPU oracle for batched forward kinematics of articulated
 * furniture parts.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: nothing in the product path links,
 * imports or calls it, and it shares no code with the GPU path.
 *
 * What it computes (Sceniris, arXiv 2512.16896): the batched scene
 * representation stores one transform per scene instance on every edge of the
 * scene graph, and a batched forward-kinematics function moves the
 * articulated parts of all instances at once (Sec. IV-B); the experiments
 * randomize the drawer joint state of every scene (Sec. V-A).
 *
 * Model (the project's reading; the paper gives no formulas): a scene has an
 * articulated base at world pose T_base and a list of joints in topological
 * order.  Joint i hangs from link parent(i) (-1: the base) at the fixed pose
 * T_i (joint frame in the parent link frame) and moves its child link by its
 * value q_i along / about the unit axis a_i given in the joint frame:
 *   prismatic  M(q) = translation by q a
 *   revolute   M(q) = rotation by angle q about a (Rodrigues' formula)
 *   link_i = link_parent(i) * T_i * M(q_i),   link_-1 = T_base.
 * A box row or support row attached to link i at the local pose L has the
 * world pose link_i * L (rotation and translation of the row; the half
 * extents / support sizes are untouched).
 * Sampled joint values: q_i = lower_i + u (upper_i - lower_i), u from
 * Philox4x32-10 with key = seed and counter = (i - first joint of the scene,
 * 0x30000, 0, scene number), first output word, mapped like every other
 * uniform of the method (orc_u01 in oracle.c).
 *
 * Layouts (row-major, FP64 copies of the FP32 inputs):
 *   joint [n_joints][24]: type (0 prismatic, 1 revolute), parent (index within
 *         the scene, -1 base), lower, upper, axis[3], pad, R_j[9], t_j[3], pad[4]
 *   base  [n_scenes][12]: R[9], t[3]        (world pose of each scene's base)
 *   local [n][12]:        R[9], t[3]        (pose of a row in its link frame)
 *   link  [n_joints][12]: R[9], t[3]        (output: world pose of each child link)
 */
#include <math.h>
#include <stdint.h>

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
double orc_u01(uint32_t w);

/* C = A B for 3x4 rigid transforms [R | t] stored R[9], t[3]. */
static void compose(const double *A, const double *B, double *C)
{
    double R[9], t[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            R[3 * r + c] = A[3 * r + 0] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
        t[r] = A[3 * r + 0] * B[9] + A[3 * r + 1] * B[10] + A[3 * r + 2] * B[11] + A[9 + r];
    }
    for (int i = 0; i < 9; ++i) C[i] = R[i];
    for (int i = 0; i < 3; ++i) C[9 + i] = t[i];
}

/* Joint motion M(q) as a 3x4 transform. */
static void motion(int type, const double a[3], double q, double *M)
{
    for (int i = 0; i < 12; ++i) M[i] = 0.0;
    if (type == 0) {
        M[0] = M[4] = M[8] = 1.0;
        M[9] = q * a[0];
        M[10] = q * a[1];
        M[11] = q * a[2];
        return;
    }
    /* Rodrigues: R = I + sin(q) K + (1 - cos(q)) K^2, K the cross-product matrix of a */
    double K[9] = {0.0, -a[2], a[1], a[2], 0.0, -a[0], -a[1], a[0], 0.0};
    double K2[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            K2[3 * r + c] = K[3 * r + 0] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
    double s = sin(q), v = 1.0 - cos(q);
    for (int i = 0; i < 9; ++i) M[i] = (i % 4 == 0 ? 1.0 : 0.0) + s * K[i] + v * K2[i];
}

/* Sampled joint values of every joint (sample != 0), then the link poses of
 * every scene.  q is an input when sample == 0.                             */
void orc_fk_links(int n_scenes, const int32_t *joint_off, const double *joint,
                  const double *base, const int32_t *scene_id, uint64_t seed, int sample,
                  double *q, double *link)
{
    for (int s = 0; s < n_scenes; ++s) {
        const int j0 = joint_off[s], j1 = joint_off[s + 1];
        const uint32_t sid = scene_id ? (uint32_t)scene_id[s] : (uint32_t)s;
        for (int i = j0; i < j1; ++i) {
            const double *J = joint + 24 * i;
            if (sample) {
                uint32_t ctr[4] = {(uint32_t)(i - j0), 0x30000u, 0u, sid};
                uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
                uint32_t w[4];
                orc_philox4x32_10(ctr, key, w);
                q[i] = J[2] + orc_u01(w[0]) * (J[3] - J[2]);
            }
            const int parent = (int)J[1];
            const double *P = parent < 0 ? base + 12 * s : link + 12 * (j0 + parent);
            double Tj[12], M[12], PT[12];
            for (int k = 0; k < 9; ++k) Tj[k] = J[8 + k];
            for (int k = 0; k < 3; ++k) Tj[9 + k] = J[17 + k];
            motion((int)J[0], J + 4, q[i], M);
            compose(P, Tj, PT);
            compose(PT, M, link + 12 * i);
        }
    }
}

/* Rows (16 floats: R[9], t[3], rest untouched) attached to links: row r moves
 * to link[row_link[r]] * local[r] when row_link[r] >= 0.                     */
void orc_fk_rows(int n_rows, const int32_t *row_link, const double *local, const double *link,
                 double *rows)
{
    for (int r = 0; r < n_rows; ++r) {
        if (row_link[r] < 0) continue;
        double W[12];
        compose(link + 12 * row_link[r], local + 12 * r, W);
        for (int k = 0; k < 12; ++k) rows[16 * r + k] = W[k];
    }
}
