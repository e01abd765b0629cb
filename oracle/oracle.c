/*
 * FP64 CPU oracle for multi-robot MotionValidation (MV) and FindFirstConflict (FFC).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no source, header,
 * table or helper with the GPU library; the two meet only at the seeded input
 * arrays.
 *
 * What it computes is the plain definition of the two primitives:
 *
 *   MV  (paper §III-A, Alg. 1): a set of synchronised paths is valid iff at
 *       every timestep t in [0, T) no robot collides with an obstacle or with
 *       itself (only when environment checking is on; self-collision belongs to
 *       the robot-obstacle validation, §III-A) and no two robots collide.
 *       Hierarchical/combined ordering and rake/linear packing only change the
 *       order of the checks (§III-A), never the answer, so this scans t
 *       ascending, robots in index order, and stops at the first hit.
 *   FFC (paper §III-B, Alg. 2): the earliest robot-robot conflict.  Alg. 2
 *       visits pairs i<j in ascending order inside each batch, keeps a conflict
 *       only when its timestep is strictly earlier, and returns as soon as a
 *       batch holds one; that is exactly the lexicographic minimum of
 *       (t, i, j) over all colliding (t, i, j).  No obstacle or self checks
 *       (§III-B).  No conflict gives (-1, -1, -1).
 *
 * Paths (§III-A; PackCfgBatch and its padding note): robot i's path has
 * L_i = last waypoint time + 1 states, T = max_i L_i, and for t at or beyond
 * its last waypoint a robot holds its last configuration.  Between waypoints
 * the state is Q_k + s (Q_{k+1} - Q_k) with s = (t - tau_k)/(tau_{k+1} - tau_k),
 * evaluated as a separate multiply and add (no fused multiply-add: the build
 * uses -ffp-contract=off).
 *
 * Geometry (§II-B: robots are sets of spheres): signed clearance delta, and a
 * pair collides iff delta < 0 (touching is free):
 *   sphere-sphere    |x - y| - (r + s)
 *   sphere-box       p = R^T (x - c), e = max(|p| - h, 0);
 *                    outside: |e| - r, inside: -min_k(h_k - |p_k|) - r
 *   sphere-cylinder  v = x - c, h = v.u, w = v - h u, s = |w|;
 *                    e_r = max(s - R, 0), e_a = max(|h| - hl, 0);
 *                    outside: sqrt(e_r^2 + e_a^2) - r, inside: -min(R - s, hl - |h|) - r
 *   sphere-point     |x - p| - (r + r_p)
 *
 * Kinematics: Frame_0 = base, Frame_k = (Frame_{k-1} F_k) J_k(q_k) with J a
 * rotation about z (REV_Z) or a translation along x/y/z (PRI_*); a sphere on
 * frame f with local centre c sits at Frame_f c.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { J_REV_Z = 0, J_PRI_X = 1, J_PRI_Y = 2, J_PRI_Z = 3 };

#define ORC_MAX_JOINTS 16

/* ------------------------------------------------------------------------- */
/* rigid transforms as 3x4 row-major [R | p]                                  */

typedef struct { double m[12]; } xf;

static void xf_mul(const xf* A, const xf* B, xf* C)
{
    /* C = A * B for 3x4 homogeneous transforms. */
    xf r;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            double s = A->m[i * 4 + 0] * B->m[0 * 4 + j];
            s = s + A->m[i * 4 + 1] * B->m[1 * 4 + j];
            s = s + A->m[i * 4 + 2] * B->m[2 * 4 + j];
            r.m[i * 4 + j] = s;
        }
        double t = A->m[i * 4 + 0] * B->m[3];
        t = t + A->m[i * 4 + 1] * B->m[7];
        t = t + A->m[i * 4 + 2] * B->m[11];
        r.m[i * 4 + 3] = t + A->m[i * 4 + 3];
    }
    *C = r;
}

static void xf_joint(int type, double q, xf* J)
{
    memset(J, 0, sizeof(*J));
    J->m[0] = 1.0; J->m[5] = 1.0; J->m[10] = 1.0;
    switch (type) {
    case J_REV_Z: {
        double c = cos(q), s = sin(q);
        J->m[0] = c;  J->m[1] = -s;
        J->m[4] = s;  J->m[5] = c;
        break;
    }
    case J_PRI_X: J->m[3] = q; break;
    case J_PRI_Y: J->m[7] = q; break;
    case J_PRI_Z: J->m[11] = q; break;
    default: break;
    }
}

static void xf_apply(const xf* A, const double* c, double* out)
{
    for (int i = 0; i < 3; ++i) {
        double s = A->m[i * 4 + 0] * c[0];
        s = s + A->m[i * 4 + 1] * c[1];
        s = s + A->m[i * 4 + 2] * c[2];
        out[i] = s + A->m[i * 4 + 3];
    }
}

/* ------------------------------------------------------------------------- */
/* team and environment as flat arrays                                        */

typedef struct {
    int32_t n_robots;
    const int32_t* n_joints;      /* [n_robots] */
    const int32_t* joint_off;     /* [n_robots] offset into joint arrays */
    const int32_t* joint_type;    /* [total joints] */
    const double*  joint_fixed;   /* [total joints][12] */
    const int32_t* sphere_off;    /* [n_robots + 1] */
    const int32_t* sphere_frame;  /* [total spheres] */
    const double*  sphere_xyzr;   /* [total spheres][4] */
    const int32_t* self_off;      /* [n_robots + 1] */
    const int32_t* self_pairs;    /* [total pairs][2], robot-local sphere indices */
    const double*  base;          /* [n_robots][12] */
} orc_team;

typedef struct {
    int32_t n_spheres; const double* spheres;     /* [n][4] */
    int32_t n_boxes;   const double* boxes;       /* [n][15] c, R row-major, h */
    int32_t n_cyls;    const double* cyls;        /* [n][8] c, u, hl, R */
    int64_t n_points;  const double* points;      /* [n][3] */
    double point_radius;
    /* point index (k-d tree) built by orc_env_build */
    int64_t* kd_perm;
    double* kd_split;
    int32_t* kd_axis;
    int64_t kd_nodes;
} orc_env;

typedef struct {
    int32_t n_queries;
    int32_t n_robots;
    int32_t dof_stride;
    const int64_t* wp_begin;      /* [n_queries * n_robots + 1] */
    const int32_t* wp_t;
    const double*  wp_q;          /* [n_wp][dof_stride] */
} orc_paths;

/* ------------------------------------------------------------------------- */
/* clearances                                                                 */

double orc_clear_sphere_sphere(const double* x, double r, const double* y, double s)
{
    double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    return sqrt(dx * dx + dy * dy + dz * dz) - (r + s);
}

double orc_clear_sphere_box(const double* x, double r, const double* box)
{
    const double* c = box;
    const double* R = box + 3;
    const double* h = box + 12;
    double v[3] = { x[0] - c[0], x[1] - c[1], x[2] - c[2] };
    double p[3], e[3];
    int inside = 1;
    for (int k = 0; k < 3; ++k) {
        /* p = R^T v: column k of R dotted with v */
        p[k] = R[0 * 3 + k] * v[0] + R[1 * 3 + k] * v[1] + R[2 * 3 + k] * v[2];
        double ek = fabs(p[k]) - h[k];
        e[k] = ek > 0.0 ? ek : 0.0;
        if (e[k] > 0.0) inside = 0;
    }
    if (inside) {
        double m = h[0] - fabs(p[0]);
        for (int k = 1; k < 3; ++k) {
            double mk = h[k] - fabs(p[k]);
            if (mk < m) m = mk;
        }
        return -m - r;
    }
    return sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) - r;
}

double orc_clear_sphere_cylinder(const double* x, double r, const double* cyl)
{
    const double* c = cyl;
    const double* u = cyl + 3;
    double hl = cyl[6], R = cyl[7];
    double v[3] = { x[0] - c[0], x[1] - c[1], x[2] - c[2] };
    double h = v[0] * u[0] + v[1] * u[1] + v[2] * u[2];
    double w[3] = { v[0] - h * u[0], v[1] - h * u[1], v[2] - h * u[2] };
    double s = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double er = s - R > 0.0 ? s - R : 0.0;
    double ea = fabs(h) - hl > 0.0 ? fabs(h) - hl : 0.0;
    if (er == 0.0 && ea == 0.0) {
        double m1 = R - s, m2 = hl - fabs(h);
        return -(m1 < m2 ? m1 : m2) - r;
    }
    return sqrt(er * er + ea * ea) - r;
}

double orc_clear_sphere_point(const double* x, double r, const double* p, double rp)
{
    double dx = x[0] - p[0], dy = x[1] - p[1], dz = x[2] - p[2];
    return sqrt(dx * dx + dy * dy + dz * dz) - (r + rp);
}

/* ------------------------------------------------------------------------- */
/* kinematics                                                                 */

/* World-frame sphere centres (and radii) of robot `r` at configuration q.
 * out: [n_spheres][4].  frames_out (optional): [n_joints + 1][12]. */
void orc_fk_robot(const orc_team* tm, int r, const double* q, double* out, double* frames_out)
{
    int nj = tm->n_joints[r];
    const int32_t* jt = tm->joint_type + tm->joint_off[r];
    const double* jf = tm->joint_fixed + (int64_t)tm->joint_off[r] * 12;
    xf frames[ORC_MAX_JOINTS + 1];
    memcpy(frames[0].m, tm->base + (int64_t)r * 12, sizeof(double) * 12);
    for (int k = 1; k <= nj; ++k) {
        xf F, J, tmp;
        memcpy(F.m, jf + (int64_t)(k - 1) * 12, sizeof(double) * 12);
        xf_joint(jt[k - 1], q[k - 1], &J);
        xf_mul(&frames[k - 1], &F, &tmp);
        xf_mul(&tmp, &J, &frames[k]);
    }
    if (frames_out)
        for (int k = 0; k <= nj; ++k) memcpy(frames_out + k * 12, frames[k].m, sizeof(double) * 12);
    int s0 = tm->sphere_off[r], s1 = tm->sphere_off[r + 1];
    for (int s = s0; s < s1; ++s) {
        const double* c = tm->sphere_xyzr + (int64_t)s * 4;
        xf_apply(&frames[tm->sphere_frame[s]], c, out + (int64_t)(s - s0) * 4);
        out[(int64_t)(s - s0) * 4 + 3] = c[3];
    }
}

/* ------------------------------------------------------------------------- */
/* path states                                                                */

/* Configuration of one path at integer timestep t (dof values written to q). */
void orc_path_state(const int32_t* wt, const double* wq, int64_t n_wp, int32_t dof_stride,
                    int32_t dof, int64_t t, double* q)
{
    if (t >= wt[n_wp - 1]) {
        for (int d = 0; d < dof; ++d) q[d] = wq[(n_wp - 1) * dof_stride + d];
        return;
    }
    int64_t k = 0;
    while (k + 1 < n_wp && wt[k + 1] <= t) ++k;
    double s = (double)(t - wt[k]) / (double)(wt[k + 1] - wt[k]);
    for (int d = 0; d < dof; ++d) {
        double a = wq[k * dof_stride + d], b = wq[(k + 1) * dof_stride + d];
        double step = s * (b - a);
        q[d] = a + step;
    }
}

static int64_t path_len(const orc_paths* P, int64_t qi, int r)
{
    int64_t e = P->wp_begin[qi * P->n_robots + r + 1];
    return (int64_t)P->wp_t[e - 1] + 1;
}

int64_t orc_query_horizon(const orc_paths* P, int64_t qi)
{
    int64_t T = 0;
    for (int r = 0; r < P->n_robots; ++r) {
        int64_t L = path_len(P, qi, r);
        if (L > T) T = L;
    }
    return T;
}

static void robot_spheres_at(const orc_team* tm, const orc_paths* P, int64_t qi, int r, int64_t t,
                             double* out)
{
    double q[ORC_MAX_JOINTS];
    int64_t b = P->wp_begin[qi * P->n_robots + r], e = P->wp_begin[qi * P->n_robots + r + 1];
    orc_path_state(P->wp_t + b, P->wp_q + b * P->dof_stride, e - b, P->dof_stride,
                   tm->n_joints[r], t, q);
    orc_fk_robot(tm, r, q, out, NULL);
}

/* ------------------------------------------------------------------------- */
/* point cloud: k-d tree (median splits, implicit balanced layout)            */

#define KD_LEAF 16

typedef struct { const double* pts; int axis; } kd_sort_ctx;
static __thread const double* g_kd_pts;
static __thread int g_kd_axis;

static int kd_cmp(const void* a, const void* b)
{
    double va = g_kd_pts[*(const int64_t*)a * 3 + g_kd_axis];
    double vb = g_kd_pts[*(const int64_t*)b * 3 + g_kd_axis];
    return (va > vb) - (va < vb);
}

static void kd_build_rec(orc_env* E, int64_t node, int64_t lo, int64_t hi)
{
    if (hi - lo <= KD_LEAF || node >= E->kd_nodes) return;
    double mn[3], mx[3];
    for (int a = 0; a < 3; ++a) { mn[a] = INFINITY; mx[a] = -INFINITY; }
    for (int64_t i = lo; i < hi; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = E->points[E->kd_perm[i] * 3 + a];
            if (v < mn[a]) mn[a] = v;
            if (v > mx[a]) mx[a] = v;
        }
    int axis = 0;
    for (int a = 1; a < 3; ++a) if (mx[a] - mn[a] > mx[axis] - mn[axis]) axis = a;
    g_kd_pts = E->points;
    g_kd_axis = axis;
    qsort(E->kd_perm + lo, (size_t)(hi - lo), sizeof(int64_t), kd_cmp);
    int64_t mid = lo + (hi - lo) / 2;
    E->kd_axis[node] = axis;
    E->kd_split[node] = E->points[E->kd_perm[mid] * 3 + axis];
    kd_build_rec(E, 2 * node + 1, lo, mid);
    kd_build_rec(E, 2 * node + 2, mid, hi);
}

/* Any point within distance `reach` of x (strictly closer than reach)? Exact: the
 * tree only prunes subtrees whose split plane is farther than reach. */
static int kd_any_hit(const orc_env* E, int64_t node, int64_t lo, int64_t hi, const double* x,
                      double r)
{
    if (hi - lo <= KD_LEAF || node >= E->kd_nodes || E->kd_axis[node] < 0) {
        for (int64_t i = lo; i < hi; ++i)
            if (orc_clear_sphere_point(x, r, E->points + E->kd_perm[i] * 3, E->point_radius) < 0.0)
                return 1;
        return 0;
    }
    int64_t mid = lo + (hi - lo) / 2;
    int axis = E->kd_axis[node];
    double d = x[axis] - E->kd_split[node];
    double reach = r + E->point_radius;
    /* left subtree holds values <= split, right subtree values >= split */
    if (d <= reach && kd_any_hit(E, 2 * node + 1, lo, mid, x, r)) return 1;
    if (-d <= reach && kd_any_hit(E, 2 * node + 2, mid, hi, x, r)) return 1;
    return 0;
}

int orc_env_build(orc_env* E)
{
    E->kd_perm = NULL; E->kd_split = NULL; E->kd_axis = NULL; E->kd_nodes = 0;
    if (E->n_points <= 0) return 0;
    int64_t nodes = 1;
    while (nodes * KD_LEAF < E->n_points) nodes *= 2;
    nodes = nodes * 2;
    E->kd_nodes = nodes;
    E->kd_perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)E->n_points);
    E->kd_split = (double*)malloc(sizeof(double) * (size_t)nodes);
    E->kd_axis = (int32_t*)malloc(sizeof(int32_t) * (size_t)nodes);
    if (!E->kd_perm || !E->kd_split || !E->kd_axis) return -1;
    for (int64_t i = 0; i < E->n_points; ++i) E->kd_perm[i] = i;
    for (int64_t i = 0; i < nodes; ++i) E->kd_axis[i] = -1;
    kd_build_rec(E, 0, 0, E->n_points);
    return 0;
}

void orc_env_free(orc_env* E)
{
    free(E->kd_perm); free(E->kd_split); free(E->kd_axis);
    E->kd_perm = NULL; E->kd_split = NULL; E->kd_axis = NULL; E->kd_nodes = 0;
}

/* Brute-force point check (used by the tests to pin the tree). */
int orc_points_any_hit_brute(const orc_env* E, const double* x, double r)
{
    for (int64_t i = 0; i < E->n_points; ++i)
        if (orc_clear_sphere_point(x, r, E->points + i * 3, E->point_radius) < 0.0) return 1;
    return 0;
}

int orc_points_any_hit(const orc_env* E, const double* x, double r)
{
    if (E->n_points <= 0) return 0;
    if (!E->kd_perm) return orc_points_any_hit_brute(E, x, r);
    return kd_any_hit(E, 0, 0, E->n_points, x, r);
}

/* ------------------------------------------------------------------------- */
/* single-state checks                                                        */

/* Robot-obstacle and self collision of one robot state (spheres in world frame). */
/* Robot r's self pairs and obstacles at one state.  all = 0 stops at the first
 * collision; all = 1 evaluates every relation (exhaustive validation, paper
 * Sec. IV-A: every collision relation at every intermediate state). */
static int env_self_hit(const orc_team* tm, const orc_env* E, int r, const double* sph, int all)
{
    int s0 = tm->sphere_off[r], ns = tm->sphere_off[r + 1] - s0;
    int hit = 0;
    for (int p = tm->self_off[r]; p < tm->self_off[r + 1]; ++p) {
        int a = tm->self_pairs[2 * p], b = tm->self_pairs[2 * p + 1];
        if (orc_clear_sphere_sphere(sph + a * 4, sph[a * 4 + 3], sph + b * 4, sph[b * 4 + 3]) < 0.0) {
            hit = 1;
            if (!all) return 1;
        }
    }
    if (!E) return hit;
    for (int a = 0; a < ns; ++a) {
        const double* x = sph + a * 4;
        double rad = x[3];
        for (int o = 0; o < E->n_spheres; ++o)
            if (orc_clear_sphere_sphere(x, rad, E->spheres + o * 4, E->spheres[o * 4 + 3]) < 0.0) {
                hit = 1;
                if (!all) return 1;
            }
        for (int o = 0; o < E->n_boxes; ++o)
            if (orc_clear_sphere_box(x, rad, E->boxes + o * 15) < 0.0) {
                hit = 1;
                if (!all) return 1;
            }
        for (int o = 0; o < E->n_cyls; ++o)
            if (orc_clear_sphere_cylinder(x, rad, E->cyls + o * 8) < 0.0) {
                hit = 1;
                if (!all) return 1;
            }
        if (orc_points_any_hit(E, x, rad)) {
            hit = 1;
            if (!all) return 1;
        }
    }
    return hit;
}

static int pair_hit(const double* si, int ni, const double* sj, int nj, int all)
{
    int hit = 0;
    for (int a = 0; a < ni; ++a)
        for (int b = 0; b < nj; ++b)
            if (orc_clear_sphere_sphere(si + a * 4, si[a * 4 + 3], sj + b * 4, sj[b * 4 + 3]) < 0.0) {
                hit = 1;
                if (!all) return 1;
            }
    return hit;
}

static int team_total_spheres(const orc_team* tm) { return tm->sphere_off[tm->n_robots]; }

/* ------------------------------------------------------------------------- */
/* MV and FFC                                                                 */

/* MV of one query.  Returns 1 valid, 0 invalid.  first_hit (optional) gets the
 * first colliding timestep of the ascending scan, -1 if valid.  exhaustive = 1
 * evaluates every relation at every state instead of stopping (same answer). */
/* Prioritised MV (PP-ST-RRT, §III-C): a robot is planned against the fixed paths
 * of others.  Robot r is in focus iff bit r of focus is set; focus = 0 puts every
 * robot in focus (plain MV). */
static int in_focus(uint32_t focus, int r)
{
    return focus == 0 || ((focus >> r) & 1u);
}

/* MV of one query (Alg. 1 as a plain scan): at every timestep, the obstacle and
 * self tests of each robot in focus, then every robot pair with at least one
 * robot in focus. */
static int mv_one(const orc_team* tm, const orc_env* E, const orc_paths* P, int64_t qi,
                  int check_env, int exhaustive, uint32_t focus, double* buf, int64_t* first_hit)
{
    int n = tm->n_robots;
    int64_t T = orc_query_horizon(P, qi);
    int64_t fh = -1;
    for (int64_t t = 0; t < T; ++t) {
        int hit = 0;
        for (int r = 0; r < n; ++r)
            robot_spheres_at(tm, P, qi, r, t, buf + (int64_t)tm->sphere_off[r] * 4);
        if (check_env)
            for (int r = 0; r < n && (exhaustive || !hit); ++r)
                if (in_focus(focus, r))
                    hit |= env_self_hit(tm, E, r, buf + (int64_t)tm->sphere_off[r] * 4, exhaustive);
        for (int i = 0; i + 1 < n && (exhaustive || !hit); ++i)
            for (int j = i + 1; j < n && (exhaustive || !hit); ++j)
                if (in_focus(focus, i) || in_focus(focus, j))
                    hit |= pair_hit(buf + (int64_t)tm->sphere_off[i] * 4, tm->sphere_off[i + 1] - tm->sphere_off[i],
                                buf + (int64_t)tm->sphere_off[j] * 4, tm->sphere_off[j + 1] - tm->sphere_off[j],
                                exhaustive);
        if (hit && fh < 0) {
            fh = t;
            if (!exhaustive) break;
        }
    }
    if (first_hit) *first_hit = fh;
    return fh < 0;
}

static void ffc_one(const orc_team* tm, const orc_paths* P, int64_t qi, double* buf, int32_t* out)
{
    int n = tm->n_robots;
    int64_t T = orc_query_horizon(P, qi);
    for (int64_t t = 0; t < T; ++t) {
        for (int r = 0; r < n; ++r)
            robot_spheres_at(tm, P, qi, r, t, buf + (int64_t)tm->sphere_off[r] * 4);
        for (int i = 0; i + 1 < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if (pair_hit(buf + (int64_t)tm->sphere_off[i] * 4, tm->sphere_off[i + 1] - tm->sphere_off[i],
                             buf + (int64_t)tm->sphere_off[j] * 4, tm->sphere_off[j + 1] - tm->sphere_off[j], 0)) {
                    out[0] = (int32_t)t; out[1] = i; out[2] = j;
                    return;
                }
    }
    out[0] = -1; out[1] = -1; out[2] = -1;
}

/* Threads of one call: nthreads if positive, else the OpenMP default; given to
 * that call's parallel region only, so the process-wide default is unchanged. */
static int set_threads(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* MV over queries [q0, q1).  env may be NULL (no obstacles).  check_env = 0 skips
 * robot-obstacle and self checks; exhaustive = 1 evaluates every relation at every
 * state; focus selects the robots validated (in_focus).  valid_out[q - q0];
 * first_hit_out optional. */
int orc_mv(const orc_team* tm, const orc_env* E, const orc_paths* P, int64_t q0, int64_t q1,
           int32_t check_env, int32_t exhaustive, uint32_t focus, uint8_t* valid_out, int64_t* first_hit_out,
           int32_t nthreads)
{
    const int nt = set_threads(nthreads);
    int S = team_total_spheres(tm);
    int err = 0;
#pragma omp parallel num_threads(nt)
    {
        double* buf = (double*)malloc(sizeof(double) * 4 * (size_t)(S > 0 ? S : 1));
        if (!buf) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int64_t qi = q0; qi < q1; ++qi) {
                int64_t fh = -1;
                valid_out[qi - q0] = (uint8_t)mv_one(tm, E, P, qi, check_env, exhaustive, focus, buf, &fh);
                if (first_hit_out) first_hit_out[qi - q0] = fh;
            }
            free(buf);
        }
    }
    return err ? -1 : 0;
}

/* FFC over queries [q0, q1).  out: [q1 - q0][3] = (t, ri, rj). */
int orc_ffc(const orc_team* tm, const orc_paths* P, int64_t q0, int64_t q1, int32_t* out,
            int32_t nthreads)
{
    const int nt = set_threads(nthreads);
    int S = team_total_spheres(tm);
    int err = 0;
#pragma omp parallel num_threads(nt)
    {
        double* buf = (double*)malloc(sizeof(double) * 4 * (size_t)(S > 0 ? S : 1));
        if (!buf) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int64_t qi = q0; qi < q1; ++qi) ffc_one(tm, P, qi, buf, out + (qi - q0) * 3);
            free(buf);
        }
    }
    return err ? -1 : 0;
}

/* World sphere positions of every robot of query qi at timestep t: out [S][4]. */
void orc_team_spheres(const orc_team* tm, const orc_paths* P, int64_t qi, int64_t t, double* out)
{
    for (int r = 0; r < tm->n_robots; ++r)
        robot_spheres_at(tm, P, qi, r, t, out + (int64_t)tm->sphere_off[r] * 4);
}

/* Timesteps for one straight-line motion: ceil(d / step), d the L2 (metric 0) or
 * L-infinity (metric 1) norm of dq (paper §IV-A: bounded C-space motion per
 * timestep). */
int64_t orc_motion_steps(const double* dq, int32_t dof, double step, int32_t metric)
{
    double d = 0.0;
    if (metric == 0) {
        for (int k = 0; k < dof; ++k) d = d + dq[k] * dq[k];
        d = sqrt(d);
    } else {
        for (int k = 0; k < dof; ++k) if (fabs(dq[k]) > d) d = fabs(dq[k]);
    }
    return (int64_t)ceil(d / step);
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
