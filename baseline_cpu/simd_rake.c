/* CPU SIMD baseline in the style of the paper's own implementation (§III-A,
 * §IV-A): MotionValidation with rake packing, W = 8 timesteps per batch (one
 * configuration per lane of an 8-wide FP32 vector), forward kinematics and
 * sphere tests in FP32, Alg. 1's combined order (each batch: every robot's
 * obstacle and self tests, then every robot pair) and early exit on the first
 * collision.  Queries run in parallel over host threads.
 *
 * A measurement baseline only: it answers in plain FP32 (no near-contact
 * re-evaluation), so a test within rounding of contact may differ from the FP64
 * definition.  The GPU library never calls it.
 *
 * Geometry conventions match the library's inputs: a joint's fixed transform F_k
 * is a row-major 3x4 matrix applied before the joint motion J_k(q) (REV_Z: rotation
 * about z; PRI_X/Y/Z: translation along an axis); a sphere lives in frame f
 * (0 = base); a box is (centre, R row-major, half-extents) with local point
 * p = R^T (x - c); a cylinder is (centre, unit axis, half-length, radius). */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define W 8
typedef float v8 __attribute__((vector_size(32)));
typedef int v8i __attribute__((vector_size(32)));

enum { J_REV_Z = 0, J_PRI_X = 1, J_PRI_Y = 2, J_PRI_Z = 3 };

typedef struct {
    int n;                  /* robots */
    const int* nj;          /* [n] joints */
    const int* j_off;       /* [n] first joint */
    const int* jtype;       /* [joints] */
    float* jfixed;          /* [joints][12] */
    float* base;            /* [n][12] */
    const int* s_off;       /* [n + 1] first sphere */
    const int* sframe;      /* [S] frame 0..nj */
    float* sxyzr;           /* [S][4] */
    const int* p_off;       /* [n + 1] first self pair */
    const int* pairs;       /* [P][2] robot-local sphere indices */
    int n_sph, n_box, n_cyl;
    float *sph, *box, *cyl; /* sph [n][4]; box [n][15] as c, R^T rows, h; cyl [n][8] */
} Scene;

static inline v8 splat(float x) { return (v8){x, x, x, x, x, x, x, x}; }
static inline int any(v8i m)
{
    int r = 0;
    for (int k = 0; k < W; ++k) r |= m[k];
    return r != 0;
}
/* lanewise max(a, 0) and |a| by bit operations */
static inline v8 vmax0(v8 a) { return (v8)((v8i)a & (a > 0.f)); }
static inline v8 vabs(v8 a) { return (v8)((v8i)a & (v8i){0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff,
                                                          0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff}); }

/* Configuration of robot r of query q at timestep t: interpolation of its
 * waypoints, rounded once to FP32 (padding past the last waypoint). */
static void config_at(const long long* wb, const int* wt, const double* wq, int dof_stride, long long p, int dof,
                      int t, float* out)
{
    long long b = wb[p], e = wb[p + 1];
    if (t >= wt[e - 1]) {
        for (int d = 0; d < dof; ++d) out[d] = (float)wq[(e - 1) * dof_stride + d];
        return;
    }
    long long lo = b, hi = e - 1;
    while (hi - lo > 1) {
        long long mid = (lo + hi) / 2;
        if (wt[mid] <= t) lo = mid; else hi = mid;
    }
    double s = (double)(t - wt[lo]) / (double)(wt[lo + 1] - wt[lo]);
    for (int d = 0; d < dof; ++d) {
        double a = wq[lo * dof_stride + d];
        out[d] = (float)(a + s * (wq[(lo + 1) * dof_stride + d] - a));
    }
}

/* Sphere centres of robot r for the W lanes' configurations q[lane][joint]. */
static void robot_spheres(const Scene* sc, int r, float q[W][8], v8* cx, v8* cy, v8* cz)
{
    v8 F[9][12];
    for (int i = 0; i < 12; ++i) F[0][i] = splat(sc->base[r * 12 + i]);
    for (int k = 0; k < sc->nj[r]; ++k) {
        const float* X = sc->jfixed + (size_t)(sc->j_off[r] + k) * 12;
        v8 A[12];
        for (int row = 0; row < 3; ++row)
            for (int col = 0; col < 4; ++col) {
                v8 v = F[k][row * 4] * X[col] + F[k][row * 4 + 1] * X[4 + col] + F[k][row * 4 + 2] * X[8 + col];
                A[row * 4 + col] = col == 3 ? v + F[k][row * 4 + 3] : v;
            }
        v8 qv;
        for (int l = 0; l < W; ++l) qv[l] = q[l][k];
        const int jt = sc->jtype[sc->j_off[r] + k];
        if (jt == J_REV_Z) {
            v8 cs, sn;
            for (int l = 0; l < W; ++l) {
                cs[l] = cosf(qv[l]);
                sn[l] = sinf(qv[l]);
            }
            for (int row = 0; row < 3; ++row) {
                v8 a0 = A[row * 4], a1 = A[row * 4 + 1];
                F[k + 1][row * 4] = a0 * cs + a1 * sn;
                F[k + 1][row * 4 + 1] = a1 * cs - a0 * sn;
                F[k + 1][row * 4 + 2] = A[row * 4 + 2];
                F[k + 1][row * 4 + 3] = A[row * 4 + 3];
            }
        } else {
            const int ax = jt - 1;
            for (int row = 0; row < 3; ++row) {
                for (int col = 0; col < 3; ++col) F[k + 1][row * 4 + col] = A[row * 4 + col];
                F[k + 1][row * 4 + 3] = A[row * 4 + 3] + A[row * 4 + ax] * qv;
            }
        }
    }
    for (int s = sc->s_off[r]; s < sc->s_off[r + 1]; ++s) {
        const v8* M = F[sc->sframe[s]];
        const float* L = sc->sxyzr + (size_t)s * 4;
        cx[s] = M[0] * L[0] + M[1] * L[1] + M[2] * L[2] + M[3];
        cy[s] = M[4] * L[0] + M[5] * L[1] + M[6] * L[2] + M[7];
        cz[s] = M[8] * L[0] + M[9] * L[1] + M[10] * L[2] + M[11];
    }
}

/* Lanes (valid mask) where a sphere of robot r hits an obstacle or a self pair hits. */
static int env_self_hit(const Scene* sc, int r, const v8* cx, const v8* cy, const v8* cz, v8i lanes)
{
    for (int s = sc->s_off[r]; s < sc->s_off[r + 1]; ++s) {
        const float rad = sc->sxyzr[(size_t)s * 4 + 3];
        v8i hit = (v8i){0};
        for (int o = 0; o < sc->n_sph; ++o) {
            const float* O = sc->sph + o * 4;
            v8 dx = cx[s] - O[0], dy = cy[s] - O[1], dz = cz[s] - O[2];
            const float R = rad + O[3];
            hit |= (dx * dx + dy * dy + dz * dz < R * R);
        }
        for (int o = 0; o < sc->n_box; ++o) {
            const float* B = sc->box + o * 15;
            v8 dx = cx[s] - B[0], dy = cy[s] - B[1], dz = cz[s] - B[2];
            v8 e0 = vmax0(vabs(dx * B[3] + dy * B[4] + dz * B[5]) - B[12]);
            v8 e1 = vmax0(vabs(dx * B[6] + dy * B[7] + dz * B[8]) - B[13]);
            v8 e2 = vmax0(vabs(dx * B[9] + dy * B[10] + dz * B[11]) - B[14]);
            hit |= (e0 * e0 + e1 * e1 + e2 * e2 < rad * rad);
        }
        for (int o = 0; o < sc->n_cyl; ++o) {
            const float* Y = sc->cyl + o * 8;
            v8 vx = cx[s] - Y[0], vy = cy[s] - Y[1], vz = cz[s] - Y[2];
            v8 h = vx * Y[3] + vy * Y[4] + vz * Y[5];
            v8 wx = vx - h * Y[3], wy = vy - h * Y[4], wz = vz - h * Y[5];
            v8 sr;
            v8 w2 = wx * wx + wy * wy + wz * wz;
            for (int l = 0; l < W; ++l) sr[l] = sqrtf(w2[l]);
            v8 er = vmax0(sr - Y[7]), ea = vmax0(vabs(h) - Y[6]);
            hit |= (er * er + ea * ea < rad * rad);
        }
        if (any(hit & lanes)) return 1;
    }
    const int s0 = sc->s_off[r];
    for (int p = sc->p_off[r]; p < sc->p_off[r + 1]; ++p) {
        const int a = s0 + sc->pairs[2 * p], b = s0 + sc->pairs[2 * p + 1];
        v8 dx = cx[a] - cx[b], dy = cy[a] - cy[b], dz = cz[a] - cz[b];
        const float R = sc->sxyzr[(size_t)a * 4 + 3] + sc->sxyzr[(size_t)b * 4 + 3];
        if (any((dx * dx + dy * dy + dz * dz < R * R) & lanes)) return 1;
    }
    return 0;
}

static int pair_hit(const Scene* sc, int i, int j, const v8* cx, const v8* cy, const v8* cz, v8i lanes)
{
    for (int a = sc->s_off[i]; a < sc->s_off[i + 1]; ++a) {
        const float ra = sc->sxyzr[(size_t)a * 4 + 3];
        v8i hit = (v8i){0};
        for (int b = sc->s_off[j]; b < sc->s_off[j + 1]; ++b) {
            v8 dx = cx[a] - cx[b], dy = cy[a] - cy[b], dz = cz[a] - cz[b];
            const float R = ra + sc->sxyzr[(size_t)b * 4 + 3];
            hit |= (dx * dx + dy * dy + dz * dz < R * R);
        }
        if (any(hit & lanes)) return 1;
    }
    return 0;
}

/* MV over queries [0, n_queries): valid_out[q] = 1 valid, 0 invalid.  check_env
 * adds obstacle and self tests; exhaustive evaluates every batch (no early exit;
 * same answers).  *states_out receives the robot-states evaluated.  Returns 0, or
 * -1 on a malformed argument. */
int simd_mv(int n_robots, const int* nj, const int* jtype, const double* jfixed, const double* base,
            const int* ns, const int* sframe, const double* sxyzr, const int* nself, const int* self_pairs,
            int n_sph, const double* sph, int n_box, const double* box, int n_cyl, const double* cyl,
            int check_env, int exhaustive, long long n_queries, int dof_stride, const long long* wp_begin,
            const int* wp_t, const double* wp_q, unsigned char* valid_out, long long* states_out, int nthreads)
{
    if (n_robots < 1 || n_robots > 32 || dof_stride < 1) return -1;
    int* j_off = calloc((size_t)n_robots, sizeof(int));
    int* s_off = calloc((size_t)n_robots + 1, sizeof(int));
    int* p_off = calloc((size_t)n_robots + 1, sizeof(int));
    int J = 0;
    for (int r = 0; r < n_robots; ++r) {
        if (nj[r] < 0 || nj[r] > 8 || nj[r] > dof_stride) { free(j_off); free(s_off); free(p_off); return -1; }
        j_off[r] = J;
        J += nj[r];
        s_off[r + 1] = s_off[r] + ns[r];
        p_off[r + 1] = p_off[r] + nself[r];
    }
    const int S = s_off[n_robots];
    Scene sc = {n_robots, nj, j_off, jtype, malloc(sizeof(float) * 12 * (size_t)(J + 1)),
                malloc(sizeof(float) * 12 * (size_t)n_robots), s_off, sframe, malloc(sizeof(float) * 4 * (size_t)(S + 1)),
                p_off, self_pairs, n_sph, n_box, n_cyl, malloc(sizeof(float) * 4 * (size_t)(n_sph + 1)),
                malloc(sizeof(float) * 15 * (size_t)(n_box + 1)), malloc(sizeof(float) * 8 * (size_t)(n_cyl + 1))};
    for (int i = 0; i < 12 * J; ++i) sc.jfixed[i] = (float)jfixed[i];
    for (int i = 0; i < 12 * n_robots; ++i) sc.base[i] = (float)base[i];
    for (int i = 0; i < 4 * S; ++i) sc.sxyzr[i] = (float)sxyzr[i];
    for (int i = 0; i < 4 * n_sph; ++i) sc.sph[i] = (float)sph[i];
    for (int o = 0; o < n_box; ++o) {
        const double* B = box + o * 15;
        float* D = sc.box + o * 15;
        for (int k = 0; k < 3; ++k) D[k] = (float)B[k];
        for (int k = 0; k < 3; ++k)          /* row k of R^T = column k of R */
            for (int j = 0; j < 3; ++j) D[3 + 3 * k + j] = (float)B[3 + 3 * j + k];
        for (int k = 0; k < 3; ++k) D[12 + k] = (float)B[12 + k];
    }
    for (int i = 0; i < 8 * n_cyl; ++i) sc.cyl[i] = (float)cyl[i];

    long long states = 0;
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();   /* this call only */
#pragma omp parallel num_threads(nt) reduction(+ : states)
#endif
    {
        /* 32-byte aligned: the vectors are moved with aligned AVX loads and stores */
        v8* cx = aligned_alloc(32, sizeof(v8) * (size_t)(S + 1));
        v8* cy = aligned_alloc(32, sizeof(v8) * (size_t)(S + 1));
        v8* cz = aligned_alloc(32, sizeof(v8) * (size_t)(S + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (long long qi = 0; qi < n_queries; ++qi) {
            const long long p0 = qi * n_robots;
            int T = 0;
            for (int r = 0; r < n_robots; ++r) {
                const int last = wp_t[wp_begin[p0 + r + 1] - 1] + 1;
                if (last > T) T = last;
            }
            const int nb = (T + W - 1) / W;        /* batches; lane k of batch b: t = b + k nb */
            int valid = 1;
            for (int b = 0; b < nb && (valid || exhaustive); ++b) {
                int ts[W];
                v8i lanes;
                for (int k = 0; k < W; ++k) {
                    const int t = b + k * nb;
                    lanes[k] = t < T ? -1 : 0;
                    ts[k] = t < T ? t : T - 1;
                    if (t < T) states += n_robots;
                }
                for (int r = 0; r < n_robots; ++r) {
                    float q[W][8];
                    for (int k = 0; k < W; ++k) config_at(wp_begin, wp_t, wp_q, dof_stride, p0 + r, nj[r], ts[k], q[k]);
                    robot_spheres(&sc, r, q, cx, cy, cz);
                }
                int hit = 0;
                if (check_env)
                    for (int r = 0; r < n_robots && (!hit || exhaustive); ++r) hit |= env_self_hit(&sc, r, cx, cy, cz, lanes);
                for (int i = 0; i + 1 < n_robots && (!hit || exhaustive); ++i)
                    for (int j = i + 1; j < n_robots && (!hit || exhaustive); ++j) hit |= pair_hit(&sc, i, j, cx, cy, cz, lanes);
                if (hit) valid = 0;
            }
            valid_out[qi] = (unsigned char)valid;
        }
        free(cx);
        free(cy);
        free(cz);
    }
    if (states_out) *states_out = states;
    free(sc.jfixed); free(sc.base); free(sc.sxyzr); free(sc.sph); free(sc.box); free(sc.cyl);
    free(j_off); free(s_off); free(p_off);
    return 0;
}
