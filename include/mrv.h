/*
 * mrv.h -- C ABI of libmrv: multi-robot MotionValidation (MV) and
 * FindFirstConflict (FFC) on an AMD Instinct MI355X (gfx950).
 *
 * The problem (paper §III-A, Alg. 1 input; §III-B, Alg. 2 input): a team of
 * robots, each a set of spheres attached to a kinematic chain (paper §II-B:
 * sphere-based robot representation), an obstacle set, and one timed path per
 * robot.  The state of robot i at integer timestep t is the linear
 * interpolation of its waypoints around t, and its last waypoint for every t at
 * or after the last waypoint time (padding, §III-A).  T = max_i L_i with
 * L_i = last waypoint time + 1.
 *
 *   MV  = true iff at every t in [0, T) no robot collides with an obstacle or
 *         itself (only with MRV_CHECK_ENV) and no two robots collide (§III-A).
 *   FFC = the lexicographically smallest (t, i, j), i < j, such that robots i
 *         and j collide at t; (-1, -1, -1) when there is none (§III-B).
 *
 * A pair of spheres collides iff its signed clearance is < 0 (touching is
 * free).  Arithmetic is FP32 with an FP64 re-evaluation of every test whose FP32
 * clearance lies within a near band of zero, so the booleans and (t, i, j)
 * equal those of an FP64 evaluation.  FP32 coordinates are formed relative to
 * the team's origin (the centre of its bases' bounding box) and the
 * environment's (the centre of its obstacles' bounding box), each subtracted in
 * FP64, so where the cell sits in the world costs no precision.  The band is
 * `near_eps` for a query whose relative coordinates stay within 4 m (every
 * frame and sphere of the team, prismatic joint values included, and every
 * obstacle part); beyond that it widens in proportion to the largest such
 * magnitude, as FP32 rounding does.
 *
 * Conventions for every entry point:
 *  - Return value: MRV_OK (0) or a negative mrv_status.  On error nothing is
 *    written to any output and mrv_last_error() describes the failure.  No
 *    C++ exception crosses this boundary.
 *  - Ownership: the caller owns every array it passes.  Host arrays are read
 *    (and copied where needed) before the call returns.  Device arrays passed to
 *    the *_device entry points must stay valid until the work on the context
 *    stream has completed (mrv_sync).
 *  - Threading: mrv_submit, mrv_poll, mrv_wait and mrv_cancel may be called from
 *    any thread.  Every other call on one context must come from one thread at a
 *    time.
 *  - Layouts: all transforms are 3x4 row-major [R | p] (12 doubles).  All
 *    arrays are dense and C-ordered.
 */
#ifndef MRV_H
#define MRV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mrv_status;
enum {
    MRV_OK = 0,
    MRV_PENDING = 1,         /* mrv_poll: the request has not finished yet */
    MRV_E_INVALID = -1,      /* malformed argument or input data */
    MRV_E_NOMEM = -2,        /* device or host allocation failed */
    MRV_E_DEVICE = -3,       /* a HIP runtime call failed */
    MRV_E_BUSY = -4,         /* request queue full, or handle still in use */
    MRV_E_HANDLE = -5,       /* unknown context, team, environment or ticket */
    MRV_E_CANCELLED = -6,    /* the request was cancelled */
    MRV_E_TIMEOUT = -7       /* mrv_wait ran out of time */
};

/* Limits enforced by validation. */
#define MRV_MAX_ROBOTS 32
#define MRV_MAX_JOINTS 8
#define MRV_MAX_SPHERES_PER_ROBOT 256
#define MRV_MAX_TEAM_SPHERES 2048
#define MRV_MAX_T (1 << 20)
/* Every floating-point input (team geometry, obstacles, points, waypoint
 * configurations) must be finite with magnitude <= MRV_MAX_COORD (metres or
 * radians); the kernels' FP32 arithmetic then cannot overflow. */
#define MRV_MAX_COORD 1.0e6

typedef struct mrv_ctx_s* mrv_ctx;

typedef struct {
    int32_t device;        /* HIP device ordinal */
    void* stream;          /* hipStream_t to order all work on; NULL = the library creates one */
    void* device_arena;    /* caller-owned device memory of `device` (e.g. a torch uint8 tensor) from
                            * which every device buffer of the context is sub-allocated: resident teams
                            * and environments, per-call scratch, the near-contact queue, captured
                            * graphs and the serving loop's batches.  The library then never calls
                            * hipMalloc; a call whose memory does not fit fails with MRV_E_NOMEM and
                            * leaves its outputs untouched, and served requests wait until running
                            * batches give memory back.  The arena must outlive the context.  NULL:
                            * the library allocates with hipMalloc as needed. */
    size_t arena_bytes;    /* size of device_arena (0 iff device_arena is NULL) */
    double near_eps;       /* near-contact band in metres (widened per query for large relative
                            * coordinates, see above); <= 0 selects 1e-5; must be < 0.01 */
    int32_t max_inflight;  /* serving: queue capacity in requests; <= 0 selects 1024 */
    size_t serve_bytes;    /* serving: the most device bytes the batches in flight may hold at once
                            * (inputs, outputs and scratch as allocated); 0 = no limit besides the
                            * arena (with an arena) or 1 GiB (without one) */
    int64_t recheck_records; /* initial length of the near-contact re-evaluation queue in
                              * 16-byte records; <= 0 selects 2^21.  Calls that overflow it
                              * enlarge it, up to 2^27 (see mrv_mv, mrv_sync). */
    uint32_t flags;        /* reserved, must be 0 */
} mrv_ctx_opts;

/* Create a context on opts->device.  *out receives the handle. */
mrv_status mrv_create(const mrv_ctx_opts* opts, mrv_ctx* out);
/* Release the context, its resident teams and environments, and its device memory.
 * Pending requests are cancelled.  NULL is accepted. */
mrv_status mrv_destroy(mrv_ctx ctx);
/* Message for the last failing call on this thread ("" if none).  Valid until the
 * next call on this thread. */
const char* mrv_last_error(void);

/* Device memory of the context in bytes: now allocated, the most ever allocated
 * at once, and the arena's usable size (0 without an arena).  Any pointer may be
 * NULL. */
mrv_status mrv_memory_stats(mrv_ctx ctx, size_t* used, size_t* peak, size_t* capacity);

/* ---------------------------------------------------------------- robots */
enum { MRV_REV_Z = 0, MRV_PRI_X = 1, MRV_PRI_Y = 2, MRV_PRI_Z = 3 };

/* One robot: a serial chain and the spheres on its frames (paper §II-B).
 * Frame_0 = base, Frame_k = Frame_{k-1} F_k J_k(q_k), J a rotation about local z
 * (MRV_REV_Z) or a translation along local x/y/z (MRV_PRI_*).  Sphere s sits at
 * Frame_{sphere_frame[s]} c_s. */
typedef struct {
    int32_t n_joints;               /* 0..MRV_MAX_JOINTS; also the robot's dof */
    const int32_t* joint_type;      /* [n_joints] */
    const double* joint_fixed;      /* [n_joints][12] F_k */
    int32_t n_spheres;              /* 1..MRV_MAX_SPHERES_PER_ROBOT */
    const int32_t* sphere_frame;    /* [n_spheres] in 0..n_joints */
    const double* sphere_xyzr;      /* [n_spheres][4] local centre and radius (> 0) */
    int32_t n_self_pairs;           /* >= 0 */
    const int32_t* self_pairs;      /* [n_self_pairs][2] sphere indices a != b: self-collision pairs */
    double base[12];                /* world-from-base transform */
} mrv_robot_desc;

/* Upload a team (host arrays, copied) and keep it resident.  Robot order
 * defines the robot indices reported by FFC.  *team_out receives the handle. */
mrv_status mrv_load_team(mrv_ctx ctx, const mrv_robot_desc* robots, int32_t n_robots,
                         int32_t* team_out);

/* ---------------------------------------------------------- environments */
/* Obstacles in the world frame.  The paper keeps a copy per robot base frame
 * (§III-A, Alg. 1 input); here one world-frame copy serves every robot, because
 * the robot-robot tests need world-frame sphere centres anyway. */
typedef struct {
    int32_t n_spheres; const double* spheres;      /* [n][4] centre, radius */
    int32_t n_boxes;   const double* boxes;        /* [n][15] centre, R (row-major 3x3), half-extents */
    int32_t n_cyls;    const double* cylinders;    /* [n][8] centre, unit axis, half-length, radius */
    int64_t n_points;  const double* points;       /* [n][3] point obstacles of radius point_radius */
    double point_radius;                           /* >= 0 */
    double grid_cell;                              /* point-grid cell size in metres; <= 0 selects 0.05 */
} mrv_env_desc;

/* Upload an environment (host arrays, copied).  *env_out receives the handle. */
mrv_status mrv_load_env(mrv_ctx ctx, const mrv_env_desc* env, int32_t* env_out);

/* Drop a team or environment handle.  MRV_E_BUSY while a served request or a
 * captured graph (mrv_graph_create) uses it. */
mrv_status mrv_unload(mrv_ctx ctx, int32_t handle);

/* ----------------------------------------------------------------- paths */
/* Query-major CSR over per-robot timed waypoint lists.  Path (q, r) is
 * waypoints [wp_begin[q*n_robots + r], wp_begin[q*n_robots + r + 1]).  Its first
 * time is 0, times strictly increase, the last time is < MRV_MAX_T, and the
 * configuration values are finite and within MRV_MAX_COORD.  wp_q rows hold dof_stride doubles (the team's
 * largest dof; a robot reads its first n_joints values). */
typedef struct {
    int32_t n_queries;
    int32_t dof_stride;
    const int64_t* wp_begin;   /* [n_queries * n_robots + 1], wp_begin[0] = 0 */
    const int32_t* wp_t;       /* [n_wp] */
    const double* wp_q;        /* [n_wp][dof_stride] */
    int64_t n_wp;              /* number of waypoints = wp_begin[last] */
} mrv_paths;

typedef struct { int32_t t, ri, rj; } mrv_conflict;   /* (-1, -1, -1): no conflict */

/* Per-call flags. */
enum {
    MRV_CHECK_ENV = 1,       /* MV: check robot-obstacle and self collision too */
    MRV_EXHAUSTIVE = 2,      /* evaluate every test (no early termination); same answers */
    MRV_HIERARCHICAL = 4,    /* MV: all environment tiles before robot-robot tiles (Alg. 1) */
    MRV_ORDER_BISECT = 0,    /* MV tile order: rake tiles in golden-ratio interleave (default) */
    MRV_ORDER_RAKE = 8,      /* MV tile order: the paper's rake, batches in index order */
    MRV_ORDER_LINEAR = 16,   /* MV tile order: consecutive timesteps (FFC always uses this) */
    MRV_PAIRS_FIRST = 32,    /* early-terminating MV: within a tile, robot-robot (and self) tests
                                before robot-obstacle tests */
    MRV_OBSTACLES_FIRST = 64, /* early-terminating MV: robot-obstacle tests first.  With neither
                                flag, pairs go first when the environment has a point cloud (its
                                tests cost most) and obstacles first otherwise.  The order
                                changes only how soon a collision ends a query, never the answer;
                                exhaustive calls always test obstacles first. */
    MRV_PAIR_PRIORITY = 128  /* early-terminating MV without a focus set: within a tile, first the
                                self tests and the robot pairs likeliest to collide -- bases
                                adjacent, within 1.25 times the team's smallest base distance
                                (paper §III-A) -- then, only if none collides, the other pairs.
                                Other calls ignore it; it never changes an answer. */
};

/* Near contact.  A test whose FP32 clearance lies within near_eps of zero is
 * queued and re-evaluated in FP64.  A queued test whose outcome can no longer
 * change the answer (MV: the query already collides; FFC: a conflict at an
 * earlier or equal (t, i, j) is known) is dropped.  When the queue overflows,
 * queries whose answer might still depend on a dropped test are unresolved:
 * the synchronous calls enlarge the queue and run again; device calls report
 * them as valid_out = 3 / t = -3 and through mrv_sync. */

/* MV over host arrays; synchronous.  valid_out[q] = 1 valid, 0 invalid.
 * env = -1 runs without obstacles (self checks still run with MRV_CHECK_ENV). */
mrv_status mrv_mv(mrv_ctx ctx, int32_t team, int32_t env, const mrv_paths* paths, uint32_t flags,
                  uint8_t* valid_out);
/* FFC over host arrays; synchronous.  out[q] = earliest conflict of query q. */
mrv_status mrv_ffc(mrv_ctx ctx, int32_t team, const mrv_paths* paths, uint32_t flags,
                   mrv_conflict* out);

/* Device-resident variants: every pointer in *paths and the output point to
 * device memory of the context's device.  Work is queued on the context stream
 * and the call returns without waiting.  Inputs are checked on the device; a
 * query whose path data break the rules above gets valid_out = 2 (MV) or
 * t = -2 (FFC), and the next mrv_sync returns MRV_E_INVALID.  The context
 * keeps per-call scratch, so results are complete only after mrv_sync or an
 * equivalent stream synchronisation. */
mrv_status mrv_mv_device(mrv_ctx ctx, int32_t team, int32_t env, const mrv_paths* paths,
                         uint32_t flags, uint8_t* valid_out);
mrv_status mrv_ffc_device(mrv_ctx ctx, int32_t team, const mrv_paths* paths, uint32_t flags,
                          mrv_conflict* out);

/* Allocation-free MV, for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  As
 * mrv_mv_device (same arguments, answers and asynchrony), but the call's scratch
 * (control words, tile enumeration, per-query state, near-contact queue) lives
 * in one fixed array of about 29 MiB (at most 30 MiB) that the library holds on
 * every device it runs on until the process ends, and the call neither allocates
 * nor frees device memory.  Limits: n_queries <= MRV_NOALLOC_MAX_QUERIES
 * (larger calls fail with MRV_E_INVALID and leave valid_out untouched); the
 * near-contact queue holds MRV_NOALLOC_RECHECK_RECORDS tests, and a query whose
 * answer depends on a test that did not fit gets valid_out = 3 (repeat it with
 * mrv_mv_device).  A query with malformed path data gets valid_out = 2.  Neither
 * is reported by mrv_sync, and mrv_last_stats does not describe these calls.
 * Every call on a device shares that device's array and leaves its contents
 * behind (each call clears what must start at zero): calls that overlap on one
 * device, from any context or thread, race and give undefined results, so
 * order them on one stream or synchronise between them. */
#define MRV_NOALLOC_MAX_QUERIES (1 << 18)
#define MRV_NOALLOC_RECHECK_RECORDS (1 << 18)
mrv_status mrv_mv_device_noalloc(mrv_ctx ctx, int32_t team, int32_t env, const mrv_paths* paths,
                                 uint32_t flags, uint8_t* valid_out);

/* Prioritised MV (the PP-ST-RRT use of MV in §III-C: a robot is planned against
 * the fixed paths of higher-priority robots).  As mrv_mv / mrv_mv_device, but
 * only the robots in `focus` (bit r = robot r of the team) are validated: their
 * obstacle and self tests (with MRV_CHECK_ENV) and every robot pair with at
 * least one robot in focus.  Pairs of robots outside focus are not tested, so
 * collisions among the fixed paths do not invalidate the motion.  focus = 0, or
 * every robot of the team, is plain MV; bits at or above the team's robot count
 * are ignored. */
mrv_status mrv_mv_focus(mrv_ctx ctx, int32_t team, int32_t env, const mrv_paths* paths, uint32_t flags,
                        uint32_t focus, uint8_t* valid_out);
mrv_status mrv_mv_focus_device(mrv_ctx ctx, int32_t team, int32_t env, const mrv_paths* paths,
                               uint32_t flags, uint32_t focus, uint8_t* valid_out);

/* Wait for the context stream; report device-side input errors since the last
 * sync (MRV_E_INVALID), then unresolved queries (MRV_E_NOMEM; the queue is then
 * enlarged to what the largest of those calls needed, so repeating them
 * succeeds). */
mrv_status mrv_sync(mrv_ctx ctx);

/* FP32 world-frame sphere centres of the team at n_states (query, timestep)
 * pairs of host paths, as the validation kernels compute them (paper §III-A,
 * SpheresFK), i.e. relative to the team origin, plus the origin added in FP32:
 * out[k][s] = (x, y, z, radius) for sphere s of the flattened team
 * (robots in order), k < n_states; out holds n_states * S * 4 floats, S = the
 * team's total sphere count.  state_query[k] must index a query of paths and
 * state_t[k] >= 0 (timesteps past a path's end give its last configuration). */
mrv_status mrv_spheres(mrv_ctx ctx, int32_t team, const mrv_paths* paths, int32_t n_states,
                       const int32_t* state_query, const int32_t* state_t, float* out);

/* Timesteps for a straight-line motion dq: ceil(|dq| / step) with the L2
 * (metric 0) or L-infinity (metric 1) norm (paper §IV-A: bounded C-space motion
 * per timestep).  Returns -1 on invalid arguments. */
int64_t mrv_motion_steps(const double* dq, int32_t dof, double step, int32_t metric);

/* ------------------------------------------------------------- tuning/stats */
typedef struct {
    int32_t chunk;           /* timesteps per tile; 0 = automatic */
    int32_t wg_per_cu;       /* persistent workgroups per compute unit; 0 = occupancy limit */
    int32_t interleave;      /* MV tile order of the calls that ask for MRV_ORDER_BISECT (the default):
                              * 0 or 1 = golden-ratio bisection, 2 = rake (as MRV_ORDER_RAKE),
                              * 3 = consecutive timesteps (as MRV_ORDER_LINEAR); FFC ignores it */
    int32_t claim;           /* tiles a workgroup takes per claim on the launch's tile counter:
                              * 0 = automatic (at most 4 for exhaustive calls and 8 otherwise, fewer
                              * when a call has under 8 claims' worth of tiles per workgroup),
                              * else 1..16 */
} mrv_tiling;
/* Set the tiling used for (team, kind), kind 0 = MV, 1 = FFC, by the calls whose
 * MRV_EXHAUSTIVE flag equals that of flags (other flag bits are ignored): calls
 * that run every test favour tiles sized for occupancy, early-terminating calls
 * longer tiles with less fixed cost per tile, so each mode keeps its own.
 * Waits for the work queued on the context stream.  MRV_E_BUSY while a served
 * request or a captured graph uses the team. */
mrv_status mrv_set_tiling(mrv_ctx ctx, int32_t team, int32_t kind, uint32_t flags, const mrv_tiling* tiling);
mrv_status mrv_get_tiling(mrv_ctx ctx, int32_t team, int32_t kind, uint32_t flags, mrv_tiling* tiling);

/* Search the tiling for (team, env, kind, flags) by timing the validation kernel on
 * the given host paths (a representative sample of the workload), one field at a
 * time from the team's current tiling: every chunk size that fits in LDS, then
 * workgroups per compute unit, then tiles per claim, then (early-terminating MV)
 * the interleave, each trial the best of two timed runs after a warm-up.  The
 * search stops after MRV_TUNE_BUDGET_MS of trial time and keeps the best tiling
 * found so far; the fastest is set for the team (as mrv_set_tiling with the same
 * flags would) and returned in *best.  Early-terminating calls skip tiles on
 * outcomes other queries' tiles found, so their sample should come near the batch
 * size the tiling is for (FFC of the 16-robot cloud team: tuned on 1,024 path sets
 * the choice lost on 131,072; on 8,192 the default was kept).
 * Results are cached per context by the team's shape (spheres, frames, groups,
 * robots), the environment's obstacle counts and the flags: a later call with
 * an equal key returns the cached tiling without timing.  The answers of MV/FFC
 * never depend on the tiling.  Trials run on a private copy of the team's
 * descriptor; MRV_E_BUSY while a served request or a captured graph uses the
 * team. */
#define MRV_TUNE_BUDGET_MS 8000
mrv_status mrv_autotune(mrv_ctx ctx, int32_t team, int32_t env, int32_t kind, const mrv_paths* sample,
                        uint32_t flags, mrv_tiling* best);

/* Captured call graphs.  mrv_graph_create records the complete pipeline of one
 * device-array call (the same arguments as mrv_mv_device / mrv_ffc_device, kind
 * 0 = MV, 1 = FFC) into a HIP graph with its own scratch; mrv_graph_launch
 * replays it on the context stream with one launch.  The graph reads the path
 * arrays and writes the output at replay time, so the caller may refill the same
 * buffers (same n_queries, no more than n_wp waypoints) between replays.
 * The graph's near-contact queue keeps its size (the context's at creation):
 * a replay that overflows it leaves valid_out = 3 / t = -3 for the queries
 * concerned and reports nothing else.
 * Replays of one graph must not overlap each other.  Destroy graphs before their
 * context; a graph keeps its team and environment loaded until it is destroyed. */
typedef struct mrv_graph_s* mrv_graph;
mrv_status mrv_graph_create(mrv_ctx ctx, int32_t team, int32_t env, int32_t kind, const mrv_paths* paths,
                            uint32_t flags, void* out, mrv_graph* graph);
mrv_status mrv_graph_launch(mrv_ctx ctx, mrv_graph graph);
mrv_status mrv_graph_destroy(mrv_ctx ctx, mrv_graph graph);

typedef struct {
    uint64_t tiles_run, tiles_skipped;
    uint64_t states_evaluated;   /* robot-states run through FK and tests */
    uint64_t states_covered;     /* sum over queries of n_robots * T */
    uint64_t rr_tests, env_tests, self_tests;   /* sphere tests executed: robot-robot, robot-obstacle
                                                   (sphere, box and cylinder obstacles; those skipped by
                                                   the bounding-box cull are not counted), self */
    uint64_t near_rechecks;      /* tests re-evaluated in FP64 */
    double kernel_ms;            /* validation kernel time of the last call (device events) */
    uint64_t point_tests;        /* sphere-point pairs tested (point clouds: each 16-sphere group's spheres
                                    against the points its blocks take, 16 at a time, from the grid cell
                                    rows its spheres reach) */
} mrv_stats;
/* Counters of the last MV/FFC call on this context (synchronises the stream). */
mrv_status mrv_last_stats(mrv_ctx ctx, mrv_stats* out);

/* --------------------------------------------------------------- serving */
typedef struct {
    int32_t kind;            /* 0 = MV, 1 = FFC */
    int32_t team, env;       /* env = -1: none */
    uint32_t flags;
    mrv_paths paths;         /* host arrays, copied by mrv_submit */
    uint32_t focus;          /* MV: robots validated as in mrv_mv_focus; 0 = all (FFC: ignored) */
} mrv_request;

/* Queue a request for the serving loop; returns once its inputs are copied.
 * MRV_E_BUSY when max_inflight requests are queued or running. */
mrv_status mrv_submit(mrv_ctx ctx, const mrv_request* req, uint64_t* ticket);
/* MRV_OK and the result in out (uint8[n_queries] for MV, mrv_conflict[n_queries]
 * for FFC; the ticket is then released), MRV_PENDING, or an error. */
mrv_status mrv_poll(mrv_ctx ctx, uint64_t ticket, void* out);
/* Like mrv_poll but waits up to timeout_ms (< 0: forever). */
mrv_status mrv_wait(mrv_ctx ctx, uint64_t ticket, int32_t timeout_ms, void* out);
/* Cancel a queued or running request; its ticket then reports MRV_E_CANCELLED once. */
mrv_status mrv_cancel(mrv_ctx ctx, uint64_t ticket);

#ifdef __cplusplus
}
#endif

#endif /* MRV_H */
