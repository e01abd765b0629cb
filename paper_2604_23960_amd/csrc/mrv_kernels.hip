// Device kernels of libmrv for gfx950 (MI355X).
//
// One MV/FFC call runs five kernels on one stream:
//   k_reset        clears the call's control words and counters,
//   k_query_info   per query: checks the path data, T = max_i L_i, tile count,
//                  interleave step; histogram of tile counts,
//   k_scan         one workgroup: orders queries by tile count (descending) and
//                  builds the rank-major tile offsets,
//   k_assign       per query: its slot in that order,
//   k_validate     persistent workgroups draining (query, tile) work in rank-major
//                  order: every query's first tile, then every query's second, ...
//                  so MV early exit (paper §III-A) and FFC pruning (§III-B) see
//                  the results of earlier tiles before later tiles start,
//   k_finalize     per query: writes the answer.
//
// A tile is C timesteps of one query.  Its workgroup interpolates each robot's
// configuration (FP64, rounded to FP32), runs the robot's chain in FP32 registers
// (paper §II-B: FK of the sphere model), stages every sphere of every robot at
// every timestep of the tile in LDS, then runs the robot-obstacle/self tests
// (MV with environment checking) and the robot-robot tests with one lane per
// sphere of a timestep.  Tests whose FP32 clearance lies within eps of zero are
// queued and re-evaluated in FP64 from the FP64 waypoints and model.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "../../include/mrv.h"
#include "mrv_internal.hpp"

namespace mrv {

namespace {

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ unsigned wave_min_u32(unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned w = (unsigned)__shfl_xor((int)v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ unsigned pair_index(int i, int j, int n)
{
    return (unsigned)(i * (2 * n - i - 1) / 2 + (j - i - 1));
}

__device__ __forceinline__ unsigned load_word(const unsigned* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Locate the waypoint segment of path [b, e) for timestep t: returns k with
// wp_t[k] <= t < wp_t[k+1], or e-1 when t is at or past the last waypoint.
__device__ __forceinline__ long long find_segment(const int* wt, long long b, long long e, int t)
{
    if (t >= wt[e - 1]) return e - 1;
    long long lo = b, hi = e - 1;   // wt[lo] <= t < wt[hi]
    while (hi - lo > 1) {
        long long mid = (lo + hi) >> 1;
        if (wt[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// FP64 re-evaluation of a near-contact test.  The configuration is the
// interpolation q = Q_k + s (Q_{k+1} - Q_k), s = (t - tau_k) / (tau_{k+1} - tau_k),
// as one multiply then one add; frames are composed as (Frame F_k) J_k(q_k); no
// operation is fused.

__device__ void fk64_sphere(const TeamDev& tm, const CallDev& cd, int q, int t, int s, double* out)
{
#pragma clang fp contract(off)
    const int r = tm.s_robot[s];
    const int f = tm.s_lframe[s];
    const long long pb = cd.wp_begin[(long long)q * cd.n_robots + r];
    const long long pe = cd.wp_begin[(long long)q * cd.n_robots + r + 1];
    const long long k = find_segment(cd.wp_t, pb, pe, t);
    const bool last = (k == pe - 1);
    double sfrac = 0.0;
    if (!last) sfrac = (double)(t - cd.wp_t[k]) / (double)(cd.wp_t[k + 1] - cd.wp_t[k]);
    double M[12];
    for (int i = 0; i < 12; ++i) M[i] = tm.r_base64[r * 12 + i];
    const int j0 = tm.r_joint_off[r];
    for (int j = 0; j < f; ++j) {
        double qa = cd.wp_q[k * cd.dof_stride + j];
        double qj = qa;
        if (!last) {
            double qb = cd.wp_q[(k + 1) * cd.dof_stride + j];
            double step = sfrac * (qb - qa);
            qj = qa + step;
        }
        const double* F = tm.j_fixed64 + (long long)(j0 + j) * 12;
        double A[12];
        for (int row = 0; row < 3; ++row) {
            for (int col = 0; col < 3; ++col) {
                double v = M[row * 4 + 0] * F[0 * 4 + col];
                v = v + M[row * 4 + 1] * F[1 * 4 + col];
                v = v + M[row * 4 + 2] * F[2 * 4 + col];
                A[row * 4 + col] = v;
            }
            double p = M[row * 4 + 0] * F[3];
            p = p + M[row * 4 + 1] * F[7];
            p = p + M[row * 4 + 2] * F[11];
            A[row * 4 + 3] = p + M[row * 4 + 3];
        }
        const int jt = tm.j_type[j0 + j];
        if (jt == MRV_REV_Z) {
            double c = cos(qj), sn = sin(qj);
            for (int row = 0; row < 3; ++row) {
                double a0 = A[row * 4 + 0], a1 = A[row * 4 + 1];
                double n0 = a0 * c + a1 * sn;
                double n1 = a0 * (-sn) + a1 * c;
                M[row * 4 + 0] = n0;
                M[row * 4 + 1] = n1;
                M[row * 4 + 2] = A[row * 4 + 2];
                M[row * 4 + 3] = A[row * 4 + 3];
            }
        } else {
            const int ax = jt - 1;   // PRI_X/Y/Z translate along column ax
            for (int row = 0; row < 3; ++row) {
                M[row * 4 + 0] = A[row * 4 + 0];
                M[row * 4 + 1] = A[row * 4 + 1];
                M[row * 4 + 2] = A[row * 4 + 2];
                M[row * 4 + 3] = A[row * 4 + ax] * qj + A[row * 4 + 3];
            }
        }
    }
    const double* c = tm.s_local64 + (long long)s * 4;
    for (int row = 0; row < 3; ++row) {
        double v = M[row * 4 + 0] * c[0];
        v = v + M[row * 4 + 1] * c[1];
        v = v + M[row * 4 + 2] * c[2];
        out[row] = v + M[row * 4 + 3];
    }
}

__device__ double clear_ss64(const double* x, double r, const double* y, double s)
{
#pragma clang fp contract(off)
    double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    return sqrt(dx * dx + dy * dy + dz * dz) - (r + s);
}

__device__ double clear_box64(const double* x, double r, const double* box)
{
#pragma clang fp contract(off)
    const double* c = box;
    const double* R = box + 3;
    const double* h = box + 12;
    double v0 = x[0] - c[0], v1 = x[1] - c[1], v2 = x[2] - c[2];
    double p[3], e[3];
    bool inside = true;
    for (int k = 0; k < 3; ++k) {
        p[k] = R[0 * 3 + k] * v0 + R[1 * 3 + k] * v1 + R[2 * 3 + k] * v2;
        double ek = fabs(p[k]) - h[k];
        e[k] = ek > 0.0 ? ek : 0.0;
        if (e[k] > 0.0) inside = false;
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

__device__ double clear_cyl64(const double* x, double r, const double* cyl)
{
#pragma clang fp contract(off)
    const double* c = cyl;
    const double* u = cyl + 3;
    double hl = cyl[6], R = cyl[7];
    double v0 = x[0] - c[0], v1 = x[1] - c[1], v2 = x[2] - c[2];
    double h = v0 * u[0] + v1 * u[1] + v2 * u[2];
    double w0 = v0 - h * u[0], w1 = v1 - h * u[1], w2 = v2 - h * u[2];
    double s = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    double er = s - R > 0.0 ? s - R : 0.0;
    double ea = fabs(h) - hl > 0.0 ? fabs(h) - hl : 0.0;
    if (er == 0.0 && ea == 0.0) {
        double m1 = R - s, m2 = hl - fabs(h);
        return -(m1 < m2 ? m1 : m2) - r;
    }
    return sqrt(er * er + ea * ea) - r;
}

// True iff the FP64 evaluation of the queued test collides.
__device__ bool recheck64(const TeamDev& tm, const EnvDev& env, const CallDev& cd, int q, int t,
                          int kind, int a, int b)
{
    double pa[3];
    fk64_sphere(tm, cd, q, t, a, pa);
    const double ra = tm.s_local64[(long long)a * 4 + 3];
    switch (kind) {
    case RK_RR:
    case RK_SELF: {
        double pb[3];
        fk64_sphere(tm, cd, q, t, b, pb);
        return clear_ss64(pa, ra, pb, tm.s_local64[(long long)b * 4 + 3]) < 0.0;
    }
    case RK_ENV_SPH:
        return clear_ss64(pa, ra, env.sph64 + (long long)b * 4, env.sph64[(long long)b * 4 + 3]) < 0.0;
    case RK_ENV_BOX:
        return clear_box64(pa, ra, env.box64 + (long long)b * 15) < 0.0;
    case RK_ENV_CYL:
        return clear_cyl64(pa, ra, env.cyl64 + (long long)b * 8) < 0.0;
    case RK_ENV_PT:
        return clear_ss64(pa, ra, env.pts64 + (long long)b * 3, env.pt_radius64) < 0.0;
    default:
        return false;
    }
}

// ---------------------------------------------------------------------------
// call preparation

__device__ int golden_step(int nt)
{
    if (nt <= 2) return 1;
    int g = (int)(nt * 0.6180339887498949);
    if (g < 1) g = 1;
    for (;; ++g) {
        int a = g, b = nt;
        while (b) { int r = a % b; a = b; b = r; }
        if (a == 1) return g;
    }
}

__global__ void k_reset(CallDev cd)
{
    int i = threadIdx.x;
    if (i < 4) cd.ctrl[i] = (i == 3) ? cd.ctrl[3] : 0;
    if (i < ST_COUNT) cd.stats[i] = 0ull;
    if (i == 0) {
        // tile counter and total live in 64-bit words after ctrl[0..3]
        unsigned long long* w = reinterpret_cast<unsigned long long*>(cd.ctrl + 4);
        w[0] = 0ull;   // total tiles
        w[1] = 0ull;   // next tile
    }
}

__global__ void k_query_info(TeamDev tm, CallDev cd)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cd.n_queries) return;
    const int n = cd.n_robots;
    int T = 0;
    bool ok = true;
    for (int r = 0; r < n && ok; ++r) {
        const long long b = cd.wp_begin[(long long)q * n + r];
        const long long e = cd.wp_begin[(long long)q * n + r + 1];
        if (b < 0 || e <= b || e > cd.n_wp) { ok = false; break; }
        int prev = cd.wp_t[b];
        if (prev != 0) { ok = false; break; }
        const int dof = tm.r_nj[r];
        for (long long i = b; i < e && ok; ++i) {
            const int ti = cd.wp_t[i];
            if (i > b && ti <= prev) ok = false;
            prev = ti;
            for (int d = 0; d < dof; ++d)
                if (!isfinite(cd.wp_q[i * cd.dof_stride + d])) ok = false;
        }
        if (prev >= MRV_MAX_T) ok = false;
        if (prev + 1 > T) T = prev + 1;
    }
    int nt = 0, g = 1;
    if (ok) {
        nt = (T + cd.chunk - 1) / cd.chunk;
        g = golden_step(nt);
    }
    cd.T[q] = ok ? T : 0;
    cd.nt[q] = nt;
    cd.gstep[q] = g;
    cd.status[q] = ok ? 0 : 1;
    cd.word[q] = cd.kind == 1 ? 0xFFFFFFFFu : 0u;
    if (!ok) {
        atomicAdd(&cd.ctrl[3], 1);
    } else {
        atomicAdd(&cd.hist[nt], 1);
        atomicMax(&cd.ctrl[0], nt);
        atomicAdd(&cd.stats[ST_STATES_COVERED], (unsigned long long)n * (unsigned long long)T);
    }
}

// One workgroup.  start[n] = number of queries with more than n tiles (the first
// slot of tile-count bin n in descending order), off[k] = number of tiles of
// rank < k (rank k holds the k-th tile of every query with more than k tiles).
__global__ __launch_bounds__(256) void k_scan(CallDev cd)
{
    __shared__ long long sbuf[256];
    __shared__ long long carry;
    const int tid = threadIdx.x;
    const int M = cd.ctrl[0];
    if (tid == 0) carry = 0;
    __syncthreads();
    // reverse exclusive scan of hist over n = M..0
    for (int base = 0; base <= M; base += 256) {
        const int idx = M - (base + tid);
        long long v = (idx >= 0) ? cd.hist[idx] : 0;
        sbuf[tid] = v;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            long long add = tid >= o ? sbuf[tid - o] : 0;
            __syncthreads();
            sbuf[tid] += add;
            __syncthreads();
        }
        if (idx >= 0) {
            cd.start[idx] = (int)(carry + sbuf[tid] - v);
            cd.hist[idx] = 0;
        }
        __syncthreads();
        if (tid == 255) carry += sbuf[255];
        __syncthreads();
    }
    if (tid == 0) carry = 0;
    __syncthreads();
    long long* off = reinterpret_cast<long long*>(cd.off);
    // forward exclusive scan of start[0..M] into off[0..M]
    for (int base = 0; base <= M; base += 256) {
        const int idx = base + tid;
        long long v = (idx <= M) ? cd.start[idx] : 0;
        sbuf[tid] = v;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            long long add = tid >= o ? sbuf[tid - o] : 0;
            __syncthreads();
            sbuf[tid] += add;
            __syncthreads();
        }
        if (idx <= M) off[idx] = carry + sbuf[tid] - v;
        __syncthreads();
        if (tid == 255) carry += sbuf[255];
        __syncthreads();
    }
    if (tid == 0) {
        unsigned long long* w = reinterpret_cast<unsigned long long*>(cd.ctrl + 4);
        w[0] = (unsigned long long)off[M];
    }
}

__global__ void k_assign(CallDev cd)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cd.n_queries) return;
    const int nt = cd.nt[q];
    if (nt > 0) {
        const int p = atomicAdd(&cd.start[nt], 1);
        cd.sorted_q[p] = q;
    }
}

__global__ void k_finalize(TeamDev tm, CallDev cd)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cd.n_queries) return;
    const bool bad = cd.status[q] != 0;
    const unsigned w = cd.word[q];
    if (cd.kind == 0) {
        cd.valid_out[q] = bad ? 2 : (w == 0u ? 1 : 0);
        return;
    }
    int t = -1, ri = -1, rj = -1;
    if (bad) {
        t = ri = rj = -2;
    } else if (w != 0xFFFFFFFFu) {
        const int n = tm.n_robots;
        const unsigned P = (unsigned)tm.P;
        t = (int)(w / P);
        int p = (int)(w % P);
        int i = 0;
        while (p >= n - 1 - i) { p -= n - 1 - i; ++i; }
        ri = i;
        rj = i + 1 + p;
    }
    cd.conflict_out[3 * q + 0] = t;
    cd.conflict_out[3 * q + 1] = ri;
    cd.conflict_out[3 * q + 2] = rj;
}

__global__ void k_fill_u32(unsigned* p, unsigned v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// validation

struct Tile {
    int q, k, phase, nv;
};

__device__ __forceinline__ void push_recheck(int4* rq, int* rqn, int kind, int c, int a, int b,
                                             bool& overflow)
{
    const int i = atomicAdd(rqn, 1);
    if (i < kRecheckCap) rq[i] = make_int4(kind | (c << 8), a, b, 0);
    else overflow = true;
}

template <int KIND>
__global__ __launch_bounds__(kWG) void k_validate(TeamDev tm, EnvDev env, CallDev cd)
{
    extern __shared__ float4 dyn[];
    const int C = cd.chunk;
    const int S = tm.S;
    const int F = tm.F;
    const int n = tm.n_robots;
    float4* sph = dyn;                 // [C][S] centre xyz, radius
    float4* fr = dyn + C * S;          // [C][F][3] frame rows (R row, p)

    __shared__ int s_t[kMaxChunk];
    __shared__ int s_q, s_k, s_nv, s_phase, s_hit, s_rqn;
    __shared__ unsigned s_key;
    __shared__ int4 s_rq[kRecheckCap];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_uniform(tid >> 6);
    const unsigned flags = cd.flags;
    const bool exhaustive = (flags & MRV_EXHAUSTIVE) != 0;
    const bool check_env = KIND == 0 && (flags & MRV_CHECK_ENV) != 0;
    const bool hier = check_env && (flags & MRV_HIERARCHICAL) != 0;
    const float eps = cd.eps32;

    unsigned long long* w64 = reinterpret_cast<unsigned long long*>(cd.ctrl + 4);
    const long long total = (long long)__hip_atomic_load(&w64[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long gtotal = hier ? 2 * total : total;
    const long long* off = reinterpret_cast<const long long*>(cd.off);
    const int M = cd.ctrl[0];

    long long k_cur = 0;
    int phase_cur = 0;
    unsigned long long n_rr = 0, n_env = 0, n_self = 0;
    unsigned long long n_run = 0, n_skip = 0, n_states = 0, n_re = 0;

    if (tid == 0) { s_rqn = 0; }

    for (;;) {
        if (tid == 0) {
            const long long g = (long long)atomicAdd(&w64[1], 1ull);
            int q = -1, k = 0, phase = 0, nv = 0;
            if (g < gtotal) {
                long long gg = g;
                if (hier) {
                    phase = g >= total ? 1 : 0;
                    gg = g - (long long)phase * total;
                    if (phase != phase_cur) { phase_cur = phase; k_cur = 0; }
                }
                // largest rank k with off[k] <= gg (ranks are non-empty below M; off[M] = total)
                long long lo = k_cur;
                if (off[lo + 1] <= gg) {
                    long long step = 1, hi;
                    lo = lo + 1;
                    for (;;) {
                        hi = lo + step;
                        if (hi >= M || off[hi] > gg) break;
                        lo = hi;
                        step <<= 1;
                    }
                    if (hi > M) hi = M;
                    while (hi - lo > 1) {
                        long long mid = (lo + hi) >> 1;
                        if (off[mid] <= gg) lo = mid; else hi = mid;
                    }
                }
                k_cur = lo;
                k = (int)lo;
                q = cd.sorted_q[gg - off[lo]];
                const int T = cd.T[q];
                const int nt = cd.nt[q];
                int base, stride;
                if (KIND == 1 || (flags & MRV_ORDER_LINEAR)) {
                    base = k * C; stride = 1;
                } else {
                    base = (flags & MRV_ORDER_RAKE) ? k : (int)(((long long)k * cd.gstep[q]) % nt);
                    stride = nt;
                }
                for (int c = 0; c < C; ++c) {
                    const long long t = (long long)base + (long long)c * stride;
                    if (t < T) { s_t[c] = (int)t; nv = c + 1; }
                }
                bool skip = false;
                if (!exhaustive) {
                    const unsigned w = load_word(cd.word + q);
                    if (KIND == 0) skip = (w != 0u);
                    else skip = (w != 0xFFFFFFFFu) && (w < (unsigned)base * (unsigned)tm.P);
                }
                if (skip) { nv = 0; ++n_skip; }
                else { ++n_run; n_states += (unsigned long long)nv * n; }
            } else {
                q = -1;
            }
            s_q = q; s_k = k; s_phase = phase; s_nv = nv;
            s_hit = 0; s_key = 0xFFFFFFFFu;
        }
        __syncthreads();
        const int q = s_q;
        if (q < 0) break;
        const int nv = s_nv;
        if (nv == 0) { __syncthreads(); continue; }
        const int phase = s_phase;
        const bool do_env = check_env && (!hier || phase == 0);
        const bool do_rr = !hier || phase == 1;

        // --- configurations and FP32 forward kinematics: one lane per (timestep, robot)
        for (int idx = tid; idx < nv * n; idx += kWG) {
            const int c = idx / n;
            const int r = idx - c * n;
            const int t = s_t[c];
            const long long pb = cd.wp_begin[(long long)q * n + r];
            const long long pe = cd.wp_begin[(long long)q * n + r + 1];
            const long long kseg = find_segment(cd.wp_t, pb, pe, t);
            const bool last = (kseg == pe - 1);
            double sfrac = 0.0;
            if (!last) sfrac = (double)(t - cd.wp_t[kseg]) / (double)(cd.wp_t[kseg + 1] - cd.wp_t[kseg]);
            const int nj = tm.r_nj[r];
            float qv[kMaxJoints];
#pragma unroll
            for (int j = 0; j < kMaxJoints; ++j) {
                qv[j] = 0.f;
                if (j < nj) {
                    double qa = cd.wp_q[kseg * cd.dof_stride + j];
                    double qj = qa;
                    if (!last) qj = qa + sfrac * (cd.wp_q[(kseg + 1) * cd.dof_stride + j] - qa);
                    qv[j] = (float)qj;
                }
            }
            float Mx[12];
#pragma unroll
            for (int i = 0; i < 12; ++i) Mx[i] = tm.r_base32[r * 12 + i];
            const int f0 = tm.r_frame_off[r];
            float4* out = fr + ((long long)c * F + f0) * 3;
            out[0] = make_float4(Mx[0], Mx[1], Mx[2], Mx[3]);
            out[1] = make_float4(Mx[4], Mx[5], Mx[6], Mx[7]);
            out[2] = make_float4(Mx[8], Mx[9], Mx[10], Mx[11]);
            const int j0 = tm.r_joint_off[r];
#pragma unroll
            for (int j = 0; j < kMaxJoints; ++j) {
                if (j < nj) {
                    const float* Fj = tm.j_fixed32 + (long long)(j0 + j) * 12;
                    float A[12];
#pragma unroll
                    for (int row = 0; row < 3; ++row) {
#pragma unroll
                        for (int col = 0; col < 4; ++col) {
                            float v = Mx[row * 4 + 0] * Fj[col] + Mx[row * 4 + 1] * Fj[4 + col] +
                                      Mx[row * 4 + 2] * Fj[8 + col];
                            A[row * 4 + col] = (col == 3) ? v + Mx[row * 4 + 3] : v;
                        }
                    }
                    const int jt = tm.j_type[j0 + j];
                    if (jt == MRV_REV_Z) {
                        float sn, cs;
                        sincosf(qv[j], &sn, &cs);
#pragma unroll
                        for (int row = 0; row < 3; ++row) {
                            const float a0 = A[row * 4 + 0], a1 = A[row * 4 + 1];
                            Mx[row * 4 + 0] = a0 * cs + a1 * sn;
                            Mx[row * 4 + 1] = a1 * cs - a0 * sn;
                            Mx[row * 4 + 2] = A[row * 4 + 2];
                            Mx[row * 4 + 3] = A[row * 4 + 3];
                        }
                    } else {
                        const int ax = jt - 1;
#pragma unroll
                        for (int row = 0; row < 3; ++row) {
                            const float axv = ax == 0 ? A[row * 4 + 0] : (ax == 1 ? A[row * 4 + 1] : A[row * 4 + 2]);
                            Mx[row * 4 + 0] = A[row * 4 + 0];
                            Mx[row * 4 + 1] = A[row * 4 + 1];
                            Mx[row * 4 + 2] = A[row * 4 + 2];
                            Mx[row * 4 + 3] = axv * qv[j] + A[row * 4 + 3];
                        }
                    }
                    float4* o = out + (j + 1) * 3;
                    o[0] = make_float4(Mx[0], Mx[1], Mx[2], Mx[3]);
                    o[1] = make_float4(Mx[4], Mx[5], Mx[6], Mx[7]);
                    o[2] = make_float4(Mx[8], Mx[9], Mx[10], Mx[11]);
                }
            }
        }
        __syncthreads();

        // --- sphere placement: one lane per (timestep, sphere)
        for (int idx = tid; idx < nv * S; idx += kWG) {
            const int c = idx / S;
            const int s = idx - c * S;
            const float4 L = tm.s_local32[s];
            const float4* Fp = fr + ((long long)c * F + tm.s_slot[s]) * 3;
            const float4 r0 = Fp[0], r1 = Fp[1], r2 = Fp[2];
            sph[idx] = make_float4(r0.x * L.x + r0.y * L.y + r0.z * L.z + r0.w,
                                   r1.x * L.x + r1.y * L.y + r1.z * L.z + r1.w,
                                   r2.x * L.x + r2.y * L.y + r2.z * L.z + r2.w, L.w);
        }
        __syncthreads();

        bool overflow = false;   // this lane queued more than the tile capacity

        // --- robot-obstacle and self tests (MV with environment checking)
        if (do_env) {
            const int nslots = tm.n_slots;
            const int ntask = nv * nslots;
            for (int task = wave; task < ntask; task += kWavesPerWG) {
                if (!exhaustive && *(volatile int*)&s_hit) break;
                const int c = task / nslots;
                const int slot = task - c * nslots;
                const int a = slot * 64 + lane;
                bool hit = false;
                if (a < S) {
                    const float4 X = sph[c * S + a];
                    const float rlo = X.w - eps, rhi = X.w + eps;
                    const float lo2 = rlo * rlo, hi2 = rhi * rhi;
                    for (int o = 0; o < env.n_sph; ++o) {
                        const float4 O = env.sph32[o];
                        const float dx = X.x - O.x, dy = X.y - O.y, dz = X.z - O.z;
                        const float d2 = dx * dx + dy * dy + dz * dz;
                        const float R = X.w + O.w;
                        const float Rh = R + eps;
                        if (d2 <= Rh * Rh) {
                            const float Rl = R - eps;
                            if (d2 < Rl * Rl) hit = true;
                            else push_recheck(s_rq, &s_rqn, RK_ENV_SPH, c, a, o, overflow);
                        }
                    }
                    for (int o = 0; o < env.n_box; ++o) {
                        const float* B = env.box32 + o * 16;
                        const float vx = X.x - B[0], vy = X.y - B[1], vz = X.z - B[2];
                        const float p0 = B[3] * vx + B[4] * vy + B[5] * vz;
                        const float p1 = B[6] * vx + B[7] * vy + B[8] * vz;
                        const float p2 = B[9] * vx + B[10] * vy + B[11] * vz;
                        const float e0 = fmaxf(fabsf(p0) - B[12], 0.f);
                        const float e1 = fmaxf(fabsf(p1) - B[13], 0.f);
                        const float e2 = fmaxf(fabsf(p2) - B[14], 0.f);
                        const float val = e0 * e0 + e1 * e1 + e2 * e2;
                        if (val <= hi2) {
                            if (val < lo2) hit = true;
                            else push_recheck(s_rq, &s_rqn, RK_ENV_BOX, c, a, o, overflow);
                        }
                    }
                    for (int o = 0; o < env.n_cyl; ++o) {
                        const float* Y = env.cyl32 + o * 8;
                        const float vx = X.x - Y[0], vy = X.y - Y[1], vz = X.z - Y[2];
                        const float h = vx * Y[3] + vy * Y[4] + vz * Y[5];
                        const float wx = vx - h * Y[3], wy = vy - h * Y[4], wz = vz - h * Y[5];
                        const float sr = sqrtf(wx * wx + wy * wy + wz * wz);
                        const float er = fmaxf(sr - Y[7], 0.f);
                        const float ea = fmaxf(fabsf(h) - Y[6], 0.f);
                        const float val = er * er + ea * ea;
                        if (val <= hi2) {
                            if (val < lo2) hit = true;
                            else push_recheck(s_rq, &s_rqn, RK_ENV_CYL, c, a, o, overflow);
                        }
                    }
                    if (env.n_pts > 0) {
                        // uniform grid: visit cells overlapping the sphere's reach
                        const float reach = X.w + env.pt_radius + eps;
                        int lo3[3], hi3[3];
                        const float xs[3] = { X.x, X.y, X.z };
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            int l = (int)floorf((xs[d] - reach - env.grid_lo[d]) * env.grid_inv);
                            int h = (int)floorf((xs[d] + reach - env.grid_lo[d]) * env.grid_inv);
                            lo3[d] = l < 0 ? 0 : l;
                            hi3[d] = h >= env.grid_dim[d] ? env.grid_dim[d] - 1 : h;
                        }
                        const float Rp = X.w + env.pt_radius;
                        const float plo = (Rp - eps) * (Rp - eps), phi = (Rp + eps) * (Rp + eps);
                        for (int cz = lo3[2]; cz <= hi3[2]; ++cz)
                            for (int cy = lo3[1]; cy <= hi3[1]; ++cy) {
                                const int row = (cz * env.grid_dim[1] + cy) * env.grid_dim[0];
                                if (lo3[0] > hi3[0]) continue;
                                const int pb = env.cell_start[row + lo3[0]];
                                const int pe = env.cell_start[row + hi3[0] + 1];
                                for (int p = pb; p < pe; ++p) {
                                    const float4 Pt = env.pts32[p];
                                    const float dx = X.x - Pt.x, dy = X.y - Pt.y, dz = X.z - Pt.z;
                                    const float d2 = dx * dx + dy * dy + dz * dz;
                                    if (d2 <= phi) {
                                        if (d2 < plo) hit = true;
                                        else push_recheck(s_rq, &s_rqn, RK_ENV_PT, c, a, p, overflow);
                                    }
                                }
                            }
                    }
                    n_env += (unsigned long long)(env.n_sph + env.n_box + env.n_cyl);
                }
                if (__ballot(hit) && lane == 0) s_hit = 1;
            }
            // self-collision pairs
            const int nsc = (tm.n_self + 63) >> 6;
            const int ntask2 = nv * nsc;
            for (int task = wave; task < ntask2; task += kWavesPerWG) {
                if (!exhaustive && *(volatile int*)&s_hit) break;
                const int c = task / nsc;
                const int p = (task - c * nsc) * 64 + lane;
                bool hit = false;
                if (p < tm.n_self) {
                    const int2 pr = tm.self_pairs[p];
                    const float4 A = sph[c * S + pr.x];
                    const float4 B = sph[c * S + pr.y];
                    const float dx = A.x - B.x, dy = A.y - B.y, dz = A.z - B.z;
                    const float d2 = dx * dx + dy * dy + dz * dz;
                    const float R = A.w + B.w;
                    const float Rh = R + eps;
                    if (d2 <= Rh * Rh) {
                        const float Rl = R - eps;
                        if (d2 < Rl * Rl) hit = true;
                        else push_recheck(s_rq, &s_rqn, RK_SELF, c, pr.x, pr.y, overflow);
                    }
                    ++n_self;
                }
                if (__ballot(hit) && lane == 0) s_hit = 1;
            }
        }

        // --- robot-robot tests: lane = sphere a of the lower robot, loop over the partner's spheres
        if (do_rr && !(KIND == 0 && !exhaustive && do_env && *(volatile int*)&s_hit)) {
            const int ntk = tm.n_rr_tasks;
            const int ntask = nv * ntk;
            for (int task = wave; task < ntask; task += kWavesPerWG) {
                const int c = task / ntk;
                if (KIND == 0) {
                    if (!exhaustive && *(volatile int*)&s_hit) break;
                } else if (!exhaustive) {
                    const unsigned best = *(volatile unsigned*)&s_key;
                    if (best != 0xFFFFFFFFu && best < (unsigned)s_t[c] * (unsigned)tm.P) break;
                }
                const int2 tk = tm.rr_tasks[task - c * ntk];
                const int slot = tk.x;
                const int rb = tk.y;
                const int a = slot * 64 + lane;
                const bool act = a < S && tm.s_robot[a] < rb;
                const float4 A = act ? sph[c * S + a] : make_float4(3e18f, 3e18f, 3e18f, 0.f);
                const float rae = A.w + eps;
                const int b0 = tm.r_sphere_off[rb];
                const int b1 = tm.r_sphere_off[rb + 1];
                const float4* Bp = sph + c * S;
                bool maybe = false;
                for (int b = b0; b < b1; ++b) {
                    const float4 B = Bp[b];
                    const float dx = A.x - B.x, dy = A.y - B.y, dz = A.z - B.z;
                    const float d2 = dx * dx + dy * dy + dz * dz;
                    const float R = rae + B.w;
                    maybe |= d2 < R * R;
                }
                if (act) n_rr += (unsigned long long)(b1 - b0);
                bool hit = false;
                if (__ballot(maybe)) {
                    if (maybe) {
                        for (int b = b0; b < b1; ++b) {
                            const float4 B = Bp[b];
                            const float dx = A.x - B.x, dy = A.y - B.y, dz = A.z - B.z;
                            const float d2 = dx * dx + dy * dy + dz * dz;
                            const float R = A.w + B.w;
                            const float Rh = R + eps;
                            if (d2 <= Rh * Rh) {
                                const float Rl = R - eps;
                                if (d2 < Rl * Rl) hit = true;
                                else push_recheck(s_rq, &s_rqn, RK_RR, c, a, b, overflow);
                            }
                        }
                    }
                    if (KIND == 0) {
                        if (__ballot(hit) && lane == 0) s_hit = 1;
                    } else {
                        unsigned key = 0xFFFFFFFFu;
                        if (hit) key = (unsigned)s_t[c] * (unsigned)tm.P + pair_index(tm.s_robot[a], rb, n);
                        key = wave_min_u32(key);
                        if (lane == 0 && key != 0xFFFFFFFFu) atomicMin(&s_key, key);
                    }
                }
            }
        }

        // --- FP64 re-evaluation of near-contact tests
        __syncthreads();
        {
            const int nq = min(s_rqn, kRecheckCap);
            for (int i = tid; i < nq; i += kWG) {
                const int4 rec = s_rq[i];
                const int kind = rec.x & 0xff;
                const int c = rec.x >> 8;
                const int t = s_t[c];
                if (recheck64(tm, env, cd, q, t, kind, rec.y, rec.z)) {
                    if (KIND == 0) s_hit = 1;
                    else atomicMin(&s_key, (unsigned)t * (unsigned)tm.P +
                                               pair_index(tm.s_robot[rec.y], tm.s_robot[rec.z], n));
                }
            }
            n_re += (unsigned long long)(nq > tid ? (nq - tid + kWG - 1) / kWG : 0);
        }
        // records beyond the queue capacity: re-evaluate them by walking the tile again
        if (__syncthreads_or(overflow ? 1 : 0)) {
            // Rare path: every test of this tile is revisited and each near-contact
            // one re-evaluated in FP64 by its own lane.
            if (do_env) {
                const int nslots = tm.n_slots;
                for (int idx = tid; idx < nv * S; idx += kWG) {
                    const int c = idx / S;
                    const int a = idx - c * S;
                    const float4 X = sph[c * S + a];
                    const int t = s_t[c];
                    (void)nslots;
                    for (int o = 0; o < env.n_sph; ++o) {
                        const float4 O = env.sph32[o];
                        const float dx = X.x - O.x, dy = X.y - O.y, dz = X.z - O.z;
                        const float d2 = dx * dx + dy * dy + dz * dz;
                        const float R = X.w + O.w;
                        if (d2 <= (R + eps) * (R + eps) && d2 >= (R - eps) * (R - eps))
                            if (recheck64(tm, env, cd, q, t, RK_ENV_SPH, a, o)) s_hit = 1;
                    }
                    for (int o = 0; o < env.n_box; ++o)
                        if (recheck64(tm, env, cd, q, t, RK_ENV_BOX, a, o)) s_hit = 1;
                    for (int o = 0; o < env.n_cyl; ++o)
                        if (recheck64(tm, env, cd, q, t, RK_ENV_CYL, a, o)) s_hit = 1;
                }
                for (int idx = tid; idx < nv * tm.n_self; idx += kWG) {
                    const int c = idx / tm.n_self;
                    const int2 pr = tm.self_pairs[idx - c * tm.n_self];
                    if (recheck64(tm, env, cd, q, s_t[c], RK_SELF, pr.x, pr.y)) s_hit = 1;
                }
                if (env.n_pts > 0) {
                    for (int idx = tid; idx < nv * S; idx += kWG) {
                        const int c = idx / S;
                        const int a = idx - c * S;
                        const float4 X = sph[c * S + a];
                        const float Rp = X.w + env.pt_radius;
                        for (long long p = 0; p < env.n_pts; ++p) {
                            const float4 Pt = env.pts32[p];
                            const float dx = X.x - Pt.x, dy = X.y - Pt.y, dz = X.z - Pt.z;
                            const float d2 = dx * dx + dy * dy + dz * dz;
                            if (d2 <= (Rp + eps) * (Rp + eps))
                                if (recheck64(tm, env, cd, q, s_t[c], RK_ENV_PT, a, (int)p)) s_hit = 1;
                        }
                    }
                }
            }
            if (do_rr) {
                for (int idx = tid; idx < nv * S; idx += kWG) {
                    const int c = idx / S;
                    const int a = idx - c * S;
                    const int ra = tm.s_robot[a];
                    const float4 A = sph[c * S + a];
                    for (int b = tm.r_sphere_off[ra + 1]; b < S; ++b) {
                        const float4 B = sph[c * S + b];
                        const float dx = A.x - B.x, dy = A.y - B.y, dz = A.z - B.z;
                        const float d2 = dx * dx + dy * dy + dz * dz;
                        const float R = A.w + B.w;
                        if (d2 <= (R + eps) * (R + eps) && d2 >= (R - eps) * (R - eps)) {
                            const int t = s_t[c];
                            if (recheck64(tm, env, cd, q, t, RK_RR, a, b)) {
                                if (KIND == 0) s_hit = 1;
                                else atomicMin(&s_key, (unsigned)t * (unsigned)tm.P +
                                                           pair_index(ra, tm.s_robot[b], n));
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();

        if (tid == 0) {
            s_rqn = 0;
            if (KIND == 0) {
                if (s_hit) atomicOr(cd.word + q, 1u);
            } else {
                if (s_key != 0xFFFFFFFFu) atomicMin(cd.word + q, s_key);
            }
        }
        __syncthreads();
    }

    // counters
    atomicAdd(&cd.stats[ST_RR_TESTS], n_rr);
    if (n_env) atomicAdd(&cd.stats[ST_ENV_TESTS], n_env);
    if (n_self) atomicAdd(&cd.stats[ST_SELF_TESTS], n_self);
    if (n_re) atomicAdd(&cd.stats[ST_RECHECKS], n_re);
    if (tid == 0) {
        atomicAdd(&cd.stats[ST_TILES_RUN], n_run);
        atomicAdd(&cd.stats[ST_TILES_SKIPPED], n_skip);
        atomicAdd(&cd.stats[ST_STATES_EVAL], n_states);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

hipError_t fill_u32(void* p, unsigned v, size_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, stream, (unsigned*)p, v, n);
    return hipGetLastError();
}

hipError_t launch_prepare(const TeamDev& tm, const CallDev& cd, hipStream_t stream)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, cd);
    if (cd.n_queries > 0) {
        const unsigned blocks = (unsigned)((cd.n_queries + 255) / 256);
        hipLaunchKernelGGL(k_query_info, dim3(blocks), dim3(256), 0, stream, tm, cd);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(256), 0, stream, cd);
        hipLaunchKernelGGL(k_assign, dim3(blocks), dim3(256), 0, stream, cd);
    }
    return hipGetLastError();
}

hipError_t launch_validate(const TeamDev& tm, const EnvDev& env, const CallDev& cd, int grid,
                           size_t lds_bytes, hipStream_t stream)
{
    if (cd.n_queries == 0) return hipSuccess;
    if (cd.kind == 0)
        hipLaunchKernelGGL(k_validate<0>, dim3(grid), dim3(kWG), lds_bytes, stream, tm, env, cd);
    else
        hipLaunchKernelGGL(k_validate<1>, dim3(grid), dim3(kWG), lds_bytes, stream, tm, env, cd);
    return hipGetLastError();
}

hipError_t launch_finalize(const TeamDev& tm, const CallDev& cd, hipStream_t stream)
{
    if (cd.n_queries == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((cd.n_queries + 255) / 256);
    hipLaunchKernelGGL(k_finalize, dim3(blocks), dim3(256), 0, stream, tm, cd);
    return hipGetLastError();
}

int validate_blocks_per_cu(int kind, size_t lds_bytes)
{
    int nb = 0;
    hipError_t e = kind == 0
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_validate<0>, kWG, lds_bytes)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_validate<1>, kWG, lds_bytes);
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

}  // namespace mrv
