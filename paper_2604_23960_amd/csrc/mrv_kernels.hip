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

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <mutex>

#include "../../include/mrv.h"
#include "mrv_internal.hpp"


namespace mrv {

namespace {

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v)
{
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (unsigned long long)lo | ((unsigned long long)hi << 32);
}

// Copy of a descriptor that no kernel writes, read through the constant address
// space so that a wave-uniform address turns into scalar loads.
template <class T>
__device__ __forceinline__ T load_descriptor(unsigned long long p)
{
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    T out;
    typedef const __attribute__((address_space(4))) unsigned cu32;
    cu32* src = (cu32*)p;
    unsigned* dst = reinterpret_cast<unsigned*>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
    return out;
}

// Reads of read-only tables at wave-uniform addresses, as scalar loads.
typedef const __attribute__((address_space(4))) float CFloat;
typedef const __attribute__((address_space(4))) int CInt;
typedef const __attribute__((address_space(4))) unsigned long long CU64;
__device__ __forceinline__ int cload(const int* p) { return *(CInt*)p; }
__device__ __forceinline__ float cloadf(const float* p) { return *(CFloat*)p; }
__device__ __forceinline__ unsigned long long cload64(const unsigned long long* p) { return *(CU64*)p; }
typedef int int8v __attribute__((ext_vector_type(8)));
typedef const __attribute__((address_space(4))) int8v CInt8;
// Eight ints at a 32-byte aligned wave-uniform address, as one scalar load.
__device__ __forceinline__ int8v cload8(const int* p) { return *(CInt8*)p; }
typedef int int16v __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(4))) int16v CInt16;
// Sixteen ints at a 64-byte aligned wave-uniform address, as one scalar load.
__device__ __forceinline__ int16v cload16(const int* p) { return *(CInt16*)p; }
typedef float float8v __attribute__((ext_vector_type(8)));
typedef float float16v __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(4))) float8v CFloat8;
typedef const __attribute__((address_space(4))) float16v CFloat16;
__device__ __forceinline__ unsigned long long u64_of(int lo, int hi)
{
    return (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32);
}

// Descriptors read in place through the constant address space (scalar loads).
// A phase takes its own pointer from at(): the address is opaque to the compiler,
// so each phase loads the fields it uses where it uses them instead of every
// field staying in scalar registers for a whole tile.
typedef const __attribute__((address_space(4))) TeamDev CTeam;
typedef const __attribute__((address_space(4))) EnvDev CEnv;
__device__ __forceinline__ unsigned long long opaque_u64(unsigned long long p)
{
    asm volatile("" : "+s"(p));
    return p;
}
__device__ __forceinline__ CTeam* team_at(unsigned long long p) { return (CTeam*)opaque_u64(p); }
__device__ __forceinline__ CEnv* env_at(unsigned long long p) { return (CEnv*)opaque_u64(p); }
// The validation kernel's CallDev argument in place (explicit kernel arguments
// start the kernarg segment), from a new opaque address for each phase.
typedef const __attribute__((address_space(4))) CallDev CCall;
__device__ __forceinline__ CCall& call_at()
{
    return *(CCall*)opaque_u64((unsigned long long)__builtin_amdgcn_kernarg_segment_ptr());
}

// A workgroup flag written by other waves (an LDS load each time).
__device__ __forceinline__ int flag_read(int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ __forceinline__ unsigned flag_read(unsigned* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// (CD: CallDev, or the kernel's arguments read in place, see call_at)
template <class CD>
__device__ __forceinline__ const TeamDev* team_of(const CD& cd, int q) { return cd.q_team ? cd.q_team[q] : cd.team0; }
template <class CD>
__device__ __forceinline__ const EnvDev* env_of(const CD& cd, int q) { return cd.q_env ? cd.q_env[q] : cd.env0; }
template <class CD>
__device__ __forceinline__ long long path_of(const CD& cd, int n_robots, int q)
{
    return cd.q_pathoff ? cd.q_pathoff[q] : (long long)q * n_robots;
}

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
// |v| <= MRV_MAX_COORD, false for NaN and infinities.  An integer test: the
// kernels are compiled assuming no NaN, so a floating-point test could be folded.
// Non-negative doubles order as their bit patterns, and NaN and infinity lie above.
__device__ __forceinline__ bool bounded64(double v)
{
    return (__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFLL) <= __double_as_longlong(MRV_MAX_COORD);
}

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
    const long long p0 = path_of(cd, tm.n_robots, q);
    const long long pb = cd.wp_begin[p0 + r];
    const long long pe = cd.wp_begin[p0 + r + 1];
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
    if (i < 3) cd.ctrl[i] = 0;
    if (i < ST_COUNT) cd.stats[i] = 0ull;
    if (i == 0) {
        // tile counter and total live in 64-bit words after ctrl[0..3]
        unsigned long long* w = reinterpret_cast<unsigned long long*>(cd.ctrl + 4);
        w[0] = 0ull;   // total tiles
        w[1] = 0ull;   // next tile
    }
}

__global__ void k_query_info(CallDev cd)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cd.n_queries) return;
    const TeamDev& tm = *team_of(cd, q);
    const int n = tm.n_robots;
    const long long p0 = path_of(cd, n, q);
    const int chunk = query_chunk(tm.chunk[cd.kind][(cd.flags & MRV_EXHAUSTIVE) ? 1 : 0], cd.lds_bytes, tm.lds_per_t,
                                  cd.chunk_floor, kMaxChunk);
    int T = 0;
    bool ok = chunk * tm.lds_per_t + 64 <= cd.lds_bytes;   // holds by the plan; checked, never assumed
    double mag = 0.0;            // bound on the |FP32 coordinates| of the query's frames and spheres
    for (int r = 0; r < n && ok; ++r) {
        const long long b = cd.wp_begin[p0 + r];
        const long long e = cd.wp_begin[p0 + r + 1];
        if (b < 0 || e <= b || e > cd.n_wp) { ok = false; break; }
        int prev = cd.wp_t[b];
        if (prev != 0) { ok = false; break; }
        const int dof = tm.r_nj[r];
        const int j0 = tm.r_joint_off[r];
        double prism = 0.0;      // largest sum of |prismatic joint value| over the robot's waypoints
        for (long long i = b; i < e && ok; ++i) {
            const int ti = cd.wp_t[i];
            if (i > b && ti <= prev) ok = false;
            prev = ti;
            double ps = 0.0;
            for (int d = 0; d < dof; ++d) {
                const double v = cd.wp_q[i * cd.dof_stride + d];
                if (!bounded64(v)) ok = false;
                else if (tm.j_type[j0 + d] != MRV_REV_Z) ps += fabs(v);
            }
            prism = fmax(prism, ps);
        }
        if (prev >= MRV_MAX_T) ok = false;
        if (prev + 1 > T) T = prev + 1;
        mag = fmax(mag, (double)tm.r_mag[r] + prism);
    }
    long long nt = 0;
    int g = 1;
    if (ok) {
        nt = tiles_of(T, chunk);
        if (nt > cd.max_nt) ok = false;     // cannot happen: T <= max_T and chunk >= chunk_floor
        else {
            // tile order: FFC and MRV_ORDER_LINEAR consecutive timesteps (g = 0), MRV_ORDER_RAKE
            // the paper's rake (g = 1), else the team's tuned interleave, by default the
            // golden-ratio step that spreads every prefix of a query's tiles over its motion
            const unsigned of = cd.flags & (MRV_ORDER_RAKE | MRV_ORDER_LINEAR);
            const int order = cd.kind == 1 || (of & MRV_ORDER_LINEAR) ? 3 : (of & MRV_ORDER_RAKE) ? 2
                            : tm.interleave[0][(cd.flags & MRV_EXHAUSTIVE) ? 1 : 0];
            g = order == 3 ? 0 : order == 2 ? 1 : golden_step((int)nt);
        }
    }
    // Near band.  Every FP32 coordinate the kernels form is relative to the team's
    // origin (frames, spheres) or to the environment's (obstacles, and the spheres
    // moved there by the FP64-rounded offset of the two origins), so FP32 rounding
    // grows with those relative magnitudes, never with where the cell sits in the
    // world.  The band eps holds with a wide margin up to kEpsRefScale metres
    // (measured); beyond it the band grows in proportion, as FP32 error does.
    double m = mag;
    const EnvDev* ep = cd.kind == 0 && (cd.flags & MRV_CHECK_ENV) ? env_of(cd, q) : nullptr;
    if (ep) {
        const double dx = tm.origin64[0] - ep->origin64[0], dy = tm.origin64[1] - ep->origin64[1],
                     dz = tm.origin64[2] - ep->origin64[2];
        m = fmax(m + sqrt(dx * dx + dy * dy + dz * dz), (double)ep->mag);
    }
    const float eps_q = (float)((double)cd.eps32 * fmax(1.0, m / kEpsRefScale));
    cd.T[q] = ok ? T : 0;
    cd.nt[q] = ok ? (int)nt : 0;
    cd.gstep[q] = g;
    cd.q_chunk[q] = chunk;
    cd.q_eps[q] = eps_q;
    cd.status[q] = ok ? 0 : 1;
    cd.word[q] = cd.kind == 1 ? 0xFFFFFFFFu : 0u;
    cd.drop[q] = 0xFFFFFFFFu;
    if (!ok) {
        atomicAdd(&cd.ctrl[3], 1);
    } else {
        atomicAdd(&cd.hist[nt], 1);
        atomicMax(&cd.ctrl[0], (int)nt);
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

__global__ void k_finalize(CallDev cd)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cd.n_queries) return;
    const TeamDev& tm = *team_of(cd, q);
    if (q == 0) atomicMax(&cd.ctrl[8], cd.ctrl[2]);
    const bool bad = cd.status[q] != 0;
    const unsigned w = cd.word[q];
    const unsigned dk = cd.drop[q];
    // a dropped near test matters only if it could still change the answer:
    // MV while no hit is known, FFC when its key is below the best conflict
    const bool unresolved = !bad && (cd.kind == 0 ? (dk != 0xFFFFFFFFu && w == 0u) : dk < w);
    if (unresolved) {
        atomicAdd(&cd.ctrl[1], 1);
        atomicAdd(&cd.ctrl[9], 1);
    }
    if (cd.kind == 0) {
        cd.valid_out[q] = bad ? 2 : unresolved ? 3 : (w == 0u ? 1 : 0);
        return;
    }
    int t = -1, ri = -1, rj = -1;
    if (bad || unresolved) {
        t = ri = rj = (bad ? -2 : -3);
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

// Queue a near-contact test for FP64 re-evaluation by k_recheck, which runs after
// the validation kernel.  key orders the test's possible outcome (MV: 0, FFC:
// t*P + pair); when the call's queue is full the smallest dropped key is kept
// per query and k_finalize decides whether the drop leaves the answer open.
template <class CD>
__device__ __forceinline__ void push_recheck(const CD& cd, int q, int t, int kind, int a, int b, unsigned key)
{
    const unsigned g = atomicAdd(reinterpret_cast<unsigned*>(cd.ctrl + 2), 1u);
    if (g < (unsigned)cd.gq_cap) cd.gq[g] = make_int4(q, t | (kind << 24), a, b);
    else atomicMin(cd.drop + q, key);
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr float kFar = 1.0e30f;     // w of an unused slot: its tests never reach zero

// on where bit `lane` of the wave-uniform mask m is set, else off (the mask acts
// as the lane predicate of one v_cndmask)
__device__ __forceinline__ float lane_select(unsigned long long m, float on, float off)
{
    return __builtin_amdgcn_inverse_ballot_w64(m) ? on : off;
}

// Smallest D in a lane's share of a block: its four rows share the column b, so
// w_b is added once, after the minimum (rounding to nearest is monotonic, so this
// equals the minimum of the four sums).
// The four lane masks of self block sb (one per accumulator register), inline in
// its 64-byte record after the group indices, so one scalar load brings both.
__device__ __forceinline__ const unsigned long long* sb_masks(CTeam* tm, int sb)
{
    return reinterpret_cast<const unsigned long long*>(tm->sblocks + 16 * sb + 8);
}

__device__ __forceinline__ float col_min(floatx4 d, float wb)
{
    return fminf(fminf(fminf(d[0], d[1]), d[2]), d[3]) + wb;
}

__device__ __forceinline__ float block_min(floatx4 d, float wb, float best)
{
    return fminf(best, col_min(d, wb));
}

// Minimum and maximum over each row of 16 lanes, in every lane of the row: lanes
// exchanged within quads, then rows rotated by 4 and 8 (DPP; all lanes active).
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float row_min16(float v)
{
    v = fminf(v, dpp_f32<0xB1>(v));         // quad_perm [1, 0, 3, 2]
    v = fminf(v, dpp_f32<0x4E>(v));         // quad_perm [2, 3, 0, 1]
    v = fminf(v, dpp_f32<0x124>(v));        // row_ror 4
    return fminf(v, dpp_f32<0x128>(v));     // row_ror 8
}

__device__ __forceinline__ float row_max16(float v)
{
    v = fmaxf(v, dpp_f32<0xB1>(v));
    v = fmaxf(v, dpp_f32<0x4E>(v));
    v = fmaxf(v, dpp_f32<0x124>(v));
    return fmaxf(v, dpp_f32<0x128>(v));
}

// Squared distance from x to a box surface region (0 inside), box in the
// precomputed row form of EnvDev::box32.
template <class V>
__device__ __forceinline__ float box_val(float x, float y, float z, const V& B)
{
    const float p0 = fmaf(B[0], x, fmaf(B[1], y, fmaf(B[2], z, B[3])));
    const float p1 = fmaf(B[4], x, fmaf(B[5], y, fmaf(B[6], z, B[7])));
    const float p2 = fmaf(B[8], x, fmaf(B[9], y, fmaf(B[10], z, B[11])));
    const float e0 = fmaxf(fabsf(p0) - B[12], 0.f);
    const float e1 = fmaxf(fabsf(p1) - B[13], 0.f);
    const float e2 = fmaxf(fabsf(p2) - B[14], 0.f);
    return fmaf(e0, e0, fmaf(e1, e1, e2 * e2));
}

template <class V>
__device__ __forceinline__ float cyl_val(float x, float y, float z, const V& Y)
{
    const float vx = x - Y[0], vy = y - Y[1], vz = z - Y[2];
    const float h = fmaf(vx, Y[3], fmaf(vy, Y[4], vz * Y[5]));
    const float wx = fmaf(-h, Y[3], vx), wy = fmaf(-h, Y[4], vy), wz = fmaf(-h, Y[5], vz);
    // hardware square root (within 1 ulp): the near band absorbs far more
    const float sr = __builtin_amdgcn_sqrtf(fmaf(wx, wx, fmaf(wy, wy, wz * wz)));
    const float er = fmaxf(sr - Y[7], 0.f);
    const float ea = fmaxf(fabsf(h) - Y[6], 0.f);
    return fmaf(er, er, ea * ea);
}

// 0 free, 1 hit, 2 near contact, for a squared distance d2 against a contact distance R.
__device__ __forceinline__ int classify(float d2, float R, float eps)
{
    const float hi = R + eps;
    if (d2 > hi * hi) return 0;
    const float lo = fmaxf(R - eps, 0.f);
    return d2 < lo * lo ? 1 : 2;
}

// The pairs one lane covers in block (ga, gb) -- rows 4 (lane / 16) .. + 3 of ga
// against column lane % 16 of gb -- in the direct form, masked by mk (the block's
// four per-register lane masks; null: every pair).  Near pairs below the best
// known outcome are queued.  Returns whether a pair collides.
template <class CD>
__device__ bool direct_block(const CD& cd, CTeam* tm, const float* base, int GSp, int ga, int gb, int lane,
                             const unsigned long long* mk, float eps, int q, int t, int rk, unsigned key, int* s_hit,
                             unsigned* s_key, bool mv)
{
    const int bs = gb * 16 + (lane & 15);
    const float br = base[3 * GSp + bs];
    if (!(br > 0.f)) return false;
    const float bx = base[bs], by = base[GSp + bs], bz = base[2 * GSp + bs];
    bool hit = false;
    for (int r = 0; r < 4; ++r) {
        if (mk && !((cload64(mk + r) >> lane) & 1ull)) continue;
        const int as = ga * 16 + 4 * (lane >> 4) + r;
        const float ar = base[3 * GSp + as];
        if (!(ar > 0.f)) continue;
        const float dx = base[as] - bx, dy = base[GSp + as] - by, dz = base[2 * GSp + as] - bz;
        const int cl = classify(fmaf(dx, dx, fmaf(dy, dy, dz * dz)), ar + br, eps);
        if (cl == 1) {
            hit = true;
        } else if (cl == 2) {
            // a near test matters only below the best known outcome
            const bool open = mv ? !flag_read(s_hit) : key < flag_read(s_key);
            if (open) push_recheck(cd, q, t, rk, tm->slot_sphere[as], tm->slot_sphere[bs], key);
        }
    }
    return hit;
}

// FP32 forward kinematics in two steps (the chain Frame_k = Frame_{k-1} F_k
// J_k(q_k) of the sphere model, paper §II-B), both relative to the team origin.
//
// joint_matrix32: the transform F_j J_j(q_j(t)) of global joint jg at timestep t,
// as three float4 rows [R | p].  The joint value is interpolated in FP64 from the
// robot's path waypoints of the query (paths from qp0), a revolute angle is
// reduced to [-pi, pi] in FP64, and the value is rounded once to FP32.
template <class TP, class CD>
__device__ __forceinline__ void joint_matrix32(TP tm, const CD& cd, long long qp0, int jg, int t, float4* out)
{
    const int r = tm->j_robot[jg];
    const int j = jg - tm->r_joint_off[r];
    const long long pb = cd.wp_begin[qp0 + r], pe = cd.wp_begin[qp0 + r + 1];
    const long long kseg = find_segment(cd.wp_t, pb, pe, t);
    double qj = cd.wp_q[kseg * cd.dof_stride + j];
    if (kseg != pe - 1) {
        const double sfrac = (double)(t - cd.wp_t[kseg]) / (double)(cd.wp_t[kseg + 1] - cd.wp_t[kseg]);
        qj = qj + sfrac * (cd.wp_q[(kseg + 1) * cd.dof_stride + j] - qj);
    }
    const int jt = tm->j_type[jg];
    // an angle enters only through sin and cos: take it modulo 2 pi while it is
    // exact, so its FP32 rounding error stays below 2^-24 pi
    if (jt == MRV_REV_Z) qj = fma(-6.283185307179586, rint(qj * 0.15915494309189535), qj);
    const float qf = (float)qj;
    const float4* Fp = reinterpret_cast<const float4*>(tm->j_fixed32 + (long long)jg * 12);
    float4 m[3] = { Fp[0], Fp[1], Fp[2] };
    if (jt == MRV_REV_Z) {
        // F Rz(q): columns 0 and 1 of F rotated by q
        float sn, cs;
        sincosf(qf, &sn, &cs);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float a0 = m[i].x, a1 = m[i].y;
            m[i].x = a0 * cs + a1 * sn;
            m[i].y = a1 * cs - a0 * sn;
        }
    } else {
        // F T(q e_axis): the translation column gains q times that axis' column
        const int ax = jt - 1;
#pragma unroll
        for (int i = 0; i < 3; ++i) m[i].w = fmaf(ax == 0 ? m[i].x : (ax == 1 ? m[i].y : m[i].z), qf, m[i].w);
    }
    out[0] = m[0];
    out[1] = m[1];
    out[2] = m[2];
}

// chain_row32: row `row` of every frame of robot r from the joint transforms M of
// one timestep (three float4 rows per global joint).  Row i of Frame_k depends
// only on row i of Frame_{k-1}, so the three rows of a chain run on three lanes.
// frames receives (n_joints + 1) frames as three float4 rows each, the base first.
template <class TP>
__device__ __forceinline__ void chain_row32(TP tm, int r, int row, const float4* M, float4* frames)
{
    const float4 b = *reinterpret_cast<const float4*>(&tm->r_base32[r * 12 + row * 4]);
    float x = b.x, y = b.y, z = b.z, w = b.w;
    frames[row] = b;
    const int nj = tm->r_nj[r];
    const float4* Mk = M + tm->r_joint_off[r] * 3;
    for (int k = 0; k < nj; ++k, Mk += 3) {
        const float4 m0 = Mk[0], m1 = Mk[1], m2 = Mk[2];
        const float nx = fmaf(z, m2.x, fmaf(y, m1.x, x * m0.x));
        const float ny = fmaf(z, m2.y, fmaf(y, m1.y, x * m0.y));
        const float nz = fmaf(z, m2.z, fmaf(y, m1.z, x * m0.z));
        const float nw = fmaf(z, m2.w, fmaf(y, m1.w, fmaf(x, m0.w, w)));
        x = nx;
        y = ny;
        z = nz;
        w = nw;
        frames[(k + 1) * 3 + row] = make_float4(x, y, z, w);
    }
}

// Sphere centre Frame c (radius passed through) from a frame's three rows.
__device__ __forceinline__ float4 place32(const float4* Fp, float4 L)
{
    const float4 r0 = Fp[0], r1 = Fp[1], r2 = Fp[2];
    return make_float4(fmaf(r0.x, L.x, fmaf(r0.y, L.y, fmaf(r0.z, L.z, r0.w))),
                       fmaf(r1.x, L.x, fmaf(r1.y, L.y, fmaf(r1.z, L.z, r1.w))),
                       fmaf(r2.x, L.x, fmaf(r2.y, L.y, fmaf(r2.z, L.z, r2.w))), L.w);
}

// Value of v in lane src (every lane active).
__device__ __forceinline__ float lane_get(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

__device__ __forceinline__ float readlane_f32(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Maximum over the wave, in every lane (every lane active): the row maxima, then
// the four rows' values read from their first lanes.
__device__ __forceinline__ float wave_max_f32(float v)
{
    v = row_max16(v);
    return fmaxf(fmaxf(readlane_f32(v, 0), readlane_f32(v, 16)), fmaxf(readlane_f32(v, 32), readlane_f32(v, 48)));
}

// Grid cell of coordinate offset v (metres past the grid's low corner) along an axis
// of dim cells at 1 / cell = inv, as an int in [-1, dim] (clamped before conversion).
__device__ __forceinline__ int cell_of(float v, float inv, int dim)
{
    return (int)floorf(fminf(fmaxf(v * inv, -1.f), (float)dim));
}

// Sphere-point tests of one wave's 64 slots (four groups of 16) against the point
// cloud, as 16 x 16 blocks on the matrix cores.  For a sphere (centre c, radius
// r_s) and a point p of the cloud (radius r_p), with R = r_s + r_p,
//   D = |c|^2 - R^2 - 2 c.p + |p|^2 = |p - c|^2 - R^2,
// one MFMA per block: K = 4 rows (-2c, 1) of 16 spheres, columns (p, |p|^2) of 16
// consecutive points of the sorted cloud (|p|^2 is stored with each point), the
// accumulator preset to |c|^2 - R^2.  Group by group, the points are those of the
// grid's cell rows that meet the group's bounding box widened by R + eps, each row
// cut to the union of the group's chords on it (a point within R + eps of a sphere
// lies in that union: the cut rounds by about 1e-7 m, far inside eps); each row is
// a contiguous run of the cloud, taken 32 points at a time (16 at its end), so a step may
// run past its row's end into the next points of the cloud, which are real points
// as well (the cloud is padded past its end with copies of its last point): a hit
// among them is a real collision and a clear one changes nothing.  A lane whose
// smallest D lies within the rounding bound of the band revisits its pairs in the
// direct form |p - c|^2 against (R -+ eps)^2, the FP32 test of every other
// sphere-obstacle pair, and queues those within the band for FP64.  a0: slot of
// lane 0; x, y, z: the lane's centre in the environment's frame.  Returns whether
// one of the lane's tests is a sure collision; adds the pairs tested to *s_npt.
template <class CD>
__device__ bool point_blocks(const CD& cd, CTeam* tm, CEnv* env, int a0, float x, float y, float z, float rad,
                             bool act, float eps, bool exhaustive, int q, int t, int* s_hit,
                             unsigned long long* s_npt, int lane)
{
    const float rp = env->pt_radius;
    const float R = rad + rp;
    const float reach = R + eps;
    const float w_own = act ? fmaf(-R, R, fmaf(x, x, fmaf(y, y, z * z))) : kFar;
    const float lx = row_min16(act ? x - reach : 3.0e38f), hx = row_max16(act ? x + reach : -3.0e38f);
    const float ly = row_min16(act ? y - reach : 3.0e38f), hy = row_max16(act ? y + reach : -3.0e38f);
    const float lz = row_min16(act ? z - reach : 3.0e38f), hz = row_max16(act ? z + reach : -3.0e38f);
    const float cell = env->grid_cell;
    constexpr int kPtSteps = 2;
    // |D_fp32 - D| for |c|, |p| <= rho and R <= Rm: the accumulator's |c|^2 - R^2 within
    // 3 u (rho^2 + Rm^2), the stored |p|^2 within u rho^2, and the MFMA's products and
    // four additions, whose partial sums stay below (|c| + |p|)^2 + R^2 <= 4 rho^2 + Rm^2,
    // within 2 u rho^2 + 4 u (4 rho^2 + Rm^2): 22 u rho^2 + 7 u Rm^2 in all; 40 u leaves a margin
    const float c2 = wave_max_f32(act ? fmaf(x, x, fmaf(y, y, z * z)) : 0.f);
    const float rho2 = fmaxf(c2, env->mag * env->mag);
    const float Rm = tm->r_max + rp;
    const float e_err = 40.f * 5.9604645e-8f * (rho2 + Rm * Rm) + 1.0e-30f;
    const float e_hi = e_err + fmaf(2.f * Rm, eps, eps * eps);
    const float e_lo = -(e_err + 2.f * Rm * eps);
    const unsigned long long am = __ballot(act);
    const int i16 = lane & 15, q4 = lane >> 4;
    const float* ptsf = reinterpret_cast<const float*>(env->pts32);
    const unsigned lane_off = (unsigned)(i16 * 4 + q4);
    const float ginv = env->grid_inv;
    const int d0 = env->grid_dim[0], d1 = env->grid_dim[1], d2 = env->grid_dim[2];
    bool hit = false;
    unsigned long long tests = 0;
    for (int g = 0; g < 4; ++g) {
        const unsigned gm = (unsigned)(am >> (16 * g)) & 0xFFFFu;
        if (gm == 0u) continue;
        if (!exhaustive && flag_read(s_hit)) break;
        // cells of the group's box (wave-uniform)
        const int cx0 = max(cell_of(readlane_f32(lx, 16 * g) - env->grid_lo[0], ginv, d0), 0);
        const int cx1 = min(cell_of(readlane_f32(hx, 16 * g) - env->grid_lo[0], ginv, d0), d0 - 1);
        const int cy0 = max(cell_of(readlane_f32(ly, 16 * g) - env->grid_lo[1], ginv, d1), 0);
        const int cy1 = min(cell_of(readlane_f32(hy, 16 * g) - env->grid_lo[1], ginv, d1), d1 - 1);
        const int cz0 = max(cell_of(readlane_f32(lz, 16 * g) - env->grid_lo[2], ginv, d2), 0);
        const int cz1 = min(cell_of(readlane_f32(hz, 16 * g) - env->grid_lo[2], ginv, d2), d2 - 1);
        if (cx0 > cx1 || cy0 > cy1 || cz0 > cz1) continue;
        const int ny = cy1 - cy0 + 1;
        const int n_rows = ny * (cz1 - cz0 + 1);
        // operands: A row i = sphere i of the group, component q4; accumulator rows 4 q4 + r
        const int src = 16 * g + i16;
        const float ax = lane_get(x, src), ay = lane_get(y, src), az = lane_get(z, src);
        const float aop = q4 == 0 ? -2.f * ax : (q4 == 1 ? -2.f * ay : (q4 == 2 ? -2.f * az : 1.f));
        const int s0 = 16 * g + 4 * q4;
        const floatx4 acc = { lane_get(w_own, s0), lane_get(w_own, s0 + 1), lane_get(w_own, s0 + 2),
                              lane_get(w_own, s0 + 3) };
        const unsigned nact = (unsigned)__popc(gm);
        const float half = 0.5f * cell;
        const float ymid0 = env->grid_lo[1] + half, zmid0 = env->grid_lo[2] + half;
        float best = 3.0e38f;
        unsigned long long gpts = 0;   // points taken by the steps (wave-uniform)
        // rows 64 at a time, one per lane, each cut to the x extent the group can reach
        // on it; then the non-empty rows by the whole wave
        auto rows = [&](auto&& batch) {
            for (int r0 = 0; r0 < n_rows; r0 += kWave) {
                const int rr = r0 + lane;
                int pb = 0, pe = 0;
                if (rr < n_rows) {
                    const int cz = cz0 + rr / ny;
                    const int cy = cy0 + (rr - (cz - cz0) * ny);
                    // the row's y and z cell centres; a sphere's distance to the row's slab is
                    // |centre - mid| - cell / 2 per axis (0 inside)
                    const float ym = fmaf((float)cy, cell, ymid0), zm = fmaf((float)cz, cell, zmid0);
                    float xa = 3.0e38f, xb = -3.0e38f;
                    for (unsigned gs = gm; gs; gs &= gs - 1u) {
                        const int sl = 16 * g + __builtin_ctz(gs);
                        const float sx = readlane_f32(x, sl), sy = readlane_f32(y, sl), sz = readlane_f32(z, sl);
                        const float sr = readlane_f32(reach, sl);
                        const float dz = fmaxf(fabsf(sz - zm) - half, 0.f);
                        const float dy = fmaxf(fabsf(sy - ym) - half, 0.f);
                        const float rem = fmaf(sr, sr, -fmaf(dy, dy, dz * dz));
                        // no chord: a half-width of -3e38 leaves both ends unchanged
                        const float hw = rem >= 0.f ? __builtin_amdgcn_sqrtf(rem) : -3.0e38f;
                        xa = fminf(xa, sx - hw);
                        xb = fmaxf(xb, sx + hw);
                    }
                    const int ax = max(cell_of(xa - env->grid_lo[0], ginv, d0), cx0);
                    const int bx = min(cell_of(xb - env->grid_lo[0], ginv, d0), cx1);
                    if (ax <= bx) {
                        const int crow = (cz * d1 + cy) * d0;
                        pb = env->cell_start[crow + ax];
                        pe = env->cell_start[crow + bx + 1];
                    }
                }
                batch(pb, pe);
            }
        };
        // the rows' points in steps of 32 (16 where a row has no more), the loads of
        // kPtSteps steps in flight at a time
        rows([&](int pb, int pe) {
            unsigned long long m = __ballot(pe > pb);
            int b = 0, se = 0;
            for (;;) {
                float v0[kPtSteps], v1[kPtSteps];
                bool two[kPtSteps];     // the step's second 16 points hold some of the row's
                int n = 0;
#pragma unroll
                for (int k = 0; k < kPtSteps; ++k) {
                    if (b >= se) {
                        if (!m) break;
                        const int L = __builtin_ctzll(m);
                        m &= m - 1;
                        b = __builtin_amdgcn_readlane(pb, L);
                        se = __builtin_amdgcn_readlane(pe, L);
                        gpts += (unsigned)((se - b + 15) & ~15);
                    }
                    two[k] = se - b > 16;
                    // a wave-uniform base and a fixed lane offset: component q4 of point b + i16
                    const float* step = ptsf + (size_t)(unsigned)b * 4;
                    v0[k] = step[lane_off];
                    v1[k] = two[k] ? step[lane_off + 64] : 0.f;
                    b += 32;
                    n = k + 1;
                }
                if (n == 0) break;
#pragma unroll
                for (int k = 0; k < kPtSteps; ++k) {
                    if (k < n) {
                        const floatx4 e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, v0[k], acc, 0, 0, 0);
                        best = fminf(best, fminf(fminf(e0[0], e0[1]), fminf(e0[2], e0[3])));
                        if (two[k]) {
                            const floatx4 e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, v1[k], acc, 0, 0, 0);
                            best = fminf(best, fminf(fminf(e1[0], e1[1]), fminf(e1[2], e1[3])));
                        }
                    }
                }
                if (n < kPtSteps) break;
            }
        });
        tests += (unsigned long long)nact * gpts;
        const bool sure = best < e_lo;
        const bool unsure = !sure && best < e_hi;
        hit = hit || sure;
        // rare: pairs within the band and no collision known
        if (__ballot(unsure) && !__ballot(hit) && !flag_read(s_hit)) {
            const long long last = env->n_pts - 1;
            // sphere by sphere of the lane's four rows, to keep few values live
#pragma unroll 1
            for (int r = 0; r < 4; ++r) {
                const float sx = lane_get(x, s0 + r), sy = lane_get(y, s0 + r), sz = lane_get(z, s0 + r);
                const float sr = lane_get(act ? rad : -1.f, s0 + r);
                if (!__ballot(unsure && sr >= 0.f)) continue;
                const float Rp = sr + rp;
                const float plo = fmaxf(Rp - eps, 0.f), phi = Rp + eps;
                // (read only for a real sphere: the wave's last chunk may end past the slots)
                const int sphere = sr >= 0.f ? tm->slot_sphere[a0 + s0 + r] : -1;
                rows([&](int pb, int pe) {
                    for (unsigned long long m = __ballot(pe > pb); m; m &= m - 1) {
                    const int L = __builtin_ctzll(m);
                    const int sb = __builtin_amdgcn_readlane(pb, L), se = __builtin_amdgcn_readlane(pe, L);
                    for (int b = sb; b < se; b += 16) {
                        const int p = b + i16;
                        const float4 P = env->pts32[p];
                        const float dx = sx - P.x, dy = sy - P.y, dz = sz - P.z;
                        const float dd = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        if (unsure && sr >= 0.f && dd <= phi * phi) {
                            if (dd < plo * plo) hit = true;
                            else if (!hit && !flag_read(s_hit))
                                push_recheck(cd, q, t, RK_ENV_PT, sphere, (int)min((long long)p, last), 0u);
                        }
                    }
                    }
                });
            }
        }
    }
    if (lane == 0 && tests) atomicAdd(s_npt, tests);
    return hit;
}

// Robot-obstacle tests of J (timestep, 64-slot chunk) tasks of one wave, one lane
// per slot, in the environment's frame (`off` = team origin minus environment
// origin), obstacle parameters in wave-uniform scalar loads (each sphere
// obstacle's loaded once for all J tasks).  Sets *s_hit on a confirmed hit; near
// tests below the known outcome are queued for FP64 re-evaluation.  The kernel
// passes one task at a time: with boxes and cylinders selected per task, larger
// J only adds register pressure.
// World boxes of obstacles ob + lane % 16 and ob + 16 + lane % 16 (empty past nbc).
struct ObBoxes {
    float3 lo[2], hi[2];
};
__device__ __forceinline__ ObBoxes ob_boxes(CEnv* env, int nbc, int ob, int lane)
{
    ObBoxes r;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int o = ob + 16 * k + (lane & 15);
        r.lo[k] = make_float3(3.0e38f, 3.0e38f, 3.0e38f);
        r.hi[k] = make_float3(-3.0e38f, -3.0e38f, -3.0e38f);
        if (o < nbc) {
            const float4 a = env->bc_box[2 * o], b = env->bc_box[2 * o + 1];
            r.lo[k] = make_float3(a.x, a.y, a.z);
            r.hi[k] = make_float3(b.x, b.y, b.z);
        }
    }
    return r;
}

template <int J, bool PTS, class CD>
__device__ __forceinline__ void env_tasks(const CD& cd, CTeam* tm, CEnv* env, const float* sp,
                                          const int* task, int nch, float ro_max, float eps, bool exhaustive, int q,
                                          unsigned focus, bool fall, const int* s_t, int* s_hit,
                                          unsigned& c_env, unsigned long long* s_npt, int lane, float3 off,
                                          const ObBoxes& pre)
{
    const int GS = tm->GS, GSp = tm->GSp, TS = tm->TS;
    int c[J], a[J];
    float x[J], y[J], z[J], rad[J], mb[J], ms[J];
    bool act[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        c[j] = task[j] / nch;
        a[j] = (task[j] - c[j] * nch) * kWave + lane;     // slot
        const float* row = sp + (long long)c[j] * TS + a[j];
        rad[j] = a[j] < GS ? row[3 * GSp] : 0.f;
        act[j] = rad[j] > 0.f;
        if (act[j] && !fall) act[j] = ((focus >> tm->s_robot[tm->slot_sphere[a[j]]]) & 1u) != 0;
        x[j] = 1.0e18f; y[j] = 1.0e18f; z[j] = 1.0e18f;
        if (act[j]) {
            // team-origin coordinates moved to the environment's frame
            x[j] = row[0] + off.x;
            y[j] = row[GSp] + off.y;
            z[j] = row[2 * GSp] + off.z;
        }
        mb[j] = 3.0e38f;
        ms[j] = 3.0e38f;
    }
    // Boxes and cylinders, task by task, each only where its world-axis box meets
    // the box of one of the task's four rows of 16 slots, the spheres widened by
    // 2 eps: every other test lies beyond the near band (the FP32 centres are far
    // closer than eps to the FP64 ones) and so is clear in FP64 as well.
    const int nbc = env->n_box + env->n_cyl;
    unsigned n_tested[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        n_tested[j] = (unsigned)env->n_sph;
        if (nbc == 0) continue;
        const float w = rad[j] + 2.f * eps;
        const float lx = row_min16(act[j] ? x[j] - w : 3.0e38f), hx = row_max16(act[j] ? x[j] + w : -3.0e38f);
        const float ly = row_min16(act[j] ? y[j] - w : 3.0e38f), hy = row_max16(act[j] ? y[j] + w : -3.0e38f);
        const float lz = row_min16(act[j] ? z[j] - w : 3.0e38f), hz = row_max16(act[j] ? z[j] + w : -3.0e38f);
        // lane l compares the box of its own row with obstacle ob + l % 16, so a
        // ballot covers 16 obstacles against all four rows
        auto group = [&](int ob, float3 olo, float3 ohi) {
            const unsigned long long m4 = __ballot((olo.x <= hx) & (ohi.x >= lx) & (olo.y <= hy) & (ohi.y >= ly) &
                                                   (olo.z <= hz) & (ohi.z >= lz));
            const unsigned m = (unsigned)((m4 | (m4 >> 16) | (m4 >> 32) | (m4 >> 48)) & 0xFFFFull);
            n_tested[j] += (unsigned)__popc(m);
            const int nb = min(max(env->n_box - ob, 0), 16);
            const unsigned low = (1u << nb) - 1u;
            // each box's (cylinder's) row form in one scalar load
            for (unsigned mm = m & low; mm; mm &= mm - 1u) {
                const int b = ob + __builtin_ctz(mm);
                const float16v B = *(CFloat16*)(env->box32 + b * 16);
                mb[j] = fminf(mb[j], box_val(x[j], y[j], z[j], B));
            }
            for (unsigned mm = m & ~low; mm; mm &= mm - 1u) {
                const int b = ob + __builtin_ctz(mm) - env->n_box;
                const float8v Y = *(CFloat8*)(env->cyl32 + b * 8);
                mb[j] = fminf(mb[j], cyl_val(x[j], y[j], z[j], Y));
            }
        };
        // the first 32 obstacles' world boxes come in registers (loaded once per tile;
        // not in the point-cloud build, whose grid walk needs the registers), the rest
        // from memory
        int ob = 0;
        if constexpr (!PTS) {
            group(0, pre.lo[0], pre.hi[0]);
            if (nbc > 16) group(16, pre.lo[1], pre.hi[1]);
            ob = 32;
        }
        for (; ob < nbc; ob += 16) {
            const ObBoxes more = ob_boxes(env, nbc, ob, lane);
            group(ob, more.lo[0], more.hi[0]);
        }
    }
    for (int o = 0; o < env->n_sph; ++o) {
        const float* ob = &env->sph32[o].x;
        const float ocx = cloadf(ob), ocy = cloadf(ob + 1), ocz = cloadf(ob + 2), orad = cloadf(ob + 3);
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const float Rs = rad[j] + orad;
            const float dx = x[j] - ocx, dy = y[j] - ocy, dz = z[j] - ocz;
            ms[j] = fminf(ms[j], fmaf(-Rs, Rs, fmaf(dx, dx, fmaf(dy, dy, dz * dz))));
        }
    }
    bool any_hit = false;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (act[j]) c_env += n_tested[j];
        const float rlo = fmaxf(rad[j] - eps, 0.f), rhi = rad[j] + eps;
        const float Rb = rad[j] + ro_max;
        // common case first: no lane within the near band of a box, cylinder or sphere
        bool hit = false, unsure = false;
        const bool near = act[j] && ((mb[j] <= rhi * rhi) || (ms[j] <= fmaf(2.f * Rb, eps, eps * eps)));
        if (__ballot(near)) {
            hit = near && ((mb[j] < rlo * rlo) || (ms[j] < -2.f * Rb * eps));
            unsure = near && !hit;
        }
        // the sphere index and timestep of a queued test, read only when one is queued
        auto sa_of = [&]() { return tm->slot_sphere[a[j]]; };
        auto t_of = [&]() { return s_t[c[j]]; };
        if constexpr (PTS) {
            if (env->n_pts > 0 && point_blocks(cd, tm, env, a[j] - lane, x[j], y[j], z[j], rad[j], act[j], eps,
                                               exhaustive, q, t_of(), s_hit, s_npt, lane))
                hit = true;
        }
        if (unsure && !(hit && !exhaustive)) {
            // rare: find the near obstacles and queue each for FP64 re-evaluation
            const float xj = x[j], yj = y[j], zj = z[j];
            for (int o = 0; o < env->n_box; ++o) {
                const float v = box_val(xj, yj, zj, (CFloat*)(env->box32 + o * 16));
                if (v < rlo * rlo) hit = true;
                else if (v <= rhi * rhi && !hit && !flag_read(s_hit))
                    push_recheck(cd, q, t_of(), RK_ENV_BOX, sa_of(), o, 0u);
            }
            for (int o = 0; o < env->n_cyl; ++o) {
                const float v = cyl_val(xj, yj, zj, (CFloat*)(env->cyl32 + o * 8));
                if (v < rlo * rlo) hit = true;
                else if (v <= rhi * rhi && !hit && !flag_read(s_hit))
                    push_recheck(cd, q, t_of(), RK_ENV_CYL, sa_of(), o, 0u);
            }
            for (int o = 0; o < env->n_sph; ++o) {
                const float* ob = &env->sph32[o].x;
                const float dx = xj - cloadf(ob), dy = yj - cloadf(ob + 1), dz = zj - cloadf(ob + 2);
                const int cl = classify(fmaf(dx, dx, fmaf(dy, dy, dz * dz)), rad[j] + cloadf(ob + 3), eps);
                if (cl == 1) hit = true;
                else if (cl == 2 && !hit && !flag_read(s_hit))
                    push_recheck(cd, q, t_of(), RK_ENV_SPH, sa_of(), o, 0u);
            }
        }
        any_hit = any_hit || hit;
    }
    if (__ballot(any_hit) && lane == 0) *s_hit = 1;
}

// PTS: the build for calls whose environments hold point clouds (the grid walk of
// the obstacle phase); without it the walk compiles out, which keeps its registers
// out of every other call.
template <int KIND, bool PTS>
__global__ __launch_bounds__(validate_wg(KIND), KIND <= 2 ? 2 : (KIND == 3 ? (PTS ? kExhPtsWGsPerCU : kExhWGsPerCU) : (KIND == 4 ? kExhWGsPerCU : kWGsPerCU))) void k_validate(CallDev cd_arg)
{
    (void)cd_arg;   // read in place through call_at()
    CCall& cd = call_at();
    // KIND: 0 early-terminating MV, 1 early-terminating FFC, 2 early-terminating MV
    // with a focus set (prioritised MV), 3 exhaustive MV, 4 exhaustive FFC, 5
    // exhaustive MV with a focus set
    constexpr bool kMV = KIND != 1 && KIND != 4;
    constexpr bool kFocus = KIND == 2 || KIND == 5;
    // exhaustive MV runs each group's self blocks over the tile's timesteps in an
    // inner loop (no early exit to honour between timesteps)
    constexpr bool kSelfInner = KIND == 3 || KIND == 5;
    constexpr bool kPrio = KIND == 0;   // pair-prioritised order: early-terminating plain MV
    constexpr int kSI = 4;

    constexpr int WG = validate_wg(KIND);
    constexpr int kWaves = WG / kWave;
    extern __shared__ float4 dyn[];

    __shared__ int s_t[kMaxChunk];
    __shared__ int s_q, s_nv, s_phase, s_hit, s_chunk;
    __shared__ unsigned s_key, s_rho2;
    __shared__ float s_eps;
    __shared__ unsigned long long s_tp, s_ep;
    __shared__ unsigned s_focus;
    // thread 0's claim state and tile counts, kept in LDS rather than registers
    __shared__ long long s_kcur, s_off0, s_off1;   // current rank and its tile range [off[k], off[k + 1])
    __shared__ long long s_gnext, s_gend;          // tiles claimed by the last atomic and not yet run
    __shared__ int s_phase_cur;
    __shared__ unsigned long long s_nrun, s_nskip, s_nstates, s_npt;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_uniform(tid >> 6);
    const unsigned flags = cd.flags;
    const bool exhaustive = KIND >= 3;
    const bool check_env = kMV && (flags & MRV_CHECK_ENV) != 0;
    const bool hier = check_env && (flags & MRV_HIERARCHICAL) != 0;

    // the tile space, read once into LDS (thread 0's claims read it from there)
    __shared__ long long s_total, s_gtotal;
    __shared__ int s_M, s_kc;

    unsigned long long c_rr = 0, c_self = 0;    // wave-uniform counters
    unsigned c_env = 0;                         // per lane: obstacle tests of this workgroup's tiles
    if (tid == 0) {
        const long long total = (long long)__hip_atomic_load(reinterpret_cast<unsigned long long*>(cd.ctrl + 4),
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_total = total;
        s_gtotal = hier ? 2 * total : total;
        s_M = cd.ctrl[0];
        // tiles per claim: the call's value, or (automatic) at most that, keeping at
        // least 8 claims per workgroup
        const long long per = (hier ? 2 * total : total) / (8ll * (long long)gridDim.x);
        s_kc = cd.claim_auto ? (int)(per < 1 ? 1 : (per < cd.claim ? per : cd.claim)) : cd.claim;
        s_kcur = 0;
        s_gnext = 0;
        s_gend = 0;
        s_off0 = 0;
        s_off1 = -1;                    // no rank range cached yet
        s_phase_cur = 0;
        s_nrun = 0;
        s_nskip = 0;
        s_nstates = 0;
        s_npt = 0;
        s_q = -1;                       // no tile yet whose outcome is to publish
        s_nv = 0;
    }

    for (;;) {
        // Wave priorities in exhaustive calls: the serial part of a tile (claim, FK,
        // records; one busy wave per workgroup) and the obstacle phase issue first,
        // then the self blocks, while the robot-robot blocks' MFMA chains, which wait
        // on the matrix pipe anyway, fill the gaps (early-terminating calls keep one
        // level: their obstacle verdicts end queries).
        if (exhaustive) __builtin_amdgcn_s_setprio(2);
        if (tid == 0) {
            CCall& cd = call_at();
            unsigned long long* w64 = reinterpret_cast<unsigned long long*>(cd.ctrl + 4);
            const long long* off = reinterpret_cast<const long long*>(cd.off);
            const long long total = s_total, gtotal = s_gtotal;
            const int M = s_M;
            // the previous tile's outcome (all its waves passed the barrier that
            // ended it) goes to its query's word before the next claim
            if (s_q >= 0 && s_nv > 0) {
                if (kMV) {
                    if (s_hit) atomicOr(cd.word + s_q, 1u);
                } else {
                    if (s_key != 0xFFFFFFFFu) atomicMin(cd.word + s_q, s_key);
                }
            }
            // s_kc consecutive tiles per atomic (one counter serves the whole chip)
            long long g = s_gnext;
            if (g >= s_gend) {
                const int kc = s_kc;
                g = (long long)atomicAdd(&w64[1], (unsigned long long)kc);
                s_gend = g + kc;
            }
            s_gnext = g + 1;
            int q = -1, nv = 0, phase = 0, C = 1;
            unsigned known = !kMV ? 0xFFFFFFFFu : 0u, focus = 0u;
            if (g < gtotal) {
                long long gg = g;
                if (hier) {
                    phase = g >= total ? 1 : 0;
                    gg = g - (long long)phase * total;
                    if (phase != s_phase_cur) { s_phase_cur = phase; s_kcur = 0; s_off1 = -1; }
                }
                // largest rank k with off[k] <= gg (ranks are non-empty below M; off[M] =
                // total).  A workgroup's tile numbers only grow within a phase, so most
                // claims fall in the cached range of the previous rank and load nothing.
                long long lo = s_kcur, o0 = s_off0, o1 = s_off1;
                if (!(gg < o1)) {
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
                    o0 = off[lo];
                    o1 = off[lo + 1];
                    s_kcur = lo;
                    s_off0 = o0;
                    s_off1 = o1;
                }
                const int k = (int)lo;
                q = cd.sorted_q[gg - o0];
                if (kFocus) focus = cd.q_focus ? cd.q_focus[q] : cd.focus0;
                const TeamDev* tq = team_of(cd, q);
                const EnvDev* eq = env_of(cd, q);
                s_tp = (unsigned long long)tq;
                s_ep = (unsigned long long)eq;
                C = cd.q_chunk[q];
                s_eps = cd.q_eps[q];
                const int T = cd.T[q];
                const int nt = cd.nt[q];
                // tile k of the query: consecutive timesteps (g = 0), or every nt-th from
                // the interleaved base (k g) mod nt
                const int gq = cd.gstep[q];
                int base, stride;
                if (!kMV || gq == 0) {
                    base = k * C; stride = 1;
                } else {
                    base = (int)(((long long)k * gq) % nt);
                    stride = nt;
                }
                for (int c = 0; c < C; ++c) {
                    const long long t = (long long)base + (long long)c * stride;
                    if (t < T) { s_t[c] = (int)t; nv = c + 1; }
                }
                // the outcome known so far: skips the tile (early exit, pruning) or,
                // in exhaustive mode, only the queueing of near tests it decides
                known = load_word(cd.word + q);
                bool skip = false;
                if (!exhaustive) {
                    if (kMV) skip = (known != 0u);
                    else skip = (known != 0xFFFFFFFFu) && (known < (unsigned)base * (unsigned)tq->P);
                }
                if (skip) { nv = 0; ++s_nskip; }
                else { ++s_nrun; s_nstates += (unsigned long long)nv * tq->n_robots; }
            }
            s_q = q; s_phase = phase; s_nv = nv; s_chunk = C; s_focus = focus;
            s_hit = kMV && known != 0u; s_key = !kMV ? known : 0xFFFFFFFFu; s_rho2 = 0u;
        }
        __syncthreads();
        CCall& cd = call_at();
        const int q = s_q;
        if (q < 0) break;
        const int nv = s_nv;
        if (nv == 0) { __syncthreads(); continue; }
        const int phase = s_phase;
        const bool do_env = check_env && (!hier || phase == 0);
        const bool do_rr = !hier || phase == 1;
        // this tile's team and environment, and its LDS partition
        const unsigned long long tpu = uniform_u64(s_tp);
        const unsigned long long epu = uniform_u64(s_ep);
        CTeam* tm = team_at(tpu);
        const int C = wave_uniform(s_chunk);
        const float eps = __int_as_float(wave_uniform(__float_as_int(s_eps)));   // this query's near band
        // prioritised MV: robots outside the focus set only take part in pairs
        // with a robot in it
        const unsigned focus = kFocus ? (unsigned)wave_uniform((int)s_focus) : 0u;
        const int S = tm->S;
        const int F = tm->F;
        const int G = tm->G;
        const int n = tm->n_robots;
        const unsigned all_robots = n >= 32 ? 0xFFFFFFFFu : (1u << n) - 1u;
        const bool fall = !kFocus || focus == 0u || (focus & all_robots) == all_robots;
        const long long qp0 = path_of(cd, n, q);
        // LDS of this tile, TS floats per timestep c: five rows of GSp floats over the
        // sphere slots (16 per group, unused slots padded) -- x, y, z relative to the
        // team's origin, radius (0 marks padding), w = |p|^2 - r^2.  The FK frames of
        // the timestep take its last 12 F floats, past the x, y, z rows, until the
        // radius and w rows are written over them.
        const int GS = tm->GS;
        const int GSp = tm->GSp;
        const int TS = tm->TS;
        const int fr_off = TS - 12 * F;
        float* sp = reinterpret_cast<float*>(dyn);                      // [C][TS]

        // --- FP32 forward kinematics.  First each joint's transform, one lane per
        // (timestep, joint), into the start of the timestep's slice (the x, y, z rows,
        // written only later); then the chains, one lane per (timestep, robot, frame
        // row), into the frames at the slice's tail.
        const int J = tm->J;
        for (int idx = tid; idx < nv * J; idx += WG) {
            const int c = idx / J;
            const int jg = idx - c * J;
            joint_matrix32(tm, cd, qp0, jg, s_t[c], reinterpret_cast<float4*>(sp + (long long)c * TS) + jg * 3);
        }
        __syncthreads();
        for (int idx = tid; idx < nv * n * 3; idx += WG) {
            const int c = idx / (3 * n);
            const int rr = idx - c * 3 * n;
            const int r = rr / 3;
            chain_row32(tm, r, rr - 3 * r, reinterpret_cast<const float4*>(sp + (long long)c * TS),
                        reinterpret_cast<float4*>(sp + (long long)c * TS + fr_off) + tm->r_frame_off[r] * 3);
        }
        __syncthreads();

        // --- sphere records, slot-major: lane idx keeps slot idx mod GS over the
        // tile's timesteps c0, c0 + cstep, ... (c0 = idx / GS), so a slot's frame
        // index and local centre are loaded once per tile.
        const int cstep = GS < WG ? WG / GS : 1;
        const int span = cstep * GS;
        constexpr int kRec = 4;
        if (GS <= WG && nv <= kRec * cstep) {
            // one pass when every lane holds at most kRec records: the centres go out
            // at once, w = |p|^2 - r^2 waits in registers until no lane reads the frames
            // that the radius and w rows overwrite
            const bool in = tid < span;
            const int c0 = in ? tid / GS : 0;
            const int s = tid - c0 * GS;
            const int fs = in ? tm->slot_frame[s] : -1;
            const float4 L = in ? tm->slot_local[s] : make_float4(0.f, 0.f, 0.f, 0.f);
            float wv[kRec];
            float r2max = 0.f;
#pragma unroll
            for (int m = 0; m < kRec; ++m) {
                const int c = c0 + m * cstep;
                wv[m] = kFar;
                if (in && c < nv) {
                    float x = 0.f, y = 0.f, z = 0.f;
                    if (fs >= 0) {
                        const float4 X = place32(reinterpret_cast<const float4*>(sp + c * TS + fr_off) + fs * 3, L);
                        x = X.x;
                        y = X.y;
                        z = X.z;
                    }
                    float* row = sp + c * TS + s;
                    row[0] = x;
                    row[GSp] = y;
                    row[2 * GSp] = z;
                    if (L.w > 0.f) {
                        const float d2 = fmaf(x, x, fmaf(y, y, z * z));
                        wv[m] = fmaf(-L.w, L.w, d2);
                        r2max = fmaxf(r2max, d2);
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < kRec; ++m) {
                const int c = c0 + m * cstep;
                if (in && c < nv) {
                    float* row = sp + c * TS + s;
                    row[3 * GSp] = L.w;
                    row[4 * GSp] = wv[m];
                }
            }
            r2max = wave_max_f32(r2max);
            if (lane == 0) atomicMax(&s_rho2, __float_as_uint(r2max));
            __syncthreads();
        } else {
            // First the centres relative to the team origin (padding slots at the origin) ...
            for (int idx = tid; idx < span; idx += WG) {
                const int c0 = idx / GS;
                const int s = idx - c0 * GS;
                const int fs = tm->slot_frame[s];
                const float4 L = tm->slot_local[s];
                for (int c = c0; c < nv; c += cstep) {
                    float x = 0.f, y = 0.f, z = 0.f;
                    if (fs >= 0) {
                        const float4 X = place32(reinterpret_cast<const float4*>(sp + (long long)c * TS + fr_off) + fs * 3, L);
                        x = X.x;
                        y = X.y;
                        z = X.z;
                    }
                    float* row = sp + (long long)c * TS + s;
                    row[0] = x;
                    row[GSp] = y;
                    row[2 * GSp] = z;
                }
            }
            __syncthreads();

            // ... then, over the frames, the radius and w = |p|^2 - r^2 rows (radius 0 and
            // w far away for padding)
            {
                float r2max = 0.f;
                for (int idx = tid; idx < span; idx += WG) {
                    const int c0 = idx / GS;
                    const int s = idx - c0 * GS;
                    const float r = tm->slot_local[s].w;
                    for (int c = c0; c < nv; c += cstep) {
                        float* row = sp + (long long)c * TS + s;
                        float w = kFar;
                        if (r > 0.f) {
                            const float x = row[0], y = row[GSp], z = row[2 * GSp];
                            const float d2 = fmaf(x, x, fmaf(y, y, z * z));
                            w = fmaf(-r, r, d2);
                            r2max = fmaxf(r2max, d2);
                        }
                        row[3 * GSp] = r;
                        row[4 * GSp] = w;
                    }
                }
                r2max = wave_max_f32(r2max);
                if (lane == 0) atomicMax(&s_rho2, __float_as_uint(r2max));
            }
            __syncthreads();
        }

        // The obstacle phase and the pair phase, in the call's order: early-terminating
        // MV may run the pairs first (MRV_PAIRS_FIRST), so that their hits end a tile
        // before costly obstacle tests; exhaustive MV and FFC keep a fixed order.
        auto env_phase = [&]() {
            if (exhaustive) __builtin_amdgcn_s_setprio(2);
            // --- robot-obstacle tests (MV with environment checking): one lane per
            // (timestep, slot); obstacle parameters are wave-uniform scalar loads.
            if (do_env && epu) {
                CCall& cd = call_at();
                CTeam* tm = team_at(tpu);
                CEnv* env = env_at(epu);
                // the team origin in the environment's frame, rounded once from FP64
                const float3 off = make_float3((float)(tm->origin64[0] - env->origin64[0]),
                                               (float)(tm->origin64[1] - env->origin64[1]),
                                               (float)(tm->origin64[2] - env->origin64[2]));
                const int nch = (GS + kWave - 1) / kWave;
                const int ntask = nv * nch;
                float ro_max = 0.f;
                for (int o = 0; o < env->n_sph; ++o) ro_max = fmaxf(ro_max, cloadf(&env->sph32[o].w));
                // tasks wave, wave + kWaves, ... of this wave, one at a time, so that in
                // early-terminating calls a hit stops the wave before its next task
                const ObBoxes pre = PTS ? ObBoxes{} : ob_boxes(env, env->n_box + env->n_cyl, 0, lane);
                int task = wave;
                for (; task < ntask && !(!exhaustive && flag_read(&s_hit)); task += kWaves) {
                    const int tk[1] = { task };
                    env_tasks<1, PTS>(cd, tm, env, sp, tk, nch, ro_max, eps, exhaustive, q, focus, fall, s_t, &s_hit, c_env,
                                 &s_npt, lane, off, pre);
                }
            }

        };
        auto pair_phase = [&]() {
            if (exhaustive) __builtin_amdgcn_s_setprio(0);
            // --- sphere-pair tests as 16 x 16 blocks on the matrix cores.  For slots a
            // (rows, group ga) and b (columns, group gb) at one timestep,
            //   D(a, b) = w_a + w_b - 2 p_a.p_b - 2 r_a r_b = |p_a - p_b|^2 - (r_a + r_b)^2,
            // the K = 4 product by one MFMA with the accumulator preset to w_a, then a
            // column minimum plus w_b on the vector unit.  One task per group ga runs,
            // timestep by timestep, the self blocks of ga (MV with environment checking;
            // pairs outside the self list masked) and its blocks against every group of
            // the higher robots.  Lanes whose minimum lies within the bound's
            // uncertainty revisit their pairs directly.
            CCall& cd = call_at();
            CTeam* tm = team_at(tpu);
            // pair-prioritised order (early-terminating MV, MRV_PAIR_PRIORITY): a first pass
            // over the self blocks and the robot pairs whose bases are adjacent, the likeliest
            // to collide (paper §III-A), then, after a barrier and only if no collision is
            // known, a second pass over the other pairs
            const bool prio = kPrio && do_rr && (flags & MRV_PAIR_PRIORITY) != 0;
            for (int pass = 0; pass < (prio ? 2 : 1); ++pass) {
            if (pass > 0) {
                __syncthreads();                 // every wave reads the flag after the first pass
                if (flag_read(&s_hit)) break;
            }
            const bool do_self = do_env && tm->n_sblocks > 0 && pass == 0;
            if ((do_rr || do_self) && !(kMV && !exhaustive && flag_read(&s_hit))) {
                const float rho2 = __uint_as_float(s_rho2);
                const float rm = tm->r_max;
                const float u = 5.9604645e-8f;
                // |D_fp32 - D| <= 24 u (rho^2 + rm^2) for |p| <= rho, r <= rm: 4 u from each
                // of w_a and w_b, 12 u from the MFMA's four fused steps (partial sums up to
                // 3 (rho^2 + rm^2)), 4 u from adding w_b; 32 u leaves a margin
                const float e_err = 32.f * u * (rho2 + rm * rm) + 1.0e-30f;
                const float Rm = 2.f * rm;
                const float e_hi = e_err + fmaf(2.f * Rm, eps, eps * eps);
                const float e_lo = -(e_err + 2.f * Rm * eps);
                const int i16 = lane & 15;
                const int q4 = lane >> 4;
                for (int k = wave; k < G; k += kWaves) {
                    if (kMV && !exhaustive && flag_read(&s_hit)) break;
                    // the task's 32-byte record in one scalar load
                    const int8v tk = cload8(tm->gtask + 8 * k);
                    const int ga = tk[0];
                    const int ra = tk[1];
                    const bool a_in = fall || ((focus >> ra) & 1u);     // ga's robot in focus
                    const int sb0 = do_self && a_in ? tk[2] : 0;
                    const int sb1 = do_self && a_in ? tk[3] : 0;
                    const bool higher_in = ra + 1 < 32 && (focus >> (ra + 1)) != 0u;   // a higher robot in focus
                    const int gs = do_rr && (a_in || higher_in) ? tk[4] : G;
                    const unsigned long long rr_tests = do_rr && a_in && !prio ? (unsigned long long)tk[5] : 0ull;
                    const unsigned long long self_tests = do_self && a_in ? (unsigned long long)tk[6] : 0ull;
                    // spheres of group ga, for the test counts of a robot outside the focus set
                    const int ga_n = a_in && !prio ? 0 : cload(reinterpret_cast<const int*>(tm->g_range) + 2 * ga + 1) -
                                                         cload(reinterpret_cast<const int*>(tm->g_range) + 2 * ga);
                    if (sb0 == sb1 && gs >= G) continue;
                    if constexpr (kSelfInner) {
                        __builtin_amdgcn_s_setprio(1);
                        // exhaustive MV: the self blocks of ga for up to kSI timesteps at a time,
                        // each block's record loaded once and its MFMAs independent
                        if (sb0 < sb1) {
                            for (int c0 = 0; c0 < nv; c0 += kSI) {
                                float best[kSI], aop[kSI];
                                int row[kSI];
#pragma unroll
                                for (int i = 0; i < kSI; ++i) {
                                    best[i] = 3.0e38f;
                                    // past the tile's last timestep a slot repeats that timestep
                                    // (its result is dropped below), so the blocks carry no branch
                                    // and their MFMAs issue back to back
                                    row[i] = min(c0 + i, nv - 1) * TS;
                                    aop[i] = -2.f * sp[row[i] + q4 * GSp + ga * 16 + i16];
                                }
                                for (int sb = sb0; sb < sb1; ++sb) {
                                    // the block's 64-byte record (column group, lane masks) in one load
                                    const int16v rec = cload16(tm->sblocks + 16 * sb);
                                    const int gb = rec[1];
                                    const unsigned long long m0 = u64_of(rec[8], rec[9]), m1 = u64_of(rec[10], rec[11]),
                                                             m2 = u64_of(rec[12], rec[13]), m3 = u64_of(rec[14], rec[15]);
#pragma unroll
                                    for (int i = 0; i < kSI; ++i) {
                                        const float* base = sp + row[i];
                                        const float4 cw = *reinterpret_cast<const float4*>(base + 4 * GSp + ga * 16 + 4 * q4);
                                        const floatx4 acc = { lane_select(m0, cw.x, kFar), lane_select(m1, cw.y, kFar),
                                                              lane_select(m2, cw.z, kFar), lane_select(m3, cw.w, kFar) };
                                        const float bop = base[q4 * GSp + gb * 16 + i16];
                                        const float wb = base[4 * GSp + gb * 16 + i16];
                                        const floatx4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[i], bop, acc, 0, 0, 0);
                                        best[i] = block_min(d, wb, best[i]);
                                    }
                                }
                                c_self += self_tests * (unsigned long long)min(kSI, nv - c0);
                                // common case first: no lane within the band at any of the timesteps
                                // (a repeated timestep's minimum equals its original's)
                                float bmin = best[0];
#pragma unroll
                                for (int i = 1; i < kSI; ++i) bmin = fminf(bmin, best[i]);
                                if (!__ballot(bmin < e_hi)) continue;
#pragma unroll
                                for (int i = 0; i < kSI; ++i) {
                                    if (c0 + i < nv) {
                                        const int t = s_t[c0 + i];
                                        const float* base = sp + (long long)(c0 + i) * TS;
                                        bool hit = false;
                                        const bool unsure = best[i] < e_hi && !(best[i] < e_lo);
                                        if (__ballot(best[i] < e_hi)) hit = best[i] < e_lo;
                                        if (__ballot(unsure) && !__ballot(hit) && unsure) {
                                            for (int sb = sb0; sb < sb1 && !hit; ++sb) {
                                                const int gb = cload(tm->sblocks + 16 * sb + 1);
                                                hit = direct_block(cd, tm, base, GSp, ga, gb, lane, sb_masks(tm, sb), eps, q, t,
                                                                   RK_SELF, 0u, &s_hit, &s_key, true);
                                            }
                                        }
                                        if (__ballot(hit) && lane == 0) s_hit = 1;
                                    }
                                }
                            }
                        }
                        if (gs >= G) continue;
                        __builtin_amdgcn_s_setprio(0);
                    }
                    for (int c = 0; c < nv; ++c) {
                        const int t = s_t[c];
                        if (kMV) {
                            if (!exhaustive && flag_read(&s_hit)) break;
                        } else if (!exhaustive) {
                            const unsigned known = flag_read(&s_key);
                            if (known != 0xFFFFFFFFu && known < (unsigned)t * (unsigned)tm->P) break;
                        }
                        c_rr += rr_tests;
                        if (!kSelfInner) c_self += self_tests;
                        const float* base = sp + (long long)c * TS;
                        const float aop = -2.f * base[q4 * GSp + ga * 16 + i16];
                        const float4 cw = *reinterpret_cast<const float4*>(base + 4 * GSp + ga * 16 + 4 * q4);
                        bool found = false;

                        // self blocks of ga
                        if (!kSelfInner && sb0 < sb1) {
                            float best = 3.0e38f;
                            for (int sb = sb0; sb < sb1; ++sb) {
                                const int16v rec = cload16(tm->sblocks + 16 * sb);
                                const int gb = rec[1];
                                const floatx4 acc = { lane_select(u64_of(rec[8], rec[9]), cw.x, kFar), lane_select(u64_of(rec[10], rec[11]), cw.y, kFar),
                                                      lane_select(u64_of(rec[12], rec[13]), cw.z, kFar), lane_select(u64_of(rec[14], rec[15]), cw.w, kFar) };
                                const float bop = base[q4 * GSp + gb * 16 + i16];
                                const float wb = base[4 * GSp + gb * 16 + i16];
                                const floatx4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bop, acc, 0, 0, 0);
                                best = block_min(d, wb, best);
                            }
                            // common case first: every pair of the lane clear beyond the band
                            if (__ballot(best < e_hi)) {
                                bool hit = best < e_lo;
                                const bool unsure = !hit && best < e_hi;
                                if (!__ballot(hit) && __ballot(unsure) && unsure) {
                                    for (int sb = sb0; sb < sb1 && !hit; ++sb) {
                                        const int gb = cload(tm->sblocks + 16 * sb + 1);
                                        const unsigned long long* mk = sb_masks(tm, sb);
                                        hit = direct_block(cd, tm, base, GSp, ga, gb, lane, mk, eps, q, t, RK_SELF, 0u, &s_hit, &s_key, true);
                                    }
                                }
                                if (__ballot(hit)) {
                                    found = true;
                                    if (lane == 0) s_hit = 1;
                                }
                            }
                        }

                        // robot-robot blocks against the higher robots
                        if (gs < G && !(found && !exhaustive)) {
                            const floatx4 acc = { cw.x, cw.y, cw.z, cw.w };
                            // the lane's minimum of D over column groups [g0, g1)
                            auto blocks_min = [&](int g0, int g1) {
                                float best = 3.0e38f;
                                int g = g0;
                                for (; g + 4 <= g1; g += 4) {
                                    float bop[4], wb[4];
                                    floatx4 d[4];
#pragma unroll
                                    for (int v = 0; v < 4; ++v) {
                                        bop[v] = base[q4 * GSp + (g + v) * 16 + i16];
                                        wb[v] = base[4 * GSp + (g + v) * 16 + i16];
                                    }
#pragma unroll
                                    for (int v = 0; v < 4; ++v) d[v] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bop[v], acc, 0, 0, 0);
                                    best = fminf(best, fminf(fminf(col_min(d[0], wb[0]), col_min(d[1], wb[1])),
                                                             fminf(col_min(d[2], wb[2]), col_min(d[3], wb[3]))));
                                }
                                for (; g < g1; ++g) {
                                    const float bop = base[q4 * GSp + g * 16 + i16];
                                    const float wb = base[4 * GSp + g * 16 + i16];
                                    const floatx4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bop, acc, 0, 0, 0);
                                    best = block_min(d, wb, best);
                                }
                                return best;
                            };
                            // FFC with two or more higher robots: one sweep over all their groups
                            // first; the robots run one by one (each pair its own key) only where
                            // a lane of the sweep comes within the band.  The blocks' values are
                            // the same in both, so a sweep clear of the band clears every pair.
                            bool near_any = true;
                            if constexpr (!kMV)
                                if (ra + 2 < n) near_any = __ballot(blocks_min(gs, G) < e_hi) != 0ull;
                            // MV: all higher robots in one sweep, unless ga's robot is outside the
                            // focus set; then robot by robot, over those in it
                            const bool sweep = kMV && a_in && !prio;
                            const int rb_end = sweep ? ra + 2 : n;
                            const unsigned pri = prio ? (unsigned)cload(reinterpret_cast<const int*>(tm->r_pri) + ra) : 0u;
                            for (int rb = ra + 1; near_any && rb < rb_end; ++rb) {
                                if (!a_in && !((focus >> rb) & 1u)) continue;
                                if (prio && (((pri >> rb) & 1u) != 0u) != (pass == 0)) continue;
                                const int g0 = sweep ? gs : cload(tm->r_group_off + rb);
                                const int g1 = sweep ? G : cload(tm->r_group_off + rb + 1);
                                if (!a_in || prio)
                                    c_rr += (unsigned long long)ga_n *
                                            (unsigned)(cload(tm->r_sphere_off + rb + 1) - cload(tm->r_sphere_off + rb));
                                const unsigned key = kMV ? 0u : (unsigned)t * (unsigned)tm->P + pair_index(ra, rb, n);
                                if (!kMV && !exhaustive && key >= flag_read(&s_key)) break;
                                const float best = blocks_min(g0, g1);
                                // common case first: every pair of the lane clear beyond the band
                                if (!__ballot(best < e_hi)) continue;
                                bool hit = best < e_lo;
                                const bool unsure = !hit && best < e_hi;
                                if (!__ballot(hit) && __ballot(unsure) && unsure) {
                                    for (int gg = g0; gg < g1 && !hit; ++gg)
                                        hit = direct_block(cd, tm, base, GSp, ga, gg, lane, nullptr, eps, q, t, RK_RR, key,
                                                           &s_hit, &s_key, kMV);
                                }
                                if (__ballot(hit)) {
                                    found = true;
                                    if (lane == 0) {
                                        if (kMV) s_hit = 1;
                                        else atomicMin(&s_key, key);
                                    }
                                    // FFC: higher robots give larger keys; MV robot by robot: one
                                    // hit decides
                                    if (!exhaustive && (!kMV || !sweep)) break;
                                }
                            }
                        }
                        // FFC: this group's later timesteps give larger keys
                        if (!kMV && found && !exhaustive) break;
                    }
                }
            }
            }

        };
        if constexpr (KIND == 0 || KIND == 2) {
            const bool pairs_first = (flags & MRV_PAIRS_FIRST) != 0;
            for (int ph = 0; ph < 2; ++ph) {
                if ((ph == 0) != pairs_first) env_phase();
                else pair_phase();
            }
        } else {
            env_phase();
            pair_phase();
        }

        __syncthreads();
    }

    if (lane == 0) {
        if (c_rr) atomicAdd(&cd.stats[ST_RR_TESTS], c_rr);
        if (c_self) atomicAdd(&cd.stats[ST_SELF_TESTS], c_self);
    }
    if (c_env) atomicAdd(&cd.stats[ST_ENV_TESTS], (unsigned long long)c_env);
    if (tid == 0) {
        atomicAdd(&cd.stats[ST_TILES_RUN], s_nrun);
        atomicAdd(&cd.stats[ST_TILES_SKIPPED], s_nskip);
        atomicAdd(&cd.stats[ST_STATES_EVAL], s_nstates);
        if (s_npt) atomicAdd(&cd.stats[ST_PT_TESTS], s_npt);
    }
}

// FP32 sphere centres of requested (query, timestep) states, computed by the same
// device code as the validation kernel (relative to the team origin), then moved
// to the world frame by one FP32 addition of the origin.  One workgroup per state;
// LDS holds the frames of one timestep.
__global__ void k_spheres(CallDev cd, const int* st_q, const int* st_t, int n_states, float4* out, int S_out)
{
    extern __shared__ float4 frames[];
    for (int k = blockIdx.x; k < n_states; k += gridDim.x) {
        const int q = st_q[k];
        const TeamDev& tm = *team_of(cd, q);
        const long long p0 = path_of(cd, tm.n_robots, q);
        // the joint transforms first, the frames after them (the same two steps as
        // the validation kernel)
        float4* fr = frames + tm.J * 3;
        for (int jg = threadIdx.x; jg < tm.J; jg += blockDim.x) joint_matrix32(&tm, cd, p0, jg, st_t[k], frames + jg * 3);
        __syncthreads();
        for (int i = threadIdx.x; i < tm.n_robots * 3; i += blockDim.x)
            chain_row32(&tm, i / 3, i % 3, frames, fr + tm.r_frame_off[i / 3] * 3);
        __syncthreads();
        for (int s = threadIdx.x; s < tm.S; s += blockDim.x) {
            const float4 X = place32(fr + tm.s_slot[s] * 3, tm.s_local32[s]);
            out[(long long)k * S_out + s] = make_float4(X.x + tm.origin[0], X.y + tm.origin[1], X.z + tm.origin[2], X.w);
        }
        __syncthreads();
    }
}

// FP64 re-evaluation of the near-contact tests the validation kernel queued; a
// record whose outcome the answer no longer depends on is skipped.
__global__ void k_recheck(CallDev cd)
{
    const EnvDev none{};
    const unsigned n = min(*reinterpret_cast<const unsigned*>(cd.ctrl + 2), (unsigned)cd.gq_cap);
    if (blockIdx.x == 0 && threadIdx.x == 0) cd.stats[ST_RECHECKS] = n;
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int4 r0 = cd.gq[i];
        const int q = r0.x, t = r0.y & 0xffffff, kind = r0.y >> 24, a = r0.z, b = r0.w;
        const TeamDev& tm = *team_of(cd, q);
        const EnvDev* ep = env_of(cd, q);
        const unsigned key = cd.kind == 0 ? 0u
                           : (unsigned)t * (unsigned)tm.P + pair_index(tm.s_robot[a], tm.s_robot[b], tm.n_robots);
        const unsigned w = load_word(cd.word + q);
        if (cd.kind == 0 ? w != 0u : key >= w) continue;        // decided already
        if (!recheck64(tm, ep ? *ep : none, cd, q, t, kind, a, b)) continue;
        if (cd.kind == 0) atomicOr(cd.word + q, 1u);
        else atomicMin(cd.word + q, key);
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

hipError_t launch_prepare(const CallDev& cd, hipStream_t stream)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, cd);
    if (cd.n_queries > 0) {
        const unsigned blocks = (unsigned)((cd.n_queries + 255) / 256);
        hipLaunchKernelGGL(k_query_info, dim3(blocks), dim3(256), 0, stream, cd);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(256), 0, stream, cd);
        hipLaunchKernelGGL(k_assign, dim3(blocks), dim3(256), 0, stream, cd);
    }
    return hipGetLastError();
}

namespace {
template <int KIND, bool PTS>
hipError_t launch_one(const CallDev& cd, int grid, hipStream_t stream)
{
    // allow dynamic LDS beyond 64 KiB (once per instantiation and process)
    static const hipError_t lds_opt = hipFuncSetAttribute((const void*)k_validate<KIND, PTS>,
                                                          hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget - 1024);
    if (lds_opt != hipSuccess && cd.lds_bytes > 64 * 1024) return lds_opt;
    hipLaunchKernelGGL((k_validate<KIND, PTS>), dim3(grid), dim3(validate_wg(KIND)), (size_t)cd.lds_bytes, stream, cd);
    return hipGetLastError();
}

template <int KIND, bool PTS>
int occupancy_one(size_t lds_bytes)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_validate<KIND, PTS>, validate_wg(KIND), lds_bytes) != hipSuccess)
        return 0;
    return nb;
}
}  // namespace

hipError_t launch_validate(const CallDev& cd, int grid, hipStream_t stream)
{
    if (cd.n_queries == 0) return hipSuccess;
    const bool pts = cd.points != 0;
    switch (validate_variant(cd)) {
    case 1: return launch_one<1, false>(cd, grid, stream);
    case 2: return pts ? launch_one<2, true>(cd, grid, stream) : launch_one<2, false>(cd, grid, stream);
    case 3: return pts ? launch_one<3, true>(cd, grid, stream) : launch_one<3, false>(cd, grid, stream);
    case 4: return launch_one<4, false>(cd, grid, stream);
    case 5: return pts ? launch_one<5, true>(cd, grid, stream) : launch_one<5, false>(cd, grid, stream);
    default: return pts ? launch_one<0, true>(cd, grid, stream) : launch_one<0, false>(cd, grid, stream);
    }
}

hipError_t launch_finalize(const CallDev& cd, hipStream_t stream)
{
    if (cd.n_queries == 0) return hipSuccess;
    hipLaunchKernelGGL(k_recheck, dim3(256), dim3(256), 0, stream, cd);
    const unsigned blocks = (unsigned)((cd.n_queries + 255) / 256);
    hipLaunchKernelGGL(k_finalize, dim3(blocks), dim3(256), 0, stream, cd);
    return hipGetLastError();
}

hipError_t launch_spheres(const CallDev& cd, const int* st_q, const int* st_t, int n_states, float4* out, int S,
                          int n_mats, hipStream_t stream)
{
    if (n_states <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min(n_states, 4096);
    // LDS: the joint transforms and the frames of one timestep, 48 bytes each
    hipLaunchKernelGGL(k_spheres, dim3(blocks), dim3(64), (size_t)n_mats * 48, stream, cd, st_q, st_t, n_states, out, S);
    return hipGetLastError();
}

}  // namespace mrv

// The fixed scratch of mrv_mv_device_noalloc (layout in mrv_internal.hpp).  Each
// device holds its own copy from module load until the process ends.  Host code
// never passes this name to a kernel: it stands for no device address there.
// Kernels get the address that noalloc_scratch_setup looked up for the device.
static __device__ __align__(256) unsigned char scratch[mrv::kNoAllocScratchBytes];

namespace mrv {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;       // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void* noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

int validate_blocks_per_cu(int kind, bool points, size_t lds_bytes)
{
    int nb = 0;
    switch (kind) {
    case 1: nb = occupancy_one<1, false>(lds_bytes); break;
    case 2: nb = points ? occupancy_one<2, true>(lds_bytes) : occupancy_one<2, false>(lds_bytes); break;
    case 3: nb = points ? occupancy_one<3, true>(lds_bytes) : occupancy_one<3, false>(lds_bytes); break;
    case 4: nb = occupancy_one<4, false>(lds_bytes); break;
    case 5: nb = points ? occupancy_one<5, true>(lds_bytes) : occupancy_one<5, false>(lds_bytes); break;
    default: nb = points ? occupancy_one<0, true>(lds_bytes) : occupancy_one<0, false>(lds_bytes); break;
    }
    return nb < 1 ? 1 : nb;
}

}  // namespace mrv
