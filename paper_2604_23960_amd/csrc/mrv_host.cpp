// Host runtime of libmrv: context, resident teams and environments, input
// validation, scratch management and the MV/FFC call pipeline.  The C ABI is
// declared in include/mrv.h; every exported function catches everything and
// reports through mrv_last_error().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mrv.h"
#include "mrv_internal.hpp"
#include "mrv_runtime.hpp"

using namespace mrv;

namespace {

thread_local std::string g_err;

mrv_status fail(mrv_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

// Packs host arrays into one device allocation, 256-byte aligned pieces.
struct Packer {
    std::vector<unsigned char> bytes;
    size_t add(const void* src, size_t n)
    {
        size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + std::max<size_t>(n, 1), 0);
        if (n) std::memcpy(bytes.data() + off, src, n);
        return off;
    }
    template <class T>
    size_t add(const std::vector<T>& v) { return add(v.data(), v.size() * sizeof(T)); }
};

struct TeamHost {
    TeamDev dev{};
    TeamDev* d_dev = nullptr;   // device copy of dev (inside dmem)
    void* dmem = nullptr;
    std::vector<int> dof;
    int max_dof = 0;
    mrv_tiling tiling[2][2] = {};   // [kind][exhaustive]
    int inflight = 0;
};

struct EnvHost {
    EnvDev dev{};
    EnvDev* d_dev = nullptr;    // device copy of dev (inside dmem)
    void* dmem = nullptr;
    int inflight = 0;
};

}  // namespace


namespace {

size_t lds_per_t(const TeamHost& tm);
int default_chunk(const TeamHost& tm, int kind, int exhaustive);
inline int mode_of(uint32_t flags) { return (flags & MRV_EXHAUSTIVE) ? 1 : 0; }
// Tiles per claim when the tiling leaves it automatic: one atomic counter serves
// only about 80 M claims/s (the arm workload's exhaustive MV was held to 31 ms by
// it at one tile per claim), so exhaustive calls take up to 4 and early-terminating
// ones, whose tiles often end at once on a known outcome, up to 8; the kernel takes
// fewer when the call has fewer than 8 claims' worth of tiles per workgroup.  Each
// tile still reads its query's outcome when it starts.  (Early-terminating MV on
// the arm workload 6.4 ms at 8 against 7.4 ms at 1, the cloud team's 47.6 ms
// against 78.5 ms; exhaustive calls gain nothing past 4.)
inline int default_claim(uint32_t flags) { return (flags & MRV_EXHAUSTIVE) ? 4 : 8; }

inline double sq(double v) { return v * v; }

// Finite and within MRV_MAX_COORD (NaN fails the comparison).
bool bounded_all(const double* p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!(std::fabs(p[i]) <= MRV_MAX_COORD)) return false;
    return true;
}

}  // namespace

struct mrv_ctx_s {
    DevAlloc alloc;         // every device buffer of the context (caller arena or hipMalloc)
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    double eps = 1e-5;
    int n_cu = 0;
    int next_handle = 1;
    std::map<int, TeamHost> teams;
    std::map<int, EnvHost> envs;
    std::mutex handle_mu;   // guards teams/envs against the serving thread

    Scratch sc;             // scratch of the synchronous and device-array calls
    DevBuf in_begin, in_t, in_q, out_buf;
    DevBuf tune_desc;       // the autotuner's private team descriptor

    std::map<std::string, mrv_tiling> tune_cache;   // autotuned tilings by team/env shape

    std::unique_ptr<ServeLoop> serve;
    int max_inflight = 1024;
    size_t serve_bytes = 0;
    size_t recheck_records = mrv::Scratch::kGlobalRecheckCap;
};

struct mrv_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Scratch sc;
    int team = -1, env = -1, kind = 0;
};

namespace {

mrv_status guard(mrv_ctx ctx)
{
    if (!ctx) return fail(MRV_E_HANDLE, "null context");
    return MRV_OK;
}

void set_device(mrv_ctx ctx) { HIPCHK(hipSetDevice(ctx->device)); }

// ---------------------------------------------------------------------------
// teams

int build_team(mrv_ctx ctx, const mrv_robot_desc* robots, int n, TeamHost& out)
{
    if (!robots || n < 1 || n > MRV_MAX_ROBOTS)
        throw Err{MRV_E_INVALID, "team must have 1.." + std::to_string(MRV_MAX_ROBOTS) + " robots"};
    std::vector<int> r_nj(n), r_joint_off(n), r_sphere_off(n + 1, 0), r_frame_off(n);
    std::vector<float> base32(n * 12);
    std::vector<double> base64(n * 12);
    std::vector<int> j_type, j_robot;
    std::vector<float> j32;
    std::vector<double> j64;
    std::vector<int> s_robot, s_slot, s_lframe;
    std::vector<float> s_local32;
    std::vector<double> s_local64;
    std::vector<int> self_pairs;
    int F = 0, S = 0, max_dof = 0;
    for (int r = 0; r < n; ++r) {
        const mrv_robot_desc& R = robots[r];
        const std::string who = "robot " + std::to_string(r) + ": ";
        if (R.n_joints < 0 || R.n_joints > MRV_MAX_JOINTS)
            throw Err{MRV_E_INVALID, who + "n_joints out of range"};
        if (R.n_joints > 0 && (!R.joint_type || !R.joint_fixed))
            throw Err{MRV_E_INVALID, who + "null joint arrays"};
        if (R.n_spheres < 1 || R.n_spheres > MRV_MAX_SPHERES_PER_ROBOT)
            throw Err{MRV_E_INVALID, who + "n_spheres out of range"};
        if (!R.sphere_frame || !R.sphere_xyzr) throw Err{MRV_E_INVALID, who + "null sphere arrays"};
        if (R.n_self_pairs < 0 || (R.n_self_pairs > 0 && !R.self_pairs))
            throw Err{MRV_E_INVALID, who + "bad self pair list"};
        if (!bounded_all(R.base, 12)) throw Err{MRV_E_INVALID, who + "base not finite or beyond MRV_MAX_COORD"};
        if (R.n_joints > 0 && !bounded_all(R.joint_fixed, (size_t)R.n_joints * 12))
            throw Err{MRV_E_INVALID, who + "joint transform not finite or beyond MRV_MAX_COORD"};
        if (!bounded_all(R.sphere_xyzr, (size_t)R.n_spheres * 4))
            throw Err{MRV_E_INVALID, who + "sphere not finite or beyond MRV_MAX_COORD"};
        r_nj[r] = R.n_joints;
        max_dof = std::max(max_dof, R.n_joints);
        r_joint_off[r] = (int)j_type.size();
        r_frame_off[r] = F;
        F += R.n_joints + 1;
        for (int i = 0; i < 12; ++i) {
            base32[r * 12 + i] = (float)R.base[i];   // translations replaced below, relative to the origin
            base64[r * 12 + i] = R.base[i];
        }
        for (int j = 0; j < R.n_joints; ++j) {
            int jt = R.joint_type[j];
            if (jt < MRV_REV_Z || jt > MRV_PRI_Z) throw Err{MRV_E_INVALID, who + "unknown joint type"};
            j_type.push_back(jt);
            j_robot.push_back(r);
            for (int i = 0; i < 12; ++i) {
                j32.push_back((float)R.joint_fixed[j * 12 + i]);
                j64.push_back(R.joint_fixed[j * 12 + i]);
            }
        }
        for (int s = 0; s < R.n_spheres; ++s) {
            int f = R.sphere_frame[s];
            if (f < 0 || f > R.n_joints) throw Err{MRV_E_INVALID, who + "sphere frame out of range"};
            double rad = R.sphere_xyzr[s * 4 + 3];
            if (!(rad > 0.0)) throw Err{MRV_E_INVALID, who + "sphere radius must be > 0"};
            s_robot.push_back(r);
            s_slot.push_back(r_frame_off[r] + f);
            s_lframe.push_back(f);
            for (int i = 0; i < 4; ++i) {
                s_local32.push_back((float)R.sphere_xyzr[s * 4 + i]);
                s_local64.push_back(R.sphere_xyzr[s * 4 + i]);
            }
        }
        for (int p = 0; p < R.n_self_pairs; ++p) {
            int a = R.self_pairs[2 * p], b = R.self_pairs[2 * p + 1];
            if (a < 0 || b < 0 || a >= R.n_spheres || b >= R.n_spheres || a == b)
                throw Err{MRV_E_INVALID, who + "self pair index out of range"};
            self_pairs.push_back(S + a);
            self_pairs.push_back(S + b);
        }
        S += R.n_spheres;
        r_sphere_off[r + 1] = S;
    }
    if (S > MRV_MAX_TEAM_SPHERES) throw Err{MRV_E_INVALID, "team has too many spheres"};
    // sphere groups: up to 16 consecutive spheres of one robot
    std::vector<int> s_group(S), r_group_off(n + 1, 0), g_range;
    int G = 0;
    for (int r = 0; r < n; ++r) {
        r_group_off[r] = G;
        for (int b = r_sphere_off[r]; b < r_sphere_off[r + 1]; b += 16) {
            const int e = std::min(b + 16, r_sphere_off[r + 1]);
            for (int s2 = b; s2 < e; ++s2) s_group[s2] = G;
            g_range.push_back(b);
            g_range.push_back(e);
            ++G;
        }
    }
    r_group_off[n] = G;
    // slots: 16 per group, unused ones padded, so a group is one 16-wide MFMA operand
    const int GS = G * 16;
    std::vector<int> slot_sphere(GS, -1), sphere_slot(S), slot_frame(GS, -1);
    std::vector<float> slot_local((size_t)GS * 4, 0.f);
    for (int g = 0; g < G; ++g)
        for (int s2 = g_range[2 * g]; s2 < g_range[2 * g + 1]; ++s2) {
            const int sl = g * 16 + (s2 - g_range[2 * g]);
            slot_sphere[sl] = s2;
            sphere_slot[s2] = sl;
            slot_frame[sl] = s_slot[s2];
            for (int i = 0; i < 4; ++i) slot_local[(size_t)sl * 4 + i] = s_local32[(size_t)s2 * 4 + i];
        }
    // self blocks: for each pair of groups (ga <= gb) holding self pairs, one lane
    // mask per accumulator register r: bit l set when the pair (row 4 (l / 16) + r
    // of ga, column l % 16 of gb) is in the list (each unordered pair once)
    std::map<std::pair<int, int>, std::array<uint64_t, 4>> blocks;
    for (size_t p = 0; p < self_pairs.size(); p += 2) {
        int sa = sphere_slot[self_pairs[p]], sb = sphere_slot[self_pairs[p + 1]];
        if (sa > sb) std::swap(sa, sb);
        const int row = sa % 16, col = sb % 16;
        auto& m = blocks.emplace(std::make_pair(sa / 16, sb / 16), std::array<uint64_t, 4>{0, 0, 0, 0}).first->second;
        m[row & 3] |= 1ull << (16 * (row >> 2) + col);
    }
    // 64-byte records: row group, column group, pairs, robot, 4 unused ints, then the
    // four lane masks
    std::vector<int> sblocks;
    int n_self_unique = 0;
    for (const auto& kv : blocks) {
        int cnt = 0;
        for (uint64_t m : kv.second) cnt += __builtin_popcountll(m);
        int rec[16] = { kv.first.first, kv.first.second, cnt, s_robot[g_range[2 * kv.first.first]], 0, 0, 0, 0 };
        std::memcpy(rec + 8, kv.second.data(), 4 * sizeof(uint64_t));
        sblocks.insert(sblocks.end(), rec, rec + 16);
        n_self_unique += cnt;
    }
    // pair tasks, one per group ga: its self blocks [sb0, sb1) (sorted by ga) and the
    // groups of every higher robot from gstart on; 8 ints each
    std::vector<int> gtask;
    {
        size_t sbi = 0;
        const size_t nsb = sblocks.size() / 16;
        for (int g = 0; g < G; ++g) {
            const int r = s_robot[g_range[2 * g]];
            const int sb0 = (int)sbi;
            int self_tests = 0;
            while (sbi < nsb && sblocks[16 * sbi] == g) self_tests += sblocks[16 * sbi++ + 2];
            const int rec[8] = { g, r, sb0, (int)sbi, r_group_off[r + 1],
                                 (g_range[2 * g + 1] - g_range[2 * g]) * (S - r_sphere_off[r + 1]), self_tests, 0 };
            gtask.insert(gtask.end(), rec, rec + 8);
        }
        // Waves take the tasks round-robin (task k to wave k mod waves), so the tasks
        // are dealt heaviest first in a snake order over four waves: each wave gets a
        // like share of the blocks (a self block weighs 1.5 robot-robot blocks, a task
        // its own set-up one more), and eight waves see pairs of such rounds.
        std::vector<int> ord(G);
        std::vector<double> wt(G);
        for (int g = 0; g < G; ++g) {
            ord[g] = g;
            wt[g] = (G - gtask[8 * g + 4]) + 1.5 * (gtask[8 * g + 3] - gtask[8 * g + 2]) + 1.0;
        }
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return wt[a] > wt[b]; });
        std::vector<int> dealt(gtask.size());
        for (int i = 0; i < G; ++i) {
            const int round = i / 4, lane = i % 4;
            const int pos = 4 * round + ((round & 1) ? 3 - lane : lane);
            // a last, partial round keeps its tasks in the first positions it has
            const int last = std::min(G, 4 * round + 4) - 4 * round;
            const int p = (round & 1) && last < 4 ? 4 * round + (last - 1 - lane) : pos;
            std::copy(gtask.begin() + 8 * ord[i], gtask.begin() + 8 * ord[i] + 8, dealt.begin() + 8 * p);
        }
        gtask.swap(dealt);
    }
    float r_max = 0.f;
    for (int s2 = 0; s2 < S; ++s2) r_max = std::max(r_max, s_local32[s2 * 4 + 3]);
    long long rr_per_t = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            rr_per_t += (long long)(r_sphere_off[i + 1] - r_sphere_off[i]) * (r_sphere_off[j + 1] - r_sphere_off[j]);

    // team origin o: the centre of the bases' bounding box, rounded to an FP32 value
    // so that it is exact in both precisions.  The FP32 frames start from base
    // translations relative to o (subtracted in FP64, rounded once), so no FP32
    // value depends on where the team sits in the world.
    float origin32[3];
    double team_mag = 0.0;
    std::vector<float> r_mag(n);
    {
        double lo[3] = { 1e300, 1e300, 1e300 }, hi[3] = { -1e300, -1e300, -1e300 };
        for (int r = 0; r < n; ++r)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], base64[r * 12 + 4 * d + 3]);
                hi[d] = std::max(hi[d], base64[r * 12 + 4 * d + 3]);
            }
        double o[3];
        for (int d = 0; d < 3; ++d) {
            origin32[d] = (float)(0.5 * (lo[d] + hi[d]));
            o[d] = (double)origin32[d];
        }
        for (int r = 0; r < n; ++r)
            for (int d = 0; d < 3; ++d) base32[r * 12 + 4 * d + 3] = (float)(base64[r * 12 + 4 * d + 3] - o[d]);
        // magnitude bound of the FP32 coordinates relative to o: base offset, joint
        // translations and the farthest sphere centre plus radius, per robot
        for (int r = 0; r < n; ++r) {
            const double* b = base64.data() + r * 12;
            double m = std::sqrt(sq(b[3] - o[0]) + sq(b[7] - o[1]) + sq(b[11] - o[2]));
            for (int j = 0; j < r_nj[r]; ++j) {
                const double* F = j64.data() + (size_t)(r_joint_off[r] + j) * 12;
                m += std::sqrt(sq(F[3]) + sq(F[7]) + sq(F[11]));
            }
            double cmax = 0.0;
            for (int s2 = r_sphere_off[r]; s2 < r_sphere_off[r + 1]; ++s2) {
                const double* c = s_local64.data() + (size_t)s2 * 4;
                cmax = std::max(cmax, std::sqrt(sq(c[0]) + sq(c[1]) + sq(c[2])) + c[3]);
            }
            r_mag[r] = (float)(m + cmax);
            team_mag = std::max(team_mag, m + cmax);
        }
    }

    // prioritised robot pairs (MRV_PAIR_PRIORITY): bases adjacent, i.e. within 1.25 times
    // the smallest distance between two bases; none when every base coincides (the
    // pair order is then the plain one)
    std::vector<unsigned> r_pri(n, 0u);
    {
        double dmin = 1e300;
        auto bd = [&](int i, int j) {
            return std::sqrt(sq(base64[i * 12 + 3] - base64[j * 12 + 3]) + sq(base64[i * 12 + 7] - base64[j * 12 + 7]) +
                             sq(base64[i * 12 + 11] - base64[j * 12 + 11]));
        };
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) dmin = std::min(dmin, bd(i, j));
        if (dmin > 0.0 && dmin < 1e300)
            for (int i = 0; i < n; ++i)
                for (int j = i + 1; j < n; ++j)
                    if (bd(i, j) <= 1.25 * dmin) r_pri[i] |= 1u << j;
    }

    Packer pk;
    const size_t o_nj = pk.add(r_nj), o_jo = pk.add(r_joint_off), o_so = pk.add(r_sphere_off),
                 o_fo = pk.add(r_frame_off), o_b32 = pk.add(base32), o_b64 = pk.add(base64),
                 o_jt = pk.add(j_type), o_j32 = pk.add(j32), o_j64 = pk.add(j64), o_sr = pk.add(s_robot),
                 o_ss = pk.add(s_slot), o_sl = pk.add(s_lframe), o_l32 = pk.add(s_local32),
                 o_l64 = pk.add(s_local64), o_rt = pk.add(gtask), o_sg = pk.add(s_group),
                 o_gr = pk.add(g_range), o_rg = pk.add(r_group_off), o_ss2 = pk.add(slot_sphere),
                 o_sb = pk.add(sblocks), o_rm = pk.add(r_mag),
                 o_jr = pk.add(j_robot), o_sf = pk.add(slot_frame), o_slc = pk.add(slot_local),
                 o_pri = pk.add(r_pri);
    const TeamDev blank{};
    const size_t o_self = pk.add(&blank, sizeof(TeamDev));
    void* d = nullptr;
    d = ctx->alloc.alloc(pk.bytes.size());
    auto at = [&](size_t o) { return (unsigned char*)d + o; };
    TeamDev& t = out.dev;
    t.n_robots = n;
    t.S = S;
    t.F = F;
    t.n_self = n_self_unique;
    t.n_sblocks = (int)sblocks.size() / 16;
    t.GS = GS;
    t.GSp = GS + 16;
    t.J = (int)j_type.size();
    // a timestep's LDS slice holds, over one tile: the joint transforms (start) and
    // the frames (tail) during forward kinematics, then the x, y, z rows over the
    // transforms while the frames are read, then the radius and w rows over the frames
    t.TS = std::max({5 * t.GSp, 3 * t.GSp + 12 * F, 12 * (t.J + F)});
    t.P = n * (n - 1) / 2;
    t.max_dof = max_dof;
    t.G = G;
    t.r_max = r_max;
    for (int k = 0; k < 3; ++k) {
        t.origin[k] = origin32[k];
        t.origin64[k] = (double)origin32[k];
    }
    t.origin[3] = 0.f;
    t.mag = (float)team_mag;
    t.rr_tests_per_t = rr_per_t;
    t.s_group = (const int*)at(o_sg);
    t.g_range = (const int2*)at(o_gr);
    t.r_group_off = (const int*)at(o_rg);
    t.r_nj = (const int*)at(o_nj);
    t.r_joint_off = (const int*)at(o_jo);
    t.r_sphere_off = (const int*)at(o_so);
    t.r_frame_off = (const int*)at(o_fo);
    t.r_mag = (const float*)at(o_rm);
    t.r_base32 = (const float*)at(o_b32);
    t.r_base64 = (const double*)at(o_b64);
    t.j_type = (const int*)at(o_jt);
    t.j_robot = (const int*)at(o_jr);
    t.j_fixed32 = (const float*)at(o_j32);
    t.j_fixed64 = (const double*)at(o_j64);
    t.s_robot = (const int*)at(o_sr);
    t.s_slot = (const int*)at(o_ss);
    t.s_lframe = (const int*)at(o_sl);
    t.s_local32 = (const float4*)at(o_l32);
    t.s_local64 = (const double*)at(o_l64);
    t.gtask = (const int*)at(o_rt);
    t.slot_sphere = (const int*)at(o_ss2);
    t.slot_frame = (const int*)at(o_sf);
    t.r_pri = (const unsigned*)at(o_pri);
    t.slot_local = (const float4*)at(o_slc);
    t.sblocks = (const int*)at(o_sb);
    out.dmem = d;
    out.d_dev = (TeamDev*)at(o_self);
    out.dof = r_nj;
    out.max_dof = max_dof;
    t.lds_per_t = (int)lds_per_t(out);
    for (int k = 0; k < 2; ++k)
        for (int m = 0; m < 2; ++m) t.chunk[k][m] = default_chunk(out, k, m);
    std::memcpy(pk.bytes.data() + o_self, &t, sizeof(TeamDev));
    if (hipMemcpy(d, pk.bytes.data(), pk.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) {
        ctx->alloc.free(d);
        throw Err{MRV_E_DEVICE, "team upload failed"};
    }
    return 0;
}

// ---------------------------------------------------------------------------
// environments

void build_env(mrv_ctx ctx, const mrv_env_desc* e, EnvHost& out)
{
    if (!e) throw Err{MRV_E_INVALID, "null environment"};
    if (e->n_spheres < 0 || e->n_boxes < 0 || e->n_cyls < 0 || e->n_points < 0)
        throw Err{MRV_E_INVALID, "negative obstacle count"};
    if ((e->n_spheres && !e->spheres) || (e->n_boxes && !e->boxes) || (e->n_cyls && !e->cylinders) ||
        (e->n_points && !e->points))
        throw Err{MRV_E_INVALID, "null obstacle array"};
    if (e->n_spheres && !bounded_all(e->spheres, (size_t)e->n_spheres * 4)) throw Err{MRV_E_INVALID, "sphere obstacle not finite or beyond MRV_MAX_COORD"};
    if (e->n_boxes && !bounded_all(e->boxes, (size_t)e->n_boxes * 15)) throw Err{MRV_E_INVALID, "box not finite or beyond MRV_MAX_COORD"};
    if (e->n_cyls && !bounded_all(e->cylinders, (size_t)e->n_cyls * 8)) throw Err{MRV_E_INVALID, "cylinder not finite or beyond MRV_MAX_COORD"};
    if (e->n_points && !bounded_all(e->points, (size_t)e->n_points * 3)) throw Err{MRV_E_INVALID, "point not finite or beyond MRV_MAX_COORD"};
    if (!bounded_all(&e->point_radius, 1) || e->point_radius < 0) throw Err{MRV_E_INVALID, "bad point radius"};
    // Environment origin o: the centre of the bounding box of every obstacle centre
    // and point, rounded to an FP32 value.  Every FP32 coordinate of the environment
    // is taken relative to o in FP64 and rounded once.
    double o[3] = { 0.0, 0.0, 0.0 };
    {
        double lo[3] = { 1e300, 1e300, 1e300 }, hi[3] = { -1e300, -1e300, -1e300 };
        auto grow = [&](const double* c) {
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], c[k]);
                hi[k] = std::max(hi[k], c[k]);
            }
        };
        for (int i = 0; i < e->n_spheres; ++i) grow(e->spheres + i * 4);
        for (int i = 0; i < e->n_boxes; ++i) grow(e->boxes + i * 15);
        for (int i = 0; i < e->n_cyls; ++i) grow(e->cylinders + i * 8);
        for (long long i = 0; i < e->n_points; ++i) grow(e->points + i * 3);
        if (lo[0] <= hi[0])
            for (int k = 0; k < 3; ++k) o[k] = (double)(float)(0.5 * (lo[k] + hi[k]));
    }
    double env_mag = 0.0;      // largest |coordinate relative to o| of any obstacle part
    auto rel_norm = [&](const double* c) { return std::sqrt(sq(c[0] - o[0]) + sq(c[1] - o[1]) + sq(c[2] - o[2])); };
    std::vector<float> sph32;
    for (int i = 0; i < e->n_spheres; ++i) {
        const double* c = e->spheres + i * 4;
        if (c[3] < 0) throw Err{MRV_E_INVALID, "negative obstacle radius"};
        for (int k = 0; k < 3; ++k) sph32.push_back((float)(c[k] - o[k]));
        sph32.push_back((float)c[3]);
        env_mag = std::max(env_mag, rel_norm(c) + c[3]);
    }
    std::vector<float> box32;
    for (int i = 0; i < e->n_boxes; ++i) {
        const double* b = e->boxes + i * 15;
        const double* R = b + 3;
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                double dot = R[0 * 3 + a] * R[0 * 3 + c] + R[1 * 3 + a] * R[1 * 3 + c] + R[2 * 3 + a] * R[2 * 3 + c];
                if (std::fabs(dot - (a == c ? 1.0 : 0.0)) > 1e-9)
                    throw Err{MRV_E_INVALID, "box rotation is not orthonormal"};
            }
        if (b[12] < 0 || b[13] < 0 || b[14] < 0) throw Err{MRV_E_INVALID, "negative box half-extent"};
        // box frame coordinates p_k = (R^T)_k . x - (R^T (c - o))_k for x relative to o:
        // row k of R^T is column k of R
        float row[16];
        const double cr[3] = { b[0] - o[0], b[1] - o[1], b[2] - o[2] };
        for (int k = 0; k < 3; ++k) {
            row[4 * k + 0] = (float)R[0 * 3 + k];
            row[4 * k + 1] = (float)R[1 * 3 + k];
            row[4 * k + 2] = (float)R[2 * 3 + k];
            row[4 * k + 3] = (float)(-(R[0 * 3 + k] * cr[0] + R[1 * 3 + k] * cr[1] + R[2 * 3 + k] * cr[2]));
        }
        env_mag = std::max(env_mag, rel_norm(b) + std::sqrt(sq(b[12]) + sq(b[13]) + sq(b[14])));
        row[12] = (float)b[12];
        row[13] = (float)b[13];
        row[14] = (float)b[14];
        row[15] = 0.f;
        box32.insert(box32.end(), row, row + 16);
    }
    std::vector<float> cyl32;
    for (int i = 0; i < e->n_cyls; ++i) {
        const double* y = e->cylinders + i * 8;
        double nrm = y[3] * y[3] + y[4] * y[4] + y[5] * y[5];
        if (std::fabs(nrm - 1.0) > 1e-9) throw Err{MRV_E_INVALID, "cylinder axis is not a unit vector"};
        if (y[6] < 0 || y[7] < 0) throw Err{MRV_E_INVALID, "negative cylinder size"};
        for (int k = 0; k < 3; ++k) cyl32.push_back((float)(y[k] - o[k]));
        for (int k = 3; k < 8; ++k) cyl32.push_back((float)y[k]);
        env_mag = std::max(env_mag, rel_norm(y) + y[6] + y[7]);
    }
    // world-axis box of each box, then of each cylinder, in FP64, padded and rounded
    // outward to FP32: the kernel skips an obstacle whose box misses every sphere of
    // a slot row by more than the near band
    std::vector<float> bc_box;
    auto push_box = [&](const double* c, const double* ext) {
        float lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
        for (int k = 0; k < 3; ++k) {
            const double ck = c[k] - o[k];
            const double pad = 1e-7 * (1.0 + std::fabs(ck) + ext[k]);
            const double l = ck - ext[k] - pad, h = ck + ext[k] + pad;
            lo[k] = (float)l;
            if ((double)lo[k] > l) lo[k] = std::nextafter(lo[k], -HUGE_VALF);
            hi[k] = (float)h;
            if ((double)hi[k] < h) hi[k] = std::nextafter(hi[k], HUGE_VALF);
        }
        bc_box.insert(bc_box.end(), lo, lo + 4);
        bc_box.insert(bc_box.end(), hi, hi + 4);
    };
    for (int i = 0; i < e->n_boxes; ++i) {
        const double* b = e->boxes + i * 15;
        const double* R = b + 3;
        double ext[3];
        for (int k = 0; k < 3; ++k)
            ext[k] = std::fabs(R[k * 3 + 0]) * b[12] + std::fabs(R[k * 3 + 1]) * b[13] + std::fabs(R[k * 3 + 2]) * b[14];
        push_box(b, ext);
    }
    for (int i = 0; i < e->n_cyls; ++i) {
        const double* y = e->cylinders + i * 8;
        double ext[3];
        for (int k = 0; k < 3; ++k)
            ext[k] = std::fabs(y[3 + k]) * y[6] + y[7] * std::sqrt(std::max(0.0, 1.0 - y[3 + k] * y[3 + k]));
        push_box(y, ext);
    }
    // point cloud: uniform grid, points sorted by cell (x fastest)
    std::vector<float> pts32;
    std::vector<double> pts64;
    std::vector<int> cell_start(1, 0);
    float grid_lo[3] = {0, 0, 0};
    int dims[3] = {1, 1, 1};
    double cell = e->grid_cell > 0 ? e->grid_cell : 0.05;
    if (e->n_points > 0) {
        if (e->n_points > (1ll << 30)) throw Err{MRV_E_INVALID, "too many points"};
        // the grid in coordinates relative to o
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (long long i = 0; i < e->n_points; ++i) {
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], e->points[i * 3 + d] - o[d]);
                hi[d] = std::max(hi[d], e->points[i * 3 + d] - o[d]);
            }
            env_mag = std::max(env_mag, rel_norm(e->points + i * 3) + e->point_radius);
        }
        long long total = 1;
        for (int d = 0; d < 3; ++d) {
            dims[d] = (int)std::floor((hi[d] - lo[d]) / cell) + 1;
            total *= dims[d];
        }
        if (total > (1ll << 26)) throw Err{MRV_E_INVALID, "point grid too fine for the cloud extent"};
        for (int d = 0; d < 3; ++d) grid_lo[d] = (float)lo[d];
        const float inv = (float)(1.0 / cell);
        std::vector<int> cell_of(e->n_points);
        std::vector<int> count(total + 1, 0);
        for (long long i = 0; i < e->n_points; ++i) {
            int ci[3];
            for (int d = 0; d < 3; ++d) {
                // bin with the same FP32 arithmetic the kernel uses for its lookups
                int v = (int)std::floor(((float)(e->points[i * 3 + d] - o[d]) - grid_lo[d]) * inv);
                ci[d] = std::min(std::max(v, 0), dims[d] - 1);
            }
            cell_of[i] = (ci[2] * dims[1] + ci[1]) * dims[0] + ci[0];
            count[cell_of[i] + 1]++;
        }
        cell_start.assign(total + 1, 0);
        for (long long c = 0; c < total; ++c) cell_start[c + 1] = cell_start[c] + count[c + 1];
        std::vector<int> cursor(cell_start.begin(), cell_start.end() - 1);
        // FP32 points carry |p|^2 (of the FP32 coordinates, rounded once) for the
        // sphere-point blocks, and kPtsPad copies of the last point past the end, which
        // the blocks may read
        pts32.assign(((size_t)e->n_points + kPtsPad) * 4, 0.f);
        pts64.assign((size_t)e->n_points * 3, 0.0);
        for (long long i = 0; i < e->n_points; ++i) {
            int p = cursor[cell_of[i]]++;
            double n2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const float v = (float)(e->points[i * 3 + d] - o[d]);
                pts32[(size_t)p * 4 + d] = v;
                n2 += (double)v * (double)v;
                pts64[(size_t)p * 3 + d] = e->points[i * 3 + d];
            }
            pts32[(size_t)p * 4 + 3] = (float)n2;
        }
        for (size_t k = 0; k < (size_t)kPtsPad * 4; ++k)
            pts32[(size_t)e->n_points * 4 + k] = pts32[((size_t)e->n_points - 1) * 4 + k % 4];
    }
    std::vector<double> sph64(e->spheres, e->spheres + (size_t)e->n_spheres * 4);
    std::vector<double> box64(e->boxes, e->boxes + (size_t)e->n_boxes * 15);
    std::vector<double> cyl64(e->cylinders, e->cylinders + (size_t)e->n_cyls * 8);
    Packer pk;
    size_t o_s32 = pk.add(sph32), o_s64 = pk.add(sph64), o_b32 = pk.add(box32), o_b64 = pk.add(box64),
           o_c32 = pk.add(cyl32), o_c64 = pk.add(cyl64), o_p32 = pk.add(pts32), o_p64 = pk.add(pts64),
           o_cs = pk.add(cell_start), o_bc = pk.add(bc_box);
    const EnvDev blank{};
    const size_t o_self = pk.add(&blank, sizeof(EnvDev));
    void* d = nullptr;
    d = ctx->alloc.alloc(pk.bytes.size());
    auto at = [&](size_t o) { return (unsigned char*)d + o; };
    EnvDev& v = out.dev;
    v.n_sph = e->n_spheres;
    v.n_box = e->n_boxes;
    v.n_cyl = e->n_cyls;
    v.n_pts = e->n_points;
    v.sph32 = (const float4*)at(o_s32);
    v.sph64 = (const double*)at(o_s64);
    v.box32 = (const float*)at(o_b32);
    v.box64 = (const double*)at(o_b64);
    v.cyl32 = (const float*)at(o_c32);
    v.cyl64 = (const double*)at(o_c64);
    v.pts32 = (const float4*)at(o_p32);
    v.pts64 = (const double*)at(o_p64);
    v.cell_start = (const int*)at(o_cs);
    v.bc_box = (const float4*)at(o_bc);
    for (int k = 0; k < 3; ++k) {
        v.grid_lo[k] = grid_lo[k];
        v.grid_dim[k] = dims[k];
    }
    v.grid_cell = (float)cell;
    v.grid_inv = (float)(1.0 / cell);
    v.pt_radius = (float)e->point_radius;
    v.pt_radius64 = e->point_radius;
    for (int k = 0; k < 3; ++k) v.origin64[k] = o[k];
    v.mag = (float)env_mag;
    out.dmem = d;
    out.d_dev = (EnvDev*)at(o_self);
    std::memcpy(pk.bytes.data() + o_self, &v, sizeof(EnvDev));
    if (hipMemcpy(d, pk.bytes.data(), pk.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) {
        ctx->alloc.free(d);
        throw Err{MRV_E_DEVICE, "environment upload failed"};
    }
}

// ---------------------------------------------------------------------------
// calls

void check_paths_host(const TeamHost& tm, const mrv_paths* p)
{
    if (!p) throw Err{MRV_E_INVALID, "null paths"};
    if (p->n_queries < 0) throw Err{MRV_E_INVALID, "negative n_queries"};
    if (p->n_queries == 0) return;
    const int n = tm.dev.n_robots;
    if (!p->wp_begin || !p->wp_t || !p->wp_q) throw Err{MRV_E_INVALID, "null path array"};
    if (p->dof_stride < std::max(tm.max_dof, 1) && !(tm.max_dof == 0 && p->dof_stride >= 0))
        throw Err{MRV_E_INVALID, "dof_stride smaller than the team's largest dof"};
    const long long npaths = (long long)p->n_queries * n;
    if (p->wp_begin[0] != 0) throw Err{MRV_E_INVALID, "wp_begin[0] must be 0"};
    if (p->wp_begin[npaths] != p->n_wp) throw Err{MRV_E_INVALID, "wp_begin[last] must equal n_wp"};
    for (long long i = 0; i < npaths; ++i) {
        const long long b = p->wp_begin[i], e = p->wp_begin[i + 1];
        if (e <= b) throw Err{MRV_E_INVALID, "empty path (query " + std::to_string(i / n) + ")"};
        if (p->wp_t[b] != 0) throw Err{MRV_E_INVALID, "first waypoint time must be 0"};
        const int dof = tm.dof[i % n];
        for (long long w = b; w < e; ++w) {
            if (w > b && p->wp_t[w] <= p->wp_t[w - 1])
                throw Err{MRV_E_INVALID, "waypoint times must strictly increase"};
            for (int d = 0; d < dof; ++d)
                if (!bounded_all(&p->wp_q[w * p->dof_stride + d], 1))
                    throw Err{MRV_E_INVALID, "waypoint configuration not finite or beyond MRV_MAX_COORD"};
        }
        if (p->wp_t[e - 1] >= MRV_MAX_T) throw Err{MRV_E_INVALID, "path longer than MRV_MAX_T"};
    }
}

long long max_horizon(const mrv_paths* p, int n_robots)
{
    long long m = 1;
    const long long npaths = (long long)p->n_queries * n_robots;
    for (long long i = 0; i < npaths; ++i) m = std::max<long long>(m, (long long)p->wp_t[p->wp_begin[i + 1] - 1] + 1);
    return m;
}

size_t lds_per_t(const TeamHost& tm)
{
    return (size_t)tm.dev.TS * sizeof(float);
}

int default_chunk(const TeamHost& tm, int kind, int exhaustive)
{
    const size_t per_t = lds_per_t(tm);
    int cmax = (int)((kLdsBudget - 2 * 1024) / per_t);
    cmax = std::min(cmax, kMaxChunk);
    if (cmax < 1) cmax = 1;
    // early-terminating calls: the longest tiles (up to 32 timesteps) with which two
    // 8-wave workgroups fit in the CU's LDS, if that is at least 2, else as many
    // timesteps as fit for one (arm workload MV: 14 timesteps, 4.0 ms against
    // 6.2 ms at 29 with one workgroup per CU; arm+rectangle FFC: 12, 9.8 ms against
    // 13.7 ms at 24; the cloud team: 6, MV 39.1 ms and FFC 51.2 ms against 47.3 ms
    // and 87.9 ms at 12; shorter tiles are slower, 5.1 ms at 8 on the arms, 11.6 ms
    // at 8 for FFC).  Exhaustive calls: up to 8, the largest that
    // keeps as many workgroups per CU as registers allow (seven for MV and FFC)
    // within the CU's 160 KiB of LDS if that is at least 2, else one workgroup
    // fewer, ... (exhaustive FFC on the arm+rectangle team: 3 timesteps at seven
    // per CU 214 ms, 4 at five 244 ms)
    if (!exhaustive) {
        const int c2 = (int)((kLdsBudget / 2 - 1024) / per_t);
        return c2 >= 2 ? std::min(c2, 32) : std::max(1, std::min(cmax, 32));
    }
    for (int wgs = kExhWGsPerCU; wgs >= 1; --wgs) {
        const int c = (int)((160 * 1024 / wgs - 1024) / per_t);
        if (c >= 2 || wgs == 1) return std::max(1, std::min(cmax, std::min(8, c)));
    }
    return 1;
}

size_t lds_bytes_for(const TeamHost& tm, int chunk)
{
    return (size_t)chunk * lds_per_t(tm) + 64;
}

}  // namespace

namespace mrv {
// Make sc hold control words, `bins` tile-count bins and `queries` per-query slots.
// Fresh bins are zeroed here; afterwards k_scan leaves them zero after every call.
void ensure_scratch(Scratch& sc, size_t bins, size_t queries, hipStream_t stream)
{
    // fresh control words and bins are cleared by a kernel on the stream that will
    // use them (a blocking hipMemset runs on the null stream, which the library's
    // non-blocking streams do not wait for)
    if (!sc.ctrl.p) {
        sc.ctrl.ensure(64 + 8 * ST_COUNT + 64);
        HIPCHK(fill_u32(sc.ctrl.p, 0u, sc.ctrl.cap / 4, stream));
    }
    if (!sc.ev0) {
        HIPCHK(hipEventCreate(&sc.ev0));
        HIPCHK(hipEventCreate(&sc.ev1));
    }
    sc.gq.ensure(sc.gq_records * 16);
    if (bins > sc.bins) {
        sc.hist.release();
        sc.start.release();
        sc.off.release();
        sc.hist.ensure(bins * sizeof(int));
        sc.start.ensure(bins * sizeof(int));
        sc.off.ensure(bins * sizeof(long long));
        HIPCHK(fill_u32(sc.hist.p, 0u, sc.hist.cap / 4, stream));
        sc.bins = bins;
    }
    const size_t Q = std::max<size_t>(queries, 1);
    sc.q_T.ensure(Q * 4);
    sc.q_nt.ensure(Q * 4);
    sc.q_g.ensure(Q * 4);
    sc.q_chunk.ensure(Q * 4);
    sc.q_eps.ensure(Q * 4);
    sc.q_status.ensure(Q * 4);
    sc.q_word.ensure(Q * 4);
    sc.q_drop.ensure(Q * 4);
    sc.q_sorted.ensure(Q * 4);
}

bool grow_recheck(Scratch& sc, size_t pushed)
{
    if (pushed <= sc.gq_records) return false;
    size_t want = sc.gq_records;
    while (want < pushed + pushed / 4) want <<= 1;
    if (want > Scratch::kMaxRecheckCap) return false;
    sc.gq.release();
    sc.gq_records = want;
    sc.gq.ensure(want * 16);
    return true;
}
}  // namespace mrv

namespace {


// Queue the whole pipeline for one call on `stream`, with its scratch at the
// device pointers of `v`; ev0/ev1 (may be null) bracket the validation kernel.
void launch_plan(mrv_ctx ctx, const ScratchView& v, const CallPlan& pl, void* out_dev, hipStream_t stream,
                 hipEvent_t ev0, hipEvent_t ev1)
{
    const int kind = pl.kind;
    CallDev cd{};
    cd.n_queries = pl.dp.n_queries;
    cd.dof_stride = pl.dp.dof_stride;
    cd.kind = kind;
    cd.flags = pl.flags;
    cd.lds_bytes = (int)pl.lds;
    cd.team0 = pl.team0;
    cd.q_team = pl.q_team;
    cd.env0 = pl.env0;
    cd.q_env = pl.q_env;
    cd.q_pathoff = pl.q_pathoff;
    cd.focus0 = pl.focus;
    cd.q_focus = pl.q_focus;
    cd.eps32 = (float)ctx->eps;
    cd.chunk_floor = std::max(1, pl.min_chunk);
    cd.claim = pl.claim > 0 ? pl.claim : default_claim(pl.flags);
    cd.claim_auto = pl.claim > 0 ? 0 : 1;
    cd.max_nt = (long long)v.bins - 2;
    cd.n_wp = pl.dp.n_wp;
    cd.wp_begin = pl.dp.wp_begin;
    cd.wp_t = pl.dp.wp_t;
    cd.wp_q = pl.dp.wp_q;
    cd.T = v.q_T;
    cd.nt = v.q_nt;
    cd.gstep = v.q_g;
    cd.q_chunk = v.q_chunk;
    cd.q_eps = v.q_eps;
    cd.status = v.q_status;
    cd.word = v.q_word;
    cd.drop = v.q_drop;
    cd.sorted_q = v.q_sorted;
    cd.hist = v.hist;
    cd.start = v.start;
    cd.off = v.off;
    cd.ctrl = v.ctrl;
    cd.gq = v.gq;
    cd.gq_cap = (int)v.gq_records;
    cd.stats = (unsigned long long*)((char*)v.ctrl + 64);
    cd.valid_out = kind == 0 ? (unsigned char*)out_dev : nullptr;
    cd.conflict_out = kind == 1 ? (int*)out_dev : nullptr;

    cd.points = pl.points && kind == 0 && (pl.flags & MRV_CHECK_ENV) ? 1 : 0;
    const int per_cu = std::max(1, validate_blocks_per_cu(validate_variant(cd), cd.points != 0, pl.lds));
    const int want = pl.wg_per_cu > 0 ? std::min(pl.wg_per_cu, per_cu) : per_cu;
    const int grid = std::max(1, ctx->n_cu * want);

    HIPCHK(launch_prepare(cd, stream));
    if (ev0) HIPCHK(hipEventRecord(ev0, stream));
    HIPCHK(launch_validate(cd, grid, stream));
    if (ev1) HIPCHK(hipEventRecord(ev1, stream));
    HIPCHK(launch_finalize(cd, stream));
}

// Queue the whole pipeline for one call on `stream`, scratch from sc (grown to fit).
void run_plan(mrv_ctx ctx, Scratch& sc, const CallPlan& pl, void* out_dev, hipStream_t stream, bool timing = true)
{
    const int min_chunk = std::max(1, pl.min_chunk);
    ensure_scratch(sc, (size_t)tile_bins(pl.max_T, min_chunk), (size_t)pl.dp.n_queries, stream);
    launch_plan(ctx, sc.view(), pl, out_dev, stream, timing ? sc.ev0 : nullptr, timing ? sc.ev1 : nullptr);
    if (timing) sc.last_kind = pl.kind;
}

// Plan for a call whose queries all use one team and environment.
// The default phase order of an early-terminating MV call: robot-robot tests first
// when the environment has a point cloud (its tests cost most), else obstacles first.
uint32_t resolve_phase_order(int kind, uint32_t flags, const EnvHost* env)
{
    if (kind != 0 || (flags & (MRV_PAIRS_FIRST | MRV_OBSTACLES_FIRST))) return flags;
    return env && env->dev.n_pts > 0 ? flags | MRV_PAIRS_FIRST : flags;
}

CallPlan single_plan(const TeamHost& tm, const EnvHost* env, int kind, uint32_t flags, const DevPaths& dp,
                     long long max_T, uint32_t focus = 0)
{
    flags = resolve_phase_order(kind, flags, env);
    CallPlan pl{};
    pl.kind = kind;
    pl.flags = flags;
    // a focus set holding every robot is plain MV (and runs the plain MV kernel)
    const uint32_t all = tm.dev.n_robots >= 32 ? 0xFFFFFFFFu : (1u << tm.dev.n_robots) - 1u;
    pl.focus = kind == 0 && (focus & all) != all ? focus : 0u;
    pl.dp = dp;
    pl.team0 = tm.d_dev;
    pl.env0 = env ? env->d_dev : nullptr;
    pl.max_T = max_T;
    const int m = mode_of(flags);
    pl.min_chunk = tm.dev.chunk[kind][m];
    pl.lds = lds_bytes_for(tm, tm.dev.chunk[kind][m]);
    pl.wg_per_cu = tm.tiling[kind][m].wg_per_cu;
    pl.claim = tm.tiling[kind][m].claim;
    pl.points = env && env->dev.n_pts > 0;
    return pl;
}

TeamHost& find_team(mrv_ctx ctx, int h)
{
    auto it = ctx->teams.find(h);
    if (it == ctx->teams.end()) throw Err{MRV_E_HANDLE, "unknown team handle " + std::to_string(h)};
    return it->second;
}

const EnvHost* find_env(mrv_ctx ctx, int h)
{
    if (h < 0) return nullptr;
    auto it = ctx->envs.find(h);
    if (it == ctx->envs.end()) throw Err{MRV_E_HANDLE, "unknown environment handle " + std::to_string(h)};
    return &it->second;
}

// Host-array call: validate, upload, run, download, wait.
void host_call(mrv_ctx ctx, int team, int env, int kind, const mrv_paths* p, uint32_t flags, void* out_host,
               uint32_t focus = 0)
{
    set_device(ctx);
    TeamHost tm;
    EnvHost evh;
    const EnvHost* ev = nullptr;
    {
        // copy the handles' descriptors; the device data stay owned by the context
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        tm = find_team(ctx, team);
        if (kind == 0 && find_env(ctx, env)) {
            evh = *find_env(ctx, env);
            ev = &evh;
        }
    }
    check_paths_host(tm, p);
    if (p->n_queries == 0) return;
    const int n = tm.dev.n_robots;
    const size_t nb = ((size_t)p->n_queries * n + 1) * sizeof(long long);
    const size_t nt = (size_t)p->n_wp * sizeof(int);
    const size_t nq = (size_t)p->n_wp * (size_t)p->dof_stride * sizeof(double);
    const size_t nout = kind == 0 ? (size_t)p->n_queries : (size_t)p->n_queries * sizeof(mrv_conflict);
    ctx->in_begin.ensure(nb);
    ctx->in_t.ensure(nt);
    ctx->in_q.ensure(nq);
    ctx->out_buf.ensure(nout);
    HIPCHK(hipMemcpyAsync(ctx->in_begin.p, p->wp_begin, nb, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->in_t.p, p->wp_t, nt, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->in_q.p, p->wp_q, nq, hipMemcpyHostToDevice, ctx->stream));
    DevPaths dp{(const long long*)ctx->in_begin.p, (const int*)ctx->in_t.p, (const double*)ctx->in_q.p,
                p->n_wp, p->n_queries, p->dof_stride};
    const CallPlan pl = single_plan(tm, ev, kind, flags, dp, max_horizon(p, n), focus);
    // a call whose near tests overflow the queue runs again with a queue that fits
    for (int attempt = 0;; ++attempt) {
        run_plan(ctx, ctx->sc, pl, ctx->out_buf.p, ctx->stream);
        int cnt[2] = {0, 0};   // unresolved queries, near tests pushed
        HIPCHK(hipMemcpyAsync(cnt, (int*)ctx->sc.ctrl.p + 1, sizeof(cnt), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (!cnt[0]) break;
        // this call's own overflow is handled here, not by the next mrv_sync
        int since = 0;
        HIPCHK(hipMemcpy(&since, (int*)ctx->sc.ctrl.p + 9, sizeof(int), hipMemcpyDeviceToHost));
        since -= cnt[0];
        HIPCHK(hipMemcpy((int*)ctx->sc.ctrl.p + 9, &since, sizeof(int), hipMemcpyHostToDevice));
        if (attempt >= 2 || !grow_recheck(ctx->sc, (unsigned)cnt[1]))
            throw Err{MRV_E_NOMEM, std::to_string(cnt[0]) +
                                       " queries exceeded the near-contact re-evaluation queue; split the batch"};
    }
    HIPCHK(hipMemcpyAsync(out_host, ctx->out_buf.p, nout, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
}

void device_call(mrv_ctx ctx, int team, int env, int kind, const mrv_paths* p, uint32_t flags, void* out_dev,
                 uint32_t focus = 0)
{
    set_device(ctx);
    TeamHost tm;
    EnvHost evh;
    const EnvHost* ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        tm = find_team(ctx, team);
        if (kind == 0 && find_env(ctx, env)) {
            evh = *find_env(ctx, env);
            ev = &evh;
        }
    }
    if (!p) throw Err{MRV_E_INVALID, "null paths"};
    if (p->n_queries < 0) throw Err{MRV_E_INVALID, "negative n_queries"};
    if (p->n_queries == 0) return;
    if (!p->wp_begin || !p->wp_t || !p->wp_q || !out_dev) throw Err{MRV_E_INVALID, "null device pointer"};
    if (p->n_wp < 1) throw Err{MRV_E_INVALID, "n_wp must be positive"};
    if (p->dof_stride < tm.max_dof) throw Err{MRV_E_INVALID, "dof_stride smaller than the team's largest dof"};
    DevPaths dp{(const long long*)p->wp_begin, p->wp_t, p->wp_q, p->n_wp, p->n_queries, p->dof_stride};
    run_plan(ctx, ctx->sc, single_plan(tm, ev, kind, flags, dp, MRV_MAX_T, focus), out_dev, ctx->stream);
}

// Scratch view over the fixed per-device array (layout in mrv_internal.hpp), with
// `bins` tile-count bins.
ScratchView noalloc_view(void* base, size_t bins)
{
    char* b = (char*)base;
    ScratchView v{};
    v.ctrl = (int*)b;
    v.hist = (int*)(b + kNaHist);
    v.start = (int*)(b + kNaStart);
    v.off = (int*)(b + kNaOff);
    v.bins = bins;
    int** q[] = {&v.q_T, &v.q_nt, &v.q_g, &v.q_chunk, (int**)&v.q_eps, &v.q_status, (int**)&v.q_word,
                 (int**)&v.q_drop, &v.q_sorted};
    for (size_t k = 0; k < 9; ++k) *q[k] = (int*)(b + kNaQuery + k * kNaQueryBytes);
    v.gq = (int4*)(b + kNaRecheck);
    v.gq_records = MRV_NOALLOC_RECHECK_RECORDS;
    return v;
}

// mrv_mv_device on the fixed scratch: no device memory is allocated or freed.  The
// handles' descriptors are read in place under the handle lock (no copies).
void noalloc_call(mrv_ctx ctx, int team, int env, const mrv_paths* p, uint32_t flags, void* out_dev)
{
    set_device(ctx);
    if (!p) throw Err{MRV_E_INVALID, "null paths"};
    if (p->n_queries < 0) throw Err{MRV_E_INVALID, "negative n_queries"};
    if (p->n_queries > MRV_NOALLOC_MAX_QUERIES)
        throw Err{MRV_E_INVALID, "n_queries above MRV_NOALLOC_MAX_QUERIES; use mrv_mv_device"};
    if (p->n_queries == 0) return;
    if (!p->wp_begin || !p->wp_t || !p->wp_q || !out_dev) throw Err{MRV_E_INVALID, "null device pointer"};
    if (p->n_wp < 1) throw Err{MRV_E_INVALID, "n_wp must be positive"};
    void* base = noalloc_scratch(ctx->device);
    if (!base) throw Err{MRV_E_DEVICE, "fixed scratch is not set up on the context's device"};
    CallPlan pl{};
    {
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        const TeamHost& tm = find_team(ctx, team);
        const EnvHost* ev = find_env(ctx, env);
        if (p->dof_stride < tm.max_dof) throw Err{MRV_E_INVALID, "dof_stride smaller than the team's largest dof"};
        const DevPaths dp{(const long long*)p->wp_begin, p->wp_t, p->wp_q, p->n_wp, p->n_queries, p->dof_stride};
        pl = single_plan(tm, ev, 0, flags, dp, MRV_MAX_T);
    }
    const size_t bins = (size_t)tile_bins(MRV_MAX_T, std::max(1, pl.min_chunk));
    if (bins > kNaBins) throw Err{MRV_E_DEVICE, "tile bins beyond the fixed scratch"};   // chunk >= 1: never
    // control words and the bins this call may touch start at zero (k_scan leaves the
    // bins zero again, but an earlier call may not have run to its end)
    HIPCHK(fill_u32(base, 0u, (kNaHist + bins * sizeof(int)) / 4, ctx->stream));
    launch_plan(ctx, noalloc_view(base, bins), pl, out_dev, ctx->stream, nullptr, nullptr);
}

uint32_t check_flags(int kind, uint32_t flags)
{
    const uint32_t known = MRV_CHECK_ENV | MRV_EXHAUSTIVE | MRV_HIERARCHICAL | MRV_ORDER_RAKE | MRV_ORDER_LINEAR |
                           MRV_PAIRS_FIRST | MRV_OBSTACLES_FIRST | MRV_PAIR_PRIORITY;
    if (flags & ~known) throw Err{MRV_E_INVALID, "unknown flag bits"};
    if ((flags & MRV_ORDER_RAKE) && (flags & MRV_ORDER_LINEAR)) throw Err{MRV_E_INVALID, "two tile orders requested"};
    if ((flags & MRV_PAIRS_FIRST) && (flags & MRV_OBSTACLES_FIRST))
        throw Err{MRV_E_INVALID, "two phase orders requested"};
    if (kind == 1) flags &= MRV_EXHAUSTIVE;
    return flags;
}

template <class Fn>
mrv_status wrap(Fn&& fn)
{
    try {
        fn();
        return MRV_OK;
    } catch (const Err& e) {
        return fail(e.s, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(MRV_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(MRV_E_DEVICE, "unexpected internal error");
    }
}

}  // namespace

// ===========================================================================
// exported (also used by the serving loop)

namespace mrv {

void serve_run_plan(mrv_ctx ctx, Scratch& sc, const CallPlan& pl, void* out_dev, hipStream_t stream)
{
    run_plan(ctx, sc, pl, out_dev, stream);
}

}  // namespace mrv

extern "C" {

const char* mrv_last_error(void) { return g_err.c_str(); }

mrv_status mrv_memory_stats(mrv_ctx ctx, size_t* used, size_t* peak, size_t* capacity)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    ctx->alloc.stats(used, peak, capacity);
    return MRV_OK;
}

mrv_status mrv_create(const mrv_ctx_opts* opts, mrv_ctx* out)
{
    if (!out) return fail(MRV_E_INVALID, "null output handle");
    return wrap([&] {
        int ndev = 0;
        HIPCHK(hipGetDeviceCount(&ndev));
        const int dev = opts ? opts->device : 0;
        if (dev < 0 || dev >= ndev) throw Err{MRV_E_INVALID, "device ordinal out of range"};
        if (opts && opts->flags != 0) throw Err{MRV_E_INVALID, "unknown context flags"};
        std::unique_ptr<mrv_ctx_s> c(new mrv_ctx_s());
        c->device = dev;
        HIPCHK(hipSetDevice(dev));
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, dev));
        c->n_cu = prop.multiProcessorCount;
        // the device's fixed scratch (mrv_mv_device_noalloc), looked up once per device
        HIPCHK(noalloc_scratch_setup(dev));
        if (opts && opts->near_eps > 0) c->eps = opts->near_eps;
        if (!(c->eps < 1e-2)) throw Err{MRV_E_INVALID, "near_eps must be < 0.01 m"};
        if (opts && opts->max_inflight > 0) c->max_inflight = opts->max_inflight;
        if (opts && opts->serve_bytes > 0) c->serve_bytes = opts->serve_bytes;
        if (opts && (opts->device_arena != nullptr) != (opts->arena_bytes > 0))
            throw Err{MRV_E_INVALID, "device_arena and arena_bytes must be given together"};
        if (opts && opts->device_arena) {
            hipPointerAttribute_t attr{};
            if (hipPointerGetAttributes(&attr, opts->device_arena) != hipSuccess ||
                attr.type != hipMemoryTypeDevice || attr.device != dev)
                throw Err{MRV_E_INVALID, "device_arena is not device memory of the context's device"};
            c->alloc.use_arena(opts->device_arena, opts->arena_bytes);
        }
        c->sc.bind(&c->alloc);
        for (DevBuf* b : {&c->in_begin, &c->in_t, &c->in_q, &c->out_buf, &c->tune_desc}) b->a = &c->alloc;
        if (opts && opts->recheck_records > 0) {
            if ((uint64_t)opts->recheck_records > Scratch::kMaxRecheckCap)
                throw Err{MRV_E_INVALID, "recheck_records above 2^27"};
            c->recheck_records = (size_t)opts->recheck_records;
        }
        c->sc.gq_records = c->recheck_records;
        if (opts && opts->stream) {
            c->stream = (hipStream_t)opts->stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        ensure_scratch(c->sc, (size_t)MRV_MAX_T + 2, 1, c->stream);
        *out = c.release();
    });
}

mrv_status mrv_destroy(mrv_ctx ctx)
{
    if (!ctx) return MRV_OK;
    mrv_status st = wrap([&] {
        if (ctx->serve) ctx->serve.reset();
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        for (auto& kv : ctx->teams) ctx->alloc.free(kv.second.dmem);
        for (auto& kv : ctx->envs) ctx->alloc.free(kv.second.dmem);
        ctx->sc.release();
        for (DevBuf* b : {&ctx->in_begin, &ctx->in_t, &ctx->in_q, &ctx->out_buf, &ctx->tune_desc}) b->release();
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    });
    delete ctx;
    return st;
}

mrv_status mrv_load_team(mrv_ctx ctx, const mrv_robot_desc* robots, int32_t n_robots, int32_t* team_out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!team_out) return fail(MRV_E_INVALID, "null team_out");
    return wrap([&] {
        set_device(ctx);
        TeamHost th;
        build_team(ctx, robots, n_robots, th);
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        const int h = ctx->next_handle++;
        ctx->teams.emplace(h, th);
        *team_out = h;
    });
}

mrv_status mrv_load_env(mrv_ctx ctx, const mrv_env_desc* env, int32_t* env_out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!env_out) return fail(MRV_E_INVALID, "null env_out");
    return wrap([&] {
        set_device(ctx);
        EnvHost eh;
        build_env(ctx, env, eh);
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        const int h = ctx->next_handle++;
        ctx->envs.emplace(h, eh);
        *env_out = h;
    });
}

mrv_status mrv_unload(mrv_ctx ctx, int32_t handle)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    return wrap([&] {
        set_device(ctx);
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        auto t = ctx->teams.find(handle);
        if (t != ctx->teams.end()) {
            if (t->second.inflight > 0) throw Err{MRV_E_BUSY, "team is used by a queued request"};
            HIPCHK(hipStreamSynchronize(ctx->stream));
            ctx->alloc.free(t->second.dmem);
            ctx->teams.erase(t);
            return;
        }
        auto e = ctx->envs.find(handle);
        if (e != ctx->envs.end()) {
            if (e->second.inflight > 0) throw Err{MRV_E_BUSY, "environment is used by a queued request"};
            HIPCHK(hipStreamSynchronize(ctx->stream));
            ctx->alloc.free(e->second.dmem);
            ctx->envs.erase(e);
            return;
        }
        throw Err{MRV_E_HANDLE, "unknown handle " + std::to_string(handle)};
    });
}

mrv_status mrv_mv(mrv_ctx ctx, int32_t team, int32_t env, const mrv_paths* paths, uint32_t flags,
                  uint8_t* valid_out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!valid_out && paths && paths->n_queries > 0) return fail(MRV_E_INVALID, "null valid_out");
    return wrap([&] {
        const uint32_t f = check_flags(0, flags);
        host_call(ctx, team, env, 0, paths, f, valid_out);
    });
}

mrv_status mrv_mv_focus(mrv_ctx ctx, int32_t team, int32_t env, const mrv_paths* paths, uint32_t flags,
                        uint32_t focus, uint8_t* valid_out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!valid_out && paths && paths->n_queries > 0) return fail(MRV_E_INVALID, "null valid_out");
    return wrap([&] {
        const uint32_t f = check_flags(0, flags);
        host_call(ctx, team, env, 0, paths, f, valid_out, focus);
    });
}

mrv_status mrv_mv_focus_device(mrv_ctx ctx, int32_t team, int32_t env, const mrv_paths* paths, uint32_t flags,
                               uint32_t focus, uint8_t* valid_out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    return wrap([&] {
        const uint32_t f = check_flags(0, flags);
        device_call(ctx, team, env, 0, paths, f, valid_out, focus);
    });
}

mrv_status mrv_ffc(mrv_ctx ctx, int32_t team, const mrv_paths* paths, uint32_t flags, mrv_conflict* out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!out && paths && paths->n_queries > 0) return fail(MRV_E_INVALID, "null output");
    return wrap([&] {
        const uint32_t f = check_flags(1, flags);
        host_call(ctx, team, -1, 1, paths, f, out);
    });
}

mrv_status mrv_mv_device_noalloc(mrv_ctx ctx, int32_t team, int32_t env, const mrv_paths* paths, uint32_t flags,
                                 uint8_t* valid_out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    return wrap([&] {
        const uint32_t f = check_flags(0, flags);
        noalloc_call(ctx, team, env, paths, f, valid_out);
    });
}

mrv_status mrv_mv_device(mrv_ctx ctx, int32_t team, int32_t env, const mrv_paths* paths, uint32_t flags,
                         uint8_t* valid_out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    return wrap([&] {
        const uint32_t f = check_flags(0, flags);
        device_call(ctx, team, env, 0, paths, f, valid_out);
    });
}

mrv_status mrv_ffc_device(mrv_ctx ctx, int32_t team, const mrv_paths* paths, uint32_t flags, mrv_conflict* out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    return wrap([&] {
        const uint32_t f = check_flags(1, flags);
        device_call(ctx, team, -1, 1, paths, f, out);
    });
}

mrv_status mrv_sync(mrv_ctx ctx)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    int bad = 0, unresolved = 0;
    bool grown = false;
    mrv_status st = wrap([&] {
        set_device(ctx);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        int* c = (int*)ctx->sc.ctrl.p;
        int most = 0;
        HIPCHK(hipMemcpy(&bad, c + 3, sizeof(int), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(&most, c + 8, sizeof(int), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(&unresolved, c + 9, sizeof(int), hipMemcpyDeviceToHost));
        const int zero[2] = {0, 0};
        HIPCHK(hipMemcpy(c + 3, zero, sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c + 8, zero, 2 * sizeof(int), hipMemcpyHostToDevice));
        // size the queue for the largest call seen, so that repeating it succeeds
        if (unresolved) grown = grow_recheck(ctx->sc, (unsigned)most);
    });
    if (st != MRV_OK) return st;
    if (bad) return fail(MRV_E_INVALID, std::to_string(bad) + " queries had malformed path data");
    if (unresolved)
        return fail(MRV_E_NOMEM, std::to_string(unresolved) +
                                     " queries exceeded the near-contact re-evaluation queue (results 3 / t = -3)" +
                                     (grown ? "; the queue has been enlarged, repeat the calls" : ""));
    return MRV_OK;
}

int64_t mrv_motion_steps(const double* dq, int32_t dof, double step, int32_t metric)
{
    if (!dq || dof < 0 || !(step > 0) || !std::isfinite(step) || (metric != 0 && metric != 1)) {
        g_err = "invalid arguments";
        return -1;
    }
    double d = 0.0;
    for (int k = 0; k < dof; ++k) {
        if (!std::isfinite(dq[k])) {
            g_err = "non-finite dq";
            return -1;
        }
        if (metric == 0) d += dq[k] * dq[k];
        else d = std::max(d, std::fabs(dq[k]));
    }
    if (metric == 0) d = std::sqrt(d);
    const double n = std::ceil(d / step);
    if (n > (double)(MRV_MAX_T - 1)) {
        g_err = "motion needs more than MRV_MAX_T steps";
        return -1;
    }
    return (int64_t)n;
}

mrv_status mrv_set_tiling(mrv_ctx ctx, int32_t team, int32_t kind, uint32_t flags, const mrv_tiling* tiling)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    return wrap([&] {
        if (!tiling || (kind != 0 && kind != 1)) throw Err{MRV_E_INVALID, "bad tiling arguments"};
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        TeamHost& tm = find_team(ctx, team);
        if (tm.inflight > 0) throw Err{MRV_E_BUSY, "team is used by a served request or a captured graph"};
        if (tiling->chunk < 0 || tiling->chunk > kMaxChunk) throw Err{MRV_E_INVALID, "chunk out of range"};
        if (tiling->chunk > 0 && lds_bytes_for(tm, tiling->chunk) > (size_t)kLdsBudget - 2 * 1024)
            throw Err{MRV_E_INVALID, "chunk does not fit in LDS for this team"};
        if (tiling->wg_per_cu < 0 || tiling->wg_per_cu > 32) throw Err{MRV_E_INVALID, "wg_per_cu out of range"};
        if (tiling->interleave < 0 || tiling->interleave > 3) throw Err{MRV_E_INVALID, "interleave out of range"};
        if (tiling->claim < 0 || tiling->claim > 16) throw Err{MRV_E_INVALID, "claim out of range"};
        const int m = mode_of(flags);
        set_device(ctx);
        // calls queued on the context stream read the descriptor: let them finish first
        HIPCHK(hipStreamSynchronize(ctx->stream));
        tm.tiling[kind][m] = *tiling;
        tm.dev.chunk[kind][m] = tiling->chunk > 0 ? tiling->chunk : default_chunk(tm, kind, m);
        tm.dev.interleave[kind][m] = tiling->interleave;
        HIPCHK(hipMemcpy(tm.d_dev, &tm.dev, sizeof(TeamDev), hipMemcpyHostToDevice));
    });
}

mrv_status mrv_get_tiling(mrv_ctx ctx, int32_t team, int32_t kind, uint32_t flags, mrv_tiling* tiling)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    return wrap([&] {
        if (!tiling || (kind != 0 && kind != 1)) throw Err{MRV_E_INVALID, "bad tiling arguments"};
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        TeamHost& tm = find_team(ctx, team);
        const int m = mode_of(flags);
        mrv_tiling t = tm.tiling[kind][m];
        t.chunk = tm.dev.chunk[kind][m];
        t.interleave = kind == 1 ? 3 : std::max(1, t.interleave);
        if (t.claim == 0) t.claim = default_claim(flags);
        *tiling = t;
    });
}

mrv_status mrv_last_stats(mrv_ctx ctx, mrv_stats* out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!out) return fail(MRV_E_INVALID, "null output");
    return wrap([&] {
        set_device(ctx);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        unsigned long long s[ST_COUNT];
        HIPCHK(hipMemcpy(s, (char*)ctx->sc.ctrl.p + 64, sizeof(s), hipMemcpyDeviceToHost));
        mrv_stats r{};
        r.tiles_run = s[ST_TILES_RUN];
        r.tiles_skipped = s[ST_TILES_SKIPPED];
        r.states_evaluated = s[ST_STATES_EVAL];
        r.states_covered = s[ST_STATES_COVERED];
        r.rr_tests = s[ST_RR_TESTS];
        r.env_tests = s[ST_ENV_TESTS];
        r.self_tests = s[ST_SELF_TESTS];
        r.near_rechecks = s[ST_RECHECKS];
        r.point_tests = s[ST_PT_TESTS];
        float ms = 0.f;
        if (ctx->sc.last_kind >= 0 && hipEventElapsedTime(&ms, ctx->sc.ev0, ctx->sc.ev1) == hipSuccess)
            r.kernel_ms = ms;
        *out = r;
    });
}

mrv_status mrv_spheres(mrv_ctx ctx, int32_t team, const mrv_paths* paths, int32_t n_states,
                       const int32_t* state_query, const int32_t* state_t, float* out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    return wrap([&] {
        set_device(ctx);
        TeamHost tm;
        {
            std::lock_guard<std::mutex> lk(ctx->handle_mu);
            tm = find_team(ctx, team);
        }
        check_paths_host(tm, paths);
        if (n_states < 0 || (n_states > 0 && (!state_query || !state_t || !out)))
            throw Err{MRV_E_INVALID, "bad state arrays"};
        for (int k = 0; k < n_states; ++k)
            if (state_query[k] < 0 || state_query[k] >= paths->n_queries || state_t[k] < 0 || state_t[k] >= MRV_MAX_T)
                throw Err{MRV_E_INVALID, "state " + std::to_string(k) + " out of range"};
        if (n_states == 0) return;
        const int n = tm.dev.n_robots, S = tm.dev.S;
        const size_t nb = ((size_t)paths->n_queries * n + 1) * sizeof(long long);
        const size_t ntb = (size_t)paths->n_wp * sizeof(int);
        const size_t nqb = (size_t)paths->n_wp * (size_t)paths->dof_stride * sizeof(double);
        const size_t nout = (size_t)n_states * S * 16;
        ctx->in_begin.ensure(nb);
        ctx->in_t.ensure(ntb);
        ctx->in_q.ensure(nqb);
        DevBuf st, o;
        st.a = o.a = &ctx->alloc;
        st.ensure((size_t)n_states * 8);
        o.ensure(nout);
        try {
            HIPCHK(hipMemcpyAsync(ctx->in_begin.p, paths->wp_begin, nb, hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync(ctx->in_t.p, paths->wp_t, ntb, hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync(ctx->in_q.p, paths->wp_q, nqb, hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync(st.p, state_query, (size_t)n_states * 4, hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync((char*)st.p + (size_t)n_states * 4, state_t, (size_t)n_states * 4,
                                  hipMemcpyHostToDevice, ctx->stream));
            CallDev cd{};
            cd.n_queries = paths->n_queries;
            cd.dof_stride = paths->dof_stride;
            cd.team0 = tm.d_dev;
            cd.n_wp = paths->n_wp;
            cd.wp_begin = (const long long*)ctx->in_begin.p;
            cd.wp_t = (const int*)ctx->in_t.p;
            cd.wp_q = (const double*)ctx->in_q.p;
            HIPCHK(launch_spheres(cd, (const int*)st.p, (const int*)st.p + n_states, n_states, (float4*)o.p, S,
                                  tm.dev.F + tm.dev.J, ctx->stream));
            HIPCHK(hipMemcpyAsync(out, o.p, nout, hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
        } catch (...) {
            (void)hipStreamSynchronize(ctx->stream);
            st.release();
            o.release();
            throw;
        }
        st.release();
        o.release();
    });
}

// ------------------------------------------------------------ autotuning

mrv_status mrv_autotune(mrv_ctx ctx, int32_t team, int32_t env, int32_t kind, const mrv_paths* sample,
                        uint32_t flags, mrv_tiling* best)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!best || (kind != 0 && kind != 1)) return fail(MRV_E_INVALID, "bad autotune arguments");
    return wrap([&] {
        set_device(ctx);
        const uint32_t f = check_flags(kind, flags);
        TeamHost tm;
        EnvHost evh;
        const EnvHost* ev = nullptr;
        {
            std::lock_guard<std::mutex> lk(ctx->handle_mu);
            tm = find_team(ctx, team);
            if (tm.inflight > 0) throw Err{MRV_E_BUSY, "team is used by a served request or a captured graph"};
            if (kind == 0 && find_env(ctx, env)) {
                evh = *find_env(ctx, env);
                ev = &evh;
            }
        }
        check_paths_host(tm, sample);
        if (sample->n_queries == 0) throw Err{MRV_E_INVALID, "empty autotune sample"};
        const EnvDev& e = ev ? ev->dev : EnvDev{};
        const std::string key = std::to_string(tm.dev.S) + "," + std::to_string(tm.dev.F) + "," +
                                std::to_string(tm.dev.G) + "," + std::to_string(tm.dev.n_robots) + "," +
                                std::to_string(tm.dev.n_self) + "|" + std::to_string(e.n_sph) + "," +
                                std::to_string(e.n_box) + "," + std::to_string(e.n_cyl) + "," +
                                std::to_string(e.n_pts) + "|" + std::to_string(kind) + "|" + std::to_string(f);
        mrv_tiling choice{};
        auto hit = ctx->tune_cache.find(key);
        if (hit != ctx->tune_cache.end()) {
            choice = hit->second;
        } else {
            const int n = tm.dev.n_robots;
            const size_t nb = ((size_t)sample->n_queries * n + 1) * sizeof(long long);
            const size_t ntb = (size_t)sample->n_wp * sizeof(int);
            const size_t nqb = (size_t)sample->n_wp * (size_t)sample->dof_stride * sizeof(double);
            const size_t nout = kind == 0 ? (size_t)sample->n_queries : (size_t)sample->n_queries * 12;
            ctx->in_begin.ensure(nb);
            ctx->in_t.ensure(ntb);
            ctx->in_q.ensure(nqb);
            ctx->out_buf.ensure(nout);
            HIPCHK(hipMemcpyAsync(ctx->in_begin.p, sample->wp_begin, nb, hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync(ctx->in_t.p, sample->wp_t, ntb, hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync(ctx->in_q.p, sample->wp_q, nqb, hipMemcpyHostToDevice, ctx->stream));
            DevPaths dp{(const long long*)ctx->in_begin.p, (const int*)ctx->in_t.p, (const double*)ctx->in_q.p,
                        sample->n_wp, sample->n_queries, sample->dof_stride};
            const long long mT = max_horizon(sample, n);
            int cmax = (int)((kLdsBudget - 2 * 1024) / lds_per_t(tm));
            cmax = std::max(1, std::min(cmax, kMaxChunk));
            std::vector<int> chunks;
            for (int c : {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32, 48, 64})
                if (c <= cmax) chunks.push_back(c);
            if (chunks.empty() || chunks.back() != cmax) chunks.push_back(cmax);
            // trials run on a private copy of the team's descriptor, so calls and served
            // requests that use the team meanwhile keep its tiling
            TeamHost trial = tm;
            ctx->tune_desc.ensure(sizeof(TeamDev));
            trial.d_dev = (TeamDev*)ctx->tune_desc.p;
            const int m = mode_of(f);
            const auto t_start = std::chrono::steady_clock::now();
            auto over_budget = [&] {
                return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count() >
                       MRV_TUNE_BUDGET_MS;
            };
            // best of two timed runs after a warm-up
            auto run_trial = [&](const mrv_tiling& t) {
                trial.dev.chunk[kind][m] = t.chunk;
                trial.dev.interleave[kind][m] = t.interleave;
                trial.tiling[kind][m] = t;
                HIPCHK(hipMemcpyAsync(trial.d_dev, &trial.dev, sizeof(TeamDev), hipMemcpyHostToDevice, ctx->stream));
                float ms_min = 1e30f;
                for (int rep = 0; rep < 3; ++rep) {
                    run_plan(ctx, ctx->sc, single_plan(trial, ev, kind, f, dp, mT), ctx->out_buf.p, ctx->stream);
                    HIPCHK(hipStreamSynchronize(ctx->stream));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, ctx->sc.ev0, ctx->sc.ev1));
                    if (rep > 0) ms_min = std::min(ms_min, ms);
                }
                return ms_min;
            };
            choice = tm.tiling[kind][m];
            choice.chunk = tm.dev.chunk[kind][m];
            float best_ms = run_trial(choice);
            auto consider = [&](const mrv_tiling& t) {
                if (over_budget()) return;
                const float ms = run_trial(t);
                if (ms < best_ms) {
                    best_ms = ms;
                    choice = t;
                }
            };
            // one field at a time, each from the best tiling so far
            for (int c : chunks) {
                mrv_tiling t = choice;
                t.chunk = c;
                if (c != choice.chunk) consider(t);
            }
            const int variant = kind == 1 ? (m ? 4 : 1) : (m ? 3 : 0);
            const int occ = validate_blocks_per_cu(variant, ev && ev->dev.n_pts > 0 && kind == 0,
                                                   lds_bytes_for(trial, choice.chunk));
            for (int wg : {1, 2, 3, 4, 6, 8, 0}) {
                mrv_tiling t = choice;
                t.wg_per_cu = wg;
                if ((wg == 0 || wg < occ) && wg != choice.wg_per_cu) consider(t);
            }
            for (int cl : {1, 2, 4, 8}) {
                mrv_tiling t = choice;
                t.claim = cl;
                if (cl != (choice.claim ? choice.claim : default_claim(f))) consider(t);
            }
            if (kind == 0 && m == 0)
                for (int il : {1, 2, 3}) {
                    mrv_tiling t = choice;
                    t.interleave = il;
                    if (il != std::max(1, choice.interleave)) consider(t);
                }
            ctx->tune_cache[key] = choice;
        }
        // apply the choice to the team
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        TeamHost& live = find_team(ctx, team);
        if (live.inflight > 0) throw Err{MRV_E_BUSY, "team is used by a served request or a captured graph"};
        HIPCHK(hipStreamSynchronize(ctx->stream));
        live.tiling[kind][mode_of(f)] = choice;
        live.dev.chunk[kind][mode_of(f)] = choice.chunk;
        live.dev.interleave[kind][mode_of(f)] = choice.interleave;
        HIPCHK(hipMemcpy(live.d_dev, &live.dev, sizeof(TeamDev), hipMemcpyHostToDevice));
        *best = choice;
    });
}

// ---------------------------------------------------------------- graphs

mrv_status mrv_graph_create(mrv_ctx ctx, int32_t team, int32_t env, int32_t kind, const mrv_paths* paths,
                            uint32_t flags, void* out, mrv_graph* graph)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!graph || (kind != 0 && kind != 1)) return fail(MRV_E_INVALID, "bad graph arguments");
    std::unique_ptr<mrv_graph_s> g(new mrv_graph_s());
    mrv_status st = wrap([&] {
        set_device(ctx);
        const uint32_t f = check_flags(kind, flags);
        if (!paths || paths->n_queries <= 0) throw Err{MRV_E_INVALID, "a graph needs at least one query"};
        if (!paths->wp_begin || !paths->wp_t || !paths->wp_q || !out) throw Err{MRV_E_INVALID, "null device pointer"};
        if (paths->n_wp < 1) throw Err{MRV_E_INVALID, "n_wp must be positive"};
        TeamHost tm;
        EnvHost evh;
        const EnvHost* ev = nullptr;
        {
            std::lock_guard<std::mutex> lk(ctx->handle_mu);
            tm = find_team(ctx, team);
            if (kind == 0 && find_env(ctx, env)) {
                evh = *find_env(ctx, env);
                ev = &evh;
            }
            if (paths->dof_stride < tm.max_dof) throw Err{MRV_E_INVALID, "dof_stride smaller than the team's largest dof"};
        }
        DevPaths dp{(const long long*)paths->wp_begin, paths->wp_t, paths->wp_q, paths->n_wp, paths->n_queries,
                    paths->dof_stride};
        CallPlan pl = single_plan(tm, ev, kind, f, dp, MRV_MAX_T);
        // every buffer exists before capture: nothing is allocated inside the graph
        g->sc.gq_records = ctx->sc.gq_records;
        g->sc.bind(&ctx->alloc);
        ensure_scratch(g->sc, (size_t)MRV_MAX_T + 2, (size_t)paths->n_queries, ctx->stream);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        try {
            run_plan(ctx, g->sc, pl, out, ctx->stream, false);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(ctx->stream, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            throw;
        }
        HIPCHK(hipStreamEndCapture(ctx->stream, &g->graph));
        HIPCHK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        find_team(ctx, team).inflight++;
        if (ev) ctx->envs.find(env)->second.inflight++;
        g->team = team;
        g->env = ev ? env : -1;
        g->kind = kind;
    });
    if (st != MRV_OK) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        g->sc.release();
        return st;
    }
    *graph = g.release();
    return MRV_OK;
}

mrv_status mrv_graph_launch(mrv_ctx ctx, mrv_graph graph)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!graph || !graph->exec) return fail(MRV_E_HANDLE, "null graph");
    return wrap([&] {
        set_device(ctx);
        HIPCHK(hipGraphLaunch(graph->exec, ctx->stream));
    });
}

mrv_status mrv_graph_destroy(mrv_ctx ctx, mrv_graph graph)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!graph) return MRV_OK;
    mrv_status st = wrap([&] {
        set_device(ctx);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        std::lock_guard<std::mutex> lk(ctx->handle_mu);
        auto t = ctx->teams.find(graph->team);
        if (t != ctx->teams.end()) t->second.inflight--;
        if (graph->env >= 0) {
            auto e = ctx->envs.find(graph->env);
            if (e != ctx->envs.end()) e->second.inflight--;
        }
    });
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    graph->sc.release();
    delete graph;
    return st;
}

// --------------------------------------------------------------- serving

mrv_status mrv_submit(mrv_ctx ctx, const mrv_request* req, uint64_t* ticket)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!req || !ticket) return fail(MRV_E_INVALID, "null argument");
    return wrap([&] {
        if (!ctx->serve) {
            // serving budget: as given, else the arena (no further limit) or 1 GiB
            const size_t budget = ctx->serve_bytes ? ctx->serve_bytes : ctx->alloc.arena() ? SIZE_MAX : (size_t(1) << 30);
            ctx->serve.reset(new ServeLoop(ctx, ctx->device, ctx->max_inflight, budget, ctx->recheck_records,
                                           &ctx->alloc));
        }
        // validate against the resident handles, resolve their device descriptors, then copy
        ServeRefs refs{};
        mrv_request rq = *req;
        {
            std::lock_guard<std::mutex> lk(ctx->handle_mu);
            if (req->kind != 0 && req->kind != 1) throw Err{MRV_E_INVALID, "kind must be 0 (MV) or 1 (FFC)"};
            TeamHost& tm = find_team(ctx, req->team);
            const EnvHost* ev = req->kind == 0 ? find_env(ctx, req->env) : nullptr;
            rq.flags = resolve_phase_order(req->kind, check_flags(req->kind, req->flags), ev);
            check_paths_host(tm, &req->paths);
            refs.team = tm.d_dev;
            refs.env = ev ? ev->d_dev : nullptr;
            refs.points = ev && ev->dev.n_pts > 0;
            refs.n_robots = tm.dev.n_robots;
            const int m = mode_of(req->flags);
            refs.chunk = tm.dev.chunk[req->kind][m];
            refs.lds = lds_bytes_for(tm, tm.dev.chunk[req->kind][m]);
            tm.inflight++;
            if (req->kind == 0 && req->env >= 0) ctx->envs.find(req->env)->second.inflight++;
        }
        mrv_status s = ctx->serve->submit(rq, refs, ticket);
        if (s != MRV_OK) {
            std::lock_guard<std::mutex> lk(ctx->handle_mu);
            ctx->teams.find(req->team)->second.inflight--;
            if (req->kind == 0 && req->env >= 0) ctx->envs.find(req->env)->second.inflight--;
            throw Err{s, s == MRV_E_BUSY ? "request queue full" : "submit failed"};
        }
    });
}

mrv_status mrv_poll(mrv_ctx ctx, uint64_t ticket, void* out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!ctx->serve) return fail(MRV_E_HANDLE, "unknown ticket");
    std::string msg;
    mrv_status s = ctx->serve->poll(ticket, out, 0, &msg);
    if (s < 0) return fail(s, msg);
    return s;
}

mrv_status mrv_wait(mrv_ctx ctx, uint64_t ticket, int32_t timeout_ms, void* out)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!ctx->serve) return fail(MRV_E_HANDLE, "unknown ticket");
    std::string msg;
    mrv_status s = ctx->serve->poll(ticket, out, timeout_ms < 0 ? -1 : timeout_ms, &msg);
    if (s == MRV_PENDING) return fail(MRV_E_TIMEOUT, "request still running");
    if (s < 0) return fail(s, msg);
    return s;
}

mrv_status mrv_cancel(mrv_ctx ctx, uint64_t ticket)
{
    if (guard(ctx)) return MRV_E_HANDLE;
    if (!ctx->serve) return fail(MRV_E_HANDLE, "unknown ticket");
    mrv_status s = ctx->serve->cancel(ticket);
    if (s < 0) return fail(s, "unknown ticket");
    return s;
}

}  // extern "C"

// called by the serving loop when a request leaves the system
namespace mrv {
void serve_release_handles(mrv_ctx ctx, int team, int env, int kind)
{
    std::lock_guard<std::mutex> lk(ctx->handle_mu);
    auto t = ctx->teams.find(team);
    if (t != ctx->teams.end()) t->second.inflight--;
    if (kind == 0 && env >= 0) {
        auto e = ctx->envs.find(env);
        if (e != ctx->envs.end()) e->second.inflight--;
    }
}
std::mutex& serve_handle_mutex(mrv_ctx ctx) { return ctx->handle_mu; }
}  // namespace mrv
