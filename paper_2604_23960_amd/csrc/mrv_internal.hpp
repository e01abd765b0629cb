// Internal layouts shared by the host runtime (mrv_host.cpp) and the device
// kernels (mrv_kernels.hip) of libmrv.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/mrv.h"
#include "mrv_tiles.hpp"

namespace mrv {

constexpr int kWG = 256;            // threads per workgroup (4 waves of 64)
constexpr int kWave = 64;
constexpr int kWavesPerWG = kWG / kWave;
// Threads per workgroup of a validation kernel variant (0 early-terminating MV,
// 1 early-terminating FFC, 2 early-terminating MV with a focus set, 3 exhaustive
// MV, 4 exhaustive FFC, 5 exhaustive MV with a focus set): early-terminating
// calls' long tiles leave room for one workgroup per CU, which then runs 8 waves.
constexpr int validate_wg(int variant) { return variant <= 2 ? 512 : kWG; }
constexpr int kMaxRobots = 32;
constexpr int kMaxJoints = 8;
constexpr int kMaxChunk = 64;       // timesteps per tile
constexpr int kLdsBudget = 160 * 1024;   // LDS one workgroup may use on gfx950
constexpr int kWGsPerCU = 6;        // validation workgroups per CU the register budget allows (exhaustive MV with a focus set, 80 VGPRs)
constexpr int kExhWGsPerCU = 7;     // the same for the exhaustive MV and FFC kernels (72 VGPRs)
constexpr int kExhPtsWGsPerCU = 6;  // and for its build for point clouds (80 VGPRs)
// The near band of a query widens in proportion to the largest coordinate magnitude
// its FP32 arithmetic sees beyond this scale (metres); see k_query_info.
constexpr double kEpsRefScale = 4.0;

// Fixed scratch of mrv_mv_device_noalloc, one array per device (byte offsets):
// control words as in every call's scratch, then the tile-count bins (hist,
// start, off) of any call, tile_bins(MRV_MAX_T, 1) of them, so the hist bins
// directly follow the control words and one fill clears both; nine per-query
// arrays of MRV_NOALLOC_MAX_QUERIES entries; the near-contact queue.
constexpr size_t na_align(size_t v) { return (v + 255) & ~size_t(255); }
constexpr size_t kNaBins = (size_t)MRV_MAX_T + 2;
constexpr size_t kNaHist = 256;
constexpr size_t kNaStart = kNaHist + na_align(kNaBins * 4);
constexpr size_t kNaOff = kNaStart + na_align(kNaBins * 4);
constexpr size_t kNaQuery = kNaOff + na_align(kNaBins * 8);
constexpr size_t kNaQueryBytes = na_align((size_t)MRV_NOALLOC_MAX_QUERIES * 4);
constexpr size_t kNaRecheck = kNaQuery + 9 * kNaQueryBytes;
constexpr size_t kNoAllocScratchBytes = kNaRecheck + (size_t)MRV_NOALLOC_RECHECK_RECORDS * 16;
static_assert(kNoAllocScratchBytes <= (size_t(30) << 20), "fixed scratch above its stated bound of 30 MiB");

enum RecheckKind : int { RK_RR = 0, RK_SELF = 1, RK_ENV_SPH = 2, RK_ENV_BOX = 3, RK_ENV_CYL = 4, RK_ENV_PT = 5 };

// Per-call counters (uint64 each), see mrv_stats.
enum StatSlot : int {
    ST_TILES_RUN = 0, ST_TILES_SKIPPED, ST_STATES_EVAL, ST_STATES_COVERED,
    ST_RR_TESTS, ST_ENV_TESTS, ST_SELF_TESTS, ST_RECHECKS, ST_PT_TESTS, ST_COUNT
};

// Resident team.  Spheres of all robots are flattened in robot order; frames of
// one timestep are numbered robot by robot, frame 0 of a robot being its base.
struct TeamDev {
    int n_robots;
    int S;                 // total spheres
    int F;                 // frame slots per timestep: sum over robots of (n_joints + 1)
    int J;                 // joints of the team (the sum of n_joints)
    int n_self;            // distinct self-collision pairs
    int n_sblocks;         // 16 x 16 self blocks per timestep
    int P;                 // robot pairs n(n-1)/2
    int max_dof;
    int G;                 // sphere groups per timestep (16 consecutive spheres of one robot)
    int GS;                // sphere slots, 16 per group
    int GSp;               // LDS row stride of the slot arrays (GS + 16, against bank conflicts)
    int TS;                // LDS floats per timestep of a tile: five slot rows, or three and the FK frames,
                           // or the joint transforms and the frames, whichever is largest
    int chunk[2][2];       // timesteps per tile: [MV / FFC][early-terminating / exhaustive]
    int interleave[2][2];  // tuned MV tile order for calls asking for MRV_ORDER_BISECT (0, 1 golden, 2 rake,
                           // 3 consecutive), as chunk
    int lds_per_t;         // LDS bytes one timestep of a tile needs
    float r_max;           // largest sphere radius of the team
    float origin[4];       // team origin o (centre of the bases' bounding box, an FP32 value): FK, sphere
                           // records and pair tests run on coordinates relative to it
    double origin64[3];    // o exactly, for the FP64 offset to an environment's origin
    float mag;             // largest of r_mag
    long long rr_tests_per_t;   // sum_{i<j} n_i n_j
    const int* r_nj;            // [n]
    const int* r_joint_off;     // [n]
    const int* r_sphere_off;    // [n+1]
    const int* r_frame_off;     // [n]
    const float* r_mag;         // [n] bound on |FP32 coordinate| of the robot's frames and spheres relative
                                // to o, without prismatic joint values (those are added per query)
    const float* r_base32;      // [n][12]
    const double* r_base64;     // [n][12]
    const int* j_type;          // [joints]
    const int* j_robot;         // [joints] robot of each joint
    const float* j_fixed32;     // [joints][12]
    const double* j_fixed64;    // [joints][12]
    const int* s_robot;         // [S]
    const int* s_slot;          // [S] frame slot = r_frame_off[robot] + local frame
    const int* s_lframe;        // [S] local frame 0..n_joints
    const float4* s_local32;    // [S] centre, radius
    const double* s_local64;    // [S][4]
    const int* s_group;         // [S] group of each sphere
    const int2* g_range;        // [G] sphere range [begin, end) of each group
    const int* r_group_off;     // [n+1] first group of each robot
    const int* gtask;           // [G][8] pair task of group ga: ga, its robot, self blocks [sb0, sb1),
                                // first group of the higher robots, robot-robot tests, self tests, 0
    const int* slot_sphere;     // [GS] sphere of each slot, -1 for padding
    const int* slot_frame;      // [GS] frame slot of each slot's sphere, -1 for padding
    const unsigned* r_pri;      // [n] bit j of entry i (j > i): the pair (i, j) is prioritised (adjacent bases)
    const float4* slot_local;   // [GS] local centre and radius of each slot's sphere, zeros for padding
    const int* sblocks;         // [n_sblocks][16] row group, column group, pairs, robot, 0, 0, 0, 0, then
                                // four 64-bit lane masks, one per accumulator register
};

// Points stored past the end of a cloud (copies of its last point), read by the
// sphere-point blocks, which take 32 consecutive points at a time.
constexpr int kPtsPad = 64;

// Resident environment in the world frame.
struct EnvDev {
    int n_sph, n_box, n_cyl;
    long long n_pts;
    const float4* sph32;        // [n] centre, radius
    const double* sph64;        // [n][4]
    const float* box32;         // [n][16] rows (R^T row k, -(R^T c)_k) for k = 0..2, then half-extents, pad
    const double* box64;        // [n][15] as given
    const float* cyl32;         // [n][8] centre(3), axis(3), half-length, radius
    const double* cyl64;        // [n][8]
    const float4* bc_box;       // [n_box + n_cyl][2] world-axis box (lo, hi) of each box, then each cylinder
    // every FP32 coordinate above and below is relative to the environment's origin
    double origin64[3];         // the environment origin (centre of its obstacles' bounding box, an FP32 value)
    float mag;                  // bound on |FP32 coordinate| of any obstacle part relative to the origin
    // uniform grid over the point cloud (CSR by cell)
    const float4* pts32;        // [n_pts + kPtsPad] points sorted by cell (x, y, z, |p|^2), then copies of the last
    const double* pts64;        // [n_pts][3] in the same order
    const int* cell_start;      // [n_cells + 1]
    float grid_lo[3];
    float grid_inv;             // 1 / cell size
    float grid_cell;
    int grid_dim[3];
    float pt_radius;
    double pt_radius64;
};

// One MV/FFC call.  Every query has a team and an environment: either the same
// for all (team0/env0) or per query (q_team/q_env), and its paths start at
// q_pathoff[q] (or q * n_robots when all queries share team0).
struct CallDev {
    int n_queries;
    int dof_stride;
    int kind;                   // 0 = MV, 1 = FFC
    unsigned flags;
    int lds_bytes;              // dynamic LDS of the validation launch
    const TeamDev* team0;
    const TeamDev* const* q_team;
    const EnvDev* env0;         // null: no obstacles
    const EnvDev* const* q_env;
    const long long* q_pathoff;
    unsigned focus0;            // robots validated (bit r), 0 = all: prioritised MV
    const unsigned* q_focus;    // per query, or null: focus0 for every query
    float eps32;                // near band in metres before per-query scaling
    int chunk_floor;            // smallest tile length the call's scratch was sized for
    int claim;                  // tiles taken per claim on the tile counter (>= 1)
    int claim_auto;             // 1: claim is only the most taken; small calls take fewer, keeping
                                // at least 8 claims per workgroup
    int points;                 // 1: some query's environment holds a point cloud (MV with obstacles)
    long long max_nt;           // most tiles a query may have (tile bins - 2)
    long long n_wp;
    const long long* wp_begin;
    const int* wp_t;
    const double* wp_q;
    // per-query scratch
    int* T;
    int* nt;
    int* gstep;
    int* q_chunk;               // timesteps per tile chosen for each query
    float* q_eps;               // near band of each query (eps32 widened for large coordinates)
    int* status;                // 0 ok, 1 invalid input
    unsigned* word;             // MV: hit flag; FFC: best key t*P + pair
    unsigned* drop;             // smallest key (MV: 0) of a near test the full queue dropped
    int* sorted_q;
    // tile enumeration scratch: max_nt + 2 bins (see mrv_tiles.hpp)
    int* hist;
    int* start;
    int* off;
    int* ctrl;                  // [0] max nt, [1] unresolved queries, [2] near tests pushed,
                                // [3] invalid-input queries (kept until read), [4..7] u64 total tiles,
                                // u64 next tile, [8] most near tests pushed by a call and [9] unresolved
                                // queries, both kept until read
    int4* gq;                   // global recheck queue, one int4 per record
    int gq_cap;
    unsigned long long* stats;  // [ST_COUNT]
    // outputs
    unsigned char* valid_out;
    int* conflict_out;          // [n_queries][3]
};

// Kernel launchers (mrv_kernels.hip).  All launch on `stream` and return the
// first launch error.
hipError_t launch_prepare(const CallDev& cd, hipStream_t stream);
hipError_t launch_validate(const CallDev& cd, int grid, hipStream_t stream);
hipError_t launch_finalize(const CallDev& cd, hipStream_t stream);
hipError_t fill_u32(void* p, unsigned v, size_t n, hipStream_t stream);
// n_mats: the team's joints plus frames (J + F), 48 bytes of LDS each.
hipError_t launch_spheres(const CallDev& cd, const int* st_q, const int* st_t, int n_states, float4* out, int S,
                          int n_mats, hipStream_t stream);
// Occupancy-derived workgroups per CU for the validation kernel.
// Whether an MV call restricts validation to a focus set (runs the focus kernel).
inline bool has_focus(const CallDev& cd) { return cd.kind == 0 && (cd.focus0 != 0u || cd.q_focus != nullptr); }
// Validation kernel of a call (variants as for validate_wg).
inline int validate_variant(const CallDev& cd)
{
    const bool exh = (cd.flags & MRV_EXHAUSTIVE) != 0;
    if (cd.kind == 1) return exh ? 4 : 1;
    if (has_focus(cd)) return exh ? 5 : 2;
    return exh ? 3 : 0;
}
// points: the build for environments with point clouds (CallDev::points).
int validate_blocks_per_cu(int variant, bool points, size_t lds_bytes);
// Device address of the fixed scratch on `device`.  noalloc_scratch_setup looks it
// up once per device (that device current) and keeps it; noalloc_scratch returns
// the kept address, null before set-up.
hipError_t noalloc_scratch_setup(int device);
void* noalloc_scratch(int device);

}  // namespace mrv
