// Host-side pieces shared by the runtime (mrv_host.cpp) and the serving loop
// (mrv_serve.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>

#include "../../include/mrv.h"
#include "mrv_internal.hpp"

namespace mrv {

struct Err {
    mrv_status s;
    std::string msg;
};

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::mrv::Err{MRV_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// Device memory of one context.  With use_arena(), every allocation is carved
// out of caller-owned memory (first fit, 256-byte aligned, free neighbours
// merged) and nothing calls hipMalloc; otherwise each allocation is a hipMalloc.
// Thread-safe.  alloc() throws Err{MRV_E_NOMEM} when the request cannot be met.
class DevAlloc {
public:
    void use_arena(void* base, size_t bytes);
    bool arena() const { return base_ != nullptr; }
    void* alloc(size_t bytes);
    void free(void* p);
    size_t largest_free() const;                 // SIZE_MAX without an arena
    void stats(size_t* used, size_t* peak, size_t* capacity) const;

private:
    mutable std::mutex mu_;
    char* base_ = nullptr;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;              // offset -> bytes (arena only)
    std::unordered_map<uintptr_t, size_t> live_; // address -> bytes
};

// Device buffer that only grows, from an allocator (hipMalloc when a is null).
struct DevBuf {
    DevAlloc* a = nullptr;
    void* p = nullptr;
    size_t cap = 0;
    void ensure(size_t bytes);
    void release();
};

// Device pointers of one call's scratch (see CallDev): control words (64 bytes of
// ints, then ST_COUNT u64 counters), tile enumeration arrays of `bins` entries,
// per-query arrays and the near-contact queue.
struct ScratchView {
    int* ctrl;
    int *hist, *start, *off;     // off holds long long
    size_t bins;
    int *q_T, *q_nt, *q_g, *q_chunk;
    float* q_eps;
    int* q_status;
    unsigned *q_word, *q_drop;
    int* q_sorted;
    int4* gq;
    size_t gq_records;
};

// Scratch of one call in flight: control words, tile enumeration arrays and
// per-query arrays.  The synchronous entry points share the context's own set;
// each serving slot has one.
struct Scratch {
    DevBuf ctrl;            // 8 ints + ST_COUNT u64
    DevBuf hist, start, off;
    size_t bins = 0;
    DevBuf q_T, q_nt, q_g, q_chunk, q_eps, q_status, q_word, q_drop, q_sorted;
    DevBuf gq;              // near-contact queue (int4 records)
    size_t gq_records = kGlobalRecheckCap;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int last_kind = -1;
    static constexpr size_t kGlobalRecheckCap = size_t(1) << 21;   // 32 MiB
    static constexpr size_t kMaxRecheckCap = size_t(1) << 27;      // 2 GiB
    template <class Fn>
    void each_buf(Fn fn)
    {
        for (DevBuf* b : {&ctrl, &hist, &start, &off, &q_T, &q_nt, &q_g, &q_chunk, &q_eps, &q_status, &q_word,
                          &q_drop, &q_sorted, &gq})
            fn(*b);
    }
    // Take device memory from `a` from now on (buffers must be empty).
    void bind(DevAlloc* a)
    {
        each_buf([a](DevBuf& b) { b.a = a; });
    }
    // Give every device buffer back (the events stay).
    void release_buffers()
    {
        each_buf([](DevBuf& b) { b.release(); });
        bins = 0;
    }
    void release()
    {
        release_buffers();
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        ev0 = ev1 = nullptr;
        bins = 0;
    }
    ScratchView view() const
    {
        return ScratchView{(int*)ctrl.p, (int*)hist.p, (int*)start.p, (int*)off.p, bins, (int*)q_T.p, (int*)q_nt.p,
                           (int*)q_g.p, (int*)q_chunk.p, (float*)q_eps.p, (int*)q_status.p, (unsigned*)q_word.p,
                           (unsigned*)q_drop.p, (int*)q_sorted.p, (int4*)gq.p, gq_records};
    }
    size_t bytes() const
    {
        return ctrl.cap + hist.cap + start.cap + off.cap + q_T.cap + q_nt.cap + q_g.cap + q_chunk.cap + q_eps.cap +
               q_status.cap + q_word.cap + q_drop.cap + q_sorted.cap + gq.cap;
    }
};

void ensure_scratch(Scratch& sc, size_t bins, size_t queries, hipStream_t stream);
// Enlarge the near-contact queue to hold `pushed` records (with 25% headroom).
// False when it already does or the size would pass kMaxRecheckCap.  The caller
// must have drained every launch that uses sc.
bool grow_recheck(Scratch& sc, size_t pushed);

// Path arrays of one call (device pointers).
struct DevPaths {
    const long long* wp_begin;
    const int* wp_t;
    const double* wp_q;
    long long n_wp;
    int n_queries;
    int dof_stride;
};

// Everything one validation call needs besides scratch and output.
struct CallPlan {
    int kind;
    uint32_t flags;
    DevPaths dp;
    const TeamDev* team0;              // team of every query when q_team is null
    const TeamDev* const* q_team;      // device array, one per query, or null
    const EnvDev* env0;                // null: no obstacles
    const EnvDev* const* q_env;        // device array, one per query, or null
    const long long* q_pathoff;        // device array: first path of each query, or null
    uint32_t focus;                    // robots validated (bit r), 0 = all
    const unsigned* q_focus;           // device array: focus of each query, or null
    long long max_T;                   // bound on every query's horizon
    int min_chunk;                     // smallest timesteps-per-tile among the queries' teams
    size_t lds;                        // dynamic LDS: max over the queries' teams
    int wg_per_cu;                     // 0 = occupancy limit
    int claim;                         // tiles per claim, 0 = automatic
    bool points;                       // some query's environment holds a point cloud
};

// Device-side descriptors a served request needs, resolved at submit time.
struct ServeRefs {
    const TeamDev* team;
    const EnvDev* env;
    bool points;                       // the environment holds a point cloud
    int n_robots;
    int chunk;
    size_t lds;
};

void serve_run_plan(mrv_ctx ctx, Scratch& sc, const CallPlan& pl, void* out_dev, hipStream_t stream);
void serve_release_handles(mrv_ctx ctx, int team, int env, int kind);
std::mutex& serve_handle_mutex(mrv_ctx ctx);

// Request loop behind mrv_submit/mrv_poll (mrv_serve.cpp).
class ServeLoop {
public:
    ServeLoop(mrv_ctx ctx, int device, int max_inflight, size_t budget_bytes, size_t recheck_records,
              DevAlloc* alloc);
    ~ServeLoop();
    mrv_status submit(const mrv_request& req, const ServeRefs& refs, uint64_t* ticket);
    // timeout_ms: 0 = do not wait, < 0 = wait forever
    mrv_status poll(uint64_t ticket, void* out, int timeout_ms, std::string* msg);
    mrv_status cancel(uint64_t ticket);

    struct Impl;

private:
    Impl* impl_;
};

}  // namespace mrv
