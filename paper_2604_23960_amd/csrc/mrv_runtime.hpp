// Host-side pieces shared by the runtime (mrv_host.cpp) and the serving loop
// (mrv_serve.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>

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

// Device buffer that only grows.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    void ensure(size_t bytes)
    {
        if (bytes <= cap) return;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(bytes, 256);
        if (hipMalloc(&p, want) != hipSuccess) {
            p = nullptr;
            throw Err{MRV_E_NOMEM, "device allocation of " + std::to_string(want) + " bytes failed"};
        }
        cap = want;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// Scratch of one call in flight: control words, tile enumeration arrays and
// per-query arrays.  The synchronous entry points share the context's own set;
// each serving slot has one.
struct Scratch {
    DevBuf ctrl;            // 8 ints + ST_COUNT u64
    DevBuf hist, start, off;
    size_t bins = 0;
    DevBuf q_T, q_nt, q_g, q_chunk, q_status, q_word, q_drop, q_sorted;
    DevBuf gq;              // near-contact queue (int4 records)
    size_t gq_records = kGlobalRecheckCap;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int last_kind = -1;
    static constexpr size_t kGlobalRecheckCap = size_t(1) << 21;   // 32 MiB
    static constexpr size_t kMaxRecheckCap = size_t(1) << 27;      // 2 GiB
    void release()
    {
        for (DevBuf* b : {&ctrl, &hist, &start, &off, &q_T, &q_nt, &q_g, &q_chunk, &q_status, &q_word, &q_drop,
                          &q_sorted, &gq})
            b->release();
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        ev0 = ev1 = nullptr;
        bins = 0;
    }
    size_t bytes() const
    {
        return ctrl.cap + hist.cap + start.cap + off.cap + q_T.cap + q_nt.cap + q_g.cap + q_chunk.cap +
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
};

// Device-side descriptors a served request needs, resolved at submit time.
struct ServeRefs {
    const TeamDev* team;
    const EnvDev* env;
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
    ServeLoop(mrv_ctx ctx, int device, int max_inflight, size_t budget_bytes, size_t recheck_records);
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
