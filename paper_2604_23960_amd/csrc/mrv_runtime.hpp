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
    DevBuf q_T, q_nt, q_g, q_status, q_word, q_sorted;
    DevBuf gq;              // near-contact queue (int4 records)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int last_kind = -1;
    static constexpr int kGlobalRecheckCap = 1 << 21;
    void release()
    {
        for (DevBuf* b : {&ctrl, &hist, &start, &off, &q_T, &q_nt, &q_g, &q_status, &q_word, &q_sorted, &gq})
            b->release();
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        ev0 = ev1 = nullptr;
        bins = 0;
    }
    size_t bytes() const
    {
        return ctrl.cap + hist.cap + start.cap + off.cap + q_T.cap + q_nt.cap + q_g.cap + q_status.cap +
               q_word.cap + q_sorted.cap + gq.cap;
    }
};

void ensure_scratch(Scratch& sc, size_t bins, size_t queries);

// Queue one call (device arrays) on `stream` using scratch `sc`.  Caller holds
// serve_handle_mutex(ctx) while the team/environment handles are read.
void serve_run_call(mrv_ctx ctx, Scratch& sc, int team, int env, int kind, uint32_t flags,
                    const long long* wp_begin, const int* wp_t, const double* wp_q, long long n_wp,
                    int n_queries, int dof_stride, long long max_T, void* out_dev, hipStream_t stream);
void serve_release_handles(mrv_ctx ctx, int team, int env, int kind);
std::mutex& serve_handle_mutex(mrv_ctx ctx);

// Request loop behind mrv_submit/mrv_poll (mrv_serve.cpp).
class ServeLoop {
public:
    ServeLoop(mrv_ctx ctx, int device, int max_inflight, size_t budget_bytes);
    ~ServeLoop();
    mrv_status submit(const mrv_request& req, int n_robots, uint64_t* ticket);
    // timeout_ms: 0 = do not wait, < 0 = wait forever
    mrv_status poll(uint64_t ticket, void* out, int timeout_ms, std::string* msg);
    mrv_status cancel(uint64_t ticket);

    struct Impl;

private:
    Impl* impl_;
};

}  // namespace mrv
