// Serving loop behind mrv_submit / mrv_poll / mrv_wait / mrv_cancel.
//
// Requests are copied at submit time into host memory and queued.  One serve
// thread owns a few slots; each slot has its own HIP stream, scratch set, device
// buffers and pinned staging memory.  Whenever a slot is free and requests wait,
// the thread merges the waiting requests that share (kind, flags) with the oldest
// one into a single call -- requests of different teams and environments mix,
// each query carrying its own team and environment descriptor -- stages their
// paths in pinned memory, reserves the batch's device memory (inputs, outputs,
// scratch and near-contact queue) from the context's allocator, and queues one
// upload, the validation kernels and the download on the slot stream.  Batches
// on different slots overlap on the device, and requests that arrive while
// others run are admitted as soon as a slot and memory free up (continuous
// batching).  Admission counts the bytes batches actually hold: a batch starts
// only if the memory held by the batches in flight, its own included, stays
// within the serving budget and the allocator (the caller's arena, if any) can
// supply it; otherwise its requests wait for a running batch to give memory
// back.  With an arena, a slot returns its device memory when its batch ends.
// Completion is detected with HIP events; results are handed to the waiting
// pollers through a condition variable.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mrv_runtime.hpp"

namespace mrv {

namespace {

enum ReqState { RS_QUEUED = 0, RS_RUNNING = 1, RS_DONE = 2, RS_ERROR = 3, RS_CANCELLED = 4 };

struct Req {
    uint64_t id = 0;
    int kind = 0, team = 0, env = -1;
    ServeRefs refs{};
    uint32_t flags = 0;
    uint32_t focus = 0;                 // MV: robots validated, 0 = all
    int n_queries = 0, n_robots = 0, dof_stride = 0;
    long long max_T = 1;
    std::vector<long long> wp_begin;   // relative to this request's waypoints
    std::vector<int> wp_t;
    std::vector<double> wp_q;
    std::vector<unsigned char> result;  // uint8[n] (MV) or int32[3n] (FFC)
    int state = RS_QUEUED;
    bool cancel_requested = false;
    mrv_status err = MRV_OK;
    std::string msg;
};

// What a batch holds on the device, from the requests it merges.
struct BatchShape {
    int nq = 0, kind = 0, stride = 0;
    long long n_paths = 0, n_wp = 0, max_T = 1;
    int min_chunk = 1 << 30;
    void add(const Req& r)
    {
        nq += r.n_queries;
        kind = r.kind;
        stride = r.dof_stride;
        n_paths += (long long)r.n_queries * r.n_robots;
        n_wp += (long long)r.wp_t.size();
        max_T = std::max(max_T, r.max_T);
        min_chunk = std::min(min_chunk, r.refs.chunk);
    }
};

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Pinned/device input block of a batch: wp_begin | wp_t | wp_q | q_team | q_env |
// q_pathoff | q_focus, each piece 256-byte aligned.
struct InputLayout {
    size_t o_t, o_q, o_team, o_env, o_po, o_fo, total;
    explicit InputLayout(const BatchShape& b)
    {
        const size_t nb = (size_t)(b.n_paths + 1) * sizeof(long long);
        o_t = align256(nb);
        o_q = align256(o_t + (size_t)b.n_wp * sizeof(int));
        o_team = align256(o_q + (size_t)b.n_wp * b.stride * sizeof(double));
        o_env = align256(o_team + (size_t)b.nq * 8);
        o_po = align256(o_env + (size_t)b.nq * 8);
        o_fo = align256(o_po + (size_t)b.nq * 8);
        total = o_fo + (size_t)b.nq * 4;
    }
};

// Device bytes a batch of this shape holds on a slot with the given near-contact
// queue length: inputs, outputs and scratch, each buffer as the allocator rounds it.
size_t batch_bytes(const BatchShape& b, size_t gq_records)
{
    auto buf = [](size_t v) { return align256(std::max<size_t>(v, 256)); };
    const size_t Q = std::max(b.nq, 1);
    const size_t bins = (size_t)tile_bins(b.max_T, b.min_chunk == (1 << 30) ? 1 : b.min_chunk);
    return buf(InputLayout(b).total) + buf(b.kind == 0 ? Q : Q * 12) + buf(64 + 8 * ST_COUNT + 64) +
           2 * buf(bins * 4) + buf(bins * 8) + 9 * buf(Q * 4) + buf(gq_records * 16);
}

struct PinnedBuf {
    void* p = nullptr;
    size_t cap = 0;
    void ensure(size_t bytes)
    {
        if (bytes <= cap) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        const size_t want = std::max<size_t>(bytes, 4096);
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            throw Err{MRV_E_NOMEM, "pinned host allocation failed"};
        }
        cap = want;
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Scratch sc;
    DevBuf d_in, d_out;
    size_t held = 0;          // device bytes of the running batch (buffers as allocated)
    PinnedBuf h_in, h_out;
    std::vector<std::shared_ptr<Req>> batch;
    std::vector<int> q_off;   // first query of each request in the batch
    int kind = 0;
    bool busy = false;
    CallPlan plan{};          // the batch's call, kept to run it again after a queue overflow
    size_t nout = 0;
    int attempts = 0;
};

}  // namespace

struct ServeLoop::Impl {
    mrv_ctx ctx;
    int device;
    int max_inflight;
    size_t budget;                      // most device bytes the batches in flight may hold
    DevAlloc* alloc;
    bool mem_wait = false;              // the queue head waits for memory a running batch holds
    bool solo_next = false;             // the next batch is the queue head alone
    size_t recheck_records;             // initial near-contact queue length of a slot
    std::mutex mu;
    std::condition_variable cv_work;    // serve thread waits here when idle
    std::condition_variable cv_done;    // pollers wait here
    std::deque<std::shared_ptr<Req>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> tickets;
    uint64_t next_id = 1;
    int inflight = 0;                   // queued + running requests
    bool stop = false;
    std::vector<Slot> slots;
    std::thread th;

    static constexpr int kSlots = 4;
    static constexpr int kMaxBatchQueries = 1 << 16;

    Impl(mrv_ctx c, int dev, int mi, size_t b, size_t rq, DevAlloc* a)
        : ctx(c), device(dev), max_inflight(mi), budget(b), alloc(a), recheck_records(rq)
    {
        HIPCHK(hipSetDevice(device));
        slots.resize(kSlots);
        for (Slot& s : slots) {
            s.sc.gq_records = rq;
            s.sc.bind(alloc);
            s.d_in.a = s.d_out.a = alloc;
            HIPCHK(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
        }
        th = std::thread([this] { run(); });
    }

    ~Impl()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_work.notify_all();
        if (th.joinable()) th.join();
        (void)hipSetDevice(device);
        for (Slot& s : slots) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            for (auto& r : s.batch) serve_release_handles(ctx, r->team, r->env, r->kind);
            s.sc.release();
            for (DevBuf* b : {&s.d_in, &s.d_out}) b->release();
            s.h_in.release();
            s.h_out.release();
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
        }
        for (auto& r : queue) serve_release_handles(ctx, r->team, r->env, r->kind);
        cv_done.notify_all();
    }

    // ---- serve thread
    void run()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            bool progress = false;
            // completions
            for (Slot& s : slots) {
                if (!s.busy) continue;
                if (hipEventQuery(s.done) != hipSuccess) continue;
                complete(s);
                progress = true;
            }
            // admissions (none while the queue head waits for a running batch's memory)
            for (Slot& s : slots) {
                if (stop || mem_wait) break;
                if (s.busy) continue;
                drop_cancelled();
                if (queue.empty()) break;
                launch(s, lk);
                progress = true;
            }
            if (stop) {
                bool any = false;
                for (Slot& s : slots) any = any || s.busy;
                if (!any) break;
            }
            if (progress) continue;
            if (any_busy()) {
                // a batch is on the device: poll its event shortly
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                cv_work.wait(lk, [this] { return stop || !queue.empty(); });
            }
        }
    }

    void drop_cancelled()
    {
        while (!queue.empty() && queue.front()->cancel_requested) {
            auto r = queue.front();
            queue.pop_front();
            finish(r, RS_CANCELLED, MRV_E_CANCELLED, "cancelled");
        }
    }

    void finish(const std::shared_ptr<Req>& r, int state, mrv_status err, const std::string& msg)
    {
        r->state = state;
        r->err = err;
        r->msg = msg;
        r->wp_begin.clear();
        r->wp_t.clear();
        r->wp_q.clear();
        r->wp_begin.shrink_to_fit();
        r->wp_t.shrink_to_fit();
        r->wp_q.shrink_to_fit();
        inflight--;
        serve_release_handles(ctx, r->team, r->env, r->kind);
        cv_done.notify_all();
    }

    size_t held_by_batches() const
    {
        size_t h = 0;
        for (const Slot& s : slots) h += s.busy ? s.held : 0;
        return h;
    }
    bool any_busy() const
    {
        for (const Slot& s : slots)
            if (s.busy) return true;
        return false;
    }

    // Form a batch from the queue head and queue it on slot s.  Called with mu held;
    // the staging copies and launches run with mu released.  Requests join while the
    // memory the batch will hold (estimated as its allocations) keeps every batch in
    // flight within the budget; the head always joins.  If the allocator cannot
    // supply the batch, its requests go back to the queue front: they wait for a
    // running batch to return memory or, with nothing running, run one at a time,
    // and a request that cannot run even alone fails with MRV_E_NOMEM.
    void launch(Slot& s, std::unique_lock<std::mutex>& lk)
    {
        std::vector<std::shared_ptr<Req>> batch;
        const std::shared_ptr<Req> head = queue.front();
        const size_t others = held_by_batches();
        const size_t room = budget > others ? budget - others : 0;
        BatchShape sh;
        for (auto it = queue.begin(); it != queue.end();) {
            const auto& r = *it;
            const bool same = r->kind == head->kind && r->flags == head->flags && r->dof_stride == head->dof_stride &&
                              !r->cancel_requested;
            bool take = same && (batch.empty() || !solo_next);
            if (take && !batch.empty()) {
                BatchShape t = sh;
                t.add(*r);
                take = t.nq <= kMaxBatchQueries && batch_bytes(t, s.sc.gq_records) <= room;
            }
            if (take) {
                sh.add(*r);
                r->state = RS_RUNNING;
                batch.push_back(r);
                it = queue.erase(it);
            } else {
                ++it;
            }
        }
        const bool solo = solo_next;
        solo_next = false;
        if (batch_bytes(sh, s.sc.gq_records) > room && any_busy()) {
            // the head alone does not fit beside the running batches: wait for them
            requeue(batch);
            mem_wait = true;
            return;
        }
        s.busy = true;
        s.batch = batch;
        s.kind = head->kind;
        s.held = 0;
        lk.unlock();
        mrv_status err = MRV_OK;
        std::string msg;
        try {
            stage_and_run(s);
        } catch (const Err& e) {
            err = e.s;
            msg = e.msg;
        } catch (...) {
            err = MRV_E_DEVICE;
            msg = "serving launch failed";
        }
        lk.lock();
        if (err != MRV_OK) {
            (void)hipStreamSynchronize(s.stream);
            s.busy = false;
            if (alloc->arena()) release_slot(s);
            if (err == MRV_E_NOMEM && (any_busy() || (!solo && s.batch.size() > 1))) {
                // out of device memory now: back to the queue front, to run when a batch
                // returns memory, or one at a time when none is running
                requeue(s.batch);
                if (any_busy()) mem_wait = true;
                else solo_next = true;
            } else {
                for (auto& r : s.batch) finish(r, RS_ERROR, err, msg);
            }
            s.batch.clear();
        }
    }

    void requeue(std::vector<std::shared_ptr<Req>>& batch)
    {
        for (auto it = batch.rbegin(); it != batch.rend(); ++it) {
            (*it)->state = RS_QUEUED;
            queue.push_front(*it);
        }
        batch.clear();
    }

    // Give the slot's device memory back to the allocator (its events and pinned
    // staging stay).
    void release_slot(Slot& s)
    {
        s.sc.release_buffers();
        s.d_in.release();
        s.d_out.release();
        s.held = 0;
    }

    void stage_and_run(Slot& s)
    {
        const auto& head = s.batch.front();
        const int stride = head->dof_stride;
        long long n_wp = 0, max_T = 1;
        int nq = 0, min_chunk = 1 << 30;
        size_t lds = 0;
        bool points = false;
        s.q_off.clear();
        for (auto& r : s.batch) {
            s.q_off.push_back(nq);
            nq += r->n_queries;
            n_wp += (long long)r->wp_t.size();
            max_T = std::max(max_T, r->max_T);
            min_chunk = std::min(min_chunk, r->refs.chunk);
            lds = std::max(lds, r->refs.lds);
            points = points || r->refs.points;
        }
        // one pinned block: wp_begin | wp_t | wp_q | q_team | q_env | q_pathoff | q_focus
        BatchShape sh;
        for (auto& r : s.batch) sh.add(*r);
        const InputLayout L(sh);
        const size_t o_t = L.o_t, o_q = L.o_q, o_team = L.o_team, o_env = L.o_env, o_po = L.o_po, o_fo = L.o_fo;
        const size_t total = L.total;
        const size_t nout = s.kind == 0 ? (size_t)nq : (size_t)nq * 12;
        s.h_in.ensure(total);
        s.h_out.ensure(nout + 64);
        char* h = (char*)s.h_in.p;
        long long* hb = (long long*)h;
        int* ht = (int*)(h + o_t);
        double* hq = (double*)(h + o_q);
        const TeamDev** hteam = (const TeamDev**)(h + o_team);
        const EnvDev** henv = (const EnvDev**)(h + o_env);
        long long* hpo = (long long*)(h + o_po);
        unsigned* hfo = (unsigned*)(h + o_fo);
        long long wbase = 0, pbase = 0;
        int qi = 0;
        bool any_focus = false;
        for (auto& r : s.batch) {
            const size_t np = (size_t)r->n_queries * r->n_robots;
            for (size_t i = 0; i < np; ++i) hb[pbase + i] = r->wp_begin[i] + wbase;
            for (int k = 0; k < r->n_queries; ++k, ++qi) {
                hteam[qi] = r->refs.team;
                henv[qi] = r->refs.env;
                hpo[qi] = pbase + (long long)k * r->n_robots;
                hfo[qi] = r->focus;
                any_focus = any_focus || r->focus != 0u;
            }
            std::memcpy(ht + wbase, r->wp_t.data(), r->wp_t.size() * sizeof(int));
            std::memcpy(hq + wbase * stride, r->wp_q.data(), r->wp_q.size() * sizeof(double));
            pbase += (long long)np;
            wbase += (long long)r->wp_t.size();
        }
        hb[pbase] = wbase;
        s.d_in.ensure(total);
        s.d_out.ensure(nout);
        ensure_scratch(s.sc, (size_t)tile_bins(max_T, min_chunk), (size_t)nq, s.stream);
        s.held = s.sc.bytes() + s.d_in.cap + s.d_out.cap;
        char* d = (char*)s.d_in.p;
        HIPCHK(hipSetDevice(device));
        HIPCHK(hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, s.stream));
        CallPlan pl{};
        pl.kind = s.kind;
        pl.flags = head->flags;
        pl.dp = DevPaths{(const long long*)d, (const int*)(d + o_t), (const double*)(d + o_q), n_wp, nq, stride};
        pl.team0 = head->refs.team;
        pl.q_team = (const TeamDev* const*)(d + o_team);
        pl.env0 = nullptr;
        pl.q_env = (const EnvDev* const*)(d + o_env);
        pl.q_pathoff = (const long long*)(d + o_po);
        pl.q_focus = any_focus ? (const unsigned*)(d + o_fo) : nullptr;   // plain MV kernel otherwise
        pl.max_T = max_T;
        pl.min_chunk = min_chunk;
        pl.lds = lds;
        pl.wg_per_cu = 0;
        pl.claim = 0;
        pl.points = points;
        s.plan = pl;
        s.nout = nout;
        s.attempts = 0;
        run_batch(s);
    }

    // Queue the slot's call; its answers and the overflow counters (unresolved
    // queries, near tests pushed) come back to pinned memory.
    void run_batch(Slot& s)
    {
        serve_run_plan(ctx, s.sc, s.plan, s.d_out.p, s.stream);
        HIPCHK(hipMemcpyAsync(s.h_out.p, s.d_out.p, s.nout, hipMemcpyDeviceToHost, s.stream));
        HIPCHK(hipMemcpyAsync((char*)s.h_out.p + s.nout, (int*)s.sc.ctrl.p + 1, 2 * sizeof(int),
                              hipMemcpyDeviceToHost, s.stream));
        HIPCHK(hipEventRecord(s.done, s.stream));
        ++s.attempts;
    }

    void complete(Slot& s)
    {
        const size_t per = s.kind == 0 ? 1 : 12;
        int total = 0;
        for (auto& r : s.batch) total += r->n_queries;
        const size_t nout = (size_t)total * per;
        int cnt[2] = {0, 0};   // unresolved queries, near tests pushed
        std::memcpy(cnt, (char*)s.h_out.p + nout, sizeof(cnt));
        const int unresolved = cnt[0];
        bool cancelled = true;
        for (auto& r : s.batch) cancelled = cancelled && r->cancel_requested;
        if (unresolved && !cancelled && s.attempts < 3) {
            // the near-contact queue overflowed: enlarge it and run the batch again
            bool again = false;
            try {
                if (grow_recheck(s.sc, (unsigned)cnt[1])) {
                    run_batch(s);
                    again = true;
                }
            } catch (...) {
                (void)hipStreamSynchronize(s.stream);
            }
            if (again) return;
        }
        if (alloc->arena()) release_slot(s);
        mem_wait = false;            // memory came back: admissions resume
        for (size_t k = 0; k < s.batch.size(); ++k) {
            auto& r = s.batch[k];
            const size_t off = (size_t)s.q_off[k] * per;
            r->result.assign((unsigned char*)s.h_out.p + off, (unsigned char*)s.h_out.p + off + (size_t)r->n_queries * per);
            bool bad = false;
            if (unresolved) {
                for (int i = 0; i < r->n_queries && !bad; ++i) {
                    if (s.kind == 0) bad = r->result[i] == 3;
                    else bad = ((const int*)r->result.data())[3 * i] == -3;
                }
            }
            if (r->cancel_requested) finish(r, RS_CANCELLED, MRV_E_CANCELLED, "cancelled");
            else if (bad) finish(r, RS_ERROR, MRV_E_NOMEM, "near-contact re-evaluation queue overflow");
            else finish(r, RS_DONE, MRV_OK, "");
        }
        s.batch.clear();
        s.busy = false;
    }
};

ServeLoop::ServeLoop(mrv_ctx ctx, int device, int max_inflight, size_t budget_bytes, size_t recheck_records,
                     DevAlloc* alloc)
    : impl_(new Impl(ctx, device, max_inflight, budget_bytes, recheck_records, alloc))
{
}

ServeLoop::~ServeLoop() { delete impl_; }

mrv_status ServeLoop::submit(const mrv_request& req, const ServeRefs& refs, uint64_t* ticket)
{
    auto r = std::make_shared<Req>();
    r->kind = req.kind;
    r->team = req.team;
    r->env = req.kind == 0 ? req.env : -1;
    r->refs = refs;
    r->flags = req.flags;
    {
        const uint32_t all = refs.n_robots >= 32 ? 0xFFFFFFFFu : (1u << refs.n_robots) - 1u;
        r->focus = req.kind == 0 && (req.focus & all) != all ? req.focus : 0u;   // every robot: plain MV
    }
    r->n_queries = req.paths.n_queries;
    r->n_robots = refs.n_robots;
    const int n_robots = refs.n_robots;
    r->dof_stride = req.paths.dof_stride;
    const size_t np = (size_t)req.paths.n_queries * n_robots;
    if (req.paths.n_queries > 0) {
        r->wp_begin.assign(req.paths.wp_begin, req.paths.wp_begin + np + 1);
        r->wp_t.assign(req.paths.wp_t, req.paths.wp_t + req.paths.n_wp);
        r->wp_q.assign(req.paths.wp_q, req.paths.wp_q + (size_t)req.paths.n_wp * req.paths.dof_stride);
        for (size_t i = 0; i < np; ++i)
            r->max_T = std::max<long long>(r->max_T, (long long)r->wp_t[r->wp_begin[i + 1] - 1] + 1);
    }
    {
        // the request alone must fit the serving budget and the allocator's capacity
        BatchShape one;
        one.add(*r);
        const size_t need = batch_bytes(one, impl_->recheck_records);
        size_t cap = 0;
        impl_->alloc->stats(nullptr, nullptr, &cap);
        if (need > impl_->budget || (impl_->alloc->arena() && need > cap)) return MRV_E_NOMEM;
    }
    std::lock_guard<std::mutex> lk(impl_->mu);
    if (impl_->inflight >= impl_->max_inflight) return MRV_E_BUSY;
    r->id = impl_->next_id++;
    impl_->inflight++;
    impl_->tickets[r->id] = r;
    if (r->n_queries == 0) {
        r->state = RS_DONE;
        impl_->inflight--;
        serve_release_handles(impl_->ctx, r->team, r->env, r->kind);
    } else {
        impl_->queue.push_back(r);
        impl_->cv_work.notify_one();
    }
    *ticket = r->id;
    return MRV_OK;
}

mrv_status ServeLoop::poll(uint64_t ticket, void* out, int timeout_ms, std::string* msg)
{
    std::unique_lock<std::mutex> lk(impl_->mu);
    auto it = impl_->tickets.find(ticket);
    if (it == impl_->tickets.end()) {
        if (msg) *msg = "unknown ticket";
        return MRV_E_HANDLE;
    }
    std::shared_ptr<Req> r = it->second;
    auto finished = [&] { return r->state >= RS_DONE; };
    if (!finished() && timeout_ms != 0) {
        if (timeout_ms < 0) impl_->cv_done.wait(lk, [&] { return finished() || impl_->stop; });
        else impl_->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished);
    }
    if (!finished()) return MRV_PENDING;
    impl_->tickets.erase(r->id);
    if (r->state == RS_DONE) {
        if (out && !r->result.empty()) std::memcpy(out, r->result.data(), r->result.size());
        return MRV_OK;
    }
    if (msg) *msg = r->msg;
    return r->err;
}

mrv_status ServeLoop::cancel(uint64_t ticket)
{
    std::lock_guard<std::mutex> lk(impl_->mu);
    auto it = impl_->tickets.find(ticket);
    if (it == impl_->tickets.end()) return MRV_E_HANDLE;
    auto& r = it->second;
    if (r->state >= RS_DONE) return MRV_OK;
    r->cancel_requested = true;
    if (r->state == RS_QUEUED) {
        for (auto q = impl_->queue.begin(); q != impl_->queue.end(); ++q)
            if ((*q)->id == r->id) {
                impl_->queue.erase(q);
                break;
            }
        impl_->finish(r, RS_CANCELLED, MRV_E_CANCELLED, "cancelled");
    }
    return MRV_OK;
}

}  // namespace mrv
