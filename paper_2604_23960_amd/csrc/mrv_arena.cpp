// Device memory of a context: sub-allocation inside a caller-owned arena, or
// hipMalloc per buffer when the caller gives none.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <iterator>

#include "mrv_runtime.hpp"

namespace mrv {

namespace {
constexpr size_t kAlign = 256;
inline size_t round_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }
}  // namespace

void DevAlloc::use_arena(void* base, size_t bytes)
{
    std::lock_guard<std::mutex> lk(mu_);
    // the usable range starts at the first aligned address
    const uintptr_t b = (uintptr_t)base;
    const uintptr_t a = (b + kAlign - 1) & ~(uintptr_t)(kAlign - 1);
    const size_t skip = (size_t)(a - b);
    base_ = (char*)a;
    cap_ = bytes > skip ? (bytes - skip) & ~(kAlign - 1) : 0;
    free_.clear();
    if (cap_) free_[0] = cap_;
    live_.clear();
    used_ = peak_ = 0;
}

void* DevAlloc::alloc(size_t bytes)
{
    const size_t want = round_up(std::max<size_t>(bytes, 1));
    std::lock_guard<std::mutex> lk(mu_);
    if (!base_) {
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess)
            throw Err{MRV_E_NOMEM, "device allocation of " + std::to_string(want) + " bytes failed"};
        live_[(uintptr_t)p] = want;
        used_ += want;
        peak_ = std::max(peak_, used_);
        return p;
    }
    // first fit over the free ranges (offset -> size), kept coalesced
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < want) continue;
        const size_t off = it->first;
        const size_t rest = it->second - want;
        free_.erase(it);
        if (rest) free_[off + want] = rest;
        live_[(uintptr_t)(base_ + off)] = want;
        used_ += want;
        peak_ = std::max(peak_, used_);
        return base_ + off;
    }
    throw Err{MRV_E_NOMEM, "device arena exhausted: " + std::to_string(want) + " bytes requested, " +
                               std::to_string(cap_ - used_) + " of " + std::to_string(cap_) + " free"};
}

void DevAlloc::free(void* p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = live_.find((uintptr_t)p);
    if (it == live_.end()) return;
    const size_t n = it->second;
    live_.erase(it);
    used_ -= n;
    if (!base_) {
        (void)hipFree(p);
        return;
    }
    size_t off = (size_t)((char*)p - base_), len = n;
    // merge with the free neighbours
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == off + len) {
        len += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            off = prev->first;
            len += prev->second;
            free_.erase(prev);
        }
    }
    free_[off] = len;
}

size_t DevAlloc::largest_free() const
{
    std::lock_guard<std::mutex> lk(mu_);
    if (!base_) return SIZE_MAX;
    size_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
}

void DevAlloc::stats(size_t* used, size_t* peak, size_t* capacity) const
{
    std::lock_guard<std::mutex> lk(mu_);
    if (used) *used = used_;
    if (peak) *peak = peak_;
    if (capacity) *capacity = base_ ? cap_ : 0;
}

void DevBuf::ensure(size_t bytes)
{
    if (bytes <= cap) return;
    release();
    const size_t want = std::max<size_t>(bytes, 256);
    if (a) {
        p = a->alloc(want);
    } else if (hipMalloc(&p, want) != hipSuccess) {
        p = nullptr;
        throw Err{MRV_E_NOMEM, "device allocation of " + std::to_string(want) + " bytes failed"};
    }
    cap = want;
}

void DevBuf::release()
{
    if (p) {
        if (a) a->free(p);
        else (void)hipFree(p);
    }
    p = nullptr;
    cap = 0;
}

}  // namespace mrv
