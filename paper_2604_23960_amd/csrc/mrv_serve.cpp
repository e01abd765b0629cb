// Serving loop behind mrv_submit / mrv_poll.
#include "mrv_runtime.hpp"

namespace mrv {

struct ServeLoop::Impl {};

ServeLoop::ServeLoop(mrv_ctx, int, int, size_t) : impl_(nullptr) {}
ServeLoop::~ServeLoop() {}
mrv_status ServeLoop::submit(const mrv_request&, int, uint64_t*) { return MRV_E_INVALID; }
mrv_status ServeLoop::poll(uint64_t, void*, int, std::string* msg)
{
    if (msg) *msg = "unknown ticket";
    return MRV_E_HANDLE;
}
mrv_status ServeLoop::cancel(uint64_t) { return MRV_E_HANDLE; }

}  // namespace mrv
