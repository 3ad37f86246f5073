// gmt_host.hpp -- host helpers shared by the library's translation units:
// the thread-local error message, HIP error checks and device buffers drawn
// from the installed allocator (gmt_set_allocator).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "../../include/gmt.h"

namespace gmt_host {

// record a formatted message for gmt_last_error() and return `st`
gmt_status fail(gmt_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    gmt_allocator a{nullptr, nullptr, nullptr};
    bool view = false;  // a part of another buffer: never freed on its own
};

// a view of `bytes` bytes at `off` inside `block`
inline DevBuf dev_view(const DevBuf &block, size_t off, size_t bytes) {
    DevBuf v;
    v.p = (char *)block.p + off;
    v.bytes = bytes;
    v.view = true;
    return v;
}

// allocate `bytes` (rounded up to 256) with the allocator installed now
gmt_status dev_alloc(DevBuf &b, size_t bytes, hipStream_t s);
// return a buffer to the allocator that produced it (nothing after gmt_shutdown)
void dev_free(DevBuf &b, hipStream_t s);
// true once gmt_shutdown has run
bool shut_down();

}  // namespace gmt_host

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return gmt_host::fail(GMT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define TRY(expr)                      \
    do {                               \
        gmt_status st_ = (expr);       \
        if (st_ != GMT_OK) return st_; \
    } while (0)
