// Internal declarations of the helpers outside the step kernels: the fixed
// workspace of the allocation-free minimizer and the streaming-copy kernel.
#pragma once

#include <stdint.h>

#include "lqfire.h"

namespace lq {

// Device address of the fixed workspace of lq_minimize_noalloc on `device`
// (which must be current): looked up once per device, then cached.
int noalloc_workspace(int device, void** out);

// Streams of the copy-ceiling kernel (lq_stream_copy).
constexpr int STREAMS_MAX = 16;
struct StreamSet {
    const void* src[STREAMS_MAX];
    void* dst[STREAMS_MAX];
};
// Enqueues the copy of ns streams of `bytes` each (width 4 or 16 bytes per
// lane per access); the caller has checked the arguments.
int launch_stream_copy(const StreamSet& p, int ns, int64_t bytes, int width, void* stream);

}  // namespace lq
