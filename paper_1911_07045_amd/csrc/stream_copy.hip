// Streaming ceiling of the FIRE step's access pattern (lq_stream_copy): plain
// copies of up to 16 device buffers with the raw buffer accesses and the
// non-temporal store policy of the step kernel, so that its time says what
// streaming the step's traffic reaches on this device.
#include <hip/hip_runtime.h>

#include "lq_aux.h"

namespace lq {

namespace {

// Non-temporal store policy: bit 1 of the buffer instruction's cache-policy
// operand on gfx950, the policy of the step kernel's stores of q, v, F.
#ifndef LQ_COPY_POLICY
#define LQ_COPY_POLICY 2
#endif
constexpr int STORE_POLICY = LQ_COPY_POLICY;
// Blocks of one launch at most (grid-stride beyond).
#ifndef LQ_COPY_GRID
#define LQ_COPY_GRID 8192
#endif

__device__ __forceinline__ __amdgpu_buffer_rsrc_t stream_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// Stream i of `ns` goes from src[i] to dst[i], W bytes per lane per access
// (4: one FP32 value per lane, as the FP32 step kernel loads its fields; 8:
// one FP64 value; 16: whole 16-byte pieces); the loads of every stream are
// issued before the stores.
// `bytes` is at most 2^31, so the grid-stride offset never wraps.
template <int W>
__global__ __launch_bounds__(256) void k_stream_copy(StreamSet p, int ns, uint32_t bytes) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const uint32_t stride = gridDim.x * 256u * (uint32_t)W;
    for (uint32_t off = (blockIdx.x * 256u + threadIdx.x) * (uint32_t)W; off < bytes; off += stride) {
        if constexpr (W == 16) {
            u32x4 v[STREAMS_MAX];
#pragma unroll
            for (int i = 0; i < STREAMS_MAX; ++i)
                if (i < ns) v[i] = __builtin_amdgcn_raw_buffer_load_b128(stream_rsrc(p.src[i], bytes), (int)off, 0, 0);
#pragma unroll
            for (int i = 0; i < STREAMS_MAX; ++i)
                if (i < ns)
                    __builtin_amdgcn_raw_buffer_store_b128(v[i], stream_rsrc(p.dst[i], bytes), (int)off, 0,
                                                           STORE_POLICY);
        } else if constexpr (W == 8) {
            typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
            u32x2 v[STREAMS_MAX];
#pragma unroll
            for (int i = 0; i < STREAMS_MAX; ++i)
                if (i < ns) v[i] = __builtin_amdgcn_raw_buffer_load_b64(stream_rsrc(p.src[i], bytes), (int)off, 0, 0);
#pragma unroll
            for (int i = 0; i < STREAMS_MAX; ++i)
                if (i < ns)
                    __builtin_amdgcn_raw_buffer_store_b64(v[i], stream_rsrc(p.dst[i], bytes), (int)off, 0,
                                                          STORE_POLICY);
        } else {
            uint32_t v[STREAMS_MAX];
#pragma unroll
            for (int i = 0; i < STREAMS_MAX; ++i)
                if (i < ns) v[i] = __builtin_amdgcn_raw_buffer_load_b32(stream_rsrc(p.src[i], bytes), (int)off, 0, 0);
#pragma unroll
            for (int i = 0; i < STREAMS_MAX; ++i)
                if (i < ns)
                    __builtin_amdgcn_raw_buffer_store_b32(v[i], stream_rsrc(p.dst[i], bytes), (int)off, 0,
                                                          STORE_POLICY);
        }
    }
}

}  // namespace

int launch_stream_copy(const StreamSet& p, int ns, int64_t bytes, int width, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    // enough blocks to fill every compute unit many times over; grid-stride beyond
    const int64_t per_block = 256 * (int64_t)width;
    const int64_t need = (bytes + per_block - 1) / per_block;
    const int g = (int)(need < LQ_COPY_GRID ? (need > 0 ? need : 1) : LQ_COPY_GRID);
    if (width == 16) k_stream_copy<16><<<g, 256, 0, s>>>(p, ns, (uint32_t)bytes);
    else if (width == 8) k_stream_copy<8><<<g, 256, 0, s>>>(p, ns, (uint32_t)bytes);
    else k_stream_copy<4><<<g, 256, 0, s>>>(p, ns, (uint32_t)bytes);
    return hipGetLastError() == hipSuccess ? LQ_OK : LQ_EHIP;
}

}  // namespace lq
