// Buffer-resource memory access for the tiled executors.
//
// A raw buffer resource (base, size in bytes) gives 32-bit byte offsets held
// in VGPRs and hardware range checking: an offset at or past the size reads 0
// and drops a store.  The executors use that to clip tiles at the array edge
// without clamping, and to mask stores by replacing the offset with OOB.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "common.hpp"

namespace pcot {

using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int OOB = 0x7FFFFFF0;  // byte offset beyond any field the executors accept

// Cache policy of every executor access: SC1, coherent at device (agent)
// scope.  Tiles on different XCDs exchange faces through HBM/MALL; with
// device-coherent loads and write-through stores a tile only has to wait for
// its stores to be acknowledged before it signals, instead of writing back
// and invalidating its XCD's whole L2 around every tile.
constexpr int CPOL_DEV = 16;

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    // word 3: 32-bit data format, no swizzle (raw, untyped access)
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename S> struct IO;

template <> struct IO<double> {
    static __device__ __forceinline__ double ld(rsrc_t r, int off) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, CPOL_DEV));
    }
    static __device__ __forceinline__ void st(rsrc_t r, int off, double v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, CPOL_DEV);
    }
};

template <> struct IO<float> {
    static __device__ __forceinline__ float ld(rsrc_t r, int off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, CPOL_DEV));
    }
    static __device__ __forceinline__ void st(rsrc_t r, int off, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, CPOL_DEV);
    }
};

template <> struct IO<uint16_t> {
    static __device__ __forceinline__ float ld(rsrc_t r, int off) {
        return bf16_to_f32(__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, CPOL_DEV));
    }
    static __device__ __forceinline__ void st(rsrc_t r, int off, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(f32_to_bf16(v), r, off, 0, CPOL_DEV);
    }
};

}  // namespace pcot
