// Raw buffer loads of gfx950 used by the operator kernels (device code).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fr {

// Word 3 of a buffer resource for untyped (raw) loads on CDNA: only a
// non-zero data format (32-bit) is required; no swizzle, no stride.
constexpr int kRawBufferWord3 = 0x00020000;

// One value at byte offset `off` of the row whose address the resource `rs`
// holds.  The row address is wave-uniform (scalar registers) and the offset
// is the lane's, so a gather costs one instruction and no vector address
// arithmetic.
template <typename TB>
__device__ inline TB load_row(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t soff = 0) {
  if constexpr (sizeof(TB) == 8) {
    return __builtin_bit_cast(TB, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, (int)soff, 0));
  } else {
    return __builtin_bit_cast(TB, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, (int)soff, 0));
  }
}

// A buffer resource over `nrec` bytes at p, both wave-uniform, built from
// scalar registers: readfirstlane keeps the compiler from placing a value it
// cannot prove uniform in vector registers, which would turn every load
// through the resource into a loop over lanes.
__device__ inline __amdgpu_buffer_rsrc_t uniform_rsrc(const void *p, int nrec) {
  const uint64_t a = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), 0,
                                           __builtin_amdgcn_readfirstlane(nrec),
                                           kRawBufferWord3);
}

}  // namespace fr
