// Device helpers shared by the kernel sources of libtacsl (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tacsl {
namespace {

constexpr int kBufferFlags = 0x00020000;  // raw 32-bit dword access, gfx9 family

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const float4* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float4*>(p), (short)0, (int)bytes, kBufferFlags);
}

// One node record: per-lane byte offset + uniform (scalar) byte offset.
__device__ __forceinline__ float4 load_node(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

__device__ __forceinline__ float lerp(float a, float b, float t) { return fmaf(t, b - a, a); }

// Element k of a row whose base is uniform; k * 4 < 2^32 (tiles hold < 2^30 taxels).
__device__ __forceinline__ float at(const float* base, uint32_t k) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (k << 2));
}
// Outputs stream out once per step: non-temporal stores keep them from
// evicting SDF lines from L2 and the memory-side cache.
__device__ __forceinline__ void put(float* base, uint32_t k, float v) {
  __builtin_nontemporal_store(v, reinterpret_cast<float*>(reinterpret_cast<char*>(base) + (k << 2)));
}

// Sum over the 64 lanes of a wavefront (all lanes active), in registers:
// data-parallel-primitive moves within quads, half-rows and rows, then the
// row broadcasts of lanes 15 and 31; lane 63 ends with the total, returned
// to every lane.  The order of the additions is fixed.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
  const int t = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF, false);
  return v + __builtin_bit_cast(float, t);
}

__device__ __forceinline__ float wave_sum(float v) {
  v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
  v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]: quad sums
  v = dpp_add<0x141, 0xF>(v);  // row_half_mirror: 8-lane sums
  v = dpp_add<0x140, 0xF>(v);  // row_mirror: 16-lane (row) sums
  v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return v + __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// FP64 sum over the 64 lanes of a wavefront (all lanes active), in the same
// fixed order as the FP32 one, the two halves of each value moved together.
__device__ __forceinline__ double wave_sum(double v) {
  v = dpp_add<0xB1, 0xF>(v);
  v = dpp_add<0x4E, 0xF>(v);
  v = dpp_add<0x141, 0xF>(v);
  v = dpp_add<0x140, 0xF>(v);
  v = dpp_add<0x142, 0xA>(v);
  v = dpp_add<0x143, 0xC>(v);
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Trilinear interpolation of corner values (index dx + 2 dy + 4 dz).
__device__ __forceinline__ float tri(float c0, float c1, float c2, float c3, float c4, float c5, float c6, float c7,
                                     float tx, float ty, float tz) {
  const float a0 = lerp(c0, c1, tx), a1 = lerp(c2, c3, tx), a2 = lerp(c4, c5, tx), a3 = lerp(c6, c7, tx);
  return lerp(lerp(a0, a1, ty), lerp(a2, a3, ty), tz);
}

}  // namespace
}  // namespace tacsl
