// Global-memory access through buffer resources (gfx950).
//
// A buffer resource describes [base, base + bytes) of one array; loads and
// stores take a 32-bit byte offset and the hardware range-checks it: an
// out-of-range load returns 0 and an out-of-range store is dropped, so an
// indexing mistake can never touch memory outside the array.  It also keeps
// address arithmetic in 32-bit registers.  Every array addressed this way
// must be smaller than 4 GiB (the plan checks).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cplx.hpp"

namespace psatd {

using rsrc_t = __amdgpu_buffer_rsrc_t;
using u32x2 = unsigned int __attribute__((ext_vector_type(2)));
using u32x4 = unsigned int __attribute__((ext_vector_type(4)));

// Word 3 of a raw (unstrided) buffer descriptor on the gfx9 family: 32-bit data format.
constexpr int kRawBufferWord3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRawBufferWord3);
}

// Cache policy of a store (the buffer instructions' auxiliary bits on gfx950): kKeep, or
// kStream, the non-temporal hint, for output that the next pass reads back only after much
// more data than the caches hold has gone through them.
constexpr int kKeep = 0, kStream = 2;

template <typename T>
struct gm;

template <>
struct gm<float> {
  static __device__ __forceinline__ float ld(rsrc_t r, uint32_t i) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, i * 4u, 0, 0));
  }
  template <int P = kKeep>
  static __device__ __forceinline__ void st(rsrc_t r, uint32_t i, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, i * 4u, 0, P);
  }
  static __device__ __forceinline__ cx<float> ldc(rsrc_t r, uint32_t i) {
    return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, 0, 0));
  }
  template <int P = kKeep>
  static __device__ __forceinline__ void stc(rsrc_t r, uint32_t i, cx<float> v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, i * 8u, 0, P);
  }
  // complex element i at a further byte offset `so` held in a scalar register
  static __device__ __forceinline__ cx<float> ldc_s(rsrc_t r, uint32_t i, uint32_t so) {
    return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, (int)so, 0));
  }
  static __device__ __forceinline__ void stc_s(rsrc_t r, uint32_t i, uint32_t so, cx<float> v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, i * 8u, (int)so, 0);
  }
  // complex elements i and i + 1 in one 16-byte store
  template <int P = kKeep>
  static __device__ __forceinline__ void stc2(rsrc_t r, uint32_t i, cx<float> a, cx<float> b) {
    const u32x4 w = {__float_as_uint(a.re), __float_as_uint(a.im), __float_as_uint(b.re), __float_as_uint(b.im)};
    __builtin_amdgcn_raw_buffer_store_b128(w, r, i * 8u, 0, P);
  }
};

template <>
struct gm<double> {
  static __device__ __forceinline__ double ld(rsrc_t r, uint32_t i) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, 0, 0));
  }
  template <int P = kKeep>
  static __device__ __forceinline__ void st(rsrc_t r, uint32_t i, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, i * 8u, 0, P);
  }
  static __device__ __forceinline__ cx<double> ldc(rsrc_t r, uint32_t i) {
    return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, i * 16u, 0, 0));
  }
  template <int P = kKeep>
  static __device__ __forceinline__ void stc(rsrc_t r, uint32_t i, cx<double> v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, i * 16u, 0, P);
  }
  template <int P = kKeep>
  static __device__ __forceinline__ void stc2(rsrc_t r, uint32_t i, cx<double> a, cx<double> b) {
    stc<P>(r, i, a);
    stc<P>(r, i + 1u, b);
  }
  static __device__ __forceinline__ cx<double> ldc_s(rsrc_t r, uint32_t i, uint32_t so) {
    return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, i * 16u, (int)so, 0));
  }
  static __device__ __forceinline__ void stc_s(rsrc_t r, uint32_t i, uint32_t so, cx<double> v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, i * 16u, (int)so, 0);
  }
};

// Walks the flat indices e = e0, e0 + step, ... of a (rows x ncol) tile as
// (row, col) pairs without dividing: step = drow * ncol + dcol, dcol < ncol.
struct Walk {
  int row, col;
  __device__ __forceinline__ void next(int drow, int dcol, int ncol) {
    col += dcol;
    row += drow;
    if (col >= ncol) {
      col -= ncol;
      ++row;
    }
  }
};

}  // namespace psatd
