// Wave-uniform values for the tile kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "types.hpp"

namespace bsm {

// Values the whole wave agrees on, made explicit so that buffer descriptors built from them stay
// in scalar registers.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint32_t uni(uint32_t v) { return uint32_t(__builtin_amdgcn_readfirstlane(int(v))); }
__device__ inline uint64_t uni(uint64_t v) {
  uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
  uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v >> 32))));
  return (uint64_t(hi) << 32) | lo;
}
template <typename P>
__device__ inline P* uni_ptr(P* p) {
  return reinterpret_cast<P*>(uni(reinterpret_cast<uint64_t>(p)));
}
// A task, its operands and its triples are the same for the whole wave: keeping them in scalar
// registers keeps the per-chunk address arithmetic on the scalar unit.
__device__ inline Triple uni(const Triple& t) {
  Triple r;
  r.a = uni(t.a);
  r.b = uni(t.b);
  return r;
}
__device__ inline Item uni(const Item& it) {
  Item r;
  r.c_off = int64_t(uni(uint64_t(it.c_off)));
  r.tri_begin = uni(it.tri_begin);
  r.tri_count = uni(it.tri_count);
  r.r0 = uint16_t(uni(uint32_t(it.r0)));
  r.c0 = uint16_t(uni(uint32_t(it.c0)));
  r.h = uint16_t(uni(uint32_t(it.h)));
  r.w = uint16_t(uni(uint32_t(it.w)));
  r.ldc = uint16_t(uni(uint32_t(it.ldc)));
  r.ldm = uint16_t(uni(uint32_t(it.ldm)));
  r.product = uni(it.product);
  return r;
}
__device__ inline ProductArgs uni(const ProductArgs& p) {
  ProductArgs r;
  r.A = uni_ptr(p.A);
  r.B = uni_ptr(p.B);
  r.C = uni_ptr(p.C);
  r.P = uni_ptr(p.P);
  r.alpha = __builtin_bit_cast(double, uni(__builtin_bit_cast(uint64_t, p.alpha)));
  r.a_plane = int64_t(uni(uint64_t(p.a_plane)));
  r.b_plane = int64_t(uni(uint64_t(p.b_plane)));
  r.c_f32 = uni(p.c_f32);
  r.pad_ = 0;
  return r;
}

// The epilogue's store of one C element: alpha * sum (+ the previous C), rounded once to C's type.
__device__ inline void store_c(const ProductArgs& pa, int64_t e, double v, int accumulate) {
  if (pa.c_f32) {
    float* c = static_cast<float*>(pa.C);
    c[e] = float(accumulate ? v + double(c[e]) : v);
  } else {
    double* c = static_cast<double*>(pa.C);
    c[e] = accumulate ? v + c[e] : v;
  }
}

// Marks task idx as executed once more (one lane; no return value, so nothing waits on it).
__device__ inline void count_task(uint32_t* done, int idx) {
  if (done) __hip_atomic_fetch_add(done + idx, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Triple q of a k-list through the scalar cache (the address is uniform): its wait counts
// against the scalar and LDS operations only, not behind the staging loads in flight.
__device__ inline Triple scalar_triple(const Triple* tri, uint32_t q) {
  using TriK = const __attribute__((address_space(4))) Triple;
  TriK* t = (TriK*)tri;
  Triple r;
  r.a = t[q].a;
  r.b = t[q].b;
  return r;
}

}  // namespace bsm
