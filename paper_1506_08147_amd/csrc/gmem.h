// Loads and stores through pointers known to address device (global)
// memory.  Pointers read from structures or from LDS tables are generic to
// the compiler, which then emits flat memory instructions; a flat access
// counts against both the vector-memory and the LDS wait counters, so a wait
// for an LDS read also waits for every global load in flight (a prefetch
// issued before LDS work would not overlap it).  Casting to the global
// address space gives global_load / global_store instead.  Only for pointers
// into device memory.
#pragma once
#include <hip/hip_runtime.h>

namespace dg {

template <class T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

template <class T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

// HIP's double2 / float2 are structures, whose copies the compiler lowers
// through generic pointers: go through the native two-element vector.
typedef __attribute__((ext_vector_type(2))) double gv2d;
typedef __attribute__((ext_vector_type(2))) float gv2f;

template <>
__device__ __forceinline__ double2 gld(const double2* p) {
  const gv2d v = *(const __attribute__((address_space(1))) gv2d*)p;
  return make_double2(v.x, v.y);
}

template <>
__device__ __forceinline__ float2 gld(const float2* p) {
  const gv2f v = *(const __attribute__((address_space(1))) gv2f*)p;
  return make_float2(v.x, v.y);
}

template <>
__device__ __forceinline__ void gst(double2* p, double2 v) {
  gv2d w;
  w.x = v.x;
  w.y = v.y;
  *(__attribute__((address_space(1))) gv2d*)p = w;
}

template <>
__device__ __forceinline__ void gst(float2* p, float2 v) {
  gv2f w;
  w.x = v.x;
  w.y = v.y;
  *(__attribute__((address_space(1))) gv2f*)p = w;
}

}  // namespace dg
