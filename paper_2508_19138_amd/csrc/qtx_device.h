// Device-side helpers shared by the HIP kernels of the RGF library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtx {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

struct zc {               // complex128 scalar passed by value to kernels
  double re, im;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(zc s, double2 a) {
  return make_double2(s.re * a.x - s.im * a.y, s.re * a.y + s.im * a.x);
}
}  // namespace qtx
