// Complex value types of the multigrid kernels, parameterised on the real
// type (double: FP64 path; float: FP32 smoothing/transfers of the mixed form).
#pragma once

#include <hip/hip_runtime.h>

template <typename R>
struct Vec;
template <>
struct Vec<double> {
  using T = double2;
};
template <>
struct Vec<float> {
  using T = float2;
};

template <typename R>
__device__ __forceinline__ typename Vec<R>::T mkv(R x, R y);
template <>
__device__ __forceinline__ double2 mkv<double>(double x, double y) {
  return make_double2(x, y);
}
template <>
__device__ __forceinline__ float2 mkv<float>(float x, float y) {
  return make_float2(x, y);
}

template <typename R>
__device__ __forceinline__ typename Vec<R>::T axpy(R a, typename Vec<R>::T x, typename Vec<R>::T y) {
  return mkv<R>(fma(a, x.x, y.x), fma(a, x.y, y.y));
}
