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

// A device-memory pointer seen as a global-address-space pointer.  Accesses
// through it compile to global_load/global_store, which the compiler keeps
// in flight across LDS accesses; accesses through a generic pointer might
// alias LDS, so each one waits for the LDS traffic before it.
// (The host pass, which only checks the kernels' source, sees the plain
// pointer: address spaces are a device-side notion.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gbl(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
#else
template <typename T>
__device__ __forceinline__ T* gbl(T* p) {
  return p;
}
#endif
