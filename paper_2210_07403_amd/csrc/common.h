// Shared device helpers: complex arithmetic on float2/double2, precision traits, error checks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>

namespace ibdl {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };
template <typename T> using cplx = typename Cplx<T>::type;

template <typename C> __host__ __device__ __forceinline__ C mk(decltype(C::x) re, decltype(C::x) im) {
  C c; c.x = re; c.y = im; return c;
}
template <typename V, typename S> __host__ __device__ __forceinline__ V mk4(S a, S b, S c, S d) {
  V v; v.x = a; v.y = b; v.z = c; v.w = d; return v;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return mk<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return mk<C>(a.x * s, a.y * s); }
// multiply by -i (forward transforms) or +i (inverse transforms)
template <bool INV, typename C> __device__ __forceinline__ C mul_mi(C a) {
  return INV ? mk<C>(-a.y, a.x) : mk<C>(a.y, -a.x);
}
// a * (i * r)
template <typename C> __device__ __forceinline__ C mul_ir(C a, decltype(C::x) r) { return mk<C>(-a.y * r, a.x * r); }

// Workgroups are dealt to the 8 XCDs round robin (workgroup b to XCD b mod 8).  This renumbers them
// so that each XCD takes a contiguous range of [0, n): neighbouring work items, which share markers
// or cache lines, then share an L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_chunk(int b, int n) {
  constexpr int X = 8;
  const int x = b % X, j = b / X, q = n / X, r = n % X;
  return x * q + (x < r ? x : r) + j;
}

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define IBDL_HIP(call)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      throw ::ibdl::Error(e_ == hipErrorOutOfMemory ? -3 : -4,                                  \
                          std::string(#call) + ": " + hipGetErrorString(e_));                   \
  } while (0)

#define IBDL_LAUNCH_CHECK() IBDL_HIP(hipGetLastError())

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

}  // namespace ibdl
