// Shared device/host helpers of libmmf (internal header, not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include "mmf.h"

#define MMF_HIP_TRY(expr)                                   \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return MMF_ERR_HIP;               \
  } while (0)

namespace mmf {
// After every kernel launch: nonzero if the launch failed.  With the opt-in
// profiling throttle (mmf_profile_sync_every) it also waits for the device
// every n launches.
int launch_check();
}  // namespace mmf

#define MMF_LAUNCH_CHECK()                                  \
  do {                                                      \
    if (mmf::launch_check() != 0) return MMF_ERR_HIP;       \
  } while (0)
// the same with a clean-up statement before the error return
#define MMF_LAUNCH_CHECK_OR(cleanup)                        \
  do {                                                      \
    if (mmf::launch_check() != 0) {                         \
      cleanup;                                              \
      return MMF_ERR_HIP;                                   \
    }                                                       \
  } while (0)

// Global-memory pointer.  A pointer read from a device table is generic to the
// compiler, and a generic (FLAT) access counts against the same wait counter as
// LDS and scalar loads, so every wait for an LDS read would also wait for the
// HBM loads and stores still in flight.  Kernels view such pointers through
// this qualifier (all device buffers of the library are global memory).  The
// host pass, which also reads device code, takes it as a plain pointer.
#if defined(__HIP_DEVICE_COMPILE__)
#define MMF_GLOBAL __attribute__((address_space(1)))
#else
#define MMF_GLOBAL
#endif

namespace mmf {

// Value behind a global pointer (the operands of a conditional expression
// cannot mix address spaces).
template <typename T>
__device__ __forceinline__ T gload(const MMF_GLOBAL T *p) { return *p; }

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

// Complex arithmetic on interleaved (re, im) pairs of R = double or float.
template <typename R>
struct alignas(2 * sizeof(R)) cx {
  R re, im;
};
typedef cx<double> cd;
typedef cx<float> cf;

template <typename R>
__host__ __device__ inline cx<R> cmk(R r, R i) { cx<R> z; z.re = r; z.im = i; return z; }
__host__ __device__ inline cd cmake(double r, double i) { return cmk<double>(r, i); }
template <typename R>
__device__ inline cx<R> cadd(cx<R> a, cx<R> b) { return cmk<R>(a.re + b.re, a.im + b.im); }
template <typename R>
__device__ inline cx<R> csub(cx<R> a, cx<R> b) { return cmk<R>(a.re - b.re, a.im - b.im); }
template <typename R>
__device__ inline cx<R> cmul(cx<R> a, cx<R> b) {
  return cmk<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// conj(a) * b
template <typename R>
__device__ inline cx<R> cmulc(cx<R> a, cx<R> b) {
  return cmk<R>(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename R>
__device__ inline cx<R> cconj(cx<R> a) { return cmk<R>(a.re, -a.im); }
template <typename R>
__device__ inline cx<R> cscale(cx<R> a, R s) { return cmk<R>(a.re * s, a.im * s); }
template <typename R>
__device__ inline R cabs2(cx<R> a) { return a.re * a.re + a.im * a.im; }

__device__ inline cd ldz(const mmf_z *p) {
  const double2 v = *reinterpret_cast<const double2 *>(p);
  return cmake(v.x, v.y);
}
__device__ inline void stz(mmf_z *p, cd v) {
  double2 t; t.x = v.re; t.y = v.im;
  *reinterpret_cast<double2 *>(p) = t;
}
// generic complex load/store on cx<R> storage (16 B for double, 8 B for float)
template <typename R>
__device__ inline cx<R> ldc(const cx<R> *p) { return *p; }
template <typename R>
__device__ inline void stc(cx<R> *p, cx<R> v) { *p = v; }

// Wavefront-wide sum (64 lanes) with DPP/shuffle via __shfl_xor.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// 256-byte aligned carving of a caller workspace.
struct Carver {
  char *base;
  size_t off;
  explicit Carver(void *p) : base((char *)p), off(0) {}
  template <class T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *r = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return r;
  }
  size_t used() const { return (off + 255) & ~(size_t)255; }
};

}  // namespace mmf
