// Shared pieces of the HIP kernels: error reporting, dispatch over the limb
// count, wave-level reductions in a fixed order, plane addressing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "../../include/mdseries.h"
#include "md.hpp"

namespace mds {

// thread-local message behind md_last_error()
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

// check a launch; returns MD_OK or MD_EHIP
int check_launch(const char *what);

// Largest dynamic LDS (bytes) a kernel of this library may request on the
// current device: the device's per-workgroup limit less 4 KiB kept for the
// kernels' static LDS (65536 - 4096 if the attribute cannot be read).
size_t lds_limit();

inline bool valid_m(int m) {
  return m == 1 || m == 2 || m == 3 || m == 4 || m == 5 || m == 8 || m == 10;
}

// Calls f(std::integral_constant<int, M>{}) for the runtime limb count m.
template <class F>
int dispatch_m(int m, F &&f) {
  switch (m) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 10: return f(std::integral_constant<int, 10>{});
    default: return fail(MD_EINVAL, "limb count m=%d not in {1,2,3,4,5,8,10}", m);
  }
}

constexpr int WAVE = 64;

// A gate word in device memory: kernels of a step enqueued ahead of time
// return at once while it is zero (the Newton protocol switches a converged
// degree's remaining steps off this way).  NULL: always open.
__device__ __forceinline__ bool gate_closed(const int32_t *gate) {
  return gate && *gate == 0;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// The largest v over the wave, the same on every lane (all lanes active).
__device__ __forceinline__ int wave_max_int(int v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int t = __shfl_xor(v, o, WAVE);
    v = v > t ? v : t;
  }
  return __builtin_amdgcn_readfirstlane(v);
}

template <int M>
__device__ __forceinline__ mdr<M> shfl_down_r(const mdr<M> &a, int off) {
  mdr<M> z;
#pragma unroll
  for (int i = 0; i < M; ++i) z.v[i] = __shfl_down(a.v[i], off, WAVE);
  return z;
}

template <int M>
__device__ __forceinline__ mdc<M> shfl_down_c(const mdc<M> &a, int off) {
  mdc<M> z;
  z.re = shfl_down_r<M>(a.re, off);
  z.im = shfl_down_r<M>(a.im, off);
  return z;
}

template <int M>
__device__ __forceinline__ mdc<M> shfl_c(const mdc<M> &a, int src) {
  mdc<M> z;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    z.re.v[i] = __shfl(a.re.v[i], src, WAVE);
    z.im.v[i] = __shfl(a.im.v[i], src, WAVE);
  }
  return z;
}

template <int M>
__device__ __forceinline__ mdr<M> shfl_r(const mdr<M> &a, int src) {
  mdr<M> z;
#pragma unroll
  for (int i = 0; i < M; ++i) z.v[i] = __shfl(a.v[i], src, WAVE);
  return z;
}

// Sum over the lanes of a segment of `seg` lanes (a power of two <= 64):
// s_l += s_{l+o} for o = seg/2, ..., 1; the segment's first lane holds the
// sum.  The order is fixed, so the bits do not depend on timing.
template <int M>
__device__ __forceinline__ mdc<M> seg_reduce_c(mdc<M> s, int seg) {
  for (int o = seg >> 1; o > 0; o >>= 1) {
    const mdc<M> t = shfl_down_c<M>(s, o);
    if ((lane_id() & (seg - 1)) < o) s = c_add<M>(s, t);
  }
  return s;
}

template <int M>
__device__ __forceinline__ mdr<M> seg_reduce_r(mdr<M> s, int seg) {
  for (int o = seg >> 1; o > 0; o >>= 1) {
    const mdr<M> t = shfl_down_r<M>(s, o);
    if ((lane_id() & (seg - 1)) < o) s = md_add<M>(s, t);
  }
  return s;
}

__host__ __device__ inline int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

}  // namespace mds
