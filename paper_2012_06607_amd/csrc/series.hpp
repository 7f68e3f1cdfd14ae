// Truncated power series on the device (Section 3).
#pragma once

#include "common.hpp"

namespace mds {

// A series of complex multiple doubles inside a plane tensor with E
// elements: coefficient k is element base + k*stride.
struct SRef {
  const double *p;
  long E;
  long base;
  long stride;
};

template <int M>
__device__ __forceinline__ mdc<M> sload(const SRef &r, int k) {
  return cload<M>(r.p, r.E, r.base + long(k) * r.stride);
}

// Coefficient k of the product x(t) y(t) with deg x <= dx:
// z_k = x_0 y_k + x_1 y_{k-1} + ... + x_{min(k,dx)} y_{k-min(k,dx)},
// started from the first product, added in increasing i (Section 3).
template <int M>
__device__ __forceinline__ mdc<M> conv_coef(const SRef &x, int dx, const SRef &y, int k) {
  mdc<M> acc = c_mul<M>(sload<M>(x, 0), sload<M>(y, k));
  const int top = k < dx ? k : dx;
  for (int i = 1; i <= top; ++i) acc = c_add<M>(acc, c_mul<M>(sload<M>(x, i), sload<M>(y, k - i)));
  return acc;
}

// Thread p of the ceil((d+1)/2) threads of one product computes the
// coefficients k = p and k = d - p, which together cost d+2 multiplications
// whatever p is.
__device__ __forceinline__ int pairs_of(int d) { return (d + 2) / 2; }
inline int pairs_of_host(int d) { return (d + 2) / 2; }

}  // namespace mds
