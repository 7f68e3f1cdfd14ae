// A dot product spread over the four waves of a workgroup (the single-path
// stage products of the staggered solve and of its adjoint).
#pragma once

#include "gang.hpp"

namespace mds {

// A dot product of len <= 64 complex terms on the four waves of a
// 256-thread workgroup: term c = x_c y_c (conj(x_c) y_c when CONJ) on wave
// c mod 4, lanes 4 (c / 4) + q, lane q forming real product q as c_mul
// orders them (re*re, im*im, re*im, im*re), the real part of the term then
// on lane q = 0 and the imaginary part on q = 2, the sum over c in
// seg_reduce's order (seg = the power of two >= len, at least 8).  The
// result ends on wave 0, lanes 0 (re) and 2 (im), with the bits of a
// one-segment c_mul / c_add sum.  ld(c, x, y) loads the operands of term c.
template <int M, bool CONJ, class Load>
__device__ __forceinline__ mdr<M> dot4(int len, int seg, Load ld, double *xch) {
  const int lane = lane_id(), w = threadIdx.x / WAVE, q = lane & 3;
  const int c = 4 * (lane >> 2) + w;
  const bool ok = c < len;
  mdc<M> x = c_zero<M>(), y = c_zero<M>();
  if (ok) ld(c, x, y);
  mdr<M> xi = x.im;
  if (CONJ) xi = md_neg<M>(xi);
  const mdr<M> p = md_mul<M>((q & 1) ? xi : x.re, (q == 0 || q == 3) ? y.re : y.im);
  mdr<M> t = shfl_down_r<M>(p, 1);
  if (q == 0) t = md_neg<M>(t);
  const mdr<M> s = ok ? md_add<M>(p, t) : md_zero<M>();
  return lead4_sum<M>(s, seg, w, lane, true, xch);
}

}  // namespace mds
