// Single multiple-double operations, one per element (the units of Table 1),
// and the 2-norm of a complex vector (Section 2's example).
#include "common.hpp"

namespace mds {

template <int M>
__global__ void __launch_bounds__(256) k_elementwise(int op, long count,
                                                     const double *__restrict__ a,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ out) {
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < count;
       e += long(gridDim.x) * blockDim.x) {
    if (op <= MD_OP_MULD) {
      const mdr<M> x = rload<M>(a, count, e);
      mdr<M> y = md_zero<M>();
      if (op != MD_OP_SQRT && op != MD_OP_RSQRT) y = rload<M>(b, count, e);
      mdr<M> z;
      switch (op) {
        case MD_OP_ADD: z = md_add<M>(x, y); break;
        case MD_OP_SUB: z = md_sub<M>(x, y); break;
        case MD_OP_MUL: z = md_mul<M>(x, y); break;
        case MD_OP_DIV: z = md_div<M>(x, y); break;
        case MD_OP_SQRT: z = md_sqrt<M>(x); break;
        case MD_OP_RSQRT: z = md_rsqrt<M>(x); break;
        default: z = md_muld<M>(x, y.v[0]); break;
      }
      rstore<M>(out, count, e, z);
    } else {
      const mdc<M> x = cload<M>(a, count, e);
      if (op == MD_OP_CABS2) {
        rstore<M>(out, count, e, c_abs2<M>(x));
        continue;
      }
      const mdc<M> y = cload<M>(b, count, e);
      mdc<M> z;
      switch (op) {
        case MD_OP_CADD: z = c_add<M>(x, y); break;
        case MD_OP_CSUB: z = c_sub<M>(x, y); break;
        case MD_OP_CMUL: z = c_mul<M>(x, y); break;
        default: z = c_div<M>(x, y); break;
      }
      cstore<M>(out, count, e, z);
    }
  }
}

// One workgroup: thread t sums |x_e|^2 over e = t, t+256, ... in order, the
// 256 partial sums are added pairwise (s_t += s_{t+o}, o = 128, ..., 1), and
// thread 0 takes the square root.
template <int M>
__global__ void __launch_bounds__(256) k_norm2(long count, const double *__restrict__ x,
                                               double *__restrict__ out) {
  __shared__ mdr<M> sh[256];
  const int t = threadIdx.x;
  mdr<M> s = md_zero<M>();
  if (t < count) {
    s = c_abs2<M>(cload<M>(x, count, t));
    for (long e = t + 256; e < count; e += 256) s = md_add<M>(s, c_abs2<M>(cload<M>(x, count, e)));
  }
  sh[t] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) sh[t] = md_add<M>(sh[t], sh[t + o]);
    __syncthreads();
  }
  if (t == 0) rstore<M>(out, 1, 0, md_sqrt<M>(sh[0]));
}

}  // namespace mds

using namespace mds;

extern "C" int md_elementwise(int m, int op, int64_t count, const double *a, const double *b,
                              double *out, void *stream) {
  if (count < 0 || op < MD_OP_ADD || op > MD_OP_CABS2)
    return fail(MD_EINVAL, "md_elementwise: bad op %d or count %lld", op, (long long)count);
  if (!a || !out || (!b && op != MD_OP_SQRT && op != MD_OP_RSQRT && op != MD_OP_CABS2))
    return fail(MD_ENULL, "md_elementwise: null pointer");
  if (count == 0) return MD_OK;
  return dispatch_m(m, [&](auto Mc) {
    constexpr int M = decltype(Mc)::value;
    long blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_elementwise<M><<<dim3(unsigned(blocks)), dim3(256), 0, (hipStream_t)stream>>>(
        op, long(count), a, b, out);
    return check_launch("md_elementwise");
  });
}

extern "C" int md_norm2(int m, int64_t count, const double *x, double *out, void *stream) {
  if (count < 1) return fail(MD_EINVAL, "md_norm2: count %lld < 1", (long long)count);
  if (!x || !out) return fail(MD_ENULL, "md_norm2: null pointer");
  return dispatch_m(m, [&](auto Mc) {
    constexpr int M = decltype(Mc)::value;
    k_norm2<M><<<dim3(1), dim3(256), 0, (hipStream_t)stream>>>(long(count), x, out);
    return check_launch("md_norm2");
  });
}
