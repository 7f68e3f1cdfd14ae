// Truncated series products z[c] = x[c] y[c] mod t^{d+1} (Section 3).
#include "series.hpp"

namespace mds {

template <int M>
__global__ void __launch_bounds__(256) k_convolve(int d, long count, const double *__restrict__ x,
                                                  const double *__restrict__ y,
                                                  double *__restrict__ z) {
  const int P = pairs_of(d);
  const long E = count * (d + 1);
  const long total = count * P;
  for (long g = blockIdx.x * long(blockDim.x) + threadIdx.x; g < total;
       g += long(gridDim.x) * blockDim.x) {
    const long c = g / P;
    const int p = int(g - c * P);
    const SRef xs{x, E, c * (d + 1), 1};
    const SRef ys{y, E, c * (d + 1), 1};
    cstore<M>(z, E, c * (d + 1) + p, conv_coef<M>(xs, d, ys, p));
    if (d - p != p) cstore<M>(z, E, c * (d + 1) + (d - p), conv_coef<M>(xs, d, ys, d - p));
  }
}

}  // namespace mds

using namespace mds;

extern "C" int md_series_convolve(int m, int d, int64_t count, const double *x, const double *y,
                                  double *z, void *stream) {
  if (d < 0 || count < 0) return fail(MD_EINVAL, "md_series_convolve: d=%d count=%lld", d,
                                      (long long)count);
  if (count == 0) return dispatch_m(m, [](auto) { return MD_OK; });
  if (!x || !y || !z) return fail(MD_ENULL, "md_series_convolve: null pointer");
  return dispatch_m(m, [&](auto Mc) {
    constexpr int M = decltype(Mc)::value;
    const long total = long(count) * pairs_of_host(d);
    long blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_convolve<M><<<dim3(unsigned(blocks)), dim3(256), 0, (hipStream_t)stream>>>(d, long(count), x,
                                                                                  y, z);
    return check_launch("md_series_convolve");
  });
}
