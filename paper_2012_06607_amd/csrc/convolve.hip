// Truncated series products z[c] = x[c] y[c] mod t^{d+1} (Section 3).
//
// Coefficient k is z_k = x_0 y_k + x_1 y_{k-1} + ... + x_k y_0, started from
// the first product and added in increasing i.  Its k + 1 products do not
// depend on each other; only the additions form a chain.  So the workgroups
// of one series take pairs of coefficients (k, d - k), d + 2 products a
// pair, and form every product of their coefficients at once in LDS: the
// four real products of each complex product on four lanes, then its real
// part p1 - p2 and imaginary part p3 + p4 on two (as c_mul forms them);
// then one lane per coefficient and part adds them up in order of i.
// The bits are those of the sequential definition; the sequential part is
// the k additions.  Series too long for LDS take the plain form, one thread
// per pair of coefficients.
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

// Pairs p = part, part + nparts, ... < P of one series, their coefficients
// in the order p, d - p (once when equal); `base` of a coefficient is the
// number of products of the coefficients before it.
struct ConvPart {
  int d, P, part, nparts;
  // number of coefficients and products of this part
  __device__ void sizes(int &ncoef, int &nprod) const {
    ncoef = 0;
    nprod = 0;
    for (int p = part; p < P; p += nparts) {
      ncoef += 1;
      nprod += p + 1;
      if (d - p != p) {
        ncoef += 1;
        nprod += d - p + 1;
      }
    }
  }
  // coefficient j: its degree k and base
  __device__ void coef(int j, int &k, int &base) const {
    base = 0;
    int idx = 0;
    for (int p = part; p < P; p += nparts) {
      if (idx == j) {
        k = p;
        return;
      }
      base += p + 1;
      ++idx;
      if (d - p != p) {
        if (idx == j) {
          k = d - p;
          return;
        }
        base += d - p + 1;
        ++idx;
      }
    }
    k = -1;
  }
  // the coefficient that product slot s belongs to: its degree, base
  __device__ void slot(int s, int &k, int &base) const {
    base = 0;
    for (int p = part; p < P; p += nparts) {
      if (s < base + p + 1) {
        k = p;
        return;
      }
      base += p + 1;
      if (d - p != p) {
        if (s < base + d - p + 1) {
          k = d - p;
          return;
        }
        base += d - p + 1;
      }
    }
    k = -1;
  }
};

// LDS of one workgroup: x_c and y_c as planes (2, M, d+1), then the real
// products as real planes (M, 4 T): entry 4 s + q of product slot s holds
// q = 0: a.re b.re, 1: a.im b.im, 2: a.re b.im, 3: a.im b.re; the real part
// (entry 0 - entry 1) then goes to entry 0 and the imaginary part (entry 2
// + entry 3) to entry 2.  One md operation per lane in each pass keeps the
// registers few, so several workgroups share a CU.
template <int M>
__global__ void __launch_bounds__(256) k_convolve_lds(int d, long count, int nparts,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      double *__restrict__ z) {
  extern __shared__ double lds[];
  const int L = d + 1;
  const long E = count * L;
  const int P = pairs_of(d);
  double *xs = lds;
  double *ys = lds + 2 * M * L;
  double *pr = ys + 2 * M * L;
  for (long task = blockIdx.x; task < count * nparts; task += gridDim.x) {
    const long c = task / nparts;
    const ConvPart cp{d, P, int(task - c * nparts), nparts};
    int ncoef, T;
    cp.sizes(ncoef, T);
    const long T4 = 4L * T;
    for (int k = threadIdx.x; k < L; k += blockDim.x) {
      cstore<M>(xs, L, k, cload<M>(x, E, c * L + k));
      cstore<M>(ys, L, k, cload<M>(y, E, c * L + k));
    }
    __syncthreads();
    // the real products; the operands are selected, not branched on, so a
    // wave runs one instruction stream for all four
    for (long h = threadIdx.x; h < T4; h += blockDim.x) {
      const int s = int(h >> 2), q = int(h & 3);
      int k, base;
      cp.slot(s, k, base);
      const int i = s - base;
      // a.re for q = 0, 2 and a.im for q = 1, 3; b.re for q = 0, 3 and b.im for q = 1, 2
      const mdr<M> a = rload<M>(xs + size_t(q & 1) * M * L, L, i);
      const mdr<M> b = rload<M>(ys + size_t((q == 1 || q == 2) ? 1 : 0) * M * L, L, k - i);
      rstore<M>(pr, T4, h, md_mul<M>(a, b));
    }
    __syncthreads();
    // real part p1 + (-p2) into entry 0, imaginary part p3 + p4 into entry 2
    for (long h = threadIdx.x; h < 2L * T; h += blockDim.x) {
      const long e = 2 * h;  // entry 0 or 2 of its slot
      const mdr<M> u = rload<M>(pr, T4, e);
      mdr<M> v = rload<M>(pr, T4, e + 1);
      if (!(h & 1)) v = md_neg<M>(v);
      rstore<M>(pr, T4, e, md_add<M>(u, v));
    }
    __syncthreads();
    // the sums in order of i, one lane per coefficient and part; the waves
    // that hold these chains (the critical path) issue ahead of other
    // workgroups' product waves on their SIMD
    const bool chain_wave = int(threadIdx.x / WAVE) * WAVE < 2 * ncoef;
    if (chain_wave) __builtin_amdgcn_s_setprio(2);
    for (int u = threadIdx.x; u < 2 * ncoef; u += blockDim.x) {
      const int part = u & 1;
      int k, base;
      cp.coef(u >> 1, k, base);
      mdr<M> acc = rload<M>(pr, T4, 4L * base + 2 * part);
      for (int i = 1; i <= k; ++i)
        acc = md_add<M>(acc, rload<M>(pr, T4, 4L * (base + i) + 2 * part));
      rstore<M>(z + size_t(part) * M * E, E, c * L + k, acc);
    }
    if (chain_wave) __builtin_amdgcn_s_setprio(0);
    __syncthreads();
  }
}

// LDS bytes of k_convolve_lds with `nparts` parts per series
size_t conv_lds_bytes(int m, int d, int nparts) {
  const long P = (d + 2) / 2;
  const long ppp = (P + nparts - 1) / nparts;
  const long T = ppp * (d + 2);
  return sizeof(double) * size_t(m) * size_t(4L * (d + 1) + 4L * T);
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
    hipStream_t s = (hipStream_t)stream;
    const int P = pairs_of_host(d);
    // parts per series: about one workgroup per CU, so that each part's
    // chain of additions (its time, mostly) has a SIMD to itself; more
    // while the products of a part do not fit in LDS
    int nparts = 1;
    {
      int dev = 0, cus = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
          cus > 0) {
        const long want = long(cus) / count;
        nparts = int(want < P ? (want > 1 ? want : 1) : P);
      }
    }
    while (nparts < P && conv_lds_bytes(M, d, nparts) > lds_limit()) ++nparts;
    const size_t lds = conv_lds_bytes(M, d, nparts);
    if (lds <= lds_limit()) {
      const long tasks = long(count) * nparts;
      const unsigned grid = unsigned(tasks < 65536 ? tasks : 65536);
      k_convolve_lds<M><<<dim3(grid), dim3(256), lds, s>>>(d, long(count), nparts, x, y, z);
    } else {
      const long total = long(count) * P;
      long blocks = (total + 255) / 256;
      if (blocks > 65536) blocks = 65536;
      k_convolve<M><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(d, long(count), x, y, z);
    }
    return check_launch("md_series_convolve");
  });
}
