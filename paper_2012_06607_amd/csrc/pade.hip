// Division of truncated power series and Pade approximants (Section 3: a
// series with a nonzero constant term has an inverse, series divide like
// numbers, and a computed series yields rational approximations).
#include "internal.hpp"
#include "wg.hpp"

namespace mds {

// z = x / y mod t^{d+1}, one lane per series: z_0 = x_0 / y_0 and
// z_k = (x_k - (y_1 z_{k-1} + ... + y_k z_0)) / y_0, the products added in
// increasing order, each z_k read back from z (the lane's own stores).
template <int M>
__global__ void __launch_bounds__(64) k_series_divide(int d, long count,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      double *__restrict__ z, int32_t *status) {
  const long c = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= count) return;
  const long E = count * (d + 1), b = c * (d + 1);
  const mdc<M> y0 = cload<M>(y, E, b);
  if (y0.re.v[0] == 0.0 && y0.im.v[0] == 0.0 && status) atomicOr(status, MD_ST_SINGULAR);
  for (int k = 0; k <= d; ++k) {
    mdc<M> r = cload<M>(x, E, b + k);
    if (k > 0) {
      mdc<M> s = c_mul<M>(cload<M>(y, E, b + 1), cload<M>(z, E, b + k - 1));
      for (int i = 2; i <= k; ++i)
        s = c_add<M>(s, c_mul<M>(cload<M>(y, E, b + i), cload<M>(z, E, b + k - i)));
      r = c_sub<M>(r, s);
    }
    cstore<M>(z, E, b + k, c_div<M>(r, y0));
  }
}

// The same quotients with the products of each coefficient side by side:
// one wave per series, its lanes form y_i z_{k-i} for i = 1..k at once into
// LDS, then lane 0 adds them in increasing i, subtracts from x_k and
// divides by y_0 (the sequential definition's bits; the chain per
// coefficient is one product instead of k).  LDS per wave: the products
// (d) and the quotients so far (d+1), planes of complex md numbers.
template <int M>
__global__ void __launch_bounds__(256) k_series_divide_wave(int d, long count,
                                                            const double *__restrict__ x,
                                                            const double *__restrict__ y,
                                                            double *__restrict__ z,
                                                            int32_t *status) {
  extern __shared__ double lds[];
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  const long c = long(blockIdx.x) * (blockDim.x / WAVE) + wave;
  const int L = d + 1;
  double *pr = lds + size_t(wave) * 2 * M * (2 * L);  // products 1..d at 0..d-1
  double *zs = pr + size_t(2) * M * L;                 // z_0..z_d
  if (c >= count) return;  // whole waves: no barrier below spans waves
  const long E = count * L, b = c * L;
  const mdc<M> y0 = cload<M>(y, E, b);
  if (lane == 0 && y0.re.v[0] == 0.0 && y0.im.v[0] == 0.0 && status)
    atomicOr(status, MD_ST_SINGULAR);
  for (int k = 0; k <= d; ++k) {
    for (int i = 1 + lane; i <= k; i += WAVE)
      cstore<M>(pr, L, i - 1, c_mul<M>(cload<M>(y, E, b + i), cload<M>(zs, L, k - i)));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane == 0) {
      mdc<M> r = cload<M>(x, E, b + k);
      if (k > 0) {
        mdc<M> sm = cload<M>(pr, L, 0);
        for (int i = 2; i <= k; ++i) sm = c_add<M>(sm, cload<M>(pr, L, i - 1));
        r = c_sub<M>(r, sm);
      }
      const mdc<M> zk = c_div<M>(r, y0);
      cstore<M>(z, E, b + k, zk);
      cstore<M>(zs, L, k, zk);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// [L/Md] Pade approximant of one series per workgroup: the Toeplitz system
// sum_j c_{L+i-j} q_j = -c_{L+i} (i, j = 1..Md) by Householder QR (the QR
// and reflector solve of the Newton step), q_0 = 1, then
// p_k = sum_{j <= min(k, Md)} q_j c_{k-j}.
template <int M, int RPL>
__global__ void __launch_bounds__(256) k_pade(int L, int Md, long count, int seg,
                                                               const double *__restrict__ c,
                                                               double *__restrict__ p,
                                                               double *__restrict__ q,
                                                               char *__restrict__ wsb,
                                                               PadeLayout lay, int32_t *status) {
  __shared__ QrShared<M> sh;
  const long s = blockIdx.x;
  const int K = L + Md + 1;
  const long Ec = count * K, Ep = count * (L + 1), Eq = count * (Md + 1);
  const double *cs = c;
  int st = 0;
  if (Md > 0) {
    char *w = wsb + s * lay.per_series;
    double *QR = reinterpret_cast<double *>(w + lay.off_QR);
    double *vd = reinterpret_cast<double *>(w + lay.off_vd);
    double *beta = reinterpret_cast<double *>(w + lay.off_beta);
    double *invd = reinterpret_cast<double *>(w + lay.off_invd);
    double *rhs = reinterpret_cast<double *>(w + lay.off_rhs);
    double *sol = reinterpret_cast<double *>(w + lay.off_sol);
    const long E = long(Md) * Md;
    for (long e = threadIdx.x; e < E; e += blockDim.x) {
      const int i = int(e / Md) + 1, j = int(e % Md) + 1;
      const int k = L + i - j;
      cstore<M>(QR, E, e, k >= 0 ? cload<M>(cs, Ec, s * K + k) : c_zero<M>());
    }
    for (int i = threadIdx.x; i < Md; i += blockDim.x)
      cstore<M>(rhs, Md, i, c_neg<M>(cload<M>(cs, Ec, s * K + L + 1 + i)));
    __syncthreads();
    qr_wg<M, RPL>(sh, Md, Md, seg, QR, E, QR, vd, beta, st);
    inv_diag_range<M>(threadIdx.x, blockDim.x, Md, Md, QR, invd, st);
    __syncthreads();
    // q_1..q_Md by wave 0's first segment, then into q
    if (threadIdx.x < WAVE)
      qr_solve_vector<M, RPL>(lane_id() < seg, Md, Md, seg, QR, vd, beta, invd, rhs, sol);
    __syncthreads();
    for (int j = threadIdx.x; j < Md; j += blockDim.x)
      cstore<M>(q, Eq, s * (Md + 1) + 1 + j, cload<M>(sol, Md, j));
  }
  if (threadIdx.x == 0) {
    mdc<M> one = c_zero<M>();
    one.re = md_from<M>(1.0);
    cstore<M>(q, Eq, s * (Md + 1), one);
  }
  __syncthreads();
  for (int k = threadIdx.x; k <= L; k += blockDim.x) {
    mdc<M> acc = c_mul<M>(cload<M>(q, Eq, s * (Md + 1)), cload<M>(cs, Ec, s * K + k));
    const int top = k < Md ? k : Md;
    for (int j = 1; j <= top; ++j)
      acc = c_add<M>(acc, c_mul<M>(cload<M>(q, Eq, s * (Md + 1) + j), cload<M>(cs, Ec, s * K + k - j)));
    cstore<M>(p, Ep, s * (L + 1) + k, acc);
  }
  if (threadIdx.x == 0 && st && status) atomicOr(status, st);
}

}  // namespace mds

using namespace mds;

extern "C" int md_series_divide(int m, int d, int64_t count, const double *x, const double *y,
                                double *z, int32_t *status, void *stream) {
  if (d < 0 || count < 0)
    return fail(MD_EINVAL, "md_series_divide: d=%d count=%lld", d, (long long)count);
  if (count == 0) return dispatch_m(m, [](auto) { return MD_OK; });
  if (!x || !y || !z) return fail(MD_ENULL, "md_series_divide: null pointer");
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    // four series a workgroup (a wave each) while their products and
    // quotients fit in LDS, else one lane per series
    const size_t lds = sizeof(double) * 2 * Mm * 2 * size_t(d + 1) * 4;
    if (lds <= lds_limit()) {
      const long blocks = (long(count) + 3) / 4;
      if (blocks > 0x7fffffffL) return fail(MD_ESHAPE, "md_series_divide: count too large");
      k_series_divide_wave<Mm><<<dim3(unsigned(blocks)), dim3(256), lds, (hipStream_t)stream>>>(
          d, long(count), x, y, z, status);
    } else {
      const long blocks = (long(count) + 63) / 64;
      if (blocks > 0x7fffffffL) return fail(MD_ESHAPE, "md_series_divide: count too large");
      k_series_divide<Mm><<<dim3(unsigned(blocks)), dim3(64), 0, (hipStream_t)stream>>>(
          d, long(count), x, y, z, status);
    }
    return check_launch("md_series_divide");
  });
}

extern "C" int md_series_pade(int m, int L, int Md, int64_t count, const double *c, double *p,
                              double *q, void *ws, size_t ws_bytes, int32_t *status,
                              void *stream) {
  if (L < 0 || Md < 0 || count < 0)
    return fail(MD_EINVAL, "md_series_pade: L=%d M=%d count=%lld", L, Md, (long long)count);
  if (Md > 64) return fail(MD_ESHAPE, "md_series_pade: denominator degree %d above 64", Md);
  if (count == 0) return dispatch_m(m, [](auto) { return MD_OK; });
  if (!c || !p || !q) return fail(MD_ENULL, "md_series_pade: null pointer");
  if (count > 0x7fffffffL) return fail(MD_ESHAPE, "md_series_pade: count too large");
  if (!valid_m(m)) return dispatch_m(m, [](auto) { return MD_OK; });
  const PadeLayout lay(m, Md, long(count));
  if (Md > 0 && (!ws || ws_bytes < lay.bytes || !aligned256(ws)))
    return fail(MD_EWORKSPACE, "md_series_pade: workspace %zu bytes < %zu or misaligned", ws_bytes,
                lay.bytes);
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const int seg = Md >= WAVE ? WAVE : pow2_at_least(Md > 0 ? Md : 1);
    const int rpl = (Md + seg - 1) / seg;
    const dim3 grid{unsigned(count)}, blk{256u};
    hipStream_t s = (hipStream_t)stream;
    char *w = static_cast<char *>(ws);
    (void)rpl;  // Md <= 64: one row per lane
    k_pade<Mm, 1><<<grid, blk, 0, s>>>(L, Md, long(count), seg, c, p, q, w, lay, status);
    return check_launch("md_series_pade");
  });
}
