// Householder QR of A0 (Section 4: the block Toeplitz system needs one
// factorisation of A_0).  One workgroup; for column j one wave forms the
// reflector from the column's 2-norm, then every wave takes trailing columns
// and applies A[:, l] -= beta (v^H A[:, l]) v with a fixed-order wave sum.
#include "internal.hpp"

namespace mds {

template <int M>
__global__ void __launch_bounds__(256) k_qr(int N, int n, const double *__restrict__ A0, long A0E,
                                            double *__restrict__ QR, double *__restrict__ vdiag,
                                            double *__restrict__ beta, int32_t *status) {
  __shared__ mdc<M> sh_v0;
  __shared__ mdr<M> sh_beta;
  const long E = long(N) * n;
  const int lane = lane_id();
  const int wave = threadIdx.x / WAVE;
  const int nwaves = blockDim.x / WAVE;
  for (long e = threadIdx.x; e < E; e += blockDim.x) cstore<M>(QR, E, e, cload<M>(A0, A0E, e));
  __syncthreads();
  int st = 0;
  for (int j = 0; j < n; ++j) {
    if (wave == 0) {
      mdr<M> s = md_zero<M>();
      bool first = true;
      for (int i = j + lane; i < N; i += WAVE) {
        const mdr<M> t = c_abs2<M>(cload<M>(QR, E, long(i) * n + j));
        s = first ? t : md_add<M>(s, t);
        first = false;
      }
      s = seg_reduce_r<M>(s, WAVE);
      if (lane == 0) {
        const mdc<M> alpha = cload<M>(QR, E, long(j) * n + j);
        const mdr<M> a2 = c_abs2<M>(alpha);
        const mdr<M> sigma = md_sqrt<M>(s);
        const mdr<M> aabs = md_sqrt<M>(a2);
        mdc<M> phi = c_zero<M>();
        phi.re = md_from<M>(1.0);
        if (aabs.v[0] != 0.0) {
          phi.re = md_div<M>(alpha.re, aabs);
          phi.im = md_div<M>(alpha.im, aabs);
        }
        mdr<M> bet = md_zero<M>();
        mdc<M> v0 = c_zero<M>(), rjj = c_zero<M>();
        if (sigma.v[0] == 0.0) {
          st |= MD_ST_SINGULAR;
        } else {
          const mdr<M> sp = md_add<M>(aabs, sigma);
          v0 = c_mulr<M>(phi, sp);
          bet = md_div<M>(md_from<M>(1.0), md_mul<M>(sigma, sp));
          rjj = c_neg<M>(c_mulr<M>(phi, sigma));
        }
        sh_v0 = v0;
        sh_beta = bet;
        cstore<M>(vdiag, n, j, v0);
        rstore<M>(beta, n, j, bet);
        cstore<M>(QR, E, long(j) * n + j, rjj);
        if (!c_finite<M>(rjj) || !md_finite<M>(bet)) st |= MD_ST_NONFINITE;
      }
    }
    __syncthreads();
    const mdc<M> v0 = sh_v0;
    const mdr<M> bet = sh_beta;
    for (int l = j + 1 + wave; l < n; l += nwaves) {
      mdc<M> w = c_zero<M>();
      bool first = true;
      for (int i = j + lane; i < N; i += WAVE) {
        const mdc<M> vi = (i == j) ? v0 : cload<M>(QR, E, long(i) * n + j);
        const mdc<M> t = c_mul<M>(c_conj<M>(vi), cload<M>(QR, E, long(i) * n + l));
        w = first ? t : c_add<M>(w, t);
        first = false;
      }
      w = seg_reduce_c<M>(w, WAVE);
      w = shfl_c<M>(w, 0);
      const mdc<M> bw = c_mulr<M>(w, bet);
      for (int i = j + lane; i < N; i += WAVE) {
        const mdc<M> vi = (i == j) ? v0 : cload<M>(QR, E, long(i) * n + j);
        const long e = long(i) * n + l;
        cstore<M>(QR, E, e, c_sub<M>(cload<M>(QR, E, e), c_mul<M>(bw, vi)));
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && st && status) atomicOr(status, st);
}

int qr_enqueue(int m, int N, int n, const double *A0, long A0E, double *QR, double *vdiag,
               double *beta, int32_t *status, hipStream_t s) {
  if (n < 1 || N < n) return fail(MD_ESHAPE, "md_qr: need N >= n >= 1 (N=%d n=%d)", N, n);
  if (!A0 || !QR || !vdiag || !beta) return fail(MD_ENULL, "md_qr: null pointer");
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    k_qr<Mm><<<dim3(1), dim3(256), 0, s>>>(N, n, A0, A0E, QR, vdiag, beta, status);
    return check_launch("md_qr");
  });
}

}  // namespace mds

extern "C" int md_qr(int m, int N, int n, const double *A0, double *QR, double *vdiag,
                     double *beta, int32_t *status, void *stream) {
  return mds::qr_enqueue(m, N, n, A0, long(N) * n, QR, vdiag, beta, status, (hipStream_t)stream);
}
