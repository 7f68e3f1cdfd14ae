// Householder QR of A0 (Section 4: the block Toeplitz system needs one
// factorisation of A_0).  One workgroup runs the n column steps; inside a
// step the column norm and |alpha| go to two waves in parallel, one lane
// forms the reflector, and the trailing columns are spread over every
// wave, one column per segment of `seg` lanes (lanes over rows, two
// columns per wave when N <= 32), with fixed-order segment sums.
#include "internal.hpp"

namespace mds {

// 1/sqrt(a) by Newton steps y += y (1 - a y^2)/2 that double the working
// precision (2, 4, 8 limbs, then M), from the hardware value: the early
// steps cost a fraction of a full-precision step.
template <int P, int M>
__device__ __forceinline__ mdr<P> trunc(const mdr<M> &a) {
  mdr<P> z;
#pragma unroll
  for (int i = 0; i < P; ++i) z.v[i] = i < M ? a.v[i] : 0.0;
  return z;
}

template <int P, int M>
__device__ __forceinline__ mdr<P> rsqrt_step(const mdr<M> &a, const mdr<P> &y) {
  const mdr<P> ap = trunc<P, M>(a);
  mdr<P> t = md_mul<P>(y, y);
  t = md_mul<P>(ap, t);
  t = md_sub<P>(md_from<P>(1.0), t);
  t = md_mul<P>(y, t);
#pragma unroll
  for (int i = 0; i < P; ++i) t.v[i] = t.v[i] * 0.5;
  return md_add<P>(y, t);
}

template <int M>
__device__ mdr<M> rsqrt_doubling(const mdr<M> &a) {
  const double y0 = 1.0 / __builtin_sqrt(a.v[0]);
  if constexpr (M == 1) {
    return md_from<1>(y0);
  } else {
    mdr<2> y2 = rsqrt_step<2, M>(a, md_from<2>(y0));
    if constexpr (M == 2) {
      return rsqrt_step<2, 2>(a, y2);
    } else if constexpr (M <= 4) {
      return rsqrt_step<M, M>(a, trunc<M, 2>(y2));
    } else {
      mdr<4> y4 = rsqrt_step<4, M>(a, trunc<4, 2>(y2));
      if constexpr (M <= 8) {
        return rsqrt_step<M, M>(a, trunc<M, 4>(y4));
      } else {
        mdr<8> y8 = rsqrt_step<8, M>(a, trunc<8, 4>(y4));
        return rsqrt_step<M, M>(a, trunc<M, 8>(y8));
      }
    }
  }
}

template <int M>
constexpr int qr_threads() {
  return M <= 2 ? 1024 : (M <= 4 ? 512 : 256);
}

template <int M, int RPL>
__global__ void __launch_bounds__(qr_threads<M>()) k_qr(int N, int n, int seg,
                                                       const double *__restrict__ A0, long A0E,
                                                       double *__restrict__ QR,
                                                       double *__restrict__ vdiag,
                                                       double *__restrict__ beta,
                                                       int32_t *status) {
  __shared__ mdr<M> sh_s2, sh_ys, sh_a2, sh_ya;
  __shared__ mdc<M> sh_v0;
  __shared__ mdr<M> sh_beta;
  const long E = long(N) * n;
  const int lane = lane_id();
  const int wave = threadIdx.x / WAVE;
  const int nwaves = blockDim.x / WAVE;
  const int lis = lane & (seg - 1);
  const int spw = WAVE / seg;                       // column slots per wave
  const int slot = wave * spw + lane / seg;        // this lane's column slot
  const int nslots = nwaves * spw;
  for (long e = threadIdx.x; e < E; e += blockDim.x) cstore<M>(QR, E, e, cload<M>(A0, A0E, e));
  __syncthreads();
  int st = 0;
  for (int j = 0; j < n; ++j) {
    // norm of the column from the diagonal down (wave 0, first segment)
    if (wave == 0) {
      mdr<M> s = md_zero<M>();
      bool first = true;
      if (lane < seg) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int i = lis + r * seg;
          if (i >= j && i < N) {
            const mdr<M> t = c_abs2<M>(cload<M>(QR, E, long(i) * n + j));
            s = first ? t : md_add<M>(s, t);
            first = false;
          }
        }
      }
      s = seg_reduce_r<M>(s, seg);
      if (lane == 0) {
        sh_s2 = s;
        sh_ys = rsqrt_doubling<M>(s);
      }
    } else if (wave == 1 && lane == 0) {
      const mdr<M> a2 = c_abs2<M>(cload<M>(QR, E, long(j) * n + j));
      sh_a2 = a2;
      sh_ya = rsqrt_doubling<M>(a2);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const mdc<M> alpha = cload<M>(QR, E, long(j) * n + j);
      const mdr<M> s2 = sh_s2, ys = sh_ys, a2 = sh_a2, ya = sh_ya;
      const mdr<M> sigma = md_mul<M>(s2, ys);
      mdr<M> aabs = md_mul<M>(a2, ya);
      mdc<M> phi = c_zero<M>();
      phi.re = md_from<M>(1.0);
      if (a2.v[0] != 0.0) phi = c_mulr<M>(alpha, ya);
      else aabs = md_zero<M>();
      mdr<M> bet = md_zero<M>();
      mdc<M> v0 = c_zero<M>(), rjj = c_zero<M>();
      if (s2.v[0] == 0.0) {
        st |= MD_ST_SINGULAR;
      } else {
        const mdr<M> sp = md_add<M>(aabs, sigma);
        v0 = c_mulr<M>(phi, sp);
        bet = md_div<M>(ys, sp);
        rjj = c_neg<M>(c_mulr<M>(phi, sigma));
      }
      if (!c_finite<M>(rjj) || !md_finite<M>(bet)) st |= MD_ST_NONFINITE;
      sh_v0 = v0;
      sh_beta = bet;
      cstore<M>(vdiag, n, j, v0);
      rstore<M>(beta, n, j, bet);
      cstore<M>(QR, E, long(j) * n + j, rjj);
    }
    __syncthreads();
    const mdc<M> v0 = sh_v0;
    const mdr<M> bet = sh_beta;
    for (int l = j + 1 + slot; l < n; l += nslots) {
      mdc<M> vi[RPL], al[RPL];
      mdc<M> w = c_zero<M>();
      bool first = true;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lis + r * seg;
        vi[r] = c_zero<M>();
        al[r] = c_zero<M>();
        if (i >= j && i < N) {
          vi[r] = (i == j) ? v0 : cload<M>(QR, E, long(i) * n + j);
          al[r] = cload<M>(QR, E, long(i) * n + l);
          const mdc<M> t = c_mul<M>(c_conj<M>(vi[r]), al[r]);
          w = first ? t : c_add<M>(w, t);
          first = false;
        }
      }
      w = seg_reduce_c<M>(w, seg);
      w = shfl_c<M>(w, lane & ~(seg - 1));
      const mdc<M> bw = c_mulr<M>(w, bet);
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lis + r * seg;
        if (i >= j && i < N) cstore<M>(QR, E, long(i) * n + l, c_sub<M>(al[r], c_mul<M>(bw, vi[r])));
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && st && status) atomicOr(status, st);
}

int qr_enqueue(int m, int N, int n, const double *A0, long A0E, double *QR, double *vdiag,
               double *beta, int32_t *status, hipStream_t s) {
  if (n < 1 || N < n) return fail(MD_ESHAPE, "md_qr: need N >= n >= 1 (N=%d n=%d)", N, n);
  if (N > 256) return fail(MD_ESHAPE, "md_qr: N=%d above 256", N);
  if (!A0 || !QR || !vdiag || !beta) return fail(MD_ENULL, "md_qr: null pointer");
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const int seg = N >= WAVE ? WAVE : pow2_at_least(N);
    const int rpl = (N + seg - 1) / seg;
    const dim3 blk(qr_threads<Mm>());
    if (rpl == 1) k_qr<Mm, 1><<<dim3(1), blk, 0, s>>>(N, n, seg, A0, A0E, QR, vdiag, beta, status);
    else if (rpl == 2) k_qr<Mm, 2><<<dim3(1), blk, 0, s>>>(N, n, seg, A0, A0E, QR, vdiag, beta, status);
    else k_qr<Mm, 4><<<dim3(1), blk, 0, s>>>(N, n, seg, A0, A0E, QR, vdiag, beta, status);
    return check_launch("md_qr");
  });
}

}  // namespace mds

extern "C" int md_qr(int m, int N, int n, const double *A0, double *QR, double *vdiag,
                     double *beta, int32_t *status, void *stream) {
  return mds::qr_enqueue(m, N, n, A0, long(N) * n, QR, vdiag, beta, status, (hipStream_t)stream);
}
