// Householder QR of A0 (Section 4: the block Toeplitz system needs one
// factorisation of A_0), by one workgroup (qr_wg): the column norm and
// |alpha| on two waves in parallel, the reflector on one lane, and the
// trailing columns over every wave, one column per segment of lanes.
#include "internal.hpp"
#include "wg.hpp"

namespace mds {

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
                                                       int32_t *status, const int32_t *gate) {
  __shared__ QrShared<M> sh;
  if (gate_closed(gate)) return;
  int st = 0;
  qr_wg<M, RPL>(sh, N, n, seg, A0, A0E, QR, vdiag, beta, st);
  if (threadIdx.x == 0 && st && status) atomicOr(status, st);
}

int qr_enqueue(int m, int N, int n, const double *A0, long A0E, double *QR, double *vdiag,
               double *beta, int32_t *status, hipStream_t s, const int32_t *gate) {
  if (n < 1 || N < n) return fail(MD_ESHAPE, "md_qr: need N >= n >= 1 (N=%d n=%d)", N, n);
  if (N > 256) return fail(MD_ESHAPE, "md_qr: N=%d above 256", N);
  if (!A0 || !QR || !vdiag || !beta) return fail(MD_ENULL, "md_qr: null pointer");
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const int seg = N >= WAVE ? WAVE : pow2_at_least(N);
    const int rpl = (N + seg - 1) / seg;
    const dim3 blk(qr_threads<Mm>());
    if (rpl == 1) k_qr<Mm, 1><<<dim3(1), blk, 0, s>>>(N, n, seg, A0, A0E, QR, vdiag, beta, status, gate);
    else if (rpl == 2) k_qr<Mm, 2><<<dim3(1), blk, 0, s>>>(N, n, seg, A0, A0E, QR, vdiag, beta, status, gate);
    else k_qr<Mm, 4><<<dim3(1), blk, 0, s>>>(N, n, seg, A0, A0E, QR, vdiag, beta, status, gate);
    return check_launch("md_qr");
  });
}

}  // namespace mds

extern "C" int md_qr(int m, int N, int n, const double *A0, double *QR, double *vdiag,
                     double *beta, int32_t *status, void *stream) {
  return mds::qr_enqueue(m, N, n, A0, long(N) * n, QR, vdiag, beta, status, (hipStream_t)stream);
}
