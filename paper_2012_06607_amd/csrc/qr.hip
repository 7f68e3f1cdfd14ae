// Householder QR of A0 (Section 4: the block Toeplitz system needs one
// factorisation of A_0), by one workgroup (qr_wg): the column norm and
// |alpha| on two waves in parallel, the reflector on one lane, and the
// trailing columns over every wave, one column per segment of lanes.
// With a synchronisation word the trailing columns of each step go over
// several workgroups instead (qr_gang, a device-memory barrier per column
// step): one workgroup is one CU's issue rate, and a step of a 64-column
// octo-double QR is some 60 complex products a lane long on one CU.  From
// three limbs on and for N <= 64 the look-ahead column of each step (the
// step's critical path: its update, then the next reflector) goes to four
// waves of workgroup 0, one real product of each complex product a lane
// (qr_gang_lead4).  All forms give the same bits.
#include "gang.hpp"
#include "internal.hpp"

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

// The same QR by gridDim.x workgroups meeting at barriers on *ctr (zero at
// the start; k_zero_ctr clears it on the stream first).
template <int M, int RPL>
__global__ void __launch_bounds__(qr_threads<M>()) k_qr_gang(int N, int n, int seg,
                                                            const double *__restrict__ A0,
                                                            long A0E, double *__restrict__ QR,
                                                            double *__restrict__ vdiag,
                                                            double *__restrict__ beta,
                                                            int32_t *status, const int32_t *gate,
                                                            int32_t *ctr) {
  __shared__ QrShared<M> sh;
  if (gate_closed(gate)) return;
  int st = 0, round = 0;
  const int G = int(gridDim.x);
  auto gsync = [&] { gang_barrier(ctr, G, round, st); };
  qr_gang<M, RPL>(sh, N, n, seg, A0, A0E, QR, vdiag, beta, st, int(blockIdx.x), G, gsync);
  if (threadIdx.x == 0 && st && status) atomicOr(status, st);
}

// The same with the look-ahead column on four waves of workgroup 0
// (qr_gang_lead4; needs 5 <= N <= 64).
template <int M>
__global__ void __launch_bounds__(qr_threads<M>()) k_qr_gang4(int N, int n, int seg,
                                                             const double *__restrict__ A0,
                                                             long A0E, double *__restrict__ QR,
                                                             double *__restrict__ vdiag,
                                                             double *__restrict__ beta,
                                                             int32_t *status, const int32_t *gate,
                                                             int32_t *ctr) {
  __shared__ QrShared<M> sh;
  __shared__ double xch[4 * M];
  if (gate_closed(gate)) return;
  int st = 0, round = 0;
  const int G = int(gridDim.x);
  auto gsync = [&] { gang_barrier(ctr, G, round, st); };
  qr_gang_lead4<M>(sh, xch, N, n, seg, A0, A0E, QR, vdiag, beta, st, int(blockIdx.x), G, gsync);
  if (threadIdx.x == 0 && st && status) atomicOr(status, st);
}

__global__ void k_zero_ctr(int32_t *ctr) { *ctr = 0; }

// From three limbs on, a column of at most 64 rows takes the four-wave
// look-ahead form (a real md product costs a quarter of a complex one or
// more; for double and double double the barriers would cost more).
static bool qr_uses_lead4(int m, int N) { return m >= 3 && N >= 5 && N <= WAVE; }

// workgroups of the spread QR: enough slots for the trailing columns of
// the first step in one round (in the four-wave form workgroup 0 takes
// the look-ahead column alone)
int qr_gang_size(int m, int N, int n) {
  const int threads = m <= 2 ? 1024 : (m <= 4 ? 512 : 256);
  const int seg = N >= WAVE ? WAVE : pow2_at_least(N);
  const int slots = (threads / WAVE) * (WAVE / seg);
  const int G = qr_uses_lead4(m, N) ? 1 + (n - 2 + slots - 1) / slots : (n - 1 + slots - 1) / slots;
  return G < 1 ? 1 : (G > 64 ? 64 : G);
}

int qr_enqueue(int m, int N, int n, const double *A0, long A0E, double *QR, double *vdiag,
               double *beta, int32_t *status, hipStream_t s, const int32_t *gate,
               int32_t *ctr) {
  if (n < 1 || N < n) return fail(MD_ESHAPE, "md_qr: need N >= n >= 1 (N=%d n=%d)", N, n);
  if (N > 256) return fail(MD_ESHAPE, "md_qr: N=%d above 256", N);
  if (!A0 || !QR || !vdiag || !beta) return fail(MD_ENULL, "md_qr: null pointer");
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const int seg = N >= WAVE ? WAVE : pow2_at_least(N);
    const int rpl = (N + seg - 1) / seg;
    const dim3 blk(qr_threads<Mm>());
    const int G = ctr ? qr_gang_size(Mm, N, n) : 1;
    if (G > 1) {
      k_zero_ctr<<<dim3(1), dim3(1), 0, s>>>(ctr);
      if (qr_uses_lead4(Mm, N))
        k_qr_gang4<Mm><<<dim3(G), blk, 0, s>>>(N, n, seg, A0, A0E, QR, vdiag, beta, status, gate,
                                               ctr);
      else if (rpl == 1)
        k_qr_gang<Mm, 1><<<dim3(G), blk, 0, s>>>(N, n, seg, A0, A0E, QR, vdiag, beta, status,
                                                 gate, ctr);
      else if (rpl == 2)
        k_qr_gang<Mm, 2><<<dim3(G), blk, 0, s>>>(N, n, seg, A0, A0E, QR, vdiag, beta, status,
                                                 gate, ctr);
      else
        k_qr_gang<Mm, 4><<<dim3(G), blk, 0, s>>>(N, n, seg, A0, A0E, QR, vdiag, beta, status,
                                                 gate, ctr);
      return check_launch("md_qr");
    }
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

extern "C" int md_qr_gang(int m, int N, int n, const double *A0, double *QR, double *vdiag,
                          double *beta, int32_t *sync, int32_t *status, void *stream) {
  if (!sync) return mds::fail(MD_ENULL, "md_qr_gang: null synchronisation word");
  return mds::qr_enqueue(m, N, n, A0, long(N) * n, QR, vdiag, beta, status, (hipStream_t)stream,
                         nullptr, sync);
}

extern "C" int md_qr_gang_size(int m, int N, int n) {
  if (!mds::valid_m(m) || n < 1 || N < n || N > 256) return 0;
  return mds::qr_gang_size(m, N, n);
}
