// Staggered solve of A(t) dx(t) = b(t), the block lower triangular Toeplitz
// system of Section 4, by forward substitution over the degrees.
//
// Every stage solves A_0 dx_k = r_k with the same QR factors.  Applying Q^H
// (n reflectors in sequence) and then back substitution with R is a chain
// of about 2n dependent steps; here that chain runs once, on the N columns
// of the identity, giving W = R^{-1} (Q^H)_{0:n} (n x N), and every stage
// is then the product dx_k = W r_k (least squares in the first n rows when
// N > n).  After dx_k the later right hand sides are updated,
// r_{k+j} -= A_j dx_k for all j = 1..d-k at once (the paper's "one job per
// right hand side update", Section 5).
#include "internal.hpp"
#include "wg.hpp"

namespace mds {

// r = b (or -b), planes (2, m, d+1, N)
template <int M>
__global__ void __launch_bounds__(256) k_copy_rhs(long E, const double *__restrict__ b, bool neg,
                                                  double *__restrict__ r, const int32_t *gate) {
  if (gate_closed(gate)) return;
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < E;
       e += long(gridDim.x) * blockDim.x) {
    mdc<M> z = cload<M>(b, E, e);
    if (neg) z = c_neg<M>(z);
    cstore<M>(r, E, e, z);
  }
}

// 1 / R_ii for i < n (one thread each), so that the back substitution
// multiplies instead of dividing.
template <int M>
__global__ void __launch_bounds__(64) k_inv_diag(int N, int n, const double *__restrict__ QR,
                                                 double *__restrict__ invd, int32_t *status,
                                                 const int32_t *gate) {
  if (gate_closed(gate)) return;
  int st = 0;
  inv_diag_range<M>(blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, N, n, QR,
                    invd, st);
  if (st && status) atomicOr(status, st);
}

// W = R^{-1} (Q^H)_{0:n}: one segment of lanes per identity column
template <int M, int RPL>
__global__ void __launch_bounds__(256) k_pinv_cols(int N, int n, int seg,
                                                   const double *__restrict__ QR,
                                                   const double *__restrict__ vdiag,
                                                   const double *__restrict__ beta,
                                                   const double *__restrict__ invd,
                                                   double *__restrict__ W, const int32_t *gate) {
  if (gate_closed(gate)) return;
  const int gwave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int c = gwave * (WAVE / seg) + lane_id() / seg;
  pinv_column<M, RPL, true>(c < N, c, N, n, seg, QR, vdiag, beta, invd, W);
}

// dx_k = W r_k: one segment per output row
template <int M>
__global__ void __launch_bounds__(256) k_stage_dx(int k, int N, int n, int d, int seg,
                                                  const double *__restrict__ G,
                                                  const double *__restrict__ r,
                                                  double *__restrict__ dx, int32_t *status,
                                                  const int32_t *gate) {
  if (gate_closed(gate)) return;
  const int gwave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int i = gwave * (WAVE / seg) + lane_id() / seg;
  int st = 0;
  stage_dx_row<M>(i < n, i, k, N, n, d, seg, G, r, dx, st);
  if (st && status) atomicOr(status, st);
}

// r_{k+j} -= A_j dx_k for j = 1..d-k: one segment per (j, row)
template <int M>
__global__ void __launch_bounds__(256) k_stage_update(int k, int N, int n, int d, int seg,
                                                      const double *__restrict__ A,
                                                      const double *__restrict__ dx,
                                                      double *__restrict__ r, const int32_t *gate) {
  if (gate_closed(gate)) return;
  const int gwave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const long row = long(gwave) * (WAVE / seg) + lane_id() / seg;
  stage_update_row<M>(row < long(d - k) * N, row, k, N, n, d, seg, A, dx, r);
}

int pinv_enqueue(int m, int N, int n, const double *QR, const double *vdiag, const double *beta,
                 double *invd, double *W, int32_t *status, hipStream_t s, const int32_t *gate) {
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    k_inv_diag<Mm><<<dim3((n + 63) / 64), dim3(64), 0, s>>>(N, n, QR, invd, status, gate);
    const int seg = N >= WAVE ? WAVE : pow2_at_least(N);
    const long waves = (long(N) * seg + WAVE - 1) / WAVE;
    const unsigned blk = unsigned((waves + 3) / 4);
    const int rpl = (N + seg - 1) / seg;
    if (rpl == 1)
      k_pinv_cols<Mm, 1><<<dim3(blk), dim3(256), 0, s>>>(N, n, seg, QR, vdiag, beta, invd, W, gate);
    else if (rpl == 2)
      k_pinv_cols<Mm, 2><<<dim3(blk), dim3(256), 0, s>>>(N, n, seg, QR, vdiag, beta, invd, W, gate);
    else if (rpl <= 4)
      k_pinv_cols<Mm, 4><<<dim3(blk), dim3(256), 0, s>>>(N, n, seg, QR, vdiag, beta, invd, W, gate);
    else
      return fail(MD_ESHAPE, "R^{-1} Q^H: N=%d above 256", N);
    return check_launch("R^{-1} Q^H");
  });
}

int solve_enqueue(int m, int N, int n, int d, const double *QR, const double *vdiag,
                  const double *beta, const double *A, const double *b, bool negate_b,
                  double *dx, void *ws, size_t ws_bytes, int32_t *status, hipStream_t s,
                  const int32_t *gate) {
  if (d < 0) return fail(MD_EINVAL, "md_series_solve: d=%d < 0", d);
  if (n < 1 || N < n) return fail(MD_ESHAPE, "md_series_solve: need N >= n >= 1 (N=%d n=%d)", N, n);
  if (N > 256) return fail(MD_ESHAPE, "md_series_solve: N=%d above 256", N);
  if (!QR || !vdiag || !beta || !A || !b || !dx) return fail(MD_ENULL, "md_series_solve: null pointer");
  if (!valid_m(m)) return dispatch_m(m, [](auto) { return MD_OK; });
  SolveLayout lay(m, N, n, d);
  if (!ws || ws_bytes < lay.bytes || !aligned256(ws))
    return fail(MD_EWORKSPACE, "md_series_solve: workspace %zu bytes < %zu or misaligned",
                ws_bytes, lay.bytes);
  double *r = reinterpret_cast<double *>(static_cast<char *>(ws) + lay.off_r);
  double *G = reinterpret_cast<double *>(static_cast<char *>(ws) + lay.off_G);
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const long Er = long(d + 1) * N;
    long blocks = (Er + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_copy_rhs<Mm><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(Er, b, negate_b, r, gate);
    double *invd = G + size_t(2) * Mm * n * N;
    int rc = pinv_enqueue(Mm, N, n, QR, vdiag, beta, invd, G, status, s, gate);
    if (rc) return rc;
    const int seg_dx = dot_seg_latency(N);
    const int seg_up = dot_seg_latency(n);
    for (int k = 0; k <= d; ++k) {
      {
        const long waves = (long(n) * seg_dx + WAVE - 1) / WAVE;
        const long blk = (waves + 3) / 4;
        k_stage_dx<Mm><<<dim3(unsigned(blk)), dim3(256), 0, s>>>(k, N, n, d, seg_dx, G, r, dx,
                                                                  status, gate);
      }
      if (k < d) {
        const long rows = long(d - k) * N;
        const long waves = (rows * seg_up + WAVE - 1) / WAVE;
        const long blk = (waves + 3) / 4;
        k_stage_update<Mm><<<dim3(unsigned(blk)), dim3(256), 0, s>>>(k, N, n, d, seg_up, A, dx, r, gate);
      }
    }
    return check_launch("md_series_solve (stages)");
  });
}

}  // namespace mds

extern "C" int md_series_solve(int m, int N, int n, int d, const double *QR, const double *vdiag,
                               const double *beta, const double *A, const double *b, double *dx,
                               void *ws, size_t ws_bytes, int32_t *status, void *stream) {
  return mds::solve_enqueue(m, N, n, d, QR, vdiag, beta, A, b, false, dx, ws, ws_bytes, status,
                            (hipStream_t)stream);
}
