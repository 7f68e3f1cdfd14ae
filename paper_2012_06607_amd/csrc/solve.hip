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
#include "layout.hpp"

namespace mds {

// r = b (or -b), planes (2, m, d+1, N)
template <int M>
__global__ void __launch_bounds__(256) k_copy_rhs(long E, const double *__restrict__ b, bool neg,
                                                  double *__restrict__ r) {
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
                                                 double *__restrict__ invd, int32_t *status) {
  const long E = long(N) * n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const mdc<M> rii = cload<M>(QR, E, long(i) * n + i);
    if (rii.re.v[0] == 0.0 && rii.im.v[0] == 0.0 && status) atomicOr(status, MD_ST_SINGULAR);
    mdc<M> one = c_zero<M>();
    one.re = md_from<M>(1.0);
    cstore<M>(invd, n, i, c_div<M>(one, rii));
  }
}

// W = R^{-1} (Q^H)_{0:n}, column by column: column c of the identity is held
// in registers by a segment of `seg` lanes (lane l keeps rows l, l+seg, ...,
// at most RPL rows), the n reflectors are applied in order
// (w = v^H g by a fixed-order segment sum, g -= beta w v), then the back
// substitution R W_c = g_{0:n} runs with the row owner multiplying by
// 1/R_ii and broadcasting.  W: row-major n x N (plane stride n*N).
template <int M, int RPL>
__global__ void __launch_bounds__(256) k_pinv_cols(int N, int n, int seg,
                                                   const double *__restrict__ QR,
                                                   const double *__restrict__ vdiag,
                                                   const double *__restrict__ beta,
                                                   const double *__restrict__ invd,
                                                   double *__restrict__ W) {
  const long E = long(N) * n;
  const long EW = long(n) * N;
  const int lane = lane_id();
  const int lis = lane & (seg - 1);
  const int segs_per_wave = WAVE / seg;
  const int gwave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int c = gwave * segs_per_wave + lane / seg;
  const bool live = c < N;
  mdc<M> g[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    g[r] = c_zero<M>();
    if (live && lis + r * seg == c) g[r].re = md_from<M>(1.0);
  }
  for (int j = 0; j < n; ++j) {
    const mdc<M> v0 = cload<M>(vdiag, n, j);
    const mdr<M> bet = rload<M>(beta, n, j);
    mdc<M> vi[RPL];
    mdc<M> w = c_zero<M>();
    bool first = true;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lis + r * seg;
      vi[r] = c_zero<M>();
      if (i >= j && i < N) {
        vi[r] = (i == j) ? v0 : cload<M>(QR, E, long(i) * n + j);
        const mdc<M> t = c_mul<M>(c_conj<M>(vi[r]), g[r]);
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
      if (i >= j && i < N) g[r] = c_sub<M>(g[r], c_mul<M>(bw, vi[r]));
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    const int owner = i & (seg - 1), ro = i / seg;
    mdc<M> xi = c_zero<M>();
#pragma unroll
    for (int r = 0; r < RPL; ++r)
      if (r == ro && lis == owner) xi = c_mul<M>(g[r], cload<M>(invd, n, i));
    xi = shfl_c<M>(xi, (lane & ~(seg - 1)) + owner);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int l = lis + r * seg;
      if (l == i) g[r] = xi;
      else if (l < i) g[r] = c_sub<M>(g[r], c_mul<M>(cload<M>(QR, E, long(l) * n + i), xi));
    }
  }
  if (live) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lis + r * seg;
      if (i < n) cstore<M>(W, EW, long(i) * N + c, g[r]);
    }
  }
}

// dx_k = W r_k: one segment of `seg` lanes per output row, lanes over the
// N columns, fixed-order segment sum.
template <int M>
__global__ void __launch_bounds__(256) k_stage_dx(int k, int N, int n, int d, int seg,
                                                  const double *__restrict__ G,
                                                  const double *__restrict__ r,
                                                  double *__restrict__ dx, int32_t *status) {
  const long EG = long(n) * N;
  const long Er = long(d + 1) * N;
  const long Ex = long(d + 1) * n;
  const int lane = lane_id();
  const int rows_per_wave = WAVE / seg;
  const int gwave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int i = gwave * rows_per_wave + lane / seg;
  const int lis = lane & (seg - 1);
  mdc<M> s = c_zero<M>();
  if (i < n) {
    bool first = true;
    for (int c = lis; c < N; c += seg) {
      const mdc<M> t = c_mul<M>(cload<M>(G, EG, long(i) * N + c), cload<M>(r, Er, long(k) * N + c));
      s = first ? t : c_add<M>(s, t);
      first = false;
    }
  }
  s = seg_reduce_c<M>(s, seg);
  if (i < n && lis == 0) {
    cstore<M>(dx, Ex, long(k) * n + i, s);
    if (!c_finite<M>(s) && status) atomicOr(status, MD_ST_NONFINITE);
  }
}

// r_{k+j}[i] -= sum_l A_j[i][l] dx_k[l] for j = 1..d-k, i < N: one segment
// of `seg` lanes per (j, i).
template <int M>
__global__ void __launch_bounds__(256) k_stage_update(int k, int N, int n, int d, int seg,
                                                      const double *__restrict__ A,
                                                      const double *__restrict__ dx,
                                                      double *__restrict__ r) {
  const long EA = long(d + 1) * N * n;
  const long Er = long(d + 1) * N;
  const long Ex = long(d + 1) * n;
  const int lane = lane_id();
  const int rows_per_wave = WAVE / seg;
  const int gwave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const long row = long(gwave) * rows_per_wave + lane / seg;  // (j-1)*N + i
  const long nrows = long(d - k) * N;
  const int lis = lane & (seg - 1);
  const int j = int(row / N) + 1;
  const int i = int(row - long(j - 1) * N);
  mdc<M> s = c_zero<M>();
  if (row < nrows) {
    bool first = true;
    for (int l = lis; l < n; l += seg) {
      const mdc<M> t = c_mul<M>(cload<M>(A, EA, (long(j) * N + i) * n + l),
                                cload<M>(dx, Ex, long(k) * n + l));
      s = first ? t : c_add<M>(s, t);
      first = false;
    }
  }
  s = seg_reduce_c<M>(s, seg);
  if (row < nrows && lis == 0) {
    const long e = long(k + j) * N + i;
    cstore<M>(r, Er, e, c_sub<M>(cload<M>(r, Er, e), s));
  }
}

int solve_enqueue(int m, int N, int n, int d, const double *QR, const double *vdiag,
                  const double *beta, const double *A, const double *b, bool negate_b,
                  double *dx, void *ws, size_t ws_bytes, int32_t *status, hipStream_t s) {
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
    k_copy_rhs<Mm><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(Er, b, negate_b, r);
    double *invd = G + size_t(2) * Mm * n * N;
    k_inv_diag<Mm><<<dim3((n + 63) / 64), dim3(64), 0, s>>>(N, n, QR, invd, status);
    {
      const int seg = N >= WAVE ? WAVE : pow2_at_least(N);
      const long waves = (long(N) * seg + WAVE - 1) / WAVE;
      const unsigned blk = unsigned((waves + 3) / 4);
      const int rpl = (N + seg - 1) / seg;
      if (rpl == 1)
        k_pinv_cols<Mm, 1><<<dim3(blk), dim3(256), 0, s>>>(N, n, seg, QR, vdiag, beta, invd, G);
      else if (rpl == 2)
        k_pinv_cols<Mm, 2><<<dim3(blk), dim3(256), 0, s>>>(N, n, seg, QR, vdiag, beta, invd, G);
      else if (rpl <= 4)
        k_pinv_cols<Mm, 4><<<dim3(blk), dim3(256), 0, s>>>(N, n, seg, QR, vdiag, beta, invd, G);
      else
        return fail(MD_ESHAPE, "md_series_solve: N=%d above 256", N);
    }
    int rc = check_launch("md_series_solve (setup)");
    if (rc) return rc;
    const int seg_dx = N >= WAVE ? WAVE : pow2_at_least(N);
    const int seg_up = n >= WAVE ? WAVE : pow2_at_least(n);
    for (int k = 0; k <= d; ++k) {
      {
        const long waves = (long(n) * seg_dx + WAVE - 1) / WAVE;
        const long blk = (waves + 3) / 4;
        k_stage_dx<Mm><<<dim3(unsigned(blk)), dim3(256), 0, s>>>(k, N, n, d, seg_dx, G, r, dx,
                                                                  status);
      }
      if (k < d) {
        const long rows = long(d - k) * N;
        const long waves = (rows * seg_up + WAVE - 1) / WAVE;
        const long blk = (waves + 3) / 4;
        k_stage_update<Mm><<<dim3(unsigned(blk)), dim3(256), 0, s>>>(k, N, n, d, seg_up, A, dx, r);
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
