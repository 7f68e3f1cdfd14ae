// Adjoint of the converged series solution: coefficient gradients of a real
// loss.
//
// At the converged x(t) the truncated system F(x, c) = f(x(t); c) mod
// t^{d+1} vanishes; its Jacobian in the series coefficients of x is the
// block lower triangular Toeplitz matrix T(A) of Section 4.  For the
// upstream gradient G (dL/dRe x + i dL/dIm x) the coefficient gradient is
// -B^H lambda with T(A)^H lambda = G and B the derivative of F in the
// coefficients.  T(A)^H is block upper triangular, so the stages run
// backward, k = d..0:
//   lambda_k = W^H (G_k - sum_{j=1}^{d-k} A_j^H lambda_{k+j}),
// with W = R^{-1} (Q^H)_{0:n} from the one QR of A_0 (W^H = A_0^{-H}, or the
// minimum-norm solution when N > n).  A coefficient c_{tau,j} enters f_i as
// c_tau(t) x^a(t), so grad c_{tau,j} = -sum_{k>=j} conj(m_{tau,k-j})
// lambda_{k,i}, m_tau = x^a: either stored by the evaluation pass or
// recomputed term by term inside the contraction (no buffer).
#include "dot4.hpp"
#include "internal.hpp"

namespace mds {

// lambda_k[i] = sum_c conj(W[c][i]) rhs_k[c], i < N (one segment per i)
template <int M>
__global__ void __launch_bounds__(256) k_adj_lambda(int k, int N, int n, int d, int seg,
                                                    const double *__restrict__ W,
                                                    const double *__restrict__ rhs,
                                                    double *__restrict__ lam, int32_t *status) {
  const int gwave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int i = gwave * (WAVE / seg) + lane_id() / seg;
  const bool live = i < N;
  const long EW = long(n) * N, Er = long(d + 1) * n, El = long(d + 1) * N;
  const int lis = lane_id() & (seg - 1);
  mdc<M> s = c_zero<M>();
  bool first = true;
  if (live)
    for (int c = lis; c < n; c += seg) {
      const mdc<M> t =
          c_mul<M>(c_conj<M>(cload<M>(W, EW, long(c) * N + i)), cload<M>(rhs, Er, long(k) * n + c));
      s = first ? t : c_add<M>(s, t);
      first = false;
    }
  s = seg_reduce_c<M>(s, seg);
  if (live && lis == 0) {
    cstore<M>(lam, El, long(k) * N + i, s);
    if (!c_finite<M>(s) && status) atomicOr(status, MD_ST_NONFINITE);
  }
}

// rhs_{k-j}[c] -= sum_i conj(A_j[i][c]) lambda_k[i], j = 1..k, c < n (one
// segment per (j, c); row = (j-1)*n + c)
template <int M>
__global__ void __launch_bounds__(256) k_adj_update(int k, int N, int n, int d, int seg,
                                                    const double *__restrict__ A,
                                                    const double *__restrict__ lam,
                                                    double *__restrict__ rhs) {
  const int gwave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const long row = long(gwave) * (WAVE / seg) + lane_id() / seg;
  const bool live = row < long(k) * n;
  const int j = live ? int(row / n) + 1 : 1;
  const int c = live ? int(row - long(j - 1) * n) : 0;
  const long EA = long(d + 1) * N * n, Er = long(d + 1) * n, El = long(d + 1) * N;
  const int lis = lane_id() & (seg - 1);
  mdc<M> s = c_zero<M>();
  bool first = true;
  if (live)
    for (int i = lis; i < N; i += seg) {
      const mdc<M> t = c_mul<M>(c_conj<M>(cload<M>(A, EA, (long(j) * N + i) * n + c)),
                                cload<M>(lam, El, long(k) * N + i));
      s = first ? t : c_add<M>(s, t);
      first = false;
    }
  s = seg_reduce_c<M>(s, seg);
  if (live && lis == 0) {
    const long e = long(k - j) * n + c;
    cstore<M>(rhs, Er, e, c_sub<M>(cload<M>(rhs, Er, e), s));
  }
}

// The same two products with each dot product on four waves (dot4: one
// real product of each complex product a lane; same bits), from three
// limbs on while the dot products are at most 64 long: lambda_k[i], one
// workgroup per i; the update, one workgroup per (j, c), while there are
// at most 512 of them.
template <int M>
__global__ void __launch_bounds__(256) k_adj_lambda4(int k, int N, int n, int d, int seg,
                                                     const double *__restrict__ W,
                                                     const double *__restrict__ rhs,
                                                     double *__restrict__ lam, int32_t *status) {
  __shared__ double xch[4 * M];
  const long EW = long(n) * N, Er = long(d + 1) * n, El = long(d + 1) * N;
  const int i = blockIdx.x;
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  const mdr<M> s = dot4<M, true>(n, seg, [&](int c, mdc<M> &x, mdc<M> &y) {
    x = cload<M>(W, EW, long(c) * N + i);
    y = cload<M>(rhs, Er, long(k) * n + c);
  }, xch);
  if (w == 0 && (lane == 0 || lane == 2)) {
    rstore<M>(lam + size_t(lane >> 1) * M * El, El, long(k) * N + i, s);
    if (!md_finite<M>(s) && status) atomicOr(status, MD_ST_NONFINITE);
  }
}

template <int M>
__global__ void __launch_bounds__(256) k_adj_update4(int k, int N, int n, int d, int seg,
                                                     const double *__restrict__ A,
                                                     const double *__restrict__ lam,
                                                     double *__restrict__ rhs) {
  __shared__ double xch[4 * M];
  const long row = blockIdx.x;
  const int j = int(row / n) + 1;
  const int c = int(row - long(j - 1) * n);
  const long EA = long(d + 1) * N * n, Er = long(d + 1) * n, El = long(d + 1) * N;
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  const mdr<M> s = dot4<M, true>(N, seg, [&](int i, mdc<M> &x, mdc<M> &y) {
    x = cload<M>(A, EA, (long(j) * N + i) * n + c);
    y = cload<M>(lam, El, long(k) * N + i);
  }, xch);
  if (w == 0 && (lane == 0 || lane == 2)) {
    const long e = long(k - j) * n + c;
    double *rp = rhs + size_t(lane >> 1) * M * Er;
    rstore<M>(rp, Er, e, md_add<M>(rload<M>(rp, Er, e), md_neg<M>(s)));
  }
}

template <int M>
__global__ void __launch_bounds__(256) k_adj_copy(long E, const double *__restrict__ a,
                                              double *__restrict__ b) {
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < E;
       e += long(gridDim.x) * blockDim.x)
    cstore<M>(b, E, e, cload<M>(a, E, e));
}

// contraction with stored monomial series: one wave per term
template <int M>
__global__ void __launch_bounds__(64) k_adj_contract_stored(EvalArgs a, const double *lam,
                                                            double *grad) {
  const int tau = blockIdx.x;
  int i = 0;
  while (i + 1 < a.N && a.eq_ptr[i + 1] <= tau) ++i;  // the equation of term tau
  contract_wave<M>(nullptr, 0, a.mono, long(a.Mt) * (a.d + 1), long(tau) * (a.d + 1), lam, a.N,
                   i, a.d, a.dc, tau, a.Mt, grad);
}

}  // namespace mds

using namespace mds;

extern "C" int md_newton_adjoint(int m, int d, const md_system *sys, const double *x,
                                 const double *grad_x, int store_monomials, double *grad_coef,
                                 void *ws, size_t ws_bytes, int32_t *status, void *stream) {
  if (!sys) return fail(MD_ENULL, "md_newton_adjoint: null system");
  if (d < 0) return fail(MD_EINVAL, "md_newton_adjoint: d=%d < 0", d);
  if (!valid_m(m)) return dispatch_m(m, [](auto) { return MD_OK; });
  const int N = sys->N, n = sys->n;
  if (n < 1 || N < n || N > 256)
    return fail(MD_ESHAPE, "md_newton_adjoint: need 256 >= N >= n >= 1 (N=%d n=%d)", N, n);
  if (!x || !grad_x || !grad_coef) return fail(MD_ENULL, "md_newton_adjoint: null pointer");
  const bool store = store_monomials != 0;
  AdjointLayout lay(m, N, n, d, sys->M, sys->max_deg, store);
  if (!ws || ws_bytes < lay.bytes || !aligned256(ws))
    return fail(MD_EWORKSPACE, "md_newton_adjoint: workspace %zu bytes < %zu or misaligned",
                ws_bytes, lay.bytes);
  hipStream_t s = (hipStream_t)stream;
  char *w = static_cast<char *>(ws);
  const NewtonLayout &nl = lay.nl;
  double *f = reinterpret_cast<double *>(w + nl.off_f);
  double *A = reinterpret_cast<double *>(w + nl.off_A);
  double *QR = reinterpret_cast<double *>(w + nl.off_QR);
  double *vd = reinterpret_cast<double *>(w + nl.off_vd);
  double *beta = reinterpret_cast<double *>(w + nl.off_beta);
  const SolveLayout sl(m, N, n, d);
  double *rhs = reinterpret_cast<double *>(w + nl.off_solve + sl.off_r);
  double *W = reinterpret_cast<double *>(w + nl.off_solve + sl.off_G);
  double *invd = W + size_t(2) * m * n * N;
  double *lam = reinterpret_cast<double *>(w + lay.off_lam);
  double *mono = store ? reinterpret_cast<double *>(w + lay.off_mono) : nullptr;
  int rc = eval_diff_enqueue(m, d, *sys, x, f, A, w + nl.off_eval, nl.bytes - nl.off_eval, s, mono);
  if (rc) return rc;
  rc = qr_enqueue(m, N, n, A, long(d + 1) * N * n, QR, vd, beta, status, s, nullptr,
                  reinterpret_cast<int32_t *>(w + nl.off_ctr));
  if (rc) return rc;
  rc = pinv_enqueue(m, N, n, QR, vd, beta, invd, W,
                    reinterpret_cast<double *>(w + nl.off_solve + sl.off_pw), status, s);
  if (rc) return rc;
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const long Er = long(d + 1) * n;
    long blocks = (Er + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_adj_copy<Mm><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(Er, grad_x, rhs);
    const int seg_l = n >= WAVE ? WAVE : pow2_at_least(n);
    const int seg_u = N >= WAVE ? WAVE : pow2_at_least(N);
    const bool l4 = Mm >= 3 && n >= 5 && n <= WAVE, u4 = Mm >= 3 && N >= 5 && N <= WAVE;
    for (int k = d; k >= 0; --k) {
      if (l4) {
        k_adj_lambda4<Mm><<<dim3(unsigned(N)), dim3(256), 0, s>>>(k, N, n, d, seg_l, W, rhs, lam,
                                                                  status);
      } else {
        const long wl = (long(N) * seg_l + WAVE - 1) / WAVE;
        k_adj_lambda<Mm><<<dim3(unsigned((wl + 3) / 4)), dim3(256), 0, s>>>(k, N, n, d, seg_l, W,
                                                                             rhs, lam, status);
      }
      if (k > 0 && u4 && long(k) * n <= 512) {
        k_adj_update4<Mm><<<dim3(unsigned(long(k) * n)), dim3(256), 0, s>>>(k, N, n, d, seg_u, A,
                                                                            lam, rhs);
      } else if (k > 0) {
        const long wu = (long(k) * n * seg_u + WAVE - 1) / WAVE;
        k_adj_update<Mm><<<dim3(unsigned((wu + 3) / 4)), dim3(256), 0, s>>>(k, N, n, d, seg_u, A,
                                                                             lam, rhs);
      }
    }
    EvalArgs a{};
    a.d = d;
    a.N = N;
    a.n = n;
    a.Mt = sys->M;
    a.dc = sys->dc;
    a.Dmax = sys->max_deg;
    a.eq_ptr = sys->eq_ptr;
    a.term_ptr = sys->term_ptr;
    a.factors = sys->factors;
    a.coef = sys->coef;
    a.x = x;
    a.mono = mono;
    if (sys->M > 0) {
      if (store) {
        k_adj_contract_stored<Mm><<<dim3(sys->M), dim3(64), 0, s>>>(a, lam, grad_coef);
      } else {
        const int rc2 = contract_recompute_enqueue(Mm, a, lam, grad_coef, s);
        if (rc2) return rc2;
      }
    }
    return check_launch("md_newton_adjoint");
  });
}
