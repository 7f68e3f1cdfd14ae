// One Newton step on truncated power series (Section 4): evaluation and
// differentiation, b = -f, one QR of A_0, the staggered solve, x += dx, and
// the size of the update (Section 6: the modulus of the update to the last
// coefficient).
#include "internal.hpp"
#include "layout.hpp"

namespace mds {

template <int M>
__global__ void __launch_bounds__(256) k_update(long E, const double *__restrict__ dx,
                                                double *__restrict__ x) {
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < E;
       e += long(gridDim.x) * blockDim.x)
    cstore<M>(x, E, e, c_add<M>(cload<M>(x, E, e), cload<M>(dx, E, e)));
}

// max_i |dx_{d,i}| and max_{k,i} |dx_{k,i}| (maxima of |.|^2 are exact
// selections, then one square root each), written as real planes (m, 2).
// out[0] on entry is the previous step's |dx_d| (or zero): a larger one now
// sets MD_ST_DIVERGED.
template <int M>
__global__ void __launch_bounds__(256) k_norms(int d, int n, const double *__restrict__ dx,
                                               double *__restrict__ out, int32_t *status) {
  __shared__ mdr<M> sh_d[256], sh_a[256];
  const long E = long(d + 1) * n;
  const int t = threadIdx.x;
  mdr<M> bd = md_zero<M>(), ba = md_zero<M>();
  for (long e = t; e < E; e += blockDim.x) {
    const mdr<M> a2 = c_abs2<M>(cload<M>(dx, E, e));
    if (md_less<M>(ba, a2)) ba = a2;
    if (e >= long(d) * n && md_less<M>(bd, a2)) bd = a2;
  }
  sh_d[t] = bd;
  sh_a[t] = ba;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      if (md_less<M>(sh_d[t], sh_d[t + o])) sh_d[t] = sh_d[t + o];
      if (md_less<M>(sh_a[t], sh_a[t + o])) sh_a[t] = sh_a[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    const mdr<M> prev = rload<M>(out, 2, 0);
    const mdr<M> nd = md_sqrt<M>(sh_d[0]);
    if (status && prev.v[0] > 0.0 && md_less<M>(prev, nd)) atomicOr(status, MD_ST_DIVERGED);
    rstore<M>(out, 2, 0, nd);
    rstore<M>(out, 2, 1, md_sqrt<M>(sh_a[0]));
  }
}

}  // namespace mds

using namespace mds;

extern "C" int md_newton_step(int m, int d, const md_system *sys, double *x, double *dx_norm,
                              void *ws, size_t ws_bytes, int32_t *status, void *stream) {
  if (!sys) return fail(MD_ENULL, "md_newton_step: null system");
  if (d < 0) return fail(MD_EINVAL, "md_newton_step: d=%d < 0", d);
  if (!valid_m(m)) return dispatch_m(m, [](auto) { return MD_OK; });
  const int N = sys->N, n = sys->n;
  if (n < 1 || N < n) return fail(MD_ESHAPE, "md_newton_step: need N >= n >= 1 (N=%d n=%d)", N, n);
  if (!x) return fail(MD_ENULL, "md_newton_step: null x");
  NewtonLayout lay(m, N, n, d, sys->M, sys->max_deg);
  if (!ws || ws_bytes < lay.bytes || !aligned256(ws))
    return fail(MD_EWORKSPACE, "md_newton_step: workspace %zu bytes < %zu or misaligned", ws_bytes,
                lay.bytes);
  hipStream_t s = (hipStream_t)stream;
  char *w = static_cast<char *>(ws);
  double *f = reinterpret_cast<double *>(w + lay.off_f);
  double *A = reinterpret_cast<double *>(w + lay.off_A);
  double *QR = reinterpret_cast<double *>(w + lay.off_QR);
  double *vd = reinterpret_cast<double *>(w + lay.off_vd);
  double *beta = reinterpret_cast<double *>(w + lay.off_beta);
  double *dx = reinterpret_cast<double *>(w + lay.off_dx);
  int rc = eval_diff_enqueue(m, d, *sys, x, f, A, w + lay.off_eval, lay.bytes - lay.off_eval, s);
  if (rc) return rc;
  rc = qr_enqueue(m, N, n, A, long(d + 1) * N * n, QR, vd, beta, status, s);
  if (rc) return rc;
  rc = solve_enqueue(m, N, n, d, QR, vd, beta, A, f, true, dx, w + lay.off_solve,
                     lay.off_eval - lay.off_solve, status, s);
  if (rc) return rc;
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const long E = long(d + 1) * n;
    long blocks = (E + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_update<Mm><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(E, dx, x);
    if (dx_norm) k_norms<Mm><<<dim3(1), dim3(256), 0, s>>>(d, n, dx, dx_norm, status);
    return check_launch("md_newton_step (update)");
  });
}
