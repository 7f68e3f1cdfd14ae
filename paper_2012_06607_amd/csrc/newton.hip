// One Newton step on truncated power series (Section 4): evaluation and
// differentiation, b = -f, one QR of A_0, the staggered solve, x += dx, and
// the size of the update (Section 6: the modulus of the update to the last
// coefficient).
#include <mutex>

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

namespace {

int newton_step_impl(int m, int d, const md_system *sys, double *x, double *dx_norm, void *ws,
                     size_t ws_bytes, int32_t *status, hipStream_t s, const char *who) {
  const int N = sys->N, n = sys->n;
  NewtonLayout lay(m, N, n, d, sys->M, sys->max_deg);
  if (!ws || ws_bytes < lay.bytes || !aligned256(ws))
    return fail(MD_EWORKSPACE, "%s: workspace %zu bytes < %zu or misaligned", who, ws_bytes,
                lay.bytes);
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
    return check_launch(who);
  });
}

int newton_check(int m, int d, const md_system *sys, const double *x, const char *who) {
  if (!sys) return fail(MD_ENULL, "%s: null system", who);
  if (d < 0) return fail(MD_EINVAL, "%s: d=%d < 0", who, d);
  if (!valid_m(m)) return dispatch_m(m, [](auto) { return MD_OK; });
  if (sys->n < 1 || sys->N < sys->n)
    return fail(MD_ESHAPE, "%s: need N >= n >= 1 (N=%d n=%d)", who, sys->N, sys->n);
  if (!x) return fail(MD_ENULL, "%s: null x", who);
  return MD_OK;
}

// The fixed scratch of md_newton_step_noalloc: one copy per GPU, held from
// the library's load until the process ends.  Host code never passes this
// name to a kernel (on the host it is a stand-in, not a device address): it
// takes the device address from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[MD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(MD_EHIP, "md_newton_step_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(MD_EINVAL, "md_newton_step_noalloc: device %d outside 0..%d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MD_EHIP, "md_newton_step_noalloc: hipGetSymbolAddress of the scratch on device %d: %s",
                  dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MD_OK;
}

}  // namespace

extern "C" int md_newton_step(int m, int d, const md_system *sys, double *x, double *dx_norm,
                              void *ws, size_t ws_bytes, int32_t *status, void *stream) {
  const int rc = newton_check(m, d, sys, x, "md_newton_step");
  if (rc) return rc;
  return newton_step_impl(m, d, sys, x, dx_norm, ws, ws_bytes, status, (hipStream_t)stream,
                          "md_newton_step");
}

extern "C" int md_newton_step_noalloc(int m, int d, const md_system *sys, double *x,
                                      double *dx_norm, int32_t *status, void *stream) {
  const char *who = "md_newton_step_noalloc";
  int rc = newton_check(m, d, sys, x, who);
  if (rc) return rc;
  const size_t need = NewtonLayout(m, sys->N, sys->n, d, sys->M, sys->max_deg).bytes;
  if (need > MD_NOALLOC_SCRATCH_BYTES)
    return fail(MD_EWORKSPACE,
                "%s: this step needs %zu bytes of scratch, above the fixed %zu (use md_newton_step "
                "with a workspace)",
                who, need, size_t(MD_NOALLOC_SCRATCH_BYTES));
  void *ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  return newton_step_impl(m, d, sys, x, dx_norm, ws, MD_NOALLOC_SCRATCH_BYTES, status,
                          (hipStream_t)stream, who);
}
