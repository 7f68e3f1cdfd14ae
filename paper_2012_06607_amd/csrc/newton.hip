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
                                                double *__restrict__ x, const int32_t *gate) {
  if (gate_closed(gate)) return;
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
                                               double *__restrict__ out, int32_t *status,
                                               const int32_t *gate) {
  __shared__ mdr<M> sh_d[256], sh_a[256];
  if (gate_closed(gate)) return;
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

// The Newton protocol of Section 6 over increasing truncation degrees.
// flags[0]: the current degree still runs; flags[1]: an earlier degree ended
// with |dx_d| above the divergence bound, so no later degree runs.

__global__ void k_proto_init(int32_t *flags) {
  if (threadIdx.x == 0) {
    flags[0] = 0;
    flags[1] = 0;
  }
}

// Start of degree j (truncation dj): the iterate is the start point with
// zero higher coefficients (each degree starts from the given point), the
// degree's step count and norm are zero, and it runs unless stopped.
template <int M>
__global__ void __launch_bounds__(256) k_proto_begin(int j, int ndeg, int dj, int n,
                                                     const double *__restrict__ x0,
                                                     double *__restrict__ xj,
                                                     double *__restrict__ nrm,
                                                     double *__restrict__ norms,
                                                     int32_t *flags, int32_t *iters) {
  const bool run = flags[1] == 0;
  __syncthreads();
  const long E = long(dj + 1) * n;
  for (long e = threadIdx.x; e < E; e += blockDim.x)
    cstore<M>(xj, E, e, e < n ? cload<M>(x0, n, e) : c_zero<M>());
  if (threadIdx.x == 0) {
    flags[0] = run ? 1 : 0;
    iters[j] = 0;
    rstore<M>(nrm, 2, 0, md_zero<M>());
    rstore<M>(nrm, 2, 1, md_zero<M>());
    rstore<M>(norms, ndeg, j, md_zero<M>());
  }
}

// After a step of the running degree j: count it, and end the degree once
// the modulus of the update to the last coefficient is at most tol (tested
// from step min_steps on).
template <int M>
__global__ void k_proto_check(int j, int min_steps, double tol, const double *__restrict__ nrm,
                              int32_t *flags, int32_t *iters) {
  if (threadIdx.x != 0 || flags[0] == 0) return;
  const int32_t done = iters[j] + 1;
  iters[j] = done;
  if (done >= min_steps && !md_less<M>(md_from<M>(tol), rload<M>(nrm, 2, 0))) flags[0] = 0;
}

// End of degree j: if it ran, its last |dx_d| is recorded, its series goes
// to x (coefficients above dj zero), and an |dx_d| above the divergence
// bound stops the later degrees (MD_ST_DIVERGED).
template <int M>
__global__ void __launch_bounds__(256) k_proto_end(int j, int ndeg, int dj, int dmax, int n,
                                                   double diverge, const double *__restrict__ xj,
                                                   const double *__restrict__ nrm,
                                                   double *__restrict__ x,
                                                   double *__restrict__ norms, int32_t *flags,
                                                   int32_t *status) {
  const bool ran = flags[1] == 0;
  __syncthreads();
  if (!ran) return;
  const long Ej = long(dj + 1) * n, E = long(dmax + 1) * n;
  for (long e = threadIdx.x; e < E; e += blockDim.x)
    cstore<M>(x, E, e, e < Ej ? cload<M>(xj, Ej, e) : c_zero<M>());
  if (threadIdx.x == 0) {
    const mdr<M> v = rload<M>(nrm, 2, 0);
    rstore<M>(norms, ndeg, j, v);
    flags[0] = 0;
    if (md_less<M>(md_from<M>(diverge), v)) {
      flags[1] = 1;
      if (status) atomicOr(status, MD_ST_DIVERGED);
    }
  }
}

}  // namespace mds

using namespace mds;

namespace {

// gate (optional): every kernel of the step returns at once while *gate == 0;
// norm_status: where the growth of |dx_d| is reported (MD_ST_DIVERGED)
int newton_step_impl(int m, int d, const md_system *sys, double *x, double *dx_norm, void *ws,
                     size_t ws_bytes, int32_t *status, hipStream_t s, const char *who,
                     const int32_t *gate = nullptr, int32_t *norm_status = nullptr,
                     bool growth = true) {
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
  int rc = eval_diff_enqueue(m, d, *sys, x, f, A, w + lay.off_eval, lay.bytes - lay.off_eval, s,
                             nullptr, gate);
  if (rc) return rc;
  // the QR's columns over several workgroups, meeting on the word at off_ctr
  rc = qr_enqueue(m, N, n, A, long(d + 1) * N * n, QR, vd, beta, status, s, gate,
                  reinterpret_cast<int32_t *>(w + lay.off_ctr));
  if (rc) return rc;
  rc = solve_enqueue(m, N, n, d, QR, vd, beta, A, f, true, dx, w + lay.off_solve,
                     lay.off_eval - lay.off_solve, status, s, gate);
  if (rc) return rc;
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const long E = long(d + 1) * n;
    long blocks = (E + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_update<Mm><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(E, dx, x, gate);
    if (dx_norm)
      k_norms<Mm><<<dim3(1), dim3(256), 0, s>>>(d, n, dx, dx_norm,
                                                growth ? status : norm_status, gate);
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

extern "C" int md_newton_protocol(int m, const md_system *sys, const double *x0, int ndeg,
                                  const int32_t *degrees, const int32_t *maxit, int min_steps,
                                  double tol, double diverge, double *x, int32_t *iters,
                                  double *norms,
                                  void *ws, size_t ws_bytes, int32_t *status, void *stream) {
  const char *who = "md_newton_protocol";
  if (!degrees || !maxit) return fail(MD_ENULL, "%s: null degree or iteration list", who);
  if (ndeg < 1 || ndeg > MD_PROTOCOL_MAX_DEGREES)
    return fail(MD_EINVAL, "%s: ndeg=%d outside 1..%d", who, ndeg, MD_PROTOCOL_MAX_DEGREES);
  for (int j = 0; j < ndeg; ++j) {
    if (degrees[j] < 0 || (j > 0 && degrees[j] <= degrees[j - 1]))
      return fail(MD_EINVAL, "%s: degrees must increase from 0 up (degrees[%d]=%d)", who, j,
                  degrees[j]);
    if (maxit[j] < 0 || maxit[j] > 10000)
      return fail(MD_EINVAL, "%s: maxit[%d]=%d outside 0..10000", who, j, maxit[j]);
  }
  if (min_steps < 1) return fail(MD_EINVAL, "%s: min_steps=%d < 1", who, min_steps);
  if (!(tol >= 0.0) || !(diverge > 0.0) || !__builtin_isfinite(tol) || !__builtin_isfinite(diverge))
    return fail(MD_EINVAL, "%s: need tol >= 0 and diverge > 0, finite", who);
  const int dmax = degrees[ndeg - 1];
  int rc = newton_check(m, dmax, sys, x, who);
  if (rc) return rc;
  if (!x0 || !iters || !norms) return fail(MD_ENULL, "%s: null x0, iters or norms", who);
  const int N = sys->N, n = sys->n;
  const ProtocolLayout pl(m, N, n, dmax, sys->M, sys->max_deg);
  if (!ws || ws_bytes < pl.bytes || !aligned256(ws))
    return fail(MD_EWORKSPACE, "%s: workspace %zu bytes < %zu or misaligned", who, ws_bytes,
                pl.bytes);
  hipStream_t s = (hipStream_t)stream;
  char *w = static_cast<char *>(ws);
  double *xj = reinterpret_cast<double *>(w + pl.off_x);
  double *nrm = reinterpret_cast<double *>(w + pl.off_nrm);
  int32_t *flags = reinterpret_cast<int32_t *>(w + pl.off_flags);
  k_proto_init<<<dim3(1), dim3(64), 0, s>>>(flags);
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    for (int j = 0; j < ndeg; ++j) {
      const int dj = degrees[j];
      k_proto_begin<Mm><<<dim3(1), dim3(256), 0, s>>>(j, ndeg, dj, n, x0, xj, nrm, norms, flags,
                                                      iters);
      for (int it = 0; it < maxit[j]; ++it) {
        const int r = newton_step_impl(Mm, dj, sys, xj, nrm, ws, pl.nl.bytes, status, s, who,
                                       flags, nullptr, false);
        if (r) return r;
        k_proto_check<Mm><<<dim3(1), dim3(64), 0, s>>>(j, min_steps, tol, nrm, flags, iters);
      }
      k_proto_end<Mm><<<dim3(1), dim3(256), 0, s>>>(j, ndeg, dj, dmax, n, diverge, xj, nrm, x,
                                                    norms, flags, status);
    }
    return check_launch(who);
  });
}
