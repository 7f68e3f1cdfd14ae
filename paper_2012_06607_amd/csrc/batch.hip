// Many independent solution paths in one persistent launch.
//
// The paper's job queue (Section 5, Figure 1): all data is set up before
// the workers start, each job reads shared inputs and writes its own
// workspace, and a counter guarded by a lock hands out the next job.  Here
// the workers are workgroups resident on the GPU, the counter is one device
// atomic per queue, and a job is a whole path: `iters` Newton steps
// (evaluation and differentiation, QR of A_0, R^{-1} Q^H, the staggered
// solve, the update) run by that workgroup with barriers between the stages
// (the paper's stage synchronisation by terminating tasks).  Jobs are taken
// in the order the caller gives (longest first balances the load), and each
// workgroup dispatches on its path's precision.
//
// A large path may be a gang of G workgroups (G members, one job each).
// The members split the term evaluations, the Jacobian rows, the columns of
// each QR step, the columns of R^{-1} Q^H and the right-hand-side updates,
// and meet at gang barriers (a counter in device memory, with device-scope
// release and acquire).  The update of x runs on member 0; every member
// computes the stage products dx_k itself (the same bits), so a stage costs
// one gang barrier.
// With one queue per accelerator die (queue q served by the workgroups on
// die q) a gang's members share that die's L2.
#include "batch_kernel.hpp"

namespace mds {

// Before a launch: the job counters and the gang counters to zero, and every
// path marked not run (its member 0 clears the mark when it is done).
__global__ void __launch_bounds__(256) k_reset(int nq, int32_t *counters, int npaths,
                                               int32_t *gang_ctr, int32_t *status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nq) counters[t] = 0;
  if (t < npaths) {
    gang_ctr[t] = 0;
    atomicOr(status + t, MD_ST_NOTRUN);
  }
}

void launch_newton_batch_lo(int block, int grid, size_t lds, hipStream_t s, int npaths,
                            const md_path *paths, const int32_t *jobs, int nq,
                            const int32_t *qbegin, const int32_t *ints, double *reals, double *ws,
                            int iters, int32_t *counters, int32_t *gang_ctr, int32_t *status,
                            int eval_waves, int64_t *clk, int64_t *phase_clk) {
  if (block == 256)
    k_newton_batch<256, 0, false><<<dim3(grid), dim3(256), lds, s>>>(
        npaths, paths, jobs, nq, qbegin, ints, reals, ws, iters, counters, gang_ctr, status,
        eval_waves, clk, phase_clk, md_protocol{}, nullptr, nullptr);
  else
    k_newton_batch<512, 0, false><<<dim3(grid), dim3(512), lds, s>>>(
        npaths, paths, jobs, nq, qbegin, ints, reals, ws, iters, counters, gang_ctr, status,
        eval_waves, clk, phase_clk, md_protocol{}, nullptr, nullptr);
}

__global__ void k_xcc_ids(int32_t *out) {
  if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

}  // namespace mds

using namespace mds;

extern "C" size_t md_batch_lds_bytes(int max_m, int max_d, int max_deg, int eval_waves) {
  if (!(max_m >= 1 && max_m <= 4) && max_m != 5 && max_m != 8 && max_m != 10) return 0;
  if (max_d < 0 || max_deg < 0 || eval_waves < 1) return 0;
  // the evaluation's series, or a copy of one dx_k of up to 64 unknowns
  // during the stages, whichever is larger
  const size_t ev = sizeof(double) * 2 * size_t(max_m) * size_t(term_lds_series(max_deg)) *
                    (max_d + 1) * eval_waves;
  const size_t dxl = sizeof(double) * 2 * size_t(max_m) * WAVE;
  return ev > dxl ? ev : dxl;
}

namespace {

// Host checks shared by md_newton_batch and md_newton_batch_protocol; the
// evaluation's LDS bytes on success.
int batch_checks(const char *who, int npaths, const md_path *paths, int njobs,
                 const int32_t *jobs, int nq, const int32_t *qbegin, const int32_t *ints,
                 double *reals, double *ws, int iters, int32_t *counters, int32_t *gang_ctr,
                 int32_t *status, int max_m, int max_N, int max_d, int max_deg, int grid,
                 int block, int eval_waves, size_t &lds) {
  if (npaths < 0 || njobs < 0 || iters < 0 || grid < 1 || (block != 256 && block != 512) ||
      eval_waves < 1 || eval_waves > block / WAVE || nq < 1 || nq > 64)
    return fail(MD_EINVAL, "%s: npaths=%d njobs=%d iters=%d grid=%d block=%d eval_waves=%d nq=%d",
                who, npaths, njobs, iters, grid, block, eval_waves, nq);
  if (!(max_m >= 1 && max_m <= 4) && max_m != 5 && max_m != 8 && max_m != 10)
    return fail(MD_EINVAL, "%s: max_m=%d must be in 1..4 or one of 5, 8, 10", who, max_m);
  if (max_m >= 5 && block != 256)
    return fail(MD_EINVAL, "%s: penta to deca double paths run with 256 threads", who);
  if (max_N < 1 || max_N > WAVE)
    return fail(MD_ESHAPE, "%s: max_N=%d must be in 1..%d", who, max_N, WAVE);
  if (npaths == 0) return MD_OK;
  if (!paths || !jobs || !qbegin || !ints || !reals || !ws || !counters || !gang_ctr || !status)
    return fail(MD_ENULL, "%s: null pointer", who);
  lds = md_batch_lds_bytes(max_m, max_d, max_deg, eval_waves);
  if (lds == 0) return fail(MD_EINVAL, "%s: LDS size for max_m=%d", who, max_m);
  if (lds > lds_limit())
    return fail(MD_ESHAPE, "%s: %zu bytes of LDS for the evaluation exceed %zu", who, lds,
                lds_limit());
  return MD_OK;
}

}  // namespace

extern "C" int md_newton_batch(int npaths, const md_path *paths, int njobs, const int32_t *jobs,
                               int nq, const int32_t *qbegin, const int32_t *ints, double *reals,
                               double *ws, int iters, int32_t *counters, int32_t *gang_ctr,
                               int32_t *status, int max_m, int max_N, int max_d, int max_deg,
                               int grid, int block, int eval_waves, int64_t *path_clock,
                               int64_t *phase_clock, void *stream) {
  size_t lds = 0;
  const int rc = batch_checks("md_newton_batch", npaths, paths, njobs, jobs, nq, qbegin, ints,
                              reals, ws, iters, counters, gang_ctr, status, max_m, max_N, max_d,
                              max_deg, grid, block, eval_waves, lds);
  if (rc || npaths == 0) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int nr = npaths > nq ? npaths : nq;
  k_reset<<<dim3((nr + 255) / 256), dim3(256), 0, s>>>(nq, counters, npaths, gang_ctr, status);
  if (max_m <= 4)
    launch_newton_batch_lo(block, grid, lds, s, npaths, paths, jobs, nq, qbegin, ints, reals, ws,
                           iters, counters, gang_ctr, status, eval_waves, path_clock, phase_clock);
  else if (max_m == 5)
    launch_newton_batch_m5(grid, lds, s, npaths, paths, jobs, nq, qbegin, ints, reals, ws,
                           iters, counters, gang_ctr, status, eval_waves, path_clock, phase_clock);
  else if (max_m == 8)
    launch_newton_batch_m8(grid, lds, s, npaths, paths, jobs, nq, qbegin, ints, reals, ws,
                           iters, counters, gang_ctr, status, eval_waves, path_clock, phase_clock);
  else
    launch_newton_batch_m10(grid, lds, s, npaths, paths, jobs, nq, qbegin, ints, reals, ws,
                            iters, counters, gang_ctr, status, eval_waves, path_clock, phase_clock);
  return check_launch("md_newton_batch");
}

extern "C" int md_newton_batch_protocol(int npaths, const md_path *paths, int njobs,
                                        const int32_t *jobs, int nq, const int32_t *qbegin,
                                        const int32_t *ints, double *reals, double *ws,
                                        const md_protocol *proto, int32_t *counters,
                                        int32_t *gang_ctr, int32_t *status, int max_m, int max_N,
                                        int max_d, int max_deg, int grid, int block,
                                        int eval_waves, int32_t *proto_iters, double *proto_norms,
                                        void *stream) {
  const char *who = "md_newton_batch_protocol";
  if (!proto) return fail(MD_ENULL, "%s: null protocol", who);
  if (proto->ndeg < 1 || proto->ndeg > MD_PROTOCOL_MAX_DEGREES)
    return fail(MD_EINVAL, "%s: ndeg=%d outside 1..%d", who, proto->ndeg,
                MD_PROTOCOL_MAX_DEGREES);
  for (int j = 0; j < proto->ndeg; ++j) {
    if (proto->degrees[j] < 0 || (j > 0 && proto->degrees[j] <= proto->degrees[j - 1]))
      return fail(MD_EINVAL, "%s: degrees must increase from 0 up (degrees[%d]=%d)", who, j,
                  proto->degrees[j]);
    if (proto->maxit[j] < 0 || proto->maxit[j] > 10000)
      return fail(MD_EINVAL, "%s: maxit[%d]=%d outside 0..10000", who, j, proto->maxit[j]);
  }
  if (proto->min_steps < 1) return fail(MD_EINVAL, "%s: min_steps=%d < 1", who, proto->min_steps);
  if (!(proto->tol >= 0.0) || !(proto->diverge > 0.0) || !__builtin_isfinite(proto->tol) ||
      !__builtin_isfinite(proto->diverge))
    return fail(MD_EINVAL, "%s: need tol >= 0 and diverge > 0, finite", who);
  if (max_m > 4)
    return fail(MD_EINVAL, "%s: the protocol runs double to quad double paths (max_m=%d)", who,
                max_m);
  size_t lds = 0;
  const int rc = batch_checks(who, npaths, paths, njobs, jobs, nq, qbegin, ints, reals, ws, 0,
                              counters, gang_ctr, status, max_m, max_N, max_d, max_deg, grid,
                              block, eval_waves, lds);
  if (rc || npaths == 0) return rc;
  if (!proto_iters || !proto_norms) return fail(MD_ENULL, "%s: null iteration or norm output", who);
  hipStream_t s = (hipStream_t)stream;
  const int nr = npaths > nq ? npaths : nq;
  k_reset<<<dim3((nr + 255) / 256), dim3(256), 0, s>>>(nq, counters, npaths, gang_ctr, status);
  launch_newton_batch_proto(block, grid, lds, s, npaths, paths, jobs, nq, qbegin, ints, reals, ws,
                            counters, gang_ctr, status, eval_waves, nullptr, nullptr, *proto,
                            proto_iters, proto_norms);
  return check_launch(who);
}

extern "C" int md_device_dies(int32_t *ids, int nblocks, void *stream) {
  if (!ids) return fail(MD_ENULL, "md_device_dies: null pointer");
  if (nblocks < 1) return fail(MD_EINVAL, "md_device_dies: nblocks=%d", nblocks);
  k_xcc_ids<<<dim3(nblocks), dim3(64), 0, (hipStream_t)stream>>>(ids);
  return check_launch("md_device_dies");
}

extern "C" int md_wall_clock_hz(int device, int64_t *hz) {
  if (!hz) return fail(MD_ENULL, "md_wall_clock_hz: null pointer");
  int khz = 0;
  const hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device);
  if (e != hipSuccess) return fail(MD_EHIP, "md_wall_clock_hz: %s", hipGetErrorString(e));
  *hz = int64_t(khz) * 1000;
  return MD_OK;
}
