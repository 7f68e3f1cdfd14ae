// The batched persistent launch with Section 6's protocol per path (the
// kernel of batch_kernel.hpp for double to quad double with the protocol
// on), in a translation unit of its own.
#include "batch_kernel.hpp"

namespace mds {

void launch_newton_batch_proto(int block, int grid, size_t lds, hipStream_t s, int npaths,
                               const md_path *paths, const int32_t *jobs, int nq,
                               const int32_t *qbegin, const int32_t *ints, double *reals,
                               double *ws, int32_t *counters, int32_t *gang_ctr, int32_t *status,
                               int eval_waves, int64_t *clk, int64_t *phase_clk,
                               const md_protocol &proto, int32_t *proto_iters,
                               double *proto_norms) {
  if (block == 256)
    k_newton_batch<256, 0, true><<<dim3(grid), dim3(256), lds, s>>>(
        npaths, paths, jobs, nq, qbegin, ints, reals, ws, 0, counters, gang_ctr, status,
        eval_waves, clk, phase_clk, proto, proto_iters, proto_norms);
  else
    k_newton_batch<512, 0, true><<<dim3(grid), dim3(512), lds, s>>>(
        npaths, paths, jobs, nq, qbegin, ints, reals, ws, 0, counters, gang_ctr, status,
        eval_waves, clk, phase_clk, proto, proto_iters, proto_norms);
}

}  // namespace mds
