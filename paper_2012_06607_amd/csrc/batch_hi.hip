// The batched persistent launch for penta, octo and deca double paths (the
// kernel of batch_kernel.hpp instantiated for m in {5, 8, 10}, 256 threads
// per workgroup), in a translation unit of its own so that it compiles in
// parallel with the double- to quad-double one.
#include "batch_kernel.hpp"

namespace mds {

void launch_newton_batch_hi(int grid, size_t lds, hipStream_t s, int npaths, const md_path *paths,
                            const int32_t *jobs, int nq, const int32_t *qbegin,
                            const int32_t *ints, double *reals, double *ws, int iters,
                            int32_t *counters, int32_t *gang_ctr, int32_t *status, int eval_waves,
                            int64_t *clk) {
  k_newton_batch<256, true><<<dim3(grid), dim3(256), lds, s>>>(
      npaths, paths, jobs, nq, qbegin, ints, reals, ws, iters, counters, gang_ctr, status,
      eval_waves, clk);
}

}  // namespace mds
