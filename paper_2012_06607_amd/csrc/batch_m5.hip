// The batched persistent launch for penta double paths (the kernel of
// batch_kernel.hpp for m = 5, 256 threads per workgroup), in a translation
// unit of its own so that the wide precisions compile in parallel.
#include "batch_kernel.hpp"

namespace mds {

MDS_BATCH_WIDE_LAUNCH(launch_newton_batch_m5) {
  k_newton_batch<256, 5, false><<<dim3(grid), dim3(256), lds, s>>>(
      npaths, paths, jobs, nq, qbegin, ints, reals, ws, iters, counters, gang_ctr, status,
      eval_waves, clk, phase_clk, md_protocol{}, nullptr, nullptr);
}

}  // namespace mds
