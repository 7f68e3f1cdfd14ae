// Coefficient-gradient contraction that recomputes each term's monomial
// series in LDS instead of reading a stored copy (one wave per term), for
// the adjoint of the converged series solution.  A translation unit of its
// own: compiled together with the stored-series kernel it crashes the
// device compiler's inliner.
#include "internal.hpp"
#include "wg.hpp"

namespace mds {

// contraction recomputing the monomial series in LDS: one wave per term
template <int M>
__global__ void __launch_bounds__(64) k_adj_contract_recompute(EvalArgs a, int r, const double *lam,
                                                               double *grad) {
  extern __shared__ double lds_raw[];
  const int tau = blockIdx.x;
  int i = 0;
  while (i + 1 < a.N && a.eq_ptr[i + 1] <= tau) ++i;
  if (a.term_ptr[tau + 1] - a.term_ptr[tau] > a.Dmax) return;  // the host validates max_deg
  const mdc<M> *mono = monomial_wave<M>(a, tau, r, reinterpret_cast<mdc<M> *>(lds_raw),
                                        [] { __syncthreads(); });
  contract_wave<M>(mono, 1, nullptr, 0, 0, lam, a.N, i, a.d, a.dc, tau, a.Mt, grad);
}

int contract_recompute_enqueue(int m, const EvalArgs &a, const double *lam, double *grad,
                               hipStream_t s) {
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const size_t lds =
        sizeof(double) * 2 * Mm * size_t(2 * (a.Dmax > 0 ? a.Dmax : 1)) * (a.d + 1);
    if (lds > lds_limit())
      return fail(MD_ESHAPE, "md_newton_adjoint: recomputing needs %zu bytes of LDS", lds);
    k_adj_contract_recompute<Mm><<<dim3(a.Mt), dim3(64), lds, s>>>(a, eval_group(a.d), lam, grad);
    return check_launch("md_newton_adjoint (contraction)");
  });
}

}  // namespace mds
