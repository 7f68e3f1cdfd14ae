// Evaluation and reverse-mode differentiation of a polynomial system at a
// power series point (Section 4).
//
// Kernel 1 (one group of ceil((d+1)/2) threads per term, each thread owning
// the coefficients k and d-k): the forward products P_j = v_1 ... v_j and
// backward products Q_j = v_j ... v_D advance together, one factor per step
// with a workgroup barrier between steps; then the cross products
// C_j = P_{j-1} Q_{j+1}; then the value c(t) P_D(t) and the derivatives
// a_l c(t) C_{j*}(t) go to the term's workspace slots.
// Kernel 2 (one thread per output coefficient): f_i and A_{i,l} are summed
// over the terms of equation i in term order, from zero.
#include "internal.hpp"
#include "wg.hpp"

namespace mds {


template <int M>
__global__ void __launch_bounds__(256) k_eval_terms(EvalArgs a) {
  if (gate_closed(a.gate)) return;
  const int d = a.d;
  const int P = pairs_of(d);
  const int T = blockDim.x / P;
  const int slot = threadIdx.x / P;
  const int p = threadIdx.x - slot * P;
  const int tau = blockIdx.x * T + slot;
  const bool active = (slot < T) && (tau < a.Mt);
  int D = 0;
  const int *v = a.factors;
  if (active) {
    D = a.term_ptr[tau + 1] - a.term_ptr[tau];
    v = a.factors + a.term_ptr[tau];
  }
  // a term longer than the workspace was sized for is left out (its slots
  // would overlap the next term's); the host validates max_deg
  const bool active_ok = active && D <= a.Dmax;
  const long L = d + 1;
  const long Ex = L * a.n;
  const int ks[2] = {p, d - p};
  const int nk = (d - p != p) ? 2 : 1;
  auto xref = [&](int var) { return SRef{a.x, Ex, long(var), long(a.n)}; };
  auto wref = [&](int s) { return SRef{a.ws, a.Ews, (long(tau) * a.S + s) * L, 1}; };
  auto wstore = [&](int s, int k, const mdc<M> &z) {
    cstore<M>(a.ws, a.Ews, (long(tau) * a.S + s) * L + k, z);
  };
  const EvalLayout &lay = a.lay;

  // forward and backward products, one factor per step
  for (int s = 1; s <= a.Dmax - 1; ++s) {
    if (active_ok && D >= 2) {
      if (s + 1 <= D) {
        const SRef Ps = (s == 1) ? xref(v[0]) : wref(lay.P(s));
        const SRef xv = xref(v[s]);
        for (int q = 0; q < nk; ++q) wstore(lay.P(s + 1), ks[q], conv_coef<M>(Ps, d, xv, ks[q]));
      }
      const int j = D - s;
      if (j >= 2) {
        const SRef Qn = (j + 1 == D) ? xref(v[D - 1]) : wref(lay.Q(j + 1));
        const SRef xv = xref(v[j - 1]);
        for (int q = 0; q < nk; ++q) wstore(lay.Q(j), ks[q], conv_coef<M>(xv, d, Qn, ks[q]));
      }
    }
    __syncthreads();
  }
  // cross products at the first position of each variable
  if (active_ok && D >= 3) {
    for (int j = 2; j <= D - 1; ++j) {
      if (v[j - 1] == v[j - 2]) continue;
      const SRef Pp = (j == 2) ? xref(v[0]) : wref(lay.P(j - 1));
      const SRef Qn = (j + 1 == D) ? xref(v[D - 1]) : wref(lay.Q(j + 1));
      for (int q = 0; q < nk; ++q) wstore(lay.C(j), ks[q], conv_coef<M>(Pp, d, Qn, ks[q]));
    }
  }
  __syncthreads();
  if (!active_ok) return;
  // coefficient products
  const SRef cref{a.coef, long(a.Mt) * (a.dc + 1), long(tau) * (a.dc + 1), 1};
  const int dcu = a.dc < d ? a.dc : d;
  for (int q = 0; q < nk; ++q) {
    const int k = ks[q];
    mdc<M> val;
    if (D == 0) {
      val = (k <= a.dc) ? sload<M>(cref, k) : c_zero<M>();
    } else {
      const SRef PD = (D == 1) ? xref(v[0]) : wref(lay.P(D));
      val = conv_coef<M>(cref, dcu, PD, k);
    }
    wstore(lay.val(), k, val);
  }
  for (int j = 1; j <= D; ++j) {
    if (j > 1 && v[j - 1] == v[j - 2]) continue;
    int mult = 0;
    for (int r = 0; r < D; ++r) mult += (v[r] == v[j - 1]);
    SRef cross{nullptr, 0, 0, 0};
    if (D >= 2) {
      if (j == 1) cross = (D == 2) ? xref(v[1]) : wref(lay.Q(2));
      else if (j == D) cross = (D == 2) ? xref(v[0]) : wref(lay.P(D - 1));
      else cross = wref(lay.C(j));
    }
    for (int q = 0; q < nk; ++q) {
      const int k = ks[q];
      mdc<M> der;
      if (D == 1) der = (k <= a.dc) ? sload<M>(cref, k) : c_zero<M>();
      else der = conv_coef<M>(cref, dcu, cross, k);
      if (mult > 1) {
        der.re = md_muld<M>(der.re, double(mult));
        der.im = md_muld<M>(der.im, double(mult));
      }
      wstore(lay.der(j), k, der);
    }
  }
}

// One 64-lane workgroup per term (eval_term_wave): the term's series live
// in LDS in the compact layout (LDS decides how many terms a CU holds:
// octo double at degree 4 and 33 coefficients, four instead of three),
// each coefficient pair's products are split over a group of lanes.
template <int M>
__global__ void __launch_bounds__(64) k_eval_terms_wave(EvalArgs a, int r) {
  extern __shared__ double lds_raw[];
  if (gate_closed(a.gate)) return;
  eval_term_wave<M, true>(a, blockIdx.x, r, reinterpret_cast<mdc<M> *>(lds_raw),
                          [] { __syncthreads(); });
}

template <int M>
__global__ void __launch_bounds__(256) k_eval_accumulate(EvalArgs a) {
  if (gate_closed(a.gate)) return;
  const long total = long(a.N) * (a.n + 1) * (a.d + 1);
  for (long g = blockIdx.x * long(blockDim.x) + threadIdx.x; g < total;
       g += long(gridDim.x) * blockDim.x)
    eval_accumulate_elem<M>(a, g);
}

int eval_diff_enqueue(int m, int d, const md_system &sys, const double *x, double *f, double *A,
                      void *ws, size_t ws_bytes, hipStream_t s, double *mono,
                      const int32_t *gate) {
  if (d < 0) return fail(MD_EINVAL, "md_poly_eval_diff: d=%d < 0", d);
  if (sys.N < 1 || sys.n < 1 || sys.M < 0 || sys.dc < 0 || sys.max_deg < 0)
    return fail(MD_ESHAPE, "md_poly_eval_diff: bad system sizes N=%d n=%d M=%d dc=%d max_deg=%d",
                sys.N, sys.n, sys.M, sys.dc, sys.max_deg);
  if (!x || !f || !A || !sys.eq_ptr || !sys.term_ptr || !sys.coef ||
      (sys.max_deg > 0 && !sys.factors))
    return fail(MD_ENULL, "md_poly_eval_diff: null pointer");
  const int P = (d + 2) / 2;
  if (P > 256) return fail(MD_ESHAPE, "md_poly_eval_diff: degree %d above 510", d);
  if (!valid_m(m)) return dispatch_m(m, [](auto) { return MD_OK; });
  EvalLayout lay(m, sys.N, sys.n, d, sys.M, sys.max_deg);
  if (!ws || ws_bytes < lay.bytes || !aligned256(ws))
    return fail(MD_EWORKSPACE, "md_poly_eval_diff: workspace %zu bytes < %zu or misaligned",
                ws_bytes, lay.bytes);
  EvalArgs a{d, sys.N, sys.n, sys.M, sys.dc, sys.max_deg, lay.S, sys.eq_ptr, sys.term_ptr,
             sys.factors, sys.coef, x, static_cast<double *>(ws), lay.E, f, A, lay};
  a.mono = mono;
  a.gate = gate;
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    if (sys.M > 0) {
      const size_t lds =
          sizeof(double) * 2 * Mm * size_t(term_lds_series(sys.max_deg, true)) * (d + 1);
      if (lds <= lds_limit()) {
        k_eval_terms_wave<Mm><<<dim3(sys.M), dim3(64), lds, s>>>(a, eval_group(d));
      } else {
        if (mono)
          return fail(MD_ESHAPE, "stored monomials need the one-wave evaluation (%zu bytes of LDS)", lds);
        const int T = 256 / P;
        const int blocks = (sys.M + T - 1) / T;
        k_eval_terms<Mm><<<dim3(blocks), dim3(256), 0, s>>>(a);
      }
      int rc = check_launch("md_poly_eval_diff (terms)");
      if (rc) return rc;
    }
    const long total = long(d + 1) * sys.N * (sys.n + 1);
    long blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_eval_accumulate<Mm><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(a);
    return check_launch("md_poly_eval_diff (accumulate)");
  });
}

}  // namespace mds

extern "C" int md_poly_eval_diff(int m, int d, const md_system *sys, const double *x, double *f,
                                 double *A, void *ws, size_t ws_bytes, void *stream) {
  if (!sys) return mds::fail(MD_ENULL, "md_poly_eval_diff: null system");
  return mds::eval_diff_enqueue(m, d, *sys, x, f, A, ws, ws_bytes, (hipStream_t)stream);
}
