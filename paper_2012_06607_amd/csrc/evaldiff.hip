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
#include "layout.hpp"
#include "series.hpp"

namespace mds {

struct EvalArgs {
  int d, N, n, Mt, dc, Dmax, S;
  const int *eq_ptr, *term_ptr, *factors;
  const double *coef, *x;
  double *ws;
  long Ews;
  double *f, *A;
  EvalLayout lay;
};

template <int M>
__global__ void __launch_bounds__(256) k_eval_terms(EvalArgs a) {
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

// One 64-lane workgroup per term; the term's factor series, its coefficient
// series and every forward, backward and cross product live in LDS.  The
// ceil((d+1)/2) coefficient pairs (k, d-k) are spread over groups of r
// lanes (r a power of two); lane `sub` of a group adds the products with
// i = sub mod r in increasing i, and the group's partial sums are combined
// by a fixed-order tree, so the bits do not depend on timing.
struct TermLds {
  int Dmax, L;
  __device__ int xs(int q) const { return q; }                 // factor q = 0..D-1
  __device__ int cs() const { return Dmax; }
  __device__ int P(int j) const { return Dmax + 1 + (j - 2); }  // j = 2..D
  __device__ int Q(int j) const { return 2 * Dmax + (j - 2); }  // j = 2..D-1
  __device__ int C(int j) const { return 3 * Dmax - 2 + (j - 2); }  // j = 2..D-1
};

__host__ __device__ inline int term_lds_series(int Dmax) {
  return Dmax < 2 ? Dmax + 1 : 4 * Dmax - 4;
}

template <int M>
__device__ __forceinline__ mdc<M> conv_part(const mdc<M> *X, int dx, const mdc<M> *Y, int k,
                                            int sub, int r) {
  const int top = k < dx ? k : dx;
  mdc<M> acc = c_zero<M>();
  bool first = true;
  for (int i = sub; i <= top; i += r) {
    const mdc<M> t = c_mul<M>(X[i], Y[k - i]);
    acc = first ? t : c_add<M>(acc, t);
    first = false;
  }
  return acc;
}

// products z = X Y (deg X <= dx) for the coefficient pairs of this lane's
// group, written to Z (LDS or, with zs != nullptr, to the workspace slot)
template <int M>
__device__ __forceinline__ void conv_group(const mdc<M> *X, int dx, const mdc<M> *Y, mdc<M> *Z,
                                           int d, int pg, int npg, int sub, int r,
                                           double *ws, long Ews, long wbase, int mult) {
  for (int p = pg; p < (d + 2) / 2; p += npg) {
    const int k1 = p, k2 = d - p;
    mdc<M> z1 = conv_part<M>(X, dx, Y, k1, sub, r);
    mdc<M> z2 = conv_part<M>(X, dx, Y, k2, sub, r);
    z1 = seg_reduce_c<M>(z1, r);
    z2 = seg_reduce_c<M>(z2, r);
    if (sub == 0) {
      if (mult > 1) {
        z1.re = md_muld<M>(z1.re, double(mult));
        z1.im = md_muld<M>(z1.im, double(mult));
        z2.re = md_muld<M>(z2.re, double(mult));
        z2.im = md_muld<M>(z2.im, double(mult));
      }
      if (Z) {
        Z[k1] = z1;
        Z[k2] = z2;
      } else {
        cstore<M>(ws, Ews, wbase + k1, z1);
        if (k2 != k1) cstore<M>(ws, Ews, wbase + k2, z2);
      }
    }
  }
}

template <int M>
__global__ void __launch_bounds__(64) k_eval_terms_wave(EvalArgs a, int r) {
  extern __shared__ double lds_raw[];
  mdc<M> *lds = reinterpret_cast<mdc<M> *>(lds_raw);
  const int tau = blockIdx.x;
  const int d = a.d, L = d + 1;
  const TermLds T{a.Dmax, L};
  const int lane = threadIdx.x;
  const int sub = lane & (r - 1);
  const int pg = lane / r;
  const int npg = WAVE / r;
  const int D = a.term_ptr[tau + 1] - a.term_ptr[tau];
  if (D > a.Dmax) return;  // the host validates max_deg; never read past the slots
  const int *v = a.factors + a.term_ptr[tau];
  auto S = [&](int slot) { return lds + slot * L; };
  const long Ex = long(L) * a.n;
  // stage the factor series and the coefficient series
  for (int e = lane; e < D * L; e += WAVE) {
    const int q = e / L, k = e - q * L;
    S(T.xs(q))[k] = cload<M>(a.x, Ex, long(k) * a.n + v[q]);
  }
  for (int k = lane; k < L; k += WAVE)
    S(T.cs())[k] = (k <= a.dc) ? cload<M>(a.coef, long(a.Mt) * (a.dc + 1), long(tau) * (a.dc + 1) + k)
                               : c_zero<M>();
  __syncthreads();
  const int dcu = a.dc < d ? a.dc : d;
  const long wb = long(tau) * a.S * L;
  if (D == 0) {
    for (int k = lane; k < L; k += WAVE) cstore<M>(a.ws, a.Ews, wb + a.lay.val() * L + k, S(T.cs())[k]);
    return;
  }
  if (D == 1) {
    conv_group<M>(S(T.cs()), dcu, S(T.xs(0)), nullptr, d, pg, npg, sub, r, a.ws, a.Ews,
                  wb + a.lay.val() * L, 1);
    for (int k = lane; k < L; k += WAVE) cstore<M>(a.ws, a.Ews, wb + a.lay.der(1) * L + k, S(T.cs())[k]);
    return;
  }
  auto Pj = [&](int j) { return j == 1 ? S(T.xs(0)) : S(T.P(j)); };
  auto Qj = [&](int j) { return j == D ? S(T.xs(D - 1)) : S(T.Q(j)); };
  for (int st = 1; st <= D - 1; ++st) {
    conv_group<M>(Pj(st), d, S(T.xs(st)), S(T.P(st + 1)), d, pg, npg, sub, r, nullptr, 0, 0, 1);
    const int j = D - st;
    if (j >= 2) conv_group<M>(S(T.xs(j - 1)), d, Qj(j + 1), S(T.Q(j)), d, pg, npg, sub, r, nullptr, 0, 0, 1);
    __syncthreads();
  }
  for (int j = 2; j <= D - 1; ++j)
    if (v[j - 1] != v[j - 2]) conv_group<M>(Pj(j - 1), d, Qj(j + 1), S(T.C(j)), d, pg, npg, sub, r, nullptr, 0, 0, 1);
  __syncthreads();
  conv_group<M>(S(T.cs()), dcu, Pj(D), nullptr, d, pg, npg, sub, r, a.ws, a.Ews, wb + a.lay.val() * L, 1);
  for (int j = 1; j <= D; ++j) {
    if (j > 1 && v[j - 1] == v[j - 2]) continue;
    int mult = 0;
    for (int q = 0; q < D; ++q) mult += (v[q] == v[j - 1]);
    const mdc<M> *cross = (j == 1) ? Qj(2) : (j == D ? Pj(D - 1) : S(T.C(j)));
    conv_group<M>(S(T.cs()), dcu, cross, nullptr, d, pg, npg, sub, r, a.ws, a.Ews,
                  wb + a.lay.der(j) * L, mult);
  }
}

template <int M>
__global__ void __launch_bounds__(256) k_eval_accumulate(EvalArgs a) {
  const int L = a.d + 1;
  const long per_k = long(a.N) * (a.n + 1);
  const long total = per_k * L;
  for (long g = blockIdx.x * long(blockDim.x) + threadIdx.x; g < total;
       g += long(gridDim.x) * blockDim.x) {
    const int k = int(g / per_k);
    const long r = g - k * per_k;
    const int i = int(r / (a.n + 1));
    const int l = int(r - long(i) * (a.n + 1));
    mdc<M> acc = c_zero<M>();
    for (int tau = a.eq_ptr[i]; tau < a.eq_ptr[i + 1]; ++tau) {
      int slot = -1;
      if (l == a.n) {
        slot = a.lay.val();
      } else {
        const int b = a.term_ptr[tau], e = a.term_ptr[tau + 1];
        if (e - b <= a.Dmax)
          for (int q = b; q < e; ++q)
            if (a.factors[q] == l) {
              slot = a.lay.der(q - b + 1);
              break;
            }
      }
      if (slot >= 0)
        acc = c_add<M>(acc, cload<M>(a.ws, a.Ews, (long(tau) * a.S + slot) * L + k));
    }
    if (l == a.n) cstore<M>(a.f, long(L) * a.N, long(k) * a.N + i, acc);
    else cstore<M>(a.A, long(L) * a.N * a.n, (long(k) * a.N + i) * a.n + l, acc);
  }
}

int eval_diff_enqueue(int m, int d, const md_system &sys, const double *x, double *f, double *A,
                      void *ws, size_t ws_bytes, hipStream_t s) {
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
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    if (sys.M > 0) {
      const size_t lds = sizeof(double) * 2 * Mm * size_t(term_lds_series(sys.max_deg)) * (d + 1);
      if (lds <= 64 * 1024) {
        int r = 1;
        while (P * r * 2 <= WAVE) r *= 2;
        k_eval_terms_wave<Mm><<<dim3(sys.M), dim3(64), lds, s>>>(a, r);
      } else {
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
