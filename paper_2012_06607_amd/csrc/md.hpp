// Multiple-double arithmetic on the FP64 vector units of gfx950.
//
// A multiple double with M limbs is an unevaluated sum x_0 + ... + x_{M-1}
// of hardware doubles, limb 0 most significant (Section 2).  Every operation
// is built from error-free transformations (two-sum, fast two-sum, fma
// two-product) and runs fully unrolled in registers; nothing here touches
// memory.  The operation sequence of each routine is fixed (this file must be
// compiled with -ffp-contract=off), so a single operation gives the same
// bits on every run and matches any other implementation of the same
// sequence:
//   M = 1   plain double arithmetic;
//   M = 2   double-double: the accurate addition of Hida, Li and Bailey
//           (8 additions and 12 subtractions, Table 1) and the fma product;
//   M >= 3  addition: level i holds a_i, b_i and the errors carried from
//           level i-1, summed by a two-sum cascade whose errors go to level
//           i+1; the last level (M-1) is summed in plain arithmetic (its
//           rounding errors lie below the last limb), then the M level sums
//           are renormalised; multiplication: partial products a_i b_j with
//           i + j < M-1 as exact two-products, summed level by level in the
//           same way (level k: the products of level k in order of i, the low
//           parts of level k-1's products, then the carries), the last level's
//           products and sum in plain arithmetic;
//   division: long division with M+1 quotient digits (Table 1's "/" column);
//   1/sqrt: Newton steps y += y (1 - a y^2) / 2 from the hardware value,
//           ceil(log2 M)+1 of them; sqrt(a) = a * (1/sqrt(a)).
// Renormalisation of K >= M level sums: a bottom-up two-sum sweep, then a
// top-down two-sum sweep emitting limbs 0..M-2, the last limb collecting the
// remaining terms.  Multiple double times double (M >= 2): a_i b = p_i + q_i
// exactly for i < M-1, the last level plain.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace mds {

// Compile-time loop: f(integral_constant<int, I>) for I = B..E-1, so every
// limb and term index is a constant and all arrays stay in registers.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <int M>
struct mdr {
  double v[M];
};

template <int M>
struct mdc {
  mdr<M> re, im;
};

// ---------------------------------------------------------------------------
// error-free transformations

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  const double ss = a + b;
  const double bb = ss - a;
  const double ea = a - (ss - bb);
  const double eb = b - bb;
  s = ss;
  e = ea + eb;
}

__device__ __forceinline__ void fast_two_sum(double a, double b, double &s, double &e) {
  const double ss = a + b;
  e = b - (ss - a);
  s = ss;
}

__device__ __forceinline__ void two_prod(double a, double b, double &p, double &e) {
  const double pp = a * b;
  e = __builtin_fma(a, b, -pp);
  p = pp;
}

// ---------------------------------------------------------------------------
// helpers

template <int M>
__device__ __forceinline__ mdr<M> md_zero() {
  mdr<M> z;
#pragma unroll
  for (int i = 0; i < M; ++i) z.v[i] = 0.0;
  return z;
}

template <int M>
__device__ __forceinline__ mdr<M> md_from(double a) {
  mdr<M> z = md_zero<M>();
  z.v[0] = a;
  return z;
}

template <int M>
__device__ __forceinline__ mdr<M> md_neg(const mdr<M> &a) {
  mdr<M> z;
#pragma unroll
  for (int i = 0; i < M; ++i) z.v[i] = -a.v[i];
  return z;
}

// K level sums -> M limbs (K >= M)
template <int M, int K>
__device__ __forceinline__ mdr<M> renorm(const double (&x)[K]) {
  static_assert(K >= M, "renorm needs K >= M");
  double t[K];
  double s = x[K - 1];
  static_for<0, K - 1>([&](auto j) {
    constexpr int i = K - 2 - decltype(j)::value;
    double ns, e;
    two_sum(x[i], s, ns, e);
    s = ns;
    t[i + 1] = e;
  });
  t[0] = s;
  mdr<M> y;
  double e = t[0];
  static_for<0, M - 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    double r, ne;
    two_sum(e, t[i + 1], r, ne);
    y.v[i] = r;
    e = ne;
  });
  if constexpr (K > M) {
    double tail = t[K - 1];
    static_for<0, K - 1 - M>([&](auto j) {
      constexpr int i = K - 2 - decltype(j)::value;
      tail = tail + t[i];
    });
    e = e + tail;
  }
  y.v[M - 1] = e;
  return y;
}

// number of terms summed at level k of the product (k < M)
__host__ __device__ constexpr int mul_level_terms(int k) {
  return k == 0 ? 1 : (k + 1) + k + (mul_level_terms(k - 1) - 1);
}

// ---------------------------------------------------------------------------
// real operations

template <int M>
__device__ __forceinline__ mdr<M> md_add(const mdr<M> &a, const mdr<M> &b) {
  if constexpr (M == 1) {
    mdr<1> z;
    z.v[0] = a.v[0] + b.v[0];
    return z;
  } else if constexpr (M == 2) {
    double s, e, t, f;
    two_sum(a.v[0], b.v[0], s, e);
    two_sum(a.v[1], b.v[1], t, f);
    e = e + t;
    fast_two_sum(s, e, s, e);
    e = e + f;
    fast_two_sum(s, e, s, e);
    mdr<2> z;
    z.v[0] = s;
    z.v[1] = e;
    return z;
  } else {
    double carry[M + 1];
    double c[M];
    static_for<0, M>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      // terms: a_i, b_i, carry[0..i-1]
      if constexpr (i == M - 1) {
        // the last level in plain arithmetic
        double s = a.v[i] + b.v[i];
        static_for<0, i>([&](auto qc) { s = s + carry[decltype(qc)::value]; });
        c[i] = s;
      } else {
        double s = a.v[i];
        double nc[M + 1];
        {
          double ns, e;
          two_sum(s, b.v[i], ns, e);
          s = ns;
          nc[0] = e;
        }
        static_for<0, i>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          double ns, e;
          two_sum(s, carry[q], ns, e);
          s = ns;
          nc[q + 1] = e;
        });
        c[i] = s;
        static_for<0, i + 1>([&](auto qc) { carry[decltype(qc)::value] = nc[decltype(qc)::value]; });
      }
    });
    return renorm<M, M>(c);
  }
}

template <int M>
__device__ __forceinline__ mdr<M> md_sub(const mdr<M> &a, const mdr<M> &b) {
  return md_add<M>(a, md_neg<M>(b));
}

// The level sums of the product a b (M >= 3) before renormalisation: c_k
// collects level k's products and the errors carried from level k-1, and
// c_0 + ... + c_{M-1} is the product md_mul renormalises.
template <int M>
__device__ __forceinline__ void mul_levels(const mdr<M> &a, const mdr<M> &b, double (&c)[M]) {
  constexpr int CMAX = mul_level_terms(M - 1);
  double carry[CMAX];
  double lo[M];
  static_for<0, M>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int ncar = (k == 0) ? 0 : mul_level_terms(k - 1) - 1;
    constexpr int nt = (k + 1) + k + ncar;
    if constexpr (k == M - 1) {
      // the last level: plain products and a plain sum
      double s = a.v[0] * b.v[k];
      static_for<1, k + 1>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        s = s + a.v[i] * b.v[k - i];
      });
      static_for<0, k>([&](auto ic) { s = s + lo[decltype(ic)::value]; });
      static_for<0, ncar>([&](auto ic) { s = s + carry[decltype(ic)::value]; });
      c[k] = s;
    } else {
      double terms[CMAX];
      double newlo[M];
      static_for<0, k + 1>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        two_prod(a.v[i], b.v[k - i], terms[i], newlo[i]);
      });
      static_for<0, k>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        terms[k + 1 + i] = lo[i];
      });
      static_for<0, ncar>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        terms[2 * k + 1 + i] = carry[i];
      });
      double s = terms[0];
      static_for<1, nt>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        double ns, e;
        two_sum(s, terms[i], ns, e);
        s = ns;
        carry[i - 1] = e;
      });
      c[k] = s;
      static_for<0, k + 1>([&](auto ic) { lo[decltype(ic)::value] = newlo[decltype(ic)::value]; });
    }
  });
}

template <int M>
__device__ __forceinline__ mdr<M> md_mul(const mdr<M> &a, const mdr<M> &b) {
  if constexpr (M == 1) {
    mdr<1> z;
    z.v[0] = a.v[0] * b.v[0];
    return z;
  } else if constexpr (M == 2) {
    double p, e;
    two_prod(a.v[0], b.v[0], p, e);
    double t1 = a.v[0] * b.v[1];
    const double t2 = a.v[1] * b.v[0];
    t1 = t1 + t2;
    e = e + t1;
    fast_two_sum(p, e, p, e);
    mdr<2> z;
    z.v[0] = p;
    z.v[1] = e;
    return z;
  } else {
    double c[M];
    mul_levels<M>(a, b, c);
    return renorm<M, M>(c);
  }
}

// x + y + z for three sets of M level sums (limbs, or mul_levels output),
// by md_add's level cascade with three inputs a level: level i sums x_i,
// y_i, z_i and the errors carried from level i-1 by two-sums (its own
// errors going to level i+1), the last level in plain arithmetic, then one
// renormalisation.  With products as mul_levels gives them this is a fused
// multiply-add: one renormalisation instead of three.
template <int M>
__device__ __forceinline__ mdr<M> sum3_levels(const double (&x)[M], const double (&y)[M],
                                              const double (&z)[M]) {
  double carry[2 * M + 2];
  double c[M + 1];
  static_for<0, M + 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int nin = 2 * i;  // carries from level i-1
    if constexpr (i == M) {
      // a level below the last limb: the carries in plain arithmetic
      double s = carry[0];
      static_for<1, nin>([&](auto qc) { s = s + carry[decltype(qc)::value]; });
      c[i] = s;
    } else {
      double s = x[i];
      double nc[2 * M + 2];
      {
        double ns, e;
        two_sum(s, y[i], ns, e);
        s = ns;
        nc[0] = e;
        two_sum(s, z[i], ns, e);
        s = ns;
        nc[1] = e;
      }
      static_for<0, nin>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        double ns, e;
        two_sum(s, carry[q], ns, e);
        s = ns;
        nc[q + 2] = e;
      });
      c[i] = s;
      static_for<0, nin + 2>([&](auto qc) { carry[decltype(qc)::value] = nc[decltype(qc)::value]; });
    }
  });
  return renorm<M, M + 1>(c);
}

// multiple double times hardware double
template <int M>
__device__ __forceinline__ mdr<M> md_muld(const mdr<M> &a, double b) {
  if constexpr (M == 1) {
    mdr<1> z;
    z.v[0] = a.v[0] * b;
    return z;
  } else {
    double p[M], q[M];
    static_for<0, M - 1>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      two_prod(a.v[i], b, p[i], q[i]);
    });
    p[M - 1] = a.v[M - 1] * b;
    double c[M];
    double carry[M];
    c[0] = p[0];
    static_for<1, M>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      // terms: p_i, q_{i-1}, carry[0..i-2]
      if constexpr (i == M - 1) {
        // the last level in plain arithmetic
        double s = p[i] + q[i - 1];
        static_for<0, i - 1>([&](auto rc) { s = s + carry[decltype(rc)::value]; });
        c[i] = s;
      } else {
        double s = p[i];
        double nc[M];
        {
          double ns, e;
          two_sum(s, q[i - 1], ns, e);
          s = ns;
          nc[0] = e;
        }
        static_for<0, i - 1>([&](auto rc) {
          constexpr int r = decltype(rc)::value;
          double ns, e;
          two_sum(s, carry[r], ns, e);
          s = ns;
          nc[r + 1] = e;
        });
        c[i] = s;
        static_for<0, i>([&](auto rc) { carry[decltype(rc)::value] = nc[decltype(rc)::value]; });
      }
    });
    return renorm<M, M>(c);
  }
}

template <int M>
__device__ __forceinline__ mdr<M> md_div(const mdr<M> &a, const mdr<M> &b) {
  if constexpr (M == 1) {
    mdr<1> z;
    z.v[0] = a.v[0] / b.v[0];
    return z;
  } else {
    double q[M + 1];
    mdr<M> r = a;
    static_for<0, M + 1>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      q[i] = r.v[0] / b.v[0];
      if constexpr (i < M) r = md_add<M>(r, md_neg<M>(md_muld<M>(b, q[i])));
    });
    return renorm<M, M + 1>(q);
  }
}

__host__ __device__ constexpr int rsqrt_iterations(int m) {
  int it = 1, p = 1;
  while (p < m) {
    p *= 2;
    it++;
  }
  return it;
}

template <int M>
__device__ __forceinline__ mdr<M> md_rsqrt(const mdr<M> &a) {
  const double y0 = 1.0 / __builtin_sqrt(a.v[0]);
  mdr<M> y = md_from<M>(y0);
  if constexpr (M > 1) {
    const mdr<M> one = md_from<M>(1.0);
    constexpr int nit = rsqrt_iterations(M);
#pragma unroll 1
    for (int it = 0; it < nit; ++it) {
      mdr<M> t = md_mul<M>(y, y);
      t = md_mul<M>(a, t);
      t = md_sub<M>(one, t);
      t = md_mul<M>(y, t);
#pragma unroll
      for (int i = 0; i < M; ++i) t.v[i] = t.v[i] * 0.5;
      y = md_add<M>(y, t);
    }
  }
  return y;
}

template <int M>
__device__ __forceinline__ mdr<M> md_sqrt(const mdr<M> &a) {
  if constexpr (M == 1) {
    mdr<1> z;
    z.v[0] = __builtin_sqrt(a.v[0]);
    return z;
  } else {
    const mdr<M> y = md_rsqrt<M>(a);
    mdr<M> s = md_mul<M>(a, y);
    const bool zero = (a.v[0] == 0.0);
#pragma unroll
    for (int i = 0; i < M; ++i) s.v[i] = zero ? 0.0 : s.v[i];
    return s;
  }
}

// a < b on values (sign of the leading nonzero limb of a - b)
template <int M>
__device__ __forceinline__ bool md_less(const mdr<M> &a, const mdr<M> &b) {
  const mdr<M> d = md_add<M>(a, md_neg<M>(b));
  int sgn = 0;
#pragma unroll
  for (int i = M - 1; i >= 0; --i) sgn = d.v[i] < 0.0 ? -1 : (d.v[i] > 0.0 ? 1 : sgn);
  return sgn < 0;
}

template <int M>
__device__ __forceinline__ bool md_finite(const mdr<M> &a) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < M; ++i) ok = ok && __builtin_isfinite(a.v[i]);
  return ok;
}

// ---------------------------------------------------------------------------
// complex operations

template <int M>
__device__ __forceinline__ mdc<M> c_zero() {
  mdc<M> z;
  z.re = md_zero<M>();
  z.im = md_zero<M>();
  return z;
}

template <int M>
__device__ __forceinline__ mdc<M> c_conj(const mdc<M> &a) {
  mdc<M> z;
  z.re = a.re;
  z.im = md_neg<M>(a.im);
  return z;
}

template <int M>
__device__ __forceinline__ mdc<M> c_neg(const mdc<M> &a) {
  mdc<M> z;
  z.re = md_neg<M>(a.re);
  z.im = md_neg<M>(a.im);
  return z;
}

template <int M>
__device__ __forceinline__ mdc<M> c_add(const mdc<M> &a, const mdc<M> &b) {
  mdc<M> z;
  z.re = md_add<M>(a.re, b.re);
  z.im = md_add<M>(a.im, b.im);
  return z;
}

template <int M>
__device__ __forceinline__ mdc<M> c_sub(const mdc<M> &a, const mdc<M> &b) {
  return c_add<M>(a, c_neg<M>(b));
}

template <int M>
__device__ __forceinline__ mdc<M> c_mul(const mdc<M> &a, const mdc<M> &b) {
  const mdr<M> p1 = md_mul<M>(a.re, b.re);
  const mdr<M> p2 = md_mul<M>(a.im, b.im);
  const mdr<M> p3 = md_mul<M>(a.re, b.im);
  const mdr<M> p4 = md_mul<M>(a.im, b.re);
  mdc<M> z;
  z.re = md_add<M>(p1, md_neg<M>(p2));
  z.im = md_add<M>(p3, p4);
  return z;
}

// s + a b for complex multiple doubles: up to double double c_add(s, c_mul(a, b));
// from three limbs on fused: the four real products as level sums, then
// s.re + (a.re b.re) + (-(a.im b.im)) and s.im + (a.re b.im) + (a.im b.re),
// each with one renormalisation (the same value to the last limb's
// rounding, with two renormalisations fewer per part).
template <int M>
__device__ __forceinline__ mdc<M> c_fmadd(const mdc<M> &s, const mdc<M> &a, const mdc<M> &b) {
  if constexpr (M <= 2) {
    return c_add<M>(s, c_mul<M>(a, b));
  } else {
    double p1[M], p2[M], p3[M], p4[M];
    mul_levels<M>(a.re, b.re, p1);
    mul_levels<M>(a.im, b.im, p2);
    mul_levels<M>(a.re, b.im, p3);
    mul_levels<M>(a.im, b.re, p4);
#pragma unroll
    for (int i = 0; i < M; ++i) p2[i] = -p2[i];
    mdc<M> z;
    z.re = sum3_levels<M>(s.re.v, p1, p2);
    z.im = sum3_levels<M>(s.im.v, p3, p4);
    return z;
  }
}

template <int M>
__device__ __forceinline__ mdc<M> c_mulr(const mdc<M> &a, const mdr<M> &r) {
  mdc<M> z;
  z.re = md_mul<M>(a.re, r);
  z.im = md_mul<M>(a.im, r);
  return z;
}

template <int M>
__device__ __forceinline__ mdr<M> c_abs2(const mdc<M> &a) {
  const mdr<M> p1 = md_mul<M>(a.re, a.re);
  const mdr<M> p2 = md_mul<M>(a.im, a.im);
  return md_add<M>(p1, p2);
}

template <int M>
__device__ __forceinline__ mdc<M> c_div(const mdc<M> &a, const mdc<M> &b) {
  const mdr<M> den = c_abs2<M>(b);
  const mdc<M> num = c_mul<M>(a, c_conj<M>(b));
  mdc<M> z;
  z.re = md_div<M>(num.re, den);
  z.im = md_div<M>(num.im, den);
  return z;
}

template <int M>
__device__ __forceinline__ bool c_finite(const mdc<M> &a) {
  return md_finite<M>(a.re) && md_finite<M>(a.im);
}

// ---------------------------------------------------------------------------
// limb planes: a complex tensor with E elements stores real limb l of element
// e at p[l*E + e] and imaginary limb l at p[(M+l)*E + e]

template <int M>
__device__ __forceinline__ mdc<M> cload(const double *__restrict__ p, long E, long e) {
  mdc<M> z;
#pragma unroll
  for (int l = 0; l < M; ++l) {
    z.re.v[l] = p[l * E + e];
    z.im.v[l] = p[(M + l) * E + e];
  }
  return z;
}

template <int M>
__device__ __forceinline__ void cstore(double *__restrict__ p, long E, long e, const mdc<M> &z) {
#pragma unroll
  for (int l = 0; l < M; ++l) {
    p[l * E + e] = z.re.v[l];
    p[(M + l) * E + e] = z.im.v[l];
  }
}

template <int M>
__device__ __forceinline__ mdr<M> rload(const double *__restrict__ p, long E, long e) {
  mdr<M> z;
#pragma unroll
  for (int l = 0; l < M; ++l) z.v[l] = p[l * E + e];
  return z;
}

template <int M>
__device__ __forceinline__ void rstore(double *__restrict__ p, long E, long e, const mdr<M> &z) {
#pragma unroll
  for (int l = 0; l < M; ++l) p[l * E + e] = z.v[l];
}

}  // namespace mds
