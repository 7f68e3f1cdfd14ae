// Workgroup- and segment-level building blocks shared by the single-path
// kernels and the batched persistent kernel.
//
// A "segment" is a power-of-two group of `seg` lanes inside one wave; it owns
// one column (QR, R^{-1} Q^H) or one dot product (stage products), lanes over
// rows, and sums in a fixed tree order.  Every loop that contains a segment
// reduction has the same trip count for all lanes of a wave.
#pragma once

#include "layout.hpp"
#include "series.hpp"

namespace mds {

// ---------------------------------------------------------------------------
// 1/sqrt(a) by Newton steps y += y (1 - a y^2)/2 that double the working
// precision (2, 4, 8 limbs, then M), from the hardware value.  A step
// squares the relative error (times 3/2), and a double-double value is good
// to about 2^-104 rather than 2^-106, so a step from it reaches only about
// 2^-207: short of four limbs (2^-212), and a step from that short of eight
// (2^-424).  For M = 4 and M = 8 one more step at full precision follows.

template <int P, int M>
__device__ __forceinline__ mdr<P> trunc(const mdr<M> &a) {
  mdr<P> z;
#pragma unroll
  for (int i = 0; i < P; ++i) z.v[i] = i < M ? a.v[i] : 0.0;
  return z;
}

template <int P, int M>
__device__ __forceinline__ mdr<P> rsqrt_step(const mdr<M> &a, const mdr<P> &y) {
  const mdr<P> ap = trunc<P, M>(a);
  mdr<P> t = md_mul<P>(y, y);
  t = md_mul<P>(ap, t);
  t = md_sub<P>(md_from<P>(1.0), t);
  t = md_mul<P>(y, t);
#pragma unroll
  for (int i = 0; i < P; ++i) t.v[i] = t.v[i] * 0.5;
  return md_add<P>(y, t);
}

template <int M>
__device__ __forceinline__ mdr<M> rsqrt_doubling(const mdr<M> &a) {
  const double y0 = 1.0 / __builtin_sqrt(a.v[0]);
  if constexpr (M == 1) {
    return md_from<1>(y0);
  } else {
    mdr<2> y2 = rsqrt_step<2, M>(a, md_from<2>(y0));
    if constexpr (M == 2) {
      return rsqrt_step<2, 2>(a, y2);
    } else if constexpr (M == 3) {
      return rsqrt_step<M, M>(a, trunc<M, 2>(y2));
    } else if constexpr (M == 4) {
      return rsqrt_step<M, M>(a, rsqrt_step<M, M>(a, trunc<M, 2>(y2)));
    } else {
      mdr<4> y4 = rsqrt_step<4, M>(a, trunc<4, 2>(y2));
      if constexpr (M < 8) {
        return rsqrt_step<M, M>(a, trunc<M, 4>(y4));
      } else if constexpr (M == 8) {
        return rsqrt_step<M, M>(a, rsqrt_step<M, M>(a, trunc<M, 4>(y4)));
      } else {
        mdr<8> y8 = rsqrt_step<8, M>(a, trunc<8, 4>(y4));
        return rsqrt_step<M, M>(a, trunc<M, 8>(y8));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Householder QR by one workgroup (Section 4).  For column j: sigma (the
// 2-norm from the diagonal down) and alpha = A[j][j] give phi = alpha/|alpha|,
// v_j = (phi (|alpha| + sigma), tail), beta = 1/(sigma (sigma + |alpha|)),
// R_jj = -phi sigma; every trailing column l gets a_l -= beta (v^H a_l) v,
// one column per segment of lanes.
//
// Look-ahead: in step j, wave 0's first segment updates column j+1 and then,
// from the values it still holds, forms reflector j+1, while the other
// segments update the remaining columns (wave 0 takes no more than its
// first round, so that the next reflector is ready as early as possible).
// One barrier per column; the scalars of reflector j live in the LDS buffer
// j & 1.

template <int M>
struct QrShared {
  mdc<M> v0[2];
  mdr<M> beta[2];
};

template <int M>
__device__ __forceinline__ void qr_reflector_scalars(const mdr<M> &s, const mdc<M> &alpha, int j,
                                                     int n, bool keep, QrShared<M> &sh,
                                                     double *__restrict__ QR, long E,
                                                     double *__restrict__ vdiag,
                                                     double *__restrict__ beta, int &st);

// Reflector j from the column values the wave's first segment holds (rows
// lis + r*seg): the segment tree of |a_i|^2 over i >= j, alpha from the lane
// that holds row j; lane 0 of the wave stores the scalars when `keep` (all
// lanes of the wave call this).
// With HOLD false the column is read from QR (rows j.. as stored) instead of
// `col`.
template <int M, int RPL, bool HOLD = true>
__device__ __forceinline__ void qr_reflector(const mdc<M> (&col)[RPL], int j, int N, int n, int seg,
                                             bool keep, QrShared<M> &sh, double *__restrict__ QR,
                                             long E, double *__restrict__ vdiag,
                                             double *__restrict__ beta, int &st) {
  const int lane = lane_id();
  const int lis = lane & (seg - 1);
  mdr<M> s = md_zero<M>();
  mdc<M> alpha = c_zero<M>();
  bool first = true;
  auto row = [&](int i, const mdc<M> &cv) __attribute__((always_inline)) {
    if (i >= j && i < N) {
      const mdr<M> t = c_abs2<M>(cv);
      s = first ? t : md_add<M>(s, t);
      first = false;
      if (i == j) alpha = cv;
    }
  };
  if constexpr (HOLD) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) row(lis + r * seg, col[r]);
  } else {
    // rows read from QR, one at a time
#pragma unroll 1
    for (int r = 0; r < RPL; ++r) {
      const int i = lis + r * seg;
      if (i >= j && i < N) row(i, cload<M>(QR, E, long(i) * n + j));
    }
  }
  s = seg_reduce_r<M>(s, seg);
  alpha = shfl_c<M>(alpha, j & (seg - 1));
  qr_reflector_scalars<M>(s, alpha, j, n, keep, sh, QR, E, vdiag, beta, st);
}

// The scalars of reflector j from sigma^2 (on lane 0) and alpha (on every
// lane), by one wave: a short chain of md operations with the independent
// ones side by side on lanes 0..3 (lane 0 keeps the results): 1/sqrt and
// the product with it for sigma^2 (lane 0) and |alpha|^2 (lane 1), then
// phi = alpha/|alpha| (re, im on lanes 0, 1), then v_0 = phi (|alpha| +
// sigma) and R_jj = -phi sigma (lanes 0..3).
template <int M>
__device__ __forceinline__ void qr_reflector_scalars(const mdr<M> &s, const mdc<M> &alpha, int j,
                                                     int n, bool keep, QrShared<M> &sh,
                                                     double *__restrict__ QR, long E,
                                                     double *__restrict__ vdiag,
                                                     double *__restrict__ beta, int &st) {
  const int lane = lane_id();
  const int base = 0, sub = lane;
  const mdr<M> s2 = shfl_r<M>(s, base);
  const mdr<M> a2 = c_abs2<M>(alpha);
  const mdr<M> xq = sub == 0 ? s2 : a2;
  const mdr<M> yq = rsqrt_doubling<M>(xq);
  const mdr<M> zq = md_mul<M>(xq, yq);
  const mdr<M> ys = shfl_r<M>(yq, base), ya = shfl_r<M>(yq, base + 1);
  const mdr<M> sigma = shfl_r<M>(zq, base);
  const bool a_zero = a2.v[0] == 0.0;
  const mdr<M> aabs = a_zero ? md_zero<M>() : shfl_r<M>(zq, base + 1);
  const mdr<M> sp = md_add<M>(aabs, sigma);
  const mdr<M> bet_q = md_div<M>(ys, sp);
  const mdr<M> ph_q = md_mul<M>((sub & 1) ? alpha.im : alpha.re, ya);
  mdc<M> phi;
  if (a_zero) {
    phi = c_zero<M>();
    phi.re = md_from<M>(1.0);
  } else {
    phi.re = shfl_r<M>(ph_q, base);
    phi.im = shfl_r<M>(ph_q, base + 1);
  }
  const mdr<M> w_q = md_mul<M>((sub & 1) ? phi.im : phi.re, (sub & 2) ? sigma : sp);
  const mdr<M> w0 = shfl_r<M>(w_q, base), w1 = shfl_r<M>(w_q, base + 1);
  const mdr<M> w2 = shfl_r<M>(w_q, base + 2), w3 = shfl_r<M>(w_q, base + 3);
  if (keep && lane == 0) {
    mdr<M> bet = md_zero<M>();
    mdc<M> v0 = c_zero<M>(), rjj = c_zero<M>();
    if (s2.v[0] == 0.0) {
      st |= MD_ST_SINGULAR;
    } else {
      v0.re = w0;
      v0.im = w1;
      bet = bet_q;
      rjj.re = md_neg<M>(w2);
      rjj.im = md_neg<M>(w3);
    }
    if (!c_finite<M>(rjj) || !md_finite<M>(bet)) st |= MD_ST_NONFINITE;
    sh.v0[j & 1] = v0;
    sh.beta[j & 1] = bet;
    cstore<M>(vdiag, n, j, v0);
    rstore<M>(beta, n, j, bet);
    cstore<M>(QR, E, long(j) * n + j, rjj);
  }
}

// a_l -= beta (v^H a_l) v over rows i >= j by one segment; `anew` receives
// the updated values (zero outside rows j..N-1).  The diagonal entry of
// column j+1 is not stored: its reflector's R_jj replaces it.  With HOLD
// false nothing is held across the two passes: the reflector rows (v_j = v0,
// the stored tail below) and the column are read where used (twice, through
// L1), every updated entry is stored (the next reflector reads its column
// back; its R_jj then replaces the diagonal) and `anew` is not written.
template <int M, int RPL, bool HOLD = true>
__device__ __forceinline__ void qr_update_column(bool live, int l, int j, int N, int n, int seg,
                                                 const mdc<M> (&vi)[RPL], const mdc<M> &v0,
                                                 const mdr<M> &bet, double *__restrict__ QR,
                                                 long E, mdc<M> (&anew)[RPL]) {
  const int lane = lane_id();
  const int lis = lane & (seg - 1);
  if constexpr (!HOLD) {
    // one row at a time (the loops stay loops, so one row's values are live)
    auto vrow = [&](int i) __attribute__((always_inline)) {
      return i == j ? v0 : cload<M>(QR, E, long(i) * n + j);
    };
    mdc<M> w = c_zero<M>();
    bool first = true;
#pragma unroll 1
    for (int r = 0; r < RPL; ++r) {
      const int i = lis + r * seg;
      if (live && i >= j && i < N) {
        const mdc<M> t = c_mul<M>(c_conj<M>(vrow(i)), cload<M>(QR, E, long(i) * n + l));
        w = first ? t : c_add<M>(w, t);
        first = false;
      }
    }
    w = seg_reduce_c<M>(w, seg);
    w = shfl_c<M>(w, lane & ~(seg - 1));
    const mdc<M> bw = c_mulr<M>(w, bet);
#pragma unroll 1
    for (int r = 0; r < RPL; ++r) {
      const int i = lis + r * seg;
      if (live && i >= j && i < N)
        cstore<M>(QR, E, long(i) * n + l,
                  c_sub<M>(cload<M>(QR, E, long(i) * n + l), c_mul<M>(bw, vrow(i))));
    }
    return;
  }
  mdc<M> al[RPL];
  mdc<M> w = c_zero<M>();
  bool first = true;
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lis + r * seg;
    al[r] = c_zero<M>();
    if (live && i >= j && i < N) {
      al[r] = cload<M>(QR, E, long(i) * n + l);
      const mdc<M> t = c_mul<M>(c_conj<M>(vi[r]), al[r]);
      w = first ? t : c_add<M>(w, t);
      first = false;
    }
  }
  w = seg_reduce_c<M>(w, seg);
  w = shfl_c<M>(w, lane & ~(seg - 1));
  const mdc<M> bw = c_mulr<M>(w, bet);
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lis + r * seg;
    anew[r] = c_zero<M>();
    if (live && i >= j && i < N) {
      anew[r] = c_sub<M>(al[r], c_mul<M>(bw, vi[r]));
      if (!(l == j + 1 && i == l)) cstore<M>(QR, E, long(i) * n + l, anew[r]);
    }
  }
}

template <int M, int RPL>
__device__ __forceinline__ void qr_wg(QrShared<M> &sh, int N, int n, int seg, const double *__restrict__ A0,
                      long A0E, double *__restrict__ QR, double *__restrict__ vdiag,
                      double *__restrict__ beta, int &st) {
  const long E = long(N) * n;
  const int lane = lane_id();
  const int wave = threadIdx.x / WAVE;
  const int nwaves = blockDim.x / WAVE;
  const int lis = lane & (seg - 1);
  const int spw = WAVE / seg;
  const int slot = wave * spw + lane / seg;
  const int nslots = nwaves * spw;
  const int others = nslots - spw;  // slots outside wave 0
  for (long e = threadIdx.x; e < E; e += blockDim.x) cstore<M>(QR, E, e, cload<M>(A0, A0E, e));
  __syncthreads();
  // step j = -1 only loads column 0 and forms reflector 0
  for (int j = -1; j < n; ++j) {
    // with four or more rows per lane nothing is held across the rounds
    // (the reflector and column rows are read where they are used), except
    // up to double double, whose rows fit in the registers
    constexpr bool HOLD = RPL < 4 || M <= 2;
    mdc<M> vi[RPL], anew[RPL];
    mdc<M> v0 = c_zero<M>();
    mdr<M> bet = md_zero<M>();
    if (j >= 0) {
      v0 = sh.v0[j & 1];
      bet = sh.beta[j & 1];
      if constexpr (HOLD) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int i = lis + r * seg;
          vi[r] = c_zero<M>();
          if (i == j) vi[r] = v0;
          else if (i > j && i < N) vi[r] = cload<M>(QR, E, long(i) * n + j);
        }
      }
    }
    // Columns j+1.. go out round by round, one per slot.  Wave 0's first
    // segment has column j+1 in round 0 and then forms reflector j+1 (worth
    // about two rounds), so wave 0 stops after round k0 - 1 and the slots of
    // the other waves take the columns that are left.
    const int ncols = n - j - 1;
    int k0 = 0, rounds = 0;
    if (j < 0) {
      k0 = 1;
      rounds = wave == 0 ? 1 : 0;
    } else if (ncols > 0) {
      const int all = (ncols + nslots - 1) / nslots;
      if (others == 0) {
        k0 = all;
        rounds = all;
      } else {
        const int kall = (ncols + 2 * spw + nslots - 1) / nslots;
        k0 = kall > 3 ? kall - 2 : 1;
        if (k0 > all) k0 = all;
        const int rest = ncols - k0 * nslots;
        rounds = wave == 0 ? k0 : k0 + (rest > 0 ? (rest + others - 1) / others : 0);
      }
    }
    for (int k = 0; k < rounds; ++k) {
      const int l = k < k0 ? j + 1 + k * nslots + slot
                           : j + 1 + k0 * nslots + (k - k0) * others + (slot - spw);
      if (j < 0) {
        if constexpr (HOLD) {
#pragma unroll
          for (int r = 0; r < RPL; ++r) {
            const int i = lis + r * seg;
            anew[r] = (l < n && i < N) ? cload<M>(QR, E, long(i) * n + l) : c_zero<M>();
          }
        }
      } else {
        qr_update_column<M, RPL, HOLD>(l < n, l, j, N, n, seg, vi, v0, bet, QR, E, anew);
      }
      if (k == 0 && wave == 0 && j + 1 < n)
        qr_reflector<M, RPL, HOLD>(anew, j + 1, N, n, seg, true, sh, QR, E, vdiag, beta, st);
    }
    __syncthreads();
  }
}

// 1 / R_ii for i < n, threads [t0, t0 + nt) of the caller
template <int M>
__device__ __forceinline__ void inv_diag_range(int t, int nt, int N, int n, const double *__restrict__ QR,
                               double *__restrict__ invd, int &st) {
  const long E = long(N) * n;
  for (int i = t; i < n; i += nt) {
    const mdc<M> rii = cload<M>(QR, E, long(i) * n + i);
    if (rii.re.v[0] == 0.0 && rii.im.v[0] == 0.0) st |= MD_ST_SINGULAR;
    mdc<M> one = c_zero<M>();
    one.re = md_from<M>(1.0);
    cstore<M>(invd, n, i, c_div<M>(one, rii));
  }
}

// W = R^{-1} (Q^H)_{0:n} in two passes (the batched kernel's form).  Row r
// of (Q^H)_{0:n} is the
// conjugate of column r of Q, and Q e_r = H_0 H_1 ... H_r e_r because H_j
// (zero above row j) leaves e_r alone for j > r: r + 1 reflectors instead of
// n.  q_row forms that row (one segment, lanes own entries lis, lis+seg,
// ...; reflectors r, r-1, ..., 0) into W's buffer; after a barrier
// backsub_column turns column c of it into column c of W = R^{-1} (Q^H)_{0:n}
// in place.  Reflector j's rows are read where used (twice, through L1);
// the loops over a lane's entries are unrolled, so g stays in registers.
template <int M, int RPL>
__device__ __forceinline__ void q_row(bool live, int r, int N, int n, int seg,
                                      const double *__restrict__ QR,
                                      const double *__restrict__ vdiag,
                                      const double *__restrict__ beta, double *__restrict__ W) {
  const long E = long(N) * n;
  const long EW = long(n) * N;
  const int lane = lane_id();
  const int lis = lane & (seg - 1);
  auto vrow = [&](int j, int i, const mdc<M> &v0) __attribute__((always_inline)) {
    return i == j ? v0 : cload<M>(QR, E, long(i) * n + j);
  };
  mdc<M> g[RPL];
  {
    // H_r e_r = e_r - beta_r conj(v_r[r]) v_r
    const mdc<M> v0 = live ? cload<M>(vdiag, n, r) : c_zero<M>();
    const mdc<M> bw = c_mulr<M>(c_conj<M>(v0), live ? rload<M>(beta, n, r) : md_zero<M>());
    mdc<M> one = c_zero<M>();
    one.re = md_from<M>(1.0);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = lis + q * seg;
      g[q] = c_zero<M>();
      if (live && i >= r && i < N)
        g[q] = c_sub<M>(i == r ? one : c_zero<M>(), c_mul<M>(bw, vrow(r, i, v0)));
    }
  }
  // the wave runs the longest row's steps; a segment works in steps j < r
  const int rmax = wave_max_int(live ? r : 0);
  for (int j = rmax - 1; j >= 0; --j) {
    const bool act = live && j < r;
    const mdc<M> v0 = act ? cload<M>(vdiag, n, j) : c_zero<M>();
    const mdr<M> bet = act ? rload<M>(beta, n, j) : md_zero<M>();
    mdc<M> w = c_zero<M>();
    bool first = true;
    // up to double double the reflector's rows stay in registers for the
    // second pass; wider numbers read them again (registers are short)
    constexpr bool HOLDV = M <= 2;
    mdc<M> vq[HOLDV ? RPL : 1];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = lis + q * seg;
      if (act && i >= j && i < N) {
        const mdc<M> vv = vrow(j, i, v0);
        if constexpr (HOLDV) vq[q] = vv;
        const mdc<M> t = c_mul<M>(c_conj<M>(vv), g[q]);
        w = first ? t : c_add<M>(w, t);
        first = false;
      }
    }
    w = seg_reduce_c<M>(w, seg);
    w = shfl_c<M>(w, lane & ~(seg - 1));
    const mdc<M> bw = c_mulr<M>(w, bet);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = lis + q * seg;
      if (act && i >= j && i < N) {
        if constexpr (HOLDV) g[q] = c_sub<M>(g[q], c_mul<M>(bw, vq[q]));
        else g[q] = c_sub<M>(g[q], c_mul<M>(bw, vrow(j, i, v0)));
      }
    }
  }
  if (live) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = lis + q * seg;
      if (i < N) cstore<M>(W, EW, long(r) * N + i, c_conj<M>(g[q]));
    }
  }
}

// Column c of W = R^{-1} Y in place, Y = (Q^H)_{0:n} as q_row left it (lanes
// own rows lis, lis+seg, ... < n): the back substitution with the row owner
// multiplying by 1/R_ii and broadcasting.
template <int M, int RPL>
__device__ __forceinline__ void backsub_column(bool live, int c, int N, int n, int seg,
                                               const double *__restrict__ QR,
                                               const double *__restrict__ invd,
                                               double *__restrict__ W) {
  const long E = long(N) * n;
  const long EW = long(n) * N;
  const int lane = lane_id();
  const int lis = lane & (seg - 1);
  mdc<M> g[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int i = lis + q * seg;
    g[q] = (live && i < n) ? cload<M>(W, EW, long(i) * N + c) : c_zero<M>();
  }
  for (int i = n - 1; i >= 0; --i) {
    const int owner = i & (seg - 1), ro = i / seg;
    mdc<M> xi = c_zero<M>();
#pragma unroll
    for (int q = 0; q < RPL; ++q)
      if (live && q == ro && lis == owner) xi = c_mul<M>(g[q], cload<M>(invd, n, i));
    xi = shfl_c<M>(xi, (lane & ~(seg - 1)) + owner);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int l = lis + q * seg;
      if (!live) continue;
      if (l == i) g[q] = xi;
      else if (l < i) g[q] = c_sub<M>(g[q], c_mul<M>(cload<M>(QR, E, long(l) * n + i), xi));
    }
  }
  if (live) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = lis + q * seg;
      if (i < n) cstore<M>(W, EW, long(i) * N + c, g[q]);
    }
  }
}

// x = R^{-1} (Q^H b)_{0:n} for one right-hand side b (N entries) by one
// segment (lanes own rows lis, lis+seg, ...), the n reflectors are
// applied in order, then the back substitution with the row owner
// multiplying by 1/R_ii and broadcasting.  x: n entries (plane stride n).
// `live` false: the segment only joins the shuffles.
template <int M, int RPL>
__device__ __forceinline__ void qr_solve_vector(bool live, int N, int n, int seg,
                                                const double *__restrict__ QR,
                                                const double *__restrict__ vdiag,
                                                const double *__restrict__ beta,
                                                const double *__restrict__ invd,
                                                const double *__restrict__ b,
                                                double *__restrict__ x) {
  const long E = long(N) * n;
  const int lane = lane_id();
  const int lis = lane & (seg - 1);
  mdc<M> g[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lis + r * seg;
    g[r] = (live && i < N) ? cload<M>(b, N, i) : c_zero<M>();
  }
  for (int j = 0; j < n; ++j) {
    const mdc<M> v0 = cload<M>(vdiag, n, j);
    const mdr<M> bet = rload<M>(beta, n, j);
    mdc<M> vi[RPL];
    mdc<M> w = c_zero<M>();
    bool first = true;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lis + r * seg;
      vi[r] = c_zero<M>();
      if (live && i >= j && i < N) {
        vi[r] = i == j ? v0 : cload<M>(QR, E, long(i) * n + j);
        const mdc<M> t = c_mul<M>(c_conj<M>(vi[r]), g[r]);
        w = first ? t : c_add<M>(w, t);
        first = false;
      }
    }
    w = seg_reduce_c<M>(w, seg);
    w = shfl_c<M>(w, lane & ~(seg - 1));
    const mdc<M> bw = c_mulr<M>(w, bet);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lis + r * seg;
      if (live && i >= j && i < N) g[r] = c_sub<M>(g[r], c_mul<M>(bw, vi[r]));
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    const int owner = i & (seg - 1), ro = i / seg;
    mdc<M> xi = c_zero<M>();
#pragma unroll
    for (int r = 0; r < RPL; ++r)
      if (live && r == ro && lis == owner) xi = c_mul<M>(g[r], cload<M>(invd, n, i));
    xi = shfl_c<M>(xi, (lane & ~(seg - 1)) + owner);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int l = lis + r * seg;
      if (!live) continue;
      if (l == i) g[r] = xi;
      else if (l < i) g[r] = c_sub<M>(g[r], c_mul<M>(cload<M>(QR, E, long(l) * n + i), xi));
    }
  }
  if (live) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lis + r * seg;
      if (i < n) cstore<M>(x, n, i, g[r]);
    }
  }
}

// Lanes per dot product of the staggered stages (length len).  The
// single-path kernels take one product per lane (shortest chain); the
// batched kernel, where a workgroup has many rows to do, lets each lane sum
// up to eight products in sequence before the segment tree (fewest
// instructions per row).  Each choice fixes the order of the sums.
__host__ __device__ inline int dot_seg_latency(int len) {
  const int s = pow2_at_least(len);
  return s > WAVE ? WAVE : s;
}
__host__ __device__ inline int dot_seg_throughput(int len) {
  const int s = pow2_at_least((len + 7) / 8);
  return s > WAVE ? WAVE : s;
}

// dx_k[i] = sum_c W[i][c] r_k[c] by one segment
template <int M>
__device__ __forceinline__ void stage_dx_row(bool live, int i, int k, int N, int n, int d, int seg,
                             const double *__restrict__ W, const double *__restrict__ r,
                             double *__restrict__ dx, int &st, double *dxl = nullptr) {
  const long EW = long(n) * N, Er = long(d + 1) * N, Ex = long(d + 1) * n;
  const int lis = lane_id() & (seg - 1);
  mdc<M> s = c_zero<M>();
  bool first = true;
  if (live)
    for (int c = lis; c < N; c += seg) {
      const mdc<M> t = c_mul<M>(cload<M>(W, EW, long(i) * N + c), cload<M>(r, Er, long(k) * N + c));
      s = first ? t : c_add<M>(s, t);
      first = false;
    }
  s = seg_reduce_c<M>(s, seg);
  if (live && lis == 0) {
    cstore<M>(dx, Ex, long(k) * n + i, s);
    if (dxl) cstore<M>(dxl, n, i, s);  // a copy of dx_k as planes (2, M, n), in LDS
    if (!c_finite<M>(s)) st |= MD_ST_NONFINITE;
  }
}

// r_{k+j}[i] -= sum_l A_j[i][l] dx_k[l] by one segment; row = (j-1)*N + i
template <int M>
__device__ __forceinline__ void stage_update_row(bool live, long row, int k, int N, int n, int d, int seg,
                                 const double *__restrict__ A, const double *__restrict__ dx,
                                 double *__restrict__ r) {
  const long EA = long(d + 1) * N * n, Er = long(d + 1) * N, Ex = long(d + 1) * n;
  const int lis = lane_id() & (seg - 1);
  const int j = int(row / N) + 1;
  const int i = int(row - long(j - 1) * N);
  mdc<M> s = c_zero<M>();
  bool first = true;
  if (live)
    for (int l = lis; l < n; l += seg) {
      const mdc<M> t = c_mul<M>(cload<M>(A, EA, (long(j) * N + i) * n + l),
                                cload<M>(dx, Ex, long(k) * n + l));
      s = first ? t : c_add<M>(s, t);
      first = false;
    }
  s = seg_reduce_c<M>(s, seg);
  if (live && lis == 0) {
    const long e = long(k + j) * N + i;
    cstore<M>(r, Er, e, c_sub<M>(cload<M>(r, Er, e), s));
  }
}

// The same update with dx_k read from a copy in LDS (planes (2, M, n)).
template <int M>
__device__ __forceinline__ void stage_update_row_lds(bool live, long row, int k, int N, int n,
                                                     int d, int seg, const double *__restrict__ A,
                                                     const double *dxl, double *__restrict__ r) {
  const long EA = long(d + 1) * N * n, Er = long(d + 1) * N;
  const int lis = lane_id() & (seg - 1);
  const int j = int(row / N) + 1;
  const int i = int(row - long(j - 1) * N);
  mdc<M> s = c_zero<M>();
  bool first = true;
  if (live)
    for (int l = lis; l < n; l += seg) {
      const mdc<M> a = cload<M>(A, EA, (long(j) * N + i) * n + l), x = cload<M>(dxl, n, l);
      s = first ? c_mul<M>(a, x) : c_fmadd<M>(s, a, x);
      first = false;
    }
  s = seg_reduce_c<M>(s, seg);
  if (live && lis == 0) {
    const long e = long(k + j) * N + i;
    cstore<M>(r, Er, e, c_sub<M>(cload<M>(r, Er, e), s));
  }
}

// The same update with this lane's entries of dx_k already in registers
// (dxr[t] = dx_k[lis + t*seg], t < NE; seg * NE >= n): the same products
// and sums as stage_update_row, without reading dx_k again for every row.
template <int M, int NE>
__device__ __forceinline__ void stage_update_row_reg(bool live, long row, int k, int N, int n,
                                                     int d, int seg, const double *__restrict__ A,
                                                     const mdc<M> (&dxr)[NE],
                                                     double *__restrict__ r) {
  const long EA = long(d + 1) * N * n, Er = long(d + 1) * N;
  const int lis = lane_id() & (seg - 1);
  const int j = int(row / N) + 1;
  const int i = int(row - long(j - 1) * N);
  mdc<M> s = c_zero<M>();
  bool first = true;
#pragma unroll
  for (int t = 0; t < NE; ++t) {
    const int l = lis + t * seg;
    if (live && l < n) {
      const mdc<M> p = c_mul<M>(cload<M>(A, EA, (long(j) * N + i) * n + l), dxr[t]);
      s = first ? p : c_add<M>(s, p);
      first = false;
    }
  }
  s = seg_reduce_c<M>(s, seg);
  if (live && lis == 0) {
    const long e = long(k + j) * N + i;
    cstore<M>(r, Er, e, c_sub<M>(cload<M>(r, Er, e), s));
  }
}

// ---------------------------------------------------------------------------
// evaluation and differentiation

struct EvalArgs {
  int d, N, n, Mt, dc, Dmax, S;
  const int *eq_ptr, *term_ptr, *factors;
  const double *coef, *x;
  double *ws;
  long Ews;
  double *f, *A;
  EvalLayout lay;
  double *mono = nullptr;  // when set: the monomial series x^a of each term, planes (2, m, Mt, d+1)
  const int32_t *gate = nullptr;  // when set and *gate == 0, the kernels return at once
};


// LDS series of one term of degree D <= Dmax: its factor series
// x_0..x_{D-1}, its coefficient series, the forward products P_2..P_D,
// backward Q_2..Q_{D-1} and cross C_2..C_{D-1}.  In the compact layout
// (from Dmax = 3 on; the one-path evaluation, where LDS decides how many
// terms a CU holds) slots are shared where the lifetimes allow: C_j takes the slot of x_{j-1} (x_1 ..
// x_{D-2} are last read by the backward products, which end before the
// first cross product, and no cross product reads them), and the
// coefficient series takes slot D when D <= 2 (loaded first) or the slot of
// x_0 when D >= 3 (loaded after the cross products, the last readers of
// x_0): 3 Dmax - 3 series instead of 4 Dmax - 4.
struct TermLds {
  int Dmax;
  bool cmp;  // the compact layout (only with Dmax >= 3)
  __device__ bool compact() const { return cmp; }
  __device__ int xs(int q) const { return q; }
  __device__ int cs(int D) const { return compact() ? (D <= 2 ? D : 0) : Dmax; }
  __device__ bool cs_late(int D) const { return compact() && D >= 3; }
  __device__ int P(int j) const { return (compact() ? Dmax : Dmax + 1) + (j - 2); }
  __device__ int Q(int j) const { return (compact() ? 2 * Dmax - 1 : 2 * Dmax) + (j - 2); }
  __device__ int C(int j) const { return compact() ? j - 1 : 3 * Dmax - 2 + (j - 2); }
};

__host__ __device__ inline int term_lds_series(int Dmax, bool compact = false) {
  return Dmax < 2 ? Dmax + 1 : ((compact && Dmax >= 3) ? 3 * Dmax - 3 : 4 * Dmax - 4);
}

// lane r-group width for degree d: the largest power of two r with
// ceil((d+1)/2) * r <= 64
__host__ __device__ inline int eval_group(int d) {
  const int P = (d + 2) / 2;
  const int r = WAVE / P;
  return r < 1 ? 1 : r;
}

// Sum over the r lanes of a group (r need not be a power of two; sub is the
// lane's index in its group): s_sub += s_{sub+o} for o = p/2, ..., 1 with p
// the power of two at least r, where sub < o and sub + o < r.  The group's
// first lane holds the sum; the order is fixed.  For a power of two r this
// is seg_reduce_c's order.
template <int M>
__device__ __forceinline__ mdc<M> group_reduce_c(mdc<M> s, int r, int sub) {
  for (int o = pow2_at_least(r) >> 1; o > 0; o >>= 1) {
    const mdc<M> t = shfl_down_c<M>(s, o);
    if (sub < o && sub + o < r) s = c_add<M>(s, t);
  }
  return s;
}

template <int M>
__device__ __forceinline__ mdc<M> conv_part(const mdc<M> *X, int dx, const mdc<M> *Y, int k,
                                            int sub, int r) {
  const int top = k < dx ? k : dx;
  mdc<M> acc = c_zero<M>();
  bool first = true;
  for (int i = sub; i <= top; i += r) {
    if (first) {
      acc = c_mul<M>(X[i], Y[k - i]);
    } else if constexpr (M <= 4) {
      acc = c_fmadd<M>(acc, X[i], Y[k - i]);
    } else {
      // five limbs and more: the two operations (the fused form makes the
      // shared series-product routine of those kernels too long for its
      // short branches)
      acc = c_add<M>(acc, c_mul<M>(X[i], Y[k - i]));
    }
    first = false;
  }
  return acc;
}

// z = X Y (deg X <= dx) truncated at d for the coefficient pairs (k, d-k)
// of this lane's group, by the `nb` lanes of a block (`bl` is the lane's
// index in it); the group's partial sums go through a fixed-order tree;
// results (times `mult`) to LDS Z or to workspace planes.  When X has fewer
// coefficients than a group has lanes, each lane takes whole coefficients
// instead.  All lanes of the wave call this (the trees shuffle across it).
template <int M>
__device__ __forceinline__ void conv_block(int bl, int nb, const mdc<M> *X, int dx, const mdc<M> *Y,
                                           mdc<M> *Z, int d, int r, double *ws, long Ews,
                                           long wbase, int mult) {
  if (dx < r && dx < d) {
    // a short X (a coefficient series, deg X < d): one coefficient per
    // lane, its few products added in sequence.  (A full product of a short
    // series, d < r, still goes through the lane groups: one coefficient
    // per lane would make its last lane add d + 1 products in sequence.)
    for (int k = bl; k <= d; k += nb) {
      mdc<M> z = conv_part<M>(X, dx, Y, k, 0, 1);
      if (mult > 1) {
        z.re = md_muld<M>(z.re, double(mult));
        z.im = md_muld<M>(z.im, double(mult));
      }
      if (Z) Z[k] = z;
      else cstore<M>(ws, Ews, wbase + k, z);
    }
    return;
  }
  const int pg = bl / r;
  const int sub = bl - pg * r;
  const int npg = nb / r;
  const int P = (d + 2) / 2;
  for (int base = 0; base < P; base += npg) {
    const int p = base + pg;
    const bool live = p < P && pg < npg;
#pragma unroll 1
    for (int q = 0; q < 2; ++q) {
      const int k = live ? (q == 0 ? p : d - p) : 0;
      mdc<M> z = live ? conv_part<M>(X, dx, Y, k, sub, r) : c_zero<M>();
      z = group_reduce_c<M>(z, r, sub);
      if (live && sub == 0 && (q == 0 || k != p)) {
        if (mult > 1) {
          z.re = md_muld<M>(z.re, double(mult));
          z.im = md_muld<M>(z.im, double(mult));
        }
        if (Z) Z[k] = z;
        else cstore<M>(ws, Ews, wbase + k, z);
      }
    }
  }
}

// conv_block as one shared function for five or more limbs: a copy inlined
// at every call site makes those kernels very large (and slow to compile)
// for no measured gain.  A leaf without LDS variables of its own.
template <int M>
__device__ __noinline__ void conv_block_call(int bl, int nb, const mdc<M> *X, int dx,
                                             const mdc<M> *Y, mdc<M> *Z, int d, int r, double *ws,
                                             long Ews, long wbase, int mult) {
  conv_block<M>(bl, nb, X, dx, Y, Z, d, r, ws, Ews, wbase, mult);
}

template <int M>
__device__ __forceinline__ void conv_any(int bl, int nb, const mdc<M> *X, int dx, const mdc<M> *Y,
                                         mdc<M> *Z, int d, int r, double *ws, long Ews, long wbase,
                                         int mult) {
  if constexpr (M >= 5) conv_block_call<M>(bl, nb, X, dx, Y, Z, d, r, ws, Ews, wbase, mult);
  else conv_block<M>(bl, nb, X, dx, Y, Z, d, r, ws, Ews, wbase, mult);
}

// One series product by the whole wave (groups of r lanes per pair).
template <int M>
__device__ __forceinline__ void conv_group(const mdc<M> *X, int dx, const mdc<M> *Y, mdc<M> *Z,
                                           int d, int r, double *ws, long Ews, long wbase,
                                           int mult) {
  conv_any<M>(lane_id(), WAVE, X, dx, Y, Z, d, r, ws, Ews, wbase, mult);
}

// Lanes per coefficient pair when two full products share the wave (32
// lanes each), or 0 when they should go one after the other: pairing pays
// while each pair still gets two lanes of the half wave (d <= 31).
__host__ __device__ inline int eval_group2(int d) {
  const int P = (d + 2) / 2;
  return 2 * P <= WAVE / 2 ? (WAVE / 2) / P : 0;
}

// Two independent full products (deg X = d) into LDS: the first by lanes
// 0..31, the second by lanes 32..63, r2 = eval_group2(d) lanes per pair; or
// one after the other when r2 is 0, and always for five or more limbs.
template <int M>
__device__ __forceinline__ void conv_pair(const mdc<M> *X0, const mdc<M> *Y0, mdc<M> *Z0,
                                          const mdc<M> *X1, const mdc<M> *Y1, mdc<M> *Z1, int d,
                                          int r, int r2) {
  if (M >= 5 || r2 == 0) {
    conv_any<M>(lane_id(), WAVE, X0, d, Y0, Z0, d, r, nullptr, 0, 0, 1);
    conv_any<M>(lane_id(), WAVE, X1, d, Y1, Z1, d, r, nullptr, 0, 0, 1);
    return;
  }
  if constexpr (M < 5) {
    const int lane = lane_id();
    const bool hi = lane >= WAVE / 2;
    conv_block<M>(lane & (WAVE / 2 - 1), WAVE / 2, hi ? X1 : X0, d, hi ? Y1 : Y0, hi ? Z1 : Z0,
                  d, r2, nullptr, 0, 0, 1);
  }
}

// One term by one wave with its series in `lds` (term_lds_series(Dmax) x
// (d+1) complex numbers): forward and backward products one factor per step,
// cross products at first positions, then c(t) times the value and the
// derivatives into the term's workspace slots.  The wave's lanes must all
// call this; `wave_sync` orders LDS between steps.  COMPACT: the compact
// LDS layout of TermLds (sized by term_lds_series(Dmax, true)).
template <int M, bool COMPACT = false, class Sync>
__device__ __forceinline__ void eval_term_wave(const EvalArgs &a, int tau, int r, mdc<M> *lds, Sync wave_sync) {
  const int d = a.d, L = d + 1;
  const TermLds T{a.Dmax, COMPACT && a.Dmax >= 3};
  const int lane = lane_id();
  const int D = a.term_ptr[tau + 1] - a.term_ptr[tau];
  if (D > a.Dmax) return;  // the host validates max_deg
  const int *v = a.factors + a.term_ptr[tau];
  auto S = [&](int slot) { return lds + slot * L; };
  const long Ex = long(L) * a.n;
  for (int e = lane; e < D * L; e += WAVE) {
    const int q = e / L, k = e - q * L;
    S(T.xs(q))[k] = cload<M>(a.x, Ex, long(k) * a.n + v[q]);
  }
  auto load_cs = [&]() __attribute__((always_inline)) {
    for (int k = lane; k < L; k += WAVE)
      S(T.cs(D))[k] = (k <= a.dc)
                          ? cload<M>(a.coef, long(a.Mt) * (a.dc + 1), long(tau) * (a.dc + 1) + k)
                          : c_zero<M>();
  };
  if (!T.cs_late(D)) load_cs();
  wave_sync();
  const int dcu = a.dc < d ? a.dc : d;
  const long wb = long(tau) * a.S * L;
  const long Em = long(a.Mt) * L;
  if (a.mono && D <= 1)
    for (int k = lane; k < L; k += WAVE) {
      mdc<M> z = c_zero<M>();
      if (D == 1) z = S(T.xs(0))[k];
      else if (k == 0) z.re = md_from<M>(1.0);
      cstore<M>(a.mono, Em, long(tau) * L + k, z);
    }
  if (D == 0) {
    for (int k = lane; k < L; k += WAVE)
      cstore<M>(a.ws, a.Ews, wb + a.lay.val() * L + k, S(T.cs(D))[k]);
    return;
  }
  auto Pj = [&](int j) { return j == 1 ? S(T.xs(0)) : S(T.P(j)); };
  auto Qj = [&](int j) { return j == D ? S(T.xs(D - 1)) : S(T.Q(j)); };
  // c(t) times the value (slot 0) and the derivatives (slot j: the cross
  // product of the j-th factor's first occurrence times its multiplicity).
  // With a short coefficient series (dcu < r) every lane takes whole
  // (slot, coefficient) pairs of all slots at once, each sum in the order
  // of conv_part; otherwise the slots go one by one through the lane groups.
  auto coef_products = [&]() __attribute__((always_inline)) {
    if (dcu < r) {
      for (int e = lane; e < (D + 1) * L; e += WAVE) {
        const int j = e / L, k = e - j * L;
        if (j > 1 && v[j - 1] == v[j - 2]) continue;
        mdc<M> z;
        if (D == 1 && j == 1) {
          z = S(T.cs(D))[k];  // d(c x)/dx = c
        } else {
          const mdc<M> *Y = j == 0 ? Pj(D) : (j == 1 ? Qj(2) : (j == D ? Pj(D - 1) : S(T.C(j))));
          z = conv_part<M>(S(T.cs(D)), dcu, Y, k, 0, 1);
          int mult = 1;
          if (j > 0) {
            mult = 0;
            for (int q = 0; q < D; ++q) mult += (v[q] == v[j - 1]);
          }
          if (mult > 1) {
            z.re = md_muld<M>(z.re, double(mult));
            z.im = md_muld<M>(z.im, double(mult));
          }
        }
        cstore<M>(a.ws, a.Ews, wb + (j == 0 ? a.lay.val() : a.lay.der(j)) * L + k, z);
      }
      return;
    }
    conv_group<M>(S(T.cs(D)), dcu, Pj(D), nullptr, d, r, a.ws, a.Ews, wb + a.lay.val() * L, 1);
    if (D == 1) {
      for (int k = lane; k < L; k += WAVE)
        cstore<M>(a.ws, a.Ews, wb + a.lay.der(1) * L + k, S(T.cs(D))[k]);
      return;
    }
    for (int j = 1; j <= D; ++j) {
      if (j > 1 && v[j - 1] == v[j - 2]) continue;
      int mult = 0;
      for (int q = 0; q < D; ++q) mult += (v[q] == v[j - 1]);
      const mdc<M> *cross = (j == 1) ? Qj(2) : (j == D ? Pj(D - 1) : S(T.C(j)));
      conv_group<M>(S(T.cs(D)), dcu, cross, nullptr, d, r, a.ws, a.Ews, wb + a.lay.der(j) * L, mult);
    }
  };
  if (D == 1) {
    coef_products();
    return;
  }
  // forward P_{st+1} = P_st x_st and backward Q_j = x_{j-1} Q_{j+1} side by
  // side; the last forward product goes with the first cross product
  // C_j = P_{j-1} Q_{j+1} (all of whose inputs are ready by then), and the
  // other cross products go two by two
  const int r2 = eval_group2(d);
  auto cross_next = [&](int j) {
    while (j <= D - 1 && v[j - 1] == v[j - 2]) ++j;
    return j;
  };
  int jc = cross_next(2);
  for (int st = 1; st <= D - 1; ++st) {
    const int j = D - st;
    if (j >= 2) {
      conv_pair<M>(Pj(st), S(T.xs(st)), S(T.P(st + 1)), S(T.xs(j - 1)), Qj(j + 1), S(T.Q(j)), d, r, r2);
    } else if (jc <= D - 1) {
      conv_pair<M>(Pj(st), S(T.xs(st)), S(T.P(st + 1)), Pj(jc - 1), Qj(jc + 1), S(T.C(jc)), d, r, r2);
      jc = cross_next(jc + 1);
    } else {
      conv_group<M>(Pj(st), d, S(T.xs(st)), S(T.P(st + 1)), d, r, nullptr, 0, 0, 1);
    }
    wave_sync();
  }
  while (jc <= D - 1) {
    const int jn = cross_next(jc + 1);
    if (jn <= D - 1) {
      conv_pair<M>(Pj(jc - 1), Qj(jc + 1), S(T.C(jc)), Pj(jn - 1), Qj(jn + 1), S(T.C(jn)), d, r, r2);
      jc = cross_next(jn + 1);
    } else {
      conv_group<M>(Pj(jc - 1), d, Qj(jc + 1), S(T.C(jc)), d, r, nullptr, 0, 0, 1);
      jc = jn;
    }
  }
  if (a.mono)
    for (int k = lane; k < L; k += WAVE) cstore<M>(a.mono, Em, long(tau) * L + k, Pj(D)[k]);
  wave_sync();
  if (T.cs_late(D)) {
    load_cs();
    wave_sync();
  }
  coef_products();
}

// f_i[k] (g's l == n) or A_{i,l}[k], one element per call (g over
// (k, i, l)): the term slots of equation i that touch it, added in term
// order from zero.  The same sums as eval_accumulate_row, spread over more
// threads for the single-path kernel.
template <int M>
__device__ __forceinline__ void eval_accumulate_elem(const EvalArgs &a, long g) {
  const int L = a.d + 1;
  const long per_k = long(a.N) * (a.n + 1);
  const int k = int(g / per_k);
  const long rr = g - k * per_k;
  const int i = int(rr / (a.n + 1));
  const int l = int(rr - long(i) * (a.n + 1));
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
    if (slot >= 0) acc = c_add<M>(acc, cload<M>(a.ws, a.Ews, (long(tau) * a.S + slot) * L + k));
  }
  if (l == a.n) cstore<M>(a.f, long(L) * a.N, long(k) * a.N + i, acc);
  else cstore<M>(a.A, long(L) * a.N * a.n, (long(k) * a.N + i) * a.n + l, acc);
}

// Coefficient k of f_i and of row i of A: zero, then the terms of equation
// i added in term order, the value slot into f_i and, for every distinct
// factor l of a term, its derivative slot (first occurrence of l) into
// A_{i,l}.  Each sum starts from zero and adds in term order, as the
// definition reads; entries no term touches stay zero.  `zeroed`: the row
// was cleared already.
template <int M>
__device__ __forceinline__ void eval_accumulate_row(const EvalArgs &a, int i, int k, bool zeroed = false) {
  const int L = a.d + 1;
  const long EA = long(L) * a.N * a.n;
  const long rowA = (long(k) * a.N + i) * a.n;
  if (!zeroed)
    for (int l = 0; l < a.n; ++l) cstore<M>(a.A, EA, rowA + l, c_zero<M>());
  mdc<M> acc = c_zero<M>();
  for (int tau = a.eq_ptr[i]; tau < a.eq_ptr[i + 1]; ++tau) {
    const long wb = long(tau) * a.S * L + k;
    acc = c_add<M>(acc, cload<M>(a.ws, a.Ews, wb + long(a.lay.val()) * L));
    const int b = a.term_ptr[tau], e = a.term_ptr[tau + 1];
    if (e - b > a.Dmax) continue;
    for (int q = b; q < e; ++q) {
      if (q > b && a.factors[q] == a.factors[q - 1]) continue;
      const long el = rowA + a.factors[q];
      cstore<M>(a.A, EA, el,
                c_add<M>(cload<M>(a.A, EA, el),
                         cload<M>(a.ws, a.Ews, wb + long(a.lay.der(q - b + 1)) * L)));
    }
  }
  cstore<M>(a.f, long(L) * a.N, long(k) * a.N + i, acc);
}

// Rows g0 .. g0+63 of the Jacobian sums by one wave, row g being
// coefficient k = g mod (d+1) of equation i = g / (d+1) (consecutive lanes
// take consecutive coefficients of one equation, so their reads of a term's
// slots are consecutive words): the wave clears the rows' A entries
// together (lanes over the entries of a row), then each lane forms its row
// as eval_accumulate_row and writes r_k[i] = -f_k[i].  All lanes of the wave
// call this.
template <int M, class Sync>
__device__ __forceinline__ void eval_accumulate_wave(const EvalArgs &a, long g0, double *__restrict__ r,
                                                     Sync wave_sync) {
  const int L = a.d + 1;
  const long rows = long(L) * a.N;
  const long EA = rows * a.n, Er = rows;
  const int lane = lane_id();
  const long cnt = rows - g0 < WAVE ? rows - g0 : WAVE;
  for (long e = lane; e < cnt * a.n; e += WAVE) {
    const long g = g0 + e / a.n;
    const int l = int(e - (g - g0) * a.n);
    const int i = int(g / L), k = int(g - long(i) * L);
    cstore<M>(a.A, EA, (long(k) * a.N + i) * a.n + l, c_zero<M>());
  }
  wave_sync();
  const long g = g0 + lane;
  if (g < rows) {
    const int i = int(g / L), k = int(g - long(i) * L);
    eval_accumulate_row<M>(a, i, k, true);
    const long e = long(k) * a.N + i;
    cstore<M>(r, Er, e, c_neg<M>(cload<M>(a.f, Er, e)));
  }
}

// ---------------------------------------------------------------------------
// adjoint pieces

// The monomial series x^a of term tau into LDS by forward products (one
// wave); returns the slot holding it.  Slots: factor series 0..D-1, then the
// products P_2..P_D.
template <int M, class Sync>
__device__ __forceinline__ const mdc<M> *monomial_wave(const EvalArgs &a, int tau, int r,
                                                       mdc<M> *lds, Sync wave_sync) {
  const int d = a.d, L = d + 1;
  const int lane = lane_id();
  const int D = a.term_ptr[tau + 1] - a.term_ptr[tau];
  const int *v = a.factors + a.term_ptr[tau];
  auto S = [&](int slot) { return lds + slot * L; };
  const long Ex = long(L) * a.n;
  if (D == 0) {
    for (int k = lane; k < L; k += WAVE) {
      mdc<M> z = c_zero<M>();
      if (k == 0) z.re = md_from<M>(1.0);
      S(0)[k] = z;
    }
    wave_sync();
    return S(0);
  }
  for (int e = lane; e < D * L; e += WAVE) {
    const int q = e / L, k = e - q * L;
    S(q)[k] = cload<M>(a.x, Ex, long(k) * a.n + v[q]);
  }
  wave_sync();
  for (int st = 1; st <= D - 1; ++st) {
    const mdc<M> *prev = st == 1 ? S(0) : S(D + st - 2);
    conv_group<M>(prev, d, S(st), S(D + st - 1), d, r, nullptr, 0, 0, 1);
    wave_sync();
  }
  return D == 1 ? S(0) : S(2 * D - 2);
}

// grad c_{tau,j} = -sum_{k=j}^{d} conj(mono_{k-j}) lambda_{k,i}, j = 0..dc,
// by one wave (lanes over k, fixed-order wave sum); the first two limbs are
// stored (planes (2, 2, Mt, dc+1)).
template <int M>
__device__ __forceinline__ void contract_wave(const mdc<M> *mono, long mstride, const double *mono_g,
                                              long Em, long mbase, const double *lam, int N, int i,
                                              int d, int dc, int tau, int Mt, double *grad) {
  const int lane = lane_id();
  const long El = long(d + 1) * N;
  const long Eg = long(Mt) * (dc + 1);
  for (int j = 0; j <= dc; ++j) {
    mdc<M> s = c_zero<M>();
    bool first = true;
    for (int k = j + lane; k <= d; k += WAVE) {
      const mdc<M> mk = mono ? mono[(k - j) * mstride] : cload<M>(mono_g, Em, mbase + (k - j));
      const mdc<M> t = c_mul<M>(c_conj<M>(mk), cload<M>(lam, El, long(k) * N + i));
      s = first ? t : c_add<M>(s, t);
      first = false;
    }
    s = seg_reduce_c<M>(s, WAVE);
    if (lane == 0) {
      const long e = long(tau) * (dc + 1) + j;
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        grad[l * Eg + e] = l < M ? -s.re.v[l] : 0.0;
        grad[(2 + l) * Eg + e] = l < M ? -s.im.v[l] : 0.0;
      }
    }
  }
}

}  // namespace mds
