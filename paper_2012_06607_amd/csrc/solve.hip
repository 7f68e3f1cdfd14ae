// Staggered solve of A(t) dx(t) = b(t), the block lower triangular Toeplitz
// system of Section 4, by forward substitution over the degrees.
//
// Every stage solves A_0 dx_k = r_k with the same QR factors.  Applying Q^H
// (n reflectors in sequence) and then back substitution with R is a chain
// of about 2n dependent steps; here W = R^{-1} (Q^H)_{0:n} (n x N) is formed
// once, and every stage is then the product dx_k = W r_k (least squares in
// the first n rows when N > n).  W itself is formed from products with
// short dependent chains (below), not by running the 2n-step chain on the
// N columns of the identity.  After dx_k the later right hand sides are updated,
// r_{k+j} -= A_j dx_k for all j = 1..d-k at once (the paper's "one job per
// right hand side update", Section 5).
#include "dot4.hpp"
#include "internal.hpp"

namespace mds {

// r = b (or -b), planes (2, m, d+1, N)
template <int M>
__global__ void __launch_bounds__(256) k_copy_rhs(long E, const double *__restrict__ b, bool neg,
                                                  double *__restrict__ r, const int32_t *gate) {
  if (gate_closed(gate)) return;
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < E;
       e += long(gridDim.x) * blockDim.x) {
    mdc<M> z = cload<M>(b, E, e);
    if (neg) z = c_neg<M>(z);
    cstore<M>(r, E, e, z);
  }
}

// 1 / R_ii for i < n (one thread each), so that the back substitution
// multiplies instead of dividing.
template <int M>
__global__ void __launch_bounds__(64) k_inv_diag(int N, int n, const double *__restrict__ QR,
                                                 double *__restrict__ invd, int32_t *status,
                                                 const int32_t *gate) {
  if (gate_closed(gate)) return;
  int st = 0;
  inv_diag_range<M>(blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, N, n, QR,
                    invd, st);
  if (st && status) atomicOr(status, st);
}

// ---------------------------------------------------------------------------
// W = R^{-1} (Q^H)_{0:n} for one path, with short dependent chains.
//
// Q = H_0 H_1 ... H_{n-1} = I - V T V^H (the compact WY form) with V the
// reflector columns (v_j: head vdiag_j in row j, the tail below it in QR)
// and T upper triangular.  Appending H_k to I - V_k T_k V_k^H gives
// T_{k+1} = [T_k, -beta_k T_k V_k^H v_k; 0, beta_k], whose inverse is
// [T_k^{-1}, V_k^H v_k; 0, 1/beta_k]: so T^{-1} has 1/beta_j on the
// diagonal and v_a^H v_b above it (the identity of Joffrain, Low,
// Quintana-Orti, van de Geijn and Van Zee, 2006).  Then
//   (Q^H)_{0:n} = I_{0:n} - V_{0:n} T^H V^H   and   W = R^{-1} (Q^H)_{0:n}.
// T and R^{-1} come from triangular inversion by doubling blocks,
// inv [A B; 0 C] = [A^{-1}, -A^{-1} B C^{-1}; 0, C^{-1}], block size
// 1, 2, 4, ...  Every product is a set of independent dot products, one
// segment of lanes each (fixed tree order), so the longest chain of
// dependent md operations is about 2 log2(n) + 4 dot products instead of
// the 2n reflector and substitution steps of one identity column, at about
// three times the operations.
//
// Scratch (planes (2, m, *)): XT, XR (n x n: T and R^{-1}, inverted in
// place), PT, PR (n x n: B C^{-1} of the current block level), Z = T^H V^H
// and Y = (Q^H)_{0:n} (n x N).

template <int M>
__device__ __forceinline__ mdc<M> vcol(const double *__restrict__ QR,
                                       const double *__restrict__ vdiag, int N, int n, int i,
                                       int j) {
  if (i == j) return cload<M>(vdiag, n, j);
  if (i > j) return cload<M>(QR, long(N) * n, long(i) * n + j);
  return c_zero<M>();
}

// The segment's sum of term(j), j = lo .. hi-1, lanes over j (fixed tree
// order); every lane of the wave calls this, dead segments with lo >= hi.
template <int M, class F>
__device__ __forceinline__ mdc<M> seg_sum(int lo, int hi, int seg, F term) {
  const int lis = lane_id() & (seg - 1);
  mdc<M> s = c_zero<M>();
  bool first = true;
  for (int j = lo + lis; j < hi; j += seg) {
    const mdc<M> t = term(j);
    s = first ? t : c_add<M>(s, t);
    first = false;
  }
  return seg_reduce_c<M>(s, seg);
}

__device__ __forceinline__ long seg_index(int seg) {
  return (long(blockIdx.x) * blockDim.x + threadIdx.x) / seg;
}

// XT = T^{-1} before inversion (diagonal beta_j^{-1} inverted: beta_j; above
// it v_a^H v_b), XR = R (diagonal already inverted: 1/R_ii); the upper
// triangles only (a <= b), one segment each
template <int M>
__global__ void __launch_bounds__(256) k_pw_init(int N, int n, int seg,
                                                 const double *__restrict__ QR,
                                                 const double *__restrict__ vdiag,
                                                 const double *__restrict__ beta,
                                                 const double *__restrict__ invd,
                                                 double *__restrict__ XT, double *__restrict__ XR,
                                                 const int32_t *gate) {
  if (gate_closed(gate)) return;
  const long g = seg_index(seg);
  const long nn = long(n) * n;
  const bool live = g < nn;
  const int a = live ? int(g / n) : 0, b = live ? int(g - long(a) * n) : 0;
  const bool up = live && a < b;
  const mdc<M> sab = seg_sum<M>(up ? b : 0, up ? N : 0, seg, [&](int i) {
    return c_mul<M>(c_conj<M>(vcol<M>(QR, vdiag, N, n, i, a)), vcol<M>(QR, vdiag, N, n, i, b));
  });
  if (live && a <= b && (lane_id() & (seg - 1)) == 0) {
    mdc<M> t = sab, r;
    if (a == b) {
      t = c_zero<M>();
      t.re = rload<M>(beta, n, a);
      r = cload<M>(invd, n, a);
    } else {
      r = cload<M>(QR, long(N) * n, long(a) * n + b);
    }
    cstore<M>(XT, nn, long(a) * n + b, t);
    cstore<M>(XR, nn, long(a) * n + b, r);
  }
}

// One block level s of both inversions: pairs [r0, r0+s) (A, inverted) and
// [r0+s, min(r0+2s, n)) (C, inverted), r0 = 2 s p.  phase 0:
// P = B C^{-1} (B the block of X above C, still the original entries);
// phase 1: X's block above C = -A^{-1} P.  Element e of a matrix's level:
// pair e / s^2, row i = r0 + (e mod s^2) / s of A, column k = r0 + s + e mod s.
template <int M>
__global__ void __launch_bounds__(256) k_pw_level(int n, int s, int phase, int seg,
                                                  double *__restrict__ XT, double *__restrict__ XR,
                                                  double *__restrict__ PT, double *__restrict__ PR,
                                                  const int32_t *gate) {
  if (gate_closed(gate)) return;
  const long per = long((n + 2 * s - 1) / (2 * s)) * s * s;
  const long g = seg_index(seg);
  const int mat = int(g / per);
  const long e = g - long(mat) * per;
  const int p = int(e / (long(s) * s));
  const int r0 = 2 * s * p;
  const int i = r0 + int((e - long(p) * s * s) / s);
  const int k = r0 + s + int(e % s);
  const bool live = mat < 2 && k < n;
  double *X = mat == 0 ? XT : XR;
  double *P = mat == 0 ? PT : PR;
  const long nn = long(n) * n;
  mdc<M> v;
  if (phase == 0) {
    // P[i][k] = sum_{j = r0+s}^{k} X[i][j] X[j][k]
    v = seg_sum<M>(live ? r0 + s : 0, live ? k + 1 : 0, seg, [&](int j) {
      return c_mul<M>(cload<M>(X, nn, long(i) * n + j), cload<M>(X, nn, long(j) * n + k));
    });
  } else {
    // X[i][k] = -sum_{j = i}^{r0+s-1} X[i][j] P[j][k]
    v = seg_sum<M>(live ? i : 0, live ? r0 + s : 0, seg, [&](int j) {
      return c_mul<M>(cload<M>(X, nn, long(i) * n + j), cload<M>(P, nn, long(j) * n + k));
    });
    v = c_neg<M>(v);
  }
  if (live && (lane_id() & (seg - 1)) == 0) cstore<M>(phase == 0 ? P : X, nn, long(i) * n + k, v);
}

// Z[a][c] = (T^H V^H)[a][c] = sum_{b <= min(a, c)} conj(T[b][a]) conj(V[c][b])
template <int M>
__global__ void __launch_bounds__(256) k_pw_z(int N, int n, int seg,
                                              const double *__restrict__ QR,
                                              const double *__restrict__ vdiag,
                                              const double *__restrict__ XT,
                                              double *__restrict__ Z, const int32_t *gate) {
  if (gate_closed(gate)) return;
  const long g = seg_index(seg);
  const bool live = g < long(n) * N;
  const int a = live ? int(g / N) : 0, c = live ? int(g - long(a) * N) : 0;
  const int top = a < c ? a : c;
  const mdc<M> v = seg_sum<M>(0, live ? top + 1 : 0, seg, [&](int b) {
    return c_mul<M>(c_conj<M>(cload<M>(XT, long(n) * n, long(b) * n + a)),
                    c_conj<M>(vcol<M>(QR, vdiag, N, n, c, b)));
  });
  if (live && (lane_id() & (seg - 1)) == 0) cstore<M>(Z, long(n) * N, long(a) * N + c, v);
}

// Y[r][c] = (Q^H)_{0:n}[r][c] = delta_rc - sum_{a <= r} V[r][a] Z[a][c]
template <int M>
__global__ void __launch_bounds__(256) k_pw_y(int N, int n, int seg,
                                              const double *__restrict__ QR,
                                              const double *__restrict__ vdiag,
                                              const double *__restrict__ Z,
                                              double *__restrict__ Y, const int32_t *gate) {
  if (gate_closed(gate)) return;
  const long g = seg_index(seg);
  const bool live = g < long(n) * N;
  const int r = live ? int(g / N) : 0, c = live ? int(g - long(r) * N) : 0;
  const mdc<M> v = seg_sum<M>(0, live ? r + 1 : 0, seg, [&](int a) {
    return c_mul<M>(vcol<M>(QR, vdiag, N, n, r, a), cload<M>(Z, long(n) * N, long(a) * N + c));
  });
  if (live && (lane_id() & (seg - 1)) == 0) {
    mdc<M> y = c_neg<M>(v);
    if (r == c) {
      mdc<M> one = c_zero<M>();
      one.re = md_from<M>(1.0);
      y = c_sub<M>(one, v);
    }
    cstore<M>(Y, long(n) * N, long(r) * N + c, y);
  }
}

// W[r][c] = sum_{q >= r} Rinv[r][q] Y[q][c]
template <int M>
__global__ void __launch_bounds__(256) k_pw_w(int N, int n, int seg,
                                              const double *__restrict__ XR,
                                              const double *__restrict__ Y,
                                              double *__restrict__ W, const int32_t *gate) {
  if (gate_closed(gate)) return;
  const long g = seg_index(seg);
  const bool live = g < long(n) * N;
  const int r = live ? int(g / N) : 0, c = live ? int(g - long(r) * N) : 0;
  const mdc<M> v = seg_sum<M>(live ? r : 0, live ? n : 0, seg, [&](int q) {
    return c_mul<M>(cload<M>(XR, long(n) * n, long(r) * n + q),
                    cload<M>(Y, long(n) * N, long(q) * N + c));
  });
  if (live && (lane_id() & (seg - 1)) == 0) cstore<M>(W, long(n) * N, long(r) * N + c, v);
}

// dx_k = W r_k: one segment per output row
template <int M>
__global__ void __launch_bounds__(256) k_stage_dx(int k, int N, int n, int d, int seg,
                                                  const double *__restrict__ G,
                                                  const double *__restrict__ r,
                                                  double *__restrict__ dx, int32_t *status,
                                                  const int32_t *gate) {
  if (gate_closed(gate)) return;
  const int gwave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int i = gwave * (WAVE / seg) + lane_id() / seg;
  int st = 0;
  stage_dx_row<M>(i < n, i, k, N, n, d, seg, G, r, dx, st);
  if (st && status) atomicOr(status, st);
}

// dx_k = W r_k with each row's dot product on four waves (N <= 64, seg >=
// 8; dot4: one real product of each complex product a lane, the sum in
// seg_reduce's order), the bits of stage_dx_row.  The n
// dot products of a stage are too few to fill the chip one wave each, so
// four lanes a product shorten the stage's chain.
template <int M>
__global__ void __launch_bounds__(256) k_stage_dx4(int k, int N, int n, int d, int seg,
                                                   const double *__restrict__ G,
                                                   const double *__restrict__ r,
                                                   double *__restrict__ dx, int32_t *status,
                                                   const int32_t *gate) {
  __shared__ double xch[4 * M];
  if (gate_closed(gate)) return;
  const long EW = long(n) * N, Er = long(d + 1) * N, Ex = long(d + 1) * n;
  const int i = blockIdx.x;
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  const mdr<M> s = dot4<M, false>(N, seg, [&](int c, mdc<M> &x, mdc<M> &y) {
    x = cload<M>(G, EW, long(i) * N + c);
    y = cload<M>(r, Er, long(k) * N + c);
  }, xch);
  if (w == 0 && (lane == 0 || lane == 2)) {
    rstore<M>(dx + size_t(lane >> 1) * M * Ex, Ex, long(k) * n + i, s);
    if (!md_finite<M>(s) && status) atomicOr(status, MD_ST_NONFINITE);
  }
}

// r_{k+j} -= A_j dx_k with each row's dot product on four waves, as in
// k_stage_dx4 (n <= 64, seg >= 8; the bits are stage_update_row's): for
// the later stages, whose few rows leave most of the chip idle.
template <int M>
__global__ void __launch_bounds__(256) k_stage_update4(int k, int N, int n, int d, int seg,
                                                       const double *__restrict__ A,
                                                       const double *__restrict__ dx,
                                                       double *__restrict__ r,
                                                       const int32_t *gate) {
  __shared__ double xch[4 * M];
  if (gate_closed(gate)) return;
  const long EA = long(d + 1) * N * n, Er = long(d + 1) * N, Ex = long(d + 1) * n;
  const long row = blockIdx.x;
  const int j = int(row / N) + 1;
  const int i = int(row - long(j - 1) * N);
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  const mdr<M> s = dot4<M, false>(n, seg, [&](int c, mdc<M> &x, mdc<M> &y) {
    x = cload<M>(A, EA, (long(j) * N + i) * n + c);
    y = cload<M>(dx, Ex, long(k) * n + c);
  }, xch);
  if (w == 0 && (lane == 0 || lane == 2)) {
    const long e = long(k + j) * N + i;
    double *rp = r + size_t(lane >> 1) * M * Er;
    rstore<M>(rp, Er, e, md_add<M>(rload<M>(rp, Er, e), md_neg<M>(s)));
  }
}

// r_{k+j} -= A_j dx_k for j = 1..d-k: one segment per (j, row)
template <int M>
__global__ void __launch_bounds__(256) k_stage_update(int k, int N, int n, int d, int seg,
                                                      const double *__restrict__ A,
                                                      const double *__restrict__ dx,
                                                      double *__restrict__ r, const int32_t *gate) {
  if (gate_closed(gate)) return;
  const int gwave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const long row = long(gwave) * (WAVE / seg) + lane_id() / seg;
  stage_update_row<M>(row < long(d - k) * N, row, k, N, n, d, seg, A, dx, r);
}

int pinv_enqueue(int m, int N, int n, const double *QR, const double *vdiag, const double *beta,
                 double *invd, double *W, double *scratch, int32_t *status, hipStream_t s,
                 const int32_t *gate) {
  if (N > 256) return fail(MD_ESHAPE, "R^{-1} Q^H: N=%d above 256", N);
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const size_t nn = size_t(2) * Mm * n * n, nN = size_t(2) * Mm * n * N;
    double *XT = scratch, *XR = XT + nn, *PT = XR + nn, *PR = PT + nn, *Z = PR + nn, *Y = Z + nN;
    auto blocks = [](long segs, int seg) {
      return dim3(unsigned((segs * seg + 255) / 256));
    };
    k_inv_diag<Mm><<<dim3((n + 63) / 64), dim3(64), 0, s>>>(N, n, QR, invd, status, gate);
    {
      const int seg = dot_seg_latency(N);
      k_pw_init<Mm><<<blocks(long(n) * n, seg), dim3(256), 0, s>>>(N, n, seg, QR, vdiag, beta,
                                                                   invd, XT, XR, gate);
    }
    for (int bs = 1; bs < n; bs *= 2) {
      const long per = long((n + 2 * bs - 1) / (2 * bs)) * bs * bs;
      const int seg = dot_seg_latency(bs);
      for (int phase = 0; phase < 2; ++phase)
        k_pw_level<Mm><<<blocks(2 * per, seg), dim3(256), 0, s>>>(n, bs, phase, seg, XT, XR, PT,
                                                                  PR, gate);
    }
    const int seg = dot_seg_latency(n);
    k_pw_z<Mm><<<blocks(long(n) * N, seg), dim3(256), 0, s>>>(N, n, seg, QR, vdiag, XT, Z, gate);
    k_pw_y<Mm><<<blocks(long(n) * N, seg), dim3(256), 0, s>>>(N, n, seg, QR, vdiag, Z, Y, gate);
    k_pw_w<Mm><<<blocks(long(n) * N, seg), dim3(256), 0, s>>>(N, n, seg, XR, Y, W, gate);
    return check_launch("R^{-1} Q^H");
  });
}

int solve_enqueue(int m, int N, int n, int d, const double *QR, const double *vdiag,
                  const double *beta, const double *A, const double *b, bool negate_b,
                  double *dx, void *ws, size_t ws_bytes, int32_t *status, hipStream_t s,
                  const int32_t *gate) {
  if (d < 0) return fail(MD_EINVAL, "md_series_solve: d=%d < 0", d);
  if (n < 1 || N < n) return fail(MD_ESHAPE, "md_series_solve: need N >= n >= 1 (N=%d n=%d)", N, n);
  if (N > 256) return fail(MD_ESHAPE, "md_series_solve: N=%d above 256", N);
  if (!QR || !vdiag || !beta || !A || !b || !dx) return fail(MD_ENULL, "md_series_solve: null pointer");
  if (!valid_m(m)) return dispatch_m(m, [](auto) { return MD_OK; });
  SolveLayout lay(m, N, n, d);
  if (!ws || ws_bytes < lay.bytes || !aligned256(ws))
    return fail(MD_EWORKSPACE, "md_series_solve: workspace %zu bytes < %zu or misaligned",
                ws_bytes, lay.bytes);
  double *r = reinterpret_cast<double *>(static_cast<char *>(ws) + lay.off_r);
  double *G = reinterpret_cast<double *>(static_cast<char *>(ws) + lay.off_G);
  return dispatch_m(m, [&](auto Mc) {
    constexpr int Mm = decltype(Mc)::value;
    const long Er = long(d + 1) * N;
    long blocks = (Er + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_copy_rhs<Mm><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(Er, b, negate_b, r, gate);
    double *invd = G + size_t(2) * Mm * n * N;
    double *pw = reinterpret_cast<double *>(static_cast<char *>(ws) + lay.off_pw);
    int rc = pinv_enqueue(Mm, N, n, QR, vdiag, beta, invd, G, pw, status, s, gate);
    if (rc) return rc;
    const int seg_dx = dot_seg_latency(N);
    const int seg_up = dot_seg_latency(n);
    // four waves a dot product from three limbs on (a real md product a
    // quarter of a complex one or less), for the later updates while they
    // have at most two such rows a SIMD
    const bool dx4 = Mm >= 3 && N >= 5 && N <= WAVE;
    const bool up4 = Mm >= 3 && n >= 5 && n <= WAVE;
    for (int k = 0; k <= d; ++k) {
      if (dx4) {
        k_stage_dx4<Mm><<<dim3(unsigned(n)), dim3(256), 0, s>>>(k, N, n, d, seg_dx, G, r, dx,
                                                                status, gate);
      } else {
        const long waves = (long(n) * seg_dx + WAVE - 1) / WAVE;
        const long blk = (waves + 3) / 4;
        k_stage_dx<Mm><<<dim3(unsigned(blk)), dim3(256), 0, s>>>(k, N, n, d, seg_dx, G, r, dx,
                                                                  status, gate);
      }
      if (k < d && up4 && long(d - k) * N <= 512) {
        k_stage_update4<Mm><<<dim3(unsigned(long(d - k) * N)), dim3(256), 0, s>>>(
            k, N, n, d, seg_up, A, dx, r, gate);
      } else if (k < d) {
        const long rows = long(d - k) * N;
        const long waves = (rows * seg_up + WAVE - 1) / WAVE;
        const long blk = (waves + 3) / 4;
        k_stage_update<Mm><<<dim3(unsigned(blk)), dim3(256), 0, s>>>(k, N, n, d, seg_up, A, dx, r, gate);
      }
    }
    return check_launch("md_series_solve (stages)");
  });
}

}  // namespace mds

extern "C" int md_series_solve(int m, int N, int n, int d, const double *QR, const double *vdiag,
                               const double *beta, const double *A, const double *b, double *dx,
                               void *ws, size_t ws_bytes, int32_t *status, void *stream) {
  return mds::solve_enqueue(m, N, n, d, QR, vdiag, beta, A, b, false, dx, ws, ws_bytes, status,
                            (hipStream_t)stream);
}
