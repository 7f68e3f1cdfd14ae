// Several workgroups working on one path: a barrier over device memory and
// the Householder QR with its columns spread over the workgroups (the
// batched kernel's gangs, and the single-path QR of large systems).
#pragma once

#include "wg.hpp"

namespace mds {

// Gang barrier: every thread's memory operations complete, then member
// thread 0 releases at device scope (the workgroup's stores become visible
// to the other members), arrives on the counter and waits for all G
// arrivals of this round (bounded: a round that never completes sets
// MD_ST_GANG, and after that the workgroup waits no more), then acquires at
// device scope (stale cache lines dropped) before the workgroup goes on.
__device__ __forceinline__ void gang_barrier(int32_t *ctr, int G, int &round, int &st) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int target = (round + 1) * G;
    long spins = (st & MD_ST_GANG) ? (1L << 25) : 0;
    // polled with an atomic (performed where the arrivals are performed)
    while (__hip_atomic_fetch_add(ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins >= (1L << 25)) {
        st |= MD_ST_GANG;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  ++round;
}

// Householder QR of A_0 by all G workgroups of a gang: the columns of each
// step go over the slots of every member, the first wave of member 0
// updates column j+1 and forms reflector j+1 from it (as qr_wg's look-ahead
// does), and a gang barrier ends each step.  The reflector scalars are read
// back from vdiag and beta (written by member 0 before the barrier).  Each
// column is updated by one segment with the same code as in qr_wg, so the
// factors are those of qr_wg bit for bit.
template <int M, int RPL, class Sync>
__device__ __forceinline__ void qr_gang(QrShared<M> &sh, int N, int n, int seg,
                                        const double *__restrict__ A0, long A0E,
                                        double *__restrict__ QR, double *__restrict__ vdiag,
                                        double *__restrict__ beta, int &st, int member, int G,
                                        Sync gsync) {
  const long E = long(N) * n;
  const int lane = lane_id();
  const int wave = threadIdx.x / WAVE;
  const int nwaves = blockDim.x / WAVE;
  const int lis = lane & (seg - 1);
  const int spw = WAVE / seg;
  const int nslots = nwaves * spw;
  const int gs = member * nslots + wave * spw + lane / seg;  // global slot
  const int GS = G * nslots, others = GS - spw;
  const bool lead = member == 0 && wave == 0;
  for (long e = long(member) * blockDim.x + threadIdx.x; e < E; e += long(G) * blockDim.x)
    cstore<M>(QR, E, e, cload<M>(A0, A0E, e));
  gsync();
  for (int j = -1; j < n; ++j) {
    constexpr bool HOLD = RPL < 4 || M <= 2;
    mdc<M> vi[RPL], anew[RPL];
    mdc<M> v0 = c_zero<M>();
    mdr<M> bet = md_zero<M>();
    if (j >= 0) {
      v0 = cload<M>(vdiag, n, j);
      bet = rload<M>(beta, n, j);
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
    // round 0: global slot gs takes column j+1+gs; later rounds: the slots
    // outside the lead wave take the columns that are left
    const int ncols = n - j - 1;
    int rounds = 0;
    if (j < 0) {
      rounds = lead ? 1 : 0;
    } else if (ncols > 0) {
      const int rest = ncols - GS;
      rounds = lead ? 1 : 1 + (rest > 0 ? (rest + others - 1) / others : 0);
    }
    for (int k = 0; k < rounds; ++k) {
      const int l = k == 0 ? j + 1 + gs : j + 1 + GS + (k - 1) * others + (gs - spw);
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
      if (k == 0 && lead && j + 1 < n)
        qr_reflector<M, RPL, HOLD>(anew, j + 1, N, n, seg, true, sh, QR, E, vdiag, beta, st);
    }
    gsync();
  }
}

// ---------------------------------------------------------------------------
// The spread QR with its look-ahead column on four waves.  In qr_gang the
// chain of a column step is the look-ahead column's update and the next
// reflector on one wave (at octo double some 75 us of the 79 a step takes),
// while the other columns wait at the barrier.  Here member 0's first four
// waves take that column alone and the other members every other column:
// row i of the column lives on wave i mod 4, lanes 4 (i / 4) + q, q = 0..3,
// and lane q forms real product q of each complex product (re*re, im*im,
// re*im, im*re, as c_mul orders them), so a complex product takes one real
// product's time; the real part of a result then sits on lane q = 0 and
// the imaginary part on q = 2.  Sums over rows keep seg_reduce's order
// (row i adds row i + o, o = seg/2, ..., 1): for o >= 4 row i + o is lane
// + o of the same wave, the levels o = 2 and 1 pair waves through LDS.
// Every md operation is the one qr_update_column and qr_reflector apply to
// the same operands, so the factors are qr_wg's bit for bit.  Needs N <= 64
// (one row per lane of a segment), seg >= 8 and four waves in a workgroup.

// Sum over rows of a value held on lanes q = 0 and q = 2 (each its own sum)
// in seg_reduce's order; the sums end on wave 0, lanes 0 and 2.  Called by
// every thread of the workgroup (the barriers); `act`: the lane's wave is
// one of the four (wave-uniform).  xch: 4 M doubles of LDS.
template <int M>
__device__ __forceinline__ mdr<M> lead4_sum(mdr<M> s, int seg, int w, int lane, bool act,
                                            double *xch) {
  if (act) {
    for (int o = seg >> 1; o >= 4; o >>= 1) {
      const mdr<M> t = shfl_down_r<M>(s, o);
      if (lane < o) s = md_add<M>(s, t);
    }
  }
  const bool part = act && (lane == 0 || lane == 2);
  const int h = lane >> 1;
  if (part && w >= 2) {
#pragma unroll
    for (int k = 0; k < M; ++k) xch[((w - 2) * 2 + h) * M + k] = s.v[k];
  }
  __syncthreads();
  if (part && w < 2) {
    mdr<M> t;
#pragma unroll
    for (int k = 0; k < M; ++k) t.v[k] = xch[(w * 2 + h) * M + k];
    s = md_add<M>(s, t);
  }
  __syncthreads();
  if (part && w == 1) {
#pragma unroll
    for (int k = 0; k < M; ++k) xch[h * M + k] = s.v[k];
  }
  __syncthreads();
  if (part && w == 0) {
    mdr<M> t;
#pragma unroll
    for (int k = 0; k < M; ++k) t.v[k] = xch[h * M + k];
    s = md_add<M>(s, t);
  }
  __syncthreads();
  return s;
}

// The parts on wave 0's lanes 0 (re) and 2 (im) to every lane (all threads
// call this).
template <int M>
__device__ __forceinline__ mdc<M> lead4_bcast(const mdr<M> &s, int w, int lane, double *xch) {
  if (w == 0 && (lane == 0 || lane == 2)) {
#pragma unroll
    for (int k = 0; k < M; ++k) xch[(lane >> 1) * M + k] = s.v[k];
  }
  __syncthreads();
  mdc<M> z;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    z.re.v[k] = xch[k];
    z.im.v[k] = xch[M + k];
  }
  __syncthreads();
  return z;
}

// The scalars of reflector j as qr_reflector_scalars forms them, with
// |alpha|^2 from the row pass (c_abs2 of row j there) and the division for
// beta on wave 1 while wave 0 forms phi, v_0 and R_jj.  s: sigma^2 on wave
// 0, lane 0; alpha and a2 on every lane.  All threads of the workgroup call
// this; xch: 3 M doubles of LDS.
template <int M>
__device__ __forceinline__ void qr_lead4_scalars(const mdr<M> &s, const mdc<M> &alpha,
                                                 const mdr<M> &a2, int j, int n, QrShared<M> &sh,
                                                 double *__restrict__ QR, long E,
                                                 double *__restrict__ vdiag,
                                                 double *__restrict__ beta, double *xch,
                                                 int &st) {
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  const int base = 0, sub = lane;
  mdr<M> s2 = md_zero<M>(), sigma = md_zero<M>(), sp = md_zero<M>(), ya = md_zero<M>();
  if (w == 0) {
    s2 = shfl_r<M>(s, base);
    const mdr<M> xq = sub == 0 ? s2 : a2;
    const mdr<M> yq = rsqrt_doubling<M>(xq);
    const mdr<M> zq = md_mul<M>(xq, yq);
    const mdr<M> ys = shfl_r<M>(yq, base);
    ya = shfl_r<M>(yq, base + 1);
    sigma = shfl_r<M>(zq, base);
    const mdr<M> aabs = a2.v[0] == 0.0 ? md_zero<M>() : shfl_r<M>(zq, base + 1);
    sp = md_add<M>(aabs, sigma);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < M; ++k) {
        xch[k] = ys.v[k];
        xch[M + k] = sp.v[k];
      }
    }
  }
  __syncthreads();
  mdr<M> w0, w1, w2, w3;
  if (w == 1) {
    mdr<M> ys1, sp1;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      ys1.v[k] = xch[k];
      sp1.v[k] = xch[M + k];
    }
    const mdr<M> bet_q = md_div<M>(ys1, sp1);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < M; ++k) xch[2 * M + k] = bet_q.v[k];
    }
  } else if (w == 0) {
    const bool a_zero = a2.v[0] == 0.0;
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
    w0 = shfl_r<M>(w_q, base);
    w1 = shfl_r<M>(w_q, base + 1);
    w2 = shfl_r<M>(w_q, base + 2);
    w3 = shfl_r<M>(w_q, base + 3);
  }
  __syncthreads();
  if (w == 0 && lane == 0) {
    mdr<M> bet = md_zero<M>();
    mdc<M> v0 = c_zero<M>(), rjj = c_zero<M>();
    if (s2.v[0] == 0.0) {
      st |= MD_ST_SINGULAR;
    } else {
      v0.re = w0;
      v0.im = w1;
#pragma unroll
      for (int k = 0; k < M; ++k) bet.v[k] = xch[2 * M + k];
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

// Step j of member 0: column l = j + 1 updated by reflector j (j >= 0; for
// j < 0 column 0 as it is), then reflector l from it.  All threads of the
// workgroup call this; waves from the fifth on only meet the barriers.
template <int M>
__device__ __forceinline__ void qr_lead4_step(int j, int N, int n, int seg,
                                              double *__restrict__ QR, long E,
                                              double *__restrict__ vdiag,
                                              double *__restrict__ beta, QrShared<M> &sh,
                                              double *xch, int &st) {
  const int lane = lane_id(), w = threadIdx.x / WAVE, q = lane & 3;
  const bool act = w < 4;
  const int i = 4 * (lane >> 2) + w;  // the lane's row
  const bool rowok = act && i < seg && i < N;
  const int l = j + 1;
  mdr<M> part = md_zero<M>();  // updated column: re on q = 0, im on q = 2
  if (j < 0) {
    if (rowok) {
      const mdc<M> a = cload<M>(QR, E, long(i) * n + l);
      part = (q & 2) ? a.im : a.re;
    }
  } else {
    const bool live = rowok && i >= j;
    mdc<M> v = c_zero<M>(), a = c_zero<M>();
    mdr<M> bet = md_zero<M>();
    mdr<M> s = md_zero<M>();
    if (act) {
      bet = rload<M>(beta, n, j);
      if (live) {
        v = i == j ? cload<M>(vdiag, n, j) : cload<M>(QR, E, long(i) * n + j);
        a = cload<M>(QR, E, long(i) * n + l);
      }
      // conj(v_i) a_i: real product q, then re = p0 - p1 (q = 0), im = p2 + p3 (q = 2)
      const mdr<M> pq = md_mul<M>((q & 1) ? md_neg<M>(v.im) : v.re, (q == 0 || q == 3) ? a.re : a.im);
      mdr<M> t = shfl_down_r<M>(pq, 1);
      if (q == 0) t = md_neg<M>(t);
      const mdr<M> z = md_add<M>(pq, t);
      s = live ? z : md_zero<M>();
    }
    s = lead4_sum<M>(s, seg, w, lane, act, xch);
    const mdc<M> wv = lead4_bcast<M>(s, w, lane, xch);
    if (act) {
      // beta w, then (beta w) v_i the same way, then a_i minus it
      const mdr<M> bw = md_mul<M>((q & 1) ? wv.im : wv.re, bet);
      const mdr<M> pq = md_mul<M>(bw, (q == 0 || q == 3) ? v.re : v.im);
      mdr<M> t = shfl_down_r<M>(pq, 1);
      if (q == 0) t = md_neg<M>(t);
      const mdr<M> z = md_add<M>(pq, t);
      part = live ? md_add<M>((q & 2) ? a.im : a.re, md_neg<M>(z)) : md_zero<M>();
      if (live && i != l && (q == 0 || q == 2))
        rstore<M>(QR + size_t(q >> 1) * M * E, E, long(i) * n + l, part);
    }
  }
  // reflector l: |a_i|^2 = re^2 + im^2 on q = 0 over rows l..N-1, alpha = row l
  mdr<M> s = md_zero<M>(), za = md_zero<M>();
  if (act) {
    const mdr<M> pq = md_mul<M>(part, part);
    const mdr<M> t = shfl_down_r<M>(pq, 2);
    za = md_add<M>(pq, t);
    s = (rowok && i >= l) ? za : md_zero<M>();
  }
  s = lead4_sum<M>(s, seg, w, lane, act, xch);
  // alpha (re, im) and |alpha|^2 from the lanes of row l
  if (rowok && i == l && (q == 0 || q == 2)) {
#pragma unroll
    for (int k = 0; k < M; ++k) xch[(q >> 1) * M + k] = part.v[k];
    if (q == 0) {
#pragma unroll
      for (int k = 0; k < M; ++k) xch[2 * M + k] = za.v[k];
    }
  }
  __syncthreads();
  mdc<M> alpha;
  mdr<M> a2;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    alpha.re.v[k] = xch[k];
    alpha.im.v[k] = xch[M + k];
    a2.v[k] = xch[2 * M + k];
  }
  __syncthreads();
  qr_lead4_scalars<M>(s, alpha, a2, l, n, sh, QR, E, vdiag, beta, xch, st);
}

// The QR of A_0 over G >= 2 workgroups: member 0 the look-ahead column and
// the reflectors (qr_lead4_step), members 1..G-1 the columns j+2.. of step
// j, one per segment, with qr_update_column; a gang barrier ends each step.
template <int M, class Sync>
__device__ __forceinline__ void qr_gang_lead4(QrShared<M> &sh, double *xch, int N, int n, int seg,
                                              const double *__restrict__ A0, long A0E,
                                              double *__restrict__ QR,
                                              double *__restrict__ vdiag,
                                              double *__restrict__ beta, int &st, int member,
                                              int G, Sync gsync) {
  const long E = long(N) * n;
  const int lane = lane_id();
  const int wave = threadIdx.x / WAVE;
  const int nwaves = blockDim.x / WAVE;
  const int lis = lane & (seg - 1);
  const int spw = WAVE / seg;
  const int nslots = nwaves * spw;
  const int GS = (G - 1) * nslots;                                  // slots of members 1..
  const int gs = (member - 1) * nslots + wave * spw + lane / seg;  // this segment's slot
  for (long e = long(member) * blockDim.x + threadIdx.x; e < E; e += long(G) * blockDim.x)
    cstore<M>(QR, E, e, cload<M>(A0, A0E, e));
  gsync();
  for (int j = -1; j < n; ++j) {
    if (member == 0) {
      if (j + 1 < n) qr_lead4_step<M>(j, N, n, seg, QR, E, vdiag, beta, sh, xch, st);
    } else if (j >= 0 && n - j - 2 > 0) {
      mdc<M> vi[1], anew[1];
      const mdc<M> v0 = cload<M>(vdiag, n, j);
      const mdr<M> bet = rload<M>(beta, n, j);
      vi[0] = c_zero<M>();
      if (lis == j) vi[0] = v0;
      else if (lis > j && lis < N) vi[0] = cload<M>(QR, E, long(lis) * n + j);
      const int rounds = (n - j - 2 + GS - 1) / GS;
      for (int k = 0; k < rounds; ++k) {
        const int l = j + 2 + k * GS + gs;
        qr_update_column<M, 1, true>(l < n, l, j, N, n, seg, vi, v0, bet, QR, E, anew);
      }
    }
    gsync();
  }
}

}  // namespace mds
