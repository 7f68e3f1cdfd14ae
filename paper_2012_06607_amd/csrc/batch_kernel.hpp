// Many independent solution paths in one persistent launch: the kernel.
//
// The paper's job queue (Section 5, Figure 1): all data is set up before
// the workers start, each job reads shared inputs and writes its own
// workspace, and a counter guarded by a lock hands out the next job.  Here
// the workers are workgroups resident on the GPU, the counter is one device
// atomic per queue, and a job is a whole path: `iters` Newton steps
// (evaluation and differentiation, QR of A_0, R^{-1} Q^H, the staggered
// solve, the update) run by that workgroup with barriers between the stages
// (the paper's stage synchronisation by terminating tasks).  Jobs are taken
// in the order the caller gives (longest first balances the load), and each
// workgroup dispatches on its path's precision.
//
// A large path may be a gang of G workgroups (G members, one job each).
// The members split the term evaluations, the Jacobian rows, the columns of
// each QR step, the columns of R^{-1} Q^H and the right-hand-side updates,
// and meet at gang barriers (a counter in device memory, with device-scope
// release and acquire).  The update of x runs on member 0; every member
// computes the stage products dx_k itself (the same bits), so a stage costs
// one gang barrier.
// With one queue per accelerator die (queue q served by the workgroups on
// die q) a gang's members share that die's L2.
#pragma once

#include "gang.hpp"
#include "internal.hpp"

namespace mds {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// max over the workgroup of an exact selection (values are compared, the
// bits of the largest are kept), through LDS
template <int M>
__device__ __forceinline__ mdr<M> wg_max(mdr<M> v, mdr<M> *sh) {
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const mdr<M> t = shfl_down_r<M>(v, o);
    if (lane_id() < o && md_less<M>(v, t)) v = t;
  }
  const int wave = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  if (lane_id() == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < nw; ++w)
      if (md_less<M>(v, sh[w])) v = sh[w];
  __syncthreads();
  return v;
}

// Accelerator die (XCC) of the calling wave.
__device__ __forceinline__ int xcc_id() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return int(v & 0xf);
}

// Protocol control of one path's steps at one truncation degree (the
// batched form of Section 6's protocol): after each step member 0 compares
// |dx_d| with tol (from step min_steps on) and publishes the decision in
// `word` (the path's workspace) before the step's closing gang barrier, so
// every member reads the same decision.  `steps` and `norm` receive the
// steps taken and the last |dx_d| (member 0).
template <int M>
struct StepCtl {
  bool on = false;
  int min_steps = 1;
  double tol = 0.0;
  int32_t *word = nullptr;
  int *steps = nullptr;
  mdr<M> *norm = nullptr;
};

// `iters` Newton steps on the path at truncation degree d (<= p.d) with the
// series x (planes (2, m, d+1, n)), or fewer under a StepCtl.
template <int M>
__device__ __forceinline__ void newton_steps(const md_path &p, int d, double *__restrict__ x,
                            bool store_norm, int iters, const int32_t *__restrict__ ints,
                            double *__restrict__ reals, double *__restrict__ wsb,
                            int32_t *__restrict__ status, int path, double *lds_raw,
                            int eval_waves, int member, int G, int32_t *gang_ctr,
                            int64_t *pclk, int &st, int &round, const StepCtl<M> &ctl) {
  __shared__ QrShared<M> qsh;
  __shared__ mdr<M> msh[16];  // one per wave, up to 1024 threads
  __shared__ int term_next;   // the workgroup's term queue (one workgroup per path)
  const int N = p.N, n = p.n, L = d + 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid / WAVE, nwaves = nt / WAVE;
  const NewtonLayout lay(M, N, n, d, p.M, p.max_deg);
  char *w = reinterpret_cast<char *>(wsb + p.ws);
  double *f = reinterpret_cast<double *>(w + lay.off_f);
  double *A = reinterpret_cast<double *>(w + lay.off_A);
  double *QR = reinterpret_cast<double *>(w + lay.off_QR);
  double *vd = reinterpret_cast<double *>(w + lay.off_vd);
  double *beta = reinterpret_cast<double *>(w + lay.off_beta);
  double *dx = reinterpret_cast<double *>(w + lay.off_dx);
  const SolveLayout sl(M, N, n, d);
  double *r = reinterpret_cast<double *>(w + lay.off_solve + sl.off_r);
  double *W = reinterpret_cast<double *>(w + lay.off_solve + sl.off_G);
  double *invd = W + size_t(2) * M * n * N;
  int32_t *gang_terms = reinterpret_cast<int32_t *>(w + lay.off_ctr);
  EvalArgs a;
  a.d = d;
  a.N = N;
  a.n = n;
  a.Mt = p.M;
  a.dc = p.dc;
  a.Dmax = p.max_deg;
  a.lay = EvalLayout(M, N, n, d, p.M, p.max_deg);
  a.S = a.lay.S;
  a.eq_ptr = ints + p.eq_ptr;
  a.term_ptr = ints + p.term_ptr;
  a.factors = ints + p.factors;
  a.coef = reals + p.coef;
  a.x = x;
  a.ws = reinterpret_cast<double *>(w + lay.off_eval);
  a.Ews = a.lay.E;
  a.f = f;
  a.A = A;
  // stage products: up to eight products per lane, or wider segments (fewer
  // products per lane, a deeper tree) while all rows still fit in 256 lanes.
  // The choice depends on the path's sizes only, so the bits do not depend
  // on the launch shape or the gang split.
  auto stage_seg = [&](int len, long rows) {
    int sg = dot_seg_throughput(len);
    const int smax = len >= WAVE ? WAVE : pow2_at_least(len);
    while (sg < smax && rows * 2 * sg <= 4 * WAVE) sg *= 2;
    return sg;
  };
  const int seg_dx = stage_seg(N, n);
  // QR and R^{-1} Q^H: up to four rows per lane, wider segments (fewer rows
  // per lane) while all columns fit in 512 lanes; sizes only, as above
  auto col_seg = [&](int cols) {
    int sg = pow2_at_least((N + 3) / 4);
    const int smax = N >= WAVE ? WAVE : pow2_at_least(N);
    while (sg < smax && long(cols) * 2 * sg <= 8 * WAVE) sg *= 2;
    return sg;
  };
  const int seg_q = col_seg(n), seg_p = col_seg(N);
  const int spw_p = WAVE / seg_p, nslots_p = nwaves * spw_p;
  const int slot_p = wave * spw_p + lane_id() / seg_p;
  const int spw_x = WAVE / seg_dx, nslots_x = nwaves * spw_x;
  const int slot_x = wave * spw_x + lane_id() / seg_dx;
  const int rgrp = eval_group(d);
  const int per_wave = term_lds_series(p.max_deg) * L;
  mdc<M> *lds = reinterpret_cast<mdc<M> *>(lds_raw);
  // during the stages the evaluation's LDS holds a copy of dx_k (planes
  // (2, M, n); md_batch_lds_bytes leaves room for n = 64)
  double *lds_dx = reinterpret_cast<double *>(lds_raw);
  const long Ex = long(L) * n, Er = long(L) * N;
  (void)Er;
  // phase clocks (optional): member 0's thread 0 adds the device wall-clock
  // time of each phase of every step to pclk[0..6] (evaluation, Jacobian
  // sums, QR, R^{-1} Q^H, stages, update); the phases end at barriers, so
  // the gang's members are done too
  const bool timing = pclk && member == 0 && tid == 0;
  int64_t tprev = timing ? wall_clock64() : 0;
  auto phase = [&](int ph) {
    if (timing) {
      const int64_t t = wall_clock64();
      pclk[ph] += t - tprev;
      tprev = t;
    }
  };
  auto gsync = [&] {
    if (G > 1) gang_barrier(gang_ctr, G, round, st);
    else __syncthreads();
  };
  if (tid == 0) term_next = 0;
  if (G > 1) {
    if (member == 0 && tid == 0) *gang_terms = 0;
    gsync();  // the gang's term queue starts at zero for every member
  } else {
    __syncthreads();
  }
  for (int it = 0; it < iters; ++it) {
    // evaluation and differentiation: waves over terms, each wave taking
    // the next term from a queue (in LDS for a path on one workgroup, in the
    // path's workspace for a gang), so terms of unequal degree even out;
    // then the sums, one (equation, coefficient) pair per lane (each wave
    // clears its rows of A first), with r = -f written by the lane that
    // formed f
    if (wave < eval_waves) {
      auto next_term = [&](int) __attribute__((always_inline)) {
        int t = 0;
        if (lane_id() == 0) t = G > 1 ? atomicAdd(gang_terms, 1) : atomicAdd(&term_next, 1);
        return __shfl(t, 0);
      };
      for (int tau = next_term(-1); tau < p.M; tau = next_term(tau))
        eval_term_wave<M>(a, tau, rgrp, lds + wave * per_wave, [] { wave_sync(); });
    }
    gsync();
    phase(0);
    // the queues start again at zero for the next step (read after later
    // barriers, gang barriers for the gang's queue)
    if (tid == 0) term_next = 0;
    if (G > 1 && member == 0 && tid == 0) *gang_terms = 0;
    for (long g0 = long(member) * nt + wave * WAVE; g0 < long(L) * N; g0 += long(G) * nt)
      eval_accumulate_wave<M>(a, g0, r, [] { wave_sync(); });
    gsync();
    phase(1);
    // QR of A_0 (the k = 0 block of A), its columns over all members of a
    // gang, then W = R^{-1} (Q^H)_{0:n}: the rows of (Q^H)_{0:n}, then the
    // back substitution by columns, both over all members
    if (G > 1) {
      qr_gang<M, 4>(qsh, N, n, seg_q, A, long(L) * N * n, QR, vd, beta, st, member, G, gsync);
      if (member == 0) inv_diag_range<M>(tid, nt, N, n, QR, invd, st);
    } else {
      qr_wg<M, 4>(qsh, N, n, seg_q, A, long(L) * N * n, QR, vd, beta, st);
      inv_diag_range<M>(tid, nt, N, n, QR, invd, st);
    }
    gsync();
    phase(2);
    {
      // the rows of (Q^H)_{0:n}: row r costs r + 1 reflectors, so the rows
      // go out longest first and snaking over the slots of all members,
      // which evens out every slot's total
      const int T = G * nslots_p, gs = member * nslots_p + slot_p;
      for (int k = 0; k * T < n; ++k) {
        const int u = k * T + ((k & 1) ? T - 1 - gs : gs);
        q_row<M, 4>(u < n, n - 1 - u, N, n, seg_p, QR, vd, beta, W);
      }
    }
    gsync();
    for (int base = member * nslots_p; base < N; base += G * nslots_p) {
      const int c = base + slot_p;
      backsub_column<M, 4>(c < N, c, N, n, seg_p, QR, invd, W);
    }
    gsync();
    phase(3);
    // staggered substitution: every member forms dx_k, the updates of the
    // later right hand sides are split over the members
    for (int k = 0; k <= d; ++k) {
      for (int base = 0; base < n; base += nslots_x) {
        const int i = base + slot_x;
        stage_dx_row<M>(i < n, i, k, N, n, d, seg_dx, W, r, dx, st,
                        (M == 3 || M == 4) ? lds_dx : nullptr);
      }
      __syncthreads();
      if (k < d) {
        const long rows = long(d - k) * N;
        const int seg_up = stage_seg(n, rows);
        if constexpr (M >= 5) {
          const int spw_u = WAVE / seg_up, nslots_u = nwaves * spw_u;
          const int slot_u = wave * spw_u + lane_id() / seg_up;
          for (long base = long(member) * nslots_u; base < rows; base += long(G) * nslots_u) {
            const long row = base + slot_u;
            stage_update_row<M>(row < rows, row, k, N, n, d, seg_up, A, dx, r);
          }
        } else if constexpr (M >= 3) {
          // triple and quad double: dx_k from its copy in LDS (each member
          // formed all of it), not through the vector caches
          const int spw_u = WAVE / seg_up, nslots_u = nwaves * spw_u;
          const int slot_u = wave * spw_u + lane_id() / seg_up;
          for (long base = long(member) * nslots_u; base < rows; base += long(G) * nslots_u) {
            const long row = base + slot_u;
            stage_update_row_lds<M>(row < rows, row, k, N, n, d, seg_up, A, lds_dx, r);
          }
        } else {
          // double and double double: the rows stream A_j through the
          // vector caches, so each lane reads its (at most eight) entries of
          // dx_k once per stage instead of once per row.  (Four entries of
          // quad double per lane, with wider segments, measured slower: the
          // registers are not there.)
          const int spw_u = WAVE / seg_up, nslots_u = nwaves * spw_u;
          const int slot_u = wave * spw_u + lane_id() / seg_up;
          mdc<M> dxr[8];
          const int lis = lane_id() & (seg_up - 1);
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int l = lis + t * seg_up;
            dxr[t] = l < n ? cload<M>(dx, Ex, long(k) * n + l) : c_zero<M>();
          }
          for (long base = long(member) * nslots_u; base < rows; base += long(G) * nslots_u) {
            const long row = base + slot_u;
            stage_update_row_reg<M, 8>(row < rows, row, k, N, n, d, seg_up, A, dxr, r);
          }
        }
        gsync();
      }
    }
    phase(4);
    if (member == 0) {
      // x += dx and the size of the update (member 0)
      mdr<M> bd = md_zero<M>(), ba = md_zero<M>();
      for (long e = tid; e < Ex; e += nt) {
        const mdc<M> u = cload<M>(dx, Ex, e);
        cstore<M>(x, Ex, e, c_add<M>(cload<M>(x, Ex, e), u));
        const mdr<M> a2 = c_abs2<M>(u);
        if (md_less<M>(ba, a2)) ba = a2;
        if (e >= long(d) * n && md_less<M>(bd, a2)) bd = a2;
      }
      bd = wg_max<M>(bd, msh);
      ba = wg_max<M>(ba, msh);
      if (tid == 0 && store_norm && it == iters - 1) {
        rstore<M>(reals + p.dx_norm, 2, 0, md_sqrt<M>(bd));
        rstore<M>(reals + p.dx_norm, 2, 1, md_sqrt<M>(ba));
      }
      if (ctl.on && tid == 0) {
        // this step's stopping decision, for every member of the gang
        const mdr<M> nd = md_sqrt<M>(bd);
        *ctl.norm = nd;
        *ctl.steps = it + 1;
        const bool done = it + 1 >= ctl.min_steps && !md_less<M>(md_from<M>(ctl.tol), nd);
        __hip_atomic_store(ctl.word, done ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (ctl.on) {
      gsync();  // the decision is visible to every member
      const int stop = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(ctl.word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      phase(5);
      if (stop) break;
    } else {
      if (it + 1 < iters) gsync();
      else __syncthreads();
      phase(5);
    }
  }
}

// One path: `iters` Newton steps at the path's degree, or, with a protocol,
// Section 6's protocol over its degrees (each degree from the start point,
// steps until |dx_d| <= tol from step min_steps on or the degree's limit,
// the later degrees skipped once a degree ends above the divergence bound;
// the series of the last degree run ends in x, zero above that degree).
template <int M>
__device__ __forceinline__ void newton_path(const md_path &p, int iters, const int32_t *__restrict__ ints,
                            double *__restrict__ reals, double *__restrict__ wsb,
                            int32_t *__restrict__ status, int path, double *lds_raw,
                            int eval_waves, int member, int G, int32_t *gang_ctr,
                            int64_t *pclk, const md_protocol *proto, int32_t *proto_iters,
                            double *proto_norms) {
  int st = 0, round = 0;
  const int tid = threadIdx.x;
  double *x = reals + p.x;
  if (!proto) {
    newton_steps<M>(p, p.d, x, true, iters, ints, reals, wsb, status, path, lds_raw, eval_waves,
                    member, G, gang_ctr, pclk, st, round, StepCtl<M>{});
  } else {
    const ProtocolLayout pl(M, p.N, p.n, p.d, p.M, p.max_deg);
    char *w = reinterpret_cast<char *>(wsb + p.ws);
    double *xj = reinterpret_cast<double *>(w + pl.off_x);
    double *x0 = reinterpret_cast<double *>(w + pl.off_x0);
    int32_t *words = reinterpret_cast<int32_t *>(w + pl.off_flags);
    const int n = p.n, ndeg = proto->ndeg;
    const long E0 = long(p.d + 1) * n;
    auto gsync = [&] {
      if (G > 1) gang_barrier(gang_ctr, G, round, st);
      else __syncthreads();
    };
    // the start point, kept while x receives each degree's series
    if (member == 0)
      for (long e = tid; e < n; e += blockDim.x) cstore<M>(x0, n, e, cload<M>(x, E0, e));
    gsync();
    int stopped = 0;
    for (int j = 0; j < ndeg; ++j) {
      const int dj = proto->degrees[j];
      const bool run = !stopped && dj <= p.d;
      int steps = 0;
      mdr<M> nd = md_zero<M>();
      if (run) {
        const long Ej = long(dj + 1) * n;
        if (member == 0)
          for (long e = tid; e < Ej; e += blockDim.x)
            cstore<M>(xj, Ej, e, e < n ? cload<M>(x0, n, e) : c_zero<M>());
        gsync();
        StepCtl<M> ctl;
        ctl.on = true;
        ctl.min_steps = proto->min_steps;
        ctl.tol = proto->tol;
        ctl.word = words;
        ctl.steps = &steps;
        ctl.norm = &nd;
        newton_steps<M>(p, dj, xj, false, proto->maxit[j], ints, reals, wsb, status, path,
                        lds_raw, eval_waves, member, G, gang_ctr, pclk, st, round, ctl);
        // the degree's series to x (member 0), and whether the next degrees run
        if (member == 0) {
          for (long e = tid; e < E0; e += blockDim.x)
            cstore<M>(x, E0, e, e < Ej ? cload<M>(xj, Ej, e) : c_zero<M>());
          if (tid == 0) {
            const bool div = md_less<M>(md_from<M>(proto->diverge), nd);
            __hip_atomic_store(words + 1, div ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (div) st |= MD_ST_DIVERGED;
          }
        }
        gsync();
        stopped = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(words + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      }
      if (member == 0 && tid == 0) {
        proto_iters[long(path) * ndeg + j] = run ? steps : 0;
        for (int l = 0; l < 10; ++l)
          proto_norms[(long(path) * ndeg + j) * 10 + l] = (run && l < M) ? nd.v[l] : 0.0;
      }
    }
  }
  if (tid == 0) {
    if (st) atomicOr(status + path, st);
    if (member == 0) atomicAnd(status + path, ~MD_ST_NOTRUN);
  }
}

// BLOCK threads per workgroup; MS: 0 for the kernel of double to quad
// double paths (m in 1..4), else the one limb count (5, 8 or 10) the
// kernel carries (one translation unit each: these compile slowly).
template <int BLOCK, int MS, bool PROTO>
__global__ void __launch_bounds__(BLOCK) k_newton_batch(int npaths, const md_path *__restrict__ paths,
                                                        const int32_t *__restrict__ jobs, int nq,
                                                        const int32_t *__restrict__ qbegin,
                                                        const int32_t *__restrict__ ints,
                                                        double *__restrict__ reals,
                                                        double *__restrict__ wsb, int iters,
                                                        int32_t *counters, int32_t *gang_ctr,
                                                        int32_t *status, int eval_waves,
                                                        int64_t *clk, int64_t *phase_clk,
                                                        md_protocol proto, int32_t *proto_iters,
                                                        double *proto_norms) {
  extern __shared__ double lds_raw[];
  __shared__ int sh_job;
  const int q = nq == 1 ? 0 : xcc_id() % nq;
  const int begin = qbegin[q], end = qbegin[q + 1];
  // Every single-thread action of the job loop (taking the next job, the
  // status of a refused path, the path's end clock) sits in one leader block
  // between two barriers, and the loop has no other exit or back edge.  A
  // leader-only block at the loop head with a `continue` elsewhere lets the
  // compiler route the other lanes' back edge around it straight to the
  // barrier; the loop then becomes divergent and those lanes spin on a stale
  // job while the leader waits, masked off, for them to leave.
  if (threadIdx.x == 0) sh_job = begin + atomicAdd(counters + q, 1);
  __syncthreads();
  int job = __builtin_amdgcn_readfirstlane(sh_job);
  while (job < end) {
    const int path = jobs[2 * job];
    const int G = jobs[2 * job + 1] >> 8, member = jobs[2 * job + 1] & 0xff;
    const bool known = path >= 0 && path < npaths;
    bool ok = false;
    md_path p{};
    if (known) {
      p = paths[path];
      ok = G >= 1 && member < G && p.N >= p.n && p.n >= 1 && p.N <= WAVE && p.d >= 0 &&
           p.max_deg >= 0 &&
           (MS ? p.m == MS : (p.m >= 1 && p.m <= 4));
    }
    if (ok) {
      if (clk && threadIdx.x == 0 && member == 0) clk[2 * path] = wall_clock64();
      int32_t *gc = gang_ctr + path;
      int64_t *pclk = phase_clk ? phase_clk + 8 * long(path) : nullptr;
      if constexpr (MS != 0) {
        newton_path<MS>(p, iters, ints, reals, wsb, status, path, lds_raw, eval_waves, member, G, gc, pclk, PROTO ? &proto : nullptr, proto_iters, proto_norms);
      } else {
        switch (p.m) {
          case 1: newton_path<1>(p, iters, ints, reals, wsb, status, path, lds_raw, eval_waves, member, G, gc, pclk, PROTO ? &proto : nullptr, proto_iters, proto_norms); break;
          case 2: newton_path<2>(p, iters, ints, reals, wsb, status, path, lds_raw, eval_waves, member, G, gc, pclk, PROTO ? &proto : nullptr, proto_iters, proto_norms); break;
          case 3: newton_path<3>(p, iters, ints, reals, wsb, status, path, lds_raw, eval_waves, member, G, gc, pclk, PROTO ? &proto : nullptr, proto_iters, proto_norms); break;
          default: newton_path<4>(p, iters, ints, reals, wsb, status, path, lds_raw, eval_waves, member, G, gc, pclk, PROTO ? &proto : nullptr, proto_iters, proto_norms); break;
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (known && !ok) atomicOr(status + path, MD_ST_BADPATH);
      if (ok && clk && member == 0) clk[2 * path + 1] = wall_clock64();
      sh_job = begin + atomicAdd(counters + q, 1);
    }
    __syncthreads();
    job = __builtin_amdgcn_readfirstlane(sh_job);
  }
}

// Launches of the instantiations (batch.hip: m in 1..4, 256 or 512
// threads; batch_m5.hip, batch_m8.hip, batch_m10.hip: one limb count each,
// 256 threads).
void launch_newton_batch_lo(int block, int grid, size_t lds, hipStream_t s, int npaths,
                            const md_path *paths, const int32_t *jobs, int nq,
                            const int32_t *qbegin, const int32_t *ints, double *reals, double *ws,
                            int iters, int32_t *counters, int32_t *gang_ctr, int32_t *status,
                            int eval_waves, int64_t *clk, int64_t *phase_clk);
// the protocol form of the double- to quad-double kernel (batch_proto.hip)
void launch_newton_batch_proto(int block, int grid, size_t lds, hipStream_t s, int npaths,
                               const md_path *paths, const int32_t *jobs, int nq,
                               const int32_t *qbegin, const int32_t *ints, double *reals,
                               double *ws, int32_t *counters, int32_t *gang_ctr, int32_t *status,
                               int eval_waves, int64_t *clk, int64_t *phase_clk,
                               const md_protocol &proto, int32_t *proto_iters,
                               double *proto_norms);
#define MDS_BATCH_WIDE_LAUNCH(NAME)                                                              \
  void NAME(int grid, size_t lds, hipStream_t s, int npaths, const md_path *paths,              \
            const int32_t *jobs, int nq, const int32_t *qbegin, const int32_t *ints,            \
            double *reals, double *ws, int iters, int32_t *counters, int32_t *gang_ctr,         \
            int32_t *status, int eval_waves, int64_t *clk, int64_t *phase_clk)
MDS_BATCH_WIDE_LAUNCH(launch_newton_batch_m5);
MDS_BATCH_WIDE_LAUNCH(launch_newton_batch_m8);
MDS_BATCH_WIDE_LAUNCH(launch_newton_batch_m10);

}  // namespace mds
