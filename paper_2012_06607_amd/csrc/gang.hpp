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

}  // namespace mds
