// Host-side launchers shared between the entry points (one library).
#pragma once

#include "common.hpp"

namespace mds {

// mono (optional): the monomial series of every term, planes (2, m, M, d+1)
// gate (optional, device): every kernel returns at once while *gate == 0
int eval_diff_enqueue(int m, int d, const md_system &sys, const double *x, double *f, double *A,
                      void *ws, size_t ws_bytes, hipStream_t s, double *mono = nullptr,
                      const int32_t *gate = nullptr);
// ctr (optional, device int32): spread the trailing columns over several
// workgroups that meet at barriers on *ctr (same bits)
int qr_enqueue(int m, int N, int n, const double *A0, long A0_stride_planes, double *QR,
               double *vdiag, double *beta, int32_t *status, hipStream_t s,
               const int32_t *gate = nullptr, int32_t *ctr = nullptr);
int qr_gang_size(int m, int N, int n);
// invd = 1 / R_ii and W = R^{-1} (Q^H)_{0:n} (row-major n x N); N <= 256;
// scratch: SolveLayout's off_pw region (2 m (4 n^2 + 2 n N) doubles)
int pinv_enqueue(int m, int N, int n, const double *QR, const double *vdiag, const double *beta,
                 double *invd, double *W, double *scratch, int32_t *status, hipStream_t s,
                 const int32_t *gate = nullptr);
int solve_enqueue(int m, int N, int n, int d, const double *QR, const double *vdiag,
                  const double *beta, const double *A, const double *b, bool negate_b,
                  double *dx, void *ws, size_t ws_bytes, int32_t *status, hipStream_t s,
                  const int32_t *gate = nullptr);

struct EvalArgs;
// grad c (planes (2, 2, M, dc+1)) from lambda, recomputing the monomials
int contract_recompute_enqueue(int m, const EvalArgs &a, const double *lam, double *grad,
                               hipStream_t s);

inline bool aligned256(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255) == 0; }

}  // namespace mds
