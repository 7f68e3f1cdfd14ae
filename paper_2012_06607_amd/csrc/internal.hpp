// Host-side launchers shared between the entry points (one library).
#pragma once

#include "common.hpp"

namespace mds {

int eval_diff_enqueue(int m, int d, const md_system &sys, const double *x, double *f, double *A,
                      void *ws, size_t ws_bytes, hipStream_t s);
int qr_enqueue(int m, int N, int n, const double *A0, long A0_stride_planes, double *QR,
               double *vdiag, double *beta, int32_t *status, hipStream_t s);
int solve_enqueue(int m, int N, int n, int d, const double *QR, const double *vdiag,
                  const double *beta, const double *A, const double *b, bool negate_b,
                  double *dx, void *ws, size_t ws_bytes, int32_t *status, hipStream_t s);

inline bool aligned256(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255) == 0; }

}  // namespace mds
