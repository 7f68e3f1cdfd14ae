// Workspace layouts (byte offsets into the caller's device workspace).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace mds {

__host__ __device__ inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Evaluation: one block of series slots per term.  Slot 0 holds the value
// c(t) P_D(t); slots 1..Dmax the derivative at factor position j (first
// occurrences only); then the forward products P_2..P_Dmax, the backward
// products Q_2..Q_{Dmax-1} and the cross products C_2..C_{Dmax-1}.
struct EvalLayout {
  int Dmax = 0, S = 0;
  long E = 0;  // complex elements in the slot planes
  size_t bytes = 0;
  EvalLayout() = default;
  __host__ __device__ EvalLayout(int m, int N, int n, int d, int M, int max_deg) {
    (void)N;
    (void)n;
    Dmax = max_deg;
    S = 1 + Dmax + (Dmax > 1 ? Dmax - 1 : 0) + 2 * (Dmax > 2 ? Dmax - 2 : 0);
    E = long(M) * S * (d + 1);
    bytes = align256(sizeof(double) * 2 * m * (E > 0 ? E : 1));
  }
  __host__ __device__ int val() const { return 0; }
  __host__ __device__ int der(int j) const { return j; }                                       // j = 1..D
  __host__ __device__ int P(int j) const { return 1 + Dmax + (j - 2); }                         // j = 2..D
  __host__ __device__ int Q(int j) const { return 1 + Dmax + (Dmax - 1) + (j - 2); }            // j = 2..D-1
  __host__ __device__ int C(int j) const { return 1 + Dmax + (Dmax - 1) + (Dmax - 2) + (j - 2); }  // j = 2..D-1
};

// Staggered solve: the right hand sides r (d+1, N), the n x N matrix
// W = R^{-1} (Q^H)_{0:n}, then 1/R_ii (n).
// Staggered solve: the right-hand sides r (d+1 x N), W (n x N) and 1/R_ii
// (n), then the scratch of the one-path W formation (pinv_scratch_doubles).
struct SolveLayout {
  size_t off_r, off_G, off_pw, bytes;
  __host__ __device__ SolveLayout(int m, int N, int n, int d) {
    off_r = 0;
    off_G = align256(sizeof(double) * 2 * m * size_t(d + 1) * N);
    off_pw = off_G + align256(sizeof(double) * 2 * m * (size_t(n) * N + n));
    bytes = off_pw + align256(sizeof(double) * 2 * m * (4 * size_t(n) * n + 2 * size_t(n) * N));
  }
};

// Newton step: f, A, QR factors, dx, then the solve and eval workspaces.
struct NewtonLayout {
  size_t off_f, off_A, off_QR, off_vd, off_beta, off_dx, off_solve, off_eval, off_ctr, bytes;
  __host__ __device__ NewtonLayout(int m, int N, int n, int d, int M, int max_deg) {
    const size_t L = size_t(d + 1);
    size_t o = 0;
    off_f = o;
    o += align256(sizeof(double) * 2 * m * L * N);
    off_A = o;
    o += align256(sizeof(double) * 2 * m * L * N * n);
    off_QR = o;
    o += align256(sizeof(double) * 2 * m * size_t(N) * n);
    off_vd = o;
    o += align256(sizeof(double) * 2 * m * size_t(n));
    off_beta = o;
    o += align256(sizeof(double) * m * size_t(n));
    off_dx = o;
    o += align256(sizeof(double) * 2 * m * L * n);
    off_solve = o;
    o += SolveLayout(m, N, n, d).bytes;
    off_eval = o;
    o += EvalLayout(m, N, n, d, M, max_deg).bytes;
    off_ctr = o;  // a gang's term queue (batched launch), the QR's barrier word (one path)
    o += 256;
    bytes = o;
  }
};

// Adjoint: the Newton step's buffers, then lambda (d+1, N) and, when the
// monomial series are stored, (M, d+1) of them.
struct AdjointLayout {
  NewtonLayout nl;
  size_t off_lam, off_mono, bytes;
  __host__ __device__ AdjointLayout(int m, int N, int n, int d, int M, int max_deg, bool store)
      : nl(m, N, n, d, M, max_deg) {
    off_lam = nl.bytes;
    off_mono = off_lam + align256(sizeof(double) * 2 * m * size_t(d + 1) * N);
    bytes = off_mono + (store ? align256(sizeof(double) * 2 * m * size_t(M > 0 ? M : 1) * (d + 1)) : 0);
  }
};

// Newton protocol over increasing truncation degrees: a Newton step's
// buffers sized for the largest degree, the iterate of the current degree
// ((dmax+1) x n at most), the step's update norms (m, 2), the start point
// (n; kept by the batched form) and the flags (running, stopped).
struct ProtocolLayout {
  NewtonLayout nl;
  size_t off_x, off_nrm, off_x0, off_flags, bytes;
  __host__ __device__ ProtocolLayout(int m, int N, int n, int dmax, int M, int max_deg)
      : nl(m, N, n, dmax, M, max_deg) {
    off_x = nl.bytes;
    off_nrm = off_x + align256(sizeof(double) * 2 * m * size_t(dmax + 1) * n);
    off_x0 = off_nrm + align256(sizeof(double) * m * 2);
    off_flags = off_x0 + align256(sizeof(double) * 2 * m * size_t(n));
    bytes = off_flags + 256;
  }
};

// Pade approximants: per series the M x M Toeplitz matrix (factored in
// place), the reflector heads, beta, 1/R_ii, the right-hand side and the
// solution.
struct PadeLayout {
  size_t off_QR, off_vd, off_beta, off_invd, off_rhs, off_sol, per_series, bytes;
  __host__ __device__ PadeLayout(int m, int Md, long count) {
    const size_t Mq = size_t(Md > 0 ? Md : 1);
    off_QR = 0;
    off_vd = align256(sizeof(double) * 2 * m * Mq * Mq);
    off_beta = off_vd + align256(sizeof(double) * 2 * m * Mq);
    off_invd = off_beta + align256(sizeof(double) * m * Mq);
    off_rhs = off_invd + align256(sizeof(double) * 2 * m * Mq);
    off_sol = off_rhs + align256(sizeof(double) * 2 * m * Mq);
    per_series = off_sol + align256(sizeof(double) * 2 * m * Mq);
    bytes = per_series * size_t(count > 0 ? count : 1);
  }
};

}  // namespace mds
