/*
 * mdseries: one Newton step on truncated power series in complex
 * multiple-double precision, on AMD Instinct MI355X (gfx950).
 *
 * Method: J. Verschelde, "Parallel Software to Offset the Cost of Higher
 * Precision", arXiv:2012.06607.  Section 2 defines multiple doubles,
 * Section 3 truncated power series and their product, Section 4 Newton's
 * method on series: evaluation and reverse-mode differentiation of the
 * system, then the block lower triangular Toeplitz solve with one QR of A_0.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Numbers.  A multiple double with m limbs (m in {1,2,3,4,5,8,10}: double,
 *   double double, triple, quad, penta, octo, deca double) is an unevaluated
 *   sum of m doubles, limb 0 the most significant (Section 2).
 * Layout.  A complex multiple-double tensor of logical shape S is a
 *   contiguous float64 array of 2*m*|S| doubles: planes (2, m, S...), the
 *   real part first; element e (row-major index into S) has real limb l at
 *   p[l*|S| + e] and imaginary limb l at p[(m+l)*|S| + e].  Real tensors are
 *   planes (m, S...).  Series vectors are coefficient-major: a series
 *   x(t) = x_0 + x_1 t + ... + x_d t^d of n-vectors has shape (d+1, n); a
 *   matrix series has shape (d+1, N, n) (Section 4: power series with vector
 *   and matrix coefficients).  Inputs must be normalised expansions.
 * Memory.  Every double* / int32_t* argument is a DEVICE pointer (HIP device
 *   memory) owned by the caller; the library never allocates or frees device
 *   memory.  Scratch space is a caller-provided device workspace of at least
 *   md_workspace_bytes(...) bytes, 256-byte aligned.
 * Streams.  `stream` is a hipStream_t (0 = null stream).  Calls only enqueue
 *   work on it: they are asynchronous and never synchronise.
 * Errors.  Argument errors are returned at once as an MD_E* code with a
 *   message in md_last_error() (thread local); nothing is enqueued then.
 *   Numerical conditions found on the device are OR-ed into the caller's
 *   device word *status (when status is not NULL) as MD_ST_* bits; read it
 *   after synchronising the stream.  Callers clear *status before a call.
 * Aliasing.  Outputs must not overlap inputs, except the in/out x of
 *   md_newton_step.
 * Determinism.  Every reduction has a fixed order: the same call on the
 *   same inputs gives the same bits.
 */
#ifndef MDSERIES_H
#define MDSERIES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MD_OK = 0,
  MD_EINVAL = 1,     /* bad m, negative degree or count, unknown op */
  MD_ESHAPE = 2,     /* n < 1, N < n, or sizes out of the supported range */
  MD_ENULL = 3,      /* a required pointer is NULL */
  MD_EWORKSPACE = 4, /* workspace missing, too small or misaligned */
  MD_EHIP = 5        /* a kernel launch failed */
};

enum {
  MD_ST_SINGULAR = 1,  /* a Householder column or a diagonal of R is zero */
  MD_ST_NONFINITE = 2, /* an infinity or NaN reached a result */
  MD_ST_BADPATH = 4,   /* md_newton_batch: a path's sizes or precision are not supported */
  MD_ST_GANG = 8,      /* md_newton_batch: a gang barrier waited too long (results invalid) */
  MD_ST_NOTRUN = 16,   /* md_newton_batch: no workgroup took the path's jobs */
  MD_ST_DIVERGED = 32  /* the update to the last coefficient grew (md_newton_step), or a degree
                          of the adaptive driver ended with it above the divergence bound */
};

/* Polynomial system f = (f_1..f_N) in x = (x_1..x_n), N >= n, whose terms
 * are c(t) x^a with truncated power series coefficients c(t) (Section 4).
 * All pointers are device pointers.
 *   eq_ptr   int32 [N+1]: the terms of equation i are eq_ptr[i]..eq_ptr[i+1]-1
 *   term_ptr int32 [M+1]: the factors of term j are
 *            factors[term_ptr[j]..term_ptr[j+1]-1]
 *   factors  int32 [F]: variable indices in [0, n), with repetition for
 *            powers, non-decreasing within a term; a term without factors is
 *            a constant (a coefficient c(t) alone)
 *   coef     planes (2, m, M, dc+1): coefficient series, degree dc
 * max_deg must be the largest number of factors of a term (host value). */
typedef struct md_system {
  int32_t N, n, M, dc, max_deg;
  const int32_t *eq_ptr;
  const int32_t *term_ptr;
  const int32_t *factors;
  const double *coef;
} md_system;

/* Truncated series product (Section 3): z_k = sum_{i=0}^{k} x_i y_{k-i},
 * k = 0..d, for `count` independent pairs of series; each z_k starts from
 * its first product x_0 y_k and adds the others in increasing i, i.e.
 * (d+2)(d+1)/2 multiplications and (d+1)d/2 additions per pair.
 * x, y, z: planes (2, m, count, d+1).  Errors: MD_EINVAL (m, d < 0,
 * count < 0), MD_ENULL. */
int md_series_convolve(int m, int d, int64_t count, const double *x, const double *y, double *z,
                       void *stream);

/* Series division (Section 3: a series with a nonzero constant term has
 * an inverse, and series divide like numbers): z[c] = x[c] / y[c] mod
 * t^{d+1} for count independent series, planes (2, m, count, d+1).
 * z_0 = x_0 / y_0 and z_k = (x_k - (y_1 z_{k-1} + ... + y_k z_0)) / y_0,
 * the products added in increasing order (the same operations as the
 * oracle, so the bits agree).  A zero y_0 sets MD_ST_SINGULAR in *status
 * (may be NULL) and the quotient is undefined.  z must not overlap x or y.
 * Errors: MD_EINVAL (bad m, d < 0, count < 0), MD_ENULL. */
int md_series_divide(int m, int d, int64_t count, const double *x, const double *y, double *z,
                     int32_t *status, void *stream);

/* [L/M] Pade approximants of count series (Section 3: computed series give
 * rational approximations): c planes (2, m, count, L+M+1) -> p planes
 * (2, m, count, L+1) and q planes (2, m, count, M+1) with q_0 = 1 and
 * q(t) c(t) - p(t) = O(t^{L+M+1}).  The denominator solves the M x M
 * Toeplitz system sum_{j=1..M} c_{L+i-j} q_j = -c_{L+i} (i = 1..M,
 * c_k = 0 for k < 0) by the Householder QR and reflector solve of the
 * Newton step; p_k = sum_{j=0..min(k,M)} q_j c_{k-j}.  One workgroup per
 * series; M <= 64.  A singular system sets MD_ST_SINGULAR.
 * Workspace (M > 0): md_workspace_bytes(MD_FN_PADE, m, M, L, 0, count, 0).
 * Errors: MD_EINVAL, MD_ESHAPE (M > 64), MD_ENULL, MD_EWORKSPACE. */
int md_series_pade(int m, int L, int M, int64_t count, const double *c, double *p, double *q,
                   void *ws, size_t ws_bytes, int32_t *status, void *stream);

/* Evaluation and reverse-mode differentiation of a system at a series point
 * (Section 4, algorithmic differentiation: all n partial derivatives for a
 * small multiple of the cost of the value).  For each term with factor list
 * v_1..v_D the forward products P_j = v_1 ... v_j, backward products
 * Q_j = v_j ... v_D and cross products C_j = P_{j-1} Q_{j+1} give the value
 * P_D and each partial derivative a_l C_{j*} (j* the first position of x_l,
 * a_l its multiplicity); both are multiplied by c(t) and added into f_i and
 * A_{i,l} in term order.
 * x: planes (2, m, d+1, n) -> f: (2, m, d+1, N), A: (2, m, d+1, N, n)
 * (A_k = coefficient k of the Jacobian series).  Workspace:
 * md_workspace_bytes(MD_FN_EVAL, m, N, n, d, M, max_deg).
 * Errors: MD_EINVAL, MD_ESHAPE, MD_ENULL, MD_EWORKSPACE. */
int md_poly_eval_diff(int m, int d, const md_system *sys, const double *x, double *f, double *A,
                      void *ws, size_t ws_bytes, void *stream);

/* Householder QR of A0 (N x n, N >= n), the one factorisation the block
 * Toeplitz solve needs (Section 4).  A0 = Q R with Q = H_0 ... H_{n-1},
 * H_j = I - beta_j v_j v_j^H on rows j..N-1; for column j with alpha its
 * diagonal entry and sigma its 2-norm from the diagonal down:
 * phi = alpha/|alpha| (1 if alpha = 0), v_j = (phi (|alpha| + sigma), the
 * entries below the diagonal), beta_j = 1/(sigma (sigma + |alpha|)),
 * R_jj = -phi sigma.  Q is never formed.
 * A0: planes (2, m, N, n) row-major; QR: (2, m, N, n) holds R on and above
 * the diagonal and the reflector tails below it; vdiag: (2, m, n) reflector
 * heads; beta: real planes (m, n).  A zero column sets MD_ST_SINGULAR
 * (beta_j = 0, R_jj = 0).  Errors: MD_EINVAL, MD_ESHAPE, MD_ENULL. */
int md_qr(int m, int N, int n, const double *A0, double *QR, double *vdiag, double *beta,
          int32_t *status, void *stream);

/* md_qr with the trailing columns of each column step spread over
 * md_qr_gang_size(m, N, n) workgroups that meet at a barrier in device
 * memory after every step (the factorisation is the same, bit for bit;
 * Section 4).  For one large system a workgroup is one CU's issue rate, so
 * the spread shortens the factorisation (octo double, 64 x 64: the column
 * updates of a step in one round instead of sixteen).  From three limbs on
 * and for 5 <= N <= 64 one workgroup takes each step's look-ahead column
 * and the next reflector on four waves (one real product of each complex
 * product a lane) and the others the remaining columns.  sync: one device
 * int32 the call clears and uses (caller-owned; calls that share it must not
 * overlap).  The workgroups must be resident together: with the GPU full of
 * other work the barriers wait, and after a bounded wait they set
 * MD_ST_GANG in status and the factors are not valid.  Errors as md_qr, and
 * MD_ENULL for a null sync. */
int md_qr_gang(int m, int N, int n, const double *A0, double *QR, double *vdiag, double *beta,
               int32_t *sync, int32_t *status, void *stream);

/* Workgroups md_qr_gang uses for an N x n factorisation (1: it runs as
 * md_qr); 0 for invalid arguments. */
int md_qr_gang_size(int m, int N, int n);

/* Solution of the linearised system A(t) dx(t) = b(t), the block lower
 * triangular Toeplitz system of Section 4, by forward substitution over the
 * degrees: A_0 dx_k = b_k - A_1 dx_{k-1} - ... - A_k dx_0, k = 0..d, each
 * stage solved with the QR factors of A_0 (Q^H, then back substitution with
 * R; least squares in the first n rows when N > n).  The stages run in
 * order; within a stage all right hand side updates r_{k+j} -= A_j dx_k run
 * in parallel.
 * QR, vdiag, beta: outputs of md_qr; A: planes (2, m, d+1, N, n) (the A_0
 * slot is not read); b: (2, m, d+1, N) -> dx: (2, m, d+1, n).  Workspace:
 * md_workspace_bytes(MD_FN_SOLVE, m, N, n, d, 0, 0).  MD_ST_NONFINITE is set
 * when dx holds an infinity or NaN.  Errors: MD_EINVAL, MD_ESHAPE,
 * MD_ENULL, MD_EWORKSPACE. */
int md_series_solve(int m, int N, int n, int d, const double *QR, const double *vdiag,
                    const double *beta, const double *A, const double *b, double *dx, void *ws,
                    size_t ws_bytes, int32_t *status, void *stream);

/* One Newton step on truncated power series (Section 4): evaluate and
 * differentiate the system at x(t), b = -f, solve A(t) dx(t) = b(t) with one
 * QR of A_0 and the staggered substitution, then x(t) += dx(t).
 * x: in/out planes (2, m, d+1, n) with n = sys->n; dx_norm: in/out real
 * planes (m, 2) (may be NULL).  On output it holds
 * [max_i |dx_{d,i}|, max_{k,i} |dx_{k,i}|], the modulus of the update to the
 * last coefficient (Section 6) and the largest update of any coefficient.
 * On input its first entry is the previous step's |dx_d| (as an earlier
 * call wrote it) or zero: when it is positive and this step's |dx_d| is
 * larger, MD_ST_DIVERGED is set (the update grew from one step to the
 * next).  Growth is expected while the t-adic convergence of the series
 * still changes coefficient d (the first ceil(log2(d+1)) + 1 steps) and at
 * the rounding floor; the caller judges the bit with that in mind.
 * Workspace: md_workspace_bytes(MD_FN_NEWTON, m, N, n, d, M, max_deg).
 * Errors: as md_poly_eval_diff and md_series_solve. */
int md_newton_step(int m, int d, const md_system *sys, double *x, double *dx_norm, void *ws,
                   size_t ws_bytes, int32_t *status, void *stream);

/* Newton's method over increasing truncation degrees, as in the experiment
 * of Section 6: for each degree d_j of `degrees` (increasing, at most
 * MD_PROTOCOL_MAX_DEGREES of them) the iterate starts from the given point
 * (x(t) = x0, higher coefficients zero) and takes Newton steps until the
 * modulus of the update to its last coefficient, |dx_{d_j}| = max_i
 * |dx_{d_j,i}|, is at most `tol` (the paper: 1e-32) or maxit[j] steps are
 * done (the paper: 8, 8, 12, 16 for degrees 8, 16, 24, 32).  The test is
 * applied from step min_steps on (2 in the tests: the first step from a
 * constant series reaches only the coefficients its right-hand side has,
 * x_1 when t enters the equations linearly, so its update to x_{d_j} is
 * zero without saying anything about convergence).  A degree that
 * ends with |dx_{d_j}| above `diverge` stops the protocol: the later degrees
 * are not run (the paper's rule that a degree with too large an update ends
 * the computations; the bound is a reading, 1.0 in the tests) and
 * MD_ST_DIVERGED is set.  The decisions are taken on the device: the steps
 * of every degree are enqueued ahead, and each of their kernels returns at
 * once when its degree has converged or was not run, so the call never
 * synchronises and can be captured in a graph.
 * x0: planes (2, m, n) (n = sys->n); degrees, maxit: HOST int32[ndeg];
 * x: planes (2, m, dmax+1, n), dmax = degrees[ndeg-1]: the series of the last
 * degree that ran (zero above that degree); iters: device int32[ndeg], the
 * steps taken at each degree (0 for a degree not run); norms: device real
 * planes (m, ndeg), the last |dx_{d_j}| of each degree (0 if not run).
 * Each degree's steps are md_newton_step's, so its series equals iters[j]
 * calls of md_newton_step from series_start(x0, d_j) bit for bit.
 * Workspace: md_workspace_bytes(MD_FN_PROTOCOL, m, N, n, dmax, M, max_deg).
 * Errors: as md_newton_step; MD_EINVAL for an empty, too long or not
 * increasing degree list, a negative step limit, min_steps < 1, tol < 0 or
 * diverge <= 0. */
#define MD_PROTOCOL_MAX_DEGREES 16
int md_newton_protocol(int m, const md_system *sys, const double *x0, int ndeg,
                       const int32_t *degrees, const int32_t *maxit, int min_steps, double tol,
                       double diverge, double *x, int32_t *iters, double *norms, void *ws,
                       size_t ws_bytes, int32_t *status, void *stream);

/* md_newton_step without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the step's scratch is a fixed device
 * array of MD_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, taken
 * at the first call on each device (the calling thread's current device,
 * which must be the device of `stream`) and held until the process ends.
 * The call allocates and frees nothing.  Arguments, layouts, results and
 * bits are those of md_newton_step.  Every call on one GPU uses that GPU's
 * one array, which keeps the last call's contents (nothing in it needs to
 * start at zero): calls that may overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.
 * Errors: as md_newton_step; MD_EWORKSPACE when the step needs more than
 * MD_NOALLOC_SCRATCH_BYTES (md_workspace_bytes(MD_FN_NEWTON, ...) tells);
 * MD_EHIP when the array's device address cannot be had. */
#define MD_NOALLOC_SCRATCH_BYTES (32u << 20)
int md_newton_step_noalloc(int m, int d, const md_system *sys, double *x, double *dx_norm,
                           int32_t *status, void *stream);

/* Gradient of a real loss L with respect to the series coefficients of the
 * system, through a converged series solution x(t) (the implicit function
 * of the system of Section 4 at its root).  With T(A) the block lower
 * triangular Toeplitz Jacobian of the truncated system in the coefficients
 * of x and G = dL/dRe x + i dL/dIm x, the call solves T(A)^H lambda = G by
 * backward substitution over the degrees (the stages of Section 4 in
 * reverse, with the same single QR of A_0: lambda_k = (R^{-1} Q^H_{0:n})^H
 * times the updated right hand side), then contracts lambda with the
 * monomial series of every term: grad c_{tau,j} =
 * -sum_{k>=j} conj(x^a_{k-j}) lambda_{k,i} for term tau = c_tau x^a of
 * equation i.  The monomial series are either kept from the evaluation
 * pass (store_monomials != 0, M (d+1) more complex numbers of workspace) or
 * recomputed per term inside the contraction (store_monomials == 0).
 * x, grad_x: planes (2, m, d+1, n), device; grad_coef: out, planes
 * (2, 2, M, dc+1) (real/imaginary, the two leading limbs of the m-limb
 * result, term, coefficient), device.  The evaluation runs in m limbs; the
 * gradient is rounded to double double on output.  Workspace:
 * md_workspace_bytes(MD_FN_ADJOINT_STORE or MD_FN_ADJOINT, m, N, n, d, M,
 * max_deg).  N <= 256.  MD_ST_SINGULAR / MD_ST_NONFINITE as md_newton_step.
 * Errors: as md_newton_step; MD_ESHAPE when a term's series exceed 64 KiB
 * of LDS. */
int md_newton_adjoint(int m, int d, const md_system *sys, const double *x, const double *grad_x,
                      int store_monomials, double *grad_coef, void *ws, size_t ws_bytes,
                      int32_t *status, void *stream);

/* Workspace size in bytes for an entry point (fn one of MD_FN_*). */
enum {
  MD_FN_EVAL = 1,
  MD_FN_SOLVE = 2,
  MD_FN_NEWTON = 3,
  MD_FN_ADJOINT = 4,
  MD_FN_ADJOINT_STORE = 5,
  MD_FN_PROTOCOL = 6, /* md_newton_protocol; d is the largest degree */
  MD_FN_PADE = 7      /* md_series_pade: N = denominator degree, n = numerator degree,
                         M = number of series (d and max_deg unused) */
};
size_t md_workspace_bytes(int fn, int m, int N, int n, int d, int M, int max_deg);

/* One multiple-double operation per element, the units of Table 1, for
 * operation-level checks.  Real ops read planes (m, count) and write
 * (m, count); MD_OP_MULD multiplies by b's leading limb; complex ops read
 * and write (2, m, count); MD_OP_CABS2 writes real planes (m, count).
 * b is ignored by MD_OP_SQRT, MD_OP_RSQRT and MD_OP_CABS2. */
enum {
  MD_OP_ADD = 0, MD_OP_SUB = 1, MD_OP_MUL = 2, MD_OP_DIV = 3, MD_OP_SQRT = 4, MD_OP_RSQRT = 5,
  MD_OP_MULD = 6, MD_OP_CADD = 7, MD_OP_CSUB = 8, MD_OP_CMUL = 9, MD_OP_CDIV = 10,
  MD_OP_CABS2 = 11
};
int md_elementwise(int m, int op, int64_t count, const double *a, const double *b, double *out,
                   void *stream);

/* 2-norm sqrt(sum_j |x_j|^2) of a complex vector (Section 2's example: 64
 * unit complex numbers have 2-norm 8).  x: planes (2, m, count), count >= 1;
 * out: real planes (m, 1).  The sum runs over lanes in a fixed tree order. */
int md_norm2(int m, int64_t count, const double *x, double *out, void *stream);

/* ---- batched paths (extension beyond the five entry points) -------------
 *
 * Many independent solution paths in one persistent launch: the paper's job
 * queue (Section 5, Figure 1) with workgroups as workers and one device
 * atomic as the counter; a job is a whole path, `iters` Newton steps run by
 * one workgroup (or a gang of workgroups) with barriers between the stages.
 * The kernel sums its dot products in its own fixed order (more products
 * per lane than md_newton_step), so a batched path agrees with
 * md_newton_step applied `iters` times within the solve's rounding
 * tolerance, not bit for bit; within the batched kernel the order depends
 * only on the path's sizes, so every launch shape, job order, queue layout
 * and gang split gives the same bits.
 *
 * One path, in a device array of md_path (all offsets are element offsets):
 *   m in 1..4 (double to quad double, one kernel), or one of 5, 8, 10
 *   (penta, octo, deca double: a kernel each, 256-thread workgroups): a
 *   launch takes the kernel of its max_m, and a path that kernel does not
 *   carry gets MD_ST_BADPATH; 1 <= n <= N <= 64, d >= 0 (md_newton_batch refuses a
 *   batch whose max_m or max_N is outside these ranges; a path table that
 *   breaks them anyway gets MD_ST_BADPATH for that path, which is then not
 *   run);
 *   eq_ptr, term_ptr, factors: offsets into `ints` (int32) of the path's
 *   system structure, laid out as in md_system (M terms, max_deg factors at
 *   most, coefficient degree dc);
 *   coef: offset into `reals` of the coefficient planes (2, m, M, dc+1);
 *   x: offset into `reals` of the path's series (2, m, d+1, n), in/out;
 *   dx_norm: offset into `reals` of real planes (m, 2) written after the last
 *   step (as md_newton_step's dx_norm);
 *   ws: offset into `ws` (doubles, a multiple of 32) of the path's private
 *   workspace of md_workspace_bytes(MD_FN_NEWTON, m, N, n, d, M, max_deg)
 *   bytes. */
typedef struct md_path {
  int32_t m, N, n, d;
  int32_t M, dc, max_deg, reserved;
  int64_t eq_ptr, term_ptr, factors;
  int64_t coef, x, dx_norm;
  int64_t ws;
} md_path;

/* Dynamic LDS bytes the batched kernel needs: the evaluation's term series
 * (2 max_m term_lds_series(max_deg) (max_d+1) eval_waves doubles), at least
 * one dx_k of 64 unknowns (2 max_m 64 doubles); 0 for invalid arguments. */
size_t md_batch_lds_bytes(int max_m, int max_d, int max_deg, int eval_waves);

/* Runs `iters` Newton steps on each of `npaths` paths in one persistent
 * launch.  paths: device md_path[npaths].  Jobs: device int32[2*njobs],
 * job j = (path, (G << 8) | member): a path is run by G workgroups (a gang,
 * 1 <= G <= 32, members 0..G-1, one job each, consecutive in one queue).
 * nq queues: queue q holds jobs qbegin[q]..qbegin[q+1]-1 (device
 * int32[nq+1]) and is served, in order, by the workgroups running on
 * accelerator die q (md_device_dies); with nq == 1 every workgroup serves
 * the one queue.  Every queue needs at least as many resident workgroups
 * as its largest gang.  counters: device int32[nq],
 * gang_ctr: device int32[npaths], both scratch that the call resets on the
 * stream (so the call can be captured in a graph and replayed).  status:
 * device int32[npaths], MD_ST_* bits per path (cleared by the caller; the
 * call sets MD_ST_NOTRUN first and clears it when the path is done).
 * max_m, max_N, max_d, max_deg: maxima over the paths (host values; max_m
 * in 1..4 or one of 5, 8, 10, max_N at most 64, and max_d, max_deg size
 * the LDS);
 * grid: the number of persistent workgroups (each queue needs as many
 * resident workgroups on its die as its largest gang); block: threads per
 * workgroup, 256 or 512 (256 when max_m >= 5); eval_waves (1..block/64):
 * waves per workgroup that
 * evaluate terms; path_clock (may be NULL): device int64[2*npaths],
 * receives for every path the device wall clock (md_wall_clock_hz ticks per
 * second) when its member 0 took it and when it finished; phase_clock (may
 * be NULL): device int64[8*npaths], zeroed by the caller, to which member 0
 * adds the wall-clock ticks of each phase of every step: [0] evaluation of
 * the terms, [1] sums into f and A, [2] QR of A_0, [3] R^{-1} Q^H, [4] the
 * staggered stages, [5] the update of x (slots 6, 7 unused).
 * Errors: MD_EINVAL (max_m not in 1..4, 5, 8, 10; block 512 with max_m >= 5;
 * among others), MD_ENULL, MD_ESHAPE
 * (max_N outside 1..64, or LDS above md_device_lds_bytes()), MD_EHIP. */
int md_newton_batch(int npaths, const md_path *paths, int njobs, const int32_t *jobs, int nq,
                    const int32_t *qbegin, const int32_t *ints, double *reals, double *ws,
                    int iters, int32_t *counters, int32_t *gang_ctr, int32_t *status, int max_m,
                    int max_N, int max_d, int max_deg, int grid, int block, int eval_waves,
                    int64_t *path_clock, int64_t *phase_clock, void *stream);

/* Section 6's protocol (as md_newton_protocol) for every path of a batch in
 * one persistent launch, with per-path decisions taken on the device: each
 * path runs the listed degrees that are at most its own d, each from its
 * start point (coefficient 0 of its x on entry), with steps until
 * |dx_{d_j}| <= tol (from step min_steps on) or maxit[j] steps, and stops
 * after a degree that ends with |dx_{d_j}| above `diverge` (MD_ST_DIVERGED
 * for that path).  A gang's members share each decision through the path's
 * workspace.  Carries double to quad double (max_m <= 4).  Arguments as
 * md_newton_batch, except: proto (host): the protocol; each path's
 * workspace slice holds md_workspace_bytes(MD_FN_PROTOCOL, m, N, n, d, M,
 * max_deg) bytes; x ends with the series of the path's last degree that ran
 * (zero above it); proto_iters: device int32[npaths*ndeg], the steps per
 * degree (0 when not run); proto_norms: device double[npaths*ndeg*10], the
 * last |dx_{d_j}| of each degree as up to 10 limbs (zeros beyond m and for
 * degrees not run).  The dx_norm slots of the paths are not written. */
typedef struct md_protocol {
  int32_t ndeg;                              /* 1..MD_PROTOCOL_MAX_DEGREES */
  int32_t min_steps;                         /* >= 1 */
  int32_t degrees[MD_PROTOCOL_MAX_DEGREES];  /* increasing, >= 0 */
  int32_t maxit[MD_PROTOCOL_MAX_DEGREES];    /* 0..10000 */
  double tol, diverge;                       /* >= 0, > 0 */
} md_protocol;

int md_newton_batch_protocol(int npaths, const md_path *paths, int njobs, const int32_t *jobs,
                             int nq, const int32_t *qbegin, const int32_t *ints, double *reals,
                             double *ws, const md_protocol *proto, int32_t *counters,
                             int32_t *gang_ctr, int32_t *status, int max_m, int max_N, int max_d,
                             int max_deg, int grid, int block, int eval_waves, int32_t *proto_iters,
                             double *proto_norms, void *stream);

/* Writes, for each of nblocks workgroups of a small launch, the accelerator
 * die (XCC) it ran on: device int32[nblocks].  The queues of
 * md_newton_batch are indexed by these ids.  Errors: MD_ENULL, MD_EINVAL,
 * MD_EHIP. */
int md_device_dies(int32_t *ids, int nblocks, void *stream);

/* Largest dynamic LDS in bytes that the kernels may take on the current
 * device (the per-workgroup limit less 4 KiB for static LDS); bounds
 * md_batch_lds_bytes for md_newton_batch. */
size_t md_device_lds_bytes(void);

/* Ticks per second of the device wall clock that md_newton_batch records,
 * for `device`.  Errors: MD_ENULL, MD_EHIP. */
int md_wall_clock_hz(int device, int64_t *hz);

/* Message for the last error returned on this thread ("" if none). */
const char *md_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MDSERIES_H */
