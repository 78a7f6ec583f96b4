/*
 * dna.h -- C ABI of libdna: the Diagonalized Newton Algorithm (DNA) for
 * non-negative matrix factorisation under the Kullback-Leibler divergence
 * (H. Van hamme, "The Diagonalized Newton Algorithm for Non-negative Matrix
 * Factorization"), as HIP kernels for gfx950 (MI355X).
 *
 * Problem (Sec. 1, eq. 1): V (N x T) ~ W H with W (N x R), H (R x T), all
 * entries >= 0, cost d_KL(V, WH) = sum v log(v/z) - sum v + sum z, Z = W H.
 * With regularisation weights rho, lambda >= 0 (dna_opts) the cost is eq. (2),
 * d_KL(V, WH) + rho sum w + lambda sum h; rho = lambda = 0 is the setting of
 * Sec. 4 and the default.
 *
 * Conventions shared by every entry point
 *  - Matrices are float32, row-major and contiguous: V[N][T], W[N][R],
 *    H[R][T].  Every matrix pointer is DEVICE memory owned by the caller.
 *  - Scalars/vectors named d_*, margin, out are device float64 buffers;
 *    chose_newton masks are device uint8 buffers (1 = Newton candidate).
 *  - `ws` is a caller-owned device workspace of at least the number of bytes
 *    the matching *_workspace_bytes() function returns; the library never
 *    allocates, frees or synchronises (except in checked mode, below).
 *  - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *    enqueued on it; calls return before the GPU finishes.
 *  - Arguments are validated on the host before anything is enqueued; an
 *    invalid call returns a status != DNA_OK and enqueues nothing.
 *  - A kernel launch failure returns DNA_EHIP; dna_last_error() gives the
 *    HIP error text (thread-local).  No C++ exception crosses this ABI.
 *  - Output buffers overlap neither the inputs nor each other nor `ws`; the
 *    factor an update, normalisation or unrolled solve rewrites in place is
 *    the one exception.
 *  - Zeros of V contribute nothing to Q, Q-bar or any cost (end of Sec. 3).
 *  - Results are deterministic: every reduction runs in a fixed order.
 */
#ifndef DNA_H_
#define DNA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DNA_OK = 0,
  DNA_EINVAL = 1,       /* null pointer, non-positive size, bad option value  */
  DNA_EWORKSPACE = 2,   /* workspace smaller than *_workspace_bytes()         */
  DNA_EDOMAIN = 3,      /* checked mode: negative entry, zero W column / H row
                           sum, or z = 0 where v > 0 (Sec. 2 assumes nonzero
                           column sums)                                         */
  DNA_ENONFINITE = 4,   /* checked mode: NaN or Inf in an input                */
  DNA_EHIP = 5,         /* HIP runtime or launch error                         */
  DNA_EUNSUPPORTED = 6  /* valid request this library does not implement       */
} dna_status;

/* Operand type of the matrix products (the accumulation is always float32 and
 * every cost sum is float64).  The 16-bit types apply to the three products of
 * the DNA half-steps (Z = W H with its ratio epilogue, the gradient / Hessian
 * products, the candidate-cost reconstructions) in dna_update_H/W,
 * dna_gradient_hessian, dna_candidates and dna_select.  Inputs and outputs stay
 * float32 in HBM; operands are rounded to 16 bits when staged.  BF16 rounds
 * directly; FP16 first applies power-of-two scales (per rank component from the
 * W column / H row maxima, per column or row of Q, Q - 1 and Q-bar from a max
 * pass, or inside dna_iterate after its first half step from bounds that the
 * preceding cost pass leaves) that are undone in float32, so FP16 neither
 * overflows nor flushes to zero where the fp32 values are normal.  The candidates, the selection sums
 * and the update itself stay in float32 / float64.  dna_mu_update and
 * dna_kl_cost ignore the field (float32 products); the unrolled adjoint returns
 * DNA_EUNSUPPORTED for 16-bit types. */
typedef enum {
  DNA_GEMM_FP32 = 0,
  DNA_GEMM_BF16 = 1,
  DNA_GEMM_FP16 = 2
} dna_gemm_type;

typedef struct {
  float eps;     /* floor of the multiplicative Newton gain, eq. (15); Sec. 4: 0.01 */
  float alpha;   /* ceiling: additive Newton step <= alpha*x, eq. (17); Sec. 4: 4   */
  int gemm;      /* dna_gemm_type                                                  */
  int checked;   /* 1: device-side domain checks, then a stream synchronise and a
                    read-back of the check flags (tests and debugging only)        */
  float rho;     /* eq. (2) weight of sum w (W half-steps, normalisations); >= 0   */
  float lambda;  /* eq. (2) weight of sum h (H half-steps, normalisations); >= 0   */
  int select;    /* dna_select_rule: how each half-step picks its candidate         */
} dna_opts;

/* The selection of steps 7-9, 12-15 (H step; 20-22, 25-28 W step).
 * DNA_SELECT_BOTH (Algorithm 1): cost both candidates, keep Newton iff
 *   d_DNA < d_MU.
 * DNA_SELECT_NEWTON_FIRST (Sec. 5's "more refined step damping", which the
 *   paper names as its next step without a method; this is the reading built
 *   here): cost the Newton candidate only and keep it iff its column's (row's)
 *   eq. (5) objective d_DNA is not above the current state's,
 *   d_cur + sum_r c_r x_r - sum v (c including lambda, or g including rho),
 *   with d_cur formed in the ratio pass; else keep the MU candidate, which
 *   never raises it (Sec. 2.1), uncosted.  One reconstruction product per
 *   half-step instead of two.  The cost never rises.  Outputs: d_sel is NaN
 *   where MU is kept; margin = current objective - Newton objective.
 *   Supported by dna_update_H/W and dna_iterate with FP32 products and
 *   R <= 64 (DNA_EUNSUPPORTED otherwise, and from dna_select, the sparse calls
 *   and the unrolled adjoint). */
typedef enum {
  DNA_SELECT_BOTH = 0,
  DNA_SELECT_NEWTON_FIRST = 1
} dna_select_rule;

/* eps = 0.01, alpha = 4 (Sec. 4), FP32 products, unchecked, rho = lambda = 0,
 * DNA_SELECT_BOTH. */
void dna_default_opts(dna_opts* opts);

/* Bytes of workspace any call below needs for an N x T x R problem with these
 * options (one size serves every entry point except the unrolled adjoint).
 * Returns 0 for non-positive sizes. */
size_t dna_workspace_bytes(int64_t N, int64_t T, int64_t R, const dna_opts* opts);

/* Algorithm 1 steps 1, 16, 29: rescale column r of W and row r of H by
 * reciprocal factors, so W H is unchanged.  At rho = lambda = 0:
 *   side 0 (steps 1, 29): divide column r of W by its sum, multiply row r of H
 *                         by the same number.
 *   side 1 (step 16):     divide row r of H by its sum, multiply column r of W
 *                         by the same number.
 * With regularisation (eq. 2; the printed steps add lambda or rho to the sums,
 * which neither yields the unit scale the rest of the algorithm assumes nor
 * keeps eq. 2 from rising, since the penalty depends on how scale is split
 * between W and H):
 *   rho > 0, lambda > 0: either side multiplies column r of W by
 *     s_r = sqrt(lambda G_r / (rho C_r)) and divides row r of H by it
 *     (C = W^t 1, G = H 1): the split minimising rho sum w + lambda sum h, after
 *     which rho C_r = lambda G_r;
 *   lambda > 0 only: either side acts as side 0 (the unpenalised W keeps unit
 *     column sums; eq. 2 has no minimiser otherwise);
 *   rho > 0 only: either side acts as side 1.
 * W and H are updated in place.  A zero sum leaves that column/row unchanged
 * (checked mode reports it as DNA_EDOMAIN). */
dna_status dna_normalize(int side, float* W, float* H, int64_t N, int64_t T, int64_t R,
                         const dna_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* One DNA update of H with W fixed: Algorithm 1 steps 4-15 (Sec. 2-3).
 *   c = W^t 1 + lambda;  Z = W H;  Q = V/Z;  Q-bar = V/Z^2         (steps 2-3, 10)
 *   A = W^t Q / c - 1            eq. (7), step 5
 *   B = (W*W)^t Q-bar / c        eq. (14), step 10
 *   MU candidate     H (1 + A)                                      eq. (11), step 6
 *   Newton candidate a < 0:  h max(hb/(hb - a), eps)                eq. (15)
 *                    a >= 0: h + min(a/b, alpha h)                  eq. (17)
 *                    then each column scaled so sum_r c_r h_r = sum_n v_n  eq. (10)
 *   per column t: d_MU, d_DNA = sum_{v>0} v log(v/z) of each candidate  steps 9, 14
 *   H[:, t] <- Newton candidate iff d_DNA < d_MU, else MU            step 15
 * Both candidates satisfy sum_r c_r h_r = sum_n v_n (eq. 9), so with lambda > 0
 * the selection on d is also the selection on the regularised column cost.
 * H (R x T) is overwritten.  Optional outputs (NULL to skip), length T:
 *   chose_newton[t] (uint8), d_sel[t] = cost of the kept candidate,
 *   margin[t] = d_MU - d_DNA (computed directly from W (H_MU - H_DNA), so it
 *   resolves differences far below the size of the costs). */
dna_status dna_update_H(const float* V, const float* W, float* H,
                        int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                        void* ws, size_t ws_bytes, uint8_t* chose_newton,
                        double* d_sel, double* margin, void* stream);

/* One DNA update of W with H fixed: Algorithm 1 steps 17-28, the mirror of
 * dna_update_H on the transposed problem (Sec. 2: d(V, WH) = d(V^t, H^t W^t)).
 * g = H 1 + rho replaces c; rows of W replace columns of H; each Newton row n
 * is scaled so that sum_r g_r w_nr = sum_t v_nt.  W (N x R) is overwritten;
 * optional outputs have length N. */
dna_status dna_update_W(const float* V, float* W, const float* H,
                        int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                        void* ws, size_t ws_bytes, uint8_t* chose_newton,
                        double* d_sel, double* margin, void* stream);

/* `iters` full iterations of Algorithm 1 in place, each: dna_update_H
 * (steps 4-15), dna_normalize(1) (step 16), dna_update_W (steps 17-28),
 * dna_normalize(0) (step 29) -- the same kernels those entry points run, in one
 * call, with the normalisations chosen by rho and lambda as in dna_normalize.  Each normalisation also writes the partial sums of the factor it
 * rescaled, so the half-step that follows reads c = W^t 1 (or g = H 1) from
 * them instead of summing the factor again; results therefore equal those of
 * the four separate calls up to the order of those float64 sums.  Step 1 (the
 * initial dna_normalize(0)) is the caller's.  iters = 0 does nothing;
 * iters < 0 is DNA_EINVAL.  Uses the dna_workspace_bytes() workspace. */
dna_status dna_iterate(const float* V, float* W, float* H,
                       int64_t N, int64_t T, int64_t R, int iters,
                       const dna_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): dna_iterate on a scratch
 * array of DNA_NOALLOC_SCRATCH_BYTES that the library itself holds, one per GPU,
 * from the library's load until the process ends.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine); the caller passes only
 * the inputs and outputs, which are those of dna_iterate, and the current
 * device's array is used (`stream` must belong to the current device).
 * Problems whose dna_workspace_bytes() exceeds DNA_NOALLOC_SCRATCH_BYTES return
 * DNA_EUNSUPPORTED before anything is enqueued (dna_last_error() gives both
 * sizes).  Every call on one GPU shares that GPU's array and leaves its contents
 * behind; calls that overlap on one GPU (concurrent streams or host threads)
 * race on it and must be serialised by the caller.  Results equal dna_iterate's
 * on the same inputs. */
#define DNA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dna_status dna_iterate_noalloc(const float* V, float* W, float* H,
                               int64_t N, int64_t T, int64_t R, int iters,
                               const dna_opts* opts, void* stream);

/* ---- Sparse V (Sec. 4.2: term-document matrices with 0.2-0.35% nonzeros) ---
 * Only the nonzeros of V enter Q, Q-bar and the costs (end of Sec. 3), so the
 * O(NRT) products become O(nnz R) gathers.  V is described by its nonzeros (all
 * values > 0) in two orders plus segment tables; every array is device memory
 * owned by the caller (int32 indices, float32 values); the struct itself is a
 * host object:
 *   col_idx, val, row_of  [nnz]  CSR order (rows ascending, columns ascending
 *                                within a row): column, value and row of each entry
 *   csc_row, csc_col, csc_pos [nnz]  the same entries in CSC order (columns
 *                                ascending): row, column, and position in the
 *                                CSR arrays
 *   segr_start [nseg_r + 1], segr_ptr [N + 1]  the CSR positions cut into
 *                                segments of at most 64 entries of one row
 *                                (segr_start ascending from 0, last = nnz); row n
 *                                owns segments segr_ptr[n] .. segr_ptr[n+1] - 1
 *   segc_start [nseg_c + 1], segc_ptr [T + 1]  the same for the CSC positions
 *                                and the columns.
 * The Python binding builds all of them from a COO or CSR matrix.  An index out
 * of range is clamped in the kernels (wrong numbers, never an out-of-bounds
 * access); checked mode additionally rejects non-finite or negative values.
 * FP32 products only (opts->gemm must be DNA_GEMM_FP32), R <= 256, nnz < 2^31. */
typedef struct {
  int64_t nnz;
  const int32_t* col_idx;
  const float* val;
  const int32_t* row_of;
  const int32_t* csc_row;
  const int32_t* csc_col;
  const int32_t* csc_pos;
  int64_t nseg_r, nseg_c;
  const int32_t* segr_start;
  const int32_t* segr_ptr;
  const int32_t* segc_start;
  const int32_t* segc_ptr;
} dna_sparse_v;

/* Workspace for the dna_sparse_* calls below (0 on invalid sizes). */
size_t dna_sparse_workspace_bytes(int64_t N, int64_t T, int64_t R, const dna_sparse_v* V, const dna_opts* opts);

/* dna_update_H / dna_update_W (Algorithm 1 steps 4-15 / 17-28) with a sparse
 * V: the same candidates (eq. 7, 11, 14, 15, 17, 10), the same costs over the
 * nonzeros and the same selection, with the same optional outputs.  The
 * gradient sum u_c = sum_n w_nr (q_nt - 1) takes the zeros of V as q = 0: it is
 * formed as the sum over the nonzeros minus (c_r - sum of w_nr over them). */
dna_status dna_sparse_update_H(const dna_sparse_v* V, const float* W, float* H,
                               int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                               void* ws, size_t ws_bytes, uint8_t* chose_newton,
                               double* d_sel, double* margin, void* stream);
dna_status dna_sparse_update_W(const dna_sparse_v* V, float* W, const float* H,
                               int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                               void* ws, size_t ws_bytes, uint8_t* chose_newton,
                               double* d_sel, double* margin, void* stream);

/* eq. 1 with a sparse V: sum over the nonzeros of v log(v/z) - v, plus
 * sum z = sum_r c_r (H 1)_r in closed form; with rho or lambda > 0 also
 * rho sum w + lambda sum h (eq. 2).  out: one device double. */
dna_status dna_sparse_kl_cost(const dna_sparse_v* V, const float* W, const float* H,
                              int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                              void* ws, size_t ws_bytes, double* out, void* stream);

/* mu_update (eq. 11) with a sparse V, without the cost output:
 * side 0: H <- H * (W^t Q) / (W^t 1 + lambda); side 1: W <- W * (Q H^t) /
 * (H 1 + rho), Q at the nonzeros only. */
dna_status dna_sparse_mu_update(int side, const dna_sparse_v* V, float* W, float* H,
                                int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                                void* ws, size_t ws_bytes, void* stream);

/* `iters` MU iterations with a sparse V in place (the steps of mu_iterate).
 * iters < 0: DNA_EINVAL. */
dna_status dna_sparse_mu_iterate(const dna_sparse_v* V, float* W, float* H,
                                 int64_t N, int64_t T, int64_t R, int iters,
                                 const dna_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* `iters` full iterations (dna_sparse_update_H, dna_normalize(1),
 * dna_sparse_update_W, dna_normalize(0)) in place.  As in dna_iterate, each
 * normalisation hands the partial sums of the factor it rescaled to the next
 * half-step when they are that step's divisor.  As Algorithm 1 does (steps 15,
 * 28), each half-step after the first takes Z at the nonzeros from the
 * candidate the preceding selection kept (the normalisation between leaves
 * W H unchanged) instead of forming it again from the factors.  Results equal
 * the separate calls up to float rounding.  iters < 0: DNA_EINVAL. */
dna_status dna_sparse_iterate(const dna_sparse_v* V, float* W, float* H,
                              int64_t N, int64_t T, int64_t R, int iters,
                              const dna_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* Plain multiplicative update (eq. 11; Lee-Seung at rho = lambda = 0):
 *   side 0: H <- H * (W^t Q) / (W^t 1 + lambda)
 *   side 1: W <- W * (Q H^t) / (H 1 + rho)
 * with Q = V / (W H).  If with_cost != 0, d_out (length T for side 0, N for
 * side 1) receives sum_{v>0} v log(v/z) per column (row) of the INPUT state,
 * computed from the same Z ("MU with cost", Table 1); otherwise d_out is
 * ignored and no logarithm is evaluated ("MU without cost"). */
dna_status mu_update(int side, const float* V, float* W, float* H,
                     int64_t N, int64_t T, int64_t R, int with_cost, double* d_out,
                     const dna_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* `iters` MU iterations in place: mu_update(0), dna_normalize(1),
 * mu_update(1), dna_normalize(0) per iteration (the MU-labelled steps of
 * Algorithm 1).  with_cost != 0 also forms each half-step's per-column / per-row
 * cost of its input state ("MU with cost", Table 1) in the workspace; it is not
 * returned.  iters < 0: DNA_EINVAL. */
dna_status mu_iterate(const float* V, float* W, float* H,
                      int64_t N, int64_t T, int64_t R, int iters, int with_cost,
                      const dna_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* Eq. (1): *out = sum_{v>0} v log(v/z) - sum v + sum z with Z = W H, written
 * to one device double; with rho or lambda > 0, eq. (2): that plus
 * rho sum w + lambda sum h. */
dna_status kl_cost(const float* V, const float* W, const float* H,
                   int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                   void* ws, size_t ws_bytes, double* out, void* stream);

/* ---- Stages of one half-step (the same kernels dna_update_* runs) -------- */

/* Steps 2-5 and 10: A and B of eq. (7) and eq. (14) (c = W^t 1 + lambda).
 * side 0: A_out, B_out are R x T;  side 1: N x R (A = Q H^t / g - 1,
 * B = Q-bar (H*H)^t / g, g = H 1 + rho). */
dna_status dna_gradient_hessian(int side, const float* V, const float* W, const float* H,
                                int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                                float* A_out, float* B_out,
                                void* ws, size_t ws_bytes, void* stream);

/* Steps 2-6, 10-11: the MU candidate and the renormalised Newton candidate.
 * side 0: X_mu, X_newton are R x T (candidates for H); side 1: N x R. */
dna_status dna_candidates(int side, const float* V, const float* W, const float* H,
                          int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                          float* X_mu, float* X_newton,
                          void* ws, size_t ws_bytes, void* stream);

/* Steps 7-9, 12-15 given both candidates: per-column (side 0) or per-row
 * (side 1) costs, selection and the kept factor written to X_out.
 * F is the fixed factor (W for side 0, H for side 1).  rho and lambda do not
 * enter (the selection compares the log-ratio sums only). */
dna_status dna_select(int side, const float* V, const float* F,
                      const float* X_mu, const float* X_newton, float* X_out,
                      int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                      uint8_t* chose_newton, double* d_sel, double* margin,
                      void* ws, size_t ws_bytes, void* stream);

/* ---- Differentiable unrolled H-solve (K DNA H-updates with W fixed) ------ */
/* lambda != 0 returns DNA_EUNSUPPORTED from both calls (rho does not enter). */

/* Workspace for the two calls below (larger than dna_workspace_bytes). */
size_t dna_unrolled_workspace_bytes(int64_t N, int64_t T, int64_t R, const dna_opts* opts);

/* Forward: H_ckpt[0] = H_init, H_ckpt[k+1] = dna_update_H(H_ckpt[k]) for
 * k < K; sel_ckpt[k][t] is that update's selection.  H_ckpt is
 * [K+1][R][T] float32, sel_ckpt [K][T] uint8, both device. */
dna_status dna_unrolled_H_fwd(const float* V, const float* W, const float* H_init, int K,
                              int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                              float* H_ckpt, uint8_t* sel_ckpt,
                              void* ws, size_t ws_bytes, void* stream);

/* Backward: given dH_K = dL/dH_K, the vector-Jacobian product through the K
 * updates with each selection frozen at its forward value and each entry
 * differentiated along the branch it took (a < 0 or a >= 0, floor, cap).
 * Writes dW (N x R) and dV (N x T), and dH_init (R x T) unless NULL; all three
 * are overwritten.  Requires z = (W H_k)_nt > 0 everywhere; the gradient with
 * respect to v at v = 0 is that of the expressions v/z, v/z^2. */
dna_status dna_unrolled_H_bwd(const float* V, const float* W, const float* H_ckpt,
                              const uint8_t* sel_ckpt, int K,
                              int64_t N, int64_t T, int64_t R, const float* dH_K,
                              float* dW, float* dV, float* dH_init, const dna_opts* opts,
                              void* ws, size_t ws_bytes, void* stream);

/* Kept sums (for callers with memory to spare; the gradients are the same).
 * The backward above recomputes, for every update k, Z = W H_k, Q, Q-bar and
 * the sums u, u_c, y of eq. 7 and 14 (two products per update).  The _aux
 * variants instead have the forward keep them in a caller-owned device
 * buffer `aux` of dna_unrolled_aux_bytes(N, T, R, K, opts) bytes (256-byte
 * aligned; per update 3 N T + 3 s R T floats, s the split count of the
 * product), which the backward reads: the backward then skips both products.
 * The bytes are 0 for R <= 64 (there the recompute is one fused pass) and the
 * _aux calls then behave as the plain ones, `aux` unused (it may be NULL).
 * The buffer must hold, unmodified, what the _aux forward of the same V, W,
 * H_init, K and opts wrote when the _aux backward reads it; it is the
 * caller's.  Errors: DNA_EWORKSPACE if aux_bytes is too small, DNA_EINVAL if
 * aux is misaligned, otherwise as the plain calls. */
size_t dna_unrolled_aux_bytes(int64_t N, int64_t T, int64_t R, int K, const dna_opts* opts);

dna_status dna_unrolled_H_fwd_aux(const float* V, const float* W, const float* H_init, int K,
                                  int64_t N, int64_t T, int64_t R, const dna_opts* opts,
                                  float* H_ckpt, uint8_t* sel_ckpt,
                                  void* ws, size_t ws_bytes, void* aux, size_t aux_bytes, void* stream);

dna_status dna_unrolled_H_bwd_aux(const float* V, const float* W, const float* H_ckpt,
                                  const uint8_t* sel_ckpt, int K,
                                  int64_t N, int64_t T, int64_t R, const float* dH_K,
                                  float* dW, float* dV, float* dH_init, const dna_opts* opts,
                                  void* ws, size_t ws_bytes, const void* aux, size_t aux_bytes,
                                  void* stream);

/* ---- Diagnostics ---------------------------------------------------------- */

const char* dna_status_string(dna_status s);
const char* dna_last_error(void);

/* Kernel timing: while enabled, every kernel the library launches is bracketed
 * by hipEvents on its stream.  dna_profile_read() synchronises those events and
 * fills up to max_entries records (one per kernel name, aggregated over
 * launches since the last reset), returning how many exist. */
typedef struct {
  const char* name;
  int64_t launches;
  double total_ms;
} dna_kernel_stat;

void dna_profile_enable(int on);
void dna_profile_reset(void);
int dna_profile_read(dna_kernel_stat* out, int max_entries);

/* Library build identification (gfx target and compile options). */
const char* dna_build_info(void);

#ifdef __cplusplus
}
#endif

#endif /* DNA_H_ */
