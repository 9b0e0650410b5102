/*
 * qtx_rgf.h - batched recursive Green's function (RGF) selected inversion of
 * block-tridiagonal complex systems on AMD Instinct MI355X (gfx950).
 *
 * The library solves, independently at every energy E, the system of the
 * NEGF+GW paper (arXiv 2508.19138, Eq. system-solve):
 *
 *     Mt(E) X^R(E) = I,        Mt(E) X^s(E) Mt(E)^dagger = B^s(E),  s in {<,>}
 *
 * and returns the "selected" blocks of the solution: the diagonal and first
 * off-diagonal blocks of X^R, X^< and X^> (Sec. 3.2, Selected System Solver).
 * The system matrices are those of Table "quantities" / Sec. 3.2.2:
 *
 *   G-type (electrons):        Mt = E S - H - Sigma^R(E),   B^s = Sigma^s(E)
 *   W-type (screened Coulomb): Mt = I - V P^R(E),           B^s = V P^s(E) V^dagger
 *
 * For W the products are formed in block-tridiagonal (BT) form and cut back
 * to the BT pattern (blocks with |i-j| > 1 dropped).  The solve is the RGF
 * forward/backward recursion of Sec. 3.2.3 (Eqs. forward-pass, backward-pass).
 *
 * Data layout (all operands): complex128 blocks, interleaved (re, im), each
 * block row-major b x b and contiguous.  A block-tridiagonal operand is three
 * arrays: diag [n][b][b], upper [n-1][b][b] (block (i,i+1)) and
 * lower [n-1][b][b] (block (i+1,i)).  Energy-dependent operands carry a
 * leading energy axis: diag [N_E][n][b][b], upper/lower [N_E][n-1][b][b].
 * Energy-independent operands (H, S, V) have no energy axis.
 *
 * Pointers: every array pointer is a HIP device pointer to memory the caller
 * owns (for example a PyTorch complex128 tensor's data_ptr()).  The library
 * never frees, reallocates or retains caller memory beyond the call.  The
 * energies array is a host pointer.
 *
 * Symmetry contract: the paper's lesser/greater quantities are
 * anti-Hermitian, B^s_ij = -conj(B^s_ji).  The library relies on it: for
 * Sigma^s and P^s it reads the diagonal and upper blocks only (the lower
 * block is taken as -upper^dagger; a lower pointer given there is ignored),
 * and it writes the lower blocks of X^s as -upper^dagger.
 *
 * Errors: every entry point returns a qtx_status.  Call-level errors
 * (bad arguments, HIP failures, out of memory) are returned directly and no
 * problem is solved.  Numerical failures are per problem: the call returns
 * QTX_ERR_PROBLEM and each problem's `status` field says what happened
 * (QTX_ERR_SINGULAR: an exactly zero pivot; QTX_ERR_NOT_FINITE: a NaN or
 * Inf pivot), with the first failing energy and block index; the other
 * problems of the batch are unaffected.  Outputs of a failing energy are
 * unspecified.  No C++ exception crosses this interface.
 *
 * Threading: a context may be used by one host thread at a time.  The
 * request loop (qtx_rgf_submit) runs on a thread of its own with its own
 * streams and workspace; solve_batch and the request loop of one context may
 * run at the same time.
 *
 * Environment (read at qtx_rgf_create): QTX_STREAMS (1..8, default 4) sets
 * the number of streams over which a batch's lane classes are spread;
 * QTX_SPLIT (1..8, default 1) the number of streams a problem of 64 or more
 * energies is split over;
 * QTX_GRAPHS=0 disables graph capture of repeated launch segments;
 * QTX_TUNE=0 disables the tile autotuner; QTX_TUNE_CACHE names its cache
 * file; QTX_GEMM_CFG, QTX_BATCH_CLASS and QTX_SERVE_CLASS override the tile
 * and the grouping of lanes into classes (for experiments).  Results do not
 * depend on any of them.
 */
#ifndef QTX_RGF_H
#define QTX_RGF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qtx_rgf_ctx qtx_rgf_ctx;

typedef enum {
  QTX_OK = 0,
  QTX_ERR_INVALID_ARG = 1, /* null/negative/inconsistent argument          */
  QTX_ERR_SINGULAR = 2,    /* exactly zero pivot in a diagonal-block inverse */
  QTX_ERR_NOT_FINITE = 3,  /* NaN or Inf met as a pivot                      */
  QTX_ERR_NOMEM = 4,       /* one energy of one problem exceeds the budget   */
  QTX_ERR_HIP = 5,         /* a HIP runtime call failed                      */
  QTX_ERR_BUSY = 6,        /* context in use                                 */
  QTX_ERR_PROBLEM = 7      /* call done; at least one problem status != OK  */
} qtx_status;

typedef enum { QTX_KIND_G = 0, QTX_KIND_W = 1 } qtx_kind;

/* QTX_FP64: every product and inverse in complex128.
 * QTX_MIXED: the Schur-update products and all lesser/greater triple
 * products in complex64 on the FP32 matrix cores (FP32 accumulate); the
 * diagonal-block inverses and the left-connected x^R_i stay complex128. */
typedef enum { QTX_FP64 = 0, QTX_MIXED = 1 } qtx_precision;

/* One block-tridiagonal input operand (device pointers, see layout above). */
typedef struct {
  const void* diag;
  const void* upper;
  const void* lower;
} qtx_bt_in;

/* One block-tridiagonal output: [N_E][n][b][b] and [N_E][n-1][b][b]. */
typedef struct {
  void* diag;
  void* upper;
  void* lower;
} qtx_bt_out;

typedef struct {
  int32_t kind;        /* qtx_kind                                           */
  int32_t precision;   /* qtx_precision                                      */
  int32_t n_blocks;    /* n >= 1                                             */
  int32_t block_size;  /* 1 <= b <= 4096                                     */
  int32_t n_energies;  /* N_E >= 1                                           */
  int32_t flags;       /* reserved, must be 0                                */
  const double* energies; /* host, [N_E] real energies (G-type; W ignores)   */

  /* G-type inputs.  H: energy independent, Hermitian; H.lower NULL means
   * lower = upper^dagger (the library may read either coupling block
   * through the adjoint of the other, so a non-Hermitian H is not
   * supported).  S: energy independent overlap; S.diag NULL means
   * S = I (then S.upper/S.lower must be NULL); S.upper/lower NULL = zero.
   * sigma_r: retarded self-energy (scattering + OBC), per energy; upper and
   * lower NULL = zero blocks.  sigma_l / sigma_g: Sigma^< / Sigma^>, per
   * energy, anti-Hermitian; upper NULL = block-diagonal. */
  qtx_bt_in H, S, sigma_r, sigma_l, sigma_g;

  /* W-type inputs.  V: energy independent, Hermitian (lower NULL =
   * upper^dagger).  P_r: retarded polarization per energy (upper/lower NULL
   * = zero).  P_l / P_g: P^< / P^> per energy, anti-Hermitian (upper NULL =
   * block-diagonal). */
  qtx_bt_in V, P_r, P_l, P_g;

  /* Outputs (device).  XR is required.  XL / XG: diag NULL skips that
   * right-hand side altogether; upper/lower may be NULL to skip those
   * blocks.  For W-type the X^s are W^< and W^>. */
  qtx_bt_out XR, XL, XG;
  /* W-type only, optional: diagonal blocks of W^R = X^R V, [N_E][n][b][b]. */
  void* WR_diag;

  /* Written by the library. */
  int32_t status;       /* qtx_status of this problem                        */
  int32_t fail_energy;  /* first failing energy index, or -1                 */
  int32_t fail_block;   /* block index of that failure, or -1                */
  int32_t reserved;
} qtx_rgf_problem;

/* Create a context on HIP device `device`.  Workspace is allocated lazily
 * and kept below `hbm_budget_bytes` (0 = 90% of the free device memory at
 * creation); a batch larger than the budget is processed in energy chunks.
 * `hip_stream` is a hipStream_t to launch on (NULL = a stream owned by the
 * context, created non-blocking: it does not wait for work the caller
 * queued on other streams, so inputs must be complete -- e.g. the caller's
 * stream synchronised -- before a problem is solved or submitted).  `flags`
 * bit 0 (QTX_FLAG_PROFILE) records per-kernel-class launch timings (see
 * qtx_rgf_kernel_stats). */
#define QTX_FLAG_PROFILE 1u
qtx_status qtx_rgf_create(qtx_rgf_ctx** out, int device,
                          uint64_t hbm_budget_bytes, void* hip_stream,
                          uint32_t flags);

/* Solve `n_problems` independent problems (each with its own n, b, N_E,
 * kind and precision).  Synchronous: returns when every output is written
 * (the context's stream is synchronised).  Inputs must not alias outputs. */
qtx_status qtx_rgf_solve_batch(qtx_rgf_ctx* ctx, qtx_rgf_problem* problems,
                               int32_t n_problems);

/* ---- partitioned solve (nested dissection) ----------------------------- */

/* Options of qtx_rgf_solve_nested.
 *   n_partitions  P_S >= 2.  Partition p holds the contiguous blocks
 *                 [lo_p, hi_p); sizes are n / P_S, the first n % P_S of them
 *                 one larger.  The first and last partitions need >= 1
 *                 block, middle ones >= 2 (else QTX_ERR_INVALID_ARG).
 *   reduced       optional (diag NULL = not returned): the reduced system on
 *                 the ns = 2 (P_S - 1) separators, in separator order
 *                 (last block of the top partition, first and last block of
 *                 each middle partition, first block of the bottom one):
 *                 diag [N_E][ns][b][b], upper and lower [N_E][ns-1][b][b].
 *   reduced_l, reduced_g
 *                 optional (diag NULL = not returned): the reduced right-hand
 *                 sides of X^< and X^> (diag and upper as above; the lower
 *                 blocks are -upper^dagger and are not written). */
typedef struct {
  int32_t n_partitions;
  int32_t reserved;
  qtx_bt_out reduced;
  qtx_bt_out reduced_l, reduced_g;
} qtx_rgf_nested;

/* One problem solved by the partitioned scheme of Sec. 4.4 (Fig.
 * nested-dissection) on this device: the same outputs, layout, symmetry
 * contract and error reporting as qtx_rgf_solve_batch of the problem alone
 * (results agree to rounding, not bitwise).  The blocks are split into
 * n_partitions partitions (one top, P_S - 2 middle, one bottom).  Phase 1:
 * every partition eliminates its interior blocks towards its separators --
 * top-down in the top partition, bottom-up in the bottom one, top-down with
 * the fill-in coupling to its first block in a middle one -- and writes its
 * separators' blocks of the reduced system.  Phase 2: the reduced system
 * (block tridiagonal over the separators) is solved by the recursion of
 * Sec. 3.2.3.  Phase 3: every partition recovers its selected blocks from
 * its separators' solution.  The partitions of one phase are independent
 * and run in shared launches, so the longest dependent chain per energy is
 * about n / P_S + 2 P_S inverses instead of n (a single-energy solve gains
 * parallelism); the price is the fill-in work of the middle partitions and
 * the reduced system.  Workspace (inside the context's budget, in energy
 * chunks) is about (5 + 2 n_rhs) n + 26 P_S + 10 ns blocks per energy.
 * fail_block is the global block whose inverse failed.  Synchronous. */
qtx_status qtx_rgf_solve_nested(qtx_rgf_ctx* ctx, qtx_rgf_problem* problem,
                                const qtx_rgf_nested* options);

/* Release the context's workspace, streams and events.  Caller memory is
 * untouched.  Waits for work in flight, including every problem submitted
 * to the request loop. */
qtx_status qtx_rgf_destroy(qtx_rgf_ctx* ctx);

/* ---- request loop (continuous batching) -------------------------------- */

/* Completion record of one submitted problem. */
typedef struct {
  uint64_t ticket;      /* as returned by qtx_rgf_submit                       */
  int32_t status;       /* qtx_status of the problem                           */
  int32_t fail_energy;  /* first failing energy, or -1                         */
  int32_t fail_block;   /* block of that failure, or -1                        */
  int32_t n_energies;
  double queue_s;       /* submission -> first lane admitted to the GPU        */
  double latency_s;     /* submission -> all its work observed complete        */
} qtx_rgf_completion;

/* Queue one problem for the context's request loop and return at once.  The
 * loop (a host thread with its own HIP stream, workspace and launch arena,
 * started on first use) admits queued problems in arrival order as soon as
 * workspace frees up, and runs every admitted problem's remaining work in
 * the same merged launches as the others, so problems that arrive while
 * others are running overlap with them on the device.  A problem's result is
 * the same as when it is solved alone (same kernels, tiles and order of
 * operations per problem).  The problem structure is copied (including its
 * host energies); every device buffer it points to must stay valid and
 * unmodified until its completion is returned by qtx_rgf_poll.  Workspace of
 * the loop: the context's budget (0 = half of the free device memory when
 * the loop starts).  Errors: QTX_ERR_INVALID_ARG (checked as in
 * qtx_rgf_solve_batch), QTX_ERR_NOMEM if one energy of the problem cannot
 * fit the loop's workspace. */
qtx_status qtx_rgf_submit(qtx_rgf_ctx* ctx, const qtx_rgf_problem* problem,
                          uint64_t* ticket);

/* Return up to `cap` completion records (in completion order) into `out`,
 * waiting up to `wait_ms` milliseconds for at least one (0 = do not wait,
 * -1 = wait until one arrives or nothing is outstanding).  *n_out receives
 * the number returned; *n_pending (may be NULL) the number of submitted
 * problems not yet returned.  QTX_ERR_HIP if the loop stopped on a runtime
 * error (outstanding problems are then returned with that status). */
qtx_status qtx_rgf_poll(qtx_rgf_ctx* ctx, qtx_rgf_completion* out, int32_t cap,
                        int32_t* n_out, int32_t* n_pending, int32_t wait_ms);

/* Static string for a status code. */
const char* qtx_rgf_status_string(qtx_status s);

/* Human-readable detail of the last call-level error on this context
 * (empty string if none).  Valid until the next call on the context. */
const char* qtx_rgf_last_error(const qtx_rgf_ctx* ctx);

/* Algorithmic flops of one problem at one energy (8 b^3 per complex block
 * product; an inverse priced as one product), as used for TFLOP/s.
 * `bt_rhs` != 0 when Sigma^s / P^s have off-diagonal blocks. */
double qtx_rgf_flops_per_energy(int32_t kind, int32_t n_blocks,
                                int32_t block_size, int32_t n_rhs,
                                int32_t bt_rhs, int32_t want_wr);

/* Per-kernel-class launch statistics recorded under QTX_FLAG_PROFILE since
 * the last reset: number of launches, summed device time (ms, HIP events on
 * the launch stream), summed algorithmic flops and algorithmic HBM bytes.
 * Classes: 0 = complex GEMM (FP64), 1 = complex GEMM (FP32), 2 = inverse
 * panel, 3 = elementwise/assembly.  Returns QTX_ERR_INVALID_ARG for an
 * unknown class. */
qtx_status qtx_rgf_kernel_stats(qtx_rgf_ctx* ctx, int32_t kernel_class,
                                int64_t* launches, double* total_ms,
                                double* flops, double* bytes);
qtx_status qtx_rgf_reset_stats(qtx_rgf_ctx* ctx);

/* ---- building blocks, exposed for testing the kernels one at a time ---- */

/* Strided-batched complex128 product on the FP64 matrix cores:
 *   D[e] = alpha * op(A[e]) * op(B[e]) + beta * C[e],  e = 0..batch-1
 * op(X) = X (op = 'N') or X^dagger (op = 'C').  All matrices row-major with
 * leading dimensions lda..ldd (in complex elements); element strides between
 * consecutive batch entries sA..sD (0 = shared operand).  op(A) is m x k,
 * op(B) is k x n, C and D are m x n.  C may equal D (in place); C may be
 * NULL when beta == 0.  Device pointers; runs on the context's stream and
 * returns after it completes. */
qtx_status qtx_rgf_zgemm(qtx_rgf_ctx* ctx, char opa, char opb, int32_t m,
                         int32_t n, int32_t k, double alpha_re,
                         double alpha_im, const void* A, int64_t lda,
                         int64_t sA, const void* B, int64_t ldb, int64_t sB,
                         double beta_re, double beta_im, const void* C,
                         int64_t ldc, int64_t sC, void* D, int64_t ldd,
                         int64_t sD, int32_t batch);

/* The same product computed on the FP32 matrix cores, as QTX_MIXED uses it:
 * the complex128 operands are rounded to complex64 as they are read from
 * on-chip memory into the matrix cores, products
 * accumulate in FP32, and the epilogue (alpha, beta, C, D) is complex128.
 * Arguments as for qtx_rgf_zgemm. */
qtx_status qtx_rgf_cgemm(qtx_rgf_ctx* ctx, char opa, char opb, int32_t m,
                         int32_t n, int32_t k, double alpha_re,
                         double alpha_im, const void* A, int64_t lda,
                         int64_t sA, const void* B, int64_t ldb, int64_t sB,
                         double beta_re, double beta_im, const void* C,
                         int64_t ldc, int64_t sC, void* D, int64_t ldd,
                         int64_t sD, int32_t batch);

/* Batched inverse of b x b complex128 matrices by Gauss-Jordan elimination
 * with partial pivoting (largest |z| in the pivot column to a relative 0.1%
 * in |z|^2; ties to the lowest row), 1 <= b <= 4096.  Above b = 1024 the
 * pivot rows of each 16-column panel are chosen by a tournament (each chunk
 * of 768 rows proposes the rows its own elimination pivots on, and the
 * elimination of the proposed rows picks among them), which is stable in
 * practice though its worst-case growth bound is weaker.  Up to b = 128 one
 * workgroup per matrix does the whole inverse in one launch.  A [batch][b][b]
 * is used as workspace (its contents afterwards are unspecified); the
 * inverses are written to X
 * [batch][b][b].  info[batch] (device int32, may be NULL) receives 0, or
 * 1 + the column of the first exactly zero pivot, or -(1 + column) for a
 * non-finite pivot. */
qtx_status qtx_rgf_zinv(qtx_rgf_ctx* ctx, int32_t b, void* A, void* X,
                        int32_t* info, int32_t batch);

/* Allocation-free variant of qtx_rgf_zinv, for callers that cannot allocate
 * device memory (code under stream capture into a graph, serving loops that
 * forbid allocation).  Same arguments, layout and results as qtx_rgf_zinv
 * (the same kernels run in the same order, so the results are bitwise the
 * same), with three differences:
 *   - the work buffers and launch descriptors live in a static device array
 *     of QTX_NOALLOC_SCRATCH_BYTES (plus 64 KiB of descriptors) that every
 *     GPU the library runs on holds until the process ends; a call allocates,
 *     copies and clears nothing, it only launches kernels;
 *   - the call is asynchronous: it returns once the kernels are queued on
 *     the context's stream, and the results are ready when that stream's
 *     work is complete (no wait inside, so it can be captured);
 *   - for b > 128, batch * (2*16 + 2*w) * 16 * b bytes of panel buffers
 *     (w = 64 for b <= 256, else 256) plus 8 * batch * b bytes of pivot
 *     bookkeeping (each part rounded up to 256 bytes) must fit
 *     QTX_NOALLOC_SCRATCH_BYTES; larger calls return QTX_ERR_INVALID_ARG with
 *     the sizes in qtx_rgf_last_error (e.g. at most 102 matrices of 256, 15
 *     of 512, 7 of 1024); b <= 1024.  Up to b = 128 the inverse is one launch
 *     that uses no work buffers, so any batch is accepted.
 * All calls on one GPU share its array, which keeps the last call's contents
 * (nothing in it needs to start at zero): calls that overlap in time on one
 * GPU race on it and must be serialised by the caller (one stream, or
 * events).  A and X must not be shared with a concurrent call either. */
#define QTX_NOALLOC_SCRATCH_BYTES (64ull << 20)
qtx_status qtx_rgf_zinv_noalloc(qtx_rgf_ctx* ctx, int32_t b, void* A, void* X,
                                int32_t* info, int32_t batch);

/* Retarded open-boundary surface function of a lead (Sec. "Retarded OBC"):
 * the solution x of Eq. (retarded-recursion), x = (m - n x n')^{-1}, by
 * n_iter iterations of Eq. (naive),
 *     x_{i+1} = (m - n x_i n')^{-1},
 * for every energy of a batch at once.  The start is whatever x holds on
 * entry: zeros for a cold start, or the previous self-consistent
 * iteration's x (the memoized mode of Sec. "OBC Memoization", where a fixed
 * iteration count keeps the energies in step).
 *
 *   m, n, n_prime  row-major b x b complex128 device blocks (m, n, n'); the
 *                  block of energy e starts at base + e * s_* elements, and a
 *                  stride of 0 shares one block among all energies
 *                  (otherwise s_* >= b*b).  m is typically (E + i eta) S_00 -
 *                  H_00 - Sigma^R_scatt,00, n and n' the contact couplings.
 *   x              [batch][b][b] device, contiguous: start on entry, x_N on
 *                  return.
 *   sigma          [batch][b][b] device or NULL: the boundary block
 *                  n x_N n' that enters B^R_OBC.
 *   update         device double[batch] or NULL: ||x_N - x_{N-1}||_F /
 *                  ||x_N||_F per energy (the caller's convergence test;
 *                  infinite if x_N is zero).
 *   info           device int32[batch]: 0, or +k / -k for the first
 *                  iteration k (1-based) whose inverse met an exactly zero /
 *                  a non-finite pivot; that energy's outputs are then
 *                  meaningless and the others are unaffected.
 * 1 <= b <= 1024, batch >= 0, n_iter >= 1.  Inputs must be complete on the
 * device before the call; the call returns when the results are written.
 * Scratch of 3 * batch * b*b complex128 plus the inverse's panel buffers
 * comes from the context's workspace, which grows to the largest request
 * and is kept (QTX_ERR_NOMEM if growing fails).  Errors:
 * QTX_ERR_INVALID_ARG (bad sizes, strides or NULL, or x / sigma sharing
 * memory with an input or each other), QTX_ERR_BUSY, QTX_ERR_HIP. */
qtx_status qtx_rgf_obc_fixed_point(qtx_rgf_ctx* ctx, int32_t b, int32_t batch,
                                   const void* m, int64_t s_m, const void* n,
                                   int64_t s_n, const void* n_prime,
                                   int64_t s_np, void* x, void* sigma,
                                   double* update, int32_t* info,
                                   int32_t n_iter);

/* The same surface function by Sancho-Rubio decimation, the faster iterative
 * method the paper cites in Sec. "Retarded OBC" (Lopez Sancho et al., 1985):
 * n_steps steps for every energy, each eliminating every other layer of the
 * lead,
 *     g = m_b^{-1},  m_s -= n g n',  m_b -= n g n' + n' g n,
 *     n <- -n g n,   n' <- -n' g n',
 * starting from m_s = m_b = m; then x = m_s^{-1}.  The represented lead
 * length doubles per step, so the couplings shrink geometrically.
 *   m, n, n_prime, s_*  as for qtx_rgf_obc_fixed_point.
 *   x          [batch][b][b] device, contiguous: output only.
 *   sigma      [batch][b][b] device or NULL: n x n'.
 *   coupling   device double[batch] or NULL: the remaining coupling
 *              (||n_N||_F + ||n'_N||_F) / (||n||_F + ||n'||_F), the caller's
 *              convergence test.
 *   info       device int32[batch]: 0, or +k / -k for the first inverse that
 *              met an exactly zero / non-finite pivot: k = step (1-based),
 *              n_steps + 1 for the final inverse of m_s.
 * 1 <= b <= 1024, batch >= 0, n_steps >= 1.  Scratch of 11 * batch * b*b
 * complex128 plus the inverse's panel buffers comes from the context's
 * workspace.  Errors as for qtx_rgf_obc_fixed_point. */
qtx_status qtx_rgf_obc_sancho_rubio(qtx_rgf_ctx* ctx, int32_t b, int32_t batch,
                                    const void* m, int64_t s_m, const void* n,
                                    int64_t s_n, const void* n_prime,
                                    int64_t s_np, void* x, void* sigma,
                                    double* coupling, int32_t* info,
                                    int32_t n_steps);

/* Lesser/greater boundary blocks of a contact in equilibrium (Sec.
 * "Lesser/Greater OBC", electrons): by the fluctuation-dissipation theorem,
 * with Gamma = i (Sigma^R - Sigma^R^dagger),
 *     Sigma^< = i f Gamma,     Sigma^> = -i (1 - f) Gamma.
 *   sigma_r           device, block of energy e at sigma_r + e * s_sr
 *                     (s_sr = 0 shares one block, else s_sr >= b*b): the
 *                     retarded boundary block n x n'.
 *   f, one_minus_f    HOST double[batch]: the contact's occupation at each
 *                     energy and its complement, both evaluated by the
 *                     caller (so that neither rounds to zero).
 *   sigma_l, sigma_g  [batch][b][b] device outputs; either may be NULL, not
 *                     both.  Outputs must not overlap sigma_r or each other
 *                     (QTX_ERR_INVALID_ARG).
 * 1 <= b <= 1024, batch >= 0; returns when written.  Errors:
 * QTX_ERR_INVALID_ARG, QTX_ERR_BUSY, QTX_ERR_HIP. */
qtx_status qtx_rgf_obc_lesser_greater(qtx_rgf_ctx* ctx, int32_t b, int32_t batch,
                                      const void* sigma_r, int64_t s_sr,
                                      const double* f, const double* one_minus_f,
                                      void* sigma_l, void* sigma_g);

/* Observables from the selected blocks (Sec. "Observables": local density of
 * states, charge density and current follow from the diagonal and first
 * off-diagonal blocks of G^< and G^>).  Per energy e and block i, in units
 * e = hbar = 1, one spin, per unit energy:
 *     dos[e][i]     = Tr(i (G^>_ii - G^<_ii)) / (2 pi)
 *     density[e][i] = Tr(-i G^<_ii) / (2 pi)
 *     current[e][i] = 2 Re Tr(H_{i,i+1} G^<_{i+1,i}) / (2 pi),  i < n-1,
 *                     through the interface between blocks i and i+1,
 *                     positive from i to i+1.
 *   XL_diag, XG_diag  [batch][n][b][b] device: diagonal blocks of G^<, G^>
 *                     (the X^<, X^> outputs of a G-type solve).
 *   XL_lower          [batch][n-1][b][b] device: G^<_{i+1,i}.
 *   H_upper           [n-1][b][b] device: H_{i,i+1} (energy independent).
 *   dos, density      device double[batch][n] or NULL; current device
 *                     double[batch][n-1] or NULL (then XL_lower and H_upper
 *                     may be NULL).  XG_diag may be NULL if dos is.
 * Integration over energy is left to the caller.  1 <= b <= 1024, n >= 1,
 * batch >= 0; returns when written.  Scratch of (n-1) b*b complex128 (the
 * couplings' adjoints) plus batch (n-1) ceil(b*b / 2048) doubles (the
 * current's partial sums) from the context's workspace.  Errors:
 * QTX_ERR_INVALID_ARG, QTX_ERR_NOMEM, QTX_ERR_BUSY, QTX_ERR_HIP. */
/* Element-wise energy convolution of two energy-resolved quantities, the
 * form of the scattering terms P and Sigma (Sec. "Energy Convolutions",
 * Eq. interaction: B_scatt(E) is proportional to the integral over E' of
 * X1(E - E') X2(E'), the products taken entry by entry).  On uniform energy
 * grids of one spacing, with the prefactor (sign, i / 2 pi, the spacing)
 * folded into s = scale_re + i scale_im:
 *     B[k][i] = s * sum_{k'=0}^{n2-1} X1'[k + shift - k'][i] * X2[k'][i],
 *     0 <= k < n_out, 0 <= i < n_elem,
 * X1' = X1, or X1 with its energy order reversed (X1'[j] = X1[n1-1-j]) when
 * reverse1 = 1, which gives the correlation form G(E') G(E' - E); terms
 * whose X1' index lies outside [0, n1) are left out, and shift places the
 * difference grid of X1 against the output grid.
 *   X1  [n1][n_elem], X2 [n2][n_elem], B [n_out][n_elem]: complex128 device
 *       arrays, energy-major (the layout of the solve's outputs: the
 *       selected blocks of one energy, [n][b][b] or a block range of them,
 *       are n_elem consecutive entries).  B must not overlap X1 or X2.
 * Summation over k' in increasing order, in FP64.  n_elem >= 0, n1, n2 >= 1,
 * n_out >= 0, reverse1 in {0, 1}; returns when written.  Errors:
 * QTX_ERR_INVALID_ARG, QTX_ERR_BUSY, QTX_ERR_HIP. */
qtx_status qtx_rgf_energy_convolution(qtx_rgf_ctx* ctx, int64_t n_elem,
                                      const void* X1, int32_t n1,
                                      int32_t reverse1, const void* X2,
                                      int32_t n2, void* B, int32_t n_out,
                                      int32_t shift, double scale_re,
                                      double scale_im);

/* The screened interaction's lesser/greater surface function (Sec.
 * "Lesser/Greater OBC"): the solution w of Eq. (lyapunov),
 *     w = q - a w a^dagger,
 * for every energy of a batch, q and a being b x b blocks extracted from P,
 * V and w^R by the caller.  The series sum_j (-1)^j a^j q (a^dagger)^j
 * converges when the spectral radius of a is below 1.
 *
 * qtx_rgf_obc_lyapunov_fixed_point: n_iter iterations of
 * w_{i+1} = q - a w_i a^dagger from the start held in w (zeros, or the
 * previous self-consistent iteration's w: the memoized mode of Sec. "OBC
 * Memoization"); update (device double[batch] or NULL) receives
 * ||w_N - w_{N-1}||_F / ||w_N||_F.
 *
 * qtx_rgf_obc_lyapunov_doubling: doubling over the series, S_1 = q - a q
 * a^dagger, then n_steps - 1 steps A <- A A, S <- S + A S A^dagger (S_k holds
 * the first 2^k terms); w is output only; remaining (device double[batch] or
 * NULL) receives ||a^(2^n_steps)||_F / ||a||_F, the caller's convergence
 * test.
 *
 *   a, q     row-major b x b complex128 device blocks; the block of energy e
 *            at base + e * s_* elements (0 = shared, else >= b*b).
 *   w        [batch][b][b] device, contiguous; must not overlap a or q
 *            (QTX_ERR_INVALID_ARG).
 * 1 <= b <= 1024, batch >= 0, n_iter / n_steps >= 1.  Scratch of 2 (fixed
 * point) or 3 (doubling) * batch * b*b complex128 from the context's
 * workspace.  Errors:
 * QTX_ERR_INVALID_ARG, QTX_ERR_NOMEM, QTX_ERR_BUSY, QTX_ERR_HIP. */
qtx_status qtx_rgf_obc_lyapunov_fixed_point(qtx_rgf_ctx* ctx, int32_t b,
                                            int32_t batch, const void* a,
                                            int64_t s_a, const void* q,
                                            int64_t s_q, void* w,
                                            double* update, int32_t n_iter);
qtx_status qtx_rgf_obc_lyapunov_doubling(qtx_rgf_ctx* ctx, int32_t b,
                                         int32_t batch, const void* a,
                                         int64_t s_a, const void* q,
                                         int64_t s_q, void* w,
                                         double* remaining, int32_t n_steps);

qtx_status qtx_rgf_observables(qtx_rgf_ctx* ctx, int32_t n_blocks, int32_t b,
                               int32_t batch, const void* XL_diag,
                               const void* XG_diag, const void* XL_lower,
                               const void* H_upper, double* dos,
                               double* density, double* current);

#ifdef __cplusplus
}
#endif

#endif /* QTX_RGF_H */
