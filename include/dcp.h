/*
 * dcp.h -- C ABI of libdcp, the MI355X (gfx950) library for the fused
 * reaction-diffusion array program
 *
 *     u' = u + dt * (alpha * Lap7(u) - beta * u^3 + gamma * f)
 *     Lap7(u)[p] = (sum of the six face neighbours of p - 6 u[p]) / h^2
 *
 * applied T times on an (nx, ny, nz) grid, and for its adjoint.
 *
 * The program is one element-wise expression over a 7-point stencil, the
 * class of NumPy array programs whose translation is described in Sec. 2.3
 * of the paper (each operator becomes a map over the array; an expression is
 * split into single-operator statements with one temporary each) and whose
 * main GPU speed-up comes from the optimisations of Sec. 3.1 (greedy
 * subgraph fusion of maps that share an iteration space, transient
 * elimination, tiled write-conflict reductions).  The fused entry points
 * compute the whole expression in one pass over the grid with no
 * temporaries in memory; the unfused entry point runs the single-operator
 * statements one kernel each, as the unoptimised program would.
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every entry point
 *
 * Layout.  Fields are dense arrays of nx*ny*nz elements with x fastest:
 *   element (x, y, z) is at index x + nx*(y + ny*z).
 *   (A C-order array of shape (nz, ny, nx).)
 *
 * Element type.  dtype DCP_F64 (double) or DCP_F32 (float).  Every field
 *   argument of one call has that type.  In DCP_F32 the coefficients are
 *   rounded to float once per call and the arithmetic is float; the
 *   diagnostic norms and the gradient reductions are accumulated in double.
 *
 * Boundary.  DCP_DIRICHLET0: a neighbour outside [0, n) along an axis reads
 *   as 0 and every point of the grid is updated.  DCP_PERIODIC: the
 *   neighbour index is taken modulo n (n = 1 and n = 2 included).
 *
 * Memory.  Every field, norm and gradient pointer is a DEVICE pointer owned
 *   by the caller.  `coeffs` is a HOST pointer read during the call only.
 *   The library never allocates or frees device memory: scratch space comes
 *   from the caller's workspace `ws` of `ws_bytes` bytes (size it with
 *   dcp_workspace_bytes; ws may be NULL when that size is 0).  Apart from
 *   the fixed scratch of dcp_step_fused_noalloc (below), the library holds
 *   no global state; calls on different streams with disjoint buffers may
 *   run concurrently.
 *
 * Execution.  Work is enqueued on `stream` (a hipStream_t; NULL is the
 *   default stream) and the call returns without synchronising.  Results,
 *   including the double-precision norm and gradient outputs, are valid once
 *   the stream has reached the call.
 *
 * Errors.  Every entry point returns a dcp_status.  Argument errors
 *   (DCP_E_NULL .. DCP_E_ALIAS) are detected before anything is enqueued:
 *   no partial work is done and no output is touched.  DCP_E_HIP means a
 *   HIP launch or copy failed; work enqueued before the failure may have
 *   run.  Non-finite coefficients are rejected; unstable but finite ones are
 *   not (the program is the caller's).
 *
 * Empty grids (nx, ny or nz equal to 0) are valid: fields are untouched and
 * every requested norm or gradient sum is written as 0.
 *
 * Tuning.  The tile and pass choices are the library's own.  For tuning
 * runs only, the environment variables DCP_TILE_SHAPE, DCP_TILE_ZC,
 * DCP_TB_CFG, DCP_TBK_CFG, DCP_TBK_SBLK, DCP_FUSE_ZR, DCP_J1_K, DCP_J2_CFG,
 * DCP_J2_MODE and DCP_J2M_CPL force a tiling or schedule; they are read at each call
 * and honoured only while DCP_TUNING=1 is set as well.  A forced choice computes the same
 * fields bit for bit; the double norms and sums may differ in rounding (their
 * summation order follows the tiles).
 */
#ifndef DCP_H
#define DCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DCP_OK = 0,
    DCP_E_NULL = -1,      /* a required pointer is NULL                        */
    DCP_E_SHAPE = -2,     /* negative extent, or nx*ny*nz*sizeof overflows     */
    DCP_E_DTYPE = -3,     /* dtype is not DCP_F64 or DCP_F32                   */
    DCP_E_BC = -4,        /* boundary is not DCP_DIRICHLET0 or DCP_PERIODIC    */
    DCP_E_ARG = -5,       /* T < 0, ckpt_every < 1 with checkpoints, tblock
                             out of range, h <= 0, non-finite coefficient,
                             unknown impl or op                               */
    DCP_E_WORKSPACE = -6, /* ws_bytes smaller than dcp_workspace_bytes(...)    */
    DCP_E_ALIAS = -7,     /* an output overlaps an input it must not overlap   */
    DCP_E_SCRATCH = -8,   /* the call needs more than the fixed device scratch
                             of dcp_step_fused_noalloc                        */
    DCP_E_HIP = -100      /* a HIP launch or copy failed                       */
} dcp_status;

typedef enum { DCP_F64 = 0, DCP_F32 = 1 } dcp_dtype;
typedef enum { DCP_DIRICHLET0 = 0, DCP_PERIODIC = 1 } dcp_bc;
typedef enum { DCP_FUSED = 0, DCP_UNFUSED = 1 } dcp_impl;

/* Operation selector for dcp_workspace_bytes. */
typedef enum {
    DCP_OP_STEP_FUSED = 0,
    DCP_OP_STEP_UNFUSED = 1,
    DCP_OP_RUN = 2,
    DCP_OP_ADJOINT = 3
} dcp_op;

/* Scalars of the program.  h is the grid spacing on every axis (> 0). */
typedef struct {
    double alpha, beta, gamma, h, dt;
} dcp_coeffs;

/*
 * Workspace size in bytes for one call of `op` with these arguments.
 *   impl        DCP_FUSED or DCP_UNFUSED (DCP_OP_RUN only; ignored otherwise)
 *   T           number of steps (DCP_OP_RUN, DCP_OP_ADJOINT)
 *   ckpt_every  checkpoint interval k (DCP_OP_ADJOINT: >= 1; ignored otherwise)
 *   tblock      steps per pass over memory (DCP_OP_RUN fused, DCP_OP_ADJOINT;
 *               1 = one step per pass)
 *   norms       nonzero if the call will request norms (energy/resid/norms2);
 *               for DCP_OP_ADJOINT: nonzero if it will request grad_gamma
 *               without grad_f (one more field of workspace)
 * The size is an upper bound valid for any pointer alignment.  Writes it to
 * *bytes (a host pointer).  Returns DCP_OK or an argument error.
 */
int dcp_workspace_bytes(int op, int dtype, int impl, int64_t nx, int64_t ny,
                        int64_t nz, int32_t T, int32_t ckpt_every,
                        int32_t tblock, int norms, size_t *bytes);

/*
 * One fused step: u_out = u + dt*(alpha*Lap7(u) - beta*u^3 + gamma*f),
 * computed in one pass (greedy subgraph fusion and transient elimination of
 * Sec. 3.1): reads u and f once, writes u_out once, no temporaries.
 *   u, f     [N]  in   (may alias each other)
 *   u_out    [N]  out  (must not overlap u or f)
 *   norms2   [2]  out, optional: {sum u_out^2, sum (u_out - u)^2}, reduced in
 *                 double with a fixed order (bitwise reproducible), in the
 *                 tiled manner of the write-conflict reductions of Sec. 3.1
 */
int dcp_step_fused(int dtype, const void *u, const void *f, void *u_out,
                   int64_t nx, int64_t ny, int64_t nz, const dcp_coeffs *coeffs,
                   int bc, double *norms2, void *ws, size_t ws_bytes,
                   void *stream);

/*
 * dcp_step_fused without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and rules as
 * dcp_step_fused, minus ws and ws_bytes: the per-workgroup partial sums of
 * norms2 live in a fixed device array of DCP_NOALLOC_SCRATCH_BYTES (1 MiB)
 * that the library holds on every GPU it runs on until the process ends.
 * The call allocates nothing.  It uses the scratch of the current device,
 * so u, f, u_out, norms2 and stream must belong to that device.
 * The scratch is needed only when norms2 is requested (16 bytes per
 * workgroup of the one-step tiling, which covers grids of more than 10^9
 * points); a grid that needs more returns DCP_E_SCRATCH before anything is
 * enqueued.  Calls that overlap in time on one GPU (on different streams,
 * or from different threads) share the scratch and race: serialise them.
 * A call overwrites every scratch entry it reads, so nothing carries over
 * from an earlier call.
 */
#define DCP_NOALLOC_SCRATCH_BYTES ((size_t)1 << 20)
int dcp_step_fused_noalloc(int dtype, const void *u, const void *f, void *u_out,
                           int64_t nx, int64_t ny, int64_t nz,
                           const dcp_coeffs *coeffs, int bc, double *norms2,
                           void *stream);

/*
 * The same step as the unfused single-operator program of Sec. 2.3, one
 * kernel per statement with every temporary written to memory:
 *     lap = Lap7(u); u3 = (u*u)*u; t1 = alpha*lap; t2 = beta*u3; t3 = t1 - t2;
 *     t4 = gamma*f;  t5 = t3 + t4; t6 = dt*t5;     u_out = u + t6
 * (plus one reduction kernel when norms2 is requested).  Each statement
 * rounds once, with no contraction, so in DCP_F64 the result equals the
 * plain serial evaluation of the same statements bit for bit.  Same
 * arguments and rules as dcp_step_fused; the workspace holds three fields.
 */
int dcp_step_unfused(int dtype, const void *u, const void *f, void *u_out,
                     int64_t nx, int64_t ny, int64_t nz,
                     const dcp_coeffs *coeffs, int bc, double *norms2,
                     void *ws, size_t ws_bytes, void *stream);

/*
 * T steps in place (the time loop: a state-transition loop around one
 * dataflow state, Sec. 2.3).
 *   impl        DCP_FUSED or DCP_UNFUSED
 *   u     [N]   in: u_0; out: u_T
 *   f     [N]   in (must not overlap u)
 *   T           >= 0 (T = 0 leaves u unchanged)
 *   tblock      most steps fused per pass over memory (temporal blocking),
 *               1, 2 or 3; 1 = one pass per step.  Values > 1 need impl =
 *               DCP_FUSED and 16-byte aligned fields with nx a multiple of
 *               the 16-byte vector (2 doubles, 4 floats).  Passes of tblock
 *               steps run on tiles of whole x-rows, or of x-segments with a
 *               halo of recomputed points when rows are too long for a
 *               whole-row tile; T mod tblock remaining steps run as shorter
 *               passes (dcp_run_plan reports the passes).  Either way every
 *               point is computed with the same operations, so u_T is
 *               bitwise the same for every tblock.
 *   energy [T]  out, optional: energy[t-1] = sum u_t^2, t = 1..T (double)
 *   resid  [T]  out, optional: resid[t-1] = sqrt(sum (u_t - u_{t-1})^2)
 *   ckpt        out, optional: ceil(T/k) consecutive fields; slot c holds
 *               u_{c*k}, c = 0 .. ceil(T/k)-1 (must not overlap u, f or ws)
 *   ckpt_every  k >= 1 when ckpt is given; ignored otherwise
 * Every step uses the same kernel whether or not norms or checkpoints are
 * requested, so u_T is bitwise identical either way.
 */
int dcp_run(int dtype, int impl, void *u, const void *f, int64_t nx,
            int64_t ny, int64_t nz, const dcp_coeffs *coeffs, int bc,
            int32_t T, int32_t tblock, double *energy, double *resid,
            void *ckpt, int32_t ckpt_every, void *ws, size_t ws_bytes,
            void *stream);

/*
 * How a dcp_run with these arguments takes its steps, for 16-byte aligned
 * fields (what torch and hipMalloc return): passes over memory of one, two
 * and three steps, so that a caller can see when a grid falls back to
 * shorter passes.  Host only; asks the current device for its LDS size when
 * there is one.  Writes *info (a host pointer); argument errors as dcp_run.
 */
typedef struct {
    int32_t passes[3];      /* passes of 1, 2 and 3 steps                      */
    int32_t steps_per_pass; /* the most steps any pass takes (0: no steps)     */
    int32_t segmented;      /* multi-step passes over x-segments with a halo
                               (1) or over whole rows (0)                      */
    int32_t tile_rows;      /* rows per tile of the multi-step passes          */
    int32_t lanes;          /* lanes per workgroup of the multi-step passes
                               (768: the three-step passes' register-ring
                               form, whose z-neighbours stay in registers;
                               1024 or 512: the form that re-reads them from
                               LDS)                                            */
} dcp_run_info;

int dcp_run_plan(int dtype, int impl, int64_t nx, int64_t ny, int64_t nz,
                 int32_t T, int32_t tblock, int norms, dcp_run_info *info);

/*
 * Reverse-mode gradient through T fused steps, from the checkpoints that
 * dcp_run wrote.  The paper defines no adjoint: these formulas are the
 * chain rule applied to the step's statement (J_t is the Jacobian of one
 * step with respect to u_t; the parameter sums differentiate the same
 * statement with respect to alpha, beta, gamma and f), and the checkpointed
 * recomputation is the standard every-k scheme.
 * With J_t = I + dt*alpha*L - diag(3*beta*dt*u_t^2):
 *     lambda_T = lam_T
 *     lambda_t = J_t^T lambda_{t+1}                    (t = T-1 .. 0)
 *     dL/dalpha = sum_t dt * <lambda_{t+1}, L u_t>
 *     dL/dbeta  = sum_t -dt * <lambda_{t+1}, u_t^3>
 *     dL/dgamma = sum_t dt * <lambda_{t+1}, f>        (optional)
 *     dL/df     = gamma * dt * sum_t lambda_{t+1}     (optional)
 * Segments [c*k, min(T, c*k+k)) are processed last to first: the states
 * inside a segment are recomputed from its checkpoint with the forward
 * kernel, then one fused adjoint kernel per step applies J_t^T (L is
 * symmetric under both boundary rules, so L^T is the same 7-point gather)
 * and accumulates the two parameter sums in double.
 * With tblock >= 2, two adjoint steps share one pass over memory where the
 * grid allows whole-row tiles (adjoint steps are paired by global parity,
 * (2m+1, 2m), independently of k), and the recomputed forward steps take
 * passes of up to tblock steps, every state stored (as dcp_run plans them).
 *   ckpt        [ceil(T/k) fields] in: as written by dcp_run (same T, k,
 *               coefficients, boundary and dtype)
 *   f      [N]  in
 *   lam_T  [N]  in: dL/du_T
 *   tblock      1, 2 or 3 (see above)
 *   grad_u0 [N] out: dL/du_0 (must not overlap ckpt, f, lam_T or ws)
 *   grad_ab [2] out, double: {dL/dalpha, dL/dbeta}, reduced in a fixed order,
 *               so for a given tblock the result does not depend on k bit
 *               for bit (dL/du_0 does not depend on tblock either)
 *   grad_f  [N] out, optional (NULL: not computed): dL/df.  The adjoint
 *               kernels add each step's input lambda_{t+1} into it, in step
 *               order (t = T-1 .. 0) and in the field's type; it is then
 *               scaled by gamma*dt.  Does not depend on k or tblock, bit for
 *               bit.  Must not overlap any other argument.
 *   grad_gamma [1] out, double, optional: dL/dgamma = dt * <sum of the
 *               lambda_{t+1}, f>, a fixed-order double reduction.  Without
 *               grad_f the running sum lives in the workspace (size it with
 *               norms = 1).
 */
int dcp_adjoint_run(int dtype, const void *ckpt, int32_t ckpt_every,
                    const void *f, const void *lam_T, int64_t nx, int64_t ny,
                    int64_t nz, const dcp_coeffs *coeffs, int bc, int32_t T,
                    int32_t tblock, void *grad_u0, double *grad_ab,
                    void *grad_f, double *grad_gamma, void *ws,
                    size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * The Jacobi stencil programs the paper lists: jacobi_1d (Sec. 2.2, the
 * static-symbolic-typing example) and jacobi_2d (Sec. 4.3, the shared-memory
 * program that the local-view example distributes).  Both take two float64
 * arrays A and B and a step count TSTEPS and run the listings' time loop
 * for t = 1 .. TSTEPS-1 (no pass when TSTEPS <= 1); each pass
 *   1D:  B[i] = 0.33333 * ((A[i-1] + A[i]) + A[i+1])    for 1 <= i <= n-2,
 *        then A[i] from B the same way;
 *   2D:  B[i][j] = 0.2 * ((((A[i][j] + A[i][j-1]) + A[i][j+1]) + A[i+1][j])
 *                         + A[i-1][j])           for 1 <= i <= n0-2,
 *                                                    1 <= j <= n1-2,
 *        then A[i][j] from B the same way.
 * The weights are the listings' literals; the sums are added in the
 * listings' left-to-right order and every operation rounds once, so A and B
 * equal a plain serial evaluation bit for bit, for every tblock.  Elements
 * outside the interior (the ends; the outer rows and columns) are never
 * written.  An array with no interior (n < 3; n0 < 3 or n1 < 3) is left
 * unchanged.
 *
 * Layout.  1D: n contiguous doubles.  2D: row-major n0 x n1 (element (i, j)
 *   at i*n1 + j, j contiguous); the listing's case is n0 = n1 = N.
 * A, B  [N]  in/out, device, caller-owned; must not overlap each other.
 * tblock     at most this many half-steps per pass over memory (temporal
 *            blocking): 0 = the library's default; 1D: 1..256, 2D: 1..16.
 *            2D arrays need n1 < 2^30.
 * ws         device workspace of dcp_jacobi_workspace_bytes(dims, n0, n1,
 *            tsteps, tblock, &bytes) bytes (n0 = n and n1 ignored for
 *            dims = 1); two
 *            array copies when any pass runs, else 0 and ws may be NULL);
 *            must not overlap A or B.
 * Errors as for the other entry points: DCP_E_SHAPE (negative extent or
 *   overflow), DCP_E_ARG (tblock out of range, dims not 1 or 2), DCP_E_NULL,
 *   DCP_E_ALIAS, DCP_E_WORKSPACE, all before any work is enqueued;
 *   DCP_E_HIP for a failed launch.
 */
int dcp_jacobi_workspace_bytes(int dims, int64_t n0, int64_t n1,
                               int32_t tsteps, int32_t tblock, size_t *bytes);

/*
 * The pass schedule a call with these arguments would run: *passes = number
 * of passes over memory (0 when nothing runs), *halo = the most half-steps in
 * one pass (host pointers).  Passes are even in number; when tblock >= 2 and
 * TSTEPS >= 3 each holds whole iterations (an even number of half-steps) and
 * only the last one stores B.
 */
int dcp_jacobi_plan(int dims, int64_t n0, int64_t n1, int32_t tsteps,
                    int32_t tblock, int64_t *passes, int32_t *halo);

int dcp_jacobi_1d(int32_t tsteps, double *A, double *B, int64_t n,
                  int32_t tblock, void *ws, size_t ws_bytes, void *stream);

int dcp_jacobi_2d(int32_t tsteps, double *A, double *B, int64_t n0,
                  int64_t n1, int32_t tblock, void *ws, size_t ws_bytes,
                  void *stream);

/*
 * Gradient through T fused steps with a fixed number of stored states
 * (binomial checkpointing): the memory-bounded alternative to checkpoints
 * every k steps, for T much larger than memory allows.  The reverse sweep
 * follows the schedule of dcp_revolve_schedule: with nslots snapshot slots
 * it recomputes the least number of forward steps (r*T - C(c+r, c+1) with
 * c = nslots + 1 and r the least integer with C(c+r, c) >= T).
 *
 * dcp_revolve_workspace_bytes: the workspace both calls share (the caller
 *   keeps it, untouched, from the forward call to the adjoint call): the
 *   saved u_0, nslots + 1 states, one scratch and two adjoint fields, plus
 *   the reductions; lsum_field nonzero adds the field for grad_gamma without
 *   grad_f.  Writes *bytes (host pointer).
 * dcp_revolve_forward: T steps in place on u (u_0 in, u_T out), as dcp_run
 *   computes them (bitwise the same u_T), saving u_0 and the snapshots the
 *   reverse sweep starts from in ws.  tblock as in dcp_run (1, 2 or 3).
 * dcp_revolve_adjoint: the same outputs as dcp_adjoint_run (grad_u0,
 *   grad_ab, optional grad_f and grad_gamma), from lam_T = dL/du_T and the
 *   workspace of the forward call (same T, nslots, coefficients, boundary
 *   and dtype).  The reverse sweep reuses the snapshot slots, so one
 *   forward call serves one adjoint call (run the forward again for
 *   another).  The fields grad_u0 and grad_f and the sum grad_gamma equal
 *   dcp_adjoint_run's with tblock = 1 bit for bit; so does grad_ab with
 *   tblock = 1.  tblock applies to the recomputed forward steps, and with
 *   tblock >= 2 two consecutive adjoint steps whose states are both stored
 *   run as one pass, whose per-step sums are added in another order (grad_ab
 *   then differs from tblock = 1 by rounding only).  A one-step advance whose
 *   state only the next adjoint step reads is folded into that step (the
 *   state is recomputed at each point, bitwise as the advance computes it),
 *   and a chain of one-step advances into fresh buffers runs as one pass.
 * Arguments, ownership and errors as for dcp_run / dcp_adjoint_run.
 */
int dcp_revolve_workspace_bytes(int dtype, int64_t nx, int64_t ny,
                                int64_t nz, int32_t T, int32_t nslots,
                                int lsum_field, size_t *bytes);

int dcp_revolve_forward(int dtype, void *u, const void *f, int64_t nx,
                        int64_t ny, int64_t nz, const dcp_coeffs *coeffs,
                        int bc, int32_t T, int32_t nslots, int32_t tblock,
                        void *ws, size_t ws_bytes, void *stream);

int dcp_revolve_adjoint(int dtype, const void *f, const void *lam_T,
                        int64_t nx, int64_t ny, int64_t nz,
                        const dcp_coeffs *coeffs, int bc, int32_t T,
                        int32_t nslots, int32_t tblock, void *grad_u0,
                        double *grad_ab, void *grad_f, double *grad_gamma,
                        void *ws, size_t ws_bytes, void *stream);

/*
 * Binomial checkpointing schedule of the reverse sweep over T steps with
 * `nslots` snapshot slots (besides the saved u_0 and one work state); see
 * dcp_revolve_forward / dcp_revolve_adjoint.  Writes *nops and, if not NULL,
 * *forward_steps (steps recomputed by the schedule, including the initial
 * sweep to u_{T-1}); if ops is not NULL, also the ops as 5 int64 each:
 *   {0, src, dst, t0, t1}  advance the state in buffer src (time t0) to time
 *                          t1 into buffer dst
 *   {1, src, -1, t, t}     adjoint step t with u_t in buffer src
 * Buffers: -1 = the saved u_0, 0 .. nslots-1 = slots, nslots = work state.
 * DCP_E_WORKSPACE if cap (in ops) is too small.  Host only.
 */
int dcp_revolve_schedule(int64_t T, int32_t nslots, int64_t *ops, int64_t cap,
                         int64_t *nops, int64_t *forward_steps);

/* ---------------------------------------------------------------------------
 * A fusing compiler for element-wise + stencil programs (the greedy subgraph
 * fusion and transient elimination of Sec. 3.1, applied to programs in the
 * single-operator SSA form of Sec. 2.3), generating HIP for gfx950 at run
 * time.  Program text, one statement per line ('#' starts a comment):
 *     dtype f64 | f32
 *     input  NAME ...          fields in memory (nx*ny*nz, x fastest)
 *     param  NAME ...          scalars given at run time (finite doubles,
 *                              rounded to the dtype once)
 *     NAME = add|sub|mul|div A B
 *     NAME = neg A  |  NAME = copy A
 *     NAME = shift A dx dy dz  the field A at (x+dx, y+dy, z+dz), under the
 *                              run's boundary rule (DCP_DIRICHLET0: 0
 *                              outside; DCP_PERIODIC: indices mod n)
 *     output NAME ...          fields written to memory
 * Operands are names defined above or numeric literals (finite doubles,
 * rounded to the dtype once).  Every statement is
 * one map over the grid (a scalar when all its operands are scalars) and
 * rounds once, so the result equals the statement-by-statement evaluation
 * bit for bit, fused or not.
 *
 * dcp_fuse_build: parses, partitions (fuse = 1: statements go greedily to
 *   the earliest kernel whose values they can read, a shifted read of a
 *   computed value starting a new kernel, and only outputs and values read
 *   by a later kernel are written to memory; fuse = 0: one kernel per
 *   statement, every value written), generates and compiles the kernels
 *   (host only; no GPU needed).  On error returns DCP_E_ARG (program text)
 *   or DCP_E_HIP (compilation) with a message in err (errlen bytes).
 * dcp_fuse_info: info[0..5] = {dtype, inputs, params, outputs, kernels,
 *   workspace fields} (the first n of them).
 * dcp_fuse_source: the generated HIP source (NUL-terminated) into buf of
 *   len bytes; *needed = its size.
 * dcp_fuse_workspace_bytes: device workspace for a grid (the values that
 *   are written to memory but are not outputs).
 * dcp_fuse_run: inputs[] and outputs[] in declaration order (device
 *   pointers; outputs must not overlap inputs, each other or ws), params[]
 *   (host doubles).  Loads the code on the current device at its first run
 *   there (under a lock: several threads may run one program object, each
 *   on its own outputs and workspace).  Runs are asynchronous on the given
 *   stream; dcp_fuse_free first waits for every device the program was
 *   loaded on.
 */
typedef struct dcp_fused dcp_fused;

int dcp_fuse_build(const char *program, int fuse, dcp_fused **out, char *err,
                   size_t errlen);
void dcp_fuse_free(dcp_fused *program);
int dcp_fuse_info(const dcp_fused *program, int32_t *info, int32_t n);
int dcp_fuse_source(const dcp_fused *program, char *buf, size_t len,
                    size_t *needed);
int dcp_fuse_workspace_bytes(const dcp_fused *program, int64_t nx, int64_t ny,
                             int64_t nz, size_t *bytes);
int dcp_fuse_run(dcp_fused *program, const void *const *inputs,
                 const double *params, void *const *outputs, int64_t nx,
                 int64_t ny, int64_t nz, int bc, void *ws, size_t ws_bytes,
                 void *stream);

/*
 * Streaming probe: one launch of a plain streaming kernel over device
 * buffers, to measure the HBM bandwidth such a kernel reaches on this GPU
 * (the practical ceiling for the kernels above; not part of the program).
 *   kind  0: out = a (copy); 1: out = a + b (two reads, one write);
 *         2: read a (out receives at most one 16-byte flag per workgroup,
 *         65536 of them, and only for non-finite data); 3: fill out
 *   nt    nonzero: loads and stores carry the streaming (non-temporal) hint
 *   bytes size of each buffer, a multiple of 16; kind 2 needs at least
 *         1 MiB and out of 1 MiB
 * Buffers are 16-byte aligned device arrays of doubles; out must not
 * overlap a or b.  Errors: DCP_E_ARG, DCP_E_NULL, DCP_E_ALIAS, DCP_E_HIP.
 */
int dcp_stream_probe(int kind, int nt, const void *a, const void *b,
                     void *out, size_t bytes, void *stream);

/* Static, NUL-terminated description of a dcp_status value. */
const char *dcp_status_string(int status);

/* Largest tblock accepted by dcp_run for this dtype (1 if temporal
 * blocking is not available). */
int32_t dcp_max_tblock(int dtype);

#ifdef __cplusplus
}
#endif

#endif /* DCP_H */
