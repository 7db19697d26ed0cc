/*
 * cntri.h -- C ABI of the MI355X (gfx950) N-shaped partition Crank-Nicolson solver.
 *
 * Method: Lutsyshyn, Navarrete, Bauer, "The N-shaped partition method: A novel parallel
 * implementation of the Crank Nicolson algorithm", arXiv 2205.00856.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array arguments are DEVICE pointers owned by the caller (for example the storage of
 *   torch tensors on the GPU); the library never frees or keeps them past the call.
 *   Exception: cn_layout.offsets is a HOST pointer (see below).
 * - Complex values are interleaved FP64 pairs (re, im), 16 bytes, 16-byte aligned (the
 *   layout of torch.complex128 / C99 double complex).  Real values are FP64.
 * - Tridiagonal naming follows Sec. 4, Eq. (5) of the paper: row i reads
 *       b_i x_{i-1} + a_i x_i + c_i x_{i+1} = d_i,
 *   a = main diagonal, b = sub-diagonal (b[0] is ignored), c = super-diagonal (c[n-1] is
 *   ignored).  Rows are 0-based.
 * - The matrix must be factorizable without pivoting: every matrix whose Hermitian part is
 *   positive definite (all Crank-Nicolson matrices with a real potential) and every strictly
 *   diagonally dominant matrix qualifies.  There is no pivoting, as in the paper.
 * - Work is enqueued asynchronously on the caller's stream (a hipStream_t passed as void*;
 *   NULL is the default stream).  Argument errors are reported synchronously with a negative
 *   status and nothing is enqueued.  A zero or non-finite pivot makes the solution
 *   non-finite; the kernels then raise a sticky device flag that cn_get_status reports as
 *   CN_NUMERICAL_BREAKDOWN.  The library never aborts the process.
 * - Workspace: the handle owns a device workspace that grows on demand.  Inside HIP graph
 *   capture nothing may be allocated: call cn_reserve with the same layout first, else the
 *   call returns CN_ERR_NOT_RESERVED.  Growing a workspace frees the old one only while no
 *   call of the handle has been captured; after the first captured call, replaced buffers are
 *   kept until cn_destroy, so every graph captured on the handle stays valid until then
 *   (cn_handle_info reports how many are kept).
 * - Threading: a handle is used by one host thread at a time.  Calls that overlap on
 *   different streams of one handle share its workspace and must not run concurrently.
 * - All arithmetic is FP64.  Results are deterministic: no floating-point atomics.
 */
#ifndef CNTRI_H
#define CNTRI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cn_handle_s* cn_handle_t;
typedef void* cn_stream_t; /* hipStream_t */

typedef enum {
  CN_OK = 0,
  CN_NUMERICAL_BREAKDOWN = 1, /* a zero or non-finite pivot was met (sticky, per handle)  */
  CN_ERR_INVALID_ARG = -1,    /* null pointer, bad size, stride or offsets                 */
  CN_ERR_UNSUPPORTED = -2,    /* valid request the library does not implement               */
  CN_ERR_NO_MEMORY = -3,      /* device allocation failed                                   */
  CN_ERR_HIP = -4,            /* a HIP runtime call failed                                  */
  CN_ERR_NOT_RESERVED = -5,   /* workspace would have to grow during graph capture          */
  CN_ERR_SCRATCH_TOO_SMALL = -6, /* cn_tridiag_solve_noalloc: the layout needs more device
                                  memory than the library's fixed scratch array holds          */
  CN_ERR_WAIT_TIMEOUT = -7    /* cn_get_status: the workgroups of a resident propagation
                                 gave up waiting on each other (other work on the GPU kept
                                 some from running); its state is unspecified               */
} cn_status;

/* Shape of the batch of independent systems handled by one call.
 * Uniform batch (offsets == NULL): system s, row i lives at element
 *     s * batch_stride + i * elem_stride
 * of every array (a, b, c, d, x, psi, V, xgrid).  elem_stride = 1, batch_stride = n is the
 * contiguous layout (ADI x-lines); elem_stride = batch, batch_stride = 1 is the interleaved
 * layout (ADI y-lines).  The rows of different systems must not overlap.
 * Uneven batch (offsets != NULL): system s owns rows offsets[s] .. offsets[s+1]-1 of every
 * array, packed contiguously; n, elem_stride and batch_stride are ignored.  offsets is a HOST
 * array of batch+1 non-decreasing values starting at 0 (empty systems are allowed). */
typedef struct {
  int64_t n;
  int64_t batch;
  int64_t elem_stride;
  int64_t batch_stride;
  const int64_t* offsets;
  int32_t partition;       /* rows per first-level partition (one workgroup tile); a power
                              of two in [32, 16384]; 0 = automatic.  Tiles exist for 64 to
                              4096 rows (64: one row per lane, explicit solves only); the
                              explicit solve of uniform batches also takes 8192 and 16384,
                              partitions of 2 or 4 chunks of 4096 rows that one workgroup
                              reduces in turn (its second pass reads each chunk twice);
                              sizes without tiles for the call's source return
                              CN_ERR_UNSUPPORTED.  Uneven batches: 0 =
                              one launch per length class for systems of up to 4096 rows
                              and two passes over 2048-row tiles for longer ones; > 0 = one
                              persistent launch over all systems with that tile            */
  int32_t rows_per_thread; /* rows per innermost block (2, 4, 8 or 16); 0 = automatic      */
  int32_t shared_coefficients; /* uniform batches only: 1 = every system reads the
                              coefficients of system 0 (a, b, c of cn_tridiag_solve; V and
                              xgrid of cn_step / cn_propagate), so the batch is several
                              right-hand sides of one matrix, whose coefficients are read
                              from one system's elements; 0 = each system its own.  Entry
                              points that accumulate per-system gradients or materialise
                              per-system arrays (adjoints, cn_assemble, cn_rhs) return
                              CN_ERR_UNSUPPORTED for 1                                       */
  int32_t levels;          /* partition levels before the RS stage (Sec. 4.1.6, Eq. (6);
                              Sec. 5.5.1): 0 = automatic (the reduced systems are partitioned
                              again until one tile holds them); L in 1..8 = the caller's
                              systems and the reduced systems of the first L-1 levels are
                              partitioned into tiles, and the reduced system left after L
                              levels is solved by the serial RS stage of Table 1 (Thomas's
                              elimination, one thread per system).  A system that fits one
                              tile at some level needs no further level.  Zero-initialise the
                              struct so that levels is 0 by default.                         */
} cn_layout;

/* Crank-Nicolson operator of Sec. 2, Eqs. (2)-(4) on a uniform grid with Dirichlet walls:
 *   H = -1/2 d^2/dx^2 + v,  v_j = v_scale * V_j + (xgrid ? xgrid_j * E : 0),
 *   three-point Laplacian, tau = dt/2, kappa = tau / (2 dx^2):
 *   T = 1 + i tau H: diagonal 1 + i tau (1/dx^2 + v_j), off-diagonals -i kappa.
 * V and xgrid are DEVICE arrays with the layout of psi.  dx_per_system (DEVICE, batch values)
 * overrides dx when non-NULL.
 * absorb (DEVICE, layout of psi, values W_j >= 0 expected) or NULL: an absorbing potential,
 * v_j - i W_j, which makes H non-Hermitian.  T's diagonal becomes 1 + tau W_j + i tau (...) and
 * the explicit side is 1 - i tau H (diagonal 1 - tau W_j - i tau (...)), which is no longer
 * T^dagger: the step stays the Cayley form (1 + i tau H)^{-1} (1 - i tau H).  cn_assemble,
 * cn_rhs, cn_step, cn_propagate, cn_step_adjoint and cn_propagate_adjoint take it.  The steps
 * run the fused kernels with W read beside V (one pass per step in cn_propagate over two-pass
 * plans, as for real potentials; 4 rows per lane); a layout whose plan needs a configuration
 * these kernels are not built for (explicit partitions with 8 or 16 rows per lane), or
 * CN_ABSORB_FUSED=0 in the environment, runs the step materialised instead (cn_assemble, cn_rhs
 * and cn_tridiag_solve's kernels through a handle buffer of 4 * span complex values, allocated
 * on the first such call for a layout, so a captured call needs one call outside capture
 * first, else CN_ERR_NOT_RESERVED; the adjoints then return CN_ERR_UNSUPPORTED).  In reverse
 * mode T^H = 1 + tau W - i tau (...) and B^H = 1 - tau W + i tau (...) for B = 1 - i tau H:
 * the operators of a step with dt -> -dt and W -> -W.  cn_autotune returns CN_ERR_UNSUPPORTED
 * for it, as does a layout with shared coefficients.  Zero-initialise the struct so that absorb
 * is NULL by default. */
typedef struct {
  const double* V;
  double v_scale;
  double dx;
  const double* dx_per_system;
  double dt;
  const double* xgrid;
  const double* absorb;
} cn_operator;

/* Partial waves of an atom in a field along z, expanded in the m = 0 spherical harmonics (the
 * radial systems of Sec. 3): radial functions psi_l(r_j), l = l0 .. l0+nl-1, on r_j = j dr
 * (j = 1..nr; psi = 0 at r = 0 and at r = (nr+1) dr), stored l-major: element (l, j) at
 * (l - l0) * nr + j - 1.  V: DEVICE, nr values V(r_j), real. */
typedef struct {
  int64_t nr;
  int64_t l0;
  int64_t nl;
  const double* V;
  double dr;
  double dt;
} cn_radial;

/* Host-only check of a layout (no device access): CN_OK, or the negative status that every
 * entry point would return for it (null layout, batch < 1, n < 1, strides < 1, systems that
 * share elements, offsets not starting at 0 or decreasing, a partition that is not a power of two
 * in [32, 16384], rows_per_thread not in {0, 2, 4, 8, 16}, shared_coefficients not 0 or 1,
 * levels not in 0..8;
 * CN_ERR_UNSUPPORTED for shared coefficients in an uneven batch). */
cn_status cn_check_layout(const cn_layout* layout);

cn_status cn_create(cn_handle_t* handle, int device);
cn_status cn_destroy(cn_handle_t handle);
const char* cn_status_string(cn_status status);

/* Builds the plans for this layout and grows the workspaces so that later calls with the same
 * layout allocate nothing (required before HIP graph capture).  For cn_propagate_adjoint under
 * capture this covers the fused recursion; its dE rows need one call outside capture first
 * (they are sized by the segment length K). */
cn_status cn_reserve(cn_handle_t handle, const cn_layout* layout);

/* x = T^{-1} d for every system of the batch: the N-shaped partition method (Sec. 4,
 * Table 1) -- partition-local RD+JD and RU+JU sweeps, the reduced system on the joint
 * lines solved by nesting the same method (Sec. 4.1.6, Eq. (6)) and, at the top, the RS
 * stage; then SS back-substitution on every level.  x may alias d; a, b, c are read only. */
cn_status cn_tridiag_solve(cn_handle_t handle, const cn_layout* layout, const void* a,
                           const void* b, const void* c, const void* d, void* x,
                           cn_stream_t stream);

/* cn_tridiag_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same plan and kernels,
 * with the plan's tables and workspace in a fixed device array of the library instead of the
 * handle's workspace.  The array holds 32 MiB (33554432 bytes) per GPU, is set up by cn_create
 * and kept until the process ends; the call allocates no device memory (the plan of a new
 * layout is built in host memory on its first call) and copies the plan's tables into the
 * array on the caller's stream before the kernels.  Arguments, layouts and results are those of
 * cn_tridiag_solve (x may alias d; the automatic or explicit partition of the layout, never an
 * autotuned one).  A layout whose tables and workspace exceed the array returns
 * CN_ERR_SCRATCH_TOO_SMALL with nothing enqueued (a single contiguous system of up to about
 * 2^28 rows fits; cn_tridiag_solve takes any size).  Every call on one GPU, from any handle or
 * stream, uses that GPU's one array: calls that overlap in time on a GPU race and must be
 * ordered by the caller (for example, issued on one stream).  Nothing in the array needs to
 * start at zero; each call rewrites what it reads. */
cn_status cn_tridiag_solve_noalloc(cn_handle_t handle, const cn_layout* layout, const void* a,
                                   const void* b, const void* c, const void* d, void* x,
                                   cn_stream_t stream);

/* Reverse mode of cn_tridiag_solve.  Given x = T^{-1} d and gx, the gradient of a real loss
 * with respect to x in the (d/dRe + i d/dIm) convention, writes
 *   gd = lambda = T^{-H} gx   (solved with the same partitioned method on T^H),
 *   ga_i = -lambda_i conj(x_i),  gb_i = -lambda_i conj(x_{i-1}),  gc_i = -lambda_i conj(x_{i+1}).
 * ga, gb, gc may each be NULL.  gb[0] and gc[n-1] are written as 0. */
cn_status cn_tridiag_solve_adjoint(cn_handle_t handle, const cn_layout* layout, const void* a,
                                   const void* b, const void* c, const void* x, const void* gx,
                                   void* gd, void* ga, void* gb, void* gc, cn_stream_t stream);

/* Materialised coefficient assembly of T (a, b, c; b[0] = c[n-1] = 0) for the layout. */
cn_status cn_assemble(cn_handle_t handle, const cn_layout* layout, const cn_operator* op,
                      double E, void* a, void* b, void* c, cn_stream_t stream);

/* Materialised explicit half-step d = (1 - i tau H) psi (Sec. 2, Eq. (3)). */
cn_status cn_rhs(cn_handle_t handle, const cn_layout* layout, const cn_operator* op, double E,
                 const void* psi, void* d, cn_stream_t stream);

/* One Crank-Nicolson step psi_out = T^{-1} (1 - i tau H) psi_in for every system, with the
 * explicit half-step fused into the reduction sweep (Sec. 5.3).  E is the field of this
 * step, used on both sides.  psi_out may alias psi_in. */
cn_status cn_step(cn_handle_t handle, const cn_layout* layout, const cn_operator* op, double E,
                  const void* psi_in, void* psi_out, cn_stream_t stream);

/* nsteps chained cn_step calls in place on psi.  E: HOST array of nsteps field
 * values, or NULL for no field.  If ckpt is non-NULL, the state before step k is copied to
 * ckpt + (k / K) * (rows of the layout) for every k divisible by K (K >= 1).
 * Systems solved in two passes (longer than one tile) run one fused pass per step: the
 * substitution of step k and the reduction of step k+1 (whose joint rows take the left
 * neighbour's explicit half-step term in the reduced system instead).  For one system whose
 * K tile joints fill more than half of a whole-system tile of 2 rows per lane of the pass's
 * workgroup (64 W < K <= 128 W), the pass's last workgroup also solves that reduced system, so
 * a step is one launch (CN_INLINE=0 turns this off).  The result equals the chain of cn_step
 * calls up to rounding (not bit for bit); CN_FUSE=0 in the environment turns the fusion off. */
cn_status cn_propagate(cn_handle_t handle, const cn_layout* layout, const cn_operator* op,
                       int64_t nsteps, const double* E, void* psi, void* ckpt, int64_t K,
                       cn_stream_t stream);

/* All nsteps Crank-Nicolson steps of one system in ONE launch (Sec. 2, Eqs. (2)-(4), each step
 * solved by the N-shaped partition of Sec. 4 with the explicit half-step fused, Sec. 5.3): the
 * kernel keeps one tile of T rows per workgroup resident for the whole sequence, its rows in
 * registers; per step every tile publishes its Table 1 slots, waits until all tiles have, solves
 * the reduced system on the tile joints itself and substitutes.  For sequences of mid-size
 * systems, whose chained passes are bound by launch and hand-over latency rather than by
 * memory.  Same result as cn_propagate without checkpoints, up to rounding.
 *   L: one contiguous system (batch 1, elem_stride 1, no offsets, no shared coefficients or
 *      levels; rows_per_thread 0 or 8; partition 0, or 512, 1024 or 2048 rows per tile).
 *   op: one dx (no dx_per_system); a real potential, or one with an absorbing part
 *       (op->absorb, the potential V - iW, as in cn_propagate).
 *   E: HOST, nsteps field values or null (zero field); uploaded with an asynchronous copy on
 *      the stream (so E != null cannot be captured into a graph: CN_ERR_UNSUPPORTED).  A
 *      launch without a field can be captured after cn_reserve of the layout (or one call
 *      outside capture), which sizes the handle's buffer for it.
 *   psi: DEVICE, n complex values, updated in place.
 *   ckpt: DEVICE or null; as in cn_propagate, the state before step k is written to
 *      ckpt + (k / K) * n for every k divisible by K (K >= 1): the first by a copy on the
 *      stream, the others from the kernel's registers.
 * CN_ERR_UNSUPPORTED also when the system needs more tiles than fit the GPU at once or than the
 * reduced solve of one workgroup takes (128 W joints: up to 2^20 rows), or when CN_RESIDENT=0
 * is set; then cn_propagate is the call.  The workgroups wait on each other: a launch that runs
 * beside other work on the same GPU (another stream, another resident propagation) may find
 * some of its workgroups unable to start; then the waits give up after a bound, the state is
 * left unspecified and cn_get_status returns CN_ERR_WAIT_TIMEOUT.  Enqueued on stream. */
cn_status cn_propagate_resident(cn_handle_t handle, const cn_layout* layout,
                                const cn_operator* op, int64_t nsteps, const double* E,
                                void* psi, void* ckpt, int64_t K, cn_stream_t stream);

/* One step of the adjoint recursion of cn_propagate (uniform batch of one system).
 * With psi_np1 = T_n^{-1} B_n psi_n, B_n = 1 - i tau H_n, and g_np1 the gradient at psi_np1:
 *   lambda = T_n^{-H} g_np1   (T_n^H = B_n for real v),
 *   g_n = B_n^H lambda        (= T_n lambda for real v),
 *   dV_accum_j += v_scale * tau * Im(conj(lambda_j) (psi_n,j + psi_np1,j)),
 *   dE_partial[0] = sum_j xgrid_j * tau * Im(conj(lambda_j) (psi_n,j + psi_np1,j))
 * (dE_partial may be NULL; it needs xgrid).  The sum is deterministic. */
cn_status cn_step_adjoint(cn_handle_t handle, const cn_layout* layout, const cn_operator* op,
                          double E, const void* psi_n, const void* psi_np1, const void* g_np1,
                          void* g_n, double* dV_accum, double* dE_partial, cn_stream_t stream);

/* One Lie-split step of the partial waves (Sec. 3): first, for every l, the Crank-Nicolson step
 * in r with H_l = -1/2 d^2/dr^2 + V(r) + l(l+1)/(2 r^2) -- the N-shaped solve of nl contiguous
 * systems of nr rows (cn_step's kernels, with the centrifugal potential written by a kernel of
 * the library into a handle buffer); then, for every r_j, the Crank-Nicolson step in l with the
 * length-gauge coupling H_E = E r_j C, C_{l,l+1} = C_{l+1,l} = (l+1)/sqrt((2l+1)(2l+3)) (the
 * matrix of cos(theta)), whose tridiagonal systems (one per r_j, nl rows, interleaved with
 * stride nr) are solved by the column kernels with their rows and right-hand sides built from
 * psi in-kernel (nr >= 64), or, for fewer radial points, assembled into the handle buffer and
 * solved by cn_tridiag_solve's kernels.  E = 0 skips the second part (it is the identity).
 * psi_out may alias psi_in.  The handle buffer (nl*nr*8 bytes, 72 with fewer than 64 radial
 * points) is allocated on the first call for a size, so a captured call needs one call outside
 * capture first (and cn_reserve of the two layouts: contiguous nr x nl, and n = nl, batch =
 * nr, elem_stride = nr, batch_stride = 1), else CN_ERR_NOT_RESERVED. */
cn_status cn_radial_step(cn_handle_t handle, const cn_radial* op, double E, const void* psi_in,
                         void* psi_out, cn_stream_t stream);

/* Reverse mode of cn_propagate with checkpoints, for a uniform layout.  ckpt holds the states
 * that cn_propagate stored before every step k with k % K == 0 (same layout, one span each);
 * seg is scratch for K+1 states.  On entry g is the gradient of a real loss at the final state
 * ((d/dRe + i d/dIm) convention); on return it is the gradient at the initial state.  Each
 * segment of K steps is recomputed forward from its checkpoint; the recursion then runs
 * backwards through it on g itself, g_N = g and
 *   g_k = B_k^H lambda_k,  lambda_k = T_k^{-H} g_{k+1},  i.e.  g_k = T_k^{-H} B_k^H g_{k+1}
 *   (for real v: (1 - i tau H_k)^{-1} (1 + i tau H_k) g_{k+1}): a Crank-Nicolson step with
 *   dt -> -dt (and W -> -W) and E_k on both sides,
 * with lambda_k = (g_k + g_{k+1}) / 2, accumulating
 *   dV_accum_j += v_scale tau Im(conj(lambda_k,j)(psi_k,j + psi_k+1,j))   (may be NULL)
 *   dE[k] = sum_j xgrid_j tau Im(conj(lambda_k,j)(psi_k,j + psi_k+1,j))   (needs xgrid; may be NULL)
 * in fixed order; g_0 is the result.  Two-pass plans run the recompute and the recursion as
 * fused passes (see cn_propagate).  With two or more segments and a stream that is
 * not being captured, the recompute of segment s-1 runs on a second stream of the handle while
 * the recursion runs through segment s; the handle then keeps a second segment buffer and a
 * second workspace (allocated on first use).  The results are the same in either form; the
 * call is ordered on the caller's stream as usual.  Under graph capture the segments run one
 * after the other on the caller's stream, as the same fused chain when the second workspace
 * exists (cn_reserve, or an earlier call), else one step at a time (equal up to rounding). */
cn_status cn_propagate_adjoint(cn_handle_t handle, const cn_layout* layout,
                               const cn_operator* op, int64_t nsteps, const double* E,
                               const void* ckpt, int64_t K, void* seg, void* g,
                               double* dV_accum, double* dE, cn_stream_t stream);

/* The reverse mode of cn_propagate without checkpoints.  The CN step of Sec. 2 is invertible,
 * so the forward states are rebuilt backwards from the final state psi_T,
 * psi_k = (1 - i tau H_k)^{-1} (1 + i tau H_k) psi_{k+1} -- a CN step with dt -> -dt and the
 * field E_k on both sides, the exact inverse of the forward step -- one
 * segment of K steps at a time into seg, beside the gradient recursion of cn_propagate_adjoint
 * (same arguments and results otherwise: g in place from the gradient at psi_T to the gradient
 * at psi_0, dV accumulated, dE written).  The rebuild of the next segment runs on a second
 * stream while the recursion works through the current one, as the checkpoint recompute does.
 * Memory: seg holds min(K, nsteps) + 1 states; no trajectory is stored.  Rounding of the
 * rebuilt states grows with the number of steps (the steps are unitary, so it grows slowly;
 * about 1e-13 relative after 2000 steps of 2^20 rows).  psi_T: DEVICE, layout of g, read
 * only.  An absorbing potential (op->absorb) returns CN_ERR_UNSUPPORTED: its inverse step
 * amplifies. */
cn_status cn_propagate_adjoint_reconstruct(cn_handle_t handle, const cn_layout* layout,
                                           const cn_operator* op, int64_t nsteps,
                                           const double* E, const void* psi_T, int64_t K,
                                           void* seg, void* g, double* dV, double* dE,
                                           cn_stream_t stream);

/* Autotuner: times the automatic plan and the candidate tile configurations (rows per
 * first-level partition and per innermost block; for uneven batches the persistent launches)
 * of this layout on the caller's data and keeps the fastest for later calls with the same
 * layout whose partition and rows_per_thread are 0.  cn_mode = 0 times
 * cn_tridiag_solve(a, b, c, d -> x); cn_mode = 1 times cn_step(op, E, psi_in = d -> psi_out = x)
 * and ignores a, b, c; cn_mode = 2 times a sequence of 8 steps in place on x (copied from d
 * before each timing), as cn_propagate runs it (one fused pass per step over two-pass plans),
 * and reports the time per step -- the choice for sequences, where the per-step latency
 * decides.  Modes 1 and 2 tune the same automatic layout (the last call wins).  x is
 * overwritten and must not alias d.  A text report of the median timings is written to report
 * (may be NULL).  Not allowed during graph capture. */
cn_status cn_autotune(cn_handle_t handle, const cn_layout* layout, int cn_mode,
                      const cn_operator* op, double E, const void* a, const void* b,
                      const void* c, const void* d, void* x, char* report, int64_t report_len,
                      cn_stream_t stream);

/* Persistent autotune cache.  path names a JSON file (read now if it exists, rewritten by every
 * later cn_autotune of this handle), or NULL / "" to stop using one.  Entries are keyed by the
 * layout's class: the device architecture (hipDeviceProp gcnArchName without its feature
 * suffix), the source (solve or CN step) and the layout's shape in power-of-two buckets (rows
 * per system and batch for uniform batches, with unit or other strides and shared
 * coefficients; batch, total rows and longest system for uneven ones), plus levels.  A layout
 * whose partition and rows_per_thread are 0 takes the cached configuration of its class when
 * the handle has no tuned plan for it in memory.  Host only (no device access); returns
 * CN_ERR_INVALID_ARG when autotune cannot write the file. */
cn_status cn_tune_cache(cn_handle_t handle, const char* path);

/* Device memory held by the handle (workspaces and plan tables, excluding retired buffers),
 * the number of buffers retired after graph capture (freed by cn_destroy), and whether a call
 * of the handle has been captured.  Each output pointer may be NULL.  Host only. */
cn_status cn_handle_info(cn_handle_t handle, int64_t* device_bytes, int64_t* retired_buffers,
                         int32_t* captured);

/* Plan log.  With cn_profile(h, 1), every launch of a plan run by cn_tridiag_solve, cn_step
 * (one step) and the adjoint solves outside graph capture is bracketed by HIP events on the
 * caller's stream (host-side event objects are created per launch); cn_profile(h, 0) stops it.
 * cn_profile_report waits for the recorded launches and writes one line per launch, in launch
 * order: "L<level> <phase> <tile T(M,W) or -> grid=<x>x<y> threads=<n> ms=<duration>", the
 * stage times of the method (partition reductions, reduced systems, substitutions, the serial
 * RS stage); then it clears the log.  buf is truncated to buflen. */
cn_status cn_profile(cn_handle_t handle, int enable);
cn_status cn_profile_report(cn_handle_t handle, char* buf, int64_t buflen);

/* Synchronises the stream, returns CN_ERR_WAIT_TIMEOUT if a resident propagation of this
 * handle gave up a wait, else CN_NUMERICAL_BREAKDOWN if any kernel of this handle met a
 * non-finite result since the last call (and clears the flags), else CN_OK. */
cn_status cn_get_status(cn_handle_t handle, cn_stream_t stream);

/* Version string and the plan chosen for a layout (for logs and benchmarks; with CN_LOG=1 in
 * the environment every plan is also described on stderr when it is built).  cn_mode 0: the
 * plan of cn_tridiag_solve; 1: the Crank-Nicolson plan (real potential), whose description ends
 * with how cn_propagate chains its steps: one fused pass per step, and whether the pass's last
 * workgroup also solves the reduced system of the tile joints (one system whose joints fit one
 * whole-system tile), which saves a launch per step; 2: the plan of the fused steps with an
 * absorbing potential (CN_ERR_UNSUPPORTED for a layout whose absorbing steps run
 * materialised).  Other values: CN_ERR_INVALID_ARG. */
const char* cn_version(void);
cn_status cn_describe_plan(cn_handle_t handle, const cn_layout* layout, int cn_mode, char* buf,
                           int64_t buflen);

#ifdef __cplusplus
}
#endif

#endif /* CNTRI_H */
