/*
 * s7: BiCGStab for 7-point variable-coefficient stencil systems on MI355X.
 *
 * C ABI of libs7.so.  Plain pointers and sizes only.
 *
 * The problem (paper: "Fast Stencil-Code Computation on a Wafer-Scale
 * Processor", SC20).  Eq. (1), section III: solve A x = b.  A is the 7-point
 * finite-difference operator on an nx x ny x nz structured mesh (section IV,
 * "SpMV (3D)").  Each row has a main diagonal and six off-diagonals named by
 * direction and sign, as the paper names its coefficient vectors:
 *
 *   (A v)(i,j,k) = diag v(i,j,k)
 *                + xm v(i-1,j,k) + xp v(i+1,j,k)
 *                + ym v(i,j-1,k) + yp v(i,j+1,k)
 *                + zm v(i,j,k-1) + zp v(i,j,k+1).
 *
 * Values outside the mesh are zero (Dirichlet ghosts).  The coefficients of
 * those outward links are ignored, whatever their values.
 *
 * Layout.  Every per-cell array is [nz][ny][nx], x fastest: cell (i,j,k) is
 * element i + nx*(j + ny*k).  Coefficients come as seven arrays in the order
 * {diag, xm, xp, ym, yp, zm, zp}.  N = nx*ny*nz must be at most 2^31 - 2^21
 * (cell indices are 32-bit, with headroom for the grids that stride over them).
 *
 * Memory.  Every array argument is a DEVICE pointer owned by the caller, for
 * example a PyTorch tensor.  The library allocates no device memory of its
 * own (the batch engine reads its states through small pinned host
 * buffers, kept for the life of the process).  Scratch comes from a caller-provided workspace of the size that
 * s7_workspace_bytes() reports, 256-byte aligned.
 *
 * Streams.  `stream` is a hipStream_t passed as void*; 0 means the null
 * stream.  s7_stencil_apply is asynchronous on it.  The solvers are
 * synchronous: they return when the result is in x.
 *
 * Errors.  Every function returns an s7_status.  No function aborts or
 * throws across the ABI.  s7_last_error() gives a message for the calling
 * thread's last failure.
 */
#ifndef S7_H
#define S7_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
} s7_dims;

enum s7_status {
    S7_OK = 0,
    S7_NOT_CONVERGED = 1, /* iteration cap reached; x holds the last iterate */
    S7_BREAKDOWN = 2,     /* see s7_info.reason; x holds the last iterate */
    S7_EINVAL = -1,       /* null pointer, dim < 1, N > 2^31 - 2^21, rtol <= 0 or NaN,
                             max_iter < 0, workspace too small or misaligned */
    S7_ENOMEM = -2,       /* request larger than the whole queue arena */
    S7_EHIP = -3,         /* HIP runtime error (message in s7_last_error) */
    S7_EAGAIN = -4,       /* poll: not finished yet */
    S7_ENOTFOUND = -5     /* unknown ticket */
};

/* Breakdown reasons.  Each test is exact, with no threshold. */
enum s7_reason {
    S7_REASON_NONE = 0,
    S7_REASON_RHO_ZERO = 1, /* (r0, r_{i+1}) == 0 */
    S7_REASON_RS_ZERO = 2,  /* (r0, s_i) == 0 */
    S7_REASON_YY_ZERO = 3,  /* (y_i, y_i) == 0 */
    S7_REASON_NONFINITE = 4 /* a scalar became Inf or NaN */
};

/*
 * Precision of the inner iteration.
 * S7_FP32: coefficients and Krylov vectors are stored and computed in FP32.
 *   Inner products accumulate FP32 products in FP64.  b and x are FP64 at
 *   the boundary.
 * S7_BF16_IR and S7_FP16_IR: coefficients and Krylov vectors are stored in
 *   BF16 or FP16 and computed in FP32, with FP64 inner products.  This is the
 *   paper's mixed 16/32-bit scheme (section IV "AllReduce"; Table I).  It
 *   runs inside an FP64 iterative-refinement loop, the correction scheme the
 *   paper names (section VI-B).  Each outer step forms the true residual
 *   r = b - A x in FP64 with the exact FP32 coefficients, solves
 *   A d = r / scale to the inner tolerance, and updates x += scale * d in FP64.
 */
enum s7_prec { S7_FP32 = 0, S7_BF16_IR = 1, S7_FP16_IR = 2 };

typedef struct {
    int32_t jacobi;         /* 1 (default): left diagonal (Jacobi) scaling, so the
                               iterated matrix has a unit diagonal (section IV,
                               first paragraph); 0: iterate on A as given */
    int32_t graph_iters;    /* iterations per captured hipGraph launch; 0 = auto */
    int32_t stream_blocks;  /* workgroups of the streaming passes; 0 = auto (at most 256);
                               capped at 1024 */
    int32_t chunk_cells;    /* batched/queue: cells per work item of the persistent
                               kernel, rounded up to a multiple of 1024, at most 2^24;
                               0 = 16384, with the chunks of small systems halved (down
                               to 4096 cells, up to 32 chunks) while the resident set
                               has fewer work items than the grid has workgroups.  No
                               result depends on it. */
    int32_t profile;        /* 1: launch without graphs, time every pass with HIP
                               events into s7_info.pass_ms */
    int32_t inner_max_iter; /* IR: inner iteration cap per outer step; 0 = 100 */
    int32_t outer_max_iter; /* IR: outer step cap; 0 = 30 */
    int32_t schedule;       /* single-system solve: 1 three passes per iteration (q = r - alpha s
                               formed on the fly where it is used, never stored), 2 four
                               passes (q stored by a streaming pass), 3 three passes whose
                               stencil passes give each thread two x-adjacent cells (meshes with
                               an even nx; 1 otherwise), 5 three passes whose stencil passes
                               stage the operand of a 4096-cell tile and one mesh row on
                               either side in LDS (meshes with an even nx of at most 4096;
                               3 otherwise); 0 = 5 on meshes of at least 2^22 cells where
                               it applies, else 3.  With tune = 1, lds_tile and xcd_run left at
                               0 are tuned together with the schedule. */
    int32_t tune;           /* 1: the fields left at 0 among schedule and stream_blocks
                               (single solve) and chunk_cells (batched) take autotuned values
                               for the problem's size class.  An untuned class is timed first
                               on synthetic data in the caller's workspace (the caller's arrays
                               are not touched); the choice is kept for the process and, if
                               the environment variable S7_TUNE_CACHE names a file, appended
                               there and read back by later processes.  The request queue
                               does not tune: its resident set changes every step, and each
                               request's sums must not depend on it.  0: fixed defaults. */
    int32_t split_cells;    /* systems of at least this many cells run on the single-system
                               path instead of the batch engine: in the request queue on a
                               second stream, one at a time; in the batched solve after the
                               shared launch.  0 = 2^21, -1 = never */
    double inner_rtol;      /* IR: inner relative tolerance; 0 = 1e-2 (BF16), 5e-3 (FP16) */
    int32_t xcd_run;        /* single-system stencil passes (all forms): consecutive workgroup
                               tiles that one XCD sweeps in a row (workgroups are dealt to the
                               eight XCDs in turn, each with its own L2); k > 1: runs of k
                               tiles, -1: an eighth of a mesh plane's tiles (each XCD sweeps one
                               band of every plane), 0 or 1: plain order (default; the runs
                               measured no faster).  Results do not depend on it. */
    int32_t lds_tile;       /* schedule 5: cells of a workgroup's tile, 2048, 4096 or 8192
                               (8, 16 or 32 cells per thread); 0 = 4096, or the autotuned
                               value with tune = 1.  A tile whose LDS (tile + 2 nx floats) does
                               not fit takes the largest of 4096 and 2048 that does. */
} s7_options;

typedef struct {
    int32_t iters;       /* BiCGStab iterations; for IR, summed over outer steps */
    int32_t outer_iters; /* IR outer steps (1 for S7_FP32) */
    int32_t status;      /* s7_status of this solve */
    int32_t reason;      /* s7_reason when status == S7_BREAKDOWN */
    double rel_res_rec;  /* recurrence residual ||r_i|| / ||b|| of the iterated
                            (scaled) system at exit */
    double rel_res_true; /* ||b - A x|| / ||b|| of the unscaled system, FP64, at exit */
    double t_ms;         /* solver wall time (queue: submit to completion) */
    double t_wait_ms;    /* queue: submit to admission; 0 otherwise */
    double pass_ms[4];   /* profile: summed time of the iteration's kernels P1, P2a, P2b, P3
                            (P1 and P2b include the finishing kernel of a split sum) */
    int32_t pass_count[4];
    int32_t schedule;    /* the schedule it ran: 1 three passes, 2 four passes, 3 three
                            passes on cell pairs, 4 the pipelined solve, 5 three passes
                            with LDS-staged stencil operands.  Batched and queue engine solves run
                            three phases per iteration: 3 if nx is even, else 1; the
                            2D 9-point solves (single, batched, queued) report 1 */
    int32_t lds_tile;    /* schedule 5: the tile the staged passes ran with; 0 otherwise */
    int32_t xcd_run;     /* single-system solves: the XCD tile order the stencil passes ran
                            with (s7_options.xcd_run, or the tuned value); 0 otherwise */
    int32_t reserved;
} s7_info;

/* Fills *opt with the defaults described above. */
void s7_default_options(s7_options *opt);

/* Message for the calling thread's last failed call ("" if none). */
const char *s7_last_error(void);

/* ABI version: 0x010000 * major + 0x100 * minor. */
int32_t s7_version(void);

/*
 * u = A v.  This is the SpMV of section IV, "SpMV (3D)": six coefficient
 * times neighbour products plus the diagonal term.  Here the diagonal is
 * explicit: no unit-diagonal assumption.
 * coef: 7 device pointers {diag, xm, xp, ym, yp, zm, zp}, N floats each.
 * v: N floats in.  u: N floats out.  u must not alias v.
 * FP32 arithmetic with a fixed summation order:
 *   diag v + xm v(i-1) + xp v(i+1) + ym v(j-1) + yp v(j+1) + zm v(k-1) + zp v(k+1).
 * Asynchronous on `stream`.
 */
int s7_stencil_apply(s7_dims d, const float *const coef[7], const float *v, float *u,
                     void *stream);

/*
 * Bytes of workspace s7_bicgstab_solve needs for these dims, precision and
 * options.  opt may be NULL for the defaults.  Returns 0 for invalid dims.
 */
size_t s7_workspace_bytes(s7_dims d, int32_t prec, const s7_options *opt);

/*
 * Solves A x = b by BiCGStab.  This is Algorithm 1 ("Standard BiCGStab")
 * with r0 = b - A x0 and the shadow vector r0 fixed.  Optional Jacobi
 * scaling is applied (section IV).
 *   coef  7 device float arrays (see layout above), not modified.
 *   b     N device doubles.
 *   x     N device doubles: x0 on entry, the solution (or last iterate) on exit.
 *   rtol  relative tolerance, > 0.  The iteration stops when the recurrence
 *         residual ||r||/||b|| of the iterated system is <= rtol.  That is
 *         checked after each full step, and on ||q|| after the q-step.  For
 *         the IR precisions the outer loop stops on the true FP64 residual.
 *   max_iter  cap on BiCGStab iterations (>= 0).  For IR it caps the inner
 *         iterations summed over the outer steps.
 *   ws, ws_bytes  caller workspace, at least s7_workspace_bytes(), 256-byte
 *         aligned.  Its contents are scratch.
 *   opt   NULL for defaults.  info: optional, filled on return.
 * b == 0 gives x = 0, 0 iterations, S7_OK.  max_iter == 0 leaves x = x0 and
 * returns S7_NOT_CONVERGED, unless x0 already meets rtol.  The schedule and
 * the streaming split (options, or autotuned with opt->tune) change only the
 * order of rounding, not the method.
 */
int s7_bicgstab_solve(s7_dims d, const float *const coef[7], const double *b, double *x,
                      double rtol, int32_t max_iter, int32_t prec, void *ws, size_t ws_bytes,
                      const s7_options *opt, s7_info *info, void *stream);

/* Size of the fixed workspace of s7_bicgstab_solve_noalloc: 64 MiB per GPU. */
#define S7_NOALLOC_WS_BYTES (64u << 20)

/*
 * For callers that cannot allocate device memory (tight serving loops, code
 * that must not call hipMalloc): s7_bicgstab_solve with prec = S7_FP32 and
 * its workspace taken from a fixed 64 MiB array in device memory that the
 * library holds on each GPU it runs on until the process ends, instead of a
 * caller workspace.  The caller still provides coef, b and x, as for
 * s7_bicgstab_solve.  No device memory is allocated or freed: kernels are
 * launched directly (no hipGraph, no autotuning trials, no profiling events;
 * opt->tune and opt->profile are ignored), and the solver state is read back
 * with hipMemcpyAsync into host stack memory.  The results are bit for bit
 * those of s7_bicgstab_solve(prec = S7_FP32) with the same options and no
 * tuning.
 * Limit: s7_workspace_bytes(d, S7_FP32, opt) <= S7_NOALLOC_WS_BYTES (about a
 * million cells); a larger system returns S7_EINVAL.  The array keeps the
 * last call's contents; every call clears what must start at zero.  All calls
 * on one GPU share the array: calls that overlap in time on one GPU (other
 * host threads, other streams) race and must be serialised by the caller.
 * Synchronous, like s7_bicgstab_solve; same status codes.
 */
int s7_bicgstab_solve_noalloc(s7_dims d, const float *const coef[7], const double *b, double *x,
                              double rtol, int32_t max_iter, const s7_options *opt, s7_info *info,
                              void *stream);

/* Workspace for s7_bicgstab_solve_batched over these nsys systems. */
size_t s7_batched_workspace_bytes(int32_t nsys, const s7_dims *d, int32_t prec,
                                  const s7_options *opt);

/*
 * Solves nsys independent systems, of uneven mesh sizes, together in one
 * persistent launch.  This is the "many compact problems" use of section
 * VIII-B.  Per-system arguments are host arrays of length nsys:
 *   d[s]; coef[7*s + c], device float arrays in the order above; b[s] and x[s],
 *   device doubles; rtol[s]; max_iter[s].
 * info, if not NULL, is an array of nsys and receives each system's result.
 * All systems use precision prec.  The whole of each solve runs on the
 * device: the iterations (three phases each), and the refinement steps or the
 * FP32 epilogue.  Each system's sums are kept per unit of 1024 of its cells,
 * so its iterates depend only on that system: not on the rest of the batch,
 * nor on chunk_cells (the work-item size).  With opt->tune = 1 and
 * chunk_cells = 0 the work-item size and the persistent grid are autotuned
 * per size class.
 * A system of split_cells cells or more (default 2^21) is solved on its own
 * by the multi-kernel path of s7_bicgstab_solve, in its slice of the
 * workspace, after the shared launch; its iterates are those of
 * s7_bicgstab_solve with the same options.
 * Returns the worst status: a negative error, or else the largest of S7_OK,
 * S7_NOT_CONVERGED and S7_BREAKDOWN.
 */
int s7_bicgstab_solve_batched(int32_t nsys, const s7_dims *d, const float *const *coef,
                              const double *const *b, double *const *x, const double *rtol,
                              const int32_t *max_iter, int32_t prec, void *ws, size_t ws_bytes,
                              const s7_options *opt, s7_info *info, void *stream);

/* Workspace for s7_bicgstab_solve_pipelined (0 for invalid dims). */
size_t s7_workspace_bytes_pipelined(s7_dims d, const s7_options *opt);

/*
 * Pipelined BiCGStab (Cools and Vanroose, Parallel Computing 65, 2017), in the
 * form with one reduction per iteration: the iterates of Algorithm 1 in exact
 * arithmetic, with the matrix products carried by recurrences (s = A p,
 * z = A s, w = A r, t = A w, v = A z).  The paper uses the classical form;
 * this variant trades more vector traffic for fewer points where the
 * iteration waits on a global sum.  FP32 storage, FP64 inner products.  In
 * FP32 the recurrences drift from A, so every 10 iterations x (FP64) absorbs
 * the correction and r = b - A x (FP64), w, t, s, z, v and the scalars are
 * recomputed from their definitions (residual replacement).  A stop that the
 * recurrences decide is confirmed on that true residual at the next
 * replacement: S7_OK means the FP64 true residual of the iterated system
 * (Jacobi-scaled by default) is at most rtol.  If it is not, the iteration
 * continues from the replaced residual with the search direction restarted,
 * which lets the true residual fall below the FP32 storage floor (about 1e-7)
 * as in iterative refinement, until rtol or max_iter.  Readings as
 * s7_bicgstab_solve, except that the stopping test on r_i is taken in
 * iteration i's reduction (x_i is returned; the half iteration computed before
 * it is not applied).  Four passes per iteration (two streaming, two
 * stencil); info->schedule = 4.  Of the options it reads jacobi and
 * graph_iters.  Arguments, ownership and returns as s7_bicgstab_solve with
 * prec = S7_FP32.
 */
int s7_bicgstab_solve_pipelined(s7_dims d, const float *const coef[7], const double *b, double *x,
                                double rtol, int32_t max_iter, void *ws, size_t ws_bytes,
                                const s7_options *opt, s7_info *info, void *stream);

/* Workspace for s7_bicgstab_solve_batched_pipelined over these nsys systems
 * (0 for invalid arguments). */
size_t s7_batched_workspace_bytes_pipelined(int32_t nsys, const s7_dims *d, const s7_options *opt);

/*
 * The pipelined BiCGStab above for nsys independent systems in one persistent
 * launch: the many-compact-problems use of section VIII-B with the
 * one-reduction iteration.  In the persistent kernel each iteration is two
 * phases, so a system's workgroups hand off twice per iteration where the
 * classical batched solve hands off three times.  Phase A forms z at the
 * stencil's neighbour cells and v = A z, and takes all ten sums.  Phase B forms
 * w at the neighbour cells and t = A w, then updates r and d.  Residual
 * replacement runs every 10 iterations, and at once after a candidate stop.
 * The stop is verified on the FP64 true residual, as in
 * s7_bicgstab_solve_pipelined.  FP32 storage; each system's sums are kept per
 * unit of 1024 of its cells, so its iterates depend only on that system and
 * not on the rest of the batch or on chunk_cells.  Arguments are as for
 * s7_bicgstab_solve_batched with prec = S7_FP32.  Of the options it reads
 * jacobi, chunk_cells and split_cells.  A system of split_cells cells or
 * more is solved alone by s7_bicgstab_solve_pipelined in its slice of the
 * workspace.  info->schedule = 4.  Returns a negative error, or else the
 * worst status.
 */
int s7_bicgstab_solve_batched_pipelined(int32_t nsys, const s7_dims *d, const float *const *coef,
                                        const double *const *b, double *const *x, const double *rtol,
                                        const int32_t *max_iter, void *ws, size_t ws_bytes,
                                        const s7_options *opt, s7_info *info, void *stream);

/*
 * Request queue with continuous batching (serving form; section VIII-A names
 * the real-time use).  The caller supplies the device arena, which is the HBM
 * budget.  A request is admitted when its workspace fits in the arena.
 * Admitted requests join the resident batch between persistent-kernel
 * epochs.  Their Krylov state stays on the device until they finish.
 */
typedef struct s7_queue s7_queue;

typedef struct {
    s7_dims d;
    const float *coef[7]; /* device arrays, kept alive by the caller until done */
    const double *b;      /* device */
    double *x;            /* device; x0 on submit, solution when done */
    double rtol;
    int32_t max_iter;
    int32_t prec;         /* s7_prec */
} s7_request;

/* A 2D 9-point request (s7_queue_submit_2d9): an nx x ny mesh with the nine
 * coefficient arrays in the order {diag, w, e, s, n, sw, se, nw, ne}. */
typedef struct {
    int32_t nx, ny;
    const float *coef[9]; /* device arrays, kept alive by the caller until done */
    const double *b;      /* device */
    double *x;            /* device; x0 on submit, solution when done */
    double rtol;
    int32_t max_iter;
    int32_t prec;         /* s7_prec */
} s7_request_2d9;

/* Bytes at the head of a queue arena that hold the batch engine's tables
 * (3D 7-point and 2D 9-point requests share them). */
size_t s7_queue_table_bytes(void);

/*
 * Creates a queue over the caller's device arena (256-byte aligned), on the
 * current device.  The arena stays owned by the caller and must outlive the
 * queue.  Its head (s7_queue_table_bytes) holds the engine tables for up to
 * 2048 resident requests of either operator; the rest holds the admitted
 * requests' workspaces (s7_workspace_bytes of their dims and precision, or
 * s7_workspace_bytes_2d9 of their mesh).  opt->graph_iters sets the epoch: the most
 * iterations a resident request runs between two admission points; 0 (the
 * default) gives each request the iterations that fit a time slice of about
 * 2 ms at its size.
 * One serving thread and one non-blocking stream belong to the queue.
 * S7_EINVAL for a bad argument or an arena too small for the tables.
 */
int s7_queue_create(s7_queue **q, void *arena, size_t arena_bytes, const s7_options *opt);
/*
 * Copies the descriptor and returns a ticket.  The request's arrays must be
 * ready on the device (work that writes them has completed) and stay valid
 * until its result is collected.  Requests are admitted in submission order.
 * S7_ENOMEM if its workspace exceeds the arena (it could never be admitted);
 * S7_EINVAL for a bad argument; after a device error, that error.
 */
int s7_queue_submit(s7_queue *q, const s7_request *req, uint64_t *ticket);
/*
 * The same for a 2D 9-point request (section IV's operator, solved as by
 * s7_bicgstab_solve_2d9).  It shares the arena, the admission order and the
 * tickets with 3D requests; small ones run in the same persistent launches
 * as the 3D requests, meshes of split_cells cells or more on the
 * large-request thread.
 * Its workspace is s7_workspace_bytes_2d9 of its mesh and precision.
 */
int s7_queue_submit_2d9(s7_queue *q, const s7_request_2d9 *req, uint64_t *ticket);
/*
 * Non-blocking.  S7_EAGAIN while the request is queued or running; else the
 * request's s7_status, *info filled (t_ms: submit to completion, t_wait_ms:
 * submit to admission), and the ticket released: a second collection of the
 * same ticket returns S7_ENOTFOUND.
 */
int s7_queue_poll(s7_queue *q, uint64_t ticket, s7_info *info);
/* Blocks until the request is done, then collects it as s7_queue_poll does. */
int s7_queue_wait(s7_queue *q, uint64_t ticket, s7_info *info);
/*
 * Runs every submitted request to completion, stops the serving thread and
 * releases the queue (uncollected results are dropped).  Returns S7_OK, or
 * the device error that stopped the queue.  No other call on q may overlap it.
 */
int s7_queue_destroy(s7_queue *q);

/*
 * Synthetic problem generator, for benchmarks and tests on meshes too large
 * to build on the host.  It writes the seven coefficient arrays and x*, and
 * b = A x* in FP64.  Recipe: recipe 0 draws i.i.d. off-diagonals in
 * [-1, -0.5) and sets diag = fl32(sum|off| + 0.1).  Recipe 1 also scales
 * zm and zp by 1 + 9 s(k), a centred z-slab with smoothstep edges.  The
 * random numbers come from SplitMix64 (Steele, Lea, Flood 2014), indexed
 * by (seed, array, cell).  Any of coef[c], xstar and b may be NULL to skip it.
 * b needs all seven coef arrays and xstar.
 */
int s7_generate_problem(s7_dims d, uint64_t seed, int32_t recipe, float *const coef[7],
                        double *xstar, double *b, void *stream);

/*
 * Bandwidth probe (diagnostic).  These are STREAM-style kernels (McCalpin):
 * they measure the HBM rate that plain streaming code reaches, which is the
 * practical ceiling for the solver's roofline fractions.  n floats per buffer,
 * a multiple of 8, with 16-byte aligned device buffers.
 *   kind 0: read-only sum of a.  kind 1: c = a (copy).  kind 2: c = a + 0.5 b
 *   (triad).  kind 3: six n/2-float read streams (the halves of a, b and c) and
 *   two write streams (a, b updated in place).  This is the access pattern of
 *   the BiCGStab x/r update.
 * Add 4 to kind for non-temporal stores, 8 for non-temporal loads.
 * width: floats per access (1, 2 or 4).  blocks: grid size (256 threads each).
 * Asynchronous on `stream`.
 */
int s7_bandwidth_probe(int32_t kind, int32_t width, float *a, float *b, float *c, size_t n,
                       int32_t blocks, void *stream);

/*
 * P2 design probe (diagnostic).  This is the three-pass iteration's P2 of
 * Algorithm 1 (q = r - alpha s formed on the fly, y = A q, and the sums
 * (q,y), (y,y), (q,q), (r0,q), (r0,y)) on the stencil of section IV
 * ("SpMV (3D)").  It is written in the kernel designs that were measured
 * against the one the solver uses:
 *   kind 0: flat cell pairs, every neighbour of r and s loaded from memory;
 *   kind 1: one-plane tiles of 2048 cells, q staged in LDS with one row on
 *           either side and the z neighbours loaded from memory (the solver's
 *           staged form); param 1 is plain tile order, 0 is band-per-XCD order;
 *   kind 2: two-plane tiles (planes 2k and 2k+1 staged together, so the z
 *           neighbour between them comes from LDS); param as for kind 1;
 *   kind 3: z-march, in which a workgroup walks param planes of one 2048-cell
 *           in-plane tile, with q of the planes below and above in registers
 *           and the current plane in a double-buffered LDS ring.
 * coef: the six off-diagonal coefficients {w, e, s, n, b, t} of the
 * unit-diagonal (Jacobi-scaled) operator, with outward links zero on the faces.
 * r, s, rhat: device inputs; y: device output (n floats).  Every design writes
 * the same y bit for bit.  part: device buffer of at least
 * s7_p2_design_part_bytes() bytes, which receives five FP64 sums per workgroup
 * (their total is the five sums).
 * Runs one warm-up launch, then reps timed launches with HIP events on
 * `stream`.  *ms receives the average per launch.  The call waits for the
 * launches.  Limits: nx a multiple of 8 and at most 1024; all float arrays
 * 16-byte aligned.  Returns S7_EINVAL otherwise.
 */
size_t s7_p2_design_part_bytes(int32_t kind, int32_t param, s7_dims d);
int s7_p2_design_probe(int32_t kind, int32_t param, s7_dims d, const float *const coef[6], const float *r,
                       const float *s, const float *rhat, float alpha, float *y, double *part,
                       size_t part_bytes, int32_t reps, float *ms, void *stream);

/*
 * The 2D 9-point operator (section IV, "SpMV (2D)"; the paper sizes it at
 * 4800 x 4800 and 22800 x 22800 meshes).  On an nx x ny mesh, cell (i,j) is
 * element i + nx*j (x fastest) and
 *
 *   (A v)(i,j) = diag v(i,j) + w v(i-1,j) + e v(i+1,j) + s v(i,j-1) + n v(i,j+1)
 *              + sw v(i-1,j-1) + se v(i+1,j-1) + nw v(i-1,j+1) + ne v(i+1,j+1).
 *
 * Coefficients come as nine device float arrays in the order
 * {diag, w, e, s, n, sw, se, nw, ne}.  Values outside the mesh are zero and
 * the coefficients of those outward links are ignored.  nx*ny must be at
 * most 2^31 - 2^21.  Everything else (ownership, streams, errors) is as for the 3D calls.
 */

/* u = A v in FP32 (terms in the order above, fused multiply-adds).
 * Asynchronous on `stream`.  v and u must not alias. */
int s7_stencil9_apply(int32_t nx, int32_t ny, const float *const coef[9], const float *v, float *u,
                      void *stream);

/* Workspace for s7_bicgstab_solve_2d9 (0 for invalid dims or precision). */
size_t s7_workspace_bytes_2d9(int32_t nx, int32_t ny, int32_t prec, const s7_options *opt);

/*
 * BiCGStab (Algorithm 1, the readings of s7_bicgstab_solve) on the 2D 9-point
 * system; x holds x0 on entry and the solution on return, b and x FP64.
 * prec as for s7_bicgstab_solve: S7_FP32 stores and computes in FP32 with
 * FP64 inner products; S7_BF16_IR and S7_FP16_IR store in 16 bits inside FP64
 * iterative refinement (the same outer loop, tolerances and caps).  The
 * iteration is the three-pass schedule.  Of the options it reads jacobi,
 * profile, graph_iters, stream_blocks and the refinement fields.  Returns as
 * s7_bicgstab_solve.
 */
int s7_bicgstab_solve_2d9(int32_t nx, int32_t ny, const float *const coef[9], const double *b, double *x,
                          double rtol, int32_t max_iter, int32_t prec, void *ws, size_t ws_bytes,
                          const s7_options *opt, s7_info *info, void *stream);

/*
 * Synthetic 2D 9-point problem: off-diagonal a (a = 1..8, array id 19 + a)
 * is -(0.5 + m 2^-24) with m the top 23 bits of the SplitMix64 hash of
 * (seed, array id, cell); diag = fl32(sum |off| + 0.1), summed in FP64 in
 * the order above; x* as in s7_generate_problem; b = A x* in FP64.  Any of
 * coef[c], xstar and b may be NULL to skip it; b needs all nine and xstar.
 */
int s7_generate_problem_2d9(int32_t nx, int32_t ny, uint64_t seed, float *const coef[9], double *xstar,
                            double *b, void *stream);

/* Workspace for s7_bicgstab_solve_batched_2d9 over these nsys meshes
 * (0 for an invalid mesh or precision). */
size_t s7_batched_workspace_bytes_2d9(int32_t nsys, const int32_t *nx, const int32_t *ny, int32_t prec,
                                      const s7_options *opt);

/*
 * The batched form of s7_bicgstab_solve_2d9: nsys independent 2D 9-point
 * systems of uneven mesh sizes solved together in one persistent launch, as
 * s7_bicgstab_solve_batched does for the 7-point operator (section VIII-B's
 * many compact problems).  Per-system arguments are host arrays of length
 * nsys: nx[s], ny[s]; coef[9*s + c], device float arrays in the order
 * {diag, w, e, s, n, sw, se, nw, ne}; b[s] and x[s], device doubles; rtol[s];
 * max_iter[s].  info, if not NULL, is an array of nsys.  Each iteration is
 * three phases (P1, P2 with the five sums, P3); the refinement steps or the
 * FP32 epilogue also run on the device.  A system's iterates depend only on
 * that system.  A mesh of
 * split_cells cells or more (default 2^21) is solved alone by
 * s7_bicgstab_solve_2d9 after the shared launch.  Returns as
 * s7_bicgstab_solve_batched.
 */
int s7_bicgstab_solve_batched_2d9(int32_t nsys, const int32_t *nx, const int32_t *ny, const float *const *coef,
                                  const double *const *b, double *const *x, const double *rtol,
                                  const int32_t *max_iter, int32_t prec, void *ws, size_t ws_bytes,
                                  const s7_options *opt, s7_info *info, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* S7_H */
