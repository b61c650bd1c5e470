/*
 * inpaint.h - C ABI of the MI355X (gfx950) homogeneous diffusion inpainting solver.
 *
 * Operation (Kaemper, Chizhov, Weickert, "Efficient Parallel Algorithms for
 * Inpainting-Based Representations of 4K Images - Part I", Section 2.2,
 * the discrete system):  for each channel solve  A u = b  with  A = C + (I - C) L  and
 * b = C f, where C = diag(mask) and L is the 5-point negated Laplacian with
 * reflecting image boundaries (diagonal |N(i)|, -1 per direct neighbour).
 * Known pixels are Dirichlet data, every other pixel is filled by the discrete
 * Laplace equation.  The solver is the paper's reduced full multigrid
 * (Section 4.2) with an optimized restricted additive Schwarz smoother
 * (Section 3, Algorithm 2) on overlapping blocks, iterated with V-cycles until
 * the relative residual drops to the requested tolerance.
 *
 * Conventions shared by every entry point:
 *   - Images f and out are planar float32 [channels][H][W], row-major and
 *     contiguous.  mask is uint8 [H][W] (non-zero = known pixel) and is shared
 *     by all channels (Section 2.2, "Practical Considerations").
 *   - A pointer may be device memory (hipMalloc, a torch CUDA tensor) or host
 *     memory; host buffers are staged through the library's own device
 *     buffers.  The caller owns f, mask and out; the library never frees them.
 *   - out == f (the same address) is allowed; any other overlap is rejected.
 *     Values of f at unknown pixels do not influence the result and may be NaN.
 *   - Relative residual (Section 5.2, "Stopping Criterion"; the start of the
 *     decay is not named in the paper, this library uses the zero-filled start
 *     C f):  rel_res(u) = ||b - A u||_2 / ||b - A C f||_2, in float64 on the
 *     finest grid, per channel.  Where ||b - A C f|| = 0 (every known pixel
 *     next to an unknown one is 0 in that channel), C f is the exact solution:
 *     the channel stops at its first convergence test and C f is returned,
 *     with a relative residual of 0.
 *   - Guarantees on success: out equals f bit for bit at known pixels, and each
 *     channel is solved on its own (its result does not depend on the others).
 *   - Return value: an inpaint_status.  Negative values are errors and leave
 *     out unspecified; INPAINT_NOT_CONVERGED still writes the last iterate.
 *     inpaint_last_error() gives a message for the calling thread.
 *   - All entry points are thread-safe.  Calls that overlap in time on the same
 *     device use separate workspaces.
 */
#ifndef INPAINT_H
#define INPAINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum inpaint_status {
  INPAINT_OK = 0,
  INPAINT_NOT_CONVERGED = 1, /* cycle cap reached; out holds the last iterate */
  INPAINT_PENDING = 2,       /* inpaint_server_poll: the request has not finished yet */
  INPAINT_E_INVALID = -1,    /* bad argument, overlapping buffers, non-finite f at a known pixel */
  INPAINT_E_EMPTY_MASK = -2, /* no known pixel: the system is singular (any constant solves it) */
  INPAINT_E_NOMEM = -3,      /* device or pinned host allocation failed */
  INPAINT_E_DEVICE = -4,     /* a HIP runtime call failed */
  INPAINT_E_DIVERGED = -5    /* the residual became non-finite */
} inpaint_status;

/* Cycle schedules (Section 4.2).  RFMG is the paper's choice. */
typedef enum inpaint_schedule {
  INPAINT_SCHED_RFMG = 0,       /* reduced FMG: coarse-to-fine cascade with one ORAS
                                   iteration per coarse level, then V-cycles on the finest */
  INPAINT_SCHED_FMG = 1,        /* full FMG: one V-cycle on every level of the cascade */
  INPAINT_SCHED_MULTILEVEL = 2, /* cascade, then plain ORAS iterations on the finest */
  INPAINT_SCHED_SINGLE = 3,     /* ORAS iterations on the finest grid only, from C f */
  INPAINT_SCHED_CG = 4,         /* comparison (Section 5.1): plain conjugate gradients on the
                                   finest grid from C f (no multigrid, no domain decomposition),
                                   float32 only; a "cycle" is 8 CG iterations and a convergence
                                   test on the float64 true residual */
  INPAINT_SCHED_CG_MULTILEVEL = 5, /* comparison (Section 5.1): the MULTILEVEL cascade with CG
                                   in place of ORAS (pre_smooth CG iterations per coarse level,
                                   default 8), then CG on the finest grid as in SCHED_CG */
  INPAINT_SCHED_CG_MULTIGRID = 6,  /* comparison (Section 5.1): the RFMG cascade and V-cycles
                                   with CG in place of ORAS as pre- and post-smoother
                                   (pre_smooth / post_smooth CG iterations, default 2 each,
                                   each smoothing restarting CG from the current residual) */
  INPAINT_SCHED_WARM = 7          /* warm start: the RFMG V-cycles on the finest grid from an
                                   initial guess instead of the cascade.  On entry `out`
                                   holds the guess (its values at unknown pixels are used,
                                   known pixels take f; a channel whose guess is not finite
                                   there stops as INPAINT_E_DIVERGED, the others are solved);
                                   the first convergence test is on the guess itself, so a
                                   guess that already meets tol is returned after 0 cycles.  For
                                   sequences of related problems, as the next frame of a
                                   video or the next mask of an encoder's search (the
                                   temporal coherence Section 1.2 leaves unused).  Solve and
                                   batched entry points only (the server rejects it). */
  /* The three CG schedules run in float32 only (another precision is E_INVALID)
     and are not accepted by inpaint_server_create.  Float32 CG can stall with a
     relative residual between 1e-6 and 1e-5 on sparse (1-2 %) masks: a CG solve
     whose largest relative residual still above tol has not improved by 1 % in
     16 convergence tests stops there with NOT_CONVERGED (out holds the last
     iterate), as at the cycle cap. */
} inpaint_schedule;

typedef enum inpaint_rhs_restriction {
  INPAINT_RHS_MODIFIED = 0, /* known children weighted by their free neighbours (Section 4.3) */
  INPAINT_RHS_NAIVE = 1     /* plain mean of the known children (Section 4.3) */
} inpaint_rhs_restriction;

/*
 * Solver options.  Zero-initialise and set struct_size = sizeof(inpaint_opts);
 * every zero field takes its default.  A NULL opts pointer means all defaults.
 */
typedef struct inpaint_opts {
  int struct_size;     /* sizeof(inpaint_opts) */
  int block;           /* ORAS block side B: 16, 32 or 64 (default 32, Section 3.1); with 64
                          a block is solved by four wavefronts and the coarsest grid is at
                          most 32 x 32 (one level more than the rule "at most B") */
  int overlap;         /* overlap o in pixels between neighbouring blocks: even (twice the
                          per-side halo), 2 <= o <= B/2 (default 6) */
  float gamma;         /* Robin term added per cut block edge, 0 < gamma <= 1 (gamma = 1 is
                          Dirichlet RAS); the paper leaves alpha open (default 0.5) */
  float tau;           /* local CG stop: ||rho_i||^2 <= tau * ||r||^2 * |block| / N (default 0.005) */
  int max_local_iters; /* cap on local CG iterations per block (default 16) */
  int schedule;        /* inpaint_schedule (default INPAINT_SCHED_RFMG) */
  int max_cycles;      /* cap on V-cycles (or finest ORAS iterations for MULTILEVEL and
                          SINGLE, or blocks of 8 CG iterations for CG and CG_MULTILEVEL);
                          default 30 for RFMG/FMG/CG_MULTIGRID/WARM, 500 for CG and
                          CG_MULTILEVEL, 2000 otherwise */
  int pre_smooth;      /* ORAS iterations before the coarse correction, at most 16
                          (0 = default 1; a negative value = none); CG iterations for the
                          CG_MULTILEVEL and CG_MULTIGRID schedules (default 8 and 2) */
  int post_smooth;     /* ORAS iterations after it (0 = default 1; negative = none); CG
                          iterations for CG_MULTIGRID (default 2) */
  int rhs_restriction; /* inpaint_rhs_restriction (default MODIFIED) */
  float coarse_tau;    /* relative stop of the CG solve on the coarsest grid, on squared
                          norms (default 1e-8) */
  int coarse_max_iters;/* cap on that solve (default 256) */
  int profile;         /* non-zero: time every finest-grid kernel launch with HIP events on the
                          solve's stream and report it in inpaint_stats (adds event records) */
  int precision;       /* inpaint_precision of the correction fields (default FP32) */
} inpaint_opts;

/* Storage precision of the correction fields: the weighted block corrections on
   every level and every field of the coarser levels.  The finest grid's iterate,
   known values and residual stay float32, every residual is evaluated in float64
   and all arithmetic is float32, so each V-cycle is one step of iterative
   refinement whose correction is computed from 16-bit fields. */
typedef enum inpaint_precision {
  INPAINT_PREC_FP32 = 0,
  INPAINT_PREC_FP16 = 1, /* IEEE half: residuals and corrections stored scaled by the
                            reference residual's rms, the coarse levels' known values and
                            iterates of the cascade unscaled, so known values must lie within
                            the half range (|f| <= 65504; beyond it the fields overflow and
                            the solve ends with INPAINT_E_DIVERGED) */
  INPAINT_PREC_BF16 = 2  /* bfloat16 */
} inpaint_precision;

/* Kernel classes reported by the profile fields of inpaint_stats. */
typedef enum inpaint_kernel {
  INPAINT_K_STAGE = 0,       /* staging of f and mask, and the reference residual */
  INPAINT_K_PYRAMID = 1,     /* coarse masks and known values (first coarsening step) */
  INPAINT_K_BLOCK_SOLVE = 2, /* ORAS local problems */
  INPAINT_K_UPDATE = 3,      /* ORAS update + residual + norm */
  INPAINT_K_PROLONG = 4,     /* cascade prolongation or coarse-grid correction + residual + norm */
  INPAINT_K_RESTRICT = 5,    /* residual restriction to the next level */
  INPAINT_K_COARSE = 6,      /* coarsest-grid solve (only when the finest grid is the coarsest) */
  INPAINT_K_RESIDUAL = 7,    /* residual + norm only */
  INPAINT_K_OUTPUT = 8,      /* writing out */
  INPAINT_NUM_KERNELS = 9
} inpaint_kernel;

/* Per-solve statistics (all channels of one problem). */
typedef struct inpaint_stats {
  double rel_res;        /* largest relative residual over the channels (float64) */
  int cycles;            /* V-cycles run (finest ORAS iterations for MULTILEVEL/SINGLE) */
  int levels;            /* grid levels used */
  int oras_iters;        /* ORAS iterations over all levels and channels */
  double local_cg_mean;  /* mean local CG iterations per block solve */
  int local_cg_max;      /* largest local CG iteration count of any block */
  float gpu_ms;          /* device time of the solve, from HIP events */
  double local_cg_finest;/* local CG iterations summed over the finest-grid block solves */
  long long finest_block_solves; /* finest-grid block solves (blocks x channels x iterations) */
  double finest_cg_pixel_iters;  /* sum over finest-grid block solves of iterations x block pixels */
  /* with opts.profile: summed duration (ms) and number of finest-grid launches per
     inpaint_kernel class, from HIP events recorded around each launch */
  float kernel_ms[INPAINT_NUM_KERNELS];
  int kernel_calls[INPAINT_NUM_KERNELS];
  int status;            /* this problem's inpaint_status (set by the batched and served solves) */
  double t_submit_ms;    /* served requests: submission, start of the first launch and completion, */
  double t_start_ms;     /* in ms on the server's clock (0 at inpaint_server_create); 0 otherwise */
  double t_done_ms;
} inpaint_stats;

/*
 * Solve one image, synchronously, with default options.
 *   f     [channels][H][W] float32, host or device
 *   mask  [H][W] uint8, host or device
 *   W, H  >= 1;  channels in [1, 4];  tol in (0, 1): target relative residual
 *   out   [channels][H][W] float32, host or device
 */
int inpaint_solve(const float* f, const uint8_t* mask, int W, int H, int channels,
                  double tol, float* out);

/*
 * As inpaint_solve, with options, a stream (a hipStream_t passed as void*;
 * NULL = the null stream) and optional statistics.  Work is issued on that
 * stream; the call returns after the result is in out (it waits on the stream
 * once per V-cycle to read the convergence flags).
 */
int inpaint_solve_ex(const float* f, const uint8_t* mask, int W, int H, int channels,
                     double tol, float* out, const inpaint_opts* opts, void* stream,
                     inpaint_stats* stats);

/*
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the solve of inpaint_solve_ex with no
 * device allocation.  The grid hierarchy and the launch arguments live in one
 * fixed device array of INPAINT_NOALLOC_SCRATCH_BYTES bytes per GPU, which
 * the library holds from its load until the process ends; the call allocates
 * no device or pinned host memory and creates no graph, stream or event.
 *   f, mask, out  device memory only (host pointers: E_INVALID), with the
 *                 layout, ownership and aliasing rules of inpaint_solve_ex
 *   opts          as for inpaint_solve_ex; the CG schedules are rejected
 *                 (E_INVALID); opts.profile is ignored
 *   stream        hipStream_t as void*, NULL = the null stream
 *   stats         as for inpaint_solve_ex, except that gpu_ms is the host time
 *                 of the call and the local CG and kernel profile fields are 0
 * A problem whose hierarchy and launch arguments need more than the array
 * holds is rejected before any device work (E_INVALID, the message gives the
 * bytes needed): with the default block and overlap, float32 fields fit up to
 * 1920x1080 with 3 channels or 3840x2160 with 1 channel.  Every call on a GPU
 * uses that GPU's one array, whose contents are the last call's: the library
 * serialises calls on the same device (a second caller waits), so calls that
 * would overlap in time run one after the other.  Returns after the result is
 * in out.  Results are bit-identical to inpaint_solve_ex with the same
 * options.
 */
#define INPAINT_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int inpaint_solve_noalloc(const float* f, const uint8_t* mask, int W, int H, int channels,
                          double tol, float* out, const inpaint_opts* opts, void* stream,
                          inpaint_stats* stats);

/*
 * Bound on the device memory that single and batched solves keep cached
 * between calls: the grid hierarchy of each problem shape (block, overlap and
 * precision) already solved is kept for the next call of that shape, and idle
 * hierarchies are freed, least recently used first, whenever the cache would
 * otherwise exceed the limit (at the end of a call, and before a new
 * hierarchy is allocated).  A hierarchy in use by a call is never freed, so a
 * single call may exceed the limit while it runs.  The default limit is
 * 16 GiB, or INPAINT_CACHE_LIMIT_MB mebibytes when that variable is set at
 * the first call.  Servers keep their own pool, bounded by their budget.
 *   limit_bytes   new limit; 0 = keep the current one (and just trim)
 *   cached_bytes  NULL, or receives the bytes still cached after trimming
 * Always returns INPAINT_OK.
 */
int inpaint_cache_limit(size_t limit_bytes, size_t* cached_bytes);

/*
 * Relative residual (float64, per channel, see above) of u for the problem
 * (f, mask).  u, f: [channels][H][W] float32; rel_res_out: channels doubles
 * (host memory).  Computed on the device.
 */
int inpaint_rel_res(const float* u, const float* f, const uint8_t* mask, int W, int H,
                    int channels, double* rel_res_out);

/*
 * One problem of a batched or served solve, with the conventions of
 * inpaint_solve: f and out planar float32 [channels][H][W], mask uint8 [H][W],
 * each pointer host or device memory, owned by the caller.
 */
typedef struct inpaint_problem {
  const float* f;
  const uint8_t* mask;
  int W, H, channels;
  float* out;
} inpaint_problem;

/*
 * Solve n independent problems of any sizes together (the data-parallel form
 * of the method: images and channels carry no coupling, Section 2.2).  Every
 * step of the cycle runs as one launch over all problems in lockstep by level;
 * each problem keeps its own hierarchy, norms and convergence test, and one
 * V-cycle of the whole batch is replayed from a captured HIP graph.  Each
 * result is bit-identical to solving that problem alone with inpaint_solve_ex
 * and the same options.
 *   problems  host array of n problems; their outputs must not overlap each other
 *   n         >= 1
 *   tol       in (0, 1), the target relative residual of every problem
 *   opts      as for inpaint_solve_ex (opts.profile is ignored); NULL = defaults
 *   stream    hipStream_t as void*, NULL = the null stream
 *   stats     NULL or an array of n inpaint_stats, one per problem (gpu_ms is
 *             the device time of the whole batch; status is that problem's
 *             inpaint_status; the local CG and kernel profile fields are 0)
 * Returns INPAINT_OK when every problem converged; otherwise the status of the
 * first problem (lowest index) that failed, else INPAINT_NOT_CONVERGED if some
 * problem reached the cycle cap.  A bad argument of any problem rejects the
 * whole call before any work (E_INVALID, the message names the problem).  A
 * problem whose data is rejected on the device (no known pixel, non-finite f
 * at a known pixel) gets its error status in stats and is left out; the others
 * are solved.  Returns after every result is in place.
 */
int inpaint_solve_batched(const inpaint_problem* problems, int n, double tol,
                          const inpaint_opts* opts, void* stream, inpaint_stats* stats);

/*
 * Autotuner of the batched solve: picks the ORAS block side (16, 32, 64), overlap
 * (2, 4, 6, 8, at most half the block), Robin weight gamma (0.3, 0.5, 0.7),
 * local CG tolerance tau (0.002, 0.005, 0.01) and cycle schedule (RFMG, FMG)
 * for these problems by timing batched solves of them: one coordinate-descent
 * sweep from `base` (NULL = defaults), each candidate timed as the median of
 * three solves after a warm-up; a candidate counts only if every problem
 * converges.  The problems' outputs are overwritten.  The choice is cached in
 * memory per workload signature (sorted sizes and channel counts, precision,
 * tolerance, smoothing counts) and, when the environment variable
 * INPAINT_AUTOTUNE_CACHE names a file, appended to and read from that file.
 *   best     receives base with the five chosen fields set
 *   best_ms  NULL or receives the chosen configuration's time per batch (ms)
 */
int inpaint_autotune(const inpaint_problem* problems, int n, double tol,
                     const inpaint_opts* base, void* stream, inpaint_opts* best,
                     double* best_ms);

/* ---------------------------------------------------------------------------
 * Serving: a request loop with continuous batching on one device.
 *
 * Requests are admitted in submission order while a batch slot is free and
 * their hierarchy (plus staging for host buffers) fits the server's HBM
 * budget; idle hierarchies of other sizes are freed to make room, and a
 * request that does not fit waits in the queue.  Admitted requests join the
 * running batch at the next V-cycle boundary and leave it when they converge,
 * so requests that arrive while others are on the device share every batched
 * launch with them.  Hierarchies stay on the device between requests of the
 * same size.  Each request runs the same arithmetic as a solve of it alone, so
 * its result is bit-identical to inpaint_solve_ex with the server's options,
 * whatever else is in the batch.
 * ------------------------------------------------------------------------- */

typedef struct inpaint_server inpaint_server; /* opaque */

typedef struct inpaint_server_cfg {
  int struct_size;   /* sizeof(inpaint_server_cfg) */
  int max_batch;     /* requests in the running batch at most, 1..1024 (0 = 64) */
  size_t hbm_budget; /* device bytes for the requests' hierarchies and staging
                        (0 = 80 % of the device memory free at creation) */
  inpaint_opts opts; /* options of every request (opts.struct_size == 0: all
                        defaults; opts.profile is ignored) */
} inpaint_server_cfg;

/* Start a server on the calling thread's current device (cfg NULL = defaults).
   The server runs its own thread and its own HIP stream. */
int inpaint_server_create(const inpaint_server_cfg* cfg, inpaint_server** srv);

/* Queue one problem with its tolerance; returns at once with a ticket.  The
   caller keeps f, mask and out valid and unchanged until the ticket has been
   collected.  Bad arguments: E_INVALID; a hierarchy larger than the whole
   budget: E_NOMEM (nothing queued). */
int inpaint_server_submit(inpaint_server* srv, const inpaint_problem* p, double tol,
                          uint64_t* ticket);

/* INPAINT_PENDING while the request runs; afterwards its inpaint_status, with
   its statistics in *st (may be NULL) including t_submit_ms, t_start_ms and
   t_done_ms, and the ticket is collected (a later call on it is E_INVALID). */
int inpaint_server_poll(inpaint_server* srv, uint64_t ticket, inpaint_stats* st);

/* As inpaint_server_poll, but blocks until the request has finished. */
int inpaint_server_wait(inpaint_server* srv, uint64_t ticket, inpaint_stats* st);

/* Finish every submitted request, stop the loop and free the server's device
   memory.  Tickets not collected before are lost. */
void inpaint_server_destroy(inpaint_server* srv);

/* Message for the last error on the calling thread ("" if none). */
const char* inpaint_last_error(void);

/* Library version string. */
const char* inpaint_version(void);

/* ---------------------------------------------------------------------------
 * Step-level entry points.  Each runs one step of the method on the device and
 * returns its result to host buffers, synchronously, so that the step can be
 * checked on its own.  All pointers are host memory.
 * ------------------------------------------------------------------------- */

/*
 * Grid hierarchy of the coarse problems (Section 4.3; level rule of Section
 * 4.4: halve with ceil until both sides are at most `block`).
 *   levels_out      number of levels L (host int)
 *   sizes_out       2*L ints: (W_l, H_l) finest first (capacity 2*16 ints)
 *   masks_out       concatenation over levels of uint8 [H_l][W_l] coarse masks
 *                   (max pooling of the children), or NULL
 *   rhs_out         concatenation over levels of float32 [channels][H_l][W_l]
 *                   known values b_l (0 at unknown pixels), or NULL
 *   rhs_restriction inpaint_rhs_restriction
 * Buffers must hold sum_l H_l*W_l (masks) and channels * sum_l H_l*W_l (rhs)
 * elements; inpaint_hierarchy_size() gives both counts.
 */
int inpaint_hierarchy_size(int W, int H, int block, int* levels_out, size_t* pixels_out);
int inpaint_debug_pyramid(const float* f, const uint8_t* mask, int W, int H, int channels,
                          int block, int rhs_restriction, int* levels_out, int* sizes_out,
                          uint8_t* masks_out, float* rhs_out);

/*
 * One ORAS iteration (Section 3, Algorithm 2) on the finest grid:
 * r = b - A u_in;  solve A_i v_i = R_i r on every block by local CG;
 * u_out = u_in + sum_i R_i^T D_i v_i.  u_in must equal f at known pixels.
 * Block side, overlap, gamma, tau and the CG cap come from opts.
 * u_in, u_out: [channels][H][W] float32.
 */
int inpaint_debug_oras_step(const float* u_in, const float* f, const uint8_t* mask, int W,
                            int H, int channels, const inpaint_opts* opts, float* u_out);

/*
 * Residual restriction (Sections 4.1 and 4.4): for each coarse pixel X of a
 * [ceil(Hf/2)][ceil(Wf/2)] grid, r_c(X) = 4 * mean of the existing fine
 * children of r_f where mask_c(X) == 0, and 0 where mask_c(X) != 0 (the factor
 * 4 = (H/h)^2 keeps the integer 5-point stencil on every level).
 *   r_f [Hf][Wf] float32, mask_c [Hc][Wc] uint8, r_c [Hc][Wc] float32.
 */
int inpaint_debug_restrict(const float* r_f, const uint8_t* mask_c, int Wf, int Hf, float* r_c);

/*
 * Bilinear, cell-centred prolongation (Section 4.4) from a [Hc][Wc] grid with
 * Hc = ceil(Hf/2), Wc = ceil(Wf/2) to [Hf][Wf]:
 *   mode 0 (cascade):    u_out = mask_f ? b_f : P u_c
 *   mode 1 (correction): u_out = u_in + (mask_f ? 0 : P u_c)
 * u_in may be NULL for mode 0.
 */
int inpaint_debug_prolong(const float* u_c, int Wf, int Hf, const uint8_t* mask_f,
                          const float* b_f, const float* u_in, int mode, float* u_out);

#ifdef __cplusplus
}
#endif

#endif /* INPAINT_H */
