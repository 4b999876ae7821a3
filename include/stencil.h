/*
 * stencil.h -- C ABI of the MI355X (gfx950) stencil-sweep library
 * (libstencil.so).
 *
 * What it computes.  A stencil sweep replaces every cell of a d-dimensional
 * grid, once per time step, by a weighted sum of itself and a fixed set of
 * neighbours taken from the previous step (paper: Sec. 2.1 and its Alg. 1
 * "Heat-2D Stencil"; the explicit heat step of Eq. 3 is the special case of a
 * radius-1 star with centre weight 1 - 2*d*mu and neighbour weights mu).  The
 * library runs T such steps, blocked in space (tiles held on chip) and in
 * time (several steps fused per pass over memory; Sec. 4 "Locality
 * Enhancer"), and returns u_T = S^T(u_0).  Reordering and fusing the updates
 * changes only rounding, not the result (Sec. 1, the two key observations).
 *
 * Conventions shared by every entry point.
 *   Layout   dense C order, shape (nz, ny, nx) in 3D, (ny, nx) in 2D, (nx) in
 *            1D; x is unit-stride, as j is in Alg. 1.  No padding.
 *   Offsets  npoints x ndim int32, slowest axis first; the centre (all zero)
 *            must be among them.  |offset| <= 4 on every axis; npoints <= 125.
 *   Boundary ST_BC_ZERO: an index outside the grid reads 0 (a zero-Dirichlet
 *            ghost layer around the grid, so every cell evolves);
 *            ST_BC_PERIODIC: indices wrap modulo the extent.
 *   Steps    exactly `steps` updates; steps == 0 is a no-op returning ST_OK.
 *   Coeffs   host FP64, one weight per point in the caller's point order; the
 *            library rounds each to the compute precision once (FP64 for
 *            ST_F64 storage, FP32 for ST_F32 and ST_BF16 storage).
 *   Memory   grid and work buffers are device pointers owned by the caller;
 *            the library never frees them.  Plans, their device tables and
 *            any plan-owned workspace belong to the library.
 *   Streams  `stream` is a hipStream_t passed as void* (NULL = the null
 *            stream).  Runs are asynchronous and stream-ordered; the result is
 *            in `grid` once the stream reaches it.  Nothing in a run
 *            synchronises the host.
 *   Errors   every call returns st_status and never throws or aborts.
 *            Argument problems are found on the host before any launch.  A
 *            HIP failure returns ST_ERR_HIP; stencil_last_error() then names
 *            the call site and the HIP error string (thread-local).
 *   Threads  distinct plans may be used from distinct threads; one plan must
 *            not be run concurrently from two threads.
 */
#ifndef PAPER_2303_08365_AMD_STENCIL_H
#define PAPER_2303_08365_AMD_STENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ST_OK = 0,
    ST_ERR_ARG = -1,          /* NULL pointer, bad size, bad enum value         */
    ST_ERR_UNSUPPORTED = -2,  /* ndim not in 1..3, radius > 4, npoints > 125,  */
                              /* a flag the pattern cannot take               */
    ST_ERR_MISMATCH = -3,     /* shape/boundary/count differs from the plan     */
    ST_ERR_NOMEM = -4,        /* host or device allocation failed               */
    ST_ERR_HIP = -5,          /* a HIP runtime call failed (see last_error)     */
    ST_ERR_CAPTURE = -6       /* reserved: no call returns it (run calls do not */
                              /* allocate; the value keeps its number)         */
} st_status;

typedef enum { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2 } st_dtype;   /* storage type */
typedef enum { ST_BC_ZERO = 0, ST_BC_PERIODIC = 1 } st_boundary;

/* Plan flags. */
#define ST_PLAN_AUTOTUNE 0x1u  /* time candidate tilings on the device now;    */
                               /* allocates and synchronises (not capturable)  */
#define ST_PLAN_NAIVE 0x2u     /* force the one-step-per-launch kernel         */
#define ST_PLAN_GRAPH 0x8u     /* capture a run's launches in a HIP graph and */
                               /* replay it while the arguments are unchanged */
                               /* (first call per argument set captures)      */
#define ST_PLAN_VARCOEF 0x4u   /* variable-coefficient heat operator (3D,      */
                               /* radius-1 star, ST_BC_ZERO, FP64/FP32 only);  */
                               /* run with stencil_run_ckpt                    */
#define ST_PLAN_OWN_WORK 0x10u /* the plan allocates a work buffer of the      */
                               /* grid's size now; stencil_run / _flux then    */
                               /* accept work == NULL (single-grid plans)      */

typedef struct {
    int32_t ndim;             /* 1..3                                          */
    int32_t npoints;          /* 1..125                                        */
    const int32_t* offsets;   /* host, npoints*ndim, copied by the plan call  */
} st_pattern;

typedef struct st_plan_s* st_plan;

/* Kernel families a plan can select. */
#define ST_KERNEL_NAIVE 0      /* one step per launch, any pattern             */
#define ST_KERNEL_STREAM2D 1   /* 2D star/box, rows streamed through registers */
#define ST_KERNEL_STREAM3D 2   /* 3D star, planes streamed, LDS row exchange   */
#define ST_KERNEL_VARCOEF3D 3  /* 3D variable-coefficient heat                 */
#define ST_KERNEL_STREAM1D 4   /* 1D star, a wave's strip of cells in registers */
#define ST_KERNEL_BOX3D 5      /* 3D radius-1 box, planes streamed, 1-2 steps    */

typedef struct {
    int32_t kernel;           /* ST_KERNEL_*                                    */
    int32_t tb;               /* time steps fused per pass                      */
    int32_t radius;           /* max |offset|                                   */
    int32_t shape_class;      /* 0 general, 1 star, 2 box                       */
    int32_t tile_x, tile_y, tile_z;  /* output cells per work-group tile        */
    int32_t block;            /* threads per work-group                         */
    int64_t workgroups;       /* work-groups per pass launch (single grid)      */
    int64_t lds_bytes;        /* LDS per work-group                             */
    int32_t variant;          /* index of the tiling candidate                  */
    int32_t ncandidates;      /* tiling candidates valid for this plan          */
    int32_t pipeline;         /* ST_KERNEL_STREAM3D: 0 = queued planes, else    */
                              /* the partial-sum pipeline (LDS buffers * 10 +   */
                              /* prefetched planes, + 100 when the planes come  */
                              /* through an LDS queue rather than registers); */
                              /* ST_KERNEL_BOX3D: 0 = one plane queue per step, */
                              /* else the two-step partial-sum pipeline (one   */
                              /* LDS row exchange per plane), variant + 1      */
    int32_t tessellated;      /* ST_KERNEL_STREAM2D: 1 = tessellated tiling     */
                              /* along y (paper Sec. 4.1: triangles, then the   */
                              /* inverted triangles at the chunk junctions, no  */
                              /* recomputed rows; two launches per pass and a   */
                              /* band scratch the plan owns), 0 = overlapped    */
} st_plan_info;

/*
 * stencil_plan -- choose kernel, tile, fused depth and launch geometry for
 * one grid shape (paper Sec. 5.2: the scheduler is fixed from a profile of the
 * problem; Tab. 1 lists the blocking sizes per benchmark).
 *
 * Allocation.  Every device buffer a plan owns is allocated here, on the
 * current device: the outflow partial sums (zero rule), the work buffer
 * (ST_PLAN_OWN_WORK), the batch descriptor table, the capture stream
 * (ST_PLAN_GRAPH), and the plan of the transposed sweep used by
 * stencil_adjoint_run.  No run call allocates device or pinned memory or
 * waits for the device; the one exception is ST_PLAN_GRAPH, whose first run
 * with a new argument set captures and instantiates a graph.  A plan made
 * where no device is present can describe its tilings, but its run calls
 * fail with ST_ERR_HIP.
 *   out      receives the plan; *out is NULL on failure.
 *   pattern  point list (copied).  Points are evaluated in a canonical order
 *            (centre, then lexicographic by offset) by every kernel, so all
 *            tilings and depths of one plan give bit-identical results.
 *   shape    pattern->ndim extents, each >= 1.
 *   storage  ST_F64 computes in FP64; ST_F32 and ST_BF16 compute in FP32
 *            (ST_BF16 rounds every step's result to bfloat16, ties to even).
 *   flags    ST_PLAN_* bits.  With ST_PLAN_AUTOTUNE the call allocates two
 *            scratch grids, times every candidate on the current device and
 *            keeps the fastest; without it a fixed heuristic is used.  With
 *            ST_PLAN_GRAPH, stencil_run captures its passes into a HIP graph
 *            (on a plan-owned stream) the first time it sees a set of
 *            arguments (grid, work, steps, weights, candidate) and afterwards
 *            replays the graph with one hipGraphLaunch; a caller that is
 *            itself capturing its stream gets the launches recorded into its
 *            own graph instead.
 * Errors: ST_ERR_ARG, ST_ERR_UNSUPPORTED, ST_ERR_NOMEM, ST_ERR_HIP (autotune).
 */
st_status stencil_plan(st_plan* out, const st_pattern* pattern, const int64_t* shape,
                       st_dtype storage, st_boundary bc, uint32_t flags);

/*
 * stencil_autotune_cache -- remember autotuning results (paper Sec. 5.2: the
 * scheduler's choice comes from a profile of the problem, taken once).  Every
 * ST_PLAN_AUTOTUNE plan (single or batch) first looks its key up -- device
 * (architecture and compute-unit count), dimensions, storage type, boundary,
 * shape or shapes, point offsets -- and takes the stored candidate without
 * timing anything; otherwise it times the candidates and stores its choice.
 * The in-memory table lives as long as the library.
 *   path  text file, one "key<TAB>candidate<TAB>candidates" line per plan:
 *         read now when it exists (its entries join the table) and rewritten
 *         after every new tuning (a file that cannot be written is left as
 *         it is: the cache is advisory).  NULL stops writing a file.
 * Errors: ST_ERR_ARG for an empty path or a malformed file (nothing loaded).
 */
st_status stencil_autotune_cache(const char* path);

/* Release a plan and everything it owns (NULL is accepted). */
st_status stencil_plan_destroy(st_plan plan);

/* Describe the plan's current choice. */
st_status stencil_plan_info(st_plan plan, st_plan_info* info);

/*
 * stencil_plan_candidate -- describe tiling candidate `index` of the plan
 * (0 <= index < info->ncandidates of stencil_plan_info).
 */
st_status stencil_plan_candidate(st_plan plan, int32_t index, st_plan_info* info);

/*
 * stencil_plan_select -- force a kernel family, fused depth and tiling
 * candidate (used by the autotuner and by tests that compare candidates).
 * kernel = -1 keeps the family; tb <= 0 keeps the depth; variant < 0 keeps
 * the candidate.  Returns ST_ERR_UNSUPPORTED when the combination cannot run
 * this plan.
 */
st_status stencil_plan_select(st_plan plan, int32_t kernel, int32_t tb, int32_t variant);

/*
 * stencil_run -- run `steps` steps on one grid (Alg. 1 with T = steps).
 *   plan    required: the call carries no pattern, so a NULL plan could not
 *           say which stencil to apply (ST_ERR_ARG).
 *   grid    device, in: u_0, out: u_T; plan->shape cells of the storage type.
 *   work    device buffer of the same size, clobbered; NULL uses the plan's
 *           own buffer (plans made with ST_PLAN_OWN_WORK; ST_ERR_ARG
 *           otherwise).
 *   coeffs  host FP64 weights, one per pattern point, caller's order.
 *   shape   must equal the plan's shape (ST_ERR_MISMATCH otherwise).
 *   bc      must equal the plan's boundary (ST_ERR_MISMATCH otherwise).
 * The steps are grouped into passes of up to tb fused steps; passes
 * alternate between grid and work and the pass list is arranged so that the
 * last pass writes `grid`.  run(a) followed by run(b) equals run(a + b) bit
 * for bit.  Unstable coefficients are not an error.
 */
st_status stencil_run(st_plan plan, void* grid, void* work, const double* coeffs,
                      const int64_t* shape, int64_t steps, st_boundary bc, void* stream);

/*
 * stencil_run_noalloc -- stencil_run for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It takes no work buffer: the passes ping-pong between
 * `grid` and the library's static work space, a file-scope device array of
 * 64 MiB (2^26 bytes) that each device the library runs on holds from the
 * first call on that device until the process ends.  The call allocates
 * nothing (no hipMalloc, no hipFree, no allocating library routine) and does
 * not wait; its result equals stencil_run's bit for bit (same passes, same
 * kernels).  ST_PLAN_GRAPH is ignored: the launches go to `stream`, or into
 * the caller's capture.
 *   plan, grid, coeffs, shape, steps, bc  as for stencil_run.
 * Every call on one device shares that device's array and leaves it holding
 * the last call's intermediate states; the array needs no clearing (every
 * pass writes each cell it later reads).  Calls that overlap on one device
 * -- on different streams, from different threads, or a replaying graph
 * that holds such a call -- race on the array and give wrong results.
 * Errors: as stencil_run; ST_ERR_ARG also when the grid needs more than the
 * 64 MiB of work space (plan cells x storage bytes), checked before anything
 * else touches the device.
 */
st_status stencil_run_noalloc(st_plan plan, void* grid, const double* coeffs, const int64_t* shape,
                              int64_t steps, st_boundary bc, void* stream);

/*
 * stencil_run_flux -- stencil_run that also keeps account of the heat the
 * steps carry out of the grid.  Reading the zero ghost layer of Alg. 1
 * (Sec. 2.1, Eq. 3) as an absorbing boundary, a step moves w_p * u(c) from
 * cell c to the cell c - off_p that reads c through point p, and what would
 * land outside the grid has left; with weights summing to 1 the grid's total
 * then drops by exactly that amount, so total + outflow stays constant up
 * to rounding and tracks the drift of long FP32 / bfloat16 runs.
 *   flux    device pointer to ONE double; the outflow of the `steps` steps
 *           (each step's sum over the state it reads, weights rounded to the
 *           compute precision, products and sums in FP64 -- except that the
 *           fused FP32-compute 3D kernels first add, in FP32, the values of
 *           one x-face column that a lane holds: up to 4 rows of one state,
 *           or of the up to 4 states of one plane in the pipelined tiling) is
 *           ADDED to it.
 *           Under the periodic rule nothing leaves and *flux is not touched.
 *   other arguments as for stencil_run; the grid ends bit-identical to
 *           stencil_run's.
 * The sum is deterministic: partial sums go to a plan-owned device buffer
 * (allocated with the plan) and one work-group adds them in a fixed order.
 * That buffer belongs to the plan, so calls on one plan must not overlap on
 * different streams.  The fused 3D radius-1
 * kernels (FP64, FP32, bfloat16 default tilings) sum the outflow inside
 * their passes; every other plan runs one step per pass with a band kernel
 * over the state each step reads.  ST_PLAN_GRAPH is ignored here (the
 * launches go to `stream`, or into the caller's capture).
 * Errors: as stencil_run; ST_ERR_ARG for flux == NULL.
 */
st_status stencil_run_flux(st_plan plan, void* grid, void* work, const double* coeffs,
                           const int64_t* shape, int64_t steps, st_boundary bc, double* flux,
                           void* stream);

/*
 * stencil_batch_plan -- plan a batch of n independent grids that share the
 * pattern, storage type and boundary but differ in shape and coefficients
 * (an ensemble).  Each pass over all grids is ONE launch: work-groups take
 * (grid, tile) items from a device descriptor table (paper Sec. 5.2: the
 * work is split so that no worker becomes the slowest).  Supported patterns:
 * 2D radius-1 star or box.  shapes: host, n * ndim extents.  flags:
 * ST_PLAN_AUTOTUNE times every tiling candidate on scratch grids of the
 * batch's shapes (allocates, synchronises) and keeps the fastest;
 * ST_PLAN_GRAPH captures the launches of a run into a HIP graph replayed while
 * the arguments stay the same.
 * Errors: ST_ERR_ARG, ST_ERR_UNSUPPORTED, ST_ERR_NOMEM, ST_ERR_HIP.
 */
st_status stencil_batch_plan(st_plan* out, const st_pattern* pattern, int32_t n,
                             const int64_t* shapes, st_dtype storage, st_boundary bc,
                             uint32_t flags);

/*
 * stencil_batch_run -- run grid g for steps[g] steps, for every g, in about
 * ceil(max steps / tb) launches on `stream` (each launch covers every grid;
 * grid g runs the passes of its own step count, the grids with fewer passes
 * idle in the last launches).
 *   grids, works  host arrays of n device pointers (work buffers as in
 *                 stencil_run, required here).
 *   coeffs        host FP64, n * npoints, row g holds grid g's weights.
 *   steps         host, n step counts (each >= 0).
 * Results land in grids[g].  The plan's device descriptor table (one entry
 * per grid, allocated with the plan) is rewritten in stream order whenever
 * the arguments differ from what it holds: the entries travel as kernel
 * arguments, so the call neither allocates nor waits, and a graph that
 * captures the call records the table it needs and rewrites it on every
 * replay.  Once a call on a plan has been recorded into a caller's graph,
 * every later call on that plan rewrites the table (a replay may have
 * changed it at any time).  Calls on one plan must not overlap on different
 * streams, and a caller's graph that holds a call on a plan must not replay
 * concurrently with other calls on that plan.
 * Errors: ST_ERR_ARG, ST_ERR_MISMATCH (n differs from the plan), ST_ERR_HIP.
 */
st_status stencil_batch_run(st_plan plan, int32_t n, void* const* grids, void* const* works,
                            const double* coeffs, const int64_t* steps, void* stream);

/*
 * stencil_batch_run_flux -- stencil_batch_run that also adds each grid's
 * outflow across the zero-rule boundary to flux[g] (device, n doubles), as
 * stencil_run_flux does for one grid.  Radius-1 stars sum it inside the
 * batch passes (one reduction launch per pass, fixed order); other patterns
 * run grid by grid, one step per pass.  ST_PLAN_GRAPH is ignored (eager
 * launches); the partial sums use a plan-owned buffer allocated with the
 * plan.  Periodic batches leave flux untouched.
 * Errors: as stencil_batch_run; ST_ERR_ARG for flux == NULL.
 */
st_status stencil_batch_run_flux(st_plan plan, int32_t n, void* const* grids, void* const* works,
                                 const double* coeffs, const int64_t* steps, double* flux, void* stream);

/*
 * stencil_run_ckpt -- variable-coefficient heat run with checkpoints (plan
 * made with ST_PLAN_VARCOEF: 3D radius-1 star, ST_BC_ZERO, FP64 or FP32).
 * The step is not in the paper; it is the conservative form of the explicit
 * heat step of Eq. 3 with a conductivity field:
 *   u'[i] = u[i] + alpha * sum over the 6 faces f of kap_f (u[i+f] - u[i]),
 *   kap_f = (k[i] + k[i+f]) / 2, and kap_f = k[i], u = 0 across the grid edge.
 *   grid   device, in u^0, out u^steps (plan shape, plan storage type).
 *   work   device buffer of the same size, clobbered.
 *   k      device conductivity field, same shape and type.
 *   ckpts  NULL, or ceil(steps/every) device buffers of the grid's size: the
 *          call stores u^(c*every) into ckpts[c] before step c*every.
 * Errors: ST_ERR_ARG, ST_ERR_MISMATCH (plan without ST_PLAN_VARCOEF), ST_ERR_HIP.
 */
st_status stencil_run_ckpt(st_plan plan, void* grid, void* work, const void* k, double alpha,
                           int64_t steps, int64_t every, void* const* ckpts, void* stream);

/*
 * stencil_adjoint_run -- reverse-mode sweep: lambda holds dL/du^steps on
 * entry and dL/du^0 on exit.
 *   Constant-weight plan: k, grad_k NULL; coeffs as for stencil_run; runs
 *     the transpose of Alg. 1's update (Sec. 2.1): u -> sum_p w_p u(x + o_p)
 *     is linear, and its transpose is the same sweep with every offset
 *     negated under the same boundary rule (planned with the plan), applied
 *     `steps` times; ckpts, every and seg are ignored.
 *   Variable-coefficient plan: coeffs ignored; k and alpha as in the forward
 *     run; ckpts / every as stored by stencil_run_ckpt.  Each checkpoint
 *     segment is recomputed forward into `seg` (min(every, steps) - 1
 *     buffers of the grid's size, laid out back to back; NULL allowed when
 *     every == 1), then stepped back.  grad_k (NULL or a device buffer of the
 *     grid's size) receives += dL/dk.  The step's transpose is the same step
 *     (the operator is symmetric); the k derivative is gathered per cell, so
 *     no atomics are used and results are deterministic.
 *   work   device buffer of the grid's size, clobbered.
 * Errors: ST_ERR_ARG, ST_ERR_MISMATCH, ST_ERR_HIP.
 */
st_status stencil_adjoint_run(st_plan plan, const void* k, double alpha, const double* coeffs,
                              void* const* ckpts, int64_t every, int64_t steps, void* lambda,
                              void* grad_k, void* seg, void* work, void* stream);

/*
 * stencil_copy -- plain streaming device copy of `bytes` bytes (one read and
 * one write of every byte: exactly the traffic one pass of the sweep must
 * move, so its rate is the achievable-bandwidth reference for the sweep's
 * roofline; the paper's transfer-time model, Sec. 4.1, makes memory traffic
 * the dominant cost of a pass).  dst and src: device, 16-byte aligned, not
 * overlapping.  Asynchronous on `stream`.
 * Errors: ST_ERR_ARG, ST_ERR_HIP.
 */
st_status stencil_copy(void* dst, const void* src, int64_t bytes, void* stream);

/* Thread-local text of the last failure ("" if none). */
const char* stencil_last_error(void);

/* Library version string. */
const char* stencil_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_2303_08365_AMD_STENCIL_H */
