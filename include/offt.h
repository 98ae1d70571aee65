/*
 * offt.h -- C ABI of the MI355X (gfx950) 3-D complex-to-complex FFT library.
 *
 * The operation is the 3-D discrete Fourier transform of a grid A(a,b,c) with
 * Na x Nb x Nc points (Duy & Ozaki, "Performance Tuning of a Parallel 3-D FFT
 * Package OpenFFT", Sec. 2):
 *
 *   forward   X[ka,kb,kc] = sum_{a,b,c} x[a,b,c] W_Na^(a ka) W_Nb^(b kb) W_Nc^(c kc),
 *             W_n = exp(-2 pi i / n)
 *   backward  the same with W_n = exp(+2 pi i / n); unnormalised unless the plan
 *             was created with normalize_inverse = 1, then scaled by 1/(Na Nb Nc).
 *
 * It is computed as in the paper's calculation flow (Sec. 3.1.1): batched 1-D
 * transforms along one axis at a time, with the data rearranged between the
 * axis passes (the transpose order abc -> cab -> cba of Sec. 2).  On one GPU the
 * rearrangement is an in-HBM tile transpose through LDS rather than an MPI
 * exchange.  The paper's three phases map to:
 *   initialization  -> offt_plan / offt_plan_ex / offt_plan_many  (index math,
 *                      one-time allocations (Sec. 3.2.4) and auto-tuning
 *                      (Sec. 3.2.3) happen here)
 *   execution       -> offt_exec_fwd / offt_exec_bwd / offt_exec_many_*  (may be
 *                      repeated any number of times; never allocates)
 *   finalization    -> offt_destroy
 *
 * Memory layout of every grid: row-major with c fastest, offset
 * a*Nb*Nc + b*Nc + c (Sec. 2, Eq. 1); element = interleaved (re, im) of the
 * plan's precision (binary64 for OFFT_C2C_F64, binary32 for OFFT_C2C_F32).
 * A batch of grids is stored back to back: grid g starts at element g*N.
 *
 * Pointers passed to the exec calls are DEVICE pointers owned by the caller;
 * `stream` is a hipStream_t (NULL = the null stream).  Exec calls are
 * stream-ordered and asynchronous: device faults surface at the caller's next
 * synchronisation, as usual in HIP.  A plan must not be executed concurrently
 * on two streams.
 *
 * Errors: calls returning int return 0 (OFFT_SUCCESS) or a negative OFFT_ERR_*;
 * calls returning a handle return NULL on error.  The last error code of the
 * calling thread is kept and can be read with offt_last_error().
 */
#ifndef OFFT_H
#define OFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct offt_plan_s* offt_plan_t;

/* precision / transform kind */
enum { OFFT_C2C_F64 = 0, OFFT_C2C_F32 = 1 };

/* error codes */
enum {
    OFFT_SUCCESS = 0,
    OFFT_ERR_INVALID_ARG = -1,      /* NULL handle/pointer, non-positive size, bad dtype/option */
    OFFT_ERR_UNSUPPORTED_SIZE = -2, /* an axis has a prime factor > 5, or exceeds the supported length */
    OFFT_ERR_OUT_OF_MEMORY = -3,    /* device allocation failed at plan time */
    OFFT_ERR_NO_DEVICE = -4,        /* no HIP device visible */
    OFFT_ERR_HIP = -5,              /* a HIP runtime call or kernel launch failed */
    OFFT_ERR_BAD_PLAN = -6,         /* handle of the wrong kind, or a forced plan string that does not parse or fit */
    OFFT_ERR_IO = -7                /* plan cache / weights file unreadable (non-fatal inside planning) */
};

/* plan selection modes (the paper's run-time auto-tuning, Sec. 3.2.3) */
enum {
    OFFT_TUNE_NONE = 0,       /* fixed heuristic plan (the default, like the paper's default method) */
    OFFT_TUNE_EXHAUSTIVE = 1, /* time every candidate plan at init, keep the fastest */
    OFFT_TUNE_LEARNED = 2,    /* rank candidates with the learned selector, no exhaustive timing */
    OFFT_TUNE_FORCED = 3      /* use the plan string given in forced_plan (the paper's User-select) */
};

typedef struct offt_opts {
    int tune;                 /* OFFT_TUNE_* (default NONE) */
    int reps;                 /* timed runs per candidate when tuning (default 2, after 1 warm-up) */
    int normalize_inverse;    /* 1: backward multiplies by 1/(Na Nb Nc) (default 0) */
    const char* forced_plan;  /* plan string for OFFT_TUNE_FORCED (format of offt_plan_describe) */
    const char* cache_path;   /* plan cache file for tuned plans, or NULL */
    const char* weights_path; /* learned-selector weights for OFFT_TUNE_LEARNED, or NULL */
    void* stream;             /* hipStream_t for tuning runs (NULL = null stream) */
    int tune_inplace;         /* 1: time whole transforms in place (in == out) when tuning;
                                 0 (default): out of place, with a second temporary buffer */
    int use_graph;            /* 1: offt_exec_fwd/bwd replay a HIP graph of the plan's pass
                                 kernels, one per direction, captured (on a private stream
                                 made at plan time) by that direction's first exec and
                                 captured again, updating the instantiated graph in place,
                                 when an exec brings other buffers; 0 (default): the kernels
                                 are launched directly */
    int layout;               /* OFFT_LAYOUT_* (default NATURAL), see below */
} offt_opts;

/* Order of the transformed grids (offt_opts.layout).
 *   NATURAL   forward output and backward input in the input's order,
 *             Na x Nb x Nc with c fastest.
 *   REVERSED  forward output and backward input in cba order: each grid is
 *             Nc x Nb x Na with a fastest, Y[c][b][a] = X[a][b][c] -- the
 *             distribution the paper's transform finishes in (Sec. 2, the
 *             transpose order abc -> cab -> cba; Sec. 3.1.1, the output
 *             index set differs from the input's).  Forward input and
 *             backward output stay natural.  One pass of each direction
 *             transposes on the fly (it reads the lines of its axis in one
 *             order and writes them in the other), so the reversal costs no
 *             pass of its own.  The plan owns a workspace of one batch of
 *             grids (offt_workspace_bytes) that the passes route through;
 *             in == out stays allowed.  Plan strings of such plans read
 *             "<forward>|<backward>", the backward plan naming the axes of
 *             its cba input (its a is the grid's c), each with ";rev=a" or
 *             ";rev=c" for the axis whose pass transposes.  With at most one
 *             axis longer than 1 both orders are the same memory and the
 *             plan is the natural one. */
#define OFFT_LAYOUT_NATURAL 0
#define OFFT_LAYOUT_REVERSED 1

/* Fill *o with the defaults listed above. */
void offt_opts_default(offt_opts* o);

/* Create a plan for `batch` grids of Na x Nb x Nc points of precision `dtype`
 * with the heuristic plan.  Axis lengths must be >= 1, 2/3/5-smooth and at most
 * OFFT_MAX_AXIS; batch >= 1.  Allocates the twiddle tables once.  Returns NULL
 * on error (OFFT_ERR_INVALID_ARG, OFFT_ERR_UNSUPPORTED_SIZE,
 * OFFT_ERR_NO_DEVICE, OFFT_ERR_OUT_OF_MEMORY, OFFT_ERR_HIP). */
offt_plan_t offt_plan(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch);

/* As offt_plan with options `o` (NULL = defaults).  Tuning runs here, on
 * o->stream, with internally allocated temporary buffers that are freed before
 * returning.  Errors as offt_plan, plus OFFT_ERR_BAD_PLAN for an unusable
 * forced plan string. */
offt_plan_t offt_plan_ex(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch,
                         const offt_opts* o);

#define OFFT_MAX_AXIS 1024

/* ---- grids of 1 to 5 axes -------------------------------------------------
 * The decomposition method is stated for multi-dimensional transforms, axes
 * named a, b, c, ... for the first, second, third dimension (Sec. 1), and the
 * package's future work goes beyond three dimensions (Sec. 5).  A plan for
 * `batch` grids of dims[0] x ... x dims[ndim-1] points, row-major with the
 * last axis fastest (a contiguous tensor of shape (batch?, *dims)),
 * 1 <= ndim <= OFFT_MAX_DIMS, each axis as in offt_plan.
 *   ndim <= 3: the three-dimensional plan of the shape padded with leading
 *              unit axes (every option of offt_plan_ex applies).
 *   ndim 4, 5: one axis pass per axis longer than 1 on the same kernels,
 *              lines of axis i strided by the product of the later axes.
 *              The heuristic runs the passes from the last axis to the
 *              first; OFFT_TUNE_EXHAUSTIVE times every kernel and tile width
 *              of each axis, then every order of the passes (up to 5! = 120,
 *              the GPU counterpart of the paper's search over transpose
 *              orders), and above 512 MiB slab schedules (the pass over a
 *              first, the others on blocks of the trailing axes, as
 *              ";slab=S" of offt_plan_describe); OFFT_TUNE_LEARNED falls back
 *              to it.  Plan strings name the axes a..e
 *              ("order=edcba;a=...;...;e=...").  The layout must be
 *              OFFT_LAYOUT_NATURAL.
 * Executed, described and destroyed with the same calls as offt_plan.
 * Errors as offt_plan_ex. */
#define OFFT_MAX_DIMS 5
offt_plan_t offt_plan_nd(int ndim, const int64_t* dims, int dtype, int64_t batch, const offt_opts* o);

/* Plan string of a 4- or 5-axis grid without a device: with plan == NULL the
 * heuristic plan, else `plan` checked and in canonical form (as
 * offt_plan_string).  Returns the full length or INVALID_ARG /
 * UNSUPPORTED_SIZE / BAD_PLAN. */
int offt_plan_string_nd(int ndim, const int64_t* dims, int dtype, const char* plan, char* buf, size_t n);

/* Forward / backward transform of the plan's `batch` grids from `in` to `out`
 * (device pointers, layout above).  in == out is allowed (in place); any other
 * overlap is invalid.  Never allocates, never synchronises.
 * Errors: OFFT_ERR_INVALID_ARG (NULL plan or pointer), OFFT_ERR_BAD_PLAN
 * (plan made by offt_plan_many), OFFT_ERR_HIP (launch failure). */
int offt_exec_fwd(offt_plan_t p, const void* in, void* out, void* stream);
int offt_exec_bwd(offt_plan_t p, const void* in, void* out, void* stream);

/* offt_exec_bwd with the scaling chosen for this call: normalize = 1 multiplies
 * the result by 1/(Na Nb Nc), 0 leaves it unnormalised, -1 takes the plan's
 * normalize_inverse (the paper states no normalisation; the scaled inverse is
 * the backward transform divided by the grid's point count).  A use_graph plan
 * replays its graph when the choice equals the plan's and launches the pass
 * kernels directly otherwise.  Errors as offt_exec_bwd, plus INVALID_ARG for
 * normalize outside {-1, 0, 1}. */
int offt_exec_bwd_norm(offt_plan_t p, const void* in, void* out, int normalize, void* stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the forward
 * (direction OFFT_FORWARD) or backward (OFFT_BACKWARD, scaled by
 * 1/(Na Nb Nc) when normalize = 1) transform of `batch` grids of
 * Na x Nb x Nc points, natural layout, with no plan object and no device
 * allocation.  It runs the heuristic plan of offt_plan with the same kernels,
 * so its results equal offt_exec_fwd / offt_exec_bwd of such a plan bit for
 * bit.  The twiddle tables (one per distinct axis length, at most 3 of
 * OFFT_MAX_AXIS complex values) live in a file-scope device array of 48 KiB
 * that each GPU the library runs on holds until the process ends; every call
 * rewrites them on `stream` before its passes, so calls that overlap on one
 * GPU (on different streams) race and must not be issued.  Axis lengths as
 * offt_plan (2/3/5-smooth, at most OFFT_MAX_AXIS: longer axes would not fit a
 * table and are rejected with OFFT_ERR_UNSUPPORTED_SIZE).  Stream-ordered,
 * never synchronises.  Errors: INVALID_ARG, UNSUPPORTED_SIZE, NO_DEVICE,
 * HIP. */
int offt_exec_noalloc(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch, int direction, int normalize,
                      const void* in, void* out, void* stream);

/* Number of axis passes of a plan (0..3: axes of length 1 need none), or a
 * negative code. */
int offt_plan_passes(offt_plan_t p);

/* Launch only axis pass i (0-based, plan order) of the forward
 * (direction = OFFT_FORWARD) or backward (OFFT_BACKWARD) transform.  Launching
 * passes 0..n-1 in order on one stream with the same in/out gives exactly
 * the result of offt_exec_fwd / offt_exec_bwd (pass 0 reads `in`, later
 * passes work in place on `out`; in REVERSED layouts the passes route
 * through the plan's workspace exactly as exec does; a pass of a slab or
 * column-block schedule runs here over all its blocks, one launch per block,
 * where exec interleaves the passes block by block); it exists so that each
 * pass can be timed on its own.
 * Errors: INVALID_ARG (NULL plan/pointer, i out of range, bad direction),
 * BAD_PLAN, HIP. */
int offt_exec_pass(offt_plan_t p, int i, int direction, const void* in, void* out, void* stream);

/* Launch passes first .. first+count-1 (plan order) exactly as offt_exec_fwd /
 * offt_exec_bwd launches them: same buffers, conjugation and scaling as
 * offt_exec_pass, and the passes of a slab or column-block schedule
 * (offt_plan_describe's ";slab=S", ";col=W") interleaved block by block.  A range covering every pass is
 * offt_exec_fwd / offt_exec_bwd; ranges launched back to back give the same
 * result.  It exists so that the pass over a and the slab schedule after it
 * can be timed apart.  Errors: INVALID_ARG (NULL plan/pointer, count < 1,
 * range outside 0..passes-1, bad direction), BAD_PLAN, HIP. */
int offt_exec_range(offt_plan_t p, int first, int count, int direction, const void* in, void* out,
                    void* stream);

/* Copy of axis pass i's memory accesses, the measured ceiling of that pass:
 * the pass's tiles (lines per workgroup, threads, tile order, grid-data
 * access mode), every thread loading the elements its first-stage
 * butterflies read (positions b + r L/R0 of its line) in one burst and
 * storing them to the same positions of `out`; no arithmetic, no LDS
 * exchange.  Moves the same bytes as the pass (2 N s per grid).  in != out,
 * each holding batch grids.  Errors: INVALID_ARG, BAD_PLAN (not a plan of
 * kind offt_plan/offt_plan_nd, or a transposing pass), UNSUPPORTED_SIZE, HIP. */
int offt_copy_pass(offt_plan_t p, int i, const void* in, void* out, void* stream);

/* Free every plan-owned allocation.  NULL is a no-op.  The handle is invalid
 * afterwards. */
int offt_destroy(offt_plan_t p);

/* Plan string (axis order, radix sequence, tile width and pass mode of each
 * axis pass) written NUL-terminated into buf[0..n).  Returns the length of the
 * full string, or a negative code; the string is truncated if n is too small.
 * A trailing ";slab=S" marks a slab schedule: the pass over a runs first over
 * the whole grid, then the passes over b and c run S planes (Nb x Nc, counted
 * over the batch) at a time, both passes of one slab before the next slab,
 * so that a slab's second pass finds the first one's output in the
 * Infinity Cache (natural layout only; the exhaustive tuner tries it for
 * grids above 512 MiB).  A trailing ";col=W" marks the column-block
 * schedule instead: the pass over c first over the whole grid, then the
 * passes over b and a on blocks of W consecutive columns c (W a power of two
 * dividing Nc and at least their tile widths).  Every element goes through
 * the same arithmetic as without either: results are bit-identical to the
 * plan without ";slab=" or ";col=". */
int offt_plan_describe(offt_plan_t p, char* buf, size_t n);

/* Bytes of device memory the plan owns (twiddle tables, scratch). */
int64_t offt_workspace_bytes(offt_plan_t p);

/* Last error code of the calling thread, and a static text for a code. */
int offt_last_error(void);
const char* offt_error_string(int code);

/* Plan string of the heuristic plan (OFFT_TUNE_NONE) for one grid shape,
 * written like offt_plan_describe.  Needs no device: the per-workgroup LDS
 * limit is the current device's when one is visible, 64 KiB otherwise.
 * Returns the full string length or INVALID_ARG / UNSUPPORTED_SIZE. */
int offt_default_plan_string(int64_t Na, int64_t Nb, int64_t Nc, int dtype, char* buf, size_t n);

/* Plan strings of either layout without a device: with plan == NULL the
 * heuristic plan of `layout` (OFFT_LAYOUT_*) for one grid shape; otherwise
 * `plan` parsed and written back in canonical form, after checking that it
 * names compiled kernels, that exchanges in parts sit on strided lines only,
 * that the transposing axis (";rev=") has a transposing kernel and that the
 * output order matches `layout` (tile sizes are checked against the device
 * at plan time, not here).  Returns the full string length, or
 * INVALID_ARG / UNSUPPORTED_SIZE / BAD_PLAN. */
int offt_plan_string(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int layout, const char* plan, char* buf,
                     size_t n);

/* Write the device-generated forward twiddle table W_n^m, m < n, of precision
 * `dtype` to host memory `host_out` (n interleaved complex values).  The table
 * is computed in binary64 on the GPU and rounded to nearest for OFFT_C2C_F32.
 * For tests of the twiddle generator.  Errors: INVALID_ARG, NO_DEVICE, HIP. */
int offt_twiddles(int64_t n, int dtype, void* host_out);

/* ---- batches of grids of different sizes (uneven batch) ------------------
 * `count` grids, grid i of dims[3i] x dims[3i+1] x dims[3i+2], all of precision
 * `dtype`, packed back to back in one buffer; grid i starts at element offset
 * offt_many_offset(p, i) (every grid starts on a 256-byte boundary).  With
 * o->tune = OFFT_TUNE_EXHAUSTIVE each distinct grid shape gets its own tuned
 * plan.  Execution (offt_exec_many and its default forms below) runs every
 * (grid, axis pass, tile) work item of the batch in one of several launch
 * forms: one kernel per pass level, the three replayed from one HIP graph
 * (the default, fastest measured), one persistent kernel replayed from a
 * graph, or each grid's passes as separate launches.  Grids stay in natural order
 * (o->layout other than NATURAL is OFFT_ERR_INVALID_ARG).  Errors as
 * offt_plan_ex. */
offt_plan_t offt_plan_many(int count, const int64_t* dims, int dtype, const offt_opts* o);

/* Element offset of grid i in the packed buffer, total elements of the
 * packed buffer (i = count), or a negative code. */
int64_t offt_many_offset(offt_plan_t p, int i);

/* Transform every grid of the packed buffer (direction OFFT_FORWARD or
 * OFFT_BACKWARD; the plan's normalize_inverse scales each grid by 1/its N).
 * in == out allowed.  `use_graph` selects the launch (OFFT_MANY_*):
 *    1  PERSISTENT_GRAPH: one persistent kernel over every (grid, pass, tile)
 *       work item, after a counter-reset kernel, replayed from a HIP graph
 *       built on the first call; later calls with other buffers or direction
 *       update the graph's kernel arguments;
 *    0  PERSISTENT: the same two kernels launched directly;
 *    2  LEVELS_GRAPH: one kernel per pass level (all grids' first passes, then
 *       all second, then all third), one workgroup per tile, replayed from a
 *       HIP graph built on the first call;
 *    3  LEVELS: the same kernels launched directly;
 *    6  LEVELS_GROUPED_GRAPH: the level kernels group by group: consecutive
 *       grids in groups of at most 192 MiB of grid data (a larger grid
 *       alone), each group's levels one after the other before the next
 *       group's, so that a group's later levels read what its earlier ones
 *       wrote from the 256 MB Infinity Cache; replayed from a HIP graph built
 *       on the first call;
 *    5  SYNC_GRAPH: one level-synchronous persistent kernel, after a counter
 *       reset, replayed from a HIP graph: one resident workgroup per slot the
 *       device has, each level's tiles dealt round-robin in the level
 *       kernels' order, a grid barrier between levels (plain stores, one L2
 *       write-back and invalidate per workgroup per barrier);
 *    4  SYNC: the same two kernels launched directly;
 *   -1  SEPARATE_HEURISTIC: every grid's passes as ordinary launches with the
 *       heuristic plans;
 *   -2  SEPARATE_TUNED: the same with the plans chosen at plan time.
 * The level forms (2, 3, 6) run any batch whose axes are all at most 160 long;
 * the persistent forms (0, 1, 4, 5) only batches whose axis lengths all lie
 * in the set {48, 60, 64, 80, 96, 120, 128, 150, 160} (lengths 1 are fine
 * for both).
 * Never allocates device memory.  Errors: INVALID_ARG, BAD_PLAN (not a
 * many-plan), UNSUPPORTED_SIZE (use_graph >= 0 for a batch outside that
 * form's lengths), HIP. */
int offt_exec_many(offt_plan_t p, const void* in, void* out, int direction, int use_graph,
                   void* stream);

/* offt_exec_many in the default launch form: LEVELS_GRAPH when every axis
 * of the batch is at most 160 long, else SEPARATE_TUNED.  Same errors. */
int offt_exec_many_fwd(offt_plan_t p, const void* in, void* out, void* stream);
int offt_exec_many_bwd(offt_plan_t p, const void* in, void* out, void* stream);

/* After the stream that ran offt_exec_many has been synchronised: 0 if the
 * last persistent run (PERSISTENT* or SYNC*) completed every dependency or
 * barrier wait normally, OFFT_ERR_HIP if a wait hit its bounded spin limit
 * (results then invalid; for SYNC* this happens when not every workgroup of
 * the launch could be resident, e.g. while other work holds the device). */
int offt_many_status(offt_plan_t p);

/* ---- the distributed calculation flow on virtual processes ----------------
 * The paper's method itself (Sec. 2, Sec. 3.1.1, Fig. 1b) run by `nprocs`
 * virtual processes on one GPU.  Process p owns the block of Eq. 2 of the
 * linear index of the order the data is currently held in: whole N2 x N3
 * planes when nprocs <= N1, whole N3-lines when N1 < nprocs <= N1 N2 (the
 * 1-D and 2-D decompositions, Eq. 2-9), over that order's leading dimensions
 * (N1, N2, N3) = (Na, Nb, Nc) for abc, (Nc, Na, Nb) for cab, (Nc, Nb, Na) for
 * cba.  Each block is a contiguous slice of the grid held in that order, so
 * the processes' local arrays are consecutive slices of one array.
 *
 * Forward (offt_exec_fwd): `in` is the grid in abc order (process p's input
 * is its abc block); per process, the 1-D transforms of its lines along c,
 * the transpose abc -> cab, the transforms along b, the transpose
 * cab -> cba, the transforms along a; `out` receives the transform in cba
 * order, Y[c][b][a] = X[a][b][c] (process p's output is its cba block: the
 * distribution the paper's transform finishes in).  Backward
 * (offt_exec_bwd, offt_exec_bwd_norm): cba input, abc output, the steps in
 * reverse with the conjugate roots of unity.  in == out is allowed.
 *
 * A transpose packs each process's elements into one chunk per destination
 * (each chunk in the destination's order, a process's own chunk straight to
 * its place), copies the chunks that change process between the processes'
 * send and receive slices, and unpacks them into the destination's local
 * array (when a process receives only from itself its pack writes that
 * array directly).  The copies follow one of the six communication methods
 * of Sec. 3.2.1 (OFFT_COMM_*):
 *   ISEND_WAITALL        every chunk posted at once as its own copy on a
 *                        communication stream, then one wait for all, then
 *                        the unpacks;
 *   ALLTOALLV            one collective copy launch over every chunk, then
 *                        the unpacks;
 *   ISEND_WAITALL_BLOCK  the processes taken in groups of block_size
 *                        destinations (the paper's B_SIZE, 32 there): each
 *                        group's chunks posted, then waited for, group after
 *                        group; then the unpacks;
 *   ISEND_WAITSOME       every chunk posted at once; each chunk is unpacked
 *                        as soon as it has arrived (an event per chunk), while
 *                        the others are still in flight;
 *   ISEND_WAITSOME_BLOCK the same per group of block_size destinations, the
 *                        next group posted once the current one is unpacked;
 *   SENDRECV             nprocs - 1 steps after the own chunk: at step i
 *                        every process sends to process myid + i and
 *                        receives from myid - i (mod nprocs), the received
 *                        chunk unpacked before the next step.
 * OFFT_COMM_AUTO times every method at plan time on the plan's stream (one
 * warm-up and o->reps timed forward transforms each, minimum of two, median
 * of more) and keeps the fastest, ties to the lower id: the paper's
 * auto-tuning of communication in the initialization phase (Sec. 3.2.3).
 * Without it the given method is used (the paper's User-select; its default
 * is ISEND_WAITSOME).
 *
 * Limits: 1 <= nprocs <= min(64, N1 N2 of every order); block_size >= 1.
 * The plan owns three arrays of the grid's size (work, send, receive), a
 * communication stream (default priority) and its events.  Exec never
 * allocates; a plan must not run on two streams at once. */
#define OFFT_COMM_AUTO (-1)
#define OFFT_COMM_ISEND_WAITALL 0
#define OFFT_COMM_ALLTOALLV 1
#define OFFT_COMM_ISEND_WAITALL_BLOCK 2
#define OFFT_COMM_ISEND_WAITSOME 3
#define OFFT_COMM_ISEND_WAITSOME_BLOCK 4
#define OFFT_COMM_SENDRECV 5

/* Orders of offt_dist_block. */
#define OFFT_ORDER_ABC 0
#define OFFT_ORDER_CAB 1
#define OFFT_ORDER_CBA 2

/* Plan of the distributed flow for one grid over `nprocs` virtual processes
 * with communication method `method` (OFFT_COMM_*) and group size
 * block_size.  From o: normalize_inverse, reps and stream (tuning).  Errors:
 * INVALID_ARG (sizes, nprocs, method, block_size), UNSUPPORTED_SIZE,
 * NO_DEVICE, OUT_OF_MEMORY, HIP. */
offt_plan_t offt_plan_dist(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int nprocs, int method, int block_size,
                           const offt_opts* o);

/* The method a distributed plan runs (OFFT_COMM_*), or a negative code. */
int offt_dist_method(offt_plan_t p);

/* ms[0..6): time of a forward transform with each method as measured at plan
 * time by OFFT_COMM_AUTO (-1 each when the method was given).  Returns 6 or a
 * negative code. */
int offt_dist_method_times(offt_plan_t p, float* ms);

/* Elements process src sends to process dst in transpose `step` of the
 * forward (OFFT_FORWARD: 0 abc -> cab, 1 cab -> cba) or backward flow
 * (OFFT_BACKWARD: 0 cba -> cab, 1 cab -> abc), as the plan moves them
 * (src == dst: the elements that stay local).  Errors: INVALID_ARG,
 * BAD_PLAN. */
int64_t offt_dist_count(offt_plan_t p, int direction, int step, int src, int dst);

/* Block of process proc in order OFFT_ORDER_*: returns its first linear index
 * and writes one past its last to *end (if end != NULL).  Errors:
 * INVALID_ARG, BAD_PLAN. */
int64_t offt_dist_block(offt_plan_t p, int order, int proc, int64_t* end);

/* The first `steps` (1..5) steps of the forward or backward flow from `in` to
 * `out`, with `method` (OFFT_COMM_AUTO: the plan's): `out` then holds the
 * processes' local arrays after that step, concatenated in process order --
 * the grid in that step's order (forward: abc, cab, cab, cba, cba; backward:
 * cba, cab, cab, abc, abc).  For tests of every step.  Never allocates.
 * Errors: INVALID_ARG, BAD_PLAN, HIP. */
int offt_dist_exec_steps(offt_plan_t p, int direction, int steps, int method, const void* in, void* out,
                         void* stream);

/* ---- byte and volume accounting (host only, no device) --------------------
 * Per plan: HBM bytes of one axis pass.  Per decomposition: the row-wise
 * block distribution of Duy & Ozaki, Sec. 2 (Eq. 2 and the index ranges
 * derived from it) and the elements each transpose of the order sequence
 * abc -> cab -> cba (Sec. 2, Fig. 1b) moves between processes, the volume of
 * communication of Sec. 4.1.  Results are element counts or bytes (>= 0), or
 * a negative error code (also in offt_last_error()). */

/* Bytes one axis pass of a plan moves to and from HBM: every element of the
 * batch read once and written once, 2 * batch * Na * Nb * Nc * (16 | 8).
 * Twiddle tables are not counted.  Errors: INVALID_ARG, UNSUPPORTED_SIZE. */
int64_t offt_pass_bytes(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch);

/* f(N1, N2, N3, Np, id) of Eq. 2: first row-major linear index of process
 * id's block (0 <= id <= Np; id = Np gives N1 N2 N3).  Whole N2 x N3 planes
 * when Np <= N1, whole N3-lines when N1 < Np <= N1 N2.  Errors: INVALID_ARG
 * (a length < 1 or > 2^20, Np outside [1, N1 N2], id outside [0, Np]). */
int64_t offt_decomp_start(int64_t n1, int64_t n2, int64_t n3, int64_t np, int64_t id);

/* Elements process src holds before transpose `step` and process dst holds
 * after it, for an n1 x n2 x n3 grid (a, b, c) over np processes; step 0:
 * abc -> cab (each order split by Eq. 2 over its own leading lengths), step
 * 1: cab -> cba.  src == dst counts what stays local.  Errors: INVALID_ARG
 * (np above what Eq. 2 covers for either order, src or dst outside [0, np)). */
int64_t offt_transpose_count(int64_t n1, int64_t n2, int64_t n3, int64_t np, int step, int64_t src,
                             int64_t dst);

/* Elements that leave their process in transpose `step` (the sum of
 * offt_transpose_count over src != dst).  Errors as offt_transpose_count. */
int64_t offt_transpose_volume(int64_t n1, int64_t n2, int64_t n3, int64_t np, int step);

/* ---- plan selection internals: candidates, features, timings -------------
 * The learned selector chooses among a deterministic list of candidate plans
 * per grid shape (the heuristic plan first; then other radix sequences and
 * tile widths per axis; then the heuristic with one axis's tile order
 * switched between launch order and XCD-contiguous order; then the other five
 * axis orders; then the heuristic with one axis's access mode switched
 * between streaming and cached grid data).  These calls expose that list for
 * building and using the learned selector. */

/* Length of one plan feature vector. */
int offt_feature_dim(void);

/* Candidate plans of a grid: returns their number n; the first min(n, max)
 * plan strings are written NUL-separated into plans[0..plans_bytes) and their
 * feature vectors (offt_feature_dim() floats each) into features.  Host only,
 * no device needed.  Errors: INVALID_ARG (buffers too small), UNSUPPORTED_SIZE. */
int offt_candidates(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch, char* plans,
                    size_t plans_bytes, float* features, int max);

/* Times every candidate plan of a grid as the exhaustive tuner does
 * (1 warm-up + reps timed forward transforms, minimum of up to two runs,
 * median of more, HIP events on
 * `stream`), in place on the caller's device buffer `buf` of at least
 * batch*Na*Nb*Nc elements, which is filled with uniform random values before
 * each candidate (its contents are destroyed).  times_ms[i] is
 * candidate i's time for i < min(n, max).  Returns n.  Synchronises the
 * stream.  Errors: INVALID_ARG, UNSUPPORTED_SIZE, NO_DEVICE, HIP. */
int offt_tune_table(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch, int reps, void* buf,
                    size_t buf_bytes, void* stream, float* times_ms, int max);

/* Feature vector (offt_feature_dim() floats) of one plan string for a grid.
 * Host only; the plan string is not checked against this device's tile
 * limits.  Errors: INVALID_ARG, UNSUPPORTED_SIZE, BAD_PLAN. */
int offt_plan_features(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch, const char* plan,
                       float* out);

/* Predicted ln(time in ms) of n feature vectors with the network in the
 * weights file.  Host only.  Errors: INVALID_ARG, IO. */
int offt_selector_scores(const char* weights_path, const float* features, int n, float* scores);

/* The plan the learned selector picks for a grid, from the weights file at
 * weights_path (format: offt-selector 1 text; see paper_1501_07350_amd/
 * selector.py), written like offt_plan_describe.  Host only.  Errors:
 * INVALID_ARG, UNSUPPORTED_SIZE, IO (missing or corrupt weights). */
int offt_selector_choose(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch,
                         const char* weights_path, char* buf, size_t n);

/* ---- the selector's network: MLP with two hidden ReLU layers -------------
 *   a1 = relu(W1 x + b1), a2 = relu(W2 a1 + b2), y = w3 . a2 + b3,
 *   loss = mean over the minibatch of (y - t)^2.
 * Parameters: one float vector W1[H][D], b1[H], W2[H][H], b2[H], w3[H], b3. */
typedef struct offt_mlp_s* offt_mlp_t;

/* Number of parameters for input width D and hidden width H (1..256). */
int64_t offt_mlp_nparams(int in_dim, int hidden);

/* Seeded initial parameters (He-uniform weights, zero biases) into host_out. */
void offt_mlp_init_params(int in_dim, int hidden, uint64_t seed, float* host_out);

/* Network on the device with room for minibatches of up to max_batch;
 * parameters from host_params (NULL: offt_mlp_init_params(seed)).  Adam
 * moments start at zero.  Errors: INVALID_ARG, NO_DEVICE, OUT_OF_MEMORY, HIP. */
offt_mlp_t offt_mlp_create(int in_dim, int hidden, int max_batch, const float* host_params, uint64_t seed);
int offt_mlp_destroy(offt_mlp_t m);
int offt_mlp_get_params(offt_mlp_t m, float* host_out);
int offt_mlp_set_params(offt_mlp_t m, const float* host_in);   /* also resets Adam */

/* y[b] = network(X[row_b]) for b < B, row_b = idx[b] (idx == NULL: b).  X is
 * a device array of rows of D floats; y a device array of B floats. */
int offt_mlp_forward(offt_mlp_t m, const float* X, const int32_t* idx, int B, float* y, void* stream);

/* Gradient of the mean squared error over the minibatch rows idx[0..B)
 * (B <= max_batch) with targets T[row]: grad (device, nparams floats) and,
 * if loss != NULL, the loss (device float). */
int offt_mlp_gradient(offt_mlp_t m, const float* X, const float* T, const int32_t* idx, int B, float* grad,
                      float* loss, void* stream);

/* One Adam step (Kingma & Ba) with bias correction on the device parameters. */
int offt_mlp_adam(offt_mlp_t m, const float* grad, float lr, float beta1, float beta2, float eps, void* stream);

#define OFFT_MANY_SEPARATE_TUNED (-2)
#define OFFT_MANY_SEPARATE_HEURISTIC (-1)
#define OFFT_MANY_PERSISTENT 0
#define OFFT_MANY_PERSISTENT_GRAPH 1
#define OFFT_MANY_LEVELS_GRAPH 2
#define OFFT_MANY_LEVELS 3
#define OFFT_MANY_SYNC 4
#define OFFT_MANY_SYNC_GRAPH 5
#define OFFT_MANY_LEVELS_GROUPED_GRAPH 6

#define OFFT_FORWARD (-1)
#define OFFT_BACKWARD (+1)

#ifdef __cplusplus
}
#endif

#endif /* OFFT_H */
