/*
 * hx — asynchronous copies and stencil launches composed as a future graph,
 * for one AMD Instinct MI355X (gfx950).
 *
 * The paper (Diehl et al., "Integration of CUDA Processing within HPX",
 * arXiv:1810.11482) gives every accelerator operation an asynchronous return
 * value (Sec. III-A "Futurization"), organises the accelerator as a device
 * with its own work queue, buffers on that device and programs run on it
 * (Sec. IV, the device/buffer/program classes), and composes copies and kernel
 * runs through those return values so that copies overlap computation
 * (Sec. IV-B, Listing 2; Sec. V-A.2, Algorithm 1).  This header is that
 * interface as a C ABI:
 *
 *   paper                                  hx
 *   device (own async work queue)          hx_ctx (one GPU, its stream set)
 *   device.create_buffer(bytes)            hx_buffer_create
 *   buffer.enqueue_write / enqueue_read    hx_copy_async (H2D / D2H)
 *   program.run(args, grid, block)         hx_launch_* (deps = futures)
 *   hpx::future<void>                      hx_event
 *   hpx::when_all / wait_all / .get()      hx_when_all / hx_wait
 *   cudaMallocHost                         hx_host_alloc
 *
 * Conventions
 *  - Every function returns an hx_status: HX_OK (0) or a negative error.
 *  - Handles (hx_buffer, hx_event, hx_plan) are opaque 64-bit values tagged
 *    with a generation; a released or foreign handle gives HX_ERR_INVALID.
 *    The value 0 is never a valid handle; as a dependency, event 0 means
 *    "already complete" and is ignored.
 *  - Argument and validation errors are reported synchronously: nothing is
 *    enqueued and the output event is left untouched.
 *  - Operations take a list of events they depend on.  The dependency is
 *    resolved on the GPU (stream-waits on the producers' events); the host
 *    blocks only in hx_wait.  If a dependency has failed the operation is not
 *    run and its event completes with HX_ERR_DEP_FAILED (exception-carrying
 *    futures).  A dependency on a user event that is not yet set holds the
 *    operation back on the host until it is.
 *  - Byte offsets are into the buffer; element counts are in cells of the
 *    operation's dtype.
 *  - All calls on one context are thread-safe.
 */
#ifndef HX_H
#define HX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------------- status */
typedef int32_t hx_status;

#define HX_OK 0
#define HX_PENDING 1           /* event not complete yet (hx_event_query) */
#define HX_ERR_INVALID (-1)    /* unknown, released or foreign handle */
#define HX_ERR_ARG (-2)        /* invalid argument */
#define HX_ERR_NO_DEVICE (-3)  /* no GPU, or a host-only context */
#define HX_ERR_HIP (-4)        /* the HIP runtime reported an error */
#define HX_ERR_OOM (-5)        /* allocation failed */
#define HX_ERR_DEP_FAILED (-6) /* a dependency failed; the operation did not run */
#define HX_ERR_TIMEOUT (-7)    /* hx_wait timed out; the event is still pending */
#define HX_ERR_INJECTED (-8)   /* failure injected by hx_debug_inject */
#define HX_ERR_HAZARD (-9)     /* hazard checker found an unordered conflict */
#define HX_ERR_UNSUPPORTED (-10)
#define HX_ERR_RANGE (-11)     /* byte range outside a buffer */

typedef struct hx_ctx_s* hx_ctx;
typedef uint64_t hx_buffer;
typedef uint64_t hx_event;
typedef uint64_t hx_plan;

typedef enum { HX_F32 = 0, HX_F64 = 1 } hx_dtype;

/* Human-readable name of a status code (static string). */
const char* hx_status_string(hx_status s);

/* ----------------------------------------------------------------- device */
typedef struct {
    char name[64];
    char arch[64];          /* e.g. "gfx950" */
    int compute_units;
    int wavefront_size;
    int clock_khz;
    int memory_clock_khz;
    int memory_bus_bits;
    size_t hbm_bytes;
    size_t lds_bytes_per_cu;
    size_t l2_bytes;
} hx_device_info_t;

/* Number of visible GPUs (0 when there is none). */
hx_status hx_device_count(int* count);

/* Properties of device `dev`.  Stands in for the paper's device discovery with
 * a capability filter (Sec. IV-A, Listing 1), restricted to local devices. */
hx_status hx_device_info(int dev, hx_device_info_t* info);

/* ---------------------------------------------------------------- context */
typedef struct {
    int compute_streams;        /* kernel streams; 0 = two fewer than the hardware
                                   queues HIP uses (GPU_MAX_HW_QUEUES, 4 by default),
                                   so the copy streams keep queues of their own */
    void* external_stream;      /* optional hipStream_t used as compute stream 0
                                   (e.g. torch's current stream); not owned */
    int check;                  /* 1 = record accesses and run the hazard checker */
    int timing;                 /* 1 = events carry timestamps (hx_event_elapsed) */
} hx_ctx_opts;

/* Create a context on device `dev` (the paper's device with its own work
 * queue, Sec. IV).  dev = -1 creates a host-only context: events, user events,
 * hx_when_all, hx_wait and the hazard checker work, every GPU operation returns
 * HX_ERR_NO_DEVICE.  `opts` may be NULL.  On error *ctx is untouched. */
hx_status hx_ctx_create(int dev, const hx_ctx_opts* opts, hx_ctx* ctx);

/* Wait for all outstanding work, then free every buffer, plan and event the
 * context owns (wrapped memory is not freed). */
hx_status hx_ctx_destroy(hx_ctx ctx);

/* Block until every operation submitted so far has finished. */
hx_status hx_ctx_synchronize(hx_ctx ctx);

/* Last error message recorded on the context (truncated to len-1 bytes). */
hx_status hx_last_error(hx_ctx ctx, char* buf, size_t len);

/* ---------------------------------------------------------------- buffers */
/* Device allocation of `bytes` (the paper's create_buffer, Sec. IV and
 * Listing 2).  The memory is uninitialised and owned by the context. */
hx_status hx_buffer_create(hx_ctx ctx, size_t bytes, hx_buffer* buf);

/* Wrap existing device memory (e.g. a torch tensor's storage) without taking
 * ownership; hx_buffer_destroy never frees it. */
hx_status hx_buffer_wrap(hx_ctx ctx, void* dev_ptr, size_t bytes, hx_buffer* buf);

/* Release a buffer handle.  The handle is invalid at once; the memory of an
 * owned buffer is freed only after every submitted operation that uses it has
 * completed. */
hx_status hx_buffer_destroy(hx_ctx ctx, hx_buffer buf);

/* Device address and size of a buffer. */
hx_status hx_buffer_ptr(hx_ctx ctx, hx_buffer buf, void** dev_ptr, size_t* bytes);

/* Page-locked host memory (cudaMallocHost in Listing 2), which makes host
 * copies truly asynchronous.  Freed with hx_host_free or at context destroy. */
hx_status hx_host_alloc(hx_ctx ctx, size_t bytes, void** host_ptr);
hx_status hx_host_free(hx_ctx ctx, void* host_ptr);

/* ----------------------------------------------------------------- copies */
typedef enum { HX_H2D = 0, HX_D2H = 1, HX_D2D = 2 } hx_copy_dir;

typedef struct {
    int dir;                 /* hx_copy_dir */
    void* host;              /* H2D: source, D2H: destination (caller-owned; must
                                stay valid until the event completes; pinned
                                memory from hx_host_alloc makes it asynchronous) */
    hx_buffer buf;           /* H2D/D2D: destination, D2H: source */
    size_t offset;           /* byte offset into buf */
    hx_buffer src_buf;       /* D2D: source buffer */
    size_t src_offset;       /* D2D: byte offset into src_buf */
    size_t bytes;
} hx_copy_desc;

/* Asynchronous copy (the paper's enqueue_write / enqueue_read, Sec. IV and
 * Listing 2; cudaMemcpyAsync in Algorithm 1).  H2D copies run on the
 * context's host-to-device stream, D2H copies on its device-to-host stream, so
 * the two directions and the kernels of other partitions overlap.  D2D copies
 * run on a compute stream: ranges whose ends and length are multiples of 16
 * bytes take the library's one-pass vector copy kernel (one 16-byte
 * nontemporal load and store per thread), others hipMemcpyAsync.  Ranges are
 * checked against the buffer (HX_ERR_RANGE); overlapping D2D ranges of one
 * buffer are rejected (HX_ERR_ARG). */
hx_status hx_copy_async(hx_ctx ctx, const hx_copy_desc* desc, const hx_event* deps, int ndeps,
                        hx_event* out);

/* ---------------------------------------------------------------- stencil */
typedef enum {
    HX_BC_PERIODIC = 0,      /* wrap around the array (1D only, both sides) */
    HX_BC_DIRICHLET0 = 1,    /* cells outside are held at 0 at every step */
    HX_BC_GHOST = 2          /* cells outside come from a halo region */
} hx_bc;

typedef struct {
    int dims;                /* 1 = 3-point line, 2 = 5-point grid */
    int dtype;               /* hx_dtype */
    int64_t nx;              /* 1D: cells; 2D: cells per row (row-major, no padding) */
    int64_t ny;              /* 2D: rows; ignored in 1D */
    int steps;               /* explicit time steps to take */
    double r;                /* diffusion number (dt / h^2 times the diffusivity) */
    hx_buffer in;  size_t in_offset;
    hx_buffer out; size_t out_offset;   /* must not overlap in */
    hx_buffer tmp; size_t tmp_offset;   /* ping-pong space of the same size, needed only
                                           when the run takes more than one pass */
    int bc_lo;               /* 1D: left end, 2D: top edge (hx_bc) */
    int bc_hi;               /* 1D: right end, 2D: bottom edge (hx_bc) */
    hx_buffer halo_lo; size_t halo_lo_offset;  /* HX_BC_GHOST: halo_width cells (1D) or rows
                                                  (2D) that precede the first cell/row; its
                                                  last cell/row is index -1 */
    hx_buffer halo_hi; size_t halo_hi_offset;  /* HX_BC_GHOST: halo_width cells/rows that
                                                  follow the last; its first is index n */
    int halo_width;
    /* Launch geometry (the paper keeps block and grid sizes in the user's hands,
     * Sec. IV-B and Sec. VI).  0 = the tuned default. */
    int cells_per_lane;      /* 1D: 8, 16, 32 or 64; 2D: 4 or 8 */
    int time_block;          /* steps fused per kernel pass */
    int waves_per_group;     /* 1, 2 or 4 */
    int rows_per_block;      /* 2D: output rows per wave */
} hx_stencil_args;

/* Advance the heat equation `steps` explicit steps from `in` into `out`
 * (the data-parallel kernel run of Sec. IV-B / Algorithm 1, with the
 * 3-point stencil of Sec. V-A.1 in heat form):
 *   1D  u'_i  = u_i + r (u_{i-1} - 2 u_i + u_{i+1})
 *   2D  u'_ij = u_ij + r (u_{i-1,j} + u_{i+1,j} + u_{i,j-1} + u_{i,j+1} - 4 u_ij)
 * In 2D the left and right edges are always zero-Dirichlet.  With a GHOST side
 * the run is one fused pass and needs steps <= halo_width (the halo supplies
 * the whole light cone); otherwise steps may be anything and passes of
 * `time_block` steps ping-pong between out and tmp, ending in out.
 * Stable for r <= 1/2 (1D) and r <= 1/4 (2D); other r are accepted. */
hx_status hx_launch_stencil(hx_ctx ctx, const hx_stencil_args* args, const hx_event* deps,
                            int ndeps, hx_event* out);

/* ------------------------------------------------------ partitioned arrays */
typedef enum { HX_PART_GRAPH = 0, HX_PART_PLAIN = 1, HX_PART_BATCHED = 2 } hx_part_mode;

typedef struct {
    int dtype;                  /* hx_dtype */
    int parts;                  /* number of partitions */
    const int64_t* sizes;       /* cells per partition (host array of `parts`) */
    const hx_buffer* bufs_a;    /* per partition: buffer holding the initial state at offset 0 */
    const hx_buffer* bufs_b;    /* per partition: second ping-pong buffer of the same size */
    int periodic;               /* 1 = the last partition wraps to the first; 0 = the two
                                   array ends are zero-Dirichlet */
    int steps;
    double r;
    int mode;                   /* hx_part_mode */
    int time_block;             /* steps per pass (<= the smallest partition); 0 = 32 in 1D,
                                   8 in 2D */
    int cells_per_lane;         /* kernel geometry, 0 = tuned */
    int waves_per_group;
    int dims;                   /* 0 or 1 = a 1D array split into runs of cells; 2 = a grid
                                   of nx columns split into bands of sizes[p] rows (top and
                                   bottom edges zero-Dirichlet; periodic must be 0) */
    int64_t nx;                 /* 2D: cells per row */
    int rows_per_block;         /* 2D kernel geometry, 0 = tuned */
} hx_partitioned_desc;

/* Advance a device-resident array split over `parts` buffers by `steps` heat
 * steps, as a future graph (the partition benchmark of Sec. V-A.2 /
 * Algorithm 1 with the stencil of Sec. V-A.1); 1D runs of cells or 2D row
 * bands.  HX_PART_GRAPH: node (p, b) advances partition p by one time block,
 * reading `time_block` halo cells (rows) straight from its neighbours' buffers,
 * and depends on nodes (p-1, b-1),
 * (p, b-1) and (p+1, b-1); independent nodes run concurrently on the compute
 * streams.  HX_PART_PLAIN: the comparator: one step per launch, issued in
 * Algorithm 1's order and chained on one stream.  HX_PART_BATCHED (2D bands
 * only): every pass is one launch per group of up to 16 bands (one node per
 * launch, depending on every node of the previous pass); 1D partitions batch
 * through hx_plan_create_batched.  `deps` gate the first pass.
 * *out completes when the last pass has; the final state is in bufs_b if
 * *final_in_b is 1, else in bufs_a.  node_events (optional, parts x passes
 * entries, pass-major) receives every node's event; the caller releases them. */
hx_status hx_run_partitioned(hx_ctx ctx, const hx_partitioned_desc* desc, const hx_event* deps,
                             int ndeps, hx_event* out, int* final_in_b, hx_event* node_events);

typedef struct {
    hx_partitioned_desc part;   /* steps <= smallest partition; one fused pass per partition */
    const void* host_in;        /* whole array, sum(sizes) cells (pinned for overlap) */
    void* host_out;             /* result, sum(sizes) cells */
} hx_pipeline_desc;

/* Host-to-host run of Algorithm 1 with the stencil: an H2D copy of every
 * partition into bufs_a[p], one fused kernel pass per partition into bufs_b[p]
 * (its halos read from the neighbours' bufs_a, so it depends on the copies of
 * p-1, p and p+1), and a D2H copy of every partition into host_out.  Copies
 * run on the copy streams while kernels of other partitions run on the compute
 * streams.  op_events (optional, 3 x parts entries: the H2D copies, the
 * kernels, the D2H copies, each indexed by partition) receives the operations'
 * events; the caller releases them. */
hx_status hx_run_pipeline(hx_ctx ctx, const hx_pipeline_desc* desc, const hx_event* deps,
                          int ndeps, hx_event* out, hx_event* op_events);

/* ------------------------------------------------------------ batched plans */
typedef enum {
    HX_BATCH_PERSISTENT = 0,   /* one persistent launch striding over every tile */
    HX_BATCH_GRAPH = 1,        /* one launch per segment, captured once as a hipGraph */
    HX_BATCH_PLAIN = 2         /* comparator: one launch per segment per step */
} hx_batch_mode;

/* How a PERSISTENT batch evaluates its fused pass of `steps` steps. */
typedef enum {
    HX_FORM_DIRECT = 0,        /* step by step in registers (f32 and f64; any boundary) */
    HX_FORM_PROPAGATOR = 1,    /* one convolution with the steps-step propagator on the matrix
                                  cores (f32 only); the plan fails with HX_ERR_ARG unless every
                                  segment qualifies, see hx_plan_create_batched */
    HX_FORM_AUTO = 2           /* the tuned form, else PROPAGATOR where every segment qualifies,
                                  else DIRECT */
} hx_batch_form;

typedef struct {
    hx_buffer in;  size_t in_offset;      /* n cells, byte offset */
    hx_buffer out; size_t out_offset;     /* n cells; must not overlap in */
    hx_buffer tmp; size_t tmp_offset;     /* n cells; HX_BATCH_PLAIN with steps > 1 only */
    int64_t n;
    double r;
    int bc_lo, bc_hi;                     /* hx_bc of each end */
    hx_buffer halo_lo; size_t halo_lo_offset;   /* as in hx_stencil_args */
    hx_buffer halo_hi; size_t halo_hi_offset;
    int halo_width;
} hx_segment;

typedef struct {
    int dtype;                  /* hx_dtype, shared by all segments */
    int steps;                  /* steps per launch: one fused pass per segment */
    int count;
    const hx_segment* segs;     /* `count` segments (copied at plan creation) */
    int mode;                   /* hx_batch_mode */
    int cells_per_lane;         /* 0 = tuned */
    int waves_per_group;        /* 0 = tuned */
    int grid_waves_per_cu;      /* PERSISTENT: > 0 = a persistent grid of that many waves per
                                   CU striding over the tiles, each wave prefetching its next
                                   tile while it advances the current one; < 0 = one wave per
                                   tile; 0 = tuned (one wave per tile if untuned) */
    int form;                   /* hx_batch_form; 0 = DIRECT */
    int span_blocks;            /* PROPAGATOR: how waves walk the blocks of 1024 cells.  > 0 =
                                   contiguous spans of that many blocks per wave (at most
                                   256, else HX_ERR_ARG); -1 = the
                                   interleaved walk (a persistent grid, wave w taking blocks
                                   w, w + grid, ... of all segments numbered back to back);
                                   -2 = the block walk (one wave per block, the grid covering
                                   every block; at most 65535 segments; waves_per_group 1 or 4
                                   waves on consecutive blocks per workgroup, 0 = tuned, else
                                   1, other counts HX_ERR_ARG); -1 and -2 are
                                   HX_ERR_ARG unless every segment has the same n and r, and
                                   give the same bits;
                                   0 = the tuned walk, else the block walk where allowed,
                                   else spans chosen to fill the device in whole rounds */
} hx_batch_desc;

/* Build a batch: `count` 1D segments, each with its own size, r, boundaries
 * and halos, all advanced `steps` steps by one operation (the batched driver:
 * many uneven partitions or independent problems in one persistent launch or
 * one captured graph).  Buffers are resolved to addresses now: they must
 * outlive the plan.  The work table is built and uploaded once. */
hx_status hx_plan_create_batched(hx_ctx ctx, const hx_batch_desc* desc, hx_plan* plan);

/* The PROPAGATOR form advances each segment by one convolution with the
 * `steps`-step propagator of the 1D stencil (the steps-fold self-convolution of
 * [r, 1-2r, r], see hx_propagator_coefficients), a banded Toeplitz product run
 * on matrix-core tiles and accumulated in f32.  Walked in spans, every f32
 * operand takes an exact three-term bf16 split (six products per pair, each
 * within 2^-20 of itself); walked interleaved or one wave per block
 * (segments of one size and one rate), each 1152-cell window is scaled by a
 * power of two and split into two fp16 terms (three products per pair, each
 * within about 3 * 2^-22 of itself).  All walks prune product levels whose
 * taps are tiny, and the fp16
 * split has absolute floors; so every 1024-cell block checks its outputs
 * against the bound E of those absolute terms: unless every output is finite
 * and at least 2^21 E times the largest finite |x| of the block's window (E
 * is a few 2^-32 of the tap mass at r = 1/4, steps = 50), the block is
 * advanced by f32 stepping instead, in the same launch (by its wave).  Each
 * output is then either within a few 2^-22 of sum_j |p_j u_{i+j}| plus 2^-21
 * of itself, or the stepped f32 result: f32 accuracy cell by cell, also next
 * to cells many orders of magnitude larger, and a non-finite input cell
 * reaches exactly the outputs within `steps` of it, as stepping does.  A
 * segment qualifies when: dtype is HX_F32, the mode PERSISTENT,
 * 1 <= steps <= 64; both ends PERIODIC (then n >= steps) or both GHOST with
 * halo_width >= 4 * ceil(steps / 4); n is a multiple of 4; and in, out, the
 * end of the left halo and the start of the right halo are 16-byte aligned.
 * Results agree with stepping to f32 rounding (not bit for bit; the
 * interleaved and the block walk give the same bits, the span walk others). */

/* Run a batch plan once after `deps`. */
hx_status hx_launch_batched(hx_ctx ctx, hx_plan plan, const hx_event* deps, int ndeps,
                            hx_event* out);

/* The `steps`-step propagator of the 1D heat stencil with diffusion number r:
 * taps[steps + j] = p_j for -steps <= j <= steps (2*steps + 1 values), the
 * steps-fold self-convolution of [r, 1 - 2r, r], computed in FP64.  One step
 * is u'_i = u_i + r (u_{i-1} - 2 u_i + u_{i+1}), so steps steps on a periodic
 * or halo-fed segment are u^(steps)_i = sum_j p_j u_{i+j}.  Needs no device. */
hx_status hx_propagator_coefficients(double r, int steps, double* taps);

/* Free a plan (waits for the context's queued work first). */
hx_status hx_plan_destroy(hx_ctx ctx, hx_plan plan);

/* --------------------------------------------------------------- halo plans */
typedef struct {
    hx_buffer src; size_t src_offset;   /* first byte of the first run */
    hx_buffer dst; size_t dst_offset;
    int64_t rows;                       /* number of runs */
    int64_t row_bytes;                  /* bytes per run, a multiple of 4 */
    int64_t src_pitch, dst_pitch;       /* bytes between consecutive runs (rows > 1) */
} hx_halo_desc;

/* Halo pack/unpack: a table of copies between state buffers and ghost slots,
 * all run by one kernel per launch.  A contiguous halo (D boundary cells of a
 * 1D partition, D boundary rows of a row band) is one run; a column halo is
 * `rows` runs with a pitch.  Spans are range-checked at creation; a
 * descriptor's source and destination must not overlap.  Buffers must outlive
 * the plan. */
hx_status hx_plan_create_halo(hx_ctx ctx, const hx_halo_desc* descs, int n, hx_plan* plan);
hx_status hx_launch_halo(hx_ctx ctx, hx_plan plan, const hx_event* deps, int ndeps,
                         hx_event* out);

/* ------------------------------------------- variable coefficient + adjoint */
/* The gradient path: a 2D variable-coefficient heat step (h = 1, zero-Dirichlet)
 *   v_c = u_c + dt * sum_f kappa_f (u_n - u_c)   over the W, E, N, S faces,
 * kappa_f = (kappa_c + kappa_n)/2 on interior faces, kappa_f = kappa_c with a
 * ghost u_n = 0 on edge faces; and its adjoint for L = 0.5 ||u_T - y||^2:
 *   lam_t = A^T lam_{t+1},  dL/dkappa_c += -dt [ sum_{interior f} (u_n-u_c)(lam_n-lam_c)/2
 *                                                + sum_{edge f} u_c lam_c ]   (u = u_t).
 * The paper has no adjoint; this is the reverse-mode derivation of the explicit
 * scheme.  States are ny x nx row-major arrays of the dtype at offset 0. */

/* out = A(kappa) u (one forward step). */
hx_status hx_heat_vc_step(hx_ctx ctx, int dtype, int64_t nx, int64_t ny, double dt, hx_buffer u,
                          hx_buffer kappa, hx_buffer out_buf, const hx_event* deps, int ndeps,
                          hx_event* out);

/* lam_out = A(kappa)^T lam_next and gacc += this step's conductivity gradient
 * (u_t the forward state of the step). */
hx_status hx_heat_vc_adjoint_step(hx_ctx ctx, int dtype, int64_t nx, int64_t ny, double dt,
                                  hx_buffer u_t, hx_buffer lam_next, hx_buffer kappa,
                                  hx_buffer lam_out, hx_buffer gacc, const hx_event* deps,
                                  int ndeps, hx_event* out);

typedef struct {
    int dtype;
    int64_t nx, ny;
    double dt;
    int steps;                  /* T */
    int ckpt;                   /* segment length S; 0 = ceil(sqrt(T)) (hx_vc_schedule) */
    hx_buffer u0;               /* initial state; also checkpoint 0 */
    hx_buffer kappa;
    hx_buffer uT;               /* forward: final state */
    hx_buffer ckpts;            /* (segments - 1) states: u_{kS}, k = 1 .. segments-1 */
    hx_buffer work;             /* 2 states of ping-pong space (T > 1) */
    hx_buffer seg;              /* backward: S - 1 states for a recomputed segment */
    hx_buffer lamT;             /* backward input: dL/du_T */
    hx_buffer lam0;             /* backward output: dL/du_0 */
    hx_buffer gk64;             /* backward output: dL/dkappa, FP64 (cells x 8 bytes) */
    hx_buffer gacc;             /* backward: one state of the dtype, per-segment accumulator
                                   (scratch: its contents afterwards are unspecified) */
    int rows_per_block;         /* rows per wave; 0 = the library's choice: for the fused
                                   passes, the height whose grid fills the device's resident
                                   wave slots once; for single steps, 64.  Results do not
                                   depend on it. */
} hx_vc_args;

/* Segment length and number of segments of the sqrt(T) checkpoint schedule. */
hx_status hx_vc_schedule(int steps, int ckpt, int* segment_length, int* segments);

/* T forward steps from u0 into uT, keeping the checkpoints u_{kS}. */
hx_status hx_heat_vc_forward(hx_ctx ctx, const hx_vc_args* args, const hx_event* deps, int ndeps,
                             hx_event* out);

/* Reverse sweep from lamT: segment by segment from the last, recompute the
 * segment's states from its checkpoint, run its adjoint steps, fold its
 * conductivity gradient into gk64 in FP64.  Writes lam0 and gk64. */
hx_status hx_heat_vc_backward(hx_ctx ctx, const hx_vc_args* args, const hx_event* deps, int ndeps,
                              hx_event* out);

/* FP64 reductions over n cells (deterministic two-pass; `work` holds at least
 * 4096 doubles): loss out64 = 0.5 sum (u - y)^2 (resid = u - y when resid is
 * not 0), and out64 = sum a*b. */
hx_status hx_launch_loss(hx_ctx ctx, int dtype, int64_t n, hx_buffer u, hx_buffer y,
                         hx_buffer resid, hx_buffer out64, hx_buffer work, const hx_event* deps,
                         int ndeps, hx_event* out);
hx_status hx_launch_dot(hx_ctx ctx, int dtype, int64_t n, hx_buffer a, hx_buffer b,
                        hx_buffer out64, hx_buffer work, const hx_event* deps, int ndeps,
                        hx_event* out);

/* hx_launch_loss without the `work` buffer, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops): it calls no
 * hipMalloc, hipFree or other allocating routine.  The partial sums go to a
 * static device array of 4096 doubles (32 KiB) that every GPU the library
 * runs on holds until the process ends; its device address is looked up once
 * per device when a context is created.  Same kernels, same result bit for
 * bit as hx_launch_loss.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (on different streams, with no event ordering them) race
 * and give wrong losses, so order them through deps.  Nothing needs clearing
 * between calls (each call writes every partial it reads).  HX_ERR_RANGE if a
 * reduction would need more than 4096 partials (never with the library's
 * grid, capped at 4096 workgroups), HX_ERR_HIP if the array's address could
 * not be looked up on this device; otherwise as hx_launch_loss. */
hx_status hx_launch_loss_noalloc(hx_ctx ctx, int dtype, int64_t n, hx_buffer u, hx_buffer y,
                                 hx_buffer resid, hx_buffer out64, const hx_event* deps,
                                 int ndeps, hx_event* out);

/* y = x * s with s an FP64 scalar in device memory (out64 of a reduction, or a
 * gradient), and dst = (dtype) src64. */
hx_status hx_launch_scale(hx_ctx ctx, int dtype, int64_t n, hx_buffer x, hx_buffer s64,
                          hx_buffer y, const hx_event* deps, int ndeps, hx_event* out);
hx_status hx_launch_cast64(hx_ctx ctx, int dtype, int64_t n, hx_buffer src64, hx_buffer dst,
                           const hx_event* deps, int ndeps, hx_event* out);

/* ------------------------------------------------------------------ events */
/* An event that completes when every event in `events` has completed (the
 * paper's when_all, Sec. III-A); it fails with HX_ERR_DEP_FAILED if any of them
 * fails.  n = 0 gives an already-complete event. */
hx_status hx_when_all(hx_ctx ctx, const hx_event* events, int n, hx_event* out);

/* Block until `ev` completes (the paper's wait_all / future::get) or
 * `timeout_ns` elapses (< 0 = no limit).  Returns the event's final status
 * (HX_OK or its error) or HX_ERR_TIMEOUT. */
hx_status hx_wait(hx_ctx ctx, hx_event ev, int64_t timeout_ns);

/* Non-blocking: *state = HX_PENDING, HX_OK or the event's error. */
hx_status hx_event_query(hx_ctx ctx, hx_event ev, hx_status* state);

/* Drop the caller's reference.  Operations that depend on the event are not
 * affected. */
hx_status hx_event_release(hx_ctx ctx, hx_event ev);

/* Milliseconds between two completed events of a context created with
 * timing = 1 (both must be GPU operations). */
hx_status hx_event_elapsed(hx_ctx ctx, hx_event start, hx_event stop, double* ms);

/* Start and end of operation `ev`, in milliseconds after the completion of
 * `ref` (timing contexts only; both complete GPU operations).  The start is
 * taken on the operation's stream once its dependency waits are satisfied, so
 * end - start is the operation's own duration. */
hx_status hx_event_span(hx_ctx ctx, hx_event ev, hx_event ref, double* start_ms, double* end_ms);

/* A host-completed event: operations that depend on it are held back until
 * hx_user_event_set is called; status HX_OK releases them, an error fails them
 * with HX_ERR_DEP_FAILED. */
hx_status hx_user_event_create(hx_ctx ctx, hx_event* out);
hx_status hx_user_event_set(hx_ctx ctx, hx_event ev, hx_status status);

/* Host continuation (the paper's future::then / dataflow, Sec. III-A): `fn`
 * runs on the context's host worker thread once every event in `deps` has
 * completed; its return value (HX_OK or an error) completes the returned event.
 * If a dependency fails, `fn` is not called and the event completes with
 * HX_ERR_DEP_FAILED.  GPU operations may depend on the returned event; they
 * are queued when it completes.  `fn` must not block on events that depend on
 * its own completion. */
typedef hx_status (*hx_host_fn)(void* user);
hx_status hx_host_task(hx_ctx ctx, hx_host_fn fn, void* user, const hx_event* deps, int ndeps,
                       hx_event* out);

/* Interop with foreign streams (e.g. torch's current stream): an event that
 * completes when the work queued on `hip_stream` so far has, and a stream-wait
 * that makes `hip_stream` wait for `ev` on the GPU. */
hx_status hx_event_record_stream(hx_ctx ctx, void* hip_stream, hx_event* out);
hx_status hx_stream_wait_event(hx_ctx ctx, void* hip_stream, hx_event ev);

/* ------------------------------------------------------- captured graphs */
/* Record a future graph once and replay it as one operation.  The futures of
 * Sec. III-A cost host work per operation (dependency resolution, stream
 * waits and markers), which Sec. V-A.1 and V-A.2 measure against the native
 * API; a program that submits the same graph of operations many times pays
 * it once with these calls.
 *
 * hx_graph_begin opens a capture: every GPU operation submitted to the context
 * until hx_graph_end (copies, stencils, batched plans in PERSISTENT or PLAIN
 * mode, programs, when_all) is recorded into one HIP graph instead of
 * running, in submission order on one stream (so the graph replays them one
 * after another, which honours every dependency; operations that would run
 * concurrently on separate streams do not overlap in the graph).  The events those
 * calls return stand for the recorded operations: they order the later
 * operations of the same capture, may be released, and are complete once the
 * capture ends (recorded, not run).  During a capture a dependency must be an
 * operation of the capture or already complete (else HX_ERR_ARG); waiting on
 * a captured operation, hx_ctx_synchronize, the destroy and host-free calls,
 * host tasks and the foreign-stream calls return HX_ERR_ARG; timing spans are
 * not taken.  Not available on a host-only context (HX_ERR_NO_DEVICE) or one
 * created on a caller's stream (HX_ERR_UNSUPPORTED).
 *
 * hx_graph_end closes the capture and returns the instantiated graph as a
 * plan handle (freed by hx_plan_destroy); if the capture failed, every
 * captured event completes with HX_ERR_HIP and so does the call.
 * hx_graph_launch runs the whole graph once after `deps`, as one operation
 * whose event completes when every recorded operation has; the graph keeps
 * the device addresses, sizes and kernel arguments of the capture, so its
 * buffers must still exist (HX_ERR_INVALID otherwise) and hold what the
 * replay should read.  hx_graph_info gives the number of operations recorded.
 */
hx_status hx_graph_begin(hx_ctx ctx);
hx_status hx_graph_end(hx_ctx ctx, hx_plan* graph);
hx_status hx_graph_launch(hx_ctx ctx, hx_plan graph, const hx_event* deps, int ndeps,
                          hx_event* out);
hx_status hx_graph_info(hx_ctx ctx, hx_plan graph, int64_t* operations);

/* ------------------------------------------------------ diagnostics/testing */
/* Sequence number the next submitted operation will get. */
hx_status hx_debug_next_seq(hx_ctx ctx, uint64_t* seq);

/* Make the operation with sequence number `seq` fail validation: it does not
 * run and its event completes with HX_ERR_INJECTED.  The environment variable
 * HX_FAULT_INJECT=<seq> does the same at context creation. */
hx_status hx_debug_inject(hx_ctx ctx, uint64_t seq);

/* Hazard checker (contexts created with check = 1): every operation declares
 * the byte ranges it reads and writes; two accesses to overlapping ranges of a
 * buffer, at least one a write, must be ordered by the dependency graph (or by
 * an hx_wait on the earlier one).  Unordered pairs are counted and described. */
hx_status hx_hazard_count(hx_ctx ctx, int64_t* count);
hx_status hx_hazard_report(hx_ctx ctx, char* buf, size_t len);

/* -------------------------------------------------------------- autotuner */
/* Project-written autotuner: time the candidate geometries (cells per lane,
 * time block, waves per group; rows per wave in 2D) of `args` on its own
 * buffers (out and tmp are overwritten) for about `budget_ms` (at least one
 * candidate runs), store the fastest in the process-wide cache under the
 * problem's key (dims, dtype, size class, steps), and return it in *best.
 * Later launches with geometry fields 0 use the cached entry.  Each candidate
 * runs once to warm up, then three times chained on one stream: in a timing
 * context (hx_ctx_opts.timing) its time is the mean HIP-event span of those
 * launches, otherwise their host time over three. */
hx_status hx_tune_stencil(hx_ctx ctx, const hx_stencil_args* args, int budget_ms,
                          hx_stencil_args* best);

/* The same for a persistent batch (desc->mode PERSISTENT), timed the same way.
 * desc->steps is the whole run's step count T.  The search covers the pass
 * depth D (the divisors of T up to 64, from the deepest down to T/8), and per
 * depth the form (PROPAGATOR for f32, over its walks: the block walk at one
 * and four waves per group, interleaved, the plan's choice, spans of 128 and
 * 40 blocks; DIRECT over cells per lane 8..64,
 * waves per group 1, 2, 4 and a persistent grid of 16 or 64 waves per CU);
 * a candidate costs T / D times its pass.  *best is the fastest, with
 * best->steps = D: the run is T / D passes of that plan (ping-ponging in and
 * out).  It is cached under the key of T and of D. */
hx_status hx_tune_batched(hx_ctx ctx, const hx_batch_desc* desc, int budget_ms,
                          hx_batch_desc* best);

/* Write the process-wide tuned-geometry cache to `path` as JSON; the cache is
 * read back from the file named by HX_TUNE_CACHE on first use. */
hx_status hx_tune_cache_save(const char* path);
/* Forget every tuned geometry (built-in defaults apply again). */
hx_status hx_tune_cache_clear(void);

/* ------------------------------------------------------------------ programs
 * A kernel given as source text and compiled at run time for the context's
 * GPU: the paper's program object (Sec. IV, Listing 2), which compiles CUDA
 * source with NVRTC and runs a kernel with arguments, grid and block on the
 * futures of its inputs.  Here hiprtc compiles HIP C++ for the device's
 * architecture.  A program handle is an hx_plan-kind handle of the context. */
typedef uint64_t hx_program;

/* Copy `source` (NUL-terminated HIP C++; kernels declared
 * extern "C" __global__) under the file name `name` (for diagnostics; null =
 * "program.hip").  Nothing is compiled yet. */
hx_status hx_program_create(hx_ctx ctx, const char* source, const char* name, hx_program* prog);

/* Compile synchronously for the context's device (a host-only context
 * compiles for gfx950 without loading the result), with the library's
 * options (--offload-arch, -O3, packed FP32 instructions disabled) followed
 * by the caller's `nopts` strings (null when nopts = 0).  HX_ERR_ARG when the
 * source does not compile (the compiler's messages are in hx_program_log),
 * HX_ERR_HIP when the code object does not load.  A program builds once. */
hx_status hx_program_build(hx_ctx ctx, hx_program prog, const char* const* options, int nopts);

/* The last build's compiler log, NUL-terminated and truncated to len;
 * *needed (if non-null) receives the full length + 1. */
hx_status hx_program_log(hx_ctx ctx, hx_program prog, char* buf, size_t len, size_t* needed);

typedef enum { HX_ARG_BUFFER = 0, HX_ARG_VALUE = 1 } hx_arg_kind;
enum { HX_ACCESS_READ = 1, HX_ACCESS_WRITE = 2 };

/* One kernel argument.  HX_ARG_BUFFER: the device address of `buffer` +
 * `offset`; `access` (HX_ACCESS_READ | HX_ACCESS_WRITE) declares how the
 * kernel uses the bytes from `offset` to the end of the buffer, which the
 * hazard checker and deferred frees rely on.  HX_ARG_VALUE: `size` bytes
 * (1..16) from `value`, laid out as the kernel parameter's type. */
typedef struct {
    int32_t kind;
    int32_t access;
    hx_buffer buffer;
    uint64_t offset;
    uint32_t size;
    uint32_t reserved;
    uint8_t value[16];
} hx_kernel_arg;

/* Run `kernel` of a built program on grid[0..2] work-groups of
 * block[0..2] work-items with `shared_bytes` of dynamic LDS, after `deps`;
 * `args` are the kernel's parameters in order (not checked against its
 * signature: a mismatch is the caller's error).  Argument errors return
 * synchronously; launch errors complete the event with HX_ERR_HIP. */
hx_status hx_program_run(hx_ctx ctx, hx_program prog, const char* kernel, const hx_kernel_arg* args,
                         int nargs, const uint32_t grid[3], const uint32_t block[3],
                         uint32_t shared_bytes, const hx_event* deps, int ndeps, hx_event* out);

/* The hipFunction_t of a built program's kernel, for callers that launch it
 * on streams of their own; valid until the program is destroyed. */
hx_status hx_program_function(hx_ctx ctx, hx_program prog, const char* kernel, void** function);

/* Wait for the context's streams, unload the code object, free the program. */
hx_status hx_program_destroy(hx_ctx ctx, hx_program prog);

#ifdef __cplusplus
}
#endif

#endif /* HX_H */
