/*
 * set.h -- C ABI of the stream-event-triggered (SET) job-pipeline runtime for
 * AMD Instinct MI355X (gfx950).
 *
 * The method (Li, Huang, Ogras, "SET: Stream-Event-Triggered Scheduling for
 * Efficient CUDA Graph Pipelines"): every job is a host-to-device copy, a
 * chain of short kernels and a device-to-host copy (Section 3.2).  Each job
 * is replayed as a pre-instantiated graph executable bound to one worker's
 * stream and buffers (Section 4.1, "Job-as-Graph and Memory Management";
 * Section 4.2 (1) "Workers").  A submitter thread binds per-job parameters
 * and pushes ready executables into per-worker queues (Algorithm 1); a
 * dispatcher thread pairs free workers with jobs, stealing from other
 * workers' queues when its own is empty and retargeting a stolen job to the
 * thief's buffers (Algorithm 2); a completion callback returns the worker to
 * the free pool (Algorithm 3).
 *
 * Conventions for every call:
 *  - Return value: SET_OK (0) or a negative SET_E* code.  No exception ever
 *    crosses the ABI.  After the first device (HIP) failure a context is
 *    latched into SET_EDEVICE and every later call on it returns SET_EDEVICE;
 *    set_last_error() gives the message.
 *  - Pointers named host_* are host addresses; pointers named dev_* / arena
 *    are device addresses; streams are hipStream_t passed as void*.
 *  - "Borrowed" memory and streams stay owned by the caller (in the Python
 *    binding: allocated by PyTorch) and must outlive the context.
 *  - Job inputs and outputs are caller-owned pinned host buffers.  host_in
 *    must stay valid and unmodified until the job completes; host_out must
 *    not be read before completion (completion callback or set_drain).
 *  - Thread safety: set_submit / set_submit_many may be called from several
 *    threads; set_get_stats may run concurrently with everything else.
 *    set_template_define, set_drain, set_reset_stats and set_ctx_destroy must
 *    not race with each other.
 */
#ifndef SET_H
#define SET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SET_ABI_VERSION 4u

/* ---------------------------------------------------------------- status codes */
enum set_status {
    SET_OK = 0,
    SET_EINVAL = -1,       /* bad argument or configuration */
    SET_ENOMEM = -2,       /* host or device allocation failed, or arena too small */
    SET_EDEVICE = -3,      /* a HIP call failed; sticky for the context */
    SET_EAGAIN = -4,       /* SET_NONBLOCK submit found the staging ring full */
    SET_ETIMEOUT = -5,     /* set_drain timed out */
    SET_ECLOSED = -6,      /* context is shutting down */
    SET_EUNSUPPORTED = -7  /* operation not available in this mode/backend */
};

/* ---------------------------------------------------------------- run modes */
/* The method and the comparison systems of Section 5.1 ("Baseline Models"),
 * all behind the same submit/drain calls. */
enum set_mode {
    /* Event-chained per-job graphs: per-worker queues, free-worker pool,
     * work stealing, completion callbacks (Section 4.2, Algorithms 1-3). */
    SET_MODE_SET = 0,
    /* Synchronous model: each job's copies and kernels launched directly on
     * one stream, then a host synchronisation (Section 5.1, model 1).  Jobs
     * run inside set_submit, round-robin over the configured streams. */
    SET_MODE_SYNC = 1,
    /* Graph model: one pre-instantiated job graph per stream, parameters
     * updated and relaunched per job, host synchronisation per job
     * (Section 5.1, model 2). */
    SET_MODE_GRAPH = 2,
    /* Static batching model: one graph of batch_size parallel job chains on a
     * fixed stream, parameters updated per batch, host synchronisation per
     * batch (Section 2; Section 3.2 "Inter-Batch Overheads"; Section 5.1,
     * model 3). */
    SET_MODE_BATCH_SYNC = 3,
    /* Queue model: one global issue queue under a mutex; an issuer thread
     * repeatedly takes the mutex and queries every worker (O(b) per round),
     * completing finished jobs and launching the next queued job's graph on
     * each idle worker (Section 2; Section 5.1, model 4). */
    SET_MODE_QUEUE = 4
};

enum set_backend {
    SET_BACKEND_HIP = 0,  /* the MI355X path */
    SET_BACKEND_FAKE = 1  /* CPU stand-in (threads as streams) for scheduler tests; computes no pipeline */
};

/* Completion mechanism of SET mode ("AddCallback", Algorithm 2; the
 * asynchronous resource return of Algorithm 3). */
enum set_callback_mode {
    /* hipEventRecord on the worker stream after the job's graph; a library
     * completion thread observes each worker's events in launch order
     * (hipEventQuery reads a host-visible signal) and runs the release.  The
     * device queues hold only event markers.  Default: with 4 hardware queues
     * per process on MI355X, a host-function packet in a queue blocks every
     * stream sharing it, which the two variants below do. */
    SET_CB_EVENT_POLL = 0,
    /* hipEventRecord on the worker stream, hipStreamWaitEvent on a per-worker
     * callback stream, hipLaunchHostFunc there (event chaining). */
    SET_CB_EVENT_CHAIN = 1,
    /* hipLaunchHostFunc directly on the worker stream after the graph. */
    SET_CB_SAME_STREAM = 2,
    /* The job's graph ends with a one-thread kernel node that stores the
     * job's binding sequence number into the slot's word of a pinned host
     * array (system-scope release store, after the device-to-host copy node
     * has finished).  The completion thread watches each worker's oldest
     * word with plain host loads and calls no HIP function, so it never
     * contends with the dispatcher inside the HIP runtime.  SET mode only.
     * Faster than event polling for short jobs with copy kernels; with DMA
     * input copies the extra kernel costs more than it saves, and event
     * polling is the faster. */
    SET_CB_HOST_FLAG = 3,
    /* hipEventRecord on the worker stream after the job's graph, with the
     * slot's events created hipEventBlockingSync; one library thread per
     * worker waits in hipEventSynchronize on that worker's events in launch
     * order and then runs the release.  Nothing spins on the host and no
     * host-function packet enters the device queues: the waiting thread
     * sleeps until the runtime signals the event (Section 4.2, "(3) Free
     * worker pool": the pool is updated on completion, not by polling). */
    SET_CB_EVENT_BLOCKING = 4
};

enum set_submit_policy {
    SET_SUBMIT_ROUND_ROBIN = 0,  /* next queue with room, cyclically (Algorithm 1) */
    SET_SUBMIT_SHORTEST = 1,     /* queue with fewest bound jobs */
    SET_SUBMIT_SKEW0 = 2         /* everything to worker 0 (forces steals; tests) */
};

/* ---------------------------------------------------------------- pipelines */
/* The job families (synthetic stand-ins for the image and small-kernel
 * workloads of Section 5.1).  Layouts are row-major, dense. */
enum set_pipeline {
    /* in: h*w uint8 image.  3x3 box sum with zero padding (uint16) ->
     * floor(sum/9) (uint8) -> 256-bin histogram (uint32).
     * out: set_out_header + uint32[256]; with SET_TF_DEBUG also uint16 sums
     * (h*w) then uint8 quotients (h*w), each at a 64-byte aligned offset. */
    SET_PIPE_BOX_HIST_U8 = 0,
    /* in: h*w float32 image.  Separable 5x5 Gaussian (sigma 1, radius 2, taps
     * normalised then rounded to float32, replicated borders, horizontal then
     * vertical) -> Sobel magnitude sqrt(gx^2+gy^2) (unnormalised 3x3 kernels,
     * replicated borders) -> mask = mag > threshold (uint8) -> count of mask
     * (uint32) and sum of mag over all pixels (float32).
     * out: set_out_header + {uint32 count, float32 sum}; with SET_TF_DEBUG
     * also the uint8 mask (h*w) then the float32 blurred image (h*w). */
    SET_PIPE_GAUSS_SOBEL_F32 = 1,
    /* no H2D: x and y are windows [x_off, x_off+n), [y_off, y_off+n) of the
     * template's device-resident pools.  z = a*x + y -> t = tanh(z) ->
     * S = sum t (float32).  out: set_out_header + float32 S. */
    SET_PIPE_SAXPY_TANH_SUM_F32 = 2,
    /* in: n int32.  Inclusive prefix sum accumulated in int64.
     * out: set_out_header + int64[n] (or the low int32 words with
     * SET_TF_SCAN_LOW32). */
    SET_PIPE_SCAN_I32_I64 = 3,
    /* A batch of vector jobs in one launch graph: H2D of a descriptor table
     * (64-byte header + one 48-byte descriptor per job, each with its own
     * work-item size) -> a persistent
     * kernel whose blocks pull (job, tile) work items from an atomic counter
     * -> a kernel summing each job's tile partials in tile order -> D2H of
     * set_out_header + one float32 S per job, in descriptor order.  Jobs are
     * normally submitted through set_run_vector_jobs, which builds the
     * tables; per-job S depends only on (n, tile size). */
    SET_PIPE_SAXPY_BATCH_F32 = 4,
    /* The inclusive int32 -> int64 scan of SET_PIPE_SCAN_I32_I64 done by a
     * library call (rocPRIM's device scan) instead of this library's kernels:
     * the job graph is built by stream capture of [H2D] -> a kernel writing
     * the job's scalars into the slot -> the library's kernels -> a kernel
     * publishing the output header -> [D2H] (Section 4.1: templates mixing
     * explicit nodes and captured library code, with placeholders only for
     * the job's own parameters).  The captured call has a fixed length, so
     * every job has n = max_n (n = 0 in the job means max_n).  Not available
     * in SET_MODE_BATCH_SYNC, and SET_TF_SCAN_LOW32 does not apply. */
    SET_PIPE_SCAN_LIB_I32_I64 = 5,
    /* Iterative thermal grid (a memory-bound iterative workload like the
     * paper's Hotspot, Section 5.1): in = temperature grid T0 followed by
     * the power grid P (each height x width float32, row-major); max_n = the
     * number of explicit steps K (1..32), each one kernel of the chain:
     *   T' = T + 0.5*P + 0.1*(N + S - 2T) + 0.1*(W + E - 2T) + (300 - T)/640
     * with N, S, W, E the four neighbours and a neighbour outside the grid
     * taken as the cell itself (no heat crosses the border); then a kernel
     * publishing the header.  out: set_out_header + T_K (float32, row-major). */
    SET_PIPE_HOTSPOT_F32 = 6
};

/* How a job's host<->device copies execute. */
enum set_copy_mode {
    SET_COPY_KERNELS = 0, /* small-grid copy kernels, nodes of the job's graph, that pull the input from /
                             push the output to pinned host memory; host buffers must be 16-byte aligned.
                             Default: ROCm runs graph memcpy nodes as large-grid blit kernels that crowd
                             out the stage kernels */
    SET_COPY_NODES = 1,   /* graph memcpy nodes (hipMemcpyAsync in the synchronous model) */
    SET_COPY_ASYNC_IN = 2 /* the input goes by hipMemcpyAsync (the DMA engines) on the worker stream
                             right before the graph launch, or on an input-copy stream (see
                             set_config.input_copy_streams); the graph holds the stages and a
                             device-to-host copy kernel.  For link-bound jobs and long kernel chains: the
                             CUs keep the stages while the DMA engines fill the link (57 GB/s host-to-device;
                             77 GB/s in both directions with the output kernel).  One job in flight per
                             worker suits it best.  Host buffers 16-byte aligned */
};

/* template flags */
#define SET_TF_DEBUG 0x1u       /* also copy intermediate images back (parity tests) */
#define SET_TF_SCAN_LOW32 0x2u  /* scan: copy back only the low 32 bits of each sum */
#define SET_TF_CAPTURE 0x4u     /* build each slot's graph by stream capture of the job's launch sequence
                                   (Section 4.1's capture path) instead of explicit node construction */
#define SET_TF_POISON 0x8u      /* memory-safety stress of Section 4.1's rule that no job writes into a slot
                                   another job still uses: every job's graph ends, after its output copy, with
                                   a kernel that fills the slot's device buffers (header and canaries excepted)
                                   with 0xFF bytes, so a job that read what the slot's previous job left there
                                   would read NaN / all-ones values instead of plausible data */

/* steal policies (set_config.steal_policy) */
#define SET_STEAL_ANY 0
#define SET_STEAL_BUSY 1

/* submit flags */
#define SET_NONBLOCK 0x1  /* return SET_EAGAIN instead of waiting for staging room */

/* ---------------------------------------------------------------- structs */
typedef struct set_config {
    uint32_t abi_version;        /* must equal SET_ABI_VERSION */
    int32_t mode;                /* enum set_mode */
    int32_t backend;             /* enum set_backend */
    int32_t device;              /* HIP device ordinal */
    int32_t num_workers;         /* b: workers, one stream each (Section 4.2 (1)); 1..256 */
    int32_t slots_per_worker;    /* d: buffer slots (one graph exec each) per worker; 1..64 */
    int32_t queue_capacity;      /* capacity of each per-worker queue Q_i; 0 = max(1, d - inflight) */
    int32_t inflight_per_worker; /* launch permits per worker in the free pool; 0 = min(2, d) */
    int32_t work_stealing;       /* 1: FindJob steals from (w+k) mod b (Algorithm 2); 0: local only */
    int32_t batch_size;          /* SET_MODE_BATCH_SYNC: job chains per batch graph, 0 = num_workers;
                                  * at most num_workers * slots_per_worker: chain i runs in slot
                                  * i / num_workers of worker i % num_workers */
    int32_t callback_mode;       /* enum set_callback_mode (SET mode) */
    int32_t submit_policy;       /* enum set_submit_policy */
    int32_t spin_us;             /* dispatcher spin before blocking on its condition variable */
    int32_t staging_capacity;    /* bound of the submit staging ring; 0 = 4096 */
    uint64_t mem_budget_bytes;   /* admission cap on the summed slot footprint of bound jobs; 0 = none */
    void **streams;              /* num_workers borrowed hipStream_t, or NULL: the library creates them */
    uint64_t seed;               /* recorded in stats only */
    /* CPU fake backend knobs (ignored by the HIP backend) */
    int32_t fake_fail_after;     /* >0: the N-th launch fails with SET_EDEVICE (error latching tests) */
    int32_t fake_reorder_callbacks; /* 1: completion callbacks may run out of launch order */
    /* SET mode: dispatcher threads (Algorithm 2 loops); thread t owns the
     * launch permits of workers w with w % dispatch_threads == t and steals
     * from every queue.  0 or 1 = the single dispatcher of the paper; capped
     * at num_workers.  ROCm's graph launch is host-bound (about 16 us per
     * launch) but scales across threads. */
    int32_t dispatch_threads;
    /* SET_COPY_ASYNC_IN templates: the number C of library-owned streams that
     * carry the input copies, worker w's on stream w % C.  In SET mode a
     * job's copy is issued when the submitter binds it to its FREE slot, and
     * the graph waits on the copy's event at launch (a stolen job copies at
     * launch on the thief's stream, after any copy still landing in its new
     * slot); in the other modes the copy is issued at launch and the worker's
     * stream waits on its event.  At most C DMA copies then run at once.
     * 0 = each input copy on its worker's own stream, right before the graph.
     * 0..64, capped at num_workers. */
    int32_t input_copy_streams;
    /* SET_CB_EVENT_CHAIN (Algorithm 3): the number K of callback streams;
     * worker w's event waits and host functions go on stream w % K.  0 = 1.
     * 1..64, capped at num_workers.  A host function holds its hardware queue
     * until the host has run it, and ROCm maps every stream of a process onto
     * 4 hardware queues: with one callback stream a single queue carries those
     * packets, with one per worker every queue does and the worker streams
     * stall behind them (1024x1024 images, 8 workers: 13.2k against 10.3-11.0k
     * jobs/s). */
    int32_t callback_streams;
    /* SET mode with work stealing: which victims FindJob (Algorithm 2) may
     * take from, probing (w+1) ... (w+b-1) mod b after its own queue.
     * SET_STEAL_ANY (0): the first non-empty queue, as printed.
     * SET_STEAL_BUSY (1): the first non-empty queue whose worker holds no
     * free launch permit; a victim with one is about to launch that job
     * itself, and taking it costs a retarget.  With one dispatcher thread per
     * worker, the printed rule lets every dispatcher whose queue is
     * momentarily empty take its neighbour's next job, which empties the
     * neighbour's queue in turn: per-job vector jobs at 8 workers and 8
     * dispatchers ran 50-60k jobs/s with 17k steals in 20k jobs, against
     * 142-146k with stealing off. */
    int32_t steal_policy;
} set_config;

typedef struct set_job_template {
    int32_t pipeline;            /* enum set_pipeline */
    uint32_t flags;              /* SET_TF_* */
    uint32_t width, height;      /* image and thermal-grid pipelines: size; 1 <= width <= 2^20,
                                    1 <= height <= 2^19, width * height <= 2^28 (the height bound
                                    keeps every launch grid within 65,536 blocks in its second
                                    dimension); SET_EINVAL otherwise */
    uint64_t max_n;              /* vector / scan pipelines: largest n any job may use (>= 1) */
    float threshold;             /* Gaussian/Sobel mask threshold; 0 means 1.0 */
    uint32_t copy_mode;          /* enum set_copy_mode */
    void *arena;                 /* borrowed device buffer for all slots of this template, or NULL: library allocates */
    uint64_t arena_bytes;        /* size of `arena`; must be >= set_template_footprint's total */
    const float *dev_x_pool;     /* SAXPY: borrowed device pool of x values */
    const float *dev_y_pool;     /* SAXPY: borrowed device pool of y values */
    uint64_t pool_len;           /* SAXPY: elements in each pool */
    int32_t block;               /* SET_PIPE_SAXPY_BATCH_F32: threads per block of the persistent work-item
                                  * kernel, 128 / 256 / 512 / 1024 (0 = 256).  It fixes the order in which a
                                  * work item's elements are summed, so it is a property of the template: a
                                  * job's S depends on (n, its item size, this block).  Other pipelines: 0 */
    int32_t grid;                /* tuning: grid cap for streaming kernels (0 = default) */
    uint32_t batch_max;          /* SAXPY batch: most jobs per batch (descriptor table capacity) */
    uint32_t tiles_max;          /* SAXPY batch: most (job, tile) work items per batch */
    uint32_t stress_delay_us;    /* memory-safety stress: > 0 puts a one-wave kernel that waits about this many
                                  * microseconds (device clock) before the first stage of every job, widening
                                  * the window in which a slot released before its job ended would be
                                  * overwritten by the next job's input copy; 0..100000, 0 = none */
    uint32_t reserved;           /* must be 0 */
} set_job_template;

typedef struct set_job_args {
    const void *host_in;         /* pinned host input (NULL for pipelines without H2D) */
    uint64_t in_bytes;           /* must equal the pipeline's input size for this job */
    void *host_out;              /* pinned host output: set_out_header + payload */
    uint64_t out_bytes;          /* >= the pipeline's output size for this job */
    uint64_t n;                  /* vector / scan length (0 = template max_n for scan) */
    float a;                     /* SAXPY scale */
    int32_t worker_hint;         /* -1: submitter policy; else preferred worker */
    uint64_t x_off, y_off;       /* SAXPY: element offsets into the x / y pools */
    uint64_t user_tag;           /* copied into the output header */
    uint32_t grid;               /* SAXPY batch: persistent grid (blocks); 0 = template default */
    uint32_t reserved;
} set_job_args;

/* One vector job for set_run_vector_jobs (z = a*x + y over pool windows). */
typedef struct set_vec_job {
    uint64_t x_off, y_off;       /* element offsets into the template's x / y pools */
    uint64_t n;                  /* 1 <= n <= template max_n */
    float a;
    uint32_t reserved;
} set_vec_job;

/* Per size bucket b = floor(log2 n): elements per (job, tile) work item and
 * the persistent grid.  Zero entries take the defaults. */
typedef struct set_vec_tuning {
    uint32_t tile_elems[64];     /* multiple of 1024 */
    uint32_t grid[64];
} set_vec_tuning;

/* Written by the device at the start of every job output (64 bytes). */
#define SET_OUT_MAGIC 0x5E7D0A11u
typedef struct set_out_header {
    uint64_t job_id;     /* id assigned by set_submit (consecutive from 0 per context) */
    uint64_t seq;        /* per-slot binding sequence number */
    uint32_t worker;     /* worker (stream) that ran the job */
    uint32_t slot;       /* buffer slot the job ran in */
    uint32_t magic;      /* SET_OUT_MAGIC once the job's last stage ran */
    uint32_t canary_ok;  /* 1 if the slot's head and tail canaries were intact */
    uint64_t user_tag;   /* set_job_args.user_tag */
    uint64_t reserved[3];
} set_out_header;

typedef struct set_stats {
    uint64_t submitted, completed, stolen, failed;
    uint64_t launches_per_worker[64];  /* workers 0..63 (a context may have up to 256) */
    uint64_t host_ns_bind;       /* submitter (or caller) time spent binding parameters */
    uint64_t host_ns_launch;     /* dispatcher time in graph launch + callback registration */
    uint64_t host_ns_callback;   /* time spent inside completion callbacks */
    uint64_t host_ns_sync;       /* baseline modes: time blocked in host synchronisation */
    uint32_t queue_high_water;   /* most jobs ever queued in one Q_i */
    uint32_t inflight_high_water;/* most jobs ever launched and not yet completed */
    uint64_t bytes_h2d, bytes_d2h;
    uint64_t mem_in_use, mem_high_water;  /* admission accounting (bytes of bound slots) */
    uint64_t batches;            /* batch-sync mode: batch graphs launched */
    uint64_t t_first_submit_ns, t_last_done_ns;  /* steady-clock stamps */
} set_stats;

/* Per-job timestamps (steady clock, ns) for latency percentiles. */
typedef struct set_job_times {
    uint64_t job_id;
    uint64_t t_submit, t_launch, t_done;
    int32_t worker, slot, stolen, status;
} set_job_times;

typedef void (*set_completion_fn)(uint64_t job_id, int status, void *user);

typedef struct set_ctx set_ctx;

/* ---------------------------------------------------------------- calls */

/* Create a context: b workers with their streams (borrowed or created),
 * per-worker queues and callback streams, the free pool, and (SET mode) the
 * submitter thread, the dispatcher thread(s) and the completion thread
 * ("Initialization", Section 4.2).
 * cfg is copied.  *out receives the handle.  Errors: SET_EINVAL (bad sizes,
 * abi_version mismatch), SET_ENOMEM, SET_EDEVICE (no device / HIP failure). */
int set_ctx_create(const set_config *cfg, set_ctx **out);

/* The inverse of the initialisation in Section 4.2 ("Initialization": the
 * main thread sets up the queues and the workers' streams, buffers and graph
 * executables, then starts the submitter and dispatcher threads): drain
 * outstanding jobs (c_done reaches the submitted count, Algorithm 3), stop
 * the threads, destroy graphs, events and library-created streams and
 * allocations.  Never frees borrowed memory or streams.  NULL is accepted
 * (no-op).  Always returns SET_OK and frees the handle; a context latched
 * into SET_EDEVICE is not drained first (its device work is waited for by a
 * device synchronisation instead). */
int set_ctx_destroy(set_ctx *c);

/* Bytes of device memory one buffer slot of template t needs, and the total
 * for num_workers * slots_per_worker slots of cfg (what a borrowed arena must
 * hold).  Pure host computation; either output may be NULL. */
int set_template_footprint(const set_config *cfg, const set_job_template *t,
                           uint64_t *slot_bytes, uint64_t *total_bytes);

/* Define a job template: lay out one buffer slot per (worker, slot) in the
 * arena and build + instantiate + upload one graph per slot whose nodes hold
 * placeholders for per-job arguments (Section 4.1).  In batch-sync mode the
 * batch graph is built instead.  *template_id receives the id (0, 1, ...).
 * Must be called before any submit of that template. */
int set_template_define(set_ctx *c, const set_job_template *t, int *template_id);

/* Submit one job.  Returns once the job is accepted: in SET mode it is in
 * the staging ring (the submitter thread binds and queues it, Algorithm 1);
 * in SYNC / GRAPH mode it has already run; in BATCH_SYNC mode it has joined
 * the current batch (the batch runs when full or at set_drain).  *job_id
 * (may be NULL) receives the consecutive id.  SET_EAGAIN with SET_NONBLOCK
 * when the staging ring is full. */
int set_submit(set_ctx *c, int template_id, const set_job_args *a, int flags, uint64_t *job_id);

/* Submit count jobs of one template in order (same semantics as count calls
 * of set_submit; stops at the first error, which is returned). */
int set_submit_many(set_ctx *c, int template_id, const set_job_args *a, uint64_t count,
                    int flags, uint64_t *first_job_id);

/* Register a function called once per completed job, from the release step
 * of Algorithm 3 (Section 4.2, "Asynchronous Resource Return": the callback
 * that runs on a separate thread once the worker's stream has finished the
 * job's graph), after the job's output is in host memory and after c_done
 * was incremented for it.  It runs on a library or driver thread, must not
 * call back into this library or into HIP, and should return quickly: the
 * worker goes back to the free pool only after it returns.  status is SET_OK
 * or the job's error code.  fn == NULL unregisters; user is passed through
 * unchanged and stays owned by the caller. */
int set_set_completion_cb(set_ctx *c, set_completion_fn fn, void *user);

/* Block until every submitted job has completed (c_done == submitted,
 * Algorithm 3's counter).  timeout_ns < 0 waits forever.  SET_ETIMEOUT on
 * timeout (jobs keep running). */
int set_drain(set_ctx *c, int64_t timeout_ns);

/* Snapshot of the counters (may run concurrently with jobs): submitted and
 * completed jobs (Algorithm 1's c_next and Algorithm 3's c_done since the
 * last reset), steals (Algorithm 2), the host time spent binding parameters
 * (UpdateGraphParams of Algorithm 1), launching and in callbacks, and the
 * first-submit / last-completion stamps from which the throughput of
 * Section 5.2 (jobs per second) is taken.  out is caller-owned.  SET_EINVAL
 * if c or out is NULL. */
int set_get_stats(set_ctx *c, set_stats *out);

/* Zero the counters of set_get_stats and the per-job time records, so that
 * a measurement window (the throughput of Section 5.2, the overhead fraction
 * t_schedule / T_measured of Section 5.3 with Eq. 4) starts clean.  Call it
 * when drained; job ids keep counting. */
int set_reset_stats(set_ctx *c);

/* Copy up to max records of per-job times for jobs completed since the last
 * reset, in completion order; *count receives how many were written. */
int set_get_job_times(set_ctx *c, set_job_times *out, uint64_t max, uint64_t *count);

/* Measurement helper for the per-kernel terms of Section 3.2 (Eq. 1-2's
 * kernel times) and the rooflines: launch stage `stage` (0-based kernel of
 * the template's chain) of template `template_id` `reps` times back to back,
 * bracketed by two HIP events on the stream they run on; *avg_us receives the
 * mean duration per launch.  worker >= 0: every launch on worker `worker`'s
 * stream against slot 0 of that worker (its working set stays in the caches
 * when it is small).  worker == -1: launch r uses slot r mod (b*d) of the
 * template, all on worker 0's stream, so with enough slots the kernel reads
 * and writes HBM.  The slots' current contents are used as input, so run
 * jobs on them first.  stage == SET_STAGE_INPUT_COPY / SET_STAGE_OUTPUT_COPY
 * times the template's host-to-device / device-to-host copy of its largest
 * job (Eq. 1's t_in and t_out) the way a job performs it (copy kernel or DMA)
 * against a library-owned pinned buffer; 0 us for a pipeline without that
 * copy.  Requires a drained context. */
#define SET_STAGE_INPUT_COPY (-1)
#define SET_STAGE_OUTPUT_COPY (-2)
int set_time_stage(set_ctx *c, int template_id, int stage, int worker, int reps, double *avg_us);

/* Measurement helper: the bandwidth reference the stage kernels are held to.
 * A plain device copy kernel (one 16-byte word per thread, every word in
 * flight at once) moving `bytes` in all (half read, half written) is launched
 * `reps` times back to back on a library-owned stream between two HIP events;
 * launch r copies slice r' of two buffers of about 512 MiB each (r' strides
 * through the slices), so it reads and writes HBM.  *avg_us receives the mean
 * duration per launch.  The buffers are allocated for the call and freed
 * after it.  bytes: 32 .. 2^30; reps >= 1.  SET_EUNSUPPORTED on the fake
 * backend. */
int set_time_device_copy(set_ctx *c, uint64_t bytes, int reps, double *avg_us);

/* Bucketed persistent batching of vector jobs (template of pipeline
 * SET_PIPE_SAXPY_BATCH_F32): jobs are grouped by size bucket floor(log2 n),
 * each bucket in input order into batches of at most batch_max jobs and
 * tiles_max work items; every batch is one job of the context (in SET mode
 * it is queued, dispatched, stolen and released like any other job).
 * results[i] receives S of jobs[i].  Blocks until every batch has completed.
 * tuning may be NULL.  Descriptor tables and result staging are pinned host
 * memory owned by the context, kept between calls and grown only when a call
 * needs more (so repeated calls allocate nothing); concurrent calls on one
 * context are serialised.  *batches (may be NULL) receives the number of
 * batches submitted. */
int set_run_vector_jobs(set_ctx *c, int template_id, const set_vec_job *jobs, uint64_t count,
                        float *results, const set_vec_tuning *tuning, uint64_t *batches);

/* ---------------------------------------------------------------- no allocation */
#define SET_NOALLOC_MAX_JOBS 16384u       /* jobs per call */
#define SET_NOALLOC_MAX_ITEMS 1048576u    /* work items per call, counted for the worst case (below) */

/* set_run_vector_jobs for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * needs no context and calls no allocating function (no hipMalloc, hipFree or
 * pinned allocation).
 *
 * Per job: S = sum over i < n of tanh(a*x[x_off+i] + y[y_off+i]), with the
 * job's work-item size taken per size bucket floor(log2 n) from tuning (zero
 * entries and tuning == NULL: the default sizes of set_run_vector_jobs).  A
 * job's S is bit-identical to what set_run_vector_jobs returns for the same
 * (n, item size); the persistent grid (`grid`, 0 = 1024 blocks) changes no
 * result.
 *
 * device: HIP device ordinal; made current for the call, then restored.
 * stream: hipStream_t of that device (NULL = its null stream).  The call only
 *   enqueues three kernels there and returns; results are ready when the
 *   stream's work before the next synchronisation point has finished.
 * dev_x_pool, dev_y_pool: device float pools of pool_len elements each.
 * dev_jobs: device array of count set_vec_job; dev_results: device float
 *   array of count results, in job order.  Both caller-owned.
 * max_n: the largest n any job may have (1..2^31).  A job with n outside
 *   [1, max_n] or a window leaving a pool reads nothing and gets NaN.
 * tuning: host struct, read during the call (item sizes: multiples of 1024).
 *
 * Limits, checked on the host before anything is enqueued (SET_EINVAL, with
 * set_last_error(NULL) naming the limit): count <= SET_NOALLOC_MAX_JOBS, and
 * count times the most items a job of length <= max_n can need under the
 * item sizes <= SET_NOALLOC_MAX_ITEMS.  With the default sizes and max_n =
 * 4194304 a job needs at most 64 items, so 16384 jobs fit.
 *
 * Work area: one static device array of about 4.8 MiB per GPU (descriptor
 * table, item partials, work counter), held from library load until the
 * process ends and shared by every call on that GPU.  Each call rewrites it
 * from its first kernel on (the counter included), so calls on one stream
 * follow each other safely; calls that overlap on one GPU (different
 * streams, or different host threads without ordering) race on it and give
 * wrong results.  Errors: SET_EINVAL as above or for null pointers,
 * SET_EDEVICE when a HIP call fails (message in set_last_error(NULL)). */
int set_run_vector_jobs_noalloc(int device, void *stream, const float *dev_x_pool, const float *dev_y_pool,
                                uint64_t pool_len, uint64_t max_n, const set_vec_job *dev_jobs, uint64_t count,
                                float *dev_results, const set_vec_tuning *tuning, uint32_t grid);

/* ---------------------------------------------------------------- serving */
/* One request of an open-loop arrival schedule. */
typedef struct set_request {
    uint64_t t_arrival_ns;       /* arrival, ns after the start of the run; non-decreasing */
    int32_t template_id;         /* a per-job template, or a vector batch template */
    uint32_t reserved;
    set_job_args args;           /* per-job template: as for set_submit.  Vector batch template:
                                    n, a, x_off, y_off of one vector job; host buffers unused */
} set_request;

typedef struct set_serve_config {
    uint32_t vec_inflight;       /* vector batches in flight at once (0 = num_workers) */
    uint32_t vec_batch_max;      /* most vector requests per batch (0 = the template's batch_max) */
    uint64_t window_ns;          /* requests arriving later are not admitted (0 = admit all) */
    const set_vec_tuning *tuning;/* work-item size per size bucket (NULL = defaults) */
} set_serve_config;

typedef struct set_serve_stats {
    uint64_t arrived, completed, failed, not_admitted;
    uint64_t vec_batches;
    uint64_t t_start_ns, t_end_ns;  /* steady clock: first arrival slot, last completion */
    uint64_t max_backlog;        /* most arrived requests waiting for admission at once */
} set_serve_stats;

/* Serve an open-loop request schedule (SET mode only).  The calling thread
 * releases each request at its arrival time; per-job requests enter the
 * scheduler at once and are admitted as worker slots and the device-memory
 * budget (set_config.mem_budget_bytes) allow; vector requests are batched
 * continuously: whenever a vector-batch slot is free, every vector request
 * that has arrived (up to vec_batch_max) forms the next batch, mixing size
 * buckets (each job keeps its bucket's work-item size, so its result equals
 * its result alone).  Requests of different kinds overlap on the device.
 * done_ns[i] receives the completion time of request i in ns after the start
 * of the run (the arrival time is reqs[i].t_arrival_ns; 0 = not completed);
 * vec_results[i] receives S of vector request i (may be NULL if there are
 * none).  Blocks until every admitted request completed.  The per-job
 * requests' host buffers follow set_submit's rules. */
int set_serve(set_ctx *c, const set_request *reqs, uint64_t count, const set_serve_config *cfg,
              uint64_t *done_ns, float *vec_results, set_serve_stats *stats);

/* Bytes a job of length n (the vector, scan and batch pipelines; ignored by
 * the image pipelines; 0 = the template's max_n where that applies) copies in
 * (set_job_args.in_bytes must equal *in_bytes) and out (set_job_args.out_bytes
 * must be at least *out_bytes).  Either output may be NULL. */
int set_job_io_bytes(set_ctx *c, int template_id, uint64_t n, uint64_t *in_bytes, uint64_t *out_bytes);

/* Number of kernels in the template's chain and the algorithmic HBM bytes one
 * launch of each moves (reads + writes of its operands, counted once). */
int set_stage_info(set_ctx *c, int template_id, int *num_stages, uint64_t *bytes_per_stage,
                   int max_stages, char *names, int names_len);

/* Message of the last error on this context ("" if none); c == NULL gives the
 * last error on this thread of a call without a context (a failed
 * set_ctx_create, set_run_vector_jobs_noalloc).  The paper defines no error
 * channel; this one serves the latch described at the top of this file.  The
 * string is owned by the library and stays valid until the next failing call
 * on the same context (or thread, for c == NULL). */
const char *set_last_error(const set_ctx *c);

/* Static name of a status code. */
const char *set_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* SET_H */
