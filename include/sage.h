/*
 * sage.h -- C ABI of the function-setup library for one AMD MI355X (gfx950).
 *
 * The library runs many invocations of the same GPU functions with fast setup
 * and shared read-only memory, after "Towards Fast Setup and High Throughput
 * of GPU Serverless Computing" (arXiv 2404.14691):
 *
 *  - parallelized function setup (section "Parallelized Function Setup"):
 *    a function's read-only data is known from its request before it runs,
 *    so it is moved to the GPU while the function's code is loaded;
 *  - sharing-based memory management (section "Sharing-based Memory
 *    Management"): read-only data is loaded once and used by every
 *    invocation.  Here sharing works on 64 KiB blocks: each block is
 *    fingerprinted on the GPU and identical blocks, also across functions,
 *    occupy one slot of a refcounted pool.
 *
 * Conventions
 *  - Every call returns sage_status; no C++ exception crosses this boundary.
 *    sage_last_error() returns a message for the calling thread's last
 *    failure (valid until that thread's next call).
 *  - Pointers are plain host or device addresses.  "Device" means memory of
 *    the context's GPU (hipMalloc, or a torch tensor on it).  Every
 *    device address passed in must be 16-byte aligned.
 *  - Handles (sage_fn, sage_inv) are never reused; a released or
 *    unregistered handle gives SAGE_ESTATE / SAGE_ENOTFOUND.
 *  - One sage_ctx per GPU.  Its calls are serialised by an internal mutex
 *    and may come from any thread.
 *
 * Environment variables read by sage_open (tests and measurements; none is
 * needed in normal use):
 *    SAGE_TILE=<shape>[+<shape>]  fixed BF16 GEMM tile shape (and thin tail
 *                                 shape) instead of the planner's choice
 *    SAGE_DEV_CHUNK_BYTES=<n>     registration chunk of device-resident
 *                                 sources (default 1 GiB; a multiple of 64 KiB)
 *    SAGE_F32_COLS=4|8            output columns per workgroup of the FP32
 *                                 MLP layer (default 4; same bits either way)
 *    SAGE_STENCIL_FUSE=0|1        Jacobi sweeps in passes of two (default 1;
 *                                 same bits either way)
 *    SAGE_FAULT_ALLOC_AFTER=<n>   after n device allocations of the pool
 *                                 arena and workspace cache, every later one
 *                                 fails as if the device were full (ENOMEM paths)
 *    SAGE_TEST_FP_CONST=<v>       every fingerprint reads as v (forces
 *                                 collisions: the byte VERIFY decides)
 */
#ifndef SAGE_H
#define SAGE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden visibility; only this interface is exported. */
#if defined(__GNUC__)
#pragma GCC visibility push(default)
#endif

typedef struct sage_ctx sage_ctx;
typedef uint64_t sage_fn;
typedef uint64_t sage_inv;

typedef enum {
  SAGE_OK = 0,
  SAGE_EINVAL = 1,    /* bad argument, size or layout */
  SAGE_ENOMEM = 2,    /* admission failed: not enough pool or device memory */
  SAGE_EBUSY = 3,     /* object still in use (e.g. unregister with live setups) */
  SAGE_ENOTFOUND = 4, /* unknown handle */
  SAGE_ESTATE = 5,    /* handle in the wrong state (released twice, ...) */
  SAGE_EHIP = 6,      /* a HIP runtime call failed */
  SAGE_EIO = 7        /* code object missing or unreadable */
} sage_status;

/* Data access type a developer declares for each datum (section "Read-only
 * Memory Sharing": Data.Type is ReadOnly or Writable).  Only read-only blobs
 * are registered; writable data is passed to each invocation. */
typedef enum { SAGE_RO = 0, SAGE_RW = 1 } sage_access;

/* Where a blob's bytes live. */
typedef enum { SAGE_SRC_HOST = 0, SAGE_SRC_DEVICE = 1 } sage_where;

/* One datum of a request (section "Parallelizing data and context": the
 * Request lists the data to load, each with a key naming its source).
 * src/nbytes name the bytes; they must stay valid and unchanged until
 * fn_unregister, because evicted blocks are reloaded from them.  Host
 * sources may be pageable or from sage_host_alloc (then copied by DMA
 * without staging). */
typedef struct {
  const void* src;
  size_t nbytes;
  uint32_t access; /* sage_access; must be SAGE_RO for fn_register */
  uint32_t where;  /* sage_where */
  uint64_t key;    /* caller's name for the datum, kept for diagnostics */
} sage_blob;

/* Function bodies the library can run. */
typedef enum {
  SAGE_MLP_F32 = 1,     /* ReLU MLP, FP32 weights/activations */
  SAGE_MLP_BF16 = 2,    /* ReLU MLP, BF16 weights/activations, FP32 accumulate, FP32 output */
  SAGE_STENCIL7_F32 = 3, /* 7-point Jacobi relaxation with a read-only coefficient grid */
  SAGE_RELAX7_F32 = 4    /* the same sweep with one constant coefficient: no read-only data */
} sage_kind;

/* MLP: one RO blob, weights [layers][width][width] ([out][in]) row-major,
 * width a power of two >= 128 whose row (width * element size) fits in
 * 64 KiB, so every weight row lies inside one block.
 *   H_0 = X, H_l = relu(H_{l-1} W_l^T) for l < layers, Y = H_{layers-1} W_L^T.
 *   Input X [batch][width] (FP32 or BF16 bits), output Y [batch][width] FP32.
 * STENCIL7: one RO blob, c[nz][ny][nx] FP32, nx a power of two with
 *   nx*4 <= 65536, all extents >= 3.  Input u0 [batch][nz][ny][nx] FP32,
 *   output u after `sweeps` Jacobi sweeps:
 *   u'_p = u_p + c_p * (avg of 6 face neighbours - u_p) on interior cells,
 *   boundary cells unchanged.
 * RELAX7: no read-only blob (n_blobs = 0); all of its data is the writable
 *   field of each invocation, like the paper's lbm (Table 2: no read-only
 *   bytes, 330 MB writable).  The STENCIL7 sweep with c_p = coef, nx a
 *   multiple of 4, all extents >= 3. */
typedef struct {
  uint32_t kind; /* sage_kind */
  uint32_t layers, width;
  uint32_t nx, ny, nz, sweeps;
  float coef;    /* RELAX7 only */
} sage_fn_desc;

typedef struct {
  size_t ring_slots;         /* pinned staging slots for host->device (default 8; 1 = no pipelining) */
  size_t chunk_bytes;        /* bytes per staging slot, multiple of 64 KiB (default 8 MiB) */
  uint32_t streams;          /* copy/fingerprint streams (default 4) */
  uint32_t fill_threads;     /* host threads copying pageable sources into staging, and host inputs /
                                outputs of MLP launches over 1 MiB through theirs (default 4) */
  uint32_t inflight_groups;  /* grouped launches that may run concurrently (default 4) */
  uint32_t share;            /* 1 (default): shared block pool; 0: private copy per invocation */
  uint32_t batch;            /* 1 (default): grouped launches replayed from hipGraphs; 0: eager */
  uint32_t serial_setup;     /* 1: load code and move data one after the other (A/B switch) */
  size_t pool_budget_bytes;  /* pool capacity; 0 = half of free device memory at open */
  const char* tune_cache;    /* autotuner cache file, or NULL for in-memory only */
  /* Multi-stage exit (section "Multi-stage Resource Exit"), interval T in ms
   * (0 = off: unreferenced blocks stay in HBM until evicted, code objects stay
   * loaded).  A block unreferenced for T moves to a pinned host cache; a code
   * object none of whose functions was set up or released for 2 T is
   * unloaded; a host copy unreferenced for 3 T is dropped (the function's
   * source remains).  Later setups reload from where the bytes are. */
  double exit_stage_ms;
  size_t host_cache_bytes;   /* host-cache budget for demoted blocks; 0 = no limit */
  /* 1: per-kernel readiness for the MLP kinds (the kernel executor's check of
   * section "Taxon Shim", made per layer).  A setup whose reload crosses the
   * host link (host cache or host source) returns once the copies are
   * issued; layer l of the body then waits only for the copies holding
   * layer l's weights, so early layers compute while later ones are still
   * arriving.  0 (default), and reloads from device sources: fn_setup
   * returns with every block resident. */
  uint32_t progressive;
} sage_config;

typedef struct {
  uint64_t logical_bytes;   /* sum of registered RO blob sizes */
  uint64_t unique_bytes;    /* sum of lengths of all live classes */
  uint64_t shared_bytes;    /* bytes of blocks in classes with >= 2 member blocks */
  uint64_t private_bytes;   /* bytes of blocks in singleton classes */
  uint64_t resident_bytes;  /* sum of lengths of resident classes */
  uint64_t resident_slots;
  uint64_t budget_slots;
  uint64_t classes;         /* live classes */
  uint64_t h2d_bytes;       /* RO bytes moved from sources into the device (pool or private copies) */
  uint64_t refcount_sum;    /* sum of class references */
  uint64_t live_setups;
  uint64_t evictions;
  uint64_t reloads;         /* classes reloaded by fn_setup */
  uint64_t registrations;
  uint64_t invocations;
  uint64_t verify_mismatches; /* fingerprint hits whose bytes differed */
  uint64_t workspace_bytes; /* device bytes held for invocation workspaces */
  /* host wall time (ms) spent in the setup path since open, by stage */
  double t_register_ms;     /* whole fn_register calls */
  double t_code_ms;         /* code branch: module load + block-table allocation */
  double t_fp_wait_ms;      /* data branch: waiting for staged bytes + fingerprints */
  double t_dedup_ms;        /* data branch: host index lookups and commit */
  double t_verify_ms;       /* data branch: COPY/VERIFY launches and their results */
  double t_setup_ms;        /* fn_setup calls (admission, reloads, references) */
  double t_invoke_ms;       /* fn_invoke / fn_invoke_batch calls */
  /* multi-stage exit */
  uint64_t host_cached_bytes; /* pinned host bytes holding demoted blocks */
  uint64_t demotions;       /* classes moved from HBM to the host cache */
  uint64_t host_reloads;    /* classes reloaded from the host cache */
  uint64_t module_loads;    /* code objects loaded (first load included) */
  uint64_t module_unloads;  /* code objects unloaded by the multi-stage exit */
  double t_module_ms;       /* host wall time in code-object loads */
  double t_reload_ms;       /* host wall time in fn_setup reloads of missing blocks (issue only, when progressive) */
  double t_release_ms;      /* fn_release / fn_release_batch calls */
  double t_unregister_ms;   /* fn_unregister calls */
} sage_stats;

/* ----------------------------------------------------------------- context */
/* Defaults of every sage_config field (no passage in the paper: the ring,
 * stream and pool parameters are this library's own). */
void sage_config_default(sage_config* cfg);

/* Open the library on `device` (HIP ordinal).  Loads the runtime kernels and
 * allocates the staging ring; roughly SageInit() of the paper's programming
 * model (section "Programming Model").  cfg may be NULL for defaults. */
sage_status sage_open(int device, const sage_config* cfg, sage_ctx** out);
/* Wait for all work, free every resource.  Live handles become invalid.
 * The end of the per-GPU memory daemon's life (section "SAGE Architecture":
 * one daemon per GPU holds the shared data); the paper defines no call for
 * it, so this is the library's own. */
sage_status sage_close(sage_ctx* ctx);
/* Message of the calling thread's last failure (the library's own error
 * reporting; no passage in the paper). */
const char* sage_last_error(void);

/* Pinned host memory (hipHostMalloc) owned by the context; sources here are
 * copied to the device by DMA without staging. NULL on failure.  The paper
 * stages its CPU data in host memory ahead of the GPU copy (section
 * "Parallelizing data and context"); pinned sources are this library's way
 * to let that copy skip the staging ring.  Freed with sage_host_free or at
 * sage_close. */
void* sage_host_alloc(sage_ctx* ctx, size_t nbytes);
void sage_host_free(sage_ctx* ctx, void* p);

/* --------------------------------------------------------------- functions */
/* Register a function and its read-only data (sections "Parallelizing data
 * and context" and "Read-only Memory Sharing").  The code object of the
 * kind is loaded on one thread while the data moves on another: chunks of
 * `chunk_bytes` go through the pinned ring to the device on several streams,
 * each 64 KiB block is fingerprinted there, and blocks whose bytes are
 * already in the pool join that slot (verified byte for byte); the others are
 * copied into new slots.  With share=0 only the function record is made and
 * the data is copied privately at each fn_setup.
 * Returns when every block is classified (joined or new); copies of new
 * blocks may still be in flight on the library's control stream, ordered
 * before every later pool access and before any body of the function.
 * Blobs must be SAGE_RO and match the kind's layout (see sage_fn_desc);
 * sources stay borrowed until fn_unregister.  Errors: EINVAL (layout),
 * ENOMEM (pool full of referenced blocks; the function is not registered),
 * EIO (code object), EHIP. */
sage_status fn_register(sage_ctx* ctx, const sage_fn_desc* desc, const sage_blob* blobs,
                        size_t n_blobs, sage_fn* out);
/* Register n functions as fn_register would one after another (same
 * classes, same errors), pipelined across functions (the setup parallelism
 * of section "Parallelizing data and context" carried across a batch; the
 * paper defines no batch call): while the host classifies function i's
 * blocks, the fingerprints of function i + 1's device sources already run.
 * Function i takes descs[i] and blobs[i][0 .. n_blobs[i]).  On success
 * out[i] is function i's handle and, when register_ms is not NULL,
 * register_ms[i] the time from the previous function's registration (the
 * call's start for i = 0) to function i's (milliseconds).  All or nothing:
 * on an error no function of the batch stays registered and out is not
 * written.  n = 0 does nothing.  Errors: those of fn_register, EINVAL
 * (null arrays). */
sage_status fn_register_batch(sage_ctx* ctx, size_t n, const sage_fn_desc* descs, const sage_blob* const* blobs,
                              const size_t* n_blobs, sage_fn* out, double* register_ms);

/* Drop a function.  EBUSY while it has live setups.  Blocks no other
 * registered function uses leave the pool.  Returns after every copy that
 * reads the function's sources has finished: the caller may free them.
 * The last stage of section "Multi-stage Resource Exit" (everything of the
 * function is released), taken at once on the caller's request.  Requests
 * of the function still queued in the serving loop fail with ENOTFOUND. */
sage_status fn_unregister(sage_ctx* ctx, sage_fn fn);

/* Apply the multi-stage exit now (it is also applied at the start of
 * fn_register, fn_setup and sage_get_stats, and by the serving loop). */
sage_status sage_tick(sage_ctx* ctx);

/* Make one invocation of `fn` with `batch` rows (MLP) or fields (stencil)
 * runnable; the analogue of SageLoadToGPU() (section "Programming of
 * Function Handle").  Admission: the function's evicted blocks are reloaded
 * (evicting unreferenced blocks of other functions, least recently released
 * first) and each distinct block of the function gains one reference.  The
 * call returns with the blocks resident, except with `progressive` set and
 * blocks coming over the host link: then it returns once their copies are
 * issued, and the body waits for them layer by layer.  With share=0 the
 * read-only data is copied into a private buffer instead.
 * Errors: ENOMEM (cannot admit; nothing changed), ENOTFOUND, EINVAL. */
sage_status fn_setup(sage_ctx* ctx, sage_fn fn, uint32_t batch, sage_inv* out);

/* Flags for fn_invoke / fn_invoke_batch: which I/O buffers are device memory. */
#define SAGE_IO_DEVICE_IN 1u
#define SAGE_IO_DEVICE_OUT 2u

/* fn_setup for n requests (fns[i], batches[i]) in order; stops at the first
 * failure, returning its status, with out[0..k) set for the k that
 * succeeded (*n_done = k).  setup_ms (may be NULL; n entries) receives each
 * request's own setup time in ms, host wall clock inside the library: the
 * setup stage of section "Long Setup Time" (everything before compute) as
 * this library sees it.  Requests arriving together (section "Low System
 * Throughput": concurrent requests) are admitted in one call. */
sage_status fn_setup_batch(sage_ctx* ctx, size_t n, const sage_fn* fns, const uint32_t* batches, sage_inv* out,
                           size_t* n_done, double* setup_ms);

/* Run one set-up invocation: in = X / u0 as described in sage_fn_desc,
 * out = Y / u.  The body waits for the function's data (the kernel-executor
 * readiness check, section "Ensuring Function Correctness").  Blocking.
 * in_bytes/out_bytes must equal the sizes the kind implies (EINVAL). */
sage_status fn_invoke(sage_ctx* ctx, sage_inv inv, const void* in, size_t in_bytes, void* out,
                      size_t out_bytes, uint32_t io_flags);

/* Run n set-up invocations as one group: MLP invocations of the same width
 * and depth run as one grouped GEMM per layer over all their rows (replayed
 * from a captured hipGraph when batch=1); stencil invocations of one
 * function run one sweep launch for all fields.  Invocations of different
 * kinds are split into several groups.  Blocking.  Each output equals the
 * invocation's fn_invoke output.  No passage in the paper (it runs each
 * invocation on its own); batching is the compute side of sharing: one read
 * of the shared weights serves every invocation of the group.  in/out/
 * in_bytes/out_bytes are arrays of n entries, as for fn_invoke. */
sage_status fn_invoke_batch(sage_ctx* ctx, size_t n, const sage_inv* invs, const void* const* in,
                            const size_t* in_bytes, void* const* out, const size_t* out_bytes,
                            uint32_t io_flags);

/* fn_invoke for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * MLP kinds only, device I/O only (in/out are device addresses, as with
 * SAGE_IO_DEVICE_IN | SAGE_IO_DEVICE_OUT); same output bits as fn_invoke.
 * The body's metadata and activations live in one fixed scratch array per
 * GPU (kept by the library until the process ends) instead of buffers the
 * library allocates: at most 512 rows, and batch x width x 2 (BF16) or
 * x 4 (FP32) <= 4 MiB; larger invocations give SAGE_EINVAL before any work.
 * No hipMalloc / hipFree; eager launches; the tile plan comes from timings
 * the context already measured (none yet: a fixed tile shape).  Blocking.
 * Every call on one GPU, from any context, uses the same scratch: calls that
 * overlap on one GPU (two contexts on two threads) race; calls on one
 * context are serialised by its mutex.  ESTATE while the serving loop runs. */
sage_status fn_invoke_noalloc(sage_ctx* ctx, sage_inv inv, const void* in, size_t in_bytes, void* out,
                              size_t out_bytes);

/* End an invocation: drop its block references (blocks reaching zero stay
 * resident until evicted: first exit stage, section "Multi-stage Resource
 * Exit") and free its private buffers.  ESTATE if already released. */
sage_status fn_release(sage_ctx* ctx, sage_inv inv);

/* fn_release for n invocations; stops at the first failure (first exit
 * stage of section "Multi-stage Resource Exit" for each). */
sage_status fn_release_batch(sage_ctx* ctx, size_t n, const sage_inv* invs);

/* ---------------------------------------------------------- introspection
 * Counters and parity introspection (no passage in the paper): what the
 * tests compare with the oracle and what the benchmark reports. */
/* Byte accounting (shared + private = logical), residency, references,
 * H2D bytes and host time per setup stage, since open. */
sage_status sage_get_stats(sage_ctx* ctx, sage_stats* out);
/* Fingerprint of each of the function's blocks, in block order (n = count). */
sage_status sage_fn_fingerprints(sage_ctx* ctx, sage_fn fn, uint64_t* out, size_t n);
/* Per block: class id, pool slot (UINT32_MAX when evicted) and references. */
sage_status sage_fn_block_info(sage_ctx* ctx, sage_fn fn, uint32_t* cls, uint32_t* slot,
                               uint32_t* refs, size_t n);
/* Number of blocks of a function. */
sage_status sage_fn_block_count(sage_ctx* ctx, sage_fn fn, size_t* out);
/* Copy one 64 KiB pool slot to host memory. */
sage_status sage_read_slot(sage_ctx* ctx, uint32_t slot, void* host64k);

/* ------------------------------------------------------ kernel entry points
 * The data-movement kernels of the path, callable directly on device
 * buffers.  stream is a hipStream_t (NULL = the context's own stream); the
 * calls are asynchronous on it. */

/* FP64K-v1 fingerprints of the ceil(nbytes/65536) blocks at dev (the last
 * block may be short) into dev_out[]. */
sage_status sage_fingerprint(sage_ctx* ctx, const void* dev, size_t nbytes, uint64_t* dev_out,
                             void* stream);

/* Block operations, one per 64 KiB block: COPY src -> dst, or VERIFY that the
 * len bytes at src and dst are equal (result[i] = 1 when they differ). */
#define SAGE_OP_COPY 0u
#define SAGE_OP_VERIFY 1u
typedef struct {
  uint64_t src;
  uint64_t dst;
  uint32_t len; /* 1..65536 */
  uint32_t op;  /* SAGE_OP_* */
} sage_blk_op;
sage_status sage_blkcopy(sage_ctx* ctx, const sage_blk_op* dev_ops, size_t n_ops,
                         uint32_t* dev_result, void* stream);

/* ---------------------------------------------------------------- serving
 * Open-loop serving (section "Low System Throughput": Poisson arrivals;
 * section "Multi-stage Resource Exit": warm reuse; "Other Lessons Learned":
 * cache replacement).  One internal thread admits queued requests with
 * fn_setup semantics (evicting unreferenced blocks, least recently released
 * first; a request that cannot be admitted waits for releases), packs the
 * admitted requests of one body shape (and I/O flags) into one grouped
 * launch of at most `max_rows` rows, and keeps up to `inflight_groups`
 * launches on the device; requests arriving meanwhile join the next launch.
 * While the loop runs, fn_invoke / fn_invoke_batch return SAGE_ESTATE.
 * Latencies are measured from sage_submit: setup = until admitted, e2e =
 * until the output is in the caller's buffer. */
typedef struct {
  double setup_ms;
  double e2e_ms;
  uint32_t status; /* sage_status of the request */
} sage_req_info;

typedef struct {
  uint64_t completed, failed, launches, rows;
  double setup_p50_ms, setup_p99_ms; /* nearest rank */
  double e2e_p50_ms, e2e_p99_ms;
  double span_ms;    /* first arrival to last completion */
  double throughput; /* completed requests per second over span_ms */
} sage_serve_report;

sage_status sage_serve_start(sage_ctx* ctx, uint32_t max_rows /* 0 = 8192 */);
/* Drain queued and in-flight requests, then stop the loop. */
sage_status sage_serve_stop(sage_ctx* ctx);
/* Queue one request; in/out as for fn_invoke and owned by the caller until
 * sage_wait returns for it. */
sage_status sage_submit(sage_ctx* ctx, sage_fn fn, uint32_t batch, const void* in, size_t in_bytes, void* out,
                        size_t out_bytes, uint32_t io_flags, uint64_t* req_id);
/* Wait for a request (timeout_ms < 0: forever; EBUSY on timeout).  Returns
 * the request's own status. */
sage_status sage_wait(sage_ctx* ctx, uint64_t req_id, double timeout_ms, sage_req_info* info);
sage_status sage_serve_stats(sage_ctx* ctx, sage_serve_report* out);
sage_status sage_serve_reset_stats(sage_ctx* ctx);

/* --------------------------------------------------------------- timing
 * Per-kernel device time measured with HIP events on the stream each launch
 * is issued on, accumulated while timing is on.  Names: "fp64k", "blkcopy",
 * "ggemm_bf16", "mlp_f32", "stencil7".  A graph replay of L layers counts as
 * L launches of its kernel. */
sage_status sage_timing_enable(sage_ctx* ctx, int on);
sage_status sage_timing_get(sage_ctx* ctx, const char* kernel, double* total_ms, uint64_t* launches);
sage_status sage_timing_reset(sage_ctx* ctx);
/* Restrict timing to the launches of one name (one of the names above;
 * NULL or "" times every kernel again).  Each timed interval costs two event
 * records on its stream, so a caller measuring one kernel's device time
 * can leave the others untimed.  The name is copied; EINVAL for an unknown
 * name. */
sage_status sage_timing_only(sage_ctx* ctx, const char* kernel);
/* Measurement support, not part of the path (no passage of the paper): the
 * compute-side ceiling of the grouped GEMM's main tile shape.  Runs one
 * workgroup per CU, each doing what the main kernel does for one 256 x 256
 * tile of depth k (k / 32 slices; per slice, every wave reads its 12 operand
 * fragments from a four-stage LDS ring and issues its 32 MFMAs, with the
 * main kernel's barrier schedule) except the global loads: the ring is
 * filled once with random BF16 values.  reps launches back to back on the
 * context's control stream.  *us_per_launch is the mean time per launch
 * (HIP events); *shader_ghz the median over workgroups of the shader clock
 * during the last launch (s_memtime against the 100 MHz reference counter).
 * EINVAL unless k is a positive multiple of 32 up to 65536 and
 * 1 <= reps <= 1000; ENOMEM if the small workspace cannot be had. */
sage_status sage_mfma_ceiling(sage_ctx* ctx, uint32_t k, uint32_t reps, double* us_per_launch, double* shader_ghz);
/* Describe the last MLP body launch of this context as text, e.g.
 * "ggemm6p_bf16_256x256:256+ggemm3t_bf16_32x32:384" (kernel:tiles per layer;
 * a second term is the thin-tile launch over split-off ragged row tiles).
 * Writes at most cap bytes including the terminating NUL; EINVAL if the
 * text does not fit, ENOTFOUND before the first MLP launch. */
sage_status sage_last_launch(sage_ctx* ctx, char* out, size_t cap);

/* --------------------------------------------------------------- self test
 * Host-only check of the setup orchestrator: runs its two branches with
 * stand-in stages that sleep (code load = load_ms; data = host_ms then
 * copy_ms per the data branch) and reports the measured setup time.  With
 * serial != 0 the branches run one after the other.  Needs no GPU. */
sage_status sage_selftest_setup_overlap(double load_ms, double host_ms, double copy_ms, int serial,
                                        double* measured_ms);

/* Host-only check of the BF16 launch planner: the plan for a layer of width
 * `width` over groups of rows[0..n_groups) on `cus` CUs, given each listed
 * tile shape's time for one full wave of tiles (shapes not listed are not
 * considered), written to `out` as "main:tiles[+tail:tiles] cost_ms".
 * EINVAL for an unknown shape name, no fitting shape, or a short buffer.
 * Needs no GPU. */
sage_status sage_selftest_plan(uint32_t width, const uint32_t* rows, size_t n_groups, const char* const* shapes,
                               const double* wave_ms, size_t n_shapes, uint32_t cus, char* out, size_t cap);

/* Host-only check of the per-layer readiness of a reload (`progressive`):
 * first[0..n) is the first block, in the function, of each reloaded class in
 * reload order (non-decreasing); a layer's weights span layer_bytes bytes
 * from l * layer_bytes.  out[l] (layers entries) receives how many leading
 * classes hold every block of layers 0..l: layer l's launch waits for
 * exactly those copies.  EINVAL for a decreasing `first` or empty input.
 * Needs no GPU. */
sage_status sage_selftest_segments(const uint32_t* first, size_t n, uint32_t layers, uint64_t layer_bytes,
                                   size_t* out);

/* Host-only randomized check of the block pool (the structure behind
 * sections "Read-only Memory Sharing" and "Multi-stage Resource Exit":
 * shared slots, references, eviction of unreferenced blocks) and of its
 * fingerprint index.  Runs n_ops random registrations, references,
 * releases, reloads and drops on a pool of budget_slots slots (a host
 * stand-in arena: no device memory) against a plain model, checking after
 * every operation: residency and slots, no slot held twice, used slots =
 * resident classes, the eviction order, and that each fingerprint chain
 * holds exactly the resident classes of its fingerprint; then random
 * inserts and deletions of the index against a hash map.  Stops at the first
 * violation: EINVAL, *failed_op = its operation number (n_ops when all
 * passed) and the reason in sage_last_error.  Needs no GPU. */
sage_status sage_selftest_pool(uint64_t seed, uint32_t n_ops, uint32_t budget_slots, uint32_t* failed_op);

#if defined(__GNUC__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif
#endif /* SAGE_H */
