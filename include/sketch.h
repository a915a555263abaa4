/*
 * sketch.h - C ABI of the MI355X single-pass PCA library.
 *
 * The library computes the truncated SVD / PCA of a dense m x n row-major matrix A that is seen
 * once, in row blocks, following Algorithm 4 of Yu, Gu, Li, Liu and Li, "Single-Pass PCA of Large
 * High-Dimensional Data" (IJCAI 2017):
 *
 *   sketch_init / sketch_reset   Omega = randn(n, l), G = [], H = 0           (Alg. 4, steps 1-3)
 *   sketch_ingest_block          g = a Omega; G = [G; g]; H = H + a^T g       (Alg. 4, steps 4-8;
 *                                                                              Eq. 10)
 *   sketch_finalize              column-block loop with re-orthogonalisation  (Alg. 4, steps 9-15;
 *                                (Eqs. 7-9), then [U~, S, V] = svd(B),         steps 16-19)
 *                                U = Q U~, truncation to k
 *
 * Conventions
 *   - Every call returns a sketch_status and never aborts or throws across the ABI.  On failure
 *     sketch_last_error() returns a thread-local message describing the last error.
 *   - "device pointer" means memory on the GPU the handle was created on (from hipMalloc or a
 *     PyTorch CUDA tensor); "pinned host pointer" means memory from hipHostMalloc (or a PyTorch
 *     pinned tensor).  Pageable host memory is rejected with SKETCH_E_INVAL.
 *   - Matrices are row-major with an explicit leading dimension counted in elements.
 *   - The library never allocates device memory: all device state lives in a caller-owned
 *     workspace of sketch_workspace_size() bytes.  It owns one copy stream and a few events.
 *   - Kernels run on the caller's HIP stream given at init.  A handle is not thread-safe;
 *     distinct handles may be used concurrently.
 *   - Any HIP runtime error makes the handle sticky in SKETCH_E_DEVICE; only sketch_destroy is
 *     then valid.  A block holding a NaN or Inf makes it sticky in SKETCH_E_NONFINITE: the kernel
 *     that sees it sets a host-mapped flag, so the first call made after that kernel ran reports
 *     it (at the latest sketch_finalize, which waits for the pass).
 */
#ifndef SKETCH_H
#define SKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sketch_s* sketch_t;

typedef enum {
  SKETCH_OK = 0,
  SKETCH_E_INVAL = 1,      /* bad argument or unsupported combination */
  SKETCH_E_STATE = 2,      /* call not valid in the handle's state (e.g. ingest after finalize) */
  SKETCH_E_NOMEM = 3,      /* workspace too small */
  SKETCH_E_CAPACITY = 4,   /* more rows than m_capacity, or a block larger than max_block_rows */
  SKETCH_E_NONFINITE = 5,  /* an ingested block held NaN or Inf (sticky) */
  SKETCH_E_DEVICE = 6      /* a HIP runtime error (sticky) */
} sketch_status;

/* Element formats.  As a source format: the type of the rows passed to sketch_ingest_block.
 * As a compute mode: the arithmetic of the two streaming products g = a Omega and a^T g.
 *   F64        FP64 operands, FP64 accumulation (the paper's precision, Sec. 4.2).
 *   F32        FP32 operands, FP32 accumulation within a block, FP64 accumulation of H.
 *   BF16       a and Omega rounded to BF16 (RNE); g kept in FP32 and fed to a^T g as a BF16
 *              hi + lo pair; FP32 accumulation within a block, FP64 accumulation of H.
 *   BF16X2     a split as bf16(a) + bf16(a - bf16(a)); otherwise as BF16.
 *   FP8_E4M3   a scaled by a power of two per row block (largest with amax * 2^e <= 448) and
 *              rounded to OCP E4M3; Omega' = e4m3(32 fp32(Omega)) / 32; a^T g uses the same a'
 *              with g as a BF16 hi + lo pair.
 * In every mode G is stored in FP32 (FP64 in F64 mode) and everything after the pass (the
 * column-block loop and the SVD of B) runs in FP64.  Omega' (Omega rounded to the operand format)
 * is the matrix used by every step, and is what sketch_get_omega returns. */
typedef enum {
  SKETCH_F64 = 0,
  SKETCH_F32 = 1,
  SKETCH_BF16 = 2,
  SKETCH_BF16X2 = 3,
  SKETCH_FP8_E4M3 = 4
} sketch_dtype;

typedef struct {
  int64_t n;               /* columns of A (>= 1) */
  int64_t m_capacity;      /* most rows the handle will ingest in total (>= 1) */
  int64_t max_block_rows;  /* largest nrows of one sketch_ingest_block call (>= 1) */
  int32_t k;               /* number of singular triplets returned, 1 <= k <= l */
  int32_t l;               /* sketch width; l = t*b "slightly larger than k" (Alg. 4 step 2),
                              l <= n, l <= 128 */
  int32_t b;               /* column block width of the finalize loop (Alg. 4 steps 9-15); divides l,
                              1 <= b <= 32 or b = l.  With b = l the loop is one block: Cholesky
                              QR twice of the whole G and B = R^-T H^T (fastest on the GPU; the
                              workspace then holds a second m x l FP64 matrix) */
  int32_t compute;         /* sketch_dtype compute mode */
  int32_t host_slots;      /* device staging slots for pinned-host sources: 0 (device sources
                              only) or 2..4 (copies overlap compute on a side stream) */
  int32_t host_src;        /* sketch_dtype of host rows when host_slots > 0: F32, F64 or BF16 */
  int32_t want_u;          /* 1: finalize may return U (m x k) */
  int32_t omega_from_seed; /* 1: Omega drawn on the device from `seed` (Philox-4x64-10 + Box-Muller,
                              entry (r, c) from words 2(r l + c) and 2(r l + c) + 1 of the stream
                              with key (seed, 0)); 0: supplied by sketch_set_omega */
  int32_t centre;          /* 1: PCA of the column-centred A - 1 mu^T, mu = the column means (the
                              method assumes centred data, Sec. 2.1), still in one pass: the pass
                              also sums the columns of A, and sketch_finalize centres the sketch
                              (G - 1 (Omega'^T mu)^T, H - mu (G^T 1)^T) before Alg. 4 steps 9-19.
                              Needs l <= 127.  0: A as given */
  int32_t reserved;        /* 0 */
  uint64_t seed;
} sketch_config;

/* Device bytes the workspace must hold for `cfg`; 0 if cfg is invalid (see sketch_last_error). */
size_t sketch_workspace_size(const sketch_config* cfg);

/* Creates a handle whose state lives in `dev_ws` (device pointer, >= sketch_workspace_size bytes,
 * 256-byte aligned, owned by the caller and kept alive until sketch_destroy).  `hip_stream` is the
 * hipStream_t all kernels are launched on (NULL = the null stream).  With omega_from_seed = 1,
 * Omega is generated here (Alg. 4 step 3); H is zeroed.  Enqueues work and returns at once. */
sketch_status sketch_init(sketch_t* out, const sketch_config* cfg, void* dev_ws, size_t ws_bytes,
                          void* hip_stream);

/* Starts a new pass on the same handle and workspace: zero rows, H = 0, and a new Omega drawn
 * from `seed` when the handle draws its own (Alg. 4 steps 1-3).  Valid in any non-sticky state. */
sketch_status sketch_reset(sketch_t h, uint64_t seed);

/* Supplies Omega (n x l, FP64, row-major with leading dimension ld >= l, device pointer) for a
 * handle created with omega_from_seed = 0.  Must precede the first ingest.  The library rounds it
 * to the operand format of the compute mode (Omega').  The caller's buffer may be freed after the
 * call returns and the stream has passed it. */
sketch_status sketch_set_omega(sketch_t h, const double* omega_dev, int64_t ld);

/* Ingests the next nrows rows of A (Alg. 4 steps 5-7): `rows` points at an nrows x n row-major
 * block with leading dimension ld >= n, of format `src_dtype`, either in device memory
 * (src_is_device = 1; F64, F32 or BF16) or in pinned host memory (src_is_device = 0; requires
 * host_slots > 0 and src_dtype == host_src).  Asynchronous: a host block must stay unchanged until
 * sketch_poll reports its ticket done; a device block until the stream passes this point.
 * Errors: E_INVAL (bad arguments, pageable host memory), E_CAPACITY (nrows > max_block_rows or
 * the total exceeds m_capacity), E_STATE (after finalize or before Omega is set). */
sketch_status sketch_ingest_block(sketch_t h, const void* rows, int32_t src_dtype, int64_t nrows,
                                  int64_t ld, int32_t src_is_device, uint64_t* ticket);

/* *done = 1 once the host buffer of `ticket` may be reused (its copy to the device finished);
 * device-source tickets are done when their kernels finished.  Non-blocking. */
sketch_status sketch_poll(sketch_t h, uint64_t ticket, int32_t* done);

/* Runs Alg. 4 steps 9-19 on the stream and waits for it.  Outputs (device pointers):
 *   S_dev  k doubles, descending;
 *   V_dev  n x k row-major, leading dimension ldv >= k (principal components);
 *   U_dev  m x k row-major, ldu >= k, or NULL (requires want_u = 1 when non-NULL);
 *   rank_out  number of basis vectors kept (l unless the rank guard stopped the loop early).
 * Singular pairs are signed so the largest-magnitude entry of each v_j is positive (lowest index
 * on ties).  Columns past min(k, rank) are zero.  Rank guard (a reading: the paper assumes a
 * full-rank sketch): with r0 the first diagonal of the first combined R, a block keeps only its
 * leading columns whose combined R diagonal exceeds 1e-10 r0, and the loop stops there.
 * The handle then rejects ingest (E_STATE) until sketch_reset. */
sketch_status sketch_finalize(sketch_t h, double* S_dev, double* U_dev, int64_t ldu, double* V_dev,
                              int64_t ldv, int32_t* rank_out);

/* ---------------------------------------------------------------- checkpoint, restore, merge
 * The pass state after any number of ingested blocks is G (the rows seen so far), H and Omega'
 * (Alg. 4 steps 3-8).  Eq. 10 makes it mergeable: the state of the rows of A_1 followed by those
 * of A_2 is G = [G_1; G_2] and H = H_1 + H_2, given the same Omega'.  A checkpoint is a host byte
 * image of the state: a header, H and G exactly as stored on the device (so a restored pass
 * continues with the same bits), and Omega' itself only when it was supplied by sketch_set_omega
 * (a seed-drawn Omega' is drawn again from the seed).  The calls below take any host memory
 * (pinned or pageable), copy synchronously and return when done. */

/* Bytes of a checkpoint of the handle's current state; 0 (with sketch_last_error set) before
 * Omega is set, after finalize or in a sticky state. */
size_t sketch_checkpoint_size(sketch_t h);

/* Writes the current pass state to `buf` (host memory of `bytes` >= sketch_checkpoint_size bytes,
 * owned by the caller).  Waits for the handle's stream.  E_STATE before Omega is set or after
 * finalize; E_INVAL for a short buffer; E_NONFINITE if a block held NaN or Inf. */
sketch_status sketch_checkpoint(sketch_t h, void* buf, size_t bytes);

/* Replaces the handle's state by a checkpoint's (any previous rows are dropped) and leaves it
 * ingesting: further blocks continue that pass.  The handle must have the checkpoint's n, l and
 * compute mode (k, b, want_u, host staging and max_block_rows may differ) and m_capacity >= its
 * rows (else E_CAPACITY); Omega' becomes the checkpoint's.  E_INVAL for a buffer that is not a
 * checkpoint of this library version or does not fit the handle. */
sketch_status sketch_restore(sketch_t h, const void* buf, size_t bytes);

/* Adds a checkpointed sketch of further rows to the handle's (Eq. 10): H = H + H', and the
 * checkpoint's G rows are appended after the rows ingested so far.  The checkpoint must have been
 * taken with the same Omega' (checked bit for bit; E_INVAL otherwise) and the handle's n, l and
 * compute mode; E_CAPACITY if the rows would exceed m_capacity; E_STATE after finalize. */
sketch_status sketch_merge(sketch_t h, const void* buf, size_t bytes);

/* Power scheme with P = 1 (Sec. 2.2; the remark closing Sec. 3.3: the loop is run once more with
 * Omega replaced by orth(H); Sec. 4.2 reports its accuracy).  Call it after the first pass over all
 * rows of A: it replaces Omega by Omega_2 = sqrt(n) orth(H) (FP64 on the device, then rounded to
 * the operand format like any Omega') and starts a second pass (rows = 0, G = [], H = 0).  The
 * caller then ingests the rows of A again and calls sketch_finalize, which returns the triplets of
 * the randomised SVD of (A A^T) A's range applied to A (singular values of A, not cubed).
 * The scale sqrt(n) is a reading: results depend only on the span of Omega.  route: 0 = Cholesky
 * QR2 of H when its tests accept it, else shifted Cholesky QR3, else block Gram-Schmidt with
 * Householder TSQR; 2 = shifted QR3 first; 1 = Gram-Schmidt + TSQR (all give orth(H));
 * *route_used (nullable) = the route that produced it.  Waits for the stream.  A later
 * sketch_reset draws a Gaussian Omega again when the handle draws its own (it keeps Omega_2
 * otherwise), and checkpoints store Omega_2 itself.  E_STATE before any rows or after finalize. */
sketch_status sketch_power_restart(sketch_t h, int32_t route, int32_t* route_used);

/* Column means mu (n values, FP64, device pointer) of the rows ingested so far, for a handle
 * created with centre = 1: the sums of the pass over the row count before sketch_finalize, the
 * means it centred with after it.  E_STATE without centring or before any row. */
sketch_status sketch_column_mean(sketch_t h, double* mu_dev);

/* Copies Omega' (n x l, FP64, row-major, leading dimension ld >= l) into device memory. */
sketch_status sketch_get_omega(sketch_t h, double* omega_dev, int64_t ld);

/* Which orthonormalisation the last sketch_finalize used (host integers, either pointer may be
 * NULL).  *loop_path: 0 = Cholesky QR of each column block of the loop of Alg. 4 steps 9-15
 * (Sec. 3.2, Eqs. 7-9), 1 = Householder TSQR (taken when a block's Gram matrix is too
 * ill-conditioned for Cholesky QR, or a block is rank deficient).  *rb_path, for R_B of B^T before
 * the SVD of Alg. 4 steps 16-19: 0 = Cholesky QR2 (B well conditioned), 2 = shifted Cholesky QR3,
 * 1 = block Gram-Schmidt with TSQR.  -1 when the sketch was empty.  E_STATE before finalize. */
sketch_status sketch_finalize_paths(sketch_t h, int32_t* loop_path, int32_t* rb_path);

/* Test hook for the next sketch_finalize: loop_householder nonzero takes TSQR for every column
 * block without trying Cholesky QR; rb_mode 1 takes Gram-Schmidt + TSQR for R_B, 2 shifted Cholesky
 * QR3 directly, 3 forms Cholesky QR2 and the results from it, then treats it as not accepted (so
 * they are formed again from shifted Cholesky QR3, as for a rejected QR2), 4 as 3 but with QR2's
 * first Cholesky factorisation taking its failed-pivot exit (a non-positive pivot, simulated from
 * the host), 0 the normal order.  All paths compute the same factorisation.  E_INVAL for another
 * rb_mode. */
sketch_status sketch_debug_force_paths(sketch_t h, int32_t loop_householder, int32_t rb_mode);

/* Copies the pass state as FP64 into device memory: G (rows x l, row-major, ld = l) and
 * H (n x l, row-major, ld = l); either pointer may be NULL.  *rows_out = rows ingested. */
sketch_status sketch_debug_state(sketch_t h, double* G_dev, double* H_dev, int64_t* rows_out);

/* Writes `count` raw 64-bit words of the Philox-4x64-10 stream with key (seed, 0), starting at
 * word `first` (word w is lane w % 4 of the block at counter (w / 4, 0, 0, 0)), to device memory,
 * on `hip_stream`, and waits for it.  Exposes the generator behind omega_from_seed for testing. */
sketch_status sketch_philox_words(uint64_t seed, uint64_t first, int64_t count, uint64_t* out_dev,
                                  void* hip_stream);

/* The pair order of one sweep of the one-sided Jacobi SVD of R_B^T (svd(B), Alg. 4 steps 16-19),
 * computed on the host by the same code the kernel runs, for testing.  For n columns (0 <= n <= 128,
 * rounded up to even), writes rounds x 64 x 2 bytes to host memory `pairs` (capacity bytes): for
 * round r and lane group g, pairs[2 (64 r + g)] is the column the group keeps in registers and
 * pairs[2 (64 r + g) + 1] the one it takes through LDS, both 255 when the group idles that round.
 * *rounds = the number of rounds.  E_INVAL for another n or a table that does not fit. */
sketch_status sketch_jacobi_schedule(int32_t n, uint8_t* pairs, int64_t capacity, int32_t* rounds);

/* Per-kernel timing of the pass (HIP events on the launch stream, taken around every launch of
 * the two streaming products while enabled).  sketch_profile_read waits for the stream and
 * returns, for kind 0 = g = a Omega (incl. its split reduction), 1 = H += a^T g, 2 = finalize:
 * the number of launches and their summed milliseconds, then clears the counters. */
sketch_status sketch_profile_enable(sketch_t h, int32_t on);
sketch_status sketch_profile_read(sketch_t h, int32_t kind, int64_t* launches, double* total_ms);

/* Releases the handle's stream, events and host bookkeeping (not the caller's workspace).
 * Waits for outstanding work first. */
sketch_status sketch_destroy(sketch_t h);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* sketch_last_error(void);

/* ================================================================ one call, no allocation
 * For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the whole of Algorithm 4 on a device-resident A in one call, with the
 * workspace taken from a fixed device array inside the library (64 MiB on each GPU, held until
 * the process ends) instead of caller memory.  The call creates no stream, event or host
 * allocation and calls no hipMalloc/hipFree.
 *
 * Equivalent to sketch_init(cfg) + sketch_ingest_block of consecutive blocks of
 * cfg->max_block_rows rows (the last one shorter) + sketch_finalize, with the same kernels and
 * bits.  cfg: as for sketch_init with host_slots = 0, omega_from_seed = 1 and m <= m_capacity;
 * sketch_workspace_size(cfg) must not exceed 64 MiB (else E_CAPACITY, with the size in the
 * message).  A_dev: device pointer, m x n row-major, leading dimension lda >= n, format src_dtype
 * (F64, F32 or BF16 as the compute mode accepts).  Outputs as sketch_finalize (S_dev, V_dev
 * required; U_dev optional, requires want_u).  Runs on hip_stream and waits for it.
 * All calls on one GPU share its array, which keeps the last call's contents (each call clears
 * what it reads before writing): calls that overlap on the same GPU race and must be serialised
 * by the caller.  A NaN or Inf in A returns E_NONFINITE; E_DEVICE on a HIP error. */
sketch_status sketch_pca_static(const sketch_config* cfg, const void* A_dev, int32_t src_dtype,
                                int64_t m, int64_t lda, double* S_dev, double* U_dev,
                                int64_t ldu, double* V_dev, int64_t ldv, int32_t* rank_out,
                                void* hip_stream);

/* ================================================================ serving
 * Many concurrent single-pass PCA streams on one GPU.  Each stream is one instance of Algorithm 4
 * (its Omega seed, G, H resident in device memory); the server admits streams while their state
 * fits a device-memory budget (later ones wait in FIFO order and are admitted as finalized
 * streams release their memory), and runs continuous batching: a scheduler gathers one pending
 * row block from each of up to max_group streams, of any widths n, and processes them with one
 * grouped launch of each streaming product (g = a Omega, its split reduction, H = H + a^T g;
 * Alg. 4 steps 5-7, Eq. 10).  Blocks that arrive while a group runs join the next group.  Every
 * block is planned from its own shape only, so a stream's results are bitwise the same alone and
 * in any mix.  The column-block loop and SVD (Alg. 4 steps 9-19) run per stream in
 * sketch_server_finalize on a second stream, overlapping the other streams' ingestion.
 *
 * Rows are device pointers (row-major, ld >= n) in the server's source format; the caller keeps a
 * block unchanged until sketch_server_poll reports its ticket.  The server owns one scheduler
 * thread (worker = 1) or is driven by sketch_server_step (worker = 0), one finalize stream and
 * its events; all device memory is the caller's workspace.  Calls are thread-safe. */
typedef struct sketch_server_s* sketch_server_t;

typedef struct {
  int32_t compute;         /* sketch_dtype: F64, F32, BF16 or BF16X2 */
  int32_t src;             /* format of every submitted block: F32 (F64 or F32 with compute F64;
                              F32 or BF16 with compute BF16) */
  int32_t l;               /* sketch width of every stream, 1..128 */
  int32_t max_group;       /* most blocks in one grouped launch, 1..64 */
  int64_t max_n;           /* widest stream (>= l) */
  int64_t max_m;           /* most rows of one stream */
  int64_t max_block_rows;  /* largest block */
  int64_t state_bytes;     /* device memory for resident stream states (the admission budget) */
  int32_t worker;          /* 1: a library thread schedules; 0: the caller calls sketch_server_step */
  int32_t host_slots;      /* device staging slots for pinned-host blocks (0: device rows only); each
                              holds max_block_rows x max_n rows of the src format, copied on a
                              library-owned stream while earlier groups compute */
} sketch_server_config;

typedef struct {
  int64_t active;          /* streams resident on the device */
  int64_t queued;          /* streams waiting for memory */
  int64_t state_used;      /* bytes of the state budget in use */
  int64_t state_peak;      /* most bytes ever in use */
  int64_t groups;          /* grouped launches issued */
  int64_t blocks;          /* blocks processed */
  int64_t max_blocks_in_group;
  int64_t finalized;       /* streams finalized */
  int64_t queued_peak;     /* most streams ever waiting for memory at once */
} sketch_server_stats;

/* Device bytes the server's workspace must hold (shared scratch + state budget); 0 if invalid. */
size_t sketch_server_workspace_size(const sketch_server_config* cfg);

/* Device bytes of one stream's resident state (what admission charges against state_bytes);
 * cfg->l and cfg->compute must match the server's; 0 if invalid. */
size_t sketch_server_stream_bytes(const sketch_server_config* srv, const sketch_config* cfg);

/* Creates a server in `dev_ws` (device pointer, 256-byte aligned, >= workspace size, owned by the
 * caller until sketch_server_destroy); grouped launches run on `hip_stream`. */
sketch_status sketch_server_create(sketch_server_t* out, const sketch_server_config* cfg,
                                   void* dev_ws, size_t ws_bytes, void* hip_stream);

/* Opens a stream (cfg: n <= max_n, m_capacity <= max_m, max_block_rows <= the server's,
 * l and compute equal to the server's, omega_from_seed = 1, host_slots = 0).  *admitted = 1 if its
 * state was placed at once, 0 if it waits for memory (blocks may be submitted meanwhile).
 * E_CAPACITY if the stream alone exceeds the state budget. */
sketch_status sketch_server_open(sketch_server_t s, const sketch_config* cfg, uint64_t* stream_id,
                                 int32_t* admitted);

/* Queues the next nrows rows of a stream (device pointer, src format, ld >= n).  *ticket
 * identifies the block in sketch_server_poll.  E_STATE after the stream's finalize began;
 * E_CAPACITY past its m_capacity or max_block_rows.  Same as sketch_server_submit_ex with
 * src_is_device = 1 and no arrival time. */
sketch_status sketch_server_submit(sketch_server_t s, uint64_t stream_id, const void* rows,
                                   int64_t nrows, int64_t ld, uint64_t* ticket);

/* As sketch_server_submit, with the rows either in device memory (src_is_device = 1) or in pinned
 * host memory (0; needs host_slots > 0, else E_INVAL; pageable memory is rejected with E_INVAL):
 * a host block is copied into a free staging slot when its group forms, on the library's copy
 * stream, and the group's kernels wait for the copy.  arrival_s: the block's arrival time on
 * sketch_server_clock(), from which its latency is measured (< 0: the submit time).  The caller
 * keeps the rows unchanged until sketch_server_poll reports the ticket or the stream's finalize
 * returns. */
sketch_status sketch_server_submit_ex(sketch_server_t s, uint64_t stream_id, const void* rows,
                                      int32_t src_is_device, int64_t nrows, int64_t ld,
                                      double arrival_s, uint64_t* ticket);

/* Seconds on the monotonic clock the server stamps submits and completions with. */
double sketch_server_clock(void);

/* One scheduler round (worker = 0 only; with a worker it returns E_STATE): retire finished
 * groups, admit waiting streams, launch at most one new group.  *launched = blocks launched. */
sketch_status sketch_server_step(sketch_server_t s, int32_t* launched);

/* Up to `cap` finished blocks since the last call: their tickets and latencies in seconds, from
 * the block's arrival (its submit, or the arrival_s given) to the completion of its grouped
 * launch on the GPU (the group's
 * completion event, converted to host time through an anchor event recorded on the idle stream
 * at creation and refreshed every 10 s when the stream is idle; the conversion may read late by
 * the few microseconds of one stream synchronisation).  *count = entries written. */
sketch_status sketch_server_poll(sketch_server_t s, uint64_t* tickets, double* latency_s,
                                 int32_t cap, int32_t* count);

/* Waits for the stream's blocks, runs Alg. 4 steps 9-19 for it (outputs as sketch_finalize:
 * device S (k), V (n x k, ldv), U (m x k, ldu) or NULL), then releases its state.  Blocks. */
sketch_status sketch_server_finalize(sketch_server_t s, uint64_t stream_id, double* S_dev,
                                     double* U_dev, int64_t ldu, double* V_dev, int64_t ldv,
                                     int32_t* rank_out);

sketch_status sketch_server_get_stats(sketch_server_t s, sketch_server_stats* out);

/* Stops the scheduler, waits for outstanding work and releases host resources. */
sketch_status sketch_server_destroy(sketch_server_t s);

#ifdef __cplusplus
}
#endif
#endif /* SKETCH_H */
