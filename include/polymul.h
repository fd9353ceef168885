/*
 * polymul.h -- C ABI of the MI355X (gfx950) sparse polynomial product.
 *
 * Operation (Section 2 of Gastineau & Laskar, problem statement and Fig. 1):
 * for A = sum_i a_i x^{alpha_i} and B = sum_j b_j x^{beta_j}, each stored in
 * distributed format (a term list sorted by a monomial order), compute
 *     C = A * B = sum_{i,j} a_i b_j x^{alpha_i + beta_j}
 * with equal monomials grouped, like terms summed and zero terms dropped, the
 * result sorted ascending (Algorithm 1 concatenates its sorted containers in
 * ascending order to obtain the canonical form).  This is Algorithm 1's
 * mul(A, B, .) without the interval-count argument: how the work is split on
 * the device is internal.
 *
 * Term layout.  A polynomial is two device arrays of equal length n:
 *   keys[n]   uint64: packed exponent vector.  Variable v (0 <= v < nvars)
 *             occupies bits [(nvars-1-v)*bits, (nvars-1-v)*bits + bits), so
 *             variable 0 is the most significant field and the unsigned order
 *             of keys is the lexicographic monomial order (the paper packs all
 *             exponents of a term into one 64-bit word, Section 6).  Keys must
 *             be strictly ascending and bits above nvars*bits must be zero.
 *   coefs[n]  8 bytes per term, by ring:
 *             PM_MODP61  uint64 residue in [0, p), p = 2^61 - 1
 *             PM_F64     IEEE double, finite
 *             PM_I64     int64 (arithmetic is exact modulo 2^64; the result is
 *                        the exact integer product when that fits int64)
 *             PM_MODQ64  uint64 residue in [0, q), q = 2^64 - 59 (a prime)
 *             or 24 bytes per term:
 *             PM_Z192    exact integers: three uint64 words per term, the
 *                        two's-complement form of a value in [-2^191, 2^191),
 *                        least significant word first (coefs[3i..3i+2]).
 *                        pm_mul forms the product modulo 2^64, 2^61 - 1 and
 *                        2^64 - 59 and recovers each coefficient by the
 *                        Chinese remainder theorem; it returns PM_EOVERFLOW
 *                        unless bits(max|a_i|) + bits(max|b_j|) +
 *                        bits(min(n_f, n_g)) <= 187, which keeps every output
 *                        coefficient below 2^187 in magnitude (bits(x): the
 *                        bit length).  pm_mul and pm_mul_bound only: the batch,
 *                        prepared-batch, server, autotuner and no-allocation
 *                        entry points return PM_EINVAL for it.
 *   Zero input coefficients are allowed; they contribute nothing.
 * Output keys are strictly ascending; no output coefficient is zero (for
 * PM_F64: exactly +0.0 or -0.0 is dropped).
 *
 * Memory.  All term arrays are device memory owned by the caller and must stay
 * alive until the stream has executed the call.  The output arrays and the
 * workspace are caller-allocated device memory; the library allocates no
 * device memory on the product path.  `n_out` may point to device memory or
 * to pinned (hipHostMalloc) host memory.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default stream).
 * pm_mul and pm_mul_batch read back a small statistics block (validation
 * result and per-variable exponent ranges) with one synchronisation of the
 * stream, then enqueue the product and return: the output arrays and *n_out
 * are valid once the stream has completed.
 *
 * FP64 summation order.  Contributions to one output monomial are added left
 * to right in row-major (i, j) order of the operands, each product rounded
 * once; the result is therefore the same whether a product runs alone, in a
 * batch or through the server, and equals the plain row-major schoolbook sum.
 *
 * Errors are negative return codes; see pm_strerror.
 */
#ifndef POLYMUL_H
#define POLYMUL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PM_OK 0
#define PM_EINVAL (-1)     /* null pointer, bad layout, negative size, key bits outside the fields */
#define PM_EUNSORTED (-2)  /* input keys not strictly ascending */
#define PM_EOVERFLOW (-3)  /* max_f[v] + max_g[v] does not fit the field of variable v (PM_Z192: also the 2^187 bound) */
#define PM_ERANGE (-4)     /* residue >= p (PM_MODP61), >= q (PM_MODQ64) or non-finite coefficient (PM_F64) */
#define PM_ECAPACITY (-5)  /* output capacity below the bound (pm_server_submit only) */
#define PM_ENOMEM (-6)     /* workspace too small, a sparse product of more than 2^32 - 1 term pairs, or a server arena that can never hold the request */
#define PM_EDEVICE (-7)    /* HIP runtime error; pm_last_error() has the message */
#define PM_EBUSY (-8)      /* server: request queue full, retry later */

typedef enum { PM_MODP61 = 0, PM_F64 = 1, PM_I64 = 2, PM_MODQ64 = 3, PM_Z192 = 4 } pm_ring;

/* nvars >= 1, bits >= 1, nvars * bits <= 64; ring one of pm_ring. */
typedef struct {
    uint32_t nvars;
    uint32_t bits;
    int32_t ring;
    int32_t reserved; /* must be 0 */
} pm_layout;

/* Read-only operand: n terms, device pointers (may be NULL when n == 0). */
typedef struct {
    int64_t n;
    const uint64_t *keys;
    const void *coefs;
} pm_cpoly;

/* Result: device arrays of `capacity` terms; *n_out receives the term count.
 * *n_out > capacity signals truncation, and a capacity of at least *n_out
 * avoids it: *n_out is then the full term count or, on the sorted path when
 * terms cancel, the number of distinct monomials before the cancelled ones
 * are dropped (result slots are assigned before the sums are known).  A
 * truncated result holds the first terms of the product, followed by entries
 * with zero coefficients.  A capacity of at least the bound from
 * pm_mul_bound never truncates. */
typedef struct {
    int64_t capacity;
    int64_t *n_out;
    uint64_t *keys;
    void *coefs;
} pm_poly;

/*
 * Bound on the result size and the workspace size of pm_mul.
 * max_terms = min(n_f * n_g, prod_v (max_f[v] + max_g[v] - min_f[v] - min_g[v] + 1)):
 * every output monomial is some alpha_i + beta_j (Fig. 1) and lies in the
 * degree box of the two operands.  Validates the operands (same codes as
 * pm_mul).  Synchronises `stream`.
 */
int pm_mul_bound(const pm_layout *layout, const pm_cpoly *f, const pm_cpoly *g, int64_t *max_terms,
                 int64_t *workspace_bytes, void *stream);

/*
 * h = f * g.  `workspace` is device memory of at least the size returned by
 * pm_mul_bound for the same operands, 256-byte aligned (else PM_EINVAL).
 * Returns PM_OK once the product is enqueued on `stream`, or an error code
 * (nothing enqueued that writes h).  The plan depends on the operands'
 * exponent ranges, so the call synchronises `stream` once, for the
 * validation and statistics read-back, before it enqueues the product; the
 * kernels then run asynchronously.  Calls from several threads are
 * serialised by one library lock (they share a pinned staging buffer).
 * pm_batch_prepare / pm_batch_launch replay a validated plan without the
 * read-back; the server polls it instead of waiting.
 */
int pm_mul(const pm_layout *layout, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h, void *workspace,
           int64_t workspace_bytes, void *stream);

/*
 * pm_mul without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operands, result and error codes as pm_mul, but
 * the workspace is a static device array of PM_NOALLOC_SCRATCH_BYTES that
 * every device holds from library load until the process ends; the call
 * makes no device or pinned-host allocation.  A product whose pm_mul_bound
 * workspace exceeds that size is rejected with PM_ENOMEM before any kernel
 * that writes h is enqueued.  All calls on one device share the array (it
 * keeps the last call's contents; the kernels clear what must start at
 * zero): calls whose work overlaps on one device race, so serialise them on
 * one stream.  Like pm_mul it synchronises `stream` for the operand
 * validation before enqueueing the product.
 */
#define PM_NOALLOC_SCRATCH_BYTES (64ll << 20)
int pm_mul_noalloc(const pm_layout *layout, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h, void *stream);

/*
 * Batched form: `count` independent products h[k] = f[k] * g[k] sharing one
 * layout, run from a single device work queue of tiles (persistent kernels,
 * replayed from a HIP graph).  max_terms[k] receives each product's bound;
 * workspace_bytes the size pm_mul_batch needs for the whole batch.  The
 * workspace is 256-byte aligned, as for pm_mul (else PM_EINVAL).
 */
int pm_mul_batch_bound(const pm_layout *layout, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
                       int64_t *max_terms, int64_t *workspace_bytes, void *stream);
int pm_mul_batch(const pm_layout *layout, int64_t count, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h,
                 void *workspace, int64_t workspace_bytes, void *stream);

/*
 * Prepared batch: validate and plan `count` products once, upload their
 * descriptors into `workspace`, and capture the whole device pipeline (zeroing,
 * key compression, tile / pair work queues, radix passes, reduction, dense
 * compaction) in one HIP graph.  pm_batch_launch replays that graph on
 * `stream`: one graph launch runs every product of the batch.  Operands,
 * results and workspace stay bound to the batch; operand contents may change
 * between launches only if term counts, strict ordering and per-variable
 * exponent ranges stay within what was validated (prepare again otherwise).
 * Returns NULL in *out on error.
 */
/*
 * Batched products with their results drained to host memory while later
 * products run: the overlap of host-side result handling with the products
 * still in progress (Sections 4 and 6.3).  Products are taken in index order
 * in waves; a wave is the longest run of consecutive products whose planned
 * workspace and bound-sized device results fit half of `device_buffer`
 * (device memory, 256-byte aligned; the two halves alternate between waves)
 * and whose bound-sized results (16 bytes per term) fit `host_buffer` (host
 * memory of host_bytes; pinned memory from hipHostMalloc lets the copies run
 * beside the kernels, pageable memory makes them synchronous).  Each wave
 * runs as one batch (as pm_mul_batch) on `stream`; its results are copied to
 * `host_buffer` on an internal stream while the next wave's kernels run, and
 * then `fn(user, k, keys, coefs, n)` is called for each product k of the wave
 * in index order, from the calling thread, with the k-th result's n terms
 * (keys ascending, coefficients in the layout's ring).  The pointers are valid
 * only during the call.  Returns when every callback has returned; *waves
 * receives the number of waves.  PM_ENOMEM if one product alone does not fit;
 * PM_EINVAL for PM_Z192 or null / non-positive buffers; validation errors as
 * pm_mul_batch (nothing is called back then).
 */
typedef void (*pm_drain_fn)(void *user, int64_t index, const uint64_t *keys, const void *coefs, int64_t n);
int pm_mul_batch_drain(const pm_layout *layout, int64_t count, const pm_cpoly *f, const pm_cpoly *g,
                       void *device_buffer, int64_t device_bytes, void *host_buffer, int64_t host_bytes,
                       pm_drain_fn fn, void *user, void *stream, int64_t *waves);

/*
 * A prepared batch: pm_batch_prepare validates the operands, plans the batch
 * (as pm_mul_batch; workspace of the batch bound, results to h[k]), uploads
 * its descriptors and captures its kernels in a HIP graph, synchronising
 * `stream`; pm_batch_launch replays the graph on `stream` (asynchronous, no
 * validation: the operands and h must still hold what prepare saw, and a
 * replay overwrites the previous results); pm_batch_destroy frees the graph.
 * PM_EINVAL for PM_Z192, a count below 1 or null arguments.
 */
typedef struct pm_batch pm_batch;
int pm_batch_prepare(const pm_layout *layout, int64_t count, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h,
                     void *workspace, int64_t workspace_bytes, void *stream, pm_batch **out);
int pm_batch_launch(pm_batch *b, void *stream);
void pm_batch_destroy(pm_batch *b);

/*
 * Serving loop (continuous batching).  The server owns one device arena of
 * `hbm_budget_bytes`, allocated once at create, and a scheduler thread.  A
 * submitted product is admitted when its bound-sized workspace fits the free
 * part of the arena; admitted products are launched in batches on the
 * server's streams while earlier batches still run, and their memory returns
 * to the arena when they complete.  Results are identical to pm_mul's.
 *   create:  nstreams in [1, 8]; returns NULL on failure (see pm_last_error).
 *   submit:  operands and result arrays as for pm_mul (caller-owned device
 *            memory; h->capacity must be >= the bound, else PM_ECAPACITY);
 *            returns a ticket.  PM_ENOMEM if the request can never fit the
 *            arena, PM_EBUSY if the pending queue is full.
 *   poll:    *done = 1 once the result is complete and visible on the host;
 *            *status receives the request's own return code.
 *   wait:    blocks until the ticket completes.
 *   stats:   latency (submit -> completion observed by the scheduler) of all
 *            completed requests, in microseconds, up to `cap` entries, in
 *            completion order; returns the number recorded.
 *   latency: the same latency for one ticket, once it has completed (with
 *            any status): PM_EBUSY while it is still running, PM_EINVAL for
 *            an unknown ticket or a NULL pointer.
 *   destroy: waits for all outstanding work and frees the arena.
 */
typedef struct pm_server pm_server;
pm_server *pm_server_create(int64_t hbm_budget_bytes, int32_t nstreams);
int pm_server_submit(pm_server *s, const pm_layout *layout, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h,
                     uint64_t *ticket);
int pm_server_poll(pm_server *s, uint64_t ticket, int32_t *done, int32_t *status);
int pm_server_wait(pm_server *s, uint64_t ticket, int32_t *status);
int64_t pm_server_latencies(pm_server *s, double *latency_us, int64_t cap);
int pm_server_latency(pm_server *s, uint64_t ticket, double *latency_us);
void pm_server_destroy(pm_server *s);

/*
 * Host-only planning (no GPU access): the bound and workspace size that
 * pm_mul_batch_bound would return for operands with the given term counts
 * and exponent ranges.  stats holds, for each product k, 4*nvars values:
 * f's per-variable minima, f's maxima, g's minima, g's maxima.  For callers
 * that already know these ranges and want to size buffers without a
 * device round trip.  Returns PM_EOVERFLOW like pm_mul_bound.
 */
int pm_plan_from_stats(const pm_layout *layout, int64_t count, const int64_t *na, const int64_t *nb,
                       const uint64_t *stats, int64_t *max_terms, int64_t *workspace_bytes);

/*
 * Measured ceiling of the degree-box path's inner loop, for roofline
 * reporting: times (HIP events on `stream`, which it synchronises) a kernel
 * that does, per term pair, the work of the dense tile step (operand keys and
 * coefficients from LDS, one ring product, one LDS compare-and-swap into a
 * 4096-slot table at about seven pairs per monomial, one LDS atomic
 * accumulation) with no HBM traffic, on 8 workgroups per CU.  *pairs_per_second
 * receives the rate.  ring: PM_MODP61, PM_I64 or PM_MODQ64 (else PM_EINVAL).
 */
int pm_dense_ceiling(int32_t ring, double *pairs_per_second, void *stream);

/*
 * Host-only helpers of the output-key interval split (Section 5, Fig. 2;
 * Section 2's intervals), computing what the interval path's sampling and
 * splitting kernels compute on the device.  No GPU access.
 *
 * pm_ival_grid: the (l+1)^2 grid samples over an na x nb pp-matrix, sample
 *   t = r*(l+1) + c at row rows[t] = r*floor(na/l) and column cols[t] =
 *   c*floor(nb/l) + (r odd ? floor(nb/(2l)) : 0), both clamped to the matrix
 *   (l = 0: the single sample (0, 0)).  rows and cols: caller-owned host
 *   arrays of (l+1)^2 entries.  PM_EINVAL unless na, nb >= 1, 0 <= l <= 63.
 * pm_ival_splitters: for ascending packed key arrays fkeys[na], gkeys[nb]
 *   (host memory; sums must not overflow the key fields), the splitters
 *   S_0 < S_1 < ... < S_{n-1}: S_0 = fkeys[0] + gkeys[0], then the distinct
 *   grid-sample sums strictly between S_0 and the end key, then the end key
 *   fkeys[na-1] + gkeys[nb-1] + 1.  The half-open intervals [S_k, S_{k+1})
 *   hold every exponent sum fkeys[i] + gkeys[j] exactly once.  spl:
 *   caller-owned host array of (l+1)^2 + 2 entries; *nspl receives n.
 */
int pm_ival_grid(int64_t na, int64_t nb, int32_t l, int64_t *rows, int64_t *cols);
int pm_ival_splitters(const uint64_t *fkeys, int64_t na, const uint64_t *gkeys, int64_t nb, int32_t l,
                      uint64_t *spl, int64_t *nspl);

/*
 * Process-wide tuning of later calls (the autotuner's knobs):
 *   tile_cfg     -1 automatic, else 0: 32x64, 1: 64x64, 2: 128x128 term tiles
 *                (LDS tile combine and dense path)
 *   combine      sparse path: -1 automatic; 0: radix-sort term-pair indices and
 *                regenerate each product in the reduction; 1: exact rings first
 *                combine f-block x g-block tiles in LDS and sort the combined
 *                (monomial, coefficient) pairs; 2: output-key intervals (grid
 *                sample of the pp-matrix, per-interval merge in LDS, no global
 *                sort; products whose degree box has fewer than 2^32 cells);
 *                3: output-key work items (pairs counted into fine key bins,
 *                bins cut into work items of at most 8192 pairs, pair indices
 *                scattered once to their work items, each work item summed
 *                in LDS; products with fewer than 2^32 cells and pairs).
 *                Automatic selection takes 3 where it applies for the
 *                exact rings (FP64 keeps the pair-index sort unless 3 is
 *                requested).
 *   allow_dense  0: never use the degree-box path
 * Results do not depend on these settings (FP64 sums every monomial's
 * products in row-major order on every path).
 */
int pm_set_tuning(int32_t tile_cfg, int32_t combine, int32_t allow_dense);

/*
 * Radix digit schedule of later sorted calls (the autotuner's third knob):
 * -1 automatic (the autotuner's choice for the size class, else 1); 0: 8-bit
 * digits over the compressed keys' significant bits, the remainder in the
 * last pass; 1: the same number of passes with digit widths as equal as
 * possible (e.g. 8, 8, 7, 7 for 30 bits).  Results do not depend on it.
 * PM_EINVAL outside -1..1.
 */
int pm_set_radix(int32_t digits);

/*
 * Synchronises `stream`, then reports whether the last pm_mul / pm_mul_batch
 * call made by this thread hit an internal consistency check on the device
 * (a look-back wait that reached its bound, or a radix scatter position
 * outside its product's range): PM_EDEVICE if so, else PM_OK.  The workspace
 * of that call must still be allocated.  For tests and debugging.
 */
int pm_last_call_status(void *stream);

/*
 * Size facts of the last pm_mul / pm_mul_batch call on this thread, after
 * synchronising `stream`: items radix-sorted (term pairs, or combined pairs
 * after the LDS tile combine), radix passes, bytes per sort key and per sort
 * payload, and degree-box cells (dense path).  A 4-byte payload is a pair
 * index: while the launch's compressed operand keys total at most 1 MB and
 * each product's fit in 64 KB, those sorts move the index alone and
 * regenerate its key from the operands in each pass (only the last pass also
 * writes keys); otherwise keys move with the index.  An 8-byte payload is a combined coefficient moved with its key
 * in every pass.  Any pointer may be NULL.
 */
int pm_last_call_info(void *stream, int64_t *staged_pairs, int32_t *passes, int32_t *key_bytes,
                      int32_t *payload_bytes, int64_t *box_cells);

/*
 * Kernel timing.  pm_profile_enable(1) clears and starts recording a HIP
 * event pair around every kernel the library launches (on the call's own
 * stream); pm_profile_enable(0) stops.  pm_profile_read(i, ...) synchronises
 * the recorded events and returns, for the i-th distinct kernel name, the
 * name, summed duration in milliseconds and launch count; it returns the
 * number of distinct names (so i may range over [0, return value)).
 */
int pm_profile_enable(int32_t enable);
int pm_profile_read(int32_t i, char *name, int32_t name_cap, double *total_ms, int64_t *launches);

/*
 * Autotuner.  Runs h = f * g once per candidate setting (sparse path:
 * output-key work items, key intervals, pair-index sort and LDS tile combine,
 * the two radix-sorted ones
 * with both digit schedules of pm_set_radix; tile shape for the degree-box
 * path), times each with HIP events on `stream`, and remembers the fastest
 * for the product's size class (ring, path, floor(log2(term pairs))).  Later
 * calls with automatic settings (pm_set_tuning(-1, -1, ...) and
 * pm_set_radix(-1), the defaults) use the remembered choice for their
 * largest product's class.  A setting whose workspace exceeds
 * `workspace_bytes` is skipped.  *tile_cfg, *combine and *digits (each may be
 * NULL; *digits is -1 where no radix sort runs) receive the choice.  Results
 * never depend on it.  Synchronises `stream`.
 */
int pm_autotune(const pm_layout *layout, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h, void *workspace,
                int64_t workspace_bytes, void *stream, int32_t *tile_cfg, int32_t *combine, int32_t *digits);
/*
 * Keep the autotuner's choices across processes (Section 5 tunes l once, at
 * installation): pm_autotune_save writes every remembered choice to the text
 * file `path` (one line per size class: ring, path, floor(log2(term pairs)),
 * tile shape, sparse mode, digit schedule); pm_autotune_load adds the choices
 * of such a file to the remembered ones (a class already remembered takes the
 * file's choice).  Host only.  PM_EINVAL if the file cannot be written or
 * read or a line is malformed (then nothing is loaded).
 */
int pm_autotune_save(const char *path);
int pm_autotune_load(const char *path);
/* Forget every autotuner choice. */
void pm_autotune_reset(void);

/* Static message for an error code. */
const char *pm_strerror(int code);
/* Message of the last PM_EDEVICE error raised on the calling thread. */
const char *pm_last_error(void);
/* Library version string. */
const char *pm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* POLYMUL_H */
