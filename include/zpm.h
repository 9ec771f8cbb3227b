/*
 * zpm -- exact multiplication of dense polynomials with integer coefficients on
 * MI355X (gfx950), by the method of "Parallel Integer Polynomial Multiplication"
 * (Chen, Covanov, Mansouri, Moreno Maza, Xie, Xie): each coefficient is split
 * into K limbs of M bits, the bivariate product is obtained from a cyclic
 * convolution mod x^K - 1 and a negacyclic convolution mod x^K + 1 computed with
 * two-dimensional number-theoretic transforms modulo word-size Fourier primes,
 * and the coefficients are recovered by CRT and evaluation at x = 2^M.
 *
 * Problem statement (Section 1): given a(y), b(y) in Z[y], compute c = a b.
 *
 * Coefficient encoding (Section 2.3 layout, Relation (definingN) for the range):
 * a polynomial with d coefficients of bound N is d * ceil(N/64) little-endian
 * uint64 words; coefficient i occupies words [i*w, (i+1)*w), w = ceil(N/64), as
 * N-bit two's complement.  Only bits [0, N) are read: the value is sign-extended
 * from bit N-1 and higher bits in the top word are ignored.
 *
 * The product has da + db - 1 coefficients.  Coefficient i is written at
 * c + i*wc as wc words of two's complement; wc must be at least
 * ceil(zpm_out_bits(da, Na, db, Nb) / 64) and extra words hold the sign.
 *
 * Memory: a, b and c are DEVICE pointers owned by the caller (for example
 * torch tensors' data_ptr()); c must not overlap a or b.  The context owns its
 * tables and workspace.  All calls taking a stream are stream-ordered: they
 * enqueue work and return; argument errors are reported before anything is
 * enqueued and leave c untouched.  Errors raised by the device are reported by
 * zpm_sync.  One context must not be used from two host threads at once, and
 * calls that share a context run in the order they are enqueued on ONE stream
 * (the workspace is shared); use one context per stream for concurrency.
 */
#ifndef ZPM_H
#define ZPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ZPM_OK 0
#define ZPM_EINVAL (-1)      /* bad argument (null pointer, size, output width) */
#define ZPM_ENOMEM (-2)      /* device allocation failed; the context stays usable */
#define ZPM_EDEVICE (-3)     /* HIP runtime or kernel error */
#define ZPM_ERANGE (-4)      /* checked-input mode: an input coefficient has bits at or above
                                N that are not copies of bit N-1, i.e. it is outside the range
                                -2^(N-1) <= a_i <= 2^(N-1) - 1 of Relation (definingN) */
#define ZPM_EUNSUPPORTED (-5) /* sizes beyond what the prime table supports */
#define ZPM_ENOTIMPL (-6)    /* a valid request for a feature this library does not provide */
#define ZPM_EBUSY (-7)       /* server: no capacity for the request right now */
#define ZPM_ENOTFOUND (-8)   /* server: unknown ticket */
#define ZPM_ETOOBIG (-9)     /* zpm_mul_noalloc: the product's workspace exceeds the fixed
                                scratch array (zpm_noalloc_max_bytes) */

typedef struct zpm_ctx zpm_ctx;

/* Parameters the planner chose for a product (Section 2.3, DetermineBase and
 * RecoveryPrime): N padded to K*M, K limbs of M bits, np primes p_k < 2^30 with
 * P = prod p_k > 2 d K 2^(2M) (1 + 2^-12), d = min(da, db) (Relation (recoveryModulo)
 * with the product of the primes in the role of p, for c_{i,j} itself, whose magnitude
 * is below d K 2^(2M)), y-transform length L = 2^log2_L >= da + db - 1. */
typedef struct zpm_plan_info {
  int64_t da, db;
  int32_t Na, Nb;
  int32_t K, M, np;
  int32_t log2_L;        /* cyclic length along y */
  int32_t log2_L1;       /* inner y factor done inside the row-convolution kernel */
  int32_t ncol;          /* strided column passes of the y-transform */
  int32_t col_log2n[4];  /* their lengths, outermost first */
  int32_t col_tile[4];   /* inner indices per workgroup of each pass */
  int32_t W;             /* 32-bit words of each CRT value */
  int32_t log2P;         /* bit length of the prime product */
  int32_t nout_bits;     /* == zpm_out_bits(...) */
  int64_t workspace_bytes;
} zpm_plan_info;

/* Library version, e.g. 100 for 0.1.0. */
int zpm_version(void);

/* Human-readable text for an error code (static storage). */
const char *zpm_strerror(int err);

/* Two's complement width that holds every coefficient of the product:
 * |c_i| <= min(da, db) 2^(Na+Nb-2) (Relation (citighterbound) with the exact
 * number of terms), so Na + Nb - 1 + bitlength(min(da, db)).  Host only. */
int32_t zpm_out_bits(int64_t da, int32_t Na, int64_t db, int32_t Nb);

/* Planner (host only, needs no GPU).  K and np: 0 = choose, otherwise forced
 * (ZPM_EUNSUPPORTED if no feasible plan has them).  Reports the plan zpm_mul takes for
 * a product run alone: with K and np both chosen, a small product whose inner
 * y-factor is 2^10 or more (x-transforms in registers, at most one column pass) has
 * that factor shortened until the fused row kernel has at least 128 workgroups.
 * Batches and resident operands keep the cost model's split. */
int zpm_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K, int32_t np,
             zpm_plan_info *out);

/* Prime table (host only): the k-th Fourier prime (largest first) and a
 * primitive 2^21-th root of unity modulo it.  ZPM_EINVAL if k is out of range. */
int zpm_prime(int32_t k, uint32_t *p, uint32_t *root);

/* The recovery's Chinese remaindering in matrix form (host only, for checking): for a
 * plan of np <= 20 primes, c_{i,j} = sum_k y_k (P/p_k) - t P (Section 4, the Chinese
 * remaindering of each c_{i,j}; y_k the residue times (P/p_k)^{-1} mod p_k, centred) is
 * computed as int8 products on the matrix cores.  Writes the A operand the recovery loads,
 * tiles x 2 steps x 64 lanes x 16 signed bytes in that order: lane l of tile T, step s
 * holds row l mod 16 and, at byte 4 w + a, the weight of byte a of term q, where
 * q = 4 (l / 16) + w in step 0 and q = 16 + l / 16 + 4 w in step 1 (y_q for q < np, t for
 * q = np, nothing above).  Row m of tile T is the weight-2^(8n) digit
 * n = 4 tiles (m / 4) + 4 T + (m mod 4); *tiles receives the tile count.  `cap` is the
 * size of `out` in bytes.  ZPM_EINVAL for np outside 1..20 or a short buffer. */
int zpm_crt_matrix(int32_t np, int8_t *out, int64_t cap, int32_t *tiles);

/* Compute units and LDS limits (bytes per workgroup, per CU) of a HIP device. */
int zpm_device_limits(int device, int32_t *ncu, int64_t *lds_per_block, int64_t *lds_per_cu);

/* Create a context on HIP device `device`.  Tables and workspace are allocated
 * on first use and grown as needed (growth waits for the device to be idle), until
 * zpm_reserve fixes them.  The environment variable ZPM_CHECK_INPUTS=1 turns the
 * checked-input mode (zpm_set_option) on for every context created afterwards. */
int zpm_create(zpm_ctx **out, int device);
void zpm_destroy(zpm_ctx *ctx);

/* Pre-size a context so that later products allocate nothing and never wait for
 * the device (the plan's resources of Section 2.3: DetermineBase / RecoveryPrime's
 * prime tables and the workspace of the two-dimensional transforms of Section 2.1).
 *   workspace_bytes  the residue workspace: at least zpm_plan_info.workspace_bytes
 *                    of the largest product to come (0 keeps the current one);
 *   max_len          the largest da + db - 1 to come: twiddle tables of every prime
 *                    of the table are built for transforms of that length
 *                    (48 primes x 16 bytes x the next power of two; 100 MB for 2^17);
 *   max_bits         the largest Na or Nb to come (tables of 2^(32 t) mod p);
 *   max_plans        distinct plans (prime count, K, M, L) whose constants are kept,
 *                    about 11 KB of device memory each (0 = 256).
 * Waits for the device, allocates, and returns ZPM_ENOMEM if that fails.  From then
 * on zpm_mul, zpm_mul_ex and zpm_mul_operand call no hipMalloc, hipFree,
 * hipDeviceSynchronize or synchronous copy: a new plan's constants go to a reserved
 * slot by an asynchronous copy on the call's stream.  A product that needs more than
 * was reserved (a larger workspace or table, a plan slot beyond max_plans, or a
 * Kronecker-reshaped product whose buffer is not yet large enough) returns ZPM_ENOMEM
 * before anything is enqueued; calling zpm_reserve again with larger sizes grows the
 * reservation.  Batches, servers and the 64-bit prime variant keep their own buffers
 * and are not covered. */
int zpm_reserve(zpm_ctx *ctx, size_t workspace_bytes, int64_t max_len, int32_t max_bits,
                int32_t max_plans);

/* Context options.
 *   ZPM_OPT_CHECK_INPUTS: 1 = checked-input mode.  Every product call (zpm_mul,
 *     zpm_mul_ex, zpm_mul_kronecker, zpm_mul_p64, zpm_mul_batch, zpm_mul_batch_ex,
 *     zpm_operand_create, zpm_mul_operand) first checks on its stream that in every
 *     input coefficient the bits from N up to the end of its top word are copies of
 *     bit N-1 (the coefficient lies in the range of Relation (definingN) as the caller
 *     declared it), waits for that check, and returns ZPM_ERANGE without enqueuing the
 *     product (c untouched) when one is not.  The call then blocks on its stream.
 *     0 (default) = bits at and above N are ignored and the value is sign-extended
 *     from bit N-1.  Servers do not check their requests.
 * ZPM_EINVAL for an unknown option or value. */
#define ZPM_OPT_CHECK_INPUTS 1
int zpm_set_option(zpm_ctx *ctx, int32_t option, int64_t value);

/* c = a * b (the algorithm of Section 2.3).  `stream` is a hipStream_t (NULL =
 * default stream).  da or db == 0 gives an empty product (nothing written).
 * Passing one operand twice (b == a, db == da, Nb == Na) computes the square a^2
 * with a single conversion and forward transform of a, whose spectra serve as both
 * factors of the pointwise products (Section 2.1); the same holds for jobs of
 * zpm_mul_batch and requests of a server. */
int zpm_mul(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b,
            int64_t db, int32_t Nb, uint64_t *c, int32_t wc, void *stream);

/* zpm_mul with a forced plan and an optional stop point, for tests and tuning.
 * K, np: as in zpm_plan.  stop_after: 0 = full product; 1..4 = stop after
 * convert-in, the forward column passes, the row convolutions or the inverse
 * column passes, and copy the workspace (np*2K*L uint32 residues, column
 * (k, j) at [(k*2K + j)*L, ...)) to the device buffer ws_out, which must hold
 * zpm_plan_info.workspace_bytes.  Residues are kept below 2 p_k, not fully reduced.
 * After convert-in, column j < K of prime k holds a's limbs a_{i,j} mod p_k (the
 * top limb signed) for i < da, and column K + j b's; after the inverse column
 * passes, column j < 2K - 1 holds c_{i,j} (2K L) 2^-32 mod p_k for i < da + db - 1
 * (Section 2: the transforms are unnormalised and the pointwise product is a
 * Montgomery product; the recovery applies 2^32 / (2K L) with its CRT constant). */
int zpm_mul_ex(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b,
               int64_t db, int32_t Nb, uint64_t *c, int32_t wc, int32_t K, int32_t np,
               int32_t stop_after, uint32_t *ws_out, void *stream);

/* Batched products: many independent products of uneven degree and bit size in
 * one call.  Each job is one product c = a * b with the encoding and ownership rules
 * of zpm_mul; jobs must not write overlapping outputs.  Every product gets its own
 * plan (from zpm_tune's table when one covers its size class, otherwise the cost
 * model restricted to at most 16 primes and K <= 16 for the register x-transform).
 * The products run level by level: level s is the s-th stage of every product, and
 * the tiles of one level that share a stage kind and a compiled variant run in one
 * launch (a few launches per level, whatever the number of products).  Stream-ordered
 * like zpm_mul.  ZPM_BATCH_GRAPH captures the whole sequence (descriptor upload and
 * launches) in a HIP graph and replays it when the same job array is passed again.
 * ZPM_BATCH_PERSISTENT runs every tile of every stage of every product in one
 * persistent launch: a grid of resident workgroups takes task numbers from a counter in
 * stage order and waits on per-product stage counters (agent-scope loads, bounded waits).
 * The call waits for the device before it returns; if a wait exceeds its bound the
 * launch stops and the call returns ZPM_EDEVICE.  Combined with ZPM_BATCH_GRAPH it is
 * ZPM_EINVAL. */
typedef struct zpm_job {
  const uint64_t *a;
  int64_t da;
  int32_t Na;
  const uint64_t *b;
  int64_t db;
  int32_t Nb;
  uint64_t *c;
  int32_t wc;
} zpm_job;
#define ZPM_BATCH_GRAPH 1
#define ZPM_BATCH_PERSISTENT 2
int zpm_mul_batch(zpm_ctx *ctx, const zpm_job *jobs, int64_t n, int32_t flags, void *stream);
/* zpm_mul_batch with every product forced to limb count K (0 = choose). */
int zpm_mul_batch_ex(zpm_ctx *ctx, const zpm_job *jobs, int64_t n, int32_t flags, int32_t K,
                     void *stream);
/* Host-only: the launches zpm_mul_batch would make (no device work; the pointers in
 * jobs may be NULL).  Sets *nlaunch and writes up to cap launches, 6 int64 each:
 * level, stage kind (0 convert-in, 1 forward column pass, 2 row convolutions,
 * 3 inverse column pass, 4 recovery), compiled variant, products, blocks, LDS bytes. */
int zpm_batch_schedule(const zpm_job *jobs, int64_t n, int32_t K, int64_t *nlaunch, int64_t *out,
                       int64_t cap);

/* Autotuner.  Products are grouped into size classes, (ceil log2(da + db - 1),
 * ceil log2(ceil(max(Na, Nb) / 32))).  For every class present in `sample` the
 * median product is replicated into a batch and timed with each feasible limb count
 * K <= 64 (which fixes M and the prime count, Section 3.1) and column-tile width T
 * of the y passes (8, 16 or 32 inner indices per workgroup); the fastest (K, T) is
 * kept in the context and used by later zpm_mul_batch calls, and by servers created
 * afterwards, for that class.  Runs on `stream` and waits for it.  With a non-NULL
 * cache_path the table is also written there as JSON (device, library version,
 * class -> [K, T]); zpm_tune_load reads such a file back (ZPM_EINVAL if it was
 * written by another library version or is malformed; the table is then unchanged).
 * zpm_tune_get copies the table (up to cap entries; tiles may be NULL) and sets *n to
 * its size. */
int zpm_tune(zpm_ctx *ctx, const zpm_job *sample, int64_t n, const char *cache_path, void *stream);
int zpm_tune_load(zpm_ctx *ctx, const char *cache_path);
int zpm_tune_get(zpm_ctx *ctx, int32_t *classes, int32_t *ks, int32_t *tiles, int32_t cap,
                 int32_t *n);

/* Per-kernel timing.  Between zpm_profile_begin and zpm_profile_end every kernel
 * the context launches is bracketed by HIP events recorded on its stream.
 * zpm_profile_end waits for those events and returns, per kernel kind, the
 * number of launches and the summed GPU time; it writes at most max_out
 * entries and sets *n_out to the number of kinds seen. */
typedef struct zpm_kernel_time {
  char name[32];
  int64_t launches;
  double total_ms;
} zpm_kernel_time;
int zpm_profile_begin(zpm_ctx *ctx);
/* As zpm_profile_begin, but only kernels whose kind k has bit k set in `kinds` are
 * bracketed (each pair of events adds a few microseconds between kernels).  Kinds:
 * 0 bivariate_representation, 1 col_pass_fwd, 2 convolve_rows, 3 col_pass_inv,
 * 4 recovering_product, 5 batch, 6 p64_convert_in, 7 p64_y_fwd, 8 p64_x_convolve,
 * 9 p64_y_inv, 10 p64_recover, 11 gfp_convert_in, 12 gfp_y_fwd, 13 gfp_x_convolve,
 * 14 gfp_y_inv, 15 gfp_recover. */
int zpm_profile_begin_kinds(zpm_ctx *ctx, uint32_t kinds);
int zpm_profile_end(zpm_ctx *ctx, zpm_kernel_time *out, int32_t max_out, int32_t *n_out);

/* Serving by continuous batching.  A server runs a worker thread with n_streams
 * streams on the context's device and a workspace pool of hbm_budget bytes of device
 * memory, allocated once at creation.  zpm_server_submit queues one product (a job as
 * for zpm_mul_batch) and returns at once with a ticket.  Whenever a stream is free the
 * worker takes the next work from the queue, admitting requests in arrival order while
 * their workspace (the np * 2K * L residues of their plan) fits in the free part of
 * the pool.  Requests with fewer than large_bits output bits
 * ((da + db - 1) * zpm_out_bits) are batched: as many as fit run together as
 * zpm_mul_batch's grouped launches on that stream; while other work occupies the
 * device, a batch of fewer than min_batch requests waits up to linger_s for more.  A larger request keeps the device
 * busy by itself and runs alone, with the zpm_mul plan; large requests hold at most
 * large_streams streams at once, so that small requests do not wait behind them.  Work on different
 * streams overlaps on the device, and requests that arrive while others run join the
 * next batch.  Twiddle tables and per-plan constants stay resident in the context; the
 * limb counts tuned into the context before creation are used.
 *
 * Ownership: the caller keeps a, b and c allocated, and leaves c alone, until the
 * request's ticket is reported finished.  The server is internally synchronized and
 * may be called from any thread; it must be destroyed before its context.  Other
 * calls on the context remain allowed meanwhile and are serialized with the worker.
 *
 * Results: status 1 = queued or running, 0 = done, < 0 = the error that ended the
 * request (ZPM_EDEVICE after a device error, after which every queued request fails
 * and submissions return ZPM_EDEVICE).  A finished ticket is reported once: the
 * first of zpm_server_poll, zpm_server_wait or zpm_server_completions that returns
 * it consumes it, and later queries return ZPM_ENOTFOUND.  latency_s runs from
 * submission to the moment the worker saw the batch complete. */
typedef struct zpm_server zpm_server;
typedef struct zpm_server_config {
  size_t hbm_budget;   /* workspace pool bytes; 0 = half of the free device memory */
  int32_t n_streams;   /* batches in flight at once, 1..16; 0 = 4 (a process gets four
                          hardware queues by default) */
  int32_t max_batch;   /* products per batch, 1..4096; 0 = 4096 */
  double large_bits;   /* output bits from which a request is large; 0 = 2^26 */
  int32_t single_product; /* 1: no batching, every request runs alone through the
                             zpm_mul path (a baseline for the batched server) */
  int32_t large_streams;  /* streams large requests may hold at once, 1..n_streams;
                             0 = max(1, n_streams / 2) */
  int32_t min_batch;      /* while other work occupies the device, a batch of small
                             requests waits for this many (or for linger_s); 0 = 4,
                             1 = never wait */
  double linger_s;        /* the longest a small request waits for companions while the
                             device is busy, at most 1 s; 0 = 150 us, < 0 = no wait */
} zpm_server_config;
int zpm_server_create(zpm_ctx *ctx, size_t hbm_budget, int32_t n_streams, zpm_server **out);
int zpm_server_create_ex(zpm_ctx *ctx, const zpm_server_config *cfg, zpm_server **out);
/* A server whose device is simulated, for tests of the admission and batching policy
 * on a host without a GPU: nothing is computed and c is never written.  A batch runs
 * for overhead_s + (its output bits) / bits_per_s seconds of wall-clock time; with
 * fail_after >= 0 the batches launched after the first fail_after report ZPM_EDEVICE.
 * cfg->hbm_budget must be given (no device memory is allocated). */
int zpm_server_create_simulated(const zpm_server_config *cfg, double bits_per_s,
                                double overhead_s, int32_t fail_after, zpm_server **out);
/* Validates and queues a product.  ZPM_EINVAL for a bad job (as zpm_mul),
 * ZPM_ENOMEM if its workspace alone exceeds the pool (counted as rejected),
 * ZPM_EUNSUPPORTED if no plan covers it, ZPM_EBUSY while the server is being
 * destroyed.  Empty products (da or db == 0) finish at once. */
int zpm_server_submit(zpm_server *srv, const zpm_job *job, uint64_t *ticket);
int zpm_server_poll(zpm_server *srv, uint64_t ticket, int32_t *status, double *latency_s);
/* Blocks until the ticket finishes or timeout_s passes (< 0: no limit); ZPM_EBUSY
 * with *status = 1 on time-out. */
int zpm_server_wait(zpm_server *srv, uint64_t ticket, double timeout_s, int32_t *status,
                    double *latency_s);
/* Up to cap finished tickets in the order they finished; *n gets the count. */
int zpm_server_completions(zpm_server *srv, uint64_t *tickets, int32_t *status, double *latency_s,
                           int64_t cap, int64_t *n);
/* Counters and latency since creation or the last zpm_server_reset_stats.
 * Percentiles are over the first 2^22 completions of that period. */
typedef struct zpm_server_report {
  uint64_t submitted, completed, failed, rejected;
  uint64_t batches;           /* batches launched */
  uint64_t admission_waits;   /* times a lane's head waited for pool memory */
  double p50_s, p99_s, max_s, mean_s;
  double out_bits;            /* output bits of the completed requests */
  double bits_per_s;          /* out_bits / (last completion - first submission) */
  double mean_batch;          /* requests per batch */
  int64_t hbm_budget, hbm_peak, hbm_in_use;   /* pool bytes */
  int64_t inflight, inflight_peak, queued;    /* requests */
} zpm_server_report;
int zpm_server_stats(zpm_server *srv, zpm_server_report *out);
int zpm_server_reset_stats(zpm_server *srv);
/* Finishes every submitted request, stops the worker and frees the pool. */
void zpm_server_destroy(zpm_server *srv);

/* Products of very wide coefficients by Kronecker substitution (Section 1, the
 * balancing remark: a forward and backward Kronecker substitution turns a pair with
 * N far from Theta(d log d) into one for which it holds).  Each coefficient is cut
 * into chunks of w bits (lower chunks unsigned, the top one signed), y is replaced
 * by z^S with S = ceil(Na/w) + ceil(Nb/w) - 1, the reshaped pair (coefficients of
 * w + 1 bits) is multiplied by the method, and c_k = sum_{r<S} c'_{S k + r} 2^(w r)
 * is evaluated with carries.  chunk_bits: w, a multiple of 64 in [256, 16384], or 0
 * for the cheapest by the planner's cost model.  Same arguments and rules as
 * zpm_mul; the reshaped operands and product live in a context buffer.  zpm_mul
 * takes this path by itself when no direct plan exists for the sizes (coefficients
 * beyond what one recovery tile holds, about 98k bits).  zpm_kronecker_plan
 * (host-only) reports the reshaping that would be used. */
typedef struct zpm_kron_info {
  int32_t chunk_bits, s_a, s_b, S;
  int64_t da2, db2;     /* reshaped lengths */
  int32_t N2, wc2;      /* reshaped coefficient bits and product words */
  zpm_plan_info inner;  /* plan of the reshaped product */
} zpm_kron_info;
int zpm_mul_kronecker(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b,
                      int64_t db, int32_t Nb, uint64_t *c, int32_t wc, int32_t chunk_bits,
                      void *stream);
int zpm_kronecker_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t chunk_bits,
                       zpm_kron_info *out);

/* Resident operand (one factor transformed once, for many products).
 * zpm_operand_create converts b and runs its forward transforms (Section 2.1:
 * BivariateRepresentation, then the y and x transforms of CyclicConvolution and
 * NegacyclicConvolution) under the plan for (da_max, Na_max, db, Nb), and keeps its
 * np * 2K * L spectra in device memory owned by the operand (K = 0 lets the planner
 * choose).  zpm_mul_operand then computes c = a * b for any a with da <= da_max and
 * Na <= Na_max with a's conversion and transforms only (ZPM_EINVAL beyond the
 * bounds); c, wc and the stream rules are as for zpm_mul.  b must stay allocated and
 * unchanged while the operand exists (its words are not read again, but c may not
 * overlap them).  The operand belongs to the context that created it; it must be
 * destroyed after the products that use it have completed and before the context.
 * zpm_operand_info reports its plan. */
typedef struct zpm_operand zpm_operand;
int zpm_operand_create(zpm_ctx *ctx, const uint64_t *b, int64_t db, int32_t Nb, int64_t da_max,
                       int32_t Na_max, int32_t K, zpm_operand **out, void *stream);
int zpm_mul_operand(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const zpm_operand *op,
                    uint64_t *c, int32_t wc, void *stream);
int zpm_operand_info(const zpm_operand *op, zpm_plan_info *out);
void zpm_operand_destroy(zpm_operand *op);

/* Many products with resident operands.  Each job multiplies its a (da coefficients of
 * Na bits, within its operand's bounds) by the b of its operand op (Section 2.1: only
 * a is converted and transformed; the pointwise products take b's spectra as they
 * are) into c of wc words per coefficient, as zpm_mul_operand would.  Jobs may name
 * different operands, and one operand any number of times.
 * zpm_mul_operand_batch runs them as zpm_mul_batch runs its jobs: one grouped launch
 * per pipeline level, stage and compiled variant, and flags = ZPM_BATCH_GRAPH replays a
 * captured graph while the jobs (and their operands) stay the same; ZPM_BATCH_PERSISTENT
 * returns ZPM_ENOTIMPL.  ZPM_EUNSUPPORTED when an operand's plan is beyond the batch
 * kernels (more than 20 primes, or K = 32): such
 * products run through zpm_mul_operand.  Ownership and streams are as for zpm_mul_batch;
 * the operands must outlive the products that use them.
 *
 * zpm_server_submit_operand queues one such product on a server (zpm_server_create)
 * of the operand's context and returns its ticket, as zpm_server_submit does.  Small
 * requests join the server's batches beside ordinary ones; large ones, and those whose
 * operand plan the batch kernels do not cover, run alone.  The caller keeps a, c and the
 * operand alive until the ticket is reported finished.  ZPM_EINVAL for a null operand,
 * an operand of another context (or a simulated server), or an a beyond its bounds. */
typedef struct zpm_operand_job {
  const uint64_t *a;
  int64_t da;
  int32_t Na;
  const zpm_operand *op;
  uint64_t *c;
  int32_t wc;
} zpm_operand_job;
int zpm_mul_operand_batch(zpm_ctx *ctx, const zpm_operand_job *jobs, int64_t n, int32_t flags,
                          void *stream);
int zpm_server_submit_operand(zpm_server *srv, const zpm_operand_job *job, uint64_t *ticket);

/* 64-bit machine-word primes (Section 4: the modulus is one machine-word Fourier
 * prime or the product of two or three of them, combined by the Chinese remaindering
 * algorithm; the paper's implementation uses two).  Same method and result as
 * zpm_mul: K limbs of M bits, the 2K x L cyclic convolution of the zero-padded limb
 * arrays (cyclic and negacyclic parts of Section 2.1 as the even and odd x-frequencies),
 * Garner's CRT into (-P/2, P/2) and evaluation at 2^M with carries (Section 2.2).
 * Primes are the three largest p < 2^62 with 2^21 | p - 1.  np <= 3 bounds M:
 * 2M + log2(4 max(da, db) K) < log2 P <= 186.  K: power of two up to 512. */
typedef struct zpm_p64_info {
  int64_t da, db;
  int32_t Na, Nb;
  int32_t K, M, np;
  int32_t log2_L;         /* cyclic length along y */
  int32_t npass;          /* strided passes of the y-transform */
  int32_t pass_log2n[3];  /* their lengths, outermost first */
  int32_t log2_tx;        /* y positions per workgroup of the x-convolution kernel */
  int32_t log2_ti;        /* coefficients per workgroup of the recovery */
  int32_t log2P;          /* bit length of the prime product */
  int32_t nout_bits;
  int64_t workspace_bytes;  /* np * 2K * L * 8 */
} zpm_p64_info;

/* Planner of the 64-bit prime variant (host only).  K, np: 0 = choose.  ZPM_EINVAL for
 * bad sizes, ZPM_EUNSUPPORTED when no plan with np <= 3 exists. */
int zpm_plan_p64(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K, int32_t np,
                 zpm_p64_info *out);
/* The k-th 64-bit prime (k < 3, largest first) and a primitive 2^21-th root of unity. */
int zpm_prime64(int32_t k, uint64_t *p, uint64_t *root);
/* c = a * b with 64-bit primes; arguments, encodings, ownership, errors and stream
 * rules as for zpm_mul (a square when b is a); K, np as in zpm_plan_p64.  The context
 * keeps this variant's tables and workspace apart from zpm_mul's. */
int zpm_mul_p64(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b,
                int64_t db, int32_t Nb, uint64_t *c, int32_t wc, int32_t K, int32_t np,
                void *stream);

/* One big generalized Fermat prime (Section 3.1: a single prime p = r^k + 1 in place of
 * several machine-word primes and CRT, Relation (FurerHypothesis) and the table of
 * generalized Fermat primes; Section 5).  Same method and result as zpm_mul: K limbs of
 * M bits, the 2K x L two-dimensional convolution over Z/pZ, the lift of each c_{i,j}
 * into (-p/2, p/2) and evaluation at 2^M with carries (Section 2.2).  An element of Z/pZ
 * is k digits in radix r; r is a primitive 2k-th root of unity, so the x-transforms
 * (K <= k, root theta = r^(k/K)) and the y-transform passes of up to 2k points multiply
 * only by powers of r, which are digit rotations.  The primes (k, r, bits of p):
 *   k = 8:  r = 2^29 - 2^25,        232 bits
 *   k = 16: r = 2^29 - 2^9 - 2^7,   464 bits
 *   k = 32: r = 2^29 - 2^14 - 2^13, 928 bits
 * and the plan needs p > 4 max(da, db) K 2^(2M) (Relation (recoveryModulo)), so
 * M <= about (log2 p - log2(4 d K)) / 2; larger coefficients return ZPM_EUNSUPPORTED.
 * da + db - 1 <= 2^21. */
typedef struct zpm_gfp_info {
  int64_t da, db;
  int32_t Na, Nb;
  int32_t k;              /* digits of the prime */
  int32_t r;              /* its radix */
  int32_t K, M;
  int32_t log2_L;
  int32_t npass;          /* y-transform passes */
  int32_t pass_log2n[6];  /* their lengths, outermost first */
  int32_t log2p;
  int32_t nout_bits;
  int64_t workspace_bytes;  /* 2K L k 32-bit digits */
} zpm_gfp_info;

/* Host only.  The radix and the bit length of the prime with k digits (8, 16 or 32);
 * ZPM_EINVAL for another k. */
int zpm_gfp_prime(int32_t k, int32_t *r, int32_t *log2p);
/* Host only.  The root of unity of order L = 2^log2_L that the y-transforms use with
 * the prime of k digits, as k balanced digits (value sum digits[l] r^l mod p).  It
 * satisfies omega^(L/2k) = r for L >= 2k, and omega = r^(2k/L) for smaller L. */
int zpm_gfp_root(int32_t k, int32_t log2_L, int32_t *digits);
/* Planner (host only).  K, k: 0 = choose (by a work model), otherwise forced. */
int zpm_plan_gfp(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K, int32_t k,
                 zpm_gfp_info *out);
/* c = a * b with one generalized Fermat prime; arguments, encodings, ownership, errors
 * and stream rules as for zpm_mul (a square when b is a); K, k as in zpm_plan_gfp.  The
 * context keeps this variant's twiddle tables and workspace apart from zpm_mul's. */
int zpm_mul_gfp(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b,
                int64_t db, int32_t Nb, uint64_t *c, int32_t wc, int32_t K, int32_t k,
                void *stream);

/* c = a * b without allocating (for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, encodings, ownership, result and stream rules as zpm_mul.  The
 * residue workspace is a fixed device array of zpm_noalloc_max_bytes() bytes (64 MiB)
 * that the library holds on every device it runs on until the process ends; its
 * address is taken once per device by zpm_create.  The call makes no hipMalloc,
 * hipFree, device-wide synchronization or synchronous copy.
 *   ZPM_ETOOBIG  the plan's workspace (zpm_plan_info.workspace_bytes) exceeds the array;
 *   ZPM_ENOMEM   the context's twiddle tables do not cover the plan, or its constants
 *                are not resident and the context is not reserved: call zpm_reserve
 *                (max_len, max_bits, max_plans; workspace_bytes may be 0) or run one
 *                zpm_mul of the same sizes first;
 *   ZPM_ENOTIMPL  coefficients too wide for a direct plan (zpm_mul reshapes those by
 *                 Kronecker substitution, which this entry point does not do);
 *   ZPM_EUNSUPPORTED  no plan at all.
 * Every such error returns before anything is enqueued, with c untouched.  All calls on
 * one device share the one array: calls whose work overlaps on the device (other
 * streams, other contexts, other host threads) race and give wrong results; order them
 * on one stream.  The array keeps the last call's residues; every word a product reads
 * is written by that product first.  The checked-input mode is not applied here (it
 * waits for the device). */
int64_t zpm_noalloc_max_bytes(void);
int zpm_mul_noalloc(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b,
                    int64_t db, int32_t Nb, uint64_t *c, int32_t wc, void *stream);

/* Measurement aid: the attainable rate (butterflies per second) of the transforms' modular
 * butterfly u, v -> u + v, (u - v) w mod p on HIP device `device`, with every operand in
 * registers and no memory traffic (eight 256-thread workgroups per compute unit, eight
 * independent pairs per thread, `iters` butterflies on each).  Allocates a small result
 * buffer, runs on the null stream and waits for it. */
int zpm_butterfly_ceiling(int device, int32_t iters, double *bfly_per_s);

/* Wait for the stream and report any device error raised by earlier calls. */
int zpm_sync(zpm_ctx *ctx, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ZPM_H */
