/*
 * dcs.h -- C ABI of the MI355X divide-and-conquer random sampler.
 *
 * Method: Sanders, Lamm, Huebschle-Schneider, Schrade, Dachsbacher,
 * "Efficient Parallel Random Sampling -- Vectorized, Cache-Efficient, and
 * Online", ACM TOMS 44(3), 2018.
 *
 * Conventions for every entry point below:
 *   - Pointers named *_dev are device (HBM) pointers on the current HIP
 *     device; the caller allocates and owns them.  The library never frees
 *     caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     work is enqueued asynchronously on it; nothing blocks the host unless
 *     the entry point says so.
 *   - Calls without a caller workspace (dcs_sample, the _ex forms with
 *     workspace == NULL, dcs_sample_part, the graph entry points) share one
 *     library workspace per device: calls on different streams must not
 *     overlap in time (give concurrent streams their own workspaces through
 *     the _ex forms, or use one stream).
 *   - Output values are 1-based (elements of 1..N) as uint64, ascending.
 *   - Return value: a dcs_status code.  Device-side failures (a capacity
 *     bound exceeded inside a kernel) cannot be returned by an asynchronous
 *     call; they are latched in an error word that the library owns, one per
 *     stream (per device), and reported by dcs_synchronize() on that stream.
 *     A caller workspace is only touched by the call it is passed to: the
 *     library keeps no pointer to it afterwards.
 *   - The sample is a pure function of (variant, n or p, N, seed, n0,
 *     dense_ratio): launch geometry, batch composition and arrival order never
 *     change a bit of it (paper Sec. 4.5, strengthened: no dependence on the
 *     number of processing elements either).
 */
#ifndef DCS_H_
#define DCS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dcs_status {
  DCS_OK = 0,
  DCS_EINVAL = 1,    /* invalid argument (see each entry point) */
  DCS_ENOMEM = 2,    /* workspace too small / device allocation failed */
  DCS_EHIP = 3,      /* a HIP runtime call failed */
  DCS_EOVERFLOW = 4, /* Bernoulli: more hits than `capacity` */
  DCS_EDEVICE = 5,   /* a kernel latched an error (reported at synchronize) */
  DCS_ENOTSUP = 6    /* request outside what the library supports */
} dcs_status;

/* Largest universe N of the recursion tree (samples without and with
 * replacement, parts, batches, served requests, segments, G(n, m)): node ids
 * and values stay below 2^63, the split's mode and exact cases are integer
 * computations; integers above 2^53 enter the deviates' doubles rounded. */
#define DCS_MAX_UNIVERSE (1ull << 62)
/* Largest universe of Bernoulli sampling and G(n, p) (chunk positions stay
 * exact in doubles). */
#define DCS_MAX_BERNOULLI_UNIVERSE (1ull << 52)

/* Canonical parameters: part of the sample's identity (changing one changes
 * the sample).  Pass NULL for the defaults. */
typedef struct dcs_params {
  uint32_t struct_size; /* sizeof(dcs_params) */
  uint32_t n0;          /* base-case threshold: a node splits iff n_v >= n0
                           (Fig. 1, "if n < n0 then return sampleBase");
                           2 <= n0 <= 4096, default 4096 */
  uint32_t dense_ratio; /* a leaf uses Algorithm B iff dense_ratio*n_v >= N_v,
                           else Algorithm H; 2..64, default 16 */
  uint32_t reserved;
} dcs_params;

/*
 * dcs_sample -- n distinct integers drawn uniformly from 1..N, ascending
 * (paper Sec. 1-2: the problem statement; Sec. 3.1 Fig. 1: Algorithm R;
 * Sec. 3.2: the node-identity hash of Algorithm P; Sec. 4.1: sorted output).
 *   out_dev: n uint64 values (8n bytes), device memory, written in full.
 * Errors: DCS_EINVAL if n > N, N > DCS_MAX_UNIVERSE, out_dev == NULL with
 * n > 0, or bad params.  n == 0 writes nothing.  Uses a per-device workspace
 * that the library grows on demand (hipMalloc; may synchronize the device).
 */
int32_t dcs_sample(uint64_t n, uint64_t N, uint64_t seed, uint64_t* out_dev, void* stream);

/* dcs_sample with explicit canonical params and an optional caller
 * workspace (workspace == NULL: the library's own).  ws_bytes must be at
 * least dcs_workspace_size(0, n, N, params); DCS_ENOMEM otherwise. */
int32_t dcs_sample_ex(uint64_t n, uint64_t N, uint64_t seed, const dcs_params* params,
                      uint64_t* out_dev, void* workspace, size_t ws_bytes, void* stream);

/*
 * dcs_sample_noalloc -- dcs_sample_ex without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, same
 * sample bit for bit as dcs_sample_ex(n, N, seed, params, out_dev, ...).
 * Its workspace is a static device array of DCS_NOALLOC_SCRATCH_BYTES per
 * device, created when the library is loaded and held until the process
 * ends; the call makes no hipMalloc / hipFree and no allocating library
 * call.  Every call on a device shares that device's array (each call
 * clears what must start at zero), so calls on one device that overlap in
 * time race: enqueue them on one stream, or wait for one before the next.
 * Errors: those of dcs_sample_ex, and DCS_ENOMEM (nothing enqueued) when
 * the call needs more than DCS_NOALLOC_SCRATCH_BYTES, i.e. when
 * dcs_workspace_size(0, n, N, 0, params) exceeds it (with the committed
 * tuning table n = 2^28 of N = 2^40 needs about 47 MiB and fits, while any
 * n from 2^25 up at N = 2^48 needs over 200 MiB and does not).
 */
#define DCS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int32_t dcs_sample_noalloc(uint64_t n, uint64_t N, uint64_t seed, const dcs_params* params,
                           uint64_t* out_dev, void* stream);

/*
 * dcs_sample_replacement -- n integers drawn independently and uniformly
 * from 1..N, sorted non-decreasing, repeats kept (Sec. 4.6: Algorithm R with
 * a binomial instead of a hypergeometric split).
 * Errors: DCS_EINVAL if N == 0 with n > 0, N > DCS_MAX_UNIVERSE, NULL out.
 */
int32_t dcs_sample_replacement(uint64_t n, uint64_t N, uint64_t seed, uint64_t* out_dev,
                               void* stream);
int32_t dcs_sample_replacement_ex(uint64_t n, uint64_t N, uint64_t seed,
                                  const dcs_params* params, uint64_t* out_dev, void* workspace,
                                  size_t ws_bytes, void* stream);

/*
 * dcs_sample_bernoulli -- each element of 1..N is kept independently with
 * probability p; the kept elements ascending (Sec. 4.7: Bernoulli sampling
 * applied independently to fixed subranges -- chunks of
 * 2^floor(log2(n0/p)) elements clamped to [2^12, 2^32] -- each by
 * geometric skips and prefix sums).
 *   out_dev:   capacity uint64 slots; the first min(count, capacity) values
 *              are written.
 *   count_dev: one uint64 in device memory, receives the true count.
 * Errors: DCS_EINVAL if p is NaN or outside [0,1], N > DCS_MAX_BERNOULLI_UNIVERSE, or
 * a NULL pointer where one is needed.  A count above `capacity` is not an
 * error of the call (it cannot be known when the call returns): compare
 * *count_dev with capacity after synchronizing; re-running with a larger
 * buffer gives the identical sample.
 * Concurrency: the chunks' output offsets come from a decoupled look-back in
 * which a chunk waits for its predecessors' counts.  A wave that has polled
 * a silent predecessor 4096 times (its chunk may not have a running wave,
 * for instance while another kernel on another stream holds the GPU)
 * computes that chunk's hit count itself, a function of the chunk alone,
 * and goes on; so a call completes whatever runs beside it.
 */
int32_t dcs_sample_bernoulli(double p, uint64_t N, uint64_t seed, uint64_t* out_dev,
                             uint64_t capacity, uint64_t* count_dev, void* stream);
int32_t dcs_sample_bernoulli_ex(double p, uint64_t N, uint64_t seed, const dcs_params* params,
                                uint64_t* out_dev, uint64_t capacity, uint64_t* count_dev,
                                void* workspace, size_t ws_bytes, void* stream);
/*
 * dcs_sample_part -- one part of the sample that dcs_sample (variant 0) or
 * dcs_sample_replacement (variant 1) returns for (n, N, seed, params), so
 * that a sample can be produced piece by piece in sorted order with bounded
 * memory (Sec. 4.1: online sampling by splitting off subranges; Sec. 3.2:
 * every node's decisions depend only on its identity, so any part can be
 * computed on its own).  The parts are the 2^depth nodes of the recursion
 * tree at depth `depth` (node `index`, 0-based from the left, covers a
 * contiguous range of 1..N); a leaf that ends a path above that depth
 * belongs, whole, to the leftmost part below it, and the other parts below
 * it are empty.  Part 0, 1, ..., 2^depth - 1 concatenated is the full sample.
 *   out_dev:        capacity uint64 slots, device memory; the part's values,
 *                   ascending, are written from out_dev[0] if they fit.
 *   count_rank_dev: two uint64 in device memory: [0] the number of values in
 *                   the part, [1] its rank (values of the sample in the parts
 *                   before it, i.e. where the part starts in the full sample).
 * The state needed to continue a piecewise traversal is (depth, index).  If
 * the count exceeds `capacity`, nothing is written to out_dev (the count is
 * only known on the device: compare count_rank_dev[0] with capacity after
 * synchronizing; re-running with a larger buffer gives the same values).
 * Errors: DCS_EINVAL for a bad variant, the argument errors of the full
 * call, depth > DCS_MAX_PART_DEPTH, index >= 2^depth, count_rank_dev NULL,
 * or out_dev NULL with capacity > 0.  Uses the library's workspace.
 */
#define DCS_MAX_PART_DEPTH 45
int32_t dcs_sample_part(int32_t variant, uint64_t n, uint64_t N, uint64_t seed,
                        const dcs_params* params, uint32_t depth, uint64_t index,
                        uint64_t* out_dev, uint64_t capacity, uint64_t* count_rank_dev,
                        void* stream);

/*
 * dcs_online_* -- online sampling in sorted order (Sec. 4.1), as a session:
 * the sample of dcs_sample (variant 0) or dcs_sample_replacement (variant 1)
 * for (n, N, seed, params), cut into the 2^depth parts of dcs_sample_part,
 * produced in runs of consecutive parts with bounded memory.
 * dcs_online_create computes the roots of all parts at once on the device
 * (one thread per part walks the splits above it; Sec. 3.2: every split
 * depends only on its node's identity) and copies their counts and ranks
 * to the host; it synchronizes `stream` before returning.  Afterwards no
 * split above the cut is computed again: dcs_online_next samples parts
 * [first, first + count) from their roots, concatenated (their values
 * ascending) into out_dev[0 .. written), in one launch sequence on
 * `stream`, so the cost of a call follows the values it produces.
 *   counts, ranks (host, may be NULL): count values of the parts' sizes and
 *                  ranks (where each part starts in the full sample).
 *   written (host, may be NULL): the number of values of the requested
 *                  parts; known on the host, so the caller sizes the next
 *                  call without synchronizing.
 * Errors: DCS_EINVAL for the argument errors of dcs_sample_part, depth >
 * DCS_MAX_ONLINE_DEPTH, a NULL session or out_dev (with values to write),
 * or parts beyond 2^depth; DCS_ENOMEM (nothing enqueued) if the parts hold
 * more than `capacity` values.  dcs_online_next uses the library's
 * workspace (as dcs_sample does); a session holds 40 B of host memory per
 * part and no device memory.
 */
#define DCS_MAX_ONLINE_DEPTH 20
typedef struct dcs_online dcs_online; /* opaque */
int32_t dcs_online_create(int32_t variant, uint64_t n, uint64_t N, uint64_t seed,
                          const dcs_params* params, uint32_t depth, void* stream,
                          dcs_online** online);
int32_t dcs_online_counts(const dcs_online* online, uint64_t first, uint64_t count,
                          uint64_t* counts, uint64_t* ranks);
int32_t dcs_online_next(dcs_online* online, uint64_t first, uint64_t count, uint64_t* out_dev,
                        uint64_t capacity, uint64_t* written, void* stream);
int32_t dcs_online_destroy(dcs_online* online);

/*
 * dcs_sample_edges_gnm -- the edges of a uniform random graph G(n, m) on the
 * vertices 0..n_vertices-1 (Sec. 7: such a graph is a sample without
 * replacement of m of the n(n-1)/2 possible edges).  Edge index k (0-based)
 * is the pair (u, v), v < u, with k = u(u-1)/2 + v; the edges are those of
 * dcs_sample_ex(m, n(n-1)/2, seed, params) (value k+1 <-> index k), decoded
 * in place.
 *   uv_dev: 2m uint32 in device memory, 8-byte aligned: edge i is
 *           (uv_dev[2i], uv_dev[2i+1]) = (u, v), in increasing (u, v) order.
 * Errors: DCS_EINVAL if n(n-1)/2 > DCS_MAX_UNIVERSE, m > n(n-1)/2, uv_dev
 * NULL or not 8-byte aligned with m > 0, or bad params.
 */
int32_t dcs_sample_edges_gnm(uint64_t n_vertices, uint64_t m, uint64_t seed,
                             const dcs_params* params, uint32_t* uv_dev, void* stream);
/*
 * dcs_sample_edges_gnp -- the edges of a random graph G(n, p): each of the
 * n(n-1)/2 pairs independently with probability p (Sec. 7: Bernoulli
 * sampling of the possible edges), i.e. dcs_sample_bernoulli_ex over
 * 1..n(n-1)/2 decoded as for G(n, m).
 *   uv_dev:    2 * capacity uint32 (8-byte aligned); the first
 *              min(count, capacity) edges are written.
 *   count_dev: one uint64 in device memory, receives the true edge count
 *              (compare with capacity after synchronizing, as for
 *              dcs_sample_bernoulli).
 * Errors: as dcs_sample_bernoulli, plus DCS_EINVAL if n(n-1)/2 >
 * DCS_MAX_BERNOULLI_UNIVERSE or uv_dev is not 8-byte aligned.
 */
int32_t dcs_sample_edges_gnp(uint64_t n_vertices, double p, uint64_t seed,
                             const dcs_params* params, uint32_t* uv_dev, uint64_t capacity,
                             uint64_t* count_dev, void* stream);

/*
 * dcs_sample_segments -- sampling over an uneven universe (Sec. 4.3, owner
 * computes; Fig. 3): n distinct elements of the concatenation of K segments
 * of lengths[0..K-1] elements (N = their sum), ascending as elements of
 * 1..N.  The segments are the leaves of the paper's binomial tree: element
 * counts are summed bottom-up and each inner node splits its sample count
 * between its two subtrees by a hypergeometric deviate (keyed by the node);
 * segment i then samples its count of its own elements as dcs_sample_ex
 * does (Fig. 1), keyed by a seed hashed from the segment's identity.
 *   lengths:    host array of K segment sizes, read during the call only.
 *   out_dev:    n uint64 device slots: segment i's values (elements
 *               lengths[0] + ... + lengths[i-1] + 1 .. that + lengths[i])
 *               follow those of segments 0..i-1.
 *   counts_dev: NULL, or K uint64 device slots receiving each segment's
 *               number of values.
 * The sample is a pure function of (n, lengths, seed, n0, dense_ratio).
 * Errors: DCS_EINVAL if K == 0, K > DCS_MAX_SEGMENTS, lengths NULL, N >
 * DCS_MAX_UNIVERSE, n > N, out_dev NULL with n > 0, or bad params.  Uses the
 * library's workspace and a pinned host staging buffer (both grown on
 * demand; may synchronize).
 */
#define DCS_MAX_SEGMENTS (1ull << 24)
int32_t dcs_sample_segments(uint64_t n, const uint64_t* lengths, uint64_t K, uint64_t seed,
                            const dcs_params* params, uint64_t* out_dev, uint64_t* counts_dev,
                            void* stream);

/*
 * dcs_sample_wholerange -- n distinct integers of 1..N, ascending, by
 * Algorithm B over the whole range (Sec. 2; Sec. 4.7's skips and prefix
 * sums; the GPU variant of Sec. 5, with the removal of the excess hits done
 * on the device instead of on the host): a Bernoulli sample with
 * rho = min(1, (n + 8 isqrt(n) + 16)/N) by fixed chunks, repeated while it
 * holds fewer than n hits (or more than n + 16 isqrt(n) + 64), then the
 * hits whose indices are the first n' - n distinct values of a uniform
 * stream over [0, n') are removed.  A second, independent path for dense
 * samples beside dcs_sample's tree (a different sample for the same seed).
 *   out_dev: n uint64 device slots, written in full.
 * The device makes up to two attempts (both failing has probability below
 * about 1e-20); if both are rejected, dcs_synchronize reports DCS_EDEVICE.
 * Errors: DCS_EINVAL if N == 0, N > 2^32, n > N, out_dev NULL with n > 0
 * or bad params; DCS_ENOTSUP if 0 < n and rho < 2^-10 (sparse samples:
 * use dcs_sample).  Uses the library's workspace.
 */
int32_t dcs_sample_wholerange(uint64_t n, uint64_t N, uint64_t seed, const dcs_params* params,
                              uint64_t* out_dev, void* stream);

/* A capacity that the Bernoulli count exceeds with negligible probability:
 * Np + 10 sqrt(Np(1-p)) + 64. */
uint64_t dcs_bernoulli_capacity_hint(double p, uint64_t N);

/* Workspace bytes needed.  variant: 0 = without replacement (n = sample
 * size), 1 = with replacement, 2 = Bernoulli (n ignored, p given as
 * p_for_bernoulli).  Writes *bytes; DCS_EINVAL on bad arguments. */
int32_t dcs_workspace_size(int32_t variant, uint64_t n, uint64_t N, double p_for_bernoulli,
                           const dcs_params* params, size_t* bytes);

/*
 * Batched sampling: many independent instances of uneven (n, N) in one
 * launch sequence (Sec. 4.2: many atomic jobs dynamically assigned to
 * workers; Sec. 4.5: results independent of that assignment).  Instance i
 * writes its sample to out_dev + out_offset[i].  Each instance's output is
 * bit-identical to a dcs_sample_ex / dcs_sample_replacement_ex call with the
 * same (n, N, seed, n0, dense_ratio).
 */
typedef struct dcs_instance {
  uint64_t n;
  uint64_t N;
  uint64_t seed;
  uint64_t out_offset; /* in uint64 elements from out_dev */
  uint32_t variant;    /* 0 = without replacement, 1 = with replacement */
  uint32_t n0;         /* 0 = default */
  uint32_t dense_ratio;/* 0 = default */
  uint32_t reserved;
} dcs_instance;

typedef struct dcs_batch dcs_batch; /* opaque */

/* Validates and uploads the instance table (host array of `count`) and
 * sizes the batch's device workspace.  The table is copied.  Errors:
 * DCS_EINVAL for an invalid instance (its index in *bad_index if non-NULL). */
int32_t dcs_batch_create(const dcs_instance* instances, uint32_t count, dcs_batch** batch,
                         uint32_t* bad_index);
/* Enqueues the whole batch on `stream`.  use_graph != 0: the launches are
 * captured once into a hipGraph and replayed on later calls. */
int32_t dcs_batch_run(dcs_batch* batch, uint64_t* out_dev, int32_t use_graph, void* stream);
int32_t dcs_batch_destroy(dcs_batch* batch);
/* Total output elements of the batch (sum of n). */
uint64_t dcs_batch_total(const dcs_batch* batch);

/*
 * Serving: continuous batching of sampling requests (an extension of the
 * batched path; the paper's load-balancing view of many small jobs, Sec. 4.2,
 * applied to requests that arrive over time).  A server owns a device output
 * arena of `arena_bytes`; a request is admitted (first come, first served)
 * once its output footprint (8 n bytes) fits in the arena, and every request
 * admitted while earlier batches are still running joins the next batch,
 * launched on the next of `n_streams` streams, so batches overlap on the
 * device.  Each request's output equals dcs_sample_ex /
 * dcs_sample_replacement_ex with the same arguments, bit for bit, whatever
 * else shares its batch.
 *   dcs_server_create: arena_bytes > 0; max_batch >= 1 requests per batch;
 *     1 <= n_streams <= 8; auto_release != 0 frees a request's arena space
 *     as soon as it completes (its output may then be overwritten).
 *   dcs_server_submit: enqueue one request; arrival_s is the scheduled arrival
 *     time on the dcs_server_now() clock (latency is measured from it; pass a
 *     negative value for "now").  DCS_EINVAL for an invalid request or one
 *     larger than the arena.
 *   dcs_server_submit_schedule: a host thread submits requests[i] at time
 *     arrival_s[i] (open loop); returns at once.  The arrays are copied.
 *     Request i gets ticket *first_ticket + i, reserved before the call
 *     returns (it polls as queued until it arrives).  DCS_EINVAL, with
 *     nothing submitted, if any request fails dcs_server_submit's checks or
 *     another schedule is still being fed.
 *   dcs_server_poll: state 0 queued, 1 running, 2 done; out_dev (valid once
 *     done, until released) and latency_s (done only) may be NULL.
 *   dcs_server_release: frees a done request's arena space.
 *   dcs_server_drain: blocks until every submitted request is done.
 *   dcs_server_stats: completed count, samples, p50 / p99 latency (s) and the
 *     span from first arrival to last completion (s).
 */
typedef struct dcs_server dcs_server;
typedef struct dcs_request {
  uint64_t n;
  uint64_t N;
  uint64_t seed;
  uint32_t variant; /* 0 = without replacement, 1 = with replacement */
  uint32_t n0;      /* 0 = default */
} dcs_request;
typedef struct dcs_server_stats {
  uint64_t completed;
  uint64_t samples;
  double p50_s;
  double p99_s;
  double max_s;
  double span_s;
  uint64_t batches;
} dcs_server_stats;
int32_t dcs_server_create(uint64_t arena_bytes, uint32_t max_batch, uint32_t n_streams,
                          int32_t auto_release, dcs_server** server);
int32_t dcs_server_submit(dcs_server* server, const dcs_request* request, double arrival_s,
                          uint64_t* ticket);
int32_t dcs_server_submit_schedule(dcs_server* server, const dcs_request* requests,
                                   const double* arrival_s, uint64_t count, uint64_t* first_ticket);
int32_t dcs_server_poll(dcs_server* server, uint64_t ticket, int32_t* state, uint64_t** out_dev,
                        double* latency_s);
int32_t dcs_server_release(dcs_server* server, uint64_t ticket);
/* Copies a done (unreleased) request's n values to dst_dev (device memory,
 * 8 n bytes), asynchronously on `stream`. */
int32_t dcs_server_copy_out(dcs_server* server, uint64_t ticket, uint64_t* dst_dev, void* stream);
int32_t dcs_server_drain(dcs_server* server);
int32_t dcs_server_stats_read(dcs_server* server, dcs_server_stats* stats);
int32_t dcs_server_destroy(dcs_server* server);
double dcs_server_now(void);

/* Waits for `stream`, then reports and clears the errors latched by the
 * library's kernels of calls enqueued on `stream` (on the current device)
 * since the last dcs_synchronize of that stream: DCS_EDEVICE if one was
 * latched, else DCS_OK.  Calls on other streams are neither waited for nor
 * reported (the first 62 streams that launch work on a device have words of
 * their own; later ones share one word). */
int32_t dcs_synchronize(void* stream);

/*
 * Launch-geometry tuning (Sec. 4.2's load balancing is static here: the
 * geometry decides how the tree and the leaf jobs are spread over the GPU).
 * A size class is (variant: 0 without, 1 with replacement; log2_n =
 * floor(log2 n), 0..63).  cut_bias is added to the depth at which the tree
 * kernels hand subtrees to threads (2^cut threads per instance);
 * leaf_wgs_per_cu is the number of leaf work-groups per compute unit (0 =
 * the kernel's occupancy, larger values are clamped to it).  Sample calls,
 * batches and served requests take the entry of their class (a batch or a
 * served batch: the class of its total sample count for the leaf grid);
 * the DCS_CUT_BIAS and DCS_LEAF_GRID environment variables override the
 * table.  Geometry never changes a sample.  The table is per process, all
 * classes start at (0, 0); dcs_workspace_size sizes for the current table.
 * Errors: DCS_EINVAL for variant not 0/1, log2_n > 63, |cut_bias| > 16,
 * leaf_wgs_per_cu > 64 or a NULL output pointer.
 */
int32_t dcs_tune_set(int32_t variant, uint32_t log2_n, int32_t cut_bias, uint32_t leaf_wgs_per_cu);
int32_t dcs_tune_get(int32_t variant, uint32_t log2_n, int32_t* cut_bias,
                     uint32_t* leaf_wgs_per_cu);
int32_t dcs_tune_reset(void);

/*
 * Leaf-job capacity (plan of every tree call: samples, parts, batches,
 * served requests, segments, G(n, m)).  The leaf jobs of the recursion tree
 * are bounded for every outcome of its random splits (at most n, and at
 * most 2I + 1 for I internal nodes, of which at most n/n0 per level hold n0
 * or more values); a call is planned with that bound when its job records
 * take at most 48 MiB or 4x the expected-case capacity (about 1.5 n/n0
 * jobs, planned with 4 n/n0 + slack), and overflow is then impossible.
 * Otherwise it is planned with the expected-case capacity and a second
 * round on the device: a tree thread whose leaf finds the job array full is
 * marked, and after the first leaf pass the marked threads run again into
 * the emptied array (their leaves' values go to fixed places, so a leaf
 * sampled in both rounds is written twice with the same values).  Only if
 * the second round runs out of slots too does dcs_synchronize report
 * DCS_EDEVICE (the sample is incomplete); later plans in the process then
 * multiply the expected-case capacity by 4 (up to 64x), so that calling
 * again gives the sample.
 * dcs_debug_leaf_capacity -- test hook: plan every later tree call with
 * `capacity` job slots per instance (at least one more than its top-level
 * paths) and the second round; 0 restores normal planning.  *boost (if not
 * NULL) receives the current multiplier; reset_boost != 0 then sets it back
 * to 1.  DCS_EINVAL if capacity >= 2^31.
 */
int32_t dcs_debug_leaf_capacity(uint64_t capacity, int32_t reset_boost, uint32_t* boost);
/* dcs_debug_lookback_help -- test hook: a Bernoulli look-back (dcs_sample_
 * bernoulli, G(n, p)) counts a silent predecessor chunk itself after `polls`
 * polls instead of 4096 (0 restores the default; 1 makes the waiting waves
 * count nearly every predecessor they wait for).  Never changes a sample. */
int32_t dcs_debug_lookback_help(uint32_t polls);
/* dcs_debug_bernoulli_list -- test hook: double-precision Bernoulli chunks
 * (p < 2^-10, and G(n, p)) keep `words` hit positions in LDS instead of the
 * size derived from the chunk's expected hits, so that chunks with more hits
 * write the rest in their second pass; 1 to 1024 words select the one-wave
 * kernel, more the work-group kernel (0 restores the default).  Never changes
 * a sample.  DCS_EINVAL above 8256 words. */
int32_t dcs_debug_bernoulli_list(uint32_t words);
/* dcs_debug_leaf_kernels -- test hook: which specialised leaf kernels a
 * single-instance tree call (or a call of an online session, whose parts
 * are subtrees of one sample's tree) leaves out, their leaves then run in the general
 * work-group kernel: bit 0 the one-wave dense kernel, bit 1 the one-wave
 * kernel of leaves of at most 1024 values, bit 2 the one-pass kernel of
 * leaves expected to repeat.  By default (mask < 0) a call leaves out the
 * kernels whose leaves its tree cannot plausibly hold.  Never changes a
 * sample.  DCS_EINVAL for a mask above 7. */
int32_t dcs_debug_leaf_kernels(int32_t mask);
/* dcs_debug_plan -- the plan of a tree call (host only, no device work):
 * info[0] cut depth, [1] tree threads, [2] DFS stack entries per thread,
 * [3] leaf-job capacity, [4] the proven bound on leaf jobs, [5] 1 if the
 * second round is planned.  DCS_EINVAL on the argument errors of
 * dcs_sample_ex / dcs_sample_replacement_ex, a bad variant or info NULL. */
int32_t dcs_debug_plan(int32_t variant, uint64_t n, uint64_t N, const dcs_params* params,
                       uint64_t* info);

/* Human-readable name of a status code (static storage). */
const char* dcs_status_string(int32_t status);

/* Kernel timing with HIP events recorded on the stream each kernel is
 * launched on.  enable != 0 starts recording (and clears the totals).
 * dcs_profile_read: after the stream is synchronized, accumulated
 * milliseconds and launch count for kernel `kind`
 * (0 = reset, 1 = tree split, 2 = leaf stage: all leaf kernels,
 * 3 = Bernoulli chunk, 4 = leaf kernel of the sparse and with-replacement
 * jobs over power-of-two ranges,
 * 5 = work-group leaf kernel of the other jobs and of the second round's
 * jobs, 6 = one-wave-per-leaf
 * kernel of the dense jobs with ranges up to 2^16, 7 = edge-index
 * decoding of the graph entry points, 8 = the segment splits of
 * dcs_sample_segments, 9 / 10 / 11 = the count passes / the scan and
 * repair / the write passes of dcs_sample_wholerange, 12 = one-wave-per-leaf
 * kernel of the sparse and with-replacement jobs of at most 1024 values over
 * ranges that are not powers of two (and of the sparse ones over powers of
 * two that are expected to repeat), 13 = work-group kernel of the sparse jobs
 * of more than 1024 values with n_v^2 >= 2 N_v, which samples each in one
 * pass instead of repeat rounds); DCS_EINVAL for another kind. */
int32_t dcs_profile_enable(int32_t enable);
int32_t dcs_profile_read(int32_t kind, double* total_ms, uint64_t* launches);
/* Restrict the timing to the kinds whose bit is set in `mask` (bit k: kind
 * k; all kinds by default), so that a timed loop records events only around
 * the kernels it reports; always DCS_OK. */
int32_t dcs_profile_kinds(uint32_t mask);

/*
 * Diagnostics: the device primitives applied elementwise to device arrays,
 * so that tests can compare them bit for bit with an independent CPU
 * implementation.  All arrays are device memory of `count` elements; the
 * call is asynchronous on `stream`.
 *   op 0: y_f64 = ln(x_f64)            op 1: y_f64 = ln(1 + x_f64)
 *   op 2: y_f32 = ln(x_f32)            op 3: y_f64 = sqrt(x_f64)
 *   op 4: y_f64 = x_f64 / x2_f64       op 5: y_f64 = ln(a!) - ln(b!) (a = x_u64, b = x2_u64)
 *   op 6: y_u64 = Hyp(n, M, N) for node ids x_u64, params p0..p2 = n, M, N, p3 = seed
 *   op 7: y_u64 = Bin(n, l/Nv) for node ids x_u64, params p0..p2 = n, l, Nv, p3 = seed
 *   op 8: y_u32[4i..4i+3] = Philox block of counter x_u32[4i..4i+3], key (p0, p1)
 *   op 9: y_f32 = U of the geometric skip for word x_u32
 */
int32_t dcs_debug_primitive(int32_t op, const void* x_dev, const void* x2_dev, void* y_dev,
                            uint64_t count, uint64_t p0, uint64_t p1, uint64_t p2, uint64_t p3,
                            void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DCS_H_ */
