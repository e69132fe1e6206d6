/*
 * recsplit.h -- C ABI of the MI355X RecSplit construction library.
 *
 * RecSplit (Esposito et al., ALENEX 2020) as extended by Bez, Kurpicz,
 * Lehmann and Sanders, "High Performance Construction of RecSplit Based
 * Minimal Perfect Hash Functions" (arXiv 2212.09562).  A minimal perfect hash
 * function maps a set S of n keys bijectively onto [0, n); a key outside S
 * maps to some value in [0, n) or beyond, without error (Sec. 1).
 *
 * Keys are 128-bit master hash codes (Sec. 2.2: every object is first hashed
 * to a uniform fingerprint; Sec. 6 uses random 128-bit integers directly).
 * The first word selects the bucket and the leaf half A/B; the second word is
 * hashed by the splitting and bijection searches.
 *
 * Every entry point returns RS_OK (0) or a negative RS_ERR_* code and leaves
 * its out-parameters untouched (or NULL) on error.  The build runs entirely
 * in HIP kernels on the current HIP device; the library owns every rs_mphf
 * it returns and the caller owns every buffer it passes in.
 */
#ifndef RECSPLIT_H
#define RECSPLIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* w0: bucket selector (top bits) and A/B class (bit 0); w1: hashed word. */
typedef struct {
  uint64_t w0, w1;
} rs_key128;

typedef struct rs_mphf rs_mphf;

enum {
  RS_OK = 0,
  RS_PENDING = 1,           /* rs_server_poll: the request is not finished yet */
  RS_ERR_INVALID_ARG = -1,  /* leaf size, bucket size, n or a pointer out of range */
  RS_ERR_DUPLICATE = -2,    /* two keys of one bucket share w1: no bijection exists */
  RS_ERR_OOM = -3,          /* device or host allocation failed */
  RS_ERR_DEVICE = -4,       /* a HIP call failed, or the device scheduler stalled */
  RS_ERR_CORRUPT = -5,      /* serialised bytes fail validation */
  RS_ERR_SEARCH_LIMIT = -6, /* a seed search passed its bug-guard limit */
  RS_ERR_UNSUPPORTED = -7   /* a bucket holds more keys than RS_MAX_BUCKET_KEYS */
};

enum {
  RS_FLAG_ROTATION = 1u,       /* leaves use rotation fitting (Sec. 4); otherwise brute force */
  RS_FLAG_KEYS_ON_DEVICE = 2u, /* keys (and query output) are device pointers */
  RS_FLAG_KEEP_VALUES = 4u     /* keep a host copy of every node value (rs_debug_node_values) */
};

#define RS_MAX_LEAF_SIZE 24u
#define RS_MAX_BUCKET_SIZE 4096u
#define RS_MAX_BUCKET_KEYS 8192u

/*
 * Build the minimal perfect hash function of n distinct keys (Sec. 2.2:
 * bucketing, one splitting tree per bucket whose inner nodes get the
 * smallest seed that splits their keys into the prescribed part sizes and
 * whose leaves get the smallest bijection value, Sec. 4 rotation fitting,
 * Golomb-Rice and Elias-Fano encoding).
 *
 * keys:        n rs_key128, host memory, or device memory with
 *              RS_FLAG_KEYS_ON_DEVICE (read on the library's own stream,
 *              ordered after the work queued so far on the legacy default
 *              stream; work on other streams must be complete).  Read only.
 * n:           0 <= n < 2^40.
 * leaf_size:   l, 2 <= l <= 24.
 * bucket_size: b, the expected bucket size, 1 <= b <= 4096; nb = max(1, ceil(n/b)).
 * flags:       RS_FLAG_*.
 * out:         receives the new structure; release with rs_free.
 *
 * Errors: RS_ERR_INVALID_ARG, RS_ERR_DUPLICATE (some bucket holds two keys
 * with the same w1), RS_ERR_UNSUPPORTED (a bucket of more than
 * RS_MAX_BUCKET_KEYS keys), RS_ERR_OOM, RS_ERR_DEVICE, RS_ERR_SEARCH_LIMIT.
 * The result depends only on the key set, l, b and RS_FLAG_ROTATION: it is
 * identical for any key order and any launch configuration.
 *
 * With the environment variable RS_PROGRESS set to a number of seconds, a
 * build (rs_build, rs_build_batch, server launches; not rs_build_noalloc)
 * prints to stderr at that interval, while its search runs, how many tree
 * nodes of how many have their final value; searches run by the early-exit
 * kernel of leaf sizes up to 18 (about a second per million keys) print
 * nothing.  With RS_DEBUG set, a failed search prints the node that failed.
 */
int rs_build(const rs_key128 *keys, uint64_t n, uint32_t leaf_size, uint32_t bucket_size,
             uint32_t flags, rs_mphf **out);

/*
 * rs_build for callers that cannot allocate device memory: code that must not
 * call hipMalloc or hipFree (tight serving loops, harnesses that forbid
 * allocation).  The build's working memory -- staged and sorted keys, bucket
 * sizes and offsets, node values, the search's task queue, states and
 * counters, and the encoded words before they are copied out -- lies in one
 * device array of RS_NOALLOC_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends (the same array holds the
 * starting seeds and the per-leaf-size tables every entry point reads).  This
 * call makes no hipMalloc, hipFree or other device or pinned-host allocation.
 *
 * keys, n, leaf_size, bucket_size, flags: as rs_build, with
 *   n <= RS_NOALLOC_MAX_KEYS; n above it, or RS_FLAG_KEEP_VALUES, is refused
 *   with RS_ERR_INVALID_ARG before any device work.
 * words:  caller-owned host buffer of cap_words 64-bit words (cap_words >= 1)
 *         that receives the serialised structure, word for word what
 *         rs_serialize gives for rs_build of the same arguments.
 * nwords: receives the number of words written.  When the structure needs
 *         more than cap_words, nothing is written to words, *nwords receives
 *         the count needed and the call returns RS_ERR_INVALID_ARG (call
 *         again with a larger buffer; the result will be the same).
 * The array keeps the last call's contents; a call clears everything it
 * needs cleared.  Calls on one device share the array and would race, so
 * the library serialises them with a lock (a second caller waits); calls on
 * different devices, or from different processes, use different copies.
 * Other errors as rs_build; RS_ERR_OOM if the encoded words do not fit the
 * space left after the working memory (at least 8 MiB; never reached by
 * structures of 2 bits per key).
 */
#define RS_NOALLOC_MAX_KEYS (1u << 19)
#define RS_NOALLOC_SCRATCH_BYTES (128ull << 20)

int rs_build_noalloc(const rs_key128 *keys, uint64_t n, uint32_t leaf_size, uint32_t bucket_size,
                     uint32_t flags, uint64_t *words, uint64_t cap_words, uint64_t *nwords);

/*
 * Build many independent key sets at once.  Each job is what rs_build takes;
 * the buckets of all jobs are sorted job by job, then every node of every job
 * is searched by one persistent launch (one device work queue), then every
 * job is encoded.  outs[i] receives job i's structure (NULL on failure) and
 * statuses[i] its result code; a job that fails (a duplicate, an argument out
 * of range) does not affect the others, and every result is identical to
 * what rs_build makes of that job alone.  Returns RS_OK or the first non-zero
 * status.  jobs, outs and statuses have njobs entries (njobs < 65536).
 */
typedef struct {
  const rs_key128 *keys;
  uint64_t n;
  uint32_t leaf_size, bucket_size, flags;
} rs_job;

int rs_build_batch(const rs_job *jobs, uint32_t njobs, rs_mphf **outs, int *statuses);

/*
 * Construction server: continuous batching of build requests on one device
 * under a fixed HBM budget (a serving form of rs_build_batch).
 *
 * rs_server_create allocates one device pool of hbm_budget_bytes and starts
 * max_slots host threads, each with its own non-blocking HIP stream.
 * Requests queue in arrival order; a free slot takes the oldest waiting
 * requests whose combined working memory fits one free region of the pool
 * (up to max_jobs_per_launch of them; a request of 2^20 keys or more is
 * built alone, smaller ones together while their keys stay below 2^20 or,
 * when at least max_slots requests are waiting, until they reach it),
 * builds them together exactly as rs_build_batch does (one persistent
 * search launch), and frees the region.
 * Slots run concurrently, so newly arrived requests are admitted while
 * earlier ones are still on the device and their kernels overlap.  A request
 * whose own working memory exceeds the budget is refused at submission
 * (RS_ERR_OOM).  The result of every request is identical to rs_build of
 * that request alone.
 *
 * Key arrays passed to rs_server_submit (host, or device with
 * RS_FLAG_KEYS_ON_DEVICE) are read when the request is admitted and must
 * stay valid and unchanged until rs_server_poll returns its result; device
 * keys must be complete before submission (the slot's stream orders only
 * after the legacy default stream).  All entry points are thread
 * safe, except that no call may overlap rs_server_destroy, which waits for
 * the builds in progress, drops requests not yet admitted, and frees results
 * never collected.  The server runs on the device current at creation.
 */
typedef struct rs_server rs_server;

typedef struct {
  uint64_t hbm_budget_bytes;    /* device pool size, >= 1 MiB */
  uint32_t max_slots;           /* concurrent builds, 1..64 */
  uint32_t max_jobs_per_launch; /* requests per search launch, >= 1 */
  uint32_t reserve_per_cu;      /* search workgroups per compute unit that launches
                                   leave free (0: none); large launches (2^20 keys or
                                   more) run one at a time, in admission order, unless
                                   max_slots requests are waiting, and a small launch made while
                                   one runs uses only the reserve, so small requests
                                   do not wait behind large ones */
} rs_server_config;

typedef struct {
  double submit, admit, done; /* host steady-clock seconds */
  uint32_t slot;              /* slot that built the request */
  uint32_t batch_jobs;        /* requests in its launch */
} rs_request_times;

typedef struct {
  uint64_t submitted, completed, launches, keys_completed;
  uint64_t waiting, bytes_in_use, peak_bytes;
} rs_server_stats;

int rs_server_create(const rs_server_config *cfg, rs_server **out);

/* Queue one build; *ticket names it for rs_server_poll.  RS_ERR_INVALID_ARG
 * for arguments rs_build would refuse; RS_ERR_OOM when it can never fit. */
int rs_server_submit(rs_server *s, const rs_job *job, uint64_t *ticket);

/*
 * Result of a request.  With wait = 0 returns RS_PENDING while the request is
 * queued or running; otherwise (or with wait != 0, after blocking until it
 * ends) returns RS_OK, sets *status to the build's code and *out to its
 * structure (NULL when the build failed; the caller releases it with
 * rs_free), fills *times when times is not NULL, and forgets the ticket.
 * RS_ERR_INVALID_ARG for an unknown or already collected ticket; when
 * several threads poll one ticket, exactly one of them collects it and the
 * others (blocked ones included) get RS_ERR_INVALID_ARG.
 */
int rs_server_poll(rs_server *s, uint64_t ticket, int wait, rs_mphf **out, int *status,
                   rs_request_times *times);

int rs_server_get_stats(rs_server *s, rs_server_stats *st);

void rs_server_destroy(rs_server *s);

/*
 * Search schedule: how the seed search hands out attempts, never what it
 * finds (every schedule gives the same structure).  A split search is handed
 * out in chunks of rounds of 256 attempts; each worker's successive claims
 * on one search double from one round up to 2^max(0, min(8, tau -
 * chunk_shift)) rounds, tau being the node's Rice parameter (about log2 of
 * its expected attempts), so long searches take few claims and short ones
 * are not overshot.  A launch is small when it has fewer than
 * small_tasks_per_worker nodes per worker; small launches use the *_small
 * settings, others the *_large ones.
 *   chunk_shift_*:  see above (0..63)
 *   help_after_*:   rounds a split search must have handed out before idle
 *                   workers join it, >= 1
 *   inline_leaf_tau_*: a leaf child whose Rice parameter is below this is
 *                   searched by the worker that split its parent, right after
 *                   the split, instead of going through the queue (0: never)
 *   bucket_mode_max_leaf: a launch whose leaf sizes are all at most this
 *                   and whose buckets hold at most 1152 keys is run with one
 *                   worker per bucket, the whole bucket tree built in LDS,
 *                   when the buckets number at least four per four-wave
 *                   worker, or with bucket_wave also when they number at
 *                   least one per four-wave worker or hold at most 256 keys
 *                   each (0: never)
 *   stall_guard_us: a search launch in which no node finishes for this
 *                   long is stopped with RS_ERR_DEVICE (a bug guard; 0: ten
 *                   seconds)
 *   max_workers:    cap on the persistent grid (0: the occupancy limit)
 *   leaf_filter_tau: a leaf whose Rice parameter is at least this is searched
 *                   in stages that drop an attempt at the first collision
 *                   within a class of its keys (0: never)
 *   split_filter_tau: a lower or upper split search whose Rice parameter is
 *                   at least this drops an attempt once a child holds more
 *                   keys than its part size (0: never)
 *   join_leaf_tau:  in a small launch that runs the filtered searches
 *                   (leaf_filter_tau or split_filter_tau in effect for some
 *                   job), a leaf whose Rice parameter is at least this is
 *                   searched in claimed chunks, as splits are, so that idle
 *                   workers join it (0: never; other leaves have one worker)
 *   rotation_lookup: rotation-fitting leaves of at most 16 keys find the
 *                   rotation of a candidate hash function by two table
 *                   lookups (Sec. 4 "Lookup Tables") instead of the wave
 *                   testing every rotation (0: off; the filter kernel that
 *                   long searches use keeps the wave test)
 *   bucket_wave:    in whole-bucket mode, each wave builds its own bucket
 *                   trees, 64 attempts a round (1), or four waves share each
 *                   bucket, 256 attempts a round (0)
 * Process-wide; builds started afterwards use it.  rs_set_schedule(NULL)
 * restores the defaults; RS_ERR_INVALID_ARG for a value out of range.
 */
typedef struct {
  uint32_t chunk_shift_small, help_after_small, inline_leaf_tau_small;
  uint32_t chunk_shift_large, help_after_large, inline_leaf_tau_large;
  uint32_t small_tasks_per_worker;
  uint32_t bucket_mode_max_leaf;
  uint32_t stall_guard_us;
  uint32_t max_workers;
  uint32_t leaf_filter_tau;
  uint32_t join_leaf_tau;
  uint32_t split_filter_tau;
  uint32_t rotation_lookup;
  uint32_t bucket_wave;
} rs_schedule;

int rs_set_schedule(const rs_schedule *s);
int rs_get_schedule(rs_schedule *s);

/*
 * Evaluate the function on n keys (Sec. 2.2 "Query": bucket, tree descent,
 * leaf position; Sec. 4: keys of B add the rotation modulo the leaf size).
 * Runs in a HIP kernel.  keys/out are host pointers, or device pointers with
 * RS_FLAG_KEYS_ON_DEVICE.  out[i] in [0, n) for every key of the built set,
 * and the ranks of the built set are a permutation of [0, n).  Thread safe.
 */
int rs_query(const rs_mphf *f, const rs_key128 *keys, uint64_t n, uint64_t *out, uint32_t flags);

/*
 * Serialised bytes (little-endian 64-bit words): header, Elias-Fano sequence
 * of the bucket prefix sums, Elias-Fano sequence of the record bit offsets,
 * Golomb-Rice bit vector.  The representation is that of Sec. 2.2
 * "Representation": every bucket's node values in preorder, Golomb-Rice coded
 * with a Rice parameter fixed per node size, the fixed-width parts of a
 * bucket stored together and then its unary parts (Sec. 2.1 for both codes);
 * the records of all buckets in one bit vector, located through the
 * Elias-Fano coded prefix sums of bucket sizes and of record offsets (the
 * paper's one combined sequence is stored here as two sequences).  Header:
 * magic, version | rotation << 32, n, l | b << 32, nb.  Each Elias-Fano
 * section: N, U, L, lower words, upper bits, upper words, then the lower
 * bits and the upper bits.  Golomb-Rice section: bits, words, then the words.
 * *bytes stays valid until rs_free(f).
 */
int rs_serialize(const rs_mphf *f, const uint8_t **bytes, uint64_t *nbytes);

/* Rebuild a queryable structure from the bytes rs_serialize describes
 * (Sec. 2.2 "Representation"; copied).  RS_ERR_CORRUPT when the header, the
 * section sizes or the Elias-Fano sequences do not validate. */
int rs_deserialize(const uint8_t *bytes, uint64_t nbytes, rs_mphf **out);

/* Node values of one bucket in preorder, as chosen by the build (requires
 * RS_FLAG_KEEP_VALUES at build time).  *count receives the number of values;
 * RS_ERR_INVALID_ARG when cap is too small or the bucket does not exist. */
int rs_debug_node_values(const rs_mphf *f, uint64_t bucket, uint64_t *vals, uint64_t cap,
                         uint64_t *count);

/* Counters and per-stage device times (HIP events on the build's stream) of
 * the build that produced f; zero for a deserialised structure. */
typedef struct {
  uint64_t n, nb, nodes, split_nodes, leaf_nodes;
  uint64_t useful_evals_split; /* (s+1) * m per inner node */
  uint64_t useful_evals_leaf;  /* (v+1) * m per brute leaf, (floor(v/m)+1) * m per rotation leaf */
  /* leaves again, each failed attempt counted at the expected evaluations of
   * an attempt dropped at the first collision within a class of its keys
   * (the larger class first; brute force: one class), the successful one at m */
  double early_exit_evals_leaf;
  /* splits again, each failed lower or upper split attempt counted at the
   * expected evaluations of an attempt dropped once a child holds more keys
   * than its part size (rs_attempt_work), fanout-2 attempts and the
   * successful one at m */
  double early_exit_evals_split;
  uint64_t gr_bits, bytes;
  uint32_t max_bucket, workers;
  double ms_sort, ms_search, ms_encode, ms_total;
} rs_stats;

int rs_get_stats(const rs_mphf *f, rs_stats *st);

/*
 * Measurement helper for the integer roofline (not part of construction).
 * Issue rates of the VALU instruction classes a hash evaluation is made of,
 * in lane-operations per second on the current device, each measured over
 * independent dependency chains at full occupancy; and the rate of the
 * evaluation sequence itself (hash, multiply-high reduction to a position,
 * bit update: 19 VALU instructions, as in the search kernels; 16 keys in
 * registers, no memory), in hash evaluations per second, over a few
 * milliseconds and over about two seconds (the clock held under sustained
 * load).  No other side effects.
 */
typedef struct {
  double add_u32, xor_b32, mul_lo_u32, mul_hi_u32, mad_u64_u32, lshrrev_b64, lshl_add_u64,
      add3_u32;
  double hash_evals, hash_evals_sustained;
  uint32_t compute_units;
} rs_valu_rates;

int rs_calibrate_valu(rs_valu_rates *out);

/*
 * Measurement helper for the work counts (host only, no device needed):
 * expected hash evaluations of one failed attempt at a node of node_size
 * keys in a tree of leaf size leaf_size, when the attempt stops at the first
 * evidence that it fails -- a leaf (node_size <= leaf_size) at the first
 * collision within a class of its keys (flags: RS_FLAG_ROTATION for the A/B
 * classes of rotation fitting, else one class), a lower or upper split once
 * a child holds more keys than its part size, a fanout-2 split not at all
 * (node_size).  -1 for arguments out of range.
 */
double rs_attempt_work(uint32_t leaf_size, uint32_t node_size, uint32_t flags);

/*
 * Measurement and test helper (host only, no device needed): the rotation r
 * that rotation fitting finds by table lookups (Sec. 4 "Lookup Tables") for
 * the m-bit words a (hash positions of the keys of A) and b (of B): the
 * smallest r with a | rot_m^r(b) = 2^m - 1, where rot_m^r moves bit p to
 * (p + r) mod m, or m when no rotation fits.  The same tables and formula as
 * the search kernels' lookup path.  0xFFFFFFFF for m outside 2..16.
 */
uint32_t rs_rotation_lookup(uint32_t m, uint32_t a, uint32_t b);

void rs_free(rs_mphf *f);

const char *rs_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* RECSPLIT_H */
