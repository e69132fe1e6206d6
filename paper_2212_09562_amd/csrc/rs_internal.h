// Internal definitions of the MI355X RecSplit library: tree shape, hash,
// device work-queue records.  Shared by the host orchestration and the HIP
// kernels of this library only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/recsplit.h"

namespace rs {

constexpr uint32_t kMaxLeaf = RS_MAX_LEAF_SIZE;
constexpr uint32_t kMaxBucketKeys = RS_MAX_BUCKET_KEYS;
constexpr uint32_t kTable = kMaxBucketKeys + 1;  // per-size tables cover m = 0..kMaxBucketKeys
constexpr uint32_t kMaxDepth = 64;
constexpr uint32_t kMaxParts = 16;  // fanout never exceeds 9 for l <= 24
constexpr uint64_t kInf = ~0ull;
constexpr uint32_t kWG = 256;  // threads per search worker (4 wave64)
constexpr uint32_t kWaves = kWG / 64;
// Filtered leaf search: two queues of kLeafQueue attempts per wave in LDS,
// after the first kLeafQueueAt words (the leaf's keys).
constexpr uint32_t kLeafQueue = 128;
constexpr uint32_t kLeafQueueAt = 32;
constexpr uint32_t kLeafFilterWords = kLeafQueueAt + kWaves * 2 * kLeafQueue;
// Filtered split search: three such queues per wave after the node's keys
// (rounded up to 32 words).
constexpr uint32_t kSplitQueueWords = kWaves * 3 * kLeafQueue;
__host__ __device__ inline uint32_t split_queue_at(uint32_t m) { return (m + 31u) & ~31u; }

enum Kind : uint32_t { kNone = 0, kLeaf = 1, kLower = 2, kUpper = 3, kBinary = 4 };

// Splitting-tree shape (Sec. 2.2): leaf size l; lower aggregation unit
// la = l * lower fanout; upper aggregation unit ua = la * upper fanout.
struct Shape {
  uint32_t l, la, ua;
};

// Fanouts of the two levels above the leaves, max{2, ceil(0.35 l + 0.55)} and
// max{2, ceil(0.21 l + 0.9)}, evaluated exactly as ceil((35l+55)/100) and
// ceil((21l+90)/100).
inline Shape make_shape(uint32_t l) {
  uint32_t lo = (35u * l + 154u) / 100u;
  uint32_t up = (21u * l + 189u) / 100u;
  if (lo < 2) lo = 2;
  if (up < 2) up = 2;
  Shape s;
  s.l = l;
  s.la = lo * l;
  s.ua = up * s.la;
  return s;
}

__host__ __device__ inline uint32_t kind_of(const Shape& s, uint32_t m) {
  return m <= 1 ? kNone : m <= s.l ? kLeaf : m <= s.la ? kLower : m <= s.ua ? kUpper : kBinary;
}

// Children of an inner node.  Lower/upper nodes: ceil(m/unit) parts of size
// unit, the last taking the remainder.  Fanout-2 nodes: the left child gets
// the smallest multiple of ua not below floor(m/2), the right the rest.
struct Parts {
  uint32_t k;     // number of children
  uint32_t unit;  // size of every child but the last (the left size for fanout 2)
  uint32_t last;  // size of the last child
};

__host__ __device__ inline Parts parts_of(const Shape& s, uint32_t m) {
  Parts p;
  uint32_t kd = kind_of(s, m);
  if (kd == kLower || kd == kUpper) {
    uint32_t u = kd == kLower ? s.l : s.la;
    p.k = (m + u - 1) / u;
    p.unit = u;
    p.last = m - (p.k - 1) * u;
  } else if (kd == kBinary) {
    uint32_t half = m / 2;
    p.k = 2;
    p.unit = s.ua * ((half + s.ua - 1) / s.ua);
    p.last = m - p.unit;
  } else {
    p.k = 0;
    p.unit = 0;
    p.last = 0;
  }
  return p;
}

__host__ __device__ inline uint32_t part_size(const Parts& p, uint32_t j) {
  return j + 1 < p.k ? p.unit : p.last;
}

// Hash of a key word w1 under identifier x: the SplitMix64 output mixer of
// (w1 + x) mod 2^64 (Steele, Lea, Flood 2014).  Only the top 32 bits are ever
// used (positions are multiply-high reductions of them), so the device form
// returns just those.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t hash_top(uint64_t w1, uint64_t x) {
  uint64_t z = w1 + x;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  uint32_t h = (uint32_t)(z >> 32);
  return h ^ (h >> 31);
}

// floor(h * M / 2^32) for the top word h of a hash.
__device__ __forceinline__ uint32_t reduce(uint32_t h, uint32_t M) { return __umulhi(h, M); }

// Work records of the device scheduler.
struct Key {
  uint64_t w0, w1;
};

struct Task {
  uint64_t key_off;  // first key of the node in the job's work arrays
  uint64_t node;     // index of the node's value (job-relative, preorder per bucket)
  uint32_t m;        // keys in the node
  uint16_t depth;    // depth in its bucket tree (root 0)
  uint16_t job;
};

struct TaskState {
  uint64_t np;      // found bit, rounds handed out, chunks in flight (see rs_search.hip)
  uint64_t best;    // smallest valid value found so far (kInf: none)
  uint32_t closed;  // set by the one worker that finalizes the task
  uint32_t advert;  // 1 while counted in Control::long_tasks, 2 once withdrawn
  uint64_t pad;
};

// Per-job results the kernels write: largest bucket, first error, and the
// useful work of the search (hash evaluations the sequential definition
// makes), counted from the node values once the search is over.
struct JobInfo {
  uint32_t maxm;
  uint32_t error;
  uint64_t evals_split, evals_leaf, splits, leaves;
  uint64_t early_exit_leaf_fx;   // see LeafWork; in units of 2^-kLeafWorkShift evaluations
  uint64_t early_exit_split_fx;  // the same for splits (split_work_table)
  uint64_t nodes;    // stored nodes of the job (copied from its node-count scan)
  uint64_t gr_bits;  // bits of its Golomb-Rice records (copied from their scan)
  uint32_t deferred;  // some bucket was too large for the first duplicate check
  uint32_t pad;
};

// Expected hash evaluations of one failed leaf attempt of size m when the
// attempt is dropped at the first collision within a class of its keys (the
// larger class hashed first), in units of 2^-kLeafWorkShift.
constexpr uint32_t kLeafWorkShift = 12;
struct LeafWork {
  uint32_t fx[kMaxLeaf + 1];
};

struct JobDev {
  Key* keys[2];             // ping-pong key arrays: depth d reads keys[d & 1]
  JobInfo* info;
  uint64_t* vals;           // node values
  uint32_t* msz;            // node sizes
  const uint32_t* nodecnt;  // stored nodes of a subtree of size m
  const uint8_t* tau;       // Rice parameter of a node of size m
  uint32_t l, la, ua;
  uint32_t rotation;
};

// Scheduler counters, each on its own 256-byte line: every worker updates
// them with atomics and idle workers poll them, so sharing a line would make
// them contend with each other.
struct Control {
  uint64_t head;  // next queue slot to hand out
  uint64_t pad_head[31];
  uint64_t tail;  // next queue slot to fill
  uint64_t pad_tail[31];
  uint64_t finished;  // nodes whose value is final
  uint64_t pad_finished[31];
  uint64_t long_tasks;  // searches open to helpers (see TaskState::advert)
  uint64_t pad_long[31];
  uint64_t total;  // nodes of all jobs (read only during the search)
  uint32_t error;  // first RS_ERR_* seen by the search (as a positive number)
  uint32_t pad;
  // the node that raised the first error (diagnostics)
  uint64_t dbg_key_off, dbg_node, dbg_slot, dbg_np, dbg_best, dbg_chunk;
  uint32_t dbg_m, dbg_depth;
  // host-pinned word that receives the finished count at every
  // 2^kProgressShift-th node (null: progress not reported)
  uint64_t* progress;
  uint64_t pad_end[22];
};
static_assert(sizeof(Control) % 256 == 0, "Control lines");
constexpr uint32_t kProgressShift = 10;

// Rotation fitting with lookup tables (Sec. 4): for every leaf size m up to
// kRotLookupMaxM and every m-bit word x, entry (1 << m) + x holds in bits
// 0..7 the rotation t with rot_m^t(x) smallest (the first such t) and in
// bits 8..15 the period of x under rotation (m when x has no shorter one).
constexpr uint32_t kRotLookupMaxM = 16;
constexpr uint32_t kRotLookupEntries = 2u << kRotLookupMaxM;

// Whole-bucket mode: dynamic LDS of a worker = a stack of pending nodes, then
// per key its hashed word, a scratch word, its A/B class and a scratch class.
constexpr uint32_t kBucketStackBytes = 64 * 24;
constexpr uint32_t kBucketModeMaxKeys = 1152;  // largest bucket (LDS of 7 workers per CU)
constexpr uint32_t kWaveBucketSmall = 256;     // one-wave bucket workers whatever the bucket count
__host__ __device__ inline uint32_t bucket_lds_bytes(uint32_t cap) {
  return kBucketStackBytes + cap * 18u;
}
// One-wave bucket workers add, after that (8-byte aligned), the starting
// seeds (kMaxDepth words) and one job's subtree node counts (u32) and Rice
// parameters (u8) for node sizes 0..cap.
__host__ __device__ inline uint32_t wave_tables_at(uint32_t cap) {
  return (bucket_lds_bytes(cap) + 7u) & ~7u;
}
__host__ __device__ inline uint32_t wave_bucket_lds_bytes(uint32_t cap) {
  return wave_tables_at(cap) + kMaxDepth * 8u + (cap + 1u) * 5u;
}

// Search kernels: nodes as tasks; the same with staged (early-exit) leaf and
// split searches, 32-bit or 64-bit split counters; whole buckets per worker
// of four waves; whole buckets per wave.
enum : uint32_t {
  kSearchNode = 0,
  kSearchFilter = 1,
  kSearchBucket = 2,
  kSearchBucketWave = 3,
  kSearchFilterWide = 4
};

struct SearchParams {
  const JobDev* jobs;
  Task* tasks;
  TaskState* states;
  uint32_t* ready;
  int32_t* active;  // queue slot owned by each worker, -1 when none
  Control* ctl;
  const uint64_t* start;  // starting seed per depth
  uint32_t workers;
  uint32_t stage_cap;  // keys staged in LDS per worker
  uint32_t chunk_shift;   // split claims grow to 2^clamp(tau - chunk_shift, 0, 8) rounds of 256
  uint32_t help_after;    // rounds a split search hands out before helpers join
  uint32_t inline_leaf_tau;  // leaf children with tau below this skip the queue
  uint32_t mode;             // kernel: kSearchNode, kSearchFilter or kSearchBucket
  uint32_t cap_shift;    // bug guard: a node may try 2^(tau + cap_shift) attempts
  uint32_t leaf_filter_tau;  // leaves with tau at least this use the filtered search (0: none)
  uint32_t join_leaf_tau;    // leaves with tau at least this are searched in claimed chunks (0: none)
  uint32_t split_filter_tau;  // lower/upper splits with tau at least this drop attempts at an
                              // overfull child (0: never)
  uint32_t rotation_lookup;   // rotation leaves of at most kRotLookupMaxM keys find their
                              // rotation by two table lookups (0: the wave tries them all)
  uint64_t stall_ticks;  // bug guard on idle time (s_memrealtime ticks)
};

}  // namespace rs
