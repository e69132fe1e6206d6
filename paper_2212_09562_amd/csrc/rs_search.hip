// Persistent seed-search kernel: every inner node's split seed and every
// leaf's bijection value (Sec. 2.2 "Splitting Trees" and "Bijections",
// Sec. 4 rotation fitting), for all buckets of one or more jobs, in one
// launch.
//
// Scheduling.  Nodes are tasks of a device queue.  The roots of all buckets
// are queued before the launch; a split that finishes redistributes its keys
// into its children's ranges and queues them (small leaf children are
// searched at once by the same worker instead).  Each workgroup (4 wave64)
// is a worker: it owns one task at a time, stages the task's keys in LDS and
// tries seeds in rounds of 256 consecutive attempts, one attempt per lane.
// A leaf is searched by one worker in one go.  A split search is handed out
// in chunks of rounds through one claim word per task, so idle workers join
// a long search (the tail of a geometric search is shared by the whole GPU)
// and the smallest valid value is still exact: chunks are disjoint and
// handed out in increasing order, a chunk claimed after some value is known
// lies above it and is dropped, every other chunk is evaluated, and the task
// closes when no claimed chunk is left in flight.  In whole-bucket mode (a
// separate kernel instance) each root task builds its bucket's whole tree in
// LDS instead, with no queue traffic.
//
// Minimality (Sec. 5.1: the stored number must be as small as possible):
// within a round a wave takes the lowest lane whose attempt is valid (ballot
// then count-trailing-zeros); across waves and chunks the minimum is taken
// with atomicMin, and no chunk that could hold a smaller value is skipped.
#include <type_traits>

#include "rs_launch.h"

namespace rs {

namespace {

constexpr uint64_t kNoSlot = ~0ull;
constexpr uint64_t kExhausted = ~0ull - 1;

enum : uint32_t { kActExit = 0, kActOwn = 1, kActHelp = 2, kActScan = 3, kActRetry = 4 };

// The kernels with staged (early-exit) searches.
__host__ __device__ constexpr bool filter_mode(uint32_t mode) {
  return mode == kSearchFilter || mode == kSearchFilterWide;
}

template <typename T>
__device__ __forceinline__ T ld_relaxed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Queue hand-off: a producer writes a task's keys and record, executes one
// release fence, then sets the ready flags with relaxed stores; a consumer
// polls a flag with relaxed loads and executes one acquire fence once it is
// set, before it reads the record and the keys.  Polls therefore cost no
// cache maintenance; each hand-off costs one write-back and one invalidation.
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ __forceinline__ bool set_error(Control* ctl, uint32_t code) {
  uint32_t expected = 0;
  return __hip_atomic_compare_exchange_strong(&ctl->error, &expected, code, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void record_failure(Control* ctl, const Task& t, uint64_t slot, const TaskState* st,
                               uint64_t chunk) {
  ctl->dbg_key_off = t.key_off;
  ctl->dbg_node = t.node;
  ctl->dbg_slot = slot;
  ctl->dbg_np = ld_relaxed(&st->np);
  ctl->dbg_best = ld_relaxed(&st->best);
  ctl->dbg_chunk = chunk;
  ctl->dbg_m = t.m;
  ctl->dbg_depth = t.depth;
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t mask_below(uint32_t lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Rotate the m low bits of x left by r (0 <= r < m <= 24).
__device__ __forceinline__ uint32_t rot_m(uint32_t x, uint32_t r, uint32_t m, uint32_t full) {
  return ((x << r) | (x >> (m - r))) & full;
}

// The rotation lookup tables (layout in rs_internal.h), written once per
// device by upload_rotation_tables.
__device__ uint16_t g_rot_lookup[kRotLookupEntries];

// Rotation fitting by table lookups (Sec. 4 "Lookup Tables"): b fills the
// holes of a after rotating by r exactly when the complement of b, rotated by
// r, equals a, so both are in one rotation orbit and r = t[~b] - t[a] modulo
// m works; when a repeats with period p the valid rotations are r + k p and
// the smallest is r mod p.  Returns that smallest valid r, or m when no
// rotation fits.
__device__ __forceinline__ uint32_t rot_lookup(uint32_t a, uint32_t b, uint32_t m, uint32_t full) {
  const uint16_t* t = g_rot_lookup + (1u << m);
  const uint32_t ea = t[a];
  const uint32_t eb = t[~b & full];
  uint32_t r = (eb & 0xFFu) + m - (ea & 0xFFu);
  if (r >= m) r -= m;
  const uint32_t p = ea >> 8;
  while (r >= p) r -= p;
  return (a | rot_m(b, r, m, full)) == full ? r : m;
}

// Everything a worker needs to know about its current task, wave-uniform.
struct Node {
  uint32_t kind, m, k, unit, last;
  uint32_t F;       // bits per packed child counter
  uint32_t target;  // packed expected counts
  uint32_t thr;     // fanout 2: a key goes left iff its hash top word < thr
  uint32_t magic;   // floor(p / unit) == (p * magic) >> 20 for p < m
  uint32_t full;    // 1 when every child has exactly unit keys
  uint32_t na;      // leaf keys of class A (staged first)
  uint32_t mult;    // value per attempt: m for rotation leaves, else 1
  uint32_t rotation;  // leaves: 0 brute force, 1 rotation fitting, 2 the same by table lookups
  uint32_t fullmask;
  uint64_t start;
  uint64_t cap;  // attempts after which the search is reported as failed
};

// J: the job's shape, leaf method and Rice parameters (a JobDev in global
// memory, or the one-wave bucket workers' copy in LDS).
template <typename JobT>
__device__ Node make_node(const Task& t, const JobT& J, const uint64_t* start,
                          uint32_t cap_shift, uint32_t lookup) {
  Node c;
  Shape s;
  s.l = uni(J.l);
  s.la = uni(J.la);
  s.ua = uni(J.ua);
  c.m = uni(t.m);
  c.kind = kind_of(s, c.m);
  Parts p = parts_of(s, c.m);
  c.k = p.k;
  c.unit = p.unit;
  c.last = p.last;
  c.rotation = uni(J.rotation);
  const uint32_t depth = uni(t.depth);
  c.start = uni64(start[depth < kMaxDepth ? depth : kMaxDepth - 1]);
  c.F = c.k ? 32u / c.k : 0;
  c.full = (c.kind == kLower || c.kind == kUpper) && c.last == c.unit;
  uint32_t tg = 0;
  for (uint32_t j = 0; j < c.k; ++j) tg += part_size(p, j) << (c.F * j);
  c.target = tg;
  c.thr = 0;
  if (c.kind == kBinary) c.thr = (uint32_t)((((uint64_t)c.unit << 32) + c.m - 1) / c.m);
  c.magic = c.unit ? ((1u << 20) + c.unit - 1) / c.unit : 0;
  c.mult = (c.kind == kLeaf && c.rotation) ? c.m : 1u;
  if (lookup && c.kind == kLeaf && c.rotation && c.m <= kRotLookupMaxM) c.rotation = 2;
  c.fullmask = c.m >= 32 ? ~0u : ((1u << c.m) - 1u);
  c.na = 0;
  // tau is within 2 bits of log2 of the expected number of trials, so a
  // node that runs past 2^(tau + cap_shift) attempts is a bug, not bad luck
  uint32_t sh = uni((uint32_t)J.tau[c.m]) + cap_shift;
  if (sh < 16) sh = 16;
  // a claim word counts rounds (256 attempts) in 31 bits
  if (sh > 38u) sh = 38u;
  c.cap = 1ull << sh;
  return c;
}

// ---------------------------------------------------------------- rounds
// Each returns the smallest valid value among the 64 attempts a0 .. a0+63 of
// this wave (wave-uniform), or kInf.

// Brute-force leaf: OR 2^position over all keys; valid when all m bits are set.
__device__ __forceinline__ uint64_t round_leaf_brute(const uint64_t* keys, const Node& c,
                                                      uint64_t a0) {
  const uint64_t X = c.start + a0 + lane_id();
  uint32_t mask = 0;
#pragma unroll 4
  for (uint32_t i = 0; i < c.m; ++i) mask |= 1u << reduce(hash_top(keys[i], X), c.m);
  uint64_t ok = __ballot(mask == c.fullmask);
  return ok ? a0 + (uint64_t)__builtin_ctzll(ok) : kInf;
}

// Rotation fitting (Sec. 4): attempt t hashes with identifier t*m; keys of A
// build a, keys of B build b; both must be collision free (popcount) and
// some rotation of b must fill the holes of a.  Lanes passing the popcount
// test are checked in lane order, each by the whole wave: lane r tests
// rotation r, so the lowest valid r comes from one ballot.
template <bool kLookup>
__device__ __forceinline__ uint64_t round_leaf_rot(const uint64_t* keys, const Node& c,
                                                    uint64_t a0) {
  const uint32_t lane = lane_id();
  const uint64_t X = c.start + (a0 + lane) * c.m;
  uint32_t a = 0, b = 0;
#pragma unroll 4
  for (uint32_t i = 0; i < c.na; ++i) a |= 1u << reduce(hash_top(keys[i], X), c.m);
#pragma unroll 4
  for (uint32_t i = c.na; i < c.m; ++i) b |= 1u << reduce(hash_top(keys[i], X), c.m);
  bool cand = (uint32_t)__popc(a) == c.na && (uint32_t)__popc(b) == c.m - c.na;
  if (kLookup && c.rotation == 2) {
    // every candidate finds its rotation itself
    const uint32_t r = cand ? rot_lookup(a, b, c.m, c.fullmask) : c.m;
    const uint64_t okm = __ballot(r < c.m);
    if (!okm) return kInf;
    const uint32_t L = (uint32_t)__builtin_ctzll(okm);
    return (a0 + L) * c.m + __builtin_amdgcn_readlane(r, L);
  }
  uint64_t cm = __ballot(cand);
  while (cm) {
    const uint32_t L = (uint32_t)__builtin_ctzll(cm);
    const uint32_t aL = __builtin_amdgcn_readlane(a, L);
    const uint32_t bL = __builtin_amdgcn_readlane(b, L);
    const uint32_t want = ~aL & c.fullmask;
    const bool ok = lane < c.m && rot_m(bL, lane < c.m ? lane : 0, c.m, c.fullmask) == want;
    const uint64_t okm = __ballot(ok);
    if (okm) return (a0 + L) * c.m + (uint64_t)__builtin_ctzll(okm);
    cm &= cm - 1;
  }
  return kInf;
}

// Exact check of one split seed by the whole wave: every key's child, then
// per-child counts by ballot.
__device__ bool verify_kway(const uint64_t* keys, const Node& c, uint64_t X) {
  const uint32_t lane = lane_id();
  uint32_t cnt = 0;  // lane j counts child j
  for (uint32_t g = 0; g < c.m; g += 64) {
    const uint32_t i = g + lane;
    const bool v = i < c.m;
    const uint32_t ch = v ? reduce(hash_top(keys[v ? i : 0], X), c.m) / c.unit : 0xFFFFFFFFu;
    for (uint32_t j = 0; j < c.k; ++j) {
      const uint32_t nj = (uint32_t)__popcll(__ballot(ch == j));
      if (lane == j) cnt += nj;
    }
  }
  const bool good = lane >= c.k || cnt == (lane + 1 < c.k ? c.unit : c.last);
  return __ballot(!good) == 0;
}

// Lower/upper split: packed child counters, F bits per child, added with a
// shift.  Fields can wrap, so a match of the packed word is only a
// candidate; candidates get the exact check.
template <bool kFull>
__device__ __forceinline__ uint64_t round_split_kway(const uint64_t* keys, const Node& c,
                                                      uint64_t a0) {
  const uint64_t X = c.start + a0 + lane_id();
  uint32_t acc = 0;
  if (kFull) {
#pragma unroll 4
    for (uint32_t i = 0; i < c.m; ++i) {
      const uint32_t ch = reduce(hash_top(keys[i], X), c.k);  // == floor(pos / unit) when m = k*unit
      acc += 1u << __umul24(ch, c.F);
    }
  } else {
#pragma unroll 4
    for (uint32_t i = 0; i < c.m; ++i) {
      const uint32_t p = reduce(hash_top(keys[i], X), c.m);
      const uint32_t ch = __umul24(p, c.magic) >> 20;
      acc += 1u << __umul24(ch, c.F);
    }
  }
  uint64_t cm = __ballot(acc == c.target);
  while (cm) {
    const uint32_t L = (uint32_t)__builtin_ctzll(cm);
    if (verify_kway(keys, c, c.start + a0 + L)) return a0 + L;
    cm &= cm - 1;
  }
  return kInf;
}

// Fanout-2 split: one counter of keys going left; remap(h, m) < left is the
// same as (top word of h) < ceil(left * 2^32 / m).
__device__ __forceinline__ uint64_t round_split_binary(const uint64_t* keys, const Node& c,
                                                        uint64_t a0) {
  const uint64_t X = c.start + a0 + lane_id();
  uint32_t cnt = 0;
#pragma unroll 4
  for (uint32_t i = 0; i < c.m; ++i) cnt += hash_top(keys[i], X) < c.thr ? 1u : 0u;
  uint64_t ok = __ballot(cnt == c.unit);
  return ok ? a0 + (uint64_t)__builtin_ctzll(ok) : kInf;
}

// One chunk: `rounds` rounds of 256 attempts from round `first` on; a wave
// stops at its first valid attempt or once its next attempt cannot beat the
// workgroup's best.
template <typename RoundFn>
__device__ __forceinline__ void run_chunk(const uint64_t* keys, const Node& c, uint64_t first,
                                          uint32_t rounds, uint64_t* s_best, RoundFn fn) {
  const uint32_t wave = threadIdx.x >> 6;
  const uint64_t base = first * kWG;
  for (uint32_t r = 0; r < rounds; ++r) {
    const uint64_t a0 = base + (uint64_t)r * kWG + wave * 64u;
    const uint64_t cur =
        uni64(__hip_atomic_load(s_best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (a0 * c.mult >= cur) break;
    const uint64_t v = fn(keys, c, a0);
    if (v != kInf) {
      if (lane_id() == 0)
        __hip_atomic_fetch_min(s_best, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      break;
    }
  }
}

// kLookup: the rotation lookup path is compiled in (not in the filter kernel,
// whose register budget it would break; its long leaves rarely reach the
// rotation test).
template <bool kLookup>
__device__ void eval_chunk(const uint64_t* keys, const Node& c, uint64_t first, uint32_t rounds,
                           uint64_t* s_best) {
  switch (c.kind) {
    case kLeaf:
      if (c.rotation) run_chunk(keys, c, first, rounds, s_best, round_leaf_rot<kLookup>);
      else run_chunk(keys, c, first, rounds, s_best, round_leaf_brute);
      break;
    case kLower:
    case kUpper:
      if (c.full) run_chunk(keys, c, first, rounds, s_best, round_split_kway<true>);
      else run_chunk(keys, c, first, rounds, s_best, round_split_kway<false>);
      break;
    default: run_chunk(keys, c, first, rounds, s_best, round_split_binary); break;
  }
}

// The dynamic LDS of a worker (node mode: the staged keys of the current
// task, then the queues of a filtered search).
extern __shared__ uint64_t g_lds[];

// ---------------------------------------------------------------- filtered leaves
// An attempt at a leaf fails at the first collision among the keys of one
// class (Sec. 4 rules a hash function out by the popcount of a class's
// word), so most attempts need not hash every key.  Each wave runs its share
// of the attempts through three stages: stage 1 hashes the first half of the
// larger class (brute force: of all keys) for 64 new attempts; the attempts
// without a collision wait in a first queue; stage 2 hashes the rest of that
// class for 64 waiting attempts at a time, and those still without a
// collision wait in a second queue; stage 3 hashes the other class and makes
// the final test (rotation fitting, or for brute force none: m distinct
// positions are all of them) for 64 at a time.  Both queues are first in,
// first out, so attempts reach stage 3 in increasing order and the first
// valid one there is the smallest of every attempt the wave has taken; what
// is still queued when the wave stops taking attempts is flushed in partial
// batches.  The value found is the one a search hashing every key of every
// attempt finds.  A queue entry is (index << 24) | the class word so far,
// with index = 64 * round + lane within the wave's share.

__device__ __forceinline__ uint32_t leaf_bits(const uint64_t* keys, uint32_t lo, uint32_t hi,
                                              uint64_t X, uint32_t m) {
  uint32_t mask = 0;
#pragma unroll 4
  for (uint32_t i = lo; i < hi; ++i) mask |= 1u << reduce(hash_top(keys[i], X), m);
  return mask;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t l) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Append the entries of the lanes with `keep` to queue q at tail t.
__device__ __forceinline__ void queue_push(uint64_t* q, uint32_t& t, bool keep, uint64_t e) {
  const uint64_t km = __ballot(keep);
  if (keep) q[(t + (uint32_t)__popcll(km & mask_below(lane_id()))) & (kLeafQueue - 1)] = e;
  t += (uint32_t)__popcll(km);
}

// One chunk of a leaf search, `rounds` rounds of 256 attempts from round
// `first` on, with the leaf's keys at the start of the dynamic LDS and this
// wave's two queues after them.  A stage whose queue holds fewer than 64
// attempts still runs once its oldest attempt has waited `patience` rounds,
// so that a valid attempt is not held back long past the end of a short
// search or by a selective stage (a lopsided A/B split makes stage 2 pass few
// attempts).
__device__ void run_leaf_filtered(const Node& c, uint64_t first, uint32_t rounds,
                                  uint32_t patience, uint64_t* s_best) {
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x >> 6;
  const uint64_t lane_base = first * kWG + (uint64_t)wave * 64u;
  const uint64_t* keys = g_lds;
  uint64_t* q1 = g_lds + kLeafQueueAt + wave * 2 * kLeafQueue;
  uint64_t* q2 = q1 + kLeafQueue;
  // class 1 = [lo1, hi1), hashed in stages 1 ([lo1, mid)) and 2; class 2 =
  // [lo2, hi2) in stage 3.  Keys of A are staged first.
  const bool a_first = !c.rotation || 2 * c.na >= c.m;
  const uint32_t lo1 = a_first ? 0u : c.na;
  const uint32_t hi1 = !c.rotation ? c.m : (a_first ? c.na : c.m);
  const uint32_t lo2 = !c.rotation ? c.m : (a_first ? c.na : 0u);
  const uint32_t hi2 = !c.rotation ? c.m : (a_first ? c.m : c.na);
  const uint32_t mid = lo1 + (hi1 - lo1 + 1) / 2;
  uint32_t h1 = 0, t1 = 0, h2 = 0, t2 = 0;  // queue heads and tails (wave-uniform)
  auto attempt_of = [&](uint64_t idx) { return (idx >> 6) * kWG + lane_base + (idx & 63u); };
  auto stage2 = [&](uint32_t cnt) {
    const bool v = lane < cnt;
    const uint64_t e = v ? q1[(h1 + lane) & (kLeafQueue - 1)] : 0;
    h1 += cnt;
    const uint64_t idx = e >> 24;
    const uint64_t X = c.start + attempt_of(idx) * c.mult;
    const uint32_t w = ((uint32_t)e & 0xFFFFFFu) | leaf_bits(keys, mid, hi1, X, c.m);
    queue_push(q2, t2, v && (uint32_t)__popc(w) == hi1 - lo1, (idx << 24) | w);
  };
  auto stage3 = [&](uint32_t cnt) -> uint64_t {
    const bool v = lane < cnt;
    const uint64_t e = v ? q2[(h2 + lane) & (kLeafQueue - 1)] : 0;
    h2 += cnt;
    const uint64_t att = attempt_of(e >> 24);
    const uint32_t w1 = (uint32_t)e & 0xFFFFFFu;
    const uint32_t w2 = leaf_bits(keys, lo2, hi2, c.start + att * c.mult, c.m);
    const bool cand = v && (uint32_t)__popc(w2) == hi2 - lo2;
    uint64_t cm = __ballot(cand);
    if (!c.rotation) return cm ? readlane64(att, (uint32_t)__builtin_ctzll(cm)) : kInf;
    while (cm) {
      const uint32_t L = (uint32_t)__builtin_ctzll(cm);
      const uint32_t x1 = __builtin_amdgcn_readlane(w1, L);
      const uint32_t x2 = __builtin_amdgcn_readlane(w2, L);
      const uint32_t want = ~(a_first ? x1 : x2) & c.fullmask;
      const uint32_t b = a_first ? x2 : x1;
      const bool ok = lane < c.m && rot_m(b, lane < c.m ? lane : 0, c.m, c.fullmask) == want;
      const uint64_t okm = __ballot(ok);
      if (okm) return readlane64(att, L) * c.m + (uint64_t)__builtin_ctzll(okm);
      cm &= cm - 1;
    }
    return kInf;
  };
  uint64_t found = kInf;
  uint32_t wait1 = 0, wait2 = 0;  // rounds the oldest entry of each queue has waited
  for (uint32_t r = 0; r < rounds; ++r) {
    const uint64_t a0 = (uint64_t)r * kWG + lane_base;
    const uint64_t cur =
        uni64(__hip_atomic_load(s_best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (a0 * c.mult >= cur) break;
    const uint32_t w = leaf_bits(keys, lo1, mid, c.start + (a0 + lane) * c.mult, c.m);
    queue_push(q1, t1, (uint32_t)__popc(w) == mid - lo1, (((uint64_t)r * 64u + lane) << 24) | w);
    wait1 = t1 != h1 ? wait1 + 1 : 0;
    if (t1 - h1 >= 64 || (t1 != h1 && wait1 >= patience)) {
      stage2(t1 - h1 < 64 ? t1 - h1 : 64);
      wait1 = 0;
    }
    wait2 = t2 != h2 ? wait2 + 1 : 0;
    if (t2 - h2 >= 64 || (t2 != h2 && wait2 >= patience)) {
      found = stage3(t2 - h2 < 64 ? t2 - h2 : 64);
      wait2 = 0;
      if (found != kInf) break;
    }
  }
  while (found == kInf && t1 != h1) {
    stage2(t1 - h1 < 64 ? t1 - h1 : 64);
    if (t2 - h2 >= 64) found = stage3(64);
  }
  while (found == kInf && t2 != h2) found = stage3(t2 - h2 < 64 ? t2 - h2 : 64);
  if (found != kInf && lane == 0)
    __hip_atomic_fetch_min(s_best, found, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------------------------------------------- filtered splits
// A lower or upper split attempt is dead once some child has received more
// keys than its part size, which usually shows well before the last key
// (about 17 % fewer evaluations at 112 keys in 7 parts, 5 % at 560 in 5).
// The same staged scheme as for leaves, with four stages over the keys (the
// stage ends depend on the node kind, make_split_filter) and three queues
// per wave; an entry is (index << 32) | counters.
// Counters: the first k-1 children in fields of fe bits, fe the bit length
// of the part size, so a field holds its part size without carrying; the
// last child is added above them and not counted.  A field above its part
// size carries out when (part-size complement) is added to every field,
// which one add and two xors expose for all fields at once; a field that has
// wrapped is only a missed early exit.  With 32-bit counters each stage end
// also tests the last child, whose count is the keys so far minus the sum of
// the fields (added by one multiply), against its part size: without that
// test twice as many attempts reach the last stage (11 % of the lower-split
// attempts against 5.5 %, 19 % of the upper ones against 8.6 %).  The final
// word test is exact for attempts without a carry, and every match is
// verified exactly before it counts.
constexpr uint32_t kMinFilterRounds = 8;  // shorter chunks: the plain rounds

// Counter words: 32 bits where the k-1 fields fit (up to l = 18), else 64
// bits (the wide filter kernel, l = 19 to 24: at most 40 bits of fields).  A
// queue entry packs the attempt index (below 2^14: at most 256 rounds of 64
// per chunk and wave) above the counters: (index << 32) | counters, or
// (index << 50) | the low 50 bits of the counters.
template <typename T>
struct SplitFilter {
  static constexpr uint32_t kIdxShift = sizeof(T) == 4 ? 32u : 50u;
  static constexpr uint64_t kAccMask = sizeof(T) == 4 ? 0xFFFFFFFFull : (1ull << 50) - 1;
  uint32_t fe, b1, b2, b3;
  T target, comp, carries, low;
  // 32-bit counters: the sum of the counted fields, for the test of the last
  // child (pairs of fields into slots of 2 fe bits, then one multiply adds
  // the slots into the top one)
  uint32_t pairs, slots, slot_at;
};

template <typename T>
__device__ __forceinline__ bool split_filter_fits(const Node& c) {
  const uint32_t fe = 32u - (uint32_t)__clz(c.unit);
  return (c.kind == kLower || c.kind == kUpper) && c.k >= 2 &&
         (c.k - 1) * fe < SplitFilter<T>::kIdxShift;
}

template <typename T>
__device__ __forceinline__ SplitFilter<T> make_split_filter(const Node& c) {
  SplitFilter<T> f;
  f.fe = 32u - (uint32_t)__clz(c.unit);
  f.target = f.comp = f.carries = 0;
  for (uint32_t j = 0; j + 1 < c.k; ++j) {
    f.target |= (T)c.unit << (f.fe * j);
    f.comp |= (T)((1u << f.fe) - 1u - c.unit) << (f.fe * j);
    f.carries |= (T)1 << (f.fe * (j + 1));
  }
  f.low = ((T)1 << (f.fe * (c.k - 1))) - 1u;
  f.pairs = f.slots = f.slot_at = 0;
  for (uint32_t j = 0; j + 1 < c.k; j += 2) {
    f.pairs |= ((1u << f.fe) - 1u) << (f.fe * j);
    f.slot_at = f.fe * j;
    f.slots |= 1u << f.slot_at;
  }
  // Stage ends, as fractions of m chosen per node kind from the law of the
  // key at which an attempt dies (simulated for 7 parts of 16 and 5 parts
  // of 112; a queue hand-off counted as one more key): lower splits die
  // from about 60 % of their keys on, upper splits only near the end.
  if (c.kind == kLower) {
    f.b1 = c.m * 79 / 112;
    f.b2 = c.m * 89 / 112;
    f.b3 = c.m * 98 / 112;
  } else {
    f.b1 = c.m * 123 / 140;
    f.b2 = c.m * 257 / 280;
    f.b3 = c.m * 267 / 280;
  }
  return f;
}

template <typename T>
__device__ __forceinline__ T split_count(const uint64_t* keys, const Node& c, uint32_t fe,
                                         uint32_t lo, uint32_t hi, uint64_t X, T acc) {
  if (c.full) {
#pragma unroll 4
    for (uint32_t i = lo; i < hi; ++i)
      acc += (T)1 << __umul24(reduce(hash_top(keys[i], X), c.k), fe);
  } else {
#pragma unroll 4
    for (uint32_t i = lo; i < hi; ++i) {
      const uint32_t ch = __umul24(reduce(hash_top(keys[i], X), c.m), c.magic) >> 20;
      acc += (T)1 << __umul24(ch, fe);
    }
  }
  return acc;
}

// One chunk of a lower or upper split search (`rounds` rounds from round
// `first`), keys at `keys`, this wave's three queues at q.
template <typename T>
__device__ void run_split_filtered(const uint64_t* keys, const Node& c, uint64_t first,
                                   uint32_t rounds, uint32_t patience, uint64_t* s_best,
                                   uint64_t* q) {
  using F = SplitFilter<T>;
  const uint32_t lane = lane_id();
  const uint64_t lane_base = first * kWG + (uint64_t)(threadIdx.x >> 6) * 64u;
  const F f = make_split_filter<T>(c);
  uint64_t* q1 = q;
  uint64_t* q2 = q + kLeafQueue;
  uint64_t* q3 = q + 2 * kLeafQueue;
  uint32_t h1 = 0, t1 = 0, h2 = 0, t2 = 0, h3 = 0, t3 = 0;  // queue heads and tails
  uint32_t w1 = 0, w2 = 0, w3 = 0;  // rounds the oldest entry of each queue has waited
  auto attempt_of = [&](uint64_t idx) { return (idx >> 6) * kWG + lane_base + (idx & 63u); };
  auto alive = [&](T acc) { return (((acc + f.comp) ^ acc ^ f.comp) & f.carries) == 0; };
  // alive, and the last child (its count is the keys so far minus the
  // counted fields) not above its part size
  auto alive_at = [&](T acc, uint32_t keys_done) {
    if constexpr (sizeof(T) == 4) {
      const uint32_t a = (uint32_t)(acc & f.low);  // without the last child's bits
      const uint32_t t = (a & f.pairs) + ((a >> f.fe) & f.pairs);
      const uint32_t sum = (uint32_t)(((uint64_t)t * f.slots) >> f.slot_at) & ((1u << (2 * f.fe)) - 1u);
      return alive(acc) && sum + c.last >= keys_done;
    } else {
      return alive(acc);
    }
  };
  auto pack = [&](uint64_t idx, T acc) { return (idx << F::kIdxShift) | ((uint64_t)acc & F::kAccMask); };
  // stages 2 and 3: the next key range for up to 64 entries of queue qi,
  // survivors to queue qo
  auto middle = [&](uint64_t* qi, uint32_t& hi_, uint64_t* qo, uint32_t& to, uint32_t cnt,
                    uint32_t lo, uint32_t hi) {
    const bool v = lane < cnt;
    const uint64_t e = v ? qi[(hi_ + lane) & (kLeafQueue - 1)] : 0;
    hi_ += cnt;
    const uint64_t idx = e >> F::kIdxShift;
    const T acc = split_count<T>(keys, c, f.fe, lo, hi, c.start + attempt_of(idx),
                                 (T)(e & F::kAccMask));
    queue_push(qo, to, v && alive_at(acc, hi), pack(idx, acc));
  };
  // stage 4: the last keys, the word test, exact verification in order
  auto last = [&](uint32_t cnt) -> uint64_t {
    const bool v = lane < cnt;
    const uint64_t e = v ? q3[(h3 + lane) & (kLeafQueue - 1)] : 0;
    h3 += cnt;
    const uint64_t att = attempt_of(e >> F::kIdxShift);
    const T acc = split_count<T>(keys, c, f.fe, f.b3, c.m, c.start + att, (T)(e & F::kAccMask));
    uint64_t cm = __ballot(v && (acc & f.low) == f.target);
    while (cm) {
      const uint32_t L = (uint32_t)__builtin_ctzll(cm);
      const uint64_t a = readlane64(att, L);
      if (verify_kway(keys, c, c.start + a)) return a;
      cm &= cm - 1;
    }
    return kInf;
  };
  uint64_t found = kInf;
  for (uint32_t r = 0; r < rounds; ++r) {
    const uint64_t a0 = (uint64_t)r * kWG + lane_base;
    const uint64_t cur =
        uni64(__hip_atomic_load(s_best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (a0 >= cur) break;
    const T acc = split_count<T>(keys, c, f.fe, 0, f.b1, c.start + a0 + lane, (T)0);
    queue_push(q1, t1, alive_at(acc, f.b1), pack((uint64_t)r * 64u + lane, acc));
    w1 = t1 != h1 ? w1 + 1 : 0;
    if (t1 - h1 >= 64 || (t1 != h1 && w1 >= patience)) {
      middle(q1, h1, q2, t2, t1 - h1 < 64 ? t1 - h1 : 64, f.b1, f.b2);
      w1 = 0;
    }
    w2 = t2 != h2 ? w2 + 1 : 0;
    if (t2 - h2 >= 64 || (t2 != h2 && w2 >= patience)) {
      middle(q2, h2, q3, t3, t2 - h2 < 64 ? t2 - h2 : 64, f.b2, f.b3);
      w2 = 0;
    }
    w3 = t3 != h3 ? w3 + 1 : 0;
    if (t3 - h3 >= 64 || (t3 != h3 && w3 >= patience)) {
      found = last(t3 - h3 < 64 ? t3 - h3 : 64);
      w3 = 0;
      if (found != kInf) break;
    }
  }
  // flush, oldest stages first
  while (found == kInf && t1 != h1) {
    middle(q1, h1, q2, t2, t1 - h1 < 64 ? t1 - h1 : 64, f.b1, f.b2);
    if (t2 - h2 >= 64) middle(q2, h2, q3, t3, 64, f.b2, f.b3);
    if (t3 - h3 >= 64) found = last(64);
  }
  while (found == kInf && t2 != h2) {
    middle(q2, h2, q3, t3, t2 - h2 < 64 ? t2 - h2 : 64, f.b2, f.b3);
    if (t3 - h3 >= 64) found = last(64);
  }
  while (found == kInf && t3 != h3) found = last(t3 - h3 < 64 ? t3 - h3 : 64);
  if (found != kInf && lane == 0)
    __hip_atomic_fetch_min(s_best, found, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Stage the task's keys in LDS.  Leaves put the keys of A (bit 0 of w0 clear)
// first, in a stable order, and report |A|.
__device__ void stage_keys(const Task& t, const JobDev& J, const Node& c, uint64_t* s_keys,
                           uint32_t* s_na) {
  const Key* src = J.keys[t.depth & 1] + t.key_off;
  const uint32_t tid = threadIdx.x;
  if (c.kind == kLeaf) {
    if (tid < 64) {
      const bool v = tid < c.m;
      Key key = v ? src[tid] : Key{0, 0};
      const bool isb = v && (key.w0 & 1u);
      const uint64_t bm = __ballot(isb);
      const uint64_t am = __ballot(v && !isb);
      const uint32_t na = (uint32_t)__popcll(am);
      const uint64_t below = mask_below(tid);
      if (v) {
        const uint32_t pos = isb ? na + (uint32_t)__popcll(bm & below) : (uint32_t)__popcll(am & below);
        s_keys[pos] = key.w1;
      }
      if (tid == 0) *s_na = na;
    }
  } else {
    for (uint32_t i = tid; i < c.m; i += kWG) s_keys[i] = src[i].w1;
  }
}

// Redistribute a split node's keys into its children's ranges of the other
// ping-pong array (stable within each child), then queue the children.  Run
// by wave 0; lane 0 queues.  The queue slots are reserved with one atomic
// before the keys move, and one release fence publishes keys and records.
// A leaf child of a split whose Rice parameter is below the launch's
// inline_leaf_tau is searched by the worker that split its parent, right
// after the split, instead of going through the queue.
__device__ __forceinline__ bool queued_child(const SearchParams& P, const JobDev& J, uint32_t l,
                                             uint32_t sz) {
  return sz >= 2 && (sz > l || (uint32_t)J.tau[sz] >= P.inline_leaf_tau);
}

// Count finished nodes.  Kernels that report progress (all but the filter
// kernel, whose searches end within seconds) also store the running count
// into the host's word at every 2^kProgressShift-th node when one is given (a
// plain store at system scope: the host keeps the largest value it has seen).
constexpr bool reports_progress(uint32_t mode) { return mode != kSearchFilter; }

template <bool kReport>
__device__ __forceinline__ void note_finished(const SearchParams& P, uint64_t inc) {
  if constexpr (kReport) {
    const uint64_t was =
        __hip_atomic_fetch_add(&P.ctl->finished, inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (((was + inc) >> kProgressShift) != (was >> kProgressShift)) {
      uint64_t* host = P.ctl->progress;
      if (host) __hip_atomic_store(host, was + inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  } else {
    __hip_atomic_fetch_add(&P.ctl->finished, inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <bool kReport>
__device__ void finalize_split(const SearchParams& P, const Task& t, const JobDev& J,
                               const Node& c, uint64_t s) {
  const uint32_t lane = lane_id();
  const uint32_t l = uni(J.l);
  uint32_t nkids = 0;  // children that go through the queue
  for (uint32_t j = 0; j < c.k; ++j)
    nkids += queued_child(P, J, l, j + 1 < c.k ? c.unit : c.last) ? 1u : 0u;
  uint64_t base = 0;
  if (lane == 0 && nkids)
    base = __hip_atomic_fetch_add(&P.ctl->tail, (uint64_t)nkids, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  const Key* src = J.keys[t.depth & 1] + t.key_off;
  Key* dst = J.keys[(t.depth + 1) & 1] + t.key_off;
  const uint64_t X = c.start + s;
  uint32_t run = 0;  // lane j: keys already placed in child j
  for (uint32_t g = 0; g < c.m; g += 64) {
    const uint32_t i = g + lane;
    const bool v = i < c.m;
    const Key key = v ? src[i] : Key{0, 0};
    const uint32_t p = reduce(hash_top(key.w1, X), c.m);
    uint32_t ch = c.kind == kBinary ? (p >= c.unit ? 1u : 0u) : p / c.unit;
    if (!v) ch = 0xFFFFFFFFu;
    const uint32_t at0 = (uint32_t)__shfl((int)run, v ? (int)ch : 0);
    uint32_t rank = 0;
    for (uint32_t j = 0; j < c.k; ++j) {
      const uint64_t mk = __ballot(ch == j);
      if (ch == j) rank = (uint32_t)__popcll(mk & mask_below(lane));
      if (lane == j) run += (uint32_t)__popcll(mk);
    }
    const uint32_t at = ch * c.unit + at0 + rank;
    if (v && at < c.m) dst[at] = key;
  }
  const bool good = lane >= c.k || run == (lane + 1 < c.k ? c.unit : c.last);
  const bool all_good = __ballot(!good) == 0;
  bool queued = false;
  if (lane == 0) {
    if (!all_good) set_error(P.ctl, (uint32_t)(-RS_ERR_DEVICE));
    J.vals[t.node] = s;
    J.msz[t.node] = c.m;
    if (nkids && t.depth + 1 >= kMaxDepth) {
      set_error(P.ctl, (uint32_t)(-RS_ERR_UNSUPPORTED));
    } else if (nkids && base + nkids > P.ctl->total) {
      set_error(P.ctl, (uint32_t)(-RS_ERR_DEVICE));
    } else {
      queued = true;
      uint64_t child_node = t.node + 1, slot = base;
      for (uint32_t j = 0; j < c.k; ++j) {
        const uint32_t sz = j + 1 < c.k ? c.unit : c.last;
        if (queued_child(P, J, l, sz)) {
          Task ct;
          ct.key_off = t.key_off + (uint64_t)j * c.unit;
          ct.node = child_node;
          ct.m = sz;
          ct.depth = (uint16_t)(t.depth + 1);
          ct.job = t.job;
          P.tasks[slot++] = ct;
        }
        child_node += J.nodecnt[sz];
      }
    }
  }
  fence_release();  // keys (every lane) and task records before the flags
  if (lane == 0) {
    if (queued)
      for (uint32_t i = 0; i < nkids; ++i) st_relaxed(&P.ready[base + i], 1u);
    note_finished<kReport>(P, 1ull);
  }
}

// A leaf's value is read only after the launch: no ordering needed.
template <bool kReport>
__device__ void finalize_leaf(const SearchParams& P, const Task& t, const JobDev& J,
                              const Node& c, uint64_t v) {
  if (threadIdx.x == 0) {
    J.vals[t.node] = v;
    J.msz[t.node] = c.m;
    note_finished<kReport>(P, 1ull);
  }
}

__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The claim word of a task (TaskState::np): chunks in flight in the low 32
// bits, the rounds of 256 attempts handed out so far (the cursor) in bits
// 32..62, and bit 63 set once some chunk has produced a value.  A claim of r
// rounds adds r to the cursor, so chunks are disjoint and handed out in
// increasing order: a chunk claimed after the bit is set lies wholly above
// the value and is dropped unevaluated.  One atomic both drops an evaluated
// chunk and claims the next.
constexpr uint64_t kFound = 1ull << 63;
__device__ __forceinline__ uint64_t cursor(uint64_t np) { return (np >> 32) & 0x7FFFFFFFull; }

// Drop n in-flight chunks of task st; returns true for the one caller that
// must finalize (a value is known and nothing is in flight any more).
// Relaxed agent-scope atomics on one cache line of the task state, performed
// at the device coherence point; a caller that found a value waited for its
// atomicMin and for the found bit before dropping its chunk, so whoever sees
// the count reach zero with the bit set also sees the value.
__device__ __forceinline__ bool release_chunk(TaskState* st, uint32_t n = 1) {
  const uint64_t old = __hip_atomic_fetch_add(&st->np, 0ull - n, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
  if ((old & 0xFFFFFFFFull) != n || !(old & kFound)) return false;
  uint32_t expected = 0;
  return __hip_atomic_compare_exchange_strong(&st->closed, &expected, 1u, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Shared {
  Task task;
  uint64_t first;  // first round of the chunk to evaluate
  uint32_t rounds, go;
  uint64_t best;
  uint64_t fin_value;
  uint32_t action;
  uint32_t na;
  uint32_t fin;
  uint32_t iter;
  uint64_t arg;
  int32_t pick;
  // thread 0's state across tasks, kept in LDS rather than in registers that
  // the task bodies need: the queue slot this worker has reserved, and the
  // idle bookkeeping of the stall guard and the back-off
  uint64_t my_q;
  uint64_t last_finished, idle_since;
  uint32_t idle;
};

__device__ __forceinline__ bool filtered_leaf(const SearchParams& P, uint32_t tau) {
  return P.leaf_filter_tau && P.stage_cap >= kLeafFilterWords && tau >= P.leaf_filter_tau;
}

// Rounds a filter queue waits: 1/32 of the node's expected rounds (about 2^tau
// values, mult per attempt), 1 to 16.
__device__ __forceinline__ uint32_t patience(const Node& c, uint32_t tau) {
  const uint64_t expect = (1ull << (tau < 40 ? tau : 40)) / ((uint64_t)c.mult * kWG);
  const uint64_t pat = expect >> 5;
  return pat < 1 ? 1u : (pat > 16 ? 16u : (uint32_t)pat);
}

// Most leaves are short and there are many: one worker searches such a leaf
// alone, as one chunk without a bound on its rounds, with no global traffic
// until the value is known (its state is never claimed).  In small launches
// of the filter kernel, leaves whose Rice parameter reaches join_leaf_tau go
// through the claimed chunks of run_claimed instead, so that idle workers can
// join them.
template <bool kFilter, bool kReport>
__device__ void run_leaf(const SearchParams& P, Shared& sh, uint64_t* s_keys, const Task& t,
                         const JobDev& J, uint64_t slot) {
  const uint32_t tid = threadIdx.x;
  Node c = make_node(t, J, P.start, P.cap_shift, kFilter ? 0u : P.rotation_lookup);
  stage_keys(t, J, c, s_keys, &sh.na);
  if (tid == 0) sh.best = kInf;
  __syncthreads();
  c.na = uni(sh.na);
  const uint64_t max_rounds = c.cap / kWG + 1;
  const uint32_t rounds = max_rounds < 0xFFFFFFFFull ? (uint32_t)max_rounds : 0xFFFFFFFFu;
  // long leaf searches go through the filter (the queues sit in the staging
  // area, after the leaf's keys)
  const uint32_t tau = uni((uint32_t)J.tau[c.m]);
  if (kFilter && filtered_leaf(P, tau))
    run_leaf_filtered(c, 0, rounds, patience(c, tau), &sh.best);
  else
    eval_chunk<!kFilter>(s_keys, c, 0, rounds, &sh.best);
  __syncthreads();
  const uint64_t v = sh.best;
  if (v == kInf) {
    if (tid == 0 && set_error(P.ctl, (uint32_t)(-RS_ERR_SEARCH_LIMIT)))
      record_failure(P.ctl, t, slot, P.states + (slot < P.ctl->total ? slot : 0), 0);
  } else {
    finalize_leaf<kReport>(P, t, J, c, v);
  }
  __syncthreads();
}

// Whole-bucket mode (small leaves, small buckets): a worker builds a whole
// bucket tree on its own, with the keys resident in LDS.  No node goes
// through the queue and no key goes back to global memory: a split's keys
// are partitioned among its children in LDS, and every search is one
// unbounded chunk, as for a leaf.  Dynamic LDS layout: the stack of pending
// nodes, then hashed words, their scratch copy, A/B classes, their scratch.
struct Frame {
  uint32_t off, m, depth, pad;
  uint64_t node;
};
constexpr uint32_t kFrames = kBucketStackBytes / sizeof(Frame);
static_assert(kFrames * sizeof(Frame) == kBucketStackBytes, "stack layout");

// Stable partition of a split node's keys (with their A/B classes) by child
// under value v, in LDS through a scratch copy, then back.  One wave.
__device__ void partition_lds(const SearchParams& P, const Node& c, uint64_t v, uint64_t* keys,
                              uint8_t* cls, uint64_t* tmp, uint8_t* ctmp) {
  const uint32_t lane = lane_id();
  const uint64_t X = c.start + v;
  uint32_t run = 0;  // lane j: keys already placed in child j
  for (uint32_t g = 0; g < c.m; g += 64) {
    const uint32_t i = g + lane;
    const bool ok = i < c.m;
    const uint64_t w = ok ? keys[i] : 0;
    const uint8_t b = ok ? cls[i] : 0;
    const uint32_t p = reduce(hash_top(w, X), c.m);
    uint32_t ch = c.kind == kBinary ? (p >= c.unit ? 1u : 0u) : p / c.unit;
    if (!ok) ch = 0xFFFFFFFFu;
    const uint32_t at0 = (uint32_t)__shfl((int)run, ok ? (int)ch : 0);
    uint32_t rank = 0;
    for (uint32_t j = 0; j < c.k; ++j) {
      const uint64_t mk = __ballot(ch == j);
      if (ch == j) rank = (uint32_t)__popcll(mk & mask_below(lane));
      if (lane == j) run += (uint32_t)__popcll(mk);
    }
    const uint32_t at = ch * c.unit + at0 + rank;
    if (ok && at < c.m) {
      tmp[at] = w;
      ctmp[at] = b;
    }
  }
  const bool good = lane >= c.k || run == (lane + 1 < c.k ? c.unit : c.last);
  if (__ballot(!good) != 0 && lane == 0) set_error(P.ctl, (uint32_t)(-RS_ERR_DEVICE));
  for (uint32_t i = lane; i < c.m; i += 64) {
    keys[i] = tmp[i];
    cls[i] = ctmp[i];
  }
}

__device__ void run_bucket(const SearchParams& P, Shared& sh, uint64_t* lds, const Task& t,
                           const JobDev& J) {
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t cap = P.stage_cap;
  Frame* stack = reinterpret_cast<Frame*>(lds);
  uint64_t* s_keys = lds + kBucketStackBytes / sizeof(uint64_t);
  uint64_t* s_tmp = s_keys + cap;
  uint8_t* s_cls = reinterpret_cast<uint8_t*>(s_tmp + cap);
  uint8_t* s_ctmp = s_cls + cap;
  const Key* src = J.keys[0] + t.key_off;
  for (uint32_t i = tid; i < t.m; i += kWG) {
    const Key k = src[i];
    s_keys[i] = k.w1;
    s_cls[i] = (uint8_t)(k.w0 & 1u);
  }
  uint32_t sp = 0, done = 0;  // thread 0: stack depth, nodes finished
  if (tid == 0) {
    Frame f;
    f.off = 0;
    f.m = t.m;
    f.depth = t.depth;
    f.pad = 0;
    f.node = t.node;
    stack[0] = f;
    sp = 1;
  }
  for (;;) {
    __syncthreads();  // the previous node is done; every thread has read its state
    if (tid == 0) {
      sh.go = 0;
      if (sp && ld_relaxed(&P.ctl->error) == 0) {
        const Frame f = stack[--sp];
        sh.task.key_off = f.off;
        sh.task.m = f.m;
        sh.task.depth = (uint16_t)f.depth;
        sh.task.node = f.node;
        sh.go = 1;
      }
      sh.best = kInf;
    }
    __syncthreads();
    if (!sh.go) break;
    Task nt;
    nt.key_off = uni64(sh.task.key_off);
    nt.m = uni(sh.task.m);
    nt.depth = (uint16_t)uni(sh.task.depth);
    nt.node = uni64(sh.task.node);
    nt.job = t.job;
    uint64_t* keys = s_keys + nt.key_off;
    uint8_t* cls = s_cls + nt.key_off;
    Node c = make_node(nt, J, P.start, P.cap_shift, P.rotation_lookup);
    if (c.kind == kLeaf && tid < 64) {
      // the keys of A (class bit clear) first, in a stable order
      const bool v = lane < c.m;
      const uint64_t w = v ? keys[lane] : 0;
      const bool isb = v && cls[lane];
      const uint64_t bm = __ballot(isb);
      const uint64_t am = __ballot(v && !isb);
      const uint32_t na = (uint32_t)__popcll(am);
      const uint64_t below = mask_below(lane);
      if (v) keys[isb ? na + (uint32_t)__popcll(bm & below) : (uint32_t)__popcll(am & below)] = w;
      if (lane == 0) sh.na = na;
    }
    __syncthreads();
    if (c.kind == kLeaf) c.na = uni(sh.na);
    const uint64_t max_rounds = c.cap / kWG + 1;
    eval_chunk<true>(keys, c, 0, max_rounds < 0xFFFFFFFFull ? (uint32_t)max_rounds : 0xFFFFFFFFu,
               &sh.best);
    __syncthreads();
    const uint64_t v = sh.best;
    if (v == kInf) {
      if (tid == 0 && set_error(P.ctl, (uint32_t)(-RS_ERR_SEARCH_LIMIT)))
        record_failure(P.ctl, nt, kNoSlot, P.states, 0);
      continue;  // the error ends the loop at the next pop
    }
    if (c.kind != kLeaf && tid < 64)
      partition_lds(P, c, v, keys, cls, s_tmp + nt.key_off, s_ctmp + nt.key_off);
    if (tid == 0) {
      J.vals[nt.node] = v;
      J.msz[nt.node] = c.m;
      ++done;
      if (c.kind != kLeaf) {
        // children that store a node (any order: a node's index fixes where
        // its value goes)
        uint64_t cn = nt.node + 1;
        for (uint32_t j = 0; j < c.k; ++j) {
          const uint32_t sz = j + 1 < c.k ? c.unit : c.last;
          if (sz >= 2) {
            if (sp >= kFrames || nt.depth + 1 >= kMaxDepth) {
              set_error(P.ctl, (uint32_t)(-RS_ERR_UNSUPPORTED));
              break;
            }
            Frame f;
            f.off = (uint32_t)nt.key_off + j * c.unit;
            f.m = sz;
            f.depth = nt.depth + 1u;
            f.pad = 0;
            f.node = cn;
            stack[sp++] = f;
          }
          cn += J.nodecnt[sz];
        }
      }
    }
  }
  if (tid == 0 && done) note_finished<true>(P, (uint64_t)done);
  __syncthreads();
}

// Search task t (queue slot `slot`) in claimed chunks until this worker's
// claim is refused, and finalize it if this worker drops the last chunk in
// flight.  sh.my_q (thread 0) is the queue slot this worker has reserved; a
// helper leaves as soon as that slot is ready.  kLeafTask: a long leaf (the
// filter kernel only), instantiated apart so that the split searches keep
// their registers.
template <uint32_t kMode, bool kLeafTask>
__device__ void run_claimed(const SearchParams& P, Shared& sh, uint64_t* s_keys, const Task& t,
                            const JobDev& J, uint64_t slot, bool own) {
  const uint32_t tid = threadIdx.x;
  constexpr bool leaf = kLeafTask;
  Node c = make_node(t, J, P.start, P.cap_shift, filter_mode(kMode) ? 0u : P.rotation_lookup);
  stage_keys(t, J, c, s_keys, &sh.na);
  __syncthreads();
  if (leaf) c.na = uni(sh.na);
  // A worker's successive claims on a search double in length, from one round
  // up to 2^clamp(tau - chunk_shift, 0, 8) rounds (tau, the Rice parameter, is
  // about log2 of the expected attempts): a search that ends soon is not
  // overshot, a long one takes few claims.
  const uint32_t tau = uni((uint32_t)J.tau[c.m]);
  const uint32_t e = tau > P.chunk_shift ? (tau - P.chunk_shift < 8 ? tau - P.chunk_shift : 8) : 0;
  const uint32_t rmax = c.kind == kBinary ? 1u : (1u << e);
  // the filter kernels' staged split search, where the counters fit (32-bit
  // words, or 64-bit ones in the wide kernel) and the queues fit after the
  // node's keys
  using Word = typename std::conditional<kMode == kSearchFilterWide, uint64_t, uint32_t>::type;
  const bool split_filter = filter_mode(kMode) && !leaf && P.split_filter_tau &&
                            tau >= P.split_filter_tau && split_filter_fits<Word>(c) &&
                            split_queue_at(c.m) + kSplitQueueWords <= P.stage_cap;
  TaskState* st = P.states + slot;
  uint32_t r = 1;  // thread 0: rounds of this worker's next claim
  // Thread 0 turns the word returned by a claim of rr rounds into the chunk to
  // evaluate (true), or drops the claim (value known, limit passed).
  auto decide = [&](uint64_t old, uint32_t rr) -> bool {
    const uint64_t first = cursor(old);
    if (old & kFound) {
      sh.fin = release_chunk(st) ? 1u : 0u;
      return false;
    }
    // every worker may hold two claimed chunks whose results are not in yet
    if (first * kWG >= c.cap + 2ull * P.workers * rmax * kWG) {
      if (set_error(P.ctl, (uint32_t)(-RS_ERR_SEARCH_LIMIT)))
        record_failure(P.ctl, t, slot, st, first);
      sh.fin = release_chunk(st) ? 1u : 0u;
      return false;
    }
    if (first <= P.help_after && P.help_after < first + rr) {
      // the claim that takes the search past help_after rounds: count it as
      // a long search so idle workers look for it
      uint32_t expected = 0;
      if (__hip_atomic_compare_exchange_strong(&st->advert, &expected, 1u, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        __hip_atomic_fetch_add(&P.ctl->long_tasks, 1ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      wait_memory();  // counted before this chunk can be dropped
    }
    sh.first = first;
    sh.rounds = rr;
    return true;
  };
  // a helper leaves as soon as the queue slot it holds is ready
  auto leave = [&]() {
    return ld_relaxed(&P.ctl->error) != 0 ||
           (!own && sh.my_q < kExhausted && ld_relaxed(&P.ready[sh.my_q]) != 0);
  };
  if (tid == 0) {
    sh.fin = 0;
    sh.best = kInf;
    sh.go = 0;
    if (!leave()) {
      sh.go = decide(__hip_atomic_fetch_add(&st->np, ((uint64_t)r << 32) | 1ull, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT),
                     r)
                  ? 1u
                  : 0u;
      r = r * 2 < rmax ? r * 2 : rmax;
    }
  }
  // The owner claims its next chunk before evaluating the current one, so
  // that the claim's round trip to the device coherence point overlaps the
  // evaluation; it then holds two chunks in flight.  The next chunk lies
  // above the current one, so a value found in the current chunk drops it
  // unevaluated.  A helper, which may have to leave, holds one chunk only,
  // and so does the filter kernel, where the extra state would spill
  // registers to scratch memory.
  uint64_t next_old = 0;  // thread 0: the word the claim of the next chunk returned
  uint32_t next_r = 0;
  bool have_next = false;
  for (;;) {
    __syncthreads();  // thread 0's decision is visible
    if (!sh.go) break;
    if (tid == 0 && own && kMode == kSearchNode) {
      next_r = r;
      next_old = __hip_atomic_fetch_add(&st->np, ((uint64_t)r << 32) | 1ull, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
      have_next = true;
      r = r * 2 < rmax ? r * 2 : rmax;
    }
    if (leaf && filtered_leaf(P, tau))
      run_leaf_filtered(c, sh.first, sh.rounds, patience(c, tau), &sh.best);
    else if (split_filter && sh.rounds >= kMinFilterRounds)
      run_split_filtered<Word>(s_keys, c, sh.first, sh.rounds, patience(c, tau), &sh.best,
                               s_keys + split_queue_at(c.m) + (tid >> 6) * 3 * kLeafQueue);
    else
      eval_chunk<!filter_mode(kMode)>(s_keys, c, sh.first, sh.rounds, &sh.best);
    __syncthreads();  // the chunk's best is final; every thread has read the decision
    if (tid == 0) {
      const uint64_t v = sh.best;
      sh.best = kInf;
      sh.fin = 0;
      sh.go = 0;
      const uint32_t held = have_next ? 2u : 1u;
      have_next = false;
      if (v != kInf) {
        __hip_atomic_fetch_min(&st->best, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_memory();  // the value is in before the found bit
        __hip_atomic_fetch_or(&st->np, kFound, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_memory();  // and the bit before the chunks are dropped
        sh.fin = release_chunk(st, held) ? 1u : 0u;
      } else if (leave()) {
        sh.fin = release_chunk(st, held) ? 1u : 0u;
      } else if (held == 2) {
        if (next_old & kFound) {
          // the next chunk lies above a known value: drop both
          sh.fin = release_chunk(st, 2) ? 1u : 0u;
        } else {
          // drop the evaluated chunk (the next one keeps the count above
          // zero, so this cannot be the last drop) and move on
          __hip_atomic_fetch_add(&st->np, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          sh.go = decide(next_old, next_r) ? 1u : 0u;
        }
      } else {
        // drop the evaluated chunk and claim the next with one atomic
        sh.go = decide(__hip_atomic_fetch_add(&st->np, (uint64_t)r << 32, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT),
                       r)
                    ? 1u
                    : 0u;
        r = r * 2 < rmax ? r * 2 : rmax;
      }
    }
  }
  if (!sh.fin) return;
  if (tid == 0) {
    sh.fin_value = ld_relaxed(&st->best);
    uint32_t expected = 1;
    if (__hip_atomic_compare_exchange_strong(&st->advert, &expected, 2u, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      __hip_atomic_fetch_add(&P.ctl->long_tasks, ~0ull, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  const uint64_t v = sh.fin_value;
  if constexpr (leaf) {
    finalize_leaf<reports_progress(kMode)>(P, t, J, c, v);
    __syncthreads();
    return;
  }
  if (tid < 64) finalize_split<reports_progress(kMode)>(P, t, J, c, v);
  __syncthreads();
  // the leaf children kept out of the queue, searched here in order
  const uint32_t l = uni(J.l);
  uint64_t child_node = t.node + 1;
  for (uint32_t j = 0; j < c.k; ++j) {
    const uint32_t sz = j + 1 < c.k ? c.unit : c.last;
    if (sz >= 2 && !queued_child(P, J, l, sz)) {
      Task ct;
      ct.key_off = t.key_off + (uint64_t)j * c.unit;
      ct.node = child_node;
      ct.m = sz;
      ct.depth = (uint16_t)(t.depth + 1);
      ct.job = t.job;
      run_leaf<filter_mode(kMode), reports_progress(kMode)>(P, sh, s_keys, ct, J, kNoSlot);
    }
    child_node += uni(J.nodecnt[sz]);
  }
}

// Work on the task in queue slot `slot` (own: this worker took it from the
// queue; otherwise it joins another worker's search).
template <uint32_t kMode>
__device__ void run_task(const SearchParams& P, Shared& sh, uint64_t* s_keys, uint64_t slot,
                         bool own) {
  Task t = sh.task;
  t.key_off = uni64(t.key_off);
  t.node = uni64(t.node);
  t.m = uni(t.m);
  t.depth = (uint16_t)uni(t.depth);
  t.job = (uint16_t)uni(t.job);
  const JobDev& J = P.jobs[t.job];
  if constexpr (kMode == kSearchBucket) {
    run_bucket(P, sh, s_keys, t, J);
  } else {
    if (t.m > uni(J.l)) {
      run_claimed<kMode, false>(P, sh, s_keys, t, J, slot, own);
      return;
    }
    if constexpr (filter_mode(kMode)) {
      // long leaves (what the filter kernel is chosen for) can be joined
      if (P.join_leaf_tau && uni((uint32_t)J.tau[t.m]) >= P.join_leaf_tau) {
        run_claimed<kMode, true>(P, sh, s_keys, t, J, slot, own);
        return;
      }
    }
    run_leaf<filter_mode(kMode), reports_progress(kMode)>(P, sh, s_keys, t, J, slot);
  }
}

// ---------------------------------------------------------------- one wave per bucket
// Whole-bucket mode with one wave per worker (workgroups of 64 threads).
// Where leaves and buckets are small, a node's search usually ends within
// its first 64 attempts, so four waves sharing one node (256 attempts a
// round) mostly evaluate attempts above its value.  Here each wave takes
// bucket roots from the queue in turn (all of them are queued before the
// launch) and builds each tree alone in its own LDS, 64 attempts a round:
// the lowest valid lane of the first round with one is the node's value.
template <typename RoundFn>
__device__ __forceinline__ uint64_t wave_search(const uint64_t* keys, const Node& c, RoundFn fn) {
  const uint64_t rounds = c.cap / 64 + 1;
  for (uint64_t r = 0; r < rounds; ++r) {
    const uint64_t v = fn(keys, c, r * 64);
    if (v != kInf) return v;
  }
  return kInf;
}

__device__ uint64_t wave_eval(const uint64_t* keys, const Node& c) {
  switch (c.kind) {
    case kLeaf:
      return c.rotation ? wave_search(keys, c, round_leaf_rot<true>)
                        : wave_search(keys, c, round_leaf_brute);
    case kLower:
    case kUpper:
      return c.full ? wave_search(keys, c, round_split_kway<true>)
                    : wave_search(keys, c, round_split_kway<false>);
    default: return wave_search(keys, c, round_split_binary);
  }
}

// Global-memory accesses of the one-wave workers, in the global address
// space: flat accesses would count in the same wait counter as the LDS
// traffic, so every LDS wait would also wait for them.
typedef __attribute__((address_space(1))) uint64_t g_u64;
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) const uint64_t g_cu64;

// What a one-wave bucket worker reads of a job: the shape, leaf method and
// output arrays in registers (read once per job, so that no node waits on a
// global load of them), the Rice parameters in LDS.
struct WaveJob {
  uint32_t l, la, ua, rotation;
  const uint8_t* tau;
  const Key* keys;
  uint64_t* vals;
  uint32_t* msz;
};

// Stage a bucket's keys (w1 and the A/B class bit) in LDS, up to four keys
// per lane per batch: the loads of a batch are issued before its first
// write, so a bucket of up to 256 keys waits for memory once.
__device__ __forceinline__ void wave_stage_keys(const Key* src, uint32_t m, uint64_t* s_keys,
                                                uint8_t* s_cls) {
  const uint32_t lane = lane_id();
  for (uint32_t base = 0; base < m; base += 256) {
    // lanes past the end read the last key again (in bounds, not stored), so
    // the four loads need no branches and are issued back to back
    const g_cu64* kw = (const g_cu64*)src;  // w0, w1 of key i at 2i, 2i+1
    uint64_t w0[4], w1[4];
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      const uint32_t i = base + lane + 64u * u;
      const uint32_t j = i < m ? i : m - 1;
      w0[u] = kw[2 * j];
      w1[u] = kw[2 * j + 1];
    }
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      const uint32_t i = base + lane + 64u * u;
      if (i < m) {
        s_keys[i] = w1[u];
        s_cls[i] = (uint8_t)(w0[u] & 1u);
      }
    }
  }
}

// One bucket tree, built by this wave from the keys already in its LDS.  The
// starting seeds and the job's Rice parameters and subtree node counts (for
// node sizes up to the stage capacity) sit in this wave's LDS after the
// bucket's arrays (LDS reads instead of dependent global loads on the path
// of every node).  Returns the number of nodes that got a value.
__device__ uint32_t wave_bucket(const SearchParams& P, uint64_t* lds, const Task& t,
                                const WaveJob& W, const uint64_t* s_start,
                                const uint32_t* s_nodecnt) {
  const uint32_t lane = lane_id();
  const uint32_t cap = P.stage_cap;
  Frame* stack = reinterpret_cast<Frame*>(lds);
  uint64_t* s_keys = lds + kBucketStackBytes / sizeof(uint64_t);
  uint64_t* s_tmp = s_keys + cap;
  uint8_t* s_cls = reinterpret_cast<uint8_t*>(s_tmp + cap);
  uint8_t* s_ctmp = s_cls + cap;
  // the stack's contents are uniform: every lane pushes and pops alike, lane
  // 0 writes
  Frame root;
  root.off = 0;
  root.m = t.m;
  root.depth = t.depth;
  root.pad = 0;
  root.node = t.node;
  if (lane == 0) stack[0] = root;
  uint32_t sp = 1, done = 0;
  while (sp) {
    __syncthreads();  // one wave: orders the keys and the stack in LDS
    const Frame f = stack[--sp];
    Task nt;
    nt.key_off = uni(f.off);
    nt.m = uni(f.m);
    nt.depth = (uint16_t)uni(f.depth);
    nt.node = uni64(f.node);
    nt.job = t.job;
    uint64_t* keys = s_keys + nt.key_off;
    uint8_t* cls = s_cls + nt.key_off;
    Node c = make_node(nt, W, s_start, P.cap_shift, P.rotation_lookup);
    if (c.kind == kLeaf) {
      // the keys of A (class bit clear) first, in a stable order
      const bool v = lane < c.m;
      const uint64_t w = v ? keys[lane] : 0;
      const bool isb = v && cls[lane];
      const uint64_t bm = __ballot(isb);
      const uint64_t am = __ballot(v && !isb);
      c.na = (uint32_t)__popcll(am);
      const uint64_t below = mask_below(lane);
      __syncthreads();
      if (v) keys[isb ? c.na + (uint32_t)__popcll(bm & below) : (uint32_t)__popcll(am & below)] = w;
      __syncthreads();
    }
    const uint64_t v = wave_eval(keys, c);
    if (v == kInf) {
      if (lane == 0 && set_error(P.ctl, (uint32_t)(-RS_ERR_SEARCH_LIMIT)))
        record_failure(P.ctl, nt, kNoSlot, P.states, 0);
      break;
    }
    if (c.kind != kLeaf) {
      __syncthreads();
      partition_lds(P, c, v, keys, cls, s_tmp + nt.key_off, s_ctmp + nt.key_off);
    }
    if (lane == 0) {
      ((g_u64*)W.vals)[nt.node] = v;
      ((g_u32*)W.msz)[nt.node] = c.m;
    }
    ++done;
    if (c.kind != kLeaf) {
      // children that store a node (any order: a node's index fixes where its
      // value goes)
      uint64_t cn = nt.node + 1;
      for (uint32_t j = 0; j < c.k; ++j) {
        const uint32_t sz = j + 1 < c.k ? c.unit : c.last;
        if (sz >= 2) {
          if (sp >= kFrames || nt.depth + 1 >= kMaxDepth) {
            if (lane == 0) set_error(P.ctl, (uint32_t)(-RS_ERR_UNSUPPORTED));
            sp = 0;
            break;
          }
          Frame g;
          g.off = (uint32_t)nt.key_off + j * c.unit;
          g.m = sz;
          g.depth = nt.depth + 1u;
          g.pad = 0;
          g.node = cn;
          if (lane == 0) stack[sp] = g;
          ++sp;
        }
        cn += uni(s_nodecnt[sz]);
      }
    }
  }
  __syncthreads();
  return done;
}

// A task record made wave-uniform (its fields in scalar registers).
__device__ Task wave_uni(Task t) {
  t.key_off = uni64(t.key_off);
  t.node = uni64(t.node);
  t.m = uni(t.m);
  t.depth = (uint16_t)uni(t.depth);
  t.job = (uint16_t)uni(t.job);
  return t;
}

// The one-wave worker: bucket roots from the queue in turn (every root was
// queued before the launch, so the tail is final); finished nodes are
// counted once per wave.  (Claiming the next root before building the
// current tree, to overlap the two round trips, measured 25-35 % slower on
// buckets of 100 keys.)
__device__ void wave_main(const SearchParams& P) {
  extern __shared__ uint64_t lds[];
  const uint32_t lane = lane_id();
  const uint32_t cap = P.stage_cap;
  // LDS after the bucket arrays: starting seeds, the current job's Rice
  // parameters and subtree node counts for sizes 0..cap (wave_bucket_lds_bytes)
  uint64_t* s_start = lds + wave_tables_at(cap) / sizeof(uint64_t);
  uint32_t* s_nodecnt = reinterpret_cast<uint32_t*>(s_start + kMaxDepth);
  uint8_t* s_tau = reinterpret_cast<uint8_t*>(s_nodecnt + cap + 1);
  uint64_t* s_keys = lds + kBucketStackBytes / sizeof(uint64_t);
  uint8_t* s_cls = reinterpret_cast<uint8_t*>(s_keys + 2 * cap);
  for (uint32_t i = lane; i < kMaxDepth; i += 64) s_start[i] = P.start[i];
  const uint64_t tail = uni64(ld_relaxed(&P.ctl->tail));
  auto claim = [&]() {
    uint64_t q = 0;
    if (lane == 0)
      q = __hip_atomic_fetch_add(&P.ctl->head, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return uni64(readlane64(q, 0));
  };
  uint32_t job = 0xFFFFFFFFu;  // whose tables are in LDS
  WaveJob W;
  uint32_t done = 0;
  for (;;) {
    const uint64_t q = claim();
    if (q >= tail || ld_relaxed(&P.ctl->error) != 0) break;
    Task t = wave_uni(P.tasks[q]);
    if (t.job != job) {
      const JobDev& J = P.jobs[t.job];
      W.l = uni(J.l);
      W.la = uni(J.la);
      W.ua = uni(J.ua);
      W.rotation = uni(J.rotation);
      W.tau = s_tau;
      W.keys = J.keys[0];
      W.vals = J.vals;
      W.msz = J.msz;
      for (uint32_t i = lane; i <= cap; i += 64) {
        s_nodecnt[i] = J.nodecnt[i];
        s_tau[i] = J.tau[i];
      }
      job = t.job;
    }
    wave_stage_keys(W.keys + t.key_off, t.m, s_keys, s_cls);
    done += wave_bucket(P, lds, t, W, s_start, s_nodecnt);
  }
  if (lane == 0 && done) note_finished<true>(P, (uint64_t)done);
}

}  // namespace

// The persistent worker loop, one kernel per mode (kSearchNode, kSearchFilter
// with filtered leaves, kSearchBucket with whole-bucket workers), so that
// each keeps its own register budget.
template <uint32_t kMode>
__device__ __forceinline__ void search_main(const SearchParams& P) {
  extern __shared__ uint64_t s_keys[];
  __shared__ Shared sh;
  const uint32_t tid = threadIdx.x;
  const uint32_t g = blockIdx.x;
  const uint64_t total = P.ctl->total;
  if (tid == 0) {
    sh.iter = 0;
    sh.my_q = kNoSlot;
    sh.last_finished = 0;
    sh.idle_since = 0;
    sh.idle = 0;  // consecutive rounds without work
  }
  __syncthreads();
  for (;;) {
    __syncthreads();  // every thread has read the previous decision
    if (tid == 0) {
      uint32_t act = kActRetry;
      if (ld_relaxed(&P.ctl->error) != 0) {
        act = kActExit;
      } else {
        if (sh.my_q == kNoSlot) {
          const uint64_t q = __hip_atomic_fetch_add(&P.ctl->head, 1ull, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
          sh.my_q = q < total ? q : kExhausted;
        }
        if (sh.my_q < kExhausted && ld_relaxed(&P.ready[sh.my_q]) != 0) {
          fence_acquire();
          act = kActOwn;
          sh.arg = sh.my_q;
          sh.my_q = kNoSlot;
        } else if (ld_relaxed(&P.ctl->finished) >= total) {
          // every node is final (slots a worker still holds may never be
          // filled: inline leaves take none)
          act = kActExit;
        } else if (ld_relaxed(&P.ctl->long_tasks) != 0) {
          act = kActScan;
        }
      }
      sh.action = act;
      sh.pick = 0x7FFFFFFF;
      sh.iter += 1;
    }
    __syncthreads();
    uint32_t act = sh.action;
    if (act == kActExit) break;
    if (act == kActScan) {
      // look for a long search among up to 256 workers, from a rotating start
      const uint32_t W = P.workers;
      const uint32_t rot = (g * 2654435761u + sh.iter * 40503u) % W;
      if (tid < W) {
        uint32_t idx = tid + rot;
        if (idx >= W) idx -= W;
        if (ld_relaxed(&P.active[idx]) >= 0) atomicMin(&sh.pick, (int32_t)tid);
      }
      __syncthreads();
      if (tid == 0) {
        uint32_t next = kActRetry;
        if (sh.pick != 0x7FFFFFFF) {
          uint32_t idx = (uint32_t)sh.pick + rot;
          if (idx >= W) idx -= W;
          const int32_t a = ld_relaxed(&P.active[idx]);
          if (a >= 0 && ld_relaxed(&P.ready[a]) != 0) {
            // join only searches that are long already: a task that ends in
            // its first chunks gains nothing from more workers
            const TaskState* ts = P.states + a;
            const uint64_t w = ld_relaxed(&ts->np);
            if (cursor(w) >= P.help_after && !(w & kFound)) {
              fence_acquire();
              next = kActHelp;
              sh.arg = (uint64_t)a;
            }
          }
        }
        sh.action = next;
      }
      __syncthreads();
      act = sh.action;
    }
    if (act == kActRetry) {
      if (tid == 0) {
        // bug guard: no node finished for stall_ticks of the 100 MHz clock
        const uint64_t fin = ld_relaxed(&P.ctl->finished);
        const uint64_t now = __builtin_amdgcn_s_memrealtime();
        if (fin != sh.last_finished || sh.idle_since == 0) {
          sh.last_finished = fin;
          sh.idle_since = now;
        } else if (now - sh.idle_since > P.stall_ticks) {
          set_error(P.ctl, (uint32_t)(-RS_ERR_DEVICE));
        }
        // back off while idle: 1, 2, 4, 8 sleeps of 16 x 64 cycles
        const uint32_t naps = 1u << (sh.idle < 3 ? sh.idle : 3);
        for (uint32_t i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(16);
        ++sh.idle;
      }
      continue;
    }
    const uint64_t slot = sh.arg;
    if (tid == 0) {
      sh.task = P.tasks[slot];
      if (act == kActOwn) st_relaxed(&P.active[g], (int32_t)slot);
      sh.idle_since = 0;
      sh.idle = 0;
    }
    __syncthreads();
    run_task<kMode>(P, sh, s_keys, slot, act == kActOwn);
    if (tid == 0 && act == kActOwn) st_relaxed(&P.active[g], (int32_t)-1);
    __syncthreads();
  }
}

}  // namespace rs

extern "C" __global__ void __launch_bounds__(rs::kWG) rs_search_kernel(rs::SearchParams P) {
  rs::search_main<rs::kSearchNode>(P);
}

// seven waves per SIMD, as the plain kernel has: the filter's state goes to
// scalar spill lanes rather than costing occupancy
extern "C" __global__ void __launch_bounds__(rs::kWG) __attribute__((amdgpu_waves_per_eu(7)))
rs_filter_kernel(rs::SearchParams P) {
  rs::search_main<rs::kSearchFilter>(P);
}

// the same with 64-bit split counters, for leaf sizes 19 to 24 (six waves per
// SIMD: at seven the wider counters spill vector registers to memory)
extern "C" __global__ void __launch_bounds__(rs::kWG) __attribute__((amdgpu_waves_per_eu(6)))
rs_filter_wide_kernel(rs::SearchParams P) {
  rs::search_main<rs::kSearchFilterWide>(P);
}

extern "C" __global__ void __launch_bounds__(rs::kWG) rs_bucket_kernel(rs::SearchParams P) {
  rs::search_main<rs::kSearchBucket>(P);
}

extern "C" __global__ void __launch_bounds__(64) rs_wave_bucket_kernel(rs::SearchParams P) {
  rs::wave_main(P);
}

namespace rs {

static const void* search_kernel(uint32_t mode) {
  return mode == kSearchBucketWave ? reinterpret_cast<const void*>(rs_wave_bucket_kernel)
         : mode == kSearchBucket   ? reinterpret_cast<const void*>(rs_bucket_kernel)
         : mode == kSearchFilter   ? reinterpret_cast<const void*>(rs_filter_kernel)
         : mode == kSearchFilterWide ? reinterpret_cast<const void*>(rs_filter_wide_kernel)
                                   : reinterpret_cast<const void*>(rs_search_kernel);
}

uint32_t search_block(uint32_t mode) { return mode == kSearchBucketWave ? 64u : kWG; }

void rotation_tables(uint16_t* out) {
  out[0] = out[1] = 0;
  for (uint32_t m = 1; m <= kRotLookupMaxM; ++m) {
    const uint32_t full = (1u << m) - 1u;
    for (uint32_t x = 0; x <= full; ++x) {
      uint32_t best = x, t = 0, period = m;
      for (uint32_t r = 1; r < m; ++r) {
        const uint32_t y = ((x << r) | (x >> (m - r))) & full;
        if (y < best) {
          best = y;
          t = r;
        }
        if (y == x && period == m) period = r;
      }
      out[(1u << m) + x] = (uint16_t)(t | (period << 8));
    }
  }
}

hipError_t upload_rotation_tables() {
  std::vector<uint16_t> t(kRotLookupEntries);
  rotation_tables(t.data());
  return hipMemcpyToSymbol(HIP_SYMBOL(g_rot_lookup), t.data(), kRotLookupEntries * sizeof(uint16_t),
                           0, hipMemcpyHostToDevice);
}

hipError_t search_occupancy(uint32_t lds_bytes, int* blocks_per_cu, uint32_t mode) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, search_kernel(mode),
                                                      search_block(mode), lds_bytes);
}

hipError_t launch_search(const SearchParams& p, uint32_t grid, uint32_t lds_bytes, hipStream_t s) {
  void* args[] = {const_cast<SearchParams*>(&p)};
  return hipLaunchKernel(search_kernel(p.mode), dim3(grid), dim3(search_block(p.mode)), args,
                         lds_bytes, s);
}

}  // namespace rs
