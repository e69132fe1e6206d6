// Host-side launchers of the library's kernels (one translation unit each).
#pragma once

#include <vector>

#include "rs_internal.h"

namespace rs {

hipError_t fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);

// Exclusive scan: out[0..n] with out[n] the total; tmp needs scan_tmp_words(n) words.
uint64_t scan_tmp_words(uint64_t n);
hipError_t scan_excl_u32(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* tmp, hipStream_t s);
hipError_t scan_excl_u64(const uint64_t* in, uint64_t n, uint64_t* out, uint64_t* tmp, hipStream_t s);

hipError_t bucket_histogram(const Key* keys, uint64_t n, uint64_t nb, uint32_t* cnt, uint32_t* maxm,
                            hipStream_t s);
hipError_t bucket_scatter(const Key* keys, uint64_t n, uint64_t nb, const uint64_t* off,
                          uint32_t* fill, Key* out, hipStream_t s);
// cap: LDS words of the check (a power of two); buckets whose next power of
// two exceeds it are skipped and set *deferred.
hipError_t duplicate_check(const Key* keys, const uint64_t* off, uint64_t nb, uint32_t cap,
                           uint32_t* error, uint32_t* deferred, hipStream_t s);
hipError_t init_states(TaskState* st, uint64_t n, hipStream_t s);
hipError_t node_counts(const uint32_t* cnt, uint64_t nb, const uint32_t* nodecnt, uint64_t* out,
                       hipStream_t s);
hipError_t queue_roots(const uint32_t* cnt, const uint64_t* off, const uint64_t* node_base,
                       uint64_t nb, uint32_t job, uint64_t key_base, uint64_t node_off, Task* tasks,
                       uint32_t* ready, Control* ctl, hipStream_t s);

// Useful hash evaluations and node counts of a finished search (added to
// *info); split_fx: expected evaluations of a failed split attempt per node
// size, in units of 2^-kLeafWorkShift.
hipError_t work_counts(const uint64_t* vals, const uint32_t* msz, uint64_t n, uint32_t l,
                       uint32_t rotation, const uint32_t* split_fx, JobInfo* info, hipStream_t s);

// The LeafWork table of a leaf search mode (host).
LeafWork leaf_work_table(bool rotation);

// Expected evaluations of a failed split attempt, per node size m <
// kTable, for leaf size l (0 for leaf sizes; host).
std::vector<double> split_work_table(uint32_t l);

// The rotation lookup tables (kRotLookupEntries entries, host) and their
// upload to the current device's copy of the search kernels' table.
void rotation_tables(uint16_t* out);
hipError_t upload_rotation_tables();

// Seed search (persistent kernel).
hipError_t search_occupancy(uint32_t lds_bytes, int* blocks_per_cu, uint32_t mode = kSearchNode);
hipError_t launch_search(const SearchParams& p, uint32_t grid, uint32_t lds_bytes, hipStream_t s);

// Encoding.
hipError_t gr_lengths(const uint64_t* node_base, uint64_t nb, const uint64_t* vals,
                      const uint32_t* msz, const uint8_t* tau, uint64_t* len, hipStream_t s);
hipError_t gr_write(const uint64_t* node_base, uint64_t nb, const uint64_t* vals, const uint32_t* msz,
                    const uint8_t* tau, const uint64_t* pos, uint64_t* gr, hipStream_t s);
hipError_t ef_write(const uint64_t* x, uint64_t N, uint32_t L, uint64_t* lower, uint64_t* upper,
                    hipStream_t s);

// Select support: every 2^kSampleShift-th one of a bit vector.
hipError_t select_samples(const uint64_t* words, uint64_t nwords, uint64_t* scratch_counts,
                          uint64_t* scratch_prefix, uint64_t* scan_tmp, uint64_t* samples,
                          uint64_t nsamples, hipStream_t s);

struct EFView {
  const uint64_t* lower;
  const uint64_t* upper;
  const uint64_t* samples;
  uint64_t N;
  uint32_t L;
};

// One select sample (the position of a one) every 2^kSampleShift ones of an
// Elias-Fano upper vector.
constexpr uint32_t kSampleShift = 5;

struct QueryParams {
  EFView C, P;
  // the two sequences decoded, (C_j, P_j) for j = 0..nb, or null: read them
  // through C and P
  const uint64_t* offsets;
  const uint64_t* gr;
  uint64_t gr_bits;
  uint64_t nb;
  Shape shape;
  uint32_t rotation;
  const uint32_t* nodecnt;
  const uint32_t* fixedbits;
  const uint8_t* tau;
  const uint64_t* start;
  // ceil(2^32 / d) for d = l, la, ua: exact quotients of numerators below 2^14
  uint32_t magic_l, magic_la, magic_ua;
};

hipError_t launch_query(const QueryParams& q, const Key* keys, uint64_t n, uint64_t* out,
                        hipStream_t s);
// out[2j] = C_j, out[2j+1] = P_j for j < N (both sequences hold N elements):
// through select samples, or (decode_pairs) straight from upper vectors of
// c_words and p_words words that hold exactly N ones each.
hipError_t decode_offsets(const EFView& C, const EFView& P, uint64_t N, uint64_t* out,
                          hipStream_t s);
hipError_t decode_pairs(const EFView& C, uint64_t c_words, const EFView& P, uint64_t p_words,
                        uint64_t* out, hipStream_t s);

}  // namespace rs
