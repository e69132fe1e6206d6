// Host-side state of the library: per-device constants, build contexts
// (stream + working memory), and the batch build used by the public entry
// points and by the construction server.
#pragma once

#include <mutex>
#include <vector>

#include "rs_launch.h"

namespace rs {

// Per-leaf-size tables, m = 0 .. kMaxBucketKeys: stored nodes of a subtree,
// Golomb-Rice fixed bits of a subtree, the Rice parameter of a node, and the
// expected evaluations of a failed split attempt (for the work counts).
struct Tables {
  uint32_t* nodecnt = nullptr;
  uint32_t* fixedbits = nullptr;
  uint8_t* tau = nullptr;
  uint32_t* split_work = nullptr;  // split_work_table in units of 2^-kLeafWorkShift
};

struct Device;

struct Buffer {
  void* p = nullptr;
  size_t cap = 0;
};

hipError_t ensure(Buffer& b, size_t bytes);

// A stream and its working memory; one build at a time per context.
struct Context {
  Device* dev = nullptr;
  hipStream_t s = nullptr;
  Buffer arena;                  // working memory of the current build (default contexts)
  Buffer out;                    // encoded words of the structure being finished
  Buffer qkeys, qout, sc_counts, sc_prefix, sc_tmp;
  hipEvent_t ev[6] = {};
  hipEvent_t upstream = nullptr;  // orders the context after the legacy default stream
  uint64_t* progress = nullptr;   // host-pinned finished count of the running search
  uint64_t* progress_dev = nullptr;  // its device address
  std::mutex mu;
};

// Read-only after initialisation; shared by every context on the device.
// The starting seeds and the tables live in the library's fixed device array
// (`scratch` in rs_api.hip), found at initialisation; so does the working
// memory of rs_build_noalloc, which builds through `noalloc` (its lock
// serialises those calls).
struct Device {
  bool ready = false;
  int id = 0;
  int cus = 0;
  int wall_khz = 100000;
  int lds_per_block = 65536;
  char* scratch = nullptr;    // device address of the fixed array on this device
  uint64_t* start = nullptr;  // starting seed of depth d: SplitMix64(0) output d+1
  Tables tables[kMaxLeaf + 1];
  std::mutex mu;  // guards lazy initialisation of the tables
  Context noalloc;
};

int device_get(Device** out);
int context_init(Context& c, Device* d);
void context_destroy(Context& c);

// One job of a build: inputs, slices of the shared arrays, outcome.
struct JobPlan {
  const Key* keys = nullptr;
  uint64_t n = 0;
  uint32_t l = 0, b = 0, flags = 0;
  uint64_t nb = 0;
  uint64_t key_base = 0, bucket_base = 0, off_base = 0, host_base = 0;
  uint64_t node_off = 0, total = 0;
  uint32_t maxm = 0;
  int status = RS_OK;
  Tables* T = nullptr;
  rs_mphf* out = nullptr;
  // rs_build_noalloc: the serialised words go to host_words (host_cap words)
  // through dev_words (dev_cap words of the fixed array) instead of a new
  // structure; nwords receives their count
  uint64_t* host_words = nullptr;
  uint64_t host_cap = 0, nwords = 0;
  uint64_t* dev_words = nullptr;
  uint64_t dev_cap = 0;
};

// Upper bound of the device working memory of a build of these jobs
// (stored nodes never exceed keys).
size_t batch_footprint(const std::vector<JobPlan>& jobs, uint32_t workers_max);

// Worker count of the search launch: the occupancy limit, or fewer.
uint32_t max_workers(const Device& d);

// Build every job whose status is RS_OK on entry, using `region` (at least
// batch_footprint bytes) for all working arrays, on the context's stream.
// `workers` caps the search grid (0: the occupancy limit).  Each job ends
// with its status and, on success, its structure.
int build_jobs(Context& c, std::vector<JobPlan>& jobs, void* region, size_t region_bytes,
               uint32_t workers);

Context* default_context(int* rc);

bool job_args_ok(const rs_key128* keys, uint64_t n, uint32_t l, uint32_t b, uint32_t flags);

void mphf_release(rs_mphf* f);

}  // namespace rs
