// C ABI of the library (include/recsplit.h): argument checks, device memory,
// kernel orchestration, serialisation.  Every step of the construction and
// of queries runs in the kernels of rs_prep.hip, rs_search.hip and
// rs_encode.hip; this file only launches them and moves results.
//
// Work runs on per-context non-blocking streams, so several builds (the
// construction server's slots) overlap on the device.  Before touching
// caller data a context waits for the work already queued on the legacy
// default stream (where torch puts its kernels unless told otherwise).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <mutex>
#include <thread>
#include <vector>

#include "rs_host.h"

using namespace rs;

namespace {

constexpr uint64_t kMagic = 0x31564C5053434552ull;  // "RECSPLV1"
constexpr uint64_t kVersion = 1;
constexpr uint32_t kHeaderWords = 5;
constexpr uint32_t kEfHeaderWords = 6;
constexpr size_t kAlign = 256;

constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// The library's fixed device array, one copy per device, held until the
// process ends.  It holds the starting seeds, the per-leaf-size tables (each
// written once, by the first build or query of its leaf size on the device)
// and, from kNoAllocAt on, the working memory and the encoded words of
// rs_build_noalloc.  Host code never takes the array's name as an address:
// device_get asks for its device address with hipGetSymbolAddress once per
// device, with that device current, and every use goes through
// Device::scratch.
constexpr size_t kScratchBytes = RS_NOALLOC_SCRATCH_BYTES;
constexpr size_t kSeedBytes = 4096;
constexpr size_t kTableSlot = 3 * align_up(kTable * sizeof(uint32_t)) + align_up(kTable);
constexpr size_t kNoAllocAt = kSeedBytes + (kMaxLeaf + 1) * kTableSlot;
static __device__ __align__(256) uint64_t scratch[kScratchBytes / sizeof(uint64_t)];

// Working memory of one job of RS_NOALLOC_MAX_KEYS keys at its most: host
// keys staged (16 B) and two sorted copies (32 B) per key, one bucket per key
// (24 B of sizes and lengths, 24 B of prefix sums and offsets), and per
// stored node (never more than keys) 72 B of value, size, task, state and
// flag; plus 1 MiB for the scan space, counters and worker table.  The
// encoded words take what is left (at least 8 MiB: several hundred bits per
// key, against the 1.5 to 2 bits per key that builds need).
constexpr size_t kNoAllocWorkBound = (size_t)(RS_NOALLOC_MAX_KEYS + 2) * 168 + (1u << 20);
static_assert(kSeedBytes >= kMaxDepth * sizeof(uint64_t), "seed space");
static_assert(kNoAllocAt + kNoAllocWorkBound + (8u << 20) <= kScratchBytes,
              "fixed array too small for RS_NOALLOC_MAX_KEYS keys");

int from_hip(hipError_t e) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return RS_ERR_OOM;
  return e == hipSuccess ? RS_OK : RS_ERR_DEVICE;
}

#define HIPCHECK(expr)                         \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return from_hip(e_); \
  } while (0)

// log of the probability that one trial succeeds at a node of size m: a leaf
// is a bijection with probability m!/m^m; a split hits its part sizes p_j
// with the multinomial probability m!/prod p_j! * prod (p_j/m)^p_j.
double log_success(const Shape& s, uint32_t m) {
  if (kind_of(s, m) == kLeaf) return lgamma((double)m + 1.0) - (double)m * log((double)m);
  Parts p = parts_of(s, m);
  double lp = lgamma((double)m + 1.0);
  for (uint32_t j = 0; j < p.k; ++j) {
    double sz = (double)part_size(p, j);
    lp += sz * log(sz / (double)m) - lgamma(sz + 1.0);
  }
  return lp;
}

// Rice parameter minimising the expected code length of a geometric value
// with success probability p (Kiely 2004): max(0, 1 + floor(log2(ln(phi-1) /
// ln(1-p)))).  It sets the fixed width of each node's value (Sec. 2.2:
// precomputed per layer).
uint32_t rice_parameter(double log_p) {
  const double p = exp(log_p);
  const double ratio = log((sqrt(5.0) - 1.0) * 0.5) / log1p(-p);
  const double t = 1.0 + floor(log2(ratio));
  return t < 0.0 ? 0u : (uint32_t)t;
}

void compute_tables(uint32_t l, std::vector<uint32_t>& nodecnt, std::vector<uint32_t>& fixedbits,
                    std::vector<uint8_t>& tau) {
  const Shape s = make_shape(l);
  nodecnt.assign(kTable, 0);
  fixedbits.assign(kTable, 0);
  tau.assign(kTable, 0);
  for (uint32_t m = 2; m < kTable; ++m) {
    const uint32_t t = rice_parameter(log_success(s, m));
    tau[m] = (uint8_t)t;
    uint32_t nc = 1, fb = t;
    Parts p = parts_of(s, m);
    for (uint32_t j = 0; j < p.k; ++j) {
      const uint32_t sz = part_size(p, j);
      nc += nodecnt[sz];
      fb += fixedbits[sz];
    }
    nodecnt[m] = nc;
    fixedbits[m] = fb;
  }
}

uint64_t splitmix_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  return mix64(state);
}

Device g_dev[64];
std::mutex g_devices_mu;
Context g_default[64];

// autotune.py on an MI355X; leaf_filter_tau = 19 filters leaves of 16 keys and
// more (l = 16, b = 2000: 0.9 %; b = 100: 6 %; l = 18 and 20: 1.7-1.8x) and
// keeps smaller leaf sizes on the plain kernel (their leaves are too short);
// join_leaf_tau = 22: leaves of 18 keys and more are joined in small launches
// (3x to 6x on a few thousand leaves of 22 or 24 keys); split_filter_tau = 16:
// l = 16, b = 2000 8 % faster, while the shorter split searches of l <= 12
// lose 1.5-2.6 % to it
constexpr rs_schedule kDefaultSchedule = {63, 4, 13, 12, 4, 16, 8, 8, 0, 0, 19, 22, 16, 0, 1};
rs_schedule g_schedule = kDefaultSchedule;
std::mutex g_schedule_mu;

rs_schedule current_schedule() {
  std::lock_guard<std::mutex> lock(g_schedule_mu);
  return g_schedule;
}

// split_work_table per leaf size, computed once per process
const std::vector<double>& split_work_cached(uint32_t l) {
  static std::mutex mu;
  static std::vector<double> tables[kMaxLeaf + 1];
  std::lock_guard<std::mutex> lock(mu);
  if (tables[l].empty()) tables[l] = split_work_table(l);
  return tables[l];
}

int tables_for(Device& d, uint32_t l, Tables** out) {
  std::lock_guard<std::mutex> lock(d.mu);
  Tables& t = d.tables[l];
  if (!t.nodecnt) {
    std::vector<uint32_t> nc, fb;
    std::vector<uint8_t> tau;
    compute_tables(l, nc, fb, tau);
    const std::vector<double>& sw = split_work_cached(l);
    std::vector<uint32_t> swfx(kTable);
    for (uint32_t m = 0; m < kTable; ++m) swfx[m] = (uint32_t)llround(ldexp(sw[m], kLeafWorkShift));
    char* slot = d.scratch + kSeedBytes + (size_t)l * kTableSlot;
    const size_t w32 = align_up(kTable * sizeof(uint32_t));
    uint32_t* a = reinterpret_cast<uint32_t*>(slot);
    uint32_t* b = reinterpret_cast<uint32_t*>(slot + w32);
    uint32_t* w = reinterpret_cast<uint32_t*>(slot + 2 * w32);
    uint8_t* c = reinterpret_cast<uint8_t*>(slot + 3 * w32);
    HIPCHECK(hipMemcpy(a, nc.data(), kTable * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b, fb.data(), kTable * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(w, swfx.data(), kTable * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(c, tau.data(), kTable, hipMemcpyHostToDevice));
    t.fixedbits = b;
    t.split_work = w;
    t.tau = c;
    t.nodecnt = a;  // last: a non-null nodecnt means the table is complete
  }
  *out = &t;
  return RS_OK;
}

uint32_t ef_lowbits(uint64_t N, uint64_t U) {
  uint32_t L = 0;
  while (L < 63 && (U >> (L + 1)) >= N) ++L;
  return L;
}

struct EFLayout {
  uint64_t N, U, L, lw, ub, uw;
  uint64_t at;  // word offset of the section header
  uint64_t words() const { return kEfHeaderWords + lw + uw; }
};

EFLayout ef_layout(uint64_t N, uint64_t U, uint64_t at) {
  EFLayout e;
  e.N = N;
  e.U = U;
  e.L = ef_lowbits(N, U);
  e.lw = (N * e.L + 63) / 64;
  e.ub = (U >> e.L) + N;
  e.uw = (e.ub + 63) / 64;
  e.at = at;
  return e;
}

// Hands out aligned slices of one device region; `failed` records a slice
// that did not fit.
struct Carver {
  char* base;
  size_t cap, used = 0;
  bool failed = false;
  template <typename T>
  T* take(uint64_t count) {
    size_t bytes = (size_t)(count ? count : 1) * sizeof(T);
    used = (used + kAlign - 1) / kAlign * kAlign;
    if (used + bytes > cap) {
      failed = true;
      return nullptr;
    }
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

hipError_t d2h(Context& c, void* dst, const void* src, size_t bytes) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.s);
  return e == hipSuccess ? hipStreamSynchronize(c.s) : e;
}

// Order the context after the work already queued on the legacy default stream.
hipError_t after_default_stream(Context& c) {
  hipError_t e = hipEventRecord(c.upstream, 0);
  return e == hipSuccess ? hipStreamWaitEvent(c.s, c.upstream, 0) : e;
}

}  // namespace

// A structure: its serialised words on the host; the device copy queries
// use (with select samples) is made by the first rs_query, or by
// rs_deserialize, which validates it there.  Builds allocate nothing per
// structure on the device, so a finished build frees no device memory (a
// device free waits for every stream of the device).
struct rs_mphf {
  std::vector<uint64_t> words;
  uint64_t n = 0, nb = 0;
  uint32_t l = 0, b = 0, rotation = 0;
  EFLayout efc{}, efp{};
  uint64_t gr_at = 0, gr_bits = 0, gr_words = 0;
  int device = 0;
  std::mutex dev_mu;  // guards the lazily made device copy
  bool dev_ready = false;
  bool encoded = false;  // made by this library's encoder (not deserialised)
  uint64_t* d_mem = nullptr;      // the device copy, one allocation:
  uint64_t* d_words = nullptr;    //   the words,
  uint64_t* d_samples = nullptr;  //   select samples of C, then of P,
  uint64_t* d_offsets = nullptr;  //   (C_j, P_j) decoded, when no larger than the words
  uint64_t ns_c = 0, ns_p = 0;
  rs_stats stats{};
  std::vector<uint64_t> keep_vals, keep_base;
};

namespace rs {

hipError_t ensure(Buffer& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return hipSuccess;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  size_t want = bytes + bytes / 4;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    return e;
  }
  b.cap = want;
  return hipSuccess;
}

int device_get(Device** out) {
  int id = 0;
  HIPCHECK(hipGetDevice(&id));
  if (id < 0 || id >= 64) return RS_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_devices_mu);
  Device& d = g_dev[id];
  if (!d.ready) {
    d.id = id;
    HIPCHECK(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, id));
    if (hipDeviceGetAttribute(&d.lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, id) !=
            hipSuccess ||
        d.lds_per_block <= 0)
      d.lds_per_block = 65536;
    if (hipDeviceGetAttribute(&d.wall_khz, hipDeviceAttributeWallClockRate, id) != hipSuccess ||
        d.wall_khz <= 0)
      d.wall_khz = 100000;
    // this device's copy of the fixed array (the array's name is no device
    // address in host code)
    void* fixed = nullptr;
    HIPCHECK(hipGetSymbolAddress(&fixed, HIP_SYMBOL(scratch)));
    if (!fixed) return RS_ERR_DEVICE;
    d.scratch = static_cast<char*>(fixed);
    uint64_t h[kMaxDepth], st = 0;
    for (uint32_t i = 0; i < kMaxDepth; ++i) h[i] = splitmix_next(st);
    d.start = reinterpret_cast<uint64_t*>(d.scratch);
    HIPCHECK(hipMemcpy(d.start, h, sizeof h, hipMemcpyHostToDevice));
    HIPCHECK(upload_rotation_tables());
    int rc = context_init(d.noalloc, &d);
    if (rc) return rc;
    d.ready = true;
  }
  *out = &d;
  return RS_OK;
}

int context_init(Context& c, Device* d) {
  c.dev = d;
  HIPCHECK(hipStreamCreateWithFlags(&c.s, hipStreamNonBlocking));
  for (int i = 0; i < 6; ++i) HIPCHECK(hipEventCreate(&c.ev[i]));
  HIPCHECK(hipEventCreateWithFlags(&c.upstream, hipEventDisableTiming));
  return RS_OK;
}

void context_destroy(Context& c) {
  if (c.s) (void)hipStreamSynchronize(c.s);
  Buffer* bs[] = {&c.arena, &c.out, &c.qkeys, &c.qout, &c.sc_counts, &c.sc_prefix, &c.sc_tmp};
  for (Buffer* b : bs) {
    if (b->p) (void)hipFree(b->p);
    b->p = nullptr;
    b->cap = 0;
  }
  for (hipEvent_t& e : c.ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (c.upstream) (void)hipEventDestroy(c.upstream);
  c.upstream = nullptr;
  if (c.progress) (void)hipHostFree(c.progress);
  c.progress = c.progress_dev = nullptr;
  if (c.s) (void)hipStreamDestroy(c.s);
  c.s = nullptr;
}

Context* default_context(int* rc) {
  Device* d = nullptr;
  *rc = device_get(&d);
  if (*rc) return nullptr;
  Context& c = g_default[d->id];
  std::lock_guard<std::mutex> lock(g_devices_mu);
  if (!c.dev) {
    *rc = context_init(c, d);
    if (*rc) return nullptr;
  }
  return &c;
}

bool job_args_ok(const rs_key128* keys, uint64_t n, uint32_t l, uint32_t b, uint32_t flags) {
  return l >= 2 && l <= kMaxLeaf && b >= 1 && b <= RS_MAX_BUCKET_SIZE && n < (1ull << 40) &&
         (!n || keys) &&
         !(flags & ~(uint32_t)(RS_FLAG_ROTATION | RS_FLAG_KEYS_ON_DEVICE | RS_FLAG_KEEP_VALUES));
}

void mphf_release(rs_mphf* f) {
  if (!f) return;
  if (f->d_mem) (void)hipFree(f->d_mem);
  delete f;
}

uint32_t max_workers(const Device& d) {
  // occupancy of the search kernel with a small stage: the most workers any launch uses
  int per_cu = 0;
  if (search_occupancy(64 * sizeof(uint64_t), &per_cu) != hipSuccess || per_cu < 1) per_cu = 8;
  return (uint32_t)per_cu * (uint32_t)d.cus;
}

size_t batch_footprint(const std::vector<JobPlan>& jobs, uint32_t workers_max) {
  uint64_t n = 0, nb = 0, noff = 0, nhost = 0, max_nb = 1;
  for (const JobPlan& j : jobs) {
    if (j.status) continue;
    const uint64_t jb = j.n ? (j.n + j.b - 1) / j.b : 1;
    n += j.n;
    nb += jb;
    noff += jb + 1;
    if (!(j.flags & RS_FLAG_KEYS_ON_DEVICE)) nhost += j.n;
    max_nb = jb > max_nb ? jb : max_nb;
  }
  const uint64_t nodes = n + 1;  // stored nodes never exceed keys
  size_t bytes = 0;
  bytes += (nhost + 2 * n) * sizeof(Key);
  bytes += nb * (2 * sizeof(uint32_t) + 2 * sizeof(uint64_t));
  bytes += noff * 3 * sizeof(uint64_t);
  bytes += scan_tmp_words(max_nb + 1) * sizeof(uint64_t);
  bytes += nodes * (sizeof(uint64_t) + sizeof(uint32_t) + sizeof(Task) + sizeof(TaskState) +
                    sizeof(uint32_t));
  bytes += sizeof(Control) + jobs.size() * (sizeof(JobInfo) + sizeof(JobDev));
  bytes += (size_t)workers_max * sizeof(int32_t);
  bytes += 24 * kAlign;
  return bytes;
}

}  // namespace rs

namespace {

// The device views of the two Elias-Fano sequences of an attached structure.
void ef_views(const rs_mphf* f, EFView* C, EFView* P) {
  C->lower = f->d_words + f->efc.at + kEfHeaderWords;
  C->upper = C->lower + f->efc.lw;
  C->samples = f->d_samples;
  C->N = f->efc.N;
  C->L = (uint32_t)f->efc.L;
  P->lower = f->d_words + f->efp.at + kEfHeaderWords;
  P->upper = P->lower + f->efp.lw;
  P->samples = f->d_samples + f->ns_c;
  P->N = f->efp.N;
  P->L = (uint32_t)f->efp.L;
}

// The device copy a query reads: the serialised words, and the bucket
// offsets decoded into pairs or select samples of both upper vectors;
// deserialised words are checked to hold exactly N ones in each upper vector.
// Caller holds f->dev_mu.
int attach_device(Context& c, rs_mphf* f) {
  const uint64_t nw = f->words.size();
  f->ns_c = (f->efc.N + (1u << kSampleShift) - 1) >> kSampleShift;
  f->ns_p = (f->efp.N + (1u << kSampleShift) - 1) >> kSampleShift;
  // Both sequences decoded into one array when it is no larger than the
  // structure (or 1 MiB): a query then reads C_j, P_j and C_{j+1} with two
  // loads instead of three selects.
  const uint64_t N = f->efc.N;
  const bool decode = N == f->efp.N && N * 16 <= (nw * 8 > (1u << 20) ? nw * 8 : (1u << 20));
  // one allocation: the words, the samples, the decoded pairs
  const uint64_t ns = f->ns_c + f->ns_p + 2;
  f->d_mem = nullptr;
  HIPCHECK(hipMalloc(&f->d_mem, (nw + ns + (decode ? 2 * N : 0)) * sizeof(uint64_t)));
  f->d_words = f->d_mem;
  f->d_samples = f->d_mem + nw;
  f->d_offsets = decode ? f->d_samples + ns : nullptr;
  HIPCHECK(hipMemcpyAsync(f->d_words, f->words.data(), nw * sizeof(uint64_t),
                          hipMemcpyHostToDevice, c.s));
  if (decode && f->encoded) {
    // the encoder's own sequences: decoded in one launch, no select support
    // (the query reads only the pairs)
    EFView C, P;
    ef_views(f, &C, &P);
    HIPCHECK(decode_pairs(C, f->efc.uw, P, f->efp.uw, f->d_offsets, c.s));
    HIPCHECK(hipStreamSynchronize(c.s));
    f->device = c.dev->id;
    f->dev_ready = true;
    return RS_OK;
  }
  const EFLayout* efs[2] = {&f->efc, &f->efp};
  uint64_t* samp[2] = {f->d_samples, f->d_samples + f->ns_c};
  uint64_t nsamp[2] = {f->ns_c, f->ns_p};
  for (int i = 0; i < 2; ++i) {
    const EFLayout& e = *efs[i];
    const uint64_t* upper = f->d_words + e.at + kEfHeaderWords + e.lw;
    HIPCHECK(ensure(c.sc_counts, (e.uw + 1) * sizeof(uint64_t)));
    HIPCHECK(ensure(c.sc_prefix, (e.uw + 1) * sizeof(uint64_t)));
    HIPCHECK(ensure(c.sc_tmp, scan_tmp_words(e.uw + 1) * sizeof(uint64_t)));
    uint64_t* prefix = static_cast<uint64_t*>(c.sc_prefix.p);
    HIPCHECK(select_samples(upper, e.uw, static_cast<uint64_t*>(c.sc_counts.p), prefix,
                            static_cast<uint64_t*>(c.sc_tmp.p), samp[i], nsamp[i], c.s));
    // Bytes from outside (rs_deserialize) must hold exactly N ones in each
    // upper vector before a select may run over them; the encoder's own
    // words need no check (and no wait).
    if (!f->encoded) {
      uint64_t ones = 0;
      if (e.uw) HIPCHECK(d2h(c, &ones, prefix + e.uw, sizeof ones));
      if (ones != e.N) return RS_ERR_CORRUPT;
    }
  }
  if (decode) {
    EFView C, P;
    ef_views(f, &C, &P);
    HIPCHECK(decode_offsets(C, P, N, f->d_offsets, c.s));
  }
  // complete before any other stream may query the copy
  HIPCHECK(hipStreamSynchronize(c.s));
  f->device = c.dev->id;
  f->dev_ready = true;
  return RS_OK;
}

// Device pointers of one build, carved from its region.
struct Arrays {
  Key *keys_in, *k0, *k1;
  uint32_t *cnt, *fill;
  uint64_t *nodes, *len, *off, *node_base, *pos, *tmp;
  uint64_t* vals;
  uint32_t* msz;
  Task* tasks;
  TaskState* states;
  uint32_t *ready, *active_u32;
  Control* ctl;
  JobInfo* jinfo;
  JobDev* jobs;
};

hipError_t h2d_async(Context& c, void* dst, const void* src, size_t bytes) {
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c.s);
}

// Encoding, first half, for every job that succeeded: the record length of
// every bucket and their offsets; each job's record bits go to its
// JobInfo::gr_bits, read back with the other per-job results.
int encode_lengths(Context& c, const Arrays& A, const std::vector<JobPlan>& jobs) {
  const hipStream_t s = c.s;
  for (size_t i = 0; i < jobs.size(); ++i) {
    const JobPlan& jp = jobs[i];
    if (jp.status) continue;
    const uint64_t nb = jp.nb;
    const uint64_t* node_base = A.node_base + jp.off_base;
    uint64_t* len = A.len + jp.bucket_base;
    uint64_t* pos = A.pos + jp.off_base;
    if (jp.total == 0) HIPCHECK(fill_u64(len, nb, 0, s));
    else HIPCHECK(gr_lengths(node_base, nb, A.vals + jp.node_off, A.msz + jp.node_off, jp.T->tau,
                             len, s));
    HIPCHECK(scan_excl_u64(len, nb, pos, A.tmp, s));
    HIPCHECK(hipMemcpyAsync(&A.jinfo[i].gr_bits, pos + nb, sizeof(uint64_t),
                            hipMemcpyDeviceToDevice, s));
  }
  return RS_OK;
}

// Where one job's serialised words go: a new structure's host words, or
// (rs_build_noalloc) the caller's buffer; the device words they are
// assembled in.
struct Out {
  rs_mphf* f = nullptr;
  uint64_t* hw = nullptr;
  uint64_t* dw = nullptr;
  uint64_t nw = 0;
  EFLayout efc{}, efp{};
  uint64_t gr_at = 0, gr_bits = 0, gr_words = 0;
};

// Encoding, second half: header words, Golomb-Rice records and both
// Elias-Fano sequences of every job that succeeded, assembled on the device
// and copied to the host, with one wait at the end.  Sets each job's status
// and, on success, its structure.
void encode_words(Context& c, const Arrays& A, std::vector<JobPlan>& jobs,
                  const std::vector<JobInfo>& info, double ms_sort, double ms_search,
                  uint32_t workers) {
  const hipStream_t s = c.s;
  const size_t nj = jobs.size();
  std::vector<Out> outs(nj);
  uint64_t own_words = 0;  // device words of the jobs that get a new structure
  for (size_t i = 0; i < nj; ++i) {
    JobPlan& jp = jobs[i];
    if (jp.status) continue;
    Out& o = outs[i];
    o.gr_bits = info[i].gr_bits;
    o.efc = ef_layout(jp.nb + 1, jp.n, kHeaderWords);
    o.efp = ef_layout(jp.nb + 1, o.gr_bits, o.efc.at + o.efc.words());
    o.gr_at = o.efp.at + o.efp.words();
    o.gr_words = (o.gr_bits + 63) / 64;
    o.nw = o.gr_at + 2 + o.gr_words;
    if (jp.host_words) {
      jp.nwords = o.nw;
      if (o.nw > jp.host_cap) jp.status = RS_ERR_INVALID_ARG;
      else if (o.nw > jp.dev_cap) jp.status = RS_ERR_OOM;
      o.hw = jp.host_words;
      o.dw = jp.dev_words;
    } else {
      own_words += o.nw;
    }
  }
  auto fail_all = [&](int code) {
    for (size_t i = 0; i < nj; ++i) {
      if (jobs[i].status) continue;
      mphf_release(outs[i].f);
      outs[i].f = nullptr;
      jobs[i].status = code;
    }
  };
  if (own_words && ensure(c.out, own_words * sizeof(uint64_t)) != hipSuccess) {
    fail_all(RS_ERR_OOM);
    return;
  }
  uint64_t at = 0;
  for (size_t i = 0; i < nj; ++i) {
    JobPlan& jp = jobs[i];
    if (jp.status || jp.host_words) continue;
    Out& o = outs[i];
    o.dw = static_cast<uint64_t*>(c.out.p) + at;
    at += o.nw;
    rs_mphf* f = new (std::nothrow) rs_mphf();
    if (!f) {
      fail_all(RS_ERR_OOM);
      return;
    }
    f->n = jp.n;
    f->nb = jp.nb;
    f->l = jp.l;
    f->b = jp.b;
    f->rotation = (jp.flags & RS_FLAG_ROTATION) ? 1u : 0u;
    f->device = c.dev->id;
    f->efc = o.efc;
    f->efp = o.efp;
    f->gr_at = o.gr_at;
    f->gr_bits = o.gr_bits;
    f->gr_words = o.gr_words;
    f->encoded = true;
    f->words.assign(o.nw, 0);
    o.f = f;
    o.hw = f->words.data();
  }
  bool ok = hipEventRecord(c.ev[4], s) == hipSuccess;
  for (size_t i = 0; ok && i < nj; ++i) {
    JobPlan& jp = jobs[i];
    if (jp.status) continue;
    const Out& o = outs[i];
    const uint32_t rotation = (jp.flags & RS_FLAG_ROTATION) ? 1u : 0u;
    // header words, staged in the host words (alive until the copies end)
    const uint64_t hdr[kHeaderWords] = {kMagic, kVersion | ((uint64_t)rotation << 32), jp.n,
                                        (uint64_t)jp.l | ((uint64_t)jp.b << 32), jp.nb};
    memcpy(o.hw, hdr, sizeof hdr);
    const EFLayout* efs[2] = {&o.efc, &o.efp};
    for (int k = 0; k < 2; ++k) {
      const EFLayout& e = *efs[k];
      const uint64_t eh[6] = {e.N, e.U, e.L, e.lw, e.ub, e.uw};
      memcpy(o.hw + e.at, eh, sizeof eh);
    }
    o.hw[o.gr_at] = o.gr_bits;
    o.hw[o.gr_at + 1] = o.gr_words;
    // zero the structure, place the headers; kernels write the rest
    ok = fill_u64(o.dw, o.nw, 0, s) == hipSuccess &&
         h2d_async(c, o.dw, o.hw, kHeaderWords * 8) == hipSuccess;
    for (int k = 0; ok && k < 2; ++k)
      ok = h2d_async(c, o.dw + efs[k]->at, o.hw + efs[k]->at, kEfHeaderWords * 8) == hipSuccess;
    ok = ok && h2d_async(c, o.dw + o.gr_at, o.hw + o.gr_at, 16) == hipSuccess;
    if (ok && jp.total)
      ok = gr_write(A.node_base + jp.off_base, jp.nb, A.vals + jp.node_off, A.msz + jp.node_off,
                    jp.T->tau, A.pos + jp.off_base, o.dw + o.gr_at + 2, s) == hipSuccess;
    const uint64_t* xs[2] = {A.off + jp.off_base, A.pos + jp.off_base};
    for (int k = 0; ok && k < 2; ++k) {
      const EFLayout& e = *efs[k];
      ok = ef_write(xs[k], e.N, (uint32_t)e.L, o.dw + e.at + kEfHeaderWords,
                    o.dw + e.at + kEfHeaderWords + e.lw, s) == hipSuccess;
    }
  }
  ok = ok && hipEventRecord(c.ev[5], s) == hipSuccess;
  for (size_t i = 0; ok && i < nj; ++i) {
    JobPlan& jp = jobs[i];
    if (jp.status) continue;
    Out& o = outs[i];
    ok = hipMemcpyAsync(o.hw, o.dw, o.nw * 8, hipMemcpyDeviceToHost, s) == hipSuccess;
    if (ok && (jp.flags & RS_FLAG_KEEP_VALUES)) {
      o.f->keep_vals.resize(jp.total);
      o.f->keep_base.resize(jp.nb + 1);
      ok = (!jp.total || hipMemcpyAsync(o.f->keep_vals.data(), A.vals + jp.node_off, jp.total * 8,
                                        hipMemcpyDeviceToHost, s) == hipSuccess) &&
           hipMemcpyAsync(o.f->keep_base.data(), A.node_base + jp.off_base, (jp.nb + 1) * 8,
                          hipMemcpyDeviceToHost, s) == hipSuccess;
    }
  }
  ok = ok && hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    fail_all(RS_ERR_DEVICE);
    return;
  }
  float ms_enc = 0, ms_all = 0;
  (void)hipEventElapsedTime(&ms_enc, c.ev[4], c.ev[5]);
  (void)hipEventElapsedTime(&ms_all, c.ev[0], c.ev[5]);
  for (size_t i = 0; i < nj; ++i) {
    JobPlan& jp = jobs[i];
    if (jp.status || !outs[i].f) continue;
    const JobInfo& in = info[i];
    rs_stats& st = outs[i].f->stats;
    memset(&st, 0, sizeof st);
    st.n = jp.n;
    st.nb = jp.nb;
    st.nodes = jp.total;
    st.split_nodes = in.splits;
    st.leaf_nodes = in.leaves;
    st.useful_evals_split = in.evals_split;
    st.useful_evals_leaf = in.evals_leaf;
    st.early_exit_evals_leaf = ldexp((double)in.early_exit_leaf_fx, -(int)kLeafWorkShift);
    st.early_exit_evals_split = ldexp((double)in.early_exit_split_fx, -(int)kLeafWorkShift);
    st.gr_bits = outs[i].gr_bits;
    st.bytes = outs[i].nw * 8;
    st.max_bucket = jp.maxm;
    st.workers = workers;
    st.ms_sort = ms_sort;
    st.ms_search = ms_search;
    st.ms_encode = ms_enc;
    st.ms_total = ms_all;
    jp.out = outs[i].f;
  }
}

}  // namespace

namespace rs {

// Seconds between progress lines during a search (RS_PROGRESS; 0: none).
double progress_every() {
  const char* e = getenv("RS_PROGRESS");
  const double v = e ? atof(e) : 0.0;
  return v > 0.0 ? v : 0.0;
}

// Wait for the search to end, printing the finished node count to stderr
// every `every` seconds (the search kernels store it into the context's
// host-pinned word every 2^kProgressShift nodes).
void wait_with_progress(Context& c, uint64_t total, double every) {
  using clock = std::chrono::steady_clock;
  const clock::time_point t0 = clock::now();
  double next = every;
  uint64_t seen = 0;
  while (hipEventQuery(c.ev[4]) == hipErrorNotReady) {
    std::this_thread::sleep_for(std::chrono::milliseconds(20));
    const double el = std::chrono::duration<double>(clock::now() - t0).count();
    if (el < next) continue;
    const uint64_t f = __atomic_load_n(c.progress, __ATOMIC_RELAXED);
    if (f > seen) seen = f;
    fprintf(stderr, "[rs progress] search: %llu of %llu nodes final after %.0f s\n",
            (unsigned long long)seen, (unsigned long long)total, el);
    fflush(stderr);
    next += every;
  }
}

int build_jobs(Context& c, std::vector<JobPlan>& jobs, void* region, size_t region_bytes,
               uint32_t workers_cap) {
  Device& d = *c.dev;
  const hipStream_t s = c.s;
  const uint32_t nj = (uint32_t)jobs.size();
  uint64_t nkeys = 0, nbk = 0, noff = 0, nhost = 0, max_nb = 1;
  for (JobPlan& j : jobs) {
    if (j.status) continue;
    j.nb = j.n ? (j.n + j.b - 1) / j.b : 1;
    j.key_base = nkeys;
    j.bucket_base = nbk;
    j.off_base = noff;
    j.host_base = nhost;
    nkeys += j.n;
    nbk += j.nb;
    noff += j.nb + 1;
    if (!(j.flags & RS_FLAG_KEYS_ON_DEVICE)) nhost += j.n;
    max_nb = j.nb > max_nb ? j.nb : max_nb;
    int rc = tables_for(d, j.l, &j.T);
    if (rc) return rc;
  }
  const rs_schedule sched = current_schedule();
  const uint32_t wmax = max_workers(d);
  uint32_t workers = workers_cap && workers_cap < wmax ? workers_cap : wmax;
  if (sched.max_workers && sched.max_workers < workers) workers = sched.max_workers;
  if (batch_footprint(jobs, wmax) > region_bytes) return RS_ERR_OOM;
  Carver cv{static_cast<char*>(region), region_bytes};
  Arrays A;
  A.keys_in = cv.take<Key>(nhost);
  A.k0 = cv.take<Key>(nkeys);
  A.k1 = cv.take<Key>(nkeys);
  A.cnt = cv.take<uint32_t>(nbk);
  A.fill = cv.take<uint32_t>(nbk);
  A.nodes = cv.take<uint64_t>(nbk);
  A.len = cv.take<uint64_t>(nbk);
  A.off = cv.take<uint64_t>(noff);
  A.node_base = cv.take<uint64_t>(noff);
  A.pos = cv.take<uint64_t>(noff);
  A.tmp = cv.take<uint64_t>(scan_tmp_words(max_nb + 1));
  A.ctl = cv.take<Control>(1);
  A.jinfo = cv.take<JobInfo>(nj);
  A.jobs = cv.take<JobDev>(nj);
  A.active_u32 = cv.take<uint32_t>(wmax);
  const uint64_t node_cap = nkeys + 1;
  A.vals = cv.take<uint64_t>(node_cap);
  A.msz = cv.take<uint32_t>(node_cap);
  A.tasks = cv.take<Task>(node_cap);
  A.states = cv.take<TaskState>(node_cap);
  A.ready = cv.take<uint32_t>(node_cap);
  if (cv.failed) return RS_ERR_OOM;

  HIPCHECK(hipEventRecord(c.ev[0], s));
  HIPCHECK(after_default_stream(c));
  for (JobPlan& j : jobs)
    if (!j.status && !(j.flags & RS_FLAG_KEYS_ON_DEVICE) && j.n)
      HIPCHECK(hipMemcpyAsync(A.keys_in + j.host_base, j.keys, j.n * sizeof(Key),
                              hipMemcpyHostToDevice, s));
  HIPCHECK(hipEventRecord(c.ev[1], s));

  // 1. buckets: sizes, borders, scatter, duplicate check, node counts, with
  // one wait for all of them.  The duplicate check's LDS is sized before the
  // bucket sizes are known, from the expected bucket size (b + 8 sqrt(b) + 32
  // keys, rounded up to a power of two, within the LDS of a block); a bucket
  // beyond it is checked after the wait, with a second one.
  HIPCHECK(fill_u64(reinterpret_cast<uint64_t*>(A.ctl), sizeof(Control) / 8, 0, s));
  HIPCHECK(fill_u64(reinterpret_cast<uint64_t*>(A.jinfo), nj * sizeof(JobInfo) / 8, 0, s));
  HIPCHECK(fill_u32(A.cnt, nbk, 0, s));
  HIPCHECK(fill_u32(A.fill, nbk, 0, s));
  uint32_t lds_keys = 1;  // the largest power of two of keys a block can sort
  while ((uint64_t)lds_keys * 2 * 8 + 1024 <= (uint64_t)d.lds_per_block) lds_keys *= 2;
  for (uint32_t i = 0; i < nj; ++i) {
    JobPlan& j = jobs[i];
    if (j.status) continue;
    const Key* kin = (j.flags & RS_FLAG_KEYS_ON_DEVICE) ? j.keys : A.keys_in + j.host_base;
    uint32_t* cnt = A.cnt + j.bucket_base;
    uint64_t* off = A.off + j.off_base;
    HIPCHECK(bucket_histogram(kin, j.n, j.nb, cnt, &A.jinfo[i].maxm, s));
    HIPCHECK(scan_excl_u32(cnt, j.nb, off, A.tmp, s));
    HIPCHECK(bucket_scatter(kin, j.n, j.nb, off, A.fill + j.bucket_base, A.k0 + j.key_base, s));
    const double want = j.b + 8.0 * sqrt((double)j.b) + 32.0;
    uint32_t cap = 64;
    while (cap < want && cap < lds_keys) cap *= 2;
    HIPCHECK(duplicate_check(A.k0 + j.key_base, off, j.nb, cap, &A.jinfo[i].error,
                             &A.jinfo[i].deferred, s));
    HIPCHECK(node_counts(cnt, j.nb, j.T->nodecnt, A.nodes + j.bucket_base, s));
    HIPCHECK(scan_excl_u64(A.nodes + j.bucket_base, j.nb, A.node_base + j.off_base, A.tmp, s));
    HIPCHECK(hipMemcpyAsync(&A.jinfo[i].nodes, A.node_base + j.off_base + j.nb, sizeof(uint64_t),
                            hipMemcpyDeviceToDevice, s));
  }
  std::vector<JobInfo> hinfo(nj);
  HIPCHECK(d2h(c, hinfo.data(), A.jinfo, nj * sizeof(JobInfo)));
  bool again = false;
  for (uint32_t i = 0; i < nj; ++i) {
    JobPlan& j = jobs[i];
    if (j.status) continue;
    j.maxm = hinfo[i].maxm;
    uint32_t p2 = 1;
    while (p2 < j.maxm) p2 <<= 1;
    // LDS of the duplicate check (next power of two) and of the search stage
    if (j.maxm > kMaxBucketKeys || (uint64_t)p2 * 8 + 1024 > (uint64_t)d.lds_per_block) {
      j.status = RS_ERR_UNSUPPORTED;
      continue;
    }
    if (hinfo[i].deferred && !hinfo[i].error) {
      HIPCHECK(duplicate_check(A.k0 + j.key_base, A.off + j.off_base, j.nb, p2,
                               &A.jinfo[i].error, &A.jinfo[i].deferred, s));
      again = true;
    }
  }
  if (again) HIPCHECK(d2h(c, hinfo.data(), A.jinfo, nj * sizeof(JobInfo)));
  uint64_t total = 0;
  uint32_t maxm = 0;
  for (uint32_t i = 0; i < nj; ++i) {
    JobPlan& j = jobs[i];
    if (j.status) continue;
    if (hinfo[i].error) {
      j.status = -(int)hinfo[i].error;
      continue;
    }
    j.total = hinfo[i].nodes;
    j.node_off = total;
    total += j.total;
    maxm = j.maxm > maxm ? j.maxm : maxm;
  }
  if (total >= (1ull << 31) || total > node_cap) return RS_ERR_UNSUPPORTED;
  HIPCHECK(hipEventRecord(c.ev[2], s));
  // whole-bucket workers for small leaves and small buckets: with four-wave
  // workers when there are enough buckets to keep every worker busy; with
  // one-wave workers also when every bucket is small (a tree of a few dozen
  // nodes built by one wave ends sooner than the same nodes passed between
  // workers through the queue, level by level)
  bool bucket_mode = sched.bucket_mode_max_leaf != 0 && maxm <= kBucketModeMaxKeys &&
                     (nbk >= 4ull * workers ||
                      (sched.bucket_wave && (nbk >= workers || maxm <= kWaveBucketSmall)));
  for (const JobPlan& j : jobs)
    if (!j.status && j.l > sched.bucket_mode_max_leaf) bucket_mode = false;

  // the filter kernel when split searches are filtered or some job's full
  // leaves reach leaf_filter_tau; LDS for the largest node's keys and for the
  // queues of a filtered leaf or split
  bool filter = false, wide = false;
  uint32_t words = maxm < 64 ? 64 : maxm;
  for (const JobPlan& j : jobs) {
    if (j.status || bucket_mode) continue;
    const Shape sh = make_shape(j.l);
    const bool leaves = sched.leaf_filter_tau &&
                        rice_parameter(log_success(sh, j.l)) >= sched.leaf_filter_tau;
    const bool splits = sched.split_filter_tau &&
                        (rice_parameter(log_success(sh, sh.la)) >= sched.split_filter_tau ||
                         rice_parameter(log_success(sh, sh.ua)) >= sched.split_filter_tau);
    if (leaves || splits) filter = true;
    // split counters of a full lower or upper node: k-1 fields of the bit
    // length of the part size; past 31 bits the wide kernel (64-bit words)
    auto field_bits = [](uint32_t k, uint32_t unit) {
      uint32_t fe = 0;
      while ((1u << fe) <= unit) ++fe;
      return (k - 1) * fe;
    };
    if (splits && (field_bits(sh.la / sh.l, sh.l) > 31 || field_bits(sh.ua / sh.la, sh.la) > 31))
      wide = true;
    if (leaves && words < kLeafFilterWords) words = kLeafFilterWords;
    if (splits) {
      const uint32_t ua = sh.ua;
      const uint32_t need = split_queue_at(ua < j.maxm ? ua : j.maxm) + kSplitQueueWords;
      if (words < need) words = need;
    }
  }
  const uint32_t mode = bucket_mode ? (sched.bucket_wave ? kSearchBucketWave : kSearchBucket)
                       : filter    ? (wide ? kSearchFilterWide : kSearchFilter)
                                   : kSearchNode;

  // 2. seed search over all nodes of all jobs, one persistent launch
  std::vector<JobDev> jd(nj);  // read by a copy that ends before the wait after the search
  // progress lines (the filter kernel, whose searches end within seconds,
  // does not report)
  double progress = mode == kSearchFilter ? 0.0 : progress_every();
  if (total) {
    const uint32_t lds = mode == kSearchBucketWave ? wave_bucket_lds_bytes(maxm)
                         : bucket_mode             ? bucket_lds_bytes(maxm)
                                                   : words * (uint32_t)sizeof(uint64_t);
    int per_cu = 0;
    HIPCHECK(search_occupancy(lds, &per_cu, mode));
    if (per_cu < 1) per_cu = 1;
    const uint32_t occ = (uint32_t)per_cu * (uint32_t)d.cus;
    // one-wave workers: four per four-wave worker the caps allow, and no more
    // than there are buckets (a wave without a bucket would only take a slot
    // on some compute unit that a working wave could have had to itself)
    if (mode == kSearchBucketWave) {
      workers *= 4;
      if ((uint64_t)workers > nbk) workers = (uint32_t)(nbk ? nbk : 1);
    }
    if (workers > occ) workers = occ;
    HIPCHECK(init_states(A.states, total, s));
    HIPCHECK(fill_u32(A.ready, total, 0, s));
    HIPCHECK(fill_u32(A.active_u32, workers < wmax ? workers : wmax, 0xFFFFFFFFu, s));
    for (uint32_t i = 0; i < nj; ++i) {
      JobPlan& j = jobs[i];
      JobDev& g = jd[i];
      memset(&g, 0, sizeof g);
      if (j.status) continue;
      g.keys[0] = A.k0 + j.key_base;
      g.keys[1] = A.k1 + j.key_base;
      g.info = A.jinfo + i;
      g.vals = A.vals + j.node_off;
      g.msz = A.msz + j.node_off;
      g.nodecnt = j.T->nodecnt;
      g.tau = j.T->tau;
      const Shape sh = make_shape(j.l);
      g.l = sh.l;
      g.la = sh.la;
      g.ua = sh.ua;
      g.rotation = (j.flags & RS_FLAG_ROTATION) ? 1u : 0u;
    }
    // (jd and total stay alive until the wait after the search)
    HIPCHECK(h2d_async(c, A.jobs, jd.data(), nj * sizeof(JobDev)));
    HIPCHECK(h2d_async(c, &A.ctl->total, &total, sizeof(uint64_t)));
    if (progress && &c != &d.noalloc) {
      if (!c.progress) {
        void* h = nullptr;
        HIPCHECK(hipHostMalloc(&h, 64, hipHostMallocMapped | hipHostMallocCoherent));
        c.progress = static_cast<uint64_t*>(h);
        void* dp = nullptr;
        HIPCHECK(hipHostGetDevicePointer(&dp, h, 0));
        c.progress_dev = static_cast<uint64_t*>(dp);
      }
      __atomic_store_n(c.progress, 0ull, __ATOMIC_RELAXED);
      HIPCHECK(h2d_async(c, &A.ctl->progress, &c.progress_dev, sizeof(uint64_t*)));
    } else {
      progress = 0.0;
    }
    for (uint32_t i = 0; i < nj; ++i) {
      JobPlan& j = jobs[i];
      if (j.status || !j.total) continue;
      HIPCHECK(queue_roots(A.cnt + j.bucket_base, A.off + j.off_base, A.node_base + j.off_base,
                           j.nb, i, 0, 0, A.tasks, A.ready, A.ctl, s));
    }
    SearchParams P;
    memset(&P, 0, sizeof P);
    P.jobs = A.jobs;
    P.tasks = A.tasks;
    P.states = A.states;
    P.ready = A.ready;
    P.active = reinterpret_cast<int32_t*>(A.active_u32);
    P.ctl = A.ctl;
    P.start = d.start;
    P.workers = workers;
    P.stage_cap = bucket_mode ? maxm : words;
    // chunking of split searches (the result does not depend on it)
    const bool small = total < (uint64_t)sched.small_tasks_per_worker * workers;
    P.chunk_shift = small ? sched.chunk_shift_small : sched.chunk_shift_large;
    P.help_after = small ? sched.help_after_small : sched.help_after_large;
    P.inline_leaf_tau = small ? sched.inline_leaf_tau_small : sched.inline_leaf_tau_large;
    P.mode = mode;
    P.cap_shift = 10;
    P.leaf_filter_tau = filter ? sched.leaf_filter_tau : 0u;
    // joined leaves pay claims and queue flushes per chunk: worth it only when
    // the leaves are too few to keep every worker busy to the end
    P.join_leaf_tau = small ? sched.join_leaf_tau : 0u;
    P.split_filter_tau = filter ? sched.split_filter_tau : 0u;
    P.rotation_lookup = sched.rotation_lookup;
    // s_memrealtime ticks (wall_khz per millisecond)
    P.stall_ticks = sched.stall_guard_us ? (uint64_t)d.wall_khz * sched.stall_guard_us / 1000ull
                                         : (uint64_t)d.wall_khz * 1000ull * 10ull;
    if (P.stall_ticks < 1) P.stall_ticks = 1;
    HIPCHECK(hipEventRecord(c.ev[3], s));
    HIPCHECK(launch_search(P, workers, lds, s));
  } else {
    HIPCHECK(hipEventRecord(c.ev[3], s));
  }
  HIPCHECK(hipEventRecord(c.ev[4], s));
  if (progress > 0.0) wait_with_progress(c, total, progress);
  // useful work of every job, counted from its node values, and the length
  // of every bucket's record (both harmless after a stopped search, whose
  // results are dropped), read back with the control block in one wait
  for (uint32_t i = 0; i < nj; ++i) {
    const JobPlan& j = jobs[i];
    if (j.status || !j.total) continue;
    HIPCHECK(work_counts(A.vals + j.node_off, A.msz + j.node_off, j.total, j.l,
                         (j.flags & RS_FLAG_ROTATION) ? 1u : 0u, j.T->split_work, A.jinfo + i, s));
  }
  const int enc_rc = encode_lengths(c, A, jobs);
  if (enc_rc) return enc_rc;
  Control h_ctl;
  HIPCHECK(hipMemcpyAsync(&h_ctl, A.ctl, sizeof h_ctl, hipMemcpyDeviceToHost, s));
  HIPCHECK(d2h(c, hinfo.data(), A.jinfo, nj * sizeof(JobInfo)));
  if (h_ctl.error && getenv("RS_DEBUG")) {
    fprintf(stderr,
            "[rs debug] error %u: node %llu slot %llu m %u depth %u key_off %llu np %016llx "
            "best %llu chunk %llu finished %llu/%llu head %llu tail %llu\n",
            h_ctl.error, (unsigned long long)h_ctl.dbg_node, (unsigned long long)h_ctl.dbg_slot,
            h_ctl.dbg_m, h_ctl.dbg_depth, (unsigned long long)h_ctl.dbg_key_off,
            (unsigned long long)h_ctl.dbg_np, (unsigned long long)h_ctl.dbg_best,
            (unsigned long long)h_ctl.dbg_chunk, (unsigned long long)h_ctl.finished,
            (unsigned long long)total, (unsigned long long)h_ctl.head,
            (unsigned long long)h_ctl.tail);
  }
  int search_rc = RS_OK;
  if (h_ctl.error) search_rc = -(int)h_ctl.error;
  else if (h_ctl.finished != total) search_rc = RS_ERR_DEVICE;
  float ms_sort = 0, ms_search = 0;
  (void)hipEventElapsedTime(&ms_sort, c.ev[1], c.ev[2]);
  (void)hipEventElapsedTime(&ms_search, c.ev[3], c.ev[4]);
  if (search_rc) {
    for (JobPlan& j : jobs)
      if (!j.status) j.status = search_rc;
    return RS_OK;
  }

  // 3. encode every job that succeeded (its record bits came with the
  // status): the words (one wait)
  encode_words(c, A, jobs, hinfo, ms_sort, ms_search, workers);
  return RS_OK;
}

}  // namespace rs

namespace {

// Run a batch on the default context, in its growable working region.
int build_on_default(std::vector<JobPlan>& plan) {
  int rc = RS_OK;
  Context* c = default_context(&rc);
  if (!c) return rc;
  std::lock_guard<std::mutex> lock(c->mu);
  const size_t need = batch_footprint(plan, max_workers(*c->dev));
  HIPCHECK(ensure(c->arena, need));
  rc = build_jobs(*c, plan, c->arena.p, c->arena.cap, 0);
  if (rc) {
    // leave the stream usable for the next call
    (void)hipStreamSynchronize(c->s);
    (void)hipGetLastError();
  }
  return rc;
}

int parse(const uint64_t* w, uint64_t nw, rs_mphf* f) {
  if (nw < kHeaderWords || w[0] != kMagic || (w[1] & 0xFFFFFFFFull) != kVersion) return RS_ERR_CORRUPT;
  f->rotation = (uint32_t)((w[1] >> 32) & 1u);
  if (w[1] >> 33) return RS_ERR_CORRUPT;
  f->n = w[2];
  f->l = (uint32_t)(w[3] & 0xFFFFFFFFull);
  f->b = (uint32_t)(w[3] >> 32);
  f->nb = w[4];
  if (f->l < 2 || f->l > kMaxLeaf || f->b < 1 || f->b > RS_MAX_BUCKET_SIZE || f->n >= (1ull << 40))
    return RS_ERR_CORRUPT;
  const uint64_t nb = f->n ? (f->n + f->b - 1) / f->b : 1;
  if (f->nb != nb) return RS_ERR_CORRUPT;
  uint64_t at = kHeaderWords;
  EFLayout* efs[2] = {&f->efc, &f->efp};
  for (int i = 0; i < 2; ++i) {
    if (nw - at < kEfHeaderWords) return RS_ERR_CORRUPT;
    const uint64_t* h = w + at;
    if (h[0] != nb + 1 || h[2] > 63) return RS_ERR_CORRUPT;
    EFLayout e = ef_layout(h[0], h[1], at);
    if (e.L != h[2] || e.lw != h[3] || e.ub != h[4] || e.uw != h[5]) return RS_ERR_CORRUPT;
    if (nw - at < e.words()) return RS_ERR_CORRUPT;
    *efs[i] = e;
    at += e.words();
  }
  if (f->efc.U != f->n) return RS_ERR_CORRUPT;
  if (nw - at < 2) return RS_ERR_CORRUPT;
  f->gr_at = at;
  f->gr_bits = w[at];
  f->gr_words = w[at + 1];
  if (f->gr_words != (f->gr_bits + 63) / 64 || nw - at - 2 != f->gr_words) return RS_ERR_CORRUPT;
  if (f->efp.U != f->gr_bits) return RS_ERR_CORRUPT;
  return RS_OK;
}

}  // namespace

extern "C" {

int rs_build(const rs_key128* keys, uint64_t n, uint32_t leaf_size, uint32_t bucket_size,
             uint32_t flags, rs_mphf** out) {
  if (!out) return RS_ERR_INVALID_ARG;
  *out = nullptr;
  if (!job_args_ok(keys, n, leaf_size, bucket_size, flags)) return RS_ERR_INVALID_ARG;
  std::vector<JobPlan> plan(1);
  plan[0].keys = reinterpret_cast<const Key*>(keys);
  plan[0].n = n;
  plan[0].l = leaf_size;
  plan[0].b = bucket_size;
  plan[0].flags = flags;
  int rc = build_on_default(plan);
  if (rc) return rc;
  if (plan[0].status) return plan[0].status;
  *out = plan[0].out;
  return RS_OK;
}

int rs_build_noalloc(const rs_key128* keys, uint64_t n, uint32_t leaf_size, uint32_t bucket_size,
                     uint32_t flags, uint64_t* words, uint64_t cap_words, uint64_t* nwords) {
  if (!nwords) return RS_ERR_INVALID_ARG;
  *nwords = 0;
  if (!job_args_ok(keys, n, leaf_size, bucket_size, flags) || (flags & RS_FLAG_KEEP_VALUES) ||
      n > RS_NOALLOC_MAX_KEYS || !words || !cap_words)
    return RS_ERR_INVALID_ARG;
  Device* d = nullptr;
  int rc = device_get(&d);
  if (rc) return rc;
  Context& c = d->noalloc;
  std::lock_guard<std::mutex> lock(c.mu);
  std::vector<JobPlan> plan(1);
  JobPlan& j = plan[0];
  j.keys = reinterpret_cast<const Key*>(keys);
  j.n = n;
  j.l = leaf_size;
  j.b = bucket_size;
  j.flags = flags;
  j.host_words = words;
  j.host_cap = cap_words;
  // working memory, then the encoded words, in the fixed array after the
  // seeds and tables
  const size_t work = batch_footprint(plan, max_workers(*d));
  if (work > kNoAllocWorkBound) return RS_ERR_INVALID_ARG;
  const size_t out_at = align_up(kNoAllocAt + work);
  j.dev_words = reinterpret_cast<uint64_t*>(d->scratch + out_at);
  j.dev_cap = (kScratchBytes - out_at) / sizeof(uint64_t);
  rc = build_jobs(c, plan, d->scratch + kNoAllocAt, work, 0);
  if (rc) {
    (void)hipStreamSynchronize(c.s);
    (void)hipGetLastError();
    return rc;
  }
  *nwords = j.nwords;
  return j.status;
}

int rs_build_batch(const rs_job* jobs, uint32_t njobs, rs_mphf** outs, int* statuses) {
  if ((njobs && (!jobs || !outs || !statuses)) || njobs > 65535) return RS_ERR_INVALID_ARG;
  std::vector<JobPlan> plan;
  std::vector<uint32_t> index;
  for (uint32_t i = 0; i < njobs; ++i) {
    outs[i] = nullptr;
    const rs_job& j = jobs[i];
    if (!job_args_ok(j.keys, j.n, j.leaf_size, j.bucket_size, j.flags)) {
      statuses[i] = RS_ERR_INVALID_ARG;
      continue;
    }
    statuses[i] = RS_OK;
    JobPlan p;
    p.keys = reinterpret_cast<const Key*>(j.keys);
    p.n = j.n;
    p.l = j.leaf_size;
    p.b = j.bucket_size;
    p.flags = j.flags;
    plan.push_back(p);
    index.push_back(i);
  }
  if (!plan.empty()) {
    const int rc = build_on_default(plan);
    for (size_t k = 0; k < plan.size(); ++k) {
      if (rc) {
        mphf_release(plan[k].out);
        plan[k].out = nullptr;
        plan[k].status = rc;
      }
      statuses[index[k]] = plan[k].status;
      outs[index[k]] = plan[k].status ? nullptr : plan[k].out;
    }
  }
  int first = RS_OK;
  for (uint32_t i = 0; i < njobs; ++i)
    if (statuses[i] && !first) first = statuses[i];
  return first;
}

int rs_query(const rs_mphf* f, const rs_key128* keys, uint64_t n, uint64_t* out, uint32_t flags) {
  if (!f || (n && (!keys || !out)) || (flags & ~(uint32_t)RS_FLAG_KEYS_ON_DEVICE))
    return RS_ERR_INVALID_ARG;
  if (!n) return RS_OK;
  int rc = RS_OK;
  Context* c = default_context(&rc);
  if (!c) return rc;
  std::lock_guard<std::mutex> lock(c->mu);
  Device& d = *c->dev;
  Tables* T = nullptr;
  rc = tables_for(d, f->l, &T);
  if (rc) return rc;
  {
    rs_mphf* g = const_cast<rs_mphf*>(f);
    std::lock_guard<std::mutex> flock(g->dev_mu);
    if (!g->dev_ready) {
      rc = attach_device(*c, g);
      if (rc) {
        // (the stream is drained before the copy is freed)
        (void)hipStreamSynchronize(c->s);
        if (g->d_mem) (void)hipFree(g->d_mem);
        g->d_mem = g->d_words = g->d_samples = g->d_offsets = nullptr;
        return rc;
      }
    } else if (g->device != d.id) {
      return RS_ERR_INVALID_ARG;  // the device copy lives on another device
    }
  }
  const Key* kd = reinterpret_cast<const Key*>(keys);
  uint64_t* od = out;
  const bool on_dev = (flags & RS_FLAG_KEYS_ON_DEVICE) != 0;
  if (on_dev) {
    HIPCHECK(after_default_stream(*c));
  } else {
    HIPCHECK(ensure(c->qkeys, n * sizeof(Key)));
    HIPCHECK(ensure(c->qout, n * sizeof(uint64_t)));
    HIPCHECK(hipMemcpyAsync(c->qkeys.p, keys, n * sizeof(Key), hipMemcpyHostToDevice, c->s));
    kd = static_cast<const Key*>(c->qkeys.p);
    od = static_cast<uint64_t*>(c->qout.p);
  }
  QueryParams q;
  ef_views(f, &q.C, &q.P);
  q.offsets = f->d_offsets;
  q.gr = f->d_words + f->gr_at + 2;
  q.gr_bits = f->gr_bits;
  q.nb = f->nb;
  q.shape = make_shape(f->l);
  q.rotation = f->rotation;
  q.nodecnt = T->nodecnt;
  q.fixedbits = T->fixedbits;
  q.tau = T->tau;
  q.start = d.start;
  auto magic = [](uint32_t dv) { return (uint32_t)(((1ull << 32) + dv - 1) / dv); };
  q.magic_l = magic(q.shape.l);
  q.magic_la = magic(q.shape.la);
  q.magic_ua = magic(q.shape.ua);
  HIPCHECK(launch_query(q, kd, n, od, c->s));
  if (!on_dev) HIPCHECK(d2h(*c, out, od, n * sizeof(uint64_t)));
  else HIPCHECK(hipStreamSynchronize(c->s));
  return RS_OK;
}

int rs_serialize(const rs_mphf* f, const uint8_t** bytes, uint64_t* nbytes) {
  if (!f || !bytes || !nbytes) return RS_ERR_INVALID_ARG;
  *bytes = reinterpret_cast<const uint8_t*>(f->words.data());
  *nbytes = f->words.size() * sizeof(uint64_t);
  return RS_OK;
}

int rs_deserialize(const uint8_t* bytes, uint64_t nbytes, rs_mphf** out) {
  if (!out || (!bytes && nbytes)) return RS_ERR_INVALID_ARG;
  *out = nullptr;
  if (nbytes % 8) return RS_ERR_CORRUPT;
  rs_mphf* f = new (std::nothrow) rs_mphf();
  if (!f) return RS_ERR_OOM;
  f->words.resize(nbytes / 8);
  if (nbytes) memcpy(f->words.data(), bytes, nbytes);
  int rc = parse(f->words.data(), f->words.size(), f);
  if (rc) {
    mphf_release(f);
    return rc;
  }
  Context* c = default_context(&rc);
  if (c) {
    std::lock_guard<std::mutex> lock(c->mu);
    std::lock_guard<std::mutex> flock(f->dev_mu);
    rc = attach_device(*c, f);
  }
  if (rc) {
    mphf_release(f);
    return rc;
  }
  f->stats.n = f->n;
  f->stats.nb = f->nb;
  f->stats.gr_bits = f->gr_bits;
  f->stats.bytes = nbytes;
  *out = f;
  return RS_OK;
}

int rs_debug_node_values(const rs_mphf* f, uint64_t bucket, uint64_t* vals, uint64_t cap,
                         uint64_t* count) {
  if (!f || !count || f->keep_base.empty() || bucket >= f->nb) return RS_ERR_INVALID_ARG;
  const uint64_t b = f->keep_base[bucket], e = f->keep_base[bucket + 1];
  *count = e - b;
  if (e - b > cap || (e > b && !vals)) return RS_ERR_INVALID_ARG;
  for (uint64_t i = b; i < e; ++i) vals[i - b] = f->keep_vals[i];
  return RS_OK;
}

int rs_get_stats(const rs_mphf* f, rs_stats* st) {
  if (!f || !st) return RS_ERR_INVALID_ARG;
  *st = f->stats;
  return RS_OK;
}

void rs_free(rs_mphf* f) { mphf_release(f); }

int rs_set_schedule(const rs_schedule* sc) {
  rs_schedule v = sc ? *sc : kDefaultSchedule;
  if (v.chunk_shift_small > 63 || !v.help_after_small || v.chunk_shift_large > 63 ||
      !v.help_after_large || !v.small_tasks_per_worker)
    return RS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_schedule_mu);
  g_schedule = v;
  return RS_OK;
}

double rs_attempt_work(uint32_t leaf_size, uint32_t node_size, uint32_t flags) {
  if (leaf_size < 2 || leaf_size > kMaxLeaf || node_size < 2 || node_size >= kTable ||
      (flags & ~RS_FLAG_ROTATION))
    return -1.0;
  if (node_size <= leaf_size) {
    const LeafWork t = leaf_work_table((flags & RS_FLAG_ROTATION) != 0);
    return ldexp((double)t.fx[node_size], -(int)kLeafWorkShift);
  }
  return split_work_cached(leaf_size)[node_size];
}

uint32_t rs_rotation_lookup(uint32_t m, uint32_t a, uint32_t b) {
  if (m < 2 || m > kRotLookupMaxM) return 0xFFFFFFFFu;
  static std::vector<uint16_t> table;
  static std::once_flag once;
  std::call_once(once, [] {
    table.resize(kRotLookupEntries);
    rotation_tables(table.data());
  });
  const uint32_t full = (1u << m) - 1u;
  a &= full;
  b &= full;
  const uint32_t ea = table[(1u << m) + a], eb = table[(1u << m) + (~b & full)];
  uint32_t r = ((eb & 0xFFu) + m - (ea & 0xFFu)) % m;
  r %= ea >> 8;
  const uint32_t rb = r ? ((b << r) | (b >> (m - r))) & full : b;
  return (a | rb) == full ? r : m;
}

int rs_get_schedule(rs_schedule* sc) {
  if (!sc) return RS_ERR_INVALID_ARG;
  *sc = current_schedule();
  return RS_OK;
}

const char* rs_strerror(int code) {
  switch (code) {
    case RS_OK: return "ok";
    case RS_PENDING: return "not finished yet";
    case RS_ERR_INVALID_ARG: return "invalid argument";
    case RS_ERR_DUPLICATE: return "two keys of one bucket share their hashed word";
    case RS_ERR_OOM: return "out of memory";
    case RS_ERR_DEVICE: return "HIP device error";
    case RS_ERR_CORRUPT: return "corrupt serialised data";
    case RS_ERR_SEARCH_LIMIT: return "seed search limit reached";
    case RS_ERR_UNSUPPORTED: return "bucket larger than supported";
    default: return "unknown error";
  }
}

}  // extern "C"
