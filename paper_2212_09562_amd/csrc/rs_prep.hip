// Bucketing (Sec. 2.2: keys to buckets of expected size b, sorted by bucket,
// bucket borders), device-wide exclusive scans, the duplicate check, and the
// roots of the search queue.
#include <algorithm>
#include <vector>

#include "rs_launch.h"

namespace rs {

namespace {

constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanPer = 4;
constexpr uint32_t kScanBlock = kScanThreads * kScanPer;

__device__ __forceinline__ uint64_t bucket_of(uint64_t w0, uint64_t nb) { return __umul64hi(w0, nb); }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const uint32_t lane = __lane_id();
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    T o = __shfl_up(v, d);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan of the 1024 values of one block; returns the block total.
__device__ uint64_t block_excl_scan(uint64_t (&v)[kScanPer], uint64_t* s_wave) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint64_t sum = 0;
#pragma unroll
  for (uint32_t i = 0; i < kScanPer; ++i) sum += v[i];
  uint64_t incl = wave_incl_scan(sum);
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  uint64_t wbase = 0, total = 0;
  for (uint32_t w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) wbase += s_wave[w];
    total += s_wave[w];
  }
  uint64_t run = wbase + incl - sum;
#pragma unroll
  for (uint32_t i = 0; i < kScanPer; ++i) {
    uint64_t x = v[i];
    v[i] = run;
    run += x;
  }
  __syncthreads();
  return total;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_sums(const T* in, uint64_t n, uint64_t* sums) {
  __shared__ uint64_t s_wave[kScanThreads / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  uint64_t v[kScanPer];
#pragma unroll
  for (uint32_t i = 0; i < kScanPer; ++i) v[i] = base + i < n ? (uint64_t)in[base + i] : 0;
  uint64_t total = block_excl_scan(v, s_wave);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block scans the per-block sums in place (exclusive), in slices of 1024.
__global__ void __launch_bounds__(kScanThreads) k_scan_top(uint64_t* sums, uint64_t nblocks) {
  __shared__ uint64_t s_wave[kScanThreads / 64];
  uint64_t carry = 0;
  for (uint64_t s0 = 0; s0 < nblocks; s0 += kScanBlock) {
    const uint64_t base = s0 + threadIdx.x * kScanPer;
    uint64_t v[kScanPer];
#pragma unroll
    for (uint32_t i = 0; i < kScanPer; ++i) v[i] = base + i < nblocks ? sums[base + i] : 0;
    uint64_t total = block_excl_scan(v, s_wave);
#pragma unroll
    for (uint32_t i = 0; i < kScanPer; ++i)
      if (base + i < nblocks) sums[base + i] = v[i] + carry;
    carry += total;
  }
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_out(const T* in, uint64_t n,
                                                          const uint64_t* sums, uint64_t* out) {
  __shared__ uint64_t s_wave[kScanThreads / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  uint64_t v[kScanPer];
#pragma unroll
  for (uint32_t i = 0; i < kScanPer; ++i) v[i] = base + i < n ? (uint64_t)in[base + i] : 0;
  const uint64_t total = block_excl_scan(v, s_wave);
  const uint64_t add = sums ? sums[blockIdx.x] : 0;  // null: a single block
#pragma unroll
  for (uint32_t i = 0; i < kScanPer; ++i)
    if (base + i < n) out[base + i] = v[i] + add;
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = add + total;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Bucket sizes.  With few buckets each block counts in LDS and flushes once.
__global__ void k_hist(const Key* keys, uint64_t n, uint64_t nb, uint32_t* cnt, uint32_t use_lds) {
  extern __shared__ uint32_t s_h[];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  if (use_lds) {
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += stride)
      atomicAdd(&s_h[bucket_of(keys[i].w0, nb)], 1u);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x)
      if (s_h[i]) atomicAdd(&cnt[i], s_h[i]);
  } else {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += stride)
      atomicAdd(&cnt[bucket_of(keys[i].w0, nb)], 1u);
  }
}

__global__ void k_max_bucket(const uint32_t* cnt, uint64_t nb, uint32_t* maxm) {
  uint32_t mx = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nb;
       i += (uint64_t)gridDim.x * blockDim.x)
    mx = max(mx, cnt[i]);
  for (uint32_t d = 32; d > 0; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d));
  if ((threadIdx.x & 63) == 0) atomicMax(maxm, mx);
}

__global__ void k_scatter(const Key* keys, uint64_t n, uint64_t nb, const uint64_t* off,
                          uint32_t* fill, Key* out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const Key k = keys[i];
    const uint64_t b = bucket_of(k.w0, nb);
    out[off[b] + atomicAdd(&fill[b], 1u)] = k;
  }
}

// Two keys of a bucket with equal w1 hash alike under every seed, so their
// leaf could never be a bijection: sort the bucket's w1 words (bitonic, in
// LDS) and compare neighbours.  Buckets that need more than `cap` words of
// LDS are skipped and reported in *deferred.
__global__ void __launch_bounds__(256) k_dupcheck(const Key* keys, const uint64_t* off, uint64_t nb,
                                                  uint32_t cap, uint32_t* error,
                                                  uint32_t* deferred) {
  extern __shared__ uint64_t s[];
  for (uint64_t j = blockIdx.x; j < nb; j += gridDim.x) {
    const uint64_t o = off[j];
    const uint32_t m = (uint32_t)(off[j + 1] - o);
    if (m < 2) continue;
    uint32_t p2 = 1;
    while (p2 < m) p2 <<= 1;
    if (p2 > cap) {
      if (threadIdx.x == 0) atomicOr(deferred, 1u);
      continue;
    }
    for (uint32_t i = threadIdx.x; i < p2; i += blockDim.x) s[i] = i < m ? keys[o + i].w1 : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= p2; k <<= 1) {
      for (uint32_t d = k >> 1; d > 0; d >>= 1) {
        for (uint32_t i = threadIdx.x; i < p2; i += blockDim.x) {
          const uint32_t x = i ^ d;
          if (x > i) {
            const uint64_t a = s[i], b = s[x];
            const bool up = (i & k) == 0;
            if ((a > b) == up) {
              s[i] = b;
              s[x] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    bool dup = false;
    for (uint32_t i = threadIdx.x; i + 1 < m; i += blockDim.x) dup |= s[i] == s[i + 1];
    if (dup) atomicCAS(error, 0u, (uint32_t)(-RS_ERR_DUPLICATE));
    __syncthreads();
  }
}

__global__ void k_init_states(TaskState* st, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    TaskState t;
    t.np = 0;
    t.best = kInf;
    t.closed = 0;
    t.advert = 0;
    t.pad = 0;
    st[i] = t;
  }
}

// Useful work of a finished search, from its node values: the hash
// evaluations the sequential definition makes, (s+1)*m per inner node,
// (v+1)*m per brute-force leaf and (floor(v/m)+1)*m per rotation leaf, and
// the node counts.  One atomic per wave.
__global__ void __launch_bounds__(256) k_work_counts(const uint64_t* vals, const uint32_t* msz,
                                                     uint64_t n, uint32_t l, uint32_t rotation,
                                                     LeafWork lw, const uint32_t* split_fx,
                                                     JobInfo* info) {
  uint64_t es = 0, el = 0, ns = 0, nl = 0, ee = 0, se = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t m = msz[i];
    const uint64_t v = vals[i];
    if (m < 2) continue;  // no stored node has fewer than two keys (a stopped search leaves stale sizes)
    if (m > l) {
      es += (v + 1) * m;
      se += v * split_fx[m < kTable ? m : kTable - 1] + ((uint64_t)m << kLeafWorkShift);
      ns += 1;
    } else {
      const uint64_t failed = rotation ? v / m : v;
      el += (failed + 1) * m;
      ee += failed * lw.fx[m < kMaxLeaf ? m : kMaxLeaf] + ((uint64_t)m << kLeafWorkShift);
      nl += 1;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    es += __shfl_xor(es, d);
    el += __shfl_xor(el, d);
    ns += __shfl_xor(ns, d);
    nl += __shfl_xor(nl, d);
    ee += __shfl_xor(ee, d);
    se += __shfl_xor(se, d);
  }
  __shared__ uint64_t part[4][6];
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[w][0] = es;
    part[w][1] = el;
    part[w][2] = ns;
    part[w][3] = nl;
    part[w][4] = ee;
    part[w][5] = se;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const uint64_t v = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                       part[3][threadIdx.x];
    uint64_t* dst[6] = {&info->evals_split, &info->evals_leaf, &info->splits, &info->leaves,
                        &info->early_exit_leaf_fx, &info->early_exit_split_fx};
    if (v) atomicAdd(dst[threadIdx.x], v);
  }
}

__global__ void k_node_counts(const uint32_t* cnt, uint64_t nb, const uint32_t* nodecnt,
                              uint64_t* out) {
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < nb;
       j += (uint64_t)gridDim.x * blockDim.x)
    out[j] = cnt[j] <= kMaxBucketKeys ? nodecnt[cnt[j]] : 0;  // larger: refused later
}

__global__ void k_roots(const uint32_t* cnt, const uint64_t* off, const uint64_t* node_base,
                        uint64_t nb, uint32_t job, uint64_t key_base, uint64_t node_off,
                        Task* tasks, uint32_t* ready, Control* ctl) {
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < nb;
       j += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t m = cnt[j];
    if (m < 2) continue;
    const uint64_t slot = __hip_atomic_fetch_add(&ctl->tail, 1ull, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    Task t;
    t.key_off = key_base + off[j];
    t.node = node_off + node_base[j];
    t.m = m;
    t.depth = 0;
    t.job = (uint16_t)job;
    tasks[slot] = t;
    __hip_atomic_store(&ready[slot], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

uint32_t grid_for(uint64_t n, uint32_t threads, uint32_t cap) {
  uint64_t g = (n + threads - 1) / threads;
  if (g > cap) g = cap;
  return g ? (uint32_t)g : 1u;
}

}  // namespace

hipError_t fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
  if (!n) return hipSuccess;
  k_fill_u64<<<grid_for(n, 256, 4096), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (!n) return hipSuccess;
  k_fill_u32<<<grid_for(n, 256, 4096), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

uint64_t scan_tmp_words(uint64_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

template <typename T>
static hipError_t scan_impl(const T* in, uint64_t n, uint64_t* out, uint64_t* tmp, hipStream_t s) {
  if (n == 0) return fill_u64(out, 1, 0, s);
  const uint64_t nblocks = (n + kScanBlock - 1) / kScanBlock;
  if (nblocks == 1) {  // one block holds everything: one launch
    k_scan_out<T><<<1, kScanThreads, 0, s>>>(in, n, nullptr, out);
    return hipGetLastError();
  }
  k_scan_sums<T><<<(uint32_t)nblocks, kScanThreads, 0, s>>>(in, n, tmp);
  k_scan_top<<<1, kScanThreads, 0, s>>>(tmp, nblocks);
  k_scan_out<T><<<(uint32_t)nblocks, kScanThreads, 0, s>>>(in, n, tmp, out);
  return hipGetLastError();
}

hipError_t scan_excl_u32(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* tmp,
                         hipStream_t s) {
  return scan_impl<uint32_t>(in, n, out, tmp, s);
}

hipError_t scan_excl_u64(const uint64_t* in, uint64_t n, uint64_t* out, uint64_t* tmp,
                         hipStream_t s) {
  return scan_impl<uint64_t>(in, n, out, tmp, s);
}

hipError_t bucket_histogram(const Key* keys, uint64_t n, uint64_t nb, uint32_t* cnt, uint32_t* maxm,
                            hipStream_t s) {
  if (n) {
    const bool lds = nb <= 16384;
    const uint32_t grid = grid_for(n, 256 * 16, lds ? 512 : 8192);
    k_hist<<<grid, 256, lds ? (uint32_t)(nb * sizeof(uint32_t)) : 0, s>>>(keys, n, nb, cnt,
                                                                          lds ? 1u : 0u);
  }
  k_max_bucket<<<grid_for(nb, 256, 1024), 256, 0, s>>>(cnt, nb, maxm);
  return hipGetLastError();
}

hipError_t bucket_scatter(const Key* keys, uint64_t n, uint64_t nb, const uint64_t* off,
                          uint32_t* fill, Key* out, hipStream_t s) {
  if (!n) return hipSuccess;
  k_scatter<<<grid_for(n, 256, 16384), 256, 0, s>>>(keys, n, nb, off, fill, out);
  return hipGetLastError();
}

hipError_t duplicate_check(const Key* keys, const uint64_t* off, uint64_t nb, uint32_t cap,
                           uint32_t* error, uint32_t* deferred, hipStream_t s) {
  if (cap < 2) return hipSuccess;
  k_dupcheck<<<grid_for(nb, 1, 4096), 256, cap * sizeof(uint64_t), s>>>(keys, off, nb, cap, error,
                                                                        deferred);
  return hipGetLastError();
}

hipError_t init_states(TaskState* st, uint64_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  k_init_states<<<grid_for(n, 256, 4096), 256, 0, s>>>(st, n);
  return hipGetLastError();
}

hipError_t work_counts(const uint64_t* vals, const uint32_t* msz, uint64_t n, uint32_t l,
                       uint32_t rotation, const uint32_t* split_fx, JobInfo* info, hipStream_t s) {
  if (!n) return hipSuccess;
  k_work_counts<<<grid_for(n, 256 * 8, 512), 256, 0, s>>>(
      vals, msz, n, l, rotation, leaf_work_table(rotation != 0), split_fx, info);
  return hipGetLastError();
}

// Keys hashed by an attempt that stops at the first collision among j keys
// thrown into m slots: key i (0-based) is hashed when the first i are
// distinct, probability prod_{t<i} (1 - t/m).
static double early_exit_keys(uint32_t j, uint32_t m) {
  double e = 0.0, distinct = 1.0;
  for (uint32_t i = 0; i < j; ++i) {
    e += distinct;
    distinct *= 1.0 - (double)i / (double)m;
  }
  return e;
}

static double all_distinct(uint32_t j, uint32_t m) {
  double d = 1.0;
  for (uint32_t i = 0; i < j; ++i) d *= 1.0 - (double)i / (double)m;
  return d;
}

// Lower and upper splits: after t keys the child counts are multinomial with
// probabilities (part size)/m; an attempt is alive while every count is at
// most its part size, and key t+1 is hashed while it is alive.  Independent
// Poisson counts with the part sizes as means, conditioned on their sum t,
// have that multinomial law, so P(alive after t) = [x^t] prod_j T_j(x) /
// Poisson(t; m), T_j the Poisson(u_j) pmf truncated at u_j.  Parts other
// than the last are all of one size, so their product is shared by the
// node sizes with the same part count.  Long double: for m near 1300 the
// pmfs reach e^-1300.  Fanout-2 splits are credited all m keys.  About 60 ms
// at l = 16 and 0.45 s at l = 24, once per process and leaf size.
std::vector<double> split_work_table(uint32_t l) {
  const Shape s = make_shape(l);
  std::vector<double> w(kTable, 0.0);
  auto pmf = [](uint32_t u) {
    std::vector<long double> p(u + 1);
    for (uint32_t c = 0; c <= u; ++c)
      p[c] = expl((long double)c * logl((long double)u) - (long double)u - lgammal(c + 1.0L));
    return p;
  };
  auto mul = [](const std::vector<long double>& a, const std::vector<long double>& b, size_t cap) {
    std::vector<long double> r(std::min(a.size() + b.size() - 1, cap), 0.0L);
    for (size_t i = 0; i < a.size() && i < cap; ++i)
      for (size_t j = 0; j < b.size() && i + j < cap; ++j) r[i + j] += a[i] * b[j];
    return r;
  };
  // shared products of f full parts, per part size
  std::vector<long double> base;
  uint32_t base_u = 0, base_f = 0;
  std::vector<long double> full_pmf;
  for (uint32_t m = 2; m < kTable; ++m) {
    const uint32_t kd = kind_of(s, m);
    if (kd == kLeaf) continue;
    if (kd == kBinary) {
      w[m] = (double)m;
      continue;
    }
    const Parts p = parts_of(s, m);
    const uint32_t u = p.unit, f = p.k - 1;
    if (u != base_u) {
      base_u = u;
      base_f = 0;
      base.assign(1, 1.0L);
      full_pmf = pmf(u);
    }
    while (base_f < f) {
      base = mul(base, full_pmf, (size_t)kTable);
      ++base_f;
    }
    const std::vector<long double> conv = mul(base, pmf(p.last), (size_t)m);
    long double e = 0.0L;
    for (uint32_t t = 0; t < m; ++t) {
      const long double pois =
          expl((long double)t * logl((long double)m) - (long double)m - lgammal(t + 1.0L));
      const long double alive = t < conv.size() ? conv[t] / pois : 0.0L;
      e += alive < 1.0L ? alive : 1.0L;
    }
    w[m] = (double)e;
  }
  return w;
}

// Brute force: one class of m keys.  Rotation fitting (Sec. 4): class A of
// a ~ Binomial(m, 1/2) keys and class B of m - a; the larger class is hashed
// first, the other only when the first has no collision.
LeafWork leaf_work_table(bool rotation) {
  LeafWork t;
  for (uint32_t m = 0; m <= kMaxLeaf; ++m) {
    double w = 0.0;
    if (m >= 2 && !rotation) {
      w = early_exit_keys(m, m);
    } else if (m >= 2) {
      double binom = 1.0;  // C(m, a)
      for (uint32_t a = 0; a <= m; ++a) {
        const uint32_t n1 = a > m - a ? a : m - a, n2 = m - n1;
        w += binom * (early_exit_keys(n1, m) + all_distinct(n1, m) * early_exit_keys(n2, m));
        binom = binom * (double)(m - a) / (double)(a + 1);
      }
      w = ldexp(w, -(int)m);
    }
    t.fx[m] = (uint32_t)llround(ldexp(w, (int)kLeafWorkShift));
  }
  return t;
}

hipError_t node_counts(const uint32_t* cnt, uint64_t nb, const uint32_t* nodecnt, uint64_t* out,
                       hipStream_t s) {
  k_node_counts<<<grid_for(nb, 256, 4096), 256, 0, s>>>(cnt, nb, nodecnt, out);
  return hipGetLastError();
}

hipError_t queue_roots(const uint32_t* cnt, const uint64_t* off, const uint64_t* node_base,
                       uint64_t nb, uint32_t job, uint64_t key_base, uint64_t node_off, Task* tasks,
                       uint32_t* ready, Control* ctl, hipStream_t s) {
  k_roots<<<grid_for(nb, 256, 4096), 256, 0, s>>>(cnt, off, node_base, nb, job, key_base,
                                                  node_off, tasks, ready, ctl);
  return hipGetLastError();
}

}  // namespace rs
