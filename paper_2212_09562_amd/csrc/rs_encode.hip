// Encoding (Sec. 2.1 "Golomb-Rice" and "Elias-Fano", Sec. 2.2
// "Representation") and evaluation (Sec. 2.2 "Query", Sec. 4).
//
// Golomb-Rice record of a bucket: the tau low bits of every node value in
// preorder, then every unary part in preorder (floor(v / 2^tau) zeros and a
// one); records of all buckets are concatenated, least significant bit first
// in 64-bit words.  Two Elias-Fano sequences hold the bucket prefix sums C_j
// and the record offsets P_j.  One wave64 encodes one bucket; bits land with
// atomicOr in a zeroed buffer, so the result does not depend on the order of
// the writes.
#include "rs_launch.h"

namespace rs {

namespace {

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
  const uint32_t lane = __lane_id();
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(v, d);
    if (lane >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (uint32_t d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

__device__ __forceinline__ void or_bits(uint64_t* w, uint64_t pos, uint64_t value, uint32_t width) {
  if (width == 0) return;
  const uint64_t i = pos >> 6;
  const uint32_t sh = (uint32_t)(pos & 63);
  atomicOr((unsigned long long*)&w[i], (unsigned long long)(value << sh));
  if (sh + width > 64) atomicOr((unsigned long long*)&w[i + 1], (unsigned long long)(value >> (64 - sh)));
}

__device__ __forceinline__ uint64_t low_mask(uint32_t t) { return t >= 64 ? ~0ull : ((1ull << t) - 1); }

__global__ void __launch_bounds__(256) k_gr_len(const uint64_t* node_base, uint64_t nb,
                                                const uint64_t* vals, const uint32_t* msz,
                                                const uint8_t* tau, uint64_t* len) {
  const uint64_t j = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  if (j >= nb) return;
  const uint32_t lane = __lane_id();
  const uint64_t b = node_base[j], e = node_base[j + 1];
  uint64_t bits = 0;
  for (uint64_t i = b + lane; i < e; i += 64) {
    const uint32_t t = tau[msz[i]];
    bits += t + (vals[i] >> t) + 1;
  }
  bits = wave_sum64(bits);
  if (lane == 0) len[j] = bits;
}

__global__ void __launch_bounds__(256) k_gr_write(const uint64_t* node_base, uint64_t nb,
                                                  const uint64_t* vals, const uint32_t* msz,
                                                  const uint8_t* tau, const uint64_t* pos,
                                                  uint64_t* gr) {
  const uint64_t j = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  if (j >= nb) return;
  const uint32_t lane = __lane_id();
  const uint64_t b = node_base[j], e = node_base[j + 1];
  uint64_t fixed = 0;
  for (uint64_t i = b + lane; i < e; i += 64) fixed += tau[msz[i]];
  fixed = wave_sum64(fixed);
  uint64_t fpos = pos[j], upos = pos[j] + fixed;
  for (uint64_t g = b; g < e; g += 64) {
    const uint64_t i = g + lane;
    const bool v = i < e;
    const uint32_t t = v ? tau[msz[i]] : 0;
    const uint64_t val = v ? vals[i] : 0;
    const uint64_t q = v ? (t >= 64 ? 0 : val >> t) : 0;
    const uint64_t fi = wave_incl_scan64(t);
    const uint64_t ui = wave_incl_scan64(v ? q + 1 : 0);
    if (v) {
      or_bits(gr, fpos + fi - t, val & low_mask(t), t);
      const uint64_t one = upos + ui - 1;  // q zeros, then this one
      atomicOr((unsigned long long*)&gr[one >> 6], 1ull << (one & 63));
    }
    fpos += __shfl(fi, 63);
    upos += __shfl(ui, 63);
  }
}

__global__ void k_ef(const uint64_t* x, uint64_t N, uint32_t L, uint64_t* lower, uint64_t* upper) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t v = x[i];
    if (L) or_bits(lower, i * L, v & low_mask(L), L);
    const uint64_t u = (v >> L) + i;
    atomicOr((unsigned long long*)&upper[u >> 6], 1ull << (u & 63));
  }
}

// Position of the k-th (0-based) set bit of x; x has more than k set bits.
// A binary search over the popcounts of halves, quarters, ...: the same
// instructions for every lane.
__device__ __forceinline__ uint32_t select_in_word(uint64_t x, uint32_t k) {
  uint32_t pos = 0;
  uint32_t c = (uint32_t)__popc((uint32_t)x);
  if (k >= c) {
    k -= c;
    pos = 32;
  }
  uint32_t w = (uint32_t)(x >> pos);
#pragma unroll
  for (uint32_t half = 16; half >= 1; half >>= 1) {
    c = (uint32_t)__popc(w & ((1u << half) - 1u));
    if (k >= c) {
      k -= c;
      pos += half;
      w >>= half;
    }
  }
  return pos;
}

__global__ void k_popc_words(const uint64_t* w, uint64_t n, uint64_t* out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = (uint64_t)__popcll(w[i]);
}

__global__ void k_samples(const uint64_t* w, uint64_t n, const uint64_t* prefix, uint64_t* samples,
                          uint64_t nsamples) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r0 = prefix[i], r1 = prefix[i + 1];
    constexpr uint64_t step = 1ull << kSampleShift;
    for (uint64_t k = (r0 + step - 1) >> kSampleShift; (k << kSampleShift) < r1 && k < nsamples;
         ++k)
      samples[k] = i * 64 + select_in_word(w[i], (uint32_t)((k << kSampleShift) - r0));
  }
}

// Position of the i-th one of an Elias-Fano upper vector.
__device__ uint64_t ef_select(const EFView& e, uint64_t i) {
  uint64_t p = e.samples[i >> kSampleShift];
  uint32_t need = (uint32_t)(i & ((1u << kSampleShift) - 1u));
  uint64_t wi = p >> 6;
  uint64_t word = e.upper[wi] & (~0ull << (p & 63));
  for (;;) {
    const uint32_t c = (uint32_t)__popcll(word);
    if (need < c) return wi * 64 + select_in_word(word, need);
    need -= c;
    word = e.upper[++wi];
  }
}

__device__ __forceinline__ uint64_t read_bits(const uint64_t* w, uint64_t pos, uint32_t width) {
  if (width == 0) return 0;
  const uint64_t i = pos >> 6;
  const uint32_t sh = (uint32_t)(pos & 63);
  uint64_t v = w[i] >> sh;
  if (sh + width > 64) v |= w[i + 1] << (64 - sh);
  return v & low_mask(width);
}

__device__ uint64_t ef_get(const EFView& e, uint64_t i) {
  const uint64_t hi = ef_select(e, i) - i;
  return (hi << e.L) | read_bits(e.lower, i * e.L, e.L);
}

// Elements i and i + 1 (i + 1 < N): the one of element i + 1 is the next one
// after that of element i.
__device__ void ef_get2(const EFView& e, uint64_t i, uint64_t* a, uint64_t* b) {
  const uint64_t p = ef_select(e, i);
  uint64_t wi = (p + 1) >> 6;
  uint64_t word = e.upper[wi] & (~0ull << ((p + 1) & 63));
  while (!word) word = e.upper[++wi];
  const uint64_t q = wi * 64 + (uint64_t)__builtin_ctzll(word);
  *a = ((p - i) << e.L) | read_bits(e.lower, i * e.L, e.L);
  *b = ((q - i - 1) << e.L) | read_bits(e.lower, (i + 1) * e.L, e.L);
}

// v mod m for a leaf size m: through double precision while v < 2^53 (one
// correction step makes it exact), else the integer division.
__device__ __forceinline__ uint32_t mod_leaf(uint64_t v, uint32_t m) {
  if (v >> 53) return (uint32_t)(v % m);
  uint64_t q = (uint64_t)((double)v * (1.0 / (double)m));
  int64_t r = (int64_t)(v - q * m);
  if (r < 0) r += m;
  if (r >= (int64_t)m) r -= m;
  return (uint32_t)r;
}

// Count the zeros before the next one at or after *pos; advance past the one.
__device__ uint64_t read_unary(const uint64_t* w, uint64_t* pos, uint64_t end) {
  uint64_t p = *pos, q = 0;
  while (p < end) {
    const uint64_t x = w[p >> 6] >> (p & 63);
    if (x) {
      const uint32_t z = (uint32_t)__builtin_ctzll(x);
      q += z;
      *pos = p + z + 1;
      return q;
    }
    const uint32_t adv = 64 - (uint32_t)(p & 63);
    q += adv;
    p += adv;
  }
  *pos = end;
  return q;
}

// Skip k unary codes (k ones) starting at *pos.
__device__ void skip_ones(const uint64_t* w, uint64_t* pos, uint64_t k, uint64_t end) {
  uint64_t p = *pos;
  while (k && p < end) {
    const uint64_t x = w[p >> 6] >> (p & 63);
    const uint32_t c = (uint32_t)__popcll(x);
    if (c >= k) {
      p += select_in_word(x, (uint32_t)(k - 1)) + 1;
      k = 0;
      break;
    }
    k -= c;
    p += 64 - (p & 63);
  }
  *pos = p < end ? p : end;
}

__global__ void __launch_bounds__(256) k_query(QueryParams Q, const Key* keys, uint64_t n,
                                               uint64_t* out) {
  const uint64_t idx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const Key key = keys[idx];
  const uint64_t j = __umul64hi(key.w0, Q.nb);
  uint64_t cj, cj1, pj;
  if (Q.offsets) {
    cj = Q.offsets[2 * j];
    pj = Q.offsets[2 * j + 1];
    cj1 = Q.offsets[2 * j + 2];
  } else {
    ef_get2(Q.C, j, &cj, &cj1);
    pj = ef_get(Q.P, j);
  }
  uint64_t m64 = cj1 - cj;
  if (m64 > kMaxBucketKeys) m64 = 0;
  uint32_t m = (uint32_t)m64;
  const uint64_t end = Q.gr_bits;
  uint64_t fp = pj, up = pj + Q.fixedbits[m];
  uint64_t offset = 0, pos = 0;
  uint32_t depth = 0;
  for (;;) {
    const uint32_t kd = kind_of(Q.shape, m);
    if (kd == kNone || depth >= kMaxDepth) break;
    const uint32_t t = Q.tau[m];
    const uint64_t lo = fp + t <= end ? read_bits(Q.gr, fp, t) : 0;
    fp += t;
    const uint64_t q = read_unary(Q.gr, &up, end);
    const uint64_t v = (t >= 64 ? 0 : q << t) | lo;
    const uint64_t start = Q.start[depth];
    if (kd == kLeaf) {
      if (Q.rotation) {
        const uint32_t r = mod_leaf(v, m);
        pos = reduce(hash_top(key.w1, start + (v - r)), m);
        if (key.w0 & 1u) {
          pos += r;
          if (pos >= m) pos -= m;
        }
      } else {
        pos = reduce(hash_top(key.w1, start + v), m);
      }
      break;
    }
    const uint32_t p = reduce(hash_top(key.w1, start + v), m);
    // the children (parts_of, with the divisions by multiply-high): every
    // child before the last has size `unit`
    uint32_t unit, k, c;
    if (kd == kBinary) {
      const uint32_t ua = Q.shape.ua;
      unit = ua * __umulhi((m >> 1) + ua - 1, Q.magic_ua);
      k = 2;
      c = p >= unit ? 1u : 0u;
    } else {
      unit = kd == kLower ? Q.shape.l : Q.shape.la;
      const uint32_t mg = kd == kLower ? Q.magic_l : Q.magic_la;
      k = __umulhi(m + unit - 1, mg);
      c = __umulhi(p, mg);
    }
    offset += (uint64_t)c * unit;
    fp += (uint64_t)c * Q.fixedbits[unit];
    skip_ones(Q.gr, &up, (uint64_t)c * Q.nodecnt[unit], end);
    m = c + 1 < k ? unit : m - (k - 1) * unit;
    depth += 1;
  }
  out[idx] = cj + offset + pos;
}

__global__ void k_decode_offsets(EFView C, EFView P, uint64_t N, uint64_t* out) {
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < N;
       j += (uint64_t)gridDim.x * blockDim.x) {
    out[2 * j] = ef_get(C, j);
    out[2 * j + 1] = ef_get(P, j);
  }
}

// Both sequences decoded without select support, one block per sequence
// (block 0: C into out[2i], block 1: P into out[2i+1]).  The upper vector is
// read in slices of one word per thread; a block prefix sum of the words'
// popcounts numbers the ones, and the one numbered i at bit position p gives
// element i = ((p - i) << L) | its L lower bits.
constexpr uint32_t kDecodeThreads = 1024;

__global__ void __launch_bounds__(kDecodeThreads) k_decode_pairs(EFView C, uint64_t c_words,
                                                                 EFView P, uint64_t p_words,
                                                                 uint64_t* out) {
  __shared__ uint32_t s_wave[kDecodeThreads / 64];
  const uint32_t which = blockIdx.x;
  const EFView e = which ? P : C;
  const uint64_t nwords = which ? p_words : c_words;
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  uint64_t base = 0;  // ones in the slices before this one
  for (uint64_t w0 = 0; w0 < nwords; w0 += kDecodeThreads) {
    const uint64_t wi = w0 + threadIdx.x;
    uint64_t word = wi < nwords ? e.upper[wi] : 0;
    const uint32_t c = (uint32_t)__popcll(word);
    uint32_t incl = c;  // inclusive prefix sum within the wave
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
      const uint32_t o = __shfl_up(incl, d);
      if (lane >= d) incl += o;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (uint32_t w = 0; w < kDecodeThreads / 64; ++w) {
      if (w < wave) before += s_wave[w];
      total += s_wave[w];
    }
    uint64_t i = base + before + incl - c;
    while (word) {
      const uint64_t p = wi * 64 + (uint64_t)__builtin_ctzll(word);
      if (i < e.N) out[2 * i + which] = ((p - i) << e.L) | read_bits(e.lower, i * e.L, e.L);
      ++i;
      word &= word - 1;
    }
    base += total;
    __syncthreads();  // s_wave is rewritten by the next slice
  }
}

uint32_t grid_for(uint64_t n, uint32_t threads, uint32_t cap) {
  uint64_t g = (n + threads - 1) / threads;
  if (g > cap) g = cap;
  return g ? (uint32_t)g : 1u;
}

}  // namespace

hipError_t gr_lengths(const uint64_t* node_base, uint64_t nb, const uint64_t* vals,
                      const uint32_t* msz, const uint8_t* tau, uint64_t* len, hipStream_t s) {
  k_gr_len<<<(uint32_t)((nb * 64 + 255) / 256), 256, 0, s>>>(node_base, nb, vals, msz, tau, len);
  return hipGetLastError();
}

hipError_t gr_write(const uint64_t* node_base, uint64_t nb, const uint64_t* vals, const uint32_t* msz,
                    const uint8_t* tau, const uint64_t* pos, uint64_t* gr, hipStream_t s) {
  k_gr_write<<<(uint32_t)((nb * 64 + 255) / 256), 256, 0, s>>>(node_base, nb, vals, msz, tau, pos,
                                                               gr);
  return hipGetLastError();
}

hipError_t ef_write(const uint64_t* x, uint64_t N, uint32_t L, uint64_t* lower, uint64_t* upper,
                    hipStream_t s) {
  k_ef<<<grid_for(N, 256, 8192), 256, 0, s>>>(x, N, L, lower, upper);
  return hipGetLastError();
}

hipError_t select_samples(const uint64_t* words, uint64_t nwords, uint64_t* counts,
                          uint64_t* prefix, uint64_t* scan_tmp, uint64_t* samples,
                          uint64_t nsamples, hipStream_t s) {
  if (!nwords) return hipSuccess;
  k_popc_words<<<grid_for(nwords, 256, 8192), 256, 0, s>>>(words, nwords, counts);
  hipError_t e = scan_excl_u64(counts, nwords, prefix, scan_tmp, s);
  if (e != hipSuccess) return e;
  k_samples<<<grid_for(nwords, 256, 8192), 256, 0, s>>>(words, nwords, prefix, samples, nsamples);
  return hipGetLastError();
}

hipError_t decode_offsets(const EFView& C, const EFView& P, uint64_t N, uint64_t* out,
                          hipStream_t s) {
  if (!N) return hipSuccess;
  k_decode_offsets<<<grid_for(N, 256, 8192), 256, 0, s>>>(C, P, N, out);
  return hipGetLastError();
}

hipError_t decode_pairs(const EFView& C, uint64_t c_words, const EFView& P, uint64_t p_words,
                        uint64_t* out, hipStream_t s) {
  k_decode_pairs<<<2, kDecodeThreads, 0, s>>>(C, c_words, P, p_words, out);
  return hipGetLastError();
}

hipError_t launch_query(const QueryParams& q, const Key* keys, uint64_t n, uint64_t* out,
                        hipStream_t s) {
  if (!n) return hipSuccess;
  k_query<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(q, keys, n, out);
  return hipGetLastError();
}

}  // namespace rs
