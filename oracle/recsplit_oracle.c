/*
 * RecSplit construction oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded C implementation of what the GPU library
 * computes, written from the paper (Bez, Kurpicz, Lehmann, Sanders, "High
 * Performance Construction of RecSplit Based Minimal Perfect Hash Functions",
 * arXiv 2212.09562).  It exists so that the tests, the smoke check and the
 * CPU-baseline leg of the benchmark can check the GPU path against an
 * independent implementation.  The product path never links, loads or calls
 * this file; it shares no code, header or table with the HIP library.
 *
 * Every stored node value is the smallest non-negative integer that meets
 * the node's validity predicate (Sec. 5.1, "Bijections": the stored number
 * must be as small as possible).  So the output is a function of (key set,
 * leaf size, bucket size, mode) alone, and parity with the GPU is bit-exact.
 *
 * Where the paper leaves a detail open, the reading used is stated at the
 * function that implements it (readings R1..R24 of the format description).
 *
 * Parity pins (what ties each function to something other than itself) are
 * listed in the test files; the functions below whose results only our own
 * format fixes -- the start seeds, tau, the byte layout -- are "parity
 * unpinned" beyond agreement with the GPU path and the round-trip and
 * closed-form checks the tests run.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_INVALID_ARG (-1)
#define OR_ERR_DUPLICATE (-2)
#define OR_ERR_OOM (-3)
#define OR_ERR_CORRUPT (-5)
#define OR_ERR_SEARCH_LIMIT (-6)

#define OR_FLAG_ROTATION 1u
#define OR_FLAG_NAIVE 2u

#define OR_MAX_LEAF 24u
#define OR_MAX_BUCKET 4096u
#define OR_MAX_DEPTH 64u
/* Bug guard only: every search below ends with probability one once
 * duplicates are rejected; the cap turns a logic error into an error code. */
#define OR_SEARCH_CAP (1ull << 40)

/* ------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): a Weyl sequence with  */
/* increment 0x9E3779B97F4A7C15 passed through a 64-bit mixer.         */
/* ------------------------------------------------------------------ */
static uint64_t or_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t or_splitmix64_next(uint64_t *state) {
  *state += 0x9E3779B97F4A7C15ull;
  return or_mix(*state);
}

/* Reading R5: the starting seed of depth d (root = 0) is output number d+1
 * of SplitMix64 seeded with 0.  The paper only says that the starting seed is
 * constant on a level (Sec. 5.3, "Splittings"). */
uint64_t or_start_seed(uint32_t d) {
  uint64_t st = 0, v = 0;
  for (uint32_t i = 0; i <= d; ++i) v = or_splitmix64_next(&st);
  return v;
}

/* Reading R3/R4: the hash of a key under hash-function identifier x is the
 * SplitMix64 mixer applied to (w1 + x) mod 2^64, where w1 is the second word
 * of the 128-bit master hash code (Sec. 2.2 "Splitting Trees" tries "random
 * hash functions"; Sec. 6 uses random 128-bit integers as the master hash). */
uint64_t or_hash(uint64_t w1, uint64_t x) { return or_mix(w1 + x); }

/* Reading R6: a hash is reduced to [0, M) by a 32x32 multiply-high of its
 * top 32 bits ("a hash function modulo l", Sec. 2.2 "Bijections"). */
uint32_t or_remap(uint64_t h, uint32_t M) {
  return (uint32_t)(((h >> 32) * (uint64_t)M) >> 32);
}

/* Reading R2: bucket of a key = floor(w0 * nb / 2^64) ("mapped to different
 * buckets of expected size b", Sec. 2.2). */
uint64_t or_bucket_of(uint64_t w0, uint64_t nb) {
  return (uint64_t)(((unsigned __int128)w0 * nb) >> 64);
}

/* Reading R1: nb = max(1, ceil(n / b)). */
uint64_t or_num_buckets(uint64_t n, uint32_t b) {
  uint64_t nb = (n + b - 1) / b;
  return nb ? nb : 1;
}

/* Sec. 2.2 "Splitting Trees": the leaf-parent level has fanout
 * max{2, ceil(0.35 l + 0.55)}, the level above max{2, ceil(0.21 l + 0.9)}.
 * The formulas are evaluated exactly in integers (35l+55 and 21l+90 over
 * 100), so l = 7 and l = 10, where the real value is an integer, are not at
 * the mercy of binary rounding. */
void or_fanouts(uint32_t l, uint32_t *lower, uint32_t *upper) {
  uint32_t lf = (35u * l + 55u + 99u) / 100u;
  uint32_t uf = (21u * l + 90u + 99u) / 100u;
  *lower = lf < 2 ? 2 : lf;
  *upper = uf < 2 ? 2 : uf;
}

enum { OR_NONE = 0, OR_LEAF = 1, OR_LOWER = 2, OR_UPPER = 3, OR_BINARY = 4 };

typedef struct {
  uint32_t l, la, ua; /* leaf size, lower aggregation size, upper aggregation size */
} or_shape;

static or_shape or_make_shape(uint32_t l) {
  uint32_t lf, uf;
  or_fanouts(l, &lf, &uf);
  or_shape s;
  s.l = l;
  s.la = lf * l;
  s.ua = uf * s.la;
  return s;
}

static int or_kind(const or_shape *s, uint32_t m) {
  if (m <= 1) return OR_NONE;
  if (m <= s->l) return OR_LEAF;
  if (m <= s->la) return OR_LOWER;
  if (m <= s->ua) return OR_UPPER;
  return OR_BINARY;
}

/* Part sizes of an inner node (readings R8, R9).  Lower and upper nodes cut
 * m into parts of their unit (l resp. l * lower fanout), the last part taking
 * the remainder.  A fanout-2 node above them gives its left child the
 * smallest multiple of the upper unit that is at least floor(m/2), so that
 * every subtree except those on the rightmost path is full (Sec. 2.2: the
 * shape depends only on l and m; every leaf but possibly the last holds l
 * objects).  Returns the number of parts, 0 for a leaf or an empty node. */
static uint32_t or_parts(const or_shape *s, uint32_t m, uint32_t *sizes, uint32_t *unit) {
  int k = or_kind(s, m);
  if (k == OR_LOWER || k == OR_UPPER) {
    uint32_t u = (k == OR_LOWER) ? s->l : s->la;
    uint32_t np = (m + u - 1) / u;
    for (uint32_t j = 0; j + 1 < np; ++j) sizes[j] = u;
    sizes[np - 1] = m - (np - 1) * u;
    *unit = u;
    return np;
  }
  if (k == OR_BINARY) {
    uint32_t half = m / 2;
    uint32_t left = s->ua * ((half + s->ua - 1) / s->ua);
    sizes[0] = left;
    sizes[1] = m - left;
    *unit = left;
    return 2;
  }
  return 0;
}

int or_children(uint32_t m, uint32_t l, uint32_t *sizes) {
  if (l < 2 || l > OR_MAX_LEAF) return OR_ERR_INVALID_ARG;
  or_shape s = or_make_shape(l);
  uint32_t unit;
  return (int)or_parts(&s, m, sizes, &unit);
}

/* Child that a key with hash h goes to (reading R7): lower and upper nodes
 * send it to floor(remap(h, m) / unit); a fanout-2 node sends it right iff
 * remap(h, m) >= size of the left child. */
static uint32_t or_child_of(const or_shape *s, uint32_t m, uint64_t h) {
  int k = or_kind(s, m);
  uint32_t p = or_remap(h, m);
  if (k == OR_BINARY) {
    uint32_t sizes[2], left;
    or_parts(s, m, sizes, &left);
    return p >= left ? 1u : 0u;
  }
  return p / (k == OR_LOWER ? s->l : s->la);
}

/* ------------------------------------------------------------------ */
/* Rotation (Sec. 2.1): rot_m^r rotates the m low bits left by r.      */
/* ------------------------------------------------------------------ */
uint32_t or_rot(uint32_t x, uint32_t r, uint32_t m) {
  uint32_t full = (m >= 32) ? 0xFFFFFFFFu : ((1u << m) - 1u);
  if (r == 0) return x & full;
  return ((x << r) | (x >> (m - r))) & full;
}

static uint32_t or_popcount(uint32_t x) {
  uint32_t c = 0;
  while (x) {
    x &= x - 1;
    ++c;
  }
  return c;
}

/* Rotation fitting test (Sec. 4): smallest r < m with a | rot_m^r(b) having
 * all m low bits set, after the popcount checks |A| = popcount(a) and
 * |B| = popcount(b).  Returns -1 when no rotation fits. */
int or_rotation_fit(uint32_t a, uint32_t b, uint32_t na, uint32_t nbb, uint32_t m) {
  uint32_t full = (1u << m) - 1u;
  if (or_popcount(a) != na || or_popcount(b) != nbb) return -1;
  for (uint32_t r = 0; r < m; ++r)
    if ((a | or_rot(b, r, m)) == full) return (int)r;
  return -1;
}

/* ------------------------------------------------------------------ */
/* Leaf bijection search (Sec. 2.2 "Bijections", Sec. 4).              */
/* ------------------------------------------------------------------ */

/* Position of a key in a leaf of size m under stored value v, exactly as a
 * query computes it (Sec. 4: the hash index is v rounded down to a multiple
 * of m and the rotation r = v mod m is added modulo m for keys of B). */
static uint32_t or_leaf_position(uint64_t w1, int is_b, uint32_t m, uint64_t start, uint64_t v,
                                 int rotation) {
  if (!rotation) return or_remap(or_hash(w1, v + start), m);
  uint64_t r = v % m;
  uint64_t s = v - r;
  uint32_t p = or_remap(or_hash(w1, s + start), m);
  return is_b ? (uint32_t)((p + r) % m) : p;
}

/* Plain definition: the smallest v whose position map is injective,
 * checked with an explicit occupancy array ("naive" search). */
static int or_leaf_naive(const uint64_t *w1, const uint8_t *is_b, uint32_t m, uint64_t start,
                         int rotation, uint64_t *out) {
  uint8_t seen[OR_MAX_LEAF];
  for (uint64_t v = 0; v < OR_SEARCH_CAP; ++v) {
    memset(seen, 0, sizeof seen);
    uint32_t i;
    for (i = 0; i < m; ++i) {
      uint32_t p = or_leaf_position(w1[i], is_b[i], m, start, v, rotation);
      if (seen[p]) break;
      seen[p] = 1;
    }
    if (i == m) {
      *out = v;
      return OR_OK;
    }
  }
  return OR_ERR_SEARCH_LIMIT;
}

/* Brute force as the paper describes it: OR 2^(hash mod m) over all keys and
 * accept when all m bits are set (Sec. 2.2 "Bijections").  *ee counts the
 * hash evaluations a search that stops at the first collision would make. */
static int or_leaf_brute(const uint64_t *w1, uint32_t m, uint64_t start, uint64_t *out,
                         uint64_t *ee) {
  uint32_t full = (1u << m) - 1u;
  for (uint64_t v = 0; v < OR_SEARCH_CAP; ++v) {
    uint32_t mask = 0;
    int collided = 0;
    for (uint32_t i = 0; i < m; ++i) {
      uint32_t bit = 1u << or_remap(or_hash(w1[i], v + start), m);
      if (!collided) {
        if (ee) ++*ee;
        if (mask & bit) collided = 1;
      }
      mask |= bit;
    }
    if (mask == full) {
      *out = v;
      return OR_OK;
    }
  }
  return OR_ERR_SEARCH_LIMIT;
}

/* Rotation fitting (Sec. 4): only hash indices that are multiples of m are
 * tried; the keys of A set bits of a, those of B bits of b; the stored value
 * is the index plus the smallest fitting rotation. */
static int or_leaf_rotation(const uint64_t *w1, const uint8_t *is_b, uint32_t m, uint64_t start,
                            uint64_t *out) {
  uint32_t na = 0, nbb = 0;
  for (uint32_t i = 0; i < m; ++i) {
    if (is_b[i]) ++nbb;
    else ++na;
  }
  for (uint64_t t = 0; t < OR_SEARCH_CAP / m; ++t) {
    uint64_t s = t * m;
    uint32_t a = 0, b = 0;
    for (uint32_t i = 0; i < m; ++i) {
      uint32_t bit = 1u << or_remap(or_hash(w1[i], s + start), m);
      if (is_b[i]) b |= bit;
      else a |= bit;
    }
    int r = or_rotation_fit(a, b, na, nbb, m);
    if (r >= 0) {
      *out = s + (uint64_t)r;
      return OR_OK;
    }
  }
  return OR_ERR_SEARCH_LIMIT;
}

/* mode: 0 brute (bitmask), 1 brute (naive), 2 rotation (bitmask),
 * 3 rotation (naive).  ee may be NULL. */
int or_leaf_search(const uint64_t *w1, const uint8_t *is_b, uint32_t m, uint32_t depth,
                   uint32_t mode, uint64_t *out, uint64_t *ee) {
  if (m < 2 || m > OR_MAX_LEAF) return OR_ERR_INVALID_ARG;
  uint64_t start = or_start_seed(depth);
  switch (mode) {
    case 0: return or_leaf_brute(w1, m, start, out, ee);
    case 1: return or_leaf_naive(w1, is_b, m, start, 0, out);
    case 2: return or_leaf_rotation(w1, is_b, m, start, out);
    case 3: return or_leaf_naive(w1, is_b, m, start, 1, out);
    default: return OR_ERR_INVALID_ARG;
  }
}

/* ------------------------------------------------------------------ */
/* Split seed search (Sec. 2.2 "Splitting Trees"): the smallest seed s  */
/* whose child counts equal the prescribed part sizes.                  */
/* ------------------------------------------------------------------ */
static int or_split(const or_shape *sh, const uint64_t *w1, uint32_t m, uint64_t start,
                    uint64_t *out) {
  uint32_t sizes[64], unit;
  uint32_t np = or_parts(sh, m, sizes, &unit);
  uint32_t cnt[64];
  for (uint64_t s = 0; s < OR_SEARCH_CAP; ++s) {
    memset(cnt, 0, sizeof(uint32_t) * np);
    for (uint32_t i = 0; i < m; ++i) ++cnt[or_child_of(sh, m, or_hash(w1[i], s + start))];
    uint32_t j;
    for (j = 0; j < np; ++j)
      if (cnt[j] != sizes[j]) break;
    if (j == np) {
      *out = s;
      return OR_OK;
    }
  }
  return OR_ERR_SEARCH_LIMIT;
}

int or_split_search(const uint64_t *w1, uint32_t m, uint32_t l, uint32_t depth, uint64_t *out) {
  if (l < 2 || l > OR_MAX_LEAF) return OR_ERR_INVALID_ARG;
  or_shape sh = or_make_shape(l);
  if (or_kind(&sh, m) < OR_LOWER) return OR_ERR_INVALID_ARG;
  return or_split(&sh, w1, m, or_start_seed(depth), out);
}

/* ------------------------------------------------------------------ */
/* Golomb-Rice parameter (Sec. 2.2 "Representation": tau depends on the */
/* layer and is precomputed).  Reading R17: p is the probability that   */
/* one trial succeeds at the node, and tau is the optimal Rice          */
/* parameter of a geometric source with that p (Kiely 2004):            */
/* tau = max(0, 1 + floor(log2(ln(phi-1) / ln(1-p)))).                  */
/* ------------------------------------------------------------------ */
static double or_log_success(const or_shape *sh, uint32_t m) {
  int k = or_kind(sh, m);
  if (k == OR_LEAF) return lgamma((double)m + 1.0) - (double)m * log((double)m);
  uint32_t sizes[64], unit;
  uint32_t np = or_parts(sh, m, sizes, &unit);
  double lp = lgamma((double)m + 1.0);
  for (uint32_t j = 0; j < np; ++j)
    lp += -lgamma((double)sizes[j] + 1.0) + (double)sizes[j] * log((double)sizes[j] / (double)m);
  return lp;
}

/* The argument of floor() in the tau formula; exposed so the tests can check
 * that it never sits close to an integer. */
double or_tau_log2arg(uint32_t m, uint32_t l) {
  or_shape sh = or_make_shape(l);
  double p = exp(or_log_success(&sh, m));
  double golden_minus_one = (sqrt(5.0) - 1.0) / 2.0;
  return log2(log(golden_minus_one) / log1p(-p));
}

static uint32_t or_tau_shape(const or_shape *sh, uint32_t m) {
  (void)sh;
  double x = or_tau_log2arg(m, sh->l);
  double t = 1.0 + floor(x);
  return t < 0.0 ? 0u : (uint32_t)t;
}

uint32_t or_tau(uint32_t m, uint32_t l) {
  or_shape sh = or_make_shape(l);
  if (or_kind(&sh, m) == OR_NONE) return 0;
  return or_tau_shape(&sh, m);
}

/* ------------------------------------------------------------------ */
/* Bucket construction: recursion over the splitting tree, node values  */
/* emitted in preorder (Sec. 2.2 "Representation").                    */
/* ------------------------------------------------------------------ */
typedef struct {
  uint64_t *val;
  uint32_t *msz;
  uint64_t len, cap;
} or_nodes;

typedef struct {
  uint64_t evals_split, evals_leaf, nodes_split, nodes_leaf, bf_ee_evals;
} or_stats;

static int or_push(or_nodes *nd, uint64_t v, uint32_t m) {
  if (nd->len == nd->cap) {
    uint64_t nc = nd->cap ? 2 * nd->cap : 256;
    uint64_t *nv = (uint64_t *)realloc(nd->val, nc * sizeof(uint64_t));
    if (!nv) return OR_ERR_OOM;
    nd->val = nv;
    uint32_t *nm = (uint32_t *)realloc(nd->msz, nc * sizeof(uint32_t));
    if (!nm) return OR_ERR_OOM;
    nd->msz = nm;
    nd->cap = nc;
  }
  nd->val[nd->len] = v;
  nd->msz[nd->len] = m;
  ++nd->len;
  return OR_OK;
}

/* keys: m pairs (w0, w1) of this node; reordered in place by the split. */
static int or_build_node(const or_shape *sh, uint64_t *keys, uint32_t m, uint32_t depth,
                         uint32_t flags, or_nodes *nd, or_stats *st) {
  int kind = or_kind(sh, m);
  if (kind == OR_NONE) return OR_OK; /* reading R10: nothing stored */
  if (depth >= OR_MAX_DEPTH) return OR_ERR_INVALID_ARG;
  uint64_t start = or_start_seed(depth);
  uint64_t w1[OR_MAX_LEAF];
  if (kind == OR_LEAF) {
    uint8_t isb[OR_MAX_LEAF];
    for (uint32_t i = 0; i < m; ++i) {
      w1[i] = keys[2 * i + 1];
      isb[i] = (uint8_t)(keys[2 * i] & 1u); /* reading R12: B iff bit 0 of w0 */
    }
    uint64_t v;
    int rc;
    int rot = (flags & OR_FLAG_ROTATION) != 0;
    if (flags & OR_FLAG_NAIVE) rc = or_leaf_naive(w1, isb, m, start, rot, &v);
    else if (rot) rc = or_leaf_rotation(w1, isb, m, start, &v);
    else rc = or_leaf_brute(w1, m, start, &v, &st->bf_ee_evals);
    if (rc) return rc;
    /* useful hash evaluations: every tried index hashes all m keys */
    st->evals_leaf += (rot ? v / m + 1 : v + 1) * (uint64_t)m;
    st->nodes_leaf += 1;
    return or_push(nd, v, m);
  }
  uint64_t *h1 = (uint64_t *)malloc(sizeof(uint64_t) * m);
  uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * 2 * m);
  uint32_t *child = (uint32_t *)malloc(sizeof(uint32_t) * m);
  if (!h1 || !tmp || !child) {
    free(h1);
    free(tmp);
    free(child);
    return OR_ERR_OOM;
  }
  for (uint32_t i = 0; i < m; ++i) h1[i] = keys[2 * i + 1];
  uint64_t s;
  int rc = or_split(sh, h1, m, start, &s);
  if (rc == OR_OK) rc = or_push(nd, s, m);
  if (rc == OR_OK) {
    st->evals_split += (s + 1) * (uint64_t)m;
    st->nodes_split += 1;
    uint32_t sizes[64], unit;
    uint32_t np = or_parts(sh, m, sizes, &unit);
    for (uint32_t i = 0; i < m; ++i) child[i] = or_child_of(sh, m, or_hash(h1[i], s + start));
    /* stable partition by child */
    uint32_t pos = 0;
    for (uint32_t c = 0; c < np; ++c)
      for (uint32_t i = 0; i < m; ++i)
        if (child[i] == c) {
          tmp[2 * pos] = keys[2 * i];
          tmp[2 * pos + 1] = keys[2 * i + 1];
          ++pos;
        }
    memcpy(keys, tmp, sizeof(uint64_t) * 2 * m);
    uint32_t off = 0;
    for (uint32_t c = 0; c < np && rc == OR_OK; ++c) {
      rc = or_build_node(sh, keys + 2 * off, sizes[c], depth + 1, flags, nd, st);
      off += sizes[c];
    }
  }
  free(h1);
  free(tmp);
  free(child);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Bit vectors, least significant bit first in little-endian words.     */
/* ------------------------------------------------------------------ */
typedef struct {
  uint64_t *w;
  uint64_t nbits, cap; /* cap in words */
} or_bits;

static int or_bits_reserve(or_bits *b, uint64_t nbits) {
  uint64_t need = (nbits + 63) / 64;
  if (need <= b->cap) return OR_OK;
  uint64_t nc = b->cap ? b->cap : 64;
  while (nc < need) nc *= 2;
  uint64_t *nw = (uint64_t *)realloc(b->w, nc * sizeof(uint64_t));
  if (!nw) return OR_ERR_OOM;
  memset(nw + b->cap, 0, (nc - b->cap) * sizeof(uint64_t));
  b->w = nw;
  b->cap = nc;
  return OR_OK;
}

static int or_bits_put(or_bits *b, uint64_t value, uint32_t width) {
  int rc = or_bits_reserve(b, b->nbits + width);
  if (rc) return rc;
  for (uint32_t i = 0; i < width; ++i) {
    if ((value >> i) & 1u) b->w[(b->nbits + i) / 64] |= 1ull << ((b->nbits + i) % 64);
  }
  b->nbits += width;
  return OR_OK;
}

static int or_bit_get(const uint64_t *w, uint64_t pos) { return (int)((w[pos / 64] >> (pos % 64)) & 1u); }

static uint64_t or_bits_get(const uint64_t *w, uint64_t pos, uint32_t width) {
  uint64_t v = 0;
  for (uint32_t i = 0; i < width; ++i) v |= (uint64_t)or_bit_get(w, pos + i) << i;
  return v;
}

/* Golomb-Rice record of one bucket (Sec. 2.1 "Golomb-Rice", Sec. 2.2
 * "Representation", reading R18): first the tau low bits of every node
 * value in preorder, then every unary part in preorder, a unary part being
 * floor(v / 2^tau) zero bits followed by a one bit. */
static int or_gr_append(or_bits *gr, const or_shape *sh, const uint64_t *val, const uint32_t *msz,
                        uint64_t cnt) {
  int rc;
  for (uint64_t i = 0; i < cnt; ++i) {
    uint32_t t = or_tau_shape(sh, msz[i]);
    rc = or_bits_put(gr, val[i] & (t >= 64 ? ~0ull : ((1ull << t) - 1)), t);
    if (rc) return rc;
  }
  for (uint64_t i = 0; i < cnt; ++i) {
    uint32_t t = or_tau_shape(sh, msz[i]);
    uint64_t q = t >= 64 ? 0 : val[i] >> t;
    for (uint64_t z = 0; z < q; ++z) {
      rc = or_bits_put(gr, 0, 1);
      if (rc) return rc;
    }
    rc = or_bits_put(gr, 1, 1);
    if (rc) return rc;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Elias-Fano (Sec. 2.1 "Elias-Fano", reading R19): N monotone values   */
/* x_0..x_{N-1} <= U = x_{N-1}; L = largest L with N * 2^L <= U (0 if   */
/* U < N); lower L bits packed; bit (x_i >> L) + i set in the upper     */
/* vector of (U >> L) + N bits.                                         */
/* ------------------------------------------------------------------ */
static uint32_t or_ef_lowbits(uint64_t N, uint64_t U) {
  uint32_t L = 0;
  while (L < 63 && (U >> (L + 1)) >= N) ++L;
  return L;
}

typedef struct {
  uint64_t N, U, L, lower_words, upper_bits, upper_words;
  uint64_t *lower, *upper;
} or_ef;

static int or_ef_build(or_ef *ef, const uint64_t *x, uint64_t N) {
  memset(ef, 0, sizeof *ef);
  ef->N = N;
  ef->U = x[N - 1];
  ef->L = or_ef_lowbits(N, ef->U);
  ef->lower_words = (N * ef->L + 63) / 64;
  ef->upper_bits = (ef->U >> ef->L) + N;
  ef->upper_words = (ef->upper_bits + 63) / 64;
  ef->lower = (uint64_t *)calloc(ef->lower_words ? ef->lower_words : 1, sizeof(uint64_t));
  ef->upper = (uint64_t *)calloc(ef->upper_words ? ef->upper_words : 1, sizeof(uint64_t));
  if (!ef->lower || !ef->upper) return OR_ERR_OOM;
  for (uint64_t i = 0; i < N; ++i) {
    for (uint64_t j = 0; j < ef->L; ++j)
      if ((x[i] >> j) & 1u) ef->lower[(i * ef->L + j) / 64] |= 1ull << ((i * ef->L + j) % 64);
    uint64_t up = (x[i] >> ef->L) + i;
    ef->upper[up / 64] |= 1ull << (up % 64);
  }
  return OR_OK;
}

static void or_ef_free(or_ef *ef) {
  free(ef->lower);
  free(ef->upper);
}

/* ------------------------------------------------------------------ */
/* Serialised form (reading R20), all fields little-endian u64 words:   */
/*  magic, version | flags << 32, n, leaf | bucket << 32, nb,           */
/*  EF(C) = N, U, L, lower_words, upper_bits, upper_words, lower, upper */
/*  EF(P) likewise, GR = nbits, nwords, words.                          */
/* ------------------------------------------------------------------ */
#define OR_MAGIC 0x31564C5053434552ull /* "RECSPLV1" little-endian */

typedef struct {
  uint64_t *w;
  uint64_t len, cap;
} or_words;

static int or_w_put(or_words *o, uint64_t v) {
  if (o->len == o->cap) {
    uint64_t nc = o->cap ? 2 * o->cap : 1024;
    uint64_t *nw = (uint64_t *)realloc(o->w, nc * sizeof(uint64_t));
    if (!nw) return OR_ERR_OOM;
    o->w = nw;
    o->cap = nc;
  }
  o->w[o->len++] = v;
  return OR_OK;
}

static int or_w_put_ef(or_words *o, const or_ef *ef) {
  int rc = 0;
  rc |= or_w_put(o, ef->N);
  rc |= or_w_put(o, ef->U);
  rc |= or_w_put(o, ef->L);
  rc |= or_w_put(o, ef->lower_words);
  rc |= or_w_put(o, ef->upper_bits);
  rc |= or_w_put(o, ef->upper_words);
  for (uint64_t i = 0; i < ef->lower_words; ++i) rc |= or_w_put(o, ef->lower[i]);
  for (uint64_t i = 0; i < ef->upper_words; ++i) rc |= or_w_put(o, ef->upper[i]);
  return rc ? OR_ERR_OOM : OR_OK;
}

/* Bucket the keys (stable counting sort by bucket id) and reject a bucket
 * holding two keys with the same w1 (reading R21): such keys hash alike
 * under every seed, so no leaf containing both could ever be a bijection. */
static int or_bucketize(const uint64_t *keys, uint64_t n, uint64_t nb, uint64_t **sorted_out,
                        uint64_t **off_out) {
  uint64_t *off = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
  uint64_t *sorted = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (n ? n : 1));
  uint64_t *fill = (uint64_t *)calloc(nb, sizeof(uint64_t));
  if (!off || !sorted || !fill) {
    free(off);
    free(sorted);
    free(fill);
    return OR_ERR_OOM;
  }
  for (uint64_t i = 0; i < n; ++i) off[or_bucket_of(keys[2 * i], nb) + 1]++;
  for (uint64_t j = 0; j < nb; ++j) off[j + 1] += off[j];
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t j = or_bucket_of(keys[2 * i], nb);
    uint64_t p = off[j] + fill[j]++;
    sorted[2 * p] = keys[2 * i];
    sorted[2 * p + 1] = keys[2 * i + 1];
  }
  free(fill);
  *sorted_out = sorted;
  *off_out = off;
  return OR_OK;
}

static int or_cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static int or_check_duplicates(const uint64_t *sorted, const uint64_t *off, uint64_t j) {
  uint64_t m = off[j + 1] - off[j];
  if (m < 2) return OR_OK;
  uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * m);
  if (!w) return OR_ERR_OOM;
  for (uint64_t i = 0; i < m; ++i) w[i] = sorted[2 * (off[j] + i) + 1];
  qsort(w, m, sizeof(uint64_t), or_cmp_u64);
  int rc = OR_OK;
  for (uint64_t i = 1; i < m; ++i)
    if (w[i] == w[i - 1]) rc = OR_ERR_DUPLICATE;
  free(w);
  return rc;
}

static int or_check_args(uint64_t n, uint32_t l, uint32_t b) {
  if (l < 2 || l > OR_MAX_LEAF) return OR_ERR_INVALID_ARG;
  if (b < 1 || b > OR_MAX_BUCKET) return OR_ERR_INVALID_ARG;
  if (n >= (1ull << 40)) return OR_ERR_INVALID_ARG;
  return OR_OK;
}

/* Whole construction (Sec. 2.2): buckets, one splitting tree per bucket,
 * a single Golomb-Rice bit vector with all bucket records concatenated, and
 * Elias-Fano sequences of the bucket prefix sums C_j and of the record bit
 * offsets P_j (reading R19: two plain sequences).  keys holds n (w0, w1)
 * pairs.  *out is malloc'ed; release with or_free. */
int or_build(const uint64_t *keys, uint64_t n, uint32_t l, uint32_t b, uint32_t flags,
             uint8_t **out, uint64_t *out_len, or_stats *st) {
  *out = NULL;
  *out_len = 0;
  int rc = or_check_args(n, l, b);
  if (rc) return rc;
  or_stats dummy;
  if (!st) st = &dummy;
  memset(st, 0, sizeof *st);
  or_shape sh = or_make_shape(l);
  uint64_t nb = or_num_buckets(n, b);
  uint64_t *sorted = NULL, *off = NULL;
  rc = or_bucketize(keys, n, nb, &sorted, &off);
  if (rc) return rc;
  for (uint64_t j = 0; j < nb && rc == OR_OK; ++j) {
    if (off[j + 1] - off[j] > 0xFFFFFFFFull) rc = OR_ERR_INVALID_ARG;
    else rc = or_check_duplicates(sorted, off, j);
  }
  or_bits gr = {0};
  uint64_t *pos = (uint64_t *)malloc(sizeof(uint64_t) * (nb + 1));
  or_nodes nd = {0};
  if (!pos) rc = OR_ERR_OOM;
  for (uint64_t j = 0; j < nb && rc == OR_OK; ++j) {
    pos[j] = gr.nbits;
    nd.len = 0;
    rc = or_build_node(&sh, sorted + 2 * off[j], (uint32_t)(off[j + 1] - off[j]), 0, flags, &nd,
                       st);
    if (rc == OR_OK) rc = or_gr_append(&gr, &sh, nd.val, nd.msz, nd.len);
  }
  if (rc == OR_OK) pos[nb] = gr.nbits;
  or_ef efc = {0}, efp = {0};
  or_words o = {0};
  if (rc == OR_OK) rc = or_ef_build(&efc, off, nb + 1);
  if (rc == OR_OK) rc = or_ef_build(&efp, pos, nb + 1);
  if (rc == OR_OK) {
    int e = 0;
    e |= or_w_put(&o, OR_MAGIC);
    e |= or_w_put(&o, 1ull | ((uint64_t)(flags & OR_FLAG_ROTATION) << 32));
    e |= or_w_put(&o, n);
    e |= or_w_put(&o, (uint64_t)l | ((uint64_t)b << 32));
    e |= or_w_put(&o, nb);
    e |= or_w_put_ef(&o, &efc);
    e |= or_w_put_ef(&o, &efp);
    e |= or_w_put(&o, gr.nbits);
    e |= or_w_put(&o, (gr.nbits + 63) / 64);
    for (uint64_t i = 0; i < (gr.nbits + 63) / 64; ++i) e |= or_w_put(&o, gr.w[i]);
    if (e) rc = OR_ERR_OOM;
  }
  or_ef_free(&efc);
  or_ef_free(&efp);
  free(gr.w);
  free(pos);
  free(nd.val);
  free(nd.msz);
  free(sorted);
  free(off);
  if (rc) {
    free(o.w);
    return rc;
  }
  *out = (uint8_t *)o.w;
  *out_len = o.len * sizeof(uint64_t);
  return OR_OK;
}

/* Build only the trees of the selected buckets of a full key set: for every
 * selected bucket, its node values in preorder and its Golomb-Rice record.
 * vals/counts: values of bucket sel[i] follow those of sel[i-1];
 * grw: records packed likewise, each starting on a fresh word, grlen[i] bits.
 * Used to check a full-size GPU build on a sample of buckets. */
int or_build_buckets(const uint64_t *keys, uint64_t n, uint32_t l, uint32_t b, uint32_t flags,
                     const uint64_t *sel, uint32_t nsel, uint64_t *vals, uint64_t vals_cap,
                     uint64_t *counts, uint64_t *grw, uint64_t grw_cap, uint64_t *grlen,
                     uint64_t *sizes, or_stats *st) {
  int rc = or_check_args(n, l, b);
  if (rc) return rc;
  or_stats dummy;
  if (!st) st = &dummy;
  memset(st, 0, sizeof *st);
  or_shape sh = or_make_shape(l);
  uint64_t nb = or_num_buckets(n, b);
  uint64_t *sorted = NULL, *off = NULL;
  rc = or_bucketize(keys, n, nb, &sorted, &off);
  if (rc) return rc;
  or_nodes nd = {0};
  uint64_t vused = 0, wused = 0;
  for (uint32_t i = 0; i < nsel && rc == OR_OK; ++i) {
    uint64_t j = sel[i];
    if (j >= nb) {
      rc = OR_ERR_INVALID_ARG;
      break;
    }
    rc = or_check_duplicates(sorted, off, j);
    if (rc) break;
    nd.len = 0;
    sizes[i] = off[j + 1] - off[j];
    rc = or_build_node(&sh, sorted + 2 * off[j], (uint32_t)sizes[i], 0, flags, &nd, st);
    if (rc) break;
    if (vused + nd.len > vals_cap) {
      rc = OR_ERR_INVALID_ARG;
      break;
    }
    if (nd.len) memcpy(vals + vused, nd.val, nd.len * sizeof(uint64_t)); /* empty: val may be NULL */
    vused += nd.len;
    counts[i] = nd.len;
    or_bits gr = {0};
    rc = or_gr_append(&gr, &sh, nd.val, nd.msz, nd.len);
    if (rc == OR_OK) {
      uint64_t nw = (gr.nbits + 63) / 64;
      if (wused + nw > grw_cap) rc = OR_ERR_INVALID_ARG;
      else {
        if (nw) memcpy(grw + wused, gr.w, nw * sizeof(uint64_t));
        wused += nw;
        grlen[i] = gr.nbits;
      }
    }
    free(gr.w);
  }
  free(nd.val);
  free(nd.msz);
  free(sorted);
  free(off);
  return rc;
}

void or_free(void *p) { free(p); }

/* ------------------------------------------------------------------ */
/* Query (Sec. 2.2 "Query", Sec. 4 for the rotation of B keys).         */
/* ------------------------------------------------------------------ */
typedef struct {
  uint64_t n, nb;
  uint32_t l, b, rotation;
  uint64_t *C, *P; /* decoded Elias-Fano sequences, nb + 1 values each */
  const uint64_t *gr;
  uint64_t gr_bits;
  or_shape sh;
} or_view;

static int or_ef_decode(const uint64_t *w, uint64_t avail, uint64_t *used, uint64_t **out,
                        uint64_t expectN) {
  if (avail < 6) return OR_ERR_CORRUPT;
  uint64_t N = w[0], U = w[1], L = w[2], lw = w[3], ub = w[4], uw = w[5];
  if (N != expectN || L > 63 || L != or_ef_lowbits(N, U)) return OR_ERR_CORRUPT;
  if (lw != (N * L + 63) / 64 || ub != (U >> L) + N || uw != (ub + 63) / 64) return OR_ERR_CORRUPT;
  if (avail < 6 + lw + uw) return OR_ERR_CORRUPT;
  const uint64_t *lower = w + 6, *upper = w + 6 + lw;
  uint64_t *x = (uint64_t *)malloc(sizeof(uint64_t) * N);
  if (!x) return OR_ERR_OOM;
  uint64_t i = 0;
  for (uint64_t p = 0; p < ub && i < N; ++p) {
    if (or_bit_get(upper, p)) {
      x[i] = ((p - i) << L) | or_bits_get(lower, i * L, (uint32_t)L);
      ++i;
    }
  }
  if (i != N || x[N - 1] != U) {
    free(x);
    return OR_ERR_CORRUPT;
  }
  *used = 6 + lw + uw;
  *out = x;
  return OR_OK;
}

static int or_view_open(const uint8_t *bytes, uint64_t len, or_view *v) {
  memset(v, 0, sizeof *v);
  if (len % 8 || len < 5 * 8) return OR_ERR_CORRUPT;
  uint64_t nw = len / 8;
  const uint64_t *w = (const uint64_t *)bytes;
  if (w[0] != OR_MAGIC || (w[1] & 0xFFFFFFFFull) != 1) return OR_ERR_CORRUPT;
  v->rotation = (uint32_t)((w[1] >> 32) & 1u);
  v->n = w[2];
  v->l = (uint32_t)(w[3] & 0xFFFFFFFFull);
  v->b = (uint32_t)(w[3] >> 32);
  v->nb = w[4];
  if (or_check_args(v->n, v->l, v->b) || v->nb != or_num_buckets(v->n, v->b)) return OR_ERR_CORRUPT;
  v->sh = or_make_shape(v->l);
  uint64_t at = 5, used;
  int rc = or_ef_decode(w + at, nw - at, &used, &v->C, v->nb + 1);
  if (rc) return rc;
  at += used;
  rc = or_ef_decode(w + at, nw - at, &used, &v->P, v->nb + 1);
  if (rc) return rc;
  at += used;
  if (nw - at < 2) return OR_ERR_CORRUPT;
  v->gr_bits = w[at];
  if (w[at + 1] != (v->gr_bits + 63) / 64 || nw - at - 2 != w[at + 1]) return OR_ERR_CORRUPT;
  v->gr = w + at + 2;
  if (v->C[0] != 0 || v->C[v->nb] != v->n || v->P[0] != 0 || v->P[v->nb] != v->gr_bits)
    return OR_ERR_CORRUPT;
  /* both sequences are prefix sums: non-decreasing, so no bucket claims
   * more keys or record bits than the whole structure holds */
  for (uint64_t j = 0; j < v->nb; ++j)
    if (v->C[j + 1] < v->C[j] || v->P[j + 1] < v->P[j]) return OR_ERR_CORRUPT;
  return OR_OK;
}

static void or_view_close(or_view *v) {
  free(v->C);
  free(v->P);
}

/* Preorder list of the sizes of the stored nodes of a tree of size m. */
static void or_preorder(const or_shape *sh, uint32_t m, uint32_t *out, uint64_t *cnt) {
  if (or_kind(sh, m) == OR_NONE) return;
  out[(*cnt)++] = m;
  uint32_t sizes[64], unit;
  uint32_t np = or_parts(sh, m, sizes, &unit);
  for (uint32_t c = 0; c < np; ++c) or_preorder(sh, sizes[c], out, cnt);
}

int or_preorder_sizes(uint32_t m, uint32_t l, uint32_t *out, uint64_t cap, uint64_t *count) {
  if (l < 2 || l > OR_MAX_LEAF) return OR_ERR_INVALID_ARG;
  or_shape sh = or_make_shape(l);
  uint64_t c = 0;
  /* a tree of m keys stores at most 2m nodes */
  if (cap < 2 * (uint64_t)m + 2) return OR_ERR_INVALID_ARG;
  or_preorder(&sh, m, out, &c);
  *count = c;
  return OR_OK;
}

/* Decode the node values of bucket j in preorder from its record. */
static int or_decode_bucket(const or_view *v, uint64_t j, uint64_t **vals, uint32_t **msz,
                            uint64_t *cnt) {
  uint32_t m = (uint32_t)(v->C[j + 1] - v->C[j]);
  uint32_t *sz = (uint32_t *)malloc(sizeof(uint32_t) * (2 * (uint64_t)m + 2));
  uint64_t *val = (uint64_t *)malloc(sizeof(uint64_t) * (2 * (uint64_t)m + 2));
  if (!sz || !val) {
    free(sz);
    free(val);
    return OR_ERR_OOM;
  }
  uint64_t c = 0;
  or_preorder(&v->sh, m, sz, &c);
  uint64_t fp = v->P[j], fixed_total = 0;
  for (uint64_t i = 0; i < c; ++i) fixed_total += or_tau_shape(&v->sh, sz[i]);
  uint64_t up = fp + fixed_total, end = v->P[j + 1];
  for (uint64_t i = 0; i < c; ++i) {
    uint32_t t = or_tau_shape(&v->sh, sz[i]);
    if (fp + t > end) goto corrupt;
    uint64_t lo = or_bits_get(v->gr, fp, t);
    fp += t;
    uint64_t q = 0;
    while (1) {
      if (up >= end) goto corrupt;
      if (or_bit_get(v->gr, up++)) break;
      ++q;
    }
    val[i] = (q << t) | lo;
  }
  *vals = val;
  *msz = sz;
  *cnt = c;
  return OR_OK;
corrupt:
  free(sz);
  free(val);
  return OR_ERR_CORRUPT;
}

int or_bucket_values(const uint8_t *bytes, uint64_t len, uint64_t j, uint64_t *out, uint64_t cap,
                     uint64_t *count) {
  or_view v;
  int rc = or_view_open(bytes, len, &v);
  if (rc == OR_OK && j >= v.nb) rc = OR_ERR_INVALID_ARG;
  uint64_t *val = NULL;
  uint32_t *sz = NULL;
  uint64_t c = 0;
  if (rc == OR_OK) rc = or_decode_bucket(&v, j, &val, &sz, &c);
  if (rc == OR_OK) {
    if (c > cap) rc = OR_ERR_INVALID_ARG;
    else {
      memcpy(out, val, c * sizeof(uint64_t));
      *count = c;
    }
  }
  free(val);
  free(sz);
  or_view_close(&v);
  return rc;
}

/* The Golomb-Rice record of bucket j as stored in serialised bytes: the bits
 * [P_j, P_j+1) of the record vector, repacked from bit 0 of out (words
 * zero-padded), so that it can be compared word for word with a record the
 * oracle builds itself (or_build_buckets).  Reads only; no arithmetic of the
 * method. */
int or_bucket_record(const uint8_t *bytes, uint64_t len, uint64_t j, uint64_t *out, uint64_t cap,
                     uint64_t *nbits) {
  or_view v;
  int rc = or_view_open(bytes, len, &v);
  if (rc == OR_OK && j >= v.nb) rc = OR_ERR_INVALID_ARG;
  if (rc == OR_OK) {
    uint64_t lo = v.P[j], bits = v.P[j + 1] - v.P[j];
    uint64_t nw = (bits + 63) / 64;
    if (nw > cap) rc = OR_ERR_INVALID_ARG;
    else {
      for (uint64_t i = 0; i < nw; ++i) {
        uint32_t take = bits - 64 * i < 64 ? (uint32_t)(bits - 64 * i) : 64u;
        out[i] = or_bits_get(v.gr, lo + 64 * i, take);
      }
      *nbits = bits;
    }
  }
  or_view_close(&v);
  return rc;
}

/* Number of stored nodes in the subtree of size m. */
static uint64_t or_subtree_nodes(const or_shape *sh, uint32_t m) {
  if (or_kind(sh, m) == OR_NONE) return 0;
  uint32_t sizes[64], unit;
  uint32_t np = or_parts(sh, m, sizes, &unit);
  uint64_t c = 1;
  for (uint32_t k = 0; k < np; ++k) c += or_subtree_nodes(sh, sizes[k]);
  return c;
}

/* Rank of one key: descend from the bucket root, following the child the
 * split hash picks and adding the sizes of the children to its left; at the
 * leaf add the leaf position; finally add the size of earlier buckets
 * (Sec. 2.2 "Query").  Keys of B get the rotation added modulo m (Sec. 4). */
static uint64_t or_query_one(const or_view *v, const uint64_t *vals, uint64_t w0, uint64_t w1,
                             uint64_t j) {
  uint32_t m = (uint32_t)(v->C[j + 1] - v->C[j]);
  uint64_t offset = 0, node = 0;
  uint32_t depth = 0;
  while (or_kind(&v->sh, m) >= OR_LOWER) {
    uint64_t start = or_start_seed(depth);
    uint64_t h = or_hash(w1, vals[node] + start);
    uint32_t c = or_child_of(&v->sh, m, h);
    uint32_t sizes[64], unit;
    or_parts(&v->sh, m, sizes, &unit);
    node += 1;
    for (uint32_t k = 0; k < c; ++k) {
      offset += sizes[k];
      node += or_subtree_nodes(&v->sh, sizes[k]);
    }
    m = sizes[c];
    depth += 1;
  }
  uint32_t p = 0;
  if (or_kind(&v->sh, m) == OR_LEAF)
    p = or_leaf_position(w1, (int)(w0 & 1u), m, or_start_seed(depth), vals[node], (int)v->rotation);
  return v->C[j] + offset + p;
}

/* keys: n pairs (w0, w1); out: n ranks.  A key not in the original set gets
 * some value, never an out-of-range read. */
int or_query(const uint8_t *bytes, uint64_t len, const uint64_t *keys, uint64_t n,
             uint64_t *out) {
  or_view v;
  int rc = or_view_open(bytes, len, &v);
  if (rc) {
    or_view_close(&v);
    return rc;
  }
  uint64_t cached = ~0ull;
  uint64_t *val = NULL;
  uint32_t *sz = NULL;
  uint64_t c = 0;
  for (uint64_t i = 0; i < n && rc == OR_OK; ++i) {
    uint64_t j = or_bucket_of(keys[2 * i], v.nb);
    if (j != cached) {
      free(val);
      free(sz);
      val = NULL;
      sz = NULL;
      rc = or_decode_bucket(&v, j, &val, &sz, &c);
      if (rc) break;
      cached = j;
    }
    out[i] = or_query_one(&v, val, keys[2 * i], keys[2 * i + 1], j);
  }
  free(val);
  free(sz);
  or_view_close(&v);
  return rc;
}
