/*
 * Drives the CPU oracle (oracle/recsplit_oracle.c) under AddressSanitizer and
 * UndefinedBehaviorSanitizer: whole builds in both leaf modes over several
 * leaf and bucket sizes, queries of members and non-members, per-bucket
 * decoding and record extraction, the naive searches, and the error paths
 * (duplicates, arguments out of range, truncated and corrupted bytes).
 * Exits non-zero on any wrong result; the sanitizers abort on any invalid
 * access or undefined operation.  Test infrastructure only.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint64_t evals_split, evals_leaf, nodes_split, nodes_leaf, bf_ee_evals;
} or_stats;

uint64_t or_splitmix64_next(uint64_t *state);
int or_build(const uint64_t *keys, uint64_t n, uint32_t l, uint32_t b, uint32_t flags,
             uint8_t **out, uint64_t *out_len, or_stats *st);
int or_build_buckets(const uint64_t *keys, uint64_t n, uint32_t l, uint32_t b, uint32_t flags,
                     const uint64_t *sel, uint32_t nsel, uint64_t *vals, uint64_t vals_cap,
                     uint64_t *counts, uint64_t *grw, uint64_t grw_cap, uint64_t *grlen,
                     uint64_t *sizes, or_stats *st);
int or_query(const uint8_t *bytes, uint64_t len, const uint64_t *keys, uint64_t n, uint64_t *out);
int or_bucket_values(const uint8_t *bytes, uint64_t len, uint64_t j, uint64_t *out, uint64_t cap,
                     uint64_t *count);
int or_bucket_record(const uint8_t *bytes, uint64_t len, uint64_t j, uint64_t *out, uint64_t cap,
                     uint64_t *nbits);
uint64_t or_num_buckets(uint64_t n, uint32_t b);
void or_free(void *p);

static int failures = 0;
#define CHECK(cond, ...)                 \
  do {                                   \
    if (!(cond)) {                       \
      fprintf(stderr, "FAIL: " __VA_ARGS__); \
      fprintf(stderr, "\n");             \
      ++failures;                        \
    }                                    \
  } while (0)

/* n keys of the SplitMix64 stream seeded with seed, two outputs per key. */
static uint64_t *draw(uint64_t n, uint64_t seed) {
  uint64_t *k = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (n ? n : 1));
  uint64_t st = seed;
  for (uint64_t i = 0; i < 2 * n; ++i) k[i] = or_splitmix64_next(&st);
  return k;
}

static void one_case(uint64_t n, uint32_t l, uint32_t b, uint32_t flags, uint64_t seed) {
  uint64_t *k = draw(n, seed);
  uint8_t *bytes = NULL;
  uint64_t len = 0;
  or_stats st;
  int rc = or_build(k, n, l, b, flags, &bytes, &len, &st);
  CHECK(rc == 0, "build n=%llu l=%u b=%u flags=%u: %d", (unsigned long long)n, l, b, flags, rc);
  if (rc) {
    free(k);
    return;
  }
  uint64_t *r = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
  uint8_t *seen = (uint8_t *)calloc(n ? n : 1, 1);
  rc = or_query(bytes, len, k, n, r);
  CHECK(rc == 0, "query %d", rc);
  for (uint64_t i = 0; i < n && rc == 0; ++i) {
    CHECK(r[i] < n && !seen[r[i]], "rank %llu of key %llu", (unsigned long long)r[i],
          (unsigned long long)i);
    if (r[i] < n) seen[r[i]] = 1;
  }
  /* non-members: any value, no invalid access */
  uint64_t *other = draw(n ? n : 1, seed ^ 0xABCDEFull);
  rc = or_query(bytes, len, other, n ? n : 1, r);
  CHECK(rc == 0, "query of non-members %d", rc);
  /* every bucket decodes, its record extracts, and a sample rebuilds alike */
  uint64_t nb = or_num_buckets(n, b);
  uint64_t cap = 2 * 8192 + 2, cnt = 0, nbits = 0;
  uint64_t *vals = (uint64_t *)malloc(sizeof(uint64_t) * cap);
  uint64_t *words = (uint64_t *)malloc(sizeof(uint64_t) * 4096);
  for (uint64_t j = 0; j < nb; ++j) {
    CHECK(or_bucket_values(bytes, len, j, vals, cap, &cnt) == 0, "bucket %llu", (unsigned long long)j);
    CHECK(or_bucket_record(bytes, len, j, words, 4096, &nbits) == 0, "record %llu",
          (unsigned long long)j);
  }
  uint64_t sel[2] = {0, nb - 1};
  uint64_t bv[2 * (2 * 8192 + 2)], counts[2], grw[8192], grlen[2], sizes[2];
  rc = or_build_buckets(k, n, l, b, flags, sel, 2, bv, 2 * cap, counts, grw, 8192, grlen, sizes, &st);
  CHECK(rc == 0, "build_buckets %d", rc);
  if (rc == 0) {
    CHECK(or_bucket_values(bytes, len, nb - 1, vals, cap, &cnt) == 0 && cnt == counts[1] &&
              memcmp(vals, bv + counts[0], cnt * sizeof(uint64_t)) == 0,
          "last bucket values");
  }
  /* truncated and corrupted bytes are rejected, never read out of bounds */
  CHECK(or_query(bytes, len - 8, k, n < 4 ? n : 4, r) != 0, "truncated bytes accepted");
  uint8_t *bad = (uint8_t *)malloc(len);
  for (uint64_t at = 0; at < len && at < 400; at += 8) {
    memcpy(bad, bytes, len);
    bad[at] ^= 0x5A;
    (void)or_query(bad, len, k, n < 4 ? n : 4, r);
    (void)or_bucket_values(bad, len, 0, vals, cap, &cnt);
  }
  free(bad);
  free(vals);
  free(words);
  free(other);
  free(seen);
  free(r);
  or_free(bytes);
  free(k);
}

int main(void) {
  static const uint32_t ls[] = {2, 3, 5, 8, 12};
  static const uint32_t bs[] = {1, 7, 100, 1000};
  uint64_t seed = 1;
  for (uint32_t flags = 0; flags < 4; ++flags)
    for (size_t i = 0; i < sizeof ls / sizeof ls[0]; ++i)
      for (size_t j = 0; j < sizeof bs / sizeof bs[0]; ++j) {
        /* naive search (flag 2) on small sets only */
        uint64_t n = (flags & 2u) ? 300 : 3000;
        if (ls[i] == 12 && (flags & 2u)) continue;
        one_case(n, ls[i], bs[j], flags, seed++);
        one_case(0, ls[i], bs[j], flags, seed++);
        one_case(1, ls[i], bs[j], flags, seed++);
        one_case(17, ls[i], bs[j], flags, seed++);
      }
  one_case(300, 16, 300, 1, seed++);
  one_case(14, 24, 14, 1, seed++);
  /* duplicates and arguments out of range */
  uint64_t *k = draw(100, 99);
  k[2] = k[4] ^ 1u;
  k[3] = k[5];
  uint8_t *bytes = NULL;
  uint64_t len = 0;
  CHECK(or_build(k, 100, 8, 100, 1, &bytes, &len, NULL) == -2, "duplicate accepted");
  CHECK(or_build(k, 100, 1, 100, 1, &bytes, &len, NULL) == -1, "l = 1 accepted");
  CHECK(or_build(k, 100, 25, 100, 1, &bytes, &len, NULL) == -1, "l = 25 accepted");
  CHECK(or_build(k, 100, 8, 0, 1, &bytes, &len, NULL) == -1, "b = 0 accepted");
  CHECK(or_build(k, 100, 8, 4097, 1, &bytes, &len, NULL) == -1, "b = 4097 accepted");
  free(k);
  printf("oracle sanitizer driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
