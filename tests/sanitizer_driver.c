/* Exercises the C oracle (oracle/oracle.c) and the input generators
 * (gen/gen.c) on small seeded inputs, for builds with AddressSanitizer /
 * UndefinedBehaviorSanitizer and with ThreadSanitizer (the oracle's pthread
 * pool).  Test infrastructure only.  Cross-checks keep the calls honest: the
 * edge-list, CSR and neighbour-list forms of one lattice give the same labels,
 * and the batched oracle equals the per-instance one on any thread count.
 * Exit status 0 when every check holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_label_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint8_t* occ,
                       int32_t* label);
int oracle_label_csr(int64_t n, const int32_t* row_ptr, const int32_t* col, const uint8_t* occ,
                     int32_t* label);
int oracle_label_ell(int64_t n, int32_t z_max, const int32_t* nn, const uint8_t* occ, int32_t* label);
int oracle_label_batched(int32_t n_inst, const int64_t* site_off, const int64_t* bond_off, const int32_t* src,
                         const int32_t* dst, const uint8_t* occ, int32_t* label, int32_t n_threads);

void gen_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void gen_u32(uint64_t seed, uint32_t stream, uint64_t first, int64_t n, uint32_t* out);
void gen_bernoulli_mask(uint64_t seed, uint32_t stream, uint64_t first, int64_t n, double p, uint8_t* out);
void gen_permutation(uint64_t seed, uint32_t stream, int64_t n, int32_t* perm);
void gen_honeycomb_edges(int32_t L, int32_t* src, int32_t* dst);
void gen_honeycomb_csr(int32_t L, int32_t* row_ptr, int32_t* col);
void gen_triangle_edges(int32_t L, int32_t* src, int32_t* dst);
void gen_triangle_csr(int32_t L, int32_t* row_ptr, int32_t* col);
int64_t gen_cayley_size(int32_t shells);
void gen_cayley_tree(int32_t shells, int32_t* src, int32_t* dst);
int64_t gen_random_regular(int64_t n, int32_t z, uint64_t seed, int32_t* src, int32_t* dst);
void gen_apply_permutation(int64_t m, const int32_t* perm, int32_t* src, int32_t* dst);
void gen_shuffle_edges(uint64_t seed, uint32_t stream, int64_t m, int32_t* src, int32_t* dst);
void gen_random_orientation(uint64_t seed, uint32_t stream, int64_t m, int32_t* src, int32_t* dst);
uint64_t gen_mix_seed(uint64_t base, uint64_t k);
int gen_ell_from_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint8_t* occ,
                       int32_t z_max, int32_t pad, int32_t* nn, uint8_t* occ_ell);

static int failures = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

static void* xmalloc(size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  return p;
}

/* edge list, CSR and neighbour list of one lattice give one labeling */
static void lattice_forms(int honeycomb, int32_t L, double p, uint64_t seed) {
  const int64_t n = honeycomb ? 2 * (int64_t)L * L : (int64_t)L * L, m = 3 * (int64_t)L * L;
  int32_t *src = xmalloc(4 * m), *dst = xmalloc(4 * m), *col = xmalloc(4 * m), *rp = xmalloc(4 * (n + 1));
  uint8_t* occ = xmalloc(m);
  if (honeycomb) {
    gen_honeycomb_edges(L, src, dst);
    gen_honeycomb_csr(L, rp, col);
  } else {
    gen_triangle_edges(L, src, dst);
    gen_triangle_csr(L, rp, col);
  }
  gen_bernoulli_mask(seed, 0, 0, m, p, occ);
  int32_t *a = xmalloc(4 * n), *b = xmalloc(4 * n), *c = xmalloc(4 * n);
  CHECK(oracle_label_edges(n, m, src, dst, occ, a) == 0);
  if (!honeycomb) {  /* the triangle CSR lists bond b of the edge list at position b */
    CHECK(oracle_label_csr(n, rp, col, occ, b) == 0);
    CHECK(memcmp(a, b, 4 * n) == 0);
  } else {
    CHECK(oracle_label_csr(n, rp, col, NULL, b) == 0);
    CHECK(oracle_label_edges(n, m, src, dst, NULL, c) == 0);
    CHECK(memcmp(b, c, 4 * n) == 0);
  }
  const int32_t z = 6;
  int32_t* nn = xmalloc(4 * n * z);
  uint8_t* occ_ell = xmalloc(n * z);
  CHECK(gen_ell_from_edges(n, m, src, dst, occ, z, -1, nn, occ_ell) == 0);
  CHECK(oracle_label_ell(n, z, nn, occ_ell, c) == 0);
  CHECK(memcmp(a, c, 4 * n) == 0);
  for (int64_t i = 0; i < n; ++i) CHECK(a[i] <= i && a[a[i]] == a[i]);
  free(src), free(dst), free(col), free(rp), free(occ), free(a), free(b), free(c), free(nn), free(occ_ell);
}

static void random_graphs(void) {
  const int32_t zs[3] = {3, 4, 6};
  for (int k = 0; k < 3; ++k) {
    const int64_t n = 20000, m = n * zs[k] / 2;
    int32_t *src = xmalloc(4 * m), *dst = xmalloc(4 * m), *perm = xmalloc(4 * n);
    CHECK(gen_random_regular(n, zs[k], gen_mix_seed(11, k), src, dst) >= 0);  /* repairs made */
    int32_t* deg = calloc((size_t)n, sizeof(int32_t));
    for (int64_t b = 0; b < m; ++b) {
      CHECK(src[b] != dst[b]);
      ++deg[src[b]];
      ++deg[dst[b]];
    }
    for (int64_t i = 0; i < n; ++i) CHECK(deg[i] == zs[k]);
    free(deg);
    gen_permutation(5, 2, n, perm);
    gen_apply_permutation(m, perm, src, dst);
    gen_shuffle_edges(6, 3, m, src, dst);
    gen_random_orientation(7, 4, m, src, dst);
    uint8_t* occ = xmalloc(m);
    gen_bernoulli_mask(9, 0, 3, m, 1.0 / (zs[k] - 1), occ);
    int32_t* lab = xmalloc(4 * n);
    CHECK(oracle_label_edges(n, m, src, dst, occ, lab) == 0);
    int64_t clusters = 0;
    for (int64_t i = 0; i < n; ++i) clusters += lab[i] == i;
    CHECK(clusters >= 1 && clusters <= n);
    free(src), free(dst), free(perm), free(occ), free(lab);
  }
  /* a Cayley tree: clusters = sites - occupied bonds */
  const int64_t n = gen_cayley_size(12), m = n - 1;
  int32_t *src = xmalloc(4 * m), *dst = xmalloc(4 * m), *lab = xmalloc(4 * n);
  uint8_t* occ = xmalloc(m);
  gen_cayley_tree(12, src, dst);
  gen_bernoulli_mask(3, 0, 0, m, 0.5, occ);
  CHECK(oracle_label_edges(n, m, src, dst, occ, lab) == 0);
  int64_t clusters = 0, on = 0;
  for (int64_t i = 0; i < n; ++i) clusters += lab[i] == i;
  for (int64_t b = 0; b < m; ++b) on += occ[b] != 0;
  CHECK(clusters == n - on);
  /* out-of-range ids are refused, not read past */
  src[0] = (int32_t)n;
  CHECK(oracle_label_edges(n, m, src, dst, occ, lab) == -1);
  free(src), free(dst), free(lab), free(occ);
}

static void generators(void) {
  const uint32_t zero[4] = {0, 0, 0, 0}, kz[2] = {0, 0};
  uint32_t out[4];
  gen_philox4x32_10(zero, kz, out);
  CHECK(out[0] == 0x6627e8d5u && out[1] == 0xe169c58du && out[2] == 0xbc57ac4cu && out[3] == 0x9b00dbd8u);
  uint32_t* w = xmalloc(4 * 1001);
  gen_u32(gen_mix_seed(7, 3), 3, 5, 1001, w);
  uint8_t* mask = xmalloc(1003);
  for (int first = 0; first < 4; ++first) gen_bernoulli_mask(11, 0, first, 1003 - first, 0.3473, mask);
  gen_bernoulli_mask(11, 0, 0, 0, 0.5, mask);
  free(w), free(mask);
}

static void batched(int n_threads) {
  enum { K = 37 };
  int64_t so[K + 1], bo[K + 1];
  so[0] = bo[0] = 0;
  for (int k = 0; k < K; ++k) {
    const int32_t L = 4 + 3 * (k % 9);
    so[k + 1] = so[k] + (int64_t)L * L;
    bo[k + 1] = bo[k] + 3 * (int64_t)L * L;
  }
  int32_t *src = xmalloc(4 * bo[K]), *dst = xmalloc(4 * bo[K]);
  int32_t *lab = xmalloc(4 * so[K]), *one = xmalloc(4 * so[K]);
  uint8_t* occ = xmalloc(bo[K]);
  for (int k = 0; k < K; ++k) {
    const int32_t L = 4 + 3 * (k % 9);
    gen_triangle_edges(L, src + bo[k], dst + bo[k]);
    gen_bernoulli_mask(gen_mix_seed(4, k), 0, 0, bo[k + 1] - bo[k], 0.3473, occ + bo[k]);
    CHECK(oracle_label_edges(so[k + 1] - so[k], bo[k + 1] - bo[k], src + bo[k], dst + bo[k], occ + bo[k],
                             one + so[k]) == 0);
  }
  CHECK(oracle_label_batched(K, so, bo, src, dst, occ, lab, n_threads) == 0);
  CHECK(memcmp(lab, one, 4 * so[K]) == 0);
  free(src), free(dst), free(lab), free(one), free(occ);
}

int main(int argc, char** argv) {
  const int threads_only = argc > 1 && strcmp(argv[1], "threads") == 0;
  if (!threads_only) {
    generators();
    lattice_forms(0, 37, 0.3473, 1);
    lattice_forms(1, 29, 0.6527, 2);
    random_graphs();
  }
  batched(1);
  batched(8);
  batched(3);
  if (failures) fprintf(stderr, "%d checks failed\n", failures);
  else printf("all checks passed\n");
  return failures ? 1 : 0;
}
