/*
 * Seeded synthetic inputs for bond percolation (paper section 4): counter-based
 * random numbers and the graph builders for the honeycomb and triangle
 * lattices, the z = 3 Cayley tree (the "Bethe lattice" of section 4) and random
 * z-regular graphs from the configuration model.
 *
 * This module holds none of the labeling arithmetic.  Its output (edge lists,
 * CSR arrays, occupancy masks) is fed unchanged both to the CPU oracle and to
 * the GPU library, so the two sides never draw random numbers themselves.
 *
 * Random numbers: Philox4x32-10, written from its published definition
 * (J. Salmon, M. Moraes, R. Dror, D. Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): a 4x32-bit counter, a 2x32-bit key, ten rounds of two
 * 32x32->64 multiplications with the key bumped by the Weyl constants between
 * rounds.  The paper drew its numbers from cuRAND XORWOW; that generator is a
 * closed library and is replaced here.
 *
 * Word i of stream s under seed S is word (i mod 4) of
 *   philox(counter = {lo32(i/4), hi32(i/4), s, 0}, key = {lo32(S), hi32(S)}).
 * A bond b is occupied iff word b of the occupancy stream is below
 * T = floor(p * 2^32) (all bonds occupied when p >= 1).
 *
 * Build: gcc -O3 -fopenmp -shared -fPIC gen.c -o libcclgen.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static inline void philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                uint32_t k0, uint32_t k1, uint32_t out[4]) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

void gen_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox_block(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1], out);
}

/* words [first, first + n) of stream `stream` */
void gen_u32(uint64_t seed, uint32_t stream, uint64_t first, int64_t n, uint32_t* out) {
  if (n <= 0) return;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint64_t blk_lo = first >> 2, blk_hi = (first + (uint64_t)n - 1) >> 2;
#pragma omp parallel for schedule(static)
  for (int64_t b = (int64_t)blk_lo; b <= (int64_t)blk_hi; ++b) {
    uint32_t w[4];
    philox_block((uint32_t)b, (uint32_t)((uint64_t)b >> 32), stream, 0u, k0, k1, w);
    for (int j = 0; j < 4; ++j) {
      uint64_t idx = ((uint64_t)b << 2) + (uint64_t)j;
      if (idx >= first && idx < first + (uint64_t)n) out[idx - first] = w[j];
    }
  }
}

/* T with u32 < T <=> occupied; 2^32 means every bond is occupied */
uint64_t gen_threshold(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return (uint64_t)1 << 32;
  return (uint64_t)floor(p * 4294967296.0);
}

void gen_bernoulli_mask(uint64_t seed, uint32_t stream, uint64_t first, int64_t n, double p,
                        uint8_t* out) {
  if (n <= 0) return;
  const uint64_t T = gen_threshold(p);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint64_t blk_lo = first >> 2, blk_hi = (first + (uint64_t)n - 1) >> 2;
#pragma omp parallel for schedule(static)
  for (int64_t b = (int64_t)blk_lo; b <= (int64_t)blk_hi; ++b) {
    uint32_t w[4];
    philox_block((uint32_t)b, (uint32_t)((uint64_t)b >> 32), stream, 0u, k0, k1, w);
    for (int j = 0; j < 4; ++j) {
      uint64_t idx = ((uint64_t)b << 2) + (uint64_t)j;
      if (idx >= first && idx < first + (uint64_t)n) out[idx - first] = (uint64_t)w[j] < T;
    }
  }
}

/* ---- sequential draws (used where an algorithm consumes numbers in order) ---- */

typedef struct {
  uint32_t k0, k1, stream;
  uint64_t block;
  uint32_t buf[4];
  int used;
} seq_rng;

static void seq_init(seq_rng* r, uint64_t seed, uint32_t stream) {
  r->k0 = (uint32_t)seed;
  r->k1 = (uint32_t)(seed >> 32);
  r->stream = stream;
  r->block = 0;
  r->used = 4;
}

static uint32_t seq_u32(seq_rng* r) {
  if (r->used == 4) {
    philox_block((uint32_t)r->block, (uint32_t)(r->block >> 32), r->stream, 0u, r->k0, r->k1,
                 r->buf);
    r->block++;
    r->used = 0;
  }
  return r->buf[r->used++];
}

static uint64_t seq_u64(seq_rng* r) {
  uint64_t lo = seq_u32(r);
  uint64_t hi = seq_u32(r);
  return (hi << 32) | lo;
}

/* uniform integer in [0, n), n >= 1: Lemire's multiply-shift with rejection
 * (D. Lemire, "Fast random integer generation in an interval", TOMACS 2019) */
static uint64_t seq_below(seq_rng* r, uint64_t n) {
  uint64_t x = seq_u64(r);
  __uint128_t m = (__uint128_t)x * n;
  uint64_t l = (uint64_t)m;
  if (l < n) {
    uint64_t t = (0 - n) % n;
    while (l < t) {
      x = seq_u64(r);
      m = (__uint128_t)x * n;
      l = (uint64_t)m;
    }
  }
  return (uint64_t)(m >> 64);
}

/* Fisher-Yates shuffle of int32 values */
static void shuffle_i32(seq_rng* r, int32_t* a, int64_t n) {
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)seq_below(r, (uint64_t)i + 1);
    int32_t t = a[i];
    a[i] = a[j];
    a[j] = t;
  }
}

/* random permutation of [0, n) */
void gen_permutation(uint64_t seed, uint32_t stream, int64_t n, int32_t* perm) {
  seq_rng r;
  seq_init(&r, seed, stream);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  shuffle_i32(&r, perm, n);
}

/* ---- lattices (ids 0-based, periodic in both directions) ---- */

/* Honeycomb as two-site cells on an L x L torus: A(x,y) = 2(yL+x), B = A+1.
 * Cell c = yL+x owns bonds 3c..3c+2: A(x,y)-B(x,y), A(x,y)-B(x-1,y),
 * A(x,y)-B(x,y-1).  N = 2L^2 sites, 3L^2 bonds, every site has 3 neighbours. */
void gen_honeycomb_edges(int32_t L, int32_t* src, int32_t* dst) {
#pragma omp parallel for schedule(static)
  for (int64_t y = 0; y < L; ++y) {
    for (int64_t x = 0; x < L; ++x) {
      int64_t c = y * L + x;
      int32_t a = (int32_t)(2 * c);
      int64_t xm = (x + L - 1) % L, ym = (y + L - 1) % L;
      src[3 * c + 0] = a;
      dst[3 * c + 0] = a + 1;
      src[3 * c + 1] = a;
      dst[3 * c + 1] = (int32_t)(2 * (y * L + xm) + 1);
      src[3 * c + 2] = a;
      dst[3 * c + 2] = (int32_t)(2 * (ym * L + x) + 1);
    }
  }
}

/* Honeycomb in half-CSR: row A(x,y) holds its three bonds in the order above,
 * rows of B sites are empty.  row_ptr has 2L^2 + 1 entries. */
void gen_honeycomb_csr(int32_t L, int32_t* row_ptr, int32_t* col) {
  const int64_t cells = (int64_t)L * L;
#pragma omp parallel for schedule(static)
  for (int64_t y = 0; y < L; ++y) {
    for (int64_t x = 0; x < L; ++x) {
      int64_t c = y * L + x;
      int64_t xm = (x + L - 1) % L, ym = (y + L - 1) % L;
      row_ptr[2 * c] = (int32_t)(3 * c);
      row_ptr[2 * c + 1] = (int32_t)(3 * c + 3);
      col[3 * c + 0] = (int32_t)(2 * c + 1);
      col[3 * c + 1] = (int32_t)(2 * (y * L + xm) + 1);
      col[3 * c + 2] = (int32_t)(2 * (ym * L + x) + 1);
    }
  }
  row_ptr[2 * cells] = (int32_t)(3 * cells);
}

/* Triangle lattice: site yL+x, forward bonds to (x+1,y), (x,y+1), (x+1,y+1)
 * (mod L); N = L^2 sites, 3L^2 bonds, coordination 6. */
void gen_triangle_edges(int32_t L, int32_t* src, int32_t* dst) {
#pragma omp parallel for schedule(static)
  for (int64_t y = 0; y < L; ++y) {
    int64_t yp = (y + 1) % L;
    for (int64_t x = 0; x < L; ++x) {
      int64_t c = y * L + x, xp = (x + 1) % L;
      src[3 * c + 0] = (int32_t)c;
      dst[3 * c + 0] = (int32_t)(y * L + xp);
      src[3 * c + 1] = (int32_t)c;
      dst[3 * c + 1] = (int32_t)(yp * L + x);
      src[3 * c + 2] = (int32_t)c;
      dst[3 * c + 2] = (int32_t)(yp * L + xp);
    }
  }
}

/* Triangle lattice in half-CSR: row_ptr[i] = 3i, col in the order above. */
void gen_triangle_csr(int32_t L, int32_t* row_ptr, int32_t* col) {
  const int64_t n = (int64_t)L * L;
#pragma omp parallel for schedule(static)
  for (int64_t y = 0; y < L; ++y) {
    int64_t yp = (y + 1) % L;
    for (int64_t x = 0; x < L; ++x) {
      int64_t c = y * L + x, xp = (x + 1) % L;
      row_ptr[c] = (int32_t)(3 * c);
      col[3 * c + 0] = (int32_t)(y * L + xp);
      col[3 * c + 1] = (int32_t)(yp * L + x);
      col[3 * c + 2] = (int32_t)(yp * L + xp);
    }
  }
  row_ptr[n] = (int32_t)(3 * n);
}

/* ---- Cayley tree (the finite Bethe lattice of section 4), z = 3 ----
 * Centre 0, shell 1 = {1,2,3}, every site of shell g >= 1 has two children
 * in shell g+1; sites numbered shell by shell ("standard position").
 * N = 3*2^G - 2 sites, N - 1 bonds; bond v-1 joins site v to its parent. */
int64_t gen_cayley_size(int32_t shells) { return shells <= 0 ? 1 : 3 * ((int64_t)1 << shells) - 2; }

void gen_cayley_tree(int32_t shells, int32_t* src, int32_t* dst) {
  const int64_t n = gen_cayley_size(shells);
#pragma omp parallel for schedule(static)
  for (int64_t v = 1; v < n; ++v) {
    int64_t parent;
    if (v <= 3) {
      parent = 0;
    } else {
      /* shell g starts at 3*2^(g-1) - 2 */
      int g = 1;
      while (3 * ((int64_t)1 << g) - 2 <= v) ++g;
      int64_t start = 3 * ((int64_t)1 << (g - 1)) - 2;
      int64_t prev_start = 3 * ((int64_t)1 << (g - 2)) - 2;
      parent = prev_start + (v - start) / 2;
    }
    src[v - 1] = (int32_t)v;
    dst[v - 1] = (int32_t)parent;
  }
}

/* ---- random z-regular graph: configuration model, simple ----
 * Stubs s in [0, nz) belong to site s / z; a uniform shuffle pairs stub 2k
 * with stub 2k+1.  Self-loops and repeated pairs are then repaired one at a
 * time by swapping endpoints with a uniformly chosen good edge, accepting the
 * swap only if both new edges are new non-loop edges.  Streams: 1 (shuffle
 * and repairs).  Returns the number of repairs, -1 on bad arguments and -2
 * when a repair finds no admissible swap. */

typedef struct {
  uint64_t* keys;
  uint64_t mask;
} edge_set;

#define SET_EMPTY 0xFFFFFFFFFFFFFFFFull
#define SET_TOMB 0xFFFFFFFFFFFFFFFEull

static uint64_t edge_key(int32_t a, int32_t b) {
  uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
  return ((uint64_t)lo << 32) | hi;
}

static uint64_t key_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

static int set_contains(const edge_set* s, uint64_t k) {
  uint64_t h = key_hash(k) & s->mask;
  while (s->keys[h] != SET_EMPTY) {
    if (s->keys[h] == k) return 1;
    h = (h + 1) & s->mask;
  }
  return 0;
}

/* returns 1 if inserted, 0 if present */
static int set_insert(edge_set* s, uint64_t k) {
  uint64_t h = key_hash(k) & s->mask;
  int64_t tomb = -1;
  while (s->keys[h] != SET_EMPTY) {
    if (s->keys[h] == k) return 0;
    if (s->keys[h] == SET_TOMB && tomb < 0) tomb = (int64_t)h;
    h = (h + 1) & s->mask;
  }
  s->keys[tomb >= 0 ? (uint64_t)tomb : h] = k;
  return 1;
}

static void set_erase(edge_set* s, uint64_t k) {
  uint64_t h = key_hash(k) & s->mask;
  while (s->keys[h] != SET_EMPTY) {
    if (s->keys[h] == k) {
      s->keys[h] = SET_TOMB;
      return;
    }
    h = (h + 1) & s->mask;
  }
}

int64_t gen_random_regular(int64_t n, int32_t z, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n <= 0 || z <= 0 || (n * z) % 2 != 0 || n > INT32_MAX || z >= n) return -1;
  const int64_t stubs = n * z, m = stubs / 2;
  int32_t* st = (int32_t*)malloc((size_t)stubs * sizeof(int32_t));
  uint8_t* bad = (uint8_t*)calloc((size_t)m, 1);
  uint64_t cap = 1;
  while (cap < 2 * (uint64_t)m + 16) cap <<= 1;
  edge_set set = {(uint64_t*)malloc(cap * sizeof(uint64_t)), cap - 1};
  if (!st || !bad || !set.keys) {
    free(st);
    free(bad);
    free(set.keys);
    return -1;
  }
  memset(set.keys, 0xFF, cap * sizeof(uint64_t));
  for (int64_t s = 0; s < stubs; ++s) st[s] = (int32_t)(s / z);
  seq_rng r;
  seq_init(&r, seed, 1u);
  shuffle_i32(&r, st, stubs);
  int64_t n_bad = 0;
  for (int64_t k = 0; k < m; ++k) {
    src[k] = st[2 * k];
    dst[k] = st[2 * k + 1];
    if (src[k] == dst[k] || !set_insert(&set, edge_key(src[k], dst[k]))) {
      bad[k] = 1;
      ++n_bad;
    }
  }
  free(st);
  int64_t repairs = 0;
  for (int64_t k = 0; k < m && n_bad > 0; ++k) {
    if (!bad[k]) continue;
    int64_t tries = 0;
    for (;;) {
      if (++tries > 1000 * m + 1000) {
        /* no admissible swap found: give up (only tiny graphs get here) */
        free(bad);
        free(set.keys);
        return -2;
      }
      int64_t j = (int64_t)seq_below(&r, (uint64_t)m);
      if (bad[j]) continue;
      int flip = (int)(seq_u32(&r) & 1u);
      int32_t a = src[k], b = dst[k], c = flip ? dst[j] : src[j], d = flip ? src[j] : dst[j];
      /* proposal: (a,c) and (b,d) replace (a,b) and (c,d) */
      if (a == c || b == d) continue;
      uint64_t k1 = edge_key(a, c), k2 = edge_key(b, d);
      if (k1 == k2 || set_contains(&set, k1) || set_contains(&set, k2)) continue;
      set_erase(&set, edge_key(src[j], dst[j]));
      set_insert(&set, k1);
      set_insert(&set, k2);
      src[k] = a;
      dst[k] = c;
      src[j] = b;
      dst[j] = d;
      bad[k] = 0;
      --n_bad;
      ++repairs;
      break;
    }
  }
  free(bad);
  free(set.keys);
  return repairs;
}

/* ---- relabelling and shuffling of an edge list ("random position") ---- */

/* src/dst <- perm[src/dst] */
void gen_apply_permutation(int64_t m, const int32_t* perm, int32_t* src, int32_t* dst) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    src[k] = perm[src[k]];
    dst[k] = perm[dst[k]];
  }
}

/* uniform shuffle of the edge order (sequential stream `stream`) */
void gen_shuffle_edges(uint64_t seed, uint32_t stream, int64_t m, int32_t* src, int32_t* dst) {
  seq_rng r;
  seq_init(&r, seed, stream);
  for (int64_t i = m - 1; i > 0; --i) {
    int64_t j = (int64_t)seq_below(&r, (uint64_t)i + 1);
    int32_t t = src[i];
    src[i] = src[j];
    src[j] = t;
    t = dst[i];
    dst[i] = dst[j];
    dst[j] = t;
  }
}

/* swap the endpoints of edge k when bit 0 of word k of `stream` is set */
void gen_random_orientation(uint64_t seed, uint32_t stream, int64_t m, int32_t* src, int32_t* dst) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < (m + 3) / 4; ++b) {
    uint32_t w[4];
    philox_block((uint32_t)b, (uint32_t)((uint64_t)b >> 32), stream, 0u, k0, k1, w);
    for (int j = 0; j < 4; ++j) {
      int64_t k = 4 * b + j;
      if (k < m && (w[j] & 1u)) {
        int32_t t = src[k];
        src[k] = dst[k];
        dst[k] = t;
      }
    }
  }
}

/* SplitMix64 finaliser (G. Steele, D. Lea, C. Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): per-instance seeds. */
uint64_t gen_mix_seed(uint64_t base, uint64_t k) {
  uint64_t z = base + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* The paper's padded, column-major neighbour list (section 3) of an
 * undirected bond list: bond b is entered in the lists of both its ends, in
 * bond order, with occupancy occ[b] (1 when occ is NULL); slot k of site i is
 * nn[k*n + i], unused slots hold `pad` (occupancy 0).  occ_ell may be NULL.
 * Returns 0, or -1 when a site would need more than z_max slots. */
int gen_ell_from_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                       const uint8_t* occ, int32_t z_max, int32_t pad, int32_t* nn,
                       uint8_t* occ_ell) {
  int32_t* fill = (int32_t*)calloc(n > 0 ? (size_t)n : 1, sizeof(int32_t));
  if (!fill) return -1;
  for (int64_t s = 0; s < n * (int64_t)z_max; ++s) {
    nn[s] = pad;
    if (occ_ell) occ_ell[s] = 0;
  }
  for (int64_t b = 0; b < m; ++b) {
    const int32_t ends[2][2] = {{src[b], dst[b]}, {dst[b], src[b]}};
    for (int e = 0; e < 2; ++e) {
      const int32_t u = ends[e][0];
      const int32_t k = fill[u]++;
      if (k >= z_max) {
        free(fill);
        return -1;
      }
      nn[(int64_t)k * n + u] = ends[e][1];
      if (occ_ell) occ_ell[(int64_t)k * n + u] = occ ? occ[b] : 1;
    }
  }
  free(fill);
  return 0;
}
