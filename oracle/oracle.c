/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, obviously-correct labeling of the clusters of occupied
 * bonds.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the GPU library neither links nor calls it, and it
 * shares no source with the GPU library.
 *
 * What it computes (the plain definition the method reaches exactly):
 *   label[i] = min { j : j is joined to i by a path of occupied bonds }.
 * Labels come from local connection information only (paper, section 2); a
 * bond is occupied with probability p (section 4), given here as a mask; the
 * label of each cluster is the minimum site number in that cluster (section 3,
 * the remark following the description of the four steps).
 *
 * How: a textbook sequential union-find over the parent array `label`.  Sets
 * are always joined by pointing the larger root at the smaller one, so every
 * root is the minimum of its set; a final find per site writes that minimum.
 * Finds use path halving (a sequential program, so no races).
 *
 * Conventions (readings of the paper where it is silent): site ids are
 * 0-based; a NULL mask means every bond is occupied; self-loops and repeated
 * bonds are allowed and change nothing; an id outside [0, n) is an error.
 *
 * Build: gcc -O2 -pthread -shared -fPIC oracle.c -o liboracle.so
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

static int32_t root_of(int32_t* parent, int32_t x) {
  while (parent[x] != x) {
    parent[x] = parent[parent[x]];
    x = parent[x];
  }
  return x;
}

static void join(int32_t* parent, int32_t a, int32_t b) {
  int32_t ra = root_of(parent, a);
  int32_t rb = root_of(parent, b);
  if (ra < rb)
    parent[rb] = ra;
  else if (rb < ra)
    parent[ra] = rb;
}

static void finish(int32_t* label, int64_t n) {
  for (int64_t i = 0; i < n; ++i) label[i] = root_of(label, (int32_t)i);
}

/* Edge list: bond b joins src[b] and dst[b] when occ[b] != 0.
 * Returns 0, or -1 for bad sizes / ids (label contents then unspecified). */
int oracle_label_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                       const uint8_t* occ, int32_t* label) {
  if (n < 0 || m < 0 || n > INT32_MAX) return -1;
  for (int64_t b = 0; b < m; ++b)
    if (src[b] < 0 || src[b] >= n || dst[b] < 0 || dst[b] >= n) return -1;
  for (int64_t i = 0; i < n; ++i) label[i] = (int32_t)i;
  for (int64_t b = 0; b < m; ++b)
    if (occ == NULL || occ[b] != 0) join(label, src[b], dst[b]);
  finish(label, n);
  return 0;
}

/* CSR: row i holds the bonds (i, col[e]) for e in [row_ptr[i], row_ptr[i+1]),
 * with occ aligned to col. */
int oracle_label_csr(int64_t n, const int32_t* row_ptr, const int32_t* col, const uint8_t* occ,
                     int32_t* label) {
  if (n < 0 || n > INT32_MAX) return -1;
  if (n > 0 && row_ptr[0] < 0) return -1;
  for (int64_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return -1;
  for (int64_t e = n > 0 ? row_ptr[0] : 0; e < (n > 0 ? row_ptr[n] : 0); ++e)
    if (col[e] < 0 || col[e] >= n) return -1;
  for (int64_t i = 0; i < n; ++i) label[i] = (int32_t)i;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
      if (occ == NULL || occ[e] != 0) join(label, (int32_t)i, col[e]);
  finish(label, n);
  return 0;
}

/* Padded neighbour list as the paper stores it (section 3): site i reads
 * nn[i], nn[i + n], nn[i + 2n], ... up to z_max entries; entries < 0 are
 * padding.  The occupancy of the bond in slot (i, k) is occ[i + k n]; both
 * directions of a bond must carry the same value. */
int oracle_label_ell(int64_t n, int32_t z_max, const int32_t* nn, const uint8_t* occ,
                     int32_t* label) {
  if (n < 0 || n > INT32_MAX || z_max < 0) return -1;
  for (int64_t s = 0; s < n * (int64_t)z_max; ++s)
    if (nn[s] >= n) return -1;
  for (int64_t i = 0; i < n; ++i) label[i] = (int32_t)i;
  for (int64_t k = 0; k < z_max; ++k)
    for (int64_t i = 0; i < n; ++i) {
      int32_t j = nn[i + k * n];
      if (j >= 0 && (occ == NULL || occ[i + k * n] != 0)) join(label, (int32_t)i, j);
    }
  finish(label, n);
  return 0;
}

/* ---- many independent instances, one per task on a pool of threads ---- */

typedef struct {
  int32_t n_inst;
  const int64_t* site_off;
  const int64_t* bond_off;
  const int32_t* src;
  const int32_t* dst;
  const uint8_t* occ;
  int32_t* label;
  int64_t next; /* next instance to take (guarded by lock) */
  int status;
  pthread_mutex_t lock;
} batch_job;

static void* batch_worker(void* arg) {
  batch_job* job = (batch_job*)arg;
  for (;;) {
    pthread_mutex_lock(&job->lock);
    int64_t k = job->next++;
    pthread_mutex_unlock(&job->lock);
    if (k >= job->n_inst) break;
    int64_t s0 = job->site_off[k], b0 = job->bond_off[k];
    int r = oracle_label_edges(job->site_off[k + 1] - s0, job->bond_off[k + 1] - b0, job->src + b0,
                               job->dst + b0, job->occ ? job->occ + b0 : NULL, job->label + s0);
    if (r != 0) {
      pthread_mutex_lock(&job->lock);
      job->status = r;
      pthread_mutex_unlock(&job->lock);
    }
  }
  return NULL;
}

/* Instance k owns sites [site_off[k], site_off[k+1]) and bonds
 * [bond_off[k], bond_off[k+1]); src/dst hold instance-local ids and the labels
 * written are instance-local.  n_threads <= 0 means one thread. */
int oracle_label_batched(int32_t n_inst, const int64_t* site_off, const int64_t* bond_off,
                         const int32_t* src, const int32_t* dst, const uint8_t* occ,
                         int32_t* label, int32_t n_threads) {
  if (n_inst < 0) return -1;
  batch_job job = {n_inst, site_off, bond_off, src, dst, occ, label, 0, 0,
                   PTHREAD_MUTEX_INITIALIZER};
  if (n_threads <= 1) {
    batch_worker(&job);
    return job.status;
  }
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
  if (!th) return -1;
  int started = 0;
  for (int t = 0; t < n_threads; ++t)
    if (pthread_create(&th[started], NULL, batch_worker, &job) == 0) ++started;
  if (started == 0) batch_worker(&job);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(th);
  return job.status;
}
