/*
 * ccl.h -- connected-component labeling of occupied bonds on one AMD
 * Instinct MI355X (gfx950).  C ABI of libccl.so.
 *
 * Method: the generalized non-iterative labeling of Komura, "A generalized
 * GPU-based connected component labeling algorithm" (arXiv:1603.08357):
 *   (i)   every site starts as its own root, label[i] = i (section 3, step i,
 *         the case of an empty residual list);
 *   (iii) every occupied bond joins the roots of its two ends with the
 *         atomicMin label reduction of Algorithm 1 -- one pass, no
 *         convergence loop;
 *   (iv)  the analysis step follows every label to its root (section 3).
 * On return every site holds the minimum site number of its cluster (section
 * 3: the label of each cluster is its minimum site number), so the result is
 * unique and independent of thread scheduling.
 *
 * Conventions for every entry point
 *   - Site ids are 0-based int32; n_sites <= INT32_MAX.
 *   - "device" pointers are HIP device allocations owned by the caller;
 *     inputs are read, never written; labels_out is fully overwritten and is
 *     also the union-find work array, so it must not overlap any input.
 *   - occupied: one byte per bond, nonzero = occupied (section 4: each bond is
 *     occupied with probability p); NULL means every bond is occupied.
 *   - Self-loops change nothing; repeated bonds and both orientations of a
 *     bond are allowed.
 *   - stream: a hipStream_t (NULL = the default stream).  Calls only enqueue
 *     work and return; the caller synchronizes.  No call on this path
 *     allocates device memory.  Calls on different streams may overlap when
 *     they touch disjoint buffers.
 *   - Argument errors are detected on the host before any HIP call and return
 *     CCL_ERR_INVALID_VALUE.  A site id outside [0, n_sites) on the labeling
 *     path is undefined behaviour (the kernels do not check ids); use
 *     ccl_validate_edges / ccl_validate_csr first on untrusted input.
 *   - After any error the contents of labels_out are unspecified.
 */
#ifndef CCL_H
#define CCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CCL_OK = 0,
  CCL_ERR_INVALID_VALUE = 1,      /* bad size, NULL pointer, aliasing, bad plan */
  CCL_ERR_INDEX_OUT_OF_RANGE = 2, /* reported by the validation calls only */
  CCL_ERR_OUT_OF_MEMORY = 3,      /* plan creation could not allocate */
  CCL_ERR_HIP = 4,                /* a HIP call failed; see ccl_last_hip_error() */
  CCL_ERR_NOT_SUPPORTED = 5,      /* device is not gfx950 */
  CCL_ERR_TOO_LARGE = 6           /* input exceeds a fixed capacity (no-allocation entry point, capacity plan) */
} ccl_status;

/* ---------------------------------------------------------------- labeling */

/*
 * Label the clusters of an edge list.
 *   n_sites    number of sites N (0 <= N <= INT32_MAX)
 *   n_bonds    number of bonds B (>= 0)
 *   src, dst   device int32[B]: bond b joins src[b] and dst[b]
 *   occupied   device uint8[B] or NULL
 *   labels_out device int32[N]: on return, the minimum site id of each site's
 *              cluster (isolated sites keep their own id)
 * Kernels: init (step i), bond-parallel merge (step iii, Algorithm 1),
 * flatten (step iv).
 */
ccl_status ccl_label(int64_t n_sites, int64_t n_bonds, const int32_t* src, const int32_t* dst,
                     const uint8_t* occupied, int32_t* labels_out, void* stream);

/*
 * ccl_label with the occupancy drawn inside the merge kernel instead of read
 * from a mask: bond b is occupied when word b of the Philox4x32-10 stream
 * (seed, stream_id) lies below floor(p 2^32), exactly the mask
 * ccl_bernoulli(seed, stream_id, 0, n_bonds, p, ...) writes (the Monte-Carlo
 * setting of section 4, with no mask in memory).  p is NaN:
 * CCL_ERR_INVALID_VALUE; p <= 0: no bond occupied; p >= 1: every bond.  The
 * other arguments and errors are ccl_label's.
 */
ccl_status ccl_label_philox(int64_t n_sites, int64_t n_bonds, const int32_t* src, const int32_t* dst,
                            uint64_t seed, uint32_t stream_id, double p, int32_t* labels_out,
                            void* stream);

/*
 * Label the clusters of a graph given as the paper's padded neighbour list
 * (section 3): z_max entries per site, column-major, so neighbour k of site
 * i is nn_list[k*N + i].  Runs the paper's own four steps: (i) each site's
 * label becomes its lowest occupied neighbour numbered below it (or its own
 * id), (ii) analysis, (iii) label reduction with Algorithm 1 over the rest of
 * each site's lower neighbours, (iv) analysis.
 *   n_sites    N (0 <= N <= INT32_MAX)
 *   z_max      entries per site (>= 0, N * z_max <= 2^40)
 *   nn_list    device int32[z_max * N]; an entry outside [0, N) is padding.
 *              A bond is seen from its higher-numbered end, so it must be
 *              listed there (listing both ends, as the paper does, is fine)
 *   occupied   device uint8[z_max * N] aligned with nn_list (nonzero =
 *              occupied; both listings of a bond should agree), or NULL
 *   labels_out device int32[N]: the minimum site id of each site's cluster
 * Same results as ccl_label over the listed bonds.  Asynchronous on stream.
 */
ccl_status ccl_label_ell(int64_t n_sites, int32_t z_max, const int32_t* nn_list,
                         const uint8_t* occupied, int32_t* labels_out, void* stream);

/*
 * Workspace bytes ccl_label_csr and ccl_label_csr_grid need (any grid width):
 * zero for n_sites <= 65536 (one tile), else one 8-byte slot per bond (the
 * bonds leaving their tile are collected there) plus a tile table of
 * 8 (4 ceil(N / 65536) + 2) bytes rounded up to 256 bytes.
 */
size_t ccl_label_csr_workspace_size(int64_t n_sites, int64_t n_bonds);

/*
 * Label the clusters of a graph in compressed-sparse-row form: row i holds the
 * bonds (i, col[e]) for e in [row_ptr[i], row_ptr[i+1]).  Each undirected bond
 * needs to appear once (a "half" CSR such as forward neighbours only), but
 * listing it in both rows is also correct.  The paper's neighbour list
 * (section 3) is this structure with all neighbours listed.
 *   n_sites    N (0 <= N <= INT32_MAX)
 *   n_bonds    at least row_ptr[N] - row_ptr[0] (e.g. the length of col);
 *              sizes the workspace, must not be smaller
 *   row_ptr    device int32[N+1], non-decreasing, row_ptr[0] >= 0
 *   col        device int32[], entries row_ptr[0] .. row_ptr[N]-1 are read
 *   occupied   device uint8[], aligned with col, or NULL
 *   workspace  device buffer of at least ccl_label_csr_workspace_size(N,
 *              n_bonds) bytes, 8-byte aligned, contents need not be
 *              initialised and are garbage afterwards; may be NULL when that
 *              size is zero
 * Kernels: sites are cut into tiles of 65536 consecutive ids; one workgroup
 * per tile initialises its labels (step i) and joins the tile-internal bonds
 * in LDS (step iii on the tile), recording the bonds that leave the tile in
 * the workspace; then those bonds are joined in global memory (step iii,
 * Algorithm 1) and the labels flattened (step iv).
 */
ccl_status ccl_label_csr(int64_t n_sites, int64_t n_bonds, const int32_t* row_ptr,
                         const int32_t* col, const uint8_t* occupied, int32_t* labels_out,
                         void* workspace, size_t workspace_bytes, void* stream);

/*
 * ccl_label_csr for a graph whose site ids number a grid row by row: site
 * y*grid_width + x (a lattice of row length grid_width, as the paper's
 * lattices are numbered).  The result does not depend on grid_width -- any
 * CSR graph is labelled correctly with any value -- but the tiles follow the
 * grid: 32 rows of 2048 columns instead of 65536 consecutive ids, so a tile
 * has a shorter boundary and fewer bonds leave it (on the 8192-wide
 * triangular lattice a quarter as many).  Used when grid_width is a multiple
 * of 4, larger than 2048 and smaller than n_sites with at least 32 rows;
 * otherwise (grid_width = 0 included) this is ccl_label_csr.  grid_width < 0:
 * CCL_ERR_INVALID_VALUE.  The other arguments, the workspace size and the
 * errors are ccl_label_csr's.
 */
ccl_status ccl_label_csr_grid(int64_t n_sites, int64_t n_bonds, int64_t grid_width,
                              const int32_t* row_ptr, const int32_t* col, const uint8_t* occupied,
                              int32_t* labels_out, void* workspace, size_t workspace_bytes,
                              void* stream);

/*
 * ccl_label_csr with the occupancy drawn inside the tile kernel instead of
 * read from a mask: bond e (the entry col[e]) is occupied when word e of the
 * Philox4x32-10 stream (seed, stream_id) lies below floor(p 2^32), exactly
 * the mask ccl_bernoulli(seed, stream_id, 0, row_ptr[N], p, ...) writes.
 * This is the Monte-Carlo setting of section 4 (a new random configuration
 * per sample) without a mask in memory: the draw costs arithmetic, not HBM
 * traffic.  p is NaN: CCL_ERR_INVALID_VALUE; p <= 0: no bond occupied;
 * p >= 1: every bond.  The other arguments and errors are ccl_label_csr's.
 */
ccl_status ccl_label_csr_philox(int64_t n_sites, int64_t n_bonds, const int32_t* row_ptr,
                                const int32_t* col, uint64_t seed, uint32_t stream_id, double p,
                                int32_t* labels_out, void* workspace, size_t workspace_bytes,
                                void* stream);

/* ccl_label_csr_philox with the grid tiles of ccl_label_csr_grid. */
ccl_status ccl_label_csr_grid_philox(int64_t n_sites, int64_t n_bonds, int64_t grid_width,
                                     const int32_t* row_ptr, const int32_t* col, uint64_t seed,
                                     uint32_t stream_id, double p, int32_t* labels_out,
                                     void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- batches */

/*
 * Many independent instances labelled in one launch.  Instance k owns sites
 * [site_off[k], site_off[k+1]) and bonds [bond_off[k], bond_off[k+1]) of the
 * concatenated arrays; src/dst hold instance-LOCAL ids (0 <= id <
 * site_off[k+1] - site_off[k] <= INT32_MAX) and the labels written are
 * instance-local.  Offsets are int64 so a batch may exceed 2^31 sites.
 */
typedef struct ccl_plan_s* ccl_plan;

/* Tuning of the persistent batched kernel; zero fields take defaults. */
typedef struct {
  int32_t block_threads;   /* threads per workgroup (multiple of 64, <= 1024) */
  int32_t blocks_per_cu;   /* resident workgroups per compute unit */
  int32_t bonds_per_chunk; /* bonds in one merge work item */
  int32_t sites_per_chunk; /* sites in one init / flatten work item */
  int32_t small_sites;     /* instances up to this many sites (<= 65536) are
                              labelled entirely in LDS by one workgroup, two
                              bytes of LDS per site; 0 = default (fits the
                              LDS of the resident workgroups), negative =
                              never */
  int32_t schedule;        /* 1 = fused: one persistent launch in which work
                              items wait for the items they depend on;
                              2 = phased: init, merge and flatten items as
                              three launches (no waiting);
                              3 = tiled: instances above small_sites are
                              cut into 65536-site tiles, each joined in LDS
                              by one workgroup from its range of the bond
                              list (the first bond whose src reaches the
                              tile's first site starts it; bonds listed in
                              order of src keep a tile's bonds together,
                              any order stays exact), then the bonds that
                              leave a tile are joined in global memory and
                              the labels of instances of several tiles are
                              flattened; bonds_per_chunk is not used;
                              0 = default (3) */
} ccl_tuning;

/*
 * Build a plan for one batch layout: reads the host copies of the offsets,
 * builds the work-item table and allocates it plus a few counters on the
 * current device (the only allocation of the batched path).
 *   n_inst          number of instances K (>= 0)
 *   site_off_host   host int64[K+1], site_off[0] = 0, non-decreasing
 *   bond_off_host   host int64[K+1], bond_off[0] = 0, non-decreasing
 *   tuning          NULL = defaults
 *   out             receives the plan
 * Returns CCL_ERR_INVALID_VALUE for bad offsets, CCL_ERR_OUT_OF_MEMORY /
 * CCL_ERR_HIP when the device allocation fails.
 */
ccl_status ccl_plan_create(int32_t n_inst, const int64_t* site_off_host,
                           const int64_t* bond_off_host, const ccl_tuning* tuning,
                           ccl_plan* out);

/*
 * A plan for many layouts, for a loop that labels a changing group of
 * instances (the ready requests of a serving tick) with one batched launch
 * each time: the device tables are allocated once, sized for every layout of
 * at most max_inst instances, max_sites sites and max_bonds bonds in total;
 * ccl_plan_set_layout gives the plan the layout of its next launches.  Until
 * a layout is set the plan has none and ccl_label_batched does nothing.
 * Returns CCL_ERR_INVALID_VALUE for negative limits or a bad tuning,
 * CCL_ERR_TOO_LARGE when the tables would exceed the work-item fields,
 * CCL_ERR_OUT_OF_MEMORY / CCL_ERR_HIP when an allocation fails.
 */
ccl_status ccl_plan_create_capacity(int32_t max_inst, int64_t max_sites, int64_t max_bonds,
                                    const ccl_tuning* tuning, ccl_plan* out);

/*
 * Sets the layout of a capacity plan without allocating and without a device
 * synchronization: builds the work tables on the host (offsets as for
 * ccl_plan_create), copies them into the plan's pinned staging and enqueues
 * their upload on `stream`, which must be the stream of the launches that use
 * the layout (launches of the previous layout already enqueued there run
 * first).  The call waits only until the previous layout's upload has left
 * the staging.  CCL_ERR_TOO_LARGE: the layout exceeds the plan's limits;
 * CCL_ERR_INVALID_VALUE: bad offsets, or a plan made by ccl_plan_create.
 */
ccl_status ccl_plan_set_layout(ccl_plan plan, int32_t n_inst, const int64_t* site_off_host,
                               const int64_t* bond_off_host, void* stream);

/* Frees a plan (synchronizes the device first). NULL is a no-op. */
ccl_status ccl_plan_destroy(ccl_plan plan);

/* The tuning a plan resolved to (defaults filled in). */
ccl_status ccl_plan_get_tuning(ccl_plan plan, ccl_tuning* out);

/*
 * Synchronous health check after a batched launch has finished: *error_host
 * is nonzero when a work item gave up waiting for the items it depends on
 * (its spin limit was hit; the labels of that launch are then unreliable).
 * The batched kernel bounds every wait, so it always terminates.
 */
ccl_status ccl_plan_check(ccl_plan plan, int32_t* error_host);

/*
 * Label every instance of the plan's layout: a small kernel that resets the
 * plan's counters (no memset node, so the launches can be captured into a HIP
 * graph and replayed), then the persistent kernel -- one launch for the fused
 * schedule, three for the phased one; the tiled schedule adds a launch that
 * finds the tiles' bond ranges, the tile launch and the leaving-bond launch.
 *   src, dst   device int32[total bonds], instance-local ids
 *   occupied   device uint8[total bonds] or NULL
 *   labels_out device int32[total sites]
 * A plan may be in flight on one stream at a time.
 */
ccl_status ccl_label_batched(ccl_plan plan, const int32_t* src, const int32_t* dst,
                             const uint8_t* occupied, int32_t* labels_out, void* stream);

/*
 * Reference schedule for batches: one ccl_label call per instance, in order,
 * on `stream` (the "one launch per instance" baseline).  Host offsets only.
 */
ccl_status ccl_label_batched_per_instance(int32_t n_inst, const int64_t* site_off_host,
                                          const int64_t* bond_off_host, const int32_t* src,
                                          const int32_t* dst, const uint8_t* occupied,
                                          int32_t* labels_out, void* stream);

/* ------------------------------------------------- occupancy on the device */

/*
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), the counter-based
 * generator used here in place of the paper's cuRAND draws (section 4).
 * Word w of stream `stream_id` under `seed` is output word w mod 4 of the
 * block with counter (b mod 2^32, b div 2^32, stream_id, 0), b = w div 4, and
 * key (seed mod 2^32, seed div 2^32).
 *   ccl_philox_u32: out[i] = word first + i, for i < n (device uint32[n])
 *   ccl_bernoulli:  out[i] = 1 when word first + i < floor(p 2^32) (every
 *                   bond when p >= 1, none when p <= 0), else 0 (device
 *                   uint8[n]): bond occupancy with probability p
 * n >= 0, first + n must not exceed 2^64.  Asynchronous on `stream`.
 */
ccl_status ccl_philox_u32(uint64_t seed, uint32_t stream_id, uint64_t first, int64_t n,
                          uint32_t* out, void* stream);
ccl_status ccl_bernoulli(uint64_t seed, uint32_t stream_id, uint64_t first, int64_t n, double p,
                         uint8_t* out, void* stream);

/* ------------------------------------------------- cluster statistics */

/*
 * These take a finished labeling (labels[i] = minimum site id of i's
 * cluster, as every ccl_label* call returns); on anything else the results
 * are undefined, but no access leaves the buffers (labels outside [0, N) are
 * skipped).  Asynchronous on `stream`; off the labeling path.  They
 * serve the percolation application of section 4.
 */

/* Workspace bytes ccl_cluster_ids needs (4 per 4096 sites, at least 4). */
size_t ccl_cluster_ids_workspace_size(int64_t n_sites);

/*
 * Sequential cluster ids, the renumbering the paper mentions at the end of
 * section 3: the cluster whose minimum site is the k-th smallest cluster
 * minimum gets id k.
 *   ids_out         device int32[N]: ids_out[i] = id of i's cluster
 *   n_clusters_out  device int32: the number of clusters
 *   workspace       device buffer of ccl_cluster_ids_workspace_size(N)
 *                   bytes, 4-byte aligned, contents need not be initialised
 * No buffer may overlap another.
 */
ccl_status ccl_cluster_ids(int64_t n_sites, const int32_t* labels, int32_t* ids_out,
                           int32_t* n_clusters_out, void* workspace, size_t workspace_bytes,
                           void* stream);

/*
 * ccl_cluster_ids without a workspace argument and without any device
 * allocation, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * workspace lives in a fixed device array of the library, 2 MiB per device,
 * allocated when the library's code is loaded on that device and held until
 * the process ends; it covers every n_sites up to
 * ccl_cluster_ids_noalloc_max_sites() (INT32_MAX).  Larger n_sites:
 * CCL_ERR_TOO_LARGE.  Nothing needs clearing between calls, but calls that
 * overlap on one device share that array and race: serialize them (one
 * stream, or events).  Kernel timing (ccl_trace_*) skips these launches.
 * Arguments, results and other errors are ccl_cluster_ids's.
 */
size_t ccl_cluster_ids_noalloc_max_sites(void);
ccl_status ccl_cluster_ids_noalloc(int64_t n_sites, const int32_t* labels, int32_t* ids_out,
                                   int32_t* n_clusters_out, void* stream);

/*
 * Cluster sizes indexed by the cluster's minimum site: sizes_out[r] is the
 * number of sites labelled r (zero where r is not a cluster minimum).
 *   sizes_out  device int32[N], overwritten
 */
ccl_status ccl_cluster_sizes(int64_t n_sites, const int32_t* labels, int32_t* sizes_out,
                             void* stream);

/*
 * The cluster-size distribution n_s of the percolation application (section
 * 4): hist_out[s] = number of clusters of exactly s sites for 1 <= s <
 * n_bins - 1, hist_out[n_bins - 1] = number of clusters of n_bins - 1 sites
 * or more, hist_out[0] = 0.
 *   sizes      device int32[N]: cluster sizes at the cluster minima, zero
 *              elsewhere, as ccl_cluster_sizes writes them (entries <= 0 are
 *              skipped)
 *   n_bins     >= 2
 *   hist_out   device int64[n_bins], 8-byte aligned, overwritten
 * sum_s s * hist_out[s] = N when every bin is below n_bins - 1.
 */
ccl_status ccl_cluster_size_histogram(int64_t n_sites, const int32_t* sizes, int64_t n_bins,
                                      int64_t* hist_out, void* stream);

/*
 * The spanning test of section 4: *result_out = 1 when one cluster holds a
 * site of sites_a and a site of sites_b (e.g. the first and the last row of a
 * lattice), else 0.
 *   sites_a, sites_b  device int32[n_a], int32[n_b], ids in [0, N) (others
 *                     are skipped)
 *   flags             device uint8[N] workspace, contents need not be
 *                     initialised
 *   result_out        device int32
 */
ccl_status ccl_spans(int64_t n_sites, const int32_t* labels, int64_t n_a, const int32_t* sites_a,
                     int64_t n_b, const int32_t* sites_b, uint8_t* flags, int32_t* result_out,
                     void* stream);

/* ---------------------------------------------------------------- checks */

/*
 * Count bonds with an end outside [0, n_sites).  Synchronous (waits on
 * `stream`); off the labeling path.  *n_bad_host receives the count; returns
 * CCL_ERR_INDEX_OUT_OF_RANGE when it is nonzero.
 */
ccl_status ccl_validate_edges(int64_t n_sites, int64_t n_bonds, const int32_t* src,
                              const int32_t* dst, int64_t* n_bad_host, void* stream);

/*
 * Count CSR defects: decreasing row_ptr steps, row_ptr[0] < 0, and column ids
 * outside [0, n_sites).  Synchronous, like ccl_validate_edges.
 */
ccl_status ccl_validate_csr(int64_t n_sites, const int32_t* row_ptr, const int32_t* col,
                            int64_t n_col, int64_t* n_bad_host, void* stream);

/* ---------------------------------------------------------------- utilities */

const char* ccl_status_string(ccl_status s);

/* HIP error code of the last failed HIP call on this host thread (0 = none). */
int ccl_last_hip_error(void);

/* Library version, e.g. 100 for 0.1.0. */
int ccl_version(void);

/*
 * Kernel timing.  While enabled, every kernel the library launches is
 * bracketed by HIP events recorded on the stream it is launched on.
 * ccl_trace_enable(1) also clears earlier records.  ccl_trace_count()
 * synchronizes on the recorded events and returns the number of records;
 * ccl_trace_get(i, ...) returns the kernel's name (static string) and its
 * duration in milliseconds.  At most 65536 records are kept.
 */
ccl_status ccl_trace_enable(int on);
int ccl_trace_count(void);
ccl_status ccl_trace_get(int i, const char** kernel_name, float* ms);

/*
 * Plain streaming copy of `bytes` bytes (16-byte aligned pointers), used to
 * calibrate hardware traffic counters against a kernel of known traffic.
 */
ccl_status ccl_probe_copy(const void* in, void* out, size_t bytes, void* stream);

/*
 * Random-access probes, the ceilings of the random graphs' labeling (bound by
 * scattered 4-byte accesses rather than by streaming bandwidth).  table:
 * device int32[table_len]; n_ops operations at hashed addresses spread over
 * the table, sixteen independent ones in flight per lane:
 *   mode 0: loads (gather);  1: device-scope atomicMin, result discarded;
 *   2: atomicMin with its result used;  3: dependent loads, each lane
 *   following table[x] chains (fill the table with mode 4 first);
 *   4: fill the table with hashed next-indices for mode 3.
 * sink: device int32 the kernel may write (keeps the loads live).  Time the
 * launch with ccl_trace_*; rate = n_ops / time.
 */
ccl_status ccl_probe_random(int32_t* table, int64_t table_len, int64_t n_ops, int32_t mode,
                            int32_t* sink, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CCL_H */
