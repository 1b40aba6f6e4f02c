// CSR labeling with tile-local joins in LDS.
//
// Sites are cut into tiles of kCsrTile consecutive ids; a tile owns its sites
// and the bonds stored in its rows.  Three kernels:
//   1. tile kernel, one workgroup per tile: step (i) for the tile in LDS
//      (par[t] = t), step (iii) -- Algorithm 1 on LDS with ds_min -- for every
//      occupied bond whose two ends lie in the tile, a root chase in LDS, and
//      one coalesced store of the tile's labels (each site's tile-local root,
//      the tile's minimum member of its local cluster).  Rows holding an
//      occupied bond that leaves the tile are flagged in a bit mask;
//   2. cross kernel: step (iii) in global memory (Algorithm 1 with
//      device-scope atomicMin) for the occupied leaving bonds of flagged rows;
//   3. flatten: step (iv).
// Every value the tile kernel stores is a member of the site's cluster no
// larger than the site, so kernels 2-3 see a valid forest and finish the job
// exactly as the single-pass method would.
#include "common.hpp"
#include "uf.hpp"

namespace ccl {

constexpr int kTileBlock = 1024;
constexpr int kTileShift = 15;
static_assert((1 << kTileShift) == kCsrTile, "tile size");

__global__ void __launch_bounds__(kTileBlock)
    k_csr_tile(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
               const uint8_t* __restrict__ occ, int32_t* __restrict__ label,
               uint64_t* __restrict__ rowmask) {
  __shared__ int32_t par[kCsrTile];
  const int64_t lo = (int64_t)blockIdx.x << kTileShift;
  const int32_t cnt = (int32_t)min((int64_t)kCsrTile, n - lo);
  for (int t = threadIdx.x; t < kCsrTile; t += kTileBlock) par[t] = t;
  __syncthreads();

  const int lane = threadIdx.x & 63;
  for (int base = 0; base < cnt; base += kTileBlock) {
    const int t = base + threadIdx.x;
    bool leaves = false;
    if (t < cnt) {
      const int64_t r = lo + t;
      const int32_t e1 = row_ptr[r + 1];
      for (int32_t e = row_ptr[r]; e < e1; ++e) {
        if (occ != nullptr && occ[e] == 0) continue;
        const int64_t v = (int64_t)col[e] - lo;
        if (v >= 0 && v < cnt)
          lds_unite(par, t, (int32_t)v);
        else
          leaves = true;
      }
    }
    const uint64_t bits = __ballot(leaves);
    const int wave_first = base + (threadIdx.x & ~63);
    if (lane == 0 && wave_first < cnt && rowmask != nullptr) rowmask[(lo + wave_first) >> 6] = bits;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < cnt; t += kTileBlock)
    label[lo + t] = (int32_t)(lo + lds_find(par, t));
}

// One wavefront per 64-row mask word; lane j owns row 64w + j.
__global__ void __launch_bounds__(256)
    k_csr_cross(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                const uint8_t* __restrict__ occ, int32_t* label,
                const uint64_t* __restrict__ rowmask, int64_t n_words) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t w = wave; w < n_words; w += n_waves) {
    const uint64_t bits = rowmask[w];
    if (((bits >> lane) & 1ull) == 0) continue;
    const int64_t r = (w << 6) + lane;
    const int64_t tlo = (r >> kTileShift) << kTileShift;
    const int64_t thi = min(tlo + kCsrTile, n);
    const int32_t e1 = row_ptr[r + 1];
    for (int32_t e = row_ptr[r]; e < e1; ++e) {
      if (occ != nullptr && occ[e] == 0) continue;
      const int32_t v = col[e];
      if (v < tlo || v >= thi) unite(label, (int32_t)r, v);
    }
  }
}

ccl_status launch_label_csr(int64_t n, const int32_t* row_ptr, const int32_t* col,
                            const uint8_t* occ, int32_t* label, uint64_t* rowmask,
                            hipStream_t s, const DeviceInfo& d) {
  if (n == 0) return CCL_OK;
  const int64_t n_tiles = (n + kCsrTile - 1) / kCsrTile;
  // a single tile has no leaving bonds to record: the mask is not touched
  CCL_LAUNCH("ccl_csr_tile", k_csr_tile, (unsigned)n_tiles, kTileBlock, 0, s, n, row_ptr, col, occ,
             label, n_tiles == 1 ? nullptr : rowmask);
  if (n_tiles == 1) return CCL_OK;  // no bond can leave the only tile
  const int64_t n_words = (n + 63) >> 6;
  CCL_LAUNCH("ccl_csr_cross", k_csr_cross, grid_for(n_words * 64, 256, 8, d), 256, 0, s, n,
             row_ptr, col, occ, label, rowmask, n_words);
  return launch_flatten(n, label, s, d);
}

// ---------------------------------------------------------------- checks

__global__ void __launch_bounds__(256)
    k_validate_csr(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                   int64_t n_col, unsigned long long* count) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  unsigned long long bad = 0;
  for (int64_t i = tid; i < n; i += stride) {
    const int32_t a = row_ptr[i], b = row_ptr[i + 1];
    bad += (b < a) ? 1ull : 0ull;
    bad += (i == 0 && a < 0) ? 1ull : 0ull;
    bad += (i == n - 1 && (int64_t)b > n_col) ? 1ull : 0ull;
  }
  for (int64_t e = tid; e < n_col; e += stride) {
    const int32_t v = col[e];
    bad += (v < 0 || (int64_t)v >= n) ? 1ull : 0ull;
  }
  if (bad) atomicAdd(count, bad);
}

ccl_status launch_validate_csr(int64_t n, const int32_t* row_ptr, const int32_t* col,
                               int64_t n_col, unsigned long long* d_count, hipStream_t s,
                               const DeviceInfo& d) {
  const int64_t work = n > n_col ? n : n_col;
  if (work == 0) return CCL_OK;
  CCL_LAUNCH("ccl_validate_csr", k_validate_csr, grid_for(work, 256, 8, d), 256, 0, s, n, row_ptr,
             col, n_col, d_count);
  return CCL_OK;
}

}  // namespace ccl
