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
constexpr int kRowsPerThread = 4;  // rows a thread handles per iteration
constexpr int kDegFast = 4;        // bonds per row kept in registers; more take a slow loop
static_assert((1 << kTileShift) == kCsrTile, "tile size");

// Raw buffer loads (gfx9 buffer resource, 32-bit offsets): an offset past
// the resource's byte size returns 0 instead of faulting, so every load of a
// batch can be issued unconditionally and the compiler keeps them in flight
// together instead of guarding each one with a branch and a wait.
constexpr uint32_t kBufWord3 = 0x00020000;
constexpr uint32_t kOffNone = 0xFFFFFFF0u;  // beyond any resource used here
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, (int)kBufWord3);
}
__device__ __forceinline__ int32_t buf_i32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0);
}
__device__ __forceinline__ uint32_t buf_u8(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, (int)byte_off, 0, 0);
}

// One workgroup per tile.  Each iteration covers kTileBlock * kRowsPerThread
// rows (row base + k * kTileBlock + tid for k < kRowsPerThread, so every load
// instruction is coalesced across the wave); the next iteration's row_ptr
// values are requested before this iteration's joins run, and the first
// kDegFast bonds of every row are requested in one batch of buffer loads, so
// a wave keeps dozens of loads in flight instead of waiting on each row.
// The buffer resources are based at the tile's first row and first bond, so
// offsets stay small whatever the graph size (a tile holding 2^30 or more
// bonds takes the plain-load loop instead).
template <bool HAS_OCC>
__global__ void __launch_bounds__(kTileBlock)
    k_csr_tile(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
               const uint8_t* __restrict__ occ, int32_t* __restrict__ label,
               uint64_t* __restrict__ rowmask) {
  __shared__ int32_t par[kCsrTile];
  const int64_t lo = (int64_t)blockIdx.x << kTileShift;
  const int32_t cnt = (int32_t)min((int64_t)kCsrTile, n - lo);
  const int tid = threadIdx.x, lane = tid & 63;
  constexpr int kRows = kTileBlock * kRowsPerThread;
  const int32_t e_begin = row_ptr[lo];
  const int32_t e_count = row_ptr[lo + cnt] - e_begin;
  const bool fast = e_count < (1 << 30);
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(row_ptr + lo, (uint32_t)(cnt + 1) * 4u);
  const __amdgpu_buffer_rsrc_t rc = make_rsrc(col + e_begin, fast ? (uint32_t)e_count * 4u : 0u);
  const __amdgpu_buffer_rsrc_t ro =
      make_rsrc(HAS_OCC ? occ + e_begin : nullptr, fast && HAS_OCC ? (uint32_t)e_count : 0u);

  // row t's bonds are [ra, rb) relative to e_begin; rows past the tile read
  // 0 (or the end value) and so hold no bonds
  int32_t ra[kRowsPerThread], rb[kRowsPerThread];
#pragma unroll
  for (int k = 0; k < kRowsPerThread; ++k) {
    const uint32_t t = (uint32_t)(k * kTileBlock + tid);
    ra[k] = buf_i32(rp, 4u * t) - e_begin;
    rb[k] = buf_i32(rp, 4u * (t + 1)) - e_begin;
  }
  for (int t = tid; t < kCsrTile; t += kTileBlock) par[t] = t;
  __syncthreads();

  for (int base = 0; base < cnt; base += kRows) {
    int32_t cv[kRowsPerThread][kDegFast];
    uint32_t ov[kRowsPerThread][kDegFast];
#pragma unroll
    for (int k = 0; k < kRowsPerThread; ++k)
#pragma unroll
      for (int j = 0; j < kDegFast; ++j) {
        const int32_t e = ra[k] + j;
        const uint32_t off = (fast && e < rb[k] && base + k * kTileBlock + tid < cnt)
                                 ? (uint32_t)e : kOffNone;
        cv[k][j] = buf_i32(rc, off * 4u);
        ov[k][j] = HAS_OCC ? buf_u8(ro, off) : (off != kOffNone ? 1u : 0u);
      }
    int32_t na[kRowsPerThread], nb[kRowsPerThread];
#pragma unroll
    for (int k = 0; k < kRowsPerThread; ++k) {
      const uint32_t t = (uint32_t)(base + kRows + k * kTileBlock + tid);
      na[k] = buf_i32(rp, 4u * t) - e_begin;
      nb[k] = buf_i32(rp, 4u * (t + 1)) - e_begin;
    }
#pragma unroll
    for (int k = 0; k < kRowsPerThread; ++k) {
      const int t = base + k * kTileBlock + tid;
      bool leaves = false;
      if (t < cnt) {
#pragma unroll
        for (int j = 0; j < kDegFast; ++j) {
          if (ov[k][j] == 0) continue;
          const int64_t v = (int64_t)cv[k][j] - lo;
          if (v >= 0 && v < cnt)
            lds_unite(par, t, (int32_t)v);
          else
            leaves = true;
        }
        for (int32_t e = ra[k] + (fast ? kDegFast : 0); e < rb[k]; ++e) {
          const int64_t ge = (int64_t)e_begin + e;
          if (HAS_OCC && occ[ge] == 0) continue;
          const int64_t v = (int64_t)col[ge] - lo;
          if (v >= 0 && v < cnt)
            lds_unite(par, t, (int32_t)v);
          else
            leaves = true;
        }
      }
      const uint64_t bits = __ballot(leaves);
      const int wave_first = base + k * kTileBlock + (tid & ~63);
      if (lane == 0 && wave_first < cnt && rowmask != nullptr)
        rowmask[(lo + wave_first) >> 6] = bits;
    }
#pragma unroll
    for (int k = 0; k < kRowsPerThread; ++k) {
      ra[k] = na[k];
      rb[k] = nb[k];
    }
  }
  __syncthreads();
  for (int t = tid; t < cnt; t += kTileBlock) label[lo + t] = (int32_t)(lo + lds_find(par, t));
}

// Cross kernel: the 64-row mask words are split into 8 contiguous ranges, one
// per XCD, so the tiles a range joins stay in one L2; inside a range the
// XCD's wavefronts take words round-robin.  Lane j of the wave owns row
// 64w + j and joins that row's occupied bonds leaving its tile.
__global__ void __launch_bounds__(256)
    k_csr_cross(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                const uint8_t* __restrict__ occ, int32_t* label,
                const uint64_t* __restrict__ rowmask, int64_t n_words) {
  const int lane = threadIdx.x & 63;
  const XcdSlot x = xcd_slot();
  const int64_t w_lo = n_words * x.xcd / kNumXcd;
  const int64_t w_hi = n_words * (x.xcd + 1) / kNumXcd;
  const int64_t waves = (int64_t)x.count * (256 / 64);
  const int64_t me = (int64_t)x.index * (256 / 64) + (threadIdx.x >> 6);
  for (int64_t w = w_lo + me; w < w_hi; w += waves) {
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
  uint64_t* mask = n_tiles == 1 ? nullptr : rowmask;
  if (occ != nullptr)
    CCL_LAUNCH("ccl_csr_tile", k_csr_tile<true>, (unsigned)n_tiles, kTileBlock, 0, s, n, row_ptr,
               col, occ, label, mask);
  else
    CCL_LAUNCH("ccl_csr_tile", k_csr_tile<false>, (unsigned)n_tiles, kTileBlock, 0, s, n, row_ptr,
               col, occ, label, mask);
  if (n_tiles == 1) return CCL_OK;  // no bond can leave the only tile
  const int64_t n_words = (n + 63) >> 6;
  // every XCD needs workgroups: each one owns a range of the mask words
  unsigned g = grid_for(n_words * 64, 256, 8, d);
  g = (g + kNumXcd - 1) / kNumXcd * kNumXcd;
  CCL_LAUNCH("ccl_csr_cross", k_csr_cross, g, 256, 0, s, n, row_ptr, col, occ, label, rowmask,
             n_words);
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
