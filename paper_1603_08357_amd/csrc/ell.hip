// The paper's own schedule over its neighbour-list form (section 3): the
// list is padded to z_max entries per site and stored column-major, so
// neighbour k of site i is nn[k*N + i] and a wavefront reading neighbour k of
// 64 consecutive sites reads 256 contiguous bytes.  Four launches, in the
// paper's order:
//   (i)   label[i] = the lowest occupied neighbour numbered below i, or i
//         (that neighbour is thereby taken off i's residual list);
//   (ii)  analysis: every site follows its label to the root;
//   (iii) label reduction: site i runs Algorithm 1 with every neighbour left
//         on its residual list (occupied, numbered below i, not the one
//         step (i) took);
//   (iv)  analysis again.
// The residual lists are never stored: step (iii) reads site i's column of
// the list again and skips what step (i) consumed.  Steps (ii) and (iv) are
// the edge path's flatten (launch_flatten), which needs only label[x] <= x.
// An entry outside [0, N) is padding.
#include "common.hpp"
#include "uf.hpp"

namespace ccl {

constexpr int kEllBlock = 256;

// The lowest occupied neighbour of site i numbered below i, or i.
template <bool HAS_OCC>
__device__ __forceinline__ int32_t ell_lowest(int64_t n, int32_t z, const int32_t* __restrict__ nn,
                                              const uint8_t* __restrict__ occ, int64_t i) {
  int32_t m = (int32_t)i;
#pragma unroll 4
  for (int32_t k = 0; k < z; ++k) {
    const int64_t e = (int64_t)k * n + i;
    const int32_t j = nn[e];
    const bool on = !HAS_OCC || occ[e] != 0;
    if (on && j >= 0 && j < m) m = j;  // j < m <= i: below i, and entries >= N never pass
  }
  return m;
}

// Step (i).
template <bool HAS_OCC>
__global__ void __launch_bounds__(kEllBlock)
    k_ell_init(int64_t n, int32_t z, const int32_t* __restrict__ nn, const uint8_t* __restrict__ occ,
               int32_t* __restrict__ label) {
  const int64_t stride = (int64_t)gridDim.x * kEllBlock;
  for (int64_t i = (int64_t)blockIdx.x * kEllBlock + threadIdx.x; i < n; i += stride)
    st_dev(label + i, ell_lowest<HAS_OCC>(n, z, nn, occ, i));
}

// Step (iii): Algorithm 1 for site i and each neighbour left on its residual
// list.  A site whose list held at most one entry has nothing left.
template <bool HAS_OCC>
__global__ void __launch_bounds__(kEllBlock)
    k_ell_reduce(int64_t n, int32_t z, const int32_t* __restrict__ nn,
                 const uint8_t* __restrict__ occ, int32_t* label) {
  const int64_t stride = (int64_t)gridDim.x * kEllBlock;
  for (int64_t i = (int64_t)blockIdx.x * kEllBlock + threadIdx.x; i < n; i += stride) {
    const int32_t taken = ell_lowest<HAS_OCC>(n, z, nn, occ, i);
    if (taken == (int32_t)i) continue;  // the residual list was empty
    bool skipped = false;
    for (int32_t k = 0; k < z; ++k) {
      const int64_t e = (int64_t)k * n + i;
      const int32_t j = nn[e];
      if ((HAS_OCC && occ[e] == 0) || j < 0 || j >= (int32_t)i) continue;
      if (j == taken && !skipped) {  // consumed by step (i)
        skipped = true;
        continue;
      }
      unite(label, (int32_t)i, j);
    }
  }
}

ccl_status launch_label_ell(int64_t n, int32_t z, const int32_t* nn, const uint8_t* occ,
                            int32_t* label, hipStream_t s, const DeviceInfo& d) {
  const unsigned g = grid_for(n, kEllBlock, 8, d);
  if (occ != nullptr)
    CCL_LAUNCH("ccl_ell_init", k_ell_init<true>, g, kEllBlock, 0, s, n, z, nn, occ, label);
  else
    CCL_LAUNCH("ccl_ell_init", k_ell_init<false>, g, kEllBlock, 0, s, n, z, nn, occ, label);
  ccl_status st = launch_flatten(n, label, s, d);  // step (ii)
  if (st != CCL_OK) return st;
  if (occ != nullptr)
    CCL_LAUNCH("ccl_ell_reduce", k_ell_reduce<true>, g, kEllBlock, 0, s, n, z, nn, occ, label);
  else
    CCL_LAUNCH("ccl_ell_reduce", k_ell_reduce<false>, g, kEllBlock, 0, s, n, z, nn, occ, label);
  return launch_flatten(n, label, s, d);  // step (iv)
}

}  // namespace ccl
