// Device-side union-find primitives of the labeling (paper, sections 2-3).
//
// The label array is the union-find forest: label[x] <= x always, and
// label[x] == x marks a root.  Two facts make the lock-free scheme correct
// under any interleaving of threads:
//   * every write to label[x] stores a member of x's cluster that is smaller
//     than the value it replaces or equal to an ancestor of it, so a stale
//     read is still a valid (older) link and root chases always terminate
//     (indices strictly decrease along a chain);
//   * the atomicMin loop of Algorithm 1 re-joins every link it displaces.
// Hence plain (possibly stale, cached) loads are used for root chases and
// only the atomicMin has to be coherent across the chip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mem.hpp"

namespace ccl {

// ---------------------------------------------------------------- global

// Ordinary cached global load of a label.  A wavefront-scope relaxed atomic
// load compiles to a plain global_load on gfx950; using it keeps the compiler
// from caching a value across iterations of a chase.
__device__ __forceinline__ int32_t lab_ld(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
// A label store: device scope (see mem.hpp), so no later kernel's write of
// the same word can be overtaken by it.
__device__ __forceinline__ void lab_st(int32_t* p, int32_t v) { st_dev(p, v); }

// Device-coherent atomicMin returning the previous value.
__device__ __forceinline__ int32_t lab_min(int32_t* p, int32_t v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The compression store of the merge step (path halving): label[x] lowered
// to an ancestor, as a device-coherent atomicMin whose result is unused.
// It can never raise a label, so however late it lands -- even after a
// later kernel wrote x's final root, which is at most the ancestor -- it
// leaves a correct value.  A plain store can land that late: under
// concurrent kernels on other streams, a merge-step compression store was
// seen to overwrite a final root written by the following flatten kernel
// (about one request in 4000 of a serving run on MI355X had one wrong
// label; with this form none in 20000).
__device__ __forceinline__ void lab_lower(int32_t* p, int32_t v) {
  __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The analysis chase (sections 2-3): follow label until label[r] == r.
__device__ __forceinline__ int32_t find_root(const int32_t* label, int32_t x) {
  int32_t p = lab_ld(label + x);
  while (p != x) {
    x = p;
    p = lab_ld(label + x);
  }
  return x;
}

// The chase with path halving: every visited site is re-pointed at its
// grandparent (a smaller member of the same cluster), so chains that many
// concurrent joins stacked up shrink as threads walk them.  The store is an
// atomicMin (lab_lower), so it never undoes a lower link another thread made.
// For the merge step only: the flatten step stores nothing but final roots.
// This form starts from a first parent p = label[x] already loaded (lets a
// caller issue the first loads of several chases together).
// The compression atomic is issued after the load of the next link: one
// counter tracks both on gfx950, so a wait for a load also waits for every
// memory operation issued before it, and an atomic issued first would put
// its round trip on the chase's critical path.
__device__ __forceinline__ int32_t find_root_halving_from(int32_t* label, int32_t x, int32_t p) {
  while (p != x) {
    const int32_t g = lab_ld(label + p);
    if (g == p) return p;
    const int32_t pg = lab_ld(label + g);
    lab_lower(label + x, g);
    x = g;
    p = pg;
  }
  return x;
}

__device__ __forceinline__ int32_t find_root_halving(int32_t* label, int32_t x) {
  return find_root_halving_from(label, x, lab_ld(label + x));
}

// Join roots r1, r2 (any members work; roots save atomics): the label
// reduction loop of Algorithm 1.  Order so that r1 > r2, then
// old = atomicMin(label[r1], r2):
//   old == r2  : the link already existed                         -> done
//   old == r1  : r1 was a root and now points at r2               -> done
//                (one atomic earlier than the printed loop, which would
//                 repeat the atomicMin and read back r2)
//   otherwise  : r1's previous link `old` was replaced; old and r2
//                must now be joined -- continue with the pair (old, r2).
// max(r1, r2) strictly decreases each round, so the loop terminates.
__device__ __forceinline__ void join_roots(int32_t* label, int32_t r1, int32_t r2) {
  while (r1 != r2) {
    if (r1 < r2) {
      int32_t t = r1;
      r1 = r2;
      r2 = t;
    }
    int32_t old = lab_min(label + r1, r2);
    if (old == r2 || old == r1) break;
    r1 = old;
  }
}

// Step (iii) for one bond (a, b): roots of both ends, then Algorithm 1.
// Bonds whose ends already share a root issue no atomic.
__device__ __forceinline__ void unite(int32_t* label, int32_t a, int32_t b) {
  int32_t r1 = find_root_halving(label, a);
  int32_t r2 = find_root_halving(label, b);
  if (r1 != r2) join_roots(label, r1, r2);
}

// Checked variants (used where a publication error must not turn into a
// hang): a label that points upward or below zero, or an atomicMin returning
// such a value, cannot occur in a valid forest; it sets `bad` and stops.
__device__ __forceinline__ int32_t find_root_halving_checked(int32_t* label, int32_t x, int32_t p,
                                                             bool& bad) {
  while (p != x) {
    if (p > x || p < 0) {
      bad = true;
      return x;
    }
    const int32_t g = lab_ld(label + p);
    if (g == p) return p;
    if (g > p || g < 0) {
      bad = true;
      return x;
    }
    const int32_t pg = lab_ld(label + g);  // before the atomic, as above
    lab_lower(label + x, g);
    x = g;
    p = pg;
  }
  return x;
}

__device__ __forceinline__ void join_roots_checked(int32_t* label, int32_t r1, int32_t r2, bool& bad) {
  while (!bad && r1 != r2) {
    if (r1 < r2) {
      const int32_t t = r1;
      r1 = r2;
      r2 = t;
    }
    const int32_t old = lab_min(label + r1, r2);
    if (old == r2 || old == r1) break;
    if (old > r1 || old < 0) {
      bad = true;
      break;
    }
    r1 = old;
  }
}

// Step (iii) for P bonds at once, in lockstep: the first parents of all 2P
// ends are requested together, each of `rounds` chase rounds advances every
// chase by one link (a finished chase re-reads its root, a cache hit, so the
// rounds stay free of branches and their loads stay in flight together),
// longer chases finish with path halving, and the first atomicMin of every
// join is issued back to back; a join whose atomicMin displaced a link ends
// with the sequential loop.  This is only another interleaving of Algorithm
// 1, which is correct under any interleaving.  A bond with a[k] == b[k] is a
// no-op (callers map unoccupied or padding bonds to (x, x) with x a valid
// site).  CHECKED: labels that point upward or below zero (impossible in a
// valid forest) set `bad` and stop that chase instead of following it.
template <int P, int ROUNDS, bool CHECKED>
__device__ __forceinline__ void unite_lockstep(int32_t* label, int32_t (&a)[P], int32_t (&b)[P],
                                               bool& bad) {
  int32_t pa[P], pb[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    pa[k] = lab_ld(label + a[k]);
    pb[k] = lab_ld(label + b[k]);
  }
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      if (CHECKED) {
        if (pa[k] > a[k] || pa[k] < 0) { bad = true; pa[k] = a[k]; }
        if (pb[k] > b[k] || pb[k] < 0) { bad = true; pb[k] = b[k]; }
      }
      a[k] = pa[k];
      b[k] = pb[k];
      pa[k] = lab_ld(label + a[k]);
      pb[k] = lab_ld(label + b[k]);
    }
  }
  int32_t hi[P], lo[P], old[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    if (CHECKED) {
      if (pa[k] > a[k] || pa[k] < 0) { bad = true; pa[k] = a[k]; }
      if (pb[k] > b[k] || pb[k] < 0) { bad = true; pb[k] = b[k]; }
    }
    if (CHECKED) {
      if (pa[k] != a[k]) a[k] = find_root_halving_checked(label, a[k], pa[k], bad);
      if (pb[k] != b[k]) b[k] = find_root_halving_checked(label, b[k], pb[k], bad);
    } else {
      if (pa[k] != a[k]) a[k] = find_root_halving_from(label, a[k], pa[k]);
      if (pb[k] != b[k]) b[k] = find_root_halving_from(label, b[k], pb[k]);
    }
    hi[k] = max(a[k], b[k]);
    lo[k] = min(a[k], b[k]);
  }
  if (CHECKED && bad) return;
#pragma unroll
  for (int k = 0; k < P; ++k) old[k] = hi[k] != lo[k] ? lab_min(label + hi[k], lo[k]) : lo[k];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    if (old[k] == lo[k] || old[k] == hi[k]) continue;
    if (CHECKED)
      join_roots_checked(label, old[k], lo[k], bad);
    else
      join_roots(label, old[k], lo[k]);
  }
}

// ---------------------------------------------------------------- LDS

__device__ __forceinline__ int32_t lds_ld(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// ---------------------------------------------------------------- LDS, 16-bit

// A tile of up to 65536 sites keeps its parent array as 16-bit tile-relative
// ids (128 KB of LDS).  Loads and path-halving stores are 16-bit LDS accesses;
// LDS has no 16-bit atomic min: lds16_min is a compare-and-swap loop on the
// 32-bit word holding the entry (the neighbouring entry's concurrent 16-bit
// stores just make the swap retry), and the lockstep union links with a
// masked-or on the entry's half of the word instead.

__device__ __forceinline__ int32_t lds16_ld(const uint16_t* p) {
  return (int32_t)__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds16_st(uint16_t* p, int32_t v) {
  __hip_atomic_store(p, (uint16_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}


// Masked-or on 32-bit LDS words at byte offsets off[k] (LDS offsets are the
// low 32 bits of a generic pointer to shared memory): the bits of mask[k]
// take the values of bits[k], atomically, and the old words come back.  The
// P operations are issued back to back and completed by one wait inside the
// same asm statement, so every result is tied to its own wait (the compiler
// does not count inline LDS operations).  P is 1, 2 or 4.
template <int P>
__device__ __forceinline__ void lds_mskor(uint32_t (&ret)[P], const uint32_t (&off)[P],
                                          const uint32_t (&mask)[P], const uint32_t (&bits)[P]) {
  static_assert(P == 1 || P == 2 || P == 4, "lds_mskor takes 1, 2 or 4 operations");
  if constexpr (P == 1) {
    asm volatile(
        "ds_mskor_rtn_b32 %0, %1, %2, %3\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(ret[0])
        : "v"(off[0]), "v"(mask[0]), "v"(bits[0])
        : "memory");
  } else if constexpr (P == 2) {
    asm volatile(
        "ds_mskor_rtn_b32 %0, %2, %4, %6\n\t"
        "ds_mskor_rtn_b32 %1, %3, %5, %7\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(ret[0]), "=&v"(ret[1])
        : "v"(off[0]), "v"(off[1]), "v"(mask[0]), "v"(mask[1]), "v"(bits[0]), "v"(bits[1])
        : "memory");
  } else {
    asm volatile(
        "ds_mskor_rtn_b32 %0, %4, %8, %12\n\t"
        "ds_mskor_rtn_b32 %1, %5, %9, %13\n\t"
        "ds_mskor_rtn_b32 %2, %6, %10, %14\n\t"
        "ds_mskor_rtn_b32 %3, %7, %11, %15\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(ret[0]), "=&v"(ret[1]), "=&v"(ret[2]), "=&v"(ret[3])
        : "v"(off[0]), "v"(off[1]), "v"(off[2]), "v"(off[3]), "v"(mask[0]), "v"(mask[1]),
          "v"(mask[2]), "v"(mask[3]), "v"(bits[0]), "v"(bits[1]), "v"(bits[2]), "v"(bits[3])
        : "memory");
  }
}

// atomicMin of entry x with v; returns the previous value of the entry
__device__ __forceinline__ int32_t lds16_min(uint16_t* par, int32_t x, int32_t v) {
  uint32_t* w = reinterpret_cast<uint32_t*>(par) + (x >> 1);
  const uint32_t sh = (uint32_t)(x & 1) * 16u;
  uint32_t cur = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  for (;;) {
    const uint32_t old = (cur >> sh) & 0xFFFFu;
    if ((int32_t)old <= v) return (int32_t)old;
    const uint32_t next = (cur & ~(0xFFFFu << sh)) | ((uint32_t)v << sh);
    uint32_t seen = cur;
    if (__hip_atomic_compare_exchange_strong(w, &seen, next, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP))
      return (int32_t)old;
    cur = seen;
  }
}

// Root chase with path halving, given p = par[x] already loaded.
__device__ __forceinline__ int32_t lds16_find_from(uint16_t* par, int32_t x, int32_t p) {
  while (p != x) {
    const int32_t g = lds16_ld(par + p);
    if (g == p) return p;
    lds16_st(par + x, g);
    x = g;
    p = lds16_ld(par + x);
  }
  return x;
}

__device__ __forceinline__ int32_t lds16_find(uint16_t* par, int32_t x) {
  int32_t p = lds16_ld(par + x);
  while (p != x) {
    const int32_t g = lds16_ld(par + p);
    if (g == p) return p;
    lds16_st(par + x, g);
    x = g;
    p = lds16_ld(par + x);
  }
  return x;
}

__device__ __forceinline__ void lds16_unite(uint16_t* par, int32_t a, int32_t b) {
  int32_t r1 = lds16_find(par, a);
  int32_t r2 = lds16_find(par, b);
  while (r1 != r2) {
    if (r1 < r2) {
      const int32_t t = r1;
      r1 = r2;
      r2 = t;
    }
    const int32_t old = lds16_min(par, r1, r2);
    if (old == r2 || old == r1) break;
    r1 = old;
  }
}

// Step (iii) in LDS for P bonds of a lane at once (tile-relative ends; a
// bond with a[k] == b[k] does nothing): the first parent loads of all 2P ends
// are issued together, then ROUNDS pointer-following rounds in which every
// end steps (a root steps onto itself), then the rare longer chases one by
// one.  The link of Algorithm 1 is then made for all P bonds together, one
// round per LDS round trip: the higher root's 16-bit half of its word is
// overwritten with the lower root by a masked-or (one atomic, no word load,
// no compare-and-swap to lose against the neighbouring entry), and the old
// parent comes back.  Old == higher root: it was a root, done.  Old == lower
// root: already linked, done.  Otherwise the higher root had been linked to
// `old` meanwhile; that link has just been replaced, so the join loop goes on
// with (old, lower root), as Algorithm 1 does after an atomicMin that did not
// find a root.  Every overwritten link is thus rejoined by the lane that
// overwrote it, a parent always stays below its child, and the larger end of
// the pair strictly decreases each round, so the loop ends; the final
// forest, hence each tile component's root (its smallest site), is the one
// the atomicMin form gives.
template <int P, int ROUNDS>
__device__ __forceinline__ void lds16_unite_lockstep(uint16_t* par, int32_t (&a)[P], int32_t (&b)[P]) {
  int32_t pa[P], pb[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    pa[k] = lds16_ld(par + a[k]);
    pb[k] = lds16_ld(par + b[k]);
  }
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      a[k] = pa[k];
      b[k] = pb[k];
      pa[k] = lds16_ld(par + a[k]);
      pb[k] = lds16_ld(par + b[k]);
    }
  }
  int32_t hi[P], lo[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    if (pa[k] != a[k]) a[k] = lds16_find_from(par, a[k], pa[k]);
    if (pb[k] != b[k]) b[k] = lds16_find_from(par, b[k], pb[k]);
    hi[k] = max(a[k], b[k]);
    lo[k] = min(a[k], b[k]);
  }
  const uint32_t base = (uint32_t)reinterpret_cast<uintptr_t>(par);  // LDS offset
  bool go[P];
#pragma unroll
  for (int k = 0; k < P; ++k) go[k] = hi[k] != lo[k];
  for (;;) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < P; ++k) any = any || go[k];
    if (!__any(any)) break;
    // a lane with nothing left issues an empty mask on its own word, so all
    // P operations of every lane are in flight together
    uint32_t ret[P], sh[P], off[P], msk[P], bits[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      sh[k] = (uint32_t)(hi[k] & 1) * 16u;
      off[k] = base + 4u * (uint32_t)(hi[k] >> 1);
      msk[k] = go[k] ? 0xFFFFu << sh[k] : 0u;
      bits[k] = go[k] ? (uint32_t)lo[k] << sh[k] : 0u;
    }
    lds_mskor<P>(ret, off, msk, bits);
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int32_t old = (int32_t)((ret[k] >> sh[k]) & 0xFFFFu);
      if (go[k] && (old == hi[k] || old == lo[k])) go[k] = false;
      if (go[k]) {
        hi[k] = max(old, lo[k]);
        lo[k] = min(old, lo[k]);
      }
    }
  }
}

}  // namespace ccl
