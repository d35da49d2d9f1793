// lc_uf.h -- lock-free union-find of the library (device side): the same
// algorithm on parent words in HBM (uf_find / uf_union, 64-bit ids) and on
// an LDS forest (lfind / lunion, 32-bit local indices).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef LC_FLAG_GRAPH
#define LC_FLAG_GRAPH 256u  // a union-find word outside the graph (internal error)
#endif

namespace lc {

// Union-find, lock-free: roots are hooked to the smaller root with a CAS on
// the parent word (parent[x] <= x always, so no cycle can form; leaves never
// become roots again, which is what makes the finds safe without locks,
// Sec. 3.2).  Finds halve the path as they go.  The same algorithm runs on
// the LDS forest of a linking tile (lfind / lunion, 32-bit local indices)
// and on the parent words in HBM (uf_find / uf_union).
// Every word met on the way must be a node id below `n` (a finished loop's
// negative word or anything else is an inconsistent graph): the find then
// returns -1 and the union raises LC_FLAG_GRAPH instead of reading outside
// the parent words.
__device__ inline int64_t uf_find(int64_t* parent, int64_t x, int64_t n) {
  if (x < 0 || x >= n) return -1;
  int64_t p = parent[x];
  while (p != x) {
    if (p < 0 || p >= n) return -1;
    const int64_t gp = parent[p];
    if (gp != p && gp >= 0 && gp < n) parent[x] = gp;  // path halving; gp is an ancestor of x
    x = p;
    p = gp;
  }
  return x;
}

// uf_find of a and of b at once: the two walks advance one step at a time
// together, so that their reads of parent words are in flight at the same
// time (a union waits on the longer walk, not on the sum of the two).
__device__ inline void uf_find2(int64_t* parent, int64_t& a, int64_t& b, int64_t n) {
  const bool oka = a >= 0 && a < n, okb = b >= 0 && b < n;
  int64_t pa = oka ? parent[a] : -1, pb = okb ? parent[b] : -1;
  if (!oka) a = -1;
  if (!okb) b = -1;
  bool da = !oka || pa == a, db = !okb || pb == b;
  while (!da || !db) {
    if (!da && (pa < 0 || pa >= n)) {
      a = -1;
      da = true;
    }
    if (!db && (pb < 0 || pb >= n)) {
      b = -1;
      db = true;
    }
    const int64_t ga = da ? pa : parent[pa];
    const int64_t gb = db ? pb : parent[pb];
    if (!da) {
      if (ga != pa && ga >= 0 && ga < n) parent[a] = ga;  // path halving
      a = pa;
      pa = ga;
      da = pa == a;
    }
    if (!db) {
      if (gb != pb && gb >= 0 && gb < n) parent[b] = gb;
      b = pb;
      pb = gb;
      db = pb == b;
    }
  }
}

__device__ inline void uf_union(int64_t* parent, int64_t a, int64_t b, int64_t n, uint32_t* flags) {
  uf_find2(parent, a, b, n);
  while (a != b) {
    if (a < 0 || b < 0) {
      atomicOr(flags, LC_FLAG_GRAPH);
      return;
    }
    if (a < b) {
      const int64_t t = a;
      a = b;
      b = t;
    }
    // hook root a (larger) below b (smaller)
    const unsigned long long old =
        atomicCAS(reinterpret_cast<unsigned long long*>(parent + a), static_cast<unsigned long long>(a),
                  static_cast<unsigned long long>(b));
    if (static_cast<int64_t>(old) == a) return;
    a = static_cast<int64_t>(old);
    uf_find2(parent, a, b, n);
  }
}

// Words of the LDS forest change under other threads' unions and path
// halving: every read and write is a relaxed workgroup-scope atomic, so it
// is really performed (and stays an LDS instruction: a volatile pointer
// would lose the address space and go through flat memory instructions).
__device__ inline uint32_t lload(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lstore(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline uint32_t lfind(uint32_t* lp, uint32_t x) {
  uint32_t p = lload(lp + x);
  while (p != x) {
    const uint32_t gp = lload(lp + p);
    if (gp != p) lstore(lp + x, gp);
    x = p;
    p = gp;
  }
  return x;
}

__device__ inline void lunion(uint32_t* lp, uint32_t a, uint32_t b) {
  a = lfind(lp, a);
  b = lfind(lp, b);
  while (a != b) {
    if (a < b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    const uint32_t old = atomicCAS(lp + a, a, b);
    if (old == a) return;
    a = lfind(lp, old);
    b = lfind(lp, b);
  }
}

}  // namespace lc
