// lc_device.h -- device-side building blocks of the loop-cluster library
// (gfx950, wave64).  Counter-based random numbers, chain descriptors and
// small integer helpers shared by the kernels of this library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lc {

// Counter domains: the top 8 bits of counter word 1 name what a draw is for.
enum : uint32_t { DOM_INIT = 0u, DOM_INS = 1u, DOM_FLIP = 2u, DOM_SYM = 3u, DOM_VOTE = 4u };

constexpr int kMaxTable = 64;  // longest Poisson threshold table

// Parent word of every node of a loop finished inside its linking tile: a
// code below all other words that holds the loop's smallest node (its
// label) and the loop's flip decision, kClosedRoot + 2 rep + bit.  Other
// loops' nodes hold a node id (>= 0) or, at their root, the loop code
// -1 - index (>= -2^62).
constexpr int64_t kClosedRoot = INT64_MIN;
__host__ __device__ inline int64_t closed_word(int64_t rep, uint32_t bit) {
  return static_cast<int64_t>((static_cast<uint64_t>(rep) << 1) + bit + (uint64_t(1) << 63));
}
__host__ __device__ inline bool is_closed_word(int64_t w) {
  return w < kClosedRoot + (int64_t(1) << 62);
}
__host__ __device__ inline int64_t closed_rep(int64_t w) {
  return static_cast<int64_t>((static_cast<uint64_t>(w) - (uint64_t(1) << 63)) >> 1);
}
__host__ __device__ inline uint32_t closed_bit(int64_t w) {
  return static_cast<uint32_t>(static_cast<uint64_t>(w) & 1u);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products; the key advances by the Weyl increments between rounds.
struct u32x4 {
  uint32_t x, y, z, w;
};

__host__ __device__ inline u32x4 philox10(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2,
                                          uint32_t c3) {
  uint32_t k0 = static_cast<uint32_t>(key), k1 = static_cast<uint32_t>(key >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t a = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t b = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t n0 = static_cast<uint32_t>(b >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(a >> 32) ^ c3 ^ k1;
    c1 = static_cast<uint32_t>(b);
    c3 = static_cast<uint32_t>(a);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

__host__ __device__ inline uint64_t lo64(const u32x4& r) {
  return static_cast<uint64_t>(r.x) | (static_cast<uint64_t>(r.y) << 32);
}
__host__ __device__ inline uint64_t hi64(const u32x4& r) {
  return static_cast<uint64_t>(r.z) | (static_cast<uint64_t>(r.w) << 32);
}

// Description of one chain, resident in device memory.  The chain's world
// lines live in its own double-buffered arrays; `cur` selects the buffer that
// holds the current configuration and flips after every completed sweep.
struct ChainDesc {
  uint64_t seed;
  int64_t L;           // spins
  int64_t n_sites;     // subspins (2S L)
  int64_t n_bonds;     // sub-bonds ((2S)^2 L)
  int64_t nbn;         // boundary nodes: n_sites (S=1/2) or 2 n_sites
  int64_t win_base;    // first flat (bond, window) index in the engine
  int64_t site_base;   // first flat subspin index in the engine
  int64_t spin_base;   // first flat spin index in the engine
  int64_t bnode_base;  // boundary nodes of all earlier chains in the engine
  int64_t kept_cap;    // capacity of each ktime buffer
  uint8_t* s0[2];      // spins at tau = 0+, n_sites
  int64_t* kstart[2];  // kept operators per window, exclusive scan, nwin + 1
  uint64_t* ktime[2];  // kept operator times, (bond, time) order
  int64_t* perm;       // symmetrization permutation of the last sweep
  int32_t two_s;
  int32_t w;           // 2^w windows per bond
  int32_t K;           // threshold table length
  uint32_t sweep;      // sweep being run (advanced on the device)
  int32_t cur;         // which of the two state buffers is current
  int32_t tile_j;      // linking tile: spins per tile
  int32_t tile_k;      //               windows per tile
  int32_t flip_rule;   // 0: bit of the loop's label, 1: XOR of its nodes' votes
  int64_t ntj;         // tiles along the chain, ceil(L / tile_j)
  uint64_t T[kMaxTable];
};

// Per-chain quantities that change every sweep (written on the device).
struct ChainDyn {
  int64_t op_base;    // first flat operator of the chain
  int64_t n_ops;
  int64_t node_base;  // first flat loop-graph node of the chain
  int64_t n_nodes;
};

// Per-chain statistics of the sweep just run (exact integers).
enum StatIdx : int {
  ST_CAND = 0,
  ST_ACC,
  ST_OPS,
  ST_KEPT_IN,
  ST_KEPT_OUT,
  ST_NODES,
  ST_CLUSTERS,
  ST_M2,
  ST_N0SQ,
  ST_SIZE2_LO,
  ST_SIZE2_HI,
  ST_LEN2_LO,
  ST_LEN2_HI,
  ST_MAFTER,
  ST_MAXSIZE,
  ST_PAD,
  ST_WORDS  // 16 words per chain
};

// 128-bit unsigned helpers (lo, hi) kept explicit.
struct u128p {
  uint64_t lo, hi;
};
__device__ inline u128p mul64x64(uint64_t a, uint64_t b) {
  return {a * b, __umul64hi(a, b)};
}
__device__ inline void atomic_add_u128(unsigned long long* lo, unsigned long long* hi, uint64_t xlo,
                                       uint64_t xhi) {
  const unsigned long long old = atomicAdd(lo, static_cast<unsigned long long>(xlo));
  const uint64_t carry = (old + xlo < old) ? 1u : 0u;
  const uint64_t h = xhi + carry;
  if (h) atomicAdd(hi, static_cast<unsigned long long>(h));
}

// Chain owning a flat index, given sorted chain start offsets base[0..n).
__device__ inline int chain_of(const int64_t* __restrict__ base, int n, int64_t i) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

}  // namespace lc
