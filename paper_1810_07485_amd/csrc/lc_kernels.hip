// lc_kernels.hip -- HIP kernels (gfx950, wave64) of one continuous-time
// loop-cluster update of the antiferromagnetic Heisenberg chain
// (Todo, Matsuo, Shitara, arXiv:1810.07485, Sec. 2 and Sec. 3.2).
//
// Every kernel walks a flat index space that spans all resident chains
// (windows, operators, loop-graph nodes or sites) with a grid-stride loop,
// reading dynamic sizes from device memory, so one launch serves one chain
// or a batch and the whole sweep can be captured in a graph.
//
// Data layout (flat over chains, chain-contiguous):
//   window i = (chain, bond b, window k): b-major, 2^w windows per bond
//   kstart[i]  first kept off-diagonal operator of window i (exclusive scan)
//   ktime[]    kept operator times, (bond, time) order
//   opstart[i] first operator of window i; optime[], optype[] (bit 0: type
//   now, bit 1: type before the flip; 1 = off-diagonal)
//   node ids per chain: boundary nodes [0, nbn), then lower(q) = nbn + 2q,
//   upper(q) = nbn + 2q + 1 for operator q; flat id = node_base + local id.
#include "lc_kernels.h"

#include "lc_device.h"

namespace lc {

constexpr int kBlock = 256;
constexpr int kCap = 12;  // candidate times per window kept in LDS while writing; more are redrawn

// Parent word of the upper node of a closed two-node loop (see k_link_ops):
// below every root code -1 - index, so no kernel takes it for a loop index.
constexpr int64_t kPairRoot = INT64_MIN;

__device__ inline int lane_id() { return __lane_id(); }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Renumbering them so that every XCD takes a contiguous range of the
// work keeps neighbouring windows and nodes (the other bond of a site, the
// next operator of a loop) in one L2.  Identity unless the grid size is a
// multiple of 8.  Only the assignment of work changes, never a result.
__device__ inline int64_t xcd_block() {
  const int64_t p = blockIdx.x, G = gridDim.x;
  if (G & 7) return p;
  return (p & 7) * (G >> 3) + (p >> 3);
}

// Block-level flushes of per-thread statistics.  Every thread holds a
// chain c (-1: none) and a value for one statistics word of that chain; the
// values are summed over the wave with shuffles and over the block's waves
// through LDS, and one atomic per block and word reaches a striped copy of
// the counter when the whole block names one chain (per wave, or per lane,
// otherwise).  Blocks that finish together would otherwise queue thousands
// of atomics on the same few words; with kStripes copies (stripe = block
// mod kStripes, so one XCD per stripe) they spread, and k_stats_reduce folds
// the stripes into the statistics at the end of the sweep.  The stripes sit
// after the nchain * ST_WORDS statistics words.  Convergent: every thread of
// the block calls.
constexpr int kWaves = kBlock / 64;
constexpr int kStripes = LC_STAT_STRIPES;

enum FlushOp { FLUSH_ADD, FLUSH_MAX };

__device__ inline unsigned long long* stripe_word(unsigned long long* stats, int nchain, int c, int w) {
  return stats + static_cast<int64_t>(nchain) * ST_WORDS +
         (static_cast<int64_t>(c) * ST_WORDS + w) * kStripes + (blockIdx.x % kStripes);
}

// (lo, hi) += (xlo, xhi) as a 128-bit sum; hi < 0: a single 64-bit word;
// FLUSH_MAX: lo = max(lo, xlo).  Into this block's stripe.
__device__ inline void stat_apply(unsigned long long* stats, int nchain, int c, int ilo, int ihi,
                                  FlushOp op, uint64_t xlo, uint64_t xhi) {
  if (op == FLUSH_MAX) {
    if (xlo) atomicMax(stripe_word(stats, nchain, c, ilo), static_cast<unsigned long long>(xlo));
  } else if (ihi < 0) {
    if (xlo) atomicAdd(stripe_word(stats, nchain, c, ilo), static_cast<unsigned long long>(xlo));
  } else if (xlo | xhi) {
    atomic_add_u128(stripe_word(stats, nchain, c, ilo), stripe_word(stats, nchain, c, ihi), xlo, xhi);
  }
}

__device__ inline void stat_combine(FlushOp op, uint64_t& alo, uint64_t& ahi, uint64_t blo,
                                    uint64_t bhi) {
  if (op == FLUSH_MAX) {
    alo = blo > alo ? blo : alo;
  } else {
    const uint64_t s = alo + blo;
    ahi = ahi + bhi + (s < alo ? 1u : 0u);
    alo = s;
  }
}

__device__ inline void block_flush(unsigned long long* stats, int nchain, int c, int ilo, int ihi,
                                   FlushOp op, uint64_t xlo, uint64_t xhi) {
  __shared__ uint64_t slo[kWaves], shi[kWaves];
  __shared__ int sc[kWaves];
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  const int c0 = __shfl(c, 0);
  const bool uni = __all(c == c0);
  if (!uni) {  // the wave spans chains: per lane
    if (c >= 0) stat_apply(stats, nchain, c, ilo, ihi, op, xlo, xhi);
    xlo = xhi = 0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t ol = __shfl_xor(xlo, o), oh = __shfl_xor(xhi, o);
    stat_combine(op, xlo, xhi, ol, oh);
  }
  if (lane == 0) {
    slo[wv] = xlo;
    shi[wv] = xhi;
    sc[wv] = uni ? c0 : -1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bool same = sc[0] >= 0;
    for (int w = 1; w < kWaves; ++w) same = same && sc[w] == sc[0];
    if (same) {
      uint64_t tlo = slo[0], thi = shi[0];
      for (int w = 1; w < kWaves; ++w) stat_combine(op, tlo, thi, slo[w], shi[w]);
      stat_apply(stats, nchain, sc[0], ilo, ihi, op, tlo, thi);
    } else {
      for (int w = 0; w < kWaves; ++w)
        if (sc[w] >= 0) stat_apply(stats, nchain, sc[w], ilo, ihi, op, slo[w], shi[w]);
    }
  }
  __syncthreads();  // the LDS slots are reused by the next flush
}

// Per-thread partial sums of one chain's statistics.  A thread walks its
// items in increasing flat index, so it meets each chain in one stretch: the
// sums go to the chain's counters (striped copies) when the thread moves on
// to another chain (per lane; frequent in a batch of many small chains) and
// once at the end (block_flush).
template <int N>
struct Partial {
  int c;
  uint64_t v[N];
  __device__ Partial() : c(-1) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = 0;
  }
  __device__ void at(int cn, unsigned long long* stats, int nchain, const int (&idx)[N]) {
    if (cn == c) return;
    if (c >= 0) {
#pragma unroll
      for (int i = 0; i < N; ++i) stat_apply(stats, nchain, c, idx[i], -1, FLUSH_ADD, v[i], 0);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = 0;
    c = cn;
  }
  // convergent: every thread of the block must call it
  __device__ void flush(unsigned long long* stats, int nchain, const int (&idx)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) block_flush(stats, nchain, c, idx[i], -1, FLUSH_ADD, v[i], 0);
  }
};

// ---------------------------------------------------------------------------
// Bonds touching a subspin x = (j, a): the 2S "left" bonds from (j-1, a') and
// the 2S "right" bonds to (j+1, c).  For S=1/2 these are bonds j-1 and j.
__device__ inline int64_t bond_touching(const ChainDesc& D, int64_t x, int idx) {
  const int64_t ts = D.two_s;
  const int64_t j = x / ts, a = x - j * ts;
  if (idx < ts) {
    const int64_t jl = (j == 0) ? D.L - 1 : j - 1;
    return (jl * ts + idx) * ts + a;
  }
  return (j * ts + a) * ts + (idx - ts);
}
__device__ inline int64_t bond_x(const ChainDesc& D, int64_t b) { return b / D.two_s; }
__device__ inline int64_t bond_y(const ChainDesc& D, int64_t b) {
  const int64_t ts = D.two_s;
  const int64_t c = b % ts, x = b / ts, j = x / ts;
  const int64_t jn = (j + 1 == D.L) ? 0 : j + 1;
  return jn * ts + c;
}

// Event (t1, b1) strictly precedes (t2, b2) on the time axis: earlier time,
// or equal time and smaller bond index.
__device__ inline bool precedes(uint64_t t1, int64_t b1, uint64_t t2, int64_t b2) {
  return t1 < t2 || (t1 == t2 && b1 < b2);
}

// Are the spins of the two ends of bond b antiparallel just before (tc[j], b)?
// (labeling rules ii/iii: a horizontal graph only between antiparallel
// spins.)  The spins at 0+ are flipped by every kept off-diagonal operator
// that precedes (tc[j], b) in (time, bond) order on the other bonds touching
// either end; kept operators on b itself flip both ends and cancel.  Answered
// for m <= kChunk candidate times of one window (b, k) at once, as a bit
// mask: each neighbouring bond's window bounds and kept times are read once
// for all of them.
constexpr int kChunk = 8;
__device__ inline uint32_t antiparallel_mask(const ChainDesc& D, const uint8_t* __restrict__ s0,
                                             const int64_t* __restrict__ kstart,
                                             const uint64_t* __restrict__ ktime, int64_t b,
                                             uint64_t k, const uint64_t (&tc)[kChunk], int m) {
  const int64_t ends[2] = {bond_x(D, b), bond_y(D, b)};
  uint32_t base = static_cast<uint32_t>(s0[ends[0]] ^ s0[ends[1]]);
  uint32_t flips = 0;  // bit j: parity of in-window kept operators before tc[j]
  const int nt = 2 * D.two_s;
  for (int e = 0; e < 2; ++e) {
    for (int s = 0; s < nt; ++s) {
      const int64_t bb = bond_touching(D, ends[e], s);
      if (bb == b) continue;
      const int64_t i0 = bb << D.w;
      const int64_t ws = kstart[i0 + static_cast<int64_t>(k)];
      const int64_t we = kstart[i0 + static_cast<int64_t>(k) + 1];
      base ^= static_cast<uint32_t>((ws - kstart[i0]) & 1);
      for (int64_t p = ws; p < we; ++p) {
        const uint64_t tp = ktime[p];
#pragma unroll
        for (int j = 0; j < kChunk; ++j)
          if (j < m && precedes(tp, bb, tc[j], b)) flips ^= 1u << j;
      }
    }
  }
  const uint32_t live = (m >= 32) ? ~0u : ((1u << m) - 1u);
  return ((base & 1u) ? ~flips : flips) & live;
}

// Candidate j of window (b, k): the j-th uniform 64-bit draw placed in the
// window.  Draw 0 is the upper half of call 0 (its lower half decides the
// count); draws 2i-1 and 2i are the halves of call i.
__device__ inline uint64_t cand_time(const ChainDesc& D, int64_t b, uint64_t k, int j, uint64_t v0) {
  uint64_t v = v0;
  if (j > 0) {
    const uint32_t call = static_cast<uint32_t>((j + 1) >> 1);
    const u32x4 r = philox10(D.seed, static_cast<uint32_t>(k), (DOM_INS << 24) | call,
                             static_cast<uint32_t>(b), D.sweep);
    v = (j & 1) ? lo64(r) : hi64(r);
  }
  return D.w == 0 ? v : ((k << (64 - D.w)) | (v >> D.w));
}

// ---------------------------------------------------------------------------
// Insertion of diagonal operators and removal of old ones (steps 2-6):
// per (bond, window) the Poisson count from one 64-bit draw against the
// threshold table, the candidate times, the antiparallel test, then (WRITE)
// the merge with the kept operators into the operator list.  The counting
// pass leaves the acceptance mask of windows with at most 32 candidates in
// accmask, so the writing pass redraws only the times.
template <bool WRITE>
__global__ __launch_bounds__(kBlock) void k_gen(const ChainDesc* __restrict__ descs,
                                                const int64_t* __restrict__ win_bases, int nchain,
                                                int64_t nwin, int64_t* __restrict__ opstart,
                                                uint32_t* __restrict__ accmask,
                                                uint64_t* __restrict__ optime,
                                                uint8_t* __restrict__ optype, int64_t op_cap,
                                                unsigned long long* __restrict__ stats,
                                                uint32_t* __restrict__ flags) {
  // only the writing pass keeps candidate times (LDS bounds its occupancy)
  __shared__ uint64_t slot[WRITE ? kCap * kBlock : 1];
  const int tid = threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  const int64_t start = xcd_block() * kBlock + tid;
  constexpr int kIdx[2] = {ST_CAND, ST_ACC};
  Partial<2> part;
  for (int64_t i = start; i < nwin; i += stride) {
    uint32_t ncand = 0, nacc = 0;
    {
      const int c = chain_of(win_bases, nchain, i);
      if (!WRITE) part.at(c, stats, nchain, kIdx);
      const ChainDesc& D = descs[c];
      const uint8_t* __restrict__ s0 = D.s0[D.cur];
      const int64_t* __restrict__ kstart = D.kstart[D.cur];
      const uint64_t* __restrict__ ktime = D.ktime[D.cur];
      const int64_t li = i - D.win_base;
      const int64_t b = li >> D.w;
      const uint64_t k = static_cast<uint64_t>(li & ((int64_t(1) << D.w) - 1));
      const u32x4 r0 = philox10(D.seed, static_cast<uint32_t>(k), DOM_INS << 24,
                                static_cast<uint32_t>(b), D.sweep);
      const uint64_t u = lo64(r0), v0 = hi64(r0);
      int n = 0;
      while (n < D.K && u >= D.T[n]) ++n;
      ncand = static_cast<uint32_t>(n);
      const bool inlds = WRITE && n <= kCap;
      const bool known = WRITE && n <= 32;
      uint64_t accm = known ? accmask[i] : 0;
      if (known) {
        if (inlds)
          for (int j = 0; j < n; ++j) slot[j * kBlock + tid] = cand_time(D, b, k, j, v0);
      } else {
        // n > kCap here whenever WRITE, so no candidate goes to LDS
        for (int j0 = 0; j0 < n; j0 += kChunk) {
          const int m = (n - j0 < kChunk) ? n - j0 : kChunk;
          uint64_t tc[kChunk];
#pragma unroll
          for (int j = 0; j < kChunk; ++j) tc[j] = (j < m) ? cand_time(D, b, k, j0 + j, v0) : 0;
          accm |= static_cast<uint64_t>(antiparallel_mask(D, s0, kstart, ktime, b, k, tc, m)) << j0;
        }
      }
      nacc = static_cast<uint32_t>(__popcll(accm));
      const int64_t kb = kstart[li], ke = kstart[li + 1];
      if (!WRITE) {
        opstart[i] = (ke - kb) + nacc;
        accmask[i] = static_cast<uint32_t>(accm);
      } else {
        const int64_t base = opstart[i];
        if (opstart[i + 1] > op_cap) {
          atomicOr(flags, 1u);
        } else {
          auto tj = [&](int j) -> uint64_t {
            return inlds ? slot[j * kBlock + tid] : cand_time(D, b, k, j, v0);
          };
          // accepted candidates: rank among accepted + kept at or before
          for (int j = 0; j < n; ++j) {
            if (!((accm >> j) & 1)) continue;
            const uint64_t t = tj(j);
            int64_t rank = 0;
            for (int j2 = 0; j2 < n; ++j2) {
              if (!((accm >> j2) & 1) || j2 == j) continue;
              const uint64_t t2 = tj(j2);
              rank += (t2 < t || (t2 == t && j2 < j)) ? 1 : 0;
            }
            for (int64_t q = kb; q < ke; ++q) rank += (ktime[q] <= t) ? 1 : 0;
            optime[base + rank] = t;
            optype[base + rank] = 0;
          }
          // kept operators: their index + accepted candidates strictly before
          for (int64_t q = kb; q < ke; ++q) {
            const uint64_t t = ktime[q];
            int64_t rank = q - kb;
            for (int j = 0; j < n; ++j)
              if ((accm >> j) & 1) rank += (tj(j) < t) ? 1 : 0;
            optime[base + rank] = t;
            optype[base + rank] = 3;
          }
        }
      }
    }
    part.v[0] += ncand;
    part.v[1] += nacc;
  }
  if (!WRITE) part.flush(stats, nchain, kIdx);
}

// Per-chain operator and node bases after the operator scan.
__global__ void k_chain_bases(const ChainDesc* __restrict__ descs, int nchain,
                              const int64_t* __restrict__ opstart, ChainDyn* __restrict__ dyn,
                              int64_t* __restrict__ op_bases, int64_t* __restrict__ node_bases,
                              int64_t* __restrict__ totals, int64_t op_cap, int64_t node_cap,
                              unsigned long long* __restrict__ stats, uint32_t* __restrict__ flags) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nchain; c += gridDim.x * blockDim.x) {
    const ChainDesc& D = descs[c];
    const int64_t nw = D.n_bonds << D.w;
    const int64_t ob = opstart[D.win_base], oe = opstart[D.win_base + nw];
    ChainDyn d;
    d.op_base = ob;
    d.n_ops = oe - ob;
    d.node_base = D.bnode_base + 2 * ob;
    d.n_nodes = D.nbn + 2 * d.n_ops;
    dyn[c] = d;
    op_bases[c] = d.op_base;
    node_bases[c] = d.node_base;
    unsigned long long* st = stats + static_cast<int64_t>(c) * ST_WORDS;
    st[ST_OPS] = static_cast<unsigned long long>(d.n_ops);
    st[ST_NODES] = static_cast<unsigned long long>(d.n_nodes);
    st[ST_KEPT_IN] = static_cast<unsigned long long>(D.kstart[D.cur][nw]);
    if (c == nchain - 1) {
      totals[0] = oe;                          // operators of all chains
      totals[1] = d.node_base + d.n_nodes;     // loop-graph nodes of all chains
      if (oe > op_cap || totals[1] > node_cap) atomicOr(flags, 2u);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_init_parent(const int64_t* __restrict__ totals,
                                                         int64_t node_cap,
                                                         int64_t* __restrict__ parent) {
  const int64_t n = min(totals[1], node_cap);
  for (int64_t g = xcd_block() * kBlock + threadIdx.x; g < n;
       g += static_cast<int64_t>(gridDim.x) * kBlock)
    parent[g] = g;
}

// ---------------------------------------------------------------------------
// Union-find, lock-free: roots are hooked to the smaller root with a CAS on
// the parent word (parent[x] <= x always, so no cycle can form; leaves never
// become roots again, which is what makes the finds safe without locks,
// Sec. 3.2).  Finds halve the path as they go.
__device__ inline int64_t uf_find(int64_t* parent, int64_t x) {
  int64_t p = parent[x];
  while (p != x) {
    const int64_t gp = parent[p];
    if (gp != p) parent[x] = gp;  // path halving; gp is an ancestor of x
    x = p;
    p = gp;
  }
  return x;
}

__device__ inline void uf_union(int64_t* parent, int64_t a, int64_t b) {
  a = uf_find(parent, a);
  b = uf_find(parent, b);
  while (a != b) {
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
    a = uf_find(parent, static_cast<int64_t>(old));
    b = uf_find(parent, b);
  }
}

// Next event on subspin x after operator (t, b, q): the earliest operator on
// any bond touching x that comes after it in (time, bond, index) order.
// Returns a flat operator index or -1.
__device__ inline int64_t next_event(const ChainDesc& D, const int64_t* __restrict__ opstart,
                                     const uint64_t* __restrict__ optime, int64_t x, int64_t b,
                                     uint64_t k, uint64_t t, int64_t q) {
  int64_t best = -1, bestb = 0;
  uint64_t bestt = 0;
  const int nt = 2 * D.two_s;
  const int64_t W = int64_t(1) << D.w;
  for (int s = 0; s < nt; ++s) {
    const int64_t bb = bond_touching(D, x, s);
    const int64_t i0 = D.win_base + bb * W;
    const int64_t bend = opstart[i0 + W];
    int64_t cand;
    if (bb == b) {
      cand = (q + 1 < bend) ? q + 1 : -1;
    } else {
      int64_t idx = opstart[i0 + static_cast<int64_t>(k)];
      const int64_t we = opstart[i0 + static_cast<int64_t>(k) + 1];
      while (idx < we && precedes(optime[idx], bb, t, b)) ++idx;
      cand = (idx < bend) ? idx : -1;
    }
    if (cand < 0) continue;
    const uint64_t ct = optime[cand];
    if (best < 0 || ct < bestt || (ct == bestt && (bb < bestb || (bb == bestb && cand < best)))) {
      best = cand;
      bestb = bb;
      bestt = ct;
    }
  }
  return best;
}

// Earlier of two candidate events (index, time, bond) in (time, bond,
// index) order; -1 marks no candidate.
__device__ inline int64_t earlier(int64_t c1, uint64_t t1, int64_t b1, int64_t c2, uint64_t t2,
                                  int64_t b2) {
  if (c1 < 0) return c2;
  if (c2 < 0) return c1;
  if (t1 != t2) return t1 < t2 ? c1 : c2;
  if (b1 != b2) return b1 < b2 ? c1 : c2;
  return c1 < c2 ? c1 : c2;
}

// Leg linking (Sec. 2, loops as trees of world-line fragments): the upper
// node of every operator joins, on each of its two subspins, the lower node
// of the next event there, or the top node of that subspin after the last.
// For S = 1/2 the next event on a site is the bond's own next operator or
// the first operator of the neighbouring bond after it: one forward pointer
// per neighbour walks that bond's operators as the window's operators
// advance in time (a merge of three sorted lists).
//
// When the next event on both sites of operator q is the bond's own next
// operator q+1, upper(q) and lower(q+1) are joined by both of their edges
// and by nothing else: a closed loop of two nodes (nine loops in ten at low
// temperature).  It is finished here without union-find: plain stores mark
// it (kPairRoot at its smallest node upper(q), lower(q+1) -> upper(q)), and
// its estimators (size 2, no boundary node, length 2 (t_{q+1} - t_q)) go to
// the chain statistics; the root and accumulation kernels skip it.
struct PairSums {
  int c = -1;
  uint64_t n = 0, l2lo = 0, l2hi = 0;
  __device__ void flush_lane(unsigned long long* stats, int nchain) {
    if (c < 0 || n == 0) return;
    stat_apply(stats, nchain, c, ST_CLUSTERS, -1, FLUSH_ADD, n, 0);
    stat_apply(stats, nchain, c, ST_SIZE2_LO, ST_SIZE2_HI, FLUSH_ADD, 4 * n, 0);
    stat_apply(stats, nchain, c, ST_LEN2_LO, ST_LEN2_HI, FLUSH_ADD, l2lo, l2hi);
    stat_apply(stats, nchain, c, ST_MAXSIZE, -1, FLUSH_MAX, 2, 0);
    n = l2lo = l2hi = 0;
  }
  __device__ void at(int cn, unsigned long long* stats, int nchain) {
    if (cn == c) return;
    flush_lane(stats, nchain);
    c = cn;
  }
  __device__ void add(uint64_t dt) {
    n += 1;
    const uint64_t l32 = dt >> 31;  // (2 dt) >> 32
    const u128p q = mul64x64(l32, l32);
    l2lo += q.lo;
    l2hi += q.hi + (l2lo < q.lo ? 1u : 0u);
  }
  // convergent: every thread of the block must call it
  __device__ void flush(unsigned long long* stats, int nchain) {
    block_flush(stats, nchain, c, ST_CLUSTERS, -1, FLUSH_ADD, n, 0);
    block_flush(stats, nchain, c, ST_SIZE2_LO, ST_SIZE2_HI, FLUSH_ADD, 4 * n, 0);
    block_flush(stats, nchain, c, ST_LEN2_LO, ST_LEN2_HI, FLUSH_ADD, l2lo, l2hi);
    block_flush(stats, nchain, c, ST_MAXSIZE, -1, FLUSH_MAX, n ? 2 : 0, 0);
  }
};

__global__ __launch_bounds__(kBlock) void k_link_ops(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ win_bases, int nchain,
    int64_t nwin, const ChainDyn* __restrict__ dyn, const int64_t* __restrict__ opstart,
    const uint64_t* __restrict__ optime, int64_t* __restrict__ parent,
    unsigned long long* __restrict__ stats, const uint32_t* __restrict__ flags) {
  if (*flags) return;
  PairSums pairs;
  for (int64_t i = xcd_block() * kBlock + threadIdx.x; i < nwin;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int c = chain_of(win_bases, nchain, i);
    const ChainDesc& D = descs[c];
    const ChainDyn dy = dyn[c];
    const int64_t li = i - D.win_base;
    const int64_t b = li >> D.w;
    const uint64_t k = static_cast<uint64_t>(li & ((int64_t(1) << D.w) - 1));
    const int64_t xs[2] = {bond_x(D, b), bond_y(D, b)};
    if (D.two_s == 1) {
      const int64_t W = int64_t(1) << D.w;
      const int64_t bl = b == 0 ? D.L - 1 : b - 1, br = b + 1 == D.L ? 0 : b + 1;
      const int64_t il = D.win_base + bl * W, ir = D.win_base + br * W;
      const int64_t el = opstart[il + k + 1], er = opstart[ir + k + 1];  // window ends
      const int64_t lend = opstart[il + W], rend = opstart[ir + W];      // bond ends
      const int64_t bend = opstart[D.win_base + b * W + W];
      int64_t pl = opstart[il + k], pr = opstart[ir + k];
      uint64_t tl = pl < lend ? optime[pl] : 0, tr = pr < rend ? optime[pr] : 0;
      const int64_t qe = opstart[i + 1];
      for (int64_t q = opstart[i]; q < qe; ++q) {
        const uint64_t t = optime[q];
        while (pl < el && precedes(tl, bl, t, b)) {
          ++pl;
          tl = pl < lend ? optime[pl] : 0;
        }
        while (pr < er && precedes(tr, br, t, b)) {
          ++pr;
          tr = pr < rend ? optime[pr] : 0;
        }
        const int64_t own = q + 1 < bend ? q + 1 : -1;
        const uint64_t tn = own >= 0 ? optime[own] : 0;
        const int64_t nx = earlier(own, tn, b, pl < lend ? pl : -1, tl, bl);
        const int64_t ny = earlier(own, tn, b, pr < rend ? pr : -1, tr, br);
        const int64_t up = dy.node_base + D.nbn + 2 * (q - dy.op_base) + 1;
        if (own >= 0 && nx == own && ny == own) {  // closed two-node loop
          parent[up] = kPairRoot;
          parent[up + 1] = up;
          pairs.at(c, stats, nchain);
          pairs.add(tn - t);
          continue;
        }
        uf_union(parent, up, nx >= 0 ? dy.node_base + D.nbn + 2 * (nx - dy.op_base) : dy.node_base + xs[0]);
        uf_union(parent, up, ny >= 0 ? dy.node_base + D.nbn + 2 * (ny - dy.op_base) : dy.node_base + xs[1]);
      }
      continue;
    }
    for (int64_t q = opstart[i]; q < opstart[i + 1]; ++q) {
      const uint64_t t = optime[q];
      const int64_t up = dy.node_base + D.nbn + 2 * (q - dy.op_base) + 1;
      for (int e = 0; e < 2; ++e) {
        const int64_t nx = next_event(D, opstart, optime, xs[e], b, k, t, q);
        const int64_t top = (D.two_s == 1) ? xs[e] : D.n_sites + xs[e];
        const int64_t to = (nx >= 0) ? dy.node_base + D.nbn + 2 * (nx - dy.op_base)
                                     : dy.node_base + top;
        uf_union(parent, up, to);
      }
    }
  }
  pairs.flush(stats, nchain);
}

// Boundary nodes: bottom(x) joins the lower node of the first event on x;
// an empty subspin joins bottom and top directly (S=1/2: one node, no edge).
__global__ __launch_bounds__(kBlock) void k_link_sites(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ site_bases, int nchain,
    int64_t nsites, const ChainDyn* __restrict__ dyn, const int64_t* __restrict__ opstart,
    const uint64_t* __restrict__ optime, int64_t* __restrict__ parent,
    const uint32_t* __restrict__ flags) {
  if (*flags) return;
  for (int64_t gi = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; gi < nsites;
       gi += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int c = chain_of(site_bases, nchain, gi);
    const ChainDesc& D = descs[c];
    const ChainDyn dy = dyn[c];
    const int64_t x = gi - D.site_base;
    const int64_t W = int64_t(1) << D.w;
    int64_t best = -1, bestb = 0;
    uint64_t bestt = 0;
    for (int s = 0; s < 2 * D.two_s; ++s) {
      const int64_t bb = bond_touching(D, x, s);
      const int64_t i0 = D.win_base + bb * W;
      const int64_t f = opstart[i0];
      if (f >= opstart[i0 + W]) continue;
      const uint64_t ct = optime[f];
      if (best < 0 || ct < bestt || (ct == bestt && bb < bestb)) {
        best = f;
        bestb = bb;
        bestt = ct;
      }
    }
    const int64_t bottom = dy.node_base + x;
    if (best >= 0)
      uf_union(parent, bottom, dy.node_base + D.nbn + 2 * (best - dy.op_base));
    else if (D.two_s > 1)
      uf_union(parent, bottom, dy.node_base + D.n_sites + x);
  }
}

// Symmetrization of the 2S subspins of each spin (split-spin only): a
// permutation pi drawn uniformly among those that map the up (down)
// subspins at beta- onto the up (down) subspins at 0+; top(j,a) joins
// bottom(j, pi(a)).  Fisher-Yates on the SYM stream of the spin.
__global__ __launch_bounds__(kBlock) void k_symmetrize(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ spin_bases, int nchain,
    int64_t nspins, const ChainDyn* __restrict__ dyn, int64_t* __restrict__ parent,
    uint32_t* __restrict__ flags) {
  if (*flags) return;
  for (int64_t gj = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; gj < nspins;
       gj += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int c = chain_of(spin_bases, nchain, gj);
    const ChainDesc& D = descs[c];
    if (D.two_s == 1) continue;
    const ChainDyn dy = dyn[c];
    const uint8_t* __restrict__ s0 = D.s0[D.cur];
    const int64_t* __restrict__ kstart = D.kstart[D.cur];
    int64_t* __restrict__ perm = D.perm;
    const int64_t j = gj - D.spin_base;
    const int ts = D.two_s;
    const int64_t W = int64_t(1) << D.w;
    int64_t up_t[8], dn_t[8], up_b[8], dn_b[8];
    int nut = 0, ndt = 0, nub = 0, ndb = 0;
    for (int a = 0; a < ts; ++a) {
      const int64_t x = j * ts + a;
      uint32_t par = 0;
      for (int s = 0; s < 2 * ts; ++s) {
        const int64_t bb = bond_touching(D, x, s);
        const int64_t i0 = bb * W;
        par ^= static_cast<uint32_t>((kstart[i0 + W] - kstart[i0]) & 1);
      }
      const uint32_t sb = s0[x];
      if (sb ^ par)
        up_t[nut++] = x;
      else
        dn_t[ndt++] = x;
      if (sb)
        up_b[nub++] = x;
      else
        dn_b[ndb++] = x;
    }
    if (nut != nub) {
      atomicOr(flags, 4u);  // inconsistent world lines: cannot symmetrize
      continue;
    }
    uint32_t d = 0;
    uint64_t pending = 0;
    auto draw = [&](uint64_t m) -> uint64_t {
      uint64_t u;
      if ((d & 1u) == 0) {
        const u32x4 r = philox10(D.seed, static_cast<uint32_t>(j), (DOM_SYM << 24) | (d >> 1), 0u,
                                 D.sweep);
        u = lo64(r);
        pending = hi64(r);
      } else {
        u = pending;
      }
      ++d;
      return __umul64hi(u, m);
    };
    for (int i = nub - 1; i >= 1; --i) {
      const int r = static_cast<int>(draw(static_cast<uint64_t>(i + 1)));
      const int64_t tmp = up_b[i];
      up_b[i] = up_b[r];
      up_b[r] = tmp;
    }
    for (int i = ndb - 1; i >= 1; --i) {
      const int r = static_cast<int>(draw(static_cast<uint64_t>(i + 1)));
      const int64_t tmp = dn_b[i];
      dn_b[i] = dn_b[r];
      dn_b[r] = tmp;
    }
    for (int q = 0; q < nut; ++q) {
      perm[up_t[q]] = up_b[q];
      uf_union(parent, dy.node_base + D.n_sites + up_t[q], dy.node_base + up_b[q]);
    }
    for (int q = 0; q < ndt; ++q) {
      perm[dn_t[q]] = dn_b[q];
      uf_union(parent, dy.node_base + D.n_sites + dn_t[q], dy.node_base + dn_b[q]);
    }
  }
}

// Full path compression: parent[g] = root = smallest node of g's loop.
// Roots (parent[g] == g) are counted per chunk of 4,096 nodes on the way
// (each wave covers 64 consecutive nodes of one chunk): rcnt feeds the
// numbering of the loops.
__global__ __launch_bounds__(kBlock) void k_compress(const int64_t* __restrict__ totals,
                                                      int64_t* __restrict__ parent,
                                                      unsigned long long* __restrict__ rcnt,
                                                      const uint32_t* __restrict__ flags) {
  if (*flags) return;
  const int64_t n = totals[1];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  const int64_t iters = (n + stride - 1) / stride;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t g = xcd_block() * kBlock + threadIdx.x + it * stride;
    const int64_t p0 = g < n ? parent[g] : -1;
    const unsigned long long roots = __ballot(p0 == g);
    if (lane_id() == 0 && roots)
      atomicAdd(rcnt + (g >> 12), static_cast<unsigned long long>(__popcll(roots)));
    if (g >= n) continue;
    int64_t r = g, p = p0;
    while (p != r && p >= 0) {  // a negative word marks a finished two-node loop
      r = p;
      p = parent[r];
    }
    if (r != g) parent[g] = r;
  }
}

// Loop-flip bit of a chain-local label: bit (label mod 128) of the Philox
// block (label / 128) of the FLIP stream of this sweep.
__device__ inline uint32_t flip_bit(const ChainDesc& D, int64_t label) {
  const uint64_t q = static_cast<uint64_t>(label) >> 7;
  const uint32_t i = static_cast<uint32_t>(label & 127);
  const u32x4 r = philox10(D.seed, static_cast<uint32_t>(q),
                           (DOM_FLIP << 24) | static_cast<uint32_t>((q >> 32) & 0xFFFFFFu), 0u,
                           D.sweep);
  const uint32_t wsel = i >> 5;
  const uint32_t word = wsel == 0 ? r.x : (wsel == 1 ? r.y : (wsel == 2 ? r.z : r.w));
  return (word >> (i & 31)) & 1u;
}

constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t& total) {
  // wave inclusive scan
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0;
    for (int q = 0; q < kBlock / 64; ++q) {
      const int64_t t = sh[q];
      sh[q] = s;
      s += t;
    }
    sh[kBlock / 64] = s;
  }
  __syncthreads();
  const int64_t r = sh[wv] + x - v;
  total = sh[kBlock / 64];
  __syncthreads();
  return r;
}

// Roots get compact loop indices in node order: roots are counted per chunk
// of kRootChunk nodes, the counts are scanned, and each chunk numbers its
// roots from its offset (no shared counter).  A chunk is kRootPer steps of
// kBlock consecutive nodes (coalesced loads, all issued before use); a
// root's rank in its chunk is the roots of earlier steps, of earlier waves
// in its step, and of lower lanes in its wave's ballot.
constexpr int kAccWords = LC_ACC_WORDS;
constexpr int kRootPer = 16;                      // steps per chunk
constexpr int kRootChunk = kBlock * kRootPer;     // nodes per chunk (2^12, counted in k_compress)
static_assert(kRootChunk == 4096, "k_compress counts roots per 4,096 nodes");

// Roots: compact index (stored as the code -1 - index in the root's parent
// word), cleared accumulators, loop count.  A loop
// through a boundary node has a bottom boundary node as its smallest node
// (boundary ids come first, and every top node is joined to a bottom one),
// so its boundary sums live in a per-subspin record bacc[site], cleared here.
__global__ __launch_bounds__(kBlock) void k_roots(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ node_bases, int nchain,
    const int64_t* __restrict__ totals, int64_t* __restrict__ parent,
    unsigned long long* __restrict__ acc, unsigned long long* __restrict__ bacc, int64_t root_cap,
    int64_t nchunks, const int64_t* __restrict__ rbase, unsigned long long* __restrict__ stats,
    uint32_t* __restrict__ flags) {
  __shared__ int wsum[kRootPer][kWaves];
  if (*flags) return;
  if (rbase[nchunks] > root_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flags, LC_FLAG_ROOTS);
    return;
  }
  const int64_t n = totals[1];
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  constexpr int kIdx[1] = {ST_CLUSTERS};
  Partial<1> part;
  for (int64_t ch = xcd_block(); ch < nchunks; ch += gridDim.x) {
    const int64_t g0 = ch * kRootChunk + threadIdx.x;
    int64_t pv[kRootPer];
#pragma unroll
    for (int s = 0; s < kRootPer; ++s) {
      const int64_t g = g0 + s * kBlock;
      pv[s] = g < n ? parent[g] : -1;
    }
    unsigned long long m[kRootPer];
#pragma unroll
    for (int s = 0; s < kRootPer; ++s) {
      m[s] = __ballot(pv[s] == g0 + s * kBlock);
      if (lane == 0) wsum[s][wv] = __popcll(m[s]);
    }
    __syncthreads();
    int64_t idx = rbase[ch];
#pragma unroll
    for (int s = 0; s < kRootPer; ++s) {
      int woff = 0, tot = 0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) {
        const int x = wsum[s][q];
        woff += q < wv ? x : 0;
        tot += x;
      }
      const int64_t g = g0 + s * kBlock;
      if (pv[s] == g) {
        const int64_t i = idx + woff + __popcll(m[s] & below);
        const int c = chain_of(node_bases, nchain, g);
        part.at(c, stats, nchain, kIdx);
        part.v[0] += 1;
        const ChainDesc& D = descs[c];
        const int64_t v = g - node_bases[c];
        parent[g] = -1 - i;
        unsigned long long* a = acc + kAccWords * i;
        a[0] = 0;
        a[1] = 0;
        a[2] = 0;
        if (v < D.n_sites) bacc[D.site_base + v] = 0;
      }
      idx += tot;
    }
    __syncthreads();  // wsum is rewritten for the next chunk
  }
  part.flush(stats, nchain, kIdx);
}

__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t w = __shfl_xor(v, o);
    v = w > v ? w : v;
  }
  return v;
}

__device__ inline void flush_carry(unsigned long long* acc, int64_t key, uint64_t v0, uint64_t v1,
                                   uint64_t v2) {
  unsigned long long* a = acc + kAccWords * key;
  atomicAdd(a + 0, static_cast<unsigned long long>(v0));
  if (v1) atomicAdd(a + 1, static_cast<unsigned long long>(v1));
  if (v2) atomicAdd(a + 2, static_cast<unsigned long long>(v2));
}

// Per-loop accumulators (before the flip), three 64-bit words per loop:
//   [0] nodes + (top nodes << 40)
//   [1] sum of +-hi32(t), [2] sum of +-lo32(t)  over operator nodes: lower
//       nodes count +t, upper nodes -t (two vertical segments end / start)
// so the loop length is 2^64 tops + 2 (2^32 [1] + [2]) ticks.  Every word
// takes plain additions without carries between words (the sums are exact
// modulo 2^64 and their true values fit).  Bottom boundary nodes add
// 1 + (spin << 32) to bacc of their loop's root subspin.
__global__ __launch_bounds__(kBlock) void k_accum(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ node_bases, int nchain,
    const ChainDyn* __restrict__ dyn, const int64_t* __restrict__ totals,
    const int64_t* __restrict__ parent, const uint64_t* __restrict__ optime,
    unsigned long long* __restrict__ acc, unsigned long long* __restrict__ bacc,
    const uint32_t* __restrict__ flags) {
  if (*flags) return;
  const int64_t n = totals[1];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  const int64_t iters = (n + stride - 1) / stride;
  // fields of the chain of the current node, reloaded only when the node
  // leaves the chain's range [cbeg, cend)
  int64_t cbeg = 0, cend = -1, op_base = 0, nbn = 0, n_sites = 0, site_base = 0;
  int two_s = 1;
  const uint8_t* s0p = nullptr;
  // wave carry: sums of one hot loop (wave-uniform), flushed once
  int64_t ck = -1;
  uint64_t cv0 = 0, cv1 = 0, cv2 = 0;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t g = xcd_block() * kBlock + threadIdx.x + it * stride;
    bool active = g < n;
    int64_t r = -1;
    uint64_t w0 = 0, w1 = 0, w2 = 0;
    if (active) {
      if (g < cbeg || g >= cend) {
        const int c = chain_of(node_bases, nchain, g);
        const ChainDesc& D = descs[c];
        const ChainDyn dy = dyn[c];
        cbeg = dy.node_base;
        cend = dy.node_base + dy.n_nodes;
        op_base = dy.op_base;
        nbn = D.nbn;
        n_sites = D.n_sites;
        site_base = D.site_base;
        two_s = D.two_s;
        s0p = D.s0[D.cur];
      }
      const int64_t v = g - cbeg;
      const int64_t p = parent[g];
      const int64_t code = p >= 0 ? parent[p] : p;
      active = code != kPairRoot;  // two-node loops were finished while linking
      if (active) {
        r = -1 - code;
        w0 = 1;
        if (v < nbn) {
          const bool bottom = v < n_sites;
          if ((two_s == 1) || !bottom) w0 += 1ull << 40;  // top node: + 2^64
          const int64_t root = (p >= 0 ? p : g) - cbeg;
          if (bottom && root < n_sites)  // always true: the root is a bottom node
            atomicAdd(bacc + site_base + root,
                      1ull + (static_cast<uint64_t>(2 * static_cast<int64_t>(s0p[v]) - 1) << 32));
        } else {
          const int64_t q = (v - nbn) >> 1;
          const uint64_t t = optime[op_base + q];
          const uint64_t th = t >> 32, tl = t & 0xFFFFFFFFull;
          if (((v - nbn) & 1) == 0) {
            w1 = th;
            w2 = tl;
          } else {
            w1 = 0 - th;
            w2 = 0 - tl;
          }
        }
      }
    }
    // Reduce by loop within the wave: bitonic sort of one packed word per
    // lane, (loop << 6) | lane (loop indices are below 2^40), so only the key
    // moves through the 21 exchange stages; each lane then fetches the sums
    // of the element it ended up with, a segmented scan adds equal loops, and
    // the last lane of each run issues one set of atomics per distinct loop.
    // Very large loops (high spin, low temperature) meet nearly every wave:
    // the wave carries the sums of one such loop across its steps instead of
    // adding them to the same record from every wave and step.
    const int lane = lane_id();
    uint64_t sk = active ? ((static_cast<uint64_t>(r) << 6) | static_cast<uint64_t>(lane)) : ~0ull;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        const uint64_t pk = __shfl_xor(sk, j);
        const bool ascending = (lane & k) == 0, lower = (lane & j) == 0;
        const bool take = (lower == ascending) ? (pk < sk) : (pk > sk);
        sk = take ? pk : sk;
      }
    }
    const int src = static_cast<int>(sk & 63ull);
    const int64_t key = sk == ~0ull ? INT64_MAX : static_cast<int64_t>(sk >> 6);
    // per-wave node and top counts fit 16 bits each
    uint32_t c0 = static_cast<uint32_t>(__shfl(static_cast<uint32_t>((w0 & 0xFFFFull) | ((w0 >> 40) << 16)), src));
    w1 = __shfl(w1, src);
    w2 = __shfl(w2, src);
    // runs of equal loops: head lanes from one ballot, segment id = heads so far
    const int64_t pkey = __shfl_up(key, 1);
    const unsigned long long heads = __ballot(lane == 0 || pkey != key);
    const int seg = __popcll(heads & ((lane == 63) ? ~0ull : ((2ull << lane) - 1ull)));
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int qs = __shfl_up(seg, d);
      const uint32_t q0 = __shfl_up(c0, d);
      const uint64_t q1 = __shfl_up(w1, d), q2 = __shfl_up(w2, d);
      if (lane >= d && qs == seg) {
        c0 += q0;
        w1 += q1;
        w2 += q2;
      }
    }
    const bool last = lane == 63 || ((heads >> (lane + 1)) & 1ull);
    const bool seg_end = key != INT64_MAX && last;
    const uint64_t v0 = static_cast<uint64_t>(c0 & 0xFFFFu) + (static_cast<uint64_t>(c0 >> 16) << 40);
    // the carried loop absorbs its segment without atomics
    bool absorbed = seg_end && key == ck;
    unsigned long long m = __ballot(absorbed);
    if (!m) {
      // the carried loop is absent: a segment of at least 16 nodes takes over
      // the carry (the old carry is flushed); the largest such segment wins
      const uint32_t cnt = seg_end ? (c0 & 0xFFFFu) : 0u;
      const uint32_t best = wave_max_u32((cnt << 6) | static_cast<uint32_t>(lane));
      if ((best >> 6) >= 16) {
        if (ck >= 0 && lane == 0) flush_carry(acc, ck, cv0, cv1, cv2);
        ck = __shfl(key, static_cast<int>(best & 63u));
        cv0 = cv1 = cv2 = 0;
        absorbed = lane == static_cast<int>(best & 63u);
        m = __ballot(absorbed);
      }
    }
    if (m) {
      const int src = __ffsll(static_cast<long long>(m)) - 1;
      cv0 += __shfl(v0, src);
      cv1 += __shfl(w1, src);
      cv2 += __shfl(w2, src);
    }
    if (seg_end && !absorbed) {
      unsigned long long* a = acc + kAccWords * key;
      atomicAdd(a + 0, static_cast<unsigned long long>(v0));
      if (w1) atomicAdd(a + 1, static_cast<unsigned long long>(w1));
      if (w2) atomicAdd(a + 2, static_cast<unsigned long long>(w2));
    }
  }
  if (ck >= 0 && lane_id() == 0) flush_carry(acc, ck, cv0, cv1, cv2);
}

// First loop index of each chain: a chain's node 0 is always a root (the
// smallest node of its loop) and loops are numbered in node order.
__global__ void k_loop_bases(const int64_t* __restrict__ node_bases, int nchain,
                             const int64_t* __restrict__ parent, int64_t* __restrict__ loop_bases,
                             const uint32_t* __restrict__ flags) {
  if (*flags) return;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nchain; c += gridDim.x * blockDim.x)
    loop_bases[c] = -1 - parent[node_bases[c]];
}

// Per-loop squares summed into the chain statistics (walks the compact loop
// records; the chain of a loop is found from its index range).
__global__ __launch_bounds__(kBlock) void k_cluster_sums(
    const int64_t* __restrict__ loop_bases, int nchain, const int64_t* __restrict__ nloops,
    int64_t root_cap, const unsigned long long* __restrict__ acc,
    unsigned long long* __restrict__ stats, const uint32_t* __restrict__ flags) {
  if (*flags) return;
  const int64_t n = *nloops < root_cap ? *nloops : root_cap;
  int cc = -1;
  int64_t cend = 0;  // first loop index past chain cc
  uint64_t s2lo = 0, s2hi = 0, l2lo = 0, l2hi = 0, mx = 0;
  auto flush_lane = [&]() {  // into this block's stripes
    stat_apply(stats, nchain, cc, ST_SIZE2_LO, ST_SIZE2_HI, FLUSH_ADD, s2lo, s2hi);
    stat_apply(stats, nchain, cc, ST_LEN2_LO, ST_LEN2_HI, FLUSH_ADD, l2lo, l2hi);
    stat_apply(stats, nchain, cc, ST_MAXSIZE, -1, FLUSH_MAX, mx, 0);
    s2lo = s2hi = l2lo = l2hi = mx = 0;
  };
  for (int64_t i = xcd_block() * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    if (cc < 0 || i >= cend) {
      if (cc >= 0) flush_lane();
      cc = chain_of(loop_bases, nchain, i);
      cend = cc + 1 < nchain ? loop_bases[cc + 1] : n;
    }
    const unsigned long long* a = acc + kAccWords * i;
    const uint64_t sz = a[0] & ((1ull << 40) - 1), tops = a[0] >> 40;
    const u128p q2 = mul64x64(sz, sz);
    s2lo += q2.lo;
    s2hi += q2.hi + (s2lo < q2.lo ? 1u : 0u);
    // len = 2^64 tops + 2^33 S_hi + 2 S_lo as a signed 128-bit sum, then >> 32
    const int64_t shi = static_cast<int64_t>(a[1]), slo = static_cast<int64_t>(a[2]);
    uint64_t llo = static_cast<uint64_t>(slo) << 1;
    uint64_t lhi = static_cast<uint64_t>(slo >> 63);  // sign extension of 2 S_lo
    const uint64_t hlo = static_cast<uint64_t>(shi) << 33;
    const uint64_t hhi = static_cast<uint64_t>(shi >> 31);  // arithmetic: bits 31.. of shi
    const uint64_t t1 = llo + hlo;
    lhi = lhi + hhi + (t1 < llo ? 1u : 0u) + tops;
    llo = t1;
    const uint64_t l32 = (llo >> 32) | (lhi << 32);  // len >> 32, len < 2^96
    const u128p l2 = mul64x64(l32, l32);
    l2lo += l2.lo;
    l2hi += l2.hi + (l2lo < l2.lo ? 1u : 0u);
    mx = sz > mx ? sz : mx;
  }
  block_flush(stats, nchain, cc, ST_SIZE2_LO, ST_SIZE2_HI, FLUSH_ADD, s2lo, s2hi);
  block_flush(stats, nchain, cc, ST_LEN2_LO, ST_LEN2_HI, FLUSH_ADD, l2lo, l2hi);
  block_flush(stats, nchain, cc, ST_MAXSIZE, -1, FLUSH_MAX, mx, 0);
}

// Flip bit of the loop through node g, from its root (the loop's smallest
// node): after compression a non-root holds its root, a root a negative code.
__device__ inline uint32_t node_flip(const ChainDesc& D, int64_t node_base,
                                     const int64_t* __restrict__ parent, int64_t g) {
  const int64_t p = parent[g];
  return flip_bit(D, (p >= 0 ? p : g) - node_base);
}

// Cluster flip (step 7): the type of an operator changes when exactly one of
// its two loops flips; kept (off-diagonal) operators are counted per window.
__global__ __launch_bounds__(kBlock) void k_flip_ops(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ win_bases, int nchain,
    int64_t nwin, const ChainDyn* __restrict__ dyn, const int64_t* __restrict__ opstart,
    const int64_t* __restrict__ parent, uint8_t* __restrict__ optype, int64_t* __restrict__ kcnt, unsigned long long* __restrict__ stats,
    const uint32_t* __restrict__ flags) {
  if (*flags) return;
  constexpr int kIdx[1] = {ST_KEPT_OUT};
  Partial<1> part;
  for (int64_t i = xcd_block() * kBlock + threadIdx.x; i < nwin;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int c = chain_of(win_bases, nchain, i);
    part.at(c, stats, nchain, kIdx);
    const ChainDesc& D = descs[c];
    const ChainDyn dy = dyn[c];
    uint64_t kept = 0;
    for (int64_t q = opstart[i]; q < opstart[i + 1]; ++q) {
      const int64_t lo = dy.node_base + D.nbn + 2 * (q - dy.op_base);
      const uint8_t v = optype[q];
      const uint8_t ty = static_cast<uint8_t>((v & 1) ^ node_flip(D, dy.node_base, parent, lo) ^
                                              node_flip(D, dy.node_base, parent, lo + 1));
      optype[q] = static_cast<uint8_t>(ty | (v & 2));
      kept += ty;
    }
    kcnt[i] = static_cast<int64_t>(kept);
    part.v[0] += kept;
  }
  part.flush(stats, nchain, kIdx);
}

// New spins at tau = 0; the boundary estimators of every loop whose root is
// this subspin's bottom node (n0 = bottom nodes, m = their spin sum before
// the flip) are squared into the chain statistics.
__global__ __launch_bounds__(kBlock) void k_flip_sites(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ site_bases, int nchain,
    int64_t nsites, const ChainDyn* __restrict__ dyn, const int64_t* __restrict__ parent,
    const unsigned long long* __restrict__ bacc,
    unsigned long long* __restrict__ stats, const uint32_t* __restrict__ flags) {
  if (*flags) return;
  constexpr int kIdx[3] = {ST_MAFTER, ST_M2, ST_N0SQ};
  Partial<3> part;
  for (int64_t gi = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; gi < nsites;
       gi += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int c = chain_of(site_bases, nchain, gi);
    part.at(c, stats, nchain, kIdx);
    const ChainDesc& D = descs[c];
    const int64_t x = gi - D.site_base;
    const int64_t p = parent[dyn[c].node_base + x];
    const uint8_t s = D.s0[D.cur][x] ^ static_cast<uint8_t>(flip_bit(D, p >= 0 ? p - dyn[c].node_base : x));
    D.s0[D.cur ^ 1][x] = s;
    part.v[0] += static_cast<uint64_t>(2 * static_cast<int64_t>(s) - 1);
    if (p < 0) {  // root of its loop
      const uint64_t b = bacc[gi];
      const int64_t n0 = static_cast<int64_t>(b & 0xFFFFFFFFull);
      const int64_t m = static_cast<int64_t>(static_cast<int32_t>(b >> 32));
      part.v[1] += static_cast<uint64_t>(m * m);
      part.v[2] += static_cast<uint64_t>(n0 * n0);
    }
  }
  part.flush(stats, nchain, kIdx);
}

// The off-diagonal operators become the next sweep's world lines.
__global__ __launch_bounds__(kBlock) void k_compact(const ChainDesc* __restrict__ descs,
                                                     const int64_t* __restrict__ win_bases,
                                                     int nchain, int64_t nwin,
                                                     const int64_t* __restrict__ opstart,
                                                     const uint64_t* __restrict__ optime,
                                                     const uint8_t* __restrict__ optype,
                                                     const int64_t* __restrict__ kflat,
                                                     uint32_t* __restrict__ flags) {
  // a sweep with any overflow or error is discarded: kflat may be stale
  if (*flags) return;
  for (int64_t i = xcd_block() * kBlock + threadIdx.x; i < nwin;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int c = chain_of(win_bases, nchain, i);
    const ChainDesc& D = descs[c];
    const int64_t li = i - D.win_base;
    const int64_t nw = D.n_bonds << D.w;
    const int64_t kb = kflat[D.win_base];
    if (kflat[D.win_base + nw] - kb > D.kept_cap) {
      atomicOr(flags, 8u);
      continue;
    }
    int64_t* __restrict__ ks = D.kstart[D.cur ^ 1];
    uint64_t* __restrict__ kt = D.ktime[D.cur ^ 1];
    int64_t o = kflat[i] - kb;
    ks[li] = o;
    if (li == nw - 1) ks[nw] = kflat[i + 1] - kb;
    for (int64_t q = opstart[i]; q < opstart[i + 1]; ++q)
      if (optype[q] & 1) kt[o++] = optime[q];
  }
}

// Fold the striped statistics into the counters (one thread per chain and
// word; a 128-bit pair is summed with carries by the thread of its low word).
__global__ void k_stats_reduce(unsigned long long* __restrict__ stats, int nchain) {
  const int64_t nw = static_cast<int64_t>(nchain) * ST_WORDS;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nw;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int w = static_cast<int>(i % ST_WORDS);
    const unsigned long long* sp = stats + nw + i * kStripes;
    if (w == ST_SIZE2_HI || w == ST_LEN2_HI) continue;
    if (w == ST_MAXSIZE) {
      unsigned long long m = stats[i];
      for (int k = 0; k < kStripes; ++k) m = sp[k] > m ? sp[k] : m;
      stats[i] = m;
    } else if (w == ST_SIZE2_LO || w == ST_LEN2_LO) {
      const unsigned long long* sh = sp + kStripes;  // stripes of the high word
      uint64_t lo = stats[i], hi = stats[i + 1];
      for (int k = 0; k < kStripes; ++k) {
        const uint64_t t = lo + sp[k];
        hi += sh[k] + (t < lo ? 1u : 0u);
        lo = t;
      }
      stats[i] = lo;
      stats[i + 1] = hi;
    } else {
      uint64_t sum = stats[i];
      for (int k = 0; k < kStripes; ++k) sum += sp[k];
      stats[i] = sum;
    }
  }
}

__global__ void k_advance(ChainDesc* __restrict__ descs, int nchain, const uint32_t* __restrict__ flags) {
  if (*flags) return;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nchain; c += gridDim.x * blockDim.x) {
    descs[c].sweep += 1;
    descs[c].cur ^= 1;
  }
}

// Append this sweep's statistics and flags to the host-visible record ring.
__global__ void k_record(const unsigned long long* __restrict__ stats, int64_t nwords,
                         const uint32_t* __restrict__ flags, unsigned long long* __restrict__ ring,
                         uint32_t* __restrict__ ring_ctr, uint32_t ring_cap) {
  const uint32_t slot = *ring_ctr;
  __syncthreads();
  if (slot < ring_cap) {
    unsigned long long* dst = ring + static_cast<int64_t>(slot) * (nwords + 1);
    for (int64_t i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = stats[i];
    if (threadIdx.x == 0) dst[nwords] = *flags;
  }
  if (threadIdx.x == 0) *ring_ctr = slot + 1;
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// Initial world lines: Neel state with a random phase, no operators.
__global__ void k_init_chain(const ChainDesc* __restrict__ d) {
  const ChainDesc& D = *d;
  const u32x4 r = philox10(D.seed, 0u, DOM_INIT << 24, 0u, 0u);
  const int64_t nw = D.n_bonds << D.w;
  for (int64_t x = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; x < D.n_sites;
       x += static_cast<int64_t>(gridDim.x) * blockDim.x)
    D.s0[D.cur][x] = static_cast<uint8_t>(((x / D.two_s) & 1) ^ (r.x & 1u));
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i <= nw;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    D.kstart[D.cur][i] = 0;
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of int64 in place (reduce, scan of block sums,
// rescan).  a[0..n) -> exclusive prefix, a[n] = total.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int64_t* __restrict__ a, int64_t n,
                                                         int64_t per_block,
                                                         int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[kBlock / 64 + 1];
  const int64_t s = blockIdx.x * per_block, e = min(n, s + per_block);
  int64_t acc = 0;
  for (int64_t i = s + threadIdx.x; i < e; i += kBlock) acc += a[i];
  int64_t total;
  block_exclusive_scan(acc, sh, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_blocks(int64_t* __restrict__ bsum, int nb) {
  __shared__ int64_t sh[kBlock / 64 + 1];
  int64_t carry = 0;
  for (int base = 0; base < nb; base += kBlock) {
    const int i = base + threadIdx.x;
    const int64_t v = i < nb ? bsum[i] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan(v, sh, total);
    if (i < nb) bsum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(int64_t* __restrict__ a, int64_t n,
                                                        int64_t per_block,
                                                        const int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[kBlock / 64 + 1];
  const int64_t s = blockIdx.x * per_block, e = min(n, s + per_block);
  int64_t carry = bsum[blockIdx.x];
  for (int64_t t0 = s; t0 < e; t0 += kScanTile) {
    int64_t v[kScanItems];
    int64_t loc = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
      const int64_t i = t0 + static_cast<int64_t>(threadIdx.x) * kScanItems + q;
      v[q] = (i < e) ? a[i] : 0;
      loc += v[q];
    }
    int64_t total;
    int64_t run = carry + block_exclusive_scan(loc, sh, total);
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
      const int64_t i = t0 + static_cast<int64_t>(threadIdx.x) * kScanItems + q;
      if (i < e) a[i] = run;
      run += v[q];
    }
    carry += total;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) a[n] = carry;
}

}  // namespace lc

// ---------------------------------------------------------------------------
// Host-side launchers.
using namespace lc;

static int grid_for(int64_t n, int cap_blocks) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap_blocks) b = cap_blocks;
  return static_cast<int>(b);
}

hipError_t lc_launch_scan(int64_t* a, int64_t n, int64_t* bsum, hipStream_t s) {
  // a has n+1 entries; bsum has kScanBlocks+1 entries
  const int nb = LC_SCAN_BLOCKS;
  int64_t per = (n + nb - 1) / nb;
  per = ((per + kScanTile - 1) / kScanTile) * kScanTile;
  if (per < kScanTile) per = kScanTile;
  const int used = static_cast<int>((n + per - 1) / per > 0 ? (n + per - 1) / per : 1);
  hipLaunchKernelGGL(k_scan_reduce, dim3(used), dim3(kBlock), 0, s, a, n, per, bsum);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBlock), 0, s, bsum, used);
  hipLaunchKernelGGL(k_scan_apply, dim3(used), dim3(kBlock), 0, s, a, n, per, bsum);
  return hipGetLastError();
}

hipError_t lc_launch_sweep(const LcSweepArgs& A, hipStream_t s) {
  const int G = A.grid_blocks;
  unsigned long long* st = reinterpret_cast<unsigned long long*>(A.stats);
  // optional timing marks between phases (see LcPhase)
  auto mark = [&](int ph) {
    if (A.events) (void)hipEventRecord(static_cast<hipEvent_t>(A.events[ph]), s);
  };
  mark(LC_PH_SETUP);
  const int64_t stat_words = static_cast<int64_t>(A.nchain) * ST_WORDS * (1 + kStripes);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(stat_words, 1024)), dim3(kBlock), 0, s, st, stat_words, 0ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s,
                     reinterpret_cast<unsigned long long*>(A.flags), 1, 0ull);
  // 1. count operators per window, 2. scan
  mark(LC_PH_GEN_COUNT);
  hipLaunchKernelGGL((k_gen<false>), dim3(grid_for(A.nwin, G)), dim3(kBlock), 0, s, A.descs,
                     A.win_bases, A.nchain, A.nwin, A.opstart, A.accmask, A.optime, A.optype,
                     A.op_cap, st, A.flags);
  mark(LC_PH_SCAN_OPS);
  (void)lc_launch_scan(A.opstart, A.nwin, A.scan_tmp, s);
  hipLaunchKernelGGL(k_chain_bases, dim3(grid_for(A.nchain, 64)), dim3(kBlock), 0, s, A.descs,
                     A.nchain, A.opstart, A.dyn, A.op_bases, A.node_bases, A.totals, A.op_cap,
                     A.node_cap, st, A.flags);
  // 3. write operators
  mark(LC_PH_GEN_WRITE);
  hipLaunchKernelGGL((k_gen<true>), dim3(grid_for(A.nwin, G)), dim3(kBlock), 0, s, A.descs,
                     A.win_bases, A.nchain, A.nwin, A.opstart, A.accmask, A.optime, A.optype,
                     A.op_cap, st, A.flags);
  // 4. loop graph and union-find
  mark(LC_PH_INIT_PARENT);
  hipLaunchKernelGGL(k_init_parent, dim3(G), dim3(kBlock), 0, s, A.totals, A.node_cap, A.parent);
  mark(LC_PH_LINK_OPS);
  hipLaunchKernelGGL(k_link_ops, dim3(grid_for(A.nwin, G)), dim3(kBlock), 0, s, A.descs,
                     A.win_bases, A.nchain, A.nwin, A.dyn, A.opstart, A.optime, A.parent, st,
                     A.flags);
  mark(LC_PH_LINK_SITES);
  hipLaunchKernelGGL(k_link_sites, dim3(grid_for(A.nsites, G)), dim3(kBlock), 0, s, A.descs,
                     A.site_bases, A.nchain, A.nsites, A.dyn, A.opstart, A.optime, A.parent,
                     A.flags);
  if (A.any_split)
    hipLaunchKernelGGL(k_symmetrize, dim3(grid_for(A.nspins, G)), dim3(kBlock), 0, s, A.descs,
                       A.spin_bases, A.nchain, A.nspins, A.dyn, A.parent, A.flags);
  mark(LC_PH_COMPRESS);
  const int64_t nroot_chunks = (A.node_cap + kRootChunk - 1) / kRootChunk;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(nroot_chunks + 1, 1024)), dim3(kBlock), 0, s,
                     reinterpret_cast<unsigned long long*>(A.rcnt), nroot_chunks + 1, 0ull);
  hipLaunchKernelGGL(k_compress, dim3(G), dim3(kBlock), 0, s, A.totals, A.parent,
                     reinterpret_cast<unsigned long long*>(A.rcnt), A.flags);
  // 5. flips and estimators
  mark(LC_PH_ROOTS);
  {
    const int64_t nch = nroot_chunks;
    (void)lc_launch_scan(A.rcnt, nch, A.scan_tmp, s);
    hipLaunchKernelGGL(k_roots, dim3(grid_for(nch, G)), dim3(kBlock), 0, s, A.descs, A.node_bases,
                       A.nchain, A.totals, A.parent, A.acc, A.bacc, A.root_cap, nch,
                       A.rcnt, st, A.flags);
    hipLaunchKernelGGL(k_loop_bases, dim3(grid_for(A.nchain, 64)), dim3(kBlock), 0, s,
                       A.node_bases, A.nchain, A.parent, A.loop_bases, A.flags);
  }
  mark(LC_PH_ACCUM);
  hipLaunchKernelGGL(k_accum, dim3(G), dim3(kBlock), 0, s, A.descs, A.node_bases, A.nchain, A.dyn,
                     A.totals, A.parent, A.optime, A.acc, A.bacc, A.flags);
  mark(LC_PH_CLUSTER_SUMS);
  // few resident threads: each flushes its partial sums with atomics
  hipLaunchKernelGGL(k_cluster_sums, dim3(G < 2048 ? G : 2048), dim3(kBlock), 0, s, A.loop_bases, A.nchain,
                     A.rcnt + (A.node_cap + kRootChunk - 1) / kRootChunk, A.root_cap, A.acc, st,
                     A.flags);
  mark(LC_PH_FLIP);
  hipLaunchKernelGGL(k_flip_ops, dim3(grid_for(A.nwin, G)), dim3(kBlock), 0, s, A.descs,
                     A.win_bases, A.nchain, A.nwin, A.dyn, A.opstart, A.parent, A.optype,
                     A.kflat, st, A.flags);
  hipLaunchKernelGGL(k_flip_sites, dim3(grid_for(A.nsites, G)), dim3(kBlock), 0, s, A.descs,
                     A.site_bases, A.nchain, A.nsites, A.dyn, A.parent, A.bacc, st, A.flags);
  // 6. next world lines
  mark(LC_PH_SCAN_KEPT);
  (void)lc_launch_scan(A.kflat, A.nwin, A.scan_tmp, s);
  mark(LC_PH_COMPACT);
  hipLaunchKernelGGL(k_compact, dim3(grid_for(A.nwin, G)), dim3(kBlock), 0, s, A.descs,
                     A.win_bases, A.nchain, A.nwin, A.opstart, A.optime, A.optype, A.kflat,
                     A.flags);
  hipLaunchKernelGGL(k_stats_reduce, dim3(grid_for(static_cast<int64_t>(A.nchain) * ST_WORDS, 64)),
                     dim3(kBlock), 0, s, st, A.nchain);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, A.descs, A.nchain, A.flags);
  hipLaunchKernelGGL(k_record, dim3(1), dim3(kBlock), 0, s, st,
                     static_cast<int64_t>(A.nchain) * ST_WORDS, A.flags, A.ring, A.ring_ctr,
                     A.ring_cap);
  mark(LC_PH_COUNT);
  return hipGetLastError();
}

hipError_t lc_launch_init_chain(const ChainDesc* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_init_chain, dim3(grid_for(n, 1024)), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

hipError_t lc_launch_fill_u64(void* p, int64_t n, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 1024)), dim3(kBlock), 0, s,
                     reinterpret_cast<unsigned long long*>(p), n, static_cast<unsigned long long>(v));
  return hipGetLastError();
}
