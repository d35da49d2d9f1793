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
#include "lc_uf.h"

namespace lc {

constexpr int kBlock = 256;

// Chain arrays reached through pointers held in the chain descriptors are
// in HBM; the compiler cannot know it, and would use flat memory
// instructions (which also wait on LDS traffic).  These casts say it.
#define LC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ inline const LC_GLOBAL T* gin(const T* p) {
  return (const LC_GLOBAL T*)p;
}
template <class T>
__device__ inline LC_GLOBAL T* gout(T* p) {
  return (LC_GLOBAL T*)p;
}
constexpr int kCap = 12;  // candidate times per window kept in LDS while writing; more are redrawn

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
// (S = 1/2 takes a path without integer division.)
__device__ inline int64_t bond_touching(const ChainDesc& D, int64_t x, int idx) {
  const int64_t ts = D.two_s;
  if (ts == 1) return idx == 0 ? (x == 0 ? D.L - 1 : x - 1) : x;
  const int64_t j = x / ts, a = x - j * ts;
  if (idx < ts) {
    const int64_t jl = (j == 0) ? D.L - 1 : j - 1;
    return (jl * ts + idx) * ts + a;
  }
  return (j * ts + a) * ts + (idx - ts);
}
__device__ inline int64_t bond_x(const ChainDesc& D, int64_t b) {
  return D.two_s == 1 ? b : b / D.two_s;
}
__device__ inline int64_t bond_y(const ChainDesc& D, int64_t b) {
  const int64_t ts = D.two_s;
  if (ts == 1) return b + 1 == D.L ? 0 : b + 1;
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
__device__ inline uint32_t antiparallel_mask(const ChainDesc& D, const LC_GLOBAL uint8_t* __restrict__ s0,
                                             const LC_GLOBAL int64_t* __restrict__ kstart,
                                             const LC_GLOBAL uint64_t* __restrict__ ktime, int64_t b,
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

// A uniform 64-bit draw placed in window k.
__device__ inline uint64_t in_window(const ChainDesc& D, uint64_t k, uint64_t v) {
  return D.w == 0 ? v : ((k << (64 - D.w)) | (v >> D.w));
}

// Philox call i >= 1 of window (b, k): its lower half is draw 2i-1, its
// upper half draw 2i.
__device__ inline u32x4 cand_call(const ChainDesc& D, int64_t b, uint64_t k, uint32_t i) {
  return philox10(D.seed, static_cast<uint32_t>(k), (DOM_INS << 24) | i, static_cast<uint32_t>(b),
                  D.sweep);
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

// Candidate times j0 .. j0 + m - 1 of window (b, k), j0 a multiple of
// kChunk, 1 <= m <= kChunk (unused entries 0).  Even draw 2i is the upper
// half of call i (call 0's is v0), odd draw 2i + 1 the lower half of call
// i + 1: the chunk's first draw takes a call of its own when j0 > 0, and
// then each call gives two consecutive draws.  Every entry of tc is written
// once with a constant index, so the array stays in registers.
static_assert(kChunk % 2 == 0, "chunks start at even draws");
__device__ inline void chunk_times(const ChainDesc& D, int64_t b, uint64_t k, uint64_t v0, int j0,
                                   int m, uint64_t (&tc)[kChunk]) {
  const uint32_t c0 = static_cast<uint32_t>(j0 >> 1);
  tc[0] = in_window(D, k, j0 == 0 ? v0 : hi64(cand_call(D, b, k, c0)));
#pragma unroll
  for (int p = 0; p < kChunk / 2; ++p) {
    const int j = 2 * p + 1;  // draws j0 + j (lower half) and j0 + j + 1 (upper half)
    uint64_t lo = 0, hi = 0;
    if (j < m) {
      const u32x4 r = cand_call(D, b, k, c0 + 1 + static_cast<uint32_t>(p));
      lo = in_window(D, k, lo64(r));
      hi = j + 1 < m ? in_window(D, k, hi64(r)) : 0;
    }
    tc[j] = lo;
    if (j + 1 < kChunk) tc[j + 1] = hi;
  }
}

// Exclusive scan of one value per thread over the block (three barriers).
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

// ---------------------------------------------------------------------------
// Insertion of diagonal operators and removal of old ones (steps 2-6):
// per (bond, window) the Poisson count from one 64-bit draw against the
// threshold table, the candidate times, the antiparallel test, then (WRITE)
// the merge with the kept operators into the operator list.  The counting
// pass leaves the acceptance mask of windows with at most 32 candidates in
// accmask, so the writing pass redraws only the times.
//
// A workgroup takes 256 consecutive windows at a time.  In the writing
// pass the candidate times of its windows with at most kCap candidates are
// drawn first, block-wide: the Philox calls of all of them are numbered
// through a block scan and dealt out to the threads in turn, so that every
// lane draws about the mean number of times (a lane per window would make
// its wave wait for the window with the most candidates); the times land in
// LDS, draw j of window w at slot[j][w].  The counting pass draws each
// window's times in its own lane, in chunks held in registers (measured
// faster there: it needs no LDS and no barriers).
template <bool WRITE>
__global__ __launch_bounds__(kBlock, WRITE ? 5 : 4) void k_gen(const ChainDesc* __restrict__ descs,
                                                const int64_t* __restrict__ win_bases, int nchain,
                                                int64_t nwin, int64_t* __restrict__ opstart,
                                                uint32_t* __restrict__ accmask,
                                                uint64_t* __restrict__ optime,
                                                uint8_t* __restrict__ optype, int64_t op_cap,
                                                unsigned long long* __restrict__ stats,
                                                uint32_t* __restrict__ flags, int skip_split,
                                                int64_t* __restrict__ defer) {
  constexpr int kW = WRITE ? kBlock : 1;
  __shared__ uint64_t slot[kCap * kW];
  __shared__ int cfirst[kW + 1];  // first call (block-wide numbering) of each window
  __shared__ uint8_t ncnt[kW];    // candidates of each window
  __shared__ int64_t scan[kWaves + 1];
  const int tid = threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  constexpr int kIdx[2] = {ST_CAND, ST_ACC};
  Partial<2> part;
  // block-uniform: every thread takes part in the barriers of each step
  for (int64_t i0 = xcd_block() * kBlock; i0 < nwin; i0 += stride) {
    const int64_t i = i0 + tid;
    uint32_t ncand = 0, nacc = 0;
    bool live = i < nwin;
    int c = 0, n = 0;
    int64_t b = 0;
    uint64_t k = 0, u = 0, v0 = 0;
    if (live) {
      c = chain_of(win_bases, nchain, i);
      if (!WRITE) part.at(c, stats, nchain, kIdx);
      const ChainDesc& D = descs[c];
      if (!WRITE && skip_split && D.two_s > 1) {
        live = false;  // counted by k_gen_split
      } else {
        const int64_t li = i - D.win_base;
        b = li >> D.w;
        k = static_cast<uint64_t>(li & ((int64_t(1) << D.w) - 1));
        const u32x4 r0 = philox10(D.seed, static_cast<uint32_t>(k), DOM_INS << 24,
                                  static_cast<uint32_t>(b), D.sweep);
        u = lo64(r0);
        v0 = hi64(r0);
        while (n < D.K && u >= D.T[n]) ++n;
        if (WRITE && n > 0 && n <= kCap) slot[tid] = in_window(D, k, v0);
      }
    }
    // the writing pass's candidate times of the windows with n <= kCap: draw
    // 0 is v0, draws 2i-1 and 2i are the halves of call i (i = 1 .. n/2)
    const bool inlds = WRITE && live && n <= kCap;
    if constexpr (WRITE) {
      int64_t ncall;
      const int64_t cex = block_exclusive_scan(inlds ? (n >> 1) : 0, scan, ncall);
      cfirst[tid] = static_cast<int>(cex);
      ncnt[tid] = static_cast<uint8_t>(inlds ? n : 0);
      if (tid == 0) cfirst[kBlock] = static_cast<int>(ncall);
      __syncthreads();
      for (int q = tid; q < static_cast<int>(ncall); q += kBlock) {
        int lo = 0, hi = kBlock - 1;  // the last window whose first call is at or before q
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (cfirst[mid] <= q)
            lo = mid;
          else
            hi = mid - 1;
        }
        const int64_t iw = i0 + lo;
        const ChainDesc& D = descs[chain_of(win_bases, nchain, iw)];
        const int64_t lw = iw - D.win_base;
        const int64_t bw = lw >> D.w;
        const uint64_t kw = static_cast<uint64_t>(lw & ((int64_t(1) << D.w) - 1));
        const int call = q - cfirst[lo] + 1;
        const u32x4 r = cand_call(D, bw, kw, static_cast<uint32_t>(call));
        slot[(2 * call - 1) * kBlock + lo] = in_window(D, kw, lo64(r));
        if (2 * call < ncnt[lo]) slot[2 * call * kBlock + lo] = in_window(D, kw, hi64(r));
      }
      __syncthreads();
    }
    if (live) {
      const ChainDesc& D = descs[c];
      const LC_GLOBAL uint8_t* __restrict__ s0 = gin(D.s0[D.cur]);
      const LC_GLOBAL int64_t* __restrict__ kstart = gin(D.kstart[D.cur]);
      const LC_GLOBAL uint64_t* __restrict__ ktime = gin(D.ktime[D.cur]);
      const int64_t li = i - D.win_base;
      ncand = static_cast<uint32_t>(n);
      const bool known = WRITE && n <= 32;
      // windows with kCap < n <= 32 are written by k_gen_defer, a wave per
      // window, so that no wave waits on one lane's redraws (0.1 % of the
      // windows at the largest mean count, 4)
      const bool deferred = known && !inlds;
      uint64_t accm = known ? accmask[i] : 0;
      if (!known) {
        for (int j0 = 0; j0 < n; j0 += kChunk) {
          const int m = (n - j0 < kChunk) ? n - j0 : kChunk;
          uint64_t tc[kChunk];
          if (inlds) {
#pragma unroll
            for (int j = 0; j < kChunk; ++j) tc[j] = j < m ? slot[(j0 + j) * kBlock + tid] : 0;
          } else {
            chunk_times(D, b, k, v0, j0, m, tc);
          }
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
        } else if (deferred) {
          const unsigned long long at =
              atomicAdd(reinterpret_cast<unsigned long long*>(defer + nwin), 1ull);
          defer[at] = i;
        } else if (inlds) {
          // accepted candidates in draw order, then a stable insertion sort
          // (equal times keep draw order), then one merge with the kept
          // operators (a kept operator first at equal times)
          int na = 0;
          for (int j = 0; j < n; ++j)
            if ((accm >> j) & 1) slot[(na++) * kBlock + tid] = slot[j * kBlock + tid];
          for (int a1 = 1; a1 < na; ++a1) {
            const uint64_t t = slot[a1 * kBlock + tid];
            int a2 = a1 - 1;
            while (a2 >= 0 && slot[a2 * kBlock + tid] > t) {
              slot[(a2 + 1) * kBlock + tid] = slot[a2 * kBlock + tid];
              --a2;
            }
            slot[(a2 + 1) * kBlock + tid] = t;
          }
          int64_t o = base, q = kb;
          int ia = 0;
          uint64_t tk = q < ke ? ktime[q] : 0;
          while (ia < na || q < ke) {
            const uint64_t ta = ia < na ? slot[ia * kBlock + tid] : 0;
            if (q < ke && (ia >= na || tk <= ta)) {
              optime[o] = tk;
              optype[o] = 3;
              ++q;
              tk = q < ke ? ktime[q] : 0;
            } else {
              optime[o] = ta;
              optype[o] = 0;
              ++ia;
            }
            ++o;
          }
        } else {
          // more than 32 candidates: every time is redrawn where needed;
          // accepted candidates: rank among accepted + kept at or before
          for (int j = 0; j < n; ++j) {
            if (!((accm >> j) & 1)) continue;
            const uint64_t t = cand_time(D, b, k, j, v0);
            int64_t rank = 0;
            for (int j2 = 0; j2 < n; ++j2) {
              if (!((accm >> j2) & 1) || j2 == j) continue;
              const uint64_t t2 = cand_time(D, b, k, j2, v0);
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
              if ((accm >> j) & 1) rank += (cand_time(D, b, k, j, v0) < t) ? 1 : 0;
            optime[base + rank] = t;
            optype[base + rank] = 3;
          }
        }
      }
    }
    part.v[0] += ncand;
    part.v[1] += nacc;
    if constexpr (WRITE) __syncthreads();  // slot and cfirst are rewritten by the next step
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


// One bit per id of the 128-bit Philox blocks of a domain: bit (id mod 128)
// of block id / 128 of this sweep.  The loop-flip bit of a chain-local label
// (domain FLIP), or the vote of a chain-local node (domain VOTE: a loop
// flips iff the XOR of its nodes' votes is 1, the majority-vote trick of
// Sec. 3.3, independent of the order of the unions).
__device__ inline uint32_t domain_bit(const ChainDesc& D, int64_t id, uint32_t dom) {
  const uint64_t q = static_cast<uint64_t>(id) >> 7;
  const uint32_t i = static_cast<uint32_t>(id & 127);
  const u32x4 r = philox10(D.seed, static_cast<uint32_t>(q),
                           (dom << 24) | static_cast<uint32_t>((q >> 32) & 0xFFFFFFu), 0u,
                           D.sweep);
  const uint32_t wsel = i >> 5;
  const uint32_t word = wsel == 0 ? r.x : (wsel == 1 ? r.y : (wsel == 2 ? r.z : r.w));
  return (word >> (i & 31)) & 1u;
}
__device__ inline uint32_t flip_bit(const ChainDesc& D, int64_t label) {
  return domain_bit(D, label, DOM_FLIP);
}
__device__ inline uint32_t vote_bit(const ChainDesc& D, int64_t node) {
  return domain_bit(D, node, DOM_VOTE);
}

constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;


// The writing pass of the windows k_gen deferred (kCap < n <= 32
// candidates): one wave per window, one lane per candidate.  Each lane draws
// its candidate's time once; an accepted candidate's place is the number of
// accepted ones before it (earlier time, or equal time and earlier draw)
// plus the kept operators at or before its time; a kept operator's place is
// its index plus the accepted candidates strictly before it -- the order
// k_gen writes (a kept operator first at equal times).
__global__ __launch_bounds__(kBlock) void k_gen_defer(const ChainDesc* __restrict__ descs,
                                                      const int64_t* __restrict__ win_bases,
                                                      int nchain, int64_t nwin,
                                                      const int64_t* __restrict__ opstart,
                                                      const uint32_t* __restrict__ accmask,
                                                      uint64_t* __restrict__ optime,
                                                      uint8_t* __restrict__ optype,
                                                      const int64_t* __restrict__ defer) {
  const int lane = lane_id();
  const int64_t nd = defer[nwin];
  const int64_t nwave = static_cast<int64_t>(gridDim.x) * kWaves;
  for (int64_t d = xcd_block() * kWaves + (threadIdx.x >> 6); d < nd; d += nwave) {
    const int64_t i = defer[d];
    const int c = chain_of(win_bases, nchain, i);
    const ChainDesc& D = descs[c];
    const LC_GLOBAL int64_t* __restrict__ kstart = gin(D.kstart[D.cur]);
    const LC_GLOBAL uint64_t* __restrict__ ktime = gin(D.ktime[D.cur]);
    const int64_t li = i - D.win_base;
    const int64_t b = li >> D.w;
    const uint64_t k = static_cast<uint64_t>(li & ((int64_t(1) << D.w) - 1));
    const u32x4 r0 = philox10(D.seed, static_cast<uint32_t>(k), DOM_INS << 24,
                              static_cast<uint32_t>(b), D.sweep);
    const uint64_t u = lo64(r0), v0 = hi64(r0);
    int n = 0;
    while (n < D.K && u >= D.T[n]) ++n;  // kCap < n <= 32: k_gen deferred it
    const uint32_t accm = accmask[i];
    const uint64_t t = lane < n ? cand_time(D, b, k, lane, v0) : 0;
    const bool acc = lane < n && ((accm >> lane) & 1u);
    const int64_t kb = kstart[li], ke = kstart[li + 1], base = opstart[i];
    int64_t rank = 0;
    for (int l = 0; l < n; ++l) {  // wave-uniform trip count
      const uint64_t t2 = __shfl(t, l);
      const bool a2 = (accm >> l) & 1u;
      rank += (a2 && l != lane && (t2 < t || (t2 == t && l < lane))) ? 1 : 0;
    }
    if (acc) {
      for (int64_t q = kb; q < ke; ++q) rank += ktime[q] <= t ? 1 : 0;
      optime[base + rank] = t;
      optype[base + rank] = 0;
    }
    for (int64_t q0 = kb; q0 < ke; q0 += 64) {  // kept operators, 64 at a time
      const int64_t q = q0 + lane;
      const uint64_t tk = q < ke ? ktime[q] : 0;
      int64_t rk = q - kb;
      for (int l = 0; l < n; ++l) {
        const uint64_t t2 = __shfl(t, l);
        rk += (((accm >> l) & 1u) && t2 < tk) ? 1 : 0;
      }
      if (q < ke) {
        optime[base + rk] = tk;
        optype[base + rk] = 3;
      }
    }
  }
}

// Counting pass of split-spin chains, by tiles.  The antiparallel test of a
// candidate on bond b = (x, y) needs the spins of subspins x and y at its
// time, and a subspin's spin flips at every kept operator on the 2 (2S)
// bonds touching it.  Per window, the kept operators on those bonds are
// gathered once per subspin into an LDS list (time and bond of each), with
// the subspin's spin at the window's start; every bond then tests its
// candidates against the two lists of its ends instead of reading
// 2 (2 (2S) - 1) bonds' windows from HBM.  Bond b's own operators are in
// both lists and cancel, as they do in the XOR of the two spins.
//
// A tile is gj spins x gk windows of one chain, one thread per bond-window
// (gj (2S)^2 gk <= 256).  Its lists are those of the subspins of spins
// j0 .. j0 + gj (the last one holds right ends only), filled from the bonds
// of spins j0 - 1 .. j0 + gj (modulo L).  A tile whose lists exceed the LDS
// tests its windows one by one as k_gen does.  The result is the same
// integers as k_gen's counting pass: counts, acceptance masks, statistics.
constexpr int kGenLists = 256;   // subspin-window lists of a tile
constexpr int kGenEnt = 2560;    // list entries (each kept operator in up to two lists)
constexpr int kGenChains = 512;  // chains of one launch (tile bases in LDS)

__host__ __device__ inline int gen_gk(int ts, int64_t W) {
  int gk = 8;
  while (gk > 1 && (gk > W || ts * ts * gk > kBlock)) gk >>= 1;
  return gk;
}
__host__ __device__ inline int gen_gj(int ts, int gk) { return kBlock / (ts * ts * gk); }

__global__ __launch_bounds__(kBlock) void k_gen_split(const ChainDesc* __restrict__ descs,
                                                      const int* __restrict__ grp_chain, int ngrp,
                                                      int nchain, int64_t* __restrict__ opstart,
                                                      uint32_t* __restrict__ accmask,
                                                      unsigned long long* __restrict__ stats) {
  __shared__ int64_t gbase[kGenChains + 1];  // first tile of each chain of the launch
  __shared__ int lcnt[kGenLists], loff[kGenLists], lcur[kGenLists];
  __shared__ uint32_t lpar[kGenLists];       // spin of the list's subspin at its window's start
  __shared__ uint64_t et[kGenEnt];           // list entries: time
  __shared__ uint16_t eb[kGenEnt];           //               bond, as its index q / nk below
  __shared__ int64_t scan[kWaves + 1];
  const int tid = threadIdx.x;
  constexpr int kIdx[2] = {ST_CAND, ST_ACC};
  Partial<2> part;
  if (ngrp > kGenChains) return;  // the host launches within the bound
  {
    int64_t total = 0;
    for (int base = 0; base < ngrp; base += kBlock) {
      int64_t cnt = 0;
      if (base + tid < ngrp) {
        const ChainDesc& D = descs[grp_chain[base + tid]];
        const int64_t W = int64_t(1) << D.w;
        const int gk = gen_gk(D.two_s, W), gj = gen_gj(D.two_s, gk);
        cnt = ((D.L + gj - 1) / gj) * (W / gk);
      }
      int64_t t2;
      const int64_t ex = block_exclusive_scan(cnt, scan, t2);
      if (base + tid < ngrp) gbase[base + tid] = total + ex;
      total += t2;
    }
    if (tid == 0) gbase[ngrp] = total;
    __syncthreads();
  }
  const int64_t ntiles = gbase[ngrp];
  for (int64_t t = xcd_block(); t < ntiles; t += gridDim.x) {
    int lo = 0, hi = ngrp - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (gbase[mid] <= t)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int c = grp_chain[lo];
    part.at(c, stats, nchain, kIdx);
    const ChainDesc& D = descs[c];
    const LC_GLOBAL uint8_t* __restrict__ s0 = gin(D.s0[D.cur]);
    const LC_GLOBAL int64_t* __restrict__ kstart = gin(D.kstart[D.cur]);
    const LC_GLOBAL uint64_t* __restrict__ ktime = gin(D.ktime[D.cur]);
    const int ts = static_cast<int>(D.two_s), ts2 = ts * ts;
    const int64_t L = D.L, W = int64_t(1) << D.w;
    const int gk = gen_gk(ts, W), gj = gen_gj(ts, gk);
    const int64_t ntk = W / gk;  // tiles window-major: neighbours in time share cache lines
    const int64_t lt = t - gbase[lo];
    const int64_t j0 = (lt / ntk) * gj, k0 = (lt % ntk) * gk;
    const int nj = static_cast<int>(min(static_cast<int64_t>(gj), L - j0));
    const int nk = gk, lognk = __ffs(gk) - 1;  // gk is a power of two
    // spin j0 + d modulo L for -1 <= d < 2 L (no 64-bit division in the loops)
    auto spin_at = [&](int64_t d) -> int64_t {
      int64_t j = j0 + d;
      if (j < 0) j += L;
      if (j >= L) j -= L;
      return j;
    };
    const int nls = static_cast<int>(min(static_cast<int64_t>(nj + 1), L));  // spins with lists
    const int nbs = static_cast<int>(min(static_cast<int64_t>(nj + 2), L));  // spins with bonds read
    const int nlists = nls * ts * nk;  // <= kGenLists whenever gj (2S)^2 gk <= 256, 2S >= 2
    const int nq = nbs * ts2 * nk;
    const bool fit = nlists <= kGenLists;  // block-uniform
    // list of subspin (spin j0 + v, a) in window k0 + kk: (v ts + a) nk + kk
    for (int l = tid; fit && l < nlists; l += kBlock) {
      const int va = l >> lognk, v = va / ts, a = va - v * ts;
      lcnt[l] = 0;
      lpar[l] = s0[spin_at(v) * ts + a];
    }
    __syncthreads();
    // the bond-window q of the spins read: bond bl of spin j0 - 1 + u, window k0 + kk
    // (spin index u, bond bl) of a list entry, kept as u ts2 + bl
    auto ent_bond = [&](uint32_t id) -> int64_t {
      const int u = static_cast<int>(id) / ts2;
      return spin_at(u - 1) * ts2 + (static_cast<int>(id) - u * ts2);
    };
    auto bond_q = [&](int q, int64_t* bb, int* ll, int* lr, int* kk) {
      const int ub = q >> lognk, u = ub / ts2, bl = ub - u * ts2;
      *kk = q & (nk - 1);
      *bb = spin_at(u - 1) * ts2 + bl;
      // list slots of the bond's ends: spin j0 - 1 + u is slot u - 1 (mod L)
      int vl = u - 1, vr = u;
      if (vl < 0) vl += static_cast<int>(L);
      if (vr == L) vr = 0;
      const int a = bl / ts, c = bl - a * ts;
      *ll = vl < nls ? ((vl * ts + a) << lognk) + *kk : -1;
      *lr = vr < nls ? ((vr * ts + c) << lognk) + *kk : -1;
    };
    for (int q = tid; fit && q < nq; q += kBlock) {
      int64_t bb;
      int ll, lr, kk;
      bond_q(q, &bb, &ll, &lr, &kk);
      const int64_t i0 = bb * W;
      const int64_t ka = kstart[i0 + k0 + kk], kb = kstart[i0 + k0 + kk + 1];
      const int cnt = static_cast<int>(kb - ka);
      const uint32_t par = static_cast<uint32_t>((ka - kstart[i0]) & 1);
      if (ll >= 0) {
        atomicAdd(lcnt + ll, cnt);
        if (par) atomicXor(lpar + ll, 1u);
      }
      if (lr >= 0) {
        atomicAdd(lcnt + lr, cnt);
        if (par) atomicXor(lpar + lr, 1u);
      }
    }
    __syncthreads();
    int64_t nent;
    {
      const int64_t v = fit && tid < nlists ? lcnt[tid] : 0;
      const int64_t ex = block_exclusive_scan(v, scan, nent);
      if (fit && tid < nlists) loff[tid] = lcur[tid] = static_cast<int>(ex);
    }
    const bool lists = fit && nent <= kGenEnt;  // block-uniform
    __syncthreads();
    if (lists) {
      for (int q = tid; q < nq; q += kBlock) {
        int64_t bb;
        int ll, lr, kk;
        bond_q(q, &bb, &ll, &lr, &kk);
        const int64_t i0 = bb * W;
        const int64_t ka = kstart[i0 + k0 + kk], kb = kstart[i0 + k0 + kk + 1];
        for (int64_t p = ka; p < kb; ++p) {
          const uint64_t tp = ktime[p];
          const uint16_t id = static_cast<uint16_t>(q >> lognk);
          if (ll >= 0) {
            const int e = atomicAdd(lcur + ll, 1);
            et[e] = tp;
            eb[e] = id;
          }
          if (lr >= 0) {
            const int e = atomicAdd(lcur + lr, 1);
            et[e] = tp;
            eb[e] = id;
          }
        }
      }
    }
    __syncthreads();
    uint32_t ncand = 0, nacc = 0;
    if (tid < nj * ts2 * nk) {
      const int lb = tid >> lognk, kk = tid & (nk - 1);
      const int64_t b = j0 * ts2 + lb;
      const uint64_t k = static_cast<uint64_t>(k0 + kk);
      const int64_t li = b * W + static_cast<int64_t>(k);
      const u32x4 r0 = philox10(D.seed, static_cast<uint32_t>(k), DOM_INS << 24,
                                static_cast<uint32_t>(b), D.sweep);
      const uint64_t u = lo64(r0), v0 = hi64(r0);
      int n = 0;
      while (n < D.K && u >= D.T[n]) ++n;
      ncand = static_cast<uint32_t>(n);
      // the lists of the two ends: x = (j0 + lb / ts2, a), y = (next spin, c)
      const int vx = lb / ts2, ac = lb - vx * ts2, a = ac / ts, cy = ac - a * ts;
      const int vy = vx + 1 == L ? 0 : vx + 1;
      const int lx = ((vx * ts + a) << lognk) + kk, ly = ((vy * ts + cy) << lognk) + kk;
      uint64_t accm = 0;
      for (int c0 = 0; c0 < n; c0 += kChunk) {
        const int m = (n - c0 < kChunk) ? n - c0 : kChunk;
        uint64_t tc[kChunk];
        chunk_times(D, b, k, v0, c0, m, tc);
        uint32_t mask;
        if (lists) {
          uint32_t base = lpar[lx] ^ lpar[ly], flips = 0, ties = 0;
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int l = side ? ly : lx;
            for (int e = loff[l]; e < loff[l] + lcnt[l]; ++e) {
              const uint64_t tp = et[e];
#pragma unroll
              for (int j = 0; j < kChunk; ++j) {
                flips ^= (tp < tc[j] ? 1u : 0u) << j;
                ties |= (tp == tc[j] ? 1u : 0u) << j;
              }
            }
          }
          // a kept operator at exactly a candidate's time precedes it when
          // its bond is the smaller one (never met in practice: 64-bit times)
          if (ties & ((1u << m) - 1u)) {
            for (int side = 0; side < 2; ++side) {
              const int l = side ? ly : lx;
              for (int e = loff[l]; e < loff[l] + lcnt[l]; ++e)
                for (int j = 0; j < m; ++j)
                  if (et[e] == tc[j] && ent_bond(eb[e]) < b) flips ^= 1u << j;
            }
          }
          const uint32_t live = (1u << m) - 1u;
          mask = ((base & 1u) ? ~flips : flips) & live;
        } else {
          mask = antiparallel_mask(D, s0, kstart, ktime, b, k, tc, m);
        }
        accm |= static_cast<uint64_t>(mask) << c0;
      }
      nacc = static_cast<uint32_t>(__popcll(accm));
      const int64_t i = D.win_base + li;
      opstart[i] = (kstart[li + 1] - kstart[li]) + nacc;
      accmask[i] = static_cast<uint32_t>(accm);
    }
    part.v[0] += ncand;
    part.v[1] += nacc;
    __syncthreads();  // the LDS is reused by the next tile
  }
  part.flush(stats, nchain, kIdx);
}

// Boundary nodes start as their own roots (operator nodes get their parent
// words from the linking tiles).
__global__ __launch_bounds__(kBlock) void k_init_bnodes(const int64_t* __restrict__ bn_bases,
                                                         int nchain, int64_t nbn,
                                                         const ChainDyn* __restrict__ dyn,
                                                         int64_t* __restrict__ parent,
                                                         const uint32_t* __restrict__ flags) {
  if (*flags) return;
  for (int64_t i = xcd_block() * kBlock + threadIdx.x; i < nbn;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int c = chain_of(bn_bases, nchain, i);
    const int64_t g = dyn[c].node_base + (i - bn_bases[c]);
    parent[g] = g;
  }
}

// Loop length >> 32 from its per-loop sums: length = 2^64 tops
// + 2 (2^32 shi + slo), with shi and slo the sums of +-hi32(t) and +-lo32(t)
// over its operator nodes (lower nodes +t, upper nodes -t: each node ends or
// starts two vertical segments) read as signed words; length < 2^96.
__device__ inline uint64_t loop_len32(uint64_t tops, uint64_t shi_w, uint64_t slo_w) {
  const int64_t shi = static_cast<int64_t>(shi_w), slo = static_cast<int64_t>(slo_w);
  uint64_t llo = static_cast<uint64_t>(slo) << 1;
  uint64_t lhi = static_cast<uint64_t>(slo >> 63);        // sign extension of 2 slo
  const uint64_t hlo = static_cast<uint64_t>(shi) << 33;
  const uint64_t hhi = static_cast<uint64_t>(shi >> 31);  // arithmetic: bits 31.. of shi
  const uint64_t t1 = llo + hlo;
  lhi = lhi + hhi + (t1 < llo ? 1u : 0u) + tops;
  llo = t1;
  return (llo >> 32) | (lhi << 32);
}

// Per-thread sums of the loops a thread finishes (flushed per lane when the
// thread moves to another chain, per block at the end).
struct LoopSums {
  int c = -1;
  uint64_t n = 0, s2lo = 0, s2hi = 0, l2lo = 0, l2hi = 0, mx = 0;
  __device__ void flush_lane(unsigned long long* stats, int nchain) {
    if (c < 0) return;  // stat_apply skips zero words
    stat_apply(stats, nchain, c, ST_CLUSTERS, -1, FLUSH_ADD, n, 0);
    stat_apply(stats, nchain, c, ST_SIZE2_LO, ST_SIZE2_HI, FLUSH_ADD, s2lo, s2hi);
    stat_apply(stats, nchain, c, ST_LEN2_LO, ST_LEN2_HI, FLUSH_ADD, l2lo, l2hi);
    stat_apply(stats, nchain, c, ST_MAXSIZE, -1, FLUSH_MAX, mx, 0);
    n = s2lo = s2hi = l2lo = l2hi = mx = 0;
  }
  __device__ void at(int cn, unsigned long long* stats, int nchain) {
    if (cn == c) return;
    flush_lane(stats, nchain);
    c = cn;
  }
  // count = false: the loop was counted elsewhere (its root was numbered)
  __device__ void add(uint64_t size, uint64_t len32, bool count = true) {
    n += count ? 1 : 0;
    const u128p a = mul64x64(size, size);
    s2lo += a.lo;
    s2hi += a.hi + (s2lo < a.lo ? 1u : 0u);
    const u128p b = mul64x64(len32, len32);
    l2lo += b.lo;
    l2hi += b.hi + (l2lo < b.lo ? 1u : 0u);
    mx = size > mx ? size : mx;
  }
  // convergent: every thread of the block must call it
  __device__ void flush(unsigned long long* stats, int nchain) {
    block_flush(stats, nchain, c, ST_CLUSTERS, -1, FLUSH_ADD, n, 0);
    block_flush(stats, nchain, c, ST_SIZE2_LO, ST_SIZE2_HI, FLUSH_ADD, s2lo, s2hi);
    block_flush(stats, nchain, c, ST_LEN2_LO, ST_LEN2_HI, FLUSH_ADD, l2lo, l2hi);
    block_flush(stats, nchain, c, ST_MAXSIZE, -1, FLUSH_MAX, mx, 0);
  }
};

// ---------------------------------------------------------------------------
// Leg linking and union-find by tiles (Sec. 2: loops as trees of world-line
// fragments; Sec. 3.1: union-find inside a domain first, then a merge of the
// fragments that leave it).  A tile is a range of spins times a range of
// time windows of one chain.  It owns the operators on the bonds that start
// at its spins (bond ((2S j) + a) 2S + c belongs to spin j) in its windows:
// at most LC_TILE_OPS operators, whose two nodes each get a 32-bit local
// index in LDS (lower 2l, upper 2l + 1 for local operator l, bond-major).
//
// Each thread walks one (subspin, window) of the tile: a merge of the
// time-ordered operator lists of the 2 2S bonds touching the subspin, in
// (time, bond) order, gives the events on the subspin; consecutive events
// are joined upper -> lower, the first event of the subspin to its bottom
// boundary node and the last one to its top node (the walker whose window
// holds that event emits the edge, so every edge is emitted once).  An edge
// whose two ends are local nodes is a local union in LDS; any other edge is
// staged as a cross edge for the global union-find.
//
// After the local unions, the tile knows for every local component its
// smallest node (rep), its size, and whether it is open (a node with fewer
// than two local edges: the loop continues outside the tile).  A closed
// component is a whole loop: the tile finishes it -- loop count, size^2,
// length^2 into the chain statistics, and every node of it gets a code
// naming its rep and the loop's flip decision (the bit of its label, or the
// XOR of its nodes' votes under the vote rule) -- without
// any global work (closed two-node loops directly from the two times, larger
// ones through an LDS accumulator slot).  An open component is a fragment:
// its rep, size and length sums go to the fragment list, which is all the
// later phases see of it.  Every node's parent word is written once,
// coalesced: its rep in an open component (the rep points to itself), the
// finished loop's code in a closed one.
constexpr int kTileBonds = LC_TILE_BONDS;
static_assert(LC_TILE_THREADS == kBlock, "one (subspin, window) walker per thread");
static_assert(kTileBonds <= 256, "owned bonds are numbered in one byte");

// LDS capacities of a tile, per spin length.  S = 1/2 tiles hold up to
// LC_TILE_OPS operators; split-spin tiles hold fewer but, being narrow (2S
// bonds of each subspin cross a tile side), more edges leaving the tile and
// more components.
template <int TS>
struct TileCfg {
  static constexpr int kOps = TS == 1 ? LC_TILE_OPS : LC_TILE_OPS_SPLIT;
  static constexpr int kNodes = 2 * kOps;
  static constexpr int kCross = TS == 1 ? 384 : 1024;
  static constexpr int kSlots = TS == 1 ? 256 : 768;
};

// After the local compression the word of a non-rep node is its rep; the
// word of a rep holds the component's fields:
constexpr uint32_t kRepFlag = 1u << 31;   // this node is its component's rep
constexpr uint32_t kRepOpen = 1u << 30;   // the component leaves the tile
constexpr uint32_t kRepFlip = 1u << 29;   // flip decision of a closed component
constexpr uint32_t kRepSize = 0x1FFFu;    // bits 0..12: nodes of the component
constexpr int kRepSlotShift = 13;         // bits 13..22: accumulator slot + 1
constexpr uint32_t kRepSlotMask = 0x3FFu;

// Per-subspin event lists of a split-spin tile's walk (tile_walk_lists),
// held in the LDS of the accumulator slots, which are not in use until the
// walk is over.  A run is the operators of one (walker, bond slot): one
// bond's window.  S = 1/2 tiles walk serially and keep these minimal.
template <int TS>
struct TileLists {
  static constexpr int kRuns = TS == 1 ? 1 : 512;    // walkers x 2 (2S) bond slots
  static constexpr int kItems = TS == 1 ? 1 : 3584;  // events of all walkers
  int64_t rstart[kRuns];     // first flat operator of each run
  int64_t wnxt[kBlock];      // first event after each walker's window (flat), or -1
  uint16_t wlist[kItems];    // each walker's events in (time, bond) order, as their index
                             // in the walker's runs taken one after another
  uint16_t rlen[kRuns];      // operators of each run
  uint16_t roff[kRuns];      // first event of each run in its walker's concatenated runs
  int16_t rloc[kRuns];       // local index of the run's first operator, -1 if not owned
  uint16_t woff[kBlock + 1]; // first list entry of each walker
  int16_t wnl[kBlock];       // local index of wnxt, or -1
  uint8_t wflag[kBlock];     // bit 0: events before the window; bit 1: no event at all
  uint64_t rnt[kRuns];       // time of the bond's first operator after the window (rflag bit 2)
  uint16_t rtix[kRuns];      // the run's times: ltime[rtix + p] (staged when not owned)
  uint8_t rflag[kRuns];      // bit 0: operators before the window; bit 1: none on the bond;
                             // bit 2: an operator after the window
  int xcur;                  // staging cursor in ltime, after the tile's own operators
};

// Edges leaving the tile, staged during the walk and written out right
// after it.  S = 1/2 tiles keep them in the LDS of the accumulator slots,
// which come into use only later: that keeps four of their workgroups on a
// CU.  Split-spin tiles walk through lists held in those slots, so their
// staged edges have LDS of their own.
template <int TS>
struct TileCross {
  int64_t xsrc[TileCfg<TS>::kCross], xdst[TileCfg<TS>::kCross];
};
struct TileNone {};

template <int TS>
struct TileLds {
  using C = TileCfg<TS>;
  static_assert(C::kNodes <= static_cast<int>(kRepSize), "component size field");
  static_assert(C::kSlots < static_cast<int>(kRepSlotMask), "slot field");
  static_assert(C::kNodes / 2 <= 2 * C::kOps, "closed-component list fits the times' LDS");
  uint32_t lpar[C::kNodes];          // local forest, then reps and their fields
  // split spins: 2-bit counts of the edges of each node inside the tile;
  // S = 1/2: one bit per node, set when the node has an edge leaving the
  // tile (open_mark)
  static constexpr bool kOpenBits = TS == 1;
  uint32_t deg[C::kNodes / 16];
  uint64_t ltime[C::kOps];           // times of the tile's operators
  uint8_t lbond[C::kOps];            // owned bond (local index) of each tile operator
  union {
    struct {
      int64_t slot_hi[C::kSlots], slot_lo[C::kSlots];
      uint32_t slot_rep[C::kSlots];
      uint32_t slot_vote[C::kSlots];  // XOR of the votes of a slotted component
    };
    TileLists<TS> wl;                 // the walk's event lists (split spins)
    std::conditional_t<TS == 1, TileCross<TS>, TileNone> xin;  // staged edges (S = 1/2)
  };
  std::conditional_t<TS == 1, TileNone, TileCross<TS>> xout;   // staged edges (split spins)
  __device__ TileCross<TS>& cross() {
    if constexpr (TS == 1)
      return xin;
    else
      return xout;
  }
  uint32_t tpre[kTileBonds + 1];     // first local operator of each owned bond
  int64_t tos[kTileBonds];           // first (flat) operator of each owned bond in the tile
  int64_t scan[kWaves + 1];
  int64_t base[2];                   // reserved positions: cross edges, fragments
  int cnt[4];                        // staged cross edges, slots, open slots, fragment cursor
  int ncl;                           // closed components whose flip decision is drawn last
  uint32_t fl;
  int64_t sflat;                     // S = 1/2: first operator of the bond left of the tile in
  int sn;                            // its windows, and how many follow it (times in ltime
                                     // after the tile's own; 0 when owned or not staged)
};
static_assert(sizeof(TileLds<1>) <= 40 * 1024, "four S = 1/2 linking workgroups per CU");
static_assert(sizeof(TileLds<8>) <= 80 * 1024, "two split-spin linking workgroups per CU");

// Time of flat operator e whose tile-local index is li (-1: not the tile's):
// from LDS or from HBM.  The LDS read is an atomic load so that the two
// reads stay loads of their own address spaces (a select between an LDS
// and a global address would become one flat memory instruction).
__device__ inline uint64_t op_time(const uint64_t* ltime, int li, const uint64_t* __restrict__ optime,
                                   int64_t e) {
  if (li >= 0) return __hip_atomic_load(ltime + li, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return optime[e];
}

// Local operator index of flat operator e on bond bb, or -1 if the tile does
// not own it.
template <class Lds>
__device__ inline int tile_local(const Lds& S, int64_t B0, int nbt, int64_t bb, int64_t e) {
  const int64_t lb = bb - B0;
  if (lb < 0 || lb >= nbt) return -1;
  const int64_t off = e - S.tos[lb];
  if (off < 0 || off >= static_cast<int64_t>(S.tpre[lb + 1] - S.tpre[lb])) return -1;
  return static_cast<int>(S.tpre[lb] + off);
}

// Flat operator of local operator lo.
template <class Lds>
__device__ inline int64_t tile_op(const Lds& S, uint32_t lo) {
  const uint32_t lb = S.lbond[lo];
  return S.tos[lb] + static_cast<int64_t>(lo - S.tpre[lb]);
}

// An edge between nodes (gu, gv); lu, lv their local indices or -1.
// S = 1/2 tiles: local node u has an edge that leaves the tile.
template <class Lds>
__device__ inline void open_mark(Lds& S, int u) {
  atomicOr(S.deg + (u >> 5), 1u << (u & 31));
}

template <class Lds>
__device__ inline void tile_edge(Lds& S, int64_t gu, int lu, int64_t gv, int lv) {
  if (lu >= 0 && lv >= 0) {
    if constexpr (!Lds::kOpenBits) {
      atomicAdd(S.deg + (lu >> 4), 1u << ((lu & 15) * 2));
      atomicAdd(S.deg + (lv >> 4), 1u << ((lv & 15) * 2));
    }
    lunion(S.lpar, static_cast<uint32_t>(lu), static_cast<uint32_t>(lv));
  } else {
    if constexpr (Lds::kOpenBits) {
      if (lu >= 0) open_mark(S, lu);
      if (lv >= 0) open_mark(S, lv);
    }
    const int s = atomicAdd(&S.cnt[0], 1);
    if (s < Lds::C::kCross) {
      S.cross().xsrc[s] = gu;
      S.cross().xdst[s] = gv;
    }
  }
}

// The walker of spin x in window k of an S = 1/2 tile (see above): a merge
// of the two time-ordered runs of bonds x - 1 and x in window k.  nb0: node
// id of the lower node of flat operator 0 of the chain's numbering (lower(e)
// = nb0 + 2e).  Every time it reads is in LDS -- the tile's own operators,
// and those of the bond left of the tile in the tile's windows, staged
// after them (S.sflat, S.sn) -- except the first operator after the window
// when that lies beyond the tile.  Its global loads are issued in two
// batches before the walk, so that no wave waits on memory inside the loop.
__device__ inline void tile_walk_half(TileLds<1>& S, const ChainDesc& D, int64_t x, int64_t k,
                                      int64_t nb0, int64_t node_base, int64_t B0, int nbt, int nlo,
                                      const int64_t* __restrict__ opstart,
                                      const uint64_t* __restrict__ optime) {
  const int64_t W = int64_t(1) << D.w;
  const int64_t jl = (x == 0) ? D.L - 1 : x - 1;
  const int64_t bnd[2] = {jl, x};
  // LDS index of the time of flat operator idx on bond s, or -1
  auto tix = [&](int s, int64_t idx) -> int {
    const int64_t lb = bnd[s] - B0;
    if (lb >= 0 && lb < nbt) {
      const int64_t off = idx - S.tos[lb];
      return (off >= 0 && off < static_cast<int64_t>(S.tpre[lb + 1] - S.tpre[lb]))
                 ? static_cast<int>(S.tpre[lb] + off)
                 : -1;
    }
    const int64_t off = idx - S.sflat;
    return (off >= 0 && off < S.sn) ? nlo + static_cast<int>(off) : -1;
  };
  int64_t h[2], e[2], end[2];
  int hl[2], ht[2];  // node-local index of the head (owned bonds, else -1); its time's LDS index
  uint64_t th[2], tn[2];
  bool before = false, any = false, has_next[2];
  // first batch: the window's run, the bond's first and last operator
  int64_t first[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int64_t i0 = D.win_base + bnd[s] * W;
    h[s] = opstart[i0 + k];
    e[s] = opstart[i0 + k + 1];
    first[s] = opstart[i0];
    end[s] = opstart[i0 + W];
  }
  // second batch: the heads' times and the times of the first operators after
  // the window
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    before = before || first[s] < h[s];
    any = any || h[s] < e[s];
    const int64_t lb = bnd[s] - B0;
    hl[s] = (lb >= 0 && lb < nbt) ? static_cast<int>(S.tpre[lb] + (h[s] - S.tos[lb])) : -1;
    ht[s] = h[s] < e[s] ? tix(s, h[s]) : -1;
    th[s] = h[s] < e[s] ? op_time(S.ltime, ht[s], optime, h[s]) : 0;
    has_next[s] = e[s] < end[s];
    tn[s] = has_next[s] ? op_time(S.ltime, tix(s, e[s]), optime, e[s]) : 0;
  }
  if (!any) return;
  // the first event's predecessor lies before the tile's first window when
  // neither bond has an operator in the tile's windows before this one: its
  // edge is another tile's, and the first event's lower node is open
  bool ext = before;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int64_t lb = bnd[s] - B0;
    ext = ext && h[s] == ((lb >= 0 && lb < nbt) ? S.tos[lb] : S.sflat);
  }
  int64_t prev = -1;
  int lprev = -1;
  for (;;) {
    int sm = -1, lcur = -1, tcur = -1;
    uint64_t tm = 0;
    int64_t bm = 0, cur = 0, em = 0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (h[s] < e[s] && (sm < 0 || th[s] < tm || (th[s] == tm && bnd[s] < bm))) {
        sm = s;
        tm = th[s];
        bm = bnd[s];
        cur = h[s];
        em = e[s];
        lcur = hl[s];
        tcur = ht[s];
      }
    }
    if (sm < 0) break;
    const int64_t gl = nb0 + 2 * cur;
    if (prev < 0) {
      if (!before)
        tile_edge(S, node_base + x, -1, gl, lcur >= 0 ? 2 * lcur : -1);
      else if (ext && lcur >= 0)
        open_mark(S, 2 * lcur);
    } else {
      tile_edge(S, nb0 + 2 * prev + 1, lprev >= 0 ? 2 * lprev + 1 : -1, gl, lcur >= 0 ? 2 * lcur : -1);
    }
    prev = cur;
    lprev = lcur;
    // the run's next operator is the next one in the LDS of its times
    const int64_t nh = cur + 1;
    const int nl = lcur >= 0 ? lcur + 1 : -1;
    const int nt = tcur >= 0 ? tcur + 1 : -1;
    const uint64_t nth = nh < em ? op_time(S.ltime, nt, optime, nh) : 0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s == sm) {
        h[s] = nh;
        hl[s] = nl;
        ht[s] = nt;
        th[s] = nth;
      }
    }
  }
  // the event after window k on this spin: the first operator after the
  // window on either bond, earliest in (time, bond) order
  int64_t nxt = -1, bn = 0;
  uint64_t tnx = 0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (has_next[s] && (nxt < 0 || tn[s] < tnx || (tn[s] == tnx && bnd[s] < bn))) {
      nxt = e[s];
      tnx = tn[s];
      bn = bnd[s];
    }
  }
  const int64_t gu = nb0 + 2 * prev + 1;
  const int lu = lprev >= 0 ? 2 * lprev + 1 : -1;
  if (nxt >= 0) {
    const int ln = tile_local(S, B0, nbt, bn, nxt);
    tile_edge(S, gu, lu, nb0 + 2 * nxt, ln >= 0 ? 2 * ln : -1);
  } else {
    tile_edge(S, gu, lu, node_base + x, -1);
  }
}

// The walk of every (subspin, window) of a split-spin tile at once.  A
// serial walker merges its 2 (2S) time-sorted bond runs one event at a
// time; here every event takes its place in its walker's list directly:
// its position in its own run plus, for every other run, the number of
// that run's operators preceding it in (time, bond) order (a binary search).
// Consecutive list entries then give the same edges as the serial walk
// (tile_walk), emitted in parallel.  Block-cooperative; returns false,
// block-uniformly and before any edge, when the tile has more runs or more
// events than the lists hold (the caller flags the tile as too large).
template <int TS>
__device__ bool tile_walk_lists(TileLds<TS>& S, const ChainDesc& D, int64_t j0, int64_t k0, int nj,
                                int nthr, int64_t nb0, int64_t node_base, int64_t B0, int nbt, int nlo,
                                const int64_t* __restrict__ opstart,
                                const uint64_t* __restrict__ optime) {
  constexpr int NB = 2 * TS;
  using WL = TileLists<TS>;
  WL& Lw = S.wl;
  const int tid = threadIdx.x;
  const int64_t W = int64_t(1) << D.w;
  const int nx = nj * TS;  // subspins of the tile
  // bond slot q of walker w (as in tile_walk)
  auto bond_of = [&](int w, int q) -> int64_t {
    const int64_t x = j0 * TS + w % nx;
    const int64_t j = x / TS, a = x - j * TS, jl = j == 0 ? D.L - 1 : j - 1;
    return q < TS ? (jl * TS + q) * TS + a : (j * TS + a) * TS + (q - TS);
  };
  auto run_time = [&](int r, int p) -> uint64_t {
    return op_time(S.ltime, Lw.rloc[r] >= 0 ? Lw.rloc[r] + p : -1, optime, Lw.rstart[r] + p);
  };
  // the run holding a walker's event `within`: the last run starting at or before it
  auto run_of = [&](int r0, int within) -> int {
    int s = 0;
    for (int q = 1; q < NB; ++q)
      if (Lw.roff[r0 + q] <= within) s = q;
    return s;
  };
  // 1. runs of every walker, one thread per run: its operators in the window,
  // the bond's first operator after the window, whether the bond has
  // operators before the window or none at all
  const int nruns = nthr * NB;
  if (nruns > WL::kRuns) return false;  // block-uniform
  if (tid == 0) Lw.xcur = nlo;
  for (int r = tid; r < nruns; r += kBlock) {
    const int w = r / NB, q = r - w * NB;
    const int64_t k = k0 + w / nx;
    const int64_t bnd = bond_of(w, q);
    const int64_t i0 = D.win_base + bnd * W;
    const int64_t h = opstart[i0 + k], e = opstart[i0 + k + 1];
    const int64_t b0 = opstart[i0], bw = opstart[i0 + W];
    const int64_t lb = bnd - B0;
    Lw.rstart[r] = h;
    Lw.rlen[r] = static_cast<uint16_t>(min(e - h, int64_t(0xFFFF)));
    Lw.rloc[r] = static_cast<int16_t>((lb >= 0 && lb < nbt) ? S.tpre[lb] + (h - S.tos[lb]) : -1);
    uint32_t f = (b0 < h ? 1u : 0u) | (bw == b0 ? 2u : 0u);
    if (e < bw) {
      f |= 4u;
      Lw.rnt[r] = op_time(S.ltime, tile_local(S, B0, nbt, bnd, e), optime, e);
    }
    Lw.rflag[r] = static_cast<uint8_t>(f);
  }
  __syncthreads();
  // per walker: the offsets of its runs in its list, the event after its
  // window (earliest in (time, bond) order), the empty subspin
  int64_t m = 0;
  int fits = 1;
  if (tid < nthr) {
    bool before = false, empty = true;
    int64_t nxt = -1, bn = 0;
    uint64_t tn = 0;
    for (int q = 0; q < NB; ++q) {
      const int r = tid * NB + q;
      Lw.roff[r] = static_cast<uint16_t>(min(m, int64_t(0xFFFF)));
      m += Lw.rlen[r];
      const uint32_t f = Lw.rflag[r];
      before = before || (f & 1u);
      empty = empty && (f & 2u);
      if (f & 4u) {
        const int64_t bnd = bond_of(tid, q);
        const uint64_t t = Lw.rnt[r];
        if (nxt < 0 || t < tn || (t == tn && bnd < bn)) {
          nxt = Lw.rstart[r] + Lw.rlen[r];
          tn = t;
          bn = bnd;
        }
      }
    }
    fits = m <= WL::kItems;
    Lw.wnxt[tid] = nxt;
    Lw.wnl[tid] = static_cast<int16_t>(nxt >= 0 ? tile_local(S, B0, nbt, bn, nxt) : -1);
    Lw.wflag[tid] = static_cast<uint8_t>((before ? 1 : 0) | (empty ? 2 : 0));
  }
  int64_t total;
  const int64_t ex = block_exclusive_scan(m, S.scan, total);
  if (!__syncthreads_and(fits) || total > WL::kItems) return false;  // block-uniform
  if (tid < nthr) {
    Lw.woff[tid] = static_cast<uint16_t>(ex);
    // a subspin without any event: its bottom joins its top
    if (m == 0 && k0 + tid / nx == 0 && (Lw.wflag[tid] & 2)) {
      const int64_t x = j0 * TS + tid % nx;
      tile_edge(S, node_base + x, -1, node_base + D.n_sites + x, -1);
    }
  }
  if (tid == 0) Lw.woff[nthr] = static_cast<uint16_t>(total);
  // the times of runs on bonds the tile does not own go to ltime after the
  // tile's own operators, so that every run's times are in LDS
  for (int r = tid; r < nruns; r += kBlock) {
    const int n = Lw.rlen[r];
    if (Lw.rloc[r] >= 0) {
      Lw.rtix[r] = static_cast<uint16_t>(Lw.rloc[r]);
    } else if (n > 0) {
      const int at = atomicAdd(&Lw.xcur, n);
      Lw.rtix[r] = static_cast<uint16_t>(at < TileCfg<TS>::kOps ? at : 0);
      if (at + n <= TileCfg<TS>::kOps)
        for (int p = 0; p < n; ++p) S.ltime[at + p] = optime[Lw.rstart[r] + p];
    } else {
      Lw.rtix[r] = 0;
    }
  }
  __syncthreads();
  const bool staged = Lw.xcur <= TileCfg<TS>::kOps;  // block-uniform
  const int nev = static_cast<int>(total);
  auto walker_of = [&](int g) -> int {
    int lo = 0, hi = nthr - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (Lw.woff[mid] <= g)
        lo = mid;
      else
        hi = mid - 1;
    }
    return lo;
  };
  // 2. every event's place in its walker's list: its position in its own
  // run plus, for every other run, the number of the run's operators
  // preceding it in (time, bond) order (a binary search, in the staged LDS
  // times, or through run_time when they did not fit)
  for (int g = tid; g < nev; g += kBlock) {
    const int w = walker_of(g);
    const int within = g - Lw.woff[w];
    const int r0 = w * NB;
    const int s = run_of(r0, within);
    const int r = r0 + s, p = within - Lw.roff[r];
    const int64_t bnd = bond_of(w, s);
    const uint64_t t = staged ? S.ltime[Lw.rtix[r] + p] : run_time(r, p);
    int rank = p;
    for (int q = 0; q < NB; ++q) {
      const int rq = r0 + q;
      const int n = Lw.rlen[rq];
      if (q == s || n == 0) continue;
      const bool tie_before = bond_of(w, q) < bnd;  // equal times: smaller bond first
      const int base = Lw.rtix[rq];
      int a = 0, b = n;
      while (a < b) {
        const int mid = (a + b) >> 1;
        const uint64_t tm = staged ? S.ltime[base + mid] : run_time(rq, mid);
        if (tm < t || (tie_before && tm == t))
          a = mid + 1;
        else
          b = mid;
      }
      rank += a;
    }
    Lw.wlist[Lw.woff[w] + rank] = static_cast<uint16_t>(within);
  }
  __syncthreads();
  // 3. edges between consecutive events (the serial walk's edges)
  for (int g = tid; g < nev; g += kBlock) {
    const int w = walker_of(g);
    const int within = g - Lw.woff[w];
    const int mw = Lw.woff[w + 1] - Lw.woff[w];
    const int64_t x = j0 * TS + w % nx;
    auto node = [&](int entry, int h, int64_t* gn, int* ln) {
      const int r = w * NB + run_of(w * NB, entry), p = entry - Lw.roff[r];
      *gn = nb0 + 2 * (Lw.rstart[r] + p) + h;
      *ln = Lw.rloc[r] >= 0 ? 2 * (Lw.rloc[r] + p) + h : -1;
    };
    int64_t gl;
    int ll;
    node(Lw.wlist[g], 0, &gl, &ll);
    if (within == 0) {
      if (!(Lw.wflag[w] & 1)) tile_edge(S, node_base + x, -1, gl, ll);
    } else {
      int64_t gu;
      int lu;
      node(Lw.wlist[g - 1], 1, &gu, &lu);
      tile_edge(S, gu, lu, gl, ll);
    }
    if (within == mw - 1) {
      int64_t gu;
      int lu;
      node(Lw.wlist[g], 1, &gu, &lu);
      if (Lw.wnxt[w] >= 0)
        tile_edge(S, gu, lu, nb0 + 2 * Lw.wnxt[w], Lw.wnl[w] >= 0 ? 2 * Lw.wnl[w] : -1);
      else
        tile_edge(S, gu, lu, node_base + D.n_sites + x, -1);
    }
  }
  return true;
}

template <int TS>
__global__ __launch_bounds__(kBlock) void k_link_tile(
    const ChainDesc* __restrict__ descs, const ChainDyn* __restrict__ dyn, int nchain,
    const int* __restrict__ grp_chain, const int64_t* __restrict__ grp_tile_base, int ngrp,
    int64_t ntiles, const int64_t* __restrict__ opstart, const uint64_t* __restrict__ optime,
    int64_t* __restrict__ parent, int64_t* __restrict__ xedge, int64_t xcap,
    int64_t* __restrict__ frag, int64_t fcap, unsigned long long* __restrict__ dyncnt,
    unsigned long long* __restrict__ stats, uint32_t* __restrict__ flags) {
  using C = TileCfg<TS>;
  constexpr int kNodes = C::kNodes;
  __shared__ TileLds<TS> S;
  const int tid = threadIdx.x;
  // flags are read once per block: later kernels of this launch may set them
  if (tid == 0) S.fl = *flags;
  __syncthreads();
  if (S.fl) return;
  LoopSums sums;
  for (int64_t t = xcd_block(); t < ntiles; t += gridDim.x) {
    const int p = chain_of(grp_tile_base, ngrp, t);
    const int c = grp_chain[p];
    const ChainDesc& D = descs[c];
    const ChainDyn dy = dyn[c];
    const int64_t lt = t - grp_tile_base[p];
    const int64_t W = int64_t(1) << D.w;
    const int64_t ntk = (W + D.tile_k - 1) / D.tile_k;  // window-major tile order
    const int64_t tk = lt % ntk, tj = lt / ntk;
    const int64_t j0 = tj * D.tile_j, k0 = tk * D.tile_k;
    const int nj = static_cast<int>(min(static_cast<int64_t>(D.tile_j), D.L - j0));
    const int nk = static_cast<int>(min(static_cast<int64_t>(D.tile_k), W - k0));
    const int64_t B0 = j0 * TS * TS;
    const int nbt = nj * TS * TS;
    const int nthr = nj * TS * nk;
    const int64_t nb0 = dy.node_base + D.nbn - 2 * dy.op_base;
    // operators of the owned bonds in windows [k0, k0 + nk)
    int64_t cnt = 0;
    if (tid < nbt && tid < kTileBonds) {
      const int64_t i0 = D.win_base + (B0 + tid) * W + k0;
      const int64_t s = opstart[i0];
      S.tos[tid] = s;
      cnt = opstart[i0 + nk] - s;
    }
    // S = 1/2: the operators of the bond left of the tile in its windows,
    // unless the tile owns that bond (a tile over the whole ring)
    int64_t xs0 = 0, xs1 = 0;
    if (TS == 1 && tid == kBlock - 1) {
      const int64_t bl = (j0 == 0 ? D.L : j0) - 1;
      if (bl - B0 < 0 || bl - B0 >= nbt) {
        const int64_t i0 = D.win_base + bl * W + k0;
        xs0 = opstart[i0];
        xs1 = opstart[i0 + nk];
      }
    }
    int64_t total;
    const int64_t ex = block_exclusive_scan(cnt, S.scan, total);
    if (nbt > kTileBonds || nthr > kBlock || total > C::kOps) {  // block-uniform
      if (tid == 0) atomicOr(flags, LC_FLAG_TILE);
      break;
    }
    if (tid < nbt) {
      S.tpre[tid] = static_cast<uint32_t>(ex);
      for (int64_t q = 0; q < cnt; ++q) S.lbond[ex + q] = static_cast<uint8_t>(tid);
    }
    if (tid == 0) {
      S.tpre[nbt] = static_cast<uint32_t>(total);
      S.cnt[0] = S.cnt[1] = S.cnt[2] = S.cnt[3] = 0;
      S.ncl = 0;
    }
    if (TS == 1 && tid == kBlock - 1) {  // staged only when the times fit after the tile's own
      S.sflat = xs0;
      S.sn = total + (xs1 - xs0) <= C::kOps ? static_cast<int>(xs1 - xs0) : 0;
    }
    const int nlo = static_cast<int>(total);
    const int nn = 2 * nlo;
    for (int u = tid; u < nn; u += kBlock) S.lpar[u] = static_cast<uint32_t>(u);
    for (int i = tid; i < kNodes / 16; i += kBlock) S.deg[i] = 0;
    __syncthreads();
    // the tile's operator times, coalesced
    for (int lo = tid; lo < nlo; lo += kBlock) S.ltime[lo] = optime[tile_op(S, static_cast<uint32_t>(lo))];
    if constexpr (TS == 1)
      for (int q = tid; q < S.sn; q += kBlock) S.ltime[nlo + q] = optime[S.sflat + q];
    __syncthreads();
    // S = 1/2: a serial walker per (subspin, window) merges two bond runs;
    // split spins merge 2 (2S) runs through the per-subspin event lists
    if constexpr (TS > 1) {
      if (!tile_walk_lists<TS>(S, D, j0, k0, nj, nthr, nb0, dy.node_base, B0, nbt, nlo, opstart, optime)) {
        if (tid == 0) atomicOr(flags, LC_FLAG_TILE);  // block-uniform: the tile is too large
        break;
      }
    } else {
      // the nodes of the last bond's operators have their edges at the spin
      // right of the tile, which another tile walks: they are open (unless
      // the tile spans the ring)
      if (nj < D.L)
        for (int lo = static_cast<int>(S.tpre[nbt - 1]) + tid; lo < nlo; lo += kBlock)
          atomicOr(S.deg + ((2 * lo) >> 5), 3u << ((2 * lo) & 31));
      if (tid < nthr) {
        const int xs = tid % nj;
        const int kk = tid / nj;
        tile_walk_half(S, D, j0 + xs, k0 + kk, nb0, dy.node_base, B0, nbt, nlo, opstart, optime);
      }
    }
    __syncthreads();
    if (S.cnt[0] > C::kCross) {  // block-uniform
      if (tid == 0) atomicOr(flags, LC_FLAG_TILE);
      break;
    }
    const int nx = S.cnt[0];
    if (tid == 0) {  // places of the staged cross edges in the edge list
      S.base[0] = nx ? static_cast<int64_t>(atomicAdd(dyncnt + 0, static_cast<unsigned long long>(nx))) : 0;
      if (S.base[0] + nx > xcap) atomicOr(flags, LC_FLAG_XEDGE);
    }
    // full compression in two steps: every root is found by read-only walks
    // first (a halving write landing after another thread's final write
    // would leave a node below a non-root), then written; a rep's word
    // becomes its fields
    uint32_t roots[(kNodes + kBlock - 1) / kBlock];
#pragma unroll
    for (int i = 0; i < (kNodes + kBlock - 1) / kBlock; ++i) {
      const int u = tid + i * kBlock;
      uint32_t r = static_cast<uint32_t>(u);
      if (u < nn)
        while (S.lpar[r] != r) r = S.lpar[r];
      roots[i] = r;
    }
    __syncthreads();
    // the staged cross edges go out before the slots (which may share
    // their LDS) come into use
    for (int i = tid; i < nx; i += kBlock) {
      const int64_t g = S.base[0] + i;
      if (g < xcap) {
        xedge[2 * g] = S.cross().xsrc[i];
        xedge[2 * g + 1] = S.cross().xdst[i];
      }
    }
#pragma unroll
    for (int i = 0; i < (kNodes + kBlock - 1) / kBlock; ++i) {
      const int u = tid + i * kBlock;
      if (u < nn) S.lpar[u] = roots[i] == static_cast<uint32_t>(u) ? kRepFlag : roots[i];
    }
    __syncthreads();
    auto rep_of = [&](int u) -> uint32_t {
      const uint32_t w = S.lpar[u];
      return (w & kRepFlag) ? static_cast<uint32_t>(u) : w;
    };
    // component sizes; components with a node lacking a local edge are open
    for (int u = tid; u < nn; u += kBlock) {
      const uint32_t r = rep_of(u);
      const bool open = TileLds<TS>::kOpenBits ? ((S.deg[u >> 5] >> (u & 31)) & 1u) != 0
                                                : ((S.deg[u >> 4] >> ((u & 15) * 2)) & 3u) < 2;
      atomicAdd(S.lpar + r, 1u);
      if (open) atomicOr(S.lpar + r, kRepOpen);
    }
    __syncthreads();
    // closed two-node loops are finished from their two times; every other
    // component gets an accumulator slot
    sums.at(c, stats, nchain);
    for (int u = tid; u < nn; u += kBlock) {
      const uint32_t av = S.lpar[u];
      if (!(av & kRepFlag)) continue;
      const bool open = (av & kRepOpen) != 0;
      if (!open && (av & kRepSize) == 2 && (u & 1) && u + 1 < nn &&
          S.lpar[u + 1] == static_cast<uint32_t>(u)) {
        sums.add(2, (S.ltime[(u + 1) >> 1] - S.ltime[u >> 1]) >> 31);  // length 2 (t1 - t0), >> 32
        continue;  // its flip decision is drawn below
      }
      const int s = atomicAdd(&S.cnt[1], 1);
      if (s < C::kSlots) {
        S.lpar[u] = av | (static_cast<uint32_t>(s + 1) << kRepSlotShift);
        S.slot_rep[s] = static_cast<uint32_t>(u);
        S.slot_hi[s] = 0;
        S.slot_lo[s] = 0;
        S.slot_vote[s] = 0;
        if (open) atomicAdd(&S.cnt[2], 1);
      }
    }
    __syncthreads();
    if (S.cnt[1] > C::kSlots) {  // block-uniform
      if (tid == 0) atomicOr(flags, LC_FLAG_TILE);
      break;
    }
    // length sums of the slotted components: lower nodes +t, upper nodes -t;
    // their nodes' votes under the vote rule
    const bool votes = D.flip_rule != 0;
    for (int lo = tid; lo < nlo; lo += kBlock) {
      const uint64_t tq = S.ltime[lo];
      const uint64_t th = tq >> 32, tl = tq & 0xFFFFFFFFull;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const uint32_t sl = (S.lpar[rep_of(2 * lo + hh)] >> kRepSlotShift) & kRepSlotMask;
        if (!sl) continue;
        atomicAdd(reinterpret_cast<unsigned long long*>(S.slot_hi + sl - 1),
                  static_cast<unsigned long long>(hh ? 0 - th : th));
        atomicAdd(reinterpret_cast<unsigned long long*>(S.slot_lo + sl - 1),
                  static_cast<unsigned long long>(hh ? 0 - tl : tl));
        if (votes &&
            vote_bit(D, nb0 + 2 * tile_op(S, static_cast<uint32_t>(lo)) + hh - dy.node_base))
          atomicXor(S.slot_vote + sl - 1, 1u);
      }
    }
    if (tid == 0) {
      const int nf = S.cnt[2];
      S.base[1] = nf ? static_cast<int64_t>(atomicAdd(dyncnt + 1, static_cast<unsigned long long>(nf))) : 0;
      if (S.base[1] + nf > fcap) atomicOr(flags, LC_FLAG_FRAG);
    }
    __syncthreads();
    // closed components are finished here; open ones become fragments
    const int ns = S.cnt[1];
    for (int s = tid; s < ns; s += kBlock) {
      const uint32_t u = S.slot_rep[s];
      const uint32_t av = S.lpar[u];
      const uint64_t size = av & kRepSize;
      if (av & kRepOpen) {
        const int64_t f = S.base[1] + atomicAdd(&S.cnt[3], 1);
        if (f < fcap) {
          frag[4 * f + 0] = nb0 + 2 * tile_op(S, u >> 1) + (u & 1);
          frag[4 * f + 1] = static_cast<int64_t>(size | (static_cast<uint64_t>(S.slot_vote[s] & 1u) << 15) |
                                                 (static_cast<uint64_t>(c) << 16));
          frag[4 * f + 2] = S.slot_hi[s];
          frag[4 * f + 3] = S.slot_lo[s];
        }
      } else {
        sums.add(size, loop_len32(0, static_cast<uint64_t>(S.slot_hi[s]),
                                  static_cast<uint64_t>(S.slot_lo[s])));
        if (votes && (S.slot_vote[s] & 1u)) S.lpar[u] = av | kRepFlip;
      }
    }
    __syncthreads();
    // flip decisions still to draw: every closed component's under the label
    // rule (the bit of its rep, its smallest node), the two-node loops' under
    // the vote rule (the XOR of their two nodes' votes).  Listed first, so
    // that the draws fill whole waves; the list reuses the times' LDS.
    uint32_t* const clist = reinterpret_cast<uint32_t*>(S.ltime);
    for (int u = tid; u < nn; u += kBlock) {
      const uint32_t av = S.lpar[u];
      if ((av & kRepFlag) && !(av & kRepOpen) &&
          (!votes || ((av >> kRepSlotShift) & kRepSlotMask) == 0))
        clist[atomicAdd(&S.ncl, 1)] = static_cast<uint32_t>(u);
    }
    __syncthreads();
    for (int k = tid; k < S.ncl; k += kBlock) {
      const uint32_t u = clist[k];
      const int64_t v = nb0 + 2 * tile_op(S, u >> 1) + (u & 1) - dy.node_base;
      // two-node loop: v is the upper node of an operator, v + 1 the lower of the next
      if (votes ? (vote_bit(D, v) ^ vote_bit(D, v + 1)) : flip_bit(D, v)) S.lpar[u] |= kRepFlip;
    }
    __syncthreads();  // flip decisions of closed components are read below
    // parent words: an open component's nodes hold its rep (the rep itself);
    // a finished loop's nodes hold its code, smallest node and flip decision
    // (closed_word), so that the flip reads one word per node
    for (int lo = tid; lo < nlo; lo += kBlock) {
      const int64_t q = tile_op(S, static_cast<uint32_t>(lo));
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const uint32_t u = static_cast<uint32_t>(2 * lo + hh);
        const uint32_t r = rep_of(static_cast<int>(u));
        const uint32_t rw = S.lpar[r];
        const int64_t g = nb0 + 2 * q + hh;
        const int64_t gr = r == u ? g : nb0 + 2 * tile_op(S, r >> 1) + (r & 1);
        parent[g] = (rw & kRepOpen) ? gr : closed_word(gr, (rw & kRepFlip) ? 1u : 0u);
      }
    }
    __syncthreads();  // the LDS is reused by the next tile
  }
  sums.flush(stats, nchain);
}

// Edges between tiles: global unions of the nodes' components (through their
// reps, which the tiles wrote as the nodes' parents).
__global__ __launch_bounds__(kBlock) void k_link_cross(const int64_t* __restrict__ xedge,
                                                        const unsigned long long* __restrict__ dyncnt,
                                                        int64_t xcap, const int64_t* __restrict__ totals,
                                                        int64_t* __restrict__ parent,
                                                        uint32_t* __restrict__ flags) {
  if (*flags) return;
  const int64_t nx = static_cast<int64_t>(dyncnt[0]);
  const int64_t n = nx < xcap ? nx : xcap;
  const int64_t nodes = totals[1];
  for (int64_t i = xcd_block() * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    uf_union(parent, xedge[2 * i], xedge[2 * i + 1], nodes, flags);
}

// Symmetrization of the 2S subspins of each spin (split-spin only): a
// permutation pi drawn uniformly among those that map the up (down)
// subspins at beta- onto the up (down) subspins at 0+; top(j,a) joins
// bottom(j, pi(a)).  Fisher-Yates on the SYM stream of the spin.
__global__ __launch_bounds__(kBlock) void k_symmetrize(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ spin_bases, int nchain,
    int64_t nspins, const ChainDyn* __restrict__ dyn, const int64_t* __restrict__ totals,
    int64_t* __restrict__ parent, uint32_t* __restrict__ flags) {
  if (*flags) return;
  const int64_t nodes = totals[1];
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
      uf_union(parent, dy.node_base + D.n_sites + up_t[q], dy.node_base + up_b[q], nodes, flags);
    }
    for (int q = 0; q < ndt; ++q) {
      perm[dn_t[q]] = dn_b[q];
      uf_union(parent, dy.node_base + D.n_sites + dn_t[q], dy.node_base + dn_b[q], nodes, flags);
    }
  }
}

// Full path compression: parent[g] = root = smallest node of g's loop.


// ---------------------------------------------------------------------------
// After the cross-tile unions every open loop is a tree over its items: the
// reps of its fragments and its boundary nodes (every other operator node
// points at a rep, or has been halved to an ancestor rep or boundary node).
// Item i < nf is fragment i; item nf + b is flat boundary node b.
__device__ inline int64_t item_node(int64_t i, int64_t nf, const int64_t* __restrict__ frag,
                                    const int64_t* __restrict__ bn_bases, int nchain,
                                    const ChainDyn* __restrict__ dyn, int* chain) {
  if (i < nf) {
    *chain = static_cast<int>(static_cast<uint64_t>(frag[4 * i + 1]) >> 16);
    return frag[4 * i];
  }
  const int64_t b = i - nf;
  const int c = chain_of(bn_bases, nchain, b);
  *chain = c;
  return dyn[c].node_base + (b - bn_bases[c]);
}

__device__ inline int64_t items_count(const unsigned long long* __restrict__ dyncnt, int64_t fcap,
                                      int64_t nbn, int64_t* nf) {
  const int64_t f = static_cast<int64_t>(dyncnt[1]);
  *nf = f < fcap ? f : fcap;
  return *nf + nbn;
}

// Full path compression of the items: parent = root (smallest node of the
// loop).  Roots are counted per chunk of 4,096 items (each wave covers 64
// consecutive items of one chunk): rcnt feeds the numbering of the loops.
constexpr int kRootPer = 16;                   // steps per chunk
constexpr int kRootChunk = kBlock * kRootPer;  // items per chunk
static_assert(kRootChunk == 4096, "roots are counted per 4,096 items");

__global__ __launch_bounds__(kBlock) void k_compress_items(
    const int64_t* __restrict__ frag, const unsigned long long* __restrict__ dyncnt, int64_t fcap,
    const int64_t* __restrict__ bn_bases, int nchain, int64_t nbn, const ChainDyn* __restrict__ dyn,
    int64_t* __restrict__ parent, unsigned long long* __restrict__ rcnt,
    const uint32_t* __restrict__ flags) {
  if (*flags) return;
  int64_t nf;
  const int64_t n = items_count(dyncnt, fcap, nbn, &nf);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  const int64_t iters = (n + stride - 1) / stride;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t i = xcd_block() * kBlock + threadIdx.x + it * stride;
    int c = 0;
    const int64_t g = i < n ? item_node(i, nf, frag, bn_bases, nchain, dyn, &c) : -1;
    const int64_t p0 = g >= 0 ? parent[g] : -1;
    const unsigned long long roots = __ballot(g >= 0 && p0 == g);
    if (lane_id() == 0 && roots)
      atomicAdd(rcnt + (i >> 12), static_cast<unsigned long long>(__popcll(roots)));
    if (g < 0) continue;
    int64_t r = g, p = p0;
    while (p != r && p >= 0) {
      r = p;
      p = parent[r];
    }
    if (r != g) parent[g] = r;
  }
}

// Roots get compact loop indices in item order: roots are counted per chunk
// (k_compress_items), the counts are scanned, and each chunk numbers its
// roots from its offset.  A chunk is kRootPer steps of kBlock consecutive
// items; a root's rank in its chunk is the roots of earlier steps, of
// earlier waves in its step, and of lower lanes in its wave's ballot.
// The root's parent word becomes the code -1 - index; its record is cleared
// and tagged with its chain.  A loop through a boundary node has a bottom
// boundary node as its smallest node, so its boundary sums live in a
// per-subspin record bacc[site], cleared here.
constexpr int kAccWords = LC_ACC_WORDS;

__global__ __launch_bounds__(kBlock) void k_roots_items(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ frag,
    const unsigned long long* __restrict__ dyncnt, int64_t fcap, const int64_t* __restrict__ bn_bases,
    int nchain, int64_t nbn, const ChainDyn* __restrict__ dyn, int64_t* __restrict__ parent,
    unsigned long long* __restrict__ acc, unsigned long long* __restrict__ bacc, int64_t root_cap,
    int64_t nchunks, const int64_t* __restrict__ rbase, unsigned long long* __restrict__ stats,
    uint32_t* __restrict__ flags) {
  __shared__ int wsum[kRootPer][kWaves];
  __shared__ uint32_t fl;
  if (threadIdx.x == 0) fl = *flags;
  __syncthreads();
  if (fl) return;
  if (rbase[nchunks] > root_cap) {  // the same for every thread
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flags, LC_FLAG_ROOTS);
    return;
  }
  int64_t nf;
  const int64_t n = items_count(dyncnt, fcap, nbn, &nf);
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  constexpr int kIdx[1] = {ST_CLUSTERS};
  Partial<1> part;
  for (int64_t ch = xcd_block(); ch * kRootChunk < n; ch += gridDim.x) {
    const int64_t i0 = ch * kRootChunk + threadIdx.x;
    int64_t gv[kRootPer], pv[kRootPer];
    int cv[kRootPer];
#pragma unroll
    for (int s = 0; s < kRootPer; ++s) {
      const int64_t i = i0 + s * kBlock;
      cv[s] = 0;
      gv[s] = i < n ? item_node(i, nf, frag, bn_bases, nchain, dyn, &cv[s]) : -1;
      pv[s] = gv[s] >= 0 ? parent[gv[s]] : -2;
    }
    unsigned long long m[kRootPer];
#pragma unroll
    for (int s = 0; s < kRootPer; ++s) {
      m[s] = __ballot(gv[s] >= 0 && pv[s] == gv[s]);
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
      if (gv[s] >= 0 && pv[s] == gv[s]) {
        const int64_t li = idx + woff + __popcll(m[s] & below);
        const int c = cv[s];
        part.at(c, stats, nchain, kIdx);
        part.v[0] += 1;
        const ChainDesc& D = descs[c];
        const int64_t v = gv[s] - dyn[c].node_base;
        parent[gv[s]] = -1 - li;
        unsigned long long* a = acc + kAccWords * li;
        a[0] = 0;
        a[1] = 0;
        a[2] = 0;
        // the loop's label is its root: its flip bit now (label rule); the
        // vote rule XORs the nodes' votes into bit 63 later
        a[3] = static_cast<unsigned long long>(c) |
               (D.flip_rule ? 0ull : static_cast<unsigned long long>(flip_bit(D, v)) << 63);
        if (v < D.n_sites) bacc[D.site_base + v] = 0;
      }
      idx += tot;
    }
    __syncthreads();  // wsum is rewritten for the next chunk
  }
  part.flush(stats, nchain, kIdx);
}

// Per-loop records (before the flip) of the open loops, from their items:
//   [0] nodes + (top nodes << 40)
//   [1] sum of +-hi32(t), [2] sum of +-lo32(t)  over operator nodes: lower
//       nodes count +t, upper nodes -t (two vertical segments end / start)
//   [3] chain, bit 63: the loop's flip decision -- the bit of its label
//       (set when the root is numbered), or the XOR of its nodes' votes
// so the loop length is 2^64 tops + 2 (2^32 [1] + [2]) ticks.  A fragment
// brings its node count and its sums; a boundary node one node (a top node
// also 2^64 of length); every word takes plain additions (exact modulo 2^64,
// the true values fit).  Bottom boundary nodes add 1 + (spin << 32) to bacc
// of their loop's root subspin.
//
// A workgroup takes chunks of kAccHash items and sums them per loop in an
// LDS hash table (open addressing on the loop index, LDS atomics), then
// adds each distinct loop's sums to its record with one set of device
// atomics (executed at the memory side: what this pass is bound by).
// Fragments leave the linking tiles in tile order, and at S > 1/2 the loops
// are long and tiles adjacent in time hold many pieces of the same loops, so
// a chunk holds several items of most of its loops (at S = 4 this pass
// takes a fifth of the time of the per-wave reduction below).  Taken when
// any chain has S > 1/2.  A loop with items in nearly every
// chunk (the largest loops at low temperature) would still take a set of
// atomics on one record per chunk: the workgroup carries the sums of one
// such loop -- a chunk's busiest, once it holds kAccHot items there -- from
// chunk to chunk and adds them once, at the end or when the loop is absent
// from a chunk and another busy one takes its place.
constexpr int kAccHash = 1024;  // LDS slots = items per chunk: the table never fills
constexpr int kAccPer = kAccHash / kBlock;
constexpr unsigned long long kAccEmpty = ~0ull;
static_assert(kAccHash == 1024, "the slot hash takes 10 bits");
constexpr uint32_t kAccHot = 64;

__device__ inline void acc_add(unsigned long long* acc, unsigned long long key, uint64_t v0,
                               uint64_t v1, uint64_t v2, uint32_t x) {
  unsigned long long* a = acc + kAccWords * static_cast<int64_t>(key);
  atomicAdd(a + 0, static_cast<unsigned long long>(v0));
  if (v1) atomicAdd(a + 1, static_cast<unsigned long long>(v1));
  if (v2) atomicAdd(a + 2, static_cast<unsigned long long>(v2));
  if (x & 1) atomicXor(a + 3, 1ull << 63);
}

__global__ __launch_bounds__(kBlock) void k_accum_hash(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ frag,
    const unsigned long long* __restrict__ dyncnt, int64_t fcap, const int64_t* __restrict__ bn_bases,
    int nchain, int64_t nbn, const ChainDyn* __restrict__ dyn, const int64_t* __restrict__ parent,
    unsigned long long* __restrict__ acc, unsigned long long* __restrict__ bacc,
    const int64_t* __restrict__ nloops, uint32_t* __restrict__ flags) {
  __shared__ unsigned long long hkey[kAccHash];
  __shared__ unsigned long long hv0[kAccHash], hv1[kAccHash], hv2[kAccHash];
  __shared__ uint32_t hx[kAccHash];  // bit 0: XOR of votes; bits 16..: items
  __shared__ unsigned long long ck, cv0, cv1, cv2;  // the carried loop and its sums
  __shared__ uint32_t cx, cfound, wbest[kWaves];
  __shared__ uint32_t fl;
  const int tid = threadIdx.x;
  if (tid == 0) {
    fl = *flags;
    ck = kAccEmpty;
    cv0 = cv1 = cv2 = 0;
    cx = cfound = 0;
  }
  __syncthreads();
  if (fl) return;
  const int64_t nl = *nloops;
  int64_t nf;
  const int64_t n = items_count(dyncnt, fcap, nbn, &nf);
  const int64_t nchunks = (n + kAccHash - 1) / kAccHash;
  for (int64_t ch = xcd_block(); ch < nchunks; ch += gridDim.x) {
    for (int h = tid; h < kAccHash; h += kBlock) {
      hkey[h] = kAccEmpty;
      hv0[h] = hv1[h] = hv2[h] = 0;
      hx[h] = 0;
    }
    __syncthreads();
    const int lane = lane_id();
    // the items' dependent reads (node, its word, its rep's word) are issued
    // for all of a thread's items before any is used
    int64_t gq[kAccPer], pq[kAccPer], cq[kAccPer];
    int chq[kAccPer];
#pragma unroll
    for (int q = 0; q < kAccPer; ++q) {
      const int64_t i = ch * kAccHash + q * kBlock + tid;
      chq[q] = 0;
      gq[q] = i < n ? item_node(i, nf, frag, bn_bases, nchain, dyn, &chq[q]) : -1;
    }
#pragma unroll
    for (int q = 0; q < kAccPer; ++q) pq[q] = gq[q] >= 0 ? parent[gq[q]] : -1;
#pragma unroll
    for (int q = 0; q < kAccPer; ++q) cq[q] = (gq[q] >= 0 && pq[q] >= 0) ? parent[pq[q]] : pq[q];
#pragma unroll
    for (int q = 0; q < kAccPer; ++q) {
      const int64_t i = ch * kAccHash + q * kBlock + tid;
      int64_t r = -1;
      uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;  // w3: XOR of votes (bit 0)
      if (i < n) {
        const int c = chq[q];
        const int64_t g = gq[q];
        const int64_t p = pq[q];
        const int64_t code = cq[q];
        r = -1 - code;
        if (code >= 0 || r >= nl) {  // not a numbered loop: inconsistent graph
          atomicOr(flags, LC_FLAG_GRAPH);
          r = -1;
        } else if (i < nf) {
          w0 = static_cast<uint64_t>(frag[4 * i + 1]) & 0x7FFFull;
          w3 = (static_cast<uint64_t>(frag[4 * i + 1]) >> 15) & 1u;
          w1 = static_cast<uint64_t>(frag[4 * i + 2]);
          w2 = static_cast<uint64_t>(frag[4 * i + 3]);
        } else {
          const ChainDesc& D = descs[c];
          const int64_t cb = dyn[c].node_base;
          const int64_t v = g - cb;
          const bool bottom = v < D.n_sites;
          w0 = 1;
          if (D.two_s == 1 || !bottom) w0 += 1ull << 40;  // a top node: + 2^64
          if (D.flip_rule) w3 = vote_bit(D, v);
          const int64_t root = (p >= 0 ? p : g) - cb;
          if (bottom && root < D.n_sites)  // always true: the root is a bottom node
            atomicAdd(bacc + D.site_base + root,
                      1ull + (static_cast<uint64_t>(2 * static_cast<int64_t>(D.s0[D.cur][v]) - 1) << 32));
        }
      }
      // Reduce by loop within the wave first (a large loop would otherwise
      // queue many lanes on one LDS word): bitonic sort of one packed word
      // per lane, (loop << 6) | lane (loop indices are below 2^40), so only
      // the key moves through the 21 exchange stages; each lane fetches the
      // sums of the item it ended up with, a segmented scan adds equal loops,
      // and the last lane of each run adds them to the loop's slot.
      uint64_t sk = r >= 0 ? ((static_cast<uint64_t>(r) << 6) | static_cast<uint64_t>(lane)) : ~0ull;
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
      const int64_t key = sk == ~0ull ? -1 : static_cast<int64_t>(sk >> 6);
      w0 = __shfl(w0, src);
      w1 = __shfl(w1, src);
      w2 = __shfl(w2, src);
      w3 = __shfl(w3, src);
      const int64_t pkey = __shfl_up(key, 1);
      const unsigned long long heads = __ballot(lane == 0 || pkey != key);
      const int seg = __popcll(heads & ((lane == 63) ? ~0ull : ((2ull << lane) - 1ull)));
      uint32_t cnt = 1;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int qs = __shfl_up(seg, d);
        const uint64_t q0 = __shfl_up(w0, d), q1 = __shfl_up(w1, d), q2 = __shfl_up(w2, d);
        const uint64_t q3 = __shfl_up(w3, d);
        const uint32_t qc = __shfl_up(cnt, d);
        if (lane >= d && qs == seg) {
          w0 += q0;
          w1 += q1;
          w2 += q2;
          w3 ^= q3;
          cnt += qc;
        }
      }
      const bool last = lane == 63 || ((heads >> (lane + 1)) & 1ull);
      if (key < 0 || !last) continue;
      // find or claim the loop's slot (at most kAccHash keys per chunk)
      const unsigned long long uk = static_cast<unsigned long long>(key);
      uint32_t h = static_cast<uint32_t>((uk * 0x9E3779B97F4A7C15ull) >> 54);  // 10 bits
      for (;;) {
        unsigned long long kk =
            __hip_atomic_load(hkey + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (kk == kAccEmpty) {
          kk = atomicCAS(hkey + h, kAccEmpty, uk);
          if (kk == kAccEmpty) kk = uk;
        }
        if (kk == uk) break;
        h = (h + 1) & (kAccHash - 1);
      }
      atomicAdd(hv0 + h, static_cast<unsigned long long>(w0));
      if (w1) atomicAdd(hv1 + h, static_cast<unsigned long long>(w1));
      if (w2) atomicAdd(hv2 + h, static_cast<unsigned long long>(w2));
      atomicAdd(hx + h, (cnt << 16) | static_cast<uint32_t>(w3 & 1));
    }
    __syncthreads();
    // the carried loop absorbs its slot; the busiest other loop is found
    uint32_t best = 0;  // (items << 10) | slot
    for (int h = tid; h < kAccHash; h += kBlock) {
      const unsigned long long key = hkey[h];
      if (key == kAccEmpty) continue;
      if (key == ck) {  // one slot, one thread
        cv0 += hv0[h];
        cv1 += hv1[h];
        cv2 += hv2[h];
        cx ^= hx[h] & 1;
        cfound = 1;
        hkey[h] = kAccEmpty;
      } else {
        const uint32_t v = ((hx[h] >> 16) << 10) | static_cast<uint32_t>(h);
        best = v > best ? v : best;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t w = __shfl_xor(best, o);
      best = w > best ? w : best;
    }
    if (lane_id() == 0) wbest[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
      uint32_t b = 0;
      for (int w = 0; w < kWaves; ++w) b = wbest[w] > b ? wbest[w] : b;
      if (!cfound && (b >> 10) >= kAccHot) {
        if (ck != kAccEmpty) acc_add(acc, ck, cv0, cv1, cv2, cx);
        const int h = static_cast<int>(b & (kAccHash - 1));
        ck = hkey[h];
        cv0 = hv0[h];
        cv1 = hv1[h];
        cv2 = hv2[h];
        cx = hx[h] & 1;
        hkey[h] = kAccEmpty;
      }
      cfound = 0;
    }
    __syncthreads();
    for (int h = tid; h < kAccHash; h += kBlock) {
      const unsigned long long key = hkey[h];
      if (key != kAccEmpty) acc_add(acc, key, hv0[h], hv1[h], hv2[h], hx[h]);
    }
    __syncthreads();  // the table is cleared for the next chunk
  }
  if (tid == 0 && ck != kAccEmpty) acc_add(acc, ck, cv0, cv1, cv2, cx);
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
                                   uint64_t v2, uint64_t v3) {
  unsigned long long* a = acc + kAccWords * key;
  atomicAdd(a + 0, static_cast<unsigned long long>(v0));
  if (v1) atomicAdd(a + 1, static_cast<unsigned long long>(v1));
  if (v2) atomicAdd(a + 2, static_cast<unsigned long long>(v2));
  if (v3 & 1) atomicXor(a + 3, 1ull << 63);
}

// The same records without an LDS table: each wave reduces its 64 items by
// loop and issues one set of atomics per distinct loop, carrying the sums
// of one hot loop across its steps.  Taken when every chain has S = 1/2:
// there a 1,024-item chunk holds few more repeats of a loop than a wave
// does, and this kernel, free of barriers and LDS, issues fewer atomics.
__global__ __launch_bounds__(kBlock, 6) void k_accum_items(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ frag,
    const unsigned long long* __restrict__ dyncnt, int64_t fcap, const int64_t* __restrict__ bn_bases,
    int nchain, int64_t nbn, const ChainDyn* __restrict__ dyn, const int64_t* __restrict__ parent,
    unsigned long long* __restrict__ acc, unsigned long long* __restrict__ bacc,
    const int64_t* __restrict__ nloops, uint32_t* __restrict__ flags) {
  if (*flags) return;
  const int64_t nl = *nloops;
  int64_t nf;
  const int64_t n = items_count(dyncnt, fcap, nbn, &nf);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  const int64_t iters = (n + stride - 1) / stride;
  // wave carry: sums of one hot loop (wave-uniform), flushed once
  int64_t ck = -1;
  uint64_t cv0 = 0, cv1 = 0, cv2 = 0, cv3 = 0;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t i = xcd_block() * kBlock + threadIdx.x + it * stride;
    int64_t r = -1;
    uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;  // w3: XOR of votes (bit 0)
    if (i < n) {
      int c = 0;
      const int64_t g = item_node(i, nf, frag, bn_bases, nchain, dyn, &c);
      const int64_t p = parent[g];
      const int64_t code = p >= 0 ? parent[p] : p;
      r = -1 - code;
      if (code >= 0 || r >= nl) {  // not a numbered loop: inconsistent graph
        atomicOr(flags, LC_FLAG_GRAPH);
        r = -1;
      } else if (i < nf) {
        w0 = static_cast<uint64_t>(frag[4 * i + 1]) & 0x7FFFull;
        w3 = (static_cast<uint64_t>(frag[4 * i + 1]) >> 15) & 1u;
        w1 = static_cast<uint64_t>(frag[4 * i + 2]);
        w2 = static_cast<uint64_t>(frag[4 * i + 3]);
      } else {
        const ChainDesc& D = descs[c];
        const int64_t cb = dyn[c].node_base;
        const int64_t v = g - cb;
        const bool bottom = v < D.n_sites;
        w0 = 1;
        if (D.two_s == 1 || !bottom) w0 += 1ull << 40;  // a top node: + 2^64
        if (D.flip_rule) w3 = vote_bit(D, v);
        const int64_t root = (p >= 0 ? p : g) - cb;
        if (bottom && root < D.n_sites)  // always true: the root is a bottom node
          atomicAdd(bacc + D.site_base + root,
                    1ull + (static_cast<uint64_t>(2 * static_cast<int64_t>(D.s0[D.cur][v]) - 1) << 32));
      }
    }
    // Reduce by loop within the wave: bitonic sort of one packed word per
    // lane, (loop << 6) | lane (loop indices are below 2^40), so only the key
    // moves through the 21 exchange stages; each lane then fetches the sums
    // of the item it ended up with, a segmented scan adds equal loops, and
    // the last lane of each run issues one set of atomics per distinct loop.
    // Very large loops meet nearly every wave: the wave carries the sums of
    // one such loop across its steps instead of adding them to the same
    // record from every wave and step.
    const int lane = lane_id();
    uint64_t sk = r >= 0 ? ((static_cast<uint64_t>(r) << 6) | static_cast<uint64_t>(lane)) : ~0ull;
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
    w0 = __shfl(w0, src);
    w1 = __shfl(w1, src);
    w2 = __shfl(w2, src);
    w3 = __shfl(w3, src);
    // runs of equal loops: head lanes from one ballot, segment id = heads so far
    const int64_t pkey = __shfl_up(key, 1);
    const unsigned long long heads = __ballot(lane == 0 || pkey != key);
    const int seg = __popcll(heads & ((lane == 63) ? ~0ull : ((2ull << lane) - 1ull)));
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int qs = __shfl_up(seg, d);
      const uint64_t q0 = __shfl_up(w0, d), q1 = __shfl_up(w1, d), q2 = __shfl_up(w2, d);
      const uint64_t q3 = __shfl_up(w3, d);
      if (lane >= d && qs == seg) {
        w0 += q0;
        w1 += q1;
        w2 += q2;
        w3 ^= q3;
      }
    }
    const bool last = lane == 63 || ((heads >> (lane + 1)) & 1ull);
    const bool seg_end = key != INT64_MAX && last;
    // the carried loop absorbs its segment without atomics
    bool absorbed = seg_end && key == ck;
    unsigned long long m = __ballot(absorbed);
    if (!m) {
      // the carried loop is absent: a segment of at least 16 items takes over
      // the carry (the old carry is flushed); the largest such segment wins
      const int seglen = seg_end ? (lane + 1 - (63 - __clzll(static_cast<long long>(heads & ((2ull << lane) - 1ull))))) : 0;
      const uint32_t cnt = static_cast<uint32_t>(seglen);
      const uint32_t best = wave_max_u32((cnt << 6) | static_cast<uint32_t>(lane));
      if ((best >> 6) >= 16) {
        if (ck >= 0 && lane == 0) flush_carry(acc, ck, cv0, cv1, cv2, cv3);
        ck = __shfl(key, static_cast<int>(best & 63u));
        cv0 = cv1 = cv2 = cv3 = 0;
        absorbed = lane == static_cast<int>(best & 63u);
        m = __ballot(absorbed);
      }
    }
    if (m) {
      const int sl = __ffsll(static_cast<long long>(m)) - 1;
      cv0 += __shfl(w0, sl);
      cv1 += __shfl(w1, sl);
      cv2 += __shfl(w2, sl);
      cv3 ^= __shfl(w3, sl);
    }
    if (seg_end && !absorbed) {
      unsigned long long* a = acc + kAccWords * key;
      atomicAdd(a + 0, static_cast<unsigned long long>(w0));
      if (w1) atomicAdd(a + 1, static_cast<unsigned long long>(w1));
      if (w2) atomicAdd(a + 2, static_cast<unsigned long long>(w2));
      if (w3 & 1) atomicXor(a + 3, 1ull << 63);
    }
  }
  if (ck >= 0 && lane_id() == 0) flush_carry(acc, ck, cv0, cv1, cv2, cv3);
}

// Per-loop squares of the open loops summed into the chain statistics (the
// chain of a record is its word 3).
__global__ __launch_bounds__(kBlock) void k_cluster_sums(
    int nchain, const int64_t* __restrict__ nloops, int64_t root_cap,
    const unsigned long long* __restrict__ acc, unsigned long long* __restrict__ stats,
    const uint32_t* __restrict__ flags) {
  if (*flags) return;
  const int64_t n = *nloops < root_cap ? *nloops : root_cap;
  LoopSums sums;
  for (int64_t i = xcd_block() * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const unsigned long long* a = acc + kAccWords * i;
    sums.at(static_cast<int>(a[3] & ~(1ull << 63)), stats, nchain);
    const uint64_t sz = a[0] & ((1ull << 40) - 1), tops = a[0] >> 40;
    // the loop was counted when its root was numbered
    sums.add(sz, loop_len32(tops, a[1], a[2]), false);
  }
  sums.flush(stats, nchain);
}

// Flip decision of the loop through node g: from g's own word for a loop
// finished in its tile (closed_word), else the record's bit 63, found
// through the loop code in g's word, its rep's, or the root's.  The decision
// was taken once per loop (label rule: the bit of its smallest node; vote
// rule: the XOR of its nodes' votes).
__device__ inline uint32_t node_flip(const int64_t* __restrict__ parent,
                                     const unsigned long long* __restrict__ acc, int64_t g) {
  const int64_t p = parent[g];
  if (is_closed_word(p)) return closed_bit(p);
  int64_t code = p;
  if (p >= 0) {
    const int64_t pp = parent[p];
    code = pp < 0 ? pp : parent[pp];
  }
  return static_cast<uint32_t>(acc[kAccWords * (-1 - code) + 3] >> 63);
}

// The XOR of the flip decisions of an operator's two nodes, g (lower, even)
// and g + 1: node_flip for both, each step's reads of the two nodes issued
// together (one 16-byte read of the two words, then the reps' words, the
// roots' words, the loop records), so that a wave waits on one chain of
// dependent reads per operator instead of two.
__device__ inline uint32_t pair_flip(const int64_t* __restrict__ parent,
                                     const unsigned long long* __restrict__ acc, int64_t g) {
  const longlong2 w = *reinterpret_cast<const longlong2*>(parent + g);
  const int64_t x0 = w.x, x1 = w.y;
  const bool c0 = is_closed_word(x0), c1 = is_closed_word(x1);
  // an open node's word is its rep (>= 0) or, for a root, its loop code (< 0)
  int64_t y0 = x0, y1 = x1;
  if (!c0 && x0 >= 0) y0 = parent[x0];
  if (!c1 && x1 >= 0) y1 = parent[x1];
  // the rep's word: its root (>= 0) or its loop code
  int64_t z0 = y0, z1 = y1;
  if (!c0 && y0 >= 0) z0 = parent[y0];
  if (!c1 && y1 >= 0) z1 = parent[y1];
  // the loop records' flip bits (bit 63 of word 3), both read at once: a
  // closed node reads record 0 instead (the records always outnumber the
  // boundary nodes, so there is one) and ignores it
  const int64_t k0 = c0 ? 0 : -1 - z0, k1 = c1 ? 0 : -1 - z1;
  const unsigned long long r0 = acc[kAccWords * k0 + 3], r1 = acc[kAccWords * k1 + 3];
  const uint32_t f0 = c0 ? closed_bit(x0) : static_cast<uint32_t>(r0 >> 63);
  const uint32_t f1 = c1 ? closed_bit(x1) : static_cast<uint32_t>(r1 >> 63);
  return f0 ^ f1;
}

// Cluster flip (step 7): the type of an operator changes when exactly one of
// its two loops flips; kept (off-diagonal) operators are counted per window.
// A node of a loop finished in its linking tile carries the decision in its
// own word; other nodes reach their loop's record through the root.  The
// operators are taken tile by tile (the linking tiles: bonds x windows), one
// workgroup per tile and one thread per operator, so the reads of the
// operators' words are coalesced along each bond's run and the lookups of
// the roots of long loops (shared by many nodes) hit lines the workgroup has
// just read.  Kept operators are counted per window in LDS through an
// operator -> window map.
constexpr int kFlipWin = LC_TILE_BONDS * LC_MAX_TS;  // windows of a tile: its bonds x windows <= 256 TS

// NWIN: windows a tile may hold -- kBlock for S = 1/2 (one walker per
// window), kFlipWin for split spins; the smaller LDS keeps more
// workgroups of the S = 1/2 flip on a CU.
template <int NWIN>
__global__ __launch_bounds__(kBlock) void k_flip_tiles(
    const ChainDesc* __restrict__ descs, const ChainDyn* __restrict__ dyn, int nchain,
    const int* __restrict__ grp_chain, const int64_t* __restrict__ grp_tile_base, int ngrp,
    int64_t ntiles, const int64_t* __restrict__ opstart, const int64_t* __restrict__ parent,
    const unsigned long long* __restrict__ acc, uint8_t* __restrict__ optype,
    int64_t* __restrict__ kcnt, unsigned long long* __restrict__ stats, uint32_t* __restrict__ flags) {
  __shared__ uint32_t wstart[NWIN + 1];   // first local operator of each window
  __shared__ uint32_t wkept[NWIN];
  __shared__ uint16_t wop[LC_TILE_OPS];       // window of each local operator
  __shared__ int64_t bfirst[kTileBonds];      // first flat operator of each bond's run
  __shared__ int64_t scan[kWaves + 1];
  __shared__ uint32_t fl;
  const int tid = threadIdx.x;
  if (tid == 0) fl = *flags;
  __syncthreads();
  if (fl) return;
  constexpr int kIdx[1] = {ST_KEPT_OUT};
  Partial<1> part;
  for (int64_t t = xcd_block(); t < ntiles; t += gridDim.x) {
    const int p = chain_of(grp_tile_base, ngrp, t);
    const int c = grp_chain[p];
    part.at(c, stats, nchain, kIdx);
    const ChainDesc& D = descs[c];
    const ChainDyn dy = dyn[c];
    const int64_t lt = t - grp_tile_base[p];
    const int64_t W = int64_t(1) << D.w;
    const int64_t ntk = (W + D.tile_k - 1) / D.tile_k;  // window-major tile order
    const int64_t tk = lt % ntk, tj = lt / ntk;
    const int64_t j0 = tj * D.tile_j, k0 = tk * D.tile_k;
    const int nj = static_cast<int>(min(static_cast<int64_t>(D.tile_j), D.L - j0));
    const int nk = static_cast<int>(min(static_cast<int64_t>(D.tile_k), W - k0));
    const int64_t B0 = j0 * D.two_s * D.two_s;
    const int nbt = nj * D.two_s * D.two_s;
    const int nwt = nbt * nk;
    const int64_t nb0 = dy.node_base + D.nbn - 2 * dy.op_base;
    // the linking of these tiles succeeded, so they fit; checked all the same
    if (nbt > kTileBonds || nwt > NWIN) {  // block-uniform
      if (tid == 0) atomicOr(flags, LC_FLAG_TILE);
      break;
    }
    // windows in (bond, window) order are the tile's operators in local order;
    // each thread scans a contiguous chunk of them
    const int per = (nwt + kBlock - 1) / kBlock;
    int64_t cnt = 0;
    for (int m = 0; m < per; ++m) {
      const int wi = tid * per + m;
      if (wi < nwt) {
        const int lb = wi / nk, kk = wi - lb * nk;
        const int64_t i = D.win_base + (B0 + lb) * W + k0 + kk;
        const int64_t a = opstart[i];
        cnt += opstart[i + 1] - a;
        if (kk == 0) bfirst[lb] = a;
      }
    }
    int64_t total;
    int64_t run = block_exclusive_scan(cnt, scan, total);
    if (total > LC_TILE_OPS) {  // block-uniform
      if (tid == 0) atomicOr(flags, LC_FLAG_TILE);
      break;
    }
    for (int m = 0; m < per; ++m) {
      const int wi = tid * per + m;
      if (wi < nwt) {
        const int lb = wi / nk, kk = wi - lb * nk;
        const int64_t i = D.win_base + (B0 + lb) * W + k0 + kk;
        wstart[wi] = static_cast<uint32_t>(run);
        wkept[wi] = 0;
        run += opstart[i + 1] - opstart[i];
      }
    }
    if (tid == 0) wstart[nwt] = static_cast<uint32_t>(total);
    __syncthreads();
    for (int wi = tid; wi < nwt; wi += kBlock)
      for (uint32_t lo = wstart[wi]; lo < wstart[wi + 1]; ++lo) wop[lo] = static_cast<uint16_t>(wi);
    __syncthreads();
    const int nlo = static_cast<int>(total);
    for (int lo = tid; lo < nlo; lo += kBlock) {
      const int wi = wop[lo];
      const int lb = wi / nk;
      const int64_t q = bfirst[lb] + (lo - static_cast<int64_t>(wstart[lb * nk]));
      const int64_t g = nb0 + 2 * q;
      const uint8_t v = optype[q];
      const uint8_t ty = static_cast<uint8_t>((v & 1) ^ pair_flip(parent, acc, g));
      optype[q] = static_cast<uint8_t>(ty | (v & 2));
      if (ty) atomicAdd(wkept + wi, 1u);
    }
    __syncthreads();
    for (int wi = tid; wi < nwt; wi += kBlock) {
      const int lb = wi / nk, kk = wi - lb * nk;
      const uint32_t k = wkept[wi];
      kcnt[D.win_base + (B0 + lb) * W + k0 + kk] = k;
      part.v[0] += k;
    }
    __syncthreads();  // the LDS is reused by the next tile
  }
  part.flush(stats, nchain, kIdx);
}

// New spins at tau = 0; the boundary estimators of every loop whose root is
// this subspin's bottom node (n0 = bottom nodes, m = their spin sum before
// the flip) are squared into the chain statistics.
__global__ __launch_bounds__(kBlock) void k_flip_sites(
    const ChainDesc* __restrict__ descs, const int64_t* __restrict__ site_bases, int nchain,
    int64_t nsites, const ChainDyn* __restrict__ dyn, const int64_t* __restrict__ parent,
    const unsigned long long* __restrict__ acc, const unsigned long long* __restrict__ bacc,
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
    const uint8_t s =
        D.s0[D.cur][x] ^ static_cast<uint8_t>(node_flip(parent, acc, dyn[c].node_base + x));
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

// Next world lines (step 7): the kept operators of every window, in order.
// They keep the operator array's own (window, operator) order, so this is a
// stream compaction: a workgroup takes 256 windows, writes their starts, and
// moves their kept operators with a block scan of the kept flags over the
// windows' operator range (8 operators per thread, 256 apart), reading and
// writing contiguous memory.  Windows of different chains (a batch) are
// taken chain by chain.
constexpr int kCompactPer = 8;

__global__ __launch_bounds__(kBlock) void k_compact(const ChainDesc* __restrict__ descs,
                                                     const int64_t* __restrict__ win_bases,
                                                     int nchain, int64_t nwin,
                                                     const int64_t* __restrict__ opstart,
                                                     const uint64_t* __restrict__ optime,
                                                     const uint8_t* __restrict__ optype,
                                                     const int64_t* __restrict__ kflat,
                                                     uint32_t* __restrict__ flags) {
  __shared__ int wsum[kCompactPer][kWaves];
  __shared__ uint32_t fl;
  // a sweep with any overflow or error is discarded: kflat may be stale
  // (read once per block: blocks of this kernel may raise the kept flag)
  if (threadIdx.x == 0) fl = *flags;
  __syncthreads();
  if (fl) return;
  const int tid = threadIdx.x;
  const int lane = lane_id(), wv = tid >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int64_t c0 = xcd_block() * kBlock; c0 < nwin; c0 += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t cend = c0 + kBlock < nwin ? c0 + kBlock : nwin;
    for (int64_t w = c0; w < cend;) {  // block-uniform: the chains of the 256 windows
      const int c = chain_of(win_bases, nchain, w);
      const ChainDesc& D = descs[c];
      const int64_t nw = D.n_bonds << D.w;
      const int64_t wend = cend < D.win_base + nw ? cend : D.win_base + nw;
      const int64_t kb = kflat[D.win_base];
      if (kflat[D.win_base + nw] - kb > D.kept_cap) {
        if (tid == 0) atomicOr(flags, 8u);
        w = wend;
        continue;
      }
      LC_GLOBAL int64_t* __restrict__ ks = gout(D.kstart[D.cur ^ 1]);
      LC_GLOBAL uint64_t* __restrict__ kt = gout(D.ktime[D.cur ^ 1]);
      const int64_t i = w + tid;
      if (i < wend) {
        const int64_t li = i - D.win_base;
        ks[li] = kflat[i] - kb;
        if (li == nw - 1) ks[nw] = kflat[i + 1] - kb;
      }
      const int64_t qb = opstart[wend];
      int64_t out = kflat[w] - kb;
      // operator base + m 256 + tid: every load and store of a wave is one
      // contiguous run; a kept operator's place is the kept ones of earlier
      // steps, of earlier waves in its step (LDS), and of lower lanes (ballot)
      for (int64_t base = opstart[w]; base < qb; base += kBlock * kCompactPer) {
        unsigned long long bal[kCompactPer];
#pragma unroll
        for (int m = 0; m < kCompactPer; ++m) {
          const int64_t q = base + m * kBlock + tid;
          bal[m] = __ballot(q < qb && (optype[q] & 1));
          if (lane == 0) wsum[m][wv] = __popcll(bal[m]);
        }
        __syncthreads();
        int64_t o = out;
#pragma unroll
        for (int m = 0; m < kCompactPer; ++m) {
          int before = 0, all = 0;
#pragma unroll
          for (int v = 0; v < kWaves; ++v) {
            before += v < wv ? wsum[m][v] : 0;
            all += wsum[m][v];
          }
          if ((bal[m] >> lane) & 1ull) {
            const int64_t q = base + m * kBlock + tid;
            kt[o + before + __popcll(bal[m] & below)] = optime[q];
          }
          o += all;
        }
        __syncthreads();  // wsum is rewritten by the next step
        out = o;
      }
      w = wend;
    }
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



// ---------------------------------------------------------------------------
// Imaginary-time slices with open boundaries (Sec. 3.1): the time axis is cut
// into G slices of whole windows; inside each slice the loop graph of the
// most recent sweep is linked and union-found on its own, the segments
// crossing a slice boundary being cut: the first event of a subspin in the
// slice joins the slice's bottom node of that subspin, its last event the
// slice's top node, and a subspin without events in the slice joins the two
// directly.  Node ids: bottom(p, x) = 2 ns p + x, top(p, x) = 2 ns p + ns + x,
// operator node (q, h) = 2 ns G + 2 (q - op_base) + h.  What each slice
// leaves open is its 2 ns boundary nodes' components: the table a global
// merge of the slices needs (Sec. 3.1, Fig. 3; the butterfly of Sec. 3.3
// exchanges exactly these).
template <int TS>
__global__ __launch_bounds__(kBlock) void k_slice_walk(LcSliceArgs A) {
  constexpr int NB = 2 * TS;
  const int64_t W = int64_t(1) << A.w;
  const int64_t ns = A.n_sites, G = A.n_slices;
  const int64_t nodes = 2 * ns * G + 2 * A.n_ops;
  const int64_t nop0 = 2 * ns * G - 2 * A.op_base;  // node of lower(q) = nop0 + 2q
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < ns * W;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t x = i / W, k = i - x * W;
    const int64_t p = ((k + 1) * G - 1) / W;
    const int64_t kb = p * W / G, ke = (p + 1) * W / G;
    const int64_t bot = 2 * ns * p + x, top = bot + ns;
    const int64_t j = x / TS, a = x - j * TS;
    const int64_t jl = (j == 0) ? A.L - 1 : j - 1;
    int64_t bnd[NB], h[NB], e[NB], se[NB];
    uint64_t th[NB];
    bool before = false, any = false, inslice = false;
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      bnd[s] = s < TS ? (jl * TS + s) * TS + a : (j * TS + a) * TS + (s - TS);
      const int64_t i0 = A.win_base + bnd[s] * W;
      h[s] = A.opstart[i0 + k];
      e[s] = A.opstart[i0 + k + 1];
      se[s] = A.opstart[i0 + ke];  // end of the slice on this bond
      const int64_t sb = A.opstart[i0 + kb];
      before = before || sb < h[s];
      inslice = inslice || sb < se[s];
      th[s] = h[s] < e[s] ? A.optime[h[s]] : 0;
      any = any || h[s] < e[s];
    }
    if (!any) {
      if (k == kb && !inslice) uf_union(A.parent, bot, top, nodes, A.flags);
      continue;
    }
    int64_t prev = -1;
    for (;;) {
      int sm = -1;
      uint64_t tm = 0;
      int64_t bm = 0, cur = 0, em = 0;
#pragma unroll
      for (int s = 0; s < NB; ++s) {
        if (h[s] < e[s] && (sm < 0 || th[s] < tm || (th[s] == tm && bnd[s] < bm))) {
          sm = s;
          tm = th[s];
          bm = bnd[s];
          cur = h[s];
          em = e[s];
        }
      }
      if (sm < 0) break;
      if (prev < 0) {
        if (!before) uf_union(A.parent, bot, nop0 + 2 * cur, nodes, A.flags);
      } else {
        uf_union(A.parent, nop0 + 2 * prev + 1, nop0 + 2 * cur, nodes, A.flags);
      }
      prev = cur;
      const int64_t nh = cur + 1;
      const uint64_t nt = nh < em ? A.optime[nh] : 0;
#pragma unroll
      for (int s = 0; s < NB; ++s) {
        if (s == sm) {
          h[s] = nh;
          th[s] = nt;
        }
      }
    }
    // the next event on this subspin inside the slice, or its top node
    int64_t nxt = -1, bn = 0;
    uint64_t tn = 0;
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      const int64_t idx = e[s];
      if (idx < se[s]) {
        const uint64_t t = A.optime[idx];
        if (nxt < 0 || t < tn || (t == tn && bnd[s] < bn)) {
          nxt = idx;
          tn = t;
          bn = bnd[s];
        }
      }
    }
    uf_union(A.parent, nop0 + 2 * prev + 1, nxt >= 0 ? nop0 + 2 * nxt : top, nodes, A.flags);
  }
}

__global__ __launch_bounds__(kBlock) void k_slice_init(int64_t* __restrict__ parent, int64_t n) {
  for (int64_t g = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; g < n;
       g += static_cast<int64_t>(gridDim.x) * kBlock)
    parent[g] = g;
}

// label = smallest node of the slice component (read-only walk, then write)
__global__ __launch_bounds__(kBlock) void k_slice_compress(int64_t* __restrict__ parent, int64_t n) {
  for (int64_t g = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; g < n;
       g += static_cast<int64_t>(gridDim.x) * kBlock) {
    int64_t r = g, p = parent[g];
    while (p != r && p >= 0 && p < n) {
      r = p;
      p = parent[r];
    }
    parent[g] = r;
  }
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

template <int TS>
static void launch_tiles(const LcSweepArgs& A, const LcTileGroup& g, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_link_tile<TS>), dim3(grid), dim3(kBlock), 0, s, A.descs, A.dyn, A.nchain,
                     A.grp_chain + g.offset, A.grp_tile_base + g.offset, g.nchain, g.ntiles,
                     A.opstart, A.optime, A.parent, A.xedge, A.xcap, A.frag, A.fcap, A.dyncnt,
                     reinterpret_cast<unsigned long long*>(A.stats), A.flags);
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
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, A.dyncnt, 4, 0ull);
  // 1. count operators per window, 2. scan
  mark(LC_PH_GEN_COUNT);
  // split-spin chains are counted by tiles when every group fits the LDS bases
  bool split_tiles = A.any_split != 0;
  for (int gi = 0; gi < A.ngroups; ++gi)
    if (A.groups[gi].two_s > 1 && A.groups[gi].nchain > kGenChains) split_tiles = false;
  hipLaunchKernelGGL((k_gen<false>), dim3(grid_for(A.nwin, G)), dim3(kBlock), 0, s, A.descs,
                     A.win_bases, A.nchain, A.nwin, A.opstart, A.accmask, A.optime, A.optype,
                     A.op_cap, st, A.flags, split_tiles ? 1 : 0, nullptr);
  for (int gi = 0; split_tiles && gi < A.ngroups; ++gi) {
    const LcTileGroup& g = A.groups[gi];
    if (g.two_s > 1)
      hipLaunchKernelGGL(k_gen_split, dim3(G), dim3(kBlock), 0, s, A.descs, A.grp_chain + g.offset,
                         g.nchain, A.nchain, A.opstart, A.accmask, st);
  }
  mark(LC_PH_SCAN_OPS);
  (void)lc_launch_scan(A.opstart, A.nwin, A.scan_tmp, s);
  hipLaunchKernelGGL(k_chain_bases, dim3(grid_for(A.nchain, 64)), dim3(kBlock), 0, s, A.descs,
                     A.nchain, A.opstart, A.dyn, A.op_bases, A.node_bases, A.totals, A.op_cap,
                     A.node_cap, st, A.flags);
  // 3. write operators
  mark(LC_PH_GEN_WRITE);
  // the windows the writing pass defers are listed in kflat (unused until
  // the flip), their count in kflat[nwin]
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s,
                     reinterpret_cast<unsigned long long*>(A.kflat + A.nwin), 1, 0ull);
  hipLaunchKernelGGL((k_gen<true>), dim3(grid_for(A.nwin, G)), dim3(kBlock), 0, s, A.descs,
                     A.win_bases, A.nchain, A.nwin, A.opstart, A.accmask, A.optime, A.optype,
                     A.op_cap, st, A.flags, 0, A.kflat);
  hipLaunchKernelGGL(k_gen_defer, dim3(G < 2048 ? G : 2048), dim3(kBlock), 0, s, A.descs,
                     A.win_bases, A.nchain, A.nwin, A.opstart, A.accmask, A.optime, A.optype,
                     A.kflat);
  // 4. loop graph and union-find: tiles, then the edges between them
  mark(LC_PH_LINK_TILES);
  hipLaunchKernelGGL(k_init_bnodes, dim3(grid_for(A.nbn, G)), dim3(kBlock), 0, s, A.bn_bases,
                     A.nchain, A.nbn, A.dyn, A.parent, A.flags);
  for (int gi = 0; gi < A.ngroups; ++gi) {
    const LcTileGroup& g = A.groups[gi];
    const int grid = static_cast<int>(g.ntiles < G ? (g.ntiles > 0 ? g.ntiles : 1) : G);
    switch (g.two_s) {
      case 1: launch_tiles<1>(A, g, grid, s); break;
      case 2: launch_tiles<2>(A, g, grid, s); break;
      case 3: launch_tiles<3>(A, g, grid, s); break;
      case 4: launch_tiles<4>(A, g, grid, s); break;
      case 5: launch_tiles<5>(A, g, grid, s); break;
      case 6: launch_tiles<6>(A, g, grid, s); break;
      case 7: launch_tiles<7>(A, g, grid, s); break;
      case 8: launch_tiles<8>(A, g, grid, s); break;
      default: break;
    }
  }
  mark(LC_PH_LINK_CROSS);
  hipLaunchKernelGGL(k_link_cross, dim3(G), dim3(kBlock), 0, s, A.xedge, A.dyncnt, A.xcap,
                     A.totals, A.parent, A.flags);
  if (A.any_split)
    hipLaunchKernelGGL(k_symmetrize, dim3(grid_for(A.nspins, G)), dim3(kBlock), 0, s, A.descs,
                       A.spin_bases, A.nchain, A.nspins, A.dyn, A.totals, A.parent, A.flags);
  // 5. loops: compress the items (fragment reps, boundary nodes), number the roots
  mark(LC_PH_COMPRESS);
  const int64_t nchunks = (A.fcap + A.nbn + kRootChunk - 1) / kRootChunk;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(nchunks + 1, 1024)), dim3(kBlock), 0, s,
                     reinterpret_cast<unsigned long long*>(A.rcnt), nchunks + 1, 0ull);
  hipLaunchKernelGGL(k_compress_items, dim3(G), dim3(kBlock), 0, s, A.frag, A.dyncnt, A.fcap,
                     A.bn_bases, A.nchain, A.nbn, A.dyn, A.parent,
                     reinterpret_cast<unsigned long long*>(A.rcnt), A.flags);
  mark(LC_PH_ROOTS);
  (void)lc_launch_scan(A.rcnt, nchunks, A.scan_tmp, s);
  // a workgroup numbers one chunk of kRootChunk items at a time
  const int groots = static_cast<int>(nchunks < G ? (nchunks > 0 ? nchunks : 1) : G);
  hipLaunchKernelGGL(k_roots_items, dim3(groots), dim3(kBlock), 0, s, A.descs,
                     A.frag, A.dyncnt, A.fcap, A.bn_bases, A.nchain, A.nbn, A.dyn, A.parent, A.acc,
                     A.bacc, A.root_cap, nchunks, A.rcnt, st, A.flags);
  // 6. estimators of the open loops, flips
  mark(LC_PH_ACCUM);
  hipLaunchKernelGGL(A.any_split ? k_accum_hash : k_accum_items, dim3(G), dim3(kBlock), 0, s, A.descs,
                     A.frag, A.dyncnt, A.fcap, A.bn_bases, A.nchain, A.nbn, A.dyn, A.parent, A.acc,
                     A.bacc, A.rcnt + nchunks, A.flags);
  mark(LC_PH_CLUSTER_SUMS);
  // few resident threads: each flushes its partial sums with atomics
  hipLaunchKernelGGL(k_cluster_sums, dim3(G < 2048 ? G : 2048), dim3(kBlock), 0, s, A.nchain,
                     A.rcnt + nchunks, A.root_cap, A.acc, st, A.flags);
  mark(LC_PH_FLIP);
  for (int gi = 0; gi < A.ngroups; ++gi) {
    const LcTileGroup& g = A.groups[gi];
    const int grid = static_cast<int>(g.ntiles < G ? (g.ntiles > 0 ? g.ntiles : 1) : G);
    hipLaunchKernelGGL(g.two_s == 1 ? k_flip_tiles<kBlock> : k_flip_tiles<kFlipWin>, dim3(grid),
                       dim3(kBlock), 0, s, A.descs, A.dyn, A.nchain,
                       A.grp_chain + g.offset, A.grp_tile_base + g.offset, g.nchain, g.ntiles,
                       A.opstart, A.parent, A.acc, A.optype, A.kflat, st, A.flags);
  }
  hipLaunchKernelGGL(k_flip_sites, dim3(grid_for(A.nsites, G)), dim3(kBlock), 0, s, A.descs,
                     A.site_bases, A.nchain, A.nsites, A.dyn, A.parent, A.acc, A.bacc, st, A.flags);
  // 7. next world lines
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

template <int TS>
static void launch_slice_walk(const LcSliceArgs& A, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_slice_walk<TS>), dim3(grid), dim3(kBlock), 0, s, A);
}

hipError_t lc_launch_slices(const LcSliceArgs& A, hipStream_t s) {
  const int64_t n = 2 * A.n_sites * A.n_slices + 2 * A.n_ops;
  hipLaunchKernelGGL(k_slice_init, dim3(grid_for(n, 8192)), dim3(kBlock), 0, s, A.parent, n);
  const int grid = grid_for(A.n_sites * (int64_t(1) << A.w), 8192);
  switch (A.two_s) {
    case 1: launch_slice_walk<1>(A, grid, s); break;
    case 2: launch_slice_walk<2>(A, grid, s); break;
    case 3: launch_slice_walk<3>(A, grid, s); break;
    case 4: launch_slice_walk<4>(A, grid, s); break;
    case 5: launch_slice_walk<5>(A, grid, s); break;
    case 6: launch_slice_walk<6>(A, grid, s); break;
    case 7: launch_slice_walk<7>(A, grid, s); break;
    case 8: launch_slice_walk<8>(A, grid, s); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_slice_compress, dim3(grid_for(n, 8192)), dim3(kBlock), 0, s, A.parent, n);
  return hipGetLastError();
}
