// lc_sw.hip -- Swendsen-Wang cluster update of the two-dimensional Ising
// model on the library's union-find: the benchmark the paper uses for its
// union-find alone (Sec. 4.1: L x L periodic square lattice at coupling K;
// each bond between equal spins active with probability p = 1 - exp(-2K);
// clusters flipped with probability 1/2).
//
// One sweep:
//   1. k_sw_tile: per 64 x 64 tile of sites (one workgroup): spins into LDS,
//      bond draws (one Philox block per site: word 0 decides the bond to the
//      right neighbour, word 1 the one below; active iff the spins are equal
//      and the word is below T = floor(p 2^32)), unions of the bonds inside
//      the tile in an LDS union-find, local compression, component sizes;
//      every site's parent word gets its component's smallest site, and each
//      component a record (smallest site, size).  Energy, magnetization and
//      active bonds of the configuration are summed on the way.
//   2. k_sw_cross: the bonds leaving a tile (its right column, bottom row),
//      drawn again, unioned in the global forest.
//   3. k_sw_compress: records' sites point at their cluster's smallest site.
//   4. k_sw_sizes, k_sw_roots: cluster sizes from the records; count, sum of
//      squares, largest.
//   5. k_sw_flip: every site's label is parent[parent[i]]; it flips with the
//      label's bit (domain SWFLIP).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "lc.h"
#include "lc_device.h"
#include "lc_uf.h"

namespace {

using lc::philox10;
using lc::u32x4;

constexpr uint32_t kDomBond = 5u, kDomFlip = 6u;
constexpr int kT = 64;               // tile side
constexpr int kTile = kT * kT;       // sites per tile
constexpr int kSwBlock = 256;
constexpr int kRing = 64;            // sweeps per host synchronisation
constexpr int kSwPhases = 6;         // timed kernels of a sweep

enum SwStat { SW_E = 0, SW_M, SW_ACT, SW_NCL, SW_S2LO, SW_S2HI, SW_MAX, SW_FLAGS, SW_WORDS };

struct SwDev {
  int64_t L, n;
  uint64_t seed;
  uint64_t T;             // bond active iff its draw is below T (T = 2^32: always)
  uint32_t sweep;
  uint8_t* spin;           // n, 1 = up
  int64_t* parent;         // n
  unsigned long long* size;  // n: cluster size at its smallest site
  int64_t* rec;            // 2 n: (smallest site of a tile component, size)
  unsigned long long* nrec;
  unsigned long long* st;  // SW_WORDS
};

__device__ inline u32x4 bond_draw(const SwDev& S, int64_t i) {
  return philox10(S.seed, static_cast<uint32_t>(i),
                  (kDomBond << 24) | static_cast<uint32_t>(static_cast<uint64_t>(i) >> 32), 0u,
                  S.sweep);
}

__device__ inline uint32_t cluster_flip(const SwDev& S, int64_t label) {
  const uint64_t q = static_cast<uint64_t>(label) >> 7;
  const uint32_t b = static_cast<uint32_t>(label & 127);
  const u32x4 r = philox10(S.seed, static_cast<uint32_t>(q),
                           (kDomFlip << 24) | static_cast<uint32_t>((q >> 32) & 0xFFFFFFu), 0u, S.sweep);
  const uint32_t w = (b >> 5) == 0 ? r.x : ((b >> 5) == 1 ? r.y : ((b >> 5) == 2 ? r.z : r.w));
  return (w >> (b & 31)) & 1u;
}

__device__ inline int64_t block_sum(int64_t v, int64_t* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wv] = v;
  __syncthreads();
  int64_t t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kSwBlock / 64; ++w) t += sh[w];
  __syncthreads();
  return t;  // valid in thread 0
}

__global__ __launch_bounds__(kSwBlock) void k_sw_tile(SwDev S) {
  __shared__ uint32_t lpar[kTile];
  __shared__ uint32_t lsize[kTile];
  __shared__ uint8_t sp[(kT + 1) * (kT + 1)];  // tile spins and the right / lower neighbours
  __shared__ int64_t red[kSwBlock / 64];
  __shared__ int nrep;
  __shared__ int64_t rbase;
  const int64_t L = S.L, ntx = (L + kT - 1) / kT;
  const int tid = threadIdx.x;
  int64_t e_acc = 0, m_acc = 0, a_acc = 0;
  for (int64_t t = blockIdx.x; t < ntx * ntx; t += gridDim.x) {
    const int64_t x0 = (t % ntx) * kT, y0 = (t / ntx) * kT;
    const int nx = static_cast<int>(std::min<int64_t>(kT, L - x0));
    const int ny = static_cast<int>(std::min<int64_t>(kT, L - y0));
    for (int k = tid; k < (nx + 1) * (ny + 1); k += kSwBlock) {
      const int ly = k / (nx + 1), lx = k - ly * (nx + 1);
      const int64_t y = (y0 + ly) % L, x = (x0 + lx) % L;
      sp[ly * (kT + 1) + lx] = S.spin[y * L + x];
    }
    for (int u = tid; u < nx * ny; u += kSwBlock) {
      lpar[u] = static_cast<uint32_t>(u);
      lsize[u] = 0;
    }
    if (tid == 0) nrep = 0;
    __syncthreads();
    // bonds: energy, magnetization, active count; unions inside the tile
    for (int u = tid; u < nx * ny; u += kSwBlock) {
      const int ly = u / nx, lx = u - ly * nx;
      const int64_t i = (y0 + ly) * L + x0 + lx;
      const int si = sp[ly * (kT + 1) + lx], sr = sp[ly * (kT + 1) + lx + 1], sd = sp[(ly + 1) * (kT + 1) + lx];
      const u32x4 w = bond_draw(S, i);
      const int zi = 2 * si - 1;
      e_acc -= zi * (2 * sr - 1) + zi * (2 * sd - 1);
      m_acc += zi;
      const bool ar = si == sr && w.x < S.T, ad = si == sd && w.y < S.T;  // u32 vs u64 compare
      a_acc += (ar ? 1 : 0) + (ad ? 1 : 0);
      if (ar && lx + 1 < nx) lc::lunion(lpar, u, u + 1);
      if (ad && ly + 1 < ny) lc::lunion(lpar, u, u + nx);
    }
    __syncthreads();
    // compression: roots found read-only, then written
    uint32_t roots[kTile / kSwBlock];
#pragma unroll
    for (int k = 0; k < kTile / kSwBlock; ++k) {
      const int u = tid + k * kSwBlock;
      uint32_t r = static_cast<uint32_t>(u);
      if (u < nx * ny)
        while (lpar[r] != r) r = lpar[r];
      roots[k] = r;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTile / kSwBlock; ++k) {
      const int u = tid + k * kSwBlock;
      if (u < nx * ny) {
        lpar[u] = roots[k];
        atomicAdd(lsize + roots[k], 1u);
        if (roots[k] == static_cast<uint32_t>(u)) atomicAdd(&nrep, 1);
      }
    }
    __syncthreads();
    if (tid == 0) rbase = static_cast<int64_t>(atomicAdd(S.nrec, static_cast<unsigned long long>(nrep)));
    __syncthreads();
    if (tid == 0) nrep = 0;
    __syncthreads();
    // parent words: the component's smallest site (local order is global order)
    for (int u = tid; u < nx * ny; u += kSwBlock) {
      const uint32_t r = lpar[u];
      const int64_t gr = (y0 + r / nx) * L + x0 + r % nx;
      S.parent[(y0 + u / nx) * L + x0 + u % nx] = gr;
      if (r == static_cast<uint32_t>(u)) {
        const int64_t k = rbase + atomicAdd(&nrep, 1);
        S.rec[2 * k] = gr;
        S.rec[2 * k + 1] = lsize[u];
      }
    }
    __syncthreads();
  }
  const int64_t e = block_sum(e_acc, red), m = block_sum(m_acc, red), a = block_sum(a_acc, red);
  if (tid == 0) {
    atomicAdd(S.st + SW_E, static_cast<unsigned long long>(e));
    atomicAdd(S.st + SW_M, static_cast<unsigned long long>(m));
    atomicAdd(S.st + SW_ACT, static_cast<unsigned long long>(a));
  }
}

// Bonds leaving a tile: the right bond of each tile's last column and the
// lower bond of its last row (index space: column bonds, then row bonds).
__global__ __launch_bounds__(kSwBlock) void k_sw_cross(SwDev S) {
  const int64_t L = S.L, nb = (L + kT - 1) / kT, half = nb * L;
  uint32_t* flags = reinterpret_cast<uint32_t*>(S.st + SW_FLAGS);
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * kSwBlock + threadIdx.x; k < 2 * half;
       k += static_cast<int64_t>(gridDim.x) * kSwBlock) {
    const bool col = k < half;
    const int64_t q = col ? k : k - half, b = q / L, o = q - b * L;
    const int64_t edge = std::min<int64_t>(b * kT + kT - 1, L - 1);
    const int64_t x = col ? edge : o, y = col ? o : edge, i = y * L + x;
    const int64_t j = col ? y * L + (x + 1 == L ? 0 : x + 1) : (y + 1 == L ? 0 : y + 1) * L + x;
    const u32x4 w = bond_draw(S, i);
    if (S.spin[i] == S.spin[j] && (col ? w.x : w.y) < S.T) lc::uf_union(S.parent, i, j, S.n, flags);
  }
}

// Each record's site points at its cluster's smallest site (read-only walk,
// then one write); its size counter is cleared.
__global__ __launch_bounds__(kSwBlock) void k_sw_compress(SwDev S) {
  const int64_t nr = static_cast<int64_t>(*S.nrec);
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * kSwBlock + threadIdx.x; k < nr;
       k += static_cast<int64_t>(gridDim.x) * kSwBlock) {
    const int64_t g = S.rec[2 * k];
    int64_t r = g, p = S.parent[g];
    while (p != r && p >= 0 && p < S.n) {
      r = p;
      p = S.parent[r];
    }
    S.parent[g] = r;
    S.size[g] = 0;
  }
}

// Cluster sizes: every record adds its tile component's size at its
// cluster's smallest site.  Near K_c one cluster spans most tiles: its
// records are a few in every wave, and one global atomic per wave to one
// word serialises (device-scope atomics execute at the memory side).  A
// block therefore sums a chunk of records per cluster in an LDS hash table
// (open addressing, 64-bit CAS on the key), then adds each distinct
// cluster's sum once.
constexpr int kHash = 2048;                 // slots; a chunk fills at most half
constexpr int kHashChunk = kHash / 2;       // records per block and step
constexpr unsigned long long kEmpty = ~0ull;

__global__ __launch_bounds__(kSwBlock) void k_sw_sizes(SwDev S) {
  __shared__ unsigned long long hkey[kHash];
  __shared__ unsigned long long hval[kHash];
  const int64_t nr = static_cast<int64_t>(*S.nrec);
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kHashChunk; base < nr;
       base += static_cast<int64_t>(gridDim.x) * kHashChunk) {
    for (int h = threadIdx.x; h < kHash; h += kSwBlock) {
      hkey[h] = kEmpty;
      hval[h] = 0;
    }
    __syncthreads();
    const int64_t end = base + kHashChunk < nr ? base + kHashChunk : nr;
    for (int64_t k = base + threadIdx.x; k < end; k += kSwBlock) {
      const unsigned long long key = static_cast<unsigned long long>(S.parent[S.rec[2 * k]]);
      const unsigned long long val = static_cast<unsigned long long>(S.rec[2 * k + 1]);
      // Fibonacci hash of the site; at most kHashChunk keys, so a free slot exists
      uint32_t h = static_cast<uint32_t>((key * 0x9E3779B97F4A7C15ull) >> 53) & (kHash - 1);
      for (;;) {
        const unsigned long long old = atomicCAS(hkey + h, kEmpty, key);
        if (old == kEmpty || old == key) {
          atomicAdd(hval + h, val);
          break;
        }
        h = (h + 1) & (kHash - 1);
      }
    }
    __syncthreads();
    for (int h = threadIdx.x; h < kHash; h += kSwBlock)
      if (hkey[h] != kEmpty) atomicAdd(S.size + hkey[h], hval[h]);
    __syncthreads();  // the table is cleared for the next chunk
  }
}

__global__ __launch_bounds__(kSwBlock) void k_sw_roots(SwDev S) {
  const int64_t nr = static_cast<int64_t>(*S.nrec);
  uint64_t cnt = 0, s2lo = 0, s2hi = 0, mx = 0;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * kSwBlock + threadIdx.x; k < nr;
       k += static_cast<int64_t>(gridDim.x) * kSwBlock) {
    const int64_t g = S.rec[2 * k];
    if (S.parent[g] != g) continue;  // not a cluster's smallest site
    const uint64_t sz = S.size[g];
    cnt += 1;
    const uint64_t q = sz * sz, qh = __umul64hi(sz, sz);
    s2lo += q;
    s2hi += qh + (s2lo < q ? 1u : 0u);
    mx = sz > mx ? sz : mx;
  }
  for (int o = 32; o > 0; o >>= 1) {
    cnt += __shfl_xor(cnt, o);
    const uint64_t lo = __shfl_xor(s2lo, o), hi = __shfl_xor(s2hi, o), m = __shfl_xor(mx, o);
    s2lo += lo;
    s2hi += hi + (s2lo < lo ? 1u : 0u);
    mx = m > mx ? m : mx;
  }
  if ((threadIdx.x & 63) == 0 && cnt) {
    atomicAdd(S.st + SW_NCL, static_cast<unsigned long long>(cnt));
    lc::atomic_add_u128(S.st + SW_S2LO, S.st + SW_S2HI, s2lo, s2hi);
    atomicMax(S.st + SW_MAX, static_cast<unsigned long long>(mx));
  }
}

__global__ __launch_bounds__(kSwBlock) void k_sw_flip(SwDev S) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kSwBlock + threadIdx.x; i < S.n;
       i += static_cast<int64_t>(gridDim.x) * kSwBlock) {
    const int64_t label = S.parent[S.parent[i]];
    S.spin[i] ^= static_cast<uint8_t>(cluster_flip(S, label));
  }
}

__global__ void k_sw_fill(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_sw_record(const unsigned long long* st, unsigned long long* ring, uint32_t slot) {
  if (threadIdx.x < SW_WORDS) ring[static_cast<int64_t>(slot) * SW_WORDS + threadIdx.x] = st[threadIdx.x];
}

int grid_of(int64_t n, int cap) {
  int64_t b = (n + kSwBlock - 1) / kSwBlock;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(b, cap)));
}

}  // namespace

struct lc_sw {
  int64_t L = 0, n = 0;
  double K = 0;
  uint64_t seed = 0;
  uint64_t T = 0;
  uint32_t sweep = 0;
  hipStream_t s = nullptr;
  lc_alloc alloc{};
  bool user = false;
  uint8_t* spin = nullptr;
  int64_t* parent = nullptr;
  unsigned long long* size = nullptr;
  int64_t* rec = nullptr;
  unsigned long long* dev = nullptr;  // nrec, stats, ring
  lc_sw_stats last{};
  bool has_last = false;
  double phase_ms[kSwPhases] = {};   // per kernel, summed (profiling)
  int64_t prof_sweeps = 0;
  bool profiling = false;
};

namespace {

void* sw_get(lc_sw* c, size_t bytes) {
  void* p = nullptr;
  if (c->user) return c->alloc.alloc(bytes, c->s, c->alloc.ctx);
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void sw_put(lc_sw* c, void* p, size_t bytes) {
  if (!p) return;
  if (c->user)
    c->alloc.free(p, bytes, c->s, c->alloc.ctx);
  else
    (void)hipFree(p);
}

constexpr int64_t kDevWords = 1 + SW_WORDS + static_cast<int64_t>(kRing) * SW_WORDS;

SwDev sw_dev(const lc_sw* c) {
  SwDev d;
  d.L = c->L;
  d.n = c->n;
  d.seed = c->seed;
  d.T = c->T;
  d.sweep = c->sweep;
  d.spin = c->spin;
  d.parent = c->parent;
  d.size = c->size;
  d.rec = c->rec;
  d.nrec = c->dev;
  d.st = c->dev + 1;
  return d;
}

}  // namespace

extern "C" {

int lc_sw_init(int64_t L, double K, uint64_t seed, const lc_alloc* alloc, void* hip_stream,
               lc_sw** out) {
  if (!out || L < 2 || L > (int64_t(1) << 20) || !(K >= 0.0) || !std::isfinite(K)) return LC_EINVAL;
  if (alloc && (!alloc->alloc || !alloc->free)) return LC_EINVAL;
  *out = nullptr;
  lc_sw* c = new (std::nothrow) lc_sw();
  if (!c) return LC_ENOMEM;
  c->L = L;
  c->n = L * L;
  c->K = K;
  c->seed = seed;
  const double p = 1.0 - std::exp(-2.0 * K);
  // floor(p 2^32) in FP64; p = 1 gives 2^32, above every draw
  c->T = !(p > 0.0) ? 0u : (p >= 1.0 ? (uint64_t(1) << 32) : static_cast<uint64_t>(p * 4294967296.0));
  c->s = static_cast<hipStream_t>(hip_stream);
  if (alloc) {
    c->alloc = *alloc;
    c->user = true;
  }
  c->spin = static_cast<uint8_t*>(sw_get(c, c->n));
  c->parent = static_cast<int64_t*>(sw_get(c, c->n * sizeof(int64_t)));
  c->size = static_cast<unsigned long long*>(sw_get(c, c->n * sizeof(unsigned long long)));
  c->rec = static_cast<int64_t*>(sw_get(c, 2 * c->n * sizeof(int64_t)));
  c->dev = static_cast<unsigned long long*>(sw_get(c, kDevWords * sizeof(unsigned long long)));
  if (!c->spin || !c->parent || !c->size || !c->rec || !c->dev) {
    lc_sw_free(c);
    return LC_ENOMEM;
  }
  if (hipMemsetAsync(c->spin, 1, c->n, c->s) != hipSuccess || hipStreamSynchronize(c->s) != hipSuccess) {
    lc_sw_free(c);
    return LC_EDEVICE;
  }
  *out = c;
  return LC_OK;
}

int lc_sw_update(lc_sw* c, int64_t n_sweeps) {
  if (!c || n_sweeps < 0) return LC_EINVAL;
  hipEvent_t ev[kSwPhases + 1] = {};
  if (c->profiling)
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) {
        for (auto& f : ev)
          if (f) (void)hipEventDestroy(f);
        return LC_EDEVICE;
      }
  int rc = LC_OK;
  std::vector<unsigned long long> h(static_cast<size_t>(kRing) * SW_WORDS);
  const int64_t ntx = (c->L + kT - 1) / kT;
  for (int64_t done = 0; done < n_sweeps && rc == LC_OK;) {
    const int chunk = static_cast<int>(std::min<int64_t>(c->profiling ? 1 : kRing, n_sweeps - done));
    for (int q = 0; q < chunk; ++q) {
      SwDev d = sw_dev(c);
      d.sweep = c->sweep + static_cast<uint32_t>(q);
      int e = 0;
      auto mark = [&]() {
        if (c->profiling) (void)hipEventRecord(ev[e++], c->s);
      };
      hipLaunchKernelGGL(k_sw_fill, dim3(1), dim3(64), 0, c->s, c->dev, int64_t(1 + SW_WORDS), 0ull);
      mark();
      hipLaunchKernelGGL(k_sw_tile, dim3(static_cast<int>(std::min<int64_t>(ntx * ntx, 8192))),
                         dim3(kSwBlock), 0, c->s, d);
      mark();
      hipLaunchKernelGGL(k_sw_cross, dim3(grid_of(2 * ntx * c->L, 8192)), dim3(kSwBlock), 0, c->s, d);
      mark();
      hipLaunchKernelGGL(k_sw_compress, dim3(grid_of(c->n, 8192)), dim3(kSwBlock), 0, c->s, d);
      mark();
      hipLaunchKernelGGL(k_sw_sizes, dim3(static_cast<int>(std::min<int64_t>((c->n + kHashChunk - 1) / kHashChunk, 4096))),
                         dim3(kSwBlock), 0, c->s, d);
      mark();
      hipLaunchKernelGGL(k_sw_roots, dim3(grid_of(c->n, 2048)), dim3(kSwBlock), 0, c->s, d);
      mark();
      hipLaunchKernelGGL(k_sw_flip, dim3(grid_of(c->n, 8192)), dim3(kSwBlock), 0, c->s, d);
      mark();
      hipLaunchKernelGGL(k_sw_record, dim3(1), dim3(64), 0, c->s, c->dev + 1,
                         c->dev + 1 + SW_WORDS, static_cast<uint32_t>(q));
    }
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h.data(), c->dev + 1 + SW_WORDS, chunk * SW_WORDS * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, c->s) != hipSuccess ||
        hipStreamSynchronize(c->s) != hipSuccess) {
      rc = LC_EDEVICE;
      break;
    }
    for (int q = 0; q < chunk; ++q) {
      const unsigned long long* r = h.data() + q * SW_WORDS;
      if (r[SW_FLAGS]) {
        rc = LC_EDEVICE;  // inconsistent forest: internal error
        break;
      }
      lc_sw_stats& st = c->last;
      st.sweep = c->sweep;
      st.energy = static_cast<int64_t>(r[SW_E]);
      st.magnetization = static_cast<int64_t>(r[SW_M]);
      st.n_active = static_cast<int64_t>(r[SW_ACT]);
      st.n_clusters = static_cast<int64_t>(r[SW_NCL]);
      st.size2_lo = r[SW_S2LO];
      st.size2_hi = r[SW_S2HI];
      st.max_size = static_cast<int64_t>(r[SW_MAX]);
      c->has_last = true;
      c->sweep += 1;
      ++done;
    }
    if (c->profiling && rc == LC_OK) {
      for (int k = 0; k < kSwPhases; ++k) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) {
          rc = LC_EDEVICE;
          break;
        }
        c->phase_ms[k] += ms;
      }
      c->prof_sweeps += 1;
    }
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return rc;
}

int lc_sw_last(const lc_sw* c, lc_sw_stats* out) {
  if (!c || !out) return LC_EINVAL;
  if (!c->has_last) return LC_ESTATE;
  *out = c->last;
  return LC_OK;
}

int lc_sw_export(const lc_sw* c, uint8_t* spins, int64_t* labels) {
  if (!c) return LC_EINVAL;
  if (labels && !c->has_last) return LC_ESTATE;
  if (spins && hipMemcpy(spins, c->spin, c->n, hipMemcpyDeviceToHost) != hipSuccess) return LC_EDEVICE;
  if (labels) {
    std::vector<int64_t> p(static_cast<size_t>(c->n));
    if (hipMemcpy(p.data(), c->parent, c->n * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
      return LC_EDEVICE;
    for (int64_t i = 0; i < c->n; ++i) {
      const int64_t q = p[i];
      if (q < 0 || q >= c->n || p[q] < 0 || p[q] >= c->n) return LC_EDEVICE;
      labels[i] = p[q];
    }
  }
  return LC_OK;
}

int lc_sw_set_profiling(lc_sw* c, int on) {
  if (!c) return LC_EINVAL;
  c->profiling = on != 0;
  for (double& v : c->phase_ms) v = 0;
  c->prof_sweeps = 0;
  return LC_OK;
}

int lc_sw_phase_count(void) { return kSwPhases; }

const char* lc_sw_phase_name(int phase) {
  static const char* const names[kSwPhases] = {"tiles", "cross", "compress", "sizes", "roots", "flip"};
  return phase >= 0 && phase < kSwPhases ? names[phase] : nullptr;
}

int lc_sw_profile(const lc_sw* c, double* ms, int n, int64_t* sweeps) {
  if (!c || !ms || n < kSwPhases) return LC_EINVAL;
  for (int k = 0; k < kSwPhases; ++k) ms[k] = c->phase_ms[k];
  if (sweeps) *sweeps = c->prof_sweeps;
  return LC_OK;
}

int lc_sw_work(const lc_sw* c, int64_t* n_records) {
  if (!c || !n_records) return LC_EINVAL;
  if (!c->has_last) return LC_ESTATE;
  unsigned long long v = 0;
  if (hipMemcpyAsync(&v, c->dev, sizeof(v), hipMemcpyDeviceToHost, c->s) != hipSuccess ||
      hipStreamSynchronize(c->s) != hipSuccess)
    return LC_EDEVICE;
  *n_records = static_cast<int64_t>(v);
  return LC_OK;
}

void lc_sw_free(lc_sw* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->s);
  sw_put(c, c->spin, c->n);
  sw_put(c, c->parent, c->n * sizeof(int64_t));
  sw_put(c, c->size, c->n * sizeof(unsigned long long));
  sw_put(c, c->rec, 2 * c->n * sizeof(int64_t));
  sw_put(c, c->dev, kDevWords * sizeof(unsigned long long));
  delete c;
}

}  // extern "C"
