// lc_kernels.h -- launch interface between the engine (host C++) and the
// HIP kernels of one loop-cluster sweep.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lc_device.h"

#define LC_SCAN_BLOCKS 1024
#define LC_ACC_WORDS 4       // words per loop record: nodes + tops << 40, sum hi, sum lo, chain
#define LC_STAT_STRIPES 256  // striped copies of each statistics word (after the words)
#define LC_MAX_TS 8          // 2S of the largest spin (S = 4)

// Linking tiles (bond range x window range of one chain, one workgroup).
#define LC_TILE_OPS 1792     // operators of an S = 1/2 tile held in LDS (four workgroups per CU)
#define LC_TILE_OPS_SPLIT 1536  // operators of a split-spin tile held in LDS
#define LC_TILE_BONDS 256    // owned bonds of a tile
#define LC_TILE_THREADS 256  // (subspin, window) walkers of a tile

// Chains of one spin length form a group: the linking kernel is compiled per
// 2S, and each group is one launch over its chains' tiles.
struct LcTileGroup {
  int two_s;                // 2S of the group's chains
  int nchain;               // chains in the group
  int offset;               // first entry of the group in grp_chain / grp_tile_base
  int64_t ntiles;           // tiles of all the group's chains
};

struct LcSweepArgs {
  lc::ChainDesc* descs;       // nchain descriptors
  const int64_t* win_bases;   // first flat window per chain
  const int64_t* site_bases;  // first flat subspin per chain
  const int64_t* spin_bases;  // first flat spin per chain
  const int64_t* bn_bases;    // first flat boundary node per chain
  int nchain;
  int any_split;              // some chain has S > 1/2
  int64_t nwin, nsites, nspins, nbn;
  int grid_blocks;            // persistent grid size of the node/window loops
  // linking tiles, per spin-length group
  int ngroups;
  LcTileGroup groups[LC_MAX_TS];
  const int* grp_chain;       // chain index of each group entry
  const int64_t* grp_tile_base;  // first tile of each group entry (within its group)
  // flat per-sweep scratch
  int64_t* opstart;           // nwin + 1
  uint32_t* accmask;          // nwin: acceptance mask of each window (<= 32 candidates)
  int64_t* kflat;             // nwin + 1
  uint64_t* optime;           // op_cap
  uint8_t* optype;            // op_cap
  int64_t* parent;            // node_cap
  int64_t* xedge;             // 2 xcap: loop-graph edges between tiles (node, node)
  int64_t* frag;              // 4 fcap: open fragments (rep, size | chain << 16, sum hi, sum lo)
  unsigned long long* acc;    // LC_ACC_WORDS root_cap: loop records
  unsigned long long* bacc;   // nsites: boundary sums of loops rooted at each bottom node
  int64_t op_cap, node_cap, root_cap, xcap, fcap;
  int64_t* rcnt;              // roots per chunk of 4,096 items, scanned ((fcap + nbn) / 4096 + 2)
  unsigned long long* dyncnt; // 4: cross edges, fragments written this sweep
  lc::ChainDyn* dyn;          // nchain
  int64_t* op_bases;          // nchain
  int64_t* node_bases;        // nchain
  int64_t* totals;            // 2: operators, nodes over all chains
  int64_t* scan_tmp;          // LC_SCAN_BLOCKS + 1
  uint64_t* stats;            // nchain * ST_WORDS, then nchain * ST_WORDS * LC_STAT_STRIPES stripes
  uint32_t* flags;            // overflow / error bits
  unsigned long long* ring;   // ring_cap records of nchain * ST_WORDS + 1 words
  uint32_t* ring_ctr;         // next record slot
  uint32_t ring_cap;
  void** events;              // LC_PH_COUNT + 1 hipEvent_t marks, or null
};

// Phases of a sweep, in launch order; events[p] is recorded before phase p
// and events[LC_PH_COUNT] after the last.
enum LcPhase {
  LC_PH_SETUP = 0,
  LC_PH_GEN_COUNT,
  LC_PH_SCAN_OPS,
  LC_PH_GEN_WRITE,
  LC_PH_LINK_TILES,
  LC_PH_LINK_CROSS,
  LC_PH_COMPRESS,
  LC_PH_ROOTS,
  LC_PH_ACCUM,
  LC_PH_CLUSTER_SUMS,
  LC_PH_FLIP,
  LC_PH_SCAN_KEPT,
  LC_PH_COMPACT,
  LC_PH_COUNT
};

// flags bits
#define LC_FLAG_OPS 1u       // operator buffer too small
#define LC_FLAG_NODES 2u     // operator or node buffer too small
#define LC_FLAG_SYM 4u       // split-spin ends cannot be matched
#define LC_FLAG_KEPT 8u      // a chain's kept-operator buffer too small
#define LC_FLAG_ROOTS 16u    // loop-record buffer too small
#define LC_FLAG_TILE 32u     // a linking tile exceeded its LDS capacities
#define LC_FLAG_XEDGE 64u    // cross-edge buffer too small
#define LC_FLAG_FRAG 128u    // fragment buffer too small
#define LC_FLAG_GRAPH 256u   // a union-find word outside the loop graph (internal error)

// Open-boundary time slices of one chain's most recent sweep.
struct LcSliceArgs {
  int64_t L, n_sites;
  int two_s, w;
  int64_t win_base;           // flat window of the chain's bond 0, window 0
  int64_t op_base, n_ops;     // the chain's operators in the flat list
  const int64_t* opstart;
  const uint64_t* optime;
  int64_t n_slices;           // G, 1 <= G <= windows per bond
  int64_t* parent;            // 2 n_sites G + 2 n_ops words
  uint32_t* flags;            // LC_FLAG_GRAPH on an inconsistent graph
};

// Fourier-mode estimators of one chain's most recent sweep (lc_fourier.hip).
struct LcFourierArgs {
  int64_t L, n_sites, n_bonds;
  int two_s, w;
  int64_t win_base;           // flat window of the chain's bond 0, window 0
  int64_t op_base;            // the chain's first flat operator
  int64_t node_base, nbn;     // the chain's first flat node; its boundary nodes
  int64_t n_nodes;
  double beta;
  const int64_t* opstart;
  const uint64_t* optime;
  const int64_t* parent;      // the sweep's union-find words
  int64_t* loopidx;           // n_nodes + 1: loop index of each loop's smallest node (scan)
  int64_t* scan_tmp;          // LC_SCAN_BLOCKS + 1
  double* acc;                // 7 per loop
  double* out;                // 4 sums
};
hipError_t lc_launch_fourier_index(const LcFourierArgs& a, hipStream_t s);
hipError_t lc_launch_fourier_sums(const LcFourierArgs& a, int64_t n_loops, hipStream_t s);

hipError_t lc_launch_sweep(const LcSweepArgs& a, hipStream_t s);
hipError_t lc_launch_slices(const LcSliceArgs& a, hipStream_t s);
hipError_t lc_launch_scan(int64_t* a, int64_t n, int64_t* bsum, hipStream_t s);
hipError_t lc_launch_init_chain(const lc::ChainDesc* d, int64_t n, hipStream_t s);
hipError_t lc_launch_fill_u64(void* p, int64_t n, uint64_t v, hipStream_t s);
