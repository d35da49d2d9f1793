/*
 * lc.h -- C ABI of the MI355X loop-cluster library.
 *
 * One continuous-time loop-cluster Monte Carlo update of the world lines of
 * the antiferromagnetic Heisenberg chain H = J sum_j S_j . S_{j+1} (J = 1,
 * periodic boundaries), after Todo, Matsuo and Shitara, "Parallel loop
 * cluster quantum Monte Carlo simulation of quantum magnets based on global
 * union-find graph algorithm" (arXiv:1810.07485): Sec. 2 (labeling, cluster
 * flip, the continuous-time steps 1-8, union-find), Sec. 3.2 (lock-free
 * union-find on a shared forest) and Sec. 5 (spin S by 2S subspins per spin
 * and (2S)^2 sub-bonds per bond).  Every step runs in HIP kernels on one
 * gfx950 GPU; the host only launches them and reads back a few counters.
 *
 * Conventions
 *  - Every function returns LC_OK (0) or a negative LC_E* code and never
 *    throws.  A failed call leaves the chain unchanged: a sweep is
 *    transactional (the world lines are double-buffered and only the last
 *    kernel of a successful sweep makes the new buffer current).
 *  - Spin S is passed as a double: 0.5, 1.0, 1.5, ... 4.0 (2S integer in 1..8).
 *    L must be even and >= 4, and the sub-bond count (2S)^2 L below 2^32
 *    (bond indices are 32-bit Philox counter words); beta must be finite,
 *    > 0 and <= 8 * 2^32.
 *  - Imaginary time is a 64-bit fixed-point fraction of beta:
 *    tau = beta * t / 2^64.
 *  - Subspin (j, a) of spin j has index 2S j + a; sub-bond
 *    ((2S j) + a) 2S + c joins (j, a) with (j+1 mod L, c).  For S = 1/2
 *    this is bond j joining spins j and j+1.
 *  - Device memory comes from the caller's allocator when one is given (the
 *    Python binding passes PyTorch's caching allocator), otherwise from
 *    hipMalloc.  The library owns what it allocates and frees it in
 *    lc_free / lc_batch_free.  Host buffers are the caller's.
 *  - Work is queued on the caller's HIP stream (NULL = the null stream) and
 *    every call returns after that stream has finished it.
 *  - Calls on one chain or batch must not overlap; different chains may be
 *    driven from different threads when they use different streams.
 *  - Per-sweep scratch (operator lists, union-find parent words, loop
 *    records) belongs to an arena shared by every engine -- a chain run
 *    alone, or a batch -- with the same stream and allocator; sweeps on one
 *    stream run one after another, so the arena is sized for the largest
 *    engine that used it, not for the sum.  Engines sharing an arena are
 *    serialised by a lock.  The arena is freed with the last engine.
 */
#ifndef LC_H
#define LC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LC_OK 0
#define LC_EINVAL -1     /* bad argument (NULL pointer, L odd or < 4, 2S not in 1..8, bad beta) */
#define LC_ENOMEM -2     /* an allocation failed; the object is unchanged */
#define LC_ETOOLARGE -3  /* footprint exceeds the device memory */
#define LC_ECAPACITY -4  /* a caller buffer is too small; the needed size is written back */
#define LC_EDEVICE -5    /* a HIP runtime error */
#define LC_ESTATE -6     /* call not valid in this state (e.g. chain owned by a batch) */

typedef struct lc_chain lc_chain;
typedef struct lc_batch lc_batch;

/* Device allocator supplied by the caller.  alloc returns device memory of at
 * least `bytes` bytes usable on `stream`, or NULL; free releases it. */
typedef struct {
  void *(*alloc)(size_t bytes, void *stream, void *ctx);
  void (*free)(void *ptr, size_t bytes, void *stream, void *ctx);
  void *ctx;
} lc_alloc;

/* Exact integers of the most recent sweep (Sec. 2, step 8).  A loop c has
 * size_c nodes, n0_c nodes at tau = 0+, magnetization
 * m_c = sum over those of (2 s - 1) before the flip, and length len_c
 * (sum of its vertical segments, in ticks of beta / 2^64). */
typedef struct {
  int64_t sweep;         /* index of the sweep described */
  int64_t n_ops;         /* operators (horizontal graphs) */
  int64_t n_cand;        /* insertion candidates drawn */
  int64_t n_acc;         /* candidates accepted (antiparallel) */
  int64_t n_kept_in;     /* off-diagonal operators before the sweep */
  int64_t n_kept_out;    /* off-diagonal operators after the flip */
  int64_t n_nodes;       /* loop-graph nodes */
  int64_t n_clusters;    /* loops */
  uint64_t sum_m2;       /* sum_c m_c^2 */
  uint64_t sum_n0sq;     /* sum_c n0_c^2 */
  uint64_t sum_size2_lo; /* sum_c size_c^2, 128-bit */
  uint64_t sum_size2_hi;
  uint64_t sum_len2_lo;  /* sum_c (len_c >> 32)^2, 128-bit */
  uint64_t sum_len2_hi;
  int64_t m_after;       /* sum_j (2 s_j - 1) at tau = 0+ after the flip */
  int64_t max_size;      /* largest loop in nodes */
} lc_sweep_stats;

/* Observables averaged over the sweeps accumulated since the last reset
 * (FP64, from exact integer sums); N_b = (2S)^2 L sub-bonds:
 *   e           = N_b/(4L) - <n_ops>/(beta L)        energy per spin
 *   chi_u       = beta/(4L) <sum_c m_c^2>             uniform susceptibility
 *   chi_u_plain = beta/(4L) <m_after^2>
 *   s_pi        = <sum_c n0_c^2>/(4L)                 staggered structure factor
 *   chi_s       = beta/(4L) <sum_c ((len_c >> 32)/2^32)^2>  staggered susceptibility */
typedef struct {
  int64_t n_sweeps;
  double e, chi_u, chi_u_plain, s_pi, chi_s;
  double mean_ops, mean_clusters;
} lc_measurement;

/* Device bytes one chain needs when run alone (state plus per-sweep scratch),
 * an estimate of the steady-state allocation (buffers grow on overflow).
 * Used for admission; LC_EINVAL on bad parameters. */
int lc_footprint(int64_t L, double S, double beta, size_t *bytes);

/* The same estimate split into the chain's own world-line state, resident as
 * long as the chain lives, and the per-sweep scratch it asks of its arena
 * (a set of chains on one stream needs the sum of their states plus the
 * scratch of the largest engine). */
int lc_footprint_parts(int64_t L, double S, double beta, size_t *state, size_t *scratch);

/* init_lattice: a chain of L spins S at inverse temperature beta with Philox
 * key `seed`, in the Neel state with a random phase and no operators.
 * The model is Sec. 2, Eq. (1): H = J sum_j S_j . S_{j+1}, J = 1, periodic;
 * spin S > 1/2 is represented by 2S subspins per spin and (2S)^2 sub-bonds
 * per bond (Sec. 5).  The paper leaves the starting configuration open; the
 * Neel state with a Philox phase (bit 0 of the INIT block) is this library's
 * reading, shared with the oracle.  Errors: LC_EINVAL for L odd, L < 4,
 * L >= 2^32, (2S)^2 L >= 2^32, 2S not an integer in 1..8, beta not finite,
 * <= 0 or > 8 2^32; LC_ETOOLARGE when the footprint exceeds the device;
 * LC_ENOMEM, LC_EDEVICE.  alloc may be NULL (hipMalloc); hip_stream may be
 * NULL.  *out receives the handle, owned by the caller until lc_free. */
int lc_init_lattice(int64_t L, double S, double beta, uint64_t seed, const lc_alloc *alloc,
                    void *hip_stream, lc_chain **out);

/* Loop-flip rule of the following sweeps.  LC_FLIP_LABEL (default): a loop
 * flips iff the Philox bit keyed by its smallest node id is 1 (canonical
 * labels make the decision independent of how the union-find ran).
 * LC_FLIP_VOTE: the majority-vote trick of Sec. 3.3 -- every loop-graph
 * node casts a Philox vote in advance and a loop flips iff the XOR of its
 * nodes' votes is 1, a tally that needs no canonical label.  Both flip each
 * loop with probability 1/2 independently of the others; they are different
 * Markov chains with the same stationary distribution.  LC_EINVAL on an
 * unknown rule. */
#define LC_FLIP_LABEL 0
#define LC_FLIP_VOTE 1
int lc_set_flip_rule(lc_chain *c, int rule);

/* update: n_sweeps loop-cluster updates (Sec. 2 steps 1-8).  With
 * accumulate != 0 each sweep's integers are added to the measurement sums.
 * LC_ESTATE when the chain belongs to a batch. */
int lc_update(lc_chain *c, int64_t n_sweeps, int accumulate);

/* measure: FP64 observables from the accumulated sums into *out (Sec. 2,
 * step 8, the measurement after each update; the paper prints no estimator
 * formulas, so the definitions are those of lc_measurement above: the
 * energy from the operator count, the susceptibilities and structure factor
 * from per-loop sums -- the improved estimators of the loop algorithm).
 * Every average is an exact integer sum divided in FP64 at the end.  With no
 * accumulated sweep, n_sweeps = 0 and every other field is 0.  LC_EINVAL on
 * NULL.  Host-only: no device work. */
int lc_measure(const lc_chain *c, lc_measurement *out);

/* update without allocating: for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops).  The same sweeps
 * as lc_update (bit for bit), launched directly on the chain's stream, with
 * every per-sweep buffer carved from the library's static device scratch of
 * 64 MiB per GPU instead of the arena; the chain's own state buffers come
 * from lc_init_lattice.  No device or library allocation happens in the
 * call (the scratch address is looked up once per GPU).  Chains whose
 * per-sweep scratch does not fit in 64 MiB (about L beta <= 1e6 at S = 1/2)
 * are refused with LC_ETOOLARGE before any work, and so is a sweep whose
 * operators outgrow the estimate or the chain's kept-operator buffer (the
 * chain is left unchanged; lc_update can grow them).  Calls on one GPU share
 * the scratch: they must not overlap.  Exports of the operators and labels
 * of these sweeps are not available (LC_ESTATE).  LC_ESTATE for a batch
 * member. */
int lc_update_noalloc(lc_chain *c, int64_t n_sweeps, int accumulate);

/* Integers of the most recent sweep; LC_ESTATE before the first sweep. */
int lc_last_sweep(const lc_chain *c, lc_sweep_stats *out);

/* Forget the accumulated sums. */
int lc_reset_measurements(lc_chain *c);

/* World lines (checkpoint and parity).  s0[n_sites] spins at tau = 0+
 * (1 = up), bond_off[n_bonds + 1] CSR offsets and times[*n_kept] the
 * off-diagonal operators in (bond, time) order, *sweep the next sweep index.
 * *n_kept is the capacity of times on input and the count on output
 * (LC_ECAPACITY if too small; times may be NULL to query sizes).
 * n_sites = 2S L, n_bonds = (2S)^2 L. */
int lc_export_state(const lc_chain *c, uint8_t *s0, int64_t *bond_off, uint64_t *times,
                    int64_t *n_kept, int64_t *sweep);

/* Replace the world lines (same layout as lc_export_state).  Times must be
 * sorted within each bond; the configuration must be a valid world-line
 * configuration (antiparallel spins at every operator, periodic) -- the next
 * sweep reports LC_ESTATE for split spins whose ends cannot be matched.
 * Accumulated measurements are kept. */
int lc_import_state(lc_chain *c, const uint8_t *s0, const int64_t *bond_off, const uint64_t *times,
                    int64_t sweep);

/* Operators of the most recent sweep in canonical (bond, time) order:
 * op_bond, op_time, and their type before (op_type0) and after (op_type1)
 * the flip, 1 = off-diagonal.  *n_ops: capacity in, count out; all arrays
 * NULL queries the count.  Valid until the next sweep of any engine sharing
 * the chain's arena (LC_ESTATE afterwards). */
int lc_export_ops(const lc_chain *c, int64_t *op_bond, uint64_t *op_time, uint8_t *op_type0,
                  uint8_t *op_type1, int64_t *n_ops);

/* Loop labels of the most recent sweep (Sec. 2: loops are the connected
 * components of the graph of world-line fragments, identified by union-find;
 * the label of a loop is its smallest node id, the canonical representative
 * that makes the result independent of the order of the unions, Sec. 3.2):
 * labels[v] = smallest node id of the loop through node v.  Nodes: boundary nodes first (S = 1/2: one per spin;
 * split spins: bottom(x) = x and top(x) = n_sites + x), then operator q has
 * lower node nbn + 2q and upper node nbn + 2q + 1.  *n_nodes: capacity in,
 * count out.  Same validity as lc_export_ops. */
int lc_export_labels(const lc_chain *c, int64_t *labels, int64_t *n_nodes);

/* Symmetrization permutation of the most recent sweep (split spins): top
 * node of subspin x is joined to bottom node perm[x].  *n: capacity in,
 * count out. */
int lc_export_perm(const lc_chain *c, int64_t *perm, int64_t *n);

/* Open-boundary imaginary-time slices of the most recent sweep (Sec. 3.1:
 * each process identifies the loops inside its time window first; the
 * fragments crossing the window's two boundaries are what the global merge
 * joins, Fig. 3 and the butterfly of Sec. 3.3).  The windows of every bond
 * are cut into n_slices (1..2^w) contiguous slices, slice p holding windows
 * [p W / G, (p + 1) W / G).  Inside each slice the loop graph of the sweep's
 * operators is linked with the segments that cross a slice boundary cut:
 * the first event of subspin x in slice p joins the slice's bottom node
 * (p, x), its last event the top node (p, x), a subspin without events in
 * the slice joins the two directly; the components are found by the
 * library's union-find.  Every node gets the smallest id of its slice
 * component, ids numbered 2 ns p + x (bottom), 2 ns p + ns + x (top) and
 * 2 ns G + 2 q + h for node h of the chain's operator q (ns = 2S L):
 * bottom[p ns + x], top[p ns + x] (G ns entries each) and op_labels[2 q + h]
 * (2 n_ops entries).  Two boundary nodes with one label are joined inside
 * their slice; a component without boundary nodes is a loop closed inside
 * it.  *n_ops: capacity of op_labels / 2 in, operators out; all arrays NULL
 * queries the count.  Valid as lc_export_ops; allocates and frees a
 * temporary device array of that many words.  LC_EINVAL for n_slices out
 * of range. */
int lc_slice_tables(const lc_chain *c, int n_slices, int64_t *bottom, int64_t *top,
                    int64_t *op_labels, int64_t *n_ops);

/* Fourier-mode improved estimators of the most recent sweep: the
 * second-moment estimators of the correlation length and the gap, which the
 * paper cites for its S = 1 results (Sec. 5).  Along a loop the staggered
 * spin (-1)^j S^z_j is one value +-1/2, so with Q_c(d, w) the sum over the
 * loop's vertical segments (site j, tau_a to tau_b) of
 * e^{i d j} int e^{i w tau} dtau, chi(pi + d, w) = <sum_c |Q_c|^2> / (4 beta L)
 * and S(pi + d) = <sum_c |P_c|^2> / (4 L), P_c = sum over the loop's nodes at
 * tau = 0+ of e^{i d j}.  Single-sweep estimates (average them over sweeps):
 *   chi_pi    = chi(pi, 0)            (the staggered susceptibility)
 *   chi_pi_q1 = chi(pi + 2 pi / L, 0)
 *   chi_pi_w1 = chi(pi, 2 pi / beta)
 *   s_pi_q1   = S(pi + 2 pi / L)
 * and then xi = (L / 2 pi) sqrt(chi_pi / chi_pi_q1 - 1) and
 * 1 / gap = (beta / 2 pi) sqrt(chi_pi / chi_pi_w1 - 1) from the averages.
 * FP64 sums in a device-dependent order (agree with the oracle to ~1e-10
 * relative, not bit for bit).  Valid as lc_export_labels; allocates and
 * frees 8 bytes per loop-graph node plus 56 per loop of device memory
 * through the chain's allocator (LC_ENOMEM when it cannot), synchronous. */
typedef struct {
  double chi_pi, chi_pi_q1, chi_pi_w1, s_pi_q1;
  int64_t n_loops;
} lc_fourier;
int lc_fourier_last(const lc_chain *c, lc_fourier *out);

void lc_free(lc_chain *c);
const char *lc_strerror(int code);

/* ---- batching: many chains, one launch sequence per sweep ----------------
 * A batch runs every member chain through the same kernels, each kernel
 * walking a flat index space over all members (Sec. 3: independent Markov
 * chains are the preferred parallelism when memory allows).  Member chains
 * keep their own world lines; their results equal their alone-runs bit for
 * bit.  The sweep is captured once as a HIP graph and replayed. */
int lc_batch_create(const lc_alloc *alloc, void *hip_stream, lc_batch **out);
int lc_batch_add(lc_batch *b, lc_chain *c);    /* LC_ESTATE if c is in a batch */
int lc_batch_remove(lc_batch *b, lc_chain *c); /* LC_EINVAL if c is not a member */
int lc_batch_size(const lc_batch *b, int *n);
/* n_sweeps sweeps of every member; accumulate as in lc_update. */
int lc_batch_update(lc_batch *b, int64_t n_sweeps, int accumulate);
/* Launch configuration: persistent grid size (workgroups of 256) used by the
 * node and window loops, and graph capture on/off.  Schedule only: results
 * do not depend on it. */
int lc_batch_set_schedule(lc_batch *b, int grid_blocks, int use_graph);
/* Bytes of device memory held by the per-sweep scratch arena the batch uses
 * (shared with every engine on its stream and allocator).  The arena grows
 * with headroom when a sweep needs more and is released with the last
 * engine that uses it; admission policies bound their budgets with it.
 * Host-only; LC_EINVAL on NULL. */
int lc_batch_scratch_bytes(const lc_batch *b, size_t *bytes);
void lc_batch_free(lc_batch *b);

/* Capacities a chain run alone holds: *kept_cap kept operators per world-line
 * buffer (grown when a sweep keeps more) and *scratch bytes of the per-sweep
 * scratch arena of its engine (0 before its first lone sweep).  Both grow,
 * with headroom, while the chain equilibrates (each growth reallocates and
 * replays a sweep); callers timing sweeps can wait until they stop changing.
 * Host-only; LC_EINVAL on NULL. */
int lc_capacity(const lc_chain *c, int64_t *kept_cap, size_t *scratch);

/* Same launch configuration for a chain run alone. */
int lc_set_schedule(lc_chain *c, int grid_blocks, int use_graph);

/* Autotuner (schedule only): for each of the n_grids candidate grid sizes
 * grids[i] (> 0), runs trial_sweeps (>= 1) real sweeps of the batch with
 * graph replay, not accumulated, timed on the host clock after one warm-up
 * sweep; then keeps the fastest.  *best_grid and *ms_per_sweep (either may be
 * NULL) receive the choice and its time.  The sweeps advance the chains
 * exactly as lc_batch_update(b, n, 0) would. */
int lc_batch_autotune(lc_batch *b, const int *grids, int n_grids, int trial_sweeps, int *best_grid,
                      double *ms_per_sweep);
int lc_autotune(lc_chain *c, const int *grids, int n_grids, int trial_sweeps, int *best_grid,
                double *ms_per_sweep);

/* Linking-tile shape (schedule only: results do not depend on it).  The
 * loop graph is linked and union-found in tiles of spins x windows, local
 * first, then globally (Secs. 3.1-3.2); a tile takes at most max_windows
 * windows per bond (a power of two up to 16; 0: 8 for S = 1/2, 1 for split
 * spins) and about target_ops operators (64..1,792; 0: 1,500 for
 * S = 1/2, 1,400 for split spins), within the LDS capacities.  LC_EINVAL
 * otherwise.  lc_autotune_tiles / lc_batch_autotune_tiles time every shape
 * i (windows[i], targets[i]) with every grid as lc_autotune does (the
 * sweeps advance the chains) and keep the fastest pair: *best_shape (index),
 * *best_grid, *ms_per_sweep (each may be NULL). */
int lc_set_tile(lc_chain *c, int max_windows, int target_ops);
int lc_autotune_tiles(lc_chain *c, const int *windows, const int *targets, int n_shapes,
                      const int *grids, int n_grids, int trial_sweeps, int *best_shape,
                      int *best_grid, double *ms_per_sweep);
int lc_batch_autotune_tiles(lc_batch *b, const int *windows, const int *targets, int n_shapes,
                            const int *grids, int n_grids, int trial_sweeps, int *best_shape,
                            int *best_grid, double *ms_per_sweep);

/* ---- timing -------------------------------------------------------------
 * With profiling on, every sweep is launched directly (no graph) with a HIP
 * event recorded on the chain's (or batch's) stream between its phases, and
 * the host synchronises once per sweep.  lc_profile returns, for each of the
 * lc_phase_count() phases (names from lc_phase_name), the summed
 * milliseconds over the completed sweeps since profiling was switched on, and
 * that sweep count.  Results of the sweeps are unchanged. */
int lc_phase_count(void);
const char *lc_phase_name(int phase);
int lc_set_profiling(lc_chain *c, int on);
int lc_profile(const lc_chain *c, double *ms, int n, int64_t *sweeps);
int lc_batch_set_profiling(lc_batch *b, int on);
int lc_batch_profile(const lc_batch *b, double *ms, int n, int64_t *sweeps);

/* ---- Swendsen-Wang update of the 2D Ising model --------------------------
 * The benchmark the paper runs its union-find on by itself (Sec. 4.1): the
 * L x L square lattice with periodic boundaries at coupling K (energy
 * -sum over nearest-neighbour pairs of s_i s_j, weight exp(-K E)).  One sweep
 * activates each bond between equal spins with probability
 * p = 1 - exp(-2K), finds the clusters of active bonds with the library's
 * lock-free union-find, and flips every cluster with probability 1/2.
 * Sites are numbered i = y L + x.  Random numbers: Philox4x32-10 keyed by the
 * seed; site i draws one block at counter (i lo 32, 5 << 24 | i >> 32, 0,
 * sweep): word 0 < T activates the bond to (x + 1 mod L, y), word 1 < T the
 * bond to (x, y + 1 mod L), T = floor(p 2^32) from FP64 p (2^32 when p = 1);
 * the cluster whose smallest site is c flips with bit c mod 128 of the block
 * at counter (c / 128 lo 32, 6 << 24 | (c / 128) >> 32, 0, sweep).
 * lc_sw_init: L in 2..2^20, K >= 0 finite (LC_EINVAL otherwise); every spin
 * up; alloc may be NULL (hipMalloc), hip_stream may be NULL; about 33 bytes
 * of device memory per site.  lc_sw_update runs n_sweeps sweeps on the
 * stream and returns after they finished; the host reads the statistics once
 * per 64 sweeps.  lc_sw_last: the most recent sweep's integers (LC_ESTATE
 * before the first).  lc_sw_export: spins[L L] (1 = up) now and, if labels
 * is not NULL, labels[L L] of the most recent sweep's clusters, each the
 * cluster's smallest site (host arrays; either may be NULL).  Profiling:
 * with it on, lc_sw_update synchronises after every sweep and times each of
 * its lc_sw_phase_count() kernels (names from lc_sw_phase_name) with HIP
 * events; lc_sw_profile returns their summed milliseconds (n >= the phase
 * count) and the sweep count.  lc_sw_work: tile-local components of the most
 * recent sweep (the records the global phase reads; synchronous device
 * read, LC_ESTATE before the first sweep). */
typedef struct lc_sw lc_sw;
typedef struct {
  int64_t sweep;
  int64_t energy;        /* of the configuration the sweep started from */
  int64_t magnetization; /* sum of s_i, same configuration */
  int64_t n_active;      /* active bonds */
  int64_t n_clusters;
  uint64_t size2_lo, size2_hi; /* sum over clusters of size^2, 128 bit */
  int64_t max_size;
} lc_sw_stats;
int lc_sw_init(int64_t L, double K, uint64_t seed, const lc_alloc *alloc, void *hip_stream,
               lc_sw **out);
int lc_sw_update(lc_sw *c, int64_t n_sweeps);
int lc_sw_last(const lc_sw *c, lc_sw_stats *out);
int lc_sw_export(const lc_sw *c, uint8_t *spins, int64_t *labels);
int lc_sw_set_profiling(lc_sw *c, int on);
int lc_sw_phase_count(void);
const char *lc_sw_phase_name(int phase);
int lc_sw_profile(const lc_sw *c, double *ms, int n, int64_t *sweeps);
int lc_sw_work(const lc_sw *c, int64_t *n_records);
void lc_sw_free(lc_sw *c);

/* ---- measurement probes (ceilings of this device) -----------------------
 * lc_probe_cas: random 8-byte compare-and-swap on an array of 2^log2_words
 * words (10..34), the access of a lock-free union-find hook (Sec. 3.2); about
 * n_cas operations per launch, best of `repeats` timed launches after one
 * warm-up.  Every CAS succeeds and leaves the array unchanged.  *cas_per_s
 * receives the rate and *success_frac (may be NULL) the fraction of CAS that
 * found the expected word (1 by construction).  lc_probe_copy: a streaming
 * device-to-device copy of `bytes` bytes; *gb_per_s counts bytes read plus
 * bytes written per second.  Both allocate and free their own device
 * buffers (hipMalloc), run on hip_stream (may be NULL) and return LC_EINVAL,
 * LC_ENOMEM or LC_EDEVICE on failure. */
int lc_probe_cas(int log2_words, int64_t n_cas, int repeats, void *hip_stream, double *cas_per_s,
                 double *success_frac);
int lc_probe_copy(int64_t bytes, int repeats, void *hip_stream, double *gb_per_s);

/* ---- testing hooks (host code of the library, no GPU needed) ------------
 * The library's host twin of its Philox4x32-10 and its Poisson window rule:
 * w (2^w windows per bond), mu = beta / 2^(w+1) and thresholds
 * T[i] = floor(P(n <= i) 2^64) with T[*K - 1] = 2^64 - 1 (T holds 64). */
int lc_debug_philox(uint64_t seed, const uint32_t ctr[4], uint32_t out[4]);
/* Work counts of the most recent sweep of the chain's own engine (the chain
 * run alone): loop-graph edges between linking tiles and open fragments the
 * tiles left for the global union-find (the benchmark's byte model uses
 * them).  LC_ESTATE before a sweep; synchronous device read. */
int lc_debug_work(const lc_chain *c, int64_t *n_cross, int64_t *n_frags);
int lc_debug_window_table(double beta, int *w, double *mu, uint64_t *T, int *K);

#ifdef __cplusplus
}
#endif
#endif
