/*
 * lc_oracle.h -- sequential CPU oracle for one continuous-time loop-cluster
 * Monte Carlo update of the antiferromagnetic Heisenberg chain
 * (Todo, Matsuo, Shitara, arXiv:1810.07485, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * definition that the GPU library is checked against.  It shares no code,
 * header, table or constant generator with the GPU library; it is compiled
 * with gcc, and only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  Nothing in the product path calls it.
 *
 * Conventions (the readings of the paper are listed in the design doc):
 *  - Sites j in [0, n_sites).  For S=1/2, n_sites = L and bond b joins
 *    sites (b, b+1 mod L)  (Sec. 2, Eq. 1 with periodic boundaries).
 *    For spin S > 1/2 the split-spin mapping of Sec. 5 is used: each spin is
 *    2S subspins, site (j,a) -> 2S*j + a, and bond index ((2S*j)+a)*2S + c
 *    joins (j,a) with (j+1 mod L, c).
 *  - Imaginary time is a 64-bit fixed-point fraction of beta:
 *    tau = beta * t / 2^64, t in [0, 2^64).
 *  - Every random number is one output block of Philox4x32-10 keyed by the
 *    seed and a counter that names the quantity it is for.
 *  - Return codes: 0 on success, negative on error (see ORC_E*).
 */
#ifndef LC_ORACLE_H
#define LC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK        0
#define ORC_EINVAL   -1
#define ORC_ENOMEM   -2
#define ORC_ESTATE   -6
#define ORC_ECAP     -7   /* caller buffer too small; size written back */
#define ORC_EINTERNAL -8  /* BFS and union-find disagree: oracle bug */

/* Philox counter domains (top 8 bits of counter word 1). */
#define ORC_DOM_INIT 0u
#define ORC_DOM_INS  1u
#define ORC_DOM_FLIP 2u
#define ORC_DOM_SYM  3u
#define ORC_DOM_VOTE 4u
#define ORC_DOM_SWBOND 5u  /* Swendsen-Wang bonds (sw_oracle.c) */
#define ORC_DOM_SWFLIP 6u  /* Swendsen-Wang cluster flips */

/* Loop-flip rules: the loop's own Philox bit keyed by its smallest node
 * (label), or the XOR of the votes of all its nodes (vote, Sec. 3.3). */
#define ORC_FLIP_LABEL 0
#define ORC_FLIP_VOTE  1

typedef struct orc_chain orc_chain;

/* Per-sweep statistics: exact integers except where noted. */
typedef struct {
    int64_t sweep;          /* index of the sweep these numbers describe */
    int64_t n_ops;          /* operators (horizontal graphs) in the sweep */
    int64_t n_cand;         /* insertion candidates drawn */
    int64_t n_acc;          /* candidates accepted as diagonal operators */
    int64_t n_kept_in;      /* off-diagonal operators carried into the sweep */
    int64_t n_kept_out;     /* off-diagonal operators after the flip */
    int64_t n_nodes;        /* loop-graph nodes */
    int64_t n_clusters;     /* loops */
    uint64_t sum_m2;        /* sum over loops of m_c^2 */
    uint64_t sum_n0sq;      /* sum over loops of n0_c^2 */
    uint64_t sum_size2_lo;  /* sum over loops of size_c^2 (u128) */
    uint64_t sum_size2_hi;
    uint64_t sum_len2_lo;   /* sum over loops of (len_c >> 32)^2 (u128) */
    uint64_t sum_len2_hi;
    int64_t m_after;        /* sum_j (2 s_j - 1) at tau=0 after the flip */
    int64_t max_size;       /* largest loop, in nodes */
} orc_stats;

/* Philox4x32-10 (Salmon et al., SC'11): out = Philox(key = seed, ctr). */
void orc_philox(uint64_t seed, const uint32_t ctr[4], uint32_t out[4]);

/* Insertion-window rule and Poisson CDF thresholds for one beta.
 * w: windows per bond = 2^w; mu: mean candidates per (bond, window);
 * T[0..*K-1]: T[i] = floor(P(n <= i) * 2^64), last entry 2^64-1. */
int orc_window_table(double beta, int *w, double *mu, uint64_t *T, int *K);

/* Loop-flip bit of a cluster label in a sweep. */
int orc_flip_bit(uint64_t seed, int64_t sweep, int64_t label);
/* Vote of loop-graph node v in a sweep (flip rule ORC_FLIP_VOTE). */
int orc_vote_bit(uint64_t seed, int64_t sweep, int64_t node);
/* Select the loop-flip rule of the following sweeps (ORC_FLIP_*). */
int orc_set_flip_rule(orc_chain *c, int rule);
/* Fourier-mode estimators (on/off for the following sweeps), and those of
 * the most recent sweep: out = chi(pi, 0), chi(pi + 2 pi/L, 0),
 * chi(pi, 2 pi/beta), S(pi + 2 pi/L) (single-sweep improved estimates;
 * ORC_ESTATE when the last sweep did not compute them). */
int orc_set_fourier(orc_chain *c, int on);
int orc_fourier_last(const orc_chain *c, double out[4]);

int  orc_create(int64_t L, int two_s, double beta, uint64_t seed, orc_chain **out);
void orc_free(orc_chain *c);
int  orc_sweep(orc_chain *c, orc_stats *st);
int  orc_sizes(const orc_chain *c, int64_t *n_sites, int64_t *n_bonds,
               int64_t *n_kept, int64_t *sweep);

/* World-line state: s0[n_sites] (0 = down, 1 = up at tau = 0+),
 * bond_off[n_bonds+1] CSR offsets, times[n_kept] off-diagonal operator
 * times in (bond, time) order.  *cap is the capacity of times on input and
 * the number of kept operators on output. */
int orc_export_state(const orc_chain *c, uint8_t *s0, int64_t *bond_off,
                     uint64_t *times, int64_t *cap, int64_t *sweep);
int orc_import_state(orc_chain *c, const uint8_t *s0, const int64_t *bond_off,
                     const uint64_t *times, int64_t sweep);

/* Operators and loop labels of the most recent sweep.
 * op_bond/op_time/op_type0 (type before the flip: 1 = off-diagonal) for
 * *n_ops operators in canonical (bond, time) order; labels for *n_nodes nodes. */
int orc_export_ops(const orc_chain *c, int64_t *op_bond, uint64_t *op_time,
                   uint8_t *op_type0, int64_t *cap);
int orc_export_labels(const orc_chain *c, int64_t *labels, int64_t *cap);
/* Symmetrization permutations of the most recent sweep (split-spin only):
 * perm[n_sites]: top(j,a) is joined to bottom(j, perm[2S*j+a]) -- stored as
 * the global subspin index. */
int orc_export_perm(const orc_chain *c, int64_t *perm, int64_t *cap);

/* ---- Swendsen-Wang update of the 2D Ising model (sw_oracle.c; the
 * union-find benchmark of Sec. 4.1) -------------------------------------- */
typedef struct orc_sw orc_sw;

/* Per sweep: energy -sum_<ij> s_i s_j and magnetization sum_i s_i of the
 * configuration the sweep starts from; active bonds; clusters; sum of the
 * squared cluster sizes (128-bit); largest cluster. */
typedef struct {
    int64_t sweep, energy, magnetization, n_active, n_clusters;
    uint64_t size2_lo, size2_hi;
    int64_t max_size;
} orc_sw_stats;

/* floor(p 2^32) with p = 1 - exp(-2K): a bond is active iff its 32-bit
 * draw is below it (and its spins are equal). */
uint64_t orc_sw_threshold(double K);
int  orc_sw_create(int64_t L, double K, uint64_t seed, orc_sw **out); /* all spins up */
void orc_sw_free(orc_sw *c);
int  orc_sw_sweep(orc_sw *c, orc_sw_stats *st);
/* spins[L*L] (1 = up) now; labels[L*L] of the last sweep's clusters (each
 * the cluster's smallest site, row-major site ids). */
int  orc_sw_export(const orc_sw *c, uint8_t *spins, int64_t *labels);

#ifdef __cplusplus
}
#endif
#endif
