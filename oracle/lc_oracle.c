/*
 * lc_oracle.c -- sequential CPU oracle for the continuous-time loop-cluster
 * update of the antiferromagnetic Heisenberg chain
 * (Todo, Matsuo, Shitara, arXiv:1810.07485).
 *
 * TEST INFRASTRUCTURE ONLY: the plain definition the GPU library is checked
 * against.  It shares no code with the GPU library.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * One Monte Carlo step follows the continuous-time procedure of Sec. 2
 * (the enumerated steps 1-8 after Fig. 1):
 *   - walk imaginary time upward carrying the spin configuration;
 *   - an existing off-diagonal operator gets a horizontal graph and flips
 *     the two spins it joins (labeling rule i, step 3);
 *   - candidate horizontal graphs arrive as a Poisson process of rate J/2
 *     per bond (the Delta_tau/2 probability of rule ii in the Trotter limit)
 *     and are kept when the two spins are antiparallel (rule ii/iii, step 5);
 *   - old diagonal operators are not carried over (step 3 keeps only the
 *     off-diagonal ones);
 *   - the loops are the connected components of the graph of world-line
 *     fragments (Sec. 2, the rooted-tree representation), found here by
 *     breadth-first search and cross-checked with a union-find using
 *     union-by-weight and path compression (Sec. 2 and Sec. 3.2 steps 1-7);
 *   - each loop flips with probability 1/2 (cluster flipping, step 7);
 *   - improved estimators are accumulated per loop (step 8).
 *
 * The exponential clock of step 2 (one global clock of rate L/2 picking a
 * uniform bond) is realised as independent per-bond Poisson processes of
 * rate 1/2, which is the same process by superposition; each bond's process
 * is drawn window by window from Philox so that every random number has a
 * fixed address.  The readings are listed in the design doc.
 */
#include "lc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define TWO64 18446744073709551616.0 /* 2^64 as a double */
#define TMAX 64                      /* longest Poisson threshold table */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror and
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of
 * two 32x32->64 multiplications with the key bumped by the Weyl constants
 * between rounds.                                                          */
void orc_philox(uint64_t seed, const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static void philox_u64(uint64_t seed, uint32_t a, uint32_t b, uint32_t c,
                       uint32_t d, uint64_t *x, uint64_t *y)
{
    uint32_t ctr[4] = {a, b, c, d}, o[4];
    orc_philox(seed, ctr, o);
    *x = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    *y = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
}

/* ------------------------------------------------------------------------ */
/* Poisson process of rate 1/2 on one bond over [0, beta): the time axis is
 * cut into W = 2^w equal windows; the count in a window is Poisson with mean
 * mu = beta / (2W) and, given the count, the points are independent and
 * uniform in the window.  w is the smallest w >= 0 with beta / 2^w <= 8.   */
int orc_window_table(double beta, int *w_out, double *mu_out, uint64_t *T, int *K)
{
    if (!(beta > 0.0) || !isfinite(beta) || beta > 8.0 * 4294967296.0)
        return ORC_EINVAL;
    int w = 0;
    while (beta > ldexp(8.0, w))
        w++;
    double mu = ldexp(beta, -w - 1);
    /* cumulative distribution P(n <= i) summed term by term */
    double p = exp(-mu);
    double C = p, Cprev = -1.0;
    int k;
    for (k = 0; k < TMAX; k++) {
        if (k > 0) {
            volatile double pm = p * mu; /* each step rounded on its own */
            p = pm / (double)k;
            volatile double Cs = C + p;
            C = Cs;
        }
        if (C >= 1.0 || k == TMAX - 1 || C == Cprev) {
            T[k] = UINT64_MAX;
            break;
        }
        T[k] = (uint64_t)(C * TWO64);
        Cprev = C;
    }
    *w_out = w;
    *mu_out = mu;
    *K = k + 1;
    return ORC_OK;
}

/* One bit of a 128-bit Philox block of domain dom: block id/128, bit id
 * mod 128 of the block read as words 0..3, least significant first. */
static int domain_bit(uint64_t seed, int64_t sweep, int64_t id, unsigned dom)
{
    uint64_t q = (uint64_t)id >> 7;
    unsigned i = (unsigned)(id & 127);
    uint32_t ctr[4] = {(uint32_t)q, (dom << 24) | (uint32_t)((q >> 32) & 0xFFFFFFu), 0u,
                       (uint32_t)sweep},
             o[4];
    orc_philox(seed, ctr, o);
    return (int)((o[i >> 5] >> (i & 31)) & 1u);
}

/* Majority-vote trick (Sec. 3.3): every node votes in advance; a loop flips
 * iff the XOR of its nodes' votes is 1.  The tally is order-independent,
 * and each loop's decision is a fair bit independent of the other loops'
 * (disjoint sets of independent votes). */
int orc_vote_bit(uint64_t seed, int64_t sweep, int64_t node)
{
    return domain_bit(seed, sweep, node, ORC_DOM_VOTE);
}

int orc_flip_bit(uint64_t seed, int64_t sweep, int64_t label)
{
    uint64_t q = (uint64_t)label >> 7;
    unsigned i = (unsigned)(label & 127);
    uint32_t ctr[4] = {(uint32_t)q, (ORC_DOM_FLIP << 24) | (uint32_t)((q >> 32) & 0xFFFFFFu),
                       0u, (uint32_t)sweep},
             o[4];
    orc_philox(seed, ctr, o);
    return (int)((o[i >> 5] >> (i & 31)) & 1u);
}

/* ------------------------------------------------------------------------ */
struct orc_chain {
    int64_t L;
    int two_s;
    double beta;
    uint64_t seed;
    int64_t n_sites, n_bonds;
    int64_t *bx, *by; /* bond -> its two sites */
    int w;
    double mu;
    uint64_t T[TMAX];
    int K;
    uint8_t *s0;
    int64_t *koff; /* kept off-diagonal operators, CSR by bond */
    uint64_t *ktime;
    int64_t n_kept;
    int64_t sweep;
    int flip_rule; /* ORC_FLIP_LABEL or ORC_FLIP_VOTE */
    int fourier;   /* compute the Fourier-mode estimators of each sweep */
    double last_fourier[4];
    int has_fourier;
    /* last sweep, for inspection */
    int64_t last_n_ops, last_n_nodes;
    int64_t *last_bond;
    uint64_t *last_time;
    uint8_t *last_type0;
    int64_t *last_label;
    int64_t *last_perm;
};

int orc_create(int64_t L, int two_s, double beta, uint64_t seed, orc_chain **out)
{
    if (!out || L < 4 || (L & 1) || two_s < 1 || two_s > 8)
        return ORC_EINVAL;
    /* bond indices are 32-bit Philox counter words */
    if ((int64_t)two_s * two_s * L >= ((int64_t)1 << 32))
        return ORC_EINVAL;
    orc_chain *c = (orc_chain *)calloc(1, sizeof(orc_chain));
    if (!c)
        return ORC_ENOMEM;
    if (orc_window_table(beta, &c->w, &c->mu, c->T, &c->K) != ORC_OK) {
        free(c);
        return ORC_EINVAL;
    }
    c->L = L;
    c->two_s = two_s;
    c->beta = beta;
    c->seed = seed;
    c->n_sites = (int64_t)two_s * L;
    c->n_bonds = (int64_t)two_s * two_s * L;
    c->bx = (int64_t *)malloc(sizeof(int64_t) * c->n_bonds);
    c->by = (int64_t *)malloc(sizeof(int64_t) * c->n_bonds);
    c->s0 = (uint8_t *)malloc(c->n_sites);
    c->koff = (int64_t *)calloc(c->n_bonds + 1, sizeof(int64_t));
    if (!c->bx || !c->by || !c->s0 || !c->koff) {
        orc_free(c);
        return ORC_ENOMEM;
    }
    /* bond ((2S j) + a) 2S + c joins subspin (j,a) with (j+1,c); for S=1/2
     * this is bond j joining sites j and j+1 (Eq. 1, periodic). */
    for (int64_t j = 0; j < L; j++)
        for (int a = 0; a < two_s; a++)
            for (int cc = 0; cc < two_s; cc++) {
                int64_t b = ((int64_t)two_s * j + a) * two_s + cc;
                c->bx[b] = (int64_t)two_s * j + a;
                c->by[b] = (int64_t)two_s * ((j + 1) % L) + cc;
            }
    /* Neel state with a random phase; all subspins of a site equal. */
    uint32_t ctr[4] = {0u, ORC_DOM_INIT << 24, 0u, 0u}, o[4];
    orc_philox(seed, ctr, o);
    int phase = (int)(o[0] & 1u);
    for (int64_t i = 0; i < c->n_sites; i++)
        c->s0[i] = (uint8_t)(((i / two_s) & 1) ^ phase);
    c->n_kept = 0;
    c->sweep = 0;
    *out = c;
    return ORC_OK;
}

int orc_set_flip_rule(orc_chain *c, int rule)
{
    if (!c || (rule != ORC_FLIP_LABEL && rule != ORC_FLIP_VOTE))
        return ORC_EINVAL;
    c->flip_rule = rule;
    return ORC_OK;
}

static void free_last(orc_chain *c)
{
    free(c->last_bond);
    free(c->last_time);
    free(c->last_type0);
    free(c->last_label);
    free(c->last_perm);
    c->last_bond = NULL;
    c->last_time = NULL;
    c->last_type0 = NULL;
    c->last_label = NULL;
    c->last_perm = NULL;
    c->last_n_ops = c->last_n_nodes = 0;
}

void orc_free(orc_chain *c)
{
    if (!c)
        return;
    free_last(c);
    free(c->bx);
    free(c->by);
    free(c->s0);
    free(c->koff);
    free(c->ktime);
    free(c);
}

int orc_sizes(const orc_chain *c, int64_t *n_sites, int64_t *n_bonds, int64_t *n_kept,
              int64_t *sweep)
{
    if (!c)
        return ORC_EINVAL;
    if (n_sites)
        *n_sites = c->n_sites;
    if (n_bonds)
        *n_bonds = c->n_bonds;
    if (n_kept)
        *n_kept = c->n_kept;
    if (sweep)
        *sweep = c->sweep;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* An event on the imaginary-time axis: an existing off-diagonal operator
 * (kind 0) or an insertion candidate (kind 1).  Events are ordered by time;
 * equal times are ordered by bond index, then kind, then rank r (the
 * position within its bond and kind).  Equal times have probability zero in
 * the continuum; the order only has to be fixed.                          */
typedef struct {
    uint64_t t;
    int64_t bond;
    int64_t r;
    int32_t kind;
    int32_t accepted;
    int64_t op; /* canonical operator id, or -1 */
} event;

static int cmp_time_order(const void *pa, const void *pb)
{
    const event *a = (const event *)pa, *b = (const event *)pb;
    if (a->t != b->t)
        return a->t < b->t ? -1 : 1;
    if (a->bond != b->bond)
        return a->bond < b->bond ? -1 : 1;
    if (a->kind != b->kind)
        return a->kind < b->kind ? -1 : 1;
    if (a->r != b->r)
        return a->r < b->r ? -1 : 1;
    return 0;
}

static int cmp_u64_stable(const void *pa, const void *pb)
{
    const uint64_t *a = (const uint64_t *)pa, *b = (const uint64_t *)pb;
    if (a[0] != b[0])
        return a[0] < b[0] ? -1 : 1;
    return a[1] < b[1] ? -1 : (a[1] > b[1]);
}

/* Candidates of one bond in window k, sorted by time (ties: draw order).
 * Returns the count; times into buf (capacity TMAX). */
static int window_candidates(const orc_chain *c, int64_t b, uint64_t k, uint64_t *buf)
{
    uint32_t dom = ORC_DOM_INS << 24;
    uint64_t u, v[TMAX + 1];
    philox_u64(c->seed, (uint32_t)k, dom | 0u, (uint32_t)b, (uint32_t)c->sweep, &u, &v[0]);
    int n = 0;
    while (n < c->K && u >= c->T[n])
        n++;
    for (int i = 1; 2 * i - 1 < n; i++)
        philox_u64(c->seed, (uint32_t)k, dom | (uint32_t)i, (uint32_t)b, (uint32_t)c->sweep,
                   &v[2 * i - 1], &v[2 * i]);
    uint64_t pair[TMAX][2];
    for (int i = 0; i < n; i++) {
        uint64_t t = c->w == 0 ? v[i] : ((k << (64 - c->w)) | (v[i] >> c->w));
        pair[i][0] = t;
        pair[i][1] = (uint64_t)i;
    }
    qsort(pair, (size_t)n, sizeof(pair[0]), cmp_u64_stable);
    for (int i = 0; i < n; i++)
        buf[i] = pair[i][0];
    return n;
}

/* Fisher-Yates shuffle of idx[0..n) driven by the SYM stream of one site;
 * *d counts the draws consumed.  A draw in [0, m) is (u * m) >> 64.      */
static void shuffle_site(const orc_chain *c, int64_t site, int64_t *idx, int n, int *d)
{
    for (int i = n - 1; i >= 1; i--) {
        uint64_t x, y;
        philox_u64(c->seed, (uint32_t)site, (ORC_DOM_SYM << 24) | (uint32_t)(*d / 2), 0u,
                   (uint32_t)c->sweep, &x, &y);
        uint64_t u = (*d % 2 == 0) ? x : y;
        (*d)++;
        int j = (int)(((u128)u * (u128)(uint64_t)(i + 1)) >> 64);
        int64_t tmp = idx[i];
        idx[i] = idx[j];
        idx[j] = tmp;
    }
}

/* graph of world-line fragments: every node has exactly two edge ends.
 * Every edge is a vertical segment of one subspin's world line (esub, from
 * tick et0 to et0 + elen), or a zero-length symmetrization edge (esub -1);
 * esub and et0 are kept only when the Fourier-mode estimators are on. */
typedef struct {
    int64_t *nb;   /* nb[2v], nb[2v+1]: neighbours */
    int64_t n_nodes, n_edges;
    int64_t *eu, *ev;
    u128 *elen;
    uint8_t *fill;
    int64_t *esub;
    uint64_t *et0;
} graph;

static void add_edge(graph *g, int64_t u, int64_t v, u128 len, int64_t sub, uint64_t t0)
{
    int64_t e = g->n_edges++;
    g->eu[e] = u;
    g->ev[e] = v;
    g->elen[e] = len;
    if (g->esub) {
        g->esub[e] = sub;
        g->et0[e] = t0;
    }
    g->nb[2 * u + g->fill[u]++] = v;
    g->nb[2 * v + g->fill[v]++] = u;
}

static int64_t uf_find(int64_t *parent, int64_t x)
{
    int64_t r = x;
    while (parent[r] != r)
        r = parent[r];
    while (parent[x] != r) { /* path compression */
        int64_t nx = parent[x];
        parent[x] = r;
        x = nx;
    }
    return r;
}

/*
 * Fourier-mode improved estimators of the sweep's loops: the second-moment
 * estimators of the correlation length and the gap (the paper cites them
 * for Table 3).  Along a loop the staggered spin (-1)^j S^z_j is one value
 * +-1/2 (every operator joins antiparallel spins), so S^z at momentum
 * pi + d, frequency w, is a sum over loops of +-1/2 times
 *   Q_c(d, w) = sum over the loop's vertical segments (subspin x of site
 *               j = x / 2S, from tau_a to tau_b) of e^{i d j} int e^{i w tau},
 * and with independent signs chi(pi + d, w) = <sum_c |Q_c|^2> / (4 beta L).
 * Three points: (d, w) = (0, 0), (2 pi / L, 0), (0, 2 pi / beta); and the
 * equal-time structure factor S(pi + 2 pi / L) = <sum_c |P_c|^2> / (4 L),
 * P_c = sum over the loop's bottom (tau = 0+) nodes of e^{i d j}.
 * Symmetrization edges have zero length and add nothing.
 */
static int fourier_sums(orc_chain *c, const graph *g, const int64_t *label, int64_t nn, int64_t ns)
{
    const double beta = c->beta, two_pi = 2.0 * acos(-1.0);
    const double d = two_pi / (double)c->L, w = two_pi / beta;
    double *q0 = (double *)calloc(nn > 0 ? nn : 1, sizeof(double));
    double *qd = (double *)calloc(2 * (nn > 0 ? nn : 1), sizeof(double));
    double *qw = (double *)calloc(2 * (nn > 0 ? nn : 1), sizeof(double));
    double *pd = (double *)calloc(2 * (nn > 0 ? nn : 1), sizeof(double));
    if (!q0 || !qd || !qw || !pd) {
        free(q0);
        free(qd);
        free(qw);
        free(pd);
        return ORC_ENOMEM;
    }
    for (int64_t e = 0; e < g->n_edges; e++) {
        if (g->esub[e] < 0)
            continue;
        const int64_t l = label[g->eu[e]];
        const int64_t j = g->esub[e] / c->two_s;
        const u128 t1 = (u128)g->et0[e] + g->elen[e];
        const double fa = ldexp((double)g->et0[e], -64), fb = ldexp((double)t1, -64);
        const double len = ldexp((double)g->elen[e], -64) * beta;
        q0[l] += len;
        qd[2 * l] += cos(d * (double)j) * len;
        qd[2 * l + 1] += sin(d * (double)j) * len;
        /* (e^{i w tau_b} - e^{i w tau_a}) / (i w), w tau = 2 pi f */
        qw[2 * l] += (sin(two_pi * fb) - sin(two_pi * fa)) / w;
        qw[2 * l + 1] -= (cos(two_pi * fb) - cos(two_pi * fa)) / w;
    }
    for (int64_t i = 0; i < ns; i++) {
        const int64_t l = label[i], j = i / c->two_s;
        pd[2 * l] += cos(d * (double)j);
        pd[2 * l + 1] += sin(d * (double)j);
    }
    double s0 = 0, sd = 0, sw = 0, sp = 0;
    for (int64_t v = 0; v < nn; v++) {
        if (label[v] != v)
            continue;
        s0 += q0[v] * q0[v];
        sd += qd[2 * v] * qd[2 * v] + qd[2 * v + 1] * qd[2 * v + 1];
        sw += qw[2 * v] * qw[2 * v] + qw[2 * v + 1] * qw[2 * v + 1];
        sp += pd[2 * v] * pd[2 * v] + pd[2 * v + 1] * pd[2 * v + 1];
    }
    const double L = (double)c->L;
    c->last_fourier[0] = s0 / (4.0 * beta * L);
    c->last_fourier[1] = sd / (4.0 * beta * L);
    c->last_fourier[2] = sw / (4.0 * beta * L);
    c->last_fourier[3] = sp / (4.0 * L);
    c->has_fourier = 1;
    free(q0);
    free(qd);
    free(qw);
    free(pd);
    return ORC_OK;
}

int orc_set_fourier(orc_chain *c, int on)
{
    if (!c)
        return ORC_EINVAL;
    c->fourier = on != 0;
    return ORC_OK;
}

int orc_fourier_last(const orc_chain *c, double out[4])
{
    if (!c || !out)
        return ORC_EINVAL;
    if (!c->has_fourier)
        return ORC_ESTATE;
    for (int k = 0; k < 4; k++)
        out[k] = c->last_fourier[k];
    return ORC_OK;
}

int orc_sweep(orc_chain *c, orc_stats *st)
{
    if (!c)
        return ORC_EINVAL;
    const int64_t nb = c->n_bonds, ns = c->n_sites;
    const uint64_t W = (uint64_t)1 << c->w;
    int rc = ORC_ENOMEM;

    /* ---- 1. candidates of every bond (step 2 and the draw of step 5) --- */
    int64_t *coff = (int64_t *)calloc(nb + 1, sizeof(int64_t));
    uint64_t *ctime = NULL;
    int64_t ccap = 0, ncand = 0;
    uint64_t buf[TMAX];
    if (!coff)
        goto out0;
    for (int64_t b = 0; b < nb; b++) {
        coff[b] = ncand;
        for (uint64_t k = 0; k < W; k++) {
            int n = window_candidates(c, b, k, buf);
            if (ncand + n > ccap) {
                ccap = 2 * (ccap + n) + 1024;
                uint64_t *p = (uint64_t *)realloc(ctime, sizeof(uint64_t) * ccap);
                if (!p)
                    goto out1;
                ctime = p;
            }
            memcpy(ctime + ncand, buf, sizeof(uint64_t) * n);
            ncand += n;
        }
    }
    coff[nb] = ncand;

    /* ---- 2. one walk up the imaginary-time axis (steps 2-6) ------------ */
    int64_t nev = c->n_kept + ncand;
    event *ev = (event *)malloc(sizeof(event) * (nev > 0 ? nev : 1));
    uint8_t *s = (uint8_t *)malloc(ns);
    if (!ev || !s) {
        free(ev);
        free(s);
        goto out1;
    }
    {
        int64_t e = 0;
        for (int64_t b = 0; b < nb; b++) {
            for (int64_t i = c->koff[b]; i < c->koff[b + 1]; i++)
                ev[e++] = (event){c->ktime[i], b, i - c->koff[b], 0, 0, -1};
            for (int64_t i = coff[b]; i < coff[b + 1]; i++)
                ev[e++] = (event){ctime[i], b, i - coff[b], 1, 0, -1};
        }
    }
    qsort(ev, (size_t)nev, sizeof(event), cmp_time_order);
    memcpy(s, c->s0, ns);
    int64_t nacc = 0;
    for (int64_t e = 0; e < nev; e++) {
        int64_t x = c->bx[ev[e].bond], y = c->by[ev[e].bond];
        if (ev[e].kind == 0) { /* off-diagonal: horizontal graph, spins flip */
            s[x] ^= 1;
            s[y] ^= 1;
        } else if (s[x] != s[y]) { /* antiparallel: horizontal graph inserted */
            ev[e].accepted = 1;
            nacc++;
        }
    }
    int64_t nops = c->n_kept + nacc;

    /* ---- 3. operators in canonical order (bond, time, kind, rank) ------ */
    free_last(c);
    c->last_bond = (int64_t *)malloc(sizeof(int64_t) * (nops > 0 ? nops : 1));
    c->last_time = (uint64_t *)malloc(sizeof(uint64_t) * (nops > 0 ? nops : 1));
    c->last_type0 = (uint8_t *)malloc(nops > 0 ? nops : 1);
    int64_t *bop = (int64_t *)calloc(nb + 1, sizeof(int64_t));
    if (!c->last_bond || !c->last_time || !c->last_type0 || !bop) {
        free(bop);
        free(ev);
        free(s);
        goto out1;
    }
    for (int64_t e = 0; e < nev; e++)
        if (ev[e].kind == 0 || ev[e].accepted)
            bop[ev[e].bond + 1]++;
    for (int64_t b = 0; b < nb; b++)
        bop[b + 1] += bop[b];
    {
        /* within a bond, the walk visits operators in (time, kind, rank)
         * order, which is the canonical order within the bond */
        int64_t *fillb = (int64_t *)calloc(nb, sizeof(int64_t));
        if (!fillb) {
            free(bop);
            free(ev);
            free(s);
            goto out1;
        }
        for (int64_t e = 0; e < nev; e++) {
            if (!(ev[e].kind == 0 || ev[e].accepted))
                continue;
            int64_t b = ev[e].bond;
            int64_t k = bop[b] + fillb[b]++;
            ev[e].op = k;
            c->last_bond[k] = b;
            c->last_time[k] = ev[e].t;
            c->last_type0[k] = (uint8_t)(ev[e].kind == 0);
        }
        free(fillb);
    }
    c->last_n_ops = nops;

    /* ---- 4. graph of world-line fragments ------------------------------ */
    const int split = c->two_s > 1;
    const int64_t nbn = split ? 2 * ns : ns; /* boundary nodes */
    const int64_t nn = nbn + 2 * nops;
    c->last_n_nodes = nn;
    graph g;
    memset(&g, 0, sizeof(g));
    g.n_nodes = nn;
    int64_t ne_max = 2 * nops + 2 * ns;
    g.nb = (int64_t *)malloc(sizeof(int64_t) * 2 * nn);
    g.eu = (int64_t *)malloc(sizeof(int64_t) * ne_max);
    g.ev = (int64_t *)malloc(sizeof(int64_t) * ne_max);
    g.elen = (u128 *)malloc(sizeof(u128) * ne_max);
    g.fill = (uint8_t *)calloc(nn > 0 ? nn : 1, 1);
    int64_t *last_at = (int64_t *)malloc(sizeof(int64_t) * ns);
    uint64_t *last_t = (uint64_t *)malloc(sizeof(uint64_t) * ns);
    c->last_perm = (int64_t *)malloc(sizeof(int64_t) * ns);
    c->has_fourier = 0;
    if (c->fourier) {
        g.esub = (int64_t *)malloc(sizeof(int64_t) * ne_max);
        g.et0 = (uint64_t *)malloc(sizeof(uint64_t) * ne_max);
    }
    if (!g.nb || !g.eu || !g.ev || !g.elen || !g.fill || !last_at || !last_t ||
        !c->last_perm || (c->fourier && (!g.esub || !g.et0)))
        goto out2;
    for (int64_t i = 0; i < ns; i++)
        last_at[i] = -1;
    /* walk the events again in time order: each operator joins the
     * previous event on each of its two sites to its lower node. */
    for (int64_t e = 0; e < nev; e++) {
        if (ev[e].op < 0)
            continue;
        int64_t k = ev[e].op;
        int64_t site[2] = {c->bx[ev[e].bond], c->by[ev[e].bond]};
        for (int q = 0; q < 2; q++) {
            int64_t i = site[q];
            if (last_at[i] < 0)
                add_edge(&g, i /* bottom / boundary node */, nbn + 2 * k, (u128)ev[e].t, i, 0);
            else
                add_edge(&g, nbn + 2 * last_at[i] + 1, nbn + 2 * k,
                         (u128)(ev[e].t - last_t[i]), i, last_t[i]);
            last_at[i] = k;
            last_t[i] = ev[e].t;
        }
    }
    for (int64_t i = 0; i < ns; i++) {
        int64_t top = split ? ns + i : i;
        if (last_at[i] < 0)
            add_edge(&g, i, top, (u128)1 << 64, i, 0);
        else
            add_edge(&g, nbn + 2 * last_at[i] + 1, top, ((u128)1 << 64) - (u128)last_t[i], i,
                     last_t[i]);
    }
    /* symmetrization of the subspins of each spin (split-spin only):
     * top(j,a) is joined to bottom(j, pi_j(a)), pi_j drawn uniformly among
     * the permutations that map every up subspin at beta- onto an up
     * subspin at 0+ and every down one onto a down one. */
    if (split) {
        for (int64_t j = 0; j < c->L; j++) {
            int64_t up_t[8], dn_t[8], up_b[8], dn_b[8];
            int nut = 0, ndt = 0, nub = 0, ndb = 0;
            for (int a = 0; a < c->two_s; a++) {
                int64_t i = (int64_t)c->two_s * j + a;
                if (s[i])
                    up_t[nut++] = i;
                else
                    dn_t[ndt++] = i;
                if (c->s0[i])
                    up_b[nub++] = i;
                else
                    dn_b[ndb++] = i;
            }
            if (nut != nub || ndt != ndb) {
                rc = ORC_ESTATE;
                goto out2;
            }
            int d = 0;
            shuffle_site(c, j, up_b, nub, &d);
            shuffle_site(c, j, dn_b, ndb, &d);
            for (int q = 0; q < nut; q++)
                c->last_perm[up_t[q]] = up_b[q];
            for (int q = 0; q < ndt; q++)
                c->last_perm[dn_t[q]] = dn_b[q];
        }
        for (int64_t i = 0; i < ns; i++)
            add_edge(&g, ns + i, c->last_perm[i], (u128)0, -1, 0);
    } else {
        for (int64_t i = 0; i < ns; i++)
            c->last_perm[i] = i;
        /* for S=1/2 the world lines are periodic; the spins after a full
         * walk equal the initial ones */
        for (int64_t i = 0; i < ns; i++)
            if (s[i] != c->s0[i]) {
                rc = ORC_ESTATE;
                goto out2;
            }
    }

    free(ev);
    ev = NULL;
    free(s);
    s = NULL;
    free(g.fill);
    g.fill = NULL;

    /* ---- 5. loops: connected components, labelled by their minimum node */
    {
        int64_t *label = (int64_t *)malloc(sizeof(int64_t) * nn);
        int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * nn);
        int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * nn);
        int64_t *weight = (int64_t *)malloc(sizeof(int64_t) * nn);
        int64_t *minid = (int64_t *)malloc(sizeof(int64_t) * nn);
        if (!label || !queue || !parent || !weight || !minid) {
            free(label);
            free(queue);
            free(parent);
            free(weight);
            free(minid);
            goto out2;
        }
        for (int64_t v = 0; v < nn; v++)
            label[v] = -1;
        int64_t ncl = 0;
        for (int64_t v = 0; v < nn; v++) {
            if (label[v] >= 0)
                continue;
            /* v is the smallest node of a new component */
            ncl++;
            int64_t head = 0, tail = 0;
            queue[tail++] = v;
            label[v] = v;
            while (head < tail) {
                int64_t x = queue[head++];
                for (int q = 0; q < 2; q++) {
                    int64_t y = g.nb[2 * x + q];
                    if (label[y] < 0) {
                        label[y] = v;
                        queue[tail++] = y;
                    }
                }
            }
        }
        /* cross-check: union-find with union-by-weight and path compression */
        for (int64_t v = 0; v < nn; v++) {
            parent[v] = v;
            weight[v] = 1;
        }
        for (int64_t e = 0; e < g.n_edges; e++) {
            int64_t a = uf_find(parent, g.eu[e]), b = uf_find(parent, g.ev[e]);
            if (a == b)
                continue;
            if (weight[a] < weight[b]) {
                int64_t t = a;
                a = b;
                b = t;
            }
            parent[b] = a;
            weight[a] += weight[b];
        }
        for (int64_t v = 0; v < nn; v++)
            minid[v] = INT64_MAX;
        for (int64_t v = 0; v < nn; v++) {
            int64_t r = uf_find(parent, v);
            if (v < minid[r])
                minid[r] = v;
        }
        int bad = 0;
        for (int64_t v = 0; v < nn; v++)
            if (minid[uf_find(parent, v)] != label[v])
                bad = 1;
        free(queue);
        free(parent);
        free(weight);
        free(minid);
        free(g.nb);
        g.nb = NULL;
        if (bad) {
            free(label);
            rc = ORC_EINTERNAL;
            goto out2;
        }
        c->last_label = label;

        /* ---- 6a. Fourier-mode estimators (optional) -------------------- */
        if (c->fourier && fourier_sums(c, &g, label, nn, ns) != ORC_OK)
            goto out2;

        /* ---- 6. improved estimators per loop (before the flip) --------- */
        int64_t *size = (int64_t *)calloc(nn, sizeof(int64_t));
        int64_t *n0 = (int64_t *)calloc(nn, sizeof(int64_t));
        int64_t *m = (int64_t *)calloc(nn, sizeof(int64_t));
        u128 *len = (u128 *)calloc(nn, sizeof(u128));
        if (!size || !n0 || !m || !len) {
            free(size);
            free(n0);
            free(m);
            free(len);
            goto out2;
        }
        for (int64_t v = 0; v < nn; v++)
            size[label[v]]++;
        for (int64_t i = 0; i < ns; i++) { /* bottom (tau = 0+) nodes */
            n0[label[i]]++;
            m[label[i]] += 2 * (int64_t)c->s0[i] - 1;
        }
        for (int64_t e = 0; e < g.n_edges; e++)
            len[label[g.eu[e]]] += g.elen[e];
        u128 s_size2 = 0, s_len2 = 0;
        uint64_t s_m2 = 0, s_n02 = 0;
        int64_t maxsz = 0;
        for (int64_t v = 0; v < nn; v++) {
            if (label[v] != v)
                continue;
            s_size2 += (u128)size[v] * (u128)size[v];
            s_m2 += (uint64_t)(m[v] * m[v]);
            s_n02 += (uint64_t)(n0[v] * n0[v]);
            u128 a = len[v] >> 32;
            s_len2 += a * a;
            if (size[v] > maxsz)
                maxsz = size[v];
        }
        free(size);
        free(n0);
        free(m);
        free(len);

        /* ---- 7. flip every loop with probability 1/2 (step 7) --------- */
        /* flip[l] for every loop l (indexed by its label): its label's bit,
         * or the XOR of its nodes' votes */
        uint8_t *flip = (uint8_t *)calloc(nn > 0 ? nn : 1, 1);
        if (!flip)
            goto out2;
        for (int64_t v = 0; v < nn; v++) {
            if (c->flip_rule == ORC_FLIP_VOTE)
                flip[label[v]] ^= (uint8_t)orc_vote_bit(c->seed, c->sweep, v);
            else if (label[v] == v)
                flip[v] = (uint8_t)orc_flip_bit(c->seed, c->sweep, v);
        }
        int64_t nkept_out = 0;
        uint8_t *type1 = (uint8_t *)malloc(nops > 0 ? nops : 1);
        if (!type1) {
            free(flip);
            goto out2;
        }
        for (int64_t k = 0; k < nops; k++) {
            int fl = flip[label[nbn + 2 * k]];
            int fu = flip[label[nbn + 2 * k + 1]];
            type1[k] = (uint8_t)(c->last_type0[k] ^ fl ^ fu);
            nkept_out += type1[k];
        }
        int64_t mafter = 0;
        for (int64_t i = 0; i < ns; i++) {
            c->s0[i] ^= flip[label[i]];
            mafter += 2 * (int64_t)c->s0[i] - 1;
        }
        free(flip);
        /* the off-diagonal operators are the next world-line configuration */
        uint64_t *nk = (uint64_t *)malloc(sizeof(uint64_t) * (nkept_out > 0 ? nkept_out : 1));
        if (!nk) {
            free(type1);
            goto out2;
        }
        memset(c->koff, 0, sizeof(int64_t) * (nb + 1));
        int64_t q = 0;
        for (int64_t k = 0; k < nops; k++) {
            if (!type1[k])
                continue;
            nk[q++] = c->last_time[k];
            c->koff[c->last_bond[k] + 1]++;
        }
        for (int64_t b = 0; b < nb; b++)
            c->koff[b + 1] += c->koff[b];
        free(type1);
        int64_t nk_in = c->n_kept;
        free(c->ktime);
        c->ktime = nk;
        c->n_kept = nkept_out;

        if (st) {
            memset(st, 0, sizeof(*st));
            st->sweep = c->sweep;
            st->n_ops = nops;
            st->n_cand = ncand;
            st->n_acc = nacc;
            st->n_kept_in = nk_in;
            st->n_kept_out = nkept_out;
            st->n_nodes = nn;
            st->n_clusters = ncl;
            st->sum_m2 = s_m2;
            st->sum_n0sq = s_n02;
            st->sum_size2_lo = (uint64_t)s_size2;
            st->sum_size2_hi = (uint64_t)(s_size2 >> 64);
            st->sum_len2_lo = (uint64_t)s_len2;
            st->sum_len2_hi = (uint64_t)(s_len2 >> 64);
            st->m_after = mafter;
            st->max_size = maxsz;
        }
        c->sweep++;
        rc = ORC_OK;
    }
out2:
    free(g.esub);
    free(g.et0);
    free(g.nb);
    free(g.eu);
    free(g.ev);
    free(g.elen);
    free(g.fill);
    free(last_at);
    free(last_t);
    free(bop);
    free(ev);
    free(s);
out1:
    free(ctime);
    free(coff);
out0:
    return rc;
}

/* ------------------------------------------------------------------------ */
int orc_export_state(const orc_chain *c, uint8_t *s0, int64_t *bond_off, uint64_t *times,
                     int64_t *cap, int64_t *sweep)
{
    if (!c || !cap)
        return ORC_EINVAL;
    int64_t have = *cap;
    *cap = c->n_kept;
    if (sweep)
        *sweep = c->sweep;
    if (s0)
        memcpy(s0, c->s0, c->n_sites);
    if (bond_off)
        memcpy(bond_off, c->koff, sizeof(int64_t) * (c->n_bonds + 1));
    if (times) {
        if (have < c->n_kept)
            return ORC_ECAP;
        memcpy(times, c->ktime, sizeof(uint64_t) * c->n_kept);
    }
    return ORC_OK;
}

int orc_import_state(orc_chain *c, const uint8_t *s0, const int64_t *bond_off,
                     const uint64_t *times, int64_t sweep)
{
    if (!c || !s0 || !bond_off || sweep < 0)
        return ORC_EINVAL;
    if (bond_off[0] != 0)
        return ORC_EINVAL;
    for (int64_t b = 0; b < c->n_bonds; b++) {
        if (bond_off[b + 1] < bond_off[b])
            return ORC_EINVAL;
        for (int64_t i = bond_off[b] + 1; i < bond_off[b + 1]; i++)
            if (times[i] < times[i - 1])
                return ORC_EINVAL;
    }
    int64_t n = bond_off[c->n_bonds];
    uint64_t *t = (uint64_t *)malloc(sizeof(uint64_t) * (n > 0 ? n : 1));
    if (!t)
        return ORC_ENOMEM;
    if (n > 0)
        memcpy(t, times, sizeof(uint64_t) * n);
    free(c->ktime);
    c->ktime = t;
    memcpy(c->koff, bond_off, sizeof(int64_t) * (c->n_bonds + 1));
    memcpy(c->s0, s0, c->n_sites);
    c->n_kept = n;
    c->sweep = sweep;
    free_last(c);
    return ORC_OK;
}

int orc_export_ops(const orc_chain *c, int64_t *op_bond, uint64_t *op_time, uint8_t *op_type0,
                   int64_t *cap)
{
    if (!c || !cap)
        return ORC_EINVAL;
    int64_t have = *cap;
    *cap = c->last_n_ops;
    if (!op_bond && !op_time && !op_type0)
        return ORC_OK;
    if (have < c->last_n_ops)
        return ORC_ECAP;
    for (int64_t k = 0; k < c->last_n_ops; k++) {
        if (op_bond)
            op_bond[k] = c->last_bond[k];
        if (op_time)
            op_time[k] = c->last_time[k];
        if (op_type0)
            op_type0[k] = c->last_type0[k];
    }
    return ORC_OK;
}

int orc_export_labels(const orc_chain *c, int64_t *labels, int64_t *cap)
{
    if (!c || !cap)
        return ORC_EINVAL;
    int64_t have = *cap;
    *cap = c->last_label ? c->last_n_nodes : 0;
    if (!labels)
        return ORC_OK;
    if (!c->last_label)
        return ORC_ESTATE;
    if (have < c->last_n_nodes)
        return ORC_ECAP;
    memcpy(labels, c->last_label, sizeof(int64_t) * c->last_n_nodes);
    return ORC_OK;
}

int orc_export_perm(const orc_chain *c, int64_t *perm, int64_t *cap)
{
    if (!c || !cap)
        return ORC_EINVAL;
    int64_t have = *cap;
    *cap = c->last_perm ? c->n_sites : 0;
    if (!perm)
        return ORC_OK;
    if (!c->last_perm)
        return ORC_ESTATE;
    if (have < c->n_sites)
        return ORC_ECAP;
    memcpy(perm, c->last_perm, sizeof(int64_t) * c->n_sites);
    return ORC_OK;
}
