/*
 * sw_oracle.c -- sequential CPU oracle for the Swendsen-Wang cluster update
 * of the two-dimensional Ising model, the benchmark the paper uses for its
 * union-find alone (arXiv:1810.07485, Sec. 4.1).
 *
 * TEST INFRASTRUCTURE ONLY: the plain definition the GPU library's
 * Swendsen-Wang update is checked against.  It shares no code with the
 * library; only the tests and the smoke check load it.
 *
 * One update of the L x L periodic square lattice at coupling K: every
 * nearest-neighbour bond between equal spins is activated with probability
 * p = 1 - exp(-2K); the clusters are the connected components of the active
 * bonds (found here by breadth-first search, each labelled by its smallest
 * site); every cluster flips with probability 1/2.
 *
 * Random numbers (Philox4x32-10, own implementation in lc_oracle.c):
 *  - site i = y L + x holds the bond to its right neighbour (x + 1 mod L)
 *    and to the one below ((y + 1 mod L) L + x); one block per site,
 *    counter (i lo 32, SWBOND << 24 | i >> 32, 0, sweep), word 0 decides
 *    the right bond and word 1 the lower one: active iff the spins are
 *    equal and word < T, T = floor(p 2^32) with p from host libm in FP64;
 *  - the flip bit of a cluster with smallest site c is bit (c mod 128) of
 *    block c / 128 of domain SWFLIP, as for the loops.
 */
#include "lc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

struct orc_sw {
    int64_t L, n;
    double K;
    uint64_t seed, T;
    uint8_t *s; /* 1 = up */
    int64_t sweep;
    int64_t *label; /* last sweep */
};

uint64_t orc_sw_threshold(double K)
{
    double p = 1.0 - exp(-2.0 * K);
    if (!(p > 0.0))
        return 0;
    if (p >= 1.0)
        return (uint64_t)1 << 32;
    return (uint64_t)(p * 4294967296.0);
}

int orc_sw_create(int64_t L, double K, uint64_t seed, orc_sw **out)
{
    if (!out || L < 2 || L > ((int64_t)1 << 20) || !(K >= 0.0) || !isfinite(K))
        return ORC_EINVAL;
    orc_sw *c = (orc_sw *)calloc(1, sizeof(orc_sw));
    if (!c)
        return ORC_ENOMEM;
    c->L = L;
    c->n = L * L;
    c->K = K;
    c->seed = seed;
    c->T = orc_sw_threshold(K);
    c->s = (uint8_t *)malloc(c->n);
    if (!c->s) {
        free(c);
        return ORC_ENOMEM;
    }
    memset(c->s, 1, c->n); /* all spins up */
    *out = c;
    return ORC_OK;
}

void orc_sw_free(orc_sw *c)
{
    if (!c)
        return;
    free(c->s);
    free(c->label);
    free(c);
}

static void bond_words(const orc_sw *c, int64_t i, uint32_t *right, uint32_t *down)
{
    uint32_t ctr[4] = {(uint32_t)i, (ORC_DOM_SWBOND << 24) | (uint32_t)((uint64_t)i >> 32), 0u,
                       (uint32_t)c->sweep},
             o[4];
    orc_philox(c->seed, ctr, o);
    *right = o[0];
    *down = o[1];
}

static int flip_of(const orc_sw *c, int64_t label)
{
    uint64_t q = (uint64_t)label >> 7;
    unsigned b = (unsigned)(label & 127);
    uint32_t ctr[4] = {(uint32_t)q, (ORC_DOM_SWFLIP << 24) | (uint32_t)((q >> 32) & 0xFFFFFFu), 0u,
                       (uint32_t)c->sweep},
             o[4];
    orc_philox(c->seed, ctr, o);
    return (int)((o[b >> 5] >> (b & 31)) & 1u);
}

int orc_sw_sweep(orc_sw *c, orc_sw_stats *st)
{
    if (!c)
        return ORC_EINVAL;
    const int64_t L = c->L, n = c->n;
    uint8_t *act = (uint8_t *)malloc(n); /* bit 0: right bond, bit 1: lower bond */
    int64_t *label = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *size = (int64_t *)calloc(n, sizeof(int64_t));
    if (!act || !label || !queue || !size) {
        free(act);
        free(label);
        free(queue);
        free(size);
        return ORC_ENOMEM;
    }
    /* configuration the sweep starts from; active bonds */
    int64_t energy = 0, mag = 0, nact = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t y = i / L, x = i % L;
        int64_t r = y * L + (x + 1) % L, d = ((y + 1) % L) * L + x;
        uint32_t wr, wd;
        bond_words(c, i, &wr, &wd);
        int si = 2 * c->s[i] - 1;
        energy -= si * (2 * c->s[r] - 1) + si * (2 * c->s[d] - 1);
        mag += si;
        act[i] = (uint8_t)(((c->s[i] == c->s[r]) && wr < c->T) | (((c->s[i] == c->s[d]) && wd < c->T) << 1));
        nact += (act[i] & 1) + (act[i] >> 1);
    }
    /* clusters: breadth-first search from the smallest unvisited site */
    for (int64_t i = 0; i < n; i++)
        label[i] = -1;
    int64_t ncl = 0;
    for (int64_t v = 0; v < n; v++) {
        if (label[v] >= 0)
            continue;
        ncl++;
        int64_t head = 0, tail = 0;
        queue[tail++] = v;
        label[v] = v;
        while (head < tail) {
            int64_t i = queue[head++];
            int64_t y = i / L, x = i % L;
            int64_t nb[4] = {y * L + (x + 1) % L, ((y + 1) % L) * L + x, y * L + (x + L - 1) % L,
                             ((y + L - 1) % L) * L + x};
            int on[4] = {act[i] & 1, act[i] >> 1, act[nb[2]] & 1, act[nb[3]] >> 1};
            for (int q = 0; q < 4; q++)
                if (on[q] && label[nb[q]] < 0) {
                    label[nb[q]] = v;
                    queue[tail++] = nb[q];
                }
        }
    }
    for (int64_t i = 0; i < n; i++)
        size[label[i]]++;
    u128 s2 = 0;
    int64_t mx = 0;
    for (int64_t i = 0; i < n; i++)
        if (size[i]) {
            s2 += (u128)size[i] * (u128)size[i];
            if (size[i] > mx)
                mx = size[i];
        }
    /* flips */
    for (int64_t i = 0; i < n; i++)
        c->s[i] ^= (uint8_t)flip_of(c, label[i]);
    if (st) {
        memset(st, 0, sizeof(*st));
        st->sweep = c->sweep;
        st->energy = energy;
        st->magnetization = mag;
        st->n_active = nact;
        st->n_clusters = ncl;
        st->size2_lo = (uint64_t)s2;
        st->size2_hi = (uint64_t)(s2 >> 64);
        st->max_size = mx;
    }
    free(c->label);
    c->label = label;
    c->sweep++;
    free(act);
    free(queue);
    free(size);
    return ORC_OK;
}

int orc_sw_export(const orc_sw *c, uint8_t *spins, int64_t *labels)
{
    if (!c)
        return ORC_EINVAL;
    if (spins)
        memcpy(spins, c->s, c->n);
    if (labels) {
        if (!c->label)
            return ORC_ESTATE;
        memcpy(labels, c->label, sizeof(int64_t) * c->n);
    }
    return ORC_OK;
}
