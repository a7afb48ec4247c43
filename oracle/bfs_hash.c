/*
 * ORACLE (test infrastructure only). Plain, slow, obviously correct CPU BFS.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library. The GPU path never calls it, and it shares no
 * code, header or table with the GPU path: it has its own packing, its own
 * hash set and its own generator application.
 *
 * What it computes (paper, section "Reminder on Cayley graphs, diameters,
 * growth", definition of Growth): the number of vertices at each distance m
 * from a fixed start vertex, gamma(m) = |{v : d(v, v0) = m}|, where d is the
 * shortest-path length and an edge joins v and v.g for every generator g
 * (section "Examples and Tutorials": generators are applied to state
 * vectors; one-line notation, 0-based).
 *
 * Action convention (a reading; the paper only says generators act on
 * vectors): gather, t[i] = s[g[i]].
 *
 * Algorithm: textbook breadth-first search. visited = {v0}; for every state
 * of the current layer and every generator in the given order, form the
 * neighbour; if it has not been visited, insert it and append it to the next
 * layer. The visited set is the FULL history, so the oracle is also correct
 * for generating sets that are not closed under inverses.
 *
 * Stop rules: at most max_layers layers are recorded; if max_frontier > 0,
 * the first layer whose size is strictly greater than max_frontier is
 * recorded and not expanded.
 *
 * Return: 0 complete (an empty next layer was found), 1 truncated (a stop
 * rule ended the search while the last layer was non-empty), negative on
 * error (-1 bad argument, -2 out of memory).
 *
 * Storage: each state is a vector of n <= 16 entries in 0..15, stored as a
 * uint64 with entry i in bits [4i, 4i+4) (least-significant first). The
 * hash set is open addressing with linear probing and exact key compare;
 * the all-ones word marks an empty slot, and the one vector that packs to
 * the all-ones word (n = 16, every entry 15) is tracked by a separate flag.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EMPTY_SLOT UINT64_MAX

typedef struct {
    uint64_t *slot;
    uint64_t mask;      /* capacity - 1, capacity a power of two */
    uint64_t used;
    int has_all_ones;   /* the key equal to EMPTY_SLOT is a member */
} oset;

static uint64_t mix64(uint64_t x)
{
    /* splitmix64 finaliser (Steele, Lea, Flood 2014) */
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

static int oset_init(oset *s, uint64_t cap)
{
    uint64_t c = 1024;
    while (c < cap) c <<= 1;
    s->slot = (uint64_t *)malloc(c * sizeof(uint64_t));
    if (!s->slot) return -2;
    memset(s->slot, 0xff, c * sizeof(uint64_t));
    s->mask = c - 1;
    s->used = 0;
    s->has_all_ones = 0;
    return 0;
}

static void oset_free(oset *s)
{
    free(s->slot);
    s->slot = NULL;
}

/* insert without growth; returns 1 if newly inserted, 0 if present */
static int oset_put(oset *s, uint64_t key)
{
    if (key == EMPTY_SLOT) {
        if (s->has_all_ones) return 0;
        s->has_all_ones = 1;
        return 1;
    }
    uint64_t i = mix64(key) & s->mask;
    for (;;) {
        uint64_t v = s->slot[i];
        if (v == key) return 0;
        if (v == EMPTY_SLOT) {
            s->slot[i] = key;
            s->used++;
            return 1;
        }
        i = (i + 1) & s->mask;
    }
}

static int oset_grow(oset *s)
{
    oset bigger;
    if (oset_init(&bigger, (s->mask + 1) * 2) != 0) return -2;
    for (uint64_t i = 0; i <= s->mask; i++)
        if (s->slot[i] != EMPTY_SLOT) oset_put(&bigger, s->slot[i]);
    bigger.has_all_ones = s->has_all_ones;
    oset_free(s);
    *s = bigger;
    return 0;
}

/* insert with growth at load factor 1/2; returns 1 new, 0 present, <0 error */
static int oset_insert(oset *s, uint64_t key)
{
    if (2 * (s->used + 1) > s->mask + 1) {
        int rc = oset_grow(s);
        if (rc) return rc;
    }
    return oset_put(s, key);
}

static uint64_t pack_lsb_first(const uint8_t *v, int n)
{
    uint64_t x = 0;
    for (int i = 0; i < n; i++) x |= (uint64_t)v[i] << (4 * i);
    return x;
}

static void unpack_lsb_first(uint64_t x, int n, uint8_t *v)
{
    for (int i = 0; i < n; i++) v[i] = (uint8_t)((x >> (4 * i)) & 15u);
}

typedef struct {
    uint64_t *a;
    uint64_t len, cap;
} ovec;

static int ovec_push(ovec *q, uint64_t x)
{
    if (q->len == q->cap) {
        uint64_t nc = q->cap ? q->cap * 2 : 1024;
        uint64_t *na = (uint64_t *)realloc(q->a, nc * sizeof(uint64_t));
        if (!na) return -2;
        q->a = na;
        q->cap = nc;
    }
    q->a[q->len++] = x;
    return 0;
}

/*
 * n          number of entries per state, 1..16
 * gens       k rows of n bytes; row g holds the images g[0..n-1]
 * k          number of generator rows, >= 1
 * start      n bytes (entries 0..15) or NULL for the identity 0,1,..,n-1
 * max_layers capacity of `sizes`, >= 1
 * max_frontier  0 = no limit
 * sizes      out, max_layers entries; entries after the last layer are 0
 * num_layers out, number of recorded layers
 * states_out optional (may be NULL): every visited state as n bytes, in
 *            discovery order, layer after layer; at most states_cap rows are
 *            written (the count still covers every state)
 * n_visited  out (may be NULL): total number of visited states
 */
int oracle_growth(int n, const uint8_t *gens, int k, const uint8_t *start,
                  int max_layers, uint64_t max_frontier, uint64_t *sizes,
                  int *num_layers, uint8_t *states_out, uint64_t states_cap,
                  uint64_t *n_visited)
{
    if (n < 1 || n > 16 || k < 1 || max_layers < 1 || !gens || !sizes || !num_layers)
        return -1;
    for (int g = 0; g < k; g++) {
        int seen[16] = {0};
        for (int i = 0; i < n; i++) {
            uint8_t x = gens[g * n + i];
            if (x >= n || seen[x]) return -1;
            seen[x] = 1;
        }
    }
    uint8_t s0[16];
    for (int i = 0; i < n; i++) {
        s0[i] = start ? start[i] : (uint8_t)i;
        if (s0[i] > 15) return -1;
    }
    memset(sizes, 0, (size_t)max_layers * sizeof(uint64_t));

    oset seen;
    if (oset_init(&seen, 1 << 16)) return -2;
    ovec cur = {0}, nxt = {0};
    int rc = 0;
    uint64_t written = 0;

    uint64_t key0 = pack_lsb_first(s0, n);
    oset_insert(&seen, key0);
    if (ovec_push(&cur, key0)) { rc = -2; goto done; }
    if (states_out && written < states_cap) memcpy(states_out + written * n, s0, n);
    written++;
    sizes[0] = 1;
    int layers = 1;
    int status = 1;

    for (;;) {
        if (max_frontier > 0 && sizes[layers - 1] > max_frontier) { status = 1; break; }
        if (layers == max_layers) { status = 1; break; }
        nxt.len = 0;
        for (uint64_t f = 0; f < cur.len; f++) {
            uint8_t s[16], t[16];
            unpack_lsb_first(cur.a[f], n, s);
            for (int g = 0; g < k; g++) {
                const uint8_t *img = gens + (size_t)g * n;
                for (int i = 0; i < n; i++) t[i] = s[img[i]];
                uint64_t key = pack_lsb_first(t, n);
                int fresh = oset_insert(&seen, key);
                if (fresh < 0) { rc = fresh; goto done; }
                if (fresh) {
                    if (ovec_push(&nxt, key)) { rc = -2; goto done; }
                    if (states_out && written < states_cap) memcpy(states_out + written * n, t, n);
                    written++;
                }
            }
        }
        if (nxt.len == 0) { status = 0; break; }
        sizes[layers++] = nxt.len;
        ovec tmp = cur; cur = nxt; nxt = tmp;
    }
    *num_layers = layers;
    rc = status;
done:
    if (n_visited) *n_visited = written;
    oset_free(&seen);
    free(cur.a);
    free(nxt.a);
    return rc;
}
