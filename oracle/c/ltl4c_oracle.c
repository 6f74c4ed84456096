/*
 * Oracle, part 3: plain single-threaded C evaluator of LTL4-C properties.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It includes no header
 * of the product library and shares no code with it.
 *
 * What it computes (paper sections in brackets):
 *   1. the value vector of every event from its key fields (Eq. 5,
 *      Section 4.1); an event that lacks a key joins no cluster, except, when
 *      the layout asks for parent events, one that carries every key but the
 *      innermost: it joins the cluster of every instance under its parent
 *      (reading stated below); its letter
 *      from its type and, when declared, from comparisons of record fields
 *      with constants (the data predicates of Section 5's cloud-storage
 *      case study);
 *   2. the clusters u^D: events grouped by vector, trace order kept inside a
 *      group (Section 2.4.3) -- a plain qsort on (vector, position); with
 *      parent events, u^D is the merge by trace position of D's own events
 *      and the parent events whose keys equal the first n-1 values of D;
 *   3. the leaf verdict lambda(delta(q0, u^D)) of every instance (Def. 6),
 *      stepping the monitor table one event at a time; on the way, the
 *      verdict after every event (stored at the event's trace position) and
 *      the length of each instance's first prefix with a T or F verdict;
 *   4. for every quantifier level from the innermost out, the 6-bin count of
 *      child verdicts of each node (Def. 8) and its verdict by Def. 7 with the
 *      numerical constraint of Eq. 6 and the permanence rules (Table 1 and
 *      the rule for the default A=1), in exact 128-bit integer arithmetic.
 *
 * The readings of Def. 7 are the ones stated in oracle/counting.py; this file
 * restates them in C and is checked against that module on random inputs.
 *
 * Nodes and instances are reported in lexicographic order of their vectors.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { V_BOT = 0, V_BOT_C = 1, V_BOT_P = 2, V_TOP_P = 3, V_TOP_C = 4, V_TOP = 5 };
#define ORA_NEVER 0xFFFFFFFFu
enum { Q_PERCENT = 0, Q_COUNT = 1 };
enum { OP_LT = 0, OP_LE = 1, OP_GT = 2, OP_GE = 3, OP_EQ = 4 };

typedef struct {
    uint32_t record_bytes;
    uint32_t type_offset, type_bytes;
    uint32_t n_keys;                  /* quantifier levels, 1..4 */
    uint32_t key_offset[4], key_bytes[4];
    const uint8_t *class_of_type;     /* [256] */
    const uint8_t *key_present;       /* [256]: bit m set = the type carries key m */
    /* data predicates (propositions read off a record's data, as in the
     * cloud-storage case study of Section 5): predicate i holds when the
     * unsigned field at pred_offset[i] compares true with pred_value[i];
     * the letter of the event is then its type's letter plus
     * 2^(pred_shift + i) for every holding predicate i */
    uint32_t n_preds, pred_shift;
    uint32_t pred_offset[3], pred_bytes[3], pred_op[3], pred_value[3];
    /* parent events (the proxy-cache case study of Section 5: per-video
     * events observed by every request of the video): when set, an event
     * whose type carries keys 0..n_keys-2 and not key n_keys-1 (for one
     * level: no key) belongs to the cluster u^D of every instance D whose
     * first n_keys-1 values equal its own, at its trace position.  It makes
     * no instance and no node, as the set of value vectors of Eq. 5 holds
     * only complete vectors.  Such events report no per-event verdict. */
    uint32_t parent_events;
} ora_layout;

/* comparison codes of a data predicate: < <= > >= == != */
static int pred_true(uint32_t op, uint32_t x, uint32_t v) {
    if (op == 0) return x < v;
    if (op == 1) return x <= v;
    if (op == 2) return x > v;
    if (op == 3) return x >= v;
    if (op == 4) return x == v;
    return x != v;
}

typedef struct {
    uint32_t n_states, n_classes, q0, pad;
    const uint32_t *delta;            /* [n_states * n_classes] */
    const uint8_t *label;             /* [n_states] */
    uint8_t kind[4], op[4];
    uint64_t num[4], den[4];          /* percentage: num/den; count: num */
} ora_property;

typedef struct {
    int n_props, n_levels;
    uint64_t n_inst;
    uint32_t *inst_keys;              /* [n_inst * n_levels] */
    uint8_t *inst_verdict;            /* [n_props * n_inst] */
    uint32_t *inst_conc;              /* [n_props * n_inst]: events of the instance read when its
                                         verdict was first T or F (0: before any), or ORA_NEVER */
    uint64_t n_events;
    uint8_t *event_verdict;           /* [n_props * n_events], trace order: the verdict of the
                                         event's instance on its prefix ending at the event;
                                         0xFF for an event of no cluster and for a
                                         parent event (it is in several) */
    uint64_t level_nodes[4];          /* nodes at level m (prefix length m) */
    uint32_t *level_keys[4];          /* [nodes * m] */
    uint64_t *level_counts[4];        /* [n_props * nodes * 6] */
    uint8_t *level_verdict[4];        /* [n_props * nodes] */
} ora_result;

static uint32_t read_field(const uint8_t *rec, uint32_t off, uint32_t bytes) {
    uint32_t v = 0;
    for (uint32_t b = 0; b < bytes; ++b) v |= (uint32_t)rec[off + b] << (8 * b);
    return v;
}

/* --- Eq. 6 and Def. 7 ---------------------------------------------------- */
typedef unsigned __int128 u128;

static int cmp_op(u128 a, int op, u128 b) {
    switch (op) {
    case OP_LT: return a < b;
    case OP_LE: return a <= b;
    case OP_GT: return a > b;
    case OP_GE: return a >= b;
    default: return a == b;
    }
}

/* S of Eq. 6: k children in the set, n children in total */
static int sat_S(int kind, int op, uint64_t num, uint64_t den, uint64_t k, uint64_t n) {
    if (kind == Q_PERCENT) return cmp_op((u128)k * den, op, (u128)num * n);
    return cmp_op(k, op, num);
}

static int perm_sat(int kind, int op, uint64_t num, uint64_t den, const uint64_t *v) {
    uint64_t top = v[V_TOP], bot = v[V_BOT];
    if (kind == Q_COUNT) {
        if (op == OP_GT) return top > num;
        if (op == OP_GE) return top >= num;
        return 0;
    }
    int c_zero = (num == 0), c_one = (num == den);
    switch (op) {
    case OP_GE: return c_zero;
    case OP_GT: return c_zero && top >= 1;
    case OP_LE: return c_one;
    case OP_LT: return c_one && bot >= 1;
    default: return 0;
    }
}

static int perm_viol(int kind, int op, uint64_t num, uint64_t den, const uint64_t *v) {
    uint64_t top = v[V_TOP], bot = v[V_BOT];
    if (kind == Q_COUNT) {
        if (op == OP_EQ || op == OP_LE) return top > num;
        if (op == OP_LT) return top >= num;
        return 0;
    }
    int c_zero = (num == 0), c_one = (num == den);
    switch (op) {
    case OP_GE: return c_one && bot >= 1;
    case OP_GT: return c_one;
    case OP_LE: return c_zero && top >= 1;
    case OP_LT: return c_zero;
    default: return (c_one && bot >= 1) || (c_zero && top >= 1);
    }
}

static uint8_t valuate(int kind, int op, uint64_t num, uint64_t den, const uint64_t *v) {
    uint64_t n = v[0] + v[1] + v[2] + v[3] + v[4] + v[5];
    uint64_t k1 = v[V_TOP];
    uint64_t k2 = k1 + v[V_TOP_C];
    uint64_t k3 = k2 + v[V_TOP_P];
    uint64_t k4 = k3 + v[V_BOT_P];
    uint64_t k5 = k4 + v[V_BOT_C];
    if (sat_S(kind, op, num, den, k1, n) && perm_sat(kind, op, num, den, v)) return V_TOP;
    if (sat_S(kind, op, num, den, k2, n)) return V_TOP_C;
    if (sat_S(kind, op, num, den, k3, n)) return V_TOP_P;
    if (sat_S(kind, op, num, den, k4, n)) return V_BOT_P;
    if (!sat_S(kind, op, num, den, k5, n) && perm_viol(kind, op, num, den, v)) return V_BOT;
    return V_BOT_C;
}

uint8_t ora_valuate(int kind, int op, uint64_t num, uint64_t den, const uint64_t *v) {
    return valuate(kind, op, num, den, v);
}

/* --- clustering ---------------------------------------------------------- */
typedef struct {
    uint32_t key[4];
    uint64_t pos;
    uint8_t cls;
} ev_t;

/* key count for the comparator; one per thread, so that evaluations of
   disjoint partitions may run concurrently */
static _Thread_local int g_nk;

static int ev_cmp(const void *a, const void *b) {
    const ev_t *x = (const ev_t *)a, *y = (const ev_t *)b;
    for (int m = 0; m < g_nk; ++m) {
        if (x->key[m] != y->key[m]) return x->key[m] < y->key[m] ? -1 : 1;
    }
    return x->pos < y->pos ? -1 : (x->pos > y->pos ? 1 : 0);
}

/* lexicographic a < b on the first m values */
static int prefix_less(const uint32_t *a, const uint32_t *b, int m) {
    for (int i = 0; i < m; ++i)
        if (a[i] != b[i]) return a[i] < b[i];
    return 0;
}

static int same_prefix(const uint32_t *a, const uint32_t *b, int m) {
    for (int i = 0; i < m; ++i)
        if (a[i] != b[i]) return 0;
    return 1;
}

void ora_free(ora_result *r) {
    if (!r) return;
    free(r->inst_keys);
    free(r->inst_verdict);
    free(r->inst_conc);
    free(r->event_verdict);
    for (int m = 0; m < 4; ++m) {
        free(r->level_keys[m]);
        free(r->level_counts[m]);
        free(r->level_verdict[m]);
    }
    free(r);
}

ora_result *ora_eval(const uint8_t *records, uint64_t n, const ora_layout *L,
                     const ora_property *P, int n_props) {
    int nk = (int)L->n_keys;
    if (nk < 1 || nk > 4 || n_props < 1) return NULL;
    uint32_t need = (1u << nk) - 1;
    ev_t *ev = (ev_t *)malloc(sizeof(ev_t) * (n ? n : 1));
    ev_t *pev = (ev_t *)malloc(sizeof(ev_t) * (L->parent_events && n ? n : 1));
    if (!ev || !pev) {
        free(ev);
        free(pev);
        return NULL;
    }
    uint64_t ne = 0, npe = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint8_t *rec = records + i * L->record_bytes;
        uint32_t type = read_field(rec, L->type_offset, L->type_bytes);
        if (type >= 256) continue;
        const uint32_t kp = L->key_present[type] & need;
        const int parent = L->parent_events && kp == (need >> 1);
        if (kp != need && !parent) continue;
        ev_t e;
        memset(&e, 0, sizeof e);
        for (int m = 0; m < nk - parent; ++m) e.key[m] = read_field(rec, L->key_offset[m], L->key_bytes[m]);
        e.pos = i;
        e.cls = L->class_of_type[type];
        for (uint32_t q = 0; q < L->n_preds && q < 3; ++q)
            if (pred_true(L->pred_op[q], read_field(rec, L->pred_offset[q], L->pred_bytes[q]), L->pred_value[q]))
                e.cls += 1u << (L->pred_shift + q);
        if (parent) pev[npe++] = e;
        else ev[ne++] = e;
    }
    g_nk = nk;
    qsort(ev, ne, sizeof(ev_t), ev_cmp);
    g_nk = nk - 1;   /* parent events: by (first n-1 values, position) */
    qsort(pev, npe, sizeof(ev_t), ev_cmp);

    ora_result *r = (ora_result *)calloc(1, sizeof(ora_result));
    r->n_props = n_props;
    r->n_levels = nk;
    uint64_t ni = 0;
    for (uint64_t i = 0; i < ne; ++i)
        if (i == 0 || !same_prefix(ev[i].key, ev[i - 1].key, nk)) ++ni;
    r->n_inst = ni;
    r->inst_keys = (uint32_t *)malloc(sizeof(uint32_t) * nk * (ni ? ni : 1));
    r->inst_verdict = (uint8_t *)malloc((size_t)n_props * (ni ? ni : 1));
    r->inst_conc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n_props * (ni ? ni : 1));
    r->n_events = n;
    r->event_verdict = (uint8_t *)malloc((size_t)n_props * (n ? n : 1));
    memset(r->event_verdict, 0xFF, (size_t)n_props * (n ? n : 1));

    /* leaves: step every property's table over each cluster (Def. 6) */
    uint32_t *state = (uint32_t *)malloc(sizeof(uint32_t) * n_props);
    uint64_t inst = 0;
    for (uint64_t i = 0; i < ne;) {
        uint64_t j = i;
        for (int p = 0; p < n_props; ++p) {
            state[p] = P[p].q0;
            /* the prefix verdict timeline: the first prefix (by its length)
               whose verdict is T or F */
            const uint8_t l0 = P[p].label[state[p]];
            r->inst_conc[(uint64_t)p * ni + inst] = (l0 == V_TOP || l0 == V_BOT) ? 0u : ORA_NEVER;
        }
        /* the parent events of this instance: those whose n-1 values equal
           its first n-1 values (a contiguous run of pev, found by a plain
           binary search for the first one not below the prefix) */
        uint64_t pa = npe, pb = npe;
        if (npe) {
            uint64_t lo = 0, hi = npe;
            while (lo < hi) {
                const uint64_t mid = (lo + hi) / 2;
                if (prefix_less(pev[mid].key, ev[i].key, nk - 1)) lo = mid + 1;
                else hi = mid;
            }
            pa = pb = lo;
            while (pb < npe && same_prefix(pev[pb].key, ev[i].key, nk - 1)) ++pb;
        }
        /* walk u^D: own events and parent events merged by trace position */
        uint64_t steps = 0;
        while ((j < ne && same_prefix(ev[j].key, ev[i].key, nk)) || pa < pb) {
            const int own_left = j < ne && same_prefix(ev[j].key, ev[i].key, nk);
            const int take_own = own_left && (pa >= pb || ev[j].pos < pev[pa].pos);
            const ev_t *e = take_own ? &ev[j] : &pev[pa];
            ++steps;
            for (int p = 0; p < n_props; ++p) {
                state[p] = P[p].delta[(uint64_t)state[p] * P[p].n_classes + e->cls];
                const uint8_t l = P[p].label[state[p]];
                if (take_own) r->event_verdict[(uint64_t)p * n + e->pos] = l;
                uint32_t *c = &r->inst_conc[(uint64_t)p * ni + inst];
                if (*c == ORA_NEVER && (l == V_TOP || l == V_BOT)) *c = (uint32_t)steps;
            }
            if (take_own) ++j;
            else ++pa;
        }
        memcpy(r->inst_keys + inst * nk, ev[i].key, sizeof(uint32_t) * nk);
        for (int p = 0; p < n_props; ++p) r->inst_verdict[(uint64_t)p * ni + inst] = P[p].label[state[p]];
        ++inst;
        i = j;
    }
    free(state);
    free(ev);
    free(pev);

    /* quantifier levels from the innermost (nk-1) out to the root (0) */
    const uint32_t *child_keys = r->inst_keys;
    const uint8_t *child_verdict = r->inst_verdict;
    uint64_t n_child = ni;
    int child_width = nk;
    for (int m = nk - 1; m >= 0; --m) {
        uint64_t nodes = 0;
        for (uint64_t c = 0; c < n_child; ++c)
            if (c == 0 || !same_prefix(child_keys + c * child_width, child_keys + (c - 1) * child_width, m)) ++nodes;
        if (m == 0) nodes = 1; /* the root exists even when there are no instances */
        r->level_nodes[m] = nodes;
        r->level_keys[m] = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1) * (nodes ? nodes : 1));
        r->level_counts[m] = (uint64_t *)calloc((size_t)n_props * nodes * 6, sizeof(uint64_t));
        r->level_verdict[m] = (uint8_t *)malloc((size_t)n_props * (nodes ? nodes : 1));
        uint64_t node = 0;
        for (uint64_t c = 0; c < n_child; ++c) {
            if (c > 0 && !same_prefix(child_keys + c * child_width, child_keys + (c - 1) * child_width, m)) ++node;
            if (m > 0) memcpy(r->level_keys[m] + node * m, child_keys + c * child_width, sizeof(uint32_t) * m);
            for (int p = 0; p < n_props; ++p)
                r->level_counts[m][((uint64_t)p * nodes + node) * 6 + child_verdict[(uint64_t)p * n_child + c]] += 1;
        }
        for (int p = 0; p < n_props; ++p)
            for (uint64_t k = 0; k < nodes; ++k)
                r->level_verdict[m][(uint64_t)p * nodes + k] =
                    valuate(P[p].kind[m], P[p].op[m], P[p].num[m], P[p].den[m],
                            r->level_counts[m] + ((uint64_t)p * nodes + k) * 6);
        child_keys = r->level_keys[m];
        child_verdict = r->level_verdict[m];
        n_child = nodes;
        child_width = m;
    }
    return r;
}

/* accessors for the ctypes wrapper */
uint64_t ora_n_inst(const ora_result *r) { return r->n_inst; }
uint64_t ora_level_nodes(const ora_result *r, int m) { return r->level_nodes[m]; }
const uint32_t *ora_inst_keys(const ora_result *r) { return r->inst_keys; }
const uint8_t *ora_inst_verdict(const ora_result *r) { return r->inst_verdict; }
const uint32_t *ora_inst_conc(const ora_result *r) { return r->inst_conc; }
const uint8_t *ora_event_verdict(const ora_result *r) { return r->event_verdict; }
const uint32_t *ora_level_keys(const ora_result *r, int m) { return r->level_keys[m]; }
const uint64_t *ora_level_counts(const ora_result *r, int m) { return r->level_counts[m]; }
const uint8_t *ora_level_verdict(const ora_result *r, int m) { return r->level_verdict[m]; }
