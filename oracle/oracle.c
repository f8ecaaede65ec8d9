/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library; the product path
 * never does.
 *
 * A plain, sequential, leftmost-innermost normaliser for left-linear term
 * rewrite systems, written from the paper's definitions:
 *
 *   - terms, substitution, match and redex: Section 2, Definitions 1 and 2;
 *   - a rule l -> r needs l not a variable and Var(r) a subset of Var(l)
 *     (Definition 1), and each variable at most once in l (the paper's
 *     left-linearity assumption right after Definition 1);
 *   - the innermost strategy and the derive / rewrite_f procedures of
 *     Section 2: a term is rewritten only once all its subterms are in
 *     normal form, subterms are visited left to right, and for a head symbol
 *     the rules are tried in their order, the first match wins; when none
 *     matches the term is in normal form.
 *
 * Representation.  Terms live in a node store (symbol, argument indices,
 * normal-form flag, reference count).  Substitutions share the nodes bound
 * to variables instead of copying them; those nodes are always in normal
 * form under the innermost strategy, so sharing them cannot change any
 * rewrite.  Every non-variable subterm of a right-hand side becomes a fresh
 * node (no sharing between equal subterms), so the oracle performs exactly
 * the rewrites of plain tree rewriting.  A rewrite replaces the *reference*
 * held by the parent position (or the root cell) with the instantiated
 * right-hand side and releases the old redex; the explicit stack holds
 * positions, so recursion depth is not bounded by the C stack (numerals can
 * be millions of symbols deep).  Nodes whose count drops to zero are freed
 * and reused.
 *
 * Output: the canonical serialisation of the normal form, i.e. the prefix
 * sequence of symbol ids with all sharing expanded, plus the count of rule
 * applications, per rule.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_RULE (-3)
#define ORC_E_TERM (-4)
#define ORC_E_STEPS (-6)
#define ORC_E_MEM (-9)

typedef struct {
    int32_t n_sym;
    int32_t *arity;
    int32_t n_rules;
    int32_t **lhs, *lhs_len;  /* prefix codes; variables are -1-k */
    int32_t **rhs, *rhs_len;
    int32_t *n_vars;
    int32_t max_vars;
    int32_t A; /* highest arity, stride of the argument store */

    /* node store */
    int32_t *sym, *args, *rc;
    uint8_t *nf;
    int64_t cap, used;
    int32_t *freelist;
    int64_t nfree, freecap;
    int64_t live, peak_live;

    /* per-run results */
    int64_t *counts;
    int64_t steps;
    int32_t *out;
    int64_t out_len, out_cap;
    double seconds;
} Oracle;

/* ------------------------------------------------------------------ store */

static int grow_store(Oracle *o, int64_t need) {
    if (need <= o->cap) return 0;
    int64_t nc = o->cap ? o->cap : 1024;
    while (nc < need) nc *= 2;
    int32_t *s = realloc(o->sym, (size_t)nc * sizeof(int32_t));
    if (!s) return -1;
    o->sym = s;
    int32_t *a = realloc(o->args, (size_t)nc * (size_t)(o->A ? o->A : 1) * sizeof(int32_t));
    if (!a) return -1;
    o->args = a;
    int32_t *r = realloc(o->rc, (size_t)nc * sizeof(int32_t));
    if (!r) return -1;
    o->rc = r;
    uint8_t *f = realloc(o->nf, (size_t)nc);
    if (!f) return -1;
    o->nf = f;
    o->cap = nc;
    return 0;
}

/* returns a fresh node id (> 0) with rc = 0, or 0 when out of memory */
static int32_t new_node(Oracle *o, int32_t s) {
    int32_t id;
    if (o->nfree > 0) {
        id = o->freelist[--o->nfree];
    } else {
        if (o->used >= INT32_MAX) return 0;
        if (grow_store(o, o->used + 1)) return 0;
        id = (int32_t)o->used++;
    }
    o->sym[id] = s;
    o->rc[id] = 0;
    o->nf[id] = 0;
    for (int j = 0; j < o->A; j++) o->args[(int64_t)id * o->A + j] = 0;
    o->live++;
    if (o->live > o->peak_live) o->peak_live = o->live;
    return id;
}

static int push_free(Oracle *o, int32_t id) {
    if (o->nfree == o->freecap) {
        int64_t nc = o->freecap ? o->freecap * 2 : 1024;
        int32_t *f = realloc(o->freelist, (size_t)nc * sizeof(int32_t));
        if (!f) return -1;
        o->freelist = f;
        o->freecap = nc;
    }
    o->freelist[o->nfree++] = id;
    o->live--;
    return 0;
}

/* drop one reference to x; free every node that becomes unreferenced */
static int release(Oracle *o, int32_t x, int32_t **work, int64_t *wcap) {
    int64_t wn = 0;
    if (*wcap < 16) {
        int32_t *w = realloc(*work, 16 * sizeof(int32_t));
        if (!w) return -1;
        *work = w;
        *wcap = 16;
    }
    (*work)[wn++] = x;
    while (wn > 0) {
        int32_t y = (*work)[--wn];
        if (--o->rc[y] > 0) continue;
        int32_t ar = o->arity[o->sym[y]];
        for (int j = 0; j < ar; j++) {
            if (wn == *wcap) {
                int32_t *w = realloc(*work, (size_t)(*wcap * 2) * sizeof(int32_t));
                if (!w) return -1;
                *work = w;
                *wcap *= 2;
            }
            (*work)[wn++] = o->args[(int64_t)y * o->A + j];
        }
        if (push_free(o, y)) return -1;
    }
    return 0;
}

/* ---------------------------------------------------------------- parsing */

/* length of the prefix-coded (sub)term starting at code[p]; -1 if malformed */
static int64_t term_len(const Oracle *o, const int32_t *code, int64_t p, int64_t end) {
    int64_t need = 1, q = p;
    while (need > 0) {
        if (q >= end) return -1;
        int32_t c = code[q++];
        need--;
        if (c >= 0) {
            if (c >= o->n_sym) return -1;
            need += o->arity[c];
        }
    }
    return q - p;
}

/* ---------------------------------------------------------------- rules */

static int validate_rule(Oracle *o, int r) {
    const int32_t *l = o->lhs[r];
    const int32_t *rh = o->rhs[r];
    /* Definition 1 (1): the left-hand side is not a variable */
    if (l[0] < 0) return ORC_E_RULE;
    int32_t nv = 0;
    char seen[256];
    memset(seen, 0, sizeof seen);
    for (int32_t i = 0; i < o->lhs_len[r]; i++) {
        if (l[i] < 0) {
            int32_t k = -1 - l[i];
            if (k >= 256) return ORC_E_RULE;
            /* left-linearity: each variable at most once in the lhs */
            if (seen[k]) return ORC_E_RULE;
            seen[k] = 1;
            if (k + 1 > nv) nv = k + 1;
        }
    }
    for (int32_t i = 0; i < o->rhs_len[r]; i++) {
        if (rh[i] < 0) {
            int32_t k = -1 - rh[i];
            /* Definition 1 (2): Var(r) is a subset of Var(l) */
            if (k >= 256 || !seen[k]) return ORC_E_RULE;
        }
    }
    o->n_vars[r] = nv;
    if (nv > o->max_vars) o->max_vars = nv;
    return ORC_OK;
}

/* match pattern l (prefix code) against node t; on success fill bind[] */
static int match(const Oracle *o, const int32_t *l, int32_t llen, int32_t t, int32_t *bind,
                 int32_t *stk) {
    /* walk the pattern in prefix order alongside a stack of term nodes */
    int32_t sp = 0;
    stk[sp++] = t;
    for (int32_t i = 0; i < llen; i++) {
        int32_t node = stk[--sp];
        int32_t c = l[i];
        if (c < 0) {
            bind[-1 - c] = node;
            continue;
        }
        if (o->sym[node] != c) return 0;
        int32_t ar = o->arity[c];
        for (int32_t j = ar - 1; j >= 0; j--) stk[sp++] = o->args[(int64_t)node * o->A + j];
    }
    return 1;
}

/* instantiate rhs (prefix code) under bind[]; returns the node holding one
 * reference owned by the caller, or 0 when out of memory */
static int32_t instantiate(Oracle *o, const int32_t *r, int32_t rlen, const int32_t *bind,
                           int32_t *pend_node, int32_t *pend_fill) {
    /* iterative prefix build: pend_node/pend_fill form a stack of nodes that
     * still miss arguments */
    int32_t sp = 0, root = 0;
    for (int32_t i = 0; i < rlen; i++) {
        int32_t c = r[i], node;
        if (c < 0) {
            node = bind[-1 - c];
            o->rc[node]++;
        } else {
            node = new_node(o, c);
            if (!node) return 0;
            o->rc[node] = 1;
        }
        if (sp == 0) {
            root = node;
        } else {
            int32_t p = pend_node[sp - 1];
            o->args[(int64_t)p * o->A + pend_fill[sp - 1]] = node;
            pend_fill[sp - 1]++;
        }
        if (c >= 0 && o->arity[c] > 0) {
            pend_node[sp] = node;
            pend_fill[sp] = 0;
            sp++;
        }
        while (sp > 0 && pend_fill[sp - 1] == o->arity[o->sym[pend_node[sp - 1]]]) sp--;
    }
    return root;
}

/* ----------------------------------------------------------------- public */

void orc_free(void *h);

void *orc_new(int32_t n_sym, const int32_t *arity, int32_t n_rules, const int32_t *rule_off,
              const int32_t *rule_code, int32_t *status) {
    *status = ORC_E_ARG;
    if (n_sym <= 0 || n_rules < 0 || !arity || (n_rules > 0 && (!rule_off || !rule_code)))
        return NULL;
    Oracle *o = calloc(1, sizeof(Oracle));
    if (!o) return NULL;
    o->n_sym = n_sym;
    o->arity = malloc(sizeof(int32_t) * (size_t)n_sym);
    o->A = 0;
    for (int32_t i = 0; i < n_sym; i++) {
        if (arity[i] < 0 || arity[i] > 64) {
            orc_free(o);
            return NULL;
        }
        o->arity[i] = arity[i];
        if (arity[i] > o->A) o->A = arity[i];
    }
    if (o->A == 0) o->A = 1;
    o->n_rules = n_rules;
    o->lhs = calloc((size_t)n_rules + 1, sizeof(int32_t *));
    o->rhs = calloc((size_t)n_rules + 1, sizeof(int32_t *));
    o->lhs_len = calloc((size_t)n_rules + 1, sizeof(int32_t));
    o->rhs_len = calloc((size_t)n_rules + 1, sizeof(int32_t));
    o->n_vars = calloc((size_t)n_rules + 1, sizeof(int32_t));
    o->counts = calloc((size_t)n_rules + 1, sizeof(int64_t));
    for (int32_t r = 0; r < n_rules; r++) {
        int64_t b = rule_off[r], e = rule_off[r + 1];
        if (e <= b) {
            *status = ORC_E_RULE;
            orc_free(o);
            return NULL;
        }
        int64_t ll = term_len(o, rule_code, b, e);
        if (ll < 0) {
            *status = ORC_E_RULE;
            orc_free(o);
            return NULL;
        }
        int64_t rl = term_len(o, rule_code, b + ll, e);
        if (rl < 0 || b + ll + rl != e) {
            *status = ORC_E_RULE;
            orc_free(o);
            return NULL;
        }
        o->lhs_len[r] = (int32_t)ll;
        o->rhs_len[r] = (int32_t)rl;
        o->lhs[r] = malloc(sizeof(int32_t) * (size_t)ll);
        o->rhs[r] = malloc(sizeof(int32_t) * (size_t)rl);
        memcpy(o->lhs[r], rule_code + b, sizeof(int32_t) * (size_t)ll);
        memcpy(o->rhs[r], rule_code + b + ll, sizeof(int32_t) * (size_t)rl);
        int st = validate_rule(o, r);
        if (st != ORC_OK) {
            *status = st;
            orc_free(o);
            return NULL;
        }
    }
    *status = ORC_OK;
    return o;
}

void orc_free(void *h) {
    Oracle *o = h;
    if (!o) return;
    for (int32_t r = 0; r < o->n_rules; r++) {
        if (o->lhs) free(o->lhs[r]);
        if (o->rhs) free(o->rhs[r]);
    }
    free(o->lhs);
    free(o->rhs);
    free(o->lhs_len);
    free(o->rhs_len);
    free(o->n_vars);
    free(o->arity);
    free(o->sym);
    free(o->args);
    free(o->rc);
    free(o->nf);
    free(o->freelist);
    free(o->counts);
    free(o->out);
    free(o);
}

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* serialise the term held by node `root`, expanding sharing */
static int serialise(Oracle *o, int32_t root) {
    o->out_len = 0;
    int64_t scap = 1024, sp = 0;
    int32_t *stk = malloc(sizeof(int32_t) * (size_t)scap);
    if (!stk) return ORC_E_MEM;
    stk[sp++] = root;
    while (sp > 0) {
        int32_t x = stk[--sp];
        if (o->out_len == o->out_cap) {
            int64_t nc = o->out_cap ? o->out_cap * 2 : 1024;
            int32_t *no = realloc(o->out, sizeof(int32_t) * (size_t)nc);
            if (!no) {
                free(stk);
                return ORC_E_MEM;
            }
            o->out = no;
            o->out_cap = nc;
        }
        o->out[o->out_len++] = o->sym[x];
        int32_t ar = o->arity[o->sym[x]];
        if (sp + ar > scap) {
            while (sp + ar > scap) scap *= 2;
            int32_t *ns = realloc(stk, sizeof(int32_t) * (size_t)scap);
            if (!ns) {
                free(stk);
                return ORC_E_MEM;
            }
            stk = ns;
        }
        for (int32_t j = ar - 1; j >= 0; j--) stk[sp++] = o->args[(int64_t)x * o->A + j];
    }
    free(stk);
    return ORC_OK;
}

/*
 * Normalise one ground term given by its prefix code.  max_steps bounds the
 * number of rule applications (termination is undecidable, Section 2);
 * exceeding it returns ORC_E_STEPS.
 */
int32_t orc_run(void *h, const int32_t *term, int64_t len, int64_t max_steps) {
    Oracle *o = h;
    if (!o || !term || len <= 0) return ORC_E_ARG;
    /* reset the store: node 0 is never used, as in the paper's arrays */
    o->used = 1;
    o->nfree = 0;
    o->live = 0;
    o->peak_live = 0;
    o->steps = 0;
    o->out_len = 0;
    for (int32_t r = 0; r < o->n_rules; r++) o->counts[r] = 0;
    if (term_len(o, term, 0, len) != len) return ORC_E_TERM;
    for (int64_t i = 0; i < len; i++)
        if (term[i] < 0) return ORC_E_TERM; /* input must be ground */
    if (grow_store(o, len + 1)) return ORC_E_MEM;

    /* build the input tree (iterative prefix build; every node rc = 1) */
    int32_t *pend = malloc(sizeof(int32_t) * (size_t)(len + 1));
    int32_t *fill = malloc(sizeof(int32_t) * (size_t)(len + 1));
    if (!pend || !fill) {
        free(pend);
        free(fill);
        return ORC_E_MEM;
    }
    int32_t root_cell = 0;
    {
        int64_t sp = 0;
        for (int64_t i = 0; i < len; i++) {
            int32_t node = new_node(o, term[i]);
            o->rc[node] = 1;
            if (sp == 0) {
                root_cell = node;
            } else {
                o->args[(int64_t)pend[sp - 1] * o->A + fill[sp - 1]] = node;
                fill[sp - 1]++;
            }
            if (o->arity[term[i]] > 0) {
                pend[sp] = node;
                fill[sp] = 0;
                sp++;
            }
            while (sp > 0 && fill[sp - 1] == o->arity[o->sym[pend[sp - 1]]]) sp--;
        }
    }
    free(pend);
    free(fill);

    int32_t maxpat = 1;
    for (int32_t r = 0; r < o->n_rules; r++) {
        if (o->lhs_len[r] > maxpat) maxpat = o->lhs_len[r];
        if (o->rhs_len[r] > maxpat) maxpat = o->rhs_len[r];
    }
    int32_t *bind = malloc(sizeof(int32_t) * (size_t)(o->max_vars + 1));
    int32_t *mstk = malloc(sizeof(int32_t) * (size_t)(maxpat * (o->A + 1) + 1));
    int32_t *pn = malloc(sizeof(int32_t) * (size_t)(maxpat + 1));
    int32_t *pf = malloc(sizeof(int32_t) * (size_t)(maxpat + 1));
    int32_t *work = NULL;
    int64_t wcap = 0;
    /* the derivation stack holds positions: (parent node, argument index);
     * parent 0 denotes the root cell */
    int64_t scap = 1024, sp = 0;
    int32_t *sp_par = malloc(sizeof(int32_t) * (size_t)scap);
    int32_t *sp_pos = malloc(sizeof(int32_t) * (size_t)scap);
    int32_t status = ORC_OK;
    if (!bind || !mstk || !pn || !pf || !sp_par || !sp_pos) {
        status = ORC_E_MEM;
        goto done;
    }

    double t0 = now_s();
    sp_par[0] = 0;
    sp_pos[0] = 0;
    sp = 1;
    while (sp > 0) {
        int32_t par = sp_par[sp - 1], pos = sp_pos[sp - 1];
        int32_t t = par ? o->args[(int64_t)par * o->A + pos] : root_cell;
        if (o->nf[t]) {
            sp--;
            continue;
        }
        /* innermost, left to right: descend into the first subterm not yet
         * in normal form */
        int32_t ar = o->arity[o->sym[t]], desc = -1;
        for (int32_t j = 0; j < ar; j++) {
            if (!o->nf[o->args[(int64_t)t * o->A + j]]) {
                desc = j;
                break;
            }
        }
        if (desc >= 0) {
            if (sp == scap) {
                scap *= 2;
                int32_t *a = realloc(sp_par, sizeof(int32_t) * (size_t)scap);
                int32_t *b = a ? realloc(sp_pos, sizeof(int32_t) * (size_t)scap) : NULL;
                if (!a || !b) {
                    if (a) sp_par = a;
                    status = ORC_E_MEM;
                    goto done;
                }
                sp_par = a;
                sp_pos = b;
            }
            sp_par[sp] = t;
            sp_pos[sp] = desc;
            sp++;
            continue;
        }
        /* all subterms are normal forms: rewrite_{hs(t)} */
        int32_t hit = -1;
        for (int32_t r = 0; r < o->n_rules; r++) {
            if (o->lhs[r][0] != o->sym[t]) continue;
            if (match(o, o->lhs[r], o->lhs_len[r], t, bind, mstk)) {
                hit = r;
                break;
            }
        }
        if (hit < 0) {
            o->nf[t] = 1;
            sp--;
            continue;
        }
        if (o->steps >= max_steps) {
            status = ORC_E_STEPS;
            goto done;
        }
        o->steps++;
        o->counts[hit]++;
        int32_t repl = instantiate(o, o->rhs[hit], o->rhs_len[hit], bind, pn, pf);
        if (!repl) {
            status = ORC_E_MEM;
            goto done;
        }
        if (par)
            o->args[(int64_t)par * o->A + pos] = repl;
        else
            root_cell = repl;
        if (release(o, t, &work, &wcap)) {
            status = ORC_E_MEM;
            goto done;
        }
        /* the position now holds the contractum; the loop examines it again */
    }
    o->seconds = now_s() - t0;
    status = serialise(o, root_cell);

done:
    free(bind);
    free(mstk);
    free(pn);
    free(pf);
    free(work);
    free(sp_par);
    free(sp_pos);
    return status;
}

int64_t orc_result_len(void *h) { return ((Oracle *)h)->out_len; }

void orc_result_copy(void *h, int32_t *out) {
    Oracle *o = h;
    memcpy(out, o->out, sizeof(int32_t) * (size_t)o->out_len);
}

/* FNV-1a 64 over the little-endian bytes of the serialisation */
uint64_t orc_result_fnv(void *h) {
    Oracle *o = h;
    uint64_t x = 1469598103934665603ULL;
    for (int64_t i = 0; i < o->out_len; i++) {
        uint32_t v = (uint32_t)o->out[i];
        for (int b = 0; b < 4; b++) {
            x ^= (v >> (8 * b)) & 0xffu;
            x *= 1099511628211ULL;
        }
    }
    return x;
}

void orc_counts(void *h, int64_t *out) {
    Oracle *o = h;
    for (int32_t r = 0; r < o->n_rules; r++) out[r] = o->counts[r];
}

int64_t orc_steps(void *h) { return ((Oracle *)h)->steps; }
double orc_seconds(void *h) { return ((Oracle *)h)->seconds; }
int64_t orc_peak_live(void *h) { return ((Oracle *)h)->peak_live; }
