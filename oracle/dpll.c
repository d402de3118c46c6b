/*
 * Plain CPU DPLL oracle: TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this library.  It shares no source, header or helper with the GPU path; it
 * reads the same CNF bytes (and cube lists) as plain data.
 *
 * What it computes (the readings are the ones stated in the design notes):
 *  - unit propagation to its fixpoint by repeated full scans;
 *  - DPLL with unit propagation: a decide mode (SAT + model / UNSAT) and a
 *    model-counting mode (#DPLL) with an arbitrary-precision count;
 *  - the canonical leaf of a cube: conflict after propagation ("refuted"),
 *    else the active variables (unassigned and in some unsatisfied clause),
 *    their number f, the number m of other unassigned variables, the number of
 *    assignments to the active variables that satisfy every unsatisfied clause,
 *    and the smallest satisfying assignment index when slot j (the j-th active
 *    variable in increasing order) is bit j of the index.
 *
 * The paper decides each access's constraint set with a SAT solver
 * (Sec. 5.2); a query is out-of-bounds iff the set is satisfiable.  Branching
 * here is MOMs (most occurrences in the shortest unsatisfied clauses), ties to
 * the lowest variable, 0-branch first: deliberately not the GPU path's order.
 *
 * CNF: variables 1..n, DIMACS literals, clause c = lits[off[c] .. off[c+1]).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n;              /* variables */
    int64_t nc;             /* clauses */
    const uint64_t *off;
    const int32_t *lits;
} cnf_t;

/* value of a literal under a: 1 true, 0 false, -1 unassigned */
static int lit_value(const int8_t *a, int32_t l)
{
    int v = a[l > 0 ? l : -l];
    if (v < 0) return -1;
    return l > 0 ? v : !v;
}

/* Unit propagation by full scans until nothing changes.  Returns 1 on a
 * conflict (some clause has every literal false), else 0. */
static int unit_propagate(const cnf_t *f, int8_t *a)
{
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int64_t c = 0; c < f->nc; c++) {
            int open = 0, sat = 0;
            int32_t last = 0;
            for (uint64_t i = f->off[c]; i < f->off[c + 1]; i++) {
                int v = lit_value(a, f->lits[i]);
                if (v == 1) { sat = 1; break; }
                if (v < 0) { open++; last = f->lits[i]; }
            }
            if (sat) continue;
            if (open == 0) return 1;
            if (open == 1) {
                a[last > 0 ? last : -last] = (int8_t)(last > 0);
                changed = 1;
            }
        }
    }
    return 0;
}

static int clause_satisfied(const cnf_t *f, const int8_t *a, int64_t c)
{
    for (uint64_t i = f->off[c]; i < f->off[c + 1]; i++)
        if (lit_value(a, f->lits[i]) == 1) return 1;
    return 0;
}

/* MOMs choice over unsatisfied clauses; 0 when every clause is satisfied. */
static int32_t choose_moms(const cnf_t *f, const int8_t *a, int32_t *score)
{
    int best_len = 1 << 30;
    for (int64_t c = 0; c < f->nc; c++) {
        if (clause_satisfied(f, a, c)) continue;
        int open = 0;
        for (uint64_t i = f->off[c]; i < f->off[c + 1]; i++)
            if (lit_value(a, f->lits[i]) < 0) open++;
        if (open < best_len) best_len = open;
    }
    if (best_len == (1 << 30)) return 0;
    memset(score, 0, sizeof(int32_t) * (size_t)(f->n + 1));
    for (int64_t c = 0; c < f->nc; c++) {
        if (clause_satisfied(f, a, c)) continue;
        int open = 0;
        for (uint64_t i = f->off[c]; i < f->off[c + 1]; i++)
            if (lit_value(a, f->lits[i]) < 0) open++;
        if (open != best_len) continue;
        for (uint64_t i = f->off[c]; i < f->off[c + 1]; i++) {
            int32_t l = f->lits[i];
            if (lit_value(a, l) < 0) score[l > 0 ? l : -l]++;
        }
    }
    int32_t best = 0;
    for (int32_t v = 1; v <= f->n; v++)
        if (score[v] > 0 && (best == 0 || score[v] > score[best])) best = v;
    return best;
}

/* ---------------------------------------------------------------- decide */

typedef struct {
    const cnf_t *f;
    int64_t nodes, max_nodes;
    int32_t *score;
} search_t;

/* 1 SAT (a holds a model), 0 UNSAT, 2 budget exhausted */
static int dpll(search_t *s, int8_t *a)
{
    if (++s->nodes > s->max_nodes) return 2;
    if (unit_propagate(s->f, a)) return 0;
    int32_t v = choose_moms(s->f, a, s->score);
    if (v == 0) {
        for (int32_t x = 1; x <= s->f->n; x++) if (a[x] < 0) a[x] = 0;
        return 1;
    }
    size_t bytes = (size_t)s->f->n + 1;
    int8_t *b = (int8_t *)malloc(bytes);
    int unknown = 0;
    for (int val = 0; val <= 1; val++) {
        memcpy(b, a, bytes);
        b[v] = (int8_t)val;
        int r = dpll(s, b);
        if (r == 1) { memcpy(a, b, bytes); free(b); return 1; }
        if (r == 2) { unknown = 1; break; }
    }
    free(b);
    return unknown ? 2 : 0;
}

/* Returns 1 SAT, 0 UNSAT, 2 UNKNOWN (node budget).  model: n+1 bytes. */
int oracle_solve(int32_t n, int64_t nc, const uint64_t *off, const int32_t *lits,
                 int64_t max_nodes, uint8_t *model, int64_t *nodes_out)
{
    cnf_t f = {n, nc, off, lits};
    search_t s = {&f, 0, max_nodes, (int32_t *)calloc((size_t)n + 1, 4)};
    int8_t *a = (int8_t *)malloc((size_t)n + 1);
    memset(a, -1, (size_t)n + 1);
    int r = dpll(&s, a);
    if (r == 1 && model) {
        model[0] = 0;
        for (int32_t x = 1; x <= n; x++) model[x] = (uint8_t)a[x];
    }
    if (nodes_out) *nodes_out = s.nodes;
    free(a);
    free(s.score);
    return r;
}

/* ---------------------------------------------------------------- count */

/* little-endian base-2^32 accumulator: acc += 2^e */
static int big_add_pow2(uint32_t *acc, int words, int64_t e)
{
    int64_t w = e / 32;
    if (w >= words) return 1;
    uint64_t carry = (uint64_t)1 << (e % 32);
    for (int64_t i = w; i < words && carry; i++) {
        uint64_t t = (uint64_t)acc[i] + carry;
        acc[i] = (uint32_t)t;
        carry = t >> 32;
    }
    return carry ? 1 : 0;
}

typedef struct {
    const cnf_t *f;
    int64_t nodes, max_nodes;
    int32_t *score;
    const uint8_t *counted;   /* NULL: every variable counts */
    uint32_t *acc;
    int words;
    int overflow;
} count_t;

/* 0 done, 2 budget exhausted */
static int count_rec(count_t *s, int8_t *a)
{
    if (++s->nodes > s->max_nodes) return 2;
    if (unit_propagate(s->f, a)) return 0;
    int32_t v = choose_moms(s->f, a, s->score);
    if (v == 0) {
        int64_t free_vars = 0;
        for (int32_t x = 1; x <= s->f->n; x++)
            if (a[x] < 0 && (!s->counted || s->counted[x])) free_vars++;
        s->overflow |= big_add_pow2(s->acc, s->words, free_vars);
        return 0;
    }
    size_t bytes = (size_t)s->f->n + 1;
    int8_t *b = (int8_t *)malloc(bytes);
    for (int val = 0; val <= 1; val++) {
        memcpy(b, a, bytes);
        b[v] = (int8_t)val;
        if (count_rec(s, b) == 2) { free(b); return 2; }
    }
    free(b);
    return 0;
}

/* Number of models of the CNF over all n variables (#DPLL) into count[words]
 * (little-endian 32-bit words).  Returns 0 done, 2 budget, 3 overflow. */
int oracle_count(int32_t n, int64_t nc, const uint64_t *off, const int32_t *lits,
                 int64_t max_nodes, uint32_t *count, int32_t words, int64_t *nodes_out)
{
    cnf_t f = {n, nc, off, lits};
    memset(count, 0, sizeof(uint32_t) * (size_t)words);
    count_t s = {&f, 0, max_nodes, (int32_t *)calloc((size_t)n + 1, 4), NULL,
                 count, words, 0};
    int8_t *a = (int8_t *)malloc((size_t)n + 1);
    memset(a, -1, (size_t)n + 1);
    int r = count_rec(&s, a);
    if (nodes_out) *nodes_out = s.nodes;
    free(a);
    free(s.score);
    if (r == 2) return 2;
    return s.overflow ? 3 : 0;
}

/* ---------------------------------------------------------------- leaf */

/* Apply the cube's literals; 1 if two of them clash. */
static int apply_cube(int8_t *a, const int32_t *cube, int32_t len)
{
    for (int32_t i = 0; i < len; i++) {
        int32_t l = cube[i], v = l > 0 ? l : -l;
        int8_t val = (int8_t)(l > 0);
        if (a[v] >= 0 && a[v] != val) return 1;
        a[v] = val;
    }
    return 0;
}

/* Unit propagation to the fixpoint of (F, cube).  assign: n+1 bytes,
 * -1/0/1.  Returns 1 on conflict. */
int oracle_up(int32_t n, int64_t nc, const uint64_t *off, const int32_t *lits,
              const int32_t *cube, int32_t cube_len, int8_t *assign)
{
    cnf_t f = {n, nc, off, lits};
    memset(assign, -1, (size_t)n + 1);
    if (apply_cube(assign, cube, cube_len)) return 1;
    return unit_propagate(&f, assign);
}

typedef struct {
    const cnf_t *f;
    const int32_t *slot_var;
    int32_t nf;
    int64_t nodes, max_nodes;
} lexmin_t;

/* Smallest index over the slots: branch on the highest unassigned slot,
 * 0 first.  1 found (a completed), 0 none, 2 budget. */
static int lexmin_rec(lexmin_t *s, int8_t *a)
{
    if (++s->nodes > s->max_nodes) return 2;
    if (unit_propagate(s->f, a)) return 0;
    int all_sat = 1;
    for (int64_t c = 0; c < s->f->nc && all_sat; c++)
        if (!clause_satisfied(s->f, a, c)) all_sat = 0;
    if (all_sat) {
        for (int32_t j = 0; j < s->nf; j++)
            if (a[s->slot_var[j]] < 0) a[s->slot_var[j]] = 0;
        return 1;
    }
    int32_t v = 0;
    for (int32_t j = s->nf - 1; j >= 0; j--)
        if (a[s->slot_var[j]] < 0) { v = s->slot_var[j]; break; }
    if (v == 0) return 0;   /* cannot happen at a fixpoint without conflict */
    size_t bytes = (size_t)s->f->n + 1;
    int8_t *b = (int8_t *)malloc(bytes);
    for (int val = 0; val <= 1; val++) {
        memcpy(b, a, bytes);
        b[v] = (int8_t)val;
        int r = lexmin_rec(s, b);
        if (r != 0) {
            if (r == 1) memcpy(a, b, bytes);
            free(b);
            return r;
        }
    }
    free(b);
    return 0;
}

/*
 * Canonical leaf of a cube.
 * Outputs: *refuted (1 if propagation conflicts), *f_out, *m_out,
 * slot_var[f] (active variables, increasing), *count_out (satisfying
 * assignments of the active variables; f <= 62 required), *first_out
 * (smallest satisfying index, -1 if none).  Returns 0, or 2 on budget,
 * 1 when f > cap or f > 62.
 */
int oracle_leaf(int32_t n, int64_t nc, const uint64_t *off, const int32_t *lits,
                const int32_t *cube, int32_t cube_len, int64_t max_nodes,
                int32_t *refuted, int32_t *f_out, int32_t *m_out,
                int32_t *slot_var, int32_t cap, uint64_t *count_out,
                int64_t *first_out)
{
    cnf_t f = {n, nc, off, lits};
    size_t bytes = (size_t)n + 1;
    int8_t *a = (int8_t *)malloc(bytes);
    memset(a, -1, bytes);
    *refuted = 0; *f_out = 0; *m_out = 0; *count_out = 0; *first_out = -1;
    if (apply_cube(a, cube, cube_len) || unit_propagate(&f, a)) {
        *refuted = 1;
        free(a);
        return 0;
    }
    uint8_t *active = (uint8_t *)calloc(bytes, 1);
    for (int64_t c = 0; c < nc; c++) {
        if (clause_satisfied(&f, a, c)) continue;
        for (uint64_t i = off[c]; i < off[c + 1]; i++) {
            int32_t l = lits[i];
            if (lit_value(a, l) < 0) active[l > 0 ? l : -l] = 1;
        }
    }
    int32_t nf = 0, nm = 0;
    for (int32_t x = 1; x <= n; x++) {
        if (a[x] >= 0) continue;
        if (active[x]) {
            if (nf < cap) slot_var[nf] = x;
            nf++;
        } else {
            nm++;
        }
    }
    *f_out = nf;
    *m_out = nm;
    if (nf > cap || nf > 62) { free(a); free(active); return 1; }

    /* count assignments of the active variables: #DPLL from the fixpoint,
     * counting only the active variables at satisfied nodes */
    uint32_t acc[4] = {0, 0, 0, 0};
    count_t cs = {&f, 0, max_nodes, (int32_t *)calloc(bytes, 4), active, acc, 4, 0};
    int8_t *b = (int8_t *)malloc(bytes);
    memcpy(b, a, bytes);
    int r = count_rec(&cs, b);
    free(cs.score);
    if (r == 2) { free(a); free(b); free(active); return 2; }
    *count_out = (uint64_t)acc[0] | ((uint64_t)acc[1] << 32);

    if (*count_out) {
        lexmin_t ls = {&f, slot_var, nf, 0, max_nodes};
        memcpy(b, a, bytes);
        r = lexmin_rec(&ls, b);
        if (r == 2) { free(a); free(b); free(active); return 2; }
        if (r == 1) {
            int64_t idx = 0;
            for (int32_t j = 0; j < nf; j++)
                if (b[slot_var[j]] == 1) idx |= (int64_t)1 << j;
            *first_out = idx;
        }
    }
    free(a); free(b); free(active);
    return 0;
}
