/*
 * HWPM oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of the heavy-weight
 * perfect matching method of Azad, Buluc, Li, Wang and Langguth,
 * "A distributed-memory algorithm for computing a heavy-weight perfect
 * matching on bipartite graphs" (arXiv 1801.09809).  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load this
 * library; the product path (the HIP library) never does, and the two share
 * no code.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (plain IEEE-754 binary64,
 * round to nearest even, no contraction, no fast-math).
 *
 * Contents
 *   oracle_tree_sum   fixed pairwise-tree FP64 sum (the summation order the
 *                     paper leaves open; read as a perfect binary tree).
 *   oracle_improve    the weight-increasing alternating 4-cycle (WIAC)
 *                     rounds, Section 5.3 (Algorithms 2-6), bulk-synchronous.
 *   oracle_greedy     Phase I.1: greedy maximal matching with the heavy-edge
 *                     tie-break of Section 5.2.
 *   oracle_mcm        Phase I.2: maximum-cardinality matching by
 *                     multi-source BFS phases with the "max" tie-break of
 *                     Section 5.2.
 *   oracle_match      Phase I then the WIAC rounds (the HWPM pipeline of
 *                     Section 5.1).
 *
 * Conventions (Section 3): an n x n matrix A in compressed sparse column
 * form (col_ptr[n+1], row_idx[nnz] strictly increasing inside a column,
 * w[nnz] finite).  Columns are the vertices C, rows the vertices R, and each
 * nonzero a_ij is the edge {i,j} of weight w(i,j).  For a perfect matching,
 * mc[j] is the row matched to column j (m_j) and mr[i] the column matched
 * to row i (m_i).
 *
 * Pins: every function here is pinned by tests/test_oracle_*.py against
 * brute-force enumeration, hand-derived cases, closed forms and the 6-cycle
 * counterexample of Section 4.  Phase I (greedy + MCM) is pinned for
 * cardinality (a maximum matching, checked against a library
 * Hopcroft-Karp) and maximality, and each of its rules (heavy-edge
 * preference, equal-weight ties by index, the heavier BFS parent, the
 * smallest endpoint per tree, a tree stopping at its first endpoint) by a
 * hand-derived case whose misreadings give a different matching or a
 * different phase and level count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_ROUND_STATS 256

typedef struct {
    int32_t rounds;        /* search passes executed (the last finds nothing) */
    int32_t hit_round_cap; /* 1 if max_rounds stopped the loop */
    int64_t cycles_applied;
    double init_weight;    /* tree sum of the initial matched weights */
    double final_weight;
    int32_t round_candidates[ORACLE_MAX_ROUND_STATS]; /* |S| per round */
    int32_t round_applied[ORACLE_MAX_ROUND_STATS];    /* |D(S)| per round */
    /* Phase I counts (oracle_match only; 0 otherwise) */
    int32_t greedy_rounds;      /* proposal rounds, the last one finding no proposal */
    int32_t greedy_cardinality; /* size of the greedy maximal matching */
    int32_t mcm_phases;         /* BFS phases started with an unmatched column */
    int32_t mcm_levels;         /* BFS levels with a nonempty frontier, all phases */
} oracle_stats;

/* ------------------------------------------------------------------------ */
/* Fixed summation order.  The paper sums matched weights (Section 3) without
 * saying in which order; the reading used here is a perfect binary tree over
 * x[0..n) padded with +0.0 up to the next power of two, adding the pair
 * (2t, 2t+1) at every level.  n == 0 gives +0.0. */
double oracle_tree_sum(const double* x, int64_t n)
{
    if (n <= 0) return 0.0;
    int64_t size = 1;
    while (size < n) size *= 2;
    double* buf = (double*)malloc((size_t)size * sizeof(double));
    if (!buf) return 0.0;
    for (int64_t t = 0; t < size; ++t) buf[t] = (t < n) ? x[t] : 0.0;
    for (int64_t len = size; len > 1; len /= 2)
        for (int64_t t = 0; t < len / 2; ++t) buf[t] = buf[2 * t] + buf[2 * t + 1];
    double s = buf[0];
    free(buf);
    return s;
}

/* Position of row r inside column c, or -1 when the edge {r,c} is absent.
 * Rows are strictly increasing inside a column, so the library bsearch
 * applies. */
static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static int64_t edge_pos(const int64_t* col_ptr, const int32_t* row_idx, int32_t r, int32_t c)
{
    int64_t lo = col_ptr[c], hi = col_ptr[c + 1];
    if (hi <= lo) return -1;
    const int32_t* hit =
        (const int32_t*)bsearch(&r, row_idx + lo, (size_t)(hi - lo), sizeof(int32_t), cmp_i32);
    return hit ? (int64_t)(hit - row_idx) : -1;
}

/* ------------------------------------------------------------------------ */
/* The WIAC rounds (Section 5.3, Algorithms 2-6), started from the perfect
 * matching mate_in (mate_in[j] = m_j).
 *
 * One round reads only the matching as it stood when the round began
 * (the algorithm is bulk-synchronous, Section 5.1):
 *
 *  Steps A+B.  Cycles are rooted at columns j only (the matrix is stored by
 *    columns) and, for a root j, only rows i > m_j of column j are taken, so
 *    each alternating 4-cycle is found from exactly one of its two columns.
 *    For such an edge {i,j} the cycle closes if the edge {m_j, m_i} exists;
 *    its gain (Section 3) is
 *        g = w(i,j) + w(m_j,m_i) - w(i,m_i) - w(m_j,j),
 *    evaluated in binary64 as (w(i,j) + w(m_j,m_i)) - (w(i,m_i) + w(m_j,j)).
 *    A cycle with g > 0 (strictly) is a candidate.
 *  Step C.  Per matched edge {m_j, j}, i.e. per root column j, keep the
 *    candidate of largest gain; equal gains go to the smallest row i.
 *  Step D.  Per matched edge {i, m_i}, i.e. per column c = m_i: if c kept a
 *    cycle of its own in Step C, c accepts nothing; otherwise c accepts,
 *    among the Step-C winners whose other matched edge is {m_c, c}, the one
 *    of largest gain, equal gains going to the smallest root column j.
 *  Flip.  Every accepted cycle is applied: m_j = i, m_i = j, m_c = old m_j,
 *    m_(old m_j) = c.  Accepted cycles are vertex-disjoint, so applying them
 *    one after another equals applying them at once.
 *
 * The loop ends after a round that applies nothing, or after max_rounds
 * rounds when max_rounds > 0 (the paper's maxiters, Section 4).
 *
 * Returns 0.  The caller guarantees a well-formed CSC and a perfect matching
 * contained in the pattern. */
int oracle_improve(int32_t n, const int64_t* col_ptr, const int32_t* row_idx, const double* w,
                   const int32_t* mate_in, int32_t max_rounds, int32_t* perm_out,
                   double* total_out, oracle_stats* st)
{
    oracle_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    if (n <= 0) {
        if (total_out) *total_out = 0.0;
        return 0;
    }
    size_t N = (size_t)n;
    int32_t* mc = (int32_t*)malloc(N * sizeof(int32_t));   /* m_j for column j */
    int32_t* mr = (int32_t*)malloc(N * sizeof(int32_t));   /* m_i for row i */
    double* wm = (double*)malloc(N * sizeof(double));      /* w(m_j, j) */
    int32_t* old_mc = (int32_t*)malloc(N * sizeof(int32_t));
    /* Step C winner of each root column */
    double* best_g = (double*)malloc(N * sizeof(double));
    int32_t* best_i = (int32_t*)malloc(N * sizeof(int32_t));
    int32_t* best_c = (int32_t*)malloc(N * sizeof(int32_t)); /* c = m_i */
    int64_t* best_k = (int64_t*)malloc(N * sizeof(int64_t)); /* position of {i,j} */
    int64_t* best_p = (int64_t*)malloc(N * sizeof(int64_t)); /* position of {m_j,m_i} */
    int32_t* accepted = (int32_t*)malloc(N * sizeof(int32_t)); /* Step D choice per column */

    for (int32_t j = 0; j < n; ++j) {
        mc[j] = mate_in[j];
        mr[mate_in[j]] = j;
        wm[j] = w[edge_pos(col_ptr, row_idx, mate_in[j], j)];
    }
    st->init_weight = oracle_tree_sum(wm, n);

    int32_t round = 0;
    for (;;) {
        if (max_rounds > 0 && round >= max_rounds) {
            st->hit_round_cap = 1;
            break;
        }
        /* Steps A, B and C for every root column j. */
        int32_t n_candidates = 0;
        for (int32_t j = 0; j < n; ++j) {
            int32_t m_j = mc[j];
            best_g[j] = 0.0;
            best_i[j] = -1;
            for (int64_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k) {
                int32_t i = row_idx[k];
                if (i <= m_j) continue;           /* rows i > m_j only */
                int32_t m_i = mr[i];
                int64_t p = edge_pos(col_ptr, row_idx, m_j, m_i); /* edge {m_j, m_i} */
                if (p < 0) continue;
                double g = (w[k] + w[p]) - (wm[m_i] + wm[j]);
                /* g > 0 and strictly better: ascending i keeps the smallest
                 * row among equal gains. */
                if (g > best_g[j]) {
                    best_g[j] = g;
                    best_i[j] = i;
                    best_c[j] = m_i;
                    best_k[j] = k;
                    best_p[j] = p;
                }
            }
            if (best_i[j] >= 0) ++n_candidates;
        }
        /* Step D for every column c. */
        for (int32_t c = 0; c < n; ++c) accepted[c] = -1;
        for (int32_t j = 0; j < n; ++j) {
            if (best_i[j] < 0) continue;
            int32_t c = best_c[j];
            if (best_i[c] >= 0) continue;          /* c kept its own cycle */
            int32_t a = accepted[c];
            /* ascending j keeps the smallest root among equal gains */
            if (a < 0 || best_g[j] > best_g[a]) accepted[c] = j;
        }
        /* Flip every accepted cycle, reading the round-start matching. */
        memcpy(old_mc, mc, N * sizeof(int32_t));
        int32_t n_applied = 0;
        for (int32_t c = 0; c < n; ++c) {
            int32_t j = accepted[c];
            if (j < 0) continue;
            int32_t i = best_i[j];
            int32_t l = old_mc[j];                 /* old m_j */
            mc[j] = i;
            mr[i] = j;
            mc[c] = l;
            mr[l] = c;
            wm[j] = w[best_k[j]];                  /* w(i, j) */
            wm[c] = w[best_p[j]];                  /* w(old m_j, c) */
            ++n_applied;
        }
        if (round < ORACLE_MAX_ROUND_STATS) {
            st->round_candidates[round] = n_candidates;
            st->round_applied[round] = n_applied;
        }
        st->cycles_applied += n_applied;
        ++round;
        if (n_applied == 0) break;
    }
    st->rounds = round;
    st->final_weight = oracle_tree_sum(wm, n);
    if (perm_out) memcpy(perm_out, mc, N * sizeof(int32_t));
    if (total_out) *total_out = st->final_weight;

    free(mc); free(mr); free(wm); free(old_mc);
    free(best_g); free(best_i); free(best_c); free(best_k); free(best_p); free(accepted);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Phase I.1: greedy maximal matching with the heavy-edge tie-break
 * (Section 5.2: when edges are picked greedily, heavier ones take
 * precedence).  Read here as bulk-synchronous proposal rounds:
 *   1. every unmatched column proposes to its unmatched row of largest
 *      weight (equal weights: smallest row);
 *   2. every row that received proposals accepts the proposer of largest
 *      weight (equal weights: smallest column);
 *   3. accepted pairs are matched.
 * The rounds stop when no unmatched column has an unmatched neighbour, so
 * the result is maximal.  With heavy == 0 the weights are ignored (the
 * ablation "without heuristic", Section 6.2): only the index order decides.
 * mc[j] / mr[i] receive the mates or -1; *rounds_out (nullable) the number
 * of proposal rounds run, counting the last one, which finds no proposal.
 * Returns the cardinality. */
int32_t oracle_greedy(int32_t n, const int64_t* col_ptr, const int32_t* row_idx,
                      const double* w, int32_t heavy, int32_t* mc, int32_t* mr,
                      int32_t* rounds_out)
{
    for (int32_t v = 0; v < n; ++v) { mc[v] = -1; mr[v] = -1; }
    if (rounds_out) *rounds_out = 0;
    if (n <= 0) return 0;
    size_t N = (size_t)n;
    int32_t* prop_row = (int32_t*)malloc(N * sizeof(int32_t)); /* row column j proposes to */
    double* prop_w = (double*)malloc(N * sizeof(double));
    int32_t* acc_col = (int32_t*)malloc(N * sizeof(int32_t));  /* proposer a row accepts */
    int32_t card = 0;
    for (;;) {
        int32_t any = 0;
        if (rounds_out) ++*rounds_out;
        for (int32_t j = 0; j < n; ++j) {
            prop_row[j] = -1;
            if (mc[j] >= 0) continue;
            for (int64_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k) {
                int32_t r = row_idx[k];
                if (mr[r] >= 0) continue;
                /* ascending rows: a strictly larger weight replaces */
                if (prop_row[j] < 0 || (heavy && w[k] > prop_w[j])) {
                    prop_row[j] = r;
                    prop_w[j] = w[k];
                }
            }
            if (prop_row[j] >= 0) any = 1;
        }
        if (!any) break;
        for (int32_t r = 0; r < n; ++r) acc_col[r] = -1;
        for (int32_t j = 0; j < n; ++j) {
            int32_t r = prop_row[j];
            if (r < 0) continue;
            int32_t a = acc_col[r];
            /* ascending columns: a strictly larger weight replaces */
            if (a < 0 || (heavy && prop_w[j] > prop_w[a])) acc_col[r] = j;
        }
        for (int32_t r = 0; r < n; ++r) {
            int32_t j = acc_col[r];
            if (j < 0) continue;
            mc[j] = r;
            mr[r] = j;
            ++card;
        }
    }
    free(prop_row); free(prop_w); free(acc_col);
    return card;
}

/* ------------------------------------------------------------------------ */
/* Phase I.2: maximum-cardinality matching by multi-source BFS phases
 * (Section 5.1: augmenting paths found by a frontier expansion, SpMSpV in
 * the paper; Section 5.2: the semiring "addition" is max, so among several
 * ways to reach a vertex the heavier edge wins).  One phase:
 *   - every unmatched column is the root of its own search tree and forms
 *     the first frontier;
 *   - level step: every row not yet visited in this phase that is adjacent
 *     to a frontier column of a still-growing tree is visited; its parent is
 *     the adjacent frontier column of largest edge weight (equal weights:
 *     smallest column), and it joins that column's tree;
 *   - a visited unmatched row ends a path; after the level, each tree that
 *     reached unmatched rows keeps the smallest such row and stops growing;
 *   - the next frontier is the mates of the newly visited matched rows of
 *     trees that are still growing;
 *   - when the frontier is empty, every recorded path is augmented (trees
 *     are vertex-disjoint, so the paths are too).
 * Phases repeat until one finds no path.  mc/mr hold a matching on entry
 * (e.g. from oracle_greedy) and the maximum matching on return.
 * *phases_out (nullable) receives the number of phases started with an
 * unmatched column (the last of them finds no path unless the matching
 * became perfect), *levels_out (nullable) the number of levels with a
 * nonempty frontier over all phases.  Returns the cardinality. */
int32_t oracle_mcm(int32_t n, const int64_t* col_ptr, const int32_t* row_idx, const double* w,
                   int32_t heavy, int32_t* mc, int32_t* mr, int32_t* phases_out,
                   int32_t* levels_out)
{
    if (phases_out) *phases_out = 0;
    if (levels_out) *levels_out = 0;
    if (n <= 0) return 0;
    size_t N = (size_t)n;
    int32_t* parent = (int32_t*)malloc(N * sizeof(int32_t));   /* row -> column it was reached from */
    double* parent_w = (double*)malloc(N * sizeof(double));
    int32_t* tree_of_row = (int32_t*)malloc(N * sizeof(int32_t));
    int32_t* tree_of_col = (int32_t*)malloc(N * sizeof(int32_t)); /* root column of the tree */
    int32_t* end_row = (int32_t*)malloc(N * sizeof(int32_t));     /* per root: chosen endpoint */
    int32_t* frontier = (int32_t*)malloc(N * sizeof(int32_t));
    int32_t* next = (int32_t*)malloc(N * sizeof(int32_t));
    int32_t* level_rows = (int32_t*)malloc(N * sizeof(int32_t));
    for (;;) {
        for (int32_t v = 0; v < n; ++v) {
            parent[v] = -1; tree_of_row[v] = -1; tree_of_col[v] = -1; end_row[v] = -1;
        }
        int32_t nf = 0;
        for (int32_t j = 0; j < n; ++j)
            if (mc[j] < 0) { frontier[nf++] = j; tree_of_col[j] = j; }
        if (nf == 0) break;                       /* already perfect */
        if (phases_out) ++*phases_out;
        int32_t found_any = 0;
        while (nf > 0) {
            if (levels_out) ++*levels_out;
            /* visit rows adjacent to the frontier; pick the parent by (w desc, col asc) */
            int32_t nl = 0;
            for (int32_t f = 0; f < nf; ++f) {
                int32_t c = frontier[f];
                int32_t t = tree_of_col[c];
                if (end_row[t] >= 0) continue;       /* tree already stopped */
                for (int64_t k = col_ptr[c]; k < col_ptr[c + 1]; ++k) {
                    int32_t r = row_idx[k];
                    if (tree_of_row[r] >= 0) continue; /* visited in an earlier level */
                    if (parent[r] < 0) {
                        parent[r] = c; parent_w[r] = w[k]; level_rows[nl++] = r;
                    } else if (heavy ? (w[k] > parent_w[r] || (w[k] == parent_w[r] && c < parent[r]))
                                     : (c < parent[r])) {
                        parent[r] = c; parent_w[r] = w[k];
                    }
                }
            }
            /* the level's rows join their parents' trees */
            for (int32_t q = 0; q < nl; ++q) {
                int32_t r = level_rows[q];
                tree_of_row[r] = tree_of_col[parent[r]];
            }
            /* endpoints: each tree keeps its smallest unmatched row */
            for (int32_t q = 0; q < nl; ++q) {
                int32_t r = level_rows[q];
                if (mr[r] >= 0) continue;
                int32_t t = tree_of_row[r];
                if (end_row[t] < 0 || r < end_row[t]) end_row[t] = r;
            }
            /* next frontier: mates of matched rows in trees still growing */
            int32_t nn = 0;
            for (int32_t q = 0; q < nl; ++q) {
                int32_t r = level_rows[q];
                if (mr[r] < 0) continue;
                int32_t t = tree_of_row[r];
                if (end_row[t] >= 0) continue;
                int32_t c = mr[r];
                tree_of_col[c] = t;
                next[nn++] = c;
            }
            for (int32_t q = 0; q < nn; ++q) frontier[q] = next[q];
            nf = nn;
        }
        /* augment every recorded path: walk from the endpoint up to the root */
        for (int32_t t = 0; t < n; ++t) {
            int32_t r = end_row[t];
            if (r < 0) continue;
            found_any = 1;
            while (r >= 0) {
                int32_t c = parent[r];
                int32_t r_next = mc[c];           /* -1 at the root */
                mc[c] = r;
                mr[r] = c;
                r = r_next;
            }
        }
        if (!found_any) break;
    }
    int32_t card = 0;
    for (int32_t j = 0; j < n; ++j) card += (mc[j] >= 0);
    free(parent); free(parent_w); free(tree_of_row); free(tree_of_col); free(end_row);
    free(frontier); free(next); free(level_rows);
    return card;
}

/* ------------------------------------------------------------------------ */
/* The HWPM pipeline (Section 5.1): greedy maximal matching, maximum
 * cardinality matching, then the WIAC rounds.  Returns 0, or -2 when the
 * matrix has no perfect matching (structurally singular, Section 3); the
 * outputs are untouched in that case. */
int oracle_match(int32_t n, const int64_t* col_ptr, const int32_t* row_idx, const double* w,
                 int32_t heavy, int32_t max_rounds, int32_t* perm_out, double* total_out,
                 oracle_stats* st, int32_t* mcm_card_out)
{
    if (n <= 0) {
        if (st) memset(st, 0, sizeof(*st));
        if (total_out) *total_out = 0.0;
        if (mcm_card_out) *mcm_card_out = 0;
        return 0;
    }
    size_t N = (size_t)n;
    int32_t* mc = (int32_t*)malloc(N * sizeof(int32_t));
    int32_t* mr = (int32_t*)malloc(N * sizeof(int32_t));
    int32_t g_rounds = 0, phases = 0, levels = 0;
    const int32_t g_card = oracle_greedy(n, col_ptr, row_idx, w, heavy, mc, mr, &g_rounds);
    int32_t card = oracle_mcm(n, col_ptr, row_idx, w, heavy, mc, mr, &phases, &levels);
    if (mcm_card_out) *mcm_card_out = card;
    int rc = 0;
    if (card < n) {
        rc = -2;
        if (st) memset(st, 0, sizeof(*st));
    } else {
        rc = oracle_improve(n, col_ptr, row_idx, w, mc, max_rounds, perm_out, total_out, st);
    }
    if (st) {
        st->greedy_rounds = g_rounds;
        st->greedy_cardinality = g_card;
        st->mcm_phases = phases;
        st->mcm_levels = levels;
    }
    free(mc); free(mr);
    return rc;
}
