/* Oracle search: serial cost-bounded depth-first search (CB-DFS) driving IDA*
 * and Budgeted Tree Search.  TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * IDA* (Background, Search Algorithms; Batch IDA* algorithm): the first bound
 * is h(start); each iteration is a depth-first search that expands a node when
 * g + h <= bound (the expansion condition of the correctness proof) and
 * records the smallest f of the pruned nodes; the next bound is that minimum.
 * The goal test is made when a node is taken for expansion.  Counters per
 * iteration: expanded = nodes taken with f <= bound that are not the goal;
 * generated = children created by those expansions.
 *
 * Budgeted Tree Search (Background; Batch BTS enhancements): repeated CB-DFS
 * with a cost bound and an expansion limit, searching over cost bounds so that
 * each accepted iteration's tree is at least c1 times the previous accepted
 * one, within a limit of c2 times it; the first budget is b0 = 10,000
 * expansions and the first bound h(root) + 1.  The exact control flow is this
 * library's reading (the cited BTS papers are not reproduced here):
 *   lo_next = h(root) (a lower bound on the optimal cost), b = b0,
 *   probe = h(root) + 1;
 *   repeat: run CB-DFS(probe, limit c2*b) to completion or to the limit;
 *     solution found (complete)   -> hi = probe; if lo_next >= probe stop
 *                                    (cost = probe), else bisect;
 *     complete, no solution, T    -> lo_next = min pruned f; accept the bound
 *                                    if T >= c1*b (b = T, probe = lo_next),
 *                                    else double the step (no hi yet) or bisect;
 *     exceeded                    -> hi = probe, bisect;
 *   bisect: if lo_next >= hi, run hi without a limit (its outcome is final for
 *   this window); else probe = lo_next + (hi - lo_next) / 2.
 * A search that finds the goal is always run to completion (so its counts do
 * not depend on the order in which solutions are met).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"

typedef struct {
    int kind;                /* 0 zero, 1 Manhattan, 2 table over 8-puzzle ranks, 3 corner PDB,
                                4 additive 15-puzzle PDB */
    const int32_t* table8;   /* kind 2: h by perm9 rank */
    int pdb_k;               /* kind 3 */
    const uint8_t* pdb;
    int apdb_groups;         /* kind 4: groups of at most 4 tiles (see orc_apdb_h) */
    const int32_t* apdb_tiles;
    const uint8_t* apdb_tables;
} orc_hspec;

typedef struct {
    int32_t bound;
    int64_t expanded, generated;
    int32_t complete; /* 1 complete, 0 stopped at a solution or at the limit */
    int32_t found;
    int64_t limit;
} orc_iter;

static int h_of(int d, const orc_hspec* h, const uint8_t* s) {
    switch (h->kind) {
    case 1: return orc_manhattan(d, s);
    case 2: return h->table8[orc_perm9_rank(s)];
    case 3: { int64_t i; orc_corner_k_index(s, h->pdb_k, &i); return h->pdb[i]; }
    case 4: return orc_apdb_h(s, h->apdb_groups, h->apdb_tiles, h->apdb_tables);
    default: return 0;
    }
}

typedef struct {
    int d;
    const orc_hspec* h;
    int32_t bound;
    int32_t next;        /* min pruned f */
    int64_t expanded, generated;
    int64_t limit;       /* expansions; < 0 = none */
    int exceeded;
    int stop_at_goal;
    int found;
    int8_t path[512];
    int path_len;
    int8_t cur[512];
} dfs_ctx;

static int dfs(dfs_ctx* c, const uint8_t* s, int g, int prev) {
    int f = g + h_of(c->d, c->h, s);
    if (f > c->bound) {
        if (f < c->next) c->next = f;
        return 0;
    }
    if (orc_is_goal(c->d, s)) {
        if (!c->found) {
            c->found = 1;
            c->path_len = g;
            memcpy(c->path, c->cur, (size_t)g);
        }
        return c->stop_at_goal;
    }
    if (c->limit >= 0 && c->expanded >= c->limit) { c->exceeded = 1; return 1; }
    c->expanded++;
    int na = orc_n_actions(c->d);
    for (int a = 0; a < na; a++) {
        if (!orc_allowed(c->d, prev, a)) continue;
        uint8_t ch[54];
        if (!orc_apply(c->d, s, a, ch)) continue;
        c->generated++;
        if (g >= 511) continue;
        c->cur[g] = (int8_t)a;
        if (dfs(c, ch, g + 1, a)) return 1;
    }
    return 0;
}

/* One cost-bounded DFS.  Returns 1 on completion (or solution when
 * stop_at_goal), 0 when the expansion limit was exceeded. */
static int cbdfs(dfs_ctx* c, const uint8_t* start, int32_t bound) {
    c->bound = bound;
    c->next = INT32_MAX;
    c->expanded = c->generated = 0;
    c->exceeded = 0;
    c->found = 0;
    dfs(c, start, 0, -1);
    return !c->exceeded;
}

/* Serial IDA*.  complete_final: finish the final iteration instead of
 * stopping at the first solution.  Returns 1 solved, 0 no solution, -1 node
 * budget hit (node_limit < 0: none). */
int orc_ida(int d, const uint8_t* start, const orc_hspec* h, int complete_final, int max_iters,
            int64_t node_limit, orc_iter* iters, int* n_iters, int32_t* cost, int8_t* path, int* path_len) {
    dfs_ctx c;
    memset(&c, 0, sizeof(c));
    c.d = d;
    c.h = h;
    c.stop_at_goal = !complete_final;
    int32_t bound = h_of(d, h, start);
    int64_t total = 0;
    *n_iters = 0;
    *cost = -1;
    for (int it = 0; it < max_iters; it++) {
        c.limit = node_limit >= 0 ? node_limit - total : -1;
        int ok = cbdfs(&c, start, bound);
        iters[it].bound = bound;
        iters[it].expanded = c.expanded;
        iters[it].generated = c.generated;
        iters[it].found = c.found;
        iters[it].complete = ok && (complete_final || !c.found);
        iters[it].limit = c.limit;
        *n_iters = it + 1;
        total += c.expanded;
        if (!ok) return -1;
        if (c.found) {
            *cost = c.path_len;
            *path_len = c.path_len;
            memcpy(path, c.path, (size_t)c.path_len);
            return 1;
        }
        if (c.next == INT32_MAX) return 0;
        bound = c.next;
    }
    return -1;
}

/* Serial Budgeted Tree Search (reading in the file header).  Each search run is
 * recorded in iters (bound, limit, complete, found, counts).  Returns 1 solved,
 * 0 no solution, -1 ran out of iteration slots or max_total expansions. */
int orc_bts(int d, const uint8_t* start, const orc_hspec* h, int64_t b0, int c1, int c2, int plus_one,
            int max_iters, int64_t max_total, orc_iter* iters, int* n_iters, int32_t* cost,
            int8_t* path, int* path_len) {
    dfs_ctx c;
    memset(&c, 0, sizeof(c));
    c.d = d;
    c.h = h;
    c.stop_at_goal = 0;
    int32_t hroot = h_of(d, h, start);
    int64_t b = b0, total = 0;
    int32_t lo_next = hroot;
    int32_t probe = hroot + (plus_one ? 1 : 0);
    int32_t hi = INT32_MAX;
    int32_t step = 1;
    int n = 0;
    *cost = -1;
    *n_iters = 0;
    while (n < max_iters) {
        int unlimited = 0;
        if (hi != INT32_MAX && lo_next >= hi) { probe = hi; unlimited = 1; }
        c.limit = unlimited ? -1 : (int64_t)c2 * b;
        int ok = cbdfs(&c, start, probe);
        iters[n].bound = probe;
        iters[n].limit = c.limit;
        iters[n].complete = ok;
        iters[n].found = ok && c.found;
        iters[n].expanded = c.expanded;
        iters[n].generated = c.generated;
        n++;
        *n_iters = n;
        total += c.expanded;
        if (max_total >= 0 && total > max_total) return -1;
        if (ok && c.found) {
            hi = probe;
            if (lo_next >= probe) {
                *cost = c.path_len;
                *path_len = c.path_len;
                memcpy(path, c.path, (size_t)c.path_len);
                return 1;
            }
        } else if (ok) {
            if (c.next == INT32_MAX) return 0;
            lo_next = c.next;
            if (unlimited || c.expanded >= (int64_t)c1 * b) {
                /* accepted iteration */
                if (c.expanded > b) b = c.expanded;
                hi = INT32_MAX;
                step = 1;
                probe = lo_next;
                continue;
            }
            if (hi == INT32_MAX) {
                probe = lo_next + step - 1;
                if (probe < lo_next) probe = lo_next;
                step *= 2;
                continue;
            }
        } else {
            hi = probe;
        }
        if (hi != INT32_MAX && lo_next < hi) probe = lo_next + (hi - lo_next) / 2;
    }
    return -1;
}
