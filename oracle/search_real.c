/* Oracle search with a real-valued heuristic (Regression-Based Neural
 * Heuristics experiment: a regression network's output, less an offset, used
 * as h without rounding).  TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The same serial CB-DFS, IDA* and Budgeted Tree Search as search.c, with
 * f = g + h, the cost bounds and the minimum pruned f held as doubles (g is an
 * integer and h a float, so g + h is exact in double precision).  IDA*'s next
 * bound is the smallest pruned f, so with real values the bound grows by the
 * smallest f gap each iteration; BTS chooses bounds by expansion counts and
 * bisects over real bounds: probe = lo + (hi - lo) / 2.  h is read from a
 * table over 8-puzzle permutation ranks, or (any domain) computed per node as
 * max(0, y - offset) from the oracle's own double-precision network.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include "orc.h"

typedef struct {
    double bound;
    int64_t expanded, generated;
    int32_t complete;
    int32_t found;
    int64_t limit;
} orc_iter_real;

int orc_net_forward(const orc_net* m, const uint8_t* states, int64_t n, int mode, const double* act_scale,
                    double* y_out, double* act_max);

typedef struct {
    int domain;
    const float* table8f;
    const orc_net* net;
    double offset;
    double bound, next;
    int64_t expanded, generated, limit;
    int exceeded, stop_at_goal, found;
    int8_t path[512], cur[512];
    int path_len;
} rctx;

static double h_real(const rctx* c, const uint8_t* s) {
    if (!c->net) return (double)c->table8f[orc_perm9_rank(s)];
    double y;
    orc_net_forward(c->net, s, 1, 0, NULL, &y, NULL);
    const double v = y - c->offset;
    return v > 0.0 ? v : 0.0;
}

static int rdfs(rctx* c, const uint8_t* s, int g, int prev) {
    const double f = (double)g + h_real(c, s);
    if (f > c->bound) {
        if (f < c->next) c->next = f;
        return 0;
    }
    if (orc_is_goal(c->domain, s)) {
        if (!c->found) {
            c->found = 1;
            c->path_len = g;
            memcpy(c->path, c->cur, (size_t)g);
        }
        return c->stop_at_goal;
    }
    if (c->limit >= 0 && c->expanded >= c->limit) { c->exceeded = 1; return 1; }
    c->expanded++;
    for (int a = 0; a < orc_n_actions(c->domain); a++) {
        if (!orc_allowed(c->domain, prev, a)) continue;
        uint8_t ch[54];
        if (!orc_apply(c->domain, s, a, ch)) continue;
        c->generated++;
        if (g >= 511) continue;
        c->cur[g] = (int8_t)a;
        if (rdfs(c, ch, g + 1, a)) return 1;
    }
    return 0;
}

static int rcbdfs(rctx* c, const uint8_t* start, double bound) {
    c->bound = bound;
    c->next = INFINITY;
    c->expanded = c->generated = 0;
    c->exceeded = c->found = 0;
    rdfs(c, start, 0, -1);
    return !c->exceeded;
}

static int ida_real(rctx* cp, const uint8_t* start, int complete_final, int max_iters, int64_t node_limit,
                    orc_iter_real* iters, int* n_iters, int32_t* cost, int8_t* path, int* path_len);
static int bts_real(rctx* cp, const uint8_t* start, int64_t b0, int c1, int c2, int plus_one, int max_iters,
                    int64_t max_total, orc_iter_real* iters, int* n_iters, int32_t* cost, int8_t* path, int* path_len);

/* Serial IDA* on the 8-puzzle with a real-valued h table.  Returns as orc_ida. */
int orc_ida_real(const uint8_t* start, const float* table8f, int complete_final, int max_iters, int64_t node_limit,
                 orc_iter_real* iters, int* n_iters, int32_t* cost, int8_t* path, int* path_len) {
    rctx c;
    memset(&c, 0, sizeof(c));
    c.table8f = table8f;
    return ida_real(&c, start, complete_final, max_iters, node_limit, iters, n_iters, cost, path, path_len);
}

/* Serial IDA* on any domain with h = max(0, y - offset), y the network's
 * double-precision output for the state. */
int orc_ida_real_net(const orc_net* net, double offset, const uint8_t* start, int complete_final, int max_iters,
                     int64_t node_limit, orc_iter_real* iters, int* n_iters, int32_t* cost, int8_t* path,
                     int* path_len) {
    rctx c;
    memset(&c, 0, sizeof(c));
    c.domain = net->domain;
    c.net = net;
    c.offset = offset;
    return ida_real(&c, start, complete_final, max_iters, node_limit, iters, n_iters, cost, path, path_len);
}

static int ida_real(rctx* cp, const uint8_t* start, int complete_final, int max_iters, int64_t node_limit,
                    orc_iter_real* iters, int* n_iters, int32_t* cost, int8_t* path, int* path_len) {
    rctx c = *cp;
    c.stop_at_goal = !complete_final;
    double bound = h_real(&c, start);
    int64_t total = 0;
    *n_iters = 0;
    *cost = -1;
    for (int it = 0; it < max_iters; it++) {
        c.limit = node_limit >= 0 ? node_limit - total : -1;
        const int ok = rcbdfs(&c, start, bound);
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
        if (isinf(c.next)) return 0;
        bound = c.next;
    }
    return -1;
}

/* Serial BTS on the 8-puzzle with a real-valued h table (the control flow of
 * search.c's orc_bts over real bounds).  Returns as orc_bts. */
int orc_bts_real(const uint8_t* start, const float* table8f, int64_t b0, int c1, int c2, int plus_one, int max_iters,
                 int64_t max_total, orc_iter_real* iters, int* n_iters, int32_t* cost, int8_t* path, int* path_len) {
    rctx c;
    memset(&c, 0, sizeof(c));
    c.table8f = table8f;
    return bts_real(&c, start, b0, c1, c2, plus_one, max_iters, max_total, iters, n_iters, cost, path, path_len);
}

/* Serial BTS on any domain with h = max(0, y - offset) from the network. */
int orc_bts_real_net(const orc_net* net, double offset, const uint8_t* start, int64_t b0, int c1, int c2, int plus_one,
                     int max_iters, int64_t max_total, orc_iter_real* iters, int* n_iters, int32_t* cost, int8_t* path,
                     int* path_len) {
    rctx c;
    memset(&c, 0, sizeof(c));
    c.domain = net->domain;
    c.net = net;
    c.offset = offset;
    return bts_real(&c, start, b0, c1, c2, plus_one, max_iters, max_total, iters, n_iters, cost, path, path_len);
}

static int bts_real(rctx* cp, const uint8_t* start, int64_t b0, int c1, int c2, int plus_one, int max_iters,
                    int64_t max_total, orc_iter_real* iters, int* n_iters, int32_t* cost, int8_t* path, int* path_len) {
    rctx c = *cp;
    c.stop_at_goal = 0;
    const double hroot = h_real(&c, start);
    int64_t b = b0, total = 0;
    double lo_next = hroot;
    double probe = hroot + (plus_one ? 1.0 : 0.0);
    double hi = INFINITY;
    double step = 1.0;
    int n = 0;
    *cost = -1;
    *n_iters = 0;
    while (n < max_iters) {
        int unlimited = 0;
        if (!isinf(hi) && lo_next >= hi) { probe = hi; unlimited = 1; }
        c.limit = unlimited ? -1 : (int64_t)c2 * b;
        const int ok = rcbdfs(&c, start, probe);
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
            if (isinf(c.next)) return 0;
            lo_next = c.next;
            if (unlimited || c.expanded >= (int64_t)c1 * b) {
                if (c.expanded > b) b = c.expanded;
                hi = INFINITY;
                step = 1.0;
                probe = lo_next;
                continue;
            }
            if (isinf(hi)) {
                probe = lo_next + step - 1.0;
                step *= 2.0;
                continue;
            }
        } else {
            hi = probe;
        }
        if (!isinf(hi) && lo_next < hi) probe = lo_next + (hi - lo_next) / 2.0;
    }
    return -1;
}
