/* Oracle domains: sliding-tile puzzles and the 3x3x3 Rubik's cube.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The paper's problem statement is a graph search from a start to a goal with
 * unit edge costs (Background, problem tuple); its domains are the 4x4 sliding
 * tile puzzle and the 3x3 Rubik's cube (Experimental Setup), plus the 8-puzzle
 * used here as the exhaustively checkable case.
 *
 * Sliding tile: byte p = tile at cell p (row-major), 0 = blank, goal tile p at
 * cell p.  Moves move the blank: 0 up, 1 left, 2 right, 3 down.  A move may not
 * undo the previous move (path information that keeps the search from going
 * back to the parent, AIDA* distributed node assignment).
 *
 * Rubik's cube: 54 stickers, sticker p = 9*f + 3*r + c on face f in
 * (U, D, L, R, F, B); byte p = colour (face index of the colour's home face).
 * This model is geometric: a sticker is a cubie position in {-1,0,1}^3 plus an
 * outward normal; a face turn rotates every sticker whose position lies in the
 * turning layer.  Face frame (normal n, column direction u, row direction v),
 * with x pointing L->R, y D->U, z B->F:
 *   U: n=+y u=+x v=+z     D: n=-y u=+x v=-z     L: n=-x u=+z v=-y
 *   R: n=+x u=-z v=-y     F: n=+z u=+x v=-y     B: n=-z u=-x v=-y
 * Sticker (f,r,c) sits at n + (c-1) u + (r-1) v.  Move m turns face m/3
 * clockwise (seen from outside the face), counter-clockwise or by a half turn
 * for m%3 = 0, 1, 2.  Canonical pruning (implied by the paper's reported
 * generated/expanded ratio on the cube): no two turns of the same face in a
 * row, and no turn of U, L or F directly after a turn of D, R or B.
 */
#include <string.h>
#include <stdlib.h>
#include "orc.h"

static const int FN[6][3] = {{0,1,0},{0,-1,0},{-1,0,0},{1,0,0},{0,0,1},{0,0,-1}};
static const int FU[6][3] = {{1,0,0},{1,0,0},{0,0,1},{0,0,-1},{1,0,0},{-1,0,0}};
static const int FV[6][3] = {{0,0,1},{0,0,-1},{0,-1,0},{0,-1,0},{0,-1,0},{0,-1,0}};

int orc_state_len(int d) { return d == ORC_STP3 ? 9 : d == ORC_STP4 ? 16 : 54; }
int orc_n_actions(int d) { return d == ORC_RUBIK ? 18 : 4; }

static int stp_side(int d) { return d == ORC_STP3 ? 3 : 4; }

static int stp_apply(int n, const uint8_t* s, int move, uint8_t* out) {
    int b = -1;
    for (int p = 0; p < n * n; p++) if (s[p] == 0) b = p;
    if (b < 0) return 0;
    int r = b / n, c = b % n;
    if (move == 0) r--; else if (move == 1) c--; else if (move == 2) c++; else if (move == 3) r++; else return 0;
    if (r < 0 || r >= n || c < 0 || c >= n) return 0;
    memcpy(out, s, (size_t)(n * n));
    out[b] = s[r * n + c];
    out[r * n + c] = 0;
    return 1;
}

static void sticker_geom(int p, int pos[3], int nrm[3]) {
    int f = p / 9, r = (p % 9) / 3, c = p % 3;
    for (int i = 0; i < 3; i++) {
        pos[i] = FN[f][i] + (c - 1) * FU[f][i] + (r - 1) * FV[f][i];
        nrm[i] = FN[f][i];
    }
}

static int sticker_index(const int pos[3], const int nrm[3]) {
    for (int f = 0; f < 6; f++) {
        if (FN[f][0] == nrm[0] && FN[f][1] == nrm[1] && FN[f][2] == nrm[2]) {
            int d[3] = {pos[0] - FN[f][0], pos[1] - FN[f][1], pos[2] - FN[f][2]};
            int c = d[0] * FU[f][0] + d[1] * FU[f][1] + d[2] * FU[f][2] + 1;
            int r = d[0] * FV[f][0] + d[1] * FV[f][1] + d[2] * FV[f][2] + 1;
            return 9 * f + 3 * r + c;
        }
    }
    return -1;
}

/* Rodrigues rotation of an integer vector about a unit axis by q quarter
 * turns, counter-clockwise when seen from the tip of the axis. */
static void rotate(const int a[3], int q, const int v[3], int out[3]) {
    static const int COS[4] = {1, 0, -1, 0}, SIN[4] = {0, 1, 0, -1};
    int c = COS[q & 3], s = SIN[q & 3];
    int cr[3] = {a[1] * v[2] - a[2] * v[1], a[2] * v[0] - a[0] * v[2], a[0] * v[1] - a[1] * v[0]};
    int dot = a[0] * v[0] + a[1] * v[1] + a[2] * v[2];
    for (int i = 0; i < 3; i++) out[i] = v[i] * c + cr[i] * s + a[i] * dot * (1 - c);
}

static int rc_apply_geometric(const uint8_t* s, int move, uint8_t* out) {
    int f = move / 3, kind = move % 3;
    int q = kind == 0 ? 3 : kind == 1 ? 1 : 2; /* clockwise = -90 degrees about the normal */
    uint8_t tmp[54];
    for (int p = 0; p < 54; p++) {
        int pos[3], nrm[3];
        sticker_geom(p, pos, nrm);
        int layer = pos[0] * FN[f][0] + pos[1] * FN[f][1] + pos[2] * FN[f][2];
        if (layer == 1) {
            int p2[3], n2[3];
            rotate(FN[f], q, pos, p2);
            rotate(FN[f], q, nrm, n2);
            tmp[sticker_index(p2, n2)] = s[p];
        } else {
            tmp[p] = s[p];
        }
    }
    memcpy(out, tmp, 54);
    return 1;
}

/* The geometric turn is a fixed permutation of sticker positions; it is
 * computed once per move from the geometry (by turning a state whose byte p
 * is p) and then applied by lookup. */
static uint8_t rc_perm[18][54];

__attribute__((constructor)) static void rc_perm_init(void) {
    uint8_t id[54];
    for (int p = 0; p < 54; p++) id[p] = (uint8_t)p;
    for (int m = 0; m < 18; m++) rc_apply_geometric(id, m, rc_perm[m]);
}

static int rc_apply(const uint8_t* s, int move, uint8_t* out) {
    const uint8_t (*perm)[54] = rc_perm;
    if (move < 0 || move >= 18) return 0;
    uint8_t tmp[54];
    for (int p = 0; p < 54; p++) tmp[p] = s[perm[move][p]];
    memcpy(out, tmp, 54);
    return 1;
}

int orc_apply(int d, const uint8_t* s, int move, uint8_t* out) {
    if (d == ORC_RUBIK) return rc_apply(s, move, out);
    return stp_apply(stp_side(d), s, move, out);
}

int orc_allowed(int d, int prev, int move) {
    if (prev < 0) return 1;
    if (d == ORC_RUBIK) {
        int f = move / 3, pf = prev / 3;
        if (f == pf) return 0;
        if (f % 2 == 0 && pf == f + 1) return 0;
        return 1;
    }
    return move != 3 - prev;
}

void orc_goal(int d, uint8_t* out) {
    if (d == ORC_RUBIK) { for (int p = 0; p < 54; p++) out[p] = (uint8_t)(p / 9); return; }
    int n = stp_side(d);
    for (int p = 0; p < n * n; p++) out[p] = (uint8_t)p;
}

int orc_is_goal(int d, const uint8_t* s) {
    uint8_t g[54];
    orc_goal(d, g);
    return memcmp(g, s, (size_t)orc_state_len(d)) == 0;
}

/* Manhattan distance: sum over non-blank tiles of row and column offsets from
 * the tile's goal cell. */
int orc_manhattan(int d, const uint8_t* s) {
    if (d == ORC_RUBIK) return 0;
    int n = stp_side(d), md = 0;
    for (int p = 0; p < n * n; p++) {
        int t = s[p];
        if (t == 0) continue;
        md += abs(p / n - t / n) + abs(p % n - t % n);
    }
    return md;
}

/* Lehmer-code rank of a permutation of 0..8 (9! values). */
int64_t orc_perm9_rank(const uint8_t* s) {
    static const int64_t FACT[10] = {1, 1, 2, 6, 24, 120, 720, 5040, 40320, 362880};
    int64_t r = 0;
    for (int i = 0; i < 9; i++) {
        int smaller = 0;
        for (int j = i + 1; j < 9; j++) if (s[j] < s[i]) smaller++;
        r += smaller * FACT[8 - i];
    }
    return r;
}

/* ------------------------------------------------------------------------
 * Exported helpers (ctypes)
 * ---------------------------------------------------------------------- */
int orc_apply_seq(int d, const uint8_t* start, const int8_t* moves, int n, uint8_t* out) {
    uint8_t cur[54], nxt[54];
    memcpy(cur, start, (size_t)orc_state_len(d));
    for (int i = 0; i < n; i++) {
        if (moves[i] < 0) break;
        if (!orc_apply(d, cur, moves[i], nxt)) return 0;
        memcpy(cur, nxt, (size_t)orc_state_len(d));
    }
    memcpy(out, cur, (size_t)orc_state_len(d));
    return 1;
}

/* Apply padded move sequences (rows of length L, -1 = end) to the goal. */
int orc_apply_seq_batch(int d, const int8_t* moves, int64_t count, int L, uint8_t* out) {
    uint8_t g[54];
    orc_goal(d, g);
    int sl = orc_state_len(d);
    for (int64_t i = 0; i < count; i++)
        if (!orc_apply_seq(d, g, moves + i * L, L, out + i * sl)) return 0;
    return 1;
}

int orc_manhattan_batch(int d, const uint8_t* s, int64_t n, int32_t* out) {
    int sl = orc_state_len(d);
    for (int64_t i = 0; i < n; i++) out[i] = orc_manhattan(d, s + i * sl);
    return 1;
}

/* Breadth-first search from the goal over every reachable 8-puzzle state.
 * dist[rank] = distance, or -1 for the 9!/2 unreachable permutations.
 * Returns the number of reached states. */
int64_t orc_bfs8(int8_t* dist) {
    const int64_t N = 362880;
    for (int64_t i = 0; i < N; i++) dist[i] = -1;
    uint8_t* q = (uint8_t*)malloc((size_t)N * 9);
    int64_t head = 0, tail = 0;
    orc_goal(ORC_STP3, q);
    dist[orc_perm9_rank(q)] = 0;
    tail = 1;
    while (head < tail) {
        uint8_t* s = q + head * 9;
        int ds = dist[orc_perm9_rank(s)];
        head++;
        for (int m = 0; m < 4; m++) {
            uint8_t c[9];
            if (!orc_apply(ORC_STP3, s, m, c)) continue;
            int64_t r = orc_perm9_rank(c);
            if (dist[r] >= 0) continue;
            dist[r] = (int8_t)(ds + 1);
            memcpy(q + tail * 9, c, 9);
            tail++;
        }
    }
    free(q);
    return tail;
}

/* Every 8-puzzle state reachable from the goal, in BFS order. */
int64_t orc_all8(uint8_t* out) {
    const int64_t N = 362880;
    int8_t* seen = (int8_t*)calloc((size_t)N, 1);
    int64_t head = 0, tail = 1;
    orc_goal(ORC_STP3, out);
    seen[orc_perm9_rank(out)] = 1;
    while (head < tail) {
        uint8_t* s = out + head * 9;
        head++;
        for (int m = 0; m < 4; m++) {
            uint8_t c[9];
            if (!orc_apply(ORC_STP3, s, m, c)) continue;
            int64_t r = orc_perm9_rank(c);
            if (seen[r]) continue;
            seen[r] = 1;
            memcpy(out + tail * 9, c, 9);
            tail++;
        }
    }
    free(seen);
    return tail;
}

/* ------------------------------------------------------------------------
 * Corner pattern database on the cube (abstraction: where the first k corner
 * cubies are and how they are twisted).  Corner position i has coordinates
 * x = (i&1 ? 1 : -1), y = (i&2 ? 1 : -1), z = (i&4 ? 1 : -1).  The cubie that
 * is home at position j is tracked for j < k; it is recognised by the set of
 * its three colours.  Its twist is the axis (y = 0, x = 1, z = 2) on which its
 * U- or D-coloured sticker currently lies.
 * ---------------------------------------------------------------------- */
static void corner_stickers(int i, int st[3]) {
    int x = (i & 1) ? 1 : -1, y = (i & 2) ? 1 : -1, z = (i & 4) ? 1 : -1;
    int pos[3] = {x, y, z};
    int ny[3] = {0, y, 0}, nx[3] = {x, 0, 0}, nz[3] = {0, 0, z};
    st[0] = sticker_index(pos, ny);
    st[1] = sticker_index(pos, nx);
    st[2] = sticker_index(pos, nz);
}

static int colour_set(const uint8_t* s, int i) {
    int st[3];
    corner_stickers(i, st);
    return (1 << s[st[0]]) | (1 << s[st[1]]) | (1 << s[st[2]]);
}

/* Abstract index = rank of (positions of cubies 0..k-1 as a partial
 * permutation of 8) * 3^k + sum twist_j * 3^j. */
static int home_set[8];

__attribute__((constructor)) static void home_set_init(void) {
    uint8_t g[54];
    orc_goal(ORC_RUBIK, g);
    for (int j = 0; j < 8; j++) home_set[j] = colour_set(g, j);
}

int orc_corner_k_index(const uint8_t* s, int k, int64_t* idx) {
    int pos[8], tw[8];
    for (int j = 0; j < k; j++) pos[j] = -1;
    for (int i = 0; i < 8; i++) {
        int cs = colour_set(s, i);
        for (int j = 0; j < k; j++) {
            if (cs == home_set[j]) {
                int st[3];
                corner_stickers(i, st);
                pos[j] = i;
                tw[j] = (s[st[0]] <= 1) ? 0 : (s[st[1]] <= 1) ? 1 : 2;
            }
        }
    }
    int64_t r = 0;
    int used[8] = {0};
    for (int j = 0; j < k; j++) {
        if (pos[j] < 0) return 0;
        int smaller = 0;
        for (int t = 0; t < pos[j]; t++) if (!used[t]) smaller++;
        used[pos[j]] = 1;
        r = r * (8 - j) + smaller;
    }
    for (int j = k - 1; j >= 0; j--) r = r * 3 + tw[j];
    *idx = r;
    return 1;
}

int64_t orc_corner_k_size(int k) {
    int64_t n = 1;
    for (int j = 0; j < k; j++) n *= (8 - j);
    for (int j = 0; j < k; j++) n *= 3;
    return n;
}

/* Breadth-first search over the abstract corner space.  Each abstract state
 * keeps a full sticker state that maps to it; applying a turn to that state and
 * abstracting again gives the abstract successor, because corner cubies move
 * independently of the rest of the cube.  Returns the number of reached
 * entries; table entries are distances (255 = unreached). */
int64_t orc_corner_pdb(int k, uint8_t* table) {
    int64_t size = orc_corner_k_size(k);
    memset(table, 255, (size_t)size);
    int64_t cap = 1 << 20;
    uint8_t* cur = (uint8_t*)malloc((size_t)cap * 54);
    uint8_t* nxt = (uint8_t*)malloc((size_t)cap * 54);
    int64_t ncur = 1, reached = 1;
    orc_goal(ORC_RUBIK, cur);
    int64_t idx;
    orc_corner_k_index(cur, k, &idx);
    table[idx] = 0;
    for (int depth = 0; ncur > 0; depth++) {
        int64_t nn = 0;
        for (int64_t i = 0; i < ncur; i++) {
            for (int m = 0; m < 18; m++) {
                uint8_t c[54];
                orc_apply(ORC_RUBIK, cur + i * 54, m, c);
                orc_corner_k_index(c, k, &idx);
                if (table[idx] != 255) continue;
                table[idx] = (uint8_t)(depth + 1);
                reached++;
                if (nn == cap) {
                    cap *= 2;
                    nxt = (uint8_t*)realloc(nxt, (size_t)cap * 54);
                    cur = (uint8_t*)realloc(cur, (size_t)cap * 54);
                }
                memcpy(nxt + nn * 54, c, 54);
                nn++;
            }
        }
        uint8_t* t = cur; cur = nxt; nxt = t;
        ncur = nn;
    }
    free(cur);
    free(nxt);
    return reached;
}

int orc_corner_k_index_batch(const uint8_t* s, int64_t n, int k, int64_t* out) {
    for (int64_t i = 0; i < n; i++) if (!orc_corner_k_index(s + i * 54, k, out + i)) return 0;
    return 1;
}

/* ------------------------------------------------------------------------
 * Additive pattern database of the 15-puzzle (the paper's classic
 * sliding-tile heuristic, Experimental Setup), for test-sized groups of at
 * most 4 tiles.  A group's abstract state is the cells of its tiles plus the
 * blank's cell, coded densely as digits base 16 (tile i's cell is digit i, the
 * blank the top digit).  Moving the blank into a cell that holds none of the
 * group's tiles costs 0; sliding one of the group's tiles into the blank costs
 * 1.  Distances from the goal come from a 0-1 breadth-first search with one
 * bucket per distance; the table keeps, per placement of the tiles, the least
 * distance over the blank's cells (255 where two tiles share a cell).
 * ---------------------------------------------------------------------- */
int orc_apdb_group(int k, const int32_t* tiles, uint8_t* table) {
    if (k < 1 || k > 6) return 0;
    int64_t n_place = 1;
    for (int i = 0; i < k; i++) n_place *= 16;
    const int64_t n_state = n_place * 16;
    uint8_t* dist = (uint8_t*)malloc((size_t)n_state);
    if (!dist) return 0;
    memset(dist, 255, (size_t)n_state);
    /* buckets[d] = states first reached at distance d (a state may appear in
       a later bucket too; stale copies are skipped) */
    int64_t* bucket[256];
    int64_t fill[256], cap[256];
    for (int d = 0; d < 256; d++) { bucket[d] = NULL; fill[d] = 0; cap[d] = 0; }
    int64_t goal = 0, mul = 1;
    for (int i = 0; i < k; i++) { goal += (int64_t)tiles[i] * mul; mul *= 16; }
    goal += 0 * n_place; /* blank at cell 0 */
    dist[goal] = 0;
    cap[0] = 1024; bucket[0] = (int64_t*)malloc(sizeof(int64_t) * 1024);
    if (!bucket[0]) { free(dist); return 0; }
    bucket[0][fill[0]++] = goal;
    for (int d = 0; d < 255; d++) {
        for (int64_t q = 0; q < fill[d]; q++) {
            const int64_t st = bucket[d][q];
            if (dist[st] != d) continue;
            int cell[6];
            int64_t rest = st;
            for (int i = 0; i < k; i++) { cell[i] = (int)(rest % 16); rest /= 16; }
            const int blank = (int)rest;
            const int br = blank / 4, bc = blank % 4;
            const int dr[4] = {-1, 1, 0, 0}, dc[4] = {0, 0, -1, 1};
            for (int m = 0; m < 4; m++) {
                const int r = br + dr[m], c = bc + dc[m];
                if (r < 0 || r > 3 || c < 0 || c > 3) continue;
                const int nb = r * 4 + c;
                int who = -1;
                for (int i = 0; i < k; i++) if (cell[i] == nb) who = i;
                int ncell[6];
                for (int i = 0; i < k; i++) ncell[i] = cell[i];
                int step = 0;
                if (who >= 0) { ncell[who] = blank; step = 1; }
                int64_t ns = 0, mm = 1;
                for (int i = 0; i < k; i++) { ns += (int64_t)ncell[i] * mm; mm *= 16; }
                ns += (int64_t)nb * n_place;
                const int nd = d + step;
                if (dist[ns] <= nd) continue;
                dist[ns] = (uint8_t)nd;
                if (fill[nd] == cap[nd]) {
                    cap[nd] = cap[nd] ? 2 * cap[nd] : 1024;
                    int64_t* grown = (int64_t*)realloc(bucket[nd], sizeof(int64_t) * (size_t)cap[nd]);
                    if (!grown) {
                        for (int e = 0; e < 256; e++) free(bucket[e]);
                        free(dist);
                        return 0;
                    }
                    bucket[nd] = grown;
                }
                bucket[nd][fill[nd]++] = ns;
            }
        }
        free(bucket[d]);
        bucket[d] = NULL;
    }
    for (int64_t p = 0; p < n_place; p++) {
        uint8_t best = 255;
        for (int b = 0; b < 16; b++) if (dist[p + (int64_t)b * n_place] < best) best = dist[p + (int64_t)b * n_place];
        table[p] = best;
    }
    free(dist);
    return 1;
}

/* h of a 15-puzzle state under an additive PDB: groups of at most 4 tiles,
 * tiles[g*4 + i] (-1 past the group's end), tables[g * 65536 + code] with
 * code = sum over the group's tiles of cell * 16^i. */
int orc_apdb_h(const uint8_t* s, int n_groups, const int32_t* tiles, const uint8_t* tables) {
    int where[16];
    for (int c = 0; c < 16; c++) where[s[c]] = c;
    int h = 0;
    for (int g = 0; g < n_groups; g++) {
        int64_t code = 0, mul = 1;
        for (int i = 0; i < 4 && tiles[g * 4 + i] >= 0; i++) { code += (int64_t)where[tiles[g * 4 + i]] * mul; mul *= 16; }
        h += tables[(int64_t)g * 65536 + code];
    }
    return h;
}

/* One group's table of any size (1 to 6 tiles): out[i] = table[code] for
 * state i, code = sum over the group's tiles of cell * 16^i. */
int orc_apdb_group_lookup(int k, const int32_t* tiles, const uint8_t* table, const uint8_t* s, int64_t n,
                          int32_t* out) {
    for (int64_t b = 0; b < n; b++) {
        int where[16];
        for (int c = 0; c < 16; c++) where[s[b * 16 + c]] = c;
        int64_t code = 0, mul = 1;
        for (int i = 0; i < k; i++) { code += (int64_t)where[tiles[i]] * mul; mul *= 16; }
        out[b] = table[code];
    }
    return 1;
}

int orc_apdb_h_batch(const uint8_t* s, int64_t n, int n_groups, const int32_t* tiles, const uint8_t* tables,
                     int32_t* out) {
    for (int64_t i = 0; i < n; i++) out[i] = orc_apdb_h(s + i * 16, n_groups, tiles, tables);
    return 1;
}
