// Host-side domains: sliding tile and the 3x3x3 cube (sticker model driven by
// per-face permutation tables), packed encoding, Manhattan distance, corner
// pattern database.
#include "domain.hpp"

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <thread>

namespace hb {

static const Domain kDomains[3] = {
    {HB_STP3, 3, 9, 8, 4},
    {HB_STP4, 4, 16, 8, 4},
    {HB_RUBIK3, 0, 54, 24, 18},
};

const Domain* domain_of(hb_domain d) {
    if ((int)d < 0 || (int)d > 2) return nullptr;
    return &kDomains[(int)d];
}

// ----------------------------------------------------------------- cube
// A clockwise quarter turn of face f rotates the face's own stickers
// (r, c) -> (c, 2 - r) and carries four strips of three side stickers one step
// around the face: strip k moves onto strip k+1, element i onto element i.
static const int kStrips[6][4][3] = {
    /* U */ {{36, 37, 38}, {18, 19, 20}, {45, 46, 47}, {27, 28, 29}},
    /* D */ {{42, 43, 44}, {33, 34, 35}, {51, 52, 53}, {24, 25, 26}},
    /* L */ {{0, 3, 6}, {36, 39, 42}, {9, 12, 15}, {53, 50, 47}},
    /* R */ {{38, 41, 44}, {2, 5, 8}, {51, 48, 45}, {11, 14, 17}},
    /* F */ {{6, 7, 8}, {27, 30, 33}, {11, 10, 9}, {26, 23, 20}},
    /* B */ {{0, 1, 2}, {24, 21, 18}, {17, 16, 15}, {29, 32, 35}},
};

struct CubeTables {
    uint8_t src[18][54];  // new[p] = old[src[m][p]]
    uint8_t dst[18][54];  // sticker at p moves to dst[m][p]
    CubeTables() {
        for (int f = 0; f < 6; f++) {
            uint8_t cw[54];  // dst map of the clockwise turn
            for (int p = 0; p < 54; p++) cw[p] = (uint8_t)p;
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) cw[9 * f + 3 * r + c] = (uint8_t)(9 * f + 3 * c + (2 - r));
            for (int k = 0; k < 4; k++)
                for (int i = 0; i < 3; i++) cw[kStrips[f][k][i]] = (uint8_t)kStrips[f][(k + 1) % 4][i];
            // quarter, inverse quarter (three quarters), half (two quarters)
            for (int kind = 0; kind < 3; kind++) {
                int reps = kind == 0 ? 1 : kind == 1 ? 3 : 2;
                uint8_t d[54];
                for (int p = 0; p < 54; p++) {
                    int q = p;
                    for (int t = 0; t < reps; t++) q = cw[q];
                    d[p] = (uint8_t)q;
                }
                int m = 3 * f + kind;
                for (int p = 0; p < 54; p++) {
                    dst[m][p] = d[p];
                    src[m][d[p]] = (uint8_t)p;
                }
            }
        }
    }
};
static const CubeTables kCube;

// Sticker indices of the cubie at (x, y, z): its faces on the y axis (U/D),
// the x axis (L/R) and the z axis (F/B); -1 where the coordinate is 0.
static void cubie_stickers(int x, int y, int z, int st[3]) {
    st[0] = y == 1 ? 3 * (z + 1) + (x + 1) : y == -1 ? 9 + 3 * (1 - z) + (x + 1) : -1;
    st[1] = x == -1 ? 18 + 3 * (1 - y) + (z + 1) : x == 1 ? 27 + 3 * (1 - y) + (1 - z) : -1;
    st[2] = z == 1 ? 36 + 3 * (1 - y) + (x + 1) : z == -1 ? 45 + 3 * (1 - y) + (1 - x) : -1;
}

static void corner_pos(int i, int* x, int* y, int* z) {
    *x = (i & 1) ? 1 : -1;
    *y = (i & 2) ? 1 : -1;
    *z = (i & 4) ? 1 : -1;
}

int rc_noncentre_sticker(int i) { return i + i / 8 + (i % 8 >= 4 ? 1 : 0); }

// ---------------------------------------------------------------- common
void goal_state(const Domain& D, uint8_t* out) {
    if (D.id == HB_RUBIK3) {
        for (int p = 0; p < 54; p++) out[p] = (uint8_t)(p / 9);
    } else {
        for (int p = 0; p < D.state_bytes; p++) out[p] = (uint8_t)p;
    }
}

bool is_goal(const Domain& D, const uint8_t* s) {
    if (D.id == HB_RUBIK3) {
        for (int p = 0; p < 54; p++)
            if (s[p] != p / 9) return false;
        return true;
    }
    for (int p = 0; p < D.state_bytes; p++)
        if (s[p] != p) return false;
    return true;
}

bool apply_move(const Domain& D, const uint8_t* s, int move, uint8_t* out) {
    if (move < 0 || move >= D.n_actions) return false;
    if (D.id == HB_RUBIK3) {
        const uint8_t* src = kCube.src[move];
        for (int p = 0; p < 54; p++) out[p] = s[src[p]];
        return true;
    }
    const int n = D.side;
    int b = 0;
    while (b < n * n && s[b] != 0) b++;
    if (b == n * n) return false;
    int r = b / n, c = b % n;
    switch (move) {
        case 0: if (r == 0) return false; r--; break;
        case 1: if (c == 0) return false; c--; break;
        case 2: if (c == n - 1) return false; c++; break;
        default: if (r == n - 1) return false; r++; break;
    }
    std::memcpy(out, s, (size_t)(n * n));
    out[b] = s[r * n + c];
    out[r * n + c] = 0;
    return true;
}

bool move_allowed(const Domain& D, int prev, int move) {
    if (prev < 0) return true;
    if (D.id == HB_RUBIK3) {
        const int f = move / 3, pf = prev / 3;
        if (f == pf) return false;
        return !((f & 1) == 0 && pf == f + 1);
    }
    return move != 3 - prev;
}

int manhattan(const Domain& D, const uint8_t* s) {
    if (D.id == HB_RUBIK3) return 0;
    const int n = D.side;
    int md = 0;
    for (int p = 0; p < n * n; p++) {
        const int t = s[p];
        if (t) md += std::abs(p / n - t / n) + std::abs(p % n - t % n);
    }
    return md;
}

bool valid_state(const Domain& D, const uint8_t* s, const char** why) {
    if (D.id == HB_RUBIK3) {
        int cnt[6] = {0};
        for (int p = 0; p < 54; p++) {
            if (s[p] > 5) { *why = "colour out of range 0..5"; return false; }
            cnt[s[p]]++;
        }
        for (int c = 0; c < 6; c++)
            if (cnt[c] != 9) { *why = "each colour must appear nine times"; return false; }
        for (int f = 0; f < 6; f++)
            if (s[9 * f + 4] != f) { *why = "centre stickers must stay in place"; return false; }
        return true;
    }
    unsigned seen = 0;
    for (int p = 0; p < D.state_bytes; p++) {
        if (s[p] >= D.state_bytes) { *why = "tile out of range"; return false; }
        seen |= 1u << s[p];
    }
    if (seen != (1u << D.state_bytes) - 1u) { *why = "tiles must form a permutation"; return false; }
    return true;
}

static int perm_parity(const int* a, int n) {
    int inv = 0;
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) inv += a[i] > a[j];
    return inv & 1;
}

bool solvable(const Domain& D, const uint8_t* s, const char** why) {
    if (!valid_state(D, s, why)) return false;
    if (D.id != HB_RUBIK3) {
        // Each move swaps the blank with a neighbour: the permutation parity
        // and the parity of the blank's distance from its goal cell change together.
        const int n = D.side;
        int a[16], b = 0;
        for (int p = 0; p < n * n; p++) { a[p] = s[p]; if (!s[p]) b = p; }
        const int dist = b / n + b % n;
        if (perm_parity(a, n * n) != (dist & 1)) { *why = "unreachable sliding-tile permutation"; return false; }
        return true;
    }
    // Cube: identify corner and edge cubies by colour sets; twist and flip sums
    // and the permutation parities must match those of reachable states.
    uint8_t g[54];
    goal_state(D, g);
    int cperm[8], ctw = 0;
    for (int i = 0; i < 8; i++) {
        int x, y, z, st[3];
        corner_pos(i, &x, &y, &z);
        cubie_stickers(x, y, z, st);
        // clockwise order of the three faces around the corner
        int ord[3] = {st[0], st[1], st[2]};
        if (x * y * z < 0) std::swap(ord[1], ord[2]);
        int set = (1 << s[st[0]]) | (1 << s[st[1]]) | (1 << s[st[2]]);
        cperm[i] = -1;
        for (int j = 0; j < 8; j++) {
            int xj, yj, zj, sj[3];
            corner_pos(j, &xj, &yj, &zj);
            cubie_stickers(xj, yj, zj, sj);
            if (set == ((1 << g[sj[0]]) | (1 << g[sj[1]]) | (1 << g[sj[2]]))) cperm[i] = j;
        }
        if (cperm[i] < 0) { *why = "impossible corner colours"; return false; }
        for (int t = 0; t < 3; t++)
            if (s[ord[t]] <= 1) ctw += t;
    }
    int used = 0;
    for (int i = 0; i < 8; i++) used |= 1 << cperm[i];
    if (used != 255) { *why = "duplicate corner cubie"; return false; }
    if (ctw % 3) { *why = "twisted corner"; return false; }
    int eperm[12], ne = 0, eflip = 0;
    int ehome[12][2];
    for (int x = -1; x <= 1; x++)
        for (int y = -1; y <= 1; y++)
            for (int z = -1; z <= 1; z++) {
                if ((x == 0) + (y == 0) + (z == 0) != 1) continue;
                int st[3], a[2], k = 0;
                cubie_stickers(x, y, z, st);
                for (int t = 0; t < 3; t++) if (st[t] >= 0) a[k++] = st[t];
                ehome[ne][0] = a[0];
                ehome[ne][1] = a[1];
                ne++;
            }
    for (int e = 0; e < 12; e++) {
        const int set = (1 << s[ehome[e][0]]) | (1 << s[ehome[e][1]]);
        eperm[e] = -1;
        for (int j = 0; j < 12; j++)
            if (set == ((1 << g[ehome[j][0]]) | (1 << g[ehome[j][1]]))) eperm[e] = j;
        if (eperm[e] < 0) { *why = "impossible edge colours"; return false; }
        // reference facelet: U/D if present, else F/B; reference colour likewise
        const int c0 = s[ehome[e][0]], c1 = s[ehome[e][1]];
        const int ref_colour = (c0 <= 1 || c1 <= 1) ? (c0 <= 1 ? c0 : c1) : (c0 >= 4 ? c0 : c1);
        // ehome[e][0] is the facelet on the lowest axis in (y, x, z) order
        eflip += (s[ehome[e][0]] == ref_colour) ? 0 : 1;
    }
    int eused = 0;
    for (int e = 0; e < 12; e++) eused |= 1 << eperm[e];
    if (eused != 4095) { *why = "duplicate edge cubie"; return false; }
    if (eflip & 1) { *why = "flipped edge"; return false; }
    if (perm_parity(cperm, 8) != perm_parity(eperm, 12)) { *why = "odd cubie permutation"; return false; }
    return true;
}

// --------------------------------------------------------------- packing
void encode(const Domain& D, const uint8_t* s, uint8_t* packed) {
    if (D.id == HB_RUBIK3) {
        uint64_t w[3] = {0, 0, 0};
        for (int q = 0; q < 48; q++) w[q / 16] |= (uint64_t)(s[rc_noncentre_sticker(q)] & 7) << (3 * (q % 16));
        std::memcpy(packed, w, 24);
        return;
    }
    uint64_t w = 0;
    for (int p = 0; p < D.state_bytes; p++) w |= (uint64_t)(s[p] & 15) << (4 * p);
    std::memcpy(packed, &w, 8);
}

void decode(const Domain& D, const uint8_t* packed, uint8_t* s) {
    if (D.id == HB_RUBIK3) {
        uint64_t w[3];
        std::memcpy(w, packed, 24);
        for (int f = 0; f < 6; f++) s[9 * f + 4] = (uint8_t)f;
        for (int q = 0; q < 48; q++) s[rc_noncentre_sticker(q)] = (uint8_t)((w[q / 16] >> (3 * (q % 16))) & 7);
        return;
    }
    uint64_t w;
    std::memcpy(&w, packed, 8);
    for (int p = 0; p < D.state_bytes; p++) s[p] = (uint8_t)((w >> (4 * p)) & 15);
}

// -------------------------------------------------- corner pattern database
// Cubie j (j < k) is the corner whose home position has x = (j&1 ? +1 : -1),
// y = (j&2 ? +1 : -1), z = (j&4 ? +1 : -1).  Its twist is the axis (y 0, x 1,
// z 2) of the face that shows its U- or D-coloured sticker.  Index = mixed-radix
// rank of the positions (radices 8, 7, ...) * 3^k + twists (cubie 0 lowest).
struct CornerMoves {
    uint8_t to[18][8][3];  // (position, twist) -> packed (position << 2 | twist)
    int home_set[8];
    CornerMoves() {
        uint8_t g[54];
        goal_state(kDomains[2], g);
        int slot_pos[54], slot_axis[54];
        for (int p = 0; p < 54; p++) slot_pos[p] = slot_axis[p] = -1;
        for (int i = 0; i < 8; i++) {
            int x, y, z, st[3];
            corner_pos(i, &x, &y, &z);
            cubie_stickers(x, y, z, st);
            for (int a = 0; a < 3; a++) { slot_pos[st[a]] = i; slot_axis[st[a]] = a; }
            home_set[i] = (1 << g[st[0]]) | (1 << g[st[1]]) | (1 << g[st[2]]);
        }
        for (int m = 0; m < 18; m++)
            for (int i = 0; i < 8; i++) {
                int x, y, z, st[3];
                corner_pos(i, &x, &y, &z);
                cubie_stickers(x, y, z, st);
                for (int a = 0; a < 3; a++) {
                    const int d = kCube.dst[m][st[a]];
                    to[m][i][a] = (uint8_t)(slot_pos[d] << 2 | slot_axis[d]);
                }
            }
    }
};
static const CornerMoves kCorner;

static int64_t corner_size(int k) {
    int64_t n = 1;
    for (int j = 0; j < k; j++) n *= 8 - j;
    for (int j = 0; j < k; j++) n *= 3;
    return n;
}

static int64_t corner_rank(int k, const int* pos, const int* tw) {
    int64_t r = 0;
    int used = 0;
    for (int j = 0; j < k; j++) {
        const int smaller = __builtin_popcount((unsigned)(~used) & ((1u << pos[j]) - 1u));
        used |= 1 << pos[j];
        r = r * (8 - j) + smaller;
    }
    for (int j = k - 1; j >= 0; j--) r = r * 3 + tw[j];
    return r;
}

static void corner_unrank(int k, int64_t r, int* pos, int* tw) {
    for (int j = 0; j < k; j++) { tw[j] = (int)(r % 3); r /= 3; }
    int digit[8];
    for (int j = k - 1; j >= 0; j--) { digit[j] = (int)(r % (8 - j)); r /= (8 - j); }
    int used = 0;
    for (int j = 0; j < k; j++) {
        int cnt = -1, p = 0;
        for (p = 0; p < 8; p++) {
            if (used & (1 << p)) continue;
            if (++cnt == digit[j]) break;
        }
        pos[j] = p;
        used |= 1 << p;
    }
}

int CornerPdb::lookup(const uint8_t* s) const {
    int pos[8], tw[8];
    for (int i = 0; i < 8; i++) {
        int x, y, z, st[3];
        corner_pos(i, &x, &y, &z);
        cubie_stickers(x, y, z, st);
        const int set = (1 << s[st[0]]) | (1 << s[st[1]]) | (1 << s[st[2]]);
        for (int j = 0; j < k; j++)
            if (set == kCorner.home_set[j]) {
                pos[j] = i;
                tw[j] = s[st[0]] <= 1 ? 0 : s[st[1]] <= 1 ? 1 : 2;
            }
    }
    return table[(size_t)corner_rank(k, pos, tw)];
}

bool corner_pdb_build(int k, int threads, CornerPdb* out) {
    if (k < 1 || k > 8) return false;
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    threads = std::min(threads, 256);
    out->k = k;
    out->size = corner_size(k);
    out->table.assign((size_t)out->size, 255);
    uint8_t* T = out->table.data();
    int pos0[8], tw0[8];
    for (int j = 0; j < k; j++) { pos0[j] = j; tw0[j] = 0; }
    T[corner_rank(k, pos0, tw0)] = 0;
    for (int depth = 0;; depth++) {
        std::atomic<int64_t> added{0};
        auto work = [&](int64_t lo, int64_t hi) {
            int64_t local = 0;
            int pos[8], tw[8], np[8], nt[8];
            for (int64_t r = lo; r < hi; r++) {
                // other threads fill level depth + 1 meanwhile: read atomically
                if (__atomic_load_n(&T[r], __ATOMIC_RELAXED) != depth) continue;
                corner_unrank(k, r, pos, tw);
                for (int m = 0; m < 18; m++) {
                    for (int j = 0; j < k; j++) {
                        const int t = kCorner.to[m][pos[j]][tw[j]];
                        np[j] = t >> 2;
                        nt[j] = t & 3;
                    }
                    const int64_t nr = corner_rank(k, np, nt);
                    uint8_t expect = 255;
                    if (__atomic_load_n(&T[nr], __ATOMIC_RELAXED) == 255 &&
                        __atomic_compare_exchange_n(&T[nr], &expect, (uint8_t)(depth + 1), false, __ATOMIC_RELAXED,
                                                    __ATOMIC_RELAXED))
                        local++;
                }
            }
            added += local;
        };
        std::vector<std::thread> pool;
        const int64_t chunk = (out->size + threads - 1) / threads;
        for (int t = 0; t < threads; t++) {
            const int64_t lo = t * chunk, hi = std::min(out->size, lo + chunk);
            if (lo < hi) pool.emplace_back(work, lo, hi);
        }
        for (auto& th : pool) th.join();
        if (added.load() == 0) break;
    }
    return true;
}

// ------------------------------------------------------------ 15-puzzle additive PDB
// Placement of k tiles: digit i is tile i's cell counted among the cells not
// taken by tiles 0..i-1 (mixed radix 16, 15, ...), rank = digits in that radix.
static int64_t placement_count(int k) {
    int64_t n = 1;
    for (int i = 0; i < k; i++) n *= 16 - i;
    return n;
}

static int64_t placement_rank(int k, const int* cell) {
    int64_t r = 0;
    uint32_t used = 0;
    for (int i = 0; i < k; i++) {
        const int d = cell[i] - __builtin_popcount(used & ((1u << cell[i]) - 1));
        r = r * (16 - i) + d;
        used |= 1u << cell[i];
    }
    return r;
}

static void placement_unrank(int k, int64_t r, int* cell) {
    int d[8];
    for (int i = k - 1; i >= 0; i--) {
        d[i] = (int)(r % (16 - i));
        r /= 16 - i;
    }
    uint32_t used = 0;
    for (int i = 0; i < k; i++) {
        int c = 0, left = d[i];
        for (;; c++) {
            if (used & (1u << c)) continue;
            if (left-- == 0) break;
        }
        cell[i] = c;
        used |= 1u << c;
    }
}

static inline bool lower_to(uint8_t* p, uint8_t v) {  // atomic min; true if the cell was unset
    uint8_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (cur > v) {
        if (__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) return cur == 255;
    }
    return false;
}

// Breadth-first over (placement, blank cell) in levels of pattern-tile moves.
// A level-c pass takes each placement with a cell at distance c, spreads c
// over the blank's region of free cells (blank moves into free cells cost
// nothing) and gives c + 1 to the placements one tile move away.  Distances
// only decrease to their final values, with atomic minima between threads.
static void build_group(const std::vector<int>& tiles, int threads, std::vector<uint8_t>* table) {
    const int k = (int)tiles.size();
    const int64_t n = placement_count(k);
    std::vector<uint8_t> dist((size_t)n * 16, 255);
    uint8_t* D = dist.data();
    {
        int cell[8];
        for (int i = 0; i < k; i++) cell[i] = tiles[i];  // tile t's home is cell t
        const int64_t r = placement_rank(k, cell);
        // the blank's region from cell 0 in the goal placement
        uint32_t occ = 0;
        for (int i = 0; i < k; i++) occ |= 1u << cell[i];
        uint32_t region = 1u, frontier = 1u;
        while (frontier) {
            uint32_t next = 0;
            for (int b = 0; b < 16; b++) {
                if (!(frontier & (1u << b))) continue;
                const int row = b >> 2, col = b & 3;
                if (row > 0) next |= 1u << (b - 4);
                if (row < 3) next |= 1u << (b + 4);
                if (col > 0) next |= 1u << (b - 1);
                if (col < 3) next |= 1u << (b + 1);
            }
            next &= ~occ & ~region;
            region |= next;
            frontier = next;
        }
        for (int b = 0; b < 16; b++)
            if (region & (1u << b)) D[r * 16 + b] = 0;
    }
    // Rows to visit at the next level: a bit per placement, set when a cell of
    // the row receives the next level's distance (only such rows can hold
    // cells at that level; a row whose cells were lowered further meanwhile
    // is skipped by its row test).
    const int64_t nwords = (n + 63) / 64;
    std::vector<uint64_t> cur_rows((size_t)nwords, 0), next_rows((size_t)nwords, 0);
    {
        int cell[8];
        for (int i = 0; i < k; i++) cell[i] = tiles[i];
        const int64_t r = placement_rank(k, cell);
        cur_rows[(size_t)(r >> 6)] |= 1ull << (r & 63);
    }
    for (int c = 0; c < 254; c++) {
        std::atomic<int64_t> added{0};
        uint64_t* NR = next_rows.data();
        auto work = [&](int64_t wlo, int64_t whi) {
            int64_t local = 0;
            int cell[8];
            const uint64_t cc8 = 0x0101010101010101ull * (uint64_t)c;
            for (int64_t wi = wlo; wi < whi; wi++) {
                uint64_t bits = cur_rows[(size_t)wi];
                while (bits) {
                const int64_t r = wi * 64 + __builtin_ctzll(bits);
                bits &= bits - 1;
                uint8_t* row = D + r * 16;
                // the row as two relaxed 64-bit loads (other threads lower
                // cells meanwhile); a byte equals c exactly where its XOR with
                // c is zero, found word-wide without carries between bytes
                uint64_t w[2] = {__atomic_load_n(reinterpret_cast<uint64_t*>(row), __ATOMIC_RELAXED),
                                 __atomic_load_n(reinterpret_cast<uint64_t*>(row) + 1, __ATOMIC_RELAXED)};
                uint32_t at_c = 0;
                for (int h = 0; h < 2; h++) {
                    const uint64_t x = w[h] ^ cc8;
                    const uint64_t z = ~(((x & 0x7F7F7F7F7F7F7F7Full) + 0x7F7F7F7F7F7F7F7Full) | x | 0x7F7F7F7F7F7F7F7Full);
                    if (!z) continue;
                    for (int b = 0; b < 8; b++)
                        if (z & (0x80ull << (8 * b))) at_c |= 1u << (8 * h + b);
                }
                if (!at_c) continue;
                placement_unrank(k, r, cell);
                uint32_t occ = 0;
                int tile_at[16];
                for (int b = 0; b < 16; b++) tile_at[b] = -1;
                for (int i = 0; i < k; i++) {
                    occ |= 1u << cell[i];
                    tile_at[cell[i]] = i;
                }
                // spread c over the free cells reachable from the level-c cells
                uint32_t region = at_c & ~occ, frontier = region;
                while (frontier) {
                    uint32_t next = 0;
                    for (int b = 0; b < 16; b++) {
                        if (!(frontier & (1u << b))) continue;
                        const int rr = b >> 2, cc = b & 3;
                        if (rr > 0) next |= 1u << (b - 4);
                        if (rr < 3) next |= 1u << (b + 4);
                        if (cc > 0) next |= 1u << (b - 1);
                        if (cc < 3) next |= 1u << (b + 1);
                    }
                    next &= ~occ & ~region;
                    region |= next;
                    frontier = next;
                }
                for (int b = 0; b < 16; b++)
                    if ((region & (1u << b)) && lower_to(&row[b], (uint8_t)c)) local++;
                // one pattern-tile move: the tile next to the blank slides into it
                // (all of the row's targets are found and prefetched first, so
                // their cache misses overlap)
                int64_t tgt[64];
                int nt = 0;
                for (int b = 0; b < 16; b++) {
                    if (!(region & (1u << b))) continue;
                    const int rr = b >> 2, cc = b & 3;
                    const int nb4[4] = {rr > 0 ? b - 4 : -1, rr < 3 ? b + 4 : -1, cc > 0 ? b - 1 : -1,
                                        cc < 3 ? b + 1 : -1};
                    for (int e = 0; e < 4; e++) {
                        const int t = nb4[e] < 0 ? -1 : tile_at[nb4[e]];
                        if (t < 0) continue;
                        int moved[8];
                        for (int i = 0; i < k; i++) moved[i] = cell[i];
                        moved[t] = b;  // the tile takes the blank's cell, the blank takes the tile's
                        const int64_t nr = placement_rank(k, moved);
                        tgt[nt++] = nr * 16 + nb4[e];
                        __builtin_prefetch(&D[nr * 16], 1);
                    }
                }
                for (int q = 0; q < nt; q++)
                    if (lower_to(&D[tgt[q]], (uint8_t)(c + 1))) {
                        local++;
                        const int64_t nr = tgt[q] >> 4;
                        __atomic_fetch_or(&NR[nr >> 6], 1ull << (nr & 63), __ATOMIC_RELAXED);
                    }
                }
            }
            added += local;
        };
        std::vector<std::thread> pool;
        const int64_t chunk = (nwords + threads - 1) / threads;
        for (int t = 0; t < threads; t++) {
            const int64_t lo = t * chunk, hi = std::min(nwords, lo + chunk);
            if (lo < hi) pool.emplace_back(work, lo, hi);
        }
        for (auto& th : pool) th.join();
        if (added.load() == 0) break;
        cur_rows.swap(next_rows);
        std::fill(next_rows.begin(), next_rows.end(), 0ull);
    }
    table->assign((size_t)n, 255);
    for (int64_t r = 0; r < n; r++) {
        uint8_t m = 255;
        for (int b = 0; b < 16; b++) m = std::min(m, D[r * 16 + b]);
        (*table)[r] = m;
    }
}

bool stp_apdb_build(const int32_t* group_of_tile, int threads, StpApdb* out) {
    if (!group_of_tile) return false;
    int n_groups = 0;
    for (int t = 1; t < 16; t++) {
        if (group_of_tile[t] < 0 || group_of_tile[t] > 14) return false;
        n_groups = std::max(n_groups, group_of_tile[t] + 1);
    }
    out->tiles.assign(n_groups, {});
    for (int t = 1; t < 16; t++) out->tiles[group_of_tile[t]].push_back(t);
    for (auto& g : out->tiles)
        if (g.empty() || g.size() > 8) return false;
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    threads = std::min(threads, 256);
    out->tables.assign(n_groups, {});
    for (int g = 0; g < n_groups; g++) build_group(out->tiles[g], threads, &out->tables[g]);
    return true;
}

int StpApdb::lookup(const uint8_t* s) const {
    int where[16];
    for (int c = 0; c < 16; c++) where[s[c]] = c;
    int h = 0;
    for (size_t g = 0; g < tiles.size(); g++) {
        int cell[8];
        const int k = (int)tiles[g].size();
        for (int i = 0; i < k; i++) cell[i] = where[tiles[g][i]];
        h += tables[g][placement_rank(k, cell)];
    }
    return h;
}

}  // namespace hb
