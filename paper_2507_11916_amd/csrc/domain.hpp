// Host-side puzzle domains of the library: state validation, moves, packed
// encoding (the TensorRepresentation of the subtree-expansion algorithm),
// Manhattan distance and the corner pattern database.
#pragma once
#include <cstdint>
#include <vector>

#include "hb.h"

namespace hb {

constexpr int kMaxStateBytes = 54;
constexpr int kMaxActions = 18;

struct Domain {
    hb_domain id;
    int side;        // sliding tile: 3 or 4; cube: 0
    int state_bytes; // 9, 16, 54
    int packed_bytes;
    int n_actions;   // 4 or 18
};

const Domain* domain_of(hb_domain d);

void goal_state(const Domain& D, uint8_t* out);
bool is_goal(const Domain& D, const uint8_t* s);
// Returns false if the move is not applicable (blank would leave the board).
bool apply_move(const Domain& D, const uint8_t* s, int move, uint8_t* out);
// Parent pruning (sliding tile) or canonical pruning (cube).
bool move_allowed(const Domain& D, int prev_move, int move);
// Validation of a state's contents; `why` receives a message on failure.
bool valid_state(const Domain& D, const uint8_t* s, const char** why);
// Solvability (sliding-tile permutation parity; cube: corner/edge invariants).
bool solvable(const Domain& D, const uint8_t* s, const char** why);
int manhattan(const Domain& D, const uint8_t* s);

void encode(const Domain& D, const uint8_t* s, uint8_t* packed);
void decode(const Domain& D, const uint8_t* packed, uint8_t* s);

// Sticker index of the i-th non-centre sticker of the cube (i < 48).
int rc_noncentre_sticker(int i);

// Corner pattern database (cube).
struct CornerPdb {
    int k;
    std::vector<uint8_t> table;  // indexed by corner_index
    int64_t size;
    int lookup(const uint8_t* s) const;
};
bool corner_pdb_build(int k, int threads, CornerPdb* out);

// Additive (disjoint) pattern database of the 15-puzzle: tiles split into
// groups; table g holds, per placement of group g's tiles, the fewest moves of
// those tiles that bring them home (other tiles' moves free), minimised over
// the blank's cell.  h = sum over the groups.
struct StpApdb {
    std::vector<std::vector<int>> tiles;        // tiles of each group, ascending
    std::vector<std::vector<uint8_t>> tables;   // per group, indexed by placement rank
    int lookup(const uint8_t* s) const;
};
// group_of_tile[t] for t = 1..15 (entry 0 ignored): group 0..n-1, every group
// non-empty and at most 8 tiles.  Returns false on a bad grouping.
bool stp_apdb_build(const int32_t* group_of_tile, int threads, StpApdb* out);

}  // namespace hb

// Opaque handle of include/hb.h.
struct hb_pdb {
    int kind = 0;  // 0 cube corners, 1 15-puzzle additive
    hb::CornerPdb corner;
    hb::StpApdb stp;
};
