/* Oracle internals.  TEST INFRASTRUCTURE ONLY: the oracle is a plain, slow,
 * double-precision CPU model of what the batched-heuristic search computes.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no source with the library in paper_2507_11916_amd/.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#define ORC_STP3 0
#define ORC_STP4 1
#define ORC_RUBIK 2

/* domain.c */
int orc_state_len(int domain);
int orc_n_actions(int domain);
int orc_apply(int domain, const uint8_t* s, int move, uint8_t* out);
int orc_allowed(int domain, int prev_move, int move);
int orc_is_goal(int domain, const uint8_t* s);
void orc_goal(int domain, uint8_t* out);
int orc_manhattan(int domain, const uint8_t* s);
int64_t orc_perm9_rank(const uint8_t* s);
int orc_corner_k_index(const uint8_t* s, int k, int64_t* idx);
int orc_apdb_h(const uint8_t* s, int n_groups, const int32_t* tiles, const uint8_t* tables);

/* mlp.c */
#define ORC_MAXT 64
typedef struct {
    int domain, n_in, n_dense, dims[8], n_res, n_out, head_kind;
    int P, S, nt;
    int rows[ORC_MAXT], cols[ORC_MAXT];
    double* T[ORC_MAXT]; /* tensors in file order */
} orc_net;
double orc_bf16_round(double x);
double orc_e4m3_round(double x);

#endif
