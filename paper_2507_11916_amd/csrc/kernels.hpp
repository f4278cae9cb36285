// Launch descriptors of the network kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hb {

struct GatherLaunch {
    int domain;             // 0 3x3, 1 4x4, 2 cube
    int prec;               // output type: 0 fp32, 1 bf16, 2 fp8
    const void* packed;     // device, packed states
    const int32_t* n_dev;   // device state count or null
    int n_host;
    int m_rows;             // rows written (>= n, padded rows are zero)
    const void* table;      // [t_rows][N] layer-1 table
    int table_f32;          // 1: float32 table, 0: bfloat16 table
    int t_rows;             // table rows (P * S)
    const float* bias;      // [N]
    int N;                  // padded width (multiple of 64)
    int ld_out;             // elements
    void* out;
    float out_inv_scale;    // fp8 output
};

struct GemmLaunch {
    int prec;               // 0 fp32, 1 bf16, 2 fp8
    int tile;               // index into the tile table
    const void* A;
    const void* Bt;
    void* C;
    const void* R;
    const float* bias;
    const float* colscale;
    const int32_t* m_dev;
    int m_host;
    int m_cap;              // largest M (grid shape)
    int N, K, lda, ldb, ldc;
    float a_scale, r_scale, out_inv_scale;
    int relu;
    int persistent_grid;    // > 0: at most this many blocks, striding over tiles
    int out_type = -1;      // type of C/R/Mk: -1 same as prec; 0 f32 (weight gradients from bf16)
    const void* Mk = nullptr;  // zero the result where this tensor (C's layout) is <= 0
    // Grouped product (ensembles): columns [g*group_n, (g+1)*group_n) of C use
    // A's columns [g*group_k, (g+1)*group_k).  0: one group.
    int group_n = 0, group_k = 0;
    // Split-K (tile ids 14-16 only; K / split a multiple of one 128-byte
    // stage): slice s multiplies K elements [s K / split, (s + 1) K / split)
    // into C + s * c_split elements (partial products, summed by the caller).
    int split = 1;
    int64_t c_split = 0;
    // Two zeroed ints per stream: with a persistent grid, blocks take tiles
    // after their first off tile_ctr[0] (each launch leaves both at zero).
    // Null: a persistent grid strides over the tiles statically.
    int* tile_ctr = nullptr;
    // Optional transposed copy of C (tile 14, float32 or bf16 outputs, no
    // split or persistent grid): element (m, n) also written at
    // Ct[n * ldct + m]; ldct a multiple of 8 and at least M rounded up to 256
    // (the rows the tiles cover).  Null: none.
    void* Ct = nullptr;
    int ldct = 0;
    int ct_rows = 0;  // rows of Ct written (the first ct_rows columns of C); 0: all N
    // Optional timing: the launch records the kernel's own start and end on
    // these two events (hipExtLaunchKernelGGL), so their elapsed time excludes
    // the dispatch.  Null: a plain launch.
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
};

struct HeadArgs {
    const void* X;          // [n][ldx] final activation
    int ldx, K;
    const void* W;          // [n_out][K]
    const float* b;         // [n_out]
    int n_out;
    float x_scale;          // fp8 activation scale
    const int32_t* n_dev;
    int n_host;
    int m_cap;              // rows the launch covers (clamps *n_dev)
    const void* packed;     // for the Manhattan minimum
    int domain;
    int mode;               // hb_out_mode
    float q, offset;
    int combine_md;         // 0 none, 1 min, 2 max, 3 plus (with Manhattan distance)
    int members;            // ensemble members (regression): x holds members * K values
    int ens_rule;           // 0 min, 1 sum of the members' outputs
    int32_t* h_out;
    float* raw;             // nullable
};

// The whole forward pass in one persistent launch (fused_forward_kernel):
// `grid` one-wave blocks; `sync` points at 4 + (n_layers + 1) * rb_cap zeroed
// ints that the launch leaves zeroed (rb_cap >= m_cap / 32 rounded up).
struct FusedLaunch {
    int domain, prec;
    const void* packed;
    const int32_t* n_dev;
    int n_host, m_cap;
    const void* table;      // float32 layer-1 table
    const float* bias1;
    int N1, ld1;
    void* out1;
    float out1_inv_scale;
    int n_layers;
    GemmLaunch layers[12];
    HeadArgs head;
    int* sync;
    int rb_cap;
    int spin_limit;
    int grid;
};

bool launch_gather(const GatherLaunch& L, hipStream_t s);
bool launch_fused(const FusedLaunch& L, hipStream_t s);
int fused_max_layers();
bool fused_enabled();  // false: the fused kernel is switched off and launch_fused refuses
bool launch_gemm(const GemmLaunch& L, hipStream_t s);
bool launch_head(const HeadArgs& H, int prec, int m_cap, hipStream_t s);
void launch_absmax(const float* x, int n, int N, int ld, unsigned* out, hipStream_t s);
int gemm_tile_count();
void gemm_tile_shape(int id, int* bm, int* bn);
hipError_t gemm_prepare_attributes();

}  // namespace hb
