// Launch descriptors of the training kernels (train.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hb {

struct HeadTrainArgs {
    const void* X;        // [m_pad][ldx] last hidden activation (type t)
    int ldx, K;           // K: padded width, multiple of 256, <= 1024
    const void* W;        // [K] head weights (type t), zero past the true width
    const float* b;       // [1]
    const float* labels;  // [n]
    int n, m_pad;
    float inv_n;
    int asym;
    float alpha;
    void* delta;          // [m_pad][ldx] output (type t)
    float* part;          // [head_train_blocks(m_pad)][K + 2] per-block partial sums
    float* dWo;           // [K] written
    float* dbo_loss;      // [2] written: output bias gradient, loss
    float* y_out;         // [n] or null
};

struct TransposeArgs {
    const void* in;
    int ld_in;
    void* out;
    int ld_out;
    int R, C;
    float* colsum;   // null or [C], written: column sums over rows < rows_sum
    int rows_sum;
    float* colpart;  // [ceil(rows_sum / 64)][C] scratch when colsum is set
};

struct ScatterArgs {
    const void* dz;      // [n][ld] gradient at layer 1's pre-activation (type t)
    int ld;
    const void* packed;  // [n] packed states (hb_encode layout)
    int n, N1;           // N1: padded width, multiple of 128
    float* partial;      // [chunks][table rows + 1][N1] per-chunk sums (last row: bias)
    int chunk;           // states per chunk
    float* dW1;          // [gradient rows][ld_w], the weight file's row order
    int ld_w;
    float* db1;          // [N1]
};


void launch_fill(float* p, int64_t n, float v, hipStream_t s);
bool launch_head_train(const HeadTrainArgs& a, int t, hipStream_t s);
int head_train_blocks(int m_pad);
void launch_column_sum(const float* part, int rows, int cols, int ld, float* out, hipStream_t s);
// Fixed-order sum of `split` partial matrices (split-K weight gradients).
void launch_splitk_sum(const float* part, int split, int64_t stride, int rows, int cols, int ldp, float* out, int ldo,
                       hipStream_t s);
void launch_transpose(const TransposeArgs& a, int t, hipStream_t s);
// Layer-1 weight and bias gradients (transpose of the gather-sum), in a fixed
// summation order: bitwise repeatable.
bool launch_scatter_l1(const ScatterArgs& a, int t, int domain, int chunks, hipStream_t s);
// out[r] = sum over b < n of X[r * ld + b] (type t), r < rows, in a fixed order.
void launch_row_sum(const void* X, int ld, int rows, int n, float* out, int t, hipStream_t s);

// Every parameter tensor's Adam step in one launch (one grid row per tensor).
struct AdamTensor {
    float* master;
    float* m;
    float* v;
    const float* grad;
    int64_t gk, gn;
    int K, N;
    void* out1;
    int64_t s1k, s1n;
    void* out2;
    int64_t s2k, s2n;
};
void launch_multi_adam(const AdamTensor* d_tensors, int count, float lr, float b1, float b2, float eps, float c1,
                       float c2, int t, hipStream_t s);

// Cube layer 1: the working table (48 non-centre stickers x 6 colours, type t,
// row stride N1_pad) and folded bias (bias + the six centre rows) from the
// master weights [54 * 6][N1].
void launch_cube_fold(const float* master, const float* bias, int N1, int N1_pad, void* table, float* bias_work, int t,
                      hipStream_t s);
int scatter_table_rows(int domain);  // 81, 256, 288
hipError_t train_prepare_attributes();

}  // namespace hb
