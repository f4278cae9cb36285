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
    float* dWo;           // [K] accumulated
    float* dbo;           // [1] accumulated
    float* loss;          // [1] accumulated
    float* y_out;         // [n] or null
};

struct TransposeArgs {
    const void* in;
    int ld_in;
    void* out;
    int ld_out;
    int R, C;
    float* colsum;  // null or [C], accumulated over rows < rows_sum
    int rows_sum;
};

struct ScatterArgs {
    const void* dz;      // [n][ld] gradient at layer 1's pre-activation (type t)
    int ld;
    const void* packed;  // [n] sliding-tile packed states
    int n, N1;           // N1: padded width, multiple of 64
    float* dW1;          // [P*S][ld_w]
    int ld_w;
    float* db1;          // [N1]
    int states_per_block;
};

struct AdamArgs {
    float* master;
    float* m;
    float* v;
    const float* grad;
    int64_t gk, gn;
    int K, N;
    float lr, b1, b2, eps, c1, c2;
    void* out1;
    int64_t s1k, s1n;
    void* out2;
    int64_t s2k, s2n;
};

void launch_fill(float* p, int64_t n, float v, hipStream_t s);
bool launch_head_train(const HeadTrainArgs& a, int t, hipStream_t s);
void launch_transpose(const TransposeArgs& a, int t, hipStream_t s);
bool launch_scatter_l1(const ScatterArgs& a, int t, int side, hipStream_t s);
void launch_adam(const AdamArgs& a, int t, hipStream_t s);

}  // namespace hb
