// HIP kernels of on-GPU training of the heuristic network (regression head,
// sliding-tile inputs): loss and output-layer gradient, transposes with fused
// bias-gradient column sums, the layer-1 scatter-add (transpose of the
// gather-sum), Adam with re-cast of the working weights, and a fill kernel.
// The matrix products (forward, input gradients, weight gradients) run on the
// MFMA GEMM of kernels.hip.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "train.hpp"

namespace hb {

__device__ __forceinline__ float tr_bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t tr_f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
template <int T>
__device__ __forceinline__ float ld_t(const void* p, size_t i) {
    return T == 0 ? reinterpret_cast<const float*>(p)[i] : tr_bf16_to_f32(reinterpret_cast<const uint16_t*>(p)[i]);
}
template <int T>
__device__ __forceinline__ void st_t(void* p, size_t i, float v) {
    if (T == 0) reinterpret_cast<float*>(p)[i] = v;
    else reinterpret_cast<uint16_t*>(p)[i] = tr_f32_to_bf16(v);
}

__global__ void fill_kernel(float* p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ------------------------------------------------------------------ head
// One wave per row, 8 rows per wave, 4 waves per block.  y = w.x + b;
// loss += w_b (y - t)^2 / n; dy = 2 w_b (y - t) / n; delta_k = dy * w_k where
// x_k > 0 (gradient at the pre-activation of the last hidden layer).  Rows >= n
// get delta = 0.  dWo and dbo are reduced over the block's rows in LDS and then
// added atomically.
constexpr int kHeadRowsPerWave = 8;
constexpr int kHeadMaxGroups = 4;  // K <= 1024

template <int T>
__global__ __launch_bounds__(256) void head_train_kernel(HeadTrainArgs a) {
    __shared__ float s_w[4][kHeadMaxGroups * 256];
    __shared__ float s_b[4], s_l[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int groups = (a.K + 255) / 256;  // lanes own 4 columns per group; columns >= K are skipped
    float accw[kHeadMaxGroups][4];
    for (int gi = 0; gi < kHeadMaxGroups; gi++)
        for (int e = 0; e < 4; e++) accw[gi][e] = 0.f;
    float accb = 0.f, accl = 0.f;
    const int row0 = (blockIdx.x * 4 + wave) * kHeadRowsPerWave;
    for (int rr = 0; rr < kHeadRowsPerWave; rr++) {
        const int r = row0 + rr;
        if (r >= a.m_pad) break;
        float x[kHeadMaxGroups][4];
        float part = 0.f;
        for (int gi = 0; gi < groups; gi++)
            for (int e = 0; e < 4; e++) {
                const int k = gi * 256 + lane * 4 + e;
                x[gi][e] = k < a.K ? ld_t<T>(a.X, (size_t)r * a.ldx + k) : 0.f;
                if (k < a.K) part += x[gi][e] * ld_t<T>(a.W, k);
            }
        for (int s = 32; s >= 1; s >>= 1) part += __shfl_xor(part, s, 64);
        float dy = 0.f;
        if (r < a.n) {
            const float y = part + a.b[0];
            const float d = y - a.labels[r];
            const float wgt = (a.asym && d > 0.f) ? a.alpha : 1.f;
            dy = 2.f * wgt * d * a.inv_n;
            accl += wgt * d * d * a.inv_n;
            accb += dy;
            if (a.y_out && lane == 0) a.y_out[r] = y;
        }
        for (int gi = 0; gi < groups; gi++)
            for (int e = 0; e < 4; e++) {
                const int k = gi * 256 + lane * 4 + e;
                if (k >= a.K) continue;
                const float dlt = x[gi][e] > 0.f ? dy * ld_t<T>(a.W, k) : 0.f;
                st_t<T>(a.delta, (size_t)r * a.ldx + k, dlt);
                accw[gi][e] += x[gi][e] * dy;
            }
    }
    for (int gi = 0; gi < kHeadMaxGroups; gi++)
        for (int e = 0; e < 4; e++) s_w[wave][gi * 256 + lane * 4 + e] = accw[gi][e];
    if (lane == 0) { s_b[wave] = accb; s_l[wave] = accl; }
    __syncthreads();
    for (int k = threadIdx.x; k < a.K; k += 256) {
        const float v = s_w[0][k] + s_w[1][k] + s_w[2][k] + s_w[3][k];
        if (v != 0.f) atomicAdd(&a.dWo[k], v);
    }
    if (threadIdx.x == 0) {
        atomicAdd(a.dbo, s_b[0] + s_b[1] + s_b[2] + s_b[3]);
        atomicAdd(a.loss, s_l[0] + s_l[1] + s_l[2] + s_l[3]);
    }
}

// ------------------------------------------------------------- transpose
// out[c][r] = in[r][c] for r < R, c < C through a 64 x 64 LDS tile; with
// colsum, every column's sum over rows < rows_sum is added atomically.
template <int T>
__global__ __launch_bounds__(256) void transpose_kernel(TransposeArgs a) {
    __shared__ float tile[64][65];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    for (int i = ty; i < 64; i += 4) {
        const int r = r0 + i, c = c0 + tx;
        tile[i][tx] = (r < a.R && c < a.C) ? ld_t<T>(a.in, (size_t)r * a.ld_in + c) : 0.f;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int c = c0 + i, r = r0 + tx;
        if (c < a.C && r < a.R) st_t<T>(a.out, (size_t)c * a.ld_out + r, tile[tx][i]);
    }
    if (a.colsum && ty == 0) {
        float s = 0.f;
        for (int i = 0; i < 64; i++)
            if (r0 + i < a.rows_sum) s += tile[i][tx];
        if (c0 + tx < a.C && s != 0.f) atomicAdd(&a.colsum[c0 + tx], s);
    }
}

// ------------------------------------------------------------ layer 1
// dW1[p*S + s_p][c] += dz[b][c] and db1[c] += dz[b][c] over the states.  A
// block of 64 threads owns 64 columns (one each) and a run of states; the
// per-row partial sums live in LDS (no two threads share a column), then every
// non-zero partial is added atomically.
template <int T, int SIDE>
__global__ __launch_bounds__(64) void scatter_l1_kernel(ScatterArgs a) {
    constexpr int P = SIDE * SIDE, S = SIDE * SIDE, ROWS = P * S;
    __shared__ float acc[ROWS][64];
    const int c = blockIdx.x * 64 + threadIdx.x;
    for (int r = 0; r < ROWS; r++) acc[r][threadIdx.x] = 0.f;
    float bsum = 0.f;
    const int b0 = blockIdx.y * a.states_per_block;
    const int b1 = min(b0 + a.states_per_block, a.n);
    for (int b = b0; b < b1; b++) {
        const uint64_t w = reinterpret_cast<const uint64_t*>(a.packed)[b];
        const float v = ld_t<T>(a.dz, (size_t)b * a.ld + c);
        if (v == 0.f) continue;
        bsum += v;
        for (int p = 0; p < P; p++) {
            const int s = min((int)((w >> (4 * p)) & 15), S - 1);
            acc[p * S + s][threadIdx.x] += v;
        }
    }
    for (int r = 0; r < ROWS; r++) {
        const float v = acc[r][threadIdx.x];
        if (v != 0.f) atomicAdd(&a.dW1[(size_t)r * a.ld_w + c], v);
    }
    if (bsum != 0.f) atomicAdd(&a.db1[c], bsum);
}

// ------------------------------------------------------------------ Adam
// master[k][n] (float32, K x N) updated from grad[k*gk + n*gn]; the working
// copies out1 (type T) at k*s1k + n*s1n and out2 at k*s2k + n*s2n are rewritten.
template <int T>
__global__ void adam_kernel(AdamArgs a) {
    const int64_t total = (int64_t)a.K * a.N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(i / a.N), n = (int)(i % a.N);
        const float g = a.grad[(size_t)k * a.gk + (size_t)n * a.gn];
        const float m = a.b1 * a.m[i] + (1.f - a.b1) * g;
        const float v = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
        a.m[i] = m;
        a.v[i] = v;
        const float w = a.master[i] - a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
        a.master[i] = w;
        if (a.out1) st_t<T>(a.out1, (size_t)k * a.s1k + (size_t)n * a.s1n, w);
        if (a.out2) st_t<T>(a.out2, (size_t)k * a.s2k + (size_t)n * a.s2n, w);
    }
}

// ------------------------------------------------------------ launchers
void launch_fill(float* p, int64_t n, float v, hipStream_t s) {
    int blocks = (int)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, s, p, n, v);
}

bool launch_head_train(const HeadTrainArgs& a, int t, hipStream_t s) {
    if (a.K % 4 || a.K > kHeadMaxGroups * 256) return false;
    const int blocks = (a.m_pad + 4 * kHeadRowsPerWave - 1) / (4 * kHeadRowsPerWave);
    if (t == 0) hipLaunchKernelGGL(head_train_kernel<0>, dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(head_train_kernel<1>, dim3(blocks), dim3(256), 0, s, a);
    return true;
}

void launch_transpose(const TransposeArgs& a, int t, hipStream_t s) {
    dim3 grid((a.C + 63) / 64, (a.R + 63) / 64);
    if (t == 0) hipLaunchKernelGGL(transpose_kernel<0>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(transpose_kernel<1>, grid, dim3(256), 0, s, a);
}

bool launch_scatter_l1(const ScatterArgs& a, int t, int side, hipStream_t s) {
    if (a.N1 % 64) return false;
    dim3 grid(a.N1 / 64, (a.n + a.states_per_block - 1) / a.states_per_block);
    if (grid.y == 0) return true;
    if (side == 3) {
        if (t == 0) hipLaunchKernelGGL((scatter_l1_kernel<0, 3>), grid, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((scatter_l1_kernel<1, 3>), grid, dim3(64), 0, s, a);
    } else if (side == 4) {
        if (t == 0) hipLaunchKernelGGL((scatter_l1_kernel<0, 4>), grid, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((scatter_l1_kernel<1, 4>), grid, dim3(64), 0, s, a);
    } else {
        return false;
    }
    return true;
}

void launch_adam(const AdamArgs& a, int t, hipStream_t s) {
    const int64_t total = (int64_t)a.K * a.N;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    if (t == 0) hipLaunchKernelGGL(adam_kernel<0>, dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(adam_kernel<1>, dim3(blocks), dim3(256), 0, s, a);
}

}  // namespace hb
