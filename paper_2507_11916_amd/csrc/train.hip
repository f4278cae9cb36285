// HIP kernels of on-GPU training of the heuristic network (regression head,
// sliding-tile or cube inputs): loss and output-layer gradient, transposes with fused
// bias-gradient column sums, the layer-1 scatter-add (transpose of the
// gather-sum), Adam with re-cast of the working weights, and a fill kernel.
// The matrix products (forward, input gradients, weight gradients) run on the
// MFMA GEMM of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
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
// Rows in turn, 2 rows per wave, 4 waves per block.  y = w.x + b;
// loss += w_b (y - t)^2 / n; dy = 2 w_b (y - t) / n; delta_k = dy * w_k where
// x_k > 0 (gradient at the pre-activation of the last hidden layer).  Rows >= n
// get delta = 0.  dWo, dbo and the loss are reduced over the block's rows in
// LDS; each block writes its partial sums, which column_sum_kernel adds in
// block order.  A wave loads all of its rows (4 consecutive values per lane
// and group, one vector access) before it reduces the first, so the rows'
// loads are in flight together; the per-row arithmetic and the row order of
// the accumulations are fixed.  Few rows per wave make many blocks: 8 rows per
// wave (a quarter of the blocks) took 1.5x as long, with the partial sums.
constexpr int kHeadRowsPerWave = 2;
constexpr int kHeadMaxGroups = 4;  // K <= 1024

// four consecutive elements (float32 or bfloat16) starting at element i
template <int T>
__device__ __forceinline__ void ld4_t(const void* p, size_t i, float (&v)[4]) {
    if (T == 0) {
        const float4 q = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(p) + i);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
        const uint2 q = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(p) + i);
        v[0] = __uint_as_float(q.x << 16); v[1] = __uint_as_float(q.x & 0xFFFF0000u);
        v[2] = __uint_as_float(q.y << 16); v[3] = __uint_as_float(q.y & 0xFFFF0000u);
    }
}
template <int T>
__device__ __forceinline__ void st4_t(void* p, size_t i, const float (&v)[4]) {
    if (T == 0) {
        *reinterpret_cast<float4*>(reinterpret_cast<float*>(p) + i) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        uint2 q;
        q.x = (uint32_t)tr_f32_to_bf16(v[0]) | ((uint32_t)tr_f32_to_bf16(v[1]) << 16);
        q.y = (uint32_t)tr_f32_to_bf16(v[2]) | ((uint32_t)tr_f32_to_bf16(v[3]) << 16);
        *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(p) + i) = q;
    }
}

template <int T>
__global__ __launch_bounds__(256) void head_train_kernel(HeadTrainArgs a) {
    constexpr int RW = kHeadRowsPerWave;
    __shared__ float s_w[4][kHeadMaxGroups * 256];
    __shared__ float s_b[4], s_l[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int groups = (a.K + 255) / 256;  // lanes own 4 columns per group; columns >= K are skipped
    // Loads are unconditional (clamped addresses) and out-of-range values are
    // zeroed afterwards, so no load waits behind a branch.  K % 4 == 0: a
    // lane's four columns are all in range or all out.
    float accw[kHeadMaxGroups][4], w[kHeadMaxGroups][4];
    _Pragma("unroll") for (int gi = 0; gi < kHeadMaxGroups; gi++) {
        const int k0 = gi * 256 + lane * 4;
        _Pragma("unroll") for (int e = 0; e < 4; e++) accw[gi][e] = 0.f;
        ld4_t<T>(a.W, min(k0, a.K - 4), w[gi]);
        if (k0 >= a.K) _Pragma("unroll") for (int e = 0; e < 4; e++) w[gi][e] = 0.f;
    }
    float accb = 0.f, accl = 0.f;
    const int row0 = (blockIdx.x * 4 + wave) * RW;
    float x[RW][kHeadMaxGroups][4];
    _Pragma("unroll") for (int rr = 0; rr < RW; rr++) {
        const int r = min(row0 + rr, a.m_pad - 1);
        _Pragma("unroll") for (int gi = 0; gi < kHeadMaxGroups; gi++)
            ld4_t<T>(a.X, (size_t)r * a.ldx + min(gi * 256 + lane * 4, a.K - 4), x[rr][gi]);
    }
    // the rows' labels and the output bias, loaded with the rows (a label read
    // after each row's reduction would put one memory latency per row in series)
    float lab[RW];
    _Pragma("unroll") for (int rr = 0; rr < RW; rr++) lab[rr] = a.labels[max(0, min(row0 + rr, a.n - 1))];
    const float bias_o = a.b[0];
    _Pragma("unroll") for (int rr = 0; rr < RW; rr++)
        _Pragma("unroll") for (int gi = 0; gi < kHeadMaxGroups; gi++)
            if (gi * 256 + lane * 4 >= a.K) _Pragma("unroll") for (int e = 0; e < 4; e++) x[rr][gi][e] = 0.f;
    // (every array index below is a compile-time constant, so x, w and accw stay
    // in registers; `groups` only masks whole unrolled iterations)
    _Pragma("unroll") for (int rr = 0; rr < RW; rr++) {
        const int r = row0 + rr;
        if (r >= a.m_pad) continue;  // uniform
        float part = 0.f;
        _Pragma("unroll") for (int gi = 0; gi < kHeadMaxGroups; gi++)
            if (gi < groups)
                _Pragma("unroll") for (int e = 0; e < 4; e++)
                    if (gi * 256 + lane * 4 + e < a.K) part += x[rr][gi][e] * w[gi][e];
        for (int s = 32; s >= 1; s >>= 1) part += __shfl_xor(part, s, 64);
        float dy = 0.f;
        if (r < a.n) {
            const float y = part + bias_o;
            const float d = y - lab[rr];
            const float wgt = (a.asym && d > 0.f) ? a.alpha : 1.f;
            dy = 2.f * wgt * d * a.inv_n;
            accl += wgt * d * d * a.inv_n;
            accb += dy;
            if (a.y_out && lane == 0) a.y_out[r] = y;
        }
        _Pragma("unroll") for (int gi = 0; gi < kHeadMaxGroups; gi++) {
            const int k0 = gi * 256 + lane * 4;
            if (gi >= groups || k0 >= a.K) continue;
            float dl[4];
            _Pragma("unroll") for (int e = 0; e < 4; e++) {
                dl[e] = x[rr][gi][e] > 0.f ? dy * w[gi][e] : 0.f;
                accw[gi][e] += x[rr][gi][e] * dy;
            }
            st4_t<T>(a.delta, (size_t)r * a.ldx + k0, dl);
        }
    }
    _Pragma("unroll") for (int gi = 0; gi < kHeadMaxGroups; gi++)
        _Pragma("unroll") for (int e = 0; e < 4; e++) s_w[wave][gi * 256 + lane * 4 + e] = accw[gi][e];
    if (lane == 0) { s_b[wave] = accb; s_l[wave] = accl; }
    __syncthreads();
    // the block's partial sums (output weights, bias, loss) into its row of
    // `part`; column_sum_kernel adds the rows in block order
    float* part = a.part + (size_t)blockIdx.x * (a.K + 2);
    for (int k = threadIdx.x; k < a.K; k += 256) part[k] = s_w[0][k] + s_w[1][k] + s_w[2][k] + s_w[3][k];
    if (threadIdx.x == 0) {
        part[a.K] = s_b[0] + s_b[1] + s_b[2] + s_b[3];
        part[a.K + 1] = s_l[0] + s_l[1] + s_l[2] + s_l[3];
    }
}

// out[c] = sum over r < rows of part[r * ld + c], in row order (the fixed-order
// second pass of every reduction over blocks: no float atomics, so results are
// bitwise repeatable).
// A block takes 64 columns; its 16 row groups each sum a contiguous quarter..
// sixteenth of the rows in order (loads issued 8 ahead), then the group sums
// are added in group order.
__global__ __launch_bounds__(1024) void column_sum_kernel(const float* part, int rows, int cols, int ld, float* out) {
    __shared__ float gs[16][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + tx;
    const int per = (rows + 15) / 16, r0 = ty * per, r1 = min(rows, r0 + per);
    float s = 0.f;
    if (c < cols) {
        int r = r0;
        for (; r + 8 <= r1; r += 8) {
            float v[8];
            _Pragma("unroll") for (int u = 0; u < 8; u++) v[u] = part[(size_t)(r + u) * ld + c];
            _Pragma("unroll") for (int u = 0; u < 8; u++) s += v[u];
        }
        for (; r < r1; r++) s += part[(size_t)r * ld + c];
    }
    gs[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && c < cols) {
        float t = 0.f;
        for (int g = 0; g < 16; g++) t += gs[g][tx];
        out[c] = t;
    }
}

// ------------------------------------------------------------- transpose
// out[c][r] = in[r][c] for r < R, c < C through a 64 x 64 LDS tile, four
// consecutive elements per thread and access (16 x 16 threads); with colpart,
// the block's column sums over rows < rows_sum go to row blockIdx.y of colpart
// (row stride C), for column_sum_kernel.  ld_in and ld_out are multiples of 4.
template <int T>
__global__ __launch_bounds__(256) void transpose_kernel(TransposeArgs a) {
    __shared__ float tile[64][65];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tq = threadIdx.x & 15, tr = threadIdx.x >> 4;
    for (int i = tr; i < 64; i += 16) {
        const int r = r0 + i, c = c0 + 4 * tq;
        float v[4];
        if (r < a.R && c + 3 < a.C) {
            ld4_t<T>(a.in, (size_t)r * a.ld_in + c, v);
        } else {
            _Pragma("unroll") for (int e = 0; e < 4; e++)
                v[e] = (r < a.R && c + e < a.C) ? ld_t<T>(a.in, (size_t)r * a.ld_in + c + e) : 0.f;
        }
        _Pragma("unroll") for (int e = 0; e < 4; e++) tile[i][4 * tq + e] = v[e];
    }
    __syncthreads();
    for (int i = tr; i < 64; i += 16) {
        const int c = c0 + i, r = r0 + 4 * tq;
        float v[4];
        _Pragma("unroll") for (int e = 0; e < 4; e++) v[e] = tile[4 * tq + e][i];
        if (c < a.C && r + 3 < a.R) {
            st4_t<T>(a.out, (size_t)c * a.ld_out + r, v);
        } else if (c < a.C) {
            _Pragma("unroll") for (int e = 0; e < 4; e++)
                if (r + e < a.R) st_t<T>(a.out, (size_t)c * a.ld_out + r + e, v[e]);
        }
    }
    if (a.colpart && threadIdx.x < 64) {
        const int tx = threadIdx.x;
        float s = 0.f;
        for (int i = 0; i < 64; i++)
            if (r0 + i < a.rows_sum) s += tile[i][tx];
        if (c0 + tx < a.C) a.colpart[(size_t)blockIdx.y * a.C + c0 + tx] = s;
    }
}

// ------------------------------------------------------------ layer 1
// dW1[row][c] = sum over states b whose one-hot input has `row` of dz[b][c]
// (the transpose of the gather-sum), db1[c] = sum_b dz[b][c].  Two passes:
// per-chunk partial sums (scatter_bucket_kernel), then the chunks' partials
// added in chunk order (scatter_sum_kernel).  No atomics: the gradient is
// bitwise repeatable.
template <int DOM>
struct TrCells {
    static constexpr int P = DOM == 0 ? 9 : DOM == 1 ? 16 : 48;  // gathered cells
    static constexpr int S = DOM == 0 ? 9 : DOM == 1 ? 16 : 6;
    static constexpr int W = DOM == 2 ? 3 : 1;                   // 64-bit words per packed state
    // symbol of cell p of a packed state given as its words (by value, so the
    // words stay in registers; the word is selected, p varies per wave)
    __device__ static int sym(uint64_t w0, uint64_t w1, uint64_t w2, int p) {
        if (DOM != 2) return min((int)((w0 >> (4 * p)) & 15), S - 1);
        const uint64_t word = (p >> 4) == 0 ? w0 : (p >> 4) == 1 ? w1 : w2;
        return min((int)((word >> (3 * (p & 15))) & 7), S - 1);
    }
};

int scatter_table_rows(int domain) { return domain == 0 ? 81 : domain == 1 ? 256 : 288; }

// Pass 1 (scatter_bucket_kernel): a block owns 128 columns of
// one chunk of states and takes the chunk SUB states at a time: their gradient
// rows (these 128 columns, as float32) and packed records are staged in LDS,
// after one all-zero row.  Wave w owns the cells p = w, w + NW, ...; per cell
// it sorts the staged states by the cell's symbol (a stable counting sort on
// wave ballots), each symbol's bucket padded with the zero row to a multiple
// of 8 entries, then walks each bucket in order, adding the staged rows into
// that symbol's two column sums, which stay in registers across the chunk
// (adding the zero row leaves a sum's bits unchanged).  Each row's partial is
// thus added in state order; wave 0 also sums every state's row, in order, for
// the bias.
template <int DOM>
struct TrBucket {
    static constexpr int P = TrCells<DOM>::P, S = TrCells<DOM>::S, W = TrCells<DOM>::W;
    static constexpr int NW = P < 16 ? P : 16;   // waves of a block
    static constexpr int CPW = P / NW;           // cells per wave
    static constexpr int SUB = DOM == 2 ? 128 : 256;  // states staged at a time
    static constexpr int LIST = SUB + 8 * S;     // a cell's list entries (u16)
    static constexpr int RB = 512;               // bytes of a staged row (128 float32)
    static_assert(P % NW == 0, "cells split evenly over the waves");
};

template <int DOM>
constexpr size_t scatter_bucket_lds_bytes() {
    using B = TrBucket<DOM>;
    return (size_t)(B::SUB + 1) * B::RB + (size_t)B::SUB * B::W * 8 + (size_t)B::P * B::LIST * 2;
}

template <int T, int DOM>
__global__ __launch_bounds__(64 * TrBucket<DOM>::NW) void scatter_bucket_kernel(ScatterArgs a) {
    using D = TrCells<DOM>;
    using B = TrBucket<DOM>;
    constexpr int ROWS = D::P * D::S, S = B::S, SUB = B::SUB, CPW = B::CPW, NW = B::NW, RB = B::RB;
    extern __shared__ __attribute__((aligned(16))) uint8_t sm[];
    uint8_t* rows = sm;                                                        // [SUB + 1][RB], row SUB all zero
    uint64_t* recs = reinterpret_cast<uint64_t*>(sm + (size_t)(SUB + 1) * RB);  // [SUB][W]
    uint16_t* lists = reinterpret_cast<uint16_t*>(sm + (size_t)(SUB + 1) * RB + (size_t)SUB * B::W * 8);  // [P][LIST]
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col0 = blockIdx.x * 128;
    const int b0 = blockIdx.y * a.chunk, b1 = min(b0 + a.chunk, a.n);
    if (threadIdx.x < RB / 4) reinterpret_cast<float*>(rows + (size_t)SUB * RB)[threadIdx.x] = 0.f;
    float acc[CPW][S][2];
    _Pragma("unroll") for (int j = 0; j < CPW; j++)
        _Pragma("unroll") for (int v = 0; v < S; v++) acc[j][v][0] = acc[j][v][1] = 0.f;
    float bs0 = 0.f, bs1 = 0.f;
    for (int sb = b0; sb < b1; sb += SUB) {
        const int ns = min(SUB, b1 - sb);
        // stage the rows as float32 (16-byte pieces of the source, every load in
        // flight before the first store; rows past the chunk repeat its last
        // row) and the records
        constexpr int EPP = T == 0 ? 4 : 8;               // elements per 16-byte source piece
        constexpr int PPR = 128 / EPP;                    // pieces per row
        constexpr int PT = (SUB * PPR + 64 * NW - 1) / (64 * NW);  // pieces per thread
        uint4 pc[PT];
        _Pragma("unroll") for (int k = 0; k < PT; k++) {
            const int i = min((int)threadIdx.x + k * 64 * NW, SUB * PPR - 1);
            const int r = min(i / PPR, ns - 1), q = i % PPR;
            pc[k] = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint8_t*>(a.dz) +
                                                    ((size_t)(sb + r) * a.ld + col0 + q * EPP) * (T == 0 ? 4 : 2));
        }
        for (int i = threadIdx.x; i < ns * D::W; i += 64 * NW)
            recs[i] = reinterpret_cast<const uint64_t*>(a.packed)[(size_t)sb * D::W + i];
        _Pragma("unroll") for (int k = 0; k < PT; k++) {
            const int i = (int)threadIdx.x + k * 64 * NW;
            if (i < SUB * PPR) {
                float* dst = reinterpret_cast<float*>(rows + (size_t)(i / PPR) * RB) + (i % PPR) * EPP;
                if (T == 0) {
                    *reinterpret_cast<uint4*>(dst) = pc[k];
                } else {
                    const uint32_t w[4] = {pc[k].x, pc[k].y, pc[k].z, pc[k].w};
                    float4 lo, hi;
                    lo.x = __uint_as_float(w[0] << 16); lo.y = __uint_as_float(w[0] & 0xffff0000u);
                    lo.z = __uint_as_float(w[1] << 16); lo.w = __uint_as_float(w[1] & 0xffff0000u);
                    hi.x = __uint_as_float(w[2] << 16); hi.y = __uint_as_float(w[2] & 0xffff0000u);
                    hi.z = __uint_as_float(w[3] << 16); hi.w = __uint_as_float(w[3] & 0xffff0000u);
                    reinterpret_cast<float4*>(dst)[0] = lo;
                    reinterpret_cast<float4*>(dst)[1] = hi;
                }
            }
        }
        __syncthreads();
        _Pragma("unroll") for (int j = 0; j < CPW; j++) {
            const int p = wave + NW * j;
            uint16_t* list = lists + (size_t)p * B::LIST;
            // counting sort of the staged states by cell p's symbol
            int cnt[S];
            _Pragma("unroll") for (int v = 0; v < S; v++) cnt[v] = 0;
            _Pragma("unroll") for (int q = 0; q < SUB / 64; q++) {
                const int b = q * 64 + lane;
                const uint64_t* rc = recs + (size_t)min(b, ns - 1) * D::W;
                const int sy = b < ns ? D::sym(rc[0], rc[D::W > 1 ? 1 : 0], rc[D::W > 2 ? 2 : 0], p) : S;
                _Pragma("unroll") for (int v = 0; v < S; v++) cnt[v] += __popcll(__ballot(sy == v));
            }
            int off[S + 1];
            off[0] = 0;
            _Pragma("unroll") for (int v = 0; v < S; v++) off[v + 1] = off[v] + ((cnt[v] + 7) & ~7);
            _Pragma("unroll") for (int v = 0; v < S; v++)  // the padding: the zero row
                if (lane < off[v + 1] - off[v] - cnt[v]) list[off[v] + cnt[v] + lane] = (uint16_t)SUB;
            int run[S];
            _Pragma("unroll") for (int v = 0; v < S; v++) run[v] = off[v];
            _Pragma("unroll") for (int q = 0; q < SUB / 64; q++) {
                const int b = q * 64 + lane;
                const uint64_t* rc = recs + (size_t)min(b, ns - 1) * D::W;
                const int sy = b < ns ? D::sym(rc[0], rc[D::W > 1 ? 1 : 0], rc[D::W > 2 ? 2 : 0], p) : S;
                int pos = 0;
                _Pragma("unroll") for (int v = 0; v < S; v++) {
                    const uint64_t m = __ballot(sy == v);
                    const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
                    pos = sy == v ? run[v] + below : pos;
                    run[v] += __popcll(m);
                }
                if (sy < S) list[pos] = (uint16_t)b;
            }
            // each bucket in order, eight staged rows in flight
            _Pragma("unroll") for (int v = 0; v < S; v++) {
                for (int k = off[v]; k < off[v + 1]; k += 8) {
                    float2 x[8];
                    _Pragma("unroll") for (int i = 0; i < 8; i++)
                        x[i] = *reinterpret_cast<const float2*>(rows + (size_t)list[k + i] * RB + lane * 8);
                    _Pragma("unroll") for (int i = 0; i < 8; i++) {
                        acc[j][v][0] += x[i].x;
                        acc[j][v][1] += x[i].y;
                    }
                }
            }
        }
        if (wave == 0) {  // the bias partial: every staged state, in order
            for (int b = 0; b < ns; b += 8) {
                float2 x[8];
                _Pragma("unroll") for (int i = 0; i < 8; i++)
                    x[i] = *reinterpret_cast<const float2*>(rows + (size_t)(b + i < ns ? b + i : SUB) * RB + lane * 8);
                _Pragma("unroll") for (int i = 0; i < 8; i++) {
                    bs0 += x[i].x;
                    bs1 += x[i].y;
                }
            }
        }
        __syncthreads();  // the next stage overwrites rows, records and lists
    }
    float* out = a.partial + (size_t)blockIdx.y * (ROWS + 1) * a.N1 + col0 + 2 * lane;
    _Pragma("unroll") for (int j = 0; j < CPW; j++)
        _Pragma("unroll") for (int v = 0; v < S; v++)
            *reinterpret_cast<float2*>(out + (size_t)((wave + NW * j) * S + v) * a.N1) = make_float2(acc[j][v][0], acc[j][v][1]);
    if (wave == 0) *reinterpret_cast<float2*>(out + (size_t)ROWS * a.N1) = make_float2(bs0, bs1);
}

// Table row -> gradient row (the weight file's order).  Cube: non-centre
// sticker q of the table is sticker q + q/8 + (q%8 >= 4) of the file.
template <int DOM>
__device__ __forceinline__ int grad_row(int r) {
    if (DOM != 2) return r;
    const int q = r / 6, col = r % 6;
    return (q + q / 8 + (q % 8 >= 4 ? 1 : 0)) * 6 + col;
}

// Pass 2: a thread takes four columns of one row and adds the chunks'
// partials in chunk order (eight loads in flight), then writes the gradient
// row (the bias row to db1).
template <int DOM>
__global__ __launch_bounds__(256) void scatter_sum_kernel(ScatterArgs a, int chunks) {
    using D = TrCells<DOM>;
    constexpr int ROWS = D::P * D::S;
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int c4 = a.N1 / 4;
    const int64_t total = (int64_t)(ROWS + 1) * c4;
    for (int64_t t = blockIdx.x * 256LL + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
        const int r = (int)(t / c4), c = (int)(t % c4) * 4;
        const float* p = a.partial + (size_t)r * a.N1 + c;
        const size_t stride = (size_t)(ROWS + 1) * a.N1;
        f4 acc = *reinterpret_cast<const f4*>(p);
        for (int k0 = 1; k0 < chunks; k0 += 8) {
            const int cnt = min(8, chunks - k0);
            f4 v[8];
            _Pragma("unroll") for (int u = 0; u < 8; u++)
                if (u < cnt) v[u] = *reinterpret_cast<const f4*>(p + (size_t)(k0 + u) * stride);
            _Pragma("unroll") for (int u = 0; u < 8; u++)
                if (u < cnt) acc += v[u];
        }
        if (r < ROWS) {
            *reinterpret_cast<f4*>(a.dW1 + (size_t)grad_row<DOM>(r) * a.ld_w + c) = acc;
        } else {
            *reinterpret_cast<f4*>(a.db1 + c) = acc;
            if (DOM == 2)  // centre f always shows colour f: its row's gradient is the bias gradient
                for (int f = 0; f < 6; f++)
                    for (int col = 0; col < 6; col++)
                        *reinterpret_cast<f4*>(a.dW1 + (size_t)((9 * f + 4) * 6 + col) * a.ld_w + c) = col == f ? acc : f4{0.f, 0.f, 0.f, 0.f};
        }
    }
}

// Cube: working table and folded bias from the master weights, in the order
// the inference model folds them (bias, then the centres of faces 0..5).
template <int T>
__global__ void cube_fold_kernel(const float* master, const float* bias, int N1, int N1_pad, void* table, float* bias_work) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N1_pad; j += gridDim.x * blockDim.x) {
        for (int r = 0; r < 288; r++) {
            const float w = j < N1 ? master[(size_t)grad_row<2>(r) * N1 + j] : 0.f;
            st_t<T>(table, (size_t)r * N1_pad + j, w);
        }
        float b = j < N1 ? bias[j] : 0.f;
        for (int f = 0; f < 6; f++) {
            const float w = j < N1 ? master[(size_t)((9 * f + 4) * 6 + f) * N1 + j] : 0.f;
            b += T == 0 ? w : tr_bf16_to_f32(tr_f32_to_bf16(w));
        }
        bias_work[j] = b;
    }
}

// ------------------------------------------------------------------ Adam
// master[k][n] (float32, K x N) updated from grad[k*gk + n*gn]; the working
// copies out1 (type T) at k*s1k + n*s1n and out2 at k*s2k + n*s2n are rewritten.
// One grid row per tensor, so every tensor's step is one launch.
// Blocks take 32 x 64 tiles (k, n) of one tensor: the master, moments and
// gradient are read and written along n, and a working copy that is stored
// transposed (element stride along n > 1, as the forward operand W^T) is
// written from an LDS tile along k, so every global access is coalesced.
// Small tiles and a grid of 512 blocks per tensor keep many blocks in flight
// (one 64 x 64 tile per block left the kernel 13% slower, two 45%).
template <int T>
__global__ __launch_bounds__(256) void multi_adam_kernel(const AdamTensor* ts, float lr, float b1, float b2, float eps,
                                                        float c1, float c2) {
    constexpr int TK = 32;  // tile rows (k); 64 columns (n)
    __shared__ float tile[TK][65];
    const AdamTensor d = ts[blockIdx.y];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int tk = (d.K + TK - 1) / TK, tn = (d.N + 63) / 64;
    constexpr int U = 4;  // k rows whose loads are issued together (clamped in range, results masked)
    for (int t = blockIdx.x; t < tk * tn; t += gridDim.x) {
        const int k0 = (t / tn) * TK, n0 = (t % tn) * 64;
        const int n = n0 + tx;
        for (int kb = ty; kb < TK; kb += 4 * U) {
            float g[U], m0[U], v0[U], w0[U];
            bool ok[U];
            size_t idx[U];
            _Pragma("unroll") for (int u = 0; u < U; u++) {
                const int k = k0 + kb + 4 * u;
                ok[u] = k < d.K && n < d.N;
                idx[u] = ok[u] ? (size_t)k * d.N + n : 0;
                g[u] = d.grad[ok[u] ? (size_t)k * d.gk + (size_t)n * d.gn : 0];
                m0[u] = d.m[idx[u]];
                v0[u] = d.v[idx[u]];
                w0[u] = d.master[idx[u]];
            }
            _Pragma("unroll") for (int u = 0; u < U; u++) {
                const int k = k0 + kb + 4 * u;
                float w = 0.f;
                if (ok[u]) {
                    const size_t i = idx[u];
                    const float m = b1 * m0[u] + (1.f - b1) * g[u];
                    const float v = b2 * v0[u] + (1.f - b2) * g[u] * g[u];
                    d.m[i] = m;
                    d.v[i] = v;
                    w = w0[u] - lr * (m / c1) / (sqrtf(v / c2) + eps);
                    d.master[i] = w;
                    if (d.out1 && d.s1n == 1) st_t<T>(d.out1, (size_t)k * d.s1k + n, w);
                    if (d.out2 && d.s2n == 1) st_t<T>(d.out2, (size_t)k * d.s2k + n, w);
                }
                tile[kb + 4 * u][tx] = w;
            }
        }
        const bool t1 = d.out1 && d.s1n != 1, t2 = d.out2 && d.s2n != 1;
        if (t1 || t2) {
            __syncthreads();
            // a wave writes 64 / TK columns per pass, TK consecutive k each
            const int kl = tx % TK, k = k0 + kl;
            for (int nn = ty * (64 / TK) + tx / TK; nn < 64; nn += 256 / TK) {
                const int n2 = n0 + nn;
                if (k < d.K && n2 < d.N) {
                    if (t1) st_t<T>(d.out1, (size_t)k * d.s1k + (size_t)n2 * d.s1n, tile[kl][nn]);
                    if (t2) st_t<T>(d.out2, (size_t)k * d.s2k + (size_t)n2 * d.s2n, tile[kl][nn]);
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ launchers
void launch_fill(float* p, int64_t n, float v, hipStream_t s) {
    int blocks = (int)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, s, p, n, v);
}

int head_train_blocks(int m_pad) { return (m_pad + 4 * kHeadRowsPerWave - 1) / (4 * kHeadRowsPerWave); }

bool launch_head_train(const HeadTrainArgs& a, int t, hipStream_t s) {
    if (a.K % 4 || a.K > kHeadMaxGroups * 256) return false;
    const int blocks = head_train_blocks(a.m_pad);
    if (t == 0) hipLaunchKernelGGL(head_train_kernel<0>, dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(head_train_kernel<1>, dim3(blocks), dim3(256), 0, s, a);
    // output-weight gradient, bias gradient and loss: the blocks' partials in order
    if (a.dbo_loss == a.dWo + a.K) {  // contiguous: one launch
        launch_column_sum(a.part, blocks, a.K + 2, a.K + 2, a.dWo, s);
    } else {
        launch_column_sum(a.part, blocks, a.K, a.K + 2, a.dWo, s);
        launch_column_sum(a.part + a.K, blocks, 2, a.K + 2, a.dbo_loss, s);
    }
    return true;
}

void launch_transpose(const TransposeArgs& a, int t, hipStream_t s) {
    dim3 grid((a.C + 63) / 64, (a.R + 63) / 64);
    if (t == 0) hipLaunchKernelGGL(transpose_kernel<0>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(transpose_kernel<1>, grid, dim3(256), 0, s, a);
    if (a.colpart) launch_column_sum(a.colpart, (a.rows_sum + 63) / 64, a.C, a.C, a.colsum, s);
}

// out[r] = sum over b < n of X[r * ld + b] (X float32 or bf16, ld a multiple
// of 8), for r < rows: the bias gradient from a transposed gradient.  A block
// of four waves takes one row, wave w the w-th quarter of the 16-byte pieces
// (pieces w, w + 4, ... per lane-position); a lane adds its pieces in order
// (eight loads in flight), the lanes' sums meet in a fixed butterfly and the
// four wave sums are added in wave order, so the result is bitwise repeatable.
template <int T>
__global__ __launch_bounds__(256) void row_sum_kernel(const void* X, int ld, int rows, int n, float* out) {
    __shared__ float ws[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = blockIdx.x;
    const size_t base = (size_t)r * ld;
    constexpr int E = T == 0 ? 4 : 8;  // elements per 16-byte load
    float acc = 0.f;
    for (int b0 = E * (wave * 64 + lane); b0 < n; b0 += 8 * 256 * E) {
        float x[8][E];
        _Pragma("unroll") for (int u = 0; u < 8; u++) {
            const int b = min(b0 + u * 256 * E, ld - E);  // in bounds; elements at or past n are masked
            const uint4 v = T == 0 ? *reinterpret_cast<const uint4*>(reinterpret_cast<const float*>(X) + base + b)
                                   : *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(X) + base + b);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            _Pragma("unroll") for (int i = 0; i < 4; i++) {
                if (T == 0) {
                    x[u][i] = __uint_as_float(w[i]);
                } else {
                    x[u][2 * i] = __uint_as_float(w[i] << 16);
                    x[u][2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
                }
            }
        }
        _Pragma("unroll") for (int u = 0; u < 8; u++)
            _Pragma("unroll") for (int i = 0; i < E; i++)
                acc += b0 + u * 256 * E + i < n ? x[u][i] : 0.f;
    }
    _Pragma("unroll") for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) ws[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[r] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

void launch_row_sum(const void* X, int ld, int rows, int n, float* out, int t, hipStream_t s) {
    const int blocks = rows;
    if (t == 0) hipLaunchKernelGGL(row_sum_kernel<0>, dim3(blocks), dim3(256), 0, s, X, ld, rows, n, out);
    else hipLaunchKernelGGL(row_sum_kernel<1>, dim3(blocks), dim3(256), 0, s, X, ld, rows, n, out);
}

// out[r][c] = sum over slices s < split of part[s * stride + r * ldp + c], added
// in slice order (the fixed-order second pass of a split-K weight gradient).
// cols, ldp and ldo are multiples of 4.
__global__ __launch_bounds__(256) void splitk_sum_kernel(const float* __restrict__ part, int split, int64_t stride,
                                                         int rows, int cols, int ldp, float* __restrict__ out, int ldo) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int c4 = cols / 4;
    const int64_t total = (int64_t)rows * c4;
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int r = (int)(i / c4), c = (int)(i % c4) * 4;
        const float* p = part + (size_t)r * ldp + c;
        f4 v[8];
        f4 acc = *reinterpret_cast<const f4*>(p);
        for (int s0 = 1; s0 < split; s0 += 8) {  // up to eight slices' loads in flight, added in order
            const int cnt = min(8, split - s0);
            _Pragma("unroll") for (int u = 0; u < 8; u++)
                if (u < cnt) v[u] = *reinterpret_cast<const f4*>(p + (size_t)(s0 + u) * stride);
            _Pragma("unroll") for (int u = 0; u < 8; u++)
                if (u < cnt) acc += v[u];
        }
        *reinterpret_cast<f4*>(out + (size_t)r * ldo + c) = acc;
    }
}

void launch_splitk_sum(const float* part, int split, int64_t stride, int rows, int cols, int ldp, float* out, int ldo,
                       hipStream_t s) {
    const int64_t work = (int64_t)rows * (cols / 4);
    const int blocks = (int)std::min<int64_t>(2048, (work + 255) / 256);
    hipLaunchKernelGGL(splitk_sum_kernel, dim3(blocks), dim3(256), 0, s, part, split, stride, rows, cols, ldp, out, ldo);
}

void launch_column_sum(const float* part, int rows, int cols, int ld, float* out, hipStream_t s) {
    const int blocks = (cols + 63) / 64;
    hipLaunchKernelGGL(column_sum_kernel, dim3(blocks), dim3(1024), 0, s, part, rows, cols, ld, out);
}

template <int T, int DOM>
static void launch_scatter_t(const ScatterArgs& a, int chunks, hipStream_t s) {
    hipLaunchKernelGGL((scatter_bucket_kernel<T, DOM>), dim3(a.N1 / 128, chunks), dim3(64 * TrBucket<DOM>::NW),
                       scatter_bucket_lds_bytes<DOM>(), s, a);
    const int blocks = (int)std::min<int64_t>(2048, ((int64_t)(scatter_table_rows(DOM) + 1) * (a.N1 / 4) + 255) / 256);
    hipLaunchKernelGGL((scatter_sum_kernel<DOM>), dim3(blocks), dim3(256), 0, s, a, chunks);
}

bool launch_scatter_l1(const ScatterArgs& a, int t, int domain, int chunks, hipStream_t s) {
    if (a.N1 % 128 || chunks < 1 || domain < 0 || domain > 2 || t < 0 || t > 1) return false;
    switch (domain * 2 + t) {
        case 0: launch_scatter_t<0, 0>(a, chunks, s); break;
        case 1: launch_scatter_t<1, 0>(a, chunks, s); break;
        case 2: launch_scatter_t<0, 1>(a, chunks, s); break;
        case 3: launch_scatter_t<1, 1>(a, chunks, s); break;
        case 4: launch_scatter_t<0, 2>(a, chunks, s); break;
        case 5: launch_scatter_t<1, 2>(a, chunks, s); break;
    }
    return true;
}

void launch_multi_adam(const AdamTensor* d_tensors, int count, float lr, float b1, float b2, float eps, float c1,
                       float c2, int t, hipStream_t s) {
    const dim3 grid(512, count);
    if (t == 0) hipLaunchKernelGGL(multi_adam_kernel<0>, grid, dim3(256), 0, s, d_tensors, lr, b1, b2, eps, c1, c2);
    else hipLaunchKernelGGL(multi_adam_kernel<1>, grid, dim3(256), 0, s, d_tensors, lr, b1, b2, eps, c1, c2);
}

template <int T, int DOM>
static hipError_t set_scatter_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&scatter_bucket_kernel<T, DOM>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)scatter_bucket_lds_bytes<DOM>());
}

// The layer-1 scatter holds up to 289 x 64 floats and 256 staged records of LDS per block.
hipError_t train_prepare_attributes() {
    hipError_t e = set_scatter_attr<0, 0>();
    if (e == hipSuccess) e = set_scatter_attr<1, 0>();
    if (e == hipSuccess) e = set_scatter_attr<0, 1>();
    if (e == hipSuccess) e = set_scatter_attr<1, 1>();
    if (e == hipSuccess) e = set_scatter_attr<0, 2>();
    if (e == hipSuccess) e = set_scatter_attr<1, 2>();
    return e;
}

void launch_cube_fold(const float* master, const float* bias, int N1, int N1_pad, void* table, float* bias_work, int t,
                      hipStream_t s) {
    const int blocks = (N1_pad + 255) / 256;
    if (t == 0) hipLaunchKernelGGL(cube_fold_kernel<0>, dim3(blocks), dim3(256), 0, s, master, bias, N1, N1_pad, table, bias_work);
    else hipLaunchKernelGGL(cube_fold_kernel<1>, dim3(blocks), dim3(256), 0, s, master, bias, N1, N1_pad, table, bias_work);
}


}  // namespace hb
