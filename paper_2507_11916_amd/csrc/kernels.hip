// HIP kernels of the heuristic network for gfx950 (CDNA4).
//
// Forward pass of h_M over a batch of packed states (ProcessBatch step 2 of
// SingleGPU Batch CB-DFS):
//   gather_l1   decode packed states, layer 1 as a gather-sum of weight rows
//               (the one-hot input is never materialised), bias, ReLU, cast;
//   gemm        dense / residual layers on MFMA with LDS-staged tiles and a
//               fused epilogue (column scale, bias, residual, ReLU, cast);
//   head        output layer and the output rule (floor / round / real,
//               Manhattan minimum; softmax-quantile / arg-max).
// Every kernel computes each row independently and in a fixed order, so a
// state's heuristic does not depend on the batch it is evaluated in.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>

#include "kernels.hpp"

namespace hb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef int intx8 __attribute__((ext_vector_type(8)));
// Native vector (not HIP's uint4 class type): arrays of it stay in registers.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ conversions
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    const uint32_t rounded = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    const uint32_t quiet = (u >> 16) | 0x40u;
    return (uint16_t)((u & 0x7FFFFFFFu) > 0x7F800000u ? quiet : rounded);
}

// OCP e4m3, round to nearest even, saturating at +-448.  The hardware
// conversion rounds to nearest even but maps overflow to NaN, so the value is
// clamped first.
__device__ __forceinline__ uint32_t f32x2_to_fp8x2(float a, float b) {
    a = fminf(fmaxf(a, -448.f), 448.f);
    b = fminf(fmaxf(b, -448.f), 448.f);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xFFFFu;
}

__device__ __forceinline__ float fp8_to_f32(uint32_t byte) {
    return __builtin_amdgcn_cvt_f32_fp8((int)byte, 0);
}

// ------------------------------------------------------------ coherent access
// Data handed between waves of one launch on different XCDs (the fused forward
// kernel) goes through device-coherent accesses: relaxed agent-scope atomic
// loads and stores, which this target issues with the sc1 cache policy (read
// from, and written through to, the level that all XCDs share) instead of
// through an XCD's own L2.  Ordering then needs only a wait for the stores and
// a compiler fence, not the agent-scope fences that write back or invalidate a
// whole L2.
template <typename T>
__device__ __forceinline__ T ld_coh(const T* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
template <typename T>
__device__ __forceinline__ void st_coh(T* p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// 16 bytes (two 8-byte accesses when coherent)
template <bool COH>
__device__ __forceinline__ u32x4 ld16(const uint8_t* p) {
    if (!COH) return *reinterpret_cast<const u32x4*>(p);
    const uint64_t* q = reinterpret_cast<const uint64_t*>(p);
    const uint64_t a = ld_coh(q), b = ld_coh(q + 1);
    return u32x4{(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
}
template <bool COH>
__device__ __forceinline__ void st16(uint8_t* p, u32x4 v) {
    if (!COH) { *reinterpret_cast<u32x4*>(p) = v; return; }
    uint64_t* q = reinterpret_cast<uint64_t*>(p);
    st_coh(q, (uint64_t)v.x | ((uint64_t)v.y << 32));
    st_coh(q + 1, (uint64_t)v.z | ((uint64_t)v.w << 32));
}

// ------------------------------------------------------------ decoding
// Symbol of cell/sticker row g of the folded layer-1 table.  Sliding tile:
// P cells, symbol = tile; row = p * S + tile.  Cube: 48 non-centre stickers,
// row = q * 6 + colour (the centres are folded into the bias).
template <int DOM>
struct Dec;
// Symbols are clamped to S - 1 so that a corrupt record cannot index past the
// table (hb_encode never produces one).
template <>
struct Dec<0> {  // 3x3
    static constexpr int P = 9, S = 9, WORDS = 1;
    __device__ static int row(const uint64_t* w, int p) { return p * S + min((int)((w[0] >> (4 * p)) & 15), S - 1); }
};
template <>
struct Dec<1> {  // 4x4
    static constexpr int P = 16, S = 16, WORDS = 1;
    __device__ static int row(const uint64_t* w, int p) { return p * S + (int)((w[0] >> (4 * p)) & 15); }
};
template <>
struct Dec<2> {  // cube
    static constexpr int P = 48, S = 6, WORDS = 3;
    __device__ static int row(const uint64_t* w, int q) {
        return q * S + min((int)((w[q >> 4] >> (3 * (q & 15))) & 7), S - 1);
    }
};

// s_waitcnt vmcnt(N) with the expcnt and lgkmcnt fields at their maxima (no
// wait on them); vmcnt is split over bits 3:0 and 15:14.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit field");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// ------------------------------------------------------------ layer 1
// Gather-sum over a column slice.  A block owns GCOLS columns of the table for
// GROWS consecutive states: it copies the table's column slice (all
// P * S rows, a few tens of KiB) and the states' packed records into LDS once,
// then each thread forms 4 columns of one state at a time by summing the
// state's P rows out of LDS.  The slice is copied with global_load_lds_dwordx4
// (16 bytes per lane straight into LDS at the instruction's base + 16 * lane):
// the slice is row-major with 16-byte pieces in order, so the 64 pieces of one
// instruction are 1 KiB of consecutive LDS, and every piece of the slice is in
// flight at once instead of one register round trip per piece.
// Reading the slice once per block instead of once per state cuts the
// gathered L2 traffic by about GROWS / S.  Sum order per output: bias, then
// the cells in order.  Rows in [n, m_rows) are written as zeros.
constexpr int GCOLS = 64, GROWS = 256;

template <int DOM, int WT /*0 f32, 1 bf16 table*/, int OUT /*0 f32, 1 bf16, 2 fp8*/>
__global__ __launch_bounds__(256) void gather_l1_kernel(const uint64_t* __restrict__ packed, const int32_t* n_dev,
                                                        int n_host, int m_rows, const void* __restrict__ table,
                                                        int t_rows, const float* __restrict__ bias, int N,
                                                        int ld_out, void* __restrict__ out, float out_inv_scale) {
    using D = Dec<DOM>;
    constexpr int TB = WT == 0 ? 4 : 2;             // table bytes per element
    constexpr int ROWB = GCOLS * TB;                // bytes of one table row's slice
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    __shared__ uint64_t recs[GROWS * D::WORDS];     // packed records of the block's states
    const int tid = threadIdx.x;
    const int c0 = blockIdx.x * GCOLS;
    const int r0 = blockIdx.y * GROWS;
    const int n = min(n_dev ? *n_dev : n_host, m_rows);

    // table slice -> LDS, 16-byte pieces; wave w issues pieces [64 j, 64 j + 64)
    // for j = w, w + 4, ...  (lanes past the last piece are masked off)
    const int pieces = t_rows * (ROWB / 16);
    const int lane = tid & 63;
    for (int i0 = (tid >> 6) * 64; i0 < pieces; i0 += 256) {
        const int i = i0 + lane;
        if (i < pieces) {
            const int r = i / (ROWB / 16), q = i % (ROWB / 16);
            const uint8_t* src = reinterpret_cast<const uint8_t*>(table) + ((size_t)r * N + c0) * TB + q * 16;
            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(smem + i0 * 16), 16, 0, 0);
        }
    }
    for (int i = tid; i < GROWS * D::WORDS; i += 256) {
        const int r = r0 + i / D::WORDS;
        recs[i] = r < n ? packed[(size_t)r0 * D::WORDS + i] : 0;
    }
    wait_vmcnt<0>();
    __syncthreads();

    // 16 lanes per state, 4 columns per lane: a 16-lane group reads one
    // table row's slice contiguously (a full bank line for float32 entries).
    const int chunk = tid & 15;
    const int col = c0 + 4 * chunk;
    float b[4];
    _Pragma("unroll") for (int j = 0; j < 4; j++) b[j] = bias[col + j];
    // Two states per pass (rr and rr + 16), rows in chunks of CH: the 2 * CH
    // LDS reads of a chunk are issued before it is summed (per state in cell
    // order), so one LDS latency is paid per chunk.  States past n have zero
    // records (valid row indices) and are written as zeros.
    constexpr int CH = D::P < 16 ? D::P : 16;
    static_assert(D::P % CH == 0, "cells per chunk");
    for (int rr = tid >> 4; rr < GROWS; rr += 32) {
        if (r0 + rr >= m_rows) break;
        uint64_t w[2][D::WORDS];
        float acc[2][4];
        _Pragma("unroll") for (int u = 0; u < 2; u++) {
            _Pragma("unroll") for (int i = 0; i < D::WORDS; i++) w[u][i] = recs[(rr + 16 * u) * D::WORDS + i];
            _Pragma("unroll") for (int j = 0; j < 4; j++) acc[u][j] = b[j];
        }
        _Pragma("unroll") for (int p0 = 0; p0 < D::P; p0 += CH) {
            if (WT == 0) {
                float4 v[2][CH];
                _Pragma("unroll") for (int u = 0; u < 2; u++)
                    _Pragma("unroll") for (int k = 0; k < CH; k++)
                        v[u][k] = *reinterpret_cast<const float4*>(smem + D::row(w[u], p0 + k) * ROWB + chunk * 16);
                __builtin_amdgcn_sched_group_barrier(0x100, 2 * CH, 0);
                _Pragma("unroll") for (int u = 0; u < 2; u++)
                    _Pragma("unroll") for (int k = 0; k < CH; k++) {
                        acc[u][0] += v[u][k].x; acc[u][1] += v[u][k].y;
                        acc[u][2] += v[u][k].z; acc[u][3] += v[u][k].w;
                    }
            } else {
                uint2 v[2][CH];
                _Pragma("unroll") for (int u = 0; u < 2; u++)
                    _Pragma("unroll") for (int k = 0; k < CH; k++)
                        v[u][k] = *reinterpret_cast<const uint2*>(smem + D::row(w[u], p0 + k) * ROWB + chunk * 8);
                __builtin_amdgcn_sched_group_barrier(0x100, 2 * CH, 0);
                _Pragma("unroll") for (int u = 0; u < 2; u++)
                    _Pragma("unroll") for (int k = 0; k < CH; k++) {
                        acc[u][0] += bf16_to_f32((uint16_t)(v[u][k].x & 0xFFFF));
                        acc[u][1] += bf16_to_f32((uint16_t)(v[u][k].x >> 16));
                        acc[u][2] += bf16_to_f32((uint16_t)(v[u][k].y & 0xFFFF));
                        acc[u][3] += bf16_to_f32((uint16_t)(v[u][k].y >> 16));
                    }
            }
        }
        _Pragma("unroll") for (int u = 0; u < 2; u++) {
            const int r = r0 + rr + 16 * u;
            if (r >= m_rows) break;
            float a[4];
            _Pragma("unroll") for (int j = 0; j < 4; j++) a[j] = r < n ? fmaxf(acc[u][j], 0.f) : 0.f;
            const size_t o = (size_t)r * ld_out + col;
            if (OUT == 0) {
                *reinterpret_cast<float4*>((float*)out + o) = make_float4(a[0], a[1], a[2], a[3]);
            } else if (OUT == 1) {
                uint2 v;
                v.x = (uint32_t)f32_to_bf16(a[0]) | ((uint32_t)f32_to_bf16(a[1]) << 16);
                v.y = (uint32_t)f32_to_bf16(a[2]) | ((uint32_t)f32_to_bf16(a[3]) << 16);
                *reinterpret_cast<uint2*>((uint16_t*)out + o) = v;
            } else {
                *reinterpret_cast<uint32_t*>((uint8_t*)out + o) =
                    f32x2_to_fp8x2(a[0] * out_inv_scale, a[1] * out_inv_scale) |
                    (f32x2_to_fp8x2(a[2] * out_inv_scale, a[3] * out_inv_scale) << 16);
            }
        }
    }
}

// ------------------------------------------------------------ GEMM
// C[M][N] = epi(A[M][K] * B[K][N]) with A row-major (activations) and B given
// transposed, Bt[N][K] (weights, K contiguous).  Block tile BM x BN, 4 waves in
// a 2 x 2 grid, each wave (BM/2) x (BN/2) built from 32x32 MFMA tiles.  Each
// K stage moves 128 bytes of every A and Bt row through LDS (double-buffered);
// 16-byte chunks are XOR-swizzled with key (row / 2) mod 8: one 16-lane group of
// a 128-bit LDS access spans 16 consecutive rows, two rows per 256-byte line of
// banks, and the key gives the 8 rows of each parity 8 distinct chunk slots, so
// both the global->LDS stores and the MFMA operand reads are conflict-free.
// (Keyed on row mod 8, a third of the LDS cycles went to bank conflicts.)
//   PREC 0: fp32, v_mfma_f32_32x32x2_f32 (a lane reads 4 K values, one per MFMA);
//   PREC 1: bf16, v_mfma_f32_32x32x16_bf16 (8 K values per lane);
//   PREC 2: fp8,  v_mfma_scale_f32_32x32x64_f8f6f4 with unit block scales
//           (32 K values per lane; column/tensor scales in the epilogue).
// A and Bt use the same per-lane K assignment, so every K index is paired
// once with itself.
struct GemmArgs {
    const uint8_t* A;
    const uint8_t* Bt;
    uint8_t* C;
    const uint8_t* R;        // residual (same type and layout as C) or null
    const float* bias;       // [N]
    const float* colscale;   // [N] fp8 weight scales or null
    const int32_t* m_dev;    // device row count or null
    int m_host;              // row count when m_dev is null
    int m_tiles_cap;         // tiles available in M (grid shape)
    int N, K;                // N and K elements (padded)
    int lda, ldb, ldc;       // elements
    float a_scale;           // fp8: scale of A
    float r_scale;           // fp8: scale of R
    float out_inv_scale;     // fp8: 1 / scale of C
    int relu;
    int persistent;          // loop over tiles with a grid stride
    const uint8_t* Mk;       // mask (C's type and layout) or null: zero where Mk <= 0
    int group_n, group_k;    // grouped product: C columns of group g read A columns from g * group_k
    // split-K (wide tiles only): slice s of `split` multiplies K elements
    // [s K / split, (s + 1) K / split) into C + s * c_split elements
    int split = 1;
    int64_t c_split = 0;
    // dynamic tile schedule (a persistent grid): tiles after a block's first
    // come off tile_ctr[0]; tile_ctr[1] counts the blocks that have left
    int* tile_ctr = nullptr;
    // optional transposed copy of C (wide tile only): element (m, n) also at
    // Ct[n * ldct + m]; every row a tile writes is below ldct
    uint8_t* Ct = nullptr;
    int ldct = 0;
    int ct_rows = 0;  // rows of Ct written (columns of C below it); 0: all
};

// Dynamic tile schedule.  A block's first tile is its own (the XCD-aware order
// below), later ones come off an atomic counter: tile_fetch is issued by thread
// 0 when a tile starts, so its latency hides behind that tile.  Nothing ever
// waits on another block: the last block to leave resets the counter pair, so
// the next launch on the stream finds both at zero.
__device__ __forceinline__ int tile_fetch(const GemmArgs& g, int grid) {
    return __hip_atomic_fetch_add(g.tile_ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + grid;
}
__device__ __forceinline__ void tile_sched_exit(const GemmArgs& g) {
    if (__hip_atomic_fetch_add(g.tile_ctr + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == (int)gridDim.x - 1) {
        __hip_atomic_store(g.tile_ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(g.tile_ctr + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Column offset in A of the group that output column n0 belongs to.
__device__ __forceinline__ size_t group_a_col(const GemmArgs& g, int n0) {
    return g.group_n ? (size_t)(n0 / g.group_n) * g.group_k : 0;
}

template <int PREC>
struct Ty {
    static constexpr int EB = PREC == 0 ? 4 : PREC == 1 ? 2 : 1;  // bytes per element
};

__device__ __forceinline__ int swz(int row, int chunk) { return row * 128 + ((chunk ^ ((row >> 1) & 7)) << 4); }

// OUTT is the type of C, R and Mk (0 f32, 1 bf16, 2 fp8): equal to PREC for the
// forward and input-gradient products, float32 for weight gradients.
template <int OUTT>
__device__ __forceinline__ float load_out_t(const uint8_t* p, int o, float fp8_scale) {
    if (OUTT == 0) return reinterpret_cast<const float*>(p)[o];
    if (OUTT == 1) return bf16_to_f32(reinterpret_cast<const uint16_t*>(p)[o]);
    return fp8_to_f32(p[o]) * fp8_scale;
}

// Fused epilogue of one 32x32 MFMA tile held by a wave (lane: column n, rows
// 8a + 4*(lane/32) + b for element 4a + b), shared by every GEMM kernel so that
// they round identically: column scale and bias, residual, ReLU, mask, cast.
// o0: element offset of the lane's first element in C, R and Mk; element 4a + b
// sits (8a + b) rows further.  Offsets are formed as unsigned 32-bit byte
// offsets from the (uniform) base pointers, which the compiler turns into
// scalar-base + 32-bit-offset accesses (the buffers are below 4 GiB).  The
// residual and mask values are all loaded before any store: R may be C itself
// (in-place residual), and reading first lets the 16 loads overlap instead of
// each waiting behind the previous store.
template <int OUTT, bool COH = false>
__device__ __forceinline__ float load_at(const uint8_t* p, uint32_t byte_off, float fp8_scale) {
    if (COH) {
        if (OUTT == 0) return __uint_as_float(ld_coh(reinterpret_cast<const uint32_t*>(p + byte_off)));
        if (OUTT == 1) return bf16_to_f32(ld_coh(reinterpret_cast<const uint16_t*>(p + byte_off)));
        return fp8_to_f32(ld_coh(p + byte_off)) * fp8_scale;
    }
    if (OUTT == 0) return *reinterpret_cast<const float*>(p + byte_off);
    if (OUTT == 1) return bf16_to_f32(*reinterpret_cast<const uint16_t*>(p + byte_off));
    return fp8_to_f32(p[byte_off]) * fp8_scale;
}

// epi_tile_v returns the values it stored (the wide tile's transposed copy).
template <int OUTT, bool COH = false>
__device__ __forceinline__ floatx16 epi_tile_v(const GemmArgs& g, const floatx16& acc, float sn, float bn, int o0) {
    constexpr uint32_t EO = OUTT == 0 ? 4 : OUTT == 1 ? 2 : 1;
    const uint32_t b0 = (uint32_t)o0 * EO, row = (uint32_t)g.ldc * EO;
    float rv[16], mk[16];
    if (g.R) {
        _Pragma("unroll") for (int e = 0; e < 16; e++)
            rv[e] = load_at<OUTT, COH>(g.R, b0 + (8 * (e >> 2) + (e & 3)) * row, g.r_scale);
    }
    if (g.Mk) {
        _Pragma("unroll") for (int e = 0; e < 16; e++)
            mk[e] = load_at<OUTT>(g.Mk, b0 + (8 * (e >> 2) + (e & 3)) * row, 1.f);
    }
    floatx16 vt;
    _Pragma("unroll") for (int e = 0; e < 16; e++) {
        const uint32_t o = b0 + (8 * (e >> 2) + (e & 3)) * row;
        float v = acc[e] * sn + bn;
        if (g.R) v += rv[e];
        if (g.relu) v = fmaxf(v, 0.f);
        if (g.Mk) v = mk[e] > 0.f ? v : 0.f;
        vt[e] = v;
        if (COH) {
            if (OUTT == 0) st_coh(reinterpret_cast<uint32_t*>(g.C + o), __float_as_uint(v));
            else if (OUTT == 1) st_coh(reinterpret_cast<uint16_t*>(g.C + o), f32_to_bf16(v));
            else st_coh(g.C + o, (uint8_t)(f32x2_to_fp8x2(v * g.out_inv_scale, 0.f) & 0xFF));
        } else if (OUTT == 0) {
            *reinterpret_cast<float*>(g.C + o) = v;
        } else if (OUTT == 1) {
            *reinterpret_cast<uint16_t*>(g.C + o) = f32_to_bf16(v);
        } else {
            g.C[o] = (uint8_t)(f32x2_to_fp8x2(v * g.out_inv_scale, 0.f) & 0xFF);
        }
    }
    asm volatile("" ::: "memory");  // one tile's loads at a time: bounded register use
    return vt;
}

template <int OUTT, bool COH = false>
__device__ __forceinline__ void epi_tile(const GemmArgs& g, const floatx16& acc, float sn, float bn, int o0) {
    (void)epi_tile_v<OUTT, COH>(g, acc, sn, bn, o0);
}

// MFMAs of one 128-byte K stage held in LDS (a_s: BM rows, b_s: BN rows, both
// swizzled) into the wave's (BM/2) x (BN/2) accumulator tiles.
template <int PREC, int BM, int BN>
__device__ __forceinline__ void mma_stage(const uint8_t* a_s, const uint8_t* b_s, floatx16 (&acc)[BM / 64][BN / 64],
                                          int wm, int wn, int lane) {
    constexpr int TI = BM / 64, TJ = BN / 64;
    const int half = lane >> 5, r32 = lane & 31;
    if (PREC == 2) {
        _Pragma("unroll") for (int kg = 0; kg < 2; kg++) {
            intx8 af[TI], bfr[TJ];
            _Pragma("unroll") for (int i = 0; i < TI; i++) {
                const int row = wm * (BM / 2) + i * 32 + r32;
                const u32x4 lo = *reinterpret_cast<const u32x4*>(a_s + swz(row, 4 * kg + 2 * half));
                const u32x4 hi = *reinterpret_cast<const u32x4*>(a_s + swz(row, 4 * kg + 2 * half + 1));
                af[i] = intx8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
            }
            _Pragma("unroll") for (int j = 0; j < TJ; j++) {
                const int row = wn * (BN / 2) + j * 32 + r32;
                const u32x4 lo = *reinterpret_cast<const u32x4*>(b_s + swz(row, 4 * kg + 2 * half));
                const u32x4 hi = *reinterpret_cast<const u32x4*>(b_s + swz(row, 4 * kg + 2 * half + 1));
                bfr[j] = intx8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
            }
            _Pragma("unroll") for (int i = 0; i < TI; i++)
                _Pragma("unroll") for (int j = 0; j < TJ; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af[i], bfr[j], acc[i][j], 0, 0, 0,
                                                                               127, 0, 127);
        }
    } else {
        _Pragma("unroll") for (int kg = 0; kg < 4; kg++) {
            u32x4 af[TI], bfr[TJ];
            _Pragma("unroll") for (int i = 0; i < TI; i++) {
                const int row = wm * (BM / 2) + i * 32 + r32;
                af[i] = *reinterpret_cast<const u32x4*>(a_s + swz(row, 2 * kg + half));
            }
            _Pragma("unroll") for (int j = 0; j < TJ; j++) {
                const int row = wn * (BN / 2) + j * 32 + r32;
                bfr[j] = *reinterpret_cast<const u32x4*>(b_s + swz(row, 2 * kg + half));
            }
            if (PREC == 1) {
                _Pragma("unroll") for (int i = 0; i < TI; i++)
                    _Pragma("unroll") for (int j = 0; j < TJ; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, af[i]), __builtin_bit_cast(bf16x8, bfr[j]), acc[i][j], 0, 0, 0);
            } else {
                _Pragma("unroll") for (int e = 0; e < 4; e++)
                    _Pragma("unroll") for (int i = 0; i < TI; i++)
                        _Pragma("unroll") for (int j = 0; j < TJ; j++) {
                            const uint32_t ai = e == 0 ? af[i].x : e == 1 ? af[i].y : e == 2 ? af[i].z : af[i].w;
                            const uint32_t bj = e == 0 ? bfr[j].x : e == 1 ? bfr[j].y : e == 2 ? bfr[j].z : bfr[j].w;
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(ai), __uint_as_float(bj),
                                                                             acc[i][j], 0, 0, 0);
                        }
            }
        }
    }
}

// Stage k + 1 is fetched into registers while stage k is multiplied out of
// LDS.  (A second register set fetching stage k + 2 measured slower: the extra
// registers halve the waves per SIMD, which hide latency better.)
template <int PREC, int OUTT, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    constexpr int EB = Ty<PREC>::EB;
    constexpr int TI = BM / 64, TJ = BN / 64;  // MFMA tiles per wave
    constexpr int A_BYTES = BM * 128, B_BYTES = BN * 128;
    constexpr int A_LD = BM * 8 / 256, B_LD = BN * 8 / 256;  // 16-byte chunks per thread per stage
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    constexpr int STAGE = A_BYTES + B_BYTES;
#define SA(buf) (smem + (buf) * STAGE)
#define SB(buf) (smem + (buf) * STAGE + A_BYTES)

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int M = g.m_dev ? *g.m_dev : g.m_host;
    const int m_tiles = min((M + BM - 1) / BM, g.m_tiles_cap);  // never past the launch's row capacity
    const int n_tiles = g.N / BN;
    const int total = m_tiles * n_tiles;
    const int kb = g.K * EB;  // bytes of K
    const int ktiles = kb / 128;

    // Tile order: consecutive blocks of one XCD (blocks are dealt to the 8
    // XCDs round-robin) take consecutive tiles, so the N tiles of one M row
    // block share that XCD's L2.
    const int grid = gridDim.x;
    const int grid8 = grid & ~7;
    int first = blockIdx.x;
    if (blockIdx.x < grid8) first = (blockIdx.x & 7) * (grid8 >> 3) + (blockIdx.x >> 3);

    const bool dyn = g.tile_ctr != nullptr;
    __shared__ int s_next;
    const int t_end = g.persistent ? total : (first < total ? first + 1 : 0);
    for (int t = first; dyn ? t < total : t < t_end;) {
        int nxt = 0;
        if (dyn && tid == 0) nxt = tile_fetch(g, grid);
        const int tm = t / n_tiles, tn = t % n_tiles;
        const int m0 = tm * BM, n0 = tn * BN;
        const uint8_t* Ag = g.A + ((size_t)m0 * g.lda + group_a_col(g, n0)) * EB;
        const uint8_t* Bg = g.Bt + (size_t)n0 * g.ldb * EB;

        floatx16 acc[TI][TJ];
        _Pragma("unroll") for (int i = 0; i < TI; i++)
            _Pragma("unroll") for (int j = 0; j < TJ; j++)
                _Pragma("unroll") for (int e = 0; e < 16; e++) acc[i][j][e] = 0.f;

        // Global -> registers and registers -> LDS for one K stage (macros, so
        // that the register sets stay in registers).
#define HB_GLOAD(kt_, RA, RB)                                                                           \
        {                                                                                               \
            const int kbyte = (kt_) * 128;                                                              \
            _Pragma("unroll") for (int i = 0; i < A_LD; i++) {                                          \
                const int id = i * 256 + tid, row = id >> 3, ch = id & 7;                               \
                RA[i] = *reinterpret_cast<const u32x4*>(Ag + (size_t)row * g.lda * EB + kbyte + ch * 16); \
            }                                                                                           \
            _Pragma("unroll") for (int i = 0; i < B_LD; i++) {                                          \
                const int id = i * 256 + tid, row = id >> 3, ch = id & 7;                               \
                RB[i] = *reinterpret_cast<const u32x4*>(Bg + (size_t)row * g.ldb * EB + kbyte + ch * 16); \
            }                                                                                           \
        }
#define HB_SSTORE(buf_, RA, RB)                                                                         \
        {                                                                                               \
            _Pragma("unroll") for (int i = 0; i < A_LD; i++) {                                          \
                const int id = i * 256 + tid, row = id >> 3, ch = id & 7;                               \
                *reinterpret_cast<u32x4*>(SA(buf_) + swz(row, ch)) = RA[i];                            \
            }                                                                                           \
            _Pragma("unroll") for (int i = 0; i < B_LD; i++) {                                          \
                const int id = i * 256 + tid, row = id >> 3, ch = id & 7;                               \
                *reinterpret_cast<u32x4*>(SB(buf_) + swz(row, ch)) = RB[i];                            \
            }                                                                                           \
        }

        u32x4 ra[A_LD], rb[B_LD];
        HB_GLOAD(0, ra, rb);
        __syncthreads();  // previous tile's readers of buffer 0 are done
        HB_SSTORE(0, ra, rb);
        __syncthreads();
        for (int kt = 0; kt < ktiles; kt++) {
            const int cur = kt & 1;
            if (kt + 1 < ktiles) HB_GLOAD(kt + 1, ra, rb);
            mma_stage<PREC, BM, BN>(SA(cur), SB(cur), acc, wm, wn, lane);
            if (kt + 1 < ktiles) HB_SSTORE(cur ^ 1, ra, rb);
            __syncthreads();
        }
#undef HB_GLOAD
#undef HB_SSTORE

        // Epilogue.  Lane holds, for MFMA tile (i, j), column j*32 + lane%32 and
        // rows i*32 + 8a + 4*(lane/32) + b for a, b in 0..3 (value 4a + b).
        const int half = lane >> 5, c32 = lane & 31;
        _Pragma("unroll") for (int j = 0; j < TJ; j++) {
            const int n = n0 + wn * (BN / 2) + j * 32 + c32;
            const float bn = g.bias ? g.bias[n] : 0.f;
            const float sn = PREC == 2 ? g.colscale[n] * g.a_scale : 1.f;
            _Pragma("unroll") for (int i = 0; i < TI; i++)
                epi_tile<OUTT>(g, acc[i][j], sn, bn, (m0 + wm * (BM / 2) + i * 32 + 4 * half) * g.ldc + n);
        }
        if (dyn) {
            __syncthreads();
            if (tid == 0) s_next = nxt;
            __syncthreads();
            t = s_next;
        } else {
            t += grid;
        }
    }
    if (dyn) {
        __syncthreads();
        if (tid == 0) tile_sched_exit(g);
    }
}

#undef SA
#undef SB

// ------------------------------------------------------------ GEMM, 8 waves
// 256 x 128 tile with 8 waves in a 4 x 2 grid, each wave 64 x 64: one block per
// CU holds as many waves as two 128 x 128 blocks but moves a quarter fewer
// operand bytes per MFMA through L2 and LDS.  Each pair of wave rows runs the
// same per-stage MFMA routine on its 128-row half of the A tile (the swizzle
// key of a row is unchanged by the 128-row offset), so results are bitwise
// equal to the other tiles.  LDS double buffer filled through registers.
template <int PREC, int OUTT>
__global__ __launch_bounds__(512) void gemm_w8_kernel(GemmArgs g) {
    constexpr int BM = 256, BN = 128;
    constexpr int EB = Ty<PREC>::EB;
    constexpr int A_BYTES = BM * 128, B_BYTES = BN * 128;
    constexpr int A_LD = BM * 8 / 512, B_LD = BN * 8 / 512;
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    constexpr int STAGE = A_BYTES + B_BYTES;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 3, wn = wave >> 2;
    const int M = g.m_dev ? *g.m_dev : g.m_host;
    const int m_tiles = min((M + BM - 1) / BM, g.m_tiles_cap);
    const int n_tiles = g.N / BN;
    const int total = m_tiles * n_tiles;
    const int kb = g.K * EB;
    const int ktiles = kb / 128;
    const int grid = gridDim.x;
    const int grid8 = grid & ~7;
    int first = blockIdx.x;
    if (blockIdx.x < grid8) first = (blockIdx.x & 7) * (grid8 >> 3) + (blockIdx.x >> 3);
    for (int t = first; t < (g.persistent ? total : (first < total ? first + 1 : 0)); t += grid) {
        const int tm = t / n_tiles, tn = t % n_tiles;
        const int m0 = tm * BM, n0 = tn * BN;
        const uint8_t* Ag = g.A + ((size_t)m0 * g.lda + group_a_col(g, n0)) * EB;
        const uint8_t* Bg = g.Bt + (size_t)n0 * g.ldb * EB;
        floatx16 acc[2][2];
        _Pragma("unroll") for (int i = 0; i < 2; i++)
            _Pragma("unroll") for (int j = 0; j < 2; j++)
                _Pragma("unroll") for (int e = 0; e < 16; e++) acc[i][j][e] = 0.f;
        u32x4 ra[A_LD], rb[B_LD];
        auto gload = [&](int kt_) {
            const int kbyte = kt_ * 128;
            _Pragma("unroll") for (int i = 0; i < A_LD; i++) {
                const int id = i * 512 + tid, row = id >> 3, ch = id & 7;
                ra[i] = *reinterpret_cast<const u32x4*>(Ag + (size_t)row * g.lda * EB + kbyte + ch * 16);
            }
            _Pragma("unroll") for (int i = 0; i < B_LD; i++) {
                const int id = i * 512 + tid, row = id >> 3, ch = id & 7;
                rb[i] = *reinterpret_cast<const u32x4*>(Bg + (size_t)row * g.ldb * EB + kbyte + ch * 16);
            }
        };
        auto sstore = [&](int buf) {
            uint8_t* sa = smem + buf * STAGE;
            uint8_t* sb = sa + A_BYTES;
            _Pragma("unroll") for (int i = 0; i < A_LD; i++) {
                const int id = i * 512 + tid, row = id >> 3, ch = id & 7;
                *reinterpret_cast<u32x4*>(sa + swz(row, ch)) = ra[i];
            }
            _Pragma("unroll") for (int i = 0; i < B_LD; i++) {
                const int id = i * 512 + tid, row = id >> 3, ch = id & 7;
                *reinterpret_cast<u32x4*>(sb + swz(row, ch)) = rb[i];
            }
        };
        gload(0);
        __syncthreads();
        sstore(0);
        __syncthreads();
        for (int kt = 0; kt < ktiles; kt++) {
            const int cur = kt & 1;
            if (kt + 1 < ktiles) gload(kt + 1);
            const uint8_t* sa = smem + cur * STAGE;
            mma_stage<PREC, 128, 128>(sa + (wm >> 1) * 128 * 128, sa + A_BYTES, acc, wm & 1, wn, lane);
            if (kt + 1 < ktiles) sstore(cur ^ 1);
            __syncthreads();
        }
        const int half = lane >> 5, c32 = lane & 31;
        _Pragma("unroll") for (int j = 0; j < 2; j++) {
            const int n = n0 + wn * 64 + j * 32 + c32;
            const float bn = g.bias ? g.bias[n] : 0.f;
            const float sn = PREC == 2 ? g.colscale[n] * g.a_scale : 1.f;
            _Pragma("unroll") for (int i = 0; i < 2; i++)
                epi_tile<OUTT>(g, acc[i][j], sn, bn, (m0 + wm * 64 + i * 32 + 4 * half) * g.ldc + n);
        }
    }
}


// ------------------------------------------------------------ GEMM, LDS ring
// Same tiles, MFMA sequence and epilogue as gemm_kernel (bitwise equal
// results), but the operands go from global memory straight into LDS
// (global_load_lds_dwordx4: each lane's 16 bytes land at the instruction's LDS
// base + 16 * lane, no registers involved) through a ring of NS stages, so
// NS - 1 stages are in flight while one is multiplied.  The swizzle is applied
// on the global side: the lane that fills LDS slot s of row r fetches chunk
// s ^ key(r).  Waiting: each wave issues LD load instructions per stage and
// they complete in order, so at the top of stage k the wave waits until at
// most (stages issued after k) * LD of its loads are outstanding; the barrier
// that follows makes every wave's part of stage k visible and frees the slot
// that stage k - 1 was read from, which the next issue refills.
template <int PREC, int OUTT, int BM, int BN, int NS>
__global__ __launch_bounds__(256) void gemm_ring_kernel(GemmArgs g) {
    constexpr int EB = Ty<PREC>::EB;
    constexpr int TI = BM / 64, TJ = BN / 64;
    constexpr int A_BYTES = BM * 128, B_BYTES = BN * 128;
    constexpr int STAGE = A_BYTES + B_BYTES;
    constexpr int LD_A = BM / 32, LD_B = BN / 32;  // 1 KiB (8-row) load instructions per wave per stage
    constexpr int LD = LD_A + LD_B;
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int M = g.m_dev ? *g.m_dev : g.m_host;
    const int m_tiles = min((M + BM - 1) / BM, g.m_tiles_cap);
    const int n_tiles = g.N / BN;
    const int total = m_tiles * n_tiles;
    const int ktiles = g.K * EB / 128;

    const int grid = gridDim.x;
    const int grid8 = grid & ~7;
    int first = blockIdx.x;
    if (blockIdx.x < grid8) first = (blockIdx.x & 7) * (grid8 >> 3) + (blockIdx.x >> 3);

    const int lrow = lane >> 3;  // row of this lane within an 8-row load instruction

    for (int t = first; t < (g.persistent ? total : (first < total ? first + 1 : 0)); t += grid) {
        const int tm = t / n_tiles, tn = t % n_tiles;
        const int m0 = tm * BM, n0 = tn * BN;
        const uint8_t* Ag = g.A + ((size_t)m0 * g.lda + group_a_col(g, n0)) * EB;
        const uint8_t* Bg = g.Bt + (size_t)n0 * g.ldb * EB;

        floatx16 acc[TI][TJ];
        _Pragma("unroll") for (int i = 0; i < TI; i++)
            _Pragma("unroll") for (int j = 0; j < TJ; j++)
                _Pragma("unroll") for (int e = 0; e < 16; e++) acc[i][j][e] = 0.f;

        // Stage kt into ring slot sl: this wave's instructions q = wave + 4i.
        auto issue = [&](int kt, int sl) {
            uint8_t* base = smem + sl * STAGE;
            const int kbyte = kt * 128;
            _Pragma("unroll") for (int i = 0; i < LD; i++) {
                const int q = wave + 4 * i;
                const bool isA = q < BM / 8;
                const int qq = isA ? q : q - BM / 8;
                const int row = 8 * qq + lrow;
                const int key = ((row >> 1) & 7);
                const int ch = (lane & 7) ^ key;
                const uint8_t* src = (isA ? Ag + (size_t)row * g.lda * EB : Bg + (size_t)row * g.ldb * EB) + kbyte + ch * 16;
                uint8_t* dst = base + (isA ? 0 : A_BYTES) + qq * 1024;
                __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
            }
        };

        __syncthreads();  // the previous tile's readers are done with every slot
        _Pragma("unroll") for (int s0 = 0; s0 < NS - 1; s0++)
            if (s0 < ktiles) issue(s0, s0);
        for (int kt = 0; kt < ktiles; kt++) {
            // stages issued so far: min(ktiles, kt + NS - 1); this wave may
            // leave the ones after kt in flight
            const int ahead = min(ktiles, kt + NS - 1) - (kt + 1);
            static_assert(NS >= 2 && NS <= 4, "ring depth");
            if (NS == 4 && ahead >= 2) wait_vmcnt<(NS == 4 ? 2 * LD : 0)>();
            else if (ahead >= 1) wait_vmcnt<LD>();
            else wait_vmcnt<0>();
            // A bare s_barrier: __syncthreads() would also wait for every
            // outstanding load (its release fence), draining the ring.  The
            // empty asm statements keep the compiler from moving LDS accesses
            // across the barrier.
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (kt + NS - 1 < ktiles) issue(kt + NS - 1, (kt + NS - 1) % NS);
            const uint8_t* a_s = smem + (kt % NS) * STAGE;
            mma_stage<PREC, BM, BN>(a_s, a_s + A_BYTES, acc, wm, wn, lane);
        }

        const int half = lane >> 5, c32 = lane & 31;
        _Pragma("unroll") for (int j = 0; j < TJ; j++) {
            const int n = n0 + wn * (BN / 2) + j * 32 + c32;
            const float bn = g.bias ? g.bias[n] : 0.f;
            const float sn = PREC == 2 ? g.colscale[n] * g.a_scale : 1.f;
            _Pragma("unroll") for (int i = 0; i < TI; i++)
                epi_tile<OUTT>(g, acc[i][j], sn, bn, (m0 + wm * (BM / 2) + i * 32 + 4 * half) * g.ldc + n);
        }
    }
}

// ------------------------------------------------------------ GEMM, wide blocks
// MFMAs of one 128-byte K stage for a wave's TI x TJ 32 x 32 tiles (A rows
// ar0 + 32 i, B rows br0 + 32 j), with every LDS read of the stage issued before
// the first MFMA: the MFMAs then wait only for their own operands and run while
// the rest of the stage is still arriving.  A scheduling barrier keeps the
// compiler from sinking the reads back next to their MFMAs (which it does to
// save registers, leaving one LDS round trip exposed per 32-byte K group).
// The MFMA sequence per output element is mma_stage's (same chunk, same order).
template <int PREC, int TI, int TJ>
__device__ __forceinline__ void mma_stage_pre(const uint8_t* a_s, const uint8_t* b_s, floatx16 (&acc)[TI][TJ],
                                              int ar0, int br0, int lane) {
    const int half = lane >> 5, r32 = lane & 31;
    if (PREC == 2) {
        constexpr int KB = TI * TJ > 4 ? 1 : 2;  // 64-element K groups read per batch (as below)
        _Pragma("unroll") for (int k0 = 0; k0 < 2; k0 += KB) {
            intx8 af[KB][TI], bfr[KB][TJ];
            _Pragma("unroll") for (int q = 0; q < KB; q++) {
                const int kg = k0 + q;
                _Pragma("unroll") for (int i = 0; i < TI; i++) {
                    const int row = ar0 + i * 32 + r32;
                    const u32x4 lo = *reinterpret_cast<const u32x4*>(a_s + swz(row, 4 * kg + 2 * half));
                    const u32x4 hi = *reinterpret_cast<const u32x4*>(a_s + swz(row, 4 * kg + 2 * half + 1));
                    af[q][i] = intx8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
                }
                _Pragma("unroll") for (int j = 0; j < TJ; j++) {
                    const int row = br0 + j * 32 + r32;
                    const u32x4 lo = *reinterpret_cast<const u32x4*>(b_s + swz(row, 4 * kg + 2 * half));
                    const u32x4 hi = *reinterpret_cast<const u32x4*>(b_s + swz(row, 4 * kg + 2 * half + 1));
                    bfr[q][j] = intx8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            _Pragma("unroll") for (int q = 0; q < KB; q++)
                _Pragma("unroll") for (int i = 0; i < TI; i++)
                    _Pragma("unroll") for (int j = 0; j < TJ; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af[q][i], bfr[q][j], acc[i][j], 0,
                                                                                   0, 0, 127, 0, 127);
            if (KB < 2) __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        // K groups read per batch: all four, or two at a time when the wave's
        // tile is 64 x 128 (the fragments of four would not fit beside its
        // accumulators); the MFMA order is the same either way
        constexpr int KB = TI * TJ > 4 ? 2 : 4;
        _Pragma("unroll") for (int k0 = 0; k0 < 4; k0 += KB) {
            u32x4 af[KB][TI], bfr[KB][TJ];
            _Pragma("unroll") for (int q = 0; q < KB; q++) {
                const int kg = k0 + q;
                _Pragma("unroll") for (int i = 0; i < TI; i++)
                    af[q][i] = *reinterpret_cast<const u32x4*>(a_s + swz(ar0 + i * 32 + r32, 2 * kg + half));
                _Pragma("unroll") for (int j = 0; j < TJ; j++)
                    bfr[q][j] = *reinterpret_cast<const u32x4*>(b_s + swz(br0 + j * 32 + r32, 2 * kg + half));
            }
            __builtin_amdgcn_sched_barrier(0);
            _Pragma("unroll") for (int q = 0; q < KB; q++) {
                if (PREC == 1) {
                    _Pragma("unroll") for (int i = 0; i < TI; i++)
                        _Pragma("unroll") for (int j = 0; j < TJ; j++)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, af[q][i]),
                                                                                __builtin_bit_cast(bf16x8, bfr[q][j]),
                                                                                acc[i][j], 0, 0, 0);
                } else {
                    _Pragma("unroll") for (int e = 0; e < 4; e++)
                        _Pragma("unroll") for (int i = 0; i < TI; i++)
                            _Pragma("unroll") for (int j = 0; j < TJ; j++)
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(af[q][i][e]),
                                                                                 __uint_as_float(bfr[q][j][e]), acc[i][j],
                                                                                 0, 0, 0);
                }
            }
            if (KB < 4) __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// 256 x 128 tile, one block per compute unit, NW waves in a 4 x (NW / 4) grid
// (8 waves: 64 x 64 each; 16 waves: 64 x 32 each), operands from global memory
// straight into a ring of NS LDS stages (as gemm_ring_kernel), each stage's
// fragments read whole before its MFMAs (mma_stage_pre).  With 8 waves, a wave
// raises its priority while it issues MFMAs, so that of the two waves sharing
// a SIMD the one with operands in registers goes first instead of both reading
// LDS and then both multiplying.  Same per-element MFMA sequence and epilogue
// as the other tiles: bitwise equal results.
template <int PREC, int OUTT, int NW, int NS, bool TC = false, int BNT = 128>
__global__ __launch_bounds__(NW * 64) void gemm_wide_kernel(GemmArgs g) {
    constexpr int BM = 256, BN = BNT, NT = NW * 64;
    constexpr int EB = Ty<PREC>::EB;
    constexpr int A_BYTES = BM * 128, B_BYTES = BN * 128, STAGE = A_BYTES + B_BYTES;
    constexpr int NA = A_BYTES / 1024, LD = STAGE / 1024 / NW;  // 1 KiB load instructions per wave per stage
    constexpr int TI = 2, TJ = BN / (8 * NW);  // waves in a 4 x (NW / 4) grid, 64 x (TJ 32) each
    static_assert(NW == 8 || NW == 16, "wave count");
    static_assert(NS >= 2 && NS <= 3, "ring depth");
    static_assert(BN == 128 || (BN == 256 && NW == 8), "tile width");
    static_assert(!TC || BN == 128, "the transposed copy is staged for 128-column tiles");
    static_assert((STAGE / 1024) % NW == 0, "loads per wave");
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 3, wn = wave >> 2;
    const int M = g.m_dev ? *g.m_dev : g.m_host;
    const int m_tiles = min((M + BM - 1) / BM, g.m_tiles_cap);
    const int n_tiles = g.N / BN;
    const int split = g.split > 1 ? g.split : 1;
    const int tiles_mn = m_tiles * n_tiles;
    const int total = tiles_mn * split;
    const int kslice = g.K / split;
    const int ktiles = kslice * EB / 128;
    const int grid = gridDim.x, grid8 = grid & ~7;
    int first = blockIdx.x;
    if (blockIdx.x < grid8) first = (blockIdx.x & 7) * (grid8 >> 3) + (blockIdx.x >> 3);
    const int lrow = lane >> 3;
    (void)NT;

    const bool dyn = g.tile_ctr != nullptr;
    __shared__ int s_next;
    const int t_end = g.persistent ? total : (first < total ? first + 1 : 0);
    for (int t = first; dyn ? t < total : t < t_end;) {
        int nxt = 0;
        if (dyn && tid == 0) nxt = tile_fetch(g, grid);
        const int sl = t / tiles_mn, tt = t - sl * tiles_mn;
        const int m0 = (tt / n_tiles) * BM, n0 = (tt % n_tiles) * BN;
        const uint8_t* Ag = g.A + ((size_t)m0 * g.lda + group_a_col(g, n0) + (size_t)sl * kslice) * EB;
        const uint8_t* Bg = g.Bt + ((size_t)n0 * g.ldb + (size_t)sl * kslice) * EB;
        floatx16 acc[TI][TJ];
        _Pragma("unroll") for (int i = 0; i < TI; i++)
            _Pragma("unroll") for (int j = 0; j < TJ; j++)
                _Pragma("unroll") for (int e = 0; e < 16; e++) acc[i][j][e] = 0.f;

        auto issue = [&](int kt) {
            uint8_t* base = smem + (kt % NS) * STAGE;
            const int kbyte = kt * 128;
            _Pragma("unroll") for (int i = 0; i < LD; i++) {
                const int q = wave + NW * i;
                const bool isA = q < NA;
                const int qq = isA ? q : q - NA;
                const int row = 8 * qq + lrow;
                const int ch = (lane & 7) ^ ((row >> 1) & 7);
                const uint8_t* src =
                    (isA ? Ag + (size_t)row * g.lda * EB : Bg + (size_t)row * g.ldb * EB) + kbyte + ch * 16;
                uint8_t* dst = base + (isA ? 0 : A_BYTES) + qq * 1024;
                __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
            }
        };

        __syncthreads();  // the previous tile's readers are done with every slot
        _Pragma("unroll") for (int s0 = 0; s0 < NS - 1; s0++)
            if (s0 < ktiles) issue(s0);
        for (int kt = 0; kt < ktiles; kt++) {
            // stages issued: min(ktiles, kt + NS - 1); those after kt may stay in flight
            if (NS == 3 && kt + 1 < ktiles) wait_vmcnt<(NS == 3 ? LD : 0)>();
            else wait_vmcnt<0>();
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (kt + NS - 1 < ktiles) issue(kt + NS - 1);
            const uint8_t* a_s = smem + (kt % NS) * STAGE;
            if (NW == 8) __builtin_amdgcn_s_setprio(1);
            mma_stage_pre<PREC, TI, TJ>(a_s, a_s + A_BYTES, acc, wm * 64, wn * (TJ * 32), lane);
            if (NW == 8) __builtin_amdgcn_s_setprio(0);
        }

        const int half = lane >> 5, c32 = lane & 31;
        GemmArgs gs = g;  // slice sl writes its own C
        if (sl) gs.C = g.C + (size_t)sl * g.c_split * (OUTT == 0 ? 4 : OUTT == 1 ? 2 : 1);
        floatx16 vt[TI][TJ];
        _Pragma("unroll") for (int j = 0; j < TJ; j++) {
            const int n = n0 + wn * (TJ * 32) + j * 32 + c32;
            const float bn = g.bias ? g.bias[n] : 0.f;
            const float sn = PREC == 2 ? g.colscale[n] * g.a_scale : 1.f;
            _Pragma("unroll") for (int i = 0; i < TI; i++) {
                const int o0 = (m0 + wm * 64 + i * 32 + 4 * half) * g.ldc + n;
                if (TC) vt[i][j] = epi_tile_v<OUTT>(gs, acc[i][j], sn, bn, o0);
                else epi_tile<OUTT>(gs, acc[i][j], sn, bn, o0);
            }
        }
        if (TC && OUTT != 2) {
            // Transposed copy through LDS: each wave turns its 64 x (TJ 32)
            // region into rows of Ct (MR rows of C, 128 bytes, per pass), so
            // every store is 16 bytes and a row gets whole 128-byte lines.
            constexpr int EO = OUTT == 0 ? 4 : 2, MR = 128 / EO, RS = 144;  // LDS row stride: 128 bytes + 16
            __syncthreads();  // every wave is done with the ring
            uint8_t* reg = smem + (size_t)wave * (TJ * 32) * RS;
            _Pragma("unroll") for (int rd = 0; rd < 64 / MR; rd++) {
                _Pragma("unroll") for (int i = rd * (MR / 32); i < (rd + 1) * (MR / 32); i++)
                    _Pragma("unroll") for (int j = 0; j < TJ; j++)
                        _Pragma("unroll") for (int a4 = 0; a4 < 4; a4++) {
                            const floatx16& v = vt[i][j];
                            uint8_t* d = reg + (32 * j + c32) * RS + ((i - rd * (MR / 32)) * 32 + 8 * a4 + 4 * half) * EO;
                            if (OUTT == 0) {
                                *reinterpret_cast<float4*>(d) = make_float4(v[4 * a4], v[4 * a4 + 1], v[4 * a4 + 2], v[4 * a4 + 3]);
                            } else {
                                const uint32_t lo = f32_to_bf16(v[4 * a4]) | ((uint32_t)f32_to_bf16(v[4 * a4 + 1]) << 16);
                                const uint32_t hi = f32_to_bf16(v[4 * a4 + 2]) | ((uint32_t)f32_to_bf16(v[4 * a4 + 3]) << 16);
                                *reinterpret_cast<uint2*>(d) = make_uint2(lo, hi);
                            }
                        }
                _Pragma("unroll") for (int q = 0; q < TJ * 4; q++) {
                    const int cidx = q * 64 + lane, n = cidx >> 3, part = cidx & 7;
                    const int nr = n0 + wn * (TJ * 32) + n;
                    const u32x4 val = *reinterpret_cast<const u32x4*>(reg + n * RS + part * 16);
                    uint8_t* dst = g.Ct + ((size_t)nr * g.ldct + m0 + wm * 64 + rd * MR) * EO + part * 16;
                    if (g.ct_rows <= 0 || nr < g.ct_rows) *reinterpret_cast<u32x4*>(dst) = val;
                }
            }
        }
        if (dyn) {
            __syncthreads();
            if (tid == 0) s_next = nxt;
            __syncthreads();
            t = s_next;
        } else {
            t += grid;
        }
    }
    if (dyn) {
        __syncthreads();
        if (tid == 0) tile_sched_exit(g);
    }
}

// ------------------------------------------------------------ small-batch GEMM
// One wave per 32 x 32 output tile, operands read from global memory straight
// into registers (no LDS, no barriers), several K stages prefetched ahead of
// the one being multiplied.  At a few hundred rows or fewer the tiles of
// gemm_kernel would leave most compute units idle; here every 32 x 32 tile is
// a block of its own.  Every output element goes through exactly the MFMA
// sequence of gemm_kernel (the same 16-byte chunk of each 128-byte K stage in
// each MFMA, the same order), so the two kernels give bitwise equal results
// and a state's value does not depend on the batch size that picked the kernel.
// One wave computes the 32 x 32 output tile at rows m0, columns n0 (shared by
// gemm_small_kernel and the fused forward kernel).
template <int PREC, int OUTT, bool COH = false>
__device__ __forceinline__ void small_tile(const GemmArgs& g, int m0, int n0, int lane) {
    constexpr int EB = Ty<PREC>::EB;
    const int half = lane >> 5, r32 = lane & 31;
    const uint8_t* Ar = g.A + ((size_t)(m0 + r32) * g.lda + group_a_col(g, n0)) * EB;
    const uint8_t* Br = g.Bt + (size_t)(n0 + r32) * g.ldb * EB;
    const int ktiles = g.K * EB / 128;
    // Byte offset, inside a 128-byte K stage, of this lane's register slot i.
    // fp32 / bf16: MFMA group i reads chunk 2i + half.  fp8: group kg reads
    // chunks 4kg + 2half and 4kg + 2half + 1 (slots 2kg and 2kg + 1).
    int off[4];
    _Pragma("unroll") for (int i = 0; i < 4; i++)
        off[i] = 16 * (PREC == 2 ? 4 * (i >> 1) + 2 * half + (i & 1) : 2 * i + half);

    // A ring of DEPTH K stages in registers: at a few dozen waves on the
    // chip, the loads in flight per wave decide how well memory latency is hidden.
    constexpr int DEPTH = 4;
    floatx16 acc;
    _Pragma("unroll") for (int e = 0; e < 16; e++) acc[e] = 0.f;
    u32x4 a[DEPTH][4], b[DEPTH][4];
    _Pragma("unroll") for (int j = 0; j < DEPTH; j++) {
        if (j < ktiles) {
            _Pragma("unroll") for (int i = 0; i < 4; i++) {
                a[j][i] = ld16<COH>(Ar + j * 128 + off[i]);
                b[j][i] = *reinterpret_cast<const u32x4*>(Br + j * 128 + off[i]);
            }
        }
    }
    for (int k0 = 0; k0 < ktiles; k0 += DEPTH) {
        _Pragma("unroll") for (int j = 0; j < DEPTH; j++) {
            const int kt = k0 + j;
            if (kt < ktiles) {
                if (PREC == 2) {
                    _Pragma("unroll") for (int kg = 0; kg < 2; kg++) {
                        const u32x4 al = a[j][2 * kg], ah = a[j][2 * kg + 1], bl = b[j][2 * kg], bh = b[j][2 * kg + 1];
                        const intx8 af = intx8{(int)al.x, (int)al.y, (int)al.z, (int)al.w, (int)ah.x, (int)ah.y, (int)ah.z, (int)ah.w};
                        const intx8 bf = intx8{(int)bl.x, (int)bl.y, (int)bl.z, (int)bl.w, (int)bh.x, (int)bh.y, (int)bh.z, (int)bh.w};
                        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af, bf, acc, 0, 0, 0, 127, 0, 127);
                    }
                } else if (PREC == 1) {
                    _Pragma("unroll") for (int kg = 0; kg < 4; kg++)
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[j][kg]),
                                                                      __builtin_bit_cast(bf16x8, b[j][kg]), acc, 0, 0, 0);
                } else {
                    _Pragma("unroll") for (int kg = 0; kg < 4; kg++)
                        _Pragma("unroll") for (int e = 0; e < 4; e++) {
                            const u32x4 av = a[j][kg], bv = b[j][kg];
                            const uint32_t ai = e == 0 ? av.x : e == 1 ? av.y : e == 2 ? av.z : av.w;
                            const uint32_t bj = e == 0 ? bv.x : e == 1 ? bv.y : e == 2 ? bv.z : bv.w;
                            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(ai), __uint_as_float(bj), acc, 0, 0, 0);
                        }
                }
                if (kt + DEPTH < ktiles) {
                    const int kbyte = (kt + DEPTH) * 128;
                    _Pragma("unroll") for (int i = 0; i < 4; i++) {
                        a[j][i] = ld16<COH>(Ar + kbyte + off[i]);
                        b[j][i] = *reinterpret_cast<const u32x4*>(Br + kbyte + off[i]);
                    }
                }
            }
        }
    }
    // Epilogue, as in gemm_kernel: column n0 + lane%32, rows 8a + 4*half + b.
    const int n = n0 + r32;
    const float bn = g.bias ? g.bias[n] : 0.f;
    const float sn = PREC == 2 ? g.colscale[n] * g.a_scale : 1.f;
    epi_tile<OUTT, COH>(g, acc, sn, bn, (m0 + 4 * half) * g.ldc + n);
}

template <int PREC, int OUTT>
__global__ __launch_bounds__(64) void gemm_small_kernel(GemmArgs g) {
    const int M = g.m_dev ? *g.m_dev : g.m_host;
    const int m_tiles = min((M + 31) / 32, g.m_tiles_cap);
    const int n_tiles = g.N / 32;
    const int tm = blockIdx.x / n_tiles, tn = blockIdx.x % n_tiles;
    if (tm >= m_tiles) return;
    small_tile<PREC, OUTT>(g, tm * 32, tn * 32, threadIdx.x);
}

// ------------------------------------------------------------ head
// Manhattan distance of a packed sliding-tile state (board side known at
// compile time).
template <int SIDE>
__device__ __forceinline__ int manhattan_packed(uint64_t w) {
    int md = 0;
    _Pragma("unroll") for (int p = 0; p < SIDE * SIDE; p++) {
        const int t = (int)((w >> (4 * p)) & 15);
        if (t) md += abs(p / SIDE - t / SIDE) + abs(p % SIDE - t % SIDE);
    }
    return md;
}

__device__ __forceinline__ int head_md(const HeadArgs& h, int r) {
    if (!h.combine_md || h.domain >= 2) return -1;
    const uint64_t w = reinterpret_cast<const uint64_t*>(h.packed)[r];
    return h.domain == 0 ? manhattan_packed<3>(w) : manhattan_packed<4>(w);
}

// Regression output rule: h = floor / round-half-even of y - offset, clamped
// at 0, then combined with Manhattan distance (min, max, or MD plus the
// clamped value); non-finite -> MD or 0.
__device__ __forceinline__ void regression_rule(const HeadArgs& h, int r, float y, int md) {
    const float v = y - h.offset;
    int hv;
    if (!isfinite(v)) {
        hv = md >= 0 ? md : 0;
    } else {
        const float f = h.mode == 1 ? rintf(v) : floorf(v);
        hv = f < 0.f ? 0 : f > 1e9f ? 1000000000 : (int)f;
        if (md >= 0) hv = h.combine_md == 3 ? min(hv, 1000000000 - md) + md : h.combine_md == 2 ? max(hv, md) : min(hv, md);
    }
    if (h.raw) h.raw[r] = v;
    h.h_out[r] = hv;
}

// Regression head: 16 lanes per state (4 states per wave, 16 per block), each
// lane summing x[k] * w[k] over 16-byte slices k = 16-lane stride apart, then
// a 16-lane butterfly; the first lane of each group applies the rule.  An
// ensemble's x holds the members' last activations side by side (K values
// each) and w their output weights; member outputs y_i = w_i . x_i + b_i are
// combined as min_i y_i or y_0 + y_1 + ... before the rule.
constexpr int kMaxMembers = 4;

// Row r by the 16-lane group whose lane index within the group is j (all 16
// lanes take part in the butterfly; lane j = 0 writes the result).
template <int IN /*0 f32, 1 bf16, 2 fp8*/, int HW /*0 f32, 1 bf16*/, bool COH = false>
__device__ __forceinline__ void head_reg_row(const HeadArgs& h, int n, int r, int j) {
    constexpr int CH = IN == 0 ? 4 : IN == 1 ? 8 : 16;  // elements per 16-byte load of x
    constexpr int XB = IN == 0 ? 4 : IN == 1 ? 2 : 1;
    const bool live = r < n;
    // the record for the Manhattan rule is fetched before the dot product
    const uint64_t rec = live && j == 0 && h.combine_md && h.domain < 2 ? reinterpret_cast<const uint64_t*>(h.packed)[r] : 0;
    float y[kMaxMembers] = {0.f, 0.f, 0.f, 0.f};
    if (live) {
        const uint8_t* xrow = reinterpret_cast<const uint8_t*>(h.X) + (size_t)r * h.ldx * XB;
        const int Ktot = h.K * h.members;
        for (int k = j * CH; k < Ktot; k += 16 * CH) {
            float x[CH], w[CH];
            const u32x4 xv = ld16<COH>(xrow + (size_t)k * XB);
            const uint32_t xu[4] = {xv.x, xv.y, xv.z, xv.w};
            if (IN == 0) {
                _Pragma("unroll") for (int e = 0; e < 4; e++) x[e] = __uint_as_float(xu[e]);
            } else if (IN == 1) {
                _Pragma("unroll") for (int e = 0; e < 4; e++) {
                    x[2 * e] = bf16_to_f32((uint16_t)(xu[e] & 0xFFFF));
                    x[2 * e + 1] = bf16_to_f32((uint16_t)(xu[e] >> 16));
                }
            } else {
                _Pragma("unroll") for (int e = 0; e < 16; e++) x[e] = fp8_to_f32((xu[e >> 2] >> (8 * (e & 3))) & 0xFF) * h.x_scale;
            }
            if (HW == 0) {
                _Pragma("unroll") for (int e = 0; e < CH; e++) w[e] = reinterpret_cast<const float*>(h.W)[k + e];
            } else {
                _Pragma("unroll") for (int q = 0; q < CH / 8; q++) {
                    const uint4 wv = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(h.W) + k + 8 * q);
                    const uint32_t wu[4] = {wv.x, wv.y, wv.z, wv.w};
                    _Pragma("unroll") for (int e = 0; e < 4; e++) {
                        w[8 * q + 2 * e] = bf16_to_f32((uint16_t)(wu[e] & 0xFFFF));
                        w[8 * q + 2 * e + 1] = bf16_to_f32((uint16_t)(wu[e] >> 16));
                    }
                }
            }
            float d = 0.f;
            _Pragma("unroll") for (int e = 0; e < CH; e++) d += x[e] * w[e];
            const int member = k / h.K;  // a slice never straddles members (K is a multiple of 128)
            _Pragma("unroll") for (int i = 0; i < kMaxMembers; i++)
                if (i == member) y[i] += d;
        }
    }
    _Pragma("unroll") for (int i = 0; i < kMaxMembers; i++)
        _Pragma("unroll") for (int s = 8; s >= 1; s >>= 1) y[i] += __shfl_xor(y[i], s, 64);
    if (!live || j != 0) return;
    float yc = y[0] + h.b[0];
    for (int i = 1; i < h.members && i < kMaxMembers; i++) {
        const float yi = y[i] + h.b[i];
        // minimum that keeps a NaN (the rule then falls back to Manhattan / 0)
        yc = h.ens_rule != 0 ? yc + yi : (yc != yc || yi != yi) ? yc + yi : fminf(yc, yi);
    }
    int md = -1;
    if (h.combine_md && h.domain < 2) md = h.domain == 0 ? manhattan_packed<3>(rec) : manhattan_packed<4>(rec);
    regression_rule(h, r, yc, md);
}

template <int IN, int HW>
__global__ __launch_bounds__(256) void head_reg_kernel(HeadArgs h) {
    const int n = min(h.n_dev ? *h.n_dev : h.n_host, h.m_cap);
    head_reg_row<IN, HW>(h, n, blockIdx.x * 16 + (threadIdx.x >> 4), threadIdx.x & 15);
}

// Classifier head: one wave per state.  y[o] = sum_k x[k] * Wo[o][k] + bo[o]
// for o < n_out, lanes own K slices of 4; wave-wide butterfly sums; lane 0
// applies the quantile or arg-max rule.  head_cls_row: row r (< n) by one
// whole wave.
template <int IN /*0 f32, 1 bf16, 2 fp8*/, int HW /*0 f32, 1 bf16*/, int NOUT, bool COH = false>
__device__ __forceinline__ void head_cls_row(const HeadArgs& h, int r, int lane) {
    float y[NOUT];
    for (int o = 0; o < NOUT; o++) y[o] = 0.f;
    for (int k = lane * 4; k < h.K; k += 256) {
        float x[4];
        const size_t xo = (size_t)r * h.ldx + k;
        if (IN == 0) {
            const u32x4 v = ld16<COH>(reinterpret_cast<const uint8_t*>((const float*)h.X + xo));
            x[0] = __uint_as_float(v.x); x[1] = __uint_as_float(v.y); x[2] = __uint_as_float(v.z); x[3] = __uint_as_float(v.w);
        } else if (IN == 1) {
            const uint64_t* p = reinterpret_cast<const uint64_t*>((const uint16_t*)h.X + xo);
            const uint64_t u = COH ? ld_coh(p) : *p;
            const uint32_t vx = (uint32_t)u, vy = (uint32_t)(u >> 32);
            x[0] = bf16_to_f32(vx & 0xFFFF); x[1] = bf16_to_f32(vx >> 16);
            x[2] = bf16_to_f32(vy & 0xFFFF); x[3] = bf16_to_f32(vy >> 16);
        } else {
            const uint32_t* p = reinterpret_cast<const uint32_t*>((const uint8_t*)h.X + xo);
            const uint32_t v = COH ? ld_coh(p) : *p;
            for (int i = 0; i < 4; i++) x[i] = fp8_to_f32((v >> (8 * i)) & 0xFF) * h.x_scale;
        }
        for (int o = 0; o < NOUT; o++) {
            if (o >= h.n_out) break;
            const size_t wo = (size_t)o * h.K + k;
            float w[4];
            if (HW == 0) {
                const float4 v = *reinterpret_cast<const float4*>((const float*)h.W + wo);
                w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
            } else {
                const uint2 v = *reinterpret_cast<const uint2*>((const uint16_t*)h.W + wo);
                w[0] = bf16_to_f32(v.x & 0xFFFF); w[1] = bf16_to_f32(v.x >> 16);
                w[2] = bf16_to_f32(v.y & 0xFFFF); w[3] = bf16_to_f32(v.y >> 16);
            }
            y[o] += x[0] * w[0] + x[1] * w[1] + x[2] * w[2] + x[3] * w[3];
        }
    }
    for (int o = 0; o < NOUT; o++) {
        if (o >= h.n_out) break;
        float v = y[o];
        for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
        y[o] = v + h.b[o];
    }
    if (lane != 0) return;
    const int md = head_md(h, r);
    // a NaN or +infinite logit leaves the rule undefined: classic value or 0
    bool undefined = false;
    for (int o = 0; o < NOUT; o++)
        if (o < h.n_out && (y[o] != y[o] || y[o] == INFINITY)) undefined = true;
    int hv;
    if (undefined && h.mode >= 3) {
        hv = md >= 0 ? md : 0;
    } else if (h.mode == 4) {
        int best = 0;
        for (int o = 1; o < NOUT; o++)
            if (o < h.n_out && y[o] > y[best]) best = o;
        hv = best;
    } else if (h.mode == 3) {
        float mx = y[0];
        for (int o = 1; o < NOUT; o++)
            if (o < h.n_out) mx = fmaxf(mx, y[o]);
        float e[NOUT], sum = 0.f;
        for (int o = 0; o < NOUT; o++)
            if (o < h.n_out) { e[o] = expf(y[o] - mx); sum += e[o]; }
        float cdf = 0.f;
        hv = h.n_out - 1;
        for (int o = 0; o < NOUT; o++) {
            if (o >= h.n_out) break;
            cdf += e[o] / sum;
            if (cdf >= h.q) { hv = o; break; }
        }
        if (!(sum > 0.f) || !isfinite(mx)) hv = md >= 0 ? md : 0;
    } else {
        regression_rule(h, r, y[0], md);  // a one-output network under a regression rule
        return;
    }
    if (h.raw) for (int o = 0; o < NOUT; o++) if (o < h.n_out) h.raw[(size_t)r * h.n_out + o] = y[o];
    h.h_out[r] = hv;
}

template <int IN, int HW, int NOUT>
__global__ __launch_bounds__(256) void head_cls_kernel(HeadArgs h) {
    const int n = min(h.n_dev ? *h.n_dev : h.n_host, h.m_cap);
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    head_cls_row<IN, HW, NOUT>(h, r, threadIdx.x & 63);
}

// ------------------------------------------------------------ fused forward
// The whole forward pass of one batch in a single persistent launch, for small
// and medium batches where each separate kernel would cost about its launch and
// ramp.  A grid of one-wave blocks pulls work items off an atomic counter in a
// fixed order: the layer-1 gather tiles (32 rows x 32 columns) of every
// 32-row block, then each matrix layer's 32 x 32 output tiles, then the head
// per 32-row block.  An item of stage s on row block b first waits until every
// stage s - 1 tile of block b has been counted done (a row's outputs need all
// of its inputs' columns), then computes with exactly the arithmetic of the
// separate kernels (gather: bias then cells in order; tiles: small_tile; head:
// head_reg_row / head_cls_row), so results are bitwise equal to theirs.  Items
// are taken in order and each waits only on earlier items, which running waves
// hold and finish without waiting on later ones: the wait always ends, with no
// assumption about how many waves are resident.  Activations pass between
// waves through device-coherent loads and stores (ld_coh / st_coh): a tile is
// counted done (atomic add) after its stores have completed, and a waiting
// wave polls the count with coherent loads before reading the tile's rows
// coherently; weights and tables are read through the caches as usual.  The
// agent-scope fences that would do the same write back or invalidate a whole
// L2 and, issued by every polling wave, stall the device.  Every wait is bounded
// (spin_limit sleeps); a wait that runs out sets a flag, and the launch then
// writes h = -1 for every row so the caller sees the failure.  The last wave
// to finish returns the counters to zero for the next launch, so a captured
// graph can replay the kernel with no memset node.
constexpr int kFusedMaxLayers = 12;
// Switched off: on the GPU, launches of this kernel did not return within 90 to
// 120 s (no fault, no wrong value seen), first with agent-scope acquire polls,
// then with device-coherent polls.  launch_fused refuses every launch until
// the cause is shown; the kernel is not instantiated meanwhile.
constexpr bool kFusedEnabled = false;

struct FusedArgs {
    const uint64_t* packed;
    const int32_t* n_dev;
    int n_host, m_cap;
    const float* table;      // layer-1 table [t_rows][N1], float32
    const float* bias1;
    int N1, ld1;             // padded layer-1 width, row stride of its output (elements)
    uint8_t* out1;
    float out1_inv_scale;
    int n_layers;
    int* sync;               // [0] next item, [1] waves done, [2] timeout flag, [4 + s * rb_cap + b] tiles done
    int rb_cap;
    int spin_limit;
    HeadArgs head;
    GemmArgs layer[kFusedMaxLayers];
};

static_assert(sizeof(FusedArgs) <= 4096, "kernel arguments are passed by value");

// Layer 1 for rows [32 rb, 32 rb + 32), columns [32 ct, 32 ct + 32): lane l
// takes row l % 32 and 16 columns; the sum order per output (bias, then the
// cells in order) is gather_l1_kernel's.
template <int DOM, int OUT>
__device__ __forceinline__ void gather_tile(const FusedArgs& f, int n, int rb, int ct, int lane) {
    using D = Dec<DOM>;
    const int r = rb * 32 + (lane & 31);
    const int c0 = ct * 32 + (lane >> 5) * 16;
    uint64_t w[D::WORDS];
    _Pragma("unroll") for (int i = 0; i < D::WORDS; i++) w[i] = r < n ? f.packed[(size_t)r * D::WORDS + i] : 0;
    float acc[16];
    _Pragma("unroll") for (int j = 0; j < 16; j++) acc[j] = f.bias1[c0 + j];
    constexpr int CH = 4;  // cells whose 64-byte row slices are in flight at once
    _Pragma("unroll") for (int p0 = 0; p0 < D::P; p0 += CH) {
        float4 v[CH][4];
        _Pragma("unroll") for (int k = 0; k < CH; k++) {
            if (p0 + k < D::P) {
                const float4* row = reinterpret_cast<const float4*>(f.table + (size_t)D::row(w, p0 + k) * f.N1 + c0);
                _Pragma("unroll") for (int q = 0; q < 4; q++) v[k][q] = row[q];
            }
        }
        _Pragma("unroll") for (int k = 0; k < CH; k++) {
            if (p0 + k < D::P) {
                _Pragma("unroll") for (int q = 0; q < 4; q++) {
                    acc[4 * q] += v[k][q].x; acc[4 * q + 1] += v[k][q].y;
                    acc[4 * q + 2] += v[k][q].z; acc[4 * q + 3] += v[k][q].w;
                }
            }
        }
    }
    _Pragma("unroll") for (int j = 0; j < 16; j++) acc[j] = r < n ? fmaxf(acc[j], 0.f) : 0.f;
    // the output goes to waves on other XCDs: device-coherent stores
    constexpr int EO = OUT == 0 ? 4 : OUT == 1 ? 2 : 1;
    uint8_t* dst = f.out1 + ((size_t)r * f.ld1 + c0) * EO;
    if (OUT == 0) {
        _Pragma("unroll") for (int q = 0; q < 4; q++)
            st16<true>(dst + 16 * q, u32x4{__float_as_uint(acc[4 * q]), __float_as_uint(acc[4 * q + 1]),
                                           __float_as_uint(acc[4 * q + 2]), __float_as_uint(acc[4 * q + 3])});
    } else if (OUT == 1) {
        uint32_t u[8];
        _Pragma("unroll") for (int e = 0; e < 8; e++)
            u[e] = (uint32_t)f32_to_bf16(acc[2 * e]) | ((uint32_t)f32_to_bf16(acc[2 * e + 1]) << 16);
        st16<true>(dst, u32x4{u[0], u[1], u[2], u[3]});
        st16<true>(dst + 16, u32x4{u[4], u[5], u[6], u[7]});
    } else {
        uint32_t u[4];
        _Pragma("unroll") for (int e = 0; e < 4; e++)
            u[e] = f32x2_to_fp8x2(acc[4 * e] * f.out1_inv_scale, acc[4 * e + 1] * f.out1_inv_scale) |
                   (f32x2_to_fp8x2(acc[4 * e + 2] * f.out1_inv_scale, acc[4 * e + 3] * f.out1_inv_scale) << 16);
        st16<true>(dst, u32x4{u[0], u[1], u[2], u[3]});
    }
}

__device__ __forceinline__ int fused_stage_tiles(const FusedArgs& f, int s) {
    return s == 0 ? f.N1 / 32 : s <= f.n_layers ? f.layer[s - 1].N / 32 : 1;
}

template <int DOM, int PREC, int CLS>
__global__ __launch_bounds__(64) void fused_forward_kernel(FusedArgs f) {
    constexpr int HW = PREC == 0 ? 0 : 1;
    const int lane = threadIdx.x;
    const int n = max(0, min(f.n_dev ? *f.n_dev : f.n_host, f.m_cap));
    const int rbs = (n + 31) / 32;
    const int n_stages = f.n_layers + 2;
    int total = 0;
    for (int s = 0; s < n_stages; s++) total += rbs * fused_stage_tiles(f, s);
    int* const work = f.sync;
    int* const fin = f.sync + 1;
    int* const flag = f.sync + 2;
    int* const done = f.sync + 4;
    for (;;) {
        int item = 0;
        if (lane == 0) item = __hip_atomic_fetch_add(work, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        item = __shfl(item, 0, 64);
        if (item >= total) break;
        int s = 0, tiles = fused_stage_tiles(f, 0);
        while (item >= rbs * tiles) {
            item -= rbs * tiles;
            s++;
            tiles = fused_stage_tiles(f, s);
        }
        const int rb = item / tiles, t = item % tiles;
        if (s > 0) {
            // poll with device-coherent loads (no cache invalidation per poll)
            const int* const cnt = done + (s - 1) * f.rb_cap + rb;
            const int need = fused_stage_tiles(f, s - 1);
            int spins = 0;
            while (ld_coh(cnt) < need) {
                if (++spins > f.spin_limit) {
                    if (lane == 0) st_coh(flag, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // orders the loads below after the poll
        }
        if (s == 0) {
            gather_tile<DOM, PREC>(f, n, rb, t, lane);
        } else if (s <= f.n_layers) {
            small_tile<PREC, PREC, true>(f.layer[s - 1], rb * 32, t * 32, lane);
        } else if (CLS) {
            for (int r = rb * 32; r < min(rb * 32 + 32, n); r++) head_cls_row<PREC, HW, 32, true>(f.head, r, lane);
        } else {
            for (int i = 0; i < 8; i++)
                head_reg_row<PREC, HW, true>(f.head, n, rb * 32 + 4 * i + (lane >> 4), lane & 15);
        }
        if (s <= f.n_layers) {
            // every lane's coherent stores have completed before the tile is counted
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            wait_vmcnt<0>();
            if (lane == 0)
                __hip_atomic_fetch_add(done + s * f.rb_cap + rb, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // The last wave to finish clears the counters (every other wave has made
    // its last access to them, all coherent, before counting itself done).
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    wait_vmcnt<0>();
    int last = 0;
    if (lane == 0) last = __hip_atomic_fetch_add(fin, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (int)gridDim.x - 1;
    last = __shfl(last, 0, 64);
    if (!last) return;
    if (ld_coh(flag) != 0)
        for (int r = lane; r < n; r += 64) f.head.h_out[r] = -1;
    for (int s = 0; s < n_stages - 1; s++)
        for (int b = lane; b < rbs; b += 64) st_coh(done + s * f.rb_cap + b, 0);
    if (lane == 0) {
        st_coh(flag, 0);
        st_coh(fin, 0);
        st_coh(work, 0);
    }
}

// ------------------------------------------------------------ calibration
// Largest value of rows < n, columns < N of a float32 activation tensor,
// accumulated with an atomic max on the (non-negative) float bits.
__global__ void absmax_kernel(const float* __restrict__ x, int n, int N, int ld, unsigned* out) {
    float m = 0.f;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * N; i += gridDim.x * blockDim.x) {
        const int r = i / N, c = i % N;
        m = fmaxf(m, fabsf(x[(size_t)r * ld + c]));
    }
    for (int s = 32; s >= 1; s >>= 1) m = fmaxf(m, __shfl_xor(m, s, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// ------------------------------------------------------------ launchers
template <int DOM, int WT, int OUT>
static void launch_gather_t(const GatherLaunch& L, hipStream_t s) {
    const dim3 grid(L.N / GCOLS, (L.m_rows + GROWS - 1) / GROWS);
    const size_t lds = (size_t)L.t_rows * GCOLS * (WT == 0 ? 4 : 2);
    hipLaunchKernelGGL((gather_l1_kernel<DOM, WT, OUT>), grid, dim3(256), lds, s,
                       reinterpret_cast<const uint64_t*>(L.packed), L.n_dev, L.n_host, L.m_rows, L.table, L.t_rows,
                       L.bias, L.N, L.ld_out, L.out, L.out_inv_scale);
}

template <int DOM>
static bool launch_gather_d(const GatherLaunch& L, hipStream_t s) {
    if (L.table_f32) {
        if (L.prec == 0) launch_gather_t<DOM, 0, 0>(L, s);
        else if (L.prec == 1) launch_gather_t<DOM, 0, 1>(L, s);
        else launch_gather_t<DOM, 0, 2>(L, s);
    } else {
        if (L.prec == 1) launch_gather_t<DOM, 1, 1>(L, s);
        else if (L.prec == 2) launch_gather_t<DOM, 1, 2>(L, s);
        else return false;
    }
    return true;
}

bool launch_gather(const GatherLaunch& L, hipStream_t s) {
    switch (L.domain) {
        case 0: return launch_gather_d<0>(L, s);
        case 1: return launch_gather_d<1>(L, s);
        case 2: return launch_gather_d<2>(L, s);
    }
    return false;
}

// A GEMM launch; with the caller's timing events, the kernel's own start and
// end are recorded on them.
template <typename K>
static void launch_k(K kern, dim3 grid, dim3 block, size_t lds, hipStream_t s, const GemmLaunch& L, const GemmArgs& g) {
    if (L.ev_start && L.ev_stop)
        hipExtLaunchKernelGGL(kern, grid, block, (std::uint32_t)lds, s, L.ev_start, L.ev_stop, 0, g);
    else
        hipLaunchKernelGGL(kern, grid, block, lds, s, g);
}

template <int PREC, int OUTT, int BM, int BN>
static void launch_gemm_t(const GemmLaunch& L, hipStream_t s) {
    GemmArgs g;
    g.A = (const uint8_t*)L.A; g.Bt = (const uint8_t*)L.Bt; g.C = (uint8_t*)L.C; g.R = (const uint8_t*)L.R;
    g.Mk = (const uint8_t*)L.Mk;
    g.bias = L.bias; g.colscale = L.colscale; g.m_dev = L.m_dev; g.m_host = L.m_host;
    g.N = L.N; g.K = L.K; g.lda = L.lda; g.ldb = L.ldb; g.ldc = L.ldc;
    g.a_scale = L.a_scale; g.r_scale = L.r_scale; g.out_inv_scale = L.out_inv_scale; g.relu = L.relu;
    g.group_n = L.group_n; g.group_k = L.group_k;
    g.Ct = (uint8_t*)L.Ct; g.ldct = L.ldct; g.ct_rows = L.ct_rows;
    const int m_tiles = (L.m_cap + BM - 1) / BM;
    const int tiles = m_tiles * (L.N / BN);
    g.m_tiles_cap = m_tiles;
    int grid = tiles;
    g.persistent = 0;
    if (L.persistent_grid > 0 && L.persistent_grid < tiles) {
        grid = L.persistent_grid;
        g.persistent = 1;
        g.tile_ctr = L.tile_ctr;  // dynamic schedule when the caller supplies the counters
    }
    if (L.m_dev) g.persistent = 1;  // tile count known only on the device: stride over the cap
    const size_t lds = 2 * (size_t)(BM + BN) * 128;
    launch_k(gemm_kernel<PREC, OUTT, BM, BN>, dim3(grid), dim3(256), lds, s, L, g);
}

template <int PREC, int OUTT>
static void launch_gemm_small(const GemmLaunch& L, hipStream_t s) {
    GemmArgs g;
    g.A = (const uint8_t*)L.A; g.Bt = (const uint8_t*)L.Bt; g.C = (uint8_t*)L.C; g.R = (const uint8_t*)L.R;
    g.Mk = (const uint8_t*)L.Mk;
    g.bias = L.bias; g.colscale = L.colscale; g.m_dev = L.m_dev; g.m_host = L.m_host;
    g.N = L.N; g.K = L.K; g.lda = L.lda; g.ldb = L.ldb; g.ldc = L.ldc;
    g.a_scale = L.a_scale; g.r_scale = L.r_scale; g.out_inv_scale = L.out_inv_scale; g.relu = L.relu;
    g.group_n = L.group_n; g.group_k = L.group_k;
    g.Ct = (uint8_t*)L.Ct; g.ldct = L.ldct; g.ct_rows = L.ct_rows;
    g.m_tiles_cap = (L.m_cap + 31) / 32;
    g.persistent = 0;
    launch_k(gemm_small_kernel<PREC, OUTT>, dim3(g.m_tiles_cap * (L.N / 32)), dim3(64), 0, s, L, g);
}

template <int PREC, int OUTT, int BM, int BN, int NS>
static void launch_gemm_ring(const GemmLaunch& L, hipStream_t s) {
    GemmArgs g;
    g.A = (const uint8_t*)L.A; g.Bt = (const uint8_t*)L.Bt; g.C = (uint8_t*)L.C; g.R = (const uint8_t*)L.R;
    g.Mk = (const uint8_t*)L.Mk;
    g.bias = L.bias; g.colscale = L.colscale; g.m_dev = L.m_dev; g.m_host = L.m_host;
    g.N = L.N; g.K = L.K; g.lda = L.lda; g.ldb = L.ldb; g.ldc = L.ldc;
    g.a_scale = L.a_scale; g.r_scale = L.r_scale; g.out_inv_scale = L.out_inv_scale; g.relu = L.relu;
    g.group_n = L.group_n; g.group_k = L.group_k;
    g.Ct = (uint8_t*)L.Ct; g.ldct = L.ldct; g.ct_rows = L.ct_rows;
    const int m_tiles = (L.m_cap + BM - 1) / BM;
    const int tiles = m_tiles * (L.N / BN);
    g.m_tiles_cap = m_tiles;
    int grid = tiles;
    g.persistent = 0;
    if (L.persistent_grid > 0 && L.persistent_grid < tiles) { grid = L.persistent_grid; g.persistent = 1; }
    if (L.m_dev) g.persistent = 1;
    const size_t lds = (size_t)NS * (BM + BN) * 128;
    launch_k(gemm_ring_kernel<PREC, OUTT, BM, BN, NS>, dim3(grid), dim3(256), lds, s, L, g);
}

template <int PREC, int OUTT>
static void launch_gemm_w8(const GemmLaunch& L, hipStream_t s) {
    GemmArgs g;
    g.A = (const uint8_t*)L.A; g.Bt = (const uint8_t*)L.Bt; g.C = (uint8_t*)L.C; g.R = (const uint8_t*)L.R;
    g.Mk = (const uint8_t*)L.Mk;
    g.bias = L.bias; g.colscale = L.colscale; g.m_dev = L.m_dev; g.m_host = L.m_host;
    g.N = L.N; g.K = L.K; g.lda = L.lda; g.ldb = L.ldb; g.ldc = L.ldc;
    g.a_scale = L.a_scale; g.r_scale = L.r_scale; g.out_inv_scale = L.out_inv_scale; g.relu = L.relu;
    g.group_n = L.group_n; g.group_k = L.group_k;
    g.Ct = (uint8_t*)L.Ct; g.ldct = L.ldct; g.ct_rows = L.ct_rows;
    const int m_tiles = (L.m_cap + 255) / 256;
    const int tiles = m_tiles * (L.N / 128);
    g.m_tiles_cap = m_tiles;
    int grid = tiles;
    g.persistent = 0;
    if (L.persistent_grid > 0 && L.persistent_grid < tiles) { grid = L.persistent_grid; g.persistent = 1; }
    if (L.m_dev) g.persistent = 1;
    launch_k(gemm_w8_kernel<PREC, OUTT>, dim3(grid), dim3(512), (size_t)2 * (256 + 128) * 128, s, L, g);
}

template <int PREC, int OUTT, int NW, int NS, bool TC = false, int BN = 128>
static void launch_gemm_wide(const GemmLaunch& L, hipStream_t s) {
    GemmArgs g;
    g.A = (const uint8_t*)L.A; g.Bt = (const uint8_t*)L.Bt; g.C = (uint8_t*)L.C; g.R = (const uint8_t*)L.R;
    g.Mk = (const uint8_t*)L.Mk;
    g.bias = L.bias; g.colscale = L.colscale; g.m_dev = L.m_dev; g.m_host = L.m_host;
    g.N = L.N; g.K = L.K; g.lda = L.lda; g.ldb = L.ldb; g.ldc = L.ldc;
    g.a_scale = L.a_scale; g.r_scale = L.r_scale; g.out_inv_scale = L.out_inv_scale; g.relu = L.relu;
    g.group_n = L.group_n; g.group_k = L.group_k;
    g.Ct = (uint8_t*)L.Ct; g.ldct = L.ldct; g.ct_rows = L.ct_rows;
    g.split = L.split > 1 ? L.split : 1;
    g.c_split = L.c_split;
    const int m_tiles = (L.m_cap + 255) / 256;
    const int tiles = m_tiles * (L.N / BN) * g.split;
    g.m_tiles_cap = m_tiles;
    int grid = tiles;
    g.persistent = 0;
    if (L.persistent_grid > 0 && L.persistent_grid < tiles) {
        grid = L.persistent_grid;
        g.persistent = 1;
        g.tile_ctr = L.tile_ctr;
    }
    if (L.m_dev) g.persistent = 1;
    launch_k(gemm_wide_kernel<PREC, OUTT, NW, NS, TC, BN>, dim3(grid), dim3(NW * 64), (size_t)NS * (256 + BN) * 128, s,
             L, g);
}

// Tile ids: 0-3 LDS double buffer fed through registers (4 waves), 4 the
// small-batch kernel (one wave per 32 x 32 tile), 5-8 the LDS ring fed by
// direct loads, 9 the 8-wave 256 x 128 tile, 10-13 the fused persistent
// forward kernel (one-wave 32 x 32 tiles; 2, 4, 8 or 12 waves per compute
// unit), which replaces the whole forward pass rather than one layer;
// 14-16 the wide-block ring kernels (8 waves with a 2- or 3-stage ring, 16
// waves with a 2-stage ring); 17 and 18 persistent grids (one 8-wave wide
// block per compute unit, two 128x128 blocks per compute unit) taking tiles
// off an atomic counter when the caller supplies one; 19 the wide ring kernel
// on 256 x 256 tiles (8 waves of 64 x 128, a third fewer operand bytes per
// MFMA than 256 x 128: for large batches, where every compute unit gets
// several tiles).
int gemm_tile_count() { return 20; }
void gemm_tile_shape(int id, int* bm, int* bn) {
    static const int T[20][2] = {{128, 128}, {128, 256}, {64, 128}, {256, 128}, {32, 32},
                                 {256, 128}, {128, 128}, {128, 256}, {64, 128}, {256, 128},
                                 {32, 32}, {32, 32}, {32, 32}, {32, 32},
                                 {256, 128}, {256, 128}, {256, 128}, {256, 128}, {128, 128}, {256, 256}};
    *bm = T[id][0];
    *bn = T[id][1];
}

// Compute units of the current device (cached per device).
static int compute_units() {
    static int cu[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (!cu[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cu[dev] = n;
    }
    return cu[dev];
}

template <int PREC, int OUTT>
static bool launch_gemm_p(const GemmLaunch& L, hipStream_t s) {
    switch (L.tile) {
        case 0: launch_gemm_t<PREC, OUTT, 128, 128>(L, s); return true;
        case 1: launch_gemm_t<PREC, OUTT, 128, 256>(L, s); return true;
        case 2: launch_gemm_t<PREC, OUTT, 64, 128>(L, s); return true;
        case 3: launch_gemm_t<PREC, OUTT, 256, 128>(L, s); return true;
        case 4: case 10: case 11: case 12: case 13: launch_gemm_small<PREC, OUTT>(L, s); return true;
        case 5: launch_gemm_ring<PREC, OUTT, 256, 128, 3>(L, s); return true;
        case 6: launch_gemm_ring<PREC, OUTT, 128, 128, 3>(L, s); return true;
        case 7: launch_gemm_ring<PREC, OUTT, 128, 256, 3>(L, s); return true;
        case 8: launch_gemm_ring<PREC, OUTT, 64, 128, 4>(L, s); return true;
        case 9: launch_gemm_w8<PREC, OUTT>(L, s); return true;
        case 14:
            if (L.Ct) {
                if constexpr (OUTT != 2) launch_gemm_wide<PREC, OUTT, 8, 2, true>(L, s);
            } else {
                launch_gemm_wide<PREC, OUTT, 8, 2>(L, s);
            }
            return true;
        case 15: launch_gemm_wide<PREC, OUTT, 8, 3>(L, s); return true;
        case 16: launch_gemm_wide<PREC, OUTT, 16, 2>(L, s); return true;
        case 17: {
            GemmLaunch P = L;
            P.persistent_grid = compute_units();
            launch_gemm_wide<PREC, OUTT, 8, 2>(P, s);
            return true;
        }
        case 18: {
            GemmLaunch P = L;
            P.persistent_grid = 2 * compute_units();
            launch_gemm_t<PREC, OUTT, 128, 128>(P, s);
            return true;
        }
        case 19:
            if (L.N % 256) return false;
            launch_gemm_wide<PREC, OUTT, 8, 2, false, 256>(L, s);
            return true;
    }
    return false;
}

bool launch_gemm(const GemmLaunch& L, hipStream_t s) {
    const int out = L.out_type < 0 ? L.prec : L.out_type;
    if (L.split > 1) {  // split-K: wide tiles, whole 128-byte stages per slice, host row count
        const int eb = L.prec == 0 ? 4 : L.prec == 1 ? 2 : 1;
        if (L.tile < 14 || L.tile > 17 || L.K % L.split != 0 || (L.K / L.split) * eb % 128 != 0 || L.m_dev ||
            L.R || L.Mk)
            return false;
    }
    if (L.Ct) {  // transposed copy: tile 14, float32 or bf16 C, host row count, whole tiles below ldct
        if (L.tile != 14 || out == 2 || L.split > 1 || L.m_dev || L.persistent_grid > 0 || L.ldct % 8 ||
            L.ldct < (L.m_cap + 255) / 256 * 256)
            return false;
    }
    if (L.prec == 0 && out == 0) return launch_gemm_p<0, 0>(L, s);
    if (L.prec == 1 && out == 1) return launch_gemm_p<1, 1>(L, s);
    if (L.prec == 1 && out == 0) return launch_gemm_p<1, 0>(L, s);
    if (L.prec == 2 && out == 2) return launch_gemm_p<2, 2>(L, s);
    return false;
}

template <int IN, int HW>
static bool launch_head_t(HeadArgs H, int m_cap, hipStream_t s) {
    H.m_cap = m_cap;
    if (H.n_out == 1 && H.mode <= 2)
        hipLaunchKernelGGL((head_reg_kernel<IN, HW>), dim3((m_cap + 15) / 16), dim3(256), 0, s, H);
    else if (H.n_out <= 32)
        hipLaunchKernelGGL((head_cls_kernel<IN, HW, 32>), dim3((m_cap + 3) / 4), dim3(256), 0, s, H);
    else
        return false;
    return true;
}

bool launch_head(const HeadArgs& H, int prec, int m_cap, hipStream_t s) {
    if (prec == 0) return launch_head_t<0, 0>(H, m_cap, s);
    if (prec == 1) return launch_head_t<1, 1>(H, m_cap, s);
    return launch_head_t<2, 1>(H, m_cap, s);
}

static GemmArgs gemm_args_of(const GemmLaunch& L) {
    GemmArgs g;
    g.A = (const uint8_t*)L.A; g.Bt = (const uint8_t*)L.Bt; g.C = (uint8_t*)L.C; g.R = (const uint8_t*)L.R;
    g.Mk = (const uint8_t*)L.Mk;
    g.bias = L.bias; g.colscale = L.colscale; g.m_dev = L.m_dev; g.m_host = L.m_host;
    g.N = L.N; g.K = L.K; g.lda = L.lda; g.ldb = L.ldb; g.ldc = L.ldc;
    g.a_scale = L.a_scale; g.r_scale = L.r_scale; g.out_inv_scale = L.out_inv_scale; g.relu = L.relu;
    g.group_n = L.group_n; g.group_k = L.group_k;
    g.Ct = (uint8_t*)L.Ct; g.ldct = L.ldct; g.ct_rows = L.ct_rows;
    g.m_tiles_cap = (L.m_cap + 31) / 32;
    g.persistent = 0;
    return g;
}

int fused_max_layers() { return kFusedMaxLayers; }

template <int DOM, int PREC>
static void launch_fused_t(const FusedArgs& f, int cls, int grid, hipStream_t s) {
    if (cls) hipLaunchKernelGGL((fused_forward_kernel<DOM, PREC, 1>), dim3(grid), dim3(64), 0, s, f);
    else hipLaunchKernelGGL((fused_forward_kernel<DOM, PREC, 0>), dim3(grid), dim3(64), 0, s, f);
}

bool launch_fused(const FusedLaunch& L, hipStream_t s) {
    if constexpr (!kFusedEnabled) {
        (void)L;
        (void)s;
        return false;
    } else {
    if (L.n_layers < 1 || L.n_layers > kFusedMaxLayers || L.grid < 1 || L.head.n_out > 32) return false;
    const bool cls = !(L.head.n_out == 1 && L.head.mode <= 2);
    FusedArgs f;
    f.packed = reinterpret_cast<const uint64_t*>(L.packed);
    f.n_dev = L.n_dev;
    f.n_host = L.n_host;
    f.m_cap = L.m_cap;
    f.table = reinterpret_cast<const float*>(L.table);
    f.bias1 = L.bias1;
    f.N1 = L.N1;
    f.ld1 = L.ld1;
    f.out1 = reinterpret_cast<uint8_t*>(L.out1);
    f.out1_inv_scale = L.out1_inv_scale;
    f.n_layers = L.n_layers;
    f.sync = L.sync;
    f.rb_cap = L.rb_cap;
    f.spin_limit = L.spin_limit;
    f.head = L.head;
    f.head.m_cap = L.m_cap;
    for (int i = 0; i < L.n_layers; i++) {
        if (L.layers[i].N % 32 || L.layers[i].prec != L.prec) return false;
        f.layer[i] = gemm_args_of(L.layers[i]);
    }
    const int c = cls ? 1 : 0;
    switch (L.domain * 3 + L.prec) {
        case 0: launch_fused_t<0, 0>(f, c, L.grid, s); return true;
        case 1: launch_fused_t<0, 1>(f, c, L.grid, s); return true;
        case 2: launch_fused_t<0, 2>(f, c, L.grid, s); return true;
        case 3: launch_fused_t<1, 0>(f, c, L.grid, s); return true;
        case 4: launch_fused_t<1, 1>(f, c, L.grid, s); return true;
        case 5: launch_fused_t<1, 2>(f, c, L.grid, s); return true;
        case 6: launch_fused_t<2, 0>(f, c, L.grid, s); return true;
        case 7: launch_fused_t<2, 1>(f, c, L.grid, s); return true;
        case 8: launch_fused_t<2, 2>(f, c, L.grid, s); return true;
    }
    return false;
    }
}

bool fused_enabled() { return kFusedEnabled; }

template <int PREC, int OUTT, int BM, int BN>
static hipError_t set_lds_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_kernel<PREC, OUTT, BM, BN>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 2 * (BM + BN) * 128);
}

template <int PREC, int OUTT, int BM, int BN, int NS>
static hipError_t set_ring_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_ring_kernel<PREC, OUTT, BM, BN, NS>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, NS * (BM + BN) * 128);
}

template <int PREC, int OUTT, int NW, int NS>
static hipError_t set_wide_attr() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_wide_kernel<PREC, OUTT, NW, NS>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, NS * (256 + 128) * 128);
    if constexpr (OUTT != 2 && NW == 8 && NS == 2)
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_wide_kernel<PREC, OUTT, NW, NS, true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, NS * (256 + 128) * 128);
    return e;
}

template <int PREC, int OUTT>
static hipError_t set_lds_attr_p() {
    hipError_t e = set_lds_attr<PREC, OUTT, 128, 128>();
    if (e == hipSuccess) e = set_lds_attr<PREC, OUTT, 128, 256>();
    if (e == hipSuccess) e = set_lds_attr<PREC, OUTT, 64, 128>();
    if (e == hipSuccess) e = set_lds_attr<PREC, OUTT, 256, 128>();
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_w8_kernel<PREC, OUTT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 2 * (256 + 128) * 128);

    if (e == hipSuccess) e = set_ring_attr<PREC, OUTT, 256, 128, 3>();
    if (e == hipSuccess) e = set_ring_attr<PREC, OUTT, 128, 128, 3>();
    if (e == hipSuccess) e = set_ring_attr<PREC, OUTT, 128, 256, 3>();
    if (e == hipSuccess) e = set_ring_attr<PREC, OUTT, 64, 128, 4>();
    if (e == hipSuccess) e = set_wide_attr<PREC, OUTT, 8, 2>();
    if (e == hipSuccess) e = set_wide_attr<PREC, OUTT, 8, 3>();
    if (e == hipSuccess) e = set_wide_attr<PREC, OUTT, 16, 2>();
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_wide_kernel<PREC, OUTT, 8, 2, false, 256>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 2 * (256 + 256) * 128);
    return e;
}

template <int DOM, int WT, int OUT>
static hipError_t set_gather_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&gather_l1_kernel<DOM, WT, OUT>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 288 * GCOLS * 4);
}

template <int DOM>
static hipError_t set_gather_attr_d() {
    hipError_t e = set_gather_attr<DOM, 0, 0>();
    if (e == hipSuccess) e = set_gather_attr<DOM, 0, 1>();
    if (e == hipSuccess) e = set_gather_attr<DOM, 0, 2>();
    if (e == hipSuccess) e = set_gather_attr<DOM, 1, 1>();
    if (e == hipSuccess) e = set_gather_attr<DOM, 1, 2>();
    return e;
}

// Kernels whose blocks may use more than 64 KiB of LDS (gfx950 has 160 KiB).
hipError_t gemm_prepare_attributes() {
    hipError_t e = set_gather_attr_d<0>();
    if (e == hipSuccess) e = set_gather_attr_d<1>();
    if (e == hipSuccess) e = set_gather_attr_d<2>();
    if (e == hipSuccess) e = set_lds_attr_p<0, 0>();
    if (e == hipSuccess) e = set_lds_attr_p<1, 1>();
    if (e == hipSuccess) e = set_lds_attr_p<1, 0>();
    if (e == hipSuccess) e = set_lds_attr_p<2, 2>();
    return e;
}

void launch_absmax(const float* x, int n, int N, int ld, unsigned* out, hipStream_t s) {
    int blocks = (int)((int64_t)n * N / 256 + 1);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(absmax_kernel, dim3(blocks), dim3(256), 0, s, x, n, N, ld, out);
}

}  // namespace hb
