// On-GPU training of a sliding-tile regression network (hb_trainer, include/hb.h).
//
// Step: forward with every activation saved (the products' epilogues also
// write each activation transposed, the operand layout of the weight
// gradients); head kernel (loss, dL/dy, output-layer gradient); backward
// through residual blocks and dense layers with input-gradient GEMMs (fused
// ReLU mask and residual add, transposed copy) and weight-gradient GEMMs
// (FP32 output; bias gradients as row sums of the transposed gradients);
// layer-1 gradient by scatter-add; Adam on FP32 master weights, re-casting
// the working copies.
#include <algorithm>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <fstream>
#include <memory>
#include <vector>

#include "common.hpp"
#include "hb.h"
#include "kernels.hpp"
#include "model.hpp"
#include "train.hpp"

namespace hb {
namespace {

constexpr int kScatterChunks = 32;  // state chunks of the layer-1 scatter (its blocks: chunks x N1 / 128)
constexpr int kSplitMax = 8;       // K slices of a split-K weight gradient

struct TLayer {
    int K, N, K_pad, N_pad;
    float *master, *m, *v;     // K*N
    float *bias, *bm, *bv;     // N_pad (the working bias is the master)
    void* Wt;                  // [N_pad][K_pad] forward operand
    void* Wkn;                 // [K_pad][N_pad] input-gradient operand
    float* dW;                 // [K_pad][N_pad]
    float* db;                 // [N_pad]
    // K < K_pad: row K of the input's transposed copy is all ones, so row K of
    // dW is the bias gradient (dbp points there); else dbp = db, a row sum
    bool ones = false;
    float* dbp = nullptr;
    int in_act, out_act, res_act;
};

uint16_t host_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace
}  // namespace hb

struct hb_trainer {
    int device = 0;
    hb_train_opts o{};
    hb::NetSpec spec;
    int t = 1, eb = 2;
    int side = 4, P = 16, S = 16, rows1 = 256;  // rows1: layer-1 weight rows in the file (cube: 54 x 6)
    int dom = 1, trows = 256;                    // trows: gathered table rows (cube: 48 x 6, centres folded)
    float* l1_bias_work = nullptr;               // cube: bias + the six centre rows (the gather's bias)
    float* partial = nullptr;                    // layer-1 scatter: per-chunk partial sums
    float* wsplit = nullptr;                     // split-K weight-gradient partials (BF16 training)
    int64_t wsplit_elems = 0;
    float* head_part = nullptr;                  // output layer: per-block partial gradients and loss
    float* colpart = nullptr;                    // bias gradients: per-row-block column sums
    hb::AdamTensor* d_adam = nullptr;            // every parameter tensor's Adam descriptor (device)
    int n_adam = 0;
    int N1 = 0, N1_pad = 0, H = 0, H_pad = 0, M_pad = 0, W_pad = 0;
    float *l1_master = nullptr, *l1_m = nullptr, *l1_v = nullptr;
    void* l1_table = nullptr;
    float *l1_bias = nullptr, *l1_bm = nullptr, *l1_bv = nullptr;
    float *dW1 = nullptr, *db1 = nullptr;
    float *ho_master = nullptr, *ho_m = nullptr, *ho_v = nullptr;
    void* ho_W = nullptr;
    float *ho_b = nullptr, *ho_bm = nullptr, *ho_bv = nullptr;
    float *dWo = nullptr, *dbo = nullptr;
    std::vector<hb::TLayer> L;
    int n_act = 0;
    std::vector<void*> act;
    void *G = nullptr, *G2 = nullptr, *GT = nullptr, *GT2 = nullptr;
    // transposed activations ([W_pad][M_pad]) for the weight-gradient products:
    // written by the forward products' epilogues (act 0 by a transpose); null
    // for activations no layer reads
    std::vector<void*> actT;

    // releases every device allocation (also when creation fails part way)
    ~hb_trainer() {
        (void)hipSetDevice(device);
        (void)hipDeviceSynchronize();
        for (void* p : allocs) (void)hipFree(p);
    }
    float* d_loss = nullptr;
    int step = 0;
    std::vector<void*> allocs;
};

namespace hb {
namespace {

hb_status dalloc(hb_trainer* tr, size_t bytes, void** p) {
    if (hipMalloc(p, bytes ? bytes : 4) != hipSuccess) return fail(HB_E_NOMEM, "hipMalloc of %zu bytes", bytes);
    tr->allocs.push_back(*p);
    HB_HIP(hipMemset(*p, 0, bytes ? bytes : 4));
    return HB_OK;
}

template <class T>
hb_status dalloc_t(hb_trainer* tr, size_t count, T** p) {
    void* q = nullptr;
    hb_status st = dalloc(tr, count * sizeof(T), &q);
    *p = (T*)q;
    return st;
}

// Upload a float32 host array and return device pointer.
hb_status up_f32(hb_trainer* tr, const std::vector<float>& h, float** d) {
    hb_status st = dalloc_t(tr, h.size(), d);
    if (st != HB_OK) return st;
    HB_HIP(hipMemcpy(*d, h.data(), h.size() * 4, hipMemcpyHostToDevice));
    return HB_OK;
}

// Upload a working copy (fp32 or bf16) of `vals` (float32, already padded).
hb_status up_work(hb_trainer* tr, const std::vector<float>& vals, void** d) {
    hb_status st = dalloc(tr, vals.size() * tr->eb, d);
    if (st != HB_OK) return st;
    if (tr->eb == 4) {
        HB_HIP(hipMemcpy(*d, vals.data(), vals.size() * 4, hipMemcpyHostToDevice));
    } else {
        std::vector<uint16_t> b(vals.size());
        for (size_t i = 0; i < vals.size(); i++) b[i] = host_bf16(vals[i]);
        HB_HIP(hipMemcpy(*d, b.data(), b.size() * 2, hipMemcpyHostToDevice));
    }
    return HB_OK;
}

hb_status gemm(hb_trainer* tr, const void* A, int lda, const void* Bt, int ldb, void* C, int ldc, const void* R,
               const void* Mk, const float* bias, int M, int N, int K, int relu, int out_type, hipStream_t s,
               void* Ct = nullptr, int ct_rows = 0) {
    GemmLaunch g{};
    g.prec = tr->t;
    g.out_type = out_type;
    g.A = A; g.Bt = Bt; g.C = C; g.R = R; g.Mk = Mk; g.bias = bias;
    g.m_host = M; g.m_cap = M;
    g.N = N; g.K = K; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.a_scale = g.r_scale = g.out_inv_scale = 1.f;
    g.relu = relu;
    g.Ct = Ct;  // transposed copy of C (rows below M_pad), its first ct_rows rows
    g.ldct = tr->M_pad;
    g.ct_rows = ct_rows;
    // Forward and input-gradient products: the 8-wave 256x128 ring tile (the
    // one that writes a transposed copy), or 64x128 for small batches without
    // one.  Weight gradients (K, the batch, far longer than
    // M and N): FP32 takes the one-wave 32x32 tile (8x the tiles of 64x128 on a
    // 1000 x 1000 output; 12% faster per FP32 step), BF16 the 64x128 tile with a
    // 4-stage LDS ring (more of the long K in flight; 8% faster per BF16 step).
    const bool wgrad = out_type == 0 && K >= 4 * std::max(M, N);  // (the weight-gradient calls ask for FP32 C)
    g.tile = wgrad ? (tr->t == 0 ? 4 : 8) : (Ct || (N % 128 == 0 && M >= 2048)) ? 14 : 2;  // (a transposed copy: tile 14)
    // BF16 weight gradients of wide layers: split-K on the 256x128 tile (the
    // 1000 x 1000 output alone is 32 such tiles), partial products in wsplit,
    // then summed in slice order (deterministic).
    int split = 0;
    if (wgrad && tr->t == 1 && tr->wsplit && M % 256 == 0 && N % 128 == 0 && out_type == 0 && !R && !Mk &&
        (int64_t)M * N <= tr->wsplit_elems / kSplitMax) {
        for (int sp = kSplitMax; sp >= 2; sp /= 2)
            if (K % (sp * 64) == 0 && (M / 256) * (N / 128) * sp <= 512) { split = sp; break; }
    }
    if (split) {
        g.tile = 14;
        g.split = split;
        g.C = tr->wsplit;
        g.ldc = N;
        g.c_split = (int64_t)M * N;
        g.bias = nullptr;
    }
    if (!launch_gemm(g, s)) return fail(HB_E_UNSUPPORTED, "no GEMM for this precision");
    HB_HIP(hipGetLastError());
    if (split) {
        launch_splitk_sum(tr->wsplit, split, (int64_t)M * N, M, N, N, static_cast<float*>(C), ldc, s);
        HB_HIP(hipGetLastError());
    }
    return HB_OK;
}

hb_status transpose(hb_trainer* tr, const void* in, int ld_in, void* out, int ld_out, int R, int C, float* colsum,
                    int rows_sum, hipStream_t s) {
    TransposeArgs a{in, ld_in, out, ld_out, R, C, colsum, rows_sum, colsum ? tr->colpart : nullptr};
    launch_transpose(a, tr->t, s);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

// Forward (activations saved) + backward; gradients left in the grad buffers.
hb_status fwd_bwd(hb_trainer* tr, const uint8_t* d_packed, const float* d_labels, int n, hipStream_t s) {
    const int Me = (int)round_up(n, 128);
    const int t = tr->t;
    // every gradient buffer is written (not accumulated) by a fixed-order reduction
    // forward
    GatherLaunch G{};
    G.domain = tr->spec.domain;
    G.prec = t;
    G.packed = d_packed;
    G.n_host = n;
    G.m_rows = Me;
    G.table = tr->l1_table;
    G.table_f32 = t == 0;
    G.t_rows = tr->trows;
    G.bias = tr->dom == 2 ? tr->l1_bias_work : tr->l1_bias;
    G.N = tr->N1_pad;
    G.ld_out = tr->W_pad;
    G.out = tr->act[0];
    G.out_inv_scale = 1.f;
    if (!launch_gather(G, s)) return fail(HB_E_UNSUPPORTED, "layer-1 kernel");
    HB_HIP(hipGetLastError());
    hb_status st;
    for (auto& l : tr->L) {
        st = gemm(tr, tr->act[l.in_act], tr->W_pad, l.Wt, l.K_pad, tr->act[l.out_act], tr->W_pad,
                  l.res_act >= 0 ? tr->act[l.res_act] : nullptr, nullptr, l.bias, Me, l.N_pad, l.K_pad, 1, -1, s,
                  tr->actT[l.out_act], l.N);  // (its padding rows keep their zeros or ones)
        if (st != HB_OK) return st;
    }
    HeadTrainArgs h{};
    h.X = tr->act[tr->n_act - 1];
    h.ldx = tr->W_pad;
    h.K = tr->H_pad;
    h.W = tr->ho_W;
    h.b = tr->ho_b;
    h.labels = d_labels;
    h.n = n;
    h.m_pad = Me;
    h.inv_n = 1.f / (float)n;
    h.asym = tr->o.asym;
    h.alpha = tr->o.alpha;
    h.delta = tr->G;
    h.part = tr->head_part;
    h.dWo = tr->dWo;
    h.dbo_loss = tr->dbo;  // dbo, then the loss
    if (!launch_head_train(h, t, s)) return fail(HB_E_UNSUPPORTED, "head width");
    HB_HIP(hipGetLastError());
    // backward: cur holds the gradient at the pre-activation of the current layer
    // output, curT its transpose ([N][M_pad], the weight-gradient operand).  The
    // input-gradient products write both; the head's gradient is transposed
    // here, its column sums giving the last layer's bias gradient.
    const int ldT = tr->M_pad;
    if ((st = transpose(tr, tr->act[0], tr->W_pad, tr->actT[0], ldT, Me, tr->L[0].K, nullptr, 0, s)) != HB_OK)
        return st;
    void* cur = tr->G;
    void* other = tr->G2;
    void* curT = tr->GT;
    void* otherT = tr->GT2;
    if ((st = transpose(tr, cur, tr->W_pad, curT, ldT, Me, tr->L.back().N_pad, tr->L.back().ones ? nullptr : tr->L.back().db,
                        n, s)) != HB_OK)
        return st;
    bool db_done = true;
    for (int j = (int)tr->L.size() - 1; j >= 0; j--) {
        TLayer& l = tr->L[j];
        const bool res_b = l.res_act >= 0;
        // weight and bias gradient: dW = X^T cur, db = column sums of cur
        if (!db_done && !l.ones) {
            launch_row_sum(curT, ldT, l.N_pad, n, l.db, t, s);
            HB_HIP(hipGetLastError());
        }
        db_done = false;
        if ((st = gemm(tr, tr->actT[l.in_act], ldT, curT, ldT, l.dW, l.N_pad, nullptr, nullptr, nullptr, l.K_pad, l.N_pad, Me,
                       0, 0, s)) != HB_OK)
            return st;
        // input gradient, masked by the input activation (post-ReLU, so > 0 marks the active units)
        if (res_b) {
            // t-gradient of a residual block: (cur W_b^T) * [t > 0]; keep cur for the identity path
            if ((st = gemm(tr, cur, tr->W_pad, l.Wkn, l.N_pad, other, tr->W_pad, nullptr, tr->act[l.in_act], nullptr, Me,
                           l.K_pad, l.N_pad, 0, -1, s, otherT)) != HB_OK)
                return st;
            TLayer& la = tr->L[j - 1];
            if (!la.ones) {
                launch_row_sum(otherT, ldT, la.N_pad, n, la.db, t, s);
                HB_HIP(hipGetLastError());
            }
            if ((st = gemm(tr, tr->actT[la.in_act], ldT, otherT, ldT, la.dW, la.N_pad, nullptr, nullptr, nullptr, la.K_pad,
                           la.N_pad, Me, 0, 0, s)) != HB_OK)
                return st;
            // x-gradient: (t-grad W_a^T + cur) * [x_in > 0], written over cur (and its transpose when a layer is below)
            if ((st = gemm(tr, other, tr->W_pad, la.Wkn, la.N_pad, cur, tr->W_pad, cur, tr->act[la.in_act], nullptr, Me,
                           la.K_pad, la.N_pad, 0, -1, s, j - 1 > 0 ? curT : nullptr)) != HB_OK)
                return st;
            j--;  // the block's first layer is done
        } else {
            if ((st = gemm(tr, cur, tr->W_pad, l.Wkn, l.N_pad, other, tr->W_pad, nullptr, tr->act[l.in_act], nullptr, Me,
                           l.K_pad, l.N_pad, 0, -1, s, j > 0 ? otherT : nullptr)) != HB_OK)
                return st;
            std::swap(cur, other);
            std::swap(curT, otherT);
        }
    }
    ScatterArgs sa{};
    sa.dz = cur;
    sa.ld = tr->W_pad;
    sa.packed = d_packed;
    sa.n = n;
    sa.N1 = tr->N1_pad;
    sa.partial = tr->partial;
    sa.chunk = (n + kScatterChunks - 1) / kScatterChunks;
    sa.dW1 = tr->dW1;
    sa.ld_w = tr->N1_pad;
    sa.db1 = tr->db1;
    if (!launch_scatter_l1(sa, t, tr->dom, (n + sa.chunk - 1) / sa.chunk, s))
        return fail(HB_E_UNSUPPORTED, "layer-1 gradient");
    HB_HIP(hipGetLastError());
    return HB_OK;
}

AdamTensor adam_tensor(float* master, float* m, float* v, const float* grad, int64_t gk, int64_t gn, int K, int N,
                       void* out1, int64_t s1k, int64_t s1n, void* out2, int64_t s2k, int64_t s2n) {
    return AdamTensor{master, m, v, grad, gk, gn, K, N, out1, s1k, s1n, out2, s2k, s2n};
}

// The descriptors of every parameter tensor (fixed at creation): master
// weights, moments, gradient, and the working copies Adam rewrites.  The
// cube's layer-1 table and bias are rebuilt from the masters after the step.
hb_status upload_adam_table(hb_trainer* tr) {
    std::vector<AdamTensor> ts;
    const bool cube = tr->dom == 2;
    ts.push_back(adam_tensor(tr->l1_master, tr->l1_m, tr->l1_v, tr->dW1, tr->N1_pad, 1, tr->rows1, tr->N1,
                             cube ? nullptr : tr->l1_table, tr->N1_pad, 1, nullptr, 0, 0));
    ts.push_back(adam_tensor(tr->l1_bias, tr->l1_bm, tr->l1_bv, tr->db1, 0, 1, 1, tr->N1, nullptr, 0, 0, nullptr, 0, 0));
    for (auto& l : tr->L) {
        ts.push_back(adam_tensor(l.master, l.m, l.v, l.dW, l.N_pad, 1, l.K, l.N, l.Wt, 1, l.K_pad, l.Wkn, l.N_pad, 1));
        ts.push_back(adam_tensor(l.bias, l.bm, l.bv, l.dbp, 0, 1, 1, l.N, nullptr, 0, 0, nullptr, 0, 0));
    }
    ts.push_back(adam_tensor(tr->ho_master, tr->ho_m, tr->ho_v, tr->dWo, 1, 0, tr->H, 1, tr->ho_W, 1, 0, nullptr, 0, 0));
    ts.push_back(adam_tensor(tr->ho_b, tr->ho_bm, tr->ho_bv, tr->dbo, 0, 1, 1, 1, nullptr, 0, 0, nullptr, 0, 0));
    void* d = nullptr;
    hb_status st = dalloc(tr, ts.size() * sizeof(AdamTensor), &d);
    if (st != HB_OK) return st;
    HB_HIP(hipMemcpy(d, ts.data(), ts.size() * sizeof(AdamTensor), hipMemcpyHostToDevice));
    tr->d_adam = static_cast<AdamTensor*>(d);
    tr->n_adam = (int)ts.size();
    return HB_OK;
}

void apply_adam(hb_trainer* tr, hipStream_t s) {
    tr->step++;
    const float c1 = 1.f - std::pow(tr->o.beta1, (float)tr->step);
    const float c2 = 1.f - std::pow(tr->o.beta2, (float)tr->step);
    launch_multi_adam(tr->d_adam, tr->n_adam, tr->o.lr, tr->o.beta1, tr->o.beta2, tr->o.eps, c1, c2, tr->t, s);
    if (tr->dom == 2)
        launch_cube_fold(tr->l1_master, tr->l1_bias, tr->N1, tr->N1_pad, tr->l1_table, tr->l1_bias_work, tr->t, s);
}

// Copy rows x cols floats from a padded device array (row stride ld) to dst.
hb_status copy2d(float* dst, const float* src, int rows, int cols, int ld, hipStream_t s) {
    HB_HIP(hipMemcpy2DAsync(dst, (size_t)cols * 4, src, (size_t)ld * 4, (size_t)cols * 4, rows, hipMemcpyDeviceToDevice, s));
    return HB_OK;
}

hb_status check_batch(hb_trainer* tr, const uint8_t* d_packed, const float* d_labels, int64_t n) {
    if (!d_packed || !d_labels) return fail(HB_E_INVAL, "null device buffer");
    if (n < 1 || n > tr->o.max_batch) return fail(HB_E_INVAL, "n must be in 1..%d", tr->o.max_batch);
    return HB_OK;
}

}  // namespace
}  // namespace hb

using namespace hb;

extern "C" {

hb_status hb_trainer_create(const char* path, const hb_train_opts* opts, hb_trainer** out) {
    if (!path || !out) return fail(HB_E_INVAL, "null argument");
    hb_train_opts o{HB_BF16, 0, 8192, 1e-3f, 0.9f, 0.999f, 1e-8f, 0, 4.f};
    if (opts) o = *opts;
    if (o.prec != HB_BF16 && o.prec != HB_FP32) return fail(HB_E_UNSUPPORTED, "training runs in BF16 or FP32");
    if (o.max_batch < 1 || o.max_batch > (1 << 20)) return fail(HB_E_INVAL, "max_batch out of range");
    NetSpec spec;
    const char* why = "";
    if (!read_weight_file(path, &spec, &why)) return fail(HB_E_INVAL, "%s: %s", path, why);
    if (spec.head_kind != 0 || spec.n_out != 1) return fail(HB_E_UNSUPPORTED, "training needs a regression head");
    for (int d : spec.dims)
        if (d > 1024) return fail(HB_E_UNSUPPORTED, "hidden widths above 1024 are not supported in training");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(HB_E_DEVICE, "no HIP device available");
    if (o.device < 0 || o.device >= ndev) return fail(HB_E_INVAL, "device out of range");
    HB_HIP(hipSetDevice(o.device));
    static bool attrs = false;
    if (!attrs) {
        HB_HIP(gemm_prepare_attributes());
        HB_HIP(train_prepare_attributes());
        attrs = true;
    }
    auto tr = std::make_unique<hb_trainer>();
    hb_trainer* T = tr.get();
    T->device = o.device;
    T->o = o;
    T->spec = spec;
    T->t = o.prec == HB_FP32 ? 0 : 1;
    T->eb = o.prec == HB_FP32 ? 4 : 2;
    T->dom = spec.domain;
    T->side = spec.domain == 0 ? 3 : 4;
    T->P = spec.domain == 2 ? 54 : T->side * T->side;
    T->S = spec.domain == 2 ? 6 : T->side * T->side;
    T->rows1 = T->P * T->S;
    T->trows = scatter_table_rows(spec.domain);
    auto pad = [](int v) { return (int)round_up(v, 128); };
    T->N1 = spec.dims[0];
    T->N1_pad = pad(T->N1);
    T->H = spec.dims.back();
    T->H_pad = pad(T->H);
    T->M_pad = (int)round_up(o.max_batch, 256);  // whole 256-row GEMM tiles
    int wmax = T->N1_pad;
    for (int d : spec.dims) wmax = std::max(wmax, pad(d));
    T->W_pad = wmax;
    const auto& TS = spec.tensors;
    hb_status st;
    // layer 1
    if ((st = up_f32(T, TS[0], &T->l1_master)) != HB_OK) return st;
    if ((st = dalloc_t(T, TS[0].size(), &T->l1_m)) != HB_OK || (st = dalloc_t(T, TS[0].size(), &T->l1_v)) != HB_OK) return st;
    {
        std::vector<float> b(T->N1_pad, 0.f);
        for (int j = 0; j < T->N1; j++) b[j] = TS[1][j];
        if ((st = up_f32(T, b, &T->l1_bias)) != HB_OK) return st;
        if (T->dom == 2) {
            // the working table and folded bias are built from the masters on the device
            if ((st = dalloc(T, (size_t)T->trows * T->N1_pad * T->eb, &T->l1_table)) != HB_OK) return st;
            if ((st = dalloc_t(T, T->N1_pad, &T->l1_bias_work)) != HB_OK) return st;
            launch_cube_fold(T->l1_master, T->l1_bias, T->N1, T->N1_pad, T->l1_table, T->l1_bias_work, T->t, nullptr);
            HB_HIP(hipGetLastError());
            HB_HIP(hipDeviceSynchronize());
        } else {
            std::vector<float> tab((size_t)T->rows1 * T->N1_pad, 0.f);
            for (int r = 0; r < T->rows1; r++)
                for (int j = 0; j < T->N1; j++) tab[(size_t)r * T->N1_pad + j] = TS[0][(size_t)r * T->N1 + j];
            if ((st = up_work(T, tab, &T->l1_table)) != HB_OK) return st;
        }
    }
    if ((st = dalloc_t(T, T->N1_pad, &T->l1_bm)) != HB_OK || (st = dalloc_t(T, T->N1_pad, &T->l1_bv)) != HB_OK) return st;
    if ((st = dalloc_t(T, (size_t)T->rows1 * T->N1_pad, &T->dW1)) != HB_OK || (st = dalloc_t(T, T->N1_pad, &T->db1)) != HB_OK)
        return st;
    // matrix layers
    const int nd = (int)spec.dims.size();
    T->n_act = nd + 2 * spec.n_res;
    int ti = 2;
    auto add = [&](int K, int N, int in_act, int out_act, int res_act) -> hb_status {
        TLayer l{};
        l.K = K; l.N = N; l.K_pad = pad(K); l.N_pad = pad(N);
        l.in_act = in_act; l.out_act = out_act; l.res_act = res_act;
        hb_status s2;
        if ((s2 = up_f32(T, TS[ti], &l.master)) != HB_OK) return s2;
        if ((s2 = dalloc_t(T, TS[ti].size(), &l.m)) != HB_OK || (s2 = dalloc_t(T, TS[ti].size(), &l.v)) != HB_OK) return s2;
        std::vector<float> b(l.N_pad, 0.f);
        for (int j = 0; j < N; j++) b[j] = TS[ti + 1][j];
        if ((s2 = up_f32(T, b, &l.bias)) != HB_OK) return s2;
        if ((s2 = dalloc_t(T, l.N_pad, &l.bm)) != HB_OK || (s2 = dalloc_t(T, l.N_pad, &l.bv)) != HB_OK) return s2;
        std::vector<float> wt((size_t)l.N_pad * l.K_pad, 0.f), wkn((size_t)l.K_pad * l.N_pad, 0.f);
        for (int k = 0; k < K; k++)
            for (int n = 0; n < N; n++) {
                wt[(size_t)n * l.K_pad + k] = TS[ti][(size_t)k * N + n];
                wkn[(size_t)k * l.N_pad + n] = TS[ti][(size_t)k * N + n];
            }
        if ((s2 = up_work(T, wt, &l.Wt)) != HB_OK || (s2 = up_work(T, wkn, &l.Wkn)) != HB_OK) return s2;
        if ((s2 = dalloc_t(T, (size_t)l.K_pad * l.N_pad, &l.dW)) != HB_OK || (s2 = dalloc_t(T, l.N_pad, &l.db)) != HB_OK) return s2;
        T->L.push_back(l);
        ti += 2;
        return HB_OK;
    };
    for (int i = 1; i < nd; i++)
        if ((st = add(spec.dims[i - 1], spec.dims[i], i - 1, i, -1)) != HB_OK) return st;
    int x_act = nd - 1;
    for (int r = 0; r < spec.n_res; r++) {
        if ((st = add(T->H, T->H, x_act, nd + 2 * r, -1)) != HB_OK) return st;
        if ((st = add(T->H, T->H, nd + 2 * r, nd + 2 * r + 1, x_act)) != HB_OK) return st;
        x_act = nd + 2 * r + 1;
    }
    // head
    if ((st = up_f32(T, TS[ti], &T->ho_master)) != HB_OK) return st;
    if ((st = dalloc_t(T, T->H, &T->ho_m)) != HB_OK || (st = dalloc_t(T, T->H, &T->ho_v)) != HB_OK) return st;
    {
        std::vector<float> hw(T->H_pad, 0.f);
        for (int k = 0; k < T->H; k++) hw[k] = TS[ti][k];
        if ((st = up_work(T, hw, &T->ho_W)) != HB_OK) return st;
    }
    if ((st = up_f32(T, TS[ti + 1], &T->ho_b)) != HB_OK) return st;
    if ((st = dalloc_t(T, 1, &T->ho_bm)) != HB_OK || (st = dalloc_t(T, 1, &T->ho_bv)) != HB_OK) return st;
    // dWo [H_pad], then dbo and the loss: one column-sum launch writes all three
    if ((st = dalloc_t(T, (size_t)T->H_pad + 2, &T->dWo)) != HB_OK) return st;
    T->dbo = T->dWo + T->H_pad;
    T->d_loss = T->dbo + 1;
    if ((st = dalloc_t(T, (size_t)head_train_blocks(T->M_pad) * (T->H_pad + 2), &T->head_part)) != HB_OK) return st;
    // activations and scratch
    const size_t abytes = (size_t)T->M_pad * T->W_pad * T->eb;
    T->act.resize(T->n_act);
    for (int a = 0; a < T->n_act; a++)
        if ((st = dalloc(T, abytes, &T->act[a])) != HB_OK) return st;
    if ((st = dalloc(T, abytes, &T->G)) != HB_OK || (st = dalloc(T, abytes, &T->G2)) != HB_OK ||
        (st = dalloc(T, abytes, &T->GT)) != HB_OK || (st = dalloc(T, abytes, &T->GT2)) != HB_OK)
        return st;
    T->actT.assign(T->n_act, nullptr);
    for (auto& l : T->L) {
        if (!T->actT[l.in_act] && (st = dalloc(T, abytes, &T->actT[l.in_act])) != HB_OK) return st;
        l.ones = l.K < l.K_pad;
        l.dbp = l.ones ? l.dW + (size_t)l.K * l.N_pad : l.db;
        if (l.ones) {  // row K of the input's transposed copy: ones (no writer touches rows >= K)
            std::vector<uint8_t> row((size_t)T->M_pad * T->eb);
            for (int b = 0; b < T->M_pad; b++) {
                if (T->eb == 4) {
                    const float one = 1.f;
                    std::memcpy(&row[(size_t)b * 4], &one, 4);
                } else {
                    const uint16_t one = host_bf16(1.f);
                    std::memcpy(&row[(size_t)b * 2], &one, 2);
                }
            }
            HB_HIP(hipMemcpy(static_cast<uint8_t*>(T->actT[l.in_act]) + (size_t)l.K * T->M_pad * T->eb, row.data(),
                             row.size(), hipMemcpyHostToDevice));
        }
    }
    if ((st = dalloc_t(T, (size_t)(T->M_pad / 64 + 1) * T->W_pad, &T->colpart)) != HB_OK) return st;
    if ((st = dalloc_t(T, (size_t)kScatterChunks * (T->trows + 1) * T->N1_pad, &T->partial)) != HB_OK) return st;
    if (T->t == 1) {
        T->wsplit_elems = (int64_t)kSplitMax * round_up(T->W_pad, 256) * T->W_pad;
        if ((st = dalloc_t(T, (size_t)T->wsplit_elems, &T->wsplit)) != HB_OK) return st;
    }
    if ((st = upload_adam_table(T)) != HB_OK) return st;
    *out = tr.release();
    return HB_OK;
}

void hb_trainer_free(hb_trainer* t) { delete t; }  // (null: nothing)

int64_t hb_trainer_n_params(const hb_trainer* t) {
    if (!t) return -1;
    int64_t n = 0;
    for (const auto& v : t->spec.tensors) n += (int64_t)v.size();
    return n;
}

hb_status hb_train_step(hb_trainer* t, const uint8_t* d_packed, const float* d_labels, int64_t n, float* loss_out,
                        void* stream) {
    if (!t) return fail(HB_E_INVAL, "null trainer");
    hb_status st = check_batch(t, d_packed, d_labels, n);
    if (st != HB_OK) return st;
    HB_HIP(hipSetDevice(t->device));
    hipStream_t s = (hipStream_t)stream;
    if ((st = fwd_bwd(t, d_packed, d_labels, (int)n, s)) != HB_OK) return st;
    apply_adam(t, s);
    HB_HIP(hipGetLastError());
    if (loss_out) {
        HB_HIP(hipMemcpyAsync(loss_out, t->d_loss, 4, hipMemcpyDeviceToHost, s));
        HB_HIP(hipStreamSynchronize(s));
    }
    return HB_OK;
}

hb_status hb_train_grad(hb_trainer* t, const uint8_t* d_packed, const float* d_labels, int64_t n, float* d_grads,
                        float* loss_out) {
    if (!t || !d_grads) return fail(HB_E_INVAL, "null argument");
    hb_status st = check_batch(t, d_packed, d_labels, n);
    if (st != HB_OK) return st;
    HB_HIP(hipSetDevice(t->device));
    hipStream_t s = nullptr;
    if ((st = fwd_bwd(t, d_packed, d_labels, (int)n, s)) != HB_OK) return st;
    float* p = d_grads;
    if ((st = copy2d(p, t->dW1, t->rows1, t->N1, t->N1_pad, s)) != HB_OK) return st;
    p += (size_t)t->rows1 * t->N1;
    HB_HIP(hipMemcpyAsync(p, t->db1, (size_t)t->N1 * 4, hipMemcpyDeviceToDevice, s));
    p += t->N1;
    for (auto& l : t->L) {
        if ((st = copy2d(p, l.dW, l.K, l.N, l.N_pad, s)) != HB_OK) return st;
        p += (size_t)l.K * l.N;
        HB_HIP(hipMemcpyAsync(p, l.dbp, (size_t)l.N * 4, hipMemcpyDeviceToDevice, s));
        p += l.N;
    }
    HB_HIP(hipMemcpyAsync(p, t->dWo, (size_t)t->H * 4, hipMemcpyDeviceToDevice, s));
    p += t->H;
    HB_HIP(hipMemcpyAsync(p, t->dbo, 4, hipMemcpyDeviceToDevice, s));
    if (loss_out) HB_HIP(hipMemcpyAsync(loss_out, t->d_loss, 4, hipMemcpyDeviceToHost, s));
    HB_HIP(hipStreamSynchronize(s));
    return HB_OK;
}

hb_status hb_trainer_get_params(hb_trainer* t, float* out) {
    if (!t || !out) return fail(HB_E_INVAL, "null argument");
    HB_HIP(hipSetDevice(t->device));
    HB_HIP(hipDeviceSynchronize());
    float* p = out;
    HB_HIP(hipMemcpy(p, t->l1_master, (size_t)t->rows1 * t->N1 * 4, hipMemcpyDeviceToHost));
    p += (size_t)t->rows1 * t->N1;
    HB_HIP(hipMemcpy(p, t->l1_bias, (size_t)t->N1 * 4, hipMemcpyDeviceToHost));
    p += t->N1;
    for (auto& l : t->L) {
        HB_HIP(hipMemcpy(p, l.master, (size_t)l.K * l.N * 4, hipMemcpyDeviceToHost));
        p += (size_t)l.K * l.N;
        HB_HIP(hipMemcpy(p, l.bias, (size_t)l.N * 4, hipMemcpyDeviceToHost));
        p += l.N;
    }
    HB_HIP(hipMemcpy(p, t->ho_master, (size_t)t->H * 4, hipMemcpyDeviceToHost));
    p += t->H;
    HB_HIP(hipMemcpy(p, t->ho_b, 4, hipMemcpyDeviceToHost));
    return HB_OK;
}

hb_status hb_trainer_save(hb_trainer* t, const char* path) {
    if (!t || !path) return fail(HB_E_INVAL, "null argument");
    std::vector<float> flat((size_t)hb_trainer_n_params(t));
    hb_status st = hb_trainer_get_params(t, flat.data());
    if (st != HB_OK) return st;
    std::ofstream f(path, std::ios::binary);
    if (!f) return fail(HB_E_INVAL, "cannot write %s", path);
    std::vector<uint32_t> hdr = {0x31574248u, 1u, (uint32_t)t->spec.domain, (uint32_t)t->spec.n_in,
                                 (uint32_t)t->spec.dims.size()};
    for (int d : t->spec.dims) hdr.push_back((uint32_t)d);
    hdr.push_back((uint32_t)t->spec.n_res);
    hdr.push_back(1u);
    hdr.push_back(0u);
    f.write(reinterpret_cast<const char*>(hdr.data()), (std::streamsize)(hdr.size() * 4));
    f.write(reinterpret_cast<const char*>(flat.data()), (std::streamsize)(flat.size() * 4));
    if (!f) return fail(HB_E_INVAL, "write failed: %s", path);
    return HB_OK;
}

}  // extern "C"
