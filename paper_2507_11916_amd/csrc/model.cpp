// Model loading (weight file -> device operands in the chosen precision),
// workspace management and the forward pass: gather layer 1, a chain of MFMA
// GEMMs, head with the output rule.
#include "model.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>

#include "common.hpp"
#include "kernels.hpp"

namespace hb {

static int dom_P(int d) { return d == 0 ? 9 : d == 1 ? 16 : 54; }
static int dom_S(int d) { return d == 0 ? 9 : d == 1 ? 16 : 6; }

bool read_weight_file(const char* path, NetSpec* out, const char** why) {
    std::ifstream f(path, std::ios::binary);
    if (!f) { *why = "cannot open weight file"; return false; }
    auto rd = [&](uint32_t* v, size_t cnt) { return (bool)f.read(reinterpret_cast<char*>(v), (std::streamsize)(cnt * 4)); };
    uint32_t h[5];
    if (!rd(h, 5) || h[0] != 0x31574248u) { *why = "bad weight-file magic"; return false; }
    if (h[1] != 1) { *why = "unsupported weight-file version"; return false; }
    if (h[2] > 2 || h[4] < 1 || h[4] > 8) { *why = "bad weight-file header"; return false; }
    out->domain = (int)h[2];
    out->n_in = (int)h[3];
    std::vector<uint32_t> d(h[4]);
    if (!rd(d.data(), d.size())) { *why = "truncated header"; return false; }
    out->dims.assign(d.begin(), d.end());
    uint32_t t3[3];
    if (!rd(t3, 3)) { *why = "truncated header"; return false; }
    out->n_res = (int)t3[0];
    out->n_out = (int)t3[1];
    out->head_kind = (int)t3[2];
    if (out->n_in != dom_P(out->domain) * dom_S(out->domain)) { *why = "n_in does not match the domain"; return false; }
    if (out->n_out < 1 || out->n_out > 32 || out->n_res > 64) { *why = "unsupported output width or depth"; return false; }
    for (int v : out->dims)
        if (v < 1 || v > 8192) { *why = "unsupported layer width"; return false; }
    std::vector<std::pair<int, int>> shp;
    int prev = out->n_in;
    for (int v : out->dims) { shp.push_back({prev, v}); shp.push_back({1, v}); prev = v; }
    for (int r = 0; r < out->n_res; r++)
        for (int j = 0; j < 2; j++) { shp.push_back({prev, prev}); shp.push_back({1, prev}); }
    shp.push_back({prev, out->n_out});
    shp.push_back({1, out->n_out});
    out->tensors.clear();
    for (auto& s : shp) {
        std::vector<float> t((size_t)s.first * s.second);
        if (!f.read(reinterpret_cast<char*>(t.data()), (std::streamsize)(t.size() * 4))) { *why = "truncated tensors"; return false; }
        out->tensors.push_back(std::move(t));
    }
    return true;
}

// ---------------------------------------------------------------- rounding
static uint16_t bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
static float bf16_val(float f) {
    uint32_t u = (uint32_t)bf16_bits(f) << 16;
    float o;
    std::memcpy(&o, &u, 4);
    return o;
}

// OCP e4m3: 4 exponent bits (bias 7), 3 mantissa bits, max 448, round to
// nearest even, saturating.
static uint8_t e4m3_bits(float x) {
    uint8_t sign = std::signbit(x) ? 0x80 : 0;
    float a = std::fabs(x);
    if (std::isnan(x)) return 0x7F;
    if (a >= 448.f) return sign | 0x7E;
    if (a < 0.015625f) {  // below 2^-6: subnormal step 2^-9
        const int m = (int)std::nearbyint(a * 512.f);
        return sign | (uint8_t)m;  // m == 8 is the smallest normal, same bits
    }
    int e;
    const float fr = std::frexp(a, &e);  // a = fr * 2^e, fr in [0.5, 1)
    int E = e - 1;                        // a = (2 fr) * 2^E
    int m = (int)std::nearbyint((2.f * fr - 1.f) * 8.f);
    if (m == 8) { m = 0; E++; }
    int code = ((E + 7) << 3) | m;
    if (code > 0x7E) code = 0x7E;
    return sign | (uint8_t)code;
}

// --------------------------------------------------------------- loading
static hb_status dev_upload(hb_model* m, const void* host, size_t bytes, void** dst) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return fail(HB_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    m->allocs.push_back(p);
    HB_HIP(hipMemcpy(p, host, bytes, hipMemcpyHostToDevice));
    *dst = p;
    return HB_OK;
}

int choose_tile(const hb_model* m, int64_t M, int N_pad) {
    if (m->tile > 0) {
        if (fused_tile(m->tile - 1)) return m->tile - 1;
        int bm, bn;
        gemm_tile_shape(m->tile - 1, &bm, &bn);
        if (N_pad % bn == 0) return m->tile - 1;
    }
    int bucket = 0;
    while ((1LL << (bucket + 1)) <= M) bucket++;
    auto it = m->tuned.find(bucket);
    if (it != m->tuned.end()) {
        if (fused_tile(it->second)) return it->second;
        int bm, bn;
        gemm_tile_shape(it->second, &bm, &bn);
        if (N_pad % bn == 0) return it->second;
    }
    // Up to a few hundred rows: one wave per 32 x 32 tile (bitwise the same
    // results as the large tiles).  Beyond: the biggest tile that still gives
    // every compute unit a block.
    if (M <= 512 && N_pad % 32 == 0) return 4;
    const int order[4] = {14, 1, 0, 2};
    for (int id : order) {
        int bm, bn;
        gemm_tile_shape(id, &bm, &bn);
        if (N_pad % bn) continue;
        const int64_t tiles = ((M + bm - 1) / bm) * (N_pad / bn);
        if (tiles >= 240) return id;
    }
    return N_pad % 128 == 0 ? 2 : 0;
}

hb_status model_load(const char* path, const hb_model_opts& o, hb_model** out) {
    return model_load_members(std::vector<std::string>{path}, 0, o, out);
}

// One network, or an ensemble of networks with the same architecture fused
// into one model: layer-1 tables side by side, every matrix layer one grouped
// product over the members (weights stacked), the members' outputs combined in
// the head.
hb_status model_load_members(const std::vector<std::string>& paths, int rule, const hb_model_opts& o, hb_model** out) {
    const int k = (int)paths.size();
    if (k < 1 || k > 4) return fail(HB_E_INVAL, "an ensemble has 1 to 4 members");
    if (rule < 0 || rule > 1) return fail(HB_E_INVAL, "unknown ensemble rule %d", rule);
    std::vector<NetSpec> specs(k);
    for (int i = 0; i < k; i++) {
        const char* why = "";
        if (!read_weight_file(paths[i].c_str(), &specs[i], &why)) return fail(HB_E_INVAL, "%s: %s", paths[i].c_str(), why);
    }
    const NetSpec& spec = specs[0];
    for (int i = 1; i < k; i++) {
        const NetSpec& t = specs[i];
        if (t.domain != spec.domain || t.n_in != spec.n_in || t.dims != spec.dims || t.n_res != spec.n_res ||
            t.n_out != spec.n_out || t.head_kind != spec.head_kind)
            return fail(HB_E_INVAL, "ensemble member %d has another architecture than member 0", i);
    }
    if (k > 1 && (spec.head_kind != 0 || spec.n_out != 1)) return fail(HB_E_INVAL, "ensembles are of regression networks");
    if (o.prec < HB_FP32 || o.prec > HB_FP8_E4M3) return fail(HB_E_INVAL, "unknown precision %d", (int)o.prec);
    if (o.out < HB_OUT_REG_FLOOR || o.out > HB_OUT_CLS_ARGMAX) return fail(HB_E_INVAL, "unknown output mode");
    const bool cls_mode = o.out >= HB_OUT_CLS_QUANTILE;
    if (cls_mode != (spec.head_kind == 1)) return fail(HB_E_INVAL, "output mode does not match the network head");
    if (!cls_mode && spec.n_out != 1) return fail(HB_E_INVAL, "a regression head has one output");
    if (o.combine_md < 0 || o.combine_md > 3) return fail(HB_E_INVAL, "combine_md must be 0..3");
    if (o.combine_md && spec.domain == 2) return fail(HB_E_INVAL, "Manhattan distance applies to sliding tiles only");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(HB_E_DEVICE, "no HIP device available");
    if (o.device < 0 || o.device >= ndev) return fail(HB_E_INVAL, "device %d out of range", o.device);
    HB_HIP(hipSetDevice(o.device));
    static bool attrs = false;
    if (!attrs) { HB_HIP(gemm_prepare_attributes()); attrs = true; }

    auto m = std::make_unique<hb_model>();
    m->device = o.device;
    HB_HIP(hipDeviceGetAttribute(&m->cus, hipDeviceAttributeMultiprocessorCount, o.device));
    m->opts = o;
    if (m->opts.max_batch <= 0) m->opts.max_batch = 16384;
    m->spec = spec;
    m->path = paths[0];
    m->paths = paths;
    m->members = k;
    m->ens_rule = rule;
    const int prec = (int)o.prec;
    const int eb = prec == 0 ? 4 : prec == 1 ? 2 : 1;
    auto pad = [](int v) { return (int)round_up(v, 128); };

    // Layer 1: table of gathered rows (cube: non-centre stickers only, the
    // constant centre rows folded into the bias).
    m->P = dom_P(spec.domain);
    m->S = dom_S(spec.domain);
    m->N1 = spec.dims[0];
    m->N1_pad = pad(m->N1);
    const int P_eff = spec.domain == 2 ? 48 : m->P;
    m->table_rows = P_eff * m->S;
    auto wq = [&](float v) { return prec == 0 ? v : bf16_val(v); };  // layer-1 / head weight rounding
    const int W1 = k * m->N1_pad;  // member i owns columns [i * N1_pad, i * N1_pad + N1)
    std::vector<float> bias1(W1, 0.f);
    std::vector<float> tab((size_t)m->table_rows * W1, 0.f);
    for (int i = 0; i < k; i++) {
        const auto& T = specs[i].tensors;
        const int c0 = i * m->N1_pad;
        for (int j = 0; j < m->N1; j++) bias1[c0 + j] = T[1][j];
        for (int q = 0; q < P_eff; q++) {
            const int p = spec.domain == 2 ? q + q / 8 + (q % 8 >= 4 ? 1 : 0) : q;
            for (int s = 0; s < m->S; s++)
                for (int j = 0; j < m->N1; j++)
                    tab[((size_t)q * m->S + s) * W1 + c0 + j] = wq(T[0][((size_t)p * m->S + s) * m->N1 + j]);
        }
        if (spec.domain == 2)
            for (int f = 0; f < 6; f++) {
                const int p = 9 * f + 4;
                for (int j = 0; j < m->N1; j++) bias1[c0 + j] += wq(T[0][((size_t)p * 6 + f) * m->N1 + j]);
            }
    }
    // The table is kept in float32 at every precision (at BF16/FP8 holding the
    // bfloat16-rounded values, which float32 represents exactly): the gather
    // is bound by vector ALU work, and float32 entries need no conversion.
    hb_status st = dev_upload(m.get(), tab.data(), tab.size() * 4, &m->l1_table);
    if (st != HB_OK) return st;
    if ((st = dev_upload(m.get(), bias1.data(), bias1.size() * 4, (void**)&m->l1_bias)) != HB_OK) return st;
    m->weight_bytes += (int64_t)tab.size() * 4;
    m->flops = (double)k * P_eff * m->N1;  // gathered adds

    // Matrix layers: dense layers 2..n_dense, then residual pairs.
    const int n_dense = (int)spec.dims.size();
    m->n_act = n_dense + 2 * spec.n_res;
    int ti = 2, act = 0;
    int width_cap = W1;
    // Tensor `t` of every member as one matrix layer: member i's output
    // columns are rows [i * N_pad, (i + 1) * N_pad) of Wt.
    auto add_layer = [&](int t, int K, int N, int in_act, int out_act, int res_act) -> hb_status {
        MatLayer L;
        L.K = K; L.N = N; L.K_pad = pad(K); L.N_pad = pad(N);
        L.in_act = in_act; L.out_act = out_act; L.res_act = res_act;
        L.groups = k;
        const int NT = k * L.N_pad;
        std::vector<float> bp(NT, 0.f);
        for (int i = 0; i < k; i++)
            for (int j = 0; j < N; j++) bp[i * L.N_pad + j] = specs[i].tensors[t + 1][j];
        hb_status s2 = dev_upload(m.get(), bp.data(), bp.size() * 4, (void**)&L.bias);
        if (s2 != HB_OK) return s2;
        const size_t cnt = (size_t)NT * L.K_pad;
        auto w_at = [&](int i, int kk, int n) { return specs[i].tensors[t][(size_t)kk * N + n]; };
        if (prec == 0) {
            std::vector<float> wt(cnt, 0.f);
            for (int i = 0; i < k; i++)
                for (int kk = 0; kk < K; kk++)
                    for (int n = 0; n < N; n++) wt[(size_t)(i * L.N_pad + n) * L.K_pad + kk] = w_at(i, kk, n);
            s2 = dev_upload(m.get(), wt.data(), cnt * 4, &L.Wt);
        } else if (prec == 1) {
            std::vector<uint16_t> wt(cnt, 0);
            for (int i = 0; i < k; i++)
                for (int kk = 0; kk < K; kk++)
                    for (int n = 0; n < N; n++) wt[(size_t)(i * L.N_pad + n) * L.K_pad + kk] = bf16_bits(w_at(i, kk, n));
            s2 = dev_upload(m.get(), wt.data(), cnt * 2, &L.Wt);
        } else {
            std::vector<uint8_t> wt(cnt, 0);
            std::vector<float> cs(NT, 0.f);
            for (int i = 0; i < k; i++)
                for (int n = 0; n < N; n++) {
                    float mx = 0.f;
                    for (int kk = 0; kk < K; kk++) mx = std::max(mx, std::fabs(w_at(i, kk, n)));
                    const float s = mx / 448.f;
                    cs[i * L.N_pad + n] = s;
                    if (s > 0.f)
                        for (int kk = 0; kk < K; kk++)
                            wt[(size_t)(i * L.N_pad + n) * L.K_pad + kk] = e4m3_bits(w_at(i, kk, n) / s);
                }
            s2 = dev_upload(m.get(), wt.data(), cnt, &L.Wt);
            if (s2 == HB_OK) s2 = dev_upload(m.get(), cs.data(), cs.size() * 4, (void**)&L.colscale);
        }
        if (s2 != HB_OK) return s2;
        m->weight_bytes += (int64_t)cnt * eb;
        m->flops += 2.0 * k * K * N;
        width_cap = std::max(width_cap, k * std::max(L.K_pad, L.N_pad));
        m->layers.push_back(L);
        return HB_OK;
    };
    for (int i = 1; i < n_dense; i++) {
        if ((st = add_layer(ti, spec.dims[i - 1], spec.dims[i], act, act + 1, -1)) != HB_OK) return st;
        ti += 2;
        act++;
    }
    const int H = spec.dims.back();
    for (int r = 0; r < spec.n_res; r++) {
        const int x_act = act;
        if ((st = add_layer(ti, H, H, x_act, n_dense + 2 * r, -1)) != HB_OK) return st;
        if ((st = add_layer(ti + 2, H, H, n_dense + 2 * r, n_dense + 2 * r + 1, x_act)) != HB_OK) return st;
        m->layers.back().res_in_place = true;
        ti += 4;
        act = n_dense + 2 * r + 1;
    }
    // Head: [n_out][K_pad] per member (members side by side), float32 or bfloat16.
    m->K_last_pad = pad(H);
    std::vector<float> hw((size_t)k * spec.n_out * m->K_last_pad, 0.f);
    std::vector<float> hbias((size_t)k * spec.n_out, 0.f);
    for (int i = 0; i < k; i++) {
        const auto& T = specs[i].tensors;
        for (int kk = 0; kk < H; kk++)
            for (int oo = 0; oo < spec.n_out; oo++)
                hw[((size_t)i * spec.n_out + oo) * m->K_last_pad + kk] = wq(T[ti][(size_t)kk * spec.n_out + oo]);
        for (int oo = 0; oo < spec.n_out; oo++) hbias[(size_t)i * spec.n_out + oo] = T[ti + 1][oo];
    }
    if (prec == 0) {
        st = dev_upload(m.get(), hw.data(), hw.size() * 4, &m->head_W);
    } else {
        std::vector<uint16_t> hb16(hw.size());
        for (size_t i = 0; i < hw.size(); i++) hb16[i] = bf16_bits(hw[i]);
        st = dev_upload(m.get(), hb16.data(), hb16.size() * 2, &m->head_W);
    }
    if (st != HB_OK) return st;
    if ((st = dev_upload(m.get(), hbias.data(), hbias.size() * 4, (void**)&m->head_b)) != HB_OK) return st;
    m->weight_bytes += (int64_t)hw.size() * (prec == 0 ? 4 : 2);
    m->flops += 2.0 * k * H * spec.n_out;
    m->width_cap = width_cap;
    m->act_scale.assign(m->n_act, 1.f);
    m->calibrated = prec != 2;
    *out = m.release();
    return HB_OK;
}

void model_free(hb_model* m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : m->ws) {
        (void)hipFree(kv.second.x);
        (void)hipFree(kv.second.t);
        (void)hipFree(kv.second.absmax);
        (void)hipFree(kv.second.sync);
    }
    for (void* p : m->allocs) (void)hipFree(p);
    delete m;
}

static hb_status get_ws(hb_model* m, hipStream_t s, Workspace** out) {
    std::lock_guard<std::mutex> lk(m->mu);
    auto it = m->ws.find(s);
    if (it != m->ws.end()) { *out = &it->second; return HB_OK; }
    Workspace w;
    const int eb = m->opts.prec == HB_FP32 ? 4 : m->opts.prec == HB_BF16 ? 2 : 1;
    w.rows_cap = (int)round_up(m->opts.max_batch, 256);
    const size_t bytes = (size_t)w.rows_cap * m->width_cap * eb;
    w.rb_cap = w.rows_cap / 32;
    const size_t sync_ints = 4 + (size_t)(fused_max_layers() + 1) * w.rb_cap;
    const size_t sync_bytes = (sync_ints + 2) * sizeof(int);  // then the GEMMs' tile counter pair
    if (hipMalloc(&w.x, bytes) != hipSuccess || hipMalloc(&w.t, bytes) != hipSuccess ||
        hipMalloc((void**)&w.absmax, 64 * sizeof(unsigned)) != hipSuccess ||
        hipMalloc((void**)&w.sync, sync_bytes) != hipSuccess) {
        (void)hipFree(w.x);
        (void)hipFree(w.t);
        (void)hipFree(w.absmax);
        return fail(HB_E_NOMEM, "workspace allocation of 2 x %zu bytes failed", bytes);
    }
    // the fused kernel's counters and the tile counters start at zero; each
    // launch leaves them zero
    HB_HIP(hipMemset(w.sync, 0, sync_bytes));
    w.tile_ctr = w.sync + sync_ints;
    auto r = m->ws.emplace(s, w);
    *out = &r.first->second;
    return HB_OK;
}

hb_status model_prepare(hb_model* m, hipStream_t s) {
    HB_HIP(hipSetDevice(m->device));
    Workspace* w = nullptr;
    return get_ws(m, s, &w);
}

// Per-kernel timing (hb_model_profile): events bracket each launch on its
// stream, or (GEMMs: `attach` given) are handed to the launch, which records
// the kernel's own start and end on them.
static int prof_begin(hb_model* m, int kind, hipStream_t s, GemmLaunch* attach = nullptr) {
    if (!m->profiling) return -1;
    hb_model::Timed t{kind, nullptr, nullptr, 0.0};
    if (hipEventCreate(&t.a) != hipSuccess || hipEventCreate(&t.b) != hipSuccess) return -1;
    if (attach) {
        attach->ev_start = t.a;
        attach->ev_stop = t.b;
    } else {
        (void)hipEventRecord(t.a, s);
    }
    std::lock_guard<std::mutex> lk(m->mu);
    m->timed.push_back(t);
    return (int)m->timed.size() - 1;
}

static void prof_end(hb_model* m, int idx, double flops, hipStream_t s, bool attached = false) {
    if (idx < 0) return;
    std::lock_guard<std::mutex> lk(m->mu);
    m->timed[idx].flops = flops;
    if (!attached) (void)hipEventRecord(m->timed[idx].b, s);
}

hb_status model_profile(hb_model* m, bool enable) {
    hb_profile dummy;
    if (!enable) { model_profile_read(m, &dummy); m->profiling = false; return HB_OK; }
    model_profile_read(m, &dummy);
    for (int k = 0; k < 3; k++) { m->prof_ms[k] = 0; m->prof_n[k] = 0; }
    m->prof_flops = 0;
    m->profiling = true;
    return HB_OK;
}

hb_status model_profile_read(hb_model* m, hb_profile* out) {
    std::lock_guard<std::mutex> lk(m->mu);
    for (auto& t : m->timed) {
        float ms = 0.f;
        if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            m->prof_ms[t.kind] += ms;
            m->prof_n[t.kind] += 1;
            if (t.kind == 1) m->prof_flops += t.flops;
        }
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    m->timed.clear();
    out->gather_ms = m->prof_ms[0];
    out->gemm_ms = m->prof_ms[1];
    out->head_ms = m->prof_ms[2];
    out->gather_launches = m->prof_n[0];
    out->gemm_launches = m->prof_n[1];
    out->head_launches = m->prof_n[2];
    out->gemm_flops = m->prof_flops;
    return HB_OK;
}

// Fused persistent forward (tile ids 10..13): waves per compute unit.
bool fused_tile(int id) { return id >= 10 && id <= 13; }
int fused_waves_per_cu(int id) {
    static const int W[4] = {2, 4, 8, 12};
    return W[id - 10];
}

// The whole forward pass of one chunk as one launch of fused_forward_kernel;
// buffers and arithmetic as in eval_chunk's kernel-per-layer path.
static hb_status eval_fused(hb_model* m, Workspace* w, const uint8_t* d_packed, int n, const int32_t* d_n, int m_cap,
                            int32_t* d_h, float* d_raw, hipStream_t s, int waves_per_cu, bool timed) {
    const int prec = (int)m->opts.prec;
    FusedLaunch F{};
    F.domain = m->spec.domain;
    F.prec = prec;
    F.packed = d_packed;
    F.n_dev = d_n;
    F.n_host = n;
    F.m_cap = m_cap;
    F.table = m->l1_table;
    F.bias1 = m->l1_bias;
    F.N1 = m->members * m->N1_pad;
    F.ld1 = m->width_cap;
    void* X = w->x;
    void* Tb = w->t;
    F.out1 = X;
    F.out1_inv_scale = 1.f / m->act_scale[0];
    F.n_layers = (int)m->layers.size();
    const int n_dense = (int)m->spec.dims.size();
    for (int i = 0; i < F.n_layers; i++) {
        const MatLayer& L = m->layers[i];
        const bool res_first = !L.res_in_place && L.out_act >= n_dense;
        GemmLaunch& g = F.layers[i];
        g = GemmLaunch{};
        g.prec = prec;
        g.tile = 4;
        g.Bt = L.Wt;
        if (L.res_in_place) { g.A = Tb; g.R = X; g.C = X; }
        else { g.A = X; g.R = nullptr; g.C = Tb; }
        g.bias = L.bias;
        g.colscale = L.colscale;
        g.m_dev = d_n;
        g.m_host = n;
        g.m_cap = m_cap;
        g.N = L.N_pad * L.groups;
        g.K = L.K_pad;
        if (L.groups > 1) { g.group_n = L.N_pad; g.group_k = L.K_pad; }
        g.lda = m->width_cap;
        g.ldb = L.K_pad;
        g.ldc = m->width_cap;
        g.a_scale = m->act_scale[L.in_act];
        g.r_scale = L.res_act >= 0 ? m->act_scale[L.res_act] : 1.f;
        g.out_inv_scale = 1.f / m->act_scale[L.out_act];
        g.relu = 1;
        if (!L.res_in_place && !res_first) std::swap(X, Tb);
    }
    HeadArgs& H = F.head;
    H.X = X;
    H.ldx = m->width_cap;
    H.K = m->K_last_pad;
    H.W = m->head_W;
    H.b = m->head_b;
    H.n_out = m->spec.n_out;
    H.x_scale = m->act_scale[m->n_act - 1];
    H.n_dev = d_n;
    H.n_host = n;
    H.packed = d_packed;
    H.domain = m->spec.domain;
    H.mode = (int)m->opts.out;
    H.q = m->opts.q;
    H.offset = m->opts.offset;
    H.combine_md = m->opts.combine_md;
    H.members = m->members;
    H.ens_rule = m->ens_rule;
    H.h_out = d_h;
    H.raw = d_raw;
    F.sync = w->sync;
    F.rb_cap = w->rb_cap;
    F.spin_limit = 1 << 18;  // polls of about 1 us: a wait gives up after about 0.3 s
    F.grid = std::max(1, m->cus) * waves_per_cu;
    if ((m_cap + 31) / 32 > w->rb_cap) return fail(HB_E_INVAL, "batch exceeds the fused kernel's counters");
    const int pi = timed ? prof_begin(m, 1, s) : -1;
    if (!launch_fused(F, s)) return fail(HB_E_UNSUPPORTED, "no fused forward kernel for this network");
    HB_HIP(hipGetLastError());
    prof_end(m, pi, m->flops * (d_n ? m_cap : n), s);
    return HB_OK;
}

// Forward pass over one chunk of at most max_batch states.
static hb_status eval_chunk(hb_model* m, Workspace* w, const uint8_t* d_packed, int n, const int32_t* d_n, int m_cap,
                            int32_t* d_h, float* d_raw, hipStream_t s, CalibCapture* cap, int force_tile,
                            bool timed = true, const ActCopy* ac = nullptr) {
    const int eb_act = m->opts.prec == HB_FP32 ? 4 : m->opts.prec == HB_BF16 ? 2 : 1;
    auto copy_act = [&](int act, const void* buf, int width) -> hb_status {
        if (!ac || ac->act != act) return HB_OK;
        HB_HIP(hipMemcpy2DAsync(ac->out, (size_t)ac->ld_bytes, buf, (size_t)m->width_cap * eb_act,
                                (size_t)width * eb_act, (size_t)n, hipMemcpyDeviceToDevice, s));
        return HB_OK;
    };
    const int prec = (int)m->opts.prec;
    if (cap && prec != 0) return fail(HB_E_INVAL, "calibration runs on a float32 model");
    const int rows = (int)round_up(m_cap, 128);
    void* X = w->x;
    void* Tb = w->t;
    if (cap) HB_HIP(hipMemsetAsync(w->absmax, 0, 64 * sizeof(unsigned), s));
    const int t0 = force_tile >= 0 ? force_tile : choose_tile(m, m_cap, 128);
    if (fused_tile(t0) && fused_enabled() && !cap && !ac && w->sync && !m->layers.empty() &&
        (int)m->layers.size() <= fused_max_layers() && m->spec.n_out <= 32)
        return eval_fused(m, w, d_packed, n, d_n, m_cap, d_h, d_raw, s, fused_waves_per_cu(t0), timed);
    GatherLaunch G{};
    G.domain = m->spec.domain;
    G.prec = prec;
    G.packed = d_packed;
    G.n_dev = d_n;
    G.n_host = n;
    G.m_rows = rows;
    G.table = m->l1_table;
    G.table_f32 = 1;
    G.t_rows = m->table_rows;
    G.bias = m->l1_bias;
    G.N = m->members * m->N1_pad;
    G.ld_out = m->width_cap;
    G.out = X;
    G.out_inv_scale = 1.f / m->act_scale[0];
    int pi = timed ? prof_begin(m, 0, s) : -1;
    if (!launch_gather(G, s)) return fail(HB_E_UNSUPPORTED, "no layer-1 kernel for this domain/precision");
    HB_HIP(hipGetLastError());
    prof_end(m, pi, 0.0, s);
    if (hb_status st = copy_act(0, X, m->members * m->N1_pad); st != HB_OK) return st;
    if (cap) launch_absmax((const float*)X, n, m->members * m->N1_pad, m->width_cap, w->absmax + 0, s);
    // X holds the running activation x, Tb is scratch.  A dense layer writes
    // Tb and the two swap roles; the first layer of a residual block writes
    // t into Tb and keeps x in X; the second reads t, adds x and overwrites x
    // in place (each element of x is read and written by the same lane).
    const int n_dense = (int)m->spec.dims.size();
    for (const MatLayer& L : m->layers) {
        const bool res_first = !L.res_in_place && L.out_act >= n_dense;
        GemmLaunch g{};
        g.prec = prec;
        g.tile = force_tile >= 0 ? force_tile : choose_tile(m, m_cap, L.N_pad);
        if (fused_tile(g.tile)) g.tile = 4;  // same arithmetic, one launch per layer
        g.Bt = L.Wt;
        if (L.res_in_place) { g.A = Tb; g.R = X; g.C = X; }
        else { g.A = X; g.R = nullptr; g.C = Tb; }
        g.bias = L.bias;
        g.colscale = L.colscale;
        g.m_dev = d_n;
        g.m_host = n;
        g.m_cap = m_cap;
        g.N = L.N_pad * L.groups;
        g.K = L.K_pad;
        if (L.groups > 1) { g.group_n = L.N_pad; g.group_k = L.K_pad; }
        g.lda = m->width_cap;
        g.ldb = L.K_pad;
        g.ldc = m->width_cap;
        g.a_scale = m->act_scale[L.in_act];
        g.r_scale = L.res_act >= 0 ? m->act_scale[L.res_act] : 1.f;
        g.out_inv_scale = 1.f / m->act_scale[L.out_act];
        g.relu = 1;
        g.tile_ctr = w->tile_ctr;  // used by the persistent-grid tiles
        pi = timed ? prof_begin(m, 1, s, &g) : -1;
        if (!launch_gemm(g, s)) return fail(HB_E_UNSUPPORTED, "no GEMM kernel for this precision/tile");
        HB_HIP(hipGetLastError());
        prof_end(m, pi, 2.0 * (d_n ? m_cap : n) * L.K * L.N * L.groups, s, true);
        if (hb_status st = copy_act(L.out_act, g.C, L.N_pad * L.groups); st != HB_OK) return st;
        if (cap) launch_absmax((const float*)g.C, n, L.N_pad * L.groups, m->width_cap, w->absmax + L.out_act, s);
        if (!L.res_in_place && !res_first) std::swap(X, Tb);
    }
    HeadArgs H{};
    H.X = X;
    H.ldx = m->width_cap;
    H.K = m->K_last_pad;
    H.W = m->head_W;
    H.b = m->head_b;
    H.n_out = m->spec.n_out;
    H.x_scale = m->act_scale[m->n_act - 1];
    H.n_dev = d_n;
    H.n_host = n;
    H.packed = d_packed;
    H.domain = m->spec.domain;
    H.mode = (int)m->opts.out;
    H.q = m->opts.q;
    H.offset = m->opts.offset;
    H.combine_md = m->opts.combine_md;
    H.members = m->members;
    H.ens_rule = m->ens_rule;
    H.h_out = d_h;
    H.raw = d_raw;
    pi = timed ? prof_begin(m, 2, s) : -1;
    if (!launch_head(H, prec, m_cap, s)) return fail(HB_E_UNSUPPORTED, "no head kernel for %d outputs", H.n_out);
    HB_HIP(hipGetLastError());
    prof_end(m, pi, 0.0, s);
    if (cap) {
        std::vector<unsigned> bits(m->n_act);
        HB_HIP(hipMemcpyAsync(bits.data(), w->absmax, m->n_act * sizeof(unsigned), hipMemcpyDeviceToHost, s));
        HB_HIP(hipStreamSynchronize(s));
        cap->act_max->resize(m->n_act);
        for (int a = 0; a < m->n_act; a++) {
            float v;
            std::memcpy(&v, &bits[a], 4);
            (*cap->act_max)[a] = std::max((*cap->act_max)[a], v);
        }
    }
    return HB_OK;
}

hb_status model_eval(hb_model* m, const uint8_t* d_packed, int64_t n, const int32_t* d_n, int64_t max_n, int32_t* d_h,
                     float* d_raw, hipStream_t s, CalibCapture* cap, int force_tile, const ActCopy* act_copy) {
    if (!m) return fail(HB_E_INVAL, "null model");
    if (!m->calibrated) return fail(HB_E_INVAL, "FP8 model has no activation scales: call hb_model_calibrate first");
    HB_HIP(hipSetDevice(m->device));
    Workspace* w = nullptr;
    hb_status st = get_ws(m, s, &w);
    if (st != HB_OK) return st;
    const int pb = m->spec.domain == 2 ? 24 : 8;
    if (d_n) {
        if (max_n > m->opts.max_batch) return fail(HB_E_INVAL, "max_n %lld exceeds the model's max_batch %d", (long long)max_n, m->opts.max_batch);
        if (max_n <= 0) return HB_OK;
        return eval_chunk(m, w, d_packed, 0, d_n, (int)max_n, d_h, d_raw, s, cap, force_tile);
    }
    for (int64_t off = 0; off < n; off += m->opts.max_batch) {
        const int c = (int)std::min<int64_t>(m->opts.max_batch, n - off);
        ActCopy ac;
        if (act_copy) { ac = *act_copy; ac.out += off * ac.ld_bytes; }
        st = eval_chunk(m, w, d_packed + off * pb, c, nullptr, c, d_h + off,
                        d_raw ? d_raw + off * m->spec.n_out : nullptr, s, cap, force_tile, true,
                        act_copy ? &ac : nullptr);
        if (st != HB_OK) return st;
    }
    return HB_OK;
}

// ------------------------------------------------ allocation-free evaluation
// The activation buffers of hb_eval_batch_noalloc live in this fixed device
// array (one copy per GPU, held until the process ends).  In host code the
// name `scratch` is a host-side stand-in, not a device address: kernels are
// given the address hipGetSymbolAddress returns with the device current, kept
// per device in scratch_dev.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex scratch_mu;
static unsigned char* scratch_dev[kScratchDevices];

static hb_status scratch_address(int device, unsigned char** out) {
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[device]) {
        void* p = nullptr;
        HB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(HB_E_DEVICE, "no device address for the allocation-free scratch array");
        scratch_dev[device] = static_cast<unsigned char*>(p);
    }
    *out = scratch_dev[device];
    return HB_OK;
}

int64_t model_noalloc_capacity(const hb_model* m) {
    const int eb = m->opts.prec == HB_FP32 ? 4 : m->opts.prec == HB_BF16 ? 2 : 1;
    const size_t row_bytes = (size_t)m->width_cap * eb;
    return (int64_t)(kScratchBytes / 2 / row_bytes) / 256 * 256;  // whole 256-row GEMM tiles
}

hb_status model_eval_noalloc(hb_model* m, const uint8_t* d_packed, int64_t n, int32_t* d_h, float* d_raw,
                             hipStream_t s) {
    if (!m->calibrated) return fail(HB_E_INVAL, "FP8 model has no activation scales: call hb_model_calibrate first");
    if (m->device < 0 || m->device >= kScratchDevices) return fail(HB_E_INVAL, "device %d out of range", m->device);
    const int64_t cap = model_noalloc_capacity(m);
    if (n > cap)
        return fail(HB_E_INVAL, "n = %lld exceeds the allocation-free limit of %lld states for this model "
                    "(two activation rows of %d elements per state in a %zu-byte array)",
                    (long long)n, (long long)cap, m->width_cap, kScratchBytes);
    if (n == 0) return HB_OK;
    HB_HIP(hipSetDevice(m->device));
    unsigned char* base = nullptr;
    hb_status st = scratch_address(m->device, &base);
    if (st != HB_OK) return st;
    Workspace w;
    w.x = base;
    w.t = base + kScratchBytes / 2;
    w.rows_cap = (int)cap;
    const int pb = m->spec.domain == 2 ? 24 : 8;
    for (int64_t off = 0; off < n; off += m->opts.max_batch) {
        const int c = (int)std::min<int64_t>(m->opts.max_batch, n - off);
        st = eval_chunk(m, &w, d_packed + off * pb, c, nullptr, c, d_h + off,
                        d_raw ? d_raw + off * m->spec.n_out : nullptr, s, nullptr, -1, false);
        if (st != HB_OK) return st;
    }
    return HB_OK;
}

hb_status model_calibrate(hb_model* m, const uint8_t* d_packed, int64_t n) {
    if (m->opts.prec != HB_FP8_E4M3) return fail(HB_E_INVAL, "calibration applies to FP8 models");
    if (n <= 0) return fail(HB_E_INVAL, "calibration needs at least one state");
    hb_model_opts o = m->opts;
    o.prec = HB_FP32;
    hb_model* f = nullptr;
    hb_status st = model_load_members(m->paths, m->ens_rule, o, &f);
    if (st != HB_OK) return st;
    std::vector<float> mx(f->n_act, 0.f);
    CalibCapture cap{&mx};
    int32_t* d_h = nullptr;
    if (hipMalloc((void**)&d_h, (size_t)std::min<int64_t>(n, f->opts.max_batch) * 4) != hipSuccess) {
        model_free(f);
        return fail(HB_E_NOMEM, "calibration buffer");
    }
    st = model_eval(f, d_packed, n, nullptr, 0, d_h, nullptr, nullptr, &cap);
    (void)hipFree(d_h);
    model_free(f);
    if (st != HB_OK) return st;
    for (int a = 0; a < m->n_act; a++) {
        const double v = mx[a];
        if (!(v > 0)) { m->act_scale[a] = 1.f; continue; }
        int e = 0;
        while (448.0 * std::ldexp(1.0, e) < v) e++;
        while (448.0 * std::ldexp(1.0, e - 1) >= v) e--;
        m->act_scale[a] = (float)std::ldexp(1.0, e);
    }
    m->calibrated = true;
    return HB_OK;
}

// Device buffers and events of one tuning session, released on every path.
struct TuneScratch {
    int32_t* d_h = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneScratch() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(d_h);
    }
};

static int bucket_of(int64_t n) {
    int b = 0;
    while ((1LL << (b + 1)) <= n) b++;
    return b;
}

// Times every tile shape on the first n states; the fastest goes to *best_id
// (internal id) and *best_us.  Pairs (set_tile id, us) go to report.
static hb_status time_tiles(hb_model* m, const uint8_t* d_packed, int64_t n, TuneScratch& t, int* best_id,
                            double* best_us, double* report, int cap) {
    hipStream_t s = nullptr;
    *best_id = -1;
    *best_us = 1e30;
    const int count = gemm_tile_count();
    std::vector<double> us_of(count, 1e30);
    // Two rounds over the tiles, each tile keeping its faster round: close
    // tiles are not decided by the order they were timed in.
    for (int round = 0; round < 2; round++) {
        for (int id = 0; id < count; id++) {
            if (fused_tile(id) && !fused_enabled()) continue;
            int bm, bn;
            gemm_tile_shape(id, &bm, &bn);
            bool ok = true;
            for (const MatLayer& L : m->layers) ok &= (L.N_pad % bn == 0);
            if (!ok) continue;
            for (int w = 0; w < 2; w++) {
                hb_status st = model_eval(m, d_packed, n, nullptr, 0, t.d_h, nullptr, s, nullptr, id);
                if (st != HB_OK) return st;
            }
            // about 2 ms of work per tile and round, 3 to 50 repetitions
            const int reps = (int)std::max<int64_t>(3, std::min<int64_t>(50, 2000000 / std::max<int64_t>(1, n * 20)));
            HB_HIP(hipEventRecord(t.e0, s));
            for (int r = 0; r < reps; r++) {
                hb_status st = model_eval(m, d_packed, n, nullptr, 0, t.d_h, nullptr, s, nullptr, id);
                if (st != HB_OK) return st;
            }
            HB_HIP(hipEventRecord(t.e1, s));
            HB_HIP(hipEventSynchronize(t.e1));
            float ms = 0.f;
            HB_HIP(hipEventElapsedTime(&ms, t.e0, t.e1));
            us_of[id] = std::min(us_of[id], 1000.0 * ms / reps);
        }
    }
    int nrep = 0;
    for (int id = 0; id < count; id++) {
        if (us_of[id] >= 1e30) continue;
        if (report && 2 * nrep + 1 < cap) { report[2 * nrep] = id + 1; report[2 * nrep + 1] = us_of[id]; }
        nrep++;
        if (us_of[id] < *best_us) { *best_us = us_of[id]; *best_id = id; }
    }
    return HB_OK;
}

static hb_status tune_prepare(hb_model* m, int64_t n, TuneScratch& t) {
    HB_HIP(hipSetDevice(m->device));
    if (hipMalloc((void**)&t.d_h, (size_t)n * 4) != hipSuccess) return fail(HB_E_NOMEM, "tuning buffer");
    HB_HIP(hipEventCreate(&t.e0));
    HB_HIP(hipEventCreate(&t.e1));
    return HB_OK;
}

hb_status model_tune(hb_model* m, const uint8_t* d_packed, int64_t n, double* report, int cap) {
    if (n <= 0 || n > m->opts.max_batch) return fail(HB_E_INVAL, "tuning batch must be in 1..max_batch");
    TuneScratch t;
    hb_status st = tune_prepare(m, n, t);
    if (st != HB_OK) return st;
    int best_id;
    double best_us;
    st = time_tiles(m, d_packed, n, t, &best_id, &best_us, report, cap);
    if (st != HB_OK) return st;
    if (best_id >= 0) m->tuned[bucket_of(n)] = best_id;
    return HB_OK;
}

hb_status model_autotune(hb_model* m, const uint8_t* d_packed, int64_t n, hb_tune_entry* table, int cap, int* rows,
                         int32_t* recommended) {
    const int64_t top = std::min<int64_t>(n, m->opts.max_batch);
    if (top <= 0) return fail(HB_E_INVAL, "autotuning needs at least one state");
    std::vector<int64_t> batches;
    for (int64_t b = 1; b <= top; b *= 2) batches.push_back(b);
    if (batches.back() != top) batches.push_back(top);
    TuneScratch t;
    hb_status st = tune_prepare(m, top, t);
    if (st != HB_OK) return st;
    std::vector<hb_tune_entry> out;
    for (int64_t b : batches) {
        int best_id;
        double best_us;
        st = time_tiles(m, d_packed, b, t, &best_id, &best_us, nullptr, 0);
        if (st != HB_OK) return st;
        if (best_id < 0) return fail(HB_E_UNSUPPORTED, "no tile shape fits this network");
        m->tuned[bucket_of(b)] = best_id;
        out.push_back(hb_tune_entry{(int32_t)b, best_id + 1, best_us, b / (best_us * 1e-6)});
    }
    double best_rate = 0;
    for (const auto& e : out) best_rate = std::max(best_rate, e.evals_per_s);
    int32_t rec = out.back().batch;
    for (const auto& e : out)
        if (e.evals_per_s >= 0.9 * best_rate) { rec = e.batch; break; }
    if (recommended) *recommended = rec;
    const int k = (int)std::min<size_t>(out.size(), (size_t)std::max(0, cap));
    if (table) std::copy(out.begin(), out.begin() + k, table);
    if (rows) *rows = table ? k : (int)out.size();
    return HB_OK;
}

// Tuning file: "hbtune 1", "arch <gcnArchName>", "model <signature>", then
// "bucket <log2> tile <internal id>" lines.
static std::string model_signature(const hb_model* m) {
    std::string sig = "d" + std::to_string(m->spec.domain) + " in" + std::to_string(m->spec.n_in) + " dims";
    for (int d : m->spec.dims) sig += "_" + std::to_string(d);
    sig += " res" + std::to_string(m->spec.n_res) + " out" + std::to_string(m->spec.n_out) + " prec" +
           std::to_string((int)m->opts.prec) + " members" + std::to_string(m->members);
    return sig;
}

static hb_status device_arch(int device, std::string* arch) {
    hipDeviceProp_t prop;
    HB_HIP(hipGetDeviceProperties(&prop, device));
    *arch = prop.gcnArchName;
    const size_t colon = arch->find(':');
    if (colon != std::string::npos) arch->resize(colon);
    return HB_OK;
}

hb_status model_save_tuning(const hb_model* m, const char* path) {
    std::string arch;
    hb_status st = device_arch(m->device, &arch);
    if (st != HB_OK) return st;
    FILE* f = fopen(path, "w");
    if (!f) return fail(HB_E_INVAL, "cannot write %s", path);
    fprintf(f, "hbtune 1\narch %s\nmodel %s\n", arch.c_str(), model_signature(m).c_str());
    for (const auto& kv : m->tuned) fprintf(f, "bucket %d tile %d\n", kv.first, kv.second);
    const bool ok = fclose(f) == 0;
    return ok ? HB_OK : fail(HB_E_INVAL, "cannot write %s", path);
}

hb_status model_load_tuning(hb_model* m, const char* path) {
    std::string arch;
    hb_status st = device_arch(m->device, &arch);
    if (st != HB_OK) return st;
    FILE* f = fopen(path, "r");
    if (!f) return fail(HB_E_INVAL, "cannot read %s", path);
    std::vector<std::string> lines;
    char buf[512];
    while (fgets(buf, sizeof buf, f)) {
        std::string l(buf);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        lines.push_back(l);
    }
    fclose(f);
    if (lines.size() < 3 || lines[0] != "hbtune 1") return fail(HB_E_INVAL, "%s is not a tuning file", path);
    if (lines[1] != "arch " + arch) return fail(HB_E_INVAL, "%s was tuned on %s, this device is %s", path, lines[1].c_str() + 5, arch.c_str());
    if (lines[2] != "model " + model_signature(m)) return fail(HB_E_INVAL, "%s was tuned for another network or precision", path);
    std::map<int, int> tuned;
    for (size_t i = 3; i < lines.size(); i++) {
        int b = -1, id = -1;
        if (sscanf(lines[i].c_str(), "bucket %d tile %d", &b, &id) != 2 || b < 0 || b > 40 || id < 0 ||
            id >= gemm_tile_count() || (fused_tile(id) && !fused_enabled()))
            return fail(HB_E_INVAL, "%s: bad line %zu", path, i + 1);
        tuned[b] = id;
    }
    m->tuned = tuned;
    return HB_OK;
}

}  // namespace hb
