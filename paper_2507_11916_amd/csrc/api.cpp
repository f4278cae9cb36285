// C ABI entry points (include/hb.h): argument checks, error text, dispatch.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "common.hpp"
#include "domain.hpp"
#include "hb.h"
#include "kernels.hpp"
#include "model.hpp"

namespace hb {

static thread_local std::string g_err = "no error";

hb_status fail(hb_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

void clear_error() { g_err = "no error"; }

}  // namespace hb

using namespace hb;

extern "C" {

const char* hb_last_error(void) { return g_err.c_str(); }

int hb_state_bytes(hb_domain d) {
    const Domain* D = domain_of(d);
    return D ? D->state_bytes : -1;
}

int hb_packed_bytes(hb_domain d) {
    const Domain* D = domain_of(d);
    return D ? D->packed_bytes : -1;
}

hb_status hb_encode(hb_domain d, const uint8_t* states, int64_t n, uint8_t* packed_out) {
    const Domain* D = domain_of(d);
    if (!D) return fail(HB_E_INVAL, "unknown domain %d", (int)d);
    if (n < 0 || (n > 0 && (!states || !packed_out))) return fail(HB_E_INVAL, "bad buffers or count");
    for (int64_t i = 0; i < n; i++) {
        const char* why = "";
        if (!valid_state(*D, states + i * D->state_bytes, &why))
            return fail(HB_E_INVAL, "state %lld: %s", (long long)i, why);
        encode(*D, states + i * D->state_bytes, packed_out + i * D->packed_bytes);
    }
    return HB_OK;
}

hb_status hb_decode(hb_domain d, const uint8_t* packed, int64_t n, uint8_t* states_out) {
    const Domain* D = domain_of(d);
    if (!D) return fail(HB_E_INVAL, "unknown domain %d", (int)d);
    if (n < 0 || (n > 0 && (!packed || !states_out))) return fail(HB_E_INVAL, "bad buffers or count");
    for (int64_t i = 0; i < n; i++) decode(*D, packed + i * D->packed_bytes, states_out + i * D->state_bytes);
    return HB_OK;
}

hb_status hb_apply_moves(hb_domain d, const int8_t* moves, int64_t count, int32_t len, uint8_t* states_out) {
    const Domain* D = domain_of(d);
    if (!D) return fail(HB_E_INVAL, "unknown domain %d", (int)d);
    if (count < 0 || len < 0 || (count > 0 && (!states_out || (len > 0 && !moves))))
        return fail(HB_E_INVAL, "bad buffers or count");
    uint8_t cur[kMaxStateBytes], nxt[kMaxStateBytes];
    for (int64_t i = 0; i < count; i++) {
        goal_state(*D, cur);
        for (int j = 0; j < len; j++) {
            const int m = moves[i * len + j];
            if (m < 0) break;
            if (!apply_move(*D, cur, m, nxt))
                return fail(HB_E_INVAL, "row %lld move %d (%d) is not applicable", (long long)i, j, m);
            std::memcpy(cur, nxt, (size_t)D->state_bytes);
        }
        std::memcpy(states_out + i * D->state_bytes, cur, (size_t)D->state_bytes);
    }
    return HB_OK;
}

hb_status hb_manhattan(hb_domain d, const uint8_t* states, int64_t n, int32_t* out) {
    const Domain* D = domain_of(d);
    if (!D || D->id == HB_RUBIK3) return fail(HB_E_INVAL, "Manhattan distance needs a sliding-tile domain");
    if (n < 0 || (n > 0 && (!states || !out))) return fail(HB_E_INVAL, "bad buffers or count");
    for (int64_t i = 0; i < n; i++) out[i] = manhattan(*D, states + i * D->state_bytes);
    return HB_OK;
}

hb_status hb_pdb_build_corner(int k, int threads, hb_pdb** out) {
    if (!out) return fail(HB_E_INVAL, "null output");
    if (k < 1 || k > 8) return fail(HB_E_INVAL, "k must be in 1..8");
    hb_pdb* p = new (std::nothrow) hb_pdb;
    if (!p) return fail(HB_E_NOMEM, "pdb");
    try {
        if (!corner_pdb_build(k, threads, &p->corner)) { delete p; return fail(HB_E_INVAL, "bad k"); }
    } catch (const std::bad_alloc&) {
        delete p;
        return fail(HB_E_NOMEM, "pattern database table");
    }
    *out = p;
    return HB_OK;
}

hb_status hb_pdb_build_stp_additive(const int32_t* group_of_tile, int threads, hb_pdb** out) {
    if (!out) return fail(HB_E_INVAL, "null output");
    if (!group_of_tile) return fail(HB_E_INVAL, "null grouping");
    hb_pdb* p = new (std::nothrow) hb_pdb;
    if (!p) return fail(HB_E_NOMEM, "pdb");
    p->kind = 1;
    try {
        if (!stp_apdb_build(group_of_tile, threads, &p->stp)) {
            delete p;
            return fail(HB_E_INVAL, "tiles 1..15 must form groups 0..n-1 of 1 to 8 tiles");
        }
    } catch (const std::bad_alloc&) {
        delete p;
        return fail(HB_E_NOMEM, "pattern database table");
    }
    *out = p;
    return HB_OK;
}

hb_status hb_pdb_lookup(const hb_pdb* pdb, const uint8_t* states, int64_t n, int32_t* out) {
    if (!pdb) return fail(HB_E_INVAL, "null pdb");
    if (n < 0 || (n > 0 && (!states || !out))) return fail(HB_E_INVAL, "bad buffers or count");
    const Domain* D = domain_of(pdb->kind == 0 ? HB_RUBIK3 : HB_STP4);
    const int sb = D->state_bytes;
    for (int64_t i = 0; i < n; i++) {
        const char* why = "";
        if (!valid_state(*D, states + i * sb, &why)) return fail(HB_E_INVAL, "state %lld: %s", (long long)i, why);
        out[i] = pdb->kind == 0 ? pdb->corner.lookup(states + i * sb) : pdb->stp.lookup(states + i * sb);
    }
    return HB_OK;
}

hb_status hb_pdb_value_counts(const hb_pdb* pdb, int64_t* counts, int32_t n_counts, int32_t* max_value) {
    if (!pdb) return fail(HB_E_INVAL, "null pdb");
    if (n_counts < 1 || !counts) return fail(HB_E_INVAL, "bad counts buffer");
    std::fill(counts, counts + n_counts, int64_t{0});
    int vmax = 0;
    auto add = [&](const std::vector<uint8_t>& table) {
        for (uint8_t v : table) {
            if (v == 255) continue;  // unreachable index (for k = 8 corners the last twist is implied)
            if (v < n_counts) counts[v]++;
            vmax = std::max(vmax, (int)v);
        }
    };
    if (pdb->kind == 0) add(pdb->corner.table);
    else
        for (const auto& t : pdb->stp.tables) add(t);
    if (max_value) *max_value = vmax;
    return HB_OK;
}

void hb_pdb_free(hb_pdb* pdb) { delete pdb; }

hb_status hb_model_load(const char* weights_path, const hb_model_opts* opts, hb_model** out) {
    if (!weights_path || !out) return fail(HB_E_INVAL, "null path or output");
    hb_model_opts o{HB_FP32, 0, HB_OUT_REG_FLOOR, 0.99f, 0.f, 0, 16384};
    if (opts) o = *opts;
    if (o.max_batch < 0 || o.max_batch > (1 << 22)) return fail(HB_E_INVAL, "max_batch out of range");
    try {
        return model_load(weights_path, o, out);
    } catch (const std::bad_alloc&) {
        return fail(HB_E_NOMEM, "host allocation while loading the model");
    }
}

hb_status hb_model_load_ensemble(const char* const* weights_paths, int k, hb_ensemble_rule rule,
                                 const hb_model_opts* opts, hb_model** out) {
    if (!weights_paths || !out || k < 1) return fail(HB_E_INVAL, "null paths or output, or k < 1");
    hb_model_opts o{HB_FP32, 0, HB_OUT_REG_FLOOR, 0.99f, 0.f, 0, 16384};
    if (opts) o = *opts;
    if (o.max_batch < 0 || o.max_batch > (1 << 22)) return fail(HB_E_INVAL, "max_batch out of range");
    std::vector<std::string> paths;
    for (int i = 0; i < k; i++) {
        if (!weights_paths[i]) return fail(HB_E_INVAL, "null path %d", i);
        paths.emplace_back(weights_paths[i]);
    }
    try {
        return model_load_members(paths, (int)rule, o, out);
    } catch (const std::bad_alloc&) {
        return fail(HB_E_NOMEM, "host allocation while loading the model");
    }
}

void hb_model_free(hb_model* m) { model_free(m); }

hb_status hb_model_get_info(const hb_model* m, hb_model_info* out) {
    if (!m || !out) return fail(HB_E_INVAL, "null argument");
    std::memset(out, 0, sizeof *out);
    out->domain = m->spec.domain;
    out->n_in = m->spec.n_in;
    out->n_dense = (int)m->spec.dims.size();
    out->n_res = m->spec.n_res;
    out->n_out = m->spec.n_out;
    out->head_kind = m->spec.head_kind;
    out->n_act = m->n_act;
    out->prec = (int)m->opts.prec;
    for (int i = 0; i < out->n_dense && i < 8; i++) out->dims[i] = m->spec.dims[i];
    out->weight_bytes = m->weight_bytes;
    out->flops_per_eval = m->flops;
    return HB_OK;
}

hb_status hb_model_calibrate(hb_model* m, const uint8_t* d_packed, int64_t n) {
    if (!m || (n > 0 && !d_packed)) return fail(HB_E_INVAL, "null argument");
    return model_calibrate(m, d_packed, n);
}

hb_status hb_model_get_act_scales(const hb_model* m, float* out, int cap) {
    if (!m || !out || cap < m->n_act) return fail(HB_E_INVAL, "need room for %d scales", m ? m->n_act : 0);
    for (int a = 0; a < m->n_act; a++) out[a] = m->act_scale[a];
    return HB_OK;
}

hb_status hb_model_set_act_scales(hb_model* m, const float* scales, int n) {
    if (!m || !scales || n != m->n_act) return fail(HB_E_INVAL, "expected %d scales", m ? m->n_act : 0);
    for (int a = 0; a < n; a++)
        if (!(scales[a] > 0.f) || !std::isfinite(scales[a])) return fail(HB_E_INVAL, "scale %d is not positive", a);
    for (int a = 0; a < n; a++) m->act_scale[a] = scales[a];
    m->calibrated = true;
    return HB_OK;
}

hb_status hb_eval_batch(hb_model* m, const uint8_t* d_packed, int64_t n, int32_t* d_h_out, float* d_raw_out,
                        void* stream) {
    if (!m) return fail(HB_E_INVAL, "null model");
    if (n < 0) return fail(HB_E_INVAL, "negative count");
    if (n == 0) return HB_OK;
    if (!d_packed || !d_h_out) return fail(HB_E_INVAL, "null device buffer");
    return model_eval(m, d_packed, n, nullptr, 0, d_h_out, d_raw_out, (hipStream_t)stream, nullptr);
}

hb_status hb_model_activation(hb_model* m, const uint8_t* d_packed, int64_t n, int act, void* d_out,
                              int64_t ld_out, void* stream) {
    if (!m || !d_packed || !d_out) return fail(HB_E_INVAL, "null argument");
    if (n < 0) return fail(HB_E_INVAL, "negative count");
    if (act < 0 || act >= m->n_act) return fail(HB_E_INVAL, "activation index %d outside 0..%d", act, m->n_act - 1);
    const int width = act == 0 ? m->members * m->N1_pad : m->layers[act - 1].N_pad * m->layers[act - 1].groups;
    if (ld_out < width) return fail(HB_E_INVAL, "row stride %lld below the activation width %d", (long long)ld_out, width);
    if (n == 0) return HB_OK;
    const int eb = m->opts.prec == HB_FP32 ? 4 : m->opts.prec == HB_BF16 ? 2 : 1;
    int32_t* d_h = nullptr;
    HB_HIP(hipSetDevice(m->device));
    HB_HIP(hipMalloc((void**)&d_h, (size_t)n * 4));
    ActCopy ac{act, static_cast<uint8_t*>(d_out), ld_out * eb};
    hb_status st = model_eval(m, d_packed, n, nullptr, 0, d_h, nullptr, (hipStream_t)stream, nullptr, -1, &ac);
    const hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(d_h);
    if (st == HB_OK && e != hipSuccess) return fail(HB_E_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return st;
}

hb_status hb_eval_batch_noalloc(hb_model* m, const uint8_t* d_packed, int64_t n, int32_t* d_h_out,
                                float* d_raw_out, void* stream) {
    if (!m) return fail(HB_E_INVAL, "null model");
    if (n < 0) return fail(HB_E_INVAL, "negative count");
    if (n > 0 && (!d_packed || !d_h_out)) return fail(HB_E_INVAL, "null device buffer");
    return model_eval_noalloc(m, d_packed, n, d_h_out, d_raw_out, (hipStream_t)stream);
}

hb_status hb_eval_batch_dev_n(hb_model* m, const uint8_t* d_packed, const int32_t* d_n, int64_t max_n,
                              int32_t* d_h_out, float* d_raw_out, void* stream) {
    if (!m || !d_n || !d_packed || !d_h_out) return fail(HB_E_INVAL, "null argument");
    if (max_n < 0) return fail(HB_E_INVAL, "negative max_n");
    return model_eval(m, d_packed, 0, d_n, max_n, d_h_out, d_raw_out, (hipStream_t)stream, nullptr);
}

hb_status hb_model_set_tile(hb_model* m, int tile_id) {
    if (!m || tile_id < 0 || tile_id > gemm_tile_count()) return fail(HB_E_INVAL, "tile id out of range");
    if (tile_id > 0 && fused_tile(tile_id - 1) && !fused_enabled())
        return fail(HB_E_UNSUPPORTED, "tile %d (the fused persistent forward kernel) is switched off", tile_id);
    m->tile = tile_id;
    return HB_OK;
}

hb_status hb_model_tune(hb_model* m, const uint8_t* d_packed, int64_t n, double* report, int cap) {
    if (!m || !d_packed) return fail(HB_E_INVAL, "null argument");
    return model_tune(m, d_packed, n, report, cap);
}

hb_status hb_model_autotune(hb_model* m, const uint8_t* d_packed, int64_t n, hb_tune_entry* table, int cap,
                            int* rows, int32_t* recommended_batch) {
    if (!m || !d_packed) return fail(HB_E_INVAL, "null argument");
    return model_autotune(m, d_packed, n, table, cap, rows, recommended_batch);
}

hb_status hb_model_tile_for(const hb_model* m, int64_t n, int* tile) {
    if (!m || !tile || n < 1) return fail(HB_E_INVAL, "bad argument");
    int id = -1;
    for (const MatLayer& L : m->layers) {  // every layer uses the same rule; report the first
        id = choose_tile(m, n, L.N_pad);
        break;
    }
    *tile = id + 1;
    return HB_OK;
}

hb_status hb_model_save_tuning(const hb_model* m, const char* path) {
    if (!m || !path) return fail(HB_E_INVAL, "null argument");
    return model_save_tuning(m, path);
}

hb_status hb_model_load_tuning(hb_model* m, const char* path) {
    if (!m || !path) return fail(HB_E_INVAL, "null argument");
    return model_load_tuning(m, path);
}

hb_status hb_model_profile(hb_model* m, int enable) {
    if (!m) return fail(HB_E_INVAL, "null model");
    return model_profile(m, enable != 0);
}

hb_status hb_model_profile_read(hb_model* m, hb_profile* out) {
    if (!m || !out) return fail(HB_E_INVAL, "null argument");
    return model_profile_read(m, out);
}

}  // extern "C"
