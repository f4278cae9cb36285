// Device-resident heuristic network (hb_model) and its forward pass.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "hb.h"

namespace hb {

struct NetSpec {
    int domain = 0, n_in = 0, n_res = 0, n_out = 0, head_kind = 0;
    std::vector<int> dims;
    std::vector<std::vector<float>> tensors;  // file order, float32
};

bool read_weight_file(const char* path, NetSpec* out, const char** why);

struct MatLayer {
    void* Wt = nullptr;         // [groups * N_pad][K_pad] in the operand type (ensembles: members stacked)
    float* bias = nullptr;      // [N_pad]
    float* colscale = nullptr;  // [N_pad] fp8 only
    int K = 0, N = 0, K_pad = 0, N_pad = 0;
    int in_act = 0, out_act = 0, res_act = -1;  // activation tensor ids
    bool res_in_place = false;
    int groups = 1;             // ensemble members evaluated by this layer's one launch
};

struct Workspace {
    void* x = nullptr;  // activation buffers: rows_cap x width_cap elements
    void* t = nullptr;
    int rows_cap = 0;
    unsigned* absmax = nullptr;  // calibration scratch (n_act entries)
    int* sync = nullptr;         // counters of the fused forward kernel (zero between launches), or null
    int rb_cap = 0;              // 32-row blocks the counters cover
    int* tile_ctr = nullptr;     // two zeroed ints: the GEMMs' dynamic tile schedule, or null
};

struct ActCopy {  // copy of one stored activation tensor (hb_model_activation)
    int act;
    uint8_t* out;
    int64_t ld_bytes;
};

struct CalibCapture {
    std::vector<float>* act_max;  // filled per activation tensor
};

}  // namespace hb

struct hb_model {
    int device = 0;
    hb_model_opts opts{};
    hb::NetSpec spec;                 // member 0's (all members share the architecture)
    std::string path;                 // member 0's weight file
    std::vector<std::string> paths;   // every member's weight file
    int members = 1;                  // ensemble size
    int ens_rule = 0;                 // 0 min, 1 sum of the members' outputs
    int P = 0, S = 0, table_rows = 0;
    void* l1_table = nullptr;
    float* l1_bias = nullptr;
    int N1 = 0, N1_pad = 0;
    std::vector<hb::MatLayer> layers;
    void* head_W = nullptr;
    float* head_b = nullptr;
    int K_last_pad = 0;
    int width_cap = 0;
    int n_act = 0;
    std::vector<float> act_scale;
    bool calibrated = false;
    int tile = 0;                       // 0 automatic, else tile id + 1
    int cus = 0;                        // compute units of the device (fused-kernel grid)
    std::map<int, int> tuned;           // batch bucket (log2) -> tile id
    int64_t weight_bytes = 0;
    double flops = 0;
    std::mutex mu;
    std::map<hipStream_t, hb::Workspace> ws;
    std::vector<void*> allocs;
    // per-kernel timing
    bool profiling = false;
    struct Timed { int kind; hipEvent_t a, b; double flops; };  // kind 0 gather, 1 gemm, 2 head
    std::vector<Timed> timed;
    double prof_ms[3] = {0, 0, 0};
    int64_t prof_n[3] = {0, 0, 0};
    double prof_flops = 0;
};

namespace hb {

hb_status model_load(const char* path, const hb_model_opts& o, hb_model** out);
hb_status model_load_members(const std::vector<std::string>& paths, int rule, const hb_model_opts& o, hb_model** out);
void model_free(hb_model* m);
hb_status model_eval(hb_model* m, const uint8_t* d_packed, int64_t n, const int32_t* d_n, int64_t max_n,
                     int32_t* d_h, float* d_raw, hipStream_t s, CalibCapture* cap, int force_tile = -1,
                     const ActCopy* act_copy = nullptr);
hb_status model_eval_noalloc(hb_model* m, const uint8_t* d_packed, int64_t n, int32_t* d_h, float* d_raw,
                             hipStream_t s);
int64_t model_noalloc_capacity(const hb_model* m);
hb_status model_calibrate(hb_model* m, const uint8_t* d_packed, int64_t n);
hb_status model_prepare(hb_model* m, hipStream_t s);  // allocate the stream's workspace now
hb_status model_tune(hb_model* m, const uint8_t* d_packed, int64_t n, double* report, int cap);
hb_status model_autotune(hb_model* m, const uint8_t* d_packed, int64_t n, hb_tune_entry* table, int cap, int* rows,
                         int32_t* recommended);
hb_status model_save_tuning(const hb_model* m, const char* path);
hb_status model_load_tuning(hb_model* m, const char* path);
int choose_tile(const hb_model* m, int64_t M, int N_pad);
bool fused_tile(int id);           // tile ids 10..13: the fused persistent forward kernel
int fused_waves_per_cu(int id);
hb_status model_profile(hb_model* m, bool enable);
hb_status model_profile_read(hb_model* m, hb_profile* out);

}  // namespace hb
