// Parallel cost-bounded DFS with batched heuristic evaluation: Batch IDA* and
// Batch BTS (cbdfs_solve in include/hb.h).
//
// Structure (SingleGPU Batch CB-DFS):
//  * GenerateWork: the tree below the start is built to depth d_init once; the
//    states at depth d_init are the work units of the shared work queue
//    (AIDA*'s initial data partitioning and distributed node assignment).
//  * Each iteration (cost bound T) runs `threads` search threads.  A thread
//    keeps work_num subtrees (Parallel CB-DFS algorithm) and round-robins over
//    them; a subtree whose top node still waits for its heuristic is skipped
//    (Subtree expansion algorithm), so one thread keeps several subtrees
//    feeding the batch.
//  * Generated children are parked in a shared batch (a host slab); a batch
//    thread seals a slab when it is full, when the timeout passes since its
//    first record, or when every search thread is waiting on h; it copies the
//    slab to the GPU, evaluates the network and writes each h back into the
//    owning node record (ProcessBatch).  Several slabs exist so that the search
//    threads keep filling while one is evaluated.  On the GPU the copy in, the
//    forward pass and the copy out of a batch are one hipGraph launch: a graph
//    per power-of-two size bucket, captured on first use, reads the state count
//    from device memory, so one graph serves every batch size of its bucket.
//  * Counting matches serial IDA*: in iteration T a node of the initial tree is
//    generated iff every strict ancestor has f <= T and is not the goal; such a
//    node with f <= T is expanded (or is the solution), with f > T it is pruned
//    and feeds the next bound; a generated depth-d_init node becomes a subtree
//    root whose own f test happens inside the subtree search.  Hence per
//    iteration (expanded, generated) equal the serial search's whenever the
//    heuristic values are the same.
// Real-valued heuristics (HB_H_NN_REAL): a node record holds the float bits of
// h = max(0, y - offset); f = g + h and the bounds are doubles (exact, as g is
// an integer and h a float), IDA*'s next bound is the smallest pruned f and BTS
// bisects over real bounds.  Integer heuristics run the same code with
// integer-valued doubles.
// Readings of the pseudo-code: the expansion test is f = g + h <= T (the proof's
// expansion condition), pruned nodes are popped and their f feeds the next
// bound, the round-robin counter wraps modulo workNum, and `miss` counts the
// distinct terminated slots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_set>
#include <vector>

#include "common.hpp"
#include "domain.hpp"
#include "hb.h"
#include "model.hpp"

namespace hb {
namespace {

using Clock = std::chrono::steady_clock;
constexpr int32_t kPending = INT32_MIN;
constexpr int kMaxDepth = 510;     // deepest path a subtree search may hold
constexpr int64_t kFlushEvery = 64; // expansions between publications of a thread's count

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

struct NodeRec {
    std::atomic<int32_t> h{kPending};  // network / batched-classic value
    int32_t hc = 0;                     // classic value
    int32_t parent = -1;                // index in the slot stack, -1 = subtree root
    int16_t g = 0;
    int8_t move = -1;
    uint8_t expanded = 0;
    uint8_t s[kMaxStateBytes];
};

// ------------------------------------------------------------------ batcher
struct Slab {
    uint8_t* packed = nullptr;  // pinned, cap * pb
    int32_t* h = nullptr;       // pinned, cap
    std::vector<NodeRec*> owners;
    int reserved = 0;
    std::atomic<int> committed{0};
    double t_first = 0;
};

struct Shared;

class Batcher {
public:
    // flush_mode: 0 full slab or timeout; 1 also when every search thread
    // waits on h; 2 also whenever the batch thread is free (eager).
    // gpu_depth: batches on the GPU at once (1 or 2); with 2 the next batch is
    // staged and launched while the previous one is still being evaluated.
    Batcher(Shared* sh, int cap, int n_slabs, double timeout_s, int flush_mode, bool graphs, int gpu_depth)
        : sh_(sh), cap_(cap), timeout_(timeout_s), idle_flush_(flush_mode >= 1), eager_(flush_mode >= 2),
          use_graphs_(graphs), n_slabs_(n_slabs),
          depth_(std::max(1, std::min(kMaxGpuDepth, std::min(gpu_depth, n_slabs - 1)))) {}
    hb_status init();
    void start();
    void stop();
    ~Batcher();
    // Reserve up to k consecutive records in the current slab; blocks while no
    // slab is free.  Returns the slab and first index; *got receives the count.
    Slab* reserve(int k, int* first, int* got);
    void commit(Slab* s, int n) { s->committed.fetch_add(n, std::memory_order_release); }
    void drain();  // flush and wait until every reserved record has been evaluated
    // Flush-when-idle bookkeeping.  gen() advances every time a slab's values
    // are handed back (before the values are written).  A search thread marks
    // itself idle with the generation it read before a full round over its
    // subtrees found nothing to do; it counts as idle only while no slab has
    // returned since, so a thread that was just given results is never taken
    // for idle.
    int64_t gen() const { return gen_.load(); }
    void set_active(int n) {
        if (n > idle_cap_) {
            idle_gen_.reset(new std::atomic<int64_t>[n]);
            idle_cap_ = n;
        }
        for (int t = 0; t < n; t++) idle_gen_[t].store(kBusy);
        n_search_ = n;
    }
    // The notification is sent under the mutex: the batch thread either
    // already waits (and wakes) or has yet to test all_idle() (and sees it).
    void mark_idle(int t, int64_t g) {
        idle_gen_[t].store(g);
        if (idle_flush_ && all_idle()) wake();
    }
    void mark_busy(int t) { idle_gen_[t].store(kBusy); }
    void thread_done(int t) {
        idle_gen_[t].store(kDone);
        if (idle_flush_ && all_idle()) wake();
    }
    hb_status eval_now(const std::vector<uint8_t>& packed, int64_t n, std::vector<int32_t>* h);  // synchronous
    std::atomic<int64_t> evals{0}, batches{0};
    double gpu_busy = 0;
    hb_status error = HB_OK;
    std::string error_text;

private:
    void wake() {
        std::lock_guard<std::mutex> lk(mu_);
        cv_.notify_all();
    }
    struct Launched {  // a batch on the GPU (batch thread only)
        Slab* s;
        int n, k;          // states, buffer set
    };
    void loop();
    hb_status process(Slab* s, int n);   // synchronous: evaluate and hand back
    void hand_back(Slab* s, int n);      // write the values to their owners
    void complete(Slab* s, hb_status st);  // under mu_: slab free again, errors recorded
    hb_status gpu_launch(int k, const uint8_t* packed, int n);
    void gpu_collect(int k, int n, int32_t* h_out);
    hb_status gpu_eval(const uint8_t* packed, int n, int32_t* h_out);
    hb_status capture(int k, int bi);
    Shared* sh_;
    int cap_;
    double timeout_;
    bool idle_flush_, eager_;
    bool use_graphs_;
    int n_slabs_;
    static constexpr int kMaxGpuDepth = 2;
    int depth_;
    std::vector<std::unique_ptr<Slab>> slabs_;
    std::vector<Slab*> free_;
    Slab* cur_ = nullptr;
    int in_flight_ = 0;  // sealed, not yet returned
    std::mutex mu_;
    std::condition_variable cv_;
    std::thread th_;
    bool all_idle() const {
        const int64_t g = gen_.load();
        bool any = false;
        for (int t = 0; t < n_search_; t++) {
            const int64_t v = idle_gen_[t].load();
            if (v == kDone) continue;
            if (v != g) return false;
            any = true;
        }
        return any;
    }
    static constexpr int64_t kBusy = -1, kDone = -2;
    static constexpr int kSpin = 64;  // polling rounds (16 yields each) before sleeping
    bool stop_ = false;
    bool draining_ = false;
    std::atomic<int64_t> gen_{0};
    std::unique_ptr<std::atomic<int64_t>[]> idle_gen_;
    int idle_cap_ = 0, n_search_ = 0;
    // GPU side: [count | pad | packed states] staged in pinned memory and
    // copied as one block; h comes back into pinned memory.
    // One buffer set per batch that may be on the GPU at once; every batch
    // runs on the one stream, so they are evaluated in launch order and share
    // the model's activation workspace.
    static constexpr int kHdr = 256;
    uint8_t* stage_[kMaxGpuDepth] = {};    // pinned, kHdr + cap * pb
    int32_t* h_stage_[kMaxGpuDepth] = {};  // pinned, cap
    uint8_t* d_stage_[kMaxGpuDepth] = {};  // device, kHdr + cap * pb
    int32_t* d_h_[kMaxGpuDepth] = {};
    float* d_raw_[kMaxGpuDepth] = {};      // device, cap: the network's y - offset (real-valued h)
    hipEvent_t done_[kMaxGpuDepth] = {};   // recorded after a batch's copy back
    hipStream_t stream_ = nullptr;
    std::vector<int> buckets_;                          // ascending batch capacities, the last is cap
    std::vector<hipGraphExec_t> execs_[kMaxGpuDepth];   // per buffer set and bucket, null until captured
    bool graphs_ok_ = true;
    std::deque<Launched> launched_;  // oldest first
    int next_k_ = 0;
    double busy_from_ = 0;           // start of the GPU's current busy period
};

struct Shared {
    const Domain* D = nullptr;
    hb_combine combine = HB_H_CLASSIC;
    hb_classic classic = HB_CLASSIC_MD;
    const hb_pdb* pdb = nullptr;
    hb_model* model = nullptr;
    bool uses_batches = false;
    bool uses_gpu = false;
    bool real = false;  // h values are float bits (HB_H_NN_REAL)
    int classic_h(const uint8_t* s) const;
    double hval(int32_t bits) const {
        if (!real) return (double)bits;
        float f;
        std::memcpy(&f, &bits, 4);
        return (double)f;
    }
};

// Float bits of a real-valued heuristic value max(0, v) (+0.0 for v <= 0 or NaN).
static int32_t real_bits(float v) {
    const float h = v > 0.f ? v : 0.f;
    int32_t b;
    std::memcpy(&b, &h, 4);
    return b;
}

int Shared::classic_h(const uint8_t* s) const {
    switch (classic) {
        case HB_CLASSIC_MD: return manhattan(*D, s);
        case HB_CLASSIC_PDB: return pdb->kind == 0 ? pdb->corner.lookup(s) : pdb->stp.lookup(s);
        default: return 0;
    }
}

hb_status Batcher::init() {
    const int pb = sh_->D->packed_bytes;
    for (int i = 0; i < n_slabs_; i++) {
        auto s = std::make_unique<Slab>();
        s->owners.resize(cap_);
        if (sh_->uses_gpu) {
            HB_HIP(hipHostMalloc((void**)&s->packed, (size_t)cap_ * pb, hipHostMallocDefault));
            HB_HIP(hipHostMalloc((void**)&s->h, (size_t)cap_ * 4, hipHostMallocDefault));
        } else {
            s->packed = new uint8_t[(size_t)cap_ * pb];
            s->h = new int32_t[cap_];
        }
        free_.push_back(s.get());
        slabs_.push_back(std::move(s));
    }
    cur_ = free_.back();
    free_.pop_back();
    if (sh_->uses_gpu) {
        HB_HIP(hipSetDevice(sh_->model->device));
        HB_HIP(hipStreamCreate(&stream_));
        for (int k = 0; k < depth_; k++) {
            HB_HIP(hipHostMalloc((void**)&stage_[k], kHdr + (size_t)cap_ * pb, hipHostMallocDefault));
            HB_HIP(hipHostMalloc((void**)&h_stage_[k], (size_t)cap_ * 4, hipHostMallocDefault));
            HB_HIP(hipMalloc((void**)&d_stage_[k], kHdr + (size_t)cap_ * pb));
            HB_HIP(hipMalloc((void**)&d_h_[k], (size_t)cap_ * 4));
            if (sh_->real) HB_HIP(hipMalloc((void**)&d_raw_[k], (size_t)cap_ * 4));
            HB_HIP(hipEventCreateWithFlags(&done_[k], hipEventDisableTiming));
        }
        hb_status st = model_prepare(sh_->model, stream_);  // workspace exists before any capture
        if (st != HB_OK) return st;
        for (int b = 32; b < cap_; b *= 2) buckets_.push_back(b);
        buckets_.push_back(cap_);
        for (int k = 0; k < depth_; k++) execs_[k].assign(buckets_.size(), nullptr);
    }
    return HB_OK;
}

Batcher::~Batcher() {
    stop();
    for (auto& s : slabs_) {
        if (sh_->uses_gpu) {
            (void)hipHostFree(s->packed);
            (void)hipHostFree(s->h);
        } else {
            delete[] s->packed;
            delete[] s->h;
        }
    }
    if (sh_->uses_gpu) {
        if (stream_) (void)hipStreamSynchronize(stream_);
        for (int k = 0; k < kMaxGpuDepth; k++) {
            for (hipGraphExec_t e : execs_[k])
                if (e) (void)hipGraphExecDestroy(e);
            (void)hipHostFree(stage_[k]);
            (void)hipHostFree(h_stage_[k]);
            (void)hipFree(d_stage_[k]);
            (void)hipFree(d_h_[k]);
            (void)hipFree(d_raw_[k]);
            if (done_[k]) (void)hipEventDestroy(done_[k]);
        }
        if (stream_) (void)hipStreamDestroy(stream_);
    }
}

void Batcher::start() { th_ = std::thread([this] { loop(); }); }

void Batcher::stop() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    if (th_.joinable()) th_.join();
}

Slab* Batcher::reserve(int k, int* first, int* got) {
    std::unique_lock<std::mutex> lk(mu_);
    while (!cur_ && !stop_) cv_.wait(lk);
    if (!cur_) { *got = 0; return nullptr; }
    Slab* s = cur_;
    const int i = s->reserved;
    const int n = std::min(k, cap_ - i);
    if (i == 0) s->t_first = now_s();
    s->reserved += n;
    *first = i;
    *got = n;
    if (s->reserved == cap_) cv_.notify_all();
    return s;
}

void Batcher::drain() {
    std::unique_lock<std::mutex> lk(mu_);
    draining_ = true;
    while (!stop_ && ((cur_ && cur_->reserved > 0) || in_flight_ > 0 || !cur_)) {
        cv_.notify_all();
        cv_.wait_for(lk, std::chrono::microseconds(200));
        if (error != HB_OK) break;
    }
    draining_ = false;
}

// Captures copy-in, forward pass and copy-out of buffer set k for batches of
// up to buckets_[bi] states; the state count is read on the device.
hb_status Batcher::capture(int k, int bi) {
    const int B = buckets_[bi];
    const int pb = sh_->D->packed_bytes;
    hipGraph_t g = nullptr;
    HB_HIP(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipMemcpyAsync(d_stage_[k], stage_[k], kHdr + (size_t)B * pb, hipMemcpyHostToDevice, stream_);
    hb_status st = e == hipSuccess ? model_eval(sh_->model, d_stage_[k] + kHdr, 0,
                                                reinterpret_cast<const int32_t*>(d_stage_[k]), B, d_h_[k], d_raw_[k],
                                                stream_, nullptr)
                                   : fail(HB_E_DEVICE, "capture: %s", hipGetErrorString(e));
    if (st == HB_OK) {
        const void* src = sh_->real ? (const void*)d_raw_[k] : (const void*)d_h_[k];
        e = hipMemcpyAsync(h_stage_[k], src, (size_t)B * 4, hipMemcpyDeviceToHost, stream_);
        if (e != hipSuccess) st = fail(HB_E_DEVICE, "capture: %s", hipGetErrorString(e));
    }
    const hipError_t ee = hipStreamEndCapture(stream_, &g);
    if (st == HB_OK && ee != hipSuccess) st = fail(HB_E_DEVICE, "end capture: %s", hipGetErrorString(ee));
    if (st == HB_OK) {
        e = hipGraphInstantiate(&execs_[k][bi], g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            execs_[k][bi] = nullptr;
            st = fail(HB_E_DEVICE, "graph instantiation: %s", hipGetErrorString(e));
        }
    }
    if (g) (void)hipGraphDestroy(g);
    return st;
}

// Stages a batch in buffer set k and launches it (a graph launch when graphs
// are on, else the same copy / forward / copy sequence issued directly); done_[k]
// is recorded behind it.  Returns without waiting.
hb_status Batcher::gpu_launch(int k, const uint8_t* packed, int n) {
    const int pb = sh_->D->packed_bytes;
    std::memcpy(stage_[k] + kHdr, packed, (size_t)n * pb);
    *reinterpret_cast<int32_t*>(stage_[k]) = n;
    bool launched = false;
    if (use_graphs_ && graphs_ok_ && !sh_->model->profiling) {
        const int bi = (int)(std::lower_bound(buckets_.begin(), buckets_.end(), n) - buckets_.begin());
        if (!execs_[k][bi] && capture(k, bi) != HB_OK) {
            graphs_ok_ = false;  // keep searching with direct launches
            (void)hipGetLastError();
        }
        if (execs_[k][bi]) {
            HB_HIP(hipGraphLaunch(execs_[k][bi], stream_));
            launched = true;
        }
    }
    if (!launched) {
        HB_HIP(hipMemcpyAsync(d_stage_[k], stage_[k], kHdr + (size_t)n * pb, hipMemcpyHostToDevice, stream_));
        hb_status st = model_eval(sh_->model, d_stage_[k] + kHdr, n, nullptr, 0, d_h_[k], d_raw_[k], stream_, nullptr);
        if (st != HB_OK) return st;
        const void* src = sh_->real ? (const void*)d_raw_[k] : (const void*)d_h_[k];
        HB_HIP(hipMemcpyAsync(h_stage_[k], src, (size_t)n * 4, hipMemcpyDeviceToHost, stream_));
    }
    HB_HIP(hipEventRecord(done_[k], stream_));
    return HB_OK;
}

// The values of a finished batch in buffer set k (done_[k] has completed).
void Batcher::gpu_collect(int k, int n, int32_t* h_out) {
    if (sh_->real) {
        const float* v = reinterpret_cast<const float*>(h_stage_[k]);
        for (int i = 0; i < n; i++) h_out[i] = real_bits(v[i]);
    } else {
        std::memcpy(h_out, h_stage_[k], (size_t)n * 4);
    }
}

// One batch, waited for (the main thread's evaluation of the initial tree).
hb_status Batcher::gpu_eval(const uint8_t* packed, int n, int32_t* h_out) {
    const double t0 = now_s();
    hb_status st = gpu_launch(0, packed, n);
    if (st != HB_OK) return st;
    HB_HIP(hipEventSynchronize(done_[0]));
    gpu_collect(0, n, h_out);
    gpu_busy += now_s() - t0;
    return HB_OK;
}

void Batcher::hand_back(Slab* s, int n) {
    gen_.fetch_add(1);  // before any value becomes visible: idle marks taken so far are stale
    for (int i = 0; i < n; i++) {
        NodeRec* r = s->owners[i];
        int32_t v = s->h[i];
        if (sh_->combine == HB_H_MIN_NN_CLASSIC) v = std::min(v, r->hc);
        r->h.store(v, std::memory_order_release);
    }
    evals += n;
    batches += 1;
}

hb_status Batcher::process(Slab* s, int n) {
    const int pb = sh_->D->packed_bytes;
    if (sh_->uses_gpu) {
        hb_status st = gpu_eval(s->packed, n, s->h);
        if (st != HB_OK) return st;
    } else {
        uint8_t st[kMaxStateBytes];
        for (int i = 0; i < n; i++) {
            decode(*sh_->D, s->packed + (size_t)i * pb, st);
            s->h[i] = sh_->classic_h(st);
        }
    }
    hand_back(s, n);
    return HB_OK;
}

void Batcher::complete(Slab* s, hb_status st) {
    if (st != HB_OK && error == HB_OK) {
        error = st;
        error_text = hb_last_error();
    }
    s->reserved = 0;
    s->committed.store(0, std::memory_order_relaxed);
    if (!cur_) cur_ = s;
    else free_.push_back(s);
    in_flight_--;
}

// The batch thread.  It seals the filling slab when it is full, its oldest
// record has waited `timeout`, every search thread waits on h (idle flush),
// or (eager) whenever it may launch, as long as fewer than depth_ batches are
// on the GPU; it hands back the oldest launched batch as soon as its values
// have arrived.  With depth 1 each batch is evaluated and handed back before
// the next is sealed.
void Batcher::loop() {
    if (sh_->uses_gpu) (void)hipSetDevice(sh_->model->device);
    const bool pipelined = sh_->uses_gpu && depth_ > 1;
    std::unique_lock<std::mutex> lk(mu_);
    int spin = 0;
    for (;;) {
        if (stop_ || error != HB_OK) {
            // drain() has handed back every batch before a regular stop; after an
            // error the launched batches are waited for and dropped
            if (!launched_.empty()) {
                lk.unlock();
                (void)hipStreamSynchronize(stream_);
                lk.lock();
                while (!launched_.empty()) {
                    complete(launched_.front().s, HB_OK);
                    launched_.pop_front();
                }
            }
            stop_ = true;
            cv_.notify_all();
            return;
        }
        if (!launched_.empty()) {
            const hipError_t q = hipEventQuery(done_[launched_.front().k]);
            if (q != hipErrorNotReady) {
                const Launched f = launched_.front();
                launched_.pop_front();
                lk.unlock();
                const double t = now_s();
                gpu_busy += t - busy_from_;
                busy_from_ = t;
                hb_status st = HB_OK;
                if (q == hipSuccess) {
                    gpu_collect(f.k, f.n, f.s->h);
                    hand_back(f.s, f.n);
                } else {
                    st = fail(HB_E_DEVICE, "batch evaluation: %s", hipGetErrorString(q));
                }
                lk.lock();
                complete(f.s, st);
                cv_.notify_all();
                spin = 0;
                continue;
            }
        }
        const bool can_seal = (int)launched_.size() < (pipelined ? depth_ : 1) && cur_ && cur_->reserved > 0;
        if (can_seal) {
            const bool full = cur_->reserved == cap_;
            const double left = cur_->t_first + timeout_ - now_s();
            const bool idle = idle_flush_ && all_idle();
            // eager: the GPU may take a batch now, so whatever arrived goes at once
            if (full || left <= 0 || idle || eager_ || draining_) {
                Slab* s = cur_;
                const int n = s->reserved;
                if (!free_.empty()) {
                    cur_ = free_.back();
                    free_.pop_back();
                } else {
                    cur_ = nullptr;
                }
                in_flight_++;
                lk.unlock();
                cv_.notify_all();
                while (s->committed.load(std::memory_order_acquire) < n) std::this_thread::yield();
                hb_status st = HB_OK;
                if (pipelined) {
                    const int k = next_k_;
                    if (launched_.empty()) busy_from_ = now_s();
                    st = gpu_launch(k, s->packed, n);
                    lk.lock();
                    if (st == HB_OK) {
                        launched_.push_back(Launched{s, n, k});
                        next_k_ = (k + 1) % depth_;
                    } else {
                        complete(s, st);
                        cv_.notify_all();
                    }
                } else {
                    st = process(s, n);
                    lk.lock();
                    complete(s, st);
                    cv_.notify_all();
                }
                spin = 0;
                continue;
            }
        }
        if (!launched_.empty()) {
            // a batch is on the GPU: poll it (and the flush conditions) without sleeping
            lk.unlock();
            for (int i = 0; i < 4; i++) std::this_thread::yield();
            lk.lock();
            continue;
        }
        if (cur_ && cur_->reserved > 0) {
            // Poll briefly first (a sleeping batch thread adds a wake-up to every
            // round trip), then sleep until notified by reserve() (full slab),
            // mark_idle() or thread_done(), or the timeout.
            if (idle_flush_ && spin < kSpin) {
                lk.unlock();
                for (int i = 0; i < 16 && !all_idle(); i++) std::this_thread::yield();
                lk.lock();
                spin++;
                continue;
            }
            const double left = cur_->t_first + timeout_ - now_s();
            cv_.wait_for(lk, std::chrono::microseconds(std::max<int64_t>(1, std::min<int64_t>(1000, (int64_t)(left * 1e6)))));
        } else {
            cv_.wait_for(lk, std::chrono::microseconds(200));
        }
    }
}

hb_status Batcher::eval_now(const std::vector<uint8_t>& packed, int64_t n, std::vector<int32_t>* h) {
    const int pb = sh_->D->packed_bytes;
    h->resize(n);
    std::lock_guard<std::mutex> lk(mu_);  // the batch thread is idle while the main thread does this
    for (int64_t off = 0; off < n; off += cap_) {
        const int c = (int)std::min<int64_t>(cap_, n - off);
        if (sh_->uses_gpu) {
            hb_status st = gpu_eval(packed.data() + off * pb, c, h->data() + off);
            if (st != HB_OK) return st;
        } else {
            uint8_t st[kMaxStateBytes];
            for (int i = 0; i < c; i++) {
                decode(*sh_->D, packed.data() + (off + i) * pb, st);
                (*h)[off + i] = sh_->classic_h(st);
            }
        }
        evals += c;
        batches += 1;
    }
    return HB_OK;
}

// ------------------------------------------------------------- prefix tree
struct PNode {
    uint8_t s[kMaxStateBytes];
    int32_t parent;
    int16_t g;
    int8_t move;
    uint8_t goal;
    double h;        // pruning value
    int32_t h_eval;  // network / batched value as stored in a node record
    int32_t hc;
    int32_t n_children;
};

struct Solver;

// --------------------------------------------------------------- one search
struct IterOut {
    int64_t expanded = 0, generated = 0;
    int64_t batches = 0, evals = 0;  // batches and states evaluated during the iteration
    double next = INFINITY;
    bool found = false, exceeded = false, aborted = false, timed_out = false;
    std::vector<int8_t> path;
};

struct Solver {
    Shared sh;
    const cbdfs_params* P = nullptr;
    int threads = 1;
    std::vector<PNode> tree;  // initial tree, BFS order
    int d_init = 0;
    int first_frontier = 0;   // index of the first depth-d_init node
    std::unique_ptr<Batcher> batcher;
    double t_start = 0;
    int64_t total_expanded = 0, total_generated = 0;
    int64_t peak_nodes = 0;
    int stack_cap = 0;
    // per-search state
    std::atomic<int> work_next{0};
    std::vector<int> work;
    std::atomic<bool> stop{false};
    std::atomic<bool> found_flag{false};
    std::atomic<int64_t> expanded_shared{0};
    std::atomic<bool> exceeded_flag{false};
    std::atomic<bool> depth_error{false};
    std::atomic<bool> timed_out{false};
    double deadline = 0;  // wall-clock stop (now_s() scale), 0 = none
    int64_t limit = -1;
    bool stop_at_goal = true;
    double bound = 0;
    std::mutex sol_mu;
    std::vector<int8_t> sol_path;
    bool budget_hit = false;
    // Node stacks of each search thread.  A thread that stops early can leave
    // children parked in a batch; the batch thread later writes their h through
    // the slab's owner pointers, so the stacks live until run() has drained the
    // batcher, not just until their thread returns.
    std::vector<std::vector<std::unique_ptr<NodeRec[]>>> stacks_of;

    double prune_h(const NodeRec& r) const {
        switch (sh.combine) {
            case HB_H_FIXED_TREE: case HB_H_CLASSIC: return (double)r.hc;
            default: return sh.hval(r.h.load(std::memory_order_relaxed));
        }
    }
    hb_status build_tree(const uint8_t* start);
    IterOut run(double T, int64_t lim, bool stop_goal);
    void thread_main(int tid, IterOut* out, int64_t* peak);
};

hb_status Solver::build_tree(const uint8_t* start) {
    const Domain& D = *sh.D;
    PNode root{};
    std::memcpy(root.s, start, D.state_bytes);
    root.parent = -1;
    root.g = 0;
    root.move = -1;
    tree.clear();
    tree.push_back(root);
    int level_begin = 0, level_end = 1;
    // Automatic depth: the early iterations of IDA* reach only a small part of
    // the initial tree, so the tree is grown until it holds many more work
    // units than there are subtree slots (at most about 3M nodes).
    const int want = P->d_init >= 0 ? -1 : (int)std::min<int64_t>(1 << 20, 1024LL * threads * std::max(1, P->work_num));
    int depth = 0;
    const int max_depth = P->d_init >= 0 ? P->d_init : 40;
    while (depth < max_depth) {
        if (want > 0 && level_end - level_begin >= want) break;
        if ((int64_t)tree.size() + (int64_t)(level_end - level_begin) * D.n_actions > 3000000) break;
        for (int i = level_begin; i < level_end; i++) {
            int nc = 0;
            if (is_goal(D, tree[i].s)) { tree[i].n_children = 0; continue; }  // goals are never expanded
            for (int a = 0; a < D.n_actions; a++) {
                if (!move_allowed(D, tree[i].move, a)) continue;
                PNode c{};
                if (!apply_move(D, tree[i].s, a, c.s)) continue;
                c.parent = i;
                c.g = (int16_t)(tree[i].g + 1);
                c.move = (int8_t)a;
                tree.push_back(c);
                nc++;
            }
            tree[i].n_children = nc;
        }
        level_begin = level_end;
        level_end = (int)tree.size();
        depth++;
        if (level_end == level_begin) break;
    }
    d_init = depth;
    first_frontier = level_begin;
    for (size_t i = first_frontier; i < tree.size(); i++) tree[i].n_children = 0;
    // Heuristic values of every node of the initial tree (one bulk evaluation).
    for (auto& n : tree) {
        n.goal = is_goal(D, n.s);
        n.hc = (sh.combine == HB_H_NN || sh.combine == HB_H_NN_REAL) ? 0 : sh.classic_h(n.s);
    }
    if (sh.uses_batches) {
        std::vector<uint8_t> packed(tree.size() * D.packed_bytes);
        for (size_t i = 0; i < tree.size(); i++) encode(D, tree[i].s, packed.data() + i * D.packed_bytes);
        std::vector<int32_t> h;
        hb_status st = batcher->eval_now(packed, (int64_t)tree.size(), &h);
        if (st != HB_OK) return st;
        for (size_t i = 0; i < tree.size(); i++) {
            int32_t v = h[i];
            if (sh.combine == HB_H_MIN_NN_CLASSIC) v = std::min(v, tree[i].hc);
            tree[i].h_eval = v;
        }
    } else {
        for (auto& n : tree) n.h_eval = n.hc;
    }
    for (auto& n : tree) n.h = (sh.combine == HB_H_FIXED_TREE || sh.combine == HB_H_CLASSIC) ? (double)n.hc : sh.hval(n.h_eval);
    return HB_OK;
}

void Solver::thread_main(int tid, IterOut* out, int64_t* peak) {
    const Domain& D = *sh.D;
    const int W = std::max(1, P->work_num);
    const int pb = D.packed_bytes;
    std::vector<std::unique_ptr<NodeRec[]>>& stacks = stacks_of[tid];  // freed by run() after drain()
    stacks.resize(W);
    std::vector<int> top(W, 0);
    for (int w = 0; w < W; w++) stacks[w].reset(new NodeRec[stack_cap]);
    std::vector<char> terminated(W, 0);
    std::vector<char> has_work(W, 0);
    int64_t expanded = 0, generated = 0, flushed = 0;
    double next = INFINITY;
    int64_t local_peak = 0;
    int miss = 0;
    bool idle = false;

    auto load_work = [&](int w) -> bool {
        const int k = work_next.fetch_add(1);
        if (k >= (int)work.size()) return false;
        const PNode& pn = tree[work[k]];
        NodeRec& r = stacks[w][0];
        std::memcpy(r.s, pn.s, D.state_bytes);
        r.g = pn.g;
        r.move = pn.move;
        r.parent = -(work[k] + 2);  // encodes the initial-tree node for path reconstruction
        r.expanded = 0;
        r.hc = pn.hc;
        r.h.store(pn.h_eval, std::memory_order_relaxed);
        top[w] = 1;
        return true;
    };
    auto record_solution = [&](int w, int idx) {
        std::vector<int8_t> tail;
        int i = idx;
        int root_node = -1;
        while (i >= 0) {
            const NodeRec& r = stacks[w][i];
            if (r.parent < 0) {
                root_node = -(r.parent + 2);
                break;
            }
            tail.push_back(r.move);
            i = r.parent;
        }
        std::vector<int8_t> head;
        for (int t = root_node; t > 0; t = tree[t].parent) head.push_back(tree[t].move);
        std::reverse(head.begin(), head.end());
        std::reverse(tail.begin(), tail.end());
        head.insert(head.end(), tail.begin(), tail.end());
        std::lock_guard<std::mutex> lk(sol_mu);
        if (!found_flag.load()) {
            sol_path = head;
            found_flag.store(true);
        }
    };

    // Returns 0 = blocked on h, 1 = progress, 2 = slot finished.
    auto do_iteration = [&](int w) -> int {
        NodeRec* S = stacks[w].get();
        for (;;) {
            if (top[w] == 0) return 2;
            NodeRec& r = S[top[w] - 1];
            if (r.expanded) { top[w]--; continue; }
            const int32_t hv = r.h.load(std::memory_order_acquire);
            if (hv == kPending) return 0;  // heuristic not ready: switch subtree
            const double f = (double)r.g + prune_h(r);
            if (f > bound) {
                next = std::min(next, f);
                top[w]--;
                continue;
            }
            if (is_goal(D, r.s)) {
                record_solution(w, top[w] - 1);
                if (stop_at_goal) stop.store(true);
                top[w]--;
                continue;
            }
            // Expansion limit (Batch BTS): local counts are published every
            // kFlushEvery expansions, so the search stops within
            // threads * kFlushEvery expansions of the limit.  The node about to
            // be expanded would make the total exceed the limit when the
            // observed total has reached it, so "exceeded" is declared only
            // when the complete search's count is larger than the limit.
            if (limit >= 0) {
                if (expanded - flushed >= kFlushEvery) {
                    expanded_shared.fetch_add(expanded - flushed);
                    flushed = expanded;
                }
                if (expanded_shared.load(std::memory_order_relaxed) + (expanded - flushed) >= limit) {
                    expanded_shared.fetch_add(expanded - flushed);
                    flushed = expanded;
                    exceeded_flag.store(true);
                    stop.store(true);
                    return 2;
                }
            }
            if (deadline > 0 && (expanded & 255) == 0 && now_s() > deadline) {
                timed_out.store(true);
                stop.store(true);
                return 2;
            }
            if (top[w] + D.n_actions > stack_cap) {  // deeper than kMaxDepth
                depth_error.store(true);
                stop.store(true);
                return 2;
            }
            r.expanded = 1;
            expanded++;
            const int parent = top[w] - 1;
            int kids[kMaxActions];
            int nk = 0;
            for (int a = 0; a < D.n_actions; a++) {
                if (!move_allowed(D, r.move, a)) continue;
                NodeRec& c = S[top[w]];
                if (!apply_move(D, r.s, a, c.s)) continue;
                c.g = (int16_t)(r.g + 1);
                c.move = (int8_t)a;
                c.parent = parent;
                c.expanded = 0;
                c.hc = (sh.combine == HB_H_NN || sh.combine == HB_H_NN_REAL) ? 0 : sh.classic_h(c.s);
                if (sh.uses_batches) c.h.store(kPending, std::memory_order_relaxed);
                else c.h.store(c.hc, std::memory_order_relaxed);
                kids[nk++] = top[w];
                top[w]++;
            }
            generated += nk;
            local_peak = std::max<int64_t>(local_peak, top[w]);
            if (sh.uses_batches) {
                int done = 0;
                while (done < nk) {
                    int first = 0, got = 0;
                    Slab* s = batcher->reserve(nk - done, &first, &got);
                    if (!s) { stop.store(true); return 2; }
                    for (int j = 0; j < got; j++) {
                        NodeRec& c = S[kids[done + j]];
                        encode(D, c.s, s->packed + (size_t)(first + j) * pb);
                        s->owners[first + j] = &c;
                    }
                    batcher->commit(s, got);
                    done += got;
                }
            }
            return 1;
        }
    };

    for (int w = 0; w < W; w++) has_work[w] = load_work(w);
    for (int w = 0; w < W; w++)
        if (!has_work[w]) { terminated[w] = 1; miss++; }
    int counter = 0;
    int stalled = 0;
    int64_t streak_gen = 0, marked_gen = INT64_MIN;
    while (miss < W) {
        if (stop.load(std::memory_order_relaxed)) break;
        const int64_t g_before = batcher ? batcher->gen() : 0;
        int res = 0;  // a terminated slot neither progresses nor blocks
        if (!terminated[counter]) {
            res = do_iteration(counter);
            if (res == 2) {
                if (stop.load(std::memory_order_relaxed)) break;
                if (!load_work(counter)) {
                    terminated[counter] = 1;
                    miss++;
                }
                res = 1;
            }
        }
        if (res == 1) {
            stalled = 0;
            if (idle) { batcher->mark_busy(tid); idle = false; }
        } else {
            if (stalled == 0) streak_gen = g_before;
            if (++stalled >= W) {
                // a full round found every subtree of this thread waiting on h
                if (batcher && (!idle || marked_gen != streak_gen)) {
                    batcher->mark_idle(tid, streak_gen);
                    idle = true;
                    marked_gen = streak_gen;
                }
                std::this_thread::yield();
                stalled = 0;
            }
        }
        counter = (counter + 1) % W;
    }
    if (batcher) batcher->thread_done(tid);
    if (limit >= 0) expanded_shared.fetch_add(expanded - flushed);
    std::lock_guard<std::mutex> lk(sol_mu);
    out->expanded += expanded;
    out->generated += generated;
    out->next = std::min(out->next, next);
    *peak += local_peak;
}

IterOut Solver::run(double T, int64_t lim, bool stop_goal) {
    IterOut out;
    const int64_t batches0 = batcher ? batcher->batches.load() : 0;
    const int64_t evals0 = batcher ? batcher->evals.load() : 0;
    bound = T;
    limit = lim;
    stop_at_goal = stop_goal;
    stop.store(false);
    found_flag.store(false);
    expanded_shared.store(0);
    sol_path.clear();
    exceeded_flag.store(false);
    depth_error.store(false);
    timed_out.store(false);
    // Accounting on the initial tree.  A node is generated in this iteration
    // iff its parent is generated, is not the goal and has f <= T (the tree is
    // in breadth-first order, so parents precede children).
    const int N = (int)tree.size();
    std::vector<char> reach(N, 0);
    if (N > 0) reach[0] = 1;
    for (int i = 1; i < N; i++) {
        const PNode& n = tree[i];
        const PNode& p = tree[n.parent];
        reach[i] = reach[n.parent] && !p.goal && (p.g + p.h <= T) && n.parent < first_frontier;
    }
    work.clear();
    for (int i = 0; i < N; i++) {
        if (!reach[i]) continue;
        const PNode& n = tree[i];
        if (i >= first_frontier) { work.push_back(i); continue; }
        const double f = (double)n.g + n.h;
        if (f > T) { out.next = std::min(out.next, f); continue; }
        if (n.goal) {
            if (!found_flag.load()) {
                std::vector<int8_t> p;
                for (int t = i; t > 0; t = tree[t].parent) p.push_back(tree[t].move);
                std::reverse(p.begin(), p.end());
                sol_path = p;
                found_flag.store(true);
                if (stop_goal) stop.store(true);
            }
            continue;
        }
        out.expanded++;
        out.generated += n.n_children;
    }
    if (limit >= 0) {
        expanded_shared.store(out.expanded);
        if (out.expanded > limit) exceeded_flag.store(true);
    }
    // A path never holds more than T + 1 expanded nodes (h >= 0), each leaving
    // at most n_actions children on the stack.
    const int depth_cap = T <= 0 ? 0 : T >= kMaxDepth ? kMaxDepth : (int)std::floor(T);
    stack_cap = (depth_cap + 2) * sh.D->n_actions + 2;
    work_next.store(0);
    int64_t peak = 0;
    if (!stop.load() && !exceeded_flag.load() && !work.empty()) {
        std::vector<std::thread> pool;
        if (batcher) batcher->set_active(threads);
        stacks_of.clear();
        stacks_of.resize(threads);
        for (int t = 0; t < threads; t++) pool.emplace_back([this, t, &out, &peak] { thread_main(t, &out, &peak); });
        for (auto& th : pool) th.join();
        // Every parked record gets its value (or the batcher stops on an
        // error) before the stacks holding the records are released.
        if (batcher) batcher->drain();
        stacks_of.clear();
    }
    peak_nodes = std::max(peak_nodes, peak);
    if (limit >= 0 && expanded_shared.load() > limit) exceeded_flag.store(true);
    out.exceeded = exceeded_flag.load();
    out.timed_out = timed_out.load();
    if (depth_error.load()) out.aborted = true;
    if (batcher && batcher->error != HB_OK) out.aborted = true;
    out.found = found_flag.load();
    out.path = sol_path;
    if (batcher) {
        out.batches = batcher->batches.load() - batches0;
        out.evals = batcher->evals.load() - evals0;
    }
    total_expanded += out.expanded;
    total_generated += out.generated;
    return out;
}

}  // namespace
}  // namespace hb

using namespace hb;

extern "C" {

void cbdfs_params_default(cbdfs_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->batch_size = 8000;
    p->work_num = 8;
    p->d_init = -1;
    p->timeout_us = 4000;
    p->n_slabs = 4;
    p->flush_when_idle = 1;
    p->gpu_depth = 1;
    p->node_limit = 0;
    p->time_limit_s = 0;
    p->bts_b0 = 10000;
    p->bts_c1 = 2;
    p->bts_c2 = 8;
    p->bts_root_plus_one = 1;
    p->dedup_frontier = 0;
    p->complete_final_iter = 0;
    p->start_bound = -1;
    p->max_iters = 1000;
    p->use_graphs = 1;
}

void cbdfs_result_free(cbdfs_result* r) {
    if (!r) return;
    delete[] r->path;
    delete[] r->iters;
    r->path = nullptr;
    r->iters = nullptr;
}

hb_status cbdfs_solve(hb_domain d, const uint8_t* start, const hb_heuristic* h, hb_algo algo, int threads,
                      const cbdfs_params* p_in, cbdfs_result* out) {
    if (!out) return fail(HB_E_INVAL, "null result");
    std::memset(out, 0, sizeof *out);
    out->cost = -1;
    const Domain* D = domain_of(d);
    if (!D) return fail(HB_E_INVAL, "unknown domain %d", (int)d);
    if (!start || !h) return fail(HB_E_INVAL, "null start or heuristic");
    if (algo != HB_IDA && algo != HB_BTS) return fail(HB_E_INVAL, "unknown algorithm");
    if (threads < 1 || threads > 1024) return fail(HB_E_INVAL, "threads must be in 1..1024");
    const char* why = "";
    if (!solvable(*D, start, &why)) return fail(HB_E_INVAL, "start state: %s", why);
    cbdfs_params P;
    cbdfs_params_default(&P);
    if (p_in) P = *p_in;
    if (P.batch_size < 1 || P.work_num < 1 || P.n_slabs < 2 || P.timeout_us < 0 || P.max_iters < 1 ||
        P.flush_when_idle < 0 || P.flush_when_idle > 2 || P.gpu_depth < 1 || P.gpu_depth > 2)
        return fail(HB_E_INVAL, "bad parameters");
    if (algo == HB_BTS && (P.bts_b0 < 1 || P.bts_c1 < 1 || P.bts_c2 <= P.bts_c1))
        return fail(HB_E_INVAL, "bad BTS parameters (need b0 >= 1, c2 > c1 >= 1)");

    auto S = std::make_unique<Solver>();
    S->sh.D = D;
    S->sh.combine = h->combine;
    S->sh.classic = h->classic;
    S->sh.pdb = h->pdb;
    S->sh.model = h->model;
    if ((int)h->combine < 0 || (int)h->combine > 5) return fail(HB_E_INVAL, "unknown combine mode");
    if (h->classic == HB_CLASSIC_MD && d == HB_RUBIK3) return fail(HB_E_INVAL, "Manhattan distance needs a sliding tile");
    if (h->classic == HB_CLASSIC_PDB &&
        (!h->pdb || !((h->pdb->kind == 0 && d == HB_RUBIK3) || (h->pdb->kind == 1 && d == HB_STP4))))
        return fail(HB_E_INVAL, "PDB heuristic needs a corner PDB for the cube or an additive PDB for the 15-puzzle");
    const bool nn = h->combine == HB_H_NN || h->combine == HB_H_MIN_NN_CLASSIC || h->combine == HB_H_FIXED_TREE ||
                    h->combine == HB_H_NN_REAL;
    if (nn) {
        if (!h->model) return fail(HB_E_INVAL, "this combine mode needs a model");
        if (h->model->spec.domain != (int)d) return fail(HB_E_INVAL, "model domain does not match");
    }
    if (h->combine == HB_H_NN_REAL &&
        (h->model->opts.out != HB_OUT_REG_REAL || h->model->spec.n_out != 1))
        return fail(HB_E_INVAL, "a real-valued heuristic needs a regression model in the REAL output mode");
    if (h->combine == HB_H_NN_REAL && h->model->opts.combine_md != 0)
        return fail(HB_E_INVAL, "a real-valued heuristic uses the network's value alone: load the model with combine_md = 0");
    S->sh.real = h->combine == HB_H_NN_REAL;
    S->sh.uses_gpu = nn;
    S->sh.uses_batches = nn || h->combine == HB_H_CLASSIC_BATCHED;
    S->P = &P;
    S->threads = threads;
    S->t_start = now_s();
    S->deadline = P.time_limit_s > 0 ? S->t_start + P.time_limit_s : 0;
    if (S->sh.uses_batches) {
        int cap = P.batch_size;
        if (nn) cap = std::min(cap, h->model->opts.max_batch);
        S->batcher = std::make_unique<Batcher>(&S->sh, cap, P.n_slabs, P.timeout_us * 1e-6, P.flush_when_idle,
                                               P.use_graphs != 0, P.gpu_depth);
        hb_status st = S->batcher->init();
        if (st != HB_OK) return st;
    }
    hb_status st = S->build_tree(start);
    if (st != HB_OK) return st;
    if (S->batcher) S->batcher->start();

    std::vector<cbdfs_iter> iters;
    std::vector<int8_t> path;
    hb_status result = HB_E_BUDGET;
    int32_t cost = -1;
    const double h_root = S->tree[0].h;
    const bool real = S->sh.real;
    auto over_time = [&] { return P.time_limit_s > 0 && now_s() - S->t_start > P.time_limit_s; };
    auto over_nodes = [&] { return P.node_limit > 0 && S->total_expanded >= P.node_limit; };
    auto remaining = [&]() -> int64_t { return P.node_limit > 0 ? std::max<int64_t>(0, P.node_limit - S->total_expanded) : -1; };
    auto push_iter = [&](double b, int64_t lim, const IterOut& o, bool complete) {
        cbdfs_iter it{};
        it.bound = (int32_t)std::floor(b);
        it.bound_real = b;
        it.limit = lim;
        it.expanded = o.expanded;
        it.generated = o.generated;
        it.complete = complete;
        it.found = o.found;
        it.batches = o.batches;
        it.evals = o.evals;
        iters.push_back(it);
    };

    if (algo == HB_IDA) {
        double bound = P.start_bound >= 0 ? (double)P.start_bound : h_root;
        for (int k = 0; k < P.max_iters; k++) {
            const int64_t lim = remaining();
            const bool stop_goal = !P.complete_final_iter;
            IterOut o = S->run(bound, lim, stop_goal);
            if (o.aborted) { result = HB_E_DEVICE; break; }
            const bool complete = !o.exceeded && !o.timed_out && !(o.found && stop_goal);
            push_iter(bound, lim, o, complete);
            if (o.found) {  // any solution at bound T costs T, the optimum (no smaller bound had one)
                cost = (int32_t)o.path.size();
                path = o.path;
                result = HB_OK;
                break;
            }
            if (o.timed_out || o.exceeded || over_nodes() || over_time()) { result = HB_E_BUDGET; break; }
            if (std::isinf(o.next)) { result = HB_E_NOSOLUTION; break; }
            bound = o.next;
        }
    } else {
        // Budgeted Tree Search (reading stated in the oracle and the design notes).
        int64_t b = P.bts_b0;
        // Integer heuristics bisect over integers; real-valued ones over reals.
        double lo_next = h_root;
        double probe = P.start_bound >= 0 ? (double)P.start_bound : h_root + (P.bts_root_plus_one ? 1 : 0);
        double hi = INFINITY;
        double step = 1;
        for (int k = 0; k < P.max_iters; k++) {
            if (over_nodes() || over_time()) { result = HB_E_BUDGET; break; }
            bool unlimited = false;
            if (!std::isinf(hi) && lo_next >= hi) { probe = hi; unlimited = true; }
            int64_t lim = unlimited ? -1 : (int64_t)P.bts_c2 * b;
            const int64_t rem = remaining();
            const bool budget_cut = rem >= 0 && (lim < 0 || rem < lim);
            if (budget_cut) lim = rem;
            IterOut o = S->run(probe, lim, false);
            if (o.aborted) { result = HB_E_DEVICE; break; }
            if (o.timed_out) {
                push_iter(probe, lim, o, false);
                result = HB_E_BUDGET;
                break;
            }
            push_iter(probe, lim, o, !o.exceeded);
            if (o.exceeded && budget_cut) { result = HB_E_BUDGET; break; }
            if (!o.exceeded && o.found) {
                hi = probe;
                if (lo_next >= probe) {
                    cost = (int32_t)o.path.size();
                    path = o.path;
                    result = HB_OK;
                    break;
                }
            } else if (!o.exceeded) {
                if (std::isinf(o.next)) { result = HB_E_NOSOLUTION; break; }
                lo_next = o.next;
                if (unlimited || o.expanded >= (int64_t)P.bts_c1 * b) {
                    if (o.expanded > b) b = o.expanded;
                    hi = INFINITY;
                    step = 1;
                    probe = lo_next;
                    continue;
                }
                if (std::isinf(hi)) {
                    probe = lo_next + step - 1;
                    if (probe < lo_next) probe = lo_next;
                    step *= 2;
                    continue;
                }
            } else {
                hi = probe;
            }
            if (!std::isinf(hi) && lo_next < hi)
                probe = real ? lo_next + (hi - lo_next) / 2 : lo_next + std::floor((hi - lo_next) / 2);
        }
    }
    std::string err_text = S->batcher ? S->batcher->error_text : "";
    double gpu = 0;
    int64_t evals = 0, batches = 0;
    if (S->batcher) {
        S->batcher->stop();
        gpu = S->batcher->gpu_busy;
        evals = S->batcher->evals.load();
        batches = S->batcher->batches.load();
    }
    out->cost = cost;
    out->path_len = (int32_t)path.size();
    out->path = new int8_t[std::max<size_t>(1, path.size())];
    std::copy(path.begin(), path.end(), out->path);
    out->n_iter = (int32_t)iters.size();
    out->iters = new cbdfs_iter[std::max<size_t>(1, iters.size())];
    std::copy(iters.begin(), iters.end(), out->iters);
    out->evals = evals;
    out->batches = batches;
    out->mean_batch = batches ? (double)evals / batches : 0.0;
    out->wall_s = now_s() - S->t_start;
    out->gpu_busy_s = gpu;
    out->expanded = S->total_expanded;
    out->generated = S->total_generated;
    out->frontier = (int32_t)(S->tree.size() - S->first_frontier);
    out->peak_nodes = S->peak_nodes;
    if (result == HB_E_DEVICE) return fail(HB_E_DEVICE, "batch evaluation failed: %s", err_text.c_str());
    if (result == HB_E_BUDGET) return fail(HB_E_BUDGET, "node, time or iteration limit reached");
    if (result == HB_E_NOSOLUTION) return fail(HB_E_NOSOLUTION, "no solution");
    clear_error();
    return HB_OK;
}

}  // extern "C"
