// Serving: continuous batching of depth frames of mixed sizes.
//
// Requests wait in a FIFO queue.  A request is admitted when its slot (its
// outputs, plus its depth when it comes from host memory, plus its counts)
// fits in the HBM budget; admission starts its host-to-device copy on a copy
// stream, or makes it launchable at once when its depth is already in
// device memory (the launch stores its counts, so nothing needs zeroing).
// Whenever fewer than `max_batches_in_flight` launches are queued on the GPU,
// every admitted request whose input is on the device (up to `max_batch`)
// goes into one batch-plan launch on the compute stream.  So new
// requests are admitted and copied while earlier batches run, and each
// launch takes whatever is ready: continuous batching.  A request's slot is
// returned to the budget when the client releases the request.
//
// The scheduling core is independent of the GPU: the HIP backend drives real
// streams and events from a worker thread; the fake backend simulates copy
// and kernel durations on a virtual clock and can fail chosen requests, so
// that admission order, budget accounting and failure isolation are tested
// on the CPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <random>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bn_internal.h"
#include "bnormals.h"

namespace bn {
namespace serve {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, capacity) with coalescing.
class Arena {
  public:
    explicit Arena(size_t capacity) : capacity_(capacity) {
        if (capacity) free_[0] = capacity;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        size_t start = off, size = bytes;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                size += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + bytes == next->first) {
            size += next->second;
            free_.erase(next);
        }
        free_[start] = size;
    }
    size_t used() const { return used_; }
    size_t capacity() const { return capacity_; }

  private:
    size_t capacity_;
    size_t used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> size
};

struct Request {
    uint64_t id = 0;
    int32_t H = 0, W = 0;
    int64_t stride = 0;
    float fx = 0, fy = 0, cx = 0, cy = 0;
    const float *host_depth = nullptr;  // copied into the slot at admission
    const float *dev_depth = nullptr;   // the client's device depth, or the slot's copy
    size_t slot_off = 0, slot_bytes = 0;
    float *normals = nullptr;
    uint8_t *mask = nullptr;
    bn_frame_stats *stats = nullptr;
    int32_t state = BN_REQ_PENDING;
    int32_t status = BN_OK;
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
    uint64_t batch = 0;
    int32_t batch_size = 0;
    hipEvent_t copy_ev = nullptr;  // HIP backend
    double copy_done_at = 0;       // fake backend
    bool released = false;
};

// Slot layout: normals | mask | stats | depth copy (host requests only).
struct SlotLayout {
    size_t normals, mask, stats, depth, total;
};

SlotLayout slot_layout(int32_t H, int32_t W, bool copy_depth) {
    const size_t px = (size_t)H * (size_t)W;
    SlotLayout l;
    l.normals = 0;
    l.mask = align_up(l.normals + 12 * px);
    l.stats = align_up(l.mask + px);
    l.depth = align_up(l.stats + sizeof(bn_frame_stats));
    l.total = l.depth + (copy_depth ? align_up(4 * px) : 0);
    return l;
}

class Backend {
  public:
    virtual ~Backend() {}
    virtual double now() = 0;
    virtual char *base() = 0;  // arena base address
    virtual int start_copy(Request &r) = 0;  // copy a host depth to its slot
    virtual bool copy_done(Request &r) = 0;
    virtual int launch(const std::vector<Request *> &batch, uint64_t id) = 0;
    virtual bool batch_done(uint64_t id) = 0;
    virtual int request_status(const Request &r) { return BN_OK; }
    virtual void forget(Request &r) {}
    virtual bool threaded() = 0;
};

// ----------------------------------------------------------------------------
// HIP backend
// ----------------------------------------------------------------------------
class HipBackend : public Backend {
  public:
    // A ring of max_batches_in_flight + 1 batch plans: the server never has
    // more launches queued than that, so the plan a launch takes is idle and
    // its descriptor table can be rewritten while the other plans' kernels
    // run.  Tables are uploaded on their own stream; the compute stream
    // waits for the upload, not for unrelated host-to-device depth copies.
    int init(size_t budget, int32_t max_batch, int32_t in_flight, const bn_params &params) {
        params_ = params;
        // each request's counts are its own: the batch stores them
        params_.flags &= ~BN_FLAG_COUNTS_ACCUMULATE;
        max_batch_ = max_batch;
        plans_.assign((size_t)in_flight + 1, nullptr);
        if (hipMalloc(&arena_, budget ? budget : 1) != hipSuccess) return BN_ERR_OOM;
        if (hipStreamCreateWithFlags(&copy_, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&upload_, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&compute_, hipStreamNonBlocking) != hipSuccess)
            return BN_ERR_DEVICE;
        return BN_OK;
    }
    ~HipBackend() override {
        if (compute_) (void)hipStreamSynchronize(compute_);
        if (upload_) (void)hipStreamSynchronize(upload_);
        if (copy_) (void)hipStreamSynchronize(copy_);
        for (auto &kv : batches_) (void)hipEventDestroy(kv.second);
        for (hipEvent_t e : uploads_) (void)hipEventDestroy(e);
        for (hipEvent_t e : event_pool_) (void)hipEventDestroy(e);
        for (bn_batch_plan *p : plans_)
            if (p) bn_batch_plan_destroy(p);
        if (copy_) (void)hipStreamDestroy(copy_);
        if (upload_) (void)hipStreamDestroy(upload_);
        if (compute_) (void)hipStreamDestroy(compute_);
        if (arena_) (void)hipFree(arena_);
    }
    double now() override {
        return std::chrono::duration<double>(
                   std::chrono::steady_clock::now().time_since_epoch())
            .count();
    }
    char *base() override { return static_cast<char *>(arena_); }
    bool threaded() override { return true; }

    int start_copy(Request &r) override {
        r.copy_ev = take_event();
        if (!r.copy_ev) return BN_ERR_DEVICE;
        float *dst = const_cast<float *>(r.dev_depth);
        if (hipMemcpy2DAsync(dst, (size_t)r.W * 4, r.host_depth, (size_t)r.stride * 4,
                             (size_t)r.W * 4, (size_t)r.H, hipMemcpyHostToDevice,
                             copy_) != hipSuccess)
            return BN_ERR_DEVICE;
        if (hipEventRecord(r.copy_ev, copy_) != hipSuccess) return BN_ERR_DEVICE;
        return BN_OK;
    }
    bool copy_done(Request &r) override {
        if (!r.copy_ev) return true;
        if (hipEventQuery(r.copy_ev) != hipSuccess) return false;
        give_event(r.copy_ev);
        r.copy_ev = nullptr;
        return true;
    }
    int launch(const std::vector<Request *> &batch, uint64_t id) override {
        std::vector<bn_frame> fr(batch.size());
        for (size_t k = 0; k < batch.size(); ++k) {
            const Request &r = *batch[k];
            fr[k] = bn_frame{r.dev_depth, r.H,       r.W,      r.host_depth ? (int64_t)r.W : r.stride,
                             r.fx,        r.fy,      r.cx,     r.cy,
                             r.normals,   r.mask,    r.stats};
        }
        int rc;
        const size_t j = next_plan_++ % plans_.size();
        bn_batch_plan *&plan = plans_[j];
        if (!plan) {
            // capacity max_batch: later lists reuse the plan's graph
            std::vector<bn_frame> cap(fr);
            while ((int32_t)cap.size() < max_batch_) cap.push_back(fr[0]);
            rc = bn_batch_plan_create(cap.data(), (int32_t)cap.size(), &params_, &plan);
            if (rc != BN_OK) return rc;
        }
        rc = bn_batch_plan_update(plan, fr.data(), (int32_t)fr.size(), upload_);
        if (rc != BN_OK) return rc;
        if (batch_plan_uploads(plan)) {
            hipEvent_t up = take_event();
            if (!up || hipEventRecord(up, upload_) != hipSuccess ||
                hipStreamWaitEvent(compute_, up, 0) != hipSuccess)
                return BN_ERR_DEVICE;
            uploads_.push_back(up);
        }
        // plain launches: a graph replay costs more host time than the
        // kernels of a typical batch of requests take on the GPU
        rc = bn_batch_launch(plan, compute_);
        if (rc != BN_OK) return rc;
        hipEvent_t e = take_event();
        if (!e || hipEventRecord(e, compute_) != hipSuccess) return BN_ERR_DEVICE;
        batches_[id] = e;
        return BN_OK;
    }
    bool batch_done(uint64_t id) override {
        auto it = batches_.find(id);
        if (it == batches_.end()) return true;
        if (hipEventQuery(it->second) != hipSuccess) return false;
        give_event(it->second);
        batches_.erase(it);
        // upload events older than a finished launch are complete too
        while (!uploads_.empty() && hipEventQuery(uploads_.front()) == hipSuccess) {
            give_event(uploads_.front());
            uploads_.pop_front();
        }
        return true;
    }
    void forget(Request &r) override {
        if (r.copy_ev) {
            (void)hipEventSynchronize(r.copy_ev);
            give_event(r.copy_ev);
            r.copy_ev = nullptr;
        }
    }

  private:
    hipEvent_t take_event() {
        if (!event_pool_.empty()) {
            hipEvent_t e = event_pool_.back();
            event_pool_.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
    void give_event(hipEvent_t e) { event_pool_.push_back(e); }

    bn_params params_{};
    int32_t max_batch_ = 1;
    void *arena_ = nullptr;
    hipStream_t copy_ = nullptr, upload_ = nullptr, compute_ = nullptr;
    std::vector<bn_batch_plan *> plans_;
    size_t next_plan_ = 0;
    std::deque<hipEvent_t> uploads_;
    std::unordered_map<uint64_t, hipEvent_t> batches_;
    std::vector<hipEvent_t> event_pool_;
};

// ----------------------------------------------------------------------------
// Fake backend: virtual clock, simulated copy and kernel times, failures
// ----------------------------------------------------------------------------
class FakeBackend : public Backend {
  public:
    FakeBackend(size_t budget, const bn_server_config &c)
        : ns_per_px_(c.fake_ns_per_pixel),
          launch_ns_(c.fake_launch_ns), copy_gbs_(c.fake_copy_gbs > 0 ? c.fake_copy_gbs : 25.0) {}
    double now() override { return t_; }
    // slots are never dereferenced: a fixed, recognisable fake base address
    char *base() override { return reinterpret_cast<char *>(uintptr_t(1) << 40); }
    bool threaded() override { return false; }
    int start_copy(Request &r) override {
        const double bytes = 4.0 * r.H * (double)r.W;
        copy_free_ = std::max(copy_free_, t_) + bytes / (copy_gbs_ * 1e9);
        r.copy_done_at = copy_free_;
        return BN_OK;
    }
    bool copy_done(Request &r) override { return t_ >= r.copy_done_at; }
    int launch(const std::vector<Request *> &batch, uint64_t id) override {
        double px = 0;
        for (const Request *r : batch) px += (double)r->H * r->W;
        gpu_free_ = std::max(gpu_free_, t_) + (launch_ns_ + ns_per_px_ * px) * 1e-9;
        done_at_[id] = gpu_free_;
        return BN_OK;
    }
    bool batch_done(uint64_t id) override {
        auto it = done_at_.find(id);
        if (it == done_at_.end()) return true;
        if (t_ < it->second) return false;
        done_at_.erase(it);
        return true;
    }
    int request_status(const Request &r) override {
        return fail_.count(r.id) ? BN_ERR_DEVICE : BN_OK;
    }
    void advance(double s) { t_ += s; }
    void fail(uint64_t id) { fail_.insert(id); }

  private:
    double t_ = 0, copy_free_ = 0, gpu_free_ = 0;
    double ns_per_px_, launch_ns_, copy_gbs_;
    std::unordered_map<uint64_t, double> done_at_;
    std::set<uint64_t> fail_;
};

// ----------------------------------------------------------------------------
// The scheduler
// ----------------------------------------------------------------------------
class Server {
  public:
    Server(const bn_server_config &c, std::unique_ptr<Backend> be)
        : cfg_(c), be_(std::move(be)), arena_((size_t)c.hbm_budget_bytes) {}

    ~Server() { stop(); }

    void start() {
        if (be_->threaded()) worker_ = std::thread([this] { loop(); });
    }
    void stop() {
        {
            std::lock_guard<std::mutex> g(mu_);
            if (stopping_) return;
            stopping_ = true;
        }
        cv_.notify_all();
        if (worker_.joinable()) worker_.join();
        // let queued work finish before the backend goes away
        std::lock_guard<std::mutex> g(mu_);
        for (auto &kv : all_) be_->forget(*kv.second);
    }

    int submit(const float *depth, bool host, int32_t H, int32_t W, int64_t stride, float fx,
               float fy, float cx, float cy, uint64_t *out_id) {
        // the outputs live in the server's slots: stand-in aligned pointers
        int rc = check_frame_args(depth, H, W, stride, fx, fy, cx, cy,
                                  reinterpret_cast<const float *>(uintptr_t(256)),
                                  reinterpret_cast<const uint8_t *>(uintptr_t(256)));
        if (rc != BN_OK) return rc;
        if (H == 0 || W == 0) return BN_ERR_INVALID_ARG;
        const SlotLayout l = slot_layout(H, W, host);
        if (align_up(l.total) > arena_.capacity()) return BN_ERR_OOM;  // can never fit
        auto r = std::make_unique<Request>();
        r->H = H;
        r->W = W;
        r->stride = stride;
        r->fx = fx;
        r->fy = fy;
        r->cx = cx;
        r->cy = cy;
        if (host)
            r->host_depth = depth;
        else
            r->dev_depth = depth;
        r->slot_bytes = l.total;
        {
            std::lock_guard<std::mutex> g(mu_);
            r->id = ++next_id_;
            r->t_submit = be_->now();
            *out_id = r->id;
            pending_.push_back(r.get());
            all_[r->id] = std::move(r);
            ++n_submitted_;
        }
        cv_.notify_all();
        return BN_OK;
    }

    int query(uint64_t id, bn_request_info *info) {
        std::lock_guard<std::mutex> g(mu_);
        return fill_info(id, info);
    }

    int wait(uint64_t id, double timeout_s, bn_request_info *info) {
        std::unique_lock<std::mutex> g(mu_);
        auto it = all_.find(id);
        if (it == all_.end()) return BN_ERR_INVALID_ARG;
        Request *r = it->second.get();
        const auto deadline = std::chrono::steady_clock::now() +
                              std::chrono::duration<double>(timeout_s < 0 ? 1e9 : timeout_s);
        while (r->state != BN_REQ_DONE && r->state != BN_REQ_FAILED) {
            if (!be_->threaded()) return BN_ERR_UNSUPPORTED;  // drive with bn_server_progress
            if (done_cv_.wait_until(g, deadline) == std::cv_status::timeout &&
                r->state != BN_REQ_DONE && r->state != BN_REQ_FAILED)
                return BN_ERR_TIMEOUT;
        }
        return fill_info(id, info);
    }

    int release(uint64_t id) {
        {
            std::lock_guard<std::mutex> g(mu_);
            auto it = all_.find(id);
            if (it == all_.end()) return BN_ERR_INVALID_ARG;
            Request *r = it->second.get();
            if (r->state != BN_REQ_DONE && r->state != BN_REQ_FAILED) return BN_ERR_UNSUPPORTED;
            if (r->normals) arena_.release(r->slot_off, r->slot_bytes);
            all_.erase(it);
            ++n_released_;
        }
        cv_.notify_all();
        return BN_OK;
    }

    // Scheduling passes until nothing changes at the current time.
    // Runs fn(backend) under the scheduler's lock (the fake backend's clock
    // and failure set are read by every scheduling pass).
    template <class F>
    void locked(F fn) {
        std::lock_guard<std::mutex> g(mu_);
        fn(*be_);
    }

    int progress() {
        std::lock_guard<std::mutex> g(mu_);
        int total = 0;
        for (int k = 0; k < 1000; ++k) {
            const int c = step_locked();
            if (!c) break;
            total += c;
        }
        return total;
    }

    void info(bn_server_stats *s) {
        std::lock_guard<std::mutex> g(mu_);
        s->submitted = n_submitted_;
        s->completed = n_completed_;
        s->failed = n_failed_;
        s->released = n_released_;
        s->batches = n_batches_;
        s->pending = (int64_t)pending_.size();
        s->in_flight_batches = (int64_t)running_.size();
        s->bytes_in_use = (int64_t)arena_.used();
        s->peak_bytes_in_use = (int64_t)peak_used_;
        s->max_batch_seen = max_batch_seen_;
    }

    Backend *backend() { return be_.get(); }

  private:
    int fill_info(uint64_t id, bn_request_info *info) {
        auto it = all_.find(id);
        if (it == all_.end()) return BN_ERR_INVALID_ARG;
        const Request &r = *it->second;
        if (info) {
            info->state = r.state;
            info->status = r.status;
            info->batch_size = r.batch_size;
            info->batch = r.batch;
            info->t_submit = r.t_submit;
            info->t_admit = r.t_admit;
            info->t_launch = r.t_launch;
            info->t_done = r.t_done;
            info->normals = r.normals;
            info->mask = r.mask;
            info->stats = r.stats;
        }
        return BN_OK;
    }

    // One scheduling pass; returns how many state changes it made.
    int step_locked() {
        int changes = 0;
        const double now = be_->now();
        // 1. finished launches
        for (auto it = running_.begin(); it != running_.end();) {
            if (!be_->batch_done(it->first)) {
                ++it;
                continue;
            }
            for (Request *r : it->second) {
                r->t_done = now;
                r->status = be_->request_status(*r);
                r->state = r->status == BN_OK ? BN_REQ_DONE : BN_REQ_FAILED;
                if (r->status == BN_OK)
                    ++n_completed_;
                else
                    ++n_failed_;
            }
            it = running_.erase(it);
            ++changes;
            done_cv_.notify_all();
        }
        // 2. inputs that reached the device
        for (auto it = copying_.begin(); it != copying_.end();) {
            if (be_->copy_done(**it)) {
                (*it)->state = BN_REQ_READY;
                ready_.push_back(*it);
                it = copying_.erase(it);
                ++changes;
            } else {
                ++it;
            }
        }
        // 3. admission, first come first served, by HBM budget
        while (!pending_.empty()) {
            Request *r = pending_.front();
            size_t off;
            if (!arena_.alloc(r->slot_bytes, &off)) break;  // wait for releases
            peak_used_ = std::max(peak_used_, arena_.used());
            const SlotLayout l = slot_layout(r->H, r->W, r->host_depth != nullptr);
            char *b = be_->base() + off;
            r->slot_off = off;
            r->normals = reinterpret_cast<float *>(b + l.normals);
            r->mask = reinterpret_cast<uint8_t *>(b + l.mask);
            r->stats = reinterpret_cast<bn_frame_stats *>(b + l.stats);
            if (r->host_depth) r->dev_depth = reinterpret_cast<const float *>(b + l.depth);
            r->t_admit = now;
            pending_.pop_front();
            if (!r->host_depth) {
                // input already on the device: launchable at once
                r->state = BN_REQ_READY;
                ready_.push_back(r);
                ++changes;
                continue;
            }
            const int rc = be_->start_copy(*r);
            if (rc != BN_OK) {
                r->status = rc;
                r->state = BN_REQ_FAILED;
                r->t_done = now;
                ++n_failed_;
                done_cv_.notify_all();
            } else {
                r->state = BN_REQ_ADMITTED;
                copying_.push_back(r);
            }
            ++changes;
        }
        // 4. launches: everything ready, while the GPU queue has room
        while (!ready_.empty() && (int32_t)running_.size() < cfg_.max_batches_in_flight) {
            std::vector<Request *> batch;
            while (!ready_.empty() && (int32_t)batch.size() < cfg_.max_batch) {
                batch.push_back(ready_.front());
                ready_.pop_front();
            }
            const uint64_t id = ++next_batch_;
            const int rc = be_->launch(batch, id);
            for (Request *r : batch) {
                r->batch = id;
                r->batch_size = (int32_t)batch.size();
                r->t_launch = now;
                if (rc == BN_OK) {
                    r->state = BN_REQ_RUNNING;
                } else {
                    r->status = rc;
                    r->state = BN_REQ_FAILED;
                    r->t_done = now;
                    ++n_failed_;
                }
            }
            if (rc == BN_OK) running_[id] = batch;
            max_batch_seen_ = std::max<int64_t>(max_batch_seen_, (int64_t)batch.size());
            ++n_batches_;
            ++changes;
            if (rc != BN_OK) done_cv_.notify_all();
        }
        return changes;
    }

    void loop() {
        std::unique_lock<std::mutex> g(mu_);
        while (!stopping_) {
            const int changes = step_locked();
            const bool busy = !running_.empty() || !copying_.empty();
            if (changes) continue;
            if (busy) {
                // GPU work in flight: poll its events again shortly
                g.unlock();
                std::this_thread::yield();
                g.lock();
            } else {
                cv_.wait_for(g, std::chrono::milliseconds(2));
            }
        }
    }

    bn_server_config cfg_;
    std::unique_ptr<Backend> be_;
    Arena arena_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::thread worker_;
    bool stopping_ = false;
    uint64_t next_id_ = 0, next_batch_ = 0;
    std::deque<Request *> pending_, ready_;
    std::vector<Request *> copying_;
    std::map<uint64_t, std::vector<Request *>> running_;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all_;
    size_t peak_used_ = 0;
    int64_t n_submitted_ = 0, n_completed_ = 0, n_failed_ = 0, n_released_ = 0, n_batches_ = 0;
    int64_t max_batch_seen_ = 0;
};

}  // namespace serve
}  // namespace bn

using namespace bn;
using namespace bn::serve;

struct bn_server {
    std::unique_ptr<Server> s;
    FakeBackend *fake = nullptr;
};

extern "C" {

int bn_server_create(const bn_server_config *cfg, bn_server **out) {
    if (!out) return BN_ERR_INVALID_ARG;
    *out = nullptr;
    if (!cfg || cfg->hbm_budget_bytes <= 0 || cfg->max_batch < 1 ||
        cfg->max_batches_in_flight < 1)
        return BN_ERR_INVALID_ARG;
    if (cfg->backend != BN_BACKEND_HIP && cfg->backend != BN_BACKEND_FAKE)
        return BN_ERR_INVALID_ARG;
    int rc = check_params_args(&cfg->params);
    if (rc != BN_OK) return rc;
    if (cfg->params.variant != 0) return BN_ERR_UNSUPPORTED;
    bn_server *srv = new (std::nothrow) bn_server();
    if (!srv) return BN_ERR_OOM;
    std::unique_ptr<Backend> be;
    if (cfg->backend == BN_BACKEND_HIP) {
        auto h = std::make_unique<HipBackend>();
        rc = h->init((size_t)cfg->hbm_budget_bytes, cfg->max_batch, cfg->max_batches_in_flight,
                     cfg->params);
        if (rc != BN_OK) {
            delete srv;
            return rc;
        }
        be = std::move(h);
    } else {
        auto f = std::make_unique<FakeBackend>((size_t)cfg->hbm_budget_bytes, *cfg);
        (void)0;
        srv->fake = f.get();
        be = std::move(f);
    }
    srv->s = std::make_unique<Server>(*cfg, std::move(be));
    srv->s->start();
    *out = srv;
    return BN_OK;
}

int bn_server_submit(bn_server *srv, const float *depth, int32_t depth_on_host, int32_t height,
                     int32_t width, int64_t depth_stride, float fx, float fy, float cx, float cy,
                     uint64_t *request_id) {
    if (!srv || !request_id) return BN_ERR_INVALID_ARG;
    return srv->s->submit(depth, depth_on_host != 0, height, width, depth_stride, fx, fy, cx, cy,
                          request_id);
}

int bn_server_query(bn_server *srv, uint64_t request_id, bn_request_info *info) {
    if (!srv) return BN_ERR_INVALID_ARG;
    return srv->s->query(request_id, info);
}

int bn_server_wait(bn_server *srv, uint64_t request_id, double timeout_s,
                   bn_request_info *info) {
    if (!srv) return BN_ERR_INVALID_ARG;
    return srv->s->wait(request_id, timeout_s, info);
}

int bn_server_release(bn_server *srv, uint64_t request_id) {
    if (!srv) return BN_ERR_INVALID_ARG;
    return srv->s->release(request_id);
}

int bn_server_progress(bn_server *srv) {
    if (!srv) return BN_ERR_INVALID_ARG;
    return srv->s->progress();
}

int bn_server_get_stats(bn_server *srv, bn_server_stats *stats) {
    if (!srv || !stats) return BN_ERR_INVALID_ARG;
    srv->s->info(stats);
    return BN_OK;
}

int bn_server_fake_advance(bn_server *srv, double seconds) {
    if (!srv || !srv->fake || !(seconds >= 0)) return BN_ERR_INVALID_ARG;
    FakeBackend *fb = srv->fake;
    srv->s->locked([fb, seconds](Backend &) { fb->advance(seconds); });
    return BN_OK;
}

int bn_server_fake_fail(bn_server *srv, uint64_t request_id) {
    if (!srv || !srv->fake) return BN_ERR_INVALID_ARG;
    FakeBackend *fb = srv->fake;
    srv->s->locked([fb, request_id](Backend &) { fb->fail(request_id); });
    return BN_OK;
}

void bn_server_destroy(bn_server *srv) {
    if (!srv) return;
    srv->s->stop();
    srv->s.reset();
    delete srv;
}

// Open-loop Poisson load: n requests drawn uniformly from `pool` (device
// frames), inter-arrival times exponential with mean 1/rate; each request
// is submitted at its arrival time and released as soon as it completes.
// latency_s[i] = completion - scheduled arrival of request i.
int bn_server_run_poisson(bn_server *srv, const bn_frame *pool, int32_t n_pool, double rate_hz,
                          int32_t n_requests, uint64_t seed, double *latency_s,
                          double *wall_s, int64_t *pixels) {
    if (!srv || !pool || n_pool < 1 || !(rate_hz > 0) || n_requests < 1 || !latency_s)
        return BN_ERR_INVALID_ARG;
    if (srv->fake) return BN_ERR_UNSUPPORTED;
    std::mt19937_64 rng(seed);
    std::exponential_distribution<double> gap(rate_hz);
    std::uniform_int_distribution<int32_t> pick(0, n_pool - 1);
    std::vector<double> arrival(n_requests);
    std::vector<int32_t> which(n_requests);
    double t = 0;
    for (int32_t i = 0; i < n_requests; ++i) {
        t += gap(rng);
        arrival[i] = t;
        which[i] = pick(rng);
    }
    Server &s = *srv->s;
    std::vector<uint64_t> ids(n_requests, 0);
    std::atomic<int32_t> submitted{0};
    std::atomic<int> error{BN_OK};
    const double t0 = s.backend()->now();
    int64_t px = 0;
    for (int32_t i = 0; i < n_requests; ++i)
        px += (int64_t)pool[which[i]].height * pool[which[i]].width;
    // completion side: wait for each request in order, record, release
    std::thread reaper([&] {
        for (int32_t i = 0; i < n_requests; ++i) {
            while (submitted.load(std::memory_order_acquire) <= i && error.load() == BN_OK)
                std::this_thread::yield();
            if (error.load() != BN_OK) return;
            bn_request_info info;
            int rc = s.wait(ids[i], 60.0, &info);
            if (rc != BN_OK || info.state != BN_REQ_DONE) {
                error.store(rc != BN_OK ? rc : info.status);
                return;
            }
            latency_s[i] = info.t_done - (t0 + arrival[i]);
            s.release(ids[i]);
        }
    });
    for (int32_t i = 0; i < n_requests && error.load() == BN_OK; ++i) {
        const double at = t0 + arrival[i];
        while (s.backend()->now() < at) {
        }
        const bn_frame &f = pool[which[i]];
        uint64_t id = 0;
        int rc = s.submit(f.depth, false, f.height, f.width, f.depth_stride, f.fx, f.fy, f.cx,
                          f.cy, &id);
        if (rc != BN_OK) {
            error.store(rc);
            break;
        }
        ids[i] = id;
        submitted.store(i + 1, std::memory_order_release);
    }
    reaper.join();
    if (wall_s) *wall_s = s.backend()->now() - t0;
    if (pixels) *pixels = px;
    return error.load();
}

}  // extern "C"
