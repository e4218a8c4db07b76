// server.cpp -- serving loop: continuous batching of evaluation requests.
//
// Requests are admitted in arrival order to free worker slots once their HBM
// footprint fits in the remaining budget of one device pool; every slot owns a
// context with its own stream, so admitted requests overlap on the device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "vlg.h"

namespace vlg {
size_t evaluation_footprint(vlg_formula *f, const vlg_image *img);
int evaluate_all_on(vlg_ctx *c, vlg_formula *f, const vlg_image *img, void *const *outs, void *ws, size_t ws_size);
const char *last_error_text();
int set_last_error(int code, const std::string &msg);
size_t formula_outputs(const vlg_formula *f);
}  // namespace vlg

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over one device buffer; offsets aligned to 256 bytes.
class Pool {
  public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
        reserved_ = 0;
    }
    bool alloc(size_t n, size_t *off) {
        n = (n + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n;
            const size_t start = it->first + n;
            free_.erase(it);
            if (rest) free_[start] = rest;
            reserved_ += n;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = (n + 255) & ~(size_t)255;
        reserved_ -= n;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t reserved() const { return reserved_; }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t reserved_ = 0;
};

struct Request {
    int64_t id = 0;
    vlg_formula *f = nullptr;
    const vlg_image *img = nullptr;
    std::vector<void *> outs;
    size_t footprint = 0;
    Clock::time_point t_submit, t_admit, t_done;
    bool done = false;
    int status = VLG_OK;
    std::string err;
};

}  // namespace

struct vlg_server {
    int device = 0;
    size_t budget = 0;
    void *pool_mem = nullptr;
    Pool pool;
    std::vector<vlg_ctx *> slots;
    std::vector<std::thread> workers;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<int64_t, std::shared_ptr<Request>> reqs;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    int64_t next_id = 1;
    int inflight = 0;
    vlg_server_stats st{};

    void worker(int k) {
        vlg_ctx *ctx = slots[(size_t)k];
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            size_t off = 0;
            bool admitted = false;
            // admit the oldest waiting request once its footprint fits
            cv_work.wait(lk, [&] {
                if (stop) return true;
                if (!queue.empty() && pool.alloc(queue.front()->footprint, &off)) admitted = true;
                return admitted;
            });
            if (!admitted) return;
            std::shared_ptr<Request> r = queue.front();
            queue.pop_front();
            inflight++;
            st.max_inflight = std::max<int64_t>(st.max_inflight, inflight);
            st.peak_reserved_bytes = std::max<int64_t>(st.peak_reserved_bytes, (int64_t)pool.reserved());
            r->t_admit = Clock::now();
            lk.unlock();
            const int rc = vlg::evaluate_all_on(ctx, r->f, r->img, r->outs.data(), (char *)pool_mem + off,
                                                r->footprint);
            std::string err = rc == VLG_OK ? std::string() : std::string(vlg::last_error_text());
            lk.lock();
            pool.release(off, r->footprint);
            inflight--;
            r->t_done = Clock::now();
            r->status = rc;
            r->err = err;
            r->done = true;
            st.completed++;
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

namespace {
int sfail(int code, const std::string &m) { return vlg::set_last_error(code, m); }
}  // namespace

extern "C" {

int vlg_server_create(vlg_server **out, int device, int nslots, int64_t hbm_budget_bytes) {
    if (!out || nslots < 1 || nslots > 64 || hbm_budget_bytes <= 0) return sfail(VLG_EINVAL, "bad server arguments");
    *out = nullptr;
    auto s = std::make_unique<vlg_server>();
    s->device = device;
    s->budget = (size_t)hbm_budget_bytes;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return sfail(VLG_EINVAL, "bad device");
    if (hipMalloc(&s->pool_mem, s->budget) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipSetDevice(prev);
        return sfail(VLG_ENOMEM, "server pool allocation failed");
    }
    s->pool.reset(s->budget);
    s->st.budget_bytes = hbm_budget_bytes;
    for (int k = 0; k < nslots; k++) {
        vlg_ctx *c = nullptr;
        int rc = vlg_create(&c, device, nullptr);
        if (rc != VLG_OK) {
            for (vlg_ctx *x : s->slots) vlg_destroy(x);
            (void)hipFree(s->pool_mem);
            (void)hipSetDevice(prev);
            return rc;
        }
        vlg_set_mode(c, VLG_MODE_FUSED);
        s->slots.push_back(c);
    }
    (void)hipSetDevice(prev);
    vlg_server *raw = s.get();
    for (int k = 0; k < nslots; k++) s->workers.emplace_back([raw, k] { raw->worker(k); });
    *out = s.release();
    return VLG_OK;
}

int vlg_evaluation_bytes(const vlg_formula *f, const vlg_image *img, int64_t *bytes) {
    if (!f || !img || !bytes) return sfail(VLG_EINVAL, "null argument");
    *bytes = (int64_t)vlg::evaluation_footprint(const_cast<vlg_formula *>(f), img);
    return VLG_OK;
}

int vlg_server_submit(vlg_server *s, const vlg_formula *cf, const vlg_image *img, void *const *outs,
                      int64_t *request_id) {
    if (!s || !cf || !img || !outs || !request_id) return sfail(VLG_EINVAL, "null argument");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    auto r = std::make_shared<Request>();
    r->f = f;
    r->img = img;
    r->outs.assign(outs, outs + vlg::formula_outputs(cf));
    r->footprint = vlg::evaluation_footprint(f, img);
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    *request_id = r->id;
    s->reqs[r->id] = r;
    s->st.submitted++;
    if (r->footprint > s->budget) {
        r->t_admit = r->t_done = r->t_submit;
        r->status = VLG_ENOMEM;
        r->err = "request footprint " + std::to_string(r->footprint) + " B exceeds the server budget";
        r->done = true;
        s->st.rejected++;
        s->st.completed++;
        s->cv_done.notify_all();
        return VLG_OK;
    }
    s->queue.push_back(r);
    s->st.max_queued = std::max<int64_t>(s->st.max_queued, (int64_t)s->queue.size());
    s->cv_work.notify_all();
    return VLG_OK;
}

int vlg_server_wait(vlg_server *s, int64_t request_id, double *queue_ms, double *run_ms) {
    if (!s) return sfail(VLG_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return sfail(VLG_EINVAL, "unknown request id");
    std::shared_ptr<Request> r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->reqs.erase(request_id);
    using ms = std::chrono::duration<double, std::milli>;
    if (queue_ms) *queue_ms = ms(r->t_admit - r->t_submit).count();
    if (run_ms) *run_ms = ms(r->t_done - r->t_admit).count();
    if (r->status != VLG_OK) return sfail(r->status, r->err);
    return VLG_OK;
}

int vlg_server_read_stats(vlg_server *s, vlg_server_stats *out) {
    if (!s || !out) return sfail(VLG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return VLG_OK;
}

int vlg_server_destroy(vlg_server *s) {
    if (!s) return VLG_OK;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->queue.empty() && s->inflight == 0; });
        s->stop = true;
        s->cv_work.notify_all();
    }
    for (auto &t : s->workers) t.join();
    for (vlg_ctx *c : s->slots) vlg_destroy(c);
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    (void)hipFree(s->pool_mem);
    (void)hipSetDevice(prev);
    delete s;
    return VLG_OK;
}

}  // extern "C"
