// Continuous-batching server for independent density-matrix solves.
//
// Requests are queued with a host copy of Hp.  An admission thread admits
// the queue head as soon as an executor is idle and the request's device
// footprint (Hp + D + solver workspace, all proportional to N^2) fits in the
// remaining budget; requests that arrive while others run join immediately,
// and their kernels overlap on the device because every executor owns its
// own stream.  Device blocks come from a caching allocator (so no hipFree,
// which would synchronise the whole device, sits on the hot path).  Each
// solve is deterministic (fixed tile order, fixed-order reductions, tile
// shape chosen from N only), so a request's result does not depend on what
// else is running.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fdm_internal.h"

namespace fdm {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t id = 0;
    int64_t n = 0;
    double n_occ = 0, kT = 0, tol = 0;
    int precision = 0;
    std::vector<double> hp;  // host copy, released at admission
    size_t footprint = 0;
    size_t ws_bytes = 0;
    double *d_dev = nullptr;  // result, held until fdm_result
    double e_band = 0;
    fdm_stats stats;
    int status = 1;  // 1 pending, else solve status
    double t_submit = 0, t_start = 0, t_finish = 0;
};

// Size-keyed cache of device blocks.  Blocks are only returned to HIP when
// the budget needs the room.
class BlockCache {
   public:
    void *get(size_t bytes) {
        auto it = free_.lower_bound(bytes);
        if (it != free_.end() && it->first <= bytes + bytes / 8) {
            void *p = it->second;
            free_.erase(it);
            return p;
        }
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            trim_all();
            if (hipMalloc(&p, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        sizes_[p] = bytes;
        held_ += bytes;
        return p;
    }
    void put(void *p) {
        if (!p) return;
        free_.emplace(sizes_[p], p);
    }
    size_t held() const { return held_; }
    size_t cached() const {
        size_t s = 0;
        for (auto &kv : free_) s += kv.first;
        return s;
    }
    void trim_all() {
        if (free_.empty()) return;
        hipDeviceSynchronize();
        for (auto &kv : free_) {
            hipFree(kv.second);
            held_ -= kv.first;
            sizes_.erase(kv.second);
        }
        free_.clear();
    }
    ~BlockCache() {
        for (auto &kv : sizes_) hipFree(kv.first);
    }

   private:
    std::multimap<size_t, void *> free_;
    std::unordered_map<void *, size_t> sizes_;
    size_t held_ = 0;
};

}  // namespace
}  // namespace fdm

using namespace fdm;

struct fdm_server {
    int device = 0;
    size_t budget = 0;
    int max_active = 4;
    int default_prec = 0;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;       // state changes (queue, finishes, shutdown)
    std::deque<uint64_t> queue;       // FIFO of pending request ids
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    size_t reserved = 0;              // footprint of admitted, unreleased requests
    uint64_t next_id = 1;
    bool stop = false;
    int idle = 0;
    std::deque<uint64_t> ready;       // admitted ids waiting for an executor
    BlockCache cache;                 // guarded by mu
    std::vector<std::thread> workers;
    std::thread admitter;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

static size_t request_footprint(int64_t n, double kT, int prec, size_t *ws) {
    *ws = fdm_workspace_bytes(n, kT, prec);
    return *ws + 2 * (size_t)n * (size_t)n * sizeof(double);
}

static void admission_loop(fdm_server *s) {
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        bool admitted = false;
        if (!s->queue.empty() && s->idle > (int)s->ready.size()) {
            Request *r = s->reqs[s->queue.front()].get();
            if (s->reserved + r->footprint <= s->budget) {
                s->reserved += r->footprint;
                s->ready.push_back(r->id);
                s->queue.pop_front();
                admitted = true;
                s->cv.notify_all();
            }
        }
        if (!admitted) s->cv.wait(lk);
    }
}

static void executor_loop(fdm_server *s) {
    hipSetDevice(s->device);
    hipStream_t stream = nullptr;
    hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    std::unique_lock<std::mutex> lk(s->mu);
    s->idle += 1;
    s->cv.notify_all();
    while (true) {
        while (!s->stop && s->ready.empty()) s->cv.wait(lk);
        if (s->stop && s->ready.empty()) break;
        const uint64_t id = s->ready.front();
        s->ready.pop_front();
        s->idle -= 1;
        Request *r = s->reqs[id].get();
        r->t_start = s->now();
        const size_t mat = (size_t)r->n * (size_t)r->n * sizeof(double);
        double *hp = (double *)s->cache.get(mat);
        double *d = (double *)s->cache.get(mat);
        void *ws = s->cache.get(r->ws_bytes);
        lk.unlock();
        int rc = FDM_OK;
        if (!hp || !d || !ws) {
            rc = FDM_ENOMEM;
        } else {
            hipError_t e = hipMemcpyAsync(hp, r->hp.data(), mat, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) rc = FDM_EHIP;
        }
        if (rc == FDM_OK) {
            fdm_options opt;
            fdm_options_default(&opt);
            opt.precision = r->precision;
            opt.workspace = ws;
            opt.workspace_bytes = r->ws_bytes;
            rc = fermi_dm_solve(hp, r->n, r->n, r->n_occ, r->kT, r->tol, d, r->n, &r->e_band,
                                &opt, &r->stats, stream);
        }
        hipStreamSynchronize(stream);
        lk.lock();
        std::vector<double>().swap(r->hp);
        s->cache.put(hp);
        s->cache.put(ws);
        if (rc != FDM_OK && rc != FDM_ENOCONV) {
            s->cache.put(d);
            d = nullptr;
        }
        r->d_dev = d;
        r->status = rc;
        r->t_finish = s->now();
        // Hp and the workspace are released now; D stays until fdm_result
        s->reserved -= r->footprint - (d ? mat : 0);
        r->footprint = d ? mat : 0;
        s->idle += 1;
        s->cv.notify_all();
    }
    lk.unlock();
    hipStreamDestroy(stream);
}

extern "C" {

fdm_server *fdm_server_create(const fdm_server_options *opt) {
    set_error("");
    if (!opt || opt->budget_bytes == 0 || opt->max_active < 0) {
        set_error("invalid server options");
        return nullptr;
    }
    std::unique_ptr<fdm_server> s(new fdm_server());
    if (hipGetDevice(&s->device) != hipSuccess) {
        set_error("hipGetDevice failed");
        return nullptr;
    }
    s->budget = opt->budget_bytes;
    s->max_active = opt->max_active > 0 ? opt->max_active : 4;
    s->default_prec = opt->precision;
    s->t0 = Clock::now();
    fdm_server *raw = s.get();
    for (int i = 0; i < s->max_active; ++i) s->workers.emplace_back(executor_loop, raw);
    s->admitter = std::thread(admission_loop, raw);
    return s.release();
}

int fdm_submit(fdm_server *s, const double *Hp, int32_t hp_on_host, int64_t N, double n_occ,
               double kT, double tol, int32_t precision, uint64_t *ticket) {
    set_error("");
    if (!s || !Hp || !ticket || N <= 0 || !(tol > 0.0) || !(kT >= 0.0) || precision < -1 ||
        precision >= FDM_NPREC)
        return FDM_EINVAL;
    if (precision < 0) precision = s->default_prec;
    std::unique_ptr<Request> r(new Request());
    r->n = N;
    r->n_occ = n_occ;
    r->kT = kT;
    r->tol = tol;
    r->precision = precision;
    r->footprint = request_footprint(N, kT, precision, &r->ws_bytes);
    if (r->ws_bytes == 0) return FDM_EINVAL;
    if (r->footprint > s->budget) {
        set_error("request footprint exceeds the server budget");
        return FDM_ENOMEM;
    }
    const size_t mat = (size_t)N * (size_t)N;
    r->hp.resize(mat);
    if (hp_on_host) {
        memcpy(r->hp.data(), Hp, mat * sizeof(double));
    } else {
        hipError_t e = hipMemcpy(r->hp.data(), Hp, mat * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return FDM_EHIP;
    }
    memset(&r->stats, 0, sizeof(r->stats));
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    r->t_submit = s->now();
    *ticket = r->id;
    s->queue.push_back(r->id);
    s->reqs[r->id] = std::move(r);
    s->cv.notify_all();
    return FDM_OK;
}

int fdm_poll(fdm_server *s, uint64_t ticket) {
    if (!s) return FDM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return FDM_EINVAL;
    return it->second->status == 1 ? 1 : 0;
}

int fdm_result(fdm_server *s, uint64_t ticket, double *D_out, int32_t out_on_host, int64_t ldd,
               double *E_band, fdm_stats *stats, double *times) {
    set_error("");
    if (!s) return FDM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return FDM_EINVAL;
    Request *r = it->second.get();
    while (r->status == 1) s->cv.wait(lk);
    if (D_out && ldd < r->n) return FDM_EINVAL;
    int rc = r->status;
    const double t_result = s->now();
    if (r->d_dev && D_out) {
        const size_t row = (size_t)r->n * sizeof(double);
        hipError_t e = hipMemcpy2D(D_out, (size_t)ldd * sizeof(double), r->d_dev, row, row,
                                   (size_t)r->n,
                                   out_on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice);
        if (e != hipSuccess) rc = FDM_EHIP;
    }
    if (E_band) *E_band = r->e_band;
    if (stats) *stats = r->stats;
    if (times) {
        times[0] = r->t_submit;
        times[1] = r->t_start;
        times[2] = r->t_finish;
        times[3] = t_result;
    }
    if (r->d_dev) s->cache.put(r->d_dev);
    s->reserved -= r->footprint;
    s->reqs.erase(it);
    s->cv.notify_all();
    return rc;
}

void fdm_server_destroy(fdm_server *s) {
    if (!s) return;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        // let queued and running requests finish
        while (!s->queue.empty() || !s->ready.empty() || s->idle < s->max_active) s->cv.wait(lk);
        s->stop = true;
        s->cv.notify_all();
    }
    for (auto &t : s->workers) t.join();
    s->admitter.join();
    for (auto &kv : s->reqs)
        if (kv.second->d_dev) s->cache.put(kv.second->d_dev);
    delete s;
}

}  // extern "C"
