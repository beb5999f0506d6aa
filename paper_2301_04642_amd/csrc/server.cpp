// Continuous-batching server for independent density-matrix solves.
//
// Requests are queued with a host copy of Hp.  An admission thread admits
// the queue head as soon as an executor is idle and the request's device
// footprint (Hp + D + solver workspace, all proportional to N^2) fits in the
// remaining budget; requests that arrive while others run join immediately,
// and their kernels overlap on the device because every executor owns its
// own stream.  Device blocks come from a pool of size classes whose held
// bytes (in use and pooled) stay within the budget.  Each solve is
// deterministic (fixed tile order, fixed-order reductions, tile shape chosen
// from N only), so a request's result does not depend on what else is
// running.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fdm_internal.h"
#include "solver_internal.h"

namespace fdm {
namespace {

using Clock = std::chrono::steady_clock;

// Requests from this size up tick in the large-size group.
constexpr int64_t kTickLargeN = 2048;

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
    bool collecting = false;  // an fdm_result call is copying D out
    double t_submit = 0, t_start = 0, t_finish = 0;
};

// Device blocks come in size classes (eight per octave above 1 MiB, so at
// most 12.5% is lost to rounding; multiples of 64 KiB below), and a freed
// block stays in the pool of its class for the next request of a similar
// size.  Every held byte -- blocks in use and pooled ones -- counts against
// the server's budget: before a new block is allocated, pooled blocks are
// evicted until the held bytes plus the new block fit.  Admission reserves a
// request's footprint in class sizes, so the blocks in use never exceed the
// reservations and eviction can always make room.  Eviction and allocation
// run outside the server mutex (hipFree can wait for the device).
size_t size_class(size_t bytes) {
    const size_t kSmall = (size_t)1 << 20, kGran = (size_t)1 << 16;
    if (bytes <= kSmall) return (bytes + kGran - 1) / kGran * kGran;
    int e = 63 - __builtin_clzll((unsigned long long)bytes);
    const size_t step = (size_t)1 << (e - 3);
    return (bytes + step - 1) / step * step;
}

class BlockPool {
   public:
    // A pooled block of exactly this class, or nullptr.
    void *take(size_t cls) {
        auto it = free_.find(cls);
        if (it == free_.end()) return nullptr;
        void *p = it->second;
        free_.erase(it);
        pooled_ -= cls;
        return p;
    }
    // Makes room for `need` more held bytes under `budget`: pooled blocks
    // (largest first) move to *evict, to be freed by the caller outside the
    // lock; the new bytes are counted as held at once.
    bool reserve(size_t need, size_t budget, std::vector<std::pair<void *, size_t>> *evict) {
        while (held_ + need > budget && !free_.empty()) {
            auto it = std::prev(free_.end());
            evict->push_back({it->second, it->first});
            held_ -= it->first;
            pooled_ -= it->first;
            sizes_.erase(it->second);
            free_.erase(it);
        }
        if (held_ + need > budget) return false;
        held_ += need;
        return true;
    }
    void adopt(void *p, size_t cls) { sizes_[p] = cls; }      // a block allocated by the caller
    void unreserve(size_t cls) { held_ -= cls; }              // an allocation that failed
    void put(void *p) {
        if (!p) return;
        const size_t cls = sizes_[p];
        free_.emplace(cls, p);
        pooled_ += cls;
    }
    size_t held() const { return held_; }
    size_t pooled() const { return pooled_; }
    void release_all() {
        for (auto &kv : sizes_) hipFree(kv.first);
        sizes_.clear();
        free_.clear();
        held_ = pooled_ = 0;
    }

   private:
    std::multimap<size_t, void *> free_;
    std::unordered_map<void *, size_t> sizes_;
    size_t held_ = 0, pooled_ = 0;
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
    BlockPool pool;                   // guarded by mu
    std::vector<std::thread> workers;
    std::thread admitter;
    // grouped hot-loop steps, one tick group per size class (nullptr:
    // independent streams): a tick lasts as long as its largest product, so
    // small requests tick with small ones at their own pace, on their own
    // stream, beside the large ones
    TickGroup *group[2] = {nullptr, nullptr};

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

// Device bytes a request holds while it runs, in block size classes: Hp,
// D and the solver workspace.
static size_t request_footprint(int64_t n, double kT, int prec, size_t *ws) {
    *ws = fdm_workspace_bytes(n, kT, prec);
    const size_t mat = (size_t)n * (size_t)n * sizeof(double);
    return size_class(*ws) + 2 * size_class(mat);
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

// Blocks of the given classes for one request: pooled ones where they
// exist, the rest allocated after evicting pooled blocks to stay within the
// budget.  Called with the lock held; drops it while freeing and allocating.
static bool acquire_blocks(fdm_server *s, std::unique_lock<std::mutex> &lk, const size_t *cls,
                           void **out, int count) {
    size_t need = 0;
    for (int i = 0; i < count; ++i) {
        out[i] = s->pool.take(cls[i]);
        if (!out[i]) need += cls[i];
    }
    if (need == 0) return true;
    std::vector<std::pair<void *, size_t>> evict;
    if (!s->pool.reserve(need, s->budget, &evict)) {
        for (int i = 0; i < count; ++i) s->pool.put(out[i]), out[i] = nullptr;
        return false;
    }
    lk.unlock();
    for (auto &b : evict) hipFree(b.first);
    bool ok = true;
    size_t failed = 0;
    for (int i = 0; i < count; ++i) {
        if (out[i]) continue;
        if (hipMalloc(&out[i], cls[i]) != hipSuccess) {
            (void)hipGetLastError();
            out[i] = nullptr;
            failed += cls[i];
            ok = false;
        }
    }
    lk.lock();
    for (int i = 0; i < count; ++i)
        if (out[i]) s->pool.adopt(out[i], cls[i]);
    if (failed) s->pool.unreserve(failed);
    return ok;
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
        const size_t cls[3] = {size_class(mat), size_class(mat), size_class(r->ws_bytes)};
        void *blk[3] = {nullptr, nullptr, nullptr};
        const bool got = acquire_blocks(s, lk, cls, blk, 3);
        double *hp = (double *)blk[0], *d = (double *)blk[1];
        void *ws = blk[2];
        lk.unlock();
        int rc = FDM_OK;
        if (!got) {
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
            opt.workspace_bytes = cls[2];
            rc = solve_impl(hp, r->n, r->n, r->n_occ, r->kT, r->tol, d, r->n, &r->e_band, &opt,
                            &r->stats, stream, s->group[r->n >= kTickLargeN ? 1 : 0]);
        }
        hipStreamSynchronize(stream);
        lk.lock();
        std::vector<double>().swap(r->hp);
        s->pool.put(hp);
        s->pool.put(ws);
        if (rc != FDM_OK && rc != FDM_ENOCONV) {
            s->pool.put(d);
            d = nullptr;
        }
        r->d_dev = d;
        r->status = rc;
        r->t_finish = s->now();
        // Hp and the workspace are released now; D stays until fdm_result
        s->reserved -= r->footprint - (d ? cls[1] : 0);
        r->footprint = d ? cls[1] : 0;
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
    if (s->max_active > kMaxGroup) {
        set_error("max_active above " + std::to_string(kMaxGroup));
        return nullptr;
    }
    s->default_prec = opt->precision;
    s->t0 = Clock::now();
    if (!opt->independent) {
        for (TickGroup *&g : s->group) {
            g = tick_group_create(s->device);
            if (!g) {
                for (TickGroup *h : s->group) tick_group_destroy(h);
                set_error("could not create the serving tick groups");
                return nullptr;
            }
        }
    }
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
    // Look the ticket up again after every wait: another fdm_result call on
    // the same ticket may have collected (and erased) it meanwhile.
    Request *r = nullptr;
    while (true) {
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end() || it->second->collecting) return FDM_EINVAL;
        r = it->second.get();
        if (r->status != 1) break;
        s->cv.wait(lk);
    }
    if (D_out && ldd < r->n) return FDM_EINVAL;
    // copy D out without the lock: the other requests keep running and
    // being admitted meanwhile
    r->collecting = true;
    const int64_t n = r->n;
    double *d_dev = r->d_dev;
    lk.unlock();
    int rc = r->status;
    if (d_dev && D_out) {
        const size_t row = (size_t)n * sizeof(double);
        hipError_t e = hipMemcpy2D(D_out, (size_t)ldd * sizeof(double), d_dev, row, row,
                                   (size_t)n,
                                   out_on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice);
        if (e != hipSuccess) rc = FDM_EHIP;
    }
    const double t_result = s->now();
    lk.lock();
    if (E_band) *E_band = r->e_band;
    if (stats) *stats = r->stats;
    if (times) {
        times[0] = r->t_submit;
        times[1] = r->t_start;
        times[2] = r->t_finish;
        times[3] = t_result;
    }
    if (d_dev) s->pool.put(d_dev);
    s->reserved -= r->footprint;
    s->reqs.erase(ticket);
    s->cv.notify_all();
    return rc;
}

int fdm_server_memory(fdm_server *s, size_t *held, size_t *reserved, size_t *pooled) {
    if (!s) return FDM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (held) *held = s->pool.held();
    if (reserved) *reserved = s->reserved;
    if (pooled) *pooled = s->pool.pooled();
    return FDM_OK;
}

void fdm_server_destroy(fdm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        // Requests that never started are dropped (queued ones hold nothing;
        // admitted ones give back their reservation); running ones finish.
        s->stop = true;
        for (uint64_t id : s->queue) s->reqs.erase(id);
        for (uint64_t id : s->ready) {
            s->reserved -= s->reqs[id]->footprint;
            s->reqs.erase(id);
        }
        s->queue.clear();
        s->ready.clear();
        s->cv.notify_all();
    }
    for (auto &t : s->workers) t.join();
    s->admitter.join();
    for (TickGroup *g : s->group) tick_group_destroy(g);
    // results nobody collected, and every pooled block
    s->pool.release_all();
    delete s;
}

}  // extern "C"
