// Serving tick: the hot-loop steps of the solves that run at the same time
// are launched together.
//
// Every executor thread runs its own solve; inside a hot loop (SP2 and
// McWeeny steps, finite-temperature evaluations) its launches are recorded
// as steps and posted here instead of going to its stream.  A ticker thread
// forms ticks: it takes the next posted step of every member, launches the
// members' products of one precision, tile edge and staging path as ONE
// grouped product over their concatenated upper-tile lists, and their
// decisions as ONE grouped decision (one block per solve), on the group's
// stream.  Each tile and each decision is computed exactly as in a solve of
// its own, so results do not depend on the grouping.  At most two ticks are
// in flight, so members that post after a tick finishes join the next one.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "fdm_internal.h"
#include "solver_internal.h"

namespace fdm {

struct TickGroup {
    int device = 0;
    hipStream_t gs = nullptr;
    hipEvent_t tick_ev[2] = {nullptr, nullptr};
    std::mutex mu;
    std::condition_variable cv;     // posts (ticker waits) and launches (members wait)
    std::vector<TickMember *> members;
    bool stop = false;
    int error = 0;
    std::string error_msg;          // the ticker's message for the failed members
    std::thread ticker;
    void run();
};

namespace {

// How long a tick waits for members that have not posted their next step.
constexpr auto kBatchWait = std::chrono::microseconds(40);

struct Taken {
    TickMember *m;
    int seq;
    Step step;
    bool enter;
};

int launch_tick(hipStream_t gs, std::vector<Taken> &tk) {
    hipError_t e;
    for (Taken &t : tk) {
        if (!t.enter) continue;
        e = hipStreamWaitEvent(gs, t.m->entry, 0);
        if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent (tick entry)");
    }
    size_t maxops = 0;
    for (Taken &t : tk) maxops = std::max(maxops, t.step.ops.size());
    for (size_t i = 0; i < maxops; ++i) {
        // launches that are neither products nor decisions, member by member
        for (Taken &t : tk) {
            if (i >= t.step.ops.size() || t.step.ops[i].kind != StepOp::CUSTOM) continue;
            e = t.step.ops[i].custom(gs);
            if (e != hipSuccess) return hip_fail(e, "tick launch");
        }
        // products, grouped by precision, tile edge and staging path
        std::map<std::tuple<int, int, bool>, std::vector<const ProdArgs *>> prods;
        for (Taken &t : tk) {
            if (i >= t.step.ops.size() || t.step.ops[i].kind != StepOp::PRODUCT) continue;
            const StepOp &o = t.step.ops[i];
            prods[std::make_tuple(o.prec, o.bt, o.direct)].push_back(&o.a);
        }
        for (auto &kv : prods) {
            const std::vector<const ProdArgs *> &v = kv.second;
            for (size_t j0 = 0; j0 < v.size(); j0 += kMaxGroup) {
                ProdGroup g;
                memset(&g, 0, sizeof(g));
                g.njobs = (int)std::min<size_t>(kMaxGroup, v.size() - j0);
                g.first[0] = 0;
                for (int j = 0; j < g.njobs; ++j) {
                    g.job[j] = *v[j0 + j];
                    g.first[j + 1] = g.first[j] + g.job[j].ntiles;
                }
                e = launch_symprod_grouped(std::get<0>(kv.first), std::get<1>(kv.first),
                                           std::get<2>(kv.first), g, gs);
                if (e != hipSuccess) return hip_fail(e, "grouped product launch");
            }
        }
        // decisions, one block per solve
        DecideGroup dg;
        memset(&dg, 0, sizeof(dg));
        for (Taken &t : tk) {
            if (i >= t.step.ops.size() || t.step.ops[i].kind != StepOp::DECIDE) continue;
            dg.job[dg.njobs++] = t.step.ops[i].d;
            if (dg.njobs == kMaxGroup) {
                e = launch_decide_grouped(dg, gs);
                if (e != hipSuccess) return hip_fail(e, "grouped decide launch");
                dg.njobs = 0;
            }
        }
        if (dg.njobs) {
            e = launch_decide_grouped(dg, gs);
            if (e != hipSuccess) return hip_fail(e, "grouped decide launch");
        }
    }
    for (Taken &t : tk) {
        e = hipEventRecord(t.m->ev[t.seq % kEvRing], gs);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord (tick)");
    }
    return FDM_OK;
}

}  // namespace

void TickGroup::run() {
    (void)hipSetDevice(device);
    int inflight = 0;  // ticks launched and not yet waited for (tick_ev[t & 1])
    long tick = 0;
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        auto any_posted = [&] {
            for (TickMember *m : members)
                if (!m->posted.empty()) return true;
            return false;
        };
        auto all_posted = [&] {
            for (TickMember *m : members)
                if (m->posted.empty()) return false;
            return true;
        };
        cv.wait(lk, [&] { return stop || any_posted(); });
        if (stop) break;
        if (!all_posted()) cv.wait_for(lk, kBatchWait, [&] { return stop || all_posted(); });
        if (stop) break;
        std::vector<Taken> tk;
        for (TickMember *m : members) {
            if (m->posted.empty()) continue;
            tk.push_back({m, m->posted.front().first, std::move(m->posted.front().second),
                          !m->entered});
            m->entered = true;
            m->taken += 1;
            m->posted.pop_front();
        }
        lk.unlock();
        // keep at most two ticks in flight
        int rc = FDM_OK;
        if (inflight == 2) {
            hipError_t e = hipEventSynchronize(tick_ev[tick & 1]);
            if (e != hipSuccess) rc = hip_fail(e, "hipEventSynchronize (tick)");
            inflight = 1;
        }
        if (rc == FDM_OK) rc = launch_tick(gs, tk);
        if (rc == FDM_OK) {
            hipError_t e = hipEventRecord(tick_ev[tick & 1], gs);
            if (e != hipSuccess) rc = hip_fail(e, "hipEventRecord (tick)");
            ++inflight;
            ++tick;
        }
        lk.lock();
        for (Taken &t : tk) {
            t.m->launched = t.seq;
            t.m->taken -= 1;
            t.m->steps += 1;
            if (tk.size() > 1) t.m->shared += 1;
            if (rc) t.m->error = rc;
        }
        if (rc) {
            error = rc;
            error_msg = last_error();  // set on this thread; members report it on theirs
        }
        cv.notify_all();
    }
}

TickGroup *tick_group_create(int device) {
    std::unique_ptr<TickGroup> g(new TickGroup());
    g->device = device;
    auto undo = [&g] {
        for (hipEvent_t e : g->tick_ev)
            if (e) (void)hipEventDestroy(e);
        if (g->gs) (void)hipStreamDestroy(g->gs);
        return nullptr;
    };
    if (hipStreamCreateWithFlags(&g->gs, hipStreamNonBlocking) != hipSuccess) return undo();
    for (int i = 0; i < 2; ++i)
        if (hipEventCreateWithFlags(&g->tick_ev[i], hipEventDisableTiming) != hipSuccess)
            return undo();
    TickGroup *raw = g.get();
    g->ticker = std::thread([raw] { raw->run(); });
    return g.release();
}

void tick_group_destroy(TickGroup *g) {
    if (!g) return;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        g->stop = true;
        g->cv.notify_all();
    }
    if (g->ticker.joinable()) g->ticker.join();
    (void)hipStreamSynchronize(g->gs);
    for (hipEvent_t e : g->tick_ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(g->gs);
    delete g;
}

int tick_join(TickGroup *g, TickMember *m, hipStream_t s) {
    hipError_t e = hipEventRecord(m->entry, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord (tick join)");
    std::lock_guard<std::mutex> lk(g->mu);
    m->entered = false;
    m->launched = -1;
    m->error = 0;
    m->posted.clear();
    g->members.push_back(m);
    return FDM_OK;
}

void tick_post(TickGroup *g, TickMember *m, int seq, Step &&st) {
    std::lock_guard<std::mutex> lk(g->mu);
    m->posted.emplace_back(seq, std::move(st));
    g->cv.notify_all();
}

int tick_wait(TickGroup *g, TickMember *m, int seq) {
    {
        std::unique_lock<std::mutex> lk(g->mu);
        g->cv.wait(lk, [&] { return m->launched >= seq || m->error != 0 || g->stop; });
        if (m->error) {
            set_error(g->error_msg);
            return m->error;
        }
        if (m->launched < seq) {
            set_error("serving tick group stopped");
            return FDM_EHIP;
        }
    }
    hipError_t e = hipEventSynchronize(m->ev[seq % kEvRing]);
    return e == hipSuccess ? FDM_OK : hip_fail(e, "hipEventSynchronize (tick step)");
}

int tick_leave(TickGroup *g, TickMember *m) {
    int last;
    {
        std::unique_lock<std::mutex> lk(g->mu);
        m->posted.clear();  // steps after the phase's decision: no-ops on the device
        g->members.erase(std::remove(g->members.begin(), g->members.end(), m), g->members.end());
        // a step the ticker has taken is launched before the member may go
        g->cv.wait(lk, [&] { return m->taken == 0; });
        last = m->launched;
        if (m->error) {
            set_error(g->error_msg);
            return m->error;
        }
    }
    if (last < 0) return FDM_OK;
    hipError_t e = hipEventSynchronize(m->ev[last % kEvRing]);
    return e == hipSuccess ? FDM_OK : hip_fail(e, "hipEventSynchronize (tick leave)");
}

}  // namespace fdm
