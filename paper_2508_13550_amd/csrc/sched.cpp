// Continuous-batching scheduler for serving CSFMM evaluations (host only).
//
// The scheduler decides; the caller executes.  Requests arrive with a plan
// key (the geometry and method parameters of their plan), the device bytes of
// that plan and of one eval workspace, and an estimate of their cost.  Each
// step starts a batch (one packed launch) with the oldest waiting request and
// adds, in arrival order, the waiting requests of the same cost class (within
// a factor kClassRatio of its cost) while their memory fits the HBM budget;
// requests of other classes wait for a later batch, which the caller may run
// beside this one on another stream, so a small request is not held for the
// length of a large one's launches:
//   * a plan stays resident after its requests finish (plan cache); a request
//     whose plan is resident needs no plan build;
//   * each resident plan owns a pool of workspaces as large as the largest
//     number of its requests in flight at once; a request that finds a free
//     pooled workspace needs no new memory;
//   * when memory is short, resident plans with nothing in flight are evicted
//     least recently used first; plans with requests in flight are never
//     evicted;
//   * within a class admission is first-come first-served, and when the
//     oldest waiting request does not fit, no younger request overtakes it;
//   * a request that cannot fit even in an empty device is rejected.
// Completions return the request's workspace to its plan's pool.
#include <cstdint>
#include <cstring>
#include <deque>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/csfmm.h"

namespace {

struct PlanEntry {
    int64_t plan_bytes = 0;
    int64_t ws_bytes = 0;
    int pool = 0;       // workspaces owned by the plan
    int inflight = 0;   // requests using the plan now
    double last_used = 0.0;
};

struct Req {
    int64_t id;
    uint64_t key;
    int64_t plan_bytes, ws_bytes;
    double t_arrival;
    double cost;
};

// Requests within this factor of the batch head's cost share its batch.
constexpr double kClassRatio = 4.0;

}  // namespace

struct csfmm_sched_s {
    int64_t budget = 0;
    int max_batch = 32;
    int64_t used = 0;
    std::deque<Req> queue;
    std::unordered_map<uint64_t, PlanEntry> plans;
    std::unordered_map<int64_t, uint64_t> inflight;  // request id -> plan key
    csfmm_sched_stats st{};

    int64_t entry_bytes(const PlanEntry& e) const { return e.plan_bytes + e.pool * e.ws_bytes; }

    // Evicts idle plans (LRU) other than `keep` until `need` more bytes fit.
    bool make_room(int64_t need, uint64_t keep, uint64_t* evict, int* n_evict, int cap) {
        while (used + need > budget) {
            uint64_t victim = 0;
            bool found = false;
            double oldest = 0.0;
            for (auto& kv : plans) {
                if (kv.first == keep || kv.second.inflight > 0) continue;
                if (!found || kv.second.last_used < oldest) {
                    victim = kv.first;
                    oldest = kv.second.last_used;
                    found = true;
                }
            }
            if (!found || *n_evict >= cap) return false;
            used -= entry_bytes(plans[victim]);
            plans.erase(victim);
            evict[(*n_evict)++] = victim;
            st.evictions += 1;
        }
        return true;
    }
};

extern "C" {

int csfmm_sched_create(int64_t hbm_budget_bytes, int max_batch, csfmm_sched_t* out) {
    if (!out || hbm_budget_bytes <= 0 || max_batch < 1) return CSFMM_E_INVALID;
    csfmm_sched_s* s = new (std::nothrow) csfmm_sched_s();
    if (!s) return CSFMM_E_OOM;
    s->budget = hbm_budget_bytes;
    s->max_batch = max_batch;
    *out = s;
    return CSFMM_OK;
}

int csfmm_sched_destroy(csfmm_sched_t s) {
    delete s;
    return CSFMM_OK;
}

int csfmm_sched_submit(csfmm_sched_t s, int64_t req_id, uint64_t plan_key, int64_t plan_bytes,
                       int64_t ws_bytes, double t_arrival, double cost) {
    if (!s || plan_bytes < 0 || ws_bytes < 0 || !(cost >= 0.0)) return CSFMM_E_INVALID;
    s->queue.push_back(Req{req_id, plan_key, plan_bytes, ws_bytes, t_arrival, cost});
    s->st.submitted += 1;
    return CSFMM_OK;
}

int csfmm_sched_step(csfmm_sched_t s, double now, csfmm_sched_decision* d) {
    if (!s || !d) return CSFMM_E_INVALID;
    d->n_launch = d->n_build = d->n_evict = d->n_reject = d->n_new_ws = 0;
    double c0 = -1.0;  // cost of the batch's first request
    size_t pos = 0;    // queue position examined next
    while (pos < s->queue.size() && d->n_launch < s->max_batch && d->n_launch < d->cap_launch) {
        const Req q = s->queue[pos];
        if (q.t_arrival > now) break;
        if (c0 >= 0.0 && (q.cost > c0 * kClassRatio || q.cost * kClassRatio < c0)) {
            ++pos;  // another class: a later batch takes it
            continue;
        }
        auto it = s->plans.find(q.key);
        const bool resident = it != s->plans.end();
        const bool free_ws = resident && it->second.inflight < it->second.pool;
        const int64_t need = (resident ? 0 : q.plan_bytes) + (free_ws ? 0 : q.ws_bytes);
        if (q.plan_bytes + q.ws_bytes > s->budget) {
            s->queue.erase(s->queue.begin() + pos);
            if (d->n_reject < d->cap_reject) d->reject_ids[d->n_reject++] = q.id;
            s->st.rejected += 1;
            continue;
        }
        if (s->used + need > s->budget &&
            !s->make_room(need, q.key, d->evict_keys, &d->n_evict, d->cap_evict))
            break;  // wait for completions; nobody in the class overtakes
        if (!resident && d->n_build >= d->cap_build) break;
        if (!free_ws && d->n_new_ws >= d->cap_launch) break;
        s->queue.erase(s->queue.begin() + pos);
        if (c0 < 0.0) c0 = q.cost;
        PlanEntry& e = s->plans[q.key];
        if (!resident) {
            e.plan_bytes = q.plan_bytes;
            e.ws_bytes = q.ws_bytes;
            d->build_keys[d->n_build++] = q.key;
            s->used += q.plan_bytes;
            s->st.plan_misses += 1;
        } else {
            s->st.plan_hits += 1;
        }
        if (!free_ws) {
            e.pool += 1;
            s->used += e.ws_bytes;
            d->new_ws_keys[d->n_new_ws++] = q.key;
        }
        e.inflight += 1;
        e.last_used = now;
        s->inflight[q.id] = q.key;
        d->launch_ids[d->n_launch++] = q.id;
        s->st.launched += 1;
    }
    if (d->n_launch > 0) s->st.batches += 1;
    return CSFMM_OK;
}

int csfmm_sched_complete(csfmm_sched_t s, int64_t req_id, double now) {
    if (!s) return CSFMM_E_INVALID;
    auto it = s->inflight.find(req_id);
    if (it == s->inflight.end()) return CSFMM_E_INVALID;
    PlanEntry& e = s->plans[it->second];
    e.inflight -= 1;
    e.last_used = now;
    s->inflight.erase(it);
    s->st.completed += 1;
    return CSFMM_OK;
}

int csfmm_sched_get_stats(csfmm_sched_t s, csfmm_sched_stats* out) {
    if (!s || !out) return CSFMM_E_INVALID;
    *out = s->st;
    out->used_bytes = s->used;
    out->budget_bytes = s->budget;
    out->queued = int64_t(s->queue.size());
    out->in_flight = int64_t(s->inflight.size());
    out->resident_plans = int64_t(s->plans.size());
    return CSFMM_OK;
}

}  // extern "C"
