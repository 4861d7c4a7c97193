// sa_server.cpp -- continuous-batching server (include/sa.h, serving).
//
// Requests arrive through sa_server_submit (the problem is copied) or sa_server_submit_plan (a
// prepared plan is shared).  Prep threads canonicalise, pack and upload them.  One scheduler thread
// owns the device work: it admits prepared requests in arrival order while a slot is free and
// their device footprint (plan, states, schedule) fits the memory budget, then advances every
// admitted request by one chunk of sweeps in a single launch of the batched kernel.  States and
// their exact energies stay on the device between chunks (each chunk resumes from them), so
// requests that arrive while others run join at the next chunk boundary, and a request's result
// does not depend on which requests shared its chunks: the draws are keyed by (variable, sweep,
// read, instance id) and the energy changes are exact integers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "sa_plan.h"

using sa::align256;
using sa::fail;
using sa::hip_fail;

namespace {

enum class Phase { Queued, Prepared, Active, Done };

struct Request {
    uint64_t id = 0;
    // owned copy of a submitted problem (unused with a shared plan)
    std::vector<int64_t> term_ptr, coef;
    std::vector<int32_t> factor_var, lo, hi;
    std::vector<double> beta_in;
    int32_t n_vars = 0;
    int64_t n_terms = 0;
    int32_t rule = 0, n_reads = 0, n_sweeps = 0;
    uint64_t seed = 0;
    uint32_t instance_id = 0;
    sa_result result{};
    sa_plan *plan = nullptr;
    bool own_plan = false;
    bool cached = false;              // plan shared through the server's plan cache
    std::array<uint64_t, 3> cache_key{};
    std::vector<double> beta;
    // device state of an admitted request
    void *mem = nullptr;  // beta | states | energies
    double *beta_dev = nullptr;
    int32_t *z_dev = nullptr;
    int64_t *e_dev = nullptr;
    size_t footprint = 0;
    bool accounted = false;  // footprint counted in the server's memory in use
    int32_t next_sweep = 0;
    Phase phase = Phase::Queued;
    bool cancel = false;
    int32_t status = SA_EBUSY;
    std::string error;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

double cost_of_update(const sa_plan &p) {
    const double chunks = 1.0 + (double)p.info.n_incidences / std::max(1, p.info.n_vars) / 64.0;
    const double per_lane = std::ceil(p.info.max_width / 64.0);
    if (p.rule == SA_HEAT_BATH_CLOSED && p.info.max_exponent <= 1) return chunks + 2.0;
    if (p.rule == SA_HEAT_BATH || p.rule == SA_HEAT_BATH_CLOSED) return chunks + 3.0 * per_lane;
    if (p.rule == SA_OPT_METROPOLIS) return chunks + 1.0 + 0.5 * per_lane;
    return chunks + 1.0;
}

}  // namespace

struct sa_server {
    sa_server_opts opts{};
    int device = 0, cus = 256, max_lds = 65536;
    hipStream_t stream = nullptr;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_prep, cv_sched, cv_done;
    std::deque<Request *> pending;           // waiting for a prep thread
    std::map<uint64_t, Request *> ready;     // prepared, admitted in arrival (id) order
    std::vector<Request *> active;           // owned by the scheduler thread
    std::map<uint64_t, std::unique_ptr<Request>> all;
    std::vector<std::thread> preppers;
    std::thread scheduler;
    bool stop = false;
    int in_prep = 0;
    uint64_t next_id = 1;
    size_t mem_used = 0;
    int64_t n_submitted = 0, n_completed = 0, n_canceled = 0, n_rejected = 0, n_chunks = 0;
    int64_t updates_done = 0;
    // chunk launch buffers (scheduler thread only)
    sa::DevArena chunk_mem;
    size_t chunk_cap = 0;
    // plans of recently submitted instances, reused by later requests with the same instance,
    // bounds and rule (content hash).  A plan's device bytes count in mem_used while at least one
    // admitted request uses it; idle cached plans are bounded by the cache limits instead.
    struct Cached {
        sa_plan *plan = nullptr;
        int64_t refs = 0;      // requests holding the plan (prepared, admitted or running)
        int64_t active = 0;    // admitted requests among them
        uint64_t last_use = 0;
        size_t bytes = 0;
    };
    std::map<std::array<uint64_t, 3>, Cached> plan_cache;
    uint64_t cache_tick = 0;
    int64_t plans_reused = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void finish_locked(sa_server *S, Request *r, int32_t status) {
    r->status = status;
    r->phase = Phase::Done;
    r->t_done = S->now();
    if (status == SA_OK) S->n_completed++;
    else if (status == SA_ECANCELED) S->n_canceled++;
    else S->n_rejected++;
    S->cv_done.notify_all();
}

constexpr size_t kMaxCachedPlans = 64;
// Cost units (cost_of_update x variables) of the median sweep a chunk is sized by, at most: about
// one sweep of a 2000-variable sparse request.
constexpr double kSweepCostCap = 8192.0;

// Frees cached plans no request holds, least recently used first, down to the cache limits
// (entry count, and a quarter of the memory budget).  S->mu held.
void evict_plans_locked(sa_server *S) {
    size_t cached_bytes = 0;
    for (auto &kv : S->plan_cache) cached_bytes += kv.second.bytes;
    for (;;) {
        const bool over = S->plan_cache.size() > kMaxCachedPlans || cached_bytes > S->opts.mem_budget_bytes / 4;
        if (!over) return;
        auto victim = S->plan_cache.end();
        for (auto it = S->plan_cache.begin(); it != S->plan_cache.end(); ++it)
            if (it->second.refs == 0 &&
                (victim == S->plan_cache.end() || it->second.last_use < victim->second.last_use))
                victim = it;
        if (victim == S->plan_cache.end()) return;   // every cached plan is in use
        cached_bytes -= victim->second.bytes;
        delete victim->second.plan;
        S->plan_cache.erase(victim);
    }
}


// Gives up the request's plan: deletes an owned one, releases a cached one.  S->mu held.
void drop_plan_locked(sa_server *S, Request *r) {
    if (r->own_plan && r->plan) delete r->plan;
    if (r->cached) {
        auto it = S->plan_cache.find(r->cache_key);
        if (it != S->plan_cache.end()) {
            it->second.refs--;
            it->second.last_use = ++S->cache_tick;
        }
        r->cached = false;
        evict_plans_locked(S);
    }
    r->plan = nullptr;
    r->own_plan = false;
}

void release_device(sa_server *S, Request *r) {
    if (r->mem) {
        (void)hipFree(r->mem);
        r->mem = nullptr;
    }
    if (r->accounted) {
        S->mem_used -= r->footprint;
        if (r->cached) {
            auto it = S->plan_cache.find(r->cache_key);
            if (it != S->plan_cache.end() && --it->second.active == 0) S->mem_used -= it->second.bytes;
        }
        r->accounted = false;
    }
    drop_plan_locked(S, r);
}

// Content hash of a submitted problem (two independent 64-bit streams plus the rule).
std::array<uint64_t, 3> problem_key(const Request &r) {
    uint64_t h1 = 0x243F6A8885A308D3ull, h2 = 0x13198A2E03707344ull;
    auto mix = [&](uint64_t w) {
        h1 = (h1 ^ w) * 0x9E3779B97F4A7C15ull;
        h1 ^= h1 >> 29;
        h2 = (h2 + w) * 0xC2B2AE3D27D4EB4Full;
        h2 = (h2 << 31) | (h2 >> 33);
    };
    auto bytes = [&](const void *p, size_t n) {
        const unsigned char *c = (const unsigned char *)p;
        size_t i = 0;
        for (; i + 8 <= n; i += 8) {
            uint64_t w;
            std::memcpy(&w, c + i, 8);
            mix(w);
        }
        uint64_t tail = 0;
        std::memcpy(&tail, c + i, n - i);
        mix(tail ^ ((uint64_t)n << 56));
    };
    mix((uint64_t)r.n_vars);
    mix((uint64_t)r.n_terms);
    bytes(r.term_ptr.data(), sizeof(int64_t) * r.term_ptr.size());
    bytes(r.factor_var.data(), sizeof(int32_t) * r.factor_var.size());
    bytes(r.coef.data(), sizeof(int64_t) * r.coef.size());
    bytes(r.lo.data(), sizeof(int32_t) * r.lo.size());
    bytes(r.hi.data(), sizeof(int32_t) * r.hi.size());
    return {h1, h2, (uint64_t)(uint32_t)r.rule};
}

void prep_loop(sa_server *S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_prep.wait(lk, [&] { return S->stop || !S->pending.empty(); });
            if (S->pending.empty()) return;
            r = S->pending.front();
            S->pending.pop_front();
            if (r->cancel) {
                finish_locked(S, r, SA_ECANCELED);
                continue;
            }
            S->in_prep++;
        }
        int rc = SA_OK;
        std::string err;
        if (!r->plan) {
            // a plan of the same instance, bounds and rule may be cached from an earlier request
            const std::array<uint64_t, 3> key = problem_key(*r);
            {
                std::lock_guard<std::mutex> lk(S->mu);
                auto it = S->plan_cache.find(key);
                if (it != S->plan_cache.end()) {
                    it->second.refs++;
                    r->plan = it->second.plan;
                    r->cached = true;
                    r->cache_key = key;
                    S->plans_reused++;
                }
            }
            if (!r->plan) {
                sa_instance inst{r->n_vars, r->n_terms, r->term_ptr.data(), r->factor_var.data(), r->coef.data()};
                sa_bounds bounds{r->lo.data(), r->hi.data()};
                sa_plan *p = nullptr;
                rc = sa::build_plan(&inst, &bounds, r->rule, &p);
                if (rc == SA_OK) {
                    std::lock_guard<std::mutex> lk(S->mu);
                    auto it = S->plan_cache.find(key);
                    if (it != S->plan_cache.end()) {
                        // another preparer cached the same instance meanwhile: use that one
                        delete p;
                        it->second.refs++;
                        r->plan = it->second.plan;
                        S->plans_reused++;
                    } else {
                        auto &e = S->plan_cache[key];
                        e.plan = p;
                        e.refs = 1;
                        e.last_use = ++S->cache_tick;
                        e.bytes = p->arena.bytes;
                        r->plan = p;
                    }
                    r->cached = true;
                    r->cache_key = key;
                } else {
                    err = sa_last_error();
                }
            }
        }
        if (rc == SA_OK) {
            sa_schedule sc{r->n_sweeps, r->beta_in.empty() ? nullptr : r->beta_in.data()};
            rc = sa::resolve_schedule(r->plan, &sc, r->beta);
            if (rc != SA_OK) err = sa_last_error();
        }
        if (rc == SA_OK) {
            // schedules for every team size the scheduler may pick, built here off the hot loop
            for (int G : {1, 2, 4, 8}) {
                sa_plan::Sched *sc = nullptr;
                if (sa::get_schedule(r->plan, G, &sc) != SA_OK) {
                    rc = SA_ENOMEM;
                    err = sa_last_error();
                    break;
                }
            }
        }
        if (rc == SA_OK) {
            const size_t zb = sizeof(int32_t) * (size_t)r->n_reads * (size_t)r->plan->dp.n;
            // a cached plan's arena is counted once, while admitted requests use it (admission)
            r->footprint = align256(sizeof(double) * r->beta.size()) + align256(zb) +
                           align256(sizeof(int64_t) * (size_t)r->n_reads) +
                           (r->own_plan ? r->plan->arena.bytes : 0);
        }
        std::lock_guard<std::mutex> lk(S->mu);
        S->in_prep--;
        if (rc != SA_OK) {
            r->error = err;
            drop_plan_locked(S, r);
            finish_locked(S, r, rc);
        } else if (r->cancel) {
            drop_plan_locked(S, r);
            finish_locked(S, r, SA_ECANCELED);
        } else {
            r->phase = Phase::Prepared;
            S->ready[r->id] = r;
        }
        S->cv_sched.notify_all();
    }
}

// Allocates and fills the device state of an admitted request (scheduler thread, unlocked).
int admit_device(Request *r) {
    const size_t bb = align256(sizeof(double) * r->beta.size());
    const size_t zb = align256(sizeof(int32_t) * (size_t)r->n_reads * (size_t)r->plan->dp.n);
    const size_t eb = align256(sizeof(int64_t) * (size_t)r->n_reads);
    hipError_t e = hipMalloc(&r->mem, bb + zb + eb);
    if (e != hipSuccess) {
        r->mem = nullptr;
        return SA_ENOMEM;
    }
    r->beta_dev = (double *)r->mem;
    r->z_dev = (int32_t *)((char *)r->mem + bb);
    r->e_dev = (int64_t *)((char *)r->mem + bb + zb);
    e = hipMemcpy(r->beta_dev, r->beta.data(), sizeof(double) * r->beta.size(), hipMemcpyHostToDevice);
    return e == hipSuccess ? SA_OK : SA_EDEVICE;
}

// One chunk: every active request advances by up to chunk_sweeps sweeps in one batched launch.
int run_chunk(sa_server *S, const std::vector<Request *> &act, std::string &err) {
    const int n = (int)act.size();
    const int C = S->opts.chunk_sweeps;
    int maxe = 1;
    bool narrow = true, z16 = true;
    for (Request *r : act) {
        maxe = std::max(maxe, sa::maxe_class_of(r->plan->info.max_exponent));
        narrow = narrow && r->plan->narrow_ok;
        for (int32_t k = 0; k < r->plan->dp.n && z16; ++k)
            z16 = r->plan->lo[k] >= INT16_MIN && r->plan->hi[k] <= INT16_MAX;
    }
    const int zsize = z16 ? 2 : 4;
    const int groups_per_cu = 2;
    const int64_t budget = std::min<int64_t>(S->max_lds, 160 * 1024 / groups_per_cu) - 64;
    // sweeps per request in this chunk: a chunk lasts as long as its slowest replica, so every
    // request gets about the same time (C sweeps of the median request), not the same sweeps
    std::vector<double> per_sweep(n);
    for (int i = 0; i < n; ++i) per_sweep[i] = act[i]->plan->dp.n * cost_of_update(*act[i]->plan);
    std::vector<double> sorted(per_sweep);
    std::nth_element(sorted.begin(), sorted.begin() + n / 2, sorted.end());
    // capped, so that a chunk of heavy requests alone stays short: requests are admitted only
    // between chunks, and a long chunk would hold back every arrival behind it
    const double budget_time = C * std::min(sorted[n / 2], kSweepCostCap);
    std::vector<int32_t> sweeps(n);
    for (int i = 0; i < n; ++i) {
        const int32_t left = act[i]->n_sweeps - act[i]->next_sweep;
        const int32_t want = (int32_t)std::max(1.0, std::floor(budget_time / per_sweep[i]));
        sweeps[i] = std::min(left, std::min(want, 16 * C));
    }
    // team sizes: replicas on the chunk's critical path get more cooperating waves
    std::vector<double> cost(n);
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
        cost[i] = (double)sweeps[i] * per_sweep[i];
        total += cost[i] * act[i]->n_reads;
    }
    const double share = total / ((double)S->cus * groups_per_cu * sa::kBatchWaves);
    std::vector<sa::BatchInst> insts(n);
    std::vector<int> team(n);
    int64_t lds_elems = 0;
    for (int i = 0; i < n; ++i) {
        Request *r = act[i];
        sa_plan &p = *r->plan;
        int G = 1;
        while (G < sa::kBatchWaves && cost[i] > 0.25 * share * G) G *= 2;
        for (;;) {
            sa_plan::Sched *sc = &p.sched[G];
            if (G == 1 || (sc->n_win > 0 && (double)sc->n_active / sc->n_win >= 0.6 * G)) break;
            G /= 2;
        }
        const int64_t stride = ((int64_t)p.dp.n + 3) & ~(int64_t)3;
        while (G < sa::kBatchWaves && (int64_t)(sa::kBatchWaves / G) * stride * zsize > budget) G *= 2;
        if ((int64_t)(sa::kBatchWaves / G) * stride * zsize > budget) {
            err = "request state does not fit LDS";
            return SA_EUNSUPPORTED;
        }
        team[i] = G;
        lds_elems = std::max<int64_t>(lds_elems, (int64_t)(sa::kBatchWaves / G) * stride);
        sa::BatchInst &d = insts[i];
        d.P = p.dp;
        d.beta = r->beta_dev;
        d.sched = p.sched[G].dev;
        d.n_win = p.sched[G].n_win;
        d.team = G;
        d.slot_stride = (int32_t)stride;
        d.n_reads = r->n_reads;
        d.n_sweeps = r->n_sweeps;
        d.s_begin = r->next_sweep;
        d.s_end = r->next_sweep + sweeps[i];
        d.resume = r->next_sweep > 0 ? 1 : 0;
        d.rule = p.rule;
        const int cls = sa::reg_chunk_class(p.info.max_width);
        d.chunk = cls == 32 ? 0 : cls;
        d.key0 = (uint32_t)r->seed;
        d.key1 = (uint32_t)(r->seed >> 32);
        d.instance_id = r->instance_id;
        d.z_out = r->z_dev;
        d.e_out = r->e_dev;
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return cost[x] / team[x] > cost[y] / team[y]; });
    std::vector<sa::BatchTask> tasks;
    for (int i : order)
        for (int32_t rd = 0; rd < act[i]->n_reads; rd += sa::kBatchWaves / team[i])
            tasks.push_back(sa::BatchTask{i, rd});
    const size_t o_task = align256(sizeof(sa::BatchInst) * n);
    const size_t o_ctr = o_task + align256(sizeof(sa::BatchTask) * tasks.size());
    const size_t need = o_ctr + 256;
    if (need > S->chunk_cap) {
        if (S->chunk_mem.base) (void)hipFree(S->chunk_mem.base);
        S->chunk_mem.base = nullptr;
        S->chunk_cap = 0;
        hipError_t e = hipMalloc(&S->chunk_mem.base, need * 2);
        if (e != hipSuccess) {
            S->chunk_mem.base = nullptr;
            err = "hipMalloc(chunk)";
            return SA_ENOMEM;
        }
        S->chunk_cap = need * 2;
    }
    char *base = (char *)S->chunk_mem.base;
    std::vector<char> staging(o_ctr, 0);
    std::memcpy(staging.data(), insts.data(), sizeof(sa::BatchInst) * n);
    std::memcpy(staging.data() + o_task, tasks.data(), sizeof(sa::BatchTask) * tasks.size());
    hipError_t e = hipMemcpyAsync(base, staging.data(), o_ctr, hipMemcpyHostToDevice, S->stream);
    if (e != hipSuccess) {
        err = std::string("hipMemcpyAsync(chunk): ") + hipGetErrorString(e);
        return SA_EDEVICE;
    }
    sa::BatchArgs a{};
    a.insts = (const sa::BatchInst *)base;
    a.tasks = (const sa::BatchTask *)(base + o_task);
    a.n_tasks = (int32_t)tasks.size();
    a.counter = (uint32_t *)(base + o_ctr);
    const int32_t state_words = (int32_t)((lds_elems * zsize + 7) / 8 * 2);
    a.parts_words = state_words;
    a.lds_words = state_words + 2 * sa::kBatchWaves;
    a.sweep_limit = 0;
    sa::BatchLaunch bl;
    bl.maxe_class = maxe;
    bl.narrow = narrow && maxe <= 2;
    bl.z16 = z16;
    bl.groups = S->cus * groups_per_cu;
    int rc = sa::launch_batch(a, bl, S->stream, err);
    if (rc != SA_OK) return rc;
    e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) {
        err = std::string("chunk: ") + hipGetErrorString(e);
        return SA_EDEVICE;
    }
    for (int i = 0; i < n; ++i) {
        Request *r = act[i];
        S->updates_done += (int64_t)sweeps[i] * r->n_reads * r->plan->dp.n;
        r->next_sweep += sweeps[i];
    }
    return SA_OK;
}

void scheduler_loop(sa_server *S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        std::vector<Request *> admit;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                // admission in arrival order, by free slots and device-memory footprint
                while (!S->ready.empty() && (int)(S->active.size() + admit.size()) < S->opts.max_slots) {
                    Request *r = S->ready.begin()->second;
                    if (r->cancel) {
                        S->ready.erase(S->ready.begin());
                        release_device(S, r);
                        finish_locked(S, r, SA_ECANCELED);
                        continue;
                    }
                    // the plan's bytes count with the first admitted request that uses it
                    size_t plan_bytes = 0, plan_need = 0;
                    if (r->cached) {
                        auto it = S->plan_cache.find(r->cache_key);
                        if (it != S->plan_cache.end()) {
                            plan_bytes = it->second.bytes;
                            plan_need = it->second.active == 0 ? plan_bytes : 0;
                        }
                    }
                    if (r->footprint + plan_bytes > S->opts.mem_budget_bytes) {
                        S->ready.erase(S->ready.begin());
                        r->error = "request footprint exceeds the server's memory budget";
                        release_device(S, r);
                        finish_locked(S, r, SA_ENOMEM);
                        continue;
                    }
                    if (S->mem_used + r->footprint + plan_need > S->opts.mem_budget_bytes) break;
                    S->ready.erase(S->ready.begin());
                    S->mem_used += r->footprint + plan_need;
                    if (r->cached) {
                        auto it = S->plan_cache.find(r->cache_key);
                        if (it != S->plan_cache.end()) it->second.active++;
                    }
                    r->accounted = true;
                    r->phase = Phase::Active;
                    r->t_admit = S->now();
                    admit.push_back(r);
                }
                if (!S->active.empty() || !admit.empty()) break;
                if (S->stop && S->pending.empty() && S->ready.empty() && S->in_prep == 0) return;
                S->cv_sched.wait(lk);
            }
        }
        for (Request *r : admit) {
            int rc = admit_device(r);
            std::lock_guard<std::mutex> lk(S->mu);
            if (rc != SA_OK) {
                r->error = "device allocation for an admitted request failed";
                release_device(S, r);
                finish_locked(S, r, rc);
            } else {
                S->active.push_back(r);
            }
        }
        if (S->active.empty()) continue;
        std::string err;
        int rc = run_chunk(S, S->active, err);
        std::vector<Request *> keep;
        for (Request *r : S->active) {
            const bool done = rc != SA_OK || r->next_sweep >= r->n_sweeps || r->cancel;
            if (!done) {
                keep.push_back(r);
                continue;
            }
            int32_t status = rc != SA_OK ? rc : (r->next_sweep >= r->n_sweeps ? SA_OK : SA_ECANCELED);
            if (status == SA_OK) {
                const size_t zb = sizeof(int32_t) * (size_t)r->n_reads * (size_t)r->plan->dp.n;
                hipError_t e = hipMemcpy(r->result.states, r->z_dev, zb, hipMemcpyDeviceToHost);
                if (e == hipSuccess)
                    e = hipMemcpy(r->result.energies, r->e_dev, sizeof(int64_t) * (size_t)r->n_reads,
                                  hipMemcpyDeviceToHost);
                if (e != hipSuccess) status = SA_EDEVICE;
            }
            std::lock_guard<std::mutex> lk(S->mu);
            if (status != SA_OK && !err.empty()) r->error = err;
            r->result.status = status;
            release_device(S, r);
            finish_locked(S, r, status);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->active.swap(keep);
            S->n_chunks++;
        }
    }
}

uint64_t enqueue(sa_server *S, std::unique_ptr<Request> req) {
    std::lock_guard<std::mutex> lk(S->mu);
    Request *r = req.get();
    r->id = S->next_id++;
    r->t_submit = S->now();
    S->all[r->id] = std::move(req);
    S->pending.push_back(r);
    S->n_submitted++;
    S->cv_prep.notify_one();
    return r->id;
}

int check_request(const sa_schedule *sched, int32_t rule, int32_t n_reads, const sa_result *result) {
    if (!result || !result->states || !result->energies) return fail(SA_EINVAL, "result buffers are required");
    if (n_reads < 1) return fail(SA_EINVAL, "n_reads must be >= 1");
    if (rule < SA_METROPOLIS || rule > SA_HEAT_BATH_CLOSED) return fail(SA_EINVAL, "unknown rule");
    if (!sched || sched->n_sweeps < 1) return fail(SA_EINVAL, "n_sweeps must be >= 1");
    if (sched->beta)
        for (int32_t s = 0; s < sched->n_sweeps; ++s)
            if (!(sched->beta[s] >= 0.0) || std::isinf(sched->beta[s])) return fail(SA_EINVAL, "beta must be finite and >= 0");
    return SA_OK;
}

}  // namespace

extern "C" {

int32_t sa_server_create(const sa_server_opts *opts, sa_server **out) {
    if (!out) return fail(SA_EINVAL, "server output pointer is NULL");
    *out = nullptr;
    std::unique_ptr<sa_server> S(new sa_server());
    if (opts) S->opts = *opts;
    if (S->opts.mem_budget_bytes == 0) S->opts.mem_budget_bytes = (size_t)16 << 30;
    if (S->opts.max_slots <= 0) S->opts.max_slots = 256;
    if (S->opts.chunk_sweeps <= 0) S->opts.chunk_sweeps = 50;
    if (S->opts.prep_threads <= 0) S->opts.prep_threads = 4;
    hipError_t e = hipGetDevice(&S->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    (void)hipDeviceGetAttribute(&S->cus, hipDeviceAttributeMultiprocessorCount, S->device);
    (void)hipDeviceGetAttribute(&S->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, S->device);
    e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    S->t0 = std::chrono::steady_clock::now();
    sa_server *raw = S.get();
    for (int i = 0; i < S->opts.prep_threads; ++i) S->preppers.emplace_back(prep_loop, raw);
    S->scheduler = std::thread(scheduler_loop, raw);
    *out = S.release();
    return SA_OK;
}

int32_t sa_server_submit(sa_server *S, const sa_problem *q, sa_result *result, uint64_t *ticket) {
    if (!S || !q || !ticket) return fail(SA_EINVAL, "server, problem and ticket are required");
    int rc = check_request(&q->sched, q->rule, q->n_reads, result);
    if (rc != SA_OK) return rc;
    const sa_instance &in = q->inst;
    if (in.n_vars < 1 || in.n_terms < 0 || !q->bounds.lower || !q->bounds.upper ||
        (in.n_terms > 0 && (!in.term_ptr || !in.factor_var || !in.coef)))
        return fail(SA_EINVAL, "malformed instance");
    if (in.n_vars > 40960) return fail(SA_EUNSUPPORTED, "served instances need N <= 40960");
    const size_t state = sizeof(int32_t) * (size_t)q->n_reads * (size_t)in.n_vars;
    if (state > S->opts.mem_budget_bytes) return fail(SA_ENOMEM, "request states exceed the memory budget");
    std::unique_ptr<Request> r(new Request());
    try {
        const int64_t nf = in.n_terms > 0 ? in.term_ptr[in.n_terms] : 0;
        r->term_ptr.assign(in.term_ptr, in.term_ptr + (in.n_terms > 0 ? in.n_terms + 1 : 0));
        if (r->term_ptr.empty()) r->term_ptr.push_back(0);
        r->factor_var.assign(in.factor_var, in.factor_var + nf);
        r->coef.assign(in.coef, in.coef + in.n_terms);
        r->lo.assign(q->bounds.lower, q->bounds.lower + in.n_vars);
        r->hi.assign(q->bounds.upper, q->bounds.upper + in.n_vars);
        if (q->sched.beta) r->beta_in.assign(q->sched.beta, q->sched.beta + q->sched.n_sweeps);
    } catch (const std::bad_alloc &) {
        return fail(SA_ENOMEM, "host allocation failed");
    }
    r->n_vars = in.n_vars;
    r->n_terms = in.n_terms;
    r->rule = q->rule;
    r->n_reads = q->n_reads;
    r->n_sweeps = q->sched.n_sweeps;
    r->seed = q->seed;
    r->instance_id = q->instance_id;
    r->result = *result;
    *ticket = enqueue(S, std::move(r));
    return SA_OK;
}

int32_t sa_server_submit_plan(sa_server *S, sa_plan *plan, const sa_schedule *sched, int32_t n_reads,
                              uint64_t seed, uint32_t instance_id, sa_result *result, uint64_t *ticket) {
    if (!S || !plan || !ticket) return fail(SA_EINVAL, "server, plan and ticket are required");
    int rc = check_request(sched, plan->rule, n_reads, result);
    if (rc != SA_OK) return rc;
    if (plan->device != S->device) return fail(SA_EINVAL, "plan belongs to another device");
    if (plan->dp.n > 40960) return fail(SA_EUNSUPPORTED, "served instances need N <= 40960");
    std::unique_ptr<Request> r(new Request());
    r->plan = plan;
    r->own_plan = false;
    if (sched->beta) r->beta_in.assign(sched->beta, sched->beta + sched->n_sweeps);
    r->n_vars = plan->dp.n;
    r->rule = plan->rule;
    r->n_reads = n_reads;
    r->n_sweeps = sched->n_sweeps;
    r->seed = seed;
    r->instance_id = instance_id;
    r->result = *result;
    *ticket = enqueue(S, std::move(r));
    return SA_OK;
}

int32_t sa_server_poll(sa_server *S, uint64_t ticket, int32_t *done, sa_timing *timing) {
    if (!S || !done) return fail(SA_EINVAL, "server and done are required");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(SA_EINVAL, "unknown ticket");
    Request *r = it->second.get();
    *done = r->phase == Phase::Done ? 1 : 0;
    if (timing) {
        timing->t_submit = r->t_submit;
        timing->t_admit = r->t_admit;
        timing->t_done = r->t_done;
        timing->updates = (uint64_t)r->n_reads * (uint64_t)r->n_sweeps * (uint64_t)r->n_vars;
        timing->status = r->phase == Phase::Done ? r->status : SA_EBUSY;
    }
    if (r->phase == Phase::Done && r->status != SA_OK && !r->error.empty()) fail(r->status, r->error);
    return SA_OK;
}

int32_t sa_server_wait(sa_server *S, uint64_t ticket, sa_timing *timing) {
    if (!S) return fail(SA_EINVAL, "server is required");
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return fail(SA_EINVAL, "unknown ticket");
        Request *r = it->second.get();
        S->cv_done.wait(lk, [&] { return r->phase == Phase::Done; });
    }
    int32_t done = 0;
    sa_timing t{};
    int32_t rc = sa_server_poll(S, ticket, &done, &t);
    if (timing) *timing = t;
    return rc == SA_OK ? t.status : rc;
}

int32_t sa_server_cancel(sa_server *S, uint64_t ticket) {
    if (!S) return fail(SA_EINVAL, "server is required");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(SA_EINVAL, "unknown ticket");
    Request *r = it->second.get();
    if (r->phase == Phase::Done) return SA_OK;
    r->cancel = true;  // honoured at the next hand-over (prep, admission or chunk boundary)
    S->cv_sched.notify_all();
    return SA_OK;
}

int32_t sa_server_get_stats(sa_server *S, sa_server_stats *st) {
    if (!S || !st) return fail(SA_EINVAL, "server and stats are required");
    std::lock_guard<std::mutex> lk(S->mu);
    st->submitted = S->n_submitted;
    st->completed = S->n_completed;
    st->canceled = S->n_canceled;
    st->failed = S->n_rejected;
    st->active = (int64_t)S->active.size();
    st->queued = (int64_t)(S->pending.size() + S->ready.size()) + S->in_prep;
    st->chunks = S->n_chunks;
    st->updates = S->updates_done;
    st->mem_in_use = S->mem_used;
    st->elapsed_s = S->now();
    st->plans_reused = S->plans_reused;
    return SA_OK;
}

void sa_server_destroy(sa_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (auto &kv : S->all)
            if (kv.second->phase != Phase::Done) kv.second->cancel = true;
        S->cv_prep.notify_all();
        S->cv_sched.notify_all();
    }
    for (auto &t : S->preppers) t.join();
    if (S->scheduler.joinable()) S->scheduler.join();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto &kv : S->all) {
            Request *r = kv.second.get();
            if (r->phase != Phase::Done) {
                release_device(S, r);
                finish_locked(S, r, SA_ECANCELED);
            }
        }
    }
    for (auto &kv : S->plan_cache) delete kv.second.plan;
    S->plan_cache.clear();
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
}

}  // extern "C"
