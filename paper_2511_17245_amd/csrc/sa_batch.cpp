// sa_batch.cpp -- many problems annealed by one persistent launch (include/sa.h, batches).
//
// Each problem becomes an ordinary plan (canonical, checked, packed, uploaded) plus its inverse
// temperatures and one-wave schedule; the batch adds a descriptor per problem, a task list of
// (problem, read) ordered longest first, a device task counter and one output arena.  The launch
// geometry (waves per workgroup, persistent workgroups) is either chosen by rule of thumb or tuned
// by timing short trial runs of the real batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "sa_plan.h"

using sa::align256;
using sa::fail;
using sa::hip_fail;

struct sa_batch {
    int device = 0;
    std::vector<std::unique_ptr<sa_plan>> plans;
    std::vector<int32_t> n_reads, n_vars, n_sweeps;
    std::vector<double> replica_cost;  // relative cost of one replica of each problem
    std::vector<size_t> z_off, e_off;  // element offsets of each problem's outputs
    std::vector<sa::BatchInst> insts;  // host copy (team sizes and schedules change with tuning)
    std::vector<int32_t> team;         // chosen waves per replica of each problem
    sa::DevArena arena;
    sa::BatchArgs args{};
    sa::BatchLaunch launch;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t n_tasks = 0, total_updates = 0, max_tasks = 0;
    double tune_ms = 0.0, policy = 0.0;
    int cus = 256, max_lds = 65536;
    bool z16 = false;
    char *base = nullptr;
    size_t o_inst = 0, o_task = 0;
    int32_t *z_dev = nullptr;
    int64_t *e_dev = nullptr;
    ~sa_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

std::mutex g_tune_mu;
struct Tuned {
    double policy;
    int groups_per_cu;
};
std::map<std::string, Tuned> g_tune_cache;  // batch shape -> tuned choice

// Relative cost of one update of a plan's variable (used only to order and size the tasks).
double update_cost(const sa_plan &p) {
    const double chunks = 1.0 + (double)p.info.n_incidences / std::max(1, p.info.n_vars) / 64.0;
    const double per_lane = std::ceil(p.info.max_width / 64.0);
    if (p.rule == SA_HEAT_BATH_CLOSED && p.info.max_exponent <= 1) return chunks + 2.0;
    if (p.rule == SA_HEAT_BATH || p.rule == SA_HEAT_BATH_CLOSED) return chunks + 3.0 * per_lane;
    if (p.rule == SA_OPT_METROPOLIS) return chunks + 1.0 + 0.5 * per_lane;
    return chunks + 1.0;
}

std::string shape_key(const sa_batch &b) {
    return std::to_string(b.plans.size()) + ":" + std::to_string(b.max_tasks) + ":" +
           std::to_string(b.total_updates) + ":" + std::to_string(b.launch.maxe_class) + ":" +
           std::to_string(b.launch.narrow) + ":" + std::to_string(b.z16);
}

// Team sizes, tasks and LDS layout for a policy strength and a workgroup count, uploaded to the
// device.  A replica whose cost exceeds `policy` times a wave's fair share of the batch gets more
// cooperating waves (up to kBatchWaves), as far as its windows keep them busy; every team's state
// must fit the workgroup's share of LDS.  policy = 0 keeps one wave per replica.
int configure(sa_batch &b, double policy, int groups_per_cu) {
    const int32_t n = (int32_t)b.plans.size();
    const int zsize = b.z16 ? 2 : 4;
    const int64_t budget = std::min<int64_t>(b.max_lds, 160 * 1024 / groups_per_cu) - 64;
    const double waves = (double)b.cus * groups_per_cu * sa::kBatchWaves;
    double total = 0.0;
    for (int32_t i = 0; i < n; ++i) total += b.n_reads[i] * b.replica_cost[i];
    const double share = total / waves;
    int64_t lds_elems_max = 0;
    for (int32_t i = 0; i < n; ++i) {
        sa_plan &p = *b.plans[i];
        int G = 1;
        if (policy > 0.0)
            while (G < sa::kBatchWaves && b.replica_cost[i] > policy * share * G) G *= 2;
        while (G > 1) {  // keep cooperating waves busy
            sa_plan::Sched *sc = nullptr;
            int rc = sa::get_schedule(&p, G, &sc);
            if (rc != SA_OK) return rc;
            if (sc->n_win > 0 && (double)sc->n_active / sc->n_win >= 0.6 * G) break;
            G /= 2;
        }
        const int64_t stride = ((int64_t)p.dp.n + 3) & ~(int64_t)3;  // state elements per slot
        while (G < sa::kBatchWaves && (int64_t)(sa::kBatchWaves / G) * stride * zsize > budget) G *= 2;
        if ((int64_t)(sa::kBatchWaves / G) * stride * zsize > budget) return fail(SA_EUNSUPPORTED, "state does not fit");
        sa_plan::Sched *sc = nullptr;
        int rc = sa::get_schedule(&p, G, &sc);
        if (rc != SA_OK) return rc;
        b.team[i] = G;
        b.insts[i].team = G;
        b.insts[i].sched = sc->dev;
        b.insts[i].n_win = sc->n_win;
        b.insts[i].slot_stride = (int32_t)stride;
        lds_elems_max = std::max<int64_t>(lds_elems_max, (int64_t)(sa::kBatchWaves / G) * stride);
    }
    // tasks: problems by decreasing cost of one replica, kBatchWaves / G_p reads per task
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return b.replica_cost[x] / b.team[x] > b.replica_cost[y] / b.team[y]; });
    std::vector<sa::BatchTask> tasks;
    for (int32_t i : order) {
        const int per = sa::kBatchWaves / b.team[i];
        for (int32_t r = 0; r < b.n_reads[i]; r += per) tasks.push_back(sa::BatchTask{i, r});
    }
    b.n_tasks = (int64_t)tasks.size();
    hipError_t e = hipMemcpy(b.base + b.o_inst, b.insts.data(), sizeof(sa::BatchInst) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b.base + b.o_task, tasks.data(), sizeof(sa::BatchTask) * tasks.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(batch tasks)");
    const int32_t state_words = (int32_t)((lds_elems_max * zsize + 7) / 8 * 2);
    b.args.n_tasks = (int32_t)b.n_tasks;
    b.args.parts_words = state_words;
    b.args.lds_words = state_words + 2 * sa::kBatchWaves;
    b.launch.groups = b.cus * groups_per_cu;
    b.launch.waves_per_group = sa::kBatchWaves;
    b.policy = policy;
    if ((int64_t)b.args.lds_words * 4 > b.max_lds) return fail(SA_EUNSUPPORTED, "workgroup LDS too large");
    return SA_OK;
}

int timed_trial(sa_batch &b, int32_t sweep_limit, float *ms) {
    sa::BatchArgs a = b.args;
    a.sweep_limit = sweep_limit;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(SA_EDEVICE, "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SA_EDEVICE, "hipEventCreate");
    }
    std::string err;
    int rc = SA_OK;
    (void)hipEventRecord(e0, b.stream);
    rc = sa::launch_batch(a, b.launch, b.stream, err);
    (void)hipEventRecord(e1, b.stream);
    if (rc == SA_OK) {
        hipError_t e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
        if (e != hipSuccess) rc = hip_fail(e, "batch trial");
    } else {
        fail(rc, err);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int create(const sa_problem *problems, int32_t n, const sa_batch_opts *opts_in, sa_batch **out) {
    if (!out) return fail(SA_EINVAL, "batch output pointer is NULL");
    *out = nullptr;
    if (!problems || n < 1) return fail(SA_EINVAL, "at least one problem is required");
    sa_batch_opts opts{};
    if (opts_in) opts = *opts_in;
    if (opts.waves_per_group != 0 && opts.waves_per_group != sa::kBatchWaves)
        return fail(SA_EINVAL, "waves_per_group must be 0 or 8");
    if (opts.groups < 0) return fail(SA_EINVAL, "groups must be >= 0");
    // host-side checks of every problem before any device work
    for (int32_t i = 0; i < n; ++i) {
        const sa_problem &q = problems[i];
        if (q.n_reads < 1) return fail(SA_EINVAL, "problem " + std::to_string(i) + ": n_reads must be >= 1");
        if (q.sched.n_sweeps < 1) return fail(SA_EINVAL, "problem " + std::to_string(i) + ": n_sweeps must be >= 1");
        if (q.sched.beta)
            for (int32_t s = 0; s < q.sched.n_sweeps; ++s)
                if (!(q.sched.beta[s] >= 0.0) || std::isinf(q.sched.beta[s]))
                    return fail(SA_EINVAL, "problem " + std::to_string(i) + ": beta must be finite and >= 0");
        if (q.inst.n_vars > 40960)
            return fail(SA_EUNSUPPORTED, "problem " + std::to_string(i) + ": batched instances need N <= 40960");
    }
    std::unique_ptr<sa_batch> b(new sa_batch());
    std::vector<std::vector<double>> betas(n);
    int32_t maxe = 1;
    bool narrow = true, z16 = true;
    for (int32_t i = 0; i < n; ++i) {
        const sa_problem &q = problems[i];
        sa_plan *raw = nullptr;
        int rc = sa::build_plan(&q.inst, &q.bounds, q.rule, &raw);
        if (rc != SA_OK) return fail(rc, "problem " + std::to_string(i) + ": " + sa_last_error());
        b->plans.emplace_back(raw);
        rc = sa::resolve_schedule(raw, &q.sched, betas[i]);
        if (rc != SA_OK) return fail(rc, "problem " + std::to_string(i) + ": " + sa_last_error());
        maxe = std::max(maxe, sa::maxe_class_of(raw->info.max_exponent));
        narrow = narrow && raw->narrow_ok;
        for (int32_t k = 0; k < raw->dp.n; ++k) z16 = z16 && raw->lo[k] >= INT16_MIN && raw->hi[k] <= INT16_MAX;
    }
    b->device = b->plans[0]->device;
    (void)hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device);
    (void)hipDeviceGetAttribute(&b->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device);
    b->launch.maxe_class = maxe;
    b->launch.narrow = narrow && maxe <= 2;
    b->launch.z16 = z16;
    b->z16 = z16;

    // device arena: descriptors, tasks (at most one per read), counter, betas, outputs
    b->insts.resize(n);
    b->team.assign(n, 1);
    std::vector<size_t> beta_off(n);
    size_t beta_total = 0, z_total = 0, e_total = 0;
    b->z_off.resize(n);
    b->e_off.resize(n);
    for (int32_t i = 0; i < n; ++i) {
        beta_off[i] = beta_total;
        beta_total += betas[i].size();
        b->z_off[i] = z_total;
        b->e_off[i] = e_total;
        z_total += (size_t)problems[i].n_reads * (size_t)b->plans[i]->dp.n;
        e_total += (size_t)problems[i].n_reads;
        b->n_reads.push_back(problems[i].n_reads);
        b->n_vars.push_back(b->plans[i]->dp.n);
        b->n_sweeps.push_back(problems[i].sched.n_sweeps);
        b->replica_cost.push_back((double)problems[i].sched.n_sweeps * b->plans[i]->dp.n * update_cost(*b->plans[i]));
        b->total_updates += (int64_t)problems[i].n_reads * problems[i].sched.n_sweeps * b->plans[i]->dp.n;
        b->max_tasks += problems[i].n_reads;
    }
    if (b->max_tasks > INT32_MAX) return fail(SA_EINVAL, "too many replicas in one batch");
    b->o_inst = 0;
    b->o_task = b->o_inst + align256(sizeof(sa::BatchInst) * n);
    const size_t o_ctr = b->o_task + align256(sizeof(sa::BatchTask) * (size_t)b->max_tasks);
    const size_t o_beta = o_ctr + 256;
    const size_t o_z = o_beta + align256(sizeof(double) * beta_total);
    const size_t o_e = o_z + align256(sizeof(int32_t) * z_total);
    const size_t total = o_e + align256(sizeof(int64_t) * e_total);
    hipError_t e = hipMalloc(&b->arena.base, total);
    if (e != hipSuccess) {
        b->arena.base = nullptr;
        return fail(SA_ENOMEM, std::string("hipMalloc(batch): ") + hipGetErrorString(e));
    }
    b->arena.bytes = total;
    b->base = (char *)b->arena.base;
    b->z_dev = (int32_t *)(b->base + o_z);
    b->e_dev = (int64_t *)(b->base + o_e);
    std::vector<double> beta_all(beta_total);
    for (int32_t i = 0; i < n; ++i) std::copy(betas[i].begin(), betas[i].end(), beta_all.begin() + beta_off[i]);
    if (beta_total) {
        e = hipMemcpy(b->base + o_beta, beta_all.data(), sizeof(double) * beta_total, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(batch betas)");
    }
    for (int32_t i = 0; i < n; ++i) {
        sa_plan &p = *b->plans[i];
        sa::BatchInst &d = b->insts[i];
        d.P = p.dp;
        d.beta = (const double *)(b->base + o_beta) + beta_off[i];
        d.n_reads = problems[i].n_reads;
        d.n_sweeps = problems[i].sched.n_sweeps;
        d.s_begin = 0;
        d.s_end = d.n_sweeps;
        d.resume = 0;
        d.rule = p.rule;
        const int rc_class = sa::reg_chunk_class(p.info.max_width);
        d.chunk = rc_class == 32 ? 0 : rc_class;
        d.key0 = (uint32_t)problems[i].seed;
        d.key1 = (uint32_t)(problems[i].seed >> 32);
        d.instance_id = problems[i].instance_id;
        d.z_out = b->z_dev + b->z_off[i];
        d.e_out = b->e_dev + b->e_off[i];
    }
    b->args.insts = (const sa::BatchInst *)(b->base + b->o_inst);
    b->args.tasks = (const sa::BatchTask *)(b->base + b->o_task);
    b->args.counter = (uint32_t *)(b->base + o_ctr);
    b->args.sweep_limit = 0;

    if (opts.hip_stream) {
        b->stream = (hipStream_t)opts.hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        b->own_stream = true;
    }

    // choose the team-size policy and the number of persistent workgroups
    Tuned choice{0.5, 2};
    const std::string key = shape_key(*b);
    bool cached = false;
    if (opts.autotune) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            choice = it->second;
            cached = true;
        }
    }
    if (opts.autotune && !cached) {
        int32_t max_s = 1;
        for (int32_t i = 0; i < n; ++i) max_s = std::max(max_s, problems[i].sched.n_sweeps);
        const int32_t trial_sweeps = std::max<int32_t>(1, std::min<int32_t>(max_s, std::max(10, max_s / 20)));
        float best_ms = 1e30f;
        for (double policy : {0.0, 0.25, 0.5, 1.0}) {
            for (int gpc : {1, 2}) {
                if (configure(*b, policy, gpc) != SA_OK) continue;
                float ms = 0.f;
                int rc = timed_trial(*b, trial_sweeps, &ms);
                if (rc != SA_OK) return rc;
                b->tune_ms += ms;
                if (ms < best_ms) {
                    best_ms = ms;
                    choice = Tuned{policy, gpc};
                }
            }
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = choice;
    }
    int rc = configure(*b, choice.policy, choice.groups_per_cu);
    if (rc != SA_OK && choice.groups_per_cu > 1) rc = configure(*b, choice.policy, 1);
    if (rc != SA_OK) return rc;
    if (opts.groups) b->launch.groups = opts.groups;

    if (opts.use_graph) {
        e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        std::string err;
        rc = sa::launch_batch(b->args, b->launch, b->stream, err);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->stream, &g);
        if (rc != SA_OK) {
            if (g) (void)hipGraphDestroy(g);
            return fail(rc, err);
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    }
    *out = b.release();
    return SA_OK;
}

int run(sa_batch *b) {
    if (!b) return fail(SA_EINVAL, "batch is NULL");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != b->device) return fail(SA_EINVAL, "batch belongs to another device");
    if (b->exec) {
        hipError_t e = hipGraphLaunch(b->exec, b->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        return SA_OK;
    }
    std::string err;
    int rc = sa::launch_batch(b->args, b->launch, b->stream, err);
    return rc == SA_OK ? SA_OK : fail(rc, err);
}

int wait(sa_batch *b) {
    if (!b) return fail(SA_EINVAL, "batch is NULL");
    hipError_t e = hipStreamSynchronize(b->stream);
    return e == hipSuccess ? SA_OK : hip_fail(e, "batch run");
}

int results(sa_batch *b, sa_result *res) {
    if (!b || !res) return fail(SA_EINVAL, "batch and results are required");
    const int32_t n = (int32_t)b->plans.size();
    for (int32_t i = 0; i < n; ++i)
        if (!res[i].states || !res[i].energies) return fail(SA_EINVAL, "result " + std::to_string(i) + " has no buffers");
    int rc = wait(b);
    if (rc != SA_OK) return rc;
    for (int32_t i = 0; i < n; ++i) {
        const size_t zb = sizeof(int32_t) * (size_t)b->n_reads[i] * (size_t)b->n_vars[i];
        hipError_t e = hipMemcpy(res[i].states, b->z_dev + b->z_off[i], zb, hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(res[i].energies, b->e_dev + b->e_off[i], sizeof(int64_t) * (size_t)b->n_reads[i],
                          hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "batch results");
        res[i].status = SA_OK;
    }
    return SA_OK;
}

}  // namespace

extern "C" {

int32_t sa_batch_create(const sa_problem *problems, int32_t n_problems, const sa_batch_opts *opts,
                        sa_batch **out) {
    try {
        return create(problems, n_problems, opts, out);
    } catch (const std::bad_alloc &) {
        return fail(SA_ENOMEM, "host allocation failed");
    } catch (const std::exception &ex) {
        return fail(SA_EINVAL, ex.what());
    }
}

int32_t sa_batch_run(sa_batch *batch) { return run(batch); }
int32_t sa_batch_wait(sa_batch *batch) { return wait(batch); }
int32_t sa_batch_results(sa_batch *batch, sa_result *results_out) { return results(batch, results_out); }

int32_t sa_batch_get_info(const sa_batch *b, sa_batch_info *info) {
    if (!b || !info) return fail(SA_EINVAL, "batch and info are required");
    info->n_problems = (int32_t)b->plans.size();
    info->n_tasks = b->n_tasks;
    info->total_updates = b->total_updates;
    info->waves_per_group = b->launch.waves_per_group;
    info->groups = b->launch.groups;
    info->slot_bytes = b->args.lds_words * 4;
    int32_t tmax = 1;
    for (int32_t t : b->team) tmax = std::max(tmax, t);
    info->max_team = tmax;
    info->policy = b->policy;
    info->kernel_maxe = b->launch.maxe_class;
    info->kernel_bits = b->launch.narrow ? 32 : 64;
    info->state_bits = b->launch.z16 ? 16 : 32;
    info->graph = b->exec ? 1 : 0;
    info->tune_ms = b->tune_ms;
    return SA_OK;
}

void sa_batch_destroy(sa_batch *batch) { delete batch; }

int32_t sa_anneal_batch(const sa_problem *problems, int32_t n_problems, sa_result *results_out,
                        const sa_batch_opts *opts) {
    sa_batch *b = nullptr;
    int32_t rc = sa_batch_create(problems, n_problems, opts, &b);
    if (rc != SA_OK) return rc;
    rc = sa_batch_run(b);
    if (rc == SA_OK) rc = sa_batch_results(b, results_out);
    sa_batch_destroy(b);
    return rc;
}

}  // extern "C"
