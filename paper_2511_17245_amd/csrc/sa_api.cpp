// sa_api.cpp -- the C ABI of include/sa.h: plans (a canonical instance packed in device memory),
// one-shot annealing, energies and error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "sa_plan.h"

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace sa {

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(SA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

}  // namespace sa

using sa::align256;
using sa::fail;
using sa::hip_fail;

namespace {

int upload_packed(const sa::Packed &pk, sa_plan *plan) {
    const sa::PackedLayout L = sa::packed_layout(pk);
    hipError_t e = hipMalloc(&plan->arena.base, L.total);
    if (e != hipSuccess) return fail(SA_ENOMEM, std::string("hipMalloc(plan): ") + hipGetErrorString(e));
    plan->arena.bytes = L.total;
    std::vector<char> staging(L.total, 0);
    sa::stage_packed(pk, L, staging.data());
    e = hipMemcpy(plan->arena.base, staging.data(), L.total, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(plan)");
    sa::bind_packed(pk, L, (char *)plan->arena.base, plan->dp);
    return SA_OK;
}

}  // namespace

namespace sa {

namespace {
// the parts of a packed instance in their device order
std::vector<std::pair<const void *, size_t>> packed_parts(const Packed &pk) {
    return {
        {pk.var.data(), pk.var.size() * sizeof(VarRec)},
        {pk.emask.data(), pk.emask.size() * sizeof(uint32_t)},
        {pk.inc.data(), pk.inc.size() * sizeof(IncRec)},
        {pk.inc_coef.data(), pk.inc_coef.size() * sizeof(int64_t)},
        {pk.overflow.data(), pk.overflow.size() * sizeof(int32_t)},
        {pk.t_off.data(), pk.t_off.size() * sizeof(int32_t)},
        {pk.t_var.data(), pk.t_var.size() * sizeof(int32_t)},
        {pk.t_coef.data(), pk.t_coef.size() * sizeof(int64_t)},
        {pk.jbytes == 1 ? (const void *)pk.jd8.data() : (const void *)pk.jd32.data(),
         pk.jbytes == 1 ? pk.jd8.size() : pk.jd32.size() * sizeof(int32_t)},
        {pk.h.data(), pk.h.size() * sizeof(int64_t)},
        {pk.d.data(), pk.d.size() * sizeof(int64_t)},
        {pk.pair.data(), pk.pair.size() * sizeof(PairRec)},
    };
}
}  // namespace

PackedLayout packed_layout(const Packed &pk) {
    // the incidence records and their coefficients are followed by one zero record, which lanes
    // past the end of a row read
    const auto parts = packed_parts(pk);
    const size_t extra[PackedLayout::kParts] = {0, 0, sizeof(IncRec), sizeof(int64_t), 0, 0, 0, 0, 0, 0, 0, 0};
    PackedLayout L;
    size_t total = 0;
    for (int i = 0; i < PackedLayout::kParts; ++i) {
        L.off[i] = total;
        const size_t b = parts[(size_t)i].second + extra[i];
        total += align256(b > 0 ? b : 1);
    }
    L.total = total;
    return L;
}

void stage_packed(const Packed &pk, const PackedLayout &L, char *image) {
    const auto parts = packed_parts(pk);
    for (int i = 0; i < PackedLayout::kParts; ++i) {
        const size_t end = i + 1 < PackedLayout::kParts ? L.off[i + 1] : L.total;
        std::memset(image + L.off[i], 0, end - L.off[i]);
        if (parts[(size_t)i].second) std::memcpy(image + L.off[i], parts[(size_t)i].first, parts[(size_t)i].second);
    }
}

void bind_packed(const Packed &pk, const PackedLayout &L, char *b, DevProblem &d) {
    d.n = pk.n;
    d.n_terms = pk.n_terms;
    d.var = (const VarRec *)(b + L.off[0]);
    d.emask = (const uint32_t *)(b + L.off[1]);
    d.inc = (const IncRec *)(b + L.off[2]);
    d.inc_coef = (const int64_t *)(b + L.off[3]);
    d.overflow = (const int32_t *)(b + L.off[4]);
    d.t_off = (const int32_t *)(b + L.off[5]);
    d.t_var = (const int32_t *)(b + L.off[6]);
    d.t_coef = (const int64_t *)(b + L.off[7]);
    d.max_other = pk.max_other;
    d.inc_pad = (int32_t)pk.inc.size();
    d.dense = pk.dense ? 1 : 0;
    d.jbytes = pk.jbytes;
    d.row_stride = pk.row_stride;
    d.jd = (const void *)(b + L.off[8]);
    d.h = (const int64_t *)(b + L.off[9]);
    d.d = (const int64_t *)(b + L.off[10]);
    d.pair = pk.pair_row.empty() ? nullptr : (const PairRec *)(b + L.off[11]);
}

}  // namespace sa

namespace sa {

int check_rule_support(int rule, int32_t max_exp) {
    if (rule < SA_METROPOLIS || rule > SA_HEAT_BATH_CLOSED) return fail(SA_EINVAL, "unknown rule");
    if (rule == SA_OPT_METROPOLIS && max_exp > 4)
        return fail(SA_EUNSUPPORTED,
                    "optimal-transition Metropolis needs every exponent <= 4 (energy difference of "
                    "degree <= 4)");
    if ((rule == SA_HEAT_BATH || rule == SA_HEAT_BATH_CLOSED) && max_exp > sa::kMaxExpPoly)
        return fail(SA_EUNSUPPORTED, "heat bath supports exponents up to 16 on the GPU");
    return SA_OK;
}

// Waves per replica.  The sweep is latency-bound (one dependent chain per replica), so the widest
// window G in {16, 8, 4, 2} is taken whose waves stay busy (mean window size >= 0.6 G), whose
// shared state fits in LDS and whose n_reads x G waves are all resident at once; otherwise G = 1.
// The annealing variants use 84 to 128 VGPRs, which leaves room for 4 waves per SIMD: a wider G
// would run the replicas in two rounds (measured slower, e.g. 8 against 4 waves per replica for
// 1024 replicas of the N = 2000 HUIO problem: 573 against 508 ms).
int pick_waves_per_replica(int32_t n, int32_t n_reads, int device,
                           const std::function<bool(int, int32_t &, int32_t &)> &windows) {
    int cus = 256, max_lds = 65536;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    const int64_t max_waves = (int64_t)cus * 4 * 4;
    for (int G = 16; G > 1; G /= 2) {
        if ((int64_t)n_reads * G > max_waves) continue;
        if (shared_state_bytes(n, G) > max_lds) continue;
        int32_t n_win = 0, n_active = 0;
        if (!windows(G, n_win, n_active) || n_win == 0) continue;
        if ((double)n_active / (double)n_win >= 0.6 * G) return G;
    }
    return 1;
}

}  // namespace sa

namespace sa {

int build_plan(const sa_instance *inst, const sa_bounds *bounds, int32_t rule, sa_plan **out) {
    if (!out) return fail(SA_EINVAL, "plan output pointer is NULL");
    *out = nullptr;
    std::string err;
    sa::Canonical canon;
    int rc = sa::canonicalize(inst, bounds, canon, err);
    if (rc != SA_OK) return fail(rc, err);
    double bound = 0.0;
    rc = sa::check_int64_bound(canon, err, &bound);
    if (rc != SA_OK) return fail(rc, err);
    sa::Packed pk;
    rc = sa::pack(canon, pk, err);
    if (rc != SA_OK) return fail(rc, err);
    rc = check_rule_support(rule, pk.max_exp);
    if (rc != SA_OK) return rc;
    std::unique_ptr<sa_plan> plan(new sa_plan());
    hipError_t e = hipGetDevice(&plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    plan->rule = rule;
    plan->lo = canon.lo;
    plan->hi = canon.hi;
    plan->narrow_ok = sa::dE_fits_32(canon);
    plan->auto_status = sa::auto_temperatures(canon, &plan->t_init, &plan->t_final, plan->auto_error);
    rc = upload_packed(pk, plan.get());
    if (rc != SA_OK) return rc;
    plan->dp.coef32 = sa::coefs_fit_32(canon) ? 1 : 0;
    sa_plan_info &in = plan->info;
    in.n_vars = pk.n;
    in.n_terms = pk.n_terms;
    in.n_incidences = pk.dense ? 2 * pk.n_pairs : (int64_t)pk.inc.size();
    in.dense = pk.dense ? 1 : 0;
    int64_t slots = (int64_t)pk.overflow.size();
    for (const auto &r : pk.inc) slots += std::min<int64_t>(r.meta >> 8, 3);
    in.n_factor_slots = slots;
    in.max_exponent = pk.max_exp;
    in.max_width = pk.max_width;
    in.device_bytes = (int64_t)plan->arena.bytes;
    in.coef_bits = 64;
    in.arith_bits = plan->narrow_ok && pk.max_exp <= 2 ? 32 : 64;
    plan->packed = std::move(pk);
    *out = plan.release();
    return SA_OK;
}

int resolve_schedule(sa_plan *plan, const sa_schedule *sched, std::vector<double> &beta) {
    if (!sched || sched->n_sweeps < 1) return fail(SA_EINVAL, "schedule with n_sweeps >= 1 is required");
    beta.resize((size_t)sched->n_sweeps);
    if (sched->beta) {
        for (int32_t s = 0; s < sched->n_sweeps; ++s) {
            double b = sched->beta[s];
            if (!(b >= 0.0) || std::isinf(b)) return fail(SA_EINVAL, "beta must be finite and >= 0");
            beta[s] = b;
        }
    } else {
        if (plan->auto_status != SA_OK) return fail(plan->auto_status, plan->auto_error);
        sa::geometric_betas(plan->t_init, plan->t_final, sched->n_sweeps, beta.data());
    }
    return SA_OK;
}

int stage_beta(sa_plan *plan, const std::vector<double> &beta, hipStream_t stream) {
    const int32_t S = (int32_t)beta.size();
    if (plan->beta_dev && plan->beta_host == beta) return SA_OK;
    if (S > plan->beta_cap) {
        if (plan->beta_dev) (void)hipFree(plan->beta_dev);
        plan->beta_dev = nullptr;
        plan->beta_cap = 0;
        hipError_t e = hipMalloc(&plan->beta_dev, sizeof(double) * (size_t)S);
        if (e != hipSuccess) return fail(SA_ENOMEM, std::string("hipMalloc(beta): ") + hipGetErrorString(e));
        plan->beta_cap = S;
    }
    hipError_t e = hipMemcpyAsync(plan->beta_dev, beta.data(), sizeof(double) * (size_t)S,
                                  hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(beta)");
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(beta)");
    plan->beta_host = beta;
    return SA_OK;
}

int get_schedule(sa_plan *plan, int G, sa_plan::Sched **out) {
    std::lock_guard<std::mutex> lk(plan->sched_mu);
    sa_plan::Sched &sc = plan->sched[G];
    if (!sc.dev) {
        std::vector<sa::SchedRec> host;
        const int32_t n_win = sa::build_schedule(plan->packed, G, host);
        int32_t active = 0;
        for (const auto &vr : plan->packed.var) active += vr.width > 1 ? 1 : 0;
        const size_t bytes = std::max<size_t>(host.size(), 1) * sizeof(sa::SchedRec);
        hipError_t e = hipMalloc(&sc.dev, bytes);
        if (e != hipSuccess) {
            sc.dev = nullptr;
            return fail(SA_ENOMEM, std::string("hipMalloc(schedule): ") + hipGetErrorString(e));
        }
        if (!host.empty()) {
            e = hipMemcpy(sc.dev, host.data(), host.size() * sizeof(sa::SchedRec), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy(schedule)");
        }
        sc.n_win = n_win;
        sc.n_active = active;
    }
    *out = &sc;
    return SA_OK;
}

int get_levels(sa_plan *plan, sa_plan::Levels **out) {
    std::lock_guard<std::mutex> lk(plan->sched_mu);
    sa_plan::Levels &lv = plan->levels;
    if (lv.n_levels < 0) {
        std::vector<int32_t> start;
        std::vector<SchedRec> slots;
        const bool mo = plan->rule == SA_METROPOLIS || plan->rule == SA_OPT_METROPOLIS;
        int32_t n_real = 0;
        const int32_t nl = mo ? build_rounds(plan->packed, slots, n_real)
                              : build_levels(plan->packed,
                                             quad_waves(plan->rule, plan->packed.max_width, plan->packed.max_exp,
                                                        quad_uniform_width(plan->packed)) * 16,
                                             start, slots);
        if (!mo) n_real = (int32_t)slots.size();
        std::vector<MoRec> mrec;
        std::vector<uint8_t> mcoef;
        if (mo) build_mo_records(plan->packed, slots, plan->dp.coef32 != 0, mrec, mcoef);
        const size_t sb = align256(start.size() * sizeof(int32_t));
        const size_t rb = sb + align256(std::max<size_t>(slots.size(), 1) * sizeof(SchedRec));
        const size_t cb = rb + align256(mrec.size() * sizeof(MoRec));
        const size_t bytes = cb + std::max<size_t>(mcoef.size(), 1);
        hipError_t e = hipMalloc(&lv.dev, bytes);
        if (e != hipSuccess) {
            lv.dev = nullptr;
            return fail(SA_ENOMEM, std::string("hipMalloc(levels): ") + hipGetErrorString(e));
        }
        std::vector<char> img(bytes, 0);
        std::memcpy(img.data(), start.data(), start.size() * sizeof(int32_t));
        if (!slots.empty()) std::memcpy(img.data() + sb, slots.data(), slots.size() * sizeof(SchedRec));
        if (!mrec.empty()) std::memcpy(img.data() + rb, mrec.data(), mrec.size() * sizeof(MoRec));
        if (!mcoef.empty()) std::memcpy(img.data() + cb, mcoef.data(), mcoef.size());
        e = hipMemcpy(lv.dev, img.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(levels)");
        lv.start = (const int32_t *)lv.dev;
        lv.slots = (const SchedRec *)((char *)lv.dev + sb);
        lv.mrec = mo ? (const MoRec *)((char *)lv.dev + rb) : nullptr;
        lv.mcoef = mo ? (const void *)((char *)lv.dev + cb) : nullptr;
        lv.n_slots = n_real;
        lv.n_rounds = mo ? (int32_t)(slots.size() / kRoundQuads) : 0;
        lv.uniform_width = mo ? 0 : uniform_width(slots);
        lv.n_levels = nl;
    }
    *out = &lv;
    return SA_OK;
}

int32_t uniform_width(const std::vector<SchedRec> &slots) {
    if (slots.empty()) return 0;
    for (const auto &sl : slots)
        if (sl.width != slots[0].width) return 0;
    return slots[0].width;
}

bool quad_eligible(int rule, const Packed &pk, int device) {
    const bool heat_bath = rule == SA_HEAT_BATH || rule == SA_HEAT_BATH_CLOSED;
    if (pk.dense || pk.max_exp > (heat_bath ? 2 : 4) || pk.max_width > 4 * kQuadMaxR) return false;
    int max_lds = 65536;
    (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    const bool mo = rule == SA_METROPOLIS || rule == SA_OPT_METROPOLIS;   // + the constant 1 after the state
    return shared_state_bytes(pk.n + (mo ? 1 : 0), quad_waves(rule, pk.max_width, pk.max_exp, quad_uniform_width(pk))) <=
           max_lds;
}

int choose_lanes(int32_t quads, int requested, int waves_per_replica, bool eligible, int32_t n_levels,
                 int32_t n_slots) {
    if (requested != 0 && requested != 4 && requested != 64)
        return fail(SA_EINVAL, "lanes_per_update must be 0, 4 or 64"), -1;
    if (requested == 64) return 64;
    if (requested == 4) {
        if (!eligible || waves_per_replica != 0)
            return fail(SA_EINVAL, "lanes_per_update = 4 needs a sparse problem with ranges of at most 128 "
                                   "values, exponents <= 2 (heat bath) or <= 4 (Metropolis, optimal "
                                   "transition), its state in LDS and waves_per_replica = 0"),
                   -1;
        return 4;
    }
    if (!eligible || waves_per_replica != 0 || n_levels <= 0) return 64;
    // the quad kernel when its levels fill, on average, half a workgroup's quads
    return (int64_t)n_slots * 2 >= (int64_t)quads * (int64_t)n_levels ? 4 : 64;
}

int reg_chunk_class(int32_t max_width) {
    const int64_t chunk = ((int64_t)max_width + 63) / 64;
    return chunk <= 1 ? 1 : chunk <= 2 ? 2 : chunk <= 8 ? 8 : chunk <= kHeatBathRegChunk ? 32 : 0;
}

}  // namespace sa

namespace {

using sa::get_schedule;
using sa::stage_beta;
using sa::resolve_schedule;

int auto_waves_per_replica(sa_plan *plan, int32_t n_reads, int device) {
    return sa::pick_waves_per_replica(plan->dp.n, n_reads, device, [&](int G, int32_t &n_win, int32_t &n_active) {
        sa_plan::Sched *sc = nullptr;
        if (get_schedule(plan, G, &sc) != SA_OK) return false;
        n_win = sc->n_win;
        n_active = sc->n_active;
        return true;
    });
}

int plan_run(sa_plan *plan, const sa_schedule *sched, int32_t n_reads, uint64_t seed,
             int32_t *out_states, int64_t *out_energies, const sa_opts *opts_in) {
    if (!plan) return fail(SA_EINVAL, "plan is NULL");
    sa_opts opts;
    sa_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    if (n_reads < 1) return fail(SA_EINVAL, "n_reads must be >= 1");
    if (!out_states || !out_energies) return fail(SA_EINVAL, "output buffers are required");
    std::vector<double> beta;
    int rc = resolve_schedule(plan, sched, beta);
    if (rc != SA_OK) return rc;
    const int32_t S = sched->n_sweeps;
    const int32_t s0 = opts.sweep_begin;
    const int32_t s1 = opts.sweep_end <= 0 ? S : opts.sweep_end;
    if (s0 < 0 || s1 < s0 || s1 > S) return fail(SA_EINVAL, "sweep range outside the schedule");
    const int32_t n = plan->dp.n;
    if (opts.init_states && !opts.device_buffers) {
        // host start states are checked against the box before any device work
        for (int64_t r = 0; r < n_reads; ++r)
            for (int32_t k = 0; k < n; ++k) {
                const int32_t v = opts.init_states[r * n + k];
                if (v < plan->lo[k] || v > plan->hi[k]) return fail(SA_EINVAL, "init_states outside the bounds");
            }
    }
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != plan->device) return fail(SA_EINVAL, "plan was created on another device");
    hipStream_t stream = (hipStream_t)opts.hip_stream;
    rc = stage_beta(plan, beta, stream);
    if (rc != SA_OK) return rc;

    const size_t zbytes = (size_t)n_reads * (size_t)n * sizeof(int32_t);
    const size_t ebytes = (size_t)n_reads * sizeof(int64_t);
    const int32_t n_traced = s1 - s0;
    const size_t tbytes = opts.trace_hashes ? (size_t)n_reads * (size_t)n_traced * sizeof(uint64_t) : 0;
    int32_t *z_dev = out_states;
    int64_t *e_dev = out_energies;
    uint64_t *t_dev = opts.trace_hashes;
    const int32_t *zi_dev = opts.init_states;
    void *tmp = nullptr;
    if (!opts.device_buffers) {
        size_t need = align256(zbytes) + align256(ebytes) + (opts.init_states ? align256(zbytes) : 0) +
                      align256(tbytes);
        e = hipMalloc(&tmp, need);
        if (e != hipSuccess) return fail(SA_ENOMEM, std::string("hipMalloc(run): ") + hipGetErrorString(e));
        z_dev = (int32_t *)tmp;
        e_dev = (int64_t *)((char *)tmp + align256(zbytes));
        size_t off = align256(zbytes) + align256(ebytes);
        if (opts.init_states) {
            int32_t *zi = (int32_t *)((char *)tmp + off);
            off += align256(zbytes);
            e = hipMemcpyAsync(zi, opts.init_states, zbytes, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) {
                (void)hipFree(tmp);
                return hip_fail(e, "hipMemcpyAsync(init)");
            }
            zi_dev = zi;
        }
        if (opts.trace_hashes) t_dev = (uint64_t *)((char *)tmp + off);
    }
    if (t_dev) {
        std::string zerr;
        rc = sa::launch_zero_u64(t_dev, (int64_t)n_reads * n_traced, stream, zerr);
        if (rc != SA_OK) {
            if (tmp) (void)hipFree(tmp);
            return fail(rc, zerr);
        }
    }
    sa::AnnealArgs a{};
    a.P = plan->dp;
    a.beta = plan->beta_dev;
    a.n_sweeps = S;
    a.s_begin = s0;
    a.s_end = s1;
    a.n_reads = n_reads;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.instance_id = opts.instance_id;
    a.otm_r = opts.otm_r;
    if (opts.otm_enum_max < 0) {
        if (tmp) (void)hipFree(tmp);
        return fail(SA_EINVAL, "otm_enum_max must be >= 0");
    }
    a.otm_enum_max = opts.otm_enum_max > 0 ? opts.otm_enum_max : sa::kOtmEnumMax;
    a.z_init = zi_dev;
    a.z_out = z_dev;
    a.e_out = e_dev;
    a.trace = t_dev;
    int G = opts.waves_per_replica;
    if (G != 0 && G != 1 && G != 2 && G != 4 && G != 8 && G != 16) {
        if (tmp) (void)hipFree(tmp);
        return fail(SA_EINVAL, "waves_per_replica must be 0, 1, 2, 4, 8 or 16");
    }
    const bool eligible = sa::quad_eligible(plan->rule, plan->packed, plan->device);
    sa_plan::Levels *lv = nullptr;
    if (eligible && G == 0 && opts.lanes_per_update != 64) {
        rc = sa::get_levels(plan, &lv);
        if (rc != SA_OK) {
            if (tmp) (void)hipFree(tmp);
            return rc;
        }
    }
    const int qwaves = sa::quad_waves(plan->rule, plan->packed.max_width, plan->packed.max_exp,
                                      sa::quad_uniform_width(plan->packed));
    const int lanes = sa::choose_lanes(qwaves * 16, opts.lanes_per_update, G, eligible, lv ? lv->n_levels : 0,
                                       lv ? lv->n_slots : 0);
    if (lanes < 0) {
        if (tmp) (void)hipFree(tmp);
        return SA_EINVAL;
    }
    if (lanes == 4) {
        sa::QuadArgs q{};
        q.P = plan->dp;
        q.beta = plan->beta_dev;
        q.n_sweeps = S;
        q.s_begin = s0;
        q.s_end = s1;
        q.n_reads = n_reads;
        q.key0 = a.key0;
        q.key1 = a.key1;
        q.instance_id = a.instance_id;
        q.level_start = lv->start;
        q.slots = lv->slots;
        q.n_levels = lv->n_levels;
        q.n_rounds = lv->n_rounds;
        q.mrec = lv->mrec;
        q.mcoef = lv->mcoef;
        q.uniform_width = lv->uniform_width;
        q.otm_r = a.otm_r;
        q.z_init = zi_dev;
        q.z_out = z_dev;
        q.e_out = e_dev;
        q.trace = t_dev;
        std::string err;
        const bool mo = plan->rule == SA_METROPOLIS || plan->rule == SA_OPT_METROPOLIS;
        rc = (mo ? sa::launch_quad_mo : sa::launch_quad)(plan->rule, q, plan->info.max_width,
                                                          plan->info.max_exponent, plan->narrow_ok, stream, err);
        if (rc == SA_OK && t_dev) rc = sa::launch_trace_prefix(t_dev, n_reads, n_traced, stream, err);
        if (rc != SA_OK) {
            if (tmp) (void)hipFree(tmp);
            return fail(rc, err);
        }
        plan->last = sa_launch_info{};
        const int qw = qwaves;
        plan->last.waves_per_group = qw;
        plan->last.groups = n_reads;
        plan->last.lds_bytes = (int32_t)sa::shared_state_bytes(n, qw);
        plan->last.state_in_lds = 1;
        plan->last.kernel_variant = 2000000 + plan->rule * 100000;
        plan->last.waves_per_replica = qw;
        plan->last.lanes_per_update = 4;
        plan->last.n_levels = lv->n_levels;
    } else {
        if (G == 0) G = auto_waves_per_replica(plan, n_reads, plan->device);
        sa::LaunchChoice lc = sa::choose_launch(plan->rule, n, n_reads, plan->info.max_width,
                                                plan->info.max_exponent, plan->device, G, plan->narrow_ok,
                                                a.otm_enum_max, plan->packed.dense);
        sa_plan::Sched *sc = nullptr;
        rc = get_schedule(plan, lc.win_waves, &sc);
        if (rc != SA_OK) {
            if (tmp) (void)hipFree(tmp);
            return rc;
        }
        a.sched = sc->dev;
        a.n_win = sc->n_win;
        a.win_waves = lc.win_waves;
        a.waves_per_group = lc.waves_per_group;
        a.dense_cache = lc.dense_cache ? 1 : 0;
        std::string err;
        rc = sa::launch_anneal(plan->rule, a, lc, stream, err);
        if (rc == SA_OK && t_dev) rc = sa::launch_trace_prefix(t_dev, n_reads, n_traced, stream, err);
        if (rc != SA_OK) {
            if (tmp) (void)hipFree(tmp);
            return fail(rc, err);
        }
        plan->last.waves_per_group = lc.waves_per_group;
        plan->last.groups = lc.groups;
        plan->last.lds_bytes = lc.lds_bytes;
        plan->last.state_in_lds = lc.state_in_lds ? 1 : 0;
        plan->last.kernel_variant = lc.variant;
        plan->last.waves_per_replica = lc.win_waves;
        plan->last.n_windows = sc->n_win;
        plan->last.lanes_per_update = 64;
        plan->last.n_levels = 0;
    }
    if (!opts.device_buffers) {
        e = hipMemcpyAsync(out_states, z_dev, zbytes, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(out_energies, e_dev, ebytes, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess && tbytes)
            e = hipMemcpyAsync(opts.trace_hashes, t_dev, tbytes, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        (void)hipFree(tmp);
        if (e != hipSuccess) return hip_fail(e, "annealing run");
    }
    return SA_OK;
}

}  // namespace

extern "C" {

void sa_opts_default(sa_opts *opts) {
    if (!opts) return;
    std::memset(opts, 0, sizeof(*opts));
    opts->otm_r = -1.0;
}

int32_t sa_plan_create(const sa_instance *inst, const sa_bounds *bounds, int32_t rule, sa_plan **out) {
    g_last_error.clear();
    try {
        return sa::build_plan(inst, bounds, rule, out);
    } catch (const std::bad_alloc &) {
        return fail(SA_ENOMEM, "host allocation failed");
    } catch (const std::exception &ex) {
        return fail(SA_EINVAL, ex.what());
    }
}

int32_t sa_plan_run(sa_plan *plan, const sa_schedule *sched, int32_t n_reads, uint64_t seed,
                    int32_t *out_states, int64_t *out_energies, const sa_opts *opts) {
    g_last_error.clear();
    try {
        return plan_run(plan, sched, n_reads, seed, out_states, out_energies, opts);
    } catch (const std::bad_alloc &) {
        return fail(SA_ENOMEM, "host allocation failed");
    } catch (const std::exception &ex) {
        return fail(SA_EINVAL, ex.what());
    }
}

void sa_plan_destroy(sa_plan *plan) { delete plan; }

int32_t sa_plan_get_info(const sa_plan *plan, sa_plan_info *info) {
    if (!plan || !info) return fail(SA_EINVAL, "plan and info are required");
    *info = plan->info;
    return SA_OK;
}

int32_t sa_plan_last_launch(const sa_plan *plan, sa_launch_info *info) {
    if (!plan || !info) return fail(SA_EINVAL, "plan and info are required");
    *info = plan->last;
    return SA_OK;
}

int32_t sa_anneal_ex(const sa_instance *inst, const sa_bounds *bounds, const sa_schedule *sched,
                     int32_t rule, int32_t n_reads, uint64_t seed, int32_t *out_states,
                     int64_t *out_energies, const sa_opts *opts) {
    g_last_error.clear();
    // argument checks that need no canonical form come first
    if (n_reads < 1) return fail(SA_EINVAL, "n_reads must be >= 1");
    if (!sched || sched->n_sweeps < 1) return fail(SA_EINVAL, "schedule with n_sweeps >= 1 is required");
    if (!out_states || !out_energies) return fail(SA_EINVAL, "output buffers are required");
    if (sched->beta)
        for (int32_t s = 0; s < sched->n_sweeps; ++s)
            if (!(sched->beta[s] >= 0.0) || std::isinf(sched->beta[s]))
                return fail(SA_EINVAL, "beta must be finite and >= 0");
    if (opts) {
        const int32_t s1 = opts->sweep_end <= 0 ? sched->n_sweeps : opts->sweep_end;
        if (opts->sweep_begin < 0 || s1 < opts->sweep_begin || s1 > sched->n_sweeps)
            return fail(SA_EINVAL, "sweep range outside the schedule");
    }
    if (opts && opts->init_states && !opts->device_buffers && inst && bounds && bounds->lower &&
        bounds->upper && inst->n_vars > 0) {
        for (int64_t r = 0; r < n_reads; ++r)
            for (int32_t k = 0; k < inst->n_vars; ++k) {
                int32_t v = opts->init_states[r * inst->n_vars + k];
                if (v < bounds->lower[k] || v > bounds->upper[k])
                    return fail(SA_EINVAL, "init_states outside the bounds");
            }
    }
    sa_plan *plan = nullptr;
    int32_t rc = sa_plan_create(inst, bounds, rule, &plan);
    if (rc != SA_OK) return rc;
    rc = sa_plan_run(plan, sched, n_reads, seed, out_states, out_energies, opts);
    if (rc == SA_OK && opts && opts->device_buffers) {
        // the plan's device memory must outlive the queued kernel
        hipError_t e = hipStreamSynchronize((hipStream_t)opts->hip_stream);
        if (e != hipSuccess) rc = hip_fail(e, "annealing run");
    }
    sa_plan_destroy(plan);
    return rc;
}

int32_t sa_anneal(const sa_instance *inst, const sa_bounds *bounds, const sa_schedule *sched,
                  int32_t rule, int32_t n_reads, uint64_t seed, int32_t *out_states,
                  int64_t *out_energies) {
    return sa_anneal_ex(inst, bounds, sched, rule, n_reads, seed, out_states, out_energies, nullptr);
}

int32_t sa_auto_schedule(const sa_instance *inst, const sa_bounds *bounds, int32_t n_sweeps,
                         double *beta_out) {
    g_last_error.clear();
    if (n_sweeps < 1 || !beta_out) return fail(SA_EINVAL, "n_sweeps >= 1 and beta_out are required");
    try {
        std::string err;
        sa::Canonical canon;
        int rc = sa::canonicalize(inst, bounds, canon, err);
        if (rc != SA_OK) return fail(rc, err);
        double ti = 0, tf = 0;
        rc = sa::auto_temperatures(canon, &ti, &tf, err);
        if (rc != SA_OK) return fail(rc, err);
        sa::geometric_betas(ti, tf, n_sweeps, beta_out);
        return SA_OK;
    } catch (const std::bad_alloc &) {
        return fail(SA_ENOMEM, "host allocation failed");
    }
}

int32_t sa_energy(const sa_instance *inst, const sa_bounds *bounds, int32_t n_states,
                  const int32_t *states, int64_t *out_energies) {
    g_last_error.clear();
    if (n_states < 1 || !states || !out_energies) return fail(SA_EINVAL, "states and outputs are required");
    sa_plan *plan = nullptr;
    int32_t rc = sa_plan_create(inst, bounds, SA_METROPOLIS, &plan);
    if (rc != SA_OK) return rc;
    const int32_t n = plan->dp.n;
    for (int64_t i = 0; i < (int64_t)n_states * n; ++i) {
        int32_t k = (int32_t)(i % n);
        if (states[i] < bounds->lower[k] || states[i] > bounds->upper[k]) {
            sa_plan_destroy(plan);
            return fail(SA_EINVAL, "state outside the bounds");
        }
    }
    const size_t zb = (size_t)n_states * n * sizeof(int32_t), eb = (size_t)n_states * sizeof(int64_t);
    void *tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, align256(zb) + eb);
    if (e != hipSuccess) {
        sa_plan_destroy(plan);
        return fail(SA_ENOMEM, "hipMalloc(energy)");
    }
    int32_t *zd = (int32_t *)tmp;
    int64_t *ed = (int64_t *)((char *)tmp + align256(zb));
    e = hipMemcpy(zd, states, zb, hipMemcpyHostToDevice);
    std::string err;
    if (e == hipSuccess) {
        rc = sa::launch_energy(plan->dp, zd, n_states, ed, nullptr, err);
        if (rc == SA_OK) {
            e = hipMemcpy(out_energies, ed, eb, hipMemcpyDeviceToHost);
            if (e != hipSuccess) rc = hip_fail(e, "energy copy");
        } else {
            fail(rc, err);
        }
    } else {
        rc = hip_fail(e, "hipMemcpy(states)");
    }
    (void)hipFree(tmp);
    sa_plan_destroy(plan);
    return rc;
}

const char *sa_last_error(void) { return g_last_error.c_str(); }

int32_t sa_version(void) { return 100; }

}  // extern "C"
