// sa_noalloc.hip -- sa_anneal_noalloc: the run of sa_anneal_ex with device outputs for callers that
// cannot allocate device memory.  What the kernels read beyond the caller's inputs and outputs --
// the packed instance, the inverse temperatures and the sweep schedule, which sa_anneal_ex puts in
// allocations of its own -- is staged in one static device array per GPU.  The host does the same
// canonicalisation, checks, packing and launch choice as sa_anneal_ex, so the results are the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sa_plan.h"

namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;

// The staging area.  Its name is a host-side stand-in: host code uses only the address that
// hipGetSymbolAddress returns for the current device (scratch_address below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// The device address of this GPU's staging area, looked up once per device (the device current).
int scratch_address(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return sa::fail(SA_EDEVICE, "device index above 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return sa::hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return SA_OK;
}

int run_noalloc(const sa_instance *inst, const sa_bounds *bounds, const sa_schedule *sched, int32_t rule,
                int32_t n_reads, uint64_t seed, int32_t *out_states, int64_t *out_energies,
                const sa_opts *opts_in) {
    sa_opts opts;
    sa_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    if (!opts_in || !opts.device_buffers)
        return sa::fail(SA_EINVAL, "sa_anneal_noalloc needs device_buffers = 1 (outputs in device memory)");
    if (n_reads < 1) return sa::fail(SA_EINVAL, "n_reads must be >= 1");
    if (!sched || sched->n_sweeps < 1) return sa::fail(SA_EINVAL, "schedule with n_sweeps >= 1 is required");
    if (!out_states || !out_energies) return sa::fail(SA_EINVAL, "output buffers are required");
    const int32_t S = sched->n_sweeps;
    const int32_t s0 = opts.sweep_begin;
    const int32_t s1 = opts.sweep_end <= 0 ? S : opts.sweep_end;
    if (s0 < 0 || s1 < s0 || s1 > S) return sa::fail(SA_EINVAL, "sweep range outside the schedule");
    if (opts.otm_enum_max < 0) return sa::fail(SA_EINVAL, "otm_enum_max must be >= 0");
    int G = opts.waves_per_replica;
    if (G != 0 && G != 1 && G != 2 && G != 4 && G != 8 && G != 16)
        return sa::fail(SA_EINVAL, "waves_per_replica must be 0, 1, 2, 4, 8 or 16");

    // host side: as sa_plan_create + sa_plan_run
    std::string err;
    sa::Canonical canon;
    int rc = sa::canonicalize(inst, bounds, canon, err);
    if (rc != SA_OK) return sa::fail(rc, err);
    double bound = 0.0;
    rc = sa::check_int64_bound(canon, err, &bound);
    if (rc != SA_OK) return sa::fail(rc, err);
    sa::Packed pk;
    rc = sa::pack(canon, pk, err);
    if (rc != SA_OK) return sa::fail(rc, err);
    rc = sa::check_rule_support(rule, pk.max_exp);
    if (rc != SA_OK) return rc;
    std::vector<double> beta((size_t)S);
    if (sched->beta) {
        for (int32_t s = 0; s < S; ++s) {
            const double b = sched->beta[s];
            if (!(b >= 0.0) || std::isinf(b)) return sa::fail(SA_EINVAL, "beta must be finite and >= 0");
            beta[(size_t)s] = b;
        }
    } else {
        double ti = 0.0, tf = 0.0;
        rc = sa::auto_temperatures(canon, &ti, &tf, err);
        if (rc != SA_OK) return sa::fail(rc, err);
        sa::geometric_betas(ti, tf, S, beta.data());
    }
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return sa::hip_fail(e, "hipGetDevice");
    void *area = nullptr;
    rc = scratch_address(device, &area);
    if (rc != SA_OK) return rc;

    // lanes per update, as sa_anneal_ex chooses them
    const bool eligible = sa::quad_eligible(rule, pk, device);
    // the levels (heat bath) or the rounds (Metropolis, optimal transition) of the quad kernel
    const bool mo = rule == SA_METROPOLIS || rule == SA_OPT_METROPOLIS;
    const int qwaves = sa::quad_waves(rule, pk.max_width, pk.max_exp, sa::quad_uniform_width(pk));
    std::vector<int32_t> lv_start;
    std::vector<sa::SchedRec> lv_slots;
    int32_t n_levels = 0, n_real = 0;
    if (eligible && G == 0 && opts.lanes_per_update != 64) {
        n_levels = mo ? sa::build_rounds(pk, lv_slots, n_real) : sa::build_levels(pk, qwaves * 16, lv_start, lv_slots);
        if (!mo) n_real = (int32_t)lv_slots.size();
    }
    int lanes = sa::choose_lanes(qwaves * 16, opts.lanes_per_update, G, eligible, n_levels, n_real);
    if (lanes < 0) return SA_EINVAL;
    if (lanes == 4 && mo && opts.lanes_per_update == 0) {
        // the rounds' record copy takes 64 kMoAhead records per round; when the image would not fit
        // the static area, the automatic choice takes the windows instead (the same results)
        const size_t cw = sa::coefs_fit_32(canon) ? 4 : 8;
        const size_t need = sa::packed_layout(pk).total + sa::align256(sizeof(double) * (size_t)S) +
                            sa::align256(lv_slots.size() * sizeof(sa::SchedRec)) +
                            (lv_slots.size() / (size_t)sa::kRoundQuads) * (size_t)sa::kMoAhead * 64 *
                                (sizeof(sa::MoRec) + cw) + 1024;
        if (need > kScratchBytes) lanes = 64;
    }
    std::vector<sa::MoRec> mrec;
    std::vector<uint8_t> mcoef;
    if (lanes == 4 && mo) sa::build_mo_records(pk, lv_slots, sa::coefs_fit_32(canon), mrec, mcoef);

    int32_t active = 0;
    for (const auto &vr : pk.var) active += vr.width > 1 ? 1 : 0;
    if (lanes == 64 && G == 0)
        G = sa::pick_waves_per_replica(pk.n, n_reads, device, [&](int g, int32_t &n_win, int32_t &n_act) {
            std::vector<sa::SchedRec> tmp;
            n_win = sa::build_schedule(pk, g, tmp);
            n_act = active;
            return true;
        });
    const int32_t enum_max = opts.otm_enum_max > 0 ? opts.otm_enum_max : sa::kOtmEnumMax;
    const sa::LaunchChoice lc = sa::choose_launch(rule, pk.n, n_reads, pk.max_width, pk.max_exp, device, G,
                                                  sa::dE_fits_32(canon), enum_max, pk.dense);
    std::vector<sa::SchedRec> sch;
    const int32_t n_win = lanes == 64 ? sa::build_schedule(pk, lc.win_waves, sch) : 0;

    // one image: packed instance | inverse temperatures | schedule (windows, or level offsets then
    // level slots)
    const sa::PackedLayout L = sa::packed_layout(pk);
    const size_t off_beta = L.total;
    const size_t off_sched = off_beta + sa::align256(sizeof(double) * (size_t)S);
    const size_t off_slots = off_sched + sa::align256(lv_start.size() * sizeof(int32_t));
    const size_t off_mrec = off_slots + sa::align256(std::max<size_t>(lv_slots.size(), 1) * sizeof(sa::SchedRec));
    const size_t off_mcoef = off_mrec + sa::align256(mrec.size() * sizeof(sa::MoRec));
    const size_t total = lanes == 64
                             ? off_sched + sa::align256(std::max<size_t>(sch.size(), 1) * sizeof(sa::SchedRec))
                             : off_mcoef + sa::align256(std::max<size_t>(mcoef.size(), 1));
    if (total > kScratchBytes)
        return sa::fail(SA_ENOMEM, "sa_anneal_noalloc: the problem needs " + std::to_string(total) +
                                       " bytes of staging; the static area holds " +
                                       std::to_string(kScratchBytes));
    std::vector<char> image(total, 0);
    sa::stage_packed(pk, L, image.data());
    std::memcpy(image.data() + off_beta, beta.data(), sizeof(double) * (size_t)S);
    // only the schedule the chosen kernel reads: the levels are built whenever the quad kernel is
    // eligible, also when the choice falls on the windows, and share their offset
    if (lanes == 64) {
        if (!sch.empty()) std::memcpy(image.data() + off_sched, sch.data(), sch.size() * sizeof(sa::SchedRec));
    } else {
        if (!lv_start.empty())
            std::memcpy(image.data() + off_sched, lv_start.data(), lv_start.size() * sizeof(int32_t));
        if (!lv_slots.empty())
            std::memcpy(image.data() + off_slots, lv_slots.data(), lv_slots.size() * sizeof(sa::SchedRec));
        if (!mrec.empty()) std::memcpy(image.data() + off_mrec, mrec.data(), mrec.size() * sizeof(sa::MoRec));
        if (!mcoef.empty()) std::memcpy(image.data() + off_mcoef, mcoef.data(), mcoef.size());
    }
    hipStream_t stream = (hipStream_t)opts.hip_stream;
    e = hipMemcpyAsync(area, image.data(), total, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);   // the host image is freed on return
    if (e != hipSuccess) return sa::hip_fail(e, "staging copy");

    sa::AnnealArgs a{};
    sa::bind_packed(pk, L, (char *)area, a.P);
    a.P.coef32 = sa::coefs_fit_32(canon) ? 1 : 0;
    a.beta = (const double *)((char *)area + off_beta);
    a.n_sweeps = S;
    a.s_begin = s0;
    a.s_end = s1;
    a.n_reads = n_reads;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.instance_id = opts.instance_id;
    a.otm_r = opts.otm_r;
    a.otm_enum_max = enum_max;
    a.z_init = opts.init_states;
    a.z_out = out_states;
    a.e_out = out_energies;
    a.trace = opts.trace_hashes;
    a.sched = (const sa::SchedRec *)((char *)area + off_sched);
    a.n_win = n_win;
    a.win_waves = lc.win_waves;
    a.waves_per_group = lc.waves_per_group;
    a.dense_cache = lc.dense_cache ? 1 : 0;
    if (a.trace) {
        rc = sa::launch_zero_u64(a.trace, (int64_t)n_reads * (s1 - s0), stream, err);
        if (rc != SA_OK) return sa::fail(rc, err);
    }
    if (lanes == 4) {
        sa::QuadArgs q{};
        q.P = a.P;
        q.beta = a.beta;
        q.n_sweeps = S;
        q.s_begin = s0;
        q.s_end = s1;
        q.n_reads = n_reads;
        q.key0 = a.key0;
        q.key1 = a.key1;
        q.instance_id = a.instance_id;
        q.level_start = (const int32_t *)((char *)area + off_sched);
        q.slots = (const sa::SchedRec *)((char *)area + off_slots);
        q.n_levels = n_levels;
        q.n_rounds = mo ? (int32_t)(lv_slots.size() / sa::kRoundQuads) : 0;
        q.mrec = mo ? (const sa::MoRec *)((char *)area + off_mrec) : nullptr;
        q.mcoef = mo ? (const void *)((char *)area + off_mcoef) : nullptr;
        q.uniform_width = mo ? 0 : sa::uniform_width(lv_slots);
        q.otm_r = a.otm_r;
        q.z_init = a.z_init;
        q.z_out = a.z_out;
        q.e_out = a.e_out;
        q.trace = a.trace;
        rc = (mo ? sa::launch_quad_mo : sa::launch_quad)(rule, q, pk.max_width, pk.max_exp, sa::dE_fits_32(canon),
                                                         stream, err);
    } else {
        rc = sa::launch_anneal(rule, a, lc, stream, err);
    }
    if (rc == SA_OK && a.trace) rc = sa::launch_trace_prefix(a.trace, n_reads, s1 - s0, stream, err);
    if (rc != SA_OK) return sa::fail(rc, err);
    return SA_OK;
}

}  // namespace

extern "C" int32_t sa_anneal_noalloc(const sa_instance *inst, const sa_bounds *bounds,
                                     const sa_schedule *sched, int32_t rule, int32_t n_reads, uint64_t seed,
                                     int32_t *out_states, int64_t *out_energies, const sa_opts *opts) {
    sa::clear_error();
    try {
        return run_noalloc(inst, bounds, sched, rule, n_reads, seed, out_states, out_energies, opts);
    } catch (const std::bad_alloc &) {
        return sa::fail(SA_ENOMEM, "host allocation failed");
    } catch (const std::exception &ex) {
        return sa::fail(SA_EINVAL, ex.what());
    }
}
