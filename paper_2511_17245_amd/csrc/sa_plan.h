// sa_plan.h -- the plan object shared by the C ABI's one-shot, batched and served paths.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "sa_internal.h"

namespace sa {

// One device allocation holding several arrays, each 256-byte aligned.
struct DevArena {
    void *base = nullptr;
    size_t bytes = 0;
    DevArena() = default;
    DevArena(const DevArena &) = delete;
    DevArena &operator=(const DevArena &) = delete;
    ~DevArena() {
        if (base) (void)hipFree(base);
    }
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace sa

struct sa_plan {
    int device = 0;
    int rule = 0;
    sa::DevProblem dp{};
    sa::DevArena arena;
    sa_plan_info info{};
    sa_launch_info last{};
    std::vector<int32_t> lo, hi;  // host copy of the box (checks of host start states)
    bool narrow_ok = false;       // every |dE| < 2^30: 32-bit integer kernels are exact
    double t_init = 0.0, t_final = 0.0;
    int auto_status = SA_OK;
    std::string auto_error;
    // device copy of the last schedule, reused while the schedule is unchanged
    double *beta_dev = nullptr;
    int32_t beta_cap = 0;
    std::vector<double> beta_host;
    // host packing (kept to build sweep schedules) and the device schedules built so far, by G
    sa::Packed packed;
    struct Sched {
        sa::SchedRec *dev = nullptr;
        int32_t n_win = 0;
        int32_t n_active = 0;  // variables that are not fixed
    };
    Sched sched[17];  // index G = 1, 2, 4, 8, 16
    // dependency levels of the sweep (the quad kernel), built on first use
    struct Levels {
        void *dev = nullptr;          // level_start (n_levels + 1 int32) then the slots, or the rounds
        const int32_t *start = nullptr;
        const sa::SchedRec *slots = nullptr;
        int32_t n_levels = -1;        // -1: not built
        int32_t n_slots = 0;          // variables placed (idle slots of the rounds not counted)
        int32_t n_rounds = 0;         // Metropolis / optimal transition: rounds of kRoundQuads slots
        const sa::MoRec *mrec = nullptr;   // and their records' round-major copy (build_mo_records)
        const void *mcoef = nullptr;
        int32_t uniform_width = 0;    // common width of every slot, 0 when they differ
    };
    Levels levels;
    std::mutex sched_mu;  // guards the lazy building of sched and levels (a server's preparers share plans)
    ~sa_plan() {
        if (beta_dev) (void)hipFree(beta_dev);
        for (auto &sc : sched)
            if (sc.dev) (void)hipFree(sc.dev);
        if (levels.dev) (void)hipFree(levels.dev);
    }
};


namespace sa {

// Records msg as this thread's last error and returns code.
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
// Clears this thread's last error (at the start of an entry point).
void clear_error();
// Canonicalise, check, pack and upload; *out owns the result.
int build_plan(const sa_instance *inst, const sa_bounds *bounds, int32_t rule, sa_plan **out);
// Inverse temperatures of a schedule (explicit or automatic) for the plan's instance.
int resolve_schedule(sa_plan *plan, const sa_schedule *sched, std::vector<double> &beta);
// The plan's sweep schedule for G waves per replica (built on first use, kept on the device).
int get_schedule(sa_plan *plan, int G, sa_plan::Sched **out);
// Uploads the inverse temperatures unless the device already holds the same array.
int stage_beta(sa_plan *plan, const std::vector<double> &beta, hipStream_t stream);
// Heat-bath register chunk class of a plan's widest range (1, 2, 8, 32, or 0 = recompute).
int reg_chunk_class(int32_t max_width);
// The plan's dependency levels (built and uploaded on first use).
int get_levels(sa_plan *plan, sa_plan::Levels **out);
// The common width of the level slots, or 0 when widths differ.
int32_t uniform_width(const std::vector<SchedRec> &slots);
// Whether the quad kernel can run `rule` on this packed problem with n replicas' state in LDS.
bool quad_eligible(int rule, const Packed &pk, int device);
// Lanes per update (64 or 4) for a run: `requested` (0 = automatic) checked against eligibility;
// the automatic choice takes the quad kernel when its levels fill half of a workgroup's `quads`
// on average (64 or 128 variables for the heat bath's 128 or 256 quads, 8 for the 16 quads of
// Metropolis and the optimal transition).
// Returns -1 (with the error recorded) for a request the problem cannot take.
int choose_lanes(int32_t quads, int requested, int waves_per_replica, bool eligible, int32_t n_levels,
                 int32_t n_slots);
// SA_EUNSUPPORTED / SA_EINVAL (with the message recorded) when the GPU kernels cannot run `rule`
// on a problem whose largest exponent is max_exp.
int check_rule_support(int rule, int32_t max_exp);
// Automatic waves per replica; windows(G, n_win, n_active) reports the window count of a G-wide
// schedule and the number of variables that are not fixed (false: no such schedule).
int pick_waves_per_replica(int32_t n, int32_t n_reads, int device,
                           const std::function<bool(int, int32_t &, int32_t &)> &windows);

}  // namespace sa
