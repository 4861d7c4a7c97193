// sa_internal.h -- contract between the host packer (sa_host.cpp), the C ABI (sa_api.cpp) and the
// HIP kernels (sa_kernels.hip).  Not installed; include/sa.h is the public interface.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sa.h"

namespace sa {

// Largest exponent of one variable inside one term that the heat-bath and optimal-transition
// kernels accept (their per-variable polynomial dE(v) = sum_m a_m (v^m - z^m) keeps m <= this).
constexpr int kMaxExpPoly = 16;
// Largest exponent stored at all (8-bit field of the incidence record).
constexpr int kMaxExpStored = 255;
// Heat-bath weights kept in registers when ceil(W/64) <= this; wider ranges recompute them.
constexpr int kHeatBathRegChunk = 32;
// Optimal transition: ranges up to this width take the argmin by enumeration, wider ones from the
// sign changes of the energy difference's forward differences (the same value).
constexpr int kOtmEnumMax = 2048;

// Canonical polynomial: merged terms, nonzero coefficients, factors sorted (a power is a
// repeated index).
struct Canonical {
    int32_t n = 0;
    std::vector<int64_t> t_off;   // n_terms + 1 offsets into t_var
    std::vector<int32_t> t_var;   // factor indices, ascending inside a term
    std::vector<int64_t> t_coef;  // nonzero coefficients
    std::vector<int32_t> lo, hi;  // integer box
    int64_t n_terms() const { return (int64_t)t_coef.size(); }
};

// Validates and canonicalises; returns an SA_* status and fills err on failure.
int canonicalize(const sa_instance *inst, const sa_bounds *bounds, Canonical &out, std::string &err);
// SA_ERANGE when sum_t |J_t| prod zmax^e >= 2^62.  Also reports the largest |dE| bound.
int check_int64_bound(const Canonical &c, std::string &err, double *bound_out);
// True when max_k sum_{t containing k} |J_t| prod_{factors} zmax^e < 2^29, so every energy
// difference |dE| < 2^30 and the difference of two of them fit 32-bit signed arithmetic.
bool dE_fits_32(const Canonical &c);
// every coefficient a_k^(m) (and each incidence record's product) below 2^31 in magnitude
bool coefs_fit_32(const Canonical &c);
// Sec. 3.4 temperature range (T_init, T_final); SA_EINVAL if the problem has no energy scale.
int auto_temperatures(const Canonical &c, double *t_init, double *t_final, std::string &err);
// Geometric cooling of Sec. 3.1 between the two temperatures, as inverse temperatures.
void geometric_betas(double t_init, double t_final, int32_t n_sweeps, double *beta_out);

// Variable record: {lower bound, width W = u - l + 1, first incidence, number of incidences}.
struct VarRec {
    int32_t lo, width, row, deg;
};
// Incidence record of variable k in term t: meta = e_k(t) | (n_other << 8); the other factors
// (indices repeated by exponent) inline in o[0..2] when n_other <= 3, else o[0] is the offset of
// n_other indices in the overflow array (a multiple of four; the list is padded with -1 to a
// multiple of four entries).
struct IncRec {
    uint32_t meta;
    int32_t o[3];
};

// Compact incidence record of a pair term J z_k z_j (index of the other factor j, coefficient J).
struct PairRec {
    int32_t j;
    int32_t J;
};
// a variable's pair records are padded with zero records to a multiple of this many
constexpr int32_t kPairBlock = 16;

// Host-side packed image of a plan (uploaded as one device allocation).
struct Packed {
    int32_t n = 0;
    int32_t n_terms = 0;
    std::vector<VarRec> var;
    std::vector<uint32_t> emask;    // bit m set: some term holds z_k^m (m = 1..31; 31 = ">= 31")
    std::vector<IncRec> inc;
    std::vector<int64_t> inc_coef;
    std::vector<int32_t> overflow;  // other-factor indices of incidences with > 3 others
    int32_t max_other = 0;          // most other factors of any incidence (1: pair terms only)
    std::vector<int32_t> t_off;     // term-major copy for energies
    std::vector<int32_t> t_var;
    std::vector<int64_t> t_coef;
    int32_t max_exp = 0;
    int32_t max_width = 1;
    // dense QUIO form (no incidence records): E = sum_k h_k z_k + d_k z_k^2 + sum_{j<k} J_kj z_j z_k
    // with J stored as a symmetric n x row_stride matrix (zero diagonal and padding)
    bool dense = false;
    int32_t jbytes = 0;             // 1 (int8) or 4 (int32)
    int32_t row_stride = 0;         // elements per matrix row (multiple of 16)
    std::vector<int8_t> jd8;
    std::vector<int32_t> jd32;
    std::vector<int64_t> h, d;
    int64_t n_pairs = 0;
    // compact form of a multilinear QUIO whose coefficients fit int32 (empty otherwise): per
    // variable its pair records (row pair_row[k], pair_deg[k] of them, followed by zero records
    // {0, 0} up to a multiple of kPairBlock) and its linear coefficient
    std::vector<PairRec> pair;
    std::vector<int32_t> pair_row, pair_deg, pair_h;
};
int pack(const Canonical &c, Packed &out, std::string &err);
int maxe_class_of(int32_t max_exp);

// One slot of the sweep schedule: in window w, wave g of a replica updates variable k (k = -1:
// the wave idles in that window).  Variables of one window share no term, so their updates
// commute and may run at the same time; windows follow the index order of the sweep (Sec. 3.1)
// and fixed variables (l = u) are left out.
struct SchedRec {
    int32_t k;
    int32_t lo, width, row, deg;
    uint32_t emask;
    int32_t pad[2];
};
// Greedy windows of at most G mutually non-interacting variables, stored wave-major
// (slot g * n_win + w).  Returns the number of windows.
int32_t build_schedule(const Packed &p, int G, std::vector<SchedRec> &out);

// Dependency levels of one sweep: a level holds, in index order, variables (not fixed) none of
// which shares a term with another, each placed after all of its lower-index neighbours' levels.
// Updating the levels one after another, the variables of a level in any order or at once, reads
// every neighbour exactly as the sequential index-order sweep does: a lower-index neighbour
// already updated in this sweep, a higher-index one not yet.  The number of levels is the
// longest chain of neighbours in index order; each variable goes to a level between its earliest
// and its latest, and levels are filled up to whole rounds of `quads` updates where the slack
// allows.  Returns the number of levels; slots are level-major, level_start has one more entry.
int32_t build_levels(const Packed &p, int32_t quads, std::vector<int32_t> &level_start,
                     std::vector<SchedRec> &slots);
// Rounds of the one-wave quad kernel: the levels of 16 (one wavefront of quads), each cut into
// rounds of 16 slots and padded to whole rounds with idle slots (k = -1, no records), and the sweep
// padded with idle rounds to a multiple of kRoundBatch rounds.  Every slot points at its
// variable's incidence records.  Returns the number of levels; n_real counts the variables placed.
constexpr int32_t kRoundQuads = 16;
constexpr int32_t kRoundBatch = 4;
int32_t build_rounds(const Packed &p, std::vector<SchedRec> &rounds, int32_t &n_real);
// Records per lane that the Metropolis / OTM quad kernel reads for one round (a row of up to
// 4 kMoAhead incidences; longer rows take the rest from the incidence records).
constexpr int32_t kMoAhead = 16;
// A round's record as that kernel reads it: meta as in IncRec, and the LDS byte offsets of the
// other factors' values -- 4 n (the state's element n, which holds 1) for an unused place.
struct MoRec {
    uint32_t meta;
    uint32_t zoff[3];
};
// Round-major copy of the rounds' records: record u of lane L (quad L / 4, its record 4 u + L % 4)
// of round r at ((r kMoAhead + u) 64 + L), with zero coefficients past a row and for records with
// more than three other factors (coefficients as int32 when coef32, else int64).  Marks in
// pad[0] of a round's slot whether its row needs the rest read from the incidence records (more
// than 4 kMoAhead records, or a long record).
void build_mo_records(const Packed &p, std::vector<SchedRec> &rounds, bool coef32, std::vector<MoRec> &rec,
                      std::vector<uint8_t> &coef);

// Device view of a packed plan.
struct DevProblem {
    int32_t n;
    int32_t n_terms;
    const VarRec *var;
    const uint32_t *emask;
    const IncRec *inc;       // incidence records, then one zero record at index inc_pad
    const int64_t *inc_coef;
    const int32_t *overflow;
    const int32_t *t_off;
    const int32_t *t_var;
    const int64_t *t_coef;
    int32_t max_other;       // most other factors of any incidence
    int32_t inc_pad;         // index of the zero record (coefficient 0, no factors)
    int32_t coef32;          // every coefficient a_k^(m) fits int32 (coefs_fit_32)
    // dense QUIO form (dense != 0)
    int32_t dense;
    int32_t jbytes;
    int32_t row_stride;
    const void *jd;
    const int64_t *h;
    const int64_t *d;
    const PairRec *pair;     // compact pair records (nullptr when the problem has none)
};

// Kernel arguments of one annealing launch.
struct AnnealArgs {
    DevProblem P;
    const double *beta;      // S inverse temperatures (device)
    int32_t n_sweeps;        // S
    int32_t s_begin, s_end;  // sweeps to run
    int32_t n_reads;
    int32_t waves_per_group;
    uint32_t key0, key1;     // Philox key (seed)
    uint32_t instance_id;
    double otm_r;            // < 0: r = s/(S-1)
    int32_t otm_enum_max;    // widest range whose optimal transition is found by enumeration
    const SchedRec *sched;   // G * n_win schedule slots (device)
    int32_t n_win;           // windows per sweep
    int32_t win_waves;       // G: waves per replica (1: each wave is an independent replica)
    const int32_t *z_init;   // device, n_reads * n, or nullptr
    int32_t *z_out;          // device, n_reads * n (also the working state when not in LDS)
    int64_t *e_out;          // device, n_reads
    int32_t dense_cache;     // 1: dense form with one wave per replica and the state in LDS keeps the
                             // coefficient cache c1 (int64 per variable) in LDS after the states
    uint64_t *trace;         // device, n_reads * (s_end - s_begin) zeroed words, or nullptr: each
                             // wave adds its share of the state hash's change per sweep (and of the
                             // initial state's hash into the first sweep); a prefix pass then turns
                             // them into the hash after every sweep
};

// Kernel arguments of one launch of the quad kernel (one update per four lanes, dependency levels).
struct QuadArgs {
    DevProblem P;
    const double *beta;          // S inverse temperatures (device)
    int32_t n_sweeps;
    int32_t s_begin, s_end;
    int32_t n_reads;
    uint32_t key0, key1;
    uint32_t instance_id;
    const int32_t *level_start;  // n_levels + 1 offsets into slots (device)
    const SchedRec *slots;       // level-major variables, or n_rounds rounds of kRoundQuads (device)
    int32_t n_levels;
    int32_t n_rounds;            // Metropolis / optimal transition: rounds per sweep (build_rounds)
    const MoRec *mrec;           // Metropolis / optimal transition: the rounds' records (build_mo_records)
    const void *mcoef;           // and their coefficients (int32 when P.coef32, else int64)
    int32_t uniform_width;       // the common width W of every slot, or 0 when widths differ
    double otm_r;                // < 0: r = s/(S-1); else a fixed r (optimal transition)
    const int32_t *z_init;
    int32_t *z_out;
    int64_t *e_out;
    uint64_t *trace;             // as AnnealArgs::trace
};
// Waves of the quad kernel's workgroup (one replica): heat bath, 8 or 16 (below), and Metropolis /
// optimal transition, one (a HUIO level holds about 16 variables, and a single wave needs no
// barrier between levels); the most values per lane it keeps in registers.
constexpr int kQuadWaves = 8;
constexpr int kQuadWavesHigh = 16;
constexpr int kQuadWavesMO = 1;
constexpr int kQuadMaxR = 32;
// Values per lane of the quad heat bath: the smallest class of 8, 16, 26, 32 holding ceil(W / 4)
// (W = 101 takes 26: 104 places).
constexpr int32_t quad_r_class(int32_t max_width) {
    const int32_t c = (max_width + 3) / 4;
    return c <= 8 ? 8 : c <= 16 ? 16 : c <= 26 ? 26 : kQuadMaxR;
}
// The factored weights of linear variables (sa_quad.h): heat bath, one width W for every variable,
// r >= 16 values per lane and at most r / 4 of the quad's 4 r places past the range.
constexpr bool quad_factored(int rule, int32_t r, int32_t uniform_width) {
    return rule == SA_HEAT_BATH && r >= 16 && uniform_width > 0 && 4 * r - uniform_width >= 0 &&
           4 * r - uniform_width <= r / 4;
}
// The heat-bath variants that hold at most 128 VGPRs, so that a workgroup of 16 waves (four per
// SIMD, rounds of 256 updates) fits without spilling: they run 16 waves, the others 8.
constexpr bool quad_high(int rule, int32_t r, int32_t max_exp, bool fact) {
    return rule == SA_HEAT_BATH_CLOSED ? (max_exp <= 1 || r == 8)
                                       : (r == 8 || (fact && (max_exp <= 1 ? r <= 26 : r == 16)));
}
// Waves per replica of the quad kernel for a problem whose widest range is max_width, whose
// exponents are at most max_exp and whose variables all have width uniform_width (0: not one width).
constexpr int quad_waves(int rule, int32_t max_width, int32_t max_exp, int32_t uniform_width) {
    if (rule == SA_METROPOLIS || rule == SA_OPT_METROPOLIS) return kQuadWavesMO;
    const int32_t r = quad_r_class(max_width);
    return quad_high(rule, r, max_exp, quad_factored(rule, r, uniform_width)) ? kQuadWavesHigh : kQuadWaves;
}
// The common width of the variables that are not fixed, or 0 when they differ (or there are none).
int32_t quad_uniform_width(const Packed &p);
// Launches the quad kernel for rule (SA_HEAT_BATH or SA_HEAT_BATH_CLOSED), a problem whose widest
// range is max_width <= 4 * kQuadMaxR and whose exponents are <= max_exp <= 2 (defined in
// sa_kernels_quad.hip).
int launch_quad(int rule, const QuadArgs &a, int32_t max_width, int32_t max_exp, bool narrow, void *stream,
                std::string &err);
// The same for SA_METROPOLIS and SA_OPT_METROPOLIS, exponents <= max_exp <= 4, kQuadWavesMO waves
// (defined in sa_kernels_quad_mo.hip).
int launch_quad_mo(int rule, const QuadArgs &a, int32_t max_width, int32_t max_exp, bool narrow, void *stream,
                   std::string &err);

struct LaunchChoice {
    int win_waves = 1;         // waves per replica (window width)
    int waves_per_group = 1;
    int groups = 1;
    int lds_bytes = 0;
    bool state_in_lds = true;
    int reg_chunk = 0;         // heat bath: weights per lane kept in registers (0: recomputed)
    int maxe_class = 1;        // kernel's largest exponent (1, 2, 4 or 16)
    bool narrow = false;       // energy differences in 32-bit arithmetic
    bool dense_cache = false;  // dense form: coefficient cache in LDS (one wave per replica)
    int variant = 0;
};

// Byte layout of a packed instance in one device area, each part 256-byte aligned (the records
// and their coefficients are followed by one zero record).
struct PackedLayout {
    static constexpr int kParts = 12;
    size_t off[kParts];
    size_t total;
};
PackedLayout packed_layout(const Packed &pk);
// Writes the packed instance into a host image of L.total bytes (padding zeroed).
void stage_packed(const Packed &pk, const PackedLayout &L, char *image);
// Points d at the parts of an image copied to device address base.
void bind_packed(const Packed &pk, const PackedLayout &L, char *base, DevProblem &d);

// Launches one annealing pass (defined in sa_kernels.hip).  Returns an SA_* status.
int launch_anneal(int rule, const AnnealArgs &a, const LaunchChoice &lc, void *stream,
                  std::string &err);
// Picks the launch geometry for n_reads replicas of an n-variable problem on `device`.
LaunchChoice choose_launch(int rule, int32_t n, int32_t n_reads, int32_t max_width, int32_t max_exp,
                           int device, int win_waves, bool narrow_ok, int32_t otm_enum_max, bool dense);
// LDS bytes of one replica's state when its G waves share it (state + per-wave energy slots).
int64_t shared_state_bytes(int32_t n, int G);
// Waves of one batch workgroup; a task runs kBatchWaves / G_p reads of problem p.
constexpr int kBatchWaves = 8;

// One problem of a batch as the persistent kernel sees it.
struct BatchInst {
    DevProblem P;
    const double *beta;      // S inverse temperatures (device)
    const SchedRec *sched;   // schedule for `team` waves per replica
    int32_t n_win;
    int32_t team;            // G_p: waves per replica (1, 2, 4 or 8)
    int32_t slot_stride;     // state elements between the teams' LDS slots
    int32_t n_reads;
    int32_t n_sweeps;
    int32_t s_begin, s_end;  // sweeps of this launch (a server chunk, or the whole schedule)
    int32_t resume;          // 1: start from the states in z_out and energies in e_out (an earlier chunk's)
    int32_t rule;
    int32_t chunk;           // heat bath: register chunk class (1, 2, 8; 0 = recompute)
    uint32_t key0, key1, instance_id;
    int32_t *z_out;          // n_reads x n (device)
    int64_t *e_out;          // n_reads (device)
};
struct BatchTask {
    int32_t inst;
    int32_t read;            // first read of the task (kBatchWaves / G_p reads)
};
struct BatchArgs {
    const BatchInst *insts;
    const BatchTask *tasks;  // ordered longest first
    int32_t n_tasks;
    uint32_t *counter;       // next task (device)
    int32_t lds_words;       // dynamic LDS of a workgroup, 32-bit words
    int32_t parts_words;     // offset of the waves' energy parts (kBatchWaves int64)
    int32_t sweep_limit;     // > 0: only the first sweep_limit sweeps (autotuning trials)
};
struct BatchLaunch {
    int waves_per_group = kBatchWaves;
    int groups = 1;
    int maxe_class = 1;
    bool narrow = false;
    bool z16 = false;        // states held as int16 in LDS (every bound within int16)
};
// Queues the counter reset and the persistent kernel (both plain kernel launches).
int launch_batch(const BatchArgs &b, const BatchLaunch &bl, void *stream, std::string &err);

// Zeroes n words of device memory with a kernel (no memset node, so the work may be captured).
int launch_zero_u64(uint64_t *p, int64_t n, void *stream, std::string &err);
// Turns per-sweep hash changes into the hash after each sweep: row r of `trace` (n_reads rows of
// n_cols) becomes its own inclusive prefix sum.
int launch_trace_prefix(uint64_t *trace, int32_t n_reads, int32_t n_cols, void *stream, std::string &err);

// Energies of n_states device-resident states (one wavefront per state).
int launch_energy(const DevProblem &P, const int32_t *states, int32_t n_states, int64_t *out,
                  void *stream, std::string &err);

}  // namespace sa
