// sa_quad_mo.h -- Metropolis and the optimal transition with one update per four lanes and one
// wavefront per replica, over the rounds of build_rounds (Sec. 3.2 sweeps, Sec. 3.3.1 and 3.3.3
// rules).
//
// A replica's wavefront holds 16 quads.  A round updates up to 16 mutually independent variables
// of one dependency level; the rounds of a sweep follow one another in the order the levels
// prescribe, so every variable reads its neighbours as the sequential index-order sweep does.
// One wavefront per replica is all the parallelism a HUIO sweep of 2000 variables offers 1024
// replicas, so there is one wave per SIMD and nothing else to hide memory latency behind: the
// kernel does it itself.  Each round issues the loads of the next round's records (16 per lane:
// rows of up to 64 records) before it works on its own, and every second round reloads the
// schedule slots of the next batch of four rounds, so a round waits only on LDS.  The records
// come from a round-major copy (build_mo_records) whose places are addressed by the round index
// alone and hold the other factors as LDS byte offsets, an unused one pointing at the constant 1
// kept after the state: a record's product is three multiplies, with no index arithmetic or
// selects.  The records hold no state; only their other factors' values, read from LDS in the
// round that uses them, do.
//
// Random words: lane q of a quad draws Philox for round q of the batch (the counter of the
// variable of that round); the quad reads them from lane q in round q.  x0 chooses the branch of
// the optimal transition, x1 the Metropolis proposal, (x2, x3) the acceptance uniform -- the same
// words, for the same counters, as the one-wavefront kernel.
#pragma once
#include <type_traits>

#include "sa_quad.h"

namespace sa {
namespace {

// s_waitcnt operand (gfx9 encoding): vmcnt 0, expcnt and lgkmcnt at their maxima (no wait)
constexpr int kWaitVmcnt0 = 0x0F70;

// One round's records for this lane (the round-major copy of build_mo_records): record u holds the
// quad's incidence 4 u + ql, or a zero record past the row.  kNarrow: every coefficient fits 32
// bits and the copy holds them as int32.
template <bool kNarrow>
struct RoundRecs {
    uint4 r[kMoAhead];   // meta, then the LDS byte offsets of the three other factors
    std::conditional_t<kNarrow, uint32_t, uint64_t> c[kMoAhead];
};

// A round's records sit at one offset from the copy's base per lane (record u a further u * 64
// records on), so the loads take no per-record arithmetic; every load is issued, so that the count
// of loads in flight is the same in every round (the waits the compiler places for the current
// round then leave the next round's loads in flight).
template <bool kNarrow>
__device__ __forceinline__ void load_round(const QuadArgs &A, int32_t r, int lane, RoundRecs<kNarrow> &R) {
    using Coef = std::conditional_t<kNarrow, uint32_t, uint64_t>;
    const size_t base = (size_t)r * kMoAhead * 64 + (size_t)lane;
    const uint4 *rec = (const uint4 *)A.mrec + base;
    const Coef *coef = (const Coef *)A.mcoef + base;
#pragma unroll
    for (int u = 0; u < kMoAhead; ++u) {
        R.r[u] = rec[u * 64];
        R.c[u] = coef[u * 64];
    }
}

// The LDS reads of group g (records 4g .. 4g + 3) of this lane: the other factors' values, 1 for
// an unused place (the state's element n).
template <bool kNarrow>
__device__ __forceinline__ void read_group(const int32_t *z, const RoundRecs<kNarrow> &R, int g,
                                           int32_t (&zv)[4][3]) {
    const char *zb = (const char *)z;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint4 &r = R.r[4 * g + u];
        zv[u][0] = *(const int32_t *)(zb + r.y);
        zv[u][1] = *(const int32_t *)(zb + r.z);
        zv[u][2] = *(const int32_t *)(zb + r.w);
    }
}

// a[m] += the products J_t prod(other factors) of group g's records whose exponent of z_k is m
// (Sec. 3.2: a_k^(m)); long records are zero in the copy and added by the caller.  `linear`: no
// quad of the wave has a term with z_k to a power above one, and every product goes to a_k^(1)
// (a zero record adds 0).
template <int kMaxE, typename Part, bool kNarrow>
__device__ __forceinline__ void add_group(const RoundRecs<kNarrow> &R, int g, const int32_t (&zv)[4][3],
                                          Part (&a)[kMaxE + 1], bool linear) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        Part p = (Part)R.c[4 * g + u];
        p *= (Part)(int64_t)zv[u][0];
        p *= (Part)(int64_t)zv[u][1];
        p *= (Part)(int64_t)zv[u][2];
        if (kMaxE == 1 || linear) {
            a[1] += p;
        } else {
            const uint32_t e = R.r[4 * g + u].x & 0xFFu;
#pragma unroll
            for (int m = 1; m <= kMaxE; ++m) a[m] += e == (uint32_t)m ? p : (Part)0;
        }
    }
}

// All groups a quad's row reaches (the wave runs as many as its longest row needs); the LDS reads
// of the next group go out before the current group's products.
template <int kMaxE, typename Part, bool kNarrow>
__device__ __forceinline__ void add_records(const int32_t *z, const RoundRecs<kNarrow> &R, int32_t deg,
                                            Part (&a)[kMaxE + 1], bool linear) {
    constexpr int kGroups = kMoAhead / 4;
    int32_t zA[4][3], zB[4][3];
    read_group<kNarrow>(z, R, 0, zA);
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
        const bool more = g + 1 < kGroups && __ballot(deg > 16 * (g + 1)) != 0;   // uniform
        if (more) read_group<kNarrow>(z, R, g + 1, (g & 1) ? zA : zB);
        add_group<kMaxE, Part, kNarrow>(R, g, (g & 1) ? zB : zA, a, linear);
        if (!more) break;
    }
}

// kRule: SA_METROPOLIS or SA_OPT_METROPOLIS.  kR: values per lane of the optimal transition's
// enumeration (W <= 4 kR).  kNarrow: record products and coefficient sums in 32-bit arithmetic
// (exact: every coefficient and partial sum is below 2^31).  Acc: energy differences (32-bit
// when they fit).
template <int kRule, int kR, int kMaxE, bool kNarrow, typename Acc>
__global__ void __launch_bounds__(kWave) quad_mo_kernel(QuadArgs A) {
    extern __shared__ int32_t lds_state[];
    const int lane = (int)threadIdx.x;
    const int ql = lane & 3, qid = lane >> 2;
    const int read = (int)blockIdx.x;
    if (read >= A.n_reads) return;
    const DevProblem &P = A.P;
    const int32_t n = P.n;
    int32_t *z = lds_state;
    using Part = std::conditional_t<kNarrow, uint32_t, uint64_t>;

    init_state(P, z, A.z_init ? A.z_init + (size_t)read * n : nullptr, (uint32_t)read, A.instance_id, A.key0,
               A.key1, lane, kWave);
    if (lane == 0) z[n] = 1;   // the value of an unused factor place in the records' copy
    window_barrier();
    int64_t E = energy_part(P, z, lane, kWave);
    uint64_t *trace = A.trace ? A.trace + (size_t)read * (size_t)(A.s_end - A.s_begin) : nullptr;
    if (trace && A.s_end > A.s_begin) {
        uint64_t h0 = 0;
        for (int32_t k = lane; k < n; k += kWave) h0 += hash_word(k, z[k]);
        h0 = wave_sum_u64(h0);
        if (lane == 0) atomicAdd((unsigned long long *)&trace[0], (unsigned long long)h0);
    }

    int64_t dE = 0;   // this quad's applied energy changes (the same in its four lanes)
    uint64_t H = 0;   // this quad's change of the state hash in the current sweep (tracing)
    const int32_t R = A.n_rounds;   // a multiple of kRoundBatch
    if (R > 0) {
        // this lane's slot of the batch starting at round b: round b + ql, quad qid
        auto slot_at = [&](int32_t b) { return A.slots[(size_t)(b + ql) * kRoundQuads + qid]; };
        auto from = [&](int q, int32_t v) { return __builtin_amdgcn_ds_bpermute(((lane & ~3) | q) << 2, v); };
        SchedRec ms, msN = slot_at(0);
        RoundRecs<kNarrow> RA, RB;
        load_round<kNarrow>(A, 0, lane, RA);
        uint32_t y0 = 0, y1 = 0, y2 = 0, y3 = 0;

        for (int32_t s = A.s_begin; s < A.s_end; ++s) {
            const double beta = __ldg(&A.beta[s]);
            const double r_opt =
                A.otm_r >= 0.0 ? A.otm_r : (A.n_sweeps > 1 ? (double)s / (double)(A.n_sweeps - 1) : 0.0);

            // round q of the batch, its records in `cur`
            auto round = [&](int q, const RoundRecs<kNarrow> &cur) {
                const int32_t k = from(q, ms.k);
                const int64_t lo = from(q, ms.lo);
                const int64_t W = from(q, ms.width);
                const int32_t row = from(q, ms.row);
                const int32_t deg = from(q, ms.deg);
                const uint32_t emask = (uint32_t)from(q, (int32_t)ms.emask);
                const int32_t rest = from(q, ms.pad[0]);   // the row continues past the copy
                const uint32_t x0 = (uint32_t)from(q, (int32_t)y0), x1 = (uint32_t)from(q, (int32_t)y1);
                const uint32_t x2 = (uint32_t)from(q, (int32_t)y2), x3 = (uint32_t)from(q, (int32_t)y3);
                const bool valid = k >= 0;
                const int64_t zk = z[valid ? k : 0];

                const bool linear = kMaxE == 1 || (emask & ~2u) == 0;
                Part a[kMaxE + 1];
#pragma unroll
                for (int m = 0; m <= kMaxE; ++m) a[m] = 0;
                // no quad of the wave has a term with z_k to a power above one (uniform)
                const bool all_linear = kMaxE == 1 || __ballot(!linear) == 0;
                add_records<kMaxE, Part, kNarrow>(z, cur, deg, a, all_linear);
                if (__ballot(rest != 0) != 0) {
                    // records with more than three other factors, and rows longer than the copy
                    // covers: one by one from the incidence records
                    for (int32_t i = ql; rest && i < deg; i += 4) {
                        const IncRec r = P.inc[row + i];
                        if (i >= 4 * kMoAhead || (r.meta >> 8) > 3u) {
                            int e;
                            const Part p = record_product<Part, int32_t>(P, z, r, (uint64_t)P.inc_coef[row + i], e);
#pragma unroll
                            for (int m = 1; m <= kMaxE; ++m) a[m] += (kMaxE == 1 || e == m) ? p : (Part)0;
                        }
                    }
                    // every load of this path complete here, so that the common path that follows
                    // inherits none of them in flight (a wait for one would take the next round's too)
                    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
                }
                Coeffs<kMaxE, Acc> C;
                C.a[0] = 0;
#pragma unroll
                for (int m = 1; m <= kMaxE; ++m) {
                    const Part sum = quad_sum<Part>(a[m]);
                    C.a[m] = kNarrow ? (Acc)(int64_t)(int32_t)(uint32_t)sum : (Acc)sum;
                }
                const double U = (double)((((uint64_t)x2 << 32) | x3) >> 11) * 0x1p-53;
                int64_t v, d;
                if (kRule == SA_OPT_METROPOLIS && (double)x0 * 0x1p-32 < r_opt) {
                    if (linear) {
                        // dE = a1 (v - z_k): the lowest value for a1 >= 0, the highest for a1 < 0
                        v = to_i64<Acc>(C.a[1]) >= 0 ? lo : lo + W - 1;
                        d = to_i64<Acc>(C.a[1] * (Acc)(v - zk));
                    } else {
                        v = (emask & ~6u) == 0 ? quad_argmin_quadratic<kMaxE, Acc>(C, lo, W, zk, ql, d)
                                               : quad_argmin<kR, kMaxE, Acc>(C, lo, W, zk, ql, d);
                    }
                } else {
                    v = lo + (int64_t)(((uint64_t)x1 * (uint64_t)(W - 1)) >> 32);
                    if (v >= zk) v += 1;
                    // a linear variable's a_k^(m), m >= 2, are zero: dE = a1 (v - z_k), the same ring value
                    d = all_linear ? to_i64<Acc>(C.a[1] * (Acc)(v - zk)) : poly_delta(C, zk, v);
                }
                if (valid && v != zk && metropolis_accept(d, beta, U)) {
                    z[k] = (int32_t)v;   // the quad's four lanes store the same value
                    dE += d;
                    if (trace) H += hash_word(k, v) - hash_word(k, zk);
                }
            };

            for (int32_t t = 0; t < R; t += 2) {
                if ((t & 3) == 0) {
                    // a new batch: its slots arrived during the last one; its random words
                    ms = msN;
                    y0 = (uint32_t)ms.k;
                    y1 = (uint32_t)s;
                    y2 = (uint32_t)read;
                    y3 = A.instance_id;
                    philox4x32_10(y0, y1, y2, y3, A.key0, A.key1);
                }
                // the next batch's slots (after the last batch, the first: the next sweep's), loaded
                // in every pair of rounds so that no load depends on a branch
                const int32_t nb = (t | 3) + 1;
                msN = slot_at(nb < R ? nb : 0);
                // round t: the records of round t + 1 go out first
                load_round<kNarrow>(A, t + 1, lane, RB);
                round(t & 3, RA);
                // round t + 1: the records of round t + 2 (after the last round, the next sweep's first)
                load_round<kNarrow>(A, t + 2 < R ? t + 2 : 0, lane, RA);
                round((t + 1) & 3, RB);
            }
            if (trace) {
                const uint64_t hw = wave_sum_u64(ql == 0 ? H : 0ull);
                if (lane == 0) atomicAdd((unsigned long long *)&trace[s - A.s_begin], (unsigned long long)hw);
                H = 0;
            }
        }
    }
    E += (int64_t)wave_sum_u64(ql == 0 ? (uint64_t)dE : 0ull);
    if (lane == 0) A.e_out[read] = E;
    int32_t *zo = A.z_out + (size_t)read * n;
    for (int32_t k = lane; k < n; k += kWave) zo[k] = z[k];
}

}  // namespace
}  // namespace sa
