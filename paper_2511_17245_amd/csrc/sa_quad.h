// sa_quad.h -- the heat-bath sweep with one update per four lanes (a "quad"), for sparse problems.
//
// Mapping: a workgroup of kWaves wavefronts anneals one replica, its state z in LDS.  The sweep
// visits the dependency levels of the variables one after another (build_levels: a level holds
// variables none of which shares a term with another, and all of whose lower-index neighbours lie
// in earlier levels), with a workgroup barrier between levels; inside a level the 16 kWaves quads
// of the workgroup take its variables in turn, each quad updating one variable on its own.  This
// reads every neighbour as the sequential index-order sweep (Sec. 3.1) does, so the result is the
// sequential sweep's.
//
// One update (Sec. 3.2, 3.3.2): the quad's four lanes split the variable's incidence records and
// sum the coefficient a_k^(1) (and a_k^(2)) across the quad; lane q holds the values
// l + q c .. l + q c + c - 1 (c = ceil(W / 4)) and their weights w_v = exp(-beta (dE_v - dE_min))
// in registers (c = kR, the launch's class for its widest range; values past a variable's own
// range weigh zero); the cumulative weights C_v are formed in value order, one value at a time --
// lane 0 adds its c weights, hands the running sum to lane 1, and so on -- so they are the exact
// sums of the plain sequential definition; the drawn value is the first v with C_v > U * C_u,
// i.e. the number of C_v <= U * C_u (C never decreases), summed over the quad.  The factored
// variant (every variable of the launch has one width) forms a linear variable's weights as
// products of an exponential and powers of another, in order of distance from the minimising
// end, and adds them in lane blocks (quad_heat_bath): its sums differ from the sequential ones
// by rounding.
#pragma once

#include "sa_device.h"

namespace sa {
namespace {

// DPP quad_perm controls: lane i of each quad reads lane perm[i] of that quad.
constexpr int kQuadXor1 = 0xB1;   // [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;   // [2, 3, 0, 1]

template <int kCtrl>
__device__ __forceinline__ uint32_t qperm32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kCtrl, 0xf, 0xf, false);
}
template <int kCtrl>
__device__ __forceinline__ uint64_t qperm64(uint64_t x) {
    return ((uint64_t)qperm32<kCtrl>((uint32_t)(x >> 32)) << 32) | qperm32<kCtrl>((uint32_t)x);
}
// every lane of a quad takes lane kQ's value
template <int kQ>
__device__ __forceinline__ double quad_bcast(double x) {
    return __longlong_as_double((long long)qperm64<kQ * 0x55>((uint64_t)__double_as_longlong(x)));
}

template <typename Acc>
__device__ __forceinline__ Acc quad_sum(Acc x) {
    if (sizeof(Acc) == 4) {
        uint32_t y = (uint32_t)x;
        y += qperm32<kQuadXor1>(y);
        y += qperm32<kQuadXor2>(y);
        return (Acc)y;
    }
    uint64_t y = (uint64_t)x;
    y += qperm64<kQuadXor1>(y);
    y += qperm64<kQuadXor2>(y);
    return (Acc)y;
}

__device__ __forceinline__ int64_t quad_min_i64(int64_t x) {
    int64_t y = (int64_t)qperm64<kQuadXor1>((uint64_t)x);
    x = y < x ? y : x;
    y = (int64_t)qperm64<kQuadXor2>((uint64_t)x);
    return y < x ? y : x;
}

// One step of the value-order walk: lane kQ of each quad turns its weights into cumulative
// weights, starting from `carry` (the sum of the quad's earlier lanes' weights); every lane then
// takes lane kQ's new running sum as the carry.
template <int kQ, int kR>
__device__ __forceinline__ void walk_step(double (&w)[kR], int ql, double &carry) {
    if (ql == kQ) {
        double run = carry;
#pragma unroll
        for (int i = 0; i < kR; ++i) {
            run += w[i];
            w[i] = run;
        }
        carry = run;
    }
    carry = quad_bcast<kQ>(carry);
}

// Values per lane of the cold heat-bath draw (at most 4 kCold values of nonzero weight).
constexpr int kCold = 7;

// Heat-bath draw (Sec. 3.3.2) of one quad: returns the new value.  C: the quad's coefficients.
// kR: values per lane (4 kR >= W).  jinf[i]: the lane's value index q kR + i as a double when
// it lies inside this variable's range, +inf past it.
template <int kR, int kMaxE, typename Acc, bool kFact>
__device__ __forceinline__ int64_t quad_heat_bath(const Coeffs<kMaxE, Acc> &C, int64_t lo, int64_t W, int64_t zk,
                                                  double beta, double U, int ql, bool linear_in,
                                                  const double (&jinf)[kR], uint32_t Wu) {
    const uint32_t W32 = (uint32_t)W;
    const uint32_t j0 = (uint32_t)ql * (uint32_t)kR;
    const bool linear = kMaxE == 1 || linear_in;
    double w[kR];
    bool rev = false;    // the weights run in distance order from the top of the range down
    bool summed = false; // w already holds the lane's running sums
    if (linear) {
        // dE(v) = a1 (v - z_k): its minimum is at an end of the range, and dE_v - dE_min is |a1|
        // times the distance of v from that end (an exact integer, converted to double with one
        // rounding as the integer difference would be)
        const bool from_top = to_i64<Acc>(C.a[1]) < 0;
        const Acc slope = from_top ? (Acc)0 - C.a[1] : C.a[1];
        const double slope_d = sizeof(Acc) == 4 ? (double)(uint32_t)slope : (double)(int64_t)slope;
        if (!(beta * slope_d > 0.0)) {
            // every weight is exp(-0) = 1: C_v = v - l + 1 exactly, and the draw is the count of
            // those <= U W
            const double thr = U * (double)W32;
            const uint32_t below = (uint32_t)thr;   // floor: thr >= 0
            return lo + (int64_t)(below < W32 ? below : W32 - 1u);
        }
        // Cold draws.  The value at distance d from the minimising end has x = |a1| d, and when
        // beta x >= 746 its weight is exactly 0 (the exponential clamps its argument at -746, where
        // the result rounds to 0, as the oracle's exp underflows to 0).  D, the number of distances
        // with beta x < 746, is found with that same comparison.  When D <= 4 kCold for every
        // active quad of the wave, only those D values are evaluated, kc per lane (kc from the
        // wave's largest D, so that the steps skipped are the same for the whole wave), in value
        // order: the zero weights add nothing to any cumulative sum, and the W - D values outside
        // the block have C = 0 (minimum at the top) or C = total (minimum at the bottom) and are
        // counted as the full walk counts them.
        if (kR >= 16 && kMaxE == 1) {
            auto pass = [&](uint32_t d) { return beta * (slope_d * (double)d) < 746.0; };
            // pass is monotone in d, so D > 4 kCold exactly when the range holds more than 4 kCold
            // values and distance 4 kCold passes: D itself is needed only for the cold draw
            const bool wide = W32 > 4u * kCold && pass(4u * kCold);
            if (__ballot(wide) == 0) {
                const double t = 746.0 * __builtin_amdgcn_rcp(beta * slope_d);
                uint32_t D = t < (double)W32 ? (uint32_t)__builtin_ceil(t) : W32;
                D = D < 1u ? 1u : D;
                if (D < W32 && pass(D)) ++D;
                if (D < W32 && pass(D)) ++D;
                if (D > 1u && !pass(D - 1u)) --D;
                if (D > 1u && !pass(D - 1u)) --D;
                // the largest D over the active lanes, one bit at a time (D <= 4 kCold < 32)
                uint32_t dmax = 0;
#pragma unroll
                for (int bit = 4; bit >= 0; --bit) {
                    const uint32_t c = dmax | (1u << bit);
                    if (__ballot(D >= c) != 0) dmax = c;
                }
                const uint32_t kc = (dmax + 3u) / 4u;   // uniform over the wave
                double wc[kCold];
                bool valid[kCold];
#pragma unroll
                for (int i = 0; i < kCold; ++i) {
                    wc[i] = 0.0;
                    valid[i] = false;
                    if ((uint32_t)i < kc) {   // uniform over the wave
                        const uint32_t pos = (uint32_t)ql * kc + (uint32_t)i;   // position in the block
                        valid[i] = pos < D;
                        // block in value order: distance pos from the bottom, or D - 1 - pos from the top
                        const uint32_t d = from_top ? (valid[i] ? D - 1u - pos : 0u) : pos;
                        const double wv = exp_nonpos(-(beta * (slope_d * (double)d)));
                        wc[i] = valid[i] ? wv : 0.0;
                    }
                }
                double carry = 0.0;
                walk_step<0, kCold>(wc, ql, carry);
                walk_step<1, kCold>(wc, ql, carry);
                walk_step<2, kCold>(wc, ql, carry);
                walk_step<3, kCold>(wc, ql, carry);
                const double thr = U * carry;
                uint32_t below = 0;
#pragma unroll
                for (int i = 0; i < kCold; ++i) below += valid[i] && wc[i] <= thr ? 1u : 0u;
                below = quad_sum<uint32_t>(below);
                // the W - D values outside the block: C = 0 below a top block, C = total above a
                // bottom block
                below += (from_top || carry <= thr) ? W32 - D : 0u;
                return lo + (int64_t)(below < W32 ? below : W32 - 1u);
            }
        }
        // Factored weights (kFact: every variable of the launch has the same width W, kR >= 16 and
        // nd = 4 kR - W <= kR / 4).  The weight at distance d from the minimising end is e^(-c d),
        // c = beta |a1|.  The layout is by distance in both orientations: lane q holds distances
        // q kR .. q kR + kR - 1 (the places past the range are the last nd of lane 3, left out of
        // the total below), and a minimum at the top makes the walk run from the top of the range
        // down.  Place i = 8m + t of lane q is at distance q kR + 8m + t, and its weight is the
        // product G_q H_m E_t of e^(-c q kR), e^(-8 c m) and e^(-c t): G_q is one exponential, and
        // E_t and H_m are powers of another, e^(-c), formed by repeated products (at most 3 + kR / 8
        // deep).  The products are accumulated with fused multiply-adds into the running sums.  The
        // weights are rounded apart from the oracle's direct exponentials, by some ulp per product
        // level, so a draw can differ only where U C_u falls within some tens of ulp of a
        // cumulative weight.
        if constexpr (kFact) {
            constexpr int kG = kR / 8, kRest = kR % 8;
            auto wexp = [&](uint32_t d) { return exp_nonpos(-(beta * (slope_d * (double)d))); };
            const double e1 = wexp(1u);
            const double G = wexp((uint32_t)ql * (uint32_t)kR);
            double E[8];
            E[0] = 1.0;
            E[1] = e1;
            E[2] = e1 * e1;
            E[3] = E[2] * e1;
            E[4] = E[2] * E[2];
            E[5] = E[4] * e1;
            E[6] = E[4] * E[2];
            E[7] = E[4] * E[3];
            const double H8 = E[4] * E[4];
            // group m (places 8m .. 8m + 7) takes F_m = G_q H_m; the kR mod 8 places after the whole
            // groups start at distance 8 kG - 8 + kR mod 8 and take E_t for t = 8 - kR % 8 + r
            double F[kG + 1];
            F[0] = G;
            double Hm = 1.0;
#pragma unroll
            for (int m = 1; m < kG; ++m) {
                Hm = m == 1 ? H8 : Hm * H8;
                F[m] = G * Hm;
            }
            if (kRest) F[kG] = G * (Hm * E[kRest]);
            double run = 0.0;
#pragma unroll
            for (int i = 0; i < kR; ++i) {
                run = i < 8 * kG ? fma(F[i / 8], E[i % 8], run) : fma(F[kG], E[8 - kRest + (i - 8 * kG)], run);
                w[i] = run;
            }
            rev = from_top;
            summed = true;
        } else {
            // |a1| times the distance: one rounding of the exact product, as the oracle's conversion of
            // the integer difference (slope * (W - 1) is exact in double: W <= 128)
            const double s_slope = from_top ? -slope_d : slope_d;
            const double o_slope = from_top ? slope_d * (double)(W32 - 1u) : 0.0;
#pragma unroll
            for (int i = 0; i < kR; ++i) {
                // a value past the range has index +inf, so x = +inf and the argument -(beta x) = -inf
                // (beta x > 0 here), which the exponential clamps to a weight of exactly 0
                const double x = __builtin_fabs(fma(jinf[i], s_slope, o_slope));
                w[i] = exp_nonpos(-(beta * x));
            }
        }
    } else {
        int64_t dmin = INT64_MAX;
#pragma unroll
        for (int i = 0; i < kR; ++i) {
            const uint32_t j = j0 + (uint32_t)i;
            const int64_t d = poly_delta(C, zk, lo + (int64_t)(j < W32 ? j : W32 - 1u));
            dmin = d < dmin ? d : dmin;
        }
        dmin = quad_min_i64(dmin);
#pragma unroll
        for (int i = 0; i < kR; ++i) {
            // evaluated at a clamped index past the range, so that the exponentials of a lane are
            // independent instructions; such values weigh zero
            const uint32_t j = j0 + (uint32_t)i;
            const uint32_t jc = j < W32 ? j : W32 - 1u;
            const int64_t d = poly_delta(C, zk, lo + (int64_t)jc);
            const double x = sizeof(Acc) == 4 ? (double)(int32_t)((uint32_t)d - (uint32_t)dmin) : (double)(d - dmin);
            const double wv = exp_nonpos(-(beta * x));
            w[i] = j < W32 ? wv : 0.0;
        }
    }
    uint32_t below = 0;
    if constexpr (kFact) {
        // Blocked sums (the factored weights already differ from the oracle's by rounding):
        // every lane forms the running sums of its own values at once, the quad adds the lanes'
        // totals in walk order, and a lane counts its places with run <= U S - (the sum of the
        // earlier lanes' weights).  Lane 3's last nd places lie past the range (nd the same for
        // every quad): its total is its running sum at the last place inside, and a place past the
        // range is counted only where every place inside is.  In reverse (minimum at the top) the
        // cumulative weight from the top R_d stands for C: v_j is drawn for the first d = W - 1 - j
        // with R_d >= (1 - U) S, so j = W - 1 - #{d : R_d < (1 - U) S}, counted as run <= the
        // next double below the limit.
        if (!summed) {
            double run = 0.0;
#pragma unroll
            for (int i = 0; i < kR; ++i) {
                run += w[i];
                w[i] = run;
            }
        }
        const double run = w[kR - 1];
        const uint32_t nd = 4u * (uint32_t)kR - Wu;
        double last = run;
#pragma unroll
        for (int e = 1; e <= kR / 4; ++e) last = nd == (uint32_t)e ? w[kR - 1 - e] : last;
        const double t0 = quad_bcast<0>(run), t1 = quad_bcast<1>(run), t2 = quad_bcast<2>(run);
        const double c1 = t0, c2 = c1 + t1, c3 = c2 + t2;
        const double total = c3 + quad_bcast<3>(last);
        const double before = ql == 0 ? 0.0 : ql == 1 ? c1 : ql == 2 ? c2 : c3;
        double lim = (rev ? 1.0 - U : U) * total - before;
        if (rev) {
            // the largest double below lim (finite): one step of its representation toward -inf
            const int64_t b = (int64_t)__double_as_longlong(lim);
            lim = __longlong_as_double(b > 0 ? b - 1 : b == 0 ? (long long)0x8000000000000001ull : b + 1);
        }
#pragma unroll
        for (int i = 0; i < kR; ++i) below += w[i] <= lim ? 1u : 0u;
        below = quad_sum<uint32_t>(below);
        if (rev) below = below < W32 ? W32 - 1u - below : 0u;
    } else {
        double carry = 0.0;
        walk_step<0, kR>(w, ql, carry);
        walk_step<1, kR>(w, ql, carry);
        walk_step<2, kR>(w, ql, carry);
        walk_step<3, kR>(w, ql, carry);
        const double thr = U * carry;   // carry: the sum of all W weights, C at the last value
#pragma unroll
        for (int i = 0; i < kR; ++i) below += w[i] <= thr ? 1u : 0u;
        below = quad_sum<uint32_t>(below);
    }
    return lo + (int64_t)(below < W32 ? below : W32 - 1u);
}

// The quad's coefficients a_k^(m) of variable k (row `row`, `deg` incidence records): lane q takes
// records q, q + 4, ...; lanes past the row read the zero record.
template <int kMaxE, typename Acc>
__device__ __forceinline__ void quad_coeffs(const DevProblem &P, const int32_t *z, int32_t row, int32_t deg,
                                            uint32_t emask, int ql, Coeffs<kMaxE, Acc> &C) {
    Acc part[kMaxE + 1];
#pragma unroll
    for (int m = 0; m <= kMaxE; ++m) part[m] = 0;
    for (int32_t c0 = 0; c0 < deg; c0 += 4) {
        const int32_t i = c0 + ql;
        const int32_t idx = i < deg ? row + i : P.inc_pad;
        int e;
        const Acc prod = record_product<Acc, int32_t>(P, z, P.inc[idx], (uint64_t)P.inc_coef[idx], e);
#pragma unroll
        for (int m = 1; m <= kMaxE; ++m) part[m] += (kMaxE == 1 || e == m) ? prod : (Acc)0;
    }
    C.a[0] = 0;
#pragma unroll
    for (int m = 1; m <= kMaxE; ++m) C.a[m] = (emask & (1u << m)) ? quad_sum<Acc>(part[m]) : (Acc)0;
}

// a_k^(1) of variable k from its compact pair records (multilinear QUIO): h_k + sum_j J_kj z_j.
// Lane q takes records q, q + 4, ...; sixteen records of the row are loaded before any is used,
// so a typical row costs one round trip to memory and one to LDS.  Rows are padded with zero
// records (J = 0, j = 0) to a multiple of sixteen, so every load lies inside the array.
template <typename Acc>
__device__ __forceinline__ Acc quad_a1_pairs(const DevProblem &P, const int32_t *z, int32_t row, int32_t deg,
                                             int32_t h, int ql) {
    static_assert(kPairBlock == 16, "one pass loads sixteen records");
    Acc part = ql == 0 ? (Acc)(int64_t)h : (Acc)0;
    for (int32_t c0 = 0; c0 < deg; c0 += 16) {
        PairRec pr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pr[u] = P.pair[row + c0 + 4 * u + ql];
#pragma unroll
        for (int u = 0; u < 4; ++u) part += (Acc)(int64_t)pr[u].J * (Acc)(int64_t)z[pr[u].j];
    }
    return quad_sum<Acc>(part);
}

// Optimal transition of one quad (Sec. 3.3.3, as read here): the value of smallest dE over the
// whole range, z_k included, ties to the lowest value.  Lane q evaluates values q kR .. q kR +
// kR - 1; returns the value, and its dE in dbest.
template <int kR, int kMaxE, typename Acc>
__device__ __forceinline__ int64_t quad_argmin(const Coeffs<kMaxE, Acc> &C, int64_t lo, int64_t W, int64_t zk,
                                               int ql, int64_t &dbest) {
    int64_t best = INT64_MAX;
    int64_t bv = INT64_MAX;
    const uint32_t W32 = (uint32_t)W;
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const uint32_t j = (uint32_t)ql * (uint32_t)kR + (uint32_t)i;
        if (j < W32) {
            const int64_t d = poly_delta(C, zk, lo + (int64_t)j);
            if (d < best) {   // values ascend within the lane: the first minimiser is the lowest
                best = d;
                bv = lo + (int64_t)j;
            }
        }
    }
    dbest = quad_min_i64(best);
    return quad_min_i64(best == dbest ? bv : INT64_MAX);
}

// The same optimal transition for a variable whose dE holds only the exponents 1 and 2:
// dE(v) = a2 v^2 + a1 v + const.  Its smallest value over the range is at an end, or (a2 > 0) at
// an integer next to the vertex -a1 / (2 a2); the vertex's computed value is within one of the
// exact one, so floor(t) - 1 .. floor(t) + 2 hold those integers.  With z_k (dE = 0) added, the
// seven candidates hold every value of smallest dE that the enumeration's lowest-value rule can
// pick; each is evaluated exactly, two per lane, ties to the lowest value.
template <int kMaxE, typename Acc>
__device__ __forceinline__ int64_t quad_argmin_quadratic(const Coeffs<kMaxE, Acc> &C, int64_t lo, int64_t W,
                                                         int64_t zk, int ql, int64_t &dbest) {
    const int64_t hi = lo + W - 1;
    const int64_t a1 = to_i64<Acc>(C.a[1]), a2 = to_i64<Acc>(C.a[kMaxE >= 2 ? 2 : 1]);
    int64_t f = lo;
    if (kMaxE >= 2 && a2 > 0) {
        const double t = -(double)a1 / (2.0 * (double)a2);
        f = t < (double)lo ? lo : t > (double)hi ? hi : (int64_t)__builtin_floor(t);
    }
    int64_t best = INT64_MAX, bv = INT64_MAX;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = ql + 4 * u;   // candidates 0..6: lo, hi, z_k, f - 1 .. f + 2
        if (i < 7) {
            int64_t v = i == 0 ? lo : i == 1 ? hi : i == 2 ? zk : f + (int64_t)(i - 4);
            v = v < lo ? lo : v > hi ? hi : v;
            const int64_t d = poly_delta(C, zk, v);
            if (d < best || (d == best && v < bv)) {
                best = d;
                bv = v;
            }
        }
    }
    dbest = quad_min_i64(best);
    return quad_min_i64(best == dbest ? bv : INT64_MAX);
}

// kRule: SA_HEAT_BATH, or SA_HEAT_BATH_CLOSED (the O(1) draw of Sec. 3.3.2 for variables whose
// energy difference is linear, the enumeration for the others).  kR: values per lane (W <= 4 kR).
// kFact: the factored weights of linear variables (quad_heat_bath), for launches whose variables
// all have one width W with 4 kR - W <= kR / 4.  Metropolis and the optimal transition have a
// kernel of their own (sa_quad_mo.h).
template <int kRule, int kR, int kMaxE, typename Acc, int kWaves, bool kFact = false>
__global__ void __launch_bounds__(kWaves * 64) quad_kernel(QuadArgs A) {
    extern __shared__ int32_t lds_state[];
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int wave = (int)(threadIdx.x / kWave);
    const int ql = lane & 3;
    constexpr int kQuads = kWaves * 16;
    const int qid = wave * 16 + (lane >> 2);
    const int read = (int)blockIdx.x;
    if (read >= A.n_reads) return;   // uniform over the workgroup
    const DevProblem &P = A.P;
    const int32_t n = P.n;
    int32_t *z = lds_state;
    const int tid = (int)threadIdx.x, nthr = kWaves * kWave;

    init_state(P, z, A.z_init ? A.z_init + (size_t)read * n : nullptr, (uint32_t)read, A.instance_id, A.key0,
               A.key1, tid, nthr);
    window_barrier();
    int64_t E = energy_part(P, z, tid, nthr);   // this wave's share of E(z0)
    uint64_t *trace = A.trace ? A.trace + (size_t)read * (size_t)(A.s_end - A.s_begin) : nullptr;
    if (trace && A.s_end > A.s_begin) {
        uint64_t h0 = 0;
        for (int32_t k = tid; k < n; k += nthr) h0 += hash_word(k, z[k]);
        h0 = wave_sum_u64(h0);
        if (lane == 0) atomicAdd((unsigned long long *)&trace[0], (unsigned long long)h0);
    }

    // this lane's value indexes q kR + i as doubles, +inf past the range: set once when every
    // variable has the same width, else per update
    const uint32_t Wu = (uint32_t)A.uniform_width;
    double jinf[kR];
    auto set_jinf = [&](uint32_t W32) {
#pragma unroll
        for (int i = 0; i < kR; ++i) {
            const uint32_t j = (uint32_t)(ql * kR + i);
            jinf[i] = j < W32 ? (double)j : __builtin_huge_val();
        }
    };
    static_assert(kRule == SA_HEAT_BATH || kRule == SA_HEAT_BATH_CLOSED, "heat-bath rules only");
    if (!kFact && Wu) set_jinf(Wu);   // the factored weights need no indexes
    int64_t dE = 0;    // this quad's applied energy changes (the same in its four lanes)
    uint64_t H = 0;    // this quad's change of the state hash in the current sweep (tracing)
    for (int32_t s = A.s_begin; s < A.s_end; ++s) {
        const double beta = A.beta[s];
        // the slot this lane fetches for round ql of the batch at `batch` (a level ending at b1)
        auto slot_of = [&](int32_t batch, int32_t b1) {
            const int32_t my_idx = batch + ql * kQuads + qid;
            SchedRec m;
            if (my_idx < b1) {
                m = A.slots[my_idx];
            } else {
                m.k = 0;
                m.lo = 0;
                m.width = 1;
                m.row = 0;
                m.deg = 0;
                m.emask = 0;
                m.pad[0] = 0;
            }
            return m;
        };
        for (int32_t l = 0; l < A.n_levels; ++l) {
            const int32_t b0 = A.level_start[l], b1 = A.level_start[l + 1];
            // batches of four rounds: lane q of a quad fetches the slot of the batch's round q and
            // draws its random words; in round q the quad reads them from lane q
            for (int32_t batch = b0; batch < b1; batch += 4 * kQuads) {
                const SchedRec ms = slot_of(batch, b1);
                uint32_t y0 = (uint32_t)ms.k, y1 = (uint32_t)s, y2 = (uint32_t)read, y3 = A.instance_id;
                // the round keys are formed again at each draw (scalar adds) rather than held in
                // registers across the sweep
                uint32_t k0 = A.key0, k1 = A.key1;
                asm volatile("" : "+s"(k0), "+s"(k1));
                philox4x32_10(y0, y1, y2, y3, k0, k1);
                for (int q = 0; q < 4; ++q) {
                    const int32_t idx = batch + q * kQuads + qid;
                    if (batch + q * kQuads >= b1) break;   // uniform: the level has no round q here
                    // the round's reads go out at a raised wave priority, so that they start under
                    // the other waves' arithmetic; the arithmetic runs at the normal priority
                    __builtin_amdgcn_s_setprio(2);
                    const int src = ((lane & ~3) | q) << 2;
                    auto from_q = [&](uint32_t v) { return (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)v); };
                    const int32_t k = (int32_t)from_q((uint32_t)ms.k);
                    const int64_t lo = (int32_t)from_q((uint32_t)ms.lo);
                    const int64_t W = (int32_t)from_q((uint32_t)ms.width);
                    const int32_t row = (int32_t)from_q((uint32_t)ms.row);
                    const int32_t deg = (int32_t)from_q((uint32_t)ms.deg);
                    const uint32_t emask = from_q(ms.emask);
                    const int32_t h = (int32_t)from_q((uint32_t)ms.pad[0]);
                    const uint32_t x1 = from_q(y1), x2 = from_q(y2), x3 = from_q(y3);
                    if (idx < b1) {
                        const double U = (double)((((uint64_t)x2 << 32) | x3) >> 11) * 0x1p-53;
                        const int64_t zk = z[k];
                        Coeffs<kMaxE, Acc> C;
                        if (kMaxE == 1 && P.pair) {
                            C.a[0] = 0;
                            C.a[1] = quad_a1_pairs<Acc>(P, z, row, deg, h, ql);
                        } else {
                            quad_coeffs<kMaxE, Acc>(P, z, row, deg, emask, ql, C);
                        }
                        __builtin_amdgcn_s_setprio(0);
                        const bool linear = kMaxE == 1 || (emask & ~2u) == 0;
                        int64_t v;
                        if (kRule == SA_HEAT_BATH_CLOSED && linear) {
                            v = heat_bath_closed(to_i64<Acc>(C.a[1]), lo, W, beta, U, x1);
                        } else {
                            if (!kFact && !Wu) set_jinf((uint32_t)W);
                            v = quad_heat_bath<kR, kMaxE, Acc, kFact>(C, lo, W, zk, beta, U, ql, linear, jinf, Wu);
                        }
                        if (v != zk) {
                            z[k] = (int32_t)v;   // the quad's four lanes store the same value
                            dE += poly_delta(C, zk, v);
                            if (trace) H += hash_word(k, v) - hash_word(k, zk);
                        }
                    }
                }
            }
            // the next level reads what this one wrote: a workgroup barrier between waves (one
            // wave's LDS accesses complete in order, so a single wave needs none)
            if constexpr (kWaves > 1) window_barrier();
        }
        if (trace) {
            const uint64_t hw = wave_sum_u64(ql == 0 ? H : 0ull);
            if (lane == 0) atomicAdd((unsigned long long *)&trace[s - A.s_begin], (unsigned long long)hw);
            H = 0;
        }
    }
    E += (int64_t)wave_sum_u64(ql == 0 ? (uint64_t)dE : 0ull);
    int64_t *parts = (int64_t *)(lds_state + (((size_t)n + 1) & ~(size_t)1));
    if (lane == 0) parts[wave] = E;
    window_barrier();
    if (wave == 0 && lane == 0) {
        int64_t tot = 0;
        for (int q = 0; q < kWaves; ++q) tot += parts[q];
        A.e_out[read] = tot;
    }
    int32_t *zo = A.z_out + (size_t)read * n;
    for (int32_t k = tid; k < n; k += nthr) zo[k] = z[k];
}

}  // namespace
}  // namespace sa
