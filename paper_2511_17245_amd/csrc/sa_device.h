// sa_device.h -- gfx950 device code of the single-variable update sweep (Sec. 3.1) for QUIO/HUIO.
//
// Mapping: a replica (read) is updated by one 64-lane wavefront, or by G = 2, 4, 8 or 16 waves of
// a workgroup that update the G mutually non-interacting variables of a schedule window at once
// (a barrier closes each window; the result equals the sequential sweep).  With G = 1 the waves of
// a workgroup are independent replicas.  A replica's state z lives in LDS when it fits, else in
// its row of the output buffer.  For the visited variable k the lanes split the terms containing
// z_k (each lane forms one term's product of the other factors) and, for the heat bath and the
// optimal transition, the candidate values v in [l_k, u_k].  Energies and energy differences are
// exact integers (two's-complement wrap-around arithmetic, exact whenever the true value fits
// int64, which the host checks); FP64 is used only for the exponentials and logarithms of the
// acceptance test and the heat-bath draws.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) with counter (k, s, read, instance) and key
// = seed; for each block of 64 windows, lane j computes the words of this wave's slot in window
// j, and the update reads them from lane j.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "sa_internal.h"

namespace sa {
namespace {

constexpr int kWave = 64;

// ------------------------------------------------------------------------------------------------
// Philox4x32-10 block function.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                              uint32_t &c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        // both words of each product from one 32 x 32 -> 64-bit multiply
        const uint64_t p0 = (uint64_t)m0 * c0, p1 = (uint64_t)m1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// ------------------------------------------------------------------------------------------------
// Wavefront collectives.  Integer reductions are order-independent (wrap-around sums, min), so any
// exchange pattern gives the same value.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t uni32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint32_t lane_read32(uint32_t x, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}

__device__ __forceinline__ uint64_t lane_read64(uint64_t x, int lane) {
    return ((uint64_t)lane_read32((uint32_t)(x >> 32), lane) << 32) | lane_read32((uint32_t)x, lane);
}

// DPP move of a 64-bit value (two 32-bit halves); lanes without a valid source take `identity`.
template <int kCtrl, int kRowMask, int kBankMask>
__device__ __forceinline__ uint64_t dpp64(uint64_t x, uint64_t identity) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)identity, (int)(uint32_t)x,
                                                              kCtrl, kRowMask, kBankMask, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(identity >> 32),
                                                              (int)(uint32_t)(x >> 32), kCtrl, kRowMask,
                                                              kBankMask, false);
    return ((uint64_t)hi << 32) | lo;
}
// DPP move of a 64-bit value over all rows; lanes whose source lies outside their row read zero
// (bound_ctrl), so no old value is needed.
template <int kCtrl>
__device__ __forceinline__ uint64_t dpp64_zero(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)x, kCtrl, 0xf, 0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(x >> 32), kCtrl, 0xf, 0xf, true);
    return ((uint64_t)hi << 32) | lo;
}
template <int kCtrl, int kRowMask, int kBankMask>
__device__ __forceinline__ uint32_t dpp32(uint32_t x, uint32_t identity) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)x, kCtrl, kRowMask, kBankMask, false);
}

// GFX9 DPP controls: row_shr:n = 0x110 + n, row_bcast:15 = 0x142, row_bcast:31 = 0x143,
// wave_shr:1 = 0x138.  The six steps below form an inclusive scan whose lane 63 holds the
// reduction of all 64 lanes (rows of 16 lanes, then the row broadcasts).
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
    x += dpp64<0x111, 0xf, 0xf>(x, 0);
    x += dpp64<0x112, 0xf, 0xf>(x, 0);
    x += dpp64<0x114, 0xf, 0xf>(x, 0);
    x += dpp64<0x118, 0xf, 0xf>(x, 0);
    x += dpp64<0x142, 0xa, 0xf>(x, 0);
    x += dpp64<0x143, 0xc, 0xf>(x, 0);
    return lane_read64(x, kWave - 1);
}

__device__ __forceinline__ int64_t min64(int64_t a, uint64_t b) { return (int64_t)b < a ? (int64_t)b : a; }

__device__ __forceinline__ int64_t wave_min_i64(int64_t x) {
    const uint64_t id = (uint64_t)INT64_MAX;
    x = min64(x, dpp64<0x111, 0xf, 0xf>((uint64_t)x, id));
    x = min64(x, dpp64<0x112, 0xf, 0xf>((uint64_t)x, id));
    x = min64(x, dpp64<0x114, 0xf, 0xf>((uint64_t)x, id));
    x = min64(x, dpp64<0x118, 0xf, 0xf>((uint64_t)x, id));
    x = min64(x, dpp64<0x142, 0xa, 0xf>((uint64_t)x, id));
    x = min64(x, dpp64<0x143, 0xc, 0xf>((uint64_t)x, id));
    return (int64_t)lane_read64((uint64_t)x, kWave - 1);
}

__device__ __forceinline__ int32_t min32(int32_t a, uint32_t b) { return (int32_t)b < a ? (int32_t)b : a; }

__device__ __forceinline__ int32_t wave_min_i32(int32_t x) {
    const uint32_t id = (uint32_t)INT32_MAX;
    x = min32(x, dpp32<0x111, 0xf, 0xf>((uint32_t)x, id));
    x = min32(x, dpp32<0x112, 0xf, 0xf>((uint32_t)x, id));
    x = min32(x, dpp32<0x114, 0xf, 0xf>((uint32_t)x, id));
    x = min32(x, dpp32<0x118, 0xf, 0xf>((uint32_t)x, id));
    x = min32(x, dpp32<0x142, 0xa, 0xf>((uint32_t)x, id));
    x = min32(x, dpp32<0x143, 0xc, 0xf>((uint32_t)x, id));
    return (int32_t)lane_read32((uint32_t)x, kWave - 1);
}

// Orders a lane's LDS/global state write before later reads by other lanes of the same wave.
template <bool kStateInLds>
__device__ __forceinline__ void state_write_fence() {
    if (kStateInLds) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// Integer arithmetic of energy differences is done modulo 2^32 (Acc = uint32_t) or 2^64
// (Acc = uint64_t).  Sums and products of a ring are exact modulo its size, so a result whose
// true value fits the signed range is exact whatever the intermediate wrap-arounds; the host
// picks 32 bits only when every |dE| of the problem is below 2^30 (differences of two values
// then fit too).
template <typename Acc>
__device__ __forceinline__ int64_t to_i64(Acc x) {
    if (sizeof(Acc) == 4) return (int64_t)(int32_t)(uint32_t)x;
    return (int64_t)(uint64_t)x;
}

template <typename Acc>
__device__ __forceinline__ Acc wave_sum(Acc x);
template <>
__device__ __forceinline__ uint64_t wave_sum<uint64_t>(uint64_t x) { return wave_sum_u64(x); }
template <>
__device__ __forceinline__ uint32_t wave_sum<uint32_t>(uint32_t x) {
    x += dpp32<0x111, 0xf, 0xf>(x, 0);
    x += dpp32<0x112, 0xf, 0xf>(x, 0);
    x += dpp32<0x114, 0xf, 0xf>(x, 0);
    x += dpp32<0x118, 0xf, 0xf>(x, 0);
    x += dpp32<0x142, 0xa, 0xf>(x, 0);
    x += dpp32<0x143, 0xc, 0xf>(x, 0);
    return lane_read32(x, kWave - 1);
}

// x^e with wrap-around
template <typename Acc>
__device__ __forceinline__ Acc upow(Acc x, int e) {
    Acc r = 1;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// State hash for tracing: the hash of z is sum_k mix(k 2^32 + (uint32)z_k) modulo 2^64, with mix the
// 64-bit finaliser of SplitMix64 (Stafford's variant 13).  Being a sum, it is kept up to date from
// the accepted moves alone, whichever wave makes them.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ __forceinline__ uint64_t hash_word(int32_t k, int64_t v) {
    return mix64(((uint64_t)(uint32_t)k << 32) | (uint64_t)(uint32_t)(int32_t)v);
}

// J_t times the product of the term's other factors, for one incidence record of the row being
// visited.  Sets e to the exponent of the visited variable in the term.  A zero record (meta = 0,
// coef = 0) contributes nothing, so lanes beyond the row hold one.
template <typename Acc, typename ZT>
__device__ __forceinline__ Acc record_product(const DevProblem &P, const ZT *z, const IncRec &r,
                                              uint64_t coef, int &e) {
    e = (int)(r.meta & 0xFFu);
    const int no = (int)(r.meta >> 8);
    Acc prod = (Acc)coef;
    if (P.max_other <= 1) {
        // pair terms only (QUIO): at most one other factor
        const int64_t z0 = z[r.o[0]];
        prod *= no > 0 ? (Acc)z0 : (Acc)1;
    } else if (no <= 3) {
        // all three reads issued together (unused slots hold index 0, a valid variable)
        const int64_t z0 = z[r.o[0]], z1 = z[r.o[1]], z2 = z[r.o[2]];
        prod *= no > 0 ? (Acc)z0 : (Acc)1;
        prod *= no > 1 ? (Acc)z1 : (Acc)1;
        prod *= no > 2 ? (Acc)z2 : (Acc)1;
    } else {
        // the list is 16-byte aligned and padded with -1 to whole int4: four indices per load (a
        // wider round of loads raises the register count of every kernel that holds this path),
        // and a pad index multiplies by one
        const int4 *o = (const int4 *)(P.overflow + r.o[0]);
        for (int f0 = 0; f0 < no; f0 += 4) {
            const int4 q = o[f0 / 4];
            const int32_t ix[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int64_t zv = z[ix[c] < 0 ? 0 : ix[c]];
                prod *= ix[c] < 0 ? (Acc)1 : (Acc)zv;
            }
        }
    }
    return prod;
}

// Loads this lane's record of chunk [c0, c0 + 64) of a row; lanes past the row's end read the zero
// record kept after the last row, so every lane loads.
__device__ __forceinline__ void load_record(const DevProblem &P, int32_t row, int32_t deg, int32_t c0,
                                            int lane, IncRec &r, uint64_t &coef) {
    const int32_t idx = lane < deg - c0 ? row + c0 + lane : P.inc_pad;
    r = P.inc[idx];
    coef = (uint64_t)P.inc_coef[idx];
}

// Dense form, one window ahead: this lane's first 16 bytes of row k, h_k and the diagonal d_k.
__device__ __forceinline__ void prefetch_dense(const DevProblem &P, int32_t k, int lane, int4 &first,
                                               uint64_t &h, int64_t &dk) {
    first = make_int4(0, 0, 0, 0);
    h = 0;
    dk = 0;
    if (k < 0) return;
    const int32_t j0 = lane * 16;
    if (j0 < P.n) {
        const char *row = (const char *)P.jd + (size_t)k * P.row_stride * P.jbytes;
        first = *(const int4 *)(row + (size_t)j0 * P.jbytes);
    }
    h = (uint64_t)P.h[k];
    dk = P.d[k];
}

// Dense form: this lane's part of sum_j J_kj z_j over row k of the coupling matrix.  Lane l reads
// elements 16l.. of each 1024-element block (one 16-byte load for int8 rows, four for int32); the
// row's padding is zero, so indexes past N are clamped instead of tested.
// `first`, when given, holds the lane's first 16 bytes of the row, loaded one window ahead.
template <typename Acc, typename ZT>
__device__ __forceinline__ Acc dense_dot(const DevProblem &P, const ZT *z, int32_t k, int lane,
                                         const int4 *first) {
    const int32_t n = P.n;
    Acc acc = 0;
    if (P.jbytes == 1) {
        const int8_t *row = (const int8_t *)P.jd + (size_t)k * P.row_stride;

        for (int32_t j0 = lane * 16; j0 < n; j0 += kWave * 16) {
            const int4 q = (first && j0 < kWave * 16) ? *first : *(const int4 *)(row + j0);
            const uint32_t w[4] = {(uint32_t)q.x, (uint32_t)q.y, (uint32_t)q.z, (uint32_t)q.w};
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int32_t jv = (int32_t)(int8_t)(w[u >> 2] >> (8 * (u & 3)));
                const int32_t j = j0 + u < n ? j0 + u : n - 1;
                acc += (Acc)(int64_t)jv * (Acc)(int64_t)z[j];
            }
        }
    } else {
        const int32_t *row = (const int32_t *)P.jd + (size_t)k * P.row_stride;

        for (int32_t j0 = lane * 16; j0 < n; j0 += kWave * 16) {
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const int4 q = (first && q4 == 0 && j0 < kWave * 16) ? *first
                                                                     : *(const int4 *)(row + j0 + 4 * q4);
                const int32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int32_t j = j0 + 4 * q4 + u < n ? j0 + 4 * q4 + u : n - 1;
                    acc += (Acc)(int64_t)w[u] * (Acc)(int64_t)z[j];
                }
            }
        }
    }
    return acc;
}

// Dense form, the paper's coefficient cache (Sec. 3.2): c1_i = h_i + sum_j J_ij z_j for every
// variable of one replica, in LDS.  Threads tid, tid + nthr, ... fill their rows from the state.
template <typename ZT>
__device__ __forceinline__ void dense_cache_init(const DevProblem &P, const ZT *z, int64_t *c1, int tid, int nthr) {
    const int32_t n = P.n;
    for (int32_t i = tid; i < n; i += nthr) {
        uint64_t acc = (uint64_t)P.h[i];
        if (P.jbytes == 1) {
            const int8_t *row = (const int8_t *)P.jd + (size_t)i * P.row_stride;
            for (int32_t j = 0; j < n; ++j) acc += (uint64_t)(int64_t)row[j] * (uint64_t)(int64_t)z[j];
        } else {
            const int32_t *row = (const int32_t *)P.jd + (size_t)i * P.row_stride;
            for (int32_t j = 0; j < n; ++j) acc += (uint64_t)(int64_t)row[j] * (uint64_t)(int64_t)z[j];
        }
        c1[i] = (int64_t)acc;
    }
}

// Dense form with the coefficient cache, one window ahead: this lane's couplings J_k,lane and
// J_k,lane+64 of row k (zero past N), h_k and the diagonal d_k.
__device__ __forceinline__ void prefetch_dense_col(const DevProblem &P, int32_t k, int lane, int4 &jcol, uint64_t &h,
                                                   int64_t &dk) {
    jcol = make_int4(0, 0, 0, 0);
    h = 0;
    dk = 0;
    if (k < 0) return;
    const int32_t n = P.n;
    if (P.jbytes == 1) {
        const int8_t *row = (const int8_t *)P.jd + (size_t)k * P.row_stride;
        jcol.y = lane < n ? row[lane] : 0;
        jcol.z = lane + kWave < n ? row[lane + kWave] : 0;
    } else {
        const int32_t *row = (const int32_t *)P.jd + (size_t)k * P.row_stride;
        jcol.y = lane < n ? row[lane] : 0;
        jcol.z = lane + kWave < n ? row[lane + kWave] : 0;
    }
    h = (uint64_t)P.h[k];
    dk = P.d[k];
}

// After z_k moved by dz: c1_i += J_ik dz for every i (the matrix's diagonal is zero, so c1_k does not
// change).  Lane l owns i = l, l + 64, ...; `jcol`, when given, holds J_k,l and J_k,l+64 (loaded one
// window ahead), which cover N <= 128.
__device__ __forceinline__ void dense_cache_update(const DevProblem &P, int64_t *c1, int32_t k, int64_t dz, int lane,
                                                   const int4 *jcol) {
    const int32_t n = P.n;
    if (jcol && n <= 2 * kWave) {
        if (lane < n) atomicAdd((unsigned long long *)&c1[lane], (unsigned long long)((int64_t)jcol->y * dz));
        if (lane + kWave < n)
            atomicAdd((unsigned long long *)&c1[lane + kWave], (unsigned long long)((int64_t)jcol->z * dz));
        return;
    }
    for (int32_t i = lane; i < n; i += kWave) {
        const int64_t J = P.jbytes == 1 ? (int64_t)((const int8_t *)P.jd)[(size_t)k * P.row_stride + i]
                                        : (int64_t)((const int32_t *)P.jd)[(size_t)k * P.row_stride + i];
        atomicAdd((unsigned long long *)&c1[i], (unsigned long long)(J * dz));
    }
}

// Uniform coefficients a_k^(m) (Sec. 3.2, T_k = sum_m a_k^(m) z_k^m) for m = 1..kMaxE; every
// index is static so the coefficients stay in registers.
template <int kMaxE, typename Acc>
struct Coeffs {
    Acc a[kMaxE + 1];
};

// r0/coef0: the lane's first incidence record (sparse form), loaded one window ahead.
template <int kMaxE, typename Acc, typename ZT>
__device__ __forceinline__ void row_coeffs(const DevProblem &P, const ZT *z, int32_t k, int32_t row,
                                           int32_t deg, uint32_t emask, int lane, const IncRec &r0,
                                           uint64_t coef0, Coeffs<kMaxE, Acc> &C, const int64_t *c1 = nullptr) {
    if (P.dense && c1) {
        // the coefficient cache: a^(1) from LDS, a^(2) = J_kk
#pragma unroll
        for (int m = 0; m <= kMaxE; ++m) C.a[m] = 0;
        C.a[1] = (Acc)(uint64_t)c1[k];
        if (kMaxE >= 2) C.a[kMaxE >= 2 ? 2 : 1] = (Acc)P.d[k];
        return;
    }
    if (P.dense) {
        // QUIO: a^(1) = h_k + sum_j J_kj z_j, a^(2) = J_kk (Sec. 3.2, the c^(1), c^(2) of QUIO)
#pragma unroll
        for (int m = 0; m <= kMaxE; ++m) C.a[m] = 0;
        if (sizeof(Acc) == 8 && P.coef32)   // a^(1) fits 32 bits: the row product in 32-bit
            C.a[1] = (Acc)(int64_t)(int32_t)(wave_sum<uint32_t>(dense_dot<uint32_t, ZT>(P, z, k, lane, nullptr)) +
                                             (uint32_t)P.h[k]);
        else
            C.a[1] = wave_sum<Acc>(dense_dot<Acc, ZT>(P, z, k, lane, nullptr)) + (Acc)P.h[k];
        if (kMaxE >= 2) C.a[kMaxE >= 2 ? 2 : 1] = (Acc)P.d[k];
        return;
    }
    if (sizeof(Acc) == 8 && P.coef32 && deg <= kWave) {
        // every coefficient fits 32 bits: products and wave sums in 32-bit arithmetic, then
        // sign-extended (exact: the true values are below 2^31)
        uint32_t part32[kMaxE + 1];
        int e;
        const uint32_t prod = record_product<uint32_t, ZT>(P, z, r0, coef0, e);
#pragma unroll
        for (int m = 1; m <= kMaxE; ++m) part32[m] = (kMaxE == 1 || e == m) ? prod : 0u;
        C.a[0] = 0;
#pragma unroll
        for (int m = 1; m <= kMaxE; ++m)
            C.a[m] = (emask & (1u << m)) ? (Acc)(int64_t)(int32_t)wave_sum<uint32_t>(part32[m]) : (Acc)0;
        return;
    }
    Acc part[kMaxE + 1];
#pragma unroll
    for (int m = 0; m <= kMaxE; ++m) part[m] = 0;
    // kMaxE = 1: every record holds z_k to the first power (the zero record contributes 0)
    {
        int e;
        const Acc prod = record_product<Acc, ZT>(P, z, r0, coef0, e);
#pragma unroll
        for (int m = 1; m <= kMaxE; ++m) part[m] += (kMaxE == 1 || e == m) ? prod : (Acc)0;
    }
    // further chunks (dense rows): four chunks' records are loaded before any is used
    for (int32_t c0 = kWave; c0 < deg; c0 += 4 * kWave) {
        IncRec r[4];
        uint64_t coef[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) load_record(P, row, deg, c0 + u * kWave, lane, r[u], coef[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int e;
            const Acc prod = record_product<Acc, ZT>(P, z, r[u], coef[u], e);
#pragma unroll
            for (int m = 1; m <= kMaxE; ++m) part[m] += (kMaxE == 1 || e == m) ? prod : (Acc)0;
        }
    }
    C.a[0] = 0;
#pragma unroll
    for (int m = 1; m <= kMaxE; ++m) C.a[m] = (emask & (1u << m)) ? wave_sum<Acc>(part[m]) : (Acc)0;
}

// dE(v) = sum_m a^(m) (v^m - z_k^m)  (Sec. 3.2)
template <int kMaxE, typename Acc>
__device__ __forceinline__ int64_t poly_delta(const Coeffs<kMaxE, Acc> &C, int64_t zk, int64_t v) {
    Acc d = C.a[1] * (Acc)(v - zk), vp = (Acc)v, zp = (Acc)zk;
#pragma unroll
    for (int m = 2; m <= kMaxE; ++m) {
        vp *= (Acc)v;
        zp *= (Acc)zk;
        d += C.a[m] * (vp - zp);
    }
    return to_i64<Acc>(d);
}

// dE of one proposed value, directly from the row: sum over terms of J_t prod(others) (v^e - z^e).
// linear: no term holds z_k to a power above one, so dE = (sum_t J_t prod(others)) (v - z_k).
// kDensePre (dense form): r0 holds the lane's first 16 bytes of the coupling row, coef0 = h_k and
// dk = d_k, all loaded one window ahead; otherwise r0/coef0 are the first incidence record.
template <typename Acc, typename ZT, bool kDensePre>
__device__ __forceinline__ int64_t direct_delta(const DevProblem &P, const ZT *z, int32_t k, int32_t row,
                                                int32_t deg, int64_t zk, int64_t v, int lane,
                                                const IncRec &r0, uint64_t coef0, int64_t dk, bool linear) {
    if (P.dense) {
        const int4 first = make_int4((int)r0.meta, r0.o[0], r0.o[1], r0.o[2]);
        Acc a1;
        if (sizeof(Acc) == 8 && P.coef32)   // a^(1) fits 32 bits: the row product in 32-bit
            a1 = (Acc)(int64_t)(int32_t)(wave_sum<uint32_t>(dense_dot<uint32_t, ZT>(P, z, k, lane,
                                                                                   kDensePre ? &first : nullptr)) +
                                         (uint32_t)(kDensePre ? coef0 : (uint64_t)P.h[k]));
        else
            a1 = wave_sum<Acc>(dense_dot<Acc, ZT>(P, z, k, lane, kDensePre ? &first : nullptr)) +
                 (kDensePre ? (Acc)coef0 : (Acc)P.h[k]);
        const Acc dd = kDensePre ? (Acc)dk : (Acc)P.d[k];
        const Acc d = a1 * (Acc)(v - zk) + dd * ((Acc)v * (Acc)v - (Acc)zk * (Acc)zk);
        return to_i64<Acc>(d);
    }
    int e;
    if (sizeof(Acc) == 8 && P.coef32 && linear && deg <= kWave) {
        // a1 fits 32 bits: the products and the wave sum in 32-bit arithmetic, dE in 64-bit
        const uint32_t p32 = record_product<uint32_t, ZT>(P, z, r0, coef0, e);
        return (int64_t)(int32_t)wave_sum<uint32_t>(p32) * (v - zk);
    }
    Acc prod = record_product<Acc, ZT>(P, z, r0, coef0, e);
    if (linear && deg <= kWave) return to_i64<Acc>(wave_sum<Acc>(prod) * (Acc)(v - zk));
    Acc acc = prod * (upow<Acc>((Acc)v, e) - upow<Acc>((Acc)zk, e));
    for (int32_t c0 = kWave; c0 < deg; c0 += 4 * kWave) {
        IncRec r[4];
        uint64_t coef[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) load_record(P, row, deg, c0 + u * kWave, lane, r[u], coef[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            prod = record_product<Acc, ZT>(P, z, r[u], coef[u], e);
            acc += prod * (upow<Acc>((Acc)v, e) - upow<Acc>((Acc)zk, e));
        }
    }
    return to_i64<Acc>(wave_sum<Acc>(acc));
}

// e^x for x <= 0 (every exponential of the annealer has a non-positive argument): x = n ln 2 + r
// with |r| <= ln(2)/2, e^r by the degree-11 polynomial that interpolates it at the 12 Chebyshev
// nodes of that interval (relative error below 2^-55.7; gen_exp_poly.py derives the coefficients
// and checks the routine: at most about 0.83 ulp), then scaled by 2^n.  The scaling rounds once,
// so below -745.2, where e^x is under half the smallest subnormal, the result is 0 (arguments
// under -746 are clamped there first).  Within about an ulp, like the host library the oracle
// uses; a last-bit difference moves a draw only when a uniform number falls within that ulp of a
// threshold.
__device__ __forceinline__ double exp_nonpos(double x) {
    const double xc = x > -746.0 ? x : -746.0;
    const double n = rint(xc * 1.4426950408889634);     // 1 / ln 2
    double r = fma(-n, 0.6931471803691238, xc);          // ln 2 rounded to 32 bits (n * it exact)
    r = fma(-n, 1.9082149292705877e-10, r);              // the rest of ln 2
    double p = 2.5110037605963777e-08;
    p = fma(p, r, 2.763263963904103e-07);
    p = fma(p, r, 2.755724091857897e-06);
    p = fma(p, r, 2.4801485482328494e-05);
    p = fma(p, r, 0.00019841269890047113);
    p = fma(p, r, 0.0013888888952314775);
    p = fma(p, r, 0.008333333333319601);
    p = fma(p, r, 0.0416666666664881);
    p = fma(p, r, 0.1666666666666668);
    p = fma(p, r, 0.5000000000000019);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, (int)n);
}

// Metropolis acceptance min[1, exp(-dE/T)] (Sec. 3.3.1), T = 1/beta; U in [0,1).
__device__ __forceinline__ bool metropolis_accept(int64_t d, double beta, double U) {
    if (d <= 0) return true;
    return U < exp_nonpos(-(beta * (double)d));
}

// DPP destinations that keep zeros where their move does not write: each is written only by the
// one masked move it serves, so the rows (or the lane) that the move skips hold the zero they
// started with, and no zeroing instruction is needed per scan.  Kept by the caller across scans.
struct ScanCarry {
    uint64_t b15 = 0, b31 = 0, sh = 0;
};

// Inclusive scan of one double per lane in the order of the DPP network: inside each row of 16
// lanes a Kogge-Stone scan (row_shr 1, 2, 4, 8), then rows 1 and 3 add the last lane of rows 0
// and 2 (row_bcast:15), then rows 2 and 3 add lane 31 (row_bcast:31).  Lanes without a source add
// +0.0, which leaves a non-negative value unchanged.
__device__ __forceinline__ double wave_scan_rows(double x, ScanCarry &cy) {
    auto step = [](double v, uint64_t shifted) { return v + __longlong_as_double((long long)shifted); };
    x = step(x, dpp64_zero<0x111>((uint64_t)__double_as_longlong(x)));
    x = step(x, dpp64_zero<0x112>((uint64_t)__double_as_longlong(x)));
    x = step(x, dpp64_zero<0x114>((uint64_t)__double_as_longlong(x)));
    x = step(x, dpp64_zero<0x118>((uint64_t)__double_as_longlong(x)));
    cy.b15 = dpp64<0x142, 0xa, 0xf>((uint64_t)__double_as_longlong(x), cy.b15);
    x = step(x, cy.b15);
    cy.b31 = dpp64<0x143, 0xc, 0xf>((uint64_t)__double_as_longlong(x), cy.b31);
    x = step(x, cy.b31);
    return x;
}

// Lane l receives lane l-1's value, lane 0 receives +0.0 (wave_shr:1; lane 0 is never written).
__device__ __forceinline__ double wave_shift_up1_zero(double x, ScanCarry &cy) {
    cy.sh = dpp64<0x138, 0xf, 0xf>((uint64_t)__double_as_longlong(x), cy.sh);
    return __longlong_as_double((long long)cy.sh);
}

// Heat-bath choice (Sec. 3.3.2) among all W values, with the fixed summation order: value j of the
// range belongs to lane j / c (c = ceil(W/64)); lane sums are left to right; the lanes' sums are
// combined by wave_scan_rows; the first value whose cumulative weight exceeds U * total is drawn
// (the last value if rounding leaves none).  W < 2^31, so value indexes are 32-bit: j0 + i < 64 c
// <= W + 63.
template <int kRegChunk, int kMaxE, typename Acc>
__device__ __forceinline__ int64_t heat_bath_pick(const Coeffs<kMaxE, Acc> &C, int64_t lo, int64_t W,
                                                  int64_t zk, double beta, double U, int lane, bool linear_in,
                                                  ScanCarry &cy) {
    const uint32_t W32 = (uint32_t)W;
    const uint32_t c = (W32 + kWave - 1) / kWave;
    const uint32_t j0 = (uint32_t)lane * c;
    const bool linear = kMaxE == 1 || linear_in;   // no term holds z_k to a power above one
    // Weights are taken relative to the minimum energy difference.  Linear dE(v) = a1 (v - z_k)
    // has it at an end of the range, and dE(v) - dE_min = |a1| times the distance of v from that
    // end, the same integer as the difference of the two energy differences.
    int64_t dmin = 0, dlane = INT64_MAX;   // dlane: the smallest dE of this lane's values
    Acc slope = 0;
    bool from_top = false;
    if (linear) {
        from_top = to_i64<Acc>(C.a[1]) < 0;
        slope = from_top ? (Acc)0 - C.a[1] : C.a[1];
    } else if (kMaxE == 2 && c > 8) {
        // dE(v) = a2 v^2 + a1 v + const: over the lane's values its minimum is at an end or at an
        // integer next to the vertex v = -a1 / (2 a2) (a2 > 0).  The vertex's index, computed in
        // double, is within one of the exact one, so the integers floor(t) - 1 .. floor(t) + 2 hold
        // the minimisers; every candidate is evaluated exactly.
        if (j0 < W32) {
            const uint32_t jh = j0 + c - 1u < W32 ? j0 + c - 1u : W32 - 1u;
            const int64_t dl = poly_delta(C, zk, lo + (int64_t)j0), dh = poly_delta(C, zk, lo + (int64_t)jh);
            dlane = dl < dh ? dl : dh;
            const int64_t a1 = to_i64<Acc>(C.a[1]), a2 = to_i64<Acc>(C.a[kMaxE >= 2 ? 2 : 1]);
            if (a2 > 0) {
                const double t = -(double)a1 / (2.0 * (double)a2) - (double)lo;
                if (t > (double)j0 - 2.0 && t < (double)jh + 2.0) {
                    const int64_t f = (int64_t)__builtin_floor(t);
#pragma unroll
                    for (int e = -1; e <= 2; ++e) {
                        const int64_t j = f + e;
                        if (j >= (int64_t)j0 && j <= (int64_t)jh) {
                            const int64_t d = poly_delta(C, zk, lo + j);
                            dlane = d < dlane ? d : dlane;
                        }
                    }
                }
            }
        }
        dmin = wave_min_i64(dlane);
    } else {
        for (uint32_t i = 0; i < c; ++i) {
            const uint32_t j = j0 + i;
            if (j < W32) {
                const int64_t d = poly_delta(C, zk, lo + (int64_t)j);
                dlane = d < dlane ? d : dlane;
            }
        }
        dmin = wave_min_i64(dlane);
    }
    // kRegChunk = 0 evaluates the weights in groups of kGroup independent exponentials (their
    // latencies overlap); they are still added one by one in value order
    constexpr uint32_t kGroup = 4;
    // exp(-beta * (dE - dmin)); in 32-bit mode the difference is formed in 32 bits (it fits)
    auto weight = [&](uint32_t j) -> double {
        double x;
        if (linear) {
            const Acc g = slope * (Acc)(from_top ? W32 - 1u - j : j);
            x = sizeof(Acc) == 4 ? (double)(uint32_t)g : (double)(int64_t)g;
        } else {
            const int64_t d = poly_delta(C, zk, lo + (int64_t)j);
            x = sizeof(Acc) == 4 ? (double)(int32_t)((uint32_t)d - (uint32_t)dmin) : (double)(d - dmin);
        }
        return exp_nonpos(-(beta * x));
    };

    // Cold draws over wide ranges: a lane whose smallest x gives beta x >= 746 holds only weights
    // of exactly 0 (its other values have larger x, and the rounded products beta x do not
    // decrease), as R37 uses.  When the lanes holding a nonzero weight are contiguous and hold at
    // most kColdPasses * 64 values, only those values are evaluated, one per lane and 64 at a time,
    // with the same weights: the values outside add nothing to any cumulative sum, so the first
    // value whose cumulative weight exceeds U * total is the same one up to the order of the
    // additions (here the DPP scan of each pass, then the passes).  Returns false otherwise.
    constexpr uint32_t kColdPasses = 4;
    auto cold_draw = [&](int64_t &v) -> bool {
        bool live = false;
        if (j0 < W32) {
            double xl;
            if (linear) {
                // the lane's value nearest the minimising end
                const uint32_t jn = from_top ? (j0 + c - 1u < W32 ? j0 + c - 1u : W32 - 1u) : j0;
                const Acc g = slope * (Acc)(from_top ? W32 - 1u - jn : jn);
                xl = sizeof(Acc) == 4 ? (double)(uint32_t)g : (double)(int64_t)g;
            } else {
                xl = sizeof(Acc) == 4 ? (double)(int32_t)((uint32_t)dlane - (uint32_t)dmin) : (double)(dlane - dmin);
            }
            live = !(beta * xl >= 746.0);   // a NaN product counts as live
        }
        const uint64_t lmask = __ballot(live);
        if (lmask == 0) return false;
        const int first = __ffsll((unsigned long long)lmask) - 1;
        const uint64_t runs = lmask >> first;
        const uint32_t nlive = (uint32_t)__popcll(lmask);
        const uint32_t jA = (uint32_t)first * c;
        const uint32_t jE = jA + nlive * c < W32 ? jA + nlive * c : W32;
        if ((runs & (runs + 1)) != 0 || jE - jA > kColdPasses * (uint32_t)kWave) return false;   // uniform
        double incl[kColdPasses], ptot[kColdPasses];
#pragma unroll
        for (uint32_t p = 0; p < kColdPasses; ++p) {
            incl[p] = 0.0;
            ptot[p] = 0.0;
            if (jA + p * kWave < jE) {   // uniform
                const uint32_t j = jA + p * kWave + (uint32_t)lane;
                const double wv = weight(j < jE ? j : jE - 1u);
                incl[p] = wave_scan_rows(j < jE ? wv : 0.0, cy);
                ptot[p] = __longlong_as_double((long long)lane_read64((uint64_t)__double_as_longlong(incl[p]), kWave - 1));
            }
        }
        double total = 0.0;
#pragma unroll
        for (uint32_t p = 0; p < kColdPasses; ++p) total += ptot[p];
        const double thr = U * total;
        double carry = 0.0;
#pragma unroll
        for (uint32_t p = 0; p < kColdPasses; ++p) {
            if (jA + p * kWave < jE) {
                const uint32_t j = jA + p * kWave + (uint32_t)lane;
                const uint64_t hm = __ballot(j < jE && carry + incl[p] > thr);
                if (hm) {
                    v = lo + (int64_t)(jA + p * kWave) + (int64_t)(__ffsll((unsigned long long)hm) - 1);
                    return true;
                }
                carry += ptot[p];
            }
        }
        v = lo + W - 1;   // rounding left no value past the threshold
        return true;
    };

    constexpr int kR = kRegChunk > 0 ? kRegChunk : 1;
    double w[kR];
    double lane_sum = 0.0;
    // Linear dE, eight or more values per lane: once beta |a1| 64 >= 745.2, every value at
    // distance 64 or more from the minimising end weighs exactly 0 (exp_nonpos of an argument at
    // or below -745.2 is 0, and the rounded products beta |a1| d grow with d).  Lane d then
    // evaluates the weight of the value at distance d, and each slot takes its weight from that
    // lane: one exponential per lane instead of kRegChunk, the same numbers.  (With two values
    // per lane the exchange costs more than the exponential it saves: measured slower.)
    constexpr bool kGather = kRegChunk >= 8;
    const bool gather = kGather && linear && beta * ((double)slope * 64.0) >= 745.2;
    if (kGather && gather) {
        const uint32_t dl = (uint32_t)lane < W32 ? (uint32_t)lane : W32 - 1u;
        const double wl = weight(from_top ? W32 - 1u - dl : dl);
        const uint32_t lo32 = (uint32_t)__double_as_longlong(wl);
        const uint32_t hi32 = (uint32_t)((uint64_t)__double_as_longlong(wl) >> 32);
#pragma unroll
        for (int i = 0; i < kR; ++i) {
            const uint32_t j = j0 + (uint32_t)i;
            const bool valid = (uint32_t)i < c && j < W32;
            const uint32_t d = from_top ? W32 - 1u - j : j;
            const int src = (int)((valid && d < (uint32_t)kWave ? d : 0u) << 2);
            const uint64_t bits = ((uint64_t)(uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)hi32) << 32) |
                                  (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)lo32);
            w[i] = (valid && d < (uint32_t)kWave) ? __longlong_as_double((long long)bits) : 0.0;
            lane_sum = i == 0 ? w[0] : lane_sum + w[i];
        }
    } else if (kRegChunk > 0) {
        if constexpr (kRegChunk >= 8) {
            int64_t vc;
            if (cold_draw(vc)) return vc;
        }
#pragma unroll
        for (int i = 0; i < kR; ++i) {
            // evaluated for every slot (at a clamped index past the range) so that the exps of a
            // lane are independent instructions; slots past the range or the chunk weigh zero
            const uint32_t j = j0 + (uint32_t)i;
            const double wv = weight(j < W32 ? j : W32 - 1u);
            w[i] = ((uint32_t)i < c && j < W32) ? wv : 0.0;
            lane_sum = i == 0 ? w[0] : lane_sum + w[i];
        }
    } else {
        int64_t vc;
        if (cold_draw(vc)) return vc;
        for (uint32_t i = 0; i < c; i += kGroup) {
            double wv[kGroup];
#pragma unroll
            for (uint32_t u = 0; u < kGroup; ++u) {
                const uint32_t j = j0 + i + u;
                const double x = weight(j < W32 ? j : W32 - 1u);
                wv[u] = (i + u < c && j < W32) ? x : 0.0;   // adding +0.0 leaves the sum unchanged
            }
#pragma unroll
            for (uint32_t u = 0; u < kGroup; ++u) lane_sum += wv[u];
        }
    }
    const double incl = wave_scan_rows(lane_sum, cy);
    const double total = __longlong_as_double((long long)lane_read64((uint64_t)__double_as_longlong(incl), kWave - 1));
    const double before = wave_shift_up1_zero(incl, cy);
    const double thr = U * total;

    int32_t hit = -1;
    if (kRegChunk > 0) {
        // C_v = before + (running in-block sum); a slot past the range adds zero and never passes
        double run = 0.0;
#pragma unroll
        for (int i = 0; i < kR; ++i) {
            run = i == 0 ? w[0] : run + w[i];
            const bool pass = (uint32_t)i < c && j0 + (uint32_t)i < W32 && before + run > thr;
            hit = (hit < 0 && pass) ? i : hit;
        }
    } else {
        // The drawn value lies in the first block (lane) whose last value passes the threshold:
        // a block's cumulative weights never decrease, and the last one is before + lane_sum (the
        // same additions in the same order).  Only that block is walked again, 64 values at a
        // time: one weight per lane, then every lane forms the block's running sum up to its own
        // value in value order (adding +0.0 for the later values leaves it unchanged).
        const uint64_t bmask = __ballot(j0 < W32 && before + lane_sum > thr);
        if (bmask == 0) return lo + W - 1;
        const int L = __ffsll((unsigned long long)bmask) - 1;
        const double bL = __longlong_as_double((long long)lane_read64((uint64_t)__double_as_longlong(before), L));
        const uint32_t jL = (uint32_t)L * c;
        const uint32_t nL = c < W32 - jL ? c : W32 - jL;
        double carry = 0.0;   // running sum of the block's values before this part
        for (uint32_t p0 = 0; p0 < nL; p0 += kWave) {
            const uint32_t m = nL - p0 < (uint32_t)kWave ? nL - p0 : (uint32_t)kWave;
            const uint32_t jl = jL + p0 + ((uint32_t)lane < m ? (uint32_t)lane : m - 1u);
            const double wl = weight(jl);
            double run = carry;
            for (uint32_t t = 0; t < m; ++t) {
                const double wt = __longlong_as_double((long long)lane_read64((uint64_t)__double_as_longlong(wl), (int)t));
                run += t <= (uint32_t)lane ? wt : 0.0;
            }
            const uint64_t hm = __ballot((uint32_t)lane < m && bL + run > thr);
            if (hm) return lo + (int64_t)(jL + p0) + (int64_t)(__ffsll((unsigned long long)hm) - 1);
            carry = __longlong_as_double((long long)lane_read64((uint64_t)__double_as_longlong(run), (int)(m - 1)));
        }
        return lo + (int64_t)jL + (int64_t)nL - 1;   // the block's last value passes (not reached)
    }
    const uint64_t mask = __ballot(hit >= 0);
    if (mask == 0) return lo + W - 1;
    const int src = __ffsll((unsigned long long)mask) - 1;
    return lo + (int64_t)src * (int64_t)c + (int64_t)(int32_t)lane_read32((uint32_t)hit, src);
}

// Optimal transition (Sec. 3.3.3): the value of smallest dE over the whole range (z_k itself, with
// dE = 0, included), ties to the smallest value.
template <int kMaxE, typename Acc>
__device__ __forceinline__ int64_t argmin_range(const Coeffs<kMaxE, Acc> &C, int64_t lo, int64_t W,
                                                int64_t zk, int lane, int64_t &dbest) {
    int64_t best = INT64_MAX;
    int32_t bv = INT32_MAX;
    for (int64_t i = lane; i < W; i += kWave) {
        const int64_t v = lo + i;
        const int64_t d = poly_delta(C, zk, v);
        if (d < best) {
            best = d;
            bv = (int32_t)v;
        }
    }
    dbest = wave_min_i64(best);
    return wave_min_i32(best == dbest ? bv : INT32_MAX);
}

// Optimal transition over a wide range, exact by construction.  With p(v) = sum_m a_m v^m (m <= 4:
// Sec. 3.3.3 restricts the rule to energy differences of degree at most four), dE(v) = p(v) -
// p(z_k).  The forward differences D1(v) = p(v+1) - p(v), D2(v) = D1(v+1) - D1(v) and D3(v) =
// D2(v+1) - D2(v) are integer polynomials of degree 3, 2 and 1 in v, and D3 is monotone.  An
// integer sequence that is monotone on a piece changes sign at most once there, at a point a
// 64-way search finds exactly.  D3's sign change splits [lo, hi] into at most two pieces on each
// of which D2 is monotone; D2's sign changes split those into at most four pieces on which D1 is
// monotone.  Where D1 does not decrease, p falls until the first v with D1(v) >= 0 and does not
// fall after it, so that v is the piece's smallest minimiser; where D1 does not increase, p's
// minimum over the piece is at one of its ends.  The smallest minimiser over the range is the
// lexicographic (dE, v) minimum over these points and the piece ends.
//
// The differences are evaluated as polynomials in 64-bit ring arithmetic.  The energy bound gives
// |a_m| M^m < 2^62 with M = max(|lo|, |hi|), and a range of more than 64 values has M >= 32, so for
// every v of the range |D1| < 2^62 * 10 / M, |D2| < 2^62 * 20 / M^2 and |D3| < 2^62 * 30 / M^3:
// the ring results are the integers themselves.

// D_order(v), order 1..3, from the true coefficients a[1..4] (as ring elements)
__device__ __forceinline__ int64_t forward_difference(const uint64_t *a, int order, int64_t v) {
    const uint64_t x = (uint64_t)v, x2 = x * x, x3 = x2 * x;
    uint64_t r;
    if (order == 1)
        r = a[1] + a[2] * (2 * x + 1) + a[3] * (3 * x2 + 3 * x + 1) + a[4] * (4 * x3 + 6 * x2 + 4 * x + 1);
    else if (order == 2)
        r = 2 * a[2] + a[3] * (6 * x + 6) + a[4] * (12 * x2 + 24 * x + 14);
    else
        r = 6 * a[3] + a[4] * (24 * x + 36);
    return (int64_t)r;
}

// The smallest v in [x0, x1] with dir * D_order(v) >= 0, or x1 + 1 if there is none; dir * D_order
// must not decrease on [x0, x1].  Wave-uniform arguments; each round the 64 lanes test the last
// point of 64 equal blocks and the range shrinks to the first block that holds the answer (a range
// of 2^33 values needs six rounds).
__device__ __forceinline__ int64_t first_nonnegative(const uint64_t *a, int order, int dir, int64_t x0,
                                                     int64_t x1, int lane) {
    int64_t b0 = x0, b1 = x1;
    for (int round = 0; round < 8 && b1 - b0 + 1 > kWave; ++round) {
        const int64_t step = (b1 - b0 + kWave) / kWave;   // ceil(len / 64)
        const int64_t s = b0 + (int64_t)lane * step;
        const int64_t e = s + step - 1 < b1 ? s + step - 1 : b1;
        const bool hit = s <= b1 && (int64_t)dir * forward_difference(a, order, e) >= 0;
        const uint64_t mask = __ballot(hit);
        if (mask == 0) return x1 + 1;
        const int64_t j = __ffsll((unsigned long long)mask) - 1;
        const int64_t nb0 = b0 + j * step;
        b1 = nb0 + step - 1 < b1 ? nb0 + step - 1 : b1;
        b0 = nb0;
    }
    const int64_t v = b0 + lane;
    const bool hit = v <= b1 && (int64_t)dir * forward_difference(a, order, v) >= 0;
    const uint64_t mask = __ballot(hit);
    return mask == 0 ? x1 + 1 : b0 + (__ffsll((unsigned long long)mask) - 1);
}

template <int kMaxE, typename Acc>
__device__ __forceinline__ int64_t argmin_wide(const Coeffs<kMaxE, Acc> &C, int64_t lo, int64_t W,
                                               int64_t zk, int lane, int64_t &dbest) {
    const int64_t hi = lo + W - 1;
    uint64_t a[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int m = 1; m <= (kMaxE < 4 ? kMaxE : 4); ++m) a[m] = (uint64_t)to_i64<Acc>(C.a[m]);
    // candidates: the range's ends; for each piece [y0, y1] of D1's index range on which D1 is
    // monotone, the piece's ends (p over [y0, y1 + 1]) and, where D1 does not decrease, its first
    // point with D1 >= 0
    int64_t cand = lo;
    int nc = 0;
    auto add = [&](int64_t v) {
        v = v > hi ? hi : v;
        if (nc == lane) cand = v;
        ++nc;
    };
    auto piece = [&](int64_t y0, int64_t y1, int dir1) {
        add(y0);
        add(y1 + 1);
        if (dir1 > 0) add(first_nonnegative(a, 1, 1, y0, y1, lane));
    };
    add(lo);
    add(hi);
    // D3 is linear with slope 24 a4: its direction on the whole range
    const int d3 = (int64_t)a[4] >= 0 ? 1 : -1;
    const int64_t z3 = first_nonnegative(a, 3, d3, lo, hi, lane);
    // D3 has sign -d3 (strictly) on [lo, z3 - 1] and sign d3 (or is 0) on [z3, hi], so D2 is
    // monotone with direction -d3 on [lo, z3] and d3 on [z3, hi]; each is split where D2 changes
    // sign, giving the pieces where D1 is monotone
    const int64_t q0[2] = {lo, z3};
    const int64_t q1[2] = {z3 <= hi ? z3 : hi, hi};
    const int qd[2] = {-d3, d3};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        if (q0[i] > q1[i] || (i == 0 && z3 == lo)) continue;
        const int64_t z2 = first_nonnegative(a, 2, qd[i], q0[i], q1[i], lane);
        if (z2 > q0[i]) piece(q0[i], z2 <= q1[i] ? z2 : q1[i], -qd[i]);   // D2 of sign -qd
        if (z2 <= q1[i]) piece(z2, q1[i], qd[i]);                           // D2 of sign qd, or 0
    }
    int64_t best = INT64_MAX;
    int32_t bv = INT32_MAX;
    if (lane < nc) {
        best = poly_delta(C, zk, cand);
        bv = (int32_t)cand;
    }
    dbest = wave_min_i64(best);
    return wave_min_i32(best == dbest ? bv : INT32_MAX);
}

// expm1(x) for x <= 0 (the closed-form heat bath's expm1(-c W)).  Below -40, e^x is under half an
// ulp of 1 and the value is -1 exactly.  On [-0.35, 0] the Taylor series of e^x - 1 to x^14 (error
// below 2^-60 relative); otherwise e^x - 1, which cancels nothing because e^x <= 0.71.
__device__ __forceinline__ double expm1_nonpos(double x) {
    if (x < -40.0) return -1.0;
    if (x < -0.35) return exp_nonpos(x) - 1.0;
    // Horner on 1/k!, k = 14 .. 2, then x + x^2 (...)
    double p = 1.0 / 87178291200.0;            // 1/14!
    p = fma(p, x, 1.0 / 6227020800.0);         // 1/13!
    p = fma(p, x, 1.0 / 479001600.0);          // 1/12!
    p = fma(p, x, 1.0 / 39916800.0);           // 1/11!
    p = fma(p, x, 1.0 / 3628800.0);            // 1/10!
    p = fma(p, x, 1.0 / 362880.0);             // 1/9!
    p = fma(p, x, 1.0 / 40320.0);              // 1/8!
    p = fma(p, x, 1.0 / 5040.0);               // 1/7!
    p = fma(p, x, 1.0 / 720.0);                // 1/6!
    p = fma(p, x, 1.0 / 120.0);                // 1/5!
    p = fma(p, x, 1.0 / 24.0);                 // 1/4!
    p = fma(p, x, 1.0 / 6.0);                  // 1/3!
    p = fma(p, x, 0.5);                        // 1/2!
    return fma(p * x, x, x);
}

// log1p(y) for -1 < y <= 0 (the closed-form heat bath's log1p(U m)).  u = 1 + y rounded; log(u)
// from u = f 2^e with f in [sqrt(1/2), sqrt(2)) and log f = 2 atanh(s), s = (f - 1)/(f + 1),
// |s| <= 0.1716, by its odd series to s^21 (error below 2^-62 relative); the rounding of u is
// put back to first order, log1p(y) = log(u) + (y - (u - 1)) / u (Kahan's correction).
__device__ __forceinline__ double log1p_nonpos(double y) {
    if (y == 0.0) return 0.0;
    if (y <= -1.0) return -__builtin_huge_val();
    const double u = 1.0 + y;
    const double corr = (y - (u - 1.0)) * __builtin_amdgcn_rcp(u);
    int e = __builtin_amdgcn_frexp_exp(u);
    double f = __builtin_amdgcn_frexp_mant(u);  // [0.5, 1)
    if (f < 0.70710678118654752) {
        f = f + f;
        e -= 1;
    }
    const double s = (f - 1.0) / (f + 1.0);
    const double s2 = s * s;
    double r = 1.0 / 21.0;
    r = fma(r, s2, 1.0 / 19.0);
    r = fma(r, s2, 1.0 / 17.0);
    r = fma(r, s2, 1.0 / 15.0);
    r = fma(r, s2, 1.0 / 13.0);
    r = fma(r, s2, 1.0 / 11.0);
    r = fma(r, s2, 1.0 / 9.0);
    r = fma(r, s2, 1.0 / 7.0);
    r = fma(r, s2, 1.0 / 5.0);
    r = fma(r, s2, 1.0 / 3.0);
    const double ln2_hi = 0.6931471803691238;    // ln 2 rounded to 32 bits: e * ln2_hi is exact
    const double ln2_lo = 1.9082149292705877e-10;  // ln 2 - ln2_hi
    const double ed = (double)e;
    const double two_s = s + s;
    // log u = e ln2_hi + (2 s + (2 s s^2 r + e ln2_lo)) + corr
    return fma(ed, ln2_hi, two_s + (fma(two_s * s2, r, ed * ln2_lo) + corr));
}

// Heat bath for a variable whose energy difference is linear, dE(v) = a (v - z_k) (Sec. 3.3.2,
// multilinear case): the inverse of the cumulative distribution in O(1).  Index i = v - lo has
// probability proportional to exp(-beta a i); with c = beta |a| and g(q) = -log1p(q expm1(-c W)) / c
// the paper's x = -(T/a) ln[1 - U (1 - exp(-a W / T))] is g(U) for a > 0 and W - g(1 - U) for a < 0
// (the same value without overflowing exp(c W)); v = lo + ceil(x) - 1, clamped to the box.  a = 0
// or beta = 0 is the uniform distribution, drawn from x1 by a multiply-high.  Wave-uniform.
// expm1 and log1p are the functions above (about an ulp, like the host library); a last-bit
// difference moves a draw only when x lies within a few ulps of an integer.
__device__ __forceinline__ int64_t heat_bath_closed(int64_t a, int64_t lo, int64_t W, double beta, double U,
                                                    uint32_t x1) {
    const double c = beta * (double)(a < 0 ? -a : a);
    if (a == 0 || !(c > 0.0)) return lo + (int64_t)(((uint64_t)x1 * (uint64_t)W) >> 32);
    const double Wd = (double)W;
    const double m = expm1_nonpos(-(c * Wd));
    double x;
    if (a > 0)
        x = -log1p_nonpos(U * m) / c;
    else
        x = Wd + log1p_nonpos((1.0 - U) * m) / c;
    if (!(x > 0.0)) return lo;
    if (x >= Wd) return lo + W - 1;
    return lo + (int64_t)ceil(x) - 1;
}

// ------------------------------------------------------------------------------------------------
// The annealing kernel.
//
// G = A.win_waves waves per replica.  G = 1: every wave of the workgroup is an independent replica.
// G > 1: the workgroup is one replica whose state is shared in LDS; in each window of the schedule
// wave g updates the window's g-th variable, and a barrier closes the window.  The variables of a
// window share no term, so this equals the sequential index-order sweep exactly.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ void window_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// What one replica's sweeps need (shared by the plain and the batched kernels).
struct ReplicaCtx {
    DevProblem P;
    const double *beta;
    int32_t n_sweeps, s_begin, s_end;
    uint32_t key0, key1, instance_id, read;
    double otm_r;
    int32_t otm_enum_max;   // widest range whose optimal transition is enumerated
    const SchedRec *sched;  // this wave's schedule slots (window-major for one wave)
    int32_t n_win;
    bool shared;            // the replica's waves cooperate (barrier after each window)
    bool active;            // false: an idle team that only keeps the workgroup's barriers
    uint64_t *trace;        // this read's per-sweep hash words (s_end - s_begin), or nullptr
    int64_t *c1;            // dense form: this replica's coefficient cache in LDS, or nullptr
};

// Initial state (given, or uniform on each box, Sec. 3.1) written by threads tid, tid+nthr, ...
template <typename ZT>
__device__ __forceinline__ void init_state(const DevProblem &P, ZT *z, const int32_t *zi, uint32_t read,
                                           uint32_t inst, uint32_t key0, uint32_t key1, int tid, int nthr) {
    const int32_t n = P.n;
    if (zi) {
        if ((const void *)zi != (const void *)z)
            for (int32_t k = tid; k < n; k += nthr) z[k] = (ZT)zi[k];
    } else {
        for (int32_t k = tid; k < n; k += nthr) {
            uint32_t x0 = (uint32_t)k, x1 = 0xFFFFFFFFu, x2 = read, x3 = inst;
            philox4x32_10(x0, x1, x2, x3, key0, key1);
            const VarRec vr = P.var[k];
            z[k] = (ZT)(vr.lo + (int32_t)(((uint64_t)x0 * (uint64_t)(uint32_t)vr.width) >> 32));
        }
    }
}

// This wave's share of E(z) = sum_t J_t prod z (threads tid, tid+nthr, ... take the terms).
template <typename ZT>
__device__ __forceinline__ int64_t energy_part(const DevProblem &P, const ZT *z, int tid, int nthr) {
    if (P.dense) {
        // rows k = g, g + G, ... of the upper triangle, lanes across the row
        const int lane = tid & (kWave - 1), g = tid / kWave, G = nthr / kWave;
        uint64_t acc = 0;
        for (int32_t k = g; k < P.n; k += G) {
            const int64_t zk = z[k];
            if (lane == 0) acc += (uint64_t)zk * (uint64_t)(P.h[k] + P.d[k] * zk);
            uint64_t racc = 0;
            if (P.jbytes == 1) {
                const int8_t *row = (const int8_t *)P.jd + (size_t)k * P.row_stride;
                for (int32_t j = k + 1 + lane; j < P.n; j += kWave) racc += (uint64_t)(int64_t)row[j] * (uint64_t)(int64_t)z[j];
            } else {
                const int32_t *row = (const int32_t *)P.jd + (size_t)k * P.row_stride;
                for (int32_t j = k + 1 + lane; j < P.n; j += kWave) racc += (uint64_t)(int64_t)row[j] * (uint64_t)(int64_t)z[j];
            }
            acc += racc * (uint64_t)zk;
        }
        return (int64_t)wave_sum_u64(acc);
    }
    uint64_t eacc = 0;
    for (int32_t t = tid; t < P.n_terms; t += nthr) {
        uint64_t prod = (uint64_t)P.t_coef[t];
        for (int32_t f = P.t_off[t]; f < P.t_off[t + 1]; ++f) prod *= (uint64_t)(int64_t)z[P.t_var[f]];
        eacc += prod;
    }
    return (int64_t)wave_sum_u64(eacc);
}

// Sweeps [s_begin, s_end) of one replica (index order, Sec. 3.1): this wave's slots of the
// schedule.  Returns the sum of the energy changes this wave applied.
template <int kRule, bool kStateInLds, int kRegChunk, int kMaxE, typename Acc, typename ZT>
__device__ __forceinline__ int64_t sweep_replica(const ReplicaCtx &R, ZT *z, int lane) {
    const DevProblem &P = R.P;
    const int32_t n_win = R.n_win;
    const SchedRec *mine = R.sched;
    int64_t E = 0;
    uint64_t H = 0;   // change of the state hash in this sweep by this wave's moves (tracing)
    ScanCarry cy;
    if (!R.active) {
        if (R.shared)
            for (int32_t s = R.s_begin; s < R.s_end; ++s)
                for (int32_t w = 0; w < n_win; ++w) window_barrier();
        return 0;
    }
    for (int32_t s = R.s_begin; s < R.s_end; ++s) {
        const double beta = R.beta[s];
        const double r_opt =
            R.otm_r >= 0.0 ? R.otm_r : (R.n_sweeps > 1 ? (double)s / (double)(R.n_sweeps - 1) : 0.0);
        for (int32_t wb = 0; wb < n_win; wb += kWave) {
            // per block of 64 windows: lane j holds this wave's slot of window wb+j and its draws
            const int32_t wl = wb + lane;
            SchedRec sl;
            if (wl < n_win) {
                sl = mine[wl];
            } else {
                sl.k = -1;
                sl.lo = 0;
                sl.width = 1;
                sl.row = 0;
                sl.deg = 0;
                sl.emask = 0;
            }
            uint32_t x0 = (uint32_t)sl.k, x1 = (uint32_t)s, x2 = R.read, x3 = R.instance_id;
            philox4x32_10(x0, x1, x2, x3, R.key0, R.key1);
            // U in [0, 1) from words 2 and 3, formed once per lane for its window
            const double Ul = (double)((((uint64_t)x2 << 32) | x3) >> 11) * 0x1p-53;
            const int32_t wend = n_win - wb < kWave ? n_win - wb : kWave;
            // first chunk of the next slot's incidence records (the dense-form Metropolis variant,
            // kRegChunk = 1: of its coupling row, with h_k and d_k), loaded one window ahead
            IncRec nrec;
            uint64_t ncoef;
            int64_t nd = 0;
            int32_t nrow = 0, ndeg = 0;   // the prefetched slot's row and row length
            auto prefetch = [&](int32_t jj) {
                nrow = (int32_t)lane_read32((uint32_t)sl.row, jj);
                ndeg = (int32_t)lane_read32((uint32_t)sl.deg, jj);
                if (kRule == SA_METROPOLIS && kRegChunk == 1) {
                    int4 q;
                    if (R.c1)
                        prefetch_dense_col(P, (int32_t)lane_read32((uint32_t)sl.k, jj), lane, q, ncoef, nd);
                    else
                        prefetch_dense(P, (int32_t)lane_read32((uint32_t)sl.k, jj), lane, q, ncoef, nd);
                    nrec.meta = (uint32_t)q.x;
                    nrec.o[0] = q.y;
                    nrec.o[1] = q.z;
                    nrec.o[2] = q.w;
                } else {
                    load_record(P, nrow, ndeg, 0, lane, nrec, ncoef);
                }
            };
            // next(): issues the next slot's prefetch where the rule has finished with the
            // current records (the closed-form heat bath: once its coefficients are formed)
            auto visit = [&](int32_t j, const IncRec &crec, uint64_t ccoef, int64_t cd, int32_t row, int32_t deg,
                             auto &&next) {
                const int32_t k = (int32_t)lane_read32((uint32_t)sl.k, j);
                if (k < 0) next();
                if (k >= 0) {
                    const int64_t lo = (int32_t)lane_read32((uint32_t)sl.lo, j);
                    const int64_t W = (int32_t)lane_read32((uint32_t)sl.width, j);
                    const uint32_t r0 = lane_read32(x0, j), r1 = lane_read32(x1, j);
                    const double U = __longlong_as_double((long long)lane_read64((uint64_t)__double_as_longlong(Ul), j));
                    const int64_t zk = (int64_t)(int32_t)uni32((uint32_t)z[k]);
                    int64_t v, d;
                    bool accept;
                    if (kRule == SA_METROPOLIS) {
                        v = lo + (int64_t)(((uint64_t)r1 * (uint64_t)(W - 1)) >> 32);
                        if (v >= zk) v += 1;
                        // (Metropolis kernels are built with kMaxE = 1 for any problem: the
                        // variable's own exponents decide)
                        if (R.c1) {
                            // dense form with the coefficient cache: dE in O(1)
                            const Acc a1 = (Acc)(uint64_t)R.c1[k];
                            const Acc dd = kRegChunk == 1 ? (Acc)cd : (Acc)P.d[k];
                            d = to_i64<Acc>(a1 * (Acc)(v - zk) + dd * ((Acc)v * (Acc)v - (Acc)zk * (Acc)zk));
                        } else {
                            d = direct_delta<Acc, ZT, kRegChunk == 1>(P, z, k, row, deg, zk, v, lane, crec, ccoef, cd,
                                                                      (lane_read32(sl.emask, j) & ~2u) == 0);
                        }
                        accept = metropolis_accept(d, beta, U);
                    } else if (kRule == SA_HEAT_BATH || kRule == SA_HEAT_BATH_CLOSED) {
                        Coeffs<kMaxE, Acc> C;
                        const uint32_t em = lane_read32(sl.emask, j);
                        row_coeffs<kMaxE, Acc, ZT>(P, z, k, row, deg, em, lane, crec, ccoef, C, R.c1);
                        next();
                        // closed form where dE is linear in the new value (no exponent above one)
                        const bool linear = kMaxE == 1 || (em & ~2u) == 0;
                        if (kRule == SA_HEAT_BATH_CLOSED && linear)
                            v = heat_bath_closed(to_i64<Acc>(C.a[1]), lo, W, beta, U, r1);
                        else
                            v = heat_bath_pick<kRegChunk, kMaxE, Acc>(C, lo, W, zk, beta, U, lane, linear, cy);
                        d = poly_delta(C, zk, v);
                        accept = true;
                    } else {
                        if ((double)r0 * 0x1p-32 < r_opt) {
                            Coeffs<kMaxE, Acc> C;
                            const uint32_t em = lane_read32(sl.emask, j);
                            row_coeffs<kMaxE, Acc, ZT>(P, z, k, row, deg, em, lane, crec, ccoef, C, R.c1);
                            if (kMaxE == 1 || (em & ~2u) == 0) {
                                // dE = a1 (v - z_k): the lowest value for a1 >= 0 (every value ties
                                // when a1 = 0), the highest for a1 < 0
                                const int64_t a1 = to_i64<Acc>(C.a[1]);
                                v = a1 >= 0 ? lo : lo + W - 1;
                                d = to_i64<Acc>(C.a[1] * (Acc)(v - zk));
                            } else if (kRegChunk == 1 && W > R.otm_enum_max && W > kWave)
                                v = argmin_wide<kMaxE, Acc>(C, lo, W, zk, lane, d);
                            else
                                v = argmin_range<kMaxE, Acc>(C, lo, W, zk, lane, d);
                        } else {
                            v = lo + (int64_t)(((uint64_t)r1 * (uint64_t)(W - 1)) >> 32);
                            if (v >= zk) v += 1;
                            d = direct_delta<Acc, ZT, false>(P, z, k, row, deg, zk, v, lane, crec, ccoef, cd,
                                                      (lane_read32(sl.emask, j) & ~2u) == 0);
                        }
                        accept = metropolis_accept(d, beta, U);
                    }
                    if (accept && v != zk) {
                        z[k] = (ZT)v;  // every lane stores the same value
                        E += d;
                        if (R.trace) H += hash_word(k, v) - hash_word(k, zk);
                        if (R.c1) {
                            const int4 jcol = make_int4((int)crec.meta, crec.o[0], crec.o[1], crec.o[2]);
                            dense_cache_update(P, R.c1, k, v - zk, lane,
                                               kRule == SA_METROPOLIS && kRegChunk == 1 ? &jcol : nullptr);
                        }
                        if (!R.shared) state_write_fence<kStateInLds>();
                    }
                }
                if (R.shared) window_barrier();
            };
            prefetch(0);
            for (int32_t j = 0; j < wend; ++j) {
                if constexpr (kRule == SA_HEAT_BATH_CLOSED) {
                    // the loads overwrite the records in place: the draw hides their latency, and
                    // no registers are copied between slots (measured faster for this rule only)
                    visit(j, nrec, ncoef, nd, nrow, ndeg, [&] { prefetch(j + 1 < wend ? j + 1 : j); });
                } else {
                    const IncRec crec = nrec;
                    const uint64_t ccoef = ncoef;
                    const int64_t cd = nd;
                    const int32_t crow = nrow, cdeg = ndeg;
                    // unconditional (the last slot loads its own records again), so that the
                    // records need no copy on a path without the prefetch
                    prefetch(j + 1 < wend ? j + 1 : j);
                    visit(j, crec, ccoef, cd, crow, cdeg, [] {});
                }
            }
        }
        if (R.trace) {
            if (lane == 0) atomicAdd((unsigned long long *)&R.trace[s - R.s_begin], (unsigned long long)H);
            H = 0;
        }
    }
    return E;
}

// ------------------------------------------------------------------------------------------------
// Plain launch: one instance, n_reads replicas.
// ------------------------------------------------------------------------------------------------
// kThreads: 512 (up to 8 waves per replica) or 1024 (16 waves; fewer registers per lane, so only
// the variants that need no more than 128 VGPRs are built that way).
// The generic-record Metropolis and OTM variants (the HUIO workloads) are held to 128 VGPRs, four
// waves per SIMD: their cold paths (long terms, the wide-range argmin) would otherwise raise the
// register count past 128 and cost a wave per SIMD on every problem.
template <int kRule, bool kStateInLds, int kRegChunk, int kMaxE, typename Acc, int kThreads>
__global__ void __launch_bounds__(kThreads, (kThreads == 512 && kRegChunk == 0 && kRule != SA_HEAT_BATH &&
                                             kRule != SA_HEAT_BATH_CLOSED) ? 4 : 1)
    anneal_kernel(AnnealArgs A) {
    extern __shared__ int32_t lds_state[];
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int wave = (int)(threadIdx.x / kWave);
    const int G = A.win_waves;
    const bool shared = G > 1;
    const int read = shared ? (int)blockIdx.x : (int)blockIdx.x * A.waves_per_group + wave;
    const int g = shared ? wave : 0;
    if (read >= A.n_reads) return;  // uniform over the replica's waves; no barrier is skipped
    const DevProblem &P = A.P;
    const int32_t n = P.n;
    int32_t *z = kStateInLds ? lds_state + (shared ? 0 : (size_t)wave * n) : A.z_out + (size_t)read * n;
    const int tid = g * kWave + lane, nthr = G * kWave;  // threads of this replica

    init_state(P, z, A.z_init ? A.z_init + (size_t)read * n : nullptr, (uint32_t)read, A.instance_id,
               A.key0, A.key1, tid, nthr);
    if (shared) window_barrier();
    else state_write_fence<kStateInLds>();
    int64_t E = energy_part(P, z, tid, nthr);
    // dense form, one wave per replica, state in LDS: the coefficient cache follows the waves' states
    int64_t *c1 = nullptr;
    if (kStateInLds && A.dense_cache && !shared) {
        c1 = (int64_t *)(lds_state + (((size_t)A.waves_per_group * n + 1) & ~(size_t)1)) + (size_t)wave * n;
        dense_cache_init(P, z, c1, lane, kWave);
        state_write_fence<kStateInLds>();
    }
    uint64_t *trace = A.trace ? A.trace + (size_t)read * (size_t)(A.s_end - A.s_begin) : nullptr;
    if (trace && A.s_end > A.s_begin) {
        // the initial state's hash goes into the first sweep's word
        uint64_t h0 = 0;
        for (int32_t k = tid; k < n; k += nthr) h0 += hash_word(k, z[k]);
        h0 = wave_sum_u64(h0);
        if (lane == 0) atomicAdd((unsigned long long *)&trace[0], (unsigned long long)h0);
    }

    ReplicaCtx R;
    R.P = P;
    R.beta = A.beta;
    R.n_sweeps = A.n_sweeps;
    R.s_begin = A.s_begin;
    R.s_end = A.s_end;
    R.key0 = A.key0;
    R.key1 = A.key1;
    R.instance_id = A.instance_id;
    R.read = (uint32_t)read;
    R.otm_r = A.otm_r;
    R.otm_enum_max = A.otm_enum_max;
    R.sched = A.sched + (size_t)g * A.n_win;
    R.n_win = A.n_win;
    R.shared = shared;
    R.active = true;
    R.trace = trace;
    R.c1 = c1;
    E += sweep_replica<kRule, kStateInLds, kRegChunk, kMaxE, Acc, int32_t>(R, z, lane);

    if (shared) {
        // combine the waves' energy parts; LDS slots follow the state
        int64_t *parts = (int64_t *)(lds_state + (((size_t)n + 1) & ~(size_t)1));
        if (lane == 0) parts[g] = E;
        window_barrier();
        if (g == 0) {
            E = 0;
            for (int q = 0; q < G; ++q) E += parts[q];
        }
    }
    if (kStateInLds) {
        int32_t *zo = A.z_out + (size_t)read * n;
        for (int32_t k = tid; k < n; k += nthr) zo[k] = z[k];
    }
    if (g == 0 && lane == 0) A.e_out[read] = E;
}

// ------------------------------------------------------------------------------------------------
// Batched launch: one persistent kernel anneals many problems.  A workgroup of kBatchWaves waves
// repeatedly takes the next task from a global counter (tasks are ordered longest first).  A task
// is kBatchWaves / G_p consecutive reads of one problem p: each read is annealed by a team of G_p
// waves (G_p = 1: independent waves; G_p > 1: cooperating waves over the problem's window schedule,
// as in the plain kernel).  Rule and heat-bath chunk class are dispatched per task; the exponent
// class, integer width and state width are those of the whole batch.
// ------------------------------------------------------------------------------------------------
template <int kMaxE, typename Acc, typename ZT>
__global__ void __launch_bounds__(kBatchWaves * 64, 4) batch_kernel(BatchArgs B) {
    extern __shared__ int32_t lds_state[];
    __shared__ uint32_t task_slot;
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int wave = (int)(threadIdx.x / kWave);
    int64_t *parts = (int64_t *)(lds_state + B.parts_words);
    constexpr int kOtmE = kMaxE < 4 ? kMaxE : 4;
    for (;;) {
        if (threadIdx.x == 0) task_slot = atomicAdd(B.counter, 1u);
        window_barrier();
        const uint32_t t = task_slot;
        window_barrier();  // every wave has the task before the slot can change again
        if (t >= (uint32_t)B.n_tasks) break;  // uniform over the workgroup
        const BatchTask task = B.tasks[t];
        const BatchInst &D = B.insts[task.inst];
        const DevProblem P = D.P;
        const int G = D.team;
        const int team = wave / G, g = wave % G;
        const int32_t read_i = task.read + team;
        const bool active = read_i < D.n_reads;
        const uint32_t read = (uint32_t)read_i;
        ZT *z = (ZT *)lds_state + (size_t)team * D.slot_stride;
        const int tid = g * kWave + lane, nthr = G * kWave;
        int32_t *zo = D.z_out + (size_t)read * P.n;
        if (active) init_state(P, z, D.resume ? zo : nullptr, read, D.instance_id, D.key0, D.key1, tid, nthr);
        window_barrier();
        // a resumed replica continues from the exact energy its previous chunk wrote (the team's
        // first wave carries it); a new one sums its terms
        int64_t E = 0;
        if (active) E = D.resume ? (g == 0 ? D.e_out[read] : 0) : energy_part(P, z, tid, nthr);
        ReplicaCtx R;
        R.P = P;
        R.beta = D.beta;
        R.n_sweeps = D.n_sweeps;
        R.s_begin = D.s_begin;
        R.s_end = B.sweep_limit > 0 && B.sweep_limit < D.s_end ? B.sweep_limit : D.s_end;
        R.key0 = D.key0;
        R.key1 = D.key1;
        R.instance_id = D.instance_id;
        R.read = read;
        R.otm_r = -1.0;
        R.otm_enum_max = kOtmEnumMax;
        R.sched = D.sched + (size_t)g * D.n_win;
        R.n_win = D.n_win;
        R.shared = G > 1;
        R.active = active;
        R.trace = nullptr;
        R.c1 = nullptr;
        if (D.rule == SA_METROPOLIS) {
            E += sweep_replica<SA_METROPOLIS, true, 0, 1, Acc, ZT>(R, z, lane);
        } else if (D.rule == SA_HEAT_BATH) {
            switch (D.chunk) {
                case 1: E += sweep_replica<SA_HEAT_BATH, true, 1, kMaxE, Acc, ZT>(R, z, lane); break;
                case 2: E += sweep_replica<SA_HEAT_BATH, true, 2, kMaxE, Acc, ZT>(R, z, lane); break;
                case 8: E += sweep_replica<SA_HEAT_BATH, true, 8, kMaxE, Acc, ZT>(R, z, lane); break;
                default: E += sweep_replica<SA_HEAT_BATH, true, 0, kMaxE, Acc, ZT>(R, z, lane); break;
            }
        } else if (D.rule == SA_HEAT_BATH_CLOSED) {
            switch (D.chunk) {
                case 1: E += sweep_replica<SA_HEAT_BATH_CLOSED, true, 1, kMaxE, Acc, ZT>(R, z, lane); break;
                case 2: E += sweep_replica<SA_HEAT_BATH_CLOSED, true, 2, kMaxE, Acc, ZT>(R, z, lane); break;
                case 8: E += sweep_replica<SA_HEAT_BATH_CLOSED, true, 8, kMaxE, Acc, ZT>(R, z, lane); break;
                default: E += sweep_replica<SA_HEAT_BATH_CLOSED, true, 0, kMaxE, Acc, ZT>(R, z, lane); break;
            }
        } else {
            E += sweep_replica<SA_OPT_METROPOLIS, true, 0, kOtmE, Acc, ZT>(R, z, lane);
        }
        if (lane == 0) parts[wave] = E;
        window_barrier();
        if (active) {
            if (g == 0 && lane == 0) {
                int64_t tot = 0;
                for (int q = 0; q < G; ++q) tot += parts[team * G + q];
                D.e_out[read] = tot;
            }
            for (int32_t k = tid; k < P.n; k += nthr) zo[k] = (int32_t)z[k];
        }
        window_barrier();  // the slots' last reads come before the next task's writes
    }
}

// Kernel entry of the plain launch.
using AnnealKernel = void (*)(AnnealArgs);

// Heat bath: the weights of ceil(W/64) <= kRegChunk values per lane stay in registers (the
// unrolled loops then cost kRegChunk steps); wider ranges recompute them (kRegChunk = 0).
template <int kRule, int kMaxE, typename Acc>
AnnealKernel pick_heat_bath_lds(int reg_chunk) {
    switch (reg_chunk) {
        case 1: return anneal_kernel<kRule, true, 1, kMaxE, Acc, 512>;
        case 2: return anneal_kernel<kRule, true, 2, kMaxE, Acc, 512>;
        case 8: return anneal_kernel<kRule, true, 8, kMaxE, Acc, 512>;
        case 32: return anneal_kernel<kRule, true, 32, kMaxE, Acc, 512>;
        default: return anneal_kernel<kRule, true, 0, kMaxE, Acc, 512>;
    }
}
template <int kRule, int kMaxE, typename Acc>
AnnealKernel pick_heat_bath_lds_16(int reg_chunk) {
    switch (reg_chunk) {
        case 1: return anneal_kernel<kRule, true, 1, kMaxE, Acc, 1024>;
        case 2: return anneal_kernel<kRule, true, 2, kMaxE, Acc, 1024>;
        default: return anneal_kernel<kRule, true, 8, kMaxE, Acc, 1024>;
    }
}

}  // namespace
}  // namespace sa
