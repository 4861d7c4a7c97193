// Drives the host-side preparation of the GPU library (csrc/sa_host.cpp: canonicalisation, the
// int64 bound, the automatic temperatures, packing, window and level schedules) on fixtures that
// reach its edges, for a build with the address and undefined-behaviour sanitizers.  Prints "ok".
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../paper_2511_17245_amd/csrc/sa_internal.h"

namespace {

int failures = 0;
void expect(bool c, const char *what) {
    if (!c) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

struct Raw {
    int32_t n;
    std::vector<int64_t> ptr{0};
    std::vector<int32_t> fac;
    std::vector<int64_t> coef;
    std::vector<int32_t> lo, hi;
    void term(int64_t c, std::vector<int32_t> v) {
        fac.insert(fac.end(), v.begin(), v.end());
        ptr.push_back((int64_t)fac.size());
        coef.push_back(c);
    }
    sa_instance inst() const { return {n, (int64_t)coef.size(), ptr.data(), fac.data(), coef.data()}; }
    sa_bounds bounds() const { return {lo.data(), hi.data()}; }
};

int prepare(const Raw &r, sa::Packed &pk, std::string &err) {
    sa_instance in = r.inst();
    sa_bounds bd = r.bounds();
    sa::Canonical c;
    int rc = sa::canonicalize(&in, &bd, c, err);
    if (rc != SA_OK) return rc;
    double bound = 0;
    rc = sa::check_int64_bound(c, err, &bound);
    if (rc != SA_OK) return rc;
    double ti = 0, tf = 0;
    if (sa::auto_temperatures(c, &ti, &tf, err) == SA_OK) {
        std::vector<double> beta(7);
        sa::geometric_betas(ti, tf, 7, beta.data());
        expect(beta[0] > 0 && beta[6] >= beta[0], "betas increase");
    }
    (void)sa::dE_fits_32(c);
    (void)sa::coefs_fit_32(c);
    return sa::pack(c, pk, err);
}

// other-factor lists of long terms: 16-byte aligned, valid indices, padded with -1 to whole int4
// (the device reads them four at a time)
void overflow_lists(const sa::Packed &pk) {
    for (const sa::IncRec &r : pk.inc) {
        const uint32_t no = r.meta >> 8;
        if (no <= 3) continue;
        const size_t at = (size_t)r.o[0], padded = (no + 3) / 4 * 4;
        expect(at % 4 == 0 && at + padded <= pk.overflow.size(), "overflow list aligned and in range");
        if (at + padded > pk.overflow.size()) continue;
        for (uint32_t f = 0; f < padded; ++f) {
            const int32_t j = pk.overflow[at + f];
            expect(f < no ? (j >= 0 && j < pk.n) : j == -1, "overflow index or pad");
        }
    }
}

void schedules(const sa::Packed &pk) {
    overflow_lists(pk);
    for (int G : {1, 2, 4, 8, 16}) {
        std::vector<sa::SchedRec> s;
        const int32_t nw = sa::build_schedule(pk, G, s);
        expect((int64_t)s.size() == (int64_t)nw * G, "schedule size");
    }
    std::vector<int32_t> start;
    std::vector<sa::SchedRec> slots;
    const int32_t nl = sa::build_levels(pk, 128, start, slots);
    expect((int32_t)start.size() == nl + 1 && start.back() == (int32_t)slots.size(), "level offsets");
    // every variable comes after the levels of its lower-index neighbours (so no two variables of
    // a level interact), and every variable that is not fixed appears exactly once
    std::vector<int32_t> lvl(pk.n, -1);
    for (int32_t l = 0; l < nl; ++l)
        for (int32_t i = start[l]; i < start[l + 1]; ++i) {
            expect(lvl[slots[i].k] == -1, "variable placed once");
            lvl[slots[i].k] = l;
        }
    for (int32_t k = 0; k < pk.n; ++k) {
        expect((lvl[k] >= 0) == (pk.var[k].width > 1), "variables that are not fixed are placed");
        if (lvl[k] < 0 || pk.dense) continue;
        const sa::VarRec &vr = pk.var[k];
        for (int32_t q = vr.row; q < vr.row + vr.deg; ++q) {
            const sa::IncRec &r = pk.inc[q];
            const uint32_t no = r.meta >> 8;
            for (uint32_t f = 0; f < no; ++f) {
                const int32_t j = no <= 3 ? r.o[f] : pk.overflow[(size_t)r.o[0] + f];
                if (j < k && lvl[j] >= 0) expect(lvl[j] < lvl[k], "lower neighbour in an earlier level");
            }
        }
    }
    if (pk.dense) return;
    // the rounds of the Metropolis / OTM quad kernel and their records' round-major copy: place
    // (r, u, lane q * 4 + l) holds incidence 4 u + l of round r's quad q, its other factors as LDS
    // byte offsets (4 n for an unused place), a zero coefficient for a long record or past the row
    std::vector<sa::SchedRec> rounds;
    int32_t n_real = 0;
    sa::build_rounds(pk, rounds, n_real);
    expect(rounds.size() % (size_t)(sa::kRoundQuads * sa::kRoundBatch) == 0, "whole batches of rounds");
    for (bool c32 : {false, true}) {
        std::vector<sa::MoRec> rec;
        std::vector<uint8_t> coef;
        sa::build_mo_records(pk, rounds, c32, rec, coef);
        const size_t nr = rounds.size() / (size_t)sa::kRoundQuads, cw = c32 ? 4 : 8;
        expect(rec.size() == nr * (size_t)sa::kMoAhead * 64 && coef.size() == rec.size() * cw, "copy size");
        const uint32_t one = (uint32_t)pk.n * 4u;
        for (size_t r = 0; r < nr; ++r)
            for (int32_t q = 0; q < sa::kRoundQuads; ++q) {
                const sa::SchedRec &s = rounds[r * (size_t)sa::kRoundQuads + (size_t)q];
                bool rest = s.k >= 0 && s.deg > 4 * sa::kMoAhead;
                for (int32_t i = 0; i < 4 * sa::kMoAhead; ++i) {
                    const size_t idx = (r * (size_t)sa::kMoAhead + (size_t)(i / 4)) * 64 + (size_t)(q * 4 + i % 4);
                    const sa::MoRec &m = rec[idx];
                    int64_t c = 0;
                    if (c32) {
                        int32_t c4;
                        std::memcpy(&c4, coef.data() + idx * cw, 4);
                        c = c4;
                    } else {
                        std::memcpy(&c, coef.data() + idx * cw, 8);
                    }
                    if (s.k < 0 || i >= s.deg) {
                        expect(c == 0 && m.zoff[0] == one && m.zoff[1] == one && m.zoff[2] == one, "zero place");
                        continue;
                    }
                    const sa::IncRec &ir = pk.inc[(size_t)s.row + (size_t)i];
                    const uint32_t no = ir.meta >> 8;
                    expect(m.meta == ir.meta, "record meta");
                    if (no > 3) {
                        rest = true;
                        expect(c == 0, "long record zero in the copy");
                        continue;
                    }
                    const int64_t want = pk.inc_coef[(size_t)s.row + (size_t)i];
                    expect(c32 ? (int32_t)c == (int32_t)want : c == want, "record coefficient");
                    for (uint32_t f = 0; f < 3; ++f)
                        expect(m.zoff[f] == (f < no ? (uint32_t)ir.o[f] * 4u : one), "factor offsets");
                }
                expect((s.pad[0] != 0) == rest, "rest flag");
            }
    }
}

}  // namespace

int main() {
    std::string err;
    // random HUIO with powers, repeated multisets, zero and cancelling coefficients, fixed variables
    std::mt19937_64 g(7);
    for (int rep = 0; rep < 20; ++rep) {
        Raw r;
        r.n = 1 + (int32_t)(g() % 60);
        for (int32_t i = 0; i < r.n; ++i) {
            const int32_t l = -(int32_t)(g() % 50);
            r.lo.push_back(l);
            r.hi.push_back(i % 7 == 3 ? l : l + (int32_t)(g() % 100));
        }
        const int m = (int)(g() % 200);
        for (int t = 0; t < m; ++t) {
            std::vector<int32_t> v(1 + g() % 5);
            for (auto &x : v) x = (int32_t)(g() % r.n);
            const int64_t c = (int64_t)(g() % 11) - 5;
            r.term(c, v);
            if (t % 9 == 0) r.term(-c, v);   // cancels the previous term
        }
        sa::Packed pk;
        const int rc = prepare(r, pk, err);
        expect(rc == SA_OK || rc == SA_ERANGE, "random problem prepares");
        if (rc == SA_OK) schedules(pk);
    }
    // long terms: the multilinear chain of degree 30 (lists of 29 other factors) and degree 17
    // with a squared factor
    for (int32_t deg : {30, 17}) {
        Raw r;
        r.n = 40;
        for (int32_t i = 0; i < r.n; ++i) {
            r.lo.push_back(-1);
            r.hi.push_back(1);
        }
        for (int32_t i = 0; i < r.n; ++i) {
            std::vector<int32_t> v;
            for (int32_t f = 0; f < deg; ++f) v.push_back((i + f) % r.n);
            if (deg == 17) v.push_back(i);
            r.term(-1, v);
        }
        sa::Packed pk;
        expect(prepare(r, pk, err) == SA_OK, "long terms prepare");
        expect(pk.max_other == (deg == 30 ? 29 : 17), "long terms keep every other factor");
        schedules(pk);
    }
    // dense QUIO (stored as a matrix) with int8 and int32 couplings
    for (int64_t jmax : {10LL, 100000LL}) {
        Raw r;
        r.n = 40;
        r.lo.assign(40, -5);
        r.hi.assign(40, 5);
        for (int32_t i = 0; i < 40; ++i)
            for (int32_t j = i; j < 40; ++j) r.term((int64_t)(g() % (2 * jmax + 1)) - jmax, {i, j});
        sa::Packed pk;
        expect(prepare(r, pk, err) == SA_OK && pk.dense, "dense problem packs as a matrix");
        schedules(pk);
    }
    // the int64 bound at its edge: |J| z^e summed just below and at 2^62
    {
        Raw r;
        r.n = 1;
        r.lo = {-(1 << 30)};
        r.hi = {(1 << 30) - 2};
        r.term(1LL << 2, {0, 0});   // 4 * 2^60 = 2^62: rejected
        sa::Packed pk;
        expect(prepare(r, pk, err) == SA_ERANGE, "bound at 2^62 is rejected");
        Raw q = r;
        q.coef[0] = 3;              // 3 * 2^60 < 2^62: accepted
        expect(prepare(q, pk, err) == SA_OK, "bound below 2^62 is accepted");
    }
    // malformed inputs
    {
        Raw r;
        r.n = 2;
        r.lo = {0, 0};
        r.hi = {1, 1};
        r.term(1, {0, 5});          // index out of range
        sa::Packed pk;
        expect(prepare(r, pk, err) == SA_EINVAL, "index out of range is rejected");
        Raw q;
        q.n = 1;
        q.lo = {0};
        q.hi = {2147483647};        // u - l above 2^31 - 2
        expect(prepare(q, pk, err) == SA_EINVAL, "range too wide is rejected");
    }
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
