// sa_host.cpp -- host-side preparation of a problem for the annealing kernels:
// validation, canonicalisation (Sec. 2), the int64 exactness bound, the automatic temperature
// range (Sec. 3.4) and the variable-major packing the kernels read.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <set>

#include "sa_internal.h"

namespace sa {

namespace {

bool fits_i64(__int128 v) { return v >= -(__int128)INT64_MAX && v <= (__int128)INT64_MAX; }

}  // namespace

int canonicalize(const sa_instance *inst, const sa_bounds *bounds, Canonical &out, std::string &err) {
    if (!inst || !bounds) {
        err = "instance and bounds are required";
        return SA_EINVAL;
    }
    const int32_t n = inst->n_vars;
    const int64_t nt = inst->n_terms;
    if (n < 1) {
        err = "n_vars must be >= 1";
        return SA_EINVAL;
    }
    if (nt < 0) {
        err = "n_terms must be >= 0";
        return SA_EINVAL;
    }
    if (!bounds->lower || !bounds->upper) {
        err = "bounds.lower and bounds.upper are required";
        return SA_EINVAL;
    }
    for (int32_t i = 0; i < n; ++i) {
        int64_t l = bounds->lower[i], u = bounds->upper[i];
        if (l > u) {
            err = "lower bound above upper bound for variable " + std::to_string(i);
            return SA_EINVAL;
        }
        if (u - l > 2147483646LL) {
            err = "range u - l exceeds 2^31 - 2 for variable " + std::to_string(i);
            return SA_EINVAL;
        }
    }
    if (nt > 0 && (!inst->term_ptr || !inst->factor_var || !inst->coef)) {
        err = "term_ptr, factor_var and coef are required when n_terms > 0";
        return SA_EINVAL;
    }
    const int64_t *tp = inst->term_ptr;
    if (nt > 0 && tp[0] != 0) {
        err = "term_ptr[0] must be 0";
        return SA_EINVAL;
    }
    for (int64_t t = 0; t < nt; ++t) {
        if (tp[t + 1] <= tp[t]) {
            err = "term " + std::to_string(t) + " has degree < 1 (constant terms are not allowed)";
            return SA_EINVAL;
        }
    }
    const int64_t nf = nt > 0 ? tp[nt] : 0;
    for (int64_t f = 0; f < nf; ++f) {
        int32_t v = inst->factor_var[f];
        if (v < 0 || v >= n) {
            err = "factor index out of range at position " + std::to_string(f);
            return SA_EINVAL;
        }
    }

    // Sort the factors of every term, then order terms by (degree, factors) and merge equal ones.
    // Terms of degree <= 2 use a packed 64-bit key (the common case for QUIO); longer terms are
    // compared factor by factor.
    std::vector<int32_t> fac(inst->factor_var, inst->factor_var + nf);
    struct ShortKey {
        uint64_t key;
        int64_t coef;
    };
    std::vector<ShortKey> shorts;
    std::vector<int64_t> longs;
    shorts.reserve((size_t)nt);
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = tp[t], b = tp[t + 1];
        std::sort(fac.begin() + a, fac.begin() + b);
        if (b - a == 1) {
            shorts.push_back({((uint64_t)1 << 62) | (uint64_t)fac[a], inst->coef[t]});
        } else if (b - a == 2) {
            shorts.push_back({((uint64_t)2 << 62) | ((uint64_t)fac[a] << 31) | (uint64_t)fac[a + 1],
                              inst->coef[t]});
        } else {
            longs.push_back(t);
        }
    }
    std::sort(shorts.begin(), shorts.end(),
              [](const ShortKey &x, const ShortKey &y) { return x.key < y.key; });
    auto long_less = [&](int64_t x, int64_t y) {
        int64_t lx = tp[x + 1] - tp[x], ly = tp[y + 1] - tp[y];
        if (lx != ly) return lx < ly;
        return std::lexicographical_compare(fac.begin() + tp[x], fac.begin() + tp[x + 1],
                                            fac.begin() + tp[y], fac.begin() + tp[y + 1]);
    };
    std::sort(longs.begin(), longs.end(), long_less);

    out = Canonical();
    out.n = n;
    out.lo.assign(bounds->lower, bounds->lower + n);
    out.hi.assign(bounds->upper, bounds->upper + n);
    out.t_off.push_back(0);
    for (size_t a = 0; a < shorts.size();) {
        size_t b = a;
        __int128 sum = 0;
        while (b < shorts.size() && shorts[b].key == shorts[a].key) sum += shorts[b++].coef;
        if (!fits_i64(sum)) {
            err = "merged coefficient overflows int64";
            return SA_ERANGE;
        }
        if (sum != 0) {
            uint64_t key = shorts[a].key;
            if ((key >> 62) == 1) {
                out.t_var.push_back((int32_t)(key & 0x7FFFFFFFu));
            } else {
                out.t_var.push_back((int32_t)((key >> 31) & 0x7FFFFFFFu));
                out.t_var.push_back((int32_t)(key & 0x7FFFFFFFu));
            }
            out.t_coef.push_back((int64_t)sum);
            out.t_off.push_back((int64_t)out.t_var.size());
        }
        a = b;
    }
    for (size_t a = 0; a < longs.size();) {
        size_t b = a;
        __int128 sum = 0;
        while (b < longs.size() && !long_less(longs[a], longs[b]) && !long_less(longs[b], longs[a]))
            sum += inst->coef[longs[b++]];
        if (!fits_i64(sum)) {
            err = "merged coefficient overflows int64";
            return SA_ERANGE;
        }
        if (sum != 0) {
            int64_t t = longs[a];
            out.t_var.insert(out.t_var.end(), fac.begin() + tp[t], fac.begin() + tp[t + 1]);
            out.t_coef.push_back((int64_t)sum);
            out.t_off.push_back((int64_t)out.t_var.size());
        }
        a = b;
    }
    return SA_OK;
}

int check_int64_bound(const Canonical &c, std::string &err, double *bound_out) {
    const __int128 limit = (__int128)1 << 62;
    __int128 total = 0;
    for (int64_t t = 0; t < c.n_terms(); ++t) {
        __int128 term = c.t_coef[t] < 0 ? -(__int128)c.t_coef[t] : (__int128)c.t_coef[t];
        for (int64_t f = c.t_off[t]; f < c.t_off[t + 1] && term < limit; ++f) {
            int32_t i = c.t_var[f];
            int64_t zm = std::max(std::llabs((long long)c.lo[i]), std::llabs((long long)c.hi[i]));
            term *= zm;
        }
        total += term;
        if (total >= limit) {
            err = "sum_t |J_t| prod max(|l|,|u|)^e reaches 2^62: energies would not be exact in int64";
            return SA_ERANGE;
        }
    }
    if (bound_out) *bound_out = (double)total;
    return SA_OK;
}

bool dE_fits_32(const Canonical &c) {
    const __int128 limit = (__int128)1 << 29;
    std::vector<__int128> per_var(c.n, 0);
    for (int64_t t = 0; t < c.n_terms(); ++t) {
        __int128 term = c.t_coef[t] < 0 ? -(__int128)c.t_coef[t] : (__int128)c.t_coef[t];
        for (int64_t f = c.t_off[t]; f < c.t_off[t + 1] && term < limit; ++f) {
            const int32_t i = c.t_var[f];
            term *= std::max(std::llabs((long long)c.lo[i]), std::llabs((long long)c.hi[i]));
        }
        if (term >= limit) return false;
        for (int64_t f = c.t_off[t]; f < c.t_off[t + 1]; ++f) {
            if (f > c.t_off[t] && c.t_var[f] == c.t_var[f - 1]) continue;
            per_var[c.t_var[f]] += term;
            if (per_var[c.t_var[f]] >= limit) return false;
        }
    }
    return true;
}

bool coefs_fit_32(const Canonical &c) {
    // per variable k: sum over the terms holding z_k of |J| * prod over the other factors of
    // zmax^e, which bounds every coefficient a_k^(m) and every partial sum of it
    const __int128 limit = (__int128)1 << 31;
    std::vector<__int128> per_var(c.n, 0);
    for (int64_t t = 0; t < c.n_terms(); ++t) {
        const __int128 absj = c.t_coef[t] < 0 ? -(__int128)c.t_coef[t] : (__int128)c.t_coef[t];
        for (int64_t f = c.t_off[t]; f < c.t_off[t + 1]; ++f) {
            if (f > c.t_off[t] && c.t_var[f] == c.t_var[f - 1]) continue;
            const int32_t k = c.t_var[f];
            __int128 b = absj;
            for (int64_t g = c.t_off[t]; g < c.t_off[t + 1] && b < limit; ++g) {
                const int32_t i = c.t_var[g];
                if (i == k) continue;
                b *= std::max(std::llabs((long long)c.lo[i]), std::llabs((long long)c.hi[i]));
            }
            if (b >= limit) return false;
            per_var[k] += b;
            if (per_var[k] >= limit) return false;
        }
    }
    return true;
}

int auto_temperatures(const Canonical &c, double *t_init, double *t_final, std::string &err) {
    // dE_max ~ max_k sum over terms holding z_k^m of |J| * prod_{other factors} zmax^e * (u_k - l_k)^m
    // dE_min ~ min |J| over the (merged, nonzero) coefficients.
    const int32_t n = c.n;
    std::vector<double> per_var(n, 0.0);
    double min_abs = INFINITY;
    for (int64_t t = 0; t < c.n_terms(); ++t) {
        const double absj = std::fabs((double)c.t_coef[t]);
        min_abs = std::min(min_abs, absj);
        const int64_t a = c.t_off[t], b = c.t_off[t + 1];
        // walk the distinct variables of the term (factors are sorted, powers are runs)
        for (int64_t f = a; f < b;) {
            int64_t g = f;
            while (g < b && c.t_var[g] == c.t_var[f]) ++g;
            const int32_t k = c.t_var[f];
            const double m = (double)(g - f);
            double prod = absj;
            for (int64_t h = a; h < b;) {
                int64_t q = h;
                while (q < b && c.t_var[q] == c.t_var[h]) ++q;
                if (c.t_var[h] != k) {
                    const int32_t i = c.t_var[h];
                    const double zmax = std::max(std::fabs((double)c.lo[i]), std::fabs((double)c.hi[i]));
                    prod *= std::pow(zmax, (double)(q - h));
                }
                h = q;
            }
            per_var[k] += prod * std::pow((double)c.hi[k] - (double)c.lo[k], m);
            f = g;
        }
    }
    double de_max = 0.0;
    for (double v : per_var) de_max = std::max(de_max, v);
    if (!(de_max > 0.0) || !std::isfinite(min_abs)) {
        err = "automatic schedule needs a term on a variable with a nonempty range";
        return SA_EINVAL;
    }
    *t_init = -de_max / std::log(0.5);
    *t_final = -min_abs / std::log(0.001);
    return SA_OK;
}

void geometric_betas(double t_init, double t_final, int32_t n_sweeps, double *beta_out) {
    for (int32_t s = 0; s < n_sweeps; ++s) {
        double T = n_sweeps > 1
                       ? t_init * std::pow(t_final / t_init, (double)s / (double)(n_sweeps - 1))
                       : t_init;
        beta_out[s] = 1.0 / T;
    }
}

namespace {

// A QUIO whose pair terms cover at least a quarter of all pairs is packed as a dense matrix: a
// row of J costs 1 or 4 bytes per pair instead of an incidence record per pair.
bool pack_dense(const Canonical &c, Packed &p) {
    const int32_t n = c.n;
    const int64_t nt = c.n_terms();
    if (n < 32) return false;
    int64_t pairs = 0;
    int64_t jmax = 0;
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t deg = c.t_off[t + 1] - c.t_off[t];
        if (deg > 2) return false;
        if (deg == 2 && c.t_var[c.t_off[t]] != c.t_var[c.t_off[t] + 1]) {
            ++pairs;
            const int64_t a = c.t_coef[t] < 0 ? -c.t_coef[t] : c.t_coef[t];
            jmax = std::max(jmax, a);
        }
    }
    if ((double)pairs < 0.25 * (double)n * (double)(n - 1) / 2.0) return false;
    if (jmax > INT32_MAX) return false;
    const int32_t stride = (n + 15) & ~15;
    const int jbytes = jmax <= 127 ? 1 : 4;
    if ((double)n * stride * jbytes > 8.0e9) return false;
    p.dense = true;
    p.jbytes = jbytes;
    p.row_stride = stride;
    p.n_pairs = pairs;
    p.h.assign(n, 0);
    p.d.assign(n, 0);
    if (jbytes == 1) p.jd8.assign((size_t)n * stride, 0);
    else p.jd32.assign((size_t)n * stride, 0);
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t a = c.t_off[t];
        const int64_t deg = c.t_off[t + 1] - a;
        const int32_t i = c.t_var[a];
        if (deg == 1) {
            p.h[i] += c.t_coef[t];
        } else if (c.t_var[a + 1] == i) {
            p.d[i] += c.t_coef[t];
        } else {
            const int32_t j = c.t_var[a + 1];
            if (jbytes == 1) {
                p.jd8[(size_t)i * stride + j] = (int8_t)c.t_coef[t];
                p.jd8[(size_t)j * stride + i] = (int8_t)c.t_coef[t];
            } else {
                p.jd32[(size_t)i * stride + j] = (int32_t)c.t_coef[t];
                p.jd32[(size_t)j * stride + i] = (int32_t)c.t_coef[t];
            }
            p.emask[i] |= 2u;
            p.emask[j] |= 2u;
        }
    }
    for (int32_t k = 0; k < n; ++k) {
        if (p.h[k] != 0) p.emask[k] |= 2u;
        if (p.d[k] != 0) {
            p.emask[k] |= 4u;
            p.max_exp = 2;
        } else if (p.emask[k]) {
            p.max_exp = std::max(p.max_exp, 1);
        }
    }
    return true;
}

}  // namespace

int pack(const Canonical &c, Packed &p, std::string &err) {
    const int32_t n = c.n;
    const int64_t nt = c.n_terms();
    if (nt > INT32_MAX - 1 || (int64_t)c.t_var.size() > INT32_MAX - 1) {
        err = "problem too large for 32-bit term offsets";
        return SA_EINVAL;
    }
    p = Packed();
    p.n = n;
    p.n_terms = (int32_t)nt;
    p.var.resize(n);
    p.emask.assign(n, 0u);
    if (pack_dense(c, p)) {
        for (int32_t k = 0; k < n; ++k) {
            const int64_t w = (int64_t)c.hi[k] - c.lo[k] + 1;
            p.var[k] = VarRec{c.lo[k], (int32_t)w, 0, 0};
            p.max_width = std::max<int32_t>(p.max_width, (int32_t)w);
        }
        p.n_terms = 0;  // energies come from the matrix
        p.t_off.assign(1, 0);
        return SA_OK;
    }
    // count incidences (distinct variables per term)
    std::vector<int64_t> deg(n, 0);
    for (int64_t t = 0; t < nt; ++t)
        for (int64_t f = c.t_off[t]; f < c.t_off[t + 1]; ++f)
            if (f == c.t_off[t] || c.t_var[f] != c.t_var[f - 1]) deg[c.t_var[f]]++;
    int64_t total = 0;
    for (int32_t k = 0; k < n; ++k) {
        if (total > INT32_MAX || deg[k] > INT32_MAX) {
            err = "too many term incidences for 32-bit offsets";
            return SA_EINVAL;
        }
        int64_t w = (int64_t)c.hi[k] - c.lo[k] + 1;
        p.var[k] = VarRec{c.lo[k], (int32_t)w, (int32_t)total, (int32_t)deg[k]};
        p.max_width = std::max<int32_t>(p.max_width, (int32_t)w);
        total += deg[k];
    }
    if (total > INT32_MAX) {
        err = "too many term incidences for 32-bit offsets";
        return SA_EINVAL;
    }
    p.inc.resize((size_t)total);
    p.inc_coef.resize((size_t)total);
    std::vector<int64_t> fill(n);
    for (int32_t k = 0; k < n; ++k) fill[k] = p.var[k].row;
    std::vector<int32_t> others;
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t a = c.t_off[t], b = c.t_off[t + 1];
        for (int64_t f = a; f < b;) {
            int64_t g = f;
            while (g < b && c.t_var[g] == c.t_var[f]) ++g;
            const int32_t k = c.t_var[f];
            const int64_t e = g - f;
            if (e > kMaxExpStored) {
                err = "exponent above 255 is not supported";
                return SA_EUNSUPPORTED;
            }
            others.clear();
            for (int64_t h = a; h < b; ++h)
                if (c.t_var[h] != k) others.push_back(c.t_var[h]);
            IncRec r{};
            r.meta = (uint32_t)e | ((uint32_t)others.size() << 8);
            p.max_other = std::max<int32_t>(p.max_other, (int32_t)others.size());
            if (others.size() <= 3) {
                for (size_t q = 0; q < 3; ++q) r.o[q] = q < others.size() ? others[q] : 0;
            } else {
                if (others.size() >= (1u << 24) || p.overflow.size() > (size_t)INT32_MAX - others.size() - 3) {
                    err = "term too long";
                    return SA_EINVAL;
                }
                // each list starts on a 16-byte boundary and is padded with -1 to whole groups of
                // four, so that the device reads it four indices at a time
                r.o[0] = (int32_t)p.overflow.size();
                r.o[1] = r.o[2] = 0;
                p.overflow.insert(p.overflow.end(), others.begin(), others.end());
                while (p.overflow.size() % 4) p.overflow.push_back(-1);
            }
            const int64_t slot = fill[k]++;
            p.inc[slot] = r;
            p.inc_coef[slot] = c.t_coef[t];
            p.emask[k] |= 1u << std::min<int64_t>(e, 31);
            p.max_exp = std::max<int32_t>(p.max_exp, (int32_t)e);
            f = g;
        }
    }
    p.t_off.resize((size_t)nt + 1);
    for (int64_t t = 0; t <= nt; ++t) p.t_off[t] = (int32_t)c.t_off[t];
    p.t_var = c.t_var;
    p.t_coef = c.t_coef;
    // compact pair records: every incidence is z_k to the first power with at most one other
    // factor, and every coefficient and linear sum fits int32
    bool compact = p.max_exp <= 1 && p.max_other <= 1;
    for (size_t q = 0; compact && q < p.inc.size(); ++q)
        compact = p.inc_coef[q] >= INT32_MIN && p.inc_coef[q] <= INT32_MAX;
    if (compact) {
        p.pair_row.assign(n, 0);
        p.pair_deg.assign(n, 0);
        p.pair_h.assign(n, 0);
        for (int32_t k = 0; k < n && compact; ++k) {
            const VarRec &vr = p.var[k];
            int64_t h = 0;
            p.pair_row[k] = (int32_t)p.pair.size();
            for (int32_t q = vr.row; q < vr.row + vr.deg; ++q) {
                if ((p.inc[q].meta >> 8) == 0)
                    h += p.inc_coef[q];
                else
                    p.pair.push_back(PairRec{p.inc[q].o[0], (int32_t)p.inc_coef[q]});
            }
            p.pair_deg[k] = (int32_t)p.pair.size() - p.pair_row[k];
            while ((p.pair.size() - (size_t)p.pair_row[k]) % kPairBlock) p.pair.push_back(PairRec{0, 0});
            compact = h >= INT32_MIN && h <= INT32_MAX;
            p.pair_h[k] = (int32_t)h;
        }
        if (!compact) {
            p.pair.clear();
            p.pair_row.clear();
            p.pair_deg.clear();
            p.pair_h.clear();
        }
    }
    return SA_OK;
}

int32_t build_schedule(const Packed &p, int G, std::vector<SchedRec> &out) {
    const int32_t n = p.n;
    std::vector<int32_t> stamp(n, -1);
    std::vector<int32_t> starts;   // window w holds members[starts[w] .. starts[w+1])
    std::vector<int32_t> members;
    int32_t win = -1, count = G;
    for (int32_t k = 0; k < n; ++k) {
        const VarRec &vr = p.var[k];
        if (vr.width == 1) continue;
        // a dense problem couples (almost) every pair: one variable per window
        if (count == G || stamp[k] == win || p.dense) {
            ++win;
            count = 0;
            starts.push_back((int32_t)members.size());
        }
        members.push_back(k);
        ++count;
        // every variable sharing a term with k conflicts with this window
        for (int32_t q = vr.row; q < vr.row + vr.deg; ++q) {
            const IncRec &r = p.inc[q];
            const uint32_t no = r.meta >> 8;
            if (no <= 3) {
                for (uint32_t f = 0; f < no; ++f) stamp[r.o[f]] = win;
            } else {
                for (uint32_t f = 0; f < no; ++f) stamp[p.overflow[(size_t)r.o[0] + f]] = win;
            }
        }
    }
    const int32_t n_win = (int32_t)starts.size();
    starts.push_back((int32_t)members.size());
    out.assign((size_t)n_win * G, SchedRec{-1, 0, 1, 0, 0, 0u, {0, 0}});
    for (int32_t w = 0; w < n_win; ++w) {
        for (int32_t i = starts[w]; i < starts[w + 1]; ++i) {
            const int g = i - starts[w];
            const int32_t k = members[i];
            const VarRec &vr = p.var[k];
            out[(size_t)g * n_win + w] = SchedRec{k, vr.lo, vr.width, vr.row, vr.deg, p.emask[k], {0, 0}};
        }
    }
    return n_win;
}

}  // namespace sa

namespace sa {

int32_t build_levels(const Packed &p, int32_t quads, std::vector<int32_t> &level_start,
                     std::vector<SchedRec> &slots) {
    const int32_t n = p.n;
    // lower-index neighbours of every variable that is not fixed (a fixed variable never changes:
    // it orders nothing)
    std::vector<std::vector<int32_t>> lower((size_t)n), upper((size_t)n);
    for (int32_t k = 0; k < n; ++k) {
        const VarRec &vr = p.var[k];
        if (vr.width == 1) continue;
        auto see = [&](int32_t j) {
            if (j != k && p.var[j].width > 1) {
                if (j < k) lower[(size_t)k].push_back(j);
                else upper[(size_t)k].push_back(j);
            }
        };
        if (p.dense) {
            // every pair is coupled: each variable waits for all earlier ones
            for (int32_t j = 0; j < n; ++j) see(j);
        } else {
            for (int32_t q = vr.row; q < vr.row + vr.deg; ++q) {
                const IncRec &r = p.inc[q];
                const uint32_t no = r.meta >> 8;
                if (no <= 3) {
                    for (uint32_t f = 0; f < no; ++f) see(r.o[f]);
                } else {
                    for (uint32_t f = 0; f < no; ++f) see(p.overflow[(size_t)r.o[0] + f]);
                }
            }
        }
        auto &lo = lower[(size_t)k];
        std::sort(lo.begin(), lo.end());
        lo.erase(std::unique(lo.begin(), lo.end()), lo.end());
        auto &up = upper[(size_t)k];
        std::sort(up.begin(), up.end());
        up.erase(std::unique(up.begin(), up.end()), up.end());
    }
    // earliest level (longest chain of lower-index neighbours below k) and latest level (the
    // number of levels minus the longest chain above k)
    std::vector<int32_t> asap((size_t)n, -1), down((size_t)n, 0);
    int32_t n_levels = 0;
    for (int32_t k = 0; k < n; ++k) {
        if (p.var[k].width == 1) continue;
        int32_t lv = 0;
        for (int32_t j : lower[(size_t)k]) lv = std::max(lv, asap[(size_t)j] + 1);
        asap[(size_t)k] = lv;
        n_levels = std::max(n_levels, lv + 1);
    }
    for (int32_t k = n - 1; k >= 0; --k) {
        if (p.var[k].width == 1) continue;
        int32_t d = 0;
        for (int32_t j : upper[(size_t)k]) d = std::max(d, down[(size_t)j] + 1);
        down[(size_t)k] = d;
    }
    // level by level: every variable that must go now (its latest level) goes, and the level is
    // filled up to a whole number of rounds of `quads` updates with the ready variables whose
    // latest level is nearest; a variable is ready once its lower-index neighbours are placed
    std::vector<int32_t> level((size_t)n, -1), waiting((size_t)n, 0);
    std::set<std::pair<int32_t, int32_t>> ready;   // (latest level, index)
    for (int32_t k = 0; k < n; ++k) {
        if (p.var[k].width == 1) continue;
        waiting[(size_t)k] = (int32_t)lower[(size_t)k].size();
        if (waiting[(size_t)k] == 0) ready.insert({n_levels - 1 - down[(size_t)k], k});
    }
    const int32_t Q = std::max<int32_t>(quads, 1);
    for (int32_t l = 0; l < n_levels; ++l) {
        std::vector<int32_t> take;
        auto it = ready.begin();
        while (it != ready.end() && it->first == l) take.push_back((it++)->second);
        const size_t target = (take.size() + (size_t)Q - 1) / (size_t)Q * (size_t)Q;
        while (it != ready.end() && take.size() < target) take.push_back((it++)->second);
        ready.erase(ready.begin(), it);
        for (int32_t k : take) level[(size_t)k] = l;
        for (int32_t k : take)
            for (int32_t j : upper[(size_t)k])
                if (--waiting[(size_t)j] == 0) ready.insert({n_levels - 1 - down[(size_t)j], j});
    }
    // counting sort by level; index order inside a level
    level_start.assign((size_t)n_levels + 1, 0);
    for (int32_t k = 0; k < n; ++k)
        if (level[(size_t)k] >= 0) level_start[(size_t)level[(size_t)k] + 1]++;
    for (int32_t l = 0; l < n_levels; ++l) level_start[(size_t)l + 1] += level_start[(size_t)l];
    slots.assign((size_t)level_start[(size_t)n_levels], SchedRec{-1, 0, 1, 0, 0, 0u, {0, 0}});
    std::vector<int32_t> fill(level_start.begin(), level_start.end() - 1);
    for (int32_t k = 0; k < n; ++k) {
        if (level[(size_t)k] < 0) continue;
        const VarRec &vr = p.var[k];
        // with compact pair records the slot points at the variable's pairs and carries its
        // linear coefficient
        slots[(size_t)fill[(size_t)level[(size_t)k]]++] =
            p.pair.empty() && p.pair_row.empty()
                ? SchedRec{k, vr.lo, vr.width, vr.row, vr.deg, p.emask[k], {0, 0}}
                : SchedRec{k, vr.lo, vr.width, p.pair_row[k], p.pair_deg[k], p.emask[k], {p.pair_h[k], 0}};
    }
    return n_levels;
}

void build_mo_records(const Packed &p, std::vector<SchedRec> &rounds, bool coef32, std::vector<MoRec> &rec,
                      std::vector<uint8_t> &coef) {
    const size_t n_rounds = rounds.size() / (size_t)kRoundQuads;
    const size_t per_round = (size_t)kMoAhead * (size_t)kRoundQuads * 4;   // records of a round (64 lanes)
    const uint32_t one = (uint32_t)p.n * 4u;                                  // LDS offset of the constant 1
    rec.assign(n_rounds * per_round, MoRec{0u, {one, one, one}});
    const size_t cw = coef32 ? 4 : 8;
    coef.assign(n_rounds * per_round * cw, 0);
    for (size_t r = 0; r < n_rounds; ++r) {
        for (int32_t q = 0; q < kRoundQuads; ++q) {
            SchedRec &s = rounds[r * (size_t)kRoundQuads + (size_t)q];
            s.pad[0] = 0;
            if (s.k < 0) continue;
            bool rest = s.deg > 4 * kMoAhead;
            const int32_t m = std::min<int32_t>(s.deg, 4 * kMoAhead);
            for (int32_t i = 0; i < m; ++i) {
                const size_t idx = (r * (size_t)kMoAhead + (size_t)(i / 4)) * 64 + (size_t)(q * 4 + i % 4);
                const IncRec &ir = p.inc[(size_t)s.row + (size_t)i];
                const uint32_t no = ir.meta >> 8;
                MoRec &mr = rec[idx];
                mr.meta = ir.meta;
                if (no > 3) {   // a long record: added from the incidence records, zero here
                    rest = true;
                    continue;
                }
                for (uint32_t f = 0; f < no; ++f) mr.zoff[f] = (uint32_t)ir.o[f] * 4u;
                const int64_t c = p.inc_coef[(size_t)s.row + (size_t)i];
                if (coef32) {
                    const int32_t c32 = (int32_t)c;
                    std::memcpy(coef.data() + idx * cw, &c32, sizeof(c32));
                } else {
                    std::memcpy(coef.data() + idx * cw, &c, sizeof(c));
                }
            }
            s.pad[0] = rest ? 1 : 0;
        }
    }
}

int32_t quad_uniform_width(const Packed &p) {
    int32_t w = 0;
    for (const VarRec &vr : p.var) {
        if (vr.width <= 1) continue;
        if (w == 0) w = vr.width;
        else if (vr.width != w) return 0;
    }
    return w;
}

int32_t build_rounds(const Packed &p, std::vector<SchedRec> &rounds, int32_t &n_real) {
    std::vector<int32_t> start;
    std::vector<SchedRec> slots;
    const int32_t n_levels = build_levels(p, kRoundQuads, start, slots);
    const SchedRec idle{-1, 0, 1, 0, 0, 0u, {0, 0}};
    rounds.clear();
    for (int32_t l = 0; l < n_levels; ++l) {
        for (int32_t i = start[(size_t)l]; i < start[(size_t)l + 1]; ++i) {
            const int32_t k = slots[(size_t)i].k;
            const VarRec &vr = p.var[(size_t)k];
            rounds.push_back(SchedRec{k, vr.lo, vr.width, vr.row, vr.deg, p.emask[(size_t)k], {0, 0}});
        }
        while (rounds.size() % (size_t)kRoundQuads) rounds.push_back(idle);
    }
    while (rounds.size() % (size_t)(kRoundQuads * kRoundBatch)) rounds.push_back(idle);
    n_real = (int32_t)slots.size();
    return n_levels;
}

}  // namespace sa
