/*
 * sa_oracle.c -- plain sequential CPU oracle for direct simulated annealing of QUIO/HUIO
 * problems (arXiv:2511.17245).  TEST INFRASTRUCTURE ONLY: it defines what the GPU path must
 * compute and is never part of the product path.  Written for readability against the paper,
 * not for speed: every quantity is computed the way the cited passage defines it.
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *  - random initial state: z_k uniform on [l_k, u_k];
 *  - random numbers: Philox4x32-10, counter (k, s, r, instance), key = seed;
 *  - Metropolis proposal: uniform over the u_k - l_k values other than z_k;
 *  - acceptance: dE <= 0 accepts, otherwise U < exp(-(beta * dE)) with U in [0, 1);
 *  - heat bath: weights exp(-beta (dE_v - min dE)) over all u_k - l_k + 1 values, summed one
 *    value at a time in increasing value order; first cumulative weight above U * total is chosen;
 *  - optimal transition: argmin of dE over the whole range (z_k itself included, dE = 0), ties
 *    to the smallest value, with probability r = s/(S-1); otherwise the Metropolis proposal;
 *    Metropolis acceptance (the optimal move, whose dE <= 0, is always accepted);
 *  - variables with l_k = u_k are skipped; zero coefficients are dropped.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -pthread -o libsa_oracle.so sa_oracle.c -lm
 */
#define _GNU_SOURCE
#include "sa_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

struct sao_poly {
    int32_t n;          /* number of variables */
    int64_t nt;         /* number of canonical terms */
    int64_t *tptr;      /* nt+1 offsets into pvar/pexp */
    int32_t *pvar;      /* the distinct variables of a term, ascending */
    int32_t *pexp;      /* their exponents (>= 1) */
    int64_t *J;         /* nonzero coefficient of each term */
    int32_t *lo, *hi;   /* integer box */
    int64_t *iptr;      /* n+1 offsets: terms incident to each variable */
    int64_t *iterm;     /* incident term */
    int32_t *iexp;      /* exponent of the variable inside that term */
    int32_t *maxe;      /* largest exponent of each variable (0: appears nowhere) */
    int32_t max_exp;
    int64_t max_width;  /* max over k of u_k - l_k + 1 */
};

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11): ten rounds of two 32x32->64 multiplies; the key is bumped by the    */
/* Weyl constants between rounds.                                                             */
/* ------------------------------------------------------------------------------------------ */
void sao_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static void draw(uint32_t k, uint32_t s, uint32_t r, uint32_t inst, const uint32_t key[2],
                 uint32_t x[4]) {
    uint32_t ctr[4] = {k, s, r, inst};
    sao_philox(ctr, key, x);
}

/* U in [0,1) from 53 bits of words 2 and 3. */
static double uniform53(const uint32_t x[4]) {
    uint64_t bits = ((uint64_t)x[2] << 32) | (uint64_t)x[3];
    return (double)(bits >> 11) * 0x1p-53;
}

/* State hash for tracing: H(z) = sum over k of mix(k * 2^32 + (uint32)z_k) modulo 2^64, with mix
 * the 64-bit finaliser of SplitMix64 (Stafford's "variant 13" constants).  A sum is used so that
 * any partition of the variables gives the same value; the hash only localises the first sweep
 * at which two runs of the same chain part. */
static uint64_t mix64(uint64_t x) {
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static uint64_t state_hash(int32_t n, const int32_t *z) {
    uint64_t h = 0;
    for (int32_t k = 0; k < n; ++k) h += mix64(((uint64_t)(uint32_t)k << 32) | (uint64_t)(uint32_t)z[k]);
    return h;
}

uint64_t sao_state_hash(int32_t n, const int32_t *z) { return (n > 0 && z) ? state_hash(n, z) : 0; }
uint64_t sao_mix64(uint64_t x) { return mix64(x); }

/* ------------------------------------------------------------------------------------------ */
/* Canonicalisation (Sec. 2: terms with the same index multiset are one term).                 */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    const int64_t *off; /* sorted factor lists, per raw term */
    const int32_t *fac;
} term_cmp_ctx;

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int cmp_terms(const void *a, const void *b, void *vctx) {
    const term_cmp_ctx *c = (const term_cmp_ctx *)vctx;
    int64_t ta = *(const int64_t *)a, tb = *(const int64_t *)b;
    int64_t la = c->off[ta + 1] - c->off[ta], lb = c->off[tb + 1] - c->off[tb];
    if (la != lb) return la < lb ? -1 : 1;
    for (int64_t i = 0; i < la; ++i) {
        int32_t x = c->fac[c->off[ta] + i], y = c->fac[c->off[tb] + i];
        if (x != y) return x < y ? -1 : 1;
    }
    return (ta > tb) - (ta < tb);
}

void sao_poly_free(sao_poly *p) {
    if (!p) return;
    free(p->tptr);
    free(p->pvar);
    free(p->pexp);
    free(p->J);
    free(p->lo);
    free(p->hi);
    free(p->iptr);
    free(p->iterm);
    free(p->iexp);
    free(p->maxe);
    free(p);
}

static int64_t iabs64(int64_t x) { return x < 0 ? -x : x; }

int sao_poly_build(int32_t n_vars, int64_t n_terms, const int64_t *term_ptr,
                   const int32_t *factor_var, const int64_t *coef, const int32_t *lower,
                   const int32_t *upper, sao_poly **out) {
    if (!out || n_vars < 1 || n_terms < 0 || !lower || !upper) return SAO_EINVAL;
    if (n_terms > 0 && (!term_ptr || !factor_var || !coef)) return SAO_EINVAL;
    *out = NULL;
    for (int32_t i = 0; i < n_vars; ++i) {
        if (lower[i] > upper[i]) return SAO_EINVAL;
        if ((int64_t)upper[i] - (int64_t)lower[i] > 2147483646LL) return SAO_EINVAL;
    }
    if (n_terms > 0 && term_ptr[0] != 0) return SAO_EINVAL;
    for (int64_t t = 0; t < n_terms; ++t)
        if (term_ptr[t + 1] <= term_ptr[t]) return SAO_EINVAL; /* degree >= 1 */
    int64_t nf = n_terms > 0 ? term_ptr[n_terms] : 0;
    for (int64_t f = 0; f < nf; ++f)
        if (factor_var[f] < 0 || factor_var[f] >= n_vars) return SAO_EINVAL;

    int rc = SAO_ENOMEM;
    int32_t *fac = NULL;
    int64_t *order = NULL;
    sao_poly *p = (sao_poly *)calloc(1, sizeof(sao_poly));
    if (!p) return SAO_ENOMEM;
    p->n = n_vars;
    p->lo = (int32_t *)malloc(sizeof(int32_t) * n_vars);
    p->hi = (int32_t *)malloc(sizeof(int32_t) * n_vars);
    fac = (int32_t *)malloc(sizeof(int32_t) * (nf > 0 ? nf : 1));
    order = (int64_t *)malloc(sizeof(int64_t) * (n_terms > 0 ? n_terms : 1));
    if (!p->lo || !p->hi || !fac || !order) goto fail;
    memcpy(p->lo, lower, sizeof(int32_t) * n_vars);
    memcpy(p->hi, upper, sizeof(int32_t) * n_vars);
    if (nf > 0) memcpy(fac, factor_var, sizeof(int32_t) * nf);
    for (int64_t t = 0; t < n_terms; ++t) {
        qsort(fac + term_ptr[t], (size_t)(term_ptr[t + 1] - term_ptr[t]), sizeof(int32_t), cmp_i32);
        order[t] = t;
    }
    term_cmp_ctx ctx = {term_ptr, fac};
    if (n_terms > 1) qsort_r(order, (size_t)n_terms, sizeof(int64_t), cmp_terms, &ctx);

    /* merge runs of equal multisets; keep nonzero sums */
    p->tptr = (int64_t *)malloc(sizeof(int64_t) * (n_terms + 1));
    p->pvar = (int32_t *)malloc(sizeof(int32_t) * (nf > 0 ? nf : 1));
    p->pexp = (int32_t *)malloc(sizeof(int32_t) * (nf > 0 ? nf : 1));
    p->J = (int64_t *)malloc(sizeof(int64_t) * (n_terms > 0 ? n_terms : 1));
    if (!p->tptr || !p->pvar || !p->pexp || !p->J) goto fail;
    p->tptr[0] = 0;
    int64_t nt = 0, npairs = 0;
    for (int64_t a = 0; a < n_terms;) {
        int64_t b = a + 1;
        while (b < n_terms) {
            int64_t ta = order[a], tb = order[b];
            int64_t la = term_ptr[ta + 1] - term_ptr[ta];
            if (term_ptr[tb + 1] - term_ptr[tb] != la) break;
            if (memcmp(fac + term_ptr[ta], fac + term_ptr[tb], sizeof(int32_t) * la) != 0) break;
            ++b;
        }
        __int128 sum = 0;
        for (int64_t q = a; q < b; ++q) sum += coef[order[q]];
        if (sum > INT64_MAX || sum < -INT64_MAX) {
            rc = SAO_ERANGE;
            goto fail;
        }
        if (sum != 0) {
            int64_t t0 = order[a];
            for (int64_t f = term_ptr[t0]; f < term_ptr[t0 + 1];) {
                int64_t g = f;
                while (g < term_ptr[t0 + 1] && fac[g] == fac[f]) ++g;
                p->pvar[npairs] = fac[f];
                p->pexp[npairs] = (int32_t)(g - f);
                ++npairs;
                f = g;
            }
            p->J[nt] = (int64_t)sum;
            p->tptr[++nt] = npairs;
        }
        a = b;
    }
    p->nt = nt;

    /* int64 bound: B = sum_t |J_t| prod zmax_i^e must stay below 2^62 so that every energy and
     * every energy difference (|dE| <= 2B) is exact in int64. */
    {
        const __int128 LIM = (__int128)1 << 62;
        __int128 B = 0;
        for (int64_t t = 0; t < nt; ++t) {
            __int128 prod = iabs64(p->J[t]);
            for (int64_t q = p->tptr[t]; q < p->tptr[t + 1] && prod < LIM; ++q) {
                int32_t i = p->pvar[q];
                int64_t zm = iabs64(p->lo[i]) > iabs64(p->hi[i]) ? iabs64(p->lo[i]) : iabs64(p->hi[i]);
                for (int e = 0; e < p->pexp[q] && prod < LIM; ++e) prod *= zm;
            }
            B += prod;
            if (B >= LIM) {
                rc = SAO_ERANGE;
                goto fail;
            }
        }
    }

    /* incidence lists: the terms T_k that contain z_k (Sec. 3.2) */
    p->iptr = (int64_t *)calloc((size_t)n_vars + 1, sizeof(int64_t));
    p->iterm = (int64_t *)malloc(sizeof(int64_t) * (npairs > 0 ? npairs : 1));
    p->iexp = (int32_t *)malloc(sizeof(int32_t) * (npairs > 0 ? npairs : 1));
    p->maxe = (int32_t *)calloc((size_t)n_vars, sizeof(int32_t));
    if (!p->iptr || !p->iterm || !p->iexp || !p->maxe) goto fail;
    for (int64_t q = 0; q < npairs; ++q) p->iptr[p->pvar[q] + 1]++;
    for (int32_t i = 0; i < n_vars; ++i) p->iptr[i + 1] += p->iptr[i];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * n_vars);
        if (!fill) goto fail;
        memcpy(fill, p->iptr, sizeof(int64_t) * n_vars);
        for (int64_t t = 0; t < nt; ++t)
            for (int64_t q = p->tptr[t]; q < p->tptr[t + 1]; ++q) {
                int32_t i = p->pvar[q];
                p->iterm[fill[i]] = t;
                p->iexp[fill[i]] = p->pexp[q];
                fill[i]++;
                if (p->pexp[q] > p->maxe[i]) p->maxe[i] = p->pexp[q];
            }
        free(fill);
    }
    p->max_exp = 0;
    p->max_width = 1;
    for (int32_t i = 0; i < n_vars; ++i) {
        if (p->maxe[i] > p->max_exp) p->max_exp = p->maxe[i];
        int64_t w = (int64_t)p->hi[i] - p->lo[i] + 1;
        if (w > p->max_width) p->max_width = w;
    }
    free(fac);
    free(order);
    *out = p;
    return SAO_OK;
fail:
    free(fac);
    free(order);
    sao_poly_free(p);
    return rc;
}

int64_t sao_poly_n_terms(const sao_poly *p) { return p ? p->nt : -1; }
int64_t sao_poly_n_pairs(const sao_poly *p) { return p ? p->tptr[p->nt] : -1; }
int32_t sao_poly_max_exponent(const sao_poly *p) { return p ? p->max_exp : -1; }

int sao_poly_export(const sao_poly *p, int64_t *tptr, int32_t *var, int32_t *expo, int64_t *coef) {
    if (!p) return SAO_EINVAL;
    int64_t np = p->tptr[p->nt];
    if (tptr) memcpy(tptr, p->tptr, sizeof(int64_t) * (p->nt + 1));
    if (var) memcpy(var, p->pvar, sizeof(int32_t) * np);
    if (expo) memcpy(expo, p->pexp, sizeof(int32_t) * np);
    if (coef) memcpy(coef, p->J, sizeof(int64_t) * p->nt);
    return SAO_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Energy and energy differences                                                              */
/* ------------------------------------------------------------------------------------------ */
static int64_t ipow(int64_t x, int32_t e) {
    int64_t r = 1;
    for (int32_t i = 0; i < e; ++i) r *= x;
    return r;
}

/* E_p(z) = sum over canonical terms of J_t prod z_i^e (Sec. 2, the HUIO objective). */
static int64_t energy(const sao_poly *p, const int32_t *z) {
    int64_t E = 0;
    for (int64_t t = 0; t < p->nt; ++t) {
        int64_t prod = p->J[t];
        for (int64_t q = p->tptr[t]; q < p->tptr[t + 1]; ++q) prod *= ipow(z[p->pvar[q]], p->pexp[q]);
        E += prod;
    }
    return E;
}

int sao_energy(const sao_poly *p, const int32_t *z, int64_t *out) {
    if (!p || !z || !out) return SAO_EINVAL;
    *out = energy(p, z);
    return SAO_OK;
}

/* a_k^(m)(z) = sum over terms containing z_k exactly m times of J_t times the product of the
 * term's other factors (Sec. 3.2: T_k = sum_m a_k^(m) z_k^m).  a[m] for m = 1..maxe_k. */
static void coeffs_recompute(const sao_poly *p, const int32_t *z, int32_t k, int64_t *a) {
    for (int32_t m = 0; m <= p->maxe[k]; ++m) a[m] = 0;
    for (int64_t q = p->iptr[k]; q < p->iptr[k + 1]; ++q) {
        int64_t t = p->iterm[q];
        int64_t prod = p->J[t];
        for (int64_t f = p->tptr[t]; f < p->tptr[t + 1]; ++f)
            if (p->pvar[f] != k) prod *= ipow(z[p->pvar[f]], p->pexp[f]);
        a[p->iexp[q]] += prod;
    }
}

/* dE_k = sum_m a_k^(m) ((z_k + dz)^m - z_k^m) with z_k + dz = v (Sec. 3.2). */
static int64_t delta_from_coeffs(const int64_t *a, int32_t maxe, int64_t zk, int64_t v) {
    int64_t d = 0;
    for (int32_t m = 1; m <= maxe; ++m)
        if (a[m] != 0) d += a[m] * (ipow(v, m) - ipow(zk, m));
    return d;
}

int sao_delta(const sao_poly *p, const int32_t *z, int32_t k, int32_t v, int64_t *out) {
    if (!p || !z || !out || k < 0 || k >= p->n) return SAO_EINVAL;
    int64_t *a = (int64_t *)malloc(sizeof(int64_t) * (p->max_exp + 1));
    if (!a) return SAO_ENOMEM;
    coeffs_recompute(p, z, k, a);
    *out = delta_from_coeffs(a, p->maxe[k], z[k], v);
    free(a);
    return SAO_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Temperature schedule (Sec. 3.4 and the geometric cooling of Sec. 3.1).                      */
/* ------------------------------------------------------------------------------------------ */
int sao_schedule(const sao_poly *p, int32_t n_sweeps, double *beta_out, double *t_init,
                 double *t_final) {
    if (!p || n_sweeps < 1) return SAO_EINVAL;
    if (p->nt == 0) return SAO_EINVAL;
    /* dE_max ~ max_k sum_m a~_k^(m) (u_k - l_k)^m, a~ built from |J| and z^max = max(|l|,|u|) */
    double dEmax = 0.0;
    for (int32_t k = 0; k < p->n; ++k) {
        if (p->iptr[k] == p->iptr[k + 1]) continue;
        double width = (double)p->hi[k] - (double)p->lo[k];
        double sum = 0.0;
        for (int64_t q = p->iptr[k]; q < p->iptr[k + 1]; ++q) {
            int64_t t = p->iterm[q];
            double prod = fabs((double)p->J[t]);
            for (int64_t f = p->tptr[t]; f < p->tptr[t + 1]; ++f) {
                int32_t i = p->pvar[f];
                if (i == k) continue;
                double zmax = fmax(fabs((double)p->lo[i]), fabs((double)p->hi[i]));
                prod *= pow(zmax, (double)p->pexp[f]);
            }
            sum += prod * pow(width, (double)p->iexp[q]);
        }
        if (sum > dEmax) dEmax = sum;
    }
    /* dE_min ~ smallest |J| over all (nonzero, merged) coefficients */
    double dEmin = INFINITY;
    for (int64_t t = 0; t < p->nt; ++t) {
        double a = fabs((double)p->J[t]);
        if (a < dEmin) dEmin = a;
    }
    if (!(dEmax > 0.0)) return SAO_EINVAL; /* every variable fixed: no energy scale */
    double Tmax = -dEmax / log(0.5);    /* accept dE_max with probability a = 1/2 */
    double Tmin = -dEmin / log(0.001);  /* accept dE_min with probability b = 0.001 */
    if (t_init) *t_init = Tmax;
    if (t_final) *t_final = Tmin;
    if (beta_out) {
        for (int32_t s = 0; s < n_sweeps; ++s) {
            double T = n_sweeps > 1 ? Tmax * pow(Tmin / Tmax, (double)s / (double)(n_sweeps - 1)) : Tmax;
            beta_out[s] = 1.0 / T;
        }
    }
    return SAO_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* One single-variable update (Sec. 3.1 steps (1)-(2), transition rules of Sec. 3.3)           */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    const sao_poly *p;
    int rule;
    uint32_t key[2];
    uint32_t inst;
    int64_t *a;     /* max_exp+1 scratch */
    double *w;      /* max_width scratch (heat bath) */
    int64_t *cache; /* n x (max_exp+1) coefficient cache, or NULL (recompute mode) */
} chain_ctx;

/* Paper's cache update (Sec. 3.2, the b_{k,s}^(m,n) update of a_k^(m)): when z_s moves to v,
 * every other variable k of every term t containing z_s gets
 *   a_k^(e_k(t)) += J_t * prod_{i not in {k,s}} z_i^e * (v^{e_s(t)} - z_s^{e_s(t)}). */
static void cache_apply_move(chain_ctx *c, const int32_t *z, int32_t s, int64_t v) {
    const sao_poly *p = c->p;
    int32_t stride = p->max_exp + 1;
    for (int64_t q = p->iptr[s]; q < p->iptr[s + 1]; ++q) {
        int64_t t = p->iterm[q];
        int64_t ds = ipow(v, p->iexp[q]) - ipow(z[s], p->iexp[q]);
        for (int64_t f = p->tptr[t]; f < p->tptr[t + 1]; ++f) {
            int32_t k = p->pvar[f];
            if (k == s) continue;
            int64_t prod = p->J[t] * ds;
            for (int64_t g = p->tptr[t]; g < p->tptr[t + 1]; ++g) {
                int32_t i = p->pvar[g];
                if (i == k || i == s) continue;
                prod *= ipow(z[i], p->pexp[g]);
            }
            c->cache[(int64_t)k * stride + p->pexp[f]] += prod;
        }
    }
}

static void cache_init(chain_ctx *c, const int32_t *z) {
    const sao_poly *p = c->p;
    int32_t stride = p->max_exp + 1;
    for (int32_t k = 0; k < p->n; ++k) {
        int64_t *a = c->cache + (int64_t)k * stride;
        for (int32_t m = 0; m < stride; ++m) a[m] = 0;
        coeffs_recompute(p, z, k, a);
    }
}

/* Metropolis acceptance min[1, exp(-dE/T)] (Sec. 3.3.1) with T = 1/beta. */
static int metropolis_accept(int64_t d, double beta, double U) {
    if (d <= 0) return 1;
    return U < exp(-(beta * (double)d));
}

/* Uniform proposal among the W-1 nonzero changes Delta z^(i) (Sec. 3.3.1). */
static int64_t metropolis_proposal(uint32_t x1, int64_t lo, int64_t W, int64_t zk) {
    int64_t v = lo + (int64_t)(((uint64_t)x1 * (uint64_t)(W - 1)) >> 32);
    if (v >= zk) v += 1;
    return v;
}

/* Heat bath (Sec. 3.3.2): P(v) = exp(-beta dE_v) / sum_j exp(-beta dE_j) over all W values,
 * the current one included.  The weights are taken relative to the minimum dE, which leaves the
 * ratios unchanged and keeps every weight in (0, 1].  The draw inverts the cumulative
 * distribution in value order: C_v = w_lo + ... + w_v, added one value at a time from the
 * lower bound up, and the first v with C_v > U * C_hi is chosen (the last value when rounding
 * puts U * C_hi at or above every C_v). */
static int64_t heat_bath_choose(chain_ctx *c, int64_t lo, int64_t W, int32_t maxe, int64_t zk,
                                double beta, double U, sao_step_info *info) {
    const int64_t *a = c->a;
    double *w = c->w;
    int64_t dmin = INT64_MAX;
    for (int64_t j = 0; j < W; ++j) {
        int64_t d = delta_from_coeffs(a, maxe, zk, lo + j);
        if (d < dmin) dmin = d;
    }
    double total = 0.0;
    for (int64_t j = 0; j < W; ++j) {
        int64_t d = delta_from_coeffs(a, maxe, zk, lo + j);
        w[j] = exp(-(beta * (double)(d - dmin)));
        total += w[j];
    }
    double thr = U * total;
    double cum = 0.0;
    int64_t pick = W - 1;
    for (int64_t j = 0; j < W; ++j) {
        cum += w[j];
        if (cum > thr) {
            pick = j;
            break;
        }
    }
    if (info) {
        /* the decision's distance from a flip: the cumulative weight nearest to the threshold */
        double run = 0.0, best = INFINITY;
        info->total = total;
        info->threshold = thr;
        for (int64_t j = 0; j < W; ++j) {
            if (j == pick) info->c_prev = run;
            run += w[j];
            if (j == pick) info->c_at = run;
            double gap = fabs(run - thr);
            if (gap < best) best = gap;
        }
        info->margin = total > 0.0 ? best / total : 0.0;
    }
    return lo + pick;
}

/* Heat bath for a variable whose energy difference is linear in the change, dE(v) = a (v - z_k)
 * (Sec. 3.3.2, multilinear case).  Index i = v - l_k has probability proportional to
 * exp(-beta a i); the paper inverts its cumulative distribution,
 *     x = -(T/a) ln[1 - U (1 - exp(-a W / T))],   v = l_k + ceil(x) - 1,
 * (its change dz = ceil(x - (z_k - l_k + 1))).  Written with c = beta |a|:
 *   a > 0:  x = g(U)        with g(q) = -log1p(q expm1(-c W)) / c,
 *   a < 0:  x = W - g(1-U)  (the same value; the paper's form overflows exp(+c W) here),
 * and ceil(x) - 1 is clamped to [0, W-1] (rounding at the ends; NaN cannot occur for c > 0).
 * With a = 0 or beta = 0 the distribution is uniform: v = l_k + floor(x1 W / 2^32). */
static int64_t heat_bath_closed(int64_t a, int64_t lo, int64_t W, double beta, double U,
                                uint32_t x1) {
    double c = beta * (double)(a < 0 ? -a : a);
    if (a == 0 || !(c > 0.0)) return lo + (int64_t)(((uint64_t)x1 * (uint64_t)W) >> 32);
    double Wd = (double)W;
    double m = expm1(-(c * Wd));
    double x;
    if (a > 0)
        x = -log1p(U * m) / c;
    else
        x = Wd + log1p((1.0 - U) * m) / c;
    int64_t i;
    if (!(x > 0.0))
        i = 0;
    else if (x >= Wd)
        i = W - 1;
    else
        i = (int64_t)ceil(x) - 1;
    return lo + i;
}

/* Returns 1 if z_k changed; *dE is the energy change applied. */
static int update_variable(chain_ctx *c, int32_t *z, int32_t k, uint32_t s, uint32_t read,
                           double beta, double r_opt, int64_t *dE, sao_step_info *info) {
    const sao_poly *p = c->p;
    int64_t lo = p->lo[k], W = (int64_t)p->hi[k] - lo + 1;
    *dE = 0;
    if (W == 1) return 0;
    uint32_t x[4];
    draw((uint32_t)k, s, read, c->inst, c->key, x);
    double U = uniform53(x);
    int64_t zk = z[k];
    int32_t maxe = p->maxe[k];
    int64_t *a = c->a;
    if (c->cache)
        memcpy(a, c->cache + (int64_t)k * (p->max_exp + 1), sizeof(int64_t) * (maxe + 1));
    else
        coeffs_recompute(p, z, k, a);

    int64_t v, d;
    int accept;
    if (c->rule == SAO_METROPOLIS) {
        v = metropolis_proposal(x[1], lo, W, zk);
        d = delta_from_coeffs(a, maxe, zk, v);
        accept = metropolis_accept(d, beta, U);
    } else if (c->rule == SAO_HEAT_BATH_CLOSED && maxe <= 1) {
        v = heat_bath_closed(maxe == 1 ? a[1] : 0, lo, W, beta, U, x[1]);
        d = delta_from_coeffs(a, maxe, zk, v);
        accept = 1;
    } else if (c->rule == SAO_HEAT_BATH || c->rule == SAO_HEAT_BATH_CLOSED) {
        v = heat_bath_choose(c, lo, W, maxe, zk, beta, U, info);
        d = delta_from_coeffs(a, maxe, zk, v);
        accept = 1;
    } else {
        /* optimal-transition Metropolis (Sec. 3.3.3): the change of smallest dE over every value
         * of the range, the unchanged value among them */
        if ((double)x[0] * 0x1p-32 < r_opt) {
            int64_t best = INT64_MAX;
            v = lo;
            for (int64_t cand = lo; cand < lo + W; ++cand) {
                int64_t dc = delta_from_coeffs(a, maxe, zk, cand);
                if (dc < best) {
                    best = dc;
                    v = cand;
                }
            }
        } else {
            v = metropolis_proposal(x[1], lo, W, zk);
        }
        d = delta_from_coeffs(a, maxe, zk, v);
        accept = metropolis_accept(d, beta, U);
        if (info) info->branch = (double)x[0] * 0x1p-32 < r_opt;
    }
    if (info) {
        info->v = v;
        info->dE = d;
        info->accepted = accept && v != zk;
        info->U = U;
        if (c->rule == SAO_METROPOLIS || c->rule == SAO_OPT_METROPOLIS) {
            info->threshold = d <= 0 ? 1.0 : exp(-(beta * (double)d));
            info->margin = d <= 0 ? INFINITY : fabs(U - info->threshold);
        }
    }
    if (!accept || v == zk) return 0;
    if (c->cache) cache_apply_move(c, z, k, v);
    z[k] = (int32_t)v;
    *dE = d;
    return 1;
}

/* ------------------------------------------------------------------------------------------ */
/* Chains                                                                                      */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    const sao_poly *p;
    int rule;
    const double *beta;
    int32_t S, s0, s1, n_reads;
    uint64_t seed;
    uint32_t inst;
    double otm_r;
    int cache_mode;
    const int32_t *z_init;
    const uint32_t *read_ids; /* NULL: row i is read i */
    int32_t *z_out;
    int64_t *e_out;
    uint64_t *hash_out; /* NULL, or (s_end - s_begin) state hashes per read */
    int tid, nthreads;
    int status;
    /* single-step mode */
    const int32_t *z_fixed;
    int32_t k_fixed, s_fixed;
    double beta_fixed, r_fixed;
    int32_t *v_out;
} job_t;

static int ctx_init(chain_ctx *c, const sao_poly *p, int rule, uint64_t seed, uint32_t inst,
                    int cache_mode) {
    memset(c, 0, sizeof *c);
    c->p = p;
    c->rule = rule;
    c->key[0] = (uint32_t)seed;
    c->key[1] = (uint32_t)(seed >> 32);
    c->inst = inst;
    c->a = (int64_t *)malloc(sizeof(int64_t) * (p->max_exp + 1));
    if (!c->a) return SAO_ENOMEM;
    if (rule == SAO_HEAT_BATH || rule == SAO_HEAT_BATH_CLOSED) {
        c->w = (double *)malloc(sizeof(double) * p->max_width);
        if (!c->w) return SAO_ENOMEM;
    }
    if (cache_mode) {
        c->cache = (int64_t *)malloc(sizeof(int64_t) * (size_t)p->n * (p->max_exp + 1));
        if (!c->cache) return SAO_ENOMEM;
    }
    return SAO_OK;
}

static void ctx_free(chain_ctx *c) {
    free(c->a);
    free(c->w);
    free(c->cache);
}

static void *anneal_worker(void *arg) {
    job_t *j = (job_t *)arg;
    const sao_poly *p = j->p;
    chain_ctx c;
    int rc = ctx_init(&c, p, j->rule, j->seed, j->inst, j->cache_mode);
    int32_t *z = (int32_t *)malloc(sizeof(int32_t) * p->n);
    if (rc != SAO_OK || !z) {
        j->status = rc != SAO_OK ? rc : SAO_ENOMEM;
        ctx_free(&c);
        free(z);
        return NULL;
    }
    for (int32_t row = j->tid; row < j->n_reads; row += j->nthreads) {
        const uint32_t r = j->read_ids ? j->read_ids[row] : (uint32_t)row;
        if (j->z_init) {
            memcpy(z, j->z_init + (int64_t)row * p->n, sizeof(int32_t) * p->n);
        } else {
            /* random initial state (Sec. 3.1), uniform on each box */
            for (int32_t k = 0; k < p->n; ++k) {
                uint32_t x[4];
                draw((uint32_t)k, 0xFFFFFFFFu, r, j->inst, c.key, x);
                int64_t W = (int64_t)p->hi[k] - p->lo[k] + 1;
                z[k] = (int32_t)(p->lo[k] + (int64_t)(((uint64_t)x[0] * (uint64_t)W) >> 32));
            }
        }
        int64_t E = energy(p, z);
        if (c.cache) cache_init(&c, z);
        for (int32_t s = j->s0; s < j->s1; ++s) {
            double beta = j->beta[s];
            double r_opt = j->otm_r >= 0.0 ? j->otm_r
                           : (j->S > 1 ? (double)s / (double)(j->S - 1) : 0.0);
            for (int32_t k = 0; k < p->n; ++k) { /* index order (Sec. 3.1) */
                int64_t d;
                if (update_variable(&c, z, k, (uint32_t)s, r, beta, r_opt, &d, NULL)) E += d;
            }
            if (j->hash_out)
                j->hash_out[(int64_t)row * (j->s1 - j->s0) + (s - j->s0)] = state_hash(p->n, z);
        }
        if (E != energy(p, z)) {
            j->status = SAO_EINTERNAL;
            break;
        }
        memcpy(j->z_out + (int64_t)row * p->n, z, sizeof(int32_t) * p->n);
        j->e_out[row] = E;
    }
    ctx_free(&c);
    free(z);
    return NULL;
}

static void *single_step_worker(void *arg) {
    job_t *j = (job_t *)arg;
    const sao_poly *p = j->p;
    chain_ctx c;
    int rc = ctx_init(&c, p, j->rule, j->seed, j->inst, 0);
    int32_t *z = (int32_t *)malloc(sizeof(int32_t) * p->n);
    if (rc != SAO_OK || !z) {
        j->status = rc != SAO_OK ? rc : SAO_ENOMEM;
        ctx_free(&c);
        free(z);
        return NULL;
    }
    memcpy(z, j->z_fixed, sizeof(int32_t) * p->n);
    int32_t k = j->k_fixed;
    for (int32_t r = j->tid; r < j->n_reads; r += j->nthreads) {
        int64_t d;
        update_variable(&c, z, k, (uint32_t)j->s_fixed, (uint32_t)r, j->beta_fixed, j->r_fixed, &d, NULL);
        j->v_out[r] = z[k];
        z[k] = j->z_fixed[k];
    }
    ctx_free(&c);
    free(z);
    return NULL;
}

int sao_default_threads(void) {
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    const char *env = getenv("OMP_NUM_THREADS");
    if (env) {
        long cap = strtol(env, NULL, 10);
        if (cap > 0 && cap < n) n = cap;
    }
    return n > 0 ? (int)n : 1;
}

static int run_jobs(job_t *tmpl, int n_threads, void *(*fn)(void *)) {
    int T = n_threads > 0 ? n_threads : sao_default_threads();
    if (T > tmpl->n_reads) T = tmpl->n_reads;
    if (T < 1) T = 1;
    job_t *jobs = (job_t *)malloc(sizeof(job_t) * T);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * T);
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return SAO_ENOMEM;
    }
    for (int t = 0; t < T; ++t) {
        jobs[t] = *tmpl;
        jobs[t].tid = t;
        jobs[t].nthreads = T;
        jobs[t].status = SAO_OK;
    }
    for (int t = 1; t < T; ++t)
        if (pthread_create(&th[t], NULL, fn, &jobs[t]) != 0) jobs[t].status = SAO_ENOMEM, th[t] = 0;
    fn(&jobs[0]);
    int rc = jobs[0].status;
    for (int t = 1; t < T; ++t) {
        if (th[t]) pthread_join(th[t], NULL);
        else {
            /* thread could not start: do its share here */
            jobs[t].status = SAO_OK;
            fn(&jobs[t]);
        }
        if (jobs[t].status != SAO_OK) rc = jobs[t].status;
    }
    free(jobs);
    free(th);
    return rc;
}

static int check_rule(const sao_poly *p, int rule) {
    if (rule < 0 || rule > 3) return SAO_EINVAL;
    /* the optimal transition is defined for energy differences of degree <= 4 (Sec. 3.3.3) */
    if (rule == SAO_OPT_METROPOLIS && p->max_exp > 4) return SAO_EUNSUPPORTED;
    return SAO_OK;
}

int sao_anneal(const sao_poly *p, int rule, const double *beta, int32_t n_sweeps,
               int32_t s_begin, int32_t s_end, int32_t n_reads, uint64_t seed,
               uint32_t instance_id, double otm_r, int cache_mode, int n_threads,
               const int32_t *z_init, int32_t *z_out, int64_t *e_out) {
    return sao_anneal_reads(p, rule, beta, n_sweeps, s_begin, s_end, n_reads, NULL, seed,
                            instance_id, otm_r, cache_mode, n_threads, z_init, z_out, e_out, NULL);
}

int sao_anneal_reads(const sao_poly *p, int rule, const double *beta, int32_t n_sweeps,
                     int32_t s_begin, int32_t s_end, int32_t n_reads, const uint32_t *read_ids,
                     uint64_t seed, uint32_t instance_id, double otm_r, int cache_mode,
                     int n_threads, const int32_t *z_init, int32_t *z_out, int64_t *e_out,
                     uint64_t *hash_out) {
    if (!p || !beta || !z_out || !e_out || n_reads < 1 || n_sweeps < 1) return SAO_EINVAL;
    if (s_begin < 0 || s_end < s_begin || s_end > n_sweeps) return SAO_EINVAL;
    int rc = check_rule(p, rule);
    if (rc != SAO_OK) return rc;
    for (int32_t s = 0; s < n_sweeps; ++s)
        if (!(beta[s] >= 0.0) || isinf(beta[s])) return SAO_EINVAL;
    if (z_init)
        for (int64_t i = 0; i < (int64_t)n_reads * p->n; ++i) {
            int32_t k = (int32_t)(i % p->n);
            if (z_init[i] < p->lo[k] || z_init[i] > p->hi[k]) return SAO_EINVAL;
        }
    job_t j;
    memset(&j, 0, sizeof j);
    j.p = p;
    j.rule = rule;
    j.beta = beta;
    j.S = n_sweeps;
    j.s0 = s_begin;
    j.s1 = s_end;
    j.n_reads = n_reads;
    j.seed = seed;
    j.inst = instance_id;
    j.otm_r = otm_r;
    j.cache_mode = cache_mode;
    j.z_init = z_init;
    j.read_ids = read_ids;
    j.z_out = z_out;
    j.e_out = e_out;
    j.hash_out = hash_out;
    return run_jobs(&j, n_threads, anneal_worker);
}

int sao_single_step(const sao_poly *p, int rule, const int32_t *z, int32_t k, int32_t s,
                    double beta, double r_opt, int32_t n_reads, uint64_t seed,
                    uint32_t instance_id, int32_t *v_out) {
    if (!p || !z || !v_out || k < 0 || k >= p->n || n_reads < 1 || s < 0) return SAO_EINVAL;
    int rc = check_rule(p, rule);
    if (rc != SAO_OK) return rc;
    job_t j;
    memset(&j, 0, sizeof j);
    j.p = p;
    j.rule = rule;
    j.n_reads = n_reads;
    j.seed = seed;
    j.inst = instance_id;
    j.z_fixed = z;
    j.k_fixed = k;
    j.s_fixed = s;
    j.beta_fixed = beta;
    j.r_fixed = r_opt;
    j.v_out = v_out;
    return run_jobs(&j, 0, single_step_worker);
}

int sao_explain_step(const sao_poly *p, int rule, const int32_t *z, int32_t k, int32_t s,
                     uint32_t read, double beta, double r_opt, uint64_t seed, uint32_t instance_id,
                     sao_step_info *out) {
    if (!p || !z || !out || k < 0 || k >= p->n || s < 0) return SAO_EINVAL;
    int rc = check_rule(p, rule);
    if (rc != SAO_OK) return rc;
    memset(out, 0, sizeof *out);
    chain_ctx c;
    rc = ctx_init(&c, p, rule, seed, instance_id, 0);
    int32_t *zz = (int32_t *)malloc(sizeof(int32_t) * p->n);
    if (rc != SAO_OK || !zz) {
        ctx_free(&c);
        free(zz);
        return rc != SAO_OK ? rc : SAO_ENOMEM;
    }
    memcpy(zz, z, sizeof(int32_t) * p->n);
    int64_t d;
    out->v = z[k];
    update_variable(&c, zz, k, (uint32_t)s, read, beta, r_opt, &d, out);
    ctx_free(&c);
    free(zz);
    return SAO_OK;
}
