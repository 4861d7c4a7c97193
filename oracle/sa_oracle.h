/*
 * sa_oracle.h -- plain sequential CPU oracle for direct simulated annealing of QUIO/HUIO
 * problems (K. Suzuki, "Simulated Annealing for Quadratic and Higher-Order Unconstrained
 * Integer Optimization", arXiv:2511.17245).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference for the GPU path:
 * only the test-suite, the smoke entry and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU library; the two agree only
 * through the paper's definitions and the random-number contract stated below.
 *
 * Random-number contract (the paper leaves the generator open): Philox4x32-10 (Salmon,
 * Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), counter
 * (variable k, sweep s, read r, instance id), key (seed low 32 bits, seed high 32 bits).
 * The initial state uses sweep id 0xFFFFFFFF.
 *
 * Status codes: 0 ok, -1 invalid argument, -2 int64 bound exceeded, -3 unsupported
 * (optimal-transition Metropolis with an exponent above four), -4 out of memory,
 * -8 internal invariant violated (tracked energy differs from recomputation).
 */
#ifndef SA_ORACLE_H
#define SA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SAO_OK 0
#define SAO_EINVAL (-1)
#define SAO_ERANGE (-2)
#define SAO_EUNSUPPORTED (-3)
#define SAO_ENOMEM (-4)
#define SAO_EINTERNAL (-8)

#define SAO_METROPOLIS 0
#define SAO_HEAT_BATH 1
#define SAO_OPT_METROPOLIS 2
/* Heat bath with the closed-form draw of Sec. 3.3.2 for every variable whose energy
 * difference is linear in its change (it appears in no term with an exponent above one);
 * other variables use the enumeration of SAO_HEAT_BATH. */
#define SAO_HEAT_BATH_CLOSED 3

typedef struct sao_poly sao_poly;

/* Canonicalise a raw polynomial (merge equal factor multisets, drop zero coefficients,
 * Sec. 2) and check the integer box and the int64 bound.  Inputs are borrowed. */
int sao_poly_build(int32_t n_vars, int64_t n_terms, const int64_t *term_ptr,
                   const int32_t *factor_var, const int64_t *coef, const int32_t *lower,
                   const int32_t *upper, sao_poly **out);
void sao_poly_free(sao_poly *p);

/* Canonical form: number of terms, total (var, exponent) pairs, and an export of them. */
int64_t sao_poly_n_terms(const sao_poly *p);
int64_t sao_poly_n_pairs(const sao_poly *p);
int sao_poly_export(const sao_poly *p, int64_t *tptr, int32_t *var, int32_t *expo, int64_t *coef);
int32_t sao_poly_max_exponent(const sao_poly *p);

/* E(z) = sum_t J_t prod z_i^e (exact int64). */
int sao_energy(const sao_poly *p, const int32_t *z, int64_t *out);

/* Energy change of setting z_k to v, through the per-variable polynomial coefficients
 * a_k^(m) (Sec. 3.2, HUIO energy difference). */
int sao_delta(const sao_poly *p, const int32_t *z, int32_t k, int32_t v, int64_t *out);

/* The automatic schedule of Sec. 3.4 with geometric cooling (Sec. 3.1): fills beta[0..S-1]
 * and returns T_init and T_final. */
int sao_schedule(const sao_poly *p, int32_t n_sweeps, double *beta_out, double *t_init,
                 double *t_final);

/* One Philox4x32-10 block. */
void sao_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Anneal n_reads independent chains through sweeps [s_begin, s_end) of an S-sweep schedule
 * beta[0..S-1].  z_init (n_reads x n_vars) may be NULL: then the chains start from the
 * random initial state.  cache_mode 0 recomputes a_k^(m) at every visit; cache_mode 1 keeps
 * the paper's coefficient cache and updates it on accepted moves (Sec. 3.2).  otm_r < 0 uses
 * the paper's r = s/(S-1); otherwise r is held at otm_r.  n_threads <= 0 uses every core.
 * Outputs: final states (n_reads x n_vars) and tracked energies (n_reads). */
int sao_anneal(const sao_poly *p, int rule, const double *beta, int32_t n_sweeps,
               int32_t s_begin, int32_t s_end, int32_t n_reads, uint64_t seed,
               uint32_t instance_id, double otm_r, int cache_mode, int n_threads,
               const int32_t *z_init, int32_t *z_out, int64_t *e_out);

/* As sao_anneal, but output row i is the chain with read id read_ids[i] (read_ids NULL: read i),
 * so a sample of the reads of a large run can be reproduced one by one.  hash_out, when not
 * NULL, receives (s_end - s_begin) state hashes per read (row-major): the hash of the state
 * after each sweep, as sao_state_hash defines it. */
int sao_anneal_reads(const sao_poly *p, int rule, const double *beta, int32_t n_sweeps,
                     int32_t s_begin, int32_t s_end, int32_t n_reads, const uint32_t *read_ids,
                     uint64_t seed, uint32_t instance_id, double otm_r, int cache_mode,
                     int n_threads, const int32_t *z_init, int32_t *z_out, int64_t *e_out,
                     uint64_t *hash_out);

/* Hash of a state: sum over k of mix(k * 2^32 + (uint32_t)z[k]) modulo 2^64, where mix is the
 * 64-bit finaliser of SplitMix64.  Order-independent (a sum), so that runs partitioned in any
 * way can report it; used only to find the first sweep at which two runs of a chain part. */
uint64_t sao_state_hash(int32_t n, const int32_t *z);
/* The mixing function of the state hash (exported so that tests can pin it). */
uint64_t sao_mix64(uint64_t x);

/* For each read r in [0, n_reads): from the state z, perform the single update of variable
 * k at sweep index s with inverse temperature beta and OTM parameter r_opt, and report the
 * new value of z_k (read-keyed draws are independent samples of one transition). */
int sao_single_step(const sao_poly *p, int rule, const int32_t *z, int32_t k, int32_t s,
                    double beta, double r_opt, int32_t n_reads, uint64_t seed,
                    uint32_t instance_id, int32_t *v_out);

/* What one update computed, for explaining a parting of two runs of a chain. */
typedef struct {
    int64_t v;          /* value drawn (heat bath) or proposed (Metropolis, OTM) */
    int64_t dE;         /* energy change of moving z_k to v */
    int32_t accepted;   /* 1 if z_k moved to v */
    int32_t branch;     /* OTM: 1 if the optimal-transition branch was taken */
    double U;           /* the uniform number of the update */
    double threshold;   /* Metropolis, OTM: exp(-beta dE) (1 for dE <= 0); heat bath: U * total */
    double total;       /* heat bath: sum of the weights exp(-beta (dE_v - min dE)) */
    double c_prev;      /* heat bath: cumulative weight before the drawn value */
    double c_at;        /* heat bath: cumulative weight at the drawn value */
    double margin;      /* distance of the decision from a flip: heat bath min_v |C_v - U total| / total,
                           Metropolis and OTM |U - threshold| (infinite when dE <= 0) */
} sao_step_info;

/* Recomputes the update of variable k at sweep s of read `read` from state z and reports it. */
int sao_explain_step(const sao_poly *p, int rule, const int32_t *z, int32_t k, int32_t s,
                     uint32_t read, double beta, double r_opt, uint64_t seed, uint32_t instance_id,
                     sao_step_info *out);

/* Hardware threads the oracle would use for n_threads <= 0. */
int sao_default_threads(void);

#ifdef __cplusplus
}
#endif
#endif
