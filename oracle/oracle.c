/*
 * oracle.c -- plain, slow, single-threaded CPU reference of the Digital
 * Annealer (DA) parallel-trial Monte Carlo step and its parallel-tempering
 * variant (Aramon et al., "Physics-Inspired Optimization for Quadratic
 * Unconstrained Problems Using a Digital Annealer", arXiv:1806.08815).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU path: every quantity it needs (the coupling matrix W
 * and bias b derived from Q, energies, local fields, the Philox generator, the
 * temperature levels, the Metropolis threshold tables, the exchange tables) is
 * computed here from its definition.
 *
 * All energies, fields and offsets are int64, so nothing here can overflow for
 * any input the library accepts.  Every loop visits every variable; there is
 * no band short-cut, no bracket table and no lazy random draw.
 *
 * Readings of points the paper leaves open (matrix convention, schedule
 * discretisation, random-number layout, tie rules) are stated where used.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EOFF_MAX (((int64_t)1) << 30)
#define ORC_THR_MAX (((int64_t)1) << 30)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): a counter-based       */
/* generator.  Ten rounds; each round multiplies counter words 0 and 2 by   */
/* the two Philox multipliers, and the key is bumped by the two Weyl        */
/* constants between rounds.                                                */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], uint64_t seed, uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    uint32_t k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter tags: which use of the generator a draw belongs to. */
enum { ORC_TAG_METROPOLIS = 0, ORC_TAG_SELECT = 1, ORC_TAG_EXCHANGE = 2, ORC_TAG_INIT = 3 };

/* 16-bit uniform draw for the Metropolis test of variable i at step s of
 * replica r: block i>>3 of the (s, r) stream, 16-bit slice i&7 (word
 * (i&7)>>1, low half first). */
uint32_t orc_metropolis_draw(uint64_t seed, uint32_t r, uint32_t s, uint32_t i)
{
    uint32_t ctr[4] = {i >> 3, s, r, ORC_TAG_METROPOLIS};
    uint32_t out[4];
    orc_philox4x32_10(ctr, seed, out);
    uint32_t word = out[(i & 7u) >> 1];
    return (i & 1u) ? (word >> 16) : (word & 0xFFFFu);
}

/* 32-bit draw that picks one of the accepted flips at step s of replica r. */
uint32_t orc_select_draw(uint64_t seed, uint32_t r, uint32_t s)
{
    uint32_t ctr[4] = {0u, s, r, ORC_TAG_SELECT};
    uint32_t out[4];
    orc_philox4x32_10(ctr, seed, out);
    return out[0];
}

/* 16-bit draw for the replica-exchange test of pair p in round t of chain c. */
uint32_t orc_exchange_draw(uint64_t seed, uint32_t c, uint32_t t, uint32_t p)
{
    uint32_t ctr[4] = {p, t, c, ORC_TAG_EXCHANGE};
    uint32_t out[4];
    orc_philox4x32_10(ctr, seed, out);
    return out[0] & 0xFFFFu;
}

/* Bit i of the random initial state of replica r. */
uint32_t orc_init_bit(uint64_t seed, uint32_t r, uint32_t i)
{
    uint32_t ctr[4] = {i >> 7, 0u, r, ORC_TAG_INIT};
    uint32_t out[4];
    orc_philox4x32_10(ctr, seed, out);
    return (out[(i >> 5) & 3u] >> (i & 31u)) & 1u;
}

/* ------------------------------------------------------------------------ */
/* Problem: minimise E(x) = x^T Q x over x in {0,1}^N (Sec. V: the DA works  */
/* on QUBO problems; any Q, not necessarily symmetric).  Off the diagonal    */
/* the pair (i,j) contributes (Q_ij + Q_ji) x_i x_j, and x_i^2 = x_i puts    */
/* Q_ii on the linear term, so                                               */
/*   W_ij = Q_ij + Q_ji (i != j), W_ii = 0, b_i = Q_ii,                      */
/*   E(x) = sum_i b_i x_i + sum_{i<j} W_ij x_i x_j.                          */
/* ------------------------------------------------------------------------ */
void orc_derive(int N, const int32_t *Q, int64_t *W, int64_t *b)
{
    for (int i = 0; i < N; ++i) {
        b[i] = (int64_t)Q[(size_t)i * N + i];
        for (int j = 0; j < N; ++j)
            W[(size_t)i * N + j] = (i == j) ? 0
                : (int64_t)Q[(size_t)i * N + j] + (int64_t)Q[(size_t)j * N + i];
    }
}

int64_t orc_energy(int N, const int64_t *W, const int64_t *b, const uint8_t *x)
{
    int64_t E = 0;
    for (int i = 0; i < N; ++i) {
        if (!x[i]) continue;
        E += b[i];
        for (int j = i + 1; j < N; ++j)
            if (x[j]) E += W[(size_t)i * N + j];
    }
    return E;
}

/* Local (effective) field h_i = b_i + sum_j W_ij x_j; flipping x_i changes the
 * energy by (1 - 2 x_i) h_i (Sec. II.A, "effective fields"). */
void orc_fields(int N, const int64_t *W, const int64_t *b, const uint8_t *x, int64_t *h)
{
    for (int i = 0; i < N; ++i) {
        int64_t acc = b[i];
        for (int j = 0; j < N; ++j)
            if (x[j]) acc += W[(size_t)i * N + j];
        h[i] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Temperatures and Metropolis thresholds.                                   */
/*                                                                           */
/* The Metropolis acceptance of a move that changes the energy by dE is     */
/* exp(-dE / T) (Sec. III, Metropolis criterion).  The test is made exact    */
/* in integers: with U_u = (u + 1/2) / 65536 for a 16-bit draw u, the move   */
/* is accepted iff U_u < exp(-d/T), i.e. iff d < -T ln U_u, i.e. (d being an */
/* integer) iff d <= ceil(-T ln U_u) - 1.  The right-hand side is the        */
/* threshold table thr_T[u].  T <= 0 accepts only d < 0.                     */
/* ------------------------------------------------------------------------ */
enum { ORC_SCHED_GEOMETRIC = 0, ORC_SCHED_LINEAR_BETA = 1 };

/* Temperature of level l of an L-level schedule from T_hi down to T_lo.
 * Geometric: T_l = T_hi (T_lo/T_hi)^(l/(L-1)).  Linear in the inverse
 * temperature (the paper's DA setting, App. A): 1/T_l interpolates linearly
 * between 1/T_hi and 1/T_lo.  One level means T_hi throughout. */
double orc_level_temperature(double T_hi, double T_lo, int kind, int L, int l)
{
    if (L <= 1) return T_hi;
    double frac = (double)l / (double)(L - 1);
    if (kind == ORC_SCHED_LINEAR_BETA)
        return 1.0 / (1.0 / T_hi + (1.0 / T_lo - 1.0 / T_hi) * frac);
    return T_hi * pow(T_lo / T_hi, frac);
}

/* Level in force at step s of an S-step run (Algorithm 2 changes the
 * temperature at intervals during the run): the run is cut into L equal
 * parts. */
int orc_level_of_step(int64_t s, int L, int64_t S)
{
    if (S <= 0) return 0;
    return (int)((s * (int64_t)L) / S);
}

/* Largest cost d accepted by draw u at temperature T (Sec. III, R4):
 * ceil(-T ln U_u) - 1 with U_u = (u + 1/2)/65536, clamped to [-1, 2^30]. */
int32_t orc_thr_entry(double T, uint32_t u)
{
    if (!(T > 0.0)) return -1;
    double U = ((double)u + 0.5) / 65536.0;
    double y = -T * log(U);
    double c = ceil(y) - 1.0;
    int64_t t;
    if (c >= (double)ORC_THR_MAX) t = ORC_THR_MAX;
    else t = (int64_t)c;
    if (t < -1) t = -1;
    return (int32_t)t;
}

void orc_threshold_table(double T, int32_t *thr)
{
    for (int u = 0; u < 65536; ++u) thr[u] = orc_thr_entry(T, (uint32_t)u);
}

/* ------------------------------------------------------------------------ */
/* One replica's state and one DA step (Algorithm 2, Sec. II.B).             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int N;
    uint8_t *x;       /* current state            */
    int64_t *h;       /* local fields of x        */
    int64_t E;        /* energy of x              */
    int64_t eoff;     /* dynamic escape offset    */
    uint8_t *best_x;  /* lowest-energy state seen */
    int64_t best_E;
    int64_t n_acc;    /* steps that applied a flip */
} orc_rep;

/* One Monte Carlo step of replica r at step index s, against the threshold
 * table thr of the temperature in force, or, when thr is NULL, against the
 * thresholds of temperature T computed per draw.  only < 0: every variable
 * proposes its flip (the DA's parallel trial, Sec. II.B); only = i: variable i
 * alone proposes (single-trial Metropolis, Sec. III).  Returns the flipped
 * variable, or -1 when no flip was accepted. */
int orc_step_T(orc_rep *st, const int64_t *W, const int32_t *thr, double T, uint64_t seed,
               uint32_t r, uint32_t s, int64_t eoff_inc, uint8_t *acc_scratch, int only)
{
    const int N = st->N;
    /* Every proposing variable's flip is tested with dE_j - E_offset. */
    int64_t m = 0;
    for (int i = 0; i < N; ++i) {
        if (only >= 0 && i != only) { acc_scratch[i] = 0; continue; }
        int64_t dE = (st->x[i] ? -st->h[i] : st->h[i]);
        int64_t d = dE - st->eoff;
        uint32_t u = orc_metropolis_draw(seed, r, s, (uint32_t)i);
        int32_t t = thr ? thr[u] : orc_thr_entry(T, u);
        acc_scratch[i] = (d <= (int64_t)t) ? 1 : 0;
        m += acc_scratch[i];
    }
    if (m == 0) {
        /* No flip accepted: raise the offset (saturating). */
        st->eoff += eoff_inc;
        if (st->eoff > ORC_EOFF_MAX) st->eoff = ORC_EOFF_MAX;
        return -1;
    }
    /* One of the m accepted flips, uniformly: j = floor(v m / 2^32) for a
     * 32-bit draw v, then the j-th accepted variable in ascending order. */
    uint32_t v = orc_select_draw(seed, r, s);
    int64_t j = (int64_t)(((uint64_t)v * (uint64_t)m) >> 32);
    int k = -1;
    for (int i = 0; i < N; ++i) {
        if (!acc_scratch[i]) continue;
        if (j == 0) { k = i; break; }
        --j;
    }
    /* Apply it: the energy changes by dE_k, every field by W_ik * delta. */
    int64_t dEk = st->x[k] ? -st->h[k] : st->h[k];
    int64_t delta = st->x[k] ? -1 : 1;
    st->E += dEk;
    st->x[k] ^= 1;
    for (int i = 0; i < N; ++i)
        st->h[i] += W[(size_t)i * N + k] * delta;
    st->eoff = 0;
    st->n_acc += 1;
    if (st->E < st->best_E) {
        st->best_E = st->E;
        memcpy(st->best_x, st->x, (size_t)N);
    }
    return k;
}

int orc_step(orc_rep *st, const int64_t *W, const int32_t *thr, uint64_t seed,
             uint32_t r, uint32_t s, int64_t eoff_inc, uint8_t *acc_scratch)
{
    return orc_step_T(st, W, thr, 0.0, seed, r, s, eoff_inc, acc_scratch, -1);
}

/* Initial state of replica r: zeros (every run starts from the same state,
 * Algorithm 2; zeros in the paper's runs, App. A) or random bits. */
enum { ORC_INIT_ZEROS = 0, ORC_INIT_RANDOM = 1 };

static void orc_init_state(orc_rep *st, const int64_t *W, const int64_t *b,
                           int init, uint64_t seed, uint32_t r)
{
    const int N = st->N;
    for (int i = 0; i < N; ++i)
        st->x[i] = (init == ORC_INIT_RANDOM) ? (uint8_t)orc_init_bit(seed, r, (uint32_t)i) : 0;
    orc_fields(N, W, b, st->x, st->h);
    st->E = orc_energy(N, W, b, st->x);
    st->eoff = 0;
    memcpy(st->best_x, st->x, (size_t)N);
    st->best_E = st->E;
    st->n_acc = 0;
}

/* Run R replicas (ids replica_base .. replica_base+R-1) for S steps each
 * through an L-level schedule; L = 0 changes the temperature every step (the
 * paper's DA runs, App. A): step s runs at level s of an S-level schedule.
 * Outputs are [R][N] states and [R] scalars;
 * any output pointer may be NULL.  Trace arrays, when given, are [R][S]:
 * the flipped variable (or -1), and E and E_offset after the step.
 * Returns 0, or -1 on bad arguments / allocation failure. */
int orc_anneal(int N, const int32_t *Q, double T_hi, double T_lo, int kind, int L,
               int64_t eoff_inc, int init, int trial, int64_t replica_base, int R, int64_t S,
               uint64_t seed,
               uint8_t *best_x, int64_t *best_E, uint8_t *final_x, int64_t *final_E,
               int64_t *n_acc,
               int32_t *trace_k, int64_t *trace_E, int64_t *trace_eoff)
{
    if (N < 1 || R < 0 || S < 0 || L < 0) return -1;
    const int per_step = (L == 0);
    int64_t *W = malloc(sizeof(int64_t) * (size_t)N * N);
    int64_t *b = malloc(sizeof(int64_t) * (size_t)N);
    int32_t *thr = malloc(sizeof(int32_t) * (size_t)(per_step ? 1 : L) * 65536);
    uint8_t *scratch = malloc((size_t)N);
    orc_rep st;
    st.N = N;
    st.x = malloc((size_t)N);
    st.best_x = malloc((size_t)N);
    st.h = malloc(sizeof(int64_t) * (size_t)N);
    if (!W || !b || !thr || !scratch || !st.x || !st.best_x || !st.h) {
        free(W); free(b); free(thr); free(scratch); free(st.x); free(st.best_x); free(st.h);
        return -1;
    }
    orc_derive(N, Q, W, b);
    for (int l = 0; l < L; ++l)
        orc_threshold_table(orc_level_temperature(T_hi, T_lo, kind, L, l), thr + (size_t)l * 65536);
    if (per_step && S > (int64_t)1 << 30) {
        free(W); free(b); free(thr); free(scratch); free(st.x); free(st.best_x); free(st.h);
        return -1;
    }

    for (int rr = 0; rr < R; ++rr) {
        uint32_t r = (uint32_t)(replica_base + rr);
        orc_init_state(&st, W, b, init, seed, r);
        for (int64_t s = 0; s < S; ++s) {
            /* single trial: sequential sweeps, variable s mod N at step s */
            const int only = trial ? (int)(s % N) : -1;
            int k;
            if (per_step) {
                double T = orc_level_temperature(T_hi, T_lo, kind, (int)S, (int)s);
                k = orc_step_T(&st, W, NULL, T, seed, r, (uint32_t)s, eoff_inc, scratch, only);
            } else {
                int l = orc_level_of_step(s, L, S);
                k = orc_step_T(&st, W, thr + (size_t)l * 65536, 0.0, seed, r, (uint32_t)s,
                               eoff_inc, scratch, only);
            }
            if (trace_k) trace_k[(size_t)rr * S + s] = k;
            if (trace_E) trace_E[(size_t)rr * S + s] = st.E;
            if (trace_eoff) trace_eoff[(size_t)rr * S + s] = st.eoff;
        }
        if (best_x) memcpy(best_x + (size_t)rr * N, st.best_x, (size_t)N);
        if (final_x) memcpy(final_x + (size_t)rr * N, st.x, (size_t)N);
        if (best_E) best_E[rr] = st.best_E;
        if (final_E) final_E[rr] = st.E;
        if (n_acc) n_acc[rr] = st.n_acc;
    }
    free(W); free(b); free(thr); free(scratch); free(st.x); free(st.best_x); free(st.h);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Parallel tempering with DA steps (Sec. II.D; the exchange move of         */
/* Algorithm 3).  Chain c holds M replicas (ids c*M + m) at the strictly     */
/* increasing temperatures T_0 < ... < T_{M-1}; replica m starts in slot m   */
/* from a random state.  A round runs K DA steps in every replica at the     */
/* temperature of its slot (global step index t*K + q), then for p = 0..M-2  */
/* in ascending order proposes to swap the temperatures of the replicas in   */
/* slots p and p+1.  With a, b those replicas the swap is accepted with      */
/* probability min(1, exp((1/T_p - 1/T_{p+1}) (E_a - E_b))), tested as       */
/* ln U_u < (1/T_p - 1/T_{p+1}) * (E_a - E_b) with U_u = (u + 1/2)/65536.    */
/* ------------------------------------------------------------------------ */
/* One exchange sweep of a chain (the exchange move of Algorithm 3): for
 * p = 0 .. M-2 in ascending order, the replicas a, b now in slots p and p+1
 * (after any swap made earlier in the same sweep) exchange temperatures with
 * probability min(1, exp((1/T_p - 1/T_{p+1}) (E_a - E_b))), tested as
 * ln U_u < (1/T_p - 1/T_{p+1}) (E_a - E_b), u the 16-bit exchange draw of
 * (chain c, round t, pair p).  E[q] is the energy of the chain's replica q;
 * replica_in_slot is updated in place; accepted swaps of pair p are added to
 * pair_swaps[p] when it is given.  Returns the number of accepted swaps. */
int64_t orc_pt_sweep(int M, const int64_t *E, const double *temps, const double *lnU,
                     int *replica_in_slot, uint64_t seed, uint32_t c, uint32_t t,
                     int64_t *pair_swaps)
{
    int64_t swaps = 0;
    for (int p = 0; p + 1 < M; ++p) {
        int a = replica_in_slot[p], bq = replica_in_slot[p + 1];
        double dbeta = 1.0 / temps[p] - 1.0 / temps[p + 1];
        double delta = dbeta * (double)(E[a] - E[bq]);
        uint32_t u = orc_exchange_draw(seed, c, t, (uint32_t)p);
        if (lnU[u] < delta) {
            replica_in_slot[p] = bq;
            replica_in_slot[p + 1] = a;
            ++swaps;
            if (pair_swaps) pair_swaps[p] += 1;
        }
    }
    return swaps;
}

/* Parallel tempering of chains chain_base .. chain_base+chains-1 (outputs
 * indexed from 0 for the first of them).  Optional extra outputs:
 * slot_trace [chains][rounds][M], the slot of each replica after every
 * round's exchange sweep; pair_swaps [chains][M-1], accepted swaps per pair. */
int orc_pt_ex(int N, const int32_t *Q, const double *temps, int M, int64_t chain_base,
              int chains, int64_t rounds, int K, int64_t eoff_inc, uint64_t seed,
              uint8_t *best_x, int64_t *best_E, uint8_t *final_x, int64_t *final_E,
              int64_t *n_acc, int32_t *slot_of_replica, int64_t *n_swaps,
              int32_t *slot_trace, int64_t *pair_swaps)
{
    if (N < 1 || M < 1 || chains < 0 || rounds < 0 || K < 0 || chain_base < 0) return -1;
    for (int p = 0; p < M; ++p) {
        if (!(temps[p] > 0.0)) return -1;
        if (p + 1 < M && !(temps[p] < temps[p + 1])) return -1;
    }
    int64_t *W = malloc(sizeof(int64_t) * (size_t)N * N);
    int64_t *b = malloc(sizeof(int64_t) * (size_t)N);
    int32_t *thr = malloc(sizeof(int32_t) * (size_t)M * 65536);
    double *lnU = malloc(sizeof(double) * 65536);
    uint8_t *scratch = malloc((size_t)N);
    orc_rep *reps = calloc((size_t)M, sizeof(orc_rep));
    int64_t *E = malloc(sizeof(int64_t) * (size_t)M);
    int *replica_in_slot = malloc(sizeof(int) * (size_t)M);
    int fail = !W || !b || !thr || !lnU || !scratch || !reps || !E || !replica_in_slot;
    for (int q = 0; q < M && !fail; ++q) {
        reps[q].N = N;
        reps[q].x = malloc((size_t)N);
        reps[q].best_x = malloc((size_t)N);
        reps[q].h = malloc(sizeof(int64_t) * (size_t)N);
        fail = !reps[q].x || !reps[q].best_x || !reps[q].h;
    }
    if (!fail) {
        orc_derive(N, Q, W, b);
        for (int p = 0; p < M; ++p) orc_threshold_table(temps[p], thr + (size_t)p * 65536);
        for (int u = 0; u < 65536; ++u) lnU[u] = log(((double)u + 0.5) / 65536.0);
        for (int cc = 0; cc < chains; ++cc) {
            const uint32_t c = (uint32_t)(chain_base + cc);
            /* replica m of chain c has id c*M + m and starts in slot m */
            for (int m = 0; m < M; ++m) {
                orc_init_state(&reps[m], W, b, ORC_INIT_RANDOM, seed, c * (uint32_t)M + (uint32_t)m);
                replica_in_slot[m] = m;
            }
            int64_t swaps = 0;
            for (int64_t t = 0; t < rounds; ++t) {
                /* K DA steps in every replica at the temperature of its slot */
                for (int p = 0; p < M; ++p) {
                    int q = replica_in_slot[p];
                    for (int i = 0; i < K; ++i) {
                        uint32_t s = (uint32_t)(t * K + i);
                        orc_step(&reps[q], W, thr + (size_t)p * 65536, seed,
                                 c * (uint32_t)M + (uint32_t)q, s, eoff_inc, scratch);
                    }
                }
                for (int q = 0; q < M; ++q) E[q] = reps[q].E;
                swaps += orc_pt_sweep(M, E, temps, lnU, replica_in_slot, seed, c, (uint32_t)t,
                                      pair_swaps ? pair_swaps + (size_t)cc * (M - 1) : NULL);
                if (slot_trace)
                    for (int p = 0; p < M; ++p)
                        slot_trace[((size_t)cc * rounds + t) * M + replica_in_slot[p]] = p;
            }
            for (int m = 0; m < M; ++m) {
                size_t q = (size_t)cc * M + m;
                if (best_x) memcpy(best_x + q * N, reps[m].best_x, (size_t)N);
                if (final_x) memcpy(final_x + q * N, reps[m].x, (size_t)N);
                if (best_E) best_E[q] = reps[m].best_E;
                if (final_E) final_E[q] = reps[m].E;
                if (n_acc) n_acc[q] = reps[m].n_acc;
            }
            if (slot_of_replica)
                for (int p = 0; p < M; ++p) slot_of_replica[(size_t)cc * M + replica_in_slot[p]] = p;
            if (n_swaps) n_swaps[cc] = swaps;
        }
    }
    for (int q = 0; q < M && reps; ++q) {
        free(reps[q].x); free(reps[q].best_x); free(reps[q].h);
    }
    free(W); free(b); free(thr); free(lnU); free(scratch); free(reps); free(E);
    free(replica_in_slot);
    return fail ? -1 : 0;
}

int orc_pt(int N, const int32_t *Q, const double *temps, int M, int chains,
           int64_t rounds, int K, int64_t eoff_inc, uint64_t seed,
           uint8_t *best_x, int64_t *best_E, uint8_t *final_x, int64_t *final_E,
           int64_t *n_acc, int32_t *slot_of_replica, int64_t *n_swaps)
{
    return orc_pt_ex(N, Q, temps, M, 0, chains, rounds, K, eoff_inc, seed, best_x, best_E,
                     final_x, final_E, n_acc, slot_of_replica, n_swaps, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Adaptive temperature ladder (Sec. II.D: the PTDA sets its temperatures    */
/* by the adaptive scheme of Hukushima et al.; the lowest and highest        */
/* temperatures stay fixed and the ones between are moved toward equal       */
/* replica-exchange acceptance for every adjacent pair).                     */
/*                                                                           */
/* One update, in inverse temperatures beta_p = 1/T_p (decreasing in p):     */
/* with interval d_p = beta_p - beta_{p+1} and measured acceptance A_p of    */
/* pair p (accepted / proposals, floored at half a swap so that no interval  */
/* collapses), the new intervals are proportional to d_p * A_p and fill the  */
/* fixed span beta_0 - beta_{M-1}:                                           */
/*   d'_p = (beta_0 - beta_{M-1}) * (w_p / sum_q w_q),  w_p = d_p * A_p,      */
/*   beta'_0 = beta_0,  beta'_{p+1} = beta'_p - d'_p,  T'_{M-1} = T_{M-1}.    */
/* A pair that accepts more than the others gets a wider interval (which      */
/* lowers its acceptance) and one that accepts less a narrower one; equal     */
/* acceptances are the fixed point.                                          */
/* ------------------------------------------------------------------------ */
void orc_ladder_update(int M, const double *temps, const int64_t *accepted, int64_t proposals,
                       double *out)
{
    for (int p = 0; p < M; ++p) out[p] = temps[p];
    if (M < 3 || proposals < 1) return;
    double beta_lo_T = 1.0 / temps[0];          /* coldest: largest beta */
    double beta_hi_T = 1.0 / temps[M - 1];
    double floor_acc = 0.5 / (double)proposals;
    double total = 0.0;
    double *w = malloc(sizeof(double) * (size_t)(M - 1));
    if (!w) return;
    for (int p = 0; p + 1 < M; ++p) {
        double acc = (double)accepted[p] / (double)proposals;
        if (acc < floor_acc) acc = floor_acc;
        w[p] = (1.0 / temps[p] - 1.0 / temps[p + 1]) * acc;
        total += w[p];
    }
    double beta = beta_lo_T;
    for (int p = 0; p + 2 < M; ++p) {
        beta = beta - (beta_lo_T - beta_hi_T) * (w[p] / total);
        out[p + 1] = 1.0 / beta;
    }
    free(w);
}

/* Ladder adaptation by repeated PT runs: iteration i runs `chains` chains of
 * `rounds` rounds (K DA steps each, random starts, seed + i) on the current
 * ladder, measures every pair's acceptance over all chains and rounds, and
 * updates the ladder.  temps is updated in place; acceptance [iterations][M-1]
 * (nullable) receives the measured acceptances of each iteration. */
int orc_pt_adapt(int N, const int32_t *Q, double *temps, int M, int chains, int iterations,
                 int64_t rounds, int K, int64_t eoff_inc, uint64_t seed, double *acceptance)
{
    if (M < 2 || chains < 1 || iterations < 0 || rounds < 1) return -1;
    int64_t *ps = calloc((size_t)chains * (size_t)(M - 1), sizeof(int64_t));
    int64_t *acc = malloc(sizeof(int64_t) * (size_t)(M - 1));
    double *next = malloc(sizeof(double) * (size_t)M);
    if (!ps || !acc || !next) { free(ps); free(acc); free(next); return -1; }
    int rc = 0;
    for (int it = 0; it < iterations && rc == 0; ++it) {
        memset(ps, 0, sizeof(int64_t) * (size_t)chains * (size_t)(M - 1));
        rc = orc_pt_ex(N, Q, temps, M, 0, chains, rounds, K, eoff_inc, seed + (uint64_t)it,
                       NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, ps);
        if (rc) break;
        const int64_t proposals = (int64_t)chains * rounds;
        for (int p = 0; p + 1 < M; ++p) {
            acc[p] = 0;
            for (int c = 0; c < chains; ++c) acc[p] += ps[(size_t)c * (M - 1) + p];
            if (acceptance)
                acceptance[(size_t)it * (M - 1) + p] = (double)acc[p] / (double)proposals;
        }
        orc_ladder_update(M, temps, acc, proposals, next);
        for (int p = 0; p < M; ++p) temps[p] = next[p];
    }
    free(ps); free(acc); free(next);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Step-level access for the invariant tests: build a replica state, step it */
/* one Monte Carlo step at a time, read it back.                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    orc_rep st;
    int64_t *W;
    int64_t *b;
    uint8_t *scratch;
} orc_handle;

void *orc_rep_new(int N, const int32_t *Q, int init, uint64_t seed, uint32_t r)
{
    orc_handle *hd = calloc(1, sizeof(orc_handle));
    if (!hd) return NULL;
    hd->st.N = N;
    hd->st.x = malloc((size_t)N);
    hd->st.best_x = malloc((size_t)N);
    hd->st.h = malloc(sizeof(int64_t) * (size_t)N);
    hd->W = malloc(sizeof(int64_t) * (size_t)N * N);
    hd->b = malloc(sizeof(int64_t) * (size_t)N);
    hd->scratch = malloc((size_t)N);
    if (!hd->st.x || !hd->st.best_x || !hd->st.h || !hd->W || !hd->b || !hd->scratch) {
        free(hd->st.x); free(hd->st.best_x); free(hd->st.h); free(hd->W); free(hd->b);
        free(hd->scratch); free(hd);
        return NULL;
    }
    orc_derive(N, Q, hd->W, hd->b);
    orc_init_state(&hd->st, hd->W, hd->b, init, seed, r);
    return hd;
}

int orc_rep_step(void *handle, const int32_t *thr, uint64_t seed, uint32_t r, uint32_t s,
                 int64_t eoff_inc)
{
    orc_handle *hd = (orc_handle *)handle;
    return orc_step(&hd->st, hd->W, thr, seed, r, s, eoff_inc, hd->scratch);
}

/* Copies x, h and best_x out, and E, eoff, best_E, n_acc into scalars[4]. */
void orc_rep_read(void *handle, uint8_t *x, int64_t *h, uint8_t *best_x, int64_t *scalars)
{
    orc_handle *hd = (orc_handle *)handle;
    int N = hd->st.N;
    if (x) memcpy(x, hd->st.x, (size_t)N);
    if (h) memcpy(h, hd->st.h, sizeof(int64_t) * (size_t)N);
    if (best_x) memcpy(best_x, hd->st.best_x, (size_t)N);
    if (scalars) {
        scalars[0] = hd->st.E;
        scalars[1] = hd->st.eoff;
        scalars[2] = hd->st.best_E;
        scalars[3] = hd->st.n_acc;
    }
}

void orc_rep_free(void *handle)
{
    orc_handle *hd = (orc_handle *)handle;
    if (!hd) return;
    free(hd->st.x); free(hd->st.best_x); free(hd->st.h); free(hd->W); free(hd->b);
    free(hd->scratch); free(hd);
}

/* Exact minimum of E over all 2^N states (N <= 24) by Gray-code enumeration:
 * consecutive codes differ in one bit, so each new energy is the previous one
 * plus (1 - 2 x_i) h_i, with h kept up to date.  Returns the minimum energy
 * and the number of states attaining it. */
int orc_bruteforce(int N, const int32_t *Q, int64_t *E_min, int64_t *n_min, uint8_t *argmin)
{
    if (N < 1 || N > 24) return -1;
    int64_t *W = malloc(sizeof(int64_t) * (size_t)N * N);
    int64_t *b = malloc(sizeof(int64_t) * (size_t)N);
    int64_t *h = malloc(sizeof(int64_t) * (size_t)N);
    uint8_t *x = calloc((size_t)N, 1);
    if (!W || !b || !h || !x) { free(W); free(b); free(h); free(x); return -1; }
    orc_derive(N, Q, W, b);
    for (int i = 0; i < N; ++i) h[i] = b[i];
    int64_t E = 0, best = 0, count = 1;
    if (argmin) memset(argmin, 0, (size_t)N);
    uint64_t total = (uint64_t)1 << N;
    for (uint64_t g = 1; g < total; ++g) {
        int i = __builtin_ctzll(g);      /* bit that changes from code g-1 to g */
        int64_t delta = x[i] ? -1 : 1;
        E += x[i] ? -h[i] : h[i];
        x[i] ^= 1;
        for (int j = 0; j < N; ++j) h[j] += W[(size_t)j * N + i] * delta;
        if (E < best) {
            best = E; count = 1;
            if (argmin) memcpy(argmin, x, (size_t)N);
        } else if (E == best) {
            ++count;
        }
    }
    *E_min = best;
    *n_min = count;
    free(W); free(b); free(h); free(x);
    return 0;
}
