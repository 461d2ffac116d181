/*
 * Aggregate risk analysis -- CPU ORACLE (test infrastructure only).
 *
 * This file is the plain, slow, obviously-correct reference that the GPU path is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline load it; the product library never links, loads or calls it, and it
 * shares no code, header or constant with the HIP sources.
 *
 * What it computes (paper: Bahl, Baltzer, Rau-Chaplin, Varghese, "Parallel
 * Simulations for Analysing Portfolios of Catastrophic Event Risk"):
 *
 *   Inputs (Section II-A): a Year Event Table of trials, each an ordered list of
 *   event occurrences; Event Loss Tables, each a set of (event, loss) records
 *   with per-ELT financial terms I; a layer = a list of ELTs plus the layer
 *   terms T = (OccR, OccL, AggR, AggL) of Table I.
 *
 *   Analysis stage (Section II-B, "Basic Algorithm for Aggregate Risk
 *   Analysis"), for every trial of the YET, in the paper's four steps:
 *     step 1  look up each occurrence's event loss in every ELT of the layer,
 *             each ELT held as a direct access table over the whole catalog
 *             (Section III-B, absent events have loss 0);
 *     step 2  apply the ELT's financial terms to each looked-up loss and
 *             accumulate the net losses across the layer's ELTs, per occurrence;
 *     step 3  apply the occurrence terms to each occurrence independently:
 *             lo_d = min(max(lo_d - OccR, 0), OccL);
 *     step 4  take the running (inclusive) cumulative sum in time order, apply
 *             the aggregate terms to it, difference it back to per-occurrence
 *             ceded losses and sum those into the trial (year) loss lr
 *             (Section II-C: one aggregate loss per trial, the YLT).
 *   Output filters (Section II-C, PML and TVaR named in Section I): computed
 *   from the sorted YLT by the rank rule documented at oracle_rank().
 *
 * Readings where the paper is silent (documented with the design):
 *   - Financial terms are undefined in the paper beyond "terms applied at the
 *     level of each individual event loss"; read as
 *     I(l) = min(max(fx*l - R, 0), L), identity for (fx, R, L) = (1, 0, +inf).
 *   - Losses are per occurrence position d (a repeated event is a separate
 *     occurrence).  The cumulative sum is inclusive (i = 1..d); the ceded loss of
 *     the first occurrence is differenced against 0; differences are taken of the
 *     pre-difference aggregate values (separate arrays, not in place).
 *   - Event IDs are 0-based in [0, catalog_size); an ELT may not list an event
 *     twice; losses must be finite and >= 0.
 *   - ELTs are accumulated in the layer's listed order, starting from +0.0.
 *
 * Arithmetic: IEEE-754 binary64, round to nearest even, no contraction (built
 * with -ffp-contract=off), sequential loops in the order written.  An optional
 * OpenMP parallel loop over trials leaves every trial's arithmetic unchanged.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_INVALID_ARG -1
#define OR_E_EVENT_ID_RANGE -2
#define OR_E_BAD_OFFSETS -3
#define OR_E_BAD_LOSS -4
#define OR_E_DUP_EVENT -5
#define OR_E_BAD_TERMS -6
#define OR_E_EMPTY -7
#define OR_E_OOM -8

static double clamp_excess(double x, double retention, double limit) {
    /* min(max(x - R, 0), L): the excess-of-loss payout of Table I. */
    double v = x - retention;
    if (v < 0.0) v = 0.0;
    if (v > limit) v = limit;
    return v;
}

static int bad_retention(double r) { return !(r >= 0.0) || isinf(r); }
static int bad_limit(double l) { return !(l >= 0.0); } /* NaN or negative; +inf allowed */

int oracle_check_layer_terms(const double *t) {
    if (!t) return OR_E_INVALID_ARG;
    if (bad_retention(t[0]) || bad_limit(t[1]) || bad_retention(t[2]) || bad_limit(t[3])) return OR_E_BAD_TERMS;
    return OR_OK;
}

/* Direct access table of one ELT over the whole catalog (Section III-B). */
static int build_dat(int32_t catalog, const int32_t *ids, const double *losses, int64_t n,
                     int dat_f32, double *dat, unsigned char *seen) {
    memset(seen, 0, (size_t)catalog);
    for (int32_t e = 0; e < catalog; ++e) dat[e] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t id = ids[i];
        double l = losses[i];
        if (id < 0 || id >= catalog) return OR_E_EVENT_ID_RANGE;
        if (!(l >= 0.0) || isinf(l)) return OR_E_BAD_LOSS;
        if (seen[id]) return OR_E_DUP_EVENT;
        seen[id] = 1;
        dat[id] = dat_f32 ? (double)(float)l : l;
    }
    return OR_OK;
}

/*
 * Analyse trials [t_begin, t_end) of the YET against one layer.
 *
 * event_ids, trial_offsets : the YET (CSR; trial t is event_ids[off[t] .. off[t+1]) in time order)
 * catalog_size             : number of catalog events; IDs in [0, catalog_size)
 * n_elts, elt_offsets      : the layer's ELTs, ELT j = pairs [elt_offsets[j], elt_offsets[j+1])
 * pair_ids, pair_losses    : concatenated (event, loss) records of all ELTs
 * elt_terms                : n_elts x (fx, R, L) financial terms, or NULL for identity
 * dat_f32                  : nonzero = each DAT entry is stored rounded to binary32
 * layer_terms              : (OccR, OccL, AggR, AggL)
 * outputs (per trial, length t_end - t_begin; NULL to skip):
 *   ylt          lr of the algorithm (sum of the per-occurrence ceded losses)
 *   occ_total    P_k, the trial's sum of occurrence-net losses
 *   gross_total  G, the trial's sum of losses net of financial terms only
 *   ylt_closed   min(max(P_k - AggR, 0), AggL), the telescoped form of lr
 *   occ_max      the trial's largest occurrence-net loss (0 for an empty trial): the
 *                year's largest single occurrence after the occurrence terms, whose
 *                distribution over trials is the occurrence exceedance curve
 * per-event outputs (length off[t_end] - off[t_begin], position relative to off[t_begin]; NULL to skip):
 *   ev_gross  loss of the occurrence summed over the layer's ELTs (after financial terms)
 *   ev_occ    after occurrence terms;  ev_cum  inclusive cumulative sum;  ev_ceded  ceded loss
 */
int oracle_analyze(const int32_t *event_ids, const int64_t *trial_offsets, int64_t t_begin, int64_t t_end,
                   int32_t catalog_size, int32_t n_elts, const int64_t *elt_offsets,
                   const int32_t *pair_ids, const double *pair_losses, const double *elt_terms,
                   int dat_f32, const double *layer_terms,
                   double *ylt, double *occ_total, double *gross_total, double *ylt_closed, double *occ_max,
                   double *ev_gross, double *ev_occ, double *ev_cum, double *ev_ceded, int n_threads) {
    if (!trial_offsets || !layer_terms || catalog_size < 1 || n_elts < 0 || t_begin < 0 || t_end < t_begin)
        return OR_E_INVALID_ARG;
    if (n_elts > 0 && (!elt_offsets || (elt_offsets[n_elts] > 0 && (!pair_ids || !pair_losses))))
        return OR_E_INVALID_ARG;
    int rc = oracle_check_layer_terms(layer_terms);
    if (rc) return rc;
    if (elt_terms) {
        for (int32_t j = 0; j < n_elts; ++j) {
            double fx = elt_terms[3 * j], r = elt_terms[3 * j + 1], l = elt_terms[3 * j + 2];
            if (!(fx >= 0.0) || isinf(fx) || bad_retention(r) || bad_limit(l)) return OR_E_BAD_TERMS;
        }
    }
    for (int64_t t = t_begin; t < t_end; ++t)
        if (trial_offsets[t + 1] < trial_offsets[t] || trial_offsets[t] < 0) return OR_E_BAD_OFFSETS;
    const int64_t ev0 = trial_offsets[t_begin];
    int64_t kmax = 0;
    for (int64_t t = t_begin; t < t_end; ++t) {
        int64_t k = trial_offsets[t + 1] - trial_offsets[t];
        if (k > kmax) kmax = k;
        for (int64_t p = trial_offsets[t]; p < trial_offsets[t + 1]; ++p)
            if (event_ids[p] < 0 || event_ids[p] >= catalog_size) return OR_E_EVENT_ID_RANGE;
    }

    /* Preprocessing stage: the layer's ELTs as direct access tables. */
    double *dat = NULL;
    if (n_elts > 0) {
        dat = (double *)malloc(sizeof(double) * (size_t)catalog_size * (size_t)n_elts);
        unsigned char *seen = (unsigned char *)malloc((size_t)catalog_size);
        if (!dat || !seen) { free(dat); free(seen); return OR_E_OOM; }
        for (int32_t j = 0; j < n_elts && rc == OR_OK; ++j) {
            int64_t a = elt_offsets[j], b = elt_offsets[j + 1];
            if (b < a) { rc = OR_E_INVALID_ARG; break; }
            rc = build_dat(catalog_size, pair_ids + a, pair_losses + a, b - a, dat_f32,
                           dat + (size_t)j * (size_t)catalog_size, seen);
        }
        free(seen);
        if (rc) { free(dat); return rc; }
    }
    const double OccR = layer_terms[0], OccL = layer_terms[1], AggR = layer_terms[2], AggL = layer_terms[3];
    if (n_threads < 1) n_threads = 1;
    int fail = 0;

#pragma omp parallel num_threads(n_threads)
    {
        /* Per-occurrence work arrays of one trial. */
        size_t kk = (size_t)(kmax > 0 ? kmax : 1);
        double *x = (double *)malloc(sizeof(double) * kk);    /* looked-up / net loss of one ELT */
        double *lo = (double *)malloc(sizeof(double) * kk);   /* accumulated, then occurrence-net */
        double *P = (double *)malloc(sizeof(double) * kk);    /* inclusive cumulative */
        double *F = (double *)malloc(sizeof(double) * kk);    /* aggregate-capped cumulative */
        double *c = (double *)malloc(sizeof(double) * kk);    /* ceded per occurrence */
        if (!x || !lo || !P || !F || !c) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t t = t_begin; t < t_end; ++t) {
                const int64_t o = trial_offsets[t];
                const int64_t k = trial_offsets[t + 1] - o;
                const int32_t *E = event_ids + o;
                for (int64_t d = 0; d < k; ++d) lo[d] = 0.0;
                /* Steps 1 and 2, for each ELT of the layer in listed order: */
                for (int32_t j = 0; j < n_elts; ++j) {
                    const double *tab = dat + (size_t)j * (size_t)catalog_size;
                    double fx = 1.0, fr = 0.0, fl = INFINITY;
                    if (elt_terms) { fx = elt_terms[3 * j]; fr = elt_terms[3 * j + 1]; fl = elt_terms[3 * j + 2]; }
                    /* look each occurrence's event up in the ELT's direct access table, */
                    for (int64_t d = 0; d < k; ++d) x[d] = tab[E[d]];
                    /* apply the ELT's financial terms to each looked-up loss, */
                    if (elt_terms)
                        for (int64_t d = 0; d < k; ++d) x[d] = clamp_excess(fx * x[d], fr, fl);
                    /* and accumulate the net losses across ELTs. */
                    for (int64_t d = 0; d < k; ++d) lo[d] += x[d];
                }
                double gsum = 0.0;
                for (int64_t d = 0; d < k; ++d) gsum += lo[d];
                if (ev_gross) for (int64_t d = 0; d < k; ++d) ev_gross[o - ev0 + d] = lo[d];
                /* Step 3: occurrence terms, each occurrence independently. */
                for (int64_t d = 0; d < k; ++d) lo[d] = clamp_excess(lo[d], OccR, OccL);
                /* Step 4: inclusive cumulative sum in time order ... */
                double run = 0.0;
                for (int64_t d = 0; d < k; ++d) { run += lo[d]; P[d] = run; }
                /* ... aggregate terms on the cumulative loss ... */
                for (int64_t d = 0; d < k; ++d) F[d] = clamp_excess(P[d], AggR, AggL);
                /* ... back to per-occurrence ceded losses (first one against 0) ... */
                for (int64_t d = 0; d < k; ++d) c[d] = F[d] - (d > 0 ? F[d - 1] : 0.0);
                /* ... summed into the trial loss. */
                double lr = 0.0;
                for (int64_t d = 0; d < k; ++d) lr += c[d];
                const int64_t r = t - t_begin;
                if (ylt) ylt[r] = lr;
                if (occ_total) occ_total[r] = run;
                if (gross_total) gross_total[r] = gsum;
                if (ylt_closed) ylt_closed[r] = clamp_excess(run, AggR, AggL);
                if (occ_max) {
                    double m = 0.0;
                    for (int64_t d = 0; d < k; ++d) m = lo[d] > m ? lo[d] : m;
                    occ_max[r] = m;
                }
                if (ev_occ) for (int64_t d = 0; d < k; ++d) ev_occ[o - ev0 + d] = lo[d];
                if (ev_cum) for (int64_t d = 0; d < k; ++d) ev_cum[o - ev0 + d] = P[d];
                if (ev_ceded) for (int64_t d = 0; d < k; ++d) ev_ceded[o - ev0 + d] = c[d];
            }
        }
        free(x); free(lo); free(P); free(F); free(c);
    }
    free(dat);
    return fail ? OR_E_OOM : OR_OK;
}

/*
 * Rank of the order statistic that a return period selects (the paper names PML
 * and TVaR but does not define them).  For N year losses sorted in descending
 * order y(1) >= ... >= y(N), the return period RP selects the k-th largest with
 * k = ceil(N / RP) clamped to [1, N]; when N / RP is within 4 ulps of an integer
 * that integer is taken (so that e.g. 49 / 4.9 gives 10, not 11).
 * Returns -1 for N < 1 or RP < 1 or NaN.
 */
int64_t oracle_rank(int64_t n, double rp) {
    if (n < 1 || !(rp >= 1.0)) return -1;
    double q = (double)n / rp;
    double r = nearbyint(q);
    double ulp = nextafter(q, INFINITY) - q;
    double k = (fabs(q - r) <= 4.0 * ulp) ? r : ceil(q);
    if (k < 1.0) k = 1.0;
    if (k > (double)n) k = (double)n;
    return (int64_t)k;
}

static int cmp_desc(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/*
 * PML and TVaR from a YLT.  PML(RP) = y(k); TVaR(RP) = (y(1) + ... + y(k)) / k,
 * summed sequentially from the largest, with k = oracle_rank(N, RP).  A TVaR at
 * tail level alpha corresponds to RP = 1 / alpha.  ranks/sorted_desc may be NULL.
 */
int oracle_risk(const double *ylt, int64_t n, const double *rps, int32_t n_rp,
                double *pml, double *tvar, int64_t *ranks, double *sorted_desc) {
    if (n < 1) return OR_E_EMPTY;
    if (!ylt || n_rp < 0 || (n_rp > 0 && (!rps || !pml || !tvar))) return OR_E_INVALID_ARG;
    for (int32_t i = 0; i < n_rp; ++i)
        if (oracle_rank(n, rps[i]) < 0) return OR_E_INVALID_ARG;
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    if (!y) return OR_E_OOM;
    for (int64_t i = 0; i < n; ++i) y[i] = ylt[i] + 0.0; /* -0.0 -> +0.0 */
    qsort(y, (size_t)n, sizeof(double), cmp_desc);
    for (int32_t i = 0; i < n_rp; ++i) {
        int64_t k = oracle_rank(n, rps[i]);
        double s = 0.0;
        for (int64_t j = 0; j < k; ++j) s += y[j];
        pml[i] = y[k - 1];
        tvar[i] = s / (double)k;
        if (ranks) ranks[i] = k;
    }
    if (sorted_desc) memcpy(sorted_desc, y, sizeof(double) * (size_t)n);
    free(y);
    return OR_OK;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
