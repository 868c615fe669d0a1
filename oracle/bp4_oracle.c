/*
 * bp4_oracle.c -- plain FP64 CPU oracle for flooding-schedule LLR belief
 * propagation over GF(4) and the paper's three variants (Momentum-BP,
 * AdaGrad-BP, EWAInit-BP), with its own error sampler and logical-error
 * bookkeeping.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  It shares no source, header, table or
 * helper with the GPU library; the two meet only through seeded inputs.
 *
 * Paper: Chen, Yi, Liang, Wang, "Improved Belief Propagation Decoding
 * Algorithms for Surface Codes" (arXiv 2407.11523).  Every step below cites
 * the section / equation it follows.  Readings where the paper is silent or
 * garbled are marked READING and listed in the design notes.
 *
 * Conventions
 *   Pauli code per qubit: bit0 = x, bit1 = z  (I=0, X=1, Z=2, Y=3).
 *   Per-qubit LLR triples are ordered (X, Y, Z), the order of section II-B1.
 *   Canonical edge order: nonzeros of H in row-major order (check, then qubit).
 *   Syndrome bits s_c in {0,1}; the check sign is (-1)^{s_c} (eq. h_update).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (no -ffast-math: IEEE semantics needed).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC'11).  Written from the published definition: ten     */
/* rounds of two 64x64->128 multiplies with the published multipliers, key   */
/* bumped by the published Weyl constants between rounds.                    */
/* ------------------------------------------------------------------------- */

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * x0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------- */
/* Tanner graph (section II-B1): check c has neighbours N(c), qubit v has     */
/* neighbours M(v); edge label H_cv is the Pauli of stabilizer c on qubit v.  */
/* ------------------------------------------------------------------------- */

typedef struct {
    int m, n, nnz;
    int *cptr;   /* [m+1] edges of check c are cptr[c] .. cptr[c+1]-1 (canonical order) */
    int *evar;   /* [nnz] qubit of edge e */
    int *echk;   /* [nnz] check of edge e */
    int *elab;   /* [nnz] Pauli code of H_cv on edge e (1, 2 or 3) */
    int *vptr;   /* [n+1] */
    int *vedge;  /* [nnz] edges of qubit v, in increasing check order */
} or_graph;

static void graph_free(or_graph *g)
{
    free(g->cptr); free(g->evar); free(g->echk); free(g->elab);
    free(g->vptr); free(g->vedge);
}

static int graph_build(int m, int n, const uint8_t *hx, const uint8_t *hz, or_graph *g)
{
    memset(g, 0, sizeof(*g));
    g->m = m; g->n = n;
    int nnz = 0;
    for (long i = 0; i < (long)m * n; ++i) nnz += (hx[i] | hz[i]) ? 1 : 0;
    g->nnz = nnz;
    g->cptr = calloc((size_t)m + 1, sizeof(int));
    g->evar = calloc((size_t)nnz + 1, sizeof(int));
    g->echk = calloc((size_t)nnz + 1, sizeof(int));
    g->elab = calloc((size_t)nnz + 1, sizeof(int));
    g->vptr = calloc((size_t)n + 1, sizeof(int));
    g->vedge = calloc((size_t)nnz + 1, sizeof(int));
    if (!g->cptr || !g->evar || !g->echk || !g->elab || !g->vptr || !g->vedge) {
        graph_free(g);
        return -1;
    }
    int e = 0;
    for (int c = 0; c < m; ++c) {
        g->cptr[c] = e;
        for (int v = 0; v < n; ++v) {
            int lab = (hx[(long)c * n + v] & 1) | ((hz[(long)c * n + v] & 1) << 1);
            if (lab) {
                g->evar[e] = v; g->echk[e] = c; g->elab[e] = lab;
                g->vptr[v + 1]++;
                ++e;
            }
        }
    }
    g->cptr[m] = e;
    for (int v = 0; v < n; ++v) g->vptr[v + 1] += g->vptr[v];
    int *fill = calloc((size_t)n + 1, sizeof(int));
    if (!fill) { graph_free(g); return -1; }
    for (int k = 0; k < nnz; ++k) {       /* canonical order visits checks increasingly */
        int v = g->evar[k];
        g->vedge[g->vptr[v] + fill[v]++] = k;
    }
    free(fill);
    return 0;
}

/* Symplectic product of two single-qubit Pauli codes: 1 iff they anticommute. */
static int anticommute(int a, int b)
{
    return ((a & 1) & ((b >> 1) & 1)) ^ (((a >> 1) & 1) & (b & 1));
}

/* Index of a non-identity Pauli code in the (X, Y, Z) LLR triple. */
static int triple_index(int pauli)
{
    return pauli == 1 ? 0 : (pauli == 3 ? 1 : 2);
}

/* Pauli code of triple index 0,1,2 = X, Y, Z. */
static const int PAULI_OF_INDEX[3] = {1, 3, 2};

/* ------------------------------------------------------------------------- */
/* Elementary functions                                                       */
/* ------------------------------------------------------------------------- */

/* log(exp(a) + exp(b)), evaluated without overflow. */
static double lse2(double a, double b)
{
    double hi = a > b ? a : b, lo = a > b ? b : a;
    if (hi == -INFINITY) return -INFINITY;
    return hi + log1p(exp(lo - hi));
}

/*
 * lambda_H of section II-B1: the LLR that the qubit's error commutes with the
 * stabilizer entry H, given the qubit's (X, Y, Z) LLRs L:
 *     ln[(1 + e^{-L_H}) / (e^{-L_X} + e^{-L_Y} + e^{-L_Z} - e^{-L_H})].
 * The denominator is the sum over the two Paulis that anticommute with H, so
 * it is evaluated as that two-term sum (same value, no cancellation):
 *     lambda = LSE(0, -L_H) - LSE(-L_a, -L_b),  {a, b} = {X, Y, Z} \ {H}.
 */
static double lambda_h(int H, const double L[3])
{
    int h = triple_index(H);
    int a = (h + 1) % 3, b = (h + 2) % 3;
    return lse2(0.0, -L[h]) - lse2(-L[a], -L[b]);
}

/*
 * phi(x) = -ln tanh(x/2) = ln((e^x + 1)/(e^x - 1)), for x >= 0; phi(0) = +inf,
 * phi(+inf) = 0, and phi(phi(x)) = x.  With it the horizontal update (eq.
 * h_update)  2 atanh( prod_k tanh(m_k/2) )  equals
 *     (prod_k sgn m_k) * phi( sum_k phi(|m_k|) )
 * exactly; the tanh/atanh product saturates to atanh(1) in FP64 once
 * |m| > ~38 and loses digits well before, this form does not.
 */
static double phi(double x)
{
    return log1p(2.0 / expm1(x));
}

static double clampd(double x, double c)
{
    if (x > c) return c;
    if (x < -c) return -c;
    return x;
}

/* ------------------------------------------------------------------------- */
/* Decoder                                                                    */
/* ------------------------------------------------------------------------- */

enum { OR_BP = 0, OR_MOMENTUM = 1, OR_ADAGRAD = 2, OR_EWAINIT = 3, OR_AEWA = 4 };

typedef struct {
    int32_t variant;            /* OR_BP, OR_MOMENTUM, OR_ADAGRAD, OR_EWAINIT */
    int32_t max_iter;           /* iter_max >= 1 */
    int32_t stop_on_syndrome;   /* 1: halt when <H, E^> = s (Alg. 2); 0: run max_iter */
    int32_t adagrad_g_from_t1;  /* READING switch: accumulate G already at t = 1 */
    double alpha;               /* Momentum / EWAInit step or discount; AdaGrad boost rate */
    double gamma;               /* Momentum decay */
    double eps;                 /* AdaGrad epsilon */
    double clamp;               /* message magnitude bound C (INFINITY: none) */
    const double *alpha_t;      /* per-iteration alpha, alpha_t[t - 1] at iteration t, or NULL for
                                   the constant alpha: the EWAInit discount (entry 0 unused) or the
                                   Momentum step */
    double alpha_last;          /* AEWA: discount of the last attempt */
    int32_t alpha_steps;        /* AEWA: attempts; alpha_k = alpha + (alpha_last - alpha) k / (steps - 1) */
    int32_t serial;             /* 0: flooding schedule (Alg. 2); 1: serial schedule (Alg. 1) */
    const double *gamma_t;      /* Momentum: per-iteration decay, gamma_t[t - 1] at iteration t, or
                                   NULL for the constant gamma */
} or_params;

typedef struct {
    double *q_out;     /* [shots][n][3] final posterior Q, or NULL */
    double *mvc_out;   /* [shots][nnz] final variable-to-check messages, or NULL */
    double *mcv_out;   /* [shots][nnz] final check-to-variable messages, or NULL */
    double *q_trace;   /* [shots][max_iter][n][3] Q^{(t)} for t = 1..max_iter, or NULL */
    double *m_trace;   /* [shots][max_iter][n][3] M^{(t)} (sum of incoming check messages), or NULL */
} or_outputs;

/* Hard decision (section II-B1): I if every LLR is positive, else the Pauli
 * with the smallest LLR; ties resolve to the first of X, Y, Z (READING).
 * Returns -1 if an LLR is NaN. */
static int hard_decision(const double q[3])
{
    if (isnan(q[0]) || isnan(q[1]) || isnan(q[2])) return -1;
    if (q[0] > 0.0 && q[1] > 0.0 && q[2] > 0.0) return 0;
    int best = 0;
    for (int w = 1; w < 3; ++w)
        if (q[w] < q[best]) best = w;
    return PAULI_OF_INDEX[best];
}

/* Horizontal update (eq. h_update) of edge e = (c, v): combine the current
 * messages m_{v'->c} of the other neighbours v' of c. */
static double check_to_qubit(const or_graph *g, const uint8_t *s, const double *mvc, int e, double C)
{
    const int c = g->echk[e];
    const int e0 = g->cptr[c], e1 = g->cptr[c + 1];
    double ssum = 0.0;
    int neg = s[c] ? 1 : 0;
    for (int f = e0; f < e1; ++f) {
        if (f == e) continue;
        ssum += phi(fabs(mvc[f]));
        if (mvc[f] < 0.0) neg ^= 1;
    }
    double w = phi(ssum);
    return clampd(neg ? -w : w, C);
}

/* Sum of incoming check messages per Pauli: M_{v,W} = sum over c in M(v) with
 * <W, H_cv> = 1 of m_{c->v} (the sum in eqs. p_update / mombp3). */
static void qubit_sums(const or_graph *g, int v, const double *mcv, double *msum)
{
    for (int w = 0; w < 3; ++w) {
        double sum = 0.0;
        for (int k = g->vptr[v]; k < g->vptr[v + 1]; ++k) {
            int e = g->vedge[k];
            if (anticommute(PAULI_OF_INDEX[w], g->elab[e])) sum += mcv[e];
        }
        msum[3 * v + w] = sum;
    }
}

/* Posterior update of entry i = 3v + w, per variant. */
static void posterior(const or_params *p, int t, int i, const double *pi0, const double *pit,
                      const double *qprev, const double *msum, double *q,
                      double *acc, double *dev)
{
    switch (p->variant) {
    case OR_BP:        /* eq. p_update */
        q[i] = pi0[i] + msum[i];
        break;
    case OR_EWAINIT:   /* eq. p_update with Pi^{(t)} (Alg. 2) */
        q[i] = pit[i] + msum[i];
        break;
    case OR_MOMENTUM: { /* eqs. mombp1, mombp2, with the gradient of eq. mombp3 */
        const double a = p->alpha_t ? p->alpha_t[t - 1] : p->alpha;
        const double gm = p->gamma_t ? p->gamma_t[t - 1] : p->gamma;
        double grad = qprev[i] - pi0[i] - msum[i];
        acc[i] = gm * acc[i] + (1.0 - gm) * grad;
        q[i] = qprev[i] - a * acc[i];
        break;
    }
    case OR_ADAGRAD: { /* eq. boost; active from the second iteration (READING) */
        /* Carried as the deviation D = Q - Pi^{(0)} (READING: the gradient
         * g' = Q^{(t-1)} - Pi - sum m of eq. boost is then D^{(t-1)} - sum m,
         * which is exactly 0 when the incoming sums repeat). */
        double grad = dev[i] - msum[i];
        if (t == 1) {
            if (p->adagrad_g_from_t1) acc[i] += grad * grad;
            dev[i] = msum[i];
        } else {
            acc[i] += grad * grad;
            dev[i] = dev[i] - p->alpha * grad / (sqrt(acc[i]) + p->eps);
        }
        q[i] = pi0[i] + dev[i];
        break;
    }
    }
}

/* Vertical update of qubit v.  BP / EWAInit (eq. v_update): lambda over the
 * prior (Pi^{(t)} for EWAInit) plus the messages of every other check c' of v.
 * Momentum / AdaGrad (eq. mombp5, with lambda applied as in v_update,
 * READING): lambda over Q^{(t)} minus the original message of c. */
static void qubit_messages(const or_graph *g, const or_params *p, int v, const double *pi0, const double *pit,
                           const double *q, const double *mcv, double *mvc, double C)
{
    for (int k = g->vptr[v]; k < g->vptr[v + 1]; ++k) {
        int e = g->vedge[k];
        int H = g->elab[e];
        double L[3];
        for (int w = 0; w < 3; ++w) {
            int W = PAULI_OF_INDEX[w];
            if (p->variant == OR_BP || p->variant == OR_EWAINIT) {
                double base = (p->variant == OR_BP) ? pi0[3 * v + w] : pit[3 * v + w];
                double sum = 0.0;
                for (int k2 = g->vptr[v]; k2 < g->vptr[v + 1]; ++k2) {
                    int f = g->vedge[k2];
                    if (f == e) continue;
                    if (anticommute(W, g->elab[f])) sum += mcv[f];
                }
                L[w] = base + sum;
            } else {
                L[w] = q[3 * v + w] - (anticommute(W, H) ? mcv[e] : 0.0);
            }
        }
        mvc[e] = clampd(lambda_h(H, L), C);
    }
}

/* Decode one shot.  Work arrays are caller-provided (per thread). */
static void decode_one(const or_graph *g, const or_params *p, const double *pi0,
                       const uint8_t *s, uint8_t *est, uint8_t *conv_out, int32_t *iters_out,
                       double *mvc, double *mcv, double *q, double *qprev, double *pit,
                       double *acc, double *dev, double *msum, int *ehat,
                       double *q_trace, double *m_trace)
{
    const int n = g->n, m = g->m, nnz = g->nnz;
    const double C = p->clamp;
    int nan_seen = 0;

    /* Initialisation (eq. init; Alg. 1 and 2): m^{(0)}_{v->c} = lambda_{H_cv}(Pi^{(0)}_v),
     * Q^{(0)} = Pi^{(0)}, momentum / gradient accumulators g^{(0)} = G^{(0)} = 0. */
    for (int e = 0; e < nnz; ++e)
        mvc[e] = clampd(lambda_h(g->elab[e], &pi0[3 * g->evar[e]]), C);
    for (int i = 0; i < 3 * n; ++i) { q[i] = pi0[i]; pit[i] = pi0[i]; acc[i] = 0.0; dev[i] = 0.0; }

    int t_done = p->max_iter, converged = 0;
    for (int t = 1; t <= p->max_iter; ++t) {
        for (int i = 0; i < 3 * n; ++i) qprev[i] = q[i];

        /* EWA initialisation (eq. EWAInit, Alg. 2): Pi^{(1)} = Pi^{(0)};
         * Pi^{(t)} = alpha Pi^{(0)} + (1 - alpha) Q^{(t-1)} for t > 1. */
        if (p->variant == OR_EWAINIT && t > 1) {
            const double a = p->alpha_t ? p->alpha_t[t - 1] : p->alpha;
            for (int i = 0; i < 3 * n; ++i)
                pit[i] = a * pi0[i] + (1.0 - a) * qprev[i];
        }

        if (!p->serial) {
            /* Flooding ("parallel") schedule, Alg. 2: every check, then every qubit. */
            for (int e = 0; e < nnz; ++e) mcv[e] = check_to_qubit(g, s, mvc, e, C);
            for (int v = 0; v < n; ++v) qubit_sums(g, v, mcv, msum);
            for (int i = 0; i < 3 * n; ++i) posterior(p, t, i, pi0, pit, qprev, msum, q, acc, dev);
            for (int v = 0; v < n; ++v) qubit_messages(g, p, v, pi0, pit, q, mcv, mvc, C);
        } else {
            /* Serial schedule, Alg. 1: qubit by qubit in index order, each qubit's
             * incoming check messages from the current messages of the check's other
             * qubits (those earlier in the sweep already updated), then its posterior
             * and its outgoing messages. */
            for (int v = 0; v < n; ++v) {
                for (int k = g->vptr[v]; k < g->vptr[v + 1]; ++k) {
                    const int e = g->vedge[k];
                    mcv[e] = check_to_qubit(g, s, mvc, e, C);
                }
                qubit_sums(g, v, mcv, msum);
                for (int i = 3 * v; i < 3 * v + 3; ++i) posterior(p, t, i, pi0, pit, qprev, msum, q, acc, dev);
                qubit_messages(g, p, v, pi0, pit, q, mcv, mvc, C);
            }
        }

        if (q_trace) memcpy(&q_trace[(size_t)(t - 1) * 3 * n], q, sizeof(double) * 3 * n);
        if (m_trace) memcpy(&m_trace[(size_t)(t - 1) * 3 * n], msum, sizeof(double) * 3 * n);

        /* Hard decision and syndrome test (section II-B1, Alg. 2). */
        nan_seen = 0;
        for (int v = 0; v < n; ++v) {
            int hd = hard_decision(&q[3 * v]);
            if (hd < 0) { nan_seen = 1; hd = 0; }
            ehat[v] = hd;
        }
        int ok = !nan_seen;
        for (int c = 0; c < m && ok; ++c) {
            int par = 0;
            for (int e = g->cptr[c]; e < g->cptr[c + 1]; ++e)
                par ^= anticommute(g->elab[e], ehat[g->evar[e]]);
            if (par != (s[c] & 1)) ok = 0;
        }
        if (p->stop_on_syndrome && ok) {
            t_done = t;
            converged = 1;
            break;
        }
        if (t == p->max_iter) converged = ok;
    }
    for (int v = 0; v < n; ++v) est[v] = (uint8_t)ehat[v];
    *conv_out = (uint8_t)converged;
    *iters_out = t_done;
}

/*
 * Decode `shots` syndromes (s: [shots][m]) with prior LLRs pi0 ([n][3]).
 * Writes est [shots][n], conv [shots], iters [shots]; optional outputs in `o`.
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad arguments.
 */
int or_decode(int m, int n, const uint8_t *hx, const uint8_t *hz, const or_params *p,
              int64_t shots, const double *pi0, const uint8_t *synd,
              uint8_t *est, uint8_t *conv, int32_t *iters, const or_outputs *o, int nthreads)
{
    if (m <= 0 || n <= 0 || !hx || !hz || !p || !pi0 || !synd || !est || !conv || !iters)
        return -1;
    if (p->max_iter < 1 || shots < 0) return -1;
    if (p->variant == OR_AEWA && (p->alpha_steps < 1 || !p->stop_on_syndrome)) return -1;
    or_graph g;
    if (graph_build(m, n, hx, hz, &g)) return -1;
    or_outputs none = {0};
    if (!o) o = &none;
    int rc = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        const int nnz = g.nnz;
        double *mvc = malloc(sizeof(double) * (nnz + 1));
        double *mcv = malloc(sizeof(double) * (nnz + 1));
        double *q = malloc(sizeof(double) * 3 * n);
        double *qprev = malloc(sizeof(double) * 3 * n);
        double *pit = malloc(sizeof(double) * 3 * n);
        double *acc = malloc(sizeof(double) * 3 * n);
        double *dev = malloc(sizeof(double) * 3 * n);
        double *msum = malloc(sizeof(double) * 3 * n);
        int *ehat = malloc(sizeof(int) * n);
        if (!mvc || !mcv || !q || !qprev || !pit || !acc || !dev || !msum || !ehat) {
#pragma omp atomic write
            rc = -1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t i = 0; i < shots; ++i) {
                double *qt = o->q_trace ? o->q_trace + (size_t)i * p->max_iter * 3 * n : NULL;
                double *mt = o->m_trace ? o->m_trace + (size_t)i * p->max_iter * 3 * n : NULL;
                if (p->variant != OR_AEWA) {
                    decode_one(&g, p, pi0, synd + (size_t)i * m, est + (size_t)i * n, conv + i,
                               iters + i, mvc, mcv, q, qprev, pit, acc, dev, msum, ehat, qt, mt);
                } else {
                    /* AEWA-BP (appendix on adaptive MBP): EWAInit-BP with the discounts
                     * alpha_0 .. alpha_{K-1}, each attempt a fresh decode, until one
                     * satisfies the syndrome; the outputs are those of the last attempt
                     * run and the iteration count is the total over the attempts. */
                    or_params pk = *p;
                    pk.variant = OR_EWAINIT;
                    pk.alpha_t = NULL;
                    int32_t total = 0;
                    for (int k = 0; k < p->alpha_steps; ++k) {
                        pk.alpha = p->alpha_steps > 1
                                       ? p->alpha + (p->alpha_last - p->alpha) * (double)k / (double)(p->alpha_steps - 1)
                                       : p->alpha;
                        decode_one(&g, &pk, pi0, synd + (size_t)i * m, est + (size_t)i * n, conv + i,
                                   iters + i, mvc, mcv, q, qprev, pit, acc, dev, msum, ehat, qt, mt);
                        total += iters[i];
                        if (conv[i]) break;
                    }
                    iters[i] = total;
                }
                if (o->q_out) memcpy(o->q_out + (size_t)i * 3 * n, q, sizeof(double) * 3 * n);
                if (o->mvc_out) memcpy(o->mvc_out + (size_t)i * nnz, mvc, sizeof(double) * nnz);
                if (o->mcv_out) memcpy(o->mcv_out + (size_t)i * nnz, mcv, sizeof(double) * nnz);
            }
        }
        free(mvc); free(mcv); free(q); free(qprev); free(pit); free(acc); free(dev); free(msum); free(ehat);
    }
    graph_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Noise sampling and syndromes (section IV: i.i.d. Pauli channel per qubit)  */
/* ------------------------------------------------------------------------- */

/*
 * Error of qubit q in shot `gshot` (global index): Philox4x64-10 with key
 * (seed, stream) and counter (gshot, q / 8, 0, 0) gives four 64-bit words;
 * qubit q takes 32-bit half (q % 2) (0 = low) of word (q % 8) / 2.  With
 * integer thresholds t = (tX, tY, tZ): u < tX -> X, u < tX+tY -> Y,
 * u < tX+tY+tZ -> Z, else I.
 */
int or_sample(int m, int n, const uint8_t *hx, const uint8_t *hz, int64_t shots, int64_t shot0,
              const uint32_t thr[3], uint64_t seed, uint64_t stream,
              uint8_t *err, uint8_t *synd, int nthreads)
{
    if (m < 0 || n <= 0 || !hx || !hz || !thr || !err || !synd || shots < 0) return -1;
    if ((uint64_t)thr[0] + thr[1] + thr[2] > 0xFFFFFFFFULL) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const uint64_t t0 = thr[0], t1 = t0 + thr[1], t2 = t1 + thr[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < shots; ++i) {
        uint8_t *e = err + (size_t)i * n;
        uint64_t key[2] = {seed, stream};
        for (int blk = 0; blk * 8 < n; ++blk) {
            uint64_t ctr[4] = {(uint64_t)(shot0 + i), (uint64_t)blk, 0, 0}, out[4];
            or_philox4x64_10(ctr, key, out);
            for (int j = 0; j < 8 && blk * 8 + j < n; ++j) {
                uint64_t u = (j & 1) ? (out[j >> 1] >> 32) : (out[j >> 1] & 0xFFFFFFFFULL);
                uint8_t pauli = u < t0 ? 1 : (u < t1 ? 3 : (u < t2 ? 2 : 0));
                e[blk * 8 + j] = pauli;
            }
        }
        /* Syndrome: s_c = sum over qubits of <H_cv, E_v> mod 2. */
        for (int c = 0; c < m; ++c) {
            int par = 0;
            for (int v = 0; v < n; ++v) {
                int lab = (hx[(size_t)c * n + v] & 1) | ((hz[(size_t)c * n + v] & 1) << 1);
                if (lab) par ^= anticommute(lab, e[v]);
            }
            synd[(size_t)i * m + c] = (uint8_t)par;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Bookkeeping (section IV): success iff E^ E is in the stabilizer group.     */
/* ------------------------------------------------------------------------- */

/*
 * For each shot, R = E^ E (x and z bits XOR).  fail[i] = 1 ("detected") if R
 * anticommutes with some stabilizer row, 2 ("undetected", a logical error)
 * if it commutes with every row but anticommutes with one of the nlog logical
 * operators (lx, lz: [nlog][n]), else 0.  counts[k] += number of shots with
 * fail == k.
 */
int or_bookkeep(int m, int n, const uint8_t *hx, const uint8_t *hz, int nlog,
                const uint8_t *lx, const uint8_t *lz, int64_t shots,
                const uint8_t *err, const uint8_t *est, uint8_t *fail, int64_t counts[3])
{
    if (m < 0 || n <= 0 || nlog < 0 || !hx || !hz || !err || !est || !fail || !counts) return -1;
    if (nlog > 0 && (!lx || !lz)) return -1;
    int64_t c0 = 0, c1 = 0, c2 = 0;
#pragma omp parallel for schedule(static) reduction(+ : c0, c1, c2)
    for (int64_t i = 0; i < shots; ++i) {
        const uint8_t *e = err + (size_t)i * n, *h = est + (size_t)i * n;
        int kind = 0;
        for (int c = 0; c < m && !kind; ++c) {
            int par = 0;
            for (int v = 0; v < n; ++v) {
                int lab = (hx[(size_t)c * n + v] & 1) | ((hz[(size_t)c * n + v] & 1) << 1);
                if (lab) par ^= anticommute(lab, (e[v] ^ h[v]) & 3);
            }
            if (par) kind = 1;
        }
        for (int k = 0; k < nlog && !kind; ++k) {
            int par = 0;
            for (int v = 0; v < n; ++v) {
                int lab = (lx[(size_t)k * n + v] & 1) | ((lz[(size_t)k * n + v] & 1) << 1);
                if (lab) par ^= anticommute(lab, (e[v] ^ h[v]) & 3);
            }
            if (par) kind = 2;
        }
        fail[i] = (uint8_t)kind;
        if (kind == 0) ++c0; else if (kind == 1) ++c1; else ++c2;
    }
    counts[0] += c0; counts[1] += c1; counts[2] += c2;
    return 0;
}

/* Elementary functions exported for the tests that pin them. */
double or_lambda(int pauli, double lx, double ly, double lz)
{
    double L[3] = {lx, ly, lz};
    return lambda_h(pauli, L);
}

double or_phi(double x) { return phi(x); }
