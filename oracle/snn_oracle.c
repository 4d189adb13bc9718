/*
 * FP64 reference simulator of the spiking-network timestep (the oracle).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the test suite, the smoke check and the CPU
 * baseline of the benchmark use it.  It shares no code, header or table with
 * the HIP path.  Plain loops, double precision throughout, in the order in
 * which the method states its steps, so that a reader can check it by eye.
 *
 * What is simulated (Balaji, Yavuz, Nowotny, "Scalability and Optimization
 * Strategies for GPU Enhanced Neural Networks"):
 *  - Hodgkin-Huxley neurons integrated at discrete time steps (Section 2).
 *    The paper names no equations; the Traub-Miles (1991) kinetics of the
 *    insect-olfaction model it uses (Section 5.1) are taken, integrated with
 *    forward-Euler substeps whose right-hand sides all come from the
 *    substep-start state.
 *  - Synapses stored in Compressed Row Storage (Section 3): per projection a
 *    weight array and a post-index array ordered by pre-synaptic neuron, and
 *    a row-start array.  A spike of pre-synaptic neuron i adds g_scale * g of
 *    every entry of row i to the conductance of that entry's post neuron.
 *  - Poisson input sources (the non-deterministic inputs of the olfaction
 *    model, Section 4 "Discussion"), drawn from Philox-4x32-10 (Salmon et al.,
 *    SC'11) so that the draws are reproducible by a separate implementation.
 *  - Per-run spike counts and a count of neurons whose voltage became NaN or
 *    infinite, the two quantities the calibration of Fig. 1 reads
 *    (avgSpike, sumNANs).
 *  - Optional pair-based STDP with all-to-all traces on chosen projections.
 *  - Izhikevich neurons (Section 5.1's first network cites the model,
 *    reference [9], without its equations; they are taken from Izhikevich,
 *    "Simple model of spiking neurons", IEEE TNN 14, 2003): v' = 0.04 v^2 +
 *    5 v + 140 - u + I, u' = a (b v - u), and at v >= 30 mV the reset
 *    v <- c, u <- u + d, with a, b, c, d per neuron.
 *
 * Parity pins (tests that tie this code to mathematics rather than to
 * itself) live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "snn_oracle.h"


/* ------------------------------------------------------------------ */
/* Traub-Miles kinetics.  V in mV, rates in 1/ms.                      */
/* ------------------------------------------------------------------ */

/* x / (e^x - 1), whose limit at x = 0 is 1.  expm1 avoids cancellation. */
double orc_phi(double x)
{
    if (x == 0.0) return 1.0;
    return x / expm1(x);
}

double orc_alpha_m(double V) { return 1.28 * orc_phi((-52.0 - V) / 4.0); }
double orc_beta_m(double V)  { return 1.4 * orc_phi((V + 25.0) / 5.0); }
double orc_alpha_h(double V) { return 0.128 * exp((-48.0 - V) / 18.0); }
double orc_beta_h(double V)  { return 4.0 / (exp((-25.0 - V) / 5.0) + 1.0); }
double orc_alpha_n(double V) { return 0.16 * orc_phi((-50.0 - V) / 5.0); }
double orc_beta_n(double V)  { return 0.5 * exp((-55.0 - V) / 40.0); }

void orc_default_hh(double *p)
{
    p[HH_GNA] = 7.15;     /* uS */
    p[HH_ENA] = 50.0;     /* mV */
    p[HH_GK] = 1.43;      /* uS */
    p[HH_EK] = -95.0;     /* mV */
    p[HH_GL] = 0.02672;   /* uS */
    p[HH_EL] = -63.563;   /* mV */
    p[HH_CM] = 0.143;     /* nF */
}

/* Ionic current (nA) flowing out of the cell. */
double orc_i_ion(const double *p, double V, double m, double h, double n)
{
    return p[HH_GNA] * m * m * m * h * (V - p[HH_ENA])
         + p[HH_GK] * n * n * n * n * (V - p[HH_EK])
         + p[HH_GL] * (V - p[HH_EL]);
}

/* One forward-Euler substep of length hs on (V, m, h, n); i_in is the
 * injected current (synaptic + external, nA), held fixed. */
void orc_substep(const double *p, double hs, double i_in, double *V, double *m, double *h, double *n)
{
    double v = *V, mm = *m, hh = *h, nn = *n;
    double dv = (-orc_i_ion(p, v, mm, hh, nn) + i_in) / p[HH_CM];
    double dm = orc_alpha_m(v) * (1.0 - mm) - orc_beta_m(v) * mm;
    double dh = orc_alpha_h(v) * (1.0 - hh) - orc_beta_h(v) * hh;
    double dn = orc_alpha_n(v) * (1.0 - nn) - orc_beta_n(v) * nn;
    *V = v + hs * dv;
    *m = mm + hs * dm;
    *h = hh + hs * dh;
    *n = nn + hs * dn;
}

/* Whether x stays finite when held in single precision, the precision of
 * the workloads' neuron state: |x| below FLT_MAX plus half its ulp, the
 * values that round to a finite float (NaN does not). */
static int fits_fp32(double x)
{
    return fabs(x) < 0x1.ffffffp127;
}

/* One forward-Euler substep of the Izhikevich model (v in mV, u in the
 * same units, t in ms); both right-hand sides from the substep-start state,
 * i_in the injected current (synaptic + external), held fixed. */
void orc_izh_substep(double a, double b, double hs, double i_in, double *v, double *u)
{
    double vv = *v, uu = *u;
    double dv = 0.04 * vv * vv + 5.0 * vv + 140.0 - uu + i_in;
    double du = a * (b * vv - uu);
    *v = vv + hs * dv;
    *u = uu + hs * du;
}

/* Net membrane current with every gate at its steady state a/(a+b). */
double orc_i_ss(const double *p, double V)
{
    double am = orc_alpha_m(V), bm = orc_beta_m(V);
    double ah = orc_alpha_h(V), bh = orc_beta_h(V);
    double an = orc_alpha_n(V), bn = orc_beta_n(V);
    return orc_i_ion(p, V, am / (am + bm), ah / (ah + bh), an / (an + bn));
}

/* Resting potential: the root of orc_i_ss in [-80, -60] mV by bisection.
 * Returns 0 on success, -1 if the bracket holds no sign change. */
int orc_rest(const double *p, double *V, double *m, double *h, double *n)
{
    double lo = -80.0, hi = -60.0;
    double flo = orc_i_ss(p, lo), fhi = orc_i_ss(p, hi);
    if (!(flo < 0.0 && fhi > 0.0)) return -1;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        double fm = orc_i_ss(p, mid);
        if (fm < 0.0) lo = mid; else hi = mid;
    }
    double v = 0.5 * (lo + hi);
    double am = orc_alpha_m(v), bm = orc_beta_m(v);
    double ah = orc_alpha_h(v), bh = orc_beta_h(v);
    double an = orc_alpha_n(v), bn = orc_beta_n(v);
    *V = v;
    *m = am / (am + bm);
    *h = ah / (ah + bh);
    *n = an / (an + bn);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Philox-4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).              */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out)
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Source i of Poisson population pop fires at step t iff the first Philox
 * word of counter (i, t_lo, t_hi, pop) under key (seed_lo, seed_hi) is below
 * floor(p * 2^32), p = rate_hz * dt_ms * 1e-3 (a Bernoulli draw per step).
 * The population index keeps two populations of one instance independent. */
uint64_t orc_poisson_threshold(double rate_hz, double dt_ms)
{
    double p = rate_hz * dt_ms * 1e-3;
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return (uint64_t)1 << 32;
    return (uint64_t)floor(p * 4294967296.0);
}

int orc_poisson_fires(uint64_t seed, int64_t t, int32_t i, int32_t pop, uint64_t thresh)
{
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)t & 0xffffffffu), (uint32_t)((uint64_t)t >> 32),
                       (uint32_t)pop};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return (uint64_t)out[0] < thresh;
}

orc_net *orc_create(double dt, int substeps, double g_scale, uint64_t seed)
{
    if (!(dt > 0.0) || substeps < 1) return NULL;
    orc_net *net = (orc_net *)calloc(1, sizeof(orc_net));
    net->dt = dt;
    net->substeps = substeps;
    net->g_scale = g_scale;
    net->seed = seed;
    return net;
}

int orc_add_pop(orc_net *net, int kind, int n, double rate_hz, double i_ext, const double *hh)
{
    if (net->ready || net->n_pops >= ORC_MAX_POPS || n < 0) return -1;
    if (kind != ORC_POISSON && kind != ORC_HH && kind != ORC_IZH) return -1;
    opop *P = &net->pops[net->n_pops];
    memset(P, 0, sizeof(*P));
    P->kind = kind;
    P->n = n;
    P->rate_hz = rate_hz;
    P->i_ext = i_ext;
    if (hh) memcpy(P->hh, hh, sizeof(P->hh)); else orc_default_hh(P->hh);
    P->thresh = orc_poisson_threshold(rate_hz, net->dt);
    return net->n_pops++;
}

int orc_add_proj(orc_net *net, int pre, int post, int64_t nnz, const int32_t *row_ptr,
                 const int32_t *col_idx, const float *g, double e_rev, double tau,
                 int stdp, double a_plus, double a_minus, double tau_stdp, double g_max)
{
    if (net->ready || net->n_projs >= ORC_MAX_PROJS || nnz < 0 || nnz >= ((int64_t)1 << 31)) return -1;
    if (pre < 0 || pre >= net->n_pops || post < 0 || post >= net->n_pops) return -1;
    if (net->pops[post].kind == ORC_POISSON || !(tau > 0.0)) return -1;
    int npre = net->pops[pre].n, npost = net->pops[post].n;
    if (row_ptr[0] != 0 || row_ptr[npre] != nnz) return -1;
    for (int i = 0; i < npre; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return -1;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col_idx[k] < 0 || col_idx[k] >= npost) return -1;
    }
    oproj *Q = &net->projs[net->n_projs];
    memset(Q, 0, sizeof(*Q));
    Q->pre = pre;
    Q->post = post;
    Q->nnz = nnz;
    Q->row_ptr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(npre + 1));
    Q->col_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    Q->g = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    memcpy(Q->row_ptr, row_ptr, sizeof(int32_t) * (size_t)(npre + 1));
    if (nnz) memcpy(Q->col_idx, col_idx, sizeof(int32_t) * (size_t)nnz);
    for (int64_t k = 0; k < nnz; ++k) Q->g[k] = (double)g[k];
    Q->e_rev = e_rev;
    Q->tau = tau;
    Q->stdp = stdp;
    Q->a_plus = a_plus;
    Q->a_minus = a_minus;
    Q->tau_stdp = tau_stdp;
    Q->g_max = g_max;
    return net->n_projs++;
}

/* Izhikevich parameters of population pop: abcd holds a[n], b[n], c[n],
 * d[n] (parameter-major, fp32, widened exactly).  Before orc_init. */
int orc_set_izh_params(orc_net *net, int pop, const float *abcd)
{
    if (net->ready || pop < 0 || pop >= net->n_pops || net->pops[pop].kind != ORC_IZH) return -1;
    opop *P = &net->pops[pop];
    size_t n = (size_t)(P->n > 0 ? P->n : 1);
    double **dst[4] = {&P->iza, &P->izb, &P->izc, &P->izd};
    for (int k = 0; k < 4; ++k) {
        free(*dst[k]);
        *dst[k] = (double *)calloc(n, sizeof(double));
        for (int j = 0; j < P->n; ++j) (*dst[k])[j] = (double)abcd[(size_t)k * (size_t)P->n + (size_t)j];
    }
    return 0;
}

/* Allocate state; every HH neuron starts at its resting point, every
 * Izhikevich neuron at v = -65 mV, u = b v; G = 0, traces = 0, no spikes at
 * step -1. */
int orc_init(orc_net *net)
{
    for (int p = 0; p < net->n_pops; ++p) {
        opop *P = &net->pops[p];
        size_t n = (size_t)(P->n > 0 ? P->n : 1);
        P->spk_prev = (unsigned char *)calloc(n, 1);
        P->spk_now = (unsigned char *)calloc(n, 1);
        P->count = (int32_t *)calloc(n, sizeof(int32_t));
        if (P->kind == ORC_HH) {
            double v, m, h, nn;
            if (orc_rest(P->hh, &v, &m, &h, &nn) != 0) return -1;
            P->V = (double *)malloc(n * sizeof(double));
            P->m = (double *)malloc(n * sizeof(double));
            P->h = (double *)malloc(n * sizeof(double));
            P->nn = (double *)malloc(n * sizeof(double));
            P->vsum = (double *)calloc(n, sizeof(double));
            for (int j = 0; j < P->n; ++j) {
                P->V[j] = v; P->m[j] = m; P->h[j] = h; P->nn[j] = nn;
            }
        }
        if (P->kind == ORC_IZH) {
            if (!P->iza) return -1;
            P->V = (double *)malloc(n * sizeof(double));
            P->m = (double *)malloc(n * sizeof(double));
            P->vsum = (double *)calloc(n, sizeof(double));
            for (int j = 0; j < P->n; ++j) {
                P->V[j] = -65.0;
                P->m[j] = P->izb[j] * -65.0;
            }
        }
    }
    for (int q = 0; q < net->n_projs; ++q) {
        oproj *Q = &net->projs[q];
        int npre = net->pops[Q->pre].n, npost = net->pops[Q->post].n;
        Q->G = (double *)calloc((size_t)(npost > 0 ? npost : 1), sizeof(double));
        if (Q->stdp) {
            Q->x = (double *)calloc((size_t)(npre > 0 ? npre : 1), sizeof(double));
            Q->y = (double *)calloc((size_t)(npost > 0 ? npost : 1), sizeof(double));
            /* column view: for post j, the CSR positions of its synapses */
            Q->col_ptr = (int32_t *)calloc((size_t)npost + 1, sizeof(int32_t));
            Q->row_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(Q->nnz > 0 ? Q->nnz : 1));
            Q->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(Q->nnz > 0 ? Q->nnz : 1));
            for (int64_t k = 0; k < Q->nnz; ++k) Q->col_ptr[Q->col_idx[k] + 1]++;
            for (int j = 0; j < npost; ++j) Q->col_ptr[j + 1] += Q->col_ptr[j];
            int32_t *fill = (int32_t *)calloc((size_t)npost + 1, sizeof(int32_t));
            for (int i = 0; i < npre; ++i)
                for (int32_t k = Q->row_ptr[i]; k < Q->row_ptr[i + 1]; ++k) {
                    int j = Q->col_idx[k];
                    int32_t at = Q->col_ptr[j] + fill[j]++;
                    Q->row_of[at] = i;
                    Q->perm[at] = k;
                }
            free(fill);
        }
    }
    net->t = 0;
    net->nan_count = 0;
    net->ready = 1;
    return 0;
}

static void log_event(orc_net *net, int64_t t, int pop, int id)
{
    if (!net->log_events) return;
    if (net->ev_n == net->ev_cap) {
        int64_t cap = net->ev_cap ? 2 * net->ev_cap : 4096;
        net->ev_t = (int32_t *)realloc(net->ev_t, sizeof(int32_t) * (size_t)cap);
        net->ev_pop = (int32_t *)realloc(net->ev_pop, sizeof(int32_t) * (size_t)cap);
        net->ev_id = (int32_t *)realloc(net->ev_id, sizeof(int32_t) * (size_t)cap);
        net->ev_cap = cap;
    }
    net->ev_t[net->ev_n] = (int32_t)t;
    net->ev_pop[net->ev_n] = pop;
    net->ev_id[net->ev_n] = id;
    net->ev_n++;
}

/* Phase 1 of step t: deliver the spikes of step t-1 through every
 * projection; on a plastic projection, then depress each delivered synapse
 * by the post trace of step t-1 (delivery uses the weight before the
 * update). */
void orc_phase_deliver(orc_net *net)
{
    const double s = net->g_scale;
    for (int q = 0; q < net->n_projs; ++q) {
        oproj *Q = &net->projs[q];
        const opop *pre = &net->pops[Q->pre];
        for (int i = 0; i < pre->n; ++i) {
            if (!pre->spk_prev[i]) continue;
            for (int32_t k = Q->row_ptr[i]; k < Q->row_ptr[i + 1]; ++k)
                Q->G[Q->col_idx[k]] += s * Q->g[k];
            if (Q->stdp)
                for (int32_t k = Q->row_ptr[i]; k < Q->row_ptr[i + 1]; ++k) {
                    double v = Q->g[k] - Q->a_minus * Q->g_max * Q->y[Q->col_idx[k]];
                    Q->g[k] = v < 0.0 ? 0.0 : v;
                }
        }
    }
}

/* Phase 2: potentiation, every synapse onto a post neuron that spiked at
 * t-1 grows by the pre trace of step t-1. */
void orc_phase_potentiate(orc_net *net)
{
    for (int q = 0; q < net->n_projs; ++q) {
        oproj *Q = &net->projs[q];
        if (!Q->stdp) continue;
        const opop *post = &net->pops[Q->post];
        for (int j = 0; j < post->n; ++j) {
            if (!post->spk_prev[j]) continue;
            for (int32_t c = Q->col_ptr[j]; c < Q->col_ptr[j + 1]; ++c) {
                int32_t k = Q->perm[c];
                double v = Q->g[k] + Q->a_plus * Q->g_max * Q->x[Q->row_of[c]];
                Q->g[k] = v > Q->g_max ? Q->g_max : v;
            }
        }
    }
}

/* Phase 3: HH populations (synaptic current from the start-of-step V, Euler
 * substeps, upward crossing of 0 mV), conductance decay, Poisson sources of
 * step t, replayed populations. */
void orc_phase_neurons(orc_net *net)
{
    const int64_t t = net->t;
    const double hs = net->dt / net->substeps;
    for (int p = 0; p < net->n_pops; ++p) {
        opop *P = &net->pops[p];
        if (P->kind != ORC_HH) continue;
        /* Neurons are independent within a step, so the loop may run on
         * several threads; each neuron's arithmetic is the same either way. */
        int64_t nan_new = 0;
        #pragma omp parallel for schedule(static) reduction(+ : nan_new) num_threads(net->threads > 1 ? net->threads : 1) if (net->threads > 1)
        for (int j = 0; j < P->n; ++j) {
            double v0 = P->V[j];
            double isyn = 0.0;
            for (int q = 0; q < net->n_projs; ++q)
                if (net->projs[q].post == p)
                    isyn += net->projs[q].G[j] * (net->projs[q].e_rev - v0);
            double v = v0, m = P->m[j], h = P->h[j], n = P->nn[j];
            for (int k = 0; k < net->substeps; ++k)
                orc_substep(P->hh, hs, isyn + P->i_ext, &v, &m, &h, &n);
            P->V[j] = v; P->m[j] = m; P->h[j] = h; P->nn[j] = n;
            P->spk_now[j] = (v0 < 0.0 && v >= 0.0) ? 1 : 0;
            /* Fig. 1's NaN count covers overflow: a neuron counts once, at
             * the step its V leaves the range of the single-precision state */
            if (fits_fp32(v0) && !fits_fp32(v)) nan_new++;
            P->vsum[j] += v;
        }
        net->nan_count += nan_new;
    }
    /* Izhikevich populations: synaptic current from the start-of-step v,
     * Euler substeps on (v, u), then the threshold test on the step's end
     * value: v >= 30 mV is a spike, and the neuron resets. */
    for (int p = 0; p < net->n_pops; ++p) {
        opop *P = &net->pops[p];
        if (P->kind != ORC_IZH) continue;
        for (int j = 0; j < P->n; ++j) {
            double v0 = P->V[j];
            double isyn = 0.0;
            for (int q = 0; q < net->n_projs; ++q)
                if (net->projs[q].post == p)
                    isyn += net->projs[q].G[j] * (net->projs[q].e_rev - v0);
            double v = v0, u = P->m[j];
            for (int k = 0; k < net->substeps; ++k)
                orc_izh_substep(P->iza[j], P->izb[j], hs, isyn + P->i_ext, &v, &u);
            int fired = v >= 30.0;
            if (fits_fp32(v0) && !fits_fp32(v)) net->nan_count++;
            if (fired) {
                v = P->izc[j];
                u = u + P->izd[j];
            }
            P->V[j] = v;
            P->m[j] = u;
            P->spk_now[j] = (unsigned char)fired;
            P->vsum[j] += v;
        }
    }
    for (int q = 0; q < net->n_projs; ++q) {
        oproj *Q = &net->projs[q];
        double d = exp(-net->dt / Q->tau);
        for (int j = 0; j < net->pops[Q->post].n; ++j) Q->G[j] *= d;
    }
    for (int p = 0; p < net->n_pops; ++p) {
        opop *P = &net->pops[p];
        if (P->kind != ORC_POISSON) continue;
        for (int i = 0; i < P->n; ++i)
            P->spk_now[i] = (unsigned char)orc_poisson_fires(net->seed, t, i, p, P->thresh);
    }
    if (net->rp_off) {
        for (int p = 0; p < net->n_pops; ++p) {
            opop *P = &net->pops[p];
            if (!P->replay) continue;
            memset(P->spk_now, 0, (size_t)P->n);
            if (t < net->rp_T) {
                int64_t a = net->rp_off[t * net->n_pops + p], b = net->rp_off[t * net->n_pops + p + 1];
                for (int64_t e = a; e < b; ++e) P->spk_now[net->rp_ids[e]] = 1;
            }
        }
    }
}

/* Phase 4: counts, event log, STDP traces; S(t) becomes S(t-1). */
void orc_phase_finish(orc_net *net)
{
    const int64_t t = net->t;
    for (int p = 0; p < net->n_pops; ++p) {
        opop *P = &net->pops[p];
        for (int i = 0; i < P->n; ++i)
            if (P->spk_now[i]) {
                P->count[i]++;
                log_event(net, t, p, i);
            }
    }
    for (int q = 0; q < net->n_projs; ++q) {
        oproj *Q = &net->projs[q];
        if (!Q->stdp) continue;
        double d = exp(-net->dt / Q->tau_stdp);
        const opop *pre = &net->pops[Q->pre], *post = &net->pops[Q->post];
        for (int i = 0; i < pre->n; ++i) Q->x[i] = Q->x[i] * d + (pre->spk_now[i] ? 1.0 : 0.0);
        for (int j = 0; j < post->n; ++j) Q->y[j] = Q->y[j] * d + (post->spk_now[j] ? 1.0 : 0.0);
    }
    for (int p = 0; p < net->n_pops; ++p) {
        opop *P = &net->pops[p];
        unsigned char *tmp = P->spk_prev;
        P->spk_prev = P->spk_now;
        P->spk_now = tmp;
    }
    net->t = t + 1;
}

/* One timestep t = net->t: the four phases in order. */
static void orc_step1(orc_net *net)
{
    orc_phase_deliver(net);
    orc_phase_potentiate(net);
    orc_phase_neurons(net);
    orc_phase_finish(net);
}

int orc_step(orc_net *net, int64_t n_steps)
{
    if (!net->ready) return -1;
    for (int64_t k = 0; k < n_steps; ++k) orc_step1(net);
    return 0;
}

/* Run n steps, copying every HH neuron's post-step V of population pop into
 * out[k * n_pop + j] (a voltage trace for parity checks). */
int orc_step_trace(orc_net *net, int64_t n_steps, int pop, double *out)
{
    if (!net->ready || pop < 0 || pop >= net->n_pops || net->pops[pop].kind == ORC_POISSON) return -1;
    int n = net->pops[pop].n;
    for (int64_t k = 0; k < n_steps; ++k) {
        orc_step1(net);
        memcpy(out + k * n, net->pops[pop].V, sizeof(double) * (size_t)n);
    }
    return 0;
}

/* ----------------------------- accessors ------------------------------ */
enum { ORC_V = 0, ORC_M, ORC_H, ORC_N };

static double *var_ptr(orc_net *net, int pop, int var)
{
    if (pop < 0 || pop >= net->n_pops || net->pops[pop].kind == ORC_POISSON) return NULL;
    opop *P = &net->pops[pop];
    if (P->kind == ORC_IZH && var != ORC_V && var != ORC_M) return NULL;
    switch (var) {
    case ORC_V: return P->V;
    case ORC_M: return P->m;
    case ORC_H: return P->h;
    case ORC_N: return P->nn;
    default: return NULL;
    }
}

int orc_get_var(orc_net *net, int pop, int var, double *out)
{
    double *p = var_ptr(net, pop, var);
    if (!p) return -1;
    memcpy(out, p, sizeof(double) * (size_t)net->pops[pop].n);
    return 0;
}

int orc_set_var(orc_net *net, int pop, int var, const double *in)
{
    double *p = var_ptr(net, pop, var);
    if (!p) return -1;
    memcpy(p, in, sizeof(double) * (size_t)net->pops[pop].n);
    return 0;
}

int orc_get_G(orc_net *net, int proj, double *out)
{
    if (proj < 0 || proj >= net->n_projs) return -1;
    memcpy(out, net->projs[proj].G, sizeof(double) * (size_t)net->pops[net->projs[proj].post].n);
    return 0;
}

int orc_set_G(orc_net *net, int proj, const double *in)
{
    if (proj < 0 || proj >= net->n_projs) return -1;
    memcpy(net->projs[proj].G, in, sizeof(double) * (size_t)net->pops[net->projs[proj].post].n);
    return 0;
}

int orc_get_weights(orc_net *net, int proj, double *out)
{
    if (proj < 0 || proj >= net->n_projs) return -1;
    memcpy(out, net->projs[proj].g, sizeof(double) * (size_t)net->projs[proj].nnz);
    return 0;
}

int orc_get_traces(orc_net *net, int proj, double *x, double *y)
{
    if (proj < 0 || proj >= net->n_projs || !net->projs[proj].stdp) return -1;
    oproj *Q = &net->projs[proj];
    memcpy(x, Q->x, sizeof(double) * (size_t)net->pops[Q->pre].n);
    memcpy(y, Q->y, sizeof(double) * (size_t)net->pops[Q->post].n);
    return 0;
}

int orc_get_counts(orc_net *net, int pop, int32_t *out)
{
    if (pop < 0 || pop >= net->n_pops) return -1;
    memcpy(out, net->pops[pop].count, sizeof(int32_t) * (size_t)net->pops[pop].n);
    return 0;
}

int orc_get_vsum(orc_net *net, int pop, double *out)
{
    if (pop < 0 || pop >= net->n_pops || net->pops[pop].kind == ORC_POISSON) return -1;
    memcpy(out, net->pops[pop].vsum, sizeof(double) * (size_t)net->pops[pop].n);
    return 0;
}

/* Spikes of the last completed step (S(t-1)) as 0/1 bytes. */
int orc_get_last_spikes(orc_net *net, int pop, unsigned char *out)
{
    if (pop < 0 || pop >= net->n_pops) return -1;
    memcpy(out, net->pops[pop].spk_prev, (size_t)net->pops[pop].n);
    return 0;
}

int orc_set_last_spikes(orc_net *net, int pop, const unsigned char *in)
{
    if (pop < 0 || pop >= net->n_pops) return -1;
    memcpy(net->pops[pop].spk_prev, in, (size_t)net->pops[pop].n);
    return 0;
}

int64_t orc_nan_count(orc_net *net) { return net->nan_count; }
void orc_set_threads(orc_net *net, int n) { net->threads = n; }
int64_t orc_time(orc_net *net) { return net->t; }
void orc_set_g_scale(orc_net *net, double s) { net->g_scale = s; }

void orc_log_events(orc_net *net, int on) { net->log_events = on; }
int64_t orc_event_count(orc_net *net) { return net->ev_n; }

/* Copy and clear the event log. */
int64_t orc_take_events(orc_net *net, int32_t *t, int32_t *pop, int32_t *id, int64_t cap)
{
    int64_t n = net->ev_n < cap ? net->ev_n : cap;
    memcpy(t, net->ev_t, sizeof(int32_t) * (size_t)n);
    memcpy(pop, net->ev_pop, sizeof(int32_t) * (size_t)n);
    memcpy(id, net->ev_id, sizeof(int32_t) * (size_t)n);
    net->ev_n = 0;
    return n;
}

/* Replay: population pop takes its spikes of step t from ids[off[t*n_pops+pop]
 * .. off[t*n_pops+pop+1]) instead of detecting or drawing them.  The arrays
 * stay owned by the caller and must outlive the steps that read them. */
int orc_set_replay(orc_net *net, int pop, int on, const int64_t *off, const int32_t *ids, int64_t T)
{
    if (pop < 0 || pop >= net->n_pops) return -1;
    net->pops[pop].replay = on;
    net->rp_off = off;
    net->rp_ids = ids;
    net->rp_T = T;
    return 0;
}

void orc_destroy(orc_net *net)
{
    if (!net) return;
    for (int p = 0; p < net->n_pops; ++p) {
        opop *P = &net->pops[p];
        free(P->V); free(P->m); free(P->h); free(P->nn);
        free(P->spk_prev); free(P->spk_now); free(P->count); free(P->vsum);
        free(P->iza); free(P->izb); free(P->izc); free(P->izd);
    }
    for (int q = 0; q < net->n_projs; ++q) {
        oproj *Q = &net->projs[q];
        free(Q->row_ptr); free(Q->col_idx); free(Q->g); free(Q->G);
        free(Q->x); free(Q->y); free(Q->col_ptr); free(Q->row_of); free(Q->perm);
    }
    free(net->ev_t); free(net->ev_pop); free(net->ev_id);
    free(net);
}
