/*
 * FP64 reverse-time adjoint of the spiking network with the spike raster
 * held fixed (the oracle of the gradient).
 *
 * TEST INFRASTRUCTURE ONLY, like snn_oracle.c.
 *
 * Loss: any function of the time-averaged post-step voltage of one
 * population, Vbar_j = (1/T) sum_{t<T} V_j(t); the caller supplies
 * dL/dVbar.  Spikes are constants of the objective (a spike changes only
 * through a discrete event, which has no derivative), so V of the loss
 * population depends on every other population only through its fixed
 * raster: the adjoint lives on the loss population alone, and only
 * projections into it receive nonzero gradients.
 *
 * Per step t the loss neuron j computes (forward, as in snn_oracle.c):
 *   Ginj_q = G_q(t-1) + s * sum_{i in S_pre(t-1)} g_{ij}        (delivery)
 *   I      = sum_q Ginj_q (E_q - V(t-1)) + I_ext                (held fixed)
 *   x_{k+1} = x_k + h f(x_k, I), x_0 = x(t-1), x(t) = x_S        (Euler)
 *   G_q(t) = d_q Ginj_q                                          (decay)
 * and the reverse pass applies the transposed Jacobian of each of these in
 * the opposite order, accumulating dL/dg_{ij} and dL/ds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "snn_oracle.h"

/* d/dx [x / (e^x - 1)] = (e^x - 1 - x e^x) / (e^x - 1)^2; near 0 the series
 * -1/2 + x/6 - x^3/180 avoids the cancellation. */
double orc_dphi(double x)
{
    if (fabs(x) < 1e-3) return -0.5 + x / 6.0 - x * x * x / 180.0;
    double em1 = expm1(x);
    double num = em1 * (1.0 - x) - x;     /* e^x - 1 - x e^x */
    return num / (em1 * em1);
}

/* Derivatives of the six rates with respect to V. */
static void rate_derivs(double V, double *dam, double *dbm, double *dah, double *dbh, double *dan, double *dbn)
{
    *dam = 1.28 * orc_dphi((-52.0 - V) / 4.0) * (-0.25);
    *dbm = 1.4 * orc_dphi((V + 25.0) / 5.0) * 0.2;
    *dah = -orc_alpha_h(V) / 18.0;
    double ez = exp((-25.0 - V) / 5.0);
    *dbh = 4.0 * ez / ((ez + 1.0) * (ez + 1.0)) * 0.2;
    *dan = 0.16 * orc_dphi((-50.0 - V) / 5.0) * (-0.2);
    *dbn = -orc_beta_n(V) / 40.0;
}

/* Vector-Jacobian product of one substep x' = x + hs f(x, i_in) at x:
 * lam_in = lam_out^T dx'/dx, and *lam_iin += lam_out^T dx'/di_in. */
void orc_substep_vjp(const double *p, double hs, const double *x, const double *lam_out, double *lam_in,
                     double *lam_iin)
{
    const double V = x[0], m = x[1], h = x[2], n = x[3];
    const double C = p[HH_CM];
    const double am = orc_alpha_m(V), bm = orc_beta_m(V);
    const double ah = orc_alpha_h(V), bh = orc_beta_h(V);
    const double an = orc_alpha_n(V), bn = orc_beta_n(V);
    double dam, dbm, dah, dbh, dan, dbn;
    rate_derivs(V, &dam, &dbm, &dah, &dbh, &dan, &dbn);
    /* partial derivatives of f_V = (i_in - I_ion) / C */
    const double dfV_dV = -(p[HH_GNA] * m * m * m * h + p[HH_GK] * n * n * n * n + p[HH_GL]) / C;
    const double dfV_dm = -3.0 * p[HH_GNA] * m * m * h * (V - p[HH_ENA]) / C;
    const double dfV_dh = -p[HH_GNA] * m * m * m * (V - p[HH_ENA]) / C;
    const double dfV_dn = -4.0 * p[HH_GK] * n * n * n * (V - p[HH_EK]) / C;
    /* gates: f_x = a (1 - x) - b x */
    const double dfm_dV = dam * (1.0 - m) - dbm * m, dfm_dm = -(am + bm);
    const double dfh_dV = dah * (1.0 - h) - dbh * h, dfh_dh = -(ah + bh);
    const double dfn_dV = dan * (1.0 - n) - dbn * n, dfn_dn = -(an + bn);
    const double lV = lam_out[0], lm = lam_out[1], lh = lam_out[2], ln = lam_out[3];
    lam_in[0] = lV + hs * (lV * dfV_dV + lm * dfm_dV + lh * dfh_dV + ln * dfn_dV);
    lam_in[1] = lm + hs * (lV * dfV_dm + lm * dfm_dm);
    lam_in[2] = lh + hs * (lV * dfV_dh + lh * dfh_dh);
    lam_in[3] = ln + hs * (lV * dfV_dn + ln * dfn_dn);
    *lam_iin += hs * lV / C;
}

/* Run T steps from the net's current state (which must be its initial state:
 * the adjoint stops there) recording the loss population's trajectory, then
 * the reverse pass.  dLdg[q] receives nnz_q doubles for every projection q
 * (zero for projections not into loss_pop), *dLds the derivative with
 * respect to g_scale, vbar_out (may be NULL) the forward's Vbar.
 * Returns 0, or -1 for a bad argument or a plastic network. */
int orc_adjoint(orc_net *net, int64_t T, int loss_pop, const double *dLdVbar, double *const *dLdg, double *dLds,
                double *vbar_out)
{
    if (!net->ready || T < 1 || loss_pop < 0 || loss_pop >= net->n_pops) return -1;
    opop *L = &net->pops[loss_pop];
    if (L->kind != ORC_HH) return -1;
    for (int q = 0; q < net->n_projs; ++q)
        if (net->projs[q].stdp) return -1;
    const int n = L->n;
    int in[ORC_MAX_PROJS], n_in = 0;
    for (int q = 0; q < net->n_projs; ++q)
        if (net->projs[q].post == loss_pop) in[n_in++] = q;

    /* tape: x(t-1) and Ginj(t) of every loss neuron, spikes S_pre(t-1) of
     * every incoming projection */
    double *xs = (double *)malloc(sizeof(double) * (size_t)T * n * 4);
    double *ginj = (double *)malloc(sizeof(double) * (size_t)T * n * (n_in > 0 ? n_in : 1));
    unsigned char **spk = (unsigned char **)calloc((size_t)(n_in > 0 ? n_in : 1), sizeof(unsigned char *));
    for (int a = 0; a < n_in; ++a)
        spk[a] = (unsigned char *)malloc((size_t)T * net->pops[net->projs[in[a]].pre].n + 1);
    double *vsum = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));

    for (int64_t t = 0; t < T; ++t) {
        for (int j = 0; j < n; ++j) {
            double *x = xs + ((size_t)t * n + j) * 4;
            x[0] = L->V[j]; x[1] = L->m[j]; x[2] = L->h[j]; x[3] = L->nn[j];
        }
        for (int a = 0; a < n_in; ++a) {
            const opop *pre = &net->pops[net->projs[in[a]].pre];
            memcpy(spk[a] + (size_t)t * pre->n, pre->spk_prev, (size_t)pre->n);
        }
        orc_phase_deliver(net);
        for (int a = 0; a < n_in; ++a)
            for (int j = 0; j < n; ++j) ginj[((size_t)t * n_in + a) * n + j] = net->projs[in[a]].G[j];
        orc_phase_potentiate(net);
        orc_phase_neurons(net);
        orc_phase_finish(net);
        for (int j = 0; j < n; ++j) vsum[j] += L->V[j];
    }
    if (vbar_out)
        for (int j = 0; j < n; ++j) vbar_out[j] = vsum[j] / (double)T;

    for (int q = 0; q < net->n_projs; ++q) memset(dLdg[q], 0, sizeof(double) * (size_t)net->projs[q].nnz);
    double dls = 0.0;
    const double hs = net->dt / net->substeps;
    const int S = net->substeps;
    double *lam = (double *)calloc((size_t)n * 4 + 1, sizeof(double));        /* adjoint of x(t) */
    double *lamG = (double *)calloc((size_t)n * (n_in > 0 ? n_in : 1), sizeof(double));   /* of G(t) */
    double *lamGinj = (double *)calloc((size_t)n * (n_in > 0 ? n_in : 1), sizeof(double));
    double *sub = (double *)malloc(sizeof(double) * (size_t)(S + 1) * 4);
    double *decay = (double *)malloc(sizeof(double) * (size_t)(n_in > 0 ? n_in : 1));
    for (int a = 0; a < n_in; ++a) decay[a] = exp(-net->dt / net->projs[in[a]].tau);

    for (int64_t t = T - 1; t >= 0; --t) {
        for (int j = 0; j < n; ++j) {
            double *lj = lam + (size_t)j * 4;
            lj[0] += dLdVbar[j] / (double)T;                /* V(t) enters Vbar */
            const double *x0 = xs + ((size_t)t * n + j) * 4;
            double isyn = L->i_ext;
            for (int a = 0; a < n_in; ++a)
                isyn += ginj[((size_t)t * n_in + a) * n + j] * (net->projs[in[a]].e_rev - x0[0]);
            memcpy(sub, x0, sizeof(double) * 4);
            for (int k = 0; k < S; ++k) {
                double *y = sub + (size_t)(k + 1) * 4;
                memcpy(y, sub + (size_t)k * 4, sizeof(double) * 4);
                orc_substep(L->hh, hs, isyn, &y[0], &y[1], &y[2], &y[3]);
            }
            double lam_i = 0.0, tmp[4];
            for (int k = S - 1; k >= 0; --k) {
                orc_substep_vjp(L->hh, hs, sub + (size_t)k * 4, lj, tmp, &lam_i);
                memcpy(lj, tmp, sizeof tmp);
            }
            double gsum = 0.0;
            for (int a = 0; a < n_in; ++a) {
                const double gi = ginj[((size_t)t * n_in + a) * n + j];
                gsum += gi;
                lamGinj[(size_t)a * n + j] = decay[a] * lamG[(size_t)a * n + j] +
                                             lam_i * (net->projs[in[a]].e_rev - x0[0]);
            }
            lj[0] += -lam_i * gsum;                         /* I depends on V(t-1) */
        }
        /* Ginj(t) = G(t-1) + s sum_{i in S_pre(t-1)} g_ij */
        for (int a = 0; a < n_in; ++a) {
            const oproj *Q = &net->projs[in[a]];
            const int npre = net->pops[Q->pre].n;
            const unsigned char *f = spk[a] + (size_t)t * npre;
            for (int i = 0; i < npre; ++i) {
                if (!f[i]) continue;
                for (int32_t k = Q->row_ptr[i]; k < Q->row_ptr[i + 1]; ++k) {
                    const double lg = lamGinj[(size_t)a * n + Q->col_idx[k]];
                    dLdg[in[a]][k] += net->g_scale * lg;
                    dls += Q->g[k] * lg;
                }
            }
            memcpy(lamG + (size_t)a * n, lamGinj + (size_t)a * n, sizeof(double) * (size_t)n);
        }
    }
    *dLds = dls;
    free(xs); free(ginj); free(vsum); free(lam); free(lamG); free(lamGinj); free(sub); free(decay);
    for (int a = 0; a < n_in; ++a) free(spk[a]);
    free(spk);
    return 0;
}
