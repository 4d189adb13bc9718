/*
 * Private declarations of the FP64 oracle (test infrastructure only): the
 * network structures shared by the forward simulator (snn_oracle.c) and the
 * adjoint (snn_adjoint.c).
 */
#ifndef SNN_ORACLE_PRIVATE_H
#define SNN_ORACLE_PRIVATE_H

#include <stdint.h>

enum { ORC_POISSON = 0, ORC_HH = 1, ORC_IZH = 2 };
enum { HH_GNA = 0, HH_ENA, HH_GK, HH_EK, HH_GL, HH_EL, HH_CM, HH_NPARAM };

/* ------------------------------------------------------------------ */
/* Network                                                            */
/* ------------------------------------------------------------------ */
#define ORC_MAX_POPS 16
#define ORC_MAX_PROJS 32

typedef struct {
    int kind, n;
    double rate_hz, i_ext, hh[HH_NPARAM];
    uint64_t thresh;
    double *V, *m, *h, *nn;      /* HH state; Izhikevich: v in V, u in m */
    double *iza, *izb, *izc, *izd;  /* Izhikevich parameters per neuron (fp32 input widened) */
    unsigned char *spk_prev;     /* spikes of the previous step */
    unsigned char *spk_now;      /* spikes of the current step */
    int32_t *count;              /* spikes per neuron since init */
    double *vsum;                /* sum of post-step V since init */
    int replay;                  /* 1: spikes come from the replay raster */
} opop;

typedef struct {
    int pre, post;
    int64_t nnz;
    int32_t *row_ptr, *col_idx;
    double *g;                   /* fp32 input widened exactly */
    double e_rev, tau;
    double *G;                   /* post-side conductance, n_post */
    int stdp;
    double a_plus, a_minus, tau_stdp, g_max;
    double *x, *y;               /* pre and post traces */
    int32_t *col_ptr, *row_of, *perm;  /* column view for potentiation */
} oproj;

typedef struct orc_net {
    double dt;
    int substeps;
    double g_scale;
    uint64_t seed;
    int n_pops, n_projs;
    opop pops[ORC_MAX_POPS];
    oproj projs[ORC_MAX_PROJS];
    int64_t t;                   /* index of the next step */
    int64_t nan_count;           /* HH neurons whose V turned non-finite */
    int ready;
    int threads;                 /* >1: the HH neuron loop runs on that many OpenMP threads */
    /* event log: (t, pop, id) of every spike, when enabled */
    int log_events;
    int64_t ev_n, ev_cap;
    int32_t *ev_t, *ev_pop, *ev_id;
    /* replay raster for populations marked replay: per step, per pop, ids */
    const int64_t *rp_off;       /* [(t * n_pops + pop)] -> start in rp_ids; size T*n_pops+1 */
    const int32_t *rp_ids;
    int64_t rp_T;
} orc_net;


double orc_phi(double x);
double orc_alpha_m(double V);
double orc_beta_m(double V);
double orc_alpha_h(double V);
double orc_beta_h(double V);
double orc_alpha_n(double V);
double orc_beta_n(double V);
void orc_substep(const double *p, double hs, double i_in, double *V, double *m, double *h, double *n);
void orc_izh_substep(double a, double b, double hs, double i_in, double *v, double *u);
void orc_phase_deliver(orc_net *net);
void orc_phase_potentiate(orc_net *net);
void orc_phase_neurons(orc_net *net);
void orc_phase_finish(orc_net *net);

#endif
