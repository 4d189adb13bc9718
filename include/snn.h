/*
 * snn.h - C ABI of the MI355X spiking-network timestep library (libsnn.so).
 *
 * The library advances networks of Hodgkin-Huxley neurons (Traub-Miles
 * kinetics), Izhikevich neurons and Poisson input sources, coupled by
 * conductance synapses kept
 * in Compressed Row Storage, one discrete time step at a time.  This is the
 * per-timestep update that the paper (Balaji, Yavuz, Nowotny, "Scalability
 * and Optimization Strategies for GPU Enhanced Neural Networks") runs inside
 * GeNN: Hodgkin-Huxley integration at discretised time steps (Section 2),
 * sparse synapse propagation through the three CRS arrays (Section 3,
 * Eq. 1), and the many-network conductance-scaling sweep (Section 2, Fig. 1)
 * as a batch of independent instances.
 *
 * Conventions
 *  - Units: mV, ms, uS (conductance), nF, nA, Hz.
 *  - Every function returns an snn_status (0 = SNN_OK, negative = error)
 *    unless stated otherwise; snn_last_error() gives a message for the last
 *    failure on the calling thread.  No exception crosses the ABI.
 *  - A device error is sticky: once a HIP call has failed, every later call
 *    on that net returns SNN_EDEVICE.
 *  - "host" pointers are caller-owned CPU memory of the stated size;
 *    "device" pointers are caller-owned GPU memory valid on the net's stream.
 *  - A NaN or infinite membrane voltage is not an error: it is counted per
 *    instance (snn_get_nan_counts), like the sumNANs column of Fig. 1.
 */
#ifndef SNN_ABI_H_
#define SNN_ABI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct snn_net snn_net; /* opaque, library-owned */

enum snn_status {
    SNN_OK = 0,
    SNN_EINVAL = -1,  /* invalid argument or network description */
    SNN_ENOMEM = -2,  /* device or host allocation failed */
    SNN_EDEVICE = -3, /* a HIP call failed (sticky) */
    SNN_ESTATE = -4,  /* call not valid in the net's current state */
    SNN_ERANGE = -5   /* value outside the representable range */
};

enum snn_pop_kind { SNN_POISSON = 0, SNN_TRAUB_MILES = 1, SNN_IZHIKEVICH = 2 };

/* State variables: V, m, h, n of a Traub-Miles population; V and the
 * recovery variable u (SNN_U) of an Izhikevich population. */
enum snn_var { SNN_V = 0, SNN_M = 1, SNN_H = 2, SNN_N = 3, SNN_U = 1 };

/* Neuron parameters, in this order: g_Na (uS), E_Na (mV), g_K (uS),
 * E_K (mV), g_leak (uS), E_leak (mV), C_m (nF). */
enum { SNN_HH_NPARAM = 7 };

/* A population (Section 5.1: networks are built of populations of neurons).
 *  kind      SNN_POISSON: source i fires at step t iff the first output word
 *            of Philox-4x32-10 (Salmon et al., SC'11) with counter
 *            (i, t mod 2^32, t div 2^32, pop), pop the population's index in
 *            its instance, and key (seed mod 2^32,
 *            seed div 2^32) is below floor(p * 2^32), p = rate_hz * dt_ms *
 *            1e-3 evaluated left to right in double precision (p >= 1:
 *            always fires).
 *            SNN_TRAUB_MILES: Hodgkin-Huxley neuron, Traub-Miles rates
 *            (the neuron model of Section 2).
 *            SNN_IZHIKEVICH: the neuron of the 4:1 excitatory/inhibitory
 *            network of Section 5.1, the model of its reference [9]
 *            (Izhikevich, IEEE TNN 14, 2003): v' = 0.04 v^2 + 5 v + 140 -
 *            u + I and u' = a (b v - u), both right-hand sides from the
 *            substep-start state in each Euler substep; after the step's
 *            substeps, v >= 30 mV is a spike and resets v <- c, u <- u + d.
 *            I (synaptic + i_ext_nA) enters v' as is.  Starts at v = -65 mV,
 *            u = b v.
 *  n         number of neurons (>= 0).
 *  rate_hz   Poisson rate (finite, >= 0); ignored otherwise.
 *  i_ext_nA  constant injected current of every HH or Izhikevich neuron.
 *  hh        neuron parameters (see above); snn_default_hh() fills the
 *            Traub-Miles values.  C_m must be > 0.  Traub-Miles only.
 *  record_vbar  1: accumulate every neuron's post-step V in double
 *            precision (read with snn_get_vbar).
 *  izh_abcd  Izhikevich only: host float[4 * n], parameter-major (a[0..n),
 *            then b, c, d), all finite; copied at create.  NULL otherwise. */
typedef struct {
    int32_t kind;
    int32_t n;
    double rate_hz;
    double i_ext_nA;
    double hh[SNN_HH_NPARAM];
    int32_t record_vbar;
    const float *izh_abcd;
} snn_pop_desc;

/* A projection in Compressed Row Storage (Section 3): row_ptr holds the
 * start of every pre-synaptic row (n_pre + 1 entries, row_ptr[0] = 0,
 * non-decreasing, row_ptr[n_pre] = nnz); col_idx the post-synaptic index of
 * every synapse, ascending within a row; g its conductance (uS, finite,
 * >= 0).  A spike of pre neuron i at step t - 1 adds g_scale * g[k] to the
 * conductance G[col_idx[k]] of the post population for every k in row i at
 * step t; G enters the post neuron as G (e_rev_mV - V) and decays by
 * exp(-dt / tau_ms) per step.  The post population must be Traub-Miles or
 * Izhikevich.
 *
 * stdp = 1 makes the weights plastic with pair-based, all-to-all traces
 * (trace time constant tau_stdp_ms): on a pre spike, every synapse of its
 * row is depressed by a_minus * g_max * y_post after delivery; on a post
 * spike, every synapse of its column is potentiated by a_plus * g_max *
 * x_pre; weights are clipped to [0, g_max] after each update. */
typedef struct {
    int32_t pre_pop;
    int32_t post_pop;
    int64_t nnz;
    const int32_t *row_ptr; /* host, n_pre + 1 */
    const int32_t *col_idx; /* host, nnz */
    const float *g;         /* host, nnz */
    float e_rev_mV;
    float tau_ms;
    int32_t stdp;
    float a_plus, a_minus, tau_stdp_ms, g_max;
} snn_proj_desc;

/* One independent network instance.  g_scale multiplies every synaptic
 * conductance of the instance (the gScale of Section 5.1); seed keys its
 * Poisson sources. */
typedef struct {
    int32_t n_pops;
    int32_t n_projs;
    const snn_pop_desc *pops;   /* host, n_pops */
    const snn_proj_desc *projs; /* host, n_projs */
    float g_scale;
    uint64_t seed;
} snn_instance_desc;

/* Device memory hooks: alloc(bytes, ctx) returns device memory or NULL,
 * free(ptr, ctx) releases it.  Both NULL: hipMalloc / hipFree. */
typedef void *(*snn_alloc_fn)(size_t bytes, void *ctx);
typedef void (*snn_free_fn)(void *ptr, void *ctx);

/* Whole-batch configuration.
 *  dt_ms, substeps  time step and number of forward-Euler substeps (>= 1)
 *  n_instances, inst  the batch (>= 1 instance)
 *  stream        hipStream_t every call enqueues on (NULL: the null stream)
 *  raster_steps  > 0: keep the spike bitmask of the last raster_steps steps
 *                on the device (snn_get_raster); 0: no raster
 *  autotune      1: time candidate launch shapes on this network at create
 *                and keep the fastest (results do not depend on it)
 *  tune_cache    path of a JSON file that stores tuned shapes per network
 *                signature, or NULL */
typedef struct {
    double dt_ms;
    int32_t substeps;
    int32_t n_instances;
    const snn_instance_desc *inst;
    void *stream;
    snn_alloc_fn alloc;
    snn_free_fn free;
    void *alloc_ctx;
    int32_t raster_steps;
    int32_t autotune;
    const char *tune_cache;
} snn_config;

/* Launch shape of the step kernels (see snn_get_launch).  Every choice gives
 * bit-identical results (conductances are integer multiples of 2^-40 uS, so
 * the order of deliveries does not matter); they differ only in speed. */
typedef struct {
    int32_t neuron_block;   /* threads per block of the neuron update: 64..1024, multiple of 64 */
    int32_t prop_blocks;    /* blocks of the propagation kernel (persistent grid) */
    int32_t prop_block;     /* threads per block of the row-mode propagation kernel */
    int32_t chunk;          /* synapses per work item of a row or column walk, multiple of 64 */
    int32_t mode;           /* delivery: 0 rows (a wavefront per row chunk, atomics into G;
                               sparse activity), 1 tiles (a wavefront per post tile and group of
                               active spike words, LDS accumulation; dense activity; the
                               non-plastic projections of a population with at least 7/8 of
                               its neurons spiking at t-1 are pulled instead: one lane per post
                               neuron sums its column from a column-ordered copy), 2 fused
                               (no propagation kernel: each neuron-update block delivers its
                               own spikes' row chunks with atomics into a double-buffered
                               delivery buffer that the next update adds to G; only for
                               networks without plastic projections), 3 grouped (rows, except
                               that every non-plastic projection onto at most 1024 neurons,
                               with at most 60% of the (pre, post) pairs connected and rows
                               of fewer than 768 synapses on average, is delivered
                               in groups of 2 to 6 of its spiking rows (about 1536 synapses),
                               taken in spike-word order: a wavefront sums a group's synapses in
                               an LDS copy of the post population's conductances and adds
                               its nonzero entries into G with atomics; prop_block <= 512) */
} snn_launch;

/* Fill p[0..6] with the Traub-Miles parameters (7.15 uS, 50 mV, 1.43 uS,
 * -95 mV, 0.02672 uS, -63.563 mV, 0.143 nF). */
void snn_default_hh(double *p);

/* Validate the description, copy every host array to the device and set
 * every Traub-Miles neuron to its resting point (the root of the
 * steady-state membrane current in [-80, -60] mV), every Izhikevich neuron
 * to v = -65 mV, u = b v, conductances and traces
 * to 0, step counter to 0.  All-or-nothing: on failure *out = NULL.
 * SNN_ERANGE for more than 2^29 neurons in all (each population padded to a
 * multiple of 64), or for weights outside the conductance range.
 * Device memory beyond the state: the CRS arrays (8 B per synapse plus row
 * starts); for every non-plastic projection a column-ordered copy used by
 * tile mode's pull delivery (each entry a one-byte row delta, its fp32
 * weight and its 4-byte weight-pool position: 9 B per synapse, plus
 * weight-0 entries bridging row gaps above 255, padding of its 64-column
 * slices to their longest column and 4 B per column and pull unit), built
 * only while the weight pool has fewer than 2^31 synapses and for
 * projections whose bridging entries stay within a quarter of their
 * synapses (the others are always pushed); for plastic projections the column view of
 * potentiation (8 B per synapse); the tile-mode partial tiles (8 B per post
 * tile column and pre spike word); the work queues. */
int snn_create(const snn_config *cfg, snn_net **out);

/* Release every device buffer.  NULL is ignored. */
void snn_destroy(snn_net *net);

/* Enqueue n_steps timesteps on the net's stream and return (asynchronous):
 * the per-timestep update of Section 2 (Hodgkin-Huxley neurons integrated
 * at discrete time steps) with spike propagation through the CRS arrays of
 * Section 3.  Each step t: (1) deliver the spikes of step t-1 through every projection
 * (and depress plastic rows), (2) potentiate plastic columns of post neurons
 * that spiked at t-1, (3) update every neuron: synaptic current from the
 * start-of-step V, `substeps` Euler substeps, conductance decay, spike iff
 * V(t-1) < 0 <= V(t); Poisson sources draw their spikes of step t. */
int snn_step(snn_net *net, int64_t n_steps);

/* Wait for all work enqueued on the net's stream. */
int snn_sync(snn_net *net);

/* Number of steps taken so far (host-side counter). */
int64_t snn_time(const snn_net *net);

/* Spike count of every neuron of population pop of instance inst since
 * create (host int32[n]): the per-neuron counts that the avgSpike of Fig. 1
 * averages (Section 5.1).  Synchronises. */
int snn_get_spikes(snn_net *net, int32_t inst, int32_t pop, int32_t *counts);

/* Spike raster (the spike times of the discrete-time simulation of
 * Section 2) of population pop of instance inst for steps [t0, t1), which must
 * lie within the last raster_steps steps, or, after snn_forward_record and
 * until the next reset, within the recorded steps.  offsets (host int64[t1-t0+1])
 * receives the start of each step's ids in `ids` (host int32[cap]),
 * ascending within a step.  Returns SNN_ERANGE if cap is too small
 * (offsets[t1-t0] still holds the needed size).  Synchronises. */
int snn_get_raster(snn_net *net, int32_t inst, int32_t pop, int64_t t0, int64_t t1,
                   int64_t *offsets, int32_t *ids, int64_t cap);

/* Read / write one state variable (enum snn_var; the neuron state that the
 * Hodgkin-Huxley integration of Section 2 advances) of a Traub-Miles or
 * Izhikevich population (SNN_V or SNN_U for the latter; SNN_EINVAL for a
 * Poisson population) as float (host float[n]); the read returns the rounded value
 * of the stored double-float pair, the write sets the pair to the value
 * exactly.  Synchronise. */
int snn_get_state(snn_net *net, int32_t inst, int32_t pop, int32_t var, float *out);
int snn_set_state(snn_net *net, int32_t inst, int32_t pop, int32_t var, const float *in);

/* The same in double precision (host double[n]): the exact sum of the
 * stored pair on read; on write the pair (hi = fl32(x), lo = fl32(x - hi)). */
int snn_get_state_f64(snn_net *net, int32_t inst, int32_t pop, int32_t var, double *out);
int snn_set_state_f64(snn_net *net, int32_t inst, int32_t pop, int32_t var, const double *in);

/* Post-side conductance G (uS) of projection proj of instance inst (host
 * double[n_post]).  G is held as a signed 64-bit multiple of 2^-40 uS, so
 * sums of deliveries do not depend on their order; the write rounds to that
 * grid.  Synchronise. */
int snn_get_conductance(snn_net *net, int32_t inst, int32_t proj, double *out);
int snn_set_conductance(snn_net *net, int32_t inst, int32_t proj, const double *in);

/* Spikes of the last completed step of population pop as 0/1 bytes (host
 * uint8[n]); the write replaces them (they are delivered at the next step).
 * Synchronise. */
int snn_get_last_spikes(snn_net *net, int32_t inst, int32_t pop, uint8_t *out);
int snn_set_last_spikes(snn_net *net, int32_t inst, int32_t pop, const uint8_t *in);

/* Sum of post-step V (double, host double[n]) over all steps since create,
 * for a population created with record_vbar = 1.  Synchronises. */
int snn_get_vbar(snn_net *net, int32_t inst, int32_t pop, double *out);

/* Per instance, how many neurons had a V within the single-precision range
 * at the start of a step and outside it at its end (|V| at or above FLT_MAX
 * plus half its ulp, which rounds to infinity, or NaN): the sumNANs of
 * Fig. 1, whose caption says the count covers overflow.  Each neuron counts
 * once, at the step its V leaves the range (host int32[n_instances]). */
int snn_get_nan_counts(snn_net *net, int32_t *per_instance);

/* Replace every instance's g_scale (host float[n_instances], finite, >= 0).
 * Every delivery from the next step on uses the new values, including that of
 * the spikes of the last step taken.  SNN_ERANGE if a conductance could leave
 * the fixed-point range (the same rule as at create).  Synchronises. */
int snn_set_gscale(snn_net *net, const float *per_instance);

/* Current weights of projection proj of instance inst (host float[nnz]). */
int snn_get_weights(snn_net *net, int32_t inst, int32_t proj, float *out);

/* Device memory of each projection's CRS arrays in bytes, as stored:
 * 4 * (2 * nnz + n_pre + 1), i.e. Eq. (1) with a row-start array of
 * n_pre + 1 entries (host int64[total projections, instance-major]). */
int snn_memory_bytes(const snn_net *net, int64_t *per_proj_bytes);

/* Current / new launch shape; snn_set_launch validates the ranges above
 * (SNN_EINVAL, also for mode 2 on a network with plastic projections and for
 * mode 3 with prop_block above 512; the launch is then left as it was).  A
 * change of mode converts the work pending for the next step (delivers it
 * now, or folds fused deliveries into G); results are unchanged.
 * Synchronises when the mode changes. */
int snn_get_launch(const snn_net *net, snn_launch *out);
int snn_set_launch(snn_net *net, const snn_launch *in);

/* Time n_steps steps (hipEvents around the enqueued work) after restoring
 * the state in between; out_ms gets the mean milliseconds per step.  Used by
 * the autotuner; leaves the net's state as it found it. */
int snn_time_steps(snn_net *net, int64_t n_steps, double *out_ms);

/* Mean milliseconds per launch of one step kernel (which: 0 propagation,
 * 1 potentiation, 2 neuron update), timed with one hipEvent pair around
 * `launches` back-to-back launches of that kernel alone on the net's
 * current state; the state is restored afterwards.  Propagation and
 * potentiation consume the same pending work items at every launch.
 * SNN_ESTATE for the propagation (which 0) in mode 2 (fused), where the
 * neuron update delivers.  Synchronises. */
int snn_time_kernel(snn_net *net, int32_t which, int64_t launches, double *ms_per_launch);

/* Advance the network by n_steps (1..100000) steps, exactly as snn_step
 * does, but with every kernel launched directly (no graph) together with a
 * start/stop hipEvent pair that the runtime stamps with that dispatch's own
 * begin and end times.  On return ms_total[k] is the summed kernel
 * duration and launches[k] the number of launches of kernel k (0
 * propagation, 1 potentiation, 2 neuron update) over those steps: the
 * per-kernel average duration of a live sequence of steps.  Both arrays
 * are caller-owned host arrays of 3 elements.  Synchronises. */
int snn_profile_steps(snn_net *net, int64_t n_steps, double *ms_total, int64_t *launches);

/* Restore the state created by snn_create: every Traub-Miles neuron at its
 * resting point, every Izhikevich neuron at v = -65 mV, u = b v, conductances, traces, counts, Vbar sums, NaN counts and
 * spikes at zero, step counter 0.  Weights (including STDP changes) and
 * g_scale are kept.  Enqueued on the net's stream. */
int snn_reset(snn_net *net);

/* Total number of synapses of the batch (the length of the weight pool),
 * or -1 for NULL.  The pool holds the weights of every projection in
 * instance-major, projection order, each in CRS order; snn_weight_offset
 * gives where (inst, proj) starts. */
int64_t snn_weight_count(const snn_net *net);
int snn_weight_offset(const snn_net *net, int32_t inst, int32_t proj, int64_t *offset);

/* Copy the whole weight pool to / from caller-owned device memory
 * (float[snn_weight_count]) on the net's stream.  The write checks on the
 * device that every weight is finite and >= 0 (SNN_EINVAL otherwise) and
 * applies the range rules of snn_create with the current g_scale
 * (SNN_ERANGE); on either error nothing is copied.  It synchronises for
 * those checks.  New weights apply to every delivery from the next step,
 * including that of the last step's spikes (in mode 2 the pending
 * deliveries are redone). */
int snn_get_weights_device(snn_net *net, float *dst_dev);
int snn_set_weights_device(snn_net *net, const float *src_dev);

/* Forward pass recorded for the adjoint (the "differentiation" extension:
 * gradients of a loss on the time-averaged voltage Vbar of population pop
 * with respect to every weight and every g_scale).  Resets the net
 * (snn_reset), runs n_steps steps keeping the spike bitmask of every step
 * and a checkpoint of the neuron state every ckpt_every steps, and writes
 * Vbar_j = (1/n_steps) sum_t V_j(t) of population pop of every instance to
 * vbar_dev (device double[sum over instances of n_pop], instance-major).
 * Requires: population pop created with record_vbar = 1 in every instance,
 * at most 1024 neurons per instance, substeps <= 8, no plastic projection.
 * Device memory: 8 B per neuron-wave word per step (raster) + (32 B per
 * neuron + 8 B per conductance) per checkpoint. */
int snn_forward_record(snn_net *net, int32_t pop, int64_t n_steps, int32_t ckpt_every, double *vbar_dev);

/* Reverse pass of the last snn_forward_record, exact for the discrete
 * forward map with the recorded spike raster held fixed.  dL_dvbar_dev
 * (device double, same layout as vbar_dev) is the loss gradient; the call
 * writes dL/dg for every synapse into dL_dg_dev (device float[weight
 * count], weight-pool order; projections that do not reach pop get 0) and
 * dL/dg_scale into dL_dgscale_dev (device double[n_instances], accumulated
 * in double).  Each segment between checkpoints is recomputed from its
 * checkpoint; *mismatch (may be NULL; then the call stays asynchronous)
 * receives the number of state values at which a recomputed segment end
 * differs from the next stored checkpoint (0 expected). */
int snn_backward(snn_net *net, const double *dL_dvbar_dev, float *dL_dg_dev, double *dL_dgscale_dev,
                 int64_t *mismatch);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * backward pass of snn_backward, with the same kernels and results, but its
 * scratch -- the per-segment tape of recomputed states and delivered
 * conductances, their adjoints and the adjoint carried from segment to
 * segment, 8 * n_loss * (K * (4 + 2 * n_in) + 4 + n_in) + 256 bytes for
 * n_loss loss neurons over the batch, checkpoint interval K and at most
 * n_in projections into a loss neuron -- in a fixed library-wide device
 * array of SNN_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends)
 * instead of the net's buffers.  It calls no allocator and records no memset
 * (outputs and scratch are cleared by a kernel).  Arguments as snn_backward
 * (no recompute check is reported).  SNN_ERANGE if the recording needs more
 * scratch than the array holds; SNN_ESTATE without a recording.  All calls
 * on one GPU share the array and it keeps the last call's contents: calls
 * that overlap on one GPU (any nets, any streams) race and give wrong
 * gradients; serialise them. */
enum { SNN_NOALLOC_SCRATCH_BYTES = 64 << 20 };
int snn_backward_noalloc(snn_net *net, const double *dL_dvbar_dev, float *dL_dg_dev, double *dL_dgscale_dev);

/* ---------------- Conductance-scale calibration (Section 5.1) ----------------
 * Host routines over the per-run table of a conductance-scaling sweep (one
 * row per run: nConn, gScale, avgSpike, NaN count), as in Fig. 1.  They keep
 * no net, touch no GPU and allocate only host scratch. */

/* Fig. 1's selection.  n_conn, g_scale, avg_spike: host double[n_runs];
 * n_nans: host int32[n_runs] (the run's NaN count, snn_get_nan_counts);
 * ref_run: index of the reference run, whose avgSpike is the target level.
 * For every distinct nConn in ascending order, writes the nConn to
 * group_n_conn[g] and to picked[g] the index of the run with a zero NaN count
 * and a finite avgSpike closest to the reference level (ties: smaller gScale,
 * then the earlier run), or -1 when the nConn has no such run; *n_groups
 * receives the number of distinct nConn.  group_n_conn and picked are host
 * arrays of at least n_runs entries.  SNN_EINVAL if n_runs < 1, a pointer is
 * NULL, ref_run is out of range or has NaNs, or an nConn or gScale is not
 * finite. */
int snn_gscale_select(int64_t n_runs, const double *n_conn, const double *g_scale, const double *avg_spike,
                      const int32_t *n_nans, int64_t ref_run, int64_t *n_groups, double *group_n_conn,
                      int64_t *picked);

/* Least-squares fit of the inverse scaling law gScale = k1 / (k2 + nConn) + k3
 * (Section 5.1, Tables 1 and 2) to n_points points (host double[n_points]
 * each): minimises the unweighted sum of squared gScale residuals over k2 >
 * -min(nConn), so the curve has no pole over the data.  Writes k[0..2] =
 * k1, k2, k3 (host double[3]) and, if mape_percent is not NULL, the mean
 * absolute percentage error of the fitted law over the points.  SNN_EINVAL
 * for fewer than three distinct nConn, a NULL array, a non-finite value or a
 * gScale <= 0; SNN_ERANGE when the best k2 lies at the end of the searched
 * range (the pole on the smallest nConn, or k2 running to infinity because
 * the points lie on a straight line). */
int snn_gscale_fit(int64_t n_points, const double *n_conn, const double *g_scale, double *k,
                   double *mape_percent);

/* Message of the last failure on this thread ("" if none). */
const char *snn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SNN_ABI_H_ */
