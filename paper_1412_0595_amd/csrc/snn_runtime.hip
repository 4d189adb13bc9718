// Host runtime of the spiking-network library: validation, device layout,
// the step loop (direct launches or a captured hipGraph of whole steps),
// state access, the launch-shape autotuner, and the C ABI of include/snn.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/snn.h"
#include "snn_internal.h"

using namespace snn;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

int snn::set_error(int code, const char *msg) { return fail(code, "%s", msg); }

// ------------------------ scratch of snn_backward_noalloc ---------------------
// A fixed device array that snn_backward_noalloc uses in place of the net's
// backward tape, for callers that cannot allocate.  Every GPU the library
// runs on holds its own copy for the life of the process; host code reaches
// it only through the device address hipGetSymbolAddress returns on that GPU
// (the array's name is a host-side stand-in, not a device address).
namespace {

constexpr size_t kScratchBytes = (size_t)SNN_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices];
void *g_scratch_ptr[kMaxDevices];

// Looks up the array's address on device dev, which must be current, once
// per device (snn_create does it for every net's device); nullptr if the
// lookup failed.
void *scratch_on_device(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        g_scratch_ptr[dev] = p;
        g_scratch_done[dev] = true;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

namespace {

// --------------------------- Traub-Miles rest point --------------------------
// Steady-state gate value a / (a + b) and the membrane current with all gates
// at steady state; the resting potential is its root in [-80, -60] mV.
double ratio_xm1(double x) { return x == 0.0 ? 1.0 : x / std::expm1(x); }

double steady_current(const double *p, double v)
{
    const double am = 1.28 * ratio_xm1((-52.0 - v) / 4.0), bm = 1.4 * ratio_xm1((v + 25.0) / 5.0);
    const double ah = 0.128 * std::exp((-48.0 - v) / 18.0), bh = 4.0 / (std::exp((-25.0 - v) / 5.0) + 1.0);
    const double an = 0.16 * ratio_xm1((-50.0 - v) / 5.0), bn = 0.5 * std::exp((-55.0 - v) / 40.0);
    const double m = am / (am + bm), h = ah / (ah + bh), n = an / (an + bn);
    return p[0] * m * m * m * h * (v - p[1]) + p[2] * n * n * n * n * (v - p[3]) + p[4] * (v - p[5]);
}

bool resting_state(const double *p, double out[4])
{
    double lo = -80.0, hi = -60.0;
    if (!(steady_current(p, lo) < 0.0 && steady_current(p, hi) > 0.0)) return false;
    while (true) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (steady_current(p, mid) < 0.0) lo = mid; else hi = mid;
    }
    const double v = 0.5 * (lo + hi);
    const double am = 1.28 * ratio_xm1((-52.0 - v) / 4.0), bm = 1.4 * ratio_xm1((v + 25.0) / 5.0);
    const double ah = 0.128 * std::exp((-48.0 - v) / 18.0), bh = 4.0 / (std::exp((-25.0 - v) / 5.0) + 1.0);
    const double an = 0.16 * ratio_xm1((-50.0 - v) / 5.0), bn = 0.5 * std::exp((-55.0 - v) / 40.0);
    out[0] = v;
    out[1] = am / (am + bm);
    out[2] = ah / (ah + bh);
    out[3] = an / (an + bn);
    return true;
}

uint64_t poisson_threshold(double rate_hz, double dt_ms)
{
    const double p = rate_hz * dt_ms * 1e-3;
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return (uint64_t)1 << 32;
    return (uint64_t)std::floor(p * 4294967296.0);
}

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace

// ------------------------------- the net ------------------------------------
struct HostProj {            // host copy of what state access needs
    int32_t inst, pre_pop, post_pop, n_pre, n_post;
    int64_t nnz, syn_base, G_base;
    std::vector<int32_t> row_ptr;
    std::vector<int32_t> col_ptr;   // plastic only
    int stdp;
    int32_t max_col_len;            // longest column (synapses onto one post neuron)
    double decay;                   // conductance decay per step
};

struct snn_net {
    // configuration
    double dt;
    int substeps;
    int n_inst;
    hipStream_t stream;
    hipStream_t cap_stream;
    snn_alloc_fn alloc_fn;
    snn_free_fn free_fn;
    void *alloc_ctx;
    int device;
    bool sticky;
    int64_t t;                       // steps enqueued so far

    // tables
    std::vector<Seg> segs;
    std::vector<Proj> projs;
    std::vector<HostProj> hprojs;
    std::vector<std::vector<int32_t>> seg_of;   // [inst][pop] -> seg index
    std::vector<std::vector<int32_t>> proj_of;  // [inst][local proj] -> global proj
    std::vector<float> gscale;
    int64_t n_waves, n_neurons_padded;
    int64_t n_hh;                    // Traub-Miles neurons (not padded)
    int64_t n_izh;                   // Izhikevich neurons
    bool plastic;
    int64_t qcap, lcap;
    int raster_steps;

    // device memory
    std::vector<void *> allocs;
    Seg *d_segs;
    Proj *d_projs;
    int32_t *d_wave_seg;
    int32_t *d_rp, *d_cp, *d_col, *d_csc_row, *d_csc_pos, *d_tp;
    int64_t *d_partial;
    uint8_t *d_pflag;
    int4 *d_units;           // tile-mode reduction units
    uint32_t *qb_cnt;        // arena: [3][kQBuckets] counters kQBucketStride apart: reservations of
                             // the two queue slots, the fused update's per-bucket done counts
    int64_t *d_qb_base;      // kQBuckets + 1 bucket offsets into a queue slot (current block size and mode)
    std::vector<int64_t> wave_items_rows, wave_items_tiles;   // worst-case work items of each wave's neurons
    int64_t n_units;
    PullUnit *d_pull_units;  // tile-mode pull units
    int64_t n_pull_units;
    int64_t *d_pull_part;    // [unit][64] their partial sums
    PullSlice *d_pull_slices;
    int64_t n_pull_slices;
    int32_t *d_pull_col;     // [slice][64] post neuron of each lane (-1: padding)
    float4 *d_pull_w;        // sliced-ELL copies of non-plastic projections: weights, [packet][64] x 4
    uint32_t *d_pull_d;      // their one-byte row deltas, [packet][64]
    int32_t *d_pull_r0;      // [unit][64] each lane's row before the unit's first entry
    int32_t *d_pull_perm;    // each copied weight's position in the weight pool (-1: padding or bridge)
    int2 *d_grp_proj;        // grouped mode: (projection, rows per group) of those delivered in groups
    int64_t n_grp;
    int64_t pull_count;      // packets
    uint32_t *pullf;     // arena: [2][n_segs]  populations delivered by pulling
    uint32_t *awcnt;     // arena: [2][n_segs]
    uint32_t *scnt;      // arena: [2][n_segs]
    int32_t *awl;        // arena: [2][n_waves]
    uint32_t *gwsel;     // arena: [2][n_segs]  words per group chosen at emission
    int64_t *D;          // arena: [2][G pool]  fused-mode deliveries for the next update
    float *d_w;
    float *d_gscale;
    float4 *d_izp;       // Izhikevich parameters (a, b, c, d) per neuron
    int64_t w_count;
    // arena of everything a step mutates (one block, so that snapshots are one copy)
    char *d_arena;
    int64_t arena_bytes;
    float *vh, *vl, *mh, *ml, *hh, *hl, *nh, *nl;
    int32_t *counts;
    double *vsum;
    int64_t *G;
    int64_t G_count;
    int32_t *nan_count;
    uint64_t *bits, *raster;
    float *trace;
    int64_t trace_count;
    Item *queue, *lqueue;
    StepState *st;

    // initial state block (8 state arrays), for snn_reset
    float *d_init_state;

    // adjoint recording (snn_forward_record / snn_backward)
    bool recorded;
    bool rec_timeline;     // the recording describes steps [0, rec_T) of the current run
    int32_t rec_pop;
    int64_t rec_T;
    int32_t rec_K;
    int64_t rec_nseg;
    uint64_t *d_rec_raster;
    float *d_ckpt_state;
    int64_t *d_ckpt_G;
    int32_t *d_loss_seg;
    int64_t *d_loss_base;
    int32_t *d_loss_owner;
    int64_t n_loss;
    int32_t n_in_max;
    int32_t loss_block;
    int4 *d_gitems;
    int64_t n_gitems;
    double *d_tape_x, *d_tape_g, *d_lg, *d_lam;
    uint32_t *d_flag;
    uint32_t *d_wmax;        // per projection: bits of the largest weight (weight checks)
    int64_t max_nnz;

    // launch shape and captured step sequences: graphs[k] replays
    // graph_len[k] whole steps (kGraphSteps, and the remainders asked for)
    snn_launch launch;
    std::vector<hipGraphExec_t> graphs;
    std::vector<int> graph_len;
};

namespace {

void *dev_alloc(snn_net *net, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (net->alloc_fn) {
        p = net->alloc_fn(bytes, net->alloc_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p) net->allocs.push_back(p);
    return p;
}

void dev_free(snn_net *net, void *p)
{
    if (!p) return;
    for (size_t i = 0; i < net->allocs.size(); ++i)
        if (net->allocs[i] == p) {
            if (net->free_fn) net->free_fn(p, net->alloc_ctx); else (void)hipFree(p);
            net->allocs.erase(net->allocs.begin() + (long)i);
            return;
        }
}

void drop_graphs(snn_net *net)
{
    for (hipGraphExec_t g : net->graphs) (void)hipGraphExecDestroy(g);
    net->graphs.clear();
    net->graph_len.clear();
}

void release(snn_net *net)
{
    drop_graphs(net);
    for (void *p : net->allocs) {
        if (net->free_fn) net->free_fn(p, net->alloc_ctx); else (void)hipFree(p);
    }
    net->allocs.clear();
    if (net->cap_stream) {
        (void)hipStreamDestroy(net->cap_stream);
        net->cap_stream = nullptr;
    }
}

#define HIP_OK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            net->sticky = true;                                                               \
            return fail(SNN_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));          \
        }                                                                                     \
    } while (0)

int check_net(const snn_net *net)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    if (net->sticky) return fail(SNN_EDEVICE, "a previous device error left the net unusable");
    return SNN_OK;
}

NeuronArgs neuron_args(snn_net *net)
{
    NeuronArgs a{};
    a.segs = net->d_segs;
    a.wave_seg = net->d_wave_seg;
    a.n_waves = net->n_waves;
    a.vh = net->vh; a.vl = net->vl; a.mh = net->mh; a.ml = net->ml;
    a.hh = net->hh; a.hl = net->hl; a.nh = net->nh; a.nl = net->nl;
    a.G = net->G;
    a.counts = net->counts;
    a.vsum = net->vsum;
    a.nan_count = net->nan_count;
    a.bits = net->bits;
    a.raster = net->raster_steps > 0 ? net->raster : nullptr;
    a.raster_steps = net->raster_steps > 0 ? net->raster_steps : 1;
    a.trace = net->trace;
    a.projs = net->d_projs;
    a.rp_pool = net->d_rp;
    a.cp_pool = net->d_cp;
    a.queue = net->queue;
    a.qcap = net->qcap;
    a.qb_cnt = net->qb_cnt;
    a.qb_base = net->d_qb_base;
    a.lqueue = net->lqueue;
    a.lcap = net->lcap;
    a.chunk = net->launch.chunk;
    a.substeps = net->substeps;
    a.hs = net->dt / net->substeps;
    a.st = net->st;
    a.mode = net->launch.mode == kModeGrouped ? kModeRows : net->launch.mode;
    a.awcnt = net->awcnt;
    a.scnt = net->scnt;
    a.awl = net->awl;
    a.gwsel = net->gwsel;
    a.pullf = net->pullf;
    a.D = net->D;
    a.G_count = net->G_count;
    a.col_pool = net->d_col;
    a.w_pool = net->d_w;
    a.gscale = net->d_gscale;
    a.n_segs = (int32_t)net->segs.size();
    a.izp = net->d_izp;
    a.feat = 0;
    for (const Seg &S : net->segs) {
        if (S.kind == kIzh) a.feat |= kFeatIzh;
        if (S.n_tr > 0 || S.n_ltp > 0) a.feat |= kFeatPlastic;
        if (S.record_vbar) a.feat |= kFeatRec;
    }
    return a;
}

PropArgs prop_args(snn_net *net)
{
    PropArgs p{};
    p.mode = net->launch.mode == kModeGrouped ? kModeRows : net->launch.mode;
    p.grp_proj = net->d_grp_proj;
    p.n_grp = net->launch.mode == kModeGrouped ? net->n_grp : 0;
    p.projs = net->d_projs;
    p.segs = net->d_segs;
    p.queue = net->queue;
    p.qcap = net->qcap;
    p.qb_cnt = net->qb_cnt;
    p.qb_base = net->d_qb_base;
    p.rp_pool = net->d_rp;
    p.tp_pool = net->d_tp;
    p.col_pool = net->d_col;
    p.w_pool = net->d_w;
    p.gscale = net->d_gscale;
    p.partial = net->d_partial;
    p.pflag = net->d_pflag;
    p.units = net->d_units;
    p.n_units = net->n_units;
    p.G = net->G;
    p.bits = net->bits;
    p.n_waves = net->n_waves;
    p.trace = net->trace;
    p.st = net->st;
    p.awcnt = net->awcnt;
    p.scnt = net->scnt;
    p.awl = net->awl;
    p.gwsel = net->gwsel;
    p.pullf = net->pullf;
    p.n_inst = net->n_inst;
    p.pull_units = net->d_pull_units;
    p.n_pull_units = net->n_pull_units;
    p.pull_part = net->d_pull_part;
    p.pull_slices = net->d_pull_slices;
    p.n_pull_slices = net->n_pull_slices;
    p.pull_col = net->d_pull_col;
    p.pull_w = net->d_pull_w;
    p.pull_d = net->d_pull_d;
    p.pull_r0 = net->d_pull_r0;
    p.n_segs = (int32_t)net->segs.size();
    return p;
}

LtpArgs ltp_args(snn_net *net)
{
    LtpArgs l{};
    l.projs = net->d_projs;
    l.lqueue = net->lqueue;
    l.lcap = net->lcap;
    l.csc_row = net->d_csc_row;
    l.csc_pos = net->d_csc_pos;
    l.w_pool = net->d_w;
    l.trace = net->trace;
    l.st = net->st;
    return l;
}

// Enqueue one whole step on stream s.
hipError_t enqueue_step(snn_net *net, hipStream_t s)
{
    // fused mode: the neuron update delivers its own spikes
    if (net->launch.mode == kModeFused) return launch_neuron(neuron_args(net), net->launch.neuron_block, s);
    hipError_t e = launch_propagate(prop_args(net), net->launch.prop_blocks, net->launch.prop_block, s);
    if (e != hipSuccess) return e;
    if (net->plastic) {
        e = launch_potentiate(ltp_args(net), net->launch.prop_blocks, net->launch.prop_block, s);
        if (e != hipSuccess) return e;
    }
    return launch_neuron(neuron_args(net), net->launch.neuron_block, s);
}

constexpr int kGraphSteps = 64;
constexpr size_t kMaxGraphs = 8;   // the full-length graph plus a few remainders

// The captured graph of n whole steps (built on first use).  The step
// counters live on the device, so one capture serves every later replay.
int graph_for(snn_net *net, int n, hipGraphExec_t *out)
{
    for (size_t k = 0; k < net->graphs.size(); ++k)
        if (net->graph_len[k] == n) {
            *out = net->graphs[k];
            return SNN_OK;
        }
    if (net->graphs.size() >= kMaxGraphs) {
        // evict the oldest remainder; the full-length graph stays
        for (size_t k = 0; k < net->graphs.size(); ++k)
            if (net->graph_len[k] != kGraphSteps) {
                (void)hipGraphExecDestroy(net->graphs[k]);
                net->graphs.erase(net->graphs.begin() + (long)k);
                net->graph_len.erase(net->graph_len.begin() + (long)k);
                break;
            }
    }
    hipGraph_t g = nullptr;
    HIP_OK(hipStreamBeginCapture(net->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < n && e == hipSuccess; ++k) e = enqueue_step(net, net->cap_stream);
    hipError_t e2 = hipStreamEndCapture(net->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        net->sticky = true;
        return fail(SNN_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        net->sticky = true;
        return fail(SNN_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    net->graphs.push_back(x);
    net->graph_len.push_back(n);
    *out = x;
    return SNN_OK;
}

// Capture, ahead of time, every graph run_steps(n) will replay.
int prepare_graphs(snn_net *net, int64_t n)
{
    hipGraphExec_t g = nullptr;
    int rc = SNN_OK;
    if (n >= kGraphSteps) rc = graph_for(net, kGraphSteps, &g);
    if (!rc && n % kGraphSteps) rc = graph_for(net, (int)(n % kGraphSteps), &g);
    return rc;
}

// n steps as replays of captured graphs: n div 64 of the 64-step graph, then
// one graph of the remaining n mod 64 steps.
int run_steps(snn_net *net, int64_t n)
{
    int rc = prepare_graphs(net, n);
    if (rc) return rc;
    hipGraphExec_t g = nullptr;
    if (n >= kGraphSteps) {
        if ((rc = graph_for(net, kGraphSteps, &g))) return rc;
        for (; n >= kGraphSteps; n -= kGraphSteps) {
            HIP_OK(hipGraphLaunch(g, net->stream));
            net->t += kGraphSteps;
        }
    }
    if (n > 0) {
        if ((rc = graph_for(net, (int)n, &g))) return rc;
        HIP_OK(hipGraphLaunch(g, net->stream));
        net->t += n;
    }
    return SNN_OK;
}

// need_state: the population must have a membrane state (Traub-Miles or
// Izhikevich, not Poisson)
int seg_index(const snn_net *net, int32_t inst, int32_t pop, bool need_state)
{
    if (inst < 0 || inst >= net->n_inst) return fail(SNN_EINVAL, "instance %d out of range", inst);
    if (pop < 0 || pop >= (int32_t)net->seg_of[inst].size()) return fail(SNN_EINVAL, "population %d out of range", pop);
    const int s = net->seg_of[inst][pop];
    if (need_state && net->segs[s].kind == kPoisson) return fail(SNN_EINVAL, "population %d is a Poisson source (no state)", pop);
    return s;
}

int proj_index(const snn_net *net, int32_t inst, int32_t proj)
{
    if (inst < 0 || inst >= net->n_inst) return fail(SNN_EINVAL, "instance %d out of range", inst);
    if (proj < 0 || proj >= (int32_t)net->proj_of[inst].size()) return fail(SNN_EINVAL, "projection %d out of range", proj);
    return net->proj_of[inst][proj];
}

int d2h(snn_net *net, void *dst, const void *src, size_t bytes)
{
    if (bytes == 0) return SNN_OK;
    HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, net->stream));
    HIP_OK(hipStreamSynchronize(net->stream));
    return SNN_OK;
}

int h2d(snn_net *net, void *dst, const void *src, size_t bytes)
{
    if (bytes == 0) return SNN_OK;
    HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, net->stream));
    HIP_OK(hipStreamSynchronize(net->stream));
    return SNN_OK;
}

// ------------------------------- validation ---------------------------------
int validate(const snn_config *cfg)
{
    if (!cfg) return fail(SNN_EINVAL, "config is NULL");
    if (!(cfg->dt_ms > 0.0) || !std::isfinite(cfg->dt_ms)) return fail(SNN_EINVAL, "dt_ms must be finite and > 0");
    if (cfg->substeps < 1 || cfg->substeps > 64) return fail(SNN_EINVAL, "substeps must be in [1, 64]");
    if (cfg->n_instances < 1 || !cfg->inst) return fail(SNN_EINVAL, "need at least one instance");
    if (cfg->raster_steps < 0) return fail(SNN_EINVAL, "raster_steps must be >= 0");
    if ((cfg->alloc == nullptr) != (cfg->free == nullptr)) return fail(SNN_EINVAL, "alloc and free must both be set or both be NULL");
    for (int b = 0; b < cfg->n_instances; ++b) {
        const snn_instance_desc &I = cfg->inst[b];
        if (I.n_pops < 1 || I.n_pops > 64 || !I.pops) return fail(SNN_EINVAL, "instance %d: n_pops must be in [1, 64]", b);
        if (I.n_projs < 0 || I.n_projs > 256 || (I.n_projs > 0 && !I.projs))
            return fail(SNN_EINVAL, "instance %d: n_projs must be in [0, 256]", b);
        if (!(I.g_scale >= 0.0f) || !std::isfinite(I.g_scale)) return fail(SNN_EINVAL, "instance %d: g_scale must be finite and >= 0", b);
        std::vector<int> n_in(I.n_pops, 0), n_out(I.n_pops, 0), n_tr(I.n_pops, 0), n_ltp(I.n_pops, 0);
        for (int p = 0; p < I.n_pops; ++p) {
            const snn_pop_desc &P = I.pops[p];
            if (P.kind != SNN_POISSON && P.kind != SNN_TRAUB_MILES && P.kind != SNN_IZHIKEVICH)
                return fail(SNN_EINVAL, "instance %d pop %d: bad kind %d", b, p, P.kind);
            if (P.n < 0) return fail(SNN_EINVAL, "instance %d pop %d: n < 0", b, p);
            if (P.kind == SNN_POISSON && (!(P.rate_hz >= 0.0) || !std::isfinite(P.rate_hz)))
                return fail(SNN_EINVAL, "instance %d pop %d: rate must be finite and >= 0", b, p);
            if (P.kind == SNN_TRAUB_MILES) {
                for (int k = 0; k < SNN_HH_NPARAM; ++k)
                    if (!std::isfinite(P.hh[k])) return fail(SNN_EINVAL, "instance %d pop %d: parameter %d not finite", b, p, k);
                if (!(P.hh[6] > 0.0)) return fail(SNN_EINVAL, "instance %d pop %d: C_m must be > 0", b, p);
                if (!std::isfinite(P.i_ext_nA)) return fail(SNN_EINVAL, "instance %d pop %d: i_ext not finite", b, p);
                double r[4];
                if (!resting_state(P.hh, r)) return fail(SNN_EINVAL, "instance %d pop %d: no resting point in [-80, -60] mV", b, p);
            }
            if (P.kind == SNN_IZHIKEVICH) {
                if (!std::isfinite(P.i_ext_nA)) return fail(SNN_EINVAL, "instance %d pop %d: i_ext not finite", b, p);
                if (P.n > 0 && !P.izh_abcd) return fail(SNN_EINVAL, "instance %d pop %d: izh_abcd is NULL", b, p);
                for (int64_t k = 0; k < 4 * (int64_t)P.n; ++k)
                    if (!std::isfinite(P.izh_abcd[k]))
                        return fail(SNN_EINVAL, "instance %d pop %d: Izhikevich parameter %lld not finite", b, p, (long long)k);
            }
        }
        for (int q = 0; q < I.n_projs; ++q) {
            const snn_proj_desc &Q = I.projs[q];
            if (Q.pre_pop < 0 || Q.pre_pop >= I.n_pops || Q.post_pop < 0 || Q.post_pop >= I.n_pops)
                return fail(SNN_EINVAL, "instance %d proj %d: population index out of range", b, q);
            if (I.pops[Q.post_pop].kind == SNN_POISSON)
                return fail(SNN_EINVAL, "instance %d proj %d: post population must be Traub-Miles or Izhikevich", b, q);
            if (!(Q.tau_ms > 0.0f) || !std::isfinite(Q.tau_ms) || !std::isfinite(Q.e_rev_mV))
                return fail(SNN_EINVAL, "instance %d proj %d: tau must be > 0 and e_rev finite", b, q);
            const int32_t npre = I.pops[Q.pre_pop].n, npost = I.pops[Q.post_pop].n;
            if (Q.nnz < 0 || Q.nnz >= ((int64_t)1 << 31)) return fail(SNN_EINVAL, "instance %d proj %d: nnz out of range", b, q);
            if (!Q.row_ptr || (Q.nnz > 0 && (!Q.col_idx || !Q.g))) return fail(SNN_EINVAL, "instance %d proj %d: NULL CSR array", b, q);
            if (Q.row_ptr[0] != 0) return fail(SNN_EINVAL, "instance %d proj %d: row_ptr[0] != 0", b, q);
            if (Q.row_ptr[npre] != Q.nnz) return fail(SNN_EINVAL, "instance %d proj %d: row_ptr[n_pre] != nnz", b, q);
            for (int32_t i = 0; i < npre; ++i) {
                const int32_t a0 = Q.row_ptr[i], a1 = Q.row_ptr[i + 1];
                if (a1 < a0) return fail(SNN_EINVAL, "instance %d proj %d: row_ptr decreases at row %d", b, q, i);
                for (int32_t k = a0; k < a1; ++k) {
                    const int32_t c = Q.col_idx[k];
                    if (c < 0 || c >= npost) return fail(SNN_EINVAL, "instance %d proj %d: col_idx[%d] = %d out of range", b, q, k, c);
                    if (k > a0 && c <= Q.col_idx[k - 1])
                        return fail(SNN_EINVAL, "instance %d proj %d: row %d not strictly ascending (sorted, no duplicate synapse)", b, q, i);
                    if (!(Q.g[k] >= 0.0f) || !std::isfinite(Q.g[k])) return fail(SNN_EINVAL, "instance %d proj %d: g[%d] not finite and >= 0", b, q, k);
                }
            }
            n_in[Q.post_pop]++;
            n_out[Q.pre_pop]++;
            if (Q.stdp) {
                if (!std::isfinite(Q.a_plus) || !std::isfinite(Q.a_minus) || !(Q.tau_stdp_ms > 0.0f) ||
                    !std::isfinite(Q.tau_stdp_ms) || !(Q.g_max >= 0.0f) || !std::isfinite(Q.g_max))
                    return fail(SNN_EINVAL, "instance %d proj %d: bad STDP parameters", b, q);
                n_tr[Q.pre_pop]++;
                n_tr[Q.post_pop]++;
                n_ltp[Q.post_pop]++;
            }
        }
        for (int p = 0; p < I.n_pops; ++p) {
            if (n_in[p] > kMaxIn) return fail(SNN_EINVAL, "instance %d pop %d: more than %d incoming projections", b, p, kMaxIn);
            if (n_out[p] > kMaxOut) return fail(SNN_EINVAL, "instance %d pop %d: more than %d outgoing projections", b, p, kMaxOut);
            if (n_tr[p] > kMaxTr) return fail(SNN_EINVAL, "instance %d pop %d: more than %d STDP traces", b, p, kMaxTr);
            if (n_ltp[p] > kMaxLtp) return fail(SNN_EINVAL, "instance %d pop %d: more than %d plastic inputs", b, p, kMaxLtp);
        }
    }
    return SNN_OK;
}

// Largest conductance a post neuron can reach is below (sum of its column) *
// g_scale / (1 - decay); keep it well inside the 2^63 * 2^-40 uS range.
constexpr double kGLimit = 4194304.0;   // 2^22 uS
// A single delivered increment g_scale * g must stay below 2^11 uS, so that
// its fixed-point value is below 2^51, where the propagation kernels round it
// to an integer with one floating-point addition.
constexpr double kWLimit = 2048.0;      // 2^11 uS

int check_range(const snn_net *net, const std::vector<double> &colmax_sum, const std::vector<double> &wmax,
                const float *gs)
{
    for (size_t q = 0; q < net->projs.size(); ++q) {
        const double s = gs[net->projs[q].inst];
        if (!(colmax_sum[q] * s < kGLimit))
            return fail(SNN_ERANGE, "projection %zu: g_scale * column sum / (1 - decay) exceeds %g uS", q, kGLimit);
        if (!(wmax[q] * s < kWLimit))
            return fail(SNN_ERANGE, "projection %zu: g_scale * largest weight exceeds %g uS", q, kWLimit);
    }
    return SNN_OK;
}

}  // namespace

// Run `body` between a hipEvent pair on a snapshot of everything a step
// mutates, then restore the snapshot; *ms gets the elapsed milliseconds.
template <class F>
static int timed_on_snapshot(snn_net *net, F body, double *ms_out)
{
    void *snap = nullptr, *wsnap = nullptr;
    HIP_OK(hipMalloc(&snap, (size_t)net->arena_bytes));
    if (net->plastic && hipMalloc(&wsnap, 4 * (size_t)std::max<int64_t>(net->w_count, 1)) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(snap);
        return fail(SNN_ENOMEM, "snapshot allocation failed");
    }
    const int64_t t_saved = net->t;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SNN_OK;
    hipError_t e = hipMemcpyAsync(snap, net->d_arena, (size_t)net->arena_bytes, hipMemcpyDeviceToDevice, net->stream);
    if (e == hipSuccess && wsnap) e = hipMemcpyAsync(wsnap, net->d_w, 4 * (size_t)net->w_count, hipMemcpyDeviceToDevice, net->stream);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, net->stream);
    if (e == hipSuccess) rc = body();
    if (e == hipSuccess && rc == SNN_OK) e = hipEventRecord(e1, net->stream);
    if (e == hipSuccess && rc == SNN_OK) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess && rc == SNN_OK) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && rc == SNN_OK) e = hipMemcpyAsync(net->d_arena, snap, (size_t)net->arena_bytes, hipMemcpyDeviceToDevice, net->stream);
    if (e == hipSuccess && rc == SNN_OK && wsnap) e = hipMemcpyAsync(net->d_w, wsnap, 4 * (size_t)net->w_count, hipMemcpyDeviceToDevice, net->stream);
    if (e == hipSuccess && rc == SNN_OK) e = hipStreamSynchronize(net->stream);
    net->t = t_saved;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(snap);
    if (wsnap) (void)hipFree(wsnap);
    if (rc) return rc;
    if (e != hipSuccess) {
        net->sticky = true;
        return fail(SNN_EDEVICE, "timing failed: %s", hipGetErrorString(e));
    }
    *ms_out = (double)ms;
    return SNN_OK;
}

// ============================== C ABI ========================================
extern "C" {

void snn_default_hh(double *p)
{
    p[0] = 7.15;
    p[1] = 50.0;
    p[2] = 1.43;
    p[3] = -95.0;
    p[4] = 0.02672;
    p[5] = -63.563;
    p[6] = 0.143;
}

const char *snn_last_error(void) { return g_err.c_str(); }

static int update_qbuckets(snn_net *net);

int snn_create(const snn_config *cfg, snn_net **out)
{
    if (!out) return fail(SNN_EINVAL, "out is NULL");
    *out = nullptr;
    g_err.clear();
    int rc = validate(cfg);
    if (rc) return rc;

    snn_net *net = new snn_net();
    net->dt = cfg->dt_ms;
    net->substeps = cfg->substeps;
    net->n_inst = cfg->n_instances;
    net->stream = (hipStream_t)cfg->stream;
    net->alloc_fn = cfg->alloc;
    net->free_fn = cfg->free;
    net->alloc_ctx = cfg->alloc_ctx;
    net->raster_steps = cfg->raster_steps;
    net->launch = snn_launch{256, 1024, 256, 256, kModeRows};
    auto bail = [&](int code) {
        release(net);
        delete net;
        return code;
    };

    // ---- layout: segments, projections, pools
    int64_t base = 0, rp_total = 0, syn_total = 0, G_total = 0, tr_total = 0, cp_total = 0, csc_total = 0;
    int64_t P_total = 0, tp_total = 0, F_total = 0;
    net->seg_of.resize(net->n_inst);
    net->proj_of.resize(net->n_inst);
    net->gscale.resize(net->n_inst);
    net->n_hh = 0;
    net->n_izh = 0;
    net->plastic = false;
    int64_t izp_total = 0;
    std::vector<double> colsum_bound, w_bound;
    for (int b = 0; b < net->n_inst; ++b) {
        const snn_instance_desc &I = cfg->inst[b];
        net->gscale[b] = I.g_scale;
        for (int p = 0; p < I.n_pops; ++p) {
            const snn_pop_desc &P = I.pops[p];
            Seg S{};
            S.kind = P.kind == SNN_POISSON ? kPoisson : P.kind == SNN_IZHIKEVICH ? kIzh : kHH;
            S.n = P.n;
            S.base = base;
            S.inst = b;
            S.pop = p;
            S.thresh = poisson_threshold(P.rate_hz, net->dt);
            S.seed = I.seed;
            S.gna = P.hh[0]; S.ena = P.hh[1]; S.gk = P.hh[2]; S.ek = P.hh[3]; S.gl = P.hh[4]; S.el = P.hh[5];
            S.inv_c = 1.0 / P.hh[6];
            S.i_ext = P.i_ext_nA;
            S.record_vbar = P.record_vbar ? 1 : 0;
            net->seg_of[b].push_back((int32_t)net->segs.size());
            net->segs.push_back(S);
            base += align_up(P.n, kWave);
            // the neuron update addresses 8-byte per-neuron arrays by 32-bit
            // byte offsets
            if (base > kMaxNeuronsPadded)
                return bail(fail(SNN_ERANGE, "more than %lld neurons (padded to 64 per population)",
                                 (long long)kMaxNeuronsPadded));
            if (S.kind == kHH) net->n_hh += P.n;
            if (S.kind == kIzh) {
                net->segs.back().izp_base = izp_total;
                izp_total += P.n;
                net->n_izh += P.n;
            }
        }
        for (int q = 0; q < I.n_projs; ++q) {
            const snn_proj_desc &Q = I.projs[q];
            const int gi = (int)net->projs.size();
            Seg &pre = net->segs[net->seg_of[b][Q.pre_pop]];
            Seg &post = net->segs[net->seg_of[b][Q.post_pop]];
            Proj P{};
            P.pre_seg = net->seg_of[b][Q.pre_pop];
            P.post_seg = net->seg_of[b][Q.post_pop];
            P.n_pre = pre.n;
            P.n_post = post.n;
            P.inst = b;
            P.stdp = Q.stdp ? 1 : 0;
            P.rp_base = rp_total;
            rp_total += pre.n + 1;
            P.syn_base = syn_total;
            P.nnz = Q.nnz;
            syn_total += Q.nnz;
            P.G_base = G_total;
            G_total += post.n;
            P.tile_w = (int32_t)std::min<int64_t>(kTileMax, std::max<int64_t>(kWave, align_up(post.n, kWave)));
            P.n_tiles = (int32_t)((post.n + P.tile_w - 1) / P.tile_w);
            P.pre_words = (int32_t)(align_up(pre.n, kWave) / kWave);
            P.P_base = P_total;
            P_total += (int64_t)P.n_tiles * P.pre_words * P.tile_w;
            P.F_base = F_total;
            F_total += (int64_t)P.n_tiles * P.pre_words;
            P.pull_base = -1;
            P.tp_base = -1;
            if (P.n_tiles > 1) {
                P.tp_base = tp_total;
                tp_total += (int64_t)pre.n * (P.n_tiles + 1);
            }
            const double decay = std::exp(-net->dt / (double)Q.tau_ms);
            post.in_proj[post.n_in] = gi;
            post.in_G[post.n_in] = P.G_base;
            post.in_erev[post.n_in] = Q.e_rev_mV;
            post.in_decay[post.n_in] = decay;
            post.n_in++;
            pre.out_proj[pre.n_out] = gi;
            pre.out_rp[pre.n_out] = P.rp_base;
            pre.out_tiles[pre.n_out] = P.n_tiles;
            pre.n_out++;
            HostProj H{};
            H.inst = b; H.pre_pop = Q.pre_pop; H.post_pop = Q.post_pop; H.n_pre = pre.n; H.n_post = post.n;
            H.nnz = Q.nnz; H.syn_base = P.syn_base; H.G_base = P.G_base; H.stdp = P.stdp;
            H.row_ptr.assign(Q.row_ptr, Q.row_ptr + pre.n + 1);
            if (Q.stdp) {
                net->plastic = true;
                P.a_plus_gmax = Q.a_plus * Q.g_max;
                P.a_minus_gmax = Q.a_minus * Q.g_max;
                P.g_max = Q.g_max;
                const float td = (float)std::exp(-net->dt / (double)Q.tau_stdp_ms);
                P.x_base = tr_total;
                pre.tr_base[pre.n_tr] = tr_total;
                pre.tr_decay[pre.n_tr] = td;
                pre.n_tr++;
                tr_total += pre.n;
                P.y_base = tr_total;
                post.tr_base[post.n_tr] = tr_total;
                post.tr_decay[post.n_tr] = td;
                post.n_tr++;
                tr_total += post.n;
                P.cp_base = cp_total;
                cp_total += post.n + 1;
                P.csc_base = csc_total;
                csc_total += Q.nnz;
                post.ltp_proj[post.n_ltp] = gi;
                post.ltp_cp[post.n_ltp] = P.cp_base;
                post.n_ltp++;
            }
            // bound on the conductance reachable with g_scale = 1
            std::vector<double> col(post.n > 0 ? post.n : 1, 0.0);
            std::vector<int32_t> len(post.n > 0 ? post.n : 1, 0);
            for (int64_t k = 0; k < Q.nnz; ++k) {
                col[Q.col_idx[k]] += Q.g[k];
                len[Q.col_idx[k]]++;
            }
            H.max_col_len = *std::max_element(len.begin(), len.end());
            H.decay = decay;
            double mx = 0.0;
            for (double c : col) mx = std::max(mx, c);
            if (Q.stdp) mx = std::max(mx, (double)Q.g_max * (double)pre.n);
            colsum_bound.push_back(mx / (1.0 - decay));
            double wm = Q.stdp ? (double)Q.g_max : 0.0;
            for (int64_t k = 0; k < Q.nnz; ++k) wm = std::max(wm, (double)Q.g[k]);
            w_bound.push_back(wm);
            net->proj_of[b].push_back(gi);
            net->projs.push_back(P);
            net->hprojs.push_back(std::move(H));
        }
    }
    if ((rc = check_range(net, colsum_bound, w_bound, net->gscale.data()))) return bail(rc);
    // sliced-ELL copies of the non-plastic projections (weight-pool positions
    // must fit the int32 permutation), with one-byte row deltas: each column's
    // encoded length is its entry count plus the weight-0 entries that bridge
    // gaps of more than kPullMaxDelta rows; columns by decreasing encoded
    // length, 64 to a slice, a slice's depth rounded up to whole packets of 4
    // and split evenly into pull units of at most `unit_depth` entries: the
    // largest of kPullDepth, 2 kPullDepth and 4 kPullDepth that still cuts
    // all copies together into kPullUnitsMin units (a deeper unit reads more
    // per record and leaves fewer slices to partial sums, but there must be
    // enough units to fill the chip)
    std::vector<std::vector<int32_t>> pcol(net->projs.size()), pord(net->projs.size()), plen(net->projs.size());
    std::vector<int64_t> pull_slices;   // first packet of each slice
    std::vector<int32_t> slice_u0;      // first pull unit of each slice
    std::vector<PullSlice> pull_red;
    std::vector<PullUnit> pull_units;
    int64_t pull_total = 0;             // packets
    if (syn_total < ((int64_t)1 << 31)) {
        for (int b = 0, gq = 0; b < net->n_inst; ++b) {
            const snn_instance_desc &I = cfg->inst[b];
            for (int q = 0; q < I.n_projs; ++q, ++gq) {
                const snn_proj_desc &Q = I.projs[q];
                Proj &P = net->projs[gq];
                if (Q.stdp || Q.nnz == 0) continue;
                std::vector<int32_t> &cp = pcol[gq], &ord = pord[gq], &len = plen[gq];
                cp.assign(P.n_post + 1, 0);
                len.assign(P.n_post, 0);
                std::vector<int32_t> last(P.n_post, -1);
                int64_t bridges = 0;
                for (int32_t i = 0; i < P.n_pre; ++i)
                    for (int32_t k = Q.row_ptr[i]; k < Q.row_ptr[i + 1]; ++k) {
                        const int32_t c = Q.col_idx[k];
                        cp[c + 1]++;
                        if (last[c] >= 0) {
                            const int32_t nb = (i - last[c] - 1) / kPullMaxDelta;
                            len[c] += nb;
                            bridges += nb;
                        }
                        last[c] = i;
                    }
                if (bridges * 4 > Q.nnz) {   // too sparse for one-byte deltas: always pushed
                    cp.clear();
                    len.clear();
                    continue;
                }
                for (int32_t j = 0; j < P.n_post; ++j) {
                    len[j] += cp[j + 1];
                    cp[j + 1] += cp[j];
                }
                ord.resize(P.n_post);
                for (int32_t j = 0; j < P.n_post; ++j) ord[j] = j;
                std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return len[x] > len[y]; });
            }
        }
    }
    int64_t pull_entries = 0;
    for (size_t gq = 0; gq < plen.size(); ++gq)
        for (int32_t j0 = 0; j0 < (int32_t)plen[gq].size(); j0 += kWave)
            pull_entries += (int64_t)kWave * 4 * ((plen[gq][pord[gq][j0]] + 3) / 4);
    int32_t unit_depth = kPullDepth;
    while (unit_depth < 4 * kPullDepth && pull_entries / ((int64_t)kWave * 2 * unit_depth) >= kPullUnitsMin) unit_depth *= 2;
    if (syn_total < ((int64_t)1 << 31)) {
        for (int b = 0, gq = 0; b < net->n_inst; ++b) {
            const snn_instance_desc &I = cfg->inst[b];
            for (int q = 0; q < I.n_projs; ++q, ++gq) {
                Proj &P = net->projs[gq];
                if (plen[gq].empty()) continue;
                const std::vector<int32_t> &ord = pord[gq], &len = plen[gq];
                P.pull_base = (int64_t)pull_slices.size();
                const Seg &pre = net->segs[P.pre_seg];
                for (int32_t j0 = 0; j0 < P.n_post; j0 += kWave) {
                    const int32_t npk = (len[ord[j0]] + 3) / 4;   // packets of the slice
                    const int64_t sl = (int64_t)pull_slices.size();
                    pull_slices.push_back(pull_total);
                    slice_u0.push_back((int32_t)pull_units.size());
                    // depth split into equal chunks of at most unit_depth;
                    // reduction groups of up to 64 chunks
                    const int32_t nch = (4 * npk + unit_depth - 1) / unit_depth;
                    for (int32_t c0 = 0; nch > 1 && c0 < nch; c0 += kWave)
                        pull_red.push_back(PullSlice{P.G_base, (int32_t)pull_units.size() + c0, std::min(kWave, nch - c0),
                                                     (int32_t)(sl * kWave), P.pre_seg, nch > kWave ? 1 : 0, 0});
                    for (int32_t c = 0; c < nch; ++c) {
                        const int32_t p0 = (int32_t)((int64_t)c * npk / nch), p1 = (int32_t)((int64_t)(c + 1) * npk / nch);
                        PullUnit U{};
                        U.pk0 = pull_total + p0;
                        U.g_base = P.G_base;
                        U.col_off = (int32_t)(sl * kWave);
                        U.npk = p1 - p0;
                        U.pre_seg = P.pre_seg;
                        U.inst = P.inst;
                        U.wbase = (int32_t)(pre.base / kWave);
                        U.nwords = (int32_t)(align_up(pre.n, kWave) / kWave);
                        U.direct = nch == 1 ? 1 : 0;
                        U.ncols = std::min(kWave, P.n_post - j0);
                        pull_units.push_back(U);
                    }
                    pull_total += npk;
                }
                net->segs[P.pre_seg].pullable = 1;
            }
        }
    }
    net->n_neurons_padded = base;
    net->n_waves = base / kWave;
    net->w_count = syn_total;
    net->G_count = G_total;
    net->trace_count = tr_total;

    // work-queue capacity: every spike word active at once (one item per
    // projection, post tile and pre word); potentiation with the smallest chunk
    int64_t qcap_tiles = 0, qcap_rows = 0, lcap = 0;
    for (const Proj &P : net->projs) qcap_tiles += (int64_t)P.n_tiles * P.pre_words;
    for (const HostProj &H : net->hprojs)
        for (int32_t i = 0; i < H.n_pre; ++i) qcap_rows += (H.row_ptr[i + 1] - H.row_ptr[i] + kMinChunk - 1) / kMinChunk;
    const int64_t qcap = std::max(qcap_tiles, qcap_rows);
    // the same worst cases per wave of pre neurons, for the reservation buckets
    net->wave_items_rows.assign(net->n_waves, 0);
    net->wave_items_tiles.assign(net->n_waves, 0);
    for (size_t q = 0; q < net->projs.size(); ++q) {
        const Proj &P = net->projs[q];
        const HostProj &H = net->hprojs[q];
        const Seg &pre = net->segs[P.pre_seg];
        for (int32_t i = 0; i < H.n_pre; ++i)
            net->wave_items_rows[(pre.base + i) / kWave] += (H.row_ptr[i + 1] - H.row_ptr[i] + kMinChunk - 1) / kMinChunk;
        for (int64_t w = pre.base / kWave; w < (pre.base + align_up(pre.n, kWave)) / kWave; ++w)
            net->wave_items_tiles[w] += P.n_tiles;
    }
    // column lengths of plastic projections
    std::vector<std::vector<int32_t>> colptrs(net->projs.size());
    for (int b = 0, gq = 0; b < net->n_inst; ++b) {
        const snn_instance_desc &I = cfg->inst[b];
        for (int q = 0; q < I.n_projs; ++q, ++gq) {
            if (!I.projs[q].stdp) continue;
            HostProj &H = net->hprojs[gq];
            H.col_ptr.assign(H.n_post + 1, 0);
            for (int64_t k = 0; k < I.projs[q].nnz; ++k) H.col_ptr[I.projs[q].col_idx[k] + 1]++;
            for (int32_t j = 0; j < H.n_post; ++j) H.col_ptr[j + 1] += H.col_ptr[j];
            for (int32_t j = 0; j < H.n_post; ++j)
                lcap += (H.col_ptr[j + 1] - H.col_ptr[j] + kMinChunk - 1) / kMinChunk;
        }
    }
    net->qcap = std::max<int64_t>(qcap, 1);
    net->lcap = std::max<int64_t>(lcap, 1);
    if (net->qcap >= ((int64_t)1 << 32) || net->lcap >= ((int64_t)1 << 32))
        return bail(fail(SNN_ERANGE, "work queue would exceed 2^32 items"));

    // ---- device allocation (everything above is host-only checking)
    if (hipGetDevice(&net->device) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(SNN_EDEVICE, "no HIP device"));
    }
    // set-up of snn_backward_noalloc on this device (its failure only
    // disables that entry point, which then reports it)
    (void)scratch_on_device(net->device);
    if (hipStreamCreateWithFlags(&net->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        net->cap_stream = nullptr;
        return bail(fail(SNN_EDEVICE, "hipStreamCreate failed"));
    }
    const int64_t N = net->n_neurons_padded;
    const int64_t W = net->n_waves;
    bool any_vbar = false;
    for (const Seg &S : net->segs) any_vbar |= S.record_vbar != 0;
    struct Part { int64_t off, bytes; };
    int64_t off = 0;
    auto part = [&](int64_t bytes) { Part p{off, bytes}; off = align_up(off + std::max<int64_t>(bytes, 1), 256); return p; };
    Part p_state[8];
    for (auto &p : p_state) p = part(N * 4);
    Part p_counts = part(N * 4);
    Part p_vsum = part(any_vbar ? N * 8 : 8);
    Part p_G = part(G_total * 8);
    Part p_nan = part(net->n_inst * 4);
    Part p_bits = part(2 * W * 8);
    Part p_raster = part(net->raster_steps > 0 ? (int64_t)net->raster_steps * W * 8 : 8);
    Part p_trace = part(tr_total * 4);
    Part p_queue = part(2 * net->qcap * (int64_t)sizeof(Item));
    Part p_lqueue = part(2 * net->lcap * (int64_t)sizeof(Item));
    Part p_st = part(sizeof(StepState));
    Part p_qb = part(4 * 3 * (int64_t)kQBuckets * kQBucketStride);   // two queue slots, fused done counts
    Part p_awcnt = part(2 * (int64_t)net->segs.size() * 4);
    Part p_scnt = part(2 * (int64_t)net->segs.size() * 4);
    Part p_awl = part(2 * W * 4);
    Part p_gws = part(2 * (int64_t)net->segs.size() * 4);
    Part p_pullf = part(2 * (int64_t)net->segs.size() * 4);
    Part p_D = part(net->plastic ? 8 : 2 * std::max<int64_t>(G_total, 1) * 8);   // fused mode only
    net->arena_bytes = off;
    net->d_arena = (char *)dev_alloc(net, (size_t)off);
    net->d_segs = (Seg *)dev_alloc(net, sizeof(Seg) * net->segs.size());
    net->d_projs = (Proj *)dev_alloc(net, sizeof(Proj) * std::max<size_t>(net->projs.size(), 1));
    net->d_wave_seg = (int32_t *)dev_alloc(net, 4 * std::max<int64_t>(W, 1));
    // at least two entries: the neuron update reads rp[0..1] as a harmless
    // stand-in when a population has no outgoing projection
    net->d_rp = (int32_t *)dev_alloc(net, 4 * std::max<int64_t>(rp_total, 2));
    net->d_col = (int32_t *)dev_alloc(net, 4 * std::max<int64_t>(syn_total, 1));
    net->d_w = (float *)dev_alloc(net, 4 * std::max<int64_t>(syn_total, 1));
    net->d_cp = (int32_t *)dev_alloc(net, 4 * std::max<int64_t>(cp_total, 1));
    net->d_csc_row = (int32_t *)dev_alloc(net, 4 * std::max<int64_t>(csc_total, 1));
    net->d_csc_pos = (int32_t *)dev_alloc(net, 4 * std::max<int64_t>(csc_total, 1));
    net->d_gscale = (float *)dev_alloc(net, 4 * net->n_inst);
    net->d_tp = (int32_t *)dev_alloc(net, 4 * std::max<int64_t>(tp_total, 1));
    net->d_partial = (int64_t *)dev_alloc(net, 8 * std::max<int64_t>(P_total, 1));
    net->d_pflag = (uint8_t *)dev_alloc(net, std::max<int64_t>(F_total, 1));
    // reduction units of the tile mode: (projection, post tile, first of 64
    // columns, first of 64 groups) over every tile's columns and groups
    std::vector<int4> units;
    for (size_t q = 0; q < net->projs.size(); ++q) {
        const Proj &P = net->projs[q];
        for (int32_t tl = 0; tl < P.n_tiles; ++tl) {
            const int32_t cols = std::min<int32_t>(P.tile_w, P.n_post - tl * P.tile_w);
            for (int32_t c = 0; c < cols; c += kWave)
                for (int32_t g = 0; g < P.pre_words; g += kWave) units.push_back(make_int4((int)q, tl, c, g));
        }
    }
    net->n_units = (int64_t)units.size();
    net->d_units = (int4 *)dev_alloc(net, sizeof(int4) * std::max<size_t>(units.size(), 1));
    // grouped mode: every non-plastic projection onto at most kGrpTile neurons,
    // at most kGrpDense of all (pre, post) pairs connected, whose mean row
    // length allows two rows or more per group
    std::vector<int2> grp;
    for (size_t q = 0; q < net->projs.size(); ++q) {
        Proj &P = net->projs[q];
        P.grp = 0;
        if (P.stdp || P.n_post <= 0 || P.n_post > kGrpTile || P.nnz <= 0 || P.pre_words <= 0 || P.n_pre <= 0)
            continue;
        if ((double)P.nnz > kGrpDense * (double)P.n_pre * (double)P.n_post) continue;
        const int64_t k = std::min<int64_t>(kGrpRows, (int64_t)kGrpSyn * P.n_pre / P.nnz);
        if (k < 2) continue;
        P.grp = 1;
        grp.push_back(make_int2((int)q, (int)k));
    }
    net->n_grp = (int64_t)grp.size();
    net->d_grp_proj = (int2 *)dev_alloc(net, sizeof(int2) * std::max<size_t>(grp.size(), 1));
    net->d_qb_base = (int64_t *)dev_alloc(net, 8 * (size_t)(kQBuckets + 1));
    net->pull_count = pull_total;
    net->n_pull_units = (int64_t)pull_units.size();
    net->d_pull_units = (PullUnit *)dev_alloc(net, sizeof(PullUnit) * std::max<size_t>(pull_units.size(), 1));
    net->d_pull_part = (int64_t *)dev_alloc(net, 8 * (size_t)kWave * std::max<size_t>(pull_units.size(), 1));
    net->n_pull_slices = (int64_t)pull_red.size();
    net->d_pull_slices = (PullSlice *)dev_alloc(net, sizeof(PullSlice) * std::max<size_t>(pull_red.size(), 1));
    net->d_pull_col = (int32_t *)dev_alloc(net, 4 * (size_t)kWave * std::max<size_t>(pull_slices.size(), 1));
    net->d_pull_w = (float4 *)dev_alloc(net, 16 * (size_t)kWave * std::max<int64_t>(pull_total, 1));
    net->d_pull_d = (uint32_t *)dev_alloc(net, 4 * (size_t)kWave * std::max<int64_t>(pull_total, 1));
    net->d_pull_r0 = (int32_t *)dev_alloc(net, 4 * (size_t)kWave * std::max<size_t>(pull_units.size(), 1));
    net->d_pull_perm = (int32_t *)dev_alloc(net, 16 * (size_t)kWave * std::max<int64_t>(pull_total, 1));
    net->d_izp = (float4 *)dev_alloc(net, sizeof(float4) * (size_t)std::max<int64_t>(izp_total, 1));
    if (!net->d_izp) return bail(fail(SNN_ENOMEM, "device allocation failed"));
    if (!net->d_arena || !net->d_segs || !net->d_projs || !net->d_wave_seg || !net->d_rp || !net->d_col || !net->d_w ||
        !net->d_cp || !net->d_csc_row || !net->d_csc_pos || !net->d_gscale || !net->d_tp || !net->d_partial || !net->d_pflag ||
        !net->d_units || !net->d_pull_units || !net->d_pull_part || !net->d_pull_slices || !net->d_pull_col || !net->d_pull_w ||
        !net->d_pull_d || !net->d_pull_r0 || !net->d_pull_perm || !net->d_qb_base || !net->d_grp_proj)
        return bail(fail(SNN_ENOMEM, "device allocation failed"));
    char *A = net->d_arena;
    float **st_ptrs[8] = {&net->vh, &net->vl, &net->mh, &net->ml, &net->hh, &net->hl, &net->nh, &net->nl};
    for (int k = 0; k < 8; ++k) *st_ptrs[k] = (float *)(A + p_state[k].off);
    net->counts = (int32_t *)(A + p_counts.off);
    net->vsum = (double *)(A + p_vsum.off);
    net->G = (int64_t *)(A + p_G.off);
    net->nan_count = (int32_t *)(A + p_nan.off);
    net->bits = (uint64_t *)(A + p_bits.off);
    net->raster = (uint64_t *)(A + p_raster.off);
    net->trace = (float *)(A + p_trace.off);
    net->queue = (Item *)(A + p_queue.off);
    net->lqueue = (Item *)(A + p_lqueue.off);
    net->st = (StepState *)(A + p_st.off);
    net->qb_cnt = (uint32_t *)(A + p_qb.off);
    net->awcnt = (uint32_t *)(A + p_awcnt.off);
    net->scnt = (uint32_t *)(A + p_scnt.off);
    net->awl = (int32_t *)(A + p_awl.off);
    net->gwsel = (uint32_t *)(A + p_gws.off);
    net->pullf = (uint32_t *)(A + p_pullf.off);
    net->D = (int64_t *)(A + p_D.off);

    // ---- uploads
    auto up = [&](void *dst, const void *src, size_t bytes) -> int {
        if (bytes == 0) return SNN_OK;
        hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) { (void)hipGetLastError(); return fail(SNN_EDEVICE, "upload failed: %s", hipGetErrorString(e)); }
        return SNN_OK;
    };
    {
        std::vector<int32_t> wave_seg(std::max<int64_t>(W, 1), 0);
        for (size_t s = 0; s < net->segs.size(); ++s) {
            const Seg &S = net->segs[s];
            for (int64_t w = S.base / kWave; w < (S.base + align_up(S.n, kWave)) / kWave; ++w) wave_seg[w] = (int32_t)s;
        }
        if ((rc = up(net->d_wave_seg, wave_seg.data(), 4 * W))) return bail(rc);
        // Izhikevich parameters, interleaved per neuron for one 16-byte load
        std::vector<float4> izp(std::max<int64_t>(izp_total, 1), make_float4(0.f, 0.f, 0.f, 0.f));
        for (size_t s = 0; s < net->segs.size(); ++s) {
            const Seg &S = net->segs[s];
            if (S.kind != kIzh) continue;
            const float *abcd = cfg->inst[S.inst].pops[S.pop].izh_abcd;
            for (int32_t j = 0; j < S.n; ++j)
                izp[S.izp_base + j] = make_float4(abcd[j], abcd[S.n + j], abcd[2 * (int64_t)S.n + j],
                                                  abcd[3 * (int64_t)S.n + j]);
        }
        if ((rc = up(net->d_izp, izp.data(), sizeof(float4) * (size_t)izp_total))) return bail(rc);
        if ((rc = up(net->d_units, units.data(), sizeof(int4) * units.size()))) return bail(rc);
        if ((rc = up(net->d_pull_units, pull_units.data(), sizeof(PullUnit) * pull_units.size()))) return bail(rc);
        if ((rc = up(net->d_pull_slices, pull_red.data(), sizeof(PullSlice) * pull_red.size()))) return bail(rc);
        if ((rc = up(net->d_grp_proj, grp.data(), sizeof(int2) * grp.size()))) return bail(rc);
    }
    if ((rc = up(net->d_segs, net->segs.data(), sizeof(Seg) * net->segs.size()))) return bail(rc);
    if ((rc = up(net->d_projs, net->projs.data(), sizeof(Proj) * net->projs.size()))) return bail(rc);
    if ((rc = up(net->d_gscale, net->gscale.data(), 4 * net->n_inst))) return bail(rc);
    for (int b = 0, gq = 0; b < net->n_inst; ++b) {
        const snn_instance_desc &I = cfg->inst[b];
        for (int q = 0; q < I.n_projs; ++q, ++gq) {
            const snn_proj_desc &Q = I.projs[q];
            const Proj &P = net->projs[gq];
            const HostProj &H = net->hprojs[gq];
            if ((rc = up(net->d_rp + P.rp_base, Q.row_ptr, 4 * (size_t)(P.n_pre + 1)))) return bail(rc);
            if ((rc = up(net->d_col + P.syn_base, Q.col_idx, 4 * (size_t)Q.nnz))) return bail(rc);
            if ((rc = up(net->d_w + P.syn_base, Q.g, 4 * (size_t)Q.nnz))) return bail(rc);
            if (P.tp_base >= 0) {
                // start of every post tile in every row (columns ascend within a row)
                std::vector<int32_t> tp((size_t)P.n_pre * (P.n_tiles + 1));
                for (int32_t i = 0; i < P.n_pre; ++i) {
                    int32_t k = Q.row_ptr[i];
                    for (int32_t tl = 0; tl <= P.n_tiles; ++tl) {
                        const int64_t lim = (int64_t)tl * P.tile_w;
                        while (k < Q.row_ptr[i + 1] && Q.col_idx[k] < lim) ++k;
                        tp[(size_t)i * (P.n_tiles + 1) + tl] = k;
                    }
                    tp[(size_t)i * (P.n_tiles + 1) + P.n_tiles] = Q.row_ptr[i + 1];
                }
                if ((rc = up(net->d_tp + P.tp_base, tp.data(), 4 * tp.size()))) return bail(rc);
            }
            if (P.pull_base >= 0) {
                // sliced-ELL copy: lane l of slice j holds column ord[64 j + l],
                // its entries in ascending row order, each the row's delta to
                // the previous entry's row (0 for the first) with gaps above
                // kPullMaxDelta bridged by weight-0 entries; each unit's lanes
                // start from their row before its first entry
                const std::vector<int32_t> &cp = pcol[gq], &ord = pord[gq];
                std::vector<int32_t> fill(cp.begin(), cp.end() - 1), rows(Q.nnz), at(Q.nnz);
                for (int32_t i = 0; i < P.n_pre; ++i)
                    for (int32_t k = Q.row_ptr[i]; k < Q.row_ptr[i + 1]; ++k) {
                        const int32_t e = fill[Q.col_idx[k]]++;
                        rows[e] = i;
                        at[e] = k;
                    }
                const int32_t n_sl = (P.n_post + kWave - 1) / kWave;
                const int64_t gs_end = P.pull_base + n_sl;
                const int64_t pk_a = pull_slices[P.pull_base];
                const int64_t pk_b = gs_end < (int64_t)pull_slices.size() ? pull_slices[gs_end] : pull_total;
                const int32_t u_a = slice_u0[P.pull_base];
                const int32_t u_b = gs_end < (int64_t)slice_u0.size() ? slice_u0[gs_end] : (int32_t)pull_units.size();
                const size_t n_pk = (size_t)(pk_b - pk_a);
                std::vector<float> ew(n_pk * kWave * 4, 0.0f);
                std::vector<uint32_t> ed(n_pk * kWave, 0u);
                std::vector<int32_t> ep(n_pk * kWave * 4, -1), lc((size_t)n_sl * kWave, -1);
                std::vector<int32_t> er0((size_t)(u_b - u_a) * kWave, 0), rbefore;
                for (int32_t j = 0; j < P.n_post; ++j) {
                    const int32_t c = ord[j], sl = j / kWave, l = j % kWave;
                    const int64_t gs = P.pull_base + sl;
                    lc[j] = c;
                    const int64_t pb = pull_slices[gs] - pk_a;
                    const int64_t pe = (gs + 1 < (int64_t)pull_slices.size() ? pull_slices[gs + 1] : pull_total) - pk_a;
                    const int32_t depth = (int32_t)(4 * (pe - pb));
                    rbefore.assign(depth + 1, 0);
                    int32_t R = cp[c + 1] > cp[c] ? rows[cp[c]] : 0, ke = 0;
                    auto emit = [&](int32_t delta, float w, int32_t pos) {
                        const size_t idx = (size_t)(pb + ke / 4) * kWave + l;
                        rbefore[ke] = R;
                        ed[idx] |= (uint32_t)delta << (8 * (ke % 4));
                        ew[idx * 4 + ke % 4] = w;
                        ep[idx * 4 + ke % 4] = pos;
                        R += delta;
                        ++ke;
                    };
                    for (int32_t k = cp[c]; k < cp[c + 1]; ++k) {
                        int32_t gap = k == cp[c] ? 0 : rows[k] - rows[k - 1];
                        while (gap > kPullMaxDelta) {
                            emit(kPullMaxDelta, 0.0f, -1);
                            gap -= kPullMaxDelta;
                        }
                        emit(gap, Q.g[at[k]], (int32_t)(P.syn_base + at[k]));
                    }
                    for (int32_t k = ke; k <= depth; ++k) rbefore[k] = R;
                    for (int32_t u = slice_u0[gs]; u < u_b && pull_units[u].col_off == (int32_t)(gs * kWave); ++u)
                        er0[(size_t)(u - u_a) * kWave + l] = rbefore[4 * (pull_units[u].pk0 - pull_slices[gs])];
                }
                if ((rc = up(net->d_pull_w + pk_a * kWave, ew.data(), 4 * ew.size()))) return bail(rc);
                if ((rc = up(net->d_pull_d + pk_a * kWave, ed.data(), 4 * ed.size()))) return bail(rc);
                if ((rc = up(net->d_pull_perm + pk_a * kWave * 4, ep.data(), 4 * ep.size()))) return bail(rc);
                if ((rc = up(net->d_pull_r0 + (int64_t)u_a * kWave, er0.data(), 4 * er0.size()))) return bail(rc);
                if ((rc = up(net->d_pull_col + P.pull_base * kWave, lc.data(), 4 * lc.size()))) return bail(rc);
            }
            if (Q.stdp) {
                // column view: entries of column j in ascending row order
                std::vector<int32_t> fill(H.col_ptr.begin(), H.col_ptr.end() - 1), rows(Q.nnz), pos(Q.nnz);
                for (int32_t i = 0; i < P.n_pre; ++i)
                    for (int32_t k = Q.row_ptr[i]; k < Q.row_ptr[i + 1]; ++k) {
                        const int32_t at = fill[Q.col_idx[k]]++;
                        rows[at] = i;
                        pos[at] = k;
                    }
                if ((rc = up(net->d_cp + P.cp_base, H.col_ptr.data(), 4 * (size_t)(P.n_post + 1)))) return bail(rc);
                if ((rc = up(net->d_csc_row + P.csc_base, rows.data(), 4 * (size_t)Q.nnz))) return bail(rc);
                if ((rc = up(net->d_csc_pos + P.csc_base, pos.data(), 4 * (size_t)Q.nnz))) return bail(rc);
            }
        }
    }
    // initial state: rest point of every Traub-Miles population, v = -65 mV
    // and u = b v for every Izhikevich population; the rest zero
    {
        std::vector<float> hi[4], lo[4];
        for (int k = 0; k < 4; ++k) {
            hi[k].assign(N, 0.0f);
            lo[k].assign(N, 0.0f);
        }
        for (int b = 0; b < net->n_inst; ++b)
            for (int p = 0; p < cfg->inst[b].n_pops; ++p) {
                const snn_pop_desc &P = cfg->inst[b].pops[p];
                if (P.kind == SNN_IZHIKEVICH) {
                    const Seg &S = net->segs[net->seg_of[b][p]];
                    for (int32_t j = 0; j < S.n; ++j) {
                        const double v0 = -65.0, u0 = (double)P.izh_abcd[S.n + j] * v0;
                        hi[0][S.base + j] = (float)v0;
                        lo[0][S.base + j] = (float)(v0 - (double)(float)v0);
                        hi[1][S.base + j] = (float)u0;
                        lo[1][S.base + j] = (float)(u0 - (double)(float)u0);
                    }
                    continue;
                }
                if (P.kind != SNN_TRAUB_MILES) continue;
                double r[4];
                resting_state(P.hh, r);
                const Seg &S = net->segs[net->seg_of[b][p]];
                for (int k = 0; k < 4; ++k) {
                    const float h = (float)r[k], l = (float)(r[k] - (double)h);
                    std::fill(hi[k].begin() + S.base, hi[k].begin() + S.base + S.n, h);
                    std::fill(lo[k].begin() + S.base, lo[k].begin() + S.base + S.n, l);
                }
            }
        if (hipMemset(net->d_arena, 0, (size_t)net->arena_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(SNN_EDEVICE, "hipMemset failed"));
        }
        for (int k = 0; k < 4; ++k) {
            if ((rc = up(*st_ptrs[2 * k], hi[k].data(), 4 * (size_t)N))) return bail(rc);
            if ((rc = up(*st_ptrs[2 * k + 1], lo[k].data(), 4 * (size_t)N))) return bail(rc);
        }
    }
    net->d_init_state = (float *)dev_alloc(net, 4 * 8 * (size_t)N);
    net->d_flag = (uint32_t *)dev_alloc(net, 256);
    net->d_wmax = (uint32_t *)dev_alloc(net, 4 * std::max<size_t>(net->projs.size(), 1));
    net->max_nnz = 0;
    for (const HostProj &H : net->hprojs) net->max_nnz = std::max(net->max_nnz, H.nnz);
    if (!net->d_init_state || !net->d_flag || !net->d_wmax) return bail(fail(SNN_ENOMEM, "device allocation failed"));
    if (hipMemcpy(net->d_init_state, net->vh, 4 * 8 * (size_t)N, hipMemcpyDeviceToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(SNN_EDEVICE, "state copy failed"));
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(SNN_EDEVICE, "device synchronisation failed"));
    }
    if ((rc = update_qbuckets(net))) return bail(rc);
    net->t = 0;
    *out = net;
    if (cfg->autotune) {
        extern int snn_autotune_internal(snn_net *, const char *);
        rc = snn_autotune_internal(net, cfg->tune_cache);
        if (rc) {
            *out = nullptr;
            return bail(rc);
        }
    }
    return SNN_OK;
}

void snn_destroy(snn_net *net)
{
    if (!net) return;
    if (!net->sticky) (void)hipStreamSynchronize(net->stream);
    release(net);
    delete net;
}

int snn_step(snn_net *net, int64_t n_steps)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (n_steps < 0) return fail(SNN_EINVAL, "n_steps < 0");
    return run_steps(net, n_steps);
}

int snn_sync(snn_net *net)
{
    int rc = check_net(net);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(net->stream));
    StepState st;
    HIP_OK(hipMemcpy(&st, net->st, sizeof st, hipMemcpyDeviceToHost));
    if (st.overflow) {
        net->sticky = true;
        return fail(SNN_EDEVICE, "work queue overflow (flag %u)", st.overflow);
    }
    return SNN_OK;
}

int64_t snn_time(const snn_net *net) { return net ? net->t : -1; }

int snn_get_spikes(snn_net *net, int32_t inst, int32_t pop, int32_t *counts)
{
    int rc = check_net(net);
    if (rc) return rc;
    const int s = seg_index(net, inst, pop, false);
    if (s < 0) return s;
    if (!counts) return fail(SNN_EINVAL, "counts is NULL");
    return d2h(net, counts, net->counts + net->segs[s].base, 4 * (size_t)net->segs[s].n);
}

int snn_get_raster(snn_net *net, int32_t inst, int32_t pop, int64_t t0, int64_t t1, int64_t *offsets, int32_t *ids,
                   int64_t cap)
{
    int rc = check_net(net);
    if (rc) return rc;
    const int s = seg_index(net, inst, pop, false);
    if (s < 0) return s;
    // the ring of the last raster_steps steps, else the recording of the
    // last snn_forward_record
    const bool rec = net->rec_timeline && t0 >= 0 && t0 <= t1 && t1 <= net->rec_T;
    const bool ring = !rec && net->raster_steps > 0 && t0 >= 0 && t0 <= t1 && t1 <= net->t &&
                      t0 >= net->t - net->raster_steps;
    if (!ring && !rec)
        return fail(SNN_ERANGE, "steps [%lld, %lld) are not in the raster window", (long long)t0, (long long)t1);
    const uint64_t *src = ring ? net->raster : net->d_rec_raster;
    const int64_t slots = ring ? net->raster_steps : net->rec_T;
    if (!offsets || (cap > 0 && !ids)) return fail(SNN_EINVAL, "NULL output");
    const Seg &S = net->segs[s];
    const int64_t w0 = S.base / kWave, nw = align_up(S.n, kWave) / kWave;
    std::vector<uint64_t> words(nw);
    int64_t n = 0;
    offsets[0] = 0;
    for (int64_t t = t0; t < t1; ++t) {
        if ((rc = d2h(net, words.data(), src + (t % slots) * net->n_waves + w0, 8 * (size_t)nw))) return rc;
        for (int64_t w = 0; w < nw; ++w)
            for (uint64_t b = words[w]; b; b &= b - 1) {
                const int32_t id = (int32_t)(w * kWave + __builtin_ctzll(b));
                if (n < cap) ids[n] = id;
                ++n;
            }
        offsets[t - t0 + 1] = n;
    }
    return n > cap ? fail(SNN_ERANGE, "raster holds %lld ids, cap %lld", (long long)n, (long long)cap) : SNN_OK;
}

static float *state_hi(snn_net *net, int var) { float *p[4] = {net->vh, net->mh, net->hh, net->nh}; return p[var]; }
static float *state_lo(snn_net *net, int var) { float *p[4] = {net->vl, net->ml, net->hl, net->nl}; return p[var]; }

int snn_get_state_f64(snn_net *net, int32_t inst, int32_t pop, int32_t var, double *out)
{
    int rc = check_net(net);
    if (rc) return rc;
    const int s = seg_index(net, inst, pop, true);
    if (s < 0) return s;
    if (var < 0 || var > (net->segs[s].kind == kIzh ? 1 : 3))
        return fail(SNN_EINVAL, "bad variable %d for population %d", var, pop);
    if (!out) return fail(SNN_EINVAL, "out is NULL");
    const Seg &S = net->segs[s];
    std::vector<float> h(S.n), l(S.n);
    if ((rc = d2h(net, h.data(), state_hi(net, var) + S.base, 4 * (size_t)S.n))) return rc;
    if ((rc = d2h(net, l.data(), state_lo(net, var) + S.base, 4 * (size_t)S.n))) return rc;
    for (int i = 0; i < S.n; ++i) out[i] = (double)h[i] + (double)l[i];
    return SNN_OK;
}

int snn_get_state(snn_net *net, int32_t inst, int32_t pop, int32_t var, float *out)
{
    if (!out) return fail(SNN_EINVAL, "out is NULL");
    const int s = net ? seg_index(net, inst, pop, true) : -1;
    if (s < 0) return net ? s : fail(SNN_EINVAL, "net is NULL");
    std::vector<double> d(net->segs[s].n);
    int rc = snn_get_state_f64(net, inst, pop, var, d.data());
    if (rc) return rc;
    for (size_t i = 0; i < d.size(); ++i) out[i] = (float)d[i];
    return SNN_OK;
}

int snn_set_state_f64(snn_net *net, int32_t inst, int32_t pop, int32_t var, const double *in)
{
    int rc = check_net(net);
    if (rc) return rc;
    const int s = seg_index(net, inst, pop, true);
    if (s < 0) return s;
    if (var < 0 || var > (net->segs[s].kind == kIzh ? 1 : 3))
        return fail(SNN_EINVAL, "bad variable %d for population %d", var, pop);
    if (!in) return fail(SNN_EINVAL, "in is NULL");
    const Seg &S = net->segs[s];
    std::vector<float> h(S.n), l(S.n);
    for (int i = 0; i < S.n; ++i) {
        h[i] = (float)in[i];
        l[i] = (float)(in[i] - (double)h[i]);
    }
    if ((rc = h2d(net, state_hi(net, var) + S.base, h.data(), 4 * (size_t)S.n))) return rc;
    return h2d(net, state_lo(net, var) + S.base, l.data(), 4 * (size_t)S.n);
}

int snn_set_state(snn_net *net, int32_t inst, int32_t pop, int32_t var, const float *in)
{
    if (!in) return fail(SNN_EINVAL, "in is NULL");
    const int s = net ? seg_index(net, inst, pop, true) : -1;
    if (s < 0) return net ? s : fail(SNN_EINVAL, "net is NULL");
    std::vector<double> d(in, in + net->segs[s].n);
    return snn_set_state_f64(net, inst, pop, var, d.data());
}

int snn_get_conductance(snn_net *net, int32_t inst, int32_t proj, double *out)
{
    int rc = check_net(net);
    if (rc) return rc;
    const int q = proj_index(net, inst, proj);
    if (q < 0) return q;
    if (!out) return fail(SNN_EINVAL, "out is NULL");
    const HostProj &H = net->hprojs[q];
    std::vector<int64_t> g(H.n_post);
    if ((rc = d2h(net, g.data(), net->G + H.G_base, 8 * (size_t)H.n_post))) return rc;
    for (int j = 0; j < H.n_post; ++j) out[j] = (double)g[j] * kFixInv;
    return SNN_OK;
}

int snn_set_conductance(snn_net *net, int32_t inst, int32_t proj, const double *in)
{
    int rc = check_net(net);
    if (rc) return rc;
    const int q = proj_index(net, inst, proj);
    if (q < 0) return q;
    if (!in) return fail(SNN_EINVAL, "in is NULL");
    const HostProj &H = net->hprojs[q];
    std::vector<int64_t> g(H.n_post);
    for (int j = 0; j < H.n_post; ++j) {
        if (!(in[j] >= 0.0) || !(in[j] < kGLimit)) return fail(SNN_ERANGE, "conductance %d out of [0, %g) uS", j, kGLimit);
        g[j] = (int64_t)std::llrint(in[j] * kFixOne);
    }
    return h2d(net, net->G + H.G_base, g.data(), 8 * (size_t)H.n_post);
}

int snn_get_last_spikes(snn_net *net, int32_t inst, int32_t pop, uint8_t *out)
{
    int rc = check_net(net);
    if (rc) return rc;
    const int s = seg_index(net, inst, pop, false);
    if (s < 0) return s;
    if (!out) return fail(SNN_EINVAL, "out is NULL");
    const Seg &S = net->segs[s];
    const int64_t nw = align_up(S.n, kWave) / kWave;
    const int slot = (int)((net->t + 1) & 1);
    std::vector<uint64_t> words(nw);
    if ((rc = d2h(net, words.data(), net->bits + slot * net->n_waves + S.base / kWave, 8 * (size_t)nw))) return rc;
    for (int i = 0; i < S.n; ++i) out[i] = (uint8_t)((words[i / kWave] >> (i % kWave)) & 1u);
    return SNN_OK;
}

// Bucket offsets of the queue slots for the current block size and mode:
// block b of the neuron update reserves in bucket b mod kQBuckets, sized to
// the worst case of its waves' neurons.
static int update_qbuckets(snn_net *net)
{
    const int64_t wpb = net->launch.neuron_block / kWave;
    const std::vector<int64_t> &items = net->launch.mode == kModeTiles ? net->wave_items_tiles : net->wave_items_rows;
    std::vector<int64_t> base(kQBuckets + 1, 0);
    for (int64_t w = 0; w < net->n_waves; ++w) base[(w / wpb) % kQBuckets + 1] += items[w];
    for (int x = 0; x < kQBuckets; ++x) base[x + 1] += base[x];
    if (base[kQBuckets] > net->qcap) return fail(SNN_EDEVICE, "queue buckets exceed the queue (internal)");
    return h2d(net, net->d_qb_base, base.data(), 8 * base.size());
}

// Zero the reservation counters of queue slot `slot` (-1: both slots and
// the fused done counts).
static int clear_qbuckets(snn_net *net, int slot)
{
    const size_t words = (size_t)kQBuckets * kQBucketStride;
    HIP_OK(launch_fill_zero(net->qb_cnt + (slot < 0 ? 0 : (size_t)slot * words), 4 * words * (slot < 0 ? 3 : 1),
                            net->stream));
    HIP_OK(hipStreamSynchronize(net->stream));
    return SNN_OK;
}

// Rebuild the propagation work of the pending step from the spike bitmasks
// of the slot it consumes, in the current delivery mode (rows: chunk items
// per spiking row; tiles: active-word lists, spike counts and one item per
// (projection, post tile, active word)); with ltp_seg >= 0 also the
// potentiation items of that population's columns.
static int rebuild_pending(snn_net *net, int ltp_seg, const uint8_t *ltp_flags)
{
    int rc;
    const int slot = (int)((net->t + 1) & 1);
    StepState st;
    if ((rc = d2h(net, &st, net->st, sizeof st))) return rc;
    std::vector<uint64_t> all(net->n_waves);
    if ((rc = d2h(net, all.data(), net->bits + slot * net->n_waves, 8 * (size_t)net->n_waves))) return rc;
    const size_t nseg = net->segs.size();
    std::vector<uint32_t> cnt(nseg, 0), spk(nseg, 0), gws(nseg, 1);
    std::vector<int32_t> awl(net->n_waves, 0);
    std::vector<Item> items;
    const int32_t ch = net->launch.chunk;
    // tile mode: words per group from this step's own counts (the kernels
    // use whatever the emission recorded), items from each group's first word
    for (size_t g = 0; g < nseg; ++g) {
        const Seg &G = net->segs[g];
        const int64_t w0 = G.base / kWave, nwd = align_up(G.n, kWave) / kWave;
        uint32_t na = 0, ns = 0;
        for (int64_t w = 0; w < nwd; ++w)
            if (all[w0 + w]) ++na, ns += (uint32_t)__builtin_popcountll(all[w0 + w]);
        gws[g] = group_words(na, ns, (uint32_t)nwd);
    }
    for (size_t g = 0; g < nseg; ++g) {
        const Seg &G = net->segs[g];
        const int64_t w0 = G.base / kWave, gw = align_up(G.n, kWave) / kWave;
        for (int64_t w = 0; w < gw; ++w) {
            const uint64_t bits = all[w0 + w];
            if (!bits) continue;
            const int32_t slot_w = (int32_t)cnt[g]++;
            awl[w0 + slot_w] = (int32_t)w;
            spk[g] += (uint32_t)__builtin_popcountll(bits);
            for (int o = 0; o < G.n_out; ++o) {
                if (net->launch.mode == kModeTiles) {
                    if ((uint32_t)slot_w % gws[g] != 0) continue;
                    for (int32_t tl = 0; tl < G.out_tiles[o]; ++tl)
                        items.push_back(Item{G.out_proj[o], (int32_t)w, tl, slot_w, bits, 0});
                } else {
                    const HostProj &H = net->hprojs[G.out_proj[o]];
                    for (uint64_t b = bits; b; b &= b - 1) {
                        const int32_t i = (int32_t)(w * kWave + __builtin_ctzll(b));
                        for (int32_t k = H.row_ptr[i]; k < H.row_ptr[i + 1]; k += ch)
                            items.push_back(Item{G.out_proj[o], i, k, std::min(k + ch, H.row_ptr[i + 1]), 0,
                                                 (uint64_t)G.inst});
                    }
                }
            }
        }
    }
    if ((int64_t)items.size() > net->qcap) return fail(SNN_ERANGE, "too many work items");
    if ((rc = h2d(net, net->queue + (int64_t)slot * net->qcap, items.data(), sizeof(Item) * items.size()))) return rc;
    if ((rc = clear_qbuckets(net, slot))) return rc;   // the rebuilt work is all contiguous
    std::vector<uint32_t> zero(nseg, 0);
    if ((rc = h2d(net, net->awcnt + (int64_t)slot * nseg, cnt.data(), 4 * nseg))) return rc;
    if ((rc = h2d(net, net->scnt + (int64_t)slot * nseg, spk.data(), 4 * nseg))) return rc;
    if ((rc = h2d(net, net->awcnt + (int64_t)(slot ^ 1) * nseg, zero.data(), 4 * nseg))) return rc;
    if ((rc = h2d(net, net->scnt + (int64_t)(slot ^ 1) * nseg, zero.data(), 4 * nseg))) return rc;
    if ((rc = h2d(net, net->awl + (int64_t)slot * net->n_waves, awl.data(), 4 * (size_t)net->n_waves))) return rc;
    if ((rc = h2d(net, net->gwsel + (int64_t)slot * nseg, gws.data(), 4 * nseg))) return rc;
    // tile mode: populations at or above the pull threshold are pulled
    std::vector<uint32_t> pf(2 * nseg, 0);
    uint32_t np = 0;
    if (net->launch.mode == kModeTiles)
        for (size_t g = 0; g < nseg; ++g) {
            const Seg &G = net->segs[g];
            const uint32_t thr = (uint32_t)(((uint64_t)G.n * kPullNum + kPullDen - 1) / kPullDen);
            if (G.pullable && spk[g] >= thr) {
                pf[(size_t)slot * nseg + g] = 1;
                ++np;
            }
        }
    if ((rc = h2d(net, net->pullf, pf.data(), 4 * pf.size()))) return rc;
    st.npull[slot] = np;
    st.npull[slot ^ 1] = 0;
    st.qcnt[slot] = (uint32_t)items.size();
    st.grp_off[slot] = 0;   // the groups deliver S(t-1) from its bitmask words
    if (ltp_seg >= 0) {
        const Seg &S = net->segs[ltp_seg];
        const uint32_t n = st.lcnt[slot];
        Item *dq = net->lqueue + (int64_t)slot * net->lcap;
        std::vector<Item> old(n), keep;
        if ((rc = d2h(net, old.data(), dq, sizeof(Item) * n))) return rc;
        for (const Item &it : old)
            if (net->projs[it.proj].post_seg != ltp_seg) keep.push_back(it);
        for (int i = 0; i < S.n; ++i) {
            if (!ltp_flags[i]) continue;
            for (int o = 0; o < S.n_ltp; ++o) {
                const HostProj &H = net->hprojs[S.ltp_proj[o]];
                for (int32_t k = H.col_ptr[i]; k < H.col_ptr[i + 1]; k += ch)
                    keep.push_back(Item{S.ltp_proj[o], i, k, std::min(k + ch, H.col_ptr[i + 1]), 0, 0});
            }
        }
        if ((int64_t)keep.size() > net->lcap) return fail(SNN_ERANGE, "too many work items");
        if ((rc = h2d(net, dq, keep.data(), sizeof(Item) * keep.size()))) return rc;
        st.lcnt[slot] = (uint32_t)keep.size();
    }
    return h2d(net, net->st, &st, sizeof st);
}

// Both queue slots empty and no population marked for pulling: fused steps
// neither fill nor reset them, so a count left from before fused mode must not
// survive a switch in either direction.  The row groups of grouped mode,
// which read the spike words rather than the queue, are told that both slots
// are done.
static int clear_queues(snn_net *net)
{
    int rc;
    StepState st;
    if ((rc = d2h(net, &st, net->st, sizeof st))) return rc;
    st.qcnt[0] = st.qcnt[1] = 0;
    st.grp_off[0] = st.grp_off[1] = 1;
    st.lcnt[0] = st.lcnt[1] = 0;
    st.npull[0] = st.npull[1] = 0;
    if ((rc = clear_qbuckets(net, -1))) return rc;
    std::vector<uint32_t> zero(2 * net->segs.size(), 0);
    if ((rc = h2d(net, net->pullf, zero.data(), 4 * zero.size()))) return rc;
    return h2d(net, net->st, &st, sizeof st);
}

// Fused -> rows/tiles: the pending deliveries of S(t-1) sit in the fused
// buffer slot that the update of step t reads; add them into G, clear the
// slot, and leave the next propagation's queue empty.
static int leave_fused(snn_net *net)
{
    int rc;
    const int64_t n = net->G_count;
    const int64_t dslot = net->t & 1;
    if (n > 0) {
        std::vector<int64_t> g(n), d(n);
        if ((rc = d2h(net, g.data(), net->G, 8 * (size_t)n))) return rc;
        if ((rc = d2h(net, d.data(), net->D + dslot * n, 8 * (size_t)n))) return rc;
        for (int64_t i = 0; i < n; ++i) g[i] += d[i];
        std::fill(d.begin(), d.end(), 0);
        if ((rc = h2d(net, net->G, g.data(), 8 * (size_t)n))) return rc;
        if ((rc = h2d(net, net->D + dslot * n, d.data(), 8 * (size_t)n))) return rc;
    }
    if ((rc = clear_queues(net))) return rc;
    const size_t nseg = net->segs.size();
    std::vector<uint32_t> zero(2 * nseg, 0);
    if ((rc = h2d(net, net->awcnt, zero.data(), 4 * zero.size()))) return rc;
    return h2d(net, net->scnt, zero.data(), 4 * zero.size());
}

// Entering fused mode (or replacing S(t-1) in it): the pending deliveries of
// S(t-1) belong in the fused buffer slot that the update of step t reads.
// Clear that slot, then run the queued work (laid out for `mode`, rows or
// tiles) with that slot as its target instead of G, and empty the queues.
static int deliver_queued_to_fused(snn_net *net, int mode)
{
    int rc;
    const int64_t n = net->G_count;
    int64_t *slot = net->D + (net->t & 1) * n;
    if (n > 0) {
        std::vector<int64_t> zero(n, 0);
        if ((rc = h2d(net, slot, zero.data(), 8 * (size_t)n))) return rc;
    }
    const snn_launch keep = net->launch;
    net->launch.mode = mode;
    PropArgs p = prop_args(net);
    net->launch = keep;
    p.G = slot;
    hipError_t e = launch_propagate(p, net->launch.prop_blocks, net->launch.prop_block, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    if (e != hipSuccess) {
        net->sticky = true;
        return fail(SNN_EDEVICE, "delivery of the pending work failed: %s", hipGetErrorString(e));
    }
    return clear_queues(net);
}

// Replace S(t-1) of one population: rewrite its bitmask words and rebuild
// the pending work (propagation of every population, potentiation of this
// population's columns).
int snn_set_last_spikes(snn_net *net, int32_t inst, int32_t pop, const uint8_t *in)
{
    int rc = check_net(net);
    if (rc) return rc;
    const int s = seg_index(net, inst, pop, false);
    if (s < 0) return s;
    if (!in) return fail(SNN_EINVAL, "in is NULL");
    const Seg &S = net->segs[s];
    const int slot = (int)((net->t + 1) & 1);
    const int64_t nw = align_up(S.n, kWave) / kWave;
    std::vector<uint64_t> words(nw, 0);
    for (int i = 0; i < S.n; ++i)
        if (in[i]) words[i / kWave] |= (uint64_t)1 << (i % kWave);
    if ((rc = h2d(net, net->bits + slot * net->n_waves + S.base / kWave, words.data(), 8 * (size_t)nw))) return rc;
    if (net->launch.mode != kModeFused) return rebuild_pending(net, s, in);
    // fused mode: the pending deliveries become those of the new S(t-1) of
    // every population, laid out as a rows-mode queue and run into the slot
    net->launch.mode = kModeRows;
    rc = rebuild_pending(net, -1, nullptr);
    net->launch.mode = kModeFused;
    if (rc) return rc;
    return deliver_queued_to_fused(net, kModeRows);
}

int snn_get_vbar(snn_net *net, int32_t inst, int32_t pop, double *out)
{
    int rc = check_net(net);
    if (rc) return rc;
    const int s = seg_index(net, inst, pop, true);
    if (s < 0) return s;
    if (!net->segs[s].record_vbar) return fail(SNN_ESTATE, "population %d was created without record_vbar", pop);
    if (!out) return fail(SNN_EINVAL, "out is NULL");
    return d2h(net, out, net->vsum + net->segs[s].base, 8 * (size_t)net->segs[s].n);
}

int snn_get_nan_counts(snn_net *net, int32_t *per_instance)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (!per_instance) return fail(SNN_EINVAL, "out is NULL");
    return d2h(net, per_instance, net->nan_count, 4 * (size_t)net->n_inst);
}

int snn_set_gscale(snn_net *net, const float *per_instance)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (!per_instance) return fail(SNN_EINVAL, "in is NULL");
    for (int b = 0; b < net->n_inst; ++b)
        if (!(per_instance[b] >= 0.0f) || !std::isfinite(per_instance[b]))
            return fail(SNN_EINVAL, "g_scale of instance %d must be finite and >= 0", b);
    // same range rule as at create, on the stored weights' column sums
    std::vector<double> bound(net->projs.size(), 0.0), wbound(net->projs.size(), 0.0);
    for (size_t q = 0; q < net->projs.size(); ++q) {
        const HostProj &H = net->hprojs[q];
        std::vector<int32_t> col(H.nnz);
        std::vector<float> w(H.nnz);
        if ((rc = d2h(net, col.data(), net->d_col + H.syn_base, 4 * (size_t)H.nnz))) return rc;
        if ((rc = d2h(net, w.data(), net->d_w + H.syn_base, 4 * (size_t)H.nnz))) return rc;
        std::vector<double> cs(std::max(H.n_post, 1), 0.0);
        for (int64_t k = 0; k < H.nnz; ++k) cs[col[k]] += w[k];
        double wm = H.stdp ? (double)net->projs[q].g_max : 0.0;
        for (int64_t k = 0; k < H.nnz; ++k) wm = std::max(wm, (double)w[k]);
        wbound[q] = wm;
        double mx = 0.0;
        for (double c : cs) mx = std::max(mx, c);
        if (H.stdp) mx = std::max(mx, (double)net->projs[q].g_max * H.n_pre);
        const int s = net->seg_of[H.inst][H.post_pop];
        double decay = 0.0;
        for (int k = 0; k < net->segs[s].n_in; ++k)
            if (net->segs[s].in_G[k] == H.G_base) decay = net->segs[s].in_decay[k];
        bound[q] = mx / (1.0 - decay);
    }
    if ((rc = check_range(net, bound, wbound, per_instance))) return rc;
    std::copy(per_instance, per_instance + net->n_inst, net->gscale.begin());
    if ((rc = h2d(net, net->d_gscale, per_instance, 4 * (size_t)net->n_inst))) return rc;
    if (net->launch.mode != kModeFused) return SNN_OK;
    // fused mode: the pending deliveries of S(t-1) were made with the old
    // g_scale; the other modes deliver them at step t with the new one
    net->launch.mode = kModeRows;
    rc = rebuild_pending(net, -1, nullptr);
    net->launch.mode = kModeFused;
    if (rc) return rc;
    return deliver_queued_to_fused(net, kModeRows);
}

int snn_get_weights(snn_net *net, int32_t inst, int32_t proj, float *out)
{
    int rc = check_net(net);
    if (rc) return rc;
    const int q = proj_index(net, inst, proj);
    if (q < 0) return q;
    if (!out) return fail(SNN_EINVAL, "out is NULL");
    const HostProj &H = net->hprojs[q];
    return d2h(net, out, net->d_w + H.syn_base, 4 * (size_t)H.nnz);
}

int snn_memory_bytes(const snn_net *net, int64_t *per_proj_bytes)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    if (!per_proj_bytes) return fail(SNN_EINVAL, "out is NULL");
    for (size_t q = 0; q < net->hprojs.size(); ++q)
        per_proj_bytes[q] = 4 * (2 * net->hprojs[q].nnz + net->hprojs[q].n_pre + 1);
    return SNN_OK;
}

int snn_get_launch(const snn_net *net, snn_launch *out)
{
    if (!net || !out) return fail(SNN_EINVAL, "NULL argument");
    *out = net->launch;
    return SNN_OK;
}

int snn_set_launch(snn_net *net, const snn_launch *in)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (!in) return fail(SNN_EINVAL, "in is NULL");
    if (in->neuron_block < 64 || in->neuron_block > 1024 || in->neuron_block % 64)
        return fail(SNN_EINVAL, "neuron_block must be a multiple of 64 in [64, 1024]");
    if (in->prop_block < 64 || in->prop_block > 1024 || in->prop_block % 64)
        return fail(SNN_EINVAL, "prop_block must be a multiple of 64 in [64, 1024]");
    if (in->prop_blocks < 1 || in->prop_blocks > 65536) return fail(SNN_EINVAL, "prop_blocks must be in [1, 65536]");
    if (in->chunk < kMinChunk || in->chunk % kWave || in->chunk > (1 << 20))
        return fail(SNN_EINVAL, "chunk must be a multiple of 64 in [64, 2^20]");
    if (in->mode != kModeRows && in->mode != kModeTiles && in->mode != kModeFused && in->mode != kModeGrouped)
        return fail(SNN_EINVAL, "mode must be 0 (rows), 1 (tiles), 2 (fused) or 3 (grouped)");
    if (in->mode == kModeGrouped && in->prop_block > 512)
        return fail(SNN_EINVAL, "mode 3 (grouped) needs prop_block <= 512 (an 8 KiB LDS tile per wavefront)");
    if (in->mode == kModeFused && net->plastic)
        return fail(SNN_EINVAL, "mode 2 (fused) needs a network without plastic projections");
    const snn_launch prev = net->launch;
    net->launch = *in;
    if ((rc = update_qbuckets(net))) return rc;
    // The pending work of the next step was laid out for the old mode and in
    // the buckets of the old block size: it is laid out again from the spike
    // bitmasks, contiguously (entering fused mode: as rows work, run at once
    // into the fused buffer).
    if (in->mode == kModeFused) {
        if (prev.mode != kModeFused) {
            net->launch.mode = kModeRows;
            rc = rebuild_pending(net, -1, nullptr);
            net->launch.mode = kModeFused;
            if (!rc) rc = deliver_queued_to_fused(net, kModeRows);
        }
    } else if (prev.mode == kModeFused) {
        rc = leave_fused(net);
    } else if (prev.mode != in->mode || prev.neuron_block != in->neuron_block) {
        rc = rebuild_pending(net, -1, nullptr);
    }
    if (rc) return rc;
    drop_graphs(net);
    return SNN_OK;
}

int snn_time_steps(snn_net *net, int64_t n_steps, double *out_ms)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (n_steps < 1 || !out_ms) return fail(SNN_EINVAL, "need n_steps >= 1 and an output");
    // capture the graph before the clock starts: host capture time is not step time
    if ((rc = prepare_graphs(net, n_steps))) return rc;
    double ms = 0.0;
    rc = timed_on_snapshot(net, [&]() { return run_steps(net, n_steps); }, &ms);
    if (rc) return rc;
    *out_ms = ms / (double)n_steps;
    return SNN_OK;
}

int snn_time_kernel(snn_net *net, int32_t which, int64_t launches, double *ms_per_launch)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (which < 0 || which > 2) return fail(SNN_EINVAL, "which must be 0, 1 or 2");
    if (which == 1 && !net->plastic) return fail(SNN_ESTATE, "no plastic projection");
    if (which == 0 && net->launch.mode == kModeFused)
        return fail(SNN_ESTATE, "mode 2 (fused) has no propagation kernel");
    if (launches < 1 || launches > 1000000 || !ms_per_launch) return fail(SNN_EINVAL, "need 1 <= launches <= 1e6 and an output");
    PropArgs p = prop_args(net);
    LtpArgs l = ltp_args(net);
    NeuronArgs a = neuron_args(net);
    double ms = 0.0;
    rc = timed_on_snapshot(net, [&]() -> int {
        for (int64_t k = 0; k < launches; ++k) {
            hipError_t e = which == 0 ? launch_propagate(p, net->launch.prop_blocks, net->launch.prop_block, net->stream)
                         : which == 1 ? launch_potentiate(l, net->launch.prop_blocks, net->launch.prop_block, net->stream)
                                      : launch_neuron(a, net->launch.neuron_block, net->stream);
            if (e != hipSuccess) {
                net->sticky = true;
                return fail(SNN_EDEVICE, "launch failed: %s", hipGetErrorString(e));
            }
        }
        return SNN_OK;
    }, &ms);
    if (rc) return rc;
    *ms_per_launch = ms / (double)launches;
    return SNN_OK;
}

int snn_profile_steps(snn_net *net, int64_t n_steps, double *ms_total, int64_t *launches)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (n_steps < 1 || n_steps > 100000 || !ms_total || !launches)
        return fail(SNN_EINVAL, "need 1 <= n_steps <= 100000 and two output arrays");
    const bool fused = net->launch.mode == kModeFused;
    const int per_step = fused ? 1 : net->plastic ? 3 : 2;
    std::vector<hipEvent_t> ev((size_t)(2 * per_step * n_steps), nullptr);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < ev.size() && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    const PropArgs p = prop_args(net);
    const LtpArgs l = ltp_args(net);
    const NeuronArgs a = neuron_args(net);
    int64_t done = 0;
    for (; done < n_steps && e == hipSuccess; ++done) {
        hipEvent_t *E = ev.data() + 2 * per_step * done;
        if (fused) {
            e = launch_neuron(a, net->launch.neuron_block, net->stream, E[0], E[1]);
            if (e == hipSuccess) net->t += 1;
            continue;
        }
        e = launch_propagate(p, net->launch.prop_blocks, net->launch.prop_block, net->stream, E[0], E[1]);
        if (e == hipSuccess && net->plastic)
            e = launch_potentiate(l, net->launch.prop_blocks, net->launch.prop_block, net->stream, E[4], E[5]);
        if (e == hipSuccess) e = launch_neuron(a, net->launch.neuron_block, net->stream, E[2], E[3]);
        if (e == hipSuccess) net->t += 1;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    for (int k = 0; k < 3; ++k) ms_total[k] = 0.0, launches[k] = 0;
    for (int64_t t = 0; t < n_steps && e == hipSuccess; ++t) {
        hipEvent_t *E = ev.data() + 2 * per_step * t;
        for (int k = 0; k < per_step && e == hipSuccess; ++k) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, E[2 * k], E[2 * k + 1]);
            const int which = fused ? 2 : k == 0 ? 0 : k == 1 ? 2 : 1;
            ms_total[which] += (double)ms;
            launches[which] += 1;
        }
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) {
        net->sticky = true;
        return fail(SNN_EDEVICE, "profiled steps failed: %s", hipGetErrorString(e));
    }
    return SNN_OK;
}

int snn_reset(snn_net *net)
{
    int rc = check_net(net);
    if (rc) return rc;
    net->rec_timeline = false;
    HIP_OK(hipMemsetAsync(net->d_arena, 0, (size_t)net->arena_bytes, net->stream));
    HIP_OK(hipMemcpyAsync(net->vh, net->d_init_state, 4 * 8 * (size_t)net->n_neurons_padded, hipMemcpyDeviceToDevice,
                          net->stream));
    net->t = 0;
    return SNN_OK;
}

int64_t snn_weight_count(const snn_net *net) { return net ? net->w_count : -1; }

int snn_weight_offset(const snn_net *net, int32_t inst, int32_t proj, int64_t *offset)
{
    if (!net || !offset) return fail(SNN_EINVAL, "NULL argument");
    const int q = proj_index(net, inst, proj);
    if (q < 0) return q;
    *offset = net->hprojs[q].syn_base;
    return SNN_OK;
}

int snn_get_weights_device(snn_net *net, float *dst)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (!dst) return fail(SNN_EINVAL, "dst is NULL");
    HIP_OK(hipMemcpyAsync(dst, net->d_w, 4 * (size_t)net->w_count, hipMemcpyDeviceToDevice, net->stream));
    return SNN_OK;
}

int snn_set_weights_device(snn_net *net, const float *src)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (!src) return fail(SNN_EINVAL, "src is NULL");
    const size_t np = net->projs.size();
    uint32_t flag = 0;
    std::vector<uint32_t> wbits(np, 0);
    HIP_OK(hipMemsetAsync(net->d_flag, 0, 4, net->stream));
    HIP_OK(hipMemsetAsync(net->d_wmax, 0, 4 * std::max<size_t>(np, 1), net->stream));
    HIP_OK(launch_check_weights(src, net->d_projs, (int32_t)np, net->max_nnz, net->d_flag, net->d_wmax, net->stream));
    HIP_OK(hipMemcpyAsync(&flag, net->d_flag, 4, hipMemcpyDeviceToHost, net->stream));
    if (np) HIP_OK(hipMemcpyAsync(wbits.data(), net->d_wmax, 4 * np, hipMemcpyDeviceToHost, net->stream));
    HIP_OK(hipStreamSynchronize(net->stream));
    if (flag) return fail(SNN_EINVAL, "weights must be finite and >= 0");
    // the range rules of snn_create: a single increment below kWLimit, and
    // g_scale * column sum / (1 - decay) below kGLimit, checked first on the
    // bound longest column * largest weight, exactly only where that fails
    for (size_t q = 0; q < np; ++q) {
        const HostProj &H = net->hprojs[q];
        const Proj &P = net->projs[q];
        float wmf;
        std::memcpy(&wmf, &wbits[q], 4);
        const double gs = net->gscale[H.inst];
        const double wm = std::max(H.stdp ? (double)P.g_max : 0.0, (double)wmf);
        if (!(wm * gs < kWLimit))
            return fail(SNN_ERANGE, "projection %zu: g_scale * largest weight exceeds %g uS", q, kWLimit);
        double bound = (double)H.max_col_len * wm;
        if (H.stdp) bound = std::max(bound, (double)P.g_max * H.n_pre);
        if (bound * gs / (1.0 - H.decay) < kGLimit) continue;
        std::vector<int32_t> col(H.nnz);
        std::vector<float> w(H.nnz);
        if ((rc = d2h(net, col.data(), net->d_col + H.syn_base, 4 * (size_t)H.nnz))) return rc;
        if ((rc = d2h(net, w.data(), src + H.syn_base, 4 * (size_t)H.nnz))) return rc;
        std::vector<double> cs(std::max(H.n_post, 1), 0.0);
        for (int64_t k = 0; k < H.nnz; ++k) cs[col[k]] += w[k];
        double mx = *std::max_element(cs.begin(), cs.end());
        if (H.stdp) mx = std::max(mx, (double)P.g_max * H.n_pre);
        if (!(mx * gs / (1.0 - H.decay) < kGLimit))
            return fail(SNN_ERANGE, "projection %zu: g_scale * column sum / (1 - decay) exceeds %g uS", q, kGLimit);
    }
    HIP_OK(hipMemcpyAsync(net->d_w, src, 4 * (size_t)net->w_count, hipMemcpyDeviceToDevice, net->stream));
    HIP_OK(launch_gather_weights(net->d_w, net->d_pull_perm, (float *)net->d_pull_w, 4 * kWave * net->pull_count,
                                 net->stream));
    if (net->launch.mode != kModeFused) return SNN_OK;
    // fused mode: the pending deliveries of S(t-1) were made with the old
    // weights; the other modes deliver them at step t with the new ones
    net->launch.mode = kModeRows;
    rc = rebuild_pending(net, -1, nullptr);
    net->launch.mode = kModeFused;
    if (rc) return rc;
    return deliver_queued_to_fused(net, kModeRows);
}

int snn_forward_record(snn_net *net, int32_t pop, int64_t n_steps, int32_t ckpt_every, double *vbar)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (n_steps < 1 || ckpt_every < 1) return fail(SNN_EINVAL, "need n_steps >= 1 and ckpt_every >= 1");
    if (!vbar) return fail(SNN_EINVAL, "vbar is NULL");
    if (net->plastic) return fail(SNN_ESTATE, "the adjoint needs fixed weights (no STDP projection)");
    if (net->substeps > kAdjMaxSub) return fail(SNN_EINVAL, "the adjoint supports at most %d substeps", kAdjMaxSub);
    std::vector<int32_t> lseg(net->n_inst);
    std::vector<int64_t> lbase(net->n_inst + 1, 0);
    int n_in_max = 1;
    for (int b = 0; b < net->n_inst; ++b) {
        if (pop < 0 || pop >= (int32_t)net->seg_of[b].size()) return fail(SNN_EINVAL, "instance %d has no population %d", b, pop);
        const Seg &S = net->segs[net->seg_of[b][pop]];
        if (S.kind != kHH) return fail(SNN_EINVAL, "population %d of instance %d is not Traub-Miles", pop, b);
        if (!S.record_vbar) return fail(SNN_ESTATE, "population %d of instance %d was created without record_vbar", pop, b);
        if (S.n > kAdjMaxLoss) return fail(SNN_EINVAL, "the adjoint supports at most %d neurons per instance", kAdjMaxLoss);
        lseg[b] = net->seg_of[b][pop];
        lbase[b + 1] = lbase[b] + S.n;
        n_in_max = std::max(n_in_max, S.n_in);
    }
    const int64_t T = n_steps, K = std::min<int64_t>(ckpt_every, T);
    const int64_t nseg = (T + K - 1) / K;
    const int64_t N = net->n_neurons_padded, W = net->n_waves;
    const int64_t n_loss = lbase[net->n_inst];
    std::vector<int32_t> owner(std::max<int64_t>(n_loss, 1), 0);
    for (int b = 0; b < net->n_inst; ++b)
        for (int64_t c = lbase[b]; c < lbase[b + 1]; ++c) owner[c] = b;
    std::vector<int4> items;
    for (int b = 0; b < net->n_inst; ++b) {
        const Seg &S = net->segs[lseg[b]];
        for (int q = 0; q < S.n_in; ++q) {
            const Proj &P = net->projs[S.in_proj[q]];
            const int nw = (int)(align_up(net->segs[P.pre_seg].n, kWave) / kWave);
            for (int w = 0; w < nw; ++w) items.push_back(make_int4(b, q, P.pre_seg, w));
        }
    }
    // (re)allocate the recording
    void *old[] = {net->d_rec_raster, net->d_ckpt_state, net->d_ckpt_G, net->d_loss_seg, net->d_loss_base,
                   net->d_loss_owner, net->d_gitems, net->d_tape_x, net->d_tape_g, net->d_lg, net->d_lam};
    for (void *p : old) dev_free(net, p);
    net->recorded = false;
    net->d_rec_raster = (uint64_t *)dev_alloc(net, 8 * (size_t)(T * W));
    net->d_ckpt_state = (float *)dev_alloc(net, 4 * (size_t)(nseg * 8 * N));
    net->d_ckpt_G = (int64_t *)dev_alloc(net, 8 * (size_t)(nseg * std::max<int64_t>(net->G_count, 1)));
    net->d_loss_seg = (int32_t *)dev_alloc(net, 4 * (size_t)net->n_inst);
    net->d_loss_base = (int64_t *)dev_alloc(net, 8 * (size_t)(net->n_inst + 1));
    net->d_loss_owner = (int32_t *)dev_alloc(net, 4 * owner.size());
    net->d_gitems = (int4 *)dev_alloc(net, sizeof(int4) * std::max<size_t>(items.size(), 1));
    net->d_tape_x = (double *)dev_alloc(net, 8 * (size_t)(K * 4 * std::max<int64_t>(n_loss, 1)));
    net->d_tape_g = (double *)dev_alloc(net, 8 * (size_t)(K * n_in_max * std::max<int64_t>(n_loss, 1)));
    net->d_lg = (double *)dev_alloc(net, 8 * (size_t)(K * n_in_max * std::max<int64_t>(n_loss, 1)));
    net->d_lam = (double *)dev_alloc(net, 8 * (size_t)((4 + n_in_max) * std::max<int64_t>(n_loss, 1)));
    if (!net->d_rec_raster || !net->d_ckpt_state || !net->d_ckpt_G || !net->d_loss_seg || !net->d_loss_base ||
        !net->d_loss_owner || !net->d_gitems || !net->d_tape_x || !net->d_tape_g || !net->d_lg || !net->d_lam)
        return fail(SNN_ENOMEM, "allocation of the adjoint recording failed");
    if ((rc = h2d(net, net->d_loss_seg, lseg.data(), 4 * lseg.size()))) return rc;
    if ((rc = h2d(net, net->d_loss_base, lbase.data(), 8 * lbase.size()))) return rc;
    if ((rc = h2d(net, net->d_loss_owner, owner.data(), 4 * owner.size()))) return rc;
    if ((rc = h2d(net, net->d_gitems, items.data(), sizeof(int4) * items.size()))) return rc;
    net->n_loss = n_loss;
    net->n_in_max = n_in_max;
    // the recompute's block per instance: all of its wavefronts walk a step's
    // raster words and rows (the step's longest phase), then the first n
    // threads update the loss neurons; a full block of kAdjMaxLoss threads
    // spreads that walk over 16 wavefronts instead of the neurons' few
    net->loss_block = kAdjMaxLoss;
    net->n_gitems = (int64_t)items.size();
    net->rec_pop = pop;
    net->rec_T = T;
    net->rec_K = (int32_t)K;
    net->rec_nseg = nseg;

    // forward from the initial state, recording the raster and checkpoints
    if ((rc = snn_reset(net))) return rc;
    NeuronArgs na = neuron_args(net);
    na.raster = net->d_rec_raster;
    na.raster_steps = (int32_t)T;
    const PropArgs pa = prop_args(net);
    for (int64_t t = 0; t < T; ++t) {
        if (t % K == 0) {
            const int64_t sgi = t / K;
            HIP_OK(hipMemcpyAsync(net->d_ckpt_state + sgi * 8 * N, net->vh, 4 * 8 * (size_t)N, hipMemcpyDeviceToDevice,
                                  net->stream));
            HIP_OK(hipMemcpyAsync(net->d_ckpt_G + sgi * std::max<int64_t>(net->G_count, 1), net->G,
                                  8 * (size_t)net->G_count, hipMemcpyDeviceToDevice, net->stream));
        }
        HIP_OK(launch_propagate(pa, net->launch.prop_blocks, net->launch.prop_block, net->stream));
        HIP_OK(launch_neuron(na, net->launch.neuron_block, net->stream));
        net->t += 1;
    }
    HIP_OK(launch_gather_vbar(net->d_segs, net->d_loss_seg, net->d_loss_base, net->d_loss_owner, n_loss, net->vsum,
                              1.0 / (double)T, vbar, net->stream));
    net->recorded = true;
    net->rec_timeline = true;
    return SNN_OK;
}

}  // extern "C"

namespace {

// The backward pass of snn_backward and snn_backward_noalloc: per segment,
// from the last to the first, recompute the loss population from its
// checkpoint into the tape, reverse it, gather the weight gradients.  The
// tape (tape_x, tape_g, lg), the adjoint carried across segments (lam) and
// the recompute check flag are the callers' scratch; lam, the flag and the
// two outputs are cleared here, by memset nodes or (fill_kernel) by a fill
// kernel.
int run_backward(snn_net *net, const double *dL_dvbar, float *dL_dg, double *dL_dgscale, double *tape_x,
                 double *tape_g, double *lg, double *lam, uint32_t *flag, bool fill_kernel)
{
    const int64_t N = net->n_neurons_padded;
    const int64_t gstride = std::max<int64_t>(net->G_count, 1);
    const size_t lam_bytes = 8 * (size_t)((4 + net->n_in_max) * std::max<int64_t>(net->n_loss, 1));
    if (fill_kernel) {
        HIP_OK(launch_fill_zero(lam, lam_bytes, net->stream));
        HIP_OK(launch_fill_zero(dL_dg, 4 * (size_t)net->w_count, net->stream));
        HIP_OK(launch_fill_zero(dL_dgscale, 8 * (size_t)net->n_inst, net->stream));
        HIP_OK(launch_fill_zero(flag, 4, net->stream));
    } else {
        HIP_OK(hipMemsetAsync(lam, 0, lam_bytes, net->stream));
        HIP_OK(hipMemsetAsync(dL_dg, 0, 4 * (size_t)net->w_count, net->stream));
        HIP_OK(hipMemsetAsync(dL_dgscale, 0, 8 * (size_t)net->n_inst, net->stream));
        HIP_OK(hipMemsetAsync(flag, 0, 4, net->stream));
    }
    AdjArgs a{};
    a.segs = net->d_segs;
    a.projs = net->d_projs;
    a.n_inst = net->n_inst;
    a.loss_seg = net->d_loss_seg;
    a.loss_base = net->d_loss_base;
    a.loss_owner = net->d_loss_owner;
    a.n_loss = net->n_loss;
    a.n_in_max = net->n_in_max;
    a.raster = net->d_rec_raster;
    a.n_waves = net->n_waves;
    a.T = net->rec_T;
    a.n_pad = N;
    a.mismatch = flag;
    a.rp_pool = net->d_rp;
    a.col_pool = net->d_col;
    a.w_pool = net->d_w;
    a.gscale = net->d_gscale;
    a.tape_x = tape_x;
    a.tape_g = tape_g;
    a.lam = lam;
    a.lg = lg;
    a.dvbar = dL_dvbar;
    a.substeps = net->substeps;
    a.hs = net->dt / net->substeps;
    a.gitems = net->d_gitems;
    a.n_gitems = net->n_gitems;
    a.dg = dL_dg;
    a.ds = dL_dgscale;
    for (int64_t sg = net->rec_nseg - 1; sg >= 0; --sg) {
        a.t_a = sg * net->rec_K;
        a.K = (int32_t)std::min<int64_t>(net->rec_K, net->rec_T - a.t_a);
        a.ckpt_state = net->d_ckpt_state + sg * 8 * N;
        a.ckpt_G = net->d_ckpt_G + sg * gstride;
        a.next_state = sg + 1 < net->rec_nseg ? net->d_ckpt_state + (sg + 1) * 8 * N : nullptr;
        a.next_G = sg + 1 < net->rec_nseg ? net->d_ckpt_G + (sg + 1) * gstride : nullptr;
        HIP_OK(launch_adj_recompute(a, net->loss_block, net->stream));
        HIP_OK(launch_adj_reverse(a, net->stream));
        HIP_OK(launch_adj_gather(a, net->stream));
    }
    return SNN_OK;
}

// Bytes of scratch the backward of the current recording needs: the check
// flag (256 B, keeping what follows aligned), then tape_x [K][4][n_loss],
// tape_g and lg [K][n_in_max][n_loss], lam [4 + n_in_max][n_loss], doubles.
size_t backward_scratch_bytes(const snn_net *net)
{
    const size_t nl = (size_t)std::max<int64_t>(net->n_loss, 1), K = (size_t)net->rec_K;
    const size_t nin = (size_t)net->n_in_max;
    return 256 + 8 * nl * (K * 4 + 2 * K * nin + 4 + nin);
}

}  // namespace

extern "C" {

int snn_backward(snn_net *net, const double *dL_dvbar, float *dL_dg, double *dL_dgscale, int64_t *mismatch)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (!net->recorded) return fail(SNN_ESTATE, "call snn_forward_record first");
    if (!dL_dvbar || !dL_dg || !dL_dgscale) return fail(SNN_EINVAL, "NULL argument");
    if ((rc = run_backward(net, dL_dvbar, dL_dg, dL_dgscale, net->d_tape_x, net->d_tape_g, net->d_lg, net->d_lam,
                           net->d_flag, false)))
        return rc;
    if (mismatch) {
        uint32_t m = 0;
        HIP_OK(hipMemcpyAsync(&m, net->d_flag, 4, hipMemcpyDeviceToHost, net->stream));
        HIP_OK(hipStreamSynchronize(net->stream));
        *mismatch = m;
    }
    return SNN_OK;
}

int snn_backward_noalloc(snn_net *net, const double *dL_dvbar, float *dL_dg, double *dL_dgscale)
{
    int rc = check_net(net);
    if (rc) return rc;
    if (!net->recorded) return fail(SNN_ESTATE, "call snn_forward_record first");
    if (!dL_dvbar || !dL_dg || !dL_dgscale) return fail(SNN_EINVAL, "NULL argument");
    const size_t need = backward_scratch_bytes(net);
    if (need > kScratchBytes)
        return fail(SNN_ERANGE, "this recording's backward needs %zu bytes of scratch, more than the %zu of "
                                "snn_backward_noalloc (fewer loss neurons or a shorter checkpoint interval)",
                    need, kScratchBytes);
    char *base = static_cast<char *>(scratch_on_device(net->device));
    if (!base) return fail(SNN_EDEVICE, "the scratch array's device address is unknown on device %d", net->device);
    const size_t nl = (size_t)std::max<int64_t>(net->n_loss, 1), K = (size_t)net->rec_K;
    const size_t nin = (size_t)net->n_in_max;
    double *tape_x = reinterpret_cast<double *>(base + 256);
    double *tape_g = tape_x + K * 4 * nl;
    double *lg = tape_g + K * nin * nl;
    double *lam = lg + K * nin * nl;
    return run_backward(net, dL_dvbar, dL_dg, dL_dgscale, tape_x, tape_g, lg, lam, reinterpret_cast<uint32_t *>(base),
                        true);
}

}  // extern "C"

// ------------------------------- autotuner ----------------------------------
// Coordinate search over the launch shape on the real network: time a short
// run per candidate (state restored after each), keep the fastest value of
// one parameter, move to the next.  Results are bitwise independent of the
// shape, so tuning never changes what is computed.
static std::string signature(const snn_net *net)
{
    hipDeviceProp_t prop{};
    (void)hipGetDeviceProperties(&prop, net->device);
    int64_t nnz = 0;
    for (const HostProj &H : net->hprojs) nnz += H.nnz;
    char buf[256];
    snprintf(buf, sizeof buf, "%s:i%d:s%zu:n%lld:z%lld:p%d", prop.gcnArchName, net->n_inst, net->segs.size(),
             (long long)net->n_neurons_padded, (long long)nnz, net->plastic ? 1 : 0);
    return buf;
}

static bool cache_lookup(const char *path, const std::string &sig, snn_launch *out)
{
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char key[300];
        snn_launch L{};
        if (sscanf(line, " \"%299[^\"]\" : [ %d , %d , %d , %d , %d ]", key, &L.neuron_block, &L.prop_blocks,
                   &L.prop_block, &L.chunk, &L.mode) == 6 && sig == key) {
            *out = L;
            found = true;
        }
    }
    fclose(f);
    return found;
}

static void cache_store(const char *path, const std::string &sig, const snn_launch &L)
{
    if (!path) return;
    std::vector<std::string> keep;
    if (FILE *f = fopen(path, "r")) {
        char line[512];
        while (fgets(line, sizeof line, f)) {
            std::string s(line);
            if (s.find("\"") != std::string::npos && s.find("\"" + sig + "\"") == std::string::npos) {
                while (!s.empty() && (s.back() == '\n' || s.back() == ',' || s.back() == ' ')) s.pop_back();
                keep.push_back(s);
            }
        }
        fclose(f);
    }
    char buf[512];
    snprintf(buf, sizeof buf, "  \"%s\": [%d, %d, %d, %d, %d]", sig.c_str(), L.neuron_block, L.prop_blocks, L.prop_block,
             L.chunk, L.mode);
    keep.push_back(buf);
    if (FILE *f = fopen(path, "w")) {
        fprintf(f, "{\n");
        for (size_t i = 0; i < keep.size(); ++i) fprintf(f, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
        fprintf(f, "}\n");
        fclose(f);
    }
}

int snn_autotune_internal(snn_net *net, const char *cache)
{
    const std::string sig = signature(net);
    snn_launch best = net->launch;
    if (cache_lookup(cache, sig, &best)) return snn_set_launch(net, &best);
    const int64_t steps = 3 * kGraphSteps;
    double best_ms = 0.0;
    int rc = snn_time_steps(net, steps, &best_ms);   // also warms up
    if (rc) return rc;
    if ((rc = snn_time_steps(net, steps, &best_ms))) return rc;
    // modes: rows, tiles, fused (no plastic projections), grouped (some projection to group)
    int md[4] = {kModeRows, kModeTiles, 0, 0}, n_md = 2;
    if (!net->plastic) md[n_md++] = kModeFused;
    if (net->n_grp > 0) md[n_md++] = kModeGrouped;
    const int nb[] = {64, 128, 256, 512, 1024};
    const int pb[] = {256, 512, 1024, 2048, 4096, 8192};
    const int ck[] = {128, 256, 512, 1024, 2048};
    for (int dim = 0; dim < 4; ++dim) {
        const int *vals = dim == 0 ? md : dim == 1 ? nb : dim == 2 ? pb : ck;
        const int nv = dim == 0 ? n_md : dim == 1 ? 5 : dim == 2 ? 6 : 5;
        snn_launch cur_best = best;
        for (int k = 0; k < nv; ++k) {
            snn_launch L = best;
            if (dim == 0) L.mode = vals[k];
            if (dim == 1) L.neuron_block = vals[k];
            if (dim == 2) L.prop_blocks = vals[k];
            if (dim == 3) L.chunk = vals[k];
            if ((rc = snn_set_launch(net, &L))) return rc;
            double ms = 0.0;
            if ((rc = snn_time_steps(net, steps, &ms))) return rc;
            if (ms < best_ms) {
                best_ms = ms;
                cur_best = L;
            }
        }
        best = cur_best;
    }
    if ((rc = snn_set_launch(net, &best))) return rc;
    cache_store(cache, sig, best);
    return SNN_OK;
}
