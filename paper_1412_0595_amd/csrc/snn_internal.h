// Device-side tables of the spiking-network library, shared by the host
// runtime (snn_runtime.hip) and the kernels (snn_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snn {

constexpr int kWave = 64;
constexpr int kMaxIn = 4;    // incoming projections of one population
constexpr int kMaxOut = 8;   // outgoing projections of one population
constexpr int kMaxTr = 4;    // STDP traces kept by one population
constexpr int kMaxLtp = 2;   // plastic projections arriving at one population
constexpr int kMinChunk = 64;
constexpr int kTileMax = 1024;  // post neurons per propagation tile (LDS accumulator width)
constexpr int kPropWaves = 4;   // wavefronts per propagation block (one LDS tile copy each)
constexpr int kMinGroups = 16;  // groups (partial tiles) per (projection, post tile) at least
constexpr int kRowsPerGroup = 16;  // spiking rows per group aimed for when more groups are allowed

// Active spike words of a pre population are processed in groups of
// consecutive active-list slots: with na active words and `rows` spiking
// rows at the previous step, a group holds ceil(na / n_groups) words, where
// n_groups = clamp(rows / kRowsPerGroup, kMinGroups, words).  Each group
// leaves one partial tile; a reduction pass after the propagation adds the
// groups' partials of each tile into G.  The neuron update applies this rule
// to the previous step's counts when it emits the work of a step (only a
// group's first word emits items) and records the choice per population.
__host__ __device__ inline uint32_t group_words(uint32_t na, uint32_t rows, uint32_t words)
{
    uint32_t g = rows / kRowsPerGroup;
    if (g < (uint32_t)kMinGroups) g = kMinGroups;
    if (g > words) g = words;
    if (g < 1) g = 1;
    const uint32_t gw = (na + g - 1) / g;
    return gw < 1 ? 1 : gw;
}

// Conductances are signed 64-bit multiples of 2^-40 uS.  Integer addition
// is associative, so the sum of a step's deliveries does not depend on the
// order in which atomics land; the grid is far finer than fp32.
constexpr double kFixOne = 1099511627776.0;          // 2^40
constexpr double kFixInv = 1.0 / 1099511627776.0;    // 2^-40

enum { kPoisson = 0, kHH = 1, kIzh = 2 };

// Delivery strategies (bitwise the same result; chosen by measurement):
// rows = a work item per chunk of a spiking row, 64-bit atomics into G;
// tiles = a work item per (projection, post tile, group of active spike
// words), LDS tile accumulation, partial tiles added into G by a reduction.
enum { kModeRows = 0, kModeTiles = 1, kModeFused = 2, kModeGrouped = 3 };
// grouped = rows, except that every non-plastic projection onto at most
// kGrpTile post neurons, with at most kGrpDense of its (pre, post) pairs
// connected and rows of fewer than kGrpSyn / 2 synapses on average, is
// delivered in groups of its spiking rows (found in order in the pre
// population's spike words), k rows per group with k = kGrpSyn / (mean row
// length), at most kGrpRows: a wavefront sums a group's synapses in its own
// LDS tile of the post population and adds the tile's nonzero entries into G
// with atomics, a few atomics per post neuron and group instead of one per
// synapse.  Denser or longer rows already put several synapses in each
// atomic transaction, and their groups would be long serial walks.
// kGrpSlots wavefronts per such projection take its groups in turn.  Its
// row items (still emitted by the neuron update) are skipped.
constexpr int kGrpTile = 1024;
constexpr int kGrpRows = 6;
constexpr int kGrpSyn = 1536;
constexpr double kGrpDense = 0.6;
constexpr int kGrpSlots = 16;
// fused = no propagation kernel: each neuron-update block delivers its own
// spikes' rows with 64-bit atomics into the delivery buffer D of the next
// step (double-buffered), which the next update adds to G (networks without
// plasticity).
constexpr int kFusedCap = 512;     // chunks a block lists in LDS per round
// Tile mode, dense activity: when at least kPullNum/kPullDen of a population
// spiked, its non-plastic projections are delivered by pulling instead.  Each
// such projection keeps a column-ordered copy in sliced-ELL form with
// compressed row indices: a column's entries in ascending row order, each a
// one-byte row delta (to the previous entry's row; the first entry's delta is
// 0) and its fp32 weight, a gap of more than kPullMaxDelta rows bridged by
// weight-0 entries of delta kPullMaxDelta.  Columns are sorted by encoded
// length, 64 to a slice; lane l of a slice holds the l-th column.  Entries go
// in packets of four per lane: packet p of a slice is one float4 of weights
// at (slice packet base + p) * 64 + l and one word of four byte deltas at the
// same index; short columns are padded with (delta 0, weight 0) to the
// slice's depth, a multiple of 4.  A pull unit is up to kPullDepth
// consecutive entries of one slice: one wavefront, one lane per column,
// starting from its lane's row before the unit's first entry (a table of 64
// rows per unit), summing the weights of spiking rows.  5 bytes per entry
// instead of the CSR's 8.  The unit of a slice of one depth chunk adds its
// sums into G itself, one plain read-modify-write per column (no other work
// touches a pulled projection's conductances in that step); the units of
// deeper slices store one partial sum per column (a coalesced store) and the
// reduction adds them into G in groups of up to 64 units per wavefront: a
// plain read-modify-write per column when one group covers the slice, else
// one atomic per group and column.  A projection whose bridging entries would
// exceed a quarter of its synapses gets no copy (it is always pushed).
constexpr int kPullNum = 7, kPullDen = 8;
constexpr int kPullDepth = 64;
constexpr int64_t kPullUnitsMin = 32768;   // pull units of all copies together, at least (unit depth choice)
constexpr int kPullMaxDelta = 255;

struct PullUnit {
    int64_t pk0;        // the unit's first packet (global packet index; lane 0)
    int64_t g_base;     // conductance pool offset of the projection
    int32_t col_off;    // offset of the slice's 64 post neurons in the column table
    int32_t npk;        // packets (4 entries each) per lane, <= 4 kPullDepth / 4
    int32_t pre_seg;    // pre population, and of it:
    int32_t inst;       //   instance (g_scale),
    int32_t wbase;      //   first spike word (global word index),
    int32_t nwords;     //   spike words
    int32_t direct;     // 1: the slice's only unit, which adds its sums into G
    int32_t ncols;      // post neurons in the slice (64 but in a projection's last slice)
};

struct PullSlice {       // one reduction group of a slice
    int64_t g_base;     // conductance pool offset of the projection
    int32_t u0;         // its first pull unit (the others follow, one per depth chunk)
    int32_t n_units;    // <= 64
    int32_t col_off;    // offset of the slice's 64 post neurons in the column table
    int32_t pre_seg;
    int32_t atomic;     // 1: other groups share the slice's columns
    int32_t pad_;
};

// One population of one instance; its neurons occupy the global ids
// [base, base + n), base a multiple of 64, so a wavefront never spans two.
struct Seg {
    int32_t kind, n;
    int64_t base;
    int32_t inst, pop;
    int32_t n_in, n_out, n_tr, n_ltp;
    // incoming projections: id, conductance array, reversal, decay per step
    int32_t in_proj[kMaxIn];
    int64_t in_G[kMaxIn];
    double in_erev[kMaxIn];
    double in_decay[kMaxIn];
    // outgoing projections: id, row-start array (pool offset), post tiles
    int32_t out_proj[kMaxOut];
    int64_t out_rp[kMaxOut];
    int32_t pullable;   // 1: it has outgoing non-plastic projections (tile mode may pull them)
    int32_t pad3_;
    int32_t out_tiles[kMaxOut];
    // plastic projections arriving here: id and column-start array
    int32_t ltp_proj[kMaxLtp];
    int64_t ltp_cp[kMaxLtp];
    // STDP traces owned by this population: pool offset and decay per step
    int64_t tr_base[kMaxTr];
    float tr_decay[kMaxTr];
    // Poisson
    uint64_t thresh;   // fires iff Philox word < thresh (thresh may be 2^32)
    uint64_t seed;
    // Traub-Miles (i_ext also for Izhikevich)
    double gna, ena, gk, ek, gl, el, inv_c, i_ext;
    int32_t record_vbar;
    int32_t pad_;
    // Izhikevich: offset of the population's (a, b, c, d) in the parameter pool
    int64_t izp_base;
};

struct Proj {
    int32_t pre_seg, post_seg;
    int32_t n_pre, n_post;
    int32_t inst, stdp;
    int64_t rp_base;    // row_ptr pool offset (n_pre + 1 local offsets)
    int64_t syn_base;   // col_idx / weight pool offset
    int64_t nnz;
    int64_t G_base;     // conductance pool offset (n_post)
    // post tiles: tile_w posts each (a multiple of 64, <= kTileMax); with
    // more than one tile, tp_base locates n_pre x (n_tiles + 1) tile starts
    // (row-local CSR offsets of the first column >= tile * tile_w)
    int32_t tile_w, n_tiles;
    int64_t tp_base;    // -1: one tile, the row pointers bound it
    int64_t P_base;     // partial pool offset: [tile][group][tile_w] int64
    int64_t pull_base;  // first slice of the column-ordered copy (non-plastic), else -1
    int64_t F_base;     // partial flag offset: [tile][group] bytes (1: a partial tile was written)
    int32_t pre_words;  // spike words of the pre population (ceil(n_pre / 64))
    int32_t grp;        // 1: delivered in row groups in grouped mode
    // STDP
    float a_plus_gmax, a_minus_gmax, g_max, pad_;
    int64_t x_base, y_base;    // trace pool offsets (pre n_pre, post n_post)
    int64_t cp_base;           // column-start pool offset (n_post + 1)
    int64_t csc_base;          // row-of / position pool offset (nnz)
};

// Counters the kernels hand to each other from step to step.  Each kernel
// reads one step field and writes the other, so no kernel reads a field
// that one of its own blocks writes.
struct StepState {
    int64_t t_prop;      // step index seen by propagation / potentiation
    int64_t t_neuron;    // step index seen by the neuron update
    uint32_t qcnt[2];    // host-built propagation work items at the start of slot t & 1
    uint32_t lcnt[2];    // potentiation work items produced at step t
    uint32_t overflow;   // set if a queue would have overflowed (never expected)
    uint32_t fdone;      // fused mode: buckets of blocks of the running update that finished
    uint32_t npull[2];   // tile mode: populations to pull, per step slot
    uint32_t grp_off[2]; // grouped mode: 1 = the grouped deliveries of S(t-1) in slot t & 1 are already made
                         // (the host emptied the queues), so the groups skip that slot
};
// Largest total of neurons (each population padded to a multiple of 64):
// byte offsets into the 8-byte per-neuron arrays stay below 2^32.
constexpr int64_t kMaxNeuronsPadded = int64_t(1) << 29;

// Work-queue reservation.  The neuron update reserves queue space once per
// block; one returning atomic per block on a single counter serialises the
// whole grid (about 11 ns each on the MI355X: 8 400 blocks take 97 us), so
// block b reserves on counter b mod kQBuckets, the counters 4 KiB apart.
// Bucket x owns a fixed range of each queue slot, sized to the worst case of
// its blocks (every neuron spiking; rows: every outgoing row in chunks of
// kMinChunk, tiles: one item per outgoing projection and post tile), for the
// current block size and mode.  Host-built work (after a mode switch or
// spikes set from the host) sits contiguously at the start of a slot with
// its own count (StepState::qcnt) and empty buckets.
constexpr int kQBuckets = 64;
constexpr int kQBucketStride = 1024;   // uint32 words between two bucket counters

// A work item.  Row mode: synapses [k0, k1) of row `row` of projection
// `proj`, whose instance is `aux` (so that its g_scale is read alongside
// the projection record).  Tile mode: projection `proj`, post tile k0, spike word
// `row` of the pre population (64 pre neurons) with its bits, and the
// word's slot k1 in the active list (the item of a group's first slot
// processes the group).  Potentiation: synapses
// [k0, k1) of the column of post neuron `row` of plastic projection `proj`.
struct Item {
    int32_t proj, row, k0, k1;
    uint64_t bits;      // propagation: the spike word itself
    uint64_t aux;       // row mode: instance of the projection
};

struct NeuronArgs {
    const Seg *segs;
    const int32_t *wave_seg;
    int64_t n_waves;
    float *vh, *vl, *mh, *ml, *hh, *hl, *nh, *nl;
    int64_t *G;
    int32_t *counts;
    double *vsum;
    int32_t *nan_count;      // per instance
    uint64_t *bits;          // 2 slots of n_waves words
    uint64_t *raster;        // raster_steps slots of n_waves words, or null
    int32_t raster_steps;
    float *trace;
    const Proj *projs;
    const int32_t *rp_pool;
    const int32_t *cp_pool;
    Item *queue;             // 2 slots of qcap
    int64_t qcap;
    uint32_t *qb_cnt;        // [3][kQBuckets] counters kQBucketStride apart: reservations of the two
                             // queue slots, the fused update's per-bucket done counts
    const int64_t *qb_base;  // kQBuckets + 1 bucket offsets into a queue slot
    Item *lqueue;            // 2 slots of lcap
    int64_t lcap;
    int32_t chunk;
    int32_t substeps;
    double hs;               // dt / substeps
    StepState *st;
    int32_t mode;            // kModeRows / kModeTiles / kModeFused (grouped mode runs as rows)
    int64_t *D;              // fused: [2][G pool] deliveries for the next update
    int64_t G_count;
    const int32_t *col_pool;
    const float *w_pool;
    const float *gscale;
    uint32_t *gwsel;         // [2][n_segs]  words per group chosen at emission
    uint32_t *pullf;         // [2][n_segs]  1: the population's projections are pulled
    uint32_t *awcnt;         // [2][n_segs]  per step slot and population: spike words that held a spike
    uint32_t *scnt;          // [2][n_segs]  spikes
    int32_t *awl;            // [2][n_waves] which words, at the population's own word offset
    int32_t n_segs;
    const float4 *izp;       // Izhikevich (a, b, c, d) per neuron, at Seg::izp_base + index
    int32_t feat;            // kFeat* bits: what the network's populations use
};

// What a network's populations use beyond Traub-Miles and Poisson neurons;
// the neuron update is instantiated per combination, so a network without
// them runs none of their code and holds none of their values.
constexpr int kFeatIzh = 1;       // Izhikevich populations
constexpr int kFeatPlastic = 2;   // STDP traces and potentiation work
constexpr int kFeatRec = 4;       // voltage sums recorded for the adjoint's loss

struct PropArgs {
    int32_t mode;
    const Proj *projs;
    const Seg *segs;
    const Item *queue;
    int64_t qcap;
    const uint32_t *qb_cnt;  // [2][kQBuckets] items reserved in each bucket, kQBucketStride apart
    const int64_t *qb_base;  // kQBuckets + 1 bucket offsets into a queue slot
    const int32_t *rp_pool;
    const int32_t *tp_pool;
    const int32_t *col_pool;
    float *w_pool;
    const float *gscale;     // per instance
    int64_t *partial;
    uint8_t *pflag;
    int64_t *G;              // sparse items add here directly
    const uint64_t *bits;    // 2 slots of n_waves spike words
    int64_t n_waves;
    const float *trace;
    StepState *st;
    uint32_t *awcnt;         // [2][n_segs], the slot of this step is cleared here
    uint32_t *scnt;          // [2][n_segs], likewise
    const int32_t *awl;      // [2][n_waves]
    const uint32_t *gwsel;   // [2][n_segs]  words per group of each pre population
    uint32_t *pullf;         // [2][n_segs]  pull flags (the slot of this step is cleared here)
    int32_t n_segs;
    int32_t n_inst;
    const int4 *units;       // tile mode: reduction units (projection, tile, first column, first group)
    int64_t n_units;
    const PullUnit *pull_units;
    int64_t n_pull_units;
    int64_t *pull_part;      // [unit][64] partial sums of the pull units
    const PullSlice *pull_slices;
    int64_t n_pull_slices;
    const int32_t *pull_col; // [slice][64] post neuron of each lane, -1 for padding
    const float4 *pull_w;    // sliced-ELL weights, [packet][64 lanes] x 4 entries
    const uint32_t *pull_d;  // their row deltas, [packet][64 lanes], one byte per entry
    const int32_t *pull_r0;  // [unit][64] lane's row before the unit's first entry
    const int2 *grp_proj;    // grouped mode: (projection, rows per group) of those delivered in groups
    int64_t n_grp;           // 0 unless grouped mode
};

struct LtpArgs {
    const Proj *projs;
    const Item *lqueue;
    int64_t lcap;
    const int32_t *csc_row;  // pre index of each column entry
    const int32_t *csc_pos;  // CSR position of each column entry
    float *w_pool;
    const float *trace;
    StepState *st;
};

// Reverse-time adjoint of one population's time-averaged voltage with the
// spike raster held fixed (snn_adjoint.hip).  Loss neurons are numbered
// compactly, instance-major: instance b owns [loss_base[b], loss_base[b+1]).
constexpr int kAdjMaxSub = 8;       // substeps the reverse pass keeps in registers
constexpr int kAdjMaxLoss = 1024;   // loss neurons per instance (one block each)

struct AdjArgs {
    const Seg *segs;
    const Proj *projs;
    int32_t n_inst;
    const int32_t *loss_seg;     // per instance
    const int64_t *loss_base;    // per instance + 1
    const int32_t *loss_owner;   // per loss neuron: its instance
    int64_t n_loss;
    int32_t n_in_max;
    const uint64_t *raster;      // [T][n_waves] spike bitmask of the recorded steps
    int64_t n_waves;
    int64_t T;
    int64_t n_pad;               // padded neuron count (stride of the state arrays)
    const float *ckpt_state;     // checkpoint of this segment: 8 state arrays
    const int64_t *ckpt_G;       // and the conductance pool
    const float *next_state;     // checkpoint of the next segment (self-check) or null
    const int64_t *next_G;
    uint32_t *mismatch;
    int64_t t_a;                 // first step of the segment
    int32_t K;                   // steps in the segment
    const int32_t *rp_pool;
    const int32_t *col_pool;
    const float *w_pool;
    const float *gscale;
    double *tape_x;              // [K][4][n_loss]   state at the start of each step
    double *tape_g;              // [K][n_in_max][n_loss]  delivered conductance (uS)
    double *lam;                 // [4 + n_in_max][n_loss]  adjoint carried across segments
    double *lg;                  // [K][n_in_max][n_loss]   adjoint of the delivered conductance
    const double *dvbar;         // [n_loss]  dL / dVbar
    int32_t substeps;
    double hs;
    const int4 *gitems;          // gather work: (instance, input slot, pre segment, bitmask word)
    int64_t n_gitems;
    float *dg;                   // [total synapses] dL / dg, weight-pool order
    double *ds;                  // [n_inst] dL / dg_scale
};

hipError_t launch_adj_recompute(const AdjArgs &a, int block, hipStream_t s);
hipError_t launch_adj_reverse(const AdjArgs &a, hipStream_t s);
hipError_t launch_adj_gather(const AdjArgs &a, hipStream_t s);
hipError_t launch_gather_vbar(const Seg *segs, const int32_t *loss_seg, const int64_t *loss_base,
                              const int32_t *loss_owner, int64_t n_loss, const double *vsum, double inv_T,
                              double *vbar, hipStream_t s);

// Launchers (snn_kernels.hip).
hipError_t launch_neuron(const NeuronArgs &a, int block, hipStream_t s, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
hipError_t launch_propagate(const PropArgs &a, int blocks, int block, hipStream_t s, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr);
hipError_t launch_potentiate(const LtpArgs &a, int blocks, int block, hipStream_t s, hipEvent_t e0 = nullptr,
                             hipEvent_t e1 = nullptr);
hipError_t launch_gather_weights(const float *w, const int32_t *perm, float *out, int64_t n, hipStream_t s);
// Zero `bytes` (a multiple of 4) at p with a kernel.
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_check_weights(const float *w, const Proj *projs, int32_t n_projs, int64_t max_nnz, uint32_t *flag,
                                uint32_t *wmax, hipStream_t s);


// Records msg as the calling thread's last error (snn_last_error) and
// returns code; for host routines that keep no net.
int set_error(int code, const char *msg);

}  // namespace snn
