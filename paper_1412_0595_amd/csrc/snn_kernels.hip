// Step kernels of the spiking-network library, written for gfx950 (wave64).
//
//  k_neuron     one lane per neuron: Traub-Miles update (Section 2: HH at
//               discrete time steps) or Poisson draw, upward-crossing spike
//               test, wavefront ballot into the spike bitmask, and compaction
//               (wave scan + LDS block offsets + one atomic per block) of the
//               propagation work of the next step.  In fused mode the block
//               instead delivers its own spikes' rows (fused_delivery).
//  k_propagate_rows  (sparse activity) persistent grid, one wavefront per
//               chunk of a spiking row; 64-bit atomics into G.  In grouped
//               mode wavefronts first take groups of a few spiking rows of
//               each projection onto a small post population, sum them in an
//               LDS tile and add its nonzero entries into G.
//  k_propagate_tiles (dense activity) persistent grid of independent
//               wavefronts, one per work item = (projection, post tile, group
//               of active 64-neuron spike words of the pre population; only a
//               group's first word emits).  The wavefront walks the row slices
//               of the group's spiking rows in the Compressed Row Storage
//               arrays (Section 3), packed several rows to a batch of loads,
//               adds the weights into its own LDS tile (columns within a row
//               are distinct, so no atomics) and writes the tile out as the
//               group's partial.  A population with at least 7/8 of its
//               neurons spiking is pulled instead: after their items the
//               wavefronts take units of the sliced-ELL column copies of its
//               non-plastic projections, one lane per post neuron.
//  k_reduce_partials  (tile mode) adds the groups' partial tiles, and the
//               pull units' partial sums of deep slices, into G.
//  k_gather_weights, k_check_weights  weight-pool maintenance (refresh of
//               the column copies; finiteness and per-projection maxima).
//  k_potentiate persistent grid, one wavefront per slice of the column of a
//               post neuron that spiked (STDP potentiation).
//
// Conductances are int64 multiples of 2^-40 uS, so integer sums of the
// deliveries are the same in any order and in every delivery mode.
#include <algorithm>
#include <hip/hip_ext.h>

#include "snn_device.h"

namespace snn {

__device__ __forceinline__ void slice_to_global(unsigned long long *G, const int32_t *col, const float *w,
                                                int32_t k0, int32_t k1, double s, int lane);

// ---------------------------------------------------------------------------
// Fused delivery (end of the neuron update): the block lists the chunks of
// its spiking neurons' outgoing rows in LDS (rounds of kFusedCap chunks; the
// chunk count of the block is uniform, so every thread passes the same
// barriers), its wavefronts take chunks from an LDS counter and add them with
// 64-bit atomics into the delivery buffer of step t + 1.  Then each block
// counts itself done; the last one advances the step counters, once every
// block has read them (no block waits for another).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fused_delivery(const NeuronArgs &a, int64_t t, uint32_t (*s_woff)[2],
                                               uint32_t &s_tot, uint32_t &s_pop, int4 *s_fl, int sidx, int32_t j,
                                               uint32_t nq, uint32_t iq, int wid, int lane, int32_t ra0,
                                               int32_t ra1, int32_t rb0, int32_t rb1)
{
    const uint32_t total = s_tot;
    const int64_t dnext = (int64_t)((t + 1) & 1) * a.G_count;
    const int32_t ch = a.chunk;
    for (uint32_t r0 = 0; r0 < total; r0 += kFusedCap) {
        if (nq) {
            const Seg &S = a.segs[sidx];
            uint32_t pos = s_woff[wid][0] + (iq - nq);      // this lane's first chunk in the block
            auto list = [&](int o, int32_t q0, int32_t q1) {
                for (int32_t k = q0; k < q1; k += ch, ++pos)
                    if (pos >= r0 && pos < r0 + (uint32_t)kFusedCap)
                        s_fl[pos - r0] = make_int4(S.out_proj[o], k, min(k + ch, q1), 0);
            };
            if (S.n_out > 0) list(0, ra0, ra1);
            if (S.n_out > 1) list(1, rb0, rb1);
            for (int o = 2; o < S.n_out; ++o) {
                const int32_t *rp = a.rp_pool + S.out_rp[o];
                list(o, rp[j], rp[j + 1]);
            }
        }
        if (threadIdx.x == 0) s_pop = 0;
        __syncthreads();
        const uint32_t n_round = min((uint32_t)kFusedCap, total - r0);
        for (;;) {
            uint32_t idx = 0;
            if (lane == 0) idx = atomicAdd(&s_pop, 1u);
            idx = (uint32_t)__builtin_amdgcn_readfirstlane(idx);
            if (idx >= n_round) break;
            const int32_t proj = __builtin_amdgcn_readfirstlane(s_fl[idx].x);
            const int32_t k0 = __builtin_amdgcn_readfirstlane(s_fl[idx].y);
            const int32_t k1 = __builtin_amdgcn_readfirstlane(s_fl[idx].z);
            const Proj &P = a.projs[proj];
            slice_to_global((unsigned long long *)(a.D + dnext + P.G_base), a.col_pool + P.syn_base,
                            a.w_pool + P.syn_base, k0, k1, (double)a.gscale[P.inst] * kFixOne, lane);
        }
        __syncthreads();
    }
    // done counts in two levels, so that no address takes one returning
    // atomic per block: the last block of bucket blockIdx mod kQBuckets
    // (counters of the third bucket slot, 4 KiB apart) counts its bucket
    // done, the last bucket advances the step counters
    if (threadIdx.x == 0) {
        const uint32_t x = blockIdx.x % kQBuckets;
        const uint32_t in_x = (gridDim.x - 1u - x) / kQBuckets + 1u;   // blocks of bucket x
        uint32_t *c = a.qb_cnt + ((int64_t)2 * kQBuckets + x) * kQBucketStride;
        if (atomicAdd(c, 1u) == in_x - 1u) {
            *c = 0u;
            const uint32_t buckets = min(gridDim.x, (uint32_t)kQBuckets);
            if (atomicAdd(&a.st->fdone, 1u) == buckets - 1u) {
                a.st->fdone = 0;
                a.st->t_prop = t + 1;
                a.st->t_neuron = t + 1;
            }
        }
    }
}

// Element at a 32-bit byte offset from a wave-uniform base: the address is
// the base (scalar registers) plus the offset (one vector register), so the
// loads and stores of several arrays at the same index share one register
// instead of holding a 64-bit address each.
template <class T>
__device__ __forceinline__ T ld_at(const T *base, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}
template <class T>
__device__ __forceinline__ void st_at(T *base, uint32_t off, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off) = v;
}
// A conductance array of one projection (pool + offset), kept in scalar
// registers.
__device__ __forceinline__ int64_t *gbase(int64_t *pool, int64_t off)
{
    return reinterpret_cast<int64_t *>(uniform_u64(reinterpret_cast<uint64_t>(pool + off)));
}
__device__ __forceinline__ double pair_at(const float *hi, const float *lo, uint32_t off)
{
    return (double)ld_at(hi, off) + (double)ld_at(lo, off);
}
__device__ __forceinline__ void split_at(double x, float *hi, float *lo, uint32_t off)
{
    const float h = (float)x;
    st_at(hi, off, h);
    st_at(lo, off, (float)(x - (double)h));
}

// ---------------------------------------------------------------------------
// Neuron update + spike compaction
// ---------------------------------------------------------------------------
// One instantiation per delivery mode (uniform over a launch) and per set of
// population features (kFeat*, fixed at create), so that each carries only
// the code and the kernel arguments its network needs.  The plain Traub-Miles
// instantiations are held to 96 VGPRs, five wavefronts per SIMD: their state
// is addressed as one 32-bit offset from uniform bases (ld_at/st_at), and the
// two 8-byte spills this leaves sit outside the substep loop.
template <int MODE, int FEAT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(FEAT == 0 ? 5 : 4, 8)))
void k_neuron(NeuronArgs a)
{
    __shared__ uint32_t s_woff[16][2];
    __shared__ uint32_t s_base[2];
    __shared__ uint32_t s_tot, s_pop;            // fused: chunks of the block, next to take
    __shared__ int4 s_fl[MODE == kModeFused ? kFusedCap : 1];   // fused: (projection, k0, k1, -) per chunk

    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // uniform: scalar loads below
    const int nwb = blockDim.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * nwb + wid;
    const int64_t t = a.st->t_neuron;
    const int cur = (int)(t & 1);

    bool spike = false;
    uint32_t nq = 0, nl = 0;       // work items this lane emits
    uint32_t wslot = 0;            // slot of this wave's word in the active list
    uint64_t wball = 0;            // this wave's spike word
    int32_t j = 0;
    int32_t ra0 = 0, ra1 = 0, rb0 = 0, rb1 = 0;   // rows of outgoing projections 0 and 1 (spiking lanes)
    float trv[kMaxTr] = {};        // prefetched traces

    // The population record's fields that the update reads, loaded together
    // before the first branch: one round trip (read at first use, behind
    // branches, each would cost one).  Waves past the last neuron read the
    // last wave's record and store nothing.
    const int sidx = __builtin_amdgcn_readfirstlane(a.wave_seg[min(gw, a.n_waves - 1)]);
    const Seg &S = a.segs[sidx];
    constexpr bool kIzhOn = (FEAT & kFeatIzh) != 0, kPlastic = (FEAT & kFeatPlastic) != 0, kRec = (FEAT & kFeatRec) != 0;
    const int64_t s_b = S.base;
    const int32_t s_n = S.n, s_kind = S.kind, s_nout = S.n_out, s_nin = S.n_in;
    const int32_t s_ntr = kPlastic ? S.n_tr : 0, s_nltp = kPlastic ? S.n_ltp : 0, s_rec = kRec ? S.record_vbar : 0;
    const int32_t s_op0 = S.out_proj[0], s_op1 = S.out_proj[1], s_inst = S.inst;
    const int64_t s_rp0 = S.out_rp[0], s_rp1 = S.out_rp[1];
    int64_t s_inG[kMaxIn];
#pragma unroll
    for (int q = 0; q < kMaxIn; ++q) s_inG[q] = S.in_G[q];
    asm volatile("" ::"s"(s_b), "s"(s_n), "s"(s_kind), "s"(s_nout), "s"(s_nin));
    if constexpr (kPlastic) asm volatile("" ::"s"(s_ntr), "s"(s_nltp));
    if constexpr (kRec) asm volatile("" ::"s"(s_rec));
    asm volatile("" ::"s"(s_op0), "s"(s_op1), "s"(s_rp0), "s"(s_rp1), "s"(s_inG[0]), "s"(s_inG[1]), "s"(s_inG[2]),
                 "s"(s_inG[3]), "s"(s_inst));

    if (gw < a.n_waves) {
        const int64_t gid = gw * kWave + lane;
        j = (int32_t)(gid - s_b);
        const bool active = j < s_n;
        // Every load of the update is issued up front and unconditionally,
        // so that they share one memory round trip: padded arrays at gid,
        // unpadded ones (conductances, traces) at jj, the index clamped into
        // the population.  Lanes past the population compute on that data and
        // store nothing.  What only a spiking neuron needs (its spike count,
        // its outgoing row bounds) is read after the spike test, by the
        // spiking lanes alone.
        const int32_t jj = active ? j : s_n - 1;
#pragma unroll
        for (int q = 0; q < kMaxTr; ++q)
            if (q < s_ntr) trv[q] = a.trace[S.tr_base[q] + jj];

        // byte offsets of the lane's elements: padded state arrays at gid,
        // conductances at jj (stores at j), from wave-uniform bases (the
        // library keeps the padded neuron count below 2^29)
        const uint32_t o4 = (uint32_t)gid * 4u, o8 = (uint32_t)gid * 8u;
        const uint32_t g8 = (uint32_t)jj * 8u, s8 = (uint32_t)j * 8u;
        if (s_kind == kHH) {
            const double vs = s_rec ? ld_at(a.vsum, o8) : 0.0;
            double v = pair_at(a.vh, a.vl, o4);
            double m = pair_at(a.mh, a.ml, o4);
            double h = pair_at(a.hh, a.hl, o4);
            double n = pair_at(a.nh, a.nl, o4);
            const double v0 = v;
            // delivered conductance: in G (rows and tile modes), G plus this
            // step's slot of the delivery buffer (fused mode)
            const int64_t dcur = (int64_t)cur * a.G_count;
            int64_t g[kMaxIn];
#pragma unroll
            for (int q = 0; q < kMaxIn; ++q)
                if (q < s_nin) {
                    g[q] = ld_at(gbase(a.G, s_inG[q]), g8);
                    if constexpr (MODE == kModeFused) g[q] += ld_at(gbase(a.D, dcur + s_inG[q]), g8);
                }
            // synaptic current from the start-of-step voltage, held fixed
            // over the substeps; then the conductances decay
            const double iin = syn_current(S, g, v0);
            // the decayed conductances are stored before the substeps, so
            // that they are not held in registers across them
            if (active) {
#pragma unroll
                for (int q = 0; q < kMaxIn; ++q)
                    if (q < s_nin) {
                        st_at(gbase(a.G, s_inG[q]), s8, fix_decay(g[q], S.in_decay[q]));
                        if constexpr (MODE == kModeFused) st_at(gbase(a.D, dcur + s_inG[q]), s8, (int64_t)0);
                    }
            }
            const double hc = a.hs * S.inv_c;
            for (int k = 0; k < a.substeps; ++k) hh_substep(S, a.hs, hc, iin, v, m, h, n);
            if (active) {
                // the offset passes through an empty asm, so the compiler
                // forms the state addresses here instead of holding eight
                // 64-bit addresses across the substeps
                uint32_t os = o4;
                asm volatile("" : "+v"(os));
                spike = (v0 < 0.0) && (v >= 0.0);
                split_at(v, a.vh, a.vl, os);
                split_at(m, a.mh, a.ml, os);
                split_at(h, a.hh, a.hl, os);
                split_at(n, a.nh, a.nl, os);
                if (fits_fp32(v0) && !fits_fp32(v)) atomicAdd(&a.nan_count[s_inst], 1);
                if (s_rec) st_at(a.vsum, 2u * os, vs + v);
            }
        } else if (kIzhOn && s_kind == kIzh) {
            // Izhikevich: v in the V pair, u in the M pair, (a, b, c, d) from
            // the parameter pool; the same conductance handling as above
            const double vs = s_rec ? a.vsum[gid] : 0.0;
            double v = pair_load(a.vh, a.vl, gid);
            double u = pair_load(a.mh, a.ml, gid);
            const float4 pr = a.izp[S.izp_base + jj];
            const double v0 = v;
            const int64_t dcur = (int64_t)cur * a.G_count;
            int64_t g[kMaxIn];
#pragma unroll
            for (int q = 0; q < kMaxIn; ++q)
                if (q < s_nin) {
                    g[q] = a.G[s_inG[q] + jj];
                    if constexpr (MODE == kModeFused) g[q] += a.D[dcur + s_inG[q] + jj];
                }
            const double iin = syn_current(S, g, v0);
            for (int k = 0; k < a.substeps; ++k) izh_substep((double)pr.x, (double)pr.y, a.hs, iin, v, u);
            if (active) {
#pragma unroll
                for (int q = 0; q < kMaxIn; ++q)
                    if (q < s_nin) {
                        a.G[s_inG[q] + j] = fix_decay(g[q], S.in_decay[q]);
                        if constexpr (MODE == kModeFused) a.D[dcur + s_inG[q] + j] = 0;
                    }
                // threshold on the step's end value, then the reset
                spike = v >= kIzhPeak;
                if (fits_fp32(v0) && !fits_fp32(v)) atomicAdd(&a.nan_count[s_inst], 1);
                if (spike) {
                    v = (double)pr.z;
                    u = u + (double)pr.w;
                }
                pair_split(v, a.vh[gid], a.vl[gid]);
                pair_split(u, a.mh[gid], a.ml[gid]);
                if (s_rec) a.vsum[gid] = vs + v;
            }
        } else {
            if (active) {
                const uint32_t w = philox_first_word((uint32_t)j, (uint32_t)((uint64_t)t & 0xffffffffu),
                                                     (uint32_t)((uint64_t)t >> 32), (uint32_t)S.pop,
                                                     (uint32_t)(S.seed & 0xffffffffu), (uint32_t)(S.seed >> 32));
                spike = (uint64_t)w < S.thresh;
            }
        }

        const uint64_t ball = __ballot(spike);
        wball = ball;
        if (lane == 0) {
            a.bits[(int64_t)cur * a.n_waves + gw] = ball;
            if (a.raster) a.raster[(t % a.raster_steps) * a.n_waves + gw] = ball;
        }
        if (active) {
#pragma unroll
            for (int q = 0; q < kMaxTr; ++q)
                if (q < s_ntr) a.trace[S.tr_base[q] + j] = trv[q] * S.tr_decay[q] + (spike ? 1.0f : 0.0f);
        }
        if (MODE == kModeTiles && ball != 0) {
            // the word is active: record it, and queue one propagation item
            // per (outgoing projection, post tile) for the next step
            if (lane == 0) {
                const uint32_t words = (uint32_t)((s_n + kWave - 1) / kWave);
                wslot = atomicAdd(&a.awcnt[cur * a.n_segs + sidx], 1u);
                // a slot beyond the population's word count can only come
                // from repeating one step's update (kernel timing): no items
                if (wslot < words) {
                    a.awl[(int64_t)cur * a.n_waves + s_b / kWave + wslot] = (int32_t)(gw - s_b / kWave);
                    const uint32_t pc = (uint32_t)__popcll(ball);
                    const uint32_t before = atomicAdd(&a.scnt[cur * a.n_segs + sidx], pc);
                    // the wave that takes the population's spike count over
                    // the pull threshold marks the population for pulling
                    const uint32_t thr = (uint32_t)(((uint64_t)s_n * kPullNum + kPullDen - 1) / kPullDen);
                    if (S.pullable && before < thr && before + pc >= thr) {
                        a.pullf[cur * a.n_segs + sidx] = 1u;
                        atomicAdd(&a.st->npull[cur], 1u);
                    }
                    // words per group from the previous step's counts (the
                    // same for every wave of the population); only the first
                    // word of a group emits the group's items
                    const int pv = cur ^ 1;
                    const uint32_t gws = group_words(min(a.awcnt[pv * a.n_segs + sidx], words),
                                                     a.scnt[pv * a.n_segs + sidx], words);
                    a.gwsel[cur * a.n_segs + sidx] = gws;
                    if (wslot % gws == 0)
                        for (int o = 0; o < s_nout; ++o) nq += (uint32_t)S.out_tiles[o];
                }
            }
        }
        if (ball != 0 && spike) {
            a.counts[gid] += 1;
            const uint32_t ch = (uint32_t)a.chunk;
            if constexpr (MODE != kModeTiles) {
                // (a missing projection reads rp_pool[0..1])
                const int32_t *rpa = a.rp_pool + (s_nout > 0 ? s_rp0 + j : 0);
                const int32_t *rpb = a.rp_pool + (s_nout > 1 ? s_rp1 + j : 0);
                ra0 = rpa[0];
                ra1 = rpa[1];
                rb0 = rpb[0];
                rb1 = rpb[1];
                // one propagation item (fused: one chunk) per chunk of each
                // outgoing row
                if (s_nout > 0) nq += ((uint32_t)(ra1 - ra0) + ch - 1) / ch;
                if (s_nout > 1) nq += ((uint32_t)(rb1 - rb0) + ch - 1) / ch;
                for (int o = 2; o < s_nout; ++o) {
                    const int32_t *rp = a.rp_pool + S.out_rp[o];
                    nq += ((uint32_t)(rp[j + 1] - rp[j]) + ch - 1) / ch;
                }
            }
            for (int o = 0; o < s_nltp; ++o) {
                const int32_t *cp = a.cp_pool + S.ltp_cp[o];
                const uint32_t len = (uint32_t)(cp[j + 1] - cp[j]);
                nl += (len + ch - 1) / ch;
            }
        }
    }

    // Compaction: wave inclusive scans, per-wave offsets in LDS, one atomic
    // reservation per block and per queue.
    const uint32_t iq = wave_incl_sum(nq, lane);
    const uint32_t il = wave_incl_sum(nl, lane);
    if (lane == kWave - 1) {
        s_woff[wid][0] = iq;
        s_woff[wid][1] = il;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sq = 0, sl = 0;
        for (int w = 0; w < nwb; ++w) {
            const uint32_t tq = s_woff[w][0], tl = s_woff[w][1];
            s_woff[w][0] = sq;
            s_woff[w][1] = sl;
            sq += tq;
            sl += tl;
        }
        s_tot = sq;
        if constexpr (MODE != kModeFused) {
            // one reservation in this block's bucket (counters 4 KiB apart, so
            // the blocks' atomics do not queue on one address)
            const int x = (int)(blockIdx.x % kQBuckets);
            const int64_t qb0 = a.qb_base[x], qb1 = a.qb_base[x + 1];
            const uint32_t r = sq ? atomicAdd(&a.qb_cnt[((int64_t)cur * kQBuckets + x) * kQBucketStride], sq) : 0u;
            s_base[0] = (uint32_t)(qb0 + r);
            s_base[1] = sl ? atomicAdd(&a.st->lcnt[cur], sl) : 0u;
            if (sq && qb0 + (int64_t)r + sq > qb1) atomicOr(&a.st->overflow, 1u);
            if (sl && (int64_t)s_base[1] + sl > a.lcap) atomicOr(&a.st->overflow, 2u);
            if (blockIdx.x == 0) {
                a.st->qcnt[cur ^ 1] = 0;    // consumed by this step's propagation
                a.st->lcnt[cur ^ 1] = 0;
                a.st->grp_off[cur] = 0;     // this step's spikes are for the row groups to deliver
                a.st->t_prop = t + 1;
            }
        }
    }
    if constexpr (MODE != kModeFused) {
        // the buckets of the slot this step's propagation consumed
        if (blockIdx.x == 0 && threadIdx.x < kQBuckets)
            a.qb_cnt[((int64_t)(cur ^ 1) * kQBuckets + threadIdx.x) * kQBucketStride] = 0u;
    }
    __syncthreads();

    if (MODE == kModeRows && nq) {
        const int32_t ch = a.chunk;
        int64_t pos = (int64_t)s_base[0] + s_woff[wid][0] + (iq - nq);
        Item *qd = a.queue + (int64_t)cur * a.qcap;
        auto emit = [&](int32_t proj, int32_t r0, int32_t r1) {
            for (int32_t k = r0; k < r1; k += ch, ++pos)
                if (pos < a.qcap) qd[pos] = Item{proj, j, k, min(k + ch, r1), 0, (uint64_t)s_inst};
        };
        if (s_nout > 0) emit(s_op0, ra0, ra1);
        if (s_nout > 1) emit(s_op1, rb0, rb1);
        for (int o = 2; o < s_nout; ++o) {
            const int32_t *rp = a.rp_pool + S.out_rp[o];
            emit(S.out_proj[o], rp[j], rp[j + 1]);
        }
    }
    // tile mode: lane 0 counted the wave's items, all lanes write
    const uint32_t wave_nq = MODE == kModeTiles ? __shfl(nq, 0, kWave) : 0u;
    if (wave_nq) {
        const int64_t base = (int64_t)s_base[0] + s_woff[wid][0];
        const int32_t word = (int32_t)(gw - s_b / kWave);
        const int32_t slot = (int32_t)__shfl(wslot, 0, kWave);
        Item *qd = a.queue + (int64_t)cur * a.qcap;
        int32_t off = 0;
        for (int o = 0; o < s_nout; ++o) {
            const int32_t nt = S.out_tiles[o];
            for (int32_t tl = lane; tl < nt; tl += kWave) {
                const int64_t pos = base + off + tl;
                if (pos < a.qcap) qd[pos] = Item{S.out_proj[o], word, tl, slot, wball, 0};
            }
            off += nt;
        }
    }
    if (nl) {
        const int32_t ch = a.chunk;
        int64_t pos = (int64_t)s_base[1] + s_woff[wid][1] + (il - nl);
        Item *ld = a.lqueue + (int64_t)cur * a.lcap;
        for (int o = 0; o < s_nltp; ++o) {
            const int32_t *cp = a.cp_pool + S.ltp_cp[o];
            const int32_t k1 = cp[j + 1];
            for (int32_t k = cp[j]; k < k1; k += ch, ++pos)
                if (pos < a.lcap) ld[pos] = Item{S.ltp_proj[o], j, k, min(k + ch, k1), 0, 0};
        }
    }
    if constexpr (MODE == kModeFused) fused_delivery(a, t, s_woff, s_tot, s_pop, s_fl, sidx, j, nq, iq, wid, lane,
                                             ra0, ra1, rb0, rb1);
}

// A batch of up to kSlots slots of kWave consecutive synapses each, packed
// from the slices of one or more spiking rows of a spike word (a long slice
// spans several slots and batches).  Slot u holds CSR entries
// [sk[u], min(sk[u] + kWave, se[u])); all of a slot's fields are uniform.
// Slots of the same row form one phase (ph[u]); an unused slot has ph -1
// and repeats the last used slot's range, so its loads stay in bounds.
constexpr int kSlots = 8;

struct Batch {
    int32_t sk[kSlots], se[kSlots], ph[kSlots];
    int32_t nph;
};

// Fill the next batch from the row in progress [k, k1) and the spiking rows
// left in rem (lane r holds row r's slice bounds in b0, b1).  Returns false
// when nothing is left.
__device__ __forceinline__ bool fill_batch(Batch &B, uint64_t &rem, int32_t &k, int32_t &k1, int32_t b0, int32_t b1)
{
    int32_t nph = 0;
    bool fresh = true;              // the next used slot starts a new phase
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
        while (k >= k1 && rem) {
            const int r = __builtin_ctzll(rem);
            rem &= rem - 1;
            k = __builtin_amdgcn_readlane(b0, r);
            k1 = __builtin_amdgcn_readlane(b1, r);
            fresh = true;
        }
        if (k < k1) {
            if (fresh) ++nph;
            fresh = false;
            B.sk[u] = k;
            B.se[u] = k1;
            B.ph[u] = nph - 1;
            k += kWave;
        } else if (u > 0) {
            B.sk[u] = B.sk[u - 1];
            B.se[u] = B.se[u - 1];
            B.ph[u] = -1;
        } else {
            return false;
        }
    }
    B.nph = nph;
    return true;
}

// Loads of one batch: column (relative to the tile) and weight per slot, at
// indices clamped into the slot's row slice, so always in bounds.
struct BatchData {
    int32_t c[kSlots];
    float g[kSlots];
};

__device__ __forceinline__ void load_batch(BatchData &D, const Batch &B, const int32_t *col, const float *w,
                                           int32_t c0, int lane)
{
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
        // an unsigned 32-bit index lets the load use a scalar base and a
        // 32-bit lane offset (one VGPR per address instead of two)
        const uint32_t kk = (uint32_t)min(B.sk[u] + lane, B.se[u] - 1);
        D.c[u] = col[kk] - c0;
        D.g[u] = w[kk];
    }
}

// One row (phase) at a time, the tile entries are all read before the row's
// own are written: columns within one row are distinct, so this order is
// exact, and the phases run in program order, so rows sharing a column see
// each other's sums.  A clamped duplicate reads the same value and adds the
// same increment as its row's last entry, so it writes the identical sum.
__device__ __forceinline__ void batch_to_tile(long long *acc, const Batch &B, const BatchData &D, double s)
{
    long long inc[kSlots], v[kSlots];
#pragma unroll
    for (int u = 0; u < kSlots; ++u) inc[u] = fix_increment(s, D.g[u]);
    for (int32_t p = 0; p < B.nph; ++p) {
        // every slot is read, those of other phases at tile entry 0 (one
        // broadcast read; it keeps the reads free of branches), and only the
        // phase's own slots are written
#pragma unroll
        for (int u = 0; u < kSlots; ++u) v[u] = acc[B.ph[u] == p ? D.c[u] : 0];
#pragma unroll
        for (int u = 0; u < kSlots; ++u)
            if (B.ph[u] == p) acc[D.c[u]] = v[u] + inc[u];
    }
}

// Add the slices of a spike word's rows into the wavefront's LDS tile,
// software-pipelined over two explicit buffers: the loads of the next batch
// are in flight while the current batch is added (a register swap would make
// the compiler wait for them).  When there is no next batch, its buffer
// repeats the current ranges, so its loads stay in bounds and go unused.
__device__ __forceinline__ void word_to_tile(long long *acc, const int32_t *col, const float *w, uint64_t rem,
                                             int32_t b0, int32_t b1, int32_t c0, double s, int lane)
{
    int32_t k = 0, k1 = 0;
    Batch BA, BB;
    BatchData DA, DB;
    if (!fill_batch(BA, rem, k, k1, b0, b1)) return;
    load_batch(DA, BA, col, w, c0, lane);
    for (;;) {
        const bool more_b = fill_batch(BB, rem, k, k1, b0, b1);
        if (!more_b) BB = BA;
        load_batch(DB, BB, col, w, c0, lane);
        batch_to_tile(acc, BA, DA, s);
        if (!more_b) return;
        const bool more_a = fill_batch(BA, rem, k, k1, b0, b1);
        if (!more_a) BA = BB;
        load_batch(DA, BA, col, w, c0, lane);
        batch_to_tile(acc, BB, DB, s);
        if (!more_a) return;
    }
}

// The same walk for delivery straight into G with 64-bit atomics; a clamped
// duplicate must not add again, so the atomics are predicated, and the empty
// asm consumes the loaded registers so the compiler keeps all the loads ahead
// of the predicated atomics (nothing waits on an atomic without a return).
__device__ __forceinline__ void atomics_from_batch(unsigned long long *G, const int32_t *col, const float *w,
                                                   const int32_t *sk, const int32_t *se, const int32_t *ph, double s,
                                                   int lane)
{
    int32_t c[kSlots];
    float g[kSlots];
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
        const int32_t kk = min(sk[u] + lane, se[u] - 1);
        c[u] = col[kk];
        g[u] = w[kk];
    }
    asm volatile("" ::"v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]), "v"(c[7]),
                 "v"(g[0]), "v"(g[1]), "v"(g[2]), "v"(g[3]), "v"(g[4]), "v"(g[5]), "v"(g[6]), "v"(g[7]));
#pragma unroll
    for (int u = 0; u < kSlots; ++u)
        if (ph[u] >= 0 && sk[u] + lane < se[u]) atomicAdd(G + c[u], (unsigned long long)fix_increment(s, g[u]));
}

__device__ __forceinline__ void word_to_global(unsigned long long *G, const int32_t *col, const float *w, uint64_t rem,
                                               int32_t b0, int32_t b1, double s, int lane)
{
    int32_t k = 0, k1 = 0;
    Batch B;
    while (fill_batch(B, rem, k, k1, b0, b1)) atomics_from_batch(G, col, w, B.sk, B.se, B.ph, s, lane);
}

// Loads of one full-width batch of the slice [kb, kb + 8*64) ∩ [., k1), at
// indices clamped below k1 (always in bounds).
struct SliceData {
    int32_t c[kSlots];
    float g[kSlots];
};

__device__ __forceinline__ void load_slice(SliceData &D, const int32_t *col, const float *w, int32_t kb, int32_t k1,
                                           int lane)
{
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
        const int32_t k = min(kb + u * kWave + lane, k1 - 1);
        D.c[u] = col[k];
        D.g[u] = w[k];
    }
}

// The predicated atomics of a loaded batch; the empty asm consumes the loaded
// registers first, so the wait covers this batch's loads only (the next
// batch's, issued later, stay in flight).
__device__ __forceinline__ void slice_atomics(unsigned long long *G, const SliceData &D, int32_t kb, int32_t k1,
                                              double s, int lane)
{
    asm volatile("" ::"v"(D.c[0]), "v"(D.c[1]), "v"(D.c[2]), "v"(D.c[3]), "v"(D.c[4]), "v"(D.c[5]), "v"(D.c[6]),
                 "v"(D.c[7]), "v"(D.g[0]), "v"(D.g[1]), "v"(D.g[2]), "v"(D.g[3]), "v"(D.g[4]), "v"(D.g[5]),
                 "v"(D.g[6]), "v"(D.g[7]));
#pragma unroll
    for (int u = 0; u < kSlots; ++u)
        if (kb + u * kWave + lane < k1) atomicAdd(G + D.c[u], (unsigned long long)fix_increment(s, D.g[u]));
}

// One row slice [k0, k1) into G with atomics, in batches of 8 x 64 entries,
// software-pipelined over two explicit buffers: the next batch's loads are in
// flight while the current batch's atomics go out.  When there is no next
// batch its buffer reloads the current range (in bounds, unused).
__device__ __forceinline__ void slice_to_global(unsigned long long *G, const int32_t *col, const float *w,
                                                int32_t k0, int32_t k1, double s, int lane)
{
    if (k0 >= k1) return;
    constexpr int32_t kStep = kSlots * kWave;
    SliceData A, B;
    int32_t ka = k0;
    load_slice(A, col, w, ka, k1, lane);
    for (;;) {
        const int32_t kbn = ka + kStep;
        const bool more_b = kbn < k1;
        load_slice(B, col, w, more_b ? kbn : ka, k1, lane);
        slice_atomics(G, A, ka, k1, s, lane);
        if (!more_b) return;
        const int32_t kan = kbn + kStep;
        const bool more_a = kan < k1;
        load_slice(A, col, w, more_a ? kan : kbn, k1, lane);
        slice_atomics(G, B, kbn, k1, s, lane);
        if (!more_a) return;
        ka = kan;
    }
}

// Read-only tables of the propagation kernels, through the constant address
// space: nothing writes them while a kernel runs (the queue was filled by the
// step's neuron update, a previous dispatch), so the compiler may read them
// with scalar loads, several in one batch.
using CItem = const __attribute__((address_space(4))) Item;
using CProj = const __attribute__((address_space(4))) Proj;
using CFloat = const __attribute__((address_space(4))) float;
using CPullUnit = const __attribute__((address_space(4))) PullUnit;
using CPullSlice = const __attribute__((address_space(4))) PullSlice;
using CInt4 = const __attribute__((address_space(4))) int4;

// The work items of queue slot `prev` that wavefront g of nw takes: the nc
// contiguous host-built ones (g, g + nw, ...), then the reserved ones bucket
// by bucket.  With at least kQBuckets wavefronts, nw / kQBuckets of them
// share each bucket (wavefront g takes bucket g mod kQBuckets and its items
// g / kQBuckets, + nw / kQBuckets, ...); with fewer, wavefront g takes
// buckets g, g + nw, ... whole.  A count beyond its bucket's range (an
// overflow, flagged by the neuron update) is cut to the range.
template <class F>
__device__ __forceinline__ void visit_items(const PropArgs &a, int prev, uint32_t g, uint32_t nw, uint32_t nc, F &&f)
{
    using CU32 = const __attribute__((address_space(4))) uint32_t;
    using CI64 = const __attribute__((address_space(4))) int64_t;
    for (uint32_t it = g; it < nc; it += nw) f((int64_t)it);
    const uint32_t per = nw / kQBuckets;
    if (per && g >= kQBuckets * per) return;
    for (uint32_t x = per ? g % kQBuckets : g; x < (uint32_t)kQBuckets; x += per ? kQBuckets : nw) {
        const uint32_t cnt = ((CU32 *)a.qb_cnt)[((int64_t)prev * kQBuckets + x) * kQBucketStride];
        const int64_t b0 = ((CI64 *)a.qb_base)[x], b1 = ((CI64 *)a.qb_base)[x + 1];
        const int64_t n = min((int64_t)cnt, b1 - b0);
        for (int64_t k = per ? g / kQBuckets : 0; k < n; k += per ? per : 1) f(b0 + k);
    }
}

// Grouped delivery.  Wavefront slot j of grouped projection p takes groups
// j, j + kGrpSlots, ... of p's spiking rows, a group being p's k consecutive
// rows in the order of the pre population's step t - 1 spike words.  One pass over the words (64 per round, one per lane) counts the
// rows; lane r of a group holds its row r, found from the round's inclusive
// popcount scan (the word whose count passes the row's index) and the set
// bit of that rank in the word.  A complete group (or the last, partial one)
// is summed into the wavefront's LDS tile of the post population with LDS
// atomics, whose nonzero entries then go into G with 64-bit atomics.
// Integer sums: the bits equal row mode's.
__device__ __forceinline__ void group_to_global(const PropArgs &a, unsigned long long *tile, int32_t np,
                                                const int32_t *rp, const int32_t *col, const float *w, double s,
                                                unsigned long long *G, int32_t row, uint32_t nrows, int32_t n_pre,
                                                int lane)
{
    for (int i = lane; i < np; i += kWave) tile[i] = 0ull;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    int32_t b0 = 0, b1 = 0;
    if ((uint32_t)lane < nrows && row >= 0 && row < n_pre) {
        b0 = rp[row];
        b1 = rp[row + 1];
    }
    uint64_t rem = nrows >= (uint32_t)kWave ? ~0ull : ((1ull << nrows) - 1ull);
    int32_t k = 0, k1 = 0;
    Batch BA, BB;
    BatchData DA, DB;
    auto add = [&](const Batch &B, const BatchData &D) {
#pragma unroll
        for (int u = 0; u < kSlots; ++u)
            if (B.ph[u] >= 0 && B.sk[u] + lane < B.se[u])
                atomicAdd(tile + D.c[u], (unsigned long long)fix_increment(s, D.g[u]));
    };
    if (fill_batch(BA, rem, k, k1, b0, b1)) {
        load_batch(DA, BA, col, w, 0, lane);
        for (;;) {
            const bool more_b = fill_batch(BB, rem, k, k1, b0, b1);
            if (!more_b) BB = BA;
            load_batch(DB, BB, col, w, 0, lane);
            add(BA, DA);
            if (!more_b) break;
            const bool more_a = fill_batch(BA, rem, k, k1, b0, b1);
            if (!more_a) BA = BB;
            load_batch(DA, BA, col, w, 0, lane);
            add(BB, DB);
            if (!more_a) break;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int i = lane; i < np; i += kWave) {
        const unsigned long long v = tile[i];
        if (v != 0ull) atomicAdd(G + i, v);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ __forceinline__ void grouped_wave(const PropArgs &a, int prev, int64_t gslot, int lane,
                                             unsigned long long *tile)
{
    using CProjG = const __attribute__((address_space(4))) Proj;
    using CSegG = const __attribute__((address_space(4))) Seg;
    using CI32G = const __attribute__((address_space(4))) int32_t;
    const CI32G *e = (CI32G *)a.grp_proj + 2 * (gslot / kGrpSlots);   // (projection, rows per group)
    const int32_t proj = e[0];
    const uint32_t K = (uint32_t)e[1];
    const uint32_t j0 = (uint32_t)(gslot % kGrpSlots);
    CProjG &P = ((CProjG *)a.projs)[proj];
    const int32_t np = P.n_post, n_pre = P.n_pre, pre_seg = P.pre_seg, pw = P.pre_words, inst = P.inst;
    const int64_t rp_base = P.rp_base, syn_base = P.syn_base, G_base = P.G_base;
    if (np <= 0 || np > kGrpTile || pw <= 0 || inst < 0 || inst >= a.n_inst || K < 1 || K > (uint32_t)kGrpRows)
        return;   // malformed entry
    const int64_t wbase = ((CSegG *)a.segs)[pre_seg].base / kWave;
    const uint64_t *wb = a.bits + (int64_t)prev * a.n_waves + wbase;
    const double sc = (double)a.gscale[inst] * kFixOne;
    const int32_t *rp = a.rp_pool + rp_base;
    const int32_t *col = a.col_pool + syn_base;
    const float *wt = a.w_pool + syn_base;
    unsigned long long *G = (unsigned long long *)(a.G + G_base);
    uint32_t q = j0;          // this wavefront's current group
    uint32_t base = 0;        // spiking rows in the rounds before this one
    int32_t row = -1;         // lane r < kGrpRows: row r of the current group
    for (int32_t w0 = 0; w0 < pw; w0 += kWave) {
        const uint64_t word = w0 + lane < pw ? wb[w0 + lane] : 0ull;
        const uint32_t pc = (uint32_t)__popcll(word);
        const uint32_t incl = wave_incl_sum(pc, lane);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
        // rows of the current group that fall in this round, then the group
        // itself once its last row is in
        for (;;) {
            const uint32_t g0 = q * K;
            if (g0 >= base + tot) break;
            for (int r = 0; r < (int)K; ++r) {
                const uint32_t t = g0 + (uint32_t)r;
                if (t < base || t >= base + tot) continue;   // (uniform)
                const uint32_t u = t - base;
                const uint64_t over = __ballot(incl > u);
                const int L = (int)__builtin_ctzll(over);
                uint64_t bits = readlane_u64(word, (uint32_t)L);
                uint32_t n = u - ((uint32_t)__builtin_amdgcn_readlane((int)incl, L) -
                                  (uint32_t)__builtin_amdgcn_readlane((int)pc, L));
                for (; n > 0; --n) bits &= bits - 1ull;
                if (lane == r) row = (w0 + L) * kWave + (int32_t)__builtin_ctzll(bits);
            }
            if (g0 + K > base + tot) break;   // the group goes on in the next round
            group_to_global(a, tile, np, rp, col, wt, sc, G, row, K, n_pre, lane);
            row = -1;
            q += (uint32_t)kGrpSlots;
        }
        base += tot;
    }
    // the last, partial group
    const uint32_t g0 = q * K;
    if (g0 < base) group_to_global(a, tile, np, rp, col, wt, sc, G, row, base - g0, n_pre, lane);
}

// ---------------------------------------------------------------------------
// CSR propagation, row mode: one wavefront per work item = a chunk of one
// spiking row; 64-bit atomics add the fixed-point weights into G (+ the
// depression of plastic rows).  Suited to sparse activity.  In grouped mode
// the first wavefronts deliver the row groups (above) and the grouped
// projections' row items are skipped.
// ---------------------------------------------------------------------------

template <bool GRP>
__global__ __launch_bounds__(1024) void k_propagate_rows(PropArgs a)
{
    extern __shared__ unsigned long long s_grp[];   // grouped mode: a kGrpTile tile per wavefront
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    const uint32_t it0 = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    CItem *queue = (CItem *)a.queue;
    CProj *projs = (CProj *)a.projs;
    CFloat *gscale = (CFloat *)a.gscale;
    // the step counter and both slots' counts of host-built items are read
    // together; the slot of step t - 1 is picked after
    const int64_t t = a.st->t_prop;
    const uint32_t c0 = a.st->qcnt[0], c1 = a.st->qcnt[1];
    asm volatile("" ::"s"(t), "s"(c0), "s"(c1), "s"(projs), "s"(gscale), "s"(a.col_pool), "s"(a.w_pool), "s"(a.G));
    const int prev = (int)((t + 1) & 1);          // slot of step t - 1
    const uint32_t nc = min((uint32_t)a.qcap, prev ? c1 : c0);
    CItem *q = queue + (int64_t)prev * a.qcap;

    uint32_t g_it = it0, nw_it = nw;
    if (GRP && a.n_grp > 0) {
        const int64_t n_gw = a.n_grp * kGrpSlots;
        if (a.st->grp_off[prev] == 0)
            for (int64_t gs = it0; gs < n_gw; gs += nw)
                grouped_wave(a, prev, gs, lane, s_grp + (threadIdx.x >> 6) * kGrpTile);
        // with enough wavefronts, the row items go to those past the groups
        if ((int64_t)nw > 2 * n_gw) {
            if ((int64_t)it0 < n_gw) nw_it = 0;
            g_it = it0 - (uint32_t)n_gw;
            nw_it = nw_it ? nw - (uint32_t)n_gw : 0u;
        }
    }

    if (nw_it) visit_items(a, prev, g_it, nw_it, nc, [&](int64_t at) {
        if (at >= a.qcap) return;                     // malformed range
        const int32_t proj = q[at].proj, k0 = q[at].k0, k1 = q[at].k1, inst = (int32_t)q[at].aux;
        if (inst < 0 || inst >= a.n_inst) return;   // malformed item
        // the projection record's fields and the instance's g_scale, read
        // together
        CProj &P = projs[proj];
        const int64_t nnz = P.nnz, syn_base = P.syn_base, G_base = P.G_base;
        const int32_t p_inst = P.inst, stdp = P.stdp, p_grp = P.grp;
        const float gs = gscale[inst];
        asm volatile("" ::"s"(nnz), "s"(syn_base), "s"(G_base), "s"(p_inst), "s"(stdp), "s"(gs), "s"(p_grp));
        if (k0 < 0 || k1 > nnz || k0 > k1 || p_inst != inst) return;   // malformed item
        if (GRP && p_grp && a.n_grp > 0) return;                         // delivered in row groups
        const double s = (double)gs * kFixOne;
        const int32_t *col = a.col_pool + syn_base;
        float *w = a.w_pool + syn_base;
        unsigned long long *G = (unsigned long long *)(a.G + G_base);
        if (!stdp) {
            slice_to_global(G, col, w, k0, k1, s, lane);
        } else {
            // batches of 8 x 64 entries at clamped indices: column and weight,
            // then the post traces, then predicated atomics; the depressed
            // weight is stored unpredicated (a clamped duplicate stores the
            // same value as its slice's last entry)
            const float *y = a.trace + P.y_base;
            for (int32_t kb = k0; kb < k1; kb += kSlots * kWave) {
                int32_t c[kSlots], kk[kSlots];
                float g[kSlots], yv[kSlots];
#pragma unroll
                for (int u = 0; u < kSlots; ++u) {
                    kk[u] = min(kb + u * kWave + lane, k1 - 1);
                    c[u] = col[kk[u]];
                    g[u] = w[kk[u]];
                }
#pragma unroll
                for (int u = 0; u < kSlots; ++u) yv[u] = y[c[u]];
                asm volatile("" ::"v"(yv[0]), "v"(yv[1]), "v"(yv[2]), "v"(yv[3]), "v"(yv[4]), "v"(yv[5]),
                             "v"(yv[6]), "v"(yv[7]));
#pragma unroll
                for (int u = 0; u < kSlots; ++u) {
                    w[kk[u]] = fmaxf(0.0f, g[u] - P.a_minus_gmax * yv[u]);
                    if (kb + u * kWave + lane < k1) atomicAdd(G + c[u], (unsigned long long)fix_increment(s, g[u]));
                }
            }
        }
    });
    if (blockIdx.x == 0 && threadIdx.x == 0) a.st->t_neuron = t;
}

// ---------------------------------------------------------------------------
// CSR propagation (+ depression on plastic rows), tile mode: tiled by post neuron.
// Every wavefront is an independent worker with its own LDS tile.  A sparse
// item (few synapses for the tile width) adds its synapses to G with global
// atomics instead; its group's flag tells the reduction that no partial tile
// was written.
// ---------------------------------------------------------------------------
constexpr int kSparseRatio = 6;   // atomics when events * kSparseRatio < tile width

// Pull units.  A unit holds, for 64 post neurons (one per lane), up to
// kPullDepth entries of each one's column, in packets of four: a float4 of
// weights and a word of four one-byte row deltas per lane (64 lanes read
// 1 KiB and 256 contiguous bytes per packet).  A lane starts from its row
// before the unit's first entry and adds each delta in turn; then the pre
// spike word of each entry's row is looked up, from LDS when the pre
// population's words fit the wavefront's tile, else from global memory.
// Each lane adds the fixed-point increments of its spiking rows and stores
// the sum as the unit's partial for its post neuron, which the reduction
// adds into G (the only unit of a slice adds them into G itself).  Padding
// and bridging entries carry weight 0, so they add nothing.  Integer sums:
// the result equals that of pushing the same spikes.  A wavefront works
// through its units as a pipeline: while one unit's first entries are in
// flight, the next unit's record and (for a population of at most 64 words)
// its spike words are loaded.
constexpr int kPullBatch = 4;   // packets (16 entries) per batch of loads

struct PullHdr {
    int64_t pk0, g_base;
    int32_t col_off, npk, pre_seg, inst, wbase, nwords, direct, ncols;
};

__device__ __forceinline__ PullHdr pull_hdr(const PropArgs &a, int64_t u)
{
    CPullUnit &U = ((CPullUnit *)a.pull_units)[u];
    return PullHdr{U.pk0, U.g_base, U.col_off, U.npk, U.pre_seg, U.inst, U.wbase, U.nwords, U.direct, U.ncols};
}

// Spike bit of pre row r from the population's words (32-bit halves).
__device__ __forceinline__ uint32_t spike_bit(const uint64_t *wb, int32_t r)
{
    return (reinterpret_cast<const uint32_t *>(wb)[r >> 5] >> (r & 31)) & 1u;
}

template <bool kLds, class F>
__device__ __forceinline__ long long pull_entries(const float4 *pw, const uint32_t *pd, int32_t npk, int32_t r,
                                                  const uint64_t *wb, double s, F &&after_first_loads)
{
    // Two batches in flight: each iteration decodes the rows of the batch it
    // holds and issues their spike-bit lookups, then the loads of the next
    // batch, then consumes the lookups, so one batch's packets travel while
    // the previous one is added.  Packets past npk (a unit shorter than a
    // batch) repeat the last one; their rows and weights are not used.
    long long sum = 0;
    float4 w[kPullBatch];
    uint32_t d[kPullBatch];
#pragma unroll
    for (int v = 0; v < kPullBatch; ++v) {
        const int64_t i = (int64_t)min(v, npk - 1) * kWave;
        w[v] = pw[i];
        d[v] = pd[i];
    }
    after_first_loads();
    for (int32_t p = 0; p < npk; p += kPullBatch) {
        uint32_t bit[4 * kPullBatch];
#pragma unroll
        for (int v = 0; v < kPullBatch; ++v) {
            const uint32_t dv = p + v < npk ? d[v] : 0u;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                r += (int32_t)((dv >> (8 * j)) & 0xffu);
                bit[4 * v + j] = spike_bit(wb, r);
            }
        }
        const int32_t pn = p + kPullBatch;
        float4 wn[kPullBatch];
        uint32_t dn[kPullBatch];
        if (pn < npk) {
#pragma unroll
            for (int v = 0; v < kPullBatch; ++v) {
                const int64_t i = (int64_t)min(pn + v, npk - 1) * kWave;
                wn[v] = pw[i];
                dn[v] = pd[i];
            }
        }
#pragma unroll
        for (int v = 0; v < kPullBatch; ++v) {
            if (p + v < npk) {
                const float wv[4] = {w[v].x, w[v].y, w[v].z, w[v].w};
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (bit[4 * v + j]) sum += fix_increment(s, wv[j]);
            }
        }
        if (pn < npk) {
#pragma unroll
            for (int v = 0; v < kPullBatch; ++v) {
                w[v] = wn[v];
                d[v] = dn[v];
            }
        }
    }
    return sum;
}

// The pull units u = g, g + nw, g + 2 nw, ... of wavefront g whose pre
// populations are flagged; `sb`: the wavefront's LDS tile (kTileMax words).
__device__ __forceinline__ void pull_phase(const PropArgs &a, int64_t g, int64_t nw, int prev, int lane, uint64_t *sb)
{
    const uint64_t *bits = a.bits + (int64_t)prev * a.n_waves;
    int32_t loaded = -1;   // population whose spike words sb holds
    for (int64_t r = 0; g + r * nw < a.n_pull_units; r += kWave) {
        const int64_t uc = g + (r + lane) * nw;
        const int32_t seg = a.pull_units[min(uc, a.n_pull_units - 1)].pre_seg;
        const uint32_t f = a.pullf[prev * a.n_segs + seg];
        uint64_t m = __ballot(uc < a.n_pull_units && f != 0u);
        if (!m) continue;
        int64_t u = g + (r + __builtin_ctzll(m)) * nw;
        m &= m - 1;
        PullHdr h = pull_hdr(a, u);
        uint64_t word = h.nwords <= kWave ? bits[h.wbase + min(lane, h.nwords - 1)] : 0ull;
        for (;;) {
            const bool more = m != 0;
            const int64_t un = more ? g + (r + __builtin_ctzll(m)) * nw : u;
            m &= m - 1;
            const PullHdr hn = pull_hdr(a, un);
            if (h.pre_seg != loaded && h.nwords <= kTileMax) {
                if (h.nwords <= kWave) {
                    if (lane < h.nwords) sb[lane] = word;
                } else {
                    for (int32_t i = lane; i < h.nwords; i += kWave) sb[i] = bits[h.wbase + i];
                }
                loaded = h.pre_seg;
            }
            // the next unit's words, unless the tile will already hold them
            auto prefetch = [&]() {
                if (more && hn.nwords <= kWave && hn.pre_seg != h.pre_seg)
                    word = bits[hn.wbase + min(lane, hn.nwords - 1)];
            };
            const double s = (double)a.gscale[h.inst] * kFixOne;
            // lanes past a partial slice's columns re-read lane 0's entries
            // (same cache lines: no padding traffic); their sums are dropped
            const int ln = lane < h.ncols ? lane : 0;
            const int32_t r0 = a.pull_r0[u * kWave + ln];
            const float4 *pw = a.pull_w + h.pk0 * kWave + ln;
            const uint32_t *pd = a.pull_d + h.pk0 * kWave + ln;
            const long long sum = h.nwords <= kTileMax ? pull_entries<true>(pw, pd, h.npk, r0, sb, s, prefetch)
                                                       : pull_entries<false>(pw, pd, h.npk, r0, bits + h.wbase, s, prefetch);
            if (h.direct) {
                const int32_t col = a.pull_col[(int64_t)h.col_off + lane];
                if (col >= 0 && sum != 0) a.G[h.g_base + col] += sum;
            } else {
                a.pull_part[u * kWave + lane] = sum;
            }
            if (!more) break;
            u = un;
            h = hn;
        }
    }
}

__global__ __launch_bounds__(kPropWaves * kWave) void k_propagate_tiles(PropArgs a)
{
    __shared__ long long s_acc[kPropWaves][kTileMax];
    __shared__ int32_t s_rows[kPropWaves][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // uniform: scalar indexing
    const int64_t t = a.st->t_prop;
    const int prev = (int)((t + 1) & 1);          // slot of step t - 1
    const uint32_t nc = min((uint32_t)a.qcap, a.st->qcnt[prev]);
    const Item *q = a.queue + (int64_t)prev * a.qcap;
    const uint32_t nw = gridDim.x * kPropWaves;
    long long *acc = s_acc[wid];

    visit_items(a, prev, blockIdx.x * kPropWaves + wid, nw, nc, [&](int64_t at) {
        if (at >= a.qcap) return;                     // malformed range
        CItem &I = ((CItem *)q)[at];
        const int32_t proj = I.proj, word0 = I.row, tile = I.k0, slot = I.k1;
        const uint64_t bits0 = I.bits;
        CProj &P = ((CProj *)a.projs)[proj];
        if (slot >= P.pre_words || tile >= P.n_tiles || word0 >= P.pre_words) return;   // malformed item
        if (P.pull_base >= 0 && a.pullf[prev * a.n_segs + P.pre_seg]) return;         // pulled instead
        // the item of the first slot of each group processes the whole group
        const uint32_t na = min(a.awcnt[prev * a.n_segs + P.pre_seg], (uint32_t)P.pre_words);
        const uint32_t gw = max(1u, a.gwsel[prev * a.n_segs + P.pre_seg]);
        if ((uint32_t)slot % gw != 0 || (uint32_t)slot >= na) return;
        const uint32_t group = (uint32_t)slot / gw;
        const uint32_t nwords = min(gw, na - (uint32_t)slot);
        const int32_t tw = P.tile_w;
        const int32_t c0 = tile * tw;
        const double s = (double)a.gscale[P.inst] * kFixOne;
        const int32_t *col = a.col_pool + P.syn_base;
        float *w = a.w_pool + P.syn_base;
        const int32_t *rp = a.rp_pool + P.rp_base;
        const int32_t *tp = a.tp_pool + (P.tp_base < 0 ? 0 : P.tp_base);
        const int64_t stride = (int64_t)P.n_tiles + 1;
        // bounds of the first word's rows, one lane per spiking row
        int32_t b0 = 0, b1 = 0;
        if ((bits0 >> lane) & 1ull) {
            const int32_t i = word0 * kWave + lane;
            if (P.tp_base < 0) {
                b0 = rp[i];
                b1 = rp[i + 1];
            } else {
                b0 = tp[(int64_t)i * stride + tile];
                b1 = tp[(int64_t)i * stride + tile + 1];
            }
        }
        uint8_t *flag = a.pflag + P.F_base + (int64_t)tile * P.pre_words + group;
        if (nwords == 1 && !P.stdp) {
            int32_t ev = b1 - b0;
#pragma unroll
            for (int d = kWave / 2; d > 0; d >>= 1) ev += __shfl_xor(ev, d, kWave);
            if (ev * kSparseRatio < tw) {
                // sparse: straight into G with atomics
                word_to_global((unsigned long long *)(a.G + P.G_base), col, w, bits0, b0, b1, s, lane);
                if (lane == 0) *flag = 0;
                return;
            }
        }
        for (int i = lane; i < tw; i += kWave) acc[i] = 0;
        const Seg &pre = a.segs[P.pre_seg];
        const int32_t *wl = a.awl + (int64_t)prev * a.n_waves + pre.base / kWave + slot;
        if (!P.stdp) {
            // The group's spiking rows, gathered across its words into a row
            // list in LDS, up to kWave rows per chunk: one lane per word reads
            // the word's id and bits, each lane places its rows by counting
            // the set bits below it, and one lane per listed row loads the
            // row's slice bounds, so a chunk's bounds take one round trip and
            // one batch pipeline covers all of its rows.
            const uint64_t *wbits = a.bits + (int64_t)prev * a.n_waves + pre.base / kWave;
            int32_t *rows = s_rows[wid];
            for (uint32_t w0 = 0; w0 < nwords; w0 += kWave) {
                const uint32_t nwc = min((uint32_t)kWave, nwords - w0);
                const int32_t word_l = wl[w0 + min((uint32_t)lane, nwc - 1)];
                const uint64_t bl = wbits[word_l];
                const uint64_t bits_l = (uint32_t)lane < nwc ? bl : 0ull;
                const uint32_t incl = wave_incl_sum((uint32_t)__popcll(bits_l), lane);
                uint32_t ws = 0;
                while (ws < nwc) {
                    const uint32_t base = ws ? (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)ws - 1) : 0u;
                    // words ws .. we-1 hold at most kWave rows (a word holds
                    // at most kWave, so we > ws)
                    const uint64_t over =
                        __ballot((uint32_t)lane >= ws && (uint32_t)lane < nwc && incl - base > (uint32_t)kWave);
                    const uint32_t we = over ? (uint32_t)__builtin_ctzll(over) : nwc;
                    const uint32_t R = (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)we - 1) - base;
                    for (uint32_t wv = ws; wv < we; ++wv) {
                        const uint64_t bw = readlane_u64(bits_l, wv);
                        const int32_t wd = __builtin_amdgcn_readlane(word_l, (int)wv);
                        const uint32_t off = (wv ? (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)wv - 1) : 0u) - base;
                        if ((bw >> lane) & 1ull)
                            rows[off + (uint32_t)__popcll(bw & ((1ull << lane) - 1ull))] = wd * kWave + lane;
                    }
                    if (R > 0) {
                        const int32_t row = rows[min((uint32_t)lane, R - 1)];
                        int32_t rb0, rb1;
                        if (P.tp_base < 0) {
                            rb0 = rp[row];
                            rb1 = rp[row + 1];
                        } else {
                            rb0 = tp[(int64_t)row * stride + tile];
                            rb1 = tp[(int64_t)row * stride + tile + 1];
                        }
                        const uint64_t rem = R >= (uint32_t)kWave ? ~0ull : ((1ull << R) - 1ull);
                        word_to_tile(acc, col, w, rem, rb0, rb1, c0, s, lane);
                    }
                    ws = we;
                }
            }
            int64_t *out = a.partial + P.P_base + ((int64_t)tile * P.pre_words + group) * tw;
            for (int i = lane; i < tw; i += kWave) out[i] = acc[i];
            if (lane == 0) *flag = 1;
            return;
        }
        // plastic rows: one word at a time, one row at a time
        for (uint32_t wi = 0; wi < nwords; ++wi) {
            uint64_t bits = bits0;
            if (wi > 0) {
                const int32_t word = __builtin_amdgcn_readfirstlane(wl[wi]);
                bits = uniform_u64(a.bits[(int64_t)prev * a.n_waves + pre.base / kWave + word]);
                b0 = b1 = 0;
                if ((bits >> lane) & 1ull) {
                    const int32_t i = word * kWave + lane;
                    if (P.tp_base < 0) {
                        b0 = rp[i];
                        b1 = rp[i + 1];
                    } else {
                        b0 = tp[(int64_t)i * stride + tile];
                        b1 = tp[(int64_t)i * stride + tile + 1];
                    }
                }
            }
            while (bits) {
                const int r = __builtin_ctzll(bits);
                bits &= bits - 1;
                const int32_t k0 = __shfl(b0, r, kWave), k1 = __shfl(b1, r, kWave);
                // batches of 8 x 64 entries of the row at clamped indices; all
                // tile entries read before any is written (distinct columns);
                // a clamped duplicate writes the same sum and the same
                // depressed weight as the row's last entry
                const float *y = a.trace + P.y_base;
                for (int32_t kb = k0; kb < k1; kb += kSlots * kWave) {
                    int32_t c[kSlots], kk[kSlots];
                    float g[kSlots], yv[kSlots];
                    long long v[kSlots];
#pragma unroll
                    for (int u = 0; u < kSlots; ++u) {
                        kk[u] = min(kb + u * kWave + lane, k1 - 1);
                        c[u] = col[kk[u]];
                        g[u] = w[kk[u]];
                    }
#pragma unroll
                    for (int u = 0; u < kSlots; ++u) {
                        yv[u] = y[c[u]];
                        v[u] = acc[c[u] - c0];
                    }
#pragma unroll
                    for (int u = 0; u < kSlots; ++u) {
                        acc[c[u] - c0] = v[u] + fix_increment(s, g[u]);
                        w[kk[u]] = fmaxf(0.0f, g[u] - P.a_minus_gmax * yv[u]);
                    }
                }
            }
        }
        int64_t *out = a.partial + P.P_base + ((int64_t)tile * P.pre_words + group) * tw;
        for (int i = lane; i < tw; i += kWave) out[i] = acc[i];
        if (lane == 0) *flag = 1;
    });
    if (a.st->npull[prev] != 0 && a.n_pull_units > 0) {
        // pull units: wavefront g takes units g, g + nw, g + 2 nw, ... (so
        // the units of the pulled populations spread over every wavefront)
        pull_phase(a, (int64_t)blockIdx.x * kPropWaves + wid, nw, prev, lane, (uint64_t *)acc);
    }
    if (blockIdx.x == 0) {
        // active-word and spike counts of the slot the next neuron update fills
        for (int i = threadIdx.x; i < a.n_segs; i += blockDim.x) {
            a.awcnt[(int64_t)(t & 1) * a.n_segs + i] = 0;
            a.scnt[(int64_t)(t & 1) * a.n_segs + i] = 0;
            a.pullf[(int64_t)(t & 1) * a.n_segs + i] = 0;
        }
        if (threadIdx.x == 0) {
            a.st->npull[t & 1] = 0;
            a.st->t_neuron = t;
        }
    }
}

// ---------------------------------------------------------------------------
// Tile mode, after the propagation: add every group's partial tile into G.
// One wavefront per unit = (projection, post tile, 64 columns, 64 groups),
// one lane per column; flags and partials are loaded 16 groups at a time at
// group indices clamped below the group count (a group that delivered with
// atomics instead has flag 0), and each column ends with one atomic add.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_partials(PropArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t t = a.st->t_neuron;             // set by the propagation just before
    const int prev = (int)((t + 1) & 1);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int64_t g = (int64_t)blockIdx.x * (blockDim.x / kWave) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    // wavefront g takes units g, g + nw, ...: 64 at a time, one per lane, it
    // finds those with partials to add (pre population pushed at t - 1 and a
    // group chunk below its group count), then adds them one by one
    for (int64_t r = 0; g + r * nw < a.n_units; r += kWave) {
        const int64_t uc = g + (r + lane) * nw;
        const int4 Ul = a.units[min(uc, a.n_units - 1)];
        const Proj &Pl = a.projs[Ul.x];
        const int64_t pb = Pl.pull_base;
        const int32_t pseg = Pl.pre_seg, pwords = Pl.pre_words;
        const uint32_t pulled = pb >= 0 ? a.pullf[prev * a.n_segs + pseg] : 0u;
        const uint32_t nal = min(a.awcnt[prev * a.n_segs + pseg], (uint32_t)pwords);
        const uint32_t gwl = max(1u, a.gwsel[prev * a.n_segs + pseg]);
        const bool work = uc < a.n_units && pulled == 0u && nal > 0u && (uint32_t)Ul.w < (nal + gwl - 1) / gwl;
        uint64_t m = __ballot(work);
        while (m) {
            const int l = __builtin_ctzll(m);
            m &= m - 1;
            CInt4 &U = ((CInt4 *)a.units)[g + (r + l) * nw];
            const int32_t proj = U.x, tile = U.y, col0 = U.z;
            const uint32_t chunk = (uint32_t)U.w;
            CProj &P = ((CProj *)a.projs)[proj];
            const uint32_t na = min(a.awcnt[prev * a.n_segs + P.pre_seg], (uint32_t)P.pre_words);
            const uint32_t gw = max(1u, a.gwsel[prev * a.n_segs + P.pre_seg]);
            const uint32_t ng = (na + gw - 1) / gw;
            const uint32_t ge = min(ng, chunk + (uint32_t)kWave);
            const int32_t tw = P.tile_w;
            const int32_t c = col0 + lane;                  // column within the tile
            const int32_t cg = tile * tw + c;               // post neuron
            const bool valid = c < tw && cg < P.n_post;
            const int64_t *pp = a.partial + P.P_base + (int64_t)tile * P.pre_words * tw + (valid ? c : col0);
            const uint8_t *fl = a.pflag + P.F_base + (int64_t)tile * P.pre_words;
            int64_t sum = 0;
            for (uint32_t gi = chunk; gi < ge; gi += 16) {
                uint32_t f[16];
                int64_t v[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const uint32_t gg = min(gi + (uint32_t)k, ge - 1);
                    f[k] = fl[gg];
                    v[k] = pp[(int64_t)gg * tw];
                }
#pragma unroll
                for (int k = 0; k < 16; ++k) sum += (gi + (uint32_t)k < ge && f[k]) ? v[k] : 0;
            }
            if (valid && sum != 0) atomicAdd((unsigned long long *)(a.G + P.G_base + cg), (unsigned long long)sum);
        }
    }
    if (a.st->npull[prev] != 0 && a.n_pull_slices > 0) {
        // reduction groups of pulled slices: wavefront g takes groups g,
        // g + nw, ..., checks 64 at a time (one per lane) against their pre
        // populations' flags, and for each pulled group adds its units'
        // partial sums into G, one lane per post neuron
        for (int64_t r = 0; g + r * nw < a.n_pull_slices; r += kWave) {
            const int64_t sl = g + (r + lane) * nw;
            const int32_t seg = a.pull_slices[min(sl, a.n_pull_slices - 1)].pre_seg;
            const uint32_t f = a.pullf[prev * a.n_segs + seg];
            uint64_t m = __ballot(sl < a.n_pull_slices && f != 0u);
            while (m) {
                const int l = __builtin_ctzll(m);
                m &= m - 1;
                CPullSlice &S = ((CPullSlice *)a.pull_slices)[g + (r + l) * nw];
                const int64_t g_base = S.g_base;
                const int32_t u0 = S.u0, nu = S.n_units, atomic = S.atomic;
                const int32_t col = a.pull_col[(int64_t)S.col_off + lane];
                int64_t sum = 0;
                for (int32_t c = 0; c < nu; c += 8) {
                    int64_t v[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) v[k] = a.pull_part[(int64_t)(u0 + min(c + k, nu - 1)) * kWave + lane];
#pragma unroll
                    for (int k = 0; k < 8; ++k) sum += c + k < nu ? v[k] : 0;
                }
                if (col >= 0 && sum != 0) {
                    if (atomic)
                        atomicAdd((unsigned long long *)(a.G + g_base + col), (unsigned long long)sum);
                    else
                        a.G[g_base + col] += sum;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// STDP potentiation over the columns of post neurons that spiked at t - 1
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_potentiate(LtpArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t t = a.st->t_neuron;
    const int prev = (int)((t + 1) & 1);
    const uint32_t n = min((uint32_t)a.lcap, a.st->lcnt[prev]);
    const Item *q = a.lqueue + (int64_t)prev * a.lcap;
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    uint32_t it = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    for (; it < n; it += nw) {
        const int32_t proj = __builtin_amdgcn_readfirstlane(q[it].proj);
        const int32_t k0 = __builtin_amdgcn_readfirstlane(q[it].k0);
        const int32_t k1 = __builtin_amdgcn_readfirstlane(q[it].k1);
        const Proj &P = a.projs[proj];
        const int32_t *rows = a.csc_row + P.csc_base;
        const int32_t *pos = a.csc_pos + P.csc_base;
        float *w = a.w_pool + P.syn_base;
        const float *x = a.trace + P.x_base;
        // batches of 8 x 64 column entries at clamped indices: positions and
        // rows, then the weights and pre traces, then the stores (a column
        // lists each synapse once; a clamped duplicate stores the same value
        // as the chunk's last entry)
        for (int32_t kb = k0; kb < k1; kb += 8 * kWave) {
            int32_t at[8], r[8];
            float wv[8], xv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t k = min(kb + u * kWave + lane, k1 - 1);
                at[u] = pos[k];
                r[u] = rows[k];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                wv[u] = w[at[u]];
                xv[u] = x[r[u]];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) w[at[u]] = fminf(P.g_max, wv[u] + P.a_plus_gmax * xv[u]);
        }
    }
}

// out[i] = w[perm[i]], 0 where perm[i] < 0: refresh the weights of a
// column-ordered copy.
__global__ void k_gather_weights(const float *w, const int32_t *perm, float *out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = perm[i];
        out[i] = p >= 0 ? w[p] : 0.0f;
    }
}

// Flag (bit 0) any weight that is not finite or is negative; wmax[q] gets
// the bits of projection q's largest weight (block row q of the grid).
__global__ void k_check_weights(const float *w, const Proj *projs, uint32_t *flag, uint32_t *wmax)
{
    const Proj &P = projs[blockIdx.y];
    float m = 0.0f;
    uint32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.nnz; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = w[P.syn_base + i];
        if (!(x >= 0.0f) || !isfinite(x))
            bad = 1;
        else
            m = fmaxf(m, x);
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        m = fmaxf(m, __shfl_xor(m, d, kWave));
        bad |= __shfl_xor(bad, d, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (bad) atomicOr(flag, 1u);
        if (m > 0.0f) atomicMax(&wmax[blockIdx.y], __float_as_uint(m));   // non-negative floats order as their bits
    }
}

hipError_t launch_gather_weights(const float *w, const int32_t *perm, float *out, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_gather_weights, dim3((unsigned)blocks), dim3(256), 0, s, w, perm, out, n);
    return hipGetLastError();
}

hipError_t launch_check_weights(const float *w, const Proj *projs, int32_t n_projs, int64_t max_nnz, uint32_t *flag,
                                uint32_t *wmax, hipStream_t s)
{
    if (n_projs == 0 || max_nnz == 0) return hipSuccess;
    const int64_t bx = std::min<int64_t>((max_nnz + 2047) / 2048, 512);
    hipLaunchKernelGGL(k_check_weights, dim3((unsigned)bx, (unsigned)n_projs), dim3(256), 0, s, w, projs, flag, wmax);
    return hipGetLastError();
}

// With a start/stop event pair the launch goes through hipExtLaunchKernelGGL,
// which stamps the events with that dispatch's own begin and end times.
#define SNN_LAUNCH(kern, grid, blk, s, e0, e1, ...)                                               \
    do {                                                                                         \
        if (e0)                                                                                  \
            hipExtLaunchKernelGGL(kern, grid, blk, 0, s, e0, e1, 0, __VA_ARGS__);                  \
        else                                                                                     \
            hipLaunchKernelGGL(kern, grid, blk, 0, s, __VA_ARGS__);                                \
    } while (0)

hipError_t launch_neuron(const NeuronArgs &a, int block, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const int64_t wpb = block / kWave;
    const int64_t blocks = (a.n_waves + wpb - 1) / wpb;
    if (blocks == 0) return hipSuccess;
    const dim3 g((unsigned)blocks), b(block);
    switch (a.mode * 8 + (a.feat & 7)) {
#define SNN_NEURON_CASE(M, F) \
    case M * 8 + F: SNN_LAUNCH((k_neuron<M, F>), g, b, s, e0, e1, a); break;
#define SNN_NEURON_FEATS(M) \
    SNN_NEURON_CASE(M, 0) SNN_NEURON_CASE(M, 1) SNN_NEURON_CASE(M, 2) SNN_NEURON_CASE(M, 3) \
    SNN_NEURON_CASE(M, 4) SNN_NEURON_CASE(M, 5) SNN_NEURON_CASE(M, 6) SNN_NEURON_CASE(M, 7)
        SNN_NEURON_FEATS(kModeRows)
        SNN_NEURON_FEATS(kModeTiles)
        SNN_NEURON_FEATS(kModeFused)
#undef SNN_NEURON_FEATS
#undef SNN_NEURON_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Delivery of one step.  Tile mode is two kernels, the tiled propagation and
// the reduction of its partial tiles into G; an event pair then brackets both.
hipError_t launch_propagate(const PropArgs &a, int blocks, int block, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (a.mode == kModeRows) {
        if (a.n_grp > 0) {
            // grouped mode: a kGrpTile tile of int64 per wavefront
            const size_t lds = 8 * (size_t)kGrpTile * (size_t)(block / kWave);
            if (e0)
                hipExtLaunchKernelGGL(k_propagate_rows<true>, dim3(blocks), dim3(block), lds, s, e0, e1, 0, a);
            else
                hipLaunchKernelGGL(k_propagate_rows<true>, dim3(blocks), dim3(block), lds, s, a);
        } else {
            SNN_LAUNCH(k_propagate_rows<false>, dim3(blocks), dim3(block), s, e0, e1, a);
        }
        return hipGetLastError();
    }
    // the tiled kernel runs kPropWaves wavefronts per block
    if (a.n_units == 0 && a.n_pull_slices == 0) {
        SNN_LAUNCH(k_propagate_tiles, dim3(blocks), dim3(kPropWaves * kWave), s, e0, e1, a);
        return hipGetLastError();
    }
    hipEvent_t none = nullptr;
    SNN_LAUNCH(k_propagate_tiles, dim3(blocks), dim3(kPropWaves * kWave), s, e0, none, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t rb = std::min<int64_t>((std::max(a.n_units, a.n_pull_slices) + 3) / 4, 4096);
    if (e0) {
        // the stop event of the pair goes on the second kernel
        hipExtLaunchKernelGGL(k_reduce_partials, dim3((unsigned)rb), dim3(256), 0, s, nullptr, e1, 0, a);
    } else {
        hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)rb), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_potentiate(const LtpArgs &a, int blocks, int block, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    SNN_LAUNCH(k_potentiate, dim3(blocks), dim3(block), s, e0, e1, a);
    return hipGetLastError();
}

// Zero n_words 32-bit words with a kernel (a fill inside a captured graph
// stays a kernel node; no memset node): 16-byte stores over the aligned body
// when p is 16-byte aligned, 4-byte stores for the rest.
__global__ __launch_bounds__(256) void k_fill_zero(uint32_t *p, int64_t n_words, int32_t vec)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n4 = vec ? n_words / 4 : 0;
    uint4 *p4 = reinterpret_cast<uint4 *>(p);
    for (int64_t i = i0; i < n4; i += stride) p4[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = 4 * n4 + i0; i < n_words; i += stride) p[i] = 0u;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    const int64_t n_words = (int64_t)(bytes / 4);
    if (n_words == 0) return hipSuccess;
    const int32_t vec = ((uintptr_t)p & 15u) == 0 ? 1 : 0;
    const int64_t items = vec ? (n_words + 3) / 4 : n_words;
    const int64_t blocks = std::min<int64_t>((items + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p, n_words, vec);
    return hipGetLastError();
}

}  // namespace snn
