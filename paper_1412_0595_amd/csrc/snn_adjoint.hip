// Reverse-time adjoint kernels (gfx950): gradient of a loss on one
// population's time-averaged voltage with respect to every synaptic weight
// g and every instance's g_scale, exact for the discrete forward map with
// the spike raster held fixed.
//
// With the raster fixed, the loss population sees the rest of the network
// only through recorded spike times, so the backward pass touches only its
// neurons and the projections into it.  Memory stays O(T/K + K): the forward
// keeps a checkpoint every K steps and the bitmask raster; each segment is
// recomputed from its checkpoint (one block per instance, deliveries summed
// in LDS on the same 2^-40 uS grid as the forward, so the recomputation is
// bit-identical), then reversed neuron by neuron with the adjoint state in
// registers, then the weight gradients are gathered over the spiking rows.
#include "snn_device.h"

namespace snn {

// d/dx [x / (e^x - 1)] = (e^x - 1 - x e^x) / (e^x - 1)^2, by its Taylor
// series -1/2 + x/6 - x^3/180 where the closed form cancels (|x| < 1e-3).
__device__ __forceinline__ double dxexpm1_ratio(double x)
{
    if (fabs(x) < 1e-3) return -0.5 + x * (1.0 / 6.0) - x * x * x * (1.0 / 180.0);
    const double em1 = expm1(x);
    return (em1 * (1.0 - x) - x) / (em1 * em1);
}

// Transposed Jacobian of one Euler substep (x' = x + hs f(x, I)) applied to
// the adjoint (lv, lm, lh, ln) of x'; accumulates the adjoint of I into li.
__device__ __forceinline__ void hh_substep_vjp(const Seg &S, double hs, double hc, double v, double m, double h,
                                               double n, double &lv, double &lm, double &lh, double &ln, double &li)
{
    const HHRates r = hh_rates(v);
    const double dam = -0.25 * 1.28 * dxexpm1_ratio((-52.0 - v) * 0.25);
    const double dbm = 0.2 * 1.4 * dxexpm1_ratio((v + 25.0) * 0.2);
    const double dah = -r.ah * (1.0 / 18.0);
    const double ez = exp((-25.0 - v) * 0.2);
    const double dbh = 0.2 * 4.0 * ez / ((ez + 1.0) * (ez + 1.0));
    const double dan = -0.2 * 0.16 * dxexpm1_ratio((-50.0 - v) * 0.2);
    const double dbn = -r.bn * 0.025;
    const double m2 = m * m, n3 = n * n * n;
    // v' = v + hc (I - I_ion)
    const double dv_dv = 1.0 - hc * (S.gna * m2 * m * h + S.gk * n3 * n + S.gl);
    const double dv_dm = -hc * 3.0 * S.gna * m2 * h * (v - S.ena);
    const double dv_dh = -hc * S.gna * m2 * m * (v - S.ena);
    const double dv_dn = -hc * 4.0 * S.gk * n3 * (v - S.ek);
    // x' = x + hs (a (1 - x) - b x)
    const double dm_dv = hs * (dam * (1.0 - m) - dbm * m), dm_dm = 1.0 - hs * (r.am + r.bm);
    const double dh_dv = hs * (dah * (1.0 - h) - dbh * h), dh_dh = 1.0 - hs * (r.ah + r.bh);
    const double dn_dv = hs * (dan * (1.0 - n) - dbn * n), dn_dn = 1.0 - hs * (r.an + r.bn);
    li += hc * lv;
    const double nv = lv * dv_dv + lm * dm_dv + lh * dh_dv + ln * dn_dv;
    const double nm = lv * dv_dm + lm * dm_dm;
    const double nh = lv * dv_dh + lh * dh_dh;
    const double nn = lv * dv_dn + ln * dn_dn;
    lv = nv;
    lm = nm;
    lh = nh;
    ln = nn;
}

// ---------------------------------------------------------------------------
// Recompute one segment of the loss population of every instance from its
// checkpoint (block b = instance b, thread j = neuron j), writing the tape.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_adj_recompute(AdjArgs a)
{
    __shared__ long long s_acc[kMaxIn * kAdjMaxLoss];
    const int b = blockIdx.x;
    const Seg &S = a.segs[a.loss_seg[b]];
    const int n = S.n;
    const int j = threadIdx.x;
    const bool mine = j < n;
    const int64_t lb = a.loss_base[b];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6, nwb = blockDim.x >> 6;
    const double s_fix = (double)a.gscale[b] * kFixOne;
    const double hc = a.hs * S.inv_c;

    float vh = 0, vl = 0, mh = 0, ml = 0, hh = 0, hl = 0, nh = 0, nl = 0;
    int64_t g[kMaxIn] = {0, 0, 0, 0};
    if (mine) {
        const float *cs = a.ckpt_state;
        const int64_t gi = S.base + j, N = a.n_pad;
        vh = cs[gi]; vl = cs[N + gi]; mh = cs[2 * N + gi]; ml = cs[3 * N + gi];
        hh = cs[4 * N + gi]; hl = cs[5 * N + gi]; nh = cs[6 * N + gi]; nl = cs[7 * N + gi];
#pragma unroll
        for (int q = 0; q < kMaxIn; ++q)
            if (q < S.n_in) g[q] = a.ckpt_G[S.in_G[q] + j];
    }
    for (int k = 0; k < a.K; ++k) {
        const int64_t t = a.t_a + k;
        for (int idx = threadIdx.x; idx < S.n_in * n; idx += blockDim.x) s_acc[idx] = 0;
        __syncthreads();
        if (t > 0) {
            for (int q = 0; q < S.n_in; ++q) {
                const Proj &P = a.projs[S.in_proj[q]];
                const Seg &pre = a.segs[P.pre_seg];
                const int nw = (pre.n + kWave - 1) / kWave;
                const uint64_t *bits = a.raster + (t - 1) * a.n_waves + pre.base / kWave;
                const int32_t *rp = a.rp_pool + P.rp_base;
                const int32_t *col = a.col_pool + P.syn_base;
                const float *w = a.w_pool + P.syn_base;
                for (int wd = wid; wd < nw; wd += nwb) {
                    uint64_t word = uniform_u64(bits[wd]);
                    while (word) {
                        const int i = wd * kWave + __builtin_ctzll(word);
                        word &= word - 1;
                        const int32_t k1 = rp[i + 1];
                        for (int32_t kk = rp[i] + lane; kk < k1; kk += kWave)
                            atomicAdd((unsigned long long *)&s_acc[q * n + col[kk]],
                                      (unsigned long long)fix_increment(s_fix, w[kk]));
                    }
                }
            }
        }
        __syncthreads();
        if (mine) {
            int64_t gin[kMaxIn];
#pragma unroll
            for (int q = 0; q < kMaxIn; ++q)
                if (q < S.n_in) gin[q] = g[q] + s_acc[q * n + j];
            double v = (double)vh + (double)vl, m = (double)mh + (double)ml;
            double h = (double)hh + (double)hl, nn = (double)nh + (double)nl;
            const int64_t c = lb + j;
            a.tape_x[((int64_t)k * 4 + 0) * a.n_loss + c] = v;
            a.tape_x[((int64_t)k * 4 + 1) * a.n_loss + c] = m;
            a.tape_x[((int64_t)k * 4 + 2) * a.n_loss + c] = h;
            a.tape_x[((int64_t)k * 4 + 3) * a.n_loss + c] = nn;
#pragma unroll
            for (int q = 0; q < kMaxIn; ++q)
                if (q < S.n_in) a.tape_g[((int64_t)k * a.n_in_max + q) * a.n_loss + c] = (double)gin[q] * kFixInv;
            const double v0 = v;
            const double iin = syn_current(S, gin, v0);
#pragma unroll
            for (int q = 0; q < kMaxIn; ++q)
                if (q < S.n_in) g[q] = fix_decay(gin[q], S.in_decay[q]);
            for (int s = 0; s < a.substeps; ++s) hh_substep(S, a.hs, hc, iin, v, m, h, nn);
            pair_split(v, vh, vl);
            pair_split(m, mh, ml);
            pair_split(h, hh, hl);
            pair_split(nn, nh, nl);
        }
        __syncthreads();
    }
    // the recomputation must reproduce the next checkpoint bit for bit
    if (mine && a.next_state) {
        const float *cs = a.next_state;
        const int64_t gi = S.base + j, N = a.n_pad;
        uint32_t bad = 0;
        bad += __float_as_uint(cs[gi]) != __float_as_uint(vh);
        bad += __float_as_uint(cs[N + gi]) != __float_as_uint(vl);
        bad += __float_as_uint(cs[2 * N + gi]) != __float_as_uint(mh);
        bad += __float_as_uint(cs[3 * N + gi]) != __float_as_uint(ml);
        bad += __float_as_uint(cs[4 * N + gi]) != __float_as_uint(hh);
        bad += __float_as_uint(cs[5 * N + gi]) != __float_as_uint(hl);
        bad += __float_as_uint(cs[6 * N + gi]) != __float_as_uint(nh);
        bad += __float_as_uint(cs[7 * N + gi]) != __float_as_uint(nl);
#pragma unroll
        for (int q = 0; q < kMaxIn; ++q)
            if (q < S.n_in) bad += a.next_G[S.in_G[q] + j] != g[q];
        if (bad) atomicAdd(a.mismatch, bad);
    }
}

// ---------------------------------------------------------------------------
// Reverse one segment: one lane per loss neuron, adjoint state in registers.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_reverse(AdjArgs a)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_loss) return;
    const int b = a.loss_owner[c];
    const Seg &S = a.segs[a.loss_seg[b]];
    const int64_t N = a.n_loss;
    double lv = a.lam[c], lm = a.lam[N + c], lh = a.lam[2 * N + c], ln = a.lam[3 * N + c];
    double lG[kMaxIn];
#pragma unroll
    for (int q = 0; q < kMaxIn; ++q) lG[q] = q < S.n_in ? a.lam[(4 + q) * N + c] : 0.0;
    const double src = a.dvbar[c] / (double)a.T;
    const double hc = a.hs * S.inv_c;
    for (int k = a.K - 1; k >= 0; --k) {
        lv += src;    // V at the end of this step enters Vbar
        const double v0 = a.tape_x[((int64_t)k * 4 + 0) * N + c];
        double xs[kAdjMaxSub][4];
        xs[0][0] = v0;
        xs[0][1] = a.tape_x[((int64_t)k * 4 + 1) * N + c];
        xs[0][2] = a.tape_x[((int64_t)k * 4 + 2) * N + c];
        xs[0][3] = a.tape_x[((int64_t)k * 4 + 3) * N + c];
        double gin[kMaxIn];
        double iin = S.i_ext, gsum = 0.0;
#pragma unroll
        for (int q = 0; q < kMaxIn; ++q) {
            gin[q] = q < S.n_in ? a.tape_g[((int64_t)k * a.n_in_max + q) * N + c] : 0.0;
            if (q < S.n_in) {
                iin += gin[q] * (S.in_erev[q] - v0);
                gsum += gin[q];
            }
        }
        // states at the start of every substep
#pragma unroll
        for (int s = 1; s < kAdjMaxSub; ++s) {
            if (s < a.substeps) {
                double v = xs[s - 1][0], m = xs[s - 1][1], h = xs[s - 1][2], n = xs[s - 1][3];
                hh_substep(S, a.hs, hc, iin, v, m, h, n);
                xs[s][0] = v;
                xs[s][1] = m;
                xs[s][2] = h;
                xs[s][3] = n;
            }
        }
        double li = 0.0;
#pragma unroll
        for (int s = kAdjMaxSub - 1; s >= 0; --s)
            if (s < a.substeps) hh_substep_vjp(S, a.hs, hc, xs[s][0], xs[s][1], xs[s][2], xs[s][3], lv, lm, lh, ln, li);
        // I = I_ext + sum_q Ginj_q (E_q - V(t-1)); G(t) = d_q Ginj_q
#pragma unroll
        for (int q = 0; q < kMaxIn; ++q) {
            if (q < S.n_in) {
                const double lgi = S.in_decay[q] * lG[q] + li * (S.in_erev[q] - v0);
                a.lg[((int64_t)k * a.n_in_max + q) * N + c] = lgi;
                lG[q] = lgi;     // Ginj_q(t) = G_q(t-1) + deliveries
            }
        }
        lv -= li * gsum;
    }
    a.lam[c] = lv;
    a.lam[N + c] = lm;
    a.lam[2 * N + c] = lh;
    a.lam[3 * N + c] = ln;
#pragma unroll
    for (int q = 0; q < kMaxIn; ++q)
        if (q < S.n_in) a.lam[(4 + q) * N + c] = lG[q];
}

// ---------------------------------------------------------------------------
// Weight and g_scale gradients of one segment: a wavefront per 64 rows of one
// projection into the loss population; rows that spiked at t - 1 add
// g_scale * lambda_Ginj(t)[post] to dL/dg and g * lambda_Ginj(t)[post] to
// dL/dg_scale.  Each synapse belongs to one wavefront, so no atomics on dg.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_gather(AdjArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wg = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wg >= a.n_gitems) return;
    const int4 it = a.gitems[wg];
    const int b = it.x, q = it.y, wd = it.w;
    const Seg &L = a.segs[a.loss_seg[b]];
    const Proj &P = a.projs[L.in_proj[q]];
    const Seg &pre = a.segs[P.pre_seg];
    const double s = (double)a.gscale[b];
    const int64_t lb = a.loss_base[b];
    const int32_t *rp = a.rp_pool + P.rp_base;
    const int32_t *col = a.col_pool + P.syn_base;
    const float *w = a.w_pool + P.syn_base;
    float *dg = a.dg + P.syn_base;
    double acc = 0.0;
    for (int k = 0; k < a.K; ++k) {
        const int64_t t = a.t_a + k;
        if (t == 0) continue;
        uint64_t word = uniform_u64(a.raster[(t - 1) * a.n_waves + pre.base / kWave + wd]);
        const double *lgk = a.lg + ((int64_t)k * a.n_in_max + q) * a.n_loss + lb;
        while (word) {
            const int i = wd * kWave + __builtin_ctzll(word);
            word &= word - 1;
            const int32_t k1 = rp[i + 1];
            for (int32_t kk = rp[i] + lane; kk < k1; kk += kWave) {
                const double l = lgk[col[kk]];
                dg[kk] = (float)((double)dg[kk] + s * l);
                acc += (double)w[kk] * l;
            }
        }
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_down(acc, d, kWave);
    if (lane == 0 && acc != 0.0) atomicAdd(&a.ds[b], acc);
}

__global__ void k_gather_vbar(const Seg *segs, const int32_t *loss_seg, const int64_t *loss_base,
                              const int32_t *loss_owner, int64_t n_loss, const double *vsum, double inv_T, double *vbar)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_loss) return;
    const int b = loss_owner[c];
    const Seg &S = segs[loss_seg[b]];
    vbar[c] = vsum[S.base + (c - loss_base[b])] * inv_T;
}

hipError_t launch_adj_recompute(const AdjArgs &a, int block, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_recompute, dim3(a.n_inst), dim3(block), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_reverse(const AdjArgs &a, hipStream_t s)
{
    const int64_t blocks = (a.n_loss + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_reverse, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_gather(const AdjArgs &a, hipStream_t s)
{
    const int64_t blocks = (a.n_gitems + 3) / 4;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_gather, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gather_vbar(const Seg *segs, const int32_t *loss_seg, const int64_t *loss_base,
                              const int32_t *loss_owner, int64_t n_loss, const double *vsum, double inv_T,
                              double *vbar, hipStream_t s)
{
    const int64_t blocks = (n_loss + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_vbar, dim3((unsigned)blocks), dim3(256), 0, s, segs, loss_seg, loss_base, loss_owner,
                       n_loss, vsum, inv_T, vbar);
    return hipGetLastError();
}

}  // namespace snn
