// chi_kernels.h -- device code of the internal-dynamics operator chi and the
// helpers shared by the device kernels.  Included by kernels.hip (generic
// network policy, compiled ahead of time for gfx950) and by the source the
// runtime compiles per network (compiled network policy).
//
// chi (paper: Algorithm section, "Internal cell dynamics module": every cell
// updated independently over the splitting interval) runs Gillespie's
// direct method over the voxels of each cell (RDME: reactions in a voxel,
// diffusion jumps to adjacent voxels).  Two kernels compute identical bits:
//   - one lane per cell: the lane's counts (int32) and its binary sum tree of
//     voxel propensities (FP64) live in LDS, field-major with the lane index
//     fastest, so 64 lanes touching "their" element hit 64 distinct banks;
//   - one 16-lane row per cell (at most 16 voxels): lane l holds voxel l.
// Work items (<= 64 cells of one tissue) come one per workgroup or, in
// persistent mode, from a device queue every workgroup pulls from until it is
// empty; the last workgroup to leave clears the queue for the next launch.
// A launch may ask for a raised issue priority of its wavefronts (`prio`):
// where several classes' launches share the device, the arbiter then serves
// its wavefronts first on a SIMD they share with another launch's.
#pragma once

#include "device_math.h"
#include "internal.h"

namespace tissue_impl {
namespace {

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Next work item for this workgroup (one wavefront); n_items or more when
// none is left.  Persistent queue: one counter shared by the launch.
__device__ __forceinline__ uint32_t next_item(uint32_t *queue, bool persistent, uint32_t &cursor)
{
    if (!persistent) {
        uint32_t it = cursor;
        cursor = 0xFFFFFFFFu;
        return it;
    }
    uint32_t it = 0;
    if (threadIdx.x == 0) it = atomicAdd(queue, 1u);
    it = __shfl(it, 0, kWave);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)it);
}

// Called by every workgroup when it has no more items: the last one out
// resets the queue and the exit count (queue[0], queue[1]) and, if given,
// one more counter (the retry count consumed by a follow-up launch).
__device__ __forceinline__ void leave_queue(uint32_t *queue, bool persistent,
                                            uint32_t *also_reset = nullptr)
{
    if (!persistent) return;
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(queue + kQDone, 1u);
        if (done == gridDim.x - 1) {
            atomicExch(queue, 0u);
            atomicExch(queue + kQDone, 0u);
            if (also_reset) atomicExch(also_reset, 0u);
        }
    }
}

// Wave-uniform copies: the tissue record is reached through a pointer read
// from memory, so the compiler cannot prove its fields uniform; reading them
// once per work item and broadcasting lane 0's value keeps them in scalar
// registers for the whole event loop.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ double uni(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = uni((uint32_t)b), hi = uni((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ uint64_t uni(uint64_t v)
{
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

// A network policy supplies the channel structure of the chi kernels:
//   SM, RM, NDM   species slots, reaction slots, diffusion slots;
//   kFixedSpecies true when every tissue using it has exactly SM species;
//   ra(r), rb(r)  reactants of reaction r (-1: none), dsp(q) species of
//                 diffusion channel q, delta(r, s) net change;
//   rate[r], drate[q] the tissue's constants (runtime, wave-uniform);
//   load(M)       fill the runtime part from the tissue record.
// NetGeneric keeps the whole structure in scalar registers, zero-padded to
// the slot counts (a padding reaction has no reactants and rate 0, a padding
// diffusion channel rate 0: each adds exactly 0.0 to every fold and is never
// selected).  A compiled network (generated per network at tissue creation)
// makes ra, rb, dsp and delta compile-time constants.
template <int SM_, int RM_, int NDM_>
struct NetGeneric {
    static constexpr int SM = SM_, RM = RM_, NDM = NDM_;
    static constexpr bool kFixedSpecies = false;  // the tissue's species count is <= SM
    int ra_[RM], rb_[RM];
    uint32_t dlo_[RM], dhi_[RM];
    int dsp_[NDM > 0 ? NDM : 1];
    double rate[RM];
    double drate[NDM > 0 ? NDM : 1];
    __device__ __forceinline__ int ra(int r) const { return ra_[r]; }
    __device__ __forceinline__ int rb(int r) const { return rb_[r]; }
    __device__ __forceinline__ int dsp(int q) const { return dsp_[q]; }
    __device__ __forceinline__ int delta(int r, int s) const
    {
        const uint32_t w = s < 4 ? dlo_[r] : dhi_[r];
        return (int)(int8_t)((w >> (8 * (s & 3))) & 0xFFu);
    }
    __device__ __forceinline__ void load(const DevModel &M)
    {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            ra_[r] = uni((int)M.reac_a[r]);
            rb_[r] = uni((int)M.reac_b[r]);
            rate[r] = uni(M.rates[r]);
            dlo_[r] = uni(M.delta_lo[r]);
            dhi_[r] = uni(M.delta_hi[r]);
        }
#pragma unroll
        for (int q = 0; q < NDM; ++q) {
            dsp_[q] = uni((int)M.diff_species[q]);
            drate[q] = uni(M.diff_rate[q]);
        }
    }
};

// Mass-action propensity of reaction r from the voxel's counts held as
// doubles.  Counts are below 2^26, so every product of two counts is an
// exact integer below 2^52 and equals the integer product converted.
template <class NET>
__device__ __forceinline__ double reaction_prop(const NET &n, int r, const double *xd)
{
    const int a = n.ra(r), b = n.rb(r);
    if (a < 0) return n.rate[r];
    const double xa = xd[a];
    if (b < 0) return n.rate[r] * xa;
    if (a == b) return n.rate[r] * ((xa * (xa - 1.0)) * 0.5);
    return n.rate[r] * (xa * xd[b]);
}

// Fold of the voxel's channels (reactions, then diffusion D_s (x_s deg)).
template <class NET>
__device__ __forceinline__ double voxel_fold(const NET &n, const double *xd, double degd)
{
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < NET::RM; ++r) acc = acc + reaction_prop(n, r, xd);
#pragma unroll
    for (int q = 0; q < NET::NDM; ++q) acc = acc + n.drate[q] * (xd[n.dsp(q)] * degd);
    return acc;
}

// The selection scan over the same fold: the first channel with a_k > 0
// and r < prefix through k, else the last channel with a_k > 0.  Prefixes
// never decrease and a zero channel repeats its predecessor's prefix, so
// the first channel with r < prefix_k always has a_k > 0, and its index is
// the number of channels whose prefix is <= r.  Only a diffusion channel
// needs its residual (r minus the prefix before it) and a1 = D_s x_s, so
// those are tracked over the diffusion channels alone: channel k is the one
// selected exactly when r >= prefix_{k-1} and r < prefix_k.  When r is at or
// past the voxel's total (possible only through the rounding of the descent)
// a second, rarely taken pass finds the last positive channel.  Returns the
// channel slot (reactions 0..RM-1, diffusion RM + q), or the slot count when
// the voxel has no positive channel.
template <class NET>
__device__ __forceinline__ int voxel_select(const NET &n, const double *xd, double degd, double r,
                                            double &resid, double &a1)
{
    constexpr int RM = NET::RM, NDM = NET::NDM, NC = RM + NDM;
    double acc = 0.0, before = 0.0;
    int below = 0;
    bool under_prev = true;
    a1 = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const double a = k < RM ? reaction_prop(n, k, xd)
                                : n.drate[k - RM] * (xd[n.dsp(k - RM)] * degd);
        const double next = acc + a;
        const bool under = r >= next;
        below += under ? 1 : 0;
        if (k >= RM) a1 = under_prev ? n.drate[k - RM] * xd[n.dsp(k - RM)] : a1;
        if (k >= RM - 1) before = under ? next : before;
        under_prev = under;
        acc = next;
    }
    int sel = below;
    if (__builtin_expect(sel >= NC, 0)) {
        double acc2 = 0.0;
        sel = NC;
        before = 0.0;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const double a = k < RM ? reaction_prop(n, k, xd)
                                    : n.drate[k - RM] * (xd[n.dsp(k - RM)] * degd);
            if (a > 0.0) {
                sel = k;
                before = acc2;
                a1 = k < RM ? 0.0 : n.drate[k - RM] * xd[n.dsp(k - RM)];
            }
            acc2 = acc2 + a;
        }
    }
    resid = r - before;
    return sel;
}

// The fold of voxel_fold keeping, for the row kernel, every channel's
// prefix (pre[k] = the fold through channel k) and every diffusion channel's
// a1 = D_s x_s, so that a later selection on this voxel needs no products.
template <class NET>
__device__ __forceinline__ double voxel_fold_cached(const NET &n, const double *xd, double degd,
                                                    double *pre, double *ad)
{
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < NET::RM; ++r) {
        acc = acc + reaction_prop(n, r, xd);
        pre[r] = acc;
    }
#pragma unroll
    for (int q = 0; q < NET::NDM; ++q) {
        acc = acc + n.drate[q] * (xd[n.dsp(q)] * degd);
        pre[NET::RM + q] = acc;
        ad[q] = n.drate[q] * xd[n.dsp(q)];
    }
    return acc;
}

// voxel_select from the cached prefixes (same channel, residual and a1).
// Only lanes with `need` get a correct result when r is at or past the
// total (the others skip the second pass, whose cost the whole wave pays).
template <class NET>
__device__ __forceinline__ int voxel_select_cached(const NET &n, const double *pre, const double *ad,
                                                   const double *xd, double degd, double r, bool need,
                                                   double &resid, double &a1)
{
    constexpr int RM = NET::RM, NDM = NET::NDM, NC = RM + NDM;
    double before = 0.0;
    int below = 0;
    bool under_prev = true;
    a1 = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const bool under = r >= pre[k];
        below += under ? 1 : 0;
        if (k >= RM) a1 = under_prev ? ad[k - RM] : a1;
        if (k >= RM - 1) before = under ? pre[k] : before;
        under_prev = under;
    }
    resid = r - before;
    if (__builtin_expect(need && below >= NC, 0)) below = voxel_select(n, xd, degd, r, resid, a1);
    return below;
}

// The channel table of a work item's network, in LDS: per channel slot the
// net change of every species as signed bytes (species 0..3 in lo, 4..7 in
// hi) and, for a diffusion channel, its species (else -1).  Slot RM + NDM is
// all zero (no positive channel: no change).
struct ChanEntry {
    uint32_t lo, hi;
    int32_t spec, pad;
};
constexpr int kChanSlots = kMaxReactions + kMaxSpecies + 1;

template <class NET>
__device__ __forceinline__ void load_channel_table(ChanEntry *tab, const DevModel &M)
{
    constexpr int RM = NET::RM, NDM = NET::NDM;
    const int k = threadIdx.x;
    if (k <= RM + NDM) {
        ChanEntry e{0u, 0u, -1, 0};
        if (k < RM) {
            e.lo = M.delta_lo[k];
            e.hi = M.delta_hi[k];
        } else if (k < RM + NDM && k - RM < M.n_diff) {
            const int sp = M.diff_species[k - RM];
            e.spec = sp;
            if (sp < 4) e.lo = 0xFFu << (8 * sp);
            else e.hi = 0xFFu << (8 * (sp - 4));
        }
        tab[k] = e;
    }
    __builtin_amdgcn_wave_barrier();
}

// Net change of species q in a packed change (signed bytes, species 0..3
// in lo, 4..7 in hi).  Counts are kept as integers beside their exact
// doubles: a count left [0, 2^k) exactly when the OR of the counts, taken
// unsigned, is 2^k or more (a negative count has the sign bit set).
__device__ __forceinline__ int entry_delta(uint32_t lo, uint32_t hi, int q)
{
    const uint32_t w = q < 4 ? lo : hi;
    return (int)(int8_t)((w >> (8 * (q & 3))) & 0xFFu);
}

// The value unchanged, but opaque to the optimiser (an empty asm with a
// vector-register constraint; no instruction is emitted).  Used inside the
// event loops so that compares on loop-invariant per-lane values are redone
// per iteration instead of being hoisted and held live as scalar lane masks,
// which exhausts the scalar registers.
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Voxel v = y*w + x of a w x h mesh (v < 64, w <= 8): y = (v * inv_w) >> 16
// with inv_w = 65536 / w + 1, exact on that range.
struct Mesh {
    int w, h, inv_w;
};

__device__ __forceinline__ void voxel_xy(const Mesh &g, int v, int &x, int &y)
{
    y = (v * g.inv_w) >> 16;
    x = v - y * g.w;
}

__device__ __forceinline__ int voxel_degree(const Mesh &g, int v)
{
    int x, y;
    voxel_xy(g, v, x, y);
    return (x > 0) + (x < g.w - 1) + (y > 0) + (y < g.h - 1);
}

// Destination of a diffusion jump: the kdir-th present neighbour in the
// order (-x, +x, -y, +y).
__device__ __forceinline__ int neighbour_at(const Mesh &g, int v, int kdir)
{
    int x, y;
    voxel_xy(g, v, x, y);
    int out = v, idx = 0;
    if (x > 0) { if (idx == kdir) out = v - 1; ++idx; }
    if (x < g.w - 1) { if (idx == kdir) out = v + 1; ++idx; }
    if (y > 0) { if (idx == kdir) out = v - g.w; ++idx; }
    if (y < g.h - 1) { if (idx == kdir) out = v + g.w; }
    return out;
}

// Index of the diffusion direction: #{l in 1..deg-1 : resid >= l * a1}.
__device__ __forceinline__ int jump_direction(double resid, double a1, int deg)
{
    int kdir = 0;
#pragma unroll
    for (int l = 1; l <= 3; ++l)
        if (l <= deg - 1 && resid >= (double)l * a1) ++kdir;
    return kdir;
}

// Per-item uniform data of a tissue.
struct ItemCtx {
    const DevTissue *T;
    const DevModel *M;   // the item's network
    int32_t *counts;
    int S;
    uint32_t first, count, step, key0, key1, tagword, cap;
};

__device__ __forceinline__ ItemCtx item_ctx(const DevTissue *const *tbl, const ChiItem &item,
                                            uint32_t kstep, uint32_t tag)
{
    ItemCtx c;
    c.T = tbl[uni(item.tissue)];
    c.M = c.T->models + uni(item.model);
    c.counts = c.T->counts;
    c.S = uni(c.T->model.n_species);
    c.first = uni(item.first);
    c.count = uni(item.count);
    c.step = uni(c.T->step_base) + kstep;
    const uint64_t seed = uni((uint64_t)c.T->seed);
    c.key0 = (uint32_t)seed;
    c.key1 = (uint32_t)(seed >> 32);
    c.tagword = (uni(c.T->sim_id) << 2) | tag;
    c.cap = uni(c.T->event_cap);
    return c;
}

__device__ __forceinline__ void item_stats(const ItemCtx &c, uint32_t ev, uint32_t draws,
                                           bool overflow, bool capped, int stat_slot)
{
    const uint32_t ev_sum = wave_sum_u32(ev);
    const uint32_t dr_sum = wave_sum_u32(draws);
    const bool any_over = __any(overflow);
    const bool any_cap = __any(capped);
    if (threadIdx.x == 0) {
        if (ev_sum) atomicAdd(c.T->stats + stat_slot, (unsigned long long)ev_sum);
        if (dr_sum) atomicAdd(c.T->stats + 2, (unsigned long long)dr_sum);
        if (any_over) atomicOr(c.T->flags + 0, 1u);
        if (any_cap) atomicOr(c.T->flags + 1, 1u);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// chi, one lane per cell.  LDS per lane: the sum tree (2P doubles) and the
// cell's counts (P*S int32, voxel-major), field-major across lanes.
// ---------------------------------------------------------------------------
// n_items_dev: when not null the item count is read from device memory
// (the retry list of a lane16 launch) and *n_items_dev is cleared by the
// last workgroup.  first: the item of a workgroup that is not persistent
// (its index in the grid, or the item a whole-run kernel asks for).
template <class NET>
__device__ __forceinline__ void chi_lane_body(unsigned char *lds, const DevTissue *const *tbl,
                                              const ChiItem *items, uint32_t n_items, uint32_t *queue,
                                              int persistent, int cells_per_item, int log2p, double dt,
                                              uint32_t kstep, uint32_t tag, uint32_t *n_items_dev,
                                              int prio, uint32_t first)
{
    constexpr int SM = NET::SM;
    __shared__ ChanEntry tab[kChanSlots];
    if (prio) __builtin_amdgcn_s_setprio(2);
    if (n_items_dev) n_items = uni(*(volatile uint32_t *)n_items_dev);
    const int lane = threadIdx.x;
    const int stride = cells_per_item;
    const int P = 1 << log2p;
    uint32_t cursor = first;
    for (;;) {
        const uint32_t it = next_item(queue, persistent != 0, cursor);
        if (it >= n_items) break;
        const ChiItem item = items[it];
        const ItemCtx c = item_ctx(tbl, item, kstep, tag);
        NET net;
        net.load(*c.M);
        load_channel_table<NET>(tab, *c.M);
        const int S = NET::kFixedSpecies ? NET::SM : c.S;
        double *tree = reinterpret_cast<double *>(lds) + lane;  // [2P][stride]
        int32_t *cnt = reinterpret_cast<int32_t *>(lds + (size_t)2 * P * stride * 8) + lane;

        const bool active = lane < (int)c.count;
        uint32_t cell = 0;
        Mesh g{1, 1, 65537};
        long long gbase = 0;
        if (active) {
            cell = (uint32_t)c.T->cell_list[c.first + lane];
            g.w = c.T->wh[2 * cell];
            g.h = c.T->wh[2 * cell + 1];
            g.inv_w = 65536 / g.w + 1;
            gbase = (long long)c.T->vox_off[cell] * S;
            const int n = g.w * g.h * S;
            for (int i = 0; i < n; ++i) cnt[i * stride] = c.counts[gbase + i];
        }
        const int V = g.w * g.h;
        double xd[SM];

        if (active) {
            for (int v = 0; v < P; ++v) {
                double leaf = 0.0;
                if (v < V) {
#pragma unroll
                    for (int q = 0; q < SM; ++q) xd[q] = (double)cnt[(v * S + q) * stride];
                    leaf = voxel_fold(net, xd, (double)voxel_degree(g, v));
                }
                tree[(P + v) * stride] = leaf;
            }
            for (int n = P - 1; n >= 1; --n)
                tree[n * stride] = tree[(2 * n) * stride] + tree[(2 * n + 1) * stride];
        }

        double t = 0.0;
        uint32_t j = 0, ev = 0;
        bool overflow = false, capped = false;
        if (active) {
            // The draw of ordinal j depends only on the counter, so draw j+1
            // is made while event j proceeds (two independent dependency
            // chains for the scheduler); the one draw past the last is unused.
            double e1, u2;
            {
                const tdev::Words4 wds = tdev::philox4x32_10(0u, c.step, cell, c.tagword, c.key0, c.key1);
                double u1;
                tdev::two_uniforms(wds, u1, u2);
                e1 = -tdev::plog<true>(u1);
            }
            for (;;) {
                const double a0 = tree[1 * stride];
                if (a0 == 0.0) break;
                if (ev >= c.cap) {
                    capped = true;
                    break;
                }
                ++j;
                const double tn = t + e1 / a0;
                if (tn >= dt) break;
                t = tn;
                double r = u2 * a0;
                {
                    const tdev::Words4 wds = tdev::philox4x32_10(j, c.step, cell, c.tagword, c.key0, c.key1);
                    double u1;
                    tdev::two_uniforms(wds, u1, u2);
                    e1 = -tdev::plog<true>(u1);
                }

                // descend the sum tree
                int n = 1;
                for (int lvl = 0; lvl < log2p; ++lvl) {
                    const double L = tree[(2 * n) * stride];
                    const double R = tree[(2 * n + 1) * stride];
                    if (r < L || R == 0.0) {
                        n = 2 * n;
                    } else {
                        r = r - L;
                        n = 2 * n + 1;
                    }
                }
                const int v = n - P;

                // the voxel's counts, the channel, the change
                const Mesh go{opaque(g.w), opaque(g.h), opaque(g.inv_w)};
                int32_t *x = cnt + v * S * stride;
                int32_t xi[SM];
#pragma unroll
                for (int q = 0; q < SM; ++q) {
                    xi[q] = x[q * stride];
                    xd[q] = (double)xi[q];
                }
                const int deg = voxel_degree(go, v);
                double resid, a1;
                const int sel = voxel_select(net, xd, (double)deg, r, resid, a1);
                const ChanEntry e = tab[sel];
                uint32_t any_bits = 0u;  // OR of the counts: the range check
#pragma unroll
                for (int q = 0; q < SM; ++q) {
                    if (q < S) {
                        xi[q] += entry_delta(e.lo, e.hi, q);
                        x[q * stride] = xi[q];
                        xd[q] = (double)xi[q];
                        any_bits |= (uint32_t)xi[q];
                    }
                }
                overflow |= any_bits >= (uint32_t)kCountLimit;
                int dst = v;
                if (e.spec >= 0) {
                    dst = neighbour_at(go, v, jump_direction(resid, a1, deg));
                    int32_t *xdst = cnt + (dst * S + e.spec) * stride;
                    const int32_t nd = *xdst + 1;
                    *xdst = nd;
                    overflow |= nd >= kCountLimit;
                }
                tree[(P + v) * stride] = voxel_fold(net, xd, (double)deg);
                if (dst != v) {
#pragma unroll
                    for (int q = 0; q < SM; ++q) xd[q] = (double)cnt[(dst * S + q) * stride];
                    tree[(P + dst) * stride] = voxel_fold(net, xd, (double)voxel_degree(go, dst));
                }
                // ancestors of the changed leaves
                int na = (P + v) >> 1, nb = (P + dst) >> 1;
                for (int lvl = 0; lvl < log2p; ++lvl) {
                    tree[na * stride] = tree[(2 * na) * stride] + tree[(2 * na + 1) * stride];
                    na >>= 1;
                }
                if (dst != v) {
                    for (int lvl = 0; lvl < log2p; ++lvl) {
                        tree[nb * stride] = tree[(2 * nb) * stride] + tree[(2 * nb + 1) * stride];
                        nb >>= 1;
                    }
                }
                ++ev;
            }
            const int n = V * S;
            for (int i = 0; i < n; ++i) c.counts[gbase + i] = cnt[i * stride];
            if (c.T->tr_chi_ev) {
                const uint32_t ts = uni(c.T->trace_steps), nc = uni(c.T->n_cells);
                const size_t slot = (size_t)(c.step % ts) * nc + cell;
                c.T->tr_chi_ev[slot] = tag ? c.T->tr_chi_ev[slot] + ev : ev;  // 2nd half adds
                c.T->tr_chi_t[slot] = (unsigned long long)__double_as_longlong(t);
            }
        }
        item_stats(c, ev, j, overflow, capped, 0);
    }
    leave_queue(queue, persistent != 0, n_items_dev);
}

// ---------------------------------------------------------------------------
// chi, one row of 16, 32 or 64 lanes per cell (cells of at most that many
// voxels): lane l of the row holds voxel l's counts (as exact doubles) and
// leaf propensity.  The sum tree is rebuilt in registers after every event
// by four in-row DPP exchanges (pair, quad, half-row, row) and, for wider
// rows, lane exchanges across rows; the descent is evaluated by every lane
// along the path to its own leaf, and exactly one lane finds all its
// decisions consistent.  Draws are made a row's width at a time, one per
// lane.
// ---------------------------------------------------------------------------
namespace {

// The value of another lane by a DPP lane pattern (all row and bank masks
// on: every lane of an active group reads an active lane of the same row,
// so no fallback value is needed and none is initialised).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int plo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
    const int phi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
    return __hiloint2double(phi, plo);
}

constexpr int kDppPairSwap = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppPairLeft = 0xA0;   // quad_perm [0,0,2,2]
constexpr int kDppPairRight = 0xF5;  // quad_perm [1,1,3,3]
constexpr int kDppQuadLeft = 0x00;   // quad_perm [0,0,0,0]
constexpr int kDppQuadRight = 0xAA;  // quad_perm [2,2,2,2]
constexpr int kDppRowMirror = 0x140;

// OR of a 32-bit value over the lane's 16-lane row (full wave required).
__device__ __forceinline__ uint32_t row_or(uint32_t x)
{
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppPairSwap, 0xF, 0xF, false);
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppQuadSwap, 0xF, 0xF, false);
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppHalfMirror, 0xF, 0xF, false);
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowMirror, 0xF, 0xF, false);
    return x;
}

// The value of lane (lane ^ mask), mask 16 or 32: the tree levels and the
// word broadcast of rows wider than one 16-lane DPP row.  The gfx950 lane
// swaps between row pairs and wave halves, without LDS: swapping a value
// with itself leaves, in the first result, every even row's (lower half's)
// own value and every odd row's (upper half's) partner's, in the second the
// other way round.
__device__ __forceinline__ uint32_t xlane_u32(uint32_t v, int mask)
{
    const int lane = (int)threadIdx.x;
    if (mask == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return lane < 32 ? r[1] : r[0];
    }
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane & 16) == 0 ? r[1] : r[0];
}

__device__ __forceinline__ double xlane_f64(double v, int mask)
{
    const uint32_t lo = (uint32_t)__double2loint(v), hi = (uint32_t)__double2hiint(v);
    return __hiloint2double((int)xlane_u32(hi, mask), (int)xlane_u32(lo, mask));
}

// One descent level from the children L (left) and R of the lane's ancestor.
__device__ __forceinline__ void descent_children(double L, double R, int bit, double &r, bool &on)
{
    const bool left = (r < L) || (R == 0.0);
    on = on && (left == (bit == 0));
    r = left ? r : r - L;
}

// One descent level: children L (left) and R of the lane's ancestor, given
// the lane's own subtree sum and its sibling's; bit = lane's side.
__device__ __forceinline__ void descent_level(double own, double sib, int bit, double &r, bool &on)
{
    const double L = bit ? sib : own;
    const double R = bit ? own : sib;
    const bool left = (r < L) || (R == 0.0);
    on = on && (left == (bit == 0));
    r = left ? r : r - L;
}

}  // namespace

// LDS of the row kernel: per lane one pre-drawn (-plog(U1), U2) pair, and
// the channel table.
struct RowShared {
    double rng_e[kWave];
    double rng_u[kWave];
    ChanEntry chan[kChanSlots];
};

// RW: lanes per row (16, 32 or 64), one voxel per lane, 64 / RW cells per
// work item; rows of 32 and 64 lanes add one or two tree levels across the
// 16-lane DPP rows.
template <class NET, int RW>
__device__ __forceinline__ void chi_row_body(RowShared &sh, const DevTissue *const *tbl,
                                             const ChiItem *items, uint32_t n_items, uint32_t *queue,
                                             int persistent, double dt, uint32_t kstep, uint32_t tag,
                                             int prio)
{
    static_assert(RW == 16 || RW == 32 || RW == 64, "row width");
    if (prio) __builtin_amdgcn_s_setprio(2);
    constexpr int SM = NET::SM;
    constexpr int LOG_RW = RW == 64 ? 6 : RW == 32 ? 5 : 4;
    ChanEntry *tab = sh.chan;
    double *rng_e = sh.rng_e;
    double *rng_u = sh.rng_u;
    const int lane = threadIdx.x, row = lane >> LOG_RW, lv = lane & (RW - 1);
    uint32_t cursor = blockIdx.x;
    for (;;) {
        const uint32_t it = next_item(queue, persistent != 0, cursor);
        if (it >= n_items) break;
        const ChiItem item = items[it];
        const ItemCtx c = item_ctx(tbl, item, kstep, tag);
        NET net;
        net.load(*c.M);
        load_channel_table<NET>(tab, *c.M);
        const int S = NET::kFixedSpecies ? NET::SM : c.S;

        const bool has_cell = row < (int)c.count;
        uint32_t cell = 0;
        Mesh g{1, 1, 65537};
        long long vbase = 0;
        if (has_cell) {
            cell = (uint32_t)c.T->cell_list[c.first + row];
            g.w = c.T->wh[2 * cell];
            g.h = c.T->wh[2 * cell + 1];
            g.inv_w = 65536 / g.w + 1;
            vbase = (long long)(c.T->vox_off[cell] + lv) * S;
        }
        const bool vox = has_cell && lv < g.w * g.h;
        // the voxel's counts, as integers and as exact doubles
        int32_t xi[SM];
        double xd[SM];
#pragma unroll
        for (int q = 0; q < SM; ++q) {
            xi[q] = (vox && q < S) ? c.counts[vbase + q] : 0;
            xd[q] = (double)xi[q];
        }
        const int deg = vox ? voxel_degree(g, lv) : 0;
        const double degd = (double)deg;
        // cached with the leaf: the channel prefixes and D_s x_s
        double pre[NET::RM + NET::NDM], ad[NET::NDM > 0 ? NET::NDM : 1];
        double leaf = voxel_fold_cached(net, xd, degd, pre, ad);
        if (!vox) leaf = 0.0;  // (a production channel is positive even at zero counts)
        // the lane's present neighbours in jump order (-x, +x, -y, +y), and
        // the jump thresholds' multipliers l for l = 1..3 (+inf past deg - 1,
        // so that the comparison fails as the rule's range ends)
        // (packed: neighbour k in bits 8k .. 8k+7)
        uint32_t nbp = 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) nbp |= (uint32_t)(vox ? neighbour_at(g, lv, k < deg ? k : 0) : lv) << (8 * k);
        double thr[3];
#pragma unroll
        for (int l = 1; l <= 3; ++l) thr[l - 1] = l <= deg - 1 ? (double)l : __builtin_inf();

        double t = 0.0, a0 = 0.0;  // a0: the row's total, rebuilt every iteration
        uint32_t j = 0, ev = 0;
        bool run = has_cell, overflow = false, capped = false;
        // Every running row has drawn exactly once per iteration so far, so
        // its draw ordinal j equals the wave-uniform iteration count.
        for (uint32_t iter = 0;; ++iter) {
            const uint32_t slot = iter & (uint32_t)(RW - 1);
            if (slot == 0u) {
                // draws iter .. iter+RW-1 of the row, one per lane
                if (run) {
                    const tdev::Words4 wds = tdev::philox4x32_10(iter + (uint32_t)lv, c.step, cell,
                                                                 c.tagword, c.key0, c.key1);
                    double u1, uu;
                    tdev::two_uniforms(wds, u1, uu);
                    rng_e[lane] = -tdev::plog(u1);
                    rng_u[lane] = uu;
                }
                __builtin_amdgcn_wave_barrier();
            }
            // this iteration's draw of the row
            const double e1 = rng_e[(row << LOG_RW) | (int)slot];
            const double u2 = rng_u[(row << LOG_RW) | (int)slot];
            __builtin_amdgcn_sched_barrier(0);
            // the sum tree of the row, rebuilt from the leaves (full wave)
            // (the two lowest levels as left and right children directly:
            // quad permutations give every lane both, so the descent needs
            // no swap by the lane's side there)
            const double l0 = dpp_f64<kDppPairLeft>(leaf);
            const double r0 = dpp_f64<kDppPairRight>(leaf);
            const double s1 = l0 + r0;
            const double l1 = dpp_f64<kDppQuadLeft>(s1);
            const double r1 = dpp_f64<kDppQuadRight>(s1);
            const double s2 = l1 + r1;
            const double p2 = dpp_f64<kDppHalfMirror>(s2);
            const double s3 = s2 + p2;
            const double p3 = dpp_f64<kDppRowMirror>(s3);
            a0 = s3 + p3;
            double s4 = 0.0, p4 = 0.0, s5 = 0.0, p5 = 0.0;
            if (RW >= 32) {
                s4 = a0;
                p4 = xlane_f64(s4, 16);
                a0 = s4 + p4;
            }
            if (RW == 64) {
                s5 = a0;
                p5 = xlane_f64(s5, 32);
                a0 = s5 + p5;
            }
            {
                // (without branches: a row with no propensity left stops, a
                // running row at the event cap stops and is flagged)
                const bool live = run & (a0 != 0.0);
                const bool at_cap = live & (ev >= c.cap);
                capped |= at_cap;
                run = live & !at_cap;
            }
            // the draw is waited for only here, after the rebuild (whose
            // exchanges cover the read's latency), and not after the branch
            __builtin_amdgcn_sched_barrier(0);
            asm volatile("" ::"v"(e1), "v"(u2));
            if (!__any(run)) break;
            // the clock, without a branch: the division then overlaps the
            // descent below (a lane that is not running discards it)
            const double tn = t + e1 / a0;
            j += run ? 1u : 0u;
            const bool event = run && !(tn >= dt);
            run = event;
            t = event ? tn : t;
            // which lane's leaf the descent reaches
            const int lvo = opaque(lv);
            double rr = u2 * a0;
            bool on = true;
            if (RW == 64) descent_level(s5, p5, (lvo >> 5) & 1, rr, on);
            if (RW >= 32) descent_level(s4, p4, (lvo >> 4) & 1, rr, on);
            descent_level(s3, p3, (lvo >> 3) & 1, rr, on);
            descent_level(s2, p2, (lvo >> 2) & 1, rr, on);
            descent_children(l1, r1, (lvo >> 1) & 1, rr, on);
            descent_children(l0, r0, lvo & 1, rr, on);
            on = on && event;

            // every lane evaluates the selection on its own voxel (from the
            // prefixes cached by its last fold); only the lane the descent
            // reached applies it
            double resid, a1;
            int sel = voxel_select_cached(net, pre, ad, xd, degd, rr, on, resid, a1);
            sel = sel < NET::RM + NET::NDM ? sel : NET::RM + NET::NDM;
            const ChanEntry e = tab[sel];
            int kdir = 0;
#pragma unroll
            for (int l = 0; l < 3; ++l) kdir += resid >= thr[l] * a1 ? 1 : 0;
            const uint32_t dst = (nbp >> (8 * kdir)) & 0xFFu;
            // the word: bit 0 set, the species times 8 in bits 3..5, the
            // destination lane from bit 8
            uint32_t word = (on && e.spec >= 0) ? (1u | ((uint32_t)e.spec << 3) | (dst << 8)) : 0u;
            // the row's diffusion word reaches every lane of the row (it is
            // zero outside the selected lane): OR over the 16-lane DPP row,
            // then across DPP rows for wider rows
            word = row_or(word);
            if (RW >= 32) word |= xlane_u32(word, 16);
            if (RW == 64) word |= xlane_u32(word, 32);
            // (a word is set only in a row that takes its event)
            const bool recv = (word & 0xFFFFFF01u) == (((uint32_t)lvo << 8) | 1u);
            const uint64_t inc = (uint64_t)(recv ? 1u : 0u) << (word & 0x38u);
            // the source lane's change and the destination's +1 (never the
            // same lane) as one packed change
            const ChanEntry ch{(on ? e.lo : 0u) + (uint32_t)inc, (on ? e.hi : 0u) + (uint32_t)(inc >> 32), -1, 0};
            const bool changed = on || recv;
            uint32_t any_bits = 0u;  // OR of the counts: the range check
#pragma unroll
            for (int q = 0; q < SM; ++q) {
                xi[q] += entry_delta(ch.lo, ch.hi, q);
                xd[q] = (double)xi[q];
                any_bits |= (uint32_t)xi[q];
            }
            overflow |= changed & (any_bits >= (uint32_t)kCountLimit);
            leaf = voxel_fold_cached(net, xd, degd, pre, ad);
            leaf = vox ? leaf : 0.0;
            if (event) ++ev;
            __builtin_amdgcn_wave_barrier();
        }
        if (vox) {
#pragma unroll
            for (int q = 0; q < SM; ++q)
                if (q < S) c.counts[vbase + q] = xi[q];
        }
        // the cell's total propensity now (the last iteration rebuilt every
        // row's tree, and a row's leaves stay put once it stops): the key
        // of the next regroup
        if (has_cell && lv == 0) c.T->load[cell] = (float)a0;
        if (has_cell && lv == 0 && c.T->tr_chi_ev) {
            const uint32_t ts = uni(c.T->trace_steps), nc = uni(c.T->n_cells);
            const size_t slot = (size_t)(c.step % ts) * nc + cell;
            c.T->tr_chi_ev[slot] = tag ? c.T->tr_chi_ev[slot] + ev : ev;  // 2nd half adds
            c.T->tr_chi_t[slot] = (unsigned long long)__double_as_longlong(t);
        }
        item_stats(c, lv == 0 ? ev : 0u, lv == 0 ? j : 0u, overflow, capped, 0);
    }
    leave_queue(queue, persistent != 0);
}


// ---------------------------------------------------------------------------
// chi, compact LDS: G = 1, 2 or 4 lanes per cell of at most 16 G voxels.
// Lane k of a cell's group holds voxels 16k .. 16k+15: their 16 leaf
// propensities (FP64, stored as pairs so one 16-byte read fetches two) and
// their counts as uint16 -- 304 B per lane for 5 species, whatever the cell
// size, so a wavefront holds 64 / G cells and eight wavefronts fit a CU.
// Every event each lane rebuilds the four levels of its own 16-leaf subtree
// in registers; the G subtree sums are combined by one or two DPP exchanges
// inside the group (pair, then quad), which are the heap's upper nodes, so
// every node carries the bits of the P-leaf heap tree (addition is
// commutative, so both lanes of an exchange hold the same sum).  The group's
// lanes draw the same numbers and take the same decisions up to the
// descent; the descent's upper levels pick the one lane whose subtree holds
// the event, which selects and applies the channel in its voxel and
// broadcasts a diffusion jump's destination to the group; the lane holding
// the destination voxel (the same or another) adds the molecule.
// A cell whose count would reach 2^16 abandons its step without writing
// anything back and is queued (retry_items, *retry_count); a follow-up
// launch of the full-width lane kernel redoes that cell-step from the
// unchanged counts in HBM, with identical bits, since a cell-step depends
// only on its starting counts and its counters.
// ---------------------------------------------------------------------------
constexpr int kLane16Leaves = 16;
constexpr int32_t kLane16Limit = 1 << 16;

// LDS of a compact launch: `stride` lanes holding data (cells per item x G).
__host__ __device__ inline size_t lane16_lds_bytes(int S, int stride)
{
    return (size_t)stride * ((size_t)kLane16Leaves * 8 + ((size_t)kLane16Leaves * S + kMaxSpecies) * 2);
}

namespace {

// OR of a 32-bit value over the lane's group of G lanes (G = 2: lane pair,
// G = 4: lane quad); every lane of the group must be active.
template <int G>
__device__ __forceinline__ uint32_t group_or(uint32_t x)
{
    if (G >= 2) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppPairSwap, 0xF, 0xF, false);
    if (G >= 4) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppQuadSwap, 0xF, 0xF, false);
    return x;
}

}  // namespace

// The value of lane k of the lane's group of G lanes (a pair or a quad), for
// a wave-uniform k < G.
template <int G>
__device__ __forceinline__ double group_bcast_f64(double v, uint32_t k)
{
    if (G == 2)
        return k == 0 ? dpp_f64<0xA0>(v) : dpp_f64<0xF5>(v);  // quad_perm [0,0,2,2] / [1,1,3,3]
    if (k == 0) return dpp_f64<0x00>(v);                     // quad_perm [0,0,0,0]
    if (k == 1) return dpp_f64<0x55>(v);                     // [1,1,1,1]
    if (k == 2) return dpp_f64<0xAA>(v);                     // [2,2,2,2]
    return dpp_f64<0xFF>(v);                                 // [3,3,3,3]
}

template <class NET, int G>
__device__ __forceinline__ void chi_lane16_body(unsigned char *lds, const DevTissue *const *tbl,
                                                const ChiItem *items, uint32_t n_items,
                                                uint32_t *queue, int persistent, int cells_per_item,
                                                double dt, uint32_t kstep, uint32_t tag,
                                                ChiItem *retry_items, uint32_t *retry_count, int prio)
{
    static_assert(G == 1 || G == 2 || G == 4, "lanes per cell");
    if (prio) __builtin_amdgcn_s_setprio(2);
    constexpr int SM = NET::SM;
    constexpr int LOG_G = G == 4 ? 2 : G == 2 ? 1 : 0;
    __shared__ ChanEntry tab[kChanSlots];
    const int lane = threadIdx.x;
    const int slot = lane >> LOG_G;   // the lane's cell within the item
    const int sub = lane & (G - 1);   // which 16 voxels of the cell it holds
    const int v0 = kLane16Leaves * sub;
    const int stride = cells_per_item * G;
    uint32_t cursor = blockIdx.x;
    for (;;) {
        const uint32_t it = next_item(queue, persistent != 0, cursor);
        if (it >= n_items) break;
        const ChiItem item = items[it];
        const ItemCtx c = item_ctx(tbl, item, kstep, tag);
        NET net;
        net.load(*c.M);
        load_channel_table<NET>(tab, *c.M);
        const int S = NET::kFixedSpecies ? NET::SM : c.S;
        // leaf pairs: pair k of this lane at lds + (k * stride + lane) * 16
        double *leafp = reinterpret_cast<double *>(lds) + 2 * lane;
        uint16_t *cnt = reinterpret_cast<uint16_t *>(lds + (size_t)stride * kLane16Leaves * 8) + lane;

        const bool active = slot < (int)c.count;
        uint32_t cell = 0;
        Mesh g{1, 1, 65537};
        long long gbase = 0;  // the lane's first count in HBM
        int nloc = 0;         // voxels the lane holds
        bool retry = false;
        if (active) {
            cell = (uint32_t)c.T->cell_list[c.first + slot];
            g.w = c.T->wh[2 * cell];
            g.h = c.T->wh[2 * cell + 1];
            g.inv_w = 65536 / g.w + 1;
            nloc = min(max(g.w * g.h - v0, 0), kLane16Leaves);
            gbase = ((long long)c.T->vox_off[cell] + v0) * S;
            const int n = nloc * S;
            for (int i = 0; i < n; ++i) {
                const int32_t x = c.counts[gbase + i];
                retry |= x >= kLane16Limit;
                cnt[i * stride] = (uint16_t)x;
            }
        }
        if (G > 1) retry = group_or<G>(retry ? 1u : 0u) != 0u;
        double xd[SM];
        if (active && !retry) {
#pragma unroll
            for (int k = 0; k < kLane16Leaves / 2; ++k) {
                double two[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int v = 2 * k + h;
                    two[h] = 0.0;
                    if (v < nloc) {
#pragma unroll
                        for (int q = 0; q < SM; ++q) xd[q] = (double)cnt[(v * S + q) * stride];
                        two[h] = voxel_fold(net, xd, (double)voxel_degree(g, v0 + v));
                    }
                }
                double *sl = leafp + (size_t)k * stride * 2;
                sl[0] = two[0];
                sl[1] = two[1];
            }
        }

        double t = 0.0, last_a0 = 0.0;
        uint32_t j = 0, ev = 0;
        bool capped = false;
        if (active && !retry) {
            // Draws: with G lanes per cell, lane k of the group makes the
            // draw of every ordinal = k (mod G), G at a time, and the group
            // reads ordinal j's from its lane j mod G.  Every running group
            // has made exactly one draw per iteration, so j is wave-uniform.
            double e1, u2, eo = 0.0, uo = 0.0;
            {
                const tdev::Words4 wds = tdev::philox4x32_10((uint32_t)(G > 1 ? sub : 0), c.step, cell,
                                                             c.tagword, c.key0, c.key1);
                double u1;
                tdev::two_uniforms(wds, u1, uo);
                eo = -tdev::plog<true>(u1);
                e1 = eo;
                u2 = uo;
                if (G > 1) {
                    e1 = group_bcast_f64<G>(eo, 0u);
                    u2 = group_bcast_f64<G>(uo, 0u);
                }
            }
            // (it: the iteration, wave-uniform; a running cell has drawn
            // it + 1 times after this iteration's draw)
            for (uint32_t it = 0;; ++it) {
                // the lane's 16 leaves and the levels of its subtree
                double l[kLane16Leaves];
#pragma unroll
                for (int k = 0; k < kLane16Leaves / 2; ++k) {
                    const double *sl = leafp + (size_t)k * stride * 2;
                    l[2 * k] = sl[0];
                    l[2 * k + 1] = sl[1];
                }
                double q1[8], q2[4], q3[2];
#pragma unroll
                for (int k = 0; k < 8; ++k) q1[k] = l[2 * k] + l[2 * k + 1];
#pragma unroll
                for (int k = 0; k < 4; ++k) q2[k] = q1[2 * k] + q1[2 * k + 1];
#pragma unroll
                for (int k = 0; k < 2; ++k) q3[k] = q2[2 * k] + q2[2 * k + 1];
                // the heap's nodes above the lanes' subtrees: the pair's sum
                // (G >= 2), then the quad's (G = 4)
                const double s = q3[0] + q3[1];
                double a0 = s, p1 = 0.0, hs = s, p2 = 0.0;
                if (G >= 2) {
                    p1 = dpp_f64<kDppPairSwap>(s);
                    hs = s + p1;
                    a0 = hs;
                }
                if (G == 4) {
                    p2 = dpp_f64<kDppQuadSwap>(hs);
                    a0 = hs + p2;
                }
                last_a0 = a0;
                // a cell with no propensity left, or at the event cap, stops
                // at the single exit below with the cells whose next event
                // falls past the interval (its draw and descent are
                // discarded, and only read memory)
                const bool live = a0 != 0.0;
                const bool at_cap = live && ev >= c.cap;
                capped = capped || at_cap;
                const bool go = live && !at_cap;
                j += go ? 1u : 0u;
                // the clock; the stop test waits until after the descent,
                // which the division then overlaps (the descent only reads)
                const double tn = t + e1 / a0;
                double r = u2 * a0;
                if (G == 1) {
                    const tdev::Words4 wds = tdev::philox4x32_10(j, c.step, cell, c.tagword, c.key0, c.key1);
                    double u1;
                    tdev::two_uniforms(wds, u1, u2);
                    e1 = -tdev::plog<true>(u1);
                } else {
                    const uint32_t k = (it + 1u) & (uint32_t)(G - 1);
                    if (k == 0) {  // the next G ordinals, one per lane of the group
                        const tdev::Words4 wds = tdev::philox4x32_10(j + (uint32_t)sub, c.step, cell,
                                                                     c.tagword, c.key0, c.key1);
                        double u1;
                        tdev::two_uniforms(wds, u1, uo);
                        eo = -tdev::plog<true>(u1);
                    }
                    e1 = group_bcast_f64<G>(eo, k);
                    u2 = group_bcast_f64<G>(uo, k);
                }
                // descent through the group's levels: only the lane whose
                // subtree the path enters stays `on`
                bool on = true;
                if (G == 4) descent_level(hs, p2, sub >> 1, r, on);
                if (G >= 2) descent_level(s, p1, sub & 1, r, on);
                // descent inside the subtree: left if r < L or R == 0, else
                // r -= L and right
                int v = 0;
                {
                    double L = q3[0], R = q3[1];
                    bool left = (r < L) || (R == 0.0);
                    r = left ? r : r - L;
                    const int b3 = left ? 0 : 1;
                    L = b3 ? q2[2] : q2[0];
                    R = b3 ? q2[3] : q2[1];
                    left = (r < L) || (R == 0.0);
                    r = left ? r : r - L;
                    const int i2 = 2 * b3 + (left ? 0 : 1);
                    // the two lower levels from the four leaves under node
                    // i2, read back by address (the same pairwise sums as
                    // q1, so the same bits) rather than selected among
                    // registers
                    const double *pa = leafp + (size_t)(2 * i2) * stride * 2;
                    const double *pb = pa + (size_t)stride * 2;
                    const double la0 = pa[0], la1 = pa[1], lb0 = pb[0], lb1 = pb[1];
                    L = la0 + la1;
                    R = lb0 + lb1;
                    left = (r < L) || (R == 0.0);
                    r = left ? r : r - L;
                    const int i1 = 2 * i2 + (left ? 0 : 1);
                    L = left ? la0 : lb0;
                    R = left ? la1 : lb1;
                    left = (r < L) || (R == 0.0);
                    r = left ? r : r - L;
                    v = 2 * i1 + (left ? 0 : 1);
                }
                if (!go || tn >= dt) break;
                t = tn;

                const Mesh gm{opaque(g.w), opaque(g.h), opaque(g.inv_w)};
                bool wide = false;
                uint32_t word = 0;  // a jump: 1 | species << 4 | destination voxel << 8
                if (on) {
                    uint16_t *x = cnt + v * S * stride;
                    int32_t xi[SM];
#pragma unroll
                    for (int q = 0; q < SM; ++q) {
                        xi[q] = x[q * stride];
                        xd[q] = (double)xi[q];
                    }
                    const int deg = voxel_degree(gm, v0 + v);
                    double resid, a1;
                    const int sel = voxel_select(net, xd, (double)deg, r, resid, a1);
                    const ChanEntry e = tab[sel];
                    uint32_t any_bits = 0u;  // OR of the counts: the range check
#pragma unroll
                    for (int q = 0; q < SM; ++q) {
                        if (q < S) {
                            xi[q] += entry_delta(e.lo, e.hi, q);
                            x[q * stride] = (uint16_t)xi[q];
                            xd[q] = (double)xi[q];
                            any_bits |= (uint32_t)xi[q];
                        }
                    }
                    wide = any_bits >= (uint32_t)kLane16Limit;
                    if (e.spec >= 0) {
                        const int dst = neighbour_at(gm, v0 + v, jump_direction(resid, a1, deg));
                        word = 1u | ((uint32_t)e.spec << 4) | ((uint32_t)dst << 8);
                    }
                    leafp[(size_t)(v >> 1) * stride * 2 + (v & 1)] = voxel_fold(net, xd, (double)deg);
                }
                if (G > 1) word = group_or<G>(word);
                // the lane holding the jump's destination voxel adds the
                // molecule and refolds that voxel
                const int dv = (int)(word >> 8) - v0;
                if ((word & 1u) && dv >= 0 && dv < kLane16Leaves) {
                    const int spec = (int)((word >> 4) & 15u);
                    uint16_t *xdst = cnt + (dv * S + spec) * stride;
                    const int32_t nd = (int32_t)*xdst + 1;
                    wide |= nd >= kLane16Limit;
                    *xdst = (uint16_t)nd;
#pragma unroll
                    for (int q = 0; q < SM; ++q) xd[q] = (double)cnt[(dv * S + q) * stride];
                    leafp[(size_t)(dv >> 1) * stride * 2 + (dv & 1)] =
                        voxel_fold(net, xd, (double)voxel_degree(gm, v0 + dv));
                }
                if (G > 1) wide = group_or<G>(wide ? 1u : 0u) != 0u;
                if (wide) {  // redo this cell-step at full width
                    retry = true;
                    break;
                }
                ++ev;
            }
        }
        if (active && retry) {
            if (sub == 0) {
                const uint32_t at = atomicAdd(retry_count, 1u);
                retry_items[at] = ChiItem{item.tissue, c.first + (uint32_t)slot, 1u, item.model};
            }
        } else if (active) {
            const int n = nloc * S;
            for (int i = 0; i < n; ++i) c.counts[gbase + i] = (int32_t)cnt[i * stride];
            if (sub == 0 && c.T->tr_chi_ev) {
                const uint32_t ts = uni(c.T->trace_steps), nc = uni(c.T->n_cells);
                const size_t at = (size_t)(c.step % ts) * nc + cell;
                c.T->tr_chi_ev[at] = tag ? c.T->tr_chi_ev[at] + ev : ev;  // 2nd half adds
                c.T->tr_chi_t[at] = (unsigned long long)__double_as_longlong(t);
            }
            // the cell's total propensity now: the key of the next regroup
            if (sub == 0) c.T->load[cell] = (float)last_a0;
        }
        const bool counted = active && !retry && sub == 0;
        item_stats(c, counted ? ev : 0u, counted ? j : 0u, false, capped && counted, 0);
    }
    leave_queue(queue, persistent != 0);
}


// ---------------------------------------------------------------------------
// chi, compact layout with one lane per cell of at most 16 voxels, with lane
// refill (compiled networks, persistent launches).  A wavefront's lanes do not
// wait for the busiest cell of their work item: a lane whose cell-step ends
// keeps its results in LDS, and once at least `refill_min` lanes are idle
// (or all of them) the wavefront writes those cells back and hands the idle
// lanes the next cells of the launch's items, which it takes from the queue
// one item at a time.  So lanes hold cells of different items, tissues and
// rate sets at once: everything a cell needs -- its tissue, counter words,
// key schedule and rates -- lives in the lane's registers.  A cell-step is the
// same sequence of operations on the same values as in the compact layout
// above (the same contract: its draws depend only on its counters), so the
// bits are the same; only the order in which cells finish differs.
// Cells that reach 2^16 molecules are handed to the full-width redo as above.
// ---------------------------------------------------------------------------
namespace {

// The channel table of a compiled network from its compile-time structure.
template <class NET>
__device__ __forceinline__ void compiled_channel_table(ChanEntry *tab)
{
    constexpr int RM = NET::RM, NDM = NET::NDM;
    const NET n{};
    const int k = threadIdx.x;
    if (k <= RM + NDM) {
        ChanEntry e{0u, 0u, -1, 0};
#pragma unroll
        for (int r = 0; r < RM; ++r)
            if (k == r) {
#pragma unroll
                for (int s = 0; s < NET::SM; ++s) {
                    const uint32_t byte = (uint32_t)(uint8_t)(int8_t)n.delta(r, s);
                    if (s < 4) e.lo |= byte << (8 * s);
                    else e.hi |= byte << (8 * (s - 4));
                }
            }
#pragma unroll
        for (int q = 0; q < NDM; ++q)
            if (k == RM + q) {
                const int sp = n.dsp(q);
                e.spec = sp;
                if (sp < 4) e.lo = 0xFFu << (8 * sp);
                else e.hi = 0xFFu << (8 * (sp - 4));
            }
        tab[k] = e;
    }
    __builtin_amdgcn_wave_barrier();
}

// Philox4x32-10 with the key schedule precomputed (rk0[r], rk1[r]: the key
// words of round r), for keys held per lane.
__device__ __forceinline__ tdev::Words4 philox_rk(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                  const uint32_t *rk0, const uint32_t *rk1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ rk0[round];
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ rk1[round];
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
    }
    return tdev::Words4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

}  // namespace

template <class NET>
__device__ __forceinline__ void chi_refill_body(unsigned char *lds, const DevTissue *const *tbl,
                                                const ChiItem *items, uint32_t n_items,
                                                uint32_t *queue, int persistent, double dt,
                                                uint32_t kstep, uint32_t tag, ChiItem *retry_items,
                                                uint32_t *retry_count, int refill_min)
{
    static_assert(NET::kFixedSpecies, "lane refill runs compiled networks only");
    constexpr int SM = NET::SM, S = NET::SM;
    constexpr int stride = kWave;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
    __shared__ ChanEntry tab[kChanSlots];
    compiled_channel_table<NET>(tab);
    const int lane = threadIdx.x;
    double *leafp = reinterpret_cast<double *>(lds) + 2 * lane;
    uint16_t *cnt = reinterpret_cast<uint16_t *>(lds + (size_t)stride * kLane16Leaves * 8) + lane;

    // the wavefront's item being handed out (wave-uniform)
    uint32_t cursor = blockIdx.x;
    uint32_t pend_next = 0, pend_count = 0, pend_tissue = 0, pend_first = 0, pend_model = 0;
    bool drained = false;

    // the lane's cell
    bool has = false, fin = false, retry = false, capped = false;
    const DevTissue *T = nullptr;
    uint32_t tix = 0, model = 0, lidx = 0, cell = 0, step = 0, tagword = 0, cap = 0;
    uint32_t rk0[10], rk1[10];
    Mesh g{1, 1, 65537};
    int nloc = 0;
    long long gbase = 0;
    NET net;
    double t = 0.0, last_a0 = 0.0, e1 = 0.0, u2 = 0.0;
    uint32_t j = 0, ev = 0;
    double xd[SM];

    for (;;) {
        const uint64_t idle = __ballot(!has || fin);
        const int n_idle = __popcll(idle);
        if (n_idle == kWave || (!drained && n_idle >= refill_min)) {
            // write the finished cells back
            if (fin) {
                if (retry) {
                    const uint32_t at = atomicAdd(retry_count, 1u);
                    retry_items[at] = ChiItem{tix, lidx, 1u, model};
                } else {
                    int32_t *counts = T->counts;
                    const int n = nloc * S;
                    for (int i = 0; i < n; ++i) counts[gbase + i] = (int32_t)cnt[i * stride];
                    if (T->tr_chi_ev) {
                        const uint32_t ts = T->trace_steps, nc = T->n_cells;
                        const size_t at = (size_t)(step % ts) * nc + cell;
                        T->tr_chi_ev[at] = tag ? T->tr_chi_ev[at] + ev : ev;  // 2nd half adds
                        T->tr_chi_t[at] = (unsigned long long)__double_as_longlong(t);
                    }
                    T->load[cell] = (float)last_a0;  // the key of the next regroup
                }
            }
            // their totals, summed per tissue across the wavefront
            uint64_t todo = __ballot(fin && !retry);
            while (todo) {
                const int leader = __builtin_ctzll(todo);
                const uint32_t lt = (uint32_t)__builtin_amdgcn_readlane((int)tix, leader);
                const bool mine = fin && !retry && tix == lt;
                const uint32_t ev_sum = wave_sum_u32(mine ? ev : 0u);
                const uint32_t dr_sum = wave_sum_u32(mine ? j : 0u);
                const bool any_cap = __any(mine && capped);
                if (lane == leader) {
                    if (ev_sum) atomicAdd(T->stats + 0, (unsigned long long)ev_sum);
                    if (dr_sum) atomicAdd(T->stats + 2, (unsigned long long)dr_sum);
                    if (any_cap) atomicOr(T->flags + 1, 1u);
                }
                todo &= ~__ballot(mine);
            }
            has = has && !fin;
            fin = false;
            // hand the idle lanes the next cells
            bool got = false;
            while (!drained) {
                const uint64_t free = __ballot(!has);
                if (free == 0) break;
                if (pend_next >= pend_count) {
                    const uint32_t it = next_item(queue, persistent != 0, cursor);
                    if (it >= n_items) {
                        drained = true;
                        break;
                    }
                    const ChiItem item = items[it];
                    pend_tissue = uni(item.tissue);
                    pend_first = uni(item.first);
                    pend_count = uni(item.count);
                    pend_model = uni(item.model);
                    pend_next = 0;
                }
                const uint32_t rank = lanes_below(free);
                const uint32_t avail = pend_count - pend_next;
                if (!has && rank < avail) {
                    has = true;
                    got = true;
                    tix = pend_tissue;
                    model = pend_model;
                    lidx = pend_first + pend_next + rank;
                }
                pend_next += min(avail, (uint32_t)__popcll(free));
            }
            // the new cells: context, counts, leaves, first draw
            if (got) {
                T = tbl[tix];
                const DevModel *M = T->models + model;
                net.load(*M);
                step = T->step_base + kstep;
                const uint64_t seed = (uint64_t)T->seed;
                uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
                for (int r = 0; r < 10; ++r) {
                    rk0[r] = k0;
                    rk1[r] = k1;
                    k0 += kWeylA;
                    k1 += kWeylB;
                }
                tagword = (T->sim_id << 2) | tag;
                cap = T->event_cap;
                cell = (uint32_t)T->cell_list[lidx];
                g.w = T->wh[2 * cell];
                g.h = T->wh[2 * cell + 1];
                g.inv_w = 65536 / g.w + 1;
                nloc = min(g.w * g.h, kLane16Leaves);
                gbase = (long long)T->vox_off[cell] * S;
                const int32_t *counts = T->counts;
                retry = false;
                const int n = nloc * S;
                for (int i = 0; i < n; ++i) {
                    const int32_t x = counts[gbase + i];
                    retry |= x >= kLane16Limit;
                    cnt[i * stride] = (uint16_t)x;
                }
                t = 0.0;
                last_a0 = 0.0;
                j = 0;
                ev = 0;
                capped = false;
                fin = retry;  // a cell over 16 bits goes to the redo untouched
                if (!retry) {
#pragma unroll
                    for (int k = 0; k < kLane16Leaves / 2; ++k) {
                        double two[2];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int v = 2 * k + h;
                            two[h] = 0.0;
                            if (v < nloc) {
#pragma unroll
                                for (int q = 0; q < SM; ++q) xd[q] = (double)cnt[(v * S + q) * stride];
                                two[h] = voxel_fold(net, xd, (double)voxel_degree(g, v));
                            }
                        }
                        double *sl = leafp + (size_t)k * stride * 2;
                        sl[0] = two[0];
                        sl[1] = two[1];
                    }
                    const tdev::Words4 wds = philox_rk(0u, step, cell, tagword, rk0, rk1);
                    double u1;
                    tdev::two_uniforms(wds, u1, u2);
                    e1 = -tdev::plog<true>(u1);
                }
            }
            if (!__any(has)) break;
        }
        if (has && !fin) {
            // one event of the lane's cell: the 16 leaves and the subtree levels
            double l[kLane16Leaves];
#pragma unroll
            for (int k = 0; k < kLane16Leaves / 2; ++k) {
                const double *sl = leafp + (size_t)k * stride * 2;
                l[2 * k] = sl[0];
                l[2 * k + 1] = sl[1];
            }
            double q1[8], q2[4], q3[2];
#pragma unroll
            for (int k = 0; k < 8; ++k) q1[k] = l[2 * k] + l[2 * k + 1];
#pragma unroll
            for (int k = 0; k < 4; ++k) q2[k] = q1[2 * k] + q1[2 * k + 1];
#pragma unroll
            for (int k = 0; k < 2; ++k) q3[k] = q2[2 * k] + q2[2 * k + 1];
            const double a0 = q3[0] + q3[1];
            last_a0 = a0;
            const bool live = a0 != 0.0;
            const bool at_cap = live && ev >= cap;
            capped = capped || at_cap;
            const bool go = live && !at_cap;
            j += go ? 1u : 0u;
            // the clock; the stop test waits until after the descent (which
            // only reads) so that the division overlaps it
            const double tn = t + e1 / a0;
            double r = u2 * a0;
            {
                const tdev::Words4 wds = philox_rk(j, step, cell, tagword, rk0, rk1);
                double u1;
                tdev::two_uniforms(wds, u1, u2);
                e1 = -tdev::plog<true>(u1);
            }
            int v = 0;
            {
                double L = q3[0], R = q3[1];
                bool left = (r < L) || (R == 0.0);
                r = left ? r : r - L;
                const int b3 = left ? 0 : 1;
                L = b3 ? q2[2] : q2[0];
                R = b3 ? q2[3] : q2[1];
                left = (r < L) || (R == 0.0);
                r = left ? r : r - L;
                const int i2 = 2 * b3 + (left ? 0 : 1);
                const double *pa = leafp + (size_t)(2 * i2) * stride * 2;
                const double *pb = pa + (size_t)stride * 2;
                const double la0 = pa[0], la1 = pa[1], lb0 = pb[0], lb1 = pb[1];
                L = la0 + la1;
                R = lb0 + lb1;
                left = (r < L) || (R == 0.0);
                r = left ? r : r - L;
                const int i1 = 2 * i2 + (left ? 0 : 1);
                L = left ? la0 : lb0;
                R = left ? la1 : lb1;
                left = (r < L) || (R == 0.0);
                r = left ? r : r - L;
                v = 2 * i1 + (left ? 0 : 1);
            }
            if (!go || tn >= dt) {
                fin = true;
            } else {
                t = tn;
                const Mesh gm{opaque(g.w), opaque(g.h), opaque(g.inv_w)};
                uint16_t *x = cnt + v * S * stride;
                int32_t xi[SM];
#pragma unroll
                for (int q = 0; q < SM; ++q) {
                    xi[q] = x[q * stride];
                    xd[q] = (double)xi[q];
                }
                const int deg = voxel_degree(gm, v);
                double resid, a1;
                const int sel = voxel_select(net, xd, (double)deg, r, resid, a1);
                const ChanEntry e = tab[sel];
                uint32_t any_bits = 0u;  // OR of the counts: the range check
#pragma unroll
                for (int q = 0; q < SM; ++q) {
                    xi[q] += entry_delta(e.lo, e.hi, q);
                    x[q * stride] = (uint16_t)xi[q];
                    xd[q] = (double)xi[q];
                    any_bits |= (uint32_t)xi[q];
                }
                bool wide = any_bits >= (uint32_t)kLane16Limit;
                leafp[(size_t)(v >> 1) * stride * 2 + (v & 1)] = voxel_fold(net, xd, (double)deg);
                if (e.spec >= 0) {
                    const int dv = neighbour_at(gm, v, jump_direction(resid, a1, deg));
                    uint16_t *xdst = cnt + (dv * S + e.spec) * stride;
                    const int32_t nd = (int32_t)*xdst + 1;
                    wide |= nd >= kLane16Limit;
                    *xdst = (uint16_t)nd;
#pragma unroll
                    for (int q = 0; q < SM; ++q) xd[q] = (double)cnt[(dv * S + q) * stride];
                    leafp[(size_t)(dv >> 1) * stride * 2 + (dv & 1)] =
                        voxel_fold(net, xd, (double)voxel_degree(gm, dv));
                }
                if (wide) {  // redo this cell-step at full width
                    retry = true;
                    fin = true;
                } else {
                    ++ev;
                }
            }
        }
    }
    leave_queue(queue, persistent != 0);
}
}  // namespace tissue_impl
