// kernels.hip -- the two operators of one splitting step on gfx950.
//
// chi (internal cell dynamics; paper: Algorithm section, "Internal cell
// dynamics module", chi updates each cell independently over dt): one lane
// per cell runs Gillespie's direct method over the cell's voxels.  The
// lane's counts (int32) and its binary sum tree of voxel propensities (FP64)
// live in LDS, laid out field-major with the lane index fastest so that 64
// lanes touching "their" element of a field hit 64 distinct banks.
//
// S (cell signalling; paper: "Cell signaling module" and the translation
// scripts, Results > Model: Delta within reach of a single shared face turns
// into the neighbour's NICD): one lane per lattice edge gathers N, D, I of
// the two facing membrane groups, runs the pairwise SSA over dt and scatters
// the counts back.  Edges of one launch touch disjoint state (a colour class
// is a matching; with disjoint face groups all classes may share a launch).
//
// Both kernels take work items (<= 64 cells or edges of one tissue) either
// one per workgroup or, in persistent mode, from a device queue that every
// workgroup pulls from until it is empty; the last workgroup to leave clears
// the queue for the next launch.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "internal.h"
#include "kernels.h"

namespace tissue_impl {
namespace {

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Next work item for this workgroup (one wavefront).
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
// resets the queue and the exit counter (queue[0], queue[1]).
__device__ __forceinline__ void leave_queue(uint32_t *queue, bool persistent)
{
    if (!persistent) return;
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(queue + 1, 1u);
        if (done == gridDim.x - 1) {
            atomicExch(queue, 0u);
            atomicExch(queue + 1, 0u);
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

// The network of one tissue, in scalar registers.  Loops over it are
// fully unrolled to the table sizes with uniform guards, so every index is
// a compile-time constant.
struct ModelR {
    int S, R, ND;
    int ra[kMaxReactions], rb[kMaxReactions];
    uint32_t code[kMaxReactions];
    double rate[kMaxReactions];
    int dsp[kMaxSpecies];
    double drate[kMaxSpecies];
};

__device__ __forceinline__ void load_model(const DevModel &M, ModelR &m)
{
    m.S = uni(M.n_species);
    m.R = uni(M.n_reactions);
    m.ND = uni(M.n_diff);
#pragma unroll
    for (int r = 0; r < kMaxReactions; ++r) {
        m.ra[r] = uni((int)M.reac_a[r]);
        m.rb[r] = uni((int)M.reac_b[r]);
        m.code[r] = uni(M.change_code[r]);
        m.rate[r] = uni(M.rates[r]);
    }
#pragma unroll
    for (int q = 0; q < kMaxSpecies; ++q) {
        m.dsp[q] = uni((int)M.diff_species[q]);
        m.drate[q] = uni(M.diff_rate[q]);
    }
}

// Mass-action propensity of reaction r; x points at species 0 of a voxel,
// species s at x[s * stride].
__device__ __forceinline__ double reaction_propensity(const ModelR &m, int r, const int32_t *x,
                                                      int stride)
{
    const int a = m.ra[r], b = m.rb[r];
    const double c = m.rate[r];
    if (a < 0) return c;
    const long long xa = x[a * stride];
    if (b < 0) return c * (double)xa;
    if (a == b) return c * (double)(xa * (xa - 1) / 2);
    return c * (double)(xa * (long long)x[b * stride]);
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

// Propensity of voxel v: left fold over reactions, then diffusion channels.
__device__ __forceinline__ double voxel_propensity(const ModelR &m, const int32_t *cnt, int stride,
                                                   int v, const Mesh &g)
{
    const int32_t *x = cnt + v * m.S * stride;
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < kMaxReactions; ++r)
        if (r < m.R) acc = acc + reaction_propensity(m, r, x, stride);
    const int deg = voxel_degree(g, v);
    if (deg > 0) {
#pragma unroll
        for (int q = 0; q < kMaxSpecies; ++q)
            if (q < m.ND) {
                const long long xs = x[m.dsp[q] * stride];
                acc = acc + m.drate[q] * (double)(xs * deg);
            }
    }
    return acc;
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

template <int P>
__device__ __forceinline__ void update_path(double *tree, int stride, int leaf)
{
    int n = (P + leaf) >> 1;
#pragma unroll
    for (int lvl = 0; lvl < 7; ++lvl) {
        if ((1 << lvl) >= P) break;
        tree[n * stride] = tree[(2 * n) * stride] + tree[(2 * n + 1) * stride];
        n >>= 1;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// chi: one lane per cell, P = leaf count of the sum tree (power of two >= V)
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kWave) void chi_kernel(const DevTissue *const *tbl,
                                                    const ChiItem *items, uint32_t n_items,
                                                    uint32_t *queue, int persistent,
                                                    int cells_per_item, double dt,
                                                    uint32_t kstep)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x;
    const int stride = cells_per_item;
    uint32_t cursor = blockIdx.x;
    for (;;) {
        const uint32_t it = next_item(queue, persistent != 0, cursor);
        if (it >= n_items) break;
        const ChiItem item = items[it];
        const DevTissue *T = tbl[uni(item.tissue)];
        ModelR m;
        load_model(T->model, m);
        const int S = m.S;
        const uint32_t first = uni(item.first), count = uni(item.count);
        const uint32_t step = uni(T->step_base) + kstep;
        const uint64_t seed = uni((uint64_t)T->seed);
        const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
        const uint32_t tagword = (uni(T->sim_id) << 2) | 0u;
        const uint32_t cap = uni(T->event_cap);
        int32_t *counts = T->counts;
        double *tree = reinterpret_cast<double *>(lds) + lane;  // [2P][stride]
        int32_t *cnt = reinterpret_cast<int32_t *>(lds + (size_t)2 * P * stride * 8) + lane;

        const bool active = lane < (int)count;
        uint32_t cell = 0;
        Mesh g{1, 1, 65537};
        long long gbase = 0;
        if (active) {
            cell = (uint32_t)T->cell_list[first + lane];
            g.w = T->wh[2 * cell];
            g.h = T->wh[2 * cell + 1];
            g.inv_w = 65536 / g.w + 1;
            gbase = (long long)T->vox_off[cell] * S;
            const int n = g.w * g.h * S;
            for (int i = 0; i < n; ++i) cnt[i * stride] = counts[gbase + i];
        }
        const int V = g.w * g.h;

        // leaves and internal nodes
        if (active) {
#pragma unroll
            for (int v = 0; v < P; ++v)
                tree[(P + v) * stride] = v < V ? voxel_propensity(m, cnt, stride, v, g) : 0.0;
#pragma unroll
            for (int n = P - 1; n >= 1; --n)
                tree[n * stride] = tree[(2 * n) * stride] + tree[(2 * n + 1) * stride];
        }

        double t = 0.0;
        uint32_t j = 0, ev = 0;
        bool overflow = false, capped = false;
        if (active) {
            for (;;) {
                const double a0 = tree[1 * stride];
                if (a0 == 0.0) break;
                if (ev >= cap) {
                    capped = true;
                    break;
                }
                const tdev::Words4 wds = tdev::philox4x32_10(j, step, cell, tagword, key0, key1);
                ++j;
                double u1, u2;
                tdev::two_uniforms(wds, u1, u2);
                const double tau = (-tdev::plog(u1)) / a0;
                const double tn = t + tau;
                if (tn >= dt) break;
                t = tn;
                double r = u2 * a0;

                // descend the sum tree
                int n = 1;
#pragma unroll
                for (int lvl = 0; lvl < 7; ++lvl) {
                    if ((1 << lvl) >= P) break;
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

                // channel of voxel v: first with a_k > 0 and r < prefix
                // through k, else the last with a_k > 0
                int32_t *x = cnt + v * S * stride;
                const int deg = voxel_degree(g, v);
                double prefix = 0.0, resid = 0.0, last_prefix = 0.0;
                int sel = -1, last = -1;
#pragma unroll
                for (int k = 0; k < kMaxReactions; ++k) {
                    if (k < m.R) {
                        const double a = reaction_propensity(m, k, x, stride);
                        const double next = prefix + a;
                        if (a > 0.0) {
                            if (sel < 0 && r < next) {
                                sel = k;
                                resid = r - prefix;
                            }
                            last = k;
                            last_prefix = prefix;
                        }
                        prefix = next;
                    }
                }
                if (deg > 0) {
#pragma unroll
                    for (int q = 0; q < kMaxSpecies; ++q) {
                        if (q < m.ND) {
                            const long long xs = x[m.dsp[q] * stride];
                            const double a = m.drate[q] * (double)(xs * deg);
                            const double next = prefix + a;
                            if (a > 0.0) {
                                if (sel < 0 && r < next) {
                                    sel = kMaxReactions + q;
                                    resid = r - prefix;
                                }
                                last = kMaxReactions + q;
                                last_prefix = prefix;
                            }
                            prefix = next;
                        }
                    }
                }
                if (sel < 0) {
                    sel = last;
                    resid = r - last_prefix;
                }

                int dst = v;
                if (sel < kMaxReactions) {
                    uint32_t code = 0;
#pragma unroll
                    for (int k = 0; k < kMaxReactions; ++k)
                        if (k == sel) code = m.code[k];
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const uint32_t byte = (code >> (8 * b)) & 0xFFu;
                        const int delta = (int)(byte & 31u) - 16;
                        if (delta != 0) {
                            const int s = (int)(byte >> 5);
                            const int32_t nv = x[s * stride] + delta;
                            x[s * stride] = nv;
                            overflow |= (nv < 0) | (nv >= kCountLimit);
                        }
                    }
                } else {
                    int s = 0;
                    double D = 0.0;
#pragma unroll
                    for (int q = 0; q < kMaxSpecies; ++q)
                        if (kMaxReactions + q == sel) {
                            s = m.dsp[q];
                            D = m.drate[q];
                        }
                    const double a1 = D * (double)(long long)x[s * stride];
                    int kdir = 0;
#pragma unroll
                    for (int l = 1; l <= 3; ++l)
                        if (l <= deg - 1 && resid >= (double)l * a1) ++kdir;
                    dst = neighbour_at(g, v, kdir);
                    const int32_t nsrc = x[s * stride] - 1;
                    x[s * stride] = nsrc;
                    int32_t *xd = cnt + (dst * S + s) * stride;
                    const int32_t ndst = *xd + 1;
                    *xd = ndst;
                    overflow |= (nsrc < 0) | (ndst >= kCountLimit);
                }
                tree[(P + v) * stride] = voxel_propensity(m, cnt, stride, v, g);
                if (dst != v) tree[(P + dst) * stride] = voxel_propensity(m, cnt, stride, dst, g);
                update_path<P>(tree, stride, v);
                if (dst != v) update_path<P>(tree, stride, dst);
                ++ev;
            }
            const int n = V * S;
            for (int i = 0; i < n; ++i) counts[gbase + i] = cnt[i * stride];
            if (T->tr_chi_ev) {
                const uint32_t ts = uni(T->trace_steps), nc = uni(T->n_cells);
                const size_t slot = (size_t)(step % ts) * nc + cell;
                T->tr_chi_ev[slot] = ev;
                T->tr_chi_t[slot] = (unsigned long long)__double_as_longlong(t);
            }
        }
        const uint32_t ev_sum = wave_sum_u32(ev);
        const uint32_t dr_sum = wave_sum_u32(j);
        const bool any_over = __any(overflow);
        const bool any_cap = __any(capped);
        if (lane == 0) {
            if (ev_sum) atomicAdd(T->stats + 0, (unsigned long long)ev_sum);
            if (dr_sum) atomicAdd(T->stats + 2, (unsigned long long)dr_sum);
            if (any_over) atomicOr(T->flags + 0, 1u);
            if (any_cap) atomicOr(T->flags + 1, 1u);
        }
    }
    leave_queue(queue, persistent != 0);
}

// ---------------------------------------------------------------------------
// S: one lane per edge
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWave) void s_kernel(const DevTissue *const *tbl, const SItem *items,
                                                  uint32_t n_items, uint32_t *queue,
                                                  int persistent, double dt, uint32_t kstep)
{
    // per lane: N, D, I of face A (cell i) then of face B (cell j)
    __shared__ int32_t fa[3][kMaxFace][kWave];
    __shared__ int32_t fb[3][kMaxFace][kWave];
    const int lane = threadIdx.x;
    uint32_t cursor = blockIdx.x;
    for (;;) {
        const uint32_t it = next_item(queue, persistent != 0, cursor);
        if (it >= n_items) break;
        const SItem item = items[it];
        const DevTissue *T = tbl[uni(item.tissue)];
        const int S = uni(T->model.n_species);
        const int sp0 = uni(T->model.trans_n), sp1 = uni(T->model.trans_d), sp2 = uni(T->model.trans_i);
        const double c = uni(T->model.trans_rate);
        const uint32_t first = uni(item.first), count = uni(item.count);
        const uint32_t step = uni(T->step_base) + kstep;
        const uint64_t seed = uni((uint64_t)T->seed);
        const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
        const uint32_t tagword = (uni(T->sim_id) << 2) | 1u;
        const uint32_t cap = uni(T->event_cap);
        int32_t *counts = T->counts;
        const bool active = lane < (int)count;
        const uint32_t e = first + lane;
        double t = 0.0;
        uint32_t j = 0, ev = 0;
        bool overflow = false, capped = false;
        if (active) {
            const EdgeRec *er = T->edges + e;
            const int mA = er->m_a, mB = er->m_b;
            const long long gi = (long long)er->vox_i, gj = (long long)er->vox_j;
            uint8_t A[kMaxFace], B[kMaxFace];
#pragma unroll
            for (int a = 0; a < kMaxFace; ++a) {
                A[a] = er->A[a];
                B[a] = er->B[a];
            }
#pragma unroll
            for (int a = 0; a < kMaxFace; ++a)
                if (a < mA) {
                    const long long g = (gi + A[a]) * S;
                    fa[0][a][lane] = counts[g + sp0];
                    fa[1][a][lane] = counts[g + sp1];
                    fa[2][a][lane] = counts[g + sp2];
                }
#pragma unroll
            for (int b = 0; b < kMaxFace; ++b)
                if (b < mB) {
                    const long long g = (gj + B[b]) * S;
                    fb[0][b][lane] = counts[g + sp0];
                    fb[1][b][lane] = counts[g + sp1];
                    fb[2][b][lane] = counts[g + sp2];
                }
            const int half = mA * mB;
            for (;;) {
                // channels: N_i(a) D_j(b) for a, b; then N_j(b) D_i(a) for b, a
                double a0 = 0.0;
                for (int a = 0; a < mA; ++a)
                    for (int b = 0; b < mB; ++b)
                        a0 = a0 + c * (double)((long long)fa[0][a][lane] * fb[1][b][lane]);
                for (int b = 0; b < mB; ++b)
                    for (int a = 0; a < mA; ++a)
                        a0 = a0 + c * (double)((long long)fb[0][b][lane] * fa[1][a][lane]);
                if (a0 == 0.0) break;
                if (ev >= cap) {
                    capped = true;
                    break;
                }
                const tdev::Words4 wds = tdev::philox4x32_10(j, step, e, tagword, key0, key1);
                ++j;
                double u1, u2;
                tdev::two_uniforms(wds, u1, u2);
                const double tau = (-tdev::plog(u1)) / a0;
                const double tn = t + tau;
                if (tn >= dt) break;
                t = tn;
                const double r = u2 * a0;
                double prefix = 0.0;
                int sel = -1, last = -1;
                int k = 0;
                for (int a = 0; a < mA; ++a)
                    for (int b = 0; b < mB; ++b, ++k) {
                        const double p = c * (double)((long long)fa[0][a][lane] * fb[1][b][lane]);
                        const double next = prefix + p;
                        if (p > 0.0) {
                            if (sel < 0 && r < next) sel = k;
                            last = k;
                        }
                        prefix = next;
                    }
                for (int b = 0; b < mB; ++b)
                    for (int a = 0; a < mA; ++a, ++k) {
                        const double p = c * (double)((long long)fb[0][b][lane] * fa[1][a][lane]);
                        const double next = prefix + p;
                        if (p > 0.0) {
                            if (sel < 0 && r < next) sel = k;
                            last = k;
                        }
                        prefix = next;
                    }
                if (sel < 0) sel = last;
                int32_t nN, nD, nI;
                if (sel < half) {
                    const int a = sel / mB, b = sel - (sel / mB) * mB;
                    nN = --fa[0][a][lane];
                    nD = --fb[1][b][lane];
                    nI = ++fa[2][a][lane];
                } else {
                    const int kk = sel - half;
                    const int b = kk / mA, a = kk - (kk / mA) * mA;
                    nN = --fb[0][b][lane];
                    nD = --fa[1][a][lane];
                    nI = ++fb[2][b][lane];
                }
                overflow |= (nN < 0) | (nD < 0) | (nI >= kCountLimit);
                ++ev;
            }
#pragma unroll
            for (int a = 0; a < kMaxFace; ++a)
                if (a < mA) {
                    const long long g = (gi + A[a]) * S;
                    counts[g + sp0] = fa[0][a][lane];
                    counts[g + sp1] = fa[1][a][lane];
                    counts[g + sp2] = fa[2][a][lane];
                }
#pragma unroll
            for (int b = 0; b < kMaxFace; ++b)
                if (b < mB) {
                    const long long g = (gj + B[b]) * S;
                    counts[g + sp0] = fb[0][b][lane];
                    counts[g + sp1] = fb[1][b][lane];
                    counts[g + sp2] = fb[2][b][lane];
                }
            if (T->tr_s_ev) {
                const uint32_t ts = uni(T->trace_steps), ne = uni(T->n_edges);
                const size_t slot = (size_t)(step % ts) * ne + e;
                T->tr_s_ev[slot] = ev;
                T->tr_s_t[slot] = (unsigned long long)__double_as_longlong(t);
            }
        }
        const uint32_t ev_sum = wave_sum_u32(ev);
        const uint32_t dr_sum = wave_sum_u32(j);
        const bool any_over = __any(overflow);
        const bool any_cap = __any(capped);
        if (lane == 0) {
            if (ev_sum) atomicAdd(T->stats + 1, (unsigned long long)ev_sum);
            if (dr_sum) atomicAdd(T->stats + 2, (unsigned long long)dr_sum);
            if (any_over) atomicOr(T->flags + 0, 1u);
            if (any_cap) atomicOr(T->flags + 1, 1u);
        }
    }
    leave_queue(queue, persistent != 0);
}

// step_base += n for every tissue of the table
__global__ void advance_kernel(DevTissue *const *tbl, uint32_t n_tissues, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_tissues) tbl[i]->step_base += n;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t chi_lds_bytes(int P, int S, int cells_per_item)
{
    return (size_t)cells_per_item * ((size_t)2 * P * 8 + (size_t)P * S * 4);
}

hipError_t launch_chi(int P, uint32_t grid, size_t lds, hipStream_t stream,
                      const DevTissue *const *tbl, const ChiItem *items, uint32_t n_items,
                      uint32_t *queue, int persistent, int cells_per_item, double dt,
                      uint32_t kstep)
{
    dim3 g(grid), b(kWave);
    switch (P) {
#define TISSUE_CHI_CASE(PP)                                                                  \
    case PP:                                                                                 \
        hipLaunchKernelGGL(chi_kernel<PP>, g, b, lds, stream, tbl, items, n_items, queue,    \
                           persistent, cells_per_item, dt, kstep);                           \
        break;
        TISSUE_CHI_CASE(1)
        TISSUE_CHI_CASE(2)
        TISSUE_CHI_CASE(4)
        TISSUE_CHI_CASE(8)
        TISSUE_CHI_CASE(16)
        TISSUE_CHI_CASE(32)
        TISSUE_CHI_CASE(64)
#undef TISSUE_CHI_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t set_chi_lds_limit(int P, size_t lds)
{
    const void *fn = nullptr;
    switch (P) {
    case 1: fn = reinterpret_cast<const void *>(&chi_kernel<1>); break;
    case 2: fn = reinterpret_cast<const void *>(&chi_kernel<2>); break;
    case 4: fn = reinterpret_cast<const void *>(&chi_kernel<4>); break;
    case 8: fn = reinterpret_cast<const void *>(&chi_kernel<8>); break;
    case 16: fn = reinterpret_cast<const void *>(&chi_kernel<16>); break;
    case 32: fn = reinterpret_cast<const void *>(&chi_kernel<32>); break;
    case 64: fn = reinterpret_cast<const void *>(&chi_kernel<64>); break;
    default: return hipErrorInvalidValue;
    }
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_s(uint32_t grid, hipStream_t stream, const DevTissue *const *tbl,
                    const SItem *items, uint32_t n_items, uint32_t *queue, int persistent,
                    double dt, uint32_t kstep)
{
    hipLaunchKernelGGL(s_kernel, dim3(grid), dim3(kWave), 0, stream, tbl, items, n_items, queue,
                       persistent, dt, kstep);
    return hipGetLastError();
}

hipError_t launch_advance(hipStream_t stream, DevTissue *const *tbl, uint32_t n_tissues,
                          uint32_t n)
{
    const uint32_t threads = 256;
    hipLaunchKernelGGL(advance_kernel, dim3((n_tissues + threads - 1) / threads), dim3(threads), 0,
                       stream, tbl, n_tissues, n);
    return hipGetLastError();
}

}  // namespace tissue_impl
