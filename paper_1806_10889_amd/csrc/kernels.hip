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

// Mass-action propensity of reaction r; x points at species 0 of a voxel,
// species s at x[s * stride].
__device__ __forceinline__ double reaction_propensity(const DevModel &M, int r,
                                                      const int32_t *x, int stride)
{
    const int a = M.reac_a[r], b = M.reac_b[r];
    const double c = M.rates[r];
    if (a < 0) return c;
    const long long xa = x[a * stride];
    if (b < 0) return c * (double)xa;
    if (a == b) return c * (double)(xa * (xa - 1) / 2);
    return c * (double)(xa * (long long)x[b * stride]);
}

__device__ __forceinline__ int voxel_degree(int v, int w, int h)
{
    const int x = v % w, y = v / w;
    return (x > 0) + (x < w - 1) + (y > 0) + (y < h - 1);
}

// Propensity of voxel v: left fold over reactions, then diffusion channels.
__device__ __forceinline__ double voxel_propensity(const DevModel &M, const int32_t *cnt,
                                                   int stride, int S, int v, int w, int h)
{
    const int32_t *x = cnt + v * S * stride;
    double acc = 0.0;
    for (int r = 0; r < M.n_reactions; ++r) acc = acc + reaction_propensity(M, r, x, stride);
    const int deg = voxel_degree(v, w, h);
    if (deg > 0) {
        for (int q = 0; q < M.n_diff; ++q) {
            const long long xs = x[M.diff_species[q] * stride];
            acc = acc + M.diff_rate[q] * (double)(xs * deg);
        }
    }
    return acc;
}

// Destination of a diffusion jump: the kdir-th present neighbour in the
// order (-x, +x, -y, +y).
__device__ __forceinline__ int neighbour_at(int v, int w, int h, int kdir)
{
    const int x = v % w, y = v / w;
    int out = v, idx = 0;
    if (x > 0) { if (idx == kdir) out = v - 1; ++idx; }
    if (x < w - 1) { if (idx == kdir) out = v + 1; ++idx; }
    if (y > 0) { if (idx == kdir) out = v - w; ++idx; }
    if (y < h - 1) { if (idx == kdir) out = v + w; }
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
        const DevTissue *T = tbl[item.tissue];
        const DevModel &M = T->model;
        const int S = M.n_species;
        double *tree = reinterpret_cast<double *>(lds) + lane;                       // [2P][stride]
        int32_t *cnt = reinterpret_cast<int32_t *>(lds + (size_t)2 * P * stride * 8) + lane;

        const bool active = lane < (int)item.count;
        uint32_t cell = 0;
        int w = 1, h = 1;
        long long gbase = 0;
        if (active) {
            cell = (uint32_t)T->cell_list[item.first + lane];
            w = T->wh[2 * cell];
            h = T->wh[2 * cell + 1];
            gbase = (long long)T->vox_off[cell] * S;
            const int n = w * h * S;
            for (int i = 0; i < n; ++i) cnt[i * stride] = T->counts[gbase + i];
        }
        const int V = w * h;
        const uint32_t step = T->step_base + kstep;

        // leaves and internal nodes
        if (active) {
            for (int v = 0; v < P; ++v)
                tree[(P + v) * stride] = v < V ? voxel_propensity(M, cnt, stride, S, v, w, h) : 0.0;
            for (int n = P - 1; n >= 1; --n)
                tree[n * stride] = tree[(2 * n) * stride] + tree[(2 * n + 1) * stride];
        }

        double t = 0.0;
        uint32_t j = 0, ev = 0;
        bool overflow = false, capped = false;
        const uint32_t key0 = (uint32_t)T->seed, key1 = (uint32_t)(T->seed >> 32);
        const uint32_t tagword = (T->sim_id << 2) | 0u;
        const uint32_t cap = T->event_cap;
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
                const int deg = voxel_degree(v, w, h);
                double prefix = 0.0, resid = 0.0, last_prefix = 0.0;
                int sel = -1, last = -1;
                for (int k = 0; k < M.n_reactions; ++k) {
                    const double a = reaction_propensity(M, k, x, stride);
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
                if (deg > 0) {
                    for (int q = 0; q < M.n_diff; ++q) {
                        const long long xs = x[M.diff_species[q] * stride];
                        const double a = M.diff_rate[q] * (double)(xs * deg);
                        const double next = prefix + a;
                        if (a > 0.0) {
                            if (sel < 0 && r < next) {
                                sel = M.n_reactions + q;
                                resid = r - prefix;
                            }
                            last = M.n_reactions + q;
                            last_prefix = prefix;
                        }
                        prefix = next;
                    }
                }
                if (sel < 0) {
                    sel = last;
                    resid = r - last_prefix;
                }

                int dst = v;
                if (sel < M.n_reactions) {
                    uint32_t code = 0;
                    for (int k = 0; k < M.n_reactions; ++k)
                        if (k == sel) code = M.change_code[k];
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
                    const int q = sel - M.n_reactions;
                    int s = 0;
                    double D = 0.0;
                    for (int qq = 0; qq < M.n_diff; ++qq)
                        if (qq == q) {
                            s = M.diff_species[qq];
                            D = M.diff_rate[qq];
                        }
                    const double a1 = D * (double)(long long)x[s * stride];
                    int kdir = 0;
                    for (int l = 1; l <= deg - 1; ++l)
                        if (resid >= (double)l * a1) ++kdir;
                    dst = neighbour_at(v, w, h, kdir);
                    const int32_t nsrc = x[s * stride] - 1;
                    x[s * stride] = nsrc;
                    int32_t *xd = cnt + (dst * S + s) * stride;
                    const int32_t ndst = *xd + 1;
                    *xd = ndst;
                    overflow |= (nsrc < 0) | (ndst >= kCountLimit);
                }
                tree[(P + v) * stride] = voxel_propensity(M, cnt, stride, S, v, w, h);
                if (dst != v)
                    tree[(P + dst) * stride] = voxel_propensity(M, cnt, stride, S, dst, w, h);
                update_path<P>(tree, stride, v);
                if (dst != v) update_path<P>(tree, stride, dst);
                ++ev;
            }
            const int n = V * S;
            for (int i = 0; i < n; ++i) T->counts[gbase + i] = cnt[i * stride];
            if (T->tr_chi_ev) {
                const size_t slot = (size_t)(step % T->trace_steps) * T->n_cells + cell;
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
        const DevTissue *T = tbl[item.tissue];
        const DevModel &M = T->model;
        const int S = M.n_species;
        const bool active = lane < (int)item.count;
        const uint32_t e = item.first + lane;
        const uint32_t step = T->step_base + kstep;
        double t = 0.0;
        uint32_t j = 0, ev = 0;
        bool overflow = false, capped = false;
        if (active) {
            const EdgeRec &er = T->edges[e];
            const int mA = er.m_a, mB = er.m_b;
            const int sp[3] = {M.trans_n, M.trans_d, M.trans_i};
            for (int a = 0; a < mA; ++a) {
                const long long g = (long long)(er.vox_i + er.A[a]) * S;
#pragma unroll
                for (int q = 0; q < 3; ++q) fa[q][a][lane] = T->counts[g + sp[q]];
            }
            for (int b = 0; b < mB; ++b) {
                const long long g = (long long)(er.vox_j + er.B[b]) * S;
#pragma unroll
                for (int q = 0; q < 3; ++q) fb[q][b][lane] = T->counts[g + sp[q]];
            }
            const double c = M.trans_rate;
            const uint32_t key0 = (uint32_t)T->seed, key1 = (uint32_t)(T->seed >> 32);
            const uint32_t tagword = (T->sim_id << 2) | 1u;
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
                if (ev >= T->event_cap) {
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
                    const int a = sel / mB, b = sel % mB;
                    nN = --fa[0][a][lane];
                    nD = --fb[1][b][lane];
                    nI = ++fa[2][a][lane];
                } else {
                    const int kk = sel - half;
                    const int b = kk / mA, a = kk % mA;
                    nN = --fb[0][b][lane];
                    nD = --fa[1][a][lane];
                    nI = ++fb[2][b][lane];
                }
                overflow |= (nN < 0) | (nD < 0) | (nI >= kCountLimit);
                ++ev;
            }
            for (int a = 0; a < mA; ++a) {
                const long long g = (long long)(er.vox_i + er.A[a]) * S;
#pragma unroll
                for (int q = 0; q < 3; ++q) T->counts[g + sp[q]] = fa[q][a][lane];
            }
            for (int b = 0; b < mB; ++b) {
                const long long g = (long long)(er.vox_j + er.B[b]) * S;
#pragma unroll
                for (int q = 0; q < 3; ++q) T->counts[g + sp[q]] = fb[q][b][lane];
            }
            if (T->tr_s_ev) {
                const size_t slot = (size_t)(step % T->trace_steps) * T->n_edges + e;
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
