// s_device.h -- device code of the cell-signalling operator S, shared by
// the S kernel (kernels.hip) and the small-tissue kernel that the runtime
// compiles per network (the whole run of a small tissue in one launch).
//
// S (paper: "Cell signaling module" and the translation scripts, Results >
// Model: Delta within reach of a single shared face turns into the
// neighbour's NICD): one lane per lattice edge gathers N, D, I of the two
// facing membrane groups, runs the pairwise SSA over dt and scatters the
// counts back.  Edges of one launch touch disjoint state (a colour class is
// a matching; edges of later classes that share a voxel with it come in
// later passes).
#pragma once

#include "chi_kernels.h"

namespace tissue_impl {
namespace {

// The SSA of one edge over dt for face groups of MA and MB voxels known at
// compile time: the counts in registers, every channel loop unrolled, the
// same operations in the same order as the general path below (so the same
// bits).  Reads the face counts, runs the events, writes the counts back.
template <int MA, int MB>
__device__ __forceinline__ void s_edge_fixed(int32_t *counts, long long gi, long long gj,
                                             const uint8_t *A, const uint8_t *B, int S, int sp0,
                                             int sp1, int sp2, bool first_order, double c,
                                             double ci, double cj, double dt, uint32_t step,
                                             uint32_t e, uint32_t tagword, uint32_t key0,
                                             uint32_t key1, uint32_t cap, double &t, uint32_t &j,
                                             uint32_t &ev, bool &overflow, bool &capped)
{
    int32_t na[MA], da[MA], ia[MA], nb[MB], db[MB], ib[MB];
#pragma unroll
    for (int a = 0; a < MA; ++a) {
        const long long g = (gi + A[a]) * S;
        na[a] = first_order ? 0 : counts[g + sp0];
        da[a] = counts[g + sp1];
        ia[a] = counts[g + sp2];
    }
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const long long g = (gj + B[b]) * S;
        nb[b] = first_order ? 0 : counts[g + sp0];
        db[b] = counts[g + sp1];
        ib[b] = counts[g + sp2];
    }
    for (;;) {
        // channels: first order ci D_i(a), then cj D_j(b); trans
        // c N_i(a) D_j(b) for a, b, then c N_j(b) D_i(a) for b, a
        constexpr int NCH = MA * MB * 2 > MA + MB ? MA * MB * 2 : MA + MB;
        double p[NCH];
        int nch;
        if (first_order) {
#pragma unroll
            for (int a = 0; a < MA; ++a) p[a] = ci * (double)da[a];
#pragma unroll
            for (int b = 0; b < MB; ++b) p[MA + b] = cj * (double)db[b];
            nch = MA + MB;
        } else {
#pragma unroll
            for (int a = 0; a < MA; ++a)
#pragma unroll
                for (int b = 0; b < MB; ++b)
                    p[a * MB + b] = c * (double)((long long)na[a] * db[b]);
#pragma unroll
            for (int b = 0; b < MB; ++b)
#pragma unroll
                for (int a = 0; a < MA; ++a)
                    p[MA * MB + b * MA + a] = c * (double)((long long)nb[b] * da[a]);
            nch = 2 * MA * MB;
        }
        double a0 = 0.0;
#pragma unroll
        for (int k = 0; k < NCH; ++k)
            if (k < nch) a0 = a0 + p[k];
        if (a0 == 0.0) break;
        if (ev >= cap) {
            capped = true;
            break;
        }
        const tdev::Words4 wds = tdev::philox4x32_10(j, step, e, tagword, key0, key1);
        ++j;
        double u1, u2;
        tdev::two_uniforms(wds, u1, u2);
        const double tau = (-tdev::plog<true>(u1)) / a0;
        const double tn = t + tau;
        if (tn >= dt) break;
        t = tn;
        const double r = u2 * a0;
        double prefix = 0.0;
        int sel = -1, last = -1;
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            if (k < nch) {
                const double next = prefix + p[k];
                if (p[k] > 0.0) {
                    if (sel < 0 && r < next) sel = k;
                    last = k;
                }
                prefix = next;
            }
        }
        if (sel < 0) sel = last;
        if (first_order) {
            // a Delta of face voxel k of one group becomes an NICD in voxel
            // m' - 1 - floor(k m' / m) of the other
            int32_t nD = 0, nI = 0;
#pragma unroll
            for (int a = 0; a < MA; ++a)
                if (sel == a) {
                    nD = --da[a];
#pragma unroll
                    for (int b = 0; b < MB; ++b)
                        if (b == MB - 1 - (a * MB) / MA) nI = ++ib[b];
                }
#pragma unroll
            for (int b = 0; b < MB; ++b)
                if (sel == MA + b) {
                    nD = --db[b];
#pragma unroll
                    for (int a = 0; a < MA; ++a)
                        if (a == MA - 1 - (b * MA) / MB) nI = ++ia[a];
                }
            overflow |= (nD < 0) | (nI >= kCountLimit);
        } else {
            int32_t nN = 0, nD = 0, nI = 0;
#pragma unroll
            for (int a = 0; a < MA; ++a)
#pragma unroll
                for (int b = 0; b < MB; ++b)
                    if (sel == a * MB + b) {
                        nN = --na[a];
                        nD = --db[b];
                        nI = ++ia[a];
                    }
#pragma unroll
            for (int b = 0; b < MB; ++b)
#pragma unroll
                for (int a = 0; a < MA; ++a)
                    if (sel == MA * MB + b * MA + a) {
                        nN = --nb[b];
                        nD = --da[a];
                        nI = ++ib[b];
                    }
            overflow |= (nN < 0) | (nD < 0) | (nI >= kCountLimit);
        }
        ++ev;
    }
    // an edge without events leaves its face counts as they were: nothing
    // to write (most edges take no event in a step), so their lines stay
    // clean in the cache
    if (ev == 0) return;
#pragma unroll
    for (int a = 0; a < MA; ++a) {
        const long long g = (gi + A[a]) * S;
        if (!first_order) counts[g + sp0] = na[a];
        counts[g + sp1] = da[a];
        counts[g + sp2] = ia[a];
    }
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const long long g = (gj + B[b]) * S;
        if (!first_order) counts[g + sp0] = nb[b];
        counts[g + sp1] = db[b];
        counts[g + sp2] = ib[b];
    }
}

}  // namespace

// per lane: N, D, I of face A (cell i) then of face B (cell j), for face
// groups the register paths do not take
struct SShared {
    int32_t fa[3][kMaxFace][kWave];
    int32_t fb[3][kMaxFace][kWave];
};

// S on one work item (up to 64 edges of one tissue), one lane per edge.
// FIX = 2 or 1: every edge of the item has face groups of FIX and FIX
// voxels (counts in registers only: no LDS, fewer registers, more resident
// wavefronts); FIX = 0: any sizes, face groups of 2 + 2 and 1 + 1 voxels in
// registers and the others through LDS (same operations in the same order
// on every path, so the same bits).
template <int FIX>
__device__ __forceinline__ void s_item(const DevTissue *const *tbl, const SItem &item, double dt,
                                       uint32_t kstep, SShared &sh)
{
    int32_t (*const fa)[kMaxFace][kWave] = sh.fa;
    int32_t (*const fb)[kMaxFace][kWave] = sh.fb;
    const int lane = threadIdx.x;
    const DevTissue *T = tbl[uni(item.tissue)];
    const int S = uni(T->model.n_species);
    const int sp0 = uni(T->model.trans_n), sp1 = uni(T->model.trans_d), sp2 = uni(T->model.trans_i);
    // first order: D_i -> I_j into the facing voxel, N unused (slot 0 idle)
    const bool first_order = uni(T->model.signal_order) == 1;
    const double c = uni(T->model.trans_rate);
    const uint32_t first = uni(item.first), count = uni(item.count);
    const uint32_t step = uni(T->step_base) + kstep;
    const uint64_t seed = uni((uint64_t)T->seed);
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    const uint32_t tagword = (uni(T->sim_id) << 2) | 1u;
    const uint32_t cap = uni(T->event_cap);
    int32_t *counts = T->counts;
    const bool active = lane < (int)count;
    double t = 0.0;
    uint32_t j = 0, ev = 0, e = 0;
    bool overflow = false, capped = false;
    if (active) {
        const EdgeRec *er = T->edges + (first + lane);
        e = er->id;  // the edge's rank: its counters and trace slot
        const int mA = er->m_a, mB = er->m_b;
        // first order: each side's molecules signal at their own
        // cell's network's rate (the tissue's rate without per-cell models)
        const double ci = T->models[er->model_i].trans_rate;
        const double cj = T->models[er->model_j].trans_rate;
        const long long gi = (long long)er->vox_i, gj = (long long)er->vox_j;
        uint8_t A[kMaxFace], B[kMaxFace];
#pragma unroll
        for (int a = 0; a < kMaxFace; ++a) {
            A[a] = er->A[a];
            B[a] = er->B[a];
        }
        // face groups of 2 and 2 voxels (4x4 cells on the hexagonal
        // lattice) and of 1 and 1 (well-mixed cells): counts in registers
        const int fixed = FIX ? FIX : (mA == 2 && mB == 2) ? 2 : (mA == 1 && mB == 1) ? 1 : 0;
        if (fixed == 2)
            s_edge_fixed<2, 2>(counts, gi, gj, A, B, S, sp0, sp1, sp2, first_order, c, ci, cj, dt,
                               step, e, tagword, key0, key1, cap, t, j, ev, overflow, capped);
        else if (fixed == 1)
            s_edge_fixed<1, 1>(counts, gi, gj, A, B, S, sp0, sp1, sp2, first_order, c, ci, cj, dt,
                               step, e, tagword, key0, key1, cap, t, j, ev, overflow, capped);
#pragma unroll
        for (int a = 0; a < kMaxFace; ++a)
            if (fixed == 0 && a < mA) {
                const long long g = (gi + A[a]) * S;
                if (!first_order) fa[0][a][lane] = counts[g + sp0];
                fa[1][a][lane] = counts[g + sp1];
                fa[2][a][lane] = counts[g + sp2];
            }
#pragma unroll
        for (int b = 0; b < kMaxFace; ++b)
            if (fixed == 0 && b < mB) {
                const long long g = (gj + B[b]) * S;
                if (!first_order) fb[0][b][lane] = counts[g + sp0];
                fb[1][b][lane] = counts[g + sp1];
                fb[2][b][lane] = counts[g + sp2];
            }
        const int half = mA * mB;
        // first order: channels ci D_i(a) for a in A, then cj D_j(b) for
        // b in B; a Delta of face voxel k of one group becomes an NICD in
        // voxel m' - 1 - floor(k m' / m) of the other (they run in
        // opposite directions along the shared face)
        while (fixed == 0 && first_order) {
            double a0 = 0.0;
            for (int a = 0; a < mA; ++a) a0 = a0 + ci * (double)fa[1][a][lane];
            for (int b = 0; b < mB; ++b) a0 = a0 + cj * (double)fb[1][b][lane];
            if (a0 == 0.0) break;
            if (ev >= cap) {
                capped = true;
                break;
            }
            const tdev::Words4 wds = tdev::philox4x32_10(j, step, e, tagword, key0, key1);
            ++j;
            double u1, u2;
            tdev::two_uniforms(wds, u1, u2);
            const double tau = (-tdev::plog<true>(u1)) / a0;
            const double tn = t + tau;
            if (tn >= dt) break;
            t = tn;
            const double r = u2 * a0;
            double prefix = 0.0;
            int sel = -1, last = -1;
            for (int k = 0; k < mA + mB; ++k) {
                const double p = k < mA ? ci * (double)fa[1][k][lane]
                                        : cj * (double)fb[1][k - mA][lane];
                const double next = prefix + p;
                if (p > 0.0) {
                    if (sel < 0 && r < next) sel = k;
                    last = k;
                }
                prefix = next;
            }
            if (sel < 0) sel = last;
            int32_t nD, nI;
            if (sel < mA) {
                nD = --fa[1][sel][lane];
                nI = ++fb[2][mB - 1 - (sel * mB) / mA][lane];
            } else {
                const int kk = sel - mA;
                nD = --fb[1][kk][lane];
                nI = ++fa[2][mA - 1 - (kk * mA) / mB][lane];
            }
            overflow |= (nD < 0) | (nI >= kCountLimit);
            ++ev;
        }
        for (;;) {
            if (fixed != 0 || first_order) break;
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
            const double tau = (-tdev::plog<true>(u1)) / a0;
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
            if (fixed == 0 && ev != 0 && a < mA) {  // (no events: nothing changed)
                const long long g = (gi + A[a]) * S;
                if (!first_order) counts[g + sp0] = fa[0][a][lane];
                counts[g + sp1] = fa[1][a][lane];
                counts[g + sp2] = fa[2][a][lane];
            }
#pragma unroll
        for (int b = 0; b < kMaxFace; ++b)
            if (fixed == 0 && ev != 0 && b < mB) {
                const long long g = (gj + B[b]) * S;
                if (!first_order) counts[g + sp0] = fb[0][b][lane];
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

// ---------------------------------------------------------------------------
// The whole run of a small tissue in one workgroup (one wavefront).  The
// tissue's record, counts, cell tables, edge records and networks, and the
// work items, are copied into LDS, and the record's copy points at the
// copies and at event and draw totals and flags of the run kept in LDS
// (only trace rings stay in device memory), so that every read and write
// of the run's steps is an LDS access.  Then,
// step after step, the chi item (one lane per cell, the same code as the
// chi lane kernel) and the S items of every pass in order run on the
// copies, each phase closed by a workgroup barrier so that the next one
// reads the counts this one wrote; at the end the counts go back, the
// run's totals and flags are added to the tissue's, and the step counter
// advances by n_steps.  The operations and their order per
// cell and per edge are those of the step-by-step launches, so the bits
// are the same.  A small tissue spends most of a launched step on launch
// overhead (paper: at small splitting intervals the scheduling of the
// tasks dominates); here one launch covers a whole call.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void copy_words(void *dst, const void *src, uint32_t n_words)
{
    uint32_t *d = static_cast<uint32_t *>(dst);
    const uint32_t *s = static_cast<const uint32_t *>(src);
    for (uint32_t i = threadIdx.x; i < n_words; i += kWave) d[i] = s[i];
}

template <class NET>
__device__ __forceinline__ void run_small(unsigned char *lds, SShared &sh, DevTissue *T,
                                          const SmallRun &run, double dt, uint32_t n_steps)
{
    const uint32_t nc = T->n_cells, ne = T->n_edges;
    copy_words(lds + run.rec, T, sizeof(DevTissue) / 4);
    copy_words(lds + run.counts, T->counts, run.n_counts);
    copy_words(lds + run.vox_off, T->vox_off, nc);
    for (uint32_t i = threadIdx.x; i < 2 * nc; i += kWave) lds[run.wh + i] = T->wh[i];
    copy_words(lds + run.cell_list, T->cell_list, nc);
    copy_words(lds + run.edges, T->edges, ne * (sizeof(EdgeRec) / 4));
    copy_words(lds + run.models, T->models, run.n_models * (sizeof(DevModel) / 4));
    copy_words(lds + run.chi_item_lds, run.chi_item, sizeof(ChiItem) / 4);
    for (int p = 0; p < run.n_s; ++p)
        copy_words(lds + run.s_items_lds[p], run.s_items[p], run.s_n[p] * (sizeof(SItem) / 4));
    // the run's event and draw totals and flags, added to the tissue's at the end
    __shared__ unsigned long long run_stats[3];
    __shared__ uint32_t run_flags[2];
    if (threadIdx.x < 3) run_stats[threadIdx.x] = 0ull;
    if (threadIdx.x < 2) run_flags[threadIdx.x] = 0u;
    __syncthreads();  // the record's copy is whole before its pointers change
    DevTissue *L = reinterpret_cast<DevTissue *>(lds + run.rec);
    DevTissue **tbl = reinterpret_cast<DevTissue **>(lds + run.tbl);
    if (threadIdx.x == 0) {
        L->stats = run_stats;
        L->flags = run_flags;
        L->counts = reinterpret_cast<int32_t *>(lds + run.counts);
        L->vox_off = reinterpret_cast<const int32_t *>(lds + run.vox_off);
        L->wh = lds + run.wh;
        L->cell_list = reinterpret_cast<int32_t *>(lds + run.cell_list);
        L->edges = reinterpret_cast<const EdgeRec *>(lds + run.edges);
        L->models = reinterpret_cast<const DevModel *>(lds + run.models);
        tbl[0] = L;
    }
    __syncthreads();

    const DevTissue *const *ctbl = tbl;
    const ChiItem *chi_item = reinterpret_cast<const ChiItem *>(lds + run.chi_item_lds);
    const double dchi = run.strang ? dt * 0.5 : dt;
    for (uint32_t k = 0; k < n_steps; ++k) {
        chi_lane_body<NET>(lds, ctbl, chi_item, 1, nullptr, 0, run.chi_cells_per_item, run.chi_log2p,
                           dchi, k, 0u, nullptr, 0, 0u);
        __syncthreads();
        for (int p = 0; p < run.n_s; ++p) {
            const SItem *items = reinterpret_cast<const SItem *>(lds + run.s_items_lds[p]);
            for (uint32_t i = 0; i < run.s_n[p]; ++i) s_item<0>(ctbl, items[i], dt, k, sh);
            __syncthreads();
        }
        if (run.strang) {
            chi_lane_body<NET>(lds, ctbl, chi_item, 1, nullptr, 0, run.chi_cells_per_item,
                               run.chi_log2p, dchi, k, 2u, nullptr, 0, 0u);
            __syncthreads();
        }
    }

    copy_words(T->counts, lds + run.counts, run.n_counts);
    if (threadIdx.x < 3 && run_stats[threadIdx.x]) atomicAdd(T->stats + threadIdx.x, run_stats[threadIdx.x]);
    if (threadIdx.x < 2 && run_flags[threadIdx.x]) atomicOr(T->flags + threadIdx.x, 1u);
    if (threadIdx.x == 0) T->step_base += n_steps;
}

}  // namespace tissue_impl
