// kernels.hip -- the device kernels of one splitting step on gfx950, compiled
// ahead of time: the signalling operator S and the step-counter advance,
// and the launchers (the chi kernels with the generic network policy are
// compiled from chi_generic.hip).
//
// S (cell signalling; paper: "Cell signaling module" and the translation
// scripts, Results > Model: Delta within reach of a single shared face turns
// into the neighbour's NICD): one lane per lattice edge gathers N, D, I of
// the two facing membrane groups, runs the pairwise SSA over dt and scatters
// the counts back.  Edges of one launch touch disjoint state (a colour class
// is a matching; with disjoint face groups all classes may share a launch).
#include <hip/hip_runtime.h>

#include "chi_kernels.h"
#include "kernels.h"

namespace tissue_impl {

// ---------------------------------------------------------------------------
// S: one lane per edge
// ---------------------------------------------------------------------------
namespace {

// Workgroup b of n, dealt to XCD b mod 8, takes item x q + min(x, r) + b / 8
// (x = b mod 8, q = n / 8, r = n mod 8): each XCD gets one contiguous range
// of the items (a bijection on 0..n-1).
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t n)
{
    const uint32_t x = b % kXcds, k = b / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + min(x, r) + k;
}

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

// FIX = 2 or 1: every edge of the launch has face groups of FIX and FIX
// voxels (counts in registers only: no LDS, fewer registers, more resident
// wavefronts); FIX = 0: any sizes, the general path in LDS for the others.
template <int FIX>
__global__ __launch_bounds__(kWave) void s_kernel(const DevTissue *const *tbl, const SItem *items,
                                                  uint32_t n_items, double dt, uint32_t kstep)
{
    // per lane: N, D, I of face A (cell i) then of face B (cell j)
    __shared__ int32_t fa[3][kMaxFace][kWave];
    __shared__ int32_t fb[3][kMaxFace][kWave];
    const int lane = threadIdx.x;
    // one workgroup per item: consecutive items on one XCD (workgroups are
    // dealt to the XCDs in turn), so that the edges around a cell share that
    // XCD's L2
    const uint32_t it = xcd_contiguous(blockIdx.x, gridDim.x);
    if (it >= n_items) return;
    const SItem item = items[it];
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
            if (fixed == 0 && a < mA) {
                const long long g = (gi + A[a]) * S;
                if (!first_order) counts[g + sp0] = fa[0][a][lane];
                counts[g + sp1] = fa[1][a][lane];
                counts[g + sp2] = fa[2][a][lane];
            }
#pragma unroll
        for (int b = 0; b < kMaxFace; ++b)
            if (fixed == 0 && b < mB) {
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

// step_base += n for every tissue of the table
__global__ void advance_kernel(DevTissue *const *tbl, uint32_t n_tissues, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_tissues) tbl[i]->step_base += n;
}

// ---------------------------------------------------------------------------
// Regroup: reorder the cells of one leaf-count class of one tissue by their
// total propensity after the last compact chi pass, largest first, in
// buckets of 1/16 of a binary order of magnitude below the class's largest,
// so that the cells of a work item (one wavefront) carry similar numbers of
// events and the heaviest items start first.  A cell's result depends only
// on its own counts and counters, never on its item or position.  One
// workgroup per segment (up to kRegroupChunk consecutive cells of a class
// of one tissue, whole work items): every thread holds its cells and their
// loads in registers, so the list is read once and rewritten in place.
// ---------------------------------------------------------------------------
constexpr int kRegroupThreads = 1024;
constexpr int kRegroupPerThread = (int)(kRegroupChunk / kRegroupThreads);
constexpr int kRegroupBuckets = 256;
static_assert(kRegroupChunk % kRegroupThreads == 0, "regroup chunk");

__global__ __launch_bounds__(kRegroupThreads) void regroup_kernel(const DevTissue *const *tbl,
                                                                  const ChiItem *segs,
                                                                  uint32_t n_segs)
{
    __shared__ uint32_t count[kRegroupBuckets];
    __shared__ uint32_t next[kRegroupBuckets];
    __shared__ uint32_t top_bits;
    if (blockIdx.x >= n_segs) return;
    const ChiItem seg = segs[blockIdx.x];
    const DevTissue *T = tbl[seg.tissue];
    int32_t *cl = T->cell_list + seg.first;
    const float *load = T->load;
    const uint32_t n = min(seg.count, kRegroupChunk);
    const int tid = threadIdx.x;
    for (int b = tid; b < kRegroupBuckets; b += kRegroupThreads) count[b] = 0u;
    if (tid == 0) top_bits = 0u;
    // this thread's cells and loads (non-negative floats order as their bits)
    int32_t cell[kRegroupPerThread];
    float key[kRegroupPerThread];
    uint32_t mb = 0u;
#pragma unroll
    for (int r = 0; r < kRegroupPerThread; ++r) {
        const uint32_t i = (uint32_t)(r * kRegroupThreads + tid);
        cell[r] = i < n ? cl[i] : 0;
        key[r] = i < n ? load[cell[r]] : 0.0f;
        mb = max(mb, __float_as_uint(key[r]));
    }
    __syncthreads();  // counters cleared; every cell read before any is rewritten
    atomicMax(&top_bits, mb);
    __syncthreads();
    const float top = __uint_as_float(top_bits);
    int bucket[kRegroupPerThread];  // 0 = heaviest
#pragma unroll
    for (int r = 0; r < kRegroupPerThread; ++r) {
        const float x = key[r];
        int b = kRegroupBuckets - 1;
        if (x > 0.0f && top > 0.0f) {
            const float d = 16.0f * __log2f(top / x);
            b = d < (float)(kRegroupBuckets - 1) ? (int)d : kRegroupBuckets - 1;
        }
        bucket[r] = b;
        if ((uint32_t)(r * kRegroupThreads + tid) < n) atomicAdd(&count[b], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0u;
        for (int b = 0; b < kRegroupBuckets; ++b) {
            next[b] = acc;
            acc += count[b];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRegroupPerThread; ++r)
        if ((uint32_t)(r * kRegroupThreads + tid) < n) cl[atomicAdd(&next[bucket[r]], 1u)] = cell[r];
}

hipError_t launch_regroup(hipStream_t stream, const DevTissue *const *tbl, const ChiItem *segs,
                          uint32_t n_segs)
{
    if (n_segs == 0) return hipSuccess;
    hipLaunchKernelGGL(regroup_kernel, dim3(n_segs), dim3(kRegroupThreads), 0, stream, tbl, segs,
                       n_segs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t chi_lds_bytes(int mode, int P, int S, int cells_per_item)
{
    if (mode == kChiRow) return 0;  // static LDS only
    // compact: cells of P > 16 leaves take P / 16 lanes each
    if (mode == kChiLane16) return lane16_lds_bytes(S, cells_per_item * compact_lanes(P));
    // per cell: the tree (2P doubles) and P*S counts, plus slack for the
    // species-slot reads past the last voxel
    return (size_t)cells_per_item * ((size_t)2 * P * 8 + ((size_t)P * S + kMaxSpecies) * 4);
}


// table sizes of a network: species slots 4 or 8, reactions rounded up to a
// multiple of 4, diffusion channels 0, 4 or 8
void chi_variant(int S, int R, int ND, int &SM, int &RM, int &NDM)
{
    SM = S <= 4 ? 4 : 8;
    RM = R <= 4 ? 4 : R <= 8 ? 8 : R <= 12 ? 12 : 16;
    NDM = ND == 0 ? 0 : ND <= 4 ? 4 : 8;
    if (NDM > SM) SM = NDM;
}

hipError_t launch_chi(int SM, int RM, int NDM, const ChiArgs &a)
{
    // each (species slots, diffusion slots) row of variants is compiled in
    // its own translation unit (chi_generic.hip built once per part)
    if (SM == 4 && NDM == 0) return launch_chi_part0(RM, a);
    if (SM == 4 && NDM == 4) return launch_chi_part1(RM, a);
    if (SM == 8 && NDM == 0) return launch_chi_part2(RM, a);
    if (SM == 8 && NDM == 4) return launch_chi_part3(RM, a);
    if (SM == 8 && NDM == 8) return launch_chi_part4(RM, a);
    return hipErrorInvalidValue;
}

hipError_t launch_s(hipStream_t stream, const DevTissue *const *tbl, const SItem *items,
                    uint32_t n_items, double dt, uint32_t kstep, int fix)
{
    if (fix == 2)
        hipLaunchKernelGGL(s_kernel<2>, dim3(n_items), dim3(kWave), 0, stream, tbl, items, n_items,
                           dt, kstep);
    else if (fix == 1)
        hipLaunchKernelGGL(s_kernel<1>, dim3(n_items), dim3(kWave), 0, stream, tbl, items, n_items,
                           dt, kstep);
    else
        hipLaunchKernelGGL(s_kernel<0>, dim3(n_items), dim3(kWave), 0, stream, tbl, items, n_items,
                           dt, kstep);
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
