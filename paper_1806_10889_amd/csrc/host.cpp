// host.cpp -- runtime behind the C-ABI of include/tissue.h.
//
// tissue_create validates the descriptor, builds the geometry on the host
// (lattice edges ranked by (colour, i), membrane rings, face groups, the
// colour-class passes of S), cuts the work into items, lays everything out
// in the caller's device buffer and uploads it.  tissue_step enqueues the
// splitting steps -- per step one chi launch per leaf-count class and one S
// launch per pass -- either eagerly or as replays of a captured HIP graph of
// a fixed number of steps.  Batches reuse the same kernels over a table of
// many tissues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tissue.h"
#include "internal.h"
#include "jit.h"
#include "kernels.h"

using namespace tissue_impl;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(TISSUE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr size_t kChiLdsBudget = 40 * 1024;  // per workgroup: >= 4 resident per CU
// chi launches of one plan (leaf classes x networks) and their queue words:
// each launch owns a block of kQueueBlockWords words (its item queue and
// exit count, its redo count, its redo launch's queue) so that launches of
// different classes can run concurrently
constexpr int kMaxChiLaunches = 64;
constexpr int32_t kWholeRunSteps = 100;  // steps per launch of the whole-run kernel
constexpr size_t kLaunchQueueBytes = (size_t)kMaxChiLaunches * kQueueBlockWords * sizeof(uint32_t);
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr size_t kChiStaticLds = 512;  // the chi kernels' static LDS (channel table), rounded up
constexpr int kDefaultRefillMin = 0;

// Pinned host memory for the copies of the control path (tissue and batch
// creation, work-item uploads, counts and stats readback).  The runtime
// stages a copy from pageable memory through a blit kernel, which waits for
// compute units behind other streams' kernels; from pinned memory the copy
// engines serve it.  One process-wide buffer, grown on demand and held under
// its lock until the copy has completed.
struct PinnedStaging {
    std::mutex mu;
    unsigned char *buf = nullptr;
    size_t cap = 0;
};

PinnedStaging &staging()
{
    static PinnedStaging s;
    return s;
}

hipError_t staging_acquire(std::unique_lock<std::mutex> &lk, size_t n, unsigned char **out)
{
    PinnedStaging &s = staging();
    lk = std::unique_lock<std::mutex>(s.mu);
    if (s.cap < n) {
        if (s.buf) (void)hipHostFree(s.buf);
        s.buf = nullptr;
        s.cap = 0;
        const size_t c = std::max<size_t>(n, (size_t)1 << 20);
        const hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&s.buf), c, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        s.cap = c;
    }
    *out = s.buf;
    return hipSuccess;
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int pow2_at_least(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------

// lattice direction offsets (square: +x, +y, -x, -y; hex axial: E, SE, SW,
// W, NW, NE with y pointing down)
const int kSquareDir[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
const int kHexDir[6][2] = {{1, 0}, {0, 1}, {-1, 1}, {-1, 0}, {0, -1}, {1, -1}};

// perimeter of a w x h mesh, clockwise from the top-right voxel: down the
// right column, left along the bottom row, up the left column, right along
// the top row; a voxel is listed once.
std::vector<int> membrane_ring(int w, int h)
{
    std::vector<int> ring;
    std::vector<char> on(w * h, 0);
    auto push = [&](int x, int y) {
        const int v = y * w + x;
        if (!on[v]) {
            on[v] = 1;
            ring.push_back(v);
        }
    };
    for (int y = 0; y < h; ++y) push(w - 1, y);
    for (int x = w - 2; x >= 0; --x) push(x, h - 1);
    for (int y = h - 2; y >= 0; --y) push(0, y);
    for (int x = 1; x < w - 1; ++x) push(x, 0);
    return ring;
}

// voxels of the face toward lattice direction d (of nd): the d-th of nd
// consecutive slices of the ring (a one-voxel group when the slice is empty)
std::vector<int> face_voxels(const std::vector<int> &ring, int nd, int d)
{
    const int M = (int)ring.size();
    const int lo = d * M / nd, hi = (d + 1) * M / nd;
    if (hi <= lo) return {ring[lo % M]};
    return std::vector<int>(ring.begin() + lo, ring.begin() + hi);
}

struct Edge {
    int colour, i, j, d;
};

std::vector<Edge> lattice_edges(int lattice, int nx, int ny)
{
    // edges in (colour class, first cell) order, generated in that order:
    // class 2d + parity holds the edges of forward direction d whose first
    // cell has that parity of x (d = 0) or of y (d > 0)
    const int nfwd = lattice == TISSUE_LATTICE_SQUARE ? 2 : 3;
    std::vector<Edge> out;
    out.reserve((size_t)nx * ny * nfwd);
    for (int d = 0; d < nfwd; ++d) {
        const int *off = lattice == TISSUE_LATTICE_SQUARE ? kSquareDir[d] : kHexDir[d];
        for (int parity = 0; parity < 2; ++parity)
            for (int y = 0; y < ny; ++y) {
                if (d != 0 && (y & 1) != parity) continue;
                const int Y = y + off[1];
                if (Y < 0 || Y >= ny) continue;
                const int x0 = d == 0 ? parity : 0, dx = d == 0 ? 2 : 1;
                for (int x = x0; x < nx; x += dx) {
                    const int X = x + off[0];
                    if (X < 0 || X >= nx) continue;
                    out.push_back(Edge{2 * d + parity, y * nx + x, Y * nx + X, d});
                }
            }
    }
    return out;
}

// rate constants are bounded so that every propensity (at most 1e12 * 2^52)
// and every sum of them stays finite
constexpr double kMaxRate = 1e12;

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0 && x <= kMaxRate; }

// ---------------------------------------------------------------------------
// plan: everything tissue_create derives from the descriptor on the host
// ---------------------------------------------------------------------------

// cells of one leaf-count class P and one network: cell_list[first, first + count)
struct ChiGroupHost {
    int P;
    int model;
    uint32_t first, count;
};

// cells per lane-mode item: as many as fit the LDS budget (a power of two <= 64)
int lane_cells_per_item(int P, int S)
{
    const size_t per_cell = chi_lds_bytes(kChiLane, P, S, 1);
    int cpi = 64;
    while (cpi > 1 && (size_t)cpi * per_cell > kChiLdsBudget) cpi >>= 1;
    return cpi;
}

// items of a class: up to cpi cells each, tagged with the tissue index and
// the cells' network
void cut_items(uint32_t tissue, const ChiGroupHost &g, int cpi, std::vector<ChiItem> &out)
{
    for (uint32_t o = 0; o < g.count; o += (uint32_t)cpi)
        out.push_back(ChiItem{tissue, g.first + o, std::min<uint32_t>((uint32_t)cpi, g.count - o),
                              (uint32_t)g.model});
}

struct Plan {
    uint32_t lattice = 0, nx = 0, ny = 0, ncell = 0, S = 0, nvox = 0, nedge = 0;
    std::vector<uint8_t> wh;
    std::vector<int32_t> vox_off;
    std::vector<int32_t> cell_list;
    std::vector<uint8_t> cell_model;    // [ncell] each cell's network
    std::vector<EdgeRec> edges;
    std::vector<uint32_t> pass_start;   // [passes + 1] ranges of the edge records per S pass
    bool disjoint = true;               // every cell's face groups pairwise disjoint
    bool has_s = false;
    int face_kind = 0;                  // 2 or 1: every edge has face groups of 2 and 2 (1 and 1) voxels
    std::vector<ChiGroupHost> chi;
    std::vector<std::vector<SItem>> s_passes;
    // the cells' networks: [0] is the descriptor's own (with the S reaction),
    // then the extra models; per network its structure (cache key) and its
    // compiled chi kernels, if any
    std::vector<DevModel> models;
    std::vector<std::string> net_keys;
    std::vector<const JitKernels *> jits;
    bool all_jit = false;               // every network has compiled kernels
    uint32_t trace_steps = 0;
    bool strang = false;                // TISSUE_FLAG_STRANG
    // byte offsets inside dev_buf
    size_t off_tissue = 0, off_tbl = 0, off_counts = 0, off_init = 0, off_voxoff = 0, off_wh = 0,
           off_cells = 0, off_edges = 0, off_models = 0, off_chi = 0, off_s = 0, off_ctl = 0,
           off_trace = 0, off_lq = 0, off_load = 0,
           off_retry = 0, bytes = 0;
    size_t n_chi_items = 0, n_s_items = 0;
};

// One network's reaction and diffusion tables, validated and packed into M
// (n_species S; the S-reaction fields are left to the caller).
int build_model(int S, uint32_t n_reactions, const int32_t *reactants, const int32_t *stoich,
                const double *rates, const double *diffusion, DevModel &M)
{
    if (n_reactions > TISSUE_MAX_REACTIONS) return fail(TISSUE_EINVAL, "n_reactions must be <= 16");
    const int R = (int)n_reactions;
    if (R > 0 && (!reactants || !stoich || !rates)) return fail(TISSUE_EINVAL, "reaction tables are null");
    if (!diffusion) return fail(TISSUE_EINVAL, "diffusion is null");
    M.n_species = S;
    M.n_reactions = R;
    for (int r = 0; r < R; ++r) {
        const int a = reactants[2 * r], b = reactants[2 * r + 1];
        if (a < -1 || a >= S || b < -1 || b >= S) return fail(TISSUE_EINVAL, "reactant index out of range");
        if (!finite_nonneg(rates[r])) return fail(TISSUE_EINVAL, "rates must be finite, >= 0 and <= 1e12");
        // canonical order: a first reactant, b second or -1
        int ra = a, rb = b;
        if (ra < 0) std::swap(ra, rb);
        M.reac_a[r] = (int8_t)ra;
        M.reac_b[r] = (int8_t)rb;
        M.rates[r] = rates[r];
        uint32_t lo = 0, hi = 0;
        int nchg = 0;
        for (int s = 0; s < S; ++s) {
            const int delta = stoich[r * S + s];
            if (delta == 0) continue;
            if (delta < -15 || delta > 15) return fail(TISSUE_EINVAL, "stoich entries must be in -15..15");
            const int supplied = (a == s) + (b == s);
            if (delta < -supplied)
                return fail(TISSUE_EINVAL, "a reaction consumes a species it does not have as reactant");
            if (++nchg > 4) return fail(TISSUE_EINVAL, "a reaction may change at most 4 species");
            const uint32_t byte = (uint32_t)(uint8_t)(int8_t)delta;
            if (s < 4) lo |= byte << (8 * s);
            else hi |= byte << (8 * (s - 4));
        }
        M.delta_lo[r] = lo;
        M.delta_hi[r] = hi;
    }
    for (int r = R; r < kMaxReactions; ++r) {  // padding: no reactants, rate 0, no change
        M.reac_a[r] = -1;
        M.reac_b[r] = -1;
        M.rates[r] = 0.0;
        M.delta_lo[r] = 0;
        M.delta_hi[r] = 0;
    }
    M.n_diff = 0;
    for (int s = 0; s < S; ++s) {
        if (!finite_nonneg(diffusion[s])) return fail(TISSUE_EINVAL, "diffusion must be finite, >= 0 and <= 1e12");
        if (diffusion[s] > 0.0) {
            M.diff_species[M.n_diff] = (int8_t)s;
            M.diff_rate[M.n_diff] = diffusion[s];
            ++M.n_diff;
        }
    }
    for (int q = M.n_diff; q < kMaxSpecies; ++q) {  // padding: rate 0
        M.diff_species[q] = 0;
        M.diff_rate[q] = 0.0;
    }
    return TISSUE_OK;
}

// The number of forward lattice edges of an nx x ny tissue (each counted
// once): square +x and +y; hexagonal also the (-1, +1) diagonal.
uint64_t lattice_edge_count(int lattice, uint64_t nx, uint64_t ny)
{
    const uint64_t n = (nx - 1) * ny + nx * (ny - 1);
    return lattice == TISSUE_LATTICE_SQUARE ? n : n + (nx - 1) * (ny - 1);
}

// Room for the S work items: each pass's items are ceil(edges / 64), and
// there are at most as many passes as colour classes (an edge of class k
// is at most in pass k: edges of one class share no voxel), so the sum is
// at most ceil(nedge / 64) + classes - 1.  Known before the passes are.
size_t s_item_room(int lattice, uint64_t nedge)
{
    const int classes = lattice == TISSUE_LATTICE_SQUARE ? 4 : 6;
    return nedge ? (size_t)((nedge + kWave - 1) / kWave) + (size_t)(classes - 1) : 0;
}

// with_edges false: everything but the edge records and the S passes (the
// tissue's size in device memory needs only their counts, known in closed
// form); tissue_required_bytes plans this way.
int build_plan(const tissue_desc_t *d, Plan &p, bool with_edges = true)
{
    if (!d) return fail(TISSUE_EINVAL, "null descriptor");
    if (d->abi_version != TISSUE_ABI_VERSION) return fail(TISSUE_EINVAL, "abi_version mismatch");
    if (d->lattice != TISSUE_LATTICE_SQUARE && d->lattice != TISSUE_LATTICE_HEX)
        return fail(TISSUE_EINVAL, "lattice must be 0 (square) or 1 (hex)");
    if (d->nx < 1 || d->ny < 1 || (uint64_t)d->nx * d->ny > (1u << 24))
        return fail(TISSUE_EINVAL, "nx, ny must be >= 1 with nx*ny <= 2^24");
    if (d->n_species < 1 || d->n_species > TISSUE_MAX_SPECIES)
        return fail(TISSUE_EINVAL, "n_species must be in 1..8");
    if (d->sim_id >= (1u << 30)) return fail(TISSUE_EINVAL, "sim_id must be < 2^30");
    if (!d->init_counts) return fail(TISSUE_EINVAL, "init_counts is null");
    if ((d->mesh_w == nullptr) != (d->mesh_h == nullptr))
        return fail(TISSUE_EINVAL, "mesh_w and mesh_h must both be given or both be null");
    if (d->flags & ~(TISSUE_FLAG_TRACE | TISSUE_FLAG_NO_JIT | TISSUE_FLAG_STRANG |
                     TISSUE_FLAG_SIGNAL_FIRST_ORDER))
        return fail(TISSUE_EINVAL, "unknown bits in flags");
    if ((d->flags & TISSUE_FLAG_TRACE) && d->trace_steps < 1)
        return fail(TISSUE_EINVAL, "trace needs trace_steps >= 1");
    const int S = (int)d->n_species;
    if (d->n_models > TISSUE_MAX_MODELS) return fail(TISSUE_EINVAL, "n_models must be <= 7");
    if (d->n_models > 0 && !d->models) return fail(TISSUE_EINVAL, "models is null");

    p.lattice = d->lattice;
    p.nx = d->nx;
    p.ny = d->ny;
    p.ncell = d->nx * d->ny;
    p.S = (uint32_t)S;

    // networks: the descriptor's own, then the extra models
    p.models.assign(1 + d->n_models, DevModel{});
    int rc = build_model(S, d->n_reactions, d->reactants, d->stoich, d->rates, d->diffusion,
                         p.models[0]);
    if (rc != TISSUE_OK) return rc;
    for (uint32_t m = 0; m < d->n_models; ++m) {
        const tissue_model_t &md = d->models[m];
        rc = build_model(S, md.n_reactions, md.reactants, md.stoich, md.rates, md.diffusion,
                         p.models[1 + m]);
        if (rc != TISSUE_OK) return fail(rc, "model " + std::to_string(m + 1) + ": " + g_last_error);
    }
    DevModel &M = p.models[0];
    const bool first_order = (d->flags & TISSUE_FLAG_SIGNAL_FIRST_ORDER) != 0;
    p.has_s = first_order ? d->trans_d >= 0 : d->trans_n >= 0;
    M.signal_order = first_order ? 1 : 2;
    if (p.has_s) {
        const int tn = first_order ? -1 : d->trans_n, td = d->trans_d, ti = d->trans_i;
        if (first_order) {
            if (td >= S || ti < 0 || ti >= S || td == ti)
                return fail(TISSUE_EINVAL, "trans_d, trans_i must be distinct species");
        } else if (tn >= S || td < 0 || td >= S || ti < 0 || ti >= S || tn == td || tn == ti || td == ti) {
            return fail(TISSUE_EINVAL, "trans_n, trans_d, trans_i must be distinct species");
        }
        if (!finite_nonneg(d->trans_rate)) return fail(TISSUE_EINVAL, "trans_rate must be finite, >= 0 and <= 1e12");
        M.trans_n = tn;
        M.trans_d = td;
        M.trans_i = ti;
        M.trans_rate = d->trans_rate;
    } else {
        M.trans_n = M.trans_d = M.trans_i = -1;
        M.trans_rate = 0.0;
    }

    // the S reaction's species are the tissue's; under first-order
    // signalling each network carries its cells' signalling rate
    for (size_t m = 1; m < p.models.size(); ++m) {
        DevModel &X = p.models[m];
        const double k = d->models[m - 1].signal_rate;
        X.trans_n = M.trans_n;
        X.trans_d = M.trans_d;
        X.trans_i = M.trans_i;
        X.signal_order = M.signal_order;
        X.trans_rate = M.trans_rate;
        if (!p.has_s) continue;
        if (first_order) {
            if (!finite_nonneg(k))
                return fail(TISSUE_EINVAL, "model " + std::to_string(m) +
                                               ": signal_rate must be finite, >= 0 and <= 1e12");
            X.trans_rate = k;
        } else if (k != M.trans_rate) {
            return fail(TISSUE_EINVAL, "model " + std::to_string(m) +
                                           ": signal_rate must equal trans_rate under the second-order reaction");
        }
    }
    for (const DevModel &X : p.models) p.net_keys.push_back(network_key(X));
    p.jits.assign(p.models.size(), nullptr);

    // cells and voxels
    p.wh.resize(2 * (size_t)p.ncell);
    p.vox_off.resize(p.ncell);
    p.cell_model.assign(p.ncell, 0);
    uint64_t nvox = 0;
    for (uint32_t c = 0; c < p.ncell; ++c) {
        const uint32_t w = d->mesh_w ? d->mesh_w[c] : d->mesh_w0;
        const uint32_t h = d->mesh_h ? d->mesh_h[c] : d->mesh_h0;
        if (w < 1 || w > TISSUE_MAX_MESH || h < 1 || h > TISSUE_MAX_MESH)
            return fail(TISSUE_EINVAL, "mesh sides must be in 1..8");
        p.wh[2 * c] = (uint8_t)w;
        p.wh[2 * c + 1] = (uint8_t)h;
        p.vox_off[c] = (int32_t)nvox;
        nvox += (uint64_t)w * h;
    }
    if (nvox * (uint64_t)S >= (1ull << 31)) return fail(TISSUE_EINVAL, "too many voxels");
    p.nvox = (uint32_t)nvox;
    {
        // (a negative count, taken unsigned, is at or past the limit too)
        uint32_t out_of_range = 0;
        for (uint64_t i = 0; i < nvox * S; ++i)
            out_of_range |= (uint32_t)((uint32_t)d->init_counts[i] >= (uint32_t)TISSUE_COUNT_LIMIT);
        if (out_of_range) return fail(TISSUE_EINVAL, "init_counts must be in [0, 2^26)");
    }

    // chi: cells grouped by leaf count P (largest cells first); work items
    // are cut per launch mode when a launch plan is made
    // classes (P, network) in order of decreasing P, then increasing
    // network; each class's cells in increasing order (a counting sort)
    constexpr int kLogP = 7;  // P = 1, 2, ..., 64
    const int nm = 1 + (int)d->n_models;
    std::vector<uint32_t> cls(p.ncell), n_in((size_t)kLogP * nm, 0);
    for (uint32_t c = 0; c < p.ncell; ++c) {
        const int m = d->cell_model ? d->cell_model[c] : 0;
        if (m > (int)d->n_models) return fail(TISSUE_EINVAL, "cell_model entries must be <= n_models");
        p.cell_model[c] = (uint8_t)m;
        int lp = 0;
        while ((1 << lp) < p.wh[2 * c] * p.wh[2 * c + 1]) ++lp;
        cls[c] = (uint32_t)((kLogP - 1 - lp) * nm + m);
        n_in[cls[c]]++;
    }
    std::vector<uint32_t> at(n_in.size() + 1, 0);
    for (size_t k = 0; k < n_in.size(); ++k) at[k + 1] = at[k] + n_in[k];
    p.cell_list.resize(p.ncell);
    {
        std::vector<uint32_t> put(at.begin(), at.end() - 1);
        for (uint32_t c = 0; c < p.ncell; ++c) p.cell_list[put[cls[c]]++] = (int32_t)c;
    }
    for (size_t k = 0; k < n_in.size(); ++k) {
        if (!n_in[k]) continue;
        ChiGroupHost g;
        g.P = 1 << (kLogP - 1 - (int)(k / (size_t)nm));
        g.model = (int)(k % (size_t)nm);
        g.first = at[k];
        g.count = n_in[k];
        p.chi.push_back(g);
        // room for the largest cut of the class, whichever the launch plan
        // picks: lane layout, rows of max(16, P) or max(32, P) lanes, or the
        // compact lane layout (at most one item per cell)
        const uint32_t lcpi = (uint32_t)lane_cells_per_item(g.P, S);
        const uint32_t wcpi = (uint32_t)(kWave / std::max(32, g.P));  // wide rows: fewest cells per item
        uint32_t most = std::max((g.count + lcpi - 1) / lcpi, (g.count + wcpi - 1) / wcpi);
        if (g.P <= 64) most = std::max(most, g.count);
        p.n_chi_items += most + (g.count + kRegroupChunk - 1) / kRegroupChunk;  // + regroup segments
    }

    // edges, face groups, S passes
    const int nd = p.lattice == TISSUE_LATTICE_SQUARE ? 4 : 6;
    if (p.has_s) p.nedge = (uint32_t)lattice_edge_count((int)p.lattice, p.nx, p.ny);
    if (p.has_s && with_edges) {
        // per mesh (key w*16+h) its [nd] face groups (empty: mesh not present)
        std::vector<std::vector<std::vector<int>>> faces(16 * 16);
        for (uint32_t c = 0; c < p.ncell; ++c) {
            const int key = p.wh[2 * c] * 16 + p.wh[2 * c + 1];
            if (!faces[key].empty()) continue;
            const std::vector<int> ring = membrane_ring(p.wh[2 * c], p.wh[2 * c + 1]);
            std::vector<std::vector<int>> g(nd);
            for (int dd = 0; dd < nd; ++dd) g[dd] = face_voxels(ring, nd, dd);
            // disjointness of all face groups of this mesh
            std::vector<int> seen(64, 0);
            for (int dd = 0; dd < nd; ++dd)
                for (int v : g[dd]) {
                    if (seen[v]) p.disjoint = false;
                    seen[v] = 1;
                }
            faces[key] = std::move(g);
        }
        const std::vector<Edge> E = lattice_edges((int)p.lattice, (int)p.nx, (int)p.ny);
        if (E.size() != p.nedge) return fail(TISSUE_EINVAL, "internal: lattice edge count");
        p.edges.resize(E.size());
        auto group_i = [&](const Edge &ed) -> const std::vector<int> & {
            return faces[p.wh[2 * ed.i] * 16 + p.wh[2 * ed.i + 1]][ed.d];
        };
        auto group_j = [&](const Edge &ed) -> const std::vector<int> & {
            return faces[p.wh[2 * ed.j] * 16 + p.wh[2 * ed.j + 1]][(ed.d + nd / 2) % nd];
        };
        // S passes.  The colour classes run in order, each over the whole
        // interval; an edge's SSA reads and writes only its two face groups,
        // so two edges of different classes commute unless they share a
        // voxel, and any order that keeps every such pair in class order
        // gives the same bits.  Pass (level) of an edge: 0 if no edge of an
        // earlier class touched its voxels, else one more than the highest
        // pass of those that did.  With disjoint face groups every edge is in
        // pass 0 (one launch); with overlapping ones (meshes of fewer than
        // six membrane voxels on the hexagonal lattice) usually two passes
        // instead of one per class.
        std::vector<uint8_t> level(E.size(), 0);
        if (!p.disjoint) {
            std::vector<uint8_t> last(p.nvox, 0);  // highest pass + 1 that touched a voxel
            for (size_t e = 0; e < E.size(); ++e) {  // E is in (colour, i) order
                const Edge &ed = E[e];
                int lv = 0;
                for (int v : group_i(ed)) lv = std::max(lv, (int)last[p.vox_off[ed.i] + v]);
                for (int v : group_j(ed)) lv = std::max(lv, (int)last[p.vox_off[ed.j] + v]);
                if (lv >= 255) return fail(TISSUE_EINVAL, "too many signalling passes");
                level[e] = (uint8_t)lv;
                // edges of one class share no cell, so marking at once is safe
                for (int v : group_i(ed)) last[p.vox_off[ed.i] + v] = (uint8_t)(lv + 1);
                for (int v : group_j(ed)) last[p.vox_off[ed.j] + v] = (uint8_t)(lv + 1);
            }
        }
        int n_levels = 0;
        for (size_t e = 0; e < E.size(); ++e) n_levels = std::max(n_levels, (int)level[e] + 1);
        p.pass_start.assign(n_levels + 1, 0);
        for (size_t e = 0; e < E.size(); ++e) p.pass_start[level[e] + 1]++;
        for (int l = 0; l < n_levels; ++l) p.pass_start[l + 1] += p.pass_start[l];
        // record order: by pass, then by first cell and direction, so that the
        // edges around a cell are processed close together and its counts
        // are fetched into a cache once (a counting sort by pass of the
        // edges taken in (first cell, direction) order)
        const int nfwd = p.lattice == TISSUE_LATTICE_SQUARE ? 2 : 3;
        std::vector<int32_t> by_cell((size_t)p.ncell * nfwd, -1);
        for (size_t e = 0; e < E.size(); ++e) by_cell[(size_t)E[e].i * nfwd + E[e].d] = (int32_t)e;
        std::vector<uint32_t> ord(E.size());
        {
            std::vector<uint32_t> at(p.pass_start.begin(), p.pass_start.end() - 1);
            for (const int32_t e : by_cell)
                if (e >= 0) ord[at[level[e]]++] = (uint32_t)e;
        }
        for (size_t k = 0; k < ord.size(); ++k) {
            const uint32_t e = ord[k];
            const Edge &ed = E[e];
            EdgeRec r{};
            r.id = e;
            r.vox_i = p.vox_off[ed.i];
            r.vox_j = p.vox_off[ed.j];
            const auto &gi = group_i(ed);
            const auto &gj = group_j(ed);
            if (gi.size() > (size_t)kMaxFace || gj.size() > (size_t)kMaxFace)
                return fail(TISSUE_EINVAL, "face group larger than supported");
            r.m_a = (uint8_t)gi.size();
            r.m_b = (uint8_t)gj.size();
            r.model_i = p.cell_model[ed.i];
            r.model_j = p.cell_model[ed.j];
            for (size_t q = 0; q < gi.size(); ++q) r.A[q] = (uint8_t)gi[q];
            for (size_t q = 0; q < gj.size(); ++q) r.B[q] = (uint8_t)gj[q];
            p.edges[k] = r;
        }
        p.face_kind = -1;
        for (const EdgeRec &r : p.edges) {
            const int k = (r.m_a == 2 && r.m_b == 2) ? 2 : (r.m_a == 1 && r.m_b == 1) ? 1 : 0;
            p.face_kind = p.face_kind < 0 || p.face_kind == k ? k : 0;
        }
        if (p.face_kind < 0) p.face_kind = 0;
        for (int l = 0; l < n_levels; ++l) {
            std::vector<SItem> pass;
            for (uint32_t o = p.pass_start[l]; o < p.pass_start[l + 1]; o += kWave)
                pass.push_back(SItem{0, o, std::min<uint32_t>(kWave, p.pass_start[l + 1] - o), 0});
            p.s_passes.push_back(std::move(pass));
        }
        for (auto &ps : p.s_passes) p.n_s_items += ps.size();
        if (p.n_s_items > s_item_room((int)p.lattice, p.nedge))
            return fail(TISSUE_EINVAL, "internal: S work items over their room");
    }

    // device layout
    if (d->flags & TISSUE_FLAG_TRACE) p.trace_steps = d->trace_steps;
    p.strang = (d->flags & TISSUE_FLAG_STRANG) != 0;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1));
        return at;
    };
    p.off_tissue = take(sizeof(DevTissue));
    p.off_tbl = take(sizeof(DevTissue *));
    p.off_counts = take((size_t)p.nvox * S * 4);
    p.off_init = take((size_t)p.nvox * S * 4);
    p.off_voxoff = take((size_t)p.ncell * 4);
    p.off_wh = take((size_t)p.ncell * 2);
    p.off_cells = take((size_t)p.ncell * 4);
    p.off_edges = take((size_t)p.nedge * sizeof(EdgeRec));
    p.off_models = take(p.models.size() * sizeof(DevModel));
    p.off_chi = take(p.n_chi_items * sizeof(ChiItem));
    p.off_s = take(s_item_room((int)p.lattice, p.nedge) * sizeof(SItem));
    p.off_ctl = take(64);  // stats[3] u64, flags[2] u32
    p.off_lq = take(kLaunchQueueBytes);  // per-launch queue words of the chi launches
    p.off_load = take((size_t)p.ncell * 4);  // per-cell load: the regroup pass's key
    p.off_retry = take((size_t)p.ncell * sizeof(ChiItem));  // lane16 cells to redo
    p.off_trace = take((size_t)p.trace_steps * ((size_t)p.ncell * 12 + (size_t)p.nedge * 12));
    p.bytes = o;
    return TISSUE_OK;
}

// ---------------------------------------------------------------------------
// launch plan: what one "step" enqueues, for a tissue or a batch
// ---------------------------------------------------------------------------

struct ChiLaunch {
    int mode;                // kChiLane, kChiRow or kChiLane16
    int rw;                  // kChiRow: lanes per cell (16, 32 or 64)
    size_t retry_lds;        // lane16: LDS of the full-width redo launch
    const JitKernels *jit;   // compiled-network kernels, or null: generic ones
    int SM, RM, NDM;         // generic kernel instantiation (table sizes)
    int P, cells_per_item;
    size_t lds;
    const ChiItem *items;
    uint32_t n_items;
    uint32_t retry_off;      // compact layout: this launch's part of the redo list
    const ChiItem *segs;     // regroup segments (a class's cells of one member), or none
    uint32_t n_segs;
    int prio;                // nonzero: wavefronts at a raised issue priority
};

// chi mode request: lane, row, automatic, compact (lane16), or wide rows.
// Automatic: cells of at most 8 leaves take the lane layout (small in LDS,
// few tree levels; a row would idle most of its lanes); classes of 16, 32
// or 64 leaves take the compact layout when it has at least 16 lanes of
// work per SIMD of the device (cells x P / 16), else rows of P lanes, whose
// event chains are shorter (one voxel per lane) but which spend a row of
// lanes per event.  Compact: every class in the compact layout (P / 16
// lanes per cell above 16 leaves).  Wide rows: rows of max(32, P) lanes,
// half as many cells per wavefront as rows of 16 for the small cells, so
// twice the wavefronts.
enum { kModeLane = 0, kModeRow = 1, kModeAuto = 2, kModeLane16 = 3, kModeRowWide = 4 };

// Work items and launches of the chi operator over a set of tissues: one
// launch per (leaf class, kernel instantiation).  Items are written to
// items_out in launch order; ChiLaunch.items holds offsets until rebased.
void plan_chi(const std::vector<const Plan *> &members, int mode_req, int regroup, int n_simd,
              std::vector<ChiItem> &items_out, std::vector<ChiLaunch> &launches)
{
    struct Key {
        int P;
        std::string net;  // compiled network key, or the generic table sizes
        bool operator<(const Key &o) const
        {
            if (P != o.P) return P > o.P;  // largest cells first
            return net < o.net;
        }
    };
    struct Group {
        const JitKernels *jit = nullptr;
        int SM = 0, RM = 0, NDM = 0, max_s = 0;
        std::vector<std::pair<uint32_t, const ChiGroupHost *>> cells;
    };
    std::map<Key, Group> groups;
    // the network key of a class (compiled network, or generic table sizes)
    auto net_of = [](const Plan &p, const ChiGroupHost &g, int &SM, int &RM, int &NDM) {
        const DevModel &M = p.models[(size_t)g.model];
        chi_variant((int)p.S, M.n_reactions, M.n_diff, SM, RM, NDM);
        return p.jits[(size_t)g.model] ? "J" + p.net_keys[(size_t)g.model]
                                       : "G" + std::to_string(SM) + "," + std::to_string(RM) + "," +
                                             std::to_string(NDM);
    };
    // automatic: where the cells of 3 to 16 voxels of a network hold the
    // compact layout's 16 lanes of work per SIMD, the classes of 4 and 8
    // leaves join the 16-leaf class's compact launch (its tree over 16
    // leaves gives a smaller cell the same bits: padding leaves add 0), one
    // launch instead of a lane-layout launch per small class; cells of one
    // or two voxels keep the lane layout, whose trees are shorter still
    std::map<std::string, uint64_t> small_cells;
    if (mode_req == kModeAuto)
        for (const Plan *pp : members)
            for (const ChiGroupHost &g : pp->chi)
                if (g.P >= 4 && g.P <= 16) {
                    int a, b, c;
                    small_cells[net_of(*pp, g, a, b, c)] += g.count;
                }
    for (size_t i = 0; i < members.size(); ++i) {
        const Plan &p = *members[i];
        for (const ChiGroupHost &g : p.chi) {
            const JitKernels *jit = p.jits[(size_t)g.model];
            int SM, RM, NDM;
            const std::string net = net_of(p, g, SM, RM, NDM);
            int P = g.P;
            if (P >= 4 && P < 16 && mode_req == kModeAuto &&
                small_cells[net] >= 16ull * (uint64_t)std::max(n_simd, 1))
                P = 16;
            Group &G = groups[Key{P, net}];
            G.jit = jit;
            G.SM = SM;
            G.RM = RM;
            G.NDM = NDM;
            G.max_s = std::max(G.max_s, (int)p.S);
            G.cells.push_back({(uint32_t)i, &g});
        }
    }
    items_out.clear();
    launches.clear();
    std::vector<ChiItem> segs_out;  // regroup segments, appended after the items
    uint64_t retry_cells = 0;  // cells of the compact launches so far
    for (auto &kv : groups) {
        const Key &k = kv.first;
        const Group &G = kv.second;
        uint64_t cells = 0;
        for (auto &m : G.cells) cells += m.second->count;
        int mode = kChiLane;
        int rw = std::max(16, k.P);
        if (mode_req == kModeRow) mode = kChiRow;  // rows of max(16, P) lanes
        if (mode_req == kModeRowWide) {
            mode = kChiRow;
            rw = std::max(32, k.P);
        }
        if (mode_req == kModeLane16 && k.P <= 64) mode = kChiLane16;
        if (mode_req == kModeAuto && k.P >= 16 && k.P <= 64) {
            const uint64_t lanes = cells * (uint64_t)compact_lanes(k.P);
            mode = lanes >= 16ull * (uint64_t)std::max(n_simd, 1) ? kChiLane16 : kChiRow;
        }
        ChiLaunch L;
        L.mode = mode;
        L.rw = rw;
        L.jit = G.jit;
        L.SM = G.SM;
        L.RM = G.RM;
        L.NDM = G.NDM;
        L.P = k.P;
        if (mode == kChiRow) {
            L.cells_per_item = kWave / rw;
        } else if (mode == kChiLane16) {
            int cpi = kWave / compact_lanes(k.P);
            while (cpi > 1 && chi_lds_bytes(kChiLane16, k.P, G.max_s, cpi) > kChiLdsBudget) cpi >>= 1;
            L.cells_per_item = cpi;
        } else {
            L.cells_per_item = lane_cells_per_item(k.P, G.max_s);
        }
        L.lds = chi_lds_bytes(mode, k.P, G.max_s, L.cells_per_item);
        L.retry_lds = chi_lds_bytes(kChiLane, k.P, G.max_s, 1);
        L.retry_off = (uint32_t)retry_cells;
        if (mode == kChiLane16) retry_cells += cells;
        L.segs = nullptr;
        L.n_segs = 0;
        L.prio = 0;
        // regroup of a compact class: on request, or automatically when the
        // launch spans at least two wavefronts (grouping cells of similar
        // load shortens each wavefront's wait for its busiest cell and, with
        // the heaviest items first, frees SIMDs early for other classes)
        const bool rg = mode == kChiLane16 && regroup != 0 &&
                        (regroup == 1 || cells * (uint64_t)compact_lanes(k.P) >= 2ull * kWave);
        if (rg) {
            L.segs = reinterpret_cast<const ChiItem *>(segs_out.size());
            for (auto &m : G.cells)
                for (uint32_t o = 0; o < m.second->count; o += kRegroupChunk)
                    segs_out.push_back(ChiItem{m.first, m.second->first + o,
                                               std::min(kRegroupChunk, m.second->count - o),
                                               (uint32_t)m.second->model});
            L.n_segs = (uint32_t)(segs_out.size() - reinterpret_cast<uintptr_t>(L.segs));
        }
        // the row head: in a single tissue the 64-leaf cells' event chains
        // are the longest of a step, and the compact layout advances a chain
        // more slowly than a row of 64 lanes; once regrouped (heaviest
        // first), the first min(SIMDs, cells / 4) cells of the class run in
        // rows, one wavefront each, the rest compact
        uint32_t head = 0;
        if (rg && mode_req == kModeAuto && k.P == 64 && G.cells.size() == 1)
            head = (uint32_t)std::min<uint64_t>((uint64_t)std::max(n_simd, 1), cells / 4);
        const size_t off = items_out.size();
        for (auto &m : G.cells) {
            ChiGroupHost g = *m.second;
            g.first += head;
            g.count -= head;
            cut_items(m.first, g, L.cells_per_item, items_out);
        }
        L.items = reinterpret_cast<const ChiItem *>(off);
        L.n_items = (uint32_t)(items_out.size() - off);
        if (head > 0) {
            // the head first, carrying the class's regroup (in launch order
            // the regroup precedes both parts; a step graph regroups every
            // class before it forks)
            ChiLaunch R = L;
            R.mode = kChiRow;
            R.rw = 64;
            R.cells_per_item = 1;
            R.lds = chi_lds_bytes(kChiRow, k.P, G.max_s, 1);
            const size_t roff = items_out.size();
            ChiGroupHost g = *G.cells[0].second;
            g.count = head;
            cut_items(G.cells[0].first, g, 1, items_out);
            R.items = reinterpret_cast<const ChiItem *>(roff);
            R.n_items = (uint32_t)(items_out.size() - roff);
            launches.push_back(R);
            L.segs = nullptr;
            L.n_segs = 0;
        }
        launches.push_back(L);
    }
    // several classes' launches share the device (as parallel branches of a
    // step graph): the compact launches -- many wavefronts, the step's
    // longest event chains (the largest cells), issue-bound -- get a raised
    // issue priority over the rows, whose one-cell wavefronts fill the
    // SIMDs' remaining issue slots (the uneven 256x256 tissue: 9.3e9 ->
    // 1.16e10 events/s; the same bits, only the order of issue changes)
    int with_items = 0;
    for (const ChiLaunch &L : launches) with_items += L.n_items > 0;
    if (with_items > 1)
        for (ChiLaunch &L : launches) L.prio = L.mode == kChiLane16 ? 1 : 0;
    // every launch's regroup segments after all items, contiguous, so that
    // a step graph can regroup every class in one launch before it forks
    const size_t seg_base = items_out.size();
    items_out.insert(items_out.end(), segs_out.begin(), segs_out.end());
    for (ChiLaunch &L : launches)
        if (L.n_segs) L.segs = reinterpret_cast<const ChiItem *>(seg_base + reinterpret_cast<uintptr_t>(L.segs));
}

struct SLaunch {
    const SItem *items;
    uint32_t n_items;
    int fix;  // 2 or 1: every edge's face groups have 2 and 2 (1 and 1) voxels; else 0
};

struct GraphKey {
    uint64_t dt_bits;
    int32_t steps;
    bool operator<(const GraphKey &o) const
    {
        return dt_bits != o.dt_bits ? dt_bits < o.dt_bits : steps < o.steps;
    }
};

struct LaunchPlan {
    DevTissue **tbl = nullptr;  // device table of DevTissue pointers
    uint32_t n_tissues = 0;
    DevTissue *rec0 = nullptr;  // device record of the first member
    std::vector<const Plan *> members;
    ChiItem *chi_items = nullptr;  // device region for chi work items
    size_t chi_items_cap = 0;
    ChiItem *retry_items = nullptr;  // device region: compact-layout cells to redo (one per cell)
    uint32_t *lq = nullptr;     // device: kQueueBlockWords queue words per chi launch
    int chi_mode = kModeAuto;
    int regroup = 2;            // regroup pass before compact launches: 0 off, 1 on, 2 automatic
    std::vector<ChiLaunch> chi;
    std::vector<SLaunch> s;
    hipStream_t stream = nullptr;
    int persistent = 1;
    bool strang = false;        // chi over dt/2 (tag 0), S over dt, chi over dt/2 (tag 2)
    int wpc = 0;                // workgroups per CU in persistent mode (0 auto)
    int cus = 0;
    int graph_chunk = 50;
    // compact launches of cells of at most 16 voxels with compiled networks
    // and a persistent grid: a wavefront refills its idle lanes with new
    // cells once this many are idle (0: never; lanes wait for their item)
    int refill_min = kDefaultRefillMin;
    // small tissues: every step of a call in one launch of the network's
    // whole-run kernel (when the plan fits it; 0: never)
    int whole_run = 1;
    hipStream_t capture_stream = nullptr;
    std::map<GraphKey, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    // side streams and fork/join events for running the leaf-count classes'
    // chi launches of one step concurrently
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork_ev = nullptr;

    ~LaunchPlan()
    {
        clear_graphs();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        for (hipStream_t s : side) (void)hipStreamDestroy(s);
        for (hipEvent_t e : joins) (void)hipEventDestroy(e);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
    }

    // Streams and events for n concurrent chi launches (n - 1 side streams).
    int ensure_side(size_t n)
    {
        if (!fork_ev) HIP_TRY(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
        while (side.size() + 1 < n) {
            hipStream_t s = nullptr;
            hipEvent_t e = nullptr;
            HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            side.push_back(s);
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            joins.push_back(e);
        }
        return TISSUE_OK;
    }

    void clear_graphs()
    {
        for (auto &kv : graphs) {
            (void)hipGraphExecDestroy(kv.second.second);
            (void)hipGraphDestroy(kv.second.first);
        }
        graphs.clear();
    }

    // One chi launch of a group; for the compact layout also the full-width
    // redo of the cells it handed back (a persistent launch that reads the
    // count from device memory and exits at once when it is zero).  Each
    // launch uses its own queue words and its own part of the redo list.
    hipError_t launch_chi_any(const ChiLaunch &L, uint32_t grid, hipStream_t st, double dt,
                              uint32_t kstep, uint32_t tag, bool regrouped = false)
    {
        uint32_t *const q = lq + kQueueBlockWords * (size_t)(&L - chi.data());
        if (L.n_segs && !regrouped) {  // regroup the class's cells by load first (same stream)
            const hipError_t er = launch_regroup(st, tbl, L.segs, L.n_segs);
            if (er != hipSuccess) return er;
        }
        int log2p = 0;
        while ((1 << log2p) < L.P) ++log2p;
        ChiArgs a{};
        a.mode = L.mode;
        a.P = L.P;
        a.rw = L.rw;
        a.grid = grid;
        a.lds = L.lds;
        a.stream = st;
        a.tbl = tbl;
        a.items = L.items;
        a.n_items = L.n_items;
        a.queue = q + kQNext;
        a.persistent = persistent;
        a.cells_per_item = L.cells_per_item;
        a.dt = dt;
        a.kstep = kstep;
        a.tag = tag;
        a.retry_items = retry_items + L.retry_off;
        a.retry_count = q + kQRetry;
        a.prio = L.prio;
        hipError_t e = hipSuccess;
        if (!L.jit) {
            e = launch_chi(L.SM, L.RM, L.NDM, a);
        } else if (L.mode == kChiRow) {
            void *args[] = {&a.tbl, &a.items, &a.n_items, &a.queue, &a.persistent, &a.dt, &a.kstep,
                            &a.tag, &a.prio};
            hipFunction_t f = L.rw == 64 ? L.jit->row64 : L.rw == 32 ? L.jit->row32 : L.jit->row;
            e = hipModuleLaunchKernel(f, grid, 1, 1, kWave, 1, 1, 0, st, args, nullptr);
        } else if (refills(L)) {
            int rmin = refill_min;
            void *args[] = {&a.tbl, &a.items, &a.n_items, &a.queue, &a.persistent, &a.dt, &a.kstep,
                            &a.tag, &a.retry_items, &a.retry_count, &rmin};
            e = hipModuleLaunchKernel(L.jit->lane16r, grid, 1, 1, kWave, 1, 1, (unsigned)L.lds, st,
                                      args, nullptr);
        } else if (L.mode == kChiLane16) {
            void *args[] = {&a.tbl, &a.items, &a.n_items, &a.queue, &a.persistent, &a.cells_per_item,
                            &a.dt, &a.kstep, &a.tag, &a.retry_items, &a.retry_count, &a.prio};
            hipFunction_t f = L.P == 64 ? L.jit->lane16x4 : L.P == 32 ? L.jit->lane16x2 : L.jit->lane16;
            e = hipModuleLaunchKernel(f, grid, 1, 1, kWave, 1, 1, (unsigned)L.lds, st, args, nullptr);
        } else {
            uint32_t *none = nullptr;
            void *args[] = {&a.tbl, &a.items, &a.n_items, &a.queue, &a.persistent, &a.cells_per_item,
                            &log2p, &a.dt, &a.kstep, &a.tag, &none, &a.prio};
            e = hipModuleLaunchKernel(L.jit->lane, grid, 1, 1, kWave, 1, 1, (unsigned)L.lds, st,
                                      args, nullptr);
        }
        if (e != hipSuccess || L.mode != kChiLane16) return e;
        // the redo launch: one cell per item, full-width layout
        ChiArgs r = a;
        r.mode = kChiLane;
        r.grid = (uint32_t)std::max(1, cus);
        r.lds = L.retry_lds;
        r.items = retry_items + L.retry_off;
        r.n_items = 0;
        r.queue = q + kQRetryNext;
        r.persistent = 1;
        r.cells_per_item = 1;
        r.n_items_dev = q + kQRetry;
        if (!L.jit) return launch_chi(L.SM, L.RM, L.NDM, r);
        void *args[] = {&r.tbl, &r.items, &r.n_items, &r.queue, &r.persistent, &r.cells_per_item,
                        &log2p, &r.dt, &r.kstep, &r.tag, &r.n_items_dev, &r.prio};
        return hipModuleLaunchKernel(L.jit->lane, r.grid, 1, 1, kWave, 1, 1, (unsigned)r.lds, st,
                                     args, nullptr);
    }

    // whether a chi launch runs the compact layout with lane refill
    bool refills(const ChiLaunch &L) const
    {
        return L.mode == kChiLane16 && L.P <= 16 && persistent && refill_min > 0 &&
               L.cells_per_item == kWave && L.jit && L.jit->lane16r;
    }

    uint32_t chi_grid(const ChiLaunch &L) const
    {
        if (!persistent) return L.n_items;
        int per_cu = wpc;
        if (per_cu <= 0) per_cu = (int)std::min<size_t>(16, std::max<size_t>(1, kLdsPerCu / (L.lds + kChiStaticLds)));
        return std::max<uint32_t>(1, std::min<uint32_t>(L.n_items, (uint32_t)(cus * per_cu)));
    }


    // Enqueue n steps (k = 0..n-1) then step_base += n.  With events
    // (2 per launch, in launch order) each kernel is bracketed; kind gets the
    // chi launch's index in `chi`, or -1 for an S launch.
    int enqueue(hipStream_t st, double dt, int32_t n, std::vector<hipEvent_t> *ev = nullptr,
                std::vector<int> *kind = nullptr)
    {
        size_t e = 0;
        // the chi launches of one (half-)step, counter tag `tag`.  Classes
        // touch disjoint cells and every launch has its own queue words and
        // redo list, so with one workgroup per item the captured step graph
        // runs them as parallel branches: one branch on `st`, the others on
        // side streams forked from and joined back into it.  Eager launches
        // (timed runs, serving) keep every launch in order on the caller's
        // stream.
        size_t branches = 0;
        for (const ChiLaunch &L : chi) branches += L.n_items > 0;
        const bool fork = !ev && !persistent && branches > 1 && st == capture_stream;
        if (fork) {
            const int rc = ensure_side(branches);
            if (rc != TISSUE_OK) return rc;
        }
        auto chi_pass = [&](double dchi, uint32_t k, uint32_t tag) -> int {
            if (fork) {
                // every class's regroup in one launch, then the branches
                const ChiItem *segs = nullptr;
                uint32_t n_segs = 0;
                for (const ChiLaunch &L : chi)
                    if (L.n_segs) {
                        if (!segs) segs = L.segs;
                        n_segs += L.n_segs;
                    }
                if (n_segs) HIP_TRY(launch_regroup(st, tbl, segs, n_segs));
                HIP_TRY(hipEventRecord(fork_ev, st));
                size_t b = 0;
                for (const ChiLaunch &L : chi) {
                    if (L.n_items == 0) continue;
                    if (b == 0) {
                        HIP_TRY(launch_chi_any(L, chi_grid(L), st, dchi, k, tag, true));
                    } else {
                        hipStream_t ss = side[b - 1];
                        HIP_TRY(hipStreamWaitEvent(ss, fork_ev, 0));
                        HIP_TRY(launch_chi_any(L, chi_grid(L), ss, dchi, k, tag, true));
                        HIP_TRY(hipEventRecord(joins[b - 1], ss));
                    }
                    ++b;
                }
                for (size_t i = 0; i + 1 < b; ++i) HIP_TRY(hipStreamWaitEvent(st, joins[i], 0));
                return TISSUE_OK;
            }
            for (const ChiLaunch &L : chi) {
                if (L.n_items == 0) continue;
                if (ev) HIP_TRY(hipEventRecord((*ev)[e++], st));
                HIP_TRY(launch_chi_any(L, chi_grid(L), st, dchi, k, tag));
                if (ev) {
                    HIP_TRY(hipEventRecord((*ev)[e++], st));
                    kind->push_back((int)(&L - chi.data()));
                }
            }
            return TISSUE_OK;
        };
        const double dchi = strang ? dt * 0.5 : dt;
        for (int32_t k = 0; k < n; ++k) {
            int rc = chi_pass(dchi, (uint32_t)k, 0u);
            if (rc != TISSUE_OK) return rc;
            for (const SLaunch &L : s) {
                if (L.n_items == 0) continue;
                if (ev) HIP_TRY(hipEventRecord((*ev)[e++], st));
                // the S operator: one workgroup per item of 64 edges, whatever
                // the chi launch shape (its face-count gathers wait on memory,
                // and many resident workgroups hide that better than a
                // persistent grid: 2 % on the batched sweep)
                HIP_TRY(launch_s(st, tbl, L.items, L.n_items, dt, (uint32_t)k, L.fix));
                if (ev) {
                    HIP_TRY(hipEventRecord((*ev)[e++], st));
                    kind->push_back(-1);
                }
            }
            if (strang) {
                rc = chi_pass(dchi, (uint32_t)k, 2u);
                if (rc != TISSUE_OK) return rc;
            }
        }
        HIP_TRY(launch_advance(st, tbl, n_tissues, (uint32_t)n));
        return TISSUE_OK;
    }

    // (Re)plan the chi launches for a mode request and upload their items.
    int set_chi_mode(int mode)
    {
        std::vector<ChiItem> items;
        std::vector<ChiLaunch> launches;
        plan_chi(members, mode, regroup, cus * 4, items, launches);
        if (items.size() > chi_items_cap) return fail(TISSUE_EINVAL, "chi item region too small");
        if (launches.size() > (size_t)kMaxChiLaunches) return fail(TISSUE_EINVAL, "too many chi launch groups");
        HIP_TRY(hipStreamSynchronize(stream));
        if (!items.empty()) {
            std::unique_lock<std::mutex> lk;
            unsigned char *h = nullptr;
            const size_t nb = items.size() * sizeof(ChiItem);
            HIP_TRY(staging_acquire(lk, nb, &h));
            std::memcpy(h, items.data(), nb);
            HIP_TRY(hipMemcpyAsync(chi_items, h, nb, hipMemcpyHostToDevice, stream));
            HIP_TRY(hipStreamSynchronize(stream));
        }
        for (ChiLaunch &L : launches) {
            L.items = chi_items + reinterpret_cast<uintptr_t>(L.items);
            if (L.n_segs) L.segs = chi_items + reinterpret_cast<uintptr_t>(L.segs);
        }
        chi = std::move(launches);
        chi_mode = mode;
        clear_graphs();
        return TISSUE_OK;
    }

    int launches_per_step() const
    {
        int c = 0;
        for (const ChiLaunch &L : chi) c += (L.n_items > 0) * (strang ? 2 : 1);
        for (const SLaunch &L : s) c += L.n_items > 0;
        return c;
    }

    // The whole-run kernel's description of this plan: one tissue whose
    // chi operator is one work item of the one-lane-per-cell layout with a
    // compiled network, at most kSmallPasses S passes of at most
    // kSmallItems items, and copies that fit the kernel's LDS (lds: its
    // dynamic LDS, the chi item's area then the copies, 16-byte aligned).
    bool small_run(SmallRun &r, const JitKernels *&jk, size_t &lds) const
    {
        r = SmallRun{};
        jk = nullptr;
        lds = 0;
        if (n_tissues != 1 || members.size() != 1 || !rec0) return false;
        const ChiLaunch *one = nullptr;
        for (const ChiLaunch &L : chi) {
            if (L.n_items == 0) continue;
            if (one || L.n_items != 1 || L.mode != kChiLane || !L.jit || !L.jit->run_small) return false;
            one = &L;
        }
        if (!one) return false;
        jk = one->jit;
        int log2p = 0;
        while ((1 << log2p) < one->P) ++log2p;
        r.chi_item = one->items;
        r.chi_cells_per_item = one->cells_per_item;
        r.chi_log2p = log2p;
        for (const SLaunch &L : s) {
            if (L.n_items == 0) continue;
            if (r.n_s == kSmallPasses || L.n_items > (uint32_t)kSmallItems) return false;
            r.s_items[r.n_s] = L.items;
            r.s_n[r.n_s] = L.n_items;
            ++r.n_s;
        }
        // the copies in LDS, after the chi item's area
        size_t o = one->lds;
        auto take = [&](size_t bytes) {
            const size_t at = (o + 15) & ~(size_t)15;
            o = at + bytes;
            return (uint32_t)at;
        };
        const Plan &p = *members[0];
        r.n_counts = p.nvox * p.S;
        r.n_models = (uint32_t)p.models.size();
        r.rec = take(sizeof(DevTissue));
        r.counts = take((size_t)r.n_counts * 4);
        r.vox_off = take((size_t)p.ncell * 4);
        r.wh = take((size_t)p.ncell * 2);
        r.cell_list = take((size_t)p.ncell * 4);
        r.edges = take((size_t)p.nedge * sizeof(EdgeRec));
        r.models = take((size_t)r.n_models * sizeof(DevModel));
        r.tbl = take(sizeof(DevTissue *));
        r.chi_item_lds = take(sizeof(ChiItem));
        for (int c = 0; c < r.n_s; ++c) r.s_items_lds[c] = take(r.s_n[c] * sizeof(SItem));
        if (o > kSmallLds) return false;
        lds = o;
        r.strang = strang ? 1 : 0;
        return true;
    }

    int run(double dt, int32_t n)
    {
        SmallRun sr;
        const JitKernels *jk = nullptr;
        size_t lds = 0;
        if (whole_run && n > 0 && small_run(sr, jk, lds)) {
            // one workgroup runs every step; launches of at most
            // kWholeRunSteps steps keep each kernel short
            for (int32_t left = n; left > 0;) {
                uint32_t m = (uint32_t)std::min<int32_t>(left, kWholeRunSteps);
                DevTissue *rec = rec0;
                void *args[] = {&rec, &sr, &dt, &m};
                HIP_TRY(hipModuleLaunchKernel(jk->run_small, 1, 1, 1, kWave, 1, 1, (unsigned)lds,
                                              stream, args, nullptr));
                left -= (int32_t)m;
            }
            return TISSUE_OK;
        }
        int32_t left = n;
        if (graph_chunk > 0 && n >= graph_chunk) {
            uint64_t bits;
            std::memcpy(&bits, &dt, 8);
            GraphKey key{bits, graph_chunk};
            auto it = graphs.find(key);
            if (it == graphs.end()) {
                if (!capture_stream) HIP_TRY(hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking));
                hipGraph_t g = nullptr;
                hipGraphExec_t ge = nullptr;
                HIP_TRY(hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal));
                const int rc = enqueue(capture_stream, dt, graph_chunk);
                hipGraph_t captured = nullptr;
                const hipError_t ee = hipStreamEndCapture(capture_stream, &captured);
                if (rc != TISSUE_OK) {
                    if (captured) (void)hipGraphDestroy(captured);
                    return rc;
                }
                if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
                g = captured;
                HIP_TRY(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
                it = graphs.emplace(key, std::make_pair(g, ge)).first;
            }
            while (left >= graph_chunk) {
                HIP_TRY(hipGraphLaunch(it->second.second, stream));
                left -= graph_chunk;
            }
        }
        if (left > 0) return enqueue(stream, dt, left);
        return TISSUE_OK;
    }

    int run_timed(double dt, int32_t n, tissue_timing_t *out)
    {
        const size_t launches = (size_t)n * launches_per_step();
        std::vector<hipEvent_t> ev(2 * launches);
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        std::vector<int> kind;
        hipEvent_t t0, t1;
        HIP_TRY(hipEventCreate(&t0));
        HIP_TRY(hipEventCreate(&t1));
        HIP_TRY(hipEventRecord(t0, stream));
        int rc = enqueue(stream, dt, n, &ev, &kind);
        if (rc != TISSUE_OK) return rc;
        HIP_TRY(hipEventRecord(t1, stream));
        HIP_TRY(hipEventSynchronize(t1));
        tissue_timing_t T{};
        std::vector<double> per_group(chi.size(), 0.0);
        for (size_t q = 0; q < kind.size(); ++q) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[2 * q], ev[2 * q + 1]));
            if (kind[q] >= 0) {
                T.chi_ms += ms;
                T.chi_launches++;
                per_group[(size_t)kind[q]] += ms;
            } else {
                T.s_ms += ms;
                T.s_launches++;
            }
        }
        T.chi_kernel = -1;
        double longest = -1.0;
        for (size_t g = 0; g < chi.size(); ++g) {
            if (chi[g].n_items == 0 || per_group[g] <= longest) continue;
            longest = per_group[g];
            T.chi_kernel = chi[g].mode == kChiRow ? (chi[g].rw > std::max(16, chi[g].P) ? kModeRowWide : kModeRow)
                         : chi[g].mode == kChiLane16 ? kModeLane16 : kModeLane;
            T.chi_leaves = chi[g].P;
            T.chi_refill = refills(chi[g]) ? 1 : 0;
        }
        float tot = 0.f;
        HIP_TRY(hipEventElapsedTime(&tot, t0, t1));
        T.total_ms = tot;
        for (auto &e : ev) (void)hipEventDestroy(e);
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        if (out) *out = T;
        return TISSUE_OK;
    }
};

int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

}  // namespace

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------

struct tissue {
    Plan plan;
    unsigned char *dev = nullptr;
    hipStream_t stream = nullptr;
    DevTissue host_rec{};          // last uploaded DevTissue (host copy)
    uint32_t steps_done = 0;
    int batches = 0;               // live batches holding this tissue
    hipEvent_t ready = nullptr;    // marks the tissue's stream for batches on other streams
    LaunchPlan lp;
    DevTissue *d_rec() const { return reinterpret_cast<DevTissue *>(dev + plan.off_tissue); }
    int32_t *d_counts() const { return reinterpret_cast<int32_t *>(dev + plan.off_counts); }
    unsigned char *d_ctl() const { return dev + plan.off_ctl; }
};

struct tissue_batch {
    std::vector<tissue *> members;
    unsigned char *dev = nullptr;
    size_t bytes = 0;                 // dev_buf's size: the capacity of set_members
    LaunchPlan lp;
    // set_members: the image of the work lists in pinned host memory (grown
    // on demand) and the event after its last copy
    unsigned char *stage = nullptr;
    size_t stage_cap = 0;
    hipEvent_t staged = nullptr;
    ~tissue_batch()
    {
        if (staged) (void)hipEventDestroy(staged);
        if (stage) (void)hipHostFree(stage);
    }
};

extern "C" {

const char *tissue_strerror(int code)
{
    switch (code) {
    case TISSUE_OK: return "ok";
    case TISSUE_EINVAL: return "invalid argument";
    case TISSUE_ENOMEM: return "device buffer too small";
    case TISSUE_EOVERFLOW: return "a species count left [0, 2^26)";
    case TISSUE_EDEVICE: return "HIP runtime error";
    case TISSUE_EBUSY: return "busy";
    case TISSUE_ESTATE: return "invalid state";
    case TISSUE_ELIMIT: return "a unit-step reached the event cap";
    default: return "unknown error";
    }
}

const char *tissue_last_error(void) { return g_last_error.c_str(); }

int tissue_device_cus(int32_t *out)
{
    if (!out) return fail(TISSUE_EINVAL, "null output");
    const int c = device_cus();
    if (c <= 0) return fail(TISSUE_EDEVICE, "no HIP device");
    *out = c;
    return TISSUE_OK;
}

int tissue_network_check(const tissue_desc_t *d)
{
    Plan p;
    const int rc = build_plan(d, p);
    if (rc != TISSUE_OK) return rc;
    std::string err;
    for (const DevModel &M : p.models)
        if (jit_compile_check(M, err) != 0) return fail(TISSUE_EDEVICE, err);
    return TISSUE_OK;
}

size_t tissue_required_bytes(const tissue_desc_t *d)
{
    Plan p;
    if (build_plan(d, p, false) != TISSUE_OK) return 0;
    return p.bytes;
}

int tissue_create(const tissue_desc_t *d, void *dev_buf, size_t dev_bytes, void *hip_stream,
                  tissue_t **out)
{
    if (!out) return fail(TISSUE_EINVAL, "null output handle");
    *out = nullptr;
    std::unique_ptr<tissue> t(new tissue());
    int rc = build_plan(d, t->plan);
    if (rc != TISSUE_OK) return rc;
    Plan &p = t->plan;
    if (!dev_buf || ((uintptr_t)dev_buf % kAlign) != 0)
        return fail(TISSUE_EINVAL, "dev_buf must be non-null and 256-byte aligned");
    if (dev_bytes < p.bytes)
        return fail(TISSUE_ENOMEM, "dev_bytes " + std::to_string(dev_bytes) + " < required " +
                                       std::to_string(p.bytes));
    t->dev = static_cast<unsigned char *>(dev_buf);
    t->stream = static_cast<hipStream_t>(hip_stream);
    const int cus = device_cus();
    if (cus <= 0) return fail(TISSUE_EDEVICE, "no HIP device");
    if (!(d->flags & TISSUE_FLAG_NO_JIT)) {
        // each network's own chi kernels; the generic ones serve a network
        // whose compilation fails
        std::string err;
        p.all_jit = true;
        for (size_t m = 0; m < p.models.size(); ++m)
            if (jit_kernels(p.models[m], &p.jits[m], err) != 0) {
                p.jits[m] = nullptr;
                p.all_jit = false;
            }
    }

    unsigned char *base = t->dev;
    DevTissue &R = t->host_rec;
    R.counts = reinterpret_cast<int32_t *>(base + p.off_counts);
    R.vox_off = reinterpret_cast<const int32_t *>(base + p.off_voxoff);
    R.wh = reinterpret_cast<const uint8_t *>(base + p.off_wh);
    R.cell_list = reinterpret_cast<int32_t *>(base + p.off_cells);
    R.load = reinterpret_cast<float *>(base + p.off_load);
    R.edges = reinterpret_cast<const EdgeRec *>(base + p.off_edges);
    R.stats = reinterpret_cast<unsigned long long *>(base + p.off_ctl);
    R.flags = reinterpret_cast<uint32_t *>(base + p.off_ctl + 24);
    if (p.trace_steps) {
        unsigned char *tr = base + p.off_trace;
        const size_t nc = (size_t)p.trace_steps * p.ncell, ne = (size_t)p.trace_steps * p.nedge;
        R.tr_chi_t = reinterpret_cast<unsigned long long *>(tr);
        R.tr_s_t = reinterpret_cast<unsigned long long *>(tr + nc * 8);
        R.tr_chi_ev = reinterpret_cast<uint32_t *>(tr + nc * 8 + ne * 8);
        R.tr_s_ev = reinterpret_cast<uint32_t *>(tr + nc * 8 + ne * 8 + nc * 4);
    }
    R.seed = d->seed;
    R.n_cells = p.ncell;
    R.n_edges = p.nedge;
    R.sim_id = d->sim_id;
    R.step_base = d->start_step;
    R.event_cap = d->event_cap ? d->event_cap : TISSUE_DEFAULT_EVENT_CAP;
    R.trace_steps = p.trace_steps ? p.trace_steps : 1;
    R.models = reinterpret_cast<const DevModel *>(base + p.off_models);
    R.model = p.models[0];
    t->steps_done = d->start_step;

    // upload (synchronous on the tissue's stream): the buffer's image up to
    // the control block, assembled in pinned memory, in one copy
    hipStream_t st = t->stream;
    const size_t cbytes = (size_t)p.nvox * p.S * 4;
    DevTissue *d_rec = t->d_rec();
    std::vector<SItem> s_all;
    for (auto &ps : p.s_passes) s_all.insert(s_all.end(), ps.begin(), ps.end());
    {
        std::unique_lock<std::mutex> lk;
        unsigned char *h = nullptr;
        const size_t up = p.off_load + (size_t)p.ncell * 4;
        HIP_TRY(staging_acquire(lk, up, &h));
        std::memcpy(h + p.off_tissue, &R, sizeof(DevTissue));
        std::memcpy(h + p.off_tbl, &d_rec, sizeof(DevTissue *));
        std::memcpy(h + p.off_counts, d->init_counts, cbytes);
        std::memcpy(h + p.off_init, d->init_counts, cbytes);
        std::memcpy(h + p.off_voxoff, p.vox_off.data(), p.vox_off.size() * 4);
        std::memcpy(h + p.off_wh, p.wh.data(), p.wh.size());
        std::memcpy(h + p.off_cells, p.cell_list.data(), p.cell_list.size() * 4);
        if (p.nedge) std::memcpy(h + p.off_edges, p.edges.data(), p.edges.size() * sizeof(EdgeRec));
        std::memcpy(h + p.off_models, p.models.data(), p.models.size() * sizeof(DevModel));
        std::memset(h + p.off_chi, 0, p.off_s - p.off_chi);
        if (!s_all.empty()) std::memcpy(h + p.off_s, s_all.data(), s_all.size() * sizeof(SItem));
        std::memset(h + p.off_ctl, 0, up - p.off_ctl);
        HIP_TRY(hipMemcpyAsync(base, h, up, hipMemcpyHostToDevice, st));
        if (p.trace_steps)
            HIP_TRY(hipMemsetAsync(base + p.off_trace, 0,
                                   (size_t)p.trace_steps * ((size_t)p.ncell * 12 + (size_t)p.nedge * 12),
                                   st));
        HIP_TRY(hipStreamSynchronize(st));
    }

    // launch plan of this tissue alone
    LaunchPlan &L = t->lp;
    L.tbl = reinterpret_cast<DevTissue **>(base + p.off_tbl);
    L.n_tissues = 1;
    L.lq = reinterpret_cast<uint32_t *>(base + p.off_lq);
    L.stream = st;
    L.cus = cus;
    L.strang = p.strang;
    L.members = {&t->plan};
    L.rec0 = t->d_rec();
    L.retry_items = reinterpret_cast<ChiItem *>(base + p.off_retry);
    L.chi_items = reinterpret_cast<ChiItem *>(base + p.off_chi);
    L.chi_items_cap = p.n_chi_items;
    size_t off = 0;
    for (auto &ps : p.s_passes) {
        L.s.push_back(SLaunch{reinterpret_cast<const SItem *>(base + p.off_s) + off, (uint32_t)ps.size(),
                              p.face_kind});
        off += ps.size();
    }
    rc = L.set_chi_mode(kModeAuto);
    if (rc != TISSUE_OK) return rc;
    *out = t.release();
    return TISSUE_OK;
}

int tissue_step(tissue_t *t, double dt, int32_t n_steps)
{
    if (!t) return fail(TISSUE_EINVAL, "null tissue");
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(TISSUE_EINVAL, "dt must be finite and > 0");
    if (n_steps < 0) return fail(TISSUE_EINVAL, "n_steps must be >= 0");
    if (n_steps == 0) return TISSUE_OK;
    if ((uint64_t)t->steps_done + (uint64_t)n_steps > 0xFFFFFFFFull)
        return fail(TISSUE_EINVAL, "step index would exceed 2^32");
    const int rc = t->lp.run(dt, n_steps);
    if (rc == TISSUE_OK) t->steps_done += (uint32_t)n_steps;
    return rc;
}

int tissue_step_timed(tissue_t *t, double dt, int32_t n_steps, tissue_timing_t *out)
{
    if (!t) return fail(TISSUE_EINVAL, "null tissue");
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(TISSUE_EINVAL, "dt must be finite and > 0");
    if (n_steps < 0) return fail(TISSUE_EINVAL, "n_steps must be >= 0");
    if ((uint64_t)t->steps_done + (uint64_t)n_steps > 0xFFFFFFFFull)
        return fail(TISSUE_EINVAL, "step index would exceed 2^32");
    const int rc = t->lp.run_timed(dt, n_steps, out);
    if (rc == TISSUE_OK) t->steps_done += (uint32_t)n_steps;
    return rc;
}

static int check_flags(const unsigned char *ctl)
{
    uint32_t flags[2];
    std::memcpy(flags, ctl + 24, 8);
    if (flags[0]) return fail(TISSUE_EOVERFLOW, "a count left [0, 2^26)");
    if (flags[1]) return fail(TISSUE_ELIMIT, "a unit-step reached event_cap");
    return TISSUE_OK;
}

int tissue_read_counts(tissue_t *t, int32_t *host_out, size_t n_out)
{
    if (!t || !host_out) return fail(TISSUE_EINVAL, "null argument");
    const size_t n = (size_t)t->plan.nvox * t->plan.S;
    if (n_out != n) return fail(TISSUE_EINVAL, "n_out must equal n_voxels * n_species");
    unsigned char ctl[64];
    {
        std::unique_lock<std::mutex> lk;
        unsigned char *h = nullptr;
        HIP_TRY(staging_acquire(lk, n * 4 + 64, &h));
        HIP_TRY(hipMemcpyAsync(h, t->d_counts(), n * 4, hipMemcpyDeviceToHost, t->stream));
        HIP_TRY(hipMemcpyAsync(h + n * 4, t->d_ctl(), 64, hipMemcpyDeviceToHost, t->stream));
        HIP_TRY(hipStreamSynchronize(t->stream));
        std::memcpy(host_out, h, n * 4);
        std::memcpy(ctl, h + n * 4, 64);
    }
    return check_flags(ctl);
}

int tissue_read_stats(tissue_t *t, tissue_stats_t *out)
{
    if (!t || !out) return fail(TISSUE_EINVAL, "null argument");
    unsigned char ctl[64];
    {
        std::unique_lock<std::mutex> lk;
        unsigned char *h = nullptr;
        HIP_TRY(staging_acquire(lk, 64, &h));
        HIP_TRY(hipMemcpyAsync(h, t->d_ctl(), 64, hipMemcpyDeviceToHost, t->stream));
        HIP_TRY(hipStreamSynchronize(t->stream));
        std::memcpy(ctl, h, 64);
    }
    return tissue_stats_decode(t, ctl, out);
}

int tissue_stats_enqueue(tissue_t *t, void *dst)
{
    if (!t || !dst) return fail(TISSUE_EINVAL, "null argument");
    HIP_TRY(hipMemcpyAsync(dst, t->d_ctl(), TISSUE_STATS_BLOCK_BYTES, hipMemcpyDeviceToHost, t->stream));
    return TISSUE_OK;
}

int tissue_stats_decode(tissue_t *t, const void *block, tissue_stats_t *out)
{
    if (!t || !block || !out) return fail(TISSUE_EINVAL, "null argument");
    const unsigned char *ctl = static_cast<const unsigned char *>(block);
    uint64_t st[3];
    uint32_t fl[2];
    std::memcpy(st, ctl, 24);
    std::memcpy(fl, ctl + 24, 8);
    out->chi_events = st[0];
    out->s_events = st[1];
    out->draws = st[2];
    out->overflow = fl[0];
    out->capped = fl[1];
    out->steps_done = t->steps_done;
    out->n_cells = t->plan.ncell;
    out->n_edges = t->plan.nedge;
    out->n_voxels = t->plan.nvox;
    out->jit = t->plan.all_jit;
    return TISSUE_OK;
}

int tissue_read_trace(tissue_t *t, uint32_t first_step, uint32_t n_steps, uint32_t *chi_events,
                      uint64_t *chi_t_bits, uint32_t *s_events, uint64_t *s_t_bits)
{
    if (!t) return fail(TISSUE_EINVAL, "null tissue");
    const Plan &p = t->plan;
    if (!p.trace_steps) return fail(TISSUE_ESTATE, "tissue was created without TISSUE_FLAG_TRACE");
    const uint64_t end = (uint64_t)first_step + n_steps;
    if (end > t->steps_done || n_steps > p.trace_steps ||
        (uint64_t)first_step + p.trace_steps < t->steps_done)
        return fail(TISSUE_EINVAL, "requested steps are not all in the trace window");
    HIP_TRY(hipStreamSynchronize(t->stream));
    const DevTissue &R = t->host_rec;
    for (uint32_t k = 0; k < n_steps; ++k) {
        const size_t slot = (size_t)((first_step + k) % p.trace_steps);
        if (chi_events)
            HIP_TRY(hipMemcpy(chi_events + (size_t)k * p.ncell, R.tr_chi_ev + slot * p.ncell,
                              (size_t)p.ncell * 4, hipMemcpyDeviceToHost));
        if (chi_t_bits)
            HIP_TRY(hipMemcpy(chi_t_bits + (size_t)k * p.ncell, R.tr_chi_t + slot * p.ncell,
                              (size_t)p.ncell * 8, hipMemcpyDeviceToHost));
        if (p.nedge && s_events)
            HIP_TRY(hipMemcpy(s_events + (size_t)k * p.nedge, R.tr_s_ev + slot * p.nedge,
                              (size_t)p.nedge * 4, hipMemcpyDeviceToHost));
        if (p.nedge && s_t_bits)
            HIP_TRY(hipMemcpy(s_t_bits + (size_t)k * p.nedge, R.tr_s_t + slot * p.nedge,
                              (size_t)p.nedge * 8, hipMemcpyDeviceToHost));
    }
    return TISSUE_OK;
}

int tissue_restart(tissue_t *t, uint32_t sim_id, uint32_t start_step)
{
    if (!t) return fail(TISSUE_EINVAL, "null tissue");
    if (sim_id >= (1u << 30)) return fail(TISSUE_EINVAL, "sim_id must be < 2^30");
    const Plan &p = t->plan;
    // wait for earlier work so the host record can be reused as the source
    HIP_TRY(hipStreamSynchronize(t->stream));
    t->host_rec.sim_id = sim_id;
    t->host_rec.step_base = start_step;
    HIP_TRY(hipMemcpyAsync(t->d_counts(), t->dev + p.off_init, (size_t)p.nvox * p.S * 4,
                           hipMemcpyDeviceToDevice, t->stream));
    HIP_TRY(hipMemcpyAsync(t->d_rec(), &t->host_rec, sizeof(DevTissue), hipMemcpyHostToDevice, t->stream));
    HIP_TRY(hipMemsetAsync(t->d_ctl(), 0, 32, t->stream));
    HIP_TRY(hipStreamSynchronize(t->stream));
    t->steps_done = start_step;
    return TISSUE_OK;
}

int tissue_write_counts(tissue_t *t, const int32_t *host_in, size_t n_in)
{
    if (!t || !host_in) return fail(TISSUE_EINVAL, "null argument");
    const size_t n = (size_t)t->plan.nvox * t->plan.S;
    if (n_in != n) return fail(TISSUE_EINVAL, "n_in must equal n_voxels * n_species");
    for (size_t i = 0; i < n; ++i)
        if (host_in[i] < 0 || host_in[i] >= TISSUE_COUNT_LIMIT)
            return fail(TISSUE_EINVAL, "counts must be in [0, 2^26)");
    std::unique_lock<std::mutex> lk;
    unsigned char *h = nullptr;
    HIP_TRY(staging_acquire(lk, n * 4, &h));
    std::memcpy(h, host_in, n * 4);
    HIP_TRY(hipMemcpyAsync(t->d_counts(), h, n * 4, hipMemcpyHostToDevice, t->stream));
    HIP_TRY(hipStreamSynchronize(t->stream));
    return TISSUE_OK;
}

int tissue_set_launch(tissue_t *t, int32_t persistent, int32_t workgroups_per_cu)
{
    if (!t || workgroups_per_cu < 0 || workgroups_per_cu > 64) return fail(TISSUE_EINVAL, "bad launch shape");
    HIP_TRY(hipStreamSynchronize(t->stream));
    t->lp.persistent = persistent ? 1 : 0;
    t->lp.wpc = workgroups_per_cu;
    t->lp.clear_graphs();
    return TISSUE_OK;
}

int tissue_set_chi_mode(tissue_t *t, int32_t mode)
{
    if (!t || mode < kModeLane || mode > kModeRowWide) return fail(TISSUE_EINVAL, "chi mode must be 0..4");
    return t->lp.set_chi_mode(mode);
}

int tissue_set_regroup(tissue_t *t, int32_t mode)
{
    if (!t || mode < 0 || mode > 2) return fail(TISSUE_EINVAL, "regroup mode must be 0, 1 or 2");
    HIP_TRY(hipStreamSynchronize(t->stream));
    t->lp.regroup = mode;
    return t->lp.set_chi_mode(t->lp.chi_mode);
}

int tissue_set_refill(tissue_t *t, int32_t min_idle_lanes)
{
    if (!t || min_idle_lanes < 0 || min_idle_lanes > kWave) return fail(TISSUE_EINVAL, "refill must be 0..64");
    HIP_TRY(hipStreamSynchronize(t->stream));
    t->lp.refill_min = min_idle_lanes;
    t->lp.clear_graphs();
    return TISSUE_OK;
}

int tissue_set_whole_run(tissue_t *t, int32_t enable)
{
    if (!t || enable < 0 || enable > 1) return fail(TISSUE_EINVAL, "whole run must be 0 or 1");
    HIP_TRY(hipStreamSynchronize(t->stream));
    t->lp.whole_run = enable;
    return TISSUE_OK;
}

int tissue_runs_whole(tissue_t *t)
{
    if (!t) return fail(TISSUE_EINVAL, "null tissue");
    SmallRun r;
    const JitKernels *jk = nullptr;
    size_t lds = 0;
    return t->lp.whole_run && t->lp.small_run(r, jk, lds) ? 1 : 0;
}

int tissue_set_graph_chunk(tissue_t *t, int32_t steps_per_graph)
{
    if (!t || steps_per_graph < 0 || steps_per_graph > 100000) return fail(TISSUE_EINVAL, "bad graph chunk");
    HIP_TRY(hipStreamSynchronize(t->stream));
    t->lp.graph_chunk = steps_per_graph;
    t->lp.clear_graphs();
    return TISSUE_OK;
}

int tissue_destroy(tissue_t *t)
{
    if (!t) return TISSUE_OK;
    if (t->batches > 0)
        return fail(TISSUE_ESTATE, "tissue is a member of " + std::to_string(t->batches) +
                                       " live batch(es); destroy them first");
    (void)hipStreamSynchronize(t->stream);
    if (t->ready) (void)hipEventDestroy(t->ready);
    delete t;
    return TISSUE_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------

namespace {

struct BatchLayout {
    size_t off_tbl = 0, off_lq = 0, off_chi = 0, off_s = 0, off_retry = 0, bytes = 0;
    size_t chi_cap = 0;
    std::vector<std::vector<SItem>> s_passes;
    std::vector<int> s_fix;  // per pass: the face-group kind shared by every member in it, or 0
};

int plan_batch(tissue_t *const *ts, int32_t n, BatchLayout &B)
{
    if (!ts || n < 1) return fail(TISSUE_EINVAL, "batch needs >= 1 tissue");
    for (int32_t i = 0; i < n; ++i)
        if (!ts[i]) return fail(TISSUE_EINVAL, "null tissue in batch");
    {
        // a tissue twice in one launch would run its cells twice, racing on its counts
        std::vector<const tissue *> sorted(ts, ts + n);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(TISSUE_EINVAL, "a tissue appears twice in the batch");
    }
    for (int32_t i = 1; i < n; ++i)
        if (ts[i]->plan.strang != ts[0]->plan.strang)
            return fail(TISSUE_EINVAL, "batch members must share the splitting scheme");
    // chi items: room for the largest cut of every member's classes
    for (int32_t i = 0; i < n; ++i) B.chi_cap += ts[i]->plan.n_chi_items;
    // S: pass c holds every member's pass c (a member with disjoint face
    // groups has one pass)
    int max_pass = 0;
    for (int32_t i = 0; i < n; ++i) {
        const Plan &p = ts[i]->plan;
        if (!p.has_s || p.nedge == 0) continue;
        max_pass = std::max(max_pass, (int)p.pass_start.size() - 1);
    }
    B.s_passes.assign(max_pass, {});
    B.s_fix.assign(max_pass, -1);
    for (int32_t i = 0; i < n; ++i) {
        const Plan &p = ts[i]->plan;
        if (!p.has_s || p.nedge == 0) continue;
        for (size_t c = 0; c + 1 < p.pass_start.size(); ++c) {
            B.s_fix[c] = B.s_fix[c] < 0 || B.s_fix[c] == p.face_kind ? p.face_kind : 0;
            for (uint32_t o = p.pass_start[c]; o < p.pass_start[c + 1]; o += kWave)
                B.s_passes[c].push_back(SItem{(uint32_t)i, o, std::min<uint32_t>(kWave, p.pass_start[c + 1] - o), 0});
        }
    }
    for (int &f : B.s_fix) f = std::max(f, 0);
    size_t n_s = 0;
    for (auto &ps : B.s_passes) n_s += ps.size();
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1));
        return at;
    };
    B.off_tbl = take((size_t)n * sizeof(DevTissue *));
    B.off_lq = take(kLaunchQueueBytes);
    B.off_chi = take(B.chi_cap * sizeof(ChiItem));
    B.off_s = take(n_s * sizeof(SItem));
    size_t cells = 0;
    for (int32_t i = 0; i < n; ++i) cells += ts[i]->plan.ncell;
    B.off_retry = take(cells * sizeof(ChiItem));
    B.bytes = o;
    return TISSUE_OK;
}

}  // namespace

size_t tissue_batch_required_bytes(tissue_t *const *ts, int32_t n)
{
    BatchLayout B;
    if (plan_batch(ts, n, B) != TISSUE_OK) return 0;
    return B.bytes;
}

int tissue_batch_create(tissue_t *const *ts, int32_t n, void *dev_buf, size_t dev_bytes,
                        void *hip_stream, tissue_batch_t **out)
{
    if (!out) return fail(TISSUE_EINVAL, "null output handle");
    *out = nullptr;
    BatchLayout B;
    int rc = plan_batch(ts, n, B);
    if (rc != TISSUE_OK) return rc;
    if (!dev_buf || ((uintptr_t)dev_buf % kAlign) != 0)
        return fail(TISSUE_EINVAL, "dev_buf must be non-null and 256-byte aligned");
    if (dev_bytes < B.bytes) return fail(TISSUE_ENOMEM, "batch buffer too small");
    const int cus = device_cus();
    if (cus <= 0) return fail(TISSUE_EDEVICE, "no HIP device");
    std::unique_ptr<tissue_batch> b(new tissue_batch());
    b->members.assign(ts, ts + n);
    b->dev = static_cast<unsigned char *>(dev_buf);
    b->bytes = dev_bytes;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    for (int32_t i = 0; i < n; ++i) HIP_TRY(hipStreamSynchronize(ts[i]->stream));
    std::vector<DevTissue *> tbl(n);
    for (int32_t i = 0; i < n; ++i) tbl[i] = ts[i]->d_rec();
    std::vector<SItem> s_all;
    for (auto &ps : B.s_passes) s_all.insert(s_all.end(), ps.begin(), ps.end());
    {
        // the buffer's image up to the end of the S items, in one copy
        std::unique_lock<std::mutex> lk;
        unsigned char *h = nullptr;
        const size_t up = B.off_s + s_all.size() * sizeof(SItem);
        HIP_TRY(staging_acquire(lk, up, &h));
        std::memcpy(h + B.off_tbl, tbl.data(), tbl.size() * sizeof(DevTissue *));
        std::memset(h + B.off_lq, 0, B.off_chi - B.off_lq);
        if (!s_all.empty()) std::memcpy(h + B.off_s, s_all.data(), s_all.size() * sizeof(SItem));
        HIP_TRY(hipMemcpyAsync(b->dev, h, up, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    LaunchPlan &L = b->lp;
    L.tbl = reinterpret_cast<DevTissue **>(b->dev + B.off_tbl);
    L.n_tissues = (uint32_t)n;
    L.lq = reinterpret_cast<uint32_t *>(b->dev + B.off_lq);
    L.stream = st;
    L.cus = cus;
    L.strang = ts[0]->plan.strang;
    for (int32_t i = 0; i < n; ++i) L.members.push_back(&ts[i]->plan);
    L.rec0 = ts[0]->d_rec();
    L.retry_items = reinterpret_cast<ChiItem *>(b->dev + B.off_retry);
    L.chi_items = reinterpret_cast<ChiItem *>(b->dev + B.off_chi);
    L.chi_items_cap = B.chi_cap;
    size_t off = 0;
    for (auto &ps : B.s_passes) {
        L.s.push_back(SLaunch{reinterpret_cast<const SItem *>(b->dev + B.off_s) + off, (uint32_t)ps.size(),
                              B.s_fix[(size_t)(&ps - B.s_passes.data())]});
        off += ps.size();
    }
    rc = L.set_chi_mode(kModeAuto);
    if (rc != TISSUE_OK) return rc;
    for (tissue *t : b->members) t->batches++;
    *out = b.release();
    return TISSUE_OK;
}

int tissue_batch_set_members(tissue_batch_t *b, tissue_t *const *ts, int32_t n)
{
    if (!b) return fail(TISSUE_EINVAL, "null batch");
    if (n < 0 || (n > 0 && !ts)) return fail(TISSUE_EINVAL, "bad member list");
    BatchLayout B;
    if (n > 0) {
        const int rc = plan_batch(ts, n, B);
        if (rc != TISSUE_OK) return rc;
        if (B.bytes > b->bytes)
            return fail(TISSUE_EBUSY, "the batch's buffer holds " + std::to_string(b->bytes) +
                                          " bytes; these members need " + std::to_string(B.bytes));
    }
    LaunchPlan &L = b->lp;
    std::vector<const Plan *> plans;
    for (int32_t i = 0; i < n; ++i) plans.push_back(&ts[i]->plan);
    std::vector<ChiItem> items;
    std::vector<ChiLaunch> launches;
    if (n > 0) plan_chi(plans, L.chi_mode, L.regroup, L.cus * 4, items, launches);
    if (launches.size() > (size_t)kMaxChiLaunches) return fail(TISSUE_EINVAL, "too many chi launch groups");
    std::vector<SItem> s_all;
    for (auto &ps : B.s_passes) s_all.insert(s_all.end(), ps.begin(), ps.end());

    // the image up to the end of the S items (member table, cleared queue
    // words, chi and S items), copied on the batch's stream after the
    // previous image's copy has left the staging memory
    const size_t up = n > 0 ? B.off_s + s_all.size() * sizeof(SItem) : 0;
    if (!b->staged) HIP_TRY(hipEventCreateWithFlags(&b->staged, hipEventDisableTiming));
    HIP_TRY(hipEventSynchronize(b->staged));
    if (up > b->stage_cap) {
        // once, for the whole buffer: the image never outgrows it (pinned
        // allocation and release can wait for the whole device)
        if (b->stage) HIP_TRY(hipHostFree(b->stage));
        b->stage = nullptr;
        b->stage_cap = 0;
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&b->stage), b->bytes, hipHostMallocDefault));
        b->stage_cap = b->bytes;
    }
    hipStream_t st = L.stream;
    if (n > 0) {
        unsigned char *h = b->stage;
        for (int32_t i = 0; i < n; ++i) {
            DevTissue *rec = ts[i]->d_rec();
            std::memcpy(h + B.off_tbl + (size_t)i * sizeof(DevTissue *), &rec, sizeof(rec));
        }
        std::memset(h + B.off_lq, 0, B.off_chi - B.off_lq);
        if (!items.empty()) std::memcpy(h + B.off_chi, items.data(), items.size() * sizeof(ChiItem));
        if (!s_all.empty()) std::memcpy(h + B.off_s, s_all.data(), s_all.size() * sizeof(SItem));
        // members on other streams: the batch's stream waits for their work so far
        for (int32_t i = 0; i < n; ++i)
            if (ts[i]->stream != st) {
                if (!ts[i]->ready) HIP_TRY(hipEventCreateWithFlags(&ts[i]->ready, hipEventDisableTiming));
                HIP_TRY(hipEventRecord(ts[i]->ready, ts[i]->stream));
                HIP_TRY(hipStreamWaitEvent(st, ts[i]->ready, 0));
            }
        HIP_TRY(hipMemcpyAsync(b->dev, h, up, hipMemcpyHostToDevice, st));
        HIP_TRY(hipEventRecord(b->staged, st));
    }

    L.clear_graphs();
    L.tbl = reinterpret_cast<DevTissue **>(b->dev + B.off_tbl);
    L.n_tissues = (uint32_t)n;
    L.lq = reinterpret_cast<uint32_t *>(b->dev + B.off_lq);
    L.members = plans;
    L.rec0 = n > 0 ? ts[0]->d_rec() : nullptr;
    L.strang = n > 0 ? ts[0]->plan.strang : L.strang;
    L.retry_items = reinterpret_cast<ChiItem *>(b->dev + B.off_retry);
    L.chi_items = reinterpret_cast<ChiItem *>(b->dev + B.off_chi);
    L.chi_items_cap = B.chi_cap;
    for (ChiLaunch &c : launches) {
        c.items = L.chi_items + reinterpret_cast<uintptr_t>(c.items);
        if (c.n_segs) c.segs = L.chi_items + reinterpret_cast<uintptr_t>(c.segs);
    }
    L.chi = std::move(launches);
    L.s.clear();
    size_t off = 0;
    for (auto &ps : B.s_passes) {
        L.s.push_back(SLaunch{reinterpret_cast<const SItem *>(b->dev + B.off_s) + off, (uint32_t)ps.size(),
                              B.s_fix[(size_t)(&ps - B.s_passes.data())]});
        off += ps.size();
    }
    // members that leave: their own stream waits for the batch's work so far,
    // so that destroying them (which synchronises their stream) also waits
    // for the batch's steps that still read their state
    for (tissue *t : b->members) {
        if (std::find(ts, ts + n, t) != ts + n || t->stream == st) continue;
        if (!t->ready) HIP_TRY(hipEventCreateWithFlags(&t->ready, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(t->ready, st));
        HIP_TRY(hipStreamWaitEvent(t->stream, t->ready, 0));
    }
    for (tissue *t : b->members) t->batches--;
    b->members.assign(ts, ts + n);
    for (tissue *t : b->members) t->batches++;
    return TISSUE_OK;
}

static int batch_check(tissue_batch_t *b, double dt, int32_t n_steps)
{
    if (!b) return fail(TISSUE_EINVAL, "null batch");
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(TISSUE_EINVAL, "dt must be finite and > 0");
    if (n_steps < 0) return fail(TISSUE_EINVAL, "n_steps must be >= 0");
    for (tissue *t : b->members)
        if ((uint64_t)t->steps_done + (uint64_t)n_steps > 0xFFFFFFFFull)
            return fail(TISSUE_EINVAL, "step index would exceed 2^32");
    return TISSUE_OK;
}

int tissue_batch_step(tissue_batch_t *b, double dt, int32_t n_steps)
{
    int rc = batch_check(b, dt, n_steps);
    if (rc != TISSUE_OK || n_steps == 0 || b->members.empty()) return rc;
    rc = b->lp.run(dt, n_steps);
    if (rc == TISSUE_OK)
        for (tissue *t : b->members) t->steps_done += (uint32_t)n_steps;
    return rc;
}

int tissue_batch_step_timed(tissue_batch_t *b, double dt, int32_t n_steps, tissue_timing_t *out)
{
    int rc = batch_check(b, dt, n_steps);
    if (rc != TISSUE_OK) return rc;
    if (b->members.empty()) {
        if (out) *out = tissue_timing_t{};
        return TISSUE_OK;
    }
    rc = b->lp.run_timed(dt, n_steps, out);
    if (rc == TISSUE_OK)
        for (tissue *t : b->members) t->steps_done += (uint32_t)n_steps;
    return rc;
}

int tissue_batch_set_launch(tissue_batch_t *b, int32_t persistent, int32_t workgroups_per_cu)
{
    if (!b || workgroups_per_cu < 0 || workgroups_per_cu > 64) return fail(TISSUE_EINVAL, "bad launch shape");
    HIP_TRY(hipStreamSynchronize(b->lp.stream));
    b->lp.persistent = persistent ? 1 : 0;
    b->lp.wpc = workgroups_per_cu;
    b->lp.clear_graphs();
    return TISSUE_OK;
}

int tissue_batch_set_regroup(tissue_batch_t *b, int32_t mode)
{
    if (!b || mode < 0 || mode > 2) return fail(TISSUE_EINVAL, "regroup mode must be 0, 1 or 2");
    HIP_TRY(hipStreamSynchronize(b->lp.stream));
    b->lp.regroup = mode;
    return b->lp.set_chi_mode(b->lp.chi_mode);
}

int tissue_batch_set_refill(tissue_batch_t *b, int32_t min_idle_lanes)
{
    if (!b || min_idle_lanes < 0 || min_idle_lanes > kWave) return fail(TISSUE_EINVAL, "refill must be 0..64");
    HIP_TRY(hipStreamSynchronize(b->lp.stream));
    b->lp.refill_min = min_idle_lanes;
    b->lp.clear_graphs();
    return TISSUE_OK;
}

int tissue_batch_set_whole_run(tissue_batch_t *b, int32_t enable)
{
    if (!b || enable < 0 || enable > 1) return fail(TISSUE_EINVAL, "whole run must be 0 or 1");
    HIP_TRY(hipStreamSynchronize(b->lp.stream));
    b->lp.whole_run = enable;
    return TISSUE_OK;
}

int tissue_batch_runs_whole(tissue_batch_t *b)
{
    if (!b) return fail(TISSUE_EINVAL, "null batch");
    SmallRun r;
    const JitKernels *jk = nullptr;
    size_t lds = 0;
    return b->lp.whole_run && b->lp.small_run(r, jk, lds) ? 1 : 0;
}

int tissue_batch_set_graph_chunk(tissue_batch_t *b, int32_t steps_per_graph)
{
    if (!b || steps_per_graph < 0 || steps_per_graph > 100000) return fail(TISSUE_EINVAL, "bad graph chunk");
    HIP_TRY(hipStreamSynchronize(b->lp.stream));
    b->lp.graph_chunk = steps_per_graph;
    b->lp.clear_graphs();
    return TISSUE_OK;
}

int tissue_batch_set_chi_mode(tissue_batch_t *b, int32_t mode)
{
    if (!b || mode < kModeLane || mode > kModeRowWide) return fail(TISSUE_EINVAL, "chi mode must be 0..4");
    return b->lp.set_chi_mode(mode);
}

int tissue_batch_sync(tissue_batch_t *b)
{
    if (!b) return fail(TISSUE_EINVAL, "null batch");
    HIP_TRY(hipStreamSynchronize(b->lp.stream));
    return TISSUE_OK;
}

// ---------------------------------------------------------------------------
// batch steps without allocation: the batch's work lists, queue words and
// redo list in a file-scope device array instead of a caller's buffer
// ---------------------------------------------------------------------------

namespace {

// One per device, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[TISSUE_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;

int scratch_address(unsigned char **out)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TISSUE_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(TISSUE_EDEVICE, "no device address for the static workspace");
        addr[dev] = p;
    }
    *out = static_cast<unsigned char *>(addr[dev]);
    return TISSUE_OK;
}

}  // namespace

int tissue_batch_step_static(tissue_t *const *ts, int32_t n, double dt, int32_t n_steps,
                             void *hip_stream)
{
    BatchLayout B;
    int rc = plan_batch(ts, n, B);
    if (rc != TISSUE_OK) return rc;
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(TISSUE_EINVAL, "dt must be finite and > 0");
    if (n_steps < 0) return fail(TISSUE_EINVAL, "n_steps must be >= 0");
    for (int32_t i = 0; i < n; ++i)
        if ((uint64_t)ts[i]->steps_done + (uint64_t)n_steps > 0xFFFFFFFFull)
            return fail(TISSUE_EINVAL, "step index would exceed 2^32");
    if (n_steps == 0) return TISSUE_OK;
    const int cus = device_cus();
    if (cus <= 0) return fail(TISSUE_EDEVICE, "no HIP device");

    // the launch plan of the default batch: automatic layout and regroup,
    // persistent chi launches, steps launched eagerly (no graph)
    LaunchPlan L;
    for (int32_t i = 0; i < n; ++i) L.members.push_back(&ts[i]->plan);
    L.rec0 = n > 0 ? ts[0]->d_rec() : nullptr;
    std::vector<ChiItem> items;
    std::vector<ChiLaunch> launches;
    plan_chi(L.members, kModeAuto, L.regroup, cus * 4, items, launches);
    if (launches.size() > (size_t)kMaxChiLaunches) return fail(TISSUE_EINVAL, "too many chi launch groups");
    std::vector<SItem> s_all;
    for (auto &ps : B.s_passes) s_all.insert(s_all.end(), ps.begin(), ps.end());
    size_t cells = 0;
    for (int32_t i = 0; i < n; ++i) cells += ts[i]->plan.ncell;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t off_tbl = take((size_t)n * sizeof(DevTissue *));
    const size_t off_lq = take(kLaunchQueueBytes);
    const size_t off_chi = take(items.size() * sizeof(ChiItem));
    const size_t off_s = take(s_all.size() * sizeof(SItem));
    const size_t off_retry = take(cells * sizeof(ChiItem));
    if (o > (size_t)TISSUE_STATIC_WORKSPACE_BYTES)
        return fail(TISSUE_ENOMEM, "the batch needs " + std::to_string(o) +
                                       " bytes of workspace, more than the static workspace's " +
                                       std::to_string((size_t)TISSUE_STATIC_WORKSPACE_BYTES));
    unsigned char *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != TISSUE_OK) return rc;

    // the workspace image up to the end of the S items: member table, queue
    // words (zero: every launch finds its queues cleared), items; one copy,
    // waited for, so that the host image may go
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    std::vector<unsigned char> img(off_s + s_all.size() * sizeof(SItem), 0);
    for (int32_t i = 0; i < n; ++i) {
        DevTissue *rec = ts[i]->d_rec();
        std::memcpy(img.data() + off_tbl + (size_t)i * sizeof(DevTissue *), &rec, sizeof(rec));
    }
    if (!items.empty()) std::memcpy(img.data() + off_chi, items.data(), items.size() * sizeof(ChiItem));
    if (!s_all.empty()) std::memcpy(img.data() + off_s, s_all.data(), s_all.size() * sizeof(SItem));
    HIP_TRY(hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));

    L.tbl = reinterpret_cast<DevTissue **>(ws + off_tbl);
    L.n_tissues = (uint32_t)n;
    L.lq = reinterpret_cast<uint32_t *>(ws + off_lq);
    L.stream = st;
    L.cus = cus;
    L.strang = ts[0]->plan.strang;
    L.graph_chunk = 0;
    L.chi_items = reinterpret_cast<ChiItem *>(ws + off_chi);
    L.chi_items_cap = items.size();
    L.retry_items = reinterpret_cast<ChiItem *>(ws + off_retry);
    for (ChiLaunch &c : launches) {
        c.items = L.chi_items + reinterpret_cast<uintptr_t>(c.items);
        if (c.n_segs) c.segs = L.chi_items + reinterpret_cast<uintptr_t>(c.segs);
    }
    L.chi = std::move(launches);
    size_t soff = 0;
    for (auto &ps : B.s_passes) {
        L.s.push_back(SLaunch{reinterpret_cast<const SItem *>(ws + off_s) + soff, (uint32_t)ps.size(),
                              B.s_fix[(size_t)(&ps - B.s_passes.data())]});
        soff += ps.size();
    }
    rc = L.run(dt, n_steps);
    if (rc == TISSUE_OK)
        for (int32_t i = 0; i < n; ++i) ts[i]->steps_done += (uint32_t)n_steps;
    return rc;
}

int tissue_batch_destroy(tissue_batch_t *b)
{
    if (!b) return TISSUE_OK;
    (void)hipStreamSynchronize(b->lp.stream);
    for (tissue *t : b->members) t->batches--;
    delete b;
    return TISSUE_OK;
}

}  // extern "C"
