// Device-free paths of the host runtime under AddressSanitizer and
// UndefinedBehaviorSanitizer: descriptor validation and the plan of a
// tissue (lattice edges ranked by (colour, i), rings, face groups, leaf
// classes, the device layout), the chi launch plans of every mode, regroup
// setting and device size, and batch layouts, on random descriptors and on
// descriptors broken one field at a time.  Built by the CPU test suite with
// the sanitizers on the host side only; it includes the runtime's source so
// that its internal functions can be called, and takes the kernels'
// launchers and the network compiler from the library.  Besides running
// clean it checks what a plan promises: every cell in exactly one work item
// of every launch plan, items within their launch's cells per item, regroup
// segments covering their class, required bytes equal to the layout, the
// lattice's edges and the records, cells and classes in their stated orders.
#include "../paper_1806_10889_amd/csrc/host.cpp"

#include <cstdio>
#include <random>

namespace {

struct Case {
    tissue_desc_t d{};
    std::vector<uint8_t> mw, mh, cm;
    std::vector<int32_t> reactants, stoich, init;
    std::vector<double> rates, diffusion;
    std::vector<tissue_model_t> models;
    std::vector<std::vector<int32_t>> m_reac, m_stoich;
    std::vector<std::vector<double>> m_rates, m_diff;
};

int fails = 0;

void check(bool ok, const char *what, int trial)
{
    if (!ok) {
        std::fprintf(stderr, "trial %d: %s\n", trial, what);
        ++fails;
    }
}

// a random network over S species: R reactions of order 0..2 whose net
// change never removes more than a reactant supplies
void random_network(std::mt19937_64 &g, int S, int R, std::vector<int32_t> &reac,
                    std::vector<int32_t> &st, std::vector<double> &rates, std::vector<double> &diff)
{
    std::uniform_int_distribution<int> sp(-1, S - 1), dl(-1, 2);
    std::uniform_real_distribution<double> u(0.0, 2.0);
    reac.assign(2 * R, -1);
    st.assign((size_t)R * S, 0);
    rates.assign(R, 0.0);
    for (int r = 0; r < R; ++r) {
        reac[2 * r] = sp(g);
        reac[2 * r + 1] = sp(g);
        int changed = 0;
        for (int s = 0; s < S && changed < 4; ++s) {
            int v = dl(g);
            const int supplied = (reac[2 * r] == s) + (reac[2 * r + 1] == s);
            if (v < -supplied) v = -supplied;
            st[(size_t)r * S + s] = v;
            changed += v != 0;
        }
        rates[r] = u(g);
    }
    diff.assign(S, 0.0);
    for (int s = 0; s < S; ++s) diff[s] = (g() & 1) ? u(g) : 0.0;
}

void random_case(std::mt19937_64 &g, Case &c)
{
    std::uniform_int_distribution<int> side(1, 40), mesh(1, 8), spn(1, 8), rn(0, 16), cnt(0, 60);
    tissue_desc_t &d = c.d;
    d = tissue_desc_t{};
    d.abi_version = TISSUE_ABI_VERSION;
    d.lattice = g() & 1;
    d.nx = (uint32_t)side(g);
    d.ny = (uint32_t)side(g);
    const uint32_t n = d.nx * d.ny;
    const bool uneven = g() & 1;
    d.mesh_w0 = (uint32_t)mesh(g);
    d.mesh_h0 = (uint32_t)mesh(g);
    c.mw.assign(n, 0);
    c.mh.assign(n, 0);
    for (uint32_t i = 0; i < n; ++i) {
        c.mw[i] = (uint8_t)(uneven ? mesh(g) : d.mesh_w0);
        c.mh[i] = (uint8_t)(uneven ? mesh(g) : d.mesh_h0);
    }
    d.mesh_w = uneven ? c.mw.data() : nullptr;
    d.mesh_h = uneven ? c.mh.data() : nullptr;
    const int S = std::max(3, spn(g));
    d.n_species = (uint32_t)S;
    const int R = rn(g);
    random_network(g, S, R, c.reactants, c.stoich, c.rates, c.diffusion);
    d.n_reactions = (uint32_t)R;
    d.reactants = c.reactants.data();
    d.stoich = c.stoich.data();
    d.rates = c.rates.data();
    d.diffusion = c.diffusion.data();
    const bool first = g() & 1;
    d.flags = (first ? TISSUE_FLAG_SIGNAL_FIRST_ORDER : 0u) | ((g() & 1) ? TISSUE_FLAG_STRANG : 0u) |
              ((g() & 3) == 0 ? TISSUE_FLAG_TRACE : 0u) | TISSUE_FLAG_NO_JIT;
    d.trace_steps = 3;
    d.trans_n = first ? -1 : 0;
    d.trans_d = 1;
    d.trans_i = 2;
    d.trans_rate = 0.5;
    if ((g() % 5) == 0) d.trans_n = -1, d.trans_d = -1;  // no S
    size_t nvox = 0;
    for (uint32_t i = 0; i < n; ++i) nvox += (size_t)c.mw[i] * c.mh[i];
    c.init.resize(nvox * S);
    for (auto &x : c.init) x = cnt(g);
    d.init_counts = c.init.data();
    d.seed = g();
    d.sim_id = (uint32_t)(g() % 1000);
    // per-cell networks on some tissues
    const int nm = (g() % 3 == 0) ? (int)(g() % 4) : 0;
    c.models.assign(nm, tissue_model_t{});
    c.m_reac.assign(nm, {});
    c.m_stoich.assign(nm, {});
    c.m_rates.assign(nm, {});
    c.m_diff.assign(nm, {});
    for (int m = 0; m < nm; ++m) {
        const int Rm = rn(g);
        random_network(g, S, Rm, c.m_reac[m], c.m_stoich[m], c.m_rates[m], c.m_diff[m]);
        c.models[m] = tissue_model_t{(uint32_t)Rm, c.m_reac[m].data(), c.m_stoich[m].data(),
                                     c.m_rates[m].data(), c.m_diff[m].data(), first ? 0.25 : 0.5};
    }
    c.cm.assign(n, 0);
    for (uint32_t i = 0; i < n; ++i) c.cm[i] = (uint8_t)(nm ? g() % (nm + 1) : 0);
    d.n_models = (uint32_t)nm;
    d.models = nm ? c.models.data() : nullptr;
    d.cell_model = nm ? c.cm.data() : nullptr;
}

// every cell of the plan in exactly one item of one launch; items within
// their launch's cells per item; regroup segments within a class
void check_launches(const Plan &p, const std::vector<ChiItem> &items,
                    const std::vector<ChiLaunch> &ls, int trial)
{
    std::vector<int> seen(p.ncell, 0);
    for (const ChiLaunch &L : ls) {
        const size_t off = reinterpret_cast<uintptr_t>(L.items);
        check(off + L.n_items <= items.size(), "launch items out of range", trial);
        if (off + L.n_items > items.size()) return;
        for (uint32_t k = 0; k < L.n_items; ++k) {
            const ChiItem &it = items[off + k];
            check(it.tissue == 0 && it.count >= 1 && it.count <= (uint32_t)L.cells_per_item,
                  "item size", trial);
            check(it.first + it.count <= p.ncell, "item range", trial);
            for (uint32_t q = 0; q < it.count && it.first + q < p.ncell; ++q) {
                const int32_t cell = p.cell_list[it.first + q];
                const int V = p.wh[2 * cell] * p.wh[2 * cell + 1];
                check(pow2_at_least(V) <= L.P && (L.P == pow2_at_least(V) || L.P == 16),
                      "cell of another leaf class", trial);
                check((int)p.cell_model[cell] == (int)it.model, "cell of another network", trial);
                seen[cell]++;
            }
        }
        if (L.n_segs) {
            const size_t so = reinterpret_cast<uintptr_t>(L.segs);
            check(so + L.n_segs <= items.size(), "segments out of range", trial);
            for (uint32_t k = 0; k < L.n_segs && so + k < items.size(); ++k)
                check(items[so + k].count <= kRegroupChunk, "segment too long", trial);
        }
    }
    for (uint32_t c = 0; c < p.ncell; ++c) check(seen[c] == 1, "cell not in exactly one item", trial);
    check(items.size() <= p.n_chi_items, "items over the plan's room", trial);
}

// The lattice's edges, listed by brute force over (cell, direction) and
// sorted by (colour class, first cell), against lattice_edges, which makes
// them in that order directly.
void check_edges(int lattice, int nx, int ny, int trial)
{
    const int nfwd = lattice == TISSUE_LATTICE_SQUARE ? 2 : 3;
    std::vector<Edge> want;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int d = 0; d < nfwd; ++d) {
                const int *off = lattice == TISSUE_LATTICE_SQUARE ? kSquareDir[d] : kHexDir[d];
                const int X = x + off[0], Y = y + off[1];
                if (X < 0 || X >= nx || Y < 0 || Y >= ny) continue;
                want.push_back(Edge{2 * d + ((d == 0 ? x : y) & 1), y * nx + x, Y * nx + X, d});
            }
    std::sort(want.begin(), want.end(), [](const Edge &a, const Edge &b) {
        return a.colour != b.colour ? a.colour < b.colour : a.i < b.i;
    });
    const std::vector<Edge> got = lattice_edges(lattice, nx, ny);
    bool same = got.size() == want.size();
    for (size_t k = 0; same && k < got.size(); ++k)
        same = got[k].colour == want[k].colour && got[k].i == want[k].i && got[k].j == want[k].j &&
               got[k].d == want[k].d;
    check(same, "lattice edges not the sorted brute-force list", trial);
}

// Records within a pass in (first cell, direction) order; cells of a leaf
// class in increasing order, classes by decreasing P, then network.
void check_orders(const Plan &p, int trial)
{
    if (p.has_s && p.nedge) {
        const std::vector<Edge> E = lattice_edges((int)p.lattice, (int)p.nx, (int)p.ny);
        for (size_t l = 0; l + 1 < p.pass_start.size(); ++l)
            for (uint32_t k = p.pass_start[l] + 1; k < p.pass_start[l + 1]; ++k) {
                const Edge &a = E[p.edges[k - 1].id], &b = E[p.edges[k].id];
                check(a.i < b.i || (a.i == b.i && a.d < b.d), "records out of (cell, direction) order", trial);
            }
    }
    for (size_t k = 0; k < p.chi.size(); ++k) {
        const ChiGroupHost &g = p.chi[k];
        for (uint32_t q = g.first + 1; q < g.first + g.count; ++q)
            check(p.cell_list[q - 1] < p.cell_list[q], "class cells out of order", trial);
        if (k)
            check(p.chi[k - 1].P > g.P || (p.chi[k - 1].P == g.P && p.chi[k - 1].model < g.model),
                  "classes out of order", trial);
    }
}

// The S passes keep every pair of edges that share a voxel in colour-class
// order (an earlier class's edge in an earlier pass), every edge is in one
// pass, and the records' ranks are a permutation of the edge ranks.
void check_passes(const Plan &p, int trial)
{
    if (!p.has_s || p.nedge == 0) return;
    const std::vector<Edge> E = lattice_edges((int)p.lattice, (int)p.nx, (int)p.ny);
    check(E.size() == p.nedge && p.pass_start.back() == p.nedge, "pass ranges", trial);
    std::vector<int> pass_of(p.nedge, -1), seen(p.nedge, 0);
    for (size_t l = 0; l + 1 < p.pass_start.size(); ++l)
        for (uint32_t k = p.pass_start[l]; k < p.pass_start[l + 1]; ++k) pass_of[k] = (int)l;
    // per voxel: (colour, pass) of the edges touching it
    std::vector<std::vector<std::pair<int, int>>> at(p.nvox);
    for (uint32_t k = 0; k < p.nedge; ++k) {
        const EdgeRec &r = p.edges[k];
        if (r.id >= p.nedge) {
            check(false, "edge rank out of range", trial);
            return;
        }
        seen[r.id]++;
        const int colour = E[r.id].colour;
        for (int q = 0; q < r.m_a; ++q) at[r.vox_i + r.A[q]].push_back({colour, pass_of[k]});
        for (int q = 0; q < r.m_b; ++q) at[r.vox_j + r.B[q]].push_back({colour, pass_of[k]});
    }
    for (uint32_t e = 0; e < p.nedge; ++e) check(seen[e] == 1, "edge ranks not a permutation", trial);
    for (const auto &v : at)
        for (size_t a = 0; a < v.size(); ++a)
            for (size_t b = 0; b < v.size(); ++b)
                if (v[a].first < v[b].first)
                    check(v[a].second < v[b].second, "shared voxel out of class order", trial);
                else if (a != b && v[a].first == v[b].first)
                    check(false, "two edges of one class share a voxel", trial);
}

}  // namespace

int main()
{
    std::mt19937_64 g(20261203);
    int planned = 0, rejected = 0, overlapping = 0;
    std::vector<std::unique_ptr<tissue>> keep;
    for (int trial = 0; trial < 300; ++trial) {
        Case c;
        random_case(g, c);
        std::unique_ptr<tissue> t(new tissue());
        const int rc = build_plan(&c.d, t->plan);
        if (rc != TISSUE_OK) {
            ++rejected;
            check(tissue_required_bytes(&c.d) == 0, "required bytes of a rejected descriptor", trial);
            continue;
        }
        ++planned;
        const Plan &p = t->plan;
        check(tissue_required_bytes(&c.d) == p.bytes, "required bytes", trial);
        check_passes(p, trial);
        check_orders(p, trial);
        check_edges(TISSUE_LATTICE_SQUARE, (int)p.nx, (int)p.ny, trial);
        check_edges(TISSUE_LATTICE_HEX, (int)p.nx, (int)p.ny, trial);
        if (!p.disjoint) ++overlapping;
        check(p.cell_list.size() == p.ncell, "cell list", trial);
        for (int mode = kModeLane; mode <= kModeRowWide; ++mode)
            for (int regroup = 0; regroup <= 2; ++regroup)
                for (int simd : {4, 1024}) {
                    std::vector<ChiItem> items;
                    std::vector<ChiLaunch> ls;
                    plan_chi({&p}, mode, regroup, simd, items, ls);
                    check_launches(p, items, ls, trial);
                }
        if (keep.size() < 12) keep.push_back(std::move(t));
    }
    // batches of the kept tissues: layout, passes, members repeated
    for (size_t n = 1; n <= keep.size(); ++n) {
        std::vector<tissue *> ts;
        for (size_t i = 0; i < n; ++i) ts.push_back(keep[i].get());
        bool same_scheme = true;
        for (tissue *t : ts) same_scheme &= t->plan.strang == ts[0]->plan.strang;
        BatchLayout B;
        const int rc = plan_batch(ts.data(), (int32_t)n, B);
        check(rc == (same_scheme ? TISSUE_OK : TISSUE_EINVAL), "batch scheme rule", (int)n);
        if (rc == TISSUE_OK) check(B.bytes > 0 && B.s_fix.size() == B.s_passes.size(), "batch layout", (int)n);
        ts.push_back(ts[0]);
        BatchLayout B2;
        check(plan_batch(ts.data(), (int32_t)ts.size(), B2) == TISSUE_EINVAL, "duplicate member", (int)n);
    }
    // one field broken at a time: every one rejected before any device work
    {
        Case c;
        for (;;) {
            random_case(g, c);
            Plan tmp;
            if (c.d.n_reactions > 0 && c.d.trans_n >= 0 && c.d.mesh_w && c.d.n_models > 0 &&
                build_plan(&c.d, tmp) == TISSUE_OK)
                break;
        }
        const tissue_desc_t good = c.d;
        int broken = 0;
        auto bad = [&](const char *what, const tissue_desc_t &d) {
            Plan tmp;
            check(build_plan(&d, tmp) == TISSUE_EINVAL, what, -1);
            check(tissue_required_bytes(&d) == 0, what, -1);
            ++broken;
        };
        tissue_desc_t d;
        d = good; d.abi_version = 0; bad("abi version", d);
        d = good; d.lattice = 2; bad("lattice", d);
        d = good; d.nx = 0; bad("empty lattice", d);
        d = good; d.n_species = 0; bad("no species", d);
        d = good; d.n_species = 9; bad("too many species", d);
        d = good; d.sim_id = 1u << 30; bad("sim_id", d);
        d = good; d.init_counts = nullptr; bad("null counts", d);
        d = good; d.mesh_h = nullptr; bad("one mesh array", d);
        d = good; d.flags |= 1u << 10; bad("unknown flag", d);
        d = good; d.flags |= TISSUE_FLAG_TRACE; d.trace_steps = 0; bad("trace without steps", d);
        d = good; d.n_models = 8; bad("too many models", d);
        d = good; d.n_reactions = 17; bad("too many reactions", d);
        d = good; d.cell_model = nullptr; d.models = nullptr; bad("models null", d);
        std::vector<double> r2 = c.rates;
        r2[0] = std::nan("");
        d = good; d.rates = r2.data(); bad("nan rate", d);
        std::vector<double> df = c.diffusion;
        df[0] = -1.0;
        d = good; d.diffusion = df.data(); bad("negative diffusion", d);
        std::vector<int32_t> ic = c.init;
        ic.back() = -1;
        d = good; d.init_counts = ic.data(); bad("negative count", d);
        ic.back() = 1 << 26;
        d = good; d.init_counts = ic.data(); bad("count at the limit", d);
        std::vector<uint8_t> mw = c.mw;
        mw[mw.size() / 2] = 9;
        d = good; d.mesh_w = mw.data(); bad("mesh side 9", d);
        d = good; d.trans_d = d.trans_n; bad("signalling species not distinct", d);
        std::vector<int32_t> re = c.reactants;
        re[0] = (int32_t)good.n_species;
        d = good; d.reactants = re.data(); bad("reactant out of range", d);
        std::vector<int32_t> sto = c.stoich;
        std::vector<int32_t> re2 = c.reactants;
        re2[0] = -1;
        re2[1] = -1;
        sto[0] = -1;  // reaction 0 has no reactant now and removes species 0
        d = good; d.reactants = re2.data(); d.stoich = sto.data(); bad("consumes what it lacks", d);
        std::vector<uint8_t> cm = c.cm;
        cm[0] = (uint8_t)(good.n_models + 1);
        d = good; d.cell_model = cm.data(); bad("cell model out of range", d);
        std::printf("broken descriptors rejected: %d\n", broken);
    }
    check(overlapping > 10, "few tissues with overlapping face groups", -1);
    std::printf("planned %d (%d with overlapping face groups), rejected %d, failures %d\n", planned,
                overlapping, rejected, fails);
    return fails ? 1 : 0;
}
