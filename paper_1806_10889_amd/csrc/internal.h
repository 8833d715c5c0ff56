// internal.h -- device data layout shared by the host runtime and the kernels.
//
// Everything a kernel needs about one tissue is in a DevTissue record that
// lives in the tissue's own device buffer; launches see tissues through a
// table of DevTissue pointers, so one launch can cover one tissue (plain) or
// many (batch, serving).  Work is cut into items of up to 64 cells (chi) or
// 64 edges (S) of one tissue; one 64-lane wavefront runs one item, one lane
// per cell or edge.
#pragma once

#ifndef __HIPCC_RTC__
#include <stdint.h>
#endif

namespace tissue_impl {

constexpr int kMaxSpecies = 8;
constexpr int kMaxReactions = 16;
constexpr int kMaxFace = 8;       // voxels in one face group (8x8 square mesh: 7)
constexpr int kWave = 64;
constexpr int32_t kCountLimit = 1 << 26;

// Mass-action network of one tissue, zero-padded to the table sizes: a
// padding reaction has no reactants and rate 0, a padding diffusion channel
// rate 0, so it adds exactly 0.0 to every fold and is never selected.  A
// reaction's net change is packed in delta_lo/delta_hi: one signed byte per
// species (species 0..3 in delta_lo, 4..7 in delta_hi).
struct DevModel {
    int32_t n_species;
    int32_t n_reactions;
    int32_t n_diff;                      // species with D > 0
    int32_t trans_n, trans_d, trans_i;   // S species (-1: unused); no S when trans_d < 0
    int32_t signal_order;                // 2: N_i + D_j -> I_i; 1: D_i -> I_j (facing voxel)
    int8_t reac_a[kMaxReactions];        // first reactant or -1
    int8_t reac_b[kMaxReactions];        // second reactant or -1
    int8_t diff_species[kMaxSpecies];    // species of diffusion channel q
    uint32_t delta_lo[kMaxReactions];
    uint32_t delta_hi[kMaxReactions];
    double rates[kMaxReactions];
    double diff_rate[kMaxSpecies];       // D of diffusion channel q
    double trans_rate;                   // S rate; first order: of this network's cells' molecules
};

// One lattice edge (i < j) and the facing membrane groups A of cell i and
// B of cell j; the voxel offsets locate the two cells in the counts array.
// Records are stored in the order the S operator processes them, which need
// not be the edges' rank: `id` is the edge's rank in (colour, i) order, the
// edge's index in every random counter and trace.
struct EdgeRec {
    int32_t vox_i;         // first voxel of cell i (global voxel index)
    int32_t vox_j;
    uint8_t m_a, m_b;
    uint8_t model_i, model_j;  // the two cells' networks (first-order signalling rates)
    uint8_t A[kMaxFace];
    uint8_t B[kMaxFace];
    uint32_t id;
};
static_assert(sizeof(EdgeRec) == 32, "EdgeRec layout");

struct DevTissue {
    int32_t *counts;              // [n_voxels][n_species], cell order, v = y*w + x
    const int32_t *vox_off;       // [n_cells] first voxel of each cell
    const uint8_t *wh;            // [n_cells][2] mesh (w, h)
    int32_t *cell_list;           // [n_cells] cells grouped by leaf-count class (each
                                  // class's order may be regrouped between steps)
    const EdgeRec *edges;         // [n_edges] in the order S processes them
    unsigned long long *stats;    // [3] chi events, S events, draws
    uint32_t *flags;              // [2] overflow, capped
    uint32_t *tr_chi_ev;          // trace ring [trace_steps][n_cells] or null
    unsigned long long *tr_chi_t;
    uint32_t *tr_s_ev;            // [trace_steps][n_edges] or null
    unsigned long long *tr_s_t;
    const DevModel *models;       // [n_models] chi networks of the cells; [0] equals `model`
    float *load;                  // [n_cells] total propensity after the last compact chi pass
    uint64_t seed;
    uint32_t n_cells, n_edges;
    uint32_t sim_id;
    uint32_t step_base;           // global index of step k = 0 of the next launch group
    uint32_t event_cap;
    uint32_t trace_steps;
    DevModel model;               // the tissue's own network and the S reaction
};

// up to 64 cells of one tissue, all with the same leaf count P and the same
// network models[model]: cells cell_list[first .. first + count)
struct ChiItem {
    uint32_t tissue;
    uint32_t first;
    uint32_t count;
    uint32_t model;
};

// chi kernel variants: one lane per cell (any P); one row of 16, 32 or 64
// lanes per cell; the compact 16-leaf / uint16 LDS layout with 1, 2 or 4
// lanes per cell (P <= 64) and a full-width redo of cells whose counts
// outgrow 16 bits
enum ChiMode { kChiLane = 0, kChiRow = 1, kChiLane16 = 2 };

// XCDs of the device: workgroups are dealt to them in turn (workgroup b to
// XCD b mod 8), each with its own L2
constexpr uint32_t kXcds = 8;

// device control words of one chi launch (uint32 each): the persistent
// queue of the main launch (next item, workgroups that left), the redo
// count of a compact launch, and the queue of its redo launch (laid out as
// the main queue)
enum {
    kQNext = 0,
    kQDone = 1,  // relative to a queue's first word
    kQRetry = 2,
    kQRetryNext = 4,
    kQueueBlockWords = 8
};

// up to 64 consecutive edges [first, first + count) of one tissue
struct SItem {
    uint32_t tissue;
    uint32_t first;
    uint32_t count;
    uint32_t pad;
};

// The whole run of a small tissue in one launch (one workgroup): its one
// chi work item (one lane per cell, at most 64 cells of one leaf class),
// then its S passes, for every step of the call, with the tissue's state
// copied into LDS for the run.  The bounds keep the one wavefront's
// sequence of items no longer than the step-by-step launches' critical
// path, and the copies within its LDS.
constexpr int kSmallPasses = 8;   // S passes (conflict levels)
constexpr int kSmallItems = 2;    // items per S pass
constexpr uint32_t kSmallLds = 48 * 1024;  // dynamic LDS of the whole-run kernel

// (copied into LDS a 4-byte word at a time)
static_assert(sizeof(DevTissue) % 8 == 0 && sizeof(DevModel) % 4 == 0, "record sizes");
static_assert(sizeof(ChiItem) % 4 == 0 && sizeof(SItem) % 4 == 0, "item sizes");

struct SmallRun {
    // LDS byte offsets of the copies: the tissue's record, counts, cell
    // tables, edge records and networks, its table of one record pointer,
    // and the work items
    uint32_t rec, counts, vox_off, wh, cell_list, edges, models, tbl;
    uint32_t n_counts;  // int32 counts (voxels x species)
    uint32_t n_models;
    const ChiItem *chi_item;
    uint32_t chi_item_lds;
    int32_t chi_cells_per_item;
    int32_t chi_log2p;
    const SItem *s_items[kSmallPasses];
    uint32_t s_n[kSmallPasses];
    uint32_t s_items_lds[kSmallPasses];
    int32_t n_s;
    int32_t strang;
};

}  // namespace tissue_impl
