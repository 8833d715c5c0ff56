// kernels.h -- host-side launchers of the device kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tissue_impl {

// Dynamic LDS bytes of one chi workgroup (lane mode: per cell 2P FP64 tree
// nodes and P*S int32 counts; compact (lane16) mode: per lane 16 FP64 leaves
// and 16*S uint16 counts, P / 16 lanes for cells of P > 16 leaves; row mode:
// none).
size_t chi_lds_bytes(int mode, int P, int S, int cells_per_item);

// Lanes per cell of the compact layout for cells of P leaves (P <= 64).
inline int compact_lanes(int P) { return P > 16 ? P / 16 : 1; }

// Arguments of one chi launch.
struct ChiArgs {
    int mode, P;
    int rw;                  // row mode: lanes per cell (16, 32 or 64)
    uint32_t grid;
    size_t lds;
    hipStream_t stream;
    const DevTissue *const *tbl;
    const ChiItem *items;
    uint32_t n_items;
    uint32_t *queue;
    int persistent, cells_per_item;
    double dt;
    uint32_t kstep;
    uint32_t tag;            // counter tag of the chi draws: 0, or 2 for a second half-step
    uint32_t *n_items_dev;   // lane mode: item count in device memory, or null
    ChiItem *retry_items;    // lane16: cells to redo at full width
    uint32_t *retry_count;
    int prio;                // nonzero: the launch's wavefronts issue at a raised priority
};
// Table sizes (species slots, reaction slots, diffusion slots) the kernels
// are instantiated for, for a network of S species, R reactions and ND
// diffusing species.
void chi_variant(int S, int R, int ND, int &SM, int &RM, int &NDM);
hipError_t launch_chi(int SM, int RM, int NDM, const ChiArgs &a);
// The generic chi kernels of one row of table sizes (chi_generic.hip, one
// translation unit per row): species slots x diffusion slots 4x0, 4x4, 8x0,
// 8x4, 8x8, for reaction slots RM = 4, 8, 12 or 16.
hipError_t launch_chi_part0(int RM, const ChiArgs &a);
hipError_t launch_chi_part1(int RM, const ChiArgs &a);
hipError_t launch_chi_part2(int RM, const ChiArgs &a);
hipError_t launch_chi_part3(int RM, const ChiArgs &a);
hipError_t launch_chi_part4(int RM, const ChiArgs &a);
// One workgroup per item of up to 64 edges.  fix = 2 or 1: every edge of
// the launch has face groups of 2 and 2 (1 and 1) voxels, the kernel
// specialised for them; 0: any face groups.
hipError_t launch_s(hipStream_t stream, const DevTissue *const *tbl, const SItem *items,
                    uint32_t n_items, double dt, uint32_t kstep, int fix);
hipError_t launch_advance(hipStream_t stream, DevTissue *const *tbl, uint32_t n_tissues,
                          uint32_t n);
// Cells per regroup segment: a class's cells of one tissue are regrouped in
// pieces of at most this many (a multiple of every work-item size, so pieces
// hold whole items), one workgroup each.
constexpr uint32_t kRegroupChunk = 16384;

// Reorder each segment's cells (consecutive cells of a class of one tissue:
// cell_list [first, first + count) of tissue `tissue`, count <=
// kRegroupChunk) by their load, largest first.
hipError_t launch_regroup(hipStream_t stream, const DevTissue *const *tbl, const ChiItem *segs,
                          uint32_t n_segs);

}  // namespace tissue_impl
