// kernels.h -- host-side launchers of the device kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tissue_impl {

// LDS bytes of one chi workgroup: per cell 2P FP64 tree nodes + P*S counts.
size_t chi_lds_bytes(int P, int S, int cells_per_item);
hipError_t set_chi_lds_limit(int P, size_t lds);
hipError_t launch_chi(int P, uint32_t grid, size_t lds, hipStream_t stream,
                      const DevTissue *const *tbl, const ChiItem *items, uint32_t n_items,
                      uint32_t *queue, int persistent, int cells_per_item, double dt,
                      uint32_t kstep);
hipError_t launch_s(uint32_t grid, hipStream_t stream, const DevTissue *const *tbl,
                    const SItem *items, uint32_t n_items, uint32_t *queue, int persistent,
                    double dt, uint32_t kstep);
hipError_t launch_advance(hipStream_t stream, DevTissue *const *tbl, uint32_t n_tissues,
                          uint32_t n);

}  // namespace tissue_impl
