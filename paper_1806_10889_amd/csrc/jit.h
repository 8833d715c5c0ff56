// jit.h -- per-network compiled chi kernels (jit.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "internal.h"

namespace tissue_impl {

struct JitKernels {
    hipModule_t module = nullptr;
    hipFunction_t lane = nullptr;  // one lane per cell
    hipFunction_t row = nullptr;   // one 16-lane row per cell
    hipFunction_t row32 = nullptr; // one 32-lane row per cell (17..32 voxels)
    hipFunction_t row64 = nullptr; // one 64-lane row per cell (33..64 voxels)
    hipFunction_t lane16 = nullptr; // one lane per cell, compact LDS
    hipFunction_t lane16x2 = nullptr; // compact, 2 lanes per cell (17..32 voxels)
    hipFunction_t lane16x4 = nullptr; // compact, 4 lanes per cell (33..64 voxels)
    hipFunction_t lane16r = nullptr;  // compact, one lane per cell, lanes refilled (persistent)
    hipFunction_t run_small = nullptr;  // every step of a call of a small tissue, chi and S
};

// Cache key of a network's structure (not its rates).
std::string network_key(const DevModel &M);
// Source of the compiled-network policy and the two kernels.
std::string network_source(const DevModel &M);
// Compile the network's kernels without loading them (no device needed).
int jit_compile_check(const DevModel &M, std::string &err);
// Compile (or fetch from the process cache) the chi kernels of M's network.
// Returns 0 and the kernels, or -1 with a message.
int jit_kernels(const DevModel &M, const JitKernels **out, std::string &err);

}  // namespace tissue_impl
