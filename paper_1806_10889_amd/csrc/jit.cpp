// jit.cpp -- per-network compilation of the chi kernels with hipRTC.
//
// The chi kernels are templates over a network policy (chi_kernels.h).  For
// each distinct reaction network (species count, reactants, stoichiometry,
// diffusing species) this file writes a policy whose structure is a set of
// compile-time constants, compiles the chi kernels (and the whole-run
// kernel of small tissues, which runs S as well) for gfx950 with the
// same floating-point rules as the ahead-of-time library (no contraction,
// no fast-math, no packed FP32), and caches the module for the process.
// Rate constants stay runtime values read per tissue, so one compiled network
// serves every tissue (and every rate set) with that structure.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "jit.h"

namespace tissue_impl {
namespace {

#include "jit_sources.inc"  // kSrcDeviceMath, kSrcInternal, kSrcChiKernels, kSrcSDevice

std::mutex g_mu;
std::map<std::string, std::unique_ptr<JitKernels>> g_cache;

std::string array_init(const std::vector<int> &v)
{
    std::ostringstream o;
    o << "{";
    for (size_t i = 0; i < v.size(); ++i) o << (i ? ", " : "") << v[i];
    if (v.empty()) o << "0";
    o << "}";
    return o.str();
}

}  // namespace

std::string network_key(const DevModel &M)
{
    std::ostringstream o;
    o << "S" << M.n_species << "R" << M.n_reactions << "D" << M.n_diff << ":";
    for (int r = 0; r < M.n_reactions; ++r) {
        o << (int)M.reac_a[r] << "," << (int)M.reac_b[r] << ",";
        o << M.delta_lo[r] << "," << M.delta_hi[r] << ";";
    }
    for (int q = 0; q < M.n_diff; ++q) o << (int)M.diff_species[q] << ";";
    return o.str();
}

std::string network_source(const DevModel &M)
{
    const int S = M.n_species, R = M.n_reactions, ND = M.n_diff;
    std::vector<int> ra(R), rb(R), dsp(ND), delta;
    for (int r = 0; r < R; ++r) {
        ra[r] = M.reac_a[r];
        rb[r] = M.reac_b[r];
        for (int s = 0; s < S; ++s) {
            const uint32_t w = s < 4 ? M.delta_lo[r] : M.delta_hi[r];
            delta.push_back((int)(int8_t)((w >> (8 * (s & 3))) & 0xFFu));
        }
    }
    for (int q = 0; q < ND; ++q) dsp[q] = M.diff_species[q];
    std::ostringstream o;
    o << "#include \"s_device.h\"\n"
      << "namespace tissue_impl {\n"
      << "struct NetCompiled {\n"
      << "    static constexpr int SM = " << S << ", RM = " << R << ", NDM = " << ND << ";\n"
      << "    static constexpr bool kFixedSpecies = true;\n"
      << "    static constexpr int kRa[" << std::max(R, 1) << "] = " << array_init(ra) << ";\n"
      << "    static constexpr int kRb[" << std::max(R, 1) << "] = " << array_init(rb) << ";\n"
      << "    static constexpr int kDsp[" << std::max(ND, 1) << "] = " << array_init(dsp) << ";\n"
      << "    static constexpr int kDelta[" << std::max(R * S, 1) << "] = " << array_init(delta) << ";\n"
      << "    double rate[" << std::max(R, 1) << "];\n"
      << "    double drate[" << std::max(ND, 1) << "];\n"
      << "    __device__ __forceinline__ int ra(int r) const { return kRa[r]; }\n"
      << "    __device__ __forceinline__ int rb(int r) const { return kRb[r]; }\n"
      << "    __device__ __forceinline__ int dsp(int q) const { return kDsp[q]; }\n"
      << "    __device__ __forceinline__ int delta(int r, int s) const { return kDelta[r * SM + s]; }\n"
      << "    __device__ __forceinline__ void load(const DevModel &M)\n"
      << "    {\n"
      // rates as vector registers: scalar registers are the scarcer resource
      // in these kernels (lane masks), vector registers do not limit occupancy
      << "#pragma unroll\n"
      << "        for (int r = 0; r < RM; ++r) rate[r] = M.rates[r];\n"
      << "#pragma unroll\n"
      << "        for (int q = 0; q < NDM; ++q) drate[q] = M.diff_rate[q];\n"
      << "    }\n"
      << "};\n"
      << "}  // namespace tissue_impl\n"
      << "using tissue_impl::ChiItem;\nusing tissue_impl::DevTissue;\n"
      << "extern \"C\" __global__ __launch_bounds__(64) void tissue_chi_lane(\n"
      << "    const DevTissue *const *tbl, const ChiItem *items, uint32_t n_items, uint32_t *queue,\n"
      << "    int persistent, int cells_per_item, int log2p, double dt, uint32_t kstep,\n"
      << "    uint32_t tag, uint32_t *n_items_dev, int prio)\n"
      << "{\n"
      << "    extern __shared__ __align__(16) unsigned char lds[];\n"
      << "    tissue_impl::chi_lane_body<tissue_impl::NetCompiled>(lds, tbl, items, n_items, queue,\n"
      << "        persistent, cells_per_item, log2p, dt, kstep, tag, n_items_dev, prio, blockIdx.x);\n"
      << "}\n"
      ;
    for (int gl : {1, 2, 4}) {
        o << "extern \"C\" __global__ __launch_bounds__(64) void tissue_chi_lane16"
          << (gl == 1 ? std::string() : "x" + std::to_string(gl)) << "(\n"
          << "    const DevTissue *const *tbl, const ChiItem *items, uint32_t n_items, uint32_t *queue,\n"
          << "    int persistent, int cells_per_item, double dt, uint32_t kstep, uint32_t tag,\n"
          << "    ChiItem *retry_items, uint32_t *retry_count, int prio)\n"
          << "{\n"
          << "    extern __shared__ __align__(16) unsigned char lds[];\n"
          << "    tissue_impl::chi_lane16_body<tissue_impl::NetCompiled, " << gl
          << ">(lds, tbl, items, n_items,\n"
          << "        queue, persistent, cells_per_item, dt, kstep, tag, retry_items, retry_count, prio);\n"
          << "}\n";
    }
    o << "extern \"C\" __global__ __launch_bounds__(64) void tissue_chi_lane16r(\n"
      << "    const DevTissue *const *tbl, const ChiItem *items, uint32_t n_items, uint32_t *queue,\n"
      << "    int persistent, double dt, uint32_t kstep, uint32_t tag, ChiItem *retry_items,\n"
      << "    uint32_t *retry_count, int refill_min)\n"
      << "{\n"
      << "    extern __shared__ __align__(16) unsigned char lds[];\n"
      << "    tissue_impl::chi_refill_body<tissue_impl::NetCompiled>(lds, tbl, items, n_items, queue,\n"
      << "        persistent, dt, kstep, tag, retry_items, retry_count, refill_min);\n"
      << "}\n";
    o << "extern \"C\" __global__ __launch_bounds__(64) void tissue_run_small(\n"
      << "    DevTissue *T, tissue_impl::SmallRun run, double dt, uint32_t n_steps)\n"
      << "{\n"
      << "    extern __shared__ __align__(16) unsigned char lds[];\n"
      << "    __shared__ tissue_impl::SShared sh;\n"
      << "    tissue_impl::run_small<tissue_impl::NetCompiled>(lds, sh, T, run, dt, n_steps);\n"
      << "}\n";
    for (int rw : {16, 32, 64}) {
        o << "extern \"C\" __global__ __launch_bounds__(64) void tissue_chi_row"
          << (rw == 16 ? std::string() : std::to_string(rw)) << "(\n"
          << "    const DevTissue *const *tbl, const ChiItem *items, uint32_t n_items, uint32_t *queue,\n"
          << "    int persistent, double dt, uint32_t kstep, uint32_t tag, int prio)\n"
          << "{\n"
          << "    __shared__ tissue_impl::RowShared sh;\n"
          << "    tissue_impl::chi_row_body<tissue_impl::NetCompiled, " << rw
          << ">(sh, tbl, items, n_items, queue,\n"
          << "        persistent, dt, kstep, tag, prio);\n"
          << "}\n";
    }
    return o.str();
}

namespace {

// Compile the network's kernels to a gfx950 code object.
int compile_network(const DevModel &M, std::vector<char> &code, std::string &err)
{
    const std::string src = network_source(M);
    const char *hdr_src[] = {kSrcDeviceMath, kSrcInternal, kSrcChiKernels, kSrcSDevice};
    const char *hdr_name[] = {"device_math.h", "internal.h", "chi_kernels.h", "s_device.h"};
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "tissue_network.hip", 4, hdr_src, hdr_name) !=
        HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return -1;
    }
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                          "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        err = "network compile failed: " + log.substr(0, 2000);
        hiprtcDestroyProgram(&prog);
        return -1;
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    code.resize(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return 0;
}

}  // namespace

int jit_compile_check(const DevModel &M, std::string &err)
{
    std::vector<char> code;
    return compile_network(M, code, err);
}

int jit_kernels(const DevModel &M, const JitKernels **out, std::string &err)
{
    *out = nullptr;
    const std::string key = network_key(M);
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        *out = it->second.get();
        return 0;
    }
    std::vector<char> code;
    if (compile_network(M, code, err) != 0) return -1;
    std::unique_ptr<JitKernels> k(new JitKernels());
    hipError_t e = hipModuleLoadData(&k->module, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&k->lane, k->module, "tissue_chi_lane");
    if (e == hipSuccess) e = hipModuleGetFunction(&k->row, k->module, "tissue_chi_row");
    if (e == hipSuccess) e = hipModuleGetFunction(&k->row32, k->module, "tissue_chi_row32");
    if (e == hipSuccess) e = hipModuleGetFunction(&k->row64, k->module, "tissue_chi_row64");
    if (e == hipSuccess) e = hipModuleGetFunction(&k->lane16, k->module, "tissue_chi_lane16");
    if (e == hipSuccess) e = hipModuleGetFunction(&k->lane16x2, k->module, "tissue_chi_lane16x2");
    if (e == hipSuccess) e = hipModuleGetFunction(&k->lane16x4, k->module, "tissue_chi_lane16x4");
    if (e == hipSuccess) e = hipModuleGetFunction(&k->lane16r, k->module, "tissue_chi_lane16r");
    if (e == hipSuccess) e = hipModuleGetFunction(&k->run_small, k->module, "tissue_run_small");
    if (e != hipSuccess) {
        err = std::string("loading the compiled network: ") + hipGetErrorString(e);
        return -1;
    }
    *out = k.get();
    g_cache.emplace(key, std::move(k));
    return 0;
}

}  // namespace tissue_impl
