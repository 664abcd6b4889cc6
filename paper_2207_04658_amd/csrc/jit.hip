// jit.hip -- host side of scheme specialization: compiles the fused substep
// and bootstrap P2G kernels (substep.hpp) with hipRTC, the scheme and the
// simulation parameters of a context written into the source as
// compile-time DevScheme / DevParams values (and the row stride of the
// packed words), so that field kinds, bit offsets, masks, codec constants,
// parameters and row addresses fold into the instruction stream (and need
// no scalar registers).  The arithmetic is the same source
// under the same device flags, so results equal the generic kernels'.
// Code objects are cached per process by (device, dimension, scheme,
// parameters, row stride).
#include "mpmq_internal.hpp"

#include <hip/hiprtc.h>

#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace mpmq {
namespace {

#include "jit_sources.inc"

struct Entry {
    hipModule_t mod = nullptr;
    JitKernels k{};
};

std::mutex g_mu;
std::map<std::string, Entry> g_cache;

std::string hexd(double v) {
    char b[64];
    std::snprintf(b, sizeof(b), "%a", v);
    return b;
}

// C++ initializer of a DevScheme with the Philox key zeroed (the kernels
// read the key from the run-time copy).
std::string initializer(const DevScheme &d) {
    std::string s = "{" + std::to_string(d.dim) + ", " + std::to_string(d.W) + ", 0u, 0u, " +
                    std::to_string(d.dither_groups) + "u, {";
    for (int i = 0; i < 4; ++i) s += std::to_string(d.order[i]) + (i < 3 ? ", " : "}, " + std::to_string(d.mat) + ", {0, 0}, {");
    for (int i = 0; i < 4; ++i) {
        const DevField &f = d.f[i];
        s += "{" + std::to_string(f.kind) + ", " + std::to_string(f.bits) + ", " + std::to_string(f.exp_bits) + ", " +
             std::to_string(f.dither) + ", " + std::to_string(f.rel) + ", " + std::to_string(f.off) + ", " +
             std::to_string(f.emin) + ", " + std::to_string(f.emax) + ", " + std::to_string(f.mask) + "u, " +
             std::to_string(f.exp_mask) + "u, " + std::to_string(f.mag_mask) + "u, " + std::to_string(f.f32dec) +
             "u, " + hexd(f.lo) + ", " +
             hexd(f.delta) + ", " + hexd(f.inv) + ", " + hexd(f.maxc) + "}" + (i < 3 ? ", " : "}}");
    }
    return s;
}

// C++ initializer of a DevParams (floats as exact hexadecimal literals).
std::string initializer(const DevParams &p) {
    auto hf = [](float v) { return hexd((double)v) + "f"; };
    return "{" + std::to_string(p.dim) + ", " + std::to_string(p.res) + ", " + std::to_string(p.bound) + ", " +
           std::to_string(p.nb) + ", " + hf(p.dt) + ", " + hf(p.inv_dx) + ", " + hf(p.dx) + ", " + hf(p.mu) + ", " +
           hf(p.la) + ", " + hf(p.p_mass) + ", " + hf(p.stress_over_m) + ", " + hf(p.pc) + ", {" + hf(p.g[0]) + ", " +
           hf(p.g[1]) + ", " + hf(p.g[2]) + "}, 0.0f, " + hexd(p.dt_d) + ", " + hexd(p.inv_dx_d) + "}";
}

bool compile(int dim, int mat, const std::string &init, const std::string &pinit, int64_t cap,
             std::vector<char> &code, std::string lowered[3], std::string *err) {
    const std::string d = std::to_string(dim), m = std::to_string(mat);
    const std::string names[3] = {"mpmq::k_substep<" + d + ", false, " + m + ">",
                                  "mpmq::k_substep<" + d + ", true, " + m + ">", "mpmq::k_p2g<" + d + ", " + m + ">"};
    const std::string src = "#define MPMQ_SCHEME_CONST " + init + "\n#define MPMQ_PARAMS_CONST " + pinit +
                            "\n#define MPMQ_CAP_CONST " + std::to_string(cap) + "ll\n#include \"substep.hpp\"\n";
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "mpmq_specialized.hip", kJitHeaderCount, kJitHeaders,
                            kJitHeaderNames) != HIPRTC_SUCCESS) {
        *err = "hiprtcCreateProgram failed";
        return false;
    }
    for (const auto &n : names) hiprtcAddNameExpression(prog, n.c_str());
    const hiprtcResult r = hiprtcCompileProgram(prog, kJitFlagCount, kJitFlags);
    if (r != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        *err = std::string("hipRTC: ") + hiprtcGetErrorString(r) + "\n" + log.substr(0, 4000);
        hiprtcDestroyProgram(&prog);
        return false;
    }
    for (int i = 0; i < 3; ++i) {
        const char *low = nullptr;
        if (hiprtcGetLoweredName(prog, names[i].c_str(), &low) != HIPRTC_SUCCESS || !low) {
            *err = "hipRTC: no lowered name for " + names[i];
            hiprtcDestroyProgram(&prog);
            return false;
        }
        lowered[i] = low;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code.resize(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return true;
}

}  // namespace

bool jit_kernels(int dim, const DevScheme &ds, const DevParams &dp, int64_t cap, JitKernels *out,
                 std::string *err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return false;
    }
    const std::string init = initializer(ds), pinit = initializer(dp);
    const std::string key =
        std::to_string(dev) + "/" + std::to_string(dim) + "/" + init + "/" + pinit + "/" + std::to_string(cap);
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        *out = it->second.k;
        return true;
    }
    std::vector<char> code;
    std::string lowered[3];
    if (!compile(dim, ds.mat, init, pinit, cap, code, lowered, err)) return false;
    Entry e;
    hipError_t h = hipModuleLoadData(&e.mod, code.data());
    for (int i = 0; h == hipSuccess && i < 3; ++i) {
        hipFunction_t f = nullptr;
        h = hipModuleGetFunction(&f, e.mod, lowered[i].c_str());
        if (i < 2) e.k.substep[i] = f;
        else e.k.p2g = f;
    }
    if (h != hipSuccess) {
        *err = std::string("loading the specialized kernels: ") + hipGetErrorString(h);
        return false;
    }
    g_cache[key] = e;
    *out = e.k;
    return true;
}

}  // namespace mpmq
