// specialize.cpp -- network-specialised propagation kernels.
//
// A network is known only at run time, but it is fixed for every launch that
// uses it.  Compiling the propagation body with the reaction kinds, reactant
// species and packed net changes as compile-time constants removes the
// per-reaction dispatch of the generic kernels (a uniform branch and a
// register select per reactant per event); the arithmetic and its order are
// unchanged, so results are identical bit for bit.  Kernels are compiled with
// hipRTC for gfx950 with the library's floating-point flags, cached on disk
// by a hash of their source and options, and loaded per device.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <sys/stat.h>
#include <unistd.h>

#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "host.hpp"

namespace lik {

namespace {

const char *const kRtcOptions[] = {
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
    "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
};
constexpr int kRtcNumOptions = sizeof(kRtcOptions) / sizeof(kRtcOptions[0]);

uint64_t fnv1a(const std::string &s, uint64_t h = 1469598103934665603ull) {
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string cache_dir() {
    const char *d = getenv("LIK_KERNEL_CACHE");
    if (d && *d) return d;
    const char *home = getenv("HOME");
    return std::string(home && *home ? home : "/tmp") + "/.cache/lik-kernels";
}

bool read_file(const std::string &path, std::vector<char> *out) {
    FILE *f = fopen(path.c_str(), "rb");
    if (!f) return false;
    fseek(f, 0, SEEK_END);
    long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    if (n <= 0) {
        fclose(f);
        return false;
    }
    out->resize((size_t)n);
    bool ok = fread(out->data(), 1, (size_t)n, f) == (size_t)n;
    fclose(f);
    return ok;
}

void write_file_atomic(const std::string &dir, const std::string &path,
                       const std::vector<char> &data) {
    std::string cur;
    for (size_t i = 0; i <= dir.size(); ++i) {  // mkdir -p
        if (i == dir.size() || dir[i] == '/') {
            if (!cur.empty()) mkdir(cur.c_str(), 0755);
        }
        if (i < dir.size()) cur += dir[i];
    }
    std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return;
    bool ok = fwrite(data.data(), 1, data.size(), f) == data.size();
    ok = (fclose(f) == 0) && ok;
    if (ok) rename(tmp.c_str(), path.c_str());
    else unlink(tmp.c_str());
}

bool compile(const std::string &src, std::vector<char> *code, std::string *err) {
    const char *const *hdr = nullptr;
    const char *const *names = nullptr;
    int nh = rtc_headers(&hdr, &names);
    hiprtcProgram prog;
    hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "lik_spec.hip", nh, hdr, names);
    if (r != HIPRTC_SUCCESS) {
        *err = std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
        return false;
    }
    r = hiprtcCompileProgram(prog, kRtcNumOptions, kRtcOptions);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        *err = std::string("hiprtcCompileProgram: ") + hiprtcGetErrorString(r) + "\n" + log;
        hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    code->resize(n);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    return n > 0;
}

}  // namespace

namespace {

// A network's tables as compile-time constants: struct `name` in namespace lik.
void emit_spec_net(std::ostringstream &o, const lik_network &net, const char *name) {
    const int U = net.U, R = net.R, W = (U + 7) / 8;
    o << "struct " << name << " {\n  static constexpr int U = " << U << ", R = " << R << ";\n";
    auto arr = [&](const char *field, const int32_t *v) {
        o << "  static constexpr int " << field << "[" << R << "] = {";
        for (int r = 0; r < R; ++r) o << (r ? "," : "") << v[r];
        o << "};\n";
    };
    arr("kind", net.kind);
    arr("s1", net.s1);
    arr("s2", net.s2);
    o << "  static constexpr unsigned nu[" << R << "][" << W << "] = {";
    for (int r = 0; r < R; ++r) {
        o << (r ? "," : "") << "{";
        for (int w = 0; w < W; ++w) o << (w ? "," : "") << net.nu[r][w] << "u";
        o << "}";
    }
    o << "};\n};\n";
}

void emit_prelude(std::ostringstream &o) {
    o << "typedef __hip_internal::uint32_t uint32_t;\n"
         "typedef __hip_internal::uint64_t uint64_t;\n"
         "typedef __hip_internal::int32_t int32_t;\n"
         "typedef __hip_internal::int64_t int64_t;\n"
         "typedef __hip_internal::uint8_t uint8_t;\n"
         "typedef __hip_internal::uint16_t uint16_t;\n"
         "#include \"flow.hpp\"\n"
         "namespace lik {\n"
         "static_assert(sizeof(EngineArgs) == "
      << sizeof(EngineArgs) << ", \"EngineArgs layout\");\n"
         "static_assert(sizeof(FilterDesc) == "
      << sizeof(FilterDesc) << ", \"FilterDesc layout\");\n"
         "static_assert(sizeof(FlowArgs) == "
      << sizeof(FlowArgs) << ", \"FlowArgs layout\");\n";
}

}  // namespace

// One flow kernel for filters of several networks: each work item runs the
// specialised body of its filter's network (group g = index in nets; the
// branch is wave-uniform), with one LDS buffer for all of them.
std::string specialized_multi_source(const std::vector<lik_network *> &nets, int precision) {
    std::ostringstream o;
    emit_prelude(o);
    for (size_t g = 0; g < nets.size(); ++g)
        emit_spec_net(o, *nets[g], ("SpecNet" + std::to_string(g)).c_str());
    o << "constexpr int cmax(int a, int b) { return a > b ? a : b; }\n"
         "constexpr int kMultiLds = 0";
    for (size_t g = 0; g < nets.size(); ++g) {
        const int U = nets[g]->U, R = nets[g]->R;
        o << ";\nconstexpr int kMultiLds" << g << " = cmax(kMultiLds"
          << (g ? std::to_string(g - 1) : std::string("")) << ", item_lds_words<" << U << ", "
          << R << ", " << precision << ">())";
    }
    o << ";\n}  // namespace lik\n";
    o << "extern \"C\" __global__ __launch_bounds__(64) void lik_flow_spec_multi("
         "lik::EngineArgs e, const lik::FlowArgs *fa) {\n"
         "  __shared__ __attribute__((aligned(16))) uint32_t lds[lik::kMultiLds"
      << nets.size() - 1 << "];\n"
         "  lik::flow_run_with(e, *fa, [&](uint32_t item) {\n"
         "    const int g = __builtin_amdgcn_readfirstlane(e.desc[item >> 6].group);\n"
         "    switch (g) {\n";
    for (size_t g = 0; g < nets.size(); ++g) {
        const int U = nets[g]->U, R = nets[g]->R, W = (U + 7) / 8;
        o << "    case " << g << ": { const lik::SpecNet" << g << " n{}; lik::run_item<lik::SpecNet"
          << g << ", " << U << ", " << R << ", " << W << ", " << precision
          << ">(e, n, item, lds); break; }\n";
    }
    o << "    default: break;\n    }\n  });\n}\n";
    return o.str();
}

std::string specialized_source(const lik_network &net, int precision) {
    const int U = net.U, R = net.R, W = (U + 7) / 8;
    std::ostringstream o;
    o << "typedef __hip_internal::uint32_t uint32_t;\n"
         "typedef __hip_internal::uint64_t uint64_t;\n"
         "typedef __hip_internal::int32_t int32_t;\n"
         "typedef __hip_internal::int64_t int64_t;\n"
         "typedef __hip_internal::uint8_t uint8_t;\n"
         "typedef __hip_internal::uint16_t uint16_t;\n"
         "#include \"flow.hpp\"\n"
         "namespace lik {\n"
         "static_assert(sizeof(EngineArgs) == "
      << sizeof(EngineArgs) << ", \"EngineArgs layout\");\n"
         "static_assert(sizeof(FilterDesc) == "
      << sizeof(FilterDesc) << ", \"FilterDesc layout\");\n"
         "static_assert(sizeof(FlowArgs) == "
      << sizeof(FlowArgs) << ", \"FlowArgs layout\");\n";
    o << "struct SpecNet {\n  static constexpr int U = " << U << ", R = " << R << ";\n";
    auto arr = [&](const char *name, const int32_t *v) {
        o << "  static constexpr int " << name << "[" << R << "] = {";
        for (int r = 0; r < R; ++r) o << (r ? "," : "") << v[r];
        o << "};\n";
    };
    arr("kind", net.kind);
    arr("s1", net.s1);
    arr("s2", net.s2);
    o << "  static constexpr unsigned nu[" << R << "][" << W << "] = {";
    for (int r = 0; r < R; ++r) {
        o << (r ? "," : "") << "{";
        for (int w = 0; w < W; ++w) o << (w ? "," : "") << net.nu[r][w] << "u";
        o << "}";
    }
    o << "};\n};\n}  // namespace lik\n";
    o << "extern \"C\" __global__ __launch_bounds__(64) void lik_propagate_spec("
         "lik::EngineArgs e, int group) {\n"
         "  const lik::SpecNet net{};\n"
         "  lik::propagate_item<lik::SpecNet, "
      << U << ", " << R << ", " << W << ", " << precision << ">(e, net, group);\n}\n";
    // e must stay the first argument: flow_run reads it again from offset 0
    // of the kernel-argument segment
    o << "extern \"C\" __global__ __launch_bounds__(64) void lik_flow_spec("
         "lik::EngineArgs e, const lik::FlowArgs *fa) {\n"
         "  const lik::SpecNet net{};\n"
         "  lik::flow_run<lik::SpecNet, "
      << U << ", " << R << ", " << W << ", " << precision << ">(e, *fa, net);\n}\n";
    if (R <= kPersistentMaxR)
        o << "extern \"C\" __global__ __launch_bounds__(64) void lik_propagate_spec_p("
             "lik::EngineArgs e, int group) {\n"
             "  const lik::SpecNet net{};\n"
             "  lik::propagate_persistent<lik::SpecNet, "
          << U << ", " << R << ", " << W << ", " << precision << ">(e, net, group);\n}\n";
    return o.str();
}

namespace {

// Code object of a generated source: from the disk cache or compiled now.
bool code_for_source(const std::string &src, std::vector<char> *code, std::string *path_out,
                     std::string *err);

// Code object for (network, precision): from the disk cache or compiled now.
bool specialized_code(const lik_network &net, int precision, std::vector<char> *code,
                      std::string *src_out, std::string *path_out, std::string *err) {
    const std::string src = specialized_source(net, precision);
    *src_out = src;
    return code_for_source(src, code, path_out, err);
}

bool code_for_source(const std::string &src, std::vector<char> *code, std::string *path_out,
                     std::string *err) {
    // the key covers everything the code object depends on: the generated
    // source, the embedded kernel headers, the options and the compiler
    std::string key = src;
    const char *const *hdr = nullptr;
    const char *const *names = nullptr;
    const int nh = rtc_headers(&hdr, &names);
    for (int i = 0; i < nh; ++i) key += std::string(names[i]) + hdr[i];
    for (int i = 0; i < kRtcNumOptions; ++i) key += std::string(" ") + kRtcOptions[i];
    int rtc_major = 0, rtc_minor = 0;
    hiprtcVersion(&rtc_major, &rtc_minor);
    key += " hiprtc " + std::to_string(rtc_major) + "." + std::to_string(rtc_minor);
    char hex[32];
    snprintf(hex, sizeof(hex), "%016llx", (unsigned long long)fnv1a(key));
    const std::string dir = cache_dir();
    const std::string path = dir + "/prop_" + hex + ".co";

    *path_out = path;
    if (read_file(path, code)) return true;
    if (!compile(src, code, err)) return false;
    write_file_atomic(dir, path, *code);
    return true;
}

}  // namespace

bool precompile_specialized(const lik_network &net, int precision, std::string *err) {
    std::vector<char> code;
    std::string src, path;
    return specialized_code(net, precision, &code, &src, &path, err);
}

hipFunction_t specialized_kernel(lik_network &net, int precision, std::string *err,
                                 int kind) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return nullptr;
    }
    std::lock_guard<std::mutex> g(net.spec_lock);
    auto it = net.spec.find({dev, precision});
    auto pick = [kind](const lik_network::SpecKernels &k) {
        return kind == kSpecPersistent ? k.persistent : kind == kSpecFlow ? k.flow : k.item;
    };
    if (it != net.spec.end()) return pick(it->second);

    std::vector<char> code;
    std::string src, path;
    if (!specialized_code(net, precision, &code, &src, &path, err)) return nullptr;
    const std::string dir = cache_dir();
    hipModule_t mod = nullptr;
    hipError_t e = hipModuleLoadData(&mod, code.data());
    if (e != hipSuccess) {
        // a damaged cache entry: compile afresh once
        code.clear();
        if (!compile(src, &code, err)) return nullptr;
        write_file_atomic(dir, path, code);
        e = hipModuleLoadData(&mod, code.data());
        if (e != hipSuccess) {
            *err = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
            return nullptr;
        }
    }
    lik_network::SpecKernels k;
    k.mod = mod;
    e = hipModuleGetFunction(&k.item, mod, "lik_propagate_spec");
    if (e != hipSuccess) {
        *err = std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
        (void)hipModuleUnload(mod);
        return nullptr;
    }
    if (net.R <= kPersistentMaxR && hipModuleGetFunction(&k.persistent, mod,
                                                         "lik_propagate_spec_p") != hipSuccess)
        k.persistent = nullptr;
    if (hipModuleGetFunction(&k.flow, mod, "lik_flow_spec") != hipSuccess) k.flow = nullptr;
    net.spec[{dev, precision}] = k;
    return pick(k);
}

hipFunction_t loaded_specialized_kernel(lik_network &net, int precision, int kind) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> g(net.spec_lock);
    auto it = net.spec.find({dev, precision});
    if (it == net.spec.end()) return nullptr;
    const lik_network::SpecKernels &k = it->second;
    return kind == kSpecPersistent ? k.persistent : kind == kSpecFlow ? k.flow : k.item;
}

namespace {
// Multi-network flow kernels, per (device, source): loaded once and kept for
// the life of the process (a set of networks has no handle that owns them).
std::mutex g_multi_mu;
std::map<std::pair<int, std::string>, std::pair<hipModule_t, hipFunction_t>> g_multi;
}  // namespace

bool rtc_code(const std::string &src, std::vector<char> *code, std::string *err) {
    std::string path;
    return code_for_source(src, code, &path, err);
}

bool precompile_multi(const std::vector<lik_network *> &nets, int precision, std::string *err) {
    std::vector<char> code;
    std::string path;
    return code_for_source(specialized_multi_source(nets, precision), &code, &path, err);
}

hipFunction_t specialized_multi_kernel(const std::vector<lik_network *> &nets, int precision,
                                       std::string *err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return nullptr;
    }
    const std::string src = specialized_multi_source(nets, precision);
    std::lock_guard<std::mutex> g(g_multi_mu);
    auto it = g_multi.find({dev, src});
    if (it != g_multi.end()) return it->second.second;
    std::vector<char> code;
    std::string path;
    if (!code_for_source(src, &code, &path, err)) return nullptr;
    hipModule_t mod = nullptr;
    hipError_t e = hipModuleLoadData(&mod, code.data());
    if (e != hipSuccess) {
        *err = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
        return nullptr;
    }
    hipFunction_t fn = nullptr;
    e = hipModuleGetFunction(&fn, mod, "lik_flow_spec_multi");
    if (e != hipSuccess) {
        *err = std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
        (void)hipModuleUnload(mod);
        return nullptr;
    }
    g_multi[{dev, src}] = {mod, fn};
    return fn;
}

void release_specialized(lik_network &net) {
    std::lock_guard<std::mutex> g(net.spec_lock);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : net.spec) {
        (void)hipSetDevice(kv.first.first);
        (void)hipModuleUnload(kv.second.mod);
    }
    if (!net.spec.empty()) (void)hipSetDevice(cur);
    net.spec.clear();
}

}  // namespace lik
