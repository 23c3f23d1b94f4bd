// jit_rtc.cpp -- hipRTC compilation of tile-pass kernels (see jit_rtc.h).
#include "jit_rtc.h"

#include <hip/hiprtc.h>

#include <cstdio>

#include "tile_dev_src.inc"   // kTileDevSrc: the text of tile_dev.h (generated at build time)

namespace dq {
namespace {

const char *const kOpts[] = {"-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                             "-mllvm", "-simplifycfg-sink-common=false"};
constexpr int kNOpts = sizeof(kOpts) / sizeof(kOpts[0]);

uint64_t fnv1a(const std::string &s, uint64_t h = 1469598103934665603ull) {
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace

std::string jit_key(const std::string &body) {
    std::string salt(kTileDevSrc);
    for (int i = 0; i < kNOpts; ++i) salt += kOpts[i];
    char buf[32];
    snprintf(buf, sizeof buf, "dqj_%016llx", (unsigned long long)fnv1a(body, fnv1a(salt)));
    return buf;
}

bool jit_compile(const std::string &src, const std::string &arch, std::vector<char> &code, std::string &err) {
    hiprtcProgram prog;
    const char *hdr = kTileDevSrc;
    const char *hname = "tile_dev.h";
    if (hiprtcCreateProgram(&prog, src.c_str(), "dq_pass.hip", 1, &hdr, &hname) != HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return false;
    }
    std::vector<const char *> opts(kOpts, kOpts + kNOpts);
    const std::string a = "--offload-arch=" + arch;
    opts.push_back(a.c_str());
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        err = std::string("hipRTC: ") + hiprtcGetErrorString(r) + "\n" + log.substr(0, 4000);
        hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    code.resize(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return n > 0;
}

}  // namespace dq
