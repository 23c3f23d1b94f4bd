// jit.cpp -- register-tile passes compiled at plan time.
//
// The runtime turns each distinct tile pass (its operation list in tile-local
// bit positions, matrix slots relative to the pass) into the source of one
// kernel: a straight-line sequence of calls into tile_dev.h whose operand
// positions are template constants.  This file compiles such sources with
// hipRTC for the current device's architecture, keeps the loaded kernels in
// a process-wide cache keyed by a hash of (header, options, source), and
// optionally stores the code objects on disk (DQ_JIT_CACHE, default
// $HOME/.cache/dq_jit; "off" disables it).
#include "dq_internal.h"

#include <hip/hiprtc.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <thread>
#include <unistd.h>
#include <vector>

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

struct Entry {
    std::vector<char> code;
    std::map<int, hipModule_t> mod;
    std::map<int, hipFunction_t> fn;
    std::map<int, int> resident;   // device -> resident single-wave blocks (forward grid)
};

std::mutex g_mu;
std::map<std::string, Entry> g_cache;

std::string arch_of_current(std::string &err) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        err = "no current HIP device";
        return "";
    }
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

std::string cache_dir() {
    const char *e = getenv("DQ_JIT_CACHE");
    if (e && *e) return strcmp(e, "off") == 0 ? std::string() : std::string(e);
    const char *h = getenv("HOME");
    if (!h || !*h) return std::string();
    return std::string(h) + "/.cache/dq_jit";
}

bool read_file(const std::string &path, std::vector<char> &out) {
    FILE *f = fopen(path.c_str(), "rb");
    if (!f) return false;
    fseek(f, 0, SEEK_END);
    const long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    bool ok = n > 0;
    if (ok) {
        out.resize((size_t)n);
        ok = fread(out.data(), 1, (size_t)n, f) == (size_t)n;
    }
    fclose(f);
    return ok;
}

void write_file(const std::string &dir, const std::string &name, const std::vector<char> &data) {
    if (dir.empty()) return;
    // create the directory chain; failures only disable the disk cache
    for (size_t p = 1; p <= dir.size(); ++p)
        if (p == dir.size() || dir[p] == '/') mkdir(dir.substr(0, p).c_str(), 0755);
    const std::string tmp = dir + "/" + name + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return;
    const bool ok = fwrite(data.data(), 1, data.size(), f) == data.size();
    fclose(f);
    if (ok) rename(tmp.c_str(), (dir + "/" + name).c_str());
    else unlink(tmp.c_str());
}

// compile one kernel source; returns false with the compiler log in err
bool compile(const std::string &src, const std::string &arch, std::vector<char> &code, std::string &err) {
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
    return true;
}

}  // namespace

std::string jit_key(const std::string &body) {
    std::string salt(kTileDevSrc);
    for (int i = 0; i < kNOpts; ++i) salt += kOpts[i];
    char buf[32];
    snprintf(buf, sizeof buf, "dqj_%016llx", (unsigned long long)fnv1a(body, fnv1a(salt)));
    return buf;
}

bool jit_load(const std::vector<std::string> &names, const std::vector<std::string> &srcs,
              std::vector<hipFunction_t> &out, std::string &err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice failed";
        return false;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    const std::string arch = arch_of_current(err);
    if (arch.empty()) return false;
    const std::string dir = cache_dir();
    // code objects: process cache, then disk cache, then compile (in parallel)
    std::vector<size_t> todo;
    for (size_t i = 0; i < names.size(); ++i) {
        Entry &E = g_cache[names[i]];
        if (!E.code.empty()) continue;
        if (!dir.empty() && read_file(dir + "/" + names[i] + "-" + arch + ".co", E.code)) continue;
        todo.push_back(i);
    }
    if (!todo.empty()) {
        std::vector<std::vector<char>> codes(todo.size());
        std::vector<std::string> errs(todo.size());
        std::vector<char> okv(todo.size(), 0);
        std::atomic<size_t> next{0};
        unsigned nt = std::thread::hardware_concurrency();
        nt = nt < 1 ? 1 : (nt > 16 ? 16 : nt);
        if (nt > todo.size()) nt = (unsigned)todo.size();
        auto work = [&]() {
            for (size_t j; (j = next++) < todo.size();)
                okv[j] = compile(srcs[todo[j]], arch, codes[j], errs[j]) ? 1 : 0;
        };
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t) th.emplace_back(work);
        for (auto &t : th) t.join();
        for (size_t j = 0; j < todo.size(); ++j) {
            if (!okv[j]) {
                err = "compiling pass " + names[todo[j]] + ": " + errs[j];
                return false;
            }
            g_cache[names[todo[j]]].code = codes[j];
            write_file(dir, names[todo[j]] + "-" + arch + ".co", codes[j]);
        }
    }
    out.assign(names.size(), nullptr);
    for (size_t i = 0; i < names.size(); ++i) {
        Entry &E = g_cache[names[i]];
        auto it = E.fn.find(dev);
        if (it == E.fn.end()) {
            hipModule_t m = nullptr;
            hipFunction_t f = nullptr;
            hipError_t e = hipModuleLoadData(&m, E.code.data());
            if (e == hipSuccess) e = hipModuleGetFunction(&f, m, names[i].c_str());
            if (e != hipSuccess) {
                err = "loading pass " + names[i] + ": " + hipGetErrorString(e);
                return false;
            }
            E.mod[dev] = m;
            it = E.fn.emplace(dev, f).first;
            int per_cu = 0, cus = 0;
            if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 64, 0) != hipSuccess || per_cu < 1)
                per_cu = 2;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
                cus = 256;
            E.resident[dev] = per_cu * cus;
        }
        out[i] = it->second;
    }
    return true;
}

int jit_resident(hipFunction_t f, size_t lds) {
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 64, lds) != hipSuccess || per_cu < 1) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 0;
    return per_cu * cus;
}

hipError_t jit_launch(hipFunction_t f, const std::string &name, const TileArgs &a, bool adj, hipStream_t s) {
    void *args[] = {(void *)&a};
    if (adj) {
        const size_t lds = sizeof(double) * 64 * (a.nlslots > 0 ? a.nlslots : 1);
        return hipModuleLaunchKernel(f, (unsigned)a.wps, (unsigned)a.batch, 1, 64, 1, 1, (unsigned)lds, s, args, nullptr);
    }
    int resident = 0;
    {
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(name);
        if (it != g_cache.end()) resident = it->second.resident[dev];
    }
    const int64_t tiles = a.batch << (a.n - 6 - a.R);
    const int64_t cap = resident > 0 ? resident : 4096;
    const unsigned g = (unsigned)(tiles < cap ? (tiles < 1 ? 1 : tiles) : cap);
    return hipModuleLaunchKernel(f, g, 1, 1, 64, 1, 1, 0, s, args, nullptr);
}

}  // namespace dq
