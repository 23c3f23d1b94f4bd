// jit.cpp -- register-tile passes compiled at plan time.
//
// The runtime turns each distinct tile pass (its operation list in tile-local
// bit positions, matrix slots relative to the pass) into the source of one
// kernel: a straight-line sequence of calls into tile_dev.h whose operand
// positions are template constants.  This file compiles such sources with
// hipRTC for the current device's architecture (jit_rtc.cpp), keeps the
// loaded kernels in a process-wide cache keyed by a hash of (header,
// options, source), and optionally stores the code objects on disk
// (DQ_JIT_CACHE, default $HOME/.cache/dq_jit; "off" disables it).
//
// hipRTC serializes the compiles of one process, so a plan with several
// passes to compile starts helper processes (dq_jitc, installed next to the
// library), up to eight at a time, and compiles in-process whatever they did
// not deliver.
#include "dq_internal.h"
#include "jit_rtc.h"

#include <dlfcn.h>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <cerrno>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

extern char **environ;

namespace dq {
namespace {

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

// the helper program next to the shared library that holds this code, or ""
std::string helper_path() {
    Dl_info info;
    if (!dladdr((void *)&helper_path, &info) || !info.dli_fname) return std::string();
    const std::string lib(info.dli_fname);
    const size_t k = lib.rfind('/');
    const std::string p = (k == std::string::npos ? std::string(".") : lib.substr(0, k)) + "/dq_jitc";
    return access(p.c_str(), X_OK) == 0 ? p : std::string();
}

bool write_all(const std::string &path, const std::string &text) {
    FILE *f = fopen(path.c_str(), "wb");
    if (!f) return false;
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    return fclose(f) == 0 && ok;
}

// Compile srcs[i] in helper processes into codes[i] (left empty where a
// helper could not be started or failed).  Each child only runs hipRTC.
void compile_in_helpers(const std::vector<const std::string *> &srcs, const std::string &arch,
                        std::vector<std::vector<char>> &codes) {
    const std::string helper = helper_path();
    if (helper.empty()) return;
    const char *td = getenv("TMPDIR");
    std::string tmpl = std::string(td && *td ? td : "/tmp") + "/dq_jit_XXXXXX";
    std::vector<char> dbuf(tmpl.begin(), tmpl.end());
    dbuf.push_back('\0');
    if (!mkdtemp(dbuf.data())) return;
    const std::string dir(dbuf.data());
    const size_t n = srcs.size();
    std::vector<std::string> in(n), out(n);
    std::vector<char> written(n, 0);
    for (size_t i = 0; i < n; ++i) {
        in[i] = dir + "/p" + std::to_string(i) + ".hip";
        out[i] = dir + "/p" + std::to_string(i) + ".co";
        written[i] = write_all(in[i], *srcs[i]) ? 1 : 0;
    }
    unsigned par = std::thread::hardware_concurrency();
    par = par < 1 ? 1 : (par > 8 ? 8 : par);
    std::vector<std::pair<pid_t, size_t>> live;   // running helpers, oldest first
    size_t next = 0;
    while (next < n || !live.empty()) {
        while (live.size() < par && next < n) {
            const size_t i = next++;
            if (!written[i]) continue;
            std::vector<char *> argv = {const_cast<char *>(helper.c_str()), const_cast<char *>(arch.c_str()),
                                        const_cast<char *>(in[i].c_str()), const_cast<char *>(out[i].c_str()), nullptr};
            pid_t pid = 0;
            if (posix_spawn(&pid, helper.c_str(), nullptr, nullptr, argv.data(), environ) == 0)
                live.emplace_back(pid, i);
        }
        if (live.empty()) continue;
        // wait for our own children only (never waitpid(-1): the process may
        // have children of its own)
        const pid_t pid = live.front().first;
        const size_t i = live.front().second;
        live.erase(live.begin());
        int status = 0;
        pid_t r;
        do {
            r = waitpid(pid, &status, 0);
        } while (r < 0 && errno == EINTR);
        if (r == pid && WIFEXITED(status) && WEXITSTATUS(status) == 0) read_file(out[i], codes[i]);
    }
    for (size_t i = 0; i < n; ++i) {
        unlink(in[i].c_str());
        unlink(out[i].c_str());
    }
    rmdir(dir.c_str());
}

}  // namespace


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
        const auto t0 = std::chrono::steady_clock::now();
        std::vector<std::vector<char>> codes(todo.size());
        if (todo.size() > 1) {
            std::vector<const std::string *> ts;
            for (size_t j : todo) ts.push_back(&srcs[j]);
            compile_in_helpers(ts, arch, codes);
        }
        size_t by_helpers = 0;
        for (const auto &c : codes) by_helpers += c.empty() ? 0 : 1;
        for (size_t j = 0; j < todo.size(); ++j) {
            if (codes[j].empty()) {
                std::string e;
                if (!jit_compile(srcs[todo[j]], arch, codes[j], e)) {
                    err = "compiling pass " + names[todo[j]] + ": " + e;
                    return false;
                }
            }
            g_cache[names[todo[j]]].code = codes[j];
            write_file(dir, names[todo[j]] + "-" + arch + ".co", codes[j]);
        }
        const char *vb = getenv("DQ_JIT_VERBOSE");
        if (vb && *vb && strcmp(vb, "0") != 0)
            fprintf(stderr, "dq jit: compiled %zu pass kernels for %s (%zu in helper processes, %zu in process) in %.1f s\n",
                    todo.size(), arch.c_str(), by_helpers, todo.size() - by_helpers,
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
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
        if (it != g_cache.end()) {
            const auto r = it->second.resident.find(dev);
            if (r != it->second.resident.end()) resident = r->second;
        }
    }
    const int64_t tiles = a.batch << (a.n - 6 - a.R);
    // four grid-stride waves per resident slot: the waves that wait for a
    // slot fill the ramp-down of the ones before them (a 32-qubit forward
    // pass: 14.26 against 14.61 ms with one wave per slot)
    const int64_t cap = 4 * (resident > 0 ? resident : 4096);
    const unsigned g = (unsigned)(tiles < cap ? (tiles < 1 ? 1 : tiles) : cap);
    return hipModuleLaunchKernel(f, g, 1, 1, 64, 1, 1, 0, s, args, nullptr);
}

}  // namespace dq
