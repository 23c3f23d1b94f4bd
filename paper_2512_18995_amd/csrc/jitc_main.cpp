// dq_jitc -- compile one tile-pass kernel source into a code object.
//
//     dq_jitc <arch> <source file> <code object file>
//
// The library starts several of these at once when a plan has many passes to
// compile (hipRTC serializes compiles within one process).  Exit status 0 on
// success; otherwise the compiler log goes to stderr.  Touches no GPU.
#include <cstdio>
#include <string>
#include <vector>

#include "jit_rtc.h"

int main(int argc, char **argv) {
    if (argc != 4) {
        fprintf(stderr, "usage: dq_jitc <arch> <source file> <code object file>\n");
        return 2;
    }
    FILE *f = fopen(argv[2], "rb");
    if (!f) {
        fprintf(stderr, "dq_jitc: cannot read %s\n", argv[2]);
        return 2;
    }
    std::string src;
    char buf[65536];
    for (size_t k; (k = fread(buf, 1, sizeof buf, f)) > 0;) src.append(buf, k);
    fclose(f);
    std::vector<char> code;
    std::string err;
    if (!dq::jit_compile(src, argv[1], code, err)) {
        fprintf(stderr, "dq_jitc: %s\n", err.c_str());
        return 1;
    }
    const std::string tmp = std::string(argv[3]) + ".part";
    FILE *o = fopen(tmp.c_str(), "wb");
    if (!o) {
        fprintf(stderr, "dq_jitc: cannot write %s\n", tmp.c_str());
        return 2;
    }
    const bool ok = fwrite(code.data(), 1, code.size(), o) == code.size();
    if (fclose(o) != 0 || !ok || rename(tmp.c_str(), argv[3]) != 0) {
        remove(tmp.c_str());
        fprintf(stderr, "dq_jitc: writing %s failed\n", argv[3]);
        return 2;
    }
    return 0;
}
