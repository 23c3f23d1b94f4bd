// jit_rtc.h -- compiling one tile-pass kernel source with hipRTC.
//
// Shared by the library (jit.cpp) and the helper program dq_jitc, which
// compiles one source per process: hipRTC serializes the compiles of one
// process, so passes compile in parallel only in separate processes.
#pragma once

#include <string>
#include <vector>

namespace dq {

// "dqj_<16 hex digits>": a hash of the kernel body, the tile_dev.h text and
// the compiler options, so that a changed header or option renames kernels
std::string jit_key(const std::string &body);

// compile src (which includes "tile_dev.h") for arch (e.g. "gfx950") into a
// loadable code object; false with the compiler log in err
bool jit_compile(const std::string &src, const std::string &arch, std::vector<char> &code, std::string &err);

}  // namespace dq
