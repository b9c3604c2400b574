// Pass kernels compiled at run time for one pass program each (hiprtc).
//
// The library's pass kernels interpret a pass program per tile: each operation's kind and
// position are read from LDS, so every operation goes through a dispatch whose branches all
// keep the tile's amplitudes in registers, and the compiler then keeps them in one set of
// registers at the loop head and another at the end of each branch, copying one into the other
// after every operation.  A compiled pass has its program as straight-line code: the gates'
// kinds and positions and a diagonal group's register weights are constants, the copies and
// the selects on them go away.  The device code is the same (pass_dev.hpp); only the program
// comes from the generated source instead of LDS.
#pragma once
#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "sf_host.hpp"

namespace sf {

// The body of the program (the statements of pass_body's P::apply, see pass_dev.hpp) for one
// pass plan, or "" for a dense block (matrix cores, its own kernel).
std::string jit_program(const PassPlan &pp);

// Kernel source of one pass (prog1 empty) or of the two blocks' passes of one level in one launch
// (a pair, the first grid0 workgroups running prog0), complex64 or complex128 states, R register
// bits and zero-subspace skipping per pass.  The kernel's name and namespace are the placeholders
// SFJ_KERNEL and SFJ_NS, which jit_kernels fills from a hash of the source.
std::string jit_kernel(bool fp64, int R0, const std::string &prog0, bool zskip0, int R1, const std::string &prog1,
                       bool zskip1);

// The kernels of the given sources on the current device: from the process-wide cache, or
// (compile) compiled, the missing ones in parallel, a few per hiprtc program, and loaded.
// fns[i] receives the kernel of sources[i] (nullptr if not cached and compile is false);
// *compile_ms the time spent compiling in this call.  0 or an SF_ERR_* code with err set.
int jit_kernels(const std::vector<std::string> &sources, std::vector<hipFunction_t> &fns, double *compile_ms,
                std::string &err, bool compile = true);

// Compiles the sources for `arch` (e.g. "gfx950") without a device and loads nothing: the total
// code-object size, or an SF_ERR_* code with the compiler's log in err.
int jit_compile_only(const std::vector<std::string> &sources, const std::string &arch, uint64_t *code_bytes,
                     std::string &err);

}  // namespace sf
