// Plan-specialised tile-pass kernels compiled at run time (hiprtc).
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "host.h"
#include "tile_frame.h"

namespace svmi {

struct JitModule {
    std::vector<hipModule_t> mods;
    std::vector<hipFunction_t> fns;   // one kernel per pass
    ~JitModule();
};

// SVMI_JIT=0 in the environment disables run-time specialisation.
bool jit_enabled();
// Compile (or fetch from the in-memory / on-disk cache) one kernel per pass.
std::shared_ptr<JitModule> jit_get(const EncodedPlan& ep, int dtype, bool two, int nt, std::string& err);
// Compile only (no device needed); used by planning checks.
bool jit_compile_only(const EncodedPlan& ep, int dtype, bool two, int nt, std::string& err);
hipError_t jit_launch(const JitModule& jm, int pass, const TileArgs& a, uint64_t nblocks, int nt, size_t lds,
                      hipStream_t s);
std::string jit_pass_source(const EncodedPlan& ep, int pass, int dtype, bool two, int nt);

}  // namespace svmi
