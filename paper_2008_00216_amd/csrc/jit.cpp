// Plan-specialised tile passes.
//
// The runtime interpreter (tile_pass.hip) dispatches every op through a
// switch on its type and register slot; on gfx950 that costs phi copies of
// all 16 register amplitudes per op.  For large states the planner's passes
// are instead emitted as straight-line HIP source -- one kernel per pass, each
// op a call of the same device templates (tile_ops.h) with its slot mask,
// table offsets and sign tables as compile-time constants -- and compiled
// with hiprtc for gfx950.  Modules are cached per plan in memory and, as code
// objects, on disk.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <unistd.h>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.h"
#include "jit.h"

extern "C" const char* svmi_jit_header_device_common;
extern "C" const char* svmi_jit_header_plan;
extern "C" const char* svmi_jit_header_tile_ops;
extern "C" const char* svmi_jit_header_tile_frame;

namespace svmi {

namespace {

uint64_t fnv(const std::string& s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string pass_source(const EncodedPlan& ep, int pi, int dtype, bool two, int nt) {
    const DPass& P = ep.passes[pi];
    const char* R = dtype == SV_C64 ? "float" : "double";
    const char* TW = two ? "true" : "false";
    std::ostringstream o;
    // c64 forward passes: at least 4 waves per SIMD (<= 128 VGPRs), as many as
    // the tile's LDS allows
    const bool two_wg = dtype == SV_C64 && !two && P.T <= 13;
    o << "extern \"C\" __global__ __launch_bounds__(" << nt << ")"
      << (two_wg ? " __attribute__((amdgpu_waves_per_eu(4, 8)))" : "") << " void svp_" << pi
      << "(svmi::TileArgs A) {\n";
    o << "  using namespace svmi;\n  using R = " << R << ";\n  using V = V2<R>;\n";
    o << "  extern __shared__ __align__(16) unsigned char smem[];\n";
    o << "  constexpr uint32_t L = " << P.L << ", H = " << P.H << ", T = " << P.T << ";\n";
    o << "  constexpr uint32_t HP[16] = {";
    for (int t = 0; t < 16; ++t) o << P.hpos[t] << (t < 15 ? "," : "");
    o << "};\n";
    o << "  TileFrame<R, " << nt << ", " << TW << "> F;\n";
    o << "  F.begin(A, smem, L, H, T, HP, " << P.nform << "u, " << P.form0 << "u, " << P.ngrad << "u);\n";
    o << "  const uint32_t tid = F.tid;\n  const R cw = F.ptab[1].x;\n  (void)cw;\n";
    const uint32_t ngroups = 1u << (P.T - kRegBits);
    // fewer register groups than threads (whole waves, 64 | ngroups): the
    // waves past the last group skip the phases and only help move the tile
    const bool part = ngroups < (uint32_t)nt;
    const uint32_t iters = part ? 1u : ngroups / nt;
    for (uint32_t ph = 0; ph < P.nphase; ++ph) {
        const DPhase& Ph = ep.phases[P.phase0 + ph];
        const uint32_t r[4] = {Ph.rpos & 255u, (Ph.rpos >> 8) & 255u, (Ph.rpos >> 16) & 255u, Ph.rpos >> 24};
        o << "  { // phase " << ph << "\n";
        o << "    constexpr uint32_t r0 = " << r[0] << ", r1 = " << r[1] << ", r2 = " << r[2] << ", r3 = " << r[3]
          << ";\n";
        o << "    constexpr uint32_t soff[16] = {";
        for (int i = 0; i < 16; ++i) o << Ph.soff[i] << (i < 15 ? "," : "");
        o << "};\n";
        if (part) o << "    if (tid < " << ngroups << "u)\n";
        o << "    for (uint32_t it = 0; it < " << iters << "u; ++it) {\n";
        o << "      const uint32_t gg = it * " << nt << "u + tid;\n";
        o << "      const uint32_t lb = ins0(ins0(ins0(ins0(gg, r0), r1), r2), r3);\n";
        o << "      const uint32_t sb = swz<R>(lb);\n";
        o << "      V a[16]; V l[16];\n      F.load_group(sb, soff, a, l, true);\n";
        for (uint32_t oi = Ph.op0; oi < Ph.op0 + Ph.nop; ++oi) {
            const DOp& op = ep.ops[oi];
            switch (op.type) {
                case OP_DENSE:
                    o << "      op_dense<R, " << op.mask << ">(a, F.pool + " << op.arg << ");\n";
                    if (two) o << "      op_dense<R, " << op.mask << ">(l, F.pool + " << op.arg << ");\n";
                    break;
                case OP_DIAGR:
                    o << "      op_diag<R, " << op.mask << ">(a, F.pool + " << op.arg << ");\n";
                    if (two) o << "      op_diag<R, " << op.mask << ">(l, F.pool + " << op.arg << ");\n";
                    break;
                case OP_BF: {
                    const uint32_t M = op.k & 7u, S = (op.k >> 4) & 3u, RM = (op.k >> 8) & 15u;
                    const bool uni = (op.k & kBfUniform) != 0;
                    const uint64_t gm = (uni || op.arg == kNoPair) ? 0ull : ep.pairs[op.arg].m[0];
                    const bool rt = op.mask != 0 || gm != 0;
                    o << "      { ";
                    if (rt)
                        o << "const R s_ = bf_parity(lb, " << op.mask << "u, F.base, " << gm << "ull) ? R(-1) : R(1); ";
                    else
                        o << "const R s_ = R(1); ";
                    const std::string targs = std::to_string(S) + ", " + std::to_string(M) + ", " + std::to_string(RM) +
                                              ", " + (rt ? "true" : "false");
                    o << "op_bf<R, " << targs << ">(a, s_, cw);";
                    if (two) o << " op_bf<R, " << targs << ">(l, s_, cw);";
                    o << " }\n";
                    break;
                }
                case OP_D1T: {
                    const uint32_t S = op.k & 3u, RM = (op.k >> 2) & 15u, real = (op.k >> 6) & 1u, pk = op.k >> 7;
                    const uint64_t gm = pk == 0 ? 0ull : ep.pairs[pk - 1].m[0];
                    const bool rt = op.mask != 0 || gm != 0;
                    o << "      { ";
                    if (rt)
                        o << "const R s_ = bf_parity(lb, " << op.mask << "u, F.base, " << gm << "ull) ? R(-1) : R(1); ";
                    else
                        o << "const R s_ = R(1); ";
                    const std::string targs = std::to_string(S) + ", " + std::to_string(RM) + ", " +
                                              (rt ? "true" : "false") + ", " + (real ? "true" : "false");
                    o << "op_d1t<R, " << targs << ">(a, F.pool + " << op.arg << ", s_);";
                    if (two) o << " op_d1t<R, " << targs << ">(l, F.pool + " << op.arg << ", s_);";
                    o << " }\n";
                    break;
                }
                case OP_PERM: {
                    const uint32_t sa = op.mask & 3u, sb = op.k <= 2 ? sa : (op.mask >> 2) & 3u;
                    const std::string targs = std::to_string(op.k) + ", " + std::to_string(sa) + ", " +
                                              std::to_string(sb);
                    o << "      op_perm<R, " << targs << ">(a);\n";
                    if (two) o << "      op_perm<R, " << targs << ">(l);\n";
                    break;
                }
                case OP_SCALE:
                    o << "      { const R s_ = F.pool[" << op.arg << "].x; op_scale<R>(a, s_);";
                    if (two) o << " op_scale<R>(l, s_);";
                    o << " }\n";
                    break;
                case OP_SIGN:
                case OP_PHASE8: {
                    const DForm& Fm = ep.forms[op.arg];
                    o << "      { uint32_t e0, d[4];\n";
                    o << "        const uint32_t et = A.etab[" << Fm.etab << "u + gg];\n";
                    o << "        form_thread(F.fl + " << 4 * Fm.slot << ", et, lb, r0, r1, r2, r3, e0, d);\n";
                    if (op.type == OP_SIGN) {
                        o << "        op_sign<R, " << TW << ">(a, l, e0, d, " << Fm.abits << "u); }\n";
                    } else {
                        const uint64_t At = (uint64_t)Fm.a_lo | ((uint64_t)Fm.a_hi << 32);
                        o << "        op_phase8<R, " << TW << ">(a, l, e0, d, " << At << "ull, F.ptab); }\n";
                    }
                    break;
                }
                case OP_GRAD: {
                    if (!two) break;
                    if (op.k == GEN_P11) {
                        o << "      F.grad_add(" << op.arg << "u, op_grad11<R, " << op.mask << ">(a, l));\n";
                    } else {
                        const int s = __builtin_ctz(op.mask);
                        const char* gn = op.k == GEN_X ? "GEN_X" : (op.k == GEN_Y ? "GEN_Y" : "GEN_Z");
                        o << "      F.grad_add(" << op.arg << "u, op_grad1<R, " << s << ", " << gn << ">(a, l));\n";
                    }
                    break;
                }
                default:
                    break;
            }
        }
        o << "      F.store_group(sb, soff, a, l, true);\n";
        o << "    }\n    __syncthreads();\n  }\n";
    }
    o << "  F.end(A, L, H, HP);\n}\n";
    return o.str();
}

std::string cache_dir() {
    const char* d = std::getenv("SVMI_JIT_CACHE");
    std::string s = d && *d ? d : "/tmp/svmi-jit-cache";
    mkdir(s.c_str(), 0755);
    return s;
}

bool compile_one(const std::string& src, const std::string& name, std::vector<char>& code, std::string& err) {
    hiprtcProgram prog;
    const char* hs[] = {svmi_jit_header_device_common, svmi_jit_header_plan, svmi_jit_header_tile_ops,
                        svmi_jit_header_tile_frame};
    const char* hn[] = {"device_common.h", "plan.h", "tile_ops.h", "tile_frame.h"};
    if (hiprtcCreateProgram(&prog, src.c_str(), name.c_str(), 4, hs, hn) != HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return false;
    }
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-mllvm", "-simplifycfg-sink-common=false",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        err = "hiprtc: " + log.substr(0, 2000);
        hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code.resize(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return true;
}

std::mutex g_mu;
std::unordered_map<uint64_t, std::shared_ptr<JitModule>> g_mods;

}  // namespace

JitModule::~JitModule() {
    for (auto m : mods)
        if (m) (void)hipModuleUnload(m);
}

bool jit_enabled() {
    const char* e = std::getenv("SVMI_JIT");
    return !(e && e[0] == '0');
}

namespace {
// Compile every pass (using the on-disk cache); fills codes[p].
bool compile_all(const EncodedPlan& ep, int dtype, bool two, int nt, std::vector<std::string>& srcs,
                 std::vector<std::vector<char>>& codes, std::string& err);
}  // namespace

bool jit_compile_only(const EncodedPlan& ep, int dtype, bool two, int nt, std::string& err) {
    std::vector<std::string> srcs;
    std::vector<std::vector<char>> codes;
    return compile_all(ep, dtype, two, nt, srcs, codes, err);
}

namespace {
bool compile_all(const EncodedPlan& ep, int dtype, bool two, int nt, std::vector<std::string>& srcs,
                 std::vector<std::vector<char>>& codes, std::string& err) {
    const int np = (int)ep.passes.size();
    srcs.assign((size_t)np, std::string());
    for (int p = 0; p < np; ++p)
        srcs[p] = "#include \"tile_frame.h\"\n#include \"tile_ops.h\"\n" + pass_source(ep, p, dtype, two, nt);
    const std::string dir = cache_dir();
    codes.assign((size_t)np, std::vector<char>());
    std::vector<std::string> errs((size_t)np);
    std::vector<int> todo;
    auto fname = [&](int p) {
        char fn[64];
        std::snprintf(fn, sizeof(fn), "/%016llx.co",
                      (unsigned long long)fnv(srcs[p] + svmi_jit_header_tile_ops + svmi_jit_header_tile_frame +
                                              svmi_jit_header_device_common + svmi_jit_header_plan));
        return dir + fn;
    };
    for (int p = 0; p < np; ++p) {
        std::ifstream f(fname(p), std::ios::binary);
        if (f) codes[p].assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
        if (codes[p].empty()) todo.push_back(p);
    }
    if (todo.empty()) return true;
    unsigned hw = std::thread::hardware_concurrency();
    const int nthr = (int)std::max(1u, std::min<unsigned>(hw ? hw : 4, 16u));
    std::vector<std::thread> th;
    std::mutex qm;
    size_t next = 0;
    for (int t = 0; t < std::min<int>(nthr, (int)todo.size()); ++t) {
        th.emplace_back([&] {
            for (;;) {
                int p;
                {
                    std::lock_guard<std::mutex> lk(qm);
                    if (next >= todo.size()) return;
                    p = todo[next++];
                }
                compile_one(srcs[p], "svp_" + std::to_string(p) + ".hip", codes[p], errs[p]);
            }
        });
    }
    for (auto& t : th) t.join();
    for (int p : todo) {
        if (codes[p].empty()) {
            err = errs[p].empty() ? "hiprtc compile failed" : errs[p];
            return false;
        }
        const std::string fn = fname(p);
        const std::string tmp = fn + ".tmp" + std::to_string((long long)p) + "." + std::to_string((long long)getpid());
        std::ofstream f(tmp, std::ios::binary);
        f.write(codes[p].data(), (std::streamsize)codes[p].size());
        f.close();
        std::rename(tmp.c_str(), fn.c_str());
    }
    return true;
}
}  // namespace

std::shared_ptr<JitModule> jit_get(const EncodedPlan& ep, int dtype, bool two, int nt, std::string& err) {
    // one source per pass; passes are compiled in parallel
    const int np = (int)ep.passes.size();
    std::vector<std::string> srcs;
    std::vector<std::vector<char>> codes;
    std::string all;
    for (int p = 0; p < np; ++p) all += pass_source(ep, p, dtype, two, nt);
    const uint64_t key = fnv(all) ^ fnv(svmi_jit_header_tile_ops) ^ (fnv(svmi_jit_header_tile_frame) << 1) ^
                         ((uint64_t)dtype << 60) ^ ((uint64_t)two << 62);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_mods.find(key);
        if (it != g_mods.end()) return it->second;
    }
    if (!compile_all(ep, dtype, two, nt, srcs, codes, err)) return nullptr;
    auto jm = std::make_shared<JitModule>();
    jm->mods.assign((size_t)np, nullptr);
    jm->fns.assign((size_t)np, nullptr);
    for (int p = 0; p < np; ++p) {
        hipError_t e = hipModuleLoadData(&jm->mods[p], codes[p].data());
        if (e != hipSuccess) {
            err = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
            return nullptr;
        }
        e = hipModuleGetFunction(&jm->fns[p], jm->mods[p], ("svp_" + std::to_string(p)).c_str());
        if (e != hipSuccess) {
            err = std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
            return nullptr;
        }
        // passes need up to 160 KiB of LDS
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(jm->fns[p]),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_mods[key] = jm;
    return jm;
}

hipError_t jit_launch(const JitModule& jm, int pass, const TileArgs& a, uint64_t nblocks, int nt, size_t lds,
                      hipStream_t s) {
    TileArgs arg = a;
    void* params[] = {&arg};
    return hipModuleLaunchKernel(jm.fns[pass], (unsigned)nblocks, 1, 1, (unsigned)nt, 1, 1, (unsigned)lds, s, params,
                                 nullptr);
}

std::string jit_pass_source(const EncodedPlan& ep, int pass, int dtype, bool two, int nt) {
    return pass_source(ep, pass, dtype, two, nt);
}

}  // namespace svmi
