// C ABI of libsvmi: contexts, validation, plan cache, executor, reductions,
// adjoint gradients and heterogeneous batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <fstream>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <sstream>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "host.h"
#include "jit.h"
#include "kernels.h"
#include "sv.h"

namespace svmi {
sv_status run_batch_persistent(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream,
                               int32_t flags, double* energies, double* grads, const sv_opts* opts,
                               sv_stats* stats, std::string& err, const GeomTable* geoms);
sv_status batch_launch_async(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream,
                             int32_t flags, const sv_opts* opts, std::string& err, const GeomTable* geoms,
                             void** job_out);
sv_status batch_finish_async(void* job, double* energies, double* grads, sv_stats* stats, std::string& err);
bool batch_tuned_table(int dtype, bool grad, GeomTable& out);
bool batch_tuned_lookup(int dtype, bool grad, int n, BatchGeom& g);
sv_status tune_batch(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream, int32_t flags,
                     const sv_opts* opts, int32_t* widths_tuned, std::string& err);
}

using namespace svmi;

namespace {

thread_local std::string g_err;

sv_status fail(sv_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            (void)hipGetLastError(); /* do not leave the error for the caller's next call */ \
            return fail(e_ == hipErrorOutOfMemory ? SV_ENOMEM : SV_EDEVICE,                  \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                  \
        }                                                                                    \
    } while (0)

// Device memory the library allocates for one context (plans, pools,
// reduction and sampling scratch), with an optional cap (sv_opts.max_work_mib).
struct WorkAcct {
    size_t used = 0;
    size_t cap = 0;      // 0 = no cap
};

// Pinned host staging (hipHostMalloc), so that copies through it are
// asynchronous DMA; `ev` marks the last copy that used it, and the buffer
// is rewritten only after that copy has completed.
struct PinBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    PinBuf() = default;
    PinBuf(const PinBuf&) = delete;
    PinBuf& operator=(const PinBuf&) = delete;
    ~PinBuf() {
        (void)wait();
        if (p) (void)hipHostFree(p);
        if (ev) (void)hipEventDestroy(ev);
    }
    hipError_t wait() {
        if (!pending) return hipSuccess;
        pending = false;
        return hipEventSynchronize(ev);
    }
    hipError_t ensure(size_t need) {
        hipError_t e = wait();
        if (e != hipSuccess) return e;
        if (!ev) {
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) { ev = nullptr; return e; }
        }
        if (need <= bytes) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        e = hipHostMalloc(&p, need, hipHostMallocDefault);
        if (e != hipSuccess) { p = nullptr; return e; }
        bytes = need;
        return hipSuccess;
    }
    hipError_t mark(hipStream_t s) {
        const hipError_t e = hipEventRecord(ev, s);
        pending = e == hipSuccess;
        return e;
    }
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    WorkAcct* acct = nullptr;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        if (acct) acct->used -= bytes;
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t need) {
        if (need <= bytes) return hipSuccess;
        if (acct && acct->cap && acct->used - bytes + need > acct->cap) return hipErrorOutOfMemory;
        release();
        hipError_t e = hipMalloc(&p, need);
        if (e != hipSuccess) { p = nullptr; return e; }
        bytes = need;
        if (acct) acct->used += need;
        return hipSuccess;
    }
};

struct CachedPlan {
    EncodedPlan ep;
    DevBuf dev;
    std::shared_ptr<JitModule> jit;
    bool jit_tried = false;
    size_t o_pass = 0, o_phase = 0, o_op = 0, o_form = 0, o_pair = 0, o_etab = 0;
    double plan_ms = 0.0;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

hipError_t upload_plan(CachedPlan& cp, hipStream_t s) {
    const EncodedPlan& e = cp.ep;
    size_t o = 0;
    cp.o_pass = o; o = align_up(o + e.passes.size() * sizeof(DPass), 256);
    cp.o_phase = o; o = align_up(o + e.phases.size() * sizeof(DPhase), 256);
    cp.o_op = o; o = align_up(o + e.ops.size() * sizeof(DOp), 256);
    cp.o_form = o; o = align_up(o + e.forms.size() * sizeof(DForm), 256);
    cp.o_pair = o; o = align_up(o + e.pairs.size() * sizeof(DPair), 256);
    cp.o_etab = o; o = align_up(o + e.etab.size() * sizeof(uint16_t), 256);
    o = std::max<size_t>(o, 256);
    hipError_t er = cp.dev.ensure(o);
    if (er != hipSuccess) return er;
    std::vector<unsigned char> h(o, 0);
    auto cpy = [&](size_t off, const void* src, size_t n) { if (n) std::memcpy(h.data() + off, src, n); };
    cpy(cp.o_pass, e.passes.data(), e.passes.size() * sizeof(DPass));
    cpy(cp.o_phase, e.phases.data(), e.phases.size() * sizeof(DPhase));
    cpy(cp.o_op, e.ops.data(), e.ops.size() * sizeof(DOp));
    cpy(cp.o_form, e.forms.data(), e.forms.size() * sizeof(DForm));
    cpy(cp.o_pair, e.pairs.data(), e.pairs.size() * sizeof(DPair));
    cpy(cp.o_etab, e.etab.data(), e.etab.size() * sizeof(uint16_t));
    er = hipMemcpyAsync(cp.dev.p, h.data(), o, hipMemcpyHostToDevice, s);
    if (er != hipSuccess) return er;
    return hipStreamSynchronize(s);
}

}  // namespace

struct sv_ctx_s {
    int n = 0;
    int dtype = SV_C64;
    int batch = 1;
    void* state = nullptr;
    size_t state_bytes = 0;
    hipStream_t stream = nullptr;
    sv_opts opts{};
    bool known_zero = false;
    bool zero_pending = false;   // |0..0> requested but not yet written
    uint64_t in_mask = 0;        // next sweep: the state is copies of its part with these bits clear
    WorkAcct acct;               // declared before every DevBuf: outlives them
    std::unordered_map<uint64_t, std::unique_ptr<CachedPlan>> cache;
    DevBuf pool, red_part, red_out, pauli, gpart, gout, pinit;
    DevBuf smp_tree, smp_u, smp_out;   // sampling and amplitude readout
    DevBuf npart;                      // FP64 partials: the last pass's norm, the adjoint energy
    DevBuf ppmask;                     // the paper's plan: CZ masks of its diagonal clusters
    sv_ctx_s() {
        for (DevBuf* b : {&pool, &red_part, &red_out, &pauli, &gpart, &gout, &pinit, &smp_tree, &smp_u, &smp_out,
                          &npart, &ppmask})
            b->acct = &acct;
    }
    std::vector<unsigned char> pool_host;
    PinBuf pool_pin[2];   // pool uploads, alternating (the adjoint uploads two per call)
    int pool_pin_i = 0;
    PinBuf out_pin;       // gradient and energy results
    // tile-pass timing (opts.timing)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<double> ev_bytes;
    double t_ms = 0.0, t_bytes = 0.0;
    int64_t t_count = 0;
    ~sv_ctx_s() {
        for (auto& e : ev) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    }
};

namespace {

size_t amp_bytes(int dtype) { return dtype == SV_C64 ? 8 : 16; }

PlanCfg cfg_for(const sv_ctx_s* c, bool two) {
    PlanCfg p;
    p.dtype = c->dtype;
    const bool c64 = c->dtype == SV_C64;
    int T = c->opts.tile_bits > 0 ? c->opts.tile_bits : (c64 ? (two ? 12 : 13) : (two ? 11 : 12));
    T = std::max(4, std::min(T, kMaxTileBits));
    if (!c64 && T > 13) T = 13;
    p.T = T;
    // 2^L contiguous amplitudes per tile segment: 128 B (c64) or 256 B (c128)
    int L = c->opts.low_bits > 0 ? c->opts.low_bits : 4;
    L = std::max(1, std::min(L, T - 1));
    if (T - L > kMaxHigh) L = T - kMaxHigh;
    p.L = L;
    int nt = c->opts.threads > 0 ? c->opts.threads : ((c64 && !two) ? 512 : 256);
    nt = nt >= 512 ? 512 : 256;
    if (!c64 && two) nt = 256;
    p.nt = nt;
    p.max_fuse_k = c->opts.max_fuse_k > 0 ? c->opts.max_fuse_k : 4;
    p.two = two;
    // complex64 passes are ALU-bound: past 8 a wider search packs more work
    // into fewer passes without saving time; complex128 passes are held by
    // memory, so every pass saved counts
    p.beam = c->opts.plan_beam > 0 ? c->opts.plan_beam : (c64 ? 8 : 16);
    return p;
}

uint64_t opts_key(const sv_ctx_s* c, bool two, bool pinit) {
    uint64_t k = (uint64_t)c->dtype * 1315423911ull;
    k ^= (uint64_t)c->batch * 2654435761ull;
    k ^= ((uint64_t)c->opts.max_fuse_k << 1) ^ ((uint64_t)c->opts.tile_bits << 9) ^
         ((uint64_t)c->opts.low_bits << 17) ^ ((uint64_t)c->opts.plain << 25) ^
         ((uint64_t)c->opts.threads << 27) ^ ((uint64_t)c->opts.structured << 40) ^
         ((uint64_t)two << 42) ^ ((uint64_t)pinit << 43) ^ ((uint64_t)(c->opts.jit + 2) << 45) ^
         ((uint64_t)c->opts.plan_beam << 48);
    return k;
}

bool use_plain(const sv_ctx_s* c) { return c->opts.plain != 0 || c->n < 4; }

// Build (or fetch) the plan for a circuit; builds the IR with the current
// parameters in `ir` and the product-init tables in `pi`.
sv_status get_plan(sv_ctx_s* c, const sv_circuit* circ, const double* params, bool two,
                   std::vector<IRGate>& ir, ProductInit& pi, CachedPlan*& out, double& plan_ms,
                   uint64_t first_pin = 0) {
    BuildOpts bo;
    bo.batch = c->batch;
    bo.structured = c->opts.structured != 0 && !use_plain(c);
    bo.fuse = !use_plain(c);
    bo.fuse_k = use_plain(c) ? 0 : c->opts.max_fuse_k;
    bo.backward = two;
    bo.product_init = !two && !use_plain(c) && c->known_zero && c->opts.product_init != 0;
    try {
        ir = build_ir(circ, params, bo, &pi, c->n);
    } catch (const std::exception& e) {
        return fail(SV_EINVAL, std::string("IR build failed: ") + e.what());
    }
    PlanCfg cfg = cfg_for(c, two);
    cfg.first_pin = two || use_plain(c) ? 0ull : first_pin;
    const uint64_t key = circuit_hash(circ, opts_key(c, two, bo.product_init) ^ ir_signature(ir) ^
                                                (cfg.first_pin * 0x9e3779b97f4a7c15ull));
    auto it = c->cache.find(key);
    plan_ms = 0.0;
    if (it != c->cache.end()) {
        out = it->second.get();
        return SV_OK;
    }
    auto t0 = std::chrono::steady_clock::now();
    auto cp = std::make_unique<CachedPlan>();
    cp->dev.acct = &c->acct;
    try {
        if (use_plain(c)) plan_plain(ir, c->n, cfg, cp->ep);
        else plan_fused(ir, c->n, cfg, cp->ep);
    } catch (const std::exception& e) {
        return fail(SV_EUNSUPPORTED, std::string("planning failed: ") + e.what());
    }
    HIPCHK(upload_plan(*cp, c->stream));
    plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    cp->plan_ms = plan_ms;
    out = cp.get();
    c->cache[key] = std::move(cp);
    return SV_OK;
}

// Plan-specialised kernels for large states, compiled on a plan's first use.
sv_status ensure_jit(sv_ctx_s* c, CachedPlan& cp, bool two) {
    const EncodedPlan& e = cp.ep;
    if (cp.jit_tried || e.passes.empty()) return SV_OK;
    cp.jit_tried = true;
    // auto: specialise when every launch streams >= 2^24 amplitudes, where a
    // few seconds of compilation (cached on disk) pay for themselves
    const bool big = (uint64_t)c->batch << c->n >= (1ull << 24);
    bool eligible = jit_enabled() && c->opts.jit >= 0 && (c->opts.jit > 0 || big);
    // passes with fewer register groups than threads need whole idle waves
    for (const DPass& P : e.passes)
        if ((1u << (P.T - kRegBits)) < (uint32_t)e.cfg.nt && ((1u << (P.T - kRegBits)) % 64u) != 0) eligible = false;
    if (eligible) {
        std::string jerr;
        cp.jit = jit_get(e, c->dtype, two, e.cfg.nt, jerr);
        if (!cp.jit && c->opts.jit > 0) return fail(SV_EDEVICE, "run-time specialisation failed: " + jerr);
    }
    return SV_OK;
}

// Product-state tables for the first tile pass (lo: 2^nlo complex FP64,
// hi: 2^{n-nlo}); the pass computes its input instead of reading psi.
struct InitTables {
    const double* lo = nullptr;
    const double* hi = nullptr;
    uint32_t nlo = 0;
    uint64_t in_mask = 0;   // TileArgs::in_mask of the first pass
};

// Execute a plan on psi (and lambda when `lam` is non-null).  With
// norm_out (device, batch doubles) the call also leaves ||psi_b||^2 there:
// summed by the last pass as it stores its tiles when the plan ends with a
// tile pass, else by a separate reduction.
sv_status run_plan(sv_ctx_s* c, CachedPlan& cp, const std::vector<IRGate>& ir, void* psi, void* lam,
                   double* gout, uint64_t gstride, const InitTables& init = InitTables{},
                   double* norm_out = nullptr) {
    const EncodedPlan& e = cp.ep;
    const int dt = c->dtype;
    const uint64_t bstride = 1ull << c->n;
    const size_t ab = amp_bytes(dt);
    // pool
    fill_pool(e, ir, c->batch, c->pool_host);
    HIPCHK(c->pool.ensure(std::max<size_t>(c->pool_host.size(), 256)));
    {
        PinBuf& pb = c->pool_pin[c->pool_pin_i];
        c->pool_pin_i ^= 1;
        HIPCHK(pb.ensure(std::max<size_t>(c->pool_host.size(), 256)));
        std::memcpy(pb.p, c->pool_host.data(), c->pool_host.size());
        HIPCHK(hipMemcpyAsync(c->pool.p, pb.p, c->pool_host.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(pb.mark(c->stream));
    }
    const uint64_t pool_bstride = e.pool_varies ? e.pool_size : 0;
    const unsigned char* pool = reinterpret_cast<const unsigned char*>(c->pool.p);
    // gradient partials
    if (lam && e.gpart_size) HIPCHK(c->gpart.ensure(e.gpart_size * c->batch * sizeof(double)));
    const unsigned char* plan = reinterpret_cast<const unsigned char*>(cp.dev.p);
    void* states[2] = {psi, lam};
    const int nstates = lam ? 2 : 1;
    {
        sv_status js = ensure_jit(c, cp, lam != nullptr);
        if (js != SV_OK) return js;
    }
    uint64_t gslot = 0;
    const bool norm_in_pass = norm_out && !lam && !e.steps.empty() && e.steps.back().type == ST_TILE;
    uint64_t norm_ntile = 0;
    for (size_t si = 0; si < e.steps.size(); ++si) {
        const Step& st = e.steps[si];
        const bool fused_init = si == 0 && init.lo != nullptr;
        switch (st.type) {
            case ST_TILE: {
                const DPass& P = e.passes[st.pass];
                TileArgs a{};
                if (fused_init) {
                    a.init_lo = init.lo;
                    a.init_hi = init.hi;
                    a.init_nlo = init.nlo;
                }
                if (si == 0) a.in_mask = init.in_mask;
                if (norm_in_pass && si + 1 == e.steps.size()) {
                    norm_ntile = 1ull << (c->n - P.T);
                    HIPCHK(c->npart.ensure((size_t)c->batch * norm_ntile * sizeof(double)));
                    a.norm_part = reinterpret_cast<double*>(c->npart.p);
                }
                a.state = psi;
                a.lam = lam;
                a.pass = reinterpret_cast<const DPass*>(plan + cp.o_pass) + st.pass;
                a.phases = reinterpret_cast<const DPhase*>(plan + cp.o_phase);
                a.ops = reinterpret_cast<const DOp*>(plan + cp.o_op);
                a.forms = reinterpret_cast<const DForm*>(plan + cp.o_form);
                a.pairs = reinterpret_cast<const DPair*>(plan + cp.o_pair);
                a.etab = reinterpret_cast<const uint16_t*>(plan + cp.o_etab);
                a.pool = pool;
                a.pool_bstride = pool_bstride;
                a.state_bstride = bstride;
                a.phase_tab = pool;
                a.gpart = lam ? reinterpret_cast<double*>(c->gpart.p) + P.gpart_off * c->batch : nullptr;
                a.ntile_log2 = (uint32_t)(c->n - (int)P.T);
                a.nthreads = (uint32_t)e.cfg.nt;
                const uint64_t nblocks = (uint64_t)c->batch << (c->n - P.T);
                const size_t lds = tile_lds_bytes(dt, lam != nullptr, P.T, P.nform, P.ngrad, e.cfg.nt);
                if (lds > 160 * 1024) return fail(SV_EUNSUPPORTED, "tile pass needs more LDS than available");
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (c->opts.timing) {
                    HIPCHK(hipEventCreate(&e0));
                    HIPCHK(hipEventCreate(&e1));
                    HIPCHK(hipEventRecord(e0, c->stream));
                }
                if (cp.jit) HIPCHK(jit_launch(*cp.jit, st.pass, a, nblocks, e.cfg.nt, lds, c->stream));
                else HIPCHK(launch_tile_pass(dt, lam != nullptr, e.cfg.nt, a, nblocks, lds, c->stream));
                if (c->opts.timing) {
                    HIPCHK(hipEventRecord(e1, c->stream));
                    c->ev.emplace_back(e0, e1);
                    // a pass with the product-state input only writes
                    c->ev_bytes.push_back((fused_init ? 1.0 : 2.0) * (double)ab * (double)c->batch *
                                          std::ldexp(1.0, c->n) * (lam ? 2.0 : 1.0));
                }
                if (lam && P.ngrad) {
                    HIPCHK(launch_grad_reduce(reinterpret_cast<double*>(c->gpart.p) + P.gpart_off * c->batch,
                                              c->batch, 1ull << (c->n - P.T), P.ngrad, gout + gslot, gstride,
                                              c->stream));
                    gslot += P.ngrad;
                }
                break;
            }
            case ST_DENSE:
                for (int s = 0; s < nstates; ++s)
                    HIPCHK(launch_dense_plain(dt, states[s], bstride, c->batch, c->n, st.k, st.tq,
                                              pool + e.recipes[st.recipe].off * ab, pool_bstride, c->stream));
                break;
            case ST_MASKED:
                for (int s = 0; s < nstates; ++s)
                    HIPCHK(launch_masked_phase(dt, states[s], bstride, c->batch, c->n, st.mask, st.mode,
                                               st.recipe >= 0 ? pool + e.recipes[st.recipe].off * ab : nullptr,
                                               pool_bstride, c->stream));
                break;
            case ST_DIAG:
                for (int s = 0; s < nstates; ++s)
                    HIPCHK(launch_diag_plain(dt, states[s], bstride, c->batch, c->n, st.k, st.tq,
                                             pool + e.recipes[st.recipe].off * ab, pool_bstride, c->stream));
                break;
            case ST_SWAP:
                for (int s = 0; s < nstates; ++s)
                    HIPCHK(launch_pair_swap(dt, states[s], bstride, c->batch, c->n, st.mask, st.ones, st.flip,
                                            st.mode, c->stream));
                break;
            case ST_GRAD: {
                if (!lam) break;
                HIPCHK(c->red_part.ensure(reduce_partials_size(c->n, c->batch) * sizeof(double)));
                HIPCHK(launch_reduce(dt, 3, psi, lam, bstride, c->batch, c->n, nullptr, st.mode, st.mask,
                                     reinterpret_cast<double*>(c->red_part.p), gout + st.slot, gstride, c->stream));
                break;
            }
            default:
                return fail(SV_EUNSUPPORTED, "unknown plan step");
        }
    }
    if (norm_out) {
        if (norm_in_pass) {
            HIPCHK(launch_grad_reduce(reinterpret_cast<double*>(c->npart.p), c->batch, norm_ntile, 1, norm_out, 1,
                                      c->stream));
        } else {
            HIPCHK(c->red_part.ensure(reduce_partials_size(c->n, c->batch) * sizeof(double)));
            HIPCHK(launch_reduce(dt, 0, psi, nullptr, bstride, c->batch, c->n, nullptr, 0, 0,
                                 reinterpret_cast<double*>(c->red_part.p), norm_out, 1, c->stream));
        }
    }
    return SV_OK;
}

void fill_stats(sv_stats* st, const sv_ctx_s* c, const CachedPlan& cp, const sv_circuit* circ, double plan_ms,
                int folded, bool init_used, bool init_fused = false) {
    if (!st) return;
    std::memset(st, 0, sizeof(*st));
    const EncodedPlan& e = cp.ep;
    st->gates_in = circ->n_gates;
    st->passes = e.n_tile + e.n_plain + (int)e.steps.size() - e.n_tile - e.n_plain;
    st->phases = e.n_phase;
    st->dense_ops = e.n_dense;
    st->diag_ops = e.n_diag;
    st->launches = (int)e.steps.size() + (init_used && !init_fused ? 1 : 0);
    st->folded_init = folded;
    st->plan_ms = plan_ms;
    const double N = std::ldexp(1.0, c->n) * c->batch;
    const double ab = (double)amp_bytes(c->dtype);
    double bytes = 0.0;
    for (const Step& s : e.steps) {
        if (s.type == ST_TILE || s.type == ST_DENSE || s.type == ST_DIAG || s.type == ST_SWAP)
            bytes += 2.0 * N * ab * (s.type == ST_SWAP ? std::ldexp(1.0, -__builtin_popcountll(s.mask | s.ones)) * 2 : 1.0);
        else if (s.type == ST_MASKED)
            bytes += 2.0 * N * ab * std::ldexp(1.0, -__builtin_popcountll(s.mask));
    }
    if (init_used && !init_fused) bytes += N * ab;     // the product state written
    if (init_fused) bytes -= N * ab;                   // the first pass reads nothing
    st->hbm_bytes = bytes;
    st->flops = e.flops * c->batch;
    st->alu_ops = e.alu_ops * c->batch;
    // the fused product-state input: a complex FP64 product (4 instructions)
    // and its rounding (2) per amplitude
    if (init_fused) st->alu_ops += 6.0 * N;
}

// Pauli tables in the device layout: distinct x masks, the first term of
// each x group, then per term the z mask, coefficient and i^{|x&z|} exponent.
struct PauliPack {
    std::vector<unsigned char> buf;
    size_t ox = 0, og = 0, oz = 0, oc = 0, oph = 0;
    size_t ogm = 0, ohz = 0, ohc = 0, ohm = 0;   // tiled lambda = H psi tables (hpsi)
    bool hpsi = false;
    uint32_t ng = 0;
};

// hpsi: also the tables of the tiled lambda = H psi kernel.
sv_status pack_pauli(const sv_ctx_s* c, const sv_pauli_sum* h, PauliPack& pk, bool hpsi = false) {
    if (!h || h->n_terms < 0) return fail(SV_EINVAL, "observable is NULL or has n_terms < 0");
    if (h->n_terms > 0 && (!h->coeff || !h->x_mask || !h->z_mask)) return fail(SV_EINVAL, "observable arrays are NULL");
    const uint64_t qm = c->n >= 64 ? ~0ull : ((1ull << c->n) - 1ull);
    std::vector<uint64_t> xs;
    std::vector<std::vector<int>> grp;
    for (int t = 0; t < h->n_terms; ++t) {
        if ((h->x_mask[t] | h->z_mask[t]) & ~qm) return fail(SV_EINVAL, "Pauli term acts outside the register");
        if (!std::isfinite(h->coeff[t])) return fail(SV_EINVAL, "non-finite Pauli coefficient");
        size_t g = 0;
        for (; g < xs.size(); ++g) if (xs[g] == h->x_mask[t]) break;
        if (g == xs.size()) { xs.push_back(h->x_mask[t]); grp.emplace_back(); }
        grp[g].push_back(t);
    }
    const size_t ng = xs.size();
    const size_t nt = (size_t)h->n_terms;
    std::vector<uint64_t> z;
    std::vector<double> cf;
    std::vector<uint32_t> ph, g0;
    for (size_t g = 0; g < ng; ++g) {
        g0.push_back((uint32_t)z.size());
        for (int t : grp[g]) {
            z.push_back(h->z_mask[t]);
            cf.push_back(h->coeff[t]);
            ph.push_back((uint32_t)(__builtin_popcountll(h->x_mask[t] & h->z_mask[t]) & 3));
        }
    }
    g0.push_back((uint32_t)z.size());
    // tiled-kernel order: per group the even-exponent terms, then the odd
    std::vector<uint32_t> gm, hm;
    std::vector<uint64_t> hz;
    std::vector<double> hc;
    if (hpsi) {
        for (size_t g = 0; g < ng; ++g) {
            for (int odd = 0; odd < 2; ++odd) {
                if (odd) gm.push_back((uint32_t)hz.size());
                for (uint32_t t = g0[g]; t < g0[g + 1]; ++t) {
                    if ((int)(ph[t] & 1) != odd) continue;
                    hz.push_back(z[t]);
                    hc.push_back(ph[t] >= 2 ? -cf[t] : cf[t]);
                    uint32_t m = 0;
                    for (uint32_t k = 0; k < 8; ++k)
                        m |= (uint32_t)(__builtin_popcountll((z[t] >> 8) & 7ull & k) & 1) << k;
                    hm.push_back(m);
                }
            }
        }
    }
    pk.hpsi = hpsi;
    pk.ox = 0;
    pk.og = align_up(pk.ox + ng * 8, 64);
    pk.oz = align_up(pk.og + (ng + 1) * 4, 64);
    pk.oc = align_up(pk.oz + nt * 8, 64);
    pk.oph = align_up(pk.oc + nt * 8, 64);
    size_t end = pk.oph + nt * 4;
    if (hpsi) {
        pk.ogm = align_up(end, 64);
        pk.ohz = align_up(pk.ogm + ng * 4, 64);
        pk.ohc = align_up(pk.ohz + nt * 8, 64);
        pk.ohm = align_up(pk.ohc + nt * 8, 64);
        end = pk.ohm + nt * 4;
    }
    const size_t tot = align_up(end + 64, 64);
    pk.buf.assign(tot, 0);
    std::memcpy(pk.buf.data() + pk.ox, xs.data(), ng * 8);
    std::memcpy(pk.buf.data() + pk.og, g0.data(), (ng + 1) * 4);
    std::memcpy(pk.buf.data() + pk.oz, z.data(), nt * 8);
    std::memcpy(pk.buf.data() + pk.oc, cf.data(), nt * 8);
    std::memcpy(pk.buf.data() + pk.oph, ph.data(), nt * 4);
    if (hpsi) {
        std::memcpy(pk.buf.data() + pk.ogm, gm.data(), ng * 4);
        std::memcpy(pk.buf.data() + pk.ohz, hz.data(), nt * 8);
        std::memcpy(pk.buf.data() + pk.ohc, hc.data(), nt * 8);
        std::memcpy(pk.buf.data() + pk.ohm, hm.data(), nt * 4);
    }
    pk.ng = (uint32_t)ng;
    return SV_OK;
}

// Device view of packed tables copied to d.
PauliDev pauli_at(const PauliPack& pk, unsigned char* d) {
    PauliDev pd{};
    pd.x = reinterpret_cast<const uint64_t*>(d + pk.ox);
    pd.g0 = reinterpret_cast<const uint32_t*>(d + pk.og);
    pd.z = reinterpret_cast<const uint64_t*>(d + pk.oz);
    pd.c = reinterpret_cast<const double*>(d + pk.oc);
    pd.ph = reinterpret_cast<const uint32_t*>(d + pk.oph);
    pd.ngroup = pk.ng;
    if (pk.hpsi) {
        pd.gm = reinterpret_cast<const uint32_t*>(d + pk.ogm);
        pd.hz = reinterpret_cast<const uint64_t*>(d + pk.ohz);
        pd.hc = reinterpret_cast<const double*>(d + pk.ohc);
        pd.hm = reinterpret_cast<const uint32_t*>(d + pk.ohm);
    }
    return pd;
}

sv_status upload_pauli(sv_ctx_s* c, const sv_pauli_sum* h, PauliDev& pd, bool hpsi = false) {
    PauliPack pk;
    sv_status st = pack_pauli(c, h, pk, hpsi);
    if (st != SV_OK) return st;
    HIPCHK(c->pauli.ensure(pk.buf.size()));
    HIPCHK(hipMemcpyAsync(c->pauli.p, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    pd = pauli_at(pk, reinterpret_cast<unsigned char*>(c->pauli.p));
    return SV_OK;
}

// Write a pending |0...0> (sv_init(ZERO) is deferred so that a following
// product-state initialisation does not stream the state twice).
sv_status write_input_copy(sv_ctx_s* c, sv_stats* stats);

sv_status materialise(sv_ctx_s* c) {
    if (c->in_mask) {
        sv_status st = write_input_copy(c, nullptr);
        if (st != SV_OK) return st;
    }
    if (!c->zero_pending) return SV_OK;
    HIPCHK(launch_init(c->dtype, c->state, 1ull << c->n, c->batch, c->n, 1, 0, 0.0, c->stream));
    c->zero_pending = false;
    return SV_OK;
}

// The paper's own plan (opts.paper): kind clusters, one memory pass per
// diagonal cluster and per pair of one-qubit gates, the scale and phase of
// the unnormalised factors kept as counters and folded back by rescale
// passes; gates of no cluster kind run gate by gate.
sv_status apply_paper(sv_ctx_s* c, const sv_circuit* circ, const double* params, sv_stats* stats,
                      double* norm_out) {
    auto t0 = std::chrono::steady_clock::now();
    const PaperPlan pp = paper_plan(circ);
    const int n = c->n;
    const uint64_t bs = 1ull << n;
    const double pass_bytes = 2.0 * (double)bs * (double)amp_bytes(c->dtype) * c->batch;
    sv_stats acc{};
    acc.gates_in = circ->n_gates;
    // CZ masks of every diagonal cluster: one-sided, then symmetric
    std::vector<uint64_t> masks;
    std::vector<size_t> moff;
    for (const PStep& st : pp.steps) {
        if (st.type != PS_DIAG) continue;
        moff.push_back(masks.size());
        std::vector<uint64_t> sym((size_t)n, 0);
        for (int k = 0; k < n; ++k)
            for (int l = 0; l < k; ++l)
                if ((st.cz[(size_t)k] >> l) & 1) { sym[(size_t)k] |= 1ull << l; sym[(size_t)l] |= 1ull << k; }
        masks.insert(masks.end(), st.cz.begin(), st.cz.end());
        masks.insert(masks.end(), sym.begin(), sym.end());
    }
    if (!masks.empty()) {
        HIPCHK(c->ppmask.ensure(masks.size() * sizeof(uint64_t)));
        HIPCHK(hipMemcpyAsync(c->ppmask.p, masks.data(), masks.size() * sizeof(uint64_t), hipMemcpyHostToDevice,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    acc.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    const uint64_t* dmask = reinterpret_cast<const uint64_t*>(c->ppmask.p);
    size_t si = 0, di = 0;
    // a first H layer on every qubit of a deferred |0..0> is the uniform state
    // (the paper's footnote on the initial Hadamard layer)
    if (c->zero_pending && !pp.steps.empty() && pp.steps[0].type == PS_LAYER && pp.steps[0].kind == SV_OP_H &&
        (int)pp.steps[0].layer.size() == n) {
        const double v = std::ldexp(1.0, -n / 2) * ((n & 1) ? std::sqrt(0.5) : 1.0);
        HIPCHK(launch_init(c->dtype, c->state, bs, c->batch, n, 2, 0, v, c->stream));
        acc.hbm_bytes += pass_bytes / 2;
        acc.launches += 1;
        acc.folded_init = n;
        si = 1;
    } else {
        sv_status ms = materialise(c);
        if (ms != SV_OK) return ms;
    }
    c->zero_pending = false;
    c->known_zero = false;
    int p = 0, s8 = 0;     // pending (1/sqrt(2))^p and w^s8
    auto rescale = [&](bool final) -> sv_status {
        if (p == 0 && (s8 & 7) == 0) return SV_OK;
        if (!final && p <= 100) return SV_OK;
        double re = std::ldexp(1.0, -(p / 2)) * ((p & 1) ? std::sqrt(0.5) : 1.0), im = 0.0;
        if (final && (s8 & 7)) {
            const double a = M_PI / 4 * (s8 & 7);
            im = re * std::sin(a);
            re = re * std::cos(a);
            s8 = 0;
        }
        p = 0;
        HIPCHK(launch_pp_scale(c->dtype, c->state, bs, c->batch, n, re, im, c->stream));
        acc.passes += 1;
        acc.launches += 1;
        acc.hbm_bytes += pass_bytes;
        return SV_OK;
    };
    const int C = std::min(n, c->dtype == SV_C64 ? 12 : 11);
    for (size_t k = si; k < pp.steps.size(); ++k) {
        const PStep& st = pp.steps[k];
        if (st.type == PS_DIAG) {
            const uint64_t* m1 = dmask + moff[di];
            HIPCHK(launch_pp_diag(c->dtype, c->state, bs, c->batch, n, st.e8, m1, m1 + n, c->stream));
            ++di;
            acc.passes += 1;
            acc.launches += 1;
            acc.diag_ops += (int)st.gates.size();
            acc.hbm_bytes += pass_bytes;
            continue;
        }
        if (st.type == PS_LAYER) {
            // pairs in qubit order, so that paired gates act on close qubits
            std::vector<std::array<int, 4>> ops;   // (qa, ga, qb, gb), gb < 0: single
            for (size_t i = 0; i < st.layer.size(); i += 2) {
                const auto& a = st.layer[i];
                if (i + 1 < st.layer.size()) ops.push_back({a.first, a.second, st.layer[i + 1].first, st.layer[i + 1].second});
                else ops.push_back({a.first, a.second, -1, -1});
                p += pg_scale_pow(a.second);
                s8 += pg_phase8(a.second);
                if (i + 1 < st.layer.size()) {
                    p += pg_scale_pow(st.layer[i + 1].second) - (pg_pair_even(a.second, st.layer[i + 1].second) ? 2 : 0);
                    s8 += pg_phase8(st.layer[i + 1].second);
                }
            }
            std::vector<std::array<int, 4>> low;
            if (c->opts.paper == 2 && C >= 2) {
                // recursive transform: high pairs over the whole state, most
                // significant first, then the low ones chunk by chunk
                std::vector<std::array<int, 4>> high;
                for (const auto& o : ops) (std::max(o[0], o[2]) >= C ? high : low).push_back(o);
                std::reverse(high.begin(), high.end());
                ops = high;
            }
            for (const auto& o : ops) {
                HIPCHK(launch_pp_pair(c->dtype, c->state, bs, c->batch, n, o[0], o[1], o[2], o[3], c->stream));
                acc.passes += 1;
                acc.launches += 1;
                acc.hbm_bytes += pass_bytes;
            }
            for (size_t b0 = 0; b0 < low.size(); b0 += 32) {
                const size_t cnt = std::min<size_t>(32, low.size() - b0);
                std::vector<int> qa(cnt), ga(cnt), qb(cnt), gb(cnt);
                for (size_t i = 0; i < cnt; ++i) {
                    qa[i] = low[b0 + i][0]; ga[i] = low[b0 + i][1]; qb[i] = low[b0 + i][2]; gb[i] = low[b0 + i][3];
                }
                HIPCHK(launch_pp_chunk(c->dtype, c->state, bs, c->batch, n, C, (int)cnt, qa.data(), ga.data(),
                                       qb.data(), gb.data(), c->stream));
                acc.passes += 1;
                acc.launches += 1;
                acc.hbm_bytes += pass_bytes;
            }
            acc.dense_ops += (int)st.gates.size();
            sv_status rs = rescale(false);
            if (rs != SV_OK) return rs;
            continue;
        }
        // gates of no cluster kind, one kernel per gate
        std::vector<sv_gate> sub;
        for (int gi : st.gates) sub.push_back(circ->gates[gi]);
        sv_circuit sc = *circ;
        sc.n_gates = (int32_t)sub.size();
        sc.gates = sub.data();
        const int32_t plain0 = c->opts.plain;
        c->opts.plain = 1;
        std::vector<IRGate> ir;
        ProductInit pi;
        CachedPlan* cp = nullptr;
        double pms = 0.0;
        sv_status gs = get_plan(c, &sc, params, false, ir, pi, cp, pms);
        if (gs == SV_OK) gs = run_plan(c, *cp, ir, c->state, nullptr, nullptr, 0);
        c->opts.plain = plain0;
        if (gs != SV_OK) return gs;
        acc.passes += (int)cp->ep.steps.size();
        acc.launches += (int)cp->ep.steps.size();
        acc.hbm_bytes += pass_bytes * (double)cp->ep.steps.size();
        acc.plan_ms += pms;
    }
    {
        sv_status rs = rescale(true);
        if (rs != SV_OK) return rs;
    }
    if (norm_out) {
        HIPCHK(c->red_part.ensure(reduce_partials_size(n, c->batch) * sizeof(double)));
        HIPCHK(launch_reduce(c->dtype, 0, c->state, nullptr, bs, c->batch, n, nullptr, 0, 0,
                             reinterpret_cast<double*>(c->red_part.p), norm_out, 1, c->stream));
    }
    if (stats) *stats = acc;
    return SV_OK;
}

// Write the copies that c->in_mask stands for (the part with the mask's bit
// clear into the part with it set; one bit).
// The launches and algorithmic bytes of the copies are added to `stats`
// when it is given.
sv_status write_input_copy(sv_ctx_s* c, sv_stats* stats = nullptr) {
    const uint64_t m = c->in_mask;
    c->in_mask = 0;
    if (!m) return SV_OK;
    const size_t half = (size_t)m * amp_bytes(c->dtype);
    for (int b = 0; b < c->batch; ++b) {
        unsigned char* st = reinterpret_cast<unsigned char*>(c->state) + (size_t)b * (c->state_bytes / c->batch);
        HIPCHK(launch_copy(st, st + half, half, c->stream));
    }
    if (stats) {
        stats->launches += c->batch;
        stats->hbm_bytes += 2.0 * (double)half * (double)c->batch;
    }
    return SV_OK;
}

sv_status apply_internal(sv_ctx_s* c, const sv_circuit* circ, const double* params, sv_stats* stats,
                         double* norm_out = nullptr) {
    sv_stats copies{};   // a pending input copy written before the sweep
    auto add_copies = [&]() {
        if (!stats) return;
        stats->launches += copies.launches;
        stats->hbm_bytes += copies.hbm_bytes;
    };
    if (c->opts.paper) {
        sv_status ws = write_input_copy(c, &copies);
        if (ws != SV_OK) return ws;
        ws = apply_paper(c, circ, params, stats, norm_out);
        if (ws == SV_OK) add_copies();
        return ws;
    }
    std::vector<IRGate> ir;
    ProductInit pi;
    CachedPlan* cp = nullptr;
    double plan_ms = 0.0;
    sv_status st = get_plan(c, circ, params, false, ir, pi, cp, plan_ms, c->in_mask);
    if (st != SV_OK) return st;
    // a pending input copy is read by the first pass when that pass is a tile
    // pass with the copy's bit among its local bits (then every tile reads only
    // amplitudes it writes); otherwise it is written first
    uint64_t in_mask = 0;
    if (c->in_mask) {
        const EncodedPlan& e = cp->ep;
        bool fused = !pi.used && !e.steps.empty() && e.steps.front().type == ST_TILE;
        if (fused) {
            const DPass& P0 = e.passes[e.steps.front().pass];
            uint64_t local = (1ull << P0.L) - 1ull;
            for (uint32_t t = 0; t < P0.H; ++t) local |= 1ull << P0.hpos[t];
            fused = (c->in_mask & ~local) == 0;
        }
        if (fused) {
            in_mask = c->in_mask;
            c->in_mask = 0;
        } else {
            st = write_input_copy(c, &copies);
            if (st != SV_OK) return st;
        }
    }
    if (!pi.used) {
        st = materialise(c);
        if (st != SV_OK) return st;
    }
    c->zero_pending = false;
    InitTables init;
    bool init_fused = false;
    if (pi.used) {
        const size_t nlo = pi.lo.size(), nhi = pi.hi.size();
        HIPCHK(c->pinit.ensure((nlo + nhi) * 16));
        HIPCHK(hipMemcpyAsync(c->pinit.p, pi.lo.data(), nlo * 16, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(reinterpret_cast<unsigned char*>(c->pinit.p) + nlo * 16, pi.hi.data(), nhi * 16,
                              hipMemcpyHostToDevice, c->stream));
        const double* lo = reinterpret_cast<const double*>(c->pinit.p);
        // a first step that is a tile pass computes the product state as its
        // input; otherwise the state is written first
        init_fused = !cp->ep.steps.empty() && cp->ep.steps.front().type == ST_TILE && pi.nlo >= 1;
        if (init_fused) {
            init.lo = lo;
            init.hi = lo + 2 * nlo;
            init.nlo = (uint32_t)pi.nlo;
        } else {
            HIPCHK(launch_init_product(c->dtype, c->state, 1ull << c->n, c->batch, c->n, pi.nlo, lo, lo + 2 * nlo,
                                       c->stream));
        }
    }
    init.in_mask = in_mask;
    st = run_plan(c, *cp, ir, c->state, nullptr, nullptr, 0, init, norm_out);
    if (st != SV_OK) return st;
    c->known_zero = false;
    fill_stats(stats, c, *cp, circ, plan_ms, pi.folded, pi.used, init_fused);
    add_copies();
    return SV_OK;
}

}  // namespace

namespace svmi {

sv_status sf_fail(sv_status st, const std::string& msg) { return fail(st, msg); }

// The next sweep of c starts from copies of the state's part with its top
// qubit `bit` clear (the part with it set is not read): the Schroedinger-Feynman
// doubling of a half state at a path bit, left to the sweep's first pass
// when it can read it.  Any other use of the state writes the copy first.
sv_status set_input_copy(sv_ctx c, int bit) {
    if (!c || bit != c->n - 1) return fail(SV_EINVAL, "set_input_copy: bad context or bit (the top qubit only)");
    if (c->in_mask) {
        sv_status st = write_input_copy(c);
        if (st != SV_OK) return st;
    }
    c->in_mask = 1ull << bit;
    c->zero_pending = false;
    c->known_zero = false;
    return SV_OK;
}

// Plan (and compile, where specialised kernels apply) the forward sweep of
// `circ` on context c without launching it, so that the plans of many
// contexts can be prepared from several host threads before they run.
// `first_pin`: qubits the first tile pass holds locally (the qubit of a
// doubling that the sweep will read, as set_input_copy leaves it; 0: none).
sv_status prepare_apply(sv_ctx c, const sv_circuit* circ, const double* params, uint64_t first_pin) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    std::string v = validate_circuit(circ, c->n);
    if (!v.empty()) return fail(SV_EINVAL, v);
    std::vector<IRGate> ir;
    ProductInit pi;
    CachedPlan* cp = nullptr;
    double plan_ms = 0.0;
    sv_status st = get_plan(c, circ, params, false, ir, pi, cp, plan_ms, first_pin);
    if (st != SV_OK) return st;
    return ensure_jit(c, *cp, false);
}

}  // namespace svmi

extern "C" {

void sv_opts_default(sv_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_fuse_k = 4;
    o->product_init = 1;
    o->structured = 1;
}

const char* sv_last_error(void) { return g_err.c_str(); }
const char* sv_version(void) { return "svmi 0.1 (gfx950)"; }

sv_status sv_create(sv_ctx* out, int32_t n, sv_dtype dt, int32_t batch, void* d_state, size_t state_bytes,
                    void* hip_stream, const sv_opts* opts) {
    g_err.clear();
    if (!out) return fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    if (dt != SV_C64 && dt != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    const int nmax = dt == SV_C64 ? 34 : 33;
    if (n < 1 || n > nmax) {
        std::ostringstream s;
        s << "n_qubits " << n << " out of range [1," << nmax << "]";
        return fail(SV_EINVAL, s.str());
    }
    if (batch < 1 || batch > 65535) return fail(SV_EINVAL, "batch must be in [1, 65535]");
    if (!d_state) return fail(SV_EINVAL, "d_state is NULL");
    const size_t ab = amp_bytes(dt);
    if ((uintptr_t)d_state % 16 != 0) return fail(SV_EINVAL, "d_state must be 16-byte aligned");
    const size_t need = (size_t)batch * ((size_t)1 << n) * ab;
    if (state_bytes != need) {
        std::ostringstream s;
        s << "state_bytes " << state_bytes << " != batch * 2^n * " << ab << " = " << need;
        return fail(SV_EINVAL, s.str());
    }
    auto c = new (std::nothrow) sv_ctx_s();
    if (!c) return fail(SV_ENOMEM, "context allocation failed");
    c->n = n;
    c->dtype = dt;
    c->batch = batch;
    c->state = d_state;
    c->state_bytes = state_bytes;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (opts) c->opts = *opts; else sv_opts_default(&c->opts);
    if (c->opts.max_work_mib < 0) { delete c; return fail(SV_EINVAL, "max_work_mib must be >= 0"); }
    if (c->opts.paper < 0 || c->opts.paper > 2) { delete c; return fail(SV_EINVAL, "paper must be 0, 1 or 2"); }
    c->acct.cap = (size_t)c->opts.max_work_mib << 20;
    if (c->opts.max_fuse_k < 0 || c->opts.max_fuse_k > 6) { delete c; return fail(SV_EINVAL, "max_fuse_k must be 0..6"); }
    if (c->opts.tile_bits < 0 || c->opts.tile_bits > kMaxTileBits) { delete c; return fail(SV_EINVAL, "tile_bits must be 0..14"); }
    if (c->opts.plan_beam < 0 || c->opts.plan_beam > 64) { delete c; return fail(SV_EINVAL, "plan_beam must be 0..64"); }
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [] { attr_err = tile_pass_set_attrs(160 * 1024); });
    if (attr_err != hipSuccess) {
        delete c;
        return fail(SV_EDEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(attr_err));
    }
    *out = c;
    return SV_OK;
}

sv_status sv_destroy(sv_ctx c) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    (void)hipStreamSynchronize(c->stream);
    delete c;
    return SV_OK;
}

sv_status sv_set_stream(sv_ctx c, void* s) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    c->stream = reinterpret_cast<hipStream_t>(s);
    return SV_OK;
}

sv_status sv_set_opts(sv_ctx c, const sv_opts* o) {
    if (!c || !o) return fail(SV_EINVAL, "ctx or opts is NULL");
    if (o->max_fuse_k < 0 || o->max_fuse_k > 6) return fail(SV_EINVAL, "max_fuse_k must be 0..6");
    if (o->tile_bits < 0 || o->tile_bits > kMaxTileBits) return fail(SV_EINVAL, "tile_bits must be 0..14");
    if (o->plan_beam < 0 || o->plan_beam > 64) return fail(SV_EINVAL, "plan_beam must be 0..64");
    if (o->max_work_mib < 0) return fail(SV_EINVAL, "max_work_mib must be >= 0");
    if (o->paper < 0 || o->paper > 2) return fail(SV_EINVAL, "paper must be 0, 1 or 2");
    c->opts = *o;
    c->cache.clear();
    c->acct.cap = (size_t)o->max_work_mib << 20;
    return SV_OK;
}

sv_status sv_init(sv_ctx c, int32_t kind, uint64_t basis_index) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    if (kind != SV_INIT_ZERO && kind != SV_INIT_BASIS && kind != SV_INIT_UNIFORM && kind != SV_INIT_ZERO_DEFERRED)
        return fail(SV_EINVAL, "unknown init kind");
    if (kind == SV_INIT_BASIS && basis_index >= (1ull << c->n)) return fail(SV_EINVAL, "basis index out of range");
    c->in_mask = 0;   // the state is overwritten
    const double v = kind == SV_INIT_UNIFORM ? std::ldexp(1.0, -c->n / 2) * ((c->n & 1) ? std::sqrt(0.5) : 1.0) : 0.0;
    if (kind == SV_INIT_ZERO_DEFERRED) {
        c->zero_pending = true;
        c->known_zero = true;
        return SV_OK;
    }
    c->zero_pending = false;
    HIPCHK(launch_init(c->dtype, c->state, 1ull << c->n, c->batch, c->n, kind == SV_INIT_UNIFORM ? 2 : 1,
                       kind == SV_INIT_ZERO ? 0 : basis_index, v, c->stream));
    // Only SV_INIT_ZERO_DEFERRED lets the next sweep fold leading gates into
    // a product state computed without reading the buffer: after any other
    // init the buffer is the truth, caller writes to it included.
    c->known_zero = false;
    return SV_OK;
}

sv_status sv_apply_circuit(sv_ctx c, const sv_circuit* circ, const double* params, sv_stats* stats) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    std::string v = validate_circuit(circ, c->n);
    if (!v.empty()) return fail(SV_EINVAL, v);
    bool has_param = false;
    for (int i = 0; i < circ->n_gates; ++i) has_param |= circ->gates[i].param >= 0;
    if (has_param && !params) return fail(SV_EINVAL, "circuit has parameterised gates but params is NULL");
    if (params)
        for (int64_t i = 0; i < (int64_t)c->batch * circ->n_params; ++i)
            if (!std::isfinite(params[i])) return fail(SV_EINVAL, "non-finite parameter");
    return apply_internal(c, circ, params, stats);
}

sv_status sv_apply_circuit_norm(sv_ctx c, const sv_circuit* circ, const double* params, double* norm2_out,
                                sv_stats* stats) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    if (!norm2_out) return fail(SV_EINVAL, "norm2_out is NULL");
    std::string v = validate_circuit(circ, c->n);
    if (!v.empty()) return fail(SV_EINVAL, v);
    bool has_param = false;
    for (int i = 0; i < circ->n_gates; ++i) has_param |= circ->gates[i].param >= 0;
    if (has_param && !params) return fail(SV_EINVAL, "circuit has parameterised gates but params is NULL");
    if (params)
        for (int64_t i = 0; i < (int64_t)c->batch * circ->n_params; ++i)
            if (!std::isfinite(params[i])) return fail(SV_EINVAL, "non-finite parameter");
    HIPCHK(c->red_out.ensure((size_t)c->batch * sizeof(double)));
    double* dnorm = reinterpret_cast<double*>(c->red_out.p);
    sv_status st = apply_internal(c, circ, params, stats, dnorm);
    if (st != SV_OK) return st;
    HIPCHK(hipMemcpyAsync(norm2_out, dnorm, (size_t)c->batch * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return SV_OK;
}

// ---- tile-geometry autotuner
namespace {
std::mutex g_tune_mu;
std::unordered_map<uint64_t, std::array<int32_t, 3>> g_tune;   // key -> (tile_bits, low_bits, threads)

std::string tune_cache_file() {
    const char* d = std::getenv("SVMI_TUNE_CACHE");
    return d && *d ? std::string(d) : std::string("/tmp/svmi-tune.txt");
}
}  // namespace

sv_status sv_tune(sv_ctx c, const sv_circuit* circ, const double* params, sv_opts* chosen, double* best_ms) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    std::string v = validate_circuit(circ, c->n);
    if (!v.empty()) return fail(SV_EINVAL, v);
    if (use_plain(c)) {
        if (chosen) *chosen = c->opts;
        if (best_ms) *best_ms = 0.0;
        return SV_OK;
    }
    const sv_opts base = c->opts;
    uint64_t key = circuit_hash(circ, 0x5a17ull ^ ((uint64_t)c->dtype << 3) ^ ((uint64_t)c->batch << 8) ^
                                          ((uint64_t)c->n << 40) ^ ((uint64_t)base.structured << 50) ^
                                          ((uint64_t)(base.jit + 2) << 52) ^ ((uint64_t)base.max_fuse_k << 56) ^
                                          ((uint64_t)base.plan_beam * 0x9e3779b97f4a7c15ull));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tune.empty()) {   // results of earlier processes
            std::ifstream f(tune_cache_file());
            unsigned long long k;
            int32_t t, l, nt;
            while (f >> k >> t >> l >> nt) g_tune[k] = {t, l, nt};
        }
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            c->opts.tile_bits = it->second[0];
            c->opts.low_bits = it->second[1];
            c->opts.threads = it->second[2];
            if (chosen) *chosen = c->opts;
            if (best_ms) *best_ms = -1.0;
            return SV_OK;
        }
    }
    // candidates around the defaults: 2^T-amplitude tiles that fit two
    // workgroups per CU, segments of 2^L contiguous amplitudes
    const bool c64 = c->dtype == SV_C64;
    std::vector<std::array<int32_t, 3>> cand;
    const int t_hi = c64 ? 13 : 12;
    for (int T = t_hi - 1; T <= t_hi; ++T)
        for (int L = 4; L <= 5; ++L) cand.push_back({T, L, (c64 && T == 13) ? 512 : 256});
    // complex64 also 2^14-amplitude tiles: 128 KiB of LDS, one workgroup
    // per CU, fewer passes
    if (c64 && c->n >= 14)
        for (int L = 4; L <= 5; ++L) cand.push_back({14, L, 512});
    {   // defined values for the timing sweeps
        sv_status is = sv_init(c, SV_INIT_UNIFORM, 0);
        if (is != SV_OK) return is;
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best = 1e300;
    std::array<int32_t, 3> pick = {base.tile_bits, base.low_bits, base.threads};
    sv_status st = SV_OK;
    for (const auto& cd : cand) {
        c->opts = base;
        c->opts.tile_bits = cd[0];
        c->opts.low_bits = cd[1];
        c->opts.threads = cd[2];
        c->opts.timing = 0;
        c->known_zero = false;
        c->zero_pending = false;
        c->in_mask = 0;
        st = apply_internal(c, circ, params, nullptr);   // plans and compiles
        if (st != SV_OK) break;
        if (hipEventRecord(e0, c->stream) != hipSuccess) { st = fail(SV_EDEVICE, "event record failed"); break; }
        st = apply_internal(c, circ, params, nullptr);
        if (st != SV_OK) break;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            st = fail(SV_EDEVICE, "event failed");
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) { best = ms; pick = cd; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->opts = base;
    if (st != SV_OK) return st;
    c->opts.tile_bits = pick[0];
    c->opts.low_bits = pick[1];
    c->opts.threads = pick[2];
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = pick;
        std::ofstream f(tune_cache_file(), std::ios::app);
        if (f) f << (unsigned long long)key << " " << pick[0] << " " << pick[1] << " " << pick[2] << "\n";
    }
    if (chosen) *chosen = c->opts;
    if (best_ms) *best_ms = best;
    return SV_OK;
}

sv_status sv_copy_state(sv_ctx dst, sv_ctx src) {
    if (!dst || !src) return fail(SV_EINVAL, "ctx is NULL");
    if (dst->n != src->n || dst->dtype != src->dtype || dst->batch != src->batch)
        return fail(SV_EINVAL, "contexts differ in width, dtype or batch");
    if (dst == src || dst->state == src->state) return SV_OK;
    const char* lo_d = static_cast<const char*>(dst->state);
    const char* lo_s = static_cast<const char*>(src->state);
    if (lo_d < lo_s + src->state_bytes && lo_s < lo_d + dst->state_bytes)
        return fail(SV_EINVAL, "state buffers overlap");
    if (src->in_mask) {
        sv_status ws = write_input_copy(src);
        if (ws != SV_OK) return ws;
    }
    if (src->stream != dst->stream) HIPCHK(hipStreamSynchronize(src->stream));
    dst->in_mask = 0;
    if (src->zero_pending) {
        // |0..0> not yet written: the copy is deferred the same way
        dst->zero_pending = true;
        dst->known_zero = true;
        return SV_OK;
    }
    HIPCHK(launch_copy(src->state, dst->state, src->state_bytes, dst->stream));
    dst->zero_pending = false;
    dst->known_zero = src->known_zero;
    return SV_OK;
}

sv_status sv_norm(sv_ctx c, double* out) {
    if (!c || !out) return fail(SV_EINVAL, "ctx or out is NULL");
    {
        sv_status ms = materialise(c);
        if (ms != SV_OK) return ms;
    }
    HIPCHK(c->red_part.ensure(reduce_partials_size(c->n, c->batch) * sizeof(double)));
    HIPCHK(c->red_out.ensure((size_t)c->batch * sizeof(double)));
    HIPCHK(launch_reduce(c->dtype, 0, c->state, nullptr, 1ull << c->n, c->batch, c->n, nullptr, 0, 0,
                         reinterpret_cast<double*>(c->red_part.p), reinterpret_cast<double*>(c->red_out.p), 1,
                         c->stream));
    HIPCHK(hipMemcpyAsync(out, c->red_out.p, (size_t)c->batch * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return SV_OK;
}

sv_status sv_expect(sv_ctx c, const sv_pauli_sum* h, double* out) {
    if (!c || !out) return fail(SV_EINVAL, "ctx or out is NULL");
    {
        sv_status ms = materialise(c);
        if (ms != SV_OK) return ms;
    }
    PauliDev pd{};
    sv_status st = upload_pauli(c, h, pd);
    if (st != SV_OK) return st;
    HIPCHK(c->red_part.ensure(reduce_partials_size(c->n, c->batch) * sizeof(double)));
    HIPCHK(c->red_out.ensure((size_t)c->batch * sizeof(double)));
    HIPCHK(launch_reduce(c->dtype, 2, c->state, nullptr, 1ull << c->n, c->batch, c->n, &pd, 0, 0,
                         reinterpret_cast<double*>(c->red_part.p), reinterpret_cast<double*>(c->red_out.p), 1,
                         c->stream));
    HIPCHK(hipMemcpyAsync(out, c->red_out.p, (size_t)c->batch * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return SV_OK;
}

sv_status sv_expect_noalloc(sv_ctx c, const sv_pauli_sum* h, double* out) {
    if (!c || !out) return fail(SV_EINVAL, "ctx or out is NULL");
    PauliPack pk;
    sv_status st = pack_pauli(c, h, pk);
    if (st != SV_OK) return st;
    // fixed work area: Pauli tables, then the block partials, then the results
    const size_t o_part = align_up(pk.buf.size(), 256);
    const size_t n_part = reduce_partials_size(c->n, c->batch);
    const size_t o_out = align_up(o_part + n_part * sizeof(double), 256);
    const size_t need = o_out + (size_t)c->batch * sizeof(double);
    if (need > kStaticScratchBytes) {
        std::ostringstream m;
        m << "sv_expect_noalloc needs " << need << " bytes of its fixed device work area (" << kStaticScratchBytes
          << " bytes): use fewer states or Pauli terms, or sv_expect";
        return fail(SV_EINVAL, m.str());
    }
    void* base = nullptr;
    HIPCHK(static_scratch(&base));
    {
        sv_status ms = materialise(c);
        if (ms != SV_OK) return ms;
    }
    unsigned char* d = reinterpret_cast<unsigned char*>(base);
    HIPCHK(hipMemcpyAsync(d, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice, c->stream));
    const PauliDev pd = pauli_at(pk, d);
    double* part = reinterpret_cast<double*>(d + o_part);
    double* res = reinterpret_cast<double*>(d + o_out);
    HIPCHK(launch_reduce(c->dtype, 2, c->state, nullptr, 1ull << c->n, c->batch, c->n, &pd, 0, 0, part, res, 1,
                         c->stream));
    HIPCHK(hipMemcpyAsync(out, res, (size_t)c->batch * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return SV_OK;
}

// Samples (or read-back amplitudes) per call, over all states: keeps the
// one-wave-per-sample grid within 2^30 workgroups.
constexpr int64_t kMaxSamples = 1ll << 32;

sv_status sv_sample(sv_ctx c, int64_t count, const double* uniforms, uint64_t* out) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    if (count < 0) return fail(SV_EINVAL, "count < 0");
    if (count == 0) return SV_OK;
    if (!uniforms || !out) return fail(SV_EINVAL, "uniforms or out is NULL");
    if (count > kMaxSamples / c->batch) return fail(SV_EINVAL, "batch * count exceeds 2^32 samples per call");
    const size_t total = (size_t)count * (size_t)c->batch;
    for (size_t k = 0; k < total; ++k)
        if (!(uniforms[k] >= 0.0 && uniforms[k] < 1.0)) return fail(SV_EINVAL, "uniforms must lie in [0, 1)");
    {
        sv_status ms = materialise(c);
        if (ms != SV_OK) return ms;
    }
    const uint64_t tree = sample_tree_doubles(c->n, c->batch);
    HIPCHK(c->smp_tree.ensure(tree * sizeof(double)));
    HIPCHK(c->smp_u.ensure(total * sizeof(double)));
    HIPCHK(c->smp_out.ensure(total * sizeof(uint64_t)));
    HIPCHK(hipMemcpyAsync(c->smp_u.p, uniforms, total * sizeof(double), hipMemcpyHostToDevice, c->stream));
    double* d_tree = reinterpret_cast<double*>(c->smp_tree.p);
    HIPCHK(launch_sample(c->dtype, c->state, 1ull << c->n, c->batch, c->n, d_tree,
                         reinterpret_cast<const double*>(c->smp_u.p), (uint64_t)count,
                         reinterpret_cast<uint64_t*>(c->smp_out.p), c->stream));
    // the root of every state's tree (the last level) holds its total mass
    std::vector<double> root(c->batch);
    HIPCHK(hipMemcpyAsync(root.data(), d_tree + tree - c->batch, c->batch * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(out, c->smp_out.p, total * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int b = 0; b < c->batch; ++b)
        if (!(root[b] > 0.0) || !std::isfinite(root[b])) return fail(SV_EINVAL, "state has zero or non-finite norm");
    return SV_OK;
}

sv_status sv_amplitudes(sv_ctx c, int64_t count, const uint64_t* indices, double* out) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    if (count < 0) return fail(SV_EINVAL, "count < 0");
    if (count == 0) return SV_OK;
    if (!indices || !out) return fail(SV_EINVAL, "indices or out is NULL");
    if (count > kMaxSamples / c->batch) return fail(SV_EINVAL, "batch * count exceeds 2^32 amplitudes per call");
    for (int64_t k = 0; k < count; ++k)
        if (indices[k] >= (1ull << c->n)) return fail(SV_EINVAL, "amplitude index out of range");
    {
        sv_status ms = materialise(c);
        if (ms != SV_OK) return ms;
    }
    HIPCHK(c->smp_u.ensure((size_t)count * sizeof(uint64_t)));
    HIPCHK(c->smp_out.ensure((size_t)count * c->batch * 2 * sizeof(double)));
    HIPCHK(hipMemcpyAsync(c->smp_u.p, indices, (size_t)count * sizeof(uint64_t), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(launch_gather(c->dtype, c->state, 1ull << c->n, c->batch, reinterpret_cast<const uint64_t*>(c->smp_u.p),
                         (uint64_t)count, reinterpret_cast<double*>(c->smp_out.p), c->stream));
    HIPCHK(hipMemcpyAsync(out, c->smp_out.p, (size_t)count * c->batch * 2 * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return SV_OK;
}

sv_status sv_adjoint_grad(sv_ctx c, const sv_circuit* circ, const double* params, const sv_pauli_sum* h,
                          void* d_scratch, size_t scratch_bytes, double* energy_out, double* grad_out,
                          sv_stats* stats) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    std::string v = validate_circuit(circ, c->n);
    if (!v.empty()) return fail(SV_EINVAL, v);
    if (!d_scratch || scratch_bytes < c->state_bytes) return fail(SV_EINVAL, "scratch must hold batch * 2^n amplitudes");
    if (((uintptr_t)d_scratch % 16) != 0) return fail(SV_EINVAL, "d_scratch must be 16-byte aligned");
    if (!energy_out) return fail(SV_EINVAL, "energy_out is NULL");
    if (circ->n_params > 0 && (!params || !grad_out)) return fail(SV_EINVAL, "params and grad_out are required");
    for (int64_t i = 0; params && i < (int64_t)c->batch * circ->n_params; ++i)
        if (!std::isfinite(params[i])) return fail(SV_EINVAL, "non-finite parameter");
    PauliDev pd{};
    sv_status st = upload_pauli(c, h, pd, true);
    if (st != SV_OK) return st;
    // forward sweep (folds leading one-qubit gates when the state is |0...0>)
    st = apply_internal(c, circ, params, stats);
    if (st != SV_OK) return st;
    // lambda = H psi; the same kernel leaves the block partials of the
    // energy Re <psi|lambda>
    const uint64_t hblk = hpsi_blocks(c->n);
    HIPCHK(c->npart.ensure((size_t)c->batch * hblk * sizeof(double)));
    double* epart = reinterpret_cast<double*>(c->npart.p);
    HIPCHK(launch_hpsi(c->dtype, c->state, d_scratch, 1ull << c->n, c->batch, c->n, pd, epart, c->stream));
    // backward plan
    std::vector<IRGate> ir;
    ProductInit pi;
    CachedPlan* cp = nullptr;
    double plan_ms = 0.0;
    st = get_plan(c, circ, params, true, ir, pi, cp, plan_ms);
    if (st != SV_OK) return st;
    const int ns = cp->ep.ngrad_total;
    const size_t gbytes = (size_t)c->batch * (size_t)(ns + 1) * sizeof(double);
    HIPCHK(c->gout.ensure(gbytes));
    double* gdev = reinterpret_cast<double*>(c->gout.p);
    // energy goes in column ns of the (batch x (ns+1)) output block
    HIPCHK(launch_grad_reduce(epart, c->batch, hblk, 1, gdev + ns, (uint64_t)ns + 1, c->stream));
    st = run_plan(c, *cp, ir, c->state, d_scratch, gdev, (uint64_t)ns + 1);
    if (st != SV_OK) return st;
    HIPCHK(c->out_pin.ensure(gbytes));
    HIPCHK(hipMemcpyAsync(c->out_pin.p, gdev, gbytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const double* res = reinterpret_cast<const double*>(c->out_pin.p);
    const int np = circ->n_params;
    for (int b = 0; b < c->batch; ++b) {
        const double* row = res + (size_t)b * (ns + 1);
        energy_out[b] = row[ns];
        if (np > 0) {
            double* g = grad_out + (size_t)b * np;
            for (int p = 0; p < np; ++p) g[p] = 0.0;
            for (int s = 0; s < ns; ++s) g[cp->ep.grad_param[s]] += cp->ep.grad_scale[s] * row[s];
        }
    }
    if (stats) {
        stats->plan_ms += plan_ms;
        stats->alu_ops += cp->ep.alu_ops * c->batch;   // backward sweep
    }
    return SV_OK;
}

sv_status sv_timing(sv_ctx c, double* tile_ms, int64_t* tile_launches, double* tile_bytes) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < c->ev.size(); ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[i].first, c->ev[i].second));
        c->t_ms += ms;
        c->t_bytes += c->ev_bytes[i];
        c->t_count += 1;
        (void)hipEventDestroy(c->ev[i].first);
        (void)hipEventDestroy(c->ev[i].second);
    }
    c->ev.clear();
    c->ev_bytes.clear();
    if (tile_ms) *tile_ms = c->t_ms;
    if (tile_launches) *tile_launches = c->t_count;
    if (tile_bytes) *tile_bytes = c->t_bytes;
    c->t_ms = 0.0;
    c->t_bytes = 0.0;
    c->t_count = 0;
    return SV_OK;
}

sv_status sv_plan_info(const sv_circuit* circ, sv_dtype dtype, int32_t adjoint, const sv_opts* opts,
                       sv_stats* stats) {
    if (!circ || !stats) return fail(SV_EINVAL, "circuit or stats is NULL");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
    std::string v = validate_circuit(circ, circ->n_qubits);
    if (!v.empty()) return fail(SV_EINVAL, v);
    sv_ctx_s c;
    c.n = circ->n_qubits;
    c.dtype = dtype;
    c.batch = 1;
    if (opts) c.opts = *opts; else sv_opts_default(&c.opts);
    if (c.opts.plan_beam < 0 || c.opts.plan_beam > 64) return fail(SV_EINVAL, "plan_beam must be 0..64");
    c.known_zero = !adjoint;
    std::vector<double> params((size_t)std::max(1, circ->n_params), 0.0);
    std::vector<IRGate> ir;
    ProductInit pi;
    BuildOpts bo;
    bo.batch = 1;
    bo.structured = c.opts.structured != 0 && !use_plain(&c);
    bo.fuse = !use_plain(&c);
    bo.fuse_k = use_plain(&c) ? 0 : c.opts.max_fuse_k;
    bo.backward = adjoint != 0;
    bo.product_init = !adjoint && !use_plain(&c) && c.opts.product_init != 0;
    auto t0 = std::chrono::steady_clock::now();
    EncodedPlan ep;
    try {
        ir = build_ir(circ, params.data(), bo, &pi, c.n);
        if (use_plain(&c)) plan_plain(ir, c.n, cfg_for(&c, adjoint != 0), ep);
        else plan_fused(ir, c.n, cfg_for(&c, adjoint != 0), ep);
    } catch (const std::exception& e) {
        return fail(SV_EUNSUPPORTED, std::string("planning failed: ") + e.what());
    }
    CachedPlan cp;
    cp.ep = std::move(ep);
    const double plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (c.opts.jit > 0 && !use_plain(&c)) {
        // compile the specialised kernels too (host only)
        std::string jerr;
        if (!jit_compile_only(cp.ep, dtype, adjoint != 0, cp.ep.cfg.nt, jerr))
            return fail(SV_EUNSUPPORTED, "run-time specialisation failed: " + jerr);
    }
    const bool init_fused = pi.used && !cp.ep.steps.empty() && cp.ep.steps.front().type == ST_TILE && pi.nlo >= 1;
    fill_stats(stats, &c, cp, circ, 0.0, pi.folded, pi.used, init_fused);
    stats->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    stats->reserved = (int32_t)plan_ms;
    return SV_OK;
}

sv_status sv_plan_trace(const sv_circuit* circ, const double* params, sv_dtype dtype, int32_t adjoint,
                        const sv_opts* opts, char* buf, size_t cap, size_t* len) {
    if (!circ || !len) return fail(SV_EINVAL, "circuit or len is NULL");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
    std::string v = validate_circuit(circ, circ->n_qubits);
    if (!v.empty()) return fail(SV_EINVAL, v);
    if (circ->n_params > 0 && !params) return fail(SV_EINVAL, "params is NULL");
    sv_ctx_s c;
    c.n = circ->n_qubits;
    c.dtype = dtype;
    c.batch = 1;
    if (opts) c.opts = *opts; else sv_opts_default(&c.opts);
    if (c.opts.plan_beam < 0 || c.opts.plan_beam > 64) return fail(SV_EINVAL, "plan_beam must be 0..64");
    if (c.opts.paper) {
        // the paper's plan: one line per kind cluster (bitmasks in binary,
        // qubit n-1 first) and the circuit gates it applies, in order
        const std::string tr = paper_trace(paper_plan(circ));
        *len = tr.size();
        if (buf && cap) {
            const size_t m = std::min(cap - 1, tr.size());
            std::memcpy(buf, tr.data(), m);
            buf[m] = '\0';
        }
        return SV_OK;
    }
    if (use_plain(&c)) return fail(SV_EUNSUPPORTED, "the plain path has no fused plan to trace");
    BuildOpts bo;
    bo.batch = 1;
    bo.structured = c.opts.structured != 0;
    bo.fuse = true;
    bo.fuse_k = c.opts.max_fuse_k;
    bo.backward = adjoint != 0;
    bo.product_init = false;
    std::string tr;
    try {
        std::vector<IRGate> ir = build_ir(circ, params, bo, nullptr, c.n);
        EncodedPlan ep;
        plan_fused(ir, c.n, cfg_for(&c, adjoint != 0), ep, &tr);
    } catch (const std::exception& e) {
        return fail(SV_EUNSUPPORTED, std::string("planning failed: ") + e.what());
    }
    *len = tr.size();
    if (buf && cap) {
        const size_t m = std::min(cap - 1, tr.size());
        std::memcpy(buf, tr.data(), m);
        buf[m] = '\0';
    }
    return SV_OK;
}

sv_status sv_sync(sv_ctx c) {
    if (!c) return fail(SV_EINVAL, "ctx is NULL");
    {
        sv_status ms = materialise(c);
        if (ms != SV_OK) return ms;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return SV_OK;
}

sv_status sv_apply_batch(int32_t count, const sv_batch_item* items, sv_dtype dtype, void* hip_stream, int32_t flags,
                         double* energies, double* grads, const sv_opts* opts, sv_stats* stats) {
    g_err.clear();
    std::string err;
    GeomTable tuned;
    const bool use_tuned = opts && opts->batch_tuned &&
                           batch_tuned_table(dtype, (flags & SV_BATCH_GRAD) != 0, tuned);
    sv_status st = run_batch_persistent(count, items, dtype, reinterpret_cast<hipStream_t>(hip_stream), flags,
                                        energies, grads, opts, stats, err, use_tuned ? &tuned : nullptr);
    if (st != SV_OK) {
        (void)hipGetLastError();
        return fail(st, err);
    }
    return SV_OK;
}

sv_status sv_apply_batch_async(int32_t count, const sv_batch_item* items, sv_dtype dtype, void* hip_stream,
                               int32_t flags, const sv_opts* opts, sv_batch_job* job) {
    g_err.clear();
    if (!job) return fail(SV_EINVAL, "job is NULL");
    *job = nullptr;
    std::string err;
    GeomTable tuned;
    const bool use_tuned = opts && opts->batch_tuned &&
                           batch_tuned_table(dtype, (flags & SV_BATCH_GRAD) != 0, tuned);
    void* j = nullptr;
    sv_status st = batch_launch_async(count, items, dtype, reinterpret_cast<hipStream_t>(hip_stream), flags, opts,
                                      err, use_tuned ? &tuned : nullptr, &j);
    if (st != SV_OK) {
        (void)hipGetLastError();
        return fail(st, err);
    }
    *job = reinterpret_cast<sv_batch_job>(j);
    return SV_OK;
}

sv_status sv_batch_finish(sv_batch_job job, double* energies, double* grads, sv_stats* stats) {
    g_err.clear();
    if (!job) return fail(SV_EINVAL, "job is NULL");
    std::string err;
    sv_status st = batch_finish_async(reinterpret_cast<void*>(job), energies, grads, stats, err);
    if (st != SV_OK) {
        (void)hipGetLastError();
        return fail(st, err);
    }
    return SV_OK;
}

sv_status sv_tune_batch(int32_t count, const sv_batch_item* items, sv_dtype dtype, void* hip_stream, int32_t flags,
                        const sv_opts* opts, int32_t* widths_tuned) {
    g_err.clear();
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    std::string err;
    sv_status st = tune_batch(count, items, dtype, reinterpret_cast<hipStream_t>(hip_stream), flags, opts,
                              widths_tuned, err);
    if (st != SV_OK) {
        (void)hipGetLastError();
        return fail(st, err);
    }
    return SV_OK;
}

sv_status sv_batch_tuning(sv_dtype dtype, int32_t grad, int32_t n_qubits, sv_opts* out) {
    if (!out) return fail(SV_EINVAL, "out is NULL");
    BatchGeom g;
    if (!batch_tuned_lookup(dtype, grad != 0, n_qubits, g)) return fail(SV_EINVAL, "width not tuned");
    sv_opts_default(out);
    out->structured = g.structured;
    out->max_fuse_k = g.fuse_k;
    out->tile_bits = g.T;
    out->low_bits = g.L;
    out->batch_tuned = 1;
    return SV_OK;
}

}  // extern "C"
