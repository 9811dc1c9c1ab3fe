// Heterogeneous batches (circuits of different widths).
//
// This translation unit hosts the batch driver; the single-launch persistent
// kernel lives in batch_persistent.hip and is used when the batch qualifies
// (see run_batch_persistent there).  This file provides the per-item
// fallback path that the persistent path is checked against.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <string>
#include <vector>

#include "batch.h"
#include "host.h"
#include "kernels.h"
#include "sv.h"

namespace svmi {

sv_status run_batch_loop(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream,
                         int32_t flags, double* energies, double* grads, const sv_opts* opts, sv_stats* stats,
                         std::string& err) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    size_t goff = 0;
    for (int32_t i = 0; i < count; ++i) {
        const sv_batch_item& it = items[i];
        const int n = it.circuit->n_qubits;
        const size_t bytes = ((size_t)1 << n) * (dtype == SV_C64 ? 8 : 16);
        sv_ctx c = nullptr;
        sv_status st = sv_create(&c, n, dtype, 1, it.d_state, bytes, stream, opts);
        if (st != SV_OK) { err = sv_last_error(); return st; }
        if (flags & SV_BATCH_INIT_ZERO) {
            st = sv_init(c, SV_INIT_ZERO, 0);
            if (st != SV_OK) { err = sv_last_error(); sv_destroy(c); return st; }
        }
        sv_stats s1;
        if (flags & SV_BATCH_GRAD) {
            st = sv_adjoint_grad(c, it.circuit, it.params, it.observable, it.d_lambda, bytes, energies + i,
                                 grads + goff, &s1);
        } else {
            st = sv_apply_circuit(c, it.circuit, it.params, &s1);
            if (st == SV_OK && energies) st = sv_expect(c, it.observable, energies + i);
        }
        if (st != SV_OK) { err = sv_last_error(); sv_destroy(c); return st; }
        sv_destroy(c);
        goff += (size_t)it.circuit->n_params;
        if (stats) {
            stats->gates_in += s1.gates_in;
            stats->passes += s1.passes;
            stats->launches += s1.launches;
            stats->hbm_bytes += s1.hbm_bytes;
            stats->flops += s1.flops;
            stats->alu_ops += s1.alu_ops;
            stats->plan_ms += s1.plan_ms;
        }
    }
    return SV_OK;
}

}  // namespace svmi

namespace svmi {

namespace {

struct PlanKeyed {
    EncodedPlan ep;
};

std::mutex g_plan_mu;
std::unordered_map<uint64_t, std::shared_ptr<PlanKeyed>> g_plans;

// Pinned staging for the plan upload and the device work area of each
// device (plans, pools, queues and reduction scratch), grow-only and shared
// by batch calls; a call holds g_stage_mu from packing until its stream has
// synchronised.  The largest work area of each device stays allocated for
// later calls instead of being allocated and freed around every launch.
std::mutex g_stage_mu;
void* g_stage = nullptr;
size_t g_stage_bytes = 0;
struct DevArea {
    void* p = nullptr;
    size_t bytes = 0;
};
std::unordered_map<int, DevArea> g_dev;   // by device ordinal

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

PlanCfg batch_cfg(int dtype, bool two, int n, const BatchGeom& g) {
    PlanCfg p;
    p.dtype = dtype;
    int T = g.T > 0 ? g.T : (dtype == SV_C64 ? 12 : (two ? 11 : 12));
    if (dtype != SV_C64 && two) T = std::min(T, 12);   // two c128 states per tile: at most 128 KiB of LDS
    p.T = std::min(T, n);
    p.L = std::min(g.L > 0 ? g.L : 4, p.T - 1);   // default: the single-circuit tile geometry
    if (p.T - p.L > kMaxHigh) p.L = p.T - kMaxHigh;
    p.nt = 256;
    p.two = two;
    return p;
}

// Plans are cached by circuit structure, dtype, direction, the IR options
// (structured, fusion width), the tile geometry and the value-dependent
// decisions of the IR.
std::shared_ptr<PlanKeyed> get_batch_plan(const sv_circuit* c, const std::vector<IRGate>& ir, int dtype, bool two,
                                          const BuildOpts& bo, const BatchGeom& g) {
    const PlanCfg cfg = batch_cfg(dtype, two, c->n_qubits, g);
    const uint64_t key = circuit_hash(c, 0x9e3779b97f4a7c15ull ^ ((uint64_t)dtype << 8) ^ ((uint64_t)two << 12) ^
                                             ((uint64_t)bo.structured << 16) ^ ((uint64_t)(uint32_t)bo.fuse_k << 20) ^
                                             ((uint64_t)cfg.T << 28) ^ ((uint64_t)cfg.L << 34) ^ ir_signature(ir));
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plans.find(key);
        if (it != g_plans.end()) return it->second;
    }
    auto pk = std::make_shared<PlanKeyed>();
    plan_fused(ir, c->n_qubits, cfg, pk->ep);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans[key] = pk;
    return pk;
}


struct ItemHost {
    std::vector<IRGate> irf, irb;
    std::shared_ptr<PlanKeyed> pf, pb;
    std::vector<unsigned char> poolf, poolb;
    std::string err;
};

}  // namespace

sv_status run_batch_persistent(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream,
                               int32_t flags, double* energies, double* grads, const sv_opts* opts,
                               sv_stats* stats, std::string& err, const GeomTable* geoms) {
    if (count < 0) { err = "count < 0"; return SV_EINVAL; }
    if (count > 0 && !items) { err = "items is NULL"; return SV_EINVAL; }
    if (dtype != SV_C64 && dtype != SV_C128) { err = "dtype must be SV_C64 or SV_C128"; return SV_EINVAL; }
    const bool grad = (flags & SV_BATCH_GRAD) != 0;
    if (grad && (!energies || !grads)) { err = "energies and grads are required"; return SV_EINVAL; }
    bool small = false;
    for (int32_t i = 0; i < count; ++i) {
        const sv_batch_item& it = items[i];
        if (!it.circuit || !it.d_state) { err = "item " + std::to_string(i) + ": NULL circuit or state"; return SV_EINVAL; }
        std::string v = validate_circuit(it.circuit, it.circuit->n_qubits);
        if (!v.empty()) { err = "item " + std::to_string(i) + ": " + v; return SV_EINVAL; }
        const int nmax = dtype == SV_C64 ? 34 : 33;
        if (it.circuit->n_qubits < 1 || it.circuit->n_qubits > nmax) { err = "item " + std::to_string(i) + ": bad width"; return SV_EINVAL; }
        if ((uintptr_t)it.d_state % 16) { err = "item " + std::to_string(i) + ": state not 16-byte aligned"; return SV_EINVAL; }
        if (grad && (!it.d_lambda || !it.observable)) {
            err = "item " + std::to_string(i) + ": gradients need d_lambda and an observable";
            return SV_EINVAL;
        }
        if (energies && !it.observable) { err = "item " + std::to_string(i) + ": energies need an observable"; return SV_EINVAL; }
        if (it.circuit->n_params > 0 && !it.params) { err = "item " + std::to_string(i) + ": params is NULL"; return SV_EINVAL; }
        if (it.circuit->n_qubits < 4) small = true;
    }
    if (count == 0) return SV_OK;
    if (small || (opts && opts->plain)) return run_batch_loop(count, items, dtype, stream, flags, energies, grads, opts, stats, err);

    auto t0 = std::chrono::steady_clock::now();
    // ---- IR and plans (planned in parallel; plans are cached by structure)
    std::vector<ItemHost> H((size_t)count);
    {
        std::atomic<int> next{0};
        unsigned hw = std::thread::hardware_concurrency();
        const int nthr = (int)std::max(1u, std::min<unsigned>(hw ? hw : 4, 16u));
        std::vector<std::thread> th;
        for (int t = 0; t < std::min(nthr, (int)count); ++t)
            th.emplace_back([&] {
                for (;;) {
                    const int i = next++;
                    if (i >= count) return;
                    const sv_batch_item& it = items[i];
                    try {
                        // geometry and fusion: the tuned choice for this width, else the options
                        BatchGeom g;
                        g.structured = !opts || opts->structured;
                        g.fuse_k = opts ? opts->max_fuse_k : 4;
                        if (geoms) {
                            auto gi = geoms->find(it.circuit->n_qubits);
                            if (gi != geoms->end()) g = gi->second;
                        }
                        BuildOpts bo;
                        bo.batch = 1;
                        bo.structured = g.structured != 0;
                        bo.fuse = true;
                        bo.fuse_k = g.fuse_k;
                        bo.product_init = false;
                        H[i].irf = build_ir(it.circuit, it.params, bo, nullptr, it.circuit->n_qubits);
                        H[i].pf = get_batch_plan(it.circuit, H[i].irf, dtype, false, bo, g);
                        fill_pool(H[i].pf->ep, H[i].irf, 1, H[i].poolf);
                        if (grad) {
                            bo.backward = true;
                            H[i].irb = build_ir(it.circuit, it.params, bo, nullptr, it.circuit->n_qubits);
                            H[i].pb = get_batch_plan(it.circuit, H[i].irb, dtype, true, bo, g);
                            fill_pool(H[i].pb->ep, H[i].irb, 1, H[i].poolb);
                        }
                    } catch (const std::exception& e) {
                        H[i].err = e.what();
                    }
                }
            });
        for (auto& t : th) t.join();
    }
    for (int i = 0; i < count; ++i) {
        if (!H[i].err.empty()) { err = "item " + std::to_string(i) + ": planning failed: " + H[i].err; return SV_EUNSUPPORTED; }
        const EncodedPlan* eps[2] = {&H[i].pf->ep, grad ? &H[i].pb->ep : nullptr};
        for (const EncodedPlan* e : eps)
            if (e)
                for (const Step& s : e->steps)
                    if (s.type != ST_TILE)  // wide (k > 4) gates: run item by item
                        return run_batch_loop(count, items, dtype, stream, flags, energies, grads, opts, stats, err);
    }

    // ---- device layout
    const size_t ab = dtype == SV_C64 ? 8 : 16;
    struct Off {
        size_t f_pass, f_phase, f_op, f_form, f_pair, f_etab, f_pool;
        size_t b_pass, b_phase, b_op, b_form, b_pair, b_etab, b_pool;
        size_t px, pg0, pz, pc, pph;
        size_t gpart, epart;
        uint32_t ngroup, nterm;
    };
    std::vector<Off> off((size_t)count);
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align_up(o + std::max<size_t>(bytes, 1), 256); return r; };
    // scratch the kernels write before they read it (gradient and energy
    // partials, reduced outputs): placed after the uploaded part, never copied
    size_t so = 0;
    auto take_scratch = [&](size_t bytes) { const size_t r = so; so = align_up(so + std::max<size_t>(bytes, 1), 256); return r; };
    std::vector<std::vector<uint64_t>> gx((size_t)count), gz((size_t)count);
    std::vector<std::vector<uint32_t>> gg0((size_t)count), gph((size_t)count);
    std::vector<std::vector<double>> gc((size_t)count);
    std::vector<uint32_t> hT((size_t)count);
    size_t lds = 0, lds_bwd = 0;
    for (int i = 0; i < count; ++i) {
        const EncodedPlan& F = H[i].pf->ep;
        Off& f = off[i];
        f.f_pass = take(F.passes.size() * sizeof(DPass));
        f.f_phase = take(F.phases.size() * sizeof(DPhase));
        f.f_op = take(F.ops.size() * sizeof(DOp));
        f.f_form = take(F.forms.size() * sizeof(DForm));
        f.f_pair = take(F.pairs.size() * sizeof(DPair));
        f.f_etab = take(F.etab.size() * sizeof(uint16_t));
        f.f_pool = take(H[i].poolf.size());
        for (const DPass& P : F.passes) lds = std::max(lds, tile_lds_bytes(dtype, false, P.T, P.nform, 0, 256));
        if (grad) {
            const EncodedPlan& B = H[i].pb->ep;
            f.b_pass = take(B.passes.size() * sizeof(DPass));
            f.b_phase = take(B.phases.size() * sizeof(DPhase));
            f.b_op = take(B.ops.size() * sizeof(DOp));
            f.b_form = take(B.forms.size() * sizeof(DForm));
            f.b_pair = take(B.pairs.size() * sizeof(DPair));
            f.b_etab = take(B.etab.size() * sizeof(uint16_t));
            f.b_pool = take(H[i].poolb.size());
            f.gpart = take_scratch(B.gpart_size * sizeof(double));
            for (const DPass& P : B.passes) lds_bwd = std::max(lds_bwd, tile_lds_bytes(dtype, true, P.T, P.nform, P.ngrad, 256));
        }
        // observable, grouped by x mask
        const sv_pauli_sum* h = items[i].observable;
        if (h) {
            if (h->n_terms < 0 || (h->n_terms > 0 && (!h->coeff || !h->x_mask || !h->z_mask))) {
                err = "item " + std::to_string(i) + ": bad observable";
                return SV_EINVAL;
            }
            const int n = items[i].circuit->n_qubits;
            const uint64_t qm = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
            std::vector<std::vector<int>> grp;
            for (int t = 0; t < h->n_terms; ++t) {
                if ((h->x_mask[t] | h->z_mask[t]) & ~qm) { err = "item " + std::to_string(i) + ": Pauli term outside the register"; return SV_EINVAL; }
                size_t g = 0;
                for (; g < gx[i].size(); ++g) if (gx[i][g] == h->x_mask[t]) break;
                if (g == gx[i].size()) { gx[i].push_back(h->x_mask[t]); grp.emplace_back(); }
                grp[g].push_back(t);
            }
            for (size_t g = 0; g < grp.size(); ++g) {
                gg0[i].push_back((uint32_t)gz[i].size());
                for (int t : grp[g]) {
                    gz[i].push_back(h->z_mask[t]);
                    gc[i].push_back(h->coeff[t]);
                    gph[i].push_back((uint32_t)(__builtin_popcountll(h->x_mask[t] & h->z_mask[t]) & 3));
                }
            }
            gg0[i].push_back((uint32_t)gz[i].size());
        } else {
            gg0[i].push_back(0);
        }
        f.ngroup = (uint32_t)gx[i].size();
        f.nterm = (uint32_t)gz[i].size();
        f.px = take(gx[i].size() * 8);
        f.pg0 = take(gg0[i].size() * 4);
        f.pz = take(gz[i].size() * 8);
        f.pc = take(gc[i].size() * 8);
        f.pph = take(gph[i].size() * 4);
        const int n = items[i].circuit->n_qubits;
        hT[i] = (uint32_t)std::min(n, 12);
        f.epart = take_scratch(((size_t)1 << (n - hT[i])) * sizeof(double));
    }
    // records: stages per item
    std::vector<std::vector<BRec>> stages((size_t)count);
    for (int i = 0; i < count; ++i) {
        const int n = items[i].circuit->n_qubits;
        auto add = [&](uint32_t kind, uint32_t pass, uint32_t T) {
            BRec r{};
            r.item = (uint32_t)i;
            r.kind = kind;
            r.pass = pass;
            r.T = T;
            r.ntiles = 1u << (n - (int)T);
            stages[i].push_back(r);
        };
        if (flags & SV_BATCH_INIT_ZERO) add(BK_INIT, 0, hT[i]);
        const EncodedPlan& F = H[i].pf->ep;
        for (size_t p = 0; p < F.passes.size(); ++p) add(BK_FWD, (uint32_t)p, F.passes[p].T);
        if (grad) {
            add(BK_HPSI, 0, hT[i]);
            const EncodedPlan& B = H[i].pb->ep;
            for (size_t p = 0; p < B.passes.size(); ++p) add(BK_BWD, (uint32_t)p, B.passes[p].T);
        } else if (energies) {
            add(BK_ENERGY, 0, hT[i]);
        }
    }
    // queues: largest items first onto the least-loaded queue
    std::vector<int> order((size_t)count);
    for (int i = 0; i < count; ++i) order[i] = i;
    auto cost = [&](int i) {
        double c = 0.0;
        for (const BRec& r : stages[i]) c += (double)r.ntiles * std::ldexp(1.0, (int)r.T) * (r.kind == BK_BWD ? 2.0 : 1.0);
        return c;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<std::vector<int>> qitems(kQueues);
    double qload[kQueues] = {0};
    for (int i : order) {
        uint32_t best = 0;
        for (uint32_t q = 1; q < kQueues; ++q) if (qload[q] < qload[best]) best = q;
        qitems[best].push_back(i);
        qload[best] += cost(i);
    }
    // Two persistent launches on the stream: stages before the backward sweep
    // (init, forward passes, lambda / energy), then the backward passes, each
    // with the interpreter it needs (the backward one carries psi and lambda).
    std::vector<BRec> recs[2];
    BatchArgs BA[2]{};
    std::vector<std::vector<int32_t>> recid((size_t)count);
    for (int ph = 0; ph < 2; ++ph) {
        for (auto& v : recid) v.clear();
        for (uint32_t q = 0; q < kQueues; ++q) {
            BA[ph].qrec0[q] = (uint32_t)recs[ph].size();
            std::vector<int> its = qitems[q];
            std::sort(its.begin(), its.end());
            std::vector<std::vector<BRec>> st((size_t)count);
            size_t maxl = 0;
            for (int i : its) {
                for (const BRec& r : stages[i])
                    if ((r.kind == BK_BWD) == (ph == 1)) st[i].push_back(r);
                maxl = std::max(maxl, st[i].size());
            }
            uint64_t w = 0;
            for (size_t lvl = 0; lvl < maxl; ++lvl)
                for (int i : its) {
                    if (lvl >= st[i].size()) continue;
                    BRec r = st[i][lvl];
                    r.first_w = w;
                    r.dep = lvl ? recid[i][lvl - 1] : -1;
                    w += r.ntiles;
                    recid[i].push_back((int32_t)recs[ph].size());
                    recs[ph].push_back(r);
                }
            BA[ph].qtotal[q] = w;
            if (w >= (1ull << 31)) { err = "batch too large for one launch"; return SV_EUNSUPPORTED; }
        }
        BA[ph].qrec0[kQueues] = (uint32_t)recs[ph].size();
    }
    const size_t o_items = take((size_t)count * sizeof(BItem));
    size_t o_recs[2], o_cnt[2];
    for (int ph = 0; ph < 2; ++ph) {
        o_recs[ph] = take(std::max<size_t>(1, recs[ph].size()) * sizeof(BRec));
        o_cnt[ph] = take((kQueues + recs[ph].size() + 1) * sizeof(uint32_t));
    }
    // reduction tasks: energies then gradient slots
    struct Task { const double* src; uint64_t ntile; uint32_t nslot; uint32_t pad; double* dst; };
    std::vector<Task> tasks;
    size_t nout = (size_t)count;
    std::vector<size_t> gslot0((size_t)count, 0);
    for (int i = 0; i < count; ++i) {
        gslot0[i] = nout;
        if (grad) nout += (size_t)H[i].pb->ep.ngrad_total;
    }
    const size_t o_out = take_scratch(nout * sizeof(double));
    const size_t o_tasks = take(((size_t)count * 64 + 16) * sizeof(Task));
    const size_t upload = o;
    const size_t total = upload + so;
    if (opts && opts->max_work_mib > 0 && total > ((size_t)opts->max_work_mib << 20)) {
        err = "the batch work area needs " + std::to_string(total) + " bytes, above max_work_mib = " +
              std::to_string(opts->max_work_mib) + " MiB";
        return SV_ENOMEM;
    }

    std::unique_lock<std::mutex> stage_lock(g_stage_mu);
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) { err = std::string("hipGetDevice: ") + hipGetErrorString(he); return SV_EDEVICE; }
    DevArea& area = g_dev[dev];
    if (area.bytes < total) {
        // the previous call on this device has synchronised (it released the lock)
        if (area.p) (void)hipFree(area.p);
        area.p = nullptr;
        area.bytes = 0;
        he = hipMalloc(&area.p, total);
        if (he != hipSuccess) { (void)hipGetLastError(); err = std::string("hipMalloc: ") + hipGetErrorString(he); return SV_ENOMEM; }
        area.bytes = total;
    }
    unsigned char* D = reinterpret_cast<unsigned char*>(area.p);
    unsigned char* S = D + upload;   // scratch part
    // every exit below waits for the stream, so the staging buffer is never
    // handed to the next call while an upload from it is in flight
    struct SyncOnExit {
        hipStream_t s;
        ~SyncOnExit() { (void)hipStreamSynchronize(s); }
    } sync_on_exit{stream};
    if (g_stage_bytes < upload) {
        if (g_stage) (void)hipHostFree(g_stage);
        g_stage = nullptr;
        g_stage_bytes = 0;
        const size_t want = align_up(upload + upload / 4, (size_t)1 << 20);
        if (hipHostMalloc(&g_stage, want, hipHostMallocDefault) == hipSuccess) g_stage_bytes = want;
        else g_stage = nullptr;
    }
    std::vector<unsigned char> hv;
    if (!g_stage) hv.assign(upload, 0);   // pinned memory unavailable: pageable upload
    unsigned char* hp = g_stage ? reinterpret_cast<unsigned char*>(g_stage) : hv.data();
    for (int ph = 0; ph < 2; ++ph) std::memset(hp + o_cnt[ph], 0, (kQueues + recs[ph].size() + 1) * sizeof(uint32_t));
    auto put = [&](size_t at, const void* src, size_t n) { if (n) std::memcpy(hp + at, src, n); };
    std::vector<BItem> bi((size_t)count);
    auto pack_item = [&](int i) {
        const Off& f = off[i];
        const EncodedPlan& F = H[i].pf->ep;
        put(f.f_pass, F.passes.data(), F.passes.size() * sizeof(DPass));
        put(f.f_phase, F.phases.data(), F.phases.size() * sizeof(DPhase));
        put(f.f_op, F.ops.data(), F.ops.size() * sizeof(DOp));
        put(f.f_form, F.forms.data(), F.forms.size() * sizeof(DForm));
        put(f.f_pair, F.pairs.data(), F.pairs.size() * sizeof(DPair));
        put(f.f_etab, F.etab.data(), F.etab.size() * sizeof(uint16_t));
        put(f.f_pool, H[i].poolf.data(), H[i].poolf.size());
        BItem& b = bi[i];
        b.state = items[i].d_state;
        b.lam = items[i].d_lambda;
        b.n = (uint32_t)items[i].circuit->n_qubits;
        b.fwd = BPlan{reinterpret_cast<const DPass*>(D + f.f_pass), reinterpret_cast<const DPhase*>(D + f.f_phase),
                      reinterpret_cast<const DOp*>(D + f.f_op), reinterpret_cast<const DForm*>(D + f.f_form),
                      reinterpret_cast<const DPair*>(D + f.f_pair), reinterpret_cast<const uint16_t*>(D + f.f_etab),
                      D + f.f_pool};
        if (grad) {
            const EncodedPlan& B = H[i].pb->ep;
            put(f.b_pass, B.passes.data(), B.passes.size() * sizeof(DPass));
            put(f.b_phase, B.phases.data(), B.phases.size() * sizeof(DPhase));
            put(f.b_op, B.ops.data(), B.ops.size() * sizeof(DOp));
            put(f.b_form, B.forms.data(), B.forms.size() * sizeof(DForm));
            put(f.b_pair, B.pairs.data(), B.pairs.size() * sizeof(DPair));
            put(f.b_etab, B.etab.data(), B.etab.size() * sizeof(uint16_t));
            put(f.b_pool, H[i].poolb.data(), H[i].poolb.size());
            b.bwd = BPlan{reinterpret_cast<const DPass*>(D + f.b_pass), reinterpret_cast<const DPhase*>(D + f.b_phase),
                          reinterpret_cast<const DOp*>(D + f.b_op), reinterpret_cast<const DForm*>(D + f.b_form),
                          reinterpret_cast<const DPair*>(D + f.b_pair), reinterpret_cast<const uint16_t*>(D + f.b_etab),
                          D + f.b_pool};
            b.gpart = reinterpret_cast<double*>(S + f.gpart);
        }
        put(f.px, gx[i].data(), gx[i].size() * 8);
        put(f.pg0, gg0[i].data(), gg0[i].size() * 4);
        put(f.pz, gz[i].data(), gz[i].size() * 8);
        put(f.pc, gc[i].data(), gc[i].size() * 8);
        put(f.pph, gph[i].data(), gph[i].size() * 4);
        b.pd.x = reinterpret_cast<const uint64_t*>(D + f.px);
        b.pd.g0 = reinterpret_cast<const uint32_t*>(D + f.pg0);
        b.pd.z = reinterpret_cast<const uint64_t*>(D + f.pz);
        b.pd.c = reinterpret_cast<const double*>(D + f.pc);
        b.pd.ph = reinterpret_cast<const uint32_t*>(D + f.pph);
        b.pd.ngroup = f.ngroup;
        b.epart = reinterpret_cast<double*>(S + f.epart);
    };
    {
        // pack the items in parallel (disjoint ranges of the staging buffer)
        std::atomic<int> next{0};
        unsigned hw = std::thread::hardware_concurrency();
        const int nthr = (int)std::max(1u, std::min<unsigned>(hw ? hw : 4, 16u));
        std::vector<std::thread> th;
        for (int t = 0; t < std::min(nthr, (int)count); ++t)
            th.emplace_back([&] {
                for (int i = next++; i < count; i = next++) pack_item(i);
            });
        for (auto& t : th) t.join();
    }
    for (int i = 0; i < count; ++i) {
        const BItem& b = bi[i];
        const int n = items[i].circuit->n_qubits;
        double* outp = reinterpret_cast<double*>(S + o_out);
        if (energies) tasks.push_back(Task{b.epart, 1ull << (n - hT[i]), 1u, 0u, outp + i});
        if (grad) {
            const EncodedPlan& B = H[i].pb->ep;
            size_t slot = gslot0[i];
            for (const DPass& P : B.passes) {
                if (!P.ngrad) continue;
                tasks.push_back(Task{b.gpart + P.gpart_off, 1ull << (n - P.T), P.ngrad, 0u, outp + slot});
                slot += P.ngrad;
            }
        }
    }
    if (tasks.size() > (size_t)count * 64 + 16) { err = "too many reduction tasks"; return SV_EUNSUPPORTED; }
    put(o_items, bi.data(), bi.size() * sizeof(BItem));
    for (int ph = 0; ph < 2; ++ph) put(o_recs[ph], recs[ph].data(), recs[ph].size() * sizeof(BRec));
    put(o_tasks, tasks.data(), tasks.size() * sizeof(Task));
    he = hipMemcpyAsync(area.p, hp, upload, hipMemcpyHostToDevice, stream);
    if (he != hipSuccess) { err = std::string("hipMemcpyAsync: ") + hipGetErrorString(he); return SV_EDEVICE; }
    int dev0 = 0, khz = 0, ncu = 0;
    (void)hipGetDevice(&dev0);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev0) != hipSuccess || khz <= 0) khz = 100000;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev0);
    // host work up to the launch: IR, plans (cached by structure), pools, layout, upload
    const double plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int ph = 0; ph < 2; ++ph) {
        if (recs[ph].empty()) continue;
        BatchArgs& A = BA[ph];
        A.items = reinterpret_cast<const BItem*>(D + o_items);
        A.recs = reinterpret_cast<const BRec*>(D + o_recs[ph]);
        A.head = reinterpret_cast<uint32_t*>(D + o_cnt[ph]);
        A.done = A.head + kQueues;
        A.err = A.done + recs[ph].size();
        A.wait_ticks = (uint64_t)khz * 2000ull;   // 2 s per dependency wait
        const size_t lds_ph = ph ? lds_bwd : lds;
        int bpc = 0;
        he = batch_occupancy(dtype, ph == 1, lds_ph, &bpc);
        if (he != hipSuccess || bpc < 1) { err = std::string("occupancy query failed: ") + hipGetErrorString(he); return SV_EDEVICE; }
        uint32_t nblocks = (uint32_t)(bpc * std::max(ncu, 1));
        nblocks = std::max<uint32_t>(kQueues, nblocks / kQueues * kQueues);
        he = launch_batch(dtype, ph == 1, A, nblocks, lds_ph, stream);
        if (he != hipSuccess) { err = std::string("persistent launch: ") + hipGetErrorString(he); return SV_EDEVICE; }
    }
    he = launch_multi_sum(reinterpret_cast<const void*>(D + o_tasks), (uint32_t)tasks.size(), stream);
    if (he != hipSuccess) { err = std::string("reduction launch: ") + hipGetErrorString(he); return SV_EDEVICE; }
    std::vector<double> out(nout, 0.0);
    uint32_t errflag[2] = {0, 0};
    he = hipMemcpyAsync(out.data(), S + o_out, nout * sizeof(double), hipMemcpyDeviceToHost, stream);
    for (int ph = 0; ph < 2; ++ph)
        if (he == hipSuccess && !recs[ph].empty())
            he = hipMemcpyAsync(&errflag[ph], BA[ph].err, 4, hipMemcpyDeviceToHost, stream);
    if (he == hipSuccess) he = hipStreamSynchronize(stream);
    if (he != hipSuccess) { err = std::string("batch: ") + hipGetErrorString(he); return SV_EDEVICE; }
    if (errflag[0] || errflag[1]) { err = "persistent batch: a dependency wait exceeded its time budget"; return SV_EDEVICE; }
    size_t goff = 0;
    for (int i = 0; i < count; ++i) {
        if (energies) energies[i] = out[i];
        if (grad) {
            const int np = items[i].circuit->n_params;
            for (int p = 0; p < np; ++p) grads[goff + p] = 0.0;
            const EncodedPlan& B = H[i].pb->ep;
            for (int s = 0; s < B.ngrad_total; ++s)
                grads[goff + B.grad_param[s]] += B.grad_scale[s] * out[gslot0[i] + s];
            goff += (size_t)np;
        }
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        for (int i = 0; i < count; ++i) {
            stats->gates_in += items[i].circuit->n_gates;
            stats->passes += (int32_t)H[i].pf->ep.passes.size() + (grad ? (int32_t)H[i].pb->ep.passes.size() : 0);
            stats->alu_ops += H[i].pf->ep.alu_ops + (grad ? H[i].pb->ep.alu_ops : 0.0);
        }
        stats->launches = (recs[0].empty() ? 0 : 1) + (recs[1].empty() ? 0 : 1) + 1;
        stats->plan_ms = plan_ms;
        double bytes = 0.0;
        for (int i = 0; i < count; ++i)
            for (const BRec& r : stages[i])
                bytes += (double)ab * std::ldexp(1.0, items[i].circuit->n_qubits) * (r.kind == BK_BWD ? 4.0 : 2.0);
        stats->hbm_bytes = bytes;
    }
    return SV_OK;
}

}  // namespace svmi

// ---- autotuner of the batch's fusion mode and tile geometry, per width
namespace svmi {

namespace {

std::mutex g_btune_mu;
std::map<uint64_t, BatchGeom> g_btune;   // (dtype, direction, width) -> choice
bool g_btune_loaded = false;

uint64_t btune_key(int dtype, bool grad, int n) {
    return ((uint64_t)dtype << 40) | ((uint64_t)(grad ? 1 : 0) << 32) | (uint64_t)(uint32_t)n;
}

std::string btune_file() {
    const char* d = std::getenv("SVMI_BATCH_TUNE_CACHE");
    return d && *d ? std::string(d) : std::string("/tmp/svmi-batch-tune.txt");
}

// caller holds g_btune_mu
void btune_load() {
    if (g_btune_loaded) return;
    g_btune_loaded = true;
    FILE* f = std::fopen(btune_file().c_str(), "r");
    if (!f) return;
    int dt, gr, n, s, k, T, L;
    while (std::fscanf(f, "%d %d %d %d %d %d %d", &dt, &gr, &n, &s, &k, &T, &L) == 7) {
        BatchGeom g;
        g.structured = s;
        g.fuse_k = k;
        g.T = T;
        g.L = L;
        g_btune[btune_key(dt, gr != 0, n)] = g;
    }
    std::fclose(f);
}

}  // namespace

bool batch_tuned_table(int dtype, bool grad, GeomTable& out) {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    btune_load();
    out.clear();
    for (const auto& kv : g_btune)
        if ((int)(kv.first >> 40) == dtype && (((kv.first >> 32) & 1) != 0) == grad)
            out[(int)(kv.first & 0xffffffffu)] = kv.second;
    return !out.empty();
}

bool batch_tuned_lookup(int dtype, bool grad, int n, BatchGeom& g) {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    btune_load();
    auto it = g_btune.find(btune_key(dtype, grad, n));
    if (it == g_btune.end()) return false;
    g = it->second;
    return true;
}

// For every width among the items: time the persistent launch of that
// width's items under candidate fusion modes (butterflies with lazy phases,
// dense blocks of 2, 3 or 4 qubits), then tile sizes 2^T and segment lengths
// 2^L around the best, one coordinate at a time, keeping a change only when
// it saves more than 3 %.  Each candidate runs twice (plans, then timed).
sv_status tune_batch(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream, int32_t flags,
                     const sv_opts* opts, int32_t* widths_tuned, std::string& err) {
    if (count <= 0 || !items) { err = "no items"; return SV_EINVAL; }
    const bool grad = (flags & SV_BATCH_GRAD) != 0;
    const int32_t rflags = (grad ? SV_BATCH_GRAD : SV_BATCH_FORWARD) | SV_BATCH_INIT_ZERO;
    std::map<int, std::vector<int>> by_w;
    for (int32_t i = 0; i < count; ++i) {
        if (!items[i].circuit) { err = "item " + std::to_string(i) + ": NULL circuit"; return SV_EINVAL; }
        by_w[items[i].circuit->n_qubits].push_back(i);
    }
    int tuned = 0;
    for (const auto& kv : by_w) {
        const int w = kv.first;
        if (w < 4) continue;                      // gate by gate: nothing to choose
        std::vector<sv_batch_item> sub;
        size_t np = 0;
        for (int i : kv.second) {
            sub.push_back(items[i]);
            np += (size_t)std::max(0, items[i].circuit->n_params);
        }
        std::vector<double> e(sub.size() + 1), gr(np + 1);
        bool obs_all = true;
        for (const sv_batch_item& it : sub) obs_all = obs_all && it.observable;
        sv_status st = SV_OK;
        auto time_geom = [&](const BatchGeom& g) -> double {
            const GeomTable t{{w, g}};
            double best = 1e300;
            for (int rep = 0; rep < 2 && st == SV_OK; ++rep) {
                const auto t0 = std::chrono::steady_clock::now();
                st = run_batch_persistent((int32_t)sub.size(), sub.data(), dtype, stream, rflags,
                                          obs_all ? e.data() : nullptr, grad ? gr.data() : nullptr, opts, nullptr,
                                          err, &t);
                const double ms =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                if (rep > 0) best = ms;
            }
            return best;
        };
        BatchGeom best;
        best.structured = 1;
        best.fuse_k = 4;
        double best_ms = time_geom(best);
        if (st != SV_OK) return st;
        auto consider = [&](const BatchGeom& g) {
            const double ms = time_geom(g);
            if (st == SV_OK && ms < 0.97 * best_ms) {
                best_ms = ms;
                best = g;
            }
        };
        for (int k = 2; k <= 4 && st == SV_OK; ++k) {
            BatchGeom g = best;
            g.structured = 0;
            g.fuse_k = k;
            consider(g);
        }
        if (w > 10) {
            const int tmax = (dtype == SV_C128 && grad) ? 12 : 13;
            const BatchGeom base = best;
            for (int T = 11; T <= std::min(tmax, w) && st == SV_OK; ++T) {
                BatchGeom g = base;
                g.T = T;
                if (T == (dtype == SV_C64 ? 12 : (grad ? 11 : 12))) continue;   // the default, timed above
                consider(g);
            }
            const BatchGeom base2 = best;
            for (int L = 3; L <= 5 && st == SV_OK; ++L) {
                if (L == 4) continue;
                BatchGeom g = base2;
                g.L = L;
                consider(g);
            }
        }
        if (st != SV_OK) return st;
        {
            std::lock_guard<std::mutex> lk(g_btune_mu);
            btune_load();
            g_btune[btune_key(dtype, grad, w)] = best;
            if (FILE* f = std::fopen(btune_file().c_str(), "a")) {
                std::fprintf(f, "%d %d %d %d %d %d %d\n", (int)dtype, grad ? 1 : 0, w, best.structured, best.fuse_k,
                             best.T, best.L);
                std::fclose(f);
            }
        }
        ++tuned;
    }
    if (widths_tuned) *widths_tuned = tuned;
    return SV_OK;
}

}  // namespace svmi
