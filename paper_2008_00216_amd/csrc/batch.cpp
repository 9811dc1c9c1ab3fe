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
#include <functional>
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
struct Stage {
    void* p = nullptr;
    size_t bytes = 0;
};
struct DevArea {
    void* p = nullptr;
    size_t bytes = 0;
};
// The resources of one call: the device work areas the first and the second
// launch read, their pinned staging, and pinned space for the results.  A
// device has two slots, so one call can be prepared and launched while the
// previous one runs (sv_apply_batch_async).
struct Slot {
    DevArea area[2];
    Stage stage[2];
    Stage res;                  // outputs and the two wait-error flags
    hipEvent_t done = nullptr;  // recorded after the copy of the results
    bool busy = false;          // held by a job until it is finished
};
struct DevState {
    Slot slot[2];
    hipStream_t up = nullptr;   // uploads of the second areas (default priority)
    hipEvent_t ev = nullptr;
};
std::unordered_map<int, DevState> g_dev;   // by device ordinal

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
    p.beam = std::max(1, g.beam);
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
                                             ((uint64_t)cfg.T << 28) ^ ((uint64_t)cfg.L << 34) ^
                                             ((uint64_t)cfg.beam << 40) ^ ir_signature(ir));
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

// fn(i) for every item, on up to 16 host threads
void for_items(int count, const std::function<void(int)>& fn) {
    std::atomic<int> next{0};
    unsigned hw = std::thread::hardware_concurrency();
    const int nthr = (int)std::max(1u, std::min<unsigned>(hw ? hw : 4, 16u));
    std::vector<std::thread> th;
    for (int t = 0; t < std::min(nthr, count); ++t)
        th.emplace_back([&] {
            for (int i = next++; i < count; i = next++) fn(i);
        });
    for (auto& t : th) t.join();
}

}  // namespace

// A launched batch call, finished by batch_finish: where its results land
// and what turns them into energies and gradients.
struct BatchJob {
    bool immediate = false;      // ran item by item: results already in e, g
    std::vector<double> e, g;
    int dev = 0, slot = -1;
    hipStream_t stream = nullptr;
    int count = 0;
    bool grad = false, want_e = false;
    size_t nout = 0;
    const double* out = nullptr; // pinned (or job-owned) copy of the reduced outputs
    const uint32_t* errflag = nullptr;
    std::vector<double> outv;    // used when pinned memory is unavailable
    std::vector<unsigned char> hv[2];   // pageable staging when pinned memory is unavailable
    std::vector<int> nparams;
    std::vector<std::shared_ptr<PlanKeyed>> pb;
    std::vector<size_t> gslot0;
    sv_stats stats{};
};

sv_status batch_launch(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream, int32_t flags,
                       bool want_e, const sv_opts* opts, std::string& err, const GeomTable* geoms, BatchJob& job) {
    if (count < 0) { err = "count < 0"; return SV_EINVAL; }
    if (count > 0 && !items) { err = "items is NULL"; return SV_EINVAL; }
    if (dtype != SV_C64 && dtype != SV_C128) { err = "dtype must be SV_C64 or SV_C128"; return SV_EINVAL; }
    if (opts && (opts->plan_beam < 0 || opts->plan_beam > 64)) { err = "plan_beam must be 0..64"; return SV_EINVAL; }
    const bool grad = (flags & SV_BATCH_GRAD) != 0;
    if (grad) want_e = true;
    job.count = count;
    job.grad = grad;
    job.want_e = want_e;
    job.stream = stream;
    bool small = false;
    // circuit validation (every gate of every item) in parallel; the errors
    // are reported in item order, each after that item's NULL checks
    std::vector<std::string> verr((size_t)std::max(count, 0));
    for_items(count, [&](int i) {
        if (items[i].circuit) verr[i] = validate_circuit(items[i].circuit, items[i].circuit->n_qubits);
    });
    for (int32_t i = 0; i < count; ++i) {
        const sv_batch_item& it = items[i];
        if (!it.circuit || !it.d_state) { err = "item " + std::to_string(i) + ": NULL circuit or state"; return SV_EINVAL; }
        if (!verr[i].empty()) { err = "item " + std::to_string(i) + ": " + verr[i]; return SV_EINVAL; }
        const int nmax = dtype == SV_C64 ? 34 : 33;
        if (it.circuit->n_qubits < 1 || it.circuit->n_qubits > nmax) { err = "item " + std::to_string(i) + ": bad width"; return SV_EINVAL; }
        if ((uintptr_t)it.d_state % 16) { err = "item " + std::to_string(i) + ": state not 16-byte aligned"; return SV_EINVAL; }
        if (grad && (!it.d_lambda || !it.observable)) {
            err = "item " + std::to_string(i) + ": gradients need d_lambda and an observable";
            return SV_EINVAL;
        }
        if (want_e && !it.observable) { err = "item " + std::to_string(i) + ": energies need an observable"; return SV_EINVAL; }
        if (it.circuit->n_params > 0 && !it.params) { err = "item " + std::to_string(i) + ": params is NULL"; return SV_EINVAL; }
        if (it.circuit->n_qubits < 4) small = true;
    }
    // item by item, synchronously: the job holds the results
    auto immediate = [&]() -> sv_status {
        job.immediate = true;
        size_t np = 0;
        for (int i = 0; i < count; ++i) np += (size_t)items[i].circuit->n_params;
        job.e.assign((size_t)count, 0.0);
        job.g.assign(np, 0.0);
        return run_batch_loop(count, items, dtype, stream, flags, want_e ? job.e.data() : nullptr, job.g.data(),
                              opts, &job.stats, err);
    };
    if (count == 0) {
        job.immediate = true;
        return SV_OK;
    }
    if (small || (opts && opts->plain)) return immediate();

    const auto t0 = std::chrono::steady_clock::now();
    auto ms_since = [](std::chrono::steady_clock::time_point t) {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
    };
    // geometry and fusion of an item: the tuned choice for its width, else the options
    auto geom_of = [&](int i) {
        BatchGeom g;
        g.structured = !opts || opts->structured;
        g.fuse_k = opts ? opts->max_fuse_k : 4;
        if (geoms) {
            auto gi = geoms->find(items[i].circuit->n_qubits);
            if (gi != geoms->end()) g = gi->second;
        }
        g.beam = opts && opts->plan_beam > 0 ? opts->plan_beam : 8;
        return g;
    };
    // Gates wider than a register phase (input gates of more than 4 qubits,
    // or dense blocks fused beyond 4) become plain kernels in either
    // direction: such batches run item by item.  Decided before anything is
    // launched, since the backward plans are only built while the forward
    // launch runs.
    for (int i = 0; i < count; ++i) {
        const BatchGeom g = geom_of(i);
        bool wide = !g.structured && g.fuse_k > 4;
        for (int32_t k = 0; k < items[i].circuit->n_gates && !wide; ++k) wide = items[i].circuit->gates[k].nq > 4;
        if (wide) return immediate();
    }

    // ---- IR, plans (cached by structure) and pools of one direction, in parallel
    std::vector<ItemHost> H((size_t)count);
    auto plan_dir = [&](bool bwd) -> sv_status {
        for_items(count, [&](int i) {
            const sv_batch_item& it = items[i];
            try {
                const BatchGeom g = geom_of(i);
                BuildOpts bo;
                bo.batch = 1;
                bo.structured = g.structured != 0;
                bo.fuse = true;
                bo.fuse_k = g.fuse_k;
                bo.product_init = false;
                bo.backward = bwd;
                std::vector<IRGate>& ir = bwd ? H[i].irb : H[i].irf;
                ir = build_ir(it.circuit, it.params, bo, nullptr, it.circuit->n_qubits);
                std::shared_ptr<PlanKeyed>& pk = bwd ? H[i].pb : H[i].pf;
                pk = get_batch_plan(it.circuit, ir, dtype, bwd, bo, g);
                fill_pool(pk->ep, ir, 1, bwd ? H[i].poolb : H[i].poolf);
            } catch (const std::exception& e) {
                H[i].err = e.what();
            }
        });
        for (int i = 0; i < count; ++i) {
            if (!H[i].err.empty()) { err = "item " + std::to_string(i) + ": planning failed: " + H[i].err; return SV_EUNSUPPORTED; }
            const EncodedPlan& e = bwd ? H[i].pb->ep : H[i].pf->ep;
            for (const Step& s : e.steps)
                if (s.type != ST_TILE) {
                    err = "item " + std::to_string(i) + ": a plan step is not a tile pass";
                    return SV_EUNSUPPORTED;
                }
        }
        return SV_OK;
    };
    // With a cap on the work area both directions are planned first, so that
    // the whole area is known before anything runs; otherwise the backward
    // plans are built while the forward launch runs.
    const bool overlap = grad && !(opts && opts->max_work_mib > 0);
    sv_status st = plan_dir(false);
    if (st != SV_OK) return st;
    if (grad && !overlap) {
        st = plan_dir(true);
        if (st != SV_OK) return st;
    }

    const size_t ab = dtype == SV_C64 ? 8 : 16;
    // Two work areas: [0] what the first launch reads (forward plans,
    // observables, its records, energy partials), [1] what the second launch
    // and the reduction read (backward plans, records, gradient partials,
    // reduction tasks and outputs).  Each is an uploaded part followed by
    // scratch the kernels write before they read it.
    struct Layout {
        size_t up = 0, sc = 0;
        size_t take(size_t bytes) { const size_t r = up; up = align_up(up + std::max<size_t>(bytes, 1), 256); return r; }
        size_t take_scratch(size_t bytes) { const size_t r = sc; sc = align_up(sc + std::max<size_t>(bytes, 1), 256); return r; }
        size_t total() const { return up + sc; }
    };
    struct POff {
        size_t pass, phase, op, form, pair, etab, pool;
    };
    struct Off {
        POff f, b;
        size_t px, pg0, pz, pc, pph;
        size_t gpart, epart;
        uint32_t ngroup, nterm;
    };
    std::vector<Off> off((size_t)count);
    Layout LA[2];
    auto take_plan = [&](Layout& L, const EncodedPlan& E, const std::vector<unsigned char>& pool) {
        POff p;
        p.pass = L.take(E.passes.size() * sizeof(DPass));
        p.phase = L.take(E.phases.size() * sizeof(DPhase));
        p.op = L.take(E.ops.size() * sizeof(DOp));
        p.form = L.take(E.forms.size() * sizeof(DForm));
        p.pair = L.take(E.pairs.size() * sizeof(DPair));
        p.etab = L.take(E.etab.size() * sizeof(uint16_t));
        p.pool = L.take(pool.size());
        return p;
    };
    std::vector<std::vector<uint64_t>> gx((size_t)count), gz((size_t)count);
    std::vector<std::vector<uint32_t>> gg0((size_t)count), gph((size_t)count);
    std::vector<std::vector<double>> gc((size_t)count);
    std::vector<uint32_t> hT((size_t)count);
    size_t lds = 0, lds_bwd = 0;
    for (int i = 0; i < count; ++i) {
        const EncodedPlan& F = H[i].pf->ep;
        Off& f = off[i];
        f.f = take_plan(LA[0], F, H[i].poolf);
        for (const DPass& P : F.passes) lds = std::max(lds, tile_lds_bytes(dtype, false, P.T, P.nform, 0, 256));
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
        f.px = LA[0].take(gx[i].size() * 8);
        f.pg0 = LA[0].take(gg0[i].size() * 4);
        f.pz = LA[0].take(gz[i].size() * 8);
        f.pc = LA[0].take(gc[i].size() * 8);
        f.pph = LA[0].take(gph[i].size() * 4);
        const int n = items[i].circuit->n_qubits;
        hT[i] = (uint32_t)std::min(n, 12);
        f.epart = LA[0].take_scratch(((size_t)1 << (n - hT[i])) * sizeof(double));
    }
    // records (item, stage) of one launch, laid out in queues: largest items
    // first onto the least-loaded queue, then level order within a queue, so
    // that every dependency of a record precedes it in its queue
    auto build_recs = [&](bool bwd, std::vector<BRec>& recs, BatchArgs& A) -> sv_status {
        std::vector<std::vector<BRec>> st((size_t)count);
        for (int i = 0; i < count; ++i) {
            const int n = items[i].circuit->n_qubits;
            auto add = [&](uint32_t kind, uint32_t pass, uint32_t T) {
                BRec r{};
                r.item = (uint32_t)i;
                r.kind = kind;
                r.pass = pass;
                r.T = T;
                r.ntiles = 1u << (n - (int)T);
                st[i].push_back(r);
            };
            if (!bwd) {
                if (flags & SV_BATCH_INIT_ZERO) add(BK_INIT, 0, hT[i]);
                const EncodedPlan& F = H[i].pf->ep;
                for (size_t p = 0; p < F.passes.size(); ++p) add(BK_FWD, (uint32_t)p, F.passes[p].T);
                if (grad) add(BK_HPSI, 0, hT[i]);
                else if (want_e) add(BK_ENERGY, 0, hT[i]);
            } else {
                const EncodedPlan& B = H[i].pb->ep;
                for (size_t p = 0; p < B.passes.size(); ++p) add(BK_BWD, (uint32_t)p, B.passes[p].T);
            }
        }
        std::vector<int> order((size_t)count);
        std::vector<double> cost((size_t)count, 0.0);
        for (int i = 0; i < count; ++i) {
            order[i] = i;
            for (const BRec& r : st[i]) cost[i] += (double)r.ntiles * std::ldexp(1.0, (int)r.T) * (bwd ? 2.0 : 1.0);
        }
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        std::vector<std::vector<int>> qitems(kQueues);
        double qload[kQueues] = {0};
        for (int i : order) {
            uint32_t best = 0;
            for (uint32_t q = 1; q < kQueues; ++q) if (qload[q] < qload[best]) best = q;
            qitems[best].push_back(i);
            qload[best] += cost[i];
        }
        std::vector<std::vector<int32_t>> recid((size_t)count);
        for (uint32_t q = 0; q < kQueues; ++q) {
            A.qrec0[q] = (uint32_t)recs.size();
            std::vector<int> its = qitems[q];
            std::sort(its.begin(), its.end());
            size_t maxl = 0;
            for (int i : its) maxl = std::max(maxl, st[i].size());
            uint64_t w = 0;
            for (size_t lvl = 0; lvl < maxl; ++lvl)
                for (int i : its) {
                    if (lvl >= st[i].size()) continue;
                    BRec r = st[i][lvl];
                    r.first_w = w;
                    r.dep = lvl ? recid[i][lvl - 1] : -1;
                    w += r.ntiles;
                    recid[i].push_back((int32_t)recs.size());
                    recs.push_back(r);
                }
            A.qtotal[q] = w;
            if (w >= (1ull << 31)) { err = "batch too large for one launch"; return SV_EUNSUPPORTED; }
        }
        A.qrec0[kQueues] = (uint32_t)recs.size();
        return SV_OK;
    };
    std::vector<BRec> recs[2];
    BatchArgs BA[2]{};
    st = build_recs(false, recs[0], BA[0]);
    if (st != SV_OK) return st;
    const size_t o_items0 = LA[0].take((size_t)count * sizeof(BItem));
    const size_t o_recs0 = LA[0].take(std::max<size_t>(1, recs[0].size()) * sizeof(BRec));
    const size_t o_cnt0 = LA[0].take((kQueues + recs[0].size() + 1) * sizeof(uint32_t));

    // the second area: backward plans, records, partials, reduction tasks, outputs
    struct Task { const double* src; uint64_t ntile; uint32_t nslot; uint32_t pad; double* dst; };
    std::vector<size_t> gslot0((size_t)count, 0);
    size_t nout = 0, o_items1 = 0, o_recs1 = 0, o_cnt1 = 0, o_out = 0, o_tasks = 0;
    auto layout_second = [&]() -> sv_status {
        if (grad) {
            for (int i = 0; i < count; ++i) {
                const EncodedPlan& B = H[i].pb->ep;
                off[i].b = take_plan(LA[1], B, H[i].poolb);
                off[i].gpart = LA[1].take_scratch(B.gpart_size * sizeof(double));
                for (const DPass& P : B.passes) lds_bwd = std::max(lds_bwd, tile_lds_bytes(dtype, true, P.T, P.nform, P.ngrad, 256));
            }
            const sv_status s2 = build_recs(true, recs[1], BA[1]);
            if (s2 != SV_OK) return s2;
        }
        o_items1 = LA[1].take((size_t)count * sizeof(BItem));
        o_recs1 = LA[1].take(std::max<size_t>(1, recs[1].size()) * sizeof(BRec));
        o_cnt1 = LA[1].take((kQueues + recs[1].size() + 1) * sizeof(uint32_t));
        nout = (size_t)count;
        for (int i = 0; i < count; ++i) {
            gslot0[i] = nout;
            if (grad) nout += (size_t)H[i].pb->ep.ngrad_total;
        }
        o_out = LA[1].take_scratch(nout * sizeof(double));
        o_tasks = LA[1].take(((size_t)count * 64 + 16) * sizeof(Task));
        return SV_OK;
    };
    if (!overlap) {
        st = layout_second();
        if (st != SV_OK) return st;
    }
    if (opts && opts->max_work_mib > 0) {
        const size_t total = LA[0].total() + LA[1].total();
        if (total > ((size_t)opts->max_work_mib << 20)) {
            err = "the batch work area needs " + std::to_string(total) + " bytes, above max_work_mib = " +
                  std::to_string(opts->max_work_mib) + " MiB";
            return SV_ENOMEM;
        }
    }

    std::unique_lock<std::mutex> stage_lock(g_stage_mu);
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) { err = std::string("hipGetDevice: ") + hipGetErrorString(he); return SV_EDEVICE; }
    DevState& ds = g_dev[dev];
    const int si = !ds.slot[0].busy ? 0 : (!ds.slot[1].busy ? 1 : -1);
    if (si < 0) {
        err = "two batch jobs are in flight on this device: finish one first (sv_batch_finish)";
        return SV_EINVAL;
    }
    Slot& sl = ds.slot[si];
    sl.busy = true;
    job.dev = dev;
    job.slot = si;
    // every error exit below waits for the streams and frees the slot, so its
    // staging buffers and work areas are never handed to the next call while
    // a copy or kernel that uses them is in flight; a launched job keeps the
    // slot until batch_finish
    struct Guard {
        hipStream_t s;
        DevState* d;
        Slot* sl;
        bool keep = false;
        ~Guard() {
            if (keep) return;
            (void)hipStreamSynchronize(s);
            if (d->up) (void)hipStreamSynchronize(d->up);
            sl->busy = false;
        }
    } guard{stream, &ds, &sl};
    // grow-only device area `a` and pinned staging `a` of the slot
    auto reserve = [&](int a) -> unsigned char* {
        DevArea& area = sl.area[a];
        const size_t total = LA[a].total();
        if (area.bytes < total) {
            // the slot's previous job has finished (its stream has synchronised)
            if (area.p) (void)hipFree(area.p);
            area.p = nullptr;
            area.bytes = 0;
            he = hipMalloc(&area.p, total);
            if (he != hipSuccess) { (void)hipGetLastError(); err = std::string("hipMalloc: ") + hipGetErrorString(he); return nullptr; }
            area.bytes = total;
        }
        Stage& sg = sl.stage[a];
        if (sg.bytes < LA[a].up) {
            if (sg.p) (void)hipHostFree(sg.p);
            sg.p = nullptr;
            sg.bytes = 0;
            const size_t want = align_up(LA[a].up + LA[a].up / 4, (size_t)1 << 20);
            if (hipHostMalloc(&sg.p, want, hipHostMallocDefault) == hipSuccess) sg.bytes = want;
            else sg.p = nullptr;   // pinned memory unavailable: pageable upload
        }
        return reinterpret_cast<unsigned char*>(area.p);
    };
    auto staging = [&](int a) {
        if (sl.stage[a].p) return reinterpret_cast<unsigned char*>(sl.stage[a].p);
        job.hv[a].assign(LA[a].up, 0);
        return job.hv[a].data();
    };
    auto plan_ptrs = [](unsigned char* D, const POff& p) {
        return BPlan{reinterpret_cast<const DPass*>(D + p.pass), reinterpret_cast<const DPhase*>(D + p.phase),
                     reinterpret_cast<const DOp*>(D + p.op), reinterpret_cast<const DForm*>(D + p.form),
                     reinterpret_cast<const DPair*>(D + p.pair), reinterpret_cast<const uint16_t*>(D + p.etab),
                     D + p.pool};
    };
    auto put_plan = [](unsigned char* hp, const POff& p, const EncodedPlan& E, const std::vector<unsigned char>& pool) {
        auto put = [&](size_t at, const void* src, size_t n) { if (n) std::memcpy(hp + at, src, n); };
        put(p.pass, E.passes.data(), E.passes.size() * sizeof(DPass));
        put(p.phase, E.phases.data(), E.phases.size() * sizeof(DPhase));
        put(p.op, E.ops.data(), E.ops.size() * sizeof(DOp));
        put(p.form, E.forms.data(), E.forms.size() * sizeof(DForm));
        put(p.pair, E.pairs.data(), E.pairs.size() * sizeof(DPair));
        put(p.etab, E.etab.data(), E.etab.size() * sizeof(uint16_t));
        put(p.pool, pool.data(), pool.size());
    };
    int dev0 = 0, khz = 0, ncu = 0;
    (void)hipGetDevice(&dev0);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev0) != hipSuccess || khz <= 0) khz = 100000;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev0);
    auto launch = [&](int ph, unsigned char* D, size_t o_items, size_t o_recs, size_t o_cnt) -> sv_status {
        if (recs[ph].empty()) return SV_OK;
        BatchArgs& A = BA[ph];
        A.items = reinterpret_cast<const BItem*>(D + o_items);
        A.recs = reinterpret_cast<const BRec*>(D + o_recs);
        A.head = reinterpret_cast<uint32_t*>(D + o_cnt);
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
        return SV_OK;
    };

    // ---- first launch: init, forward passes, lambda / energies
    unsigned char* D0 = reserve(0);
    if (!D0) return SV_ENOMEM;
    unsigned char* S0 = D0 + LA[0].up;   // scratch part
    {
        unsigned char* hp = staging(0);
        std::memset(hp + o_cnt0, 0, (kQueues + recs[0].size() + 1) * sizeof(uint32_t));
        std::vector<BItem> bi((size_t)count);
        for_items(count, [&](int i) {   // disjoint ranges of the staging buffer
            const Off& f = off[i];
            put_plan(hp, f.f, H[i].pf->ep, H[i].poolf);
            auto put = [&](size_t at, const void* src, size_t n) { if (n) std::memcpy(hp + at, src, n); };
            put(f.px, gx[i].data(), gx[i].size() * 8);
            put(f.pg0, gg0[i].data(), gg0[i].size() * 4);
            put(f.pz, gz[i].data(), gz[i].size() * 8);
            put(f.pc, gc[i].data(), gc[i].size() * 8);
            put(f.pph, gph[i].data(), gph[i].size() * 4);
            BItem& b = bi[i];
            b = BItem{};
            b.state = items[i].d_state;
            b.lam = items[i].d_lambda;
            b.n = (uint32_t)items[i].circuit->n_qubits;
            b.fwd = plan_ptrs(D0, f.f);
            b.pd.x = reinterpret_cast<const uint64_t*>(D0 + f.px);
            b.pd.g0 = reinterpret_cast<const uint32_t*>(D0 + f.pg0);
            b.pd.z = reinterpret_cast<const uint64_t*>(D0 + f.pz);
            b.pd.c = reinterpret_cast<const double*>(D0 + f.pc);
            b.pd.ph = reinterpret_cast<const uint32_t*>(D0 + f.pph);
            b.pd.ngroup = f.ngroup;
            b.epart = reinterpret_cast<double*>(S0 + f.epart);
        });
        std::memcpy(hp + o_items0, bi.data(), bi.size() * sizeof(BItem));
        if (!recs[0].empty()) std::memcpy(hp + o_recs0, recs[0].data(), recs[0].size() * sizeof(BRec));
        he = hipMemcpyAsync(D0, hp, LA[0].up, hipMemcpyHostToDevice, stream);
        if (he != hipSuccess) { err = std::string("hipMemcpyAsync: ") + hipGetErrorString(he); return SV_EDEVICE; }
    }
    const double prep_ms = ms_since(t0);   // host work before the first launch
    st = launch(0, D0, o_items0, o_recs0, o_cnt0);
    if (st != SV_OK) return st;

    // ---- backward plans and the second area, built while the first launch runs
    if (overlap) {
        st = plan_dir(true);
        if (st == SV_OK) st = layout_second();
        if (st != SV_OK) return st;
    }
    unsigned char* D1 = reserve(1);
    if (!D1) return SV_ENOMEM;
    unsigned char* S1 = D1 + LA[1].up;
    std::vector<Task> tasks;
    {
        unsigned char* hp = staging(1);
        std::memset(hp + o_cnt1, 0, (kQueues + recs[1].size() + 1) * sizeof(uint32_t));
        std::vector<BItem> bi((size_t)count);
        for_items(count, [&](int i) {   // disjoint ranges of the staging buffer
            BItem& b = bi[i];
            b = BItem{};
            b.state = items[i].d_state;
            b.lam = items[i].d_lambda;
            b.n = (uint32_t)items[i].circuit->n_qubits;
            if (grad) {
                put_plan(hp, off[i].b, H[i].pb->ep, H[i].poolb);
                b.bwd = plan_ptrs(D1, off[i].b);
                b.gpart = reinterpret_cast<double*>(S1 + off[i].gpart);
            }
        });
        // reduction tasks: energies (partials in the first area), then gradient slots
        double* outp = reinterpret_cast<double*>(S1 + o_out);
        for (int i = 0; i < count; ++i) {
            const int n = items[i].circuit->n_qubits;
            if (want_e)
                tasks.push_back(Task{reinterpret_cast<double*>(S0 + off[i].epart), 1ull << (n - hT[i]), 1u, 0u, outp + i});
            if (grad) {
                const EncodedPlan& B = H[i].pb->ep;
                size_t slot = gslot0[i];
                for (const DPass& P : B.passes) {
                    if (!P.ngrad) continue;
                    tasks.push_back(Task{bi[i].gpart + P.gpart_off, 1ull << (n - P.T), P.ngrad, 0u, outp + slot});
                    slot += P.ngrad;
                }
            }
        }
        if (tasks.size() > (size_t)count * 64 + 16) { err = "too many reduction tasks"; return SV_EUNSUPPORTED; }
        std::memcpy(hp + o_items1, bi.data(), bi.size() * sizeof(BItem));
        if (!recs[1].empty()) std::memcpy(hp + o_recs1, recs[1].data(), recs[1].size() * sizeof(BRec));
        std::memcpy(hp + o_tasks, tasks.data(), tasks.size() * sizeof(Task));
        // upload on a side stream so the copy overlaps the first launch; the
        // stream waits for it before the second launch
        if (!ds.up) {
            he = hipStreamCreateWithFlags(&ds.up, hipStreamNonBlocking);
            if (he == hipSuccess) he = hipEventCreateWithFlags(&ds.ev, hipEventDisableTiming);
            if (he != hipSuccess) { err = std::string("upload stream: ") + hipGetErrorString(he); return SV_EDEVICE; }
        }
        he = hipMemcpyAsync(D1, hp, LA[1].up, hipMemcpyHostToDevice, ds.up);
        if (he == hipSuccess) he = hipEventRecord(ds.ev, ds.up);
        if (he == hipSuccess) he = hipStreamWaitEvent(stream, ds.ev, 0);
        if (he != hipSuccess) { err = std::string("upload: ") + hipGetErrorString(he); return SV_EDEVICE; }
    }
    st = launch(1, D1, o_items1, o_recs1, o_cnt1);
    if (st != SV_OK) return st;
    he = launch_multi_sum(reinterpret_cast<const void*>(D1 + o_tasks), (uint32_t)tasks.size(), stream);
    if (he != hipSuccess) { err = std::string("reduction launch: ") + hipGetErrorString(he); return SV_EDEVICE; }
    // results (outputs, then the two wait-error flags) into the slot's pinned buffer
    const size_t rbytes = nout * sizeof(double) + 2 * sizeof(uint32_t);
    if (sl.res.bytes < rbytes) {
        if (sl.res.p) (void)hipHostFree(sl.res.p);
        sl.res.p = nullptr;
        sl.res.bytes = 0;
        const size_t want = align_up(rbytes + rbytes / 4, (size_t)1 << 16);
        if (hipHostMalloc(&sl.res.p, want, hipHostMallocDefault) == hipSuccess) sl.res.bytes = want;
        else sl.res.p = nullptr;
    }
    unsigned char* rp = nullptr;
    if (sl.res.p) {
        rp = reinterpret_cast<unsigned char*>(sl.res.p);
    } else {
        job.outv.assign((rbytes + sizeof(double) - 1) / sizeof(double), 0.0);
        rp = reinterpret_cast<unsigned char*>(job.outv.data());
    }
    double* outp_h = reinterpret_cast<double*>(rp);
    uint32_t* flags_h = reinterpret_cast<uint32_t*>(rp + nout * sizeof(double));
    flags_h[0] = flags_h[1] = 0;
    he = hipMemcpyAsync(outp_h, S1 + o_out, nout * sizeof(double), hipMemcpyDeviceToHost, stream);
    for (int ph = 0; ph < 2; ++ph)
        if (he == hipSuccess && !recs[ph].empty())
            he = hipMemcpyAsync(&flags_h[ph], BA[ph].err, 4, hipMemcpyDeviceToHost, stream);
    if (he == hipSuccess && !sl.done) he = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventRecord(sl.done, stream);
    if (he != hipSuccess) { err = std::string("batch: ") + hipGetErrorString(he); return SV_EDEVICE; }
    job.nout = nout;
    job.out = outp_h;
    job.errflag = flags_h;
    job.nparams.resize((size_t)count);
    job.pb.resize((size_t)count);
    for (int i = 0; i < count; ++i) {
        job.nparams[i] = items[i].circuit->n_params;
        if (grad) job.pb[i] = H[i].pb;
    }
    job.gslot0 = gslot0;
    sv_stats& sts = job.stats;
    std::memset(&sts, 0, sizeof(sts));
    for (int i = 0; i < count; ++i) {
        sts.gates_in += items[i].circuit->n_gates;
        sts.passes += (int32_t)H[i].pf->ep.passes.size() + (grad ? (int32_t)H[i].pb->ep.passes.size() : 0);
        sts.alu_ops += H[i].pf->ep.alu_ops + (grad ? H[i].pb->ep.alu_ops : 0.0);
    }
    sts.launches = (recs[0].empty() ? 0 : 1) + (recs[1].empty() ? 0 : 1) + 1;
    sts.plan_ms = prep_ms;
    double bytes = 0.0;
    for (int ph = 0; ph < 2; ++ph)
        for (const BRec& r : recs[ph])
            bytes += (double)ab * std::ldexp(1.0, items[r.item].circuit->n_qubits) * (r.kind == BK_BWD ? 4.0 : 2.0);
    sts.hbm_bytes = bytes;
    guard.keep = true;
    return SV_OK;
}

// Wait for a launched job, turn its reduced outputs into energies and
// gradients (the backward plans' slot order and scale factors), release its
// slot.  energies / grads may be NULL when not wanted.
sv_status batch_finish(BatchJob& job, double* energies, double* grads, sv_stats* stats, std::string& err) {
    if (job.immediate) {
        if (energies && job.want_e) std::copy(job.e.begin(), job.e.end(), energies);
        if (grads && job.grad) std::copy(job.g.begin(), job.g.end(), grads);
        if (stats) *stats = job.stats;
        return SV_OK;
    }
    Slot* sl = nullptr;
    hipStream_t up = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        DevState& ds = g_dev[job.dev];
        sl = &ds.slot[job.slot];
        up = ds.up;
    }
    sv_status st = SV_OK;
    const hipError_t he = hipEventSynchronize(sl->done);
    if (he != hipSuccess) {
        err = std::string("batch: ") + hipGetErrorString(he);
        st = SV_EDEVICE;
    } else if (job.errflag[0] || job.errflag[1]) {
        err = "persistent batch: a dependency wait exceeded its time budget";
        st = SV_EDEVICE;
    } else {
        size_t goff = 0;
        for (int i = 0; i < job.count; ++i) {
            if (energies && job.want_e) energies[i] = job.out[i];
            if (job.grad && grads) {
                const int np = job.nparams[i];
                for (int p = 0; p < np; ++p) grads[goff + p] = 0.0;
                const EncodedPlan& B = job.pb[i]->ep;
                for (int k = 0; k < B.ngrad_total; ++k)
                    grads[goff + B.grad_param[k]] += B.grad_scale[k] * job.out[job.gslot0[i] + k];
                goff += (size_t)np;
            }
        }
        if (stats) *stats = job.stats;
    }
    if (st != SV_OK) {
        (void)hipStreamSynchronize(job.stream);
        if (up) (void)hipStreamSynchronize(up);
    }
    std::lock_guard<std::mutex> lk(g_stage_mu);
    sl->busy = false;
    return st;
}

sv_status run_batch_persistent(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream,
                               int32_t flags, double* energies, double* grads, const sv_opts* opts,
                               sv_stats* stats, std::string& err, const GeomTable* geoms) {
    if ((flags & SV_BATCH_GRAD) && (!energies || !grads)) { err = "energies and grads are required"; return SV_EINVAL; }
    BatchJob job;
    const sv_status st = batch_launch(count, items, dtype, stream, flags, energies != nullptr, opts, err, geoms, job);
    if (st != SV_OK) return st;
    return batch_finish(job, energies, grads, stats, err);
}

// Opaque jobs for the asynchronous entry points.
sv_status batch_launch_async(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream,
                             int32_t flags, const sv_opts* opts, std::string& err, const GeomTable* geoms,
                             void** job_out) {
    auto job = std::make_unique<BatchJob>();
    const sv_status st = batch_launch(count, items, dtype, stream, flags, (flags & SV_BATCH_ENERGY) != 0, opts, err,
                                      geoms, *job);
    if (st != SV_OK) return st;
    *job_out = job.release();
    return SV_OK;
}

sv_status batch_finish_async(void* job, double* energies, double* grads, sv_stats* stats, std::string& err) {
    std::unique_ptr<BatchJob> j(static_cast<BatchJob*>(job));
    if (j->grad && (!energies || !grads)) {
        // still wait for the job and release its slot
        std::string ignore;
        (void)batch_finish(*j, nullptr, nullptr, nullptr, ignore);
        err = "energies and grads are required";
        return SV_EINVAL;
    }
    if (j->want_e && !energies) {
        std::string ignore;
        (void)batch_finish(*j, nullptr, nullptr, nullptr, ignore);
        err = "energies is NULL";
        return SV_EINVAL;
    }
    return batch_finish(*j, energies, grads, stats, err);
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
            // Tiles no larger than the default: the launch gives every
            // workgroup the LDS of its largest tile, so a larger tile for one
            // width (faster when that width is timed alone) would cut the
            // occupancy of all the others in a mixed batch.
            const int tdef = dtype == SV_C64 ? 12 : (grad ? 11 : 12);
            const BatchGeom base = best;
            for (int T = 11; T < std::min(tdef, w + 1) && st == SV_OK; ++T) {
                BatchGeom g = base;
                g.T = T;
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
