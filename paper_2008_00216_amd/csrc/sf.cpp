// Schroedinger-Feynman mode (Sec. 1 and Sec. 6: the paper accelerates the
// Schroedinger sweeps inside Schroedinger-Feynman simulation, whose details
// are in a separate paper; this mode is built from the mathematics of the
// path sum).
//
// The register is cut into two halves A and B.  A gate across the cut is a
// sum of two products of one-half operators,
//   CZ(a, b)    = |0><0|_a (x) I_b + |1><1|_a (x) Z_b,
//   CP(a, b; p) = |0><0|_a (x) I_b + |1><1|_a (x) P(p)_b,
//   CNOT(c, t)  = |0><0|_c (x) I_t + |1><1|_c (x) X_t,
// so the circuit is a sum over 2^c paths (one bit per cross gate) of
// products A_s (x) B_s of half-width states, each the result of a
// half-width Schroedinger sweep:  psi[j] = sum_s A_s[jA] B_s[jB].
//
// GPU layout.  The path bits are held as extra high qubits of each half
// ("ancillas"): cross gate k adds qubit n_S + k to side S.  Before its cross
// gate an ancilla is |0>, so the sweep runs on the 2^(n_S + m) amplitudes of
// the m ancillas that exist so far; at the cross gate the half's buffer is
// doubled by a copy (both path values start from the same state, so every
// gate before the cut is applied once for all the paths that share it) and
// the cross gate's half operator becomes an ordinary gate on (ancilla,
// qubit): the projector side keeps the amplitudes whose qubit equals the
// ancilla (an explicit 2-qubit diagonal), the other side applies the
// controlled Z, phase or X from the ancilla.  Every sweep is the library's
// tile-pass sweep of a wider state.  When the buffers do not fit the work
// area, the last cross gates are enumerated instead (one path assignment at
// a time, restarting from a checkpoint of both halves taken at the first of
// them), and their half operators are fixed one-qubit gates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstring>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "host.h"
#include "kernels.h"
#include "sv.h"

namespace svmi {
sv_status sf_fail(sv_status st, const std::string& msg);
sv_status prepare_apply(sv_ctx c, const sv_circuit* circ, const double* params, uint64_t first_pin);
sv_status set_input_copy(sv_ctx c, int bit);
}

namespace {

using svmi::cd;

enum { XK_CZ = 0, XK_CP = 1, XK_CNOT = 2 };

struct Cross {
    int kind = XK_CZ;
    int proj_side = 0;      // side holding the projector (control)
    int qp = 0, qo = 0;     // local qubit on the projector side / the other side
    int param = -1;
    double theta = 0.0;
};

// One half-width circuit under construction (local qubit numbering).
struct SideCirc {
    std::vector<sv_gate> gates;
    std::vector<double> mats;
    sv_circuit view(int n, int n_params) const {
        sv_circuit c;
        c.n_qubits = n;
        c.n_gates = (int32_t)gates.size();
        c.gates = gates.data();
        c.n_mat_doubles = (int64_t)mats.size();
        c.mats = mats.empty() ? nullptr : mats.data();
        c.n_params = n_params;
        return c;
    }
};

// A gate of the suffix whose entries depend on the assignment of an
// enumerated path bit: offset of its doubles in the suffix's mats.
struct Slot {
    int side = 0;
    int cross = 0;          // cross-gate index
    bool proj = false;      // projector half of the gate
    size_t off = 0;
};

sv_gate mk_gate(int op, std::initializer_list<int> qs, int param = -1, double theta = 0.0, int mat = -1) {
    sv_gate g;
    std::memset(&g, 0, sizeof(g));
    g.op = op;
    g.nq = (int32_t)qs.size();
    int t = 0;
    for (int q : qs) g.q[t++] = q;
    g.param = param;
    g.theta = theta;
    g.mat = mat;
    return g;
}

struct SfPlan {
    int n = 0, nS[2] = {0, 0};
    int ncross = 0, ninner = 0, n_params = 0;
    std::vector<int> loc;                 // qubit -> local index on its side
    uint64_t mask = 0;                    // qubits of side A
    std::vector<Cross> cross;
    std::vector<SideCirc> pre[2];         // prefix segment m runs at width nS + m
    SideCirc suf[2];                      // after the first enumerated cross gate (width nS + ninner)
    std::vector<Slot> slots;
    bool has_suffix() const { return ncross > ninner; }
};

size_t need_bytes(const SfPlan& p, int ninner, size_t ab) {
    const size_t half = ((size_t)1 << (p.nS[0] + ninner)) + ((size_t)1 << (p.nS[1] + ninner));
    return half * ab * (ninner < p.ncross ? 2 : 1);
}

// Split the circuit into the two halves; fills everything but the segments.
std::string split(const sv_circuit* c, uint64_t mask, SfPlan& p) {
    const int n = c->n_qubits;
    const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1);
    if ((mask & ~all) != 0) return "half mask names qubits outside the register";
    p.n = n;
    p.mask = mask;
    p.n_params = c->n_params;
    p.loc.assign((size_t)n, 0);
    for (int q = 0; q < n; ++q) {
        const int s = ((mask >> q) & 1) ? 0 : 1;
        p.loc[q] = p.nS[s]++;
    }
    if (p.nS[0] < 1 || p.nS[1] < 1) return "each half needs at least one qubit";
    for (int i = 0; i < c->n_gates; ++i) {
        const sv_gate& g = c->gates[i];
        int sides = 0;
        for (int t = 0; t < g.nq; ++t) sides |= 1 << (((mask >> g.q[t]) & 1) ? 0 : 1);
        if (sides != 3) continue;
        Cross x;
        if (g.op == SV_OP_CZ || g.op == SV_OP_CP) {
            x.kind = g.op == SV_OP_CZ ? XK_CZ : XK_CP;
            const int sa = ((mask >> g.q[0]) & 1) ? 0 : 1;
            const int qa = sa == 0 ? g.q[0] : g.q[1], qb = sa == 0 ? g.q[1] : g.q[0];
            x.proj_side = 0;
            x.qp = p.loc[qa];
            x.qo = p.loc[qb];
            x.param = g.param;
            x.theta = g.theta;
        } else if (g.op == SV_OP_CNOT) {
            x.kind = XK_CNOT;
            x.proj_side = ((mask >> g.q[0]) & 1) ? 0 : 1;
            x.qp = p.loc[g.q[0]];
            x.qo = p.loc[g.q[1]];
        } else {
            std::ostringstream e;
            e << "gate " << i << " (op " << g.op << ") crosses the cut: only CZ, CP and CNOT can";
            return e.str();
        }
        p.cross.push_back(x);
    }
    p.ncross = (int)p.cross.size();
    return "";
}

// Build the segments for `ninner` path bits held in memory.
void build_segments(const sv_circuit* c, SfPlan& p, int ninner) {
    p.ninner = ninner;
    for (int s = 0; s < 2; ++s) {
        p.pre[s].assign((size_t)ninner + 1, SideCirc{});
        p.suf[s] = SideCirc{};
    }
    p.slots.clear();
    int k = 0;                                  // next cross gate
    const uint64_t mask = p.mask;
    for (int i = 0; i < c->n_gates; ++i) {
        const sv_gate& g = c->gates[i];
        int sides = 0;
        for (int t = 0; t < g.nq; ++t) sides |= 1 << (((mask >> g.q[t]) & 1) ? 0 : 1);
        if (sides != 3) {
            const int s = sides == 1 ? 0 : 1;
            // gates after the first enumerated cross gate belong to the suffix
            SideCirc& dst = (k > ninner) ? p.suf[s] : p.pre[s][(size_t)k];
            sv_gate h = g;
            for (int t = 0; t < g.nq; ++t) h.q[t] = p.loc[g.q[t]];
            if (g.op == SV_OP_MAT || g.op == SV_OP_DIAG) {
                const int d = 1 << g.nq;
                const size_t nd = (size_t)2 * d * (g.op == SV_OP_MAT ? d : 1);
                h.mat = (int32_t)dst.mats.size();
                dst.mats.insert(dst.mats.end(), c->mats + g.mat, c->mats + g.mat + nd);
            }
            dst.gates.push_back(h);
            continue;
        }
        const Cross& x = p.cross[(size_t)k];
        if (k < ninner) {
            // held in memory: ancilla nS + k of both sides, segment k + 1 starts here
            for (int s = 0; s < 2; ++s) {
                SideCirc& dst = p.pre[s][(size_t)k + 1];
                const int anc = p.nS[s] + k;
                if (s == x.proj_side) {
                    dst.gates.push_back(mk_gate(SV_OP_DIAG, {x.qp, anc}, -1, 0.0, (int)dst.mats.size()));
                    const double d[8] = {1, 0, 0, 0, 0, 0, 1, 0};   // keep the amplitudes with qubit == ancilla
                    dst.mats.insert(dst.mats.end(), d, d + 8);
                } else if (x.kind == XK_CZ) {
                    dst.gates.push_back(mk_gate(SV_OP_CZ, {anc, x.qo}));
                } else if (x.kind == XK_CP) {
                    dst.gates.push_back(mk_gate(SV_OP_CP, {anc, x.qo}, x.param, x.theta));
                } else {
                    dst.gates.push_back(mk_gate(SV_OP_CNOT, {anc, x.qo}));
                }
            }
        } else {
            // enumerated: a fixed one-qubit gate per side, entries per assignment
            for (int s = 0; s < 2; ++s) {
                SideCirc& dst = p.suf[s];
                Slot sl;
                sl.side = s;
                sl.cross = k;
                sl.proj = s == x.proj_side;
                sl.off = dst.mats.size();
                if (sl.proj || x.kind != XK_CNOT) {
                    dst.gates.push_back(mk_gate(SV_OP_DIAG, {sl.proj ? x.qp : x.qo}, -1, 0.0, (int)sl.off));
                    dst.mats.insert(dst.mats.end(), 4, 0.0);
                } else {
                    dst.gates.push_back(mk_gate(SV_OP_MAT, {x.qo}, -1, 0.0, (int)sl.off));
                    dst.mats.insert(dst.mats.end(), 8, 0.0);
                }
                p.slots.push_back(sl);
            }
        }
        ++k;
    }
}

// Entries of the enumerated gates for one assignment of their path bits.
void fill_slots(SfPlan& p, uint64_t sigma, const double* params) {
    for (const Slot& sl : p.slots) {
        const int bit = (int)((sigma >> (sl.cross - p.ninner)) & 1ull);
        const Cross& x = p.cross[(size_t)sl.cross];
        double* m = p.suf[sl.side].mats.data() + sl.off;
        if (sl.proj) {                                   // |bit><bit|
            m[0] = bit ? 0.0 : 1.0; m[1] = 0.0;
            m[2] = bit ? 1.0 : 0.0; m[3] = 0.0;
        } else if (x.kind == XK_CZ) {                    // Z^bit
            m[0] = 1.0; m[1] = 0.0;
            m[2] = bit ? -1.0 : 1.0; m[3] = 0.0;
        } else if (x.kind == XK_CP) {                    // P(theta)^bit
            const double th = x.param >= 0 ? params[x.param] : x.theta;
            m[0] = 1.0; m[1] = 0.0;
            m[2] = bit ? std::cos(th) : 1.0; m[3] = bit ? std::sin(th) : 0.0;
        } else {                                         // X^bit
            const double d = bit ? 0.0 : 1.0, o = bit ? 1.0 : 0.0;
            const double v[8] = {d, 0, o, 0, o, 0, d, 0};
            std::copy(v, v + 8, m);
        }
    }
}

size_t amp_bytes(int dt) { return dt == SV_C64 ? 8 : 16; }

int max_width(int dt) { return dt == SV_C64 ? 34 : 33; }

// Largest number of path bits held in memory that fits work_bytes.
int choose_inner(const SfPlan& p, int dt, size_t work_bytes) {
    const size_t ab = amp_bytes(dt);
    for (int m = p.ncross; m >= 0; --m) {
        if (p.nS[0] + m > max_width(dt) || p.nS[1] + m > max_width(dt)) continue;
        if (need_bytes(p, m, ab) <= work_bytes) return m;
    }
    return -1;
}

uint64_t pext(uint64_t x, uint64_t m) {
    uint64_t r = 0;
    int b = 0;
    for (int q = 0; q < 64; ++q)
        if ((m >> q) & 1) {
            if ((x >> q) & 1) r |= 1ull << b;
            ++b;
        }
    return r;
}

}  // namespace

struct sv_sf_s {
    SfPlan plan;
    int dtype = SV_C64;
    hipStream_t stream = nullptr;
    sv_opts opts{};
    unsigned char* work = nullptr;
    size_t work_bytes = 0;
    size_t off[2] = {0, 0}, ck[2] = {0, 0};       // half buffers and their checkpoints
    std::vector<sv_ctx> ctx[2];                    // widths nS .. nS + ninner
    void* d_idx = nullptr;                         // jA, jB, accumulators
    size_t d_idx_bytes = 0;
    bool prepared = false;
    ~sv_sf_s() {
        for (int s = 0; s < 2; ++s)
            for (sv_ctx c : ctx[s]) if (c) sv_destroy(c);
        if (d_idx) (void)hipFree(d_idx);
    }
};

namespace {

void add_stats(sv_stats* dst, const sv_stats& s) {
    if (!dst) return;
    dst->passes += s.passes;
    dst->phases += s.phases;
    dst->dense_ops += s.dense_ops;
    dst->diag_ops += s.diag_ops;
    dst->launches += s.launches;
    dst->folded_init += s.folded_init;
    dst->plan_ms += s.plan_ms;
    dst->hbm_bytes += s.hbm_bytes;
    dst->flops += s.flops;
    dst->alu_ops += s.alu_ops;
}

}  // namespace

extern "C" {

sv_status sv_sf_plan(const sv_circuit* circ, uint64_t half_mask, sv_dtype dtype, size_t work_bytes,
                     sv_sf_info* info) {
    using svmi::sf_fail;
    if (!circ || !info) return sf_fail(SV_EINVAL, "circuit or info is NULL");
    if (dtype != SV_C64 && dtype != SV_C128) return sf_fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    std::string v = svmi::validate_circuit(circ, circ->n_qubits);
    if (!v.empty()) return sf_fail(SV_EINVAL, v);
    SfPlan p;
    v = split(circ, half_mask, p);
    if (!v.empty()) return sf_fail(SV_EUNSUPPORTED, v);
    std::memset(info, 0, sizeof(*info));
    info->n_qubits = p.n;
    info->n_a = p.nS[0];
    info->n_b = p.nS[1];
    info->n_cross = p.ncross;
    info->paths = std::ldexp(1.0, p.ncross);
    const size_t ab = amp_bytes(dtype);
    info->work_bytes_all_inner = need_bytes(p, p.ncross, ab);
    info->work_bytes_min = need_bytes(p, 0, ab);
    const int m = choose_inner(p, dtype, work_bytes);
    info->n_inner = m;
    info->n_outer = m < 0 ? -1 : p.ncross - m;
    return SV_OK;
}

sv_status sv_sf_create(sv_sf* out, const sv_circuit* circ, uint64_t half_mask, sv_dtype dtype, void* d_work,
                       size_t work_bytes, void* hip_stream, const sv_opts* opts) {
    using svmi::sf_fail;
    if (!out) return sf_fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    if (!circ || !d_work) return sf_fail(SV_EINVAL, "circuit or d_work is NULL");
    if ((uintptr_t)d_work % 256 != 0) return sf_fail(SV_EINVAL, "d_work must be 256-byte aligned");
    if (dtype != SV_C64 && dtype != SV_C128) return sf_fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    std::string v = svmi::validate_circuit(circ, circ->n_qubits);
    if (!v.empty()) return sf_fail(SV_EINVAL, v);
    auto* f = new (std::nothrow) sv_sf_s();
    if (!f) return sf_fail(SV_ENOMEM, "allocation failed");
    v = split(circ, half_mask, f->plan);
    if (!v.empty()) { delete f; return sf_fail(SV_EUNSUPPORTED, v); }
    const int m = choose_inner(f->plan, dtype, work_bytes);
    if (m < 0) {
        std::ostringstream e;
        e << "work area of " << work_bytes << " bytes holds no path split (need at least "
          << need_bytes(f->plan, 0, amp_bytes(dtype)) << ")";
        delete f;
        return sf_fail(SV_EINVAL, e.str());
    }
    build_segments(circ, f->plan, m);
    f->dtype = dtype;
    f->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (opts) f->opts = *opts; else sv_opts_default(&f->opts);
    f->work = reinterpret_cast<unsigned char*>(d_work);
    f->work_bytes = work_bytes;
    const size_t ab = amp_bytes(dtype);
    const SfPlan& p = f->plan;
    const size_t hb[2] = {((size_t)1 << (p.nS[0] + m)) * ab, ((size_t)1 << (p.nS[1] + m)) * ab};
    f->off[0] = 0;
    f->off[1] = hb[0];
    f->ck[0] = hb[0] + hb[1];
    f->ck[1] = f->ck[0] + hb[0];
    for (int s = 0; s < 2; ++s) {
        f->ctx[s].assign((size_t)m + 1, nullptr);
        for (int w = 0; w <= m; ++w) {
            sv_status st = sv_create(&f->ctx[s][(size_t)w], p.nS[s] + w, dtype, 1, f->work + f->off[s],
                                     ((size_t)1 << (p.nS[s] + w)) * ab, hip_stream, &f->opts);
            if (st != SV_OK) { delete f; return st; }
        }
    }
    *out = f;
    return SV_OK;
}

sv_status sv_sf_destroy(sv_sf f) {
    if (!f) return svmi::sf_fail(SV_EINVAL, "sf is NULL");
    (void)hipStreamSynchronize(f->stream);
    delete f;
    return SV_OK;
}

sv_status sv_sf_amplitudes(sv_sf f, const double* params, int64_t count, const uint64_t* indices, double* out,
                           sv_stats* stats) {
    using svmi::sf_fail;
    if (!f) return sf_fail(SV_EINVAL, "sf is NULL");
    if (count < 0) return sf_fail(SV_EINVAL, "count < 0");
    if (count > 0 && (!indices || !out)) return sf_fail(SV_EINVAL, "indices or out is NULL");
    SfPlan& p = f->plan;
    if (p.n_params > 0 && !params) return sf_fail(SV_EINVAL, "circuit has parameters but params is NULL");
    for (int i = 0; p.n_params > 0 && i < p.n_params; ++i)
        if (!std::isfinite(params[i])) return sf_fail(SV_EINVAL, "non-finite parameter");
    const uint64_t top = p.n >= 64 ? ~0ull : ((1ull << p.n) - 1);
    for (int64_t k = 0; k < count; ++k)
        if (indices[k] & ~top) return sf_fail(SV_EINVAL, "amplitude index out of range");
    if (stats) std::memset(stats, 0, sizeof(*stats));
    const size_t ab = amp_bytes(f->dtype);
    const int m = p.ninner;
    // requested amplitudes -> (jA, jB) on the device, FP64 accumulators
    const size_t nidx = (size_t)std::max<int64_t>(count, 1);
    const size_t need = nidx * (2 * sizeof(uint64_t) + 2 * sizeof(double));
    if (f->d_idx_bytes < need) {
        if (f->d_idx) (void)hipFree(f->d_idx);
        f->d_idx = nullptr;
        f->d_idx_bytes = 0;
        hipError_t e = hipMalloc(&f->d_idx, need);
        if (e != hipSuccess) { (void)hipGetLastError(); return sf_fail(SV_ENOMEM, "hipMalloc of the index buffers failed"); }
        f->d_idx_bytes = need;
    }
    std::vector<uint64_t> hj(2 * nidx, 0);
    const uint64_t mb = top & ~p.mask;
    for (int64_t k = 0; k < count; ++k) {
        hj[(size_t)k] = pext(indices[k], p.mask);
        hj[nidx + (size_t)k] = pext(indices[k], mb);
    }
    uint64_t* d_j = reinterpret_cast<uint64_t*>(f->d_idx);
    double* d_acc = reinterpret_cast<double*>(d_j + 2 * nidx);
    auto hip_fail = [&](const char* what, hipError_t e) {
        (void)hipGetLastError();
        return sf_fail(e == hipErrorOutOfMemory ? SV_ENOMEM : SV_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t he = hipMemcpyAsync(d_j, hj.data(), 2 * nidx * sizeof(uint64_t), hipMemcpyHostToDevice, f->stream);
    if (he != hipSuccess) return hip_fail("index upload", he);
    for (int s = 0; s < 2; ++s) {
        sv_status st = sv_init(f->ctx[s][0], SV_INIT_ZERO_DEFERRED, 0);
        if (st != SV_OK) return st;
    }
    if (!f->prepared) {
        // plan (and compile) every segment of both halves up front, several
        // contexts at a time, instead of one after the other as they run
        if (p.has_suffix()) fill_slots(p, 0, params);
        // a segment after a doubling is planned with its path qubit local in
        // the first pass, which then reads the doubling instead of a copy
        struct Task { sv_ctx c; sv_circuit cv; uint64_t pin; };
        std::vector<Task> tasks;
        for (int s = 0; s < 2; ++s) {
            for (int w = 0; w <= m; ++w)
                if (!p.pre[s][(size_t)w].gates.empty() || w == 0)
                    tasks.push_back({f->ctx[s][(size_t)w], p.pre[s][(size_t)w].view(p.nS[s] + w, p.n_params),
                                     w > 0 ? 1ull << (p.nS[s] + w - 1) : 0ull});
            if (p.has_suffix())
                tasks.push_back({f->ctx[s][(size_t)m], p.suf[s].view(p.nS[s] + m, p.n_params), 0ull});
        }
        std::vector<sv_status> res(tasks.size(), SV_OK);
        std::vector<std::string> msg(tasks.size());
        size_t next = 0;
        std::mutex mu;
        std::vector<std::thread> th;
        const int nthr = (int)std::min<size_t>(4, tasks.size());
        for (int t = 0; t < nthr; ++t)
            th.emplace_back([&] {
                for (;;) {
                    size_t i;
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        if (next >= tasks.size()) return;
                        i = next++;
                    }
                    res[i] = svmi::prepare_apply(tasks[i].c, &tasks[i].cv, params, tasks[i].pin);
                    if (res[i] != SV_OK) msg[i] = sv_last_error();
                }
            });
        for (auto& t : th) t.join();
        for (size_t i = 0; i < tasks.size(); ++i)
            if (res[i] != SV_OK) return sf_fail(res[i], "preparing a half-width sweep: " + msg[i]);
        f->prepared = true;
    }
    // prefix: segment w at width nS + w; the buffer doubles before each w >= 1
    for (int s = 0; s < 2; ++s) {
        sv_status st = SV_OK;
        for (int w = 0; w <= m; ++w) {
            const SideCirc& sc = p.pre[s][(size_t)w];
            if (w > 0) {
                if (!sc.gates.empty()) {
                    // the segment's sweep reads the lower half for both halves
                    // when its first pass holds the new ancilla locally, and
                    // writes the copy first otherwise
                    st = svmi::set_input_copy(f->ctx[s][(size_t)w], p.nS[s] + w - 1);
                    if (st != SV_OK) return st;
                } else {
                    const size_t bytes = ((size_t)1 << (p.nS[s] + w - 1)) * ab;
                    he = svmi::launch_copy(f->work + f->off[s], f->work + f->off[s] + bytes, bytes, f->stream);
                    if (he != hipSuccess) return hip_fail("path doubling copy", he);
                    if (stats) { stats->hbm_bytes += 2.0 * (double)bytes; stats->launches += 1; }
                }
            }
            if (sc.gates.empty() && w > 0) continue;
            sv_circuit cv = sc.view(p.nS[s] + w, p.n_params);
            sv_stats ss{};
            st = sv_apply_circuit(f->ctx[s][(size_t)w], &cv, params, &ss);
            if (st != SV_OK) return st;
            add_stats(stats, ss);
        }
    }
    const uint64_t npath = 1ull << m;
    const size_t hb[2] = {((size_t)1 << (p.nS[0] + m)) * ab, ((size_t)1 << (p.nS[1] + m)) * ab};
    const uint64_t nsigma = p.has_suffix() ? (1ull << (p.ncross - m)) : 1ull;
    if (p.has_suffix()) {
        for (int s = 0; s < 2; ++s) {
            he = svmi::launch_copy(f->work + f->off[s], f->work + f->ck[s], hb[s], f->stream);
            if (he != hipSuccess) return hip_fail("checkpoint copy", he);
            if (stats) { stats->hbm_bytes += 2.0 * (double)hb[s]; stats->launches += 1; }
        }
    }
    for (uint64_t sg = 0; sg < nsigma; ++sg) {
        if (p.has_suffix()) {
            fill_slots(p, sg, params);
            for (int s = 0; s < 2; ++s) {
                if (sg > 0) {
                    he = svmi::launch_copy(f->work + f->ck[s], f->work + f->off[s], hb[s], f->stream);
                    if (he != hipSuccess) return hip_fail("checkpoint restore", he);
                    if (stats) { stats->hbm_bytes += 2.0 * (double)hb[s]; stats->launches += 1; }
                }
                sv_circuit cv = p.suf[s].view(p.nS[s] + m, p.n_params);
                sv_stats ss{};
                sv_status st = sv_apply_circuit(f->ctx[s][(size_t)m], &cv, params, &ss);
                if (st != SV_OK) return st;
                add_stats(stats, ss);
            }
        }
        he = svmi::launch_sf_contract(f->dtype, f->work + f->off[0], f->work + f->off[1], p.nS[0], p.nS[1], npath,
                                      d_j, d_j + nidx, (uint64_t)count, d_acc, sg > 0 ? 1 : 0, f->stream);
        if (he != hipSuccess) return hip_fail("path contraction", he);
        if (stats) {
            stats->hbm_bytes += (double)count * (double)npath * 2.0 * (double)ab;
            stats->launches += 1;
        }
    }
    if (count > 0) {
        he = hipMemcpyAsync(out, d_acc, (size_t)count * 2 * sizeof(double), hipMemcpyDeviceToHost, f->stream);
        if (he != hipSuccess) return hip_fail("result copy", he);
    }
    he = hipStreamSynchronize(f->stream);
    if (he != hipSuccess) return hip_fail("stream synchronise", he);
    return SV_OK;
}

}  // extern "C"
