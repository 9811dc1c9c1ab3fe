// Simulation planner: IR gates -> tile passes -> register phases -> ops.
//
// Pass formation reuses the reordering scan of Sec. 4.5.  Walking the
// remaining gates in order, every qubit is "unobstructed" until a gate that
// cannot be executed touches it; then it is "obstructed" and no later gate on
// it may move ahead.  Diagonal gates commute with each other (Sec. 4.2), so a
// pending diagonal only obstructs later non-diagonal gates.  For a candidate
// set S of local qubits, a gate is executable in the pass when it is
// unobstructed and either diagonal with 8th-root phases (any qubits: the
// kernel knows every amplitude's full index) or all its qubits are in S.  The
// greedy S of a pass comes from demand and then a swap-based local search on
// the number of gates executed; a beam search over whole sequences of such
// sets (the greedy set and its best single swaps at every step) then looks
// for fewer passes.  Register phases inside a pass are chosen the same way
// over 4-subsets of the local bits.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <stdexcept>

#include "device_common.h"
#include "host.h"

namespace svmi {

namespace {

enum Cls { C_FREE = 0, C_LOCAL = 1, C_BIG = 2 };

struct GInfo {
    uint64_t qm = 0;
    int cls = C_LOCAL;
    bool diag = false;   // commutes with other diagonals
    double w = 1.0;
};

GInfo info_of(const IRGate& g) {
    GInfo r;
    r.qm = g.qmask();
    if (g.kind == K_DIAG8 && !g.grad) {
        r.cls = C_FREE;
        r.diag = true;
        r.w = 0.05;
        return r;
    }
    if (g.grad) {
        r.cls = C_LOCAL;
        r.w = 0.5;
        return r;
    }
    if (g.kind == K_DIAGG) {
        r.cls = g.k <= kRegBits ? C_LOCAL : C_BIG;
        r.diag = true;
        r.w = 0.3;
        return r;
    }
    r.cls = g.k <= kRegBits ? C_LOCAL : C_BIG;
    r.w = g.skind ? 0.7 : (double)(1 << (g.k - 1));
    return r;
}

// Obstruction scan.  `allowed` = qubits (bits) executable for C_LOCAL gates.
// Returns score; fills `exec` if non-null.
double scan(const std::vector<int>& rem, const std::vector<GInfo>& inf, uint64_t allowed, uint64_t all,
            std::vector<int>* exec, int limit_local_fail = 1 << 30) {
    uint64_t bND = 0, bD = 0;
    double score = 0.0;
    int fails = 0;
    for (int id : rem) {
        const GInfo& g = inf[id];
        if (g.cls == C_FREE) {
            if (g.qm & bND) { bD |= g.qm; continue; }
            score += g.w;
            if (exec) exec->push_back(id);
            continue;
        }
        if (g.cls == C_BIG) {
            if (g.diag) bD |= g.qm; else bND |= g.qm;
        } else if (g.qm & (g.diag ? bND : (bND | bD))) {
            if (g.diag) bD |= g.qm; else bND |= g.qm;
        } else if ((g.qm & ~allowed) == 0) {
            score += g.w;
            if (exec) exec->push_back(id);
            continue;
        } else {
            if (g.diag) bD |= g.qm; else bND |= g.qm;
            if (++fails > limit_local_fail) break;
        }
        if ((bND & all) == all) break;
    }
    return score;
}

int popc(uint64_t x) { return __builtin_popcountll(x); }

// ---------------------------------------------------------------- forms

struct Form {
    int alpha[64];
    std::map<std::pair<int, int>, int> beta;  // (a<b) -> exponent mod 8
    int konst = 0;
    Form() { std::memset(alpha, 0, sizeof(alpha)); }
    bool empty() const {
        if (konst & 7) return false;
        for (int i = 0; i < 64; ++i) if (alpha[i] & 7) return false;
        for (auto& kv : beta) if (kv.second & 7) return false;
        return true;
    }
    bool depends(uint64_t qm) const {
        for (int i = 0; i < 64; ++i) if (((qm >> i) & 1) && (alpha[i] & 7)) return true;
        for (auto& kv : beta)
            if ((kv.second & 7) && (((qm >> kv.first.first) & 1) || ((qm >> kv.first.second) & 1))) return true;
        return false;
    }
    bool sign_only() const {
        if (konst & 3) return false;
        for (int i = 0; i < 64; ++i) if (alpha[i] & 3) return false;
        for (auto& kv : beta) if (kv.second & 3) return false;
        return true;
    }
    void add(const IRGate& g) {
        if (g.k == 1) {
            alpha[g.q[0]] = (alpha[g.q[0]] + g.alpha[0]) & 7;
        } else {
            alpha[g.q[0]] = (alpha[g.q[0]] + g.alpha[0]) & 7;
            alpha[g.q[1]] = (alpha[g.q[1]] + g.alpha[1]) & 7;
            int a = g.q[0], b = g.q[1];
            if (a > b) std::swap(a, b);
            int& v = beta[{a, b}];
            v = (v + g.beta) & 7;
        }
    }
    int beta_of(int a, int b) const {
        if (a > b) std::swap(a, b);
        auto it = beta.find({a, b});
        return it == beta.end() ? 0 : it->second & 7;
    }
    void clear() {
        std::memset(alpha, 0, sizeof(alpha));
        beta.clear();
        konst = 0;
    }
};

struct PassGeom {
    int L = 0, H = 0, T = 0;
    int hpos[16] = {0};
    int lpos[64];            // global qubit -> local position or -1
    int gq[kMaxTileBits];    // local position -> global qubit
};

PassGeom make_geom(int n, int L, uint64_t S) {
    PassGeom g;
    g.L = L;
    for (int q = 0; q < 64; ++q) g.lpos[q] = -1;
    int t = 0;
    for (int q = 0; q < L; ++q) { g.lpos[q] = q; g.gq[q] = q; }
    for (int q = L; q < n; ++q)
        if ((S >> q) & 1) {
            g.hpos[t] = q;
            g.lpos[q] = L + t;
            g.gq[L + t] = q;
            ++t;
        }
    g.H = t;
    g.T = L + t;
    return g;
}

template <class R>
void soff_for(const int r[4], uint16_t* soff) {
    for (int i = 0; i < kRegAmps; ++i) {
        uint32_t l = 0;
        for (int s = 0; s < 4; ++s)
            if ((i >> s) & 1) l |= 1u << r[s];
        soff[i] = (uint16_t)swz<R>(l);
    }
}

uint32_t deposit_skip(uint32_t x, const int r[4]) {
    for (int s = 0; s < 4; ++s) {
        const int p = r[s];
        x = ((x >> p) << (p + 1)) | (x & ((1u << p) - 1u));
    }
    return x;
}

// Encode a form for (pass geometry, phase registers) into out.
int encode_form(const Form& F, const PassGeom& G, const int r[4], int n, EncodedPlan& out, uint32_t slot) {
    DForm D;
    std::memset(&D, 0, sizeof(D));
    D.konst = (uint32_t)(F.konst & 7);
    D.slot = slot;
    const uint64_t localmask = [&] {
        uint64_t m = 0;
        for (int a = 0; a < G.T; ++a) m |= 1ull << G.gq[a];
        return m;
    }();
    // register table A[i]
    uint64_t A = 0;
    for (int i = 0; i < kRegAmps; ++i) {
        int e = 0;
        for (int s = 0; s < 4; ++s) {
            if (!((i >> s) & 1)) continue;
            e += F.alpha[G.gq[r[s]]];
            for (int s2 = s + 1; s2 < 4; ++s2)
                if ((i >> s2) & 1) e += F.beta_of(G.gq[r[s]], G.gq[r[s2]]);
        }
        A |= (uint64_t)(e & 7) << (3 * i);
    }
    D.a_lo = (uint32_t)A;
    D.a_hi = (uint32_t)(A >> 32);
    for (int i = 0; i < kRegAmps; ++i) D.abits |= (uint32_t)((A >> (3 * i + 2)) & 1u) << i;
    bool tile = false;
    // nonlocal linear terms and local <-> nonlocal pairs
    for (int q = 0; q < n; ++q) {
        if ((localmask >> q) & 1) continue;
        const int al = F.alpha[q] & 7;
        for (int c = 0; c < 3; ++c)
            if ((al >> c) & 1) { D.ka[c] |= 1ull << q; tile = true; }
    }
    for (auto& kv : F.beta) {
        const int v = kv.second & 7;
        if (!v) continue;
        const int a = kv.first.first, b = kv.first.second;
        const bool la = (localmask >> a) & 1, lb = (localmask >> b) & 1;
        if (la && lb) continue;
        tile = true;
        if (la != lb) {
            const int loc = la ? a : b, nl = la ? b : a;
            const int pa = G.lpos[loc];
            for (int c = 0; c < 3; ++c)
                if ((v >> c) & 1) D.mc[pa][c] |= 1ull << nl;
        }
    }
    // nonlocal-nonlocal pairs
    D.q0 = (uint32_t)out.pairs.size();
    std::map<int, DPair> pl;
    for (auto& kv : F.beta) {
        const int v = kv.second & 7;
        if (!v) continue;
        const int a = kv.first.first, b = kv.first.second;  // a < b
        if (((localmask >> a) & 1) || ((localmask >> b) & 1)) continue;
        DPair& p = pl[b];
        p.b = (uint32_t)b;
        for (int c = 0; c < 3; ++c)
            if ((v >> c) & 1) p.m[c] |= 1ull << a;
    }
    for (auto& kv : pl) out.pairs.push_back(kv.second);
    D.nq = (uint32_t)(out.pairs.size() - D.q0);
    D.has_tile = tile ? 1u : 0u;
    // thread-group table
    D.etab = (uint32_t)out.etab.size();
    const uint32_t ng = 1u << (G.T - kRegBits);
    std::vector<int> tau;
    for (int a = 0; a < G.T; ++a)
        if (a != r[0] && a != r[1] && a != r[2] && a != r[3]) tau.push_back(a);
    for (uint32_t gg = 0; gg < ng; ++gg) {
        const uint32_t lb = deposit_skip(gg, r);
        int e = 0;
        int d[4] = {0, 0, 0, 0};
        for (size_t i = 0; i < tau.size(); ++i) {
            const int a = tau[i];
            if (!((lb >> a) & 1)) continue;
            const int qa = G.gq[a];
            e += F.alpha[qa];
            for (size_t j = i + 1; j < tau.size(); ++j) {
                const int a2 = tau[j];
                if ((lb >> a2) & 1) e += F.beta_of(qa, G.gq[a2]);
            }
            for (int s = 0; s < 4; ++s) d[s] += F.beta_of(G.gq[r[s]], qa);
        }
        uint32_t v = (uint32_t)(e & 7);
        for (int s = 0; s < 4; ++s) v |= (uint32_t)(d[s] & 7) << (3 + 3 * s);
        out.etab.push_back((uint16_t)v);
    }
    out.forms.push_back(D);
    return (int)out.forms.size() - 1;
}

// Matrix slot permutation for a gate whose qubits sit on register slots.
void slot_perm(const IRGate& g, const int* slot_of_q, Recipe& rc, uint32_t& mask) {
    int s[6];
    mask = 0;
    for (int t = 0; t < g.k; ++t) {
        s[t] = slot_of_q[t];
        mask |= 1u << s[t];
    }
    // new local bit j <- the gate bit whose slot is the j-th smallest
    int order[6];
    for (int t = 0; t < g.k; ++t) order[t] = t;
    std::sort(order, order + g.k, [&](int a, int b) { return s[a] < s[b]; });
    for (int j = 0; j < g.k; ++j) rc.perm[j] = order[j];
    rc.k = g.k;
}

uint64_t add_recipe(EncodedPlan& out, Recipe rc, const std::vector<IRGate>& ir) {
    if (rc.type == Recipe::DENSE) {
        const int d = 1 << rc.k;
        rc.size = (uint64_t)d * d + (rc.inplace ? 11u : 0u);
        rc.varies = ir[rc.gate].m.nb > 1;
    } else if (rc.type == Recipe::DIAG) {
        rc.size = (uint64_t)1 << rc.k;
        rc.varies = ir[rc.gate].m.nb > 1;
    } else if (rc.type == Recipe::PHASETAB || rc.type == Recipe::BFTAB) {
        rc.size = 8;
    } else {
        rc.size = 1;
    }
    // keep matrices 16-byte friendly: no special alignment needed for V2
    rc.off = out.pool_size;
    out.pool_size += rc.size;
    if (rc.varies) out.pool_varies = true;
    out.recipes.push_back(rc);
    return rc.off;
}

// Butterflies between two applications of the accumulated 1/sqrt(2) factors:
// amplitudes grow by 2^60 at most in a forward sweep, and by 2^30 in an
// adjoint sweep, where the gradient terms multiply a psi and a lambda
// amplitude in the state's precision (FP32 for c64).  The factor is applied
// as soon as the count is reached, inside a pass if need be.
constexpr int kScaleEvery = 120;
constexpr int kScaleEveryAdjoint = 60;

double op_cost(const IRGate& g) {
    if (g.kind == K_DIAG8) return 0.0;
    if (g.grad) return 6.0;
    if (g.kind == K_DIAGG) return 6.0;
    if (g.skind) return 4.0;
    return 8.0 * (double)(1 << g.k);
}

}  // namespace

namespace {

// Planner trace: the plan's arithmetic in global-qubit terms, one op per line
// (pass/phase markers, butterflies with their twiddle and partner qubits,
// flushed phase forms, dense and diagonal blocks with their matrices, pass
// scales, gradient reductions).  Used to check the planner's algebra on the
// host against an independent evaluation.
void trace_matrix(std::string* tr, const char* tag, const IRGate& g, const std::string& partners = "") {
    if (!tr) return;
    char b[64];
    *tr += tag;
    std::snprintf(b, sizeof(b), " %d", g.k);
    *tr += b;
    for (int t = 0; t < g.k; ++t) { std::snprintf(b, sizeof(b), " %d", g.q[t]); *tr += b; }
    const cd* m = g.m.at(0);
    const size_t cnt = g.m.diag ? (size_t)g.m.d : (size_t)g.m.d * g.m.d;
    for (size_t i = 0; i < cnt; ++i) {
        std::snprintf(b, sizeof(b), " %.17g %.17g", m[i].real(), m[i].imag());
        *tr += b;
    }
    if (!partners.empty()) *tr += " |" + partners;
    *tr += "\n";
}

void trace_form(std::string* tr, const Form& F) {
    if (!tr) return;
    char b[64];
    std::snprintf(b, sizeof(b), "FORM %d", F.konst & 7);
    *tr += b;
    for (int q = 0; q < 64; ++q)
        if (F.alpha[q] & 7) { std::snprintf(b, sizeof(b), " a%d:%d", q, F.alpha[q] & 7); *tr += b; }
    for (auto& kv : F.beta)
        if (kv.second & 7) {
            std::snprintf(b, sizeof(b), " b%d,%d:%d", kv.first.first, kv.first.second, kv.second & 7);
            *tr += b;
        }
    *tr += "\n";
}

}  // namespace

// Local set S of one pass (|S| = T, the L low bits always local): the qubits
// of the leading unobstructed gates, filled up with the qubits that have the
// most pending local work, then improved by swapping one high local qubit
// for one non-local qubit while the scan score grows.
uint64_t greedy_local_set(const std::vector<int>& rem, const std::vector<GInfo>& inf, int n, int T, int L) {
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    uint64_t S = (1ull << L) - 1ull;
    {
        uint64_t bND = 0, bD = 0;
        for (int id : rem) {
            const GInfo& g = inf[id];
            if (g.cls == C_FREE) {
                if (g.qm & bND) bD |= g.qm;
                continue;
            }
            const uint64_t blk = g.diag ? bND : (bND | bD);
            if (g.cls == C_LOCAL && !(g.qm & blk) && popc(S | g.qm) <= T) {
                S |= g.qm;
                continue;
            }
            if (g.diag) bD |= g.qm; else bND |= g.qm;
            if ((bND & all) == all || popc(S) >= T) break;
        }
        if (popc(S) < T) {
            std::vector<int> cnt((size_t)n, 0);
            for (int id : rem)
                if (inf[id].cls == C_LOCAL)
                    for (int q = 0; q < n; ++q) if ((inf[id].qm >> q) & 1) cnt[q]++;
            while (popc(S) < T) {
                int best = -1;
                for (int q = 0; q < n; ++q)
                    if (!((S >> q) & 1) && (best < 0 || cnt[q] > cnt[best])) best = q;
                if (best < 0) break;
                S |= 1ull << best;
            }
        }
    }
    double best = scan(rem, inf, S, all, nullptr);
    for (int round = 0; round < 6 && T < n; ++round) {
        bool improved = false;
        uint64_t bestS = S;
        for (int a = L; a < n; ++a) {
            if (!((S >> a) & 1)) continue;
            for (int b = L; b < n; ++b) {
                if ((S >> b) & 1) continue;
                const uint64_t S2 = (S & ~(1ull << a)) | (1ull << b);
                const double sc = scan(rem, inf, S2, all, nullptr);
                if (sc > best + 1e-9) { best = sc; bestS = S2; improved = true; }
            }
        }
        S = bestS;
        if (!improved) break;
    }
    return S;
}

// Gates executed by a pass over local set S, in circuit order.  At most
// kMaxGradPerPass gradient reductions per pass (their per-wave partials live
// in LDS); a prefix of the executable list in circuit order is closed under
// dependencies, so the rest waits for a later pass.
std::vector<int> executable(const std::vector<IRGate>& ir, const std::vector<GInfo>& inf,
                            const std::vector<int>& rem, uint64_t S, uint64_t all) {
    std::vector<int> ex;
    scan(rem, inf, S, all, &ex);
    int ng = 0;
    for (size_t e = 0; e < ex.size(); ++e)
        if (ir[ex[e]].grad && ++ng > kMaxGradPerPass) {
            ex.resize(e);
            break;
        }
    return ex;
}

// Steps that remain after executing `ex` (a pass), or after the plain step of
// the leading gate when `ex` is empty.
std::vector<int> remove_executed(const std::vector<int>& rem, const std::vector<int>& ex, size_t nir) {
    std::vector<int> nr;
    if (ex.empty()) {
        nr.assign(rem.begin() + 1, rem.end());
        return nr;
    }
    std::vector<char> done(nir, 0);
    for (int id : ex) done[id] = 1;
    nr.reserve(rem.size() - ex.size());
    for (int id : rem) if (!done[id]) nr.push_back(id);
    return nr;
}

// Beam search over sequences of local sets.  The greedy choice maximises the
// work of the current pass only, and a pass that takes a little less can
// leave the rest of the circuit in fewer passes.  Every search state is a
// list of remaining gates after some number of steps; its children are the
// greedy set and the best single swaps away from it (by the scan score of the
// current pass), and after each step the `width` states with the least
// remaining gate weight survive (duplicates merged).  The first sequence that
// empties the list wins; the greedy sequence is the fallback, so the result
// never has more steps than greedy planning.  Returns one local set per step
// (a plain step's entry is the set that found nothing to execute).
// S with every qubit of `pin` made local, each in place of the unpinned high
// qubit whose loss leaves the most gate weight executable.
uint64_t pin_set(uint64_t S, uint64_t pin, const std::vector<int>& rem, const std::vector<GInfo>& inf, int n,
                 int L) {
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    pin &= all;
    for (int b = 0; b < n; ++b) {
        if (!((pin >> b) & 1) || ((S >> b) & 1)) continue;
        uint64_t bestS = S;
        double bw = -1.0;
        for (int a = L; a < n; ++a) {
            if (!((S >> a) & 1) || ((pin >> a) & 1)) continue;
            const uint64_t S2 = (S & ~(1ull << a)) | (1ull << b);
            const double w = scan(rem, inf, S2, all, nullptr);
            if (w > bw) { bw = w; bestS = S2; }
        }
        if (bw < 0.0) break;   // every high qubit is pinned
        S = bestS;
    }
    return S;
}

std::vector<uint64_t> beam_local_sets(const std::vector<IRGate>& ir, const std::vector<GInfo>& inf,
                                      const std::vector<int>& rem0, int n, int T, int L, int width,
                                      uint64_t pin) {
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    const int kids = std::max(2, std::min(width, 4));
    struct Node {
        std::vector<int> rem;
        std::vector<uint64_t> seq;
        double left = 0.0;
        uint64_t hash = 0;
    };
    auto finish = [&](Node& nd) {
        double w = 0.0;
        uint64_t h = 1469598103934665603ull;
        for (int id : nd.rem) {
            w += inf[id].w;
            h = (h ^ (uint64_t)id) * 1099511628211ull;
        }
        nd.left = w;
        nd.hash = h ^ (uint64_t)nd.rem.size();
    };
    // greedy sequence: the fallback and the bound
    std::vector<uint64_t> greedy;
    {
        std::vector<int> r = rem0;
        while (!r.empty()) {
            uint64_t S = greedy_local_set(r, inf, n, T, L);
            if (greedy.empty()) S = pin_set(S, pin, r, inf, n, L);
            greedy.push_back(S);
            r = remove_executed(r, executable(ir, inf, r, S, all), ir.size());
        }
    }
    std::vector<Node> beam(1);
    beam[0].rem = rem0;
    finish(beam[0]);
    while (!beam.empty() && beam[0].seq.size() + 1 < greedy.size()) {
        std::vector<Node> next;
        for (const Node& nd : beam) {
            const bool first = nd.seq.empty();
            uint64_t S0 = greedy_local_set(nd.rem, inf, n, T, L);
            if (first) S0 = pin_set(S0, pin, nd.rem, inf, n, L);
            std::vector<std::pair<double, uint64_t>> cand;
            cand.push_back({scan(nd.rem, inf, S0, all, nullptr) + 1e-6, S0});
            if (!executable(ir, inf, nd.rem, S0, all).empty() && T < n) {
                for (int a = L; a < n; ++a) {
                    if (!((S0 >> a) & 1) || (first && ((pin >> a) & 1))) continue;
                    for (int b = L; b < n; ++b) {
                        if ((S0 >> b) & 1) continue;
                        const uint64_t S2 = (S0 & ~(1ull << a)) | (1ull << b);
                        cand.push_back({scan(nd.rem, inf, S2, all, nullptr), S2});
                    }
                }
            }
            std::stable_sort(cand.begin(), cand.end(),
                             [](const std::pair<double, uint64_t>& x, const std::pair<double, uint64_t>& y) {
                                 return x.first > y.first;
                             });
            int taken = 0;
            for (const auto& c : cand) {
                if (taken == kids) break;
                const std::vector<int> ex = executable(ir, inf, nd.rem, c.second, all);
                if (ex.empty() && c.second != S0) continue;
                Node ch;
                ch.rem = remove_executed(nd.rem, ex, ir.size());
                ch.seq = nd.seq;
                ch.seq.push_back(c.second);
                if (ch.rem.empty()) return ch.seq;
                finish(ch);
                next.push_back(std::move(ch));
                ++taken;
            }
        }
        std::stable_sort(next.begin(), next.end(), [](const Node& x, const Node& y) { return x.left < y.left; });
        std::vector<Node> keep;
        for (Node& nd : next) {
            if ((int)keep.size() == width) break;
            bool dup = false;
            for (const Node& k : keep)
                if (k.hash == nd.hash && k.rem == nd.rem) { dup = true; break; }
            if (!dup) keep.push_back(std::move(nd));
        }
        beam.swap(keep);
    }
    return greedy;
}

void plan_fused(const std::vector<IRGate>& ir, int n, const PlanCfg& cfg, EncodedPlan& out, std::string* tr) {
    out = EncodedPlan();
    out.cfg = cfg;
    out.n = n;
    const bool c64 = cfg.dtype == SV_C64;
    // phase table e^{i pi e/4} at pool offset 0
    {
        Recipe r;
        r.type = Recipe::PHASETAB;
        add_recipe(out, r, ir);
    }
    std::vector<GInfo> inf(ir.size());
    for (size_t i = 0; i < ir.size(); ++i) inf[i] = info_of(ir[i]);
    const int T = std::min(cfg.T, n);
    const int L = std::min(cfg.L, T);
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    const uint64_t low = (1ull << L) - 1ull;
    // a gate whose qubits above the L low bits outnumber the tile's high bits
    // can never be local: it runs as a plain step
    for (size_t i = 0; i < ir.size(); ++i)
        if (inf[i].cls == C_LOCAL && !ir[i].grad && popc(inf[i].qm & ~low) > T - L) inf[i].cls = C_BIG;
    std::vector<int> rem(ir.size());
    for (size_t i = 0; i < ir.size(); ++i) rem[i] = (int)i;
    uint64_t grad_base = 0;
    // Diagonal phases not applied yet (Sec. 4.3's clustered T/S/Z/CZ plus the
    // side phases of the butterflies).  They stay pending across passes: a
    // butterfly on qubit q takes over the part that depends on q as its
    // twiddle, so most of them are never applied as separate ops.
    Form pending;
    // Each butterfly grows the state by sqrt(2); the factor 2^(-scale_p/2) is
    // applied when scale_p reaches its limit (FP32 keeps the growth exactly)
    // and before the state is handed back.
    int scale_p = 0;
    const int scale_every = cfg.two ? kScaleEveryAdjoint : kScaleEvery;

    // local sets of the tile passes, chosen ahead by a beam search over whole
    // pass sequences (an empty list: greedy per pass)
    const std::vector<uint64_t> seq = cfg.beam > 1 ? beam_local_sets(ir, inf, rem, n, T, L, cfg.beam, cfg.first_pin)
                                                   : std::vector<uint64_t>();
    size_t it = 0;
    while (!rem.empty()) {
        // ---- choose the local set S (|S| = T, low bits always local; the
        // first pass also holds the pinned qubits)
        uint64_t S = it < seq.size() ? seq[it] : greedy_local_set(rem, inf, n, T, L);
        if (it == 0) S = pin_set(S, cfg.first_pin, rem, inf, n, L);
        ++it;
        std::vector<int> ex = executable(ir, inf, rem, S, all);
        if (ex.empty()) {
            // the frontier is a gate wider than a register phase: plain kernel
            const int id = rem[0];
            if (inf[id].cls != C_BIG) throw std::runtime_error("planner: no progress");
            const IRGate& g = ir[id];
            Step st;
            if (g.kind == K_DIAGG) {
                st.type = ST_DIAG;
            } else {
                st.type = ST_DENSE;
            }
            int order[6];
            for (int t = 0; t < g.k; ++t) order[t] = t;
            std::sort(order, order + g.k, [&](int x, int y) { return g.q[x] < g.q[y]; });
            Recipe rc;
            rc.type = g.kind == K_DIAGG ? Recipe::DIAG : Recipe::DENSE;
            rc.gate = id;
            rc.k = g.k;
            for (int j = 0; j < g.k; ++j) { rc.perm[j] = order[j]; st.tq[j] = g.q[order[j]]; }
            st.k = g.k;
            add_recipe(out, rc, ir);
            st.recipe = (int)out.recipes.size() - 1;
            out.steps.push_back(st);
            out.n_plain++;
            trace_matrix(tr, g.kind == K_DIAGG ? "DIAG" : "DENSE", g);
            out.flops += 8.0 * (double)(1 << g.k) * (double)(1ull << n);
            rem.erase(std::find(rem.begin(), rem.end(), id));
            continue;
        }
        // ---- build the pass
        PassGeom G = make_geom(n, L, S);
        DPass P;
        std::memset(&P, 0, sizeof(P));
        P.L = (uint32_t)G.L;
        P.H = (uint32_t)G.H;
        P.T = (uint32_t)G.T;
        for (int t = 0; t < G.H; ++t) P.hpos[t] = (uint32_t)G.hpos[t];
        P.phase0 = (uint32_t)out.phases.size();
        P.form0 = (uint32_t)out.forms.size();
        uint32_t nform = 0, ngrad = 0;
        if (tr) {
            *tr += "PASS";
            for (int a = 0; a < G.T; ++a) *tr += " " + std::to_string(G.gq[a]);
            *tr += "\n";
        }

        // phases
        std::vector<int> prem = ex;
        // pending phases must be applied at the end of this pass when no pass
        // follows or a plain (wide-gate) step may come next
        bool flush_at_end = false;
        {
            std::vector<char> inpass(ir.size(), 0);
            for (int id : ex) inpass[id] = 1;
            bool any_left = false;
            for (int id : rem) {
                if (inpass[id]) continue;
                any_left = true;
                if (inf[id].cls == C_BIG) flush_at_end = true;
            }
            if (!any_left) flush_at_end = true;
        }
        std::vector<int> combos;
        for (int a = 0; a < G.T; ++a)
            for (int b = a + 1; b < G.T; ++b)
                for (int c = b + 1; c < G.T; ++c)
                    for (int d = c + 1; d < G.T; ++d) combos.push_back(a | (b << 8) | (c << 16) | (d << 24));
        // local-position masks for the phase scan (non-local qubits never
        // obstruct anything inside a pass, so they are dropped)
        std::vector<GInfo> pinf = inf;
        for (int id : prem) {
            uint64_t m = 0;
            for (int t = 0; t < ir[id].k; ++t) {
                const int lp = G.lpos[ir[id].q[t]];
                if (lp >= 0) m |= 1ull << lp;
            }
            pinf[id].qm = m;
        }
        const uint64_t lall = (1ull << G.T) - 1ull;
        while (!prem.empty()) {
            double bs = -1.0;
            int bc = combos.empty() ? 0 : combos[0];
            for (int cmb : combos) {
                const uint64_t R = (1ull << (cmb & 255)) | (1ull << ((cmb >> 8) & 255)) |
                                   (1ull << ((cmb >> 16) & 255)) | (1ull << (cmb >> 24));
                const double sc = scan(prem, pinf, R, lall, nullptr);
                if (sc > bs + 1e-9) { bs = sc; bc = cmb; }
            }
            int r[4] = {bc & 255, (bc >> 8) & 255, (bc >> 16) & 255, bc >> 24};
            const uint64_t R = (1ull << r[0]) | (1ull << r[1]) | (1ull << r[2]) | (1ull << r[3]);
            std::vector<int> pex;
            scan(prem, pinf, R, lall, &pex);
            if (pex.empty()) throw std::runtime_error("planner: empty register phase");
            DPhase Ph;
            std::memset(&Ph, 0, sizeof(Ph));
            Ph.kind = PH_REG;
            Ph.rpos = (uint32_t)(r[0] | (r[1] << 8) | (r[2] << 16) | (r[3] << 24));
            if (c64) soff_for<float>(r, Ph.soff); else soff_for<double>(r, Ph.soff);
            Ph.op0 = (uint32_t)out.ops.size();
            if (tr)
                *tr += "PHASE " + std::to_string(G.gq[r[0]]) + " " + std::to_string(G.gq[r[1]]) + " " +
                       std::to_string(G.gq[r[2]]) + " " + std::to_string(G.gq[r[3]]) + "\n";
            auto flush = [&](bool force) {
                if (pending.empty()) { pending.clear(); return; }
                (void)force;
                trace_form(tr, pending);
                const bool so = pending.sign_only();
                const int fi = encode_form(pending, G, r, n, out, nform++);
                DOp op{so ? (uint32_t)OP_SIGN : (uint32_t)OP_PHASE8, 0u, 0u, (uint32_t)fi};
                out.ops.push_back(op);
                out.n_diag++;
                out.flops += (so ? 2.0 : 6.0) * (double)(1ull << n) * (cfg.two ? 2 : 1);
                out.alu_ops += (so ? 1.0 : 4.0) * (double)(1ull << n) * (cfg.two ? 2 : 1);
                pending.clear();
            };
            auto emit_scale = [&]() {
                Recipe rc;
                rc.type = Recipe::SCALE;
                rc.scale = std::ldexp(1.0, -(scale_p / 2)) * ((scale_p & 1) ? std::sqrt(0.5) : 1.0);
                const uint64_t off = add_recipe(out, rc, ir);
                DOp op{(uint32_t)OP_SCALE, 0u, 0u, (uint32_t)off};
                out.ops.push_back(op);
                if (tr) {
                    char b[64];
                    std::snprintf(b, sizeof(b), "SCALE %.17g\n", rc.scale);
                    *tr += b;
                }
                scale_p = 0;
                out.alu_ops += 2.0 * (double)(1ull << n) * (cfg.two ? 2 : 1);
            };
            for (int id : pex) {
                const IRGate& g = ir[id];
                if (inf[id].cls == C_FREE) {
                    pending.add(g);
                    continue;
                }
                int slot_of_q[6];
                for (int t = 0; t < g.k; ++t) {
                    const int lp = G.lpos[g.q[t]];
                    int s = -1;
                    for (int u = 0; u < 4; ++u) if (r[u] == lp) s = u;
                    slot_of_q[t] = s;
                }
                // Take the part of the pending phase that depends on qubit q:
                // w^m (-1)^(sum of partner bits).  Needs every pair exponent on
                // q to be 0 or 4; otherwise the whole form is applied first.
                struct Tw { int m = 0; uint32_t RM = 0, lmask = 0, pair = kNoPair; std::string partners; };
                auto take_twiddle = [&](int q) {
                    for (auto& kv : pending.beta)
                        if ((kv.second & 3) && (kv.first.first == q || kv.first.second == q)) {
                            flush(false);
                            break;
                        }
                    Tw t;
                    t.m = pending.alpha[q] & 7;
                    uint64_t gmask = 0;
                    for (auto it = pending.beta.begin(); it != pending.beta.end();) {
                        const int a = it->first.first, b = it->first.second;
                        if (a != q && b != q) { ++it; continue; }
                        if (it->second & 7) {
                            const int p = a == q ? b : a;
                            t.partners += " " + std::to_string(p);
                            const int lp = G.lpos[p];
                            int su = -1;
                            for (int u = 0; u < 4; ++u) if (r[u] == lp) su = u;
                            if (lp < 0) gmask |= 1ull << p;
                            else if (su >= 0) t.RM |= 1u << su;
                            else t.lmask |= 1u << lp;
                        }
                        it = pending.beta.erase(it);
                    }
                    pending.alpha[q] = 0;
                    if (gmask) {
                        DPair pr;
                        std::memset(&pr, 0, sizeof(pr));
                        pr.m[0] = gmask;
                        t.pair = (uint32_t)out.pairs.size();
                        out.pairs.push_back(pr);
                    }
                    return t;
                };
                if (g.skind == OP_BF) {
                    const int q = g.q[0];
                    if (scale_p >= scale_every) emit_scale();
                    Tw t = take_twiddle(q);
                    const int M = (t.m + g.bf_pre) & 7;
                    pending.alpha[q] = g.bf_post & 7;
                    pending.konst = (pending.konst + g.bf_g) & 7;
                    DOp op{(uint32_t)OP_BF, (uint32_t)(M | (slot_of_q[0] << 4) | (t.RM << 8)), t.lmask, t.pair};
                    if (t.lmask == 0 && t.pair == kNoPair) {
                        // signs from register partners only: a per-pair sign table
                        Recipe rb;
                        rb.type = Recipe::BFTAB;
                        rb.slot = slot_of_q[0];
                        rb.rm = t.RM;
                        rb.bf_m = M;
                        op.k |= kBfUniform;
                        op.arg = (uint32_t)add_recipe(out, rb, ir);
                    }
                    out.ops.push_back(op);
                    if (tr) *tr += "BF " + std::to_string(q) + " " + std::to_string(M) + t.partners + "\n";
                    scale_p += 1;
                    out.n_dense++;
                    out.flops += ((M & 1) ? 5.0 : 2.0) * (double)(1ull << n) * (cfg.two ? 2 : 1);
                    out.alu_ops += ((M & 1) ? 3.0 : 2.0) * (double)(1ull << n) * (cfg.two ? 2 : 1);
                    continue;
                }
                if (g.perm != PK_NONE && g.kind == K_DENSE && !g.grad &&
                    g.k == ((g.perm == PK_X || g.perm == PK_Y) ? 1 : 2)) {
                    // X, Y, CNOT, SWAP: amplitudes change registers, no
                    // arithmetic (Y: a swap of real and imaginary parts and
                    // a sign); pending phases on its qubits are applied first
                    if (pending.depends(g.qmask())) flush(false);
                    const uint32_t sa = (uint32_t)slot_of_q[0], sb = g.k > 1 ? (uint32_t)slot_of_q[1] : sa;
                    DOp op{(uint32_t)OP_PERM, (uint32_t)g.perm, sa | (sb << 2), 0u};
                    out.ops.push_back(op);
                    if (tr) {
                        *tr += "PERM " + std::to_string(g.perm) + " " + std::to_string(g.q[0]);
                        if (g.k > 1) *tr += " " + std::to_string(g.q[1]);
                        *tr += "\n";
                    }
                    out.alu_ops += (g.perm == PK_Y ? 1.0 : 0.0) * (double)(1ull << n) * (cfg.two ? 2 : 1);
                    continue;
                }
                if (g.kind == K_DENSE && g.k == 1 && !g.grad) {
                    // one-qubit matrix: the pending phase of q folds into its
                    // second column, the partner signs into the kernel
                    const int q = g.q[0];
                    Tw t = take_twiddle(q);
                    const bool real = real_gate(g) && (t.m & 3) == 0;
                    Recipe rc;
                    rc.type = Recipe::DENSE;
                    rc.gate = id;
                    rc.k = 1;
                    rc.twiddle = t.m;
                    rc.inplace = true;
                    rc.slot = slot_of_q[0];
                    rc.rm = t.RM;
                    const uint64_t off = add_recipe(out, rc, ir);
                    const uint32_t pk = t.pair == kNoPair ? 0u : t.pair + 1u;
                    DOp op{(uint32_t)OP_D1T, (uint32_t)(slot_of_q[0] | (t.RM << 2) | ((real ? 1u : 0u) << 6) | (pk << 7)),
                           t.lmask, (uint32_t)off};
                    out.ops.push_back(op);
                    if (tr) {
                        IRGate tg = g;
                        tg.m = g.m;
                        const cd w = std::polar(1.0, M_PI / 4.0 * t.m);
                        for (int bb = 0; bb < tg.m.nb; ++bb) { tg.m.at(bb)[1] *= w; tg.m.at(bb)[3] *= w; }
                        trace_matrix(tr, "DENSE1", tg, t.partners);
                    }
                    out.n_dense++;
                    out.flops += (real ? 8.0 : 16.0) * (double)(1ull << n) * (cfg.two ? 2 : 1);
                    out.alu_ops += (real ? 4.0 : 8.0) * (double)(1ull << n) * (cfg.two ? 2 : 1);
                    continue;
                }
                // A diagonal gate, or a gradient term whose generator is
                // diagonal, commutes with the pending diagonal phases (which
                // psi and lambda share), so those stay pending
                const bool commutes = g.kind == K_DIAGG || (g.grad && (g.gen == GEN_Z || g.gen == GEN_P11));
                if (!commutes && pending.depends(g.qmask())) flush(false);
                if (g.grad) {
                    uint32_t mask = 0;
                    for (int t = 0; t < g.k; ++t) mask |= 1u << slot_of_q[t];
                    DOp op{(uint32_t)OP_GRAD, (uint32_t)g.gen, mask, ngrad};
                    out.ops.push_back(op);
                    if (tr) {
                        char b[64];
                        std::snprintf(b, sizeof(b), "GRAD %d %d %.17g", g.param, g.gen, std::ldexp(1.0, -scale_p));
                        *tr += b;
                        for (int t = 0; t < g.k; ++t) *tr += " " + std::to_string(g.q[t]);
                        *tr += "\n";
                    }
                    out.grad_param.push_back(g.param);
                    // psi and lambda both carry sqrt(2)^scale_p at this point of the pass
                    out.grad_scale.push_back(std::ldexp(1.0, -scale_p));
                    ++ngrad;
                    // 4 multiply-adds per register pair (a psi and a lambda amplitude each)
                    out.alu_ops += 2.0 * (double)(1ull << n);
                    continue;
                }
                Recipe rc;
                rc.gate = id;
                uint32_t mask = 0;
                slot_perm(g, slot_of_q, rc, mask);
                if (g.kind == K_DIAGG) {
                    rc.type = Recipe::DIAG;
                    const uint64_t off = add_recipe(out, rc, ir);
                    DOp op{(uint32_t)OP_DIAGR, (uint32_t)g.k, mask, (uint32_t)off};
                    out.ops.push_back(op);
                    trace_matrix(tr, "DIAG", g);
                    out.n_diag++;
                    out.flops += 6.0 * (double)(1ull << n) * (cfg.two ? 2 : 1);
                    out.alu_ops += 4.0 * (double)(1ull << n) * (cfg.two ? 2 : 1);
                } else {
                    rc.type = Recipe::DENSE;
                    const uint64_t off = add_recipe(out, rc, ir);
                    DOp op{(uint32_t)OP_DENSE, (uint32_t)g.k, mask, (uint32_t)off};
                    out.ops.push_back(op);
                    trace_matrix(tr, "DENSE", g);
                    out.n_dense++;
                    out.flops += 8.0 * (double)(1 << g.k) * (double)(1ull << n) * (cfg.two ? 2 : 1);
                    out.alu_ops += 4.0 * (double)(1 << g.k) * (double)(1ull << n) * (cfg.two ? 2 : 1);
                }
            }
            // drop executed gates from prem
            {
                std::vector<char> done(ir.size(), 0);
                for (int id : pex) done[id] = 1;
                std::vector<int> nr;
                for (int id : prem) if (!done[id]) nr.push_back(id);
                prem.swap(nr);
            }
            if (prem.empty()) {
                if (flush_at_end) flush(true);
                if (scale_p && (flush_at_end || scale_p >= scale_every)) emit_scale();
            }
            Ph.nop = (uint32_t)(out.ops.size() - Ph.op0);
            out.phases.push_back(Ph);
            out.n_phase++;
        }
        P.nphase = (uint32_t)(out.phases.size() - P.phase0);
        P.nform = nform;
        P.ngrad = ngrad;
        P.gpart_off = out.gpart_size;   // per state; the executor scales by the batch
        out.grad_slot_off.push_back(grad_base);
        grad_base += ngrad;
        out.gpart_size += (uint64_t)ngrad << (n - G.T);
        out.passes.push_back(P);
        Step st;
        st.type = ST_TILE;
        st.pass = (int)out.passes.size() - 1;
        out.steps.push_back(st);
        out.n_tile++;
        // remove executed gates
        {
            std::vector<char> done(ir.size(), 0);
            for (int id : ex) done[id] = 1;
            std::vector<int> nr;
            for (int id : rem) if (!done[id]) nr.push_back(id);
            rem.swap(nr);
        }
    }
    out.ngrad_total = (int)grad_base;
}

void plan_plain(const std::vector<IRGate>& ir, int n, const PlanCfg& cfg, EncodedPlan& out) {
    out = EncodedPlan();
    out.cfg = cfg;
    out.n = n;
    {
        Recipe r;
        r.type = Recipe::PHASETAB;
        add_recipe(out, r, ir);
    }
    const double N = (double)(1ull << n);
    int grad_slot = 0;
    for (size_t id = 0; id < ir.size(); ++id) {
        const IRGate& g = ir[id];
        Step st;
        if (g.grad) {
            st.type = ST_GRAD;
            st.k = g.k;
            for (int t = 0; t < g.k; ++t) st.tq[t] = g.q[t];
            st.mask = g.qmask();
            st.mode = g.gen;
            st.slot = grad_slot++;
            out.grad_param.push_back(g.param);
            out.grad_scale.push_back(1.0);
            out.steps.push_back(st);
            continue;
        }
        if (g.kind == K_DIAG8) {
            uint64_t mask = 0;
            int e = 0;
            if (g.k == 1) {
                mask = 1ull << g.q[0];
                e = g.alpha[0] & 7;
            } else {
                mask = (1ull << g.q[0]) | (1ull << g.q[1]);
                e = g.beta & 7;
                if ((g.alpha[0] & 7) || (g.alpha[1] & 7)) {
                    // general two-qubit 8th-root diagonal: use the diagonal kernel
                    e = -1;
                }
            }
            if (e < 0) throw std::runtime_error("planner: unfused two-qubit phase with linear terms");
            if (e == 0) continue;
            st.type = ST_MASKED;
            st.mask = mask;
            st.mode = e == 4 ? 1 : (e == 2 ? 2 : (e == 6 ? 3 : 0));
            if (st.mode == 0) {
                Recipe rc;
                rc.type = Recipe::VALUE;
                const double a = std::atan2(1.0, 1.0) * e;  // pi/4 * e
                rc.value = cd(std::cos(a), std::sin(a));
                if (e == 1) rc.value = cd(std::sqrt(0.5), std::sqrt(0.5));
                if (e == 7) rc.value = cd(std::sqrt(0.5), -std::sqrt(0.5));
                if (e == 3) rc.value = cd(-std::sqrt(0.5), std::sqrt(0.5));
                if (e == 5) rc.value = cd(-std::sqrt(0.5), -std::sqrt(0.5));
                add_recipe(out, rc, ir);
                st.recipe = (int)out.recipes.size() - 1;
            }
            out.steps.push_back(st);
            out.n_diag++;
            out.flops += 2.0 * N / (double)(1ull << popc(mask));
            continue;
        }
        int order[6];
        for (int t = 0; t < g.k; ++t) order[t] = t;
        std::sort(order, order + g.k, [&](int x, int y) { return g.q[x] < g.q[y]; });
        if (g.kind == K_DIAGG) {
            // one entry differs from 1 for every state -> masked multiply
            const int d = g.m.d;
            bool unit = true;
            for (int b = 0; b < g.m.nb && unit; ++b)
                for (int i = 0; i + 1 < d; ++i)
                    if (g.m.at(b)[i] != cd(1.0, 0.0)) { unit = false; break; }
            Recipe rc;
            rc.gate = (int)id;
            rc.k = g.k;
            for (int j = 0; j < g.k; ++j) { rc.perm[j] = order[j]; st.tq[j] = g.q[order[j]]; }
            st.k = g.k;
            if (unit) {
                st.type = ST_MASKED;
                st.mask = g.qmask();
                st.mode = 0;
                rc.type = Recipe::VALUE;
                rc.value = cd(0.0, 0.0);  // taken from the gate per state (last entry)
                rc.varies = g.m.nb > 1;
                rc.k = -1;                // marks "last diagonal entry of gate"
            } else {
                st.type = ST_DIAG;
                rc.type = Recipe::DIAG;
            }
            add_recipe(out, rc, ir);
            st.recipe = (int)out.recipes.size() - 1;
            out.steps.push_back(st);
            out.n_diag++;
            out.flops += 6.0 * N;
            continue;
        }
        if (g.perm != PK_NONE) {
            st.type = ST_SWAP;
            if (g.perm == PK_X || g.perm == PK_Y) {
                st.mask = 1ull << g.q[0];
                st.ones = 0;
                st.flip = 1ull << g.q[0];
                st.mode = g.perm == PK_Y ? 1 : 0;
            } else if (g.perm == PK_CNOT) {
                st.mask = 1ull << g.q[1];
                st.ones = 1ull << g.q[0];
                st.flip = 1ull << g.q[1];
            } else {
                st.mask = 1ull << g.q[1];
                st.ones = 1ull << g.q[0];
                st.flip = (1ull << g.q[0]) | (1ull << g.q[1]);
            }
            out.steps.push_back(st);
            out.n_plain++;
            continue;
        }
        st.type = ST_DENSE;
        Recipe rc;
        rc.type = Recipe::DENSE;
        rc.gate = (int)id;
        rc.k = g.k;
        for (int j = 0; j < g.k; ++j) { rc.perm[j] = order[j]; st.tq[j] = g.q[order[j]]; }
        st.k = g.k;
        add_recipe(out, rc, ir);
        st.recipe = (int)out.recipes.size() - 1;
        out.steps.push_back(st);
        out.n_plain++;
        out.n_dense++;
        out.flops += 8.0 * (double)(1 << g.k) * N;
    }
    out.ngrad_total = grad_slot;
}

namespace {
// Register index of the q-th pair (bit `slot` clear) in increasing order.
int pair_index(int slot, int q) {
    return (q & ((1 << slot) - 1)) | ((q >> slot) << (slot + 1));
}

template <class R>
void fill_pool_t(const EncodedPlan& p, const std::vector<IRGate>& ir, int batch, std::vector<unsigned char>& bytes) {
    const int nb = p.pool_varies ? batch : 1;
    bytes.assign((size_t)nb * p.pool_size * 2 * sizeof(R), 0);
    R* base = reinterpret_cast<R*>(bytes.data());
    const double c = std::sqrt(0.5);
    const cd tab[8] = {cd(1, 0), cd(c, c), cd(0, 1), cd(-c, c), cd(-1, 0), cd(-c, -c), cd(0, -1), cd(c, -c)};
    auto fill_one = [&](int b) {
        R* pb = base + (size_t)b * p.pool_size * 2;
        for (const Recipe& rc : p.recipes) {
            R* dst = pb + rc.off * 2;
            switch (rc.type) {
                case Recipe::PHASETAB:
                    for (int e = 0; e < 8; ++e) { dst[2 * e] = (R)tab[e].real(); dst[2 * e + 1] = (R)tab[e].imag(); }
                    break;
                case Recipe::SCALE:
                    dst[0] = (R)rc.scale;
                    dst[1] = 0;
                    break;
                case Recipe::VALUE: {
                    cd v = rc.value;
                    if (rc.k == -1) {
                        const IRGate& g = ir[rc.gate];
                        v = g.m.at(b)[g.m.d - 1];
                    }
                    dst[0] = (R)v.real();
                    dst[1] = (R)v.imag();
                    break;
                }
                case Recipe::DENSE: {
                    const IRGate& g = ir[rc.gate];
                    const int d = 1 << rc.k;
                    const cd* m = g.m.at(b);
                    for (int r = 0; r < d; ++r)
                        for (int col = 0; col < d; ++col) {
                            int orr = 0, oc = 0;
                            for (int j = 0; j < rc.k; ++j) {
                                if ((r >> j) & 1) orr |= 1 << rc.perm[j];
                                if ((col >> j) & 1) oc |= 1 << rc.perm[j];
                            }
                            cd v = m[(size_t)orr * d + oc];
                            if (rc.twiddle && (col & 1)) v *= tab[rc.twiddle & 7];
                            dst[2 * (r * d + col)] = (R)v.real();
                            dst[2 * (r * d + col) + 1] = (R)v.imag();
                        }
                    if (rc.inplace) {
                        // u = [[a, b], [c, e]] (twiddle included) as
                        // o0 = a x + b y, o1 = (c / a) o0 + (e - (c / a) b) y,
                        // usable when |a| >= |c| (then |c / a| <= 1)
                        cd u[4];
                        for (int e = 0; e < 4; ++e) {
                            u[e] = m[e];
                            if (rc.twiddle && (e & 1)) u[e] *= tab[rc.twiddle & 7];
                        }
                        cd rr(0.0, 0.0), dd(0.0, 0.0);
                        const bool ok = std::abs(u[0]) >= std::abs(u[2]) && std::abs(u[0]) > 0.0;
                        if (ok) {
                            rr = u[2] / u[0];
                            dd = u[3] - rr * u[1];
                        }
                        dst[8] = (R)rr.real();
                        dst[9] = (R)rr.imag();
                        dst[10] = (R)dd.real();
                        dst[11] = (R)dd.imag();
                        dst[12] = ok ? R(1) : R(0);
                        dst[13] = 0;
                        // real matrices: signed (b, d) per register pair
                        for (int q = 0; q < 8; ++q) {
                            const int i = pair_index(rc.slot, q);
                            const bool neg = (__builtin_popcount((unsigned)i & rc.rm) & 1) != 0;
                            dst[14 + 2 * q] = (R)(neg ? -u[1].real() : u[1].real());
                            dst[15 + 2 * q] = (R)(neg ? -dd.real() : dd.real());
                        }
                    }
                    break;
                }
                case Recipe::BFTAB: {
                    const double g = (rc.bf_m & 1) ? c : 1.0;
                    for (int q = 0; q < 8; ++q) {
                        const int i = pair_index(rc.slot, q);
                        const bool neg = (__builtin_popcount((unsigned)i & rc.rm) & 1) != 0;
                        const R gq = (R)(neg ? -g : g);
                        dst[2 * q] = gq;
                        dst[2 * q + 1] = R(-2) * gq;
                    }
                    break;
                }
                case Recipe::DIAG: {
                    const IRGate& g = ir[rc.gate];
                    const int d = 1 << rc.k;
                    const cd* m = g.m.at(b);
                    for (int r = 0; r < d; ++r) {
                        int orr = 0;
                        for (int j = 0; j < rc.k; ++j)
                            if ((r >> j) & 1) orr |= 1 << rc.perm[j];
                        dst[2 * r] = (R)m[orr].real();
                        dst[2 * r + 1] = (R)m[orr].imag();
                    }
                    break;
                }
            }
        }
    };
    // the states' pools are independent: many parameter sets fill in parallel
    if (nb >= 8 && (size_t)nb * p.recipes.size() >= 4096) {
        host_parallel_for(nb, fill_one);
    } else {
        for (int b = 0; b < nb; ++b) fill_one(b);
    }
}
}  // namespace

void fill_pool(const EncodedPlan& p, const std::vector<IRGate>& ir, int batch, std::vector<unsigned char>& bytes) {
    if (p.cfg.dtype == SV_C64) fill_pool_t<float>(p, ir, batch, bytes);
    else fill_pool_t<double>(p, ir, batch, bytes);
}

}  // namespace svmi
