// The paper's own simulation plan, kept as an ablation of the tile-pass
// design: gates are clustered by kind with the reordering scan of Sec. 4.5
// (diagonal 8th-root phases and CZ together; one-qubit gates of one kind
// together, at most one per qubit), and the clusters are encoded with the
// bitmasks of Sec. 4.2-4.3.
#include <algorithm>
#include <sstream>

#include "host.h"

namespace svmi {

namespace {

// Exponent of w = e^{i pi/4} of a one-qubit 8th-root diagonal, or -1.
int diag8_exponent(int op) {
    switch (op) {
        case SV_OP_I: return 0;
        case SV_OP_T: return 1;
        case SV_OP_S: return 2;
        case SV_OP_Z: return 4;
        case SV_OP_SDG: return 6;
        case SV_OP_TDG: return 7;
        default: return -1;
    }
}

// Cluster kind of a gate: SV_OP_T for every 8th-root diagonal and CZ, the op
// itself for H, sqrt(X), sqrt(Y) and their inverses (the paper's multiply-free
// family), -1 for a gate that stays alone (sqrt(W), which the paper does not
// use and has no multiply-free form, among them).
int kind_of(const sv_gate& g) {
    if (g.op == SV_OP_CZ || diag8_exponent(g.op) >= 0) return SV_OP_T;
    switch (g.op) {
        case SV_OP_H: case SV_OP_SQRTX: case SV_OP_SQRTXDG: case SV_OP_SQRTY: case SV_OP_SQRTYDG:
            return g.op;
        default: return -1;
    }
}

int paper_gate(int op) {
    switch (op) {
        case SV_OP_H: return PG_H;
        case SV_OP_SQRTX: return PG_SX;
        case SV_OP_SQRTXDG: return PG_SXDG;
        case SV_OP_SQRTY: return PG_SY;
        case SV_OP_SQRTYDG: return PG_SYDG;
        default: return PG_GEN;
    }
}

uint64_t qmask(const sv_gate& g) {
    uint64_t m = 0;
    for (int t = 0; t < g.nq; ++t) m |= 1ull << g.q[t];
    return m;
}

std::string bin(uint64_t m, int n) {
    std::string s;
    for (int q = n - 1; q >= 0; --q) s.push_back(((m >> q) & 1) ? '1' : '0');
    return s;
}

}  // namespace

PaperPlan paper_plan(const sv_circuit* c) {
    PaperPlan p;
    const int n = c->n_qubits;
    p.n = n;
    const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1);
    std::vector<char> done((size_t)c->n_gates, 0);
    for (int k = 0; k < c->n_gates; ++k) {
        if (done[k]) continue;
        const sv_gate& gk = c->gates[k];
        const int kind = kind_of(gk);
        done[k] = 1;
        if (kind < 0) {
            // a gate of no cluster kind: joins the previous step of such gates
            if (!p.steps.empty() && p.steps.back().type == PS_GATES) {
                p.steps.back().gates.push_back(k);
            } else {
                PStep st;
                st.type = PS_GATES;
                st.gates.push_back(k);
                p.steps.push_back(st);
            }
            continue;
        }
        std::vector<int> members{k};
        uint64_t in_cluster = qmask(gk), obstructed = 0;
        // scan the later gates not yet clustered (Sec. 4.5): a gate of the
        // kind joins when none of its qubits is obstructed (and, for a
        // one-qubit layer, its qubit has no gate of the layer yet); every
        // other gate obstructs its qubits.  Diagonal gates commute with one
        // another, gates on disjoint qubits commute, nothing else does.
        for (int l = k + 1; l < c->n_gates && obstructed != all; ++l) {
            if (done[l]) continue;
            const sv_gate& gl = c->gates[l];
            const uint64_t ql = qmask(gl);
            const bool same = kind_of(gl) == kind;
            const bool free_q = (ql & obstructed) == 0 && (kind == SV_OP_T || (ql & in_cluster) == 0);
            if (same && free_q) {
                members.push_back(l);
                in_cluster |= ql;
                done[l] = 1;
            } else {
                obstructed |= ql;
            }
        }
        PStep st;
        st.gates = members;
        st.kind = kind;
        if (kind == SV_OP_T) {
            st.type = PS_DIAG;
            st.cz.assign((size_t)n, 0);
            std::vector<int> e((size_t)n, 0);
            for (int gi : members) {
                const sv_gate& g = c->gates[gi];
                if (g.op == SV_OP_CZ) {
                    // one-sided masks, toggled: the lower qubit is the
                    // partner bit in the higher qubit's mask; CZ CZ cancels
                    const int a = std::min(g.q[0], g.q[1]), b = std::max(g.q[0], g.q[1]);
                    st.cz[(size_t)b] ^= 1ull << a;
                } else {
                    e[(size_t)g.q[0]] = (e[(size_t)g.q[0]] + diag8_exponent(g.op)) & 7;
                }
            }
            for (int q = 0; q < n; ++q)
                for (int b = 0; b < 3; ++b)
                    if ((e[(size_t)q] >> b) & 1) st.e8[b] |= 1ull << q;
        } else {
            st.type = PS_LAYER;
            for (int gi : members) st.layer.emplace_back(c->gates[gi].q[0], paper_gate(c->gates[gi].op));
            std::sort(st.layer.begin(), st.layer.end());
        }
        p.steps.push_back(st);
    }
    return p;
}

std::string paper_trace(const PaperPlan& p) {
    std::ostringstream o;
    for (const PStep& st : p.steps) {
        if (st.type == PS_DIAG) {
            o << "DIAG e8 " << bin(st.e8[0], p.n) << " " << bin(st.e8[1], p.n) << " " << bin(st.e8[2], p.n) << " cz";
            for (int q = 0; q < p.n; ++q)
                if (st.cz[(size_t)q]) o << " " << q << ":" << bin(st.cz[(size_t)q], p.n);
        } else if (st.type == PS_LAYER) {
            uint64_t m = 0;
            for (const auto& g : st.layer) m |= 1ull << g.first;
            o << "LAYER " << st.kind << " " << bin(m, p.n);
        } else {
            o << "GATES";
        }
        o << " |";
        for (int gi : st.gates) o << " " << gi;
        o << "\n";
    }
    return o.str();
}

}  // namespace svmi
