// Gate table, validation, circuit -> IR conversion and one-qubit fusion.
//
// Gate definitions follow Sec. 2 of the paper (NOT, H, Z, CNOT, CZ, P = S,
// sqrt(X), T) and Sec. 4.3 (P = T^2, Z = T^4).  sqrt(Y) is the principal
// square root (the printed matrix squares to -Y).  sqrt(W) is the principal
// root of W = (X + Y)/sqrt(2).  Rotations are exp(-i theta G / 2).
//
// Classification follows the paper's split of gates by kind (Sec. 4.2):
// diagonal gates with 8th-root phases (T, S, Z, CZ and inverses) become terms
// of a phase form, general diagonals (RZ, P, CP) stay diagonal, everything
// else is a dense (non-diagonal) gate.  With `structured`, H, sqrt(X),
// sqrt(Y) and sqrt(W) keep their factored multiply-free form (Sec. 4.4).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>
#include <stdexcept>

#include "host.h"

namespace svmi {

// True when the gate's matrix is real (for every parameter value).
bool real_gate(const IRGate& g) {
    if (g.kind == K_DIAG8) return (g.alpha[0] & 3) == 0 && (g.alpha[1] & 3) == 0 && (g.beta & 3) == 0;
    return g.real;
}

namespace {

const double kR = std::sqrt(0.5);

int op_arity(int op) {
    switch (op) {
        case SV_OP_CZ: case SV_OP_CNOT: case SV_OP_SWAP: case SV_OP_CP: return 2;
        case SV_OP_MAT: case SV_OP_DIAG: return -1;
        default: return 1;
    }
}

bool op_takes_angle(int op) {
    return op == SV_OP_RX || op == SV_OP_RY || op == SV_OP_RZ || op == SV_OP_P || op == SV_OP_CP;
}

int diag8_alpha(int op) {
    switch (op) {
        case SV_OP_I: return 0;
        case SV_OP_Z: return 4;
        case SV_OP_S: return 2;
        case SV_OP_SDG: return 6;
        case SV_OP_T: return 1;
        case SV_OP_TDG: return 7;
        default: return -1;
    }
}

void conj_transpose(std::vector<cd>& m, int d) {
    std::vector<cd> t(m.size());
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) t[(size_t)c * d + r] = std::conj(m[(size_t)r * d + c]);
    m.swap(t);
}

// C = A * B (d x d)
void matmul(const cd* a, const cd* b, cd* c, int d) {
    for (int r = 0; r < d; ++r)
        for (int col = 0; col < d; ++col) {
            cd s = 0.0;
            for (int t = 0; t < d; ++t) s += a[(size_t)r * d + t] * b[(size_t)t * d + col];
            c[(size_t)r * d + col] = s;
        }
}

}  // namespace

void gate_matrix(int op, double theta, const double* mat, int nq, std::vector<cd>& m) {
    const cd I(0.0, 1.0);
    auto set2 = [&](cd a, cd b, cd c, cd d) { m = {a, b, c, d}; };
    switch (op) {
        case SV_OP_I: set2(1, 0, 0, 1); break;
        case SV_OP_H: set2(kR, kR, kR, -kR); break;
        case SV_OP_X: set2(0, 1, 1, 0); break;
        case SV_OP_Y: set2(0, -I, I, 0); break;
        case SV_OP_Z: set2(1, 0, 0, -1); break;
        case SV_OP_S: set2(1, 0, 0, I); break;
        case SV_OP_SDG: set2(1, 0, 0, -I); break;
        case SV_OP_T: set2(1, 0, 0, cd(kR, kR)); break;
        case SV_OP_TDG: set2(1, 0, 0, cd(kR, -kR)); break;
        case SV_OP_SQRTX: case SV_OP_SQRTXDG:
            set2(cd(0.5, 0.5), cd(0.5, -0.5), cd(0.5, -0.5), cd(0.5, 0.5));
            if (op == SV_OP_SQRTXDG) conj_transpose(m, 2);
            break;
        case SV_OP_SQRTY: case SV_OP_SQRTYDG:
            set2(cd(0.5, 0.5), cd(-0.5, -0.5), cd(0.5, 0.5), cd(0.5, 0.5));
            if (op == SV_OP_SQRTYDG) conj_transpose(m, 2);
            break;
        case SV_OP_SQRTW: case SV_OP_SQRTWDG:
            set2(cd(0.5, 0.5), cd(0.0, -kR), cd(kR, 0.0), cd(0.5, 0.5));
            if (op == SV_OP_SQRTWDG) conj_transpose(m, 2);
            break;
        case SV_OP_RX: {
            const double c = std::cos(theta / 2), s = std::sin(theta / 2);
            set2(c, cd(0, -s), cd(0, -s), c);
            break;
        }
        case SV_OP_RY: {
            const double c = std::cos(theta / 2), s = std::sin(theta / 2);
            set2(c, -s, s, c);
            break;
        }
        case SV_OP_RZ: {
            const double c = std::cos(theta / 2), s = std::sin(theta / 2);
            set2(cd(c, -s), 0, 0, cd(c, s));
            break;
        }
        case SV_OP_P: set2(1, 0, 0, cd(std::cos(theta), std::sin(theta))); break;
        case SV_OP_CZ:
            m.assign(16, 0.0);
            m[0] = m[5] = m[10] = 1.0;
            m[15] = -1.0;
            break;
        case SV_OP_CP:
            m.assign(16, 0.0);
            m[0] = m[5] = m[10] = 1.0;
            m[15] = cd(std::cos(theta), std::sin(theta));
            break;
        case SV_OP_CNOT:  // control = local bit 0, target = local bit 1: 1 <-> 3
            m.assign(16, 0.0);
            m[0 * 4 + 0] = 1.0;
            m[2 * 4 + 2] = 1.0;
            m[3 * 4 + 1] = 1.0;
            m[1 * 4 + 3] = 1.0;
            break;
        case SV_OP_SWAP:  // 1 <-> 2
            m.assign(16, 0.0);
            m[0] = 1.0;
            m[3 * 4 + 3] = 1.0;
            m[2 * 4 + 1] = 1.0;
            m[1 * 4 + 2] = 1.0;
            break;
        case SV_OP_MAT: {
            const int d = 1 << nq;
            m.resize((size_t)d * d);
            for (int i = 0; i < d * d; ++i) m[i] = cd(mat[2 * i], mat[2 * i + 1]);
            break;
        }
        case SV_OP_DIAG: {
            const int d = 1 << nq;
            m.assign((size_t)d * d, 0.0);
            for (int i = 0; i < d; ++i) m[(size_t)i * d + i] = cd(mat[2 * i], mat[2 * i + 1]);
            break;
        }
        default: m.clear(); break;
    }
}

std::string validate_circuit(const sv_circuit* c, int n_qubits) {
    std::ostringstream e;
    if (!c) return "circuit is NULL";
    if (c->n_qubits != n_qubits) {
        e << "circuit has " << c->n_qubits << " qubits, context has " << n_qubits;
        return e.str();
    }
    if (c->n_gates < 0) return "n_gates < 0";
    if (c->n_gates > 0 && !c->gates) return "gates is NULL";
    if (c->n_params < 0) return "n_params < 0";
    for (int i = 0; i < c->n_gates; ++i) {
        const sv_gate& g = c->gates[i];
        if (g.op < 0 || g.op >= SV_OP_COUNT_) {
            e << "gate " << i << ": unknown op " << g.op;
            return e.str();
        }
        const int want = op_arity(g.op);
        if (g.nq < 1 || g.nq > 6 || (want > 0 && g.nq != want)) {
            e << "gate " << i << ": op " << g.op << " with nq=" << g.nq;
            return e.str();
        }
        uint64_t seen = 0;
        for (int t = 0; t < g.nq; ++t) {
            if (g.q[t] < 0 || g.q[t] >= n_qubits) {
                e << "gate " << i << ": qubit " << g.q[t] << " out of range [0," << n_qubits << ")";
                return e.str();
            }
            if ((seen >> g.q[t]) & 1ull) {
                e << "gate " << i << ": duplicate qubit " << g.q[t];
                return e.str();
            }
            seen |= 1ull << g.q[t];
        }
        if (g.param >= 0) {
            if (!op_takes_angle(g.op)) {
                e << "gate " << i << ": op " << g.op << " takes no parameter";
                return e.str();
            }
            if (g.param >= c->n_params) {
                e << "gate " << i << ": param " << g.param << " >= n_params " << c->n_params;
                return e.str();
            }
        }
        if (g.op == SV_OP_MAT || g.op == SV_OP_DIAG) {
            const int64_t need = 2ll * (1ll << g.nq) * (g.op == SV_OP_MAT ? (1ll << g.nq) : 1ll);
            if (!c->mats || g.mat < 0 || (int64_t)g.mat + need > c->n_mat_doubles) {
                e << "gate " << i << ": matrix offset " << g.mat << " out of range";
                return e.str();
            }
        }
        if (!std::isfinite(g.theta)) {
            e << "gate " << i << ": non-finite angle";
            return e.str();
        }
    }
    return "";
}

uint64_t circuit_hash(const sv_circuit* c, uint64_t seed) {
    uint64_t h = 1469598103934665603ull ^ seed;
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 255u;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)c->n_qubits);
    mix((uint64_t)c->n_gates);
    mix((uint64_t)c->n_params);
    for (int i = 0; i < c->n_gates; ++i) {
        const sv_gate& g = c->gates[i];
        mix((uint64_t)g.op | ((uint64_t)g.nq << 8) | ((uint64_t)(uint32_t)g.param << 16));
        for (int t = 0; t < g.nq; ++t) mix((uint64_t)g.q[t]);
    }
    return h;
}

// Signature of the value-dependent planning decisions of an IR list: the
// kind, structure and flags of every gate, whether its matrix is real, and
// for a general diagonal whether every entry but the last is 1 (the masked
// form of the plain sweep).  Two calls whose circuits have the same structure
// but values that change any of these decisions get different plans.
uint64_t ir_signature(const std::vector<IRGate>& ir) {
    uint64_t h = 0x243f6a8885a308d3ull;
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 255u;
            h *= 1099511628211ull;
        }
    };
    mix(ir.size());
    for (const IRGate& g : ir) {
        bool unit = false;
        if (g.kind == K_DIAGG) {
            unit = true;
            for (int b = 0; b < g.m.nb && unit; ++b)
                for (int i = 0; i + 1 < g.m.d; ++i)
                    if (g.m.at(b)[i] != cd(1.0, 0.0)) { unit = false; break; }
        }
        mix((uint64_t)g.kind | ((uint64_t)g.k << 4) | ((uint64_t)g.skind << 8) | ((uint64_t)g.perm << 16) |
            ((uint64_t)real_gate(g) << 20) | ((uint64_t)unit << 21) | ((uint64_t)g.grad << 22) |
            ((uint64_t)g.m.diag << 23) | ((uint64_t)(g.m.nb > 1) << 24) | ((uint64_t)(uint32_t)g.gen << 28) |
            ((uint64_t)(uint32_t)g.param << 32));
        mix((uint64_t)(g.alpha[0] & 7) | ((uint64_t)(g.alpha[1] & 7) << 3) | ((uint64_t)(g.beta & 7) << 6) |
            ((uint64_t)(g.bf_pre & 7) << 9) | ((uint64_t)(g.bf_post & 7) << 12) | ((uint64_t)(g.bf_g & 7) << 15));
        for (int t = 0; t < g.k; ++t) mix((uint64_t)g.q[t]);
    }
    return h;
}

namespace {

int gen_of(int op) {
    switch (op) {
        case SV_OP_RX: return GEN_X;
        case SV_OP_RY: return GEN_Y;
        case SV_OP_RZ: case SV_OP_P: return GEN_Z;
        case SV_OP_CP: return GEN_P11;
        default: return 0;
    }
}

int perm_of(int op) {
    switch (op) {
        case SV_OP_X: return PK_X;
        case SV_OP_Y: return PK_Y;
        case SV_OP_CNOT: return PK_CNOT;
        case SV_OP_SWAP: return PK_SWAP;
        default: return PK_NONE;
    }
}

// The one-qubit gates of the benchmark family as one unnormalised butterfly
// H' = [[1,1],[1,-1]] between 8th-root diagonals:  G = w^g diag(1, w^post)
// H' diag(1, w^pre) / sqrt(2),  w = e^{i pi/4}.  With the principal roots
// (sqrt(G) = ((1+i)/2) I + ((1-i)/2) G) and W = (X+Y)/sqrt(2) = T X T^dag:
//   H = H'/sqrt(2);  sqrt(X) = w S^dag H S^dag;  sqrt(Y) = w H Z;
//   sqrt(W) = T sqrt(X) T^dag = w (T S^dag) H (S^dag T^dag),
// and the conjugate transposes for the adjoint sweep.  Returns false for
// other gates.
bool butterfly_form(int op, bool inv, int& pre, int& post, int& g) {
    int a = -1, b = -1, c = 0;
    switch (op) {
        case SV_OP_H: a = 0; b = 0; c = 0; break;
        case SV_OP_SQRTX: a = 6; b = 6; c = 1; break;
        case SV_OP_SQRTY: a = 4; b = 0; c = 1; break;
        case SV_OP_SQRTW: a = 5; b = 7; c = 1; break;
        case SV_OP_SQRTXDG: a = 2; b = 2; c = 7; break;
        case SV_OP_SQRTYDG: a = 0; b = 4; c = 7; break;
        case SV_OP_SQRTWDG: a = 1; b = 3; c = 7; break;
        default: return false;
    }
    if (inv) {  // (w^c D_b H' D_a)^dag = w^-c D_-a H' D_-b
        pre = (8 - b) & 7;
        post = (8 - a) & 7;
        g = (8 - c) & 7;
    } else {
        pre = a;
        post = b;
        g = c;
    }
    return true;
}

// One IR gate from a circuit gate (inverse = conjugate transpose when `inv`).
IRGate make_ir(const sv_circuit* c, int gi, const double* params, const BuildOpts& o, bool inv) {
    const sv_gate& g = c->gates[gi];
    IRGate r;
    r.k = g.nq;
    for (int t = 0; t < g.nq; ++t) r.q[t] = g.q[t];
    r.src = gi;
    r.param = g.param;
    r.gen = gen_of(g.op);
    const int a8 = diag8_alpha(g.op);
    if (a8 >= 0 || g.op == SV_OP_CZ) {
        r.kind = K_DIAG8;
        if (g.op == SV_OP_CZ) r.beta = 4;
        else r.alpha[0] = inv ? (8 - a8) & 7 : a8;
        return r;
    }
    const bool diag = g.op == SV_OP_RZ || g.op == SV_OP_P || g.op == SV_OP_CP || g.op == SV_OP_DIAG;
    r.kind = diag ? K_DIAGG : K_DENSE;
    if (!diag && o.structured && butterfly_form(g.op, inv, r.bf_pre, r.bf_post, r.bf_g)) r.skind = OP_BF;
    r.perm = inv && g.op == SV_OP_Y ? PK_Y : perm_of(g.op);
    const int d = 1 << g.nq;
    const int nb = (g.param >= 0) ? o.batch : 1;
    r.m.d = d;
    r.m.nb = nb;
    r.m.diag = diag;
    r.m.v.resize((size_t)nb * (diag ? d : d * d));
    std::vector<cd> m;
    for (int b = 0; b < nb; ++b) {
        const double th = g.param >= 0 ? params[(size_t)b * c->n_params + g.param] : g.theta;
        gate_matrix(g.op, th, (g.op == SV_OP_MAT || g.op == SV_OP_DIAG) ? c->mats + g.mat : nullptr, g.nq, m);
        if (inv) conj_transpose(m, d);
        cd* dst = r.m.at(b);
        if (diag)
            for (int i = 0; i < d; ++i) dst[i] = m[(size_t)i * d + i];
        else
            std::copy(m.begin(), m.end(), dst);
    }
    if (g.param >= 0) {
        r.real = g.op == SV_OP_RY;   // real for every angle
    } else {
        r.real = true;
        for (const cd& v : r.m.v) if (v.imag() != 0.0) r.real = false;
    }
    return r;
}


// Dense 2x2 matrix of a one-qubit IR gate (any kind), per state.
MatB as_dense1(const IRGate& g) {
    MatB r;
    r.d = 2;
    r.diag = false;
    if (g.kind == K_DIAG8) {
        r.nb = 1;
        r.v = {1.0, 0.0, 0.0, 1.0};
        switch (g.alpha[0] & 7) {
            case 1: r.v[3] = cd(kR, kR); break;
            case 2: r.v[3] = cd(0, 1); break;
            case 3: r.v[3] = cd(-kR, kR); break;
            case 4: r.v[3] = -1.0; break;
            case 5: r.v[3] = cd(-kR, -kR); break;
            case 6: r.v[3] = cd(0, -1); break;
            case 7: r.v[3] = cd(kR, -kR); break;
            default: break;
        }
        return r;
    }
    if (g.kind == K_DIAGG) {
        r.nb = g.m.nb;
        r.v.resize((size_t)r.nb * 4);
        for (int b = 0; b < r.nb; ++b) {
            const cd* s = g.m.at(b);
            cd* t = r.at(b);
            t[0] = s[0]; t[1] = 0.0; t[2] = 0.0; t[3] = s[1];
        }
        return r;
    }
    return g.m;
}

// a := b * a for one-qubit matrices (per state)
MatB mul1(const MatB& b, const MatB& a) {
    MatB r;
    r.d = 2;
    r.diag = false;
    r.nb = std::max(a.nb, b.nb);
    r.v.resize((size_t)r.nb * 4);
    for (int s = 0; s < r.nb; ++s) matmul(b.at(s), a.at(s), r.at(s), 2);
    return r;
}

MatB diag_of(const IRGate& g) {
    // diagonal entries (2) of a one-qubit diagonal gate
    MatB r;
    r.d = 2;
    r.diag = true;
    if (g.kind == K_DIAGG) return g.m;
    MatB d = as_dense1(g);
    r.nb = 1;
    r.v = {d.v[0], d.v[3]};
    return r;
}

}  // namespace

std::vector<IRGate> build_ir(const sv_circuit* c, const double* params, const BuildOpts& o, ProductInit* pinit,
                             int n) {
    std::vector<IRGate> in;
    in.reserve((size_t)c->n_gates * (o.backward ? 2 : 1));
    std::vector<char> consumed((size_t)c->n_gates, 0);

    // Leading one-qubit gates on |0...0> become a product-state initialisation
    // (the paper turns the initial Hadamard layer into a uniform initial state,
    // Sec. 4.5 footnote and Sec. 6.1).
    if (pinit) pinit->used = false;
    if (!o.backward && o.product_init && pinit) {
        std::vector<std::vector<cd>> v((size_t)n, std::vector<cd>{1.0, 0.0});
        std::vector<char> leading((size_t)n, 1);
        int folded = 0;
        for (int i = 0; i < c->n_gates; ++i) {
            const sv_gate& g = c->gates[i];
            if (g.nq == 1 && leading[g.q[0]] && g.param < 0) {
                std::vector<cd> m;
                gate_matrix(g.op, g.theta, (g.op == SV_OP_MAT || g.op == SV_OP_DIAG) ? c->mats + g.mat : nullptr, 1, m);
                std::vector<cd>& x = v[g.q[0]];
                const cd a = m[0] * x[0] + m[1] * x[1], b = m[2] * x[0] + m[3] * x[1];
                x = {a, b};
                consumed[i] = 1;
                ++folded;
            } else {
                for (int t = 0; t < g.nq; ++t) leading[g.q[t]] = 0;
            }
        }
        if (folded > 0) {
            pinit->used = true;
            pinit->folded = folded;
            pinit->nlo = n / 2;
            const int nlo = pinit->nlo, nhi = n - nlo;
            pinit->lo.assign((size_t)1 << nlo, 1.0);
            pinit->hi.assign((size_t)1 << nhi, 1.0);
            for (uint64_t i = 0; i < (1ull << nlo); ++i) {
                cd p = 1.0;
                for (int q = 0; q < nlo; ++q) p *= v[q][(i >> q) & 1];
                pinit->lo[i] = p;
            }
            for (uint64_t i = 0; i < (1ull << nhi); ++i) {
                cd p = 1.0;
                for (int q = 0; q < nhi; ++q) p *= v[nlo + q][(i >> q) & 1];
                pinit->hi[i] = p;
            }
        }
    }

    // The gates' matrices for many parameter sets are computed in parallel
    // (make_ir is independent per gate); errors are reported in gate order.
    std::vector<IRGate> made;
    if (o.batch >= 8 && c->n_gates >= 16) {
        made.resize((size_t)c->n_gates);
        std::vector<std::string> errs((size_t)c->n_gates);
        host_parallel_for(c->n_gates, [&](int i) {
            if (consumed[i]) return;
            try {
                made[i] = make_ir(c, i, params, o, o.backward);
            } catch (const std::exception& e) {
                errs[i] = e.what();
            }
        });
        for (int i = 0; i < c->n_gates; ++i)
            if (!errs[i].empty()) throw std::runtime_error(errs[i]);
    }
    auto gate_ir = [&](int i) { return made.empty() ? make_ir(c, i, params, o, o.backward) : std::move(made[i]); };
    if (!o.backward) {
        for (int i = 0; i < c->n_gates; ++i)
            if (!consumed[i]) in.push_back(gate_ir(i));
    } else {
        // Each parametric gate exp(-i theta G / 2) commutes with its
        // generator G, so Im <lambda|G|psi> has the same value before and
        // after the gate's inverse is applied to both states.  With the
        // structured forms the term goes after it: the inverse takes over the
        // pending phases on its qubits (Sec. 4.3), and the term then finds
        // none there.  With dense blocks it goes before, where it does not
        // separate the inverse from the gates applied next on its qubits.
        for (int i = c->n_gates - 1; i >= 0; --i) {
            const sv_gate& g = c->gates[i];
            IRGate gr;
            if (g.param >= 0) {
                gr.grad = 1;
                gr.kind = K_DENSE;
                gr.k = g.nq;
                for (int t = 0; t < g.nq; ++t) gr.q[t] = g.q[t];
                gr.param = g.param;
                gr.gen = gen_of(g.op);
                gr.src = i;
                if (!o.structured) in.push_back(gr);
            }
            in.push_back(gate_ir(i));
            if (g.param >= 0 && o.structured) in.push_back(gr);
        }
    }
    if (!o.fuse) return in;

    // One-qubit fusion.  A chain on qubit q stays open while only diagonal
    // gates touch q; a dense chain cannot absorb a dense gate once a
    // multi-qubit diagonal has touched q ("blocked"), but diagonal one-qubit
    // gates commute with those and may still join.
    std::vector<IRGate> out;
    out.reserve(in.size());
    std::vector<char> alive;
    std::vector<int> open((size_t)n, -1);
    std::vector<char> open_diag((size_t)n, 0), blocked((size_t)n, 0);
    auto is_diag = [](const IRGate& g) { return g.kind != K_DENSE; };
    auto fusable = [&](const IRGate& g) {
        if (g.grad || g.k != 1) return false;
        if (o.backward && g.param >= 0) return false;
        if (g.skind) return false;
        if (o.structured && g.perm != PK_NONE) return false;   // applied as a register permutation
        if (o.structured && g.kind == K_DIAG8) return false;
        return true;
    };
    for (IRGate& g : in) {
        if (fusable(g)) {
            const int q = g.q[0];
            const int oi = open[q];
            if (oi >= 0) {
                IRGate& h = out[oi];
                if (is_diag(g) && open_diag[q]) {
                    if (g.kind == K_DIAG8 && h.kind == K_DIAG8) {
                        h.alpha[0] = (h.alpha[0] + g.alpha[0]) & 7;
                    } else {
                        MatB a = diag_of(h), b = diag_of(g), r;
                        r.d = 2; r.diag = true; r.nb = std::max(a.nb, b.nb);
                        r.v.resize((size_t)r.nb * 2);
                        for (int s = 0; s < r.nb; ++s) {
                            r.at(s)[0] = a.at(s)[0] * b.at(s)[0];
                            r.at(s)[1] = a.at(s)[1] * b.at(s)[1];
                        }
                        h.real = real_gate(h) && real_gate(g);
                        h.kind = K_DIAGG; h.m = r; h.perm = PK_NONE; h.param = -1; h.gen = 0;
                    }
                    continue;
                }
                if (open_diag[q]) {
                    // dense g after a diagonal chain: move the chain to here
                    IRGate f = g;
                    f.m = mul1(as_dense1(g), as_dense1(h));
                    f.real = real_gate(g) && real_gate(h);
                    f.kind = K_DENSE; f.perm = PK_NONE; f.param = -1; f.gen = 0; f.skind = 0;
                    f.src = h.src;
                    alive[oi] = 0;
                    out.push_back(std::move(f));
                    alive.push_back(1);
                    open[q] = (int)out.size() - 1;
                    open_diag[q] = 0;
                    blocked[q] = 0;
                    continue;
                }
                if (is_diag(g) || !blocked[q]) {
                    h.real = real_gate(g) && real_gate(h);
                    h.m = mul1(as_dense1(g), h.m);
                    h.kind = K_DENSE; h.perm = PK_NONE; h.param = -1; h.gen = 0; h.skind = 0;
                    continue;
                }
            }
            open_diag[q] = is_diag(g);
            out.push_back(std::move(g));   // `in` is not read again
            alive.push_back(1);
            open[q] = (int)out.size() - 1;
            blocked[q] = 0;
            continue;
        }
        if (!g.grad && g.kind != K_DENSE) {
            for (int t = 0; t < g.k; ++t)
                if (open[g.q[t]] >= 0 && !open_diag[g.q[t]]) blocked[g.q[t]] = 1;
        } else {
            for (int t = 0; t < g.k; ++t) open[g.q[t]] = -1;
        }
        // A diagonal one-qubit gate that cannot fuse (structured mode T) must
        // still keep later dense gates from jumping over it.
        if (g.k == 1 && g.kind != K_DENSE) open[g.q[0]] = -1;
        out.push_back(std::move(g));
        alive.push_back(1);
    }
    std::vector<IRGate> res;
    res.reserve(out.size());
    for (size_t i = 0; i < out.size(); ++i)
        if (alive[i]) res.push_back(std::move(out[i]));
    if (o.fuse_k >= 2 && !o.structured) return fuse_blocks(std::move(res), o.fuse_k, n);
    return res;
}

// Complex product without the library's inf/NaN recovery (all entries here
// are finite).
static inline cd cmul_plain(cd a, cd b) {
    return cd(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
}

// Dense blocks of at most kmax qubits (Sec. 4.2 contrasts this with its own
// clustering; used for the dense mode and its width sweep).  Open blocks have
// disjoint qubit sets, so they commute; a gate joins the blocks it touches
// when their union stays within kmax qubits, otherwise those blocks are
// closed (emitted) and the gate starts a new one.  Products are formed in
// FP64 and rounded once when the plan's matrix pool is filled.  Gradient
// pseudo-gates and wider gates close the blocks on their qubits.
//
// Block members are kept as linked lists over the input indices (merging
// blocks concatenates lists) and the products are formed in reused buffers,
// so a block costs one allocation, for its own matrix.
std::vector<IRGate> fuse_blocks(std::vector<IRGate>&& in, int kmax, int n) {
    (void)n;
    struct Blk {
        uint64_t qm;
        int head, tail, count;   // member list in circuit order (links in `nxt`)
    };
    std::vector<int> nxt(in.size(), -1);
    std::vector<IRGate> out;
    out.reserve(in.size());
    std::vector<Blk> open;
    open.reserve(64);
    std::vector<cd> U, gath;
    const double c8 = std::sqrt(0.5);
    const cd tab8[8] = {cd(1, 0), cd(c8, c8), cd(0, 1), cd(-c8, c8), cd(-1, 0), cd(-c8, -c8), cd(0, -1), cd(c8, -c8)};
    auto emit = [&](const Blk& B) {
        if (B.count == 1) {
            out.push_back(std::move(in[B.head]));
            return;
        }
        IRGate f;
        int qs[6], k = 0;
        for (int q = 0; q < 64; ++q) if ((B.qm >> q) & 1) qs[k++] = q;
        f.k = k;
        for (int t = 0; t < k; ++t) f.q[t] = qs[t];
        f.src = in[B.head].src;
        int nb = 1;
        bool diag = true, real = true;
        for (int gi = B.head; gi >= 0; gi = nxt[gi]) {
            const IRGate& g = in[gi];
            if (g.kind == K_DENSE) diag = false;
            if (!real_gate(g)) real = false;
            if (g.kind != K_DIAG8) nb = std::max(nb, g.m.nb);
        }
        const int D = 1 << k;
        f.m.d = D;
        f.m.nb = nb;
        f.m.diag = diag;
        f.m.v.assign((size_t)nb * (diag ? D : (size_t)D * D), 0.0);
        U.resize((size_t)D * D);
        gath.resize((size_t)D * D);
        for (int b = 0; b < nb; ++b) {
            std::fill(U.begin(), U.end(), cd(0.0));
            for (int i = 0; i < D; ++i) U[(size_t)i * D + i] = 1.0;
            for (int gi = B.head; gi >= 0; gi = nxt[gi]) {
                const IRGate& g = in[gi];
                const int kg = g.k, dg = 1 << kg;
                int pos[6];
                for (int t = 0; t < kg; ++t)
                    for (int s2 = 0; s2 < k; ++s2) if (qs[s2] == g.q[t]) pos[t] = s2;
                // block-local index of gate-local index l (bits deposited at pos)
                int dep[64];
                uint32_t gmask = 0;
                for (int t = 0; t < kg; ++t) gmask |= 1u << pos[t];
                for (int l = 0; l < dg; ++l) {
                    int idx = 0;
                    for (int t = 0; t < kg; ++t) if ((l >> t) & 1) idx |= 1 << pos[t];
                    dep[l] = idx;
                }
                if (g.kind == K_DIAG8 || g.m.diag) {
                    // U <- diag(G_emb) U: scale the rows
                    const cd* m = g.kind == K_DIAG8 ? nullptr : g.m.at(g.m.nb == 1 ? 0 : b);
                    for (int l = 0; l < dg; ++l) {
                        cd v;
                        if (!m) {
                            int e = 0;
                            if (l & 1) e += g.alpha[0];
                            if (kg > 1 && (l & 2)) e += g.alpha[1];
                            if (kg > 1 && (l & 3) == 3) e += g.beta;
                            v = tab8[e & 7];
                        } else {
                            v = m[l];
                        }
                        for (int base = 0; base < D; ++base) {
                            if (base & gmask) continue;
                            cd* row = U.data() + (size_t)(base | dep[l]) * D;
                            for (int c = 0; c < D; ++c) {
                                // + 0.0 keeps the zeros positive, as a sum started from 0 does
                                const cd r = cmul_plain(v, row[c]);
                                row[c] = cd(r.real() + 0.0, r.imag() + 0.0);
                            }
                        }
                    }
                    continue;
                }
                // U <- G_emb U: rows base|dep[l] mix through G, all columns at once
                const cd* G = g.m.at(g.m.nb == 1 ? 0 : b);
                for (int base = 0; base < D; ++base) {
                    if (base & gmask) continue;
                    for (int l = 0; l < dg; ++l)
                        std::copy_n(U.data() + (size_t)(base | dep[l]) * D, D, gath.data() + (size_t)l * D);
                    for (int l = 0; l < dg; ++l) {
                        cd* row = U.data() + (size_t)(base | dep[l]) * D;
                        for (int c = 0; c < D; ++c) row[c] = 0.0;
                        for (int l2 = 0; l2 < dg; ++l2) {
                            const cd x = G[(size_t)l * dg + l2];
                            const cd* src = gath.data() + (size_t)l2 * D;
                            for (int c = 0; c < D; ++c) row[c] += cmul_plain(x, src[c]);
                        }
                    }
                }
            }
            cd* dst = f.m.at(b);
            if (diag) for (int i = 0; i < D; ++i) dst[i] = U[(size_t)i * D + i];
            else std::copy(U.begin(), U.end(), dst);
        }
        f.kind = diag ? K_DIAGG : K_DENSE;
        f.real = real;
        f.param = -1;
        f.gen = 0;
        f.perm = PK_NONE;
        out.push_back(std::move(f));
    };
    // emit the open blocks that touch qm (in order) and keep the others (in order)
    auto close_touching = [&](uint64_t qm) {
        size_t w = 0;
        for (size_t r = 0; r < open.size(); ++r) {
            if (open[r].qm & qm) emit(open[r]);
            else open[w++] = open[r];
        }
        open.resize(w);
    };
    for (size_t i = 0; i < in.size(); ++i) {
        const IRGate& g = in[i];
        const uint64_t qm = g.qmask();
        if (g.grad || g.k > kmax || g.skind) {
            close_touching(qm);
            out.push_back(std::move(in[i]));
            continue;
        }
        uint64_t un = qm;
        for (const Blk& B : open) if (B.qm & qm) un |= B.qm;
        if (__builtin_popcountll(un) <= kmax) {
            // merge the touching blocks (in order) and the gate into one block at the end
            Blk nbk{un, -1, -1, 0};
            size_t w = 0;
            for (size_t r = 0; r < open.size(); ++r) {
                const Blk& B = open[r];
                if (B.qm & qm) {
                    if (nbk.head < 0) nbk.head = B.head;
                    else nxt[nbk.tail] = B.head;
                    nbk.tail = B.tail;
                    nbk.count += B.count;
                } else {
                    open[w++] = B;
                }
            }
            open.resize(w);
            if (nbk.head < 0) nbk.head = (int)i;
            else nxt[nbk.tail] = (int)i;
            nbk.tail = (int)i;
            nbk.count += 1;
            open.push_back(nbk);
        } else {
            close_touching(qm);
            open.push_back(Blk{qm, (int)i, (int)i, 1});
        }
    }
    for (const Blk& B : open) emit(B);
    return out;
}

}  // namespace svmi
