// Host-side gate IR, fusion and planning (internal to libsvmi).
#pragma once
#include <complex>
#include <cstdint>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "plan.h"
#include "sv.h"

namespace svmi {

using cd = std::complex<double>;

enum Kind { K_DENSE = 0, K_DIAG8 = 1, K_DIAGG = 2 };
enum PermKind { PK_NONE = 0, PK_X = 1, PK_Y = 2, PK_CNOT = 3, PK_SWAP = 4 };

// Per-state matrices: nb == 1 (shared by the whole batch) or nb == batch.
struct MatB {
    int d = 0;                 // rows (= columns for dense, entries for diagonal)
    int nb = 1;
    bool diag = false;         // entries are a diagonal (d values per state)
    std::vector<cd> v;         // nb * (diag ? d : d*d)
    const cd* at(int b) const { return v.data() + (size_t)(nb == 1 ? 0 : b) * (diag ? d : d * d); }
    cd* at(int b) { return v.data() + (size_t)(nb == 1 ? 0 : b) * (diag ? d : d * d); }
};

struct IRGate {
    int kind = K_DENSE;
    int k = 1;
    int q[6] = {0, 0, 0, 0, 0, 0};
    int alpha[2] = {0, 0};     // DIAG8 linear exponents (mod 8) on q[0], q[1]
    int beta = 0;              // DIAG8 pair exponent on (q[0], q[1])
    int skind = 0;             // OP_BF: w^g diag(1, w^post) H' diag(1, w^pre) / sqrt(2), else 0
    int bf_pre = 0, bf_post = 0, bf_g = 0;   // exponents of w = e^{i pi/4} (mod 8)
    bool real = false;         // the matrix is real for every parameter value
    int perm = PK_NONE;        // exact permutation gate (plain path)
    int src = -1;              // first source gate
    int param = -1;            // parameter index (unfused parameterised gate)
    int gen = 0;               // GradGen for the adjoint
    int grad = 0;              // 1 = pseudo-gate: gradient reduction (adjoint sweep)
    MatB m;                    // matrix (dense) or diagonal entries (DIAGG); empty for DIAG8
    uint64_t qmask() const {
        uint64_t r = 0;
        for (int t = 0; t < k; ++t) r |= 1ull << q[t];
        return r;
    }
};

struct BuildOpts {
    int batch = 1;
    bool structured = true;
    bool fuse = true;            // fuse one-qubit chains
    bool backward = false;       // adjoint sweep: inverse gates in reverse + gradient pseudo-gates
    bool product_init = false;   // fold leading one-qubit gates (state is |0..0>)
    int fuse_k = 0;              // dense mode: fuse gates into blocks of <= fuse_k qubits (0/1 = off)
};

struct ProductInit {
    bool used = false;
    int nlo = 0;
    std::vector<cd> lo, hi;      // tensor-product tables
    int folded = 0;
};

// Validation of a circuit (and parameter count); returns empty string when OK.
std::string validate_circuit(const sv_circuit* c, int n_qubits);

// Gate matrix (row-major, local index order q[0] = LSB) in FP64.
void gate_matrix(int op, double theta, const double* mat, int nq, std::vector<cd>& out);

// Circuit -> IR (with fusion per BuildOpts).  params: batch * n_params.
std::vector<IRGate> build_ir(const sv_circuit* c, const double* params, const BuildOpts& o,
                             ProductInit* pinit, int n_qubits);

// True when the gate's matrix is real for every parameter value.
bool real_gate(const IRGate& g);

// Dense blocks of at most kmax qubits from an IR gate list.
std::vector<IRGate> fuse_blocks(std::vector<IRGate>&& in, int kmax, int n);

// Structural hash of a circuit for the plan cache.
uint64_t circuit_hash(const sv_circuit* c, uint64_t seed);

// Hash of the value-dependent planning decisions of an IR list (real
// matrices, unit diagonals, gate kinds); combined with circuit_hash in every
// plan-cache key, so that new angles or matrices never reuse a plan made for
// values that decided differently.
uint64_t ir_signature(const std::vector<IRGate>& ir);

// ----------------------------------------------- the paper's own plan (ablation)
//
// Kind clusters of Sec. 4.2 formed by the reordering scan of Sec. 4.5, with
// the bitmask encodings of Sec. 4.3 (8th-root phases as exponent bit-planes,
// CZ gates as one mask per qubit) and one-qubit layers of one gate kind.

enum PaperStep { PS_DIAG = 0, PS_LAYER = 1, PS_GATES = 2 };

struct PStep {
    int type = PS_DIAG;
    int kind = 0;                       // the clustered gate kind (sv_op of the layer; SV_OP_T for DIAG)
    uint64_t e8[3] = {0, 0, 0};         // PS_DIAG: exponent of w per qubit, bit-planes (mod 8)
    std::vector<uint64_t> cz;           // PS_DIAG: m_k = partners l < k of the CZ gates on qubit k
    std::vector<std::pair<int, int>> layer;   // PS_LAYER: (qubit, PaperGate), sorted by qubit
    std::vector<int> gates;             // circuit gates of the step in execution order
};

struct PaperPlan {
    int n = 0;
    std::vector<PStep> steps;
};

// Cluster a circuit by kind (Sec. 4.5 scan).  Gates other than the 8th-root
// diagonals, CZ, H and the square-root family form single-gate PS_GATES steps
// (consecutive ones merged).
PaperPlan paper_plan(const sv_circuit* c);
// Text form of a paper plan (one line per step) for host-side checks.
std::string paper_trace(const PaperPlan& p);

// Geometry and fusion of the items of one width in a heterogeneous batch
// (T, L = 0: the defaults).
struct BatchGeom {
    int structured = 1;
    int fuse_k = 4;
    int T = 0;
    int L = 0;
    int beam = 8;   // planner beam width (not tuned)
};
using GeomTable = std::map<int, BatchGeom>;   // width -> choice

// ----------------------------------------------------------------- planning

struct PlanCfg {
    int dtype = SV_C64;
    int T = 13;                  // local bits per pass
    int L = 5;                   // contiguous low bits
    int nt = 512;                // threads per workgroup
    int max_fuse_k = 4;
    bool two = false;            // adjoint sweep (psi and lambda)
    int beam = 1;                // width of the local-set beam search (1 = greedy per pass)
    uint64_t first_pin = 0;      // qubits the first tile pass must hold locally
};

// Pool recipe: what goes into each pool slot (computed per call).
struct Recipe {
    enum Type { DENSE = 0, DIAG = 1, SCALE = 2, VALUE = 3, PHASETAB = 4, BFTAB = 5 } type = DENSE;
    int gate = -1;               // IR gate
    int perm[6] = {0, 1, 2, 3, 4, 5};  // slot order: new local bit t <- gate local bit perm[t]
    int k = 0;
    double scale = 1.0;          // SCALE
    int twiddle = 0;             // DENSE k = 1: multiply column 1 by e^{i pi twiddle/4}
    bool inplace = false;        // DENSE k = 1: also store the in-place form (r, d, flag, sign table)
    int slot = 0;                // DENSE k = 1 in-place / BFTAB: register slot of the qubit
    uint32_t rm = 0;             // partner register slots
    int bf_m = 0;                // BFTAB: twiddle exponent M
    cd value{1.0, 0.0};          // VALUE
    uint64_t off = 0;            // pool offset (complex elements)
    uint64_t size = 0;
    bool varies = false;         // differs per batch state
};

enum StepType { ST_TILE = 0, ST_DENSE = 1, ST_MASKED = 2, ST_DIAG = 3, ST_SWAP = 4, ST_GRAD = 5 };

struct Step {
    int type = ST_TILE;
    int pass = -1;               // ST_TILE
    int k = 0;
    int tq[6] = {0, 0, 0, 0, 0, 0};
    uint64_t mask = 0, ones = 0, flip = 0;
    int mode = 0;                // ST_MASKED/ST_SWAP mode, ST_GRAD generator
    int slot = -1;               // ST_GRAD: gradient slot
    int recipe = -1;
};

struct EncodedPlan {
    PlanCfg cfg;
    int n = 0;
    std::vector<DPass> passes;
    std::vector<DPhase> phases;
    std::vector<DOp> ops;
    std::vector<DForm> forms;
    std::vector<DPair> pairs;
    std::vector<uint16_t> etab;
    std::vector<Recipe> recipes;
    std::vector<Step> steps;
    uint64_t pool_size = 0;      // complex elements per state
    bool pool_varies = false;
    uint64_t gpart_size = 0;     // doubles per state (gradient partials)
    int ngrad_total = 0;
    std::vector<int> grad_param; // grad slot (global) -> parameter index
    std::vector<double> grad_scale; // grad slot -> factor undoing the butterflies' growth at the reduction
    std::vector<uint64_t> grad_slot_off;  // per pass: first global grad slot
    // statistics
    int n_dense = 0, n_diag = 0, n_phase = 0, n_tile = 0, n_plain = 0;
    double flops = 0.0;
    double alu_ops = 0.0;        // vector arithmetic instructions per lane (an FMA counts once), tile passes
};

// Plan a fused sweep (tile passes) for an IR gate list.
void plan_fused(const std::vector<IRGate>& ir, int n, const PlanCfg& cfg, EncodedPlan& out,
                std::string* trace = nullptr);
// Plan a plain sweep (one kernel per gate).
void plan_plain(const std::vector<IRGate>& ir, int n, const PlanCfg& cfg, EncodedPlan& out);

// Fill the pool (state dtype, batch-major when it varies) from the recipes.
// fn(i) for i in [0, n) on a persistent pool of host threads (the caller
// takes part); runs inline when the pool is busy with another loop.
void host_parallel_for(int n, const std::function<void(int)>& fn);

void fill_pool(const EncodedPlan& p, const std::vector<IRGate>& ir, int batch,
               std::vector<unsigned char>& pool_bytes);

}  // namespace svmi
