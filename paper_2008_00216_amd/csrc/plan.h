// Device-visible simulation plan.
//
// The host planner turns a circuit into a "simulation plan" (Sec. 4.5: the
// schedule of gate sets handled by the kernels) made of tile passes.  A tile
// pass streams the whole state once: every workgroup gathers one tile of 2^T
// amplitudes (T "local" qubits: the L lowest index bits, contiguous in memory,
// plus H higher bits) into LDS, applies a list of register phases, and writes
// the tile back.  A register phase gives each thread the 16 amplitudes that
// differ in 4 chosen local bits ("register slots") and runs an op list on
// them in registers: dense blocks on up to 4 slots, diagonals, twiddled H'
// butterflies (Sec. 4.4's multiply-free one-qubit gates with the pending
// diagonal phases of Sec. 4.3 folded in), the 8th-root phase form of
// clustered T/S/Z/CZ gates (Sec. 4.3) and, for the adjoint sweep, gradient
// reductions.
//
// All structures are plain data; the planner fills them on the host and
// copies them to one device buffer per plan.
#pragma once
#ifndef __HIPCC_RTC__
#include <stdint.h>
#endif

namespace svmi {

constexpr int kRegBits = 4;           // register slots per phase
constexpr int kRegAmps = 1 << kRegBits;
constexpr int kMaxTileBits = 14;      // local qubits per tile pass
constexpr int kMaxHigh = 12;          // high local bits per pass
constexpr int kMaxGradPerPass = 128;  // gradient slots reduced per pass

// Unnormalised one-qubit factors of the paper's multiply-free family (the
// paper's own plan, Sec. 4.4): H = H'/sqrt(2), sqrt(X)(dg) = sqrt(X)(dg)'/2,
// sqrt(Y)(dg) = w^(+-1) sqrt(Y)(dg)'/sqrt(2) with w = e^{i pi/4}; PG_GEN is
// any other one-qubit matrix (applied as it is).
enum PaperGate { PG_H = 0, PG_SX = 1, PG_SXDG = 2, PG_SY = 3, PG_SYDG = 4, PG_GEN = 5 };

// Entries re + i im of the unnormalised factors:
//   H' = [[1, 1], [1, -1]],  sqrt(X)' = [[1+i, 1-i], [1-i, 1+i]],
//   sqrt(X)dg' = [[1-i, 1+i], [1+i, 1-i]],  sqrt(Y)' = [[1, -1], [1, 1]],
//   sqrt(Y)dg' = [[1, 1], [-1, 1]].
struct GInt {
    int re, im;
};
constexpr GInt gmul(GInt a, GInt b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
constexpr GInt pg_fac(int g, int r, int c) {
    return g == PG_H ? ((r & c) ? GInt{-1, 0} : GInt{1, 0})
         : g == PG_SX ? (r == c ? GInt{1, 1} : GInt{1, -1})
         : g == PG_SXDG ? (r == c ? GInt{1, -1} : GInt{1, 1})
         : g == PG_SY ? ((r == 0 && c == 1) ? GInt{-1, 0} : GInt{1, 0})
                      : ((r == 1 && c == 0) ? GInt{-1, 0} : GInt{1, 0});
}
// Entry (r, c) of ga' (x) gb' (ga on local bit 0, gb on local bit 1).
constexpr GInt pg_pair(int ga, int gb, int r, int c) {
    return gmul(pg_fac(ga, r & 1, c & 1), pg_fac(gb, r >> 1, c >> 1));
}
// True when every entry of ga' (x) gb' is twice a Gaussian integer (as for
// sqrt(X)' (x) sqrt(X)'); the pair is then applied with the entries halved and
// one factor 1/2 fewer in the scale counter.
constexpr bool pg_pair_even(int ga, int gb) {
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            const GInt v = pg_pair(ga, gb, r, c);
            if ((v.re & 1) || (v.im & 1)) return false;
        }
    return true;
}
// Powers of 1/sqrt(2) factored out of one unnormalised gate, and of w.
constexpr int pg_scale_pow(int g) { return (g == PG_SX || g == PG_SXDG) ? 2 : 1; }
constexpr int pg_phase8(int g) { return g == PG_SY ? 1 : g == PG_SYDG ? 7 : 0; }

enum OpType : uint32_t {
    OP_DENSE = 1,   // k <= 4 slots (mask in `mask`), matrix at `arg` (pool elements)
    OP_DIAGR = 2,   // diagonal on slots `mask`, 2^k entries at `arg`
    OP_PHASE8 = 3,  // quadratic 8th-root phase form `arg`
    OP_SIGN = 4,    // same with every exponent in {0, 4}
    OP_GRAD = 5,    // Im<lambda|G|psi> over slots `mask`, generator `k`, pass-local slot `arg`
    OP_SCALE = 6,   // multiply by the real scalar at pool element `arg` (.x)
    OP_BF = 11,     // twiddled butterfly, see below
    OP_D1T = 12,    // one-qubit 2x2 matrix at `arg` with a +-1 input sign, see below
    OP_PERM = 13,   // exact permutation on register slots, see below
};

// OP_PERM: X (k = 1) or Y (k = 2) on slot a, CNOT (k = 3, control a, target
// b) or SWAP (k = 4) of slots a and b; mask = a | b << 2.  Amplitudes move
// between registers (renamed away in the specialised kernels); Y also
// multiplies by +-i (a swap of real and imaginary parts and one sign).

// OP_BF on register slot S: for every pair (x, y) of amplitudes that differ
// only in slot S (y has the bit set),
//     x <- x + t y,   y <- x - t y,   t = w^M (-1)^(parity of the index bits in
// the partner set),  w = e^{i pi/4}.
// Encoding: k = M | S << 4 | RM << 8 | U << 12 (RM: partner register
// slots); mask = partner tile-local positions outside the registers; arg =
// index of a DPair whose m[0] holds the partner nonlocal qubits, or kNoPair.
// U = 1 (no partner outside the registers, mask = 0): arg is instead the pool
// offset of a sign table of 8 entries, one per register pair in increasing
// index order: entry p = (g_p, -2 g_p), g_p = the real factor of the
// twiddle (1 for even M, cos(pi/4) for odd M) with the sign of the pair's
// register partner parity.
constexpr uint32_t kNoPair = 0xffffffffu;
constexpr uint32_t kBfUniform = 1u << 12;

// OP_D1T on slot S: (x, y) <- (u00 x + s u01 y, u10 x + s u11 y) with u the
// 2x2 matrix at pool offset `arg` (the pending 8th-root phase of the qubit is
// already folded into its second column) and s = (-1)^(parity of the
// partner bits).  Encoding: k = S | RM << 2 | REAL << 6 | (pair + 1) << 7
// (REAL: u is real; pair: DPair index of the partner nonlocal qubits, 0 =
// none); mask = partner tile-local positions outside the registers.
// The pool entry continues with an in-place form of u = [[a, b], [c, e]]:
// arg+4 = r = c / a, arg+5 = d = e - r b, arg+6 = flag (.x != 0 when
// |a| >= |c| and the form is valid), and for REAL, arg+7..arg+14 = per
// register pair p (increasing index order) the signed (b_p, d_p) of the
// pair's register partner parity.
enum GradGen : uint32_t { GEN_X = 1, GEN_Y = 2, GEN_Z = 3, GEN_P11 = 4 };

struct DOp {
    uint32_t type;
    uint32_t k;      // arity (dense/diag) or generator (grad)
    uint32_t mask;   // register-slot bitmask (4 bits)
    uint32_t arg;
};

enum PhaseKind : uint32_t { PH_REG = 0 };

struct DPhase {
    uint32_t kind;
    uint32_t rpos;       // register positions in the tile-local index, 4 x 8 bits, ascending
    uint32_t op0, nop;
    uint16_t soff[kRegAmps];  // swizzled LDS offsets of the 16 slots (amplitude units)
};

// 8th-root phase form relative to one pass/phase (see kernels for the
// decomposition into tile, thread and register parts).
struct DForm {
    uint64_t mc[kMaxTileBits][3];   // per local bit a: nonlocal partner masks, bit c of beta
    uint64_t ka[3];                 // nonlocal linear terms, bit c of alpha
    uint32_t konst;                 // constant exponent
    uint32_t has_tile;              // 1 if any tile-dependent term exists
    uint32_t q0, nq;                // nonlocal pair list [q0, q0+nq) in the pass's pair table
    uint32_t etab;                  // offset of the per-thread-group table (uint16 entries)
    uint32_t a_lo, a_hi;            // register-slot table A[16], 3 bits each (48 bits)
    uint32_t lam_const[3];          // Lambda_c when has_tile == 0
    uint32_t slot;                  // index of this form among the pass's forms
    uint32_t abits;                 // bit i = bit 2 of A[i] (sign-only forms)
};

// Nonlocal-nonlocal pair entry: for nonlocal bit `b`, masks of nonlocal
// partners b' < b with bit c of beta(b, b') set.
struct DPair {
    uint64_t m[3];
    uint32_t b;
    uint32_t pad;
};

struct DPass {
    uint32_t L, H, T;
    uint32_t nphase, phase0;
    uint32_t nform, form0;
    uint32_t ngrad;
    uint64_t gpart_off;   // offset of this pass's gradient partials (doubles)
    uint32_t hpos[16];
};

}  // namespace svmi
