// Register-phase operations of a tile pass.  Each operates on the 16
// amplitudes a[0..15] that a thread holds in a register phase; bit s of the
// register index is register slot s.  Shared by the runtime interpreter and
// the plan-specialised kernels compiled with hiprtc.
#pragma once
#include "device_common.h"
#include "plan.h"

namespace svmi {

// Dense 2^k x 2^k block on the slots of MASK (k = popcount(MASK) <= 4); the
// matrix is row-major with local index bit t = the t-th lowest slot of MASK.
// Each matrix element is loaded once and applied to every index set.
template <class R, int MASK, class U>
__device__ __forceinline__ void op_dense(V2<R>* a, U u) {
    constexpr int K = __builtin_popcount(MASK);
    constexpr int D = 1 << K;
    V2<R> out[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = V2<R>{R(0), R(0)};
#pragma unroll
    for (int o = 0; o < D; ++o) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const V2<R> m = ldv(u + o * D + c);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if (r & MASK) continue;
                cmac(out[r | dep4(MASK, o)], m, a[r | dep4(MASK, c)]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = out[i];
}

// Diagonal on the slots of MASK: a[i] *= d[ext(MASK, i)].
template <class R, int MASK, class U>
__device__ __forceinline__ void op_diag(V2<R>* a, U d) {
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = cmul(ldv(d + ext4(MASK, i)), a[i]);
}

// Twiddled butterfly on slot S (OP_BF): for each pair (x, y), y the member
// with the slot bit set, x <- x + t y and y <- x - t y with
// t = k w^M (-1)^(parity of the register slots RM in the pair index),
// w = e^{i pi/4}.  k = +-1 is the thread's sign from partner bits outside the
// registers (RT) or 1.  w^M y = i^(M/2) y for even M and
// i^((M-1)/2) c (y.x - y.y, y.x + y.y) for odd M (c = cos(pi/4)), so an even
// twiddle costs 4 adds or FMAs per pair and an odd one 6.  The 1/sqrt(2) of
// every butterfly is applied once per pass (op_scale).
template <class R, int S, int M, int RM, bool RT>
__device__ __forceinline__ void op_bf(V2<R>* a, R s, R c) {
    constexpr int j = (M >> 1) & 3;
    constexpr bool odd = (M & 1) != 0;
    const R kk = odd ? (RT ? s * c : c) : (RT ? s : R(1));
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & (1 << S)) continue;
        const V2<R> x = a[i], y = a[i | (1 << S)];
        const bool neg = (__builtin_popcount(i & RM) & 1) != 0;
        R z0, z1;
        if constexpr (odd) {
            z0 = y.x - y.y;
            z1 = y.x + y.y;
        } else {
            z0 = y.x;
            z1 = y.y;
        }
        // t y = (g0 p0, g1 p1) with g = +-k
        R p0, p1;
        bool n0, n1;
        if constexpr (j == 0) { p0 = z0; p1 = z1; n0 = false; n1 = false; }
        else if constexpr (j == 1) { p0 = z1; p1 = z0; n0 = true; n1 = false; }
        else if constexpr (j == 2) { p0 = z0; p1 = z1; n0 = true; n1 = true; }
        else { p0 = z1; p1 = z0; n0 = false; n1 = true; }
        n0 = n0 != neg;
        n1 = n1 != neg;
        if constexpr (!odd && !RT) {
            const R q0 = n0 ? -p0 : p0, q1 = n1 ? -p1 : p1;
            a[i] = V2<R>{x.x + q0, x.y + q1};
            a[i | (1 << S)] = V2<R>{x.x - q0, x.y - q1};
        } else {
            const R g0 = n0 ? -kk : kk, g1 = n1 ? -kk : kk;
            a[i] = V2<R>{fma_(g0, p0, x.x), fma_(g1, p1, x.y)};
            a[i | (1 << S)] = V2<R>{fma_(-g0, p0, x.x), fma_(-g1, p1, x.y)};
        }
    }
}

// Interpreter form of op_bf: M is a template argument (the interpreter
// dispatches on it), the register partner mask RM is known at run time.
template <class R, int S, int M>
__device__ __forceinline__ void op_bf_rm(V2<R>* a, uint32_t RM, R s, R c) {
    constexpr int j = (M >> 1) & 3;
    constexpr bool odd = (M & 1) != 0;
    const R kk = odd ? s * c : s;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & (1 << S)) continue;
        const V2<R> x = a[i], y = a[i | (1 << S)];
        R z0, z1;
        if constexpr (odd) {
            z0 = y.x - y.y;
            z1 = y.x + y.y;
        } else {
            z0 = y.x;
            z1 = y.y;
        }
        R p0, p1;
        bool n0, n1;
        if constexpr (j == 0) { p0 = z0; p1 = z1; n0 = false; n1 = false; }
        else if constexpr (j == 1) { p0 = z1; p1 = z0; n0 = true; n1 = false; }
        else if constexpr (j == 2) { p0 = z0; p1 = z1; n0 = true; n1 = true; }
        else { p0 = z1; p1 = z0; n0 = false; n1 = true; }
        const R g = (__builtin_popcount((uint32_t)i & RM) & 1) ? -kk : kk;
        const R g0 = n0 ? -g : g, g1 = n1 ? -g : g;
        a[i] = V2<R>{fma_(g0, p0, x.x), fma_(g1, p1, x.y)};
        a[i | (1 << S)] = V2<R>{fma_(-g0, p0, x.x), fma_(-g1, p1, x.y)};
    }
}

// v with its sign flipped when the wave-uniform bit f is set, computed on
// the scalar unit so that the result is an SGPR operand.
__device__ __forceinline__ float uneg(float v, uint32_t f) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v) ^ (int)(f << 31)));
}
__device__ __forceinline__ double uneg(double v, uint32_t f) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32) ^ (int)(f << 31));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sign pattern of a register partner mask: bit i = parity of (i & RM).
__device__ __forceinline__ uint32_t rm_pattern(uint32_t RM) {
    return ((RM & 1u) ? 0xAAAAu : 0u) ^ ((RM & 2u) ? 0xCCCCu : 0u) ^ ((RM & 4u) ? 0xF0F0u : 0u) ^
           ((RM & 8u) ? 0xFF00u : 0u);
}

// Register pair number of index i (bit S clear): i with bit S removed.
template <int S>
__device__ constexpr int pair_no(int i) {
    return (i & ((1 << S) - 1)) | ((i >> (S + 1)) << S);
}

// Interpreter form of op_bf when no partner lies outside the registers
// (OP_BF with kBfUniform): the signed twiddle factors of the 8 pairs come
// from the pool table t (entry p = (g_p, -2 g_p)) as scalar operands.  The
// outputs overwrite the inputs: x' = x + t y first, then y' = x' - 2 t y, so
// x and y end their lives at their last use and the op needs no register
// copies (y' is rounded from x' rather than from x).
template <class R, int S, int M, class U>
__device__ __forceinline__ void op_bf_t(V2<R>* a, U t) {
    constexpr int j = (M >> 1) & 3;
    constexpr bool odd = (M & 1) != 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & (1 << S)) continue;
        const V2<R> x = a[i], y = a[i | (1 << S)];
        R z0, z1;
        if constexpr (odd) {
            z0 = y.x - y.y;
            z1 = y.x + y.y;
        } else {
            z0 = y.x;
            z1 = y.y;
        }
        R p0, p1;
        bool n0, n1;
        if constexpr (j == 0) { p0 = z0; p1 = z1; n0 = false; n1 = false; }
        else if constexpr (j == 1) { p0 = z1; p1 = z0; n0 = true; n1 = false; }
        else if constexpr (j == 2) { p0 = z0; p1 = z1; n0 = true; n1 = true; }
        else { p0 = z1; p1 = z0; n0 = false; n1 = true; }
        const V2<R> gh = ldv(t + pair_no<S>(i));
        const R g0 = n0 ? -gh.x : gh.x, g1 = n1 ? -gh.x : gh.x;
        const R h0 = n0 ? -gh.y : gh.y, h1 = n1 ? -gh.y : gh.y;
        const R x0 = fma_(g0, p0, x.x), x1 = fma_(g1, p1, x.y);
        a[i] = V2<R>{x0, x1};
        a[i | (1 << S)] = V2<R>{fma_(h0, p0, x0), fma_(h1, p1, x1)};
    }
}

// One-qubit matrix u (row-major 2x2 at u, the qubit's pending phase already
// in its second column) on slot S with the input sign of y
// s * (-1)^(parity of the register slots RM in the pair index) (OP_D1T).
// REAL: u is real (8 multiply-adds per pair instead of 16).
template <class R, int S, int RM, bool RT, bool REAL>
__device__ __forceinline__ void op_d1t(V2<R>* a, const V2<R>* __restrict__ u, R s) {
    const V2<R> u00 = u[0], u10 = u[2];
    V2<R> u01 = u[1], u11 = u[3];
    if constexpr (RT) {
        u01 = V2<R>{s * u01.x, s * u01.y};
        u11 = V2<R>{s * u11.x, s * u11.y};
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & (1 << S)) continue;
        const V2<R> x = a[i], y = a[i | (1 << S)];
        const bool neg = (__builtin_popcount(i & RM) & 1) != 0;
        const R c01x = neg ? -u01.x : u01.x, c01y = neg ? -u01.y : u01.y;
        const R c11x = neg ? -u11.x : u11.x, c11y = neg ? -u11.y : u11.y;
        V2<R> o0, o1;
        if constexpr (REAL) {
            o0 = V2<R>{fma_(c01x, y.x, u00.x * x.x), fma_(c01x, y.y, u00.x * x.y)};
            o1 = V2<R>{fma_(c11x, y.x, u10.x * x.x), fma_(c11x, y.y, u10.x * x.y)};
        } else {
            o0 = cmul(u00, x);
            o1 = cmul(u10, x);
            cmac(o0, V2<R>{c01x, c01y}, y);
            cmac(o1, V2<R>{c11x, c11y}, y);
        }
        a[i] = o0;
        a[i | (1 << S)] = o1;
    }
}

// Interpreter form of op_d1t: the register partner mask RM at run time.
template <class R, int S, bool REAL, class U>
__device__ __forceinline__ void op_d1t_rm(V2<R>* a, U u, uint32_t RM, R s) {
    const V2<R> u00 = ldv(u), u10 = ldv(u + 2);
    const V2<R> u01{s * u[1].x, s * u[1].y}, u11{s * u[3].x, s * u[3].y};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & (1 << S)) continue;
        const V2<R> x = a[i], y0 = a[i | (1 << S)];
        const bool neg = (__builtin_popcount((uint32_t)i & RM) & 1) != 0;
        const V2<R> y = neg ? V2<R>{-y0.x, -y0.y} : y0;
        V2<R> o0, o1;
        if constexpr (REAL) {
            o0 = V2<R>{fma_(u01.x, y.x, u00.x * x.x), fma_(u01.x, y.y, u00.x * x.y)};
            o1 = V2<R>{fma_(u11.x, y.x, u10.x * x.x), fma_(u11.x, y.y, u10.x * x.y)};
        } else {
            o0 = cmul(u00, x);
            o1 = cmul(u10, x);
            cmac(o0, u01, y);
            cmac(o1, u11, y);
        }
        a[i] = o0;
        a[i | (1 << S)] = o1;
    }
}

// Real one-qubit matrix in the in-place form with the signed (b_p, d_p) of
// each register pair read from the pool (entries 7..14) as scalar operands.
template <class R, int S, class U>
__device__ __forceinline__ void op_d1t_t(V2<R>* a, U u) {
    const R u00 = u[0].x, r = u[4].x;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & (1 << S)) continue;
        const V2<R> x = a[i], y = a[i | (1 << S)];
        const V2<R> be = ldv(u + 7 + pair_no<S>(i));
        const V2<R> o0{fma_(be.x, y.x, u00 * x.x), fma_(be.x, y.y, u00 * x.y)};
        a[i] = o0;
        a[i | (1 << S)] = V2<R>{fma_(r, o0.x, be.y * y.x), fma_(r, o0.y, be.y * y.y)};
    }
}

// Interpreter form of op_d1t when every lane has the same input signs, with
// the outputs written over the inputs: u = [[a, b], [c, e]] is applied as
// o0 = a x + b' y, then o1 = r o0 + d' y with r = c / a and d = e - r b
// (u[4], u[5]; b' and d' carry the pair's partner sign), so that x and y end
// their lives at their last use and the op needs no register copies.  The
// planner stores this form only when |a| >= |c|.
template <class R, int S, bool REAL, class U>
__device__ __forceinline__ void op_d1t_u(V2<R>* a, U u, uint32_t pm) {
    const V2<R> u00 = ldv(u), u01 = ldv(u + 1), r = ldv(u + 4), d = ldv(u + 5);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & (1 << S)) continue;
        const V2<R> x = a[i], y = a[i | (1 << S)];
        const uint32_t neg = (pm >> i) & 1u;
        V2<R> o0, o1;
        if constexpr (REAL) {
            const R b = uneg(u01.x, neg), e = uneg(d.x, neg);
            o0 = V2<R>{fma_(b, y.x, u00.x * x.x), fma_(b, y.y, u00.x * x.y)};
            o1 = V2<R>{fma_(r.x, o0.x, e * y.x), fma_(r.x, o0.y, e * y.y)};
        } else {
            const V2<R> b{uneg(u01.x, neg), uneg(u01.y, neg)}, e{uneg(d.x, neg), uneg(d.y, neg)};
            o0 = cmul(u00, x);
            cmac(o0, b, y);
            o1 = cmul(e, y);
            cmac(o1, r, o0);
        }
        a[i] = o0;
        a[i | (1 << S)] = o1;
    }
}

// True when a pool flag entry is set (its bits are not all zero).
__device__ __forceinline__ bool uflag(float v) { return __float_as_uint(v) != 0u; }
__device__ __forceinline__ bool uflag(double v) { return __double_as_longlong(v) != 0ll; }

// Thread sign of a butterfly: (-1)^(parity of the partner bits of the
// thread's tile-local index lb and of the tile's global base).
__device__ __forceinline__ uint32_t bf_parity(uint32_t lb, uint32_t lmask, uint64_t base, uint64_t gmask) {
    return (uint32_t)(__popc(lb & lmask) + __popcll(base & gmask)) & 1u;
}

template <class R>
__device__ __forceinline__ void op_scale(V2<R>* a, R s) {
#pragma unroll
    for (int i = 0; i < 16; ++i) { a[i].x *= s; a[i].y *= s; }
}

// ---- 8th-root phase forms (Sec. 4.3) --------------------------------------
// Exponent of register amplitude i: e0 + sum_{s in i} d[s] + A_i (mod 8),
// where e0 and d[] are per thread and A (3 bits per i) is uniform.

// Per-thread parts from the per-tile masks (fl: Lambda_0..2 and K in LDS) and
// the per-thread-group table entry et (3 bits Etau, then 3 bits per slot).
__device__ __forceinline__ void form_thread(const uint32_t* fl, uint32_t et, uint32_t lb, uint32_t r0, uint32_t r1,
                                            uint32_t r2, uint32_t r3, uint32_t& e0, uint32_t d[4]) {
    const uint32_t L0 = fl[0], L1 = fl[1], L2 = fl[2], K = fl[3];
    e0 = K + (et & 7u) + __popc(lb & L0) + 2u * __popc(lb & L1) + 4u * __popc(lb & L2);
    const uint32_t rr[4] = {r0, r1, r2, r3};
#pragma unroll
    for (int s = 0; s < 4; ++s)
        d[s] = ((et >> (3 + 3 * s)) & 7u) + ((L0 >> rr[s]) & 1u) + 2u * ((L1 >> rr[s]) & 1u) +
               4u * ((L2 >> rr[s]) & 1u);
}

// Sign-only form: every exponent is 0 or 4, so the sign bit of amplitude i is
// the XOR of the bit-2's of its terms; build a 16-bit flip mask per thread.
template <class R, bool TWO>
__device__ __forceinline__ void op_sign(V2<R>* a, V2<R>* l, uint32_t e0, const uint32_t d[4], uint32_t abits) {
    uint32_t m = abits;
    m ^= ((e0 >> 2) & 1u) ? 0xFFFFu : 0u;
    m ^= ((d[0] >> 2) & 1u) ? 0xAAAAu : 0u;
    m ^= ((d[1] >> 2) & 1u) ? 0xCCCCu : 0u;
    m ^= ((d[2] >> 2) & 1u) ? 0xF0F0u : 0u;
    m ^= ((d[3] >> 2) & 1u) ? 0xFF00u : 0u;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t f = (m << (31 - i)) & 0x80000000u;
        sign_flip_mask(a[i], f);
        if constexpr (TWO) sign_flip_mask(l[i], f);
    }
}

// General form: multiply amplitude i by e^{i pi e_i / 4} from the LDS table.
template <class R, bool TWO>
__device__ __forceinline__ void op_phase8(V2<R>* a, V2<R>* l, uint32_t e0, const uint32_t d[4], uint64_t At,
                                          const V2<R>* ptab) {
    uint32_t e[16];
    e[0] = e0;
#pragma unroll
    for (int i = 1; i < 16; ++i) e[i] = e[i & (i - 1)] + d[__builtin_ctz(i)];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t ee = (e[i] + (uint32_t)(At >> (3 * i))) & 7u;
        const V2<R> t = ptab[ee];
        a[i] = cmul(t, a[i]);
        if constexpr (TWO) l[i] = cmul(t, l[i]);
    }
}

// ---- adjoint gradient terms -----------------------------------------------
// Im <lambda|G|psi> over the 16 register amplitudes, G = X, Y or Z on slot
// S.  The thread's products are accumulated with fused multiply-adds in the
// state's precision (two chains); the frame sums these partials over the
// wave in the same precision, and the wave sums over the state in FP64.
template <class R, int S, uint32_t GEN>
__device__ __forceinline__ R op_grad1(const V2<R>* p, const V2<R>* l) {
    R acc[2] = {R(0), R(0)};
    int c = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & (1 << S)) continue;
        const int j = i | (1 << S);
        const V2<R> p0 = p[i], p1 = p[j], l0 = l[i], l1 = l[j];
        R& a = acc[c++ & 1];
        if constexpr (GEN == GEN_X) {
            // Im(conj(l0) p1) + Im(conj(l1) p0)
            a = fma_(l0.x, p1.y, a); a = fma_(-l0.y, p1.x, a);
            a = fma_(l1.x, p0.y, a); a = fma_(-l1.y, p0.x, a);
        } else if constexpr (GEN == GEN_Y) {
            // (Y psi)_0 = -i psi_1, (Y psi)_1 = i psi_0: Re(conj(l1) p0) - Re(conj(l0) p1)
            a = fma_(l1.x, p0.x, a); a = fma_(l1.y, p0.y, a);
            a = fma_(-l0.x, p1.x, a); a = fma_(-l0.y, p1.y, a);
        } else {
            // Im(conj(l0) p0) - Im(conj(l1) p1)
            a = fma_(l0.x, p0.y, a); a = fma_(-l0.y, p0.x, a);
            a = fma_(-l1.x, p1.y, a); a = fma_(l1.y, p1.x, a);
        }
    }
    return acc[0] + acc[1];
}

// Generator -2 |11><11| on the two slots of MASK (controlled phase).
template <class R, int MASK>
__device__ __forceinline__ R op_grad11(const V2<R>* p, const V2<R>* l) {
    R acc = R(0);
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if ((i & MASK) == MASK) {
            acc = fma_(l[i].x, p[i].y, acc);
            acc = fma_(-l[i].y, p[i].x, acc);
        }
    return R(-2) * acc;
}

// Exact permutation on register slots (OP_PERM): KIND 1 = X on slot SA,
// 2 = Y on slot SA, 3 = CNOT (control SA, target SB), 4 = SWAP(SA, SB).
template <class R, int KIND, int SA, int SB>
__device__ __forceinline__ void op_perm(V2<R>* a) {
    constexpr uint32_t ma = 1u << SA, mb = 1u << SB;
#pragma unroll
    for (uint32_t i = 0; i < 16; ++i) {
        if constexpr (KIND == 1) {
            if (!(i & ma)) {
                const V2<R> x = a[i];
                a[i] = a[i | ma];
                a[i | ma] = x;
            }
        } else if constexpr (KIND == 2) {
            if (!(i & ma)) {   // (x, y) <- (-i y, i x)
                const V2<R> x = a[i], y = a[i | ma];
                a[i] = V2<R>{y.y, -y.x};
                a[i | ma] = V2<R>{-x.y, x.x};
            }
        } else if constexpr (KIND == 3) {
            if ((i & ma) && !(i & mb)) {
                const V2<R> x = a[i];
                a[i] = a[i | mb];
                a[i | mb] = x;
            }
        } else {
            if ((i & ma) && !(i & mb)) {
                const uint32_t j = i ^ ma ^ mb;
                const V2<R> x = a[i];
                a[i] = a[j];
                a[j] = x;
            }
        }
    }
}

}  // namespace svmi
