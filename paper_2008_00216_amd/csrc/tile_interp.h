// Runtime-interpreted tile pass body: the op list of every register phase is
// read from the plan and dispatched on its type and slot mask.  Used by the
// single-circuit tile kernel and by the persistent batched kernel.
#pragma once
#include "device_common.h"
#include "plan.h"
#include "tile_frame.h"
#include "tile_ops.h"

namespace svmi {

namespace {

template <class R>
__device__ __forceinline__ void dense_dispatch(V2<R>* a, uint32_t mask, cptr_t<V2<R>> u) {
    switch (mask) {
        case 1: op_dense<R, 1>(a, u); break;
        case 2: op_dense<R, 2>(a, u); break;
        case 3: op_dense<R, 3>(a, u); break;
        case 4: op_dense<R, 4>(a, u); break;
        case 5: op_dense<R, 5>(a, u); break;
        case 6: op_dense<R, 6>(a, u); break;
        case 7: op_dense<R, 7>(a, u); break;
        case 8: op_dense<R, 8>(a, u); break;
        case 9: op_dense<R, 9>(a, u); break;
        case 10: op_dense<R, 10>(a, u); break;
        case 11: op_dense<R, 11>(a, u); break;
        case 12: op_dense<R, 12>(a, u); break;
        case 13: op_dense<R, 13>(a, u); break;
        case 14: op_dense<R, 14>(a, u); break;
        case 15: op_dense<R, 15>(a, u); break;
        default: break;
    }
}

template <class R>
__device__ __forceinline__ void diag_dispatch(V2<R>* a, uint32_t mask, cptr_t<V2<R>> d) {
    switch (mask) {
        case 1: op_diag<R, 1>(a, d); break;
        case 2: op_diag<R, 2>(a, d); break;
        case 3: op_diag<R, 3>(a, d); break;
        case 4: op_diag<R, 4>(a, d); break;
        case 5: op_diag<R, 5>(a, d); break;
        case 6: op_diag<R, 6>(a, d); break;
        case 7: op_diag<R, 7>(a, d); break;
        case 8: op_diag<R, 8>(a, d); break;
        case 9: op_diag<R, 9>(a, d); break;
        case 10: op_diag<R, 10>(a, d); break;
        case 11: op_diag<R, 11>(a, d); break;
        case 12: op_diag<R, 12>(a, d); break;
        case 13: op_diag<R, 13>(a, d); break;
        case 14: op_diag<R, 14>(a, d); break;
        case 15: op_diag<R, 15>(a, d); break;
        default: break;
    }
}

#define SVMI_BF_CASE(S, M) \
    case (S) * 8 + (M): op_bf_rm<R, S, M>(a, RM, s, c); break;

template <class R>
__device__ __forceinline__ void bf_dispatch(V2<R>* a, uint32_t slot, uint32_t M, uint32_t RM, R s, R c) {
    switch (slot * 8 + M) {
        SVMI_BF_CASE(0, 0) SVMI_BF_CASE(0, 1) SVMI_BF_CASE(0, 2) SVMI_BF_CASE(0, 3)
        SVMI_BF_CASE(0, 4) SVMI_BF_CASE(0, 5) SVMI_BF_CASE(0, 6) SVMI_BF_CASE(0, 7)
        SVMI_BF_CASE(1, 0) SVMI_BF_CASE(1, 1) SVMI_BF_CASE(1, 2) SVMI_BF_CASE(1, 3)
        SVMI_BF_CASE(1, 4) SVMI_BF_CASE(1, 5) SVMI_BF_CASE(1, 6) SVMI_BF_CASE(1, 7)
        SVMI_BF_CASE(2, 0) SVMI_BF_CASE(2, 1) SVMI_BF_CASE(2, 2) SVMI_BF_CASE(2, 3)
        SVMI_BF_CASE(2, 4) SVMI_BF_CASE(2, 5) SVMI_BF_CASE(2, 6) SVMI_BF_CASE(2, 7)
        SVMI_BF_CASE(3, 0) SVMI_BF_CASE(3, 1) SVMI_BF_CASE(3, 2) SVMI_BF_CASE(3, 3)
        SVMI_BF_CASE(3, 4) SVMI_BF_CASE(3, 5) SVMI_BF_CASE(3, 6) SVMI_BF_CASE(3, 7)
        default: break;
    }
}
#undef SVMI_BF_CASE

#define SVMI_BFT_CASE(S, M) \
    case (S) * 8 + (M): op_bf_t<R, S, M>(a, t); break;

template <class R>
__device__ __forceinline__ void bf_dispatch_t(V2<R>* a, uint32_t slot, uint32_t M, cptr_t<V2<R>> t) {
    switch (slot * 8 + M) {
        SVMI_BFT_CASE(0, 0) SVMI_BFT_CASE(0, 1) SVMI_BFT_CASE(0, 2) SVMI_BFT_CASE(0, 3)
        SVMI_BFT_CASE(0, 4) SVMI_BFT_CASE(0, 5) SVMI_BFT_CASE(0, 6) SVMI_BFT_CASE(0, 7)
        SVMI_BFT_CASE(1, 0) SVMI_BFT_CASE(1, 1) SVMI_BFT_CASE(1, 2) SVMI_BFT_CASE(1, 3)
        SVMI_BFT_CASE(1, 4) SVMI_BFT_CASE(1, 5) SVMI_BFT_CASE(1, 6) SVMI_BFT_CASE(1, 7)
        SVMI_BFT_CASE(2, 0) SVMI_BFT_CASE(2, 1) SVMI_BFT_CASE(2, 2) SVMI_BFT_CASE(2, 3)
        SVMI_BFT_CASE(2, 4) SVMI_BFT_CASE(2, 5) SVMI_BFT_CASE(2, 6) SVMI_BFT_CASE(2, 7)
        SVMI_BFT_CASE(3, 0) SVMI_BFT_CASE(3, 1) SVMI_BFT_CASE(3, 2) SVMI_BFT_CASE(3, 3)
        SVMI_BFT_CASE(3, 4) SVMI_BFT_CASE(3, 5) SVMI_BFT_CASE(3, 6) SVMI_BFT_CASE(3, 7)
        default: break;
    }
}
#undef SVMI_BFT_CASE

template <class R>
__device__ __forceinline__ void d1t_dispatch(V2<R>* a, uint32_t slot, bool real, cptr_t<V2<R>> u, uint32_t RM, R s) {
    switch (slot * 2 + (real ? 1u : 0u)) {
        case 0: op_d1t_rm<R, 0, false>(a, u, RM, s); break;
        case 1: op_d1t_rm<R, 0, true>(a, u, RM, s); break;
        case 2: op_d1t_rm<R, 1, false>(a, u, RM, s); break;
        case 3: op_d1t_rm<R, 1, true>(a, u, RM, s); break;
        case 4: op_d1t_rm<R, 2, false>(a, u, RM, s); break;
        case 5: op_d1t_rm<R, 2, true>(a, u, RM, s); break;
        case 6: op_d1t_rm<R, 3, false>(a, u, RM, s); break;
        case 7: op_d1t_rm<R, 3, true>(a, u, RM, s); break;
        default: break;
    }
}

template <class R>
__device__ __forceinline__ void d1t_dispatch_t(V2<R>* a, uint32_t slot, cptr_t<V2<R>> u) {
    switch (slot) {
        case 0: op_d1t_t<R, 0>(a, u); break;
        case 1: op_d1t_t<R, 1>(a, u); break;
        case 2: op_d1t_t<R, 2>(a, u); break;
        case 3: op_d1t_t<R, 3>(a, u); break;
        default: break;
    }
}

template <class R>
__device__ __forceinline__ void d1t_dispatch_u(V2<R>* a, uint32_t slot, cptr_t<V2<R>> u, uint32_t pm) {
    switch (slot) {
        case 0: op_d1t_u<R, 0, false>(a, u, pm); break;
        case 1: op_d1t_u<R, 1, false>(a, u, pm); break;
        case 2: op_d1t_u<R, 2, false>(a, u, pm); break;
        case 3: op_d1t_u<R, 3, false>(a, u, pm); break;
        default: break;
    }
}

template <class R, uint32_t GEN>
__device__ __forceinline__ R grad1_dispatch(const V2<R>* p, const V2<R>* l, uint32_t mask) {
    switch (mask) {
        case 1: return op_grad1<R, 0, GEN>(p, l);
        case 2: return op_grad1<R, 1, GEN>(p, l);
        case 4: return op_grad1<R, 2, GEN>(p, l);
        case 8: return op_grad1<R, 3, GEN>(p, l);
        default: return R(0);
    }
}

template <class R>
__device__ __forceinline__ R grad_dispatch(const V2<R>* p, const V2<R>* l, uint32_t gen, uint32_t mask) {
    switch (gen) {
        case GEN_X: return grad1_dispatch<R, GEN_X>(p, l, mask);
        case GEN_Y: return grad1_dispatch<R, GEN_Y>(p, l, mask);
        case GEN_Z: return grad1_dispatch<R, GEN_Z>(p, l, mask);
        default: break;
    }
    switch (mask) {
        case 3: return op_grad11<R, 3>(p, l);
        case 5: return op_grad11<R, 5>(p, l);
        case 6: return op_grad11<R, 6>(p, l);
        case 9: return op_grad11<R, 9>(p, l);
        case 10: return op_grad11<R, 10>(p, l);
        case 12: return op_grad11<R, 12>(p, l);
        default: return R(0);
    }
}

#define SVMI_PERM1(K, S) \
    case (K) * 16 + (S) * 4 + (S): op_perm<R, K, S, S>(a); break;
#define SVMI_PERM2(K, A, B) \
    case (K) * 16 + (A) * 4 + (B): op_perm<R, K, A, B>(a); break;

template <class R>
__device__ __forceinline__ void perm_dispatch(V2<R>* a, uint32_t kind, uint32_t mask) {
    const uint32_t sa = mask & 3u, sb = (mask >> 2) & 3u;
    switch (kind * 16 + sa * 4 + (kind <= 2 ? sa : sb)) {
        SVMI_PERM1(1, 0) SVMI_PERM1(1, 1) SVMI_PERM1(1, 2) SVMI_PERM1(1, 3)
        SVMI_PERM1(2, 0) SVMI_PERM1(2, 1) SVMI_PERM1(2, 2) SVMI_PERM1(2, 3)
        SVMI_PERM2(3, 0, 1) SVMI_PERM2(3, 0, 2) SVMI_PERM2(3, 0, 3) SVMI_PERM2(3, 1, 0)
        SVMI_PERM2(3, 1, 2) SVMI_PERM2(3, 1, 3) SVMI_PERM2(3, 2, 0) SVMI_PERM2(3, 2, 1)
        SVMI_PERM2(3, 2, 3) SVMI_PERM2(3, 3, 0) SVMI_PERM2(3, 3, 1) SVMI_PERM2(3, 3, 2)
        SVMI_PERM2(4, 0, 1) SVMI_PERM2(4, 0, 2) SVMI_PERM2(4, 0, 3) SVMI_PERM2(4, 1, 0)
        SVMI_PERM2(4, 1, 2) SVMI_PERM2(4, 1, 3) SVMI_PERM2(4, 2, 0) SVMI_PERM2(4, 2, 1)
        SVMI_PERM2(4, 2, 3) SVMI_PERM2(4, 3, 0) SVMI_PERM2(4, 3, 1) SVMI_PERM2(4, 3, 2)
        default: break;
    }
}
#undef SVMI_PERM1
#undef SVMI_PERM2

__device__ __forceinline__ DOp ld_op(cptr_t<DOp> p) {
    return DOp{p->type, p->k, p->mask, p->arg};
}

// Fixed registers for the amplitudes of the two states (complex64) at the head
// of every op iteration.  Without them the compiler homes the loop-carried
// amplitudes where the dense ops leave them, and every op that only reads
// them (the gradient terms) pays two moves of all 64 registers per iteration.
#define SVMI_PIN4(V0, V1, V2_, V3, x0, x1, x2, x3) \
    "+{v" #V0 "}"(x0), "+{v" #V1 "}"(x1), "+{v" #V2_ "}"(x2), "+{v" #V3 "}"(x3)
template <class R>
__device__ __forceinline__ void pin_pair(V2<R>*, V2<R>*) {}
template <>
__device__ __forceinline__ void pin_pair<float>(V2<float>* a, V2<float>* l) {
    asm volatile("" : SVMI_PIN4(64, 65, 66, 67, a[0].x, a[0].y, a[1].x, a[1].y),
                      SVMI_PIN4(68, 69, 70, 71, a[2].x, a[2].y, a[3].x, a[3].y),
                      SVMI_PIN4(72, 73, 74, 75, a[4].x, a[4].y, a[5].x, a[5].y),
                      SVMI_PIN4(76, 77, 78, 79, a[6].x, a[6].y, a[7].x, a[7].y));
    asm volatile("" : SVMI_PIN4(80, 81, 82, 83, a[8].x, a[8].y, a[9].x, a[9].y),
                      SVMI_PIN4(84, 85, 86, 87, a[10].x, a[10].y, a[11].x, a[11].y),
                      SVMI_PIN4(88, 89, 90, 91, a[12].x, a[12].y, a[13].x, a[13].y),
                      SVMI_PIN4(92, 93, 94, 95, a[14].x, a[14].y, a[15].x, a[15].y));
    asm volatile("" : SVMI_PIN4(96, 97, 98, 99, l[0].x, l[0].y, l[1].x, l[1].y),
                      SVMI_PIN4(100, 101, 102, 103, l[2].x, l[2].y, l[3].x, l[3].y),
                      SVMI_PIN4(104, 105, 106, 107, l[4].x, l[4].y, l[5].x, l[5].y),
                      SVMI_PIN4(108, 109, 110, 111, l[6].x, l[6].y, l[7].x, l[7].y));
    asm volatile("" : SVMI_PIN4(112, 113, 114, 115, l[8].x, l[8].y, l[9].x, l[9].y),
                      SVMI_PIN4(116, 117, 118, 119, l[10].x, l[10].y, l[11].x, l[11].y),
                      SVMI_PIN4(120, 121, 122, 123, l[12].x, l[12].y, l[13].x, l[13].y),
                      SVMI_PIN4(124, 125, 126, 127, l[14].x, l[14].y, l[15].x, l[15].y));
}
#undef SVMI_PIN4

}  // namespace

// Interpreter body of one tile of one pass (blk = state * tiles + tile).
template <class R, int NT, bool TWO, bool STREAM = true>
__device__ __forceinline__ void tile_interp(const TileArgs& A, unsigned char* smem, uint64_t blk) {
    using V = V2<R>;
    const cptr_t<DPass> P = cptr(A.pass);
    const cptr_t<uint32_t> hpos = cptr(A.pass->hpos);
    // pass fields are block-uniform; readfirstlane keeps every loop that
    // contains a barrier on a scalar exit condition
    const uint32_t L = rfl(P->L), H = rfl(P->H);
    TileFrame<R, NT, TWO, STREAM> F;
    F.begin_at(A, smem, L, H, rfl(P->T), hpos, rfl(P->nform), rfl(P->form0), rfl(P->ngrad), blk);
    const uint32_t tid = F.tid;
    const uint32_t ngroups = F.NA >> kRegBits;
    const uint32_t iters = (ngroups + NT - 1) / NT;
    const uint32_t nphase = rfl(P->nphase);
    // phase records, op descriptors, pair masks and matrices are wave-uniform
    // and read through scalar loads
    const cptr_t<DPhase> phs = cptr(A.phases) + rfl(P->phase0);
    const cptr_t<DOp> ops = cptr(A.ops);
    const cptr_t<DPair> prs = cptr(A.pairs);
    const cptr_t<V> pool = cptr(F.pool);
    for (uint32_t ph = 0; ph < nphase; ++ph) {
        const uint32_t rpos = phs[ph].rpos;
        const uint32_t r0 = rpos & 255u, r1 = (rpos >> 8) & 255u, r2 = (rpos >> 16) & 255u, r3 = rpos >> 24;
        uint32_t soff[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) soff[i] = phs[ph].soff[i];
        const uint32_t op0 = phs[ph].op0, nop = phs[ph].nop;
        for (uint32_t it = 0; it < iters; ++it) {
            const uint32_t gg = it * NT + tid;
            const bool act = gg < ngroups;
            const uint32_t lb = ins0(ins0(ins0(ins0(gg, r0), r1), r2), r3);
            const uint32_t sb = swz<R>(lb);
            V a[16];
            V l[16];
            F.load_group(sb, soff, a, l, act);
            // op descriptors are fetched one op ahead so that their load
            // overlaps the arithmetic of the current op
            DOp nxt{0u, 0u, 0u, 0u};
            if (nop) nxt = ld_op(ops + op0);
            for (uint32_t o = op0; o < op0 + nop; ++o) {
                const DOp op = nxt;
                if (o + 1 < op0 + nop) nxt = ld_op(ops + o + 1);
                if constexpr (TWO) pin_pair<R>(a, l);
                const uint32_t type = rfl(op.type), mask = rfl(op.mask), arg = rfl(op.arg);
                switch (type) {
                    case OP_DENSE:
                        dense_dispatch<R>(a, mask, pool + arg);
                        if constexpr (TWO) dense_dispatch<R>(l, mask, pool + arg);
                        break;
                    case OP_DIAGR:
                        diag_dispatch<R>(a, mask, pool + arg);
                        if constexpr (TWO) diag_dispatch<R>(l, mask, pool + arg);
                        break;
                    case OP_BF: {
                        const uint32_t kk = rfl(op.k);
                        if (kk & kBfUniform) {
                            // every lane has the same twiddles: sign table at arg
                            bf_dispatch_t<R>(a, (kk >> 4) & 3u, kk & 7u, pool + arg);
                            if constexpr (TWO) bf_dispatch_t<R>(l, (kk >> 4) & 3u, kk & 7u, pool + arg);
                            break;
                        }
                        const uint64_t gm = arg == kNoPair ? 0ull : prs[arg].m[0];
                        const R sg = bf_parity(lb, mask, F.base, gm) ? R(-1) : R(1);
                        const R cw = kSqrtHalf<R>;
                        bf_dispatch<R>(a, (kk >> 4) & 3u, kk & 7u, (kk >> 8) & 15u, sg, cw);
                        if constexpr (TWO) bf_dispatch<R>(l, (kk >> 4) & 3u, kk & 7u, (kk >> 8) & 15u, sg, cw);
                        break;
                    }
                    case OP_D1T: {
                        const uint32_t kk = rfl(op.k);
                        const uint32_t pk = kk >> 7;
                        if (mask == 0u && pk == 0u && uflag(pool[arg + 6].x)) {
                            // same input signs in every lane, in-place form stored
                            if ((kk >> 6) & 1u) {
                                d1t_dispatch_t<R>(a, kk & 3u, pool + arg);
                                if constexpr (TWO) d1t_dispatch_t<R>(l, kk & 3u, pool + arg);
                            } else {
                                const uint32_t pm = rm_pattern((kk >> 2) & 15u);
                                d1t_dispatch_u<R>(a, kk & 3u, pool + arg, pm);
                                if constexpr (TWO) d1t_dispatch_u<R>(l, kk & 3u, pool + arg, pm);
                            }
                            break;
                        }
                        const uint64_t gm = pk == 0 ? 0ull : prs[pk - 1].m[0];
                        const R sg = bf_parity(lb, mask, F.base, gm) ? R(-1) : R(1);
                        const bool real = ((kk >> 6) & 1u) != 0;
                        d1t_dispatch<R>(a, kk & 3u, real, pool + arg, (kk >> 2) & 15u, sg);
                        if constexpr (TWO) d1t_dispatch<R>(l, kk & 3u, real, pool + arg, (kk >> 2) & 15u, sg);
                        break;
                    }
                    case OP_PERM:
                        perm_dispatch<R>(a, rfl(op.k), mask);
                        if constexpr (TWO) perm_dispatch<R>(l, rfl(op.k), mask);
                        break;
                    case OP_SCALE: {
                        const R s = pool[arg].x;
                        op_scale<R>(a, s);
                        if constexpr (TWO) op_scale<R>(l, s);
                        break;
                    }
                    case OP_PHASE8:
                    case OP_SIGN: {
                        const cptr_t<DForm> Fm = cptr(A.forms) + arg;
                        const uint32_t et = act ? (uint32_t)A.etab[Fm->etab + gg] : 0u;
                        uint32_t e0, d[4];
                        form_thread(F.fl + 4 * Fm->slot, et, lb, r0, r1, r2, r3, e0, d);
                        if (type == OP_SIGN) {
                            op_sign<R, TWO>(a, l, e0, d, Fm->abits);
                        } else {
                            const uint64_t At = (uint64_t)Fm->a_lo | ((uint64_t)Fm->a_hi << 32);
                            op_phase8<R, TWO>(a, l, e0, d, At, F.ptab);
                        }
                        break;
                    }
                    case OP_GRAD:
                        if constexpr (TWO) F.grad_add(arg, grad_dispatch<R>(a, l, rfl(op.k), mask));
                        break;
                    default:
                        break;
                }
            }
            F.store_group(sb, soff, a, l, act);
        }
        __syncthreads();
    }
    F.end(A, L, H, hpos);
}

}  // namespace svmi
