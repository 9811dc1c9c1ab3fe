// Fused tile pass: the hot loop of the sweep.
//
// One workgroup owns one tile: the 2^T amplitudes whose indices agree on all
// non-local bits.  The local bits are the L lowest index bits (contiguous in
// memory, so a tile is 2^H segments of 2^L amplitudes) plus H higher bits.
// This is the GPU counterpart of the paper's cache blocking (Sec. 5.1): all
// gates that act on local qubits are applied while the tile is on chip, so
// each pass costs one read and one write of the state.
//
// Inside the tile, a register phase hands every thread the 16 amplitudes that
// differ in 4 register slots and applies the phase's op list in registers:
//   - dense blocks of k <= 4 qubits (one-qubit gates stay factored, as in
//     Sec. 5.3, unless the planner multiplies them out);
//   - multiply-free kernels for the factored H', sqrt(X)', sqrt(Y)' and the
//     scaled sqrt(W) (entries +-1, +-i and e^{i pi/4}; Sec. 4.4);
//   - the 8th-root phase of a cluster of diagonal T/S/Z/CZ gates (Sec. 4.3):
//     exponent e(j) = sum_a alpha_a j_a + sum_{a<b} beta_ab j_a j_b (mod 8),
//     evaluated with popcounts and applied as one multiply by e^{i pi e/4}
//     (or as a sign-bit flip when every exponent is 0 or 4);
//   - gradient reductions Im<lambda|G|psi> for the adjoint sweep.
#include "device_common.h"
#include "kernels.h"

namespace svmi {

namespace {

template <class R, int MASK>
__device__ __forceinline__ void dense_mask(V2<R>* a, const V2<R>* __restrict__ u) {
    constexpr int K = __builtin_popcount(MASK);
    constexpr int D = 1 << K;
    V2<R> out[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = V2<R>{R(0), R(0)};
#pragma unroll
    for (int o = 0; o < D; ++o) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const V2<R> m = u[o * D + c];
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

template <class R>
__device__ __forceinline__ void dense_dispatch(V2<R>* a, uint32_t mask, const V2<R>* __restrict__ u) {
    switch (mask) {
        case 1: dense_mask<R, 1>(a, u); break;
        case 2: dense_mask<R, 2>(a, u); break;
        case 3: dense_mask<R, 3>(a, u); break;
        case 4: dense_mask<R, 4>(a, u); break;
        case 5: dense_mask<R, 5>(a, u); break;
        case 6: dense_mask<R, 6>(a, u); break;
        case 7: dense_mask<R, 7>(a, u); break;
        case 8: dense_mask<R, 8>(a, u); break;
        case 9: dense_mask<R, 9>(a, u); break;
        case 10: dense_mask<R, 10>(a, u); break;
        case 11: dense_mask<R, 11>(a, u); break;
        case 12: dense_mask<R, 12>(a, u); break;
        case 13: dense_mask<R, 13>(a, u); break;
        case 14: dense_mask<R, 14>(a, u); break;
#ifndef NO_D4
        case 15: dense_mask<R, 15>(a, u); break;
#endif
        default: break;
    }
}

// Compile-time extraction of the MASK bits of i into a dense index.
__device__ constexpr int ext4(int mask, int i) {
    int out = 0, t = 0;
    for (int b = 0; b < 4; ++b)
        if ((mask >> b) & 1) {
            if ((i >> b) & 1) out |= 1 << t;
            ++t;
        }
    return out;
}

template <class R, int MASK>
__device__ __forceinline__ void diag_mask(V2<R>* a, const V2<R>* __restrict__ d) {
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = cmul(d[ext4(MASK, i)], a[i]);
}

template <class R>
__device__ __forceinline__ void diag_dispatch(V2<R>* a, uint32_t mask, const V2<R>* __restrict__ d) {
    switch (mask) {
        case 1: diag_mask<R, 1>(a, d); break;
        case 2: diag_mask<R, 2>(a, d); break;
        case 3: diag_mask<R, 3>(a, d); break;
        case 4: diag_mask<R, 4>(a, d); break;
        case 5: diag_mask<R, 5>(a, d); break;
        case 6: diag_mask<R, 6>(a, d); break;
        case 7: diag_mask<R, 7>(a, d); break;
        case 8: diag_mask<R, 8>(a, d); break;
        case 9: diag_mask<R, 9>(a, d); break;
        case 10: diag_mask<R, 10>(a, d); break;
        case 11: diag_mask<R, 11>(a, d); break;
        case 12: diag_mask<R, 12>(a, d); break;
        case 13: diag_mask<R, 13>(a, d); break;
        case 14: diag_mask<R, 14>(a, d); break;
        case 15: diag_mask<R, 15>(a, d); break;
        default: break;
    }
}

// Multiply-free one-qubit kernels on register slot S (factored matrices of
// Sec. 4.4; their scale factors are applied once per pass by OP_SCALE).
template <class R, int S, uint32_t KIND>
__device__ __forceinline__ void struct1(V2<R>* a, R c) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & (1 << S)) continue;
        const V2<R> x = a[i], y = a[i | (1 << S)];
        V2<R> o0, o1;
        if constexpr (KIND == OP_HP) {           // [[1,1],[1,-1]]
            o0 = V2<R>{x.x + y.x, x.y + y.y};
            o1 = V2<R>{x.x - y.x, x.y - y.y};
        } else if constexpr (KIND == OP_XP) {    // [[1+i,1-i],[1-i,1+i]]: s +- i d
            const V2<R> s{x.x + y.x, x.y + y.y}, d{x.x - y.x, x.y - y.y};
            o0 = V2<R>{s.x - d.y, s.y + d.x};
            o1 = V2<R>{s.x + d.y, s.y - d.x};
        } else if constexpr (KIND == OP_YP) {    // [[1+i,-1-i],[1+i,1+i]]: (1+i)d, (1+i)s
            const V2<R> s{x.x + y.x, x.y + y.y}, d{x.x - y.x, x.y - y.y};
            o0 = V2<R>{d.x - d.y, d.x + d.y};
            o1 = V2<R>{s.x - s.y, s.x + s.y};
        } else {                                 // [[w,-i],[1,w]], w = c(1+i)
            o0 = V2<R>{fma_(c, x.x - x.y, y.y), fma_(c, x.x + x.y, -y.x)};
            o1 = V2<R>{fma_(c, y.x - y.y, x.x), fma_(c, y.x + y.y, x.y)};
        }
        a[i] = o0;
        a[i | (1 << S)] = o1;
    }
}

template <class R, uint32_t KIND>
__device__ __forceinline__ void struct_dispatch(V2<R>* a, uint32_t mask, R c) {
    switch (mask) {
        case 1: struct1<R, 0, KIND>(a, c); break;
        case 2: struct1<R, 1, KIND>(a, c); break;
        case 4: struct1<R, 2, KIND>(a, c); break;
        case 8: struct1<R, 3, KIND>(a, c); break;
        default: break;
    }
}

__device__ __forceinline__ double imcj(double ux, double uy, double vx, double vy) {
    return ux * vy - uy * vx;  // Im(conj(u) v)
}
__device__ __forceinline__ double recj(double ux, double uy, double vx, double vy) {
    return ux * vx + uy * vy;  // Re(conj(u) v)
}

// Partial Im<lambda|G|psi> over the 16 register amplitudes, FP64.
template <class R, int S>
__device__ __forceinline__ double grad1(const V2<R>* p, const V2<R>* l, uint32_t gen) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i & (1 << S)) continue;
        const int j = i | (1 << S);
        const double p0x = p[i].x, p0y = p[i].y, p1x = p[j].x, p1y = p[j].y;
        const double l0x = l[i].x, l0y = l[i].y, l1x = l[j].x, l1y = l[j].y;
        if (gen == GEN_X) {
            acc += imcj(l0x, l0y, p1x, p1y) + imcj(l1x, l1y, p0x, p0y);
        } else if (gen == GEN_Y) {
            // (Y psi)_0 = -i psi_1, (Y psi)_1 = i psi_0
            acc += -recj(l0x, l0y, p1x, p1y) + recj(l1x, l1y, p0x, p0y);
        } else {
            acc += imcj(l0x, l0y, p0x, p0y) - imcj(l1x, l1y, p1x, p1y);
        }
    }
    return acc;
}

template <class R>
__device__ __forceinline__ double grad_dispatch(const V2<R>* p, const V2<R>* l, uint32_t gen,
                                                uint32_t mask) {
    if (gen == GEN_P11) {
        // generator -2 |11><11| on the two slots of `mask`
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if ((i & mask) == mask)
                acc += -2.0 * imcj(l[i].x, l[i].y, p[i].x, p[i].y);
        return acc;
    }
    switch (mask) {
        case 1: return grad1<R, 0>(p, l, gen);
        case 2: return grad1<R, 1>(p, l, gen);
        case 4: return grad1<R, 2>(p, l, gen);
        case 8: return grad1<R, 3>(p, l, gen);
        default: return 0.0;
    }
}

__device__ __forceinline__ uint32_t ins0(uint32_t x, uint32_t p) {
    const uint32_t lo = x & ((1u << p) - 1u);
    return ((x >> p) << (p + 1)) | lo;
}

__device__ __forceinline__ uint64_t map_local(uint32_t l, uint32_t L, uint32_t H,
                                              const uint32_t* __restrict__ hpos) {
    uint64_t o = l & ((1u << L) - 1u);
    const uint32_t hi = l >> L;
    for (uint32_t t = 0; t < H; ++t) o |= (uint64_t)((hi >> t) & 1u) << hpos[t];
    return o;
}

}  // namespace

template <class R, int NT, bool TWO>
__global__ __launch_bounds__(NT) void k_tile(TileArgs A) {
    using V = V2<R>;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NW = NT / 64;
    const DPass* __restrict__ P = A.pass;
    const uint32_t L = P->L, H = P->H, T = P->T;
    const uint32_t tid = threadIdx.x;
    const uint64_t blk = blockIdx.x;
    const uint32_t b = (uint32_t)(blk >> A.ntile_log2);
    const uint64_t g = blk & ((1ull << A.ntile_log2) - 1ull);

    const uint32_t* __restrict__ hpos = P->hpos;

    // global index of local index 0: deposit g into the non-local bits
    uint64_t base = g << L;
    for (uint32_t t = 0; t < H; ++t) {
        const uint32_t h = hpos[t];
        base = (base & ((1ull << h) - 1ull)) | ((base >> h) << (h + 1));
    }

    V* __restrict__ psi = reinterpret_cast<V*>(A.state) + (uint64_t)b * A.state_bstride;
    V* __restrict__ lam = nullptr;
    if constexpr (TWO) lam = reinterpret_cast<V*>(A.lam) + (uint64_t)b * A.state_bstride;
    const V* __restrict__ pool = reinterpret_cast<const V*>(A.pool) + (uint64_t)b * A.pool_bstride;

    const uint32_t NA = 1u << T;
    V* sA = reinterpret_cast<V*>(smem);
    V* sB = sA + (TWO ? NA : 0);
    V* ptab = sA + (TWO ? 2 * NA : NA);
    uint32_t* fl = reinterpret_cast<uint32_t*>(ptab + 8);
    const uint32_t nform = P->nform;
    double* red = reinterpret_cast<double*>(fl + ((4 * nform + 1) & ~1u));
    const uint32_t ngrad = TWO ? P->ngrad : 0;

    // ---- small per-workgroup tables
    if (tid < 8) ptab[tid] = reinterpret_cast<const V*>(A.phase_tab)[tid];
    for (uint32_t i = tid; i < 4 * nform; i += NT) fl[i] = 0;
    if constexpr (TWO)
        for (uint32_t i = tid; i < ngrad * NW; i += NT) red[i] = 0.0;

    // ---- gather the tile into LDS (16-byte chunks, coalesced along the low bits)
    constexpr uint32_t APC = 16 / sizeof(V);
    const uint32_t nchunk = NA / APC;
    const uint64_t ot = map_local(APC * tid, L, H, hpos);
    for (uint32_t c0 = 0; c0 < nchunk; c0 += 8 * NT) {
        u32x4 va[8];
        u32x4 vb[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t c = c0 + j * NT + tid;
            if (c < nchunk) {
                const uint64_t gi = base + ot + map_local(APC * (c0 + j * NT), L, H, hpos);
                va[j] = *reinterpret_cast<const u32x4*>(psi + gi);
                if constexpr (TWO) vb[j] = *reinterpret_cast<const u32x4*>(lam + gi);
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t c = c0 + j * NT + tid;
            if (c < nchunk) {
                const uint32_t s = swz<R>(APC * c);
                *reinterpret_cast<u32x4*>(sA + s) = va[j];
                if constexpr (TWO) *reinterpret_cast<u32x4*>(sB + s) = vb[j];
            }
        }
    }
    __syncthreads();

    // ---- per-tile parts of the phase forms: Lambda_c masks and constants
    for (uint32_t w = tid; w < nform * 16; w += NT) {
        const uint32_t f = w >> 4, a = w & 15u;
        const DForm* F = A.forms + P->form0 + f;
        if (!F->has_tile) {
            if (a == 0) atomicAdd(&fl[4 * f + 3], F->konst);
            continue;
        }
        if (a < T) {
            const uint32_t lamv = __popcll(base & F->mc[a][0]) + 2u * __popcll(base & F->mc[a][1]) +
                                  4u * __popcll(base & F->mc[a][2]);
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                if ((lamv >> cc) & 1u) atomicOr(&fl[4 * f + cc], 1u << a);
        }
        if (a == 0) {
            const uint32_t kv = F->konst + __popcll(base & F->ka[0]) + 2u * __popcll(base & F->ka[1]) +
                                4u * __popcll(base & F->ka[2]);
            atomicAdd(&fl[4 * f + 3], kv);
        }
    }
    for (uint32_t f = 0; f < nform; ++f) {
        const DForm* F = A.forms + P->form0 + f;
        const uint32_t nq = F->nq;
        for (uint32_t e = tid; e < nq; e += NT) {
            const DPair pr = A.pairs[F->q0 + e];
            if ((base >> pr.b) & 1ull) {
                const uint32_t kv = __popcll(base & pr.m[0]) + 2u * __popcll(base & pr.m[1]) +
                                    4u * __popcll(base & pr.m[2]);
                atomicAdd(&fl[4 * f + 3], kv);
            }
        }
    }
    __syncthreads();

    // ---- register phases
    const uint32_t ngroups = NA >> kRegBits;
    const uint32_t iters = (ngroups + NT - 1) / NT;
    const uint32_t nphase = P->nphase;
    for (uint32_t ph = 0; ph < nphase; ++ph) {
        const DPhase* __restrict__ Ph = A.phases + P->phase0 + ph;
        const uint32_t rpos = Ph->rpos;
        const uint32_t r0 = rpos & 255u, r1 = (rpos >> 8) & 255u, r2 = (rpos >> 16) & 255u,
                       r3 = rpos >> 24;
        uint32_t soff[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) soff[i] = Ph->soff[i];
        const uint32_t op0 = Ph->op0, nop = Ph->nop;
        for (uint32_t it = 0; it < iters; ++it) {
            const uint32_t gg = it * NT + tid;
            const bool act = gg < ngroups;
            const uint32_t lb = ins0(ins0(ins0(ins0(gg, r0), r1), r2), r3);
            const uint32_t sb = swz<R>(lb);
            V a[16];
            V l[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                a[i] = act ? sA[sb ^ soff[i]] : V{R(0), R(0)};
                if constexpr (TWO) l[i] = act ? sB[sb ^ soff[i]] : V{R(0), R(0)};
            }
            for (uint32_t o = op0; o < op0 + nop; ++o) {
                const DOp op = A.ops[o];
                const uint32_t type = rfl(op.type), mask = rfl(op.mask), arg = rfl(op.arg);
                switch (type) {
#ifndef NO_DENSE
                    case OP_DENSE:
                        dense_dispatch<R>(a, mask, pool + arg);
                        if constexpr (TWO) dense_dispatch<R>(l, mask, pool + arg);
                        break;
#endif
                    case OP_DIAGR:
                        diag_dispatch<R>(a, mask, pool + arg);
                        if constexpr (TWO) diag_dispatch<R>(l, mask, pool + arg);
                        break;
#ifndef NO_STRUCT
                    case OP_HP:
                        struct_dispatch<R, OP_HP>(a, mask, R(0));
                        if constexpr (TWO) struct_dispatch<R, OP_HP>(l, mask, R(0));
                        break;
                    case OP_XP:
                        struct_dispatch<R, OP_XP>(a, mask, R(0));
                        if constexpr (TWO) struct_dispatch<R, OP_XP>(l, mask, R(0));
                        break;
                    case OP_YP:
                        struct_dispatch<R, OP_YP>(a, mask, R(0));
                        if constexpr (TWO) struct_dispatch<R, OP_YP>(l, mask, R(0));
                        break;
                    case OP_WP: {
                        const R c = ptab[1].x;  // cos(pi/4) in the state dtype
                        struct_dispatch<R, OP_WP>(a, mask, c);
                        if constexpr (TWO) struct_dispatch<R, OP_WP>(l, mask, c);
                        break;
                    }
#endif
                    case OP_SCALE: {
                        const R s = pool[arg].x;
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            a[i].x *= s; a[i].y *= s;
                            if constexpr (TWO) { l[i].x *= s; l[i].y *= s; }
                        }
                        break;
                    }
#ifndef NO_P8
                    case OP_PHASE8:
                    case OP_SIGN: {
                        const DForm* __restrict__ F = A.forms + arg;
                        const uint32_t fs = F->slot;
                        const uint32_t L0 = fl[4 * fs], L1 = fl[4 * fs + 1], L2 = fl[4 * fs + 2];
                        const uint32_t K = fl[4 * fs + 3];
                        const uint32_t et = act ? (uint32_t)A.etab[F->etab + gg] : 0u;
                        const uint32_t e0 = K + (et & 7u) + __popc(lb & L0) + 2u * __popc(lb & L1) +
                                            4u * __popc(lb & L2);
                        const uint32_t rr[4] = {r0, r1, r2, r3};
                        uint32_t d[4];
#pragma unroll
                        for (int s = 0; s < 4; ++s)
                            d[s] = ((et >> (3 + 3 * s)) & 7u) + ((L0 >> rr[s]) & 1u) +
                                   2u * ((L1 >> rr[s]) & 1u) + 4u * ((L2 >> rr[s]) & 1u);
                        const uint64_t At = (uint64_t)F->a_lo | ((uint64_t)F->a_hi << 32);
                        uint32_t e[16];
                        e[0] = e0;
#pragma unroll
                        for (int i = 1; i < 16; ++i) e[i] = e[i & (i - 1)] + d[__builtin_ctz(i)];
                        if (type == OP_SIGN) {
#pragma unroll
                            for (int i = 0; i < 16; ++i) {
                                const uint32_t f = ((e[i] + (uint32_t)(At >> (3 * i))) >> 2) & 1u;
                                sign_flip(a[i], f);
                                if constexpr (TWO) sign_flip(l[i], f);
                            }
                        } else {
#pragma unroll
                            for (int i = 0; i < 16; ++i) {
                                const uint32_t ee = (e[i] + (uint32_t)(At >> (3 * i))) & 7u;
                                const V t = ptab[ee];
                                a[i] = cmul(t, a[i]);
                                if constexpr (TWO) l[i] = cmul(t, l[i]);
                            }
                        }
                        break;
                    }
#endif
#ifndef NO_GRAD
                    case OP_GRAD:
                        if constexpr (TWO) {
                            double acc = grad_dispatch<R>(a, l, rfl(op.k), mask);
#pragma unroll
                            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
                            if ((tid & 63u) == 0) red[arg * NW + (tid >> 6)] += acc;
                        }
                        break;
#endif
                    default:
                        break;
                }
            }
            if (act) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    sA[sb ^ soff[i]] = a[i];
                    if constexpr (TWO) sB[sb ^ soff[i]] = l[i];
                }
            }
        }
        __syncthreads();
    }

    // ---- gradient partials of this tile
    if constexpr (TWO) {
        if (ngrad) {
            const uint64_t ntile = 1ull << A.ntile_log2;
            double* dst = A.gpart + ((uint64_t)b * ntile + g) * ngrad;
            for (uint32_t j = tid; j < ngrad; j += NT) {
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) s += red[j * NW + w];
                dst[j] = s;
            }
        }
    }

    // ---- scatter the tile back
    for (uint32_t c0 = 0; c0 < nchunk; c0 += 8 * NT) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t c = c0 + j * NT + tid;
            if (c < nchunk) {
                const uint32_t s = swz<R>(APC * c);
                const uint64_t gi = base + ot + map_local(APC * (c0 + j * NT), L, H, hpos);
                *reinterpret_cast<u32x4*>(psi + gi) = *reinterpret_cast<const u32x4*>(sA + s);
                if constexpr (TWO) *reinterpret_cast<u32x4*>(lam + gi) = *reinterpret_cast<const u32x4*>(sB + s);
            }
        }
    }
}

size_t tile_lds_bytes(int dtype, bool two, uint32_t T, uint32_t nform, uint32_t ngrad, int nt) {
    const size_t amp = dtype == 1 ? 8 : 16;
    size_t bytes = (two ? 2 : 1) * ((size_t)1 << T) * amp + 8 * amp;
    bytes += 4 * (((4 * (size_t)nform + 1) & ~(size_t)1));
    if (two) bytes += 8 * (size_t)ngrad * (nt / 64);
    return (bytes + 15) & ~(size_t)15;
}

template <class R, int NT, bool TWO>
static hipError_t launch_one(const TileArgs& a, uint64_t nblocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_tile<R, NT, TWO>), dim3((uint32_t)nblocks), dim3(NT), lds, s, a);
    return hipGetLastError();
}

hipError_t tile_pass_set_attrs(size_t max_lds) {
    const void* fns[] = {
        (const void*)&k_tile<float, 256, false>, (const void*)&k_tile<float, 256, true>,
        (const void*)&k_tile<float, 512, false>, (const void*)&k_tile<float, 512, true>,
        (const void*)&k_tile<double, 256, false>, (const void*)&k_tile<double, 256, true>,
        (const void*)&k_tile<double, 512, false>, (const void*)&k_tile<double, 512, true>,
    };
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_tile_pass(int dtype, bool two, int nt, const TileArgs& a, uint64_t nblocks,
                            size_t lds, hipStream_t s) {
    if (dtype == 1) {
        if (nt == 256) return two ? launch_one<float, 256, true>(a, nblocks, lds, s)
                                  : launch_one<float, 256, false>(a, nblocks, lds, s);
        return two ? launch_one<float, 512, true>(a, nblocks, lds, s)
                   : launch_one<float, 512, false>(a, nblocks, lds, s);
    }
    if (nt == 256) return two ? launch_one<double, 256, true>(a, nblocks, lds, s)
                              : launch_one<double, 256, false>(a, nblocks, lds, s);
    return two ? launch_one<double, 512, true>(a, nblocks, lds, s)
               : launch_one<double, 512, false>(a, nblocks, lds, s);
}

}  // namespace svmi
