// Frame of a tile pass: gather a tile into LDS, per-tile parts of the phase
// forms, register-group load/store, gradient partials and the scatter back.
// Shared by the runtime interpreter and the plan-specialised kernels.
#pragma once
#include "device_common.h"
#include "plan.h"

namespace svmi {

struct TileArgs {
    void* state;             // batch element 0 of psi
    void* lam;               // batch element 0 of lambda (adjoint sweep) or nullptr
    const DPass* pass;
    const DPhase* phases;
    const DOp* ops;
    const DForm* forms;
    const DPair* pairs;
    const uint16_t* etab;
    const void* pool;        // matrix pool (state dtype, complex), batch element 0
    uint64_t pool_bstride;   // elements between per-state pools (0 = shared)
    uint64_t state_bstride;  // amplitudes between states
    const void* phase_tab;   // 8 complex entries e^{i pi e / 4} in the state dtype
    double* gpart;           // gradient partials of this pass
    uint32_t ntile_log2;     // log2(tiles per state)
    uint32_t nthreads;
    // Product-state input (one-state passes only): when init_lo is set the
    // tile's amplitudes are not read but computed as lo[j mod 2^init_nlo] *
    // hi[j >> init_nlo] (complex FP64, rounded once), the state the leading
    // one-qubit gates make from |0..0>.
    const double* init_lo;
    const double* init_hi;
    uint32_t init_nlo;
    // One-state passes: when set, the pass also writes the FP64 sum of
    // |psi_j|^2 over each tile it stores, at norm_part[state * tiles + tile].
    double* norm_part;
    // One-state passes: index bits that read as 0 on input (the state is
    // taken as copies of its part with those bits clear, written by the pass
    // in full).  The bits must be tile-local, so that a tile reads only what
    // it writes.  0 = none.
    uint64_t in_mask;
};

template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};

__device__ __forceinline__ uint32_t ins0(uint32_t x, uint32_t p) {
    const uint32_t lo = x & ((1u << p) - 1u);
    return ((x >> p) << (p + 1)) | lo;
}

// Global offset of tile-local index l (low L bits contiguous, then the high
// positions hpos[0..H)).
template <class HP>
__device__ __forceinline__ uint64_t map_local(uint32_t l, uint32_t L, uint32_t H, HP hpos) {
    uint64_t o = l & ((1u << L) - 1u);
    const uint32_t hi = l >> L;
    for (uint32_t t = 0; t < H; ++t) o |= (uint64_t)((hi >> t) & 1u) << hpos[t];
    return o;
}

// STREAM: the tile's global loads and stores carry the non-temporal hint
// (every amplitude is read and written once per pass, so caching them only
// evicts other lines); off in the persistent batch, whose tiles hand data to
// later tiles of the same launch through the cache hierarchy.
template <class R, int NT, bool TWO, bool STREAM = true>
struct TileFrame {
    using V = V2<R>;
    static constexpr int NW = NT / 64;
    uint32_t tid, b, T, NA, ngrad;
    uint64_t g, base, ot;
    V* psi;
    V* lam;
    const V* pool;
    V* sA;
    V* sB;
    V* ptab;
    uint32_t* fl;
    double* red;
    double* nrm;   // NW per-wave norm sums (after the gradient slots)

    __device__ __forceinline__ static u32x4 gload(const u32x4* p) {
        if constexpr (STREAM) return __builtin_nontemporal_load(p);
        else return *p;
    }
    __device__ __forceinline__ static void gstore(u32x4* p, const u32x4& v) {
        if constexpr (STREAM) __builtin_nontemporal_store(v, p);
        else *p = v;
    }

    // Carve LDS, gather the tile, evaluate the per-tile form parts.
    template <class HP>
    __device__ __forceinline__ void begin(const TileArgs& A, unsigned char* smem, uint32_t L, uint32_t H,
                                          uint32_t Tn, HP hpos, uint32_t nform, uint32_t form0,
                                          uint32_t ngrad_) {
        begin_at(A, smem, L, H, Tn, hpos, nform, form0, ngrad_, blockIdx.x);
    }
    // blk = state * 2^ntile_log2 + tile
    // The 16 bytes of the product-state input at global amplitude gi (one
    // complex128 amplitude, or the complex64 pair gi, gi + 1 with gi even).
    __device__ __forceinline__ static u32x4 product_chunk(const TileArgs& A, uint64_t gi) {
        constexpr uint32_t APC = 16 / sizeof(V);
        const uint64_t amask = (1ull << A.init_nlo) - 1ull;
        union {
            V v[APC];
            u32x4 u;
        } out;
#pragma unroll
        for (uint32_t t = 0; t < APC; ++t) {
            const uint64_t j = gi + t;
            const uint64_t a = j & amask, h = j >> A.init_nlo;
            const double ar = A.init_lo[2 * a], ai = A.init_lo[2 * a + 1];
            const double br = A.init_hi[2 * h], bi = A.init_hi[2 * h + 1];
            out.v[t] = V{R(ar * br - ai * bi), R(ar * bi + ai * br)};
        }
        return out.u;
    }

    template <class HP>
    __device__ __forceinline__ void begin_at(const TileArgs& A, unsigned char* smem, uint32_t L, uint32_t H,
                                             uint32_t Tn, HP hpos, uint32_t nform, uint32_t form0,
                                             uint32_t ngrad_, uint64_t blk) {
        tid = threadIdx.x;
        T = Tn;
        NA = 1u << T;
        ngrad = TWO ? ngrad_ : 0u;
        b = (uint32_t)(blk >> A.ntile_log2);
        g = blk & ((1ull << A.ntile_log2) - 1ull);
        base = g << L;
        for (uint32_t t = 0; t < H; ++t) {
            const uint32_t h = hpos[t];
            base = (base & ((1ull << h) - 1ull)) | ((base >> h) << (h + 1));
        }
        psi = reinterpret_cast<V*>(A.state) + (uint64_t)b * A.state_bstride;
        lam = nullptr;
        if constexpr (TWO) lam = reinterpret_cast<V*>(A.lam) + (uint64_t)b * A.state_bstride;
        pool = reinterpret_cast<const V*>(A.pool) + (uint64_t)b * A.pool_bstride;
        sA = reinterpret_cast<V*>(smem);
        sB = sA + (TWO ? NA : 0);
        ptab = sA + (TWO ? 2 * NA : NA);
        fl = reinterpret_cast<uint32_t*>(ptab + 8);
        red = reinterpret_cast<double*>(fl + ((4 * nform + 1) & ~1u));
        nrm = red + (TWO ? ngrad * NW : 0u);

        if (tid < 8) ptab[tid] = reinterpret_cast<const V*>(A.phase_tab)[tid];
        for (uint32_t i = tid; i < 4 * nform; i += NT) fl[i] = 0;
        if constexpr (TWO)
            for (uint32_t i = tid; i < ngrad * NW; i += NT) red[i] = 0.0;

        constexpr uint32_t APC = 16 / sizeof(V);
        const uint32_t nchunk = NA / APC;
        ot = map_local(APC * tid, L, H, hpos);
        const bool pinit = !TWO && A.init_lo != nullptr;   // uniform over the grid
        const uint64_t imask = TWO ? 0ull : A.in_mask;     // uniform
        // 16-byte chunks in flight per thread before the first wait: all 16 of
        // a complex128 tile's share (one state), else 8
        constexpr int KB = (sizeof(V) == 16 && !TWO) ? 16 : 8;
        // (two copies of the loop: the input mask costs nothing when unused)
        auto gather = [&](auto masked) {
        for (uint32_t c0 = 0; c0 < nchunk; c0 += KB * NT) {
            u32x4 va[KB];
            u32x4 vb[TWO ? KB : 1];
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                const uint32_t c = c0 + j * NT + tid;
                if (c < nchunk) {
                    const uint64_t gi = base + ot + map_local(APC * (c0 + j * NT), L, H, hpos);
                    if constexpr (decltype(masked)::value) va[j] = gload(reinterpret_cast<const u32x4*>(psi + (gi & ~imask)));
                    else if (pinit) va[j] = product_chunk(A, gi);
                    else va[j] = gload(reinterpret_cast<const u32x4*>(psi + gi));
                    if constexpr (TWO) vb[j] = gload(reinterpret_cast<const u32x4*>(lam + gi));
                }
            }
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                const uint32_t c = c0 + j * NT + tid;
                if (c < nchunk) {
                    const uint32_t s = swz<R>(APC * c);
                    *reinterpret_cast<u32x4*>(sA + s) = va[j];
                    if constexpr (TWO) *reinterpret_cast<u32x4*>(sB + s) = vb[j];
                }
            }
        }
        };
        if (imask) gather(BoolTag<true>{});
        else gather(BoolTag<false>{});
        __syncthreads();

        // per-tile form parts: Lambda_c (local bits whose nonlocal partner sum
        // has bit c set) and the tile constant K
        for (uint32_t w = tid; w < nform * 16; w += NT) {
            const uint32_t f = w >> 4, a = w & 15u;
            const DForm* F = A.forms + form0 + f;
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
            const DForm* F = A.forms + form0 + f;
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
    }

    __device__ __forceinline__ void load_group(uint32_t sb, const uint32_t* soff, V* a, V* l, bool act) const {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            a[i] = act ? sA[sb ^ soff[i]] : V{R(0), R(0)};
            if constexpr (TWO) l[i] = act ? sB[sb ^ soff[i]] : V{R(0), R(0)};
        }
    }
    __device__ __forceinline__ void store_group(uint32_t sb, const uint32_t* soff, const V* a, const V* l,
                                                bool act) const {
        if (!act) return;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            sA[sb ^ soff[i]] = a[i];
            if constexpr (TWO) sB[sb ^ soff[i]] = l[i];
        }
    }

    // Gradient partial summed over the wave in the state's precision (DPP
    // only, the sum lands in lane 63), then added in FP64 to the per-wave slot.
    __device__ __forceinline__ void grad_add(uint32_t slot, R v) const {
        v = wave_sum_lane63(v);
        if ((tid & 63u) == 63u) red[slot * NW + (tid >> 6)] += (double)v;
    }

    // Gradient partials of this tile and the scatter back to HBM.
    template <class HP>
    __device__ __forceinline__ void end(const TileArgs& A, uint32_t L, uint32_t H, HP hpos) {
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
        constexpr uint32_t APC = 16 / sizeof(V);
        const uint32_t nchunk = NA / APC;
        const bool nsum = !TWO && A.norm_part != nullptr;   // uniform over the grid
        double nacc = 0.0;
        for (uint32_t c0 = 0; c0 < nchunk; c0 += 8 * NT) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t c = c0 + j * NT + tid;
                if (c < nchunk) {
                    const uint32_t s = swz<R>(APC * c);
                    const uint64_t gi = base + ot + map_local(APC * (c0 + j * NT), L, H, hpos);
                    const u32x4 v = *reinterpret_cast<const u32x4*>(sA + s);
                    gstore(reinterpret_cast<u32x4*>(psi + gi), v);
                    if (nsum) nacc += chunk_norm2(v);
                    if constexpr (TWO) gstore(reinterpret_cast<u32x4*>(lam + gi), *reinterpret_cast<const u32x4*>(sB + s));
                }
            }
        }
        if (nsum) {
            // fixed order: chunks per thread, the wave, the waves of the tile
            nacc = wave_sum64(nacc);
            if ((tid & 63u) == 0) nrm[tid >> 6] = nacc;
            __syncthreads();
            if (tid == 0) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) t += nrm[w];
                A.norm_part[((uint64_t)b << A.ntile_log2) + g] = t;
            }
        }
    }

    // FP64 sum of |psi_j|^2 over the amplitudes of one 16-byte chunk.
    __device__ __forceinline__ static double chunk_norm2(const u32x4& u) {
        constexpr uint32_t APC = 16 / sizeof(V);
        union {
            u32x4 u;
            V v[APC];
        } c;
        c.u = u;
        double t = 0.0;
#pragma unroll
        for (uint32_t k = 0; k < APC; ++k) {
            const double x = (double)c.v[k].x, y = (double)c.v[k].y;
            t = __builtin_fma(x, x, t);
            t = __builtin_fma(y, y, t);
        }
        return t;
    }
};

}  // namespace svmi
