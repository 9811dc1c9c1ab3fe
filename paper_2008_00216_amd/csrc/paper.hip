// Kernels of the paper's own plan (the ablation of the tile-pass design):
//
// * a diagonal cluster in one memory pass (Sec. 4.3): every amplitude's
//   phase e^{i pi e/4} from popcounts of its index against the exponent
//   bit-planes of the 8th-root gates, and the CZ sign from the one-mask-per-
//   qubit encoding, updated along a reflected Gray code as the index changes
//   one bit at a time; amplitudes whose phase is 1 are neither read nor
//   written;
// * pairs of one-qubit gates of a layer as the Kronecker product of their
//   unnormalised factors (Sec. 4.4), whose entries are small Gaussian
//   integers known at compile time, so the products are additions,
//   subtractions and real/imaginary swaps; the factored-out scale and phase
//   are kept as counters by the host (Sec. 4.1);
// * the recursive transform of Sec. 5.1 mapped to the GPU: after the pairs
//   on high qubits, the remaining gates of a layer run on contiguous chunks
//   staged in LDS (a chunk per workgroup instead of one per L2 cache);
// * the rescale pass that folds the scale counter back into the state.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace svmi {

namespace {

constexpr int kPB = 256;

// k v for a compile-time k in {-2, -1, 1, 2}: a move, a negation or an
// addition -- never a multiply.
template <int K, class R>
__device__ __forceinline__ R kx(R v) {
    static_assert(K == 1 || K == -1 || K == 2 || K == -2, "small integer coefficient");
    if constexpr (K == 1) return v;
    else if constexpr (K == -1) return -v;
    else if constexpr (K == 2) return v + v;
    else return -(v + v);
}

// a v + b w for compile-time small integers a, b (at least one non-zero)
template <int A, int B, class R>
__device__ __forceinline__ R lin(R v, R w) {
    static_assert(A != 0 || B != 0, "zero coefficient pair");
    if constexpr (A == 0) return kx<B>(w);
    else if constexpr (B == 0) return kx<A>(v);
    else return kx<A>(v) + kx<B>(w);
}

// acc (+)= (a + i b) x for compile-time small integers a, b: the real part
// is a x.re - b x.im and the imaginary part a x.im + b x.re, formed with
// additions, subtractions and swaps only.
template <class R, int A, int B, bool FIRST>
__device__ __forceinline__ void gacc(V2<R>& acc, const V2<R>& x) {
    if constexpr (A == 0 && B == 0) {
        if constexpr (FIRST) acc = V2<R>{R(0), R(0)};
        return;
    } else {
        const R re = lin<A, -B>(x.x, x.y);
        const R im = lin<A, B>(x.y, x.x);
        if constexpr (FIRST) {
            acc.x = re;
            acc.y = im;
        } else {
            acc.x += re;
            acc.y += im;
        }
    }
}

template <class R, int G>
__device__ __forceinline__ void apply1(V2<R>& x0, V2<R>& x1) {
    V2<R> y0, y1;
    gacc<R, pg_fac(G, 0, 0).re, pg_fac(G, 0, 0).im, true>(y0, x0);
    gacc<R, pg_fac(G, 0, 1).re, pg_fac(G, 0, 1).im, false>(y0, x1);
    gacc<R, pg_fac(G, 1, 0).re, pg_fac(G, 1, 0).im, true>(y1, x0);
    gacc<R, pg_fac(G, 1, 1).re, pg_fac(G, 1, 1).im, false>(y1, x1);
    x0 = y0;
    x1 = y1;
}

// Row r of GA' (x) GB' (GA on local bit 0, GB on local bit 1) times x[0..3],
// with the entries halved when all are even (pg_pair_even).
template <int GA, int GB, int R_, int C_>
constexpr GInt pentry() {
    constexpr GInt v = pg_pair(GA, GB, R_, C_);
    return pg_pair_even(GA, GB) ? GInt{v.re / 2, v.im / 2} : v;
}

template <class R, int GA, int GB, int ROW>
__device__ __forceinline__ V2<R> prow(const V2<R>* x) {
    constexpr GInt m0 = pentry<GA, GB, ROW, 0>();
    constexpr GInt m1 = pentry<GA, GB, ROW, 1>();
    constexpr GInt m2 = pentry<GA, GB, ROW, 2>();
    constexpr GInt m3 = pentry<GA, GB, ROW, 3>();
    V2<R> y;
    gacc<R, m0.re, m0.im, true>(y, x[0]);
    gacc<R, m1.re, m1.im, false>(y, x[1]);
    gacc<R, m2.re, m2.im, false>(y, x[2]);
    gacc<R, m3.re, m3.im, false>(y, x[3]);
    return y;
}

template <class R, int GA, int GB>
__device__ __forceinline__ void apply2(V2<R>* x) {
    const V2<R> y0 = prow<R, GA, GB, 0>(x), y1 = prow<R, GA, GB, 1>(x);
    const V2<R> y2 = prow<R, GA, GB, 2>(x), y3 = prow<R, GA, GB, 3>(x);
    x[0] = y0;
    x[1] = y1;
    x[2] = y2;
    x[3] = y3;
}

__device__ __forceinline__ uint64_t ins0_64(uint64_t x, uint32_t p) {
    const uint64_t lo = x & ((1ull << p) - 1ull);
    return ((x >> p) << (p + 1)) | lo;
}

// One pair of gates per pass: each thread owns the four amplitudes whose
// indices differ in bits qa and qb.
template <class R, int GA, int GB>
__global__ __launch_bounds__(kPB) void k_pp_pair(V2<R>* __restrict__ psi, uint64_t bstride, uint32_t qa, uint32_t qb,
                                                 uint64_t count) {
    V2<R>* p = psi + (uint64_t)blockIdx.y * bstride;
    const uint32_t lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
    const uint64_t ba = 1ull << qa, bb = 1ull << qb;
    for (uint64_t s = (uint64_t)blockIdx.x * kPB + threadIdx.x; s < count; s += (uint64_t)gridDim.x * kPB) {
        const uint64_t j = ins0_64(ins0_64(s, lo), hi);
        V2<R> x[4] = {p[j], p[j | ba], p[j | bb], p[j | ba | bb]};
        apply2<R, GA, GB>(x);
        p[j] = x[0];
        p[j | ba] = x[1];
        p[j | bb] = x[2];
        p[j | ba | bb] = x[3];
    }
}

template <class R, int G>
__global__ __launch_bounds__(kPB) void k_pp_one(V2<R>* __restrict__ psi, uint64_t bstride, uint32_t q,
                                                uint64_t count) {
    V2<R>* p = psi + (uint64_t)blockIdx.y * bstride;
    const uint64_t b = 1ull << q;
    for (uint64_t s = (uint64_t)blockIdx.x * kPB + threadIdx.x; s < count; s += (uint64_t)gridDim.x * kPB) {
        const uint64_t j = ins0_64(s, q);
        V2<R> x0 = p[j], x1 = p[j | b];
        apply1<R, G>(x0, x1);
        p[j] = x0;
        p[j | b] = x1;
    }
}

// e^{i pi e / 4} v: sign changes and swaps for even e, one complex
// multiply by (+-1 +- i)/sqrt(2) for odd e.
template <class R>
__device__ __forceinline__ V2<R> mul_w(V2<R> v, uint32_t e, R c) {
    switch (e) {
        case 2: return V2<R>{-v.y, v.x};
        case 4: return V2<R>{-v.x, -v.y};
        case 6: return V2<R>{v.y, -v.x};
        default: {
            const R wr = (e == 1 || e == 7) ? c : -c;
            const R wi = (e == 1 || e == 3) ? c : -c;
            return V2<R>{v.x * wr - v.y * wi, v.x * wi + v.y * wr};
        }
    }
}

// Diagonal cluster: waves own runs of 1024 consecutive amplitudes, lane =
// index bits 0..5, the four bits above visited in reflected Gray order so
// that the CZ sign is updated from one mask per step.
template <class R>
__global__ __launch_bounds__(kPB) void k_pp_diag(V2<R>* __restrict__ psi, uint64_t bstride, uint32_t n, uint64_t e0,
                                                 uint64_t e1, uint64_t e2, const uint64_t* __restrict__ m1s,
                                                 const uint64_t* __restrict__ msym, uint64_t nruns, R c) {
    V2<R>* p = psi + (uint64_t)blockIdx.y * bstride;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t run = (uint64_t)blockIdx.x * (kPB / 64) + (threadIdx.x >> 6);
    if (run >= nruns) return;
    constexpr uint32_t G = 4;
    uint64_t j = (run << (6 + G)) | lane;
    uint32_t par = 0;
    for (uint64_t r = j; r; r &= r - 1) par ^= (uint32_t)__popcll(m1s[__ffsll((long long)r) - 1] & j) & 1u;
    for (uint32_t t = 0; t < (1u << G); ++t) {
        if (t) {
            const uint32_t b = 6u + (uint32_t)__builtin_ctz(t);
            j ^= 1ull << b;
            par ^= (uint32_t)__popcll(msym[b] & j) & 1u;
        }
        const uint32_t e = ((uint32_t)__popcll(j & e0) + 2u * (uint32_t)__popcll(j & e1) +
                            4u * (uint32_t)__popcll(j & e2) + 4u * par) & 7u;
        if (e) p[j] = mul_w<R>(p[j], e, c);
    }
}

// Registers of fewer than 10 qubits: the sign of every index from scratch.
template <class R>
__global__ __launch_bounds__(kPB) void k_pp_diag_small(V2<R>* __restrict__ psi, uint64_t bstride, uint32_t n,
                                                       uint64_t e0, uint64_t e1, uint64_t e2,
                                                       const uint64_t* __restrict__ m1s, R c) {
    V2<R>* p = psi + (uint64_t)blockIdx.y * bstride;
    const uint64_t j = (uint64_t)blockIdx.x * kPB + threadIdx.x;
    if (j >= (1ull << n)) return;
    uint32_t par = 0;
    for (uint64_t r = j; r; r &= r - 1) par ^= (uint32_t)__popcll(m1s[__ffsll((long long)r) - 1] & j) & 1u;
    const uint32_t e = ((uint32_t)__popcll(j & e0) + 2u * (uint32_t)__popcll(j & e1) +
                        4u * (uint32_t)__popcll(j & e2) + 4u * par) & 7u;
    if (e) p[j] = mul_w<R>(p[j], e, c);
}

// The remaining (low-qubit) gates of a layer on chunks of 2^C contiguous
// amplitudes staged in LDS, one chunk per workgroup.  Each op carries its
// matrix of small Gaussian integers (the same entries as the pair kernels;
// products by them are exact, as the additions there are).
struct PPChunkOps {
    uint32_t n;
    uint8_t qa[32], qb[32], single[32];
    int8_t m[32][16][2];      // row-major 4 x 4 (pair) or 2 x 2 in the first 4 (single)
};

template <class R>
__device__ __forceinline__ V2<R> cmul_int(int a, int b, V2<R> x) {
    return V2<R>{R(a) * x.x - R(b) * x.y, R(a) * x.y + R(b) * x.x};
}

template <class R>
__global__ __launch_bounds__(kPB) void k_pp_chunk(V2<R>* __restrict__ psi, uint64_t bstride, uint32_t C,
                                                  PPChunkOps ops) {
    extern __shared__ __align__(16) unsigned char smem[];
    V2<R>* s = reinterpret_cast<V2<R>*>(smem);
    V2<R>* p = psi + (uint64_t)blockIdx.y * bstride + ((uint64_t)blockIdx.x << C);
    const uint32_t N = 1u << C;
    for (uint32_t i = threadIdx.x; i < N; i += kPB) s[i] = p[i];
    __syncthreads();
    for (uint32_t o = 0; o < ops.n; ++o) {
        const uint32_t qa = ops.qa[o];
        if (ops.single[o]) {
            const uint32_t b = 1u << qa;
            for (uint32_t t = threadIdx.x; t < N / 2; t += kPB) {
                const uint32_t j = (uint32_t)ins0_64(t, qa);
                const V2<R> x[2] = {s[j], s[j | b]};
                V2<R> y[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const V2<R> u = cmul_int<R>(ops.m[o][2 * r][0], ops.m[o][2 * r][1], x[0]);
                    const V2<R> v = cmul_int<R>(ops.m[o][2 * r + 1][0], ops.m[o][2 * r + 1][1], x[1]);
                    y[r] = V2<R>{u.x + v.x, u.y + v.y};
                }
                s[j] = y[0];
                s[j | b] = y[1];
            }
        } else {
            const uint32_t qb = ops.qb[o];
            const uint32_t lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
            const uint32_t ba = 1u << qa, bb = 1u << qb;
            for (uint32_t t = threadIdx.x; t < N / 4; t += kPB) {
                const uint32_t j = (uint32_t)ins0_64(ins0_64(t, lo), hi);
                const V2<R> x[4] = {s[j], s[j | ba], s[j | bb], s[j | ba | bb]};
                V2<R> y[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    V2<R> acc = cmul_int<R>(ops.m[o][4 * r][0], ops.m[o][4 * r][1], x[0]);
#pragma unroll
                    for (int cc = 1; cc < 4; ++cc) {
                        const V2<R> v = cmul_int<R>(ops.m[o][4 * r + cc][0], ops.m[o][4 * r + cc][1], x[cc]);
                        acc.x += v.x;
                        acc.y += v.y;
                    }
                    y[r] = acc;
                }
                s[j] = y[0];
                s[j | ba] = y[1];
                s[j | bb] = y[2];
                s[j | ba | bb] = y[3];
            }
        }
        __syncthreads();
    }
    for (uint32_t i = threadIdx.x; i < N; i += kPB) p[i] = s[i];
}

template <class R>
__global__ __launch_bounds__(kPB) void k_pp_scale(V2<R>* __restrict__ psi, uint64_t bstride, uint64_t count, R sr,
                                                  R si) {
    V2<R>* p = psi + (uint64_t)blockIdx.y * bstride;
    for (uint64_t j = (uint64_t)blockIdx.x * kPB + threadIdx.x; j < count; j += (uint64_t)gridDim.x * kPB) {
        const V2<R> v = p[j];
        p[j] = V2<R>{v.x * sr - v.y * si, v.x * si + v.y * sr};
    }
}

inline dim3 pp_grid(uint64_t count, int batch) {
    uint64_t g = (count + kPB - 1) / kPB;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return dim3((uint32_t)g, (uint32_t)batch);
}

template <class R, int GA>
hipError_t pair_b(V2<R>* st, uint64_t bs, int batch, int n, int qa, int qb, int gb, hipStream_t s) {
    const dim3 g = pp_grid(1ull << (n - 2), batch);
    switch (gb) {
        case PG_H: hipLaunchKernelGGL((k_pp_pair<R, GA, PG_H>), g, dim3(kPB), 0, s, st, bs, qa, qb, 1ull << (n - 2)); break;
        case PG_SX: hipLaunchKernelGGL((k_pp_pair<R, GA, PG_SX>), g, dim3(kPB), 0, s, st, bs, qa, qb, 1ull << (n - 2)); break;
        case PG_SXDG: hipLaunchKernelGGL((k_pp_pair<R, GA, PG_SXDG>), g, dim3(kPB), 0, s, st, bs, qa, qb, 1ull << (n - 2)); break;
        case PG_SY: hipLaunchKernelGGL((k_pp_pair<R, GA, PG_SY>), g, dim3(kPB), 0, s, st, bs, qa, qb, 1ull << (n - 2)); break;
        case PG_SYDG: hipLaunchKernelGGL((k_pp_pair<R, GA, PG_SYDG>), g, dim3(kPB), 0, s, st, bs, qa, qb, 1ull << (n - 2)); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class R>
hipError_t pair_t(V2<R>* st, uint64_t bs, int batch, int n, int qa, int ga, int qb, int gb, hipStream_t s) {
    if (gb < 0) {
        const dim3 g = pp_grid(1ull << (n - 1), batch);
        const uint64_t cnt = 1ull << (n - 1);
        switch (ga) {
            case PG_H: hipLaunchKernelGGL((k_pp_one<R, PG_H>), g, dim3(kPB), 0, s, st, bs, qa, cnt); break;
            case PG_SX: hipLaunchKernelGGL((k_pp_one<R, PG_SX>), g, dim3(kPB), 0, s, st, bs, qa, cnt); break;
            case PG_SXDG: hipLaunchKernelGGL((k_pp_one<R, PG_SXDG>), g, dim3(kPB), 0, s, st, bs, qa, cnt); break;
            case PG_SY: hipLaunchKernelGGL((k_pp_one<R, PG_SY>), g, dim3(kPB), 0, s, st, bs, qa, cnt); break;
            case PG_SYDG: hipLaunchKernelGGL((k_pp_one<R, PG_SYDG>), g, dim3(kPB), 0, s, st, bs, qa, cnt); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (n < 2 || qa == qb) return hipErrorInvalidValue;
    switch (ga) {
        case PG_H: return pair_b<R, PG_H>(st, bs, batch, n, qa, qb, gb, s);
        case PG_SX: return pair_b<R, PG_SX>(st, bs, batch, n, qa, qb, gb, s);
        case PG_SXDG: return pair_b<R, PG_SXDG>(st, bs, batch, n, qa, qb, gb, s);
        case PG_SY: return pair_b<R, PG_SY>(st, bs, batch, n, qa, qb, gb, s);
        case PG_SYDG: return pair_b<R, PG_SYDG>(st, bs, batch, n, qa, qb, gb, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_pp_pair(int dtype, void* state, uint64_t bstride, int batch, int n, int qa, int ga, int qb, int gb,
                          hipStream_t s) {
    if (qa < 0 || qa >= n || (gb >= 0 && (qb < 0 || qb >= n))) return hipErrorInvalidValue;
    if (dtype == 1) return pair_t<float>(reinterpret_cast<V2<float>*>(state), bstride, batch, n, qa, ga, qb, gb, s);
    return pair_t<double>(reinterpret_cast<V2<double>*>(state), bstride, batch, n, qa, ga, qb, gb, s);
}

hipError_t launch_pp_diag(int dtype, void* state, uint64_t bstride, int batch, int n, const uint64_t* e8,
                          const uint64_t* d_m1s, const uint64_t* d_msym, hipStream_t s) {
    const double c = 0.70710678118654752440;
    if (n >= 10) {
        const uint64_t nruns = 1ull << (n - 10);
        const uint64_t nb = (nruns + kPB / 64 - 1) / (kPB / 64);
        if (nb > 0x7fffffffull) return hipErrorInvalidValue;
        const dim3 g((uint32_t)nb, (uint32_t)batch);
        if (dtype == 1)
            hipLaunchKernelGGL(k_pp_diag<float>, g, dim3(kPB), 0, s, reinterpret_cast<V2<float>*>(state), bstride,
                               (uint32_t)n, e8[0], e8[1], e8[2], d_m1s, d_msym, nruns, (float)c);
        else
            hipLaunchKernelGGL(k_pp_diag<double>, g, dim3(kPB), 0, s, reinterpret_cast<V2<double>*>(state), bstride,
                               (uint32_t)n, e8[0], e8[1], e8[2], d_m1s, d_msym, nruns, c);
    } else {
        const dim3 g((uint32_t)(((1ull << n) + kPB - 1) / kPB), (uint32_t)batch);
        if (dtype == 1)
            hipLaunchKernelGGL(k_pp_diag_small<float>, g, dim3(kPB), 0, s, reinterpret_cast<V2<float>*>(state),
                               bstride, (uint32_t)n, e8[0], e8[1], e8[2], d_m1s, (float)c);
        else
            hipLaunchKernelGGL(k_pp_diag_small<double>, g, dim3(kPB), 0, s, reinterpret_cast<V2<double>*>(state),
                               bstride, (uint32_t)n, e8[0], e8[1], e8[2], d_m1s, c);
    }
    return hipGetLastError();
}

hipError_t launch_pp_chunk(int dtype, void* state, uint64_t bstride, int batch, int n, int C, int nops,
                           const int* qa, const int* ga, const int* qb, const int* gb, hipStream_t s) {
    if (nops <= 0) return hipSuccess;
    if (nops > 32 || C > n || C < 2) return hipErrorInvalidValue;
    PPChunkOps ops{};
    ops.n = (uint32_t)nops;
    for (int o = 0; o < nops; ++o) {
        if (qa[o] < 0 || qa[o] >= C || ga[o] < 0 || ga[o] >= PG_GEN) return hipErrorInvalidValue;
        if (gb[o] >= 0 && (qb[o] < 0 || qb[o] >= C || qb[o] == qa[o] || gb[o] >= PG_GEN)) return hipErrorInvalidValue;
        ops.qa[o] = (uint8_t)qa[o];
        ops.qb[o] = (uint8_t)(gb[o] >= 0 ? qb[o] : 0);
        ops.single[o] = gb[o] < 0 ? 1 : 0;
        if (gb[o] < 0) {
            for (int e = 0; e < 4; ++e) {
                const GInt v = pg_fac(ga[o], e >> 1, e & 1);
                ops.m[o][e][0] = (int8_t)v.re;
                ops.m[o][e][1] = (int8_t)v.im;
            }
        } else {
            const int h = pg_pair_even(ga[o], gb[o]) ? 2 : 1;
            for (int e = 0; e < 16; ++e) {
                const GInt v = pg_pair(ga[o], gb[o], e >> 2, e & 3);
                ops.m[o][e][0] = (int8_t)(v.re / h);
                ops.m[o][e][1] = (int8_t)(v.im / h);
            }
        }
    }
    const dim3 g((uint32_t)(1ull << (n - C)), (uint32_t)batch);
    const size_t lds = ((size_t)1 << C) * (dtype == 1 ? 8 : 16);
    if (dtype == 1)
        hipLaunchKernelGGL(k_pp_chunk<float>, g, dim3(kPB), lds, s, reinterpret_cast<V2<float>*>(state), bstride,
                           (uint32_t)C, ops);
    else
        hipLaunchKernelGGL(k_pp_chunk<double>, g, dim3(kPB), lds, s, reinterpret_cast<V2<double>*>(state), bstride,
                           (uint32_t)C, ops);
    return hipGetLastError();
}

hipError_t launch_pp_scale(int dtype, void* state, uint64_t bstride, int batch, int n, double re, double im,
                           hipStream_t s) {
    const uint64_t count = 1ull << n;
    const dim3 g = pp_grid(count, batch);
    if (dtype == 1)
        hipLaunchKernelGGL(k_pp_scale<float>, g, dim3(kPB), 0, s, reinterpret_cast<V2<float>*>(state), bstride, count,
                           (float)re, (float)im);
    else
        hipLaunchKernelGGL(k_pp_scale<double>, g, dim3(kPB), 0, s, reinterpret_cast<V2<double>*>(state), bstride,
                           count, re, im);
    return hipGetLastError();
}

}  // namespace svmi
