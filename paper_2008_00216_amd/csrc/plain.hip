// One-kernel-per-gate ("plain") kernels, initialisation and the adjoint's
// gradient reduction.
//
// The plain kernels are the baseline of Sec. 3: a gate on k qubits updates
// each of the 2^{n-k} disjoint amplitude sets independently.  Diagonal gates
// whose matrix is the identity except for one entry (CZ, Z, S, T, P, CP)
// touch only the amplitudes whose index has every gate bit set (the paper's
// "j & mask == mask" test, Sec. 3), and the permutation gates (NOT, CNOT,
// SWAP, Y) exchange amplitude pairs without arithmetic, so both are exact.
#include "device_common.h"
#include "kernels.h"

namespace svmi {

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kMaxBlocks = 1u << 20;   // grid-stride beyond 2^28 threads per state

__device__ __forceinline__ uint64_t insert_zeros(uint64_t s, const int* tq, int k) {
    for (int t = 0; t < k; ++t) {
        const int p = tq[t];
        s = ((s >> p) << (p + 1)) | (s & ((1ull << p) - 1ull));
    }
    return s;
}

__device__ __forceinline__ uint64_t insert_zeros_mask(uint64_t s, uint64_t mask) {
    while (mask) {
        const int p = __builtin_ctzll(mask);
        s = ((s >> p) << (p + 1)) | (s & ((1ull << p) - 1ull));
        mask &= mask - 1;
    }
    return s;
}

struct Targets {
    int q[6];
};

template <class R, int K>
__global__ __launch_bounds__(kBlock) void k_dense(V2<R>* state, uint64_t bstride, int n, Targets tg,
                                                  const V2<R>* __restrict__ mat, uint64_t mat_bstride,
                                                  uint64_t nsets) {
    constexpr int D = 1 << K;
    const uint32_t b = blockIdx.y;
    V2<R>* psi = state + (uint64_t)b * bstride;
    const V2<R>* u = mat + (uint64_t)b * mat_bstride;
    for (uint64_t gid = (uint64_t)blockIdx.x * kBlock + threadIdx.x; gid < nsets;
         gid += (uint64_t)gridDim.x * kBlock) {
    const uint64_t base = insert_zeros(gid, tg.q, K);
    uint64_t off[D];
#pragma unroll
    for (int l = 0; l < D; ++l) {
        uint64_t o = 0;
#pragma unroll
        for (int t = 0; t < K; ++t)
            if ((l >> t) & 1) o |= 1ull << tg.q[t];
        off[l] = base | o;
    }
    V2<R> in[D];
#pragma unroll
    for (int l = 0; l < D; ++l) in[l] = psi[off[l]];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        V2<R> acc{R(0), R(0)};
#pragma unroll
        for (int c = 0; c < D; ++c) cmac(acc, u[r * D + c], in[c]);
        psi[off[r]] = acc;
    }
    }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_masked_phase(V2<R>* state, uint64_t bstride, uint64_t mask,
                                                         int mode, const V2<R>* __restrict__ val,
                                                         uint64_t val_bstride, uint64_t count) {
    const uint32_t b = blockIdx.y;
    V2<R>* psi = state + (uint64_t)b * bstride;
    for (uint64_t gid = (uint64_t)blockIdx.x * kBlock + threadIdx.x; gid < count;
         gid += (uint64_t)gridDim.x * kBlock) {
    const uint64_t j = insert_zeros_mask(gid, mask) | mask;
    V2<R> a = psi[j];
    if (mode == 1) {
        sign_flip(a, 1u);
    } else if (mode == 2) {          // times +i
        a = V2<R>{-a.y, a.x};
    } else if (mode == 3) {          // times -i
        a = V2<R>{a.y, -a.x};
    } else {
        a = cmul(val[(uint64_t)b * val_bstride], a);
    }
    psi[j] = a;
    }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_diag(V2<R>* state, uint64_t bstride, int k, Targets tg,
                                                 const V2<R>* __restrict__ d, uint64_t d_bstride,
                                                 uint64_t count) {
    const uint32_t b = blockIdx.y;
    V2<R>* psi = state + (uint64_t)b * bstride;
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < count; j += (uint64_t)gridDim.x * kBlock) {
        uint32_t loc = 0;
        for (int t = 0; t < k; ++t) loc |= (uint32_t)((j >> tg.q[t]) & 1ull) << t;
        psi[j] = cmul(d[(uint64_t)b * d_bstride + loc], psi[j]);
    }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_pair_swap(V2<R>* state, uint64_t bstride, uint64_t fixed,
                                                      uint64_t ones, uint64_t flip, int mode,
                                                      uint64_t count) {
    const uint32_t b = blockIdx.y;
    V2<R>* psi = state + (uint64_t)b * bstride;
    for (uint64_t gid = (uint64_t)blockIdx.x * kBlock + threadIdx.x; gid < count;
         gid += (uint64_t)gridDim.x * kBlock) {
    const uint64_t j0 = insert_zeros_mask(gid, fixed) | ones;
    const uint64_t j1 = j0 ^ flip;
    const V2<R> a0 = psi[j0], a1 = psi[j1];
    if (mode == 0) {
        psi[j0] = a1;
        psi[j1] = a0;
    } else {  // Y: (a0, a1) -> (-i a1, i a0)
        psi[j0] = V2<R>{a1.y, -a1.x};
        psi[j1] = V2<R>{-a0.y, a0.x};
    }
    }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_init(V2<R>* state, uint64_t bstride, uint64_t count, int kind,
                                                 uint64_t index, R value) {
    const uint32_t b = blockIdx.y;
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < count; j += (uint64_t)gridDim.x * kBlock) {
        V2<R> v{R(0), R(0)};
        if (kind == 2) v.x = value;
        else if (j == index) v.x = R(1);
        state[(uint64_t)b * bstride + j] = v;
    }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_init_product(V2<R>* state, uint64_t bstride, uint64_t count,
                                                         int nlo, const double* __restrict__ lo,
                                                         const double* __restrict__ hi) {
    const uint32_t b = blockIdx.y;
    // two consecutive amplitudes per thread (same high part when nlo >= 1)
    const uint64_t pairs = count >> 1;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < pairs; p += (uint64_t)gridDim.x * kBlock) {
        const uint64_t j = 2 * p;
        const uint64_t a = j & ((1ull << nlo) - 1ull), h = j >> nlo;
        const double br = hi[2 * h], bi = hi[2 * h + 1];
        const double ar0 = lo[2 * a], ai0 = lo[2 * a + 1], ar1 = lo[2 * a + 2], ai1 = lo[2 * a + 3];
        V2<R> o[2] = {V2<R>{R(ar0 * br - ai0 * bi), R(ar0 * bi + ai0 * br)},
                      V2<R>{R(ar1 * br - ai1 * bi), R(ar1 * bi + ai1 * br)}};
        V2<R>* dst = state + (uint64_t)b * bstride + j;
        dst[0] = o[0];
        dst[1] = o[1];
    }
}

// Gradient partials part[b][tile][slot] are summed over tiles in two steps
// with a fixed order.  Step 1: block (slot chunk of 64, tile chunk c) sums
// tiles [c*tc, (c+1)*tc) with its 4 waves taking every 4th tile, and writes
// the chunk sum over the chunk's first row (read only by this block).
__global__ __launch_bounds__(kBlock) void k_grad_chunk(double* __restrict__ part, uint64_t ntile, uint32_t nslot,
                                                       uint64_t tc) {
    __shared__ double sh[kBlock / 64][64];
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint32_t j = blockIdx.x * 64u + lane;
    const uint64_t t0 = (uint64_t)blockIdx.y * tc;
    const uint64_t t1 = t0 + tc < ntile ? t0 + tc : ntile;
    double* p = part + (uint64_t)blockIdx.z * ntile * nslot;
    double s = 0.0;
    if (j < nslot)
        for (uint64_t t = t0 + w; t < t1; t += kBlock / 64) s += p[t * nslot + j];
    sh[w][lane] = s;
    __syncthreads();
    if (w == 0 && j < nslot) {
        double r = 0.0;
#pragma unroll
        for (int u = 0; u < kBlock / 64; ++u) r += sh[u][lane];
        p[t0 * nslot + j] = r;
    }
}

// Step 2: out[b][slot] = sum over the chunk rows, chunk order.
__global__ __launch_bounds__(kBlock) void k_grad_reduce(const double* __restrict__ part, uint64_t ntile,
                                                        uint32_t nslot, uint64_t tc, double* __restrict__ out,
                                                        uint64_t out_stride) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t b = blockIdx.y;
    if (j >= nslot) return;
    const double* p = part + (uint64_t)b * ntile * nslot + j;
    double s = 0.0;
    for (uint64_t t = 0; t < ntile; t += tc) s += p[t * nslot];
    out[(uint64_t)b * out_stride + j] = s;
}

struct SumTask {
    const double* src;
    uint64_t ntile;
    uint32_t nslot;
    uint32_t pad;
    double* dst;
};

// One block per task: dst[j] = sum_t src[t * nslot + j], t ascending.
__global__ __launch_bounds__(kBlock) void k_multi_sum(const SumTask* __restrict__ tasks) {
    const SumTask t = tasks[blockIdx.x];
    for (uint32_t j = threadIdx.x; j < t.nslot; j += kBlock) {
        double s = 0.0;
        for (uint64_t k = 0; k < t.ntile; ++k) s += t.src[k * t.nslot + j];
        t.dst[j] = s;
    }
}

// Streaming copy of n 16-byte words: grid-stride, four loads in flight per
// thread before the four stores.
__global__ __launch_bounds__(kBlock) void k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                   uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    // four 16-byte words in flight per thread, non-temporal (each word is
    // touched once)
    for (; i + 3 * stride < n; i += 4 * stride) {
        u32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

inline dim3 grid_for(uint64_t count, int batch) {
    uint64_t g = (count + kBlock - 1) / kBlock;
    if (g > kMaxBlocks) g = kMaxBlocks;
    return dim3((uint32_t)g, (uint32_t)batch);
}

}  // namespace

template <class R>
static hipError_t dense_plain_t(void* state, uint64_t bstride, int batch, int n, int k, const int* tq,
                                const void* mat, uint64_t mat_bstride, hipStream_t s) {
    Targets tg{};
    for (int t = 0; t < k; ++t) tg.q[t] = tq[t];
    const uint64_t nsets = 1ull << (n - k);
    auto* st = reinterpret_cast<V2<R>*>(state);
    auto* m = reinterpret_cast<const V2<R>*>(mat);
    const dim3 g = grid_for(nsets, batch);
    switch (k) {
        case 1: hipLaunchKernelGGL((k_dense<R, 1>), g, dim3(kBlock), 0, s, st, bstride, n, tg, m, mat_bstride, nsets); break;
        case 2: hipLaunchKernelGGL((k_dense<R, 2>), g, dim3(kBlock), 0, s, st, bstride, n, tg, m, mat_bstride, nsets); break;
        case 3: hipLaunchKernelGGL((k_dense<R, 3>), g, dim3(kBlock), 0, s, st, bstride, n, tg, m, mat_bstride, nsets); break;
        case 4: hipLaunchKernelGGL((k_dense<R, 4>), g, dim3(kBlock), 0, s, st, bstride, n, tg, m, mat_bstride, nsets); break;
        case 5: hipLaunchKernelGGL((k_dense<R, 5>), g, dim3(kBlock), 0, s, st, bstride, n, tg, m, mat_bstride, nsets); break;
        case 6: hipLaunchKernelGGL((k_dense<R, 6>), g, dim3(kBlock), 0, s, st, bstride, n, tg, m, mat_bstride, nsets); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dense_plain(int dtype, void* state, uint64_t bstride, int batch, int n, int k,
                              const int* tq, const void* mat, uint64_t mat_bstride, hipStream_t s) {
    if (mfma_dense_supported(dtype, n, k))
        return launch_dense_mfma(dtype, state, bstride, batch, n, k, tq, mat, mat_bstride, s);
    return dtype == 1 ? dense_plain_t<float>(state, bstride, batch, n, k, tq, mat, mat_bstride, s)
                      : dense_plain_t<double>(state, bstride, batch, n, k, tq, mat, mat_bstride, s);
}

hipError_t launch_masked_phase(int dtype, void* state, uint64_t bstride, int batch, int n, uint64_t mask,
                               int mode, const void* val, uint64_t val_bstride, hipStream_t s) {
    const uint64_t count = 1ull << (n - __builtin_popcountll(mask));
    const dim3 g = grid_for(count, batch);
    if (dtype == 1)
        hipLaunchKernelGGL(k_masked_phase<float>, g, dim3(kBlock), 0, s, reinterpret_cast<V2<float>*>(state),
                           bstride, mask, mode, reinterpret_cast<const V2<float>*>(val), val_bstride, count);
    else
        hipLaunchKernelGGL(k_masked_phase<double>, g, dim3(kBlock), 0, s, reinterpret_cast<V2<double>*>(state),
                           bstride, mask, mode, reinterpret_cast<const V2<double>*>(val), val_bstride, count);
    return hipGetLastError();
}

hipError_t launch_diag_plain(int dtype, void* state, uint64_t bstride, int batch, int n, int k,
                             const int* tq, const void* d, uint64_t d_bstride, hipStream_t s) {
    Targets tg{};
    for (int t = 0; t < k; ++t) tg.q[t] = tq[t];
    const uint64_t count = 1ull << n;
    const dim3 g = grid_for(count, batch);
    if (dtype == 1)
        hipLaunchKernelGGL(k_diag<float>, g, dim3(kBlock), 0, s, reinterpret_cast<V2<float>*>(state), bstride,
                           k, tg, reinterpret_cast<const V2<float>*>(d), d_bstride, count);
    else
        hipLaunchKernelGGL(k_diag<double>, g, dim3(kBlock), 0, s, reinterpret_cast<V2<double>*>(state), bstride,
                           k, tg, reinterpret_cast<const V2<double>*>(d), d_bstride, count);
    return hipGetLastError();
}

hipError_t launch_pair_swap(int dtype, void* state, uint64_t bstride, int batch, int n, uint64_t zero_mask,
                            uint64_t one_mask, uint64_t flip, int mode, hipStream_t s) {
    const uint64_t fixed = zero_mask | one_mask;
    const uint64_t count = 1ull << (n - __builtin_popcountll(fixed));
    const dim3 g = grid_for(count, batch);
    if (dtype == 1)
        hipLaunchKernelGGL(k_pair_swap<float>, g, dim3(kBlock), 0, s, reinterpret_cast<V2<float>*>(state),
                           bstride, fixed, one_mask, flip, mode, count);
    else
        hipLaunchKernelGGL(k_pair_swap<double>, g, dim3(kBlock), 0, s, reinterpret_cast<V2<double>*>(state),
                           bstride, fixed, one_mask, flip, mode, count);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
        return hipErrorInvalidValue;
    const uint64_t n = bytes / 16;
    uint64_t g = (n + kBlock - 1) / kBlock;
    if (g > 262144) g = 262144;   // enough waves to stream HBM; the rest is grid-stride
    hipLaunchKernelGGL(k_copy16, dim3((uint32_t)g), dim3(kBlock), 0, s, reinterpret_cast<const u32x4*>(src),
                       reinterpret_cast<u32x4*>(dst), n);
    return hipGetLastError();
}

hipError_t launch_init(int dtype, void* state, uint64_t bstride, int batch, int n, int kind, uint64_t index,
                       double value, hipStream_t s) {
    const uint64_t count = 1ull << n;
    const dim3 g = grid_for(count, batch);
    if (dtype == 1)
        hipLaunchKernelGGL(k_init<float>, g, dim3(kBlock), 0, s, reinterpret_cast<V2<float>*>(state), bstride,
                           count, kind, index, (float)value);
    else
        hipLaunchKernelGGL(k_init<double>, g, dim3(kBlock), 0, s, reinterpret_cast<V2<double>*>(state), bstride,
                           count, kind, index, value);
    return hipGetLastError();
}

hipError_t launch_init_product(int dtype, void* state, uint64_t bstride, int batch, int n, int nlo,
                               const double* lo, const double* hi, hipStream_t s) {
    if (nlo < 1 || n < 2) return hipErrorInvalidValue;
    const uint64_t count = 1ull << n;
    const dim3 g = grid_for(count / 2, batch);
    if (dtype == 1)
        hipLaunchKernelGGL(k_init_product<float>, g, dim3(kBlock), 0, s, reinterpret_cast<V2<float>*>(state),
                           bstride, count, nlo, lo, hi);
    else
        hipLaunchKernelGGL(k_init_product<double>, g, dim3(kBlock), 0, s, reinterpret_cast<V2<double>*>(state),
                           bstride, count, nlo, lo, hi);
    return hipGetLastError();
}

hipError_t launch_multi_sum(const void* tasks, uint32_t ntask, hipStream_t s) {
    if (ntask == 0) return hipSuccess;
    hipLaunchKernelGGL(k_multi_sum, dim3(ntask), dim3(kBlock), 0, s, reinterpret_cast<const SumTask*>(tasks));
    return hipGetLastError();
}

hipError_t launch_grad_reduce(double* part, int batch, uint64_t ntile, uint32_t nslot, double* out,
                              uint64_t out_stride, hipStream_t s) {
    if (nslot == 0 || ntile == 0) return hipSuccess;
    const uint64_t nchunk = ntile < 64 ? ntile : 64;
    const uint64_t tc = (ntile + nchunk - 1) / nchunk;
    const uint64_t nc = (ntile + tc - 1) / tc;
    const dim3 g1((nslot + 63) / 64, (uint32_t)nc, (uint32_t)batch);
    hipLaunchKernelGGL(k_grad_chunk, g1, dim3(kBlock), 0, s, part, ntile, nslot, tc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2((nslot + kBlock - 1) / kBlock, (uint32_t)batch);
    hipLaunchKernelGGL(k_grad_reduce, g2, dim3(kBlock), 0, s, part, ntile, nslot, tc, out, out_stride);
    return hipGetLastError();
}

}  // namespace svmi
