// FP64 reductions over the state: the norm check of Sec. 4.1 (accumulated in
// double precision, as the paper recommends for a float state), inner
// products, Pauli-sum expectations and lambda = H psi for the adjoint sweep.
//
// Every reduction uses a fixed grid and a fixed tree, so results are
// bit-reproducible run to run.
#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace svmi {

namespace {

constexpr int kRB = 256;            // threads per reduction block
constexpr uint32_t kMaxRBlk = 8192;  // blocks per state (enough loads in flight to stream HBM)

inline uint32_t nblk_for(int n) {
    const uint64_t N = 1ull << n;
    uint64_t b = (N + 8 * kRB - 1) / (8 * kRB);
    if (b > kMaxRBlk) b = kMaxRBlk;
    if (b < 1) b = 1;
    return (uint32_t)b;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0) {
#pragma unroll
        for (int w = 0; w < kRB / 64; ++w) s += sh[w];
    }
    return s;
}

template <class R>
__device__ __forceinline__ double term_value(const PauliDev& pd, uint64_t j, const V2<R>* psi, double ar,
                                             double ai) {
    double acc = 0.0;
    for (uint32_t g = 0; g < pd.ngroup; ++g) {
        const uint64_t x = pd.x[g];
        const uint64_t jx = j ^ x;
        const V2<R> bq = psi[jx];
        const double br = bq.x, bi = bq.y;
        const double pr = ar * br + ai * bi;   // Re conj(a) b
        const double pi = ar * bi - ai * br;   // Im conj(a) b
        const uint32_t t1 = pd.g0[g + 1];
        for (uint32_t t = pd.g0[g]; t < t1; ++t) {
            const double s = (__popcll(jx & pd.z[t]) & 1) ? -1.0 : 1.0;
            const uint32_t ph = pd.ph[t];
            const double v = (ph & 1) ? pi : pr;
            const double sg = (ph == 1 || ph == 2) ? -1.0 : 1.0;
            acc += pd.c[t] * s * sg * v;
        }
    }
    return acc;
}

template <class R>
__global__ __launch_bounds__(kRB) void k_reduce(int kind, const V2<R>* __restrict__ a,
                                                const V2<R>* __restrict__ b2, uint64_t bstride, uint64_t N,
                                                PauliDev pd, int gen, uint64_t gmask,
                                                double* __restrict__ partials) {
    __shared__ double sh[kRB / 64];
    const uint32_t b = blockIdx.y;
    const V2<R>* pa = a + (uint64_t)b * bstride;
    const V2<R>* pb = b2 ? b2 + (uint64_t)b * bstride : nullptr;
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kRB;
    uint64_t j0 = (uint64_t)blockIdx.x * kRB + threadIdx.x;
    if (kind <= 1) {
        // four amplitudes in flight per thread, fixed order
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (; j0 + 3 * stride < N; j0 += 4 * stride) {
            V2<R> v[4], w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = pa[j0 + u * stride];
            if (kind == 1) {
#pragma unroll
                for (int u = 0; u < 4; ++u) w[u] = pb[j0 + u * stride];
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) w[u] = v[u];
            }
            a0 += (double)v[0].x * (double)w[0].x + (double)v[0].y * (double)w[0].y;
            a1 += (double)v[1].x * (double)w[1].x + (double)v[1].y * (double)w[1].y;
            a2 += (double)v[2].x * (double)w[2].x + (double)v[2].y * (double)w[2].y;
            a3 += (double)v[3].x * (double)w[3].x + (double)v[3].y * (double)w[3].y;
        }
        acc = (a0 + a1) + (a2 + a3);
    }
    for (uint64_t j = j0; j < N; j += stride) {
        const V2<R> v = pa[j];
        const double vr = v.x, vi = v.y;
        if (kind == 0) {
            acc += vr * vr + vi * vi;
        } else if (kind == 1) {
            const V2<R> w = pb[j];
            acc += vr * (double)w.x + vi * (double)w.y;
        } else if (kind == 2) {
            acc += term_value<R>(pd, j, pa, vr, vi);
        } else {
            // Im <lambda|G|psi>: a = psi, b = lambda
            const V2<R> l = pb[j];
            const double lr = l.x, li = l.y;
            if (gen == GEN_Z) {
                const double s = (j & gmask) ? -1.0 : 1.0;
                acc += s * (lr * vi - li * vr);
            } else if (gen == GEN_P11) {
                if ((j & gmask) == gmask) acc += -2.0 * (lr * vi - li * vr);
            } else {
                const V2<R> w = pa[j ^ gmask];
                const double wr = w.x, wi = w.y;
                if (gen == GEN_X) {
                    acc += lr * wi - li * wr;
                } else {  // Y: (Y psi)_j = -+ i psi_{j^m}
                    const double s = (j & gmask) ? 1.0 : -1.0;
                    acc += s * (lr * wr + li * wi);
                }
            }
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[(uint64_t)b * gridDim.x + blockIdx.x] = s;
}

// Sum of the block partials of one state: strided per thread, then the
// fixed block tree.
__global__ __launch_bounds__(kRB) void k_final(const double* __restrict__ partials, uint32_t nb,
                                               double* __restrict__ out, uint64_t out_stride) {
    __shared__ double sh[kRB / 64];
    const uint32_t b = blockIdx.x;
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < nb; i += kRB) acc += partials[(uint64_t)b * nb + i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[(uint64_t)b * out_stride] = s;
}

template <class R>
__global__ __launch_bounds__(kRB) void k_hpsi(const V2<R>* __restrict__ psi, V2<R>* __restrict__ lam,
                                              uint64_t bstride, uint64_t N, PauliDev pd) {
    const uint32_t b = blockIdx.y;
    const V2<R>* p = psi + (uint64_t)b * bstride;
    for (uint64_t j = (uint64_t)blockIdx.x * kRB + threadIdx.x; j < N; j += (uint64_t)gridDim.x * kRB) {
    double lr = 0.0, li = 0.0;
    for (uint32_t g = 0; g < pd.ngroup; ++g) {
        const uint64_t jx = j ^ pd.x[g];
        const V2<R> v = p[jx];
        const double vr = v.x, vi = v.y;
        const uint32_t t1 = pd.g0[g + 1];
        for (uint32_t t = pd.g0[g]; t < t1; ++t) {
            const double s = ((__popcll(jx & pd.z[t]) & 1) ? -1.0 : 1.0) * pd.c[t];
            // multiply (vr + i vi) by s * i^{ph}
            const uint32_t ph = pd.ph[t];
            double xr = vr, xi = vi;
            if (ph & 1) { const double tmp = xr; xr = -xi; xi = tmp; }
            if (ph & 2) { xr = -xr; xi = -xi; }
            lr += s * xr;
            li += s * xi;
        }
    }
    lam[(uint64_t)b * bstride + j] = V2<R>{R(lr), R(li)};
    }
}

// ---- measurement sampling ---------------------------------------------------
// Sum of |psi_j|^2 over each chunk of 2^kChunkBits consecutive amplitudes
// (FP64, fixed block tree).
constexpr int kChunkBits = 12;

template <class R>
__global__ __launch_bounds__(kRB) void k_chunk_sums(const V2<R>* __restrict__ a, uint64_t bstride, uint32_t cbits,
                                                    double* __restrict__ sums, uint64_t nchunk) {
    __shared__ double sh[kRB / 64];
    const uint32_t b = blockIdx.y;
    const V2<R>* pa = a + (uint64_t)b * bstride + ((uint64_t)blockIdx.x << cbits);
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < (1u << cbits); i += kRB) {
        const V2<R> v = pa[i];
        acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) sums[(uint64_t)b * nchunk + blockIdx.x] = s;
}

// One block per chunk that holds samples: the chunk's inclusive prefix sums
// of |psi_j|^2 in LDS (FP64), then for every sample of the chunk the first
// index whose prefix exceeds the sample's residual target.
template <class R>
__global__ __launch_bounds__(kRB) void k_chunk_find(const V2<R>* __restrict__ a, uint64_t bstride, uint32_t cbits,
                                                    const SampleTask* __restrict__ tasks,
                                                    const double* __restrict__ target, uint64_t* __restrict__ out) {
    __shared__ double pre[1 << kChunkBits];
    __shared__ double part[kRB];
    const SampleTask t = tasks[blockIdx.x];
    const uint32_t C = 1u << cbits, per = (C + kRB - 1) / kRB;
    const V2<R>* pa = a + (uint64_t)t.state * bstride + (t.chunk << cbits);
    // each thread: a contiguous run of `per` amplitudes, prefix within the run
    double acc = 0.0;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t i = threadIdx.x * per + k;
        if (i >= C) break;
        const V2<R> v = pa[i];
        acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        pre[i] = acc;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (uint32_t w = 0; w < kRB; ++w) {
            const double v = part[w];
            part[w] = run;   // exclusive prefix of the runs
            run += v;
        }
    }
    __syncthreads();
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t i = threadIdx.x * per + k;
        if (i >= C) break;
        pre[i] += part[threadIdx.x];
    }
    __syncthreads();
    for (uint64_t s = t.s0 + threadIdx.x; s < t.s1; s += kRB) {
        const double r = target[s];
        // first i with pre[i] > r; a residual at or past the chunk's total
        // (rounding) takes the last amplitude with nonzero probability
        uint32_t lo = 0, hi = C;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pre[mid] > r) hi = mid; else lo = mid + 1;
        }
        if (lo >= C) {
            lo = C - 1;
            while (lo > 0 && pre[lo] == pre[lo - 1]) --lo;
        }
        out[t.out0 + (s - t.s0)] = (t.chunk << cbits) + lo;
    }
}

template <class R>
__global__ __launch_bounds__(kRB) void k_gather(const V2<R>* __restrict__ a, uint64_t bstride, int batch,
                                                const uint64_t* __restrict__ idx, uint64_t count,
                                                double* __restrict__ out) {
    const uint64_t k = (uint64_t)blockIdx.x * kRB + threadIdx.x;
    const uint32_t b = blockIdx.y;
    if (k >= count) return;
    const V2<R> v = a[(uint64_t)b * bstride + idx[k]];
    out[2 * ((uint64_t)b * count + k)] = (double)v.x;
    out[2 * ((uint64_t)b * count + k) + 1] = (double)v.y;
}

}  // namespace

uint32_t sample_chunk_bits(int n) { return (uint32_t)std::min(n, kChunkBits); }

hipError_t launch_chunk_sums(int dtype, const void* a, uint64_t bstride, int batch, int n, double* sums,
                             hipStream_t s) {
    const uint32_t cb = sample_chunk_bits(n);
    const uint64_t nchunk = 1ull << (n - (int)cb);
    const dim3 g((uint32_t)nchunk, (uint32_t)batch);
    if (dtype == 1)
        hipLaunchKernelGGL(k_chunk_sums<float>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<float>*>(a), bstride,
                           cb, sums, nchunk);
    else
        hipLaunchKernelGGL(k_chunk_sums<double>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<double>*>(a),
                           bstride, cb, sums, nchunk);
    return hipGetLastError();
}

hipError_t launch_chunk_find(int dtype, const void* a, uint64_t bstride, int n, const SampleTask* tasks,
                             uint32_t ntask, const double* target, uint64_t* out, hipStream_t s) {
    if (ntask == 0) return hipSuccess;
    const uint32_t cb = sample_chunk_bits(n);
    if (dtype == 1)
        hipLaunchKernelGGL(k_chunk_find<float>, dim3(ntask), dim3(kRB), 0, s, reinterpret_cast<const V2<float>*>(a),
                           bstride, cb, tasks, target, out);
    else
        hipLaunchKernelGGL(k_chunk_find<double>, dim3(ntask), dim3(kRB), 0, s,
                           reinterpret_cast<const V2<double>*>(a), bstride, cb, tasks, target, out);
    return hipGetLastError();
}

hipError_t launch_gather(int dtype, const void* a, uint64_t bstride, int batch, const uint64_t* idx, uint64_t count,
                         double* out, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const dim3 g((uint32_t)((count + kRB - 1) / kRB), (uint32_t)batch);
    if (dtype == 1)
        hipLaunchKernelGGL(k_gather<float>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<float>*>(a), bstride,
                           batch, idx, count, out);
    else
        hipLaunchKernelGGL(k_gather<double>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<double>*>(a), bstride,
                           batch, idx, count, out);
    return hipGetLastError();
}

size_t reduce_partials_size(int n, int batch) { return (size_t)nblk_for(n) * (size_t)batch; }

hipError_t launch_reduce(int dtype, int kind, const void* a, const void* b, uint64_t bstride, int batch, int n,
                         const PauliDev* pd, int gen, uint64_t gmask, double* partials, double* out,
                         uint64_t out_stride, hipStream_t s) {
    const uint32_t nb = nblk_for(n);
    const uint64_t N = 1ull << n;
    PauliDev p{};
    if (pd) p = *pd;
    const dim3 g(nb, (uint32_t)batch);
    if (dtype == 1)
        hipLaunchKernelGGL(k_reduce<float>, g, dim3(kRB), 0, s, kind, reinterpret_cast<const V2<float>*>(a),
                           reinterpret_cast<const V2<float>*>(b), bstride, N, p, gen, gmask, partials);
    else
        hipLaunchKernelGGL(k_reduce<double>, g, dim3(kRB), 0, s, kind, reinterpret_cast<const V2<double>*>(a),
                           reinterpret_cast<const V2<double>*>(b), bstride, N, p, gen, gmask, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_final, dim3((uint32_t)batch), dim3(kRB), 0, s, partials, nb, out, out_stride);
    return hipGetLastError();
}

hipError_t launch_hpsi(int dtype, const void* psi, void* lam, uint64_t bstride, int batch, int n,
                       const PauliDev& pd, hipStream_t s) {
    const uint64_t N = 1ull << n;
    uint64_t gx = (N + kRB - 1) / kRB;
    if (gx > (1u << 20)) gx = 1u << 20;
    const dim3 g((uint32_t)gx, (uint32_t)batch);
    if (dtype == 1)
        hipLaunchKernelGGL(k_hpsi<float>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<float>*>(psi),
                           reinterpret_cast<V2<float>*>(lam), bstride, N, pd);
    else
        hipLaunchKernelGGL(k_hpsi<double>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<double>*>(psi),
                           reinterpret_cast<V2<double>*>(lam), bstride, N, pd);
    return hipGetLastError();
}

}  // namespace svmi
