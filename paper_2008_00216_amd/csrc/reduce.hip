// FP64 reductions over the state: the norm check of Sec. 4.1 (accumulated in
// double precision, as the paper recommends for a float state), inner
// products, Pauli-sum expectations and lambda = H psi for the adjoint sweep.
//
// Every reduction uses a fixed grid and a fixed tree, so results are
// bit-reproducible run to run.
#include <algorithm>

#include "device_common.h"
#include "hpsi_tile.h"
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

// lambda = H psi for a Pauli sum.  With epart, each block also writes its
// FP64 partial of Re <psi|lambda> = <psi|H|psi> (lambda before rounding to
// the state precision), at epart[state * gridDim.x + block].
template <class R>
__global__ __launch_bounds__(kRB) void k_hpsi(const V2<R>* __restrict__ psi, V2<R>* __restrict__ lam,
                                              uint64_t bstride, uint64_t N, PauliDev pd,
                                              double* __restrict__ epart) {
    __shared__ double sh[kRB / 64];
    const uint32_t b = blockIdx.y;
    const V2<R>* p = psi + (uint64_t)b * bstride;
    double e = 0.0;
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
    if (epart) {
        const V2<R> v0 = p[j];
        e += (double)v0.x * lr + (double)v0.y * li;
    }
    }
    if (epart) {   // uniform over the grid
        const double t = block_sum(e, sh);
        if (threadIdx.x == 0) epart[(uint64_t)b * gridDim.x + blockIdx.x] = t;
    }
}

// lambda = H psi by tiles of 2^11 consecutive amplitudes (n >= 11), the
// same sum as k_hpsi with the work per wave cut to a few instructions per
// amplitude (hpsi_tile11).  The block's FP64 partial of Re <psi|lambda>
// (lambda before rounding) goes to epart[state * gridDim.x + block].
template <class R>
__global__ __launch_bounds__(kRB) void k_hpsi_tile(const V2<R>* __restrict__ psi, V2<R>* __restrict__ lam,
                                                   uint64_t bstride, PauliDev pd, double* __restrict__ epart) {
    __shared__ V2<R> tile[1 << kHB];
    __shared__ double sh[kRB / 64];
    const uint32_t b = blockIdx.y;
    const uint64_t t0 = (uint64_t)blockIdx.x << kHB;
    const double e = hpsi_tile11<R>(psi + (uint64_t)b * bstride, lam + (uint64_t)b * bstride, t0, pd, tile, false);
    if (epart) {
        const double s = block_sum(e, sh);
        if (threadIdx.x == 0) epart[(uint64_t)b * gridDim.x + blockIdx.x] = s;
    }
}

// ---- measurement sampling ---------------------------------------------------
// A 64-ary tree of FP64 probability masses over each state: level 0 is
// |psi_j|^2 (never stored), node i of level k+1 is the sum of nodes
// 64 i .. 64 i + 63 of level k.  One launch builds two levels; a sample
// descends from the root with one wave, choosing at every level the first
// child whose inclusive prefix exceeds the residual target.

__device__ __forceinline__ double prob(const V2<float>& v) {
    return (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}
__device__ __forceinline__ double prob(const V2<double>& v) { return v.x * v.x + v.y * v.y; }
__device__ __forceinline__ double prob(double v) { return v; }

// A block step covers 4096 consecutive nodes of level k: wave w sums groups
// 16 w .. 16 w + 15 of 64 nodes into level k+1 (coalesced loads, lane l
// holding node l of each group, a 64-lane sum per group), and the step's
// 64 level-(k+1) nodes go through LDS into one level-(k+2) node and one
// coalesced store of the level-(k+1) nodes.  Blocks stride over the steps
// with the next step's loads issued before the current step's arithmetic.
// cnt_in: nodes per state at level k (a power of two).
template <class In>
__device__ __forceinline__ void tree_load(const In* pin, uint64_t step, uint64_t cnt_in, In (&v)[16]) {
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint64_t i0 = step * 4096 + (uint64_t)w * 1024 + lane;
#pragma unroll
    for (int g = 0; g < 16; ++g) {
        const uint64_t i = i0 + (uint64_t)g * 64;
        if (i < cnt_in) v[g] = pin[i]; else v[g] = In{};
    }
}

template <class In>
__global__ __launch_bounds__(kRB) void k_tree2(const In* __restrict__ in, uint64_t stride_in, uint64_t cnt_in,
                                               double* __restrict__ out1, double* __restrict__ out2) {
    __shared__ double sh[64];
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint32_t b = blockIdx.y;
    const uint64_t cnt1 = cnt_in > 64 ? cnt_in >> 6 : 1, cnt2 = cnt1 > 64 ? cnt1 >> 6 : 1;
    const uint64_t nstep = (cnt_in + 4095) / 4096;
    const In* pin = in + (uint64_t)b * stride_in;
    uint64_t step = blockIdx.x;
    if (step >= nstep) return;   // block-uniform
    In v[16];
    tree_load(pin, step, cnt_in, v);
    for (; step < nstep; step += gridDim.x) {
        double p[16];
#pragma unroll
        for (int g = 0; g < 16; ++g) p[g] = prob(v[g]);
        const uint64_t nxt = step + gridDim.x;
        if (nxt < nstep) tree_load(pin, nxt, cnt_in, v);
#pragma unroll
        for (int g = 0; g < 16; ++g) {
            const double t = wave_sum64(p[g]);
            if (lane == 0) sh[w * 16 + g] = t;
        }
        __syncthreads();
        if (w == 0) {
            const double t = sh[lane];
            const uint64_t node = step * 64 + lane;
            if (node < cnt1) out1[(uint64_t)b * cnt1 + node] = t;
            if (out2) {
                const double t2 = wave_sum64(node < cnt1 ? t : 0.0);
                if (lane == 0) out2[(uint64_t)b * cnt2 + step] = t2;
            }
        }
        __syncthreads();
    }
}

// Levels 1 and 2 from complex64 amplitudes.  Each lane loads two adjacent
// amplitudes (16 bytes), so one wave load covers groups 2k and 2k+1 (lanes
// 0-31 and 32-63): a row sum (DPP within each 16-lane row) and two row
// pairs give both group sums, half the reduction work of one 64-lane sum
// per group.  Same node layout, launch shape and prefetch as k_tree2.
__global__ __launch_bounds__(kRB) void k_tree2_c64(const V2<float>* __restrict__ in, uint64_t stride_in,
                                                   uint64_t cnt_in, double* __restrict__ out1,
                                                   double* __restrict__ out2) {
    __shared__ double sh[64];
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint32_t b = blockIdx.y;
    const uint64_t cnt1 = cnt_in > 64 ? cnt_in >> 6 : 1, cnt2 = cnt1 > 64 ? cnt1 >> 6 : 1;
    const uint64_t nstep = (cnt_in + 4095) / 4096;
    const V2<float>* pin = in + (uint64_t)b * stride_in;
    uint64_t step = blockIdx.x;
    if (step >= nstep) return;   // block-uniform
    auto load = [&](uint64_t st, u32x4 (&v)[8]) {
        const uint64_t i0 = st * 4096 + (uint64_t)w * 1024 + 2u * lane;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint64_t i = i0 + (uint64_t)k * 128;   // even, so i + 1 < cnt_in when i < cnt_in
            if (i < cnt_in) v[k] = *reinterpret_cast<const u32x4*>(pin + i);
            else v[k] = u32x4{0u, 0u, 0u, 0u};
        }
    };
    u32x4 v[8];
    load(step, v);
    for (; step < nstep; step += gridDim.x) {
        double p[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float x0 = __uint_as_float(v[k].x), y0 = __uint_as_float(v[k].y);
            const float x1 = __uint_as_float(v[k].z), y1 = __uint_as_float(v[k].w);
            double t = (double)x0 * (double)x0;
            t = __builtin_fma((double)y0, (double)y0, t);
            t = __builtin_fma((double)x1, (double)x1, t);
            p[k] = __builtin_fma((double)y1, (double)y1, t);
        }
        const uint64_t nxt = step + gridDim.x;
        if (nxt < nstep) load(nxt, v);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            double t = p[k];
            t += dpp_f64<0xB1>(t);    // quad_perm [1,0,3,2]
            t += dpp_f64<0x4E>(t);    // quad_perm [2,3,0,1]
            t += dpp_f64<0x124>(t);   // row_ror:4
            t += dpp_f64<0x128>(t);   // row_ror:8: every lane holds its row's sum
            const double g0 = lane_f64(t, 0) + lane_f64(t, 16);
            const double g1 = lane_f64(t, 32) + lane_f64(t, 48);
            if (lane == 0) {
                sh[w * 16 + 2 * k] = g0;
                sh[w * 16 + 2 * k + 1] = g1;
            }
        }
        __syncthreads();
        if (w == 0) {
            const double t = sh[lane];
            const uint64_t node = step * 64 + lane;
            if (node < cnt1) out1[(uint64_t)b * cnt1 + node] = t;
            if (out2) {
                const double t2 = wave_sum64(node < cnt1 ? t : 0.0);
                if (lane == 0) out2[(uint64_t)b * cnt2 + step] = t2;
            }
        }
        __syncthreads();
    }
}

// Inclusive prefix sum over the 64 lanes of a wave (FP64).
__device__ __forceinline__ double wave_incl_scan(double v) {
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}

// One wave per sample.  lvl[k] (k = 1..K) points at level k of all states
// (state b's nodes at b * cnt(k)); level K has one node.  uniforms and out:
// batch * count values, row b for state b.
struct TreeLevels {
    const double* lvl[8];
    int K;
};

template <class R>
__global__ __launch_bounds__(kRB) void k_descend(const V2<R>* __restrict__ a, uint64_t bstride, int n,
                                                 TreeLevels tl, const double* __restrict__ uniforms,
                                                 uint64_t count, uint64_t total, uint64_t* __restrict__ out) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t s = (uint64_t)blockIdx.x * (kRB / 64) + (threadIdx.x >> 6);
    if (s >= total) return;   // wave-uniform
    const uint64_t b = s / count;
    double r = 0.0;
    uint64_t j = 0;   // node index at level k + 1
    for (int k = tl.K - 1; k >= 0; --k) {
        const int lb = n - 6 * k;   // log2 of the node count at level k
        const uint32_t nch = lb >= 6 ? 64u : (1u << lb);
        const uint64_t c = j * 64 + lane;
        double v = 0.0;
        if (lane < nch) {
            if (k == 0)
                v = prob(a[b * bstride + c]);
            else
                v = tl.lvl[k][(b << lb) + c];
        }
        const double incl = wave_incl_scan(v);
        if (k == tl.K - 1) r = uniforms[s] * __shfl(incl, 63, 64);   // target = u * total mass
        uint64_t m = __ballot(lane < nch && incl > r);
        uint32_t pick;
        if (m) {
            pick = (uint32_t)__builtin_ctzll(m);
        } else {
            // r at or past the children's total (rounding): the last child
            // with nonzero mass
            m = __ballot(lane < nch && v > 0.0);
            pick = m ? 63u - (uint32_t)__builtin_clzll(m) : 0u;
        }
        r -= __shfl(incl - v, (int)pick, 64);
        j = j * 64 + pick;
    }
    if (lane == 0) out[s] = j;
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

int sample_levels(int n) { return (n + 5) / 6; }

uint64_t sample_tree_doubles(int n, int batch) {
    uint64_t t = 0;
    for (int k = 1; k <= sample_levels(n); ++k) t += 1ull << std::max(0, n - 6 * k);
    return t * (uint64_t)batch;
}

hipError_t launch_sample(int dtype, const void* a, uint64_t bstride, int batch, int n, double* tree,
                         const double* uniforms, uint64_t count, uint64_t* out, hipStream_t s) {
    const int K = sample_levels(n);
    if (K > 7) return hipErrorInvalidValue;
    TreeLevels tl{};
    tl.K = K;
    double* lv[8] = {};
    uint64_t off = 0;
    for (int k = 1; k <= K; ++k) {
        lv[k] = tree + off;
        tl.lvl[k] = lv[k];
        off += (uint64_t)batch << std::max(0, n - 6 * k);
    }
    // levels 1, 2 from the amplitudes, then two more per launch
    for (int k = 0; k < K; k += 2) {
        const uint64_t cnt_in = 1ull << std::max(0, n - 6 * k);
        // 8 resident blocks per CU over the whole batch
        const uint64_t cap = std::max<uint64_t>(1, 2048 / (uint64_t)batch);
        const dim3 g((uint32_t)std::min<uint64_t>((cnt_in + 4095) / 4096, cap), (uint32_t)batch);
        double* o2 = k + 2 <= K ? lv[k + 2] : nullptr;
        if (k == 0) {
            if (dtype == 1)
                hipLaunchKernelGGL(k_tree2_c64, g, dim3(kRB), 0, s, reinterpret_cast<const V2<float>*>(a), bstride,
                                   cnt_in, lv[1], o2);
            else
                hipLaunchKernelGGL(k_tree2<V2<double>>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<double>*>(a),
                                   bstride, cnt_in, lv[1], o2);
        } else {
            hipLaunchKernelGGL(k_tree2<double>, g, dim3(kRB), 0, s, lv[k], cnt_in, cnt_in, lv[k + 1], o2);
        }
    }
    const uint64_t total = count * (uint64_t)batch;
    if (total == 0) return hipGetLastError();
    const uint32_t per = kRB / 64;
    const dim3 gd((uint32_t)((total + per - 1) / per));
    if (dtype == 1)
        hipLaunchKernelGGL(k_descend<float>, gd, dim3(kRB), 0, s, reinterpret_cast<const V2<float>*>(a), bstride, n,
                           tl, uniforms, count, total, out);
    else
        hipLaunchKernelGGL(k_descend<double>, gd, dim3(kRB), 0, s, reinterpret_cast<const V2<double>*>(a), bstride,
                           n, tl, uniforms, count, total, out);
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

uint64_t hpsi_blocks(int n) {
    if (n >= kHB) return 1ull << (n - kHB);
    const uint64_t N = 1ull << n;
    uint64_t gx = (N + kRB - 1) / kRB;
    return gx > (1u << 20) ? (1u << 20) : gx;
}

hipError_t launch_hpsi(int dtype, const void* psi, void* lam, uint64_t bstride, int batch, int n,
                       const PauliDev& pd, double* epart, hipStream_t s) {
    const uint64_t N = 1ull << n;
    const uint64_t gx = hpsi_blocks(n);
    const dim3 g((uint32_t)gx, (uint32_t)batch);
    if (n >= kHB && pd.gm && pd.hz && pd.hc && pd.hm) {
        if (dtype == 1)
            hipLaunchKernelGGL(k_hpsi_tile<float>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<float>*>(psi),
                               reinterpret_cast<V2<float>*>(lam), bstride, pd, epart);
        else
            hipLaunchKernelGGL(k_hpsi_tile<double>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<double>*>(psi),
                               reinterpret_cast<V2<double>*>(lam), bstride, pd, epart);
        return hipGetLastError();
    }
    if (n >= kHB) return hipErrorInvalidValue;   // the tiled kernel's tables are missing
    if (dtype == 1)
        hipLaunchKernelGGL(k_hpsi<float>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<float>*>(psi),
                           reinterpret_cast<V2<float>*>(lam), bstride, N, pd, epart);
    else
        hipLaunchKernelGGL(k_hpsi<double>, g, dim3(kRB), 0, s, reinterpret_cast<const V2<double>*>(psi),
                           reinterpret_cast<V2<double>*>(lam), bstride, N, pd, epart);
    return hipGetLastError();
}

}  // namespace svmi
