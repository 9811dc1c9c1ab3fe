// Dense gates on K = 5 or 6 qubits on the matrix cores (complex64: FP32
// MFMA; complex128: FP64 MFMA).
//
// A K-qubit gate updates each of the 2^{n-K} amplitude sets (Sec. 3) with the
// same 2^K x 2^K matrix U, so a chunk of C sets is the product Y = U X of U
// with the 2^K x C matrix X whose column c holds the amplitudes of set c.
// At 8 * 2^K flops per amplitude these are the only gates of the path whose
// arithmetic outweighs their memory traffic, and they run as a real FP32
// GEMM on MFMA:
//     [Re Y; Im Y] = [[Re U, -Im U], [Im U, Re U]] [Re X; Im X]
// (a 2^{K+1} x 2^{K+1} real matrix), with v_mfma_f32_32x32x2f32 tiles.
//
// One workgroup (8 waves) holds a chunk of 4096 amplitudes in LDS as separate
// real and imaginary planes X[comp][row][col]; wave w computes the 32 x 32
// output tile (row block w % RB, column block w / RB).  Its 32 rows of the
// real-expanded matrix stay in registers for all chunks the workgroup visits.
#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace svmi {

namespace {

constexpr int kMT = 512;   // 8 waves

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint64_t ins_zeros(uint64_t s, const int* tq, int k) {
    for (int t = 0; t < k; ++t) {
        const int p = tq[t];
        s = ((s >> p) << (p + 1)) | (s & ((1ull << p) - 1ull));
    }
    return s;
}

struct MTargets {
    int q[6];
};

template <int K>
__global__ __launch_bounds__(kMT) void k_dense_mfma(V2<float>* state, uint64_t bstride, MTargets tg,
                                                    const V2<float>* __restrict__ mat, uint64_t mat_bstride,
                                                    uint64_t nchunks) {
    constexpr int D = 1 << K;            // amplitude rows
    constexpr int R2 = 2 * D;            // real-expanded rows = contraction length
    constexpr int C = 4096 / D;          // sets per chunk
    constexpr int RB = R2 / 32;          // row blocks
    constexpr int STEPS = R2 / 2;        // MFMA steps (k = 2 each)
    static_assert(RB * (C / 32) == kMT / 64, "one 32x32 output tile per wave");
    __shared__ float X[2][D][C];         // [re/im][row][set]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rb = wave % RB, cb = wave / RB;
    const uint32_t b = blockIdx.y;
    V2<float>* psi = state + (uint64_t)b * bstride;
    const V2<float>* u = mat + (uint64_t)b * mat_bstride;

    // this wave's rows of the real-expanded matrix: A[i][k], i = rb*32 + lane%32,
    // k = 2*s + lane/32
    float a[STEPS];
    {
        const int i = rb * 32 + (lane & 31);
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            const int k = 2 * s + (lane >> 5);
            const V2<float> m = u[(i & (D - 1)) * D + (k & (D - 1))];
            const bool ilo = i < D, klo = k < D;
            a[s] = ilo ? (klo ? m.x : -m.y) : (klo ? m.y : m.x);
        }
    }
    uint64_t rowoff[4096 / kMT];
#pragma unroll
    for (int e = 0; e < 4096 / kMT; ++e) {
        const int r = (e * kMT + tid) / C;
        uint64_t o = 0;
#pragma unroll
        for (int t = 0; t < K; ++t)
            if ((r >> t) & 1) o |= 1ull << tg.q[t];
        rowoff[e] = o;
    }

    for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const uint64_t set0 = ch * C;
        // gather: element e -> (row r, set c), consecutive threads on consecutive sets
#pragma unroll
        for (int e = 0; e < 4096 / kMT; ++e) {
            const int idx = e * kMT + tid;
            const int r = idx / C, c = idx % C;
            const V2<float> v = psi[ins_zeros(set0 + c, tg.q, K) | rowoff[e]];
            X[0][r][c] = v.x;
            X[1][r][c] = v.y;
        }
        __syncthreads();
        f32x16 acc;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
        const int col = cb * 32 + (lane & 31);
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            const int k = 2 * s + (lane >> 5);
            const float bv = X[k >> K][k & (D - 1)][col];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], bv, acc, 0, 0, 0);
        }
        __syncthreads();   // every wave has read X
        // output tile: lane holds column lane%32, rows (j/4)*8 + (lane/32)*4 + j%4
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int i = rb * 32 + (j >> 2) * 8 + (lane >> 5) * 4 + (j & 3);
            X[i >> K][i & (D - 1)][col] = acc[j];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4096 / kMT; ++e) {
            const int idx = e * kMT + tid;
            const int r = idx / C, c = idx % C;
            psi[ins_zeros(set0 + c, tg.q, K) | rowoff[e]] = V2<float>{X[0][r][c], X[1][r][c]};
        }
        __syncthreads();   // X is reused by the next chunk
    }
}

// The same product in complex128 with v_mfma_f64_16x16x4f64 tiles.  A chunk
// holds 2048 amplitudes (32 KiB of FP64 planes in LDS); the real-expanded
// output (2^{K+1} rows x C sets) is 16 tiles of 16 x 16, two per wave, both
// in one row block so that the wave's rows of the real-expanded matrix
// (held in registers for all chunks) serve both.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int K>
__global__ __launch_bounds__(kMT) void k_dense_mfma64(V2<double>* state, uint64_t bstride, MTargets tg,
                                                      const V2<double>* __restrict__ mat, uint64_t mat_bstride,
                                                      uint64_t nchunks) {
    constexpr int D = 1 << K;            // amplitude rows
    constexpr int R2 = 2 * D;            // real-expanded rows = contraction length
    constexpr int NA = 2048;             // amplitudes per chunk
    constexpr int C = NA / D;            // sets per chunk
    constexpr int RB = R2 / 16;          // row blocks of 16
    constexpr int STEPS = R2 / 4;        // MFMA steps (k = 4 each)
    constexpr int NG = (kMT / 64) / RB;  // column groups (waves per row block)
    constexpr int CPG = (C / 16) / NG;   // column blocks per wave
    static_assert(CPG == 2 && RB * NG == kMT / 64, "two 16x16 output tiles per wave");
    __shared__ double X[2][D][C];        // [re/im][row][set]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rb = wave % RB, cg = wave / RB;
    const uint32_t b = blockIdx.y;
    V2<double>* psi = state + (uint64_t)b * bstride;
    const V2<double>* u = mat + (uint64_t)b * mat_bstride;

    // A operand of step s: lane holds A[i][k], i = rb*16 + lane%16,
    // k = 4*s + lane/16
    double a[STEPS];
    {
        const int i = rb * 16 + (lane & 15);
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            const int k = 4 * s + (lane >> 4);
            const V2<double> m = u[(i & (D - 1)) * D + (k & (D - 1))];
            const bool ilo = i < D, klo = k < D;
            a[s] = ilo ? (klo ? m.x : -m.y) : (klo ? m.y : m.x);
        }
    }
    uint64_t rowoff[NA / kMT];
#pragma unroll
    for (int e = 0; e < NA / kMT; ++e) {
        const int r = (e * kMT + tid) / C;
        uint64_t o = 0;
#pragma unroll
        for (int t = 0; t < K; ++t)
            if ((r >> t) & 1) o |= 1ull << tg.q[t];
        rowoff[e] = o;
    }

    for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const uint64_t set0 = ch * C;
#pragma unroll
        for (int e = 0; e < NA / kMT; ++e) {
            const int idx = e * kMT + tid;
            const int r = idx / C, c = idx % C;
            const V2<double> v = psi[ins_zeros(set0 + c, tg.q, K) | rowoff[e]];
            X[0][r][c] = v.x;
            X[1][r][c] = v.y;
        }
        __syncthreads();
        f64x4 acc[CPG];
#pragma unroll
        for (int t = 0; t < CPG; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[t][j] = 0.0;
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            const int k = 4 * s + (lane >> 4);
#pragma unroll
            for (int t = 0; t < CPG; ++t) {
                const int col = (cg * CPG + t) * 16 + (lane & 15);
                const double bv = X[k >> K][k & (D - 1)][col];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bv, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();   // every wave has read X
        // output tile: lane holds column lane%16, rows lane/16 + 4*j
        // (the FP64 tile interleaves its rows over the registers)
#pragma unroll
        for (int t = 0; t < CPG; ++t) {
            const int col = (cg * CPG + t) * 16 + (lane & 15);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = rb * 16 + (lane >> 4) + 4 * j;
                X[i >> K][i & (D - 1)][col] = acc[t][j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < NA / kMT; ++e) {
            const int idx = e * kMT + tid;
            const int r = idx / C, c = idx % C;
            psi[ins_zeros(set0 + c, tg.q, K) | rowoff[e]] = V2<double>{X[0][r][c], X[1][r][c]};
        }
        __syncthreads();   // X is reused by the next chunk
    }
}

}  // namespace

bool mfma_dense_supported(int dtype, int n, int k) {
    if (k != 5 && k != 6) return false;
    // at least one chunk: 4096 amplitudes (complex64) or 2048 (complex128)
    return dtype == 1 ? n >= 12 : n >= 11;
}

hipError_t launch_dense_mfma(int dtype, void* state, uint64_t bstride, int batch, int n, int k, const int* tq,
                             const void* mat, uint64_t mat_bstride, hipStream_t s) {
    if (!mfma_dense_supported(dtype, n, k)) return hipErrorInvalidValue;
    MTargets tg{};
    for (int t = 0; t < k; ++t) tg.q[t] = tq[t];
    const uint64_t nsets = 1ull << (n - k);
    if (dtype != 1) {
        const uint64_t nchunks = nsets / (2048ull >> k);
        const uint32_t grid = (uint32_t)std::min<uint64_t>(nchunks, 4096);
        auto* st = reinterpret_cast<V2<double>*>(state);
        auto* m = reinterpret_cast<const V2<double>*>(mat);
        if (k == 5)
            hipLaunchKernelGGL(k_dense_mfma64<5>, dim3(grid, (uint32_t)batch), dim3(kMT), 0, s, st, bstride, tg, m,
                               mat_bstride, nchunks);
        else
            hipLaunchKernelGGL(k_dense_mfma64<6>, dim3(grid, (uint32_t)batch), dim3(kMT), 0, s, st, bstride, tg, m,
                               mat_bstride, nchunks);
        return hipGetLastError();
    }
    const uint64_t C = 4096ull >> k;
    const uint64_t nchunks = nsets / C;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(nchunks, 4096);
    auto* st = reinterpret_cast<V2<float>*>(state);
    auto* m = reinterpret_cast<const V2<float>*>(mat);
    if (k == 5)
        hipLaunchKernelGGL(k_dense_mfma<5>, dim3(grid, (uint32_t)batch), dim3(kMT), 0, s, st, bstride, tg, m,
                           mat_bstride, nchunks);
    else if (k == 6)
        hipLaunchKernelGGL(k_dense_mfma<6>, dim3(grid, (uint32_t)batch), dim3(kMT), 0, s, st, bstride, tg, m,
                           mat_bstride, nchunks);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace svmi
