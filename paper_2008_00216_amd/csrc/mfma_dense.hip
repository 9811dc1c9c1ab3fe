// Dense gates on K = 5 or 6 qubits in complex64 on the matrix cores.
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

}  // namespace

bool mfma_dense_supported(int dtype, int n, int k) {
    return dtype == 1 && (k == 5 || k == 6) && n >= 12;   // at least one chunk of 4096 amplitudes
}

hipError_t launch_dense_mfma(void* state, uint64_t bstride, int batch, int n, int k, const int* tq, const void* mat,
                             uint64_t mat_bstride, hipStream_t s) {
    MTargets tg{};
    for (int t = 0; t < k; ++t) tg.q[t] = tq[t];
    const uint64_t nsets = 1ull << (n - k);
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
