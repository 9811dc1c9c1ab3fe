// Path-sum contraction of the Schroedinger-Feynman mode: every requested
// amplitude is the sum over cut paths s of A_s[jA] * B_s[jB], where A_s and
// B_s are the two half states of path s (stored path-major: the path index
// occupies the high index bits of each half's buffer).  FP64 accumulation.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace svmi {

namespace {

constexpr int kSB = 256;                 // 4 waves, one requested amplitude per wave

template <class R>
__global__ __launch_bounds__(kSB) void k_sf_contract(const V2<R>* __restrict__ A, const V2<R>* __restrict__ B,
                                                     uint32_t nA, uint32_t nB, uint64_t npath,
                                                     const uint64_t* __restrict__ jA, const uint64_t* __restrict__ jB,
                                                     uint64_t count, double2* __restrict__ acc, int accumulate) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t k = (uint64_t)blockIdx.x * (kSB / 64) + (threadIdx.x >> 6);
    if (k >= count) return;              // whole waves leave together
    const uint64_t a0 = jA[k], b0 = jB[k];
    double re = 0.0, im = 0.0;
    for (uint64_t s = lane; s < npath; s += 64) {
        const V2<R> a = A[(s << nA) | a0];
        const V2<R> b = B[(s << nB) | b0];
        const double ar = a.x, ai = a.y, br = b.x, bi = b.y;
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
    }
    if (lane == 0) {
        double2 v = make_double2(re, im);
        if (accumulate) {
            const double2 o = acc[k];
            v.x += o.x;
            v.y += o.y;
        }
        acc[k] = v;
    }
}

}  // namespace

hipError_t launch_sf_contract(int dtype, const void* A, const void* B, int nA, int nB, uint64_t npath,
                              const uint64_t* jA, const uint64_t* jB, uint64_t count, double* acc, int accumulate,
                              hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint64_t nblk = (count + kSB / 64 - 1) / (kSB / 64);
    if (nblk > 0x7fffffffull) return hipErrorInvalidValue;
    const dim3 g((uint32_t)nblk);
    if (dtype == 1)
        hipLaunchKernelGGL(k_sf_contract<float>, g, dim3(kSB), 0, s, reinterpret_cast<const V2<float>*>(A),
                           reinterpret_cast<const V2<float>*>(B), (uint32_t)nA, (uint32_t)nB, npath, jA, jB, count,
                           reinterpret_cast<double2*>(acc), accumulate);
    else
        hipLaunchKernelGGL(k_sf_contract<double>, g, dim3(kSB), 0, s, reinterpret_cast<const V2<double>*>(A),
                           reinterpret_cast<const V2<double>*>(B), (uint32_t)nA, (uint32_t)nB, npath, jA, jB, count,
                           reinterpret_cast<double2*>(acc), accumulate);
    return hipGetLastError();
}

}  // namespace svmi
