// Tiled lambda = H psi for a Pauli sum (Sec. 3's matrix-vector product
// with the observable, for the adjoint sweep): the body of one workgroup of
// 256 threads on a 2^11-amplitude tile.
#pragma once
#include "device_common.h"
#include "kernels.h"

namespace svmi {

constexpr int kHB = 11;                     // tile bits
constexpr int kHT = 256;                    // threads per workgroup
constexpr int kHK = (1 << kHB) / kHT;       // amplitudes per thread

__device__ __forceinline__ double flip_sign(double v, uint32_t bit) {
    return __longlong_as_double(__double_as_longlong(v) ^ ((long long)(bit & 1u) << 63));
}

// lambda = H psi on amplitudes t0 .. t0 + 2^11 - 1 of the state at p (t0 a
// multiple of 2^11; the state has at least 2^11 amplitudes), written to
// lam (none when lam is null).  Thread `tid` holds amplitudes
// t0 + k 256 + tid (k < 8), and the tile sits in LDS (`tile`, 2^11
// entries), so a group whose x mask stays below bit 11 reads its partners
// there; other groups load them from global memory.  For a group with mask
// x the partner of amplitude k has index jx = (t0 ^ x) with bits 8..10 xor k
// and bits 0..7 = (tid ^ x) & 255, so the sign (-1)^{|z & jx|} of a term
// splits into a per-lane factor (bits 0..7), a compile-time factor per k
// (bits 8..10, the table hm) and a block-uniform factor (bits >= 8 of
// t0 ^ x) computed on the scalar unit.  Per group the terms add up to one
// complex diagonal value D_k per amplitude, and lambda gains D_k times the
// partner.  Accumulation is FP64; lambda is rounded once.  Returns the
// thread's share of Re <psi|lambda> over the tile, from lambda before
// rounding, or from the rounded lambda with `rounded_energy`.  Needs the
// tables gm, hz, hc, hm of `pd`; ends with a barrier, so the tile can be
// reused at once.
template <class R>
__device__ __forceinline__ double hpsi_tile11(const V2<R>* __restrict__ p, V2<R>* __restrict__ lam, uint64_t t0,
                                              const PauliDev& pd, V2<R>* tile, bool rounded_energy) {
    const uint32_t tid = threadIdx.x;
    V2<R> v[kHK];
#pragma unroll
    for (int k = 0; k < kHK; ++k) {
        v[k] = p[t0 + (uint32_t)k * kHT + tid];
        tile[k * kHT + tid] = v[k];
    }
    __syncthreads();
    double lr[kHK], li[kHK];
#pragma unroll
    for (int k = 0; k < kHK; ++k) { lr[k] = 0.0; li[k] = 0.0; }
    const cptr_t<uint64_t> X = cptr(pd.x);
    const cptr_t<uint32_t> G0 = cptr(pd.g0);
    const cptr_t<uint32_t> GM = cptr(pd.gm);
    const cptr_t<uint64_t> HZ = cptr(pd.hz);
    const cptr_t<double> HC = cptr(pd.hc);
    const cptr_t<uint32_t> HM = cptr(pd.hm);
    for (uint32_t g = 0; g < pd.ngroup; ++g) {
        const uint64_t x = X[g];
        V2<R> w[kHK];
        if (x == 0) {
#pragma unroll
            for (int k = 0; k < kHK; ++k) w[k] = v[k];
        } else if ((x >> kHB) == 0) {
#pragma unroll
            for (int k = 0; k < kHK; ++k) w[k] = tile[((uint32_t)k * kHT + tid) ^ (uint32_t)x];
        } else {
#pragma unroll
            for (int k = 0; k < kHK; ++k) w[k] = p[(t0 + (uint32_t)k * kHT + tid) ^ x];
        }
        const uint32_t xl = (tid ^ (uint32_t)x) & 255u;
        const uint64_t xu = (t0 ^ x) & ~255ull;
        double dr[kHK], di[kHK];
#pragma unroll
        for (int k = 0; k < kHK; ++k) { dr[k] = 0.0; di[k] = 0.0; }
        const uint32_t ta = G0[g], tm = GM[g], te = G0[g + 1];
        for (uint32_t t = ta; t < tm; ++t) {
            const uint64_t z = HZ[t];
            const double c = HC[t];
            const uint32_t pm = HM[t];
            const uint32_t u = (uint32_t)__popcll(z & xu);
            const uint32_t lp = (uint32_t)__popc(xl & (uint32_t)z);
            const double ls = __longlong_as_double((long long)(0x3FF00000u | (lp << 31)) << 32);
#pragma unroll
            for (int k = 0; k < kHK; ++k) dr[k] = fma(ls, flip_sign(c, (pm >> k) ^ u), dr[k]);
        }
        for (uint32_t t = tm; t < te; ++t) {
            const uint64_t z = HZ[t];
            const double c = HC[t];
            const uint32_t pm = HM[t];
            const uint32_t u = (uint32_t)__popcll(z & xu);
            const uint32_t lp = (uint32_t)__popc(xl & (uint32_t)z);
            const double ls = __longlong_as_double((long long)(0x3FF00000u | (lp << 31)) << 32);
#pragma unroll
            for (int k = 0; k < kHK; ++k) di[k] = fma(ls, flip_sign(c, (pm >> k) ^ u), di[k]);
        }
#pragma unroll
        for (int k = 0; k < kHK; ++k) {
            const double wr = w[k].x, wi = w[k].y;
            lr[k] = fma(dr[k], wr, fma(-di[k], wi, lr[k]));
            li[k] = fma(dr[k], wi, fma(di[k], wr, li[k]));
        }
    }
    double e = 0.0;
#pragma unroll
    for (int k = 0; k < kHK; ++k) {
        const V2<R> lv{R(lr[k]), R(li[k])};
        if (lam) lam[t0 + (uint32_t)k * kHT + tid] = lv;
        if (rounded_energy) e += (double)v[k].x * (double)lv.x + (double)v[k].y * (double)lv.y;
        else e += (double)v[k].x * lr[k] + (double)v[k].y * li[k];
    }
    __syncthreads();
    return e;
}

}  // namespace svmi
