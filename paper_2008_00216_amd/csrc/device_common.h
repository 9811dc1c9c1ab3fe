// Shared device helpers for the HIP kernels (gfx950).  Also compiled at run
// time by hiprtc for plan-specialised tile passes, so it avoids host headers
// when __HIPCC_RTC__ is defined.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
typedef unsigned char uint8_t;
typedef unsigned short uint16_t;
typedef unsigned int uint32_t;
typedef int int32_t;
typedef unsigned long long uint64_t;
typedef long long int64_t;
#endif

namespace svmi {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class R>
struct alignas(2 * sizeof(R)) V2 {
    R x, y;
};

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc += u * v (complex)
template <class R>
__device__ __forceinline__ void cmac(V2<R>& acc, V2<R> u, V2<R> v) {
    acc.x = fma_(u.x, v.x, acc.x);
    acc.x = fma_(-u.y, v.y, acc.x);
    acc.y = fma_(u.x, v.y, acc.y);
    acc.y = fma_(u.y, v.x, acc.y);
}

template <class R>
__device__ __forceinline__ V2<R> cmul(V2<R> u, V2<R> v) {
    V2<R> r;
    r.x = fma_(-u.y, v.y, u.x * v.x);
    r.y = fma_(u.y, v.x, u.x * v.y);
    return r;
}

// Deposit the low bits of l into the set bits of MASK (compile time).
__host__ __device__ constexpr int dep4(int mask, int l) {
    int out = 0, t = 0;
    for (int b = 0; b < 4; ++b)
        if ((mask >> b) & 1) {
            if ((l >> t) & 1) out |= 1 << b;
            ++t;
        }
    return out;
}

// Extract the MASK bits of i into a dense index (compile time).
__host__ __device__ constexpr int ext4(int mask, int i) {
    int out = 0, t = 0;
    for (int b = 0; b < 4; ++b)
        if ((mask >> b) & 1) {
            if ((i >> b) & 1) out |= 1 << t;
            ++t;
        }
    return out;
}

// XOR-linear LDS swizzle (amplitude units).  It only flips low index bits
// as a function of higher bits, so swz(a ^ b) == swz(a) ^ swz(b); the c64
// variant keeps bit 0 so that the two amplitudes of a 16-byte chunk stay
// adjacent.  For c64, bits 1..4 (the bank within a 128-byte row) are mixed
// with bits 4..8: a register phase inserts its four slot bits among the
// thread-index bits, and mixing in the bits just above the bank bits spreads
// the 16-lane groups of its ds_read_b64 / ds_write_b64 over all 32 banks for
// almost every choice of slot positions.
template <class R>
__host__ __device__ inline constexpr uint32_t swz(uint32_t l);
template <>
__host__ __device__ inline constexpr uint32_t swz<float>(uint32_t l) {
    return l ^ ((((l >> 4) ^ (l >> 5)) & 15u) << 1);
}
template <>
__host__ __device__ inline constexpr uint32_t swz<double>(uint32_t l) {
    return l ^ (((l >> 4) ^ (l >> 8) ^ (l >> 12)) & 15u);
}

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// One DPP move of both halves of a double (every lane active; the patterns
// used here read lanes of the same row only).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    // every lane has a source lane under the controls used here (quad
    // permutes, row rotations), so no old value is needed
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// DPP moves into the rows of ROW_MASK only (the lanes of the other rows read
// 0), of a float and of both halves of a double.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_rows(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_rows(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave (all lanes active), complete in lane 63
// only: each row of 16 lanes is summed (swaps within quads, rotations by 4
// and 8 lanes), then row 1 adds the sum of row 0 and row 3 that of row 2
// (row_bcast:15), and rows 2 and 3 add the sum of rows 0 and 1
// (row_bcast:31).  No lane reads; the lanes of the other rows add 0.
template <class T>
__device__ __forceinline__ T wave_sum_lane63(T v) {
    v += dpp_rows<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += dpp_rows<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += dpp_rows<0x124, 0xF>(v);   // row_ror:4
    v += dpp_rows<0x128, 0xF>(v);   // row_ror:8
    v += dpp_rows<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_rows<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

// Sum over the 64 lanes of a wave (all lanes active), in every lane: each
// row of 16 lanes is summed with DPP (swaps within quads, then rotations by 4
// and 8 lanes), and the four row sums are read with readlane.  No LDS round
// trips, unlike a shuffle tree.
__device__ __forceinline__ double wave_sum64(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x124>(v);   // row_ror:4
    v += dpp_f64<0x128>(v);   // row_ror:8
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// 1/sqrt(2) = cos(pi/4), the state dtype's rounding of its double value
template <class R>
constexpr R kSqrtHalf = R(0.70710678118654752440);

// Plan data (op lists, matrix pools, pair masks) is written before a launch
// and only read by kernels.  Reading it through a constant-address-space
// pointer lets wave-uniform reads become scalar loads into SGPRs instead of
// vector loads into every lane.
template <class T>
using cptr_t = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ cptr_t<T> cptr(const T* p) {
    return (cptr_t<T>)p;
}
// Element-wise loads that accept generic and constant-space pointers alike.
template <class R>
__device__ __forceinline__ V2<R> ldv(const V2<R>* p) {
    return *p;
}
template <class R>
__device__ __forceinline__ V2<R> ldv(cptr_t<V2<R>> p) {
    return V2<R>{p->x, p->y};
}

// Flip the sign of both parts of an amplitude when bit 31 of `m` is set (exact).
__device__ __forceinline__ void sign_flip_mask(V2<float>& a, uint32_t m) {
    a.x = __uint_as_float(__float_as_uint(a.x) ^ m);
    a.y = __uint_as_float(__float_as_uint(a.y) ^ m);
}
__device__ __forceinline__ void sign_flip_mask(V2<double>& a, uint32_t m) {
    const long long mm = (long long)((unsigned long long)m << 32);
    a.x = __longlong_as_double(__double_as_longlong(a.x) ^ mm);
    a.y = __longlong_as_double(__double_as_longlong(a.y) ^ mm);
}
__device__ __forceinline__ void sign_flip(V2<float>& a, uint32_t flip) { sign_flip_mask(a, flip << 31); }
__device__ __forceinline__ void sign_flip(V2<double>& a, uint32_t flip) { sign_flip_mask(a, flip << 31); }

}  // namespace svmi
