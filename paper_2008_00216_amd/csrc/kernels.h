// Host-side launch interface of the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"
#include "tile_frame.h"

namespace svmi {

// Fixed device work area of the allocation-free entry point: a file-scope
// __device__ array of this many bytes per GPU, held until the process ends.
// static_scratch() returns its device address on the current device (looked
// up once per device with hipGetSymbolAddress); never pass the array's name.
constexpr size_t kStaticScratchBytes = 4u << 20;
hipError_t static_scratch(void** ptr);

// Schroedinger-Feynman path sum: acc[k] (+)= sum_{s < npath} A[(s << nA) | jA[k]] *
// B[(s << nB) | jB[k]] in FP64 (acc: count interleaved complex doubles).
hipError_t launch_sf_contract(int dtype, const void* A, const void* B, int nA, int nB, uint64_t npath,
                              const uint64_t* jA, const uint64_t* jB, uint64_t count, double* acc, int accumulate,
                              hipStream_t s);

// The paper's own plan (ablation).  Diagonal cluster in one pass: amplitude j
// times e^{i pi e/4}, e = popc(j&e8[0]) + 2 popc(j&e8[1]) + 4 popc(j&e8[2]) +
// 4 (CZ parity from the one-sided masks d_m1s; d_msym the symmetric ones),
// both device arrays of n masks.
hipError_t launch_pp_diag(int dtype, void* state, uint64_t bstride, int batch, int n, const uint64_t* e8,
                          const uint64_t* d_m1s, const uint64_t* d_msym, hipStream_t s);
// Unnormalised factor ga on qubit qa and gb on qb (gb < 0: ga alone), one pass.
hipError_t launch_pp_pair(int dtype, void* state, uint64_t bstride, int batch, int n, int qa, int ga, int qb, int gb,
                          hipStream_t s);
// nops (<= 32) pairs / single gates on qubits < C over chunks of 2^C contiguous amplitudes in LDS.
hipError_t launch_pp_chunk(int dtype, void* state, uint64_t bstride, int batch, int n, int C, int nops,
                           const int* qa, const int* ga, const int* qb, const int* gb, hipStream_t s);
// Every amplitude times (re + i im).
hipError_t launch_pp_scale(int dtype, void* state, uint64_t bstride, int batch, int n, double re, double im,
                           hipStream_t s);

// Dynamic LDS bytes a tile pass needs.
size_t tile_lds_bytes(int dtype, bool two, uint32_t T, uint32_t nform, uint32_t ngrad, int nt);
hipError_t launch_tile_pass(int dtype, bool two, int nt, const TileArgs& a, uint64_t nblocks,
                            size_t lds, hipStream_t s);
hipError_t tile_pass_set_attrs(size_t max_lds);

// Plain (one kernel per gate) kernels; `batch` states spaced `bstride` amplitudes.
// Dense k-qubit gate on ascending qubits tq[0..k), matrix row-major in that order.
// K = 5, 6 dense gates on MFMA (complex64: n >= 12, FP32 tiles; complex128:
// n >= 11, FP64 tiles); ascending targets.
bool mfma_dense_supported(int dtype, int n, int k);
hipError_t launch_dense_mfma(int dtype, void* state, uint64_t bstride, int batch, int n, int k, const int* tq,
                             const void* mat, uint64_t mat_bstride, hipStream_t s);
hipError_t launch_dense_plain(int dtype, void* state, uint64_t bstride, int batch, int n, int k,
                             const int* tq, const void* mat, uint64_t mat_bstride, hipStream_t s);
// Multiply every amplitude whose index has all bits of `mask` set by the
// complex value at `val` (per state, spaced val_bstride); mode 0 general,
// 1 sign flip (exact), 2 multiply by +i (exact), 3 by -i (exact).
hipError_t launch_masked_phase(int dtype, void* state, uint64_t bstride, int batch, int n,
                               uint64_t mask, int mode, const void* val, uint64_t val_bstride,
                               hipStream_t s);
// Diagonal on ascending qubits tq[0..k): amplitude j times d[loc(j)].
hipError_t launch_diag_plain(int dtype, void* state, uint64_t bstride, int batch, int n, int k,
                             const int* tq, const void* d, uint64_t d_bstride, hipStream_t s);
// Exact pair permutation: for every index j with bits `zero_mask` clear and
// `one_mask` set, exchange amplitudes j and j ^ flip.  mode 0: plain swap,
// mode 1: Y-type swap (a0, a1) -> (-i a1, i a0).
hipError_t launch_pair_swap(int dtype, void* state, uint64_t bstride, int batch, int n,
                            uint64_t zero_mask, uint64_t one_mask, uint64_t flip, int mode,
                            hipStream_t s);

// Initialisation.  kind: 0 zero, 1 basis(index), 2 uniform(value).
// dst[0, bytes) = src[0, bytes) (both 16-byte aligned, bytes a multiple of 16).
hipError_t launch_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s);
hipError_t launch_init(int dtype, void* state, uint64_t bstride, int batch, int n, int kind,
                       uint64_t index, double value, hipStream_t s);
// Product state psi[j] = lo[j & (2^nlo - 1)] * hi[j >> nlo] (FP64 tables).
hipError_t launch_init_product(int dtype, void* state, uint64_t bstride, int batch, int n,
                               int nlo, const double* lo, const double* hi, hipStream_t s);

// FP64 reductions.  Partials need reduce_partials_size(...) doubles.
size_t reduce_partials_size(int n, int batch);
// kind 0: ||psi||^2; kind 1: Re<a|b> (b = second); kind 2: Pauli-sum
// expectation; kind 3: Im<b|G|a> for a one/two-qubit generator G (gen,
// qubit mask gmask) -- the adjoint gradient term with a = psi, b = lambda.
// out[s * out_stride] receives state s's value.
struct PauliDev {
    const uint64_t* x;        // distinct x masks [ngroup]
    const uint32_t* g0;       // first term of each group [ngroup + 1]
    const uint64_t* z;        // z mask per term
    const double* c;          // coefficient per term
    const uint32_t* ph;       // i^{|x&z|} exponent per term
    uint32_t ngroup;
    // Tables of the tiled lambda = H psi kernel (null unless requested).
    // Within each group the terms with an even phase exponent come first,
    // up to gm[g]; per term in that order: hz = z mask, hc = coefficient
    // times the real sign of i^ph (so the term is hc, or i hc for odd ph),
    // hm bit k (k < 8) = parity of (z >> 8) & k.
    const uint32_t* gm;
    const uint64_t* hz;
    const double* hc;
    const uint32_t* hm;
};
hipError_t launch_reduce(int dtype, int kind, const void* a, const void* b, uint64_t bstride,
                         int batch, int n, const PauliDev* pd, int gen, uint64_t gmask,
                         double* partials, double* out, uint64_t out_stride, hipStream_t s);
// Measurement sampling by descent of a 64-ary FP64 tree of probability
// masses.  sample_levels(n) = K tree levels above the amplitudes; the tree
// takes sample_tree_doubles(n, batch) doubles.  out[b * count + k] = the
// smallest j whose prefix of |psi_b|^2 (tree order) exceeds
// uniforms[b * count + k] * (total mass of psi_b).
int sample_levels(int n);
uint64_t sample_tree_doubles(int n, int batch);
hipError_t launch_sample(int dtype, const void* a, uint64_t bstride, int batch, int n, double* tree,
                         const double* uniforms, uint64_t count, uint64_t* out, hipStream_t s);
hipError_t launch_gather(int dtype, const void* a, uint64_t bstride, int batch, const uint64_t* idx, uint64_t count,
                         double* out, hipStream_t s);

// lambda = H psi (FP64 accumulation, rounded once).  With epart (batch *
// hpsi_blocks(n) doubles) the blocks also leave their FP64 partials of
// Re <psi|lambda>, to be summed by launch_grad_reduce with nslot = 1.
uint64_t hpsi_blocks(int n);
hipError_t launch_hpsi(int dtype, const void* psi, void* lam, uint64_t bstride, int batch, int n,
                       const PauliDev& pd, double* epart, hipStream_t s);
// out[b * out_stride + j] = sum_t part[(b * ntile + t) * nslot + j] in a
// fixed order (chunks of tiles, then the chunk sums); part is overwritten.
hipError_t launch_grad_reduce(double* part, int batch, uint64_t ntile, uint32_t nslot,
                              double* out, uint64_t out_stride, hipStream_t s);

// Tasks {const double* src; uint64 ntile; uint32 nslot; uint32 pad; double* dst}:
// dst[j] = sum over t (ascending) of src[t * nslot + j]; one block per task.
hipError_t launch_multi_sum(const void* tasks, uint32_t ntask, hipStream_t s);

}  // namespace svmi
