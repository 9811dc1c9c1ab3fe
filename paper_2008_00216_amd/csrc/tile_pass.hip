// Fused tile pass: the hot loop of the sweep (runtime-interpreted op list).
//
// One workgroup owns one tile: the 2^T amplitudes whose indices agree on all
// non-local bits.  The local bits are the L lowest index bits (contiguous in
// memory, so a tile is 2^H segments of 2^L amplitudes) plus H higher bits.
// This is the GPU counterpart of the paper's cache blocking (Sec. 5.1): all
// gates that act on local qubits are applied while the tile is on chip, so
// each pass costs one read and one write of the state.
//
// Inside the tile, a register phase hands every thread the 16 amplitudes that
// differ in 4 register slots and applies the phase's op list in registers
// (tile_ops.h).  This kernel reads the op list from memory; the planner can
// instead emit a plan-specialised kernel per pass (jit.cpp) where every slot
// and table is a compile-time constant.
#include "device_common.h"
#include "kernels.h"
#include "tile_frame.h"
#include "tile_ops.h"

#include "tile_interp.h"

namespace svmi {

template <class R, int NT, bool TWO>
__global__ __launch_bounds__(NT) void k_tile(TileArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    tile_interp<R, NT, TWO>(A, smem, blockIdx.x);
}

size_t tile_lds_bytes(int dtype, bool two, uint32_t T, uint32_t nform, uint32_t ngrad, int nt) {
    const size_t amp = dtype == 1 ? 8 : 16;
    size_t bytes = (two ? 2 : 1) * ((size_t)1 << T) * amp + 8 * amp;
    bytes += 4 * (((4 * (size_t)nform + 1) & ~(size_t)1));
    if (two) bytes += 8 * (size_t)ngrad * (nt / 64);
    bytes += 8 * (size_t)(nt / 64);   // per-wave norm sums (one-state passes that return the norm)
    return (bytes + 15) & ~(size_t)15;
}

template <class R, int NT, bool TWO>
static hipError_t launch_one(const TileArgs& a, uint64_t nblocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_tile<R, NT, TWO>), dim3((uint32_t)nblocks), dim3(NT), lds, s, a);
    return hipGetLastError();
}

hipError_t tile_pass_set_attrs(size_t max_lds) {
    const void* fns[] = {
        (const void*)&k_tile<float, 256, false>, (const void*)&k_tile<float, 256, true>,
        (const void*)&k_tile<float, 512, false>, (const void*)&k_tile<float, 512, true>,
        (const void*)&k_tile<double, 256, false>, (const void*)&k_tile<double, 256, true>,
        (const void*)&k_tile<double, 512, false>, (const void*)&k_tile<double, 512, true>,
    };
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_tile_pass(int dtype, bool two, int nt, const TileArgs& a, uint64_t nblocks,
                            size_t lds, hipStream_t s) {
    if (dtype == 1) {
        if (nt == 256) return two ? launch_one<float, 256, true>(a, nblocks, lds, s)
                                  : launch_one<float, 256, false>(a, nblocks, lds, s);
        return two ? launch_one<float, 512, true>(a, nblocks, lds, s)
                   : launch_one<float, 512, false>(a, nblocks, lds, s);
    }
    if (nt == 256) return two ? launch_one<double, 256, true>(a, nblocks, lds, s)
                              : launch_one<double, 256, false>(a, nblocks, lds, s);
    return two ? launch_one<double, 512, true>(a, nblocks, lds, s)
               : launch_one<double, 512, false>(a, nblocks, lds, s);
}

}  // namespace svmi
