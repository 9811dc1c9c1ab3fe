// Heterogeneous batch in one persistent launch.
//
// Every item (a circuit of its own width, its state, optional lambda scratch
// and observable) is split into stages: [zero init], forward tile passes,
// lambda = H psi with the energy partials (or the energy alone), [backward
// tile passes with gradient partials].  A stage is a set of independent
// tiles; stage s of an item may start only when all tiles of stage s-1 of the
// same item are done.
//
// The batch runs as two such launches: the stages up to lambda / the energy,
// then the backward passes (which carry psi and lambda through the
// interpreter and need more registers).  The host lays the (item, stage)
// records of a launch out in 8 queues (one per XCD,
// workgroup w serves queue w % 8) in level order, so every dependency of a
// record precedes it in its queue.  The grid holds only resident
// workgroups; a workgroup pops a tile index with an atomic, finds its record,
// waits (bounded in wall-clock time) for the previous stage and runs the tile
// with the same interpreter body as the single-circuit tile pass.  Waits can
// only be on tiles popped earlier by running workgroups, so the queue always
// drains; a wait that exceeds its time budget sets an error flag and the
// workgroup skips its work, so every wave still reaches the exit.
//
// Control flow around the barriers is wave-uniform: wave 0 as a whole runs
// the scheduling step (one lane does the atomics, the results are broadcast
// with readlane/readfirstlane), the other waves skip it.  A lane-dependent
// branch next to a barrier on the loop's back edge lets the compiler build an
// inner loop that some lanes of a wave leave and others do not, which does
// not terminate on SIMD hardware.  The completion count of a tile is added
// by the same lane-0 step that pops the workgroup's next tile.
#include "device_common.h"
#include "kernels.h"
#include "tile_frame.h"
#include "tile_ops.h"
#include "tile_interp.h"
#include "batch.h"

namespace svmi {

namespace {

constexpr int kBNT = 256;

template <class R>
__device__ void init_tile(const BItem& it, uint32_t tile, uint32_t Th) {
    V2<R>* psi = reinterpret_cast<V2<R>*>(it.state);
    const uint64_t j0 = (uint64_t)tile << Th;
    const uint32_t cnt = 1u << Th;
    for (uint32_t i = threadIdx.x; i < cnt; i += kBNT) {
        V2<R> v{R(0), R(0)};
        if (j0 + i == 0) v.x = R(1);
        psi[j0 + i] = v;
    }
}

// lambda = H psi on the tile's amplitudes (FP64 accumulation) and the tile's
// partial of Re <psi|lambda>.  With `write` = false only the energy partial.
template <class R>
__device__ void hpsi_tile(const BItem& it, uint32_t tile, uint32_t Th, bool write, double* sh) {
    const V2<R>* psi = reinterpret_cast<const V2<R>*>(it.state);
    V2<R>* lam = reinterpret_cast<V2<R>*>(it.lam);
    const PauliDev& pd = it.pd;
    const uint64_t j0 = (uint64_t)tile << Th;
    const uint32_t cnt = 1u << Th;
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < cnt; i += kBNT) {
        const uint64_t j = j0 + i;
        double lr = 0.0, li = 0.0;
        for (uint32_t g = 0; g < pd.ngroup; ++g) {
            const uint64_t jx = j ^ pd.x[g];
            const V2<R> v = psi[jx];
            const double vr = v.x, vi = v.y;
            const uint32_t t1 = pd.g0[g + 1];
            for (uint32_t t = pd.g0[g]; t < t1; ++t) {
                const double s = ((__popcll(jx & pd.z[t]) & 1) ? -1.0 : 1.0) * pd.c[t];
                const uint32_t ph = pd.ph[t];
                double xr = vr, xi = vi;
                if (ph & 1) { const double tmp = xr; xr = -xi; xi = tmp; }
                if (ph & 2) { xr = -xr; xi = -xi; }
                lr += s * xr;
                li += s * xi;
            }
        }
        const V2<R> a = psi[j];
        if (write) {
            const V2<R> lv{R(lr), R(li)};
            lam[j] = lv;
            // energy from the rounded lambda, as the adjoint sweep sees it
            acc += (double)a.x * (double)lv.x + (double)a.y * (double)lv.y;
        } else {
            acc += (double)a.x * lr + (double)a.y * li;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kBNT / 64; ++w) s += sh[w];
        it.epart[tile] = s;
    }
}

__device__ __forceinline__ uint64_t rfl64(uint64_t v) {
    return (uint64_t)rfl((uint32_t)v) | ((uint64_t)rfl((uint32_t)(v >> 32)) << 32);
}

template <class T>
__device__ __forceinline__ T* uptr(T* p) {
    return reinterpret_cast<T*>(rfl64(reinterpret_cast<uint64_t>(p)));
}

// Register budgets (waves per SIMD) of the variants: two waves for complex64
// (the backward interpreter carries psi and lambda), one for complex128.
template <class R, bool BWD>
struct BatchWaves {
    static constexpr int value = sizeof(R) == 4 ? 2 : 1;
};

// Tile dependencies (a pass of a circuit needs every tile of its previous
// stage) are counted in done[].  A finished tile is published with one
// device-scope release (the L2 is written back once, after every wave's
// stores have completed) and a relaxed count; a waiting workgroup polls the
// count with relaxed loads and takes one device-scope acquire when it is
// reached.  (Fences on every poll and around every tile cost 2.5x on
// 22-qubit circuits.)
template <class R, bool BWD>
__global__ __launch_bounds__(kBNT) __attribute__((amdgpu_waves_per_eu(BatchWaves<R, BWD>::value)))
void k_batch(BatchArgs B) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_ctl[4];          // popped slot, record (-1: queue empty), skip
    __shared__ double s_red[kBNT / 64];
    const uint32_t q = blockIdx.x % kQueues;
    const uint32_t rec0 = B.qrec0[q], rec1 = B.qrec0[q + 1];
    const uint64_t total = B.qtotal[q];
    const bool wave0 = threadIdx.x < 64;   // wave-uniform
    const uint32_t lane = threadIdx.x & 63u;
    int32_t prev = -1;                     // record of the tile finished in the previous round
    for (;;) {
        if (wave0) {
            uint32_t wl = 0;
            if (lane == 0) {
                if (prev >= 0) {
                    // every wave's stores have completed (wait + barrier below)
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    __hip_atomic_fetch_add(&B.done[prev], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                wl = __hip_atomic_fetch_add(&B.head[q], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            const uint32_t w = __builtin_amdgcn_readlane(wl, 0);
            int32_t r = -1;
            if (w < total) {
                // binary search: last record with first_w <= w
                uint32_t lo = rec0, hi = rec1;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) / 2;
                    if (rfl64(B.recs[mid].first_w) <= w) lo = mid; else hi = mid;
                }
                r = (int32_t)lo;
            }
            uint32_t skip = 0;
            if (r >= 0) {
                const int32_t dep = (int32_t)rfl((uint32_t)B.recs[r].dep);
                if (dep >= 0) {
                    const uint32_t need = rfl(B.recs[dep].ntiles);
                    const uint64_t t0 = wall_clock64();
                    for (;;) {
                        const uint32_t d = rfl(__hip_atomic_load(&B.done[dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                        if (d >= need) break;
                        const uint32_t e = rfl(__hip_atomic_load(B.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                        if (e != 0u || wall_clock64() - t0 > B.wait_ticks) {
                            skip = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(4);
                    }
                    // acquire what the previous stage wrote
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
            }
            if (lane == 0) {
                if (skip) __hip_atomic_fetch_or(B.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_ctl[0] = w;
                s_ctl[1] = (uint32_t)r;
                s_ctl[2] = skip;
            }
        }
        __syncthreads();
        const int32_t r = (int32_t)rfl(s_ctl[1]);
        if (r < 0) break;
        const uint32_t skip = rfl(s_ctl[2]);
        const BRec rc = B.recs[r];
        const uint32_t tile = rfl(s_ctl[0]) - (uint32_t)rfl64(rc.first_w);
        const uint32_t kind = rfl(rc.kind);
        if (!skip) {
            const BItem& it = B.items[rfl(rc.item)];
            if (!BWD && kind == BK_INIT) {
                init_tile<R>(it, tile, rfl(rc.T));
            } else if (!BWD && (kind == BK_HPSI || kind == BK_ENERGY)) {
                hpsi_tile<R>(it, tile, rfl(rc.T), kind == BK_HPSI, s_red);
            } else {
                // the plan pointers are uniform: keep them in scalar registers so the
                // interpreter's loop bounds stay scalar, as in the single-circuit kernel
                TileArgs A{};
                const BPlan& pl = BWD ? it.bwd : it.fwd;
                A.state = uptr<void>(it.state);
                A.lam = uptr<void>(it.lam);
                A.pass = uptr<const DPass>(pl.passes) + rfl(rc.pass);
                A.phases = uptr<const DPhase>(pl.phases);
                A.ops = uptr<const DOp>(pl.ops);
                A.forms = uptr<const DForm>(pl.forms);
                A.pairs = uptr<const DPair>(pl.pairs);
                A.etab = uptr<const uint16_t>(pl.etab);
                A.pool = uptr<const void>(pl.pool);
                A.pool_bstride = 0;
                A.state_bstride = 0;
                A.phase_tab = A.pool;
                A.gpart = BWD ? uptr<double>(it.gpart) + A.pass->gpart_off : nullptr;
                A.ntile_log2 = rfl(it.n) - rfl(rc.T);
                A.nthreads = kBNT;
                tile_interp<R, kBNT, BWD, false>(A, smem, tile);
            }
        }
        // every wave's global writes have completed before wave 0 publishes
        // the tile with its next pop
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        prev = r;
    }
}

}  // namespace

template <class R, bool BWD>
static const void* batch_fn() {
    return reinterpret_cast<const void*>(&k_batch<R, BWD>);
}

hipError_t launch_batch(int dtype, bool bwd, const BatchArgs& a, uint32_t nblocks, size_t lds, hipStream_t s) {
    if (dtype == 1) {
        if (bwd) hipLaunchKernelGGL((k_batch<float, true>), dim3(nblocks), dim3(kBNT), lds, s, a);
        else hipLaunchKernelGGL((k_batch<float, false>), dim3(nblocks), dim3(kBNT), lds, s, a);
    } else {
        if (bwd) hipLaunchKernelGGL((k_batch<double, true>), dim3(nblocks), dim3(kBNT), lds, s, a);
        else hipLaunchKernelGGL((k_batch<double, false>), dim3(nblocks), dim3(kBNT), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t batch_occupancy(int dtype, bool bwd, size_t lds, int* blocks_per_cu) {
    const void* f = dtype == 1 ? (bwd ? batch_fn<float, true>() : batch_fn<float, false>())
                               : (bwd ? batch_fn<double, true>() : batch_fn<double, false>());
    // 160 KiB of LDS per workgroup minus the kernel's static shared variables
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, kBNT, lds);
}

}  // namespace svmi
