// Device-visible data of the persistent batched launch.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "plan.h"

namespace svmi {

constexpr uint32_t kQueues = 8;   // one work queue per XCD

// One direction (forward or backward) of one item's plan, device pointers.
struct BPlan {
    const DPass* passes;
    const DPhase* phases;
    const DOp* ops;
    const DForm* forms;
    const DPair* pairs;
    const uint16_t* etab;
    const void* pool;       // matrix pool; its first 8 entries are the phase table
};

struct BItem {
    void* state;
    void* lam;
    BPlan fwd, bwd;
    PauliDev pd;
    double* gpart;          // gradient partials of the backward passes
    double* epart;          // energy partial per lambda tile
    uint32_t n;
    uint32_t pad;
};

enum BKind : uint32_t { BK_INIT = 0, BK_FWD = 1, BK_HPSI = 2, BK_ENERGY = 3, BK_BWD = 4 };

// A stage of an item: `ntiles` independent tiles, queue slots [first_w, first_w + ntiles).
struct BRec {
    uint64_t first_w;
    uint32_t item, kind, pass, ntiles, T;
    int32_t dep;            // record of the previous stage (-1: none)
};

struct BatchArgs {
    const BItem* items;
    const BRec* recs;
    uint32_t qrec0[kQueues + 1];   // records of queue q: [qrec0[q], qrec0[q+1])
    uint64_t qtotal[kQueues];      // tiles in queue q
    uint32_t* head;                // per-queue pop counters
    uint32_t* done;                // per-record finished tiles
    uint32_t* err;                 // set when a dependency wait exceeds its time budget
    uint64_t wait_ticks;           // budget of one dependency wait, device wall-clock ticks
};

// bwd = false: init / forward / lambda / energy stages; true: backward stages.
hipError_t launch_batch(int dtype, bool bwd, const BatchArgs& a, uint32_t nblocks, size_t lds, hipStream_t s);
hipError_t batch_occupancy(int dtype, bool bwd, size_t lds, int* blocks_per_cu);

}  // namespace svmi
