// Heterogeneous batches (circuits of different widths).
//
// This translation unit hosts the batch driver; the single-launch persistent
// kernel lives in batch_persistent.hip and is used when the batch qualifies
// (see run_batch_persistent there).  This file provides the per-item
// fallback path that the persistent path is checked against.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "host.h"
#include "sv.h"

namespace svmi {

sv_status run_batch_loop(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream,
                         int32_t flags, double* energies, double* grads, const sv_opts* opts, sv_stats* stats,
                         std::string& err) {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    size_t goff = 0;
    for (int32_t i = 0; i < count; ++i) {
        const sv_batch_item& it = items[i];
        const int n = it.circuit->n_qubits;
        const size_t bytes = ((size_t)1 << n) * (dtype == SV_C64 ? 8 : 16);
        sv_ctx c = nullptr;
        sv_status st = sv_create(&c, n, dtype, 1, it.d_state, bytes, stream, opts);
        if (st != SV_OK) { err = sv_last_error(); return st; }
        if (flags & SV_BATCH_INIT_ZERO) {
            st = sv_init(c, SV_INIT_ZERO, 0);
            if (st != SV_OK) { err = sv_last_error(); sv_destroy(c); return st; }
        }
        sv_stats s1;
        if (flags & SV_BATCH_GRAD) {
            st = sv_adjoint_grad(c, it.circuit, it.params, it.observable, it.d_lambda, bytes, energies + i,
                                 grads + goff, &s1);
        } else {
            st = sv_apply_circuit(c, it.circuit, it.params, &s1);
            if (st == SV_OK && energies) st = sv_expect(c, it.observable, energies + i);
        }
        if (st != SV_OK) { err = sv_last_error(); sv_destroy(c); return st; }
        sv_destroy(c);
        goff += (size_t)it.circuit->n_params;
        if (stats) {
            stats->gates_in += s1.gates_in;
            stats->passes += s1.passes;
            stats->launches += s1.launches;
            stats->hbm_bytes += s1.hbm_bytes;
            stats->flops += s1.flops;
            stats->plan_ms += s1.plan_ms;
        }
    }
    return SV_OK;
}

}  // namespace svmi

namespace svmi {

sv_status run_batch_persistent(int32_t count, const sv_batch_item* items, sv_dtype dtype, hipStream_t stream,
                               int32_t flags, double* energies, double* grads, const sv_opts* opts,
                               sv_stats* stats, std::string& err) {
    if (count < 0) { err = "count < 0"; return SV_EINVAL; }
    if (count > 0 && !items) { err = "items is NULL"; return SV_EINVAL; }
    if (dtype != SV_C64 && dtype != SV_C128) { err = "dtype must be SV_C64 or SV_C128"; return SV_EINVAL; }
    if ((flags & SV_BATCH_GRAD) && (!energies || !grads)) { err = "energies and grads are required"; return SV_EINVAL; }
    for (int32_t i = 0; i < count; ++i) {
        if (!items[i].circuit || !items[i].d_state) { err = "item " + std::to_string(i) + ": NULL circuit or state"; return SV_EINVAL; }
        if ((flags & SV_BATCH_GRAD) && (!items[i].d_lambda || !items[i].observable)) {
            err = "item " + std::to_string(i) + ": gradients need d_lambda and an observable";
            return SV_EINVAL;
        }
        if (energies && !items[i].observable) { err = "item " + std::to_string(i) + ": energies need an observable"; return SV_EINVAL; }
    }
    return run_batch_loop(count, items, dtype, stream, flags, energies, grads, opts, stats, err);
}

}  // namespace svmi
