#!/usr/bin/env python
"""Benchmark: Schroedinger sweep of the 33-qubit 3x11 grid circuit (40 cycles,
1873 gates) in complex64 on one MI355X, plus the adjoint-gradient leg (20
qubits, 400 parameters, 64 parameter sets) against finite differences with
the plain per-gate kernels.

A step = initialise |0...0> + apply the whole circuit + the FP64 norm check
(summed by the sweep's last pass), with the 64 GiB state resident in HBM.
Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from tests.golden import load as golden   # stored FP64 oracle values (text), never the oracle itself

HBM_PEAK_GBS = 8000.0                 # MI355X HBM3E, GB/s
# Vector ALU issue peak without packed FP32: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
# = 39.3 T lane-instructions/s (an add, a multiply or an FMA each count once).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


PROFILE = os.path.join(ROOT, "profiles", "tile_pass_grid3x11_33q_c64.md")


def kernel_sources_hash() -> str:
    """Hash of the sources that define the tile-pass kernels and plans."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2008_00216_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload_is_default: bool, geometry):
    """HBM bytes per tile-pass launch from the committed FETCH_SIZE/WRITE_SIZE
    summary (calibrated against a device copy), or None when the kernel
    sources changed since the counters were taken, or the workload or tile
    geometry differs."""
    if not workload_is_default or not os.path.exists(PROFILE):
        return None
    vals = {}
    with open(PROFILE) as f:
        for line in f:
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_sources_sha256_16",
                                                      "tile_geometry"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256_16") != kernel_sources_hash():
        return None
    if vals.get("tile_geometry") != " ".join(str(int(x)) for x in geometry):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--qubits", type=int, default=33, help="grid 3 x (qubits/3); 33 = headline")
    p.add_argument("--cycles", type=int, default=40)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-adjoint", action="store_true")
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--no-sample", action="store_true")
    p.add_argument("--no-c128", action="store_true")
    p.add_argument("--no-sf", action="store_true")
    p.add_argument("--sf-only", action="store_true", help="only the Schroedinger-Feynman leg")
    p.add_argument("--batch-only", action="store_true", help="only the 512-circuit batch leg")
    p.add_argument("--batch-tune-file", default=None,
                   help="with --batch-only: use the batch tuning stored in this file (SVMI_BATCH_TUNE_CACHE) "
                        "instead of tuning and timing the default geometry")
    p.add_argument("--c128-only", action="store_true", help="only the complex128 sweep leg")
    p.add_argument("--dense-blocks", action="store_true",
                   help="4 random 5-qubit and 4 random 6-qubit unitaries on a 30-qubit complex128 state, one "
                        "kernel each (the MFMA dense-block kernel)")
    p.add_argument("--ksweep", action="store_true", help="30-qubit dense-width sweep instead of the benchmark")
    p.add_argument("--ablation", action="store_true",
                   help="32-qubit ablation and gate-category profile instead of the benchmark")
    p.add_argument("--calib-copy-gib", type=float, default=0.0,
                   help="run a device copy of this size first (counter calibration)")
    p.add_argument("--structured", type=int, default=1)
    p.add_argument("--tile-bits", type=int, default=0)
    p.add_argument("--low-bits", type=int, default=0)
    p.add_argument("--threads", type=int, default=0)
    p.add_argument("--jit", type=int, default=0, help="plan-specialised kernels: 0 auto, 1 always, -1 never")
    p.add_argument("--no-tune", action="store_true", help="skip the tile-geometry autotuner")
    p.add_argument("--plan-beam", type=int, default=0,
                   help="planner beam width over the passes' local sets (0 = library default, 1 = greedy)")
    return p.parse_args()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def _oracle_prefix_rate(oracle, np, circ, params, nthreads, budget_s):
    """Apply gates of circ one by one in FP64 from |0..0> until budget_s has
    passed (or the circuit ends): (gates done, seconds, amp-updates/s)."""
    n = circ.n
    psi = np.zeros(1 << n, np.complex128)
    psi[0] = 1.0
    t0 = time.perf_counter()
    done = 0
    for g in circ.gates:
        oracle.apply_matrix(psi, n, g.qubits, oracle.gate_matrix(g, params), nthreads)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return done, dt, done * float(1 << n) / dt


def cpu_baseline(circ, W, np, budget_s=8.0):
    """The FP64 oracle, gate by gate, on this host's cores (all of them and
    one), on a bounded sample of every workload; each figure is extrapolated
    from the timed sample to the whole workload by amplitude updates.  The
    headline value is the 33-qubit grid's: the amp-updates/s of its 28-qubit
    cut over 2^33."""
    import oracle
    nthreads = oracle.max_threads()
    out = {"kind": "oracle", "cores": nthreads, "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}
    cfg = {}

    def sweep_entry(name, c, params=None, whole=None):
        whole = whole if whole is not None else len(c)
        done, dt, rate = _oracle_prefix_rate(oracle, np, c, params, nthreads, budget_s)
        done1, dt1, rate1 = _oracle_prefix_rate(oracle, np, c, params, 1, budget_s / 3)
        amps = float(1 << c.n)
        cfg[name] = {"qubits": c.n, "gates": whole,
                     "all_cores": {"gates_per_s": rate / amps, "amp_updates_per_s": rate,
                                   "sweep_s_extrapolated": whole * amps / rate,
                                   "sample": f"first {done} gates, {dt:.1f} s on {nthreads} threads"},
                     "one_core": {"gates_per_s": rate1 / amps, "amp_updates_per_s": rate1,
                                  "sweep_s_extrapolated": whole * amps / rate1,
                                  "sample": f"first {done1} gates, {dt1:.1f} s on 1 thread"}}
        return rate

    # line, 12 qubits, 175 gates, whole circuit
    sweep_entry("line12_10layers", W.line_circuit(12, 10, seed=1000))
    progress("cpu baseline: line circuit done")
    # 5x6 grid, 20 cycles: its 28-qubit cut
    sweep_entry("grid5x6_20cycles_cut28", W.grid30().cut(28))
    progress("cpu baseline: 30-qubit grid cut done")
    # the headline 3x11 grid, 40 cycles: its 28-qubit cut
    rate33 = sweep_entry("grid3x11_40cycles_cut28", circ.cut(28))
    progress("cpu baseline: 33-qubit grid cut done")
    # ansatz, 20 qubits: one energy; parameter shift needs 2 per parameter
    a = W.ansatz_circuit(20, 10)
    h = W.ansatz_observable(20)
    th = W.uniform_params(64, a.n_params, 3003)
    t0 = time.perf_counter()
    oracle.energy(a, th[0], h, nthreads=nthreads)
    t_e = time.perf_counter() - t0
    done1, dt1, rate1 = _oracle_prefix_rate(oracle, np, a, th[0], 1, budget_s / 3)
    t_e1 = len(a) * float(1 << 20) / rate1
    cfg["ansatz20_400params"] = {
        "qubits": 20, "gates": len(a), "params": a.n_params,
        "energy_s": {"all_cores": t_e, "one_core_extrapolated": t_e1},
        "param_shift_2_sets_s_extrapolated": {"all_cores": 2 * (2 * a.n_params + 1) * t_e,
                                              "one_core": 2 * (2 * a.n_params + 1) * t_e1},
        "param_shift_64_sets_s_extrapolated": {"all_cores": 64 * (2 * a.n_params + 1) * t_e},
        "sample": f"one energy on {nthreads} threads (forward sweep + 39 Pauli terms); one core: first "
                  f"{done1} gates in {dt1:.1f} s"}
    progress("cpu baseline: ansatz done")
    # batch of 512 circuits: forward of every 64th circuit, scaled by amp-updates
    bc = W.batch_circuits(512, 10, 22, 20, 60, seed0=4000)
    tot_upd = sum(len(c) * float(1 << c.n) for c in bc)
    grad_upd = sum(2 * c.n_params * len(c) * float(1 << c.n) for c in bc)
    pick = []
    t0 = time.perf_counter()
    upd = 0.0
    for i in range(0, 512, 64):        # every 64th circuit, until the budget is spent
        c = bc[i]
        p = W.uniform_params(1, c.n_params, 4000 + i)[0]
        oracle.energy(c, p, W.z_sum(c.n), nthreads=nthreads)
        upd += len(c) * float(1 << c.n)
        pick.append(i)
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    rate = upd / dt
    cfg["batch512"] = {"circuits": 512, "gates": sum(len(c) for c in bc),
                       "forward_s_extrapolated": tot_upd / rate,
                       "param_shift_grads_s_extrapolated": grad_upd / rate,
                       "amp_updates_per_s": rate,
                       "sample": f"forward + energy of circuits {pick} ({upd:.3g} amp-updates) in {dt:.1f} s on "
                                 f"{nthreads} threads; gradients by parameter shift = 2 sweeps per parameter"}
    progress("cpu baseline: batch sample done")
    out["value"] = rate33 / float(1 << circ.n)
    out["unit"] = "gates/s (33-qubit equivalent)"
    out["sample"] = (f"FP64 oracle, gate by gate, on the 28-qubit cut (qubits 0-27) of the 33-qubit grid circuit, "
                     f"{budget_s:.0f} s on {nthreads} threads; value = amp-updates/s / 2^{circ.n}")
    out["configs"] = cfg
    return out


def _err_vs_fp64(got, want, n):
    import numpy as np
    err = float(np.max(np.abs(np.asarray(got) - np.asarray(want))))
    return {"max_abs_err_vs_fp64": err, "max_abs_err_x_2^(n/2)": err * 2.0 ** (n / 2)}


def adjoint_leg(sv, W, torch, np):
    """cfg: 20 qubits, 10 layers RY/RZ + CZ ladder, 400 params, batch 64."""
    n, B = 20, 64
    c = W.ansatz_circuit(n, 10)
    h = W.ansatz_observable(n)
    th = W.uniform_params(B, c.n_params, 3003)
    s = sv.StateVector(n, torch.complex64, batch=B)
    scratch = torch.empty_like(s.tensor)
    # marshalled once, as a caller reusing its circuit and observable would
    cabi, habi = sv.CircuitABI(c), sv.PauliABI(h)
    # warm up (plans)
    s.init("zero_deferred")
    s.adjoint_grad(cabi, th, habi, scratch)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.time()
    for _ in range(reps):
        s.init("zero_deferred")
        e, g = s.adjoint_grad(cabi, th, habi, scratch)
    torch.cuda.synchronize()
    t_adj = (time.time() - t0) / reps
    adj_ops = s.last_stats["alu_ops"]   # forward + backward sweeps, all 64 sets
    # finite differences with the plain per-gate kernels on the same GPU
    sp = sv.StateVector(n, torch.complex64, batch=B, opts=sv.make_opts(plain=1))
    hstep = 1e-3
    sample = [0, 137, 262, 399]
    sp.init("zero"); sp.apply(c, th); sp.expect(h)
    torch.cuda.synchronize()
    t0 = time.time()
    fd = np.zeros((B, len(sample)))
    for j, p in enumerate(sample):
        vals = []
        for sgn in (1, -1):
            tt = th.copy()
            tt[:, p] += sgn * hstep
            sp.init("zero")
            sp.apply(c, tt)
            vals.append(sp.expect(h))
        fd[:, j] = (vals[0] - vals[1]) / (2 * hstep)
    t_fd_sample = time.time() - t0
    t_fd_full = t_fd_sample / len(sample) * c.n_params      # 2 sweeps per parameter
    err_fd = float(np.max(np.abs(g[:, sample] - fd)))
    # parameter shift (exact for exp(-i theta P / 2) gates) with the fused
    # sweeps on the same GPU: 2 sweeps per parameter
    sf = sv.StateVector(n, torch.complex64, batch=B)
    sf.init("zero"); sf.apply(c, th); sf.expect(h)
    torch.cuda.synchronize()
    t0 = time.time()
    ps = np.zeros((B, len(sample)))
    for j, p in enumerate(sample):
        vals = []
        for sgn in (1, -1):
            tt = th.copy()
            tt[:, p] += sgn * math.pi / 2
            sf.init("zero")
            sf.apply(c, tt)
            vals.append(sf.expect(h))
        ps[:, j] = (vals[0] - vals[1]) / 2
    t_ps_full = (time.time() - t0) / len(sample) * c.n_params
    err_ps = float(np.max(np.abs(g[:, sample] - ps)))
    del sf, sp
    sel, en, gr = golden.ansatz20_gradients()
    fp64 = {"energy_max_abs_err_vs_fp64": max(abs(e[b] - en[b]) for b in en),
            "grad_max_abs_err_vs_fp64": max(float(np.max(np.abs(g[b][sel] - gr[b]))) for b in gr),
            "sample": f"sets {sorted(en)}: energies and parameter-shift gradients of {len(sel)} sampled "
                      "parameters from the FP64 oracle (tests/golden/ansatz20_gradients.txt)"}
    return {
        "workload": "ansatz20q-10layers-400params-batch64-c64",
        "adjoint_s": t_adj,
        "roofline_alu": {"bound": "alu", "achieved": round(adj_ops / t_adj / 1e12, 2), "peak": round(VALU_PEAK_TOPS, 2),
                         "unit": "TOP/s", "frac": round(adj_ops / t_adj / 1e12 / VALU_PEAK_TOPS, 4),
                         "note": "algorithmic vector instructions of the forward and backward sweeps / whole call"},
        "grad_vectors_per_s": B / t_adj,
        "param_grads_per_s": B * c.n_params / t_adj,
        "fd_plain_s_extrapolated": t_fd_full,
        "fd_sample": f"{len(sample)} params x 2 plain sweeps x {B} sets, h={hstep}",
        "speedup_vs_fd_plain": t_fd_full / t_adj,
        "max_abs_diff_vs_fd": err_fd,
        "param_shift_fused_s_extrapolated": t_ps_full,
        "param_shift_sample": f"{len(sample)} params x 2 fused sweeps x {B} sets, shifts +-pi/2",
        "speedup_vs_param_shift_fused": t_ps_full / t_adj,
        "max_abs_diff_vs_param_shift": err_ps,
        "fp64_check": fp64,
    }


def plain_leg(sv, W, torch, reps=20):
    """The plain method on a small state: the 12-qubit line circuit (10
    layers, 175 gates) in complex128 from |0..0>, one kernel per gate.  At
    64 KiB this is bound by launch latency, not HBM, so it is reported per
    gate; the fused sweep of the same circuit is given beside it."""
    c = W.line_circuit(12, 10, seed=1000)
    out = {"workload": f"line12-10layers-{len(c)}gates-c128"}
    for name, kw in (("one_kernel_per_gate", dict(plain=1)), ("fused", dict())):
        s = sv.StateVector(c.n, torch.complex128, opts=sv.make_opts(**kw))
        cabi = sv.CircuitABI(c)
        s.init("zero")
        st = s.apply(cabi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            s.init("zero")
            st = s.apply(cabi)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        idx, want, _ = golden.amplitudes("line12_amplitudes.txt")
        got = s.amplitudes(idx)[0]
        out[name] = {"us_per_gate": dt / len(c) * 1e6, "ms_per_sweep": dt * 1e3, "launches": st["launches"],
                     "fp64_check": _err_vs_fp64(got, want, c.n)}
        s.close()
    return out


def copy_ceiling(sv, torch, n=30, reps=5):
    """Streaming read + write bandwidth on this GPU, the practical ceiling
    of a pass that reads and writes the state once: sv_copy_state between
    two 2^n-amplitude complex64 states (8 GiB at n = 30), timed with HIP
    events on the library's stream, next to a torch device copy."""
    a = sv.StateVector(n, torch.complex64)
    b = sv.StateVector(n, torch.complex64)
    a.tensor.fill_(1.0)
    b.copy_from(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_from(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(reps):
        b.tensor.copy_(a.tensor)
    e1.record()
    torch.cuda.synchronize()
    ms_torch = e0.elapsed_time(e1) / reps
    same = bool(torch.equal(a.tensor, b.tensor))
    nb = float(a.tensor.numel() * a.tensor.element_size())
    del a, b
    torch.cuda.empty_cache()
    gbs, gbs_t = 2.0 * nb / (ms / 1e3) / 1e9, 2.0 * nb / (ms_torch / 1e3) / 1e9
    return {"GBps": round(gbs, 1), "frac_of_spec": round(gbs / HBM_PEAK_GBS, 4), "bytes": 2 * nb,
            "torch_copy_GBps": round(gbs_t, 1), "copy_exact": same,
            "what": f"sv_copy_state of a 2^{n}-amplitude complex64 state (read + write), {reps} reps, HIP events"}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batch_leg(sv, W, torch, np, count=512, tune_file=None, beam=0):
    """512 circuits, n ~ U{10..22}, 20..60 layers (RY + a random gate per qubit
    + CZ), observable sum Z_i: energies and adjoint gradients of all of them
    in one persistent launch, against the same work one circuit at a time."""
    circs_py = W.batch_circuits(count, 10, 22, 20, 60, seed0=4000)
    params = [W.uniform_params(1, c.n_params, 4000 + i)[0] for i, c in enumerate(circs_py)]
    # marshalled once, as a caller reusing its circuits would
    circs = [sv.CircuitABI(c) for c in circs_py]
    obs = [sv.PauliABI(W.z_sum(c.n)) for c in circs_py]
    states = [torch.empty(1 << c.n, dtype=torch.complex64, device="cuda") for c in circs]
    lams = [torch.empty_like(t) for t in states]
    progress(f"batch: {count} circuits generated")
    bopts = sv.make_opts(plan_beam=beam)
    if tune_file is None:
        e, g, st = sv.apply_batch(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True, opts=bopts)
        torch.cuda.synchronize()
        progress("batch: first persistent launch done (plans built)")
    reps = 3
    t_default = None
    if tune_file is None:
        t0 = time.perf_counter()
        for _ in range(reps):
            e, g, st = sv.apply_batch(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True, opts=bopts)
        torch.cuda.synchronize()
        t_default = (time.perf_counter() - t0) / reps
        progress(f"batch: {t_default * 1e3:.1f} ms per launch with the default geometry")
        # per-width fusion mode and tile geometry by measurement
        t0 = time.perf_counter()
        ntuned = sv.tune_batch(circs, params, states, obs, lambdas=lams, grad=True, opts=bopts)
        t_tune = time.perf_counter() - t0
    else:
        # choices of an earlier sv_tune_batch run, read from its file
        ntuned, t_tune = -1, 0.0
    widths = sorted({c.n for c in circs_py})
    tuning = {int(w): sv.batch_tuning(w, grad=True) for w in widths}
    topts = sv.make_opts(batch_tuned=1, plan_beam=beam)
    e, g, st = sv.apply_batch(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True, opts=topts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        e, g, st = sv.apply_batch(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True, opts=topts)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    progress(f"batch: {t_batch * 1e3:.1f} ms per launch tuned ({ntuned} widths, {t_tune:.1f} s)")
    # a stream of batches: the host validates, plans and uploads batch k + 1
    # while the GPU runs batch k (sv_apply_batch_async / sv_batch_finish)
    reps_pipe = 6
    prev = None
    pipe_equal = True
    t0 = time.perf_counter()
    for _ in range(reps_pipe):
        job = sv.apply_batch_async(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True, opts=topts)
        if prev is not None:
            ep, gp, _ = prev.finish()
            pipe_equal = pipe_equal and bool(np.array_equal(ep, e)) and all(np.array_equal(a, b) for a, b in zip(gp, g))
        prev = job
    ep, gp, _ = prev.finish()
    torch.cuda.synchronize()
    t_pipe = (time.perf_counter() - t0) / reps_pipe
    pipe_equal = pipe_equal and bool(np.array_equal(ep, e)) and all(np.array_equal(a, b) for a, b in zip(gp, g))
    progress(f"batch: {t_pipe * 1e3:.1f} ms per batch in a stream of {reps_pipe} (asynchronous calls)")
    # one circuit at a time (per-circuit launches, same library)
    sample = list(range(0, count, 8))
    ctxs = {}
    for i in sample:
        c = circs[i]
        s = sv.StateVector(c.n, torch.complex64, tensor=states[i].view(1, -1))
        s.init("zero_deferred")
        s.adjoint_grad(c, params[i][None, :], obs[i], lams[i].view(1, -1))
        ctxs[i] = s
    torch.cuda.synchronize()
    progress("batch: one-at-a-time warm-up done")
    t0 = time.perf_counter()
    e_one = {}
    for i in sample:
        s = ctxs[i]
        s.init("zero_deferred")
        ee, gg = s.adjoint_grad(circs[i], params[i][None, :], obs[i], lams[i].view(1, -1))
        e_one[i] = (ee[0], gg[0])
    torch.cuda.synchronize()
    t_one = (time.perf_counter() - t0) * count / len(sample)
    err_e = max(abs(e[i] - e_one[i][0]) for i in sample)
    err_g = max(float(np.max(np.abs(g[i] - e_one[i][1]))) for i in sample)
    gates = sum(len(c.gates) for c in circs_py)
    wide = golden.batch_wide_gradients()
    fp64 = {"energy_max_abs_err_vs_fp64": max(abs(e[i] - d["energy"]) for i, d in wide.items()),
            "grad_max_abs_err_vs_fp64": max(float(np.max(np.abs(g[i][d["params"]] - d["grad"])))
                                            for i, d in wide.items() if "grad" in d),
            "sample": f"energies of the {len(wide)} circuits of 21-22 qubits among the first 64 and parameter-"
                      "shift gradients of 6 parameters of the two widest, FP64 oracle "
                      "(tests/golden/batch_wide_gradients.txt)"}
    return {
        "workload": f"{count} circuits, n 10..22, 20..60 layers, c64, forward + adjoint of sum Z",
        "gates": gates,
        "batch_s": t_batch,
        "batch_s_default_geometry": t_default,
        "tune_s": t_tune,
        "tuning_per_width": tuning,
        "roofline_alu": {"bound": "alu", "achieved": round(st["alu_ops"] / t_batch / 1e12, 2),
                         "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s",
                         "frac": round(st["alu_ops"] / t_batch / 1e12 / VALU_PEAK_TOPS, 4),
                         "note": "algorithmic vector instructions of all forward and backward passes / whole call"},
        "batch_s_stream": t_pipe,
        "stream": f"{reps_pipe} batches through sv_apply_batch_async / sv_batch_finish, one in flight while the "
                  "host prepares the next; results equal to the synchronous call: " + str(pipe_equal),
        "roofline_alu_stream": {"bound": "alu", "achieved": round(st["alu_ops"] / t_pipe / 1e12, 2),
                                "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s",
                                "frac": round(st["alu_ops"] / t_pipe / 1e12 / VALU_PEAK_TOPS, 4),
                                "note": "algorithmic vector instructions of all passes / time per batch in the stream"},
        "circuits_per_s": count / t_batch,
        "gates_per_s": gates / t_batch,
        "one_at_a_time_s_extrapolated": t_one,
        "one_at_a_time_sample": f"{len(sample)} of {count} circuits, per-circuit launches",
        "speedup_vs_one_at_a_time": t_one / t_batch,
        "max_abs_diff_energy_vs_one_at_a_time": err_e,
        "max_abs_diff_grad_vs_one_at_a_time": err_g,
        "launches": st["launches"],
        "host_prep_ms": st["plan_ms"],
        "fp64_check": fp64,
    }


def headline_fp64_check(sv, torch, circ, geometry):
    """The 33-qubit state has no FP64 reference; its 28-qubit cut (qubits
    0-27, gates entirely inside them) runs with the same options and tile
    geometry and is compared with FP64 oracle amplitudes
    (tests/golden/grid33_cut28_amplitudes.txt)."""
    cut = circ.cut(28)
    kw = dict(zip(("tile_bits", "low_bits", "threads"), (int(x) for x in geometry)))
    s = sv.StateVector(28, torch.complex64, opts=sv.make_opts(**kw))
    s.init("zero_deferred")
    _, nrm = s.apply_norm(cut)
    idx, want, nrm_want = golden.grid33_cut28()
    got = s.amplitudes(idx)[0]
    del s
    torch.cuda.empty_cache()
    return dict(_err_vs_fp64(got, want, 28), norm_err_vs_fp64=abs(float(nrm[0]) - nrm_want),
                sample=f"{len(idx)} amplitudes and the norm of the 28-qubit cut ({len(cut)} gates)")


def sample_leg(s, W, np, n, shots=1 << 20, reps=3):
    """Measurement sampling from the final state of the sweep: `shots`
    bit strings per call.  The call reads the state once to build a 64-ary
    FP64 tree of probability masses (writing 1/64 of the state's amplitude
    count in nodes), then every sample reads 64 nodes per tree level and 64
    amplitudes at the bottom; the HBM figure counts those bytes."""
    u = W.sample_uniforms(shots, seed=16)
    s.sample(u)                                     # warm-up: buffers
    t0 = time.perf_counter()
    for _ in range(reps):
        got = s.sample(u)
    dt = (time.perf_counter() - t0) / reps
    amp = s.amplitudes(got[:8192])[0]
    xeb = float(np.mean(np.abs(amp) ** 2) * float(1 << n) - 1.0)
    levels = (n + 5) // 6
    state_bytes = float(1 << n) * 8
    tree_bytes = sum(float(1 << max(0, n - 6 * k)) * 8 for k in range(1, levels + 1))
    per_sample = 64 * 8 + sum(min(64, 1 << max(0, n - 6 * k)) * 8 for k in range(1, levels)) + 16
    moved = state_bytes + tree_bytes + shots * per_sample
    return {"shots": shots, "ms_per_call": dt * 1e3, "samples_per_s": shots / dt,
            "hbm_bytes_algorithmic": moved, "GBps_whole_call": moved / dt / 1e9,
            "hbm_frac_whole_call": moved / dt / 1e9 / HBM_PEAK_GBS, "linear_xeb_8192": xeb}


def c128_leg(sv, W, torch, steps=2, beam=0, geometry=(0, 0, 0)):
    """The same kind of sweep in complex128: the 32-qubit 4x8 grid circuit
    with 40 cycles (64 GiB state), default options, tile passes timed with
    HIP events.  FP64 arithmetic issues at the same lane rate as FP32, and
    every amplitude moves twice the bytes, so the passes run against the
    HBM roofline."""
    circ = W.grid_circuit(4, 8, 40, seed=1005)
    n = circ.n
    kw = dict(zip(("tile_bits", "low_bits", "threads"), geometry))
    s = sv.StateVector(n, torch.complex128, opts=sv.make_opts(timing=1, plan_beam=beam, **kw))
    cabi = sv.CircuitABI(circ)
    s.init("zero_deferred")
    st, _ = s.apply_norm(cabi)                         # warm-up: plan, compile
    s.timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.init("zero_deferred")
        st, nrm2 = s.apply_norm(cabi)
        nrm = float(nrm2[0])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    tile_ms, launches, tile_bytes = s.timing()
    per = tile_ms / max(1, launches)
    gbs = tile_bytes / max(1, launches) / (per / 1e3) / 1e9
    tops = st["alu_ops"] * steps / (tile_ms / 1e3) / 1e12
    del s
    torch.cuda.empty_cache()
    cut = circ.cut(24)
    sc = sv.StateVector(24, torch.complex128)
    sc.init("zero_deferred")
    sc.apply(cut)
    idx, want, nrm_want = golden.amplitudes("grid4x8_cut24_amplitudes.txt")
    fp64 = dict(_err_vs_fp64(sc.amplitudes(idx)[0], want, 24),
                sample=f"{len(idx)} amplitudes of the 24-qubit cut ({len(cut)} gates) against the FP64 oracle "
                       "(tests/golden/grid4x8_cut24_amplitudes.txt)")
    del sc
    return {"workload": f"grid4x8-40cycles-{n}q-c128", "gates": len(circ), "ms_per_step": ms, "fp64_check": fp64,
            "gates_per_s": len(circ) / (ms / 1e3), "passes": st["passes"],
            "tile_kernel": {"launches": launches, "avg_ms": per, "bytes_per_launch": tile_bytes / max(1, launches)},
            "roofline_hbm": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbs / HBM_PEAK_GBS, 4)},
            "roofline_alu": {"bound": "alu", "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                             "unit": "TOP/s", "frac": round(tops / VALU_PEAK_TOPS, 4)},
            "norm_error": abs(nrm - 1.0)}


def sf_mask(rows, cols, n_a):
    """Half A of a row-major grid: the first n_a qubits in column-major order
    (column 0 top to bottom, then column 1, ...), a cut with a short boundary."""
    order = [r * cols + c for c in range(cols) for r in range(rows)]
    return sum(1 << q for q in order[:n_a])


def sf_leg(sv, W, torch, np, reps=3, amplitudes=4096):
    """Schroedinger-Feynman mode: the 34-qubit 2x17 grid circuit (20 cycles)
    cut into two 17-qubit halves, 15 gates across the cut, 2^15 paths held in
    memory; `amplitudes` seeded output amplitudes per call.  Checked against
    the full 34-qubit Schroedinger sweep of the same circuit (complex64, 128
    GiB) and, for FP64, the same construction at 22 qubits against stored
    oracle amplitudes."""
    c = W.grid_circuit(2, 17, 20, seed=1007)
    mask = sf_mask(2, 17, 17)
    idx = np.unique(np.random.default_rng(17).integers(0, 1 << c.n, amplitudes).astype(np.uint64))
    sim = sv.SchrodingerFeynman(c, mask, torch.complex64)
    info = sim.info
    t0 = time.perf_counter()
    got, st = sim.amplitudes(idx)                 # plans and compiles every half-width sweep
    t_first = time.perf_counter() - t0
    progress(f"sf: first call {t_first:.1f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        got, st = sim.amplitudes(idx)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    progress(f"sf: {t * 1e3:.1f} ms per call")
    del sim
    torch.cuda.empty_cache()
    # the same amplitudes from the full-width sweep on this GPU
    s = sv.StateVector(c.n, torch.complex64)
    s.init("zero_deferred")
    t0 = time.perf_counter()
    s.apply(c)
    full = s.amplitudes(idx)[0]
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    s.apply(c)                                     # plans compiled: time a second sweep
    s.init("zero_deferred")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.apply(c)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    del s
    torch.cuda.empty_cache()
    # FP64: the 22-qubit version of the same construction
    c22 = W.grid_circuit(2, 11, 20, seed=1006)
    i22, want, _ = golden.amplitudes("grid2x11_amplitudes.txt")
    s22 = sv.SchrodingerFeynman(c22, sf_mask(2, 11, 11), torch.complex64)
    got22, _ = s22.amplitudes(i22)
    del s22
    torch.cuda.empty_cache()
    gbs = st["hbm_bytes"] / t / 1e9
    return {"workload": f"grid2x17-20cycles-34q-c64, halves of 17 qubits, {info['n_cross']} cross gates, "
                        f"{len(idx)} amplitudes",
            "paths": info["paths"], "paths_in_memory_bits": info["n_inner"], "s_per_call": t,
            "paths_per_s": info["paths"] / t, "amplitudes_per_s": len(idx) / t,
            "first_call_s": t_first, "passes": st["passes"], "launches": st["launches"],
            "roofline_hbm": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbs / HBM_PEAK_GBS, 4),
                             "note": "algorithmic bytes of every half-width pass (a pass that reads a doubled "
                                     "half state counts a full read), of the doubling copies not read by a "
                                     "pass, and of the path contraction / whole call"},
            "full_schroedinger_s": t_full, "speedup_vs_full_schroedinger": t_full / t,
            "max_abs_diff_vs_full_schroedinger_c64": float(np.max(np.abs(got - full))),
            "fp64_check": dict(_err_vs_fp64(got22, want, 22),
                               sample=f"{len(i22)} amplitudes of the 22-qubit 2x11 grid (20 cycles) by the same "
                                      "split against the FP64 oracle (tests/golden/grid2x11_amplitudes.txt)")}


DIAGONAL_OPS = ("CZ", "T", "TDG", "S", "SDG", "Z", "RZ", "CP", "P")


def categorize(circ, W, local_bits=13):
    """Split a grid circuit into the gate categories of the paper's runtime
    profile (Sec. 6, tab:profile), each as a circuit of its own with the
    gates in their original order:
      initial H      the leading layer of H gates, one per qubit;
      diagonal       CZ and T (and any other diagonal gate);
      low one-qubit  non-diagonal one-qubit gates on qubits below
                     `local_bits` (inside one tile of 2^local_bits amplitudes);
      high one-qubit non-diagonal one-qubit gates on the other qubits."""
    g = list(circ.gates)
    k = 0
    seen = set()
    while k < len(g) and g[k].op == "H" and g[k].qubits[0] not in seen:
        seen.add(g[k].qubits[0])
        k += 1
    cats = {"initial H": g[:k], "diagonal": [], "low one-qubit": [], "high one-qubit": [], "other": []}
    for x in g[k:]:
        if x.op in DIAGONAL_OPS:
            cats["diagonal"].append(x)
        elif len(x.qubits) == 1:
            cats["low one-qubit" if x.qubits[0] < local_bits else "high one-qubit"].append(x)
        else:
            cats["other"].append(x)
    return {name: W.Circuit(circ.n, gates, circ.n_params, f"{circ.name}:{name}")
            for name, gates in cats.items() if gates}


def ablation(sv, W, torch, np, steps=1):
    """GPU counterpart of the paper's ablation and runtime profile (Sec. 6):
    the 32-qubit 4x8 grid circuit (initial H + 26 cycles) in complex64,
    with the optimisations switched off one at a time, and the gate
    categories of tab:profile timed on their own in the fused and in the
    one-kernel-per-gate modes (the initial H layer as a product-state
    init, the other categories applied to a written |0..0>).  Each mode's final state is compared with the
    fully optimised one at 4096 fixed amplitudes.  Prints one JSON line."""
    circ = W.grid_circuit(4, 8, 26, seed=1004)
    n = circ.n
    modes = [
        ("all optimisations", dict()),
        ("no plan-specialised kernels (interpreter)", dict(jit=-1)),
        ("no product-state init", dict(product_init=0)),
        ("no butterflies or lazy phases (2x2 matrices, explicit diagonals)", dict(structured=0, max_fuse_k=1)),
        ("no tile passes (one kernel per gate)", dict(plain=1)),
        ("the paper's plan: kind clusters, gate pairs, Gray-code CZ, rescale passes (sqrt(W) gate by gate)",
         dict(paper=1)),
        ("the paper's plan with the recursive transform (a layer's low gates on LDS chunks)", dict(paper=2)),
    ]
    probe = np.unique(np.random.default_rng(17).integers(0, 1 << n, size=4096).astype(np.uint64))
    ref = None
    rows = []
    t_state = torch.empty((1, 1 << n), dtype=torch.complex64, device="cuda")

    def run(kw, c, reps, whole_step=True):
        """ms per sweep: deferred |0..0> + apply (whole_step), or apply
        alone on a written |0..0> (a category on its own)."""
        s = sv.StateVector(n, torch.complex64, opts=sv.make_opts(**kw), tensor=t_state)
        cabi = sv.CircuitABI(c)
        s.init("zero_deferred")
        st = s.apply(cabi)                             # warm-up: plan, compile
        torch.cuda.synchronize()
        dt = 0.0
        for _ in range(reps):
            if not whole_step:
                s.init("zero")
                torch.cuda.synchronize()
            t0 = time.perf_counter()
            if whole_step:
                s.init("zero_deferred")
            st = s.apply(cabi)
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
        return s, st, dt * 1e3 / reps

    for name, kw in modes:
        s, st, ms = run(kw, circ, steps)
        amp = s.amplitudes(probe)[0]
        if ref is None:
            ref = amp
        rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
        row = {"mode": name, "ms": ms, "passes": st["passes"], "launches": st["launches"],
               "max_abs_diff_vs_all": float(np.max(np.abs(amp - ref))),
               "max_diff_over_rms_amp": float(np.max(np.abs(amp - ref))) / rms}
        s.close()
        progress(f"ablation: {name}: {ms:.1f} ms")
        cats = {}
        if kw in (dict(), dict(plain=1)):
            for cname, cc in categorize(circ, W).items():
                # a category of one-qubit gates alone is a product state: it
                # would fold into the init entirely, so only the initial H
                # layer keeps the product-state init
                ckw = kw if cname == "initial H" else dict(kw, product_init=0)
                _, cst, cms = run(ckw, cc, 1, whole_step=(cname == "initial H"))
                cats[cname] = {"gates": len(cc), "ms": cms, "passes": cst["passes"]}
                progress(f"ablation:   {cname} ({len(cc)} gates): {cms:.1f} ms")
            tot = sum(v["ms"] for v in cats.values())
            for v in cats.values():
                v["pct_of_category_sum"] = 100.0 * v["ms"] / tot
            row["categories_alone"] = cats
        rows.append(row)
    base = rows[0]["ms"]
    for r in rows:
        r["x_slower_than_all"] = r["ms"] / base
    # the paper's own gate set (sqrt(X), sqrt(Y), T; no sqrt(W)), where its
    # plan needs no gate-by-gate fallback
    fam = W.grid_circuit(4, 8, 26, seed=1004, family=("SQRTX", "SQRTY", "T"))
    frows = []
    fref = None
    for name, kw in (("tile passes, all optimisations", dict()), ("the paper's plan", dict(paper=1)),
                     ("the paper's plan with the recursive transform", dict(paper=2))):
        s, st, ms = run(kw, fam, steps)
        amp = s.amplitudes(probe)[0]
        if fref is None:
            fref = amp
        frows.append({"mode": name, "ms": ms, "passes": st["passes"], "launches": st["launches"],
                      "max_abs_diff_vs_tile_passes": float(np.max(np.abs(amp - fref))),
                      "x_slower_than_tile_passes": None})
        s.close()
        progress(f"ablation (sqrt(X)/sqrt(Y)/T grid): {name}: {ms:.1f} ms")
    for r in frows:
        r["x_slower_than_tile_passes"] = r["ms"] / frows[0]["ms"]
    out = {"ablation": {"workload": f"grid4x8-26cycles-{n}q-c64", "gates": len(circ), "modes": rows},
           "paper_gate_set": {"workload": f"grid4x8-26cycles-{n}q-c64, family sqrt(X)/sqrt(Y)/T", "gates": len(fam),
                              "modes": frows}}
    print(json.dumps(out), flush=True)


def dense_blocks(sv, W, torch, np, n=30, reps=4):
    """Explicit 5- and 6-qubit unitaries (random, from a QR of complex
    Gaussians; seeded) on random targets of a 2^30-amplitude complex128
    state, one kernel per gate (the MFMA dense-block kernel), `reps` of each
    width; HIP-event time per gate."""
    rng = np.random.default_rng(30)
    s = sv.StateVector(n, torch.complex128, opts=sv.make_opts(plain=1))
    s.init("uniform")
    out = {"workload": f"{n}-qubit complex128 state, {reps} random 5-qubit and {reps} random 6-qubit unitaries"}
    for k in (5, 6):
        gates = []
        for _ in range(reps):
            z = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
            q, r = np.linalg.qr(z)
            gates.append(W.Gate("MAT", tuple(int(x) for x in rng.permutation(n)[:k]),
                                mat=(q * (np.diag(r) / np.abs(np.diag(r)))).astype(np.complex128)))
        c = sv.CircuitABI(W.Circuit(n, gates, 0, f"dense{k}"))
        s.apply(c)                                   # warm-up: plans
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        st = s.apply(c)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        flops = float(1 << n) * 8 * (1 << k)
        out[f"k{k}"] = {"ms_per_gate": ms, "fp64_TFLOPs": flops / (ms / 1e3) / 1e12,
                        "hbm_TBs": 2.0 * (1 << n) * 16 / (ms / 1e3) / 1e12}
    nrm = float(s.norm()[0])
    out["norm_error"] = abs(nrm - 1.0)
    del s
    torch.cuda.empty_cache()
    return out


def ksweep(sv, W, torch, steps=2):
    """5x6 grid, 30 qubits, 20 cycles, complex64 and complex128: the
    butterfly mode against dense blocks of at most k qubits (k = 1..6).  One
    JSON line per mode."""
    circ = W.grid30()
    cabi = sv.CircuitABI(circ)
    modes = [("butterflies", dict(structured=1))] + [(f"dense k<={k}", dict(structured=0, max_fuse_k=k))
                                                   for k in range(1, 7)]
    rows = []
    for dtype, name, kw in [(d, nm, kw) for d in (torch.complex64, torch.complex128) for nm, kw in modes]:
        s = sv.StateVector(circ.n, dtype, opts=sv.make_opts(timing=1, **kw))
        s.init("zero_deferred")
        st = s.apply(cabi)
        torch.cuda.synchronize()
        s.timing()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.init("zero_deferred")
            st = s.apply(cabi)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        tile_ms, launches, tile_bytes = s.timing()
        row = {"dtype": "c64" if dtype == torch.complex64 else "c128", "mode": name, "ms_per_sweep": ms,
               "gates_per_s": len(circ.gates) / (ms / 1e3),
               "passes": st["passes"], "dense_ops": st["dense_ops"],
               "hbm_frac_sweep": st["hbm_bytes"] / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
               "tile_avg_ms": tile_ms / max(1, launches),
               "alu_frac_tile": st["alu_ops"] * steps / (tile_ms / 1e3) / 1e12 / VALU_PEAK_TOPS if tile_ms else None}
        rows.append(row)
        print(json.dumps(row), flush=True)
        del s
        torch.cuda.empty_cache()
    return rows


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on a single MI355X; sharding is a design note only).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.batch_tune_file:
        os.environ["SVMI_BATCH_TUNE_CACHE"] = args.batch_tune_file
    import paper_2008_00216_amd as sv
    import workloads as W

    torch.cuda.set_device(0)
    if args.calib_copy_gib > 0:
        nb = int(args.calib_copy_gib * (1 << 30))
        a = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    if args.ksweep:
        ksweep(sv, W, torch)
        return
    if args.ablation:
        ablation(sv, W, torch, np)
        return
    if args.dense_blocks:
        print(json.dumps(dense_blocks(sv, W, torch, np)), flush=True)
        return
    if args.sf_only:
        print(json.dumps(sf_leg(sv, W, torch, np)), flush=True)
        return
    if args.batch_only:
        print(json.dumps(batch_leg(sv, W, torch, np, tune_file=args.batch_tune_file, beam=args.plan_beam)), flush=True)
        return
    if args.c128_only:
        print(json.dumps(c128_leg(sv, W, torch, beam=args.plan_beam,
                                  geometry=(args.tile_bits, args.low_bits, args.threads))), flush=True)
        return

    cols = args.qubits // 3
    circ = W.grid_circuit(3, cols, args.cycles, seed=1002)
    n = circ.n
    # host planning time of the circuit (IR, reordering, encoding), uncached
    plan_ms_host = sv.plan_info(circ, torch.complex64, opts=sv.make_opts(plan_beam=args.plan_beam))["plan_ms"]
    opts = sv.make_opts(timing=1, structured=args.structured, tile_bits=args.tile_bits,
                        low_bits=args.low_bits, threads=args.threads, jit=args.jit, plan_beam=args.plan_beam)
    s = sv.StateVector(n, torch.complex64, opts=opts)
    cabi = sv.CircuitABI(circ)
    st = None
    tuned = None
    if not args.no_tune and args.tile_bits == 0 and args.low_bits == 0 and args.threads == 0:
        t0 = time.perf_counter()
        chosen, best_ms = s.tune(cabi)
        tuned = {"tile_bits": chosen["tile_bits"], "low_bits": chosen["low_bits"], "threads": chosen["threads"],
                 "tune_s": time.perf_counter() - t0, "best_sweep_ms": best_ms}
        progress(f"tuned: {tuned}")
    for _ in range(args.warmup):
        s.init("zero_deferred")
        st, _ = s.apply_norm(cabi)
    s.timing()  # reset counters
    progress("sweep: warm-up done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norms = []
    for _ in range(args.steps):
        s.init("zero_deferred")
        st, nrm = s.apply_norm(cabi)      # the norm check is summed by the last pass
        norms.append(float(nrm[0]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tile_ms, tile_launches, tile_bytes = s.timing()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gates = len(circ.gates)
    gates_per_s = gates / (ms_per_step / 1e3)
    amp_upd = gates * float(1 << n) / (ms_per_step / 1e3)

    per_launch_ms = tile_ms / max(1, tile_launches)
    bytes_per_launch = tile_bytes / max(1, tile_launches)
    achieved_gbs = bytes_per_launch / (per_launch_ms / 1e3) / 1e9
    ops_tile = st["alu_ops"]                       # algorithmic vector instructions per lane, all tile passes
    achieved_tops = ops_tile * args.steps / (tile_ms / 1e3) / 1e12
    hbm_frac = achieved_gbs / HBM_PEAK_GBS
    alu_frac = achieved_tops / VALU_PEAK_TOPS
    geometry = (tuned["tile_bits"], tuned["low_bits"], tuned["threads"]) if tuned else (
        args.tile_bits, args.low_bits, args.threads)
    default_workload = (args.qubits == 33 and args.cycles == 40 and args.structured == 1 and args.jit == 0)
    traffic = recorded_traffic(default_workload, geometry)
    roofline_hbm = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm_frac, 4), "traffic": traffic}
    roofline_alu = {"bound": "alu", "achieved": round(achieved_tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                    "unit": "TOP/s", "frac": round(alu_frac, 4)}
    # the metric is the HBM fraction; the ALU fraction beside it names the
    # resource that binds the pass
    roofline = dict(roofline_hbm, binding=("alu" if alu_frac > hbm_frac else "hbm"), alu_frac=round(alu_frac, 4))

    out = {
        "metric": "gates/s & %HBM peak at 33q complex64; adjoint grads/s vs plain at stated error",
        "value": gates_per_s,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"grid3x{cols}-{args.cycles}cycles-{n}q-c64", "qubits": n, "gates": gates,
                   "state_gib": (1 << n) * 8 / 2 ** 30, "parallelism": "1 GPU"},
        "amp_updates_per_s": amp_upd,
        "passes": st["passes"], "phases": st["phases"], "plan_ms_first": plan_ms_host,
        "sweep_hbm_bytes": st["hbm_bytes"],
        "sweep_GBps_algorithmic": st["hbm_bytes"] / (ms_per_step / 1e3) / 1e9,
        "hbm_frac_whole_step": st["hbm_bytes"] / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "tile_kernel": {"launches": tile_launches, "avg_ms": per_launch_ms,
                        "bytes_per_launch": bytes_per_launch},
        "roofline": roofline,
        "roofline_hbm": roofline_hbm,
        "roofline_alu": roofline_alu,
        "norm_error": max(abs(x - 1.0) for x in norms),
        "tuned_geometry": tuned,
    }
    progress(f"sweep: {ms_per_step:.1f} ms per step")
    if default_workload:
        out["fp64_check"] = headline_fp64_check(sv, torch, circ, geometry)
        progress("sweep: 28-qubit cut checked against the FP64 oracle")
    if not args.no_sample:
        out["sample"] = sample_leg(s, W, np, n)
        progress(f"sampling: {out['sample']['ms_per_call']:.1f} ms per call")
    del s
    torch.cuda.empty_cache()
    out["copy_ceiling"] = copy_ceiling(sv, torch)
    out["roofline_hbm"]["frac_of_copy_ceiling"] = round(achieved_gbs / out["copy_ceiling"]["GBps"], 4)
    out["plain_method"] = plain_leg(sv, W, torch)
    progress("copy ceiling and plain-method leg done")
    if not args.no_c128:
        out["c128"] = c128_leg(sv, W, torch, beam=args.plan_beam)
        progress(f"c128 leg: {out['c128']['ms_per_step']:.1f} ms per step")
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(sv, W, torch, np)
        progress("adjoint leg done")
    if not args.no_batch:
        out["batch"] = batch_leg(sv, W, torch, np, beam=args.plan_beam)
    if not args.no_sf:
        out["schroedinger_feynman"] = sf_leg(sv, W, torch, np)
        progress("Schroedinger-Feynman leg done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(circ, W, np)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
