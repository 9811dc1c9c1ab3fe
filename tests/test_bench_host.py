"""Host-side pieces of bench.py (no GPU): the gate categories of the
runtime profile, the one-GPU guard and the gating of the recorded HBM
traffic on the kernel sources and tile geometry it was counted for."""
import subprocess
import sys
import os

import bench
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_categories_partition_the_circuit():
    c = W.grid_circuit(4, 8, 26, seed=1004)
    cats = bench.categorize(c, W, local_bits=13)
    assert sum(len(x) for x in cats.values()) == len(c)
    assert len(cats["initial H"]) == c.n
    assert all(g.op == "H" for g in cats["initial H"].gates)
    assert all(g.op in ("CZ", "T") for g in cats["diagonal"].gates)
    assert all(g.qubits[0] < 13 and g.op not in bench.DIAGONAL_OPS for g in cats["low one-qubit"].gates)
    assert all(g.qubits[0] >= 13 and g.op not in bench.DIAGONAL_OPS for g in cats["high one-qubit"].gates)
    # order inside a category is the circuit's order
    pos = {id(g): i for i, g in enumerate(c.gates)}
    for x in cats.values():
        idx = [pos[id(g)] for g in x.gates]
        assert idx == sorted(idx)


def test_initial_layer_stops_at_a_repeated_qubit():
    g = [W.Gate("H", (0,)), W.Gate("H", (1,)), W.Gate("H", (0,)), W.Gate("CZ", (0, 1))]
    cats = bench.categorize(W.Circuit(2, g), W)
    assert len(cats["initial H"]) == 2 and len(cats["low one-qubit"]) == 1 and len(cats["diagonal"]) == 1


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_every_leg_main_calls_is_defined():
    import ast
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    main = next(n for n in tree.body if isinstance(n, ast.FunctionDef) and n.name == "main")
    called = {c.func.id for c in ast.walk(main) if isinstance(c, ast.Call) and isinstance(c.func, ast.Name)}
    defined = {n.name for n in tree.body if isinstance(n, ast.FunctionDef)}
    builtins = set(dir(__builtins__)) if isinstance(__builtins__, dict) is False else set(__builtins__)
    missing = sorted(x for x in called - defined if x not in builtins and not hasattr(__import__("builtins"), x))
    assert not missing, missing


def test_recorded_traffic_only_for_the_profiled_sources_and_geometry(tmp_path, monkeypatch):
    prof = tmp_path / "p.md"
    prof.write_text("traffic_bytes_per_launch: 123456789\n"
                    "tile_geometry: 13 4 512\n"
                    f"kernel_sources_sha256_16: {bench.kernel_sources_hash()}\n")
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    assert bench.recorded_traffic(True, (13, 4, 512)) == 123456789.0
    assert bench.recorded_traffic(True, (12, 4, 512)) is None     # other tile geometry
    assert bench.recorded_traffic(False, (13, 4, 512)) is None    # other workload
    prof.write_text(prof.read_text().replace(bench.kernel_sources_hash(), "0" * 16))
    assert bench.recorded_traffic(True, (13, 4, 512)) is None     # sources changed since the counters


def test_committed_traffic_summary_is_close_to_the_algorithmic_bytes():
    # One launch reads and writes the 2^33-amplitude complex64 state, except
    # the first pass of the 22, which only writes it.
    vals = {}
    for line in open(bench.PROFILE):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    traffic = float(vals["traffic_bytes_per_launch"])
    algorithmic = (2 ** 33 * 8) * (2 * 21 + 1) / 22
    assert abs(traffic / algorithmic - 1) < 0.01
    assert len(vals["kernel_sources_sha256_16"]) == 16
    assert vals["tile_geometry"].split() == ["13", "4", "512"]
