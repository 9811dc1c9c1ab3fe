"""Host-side pieces of bench.py (no GPU): the gate categories of the
runtime profile and the one-GPU guard."""
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
