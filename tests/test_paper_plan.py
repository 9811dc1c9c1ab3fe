"""The paper's own plan (opts.paper), host side: the kind clusters of the
reordering scan (Sec. 4.5) and their bitmask encodings (Sec. 4.2-4.3)
reproduce the values printed in the paper, and applying the clusters' gates
in plan order (with the FP64 oracle) equals the circuit."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.golden import load as golden

m = pytest.importorskip("paper_2008_00216_amd")


def trace(c, paper=1):
    return m.plan_trace(c, None if c.n_params == 0 else np.zeros(c.n_params), opts=m.make_opts(paper=paper))


def parse(tr):
    steps = []
    for line in tr.strip().splitlines():
        head, gates = line.split("|")
        steps.append((head.split(), [int(x) for x in gates.split()]))
    return steps


def fig_reorder_circuit():
    """The four-qubit example of Fig. reorder, gates listed column by column
    (sqrt(X) and sqrt(Y) boxes as drawn, CZ controls on qubits 0 and 2)."""
    G = W.Gate
    g = [G("H", (q,)) for q in range(4)]
    g += [G("CZ", (0, 1)), G("T", (2,))]
    g += [G("T", (0,)), G("CZ", (2, 3))]
    g += [G("SQRTX", (0,)), G("T", (1,)), G("SQRTX", (2,)), G("T", (3,))]
    g += [G("SQRTX", (1,)), G("SQRTY", (2,))]
    g += [G("SQRTY", (1,)), G("SQRTY", (3,))]
    g += [G("H", (q,)) for q in range(4)]
    return W.Circuit(4, g, 0, "fig-reorder")


def test_fig_reorder_clusters_and_masks():
    c = fig_reorder_circuit()
    steps = parse(trace(c))
    kinds = [h[0] if h[0] != "LAYER" else f"LAYER{h[1]}" for h, _ in steps]
    assert kinds == [f"LAYER{m.OPS['H']}", "DIAG", f"LAYER{m.OPS['SQRTX']}", f"LAYER{m.OPS['SQRTY']}",
                     f"LAYER{m.OPS['H']}"]
    bm = golden.bitmasks()
    diag = steps[1][0]
    # T layer: exponent 1 on every qubit -> bit-plane 0 = b1111
    assert diag[2] == bm["reorder_t_mask"][0] and diag[3] == "0000" and diag[4] == "0000"
    cz = dict(x.split(":") for x in diag[6:])
    assert [cz["1"], cz["3"]] == bm["reorder_cz_masks"] and set(cz) == {"1", "3"}
    assert steps[2][0][2] == bm["reorder_sqrtx_mask"][0]
    assert steps[3][0][2] == bm["reorder_sqrty_mask"][0]


def test_cz_all_pairs_masks():
    # Sec. 4.3 example: six CZ gates on all pairs of four qubits; the
    # symmetric masks (one per qubit) follow from the one-sided ones
    c = W.Circuit(4, [W.Gate("CZ", (a, b)) for a in range(4) for b in range(a + 1, 4)], 0)
    (head, gates), = parse(trace(c))
    one = {int(k): int(v, 2) for k, v in (x.split(":") for x in head[6:])}
    sym = [0] * 4
    for k, mk in one.items():
        for l in range(4):
            if (mk >> l) & 1:
                sym[k] |= 1 << l
                sym[l] |= 1 << k
    bm = golden.bitmasks()
    assert [format(x, "04b") for x in sym] == bm["cz_all_pairs_masks"]
    assert sum(bin(x).count("1") for x in sym) == int(bm["cz_all_pairs_bitcount"][0])


def test_repeated_cz_cancels_and_diagonals_accumulate():
    c = W.Circuit(3, [W.Gate("CZ", (0, 2)), W.Gate("T", (1,)), W.Gate("CZ", (2, 0)), W.Gate("S", (1,)),
                      W.Gate("Z", (0,))], 0)
    (head, gates), = parse(trace(c))
    assert head[0] == "DIAG" and sorted(gates) == list(range(5))
    # exponents: qubit 1 gets 1 + 2 = 3 (planes 0, 1), qubit 0 gets 4 (plane 2)
    assert head[2:5] == ["010", "010", "001"]
    assert head[5:] == ["cz"]           # the two CZ gates cancel


@pytest.mark.parametrize("seed", range(6))
def test_plan_order_equals_the_circuit(seed):
    n = 6
    ops = ("H", "SQRTX", "SQRTY", "SQRTXDG", "SQRTYDG", "T", "TDG", "S", "Z", "CZ", "SQRTW", "X", "RX", "CNOT")
    c = W.random_circuit(n, 80, 900 + seed, ops=ops)
    params = W.uniform_params(1, c.n_params, seed)[0]
    order = [g for _, gs in parse(m.plan_trace(c, params if c.n_params else None, opts=m.make_opts(paper=1)))
             for g in gs]
    assert sorted(order) == list(range(len(c)))
    psi0 = W.random_state(n, seed)
    a = oracle.simulate(c, params, psi0)
    b = oracle.simulate(c, params, psi0, gates=[c.gates[i] for i in order])
    assert np.max(np.abs(a - b)) < 1e-13
