"""The C ABI library loads and exports every symbol include/mnbab.h declares (CPU only, no compute)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mnbab.h")
LIB = os.path.join(ROOT, "paper_2205_00263_amd", "libmnbab.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    txt = "\n".join(ln for ln in txt.splitlines() if not ln.strip().startswith("typedef"))
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("typedef",)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for n in ("bound_init", "bound_optimize", "branch_split", "query_submit", "query_poll",
              "mnb_net_create", "mnb_problem_create", "mnb_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_declares_only_exported_symbols():
    from paper_2205_00263_amd import _lib
    lib = ctypes.CDLL(LIB)
    assert [n for n in _lib.exported_symbols() if not hasattr(lib, n)] == []
    assert set(_lib.exported_symbols()) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
def test_split_costs_follow_appendix_b(cfg):
    """mnb_split_costs (host code of the library, no device work) against the oracle's cost model of
    Appendix B on the four full-size network shapes (configuration 4 has residual additions), with
    random multi-neuron constraint counts and without any."""
    import numpy as np
    import workloads as W
    from oracle import cost as ocost
    from paper_2205_00263_amd import split_costs
    nodes = W.make_net(cfg)
    shapes = W.node_shapes(nodes)
    layers, relu_pos = [], []
    for i in range(1, len(nodes)):
        n = nodes[i]
        d = int(np.prod(shapes[i]))
        if n["kind"] == "relu":
            layers.append({"kind": "relu", "d": d})
            relu_pos.append(len(layers) - 1)
        elif n["kind"] == "fc":
            layers.append({"kind": "fc", "d": d, "nW": int(np.asarray(n["W"]).size)})
        elif n["kind"] == "conv":
            layers.append({"kind": "conv", "d": d, "k": int(np.asarray(n["W"]).shape[2])})
        else:
            layers.append({"kind": "add", "d": d})
    rng = np.random.default_rng(cfg)
    for p in (None, rng.integers(0, 500, len(relu_pos)).astype(np.int32)):
        got = split_costs(nodes, p)
        for t, k in enumerate(relu_pos):
            layers[k]["p"] = 0 if p is None else int(p[t])
        assert got.tolist() == [float(ocost.split_cost(layers, k)) for k in relu_pos]
    with pytest.raises(Exception):
        split_costs(nodes, -np.ones(len(relu_pos), np.int32))
