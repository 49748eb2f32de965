"""Split-cost model of Appendix B (oracle; test infrastructure only).

For a split in layer k of an L-layer network the direct cost is
sum_{i=k+1}^{L} 2 d_i C_i  with  C_i = sum_{j<i} c_j, where the per-layer
back-substitution cost c_j is d_j + p_j for a ReLU layer (p_j multi-neuron
constraints), #W_j for a linear layer and d_j k_j^2 for a convolution.

Reading: the appendix lists no cost for a residual addition; passing a
coefficient through one touches each of its d_j entries once, so it is
counted as c_j = d_j.
"""
from __future__ import annotations


def layer_costs(layers):
    """layers: list of dicts {kind: relu|fc|conv|add, d: width, p: #MNC, nW: #weights, k: kernel}."""
    out = []
    for L in layers:
        if L["kind"] == "relu":
            out.append(L["d"] + L.get("p", 0))
        elif L["kind"] == "fc":
            out.append(L["nW"])
        elif L["kind"] == "conv":
            out.append(L["d"] * L["k"] ** 2)
        elif L["kind"] == "add":
            out.append(L["d"])
        else:
            raise ValueError(L["kind"])
    return out


def split_cost(layers, k):
    """sum_{i=k+1}^{L} 2 d_i C_i for layers indexed 0..L (the list order)."""
    c = layer_costs(layers)
    total = 0
    for i in range(k + 1, len(layers)):
        Ci = sum(c[:i])
        total += 2 * layers[i]["d"] * Ci
    return total
