"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module produces DATA only: network weights, input points, L-infinity
boxes, output specifications and split sets.  It holds none of the bounding
method's arithmetic.  The one computation it does perform is a plain forward
evaluation of the network at the centre point x0, used to choose the class
label of a robustness specification (the label is part of the input recipe,
not of the method).

The trained networks and datasets of the paper (MNIST, CIFAR10; ConvSmall,
ConvBig, ResNet6 of Tables 3-5) are not available; these generators stand in
for them with the same layer shapes and input ranges:

* weights He-normal N(0, 2/fan_in) in float32, biases U(+-1/sqrt(fan_in));
* inputs x0 ~ U[0,1]^d, box = [max(x0-eps,0), min(x0+eps,1)];
* spec rows logit[c] - logit[j] for the label c = argmax f(x0).

Network description format (a list of node dicts, topologically ordered,
node 0 is the input):

    {"kind": "input", "shape": (C, H, W)}
    {"kind": "fc",   "src": i, "W": [dout, din], "b": [dout]}
    {"kind": "conv", "src": i, "W": [Co, Ci, k, k], "b": [Co], "stride": s, "pad": p}
    {"kind": "bn",   "src": i, "gamma": [C], "beta": [C], "mean": [C], "var": [C], "eps": e}
    {"kind": "avgpool", "src": i, "k": k, "stride": s, "pad": p}
    {"kind": "relu", "src": i}
    {"kind": "add",  "src": i, "src2": j}

Output shapes are derived from the input shape (flattening in C,H,W order
happens implicitly at an fc node).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "node_shapes", "fc_net", "convsmall", "convbig", "resnet6", "resnet8",
    "tiny_fc", "tiny_conv", "tiny_resnet", "tiny_resnet_bn", "make_net", "make_input",
    "make_spec", "forward_logits", "make_split_sets", "Workload",
    "make_workload", "CONFIG_SEEDS",
]

# Seeds per configuration: net = 1000+cfg, input = 2000+cfg, splits = 3000+cfg.
CONFIG_SEEDS = {cfg: (1000 + cfg, 2000 + cfg, 3000 + cfg) for cfg in range(1, 6)}


# --------------------------------------------------------------------------- shapes
def node_shapes(nodes):
    """Output (C,H,W) of every node; an fc output is (dout,1,1)."""
    shapes = []
    for i, n in enumerate(nodes):
        k = n["kind"]
        if k == "input":
            shapes.append(tuple(int(v) for v in n["shape"]))
        elif k == "fc":
            shapes.append((int(n["W"].shape[0]), 1, 1))
        elif k == "conv":
            ci, hi, wi = shapes[n["src"]]
            co, ci2, kh, kw = n["W"].shape
            assert ci == ci2 and kh == kw, (i, ci, ci2)
            s, p = n["stride"], n["pad"]
            ho = (hi + 2 * p - kh) // s + 1
            wo = (wi + 2 * p - kw) // s + 1
            shapes.append((int(co), int(ho), int(wo)))
        elif k == "avgpool":
            c, hi, wi = shapes[n["src"]]
            kk, s, p = n["k"], n["stride"], n["pad"]
            shapes.append((int(c), (hi + 2 * p - kk) // s + 1, (wi + 2 * p - kk) // s + 1))
        elif k in ("relu", "bn"):
            shapes.append(shapes[n["src"]])
        elif k == "add":
            assert shapes[n["src"]] == shapes[n["src2"]], (i, shapes[n["src"]], shapes[n["src2"]])
            shapes.append(shapes[n["src"]])
        else:
            raise ValueError(k)
    return shapes


# --------------------------------------------------------------------------- layer makers
class _Builder:
    def __init__(self, in_shape, rng):
        self.nodes = [{"kind": "input", "shape": tuple(in_shape)}]
        self.rng = rng

    @property
    def last(self):
        return len(self.nodes) - 1

    def shape(self, i):
        return node_shapes(self.nodes)[i]

    def fc(self, dout, src=None):
        src = self.last if src is None else src
        c, h, w = self.shape(src)
        din = c * h * w
        W = self.rng.normal(0.0, np.sqrt(2.0 / din), size=(dout, din)).astype(np.float32)
        bnd = 1.0 / np.sqrt(din)
        b = self.rng.uniform(-bnd, bnd, size=dout).astype(np.float32)
        self.nodes.append({"kind": "fc", "src": src, "W": W, "b": b})
        return self.last

    def conv(self, cout, k, stride, pad, src=None):
        src = self.last if src is None else src
        cin = self.shape(src)[0]
        fan_in = cin * k * k
        W = self.rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(cout, cin, k, k)).astype(np.float32)
        bnd = 1.0 / np.sqrt(fan_in)
        b = self.rng.uniform(-bnd, bnd, size=cout).astype(np.float32)
        self.nodes.append({"kind": "conv", "src": src, "W": W, "b": b,
                           "stride": int(stride), "pad": int(pad)})
        return self.last

    def bn(self, src=None):
        """Batch normalisation with fixed, seeded statistics (the evaluation-mode layer)."""
        src = self.last if src is None else src
        c = self.shape(src)[0]
        r = self.rng
        self.nodes.append({"kind": "bn", "src": src,
                           "gamma": r.uniform(0.5, 1.5, c).astype(np.float32),
                           "beta": r.uniform(-0.1, 0.1, c).astype(np.float32),
                           "mean": r.normal(0.0, 0.1, c).astype(np.float32),
                           "var": r.uniform(0.5, 1.5, c).astype(np.float32), "eps": 1e-5})
        return self.last

    def avgpool(self, k, stride, pad=0, src=None):
        src = self.last if src is None else src
        self.nodes.append({"kind": "avgpool", "src": src, "k": int(k), "stride": int(stride), "pad": int(pad)})
        return self.last

    def relu(self, src=None):
        src = self.last if src is None else src
        self.nodes.append({"kind": "relu", "src": src})
        return self.last

    def add(self, a, b):
        self.nodes.append({"kind": "add", "src": a, "src2": b})
        return self.last


def fc_net(widths, seed, in_shape=None):
    """FC ReLU net with the given widths [d0, h1, ..., out]."""
    rng = np.random.default_rng(seed)
    in_shape = in_shape or (widths[0], 1, 1)
    B = _Builder(in_shape, rng)
    for i, w in enumerate(widths[1:]):
        B.fc(w)
        if i < len(widths) - 2:
            B.relu()
    return B.nodes


def convsmall(seed, in_shape=(1, 28, 28), c1=16, c2=32, hidden=100, n_out=10):
    """ConvSmall shape (Table 4): Conv c1 4x4/2/0, Conv c2 4x4/2/0, FC hidden, FC n_out."""
    B = _Builder(in_shape, np.random.default_rng(seed))
    B.conv(c1, 4, 2, 0); B.relu()
    B.conv(c2, 4, 2, 0); B.relu()
    B.fc(hidden); B.relu()
    B.fc(n_out)
    return B.nodes


def convbig(seed, in_shape=(3, 32, 32), ch=(32, 32, 64, 64), hidden=(512, 512), n_out=10):
    """ConvBig shape (Table 4, CIFAR10 column with padding 1)."""
    B = _Builder(in_shape, np.random.default_rng(seed))
    B.conv(ch[0], 3, 1, 1); B.relu()
    B.conv(ch[1], 4, 2, 1); B.relu()
    B.conv(ch[2], 3, 1, 1); B.relu()
    B.conv(ch[3], 4, 2, 1); B.relu()
    for h in hidden:
        B.fc(h); B.relu()
    B.fc(n_out)
    return B.nodes


def _res_block(B, cout, bn=False):
    x = B.last
    B.conv(cout, 3, 2, 1, src=x)
    if bn:
        B.bn()
    B.relu()
    b = B.conv(cout, 3, 1, 1)
    if bn:
        b = B.bn()
    s = B.conv(cout, 1, 2, 0, src=x)
    if bn:
        s = B.bn()
    B.add(b, s)
    return B.relu()


def resnet6(seed, in_shape=(3, 32, 32), ch=(16, 32, 64), hidden=100, n_out=10, stem_stride=2):
    """ResNet6 shape (Table 5): stem conv, two residual blocks, FC hidden, FC n_out.

    The stem is taken with stride 2 (padding 1); with that reading the ReLU
    node count equals the 10,340 of Table 3.
    """
    B = _Builder(in_shape, np.random.default_rng(seed))
    B.conv(ch[0], 3, stem_stride, 1); B.relu()
    for c in ch[1:]:
        _res_block(B, c)
    B.fc(hidden); B.relu()
    B.fc(n_out)
    return B.nodes


def resnet8(seed, in_shape=(3, 32, 32), ch=(16, 32, 64, 128), hidden=100, n_out=10, bn=False, pool=None):
    """ResNet8 shape (Table 5): stem conv 16 3x3/2/1, three residual blocks, FC hidden, FC n_out.

    bn=True puts a batch-normalisation layer after every convolution (before its ReLU or residual
    addition); pool=(k, s) an average pooling k x k / s after the last block."""
    B = _Builder(in_shape, np.random.default_rng(seed))
    B.conv(ch[0], 3, 2, 1)
    if bn:
        B.bn()
    B.relu()
    for c in ch[1:]:
        _res_block(B, c, bn=bn)
    if pool:
        B.avgpool(pool[0], pool[1])
    B.fc(hidden); B.relu()
    B.fc(n_out)
    return B.nodes


def tiny_fc(seed, widths=(3, 4, 4, 2)):
    return fc_net(list(widths), seed)


def tiny_conv(seed, in_shape=(1, 6, 6), c1=2, c2=3, hidden=4, n_out=3):
    """Small conv net: Conv c1 3x3/2/1, Conv c2 3x3/1/0 (k4 s2 when possible), FC."""
    B = _Builder(in_shape, np.random.default_rng(seed))
    B.conv(c1, 3, 2, 1); B.relu()
    B.conv(c2, 2, 1, 0); B.relu()
    B.fc(hidden); B.relu()
    B.fc(n_out)
    return B.nodes


def tiny_resnet(seed, in_shape=(1, 4, 4), ch=(2, 2), n_out=2, bn=False, pool=None):
    """Stem conv 3x3/1/1, one residual block, FC; bn=True adds batch normalisation after every
    convolution, pool=(k, s) an average pooling after the block."""
    B = _Builder(in_shape, np.random.default_rng(seed))
    B.conv(ch[0], 3, 1, 1)
    if bn:
        B.bn()
    B.relu()
    _res_block(B, ch[1], bn=bn)
    if pool:
        B.avgpool(pool[0], pool[1])
    B.fc(n_out)
    return B.nodes


def tiny_resnet_bn(seed):
    return tiny_resnet(seed, in_shape=(1, 4, 4), ch=(2, 3), bn=True, pool=(2, 2))


def make_net(cfg, seed=None, scale="full"):
    """Network of a configuration: 1 FC 784-100-100-10, 2 ConvSmall, 3 ConvBig, 4 ResNet6.

    scale="small" gives a down-scaled net of the same topology (for tests).
    """
    seed = CONFIG_SEEDS[cfg][0] if seed is None else seed
    if cfg == 1:
        if scale == "small":
            return fc_net([64, 24, 24, 10], seed, in_shape=(1, 8, 8))
        return fc_net([784, 100, 100, 10], seed, in_shape=(1, 28, 28))
    if cfg == 2:
        if scale == "small":
            return convsmall(seed, in_shape=(1, 12, 12), c1=4, c2=8, hidden=20)
        return convsmall(seed)
    if cfg == 3:
        if scale == "small":
            return convbig(seed, in_shape=(3, 8, 8), ch=(4, 4, 8, 8), hidden=(32, 32))
        return convbig(seed)
    if cfg == 4:
        if scale == "small":
            return resnet6(seed, in_shape=(3, 8, 8), ch=(4, 8, 8), hidden=20)
        return resnet6(seed)
    raise ValueError(cfg)


# --------------------------------------------------------------------------- inputs and specs
def make_input(shape, eps, seed):
    """x0 ~ U[0,1]^shape (flattened) and the clipped L-infinity box."""
    rng = np.random.default_rng(seed)
    d = int(np.prod(shape))
    x0 = rng.uniform(0.0, 1.0, size=d).astype(np.float32)
    lo = np.maximum(x0 - np.float32(eps), 0.0).astype(np.float32)
    hi = np.minimum(x0 + np.float32(eps), 1.0).astype(np.float32)
    return x0, lo, hi


def forward_logits(nodes, x):
    """Plain float64 forward evaluation f(x) of a batch of inputs x [R, d0].

    Used only to choose the label of a robustness specification."""
    shapes = node_shapes(nodes)
    x = np.asarray(x, dtype=np.float64)
    vals = [x.reshape(x.shape[0], -1)]
    for i, n in enumerate(nodes[1:], start=1):
        k = n["kind"]
        if k == "fc":
            vals.append(vals[n["src"]] @ n["W"].astype(np.float64).T + n["b"].astype(np.float64))
        elif k == "conv":
            import torch  # library convolution, float64 on the CPU
            ci, hi, wi = shapes[n["src"]]
            z = torch.from_numpy(vals[n["src"]].reshape(-1, ci, hi, wi))
            W = torch.from_numpy(n["W"].astype(np.float64))
            b = torch.from_numpy(n["b"].astype(np.float64))
            out = torch.nn.functional.conv2d(z, W, b, stride=n["stride"], padding=n["pad"])
            vals.append(out.reshape(out.shape[0], -1).numpy())
        elif k in ("bn", "avgpool"):
            import torch  # library layers, float64 on the CPU
            ci, hi, wi = shapes[n["src"]]
            z = torch.from_numpy(vals[n["src"]].reshape(-1, ci, hi, wi))
            if k == "bn":
                t = lambda key: torch.from_numpy(np.asarray(n[key], np.float64))
                out = torch.nn.functional.batch_norm(z, t("mean"), t("var"), t("gamma"), t("beta"), training=False,
                                                     eps=float(n["eps"]))
            else:
                out = torch.nn.functional.avg_pool2d(z, n["k"], n["stride"], n["pad"], count_include_pad=True)
            vals.append(out.reshape(out.shape[0], -1).numpy())
        elif k == "relu":
            vals.append(np.maximum(vals[n["src"]], 0.0))
        elif k == "add":
            vals.append(vals[n["src"]] + vals[n["src2"]])
    return vals[-1]


def make_spec(nodes, x0, n_spec=None, target=None, seed=0):
    """Robustness spec rows e_c - e_j for the label c = argmax f(x0) (ties: lowest index).

    n_spec=None gives all j != c (n_out - 1 rows); target=j gives the single row vs j;
    n_spec=1 with target=None draws j != c at random (seeded).
    Returns (C [S, n_out] float32, c0 [S] float32, label c).
    """
    logits = forward_logits(nodes, np.asarray(x0)[None, :])[0]
    n_out = logits.shape[0]
    c = int(np.argmax(logits))
    others = [j for j in range(n_out) if j != c]
    if target is not None:
        js = [int(target)]
    elif n_spec is None or n_spec == n_out - 1:
        js = others
    else:
        rng = np.random.default_rng(seed)
        js = list(rng.choice(others, size=n_spec, replace=False))
    C = np.zeros((len(js), n_out), dtype=np.float32)
    for r, j in enumerate(js):
        C[r, c] = 1.0
        C[r, j] = -1.0
    return C, np.zeros(len(js), dtype=np.float32), c


# --------------------------------------------------------------------------- split sets
def make_split_sets(unstable, n_sub, depth_lo, depth_hi, seed):
    """Random split sets among root-unstable neurons.

    unstable: list over ReLU layers of arrays of unstable neuron indices.
    Returns n_sub lists of (relu_layer, neuron, sign) with sign +1 for the
    positive phase (zhat >= 0) and -1 for the negative phase; depth ~ U{lo..hi}
    capped by the number of candidates; neurons distinct within a set.
    """
    rng = np.random.default_rng(seed)
    cand = [(k, int(j)) for k, arr in enumerate(unstable) for j in np.asarray(arr)]
    out = []
    for _ in range(n_sub):
        d = int(rng.integers(depth_lo, depth_hi + 1))
        d = min(d, len(cand))
        pick = rng.choice(len(cand), size=d, replace=False) if d > 0 else []
        signs = rng.choice([1, -1], size=d)
        out.append([(cand[p][0], cand[p][1], int(s)) for p, s in zip(pick, signs)])
    return out


# --------------------------------------------------------------------------- bundles
class Workload:
    """A verification query: net, centre point, box and spec."""

    def __init__(self, nodes, x0, lo, hi, C, c0, label, eps):
        self.nodes, self.x0, self.lo, self.hi = nodes, x0, lo, hi
        self.C, self.c0, self.label, self.eps = C, c0, label, eps

    @property
    def in_shape(self):
        return self.nodes[0]["shape"]


_EPS = {1: 0.02, 2: 0.03, 3: 2.0 / 255.0, 4: 1.0 / 255.0}


def make_workload(cfg, scale="full", eps=None, n_spec=None, seed_offset=0):
    net_seed, in_seed, _ = CONFIG_SEEDS[cfg]
    nodes = make_net(cfg, seed=net_seed + seed_offset, scale=scale)
    eps = _EPS[cfg] if eps is None else eps
    x0, lo, hi = make_input(nodes[0]["shape"], eps, in_seed + seed_offset)
    C, c0, label = make_spec(nodes, x0, n_spec=n_spec)
    return Workload(nodes, x0, lo, hi, C, c0, label, eps)
