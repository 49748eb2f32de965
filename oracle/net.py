"""Network arithmetic in float64 (oracle; test infrastructure only).

The network of Section 2.1: affine layers zhat = W z + b and ReLUs
z = max(0, zhat), generalised to a DAG of fc / conv / bn / avgpool / relu /
add nodes (Section 2.1 notes the method covers convolutional, residual,
batch-normalisation and average-pooling layers; the latter two are affine).

* bn: batch normalisation with fixed statistics, per channel c
  y = gamma_c (x - mean_c) / sqrt(var_c + eps) + beta_c;
* avgpool: the mean of each k x k window (stride s, zero padding p counted
  in the window, so the divisor is always k^2).

Everything here works on batches of row vectors [R, size]; conv tensors are
flattened in (C, H, W) order.
"""
from __future__ import annotations

import numpy as np


AFFINE_KINDS = ("fc", "conv", "bn", "avgpool")


class Net:
    """float64 copy of a node list (format documented in the workloads module)."""

    def __init__(self, nodes):
        self.nodes = []
        for n in nodes:
            m = dict(n)
            if "W" in m:
                m["W"] = np.asarray(m["W"], dtype=np.float64)
                m["b"] = np.asarray(m["b"], dtype=np.float64)
            for key in ("gamma", "beta", "mean", "var"):
                if key in m:
                    m[key] = np.asarray(m[key], dtype=np.float64)
            self.nodes.append(m)
        self.shapes = _shapes(self.nodes)
        self.sizes = [int(np.prod(s)) for s in self.shapes]
        self.relus = [i for i, n in enumerate(self.nodes) if n["kind"] == "relu"]
        self.n_out = self.sizes[-1]

    def __len__(self):
        return len(self.nodes)

    def relu_layer(self, node_idx):
        return self.relus.index(node_idx)


def _shapes(nodes):
    shapes = []
    for n in nodes:
        k = n["kind"]
        if k == "input":
            shapes.append(tuple(int(v) for v in n["shape"]))
        elif k == "fc":
            shapes.append((n["W"].shape[0], 1, 1))
        elif k == "conv":
            ci, hi, wi = shapes[n["src"]]
            co, _, kk, _ = n["W"].shape
            s, p = n["stride"], n["pad"]
            shapes.append((co, (hi + 2 * p - kk) // s + 1, (wi + 2 * p - kk) // s + 1))
        elif k == "avgpool":
            c, hi, wi = shapes[n["src"]]
            kk, s, p = n["k"], n["stride"], n["pad"]
            shapes.append((c, (hi + 2 * p - kk) // s + 1, (wi + 2 * p - kk) // s + 1))
        elif k in ("relu", "bn"):
            shapes.append(shapes[n["src"]])
        elif k == "add":
            shapes.append(shapes[n["src"]])
    return shapes


# --------------------------------------------------------------------------- conv
def conv_apply(W, z, in_shape, out_shape, stride, pad):
    """Linear part of a 2-D convolution: out[co,y,x] = sum W[co,ci,ky,kx] z[ci, s*y+ky-p, s*x+kx-p]."""
    R = z.shape[0]
    ci, hi, wi = in_shape
    co, ho, wo = out_shape
    k = W.shape[2]
    s, p = stride, pad
    zp = np.zeros((R, ci, hi + 2 * p, wi + 2 * p))
    zp[:, :, p:p + hi, p:p + wi] = z.reshape(R, ci, hi, wi)
    out = np.zeros((R, co, ho, wo))
    for ky in range(k):
        for kx in range(k):
            patch = zp[:, :, ky:ky + s * (ho - 1) + 1:s, kx:kx + s * (wo - 1) + 1:s]
            out += np.einsum("rchw,oc->rohw", patch, W[:, :, ky, kx])
    return out.reshape(R, -1)


def conv_adjoint(W, a, in_shape, out_shape, stride, pad):
    """Adjoint (transpose) of conv_apply: maps a coefficient on the output to one on the input."""
    R = a.shape[0]
    ci, hi, wi = in_shape
    co, ho, wo = out_shape
    k = W.shape[2]
    s, p = stride, pad
    a4 = a.reshape(R, co, ho, wo)
    gp = np.zeros((R, ci, hi + 2 * p, wi + 2 * p))
    for ky in range(k):
        for kx in range(k):
            gp[:, :, ky:ky + s * (ho - 1) + 1:s, kx:kx + s * (wo - 1) + 1:s] += \
                np.einsum("rohw,oc->rchw", a4, W[:, :, ky, kx])
    return gp[:, :, p:p + hi, p:p + wi].reshape(R, -1)


# --------------------------------------------------------------------------- batch norm / pooling
def bn_scale(n):
    """Per-channel slope gamma / sqrt(var + eps) of a batch-normalisation node."""
    return n["gamma"] / np.sqrt(n["var"] + n["eps"])


def avgpool_apply(z, in_shape, out_shape, k, stride, pad):
    """out[c,y,x] = (1/k^2) sum_{ky,kx} z[c, s*y+ky-p, s*x+kx-p] (zero padding counted)."""
    R = z.shape[0]
    c, hi, wi = in_shape
    _, ho, wo = out_shape
    s, p = stride, pad
    zp = np.zeros((R, c, hi + 2 * p, wi + 2 * p))
    zp[:, :, p:p + hi, p:p + wi] = z.reshape(R, c, hi, wi)
    out = np.zeros((R, c, ho, wo))
    for ky in range(k):
        for kx in range(k):
            out += zp[:, :, ky:ky + s * (ho - 1) + 1:s, kx:kx + s * (wo - 1) + 1:s]
    return (out / (k * k)).reshape(R, -1)


def avgpool_adjoint(a, in_shape, out_shape, k, stride, pad):
    """Adjoint of avgpool_apply: each output coefficient spread evenly over its window."""
    R = a.shape[0]
    c, hi, wi = in_shape
    _, ho, wo = out_shape
    s, p = stride, pad
    a4 = a.reshape(R, c, ho, wo) / (k * k)
    gp = np.zeros((R, c, hi + 2 * p, wi + 2 * p))
    for ky in range(k):
        for kx in range(k):
            gp[:, :, ky:ky + s * (ho - 1) + 1:s, kx:kx + s * (wo - 1) + 1:s] += a4
    return gp[:, :, p:p + hi, p:p + wi].reshape(R, -1)


# --------------------------------------------------------------------------- affine nodes
def affine_apply(net, i, z):
    """W z (no bias) for affine node i on a batch z [R, d_in]."""
    n = net.nodes[i]
    if n["kind"] == "fc":
        return z @ n["W"].T
    if n["kind"] == "conv":
        return conv_apply(n["W"], z, net.shapes[n["src"]], net.shapes[i], n["stride"], n["pad"])
    if n["kind"] == "bn":
        c, h, w = net.shapes[i]
        return z * np.repeat(bn_scale(n), h * w)[None, :]
    if n["kind"] == "avgpool":
        return avgpool_apply(z, net.shapes[n["src"]], net.shapes[i], n["k"], n["stride"], n["pad"])
    raise ValueError(n["kind"])


def affine_adjoint(net, i, a):
    """a W for affine node i: the Eq. 2 coefficient map a^(i-1) = ahat^(i) W^(i)."""
    n = net.nodes[i]
    if n["kind"] == "fc":
        return a @ n["W"]
    if n["kind"] == "conv":
        return conv_adjoint(n["W"], a, net.shapes[n["src"]], net.shapes[i], n["stride"], n["pad"])
    if n["kind"] == "bn":
        c, h, w = net.shapes[i]
        return a * np.repeat(bn_scale(n), h * w)[None, :]
    if n["kind"] == "avgpool":
        return avgpool_adjoint(a, net.shapes[n["src"]], net.shapes[i], n["k"], n["stride"], n["pad"])
    raise ValueError(n["kind"])


def bias_vector(net, i):
    """Bias of affine node i expanded to one entry per output neuron."""
    n = net.nodes[i]
    if n["kind"] == "fc":
        return n["b"]
    c, h, w = net.shapes[i]
    if n["kind"] == "bn":
        return np.repeat(n["beta"] - n["mean"] * bn_scale(n), h * w)
    if n["kind"] == "avgpool":
        return np.zeros(c * h * w)
    return np.repeat(n["b"], h * w)


# --------------------------------------------------------------------------- forward / IBP
def forward_all(net, x):
    """All node values of the exact forward pass f(x) (Section 2.1) for x [R, d0]."""
    vals = [np.asarray(x, dtype=np.float64).reshape(len(x), -1)]
    for i, n in enumerate(net.nodes[1:], start=1):
        k = n["kind"]
        if k in AFFINE_KINDS:
            vals.append(affine_apply(net, i, vals[n["src"]]) + bias_vector(net, i))
        elif k == "relu":
            vals.append(np.maximum(vals[n["src"]], 0.0))
        elif k == "add":
            vals.append(vals[n["src"]] + vals[n["src2"]])
    return vals


def forward(net, x):
    return forward_all(net, x)[-1]


def interval_forward(net, lo, hi, relu_bounds, upto):
    """Interval bound propagation (the cheap bounding method the paper cites for l/u).

    relu_bounds: dict relu-node -> (l, u) of its input, already known; those
    are used (intersected with the propagated interval) at each ReLU.
    Returns (L, U) lists for nodes 0..upto.
    """
    L = [np.asarray(lo, dtype=np.float64)]
    U = [np.asarray(hi, dtype=np.float64)]
    for i in range(1, upto + 1):
        n = net.nodes[i]
        k = n["kind"]
        if k in AFFINE_KINDS:
            lo_s, hi_s = L[n["src"]][None, :], U[n["src"]][None, :]
            mid = (lo_s + hi_s) / 2.0
            rad = (hi_s - lo_s) / 2.0
            c = affine_apply(net, i, mid)[0]
            r = _abs_affine(net, i, rad)[0]
            b = bias_vector(net, i)
            L.append(c - r + b)
            U.append(c + r + b)
        elif k == "relu":
            l, u = L[n["src"]], U[n["src"]]
            if i in relu_bounds:
                l = np.maximum(l, relu_bounds[i][0])
                u = np.minimum(u, relu_bounds[i][1])
            L.append(np.maximum(l, 0.0))
            U.append(np.maximum(u, 0.0))
        elif k == "add":
            L.append(L[n["src"]] + L[n["src2"]])
            U.append(U[n["src"]] + U[n["src2"]])
    return L, U


def _abs_affine(net, i, z):
    """|W| z for affine node i (the radius of the interval image)."""
    n = net.nodes[i]
    if n["kind"] == "fc":
        return z @ np.abs(n["W"]).T
    if n["kind"] == "bn":
        c, h, w = net.shapes[i]
        return z * np.repeat(np.abs(bn_scale(n)), h * w)[None, :]
    if n["kind"] == "avgpool":
        return affine_apply(net, i, z)      # nonnegative weights
    return conv_apply(np.abs(n["W"]), z, net.shapes[n["src"]], net.shapes[i], n["stride"], n["pad"])
