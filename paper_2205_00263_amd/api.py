"""Python binding of the engine: numpy in, numpy out; every step runs in the HIP library.

Names follow the C ABI (bound_init, branch_split, bound_optimize,
query_submit, query_poll).  Arrays are converted to contiguous float32 /
int32 / int64 and handed over as plain pointers.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import check, lib

__all__ = ["Net", "Problem", "use_torch_plumbing", "mnc_to_csr", "set_index", "set_kernel_variants",
           "get_kernel_variants", "VARIANTS", "split_costs", "relu_hull"]


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _ptr(a, ctype=C.c_float):
    return a.ctypes.data_as(C.POINTER(ctype))


def set_index(key):
    """Parameter-set index: 'final' -> 0, (m, +1) -> 2m-1 (lower bounds of ReLU layer m), (m, -1) -> 2m."""
    if key == "final":
        return 0
    m, s = key
    return 2 * m - 1 if s > 0 else 2 * m


# --------------------------------------------------------------------------- plumbing
_torch_hooks = {}


def use_torch_plumbing(enable=True):
    """Route device allocations through PyTorch's caching allocator and launch on torch's current stream."""
    L = lib()
    if not enable:
        check(L.mnb_set_allocator(_lib.ALLOC_FN(), _lib.FREE_FN(), None))
        check(L.mnb_set_stream(None))
        _torch_hooks.clear()
        return
    import torch
    stream = torch.cuda.current_stream()
    dev = torch.cuda.current_device()

    def _alloc(nbytes, ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream))
        except Exception:
            return None

    def _free(ptr, ctx):
        if ptr:
            torch.cuda.caching_allocator_delete(ptr)

    a, f = _lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free)
    _torch_hooks.update(alloc=a, free=f, stream=stream)
    check(L.mnb_set_allocator(a, f, None))
    check(L.mnb_set_stream(C.c_void_p(stream.cuda_stream)))


# --------------------------------------------------------------------------- network
def _layer_array(nodes):
    """ctypes array of mnb_layer for a node list (workloads format) and the buffers it points into."""
    from workloads import node_shapes  # shapes only
    shapes = node_shapes(nodes)
    arr = (_lib.Layer * len(nodes))()
    keep = []
    kinds = {"input": _lib.MNB_INPUT, "fc": _lib.MNB_FC, "conv": _lib.MNB_CONV,
             "relu": _lib.MNB_RELU, "add": _lib.MNB_ADD, "bn": _lib.MNB_BN, "avgpool": _lib.MNB_AVGPOOL}
    for i, n in enumerate(nodes):
        L = arr[i]
        L.kind = kinds[n["kind"]]
        L.src = n.get("src", -1)
        L.src2 = n.get("src2", -1)
        for t in range(3):
            L.out_chw[t] = shapes[i][t]
            if i > 0:
                L.in_chw[t] = shapes[n["src"]][t]
        if n["kind"] in ("fc", "conv"):
            W, b = _f32(n["W"]), _f32(n["b"])
            keep += [W, b]
            L.W, L.b = _ptr(W), _ptr(b)
        if n["kind"] == "conv":
            L.k = n["W"].shape[2]
            L.stride, L.pad = n["stride"], n["pad"]
        if n["kind"] == "bn":
            stats = np.ascontiguousarray(np.concatenate([np.asarray(n[k], np.float32).ravel()
                                                         for k in ("gamma", "beta", "mean", "var")]))
            keep.append(stats)
            L.W, L.eps = _ptr(stats), float(n["eps"])
        if n["kind"] == "avgpool":
            L.k, L.stride, L.pad = n["k"], n["stride"], n["pad"]
    return arr, keep


def split_costs(nodes, mnc_counts=None):
    """mnb_split_costs: direct split cost of each ReLU layer (Appendix B) of a node list, with
    mnc_counts [n_relu] multi-neuron constraints per layer (None: none); 1 / cost is a layer weight
    of Problem.branch_scores.  Host-only call of the library (no GPU needed)."""
    arr, _keep = _layer_array(nodes)
    n_relu = sum(1 for n in nodes if n["kind"] == "relu")
    p = None if mnc_counts is None else np.ascontiguousarray(mnc_counts, np.int32)
    if p is not None and p.shape != (n_relu,):
        raise ValueError("mnc_counts needs one entry per ReLU layer")
    out = np.zeros(n_relu, np.float64)
    check(lib().mnb_split_costs(arr, len(nodes), _ptr(p, C.c_int32) if p is not None else None,
                                out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


class Net:
    """A network (node list in the workloads format) copied to the device."""

    def __init__(self, nodes):
        arr, keep = _layer_array(nodes)
        h = C.c_void_p()
        check(lib().mnb_net_create(arr, len(nodes), C.byref(h)))
        self.h = h
        self.nodes = nodes
        nr = C.c_int()
        sizes = (C.c_int * 64)()
        d_in, d_out = C.c_int(), C.c_int()
        check(lib().mnb_net_info(h, C.byref(nr), sizes, C.byref(d_in), C.byref(d_out)))
        self.relu_sizes = [sizes[i] for i in range(nr.value)]
        self.d0, self.n_out = d_in.value, d_out.value
        self.relu_nodes = [i for i, n in enumerate(nodes) if n["kind"] == "relu"]

    @property
    def n_relu(self):
        return len(self.relu_sizes)

    def split_costs(self, mnc_counts=None):
        """split_costs of this net's node list."""
        return split_costs(self.nodes, mnc_counts)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                lib().mnb_net_destroy(h)
            except Exception:
                pass
            self.h = None

    # kernel-level entry points (device pointers, e.g. torch tensors' data_ptr())
    def fc_backsub(self, node, A_ptr, C_ptr, M, accumulate=False):
        check(lib().mnb_kernel_fc_backsub(self.h, node, C.c_void_p(A_ptr), C.c_void_p(C_ptr), M, int(accumulate)))

    def conv_backsub(self, node, A_ptr, C_ptr, M, accumulate=False):
        check(lib().mnb_kernel_conv_backsub(self.h, node, C.c_void_p(A_ptr), C.c_void_p(C_ptr), M,
                                            int(accumulate)))

    def fc_forward(self, node, G_ptr, C_ptr, M):
        check(lib().mnb_kernel_fc_forward(self.h, node, C.c_void_p(G_ptr), C.c_void_p(C_ptr), M))

    def conv_forward(self, node, G_ptr, C_ptr, M):
        check(lib().mnb_kernel_conv_forward(self.h, node, C.c_void_p(G_ptr), C.c_void_p(C_ptr), M))

    @staticmethod
    def sync():
        check(lib().mnb_sync())


# kernel variants (mnb_set_kernel_variants): bits forcing the more general kernel of a step
VARIANTS = {"valu_bottom": 1, "no_tap_convt": 2, "no_pair_conv": 4, "no_row_conv": 8, "no_window": 16,
            "no_fused_bottom": 32, "no_patch": 64, "no_cone": 128,
            "no_first_conv": 256, "no_win_conv": 512}


def set_kernel_variants(mask):
    """Force the general kernels selected by `mask` (bits of VARIANTS) for later calls; returns the
    previous mask.  All variants compute the same bounds to FP32 rounding."""
    return int(lib().mnb_set_kernel_variants(int(mask)))


def get_kernel_variants():
    return int(lib().mnb_get_kernel_variants())


def mnc_to_csr(P, Phat, p):
    """Dense (P, Phat, p) of one layer -> CSR arrays over the union of their nonzeros."""
    P = np.asarray(P, dtype=np.float64)
    Phat = np.asarray(Phat, dtype=np.float64)
    e = P.shape[0]
    row_ptr = [0]
    cols, pv, hv = [], [], []
    for r in range(e):
        nz = np.nonzero((P[r] != 0) | (Phat[r] != 0))[0]
        cols += list(nz)
        pv += list(P[r, nz])
        hv += list(Phat[r, nz])
        row_ptr.append(len(cols))
    return (np.asarray(row_ptr, np.int32), np.asarray(cols, np.int32), np.asarray(pv, np.float32),
            np.asarray(hv, np.float32), np.asarray(p, np.float32))


class _MncPack:
    """ctypes array of mnb_mnc plus the numpy buffers it points into."""

    def __init__(self, mncs):
        # mncs: dict relu-layer m -> (row_ptr, col, P, Phat, p)
        self.keep = []
        self.arr = (_lib.Mnc * max(1, len(mncs)))()
        for t, (m, (rp, col, P, Ph, p)) in enumerate(sorted(mncs.items())):
            rp, col = np.ascontiguousarray(rp, np.int32), np.ascontiguousarray(col, np.int32)
            P, Ph, p = _f32(P), _f32(Ph), _f32(p)
            self.keep += [rp, col, P, Ph, p]
            c = self.arr[t]
            c.layer, c.e = int(m), int(len(p))
            c.row_ptr, c.col = _ptr(rp, C.c_int32), _ptr(col, C.c_int32)
            c.P, c.Phat, c.p = _ptr(P), _ptr(Ph), _ptr(p)
        self.n = len(mncs)


# --------------------------------------------------------------------------- problem
class Problem:
    """Device-resident pool of subproblems of one network."""

    def __init__(self, net: Net, n_spec: int, capacity: int = 1024, max_mnc: int = 0):
        self.net = net
        self.S = int(n_spec)
        self.max_mnc = int(max_mnc)
        h = C.c_void_p()
        check(lib().mnb_problem_create(net.h, self.S, int(capacity), self.max_mnc, C.byref(h)))
        self.h = h
        self.total_d = sum(net.relu_sizes)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                lib().mnb_problem_destroy(h)
            except Exception:
                pass
            self.h = None

    def bound_init(self, lo, hi, Cm, c0, mncs=None):
        lo, hi, Cm, c0 = _f32(lo), _f32(hi), _f32(Cm), _f32(c0)
        assert Cm.shape == (self.S, self.net.n_out)
        pack = _MncPack(mncs or {})
        rid = C.c_int64()
        lb = np.zeros(self.S, np.float32)
        ub = np.zeros(self.S, np.float32)
        check(lib().bound_init(self.h, _ptr(lo), _ptr(hi), _ptr(Cm), _ptr(c0),
                               pack.arr if pack.n else None, pack.n, C.byref(rid), _ptr(lb), _ptr(ub)))
        return rid.value, lb, ub

    def branch_split(self, parents, layers, neurons):
        parents = np.ascontiguousarray(parents, np.int64)
        layers = np.ascontiguousarray(layers, np.int32)
        neurons = np.ascontiguousarray(neurons, np.int32)
        n = len(parents)
        child = np.zeros(2 * n, np.int64)
        check(lib().branch_split(self.h, _ptr(parents, C.c_int64), _ptr(layers, C.c_int32),
                                 _ptr(neurons, C.c_int32), n, _ptr(child, C.c_int64)))
        return child

    @staticmethod
    def opt_cfg(steps=20, lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8, recompute_intermediate=True,
                ckpt_stride=0, mem_budget=0):
        cfg = _lib.OptCfg()
        lib().mnb_opt_cfg_default(C.byref(cfg))
        cfg.steps, cfg.lr, cfg.beta1, cfg.beta2, cfg.eps = steps, lr, beta1, beta2, eps
        cfg.recompute_intermediate = int(recompute_intermediate)
        cfg.ckpt_stride = int(ckpt_stride)
        cfg.mem_budget = int(mem_budget)
        return cfg

    def bound_optimize(self, ids, want_branch=False, **kw):
        ids = np.ascontiguousarray(ids, np.int64)
        n = len(ids)
        cfg = self.opt_cfg(**kw)
        lb = np.zeros((n, self.S), np.float32)
        ub = np.zeros((n, self.S), np.float32)
        bl = np.zeros(n, np.int32) if want_branch else None
        bn = np.zeros(n, np.int32) if want_branch else None
        check(lib().bound_optimize(self.h, _ptr(ids, C.c_int64), n, C.byref(cfg), _ptr(lb), _ptr(ub),
                                   _ptr(bl, C.c_int32) if want_branch else None,
                                   _ptr(bn, C.c_int32) if want_branch else None))
        if want_branch:
            return lb, ub, bl, bn
        return lb, ub

    def optimize_begin(self, ids, **kw):
        """bound_optimize_begin: an OptSession over the subproblems `ids` (keywords as bound_optimize)."""
        return OptSession(self, ids, self.opt_cfg(**kw))

    def get_bounds(self, sid, layer):
        d = self.net.relu_sizes[layer]
        l = np.zeros(d, np.float32)
        u = np.zeros(d, np.float32)
        S = np.zeros(d, np.int8)
        check(lib().mnb_get_bounds(self.h, int(sid), int(layer), _ptr(l), _ptr(u), _ptr(S, C.c_int8)))
        return l, u, S

    def get_params(self, sid, set_idx):
        a = np.zeros(self.total_d, np.float32)
        b = np.zeros(self.total_d, np.float32)
        g = np.zeros(max(1, self.net.n_relu * self.max_mnc), np.float32)
        check(lib().mnb_get_params(self.h, int(sid), int(set_idx), _ptr(a), _ptr(b), _ptr(g)))
        return a, b, g[: self.net.n_relu * self.max_mnc]

    def set_params(self, sid, set_idx, alpha=None, beta=None, gamma=None):
        a = _f32(alpha) if alpha is not None else None
        b = _f32(beta) if beta is not None else None
        g = _f32(gamma) if gamma is not None else None
        check(lib().mnb_set_params(self.h, int(sid), int(set_idx), _ptr(a) if a is not None else None,
                                   _ptr(b) if b is not None else None, _ptr(g) if g is not None else None))

    def set_params_device(self, sid, set_idx, alpha_ptr=0, beta_ptr=0, gamma_ptr=0):
        """mnb_set_params_device: parameters from device arrays (pointers, 0 = leave unchanged)."""
        v = lambda p: C.c_void_p(p) if p else None
        check(lib().mnb_set_params_device(self.h, int(sid), int(set_idx), v(alpha_ptr), v(beta_ptr), v(gamma_ptr)))

    def bound_grad_device(self, sid, set_idx, lb_ptr=0, ga_ptr=0, gb_ptr=0, gg_ptr=0):
        """mnb_bound_grad_device: row bounds and gradients into device arrays; returns the row count."""
        v = lambda p: C.c_void_p(p) if p else None
        rows = C.c_int()
        check(lib().mnb_bound_grad_device(self.h, int(sid), int(set_idx), C.byref(rows), v(lb_ptr), v(ga_ptr),
                                          v(gb_ptr), v(gg_ptr)))
        return rows.value

    def bound_grad(self, sid, set_idx):
        rows = C.c_int()
        lbr = np.zeros(max(self.S, max(self.net.relu_sizes) * 1), np.float32)
        ga = np.zeros(self.total_d, np.float32)
        gb = np.zeros(self.total_d, np.float32)
        gg = np.zeros(max(1, self.net.n_relu * self.max_mnc), np.float32)
        check(lib().mnb_bound_grad(self.h, int(sid), int(set_idx), C.byref(rows), _ptr(lbr), _ptr(ga), _ptr(gb),
                                   _ptr(gg)))
        return lbr[: rows.value], ga, gb, gg[: self.net.n_relu * self.max_mnc]

    def branch_scores(self, ids, layer_weight=None, want_scores=False):
        """Active constraint scores (Section 3.4) of the subproblems `ids` from their spec-row
        gamma: the chosen (layer, neuron) per subproblem (-1 without a candidate) and, with
        want_scores, the scores [n, sum of ReLU widths] (-inf for non-candidates).  layer_weight
        [n_relu] multiplies layer i's scores; 1 / split_costs(...) gives cost adjusted branching."""
        ids = np.ascontiguousarray(ids, np.int64)
        n = len(ids)
        w = None if layer_weight is None else _f32(layer_weight)
        if w is not None and w.shape != (self.net.n_relu,):
            raise ValueError("layer_weight needs one entry per ReLU layer")
        sc = np.zeros((n, self.total_d), np.float32) if want_scores else None
        bl = np.zeros(n, np.int32)
        bn = np.zeros(n, np.int32)
        check(lib().mnb_branch_scores(self.h, _ptr(ids, C.c_int64), n, _ptr(w) if w is not None else None,
                                      _ptr(sc) if want_scores else None, _ptr(bl, C.c_int32), _ptr(bn, C.c_int32)))
        return (bl, bn, sc) if want_scores else (bl, bn)

    def contribution_scores(self, ids, want_scores=True):
        """mnb_contribution_scores: the alpha-contribution branching scores of bound_optimize at the
        subproblems' current parameters and bounds: (layer, neuron) per subproblem and, with
        want_scores, the scores [n, sum of ReLU widths] (-inf for non-candidates)."""
        ids = np.ascontiguousarray(ids, np.int64)
        n = len(ids)
        sc = np.zeros((n, self.total_d), np.float32) if want_scores else None
        bl = np.zeros(n, np.int32)
        bn = np.zeros(n, np.int32)
        check(lib().mnb_contribution_scores(self.h, _ptr(ids, C.c_int64), n, _ptr(sc) if want_scores else None,
                                            _ptr(bl, C.c_int32), _ptr(bn, C.c_int32)))
        return (bl, bn, sc) if want_scores else (bl, bn)

    def octahedral_bounds(self, sid, layer, groups):
        """mnb_octahedral_bounds: lb [n, 26] of the groups [n, 3] of ReLU layer `layer`."""
        g = np.ascontiguousarray(groups, np.int32).reshape(-1, 3)
        lb = np.zeros((len(g), 26), np.float32)
        check(lib().mnb_octahedral_bounds(self.h, int(sid), int(layer), _ptr(g, C.c_int32), len(g), _ptr(lb)))
        return lb

    def mnc_generate(self, sid, cap=500):
        """mnb_mnc_generate: constraints of every ReLU layer of the query of root `sid`; counts per layer."""
        e = np.zeros(self.net.n_relu, np.int32)
        check(lib().mnb_mnc_generate(self.h, int(sid), int(cap), _ptr(e, C.c_int32)))
        return e

    def get_mnc(self, sid, layer):
        """mnb_get_mnc: (row_ptr, col, P, Phat, p) of the query's constraints of one ReLU layer."""
        E = max(self.max_mnc, 1)
        e = C.c_int()
        rp = np.zeros(E + 1, np.int32)
        col = np.zeros(4 * E, np.int32)
        P_ = np.zeros(4 * E, np.float32)
        H_ = np.zeros(4 * E, np.float32)
        p = np.zeros(E, np.float32)
        check(lib().mnb_get_mnc(self.h, int(sid), int(layer), C.byref(e), _ptr(rp, C.c_int32), _ptr(col, C.c_int32),
                                _ptr(P_), _ptr(H_), _ptr(p)))
        n = e.value
        nnz = int(rp[n])
        return rp[:n + 1].copy(), col[:nnz].copy(), P_[:nnz].copy(), H_[:nnz].copy(), p[:n].copy()

    def release(self, ids):
        ids = np.ascontiguousarray(ids, np.int64)
        check(lib().mnb_release(self.h, _ptr(ids, C.c_int64), len(ids)))

    def usage(self):
        u, c = C.c_int64(), C.c_int64()
        check(lib().mnb_problem_usage(self.h, C.byref(u), C.byref(c)))
        return u.value, c.value


class OptSession:
    """bound_optimize in steps: step() is one Adam iteration (evaluation, adjoint, update) of every
    subproblem of the session; end() runs the last evaluation and returns bound_optimize's outputs."""

    def __init__(self, problem, ids, cfg):
        self.problem = problem
        self.ids = np.ascontiguousarray(ids, np.int64)
        h = C.c_void_p()
        check(lib().bound_optimize_begin(problem.h, _ptr(self.ids, C.c_int64), len(self.ids), C.byref(cfg),
                                         C.byref(h)))
        self.h = h

    def step(self):
        check(lib().bound_optimize_step(self.h))

    def end(self, want_branch=False):
        n, S = len(self.ids), self.problem.S
        lb = np.zeros((n, S), np.float32)
        ub = np.zeros((n, S), np.float32)
        bl = np.zeros(n, np.int32) if want_branch else None
        bn = np.zeros(n, np.int32) if want_branch else None
        check(lib().bound_optimize_end(self.h, _ptr(lb), _ptr(ub), _ptr(bl, C.c_int32) if want_branch else None,
                                       _ptr(bn, C.c_int32) if want_branch else None))
        self.h = None
        return (lb, ub, bl, bn) if want_branch else (lb, ub)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().mnb_opt_session_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def relu_hull(lb, max_out=4096):
    """mnb_relu_hull: constraints (Phat [k,3], P [k,3], p [k]) of the 3-neuron ReLU hull over the
    polytope of the 26 octahedral bounds lb (host-only call of the library)."""
    lb = np.ascontiguousarray(lb, np.float64)
    if lb.shape != (26,):
        raise ValueError("lb needs the 26 octahedral bounds")
    out = np.zeros((max(max_out, 1), 7), np.float64)
    n = C.c_int()
    check(lib().mnb_relu_hull(lb.ctypes.data_as(C.POINTER(C.c_double)), int(max_out),
                              out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)))
    o = out[: n.value]
    return o[:, :3].copy(), o[:, 3:6].copy(), o[:, 6].copy()


# --------------------------------------------------------------------------- kernel timer
class KernelTimer:
    """HIP-event timing of one kernel class inside the library (see mnb_timer_begin)."""

    KINDS = {"fc_backsub": 1, "conv_backsub": 2, "fc_forward": 3, "conv_forward": 4, "fold": 5, "relax": 6,
             "concretize": 7, "bottom": 8, "bottom_win": 9}

    def __init__(self, net=None, kind="conv_backsub", node=-1):
        self.kind, self.node = kind, node

    def start(self):
        check(lib().mnb_timer_begin(self.KINDS[self.kind], int(self.node)))

    def stop(self):
        n, ms, fl, by = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
        check(lib().mnb_timer_end(C.byref(n), C.byref(ms), C.byref(fl), C.byref(by)))
        return {"name": f"{self.kind}@node{self.node}", "count": n.value, "ms": ms.value, "flops": fl.value,
                "bytes": by.value}


# --------------------------------------------------------------------------- serving
VERDICTS = {1: "verified", 2: "falsified", 3: "unknown", 4: "timeout"}
REASONS = {0: "none", 1: "no_split", 2: "queue_cap", 3: "memory", 4: "error", 5: "time"}


class Server:
    """Continuous-batching verification server (query_submit / query_poll)."""

    def __init__(self, nets, max_batch=256, queue_cap=4096, mem_budget=64 << 30, steps=20, lr=0.1, max_slots=0):
        self.nets = list(nets)
        cfg = _lib.ServerCfg()
        lib().mnb_server_cfg_default(C.byref(cfg))
        cfg.max_batch, cfg.queue_cap, cfg.mem_budget = int(max_batch), int(queue_cap), int(mem_budget)
        cfg.max_slots = int(max_slots)
        cfg.opt.steps, cfg.opt.lr = int(steps), float(lr)
        arr = (C.c_void_p * len(self.nets))(*[n.h.value for n in self.nets])
        h = C.c_void_p()
        check(lib().mnb_server_create(arr, len(self.nets), C.byref(cfg), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().mnb_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query_submit(self, net_index, lo, hi, Cm, c0, mncs=None, timeout_s=60.0, mnc_cap=0):
        lo, hi, Cm, c0 = _f32(lo), _f32(hi), _f32(Cm), _f32(c0)
        pack = _MncPack(mncs or {})
        q = _lib.Query()
        q.net_index = int(net_index)
        q.x_lo, q.x_hi, q.C, q.c0 = _ptr(lo), _ptr(hi), _ptr(Cm), _ptr(c0)
        q.n_spec = int(Cm.shape[0])
        q.mnc = pack.arr if pack.n else None
        q.n_mnc = pack.n
        q.timeout_s = float(timeout_s)
        q.mnc_cap = int(mnc_cap)
        t = C.c_uint64()
        check(lib().query_submit(self.h, C.byref(q), C.byref(t)))
        return t.value

    def query_poll(self, ticket):
        r = _lib.Result()
        rc = check(lib().query_poll(self.h, C.c_uint64(ticket), C.byref(r)))
        if rc == _lib.MNB_PENDING:
            return None
        return {"verdict": VERDICTS.get(r.verdict, str(r.verdict)), "lb": r.lb, "subproblems": r.subproblems,
                "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done,
                "latency": r.t_done - r.t_submit, "reason": REASONS.get(r.reason, str(r.reason)),
                "restarts": r.restarts}

    def wait(self, ticket, timeout=600.0, poll_s=0.002):
        import time
        t0 = time.time()
        while True:
            r = self.query_poll(ticket)
            if r is not None:
                return r
            if time.time() - t0 > timeout:
                raise TimeoutError(f"query {ticket} not done after {timeout} s")
            time.sleep(poll_s)
