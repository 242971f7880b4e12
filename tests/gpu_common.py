"""Shared helpers of the GPU parity tests: build the same input on both sides
(oracle on the CPU, library on the GPU) and compare."""
from __future__ import annotations

import numpy as np

import oracle as O
import workloads as W

LINF = 1e-9  # rank parity bar (FP64, tau = 1e-10)


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def dfpr():
    import paper_2401_15870_amd as m
    m.lib()  # fails loudly when the HIP library is missing
    return m


def assert_csr_equal(g, og):
    for in_csr, off, idx in ((False, og.out_off, og.out_idx), (True, og.in_off, og.in_idx)):
        goff, gidx = g.export(in_csr=in_csr)
        assert goff.shape == off.shape and np.array_equal(goff, off), f"offsets differ (in_csr={in_csr})"
        assert gidx.shape == idx.shape and np.array_equal(gidx, idx), f"indices differ (in_csr={in_csr})"


def assert_info_equal(info, ob):
    for k in ("ins_in", "ins_effective", "del_in", "del_effective", "self_loop_dels_ignored"):
        assert info[k] == ob.info[k], (k, info[k], ob.info[k])


class Pair:
    """One graph on both sides, updated in lock-step."""

    def __init__(self, n, src, dst, fused=False, **kw):
        """fused=False keeps the launch-per-iteration loop on small graphs too
        (the library default runs them in one launch; both give the same bits)."""
        self.dfpr = dfpr()
        self.og = O.graph(n, src, dst)
        self.g = self.dfpr.Graph.from_coo(n, src, dst, **kw)
        if not fused:
            self.g.set_fused_limit(0)
        self.kw = kw
        self.og_prev = None
        self.batch = None
        self.n = n

    def apply(self, ds, dd, is_, id_, device=False):
        torch = torch_cuda()
        if device:
            args = [torch.as_tensor(np.asarray(a, np.int32)).cuda() for a in (ds, dd, is_, id_)]
        else:
            args = (ds, dd, is_, id_)
        info = self.g.apply_batch(*args)
        og2, ob = O.apply(self.og, ds, dd, is_, id_)
        assert_info_equal(info, ob)
        assert info["m_after"] == og2.m
        self.og_prev, self.og, self.batch = self.og, og2, ob
        return info

    def rank(self, mode, r_prev, **kw):
        """(gpu ranks as numpy, gpu stats, oracle Result) from the same R_prev bits."""
        torch = torch_cuda()
        rp = None if r_prev is None else torch.from_numpy(np.ascontiguousarray(r_prev)).cuda()
        r, st = self.g.update_ranks(mode, rp, **kw)
        torch.cuda.synchronize()
        okw = {k: v for k, v in kw.items() if k in ("alpha", "tol", "max_iters", "criterion")}  # dense_switch: GPU only
        if "frontier_tol" in kw:
            okw["tol_f"] = kw["frontier_tol"]
        if "prune_tol" in kw:
            okw["tol_p"] = kw["prune_tol"]
        if mode in ("df", "dfp"):
            ref = O.rank(mode, self.og, r_prev, self.og_prev, self.batch, **okw)
        else:
            ref = O.rank(mode, self.og, r_prev, **okw)
        return r.cpu().numpy(), st, ref


def rmat(scale, ef=16, seed=1):
    return W.rmat_graph(scale, ef, seed=seed)


def hub_graph(n, hub_in, hub_out, extra, seed):
    """Random graph plus one vertex with many in- and out-neighbours."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, extra)
    d = rng.integers(0, n, extra)
    ins = rng.choice(np.arange(1, n), size=hub_in, replace=False)
    outs = rng.choice(np.arange(1, n), size=hub_out, replace=False)
    src = np.concatenate([s, ins, np.zeros(hub_out, np.int64)])
    dst = np.concatenate([d, np.zeros(hub_in, np.int64), outs])
    return n, src.astype(np.int32), dst.astype(np.int32)
