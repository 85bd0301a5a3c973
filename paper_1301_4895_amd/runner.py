"""Device buffers (PyTorch) around the library's two device calls."""
from __future__ import annotations

import torch

from . import binding as B


class Runner:
    """Blocks + contraction for one batch of lanes with fixed shapes.

    props_u / props_d: complex64 or complex128 device tensors
    [batch][V][n_src][12][12]; sink_w: complex128 [n_src][V] or None;
    scale_exp: int32 [batch] or None; props_s: the strange propagator of a
    system with a Lambda.  Buffers are allocated once here; ``run`` only
    launches."""

    def __init__(self, tl: B.TermList, props_u, props_d, precision, sink_w=None, scale_exp=None,
                 err_estimate=False, props_s=None):
        self.tl = tl
        if tl._dev is None:
            tl.upload(props_u.device)
        self.batch, self.V = props_u.shape[0], props_u.shape[1]
        self.keep = (props_u, props_d, sink_w, scale_exp, props_s)
        self.p = B.problem(self.batch, self.V, props_u, props_d, precision,
                           None if sink_w is None else torch.view_as_real(sink_w), scale_exp, props_s)
        self.err_estimate = err_estimate
        nb, nbw, ncw = self._sizes()
        dev = props_u.device
        self.blocks = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.bws = torch.empty(max(nbw, 1), dtype=torch.uint8, device=dev)
        self.cws = torch.empty(max(ncw, 1), dtype=torch.uint8, device=dev)
        c = tl.counts()
        # main output, then the side nuclei's outputs, each [batch][rows][columns]
        self.out = torch.empty(self.batch * c["n_out"], dtype=torch.complex128, device=dev)
        shape = (1, 1) if c["projected"] else (c["n_delta"], c["n_alpha"])
        self.corr = self.out[:self.batch * shape[0] * shape[1]].view(self.batch, *shape)
        self.side_corr = []
        off = self.batch * shape[0] * shape[1]
        for i in range(c["n_side"]):
            stage, alphas, *_ = tl.side(i)
            n = self.batch * c["n_spin"][stage] * len(alphas)
            self.side_corr.append(self.out[off:off + n].view(self.batch, c["n_spin"][stage], len(alphas)))
            off += n
        self.exp = torch.empty(self.batch, dtype=torch.int32, device=dev)
        # error estimates (sigma, bound) of every output, as corr and side_corr
        self.err_all = (torch.empty((self.batch * c["n_out"], 2), dtype=torch.float64, device=dev)
                        if err_estimate else None)
        self.err = None if self.err_all is None else self.err_all[:self.batch * shape[0] * shape[1]].view(
            self.batch, *shape, 2)

    def _sizes(self):
        nb, nbw, ncw = B.workspace_query(self.tl, self.p)
        if self.err_estimate:
            ncw += B.workspace_query_err(self.tl, self.p)
        return nb, nbw, ncw

    def ensure_workspace(self):
        """Grows the contraction workspace when the term list's launch tuning
        needs more (two-phase steps keep their partials there)."""
        ncw = self._sizes()[2]
        if ncw > self.cws.numel():
            self.cws = None
            torch.cuda.empty_cache()
            self.cws = torch.empty(ncw, dtype=torch.uint8, device=self.blocks.device)

    def set_props(self, props_u, props_d, scale_exp=None, props_s=None):
        """Points the problem at other propagators of the same shape."""
        sink_w = self.keep[2]
        self.keep = (props_u, props_d, sink_w, scale_exp if scale_exp is not None else self.keep[3],
                     props_s if props_s is not None else self.keep[4])
        self.p.prop_u = props_u.data_ptr()
        self.p.prop_d = props_d.data_ptr()
        if scale_exp is not None:
            self.p.scale_exp = scale_exp.data_ptr()
        if props_s is not None:
            self.p.prop_s = props_s.data_ptr()

    def run_blocks(self, stream=None):
        B.make_blocks(self.tl, self.p, self.blocks, self.bws, stream)

    def run_contract(self, stream=None):
        self.ensure_workspace()
        B.contract_correlator(self.tl, self.p, self.blocks, self.out, self.exp, self.cws, stream, self.err_all)

    def run(self, stream=None):
        self.run_blocks(stream)
        self.run_contract(stream)
        return self.corr, self.exp
