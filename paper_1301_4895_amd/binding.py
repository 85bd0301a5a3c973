"""ctypes binding of libmbcontract (include/mbcontract.h).

Argument marshalling only: every step of the method runs in the library (host
term-list builder, HIP kernels).  PyTorch tensors provide device memory and
streams.  There is no fallback: a missing library raises at import of the
first call.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbcontract.so")

MB_OK, MB_EINVAL, MB_EPAULI, MB_EUNSUPPORTED, MB_ENOWORKSPACE, MB_EHIP, MB_ENOMEM = 0, -1, -2, -3, -4, -5, -6
MB_PATH_AUTO, MB_PATH_PROTONS_FIRST, MB_PATH_NEUTRONS_FIRST, MB_PATH_EXPLICIT, MB_PATH_BEST = 0, 1, 2, 3, 4
MB_C64, MB_C128 = 0, 1
MB_FP64, MB_MIXED, MB_MIXED_F32B = 0, 1, 2
MB_MAX_STAGES = 16
MB_TUNE_PASS_GROUP, MB_TUNE_LDS_BYTES, MB_TUNE_LANE_TILE, MB_TUNE_KERNEL, MB_TUNE_UNROLL, MB_TUNE_GROUP = \
    1, 2, 3, 4, 5, 6
MB_TUNE_PAIRED = 7
MB_TUNE_TWO_PHASE = 8
MB_TUNE_BLOCKS = 9
(MB_EXPORT_QUARK, MB_EXPORT_SPIN, MB_EXPORT_QSPLIT, MB_EXPORT_SSPLIT, MB_EXPORT_COEF,
 MB_EXPORT_DELTA, MB_EXPORT_ALPHA, MB_EXPORT_PROJ, MB_EXPORT_SIDE, MB_EXPORT_QUARK_S, MB_EXPORT_SPIN_L,
 MB_EXPORT_DELTA_L, MB_EXPORT_ALPHA_L) = range(1, 14)
MB_PROTON, MB_NEUTRON, MB_LAMBDA = 0, 1, 2

EXPORTED_SYMBOLS = [
    "mb_build_term_list", "mb_build_term_list_counts_only", "mb_build_term_list_path", "mb_term_list_free",
    "mb_term_list_save", "mb_term_list_load",
    "mb_term_list_counts", "mb_term_list_export", "mb_term_list_upload", "mb_workspace_query",
    "mb_make_blocks", "mb_make_blocks_noalloc", "mb_contract_correlator", "mb_contract_step", "mb_term_list_tune", "mb_workspace_query_err",
    "mb_batch_plan", "mb_batch_create", "mb_batch_launch", "mb_batch_kernel_count", "mb_batch_free",
    "mb_last_error",
]


class MBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmbcontract error {code}: {msg}")
        self.code = code


class mb_nucleus(C.Structure):
    _fields_ = [("n_P", C.c_int), ("n_N", C.c_int), ("rel", C.c_int), ("n_src", C.c_int),
                ("path", C.c_int), ("order", C.c_uint32), ("n_Lambda", C.c_int)]


class mb_spin_request(C.Structure):
    _fields_ = [("all_components", C.c_int), ("sink_P", C.c_uint32), ("sink_N", C.c_uint32),
                ("n_alpha", C.c_int), ("alpha", C.POINTER(C.c_uint32)), ("proj", C.POINTER(C.c_double)),
                ("sink_L", C.c_uint32), ("alpha_L", C.POINTER(C.c_uint32))]


class mb_side_request(C.Structure):
    _fields_ = [("stage", C.c_int), ("all_components", C.c_int), ("n_alpha", C.c_int),
                ("alpha", C.POINTER(C.c_uint32))]


class mb_counts(C.Structure):
    _fields_ = [("n_stages", C.c_int), ("path", C.c_int * MB_MAX_STAGES), ("n_lambda", C.c_int64),
                ("n_lambda_step", C.c_int64 * MB_MAX_STAGES), ("n_req", C.c_int64 * MB_MAX_STAGES),
                ("n_quark", C.c_int64 * MB_MAX_STAGES), ("n_spin", C.c_int32 * MB_MAX_STAGES),
                ("n_L", C.c_int64), ("n_U", C.c_int64), ("n_delta", C.c_int32),
                ("n_alpha", C.c_int32), ("n_psi", C.c_int32), ("n_xi", C.c_int32),
                ("device_bytes", C.c_int64), ("projected", C.c_int32), ("n_LM", C.c_int64),
                ("n_side", C.c_int32), ("n_out", C.c_int64), ("rel", C.c_int32), ("n_src", C.c_int32),
                ("n_Lambda", C.c_int32)]


class mb_problem(C.Structure):
    _fields_ = [("batch", C.c_int64), ("V", C.c_int64), ("in_dtype", C.c_int),
                ("precision", C.c_int), ("prop_u", C.c_void_p), ("prop_d", C.c_void_p),
                ("sink_w", C.c_void_p), ("scale_exp", C.c_void_p), ("prop_s", C.c_void_p)]


class mb_batch_item(C.Structure):
    _fields_ = [("tl", C.c_void_p), ("prob", mb_problem), ("blocks", C.c_void_p),
                ("blocks_bytes", C.c_size_t), ("blocks_ws", C.c_void_p), ("blocks_ws_bytes", C.c_size_t),
                ("contract_ws", C.c_void_p), ("contract_ws_bytes", C.c_size_t), ("corr_out", C.c_void_p),
                ("exp_out", C.c_void_p), ("branch", C.c_int)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.mb_build_term_list.argtypes = [C.POINTER(mb_nucleus), C.POINTER(mb_spin_request), C.POINTER(P)]
        L.mb_build_term_list_counts_only.argtypes = L.mb_build_term_list.argtypes
        L.mb_build_term_list_path.argtypes = [C.POINTER(mb_nucleus), C.POINTER(mb_spin_request), C.c_int,
                                              C.POINTER(mb_side_request), C.POINTER(P)]
        L.mb_term_list_free.argtypes = [P]
        L.mb_term_list_save.argtypes = [P, C.c_char_p]
        L.mb_term_list_load.argtypes = [C.c_char_p, C.POINTER(P)]
        L.mb_term_list_free.restype = None
        L.mb_term_list_counts.argtypes = [P, C.POINTER(mb_counts)]
        L.mb_term_list_export.argtypes = [P, C.c_int, C.c_int, P, C.POINTER(C.c_size_t)]
        L.mb_term_list_upload.argtypes = [P, P, C.c_size_t, P]
        L.mb_workspace_query.argtypes = [P, C.POINTER(mb_problem), C.POINTER(C.c_size_t),
                                         C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.mb_make_blocks.argtypes = [P, C.POINTER(mb_problem), P, C.c_size_t, P, C.c_size_t, P]
        L.mb_make_blocks_noalloc.argtypes = [P, C.POINTER(mb_problem), P, C.c_size_t, P]
        L.mb_contract_correlator.argtypes = [P, C.POINTER(mb_problem), P, C.c_size_t, P, P, P, P,
                                             C.c_size_t, P]
        L.mb_workspace_query_err.argtypes = [P, C.POINTER(mb_problem), C.POINTER(C.c_size_t)]
        L.mb_contract_step.argtypes = [P, C.POINTER(mb_problem), P, C.c_size_t, C.c_int, P, P, P,
                                       C.c_size_t, P]
        L.mb_term_list_tune.argtypes = [P, C.c_int, C.c_int, C.c_int]
        L.mb_batch_plan.argtypes = [C.POINTER(P), C.POINTER(mb_problem), C.c_int, C.c_int,
                                    C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.mb_batch_create.argtypes = [C.POINTER(mb_batch_item), C.c_int, C.c_int, C.POINTER(P)]
        L.mb_batch_launch.argtypes = [P, P]
        L.mb_batch_kernel_count.argtypes = [P, C.POINTER(C.c_int64)]
        L.mb_batch_free.argtypes = [P]
        L.mb_batch_free.restype = None
        L.mb_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != MB_OK:
        raise MBError(rc, lib().mb_last_error().decode())


class TermList:
    """Owner of an mb_term_list handle.  ``proj``: optional real weights
    [n_delta][n_alpha] of the spin projection (Sec. 5), over the sink and
    source sets of the same request without it.  ``sides``: smaller nuclei
    on the path (Sec. 7), as (stage, source sets) with source sets None for
    all of them.  ``order``: with path MB_PATH_EXPLICIT, bit i set when the
    (i+1)-th baryon added is a proton.  ``n_Lambda`` = 1 adds one Lambda
    (after the nucleons); then ``alphas`` are (proton set, neutron set,
    Lambda set) triples and ``sink_L`` is the Lambda's sink base set."""

    def __init__(self, n_P, n_N, rel, n_src=1, *, all_components=False, sink_P=0, sink_N=0,
                 alphas=(), path=MB_PATH_AUTO, order=0, counts_only=False, proj=None, sides=(),
                 n_Lambda=0, sink_L=0):
        nuc = mb_nucleus(n_P, n_N, int(rel), n_src, path, order, n_Lambda)
        width = 3 if n_Lambda else 2
        al = np.asarray(alphas, np.uint32).reshape(-1, width)
        arr = np.ascontiguousarray(al[:, :2].reshape(-1))
        arrL = np.ascontiguousarray(al[:, 2]) if n_Lambda else np.zeros(0, np.uint32)
        self._alpha_keep = (arr, arrL)
        w = None if proj is None else np.ascontiguousarray(np.asarray(proj, np.float64).reshape(-1))
        req = mb_spin_request(int(all_components), sink_P, sink_N, len(arr) // 2,
                              arr.ctypes.data_as(C.POINTER(C.c_uint32)) if len(arr) else None,
                              w.ctypes.data_as(C.POINTER(C.c_double)) if w is not None else None,
                              sink_L, arrL.ctypes.data_as(C.POINTER(C.c_uint32)) if len(arrL) else None)
        h = C.c_void_p()
        if sides:
            if counts_only:
                raise ValueError("side nuclei need a full term list")
            self._side_keep = [np.ascontiguousarray(np.asarray(a if a is not None else (), np.uint32).reshape(-1))
                               for _, a in sides]
            sr = (mb_side_request * len(sides))(*[
                mb_side_request(st, int(a is None), len(k) // 2,
                                k.ctypes.data_as(C.POINTER(C.c_uint32)) if len(k) else None)
                for (st, a), k in zip(sides, self._side_keep)])
            _check(lib().mb_build_term_list_path(C.byref(nuc), C.byref(req), len(sides), sr, C.byref(h)))
        else:
            fn = lib().mb_build_term_list_counts_only if counts_only else lib().mb_build_term_list
            _check(fn(C.byref(nuc), C.byref(req), C.byref(h)))
        self.h = h
        self.nucleus = dict(n_P=n_P, n_N=n_N, rel=bool(rel), n_src=n_src, n_Lambda=n_Lambda)
        self._dev = None

    def save(self, path):
        """Writes the host term list to a file (mb_term_list_save)."""
        _check(lib().mb_term_list_save(self.h, os.fsencode(path)))

    @classmethod
    def load(cls, path):
        """A term list read back from a file written by ``save``."""
        h = C.c_void_p()
        _check(lib().mb_term_list_load(os.fsencode(path), C.byref(h)))
        self = cls.__new__(cls)
        self.h = h
        self._dev = None
        c = self.counts()
        nP = sum(1 for t in c["path"] if t == 0)
        self.nucleus = dict(n_P=nP, n_N=c["n_stages"] - nP, rel=bool(c["rel"]), n_src=c["n_src"], n_Lambda=0)
        return self

    @classmethod
    def spin_state(cls, n_P, n_N, rel, n_src, spins, n_Lambda=0, **kw):
        """Single spin component (Sec. 8): indices listed protons first,
        then neutrons, then the Lambda's."""
        pm = sum(1 << s for s in spins[:n_P])
        nm = sum(1 << s for s in spins[n_P:n_P + n_N])
        if n_Lambda:
            lm = 1 << spins[n_P + n_N]
            return cls(n_P, n_N, rel, n_src, sink_P=pm, sink_N=nm, sink_L=lm, alphas=[(pm, nm, lm)],
                       n_Lambda=1, **kw)
        return cls(n_P, n_N, rel, n_src, sink_P=pm, sink_N=nm, alphas=[(pm, nm)], **kw)

    def close(self):
        if getattr(self, "h", None):
            lib().mb_term_list_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: module globals may be gone
            pass

    def counts(self):
        c = mb_counts()
        _check(lib().mb_term_list_counts(self.h, C.byref(c)))
        n = c.n_stages
        return dict(n_stages=n, path=list(c.path[:n]), n_lambda=c.n_lambda,
                    n_lambda_step=list(c.n_lambda_step[:n]), n_req=list(c.n_req[:n]),
                    n_quark=list(c.n_quark[:n]), n_spin=list(c.n_spin[:n]), n_L=c.n_L, n_U=c.n_U,
                    n_delta=c.n_delta, n_alpha=c.n_alpha, n_psi=c.n_psi, n_xi=c.n_xi,
                    device_bytes=c.device_bytes, projected=bool(c.projected), n_LM=c.n_LM,
                    n_side=c.n_side, n_out=c.n_out, rel=c.rel, n_src=c.n_src, n_Lambda=c.n_Lambda)

    def side(self, i):
        """Side request i: (stage, source sets [n][2], CSR row starts, quark
        part indices of its stage, integer coefficients)."""
        raw = self.export(MB_EXPORT_SIDE, i, np.uint8)
        stage, na = (int(v) for v in raw[:16].view(np.int64))
        o = 16 + 8 * na
        alphas = raw[16:o].view(np.uint32).reshape(-1, 2)
        row = raw[o:o + 8 * (na + 1)].view(np.int64)
        n = int(row[-1])
        o += 8 * (na + 1)
        col = raw[o:o + 8 * n].view(np.int64)
        val = raw[o + 8 * n:o + 16 * n].view(np.int64)
        return stage, alphas, row, col, val

    def export(self, what, stage=0, dtype=np.uint32):
        n = C.c_size_t(0)
        _check(lib().mb_term_list_export(self.h, what, stage, None, C.byref(n)))
        buf = np.zeros(max(n.value, 1), np.uint8)
        _check(lib().mb_term_list_export(self.h, what, stage, buf.ctypes.data_as(C.c_void_p), C.byref(n)))
        return buf[:n.value].view(dtype)

    def tune(self, step, what, value):
        """Launch tuning of a recursion step (results do not depend on it)."""
        _check(lib().mb_term_list_tune(self.h, step, what, value))

    def upload(self, torch_device="cuda"):
        """Allocates the device image (a torch tensor) and uploads the tables."""
        import torch
        nbytes = self.counts()["device_bytes"]
        dev = torch.empty(nbytes + 256, dtype=torch.uint8, device=torch_device)
        ptr = dev.data_ptr()
        off = (-ptr) % 256
        stream = torch.cuda.current_stream().cuda_stream
        _check(lib().mb_term_list_upload(self.h, C.c_void_p(ptr + off), nbytes, C.c_void_p(stream)))
        self._dev = dev
        return self


def problem(batch, V, props_u, props_d, precision, sink_w=None, scale_exp=None, props_s=None):
    """mb_problem for torch device tensors (props complex64 / complex128;
    props_s the strange propagator of a system with a Lambda)."""
    import torch
    in_dtype = MB_C128 if props_u.dtype == torch.complex128 else MB_C64
    return mb_problem(batch, V, in_dtype, precision, props_u.data_ptr(), props_d.data_ptr(),
                      sink_w.data_ptr() if sink_w is not None else None,
                      scale_exp.data_ptr() if scale_exp is not None else None,
                      props_s.data_ptr() if props_s is not None else None)


def workspace_query(tl: TermList, p: mb_problem):
    a, b, c = C.c_size_t(), C.c_size_t(), C.c_size_t()
    _check(lib().mb_workspace_query(tl.h, C.byref(p), C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def workspace_query_err(tl: TermList, p: mb_problem):
    """Extra contraction workspace bytes for error estimates."""
    a = C.c_size_t()
    _check(lib().mb_workspace_query_err(tl.h, C.byref(p), C.byref(a)))
    return a.value


def make_blocks(tl: TermList, p: mb_problem, blocks, ws, stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().mb_make_blocks(tl.h, C.byref(p), C.c_void_p(blocks.data_ptr()), blocks.numel() * blocks.element_size(),
                                C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), C.c_void_p(s)))


MB_NOALLOC_SCRATCH_BYTES = 64 << 20


def make_blocks_noalloc(tl: TermList, p: mb_problem, blocks, stream=None):
    """mb_make_blocks with the partial sums in the library's fixed scratch."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().mb_make_blocks_noalloc(tl.h, C.byref(p), C.c_void_p(blocks.data_ptr()),
                                        blocks.numel() * blocks.element_size(), C.c_void_p(s)))


def contract_correlator(tl: TermList, p: mb_problem, blocks, corr, exp_out, ws, stream=None, err=None):
    """err: optional float64 device tensor [batch][n_out][2] for the error
    estimates (then ws must hold workspace_query_err more bytes)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().mb_contract_correlator(
        tl.h, C.byref(p), C.c_void_p(blocks.data_ptr()), blocks.numel() * blocks.element_size(),
        C.c_void_p(corr.data_ptr()), C.c_void_p(exp_out.data_ptr()) if exp_out is not None else None,
        C.c_void_p(err.data_ptr()) if err is not None else None,
        C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), C.c_void_p(s)))


def contract_step(tl: TermList, p: mb_problem, blocks, step, corr, exp_out, ws, stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib().mb_contract_step(
        tl.h, C.byref(p), C.c_void_p(blocks.data_ptr()), blocks.numel() * blocks.element_size(), step,
        C.c_void_p(corr.data_ptr()) if corr is not None else None,
        C.c_void_p(exp_out.data_ptr()) if exp_out is not None else None,
        C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), C.c_void_p(s)))


def batch_plan(tls, probs, n_branches):
    """Branch of every item (longest first onto the least loaded branch) and
    the cost estimate of every item (algorithmic flops)."""
    n = len(tls)
    ta = (C.c_void_p * n)(*[t.h for t in tls])
    pa = (mb_problem * n)(*probs)
    br = (C.c_int * n)()
    cost = (C.c_double * n)()
    _check(lib().mb_batch_plan(ta, pa, n, n_branches, br, cost))
    return list(br), list(cost)


class Batch:
    """A recorded batch (mb_batch_create): items are dicts with keys tl,
    prob, blocks, blocks_ws, contract_ws, corr, exp (torch tensors or None)
    and branch."""

    def __init__(self, items, n_branches):
        n = len(items)
        arr = (mb_batch_item * n)()

        def nbytes(t):
            return t.numel() * t.element_size()
        for i, it in enumerate(items):
            arr[i] = mb_batch_item(it["tl"].h, it["prob"], it["blocks"].data_ptr(), nbytes(it["blocks"]),
                                   it["blocks_ws"].data_ptr(), nbytes(it["blocks_ws"]),
                                   it["contract_ws"].data_ptr(), nbytes(it["contract_ws"]),
                                   it["corr"].data_ptr(),
                                   it["exp"].data_ptr() if it.get("exp") is not None else None,
                                   it["branch"])
        h = C.c_void_p()
        _check(lib().mb_batch_create(arr, n, n_branches, C.byref(h)))
        self.h = h
        self._items = items   # keeps the buffers alive

    def launch(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        _check(lib().mb_batch_launch(self.h, C.c_void_p(s)))

    def kernel_count(self):
        n = C.c_int64()
        _check(lib().mb_batch_kernel_count(self.h, C.byref(n)))
        return n.value

    def close(self):
        if self.h:
            lib().mb_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
