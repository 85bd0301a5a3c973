"""ctypes binding of synth/libsynth.so (device twin of synth.props)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_SO = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynth.so")
_lib = None


def _l():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise ImportError(f"{_SO} is missing: run __graft_entry__.build()")
        _lib = C.CDLL(_SO)
        _lib.mb_synth_props.argtypes = [C.c_void_p, C.c_int, C.c_uint64, C.c_uint32, C.c_int64, C.c_int,
                                        C.c_int, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]
    return _lib


def fill_props(out, seed: int, stream_id: int, V: int, nsrc: int, T: int, first_bt: int, m: float = 0.5):
    """Fills the torch tensor out[nbt][V][nsrc][12][12] (complex64/128) with
    units first_bt .. first_bt+nbt-1 (unit = problem*T + t) of the dataset."""
    import torch
    from .props import decay
    dec = torch.from_numpy(decay(T, m)).to(out.device)
    nbt = out.shape[0]
    c128 = 1 if out.dtype == torch.complex128 else 0
    s = torch.cuda.current_stream().cuda_stream
    rc = _l().mb_synth_props(C.c_void_p(out.data_ptr()), c128, seed, stream_id, V, nsrc, T, first_bt, nbt,
                             C.c_void_p(dec.data_ptr()), C.c_void_p(s))
    if rc != 0:
        raise RuntimeError(f"mb_synth_props failed: hip error {rc}")
    torch.cuda.current_stream().synchronize()
    del dec
    return out
