"""Python front end: code and decoder handles over the C ABI, torch for memory and streams."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import check, load


@dataclass
class DecoderParams:
    """Mirror of ``lbp_params`` (include/lbp.h)."""
    max_iter: int = 100
    scale_mode: int = _lib.SCALE_PAPER
    scale: float = 0.625
    msg: int = _lib.MSG_INT8
    lottery: bool = True
    lottery_skip: int = 6
    flip: int = _lib.FLIP_MSG
    osd: int = _lib.OSD_0
    osd_order: int = 10
    lottery_rule: int = 0        # lottery_rule(cn, vn); 0 = Algorithm 3
    seed: int = 0

    def c(self) -> _lib.Params:
        return _lib.Params(self.max_iter, self.scale_mode, self.scale, self.msg, int(self.lottery),
                           self.lottery_skip, self.flip, self.osd, self.osd_order, self.lottery_rule,
                           self.seed & 0xFFFFFFFFFFFFFFFF)


class Code:
    """A parity-check matrix and per-column priors loaded onto the current device."""

    def __init__(self, row_ptr, col_idx, m: int, n: int, prior):
        lib = load()
        self.m, self.n = int(m), int(n)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        p = np.ascontiguousarray(np.broadcast_to(np.asarray(prior, dtype=np.float64), (self.n,)))
        h = ctypes.c_void_p()
        check(lib.lbp_code_create(self.m, self.n, rp.ctypes.data, ci.ctypes.data, p.ctypes.data, ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_scipy(cls, h, prior):
        import scipy.sparse as sp
        h = sp.csr_matrix(h)
        h.sort_indices()
        return cls(h.indptr, h.indices, h.shape[0], h.shape[1], prior)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib._lib is not None:
            _lib._lib.lbp_code_destroy(self._h)
            self._h = None


class Decoder:
    """Decoder for one code with fixed parameters and a workspace for max_batch shots."""

    def __init__(self, code: Code, params: DecoderParams, max_batch: int):
        lib = load()
        self.code = code
        self.params = params
        self.max_batch = int(max_batch)
        prm = params.c()
        h = ctypes.c_void_p()
        check(lib.lbp_decoder_create(code.handle, ctypes.byref(prm), self.max_batch, ctypes.byref(h)))
        self._h = h
        self.mw = (code.m + 31) // 32
        self.nw = (code.n + 31) // 32

    @property
    def osd_capacity(self) -> int:
        return int(load().lbp_decoder_osd_capacity(self._h))

    def set_osd_capacity(self, cap: int) -> None:
        check(load().lbp_decoder_set_osd_capacity(self._h, int(cap)))

    def set_timing(self, enable: bool) -> None:
        check(load().lbp_decoder_set_timing(self._h, int(enable)))

    def kernel_times(self):
        """(bp_ms, bp_launches, osd_ms, osd_launches) accumulated since the last call."""
        a, c = ctypes.c_double(), ctypes.c_double()
        b, d = ctypes.c_int64(), ctypes.c_int64()
        check(load().lbp_decoder_kernel_times(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                              ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def decode(self, syndromes, first_shot_id: int = 0, out=None, want_iters: bool = True,
               want_llr: bool = False, stream=None):
        """Decode a [shots, ceil(m/32)] int32/uint32 CUDA tensor of packed syndromes.

        Returns (corrections int32 [shots, ceil(n/32)], flags uint8 [shots],
        iters int32 [shots] or None, llr float32 [shots, n] or None), all on the
        syndromes' device; work is queued on ``stream`` (default: torch's current stream).
        """
        import torch
        assert syndromes.is_cuda and syndromes.dim() == 2 and syndromes.shape[1] == self.mw
        assert syndromes.dtype in (torch.int32, torch.uint32) and syndromes.is_contiguous()
        shots = syndromes.shape[0]
        dev = syndromes.device
        if out is None:
            corr = torch.empty((shots, self.nw), dtype=torch.int32, device=dev)
            flags = torch.empty(shots, dtype=torch.uint8, device=dev)
            iters = torch.empty(shots, dtype=torch.int32, device=dev) if want_iters else None
            llr = torch.empty((shots, self.code.n), dtype=torch.float32, device=dev) if want_llr else None
        else:
            corr, flags, iters, llr = out
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        check(load().lbp_decode(self._h, shots, first_shot_id & 0xFFFFFFFFFFFFFFFF, syndromes.data_ptr(),
                                corr.data_ptr(), flags.data_ptr(), iters.data_ptr() if iters is not None else None,
                                llr.data_ptr() if llr is not None else None, s.cuda_stream))
        return corr, flags, iters, llr

    def decode_noalloc(self, syndromes, out, first_shot_id: int = 0, stream=None):
        """lbp_decode_noalloc: lbp_decode on the library's static scratch (no allocation).
        ``out`` = (corrections, flags, iters or None, llr or None), preallocated CUDA tensors."""
        import torch
        assert syndromes.is_cuda and syndromes.dim() == 2 and syndromes.shape[1] == self.mw
        assert syndromes.dtype in (torch.int32, torch.uint32) and syndromes.is_contiguous()
        corr, flags, iters, llr = out
        s = stream if stream is not None else torch.cuda.current_stream(syndromes.device)
        check(load().lbp_decode_noalloc(self._h, syndromes.shape[0], first_shot_id & 0xFFFFFFFFFFFFFFFF,
                                        syndromes.data_ptr(), corr.data_ptr(), flags.data_ptr(),
                                        iters.data_ptr() if iters is not None else None,
                                        llr.data_ptr() if llr is not None else None, s.cuda_stream))
        return corr, flags, iters, llr

    def decode_keyed(self, syndromes, shot_keys, out=None, stream=None):
        """lbp_decode_keyed: shot_keys is a CUDA int64/uint64 tensor [shots, 2] of (seed, shot_id)."""
        import torch
        assert syndromes.is_cuda and syndromes.dim() == 2 and syndromes.shape[1] == self.mw
        assert syndromes.is_contiguous() and shot_keys.is_contiguous() and shot_keys.is_cuda
        assert shot_keys.shape == (syndromes.shape[0], 2) and shot_keys.element_size() == 8
        shots = syndromes.shape[0]
        dev = syndromes.device
        if out is None:
            corr = torch.empty((shots, self.nw), dtype=torch.int32, device=dev)
            flags = torch.empty(shots, dtype=torch.uint8, device=dev)
            iters = torch.empty(shots, dtype=torch.int32, device=dev)
        else:
            corr, flags, iters = out
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        check(load().lbp_decode_keyed(self._h, shots, shot_keys.data_ptr(), syndromes.data_ptr(), corr.data_ptr(),
                                      flags.data_ptr(), iters.data_ptr() if iters is not None else None, None,
                                      s.cuda_stream))
        return corr, flags, iters

    def decode_baseline(self, syndromes, first_shot_id: int = 0, stream=None):
        """lbp_decode_baseline (global-memory comparison path); returns (corr, flags, iters)."""
        import torch
        assert syndromes.is_cuda and syndromes.dim() == 2 and syndromes.shape[1] == self.mw
        assert syndromes.is_contiguous()
        shots = syndromes.shape[0]
        dev = syndromes.device
        corr = torch.empty((shots, self.nw), dtype=torch.int32, device=dev)
        flags = torch.empty(shots, dtype=torch.uint8, device=dev)
        iters = torch.empty(shots, dtype=torch.int32, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        check(load().lbp_decode_baseline(self._h, shots, first_shot_id & 0xFFFFFFFFFFFFFFFF, syndromes.data_ptr(),
                                         corr.data_ptr(), flags.data_ptr(), iters.data_ptr(), s.cuda_stream))
        return corr, flags, iters

    def shape(self) -> dict:
        """lbp_decoder_shape: the BP and OSD launch shapes chosen at creation."""
        v = [ctypes.c_int32() for _ in range(6)]
        check(load().lbp_decoder_shape(self._h, *[ctypes.byref(x) for x in v]))
        keys = ("bp_waves_per_block", "bp_blocks", "bp_group", "osd_variant", "osd_threads", "osd_blocks")
        return {k: x.value for k, x in zip(keys, v)}

    @property
    def device_bytes(self) -> int:
        return int(load().lbp_decoder_device_bytes(self._h))

    def decode_host(self, syndromes: np.ndarray, first_shot_id: int = 0, want_llr: bool = False):
        """Synchronous decode of host arrays (numpy uint32 [shots, ceil(m/32)])."""
        syn = np.ascontiguousarray(syndromes, dtype=np.uint32)
        shots = syn.shape[0]
        corr = np.zeros((shots, self.nw), dtype=np.uint32)
        flags = np.zeros(shots, dtype=np.uint8)
        iters = np.zeros(shots, dtype=np.int32)
        llr = np.zeros((shots, self.code.n), dtype=np.float32) if want_llr else None
        check(load().lbp_decode_host(self._h, shots, first_shot_id & 0xFFFFFFFFFFFFFFFF, syn.ctypes.data,
                                     corr.ctypes.data, flags.ctypes.data, iters.ctypes.data,
                                     llr.ctypes.data if llr is not None else None))
        return corr, flags, iters, llr

    def __del__(self):
        if getattr(self, "_h", None) and _lib._lib is not None:
            _lib._lib.lbp_decoder_destroy(self._h)
            self._h = None


class Plan:
    """lbp_plan: groups of shots of several decoders in one persistent launch,
    replayed from a captured HIP graph.

    ``groups`` is a list of (decoder, syndromes CUDA tensor [shots, ceil(m/32)],
    first_shot_id).  Outputs are allocated here (``outputs[g]`` = (corrections,
    flags, iters)) and bound to the plan, as are the syndrome tensors: write new
    syndromes into them in place and call ``launch``."""

    def __init__(self, groups, autotune: bool = True):
        import torch
        lib = load()
        self._keep = []
        self.outputs = []
        arr = (_lib.Group * len(groups))()
        for g, (dec, syn, first) in enumerate(groups):
            assert syn.is_cuda and syn.is_contiguous() and syn.dim() == 2 and syn.shape[1] == dec.mw
            shots = syn.shape[0]
            corr = torch.zeros((shots, dec.nw), dtype=torch.int32, device=syn.device)
            flags = torch.zeros(shots, dtype=torch.uint8, device=syn.device)
            iters = torch.zeros(shots, dtype=torch.int32, device=syn.device)
            self._keep += [dec, syn, corr, flags, iters]
            self.outputs.append((corr, flags, iters))
            arr[g] = _lib.Group(dec._h, shots, first & 0xFFFFFFFFFFFFFFFF, syn.data_ptr(), corr.data_ptr(),
                                flags.data_ptr(), iters.data_ptr())
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        check(lib.lbp_plan_create(len(groups), ctypes.cast(arr, ctypes.c_void_p),
                                  _lib.PLAN_AUTOTUNE if autotune else 0, ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        check(load().lbp_plan_launch(self._h, s.cuda_stream))

    def info(self):
        """(waves per block, blocks, measured ms of each autotuning candidate)."""
        w, b, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ms = (ctypes.c_double * 8)()
        check(load().lbp_plan_info(self._h, ctypes.byref(w), ctypes.byref(b), ctypes.byref(k), ms))
        return w.value, b.value, [ms[i] for i in range(k.value)]

    def __del__(self):
        if getattr(self, "_h", None) and _lib._lib is not None:
            _lib._lib.lbp_plan_destroy(self._h)
            self._h = None
