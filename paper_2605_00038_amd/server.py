"""Python handle of the serving loop (lbp_server_* in include/lbp.h): argument marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import LBP_ENOTREADY, LBP_OK, check, load
from .decoder import Code, DecoderParams


class Server:
    """Streaming decode server (lbp_server_*) on the current HIP device."""

    def __init__(self, device_mem_budget: int = 0, max_slots: int = 8):
        h = ctypes.c_void_p()
        check(load().lbp_server_create(int(device_mem_budget), int(max_slots), ctypes.byref(h)))
        self._h = h
        self._codes = []  # keep Code objects alive as long as the server

    def add_code(self, code: Code, params: DecoderParams) -> int:
        slot = ctypes.c_int32()
        prm = params.c()
        check(load().lbp_server_add_code(self._h, code.handle, ctypes.byref(prm), ctypes.byref(slot)))
        self._codes.append(code)
        return slot.value

    def _shape(self, slot: int):
        code = self._codes[slot]
        return (code.m + 31) // 32, (code.n + 31) // 32

    def submit(self, slot: int, syndromes: np.ndarray, seed: int, first_shot_id: int = 0) -> int:
        syn = np.ascontiguousarray(syndromes, dtype=np.uint32)
        mw, _ = self._shape(slot)
        assert syn.ndim == 2 and syn.shape[1] == mw
        t = ctypes.c_uint64()
        check(load().lbp_server_submit(self._h, int(slot), syn.shape[0], seed & 0xFFFFFFFFFFFFFFFF,
                                       first_shot_id & 0xFFFFFFFFFFFFFFFF, syn.ctypes.data, ctypes.byref(t)))
        return t.value

    def _outputs(self, slot: int, shots: int):
        _, nw = self._shape(slot)
        return (np.zeros((shots, nw), np.uint32), np.zeros(shots, np.uint8), np.zeros(shots, np.int32))

    def poll(self, ticket: int, slot: int, shots: int):
        """Results (corrections, flags, iters), or None while the request is pending."""
        corr, flags, iters = self._outputs(slot, shots)
        st = load().lbp_server_poll(self._h, ticket, corr.ctypes.data, flags.ctypes.data, iters.ctypes.data)
        if st == LBP_ENOTREADY:
            return None
        check(st)
        return corr, flags, iters

    def wait(self, ticket: int, slot: int, shots: int, timeout_us: int = -1):
        corr, flags, iters = self._outputs(slot, shots)
        st = load().lbp_server_wait(self._h, ticket, int(timeout_us), corr.ctypes.data, flags.ctypes.data,
                                    iters.ctypes.data)
        if st == LBP_ENOTREADY:
            return None
        check(st)
        return corr, flags, iters

    def cancel(self, ticket: int) -> None:
        check(load().lbp_server_cancel(self._h, ticket))

    def slot_info(self, slot: int) -> dict:
        v = [ctypes.c_int64() for _ in range(5)]
        check(load().lbp_server_slot_info(self._h, int(slot), *[ctypes.byref(x) for x in v]))
        return dict(zip(("ring_items", "bp_launches", "shots", "max_inflight", "queued_shots"), (x.value for x in v)))

    def run_load(self, slots, pools, n_requests: int, shots_per_request: int, rate: float, seed: int):
        """Open-loop Poisson load (rate requests/s; 0 = saturation) over the given slots.

        pools[k]: uint32 [pool_k, ceil(m_k/32)] host syndromes for slots[k].
        Returns (latency_us [n_requests], request_code [n_requests], elapsed_s)."""
        k = len(slots)
        arrs = [np.ascontiguousarray(p, dtype=np.uint32) for p in pools]
        slot_arr = (ctypes.c_int32 * k)(*slots)
        ptrs = (ctypes.c_void_p * k)(*[a.ctypes.data for a in arrs])
        sizes = (ctypes.c_int64 * k)(*[a.shape[0] for a in arrs])
        lat = np.zeros(n_requests, np.float64)
        code = np.zeros(n_requests, np.int32)
        el = ctypes.c_double()
        check(load().lbp_server_run_load(self._h, k, slot_arr, ptrs, sizes, int(n_requests), int(shots_per_request),
                                         float(rate), seed & 0xFFFFFFFFFFFFFFFF, code.ctypes.data, lat.ctypes.data,
                                         ctypes.byref(el)))
        return lat, code, el.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().lbp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Server", "LBP_OK"]
