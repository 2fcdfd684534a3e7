"""Python binding of the request server in include/gbs_mps.h (gbs_server_*).

Argument marshalling only: queueing, admission, the worker threads and every
kernel live in libgbs_mps.so.  Device tensors passed to `submit` are kept
alive here until `wait` returns.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib
from ._lib import BuildOpts, Request, Result, ServerStats, check, lib


@dataclasses.dataclass
class Ticket:
    id: int
    out: torch.Tensor
    gamma: torch.Tensor | None


class Server:
    """gbs_server_create / submit / wait / stats / destroy."""

    def __init__(self, slots: int = 4, budget_bytes: int | None = None, max_queue: int = 4096):
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(free * 0.6)
        h = ctypes.c_void_p()
        check(lib().gbs_server_create(int(slots), int(budget_bytes), int(max_queue), ctypes.byref(h)))
        self._h = h
        self.slots = slots
        self.budget_bytes = budget_bytes

    def submit(self, gamma: torch.Tensor, d: int, chi: int, shots: int, seed: int, precision: str = "fp32",
               dstar: float = 1.0 + 1e-10, trunc_rel: float = 0.0, out: torch.Tensor | None = None,
               keep: bool = False) -> Ticket:
        """Build (and keep the MPS resident when `keep`), then draw `shots`
        samples.  A kept MPS is named by the ticket's id (sample(), release())."""
        if not isinstance(gamma, torch.Tensor) or not gamma.is_cuda or gamma.dtype != torch.float64:
            raise ValueError("gamma must be a CUDA float64 tensor")
        gamma = gamma.contiguous()
        M = gamma.shape[0] // 2
        if out is None:
            out = torch.empty((shots, M), dtype=torch.int32, device=gamma.device)
        # the workers read gamma on their own streams: make the producer's work visible first
        torch.cuda.current_stream(gamma.device).synchronize()
        req = Request(gamma=gamma.data_ptr(), M=M,
                      opt=BuildOpts(d=d, chi=chi, dstar=dstar, prec=_lib.PRECISIONS[precision], flags=0,
                                    trunc_rel=trunc_rel),
                      shots=shots, seed=seed & (2 ** 64 - 1), out=out.data_ptr() if shots > 0 else None,
                      kind=_lib.GBS_REQ_BUILD if keep else _lib.GBS_REQ_BUILD_SAMPLE, handle=0)
        rid = ctypes.c_int64()
        check(lib().gbs_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        return Ticket(rid.value, out, gamma)

    def sample(self, handle: int, M: int, shots: int, seed: int, out: torch.Tensor | None = None,
               device="cuda") -> Ticket:
        """Draw `shots` samples from the resident MPS named `handle` (the id
        of the keep=True submit that built it); M: its mode count."""
        if out is None:
            out = torch.empty((shots, M), dtype=torch.int32, device=device)
        req = Request(gamma=None, M=M, opt=BuildOpts(), shots=shots, seed=seed & (2 ** 64 - 1),
                      out=out.data_ptr(), kind=_lib.GBS_REQ_SAMPLE, handle=int(handle))
        rid = ctypes.c_int64()
        check(lib().gbs_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        return Ticket(rid.value, out, None)

    def release(self, handle: int) -> None:
        """Free a resident MPS once the samples admitted or queued on it are done."""
        check(lib().gbs_server_release(self._h, int(handle)))

    def poll(self, t: Ticket) -> bool:
        done = ctypes.c_int32()
        check(lib().gbs_server_poll(self._h, t.id, ctypes.byref(done)))
        return bool(done.value)

    def wait(self, t: Ticket, raise_on_error: bool = True) -> dict:
        """Block until the request is done; returns its timings (ms) and
        status.  The samples are in t.out.  A failed request raises GbsError
        unless raise_on_error is False (then status < 0 and "error" is set)."""
        r = Result()
        rc = lib().gbs_server_wait(self._h, t.id, ctypes.byref(r))
        if rc != 0 and raise_on_error:
            check(rc)
        out = {f: getattr(r, f) for f, _ in Result._fields_}
        if rc != 0:
            msg = lib().gbs_last_error()
            out["error"] = msg.decode() if msg else ""
        return out

    def stats(self) -> dict:
        s = ServerStats()
        check(lib().gbs_server_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def reset_stats(self) -> None:
        check(lib().gbs_server_reset_stats(self._h))

    def close(self) -> None:
        if self._h:
            lib().gbs_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(M: int, d: int, chi: int, shots: int, precision: str = "fp32") -> int:
    """gbs_mps_footprint: upper estimate of one request's device bytes."""
    opts = BuildOpts(d=d, chi=chi, dstar=1.0 + 1e-10, prec=_lib.PRECISIONS[precision], flags=0, trunc_rel=0.0)
    return int(lib().gbs_mps_footprint(int(M), ctypes.byref(opts), int(shots)))


def run_mix(server: Server, requests, gammas, precision: str = "fp32", time_scale: float = 1.0):
    """Submit `requests` (dicts with workload, arrival [s], shots, seed) at
    their arrival times, wait for all, return (per-request results, stats).
    gammas[i] is request i's covariance on the device."""
    import time
    server.reset_stats()
    t0 = time.perf_counter()
    tickets = []
    for r, g in zip(requests, gammas):
        delay = r["arrival"] * time_scale - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        w = r["workload"]
        tickets.append(server.submit(g, w.d, w.chi, r["shots"], r["seed"], precision=precision))
    results = [server.wait(t, raise_on_error=False) for t in tickets]
    return tickets, results, server.stats()
