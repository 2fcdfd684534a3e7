"""Python-facing API: build an MPS from a covariance matrix on the GPU and
query amplitudes and samples.  Thin wrapper over the C ABI (see _lib)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import BuildOpts, GbsError, InfoT, check, lib


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class GaussianMPS:
    """Handle to a device-resident MPS built by gbs_mps_build."""

    def __init__(self, handle: ctypes.c_void_p, M: int, d: int):
        self._h = handle
        self.M = M
        self.d = d
        self.site = None  # set for a single-site build (build_site)

    # -- lifetime
    def free(self) -> None:
        if self._h:
            lib().gbs_mps_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # -- consumers
    def amplitude(self, patterns: torch.Tensor, stream=None) -> torch.Tensor:
        """Complex128 amplitudes <n|psi> for a (B, M) int32 CUDA tensor."""
        if patterns.dtype != torch.int32 or not patterns.is_cuda or patterns.dim() != 2 or patterns.shape[1] != self.M:
            raise ValueError("patterns must be a CUDA int32 tensor of shape (B, M)")
        patterns = patterns.contiguous()
        out = torch.empty((patterns.shape[0], 2), dtype=torch.float64, device=patterns.device)
        check(lib().gbs_mps_amplitude(self._h, ctypes.c_void_p(patterns.data_ptr()), patterns.shape[0],
                                      ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return torch.view_as_complex(out)

    def sample(self, shots: int, seed: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """(shots, M) int32 photon-number samples on the GPU."""
        if out is None:
            out = torch.empty((shots, self.M), dtype=torch.int32, device="cuda")
        check(lib().gbs_mps_sample(self._h, int(shots), ctypes.c_uint64(seed & (2 ** 64 - 1)),
                                   ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def sample_noalloc(self, shots: int, seed: int, out: torch.Tensor, stream=None) -> torch.Tensor:
        """sample() through gbs_mps_sample_noalloc: the same samples, drawn on
        the library's static device scratch array (no device allocation in
        the call; `out` must be given)."""
        if out.dtype != torch.int32 or not out.is_cuda or tuple(out.shape) != (shots, self.M):
            raise ValueError("out must be a CUDA int32 tensor of shape (shots, M)")
        check(lib().gbs_mps_sample_noalloc(self._h, int(shots), ctypes.c_uint64(seed & (2 ** 64 - 1)),
                                           ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def sample_timed(self, shots: int, seed: int, out: torch.Tensor | None = None, stream=None):
        """sample() with HIP events around each sampling launch; returns
        (samples, dict of launch counts and GPU milliseconds).  Synchronises
        the stream."""
        if out is None:
            out = torch.empty((shots, self.M), dtype=torch.int32, device="cuda")
        t = _lib.SampleTimingT()
        check(lib().gbs_mps_sample_timed(self._h, int(shots), ctypes.c_uint64(seed & (2 ** 64 - 1)),
                                         ctypes.c_void_p(out.data_ptr()), _stream_handle(stream), ctypes.byref(t)))
        return out, {k: getattr(t, k) for k, _ in _lib.SampleTimingT._fields_}

    def overlap(self, other: "GaussianMPS", stream=None, precision: str = "fp64") -> complex:
        """<self|other> by a transfer contraction on the GPU in the given
        arithmetic (fp64, fp32 or bf16x3)."""
        out = (ctypes.c_double * 2)()
        check(lib().gbs_mps_overlap_prec(self._h, other._h, _lib.PRECISIONS[precision], out, _stream_handle(stream)))
        return complex(out[0], out[1])

    def fidelity(self, other: "GaussianMPS", stream=None) -> float:
        """|<a|b>|^2 / (<a|a><b|b>), each term by the FP64 transfer contraction."""
        ab = self.overlap(other, stream)
        aa = self.overlap(self, stream).real
        bb = other.overlap(other, stream).real
        return abs(ab) ** 2 / (aa * bb)

    # -- diagnostics
    def info(self) -> dict:
        inf = InfoT()
        M = self.M
        bond = (ctypes.c_int32 * (M + 1))()
        ne = (ctypes.c_int32 * (M + 1))()
        eps = (ctypes.c_double * (M + 1))()
        ent = (ctypes.c_double * (M + 1))()
        check(lib().gbs_mps_info(self._h, ctypes.byref(inf), bond, ne, eps, ent))
        d = {f: getattr(inf, f) for f, _ in InfoT._fields_}
        d["bond"] = list(bond)
        d["ne"] = list(ne)
        d["eps"] = list(eps)
        d["entropy"] = list(ent)
        return d

    def export_elements(self, m: int, what: str, idx) -> np.ndarray:
        """gbs_mps_export_elements: complex values of the elements
        (alpha, p, beta) listed in idx (n x 3) of the "tensor" or "raw"
        tensor of site m."""
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1, 3))
        out = np.empty((idx.shape[0], 2), dtype=np.float64)
        check(lib().gbs_mps_export_elements(self._h, int(m), _lib.EXPORT[what], ctypes.c_void_p(idx.ctypes.data),
                                            idx.shape[0], ctypes.c_void_p(out.ctypes.data)))
        return out[:, 0] + 1j * out[:, 1]

    def export(self, m: int, what: str) -> np.ndarray:
        """gbs_mps_export: tensor / raw (kept[m-1] x d x kept[m]) / Q / basis /
        lambda / svals of site or cut m, or the (M+1) x 2 parity-sector sizes
        of the sampler ("sectors", m ignored), copied to host memory."""
        inf = self.info()
        d, chi = self.d, inf["chi"]
        bond, ne = inf["bond"], inf["ne"]
        kind = _lib.EXPORT[what]
        if what == "tensor":
            buf = np.empty(max(1, bond[m - 1] * d * bond[m]), dtype=np.complex128)
        elif what == "raw":
            n = bond[m - 1] * d * bond[m] if self.site else chi * d * chi
            buf = np.empty(max(1, n), dtype=np.complex128)
        elif what == "Q":
            k = ne[m - 1] + 1 + ne[m]
            buf = np.empty(max(1, k * k), dtype=np.complex128)
        elif what == "basis":
            buf = np.empty(max(1, chi * max(1, ne[m])), dtype=np.int32)
        elif what == "sectors":
            buf = np.empty(2 * (self.M + 1), dtype=np.int32)
        else:  # lambda, svals
            buf = np.empty(max(1, chi, ne[m]), dtype=np.float64)
        written = ctypes.c_int64(0)
        check(lib().gbs_mps_export(self._h, m, kind, ctypes.c_void_p(buf.ctypes.data), buf.nbytes,
                                   ctypes.byref(written)))
        arr = buf[:written.value // buf.itemsize].copy()
        if what == "tensor":
            return arr.reshape(bond[m - 1], d, bond[m])
        if what == "Q":
            k = ne[m - 1] + 1 + ne[m]
            return arr.reshape(k, k)
        if what == "raw":
            kl = len(self.export(m - 1, "basis"))
            return arr.reshape(kl, d, arr.size // (kl * d))
        if what == "basis":
            return arr.reshape(-1, ne[m]) if ne[m] else np.zeros((1, 0), dtype=np.int32)
        if what == "sectors":
            return arr.reshape(self.M + 1, 2)
        return arr


def build_site(gamma: torch.Tensor, d: int, chi: int, site: int, dstar: float = 1.0 + 1e-10,
               eps_target: float = 0.0, kept_heap: bool = False, stream=None) -> GaussianMPS:
    """The raw PCO tensor of one site (1-based) at bond dimension chi, in
    FP64, without the rest of the MPS: export(site, "raw") gives it as
    kept[site-1] x d x kept[site]; info() gives the phase times.
    eps_target > 0: the bond dimension of each cut is D(eps), capped at chi.
    kept_heap: enumerate the kept bases with the sequential heap."""
    if not isinstance(gamma, torch.Tensor) or not gamma.is_cuda or gamma.dtype != torch.float64:
        raise ValueError("gamma must be a CUDA float64 tensor")
    if gamma.dim() != 2 or gamma.shape[0] != gamma.shape[1] or gamma.shape[0] % 2:
        raise GbsError(_lib.GBS_E_INVAL, "gamma must be 2M x 2M")
    gamma = gamma.contiguous()
    M = gamma.shape[0] // 2
    opts = BuildOpts(d=d, chi=chi, dstar=dstar, prec=_lib.PRECISIONS["fp64"],
                     flags=_lib.GBS_KEPT_HEAP if kept_heap else 0, trunc_rel=0.0, eps_target=eps_target)
    h = ctypes.c_void_p()
    check(lib().gbs_mps_build_site(ctypes.c_void_p(gamma.data_ptr()), M, ctypes.byref(opts), int(site),
                                   _stream_handle(stream), ctypes.byref(h)))
    g = GaussianMPS(h, M, d)
    g.site = int(site)
    return g


def build(gamma: torch.Tensor, d: int, chi: int, dstar: float = 1.0 + 1e-10, precision: str = "fp64",
          keep_raw: bool = False, trunc_rel: float = 0.0, dense_sampler: bool = False,
          eps_target: float = 0.0, chi_build: int = 0, chain_gsvd: bool = False, kept_heap: bool = False,
          stream=None) -> GaussianMPS:
    """Convert the pure Gaussian state with covariance `gamma` (2M x 2M FP64
    CUDA tensor, xxpp, vacuum = I/2) into an MPS with cutoff d and bond chi.
    dense_sampler: FP32 sampling over whole bonds instead of photon-parity
    sectors.  eps_target > 0: per cut, the fewest kept states whose discarded
    weight is at most eps_target (at most chi).  chi_build > chi: kept bases
    and PCO tensors at chi_build states per cut, recompressed to chi by the
    truncation sweep.  chain_gsvd: run the Gaussian SVD as the sequential
    chain instead of every site on its own.  kept_heap: enumerate every kept
    basis with the sequential heap (for comparison)."""
    if not isinstance(gamma, torch.Tensor) or not gamma.is_cuda or gamma.dtype != torch.float64:
        raise ValueError("gamma must be a CUDA float64 tensor")
    if gamma.dim() != 2 or gamma.shape[0] != gamma.shape[1] or gamma.shape[0] % 2:
        raise GbsError(_lib.GBS_E_INVAL, "gamma must be 2M x 2M")
    gamma = gamma.contiguous()
    M = gamma.shape[0] // 2
    opts = BuildOpts(d=d, chi=chi, dstar=dstar, prec=_lib.PRECISIONS[precision],
                     flags=(_lib.GBS_KEEP_RAW if keep_raw else 0) | (_lib.GBS_DENSE_SAMPLER if dense_sampler else 0)
                     | (_lib.GBS_CHAIN_GSVD if chain_gsvd else 0) | (_lib.GBS_KEPT_HEAP if kept_heap else 0),
                     trunc_rel=trunc_rel, eps_target=eps_target, chi_build=chi_build)
    h = ctypes.c_void_p()
    check(lib().gbs_mps_build(ctypes.c_void_p(gamma.data_ptr()), M, ctypes.byref(opts), _stream_handle(stream),
                              ctypes.byref(h)))
    return GaussianMPS(h, M, d)


def filter_pure(gamma_th: torch.Tensor, eps: float = 0.0, alpha_max: float = 0.0, max_iter: int = 0,
                want_S: bool = False, stream=None):
    """gbs_filter_pure: pure part Gamma_p = S S^T / 2 of the mixed covariance
    gamma_th (2N x 2N FP64 CUDA tensor) by the descent of App. C.  Returns
    (gamma_p, S or None, info dict with iterations, converged, loss, n_eff, ms);
    0 selects the library's defaults (eps 1e-12, alpha_max 0.5, 100000 steps)."""
    if not isinstance(gamma_th, torch.Tensor) or not gamma_th.is_cuda or gamma_th.dtype != torch.float64:
        raise ValueError("gamma_th must be a CUDA float64 tensor")
    if gamma_th.dim() != 2 or gamma_th.shape[0] != gamma_th.shape[1] or gamma_th.shape[0] % 2:
        raise GbsError(_lib.GBS_E_INVAL, "gamma_th must be 2N x 2N")
    gamma_th = gamma_th.contiguous()
    n = gamma_th.shape[0]
    gp = torch.empty_like(gamma_th)
    S = torch.empty_like(gamma_th) if want_S else None
    info = _lib.FilterInfo()
    opts = _lib.FilterOpts(eps=eps, alpha_max=alpha_max, max_iter=max_iter)
    check(lib().gbs_filter_pure(ctypes.c_void_p(gamma_th.data_ptr()), n // 2, ctypes.byref(opts),
                                ctypes.c_void_p(gp.data_ptr()), ctypes.c_void_p(S.data_ptr()) if want_S else None,
                                ctypes.byref(info), _stream_handle(stream)))
    return gp, S, {f: getattr(info, f) for f, _ in _lib.FilterInfo._fields_}
