"""gbs_mps_sample_noalloc (sampling on the library's static device scratch
array, for callers that cannot allocate) against gbs_mps_sample, through the
C ABI: the samples must be identical, integer for integer.

Two calls in a row share the one scratch array: the first at the 144-mode,
chi = 256 workload with more shots than one scratch-sized sweep holds (so the
shots go through in several sweeps), the second on a smaller state with fewer
shots.  A third call samples an FP64 handle (the vector sweep)."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _build(torch, name, precision):
    from paper_2512_10643_amd import mps as gmps
    w = W.workload(name)
    g = torch.tensor(w.gamma, dtype=torch.float64, device="cuda")
    return w, gmps.build(g, w.d, w.chi, precision=precision)


def _compare(torch, h, shots, seed):
    ref = h.sample(shots, seed)
    got = torch.full((shots, h.M), -1, dtype=torch.int32, device="cuda")
    h.sample_noalloc(shots, seed, got)
    torch.cuda.synchronize()
    ref, got = ref.cpu().numpy(), got.cpu().numpy()
    diff = int(np.count_nonzero(ref != got))
    _say(f"  M={h.M} shots={shots} seed={seed}: {diff} entries differ")
    assert diff == 0
    assert np.all(got.sum(1) % 2 == 0)


def test_noalloc_sampling_equals_sample_on_two_calls(torch_cuda):
    from paper_2512_10643_amd import _lib
    torch = torch_cuda
    _say("noalloc: c3 fp32, 300077 shots (several scratch-sized sweeps)")
    w3, h3 = _build(torch, "c3", "fp32")
    # two rows of left vectors per shot, each at least the widest parity sector in FP32 complex
    per_shot = 2 * 8 * int(h3.export(0, "sectors").max())
    assert 300_077 * per_shot > _lib.GBS_SAMPLE_NOALLOC_SCRATCH_BYTES  # more than one sweep
    _compare(torch, h3, 300_077, seed=11)
    _say("noalloc: c2 fp32, 5003 shots (smaller input on the same scratch)")
    w2, h2 = _build(torch, "c2", "fp32")
    _compare(torch, h2, 5_003, seed=12)
    h3.free()
    h2.free()


def test_noalloc_vector_sweep_and_errors(torch_cuda):
    from paper_2512_10643_amd import _lib
    torch = torch_cuda
    _say("noalloc: c1 fp64 (vector sweep), 3001 shots")
    w1, h1 = _build(torch, "c1", "fp64")
    _compare(torch, h1, 3_001, seed=13)
    L = _lib.lib()
    out = torch.empty((4, w1.M), dtype=torch.int32, device="cuda")
    assert L.gbs_mps_sample_noalloc(None, 4, 0, out.data_ptr(), None) == _lib.GBS_E_INVAL
    assert L.gbs_mps_sample_noalloc(h1._h, -1, 0, out.data_ptr(), None) == _lib.GBS_E_INVAL
    assert L.gbs_mps_sample_noalloc(h1._h, 4, 0, None, None) == _lib.GBS_E_INVAL
    assert L.gbs_mps_sample_noalloc(h1._h, 0, 0, None, None) == _lib.GBS_OK
    h1.free()
