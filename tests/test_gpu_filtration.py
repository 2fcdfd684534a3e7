"""Mixed -> pure filtration on the GPU (gbs_filter_pure, App. C) against the
CPU oracle's descent and against closed forms.  FP64 throughout: Gamma_p and
N_eff within 1e-10.

Inputs: squeezers with source loss and thermal photons through a passive
interferometer (the shape of a lossy boson-sampling experiment), whose
optimum is known in closed form, and the same with correlated noise (no
closed form; the descent itself is compared, on a seed whose lowest
eigenvalue stays separated from the next one along the way, so both sides
take the same steps)."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import build as obuild, filtration as F, mps as omps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu_filter(torch, g, **kw):
    from paper_2512_10643_amd import mps as gmps
    t = torch.tensor(np.asarray(g), dtype=torch.float64, device="cuda")
    gp, S, info = gmps.filter_pure(t, want_S=True, **kw)
    return gp.cpu().numpy(), S.cpu().numpy(), info


def _closed_form(x):
    b = x["eta"] * np.exp(-2 * x["r"]) + 1 - x["eta"] + 2 * x["n_th"]
    rp = np.maximum(0.0, -0.5 * np.log(b))
    return W.gamma_of_circuit(rp, x["U"]), float(np.sum(np.sinh(rp) ** 2))


@pytest.mark.parametrize("M,circuit,seed", [(16, "haar", 3), (32, ("brick", 8), 9), (72, "haar", 10)])
def test_filtration_matches_oracle(torch_cuda, M, circuit, seed):
    _say(f"case: lossy sources M={M} {circuit} seed={seed}: GPU filtration vs oracle descent")
    x = W.lossy(M=M, circuit=circuit, seed=seed)
    gp, S, info = _gpu_filter(torch_cuda, x["gamma"])
    res = F.filter_pure(x["gamma"])
    want, neff = _closed_form(x)
    err = float(np.max(np.abs(gp - res.gamma_p)))
    _say(f"  gpu {info['iterations']} steps in {info['ms']:.1f} ms (loss {info['loss']:.1e}), oracle "
         f"{res.iterations} steps; max |Gp_gpu - Gp_oracle| = {err:.2e}; N_eff {info['n_eff']:.10f} vs "
         f"{res.n_eff:.10f} (closed form {neff:.10f})")
    assert info["converged"] == 1 and info["loss"] <= 1e-12
    assert err <= 1e-10
    assert abs(info["n_eff"] - res.n_eff) <= 1e-10
    assert np.max(np.abs(gp - want)) <= 1e-10
    om = np.block([[np.zeros((M, M)), np.eye(M)], [-np.eye(M), np.zeros((M, M))]])
    assert np.max(np.abs(S @ om @ S.T - om)) <= 1e-10


def test_filtration_at_144_modes_closed_form(torch_cuda):
    """144 lossy sources through a Haar interferometer (the size of the
    paper's Jiuzhang 2.0 benchmark and of the 144-mode workload): the GPU's
    pure part against the closed-form optimum."""
    _say("case: lossy sources M=144 haar: GPU filtration vs closed form")
    x = W.lossy(M=144, r=(0.1, 0.8), eta=(0.4, 0.8), seed=12)
    gp, S, info = _gpu_filter(torch_cuda, x["gamma"])
    want, neff = _closed_form(x)
    err = float(np.max(np.abs(gp - want)))
    _say(f"  {info['iterations']} steps in {info['ms']:.1f} ms; max |Gp - Gp*| = {err:.2e}; "
         f"N_eff {info['n_eff']:.10f} vs {neff:.10f}")
    assert info["converged"] == 1
    assert err <= 1e-10 and abs(info["n_eff"] - neff) <= 1e-10


def test_filtration_correlated_noise_matches_oracle(torch_cuda):
    _say("case: lossy sources M=8 with correlated noise: GPU vs oracle descent")
    x = W.lossy(M=8, seed=5, noise=0.05)
    res = F.filter_pure(x["gamma"])
    assert res.min_gap > 1e-8  # the two sides take the same steps
    gp, S, info = _gpu_filter(torch_cuda, x["gamma"])
    err = float(np.max(np.abs(gp - res.gamma_p)))
    _say(f"  gpu {info['iterations']} steps, oracle {res.iterations}; max |dGp| = {err:.2e}; "
         f"N_eff {info['n_eff']:.12f} vs {res.n_eff:.12f}")
    assert info["iterations"] == res.iterations
    assert err <= 1e-10 and abs(info["n_eff"] - res.n_eff) <= 1e-10


def test_filtration_special_cases_and_errors(torch_cuda):
    """A squeezed thermal mode (closed form), a state without squeezing (no
    step), a pure input (its own pure part) and the argument checks."""
    from paper_2512_10643_amd import GbsError, mps as gmps
    torch = torch_cuda
    r, nu = 0.7, 1.3
    g1 = 0.5 * nu * np.diag([np.exp(2 * r), np.exp(-2 * r)])
    gp, S, info = _gpu_filter(torch, g1)
    rp = r - 0.5 * np.log(nu)
    assert np.max(np.abs(gp - 0.5 * np.diag([np.exp(2 * rp), np.exp(-2 * rp)]))) <= 1e-10
    u = W.haar_unitary(5, np.random.default_rng(0))
    gp, S, info = _gpu_filter(torch, W.lossy_gamma(np.zeros(5), u, 0.7, n_th=0.05))
    assert info["iterations"] == 0 and np.array_equal(S, np.eye(10)) and info["n_eff"] == 0.0
    w = W.workload("c1")
    gp, S, info = _gpu_filter(torch, w.gamma)
    assert np.max(np.abs(gp - w.gamma)) <= 1e-9
    with pytest.raises(GbsError):
        gmps.filter_pure(torch.zeros((2 * 300, 2 * 300), dtype=torch.float64, device="cuda"))
    bad = np.eye(4)
    bad[0, 1] = 0.3
    with pytest.raises(GbsError):
        gmps.filter_pure(torch.tensor(bad, device="cuda"))
    gp, S, info = _gpu_filter(torch, W.lossy(M=6, seed=2)["gamma"], max_iter=3)
    assert info["iterations"] == 3 and info["converged"] == 0


def test_filtered_state_builds_the_oracles_mps(torch_cuda):
    """Lossy input -> pure part on the GPU -> MPS on the GPU, against the
    oracle's filtration and MPS build of the same input (8 modes, d=4,
    chi=16, FP64): amplitudes within 1e-10."""
    import itertools
    from paper_2512_10643_amd import mps as gmps
    torch = torch_cuda
    _say("case: lossy M=8 -> filtration -> MPS (d=4, chi=16) vs oracle")
    x = W.lossy(M=8, r=(0.5, 0.9), seed=14)
    t = torch.tensor(x["gamma"], dtype=torch.float64, device="cuda")
    gp, _, info = gmps.filter_pure(t)
    h = gmps.build(gp, 4, 16, precision="fp64")
    res = F.filter_pure(x["gamma"])
    o = obuild.build_mps(res.gamma_p, 4, 16)
    pats = [p for p in itertools.product(range(4), repeat=8) if sum(p) <= 4]
    got = h.amplitude(torch.tensor(pats, dtype=torch.int32, device="cuda")).cpu().numpy()
    ref = omps.amplitudes(o.tensors, pats)
    err = float(np.max(np.abs(got - ref)))
    _say(f"  {len(pats)} amplitudes: max |delta| = {err:.2e}; N_eff {info['n_eff']:.6f}")
    assert err <= 1e-10
    s = h.sample(2048, seed=3)
    assert int((s.sum(1) % 2).abs().sum()) == 0
    h.free()
