"""lddmm_gradient_noalloc (the gradient with the library's static scratch) gives
exactly what lddmm_gradient gives with a caller workspace, on consecutive calls
of different sizes (the scratch keeps the previous call's contents), for both
gradient kinds; a problem larger than the scratch is refused before any launch."""

import sys

import numpy as np
import pytest
import torch

from oracle import lddmm as O
from paper_1605_02060_amd import lddmm as L
from paper_1605_02060_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def _case(shape, T, h, seed):
    p = synth.blob_pair(shape, seed, max_disp=max(shape) / 10,
                        sigma=(max(shape) / 14, max(shape) / 6))
    P = tuple(O.smooth7(n) for n in shape)
    v = (h * synth.random_velocity(P, T, 600 + seed, vmax=1.5, sigma_s=3.0)).astype(np.float32)
    prm = L.Params(T=T, n_levels=1, iters=(0,), sigma=0.7, weight=(1.0, 0.5))
    return (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1)), t(v), prm


@pytest.mark.parametrize("kind", [L.GRAD_V, L.GRAD_L2])
def test_noalloc_equals_workspace_call_on_consecutive_sizes(kind):
    for shape, T, h, seed in (((32, 32, 32), 10, 0.05, 1), ((20, 18, 22), 4, 0.1, 2)):
        say(f"gradient_noalloc kind={kind} {shape} T={T}")
        imgs, v, prm = _case(shape, T, h, seed)
        g_ref, e_ref = L.lddmm_gradient(*imgs, v, prm, kind=kind, spacing=h)
        g, e = L.lddmm_gradient_noalloc(*imgs, v, prm, kind=kind, spacing=h)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), shape
        assert torch.equal(e.nan_to_num(-1.0), e_ref.nan_to_num(-1.0)), shape
        assert torch.isfinite(e[:3]).all()


def test_noalloc_refuses_a_problem_beyond_the_scratch():
    say("gradient_noalloc beyond the scratch")
    shape = (96, 96, 96)
    prm = L.Params(T=10, n_levels=1, iters=(0,))
    assert L.lddmm_workspace_size(shape, prm, 1.0) > 256 << 20
    M = torch.zeros(shape, device=DEV)
    v = torch.zeros((10, 3) + shape, device=DEV)
    grad = torch.full_like(v, 7.0)
    with pytest.raises(L.LddmmError) as e:
        L.lddmm_gradient_noalloc(M, M, None, None, v, prm, kind=L.GRAD_V, grad=grad)
    assert e.value.code == L.ESCRATCH
    torch.cuda.synchronize()
    assert bool((grad == 7.0).all())              # nothing was launched
