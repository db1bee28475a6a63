"""K over all time steps at once (LDDMM_TUNE_K_TIME_BATCH), through the C ABI.

On the levels of a registration with at most 2^21 voxels the backward sweep
keeps the T body forces and then smooths and updates all of them, one batched
launch per pass.  The sweep reads the current iterate, which the update does
not write, so the descent is the same; the batched passes transform each line
as the single-step ones do, so the results must be the same bits:

* multi-level registrations with the guard on (rejected trials replay the
  update) and off, one and two weighted channels, first order and RK4;
* T = 40, which takes two batched launches per pass (32 time steps each at most);
* the coarse levels' fused x + y passes (a 32 x 32 plane) and the separate
  passes of the other grids;
* and against the FP64 oracle on a small registration."""

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


@pytest.fixture
def restore():
    yield
    L.lddmm_set_tunable(L.TUNE_K_TIME_BATCH, 1)


def _both(args, prm, h, v0=None):
    out = {}
    for on in (0, 1):
        L.lddmm_set_tunable(L.TUNE_K_TIME_BATCH, on)
        r = L.lddmm_register(*args, params=prm, spacing=h,
                             v=None if v0 is None else v0.clone())
        torch.cuda.synchronize()
        out[on] = r
    return out[0], out[1]


def _same(a, b):
    assert a["status"] == b["status"]
    for k in ("v", "phi10", "phi01"):
        assert torch.equal(a[k], b[k]), k
    assert torch.equal(a["trace"].nan_to_num(-1.0), b["trace"].nan_to_num(-1.0))


CASES = [
    # shape, T, levels, iters, guard, weight, rk4
    ((20, 24, 28), 5, 2, (4, 3), True, (1.0, 0.0), False),
    ((20, 24, 28), 5, 2, (4, 3), False, (1.0, 0.5), False),
    ((24, 20, 30), 4, 2, (3, 3), True, (1.0, 0.0), True),
    ((64, 64, 64), 6, 2, (3, 2), True, (1.0, 0.0), False),     # 32 x 32 coarse planes: fused
    ((14, 18, 16), 40, 1, (3,), True, (1.0, 0.3), False),      # two launches per pass
]


@pytest.mark.parametrize("shape,T,levels,iters,guard,weight,rk4", CASES)
def test_time_batched_K_gives_the_same_registration(shape, T, levels, iters, guard, weight, rk4,
                                                    restore):
    say(f"time-batched K {shape} T={T} levels={levels} guard={guard} weight={weight} rk4={rk4}")
    p = synth.blob_pair(shape, 611, max_disp=max(shape) / 10,
                        sigma=(max(shape) / 16, max(shape) / 6.4))
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1))
    prm = L.Params(T=T, n_levels=levels, iters=iters, step=0.05, guard=guard, weight=weight,
                   flags=L.FLAG_RK4 if rk4 else 0)
    a, b = _both(args, prm, 0.05)
    _same(a, b)


def test_time_batched_K_from_a_given_velocity(restore):
    # a registration that starts from a nonzero v (every time step differs)
    shape, T = (20, 22, 26), 6
    say(f"time-batched K from a given v {shape} T={T}")
    p = synth.blob_pair(shape, 612, max_disp=2.0, sigma=(1.5, 4.0))
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1))
    prm = L.Params(T=T, n_levels=1, iters=(5,), step=0.05, guard=True, weight=(1.0, 0.5))
    P = L.lddmm_comp_grid(shape, prm, 0, 0.05)
    v0 = t(0.05 * synth.random_velocity(P, T, 613, vmax=2.0, sigma_s=2.0))
    a, b = _both(args, prm, 0.05, v0)
    _same(a, b)


def test_time_batched_K_matches_the_oracle(restore):
    shape, h = (16, 18, 20), 0.05
    prm = O.Params(T=5, n_levels=2, iters=(4, 3), step=0.05, spacing=h, guard=True,
                   weight=(1.0, 0.0))
    p = synth.blob_pair(shape, 614, max_disp=2.0, sigma=(1.5, 3.5))
    say(f"time-batched K vs oracle {shape}")
    ref = O.register(O.Problem(p.M0, p.M1), prm)
    L.lddmm_set_tunable(L.TUNE_K_TIME_BATCH, 1)
    lp = L.Params(alpha=prm.alpha, gamma=prm.gamma, sigma=prm.sigma, T=prm.T,
                  n_levels=prm.n_levels, iters=prm.iters, step=prm.step, guard=prm.guard,
                  weight=prm.weight)
    r = L.lddmm_register(t(p.M0), t(p.M1), params=lp, spacing=h)
    torch.cuda.synchronize()
    v = r["v"].cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(v, ref.v, atol=1e-4 * np.abs(ref.v).max())
