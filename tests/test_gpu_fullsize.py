"""Parity at the atlas size (user grid 264 x 160 x 228, T = 10, 50 um) with
the kernels the benchmark's finest level launches: the XCD-slab sweeps, the
LDS-staged backward sweep and the tiled FFT passes.  K runs on the benchmark's
finest computational grid 280 x 160 x 240; the single-level calls (energy,
gradient, and a registration without a pyramid) run on the single-level grid
270 x 160 x 240, where the backward sweep is staged as well.

The oracle cannot run whole registrations at this size in a test, so:
* K is compared on the whole grid (the oracle's FFTs take seconds);
* the regulariser of the energy is compared on the whole grid, with v a smooth
  field scaled per time step, so the expected value is one oracle evaluation;
* the maps phi_10 and phi_01 are compared on the interiors of sub-boxes: the
  value of either map at a voxel depends only on v within a few voxels per
  time step of it, so the oracle run on a box with a wide enough margin gives
  the same values there;
* the staged and the grid-stride backward sweeps (the choice only changes the
  launch) give the same bits for the energy and the V-gradient;
* E, R, D, the image SSD and 100000 sampled entries of the V-gradient of one
  velocity are compared with values the oracle computed on the whole grid
  (tests/golden/make_atlas_gradient.py wrote them).
"""

import importlib.util
import os
import sys

import numpy as np
import pytest
import torch

from oracle import lddmm as O
from paper_1605_02060_amd import lddmm as L
from paper_1605_02060_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
N = (228, 160, 264)                 # user grid [z][y][x]
P = (240, 160, 280)                 # its finest computational grid in the 3-level pyramid
P1 = (240, 160, 270)                # its computational grid without a pyramid
H = 0.05
T = 10
ALPHA, GAMMA = 0.02, 1.0
SCALES = 1.0 + 0.05 * np.arange(T)  # v_j = SCALES[j] * base


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _base_field(grid):
    """A smooth periodic field on a computational grid (physical units): a few low
    plane waves per component, at most 3 voxels per unit time (0.3 voxel per step)."""
    return synth.plane_wave_velocity(grid, 77, 3.0 * H)


PRM1 = L.Params(alpha=ALPHA, gamma=GAMMA, T=T, n_levels=1, iters=(0,))


@pytest.fixture(scope="module")
def base():
    assert L.lddmm_comp_grid(N, PRM1, 0, H) == P1
    assert L.lddmm_comp_grid(N, L.Params(T=T, n_levels=3, iters=(0, 0, 0)), 0, H) == P
    return _base_field(P1)


@pytest.fixture(scope="module")
def v_gpu(base):
    v = np.stack([s * base for s in SCALES]).astype(np.float32)
    return torch.as_tensor(v, device=DEV)


@pytest.fixture(scope="module")
def masks():
    p = synth.config_pair("atlas")
    assert p.M0.shape == N
    return p


def test_smooth_on_the_full_grid():
    say("K on 280x160x240")
    rng = np.random.default_rng(78)
    b = rng.standard_normal((3,) + P).astype(np.float32)
    got = L.lddmm_smooth(torch.as_tensor(b, device=DEV), H, ALPHA, GAMMA).cpu().numpy()
    ref = O.apply_K(b.astype(np.float64), ALPHA, GAMMA, H)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


def test_regulariser_on_the_full_grid(base, v_gpu, masks):
    say("energy R at the atlas size")
    tt = lambda a: torch.as_tensor(a, device=DEV)
    out = L.lddmm_energy(tt(masks.M0), tt(masks.M1), None, None, v_gpu, PRM1,
                         spacing=H).cpu().numpy()
    # R is quadratic in v: R(v) = (sum_j s_j^2) / T * R(base as a one-step field)
    R1 = O.reg_energy(base[None], ALPHA, GAMMA, H)
    R = (SCALES ** 2).sum() / T * R1
    assert abs(out[1] - R) <= 1e-5 * R


BOXES = [(60, 40, 60), (100, 50, 150), (120, 60, 190)]   # box corners [z][y][x]
BOX, MARGIN = 64, 24


def test_maps_on_subbox_interiors(v_gpu, masks):
    # a registration with no iterations returns the maps of the given v
    say("phi_10, phi_01 at the atlas size vs the oracle on sub-boxes")
    tt = lambda a: torch.as_tensor(a, device=DEV)
    prm = L.Params(alpha=ALPHA, gamma=GAMMA, T=T, n_levels=1, iters=(0,), guard=False)
    res = L.lddmm_register(tt(masks.M0), tt(masks.M1), params=prm, spacing=H, v=v_gpu.clone())
    torch.cuda.synchronize()
    phi10, phi01 = res["phi10"].cpu().numpy(), res["phi01"].cpu().numpy()
    v1 = v_gpu.cpu().numpy()
    for z0, y0, x0 in BOXES:
        sl = (slice(None), slice(None), slice(z0, z0 + BOX), slice(y0, y0 + BOX),
              slice(x0, x0 + BOX))
        vb = v1[sl].astype(np.float64)                          # the values the GPU holds
        u0, _ = O.forward_sweep(vb, [np.zeros(vb.shape[2:])], H, [])
        u1 = O.backward_maps(vb, H)
        core = tuple(slice(MARGIN, BOX - MARGIN) for _ in range(3))
        inner = tuple(slice(a + MARGIN, a + BOX - MARGIN) for a in (z0, y0, x0))
        e10 = np.abs(phi10[(slice(None),) + inner] - u0[T][(slice(None),) + core]).max() / H
        e01 = np.abs(phi01[(slice(None),) + inner] - u1[0][(slice(None),) + core]).max() / H
        assert e10 < 1e-4 and e01 < 1e-4, ((z0, y0, x0), e10, e01)


def test_staged_and_grid_stride_sweeps_agree_bitwise(v_gpu, masks):
    say("staged vs grid-stride backward at the atlas size")
    tt = lambda a: torch.as_tensor(a, device=DEV)
    args = (tt(masks.M0), tt(masks.M1), tt(masks.MI0), tt(masks.MI1))
    out = {}
    try:
        for name, thr in (("staged", 1), ("grid", 1 << 30)):
            L.lddmm_set_tunable(L.TUNE_STAGED_MIN_BLOCKS, thr)
            g, e = L.lddmm_gradient(*args, v_gpu, PRM1, kind=L.GRAD_V, spacing=H)
            torch.cuda.synchronize()
            out[name] = (g.cpu().numpy(), e.cpu().numpy())
    finally:
        L.lddmm_set_tunable(L.TUNE_STAGED_MIN_BLOCKS, 2048)
    np.testing.assert_array_equal(out["staged"][0], out["grid"][0])
    np.testing.assert_array_equal(out["staged"][1], out["grid"][1])
    assert np.isfinite(out["staged"][1][0])


def _golden_script():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "make_atlas_gradient.py")
    spec = importlib.util.spec_from_file_location("make_atlas_gradient", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_energy_and_gradient_against_stored_oracle(masks):
    say("E, R, D and sampled V-gradient at the atlas size vs stored oracle values")
    gs = _golden_script()
    ref = np.load(gs.OUT)
    v = gs.velocity()
    assert v.shape[2:] == P1 and gs.T == T and gs.H == H
    tt = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=DEV)
    prm = L.Params(alpha=gs.ALPHA, gamma=gs.GAMMA, sigma=gs.SIGMA, T=T, n_levels=1, iters=(0,),
                   weight=(1.0, 0.0))
    g, out = L.lddmm_gradient(tt(masks.M0), tt(masks.M1), tt(masks.MI0), tt(masks.MI1), tt(v), prm,
                              kind=L.GRAD_V, spacing=H)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    for k, name in enumerate(("E", "R", "D", "img_ssd")):
        assert abs(out[k] - float(ref[name])) <= 1e-5 * abs(float(ref[name])), name
    idx = torch.as_tensor(ref["idx"].astype(np.int64), device=DEV)
    got = g.reshape(-1)[idx].cpu().numpy().astype(np.float64)
    err = np.abs(got - ref["g"].astype(np.float64)).max() / float(ref["g_absmax"])
    assert err < 2e-5, err
