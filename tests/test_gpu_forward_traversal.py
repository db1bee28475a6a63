"""The forward sweep's two traversals: plane-marching tiles (each thread walks a
run of z-planes, the velocity's z neighbours held in registers) and the
grid-stride sweep (LDDMM_TUNE_FWD_TILES = 0).  Both compute every voxel with the
same expressions, so maps, deformed templates and the velocity after descent
steps are bitwise equal; only the order of the FP64 energy sums differs.

The tile counts used here give runs of one plane, of several planes with a
ragged last run, and of the whole column, on grids whose xy plane is not a
multiple of the block size.  The oracle pins the energies at a multi-plane
setting; the default setting on these small grids gives one-plane runs, which
the other parity tests cover.
"""

import sys

import numpy as np
import pytest
import torch

from oracle import lddmm as O
from paper_1605_02060_amd import lddmm as L
from paper_1605_02060_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
DEFAULT_TILES = 1792


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def host(x):
    return x.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.fixture
def restore_tiles():
    yield
    L.lddmm_set_tunable(L.TUNE_FWD_TILES, DEFAULT_TILES)


# user grid [z][y][x]; computational grid 30 x 40 x 45 on one level, 30 x 40 x 48
# at the finest of two: xy planes of 1800 and 1920 voxels, 8 blocks of 256 with a
# ragged last one
SHAPE = (29, 40, 45)


@pytest.mark.parametrize("rk4", [False, True])
def test_traversals_give_the_same_registration(rk4, restore_tiles):
    p = synth.blob_pair(SHAPE, 450, max_disp=2.5, sigma=(1.5, 4.0))
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1))
    prm = L.Params(T=4, n_levels=2, iters=(3, 3), step=0.02, guard=False, weight=(1.0, 0.5),
                   flags=L.FLAG_RK4 if rk4 else 0)
    out = {}
    # on the finest grid -- 0: grid-stride; 1: 8 tiles, one run of all 30 planes
    # per plane block; 16: runs of 15; 32: runs of 8 with a ragged last run of 6;
    # 3584: one plane per run; 1792, the default
    for tiles in (0, 1, 16, 32, 3584, DEFAULT_TILES):
        say(f"forward tiles {tiles} rk4={rk4}")
        L.lddmm_set_tunable(L.TUNE_FWD_TILES, tiles)
        r = L.lddmm_register(*args, params=prm, spacing=0.05)
        torch.cuda.synchronize()
        out[tiles] = r
    ref = out[0]
    for tiles, r in out.items():
        assert r["status"] == ref["status"], tiles
        for k in ("v", "phi10", "phi01"):
            assert torch.equal(r[k], ref[k]), (tiles, k)
        e, e0 = r["trace"][:, :3], ref["trace"][:, :3]
        assert torch.allclose(e, e0, rtol=1e-12, atol=0.0), tiles


def test_multi_plane_runs_match_the_oracle(restore_tiles):
    h, T = 0.05, 4
    p = synth.blob_pair(SHAPE, 451, max_disp=2.0, sigma=(2.0, 4.0))
    P = tuple(O.smooth7(n) for n in SHAPE)
    v = (h * synth.random_velocity(P, T, 121, vmax=2.0, sigma_s=3.0)).astype(np.float32)
    prm = O.Params(T=T, spacing=h, weight=(1.0, 0.3))
    ref = O.energy(O.Problem(p.M0, p.M1, p.MI0, p.MI1), prm, v.astype(np.float64))
    lp = L.Params(T=T, n_levels=1, iters=(0,), weight=(1.0, 0.3))
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1))
    for tiles in (1, 32):
        say(f"energy vs oracle, forward tiles {tiles}")
        L.lddmm_set_tunable(L.TUNE_FWD_TILES, tiles)
        out = host(L.lddmm_energy(*args, t(v), lp, spacing=h))
        assert rel(out[0], ref["E"]) < 1e-5
        assert rel(out[1], ref["R"]) < 1e-5
        assert rel(out[2], ref["D"]) < 1e-5


def test_batched_equals_single_with_multi_plane_runs(restore_tiles):
    say("batched vs single, forward tiles 32")
    L.lddmm_set_tunable(L.TUNE_FWD_TILES, 32)
    shapes = [(20, 24, 28), SHAPE, (18, 30, 22)]
    pairs = []
    for k, shp in enumerate(shapes):
        p = synth.blob_pair(shp, 460 + k, max_disp=max(shp) / 10,
                            sigma=(max(shp) / 16, max(shp) / 6.4))
        pairs.append({"M0": t(p.M0), "M1": t(p.M1), "MI0": t(p.MI0), "MI1": t(p.MI1),
                      "spacing": 0.05})
    prm = L.Params(T=5, n_levels=2, iters=(4, 3), step=0.05, guard=True, weight=(1.0, 0.3))
    res, code = L.lddmm_register_batched(pairs, prm)
    torch.cuda.synchronize()
    for d, r in zip(pairs, res):
        single = L.lddmm_register(d["M0"], d["M1"], d["MI0"], d["MI1"], params=prm,
                                  spacing=d["spacing"])
        torch.cuda.synchronize()
        assert r["status"] == single["status"]
        for k in ("v", "phi10", "phi01"):
            assert torch.equal(r[k], single[k]), k
        assert torch.equal(r["trace"].nan_to_num(-1.0), single["trace"].nan_to_num(-1.0))


def test_tunable_rejects_negative_values(restore_tiles):
    with pytest.raises(Exception):
        L.lddmm_set_tunable(L.TUNE_FWD_TILES, -1)
    L.lddmm_set_tunable(L.TUNE_FWD_TILES, 0)


# ----------------------------------------------- LDS-staged forward sweep ----
# LDDMM_TUNE_FWD_STAGED_MIN_BLOCKS = 1 stages every grid: 64 x 4 columns over
# z-slabs with a ring of u0 planes in LDS (gathers leaving the window read
# global memory).  Same expressions, so the same bits as the other traversals.

@pytest.fixture
def restore_staged():
    yield
    L.lddmm_set_tunable(L.TUNE_FWD_STAGED_MIN_BLOCKS, 2048)
    L.lddmm_set_tunable(L.TUNE_FWD_TILES, DEFAULT_TILES)


# weight (1, 0) leaves one weighted channel, whose template planes the first-order
# interior steps also stage in LDS; (1, 0.5) weights two, read from global memory
@pytest.mark.parametrize("weight", [(1.0, 0.5), (1.0, 0.0)])
@pytest.mark.parametrize("rk4", [False, True])
@pytest.mark.parametrize("vmax", [2.0, 40.0])
def test_staged_forward_gives_the_same_registration(rk4, vmax, weight, restore_staged):
    # vmax 40 voxels per unit time: 10 voxels per step at T = 4, far outside the window
    p = synth.blob_pair(SHAPE, 452, max_disp=2.5, sigma=(1.5, 4.0))
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1))
    prm = L.Params(T=4, n_levels=2, iters=(3, 3), step=0.02, guard=False, weight=weight,
                   flags=L.FLAG_RK4 if rk4 else 0)
    P = L.lddmm_comp_grid(SHAPE, prm, 0, 0.05)
    v0 = t(0.05 * synth.random_velocity(P, 4, 122, vmax=vmax, sigma_s=3.0))
    out = {}
    for name, staged, tiles in (("grid", 1 << 30, 0), ("march", 1 << 30, DEFAULT_TILES),
                                ("staged", 1, DEFAULT_TILES)):
        say(f"forward traversal {name} rk4={rk4} vmax={vmax} weight={weight}")
        L.lddmm_set_tunable(L.TUNE_FWD_TILES, tiles)
        L.lddmm_set_tunable(L.TUNE_FWD_STAGED_MIN_BLOCKS, staged)
        r = L.lddmm_register(*args, params=prm, spacing=0.05, v=v0.clone())
        torch.cuda.synchronize()
        out[name] = r
    ref = out["grid"]
    for name, r in out.items():
        assert r["status"] == ref["status"], name
        for k in ("v", "phi10", "phi01"):
            assert torch.equal(r[k], ref[k]), (name, k)
        e, e0 = r["trace"][:, :3], ref["trace"][:, :3]
        assert torch.allclose(e, e0, rtol=1e-12, atol=0.0), name


# ragged tiles (64 x 4 columns): x = 45 fills 45 columns of one tile and y = 30
# leaves two rows in the last tile; x = 225 = 3 * 64 + 33 and y = 21 one row;
# x = 450 = 7 * 64 + 2 leaves two columns, the last of whose x + 1 (periodic)
# lies in the first tile, and y = 9 one row.  (A one-column tile would need a
# 7-smooth x of 64 k + 1; the first is 2625, above the largest axis, 1024.)
RAGGED = [(10, 30, 45), (10, 21, 225), (10, 9, 450)]


@pytest.mark.parametrize("weight", [(1.0, 0.5), (1.0, 0.0)])
@pytest.mark.parametrize("shape", RAGGED)
@pytest.mark.parametrize("rk4", [False, True])
def test_staged_forward_on_ragged_tiles(shape, rk4, weight, restore_staged):
    p = synth.blob_pair(shape, 454, max_disp=2.0, sigma=(1.5, 3.0))
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1))
    prm = L.Params(T=3, n_levels=1, iters=(3,), step=0.02, guard=False, weight=weight,
                   flags=L.FLAG_RK4 if rk4 else 0)
    P = L.lddmm_comp_grid(shape, prm, 0, 0.05)
    assert P == shape
    v0 = t(0.05 * synth.random_velocity(P, 3, 124, vmax=3.0, sigma_s=2.0))
    out = {}
    for name, staged, tiles in (("grid", 1 << 30, 0), ("staged", 1, DEFAULT_TILES)):
        say(f"forward traversal {name} on ragged tiles {shape}, rk4={rk4}, weight={weight}")
        L.lddmm_set_tunable(L.TUNE_FWD_TILES, tiles)
        L.lddmm_set_tunable(L.TUNE_FWD_STAGED_MIN_BLOCKS, staged)
        r = L.lddmm_register(*args, params=prm, spacing=0.05, v=v0.clone())
        torch.cuda.synchronize()
        out[name] = r
    a, b = out["grid"], out["staged"]
    assert a["status"] == b["status"]
    for k in ("v", "phi10", "phi01"):
        assert torch.equal(a[k], b[k]), k
    assert torch.allclose(a["trace"][:, :3], b["trace"][:, :3], rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("weight", [(1.0, 0.3), (1.0, 0.0)])
def test_staged_forward_energy_matches_the_oracle(weight, restore_staged):
    h, T = 0.05, 4
    p = synth.blob_pair(SHAPE, 453, max_disp=2.0, sigma=(2.0, 4.0))
    P = tuple(O.smooth7(n) for n in SHAPE)
    v = (h * synth.random_velocity(P, T, 123, vmax=6.0, sigma_s=3.0)).astype(np.float32)
    prm = O.Params(T=T, spacing=h, weight=weight)
    ref = O.energy(O.Problem(p.M0, p.M1, p.MI0, p.MI1), prm, v.astype(np.float64))
    lp = L.Params(T=T, n_levels=1, iters=(0,), weight=weight)
    L.lddmm_set_tunable(L.TUNE_FWD_STAGED_MIN_BLOCKS, 1)
    say(f"staged forward: energy vs oracle, weight={weight}")
    out = host(L.lddmm_energy(t(p.M0), t(p.M1), t(p.MI0), t(p.MI1), t(v), lp, spacing=h))
    for k, name in enumerate(("E", "R", "D", "img_ssd")):
        assert rel(out[k], ref[name]) < 1e-5, name


def test_staged_forward_batched_equals_single(restore_staged):
    say("batched vs single, staged forward")
    L.lddmm_set_tunable(L.TUNE_FWD_STAGED_MIN_BLOCKS, 1)
    shapes = [(20, 24, 28), SHAPE, (18, 30, 22)]
    pairs = []
    for k, shp in enumerate(shapes):
        p = synth.blob_pair(shp, 470 + k, max_disp=max(shp) / 10,
                            sigma=(max(shp) / 16, max(shp) / 6.4))
        pairs.append({"M0": t(p.M0), "M1": t(p.M1), "spacing": 0.05})
    prm = L.Params(T=5, n_levels=2, iters=(4, 3), step=0.05, guard=True)
    res, code = L.lddmm_register_batched(pairs, prm)
    torch.cuda.synchronize()
    for d, r in zip(pairs, res):
        single = L.lddmm_register(d["M0"], d["M1"], params=prm, spacing=d["spacing"])
        torch.cuda.synchronize()
        for k in ("v", "phi10", "phi01"):
            assert torch.equal(r[k], single[k]), k
        assert torch.equal(r["trace"].nan_to_num(-1.0), single["trace"].nan_to_num(-1.0))
