"""Batched registration: one launch per stage for several problems of uneven
size must give exactly the results of independent single-problem calls."""

import sys
import time

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


def _pairs(shapes, seed0=400, with_img=True):
    out = []
    for k, shp in enumerate(shapes):
        p = synth.blob_pair(shp, seed0 + k, max_disp=max(shp) / 10,
                            sigma=(max(shp) / 16, max(shp) / 6.4))
        d = {"M0": t(p.M0), "M1": t(p.M1), "spacing": 0.05}
        if with_img:
            d["MI0"], d["MI1"] = t(p.MI0), t(p.MI1)
        out.append((p, d))
    return out


@pytest.mark.parametrize("guard,levels,iters,staged", [(True, 2, (6, 5), False),
                                                       (False, 1, (5,), False),
                                                       (True, 2, (6, 5), True)])
def test_batched_equals_single_calls(guard, levels, iters, staged):
    # staged: force the LDS-staged backward kernel on these small grids
    say(f"batched vs single guard={guard} levels={levels} staged={staged}")
    shapes = [(20, 24, 28), (32, 32, 32), (18, 30, 22), (26, 20, 34)]
    pairs = _pairs(shapes)
    prm = L.Params(T=5, n_levels=levels, iters=iters, step=0.05 if guard else 0.02, guard=guard,
                   weight=(1.0, 0.3))
    L.lddmm_set_tunable(L.TUNE_STAGED_MIN_BLOCKS, 1 if staged else 2048)
    try:
        res, code = L.lddmm_register_batched([d for _, d in pairs], prm)
        torch.cuda.synchronize()
        for (p, d), r in zip(pairs, res):
            single = L.lddmm_register(d["M0"], d["M1"], d["MI0"], d["MI1"], params=prm,
                                      spacing=d["spacing"])
            torch.cuda.synchronize()
            assert r["status"] == single["status"]
            assert torch.equal(r["v"], single["v"])
            assert torch.equal(r["phi10"], single["phi10"])
            assert torch.equal(r["phi01"], single["phi01"])
            assert torch.equal(r["trace"].nan_to_num(-1.0), single["trace"].nan_to_num(-1.0))
    finally:
        L.lddmm_set_tunable(L.TUNE_STAGED_MIN_BLOCKS, 2048)


def test_batched_matches_oracle_for_each_problem():
    say("batched vs oracle")
    shapes = [(16, 20, 18), (24, 16, 20)]
    pairs = _pairs(shapes, seed0=410)
    prm = L.Params(T=4, iters=(5,), step=0.02, weight=(1.0, 0.0))
    res, code = L.lddmm_register_batched([d for _, d in pairs], prm)
    torch.cuda.synchronize()
    for (p, d), r in zip(pairs, res):
        oprm = O.Params(T=4, iters=(5,), step=0.02, spacing=0.05, weight=(1.0, 0.0))
        ref = O.register(O.Problem(p.M0, p.M1, p.MI0, p.MI1), oprm)
        tr = r["trace"].cpu().numpy()
        rt = np.array(ref.trace)
        np.testing.assert_array_equal(tr[:, 6], rt[:, 6])
        assert np.all(np.abs(tr[:, 7] - rt[:, 7]) <= 1e-5 * np.abs(rt[:, 7]))
        assert np.abs(r["phi10"].cpu().numpy() - ref.phi10).max() / 0.05 < 1e-4


def test_batched_sixteen_uneven_pairs_timing():
    # the batched workload: 16 pairs, sizes from rng(4) in 64..160 per axis, T = 10;
    # iterations cut to 10 here (timing comparison only)
    dims = synth.batched_dims()
    shapes = [(int(z), int(y), int(x)) for x, y, z in dims]
    say(f"batched 16 pairs {shapes[:3]}...")
    pairs = []
    for k, shp in enumerate(shapes):
        s = min(shp) / 32.0
        p = synth.blob_pair(shp, 400 + k, max_disp=3 * s, sigma=(2 * s, 5 * s))
        pairs.append({"M0": t(p.M0), "M1": t(p.M1), "spacing": 0.05})
    prm = L.Params(T=10, iters=(10,), step=0.02, guard=False)
    wss = [L.workspace(d["M0"].shape, prm, 0.05) for d in pairs]
    res, code = L.lddmm_register_batched(pairs, prm, wss=wss, want_phi=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, code = L.lddmm_register_batched(pairs, prm, wss=wss, want_phi=False)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    for d, ws in zip(pairs, wss):
        L.lddmm_register(d["M0"], d["M1"], params=prm, spacing=0.05, ws=ws, want_phi=False)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    print(f"16 pairs x 10 iterations: batched {tb:.3f} s, sequential {ts:.3f} s")
    assert code in (L.OK, L.WFOLD)


def test_tunables_do_not_change_results():
    from paper_1605_02060_amd import tune
    say("tunables: results independent of launch shapes")
    p = synth.blob_pair((22, 30, 26), 420, max_disp=2.5, sigma=(1.5, 4.0))
    M0, M1, MI0, MI1 = t(p.M0), t(p.M1), t(p.MI0), t(p.MI1)
    prm = L.Params(T=4, iters=(3,), step=0.02, guard=False, weight=(1.0, 0.5))
    tune.set_all(tune.DEFAULTS)
    ref = L.lddmm_register(M0, M1, MI0, MI1, params=prm, spacing=0.05)
    try:
        for which, values in tune.CANDIDATES.items():
            for v in values:
                say(f"tunable {tune.NAMES[which]} = {v}")
                tune.set_all(tune.DEFAULTS)
                L.lddmm_set_tunable(which, v)
                r = L.lddmm_register(M0, M1, MI0, MI1, params=prm, spacing=0.05)
                torch.cuda.synchronize()
                assert torch.equal(r["v"], ref["v"]), (which, v)
                assert torch.equal(r["phi10"], ref["phi10"]) and torch.equal(r["phi01"], ref["phi01"])
                e, e0 = r["trace"][:, :3], ref["trace"][:, :3]
                assert torch.allclose(e, e0, rtol=1e-12, atol=0.0), (which, v)
    finally:
        tune.set_all(tune.DEFAULTS)


def test_autotune_picks_candidates_and_caches(tmp_path, monkeypatch):
    from paper_1605_02060_amd import tune
    say("autotune on three uneven pairs")
    monkeypatch.setenv("LDDMM_TUNE_CACHE", str(tmp_path / "tune.json"))
    pairs = [d for _, d in _pairs([(24, 20, 28), (30, 26, 18), (20, 32, 24)], seed0=430,
                                  with_img=False)]
    prm = L.Params(T=4, iters=(3,), step=0.02, guard=False)
    try:
        choice = tune.autotune(pairs, prm, iters=2, repeats=1)
        for which, v in choice.items():
            assert v in tune.CANDIDATES[which]
        assert (tmp_path / "tune.json").exists()
        again = tune.autotune(pairs, prm)                 # served from the cache
        assert again == choice
        res, code = L.lddmm_register_batched(pairs, prm)
        torch.cuda.synchronize()
        tune.set_all(tune.DEFAULTS)
        ref, code0 = L.lddmm_register_batched(pairs, prm)
        torch.cuda.synchronize()
        for a, b in zip(res, ref):
            assert torch.equal(a["v"], b["v"])
    finally:
        tune.set_all(tune.DEFAULTS)
