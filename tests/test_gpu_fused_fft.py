"""K with the fused x + y passes (one component's xy plane of the half spectrum
in LDS, LDDMM_TUNE_FFT_FUSED_LDS) against the FP64 oracle and against the
separate passes.  The fused passes pack two rows of one component per complex
line where the separate passes pack rows across components, so the two agree to
FP32 rounding, not bit for bit; batched calls take the same fused passes as
single calls and stay bitwise equal to them."""

import sys

import numpy as np
import pytest
import torch

from oracle import lddmm as O
from paper_1605_02060_amd import lddmm as L
from paper_1605_02060_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
FUSED_DEFAULT = 81920


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def host(x):
    return x.detach().cpu().numpy().astype(np.float64)


@pytest.fixture
def restore_fused():
    yield
    L.lddmm_set_tunable(L.TUNE_FFT_FUSED_LDS, FUSED_DEFAULT)


# grids [z][y][x] whose (x, y) has a fused plan: the middle and coarsest atlas
# levels, 32 x 32 and 64 x 64
@pytest.mark.parametrize("P,h,alpha,gamma", [
    ((120, 80, 140), 0.1, 0.02, 1.0),
    ((60, 40, 70), 0.2, 0.02, 1.0),
    ((32, 32, 32), 1.0, 0.3, 1.0),
    ((18, 64, 64), 0.5, 0.7, 0.5),
])
def test_fused_smooth_matches_oracle_and_separate_passes(P, h, alpha, gamma, restore_fused):
    b = np.random.default_rng(7).normal(size=(3,) + P)
    ref = O.apply_K(b, alpha, gamma, h)
    out = {}
    for name, lds in (("fused", FUSED_DEFAULT), ("separate", 0)):
        say(f"smooth {name} P={P}")
        L.lddmm_set_tunable(L.TUNE_FFT_FUSED_LDS, lds)
        o = L.lddmm_smooth(t(b), h, alpha, gamma)
        torch.cuda.synchronize()
        out[name] = host(o)
        err = np.abs(out[name] - ref).max() / np.abs(ref).max()
        assert err < 1e-5, (name, err)
    d = np.abs(out["fused"] - out["separate"]).max() / np.abs(ref).max()
    assert 0.0 < d < 2e-6, d          # different rounding, same transform


def test_fused_lds_limit_selects_the_separate_passes(restore_fused):
    # a limit below the plane's 12.4 KB (70 x 40) gives the separate passes' bits
    P = (60, 40, 70)
    b = t(np.random.default_rng(8).normal(size=(3,) + P))
    res = {}
    for name, lds in (("separate", 0), ("limited", 4096)):
        L.lddmm_set_tunable(L.TUNE_FFT_FUSED_LDS, lds)
        res[name] = L.lddmm_smooth(b, 0.2, 0.02, 1.0)
        torch.cuda.synchronize()
    assert torch.equal(res["separate"], res["limited"])


@pytest.mark.parametrize("fused", [FUSED_DEFAULT, 0])
def test_fused_registration_matches_oracle(fused, restore_fused):
    say(f"register blobs32, fused lds {fused}")
    L.lddmm_set_tunable(L.TUNE_FFT_FUSED_LDS, fused)
    p = synth.config_pair("blobs32")
    prm = O.Params(T=5, iters=(8,), step=0.02, spacing=0.05, guard=True)
    ref = O.register(O.Problem(p.M0, p.M1), prm)
    lp = L.Params(T=5, iters=(8,), step=0.02, guard=True)
    res = L.lddmm_register(t(p.M0), t(p.M1), params=lp, spacing=0.05)
    torch.cuda.synchronize()
    tr = host(res["trace"])
    rt = np.array(ref.trace)
    np.testing.assert_array_equal(tr[:, 6], rt[:, 6])
    assert np.all(np.abs(tr[:, :3] - rt[:, :3]) <= 1e-5 * np.abs(rt[:, :3]))
    e10 = np.abs(host(res["phi10"]) - ref.phi10).max() / 0.05
    assert e10 < 1e-4, e10


def test_fused_batched_equals_single(restore_fused):
    # one problem per kind: fused (32 x 32 and 64 x 64 planes) and separate passes
    shapes = [(32, 32, 32), (20, 24, 28), (18, 64, 64)]
    pairs = []
    for k, shp in enumerate(shapes):
        p = synth.blob_pair(shp, 490 + k, max_disp=max(shp) / 10,
                            sigma=(max(shp) / 16, max(shp) / 6.4))
        pairs.append({"M0": t(p.M0), "M1": t(p.M1), "spacing": 0.05})
    prm = L.Params(T=4, n_levels=1, iters=(5,), step=0.05, guard=True)
    say("batched with fused and separate K")
    res, code = L.lddmm_register_batched(pairs, prm)
    torch.cuda.synchronize()
    for d, r in zip(pairs, res):
        single = L.lddmm_register(d["M0"], d["M1"], params=prm, spacing=d["spacing"])
        torch.cuda.synchronize()
        assert r["status"] == single["status"]
        for k in ("v", "phi10", "phi01"):
            assert torch.equal(r[k], single[k]), k
        assert torch.equal(r["trace"].nan_to_num(-1.0), single["trace"].nan_to_num(-1.0))
