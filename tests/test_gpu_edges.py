"""GPU parity on the configurations and edge cases that the other parity tests
do not reach:

* the 32^3 workload exactly as configured (T = 10, 50 iterations);
* sigma != 1 in the energy, both gradients and a registration;
* the LDS-staged backward sweep with map gathers that leave its staged window
  (|dt v / h| between 2 and 3 voxels per step), first order and RK4;
* the exact gradient's splat radius just inside and just beyond its limit;
* the fold and guard-stop statuses of a registration, and a registration
  resumed from its returned velocity against the straight run;
* the batched workload's 16 uneven pairs: batched equals single calls, and the
  smallest pair against the oracle.
Everything is compared with the FP64 oracle on the same seeded inputs, or
bitwise between two launch choices that must not change a result."""

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


def t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(x):
    return x.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _lp(prm: O.Params, **kw):
    flags = kw.pop("flags", L.FLAG_RK4 if prm.integrator == "rk4" else 0)
    return L.Params(alpha=prm.alpha, gamma=prm.gamma, sigma=prm.sigma, T=prm.T,
                    n_levels=prm.n_levels, iters=prm.iters, step=prm.step, guard=prm.guard,
                    weight=prm.weight, flags=flags, **kw)


def _compare_trace_and_maps(res, ref, h, tol_phi=1e-4, tol_E=1e-5):
    tr = host(res["trace"])
    rt = np.array(ref.trace)
    assert tr.shape == rt.shape
    np.testing.assert_array_equal(tr[:, 6], rt[:, 6])        # same accept / reject decisions
    fin = np.isfinite(rt[:, 0])
    np.testing.assert_array_equal(np.isfinite(tr[:, 0]), fin)
    assert np.all(np.abs(tr[fin, :3] - rt[fin, :3]) <= tol_E * np.abs(rt[fin, :3]) + 1e-300)
    assert np.all(np.abs(tr[:, 7] - rt[:, 7]) <= tol_E * np.abs(rt[:, 7]))
    e10 = np.abs(host(res["phi10"]) - ref.phi10).max() / h
    e01 = np.abs(host(res["phi01"]) - ref.phi01).max() / h
    assert e10 < tol_phi and e01 < tol_phi, (e10, e01)
    assert res["status"] == ref.status, (res["status"], ref.status)


# ------------------------------------------------ the 32^3 workload ----

@pytest.mark.parametrize("h,step", [(0.05, 0.02), (1.0, 0.2)])
def test_blobs32_as_configured(h, step):
    """32^3, T = 10, 50 iterations, alpha = 0.02, gamma = sigma = 1, guard on:
    every iteration's E, R, D and accept decision, and both maps."""
    say(f"blobs32 T=10 50 iterations h={h} step={step}")
    p = synth.config_pair("blobs32")
    prm = O.Params(T=10, iters=(50,), step=step, spacing=h)
    ref = O.register(O.Problem(p.M0, p.M1, p.MI0, p.MI1), prm)
    res = L.lddmm_register(t(p.M0), t(p.M1), t(p.MI0), t(p.MI1), params=_lp(prm), spacing=h)
    torch.cuda.synchronize()
    _compare_trace_and_maps(res, ref, h)


# --------------------------------------------------------- sigma != 1 ----

def _blob_case(shape, seed, T, h, vmax, weight=(1.0, 0.5), sigma=0.5):
    p = synth.blob_pair(shape, seed, max_disp=max(shape) / 10,
                        sigma=(max(shape) / 14, max(shape) / 6))
    P = tuple(O.smooth7(n) for n in shape)
    v = (h * synth.random_velocity(P, T, 500 + seed, vmax=vmax, sigma_s=3.0)).astype(np.float32)
    prm = O.Params(T=T, spacing=h, sigma=sigma, weight=weight)
    return p, P, v, prm


def test_sigma_half_energy_and_gradients():
    say("sigma 0.5: energy, V-gradient, exact gradient")
    p, P, v, prm = _blob_case((20, 22, 24), 31, 4, 0.1, 1.5)
    prob = O.Problem(p.M0, p.M1, p.MI0, p.MI1)
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1))
    ref = O.energy(prob, prm, v.astype(np.float64))
    out = host(L.lddmm_energy(*args, t(v), _lp(prm), spacing=0.1))
    for k, name in enumerate(("E", "R", "D", "img_ssd")):
        assert rel(out[k], ref[name]) < 1e-5, name
    gV, st, _ = O.gradient(prob, prm, v.astype(np.float64), kind="V")
    g, _ = L.lddmm_gradient(*args, t(v), _lp(prm), kind=L.GRAD_V, spacing=0.1)
    assert np.abs(host(g) - gV).max() < 2e-5 * np.abs(gV).max()
    gL, _, _ = O.gradient(prob, prm, v.astype(np.float64), kind="L2")
    g, e = L.lddmm_gradient(*args, t(v), _lp(prm), kind=L.GRAD_L2, spacing=0.1)
    assert np.abs(host(g) - gL).max() < 1e-4 * np.abs(gL).max()
    assert rel(host(e)[0], st["E"]) < 1e-5


def test_sigma_half_register():
    say("sigma 0.5: registration")
    p = synth.config_pair("blobs32")
    prm = O.Params(T=10, iters=(10,), step=0.005, spacing=0.05, sigma=0.5, weight=(1.0, 0.5))
    ref = O.register(O.Problem(p.M0, p.M1, p.MI0, p.MI1), prm)
    res = L.lddmm_register(t(p.M0), t(p.M1), t(p.MI0), t(p.MI1), params=_lp(prm), spacing=0.05)
    torch.cuda.synchronize()
    _compare_trace_and_maps(res, ref, 0.05)


# ------------------------------------ staged backward beyond its window ----

@pytest.mark.parametrize("integrator", ["euler", "rk4"])
def test_staged_backward_with_gathers_outside_the_window(integrator):
    """max |dt v / h| of 2.5 voxels: most map gathers of the staged kernel leave
    its LDS window (halo 1) and read global memory."""
    say(f"staged backward, 2.5 voxels per step, {integrator}")
    shape, T, h = (40, 36, 48), 4, 0.1
    p = synth.blob_pair(shape, 33, max_disp=4.0, sigma=(3.0, 7.0))
    P = tuple(O.smooth7(n) for n in shape)
    v = (h * synth.random_velocity(P, T, 533, vmax=10.0, sigma_s=4.0)).astype(np.float32)
    assert 2.0 < np.abs(v).max() / h / T <= 2.5
    prm = O.Params(T=T, spacing=h, weight=(1.0, 0.5), integrator=integrator)
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1), t(v))
    out = {}
    try:
        for name, thr in (("staged", 1), ("grid", 1 << 30)):
            L.lddmm_set_tunable(L.TUNE_STAGED_MIN_BLOCKS, thr)
            g, e = L.lddmm_gradient(*args, _lp(prm), kind=L.GRAD_V, spacing=h)
            torch.cuda.synchronize()
            out[name] = (g.cpu().numpy(), e.cpu().numpy())
    finally:
        L.lddmm_set_tunable(L.TUNE_STAGED_MIN_BLOCKS, 2048)
    np.testing.assert_array_equal(out["staged"][0], out["grid"][0])
    np.testing.assert_array_equal(out["staged"][1], out["grid"][1])
    g_ref, st, _ = O.gradient(O.Problem(p.M0, p.M1, p.MI0, p.MI1), prm, v.astype(np.float64),
                              kind="V")
    err = np.abs(out["staged"][0] - g_ref).max() / np.abs(g_ref).max()
    assert err < 2e-5, err
    assert rel(float(out["staged"][1][0]), st["E"]) < 1e-5


@pytest.mark.parametrize("integrator", ["euler", "rk4"])
def test_staged_backward_registration_far_gathers(integrator):
    """A registration that starts from the 2.5-voxel field, with the staged kernel
    forced: the maps and the min-det column against the oracle."""
    say(f"staged registration from a 2.5-voxel field, {integrator}")
    shape, T, h = (30, 28, 34), 4, 0.1
    p = synth.blob_pair(shape, 34, max_disp=3.0, sigma=(2.5, 5.0))
    P = tuple(O.smooth7(n) for n in shape)
    v = (h * synth.random_velocity(P, T, 534, vmax=10.0, sigma_s=4.0)).astype(np.float32)
    prm = O.Params(T=T, iters=(4,), step=0.01, spacing=h, guard=False, integrator=integrator)
    ref = O.register(O.Problem(p.M0, p.M1), prm, v_init=v.astype(np.float64))
    L.lddmm_set_tunable(L.TUNE_STAGED_MIN_BLOCKS, 1)
    try:
        res = L.lddmm_register(t(p.M0), t(p.M1), params=_lp(prm), spacing=h, v=t(v))
        torch.cuda.synchronize()
    finally:
        L.lddmm_set_tunable(L.TUNE_STAGED_MIN_BLOCKS, 2048)
    _compare_trace_and_maps(res, ref, h)
    tr, rt = host(res["trace"]), np.array(ref.trace)
    np.testing.assert_allclose(tr[1:, 4], rt[1:, 4], rtol=1e-4)   # min det of each gradient


# ----------------------------------------- exact gradient splat radius ----

@pytest.mark.parametrize("dmax,ok", [(2.9, True), (3.1, False)])
def test_exact_gradient_splat_radius_limit(dmax, ok):
    """The reverse sweep gathers its splat over offsets up to 3 voxels, which
    covers |dt v / h| < 3; beyond that the energy is reported as NaN."""
    say(f"exact gradient at max |dt v/h| = {dmax}")
    shape, T, h = (20, 22, 24), 4, 1.0
    p = synth.blob_pair(shape, 35, max_disp=2.0, sigma=(2.0, 4.0))
    P = tuple(O.smooth7(n) for n in shape)
    v = synth.random_velocity(P, T, 535, vmax=1.0, sigma_s=3.0).astype(np.float64)
    v *= dmax * T * h / np.abs(v).max()
    v = v.astype(np.float32)
    assert abs(np.abs(v).max() / (T * h) - dmax) < 1e-5
    prm = O.Params(T=T, spacing=h)
    g, e = L.lddmm_gradient(t(p.M0), t(p.M1), None, None, t(v), _lp(prm), kind=L.GRAD_L2,
                            spacing=h)
    e = host(e)
    if not ok:
        assert np.isnan(e[0])
        assert np.isfinite(e[1]) and np.isfinite(e[2])
        return
    g_ref, st, _ = O.gradient(O.Problem(p.M0, p.M1), prm, v.astype(np.float64), kind="L2")
    assert np.abs(host(g) - g_ref).max() < 1e-4 * np.abs(g_ref).max()
    assert rel(e[0], st["E"]) < 1e-5


# ------------------------------------------------------------- statuses ----

def _fold_case():
    shape, T, h = (24, 24, 24), 4, 1.0
    p = synth.blob_pair(shape, 36, max_disp=2.0, sigma=(2.0, 4.0))
    P = tuple(O.smooth7(n) for n in shape)
    rng = np.random.default_rng(536)
    v_fold = (2.5 * rng.standard_normal((T, 3) + P)).astype(np.float32)
    v_smooth = synth.random_velocity(P, T, 537, vmax=1.0, sigma_s=4.0)
    return p, T, h, v_fold, v_smooth


@pytest.mark.parametrize("which,iters", [("fold", 0), ("smooth", 0), ("fold", 3)])
def test_fold_status_of_the_returned_velocity(which, iters):
    """LDDMM_WFOLD iff the returned v's maps phi_{t_j,1} have det <= 0 somewhere."""
    say(f"fold status: {which} field, {iters} iterations")
    p, T, h, v_fold, v_smooth = _fold_case()
    v = v_fold if which == "fold" else v_smooth
    prm = O.Params(T=T, iters=(iters,), step=1e-6, spacing=h, guard=False)
    ref = O.register(O.Problem(p.M0, p.M1), prm, v_init=v.astype(np.float64))
    u1 = O.backward_maps(ref.v, h)
    min_det = min(O.jacobian_det(u1[j], h).min() for j in range(T))
    assert (min_det <= 0) == (which == "fold")
    assert ref.status == (O.STATUS_WFOLD if which == "fold" else O.STATUS_OK)
    res = L.lddmm_register(t(p.M0), t(p.M1), params=_lp(prm), spacing=h, v=t(v))
    torch.cuda.synchronize()
    assert res["status"] == (L.WFOLD if which == "fold" else L.OK)
    _compare_trace_and_maps(res, ref, h)


def test_guard_stop_status():
    """A step so large that every trial raises the energy: ten halvings, then
    the level stops (LDDMM_WGUARD) and the remaining slots record nothing."""
    say("forced guard stop")
    p = synth.config_pair("blobs32")
    prm = O.Params(T=4, iters=(14,), step=1e4, spacing=0.05)
    ref = O.register(O.Problem(p.M0, p.M1), prm)
    assert ref.status == O.STATUS_WGUARD
    res = L.lddmm_register(t(p.M0), t(p.M1), params=_lp(prm), spacing=0.05)
    torch.cuda.synchronize()
    assert res["status"] == L.WGUARD
    tr = host(res["trace"])
    assert np.all(tr[1:11, 6] == 0) and np.all(np.isnan(tr[11:, 0]))
    _compare_trace_and_maps(res, ref, 0.05)


def test_resume_from_the_returned_velocity_equals_the_straight_run():
    """Four iterations, then four more from the returned v (v_init), against
    eight in one call: with every trial accepted the step size never changes, so
    the resumed call retraces the straight one bit for bit.  The oracle checks
    the same on its side."""
    say("resume: 4 + 4 iterations against 8")
    p = synth.config_pair("blobs32")
    args = (t(p.M0), t(p.M1), t(p.MI0), t(p.MI1))
    prm4 = L.Params(T=3, iters=(4,), step=0.02, guard=True)
    prm8 = L.Params(T=3, iters=(8,), step=0.02, guard=True)
    a = L.lddmm_register(*args, params=prm4, spacing=0.05)
    b = L.lddmm_register(*args, params=prm4, spacing=0.05, v=a["v"].clone())
    c = L.lddmm_register(*args, params=prm8, spacing=0.05)
    torch.cuda.synchronize()
    tc = host(c["trace"])
    assert np.all(tc[1:, 6] == 1)                     # every trial accepted
    for k in ("v", "phi10", "phi01"):
        assert torch.equal(b[k], c[k]), k
    # the resumed trace is the second half of the straight one; its row 0 (the
    # evaluation at v_init) has the energies of the straight run's row 4
    tb = host(b["trace"])
    np.testing.assert_array_equal(tb[1:], tc[5:])
    np.testing.assert_array_equal(tb[0, [0, 1, 2, 5]], tc[4, [0, 1, 2, 5]])
    assert b["status"] == c["status"] == L.OK


# ------------------------------------------- the 16-pair batched workload ----

def _c4_pairs():
    dims = synth.batched_dims()
    out = []
    for k in range(len(dims)):
        p = synth.batched_pair(k, dims)
        out.append((p, {"M0": t(p.M0), "M1": t(p.M1), "spacing": 0.05}))
    return out


def test_batched_sixteen_pairs_equal_single_calls():
    say("16 batched pairs, 10 iterations: batched == single")
    pairs = _c4_pairs()
    prm = L.Params(T=10, iters=(10,), step=0.02, guard=True)
    res, code = L.lddmm_register_batched([d for _, d in pairs], prm)
    torch.cuda.synchronize()
    for k, ((p, d), r) in enumerate(zip(pairs, res)):
        single = L.lddmm_register(d["M0"], d["M1"], params=prm, spacing=0.05)
        torch.cuda.synchronize()
        say(f"pair {k} {tuple(d['M0'].shape)} status {r['status']}")
        assert r["status"] == single["status"]
        assert torch.equal(r["v"], single["v"]), k
        assert torch.equal(r["phi10"], single["phi10"]), k
        assert torch.equal(r["phi01"], single["phi01"]), k
        assert torch.equal(r["trace"].nan_to_num(-1.0), single["trace"].nan_to_num(-1.0)), k
        del single


@pytest.mark.timeout(600)
def test_batched_smallest_pair_matches_oracle():
    say("smallest batched pair against the oracle, 3 iterations")
    dims = synth.batched_dims()
    k = int(np.argmin(np.prod(dims, axis=1)))
    p = synth.batched_pair(k, dims)
    big = synth.batched_pair(int(np.argmax(np.prod(dims, axis=1))), dims)
    pairs = [{"M0": t(p.M0), "M1": t(p.M1), "spacing": 0.05},
             {"M0": t(big.M0), "M1": t(big.M1), "spacing": 0.05}]
    prm = L.Params(T=10, iters=(3,), step=0.02, guard=True)
    res, code = L.lddmm_register_batched(pairs, prm)
    torch.cuda.synchronize()
    oprm = O.Params(T=10, iters=(3,), step=0.02, spacing=0.05)
    ref = O.register(O.Problem(p.M0, p.M1), oprm)
    _compare_trace_and_maps(res[0], ref, 0.05)
