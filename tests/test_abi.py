"""The C-ABI library loads and exports every symbol include/*.h declares
(CPU only: no compute calls without a GPU)."""

import ctypes
import os
import re

import pytest

from paper_1605_02060_amd import cnn
from paper_1605_02060_amd import lddmm as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(headers=("lddmm.h", "lddmm_cnn.h", "lddmm_masks.h")):
    names = set()
    for h in headers:
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(lddmm_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_every_header_is_checked():
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["lddmm.h", "lddmm_cnn.h",
                                                                 "lddmm_masks.h"]


def test_header_declares_the_boundary_calls():
    names = _declared()
    for n in ("lddmm_register", "lddmm_energy", "lddmm_gradient", "lddmm_apply"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTED + cnn.EXPORTED) == _declared()
    cnn._lib()                                    # every signature binds


def test_struct_layout_matches_header(tmp_path):
    # compile the header with the host C compiler and compare sizes / offsets
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "sz.c"
    src.write_text(
        "#include <stdio.h>\n#include <stddef.h>\n#include \"lddmm.h\"\n"
        "int main(){printf(\"%zu %zu %zu %zu %zu %zu\\n\", sizeof(lddmm_params),"
        " offsetof(lddmm_params, step), offsetof(lddmm_params, weight),"
        " offsetof(lddmm_params, checkpoint_every), sizeof(lddmm_problem),"
        " offsetof(lddmm_problem, workspace_bytes));"
        "printf(\"%zu %zu %zu\\n\", sizeof(lddmm_align_params), offsetof(lddmm_align_params, step),"
        " offsetof(lddmm_align_params, max_halvings));}\n")
    exe = tmp_path / "sz"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    want = [ctypes.sizeof(L._Params), L._Params.step.offset, L._Params.weight.offset,
            L._Params.checkpoint_every.offset, ctypes.sizeof(L._Problem),
            L._Problem.workspace_bytes.offset, ctypes.sizeof(L._AlignParams),
            L._AlignParams.step.offset, L._AlignParams.max_halvings.offset]
    assert got == want


def test_host_side_queries_without_gpu():
    p = L.Params(T=10, n_levels=3, iters=(200, 200, 200))
    assert L.lddmm_comp_grid((228, 160, 264), p, 0) == (240, 160, 280)
    assert L.lddmm_comp_grid((228, 160, 264), p, 2) == (60, 40, 70)
    assert L.lddmm_trace_rows(p) == 603
    assert L.lddmm_workspace_size((228, 160, 264), p) > 0
    bad = L.Params(T=0)
    assert L.lddmm_workspace_size((32, 32, 32), bad) == 0
    assert L.strerror(L.EINVAL) == "invalid argument"


def test_binding_rejects_wrongly_sized_buffers():
    # the C ABI takes bare pointers: the binding checks every shape before a call
    import torch
    N = (13, 17, 19)
    M = torch.zeros(N)
    prm = L.Params(T=3, iters=(1,))
    P = L.lddmm_comp_grid(N, prm, 0, 1.0)
    assert P != N
    with pytest.raises(ValueError, match="v:"):
        L.lddmm_register(M, M, params=prm, v=torch.zeros((3, 3) + N))
    with pytest.raises(ValueError, match="MI0"):
        L.lddmm_register(M, M, torch.zeros(N[::-1]), None, params=prm)
    with pytest.raises(ValueError, match="M1"):
        L.lddmm_register(M, torch.zeros(N, dtype=torch.float64), params=prm)
    with pytest.raises(ValueError, match="u:"):
        L.lddmm_apply(torch.zeros((3, 13, 17, 18)), M)


def test_profile_classes_match_header():
    src = open(os.path.join(ROOT, "include", "lddmm.h")).read()
    n = int(re.search(r"#define LDDMM_PROF_CLASSES\s+(\d+)", src).group(1))
    assert len(L.PROF_CLASSES) == n
    for k, name in enumerate(("FORWARD", "BACKWARD", "FFT_X", "FFT_Y", "FFT_ZK", "FFT_YINV",
                              "FFT_XINV", "OTHER", "HIST_RANGE", "HIST_COUNT", "HIST_APPLY",
                              "ALIGN", "FORWARD_EDGE", "BACKWARD_EDGE")):
        assert int(re.search(rf"#define LDDMM_PROF_{name}\s+(\d+)", src).group(1)) == k


def test_tunable_ids_match_header_and_values_are_checked():
    # process-wide launch shapes; setting them touches no GPU
    from paper_1605_02060_amd import tune
    src = open(os.path.join(ROOT, "include", "lddmm.h")).read()
    for name in ("SWEEP_BLOCKS", "FFT_X_ELEMS", "FFT_COLS", "FFT_ZCOLS", "STAGED_MIN_BLOCKS",
                 "FWD_TILES", "FWD_STAGED_MIN_BLOCKS", "FFT_FUSED_LDS", "K_TIME_BATCH"):
        val = int(re.search(rf"#define LDDMM_TUNE_{name}\s+(\d+)", src).group(1))
        assert getattr(L, f"TUNE_{name}") == val
    assert set(tune.DEFAULTS) == set(tune.CANDIDATES) == set(tune.NAMES)
    try:
        with pytest.raises(RuntimeError):
            L.lddmm_set_tunable(L.TUNE_FWD_TILES, -1)
        with pytest.raises(RuntimeError):
            L.lddmm_set_tunable(L.TUNE_SWEEP_BLOCKS, 0)
        with pytest.raises(RuntimeError):
            L.lddmm_set_tunable(99, 1)
        with pytest.raises(RuntimeError):
            L.lddmm_set_tunable(L.TUNE_FFT_FUSED_LDS, -1)
        L.lddmm_set_tunable(L.TUNE_FFT_FUSED_LDS, 0)       # 0: never fuse
        L.lddmm_set_tunable(L.TUNE_FFT_FUSED_LDS, 81920)
        for bad in (-1, 2):
            with pytest.raises(RuntimeError):
                L.lddmm_set_tunable(L.TUNE_K_TIME_BATCH, bad)
        L.lddmm_set_tunable(L.TUNE_K_TIME_BATCH, 0)        # K after each step
        L.lddmm_set_tunable(L.TUNE_K_TIME_BATCH, 1)
        L.lddmm_set_tunable(L.TUNE_FWD_TILES, 0)          # 0: the grid-stride forward sweep
        L.lddmm_set_tunable(L.TUNE_FWD_TILES, 1 << 20)    # clamped to the partial buffers
    finally:
        tune.set_all(tune.DEFAULTS)


def test_energy_and_gradient_take_v_on_the_single_level_grid():
    # the library evaluates energy and gradient on one level whatever n_levels
    # says, so the binding checks v against the single-level grid
    import torch
    N = (12, 12, 29)
    M = torch.zeros(N)
    prm = L.Params(T=2, n_levels=3, iters=(1, 1, 1))
    P2 = L.lddmm_comp_grid(N, prm, 0, 1.0)
    P1 = L.lddmm_comp_grid(N, L.Params(T=2), 0, 1.0)
    assert P1 != P2
    for call in (lambda v: L.lddmm_energy(M, M, None, None, v, prm),
                 lambda v: L.lddmm_gradient(M, M, None, None, v, prm)):
        with pytest.raises(ValueError, match="v:"):
            call(torch.zeros((2, 3) + P2))
        with pytest.raises(ValueError, match="device tensor"):   # shape accepted
            call(torch.zeros((2, 3) + P1))
