"""Write the expected energy terms and sampled V-gradient entries of one
velocity on the atlas-sized single-level grid, computed by the FP64 oracle.

Workload: the atlas-like pair (user grid 264 x 160 x 228, seed 1), computational
grid 270 x 160 x 240, T = 10, h = 0.05, alpha = 0.02, gamma = sigma = 1,
Mask-LDDMM weights (1, 0) with the masked-image channel monitored (Methods,
Registration and Preprocessing).  The velocity is v_j = (1 + j/20) w, with w the
plane-wave field of synth.plane_wave_velocity(grid, 77, 3 h) (at most 0.45 voxel
per time step).

Stored (tests/golden/atlas_264x160x228_gradient.npz):
  E, R, D, img_ssd, min_det  -- oracle scalars (float64);
  idx                        -- 100000 flat indices into g[T][3][nz][ny][nx],
                                drawn by numpy.random.default_rng(2024) without
                                replacement (uint32);
  g                          -- the oracle's g at those indices (float32);
  g_absmax                   -- max |g| over the whole field (float64).

Run: python tests/golden/make_atlas_gradient.py   (about 10 minutes, ~12 GB)
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lddmm as O  # noqa: E402
from paper_1605_02060_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "atlas_264x160x228_gradient.npz")
H, T, ALPHA, GAMMA, SIGMA = 0.05, 10, 0.02, 1.0, 1.0
GRID = (240, 160, 270)           # single-level computational grid [z][y][x]
N_SAMPLES = 100000


def velocity():
    """The velocity both sides evaluate (float32, as the GPU holds it)."""
    w = synth.plane_wave_velocity(GRID, 77, 3.0 * H)
    return np.stack([(1.0 + 0.05 * j) * w for j in range(T)]).astype(np.float32)


def sample_indices():
    n = T * 3 * int(np.prod(GRID))
    return np.random.default_rng(2024).choice(n, N_SAMPLES, replace=False).astype(np.uint32)


def main():
    t0 = time.time()
    p = synth.config_pair("atlas")
    prob = O.Problem(p.M0, p.M1, p.MI0, p.MI1)
    prm = O.Params(alpha=ALPHA, gamma=GAMMA, sigma=SIGMA, T=T, weight=(1.0, 0.0), spacing=H)
    v = velocity().astype(np.float64)
    assert v.shape[2:] == GRID
    g, st, md = O.gradient(prob, prm, v, kind="V")
    idx = sample_indices()
    np.savez(OUT, E=st["E"], R=st["R"], D=st["D"], img_ssd=st["img_ssd"], min_det=md, idx=idx,
             g=g.reshape(-1)[idx].astype(np.float32), g_absmax=np.abs(g).max())
    print(f"wrote {OUT}: E {st['E']:.9g} R {st['R']:.9g} D {st['D']:.9g} "
          f"img {st['img_ssd']:.9g} min det {md:.6g}, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
