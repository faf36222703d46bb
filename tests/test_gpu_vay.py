"""GPU parity of the push + deposit with Vay's kick in the FIDO frame
(grpic_push_deposit_vay through the C ABI) against the oracle run with the
same kick, element by element, at the FP64 bar and norms of tests/parity.py;
plus its argument checks and the force-free drift on the GPU."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2503_04558_amd import grpic
from paper_2503_04558_amd import workload as wl

from parity import assert_parity, gpu_run

pytestmark = pytest.mark.gpu

TOL = 1e-12
TILED = [pytest.param(False, id="untiled"), pytest.param(True, id="tiled")]


def _announce(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.mark.parametrize("tiled", TILED)
def test_vay_parity_small_wald_config(tiled):
    """256^2, a = 0.99, 1e5 e+- pairs, |u| uniform in [0, 1], Wald B0 = 1,
    10 steps (the small parity configuration) with the Vay kick."""
    _announce(f"vay parity 256x256 2e5 particles 10 steps tiled={tiled}")
    g = wl.make_grid(256, 256, 0.99)
    parts = wl.pairs(g, 100_000, kind="uniform", seed=0)
    e, c = assert_parity(g, wl.species_table(), parts, wl.wald_fields(g), wl.crossing_dt(g), 10, TOL, tiled=tiled,
                         kick="vay")
    _announce(f"errors {e} counters {c}")
    assert c["out"] > 0 and c["reflected"] > 0


@pytest.mark.parametrize("tiled", TILED)
def test_vay_parity_strong_field_ragged(tiled):
    """Strong field (Wald B0 = 30, so h |B| ~ 1 per kick), relativistic
    Maxwell-Juttner (T = 5), ragged count on a 40 x 100 grid, 5 steps."""
    _announce(f"vay parity strong field tiled={tiled}")
    g = wl.make_grid(40, 100, 0.9)
    parts = wl.pairs(g, 501, kind="mj", seed=3, params=dict(T=5.0))
    parts = {k: v[:1001] for k, v in parts.items()}
    assert_parity(g, wl.species_table(), parts, wl.wald_fields(g, B0=30.0), wl.crossing_dt(g), 5, TOL, tiled=tiled,
                  kick="vay")


@pytest.mark.parametrize("tiled", TILED)
def test_vay_parity_fine_grid_short_series(tiled):
    """1600 x 1280 (the kernels' short Taylor series), 6e4 particles of the
    throughput workload's recipe, 6 steps, Vay kick."""
    _announce(f"vay parity fine grid tiled={tiled}")
    g = wl.make_grid(1600, 1280, 0.99)
    parts = wl.pairs(g, 30_000, kind="mj", seed=11, params=dict(T=0.1, vphi=0.1))
    assert_parity(g, wl.species_table(), parts, wl.wald_fields(g), wl.crossing_dt(g), 6, TOL, tiled=tiled,
                  kick="vay")


def test_vay_force_free_drift_on_gpu():
    """Uniform field arrays (the CIC gather returns the constants up to
    rounding) with D = -v x B for one particle's velocity at its position in
    the Kerr metric: E + v x B = 0 there, so with the Vay kick the step is
    the zero-field (geodesic) step to round-off, while the Boris kick moves
    the momentum.  Independent of the oracle: the fields come from the
    metric and a cross product written here."""
    _announce("vay force-free drift on the GPU")
    g = wl.make_grid(64, 64, 0.9)
    i0, j0, fx, fy = 30, 20, 0.3, 0.6
    xi, eta = i0 + fx, j0 + fy
    r, th = g.r(xi), g.theta(eta)
    m = orc.metric(g.a, g.M, r, th)

    def raise_(v):
        return np.array([m["h_rr"] * v[0] + m["h_rph"] * v[2], m["h_thth"] * v[1],
                         m["h_rph"] * v[0] + m["h_phph"] * v[2]])

    u = np.array([0.8, 0.5 * r, 1.2 * r])
    uu = raise_(u) @ u
    v = raise_(u) / math.sqrt(1.0 + uu)
    B = np.array([30.0, 20.0 / r, 10.0])          # strong: the Boris error grows with (q B dt / m)^2
    vxB = m["sqrtg"] * np.array([v[1] * B[2] - v[2] * B[1], v[2] * B[0] - v[0] * B[2], v[0] * B[1] - v[1] * B[0]])
    D = -raise_(vxB)
    X = [np.full(g.shape, c) for c in (*D, *B)]
    parts = dict(cell=np.array([i0 * g.nth + j0], dtype=np.int32), xr=np.array([fx]), xth=np.array([fy]),
                 ur=np.array([u[0]]), uth=np.array([u[1]]), uph=np.array([u[2]]), w=np.array([1.0]),
                 sp=np.array([1], dtype=np.uint8))
    sp = wl.species_table()
    dt = wl.crossing_dt(g)
    zero, _, _ = gpu_run(g, sp, parts, [np.zeros(g.shape)] * 6, dt, 1)
    vay, _, _ = gpu_run(g, sp, parts, X, dt, 1, kick="vay")
    boris, _, _ = gpu_run(g, sp, parts, X, dt, 1, kick="boris")
    assert vay["cell"][0] == zero["cell"][0] >= 0
    for k in ("xr", "xth"):
        assert abs(vay[k][0] - zero[k][0]) <= 1e-13, k
    scale = math.sqrt(1.0 + uu)
    for k in ("ur", "uth", "uph"):
        assert abs(vay[k][0] - zero[k][0]) <= 1e-13 * scale * (r if k != "ur" else 1.0), k
    moved = max(abs(boris[k][0] - zero[k][0]) for k in ("ur", "uth", "uph"))
    assert moved > 1e-8 * scale, moved


def test_vay_rejects_split_particles():
    g = wl.make_grid(16, 16, 0.5)
    parts = grpic.to_device(wl.pairs(g, 4, seed=1), grpic.GRPIC_FP32_SPLIT)
    F = [torch.zeros(g.shape, dtype=torch.float32, device="cuda") for _ in range(6)]
    J = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    with pytest.raises(grpic.GrpicError, match="FP64"):
        grpic.grpic_push_deposit(grpic.make_metric(0.5), g, wl.species_table(), parts, F, J,
                                 wl.crossing_dt(g), 1, kick="vay")
