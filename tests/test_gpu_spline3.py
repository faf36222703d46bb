"""GPU parity of the push + deposit with the third-order (cubic B-spline)
shape (grpic_push_deposit_spline3 through the C ABI, untiled and tiled)
against the oracle run with order=3, element by element at the FP64 bar and norms of
tests/parity.py; the cubic charge (grpic_charge3) against the oracle's; and
per-vertex continuity on the GPU's own outputs, including moves whose
windows fold across the axes."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2503_04558_amd import grpic
from paper_2503_04558_amd import workload as wl

from parity import assert_parity, gpu_run

pytestmark = pytest.mark.gpu

TOL = 1e-12
EPS = np.finfo(np.float64).eps
TILED = [pytest.param(False, id="untiled"), pytest.param(True, id="tiled")]


def _announce(msg):
    print(f"[gpu] {msg}", flush=True)


def _axis_parts(g, n, seed):
    """Particles within two cells of an axis, driven into it; an eighth at
    each radial edge."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, g.nr, n)
    j = rng.choice([0, 1, g.nth - 2, g.nth - 1], n)
    i[: n // 8] = 0
    i[n // 8: n // 4] = g.nr - 1
    r, th = g.r(i + 0.5), g.theta(j + 0.5)
    uh = rng.normal(size=(3, n)) * 2.0
    uh[1] = np.where(j < 2, -np.abs(uh[1]), np.abs(uh[1]))
    ur, uth, uph = wl.frame_to_covariant(g.a, g.M, r, th, uh)
    return dict(cell=(i * g.nth + j).astype(np.int32), xr=rng.uniform(0, 1, n), xth=rng.uniform(0, 1, n),
                ur=ur, uth=uth, uph=uph, w=rng.uniform(0.5, 2.0, n), sp=rng.integers(0, 2, n).astype(np.uint8))


@pytest.mark.parametrize("tiled", TILED)
def test_spline3_parity_wald_config(tiled):
    """128^2, a = 0.99, guard 3, 2e4 e+- (|u| uniform in [0, 1]), Wald B0 = 1
    (columns beyond the axes from the analytic field), 10 steps; untiled,
    and through the GPU sort and the tiled kernel's LDS window."""
    _announce(f"spline3 parity 128x128 2e4 particles 10 steps tiled={tiled}")
    g = wl.make_grid(128, 128, 0.99, guard=3)
    parts = wl.pairs(g, 10_000, kind="uniform", seed=0)
    e, c = assert_parity(g, wl.species_table(), parts, wl.wald_fields(g), wl.crossing_dt(g), 10, TOL, order=3,
                         tiled=tiled)
    _announce(f"errors {e} counters {c}")
    assert c["out"] > 0 and c["reflected"] > 0


@pytest.mark.parametrize("tiled", TILED)
def test_spline3_parity_axis_and_edges(tiled):
    """Every particle within two cells of an axis (its 5 x 5 window folds)
    or at a radial edge, driven into it; 6 steps."""
    _announce(f"spline3 parity axis/edges tiled={tiled}")
    g = wl.make_grid(24, 24, 0.99, guard=3)
    parts = _axis_parts(g, 4000, 5)
    e, c = assert_parity(g, wl.species_table(), parts, wl.wald_fields(g, B0=2.0), wl.crossing_dt(g), 6, TOL,
                         max_ill_fraction=1e-2, order=3, tiled=tiled)
    assert c["reflected"] > 20 and c["out"] > 100


@pytest.mark.parametrize("tiled", TILED)
@pytest.mark.parametrize("n", [1, 65, 1001])
def test_spline3_parity_ragged(n, tiled):
    _announce(f"spline3 parity ragged n={n} tiled={tiled}")
    g = wl.make_grid(40, 100, 0.9, guard=3)
    parts = wl.pairs(g, (n + 1) // 2, kind="mj", seed=n, params=dict(T=0.5))
    parts = {k: v[:n] for k, v in parts.items()}
    assert_parity(g, wl.species_table(), parts, wl.wald_fields(g, B0=3.0), wl.crossing_dt(g), 5, TOL, order=3,
                  tiled=tiled)


def test_spline3_charge_and_continuity_on_gpu():
    """grpic_charge3 equals the oracle's cubic charge; over 5 GPU steps the
    per-vertex continuity residual of the GPU's own outputs stays at
    round-off, axis vertices included."""
    _announce("spline3 charge and continuity")
    g = wl.make_grid(48, 40, 0.99, guard=3)
    sp = wl.species_table()
    host = _axis_parts(g, 3000, 9)
    more = wl.pairs(g, 3000, kind="mj", seed=10, params=dict(T=1.0))
    host = {k: np.concatenate([host[k], more[k]]) for k in host}
    parts = grpic.to_device(host)
    Q0 = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    A0 = torch.zeros_like(Q0)
    grpic.grpic_charge(g, sp, parts, Q0, order=3)
    grpic.grpic_charge(g, [dict(s, q=1.0) for s in sp], parts, A0, order=3)
    torch.cuda.synchronize()
    want = orc.charge3(g, sp, host)
    scale = np.abs(want).max()
    assert np.abs(Q0.cpu().numpy() - want).max() <= 1e-13 * scale
    F = [torch.as_tensor(f).cuda() for f in wl.wald_fields(g, B0=2.0)]
    J = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    dt = wl.crossing_dt(g)
    nsteps = 5
    grpic.grpic_push_deposit(grpic.make_metric(g.a, g.M), g, sp, parts, F, J, dt, nsteps, order=3)
    Q1 = torch.zeros_like(Q0)
    A1 = torch.zeros_like(Q0)
    grpic.grpic_charge(g, sp, parts, Q1, order=3)
    grpic.grpic_charge(g, [dict(s, q=1.0) for s in sp], parts, A1, order=3)
    torch.cuda.synchronize()
    div = torch.zeros_like(J[0])
    div[1:, :] += J[0][1:, :] - J[0][:-1, :]
    div[:, 1:] += J[1][:, 1:] - J[1][:, :-1]
    G = g.guard
    inner = slice(G + 2, G + g.nr - 2)          # away from the rows that receive the outflow's last moves
    R = (Q1 - Q0 + dt * div)[inner]
    bound = (64 * EPS * (1 + nsteps) * (A0 + A1))[inner]
    ratio = (R.abs() / bound.clamp_min(1e-300)).max().item()
    _announce(f"continuity: max |R| / bound = {ratio:.3e}")
    assert ratio <= 1.0
    for arr in (*J, Q1):                           # nothing beyond the axes
        a = arr.cpu().numpy()
        assert not a[:, :G].any() and not a[:, G + g.nth + 1:].any()


def test_spline3_argument_checks():
    g2 = wl.make_grid(16, 16, 0.5)                 # guard 2: too narrow for the cubic window
    parts = grpic.to_device(wl.pairs(g2, 4, seed=1))
    F = [torch.zeros(g2.shape, dtype=torch.float64, device="cuda") for _ in range(6)]
    J = [torch.zeros(g2.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    with pytest.raises(grpic.GrpicError, match="guard"):
        grpic.grpic_push_deposit(grpic.make_metric(0.5), g2, wl.species_table(), parts, F, J,
                                 wl.crossing_dt(g2), 1, order=3)
    with pytest.raises(ValueError, match="order=3"):
        grpic.grpic_push_deposit(grpic.make_metric(0.5), g2, wl.species_table(), parts, F, J,
                                 wl.crossing_dt(g2), 1, order=3, kick="vay")


def test_spline3_tiled_equals_untiled_with_drift_beyond_window():
    """One sort, then 40 steps with the cubic shape: fast particles and those
    near the horizon leave their tile's LDS window (whose cubic bounds check
    works on the axis-folded columns) and deposit to global memory, and a
    share of the particles start within two cells of an axis, so their
    folded windows sit at the window's column edges.  On identical sorted
    inputs the tiled push must reproduce the untiled one bit for bit for
    every particle, and its current up to summation order; some deposits
    must have gone the global way."""
    _announce("spline3 tiled vs untiled with drift")
    g = wl.make_grid(64, 128, 0.99, guard=3)
    bulk = wl.pairs(g, 30_000, kind="uniform", seed=12, params=dict(umax=3.0))
    axis = _axis_parts(g, 20_000, seed=13)
    host = {k: np.concatenate([bulk[k], axis[k].astype(bulk[k].dtype)]) for k in bulk}
    n = len(host["cell"])
    sorter = grpic.Sorter(g, n)
    base = sorter.sort(grpic.to_device(host))
    copies = [{k: v.clone() for k, v in base.items()} for _ in range(2)]
    F = [torch.as_tensor(f).cuda() for f in wl.wald_fields(g, B0=2.0)]
    Js = [[torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)] for _ in range(2)]
    cnts = [torch.zeros(grpic.GRPIC_NCOUNTERS, dtype=torch.int64, device="cuda") for _ in range(2)]
    m = grpic.make_metric(g.a, g.M)
    dt = wl.crossing_dt(g)
    for step in range(40):
        grpic.grpic_push_deposit(m, g, wl.species_table(), copies[0], F, Js[0], dt, 1, counters=cnts[0], order=3)
        grpic.grpic_push_deposit(m, g, wl.species_table(), copies[1], F, Js[1], dt, 1, tiling=sorter.tiling,
                                 counters=cnts[1], order=3)
    torch.cuda.synchronize()
    for k in copies[0]:
        assert torch.equal(copies[0][k], copies[1][k]), k
    for a, b in zip(*Js):
        assert (a - b).abs().max().item() <= 1e-13 * a.abs().max().item()
    c0 = dict(zip(grpic.COUNTER_NAMES, cnts[0].tolist()))
    c1 = dict(zip(grpic.COUNTER_NAMES, cnts[1].tolist()))
    _announce(f"untiled {c0} tiled {c1}")
    assert {k: c0[k] for k in ("out", "bad", "reflected", "live_steps")} == \
           {k: c1[k] for k in ("out", "bad", "reflected", "live_steps")}
    assert c1["spilled"] > 1000 and c0["spilled"] == 0 and c1["reflected"] > 100
