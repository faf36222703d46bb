"""Pins of the oracle's differentiated form (forward-mode dual numbers through
the whole K-step trajectory), used to check the GPU adjoint.

Loss (the adjoint workload, adjoint_cases.py): L = sum over steps n < K and
particles of lambda . (F^r, F^th, G^ph), lambda_r = dt on the r-faces nearest
to r = 5 (the net charge through that shell), zero elsewhere.

* The loss equals lambda contracted with the currents the plain oracle run
  accumulates over the same steps.
* d L / d u_i(0) per particle and d L / d(fields) along random directions agree
  with central finite differences (h = 1e-6); points where +-h crosses a CIC
  kink (one-sided differences disagree) are skipped and counted.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2503_04558_amd import workload as wl

from adjoint_cases import K, shell_case, shell_face


@pytest.fixture(scope="module")
def setup():
    return shell_case()


def test_shell_face_index():
    g = wl.make_grid(512, 512, 0.9)
    i = shell_face(g)
    assert i == 189 and abs(g.r(i + 0.5) - 5.0) < 0.02


def test_loss_equals_lambda_dot_accumulated_current(setup):
    g, dt, fields, parts, lam = setup
    L, _, st = orc.loss_dual(g, wl.species_table(), parts, fields, lam, dt, K)
    _, J, _, _ = orc.run(g, wl.species_table(), parts, fields, dt, K)
    L2 = sum(float((l * j).sum()) for l, j in zip(lam, J))
    assert abs(L) > 1e-3                        # charge really crosses the shell
    assert L == pytest.approx(L2, rel=1e-12, abs=1e-14)


def _signature(traj):
    """Half-cell floors along a trajectory: gathers use xi and xi - 1/2, the
    shape functions kink at integer coordinates, so equal signatures mean no
    kink lies between two runs."""
    t = traj[np.isfinite(traj[:, 0])]
    return np.floor(2.0 * t).astype(np.int64).tobytes()


def test_momentum_gradient_matches_finite_differences(setup):
    """Dual-number dL/du_i(0) against the 5-point stencil with h = 1e-4 and the
    central difference with h = 1e-6, where no kink lies within +-2h.  L is a
    sum of O(1) deposit terms that cancel to ~1e-2, so its round-off is ~1e-14
    absolute: the h = 1e-6 difference carries ~1e-8 of noise (1e-4 relative
    bar), the 5-point stencil at 1e-4 is good to ~1e-8 relative (1e-6 bar)."""
    g, dt, fields, parts, lam = setup
    sp = wl.species_table()
    checked = skipped = 0
    for p in range(0, len(parts["cell"]), 10):
        xi = parts["cell"][p] // g.nth + parts["xr"][p]
        eta = parts["cell"][p] % g.nth + parts["xth"][p]
        u = np.array([parts["ur"][p], parts["uth"][p], parts["uph"][p]])
        one = {k: v[p:p + 1] for k, v in parts.items()}
        row = sp[int(parts["sp"][p])]
        for k in range(3):
            t = [np.zeros(1), np.zeros(1), np.zeros(1)]
            t[k][0] = 1.0
            L0, dL, _ = orc.loss_dual(g, sp, one, fields, lam, dt, K, tu=t)

            def run(delta):
                v = u.copy()
                v[k] += delta
                return orc.loss_particle(g, row, xi, eta, v, parts["w"][p], fields, lam, dt, K, trajectory=True)

            h = 1e-4
            runs = [run(d) for d in (-2 * h, -h, 0.0, h, 2 * h)]
            if len({(st, _signature(tr)) for _, st, tr in runs}) > 1:
                skipped += 1
                continue
            Ls = [r[0] for r in runs]
            fd5 = (Ls[0] - 8 * Ls[1] + 8 * Ls[3] - Ls[4]) / (12 * h)
            assert dL == pytest.approx(fd5, rel=1e-6, abs=1e-9), (p, k, dL, fd5)
            Lp, Lm = run(1e-6)[0], run(-1e-6)[0]
            assert dL == pytest.approx((Lp - Lm) / 2e-6, rel=1e-4, abs=1e-8), (p, k, dL)
            checked += 1
    assert checked >= 60 and skipped <= checked, (checked, skipped)


def test_field_gradient_matches_finite_differences(setup):
    g, dt, fields, parts, lam = setup
    sp = wl.species_table()
    rng = np.random.default_rng(2)
    sub = {k: v[:120] for k, v in parts.items()}
    agree = 0
    for trial in range(4):
        tF = [rng.normal(size=g.shape) * np.abs(f).max() for f in fields]
        L0, dL, _ = orc.loss_dual(g, sp, sub, fields, lam, dt, K, tF=tF)
        h = 1e-6
        Lp, _, _ = orc.loss_dual(g, sp, sub, [f + h * t for f, t in zip(fields, tF)], lam, dt, K)
        Lm, _, _ = orc.loss_dual(g, sp, sub, [f - h * t for f, t in zip(fields, tF)], lam, dt, K)
        fd = (Lp - Lm) / (2 * h)
        if abs(dL - fd) <= 1e-5 * max(abs(dL), 1e-6):
            agree += 1
    assert agree >= 3          # a random field direction may move one particle across a kink


def test_loss_with_per_step_fields_is_the_sum_over_field_epochs():
    """loss_dual_steps takes step k's fields from field_steps[k]: with the same
    fields every step it equals loss_dual bit for bit; with fields A for the
    first k steps and B after, L equals the loss of k steps in A plus that of
    the remaining steps in B from the state the first k steps reach (orc.run);
    its u-derivative matches central differences of that split value."""
    import numpy as np

    from oracle import oracle as orc
    from paper_2503_04558_amd import workload as wl
    from adjoint_cases import shell_case

    g, dt, fields, parts, lam = shell_case(60)
    sp = wl.species_table()
    K, k = 12, 5
    tu = [np.ones(60), np.zeros(60), np.zeros(60)]
    same = orc.loss_dual_steps(g, sp, parts, [fields] * K, lam, dt, tu=tu)
    ref = orc.loss_dual(g, sp, parts, fields, lam, dt, K, tu=tu)
    assert same[0] == ref[0] and same[1] == ref[1]
    B = [1.7 * f for f in fields]                                   # a stronger field after step k
    L, dL, _ = orc.loss_dual_steps(g, sp, parts, [fields] * k + [B] * (K - k), lam, dt, tu=tu)

    def split(p):
        L1, _, _ = orc.loss_dual(g, sp, p, fields, lam, dt, k)
        mid, _, _, _ = orc.run(g, sp, p, fields, dt, k)
        L2, _, _ = orc.loss_dual(g, sp, mid, B, lam, dt, K - k)
        return L1 + L2

    assert abs(L - split(parts)) <= 1e-13 * max(1.0, abs(L))
    assert abs(L - ref[0]) > 1e-6                                     # the second epoch's fields matter
    h = 1e-6
    up = dict(parts, ur=parts["ur"] + h)
    um = dict(parts, ur=parts["ur"] - h)
    fd = (split(up) - split(um)) / (2 * h)
    assert abs(fd - dL) <= 1e-5 * max(1.0, abs(dL))
