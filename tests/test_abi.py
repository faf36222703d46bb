"""CPU checks of the C ABI: libgrpic.so loads, exports every function that
include/grpic.h declares, and its host-side logic (argument validation, the
light-crossing bound) behaves as documented.  No device work is requested:
every call here returns before any HIP call."""
import ctypes
import math
import os
import re

import pytest

from paper_2503_04558_amd import grpic
from paper_2503_04558_amd import workload as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "grpic.h")).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(grpic_\w+)\s*\(", txt, flags=re.M)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert "grpic_push_deposit" in names and "grpic_sort" in names
    L = grpic.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(grpic.EXPORTED) <= set(names)


def test_crossing_time_matches_generator():
    for nr, nth, a in ((256, 256, 0.99), (512, 512, 0.9), (64, 32, 0.0)):
        g = wl.make_grid(nr, nth, a)
        t = grpic.grpic_crossing_time(grpic.make_metric(a, 1.0), g)
        assert t == pytest.approx(wl.crossing_time(g), rel=1e-12)
    bad = grpic.grpic_crossing_time(grpic.make_metric(2.0, 1.0), wl.make_grid(8, 8, 0.5))
    assert bad < 0


def test_grid_arrays_above_4gib_are_rejected():
    """Grid arrays are addressed with 32-bit byte offsets: (nr + 1 + 2 guard)
    x pitch doubles must stay below 4 GiB."""
    g = wl.make_grid(64, 32, 0.5)
    ok = grpic.make_grid(g)
    assert grpic.grpic_crossing_time(grpic.make_metric(0.5, 1.0), g) > 0
    rows = ok.nr + 1 + 2 * ok.guard
    big = grpic.grpic_grid(ok.nr, ok.nth, ok.guard, (2 ** 32) // (8 * rows) + 1, ok.lnr0, ok.dlnr, ok.dth)
    assert rows * big.pitch * 8 > 2 ** 32 - 1
    assert grpic.lib().grpic_crossing_time(ctypes.byref(grpic.make_metric(0.5, 1.0)), ctypes.byref(big)) < 0
    assert "4 GiB" in grpic.lib().grpic_last_error().decode()
    fits = grpic.grpic_grid(ok.nr, ok.nth, ok.guard, (2 ** 32 - 1) // (8 * rows), ok.lnr0, ok.dlnr, ok.dth)
    assert grpic.lib().grpic_crossing_time(ctypes.byref(grpic.make_metric(0.5, 1.0)), ctypes.byref(fits)) > 0


def _call_push(metric, grid, species, nsp, parts, fields, cur, dt, nsteps=1, ncorr=3):
    L = grpic.lib()
    return L.grpic_push_deposit(
        ctypes.byref(metric) if metric is not None else None,
        ctypes.byref(grid) if grid is not None else None,
        species, nsp,
        ctypes.byref(parts) if parts is not None else None,
        ctypes.byref(fields) if fields is not None else None,
        ctypes.byref(cur) if cur is not None else None,
        None, dt, nsteps, ncorr, None, 0, 0, None, None)


def _fake_args(g):
    """Structures with non-NULL placeholder pointers; only validated, never dereferenced."""
    fake = 0x1000
    parts = grpic.grpic_particles(10, *([fake] * 8), None, grpic.GRPIC_FP64, 0)
    fields = grpic.grpic_fields()
    for c in range(3):
        fields.D[c] = fake
        fields.B[c] = fake
    cur = grpic.grpic_current(fake, fake, fake)
    return parts, fields, cur


def test_argument_validation_errors():
    g = wl.make_grid(32, 32, 0.9)
    G = grpic.make_grid(g)
    m = grpic.make_metric(0.9, 1.0)
    sp = grpic.make_species(wl.species_table())
    parts, fields, cur = _fake_args(g)
    dt = wl.crossing_dt(g)
    L = grpic.lib()
    assert _call_push(None, G, sp, 2, parts, fields, cur, dt) == grpic.GRPIC_EINVAL
    assert _call_push(m, G, sp, 0, parts, fields, cur, dt) == grpic.GRPIC_EINVAL
    assert _call_push(m, G, sp, 9, parts, fields, cur, dt) == grpic.GRPIC_EINVAL
    assert _call_push(m, G, sp, 2, parts, fields, cur, -dt) == grpic.GRPIC_EINVAL
    assert _call_push(m, G, sp, 2, parts, fields, cur, float("nan")) == grpic.GRPIC_EINVAL
    assert _call_push(m, G, sp, 2, parts, fields, cur, dt, ncorr=-1) == grpic.GRPIC_EINVAL
    assert _call_push(m, G, sp, 2, parts, fields, None, dt) == grpic.GRPIC_EINVAL
    assert b"current" in L.grpic_last_error()
    assert _call_push(grpic.make_metric(1.5, 1.0), G, sp, 2, parts, fields, cur, dt) == grpic.GRPIC_EINVAL
    bad_grid = grpic.make_grid(g)
    bad_grid.guard = 1
    assert _call_push(m, bad_grid, sp, 2, parts, fields, cur, dt) == grpic.GRPIC_EINVAL
    bad_grid = grpic.make_grid(g)
    bad_grid.dth = 0.1
    assert _call_push(m, bad_grid, sp, 2, parts, fields, cur, dt) == grpic.GRPIC_EINVAL
    bad_grid = grpic.make_grid(g)
    bad_grid.pitch = g.nth
    assert _call_push(m, bad_grid, sp, 2, parts, fields, cur, dt) == grpic.GRPIC_EINVAL
    # dt above the light-crossing time of the smallest cell
    assert _call_push(m, G, sp, 2, parts, fields, cur, 2.01 * dt) == grpic.GRPIC_ERANGE
    assert b"crossing" in L.grpic_last_error()
    # massive species need m > 0
    sp_bad = grpic.make_species([dict(q=1.0, m=0.0)])
    assert _call_push(m, G, sp_bad, 1, parts, fields, cur, dt) == grpic.GRPIC_EINVAL
    # nothing to do is not an error (returns before any launch)
    empty = grpic.grpic_particles(0, *([None] * 9), grpic.GRPIC_FP64, 0)
    assert _call_push(m, G, sp, 2, empty, fields, cur, dt) == grpic.GRPIC_OK


def test_sort_workspace_and_validation():
    g = wl.make_grid(64, 32, 0.9)
    G = grpic.make_grid(g)
    need = grpic.grpic_sort_workspace_bytes(g, 1000)
    assert need >= 8 * (64 * 32 + 1)
    L = grpic.lib()
    fake = 0x1000
    pin = grpic.grpic_particles(10, *([fake] * 8), None, grpic.GRPIC_FP64, 0)
    pout = grpic.grpic_particles(10, *([fake + 64] * 8), None, grpic.GRPIC_FP64, 0)
    rc = L.grpic_sort(ctypes.byref(G), ctypes.byref(pin), ctypes.byref(pout), None, None, 0, fake, need - 8,
                      fake, None)
    assert rc == grpic.GRPIC_ENOMEM
    tneed = grpic.grpic_tiling_bytes(g, 10)
    rc = L.grpic_sort(ctypes.byref(G), ctypes.byref(pin), ctypes.byref(pout), None, fake, tneed - 1, fake, need,
                      fake, None)
    assert rc == grpic.GRPIC_ENOMEM
    pout.precision = grpic.GRPIC_FP32_SPLIT
    rc = L.grpic_sort(ctypes.byref(G), ctypes.byref(pin), ctypes.byref(pout), None, None, 0, fake, need, fake, None)
    assert rc == grpic.GRPIC_EINVAL


def test_push_rejects_unknown_tiling():
    g = wl.make_grid(32, 32, 0.9)
    parts, fields, cur = _fake_args(g)
    L = grpic.lib()
    rc = L.grpic_push_deposit(ctypes.byref(grpic.make_metric(0.9, 1.0)), ctypes.byref(grpic.make_grid(g)),
                              grpic.make_species(wl.species_table()), 2, ctypes.byref(parts), ctypes.byref(fields),
                              ctypes.byref(cur), 0x2000, wl.crossing_dt(g), 1, 3, None, 0, 0, None, None)
    assert rc == grpic.GRPIC_EINVAL and b"tiling" in L.grpic_last_error()


def test_checkpoint_and_backward_validation():
    g = wl.make_grid(32, 32, 0.9)
    assert grpic.grpic_checkpoint_bytes(1000, 32, 8) == 4 * (4000 + 5 * 8 * 1000)
    assert grpic.grpic_checkpoint_bytes(1000, 30, 8) == 0          # ckpt_every must divide nsteps
    rows, pitch = g.nr + 1 + 2 * g.guard, g.pitch
    assert grpic.grpic_backward_workspace_bytes(g, 1000, 8) == 320000 + 4 * (2 * rows + 2 * pitch + 2)
    parts, fields, cur = _fake_args(g)
    L = grpic.lib()
    m, G, sp = grpic.make_metric(0.9, 1.0), grpic.make_grid(g), grpic.make_species(wl.species_table())
    dt = wl.crossing_dt(g)
    # forward with a checkpoint buffer that is too small
    rc = L.grpic_push_deposit(ctypes.byref(m), ctypes.byref(G), sp, 2, ctypes.byref(parts), ctypes.byref(fields),
                              ctypes.byref(cur), None, dt, 32, 3, 0x3000, 16, 8, None, None)
    assert rc == grpic.GRPIC_ENOMEM
    rc = L.grpic_push_deposit(ctypes.byref(m), ctypes.byref(G), sp, 2, ctypes.byref(parts), ctypes.byref(fields),
                              ctypes.byref(cur), None, dt, 30, 3, 0x3000, 1 << 30, 8, None, None)
    assert rc == grpic.GRPIC_EINVAL
    gu = grpic.grpic_momentum_grads(0x1000, 0x1000, 0x1000)
    gf = grpic.grpic_field_grads()
    for c in range(3):
        gf.D[c] = 0x1000
        gf.B[c] = 0x1000
    ck = grpic.grpic_checkpoint_bytes(10, 32, 8)
    ws = grpic.grpic_backward_workspace_bytes(g, 10, 8)
    args = [ctypes.byref(m), ctypes.byref(G), sp, 2, ctypes.byref(parts), ctypes.byref(fields), ctypes.byref(cur),
            dt, 32, 3, 0x3000, ck, 8, 0x4000, ws, ctypes.byref(gu), ctypes.byref(gf), None]
    bad = list(args)
    bad[9] = 9                                                     # ncorr above the adjoint's limit
    assert L.grpic_push_deposit_backward(*bad) == grpic.GRPIC_EINVAL
    bad = list(args)
    bad[14] = ws - 8                                               # workspace too small
    assert L.grpic_push_deposit_backward(*bad) == grpic.GRPIC_ENOMEM
    bad = list(args)
    bad[7] = 2.01 * dt
    assert L.grpic_push_deposit_backward(*bad) == grpic.GRPIC_ERANGE


def test_vay_entry_validation():
    """grpic_push_deposit_vay shares the push's checks and takes FP64
    particles only; every call here returns before any launch."""
    g = wl.make_grid(32, 32, 0.9)
    G = grpic.make_grid(g)
    m = grpic.make_metric(0.9, 1.0)
    sp = grpic.make_species(wl.species_table())
    parts, fields, cur = _fake_args(g)
    dt = wl.crossing_dt(g)
    L = grpic.lib()

    def call(parts, dt, ncorr=3):
        return L.grpic_push_deposit_vay(ctypes.byref(m), ctypes.byref(G), sp, 2, ctypes.byref(parts),
                                        ctypes.byref(fields), ctypes.byref(cur), None, dt, 1, ncorr, None, None)

    split = grpic.grpic_particles(10, *([0x1000] * 8), None, grpic.GRPIC_FP32_SPLIT, 0)
    assert call(split, dt) == grpic.GRPIC_EINVAL
    assert b"FP64" in L.grpic_last_error()
    assert call(parts, -dt) == grpic.GRPIC_EINVAL
    assert call(parts, dt, ncorr=17) == grpic.GRPIC_EINVAL
    assert call(parts, 2.01 * dt) == grpic.GRPIC_ERANGE
    empty = grpic.grpic_particles(0, *([None] * 9), grpic.GRPIC_FP64, 0)
    assert call(empty, dt) == grpic.GRPIC_OK
    with pytest.raises(ValueError, match="checkpoints"):
        grpic.grpic_push_deposit(m, g, wl.species_table(), {}, [], [], dt, 1, kick="vay", ckpt=object())
    with pytest.raises(ValueError, match="kick"):
        grpic.grpic_push_deposit(m, g, wl.species_table(), {}, [], [], dt, 1, kick="leapfrog")


def test_field_step_validation():
    """The field step's host-side checks, before any device work: a theta
    grid narrower than 2 * guard (the columns beyond the axes mirror physical
    ones), tables not written for this metric and grid, a small workspace."""
    L = grpic.lib()
    m = grpic.make_metric(0.9, 1.0)
    fake = 0x1000
    state = grpic.grpic_field_state()
    for c in range(3):
        state.D[c] = fake
        state.B[c] = fake
    narrow = grpic.make_grid(wl.make_grid(9, 3, 0.9))
    ok = grpic.make_grid(wl.make_grid(9, 8, 0.9))

    def call(grid, tables, ws_bytes, dt=0.01):
        return L.grpic_field_step(ctypes.byref(m), ctypes.byref(grid), tables, ctypes.byref(state), None, dt, 0.53,
                                  7, 0, 0.0, fake, ws_bytes, None)

    assert call(narrow, fake, 1 << 30) == grpic.GRPIC_EINVAL
    assert b"nth" in L.grpic_last_error()
    assert call(ok, fake, 1 << 30) == grpic.GRPIC_EINVAL            # tables never written
    assert b"tables" in L.grpic_last_error()
    assert call(ok, fake, 1 << 30, dt=-1.0) == grpic.GRPIC_EINVAL
    assert L.grpic_field_workspace_bytes(ctypes.byref(ok)) == 18 * (9 + 1 + 2 * ok.guard) * ok.pitch * 8


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No CPU fallback: with libgrpic.so absent the binding raises."""
    monkeypatch.setattr(grpic, "_lib", None)
    monkeypatch.setattr(grpic, "LIB_PATH", str(tmp_path / "libgrpic.so"))
    with pytest.raises(RuntimeError, match="not built"):
        grpic.lib()


def test_spline3_entry_validation():
    """grpic_push_deposit_spline3 and grpic_charge3: FP64 only, guard >= 3,
    nth >= 4; every call here returns before any launch."""
    L = grpic.lib()
    m = grpic.make_metric(0.9, 1.0)
    sp = grpic.make_species(wl.species_table())
    g3 = wl.make_grid(32, 32, 0.9, guard=3)
    parts, fields, cur = _fake_args(g3)
    dt = wl.crossing_dt(g3)

    def call(grid, parts, dt):
        G = grpic.make_grid(grid)
        return L.grpic_push_deposit_spline3(ctypes.byref(m), ctypes.byref(G), sp, 2, ctypes.byref(parts),
                                            ctypes.byref(fields), ctypes.byref(cur), None, dt, 1, 3, None, None)

    assert call(wl.make_grid(32, 32, 0.9), parts, dt) == grpic.GRPIC_EINVAL        # guard 2
    assert b"guard" in L.grpic_last_error()
    assert call(wl.make_grid(32, 3, 0.9, guard=3), parts, dt) == grpic.GRPIC_EINVAL  # nth 3
    split = grpic.grpic_particles(10, *([0x1000] * 8), None, grpic.GRPIC_FP32_SPLIT, 0)
    assert call(g3, split, dt) == grpic.GRPIC_EINVAL
    assert call(g3, parts, 2.01 * dt) == grpic.GRPIC_ERANGE
    empty = grpic.grpic_particles(0, *([None] * 9), grpic.GRPIC_FP64, 0)
    assert call(g3, empty, dt) == grpic.GRPIC_OK
    G2 = grpic.make_grid(wl.make_grid(16, 16, 0.5))
    assert L.grpic_charge3(ctypes.byref(G2), sp, 2, ctypes.byref(parts), 0x1000, None) == grpic.GRPIC_EINVAL


def test_qed_entry_validation():
    """grpic_push_deposit_qed: FP64 particles with tags, a massless photon
    species and massive leptons inside the species table, 1 < gamma_thr,
    0 < eps_ph < sqrt(gamma_thr^2 - 1), tau >= 0, n_used given, and the
    push's own checks; every call here returns before any launch."""
    L = grpic.lib()
    g = wl.make_grid(32, 32, 0.9)
    G = grpic.make_grid(g)
    m = grpic.make_metric(0.9, 1.0)
    table = wl.qed_species_table()
    sp = grpic.make_species(table)
    fake = 0x1000
    parts = grpic.grpic_particles(10, *([fake] * 8), None, grpic.GRPIC_FP64, 0, fake)
    _, fields, cur = _fake_args(g)
    dt = wl.crossing_dt(g)

    def call(parts=parts, dt=dt, nsp=3, species=sp, n_used=fake, step=0, **kw):
        q = dict(gamma_thr=100.0, eps_ph=4.0, tau=2.0, seed=1, electron_sp=0, positron_sp=1, photon_sp=2)
        q.update(kw)
        Q = grpic.make_qed(**q)
        return L.grpic_push_deposit_qed(ctypes.byref(m), ctypes.byref(G), species, nsp, ctypes.byref(parts),
                                        ctypes.byref(fields), ctypes.byref(cur), None, dt, step, 3,
                                        ctypes.byref(Q), n_used, None, 0, None, None, None)

    notag = grpic.grpic_particles(10, *([fake] * 8), None, grpic.GRPIC_FP64, 0, None)
    assert call(parts=notag) == grpic.GRPIC_EINVAL and b"tags" in L.grpic_last_error()
    split = grpic.grpic_particles(10, *([fake] * 8), None, grpic.GRPIC_FP32_SPLIT, 0, fake)
    assert call(parts=split) == grpic.GRPIC_EINVAL and b"FP64" in L.grpic_last_error()
    assert call(n_used=None) == grpic.GRPIC_EINVAL and b"n_used" in L.grpic_last_error()
    assert call(photon_sp=3) == grpic.GRPIC_EINVAL
    assert call(photon_sp=1) == grpic.GRPIC_EINVAL and b"massless" in L.grpic_last_error()
    assert call(electron_sp=2) == grpic.GRPIC_EINVAL and b"massive" in L.grpic_last_error()
    assert call(gamma_thr=1.0) == grpic.GRPIC_EINVAL
    assert call(eps_ph=0.0) == grpic.GRPIC_EINVAL
    assert call(gamma_thr=3.0, eps_ph=math.sqrt(8.0)) == grpic.GRPIC_EINVAL       # eps_ph = |u| at threshold
    assert call(tau=-1.0) == grpic.GRPIC_EINVAL
    assert call(tau=float("nan")) == grpic.GRPIC_EINVAL
    assert call(step=-1) == grpic.GRPIC_EINVAL
    assert call(dt=-dt) == grpic.GRPIC_EINVAL
    assert call(dt=2.01 * dt) == grpic.GRPIC_ERANGE
    empty = grpic.grpic_particles(0, *([None] * 9), grpic.GRPIC_FP64, 0, None)
    assert call(parts=empty) == grpic.GRPIC_OK


def test_sort_noalloc_rejects_grids_beyond_its_scratch():
    """grpic_sort_noalloc: its fixed scratch holds the sort of a 2048^2 grid;
    a 4096^2 grid is rejected with GRPIC_ENOMEM before any device work."""
    L = grpic.lib()
    fake = 0x1000
    parts = grpic.grpic_particles(10, *([fake] * 8), None, grpic.GRPIC_FP64, 0, None)
    out = grpic.grpic_particles(10, *([fake * 2] * 8), None, grpic.GRPIC_FP64, 0, None)
    big = grpic.make_grid(wl.make_grid(4096, 4096, 0.9))
    assert grpic.grpic_sort_workspace_bytes(wl.make_grid(2048, 2048, 0.9), 10) <= grpic.GRPIC_SORT_SCRATCH_BYTES
    assert grpic.grpic_sort_workspace_bytes(wl.make_grid(4096, 4096, 0.9), 10) > grpic.GRPIC_SORT_SCRATCH_BYTES
    rc = L.grpic_sort_noalloc(ctypes.byref(big), ctypes.byref(parts), ctypes.byref(out), None, None, 0, fake, None)
    assert rc == grpic.GRPIC_ENOMEM and b"scratch" in L.grpic_last_error()
    ok = grpic.make_grid(wl.make_grid(64, 64, 0.9))
    rc = L.grpic_sort_noalloc(ctypes.byref(ok), ctypes.byref(parts), ctypes.byref(out), None, None, 0, None, None)
    assert rc == grpic.GRPIC_EINVAL and b"n_alive" in L.grpic_last_error()


@pytest.mark.parametrize("nr,nth,n", [(48, 200, 9000), (2048, 2048, 200_000_000), (7, 64, 0), (5, 70, 3)])
def test_tiling_bytes_follow_the_documented_layout(nr, nth, n):
    """grpic_tiling_bytes against the layout the GPU tests read back: a
    40-byte header, the 256-particle cut (16 B per entry) and its int32 live
    counts, then 8-byte aligned the 192-particle cut and its counts, then 8-byte
    aligned the anchor table (r at nr + 10 row corners, sin and cos at
    tiles * 64 + 9 column corners)."""
    g = wl.make_grid(nr, nth, 0.9)
    ntiles = nr * ((nth + 63) // 64)
    cap, cap3 = n // 256 + ntiles + 8, n // 192 + ntiles + 8
    al = lambda b: (b + 7) // 8 * 8
    s3 = al(40 + 20 * cap)
    anchors = al(s3 + 20 * cap3)
    cols = ((nth + 63) // 64) * 64 + 9
    assert grpic.grpic_tiling_bytes(g, n) == anchors + 8 * ((nr + 10) + 2 * cols)
