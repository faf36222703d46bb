"""The adjoint over the last steps of a PIC loop (push + deposit, then the
field step, every step), through grpic_push_deposit_backward_range: the
fields change from step to step and are passed as the per-step states the
forward saw (a strided stack), the backward runs in particle batches with a
workspace sized for one batch, and the forward may be the FP32-split form
(checkpoints promoted to FP64).

Against the oracle's dual numbers fed the same per-step fields
(oracle.loss_dual_steps): d L / d u_i at the start of the window for sampled
particles, at the adjoint bar of test_gpu_adjoint.py.  Per-step field
gradients against central differences of the GPU forward with the fields
of one step perturbed, and their sum over steps against the summed form.
Batches reproduce the single call bit for bit.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2503_04558_amd import grpic
from paper_2503_04558_amd import workload as wl

from adjoint_cases import shell_lambda

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
K, C, WARM = 16, 8, 4


def _announce(msg):
    print(f"[gpu] {msg}", flush=True)


def _pic_window(g, parts_np, precision, fields0, dt):
    """WARM PIC steps, then K more saving checkpoints every C steps and the
    field state each push gathers from.  Returns the particles at the window's
    start (host), the checkpoints, the (6, K, rows, pitch) field history and
    the window's loss current."""
    metric = grpic.make_metric(g.a, g.M)
    sp = wl.species_table()
    dev = grpic.to_device(parts_np, precision)
    real = torch.float64 if precision == grpic.GRPIC_FP64 else torch.float32
    state = [torch.as_tensor(f).cuda() for f in fields0]
    solver = grpic.FieldSolver(metric, g)
    n = dev["cell"].numel()
    slot = grpic.grpic_checkpoint_bytes(n, 1, 1)
    ck = torch.full((K // C * slot,), 255, dtype=torch.uint8, device="cuda")
    hist = torch.empty((6, K) + tuple(g.shape), dtype=torch.float64, device="cuda")
    Jwin = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    start = None
    for k in range(WARM + K):
        J = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
        F = [s.to(real) for s in state]
        kw = {}
        w = k - WARM
        if w == 0:
            start = grpic.to_host(dev)
        if w >= 0:
            for c in range(6):
                hist[c, w].copy_(state[c])
            if w % C == 0:
                kw = dict(ckpt=ck[(w // C) * slot:(w // C + 1) * slot], ckpt_every=1)
        grpic.grpic_push_deposit(metric, g, sp, dev, F, J, dt, 1, **kw)
        if w >= 0:
            for a, b in zip(Jwin, J):
                a += b
        solver.step(state, J, dt, 0.53, 7, damp_cells=8, damp_max=0.1)
    torch.cuda.synchronize()
    return start, ck, hist, Jwin


def _backward(g, start_np, ck, hist, lam, dt, batches, grad_fields=None, gstride=0):
    n = len(start_np["cell"])
    parts = {"w": torch.as_tensor(np.asarray(start_np["w"], dtype=np.float64)).cuda(),
             "sp": torch.as_tensor(start_np["sp"]).cuda()}
    plane = hist.shape[2] * hist.shape[3]
    lam_t = [torch.as_tensor(l).cuda() for l in lam]
    gu = np.zeros((n, 3))
    bounds = np.linspace(0, n, batches + 1).astype(np.int64)
    size = int(np.max(np.diff(bounds)))
    ws = torch.full((grpic.grpic_backward_workspace_bytes(g, size, C),), 255, dtype=torch.uint8, device="cuda")
    for b0, b1 in zip(bounds[:-1], bounds[1:]):
        out = [torch.full((int(b1 - b0),), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
        grpic.grpic_push_deposit_backward_range(grpic.make_metric(g.a, g.M), g, wl.species_table(), parts,
                                                [hist[c, 0] for c in range(6)], lam_t, dt, K, 3, ck, C,
                                                int(b0), int(b1 - b0), ws, out, grad_fields,
                                                field_step_stride=plane, grad_step_stride=gstride)
        torch.cuda.synchronize()
        gu[b0:b1] = np.stack([t.cpu().numpy() for t in out], axis=1)
    return gu


def _oracle_grad_u(g, parts, hist_np, lam, dt):
    steps = np.ascontiguousarray(hist_np)
    n = len(parts["cell"])
    out = np.zeros((n, 3))
    for p in range(n):
        one = {k: v[p:p + 1] for k, v in parts.items()}
        for d in range(3):
            t = [np.zeros(1) for _ in range(3)]
            t[d][0] = 1.0
            _, out[p, d], _ = orc.loss_dual_steps(g, wl.species_table(), one, steps, lam, dt, tu=t)
    return out


@pytest.fixture(scope="module")
def window():
    _announce("adjoint over a PIC window: 128^2, 2e4 power-law particles, 4 + 16 steps")
    g = wl.make_grid(128, 128, 0.99)
    dt = wl.crossing_dt(g)
    parts = wl.pairs(g, 10_000, kind="powerlaw", seed=3, params=dict(gmax=1e3))
    fields0 = wl.wald_fields(g, B0=1.0)
    lam = shell_lambda(g, dt)
    start, ck, hist, Jwin = _pic_window(g, parts, grpic.GRPIC_FP64, fields0, dt)
    return dict(g=g, dt=dt, parts=parts, fields0=fields0, lam=lam, start=start, ck=ck, hist=hist, Jwin=Jwin)


def test_window_gradients_match_oracle_with_per_step_fields(window):
    g, dt, lam = window["g"], window["dt"], window["lam"]
    start, hist = window["start"], window["hist"]
    gu = _backward(g, start, window["ck"], hist, lam, dt, batches=3)
    assert np.all(np.isfinite(gu))
    hist_np = hist.cpu().numpy()
    # the fields really change across the window
    assert np.abs(hist_np[:, -1] - hist_np[:, 0]).max() > 1e-6 * np.abs(hist_np[:, 0]).max()
    live = np.flatnonzero(start["cell"] >= 0)
    nz = live[np.abs(gu[live]).max(axis=1) > 0]
    rng = np.random.default_rng(4)
    pick = np.concatenate([rng.choice(nz, min(150, len(nz)), replace=False),
                           rng.choice(live, 150, replace=False)])
    sub = {k: v[pick] for k, v in start.items()}
    ref = _oracle_grad_u(g, sub, hist_np, lam, dt)
    pert = {k: np.array(v, copy=True) for k, v in sub.items()}
    for k in ("ur", "uth", "uph"):
        pert[k] *= 1.0 + 4 * EPS
    sens = np.abs(_oracle_grad_u(g, pert, hist_np, lam, dt) - ref).max(axis=1)
    err = np.abs(gu[pick] - ref).max(axis=1)
    scale = np.abs(ref).max(axis=1)
    bar = 1e-9 * scale + 1e-13 * scale.max() + 64 * sens
    _announce(f"window grad_u: {len(nz)} non-zero of {len(live)}; sampled max err/bar "
              f"{float((err / np.maximum(bar, 1e-300)).max()):.3e}")
    assert len(nz) >= 50
    assert np.all(gu[pick][scale == 0.0] == 0.0)
    assert np.all(err <= bar), np.flatnonzero(err > bar)[:5]
    # the loss the backward differentiates is the window's: L from the GPU
    # forward equals the oracle's over the same per-step fields
    L_gpu = sum(float((torch.as_tensor(l).cuda() * j).sum()) for l, j in zip(lam, window["Jwin"]))
    steps = [[hist_np[c, k] for c in range(6)] for k in range(K)]
    L_orc, _, _ = orc.loss_dual_steps(g, wl.species_table(), start, steps, lam, dt)
    assert L_gpu == pytest.approx(L_orc, rel=1e-11, abs=1e-13)


def test_batches_equal_one_call_and_step_gradients_sum(window):
    g, dt, lam = window["g"], window["dt"], window["lam"]
    start, hist, ck = window["start"], window["hist"], window["ck"]
    plane = hist.shape[2] * hist.shape[3]
    one = _backward(g, start, ck, hist, lam, dt, batches=1)
    four = _backward(g, start, ck, hist, lam, dt, batches=4)
    assert np.array_equal(one, four)
    summed = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(6)]
    per = torch.zeros((6, K) + tuple(g.shape), dtype=torch.float64, device="cuda")
    _backward(g, start, ck, hist, lam, dt, batches=2, grad_fields=summed)
    _backward(g, start, ck, hist, lam, dt, batches=2, grad_fields=[per[c, 0] for c in range(6)], gstride=plane)
    torch.cuda.synchronize()
    for c in range(6):
        a, b = per[c].sum(dim=0), summed[c]
        assert (a - b).abs().max().item() <= 1e-12 * max(b.abs().max().item(), 1e-300)
    # per-step field gradient of one step against central differences of the
    # GPU forward over the recorded fields with that step's fields moved
    metric = grpic.make_metric(g.a, g.M)
    lam_t = [torch.as_tensor(l).cuda() for l in lam]

    def loss(step, tF, h):
        dev = grpic.to_device(start)
        J = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
        for k in range(K):
            F = [hist[c, k] + (h * tF[c] if k == step else 0.0) for c in range(6)]
            grpic.grpic_push_deposit(metric, g, wl.species_table(), dev, F, J, dt, 1)
        torch.cuda.synchronize()
        return sum(float((l * j).sum()) for l, j in zip(lam_t, J))

    rng = np.random.default_rng(8)
    agree = 0
    for trial, step in enumerate((2, 9, 15)):
        tF = [torch.as_tensor(rng.normal(size=g.shape)).cuda() * hist[c, step].abs().max() for c in range(6)]
        dL = sum(float((per[c, step] * tF[c]).sum()) for c in range(6))
        h = 1e-6
        fd = (loss(step, tF, h) - loss(step, tF, -h)) / (2 * h)
        if abs(fd - dL) <= 1e-4 * max(abs(dL), 1e-4):
            agree += 1
    assert agree >= 2                       # a random direction may move one particle across a CIC kink


def test_split_forward_checkpoints_promoted(window):
    """The same window with the FP32-split forward: checkpoints hold the float
    states promoted to double and the reverse replays in FP64 from them; the
    gradients stay close to the FP64 forward's (median relative difference
    below 1e-4: the split trajectory is within ~1e-6 of the FP64 one)."""
    g, dt, lam = window["g"], window["dt"], window["lam"]
    start_s, ck_s, hist_s, _ = _pic_window(g, window["parts"], grpic.GRPIC_FP32_SPLIT, window["fields0"], dt)
    # checkpoint 0 is the split start state promoted exactly
    n = len(start_s["cell"])
    off = (n * 4 + 7) // 8 * 8
    xr = ck_s[off: off + 8 * n].view(torch.float64).cpu().numpy()
    assert np.array_equal(xr, start_s["xr"].astype(np.float64))
    gs = _backward(g, start_s, ck_s, hist_s, lam, dt, batches=2)
    gd = _backward(g, window["start"], window["ck"], window["hist"], lam, dt, batches=2)
    assert np.all(np.isfinite(gs))
    scale = np.abs(gd).max(axis=1)
    nz = scale > 0
    rel = np.abs(gs - gd).max(axis=1)[nz] / scale[nz]
    _announce(f"split vs FP64 window gradients: median rel {float(np.median(rel)):.2e}, "
              f"p90 {float(np.quantile(rel, 0.9)):.2e}")
    assert np.median(rel) < 1e-4
