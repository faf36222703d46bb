"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the oracle.

Norms (FP64, tolerance tol):
* position: |d xi|, |d eta| <= tol * max(1, |xi|)
* momentum, per covariant component i:
  |d u_i| * sqrt(gamma^ii) <= tol * sqrt(1 + gamma^jk u_j u_k)
  (the change measured in the local orthonormal frame's units)
* current, per array: max |dF| <= tol * max A_F, and per element
  |dF| <= tol * A_F, where A_F is the oracle's per-element sum of the
  contributions' magnitude scales (|q w|/dt for F^r, F^th; |q w dphi|/dt for
  G^ph).  The scale, not |contribution|, bounds the rounding of a value whose
  terms cancel (the flux at the far side of a particle's window is zero in
  exact arithmetic).
* live/removed status must agree particle by particle.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as orc
from paper_2503_04558_amd import grpic
from paper_2503_04558_amd import workload as wl


def gpu_run(grid, species, parts_np, fields_np, dt, nsteps, ncorr=3, precision=grpic.GRPIC_FP64,
            J0=None, tiled=False):
    """Push on the GPU.  tiled: sort on the GPU first (grpic_sort with a
    tiling; phi carries each particle's index through the sort) and push with
    the tiling; the result is returned in the input order."""
    n = len(parts_np["cell"])
    host = dict(parts_np)
    if tiled:
        host["phi"] = np.arange(n, dtype=np.float64)
    parts = grpic.to_device(host, precision)
    real = torch.float64 if precision == grpic.GRPIC_FP64 else torch.float32
    F = [torch.as_tensor(f).to(device="cuda", dtype=real) for f in fields_np]
    J = [torch.zeros(grid.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    if J0 is not None:
        for j, j0 in zip(J, J0):
            j.copy_(torch.as_tensor(j0))
    counters = torch.zeros(grpic.GRPIC_NCOUNTERS, dtype=torch.int64, device="cuda")
    tiling = None
    perm = None
    if tiled:
        sorter = grpic.Sorter(grid, n, precision, with_phi=True)
        parts = sorter.sort(parts)
        n_alive = int(sorter.n_alive.item())
        perm = parts["phi"][:n_alive].cpu().numpy().astype(np.int64)
        parts = {k: v for k, v in parts.items() if k != "phi"}
        tiling = sorter.tiling
    grpic.grpic_push_deposit(grpic.make_metric(grid.a, grid.M), grid, species, parts, F, J, dt, nsteps,
                             ncorr, tiling=tiling, counters=counters)
    torch.cuda.synchronize()
    cnt = dict(zip(grpic.COUNTER_NAMES, counters.cpu().numpy().tolist()))
    out = grpic.to_host(parts)
    if tiled:
        back = {k: np.array(parts_np[k], copy=True) for k in out}
        back["cell"][:] = -1
        for k in out:
            back[k][perm] = out[k][: len(perm)]
        out = back
    return out, [j.cpu().numpy() for j in J], cnt


def oracle_run(grid, species, parts_np, fields_np, dt, nsteps, ncorr=3):
    p, J, A, st = orc.run(grid, species, parts_np, fields_np, dt, nsteps, ncorr=ncorr, with_abs=True)
    return p, J, A, st


def positions(grid, p):
    ci = p["cell"] // grid.nth
    cj = p["cell"] % grid.nth
    return ci + p["xr"].astype(np.float64), cj + p["xth"].astype(np.float64)


def compare_particles(grid, pg, po, tol):
    """Returns a dict of worst normalised errors; asserts status agreement."""
    alive_g, alive_o = pg["cell"] >= 0, po["cell"] >= 0
    mism = int(np.count_nonzero(alive_g != alive_o))
    both = alive_g & alive_o
    xg, eg = positions(grid, {k: v[both] for k, v in pg.items()})
    xo, eo = positions(grid, {k: v[both] for k, v in po.items()})
    pos_err = max(np.max(np.abs(xg - xo) / np.maximum(1.0, np.abs(xo)), initial=0.0),
                  np.max(np.abs(eg - eo) / np.maximum(1.0, np.abs(eo)), initial=0.0))
    r = grid.r(xo)
    th = grid.theta(eo)
    k = wl._ks_pieces(grid.a, grid.M, r, th)
    uo = [po[c][both].astype(np.float64) for c in ("ur", "uth", "uph")]
    ug = [pg[c][both].astype(np.float64) for c in ("ur", "uth", "uph")]
    norm = np.sqrt(1.0 + k["h_rr"] * uo[0] ** 2 + 2 * k["h_rp"] * uo[0] * uo[2] + k["h_tt"] * uo[1] ** 2
                   + k["h_pp"] * uo[2] ** 2)
    hii = (k["h_rr"], k["h_tt"], k["h_pp"])
    mom_err = max((np.max(np.abs(ug[i] - uo[i]) * np.sqrt(hii[i]) / norm, initial=0.0) for i in range(3)))
    return dict(status_mismatch=mism, pos=float(pos_err), mom=float(mom_err), n_alive=int(both.sum()))


def compare_current(Jg, Jo, Ao, tol):
    worst = 0.0
    for g, o, a in zip(Jg, Jo, Ao):
        scale = max(np.abs(a).max(), 1e-300)
        worst = max(worst, np.abs(g - o).max() / scale)
        bad = np.abs(g - o) > tol * a
        assert not bad.any(), ("per-element current error above tol * A_F", int(bad.sum()),
                               float((np.abs(g - o) / np.maximum(a, 1e-300)).max()))
    return worst


def assert_parity(grid, species, parts_np, fields_np, dt, nsteps, tol=1e-12, ncorr=3, tiled=False):
    pg, Jg, cg = gpu_run(grid, species, parts_np, fields_np, dt, nsteps, ncorr, tiled=tiled)
    po, Jo, Ao, so = oracle_run(grid, species, parts_np, fields_np, dt, nsteps, ncorr)
    e = compare_particles(grid, pg, po, tol)
    assert e["status_mismatch"] == 0, e
    assert e["pos"] <= tol and e["mom"] <= tol, e
    e["J"] = compare_current(Jg, Jo, Ao, tol)
    assert e["J"] <= tol, e
    if not tiled:       # the GPU sort drops particles removed before the push; the oracle counts them
        assert cg["bad"] == so["bad"], (cg, so)
        assert cg["live_steps"] == so["live_steps"], (cg, so)
    assert cg["out"] == so["out"] and cg["reflected"] == so["reflected"], (cg, so)
    return e, cg
