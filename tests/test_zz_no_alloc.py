"""grpic_sort_noalloc (the sort with the library's static scratch in place
of a caller workspace) against grpic_sort, through the C ABI: two calls in a
row, the second on a smaller grid with fewer particles, each compared with a
grpic_sort of the same input.  Integer results bit for bit: the live count,
the cell offsets, the sorted cell array, the tiling's header and slice
table; the particles as a multiset within each cell (the order inside a cell
is not specified), matched by tag."""
import numpy as np
import pytest
import torch

from paper_2503_04558_amd import grpic
from paper_2503_04558_amd import workload as wl

pytestmark = pytest.mark.gpu


def _input(g, npairs, seed):
    host = wl.pairs(g, npairs, kind="uniform", seed=seed)
    n = len(host["cell"])
    rng = np.random.default_rng(seed)
    host["cell"][rng.random(n) < 0.1] = -1                 # some removed particles
    host["tag"] = rng.permutation(n).astype(np.uint64)     # unique keys for the multiset check
    return grpic.to_device(host)


def _sort(g, parts, noalloc):
    n = parts["cell"].numel()
    out = grpic.empty_particles(n, with_tag=True)
    offs = torch.empty(g.nr * g.nth + 1, dtype=torch.int64, device="cuda")
    n_alive = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    tiling = torch.full((grpic.grpic_tiling_bytes(g, n),), 0xAB, dtype=torch.uint8, device="cuda")
    if noalloc:
        grpic.grpic_sort_noalloc(g, parts, out, offs, n_alive, tiling)
    else:
        ws = torch.full((grpic.grpic_sort_workspace_bytes(g, n),), 0xCD, dtype=torch.uint8, device="cuda")
        grpic.grpic_sort(g, parts, out, offs, ws, n_alive, tiling)
    torch.cuda.synchronize()
    return grpic.to_host(out), offs.cpu().numpy(), int(n_alive.item()), tiling.cpu().numpy()


def _slice_tables(g, n):
    """Byte ranges of a tiling that the sort writes: the header with the cut
    into slices of at most 256 particles, and the cut into slices of at most
    192 (tiles of 64 cells of a row; each table is followed by a live count
    per entry that the push writes)."""
    ntiles = g.nr * ((g.nth + 63) // 64)
    cap, cap3 = n // 256 + ntiles + 8, n // 192 + ntiles + 8
    s3 = (40 + 20 * cap + 7) // 8 * 8
    return [(0, 40 + 16 * cap), (s3, s3 + 16 * cap3)]


def _check_same(g, a, b):
    pa, oa, na, ta = a
    pb, ob, nb, tb = b
    n = len(pa["cell"])
    assert na == nb and np.array_equal(oa, ob)
    assert np.array_equal(pa["cell"], pb["cell"])
    assert np.all(pa["cell"][na:] == -1) and np.all(pa["cell"][:na] >= 0)
    for lo, hi in _slice_tables(g, n):
        assert np.array_equal(ta[lo:hi], tb[lo:hi])
    # within each cell the same particles (sorted by cell, so order by (cell, tag))
    for p in (pa, pb):
        order = np.lexsort((p["tag"][:na], p["cell"][:na]))
        for key in p:
            p[key] = p[key][:na][order]
    for key in pa:
        assert np.array_equal(pa[key], pb[key]), key
    return na


def test_sort_noalloc_matches_sort_twice_smaller_second():
    for nr, nth, npairs, seed in ((512, 384, 400_000, 1), (96, 70, 20_000, 2)):
        print(f"[gpu] sort_noalloc {nr}x{nth}, {2 * npairs} particles", flush=True)
        g = wl.make_grid(nr, nth, 0.9)
        parts = _input(g, npairs, seed)
        ref = _sort(g, parts, noalloc=False)
        got = _sort(g, parts, noalloc=True)
        na = _check_same(g, got, ref)
        assert 0 < na < 2 * npairs


def test_sort_noalloc_feeds_the_tiled_push():
    """The tiling written by the no-allocation sort drives the tiled push to
    the same result as the tiling of grpic_sort."""
    g = wl.make_grid(128, 128, 0.99)
    host = wl.pairs(g, 30_000, kind="mj", seed=3, params=dict(T=0.5))
    n = len(host["cell"])
    host["tag"] = np.arange(n, dtype=np.uint64)            # identity through the sorts
    F = [torch.as_tensor(f).cuda() for f in wl.wald_fields(g)]
    m = grpic.make_metric(g.a, g.M)
    dt = wl.crossing_dt(g)
    res = []
    for noalloc in (False, True):
        parts = grpic.to_device(host)
        out = grpic.empty_particles(n, with_tag=True)
        n_alive = torch.zeros(1, dtype=torch.int64, device="cuda")
        tiling = torch.empty(grpic.grpic_tiling_bytes(g, n), dtype=torch.uint8, device="cuda")
        if noalloc:
            grpic.grpic_sort_noalloc(g, parts, out, None, n_alive, tiling)
        else:
            ws = torch.empty(grpic.grpic_sort_workspace_bytes(g, n), dtype=torch.uint8, device="cuda")
            grpic.grpic_sort(g, parts, out, None, ws, n_alive, tiling)
        J = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
        grpic.grpic_push_deposit(m, g, wl.species_table(), out, F, J, dt, 3, tiling=tiling)
        torch.cuda.synchronize()
        res.append((grpic.to_host(out), [j.cpu().numpy() for j in J]))
    (pa, Ja), (pb, Jb) = res

    def by_tag(p):
        live = p["cell"] >= 0
        order = np.argsort(p["tag"][live])
        return {k: v[live][order] for k, v in p.items()}

    a, b = by_tag(pa), by_tag(pb)
    assert len(a["tag"]) > 0.9 * n
    for k in ("tag", "cell", "xr", "xth", "ur", "uth", "uph"):
        assert np.array_equal(a[k], b[k]), k          # each particle's step does not depend on its slot
    for a, b in zip(Ja, Jb):
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
