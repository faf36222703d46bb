"""The adjoint workload shared by the oracle pins and the GPU adjoint tests.

Loss: L = sum over steps n < K and particles of lambda . (F^r, F^th, G^ph)_n
with lambda_r = dt on the r-faces of row i*, the face r_{i*+1/2} nearest to
r = 5 (so L is the net charge carried through that shell), zero elsewhere.
Particles: 512^2 grid, a = 0.9, Wald field B0 = 1, Maxwell-Juttner pairs
(T = 0.5); 400 of them within one cell of the shell, spread over theta.
"""
import numpy as np

from paper_2503_04558_amd import workload as wl

K = 32
CKPT_EVERY = 8


def shell_face(g, r=5.0):
    i = np.arange(g.nr)
    return int(np.argmin(np.abs(g.r(i + 0.5) - r)))


def shell_lambda(g, dt, r=5.0):
    lam = [np.zeros(g.shape) for _ in range(3)]
    lam[0][g.guard + shell_face(g, r), :] = dt
    return lam


def shell_case(npart=400):
    g = wl.make_grid(512, 512, 0.9)
    dt = wl.crossing_dt(g)
    fields = wl.wald_fields(g, B0=1.0)
    parts = wl.pairs(g, 500_000, kind="mj", seed=0, params=dict(T=0.5))
    i_star = shell_face(g)
    rows = parts["cell"] // g.nth
    near = np.flatnonzero(np.abs(rows - i_star) <= 1)
    near = near[np.linspace(0, len(near) - 1, npart).astype(int)]
    sub = {k: v[near] for k, v in parts.items()}
    return g, dt, fields, sub, shell_lambda(g, dt)
