"""Seeded synthetic inputs for the GRPIC push + deposit path.

This module builds inputs only; it holds none of the push or deposit
arithmetic.  It is the one module that both the CPU oracle tests and the HIP
path take their inputs from.

Contents
--------
* ``make_grid``: the 2D axisymmetric Kerr-Schild grid, logarithmic in r and
  uniform in theta (Sec. 2.1, boundary conditions; Sec. 3.3 and 4 use a
  log-r grid).  Vertex i sits at ln r = lnr0 + i*dlnr, vertex j at
  theta = j*pi/nth.
* ``wald_fields``: the rotating vacuum Wald solution of App. C (eqs.
  wald-vector-potential and wald-solution-ks, with the mass M written back
  in) point-sampled at the Yee stagger of Fig. Yee, with D^i obtained from
  E_i by inverting eq. E-H-B-D.  On the axis D^ph = B^th = 0 (Sec. 2.1).
* ``monopole_fields``: the vacuum monopole of App. C (the initial field of
  the Sec. 4 spark-gap runs) on the same stagger, D^i again from eq.
  E-H-B-D; ``qed_particles``: e+- and photons for that workload.
* ``crossing_dt``: the cell crossing time at the coordinate speed of light,
  minimised over cell centres.
* particle samplers: pairs placed per cell with uniform offsets; momenta
  drawn in the local orthonormal frame of gamma_ij (isotropic with |u|
  uniform, Maxwell-Juttner with a bulk phi rotation, or a power law in the
  Lorentz factor) and mapped to covariant Kerr-Schild components.

Random numbers come from numpy PCG64 streams, one per chunk of
``CHUNK_PAIRS`` pairs, keyed by (seed, chunk index), so any leading subset
of a large draw is reproduced exactly by a small draw with the same seed.

Field arrays are (nr + 1 + 2*guard) rows x pitch columns, float64; element
[i + guard, j + guard] holds grid point (i + s_r, j + s_th) of a component
with stagger (s_r, s_th).  Component order: D^r, D^th, D^ph, B^r, B^th, B^ph.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

FIELD_NAMES = ("Dr", "Dth", "Dph", "Br", "Bth", "Bph")
# Stagger (s_r, s_th) of each field component, Fig. Yee.
STAGGER = {
    "Dr": (0.5, 0.0), "Dth": (0.0, 0.5), "Dph": (0.0, 0.0),
    "Br": (0.0, 0.5), "Bth": (0.5, 0.0), "Bph": (0.5, 0.5),
}
# Current arrays in flux form share the D stagger: F^r at (i+1/2, j),
# F^th at (i, j+1/2), G^ph at (i, j).
CURRENT_NAMES = ("Fr", "Fth", "Gph")

CHUNK_PAIRS = 1 << 16

SPECIES_PAIRS = ((-1.0, 1.0), (1.0, 1.0))   # (q, m) of e-, e+


@dataclass(frozen=True)
class Grid:
    a: float
    M: float
    nr: int
    nth: int
    guard: int
    pitch: int
    lnr0: float
    dlnr: float
    dth: float

    @property
    def rows(self) -> int:
        return self.nr + 1 + 2 * self.guard

    @property
    def shape(self) -> tuple[int, int]:
        return (self.rows, self.pitch)

    @property
    def ncell(self) -> int:
        return self.nr * self.nth

    def r(self, xi):
        return np.exp(self.lnr0 + np.asarray(xi, dtype=np.float64) * self.dlnr)

    def theta(self, eta):
        return np.asarray(eta, dtype=np.float64) * self.dth

    def index(self, i, j):
        """Flat array index of grid point (i, j) (any stagger)."""
        return (np.asarray(i) + self.guard) * self.pitch + (np.asarray(j) + self.guard)


def horizon(a: float, M: float = 1.0) -> float:
    """Outer horizon r_+ = M + sqrt(M^2 - a^2)."""
    return M + math.sqrt(M * M - a * a)


def make_grid(nr: int, nth: int, a: float, M: float = 1.0, r_out: float = 50.0,
              rin_factor: float = 0.9, r_in: float | None = None, guard: int = 2,
              pitch: int | None = None) -> Grid:
    """Log-r grid from r_in (default 0.9 r_+) to r_out, theta uniform on [0, pi]."""
    if r_in is None:
        r_in = rin_factor * horizon(a, M)
    lnr0 = math.log(r_in)
    dlnr = (math.log(r_out) - lnr0) / nr
    if pitch is None:
        pitch = nth + 1 + 2 * guard
    if pitch < nth + 1 + 2 * guard:
        raise ValueError("pitch too small")
    return Grid(a=float(a), M=float(M), nr=int(nr), nth=int(nth), guard=int(guard),
                pitch=int(pitch), lnr0=lnr0, dlnr=dlnr, dth=math.pi / nth)


# --------------------------------------------------------------------------
# Kerr-Schild spatial metric pieces needed to build inputs (App. A).
# --------------------------------------------------------------------------
def _ks_pieces(a, M, r, th):
    s, c = np.sin(th), np.cos(th)
    rho2 = r * r + a * a * c * c
    z = 2.0 * M * r / rho2
    delta = r * r + a * a - 2.0 * M * r
    sigma = (r * r + a * a) ** 2 - a * a * delta * s * s
    with np.errstate(divide="ignore", invalid="ignore"):     # gamma^phph is infinite on the axis
        h_pp = 1.0 / (rho2 * s * s)
    return dict(
        s=s, c=c, rho2=rho2, z=z,
        alpha=1.0 / np.sqrt(1.0 + z), beta=z / (1.0 + z),
        g_rr=1.0 + z, g_rp=-a * s * s * (1.0 + z), g_tt=rho2, g_pp=sigma * s * s / rho2,
        h_rr=(a * a + r * r) / rho2 - 2.0 * M * r / (rho2 + 2.0 * M * r),
        h_rp=a / rho2, h_tt=1.0 / rho2, h_pp=h_pp,
    )


def wald_point(a, M, B0, r, th):
    """Rotating Wald field at points: returns dict of D^i, B^i, E_i, A_t, A_ph.

    From the Boyer-Lindquist potential A_t = B0 (a M r (1+cos^2)/rho^2 - a),
    A_ph = B0/2 sin^2 (r^2 + a^2 - 2 M a^2 r (1+cos^2)/rho^2) (App. C), which
    keep their form in Kerr-Schild coordinates, plus A_r^KS obtained from the
    coordinate change.  B^i = curl A / sqrt(gamma), E_i = d_i A_t, written
    with sin(theta) cancelled analytically so the axis is regular.
    """
    r = np.asarray(r, dtype=np.float64)
    th = np.asarray(th, dtype=np.float64)
    k = _ks_pieces(a, M, r, th)
    s, c, rho2 = k["s"], k["c"], k["rho2"]
    rho4 = rho2 * rho2
    sqz = np.sqrt(1.0 + k["z"])
    K = r * r + a * a - 2.0 * M * a * a * r * (1.0 + c * c) / rho2
    dK_dr = 2.0 * r - 2.0 * M * a * a * (1.0 + c * c) * (rho2 - 2.0 * r * r) / rho4
    # sqrt(gamma) B^i with sqrt(gamma) = rho^2 sin sqrt(1+z); sin cancelled below.
    Br = B0 * c * (K + 2.0 * M * a * a * r * s * s * (r * r - a * a) / rho4) / (rho2 * sqz)
    Bth = -0.5 * B0 * s * dK_dr / (rho2 * sqz)
    Bph = -B0 * c * (2.0 * a * M * r * (a * a - r * r) / rho4 - a) / (rho2 * sqz)
    Er = B0 * a * M * (1.0 + c * c) * (a * a * c * c - r * r) / rho4
    Eth = B0 * 2.0 * a * M * r * (a * a - r * r) * s * c / rho4
    # sqrt(gamma) B^ph and sqrt(gamma) B^th / sin^2 for the D inversion
    sg_Bph = -B0 * s * c * (2.0 * a * M * r * (a * a - r * r) / rho4 - a)
    sg_Bth_over_s2 = -0.5 * B0 * dK_dr
    # Invert E_i = alpha gamma_ij D^j + e_ijk beta^j B^k (eq. E-H-B-D):
    # alpha gamma_ij D^j = (E_r, E_th + sqrt(g) beta B^ph, -sqrt(g) beta B^th)
    al, be = k["alpha"], k["beta"]
    Dr = (k["h_rr"] * Er + k["h_rp"] * (-be * sg_Bth_over_s2 * s * s)) / al
    Dth = k["h_tt"] * (Eth + be * sg_Bph) / al
    Dph = (k["h_rp"] * Er - be * sg_Bth_over_s2 / rho2) / al
    At = B0 * (a * M * r * (1.0 + c * c) / rho2 - a)
    Aph = 0.5 * B0 * s * s * K
    return dict(Dr=Dr, Dth=Dth, Dph=Dph, Br=Br, Bth=Bth, Bph=Bph, Er=Er, Eth=Eth,
                At=At, Aph=Aph)


def monopole_point(a, M, B0, r, th):
    """Vacuum monopole of App. C at points: dict of D^i, B^i, E_i, A_t, A_r, A_ph.

    From the Kerr-Schild potential A = B0 (a cos/rho^2, a cos/rho^2, 0,
    -cos (r^2 + a^2)/rho^2) (eq. for A_mu,monopole^KS; with the mass M
    written back in only sqrt(gamma) changes): B^r = d_th A_ph / sqrt(g),
    B^th = -d_r A_ph / sqrt(g), B^ph = -d_th A_r / sqrt(g), E_i = d_i A_t,
    written with sin(theta) cancelled so the axis is regular; D^i from E_i by
    inverting eq. E-H-B-D, as for the Wald field.
    """
    r = np.asarray(r, dtype=np.float64)
    th = np.asarray(th, dtype=np.float64)
    k = _ks_pieces(a, M, r, th)
    s, c, rho2 = k["s"], k["c"], k["rho2"]
    rho4 = rho2 * rho2
    sqz = np.sqrt(1.0 + k["z"])
    q = r * r - a * a * c * c
    # sqrt(gamma) B^i, sqrt(gamma) = rho^2 sin sqrt(1+z); sin cancelled in B^i
    Br = B0 * (a * a + r * r) * q / (rho4 * rho2 * sqz)
    Bth = -B0 * 2.0 * a * a * r * s * c / (rho4 * rho2 * sqz)
    Bph = B0 * a * q / (rho4 * rho2 * sqz)
    Er = -B0 * 2.0 * a * r * c / rho4
    Eth = -B0 * a * q * s / rho4
    sg_Bph = B0 * a * q * s / rho4
    sg_Bth_over_s2 = -B0 * 2.0 * a * a * r * c / rho4
    al, be = k["alpha"], k["beta"]
    Dr = (k["h_rr"] * Er + k["h_rp"] * (-be * sg_Bth_over_s2 * s * s)) / al
    Dth = k["h_tt"] * (Eth + be * sg_Bph) / al
    Dph = (k["h_rp"] * Er - be * sg_Bth_over_s2 / rho2) / al
    At = B0 * a * c / rho2
    Aph = -B0 * c * (r * r + a * a) / rho2
    return dict(Dr=Dr, Dth=Dth, Dph=Dph, Br=Br, Bth=Bth, Bph=Bph, Er=Er, Eth=Eth, At=At, Ar=At, Aph=Aph)


def monopole_fields(grid: Grid, B0: float = 1.0, axis_bc: bool = True) -> list[np.ndarray]:
    """The vacuum monopole (App. C) as the six field arrays on the Yee stagger."""
    return wald_fields(grid, B0, axis_bc, point=monopole_point)


def wald_fields(grid: Grid, B0: float = 1.0, axis_bc: bool = True, point=None) -> list[np.ndarray]:
    """The six field arrays D^r, D^th, D^ph, B^r, B^th, B^ph on the Yee stagger
    (of the rotating Wald field, or of the field that ``point`` gives)."""
    point = wald_point if point is None else point
    rows, pitch, g = grid.rows, grid.pitch, grid.guard
    ii = np.arange(rows, dtype=np.float64)[:, None] - g
    jj = np.arange(pitch, dtype=np.float64)[None, :] - g
    by_stagger = {}
    for name in FIELD_NAMES:
        by_stagger.setdefault(STAGGER[name], []).append(name)
    out = {}
    for (sr, st), names in by_stagger.items():
        r = grid.r(ii + sr) * np.ones_like(jj)
        th = grid.theta(jj + st) * np.ones_like(ii)
        vals = point(grid.a, grid.M, B0, r, th)
        for name in names:
            v = np.ascontiguousarray(vals[name], dtype=np.float64)
            if axis_bc and st == 0.0 and name in ("Dph", "Bth"):
                v[:, g] = 0.0                 # theta = 0
                v[:, g + grid.nth] = 0.0      # theta = pi
            out[name] = v
    return [out[name] for name in FIELD_NAMES]


def zero_fields(grid: Grid) -> list[np.ndarray]:
    return [np.zeros(grid.shape, dtype=np.float64) for _ in FIELD_NAMES]


def zero_currents(grid: Grid) -> list[np.ndarray]:
    return [np.zeros(grid.shape, dtype=np.float64) for _ in CURRENT_NAMES]


def crossing_time(grid: Grid) -> float:
    """Minimum over cell centres of the light crossing time of one cell.

    In grid units a cell has unit size; light moves at most
    |dxi/dt| <= (alpha sqrt(h^rr) + |beta^r|) / (r dlnr) and
    |deta/dt| <= alpha sqrt(h^thth) / dth.
    """
    xi = np.arange(grid.nr, dtype=np.float64) + 0.5
    eta = np.arange(grid.nth, dtype=np.float64) + 0.5
    r = grid.r(xi)[:, None]
    th = grid.theta(eta)[None, :]
    k = _ks_pieces(grid.a, grid.M, r, th)
    v_xi = (k["alpha"] * np.sqrt(k["h_rr"]) + np.abs(k["beta"])) / (r * grid.dlnr)
    v_eta = k["alpha"] * np.sqrt(k["h_tt"]) / grid.dth
    return float(np.min(1.0 / np.maximum(v_xi, v_eta)))


def crossing_dt(grid: Grid, frac: float = 0.5) -> float:
    return frac * crossing_time(grid)


# --------------------------------------------------------------------------
# Particle samplers
# --------------------------------------------------------------------------
def frame_to_covariant(a, M, r, th, uhat):
    """Map momenta in the orthonormal frame of gamma_ij to covariant u_i.

    u_i = L_i^a uhat_a with L L^T = gamma_ij (lower-triangular in (ph, th, r)):
    u_th = rho uhat_th, u_ph = sqrt(g_pp) uhat_ph,
    u_r = sqrt(g_rr - g_rp^2/g_pp) uhat_r + g_rp/sqrt(g_pp) uhat_ph,
    so gamma^ij u_i u_j = |uhat|^2.
    """
    k = _ks_pieces(a, M, r, th)
    sp = np.sqrt(k["g_pp"])
    ur = np.sqrt(k["g_rr"] - k["g_rp"] ** 2 / k["g_pp"]) * uhat[0] + k["g_rp"] / sp * uhat[2]
    uth = np.sqrt(k["rho2"]) * uhat[1]
    uph = sp * uhat[2]
    return ur, uth, uph


def _isotropic_dirs(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz])   # (r, th, ph) frame axes


_MJ_CACHE: dict = {}


def _mj_inverse_cdf(theta_T: float):
    """Tabulated inverse CDF of |u| for f(u) ~ u^2 exp(-sqrt(1+u^2)/T)."""
    if theta_T in _MJ_CACHE:
        return _MJ_CACHE[theta_T]
    umax = max(1.0, theta_T) * 60.0
    u = np.linspace(0.0, umax, 400001)
    logf = 2.0 * np.log(np.maximum(u, 1e-300)) - (np.sqrt(1.0 + u * u) - 1.0) / theta_T
    f = np.exp(logf - logf.max())
    f[0] = 0.0
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(u))])
    cdf /= cdf[-1]
    _MJ_CACHE[theta_T] = (cdf, u)
    return cdf, u


def _draw_momenta(kind, rng, n, params):
    """Momenta in the local orthonormal frame, shape (3, n)."""
    d = _isotropic_dirs(rng, n)
    if kind == "uniform":
        mag = rng.uniform(0.0, params.get("umax", 1.0), n)
        return d * mag
    if kind == "mj":
        cdf, ugrid = _mj_inverse_cdf(float(params["T"]))
        mag = np.interp(rng.uniform(0.0, 1.0, n), cdf, ugrid)
        uh = d * mag
        v = float(params.get("vphi", 0.0))
        if v != 0.0:    # Lorentz boost along e_(ph) with speed v
            G = 1.0 / math.sqrt(1.0 - v * v)
            gam = np.sqrt(1.0 + mag * mag)
            uh[2] = G * (uh[2] + v * gam)
        return uh
    if kind == "powerlaw":     # dN/dgamma ~ gamma^-2 on [1, gmax]
        gmax = float(params.get("gmax", 1e3))
        U = rng.uniform(0.0, 1.0, n)
        gam = 1.0 / (1.0 - U * (1.0 - 1.0 / gmax))
        return d * np.sqrt(np.maximum(gam * gam - 1.0, 0.0))
    raise ValueError(kind)


def _chunk(grid: Grid, seed: int, c: int, p0: int, p1: int, kind: str, params: dict):
    """Pairs p0..p1-1 (global pair index) of chunk c."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(c,))))
    m = p1 - p0
    k = np.arange(p0, p1, dtype=np.int64)
    cell = (k % grid.ncell).astype(np.int32)
    off = rng.uniform(0.0, 1.0, (2, m))
    ci, cj = cell // grid.nth, cell % grid.nth
    r = grid.r(ci + off[0])
    th = grid.theta(cj + off[1])
    out = {}
    for s in range(2):                      # e- then e+ momenta
        uh = _draw_momenta(kind, rng, m, params)
        out[s] = frame_to_covariant(grid.a, grid.M, r, th, uh)
    res = dict(cell=np.repeat(cell, 2), xr=np.repeat(off[0], 2), xth=np.repeat(off[1], 2))
    for key, comp in (("ur", 0), ("uth", 1), ("uph", 2)):
        v = np.empty(2 * m)
        v[0::2] = out[0][comp]
        v[1::2] = out[1][comp]
        res[key] = v
    res["w"] = np.ones(2 * m)
    res["sp"] = np.tile(np.array([0, 1], dtype=np.uint8), m)
    return res


def pairs(grid: Grid, npairs: int, kind: str = "uniform", seed: int = 0, params: dict | None = None,
          first_pair: int = 0, workers: int = 1, sink=None):
    """e+- pairs (2*npairs particles, e- at even, e+ at odd index).

    Pair k sits in cell k mod (nr*nth) at a uniform offset shared by the two
    particles; each particle draws its own momentum.  With ``sink`` given,
    each chunk is passed to sink(start_particle, arrays) instead of being
    concatenated (for workloads that do not fit comfortably in host memory).
    """
    params = dict(params or {})
    p_end = first_pair + npairs
    jobs = []
    c = first_pair // CHUNK_PAIRS
    while c * CHUNK_PAIRS < p_end:
        lo = max(c * CHUNK_PAIRS, first_pair)
        hi = min((c + 1) * CHUNK_PAIRS, p_end)
        jobs.append((c, lo, hi))
        c += 1

    def run(job):
        c, lo, hi = job
        # Chunks are always drawn whole so that any subset is reproducible.
        d = _chunk(grid, seed, c, c * CHUNK_PAIRS, (c + 1) * CHUNK_PAIRS, kind, params)
        a0 = 2 * (lo - c * CHUNK_PAIRS)
        a1 = 2 * (hi - c * CHUNK_PAIRS)
        return {k: v[a0:a1] for k, v in d.items()}, 2 * (lo - first_pair)

    if sink is not None:
        with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
            for arrs, start in ex.map(run, jobs):
                sink(start, arrs)
        return None
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        parts = list(ex.map(run, jobs))
    return {k: np.concatenate([p[0][k] for p in parts]) for k in parts[0][0]}


def qed_species_table():
    """Species of the monopole workload: 0 = e-, 1 = e+, 2 = photon."""
    return species_table() + [dict(q=0.0, m=0.0, massless=1)]


def qed_particles(grid: Grid, npairs: int, photon_frac: float = 0.2, seed: int = 0, gmax: float = 1e3,
                  eps_range=(1.0, 10.0), workers: int = 1):
    """Inputs of the monopole workload: e+- pairs with dN/dgamma ~ gamma^-2 on
    [1, gmax] (the pair recipe above), of which a fraction photon_frac of the
    pairs' e- slots are turned into photons with FIDO energy uniform in
    eps_range along an isotropic direction; uint64 tags 0 .. n-1."""
    parts = pairs(grid, npairs, kind="powerlaw", seed=seed, params=dict(gmax=gmax), workers=workers)
    n = len(parts["cell"])
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(1 << 30,))))
    ph = np.flatnonzero((rng.uniform(0.0, 1.0, npairs) < photon_frac)) * 2
    ci, cj = parts["cell"][ph] // grid.nth, parts["cell"][ph] % grid.nth
    r = grid.r(ci + parts["xr"][ph])
    th = grid.theta(cj + parts["xth"][ph])
    eps = rng.uniform(eps_range[0], eps_range[1], len(ph))
    uh = _isotropic_dirs(rng, len(ph)) * eps
    ur, uth, uph = frame_to_covariant(grid.a, grid.M, r, th, uh)
    parts["ur"][ph], parts["uth"][ph], parts["uph"][ph] = ur, uth, uph
    parts["sp"][ph] = 2
    parts["tag"] = np.arange(n, dtype=np.uint64)
    return parts


def species_table():
    """(q, m) rows for the species indices used by ``pairs``: 0 = e-, 1 = e+."""
    return [dict(q=q, m=m, massless=0) for q, m in SPECIES_PAIRS]
