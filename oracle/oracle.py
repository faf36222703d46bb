"""ctypes front end of the FP64 CPU oracle in grpic_oracle.cpp.

TEST INFRASTRUCTURE ONLY: the plain, slow reference that the HIP library is
checked against.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark import this module; the library never does.  It imports
nothing from the HIP package: grids are duck-typed (any object with the
attributes a, M, nr, nth, guard, pitch, lnr0, dlnr, dth works).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "grpic_oracle.cpp")
SO = os.path.join(_HERE, "libgrpic_oracle.so")

_c_double_p = ctypes.POINTER(ctypes.c_double)


class Geom(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("M", ctypes.c_double),
                ("nr", ctypes.c_int32), ("nth", ctypes.c_int32),
                ("guard", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("lnr0", ctypes.c_double), ("dlnr", ctypes.c_double), ("dth", ctypes.c_double)]


class Species(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("m", ctypes.c_double),
                ("massless", ctypes.c_int32), ("pad", ctypes.c_int32)]


def build() -> str:
    """Compile the oracle (g++, no FMA contraction, OpenMP for timing mode)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
           SRC, "-o", SO + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(SO + ".tmp", SO)
    return SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            build()
        _lib = ctypes.CDLL(SO)
    return _lib


def geom(grid) -> Geom:
    return Geom(float(grid.a), float(grid.M), int(grid.nr), int(grid.nth), int(grid.guard),
                int(grid.pitch), float(grid.lnr0), float(grid.dlnr), float(grid.dth))


def _p(x: np.ndarray):
    return x.ctypes.data_as(ctypes.c_void_p)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


METRIC_KEYS = ("alpha", "beta", "g_rr", "g_rph", "g_thth", "g_phph",
               "h_rr", "h_rph", "h_thth", "h_phph", "sqrtg")
METRIC_DKEYS = ("alpha", "beta", "h_rr", "h_rph", "h_thth", "h_phph")


def metric(a: float, M: float, r: float, th: float) -> dict:
    out = np.zeros(23)
    lib().orc_metric(ctypes.c_double(a), ctypes.c_double(M), ctypes.c_double(r),
                     ctypes.c_double(th), _p(out))
    d = {k: out[i] for i, k in enumerate(METRIC_KEYS)}
    for q, k in enumerate(METRIC_DKEYS):
        d["dr_" + k] = out[11 + 2 * q]
        d["dth_" + k] = out[12 + 2 * q]
    return d


def rhs(grid, y, eps: float = 1.0) -> np.ndarray:
    g = geom(grid)
    y = _f64(y)
    f = np.zeros(6)
    lib().orc_rhs(ctypes.byref(g), ctypes.c_double(eps), _p(y), _p(f))
    return f


def boris(grid, qm, dt, xi, eta, u, D, B) -> np.ndarray:
    g = geom(grid)
    u, D, B = _f64(u), _f64(D), _f64(B)
    out = np.zeros(3)
    lib().orc_boris(ctypes.byref(g), ctypes.c_double(qm), ctypes.c_double(dt), ctypes.c_double(xi),
                    ctypes.c_double(eta), _p(u), _p(D), _p(B), _p(out))
    return out


def vay(grid, qm, dt, xi, eta, u, D, B) -> np.ndarray:
    """Vay's momentum update in the FIDO frame (the alternative kick)."""
    g = geom(grid)
    u, D, B = _f64(u), _f64(D), _f64(B)
    out = np.zeros(3)
    lib().orc_vay(ctypes.byref(g), ctypes.c_double(qm), ctypes.c_double(dt), ctypes.c_double(xi),
                  ctypes.c_double(eta), _p(u), _p(D), _p(B), _p(out))
    return out


KICKS = {"boris": 0, "vay": 1}


def push_point(grid, q, m, dt, xi, eta, u, D, B, ncorr: int = 3, massless: bool = False,
               kick: str = "boris") -> np.ndarray:
    """Kick with point fields D, B at x^n, then the geodesic PC (no boundaries).

    Returns y1 = (xi, eta, dphi, u_r, u_th, u_ph)."""
    g = geom(grid)
    sp = Species(float(q), float(m), int(massless), 0)
    u, D, B = _f64(u), _f64(D), _f64(B)
    y1 = np.zeros(6)
    lib().orc_push_point(ctypes.byref(g), ctypes.byref(sp), ctypes.c_double(dt), ctypes.c_int(ncorr),
                         ctypes.c_double(xi), ctypes.c_double(eta), _p(u), _p(D), _p(B), _p(y1),
                         ctypes.c_int(KICKS[kick]))
    return y1


def gather(grid, fields, xi, eta) -> np.ndarray:
    g = geom(grid)
    fl = [_f64(f) for f in fields]
    ptrs = (ctypes.c_void_p * 6)(*[f.ctypes.data for f in fl])
    out = np.zeros(6)
    lib().orc_gather(ctypes.byref(g), ptrs, ctypes.c_double(xi), ctypes.c_double(eta), _p(out))
    return out


def deposit_move(grid, qw, dt, xi0, eta0, xi1, eta1, dphi, J=None):
    """Deposit of one move; returns (Fr, Fth, Gph) arrays (added to J if given)."""
    g = geom(grid)
    if J is None:
        J = [np.zeros((grid.nr + 1 + 2 * grid.guard, grid.pitch)) for _ in range(3)]
    lib().orc_deposit_move(ctypes.byref(g), ctypes.c_double(qw), ctypes.c_double(dt),
                           ctypes.c_double(xi0), ctypes.c_double(eta0), ctypes.c_double(xi1),
                           ctypes.c_double(eta1), ctypes.c_double(dphi), _p(J[0]), _p(J[1]), _p(J[2]))
    return J


def gather3(grid, fields, xi, eta) -> np.ndarray:
    """The six components at (xi, eta) with the cubic spline shape."""
    g = geom(grid)
    fl = [_f64(f) for f in fields]
    ptrs = (ctypes.c_void_p * 6)(*[f.ctypes.data for f in fl])
    out = np.zeros(6)
    lib().orc_gather3(ctypes.byref(g), ptrs, ctypes.c_double(xi), ctypes.c_double(eta), _p(out))
    return out


def deposit_move3(grid, qw, dt, xi0, eta0, xi1, eta1, dphi, J=None):
    """Deposit of one move with the cubic shape, folded across the axes."""
    g = geom(grid)
    if J is None:
        J = [np.zeros((grid.nr + 1 + 2 * grid.guard, grid.pitch)) for _ in range(3)]
    lib().orc_deposit_move3(ctypes.byref(g), ctypes.c_double(qw), ctypes.c_double(dt),
                            ctypes.c_double(xi0), ctypes.c_double(eta0), ctypes.c_double(xi1),
                            ctypes.c_double(eta1), ctypes.c_double(dphi), _p(J[0]), _p(J[1]), _p(J[2]))
    return J


def charge3(grid, species, parts) -> np.ndarray:
    """Q with the cubic spline shape, folded across the axes."""
    g = geom(grid)
    sp = _species_array(species)
    cell = np.ascontiguousarray(parts["cell"], dtype=np.int32)
    xr, xth, w = _f64(parts["xr"]), _f64(parts["xth"]), _f64(parts["w"])
    spi = np.ascontiguousarray(parts["sp"], dtype=np.uint8)
    Q = np.zeros((grid.nr + 1 + 2 * grid.guard, grid.pitch))
    lib().orc_charge3(ctypes.byref(g), sp, ctypes.c_int(len(species)), ctypes.c_int64(len(cell)),
                      _p(cell), _p(xr), _p(xth), _p(w), _p(spi), _p(Q))
    return Q


def _species_array(species):
    arr = (Species * len(species))()
    for i, s in enumerate(species):
        arr[i] = Species(float(s["q"]), float(s["m"]), int(s.get("massless", 0)), 0)
    return arr


def charge(grid, species, parts) -> np.ndarray:
    """Q_ij = sum over live particles of q w S_ij(x_p)."""
    g = geom(grid)
    sp = _species_array(species)
    cell = np.ascontiguousarray(parts["cell"], dtype=np.int32)
    xr, xth, w = _f64(parts["xr"]), _f64(parts["xth"]), _f64(parts["w"])
    spi = np.ascontiguousarray(parts["sp"], dtype=np.uint8)
    Q = np.zeros((grid.nr + 1 + 2 * grid.guard, grid.pitch))
    lib().orc_charge(ctypes.byref(g), sp, ctypes.c_int(len(species)), ctypes.c_int64(len(cell)),
                     _p(cell), _p(xr), _p(xth), _p(w), _p(spi), _p(Q))
    return Q


PARTICLE_KEYS = ("cell", "xr", "xth", "ur", "uth", "uph", "w", "sp")


def run(grid, species, parts, fields, dt, nsteps, ncorr: int = 3, nthreads: int = 1,
        with_abs: bool = False, track_phi: bool = False, J=None, kick: str = "boris", order: int = 1):
    """Advance copies of the particle arrays nsteps steps.

    Returns (parts_out, J, A, stats): J = [Fr, Fth, Gph] (added to the given
    J if any); A (with_abs, serial only) = per element, the sum over the
    contributions of their magnitude scale, |q w|/dt for F^r and F^th and
    |q w dphi|/dt for G^ph; stats = dict(out, bad, reflected, live_steps).
    kick: "boris" (the generalised Boris kick) or "vay" (Vay's update in the
    FIDO frame).  order: 1 (CIC) or 3 (the cubic spline shape for gather and
    deposit, folded across the axes; the grid needs guard >= 3).
    """
    if order not in (1, 3):
        raise ValueError(f"order: expected 1 or 3, got {order}")
    if order == 3 and grid.guard < 3:
        raise ValueError("the cubic shape needs guard >= 3")
    g = geom(grid)
    sp = _species_array(species)
    p = {
        "cell": np.array(parts["cell"], dtype=np.int32, copy=True),
        "xr": np.array(parts["xr"], dtype=np.float64, copy=True),
        "xth": np.array(parts["xth"], dtype=np.float64, copy=True),
        "ur": np.array(parts["ur"], dtype=np.float64, copy=True),
        "uth": np.array(parts["uth"], dtype=np.float64, copy=True),
        "uph": np.array(parts["uph"], dtype=np.float64, copy=True),
        "w": _f64(parts["w"]),
        "sp": np.ascontiguousarray(parts["sp"], dtype=np.uint8),
    }
    n = len(p["cell"])
    if track_phi:
        p["phi"] = np.array(parts.get("phi", np.zeros(n)), dtype=np.float64, copy=True)
    shape = (grid.nr + 1 + 2 * grid.guard, grid.pitch)
    if J is None:
        J = [np.zeros(shape) for _ in range(3)]
    A = [np.zeros(shape) for _ in range(3)] if with_abs else None
    fl = [_f64(f) for f in fields]
    fptr = (ctypes.c_void_p * 6)(*[f.ctypes.data for f in fl])
    stats = np.zeros(4, dtype=np.int64)
    null = ctypes.c_void_p(0)
    lib().orc_run(ctypes.byref(g), sp, ctypes.c_int(len(species)), ctypes.c_int64(n),
                  _p(p["cell"]), _p(p["xr"]), _p(p["xth"]), _p(p["ur"]), _p(p["uth"]), _p(p["uph"]),
                  _p(p["w"]), _p(p["sp"]), _p(p["phi"]) if track_phi else null,
                  fptr, _p(J[0]), _p(J[1]), _p(J[2]),
                  _p(A[0]) if A else null, _p(A[1]) if A else null, _p(A[2]) if A else null,
                  ctypes.c_double(dt), ctypes.c_int(nsteps), ctypes.c_int(ncorr),
                  ctypes.c_int(nthreads), _p(stats), ctypes.c_int(KICKS[kick]), ctypes.c_int(order))
    st = dict(out=int(stats[0]), bad=int(stats[1]), reflected=int(stats[2]), live_steps=int(stats[3]))
    return p, J, A, st


def philox(counter, key) -> np.ndarray:
    """Philox4x64-10 of one 4-word counter under a 2-word key (uint64)."""
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint64))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox(_p(c), _p(k), _p(out))
    return out


class Qed(ctypes.Structure):
    _fields_ = [("gamma_thr", ctypes.c_double), ("eps_ph", ctypes.c_double), ("tau", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("electron_sp", ctypes.c_int32), ("positron_sp", ctypes.c_int32),
                ("photon_sp", ctypes.c_int32), ("pad", ctypes.c_int32)]


def run_qed(grid, species, parts, fields, dt, step, qed: dict, ncorr: int = 3, capacity=None, J=None):
    """One step of photon emission and pair conversion around the push
    (serial).  parts needs a uint64 "tag" array.  qed: gamma_thr, eps_ph,
    tau, seed, electron_sp, positron_sp, photon_sp.  Returns (parts_out, J,
    A, created, stats, qstats): created holds the new particles in creation
    order; stats as in run; qstats = dict(emitted, converted, lost)."""
    g = geom(grid)
    sp = _species_array(species)
    p = {
        "cell": np.array(parts["cell"], dtype=np.int32, copy=True),
        "xr": np.array(parts["xr"], dtype=np.float64, copy=True),
        "xth": np.array(parts["xth"], dtype=np.float64, copy=True),
        "ur": np.array(parts["ur"], dtype=np.float64, copy=True),
        "uth": np.array(parts["uth"], dtype=np.float64, copy=True),
        "uph": np.array(parts["uph"], dtype=np.float64, copy=True),
        "w": np.array(parts["w"], dtype=np.float64, copy=True),
        "sp": np.array(parts["sp"], dtype=np.uint8, copy=True),
        "tag": np.array(parts["tag"], dtype=np.uint64, copy=True),
    }
    n = len(p["cell"])
    cap = 2 * n if capacity is None else int(capacity)
    c = {"cell": np.full(cap, -1, dtype=np.int32), "sp": np.zeros(cap, dtype=np.uint8),
         "tag": np.zeros(cap, dtype=np.uint64)}
    for k in ("xr", "xth", "ur", "uth", "uph", "w"):
        c[k] = np.zeros(cap)
    shape = (grid.nr + 1 + 2 * grid.guard, grid.pitch)
    if J is None:
        J = [np.zeros(shape) for _ in range(3)]
    A = [np.zeros(shape) for _ in range(3)]
    fl = [_f64(f) for f in fields]
    fptr = (ctypes.c_void_p * 6)(*[f.ctypes.data for f in fl])
    q = Qed(float(qed["gamma_thr"]), float(qed["eps_ph"]), float(qed["tau"]), int(qed["seed"]),
            int(qed["electron_sp"]), int(qed["positron_sp"]), int(qed["photon_sp"]), 0)
    nc = ctypes.c_int64(0)
    stats = np.zeros(4, dtype=np.int64)
    qstats = np.zeros(3, dtype=np.int64)
    lib().orc_run_qed(ctypes.byref(g), sp, ctypes.c_int(len(species)), ctypes.c_int64(n),
                      _p(p["cell"]), _p(p["xr"]), _p(p["xth"]), _p(p["ur"]), _p(p["uth"]), _p(p["uph"]),
                      _p(p["w"]), _p(p["sp"]), _p(p["tag"]), fptr, _p(J[0]), _p(J[1]), _p(J[2]),
                      _p(A[0]), _p(A[1]), _p(A[2]), ctypes.c_double(dt), ctypes.c_int(ncorr),
                      ctypes.c_int64(int(step)), ctypes.byref(q), ctypes.c_int64(cap),
                      _p(c["cell"]), _p(c["xr"]), _p(c["xth"]), _p(c["ur"]), _p(c["uth"]), _p(c["uph"]),
                      _p(c["w"]), _p(c["sp"]), _p(c["tag"]), ctypes.byref(nc), _p(stats), _p(qstats))
    created = {k: v[: nc.value] for k, v in c.items()}
    st = dict(out=int(stats[0]), bad=int(stats[1]), reflected=int(stats[2]), live_steps=int(stats[3]))
    qs = dict(emitted=int(qstats[0]), converted=int(qstats[1]), lost=int(qstats[2]))
    return p, J, A, created, st, qs


def has_openmp() -> bool:
    return bool(lib().orc_has_openmp())


OP_NAMES = ("add", "mul", "div", "sqrt", "exp", "sin", "cos")


def count_ops(grid, species, parts, fields, dt, ncorr: int = 3, sample=None) -> dict:
    """Mean floating-point operation counts of one particle-step (gather,
    push, deposit) over the live particles listed in `sample` (default all),
    from the oracle run on a counting scalar type."""
    g = geom(grid)
    sp = _species_array(species)
    fl = [_f64(f) for f in fields]
    fptr = (ctypes.c_void_p * 6)(*[f.ctypes.data for f in fl])
    out = np.zeros(7, dtype=np.int64)
    n = 0
    idx = range(len(parts["cell"])) if sample is None else sample
    for p in idx:
        c = int(parts["cell"][p])
        if c < 0:
            continue
        xi = c // grid.nth + float(parts["xr"][p])
        eta = c % grid.nth + float(parts["xth"][p])
        u = np.array([parts["ur"][p], parts["uth"][p], parts["uph"][p]], dtype=np.float64)
        lib().orc_count_ops(ctypes.byref(g), ctypes.byref(sp[int(parts["sp"][p])]), fptr,
                            ctypes.c_double(float(parts["w"][p])), ctypes.c_double(dt), ctypes.c_int(ncorr),
                            ctypes.c_double(xi), ctypes.c_double(eta), _p(u), _p(out))
        n += 1
    d = {k: float(v) / max(n, 1) for k, v in zip(OP_NAMES, out)}
    d["total"] = sum(d[k] for k in OP_NAMES)
    d["particles"] = n
    return d


def _ptrs(arrs):
    if arrs is None:
        return None
    keep = [None if a is None else _f64(a) for a in arrs]
    ptr = (ctypes.c_void_p * len(keep))(*[0 if a is None else a.ctypes.data for a in keep])
    return ptr, keep


def loss_dual(grid, species, parts, fields, lam, dt, nsteps, ncorr: int = 3, tu=None, tF=None):
    """L = sum over particles and steps of lambda . (F^r, F^th, G^ph) and its
    derivative along the direction (tu = (t_ur, t_uth, t_uph) per particle,
    tF = six field tangent arrays), by forward-mode dual numbers through the
    oracle.  Returns (L, dL, status per particle)."""
    g = geom(grid)
    sp = _species_array(species)
    n = len(parts["cell"])
    cell = np.ascontiguousarray(parts["cell"], dtype=np.int32)
    arrs = {k: _f64(parts[k]) for k in ("xr", "xth", "ur", "uth", "uph", "w")}
    spi = np.ascontiguousarray(parts["sp"], dtype=np.uint8)
    tus = [None, None, None] if tu is None else [_f64(t) for t in tu]
    F, keepF = _ptrs(fields)
    tFp = _ptrs(tF)
    L, keepL = _ptrs(lam)
    out = np.zeros(2)
    status = np.zeros(n, dtype=np.int32)
    null = ctypes.c_void_p(0)
    lib().orc_loss_dual(ctypes.byref(g), sp, ctypes.c_int(len(species)), ctypes.c_int64(n), _p(cell),
                        _p(arrs["xr"]), _p(arrs["xth"]), _p(arrs["ur"]), _p(arrs["uth"]), _p(arrs["uph"]),
                        _p(arrs["w"]), _p(spi), *[null if t is None else _p(t) for t in tus],
                        F, tFp[0] if tFp else null, L, ctypes.c_double(dt), ctypes.c_int(nsteps),
                        ctypes.c_int(ncorr), _p(out), _p(status))
    return float(out[0]), float(out[1]), status


def loss_dual_steps(grid, species, parts, field_steps, lam, dt, ncorr: int = 3, tu=None):
    """loss_dual over the steps of field_steps, whose fields change from step
    to step: field_steps[k] holds the six arrays step k gathers from, or
    field_steps is one float64 array of shape (6, nsteps, rows, pitch)
    (inputs; the derivative is along tu only).  Returns (L, dL, status per
    particle)."""
    g = geom(grid)
    sp = _species_array(species)
    n = len(parts["cell"])
    shape = (grid.nr + 1 + 2 * grid.guard, grid.pitch)
    if isinstance(field_steps, np.ndarray):
        if field_steps.ndim != 4 or field_steps.shape[0] != 6 or field_steps.shape[2:] != shape:
            raise ValueError("field_steps: expected shape (6, nsteps, rows, pitch)")
        nsteps = field_steps.shape[1]
        stacked = [np.ascontiguousarray(field_steps[c], dtype=np.float64) for c in range(6)]
    else:
        nsteps = len(field_steps)
        stacked = [np.ascontiguousarray(np.stack([np.asarray(fs[c], dtype=np.float64).reshape(shape)
                                                  for fs in field_steps])) for c in range(6)]
    fptr = (ctypes.c_void_p * 6)(*[a.ctypes.data for a in stacked])
    cell = np.ascontiguousarray(parts["cell"], dtype=np.int32)
    arrs = {k: _f64(parts[k]) for k in ("xr", "xth", "ur", "uth", "uph", "w")}
    spi = np.ascontiguousarray(parts["sp"], dtype=np.uint8)
    tus = [None, None, None] if tu is None else [_f64(t) for t in tu]
    L, keepL = _ptrs(lam)
    out = np.zeros(2)
    status = np.zeros(n, dtype=np.int32)
    null = ctypes.c_void_p(0)
    lib().orc_loss_dual_steps(ctypes.byref(g), sp, ctypes.c_int(len(species)), ctypes.c_int64(n), _p(cell),
                              _p(arrs["xr"]), _p(arrs["xth"]), _p(arrs["ur"]), _p(arrs["uth"]), _p(arrs["uph"]),
                              _p(arrs["w"]), _p(spi), *[null if t is None else _p(t) for t in tus],
                              fptr, null, ctypes.c_long(shape[0] * shape[1]), L, ctypes.c_double(dt),
                              ctypes.c_int(nsteps), ctypes.c_int(ncorr), _p(out), _p(status))
    return float(out[0]), float(out[1]), status


def loss_particle(grid, species_row, xi, eta, u, w, fields, lam, dt, nsteps, ncorr: int = 3, trajectory=False):
    """L of one particle on plain doubles; returns (L, status) or, with
    trajectory, (L, status, positions (nsteps + 1, 2), nan after removal)."""
    g = geom(grid)
    sp = _species_array([species_row])
    F, keepF = _ptrs(fields)
    L, keepL = _ptrs(lam)
    u = _f64(u)
    out = ctypes.c_double(0.0)
    traj = np.full((nsteps + 1, 2), np.nan) if trajectory else None
    lib().orc_loss_particle.restype = ctypes.c_int
    st = lib().orc_loss_particle(ctypes.byref(g), sp, ctypes.c_double(xi), ctypes.c_double(eta), _p(u),
                                 ctypes.c_double(w), F, L, ctypes.c_double(dt), ctypes.c_int(nsteps),
                                 ctypes.c_int(ncorr), ctypes.byref(out),
                                 _p(traj) if trajectory else ctypes.c_void_p(0))
    if trajectory:
        return float(out.value), int(st), traj
    return float(out.value), int(st)


# ---------------------------------------------------------------- field solver

FIELD_KEYS = ("Dr", "Dth", "Dph", "Br", "Bth", "Bph")


def _grid_arrays(grid, arrays):
    shape = (grid.nr + 1 + 2 * grid.guard, grid.pitch)
    out = [np.ascontiguousarray(np.array(a, dtype=np.float64)).reshape(shape) for a in arrays]
    return out, shape


def _field_ptrs(arrays):
    return (ctypes.c_void_p * len(arrays))(*[_p(a) for a in arrays])


def field_areas(grid) -> list:
    """Area elements per unit phi at the locations of D^r, D^th, D^ph,
    B^r, B^th, B^ph (10-point Gauss quadrature of sqrt(gamma))."""
    shape = (grid.nr + 1 + 2 * grid.guard, grid.pitch)
    A = [np.zeros(shape) for _ in range(6)]
    lib().orc_field_areas(ctypes.byref(geom(grid)), _field_ptrs(A))
    return A


def field_circulations(grid, X) -> list:
    """C_H for D^r, D^th, D^ph and C_E for B^r, B^th, B^ph of the state X
    (six grid arrays; guard rows are filled from it first)."""
    Xs, shape = _grid_arrays(grid, X)
    C = [np.zeros(shape) for _ in range(6)]
    lib().orc_field_circulations(ctypes.byref(geom(grid)), _field_ptrs(Xs), _field_ptrs(C))
    return C


def field_step(grid, X, F=None, dt=0.0, w1=0.53, ncorr=7, damp_cells=0, damp_max=0.0) -> list:
    """One field step (predictor + ncorr correctors, weights 1 - w1, w1) of
    the state X with the flux-form currents F (three grid arrays or None);
    returns the new state (six arrays)."""
    Xs, shape = _grid_arrays(grid, X)
    Fs = None
    if F is not None:
        Fs, _ = _grid_arrays(grid, F)
    lib().orc_field_step(ctypes.byref(geom(grid)), _field_ptrs(Xs), _field_ptrs(Fs) if Fs is not None else None,
                         ctypes.c_double(dt), ctypes.c_double(w1), ctypes.c_int(ncorr), ctypes.c_int(damp_cells),
                         ctypes.c_double(damp_max))
    return Xs
