"""FP64 CPU oracle for the explicit APIC-MPM step (arXiv 1603.06188).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  The product path (the
HIP library under ``paper_1603_06188_amd/``) never imports, links or calls it,
and the two share no code.

The arithmetic lives in ``apic_oracle.c`` (plain C, binary64, no FMA
contraction); this module only marshals NumPy arrays to it.  Every function
cites the passage of the paper it follows:

* ``bspline`` / ``weights``             -- interpolation weights, Sec. 3.5
* ``neo_hookean_psi`` / ``neo_hookean_P`` -- energy density and first
  Piola-Kirchhoff stress of Sec. 3.1 (the neo-Hookean form is a reading: the
  paper names the model in Sec. 6 without writing it)
* ``p2g``                              -- transfer to grid, Sec. 3.2, plus the
  force of Sec. 3.3 at F^{n+lambda} = F^n (lambda = 0); ``transfer`` selects
  APIC, RPIC (Sec. 2.1) or PIC, the three cases of Sec. 5.6
* ``grid_update``                      -- grid evolution of Sec. 3.3, lambda = 0
* ``g2p``                              -- transfer to particles, Sec. 3.4 (RPIC:
  Sec. 2.1 with K_p and l_p as in Sec. 5.1; PIC: no affine part)
* ``particle_totals`` / ``grid_totals`` -- momenta of Sec. 3.1 with the
  particle angular momentum of Sec. 5.3 (B term included)
* ``cfl_dt``                           -- CFL rule of Sec. 4.3
* degree 1 everywhere: multilinear weights with the lagged C_p of Sec. 5.9
  (the B planes carry C_p), APIC transfer only
* ``neo_hookean_dP`` / ``forces_at`` / ``force_differential`` -- the stress
  differential and the force and force-derivative product of Sec. 3.3 with
  the nodes displaced
* ``midpoint_step``                    -- the implicit midpoint member
  (lambda = 1/2) of Sec. 3.3, solved as the minimization of Sec. 4.1 by
  Newton's method with the mass-inner-product conjugate gradient of Sec. 4.2
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "apic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OR_OK = 0
OR_E_ARG = -1
OR_E_DOMAIN = -2
OR_E_SINGULAR = -3
OR_E_INVERTED = -4

# transfer variants of Sec. 5.6: the affine part C_p is full, skew or zero
TRANSFER_APIC = 0
TRANSFER_RPIC = 1
TRANSFER_PIC = 2

_ERRORS = {
    OR_E_ARG: "invalid argument",
    OR_E_DOMAIN: "particle kernel support leaves the grid",
    OR_E_SINGULAR: "singular matrix",
    OR_E_INVERTED: "inverted element (det F <= 0)",
}


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (binary64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
             "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        G = ctypes.POINTER(_Grid)
        lib.oracle_bspline.restype = ctypes.c_double
        lib.oracle_bspline.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.oracle_bspline_deriv.restype = ctypes.c_double
        lib.oracle_bspline_deriv.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.oracle_weights.restype = ctypes.c_int
        lib.oracle_weights.argtypes = [G, _dp, _lp, _dp, _dp]
        lib.oracle_neo_hookean_psi.restype = ctypes.c_int
        lib.oracle_neo_hookean_psi.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp]
        lib.oracle_neo_hookean_P.restype = ctypes.c_int
        lib.oracle_neo_hookean_P.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp]
        lib.oracle_p2g.restype = ctypes.c_int
        lib.oracle_p2g.argtypes = [G, ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp, _dp]
        lib.oracle_grid_update.restype = ctypes.c_int
        lib.oracle_grid_update.argtypes = [G, _dp, _dp, _dp, ctypes.c_double, _dp, _ip, _dp, _dp, _dp]
        lib.oracle_g2p.restype = ctypes.c_int
        lib.oracle_g2p.argtypes = [G, ctypes.c_int64, _dp, _dp, _dp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp]
        lib.oracle_particle_totals.restype = None
        lib.oracle_particle_totals.argtypes = [ctypes.c_int, ctypes.c_int64, _dp, _dp, _dp, _dp, _dp]
        lib.oracle_grid_totals.restype = None
        lib.oracle_grid_totals.argtypes = [G, _dp, _dp, _dp, _dp]
        lib.oracle_potential.restype = ctypes.c_int
        lib.oracle_potential.argtypes = [ctypes.c_int, ctypes.c_int64, _dp, _dp, ctypes.c_double,
                                         ctypes.c_double, _dp]
        lib.oracle_cfl_dt.restype = ctypes.c_double
        lib.oracle_cfl_dt.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                      _dp, _dp]
        lib.oracle_cfl_dt_lagged.restype = ctypes.c_double
        lib.oracle_cfl_dt_lagged.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                             _dp, _dp]
        lib.oracle_neo_hookean_dP.restype = ctypes.c_int
        lib.oracle_neo_hookean_dP.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp, _dp]
        lib.oracle_forces_at.restype = ctypes.c_int
        lib.oracle_forces_at.argtypes = [G, ctypes.c_int64, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                         _dp, _dp, _dp]
        lib.oracle_force_differential.restype = ctypes.c_int
        lib.oracle_force_differential.argtypes = [G, ctypes.c_int64, _dp, _dp, _dp, ctypes.c_double,
                                                  ctypes.c_double, _dp, _dp, _dp]
        lib.oracle_node_in_band.restype = ctypes.c_int
        lib.oracle_node_in_band.argtypes = [G, _ip, _ip]
        lib.oracle_node_count.restype = ctypes.c_int64
        lib.oracle_node_count.argtypes = [G]
        lib.oracle_matrix_det.restype = ctypes.c_double
        lib.oracle_matrix_det.argtypes = [ctypes.c_int, _dp]
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_get_threads.restype = ctypes.c_int
        lib.oracle_get_threads.argtypes = []
        _lib = lib
    return _lib


def _check(rc: int) -> None:
    if rc != OR_OK:
        raise OracleError(_ERRORS.get(rc, f"oracle error {rc}"))


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


class Grid:
    """Uniform grid with ``cells[a]`` cells (``cells[a] + 1`` nodes) per axis,
    spacing ``dx``, origin 0 (Sec. 3.3: fixed Cartesian grid)."""

    def __init__(self, dim: int, degree: int, cells, dx: float):
        self.dim = int(dim)
        self.degree = int(degree)
        c = list(cells) + [0] * (3 - len(cells))
        self.cells = tuple(int(v) for v in c[: self.dim])
        self.dx = float(dx)
        self._s = _Grid(self.dim, self.degree, (ctypes.c_int32 * 3)(*[int(v) for v in c[:3]]), self.dx)

    @property
    def nodes(self):
        return tuple(c + 1 for c in self.cells)

    @property
    def node_count(self) -> int:
        return int(np.prod(self.nodes))

    def node_positions(self) -> np.ndarray:
        """Node positions x_i, node-major in the oracle's linear order."""
        axes = [np.arange(n, dtype=np.float64) * self.dx for n in self.nodes]
        mesh = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
        return np.stack([m.reshape(-1) for m in mesh], axis=1)

    def ref(self):
        return ctypes.byref(self._s)


def set_threads(n: int) -> None:
    """Threads of the transfers (1, the default, is the serial checker the
    tests use; more split the particles into blocks, for the CPU baseline)."""
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def bspline(degree: int, t: float) -> float:
    return _load().oracle_bspline(int(degree), float(t))


def bspline_deriv(degree: int, t: float) -> float:
    return _load().oracle_bspline_deriv(int(degree), float(t))


def weights(grid: Grid, xp):
    """Support of one particle: (node indices, w_ip, grad w_ip)."""
    xp = _d(xp)
    nodes = np.zeros(125, dtype=np.int64)
    w = np.zeros(125)
    gw = np.zeros(125 * grid.dim)
    m = _load().oracle_weights(grid.ref(), _ptr(xp), nodes.ctypes.data_as(_lp), _ptr(w), _ptr(gw))
    if m < 0:
        _check(m)
    return nodes[:m].copy(), w[:m].copy(), gw[: m * grid.dim].reshape(m, grid.dim).copy()


def neo_hookean_psi(F, mu: float, lam: float) -> float:
    F = _d(F)
    d = F.shape[0]
    out = ctypes.c_double()
    _check(_load().oracle_neo_hookean_psi(d, _ptr(F), mu, lam, ctypes.byref(out)))
    return out.value


def neo_hookean_P(F, mu: float, lam: float) -> np.ndarray:
    F = _d(F)
    d = F.shape[0]
    P = np.zeros((d, d))
    _check(_load().oracle_neo_hookean_P(d, _ptr(F), mu, lam, _ptr(P)))
    return P


def det(A) -> float:
    A = _d(A)
    return _load().oracle_matrix_det(A.shape[0], _ptr(A))


def p2g(grid: Grid, x, v, B, F, m, V, model: int = 0, mu: float = 0.0, lam: float = 0.0,
        want_D: bool = False, *, transfer: int = TRANSFER_APIC):
    """Transfer to grid (Sec. 3.2) plus the force f_i of Sec. 3.3 (model 1).
    ``transfer`` selects C_p = B_p D_p^{-1} (APIC), its rotation (RPIC) or
    zero (PIC), Sec. 5.6.

    Returns dict with node-major ``m`` (nodes), ``mv`` (nodes, d), ``f``
    (nodes, d) and optionally ``D`` (np, d, d)."""
    d = grid.dim
    x, v, B, F, m, V = (_d(a) for a in (x, v, B, F, m, V))
    npart = x.shape[0]
    nn = grid.node_count
    gm = np.zeros(nn)
    gmv = np.zeros((nn, d))
    gf = np.zeros((nn, d))
    D = np.zeros((max(npart, 1), d, d)) if want_D else None
    _check(_load().oracle_p2g(grid.ref(), npart, _ptr(x), _ptr(v), _ptr(B), _ptr(F), _ptr(m), _ptr(V),
                              int(model), float(mu), float(lam), int(transfer), _ptr(gm), _ptr(gmv), _ptr(gf),
                              _ptr(D) if want_D else None))
    out = {"m": gm, "mv": gmv, "f": gf}
    if want_D:
        out["D"] = D[:npart]
    return out


def grid_update(grid: Grid, gm, gmv, gf, dt: float, gravity=None, band=None):
    """Grid evolution of Sec. 3.3 at lambda = 0; returns v, vt, xt (nodes, d)."""
    d = grid.dim
    gm, gmv = _d(gm), _d(gmv)
    keep = _d(gf) if gf is not None else None
    gfp = _ptr(keep) if keep is not None else None
    g = _d(np.zeros(3) if gravity is None else list(gravity) + [0.0] * (3 - len(gravity)))
    bd = None
    if band is not None:
        bd = np.ascontiguousarray(list(band) + [0] * (6 - len(band)), dtype=np.int32)
    nn = grid.node_count
    gv, gvt, gxt = np.zeros((nn, d)), np.zeros((nn, d)), np.zeros((nn, d))
    _check(_load().oracle_grid_update(grid.ref(), _ptr(gm), _ptr(gmv), gfp, float(dt), _ptr(g),
                                      bd.ctypes.data_as(_ip) if bd is not None else None,
                                      _ptr(gv), _ptr(gvt), _ptr(gxt)))
    return {"v": gv, "vt": gvt, "xt": gxt}


def g2p(grid: Grid, x, F, gvt, gxt, *, transfer: int = TRANSFER_APIC):
    """Transfer to particles (Sec. 3.4) with the weights of time n; the affine
    state B_p is that of APIC, RPIC (Sec. 2.1) or PIC (zero) per ``transfer``."""
    d = grid.dim
    x, F, gvt, gxt = (_d(a) for a in (x, F, gvt, gxt))
    npart = x.shape[0]
    xo, vo = np.zeros((npart, d)), np.zeros((npart, d))
    Bo, Fo = np.zeros((npart, d, d)), np.zeros((npart, d, d))
    _check(_load().oracle_g2p(grid.ref(), npart, _ptr(x), _ptr(F), _ptr(gvt), _ptr(gxt), int(transfer),
                              _ptr(xo), _ptr(vo), _ptr(Bo), _ptr(Fo)))
    return {"x": xo, "v": vo, "B": Bo, "F": Fo}


def step(grid: Grid, x, v, B, F, m, V, model=0, mu=0.0, lam=0.0, dt=0.0, gravity=None, band=None,
         transfer=TRANSFER_APIC):
    """One explicit step: P2G, grid update, G2P.  Returns the grid stage
    arrays and the new particle state."""
    g = p2g(grid, x, v, B, F, m, V, model, mu, lam, transfer=transfer)
    u = grid_update(grid, g["m"], g["mv"], g["f"] if model == 1 else None, dt, gravity, band)
    p = g2p(grid, x, F, u["vt"], u["xt"], transfer=transfer)
    out = dict(g)
    out.update(u)
    out.update({"x_new": p["x"], "v_new": p["v"], "B_new": p["B"], "F_new": p["F"]})
    return out


def particle_totals(x, v, B, m):
    """[p (3), l (3), kinetic energy, mass]; l includes m_p B_p^T : eps (Sec. 5.3)."""
    x, v, m = _d(x), _d(v), _d(m)
    d = x.shape[1]
    keep = _d(B) if B is not None else None
    Bp = _ptr(keep) if keep is not None else None
    out = np.zeros(8)
    _load().oracle_particle_totals(d, x.shape[0], _ptr(x), _ptr(v), Bp, _ptr(m), _ptr(out))
    return out


def grid_totals(grid: Grid, gm, gvel, gpos=None):
    """[p (3), l (3), kinetic energy, mass] of grid velocities at gpos (x_i if None)."""
    gm, gvel = _d(gm), _d(gvel)
    keep = _d(gpos) if gpos is not None else None
    out = np.zeros(8)
    _load().oracle_grid_totals(grid.ref(), _ptr(gm), _ptr(gvel), _ptr(keep) if keep is not None else None,
                               _ptr(out))
    return out


def potential(F, V, mu: float, lam: float) -> float:
    F, V = _d(F), _d(V)
    out = ctypes.c_double()
    _check(_load().oracle_potential(F.shape[1], F.shape[0], _ptr(F), _ptr(V), mu, lam, ctypes.byref(out)))
    return out.value


def cfl_dt(dx: float, v, B, nu: float = 1.0, degree: int = 2) -> float:
    """Largest dt admitted by the CFL rule of Sec. 4.3 (degree 1: the same
    rule for the lagged C_p of Sec. 5.9, held in B)."""
    v, B = _d(v), _d(B)
    f = _load().oracle_cfl_dt_lagged if degree == 1 else _load().oracle_cfl_dt
    return f(v.shape[1], float(dx), float(nu), v.shape[0], _ptr(v), _ptr(B))


# ---------------------------------------------------------------------------
# Implicit midpoint (Sec. 3.3 at lambda = 1/2; Sec. 4.1, 4.2)
# ---------------------------------------------------------------------------

def neo_hookean_dP(F, mu: float, lam: float, dF) -> np.ndarray:
    """dP/dF : dF of the neo-Hookean stress (the product in the force
    derivative of Sec. 3.3)."""
    F, dF = _d(F), _d(dF)
    out = np.zeros_like(F)
    _check(_load().oracle_neo_hookean_dP(F.shape[0], _ptr(F), float(mu), float(lam), _ptr(dF), _ptr(out)))
    return out


def forces_at(grid: Grid, x, F, V, mu: float, lam: float, u):
    """Grid forces f_i = -dPhi/dx_i and Phi = sum_p V_p Psi(F_hat_p) with
    node i moved by u_i (Sec. 3.3).  Returns (f (nodes, d), Phi)."""
    x, F, V, u = _d(x), _d(F), _d(V), _d(u)
    f = np.zeros((grid.node_count, grid.dim))
    phi = ctypes.c_double(0.0)
    _check(_load().oracle_forces_at(grid.ref(), x.shape[0], _ptr(x), _ptr(F), _ptr(V), float(mu), float(lam),
                                    _ptr(u), _ptr(f), ctypes.byref(phi)))
    return f, phi.value


def force_differential(grid: Grid, x, F, V, mu: float, lam: float, u, du) -> np.ndarray:
    """sum_j (df_i/dx_j) du_j at the state displaced by u (Sec. 3.3, the force
    derivative and its helper)."""
    x, F, V, u, du = _d(x), _d(F), _d(V), _d(u), _d(du)
    df = np.zeros((grid.node_count, grid.dim))
    _check(_load().oracle_force_differential(grid.ref(), x.shape[0], _ptr(x), _ptr(F), _ptr(V), float(mu),
                                             float(lam), _ptr(u), _ptr(du), _ptr(df)))
    return df


def band_mask(grid: Grid, band) -> np.ndarray:
    """Nodes in the sticky band, by the rule of ``grid_update``."""
    mask = np.zeros(grid.node_count, dtype=bool)
    if band is None:
        return mask
    bd = np.ascontiguousarray(list(band) + [0] * (6 - len(band)), dtype=np.int32)
    lib = _load()
    idx = np.zeros(3, dtype=np.int32)
    for k, pos in enumerate(np.rint(grid.node_positions() / grid.dx).astype(np.int64)):
        idx[:grid.dim] = pos
        mask[k] = bool(lib.oracle_node_in_band(grid.ref(), idx.ctypes.data_as(_ip), bd.ctypes.data_as(_ip)))
    return mask


def midpoint_step(grid: Grid, x, v, B, F, m, V, model=1, mu=0.0, lam=0.0, dt=0.0, gravity=None, band=None,
                  newton_tol=1e-12, max_newton=12, cg_tol=1e-12, max_cg=400):
    """One implicit midpoint step (lambda = 1/2 of Sec. 3.3), APIC transfers.

    Grid: m_i and v_i = (m v)_i / m_i from the transfer of Sec. 3.2.  The
    unknown is dv_i = vt_i - v_i (Sec. 4.1), the minimizer of
        E(dv) = sum_i m_i/8 |dv_i|^2 - dt/4 sum_i m_i g.dv_i + Phi(x_i + u_i),
        u_i = dt/2 v_i + dt/4 dv_i,
    whose gradient (m_i/4) r_i with r_i = dv_i - dt (f_i/m_i + g) vanishes
    exactly at the midpoint equations.  Sticky-band nodes hold v_i = vt_i = 0
    and, with massless nodes, are not unknowns.

    Newton: each step solves (I - dt^2/4 M^{-1} K) delta = -r with
    K = df/dx (the operator of Sec. 4.2 that maps velocity-like vectors to
    velocity-like vectors) by the conjugate gradient of Sec. 4.2 in the mass
    inner product <a, b> = sum_i m_i a_i.b_i, starting from delta = 0 and
    stopping at <r, r> <= cg_tol^2 <b, b> or at non-positive curvature (then
    the iterate so far, or b itself on the first iteration); then a
    backtracking line search (halving from 1, at most 30 times, until E does
    not increase or |r|_M decreases: near the minimum E is flat to within its
    rounding while the gradient still falls; a trial that inverts an element
    has E = +inf, since Psi grows without bound as J -> 0+, and is halved).  Newton stops when
    |r|_M <= newton_tol |r_0|_M.

    Then vt_i = v_i + dv_i, xt_i = x_i + dt (v_i + vt_i)/2 and the transfer to
    particles of Sec. 3.4 in its general form.  Returns the new particle
    state and solver statistics."""
    d = grid.dim
    x, v, B, F, m, V = (_d(a) for a in (x, v, B, F, m, V))
    g = p2g(grid, x, v, B, F, m, V, 0)
    gm = g["m"]
    sticky = band_mask(grid, band)
    free = (gm > 0) & ~sticky
    mf = np.where(free, gm, 0.0)
    gv = np.zeros((grid.node_count, d))
    gv[free] = g["mv"][free] / gm[free, None]
    grav = np.zeros(d) if gravity is None else np.asarray(gravity, dtype=np.float64)[:d]
    Vp = V if model == 1 else V * 0.0

    def dot_m(a, b):
        return float(np.sum(mf[:, None] * a * b))

    def residual_energy(dv):
        u = 0.5 * dt * gv + 0.25 * dt * dv
        try:
            f, phi = forces_at(grid, x, F, Vp, mu, lam, u)
        except OracleError as e:
            # an inverted element: Psi -> +inf as J -> 0+, so E is +inf there
            if str(e) != _ERRORS[OR_E_INVERTED]:
                raise
            return None, np.inf
        r = np.zeros_like(dv)
        r[free] = dv[free] - dt * (f[free] / gm[free, None] + grav)
        E = float(np.sum(mf[:, None] * (0.125 * dv * dv - 0.25 * dt * grav * dv))) + phi
        return r, E

    def apply_A(dv, p):
        u = 0.5 * dt * gv + 0.25 * dt * dv
        df = force_differential(grid, x, F, Vp, mu, lam, u, p)
        s = np.zeros_like(p)
        s[free] = p[free] - 0.25 * dt * dt * df[free] / gm[free, None]
        return s

    dv = np.zeros((grid.node_count, d))
    stats = {"newton": 0, "cg": 0, "halvings": 0, "res0": 0.0, "res": 0.0}
    r, E = residual_energy(dv)
    if r is None:
        raise OracleError(_ERRORS[OR_E_INVERTED])
    res0 = np.sqrt(dot_m(r, r))
    stats["res0"] = res0
    for it in range(max_newton):
        if res0 == 0.0 or np.sqrt(dot_m(r, r)) <= newton_tol * res0:
            break
        # conjugate gradient on A delta = b, mass inner product (Sec. 4.2)
        b = -r
        delta = np.zeros_like(b)
        rc = b.copy()
        p = rc.copy()
        gamma = dot_m(rc, rc)
        gamma0 = gamma
        for k in range(max_cg):
            if gamma <= cg_tol * cg_tol * gamma0:
                break
            s = apply_A(dv, p)
            ps = dot_m(p, s)
            stats["cg"] += 1
            if ps <= 0.0:
                if k == 0:
                    delta = b.copy()
                break
            alpha = gamma / ps
            delta = delta + alpha * p
            rc = rc - alpha * s
            kappa = dot_m(rc, rc)
            p = rc + (kappa / gamma) * p
            gamma = kappa
        # backtracking line search on E; a trial with an inverted element
        # (E = +inf) is always halved
        step = 1.0
        for k in range(30):
            r_new, E_new = residual_energy(dv + step * delta)
            ok = np.isfinite(E_new) and (E_new <= E or np.sqrt(dot_m(r_new, r_new)) < np.sqrt(dot_m(r, r)))
            if ok or k == 29:
                break
            step *= 0.5
            stats["halvings"] += 1
        if not np.isfinite(E_new):
            raise OracleError(_ERRORS[OR_E_INVERTED])
        dv = dv + step * delta
        r, E = r_new, E_new
        stats["newton"] = it + 1
    stats["res"] = float(np.sqrt(dot_m(r, r)))
    gvt = np.where(free[:, None], gv + dv, 0.0)
    gxt = grid.node_positions() + dt * 0.5 * (gv + gvt)
    out = g2p(grid, x, F, gvt, gxt)
    return {"m": gm, "v": gv, "vt": gvt, "xt": gxt, "x_new": out["x"], "v_new": out["v"], "B_new": out["B"],
            "F_new": out["F"], "stats": stats}
