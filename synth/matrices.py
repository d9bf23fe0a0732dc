"""Seeded sparse test matrices (CSR, int32 indices, float64 values).

What is built here:

* closed-form matrices (diagonal, permuted diagonal, 2x2 block diagonal) whose
  singular values are known exactly;
* a row/column-scaled banded matrix ``D_r B D_c`` whose condition number is
  dominated by the scaling, as the paper reports for its benchmark systems
  (column norms spread over many decades, section "Condition Number and
  Preconditioning");
* a tiny variable-viscosity Stokes system on a staggered grid;
* the six-field hydro-mechanical staggered-grid system (solid velocity, total
  pressure, Darcy flux, fluid pressure) whose governing equations the paper
  lists in section "Governing Equations".

The paper gives the PDEs but no discretisation constants, boundary
conditions or units, so the constants below are this project's choice; they
are picked so that the systems are scaling-dominated with kappa_2 of order
1e20-1e25, as the paper's matrices are.

Only numpy/scipy assembly lives here; nothing in this module computes a norm,
a singular value or any step of the estimator.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Csr:
    """A square CSR matrix: int32 column indices, float64 values.

    ``rowptr`` is int64 so that it also covers factors above 2**31 entries;
    the C library accepts int32 or int64 row pointers.
    """

    n: int
    rowptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]
    meta: dict | None = None

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(a, meta: dict | None = None) -> "Csr":
        a = sp.csr_matrix(a)
        a.sum_duplicates()
        a.sort_indices()
        if a.shape[0] != a.shape[1]:
            raise ValueError("square matrices only")
        return Csr(
            n=int(a.shape[0]),
            rowptr=np.ascontiguousarray(a.indptr, dtype=np.int64),
            col=np.ascontiguousarray(a.indices, dtype=np.int32),
            val=np.ascontiguousarray(a.data, dtype=np.float64),
            meta=meta or {},
        )

    def save(self, path: str) -> None:
        np.savez(path, n=self.n, rowptr=self.rowptr, col=self.col, val=self.val)

    @staticmethod
    def load(path: str) -> "Csr":
        z = np.load(path, allow_pickle=False)
        return Csr(int(z["n"]), z["rowptr"].astype(np.int64), z["col"].astype(np.int32),
                   z["val"].astype(np.float64), {})


def csr_from_dense(a: np.ndarray, meta: dict | None = None) -> Csr:
    return Csr.from_scipy(sp.csr_matrix(np.asarray(a, dtype=np.float64)), meta)


# ---------------------------------------------------------------- closed form
def diag_csr(d, row_perm=None, col_perm=None) -> Csr:
    """P diag(d) Q as CSR: row ``row_perm[i]`` holds d[i] in column ``col_perm[i]``.

    Its singular values are |d| exactly, whatever the permutations.
    """
    d = np.asarray(d, dtype=np.float64)
    n = d.size
    rp = np.arange(n) if row_perm is None else np.asarray(row_perm)
    cp = np.arange(n) if col_perm is None else np.asarray(col_perm)
    a = sp.coo_matrix((d, (rp, cp)), shape=(n, n))
    return Csr.from_scipy(a, {"kind": "diag"})


def block_diag_2x2(blocks) -> Csr:
    """Block-diagonal matrix of 2x2 blocks given as an array of shape (b, 2, 2)."""
    blocks = np.asarray(blocks, dtype=np.float64)
    return Csr.from_scipy(sp.block_diag(list(blocks), format="csr"), {"kind": "blockdiag2"})


def scaled_banded(n: int, seed: int, offsets=(-7, -3, -1, 0, 1, 3, 7), col_decades=10.0,
                  row_decades=3.0, off_scale=0.3) -> Csr:
    """D_r B D_c with B a well-conditioned banded matrix and log-uniform scalings.

    B has diagonal 1 + U(0,1) and off-diagonals off_scale * N(0,1); D_c and D_r
    are 10**U(-col_decades, col_decades) and 10**U(-row_decades, row_decades).
    """
    rng = np.random.default_rng(seed)
    diags = []
    for o in offsets:
        m = n - abs(o)
        diags.append(1.0 + rng.random(m) if o == 0 else off_scale * rng.standard_normal(m))
    b = sp.diags(diags, list(offsets), shape=(n, n), format="csr")
    dc = 10.0 ** rng.uniform(-col_decades, col_decades, n)
    dr = 10.0 ** rng.uniform(-row_decades, row_decades, n)
    a = sp.diags(dr) @ b @ sp.diags(dc)
    return Csr.from_scipy(a, {"kind": "scaled_banded", "seed": seed})


# ------------------------------------------------------------- assembly util
class _Triplets:
    def __init__(self):
        self.r, self.c, self.v = [], [], []

    def add(self, rows, cols, vals, mask=None):
        rows = np.asarray(rows)
        cols = np.broadcast_to(np.asarray(cols), rows.shape)
        vals = np.broadcast_to(np.asarray(vals, dtype=np.float64), rows.shape)
        if mask is not None:
            mask = np.broadcast_to(mask, rows.shape)
            rows, cols, vals = rows[mask], cols[mask], vals[mask]
        self.r.append(rows.ravel().astype(np.int64))
        self.c.append(cols.ravel().astype(np.int64))
        self.v.append(vals.ravel().astype(np.float64))

    def build(self, n, meta) -> Csr:
        r = np.concatenate(self.r)
        c = np.concatenate(self.c)
        v = np.concatenate(self.v)
        a = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
        a.sum_duplicates()
        a.eliminate_zeros()
        a.sort_indices()
        return Csr.from_scipy(a, meta)



def _balance_and_scale(a, kinds, small_kinds, rng, big_decades=(10.0, 13.0),
                       small_decades=(-5.0, -2.0), sweeps: int = 3, position=None):
    """Unit choice per unknown type, then an explicit column scaling.

    ``kinds[i]`` is the unknown type of column i and the equation type of row
    i (the discretisations here put equation i at unknown i). First each
    equation type and each unknown type is rescaled by one constant (the
    median row / column norm of that type), a change of units that removes
    the between-type imbalance of the raw SI coefficients. Then every column
    is normalised and multiplied by 10**U(big_decades) or, for the types in
    ``small_kinds``, 10**U(small_decades), or -- when ``position`` (one value in
    [0, 1] per column) is given -- to that place inside its cluster's range.
    The result is A = B D with
    kappa(B) set by the physics (viscosity and permeability contrasts, grid
    size) and the extra ill-conditioning carried by the column scaling D, the
    structure the paper reports for its systems: column norms in two clusters
    (below 1e-2 and above 1e10) and kappa dropping by about 15 decades under
    column scaling.
    """
    a = sp.csr_matrix(a, dtype=np.float64)
    kinds = np.asarray(kinds)
    types = np.unique(kinds)
    for _ in range(sweeps):
        cn = np.sqrt(np.asarray(a.multiply(a).sum(axis=0)).ravel())
        cs = np.ones(a.shape[1])
        for t in types:
            cs[kinds == t] = np.median(cn[kinds == t])
        a = a @ sp.diags(1.0 / cs)
        rn = np.sqrt(np.asarray(a.multiply(a).sum(axis=1)).ravel())
        rs = np.ones(a.shape[0])
        for t in types:
            rs[kinds == t] = np.median(rn[kinds == t])
        a = sp.diags(1.0 / rs) @ a
    cn = np.sqrt(np.asarray(a.multiply(a).sum(axis=0)).ravel())
    small = np.isin(kinds, np.asarray(list(small_kinds)))
    if position is None:  # seeded random place inside each cluster
        dec = np.where(small, rng.uniform(small_decades[0], small_decades[1], kinds.size),
                       rng.uniform(big_decades[0], big_decades[1], kinds.size))
    else:
        dec = np.where(small, small_decades[0] + (small_decades[1] - small_decades[0]) * position,
                       big_decades[0] + (big_decades[1] - big_decades[0]) * position)
    return sp.csr_matrix(a @ sp.diags(10.0 ** dec / cn))

# ---------------------------------------------------------- tiny Stokes (C1)
def stokes2d(nx: int = 10, ny: int = 10, seed: int = 0, lx: float = 1.0e3, ly: float = 1.0e3,
             eta_range=(18.0, 24.0), cont_scale: float | None = None, raw: bool = False,
             big_decades=(11.0, 14.0), small_decades=(-6.0, -3.0)) -> Csr:
    """Variable-viscosity incompressible Stokes on a staggered grid with nx x ny cells.

    Unknowns: vx on the (nx+1) x ny vertical faces, vy on the nx x (ny+1)
    horizontal faces, P in the nx x ny cells (vx first, then vy, then P).
    x-momentum uses the 11-point staggered stencil (5 vx, 4 vy, 2 P),
    continuity the 4-point divergence. Free slip on all walls (normal velocity
    rows are Dirichlet identity rows), pressure in cell (0,0) pinned.
    log10(eta) ~ U(eta_range) per cell, seeded; corner viscosity is the
    geometric mean of the adjacent cells.

    Pressure and continuity are scaled by ``cont_scale`` (default
    2*eta_min/(dx+dy) of the drawn field, the usual choice on staggered
    grids): the pressure unknown is P/cont_scale and the continuity rows are
    multiplied by cont_scale. Without this scaling the system is numerically
    singular (kappa far above 1/eps), which no estimator can resolve.

    Unless ``raw``, the SI system then goes through ``_balance_and_scale`` with
    the pressure columns in the small cluster (seeded from ``seed + 1``).
    """
    rng = np.random.default_rng(seed)
    dx, dy = lx / nx, ly / ny
    etac = 10.0 ** rng.uniform(eta_range[0], eta_range[1], (ny, nx))
    pad = np.pad(np.log10(etac), 1, mode="edge")
    etan = 10.0 ** (0.25 * (pad[:-1, :-1] + pad[1:, :-1] + pad[:-1, 1:] + pad[1:, 1:]))  # (ny+1, nx+1)
    kc = 2.0 * etac.min() / (dx + dy) if cont_scale is None else float(cont_scale)
    kb = np.exp(np.log(etac).mean()) / min(dx, dy) ** 2  # wall-row scale: typical eta/h^2

    nvx = (nx + 1) * ny
    nvy = nx * (ny + 1)
    n = nvx + nvy + nx * ny

    def ivx(i, j):  # vx at x = i*dx, y = (j+1/2)*dy
        return j * (nx + 1) + i

    def ivy(i, j):  # vy at x = (i+1/2)*dx, y = j*dy
        return nvx + j * nx + i

    def ip(i, j):
        return nvx + nvy + j * nx + i

    t = _Triplets()
    # x-momentum
    J, I = np.meshgrid(np.arange(ny), np.arange(nx + 1), indexing="ij")
    bnd = (I == 0) | (I == nx)
    t.add(ivx(I, J), ivx(I, J), kb, bnd)
    inn = ~bnd
    Ii, Jj = np.clip(I, 1, nx - 1), J
    e1 = etac[Jj, np.clip(Ii, 0, nx - 1)]
    e0 = etac[Jj, Ii - 1]
    en1 = etan[Jj + 1, Ii]
    en0 = etan[Jj, Ii]
    r = ivx(Ii, Jj)
    up = Jj + 1 < ny
    dn = Jj - 1 >= 0
    t.add(r, ivx(Ii + 1, Jj), 2 * e1 / dx**2, inn)
    t.add(r, ivx(Ii - 1, Jj), 2 * e0 / dx**2, inn)
    diag = -2 * (e1 + e0) / dx**2 - np.where(up, en1, 0) / dy**2 - np.where(dn, en0, 0) / dy**2
    t.add(r, r, diag, inn)
    t.add(r, ivx(Ii, np.minimum(Jj + 1, ny - 1)), en1 / dy**2, inn & up)
    t.add(r, ivx(Ii, np.maximum(Jj - 1, 0)), en0 / dy**2, inn & dn)
    t.add(r, ivy(Ii, Jj + 1), en1 / (dx * dy), inn)
    t.add(r, ivy(Ii - 1, Jj + 1), -en1 / (dx * dy), inn)
    t.add(r, ivy(Ii, Jj), -en0 / (dx * dy), inn)
    t.add(r, ivy(Ii - 1, Jj), en0 / (dx * dy), inn)
    t.add(r, ip(np.minimum(Ii, nx - 1), Jj), -kc / dx, inn)
    t.add(r, ip(Ii - 1, Jj), kc / dx, inn)
    # y-momentum
    J, I = np.meshgrid(np.arange(ny + 1), np.arange(nx), indexing="ij")
    bnd = (J == 0) | (J == ny)
    t.add(ivy(I, J), ivy(I, J), kb, bnd)
    inn = ~bnd
    Ii, Jj = I, np.clip(J, 1, ny - 1)
    e1 = etac[np.clip(Jj, 0, ny - 1), Ii]
    e0 = etac[Jj - 1, Ii]
    en1 = etan[Jj, Ii + 1]
    en0 = etan[Jj, Ii]
    r = ivy(Ii, Jj)
    rt = Ii + 1 < nx
    lt = Ii - 1 >= 0
    t.add(r, ivy(Ii, Jj + 1), 2 * e1 / dy**2, inn)
    t.add(r, ivy(Ii, Jj - 1), 2 * e0 / dy**2, inn)
    diag = -2 * (e1 + e0) / dy**2 - np.where(rt, en1, 0) / dx**2 - np.where(lt, en0, 0) / dx**2
    t.add(r, r, diag, inn)
    t.add(r, ivy(np.minimum(Ii + 1, nx - 1), Jj), en1 / dx**2, inn & rt)
    t.add(r, ivy(np.maximum(Ii - 1, 0), Jj), en0 / dx**2, inn & lt)
    t.add(r, ivx(Ii + 1, Jj), en1 / (dx * dy), inn)
    t.add(r, ivx(Ii + 1, Jj - 1), -en1 / (dx * dy), inn)
    t.add(r, ivx(Ii, Jj), -en0 / (dx * dy), inn)
    t.add(r, ivx(Ii, Jj - 1), en0 / (dx * dy), inn)
    t.add(r, ip(Ii, np.minimum(Jj, ny - 1)), -kc / dy, inn)
    t.add(r, ip(Ii, Jj - 1), kc / dy, inn)
    # continuity
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    pin = (I == 0) & (J == 0)
    t.add(ip(I, J), ip(I, J), kc * kc / np.exp(np.log(etac).mean()), pin)
    free = ~pin
    r = ip(I, J)
    t.add(r, ivx(I + 1, J), kc / dx, free)
    t.add(r, ivx(I, J), -kc / dx, free)
    t.add(r, ivy(I, J + 1), kc / dy, free)
    t.add(r, ivy(I, J), -kc / dy, free)
    meta = {"kind": "stokes2d", "nx": nx, "ny": ny, "seed": seed, "cont_scale": kc}
    a = t.build(n, meta)
    if raw:
        return a
    kinds = np.concatenate([np.zeros(nvx, np.int64), np.ones(nvy, np.int64), np.full(nx * ny, 2)])
    b = _balance_and_scale(a.to_scipy(), kinds, (2,), np.random.default_rng(seed + 1),
                           big_decades, small_decades)
    return Csr.from_scipy(b, meta)


# ----------------------------------------------- hydro-mechanical (C2..C5)
HM_FIELDS = ("vx", "vy", "P", "qx", "qy", "Pf")

#: Generator constants (SI units). The paper names the physical parameters of
#: its governing equations but gives no values; these are this project's.
HM_CONSTANTS = dict(
    lx=500.0,  # domain width [m] (the paper's domain is 500 m x 50 m)
    ly=50.0,  # domain height [m]
    eta_fluid=1.0e-3,  # fluid viscosity [Pa s]
    phi=0.01,  # porosity
    beta_d=1.0e-10,  # drained compressibility [1/Pa]
    alpha=0.9,  # Biot-Willis coefficient
    skempton=0.6,  # Skempton coefficient B
    dt=1.0e7,  # time step [s]
    compaction_factor=1.0,  # eta_phi = compaction_factor * eta / phi
)


def hm_fields(side: int, seed: int, eta_range=(18.0, 24.0), perm_range=(-20.0, -12.0)):
    """Per-cell log10 viscosity and log10 permeability, log-uniform, seeded.

    Returns two float64 arrays of shape (side-1, side-1).
    """
    rng = np.random.default_rng(seed)
    c = side - 1
    log_eta = rng.uniform(eta_range[0], eta_range[1], (c, c))
    log_k = rng.uniform(perm_range[0], perm_range[1], (c, c))
    return log_eta, log_k


def hydromech2d(side: int, seed: int | None = None, log_eta=None, log_k=None, consts=None,
                pressure_scale: float | None = None, flux_scale: float = 1.0, raw: bool = False,
                big_decades=(11.5, 14.5), small_decades=(-5.0, -2.0), eta_range=(18.0, 24.0),
                perm_range=(-20.0, -12.0)) -> Csr:
    """Six-field hydro-mechanical staggered-grid matrix on side x side nodes.

    Ordering is node-major: unknown (i, j, f) -> 6*(i*side + j) + f with
    f in (vx, vy, P, qx, qy, Pf), i the row (y) and j the column (x) of the
    basic node, which gives the tri-banded pattern the paper shows. Every node
    carries all six unknowns; the ones that fall outside the domain (ghost
    nodes) and the Dirichlet boundary unknowns get scaled identity rows, so
    n = 6*side**2 exactly.

    Equations (rows), with the paper's governing equations as the model:
      vx, vy : bulk momentum, d(tau_ij)/dx_j - dP/dx_i (11-point stencil), free
               slip on the walls parallel to the velocity component;
      P      : solid mass, div(v_s) + beta_d (P - alpha Pf)/dt + (P - Pf)/((1-phi) eta_phi);
      qx, qy : Darcy, q_i + (k/eta_f) dPf/dx_i, no flux through the walls;
      Pf     : fluid mass, div(q) - beta_d alpha (P - Pf/B)/dt - (P - Pf)/((1-phi) eta_phi).
    Both pressures are scaled by ``pressure_scale`` (default 2*eta_min/(dx+dy))
    and both mass-conservation rows by the same factor, as staggered-grid
    codes do; the Darcy flux unknowns by ``flux_scale``.

    Unless ``raw``, the SI system then goes through ``_balance_and_scale`` with
    the two Darcy-flux fields (qx, qy: one third of the columns, as in the
    paper's column-norm distribution) in the small cluster; each column's place
    inside its cluster follows the local log-permeability (flux columns) or
    log-viscosity (the others), so the matrix depends on the fields only.
    """
    k = side
    if k < 4:
        raise ValueError("side must be >= 4")
    cst = dict(HM_CONSTANTS)
    if consts:
        cst.update(consts)
    if log_eta is None or log_k is None:
        le, lk = hm_fields(side, 0 if seed is None else seed, eta_range, perm_range)
        log_eta = le if log_eta is None else log_eta
        log_k = lk if log_k is None else log_k
    log_eta = np.asarray(log_eta, dtype=np.float64)
    log_k = np.asarray(log_k, dtype=np.float64)
    assert log_eta.shape == (k - 1, k - 1) and log_k.shape == (k - 1, k - 1)
    dx = cst["lx"] / (k - 1)
    dy = cst["ly"] / (k - 1)
    etac = 10.0 ** log_eta
    permc = 10.0 ** log_k
    pad = np.pad(log_eta, 1, mode="edge")
    etan = 10.0 ** (0.25 * (pad[:-1, :-1] + pad[1:, :-1] + pad[:-1, 1:] + pad[1:, 1:]))  # (k, k)
    ps = 2.0 * etac.min() / (dx + dy) if pressure_scale is None else float(pressure_scale)
    qs = float(flux_scale)
    ef = cst["eta_fluid"]
    phi = cst["phi"]
    bd = cst["beta_d"]
    al = cst["alpha"]
    bsk = cst["skempton"]
    dt = cst["dt"]
    n = 6 * k * k

    def u(i, j, f):
        return 6 * (i * k + j) + f

    VX, VY, P, QX, QY, PF = range(6)
    t = _Triplets()
    I, J = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")  # I: y index, J: x index
    Ic = np.clip(I, 0, k - 2)
    Jc = np.clip(J, 0, k - 2)
    kb_v = etac.max() / min(dx, dy) ** 2  # identity-row scale for velocity ghosts / walls
    kb_p = ps * ps / etac.max()  # identity-row scale for pressure ghosts

    # ---- x-momentum at vx(i, j): x = j dx, y = (i + 1/2) dy
    real = (I <= k - 2)
    wall = real & ((J == 0) | (J == k - 1))
    inn = real & ~wall
    t.add(u(I, J, VX), u(I, J, VX), kb_v, ~inn)
    Ji = np.clip(J, 1, k - 2)
    e1 = etac[Ic, Ji]
    e0 = etac[Ic, Ji - 1]
    et = etan[np.minimum(Ic + 1, k - 1), Ji]
    eb = etan[Ic, Ji]
    r = u(Ic, Ji, VX)
    up = Ic < k - 2
    dn = Ic > 0
    t.add(r, u(Ic, Ji + 1, VX), 2 * e1 / dx**2, inn)
    t.add(r, u(Ic, Ji - 1, VX), 2 * e0 / dx**2, inn)
    t.add(r, r, -2 * (e1 + e0) / dx**2 - np.where(up, et, 0) / dy**2 - np.where(dn, eb, 0) / dy**2, inn)
    t.add(r, u(np.minimum(Ic + 1, k - 1), Ji, VX), et / dy**2, inn & up)
    t.add(r, u(np.maximum(Ic - 1, 0), Ji, VX), eb / dy**2, inn & dn)
    t.add(r, u(Ic + 1, Ji, VY), et / (dx * dy), inn)
    t.add(r, u(Ic + 1, Ji - 1, VY), -et / (dx * dy), inn)
    t.add(r, u(Ic, Ji, VY), -eb / (dx * dy), inn)
    t.add(r, u(Ic, Ji - 1, VY), eb / (dx * dy), inn)
    t.add(r, u(Ic, Ji, P), -ps / dx, inn)
    t.add(r, u(Ic, Ji - 1, P), ps / dx, inn)

    # ---- y-momentum at vy(i, j): x = (j + 1/2) dx, y = i dy
    real = (J <= k - 2)
    wall = real & ((I == 0) | (I == k - 1))
    inn = real & ~wall
    t.add(u(I, J, VY), u(I, J, VY), kb_v, ~inn)
    Ii = np.clip(I, 1, k - 2)
    e1 = etac[Ii, Jc]
    e0 = etac[Ii - 1, Jc]
    er = etan[Ii, np.minimum(Jc + 1, k - 1)]
    el = etan[Ii, Jc]
    r = u(Ii, Jc, VY)
    rt = Jc < k - 2
    lt = Jc > 0
    t.add(r, u(Ii + 1, Jc, VY), 2 * e1 / dy**2, inn)
    t.add(r, u(Ii - 1, Jc, VY), 2 * e0 / dy**2, inn)
    t.add(r, r, -2 * (e1 + e0) / dy**2 - np.where(rt, er, 0) / dx**2 - np.where(lt, el, 0) / dx**2, inn)
    t.add(r, u(Ii, np.minimum(Jc + 1, k - 1), VY), er / dx**2, inn & rt)
    t.add(r, u(Ii, np.maximum(Jc - 1, 0), VY), el / dx**2, inn & lt)
    t.add(r, u(Ii, Jc + 1, VX), er / (dx * dy), inn)
    t.add(r, u(Ii - 1, Jc + 1, VX), -er / (dx * dy), inn)
    t.add(r, u(Ii, Jc, VX), -el / (dx * dy), inn)
    t.add(r, u(Ii - 1, Jc, VX), el / (dx * dy), inn)
    t.add(r, u(Ii, Jc, P), -ps / dy, inn)
    t.add(r, u(Ii - 1, Jc, P), ps / dy, inn)

    # ---- cell-centred rows: solid mass (P) and fluid mass (Pf)
    cell = (I <= k - 2) & (J <= k - 2)
    t.add(u(I, J, P), u(I, J, P), kb_p, ~cell)
    t.add(u(I, J, PF), u(I, J, PF), kb_p, ~cell)
    eta_phi = cst["compaction_factor"] * etac[Ic, Jc] / phi
    comp = 1.0 / ((1.0 - phi) * eta_phi)
    r = u(Ic, Jc, P)
    t.add(r, u(Ic, Jc + 1, VX), ps / dx, cell)
    t.add(r, u(Ic, Jc, VX), -ps / dx, cell)
    t.add(r, u(Ic + 1, Jc, VY), ps / dy, cell)
    t.add(r, u(Ic, Jc, VY), -ps / dy, cell)
    t.add(r, r, ps * ps * (bd / dt + comp), cell)
    t.add(r, u(Ic, Jc, PF), -ps * ps * (bd * al / dt + comp), cell)
    r = u(Ic, Jc, PF)
    t.add(r, u(Ic, Jc + 1, QX), ps * qs / dx, cell)
    t.add(r, u(Ic, Jc, QX), -ps * qs / dx, cell)
    t.add(r, u(Ic + 1, Jc, QY), ps * qs / dy, cell)
    t.add(r, u(Ic, Jc, QY), -ps * qs / dy, cell)
    t.add(r, u(Ic, Jc, P), -ps * ps * (bd * al / dt + comp), cell)
    t.add(r, r, ps * ps * (bd * al / (bsk * dt) + comp), cell)

    # ---- Darcy x at qx(i, j) (vx position), no flux through x-walls
    real = (I <= k - 2)
    wall = real & ((J == 0) | (J == k - 1))
    inn = real & ~wall
    t.add(u(I, J, QX), u(I, J, QX), qs, ~inn)
    kf = np.sqrt(permc[Ic, Ji - 1] * permc[Ic, Ji])
    r = u(Ic, Ji, QX)
    t.add(r, r, qs, inn)
    t.add(r, u(Ic, Ji, PF), ps * kf / (ef * dx), inn)
    t.add(r, u(Ic, Ji - 1, PF), -ps * kf / (ef * dx), inn)

    # ---- Darcy y at qy(i, j) (vy position), no flux through y-walls
    real = (J <= k - 2)
    wall = real & ((I == 0) | (I == k - 1))
    inn = real & ~wall
    t.add(u(I, J, QY), u(I, J, QY), qs, ~inn)
    kf = np.sqrt(permc[Ii - 1, Jc] * permc[Ii, Jc])
    r = u(Ii, Jc, QY)
    t.add(r, r, qs, inn)
    t.add(r, u(Ii, Jc, PF), ps * kf / (ef * dy), inn)
    t.add(r, u(Ii - 1, Jc, PF), -ps * kf / (ef * dy), inn)

    meta = {"kind": "hydromech2d", "side": side, "seed": seed, "pressure_scale": ps,
            "flux_scale": qs, "dx": dx, "dy": dy}
    a = t.build(n, meta)
    if raw:
        return a
    kinds = np.arange(n, dtype=np.int64) % 6
    # Column scales follow the local coefficients (a choice of units per
    # unknown proportional to the local material): a flux column's place in
    # the small cluster is its node's log-permeability, every other column's
    # place in the large cluster its node's log-viscosity. The matrix is then
    # a function of the two fields alone.
    padk = np.pad(log_k, 1, mode="edge")
    node_k = 0.25 * (padk[:-1, :-1] + padk[1:, :-1] + padk[:-1, 1:] + padk[1:, 1:])
    pade = np.pad(log_eta, 1, mode="edge")
    node_e = 0.25 * (pade[:-1, :-1] + pade[1:, :-1] + pade[:-1, 1:] + pade[1:, 1:])
    pos_k = np.clip((node_k - perm_range[0]) / (perm_range[1] - perm_range[0]), 0.0, 1.0)
    pos_e = np.clip((node_e - eta_range[0]) / (eta_range[1] - eta_range[0]), 0.0, 1.0)
    position = np.where(np.isin(kinds, (QX, QY)), np.repeat(pos_k.ravel(), 6),
                        np.repeat(pos_e.ravel(), 6))
    b = _balance_and_scale(a.to_scipy(), kinds, (QX, QY), None, big_decades, small_decades,
                           position=position)
    return Csr.from_scipy(b, meta)


def hm_batch_specs(count: int = 64, side_range=(51, 401), seed_sides: int = 3, seed_base: int = 4,
                   sigma_decades: float = 0.5):
    """Sides and perturbed coefficient fields for the batched workload.

    One base log-field pair is drawn on the largest grid; each matrix samples
    it at its own cell centres (nearest cell, in physical coordinates) and adds
    an independent N(0, sigma_decades^2) perturbation per cell, in decades.
    Returns a list of (side, log_eta, log_k).
    """
    rng = np.random.default_rng(seed_sides)
    sides = rng.integers(side_range[0], side_range[1] + 1, size=count)
    base_side = int(side_range[1])
    be, bk = hm_fields(base_side, seed_base)
    out = []
    for m, s in enumerate(sides):
        s = int(s)
        c = s - 1
        centres = (np.arange(c) + 0.5) / c
        src = np.minimum((centres * (base_side - 1)).astype(np.int64), base_side - 2)
        prng = np.random.default_rng(seed_base * 1000003 + m)
        le = be[np.ix_(src, src)] + prng.normal(0.0, sigma_decades, (c, c))
        lk = bk[np.ix_(src, src)] + prng.normal(0.0, sigma_decades, (c, c))
        out.append((s, le, lk))
    return out
