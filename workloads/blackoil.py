"""Seeded synthetic black-oil Jacobians (3x3-block BSR) and right-hand sides.

This module only *generates inputs*: it holds none of the solver's arithmetic
and is shared by the oracle tests, the GPU tests and the benchmark.  The SPE10
property data used in the paper's experiments (Section 6) is not available, so
the workloads below stand in for it with the same grid shape (60x220x85),
strong layered heterogeneity, inactive cells and channelised permeability.

Value rules (one reading of an under-determined recipe):

* cells are ordered naturally, c = i + nx*(j + ny*k); inactive cells are
  skipped and the active ones renumbered in the same order; the unknowns of a
  cell are interleaved (P, Sw, Sg);
* each face between two active cells carries a transmissibility
  T = tau * 2*k_c*k_d/(k_c + k_d) (harmonic mean, unit geometry; k_z = ratio*k
  on z faces), tau = 1e-3;
* the off-diagonal block A_cd has (0,0) = -T and its other 8 entries equal
  u*(-T) with u ~ U[-0.1, 0.1], drawn independently for A_cd and A_dc;
* the diagonal block is the accumulation diag(phi*c_t, phi, phi) minus the
  entrywise sum of the row's off-diagonal blocks, except that the saturation
  self-entries are made dominance-safe: D[a][a] = phi + sum_d sum_b |A_cd[a][b]|
  for a in {1, 2};
* RHS entries are U[-1, 1].

Block rows list their columns in ascending order and always store the
diagonal block.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TAU = 1.0e-3
PORO = 0.2
COMPRESS = 1.0e-5
U_COUPLING = 0.1


@dataclass
class BsrCase:
    """A 3x3-block sparse matrix in BSR form plus its grid description."""

    row_ptr: np.ndarray  # int32 [n_b + 1]
    col: np.ndarray  # int32 [nnz_b]
    vals: np.ndarray  # float64 [nnz_b, 3, 3], row-major blocks
    grid: tuple = (0, 0, 0)
    active: np.ndarray | None = None  # bool over the full grid (natural order)
    meta: dict = field(default_factory=dict)

    @property
    def n_b(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz_b(self) -> int:
        return int(self.col.shape[0])

    @property
    def ndof(self) -> int:
        return 3 * self.n_b


@dataclass
class FaceData:
    """Per-direction face transmissibilities and coupling draws on the full grid.

    T[d] has one entry per cell (the face to the +d neighbour; zero where that
    neighbour is outside the grid or either side is inactive).  U[d] has shape
    (ncell, 2, 8): index 0 is the block A_{c,c+d}, index 1 is A_{c+d,c}; the
    8 entries fill the block in row-major order skipping (0,0).
    """

    T: list
    U: list


# ---------------------------------------------------------------- permeability
def perm_iid_lognormal(shape, rng, mean_md=100.0, sigma=1.0):
    nx, ny, nz = shape
    return np.exp(math.log(mean_md) + sigma * rng.standard_normal(nx * ny * nz))


def perm_layered_lognormal(shape, rng, mean_md=100.0, sigma=2.0, layer_frac=0.7):
    """ln k = ln(mean) + sigma*(sqrt(f)*zeta_layer + sqrt(1-f)*xi_cell)."""
    nx, ny, nz = shape
    zeta = rng.standard_normal(nz)
    xi = rng.standard_normal(nx * ny * nz)
    layer = np.repeat(zeta, nx * ny)
    return np.exp(math.log(mean_md) + sigma * (math.sqrt(layer_frac) * layer
                                               + math.sqrt(1.0 - layer_frac) * xi))


def perm_channels(shape, rng, k_in=1000.0, k_out=1.0):
    """Per layer 4-8 sinusoidal channels at k_in on a k_out background."""
    nx, ny, nz = shape
    k = np.full((nz, ny, nx), k_out)
    ii = np.arange(nx)[None, :]
    jj = np.arange(ny)[:, None]
    for kk in range(nz):
        nch = int(rng.integers(4, 9))
        for _ in range(nch):
            y0 = rng.uniform(0.0, ny)
            amp = rng.uniform(5.0, 20.0)
            wl = rng.uniform(50.0, 200.0)
            ph = rng.uniform(0.0, 2.0 * math.pi)
            width = int(rng.integers(3, 9))
            yc = y0 + amp * np.sin(2.0 * math.pi * ii / wl + ph)
            inside = np.abs(jj - yc) <= 0.5 * width
            k[kk][inside] = k_in
    return k.reshape(-1)


def random_mask(shape, rng, frac):
    ncell = shape[0] * shape[1] * shape[2]
    active = np.ones(ncell, dtype=bool)
    n_off = int(round(frac * ncell))
    if n_off > 0:
        active[rng.choice(ncell, size=n_off, replace=False)] = False
    return active


# ---------------------------------------------------------------- faces
def _neighbour_ok(shape, d):
    nx, ny, nz = shape
    i = np.tile(np.arange(nx), ny * nz)
    j = np.tile(np.repeat(np.arange(ny), nx), nz)
    k = np.repeat(np.arange(nz), nx * ny)
    return (i < nx - 1, j < ny - 1, k < nz - 1)[d]


def make_faces(shape, perm, active, kz_ratio, rng, tau=TAU):
    nx, ny, nz = shape
    ncell = nx * ny * nz
    strides = (1, nx, nx * ny)
    T, U = [], []
    for d in range(3):
        ok = _neighbour_ok(shape, d)
        c = np.nonzero(ok)[0]
        nb = c + strides[d]
        kc, kd = perm[c], perm[nb]
        if d == 2:
            kc, kd = kz_ratio * kc, kz_ratio * kd
        t = np.zeros(ncell)
        t[c] = tau * 2.0 * kc * kd / (kc + kd)
        t[c] *= (active[c] & active[nb])
        T.append(t)
        U.append(rng.uniform(-U_COUPLING, U_COUPLING, size=(ncell, 2, 8)))
    return FaceData(T=T, U=U)


def drift_faces(faces: FaceData, rng, amp=0.05):
    """One Newton step of value drift: T and u scaled by (1 + U[-amp, amp])."""
    T, U = [], []
    for d in range(3):
        T.append(faces.T[d] * (1.0 + rng.uniform(-amp, amp, size=faces.T[d].shape)))
        U.append(faces.U[d] * (1.0 + rng.uniform(-amp, amp, size=faces.U[d].shape)))
    return FaceData(T=T, U=U)


def _fill_block(t, u):
    """Off-diagonal block: (0,0) = -t, the other eight = u*(-t)."""
    blk = np.empty((t.shape[0], 3, 3))
    flat = blk.reshape(-1, 9)
    flat[:, 0] = -t
    flat[:, 1:] = u * (-t)[:, None]
    return blk


def assemble(shape, active, faces: FaceData, poro=PORO, compress=COMPRESS) -> BsrCase:
    """Assemble the BSR Jacobian of the active cells from the face data."""
    nx, ny, nz = shape
    ncell = nx * ny * nz
    strides = (1, nx, nx * ny)
    act_idx = np.full(ncell, -1, dtype=np.int64)
    act_cells = np.nonzero(active)[0]
    n_b = act_cells.shape[0]
    act_idx[act_cells] = np.arange(n_b)

    # Seven slots per active cell in ascending column order:
    # z-, y-, x-, self, x+, y+, z+.
    slot_nb = np.full((n_b, 7), -1, dtype=np.int64)
    slot_blk = np.zeros((n_b, 7, 3, 3))
    diag = np.zeros((n_b, 3, 3))
    absrow = np.zeros((n_b, 3))  # sum_d sum_b |A_cd[a][b]| per row a
    for d in range(3):
        t = faces.T[d]
        has = np.nonzero(t != 0.0)[0]  # lower cell of each live face
        up = has + strides[d]
        lo_a, up_a = act_idx[has], act_idx[up]
        b_lu = _fill_block(t[has], faces.U[d][has, 0])  # A_{lo,up}
        b_ul = _fill_block(t[has], faces.U[d][has, 1])  # A_{up,lo}
        slot_nb[lo_a, 4 + d] = up_a
        slot_blk[lo_a, 4 + d] = b_lu
        slot_nb[up_a, 2 - d] = lo_a
        slot_blk[up_a, 2 - d] = b_ul
        # each active cell owns at most one face per direction and side, so
        # the index arrays below hold no duplicates
        diag[lo_a] -= b_lu
        diag[up_a] -= b_ul
        absrow[lo_a] += np.abs(b_lu).sum(axis=2)
        absrow[up_a] += np.abs(b_ul).sum(axis=2)
    diag[:, 0, 0] += poro * compress
    diag[:, 1, 1] = poro + absrow[:, 1]
    diag[:, 2, 2] = poro + absrow[:, 2]
    slot_nb[:, 3] = np.arange(n_b)
    slot_blk[:, 3] = diag

    present = slot_nb >= 0
    counts = present.sum(axis=1)
    row_ptr = np.zeros(n_b + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = slot_nb[present].astype(np.int32)
    vals = np.ascontiguousarray(slot_blk[present])
    return BsrCase(row_ptr=row_ptr.astype(np.int32), col=col, vals=vals,
                   grid=shape, active=active)


def rhs(n_dof, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n_dof)


# ---------------------------------------------------------------- named workloads
def case_small(seed=1000, shape=(20, 20, 5), sigma=1.0, kz_ratio=1.0):
    """20x20x5 grid, all cells active, i.i.d. log-normal permeability."""
    rng = np.random.default_rng(seed)
    perm = perm_iid_lognormal(shape, rng, sigma=sigma)
    active = np.ones(shape[0] * shape[1] * shape[2], dtype=bool)
    faces = make_faces(shape, perm, active, kz_ratio, rng)
    case = assemble(shape, active, faces)
    case.meta = dict(name=f"lognormal_{shape[0]}x{shape[1]}x{shape[2]}", seed=seed, sigma=sigma)
    return case


def case_spe10_like(seed=1100, shape=(60, 220, 85), sigma=2.0, kz_ratio=0.1,
                    inactive_frac=0.025, return_faces=False):
    """SPE10-sized grid, layered log-normal permeability, 2.5% inactive cells."""
    rng = np.random.default_rng(seed)
    perm = perm_layered_lognormal(shape, rng, sigma=sigma)
    active = random_mask(shape, np.random.default_rng(seed + 1), inactive_frac)
    faces = make_faces(shape, perm, active, kz_ratio, rng)
    case = assemble(shape, active, faces)
    case.meta = dict(name=f"spe10like_{shape[0]}x{shape[1]}x{shape[2]}", seed=seed,
                     sigma=sigma, kz_ratio=kz_ratio, inactive_frac=inactive_frac)
    if return_faces:
        return case, faces
    return case


def newton_sequence(n_steps=12, seed=1200, base_seed=1100, shape=(60, 220, 85), **kw):
    """Yield (step, case, b): successive Jacobians with fixed pattern and +-5% drift."""
    case, faces = case_spe10_like(seed=base_seed, shape=shape, return_faces=True, **kw)
    active = case.active
    for step in range(n_steps):
        if step > 0:
            faces = drift_faces(faces, np.random.default_rng(seed + step))
            case = assemble(shape, active, faces)
        b = rhs(case.ndof, seed + 100 + step)
        case.meta = dict(name=f"newton_step{step}", step=step)
        yield step, case, b


def case_channels(seed=1400, shape=(200, 200, 100), kz_ratio=0.01):
    """Channelised permeability (1000 mD channels on 1 mD), strong anisotropy."""
    rng = np.random.default_rng(seed)
    perm = perm_channels(shape, rng)
    active = np.ones(shape[0] * shape[1] * shape[2], dtype=bool)
    faces = make_faces(shape, perm, active, kz_ratio, rng)
    case = assemble(shape, active, faces)
    case.meta = dict(name=f"channels_{shape[0]}x{shape[1]}x{shape[2]}", seed=seed)
    return case


def serving_requests(n_req=512, seed=1300, cells_lo=1e4, cells_hi=1e6, repeat_frac=0.3):
    """Descriptors of a serving stream: grid sizes, sigma, repeats (no matrices yet)."""
    rng = np.random.default_rng(seed)
    reqs = []
    resident = []
    for r in range(n_req):
        if resident and rng.uniform() < repeat_frac:
            base = resident[int(rng.integers(len(resident)))]
            reqs.append(dict(req=r, case_id=base["case_id"], shape=base["shape"],
                             sigma=base["sigma"], seed=base["seed"],
                             drift_seed=int(seed * 1000 + r), repeat=True))
            continue
        cells = math.exp(rng.uniform(math.log(cells_lo), math.log(cells_hi)))
        nz = max(1, int(round(math.exp(rng.uniform(math.log(2), math.log(50))))))
        aspect = math.exp(rng.uniform(math.log(0.25), math.log(4.0)))
        area = cells / nz
        nx = max(2, int(round(math.sqrt(area * aspect))))
        ny = max(2, int(round(area / nx)))
        sigma = float(rng.uniform(1.0, 2.5))
        d = dict(req=r, case_id=r, shape=(nx, ny, nz), sigma=sigma,
                 seed=int(seed * 1000 + r), drift_seed=None, repeat=False)
        reqs.append(d)
        resident.append(d)
    return reqs


def serving_case(desc):
    """Materialise one serving request descriptor into (case, b)."""
    shape = tuple(desc["shape"])
    rng = np.random.default_rng(desc["seed"])
    perm = perm_iid_lognormal(shape, rng, sigma=desc["sigma"])
    active = np.ones(shape[0] * shape[1] * shape[2], dtype=bool)
    faces = make_faces(shape, perm, active, 1.0, rng)
    if desc.get("drift_seed") is not None:
        faces = drift_faces(faces, np.random.default_rng(desc["drift_seed"]))
    case = assemble(shape, active, faces)
    b = rhs(case.ndof, desc["seed"] + 7 if desc.get("drift_seed") is None else desc["drift_seed"] + 7)
    return case, b
