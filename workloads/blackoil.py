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


def add_wells(case: BsrCase, columns, seed, well_index=5.0, frac_hi=0.5, u=U_COUPLING) -> BsrCase:
    """Append implicit wells to a reservoir Jacobian: the [A_RR A_RW; A_WR A_WW]
    system of the paper's Section 2.2, one bottom-hole-pressure unknown per
    well, each well stored as an extra 3x3 block row after the cells so the
    matrix stays 3x3-block (slots 1 and 2 of a well are placeholder unknowns
    with identity equations).

    A well perforates every active cell of a vertical grid column (ix, iy);
    the columns must be distinct.  Its productivity at cell c is PI_c =
    well_index * (mean transmissibility of c's faces).  Cell c gains the
    block A_cw with column 0 = -PI_c * (1, f1, f2), f_a ~ U[0, frac_hi], and
    the matching diagonal terms (D[0][0] += PI_c, D[a][0] += PI_c f_a, and
    D[a][a] += PI_c f_a so the saturation rows stay dominant); the well row
    has A_wc[0, :] = -PI_c * (1, u1, u2), u ~ U[-u, u], and A_ww =
    diag(sum_c PI_c, 1, 1) (a rate-controlled well equation).  Random draws
    are taken well by well, perforation by perforation (f1, f2, u1, u2)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = case.grid
    n_b = case.n_b
    rp = case.row_ptr.astype(np.int64)
    col = case.col.astype(np.int64)
    act_idx = np.full(nx * ny * nz, -1, dtype=np.int64)
    act_idx[np.nonzero(case.active)[0]] = np.arange(n_b)
    rowlen = np.diff(rp)
    row_of = np.repeat(np.arange(n_b), rowlen)
    offd = col != row_of
    mean_t = np.bincount(row_of[offd], weights=-case.vals[offd, 0, 0], minlength=n_b) / np.maximum(rowlen - 1, 1)
    diag_pos = np.nonzero(~offd)[0]  # one diagonal block per row, in row order
    perfs = []
    for ix, iy in columns:
        cells = act_idx[ix + nx * (iy + ny * np.arange(nz))]
        perfs.append(cells[cells >= 0])
    all_cells = np.concatenate(perfs) if perfs else np.zeros(0, dtype=np.int64)
    if np.unique(all_cells).size != all_cells.size:
        raise ValueError("well columns must be distinct")
    n_w = len(perfs)
    extra = np.zeros(n_b, dtype=np.int64)
    extra[all_cells] = 1
    # new layout: the cell rows (old entries, then the well entry), then the well rows
    new_len = np.concatenate([rowlen + extra, [p.size + 1 for p in perfs]]).astype(np.int64)
    new_rp = np.zeros(n_b + n_w + 1, dtype=np.int64)
    np.cumsum(new_len, out=new_rp[1:])
    new_col = np.empty(new_rp[-1], dtype=np.int64)
    new_vals = np.zeros((new_rp[-1], 3, 3))
    old_pos = new_rp[row_of] + (np.arange(rp[-1]) - rp[row_of])
    new_col[old_pos] = col
    new_vals[old_pos] = case.vals
    for w, cells in enumerate(perfs):
        wi = n_b + w
        draws = rng.uniform(size=(cells.size, 4))
        f = frac_hi * draws[:, :2]
        uu = u * (2.0 * draws[:, 2:] - 1.0)
        pi = well_index * mean_t[cells]
        pos = new_rp[cells] + rowlen[cells]  # the last entry of each perforated row
        new_col[pos] = wi
        new_vals[pos, 0, 0] = -pi
        new_vals[pos, 1, 0] = -pi * f[:, 0]
        new_vals[pos, 2, 0] = -pi * f[:, 1]
        dp = old_pos[diag_pos[cells]]
        new_vals[dp, 0, 0] += pi
        new_vals[dp, 1, 0] += pi * f[:, 0]
        new_vals[dp, 2, 0] += pi * f[:, 1]
        new_vals[dp, 1, 1] += pi * f[:, 0]
        new_vals[dp, 2, 2] += pi * f[:, 1]
        base = new_rp[wi]
        new_col[base:base + cells.size] = cells
        new_vals[base:base + cells.size, 0, 0] = -pi
        new_vals[base:base + cells.size, 0, 1] = -pi * uu[:, 0]
        new_vals[base:base + cells.size, 0, 2] = -pi * uu[:, 1]
        new_col[base + cells.size] = wi
        new_vals[base + cells.size] = np.diag([pi.sum(), 1.0, 1.0])
    return BsrCase(row_ptr=new_rp.astype(np.int32), col=new_col.astype(np.int32), vals=new_vals, grid=case.grid,
                   active=case.active, meta=dict(case.meta, wells=[tuple(c) for c in columns]))


def five_spot(shape):
    """Well columns of a five-spot pattern: four corners (one cell in from the
    edges) and the centre."""
    nx, ny, _ = shape
    return [(1, 1), (nx - 2, 1), (1, ny - 2), (nx - 2, ny - 2), (nx // 2, ny // 2)]


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


def newton_sequence(n_steps=12, seed=1200, base_seed=1100, shape=(60, 220, 85), amp=0.05, **kw):
    """Yield (step, case, b): successive Jacobians with fixed pattern and +-amp
    (default 5%) multiplicative drift per step."""
    case, faces = case_spe10_like(seed=base_seed, shape=shape, return_faces=True, **kw)
    active = case.active
    for step in range(n_steps):
        if step > 0:
            faces = drift_faces(faces, np.random.default_rng(seed + step), amp=amp)
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
