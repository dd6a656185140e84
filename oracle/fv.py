"""Finite-volume discretisation of the cylindrical Poisson equation (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The equation is Eq. (cylindrical_poisson) of Sec. 3.1; multiplied by r
(Eq. (mode_poisson)) and integrated over a control volume it becomes the cell
balance of App. A (Eqs. (interior_face_conductances) to
(explicit_interior_cell_balance)).  The undecomposed 3-D operator is that
radial-axial balance plus the periodic three-point azimuthal difference of
Sec. 3.1 weighted by the shift coefficient mu_q (the 3-D form that the Fourier
modes diagonalise).

Grid reading (vertex-centred): ``Nr`` radial and ``Nz`` axial nodes include the
Dirichlet faces; interior node (i, k), 1 <= i <= Nr-2, 1 <= k <= Nz-2, owns the
control volume whose faces lie half-way to its neighbours.  With uniform
spacing its centre is the node, its widths are dr and dz, and a boundary
neighbour sits one full spacing away.

General geometry (``Grid.general``, ``Grid.vertex``, ``Grid.cell_centred``):
explicit, possibly non-uniform points in r and z with the faces of every
control volume.  In the cell-centred reading of App. A the unknowns sit at
cell centres and the Dirichlet values on the outer faces, half a cell from the
first centre, which gives the half-cell boundary conductance.  Pinned by the
paper's Dirichlet worked cell, SPD/M-matrix structure, dense-vs-sparse
agreement, exact mode decomposition and measured second-order convergence.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

#: Vacuum permittivity, CODATA 2018 (F/m).  The paper does not print it.
EPS0 = 8.8541878128e-12


def cell_coefficients(r_lo, r_hi, r_c, dr, dz, d_w, d_e, d_s, d_n):
    """Coefficients of one control volume, App. A.

    Arguments: radial face radii ``r_lo = r_{i-1/2}``, ``r_hi = r_{i+1/2}``,
    centre radius ``r_c = r_i``, cell widths ``dr = r_{i+1/2} - r_{i-1/2}`` and
    ``dz = z_{k+1/2} - z_{k-1/2}`` (Eq. (cell_geometry_appendix)), and the
    centre-to-centre distances to the west, east, south and north neighbours
    (``d_w = r_i - r_{i-1}`` etc.).  Returns a dict with

    * ``G_rm, G_rp, G_zm, G_zp`` -- Eq. (interior_face_conductances):
      ``G_{r,-} = r_{i-1/2} dz_k / d_w``, ``G_{r,+} = r_{i+1/2} dz_k / d_e``,
      ``G_{z,-} = r_i dr_i / d_s``, ``G_{z,+} = r_i dr_i / d_n``;
    * ``D0`` -- their sum, Eq. (interior_base_diagonal);
    * ``mu`` -- ``dr_i dz_k / r_i``, Eq. (integrated_mode_shift);
    * ``s_eps0`` -- ``r_i dr_i dz_k`` (= s_q * eps0), Eq. (integrated_charge_rhs).

    Works elementwise on arrays.
    """
    G_rm = r_lo * dz / d_w
    G_rp = r_hi * dz / d_e
    G_zm = r_c * dr / d_s
    G_zp = r_c * dr / d_n
    return {
        "G_rm": G_rm,
        "G_rp": G_rp,
        "G_zm": G_zm,
        "G_zp": G_zp,
        "D0": G_rm + G_rp + G_zm + G_zp,
        "mu": dr * dz / r_c,
        "s_eps0": r_c * dr * dz,
    }


def charge_scale(coef):
    """``s_q = r_i dr_i dz_k / eps0``, Eq. (mode_rhs) / (integrated_charge_rhs)."""
    return coef["s_eps0"] / EPS0


class Grid:
    """Vertex-centred annular grid and its per-node coefficients.

    ``nr, nz`` count nodes including the Dirichlet faces; ``ntheta`` periodic
    nodes span 2 pi.  ``dtype`` may be ``numpy.longdouble`` for extended
    precision.  Coefficient arrays have shape ``(nz-2, nr-2)`` (interior
    nodes, r fastest); with uniform z they do not depend on k but are stored
    in full to keep the stencil code plain.
    """

    def __init__(self, nr, ntheta, nz, r_in, r_out, dz, dtype=np.float64):
        if nr < 3 or nz < 3 or ntheta < 1:
            raise ValueError("need nr >= 3, nz >= 3, ntheta >= 1")
        if not (0.0 < r_in < r_out) or not dz > 0.0:
            raise ValueError("need 0 < r_in < r_out and dz > 0")
        self.nr, self.ntheta, self.nz = int(nr), int(ntheta), int(nz)
        self.dtype = dtype
        t = dtype
        self.r_in, self.r_out, self.dz = t(r_in), t(r_out), t(dz)
        self.dr = (self.r_out - self.r_in) / t(nr - 1)
        self.dtheta = t(2) * np.arccos(t(-1)) / t(ntheta)
        self.r = self.r_in + self.dr * np.arange(nr, dtype=t)
        self.z = self.dz * np.arange(nz, dtype=t)
        # Interior node centres.  Uniform spacing: the control volume of node i
        # has faces at r_i -/+ dr/2 and widths dr, dz; every neighbour (boundary
        # nodes included) is one full spacing away.
        R = self.r[None, 1:-1] * np.ones((nz - 2, 1), dtype=t)
        half = t(0.5)
        c = cell_coefficients(R - half * self.dr, R + half * self.dr, R, self.dr, self.dz,
                              self.dr, self.dr, self.dz, self.dz)
        self.coef = c
        self.G_rm, self.G_rp = c["G_rm"], c["G_rp"]
        self.G_zm, self.G_zp = c["G_zm"], c["G_zp"]
        self.D0, self.mu = c["D0"], c["mu"]
        self.s_eps0 = c["s_eps0"]

        self.uniform = True

    @classmethod
    def of(cls, problem, dtype=np.float64):
        p = problem
        return cls(p.nr, p.ntheta, p.nz, p.r_in, p.r_out, p.dz, dtype=dtype)

    @classmethod
    def general(cls, r, z, r_lo, r_hi, z_lo, z_hi, ntheta, dtype=np.float64):
        """Grid from explicit geometry (App. A with general spacing).

        ``r`` (nr) and ``z`` (nz) are the points, boundary points included;
        ``r_lo, r_hi`` (nr - 2) and ``z_lo, z_hi`` (nz - 2) are the faces of the
        control volume of each interior point.  Conductances use the distances
        between neighbouring points, so a boundary point on a face gives the
        half-cell Dirichlet conductance of Eq. (dirichlet_face_conductances).
        """
        t = dtype
        g = cls.__new__(cls)
        r = np.asarray(r, dtype=t)
        z = np.asarray(z, dtype=t)
        nr, nz = len(r), len(z)
        if nr < 3 or nz < 3 or ntheta < 1:
            raise ValueError("need nr >= 3, nz >= 3, ntheta >= 1")
        if not (r[0] > 0 and np.all(np.diff(r) > 0) and np.all(np.diff(z) > 0)):
            raise ValueError("need 0 < r[0] and increasing points")
        g.nr, g.ntheta, g.nz, g.dtype = nr, int(ntheta), nz, dtype
        g.r, g.z = r, z
        g.r_in, g.r_out = r[0], r[-1]
        g.dr = g.dz = None  # no single spacing
        g.dtheta = t(2) * np.arccos(t(-1)) / t(ntheta)
        R = np.broadcast_to(r[None, 1:-1], (nz - 2, nr - 2))
        rlo = np.broadcast_to(np.asarray(r_lo, dtype=t)[None, :], R.shape)
        rhi = np.broadcast_to(np.asarray(r_hi, dtype=t)[None, :], R.shape)
        zlo = np.asarray(z_lo, dtype=t)[:, None]
        zhi = np.asarray(z_hi, dtype=t)[:, None]
        d_w = (r[1:-1] - r[:-2])[None, :]
        d_e = (r[2:] - r[1:-1])[None, :]
        d_s = (z[1:-1] - z[:-2])[:, None]
        d_n = (z[2:] - z[1:-1])[:, None]
        c = cell_coefficients(rlo, rhi, R, rhi - rlo, zhi - zlo, d_w, d_e, d_s, d_n)
        c = {k: np.broadcast_to(v, R.shape).copy() for k, v in c.items()}
        g.coef = c
        g.G_rm, g.G_rp = c["G_rm"], c["G_rp"]
        g.G_zm, g.G_zp = c["G_zm"], c["G_zp"]
        g.D0, g.mu = c["D0"], c["mu"]
        g.s_eps0 = c["s_eps0"]
        g.uniform = False
        return g

    @classmethod
    def vertex(cls, r, z, ntheta, dtype=np.float64):
        """Vertex-centred grid on the given (possibly non-uniform) points: the
        control-volume faces lie halfway between neighbouring points."""
        r = np.asarray(r, dtype=dtype)
        z = np.asarray(z, dtype=dtype)
        h = dtype(0.5)
        return cls.general(r, z, h * (r[:-2] + r[1:-1]), h * (r[1:-1] + r[2:]),
                           h * (z[:-2] + z[1:-1]), h * (z[1:-1] + z[2:]), ntheta, dtype)

    @classmethod
    def cell_centred(cls, r_faces, z_faces, ntheta, dtype=np.float64):
        """Cell-centred grid (App. A): cells between the given faces, unknowns at
        the cell centres (face midpoints), Dirichlet values on the outer faces,
        which are the boundary points (half a cell from the first centres)."""
        rf = np.asarray(r_faces, dtype=dtype)
        zf = np.asarray(z_faces, dtype=dtype)
        h = dtype(0.5)
        r = np.concatenate([rf[:1], h * (rf[:-1] + rf[1:]), rf[-1:]])
        z = np.concatenate([zf[:1], h * (zf[:-1] + zf[1:]), zf[-1:]])
        return cls.general(r, z, rf[:-1], rf[1:], zf[:-1], zf[1:], ntheta, dtype)

    @property
    def interior_shape(self):
        return (self.ntheta, self.nz - 2, self.nr - 2)

    @property
    def shape(self):
        return (self.ntheta, self.nz, self.nr)

    @property
    def n_unknowns(self):
        return self.ntheta * (self.nz - 2) * (self.nr - 2)

    def theta_coupling(self):
        """Azimuthal conductance ``mu_q / dtheta^2`` of the 3-D operator (Sec. 3.1)."""
        return self.mu / (self.dtheta * self.dtheta)


def boundary_values(grid: Grid, bc) -> np.ndarray:
    """Full node array holding the Dirichlet values on boundary nodes, zero inside.

    ``bc = (phi_r_in, phi_r_out, phi_z0, phi_zL)``; the axial faces win at the
    (r, z) corners, which never enter the stencil.
    """
    phi = np.zeros(grid.shape, dtype=grid.dtype)
    phi[:, :, 0] = bc[0]
    phi[:, :, -1] = bc[1]
    phi[:, 0, :] = bc[2]
    phi[:, -1, :] = bc[3]
    return phi


def apply_full(grid: Grid, phi: np.ndarray) -> np.ndarray:
    """``(A_full phi)_q`` at every interior node, boundary nodes included as neighbours.

    This is the left-hand side of Eq. (explicit_interior_cell_balance) with the
    azimuthal three-point term added: ``(D0 + 2 mu/dtheta^2) u_q - G_{r,-} u_W
    - G_{r,+} u_E - G_{z,-} u_S - G_{z,+} u_N - mu/dtheta^2 (u_{j-1} + u_{j+1})``.
    Evaluated in ``grid.dtype``.  Result shape ``(ntheta, nz-2, nr-2)``.
    """
    u = np.asarray(phi, dtype=grid.dtype)
    c = u[:, 1:-1, 1:-1]
    gt = grid.theta_coupling()
    out = (grid.D0 + 2 * gt) * c
    out = out - grid.G_rm * u[:, 1:-1, :-2]
    out = out - grid.G_rp * u[:, 1:-1, 2:]
    out = out - grid.G_zm * u[:, :-2, 1:-1]
    out = out - grid.G_zp * u[:, 2:, 1:-1]
    out = out - gt * (np.roll(c, 1, axis=0) + np.roll(c, -1, axis=0))
    return out


def charge_from_potential(grid: Grid, phi: np.ndarray) -> np.ndarray:
    """The charge density whose discrete solution is ``phi``: ``rho = (A_full phi)/s_q``.

    Returned as a full node array (boundary nodes zero) in ``grid.dtype``;
    pass an extended-precision grid to round only once when casting to FP64.
    """
    rho = np.zeros(grid.shape, dtype=grid.dtype)
    rho[:, 1:-1, 1:-1] = apply_full(grid, phi) * grid.dtype(EPS0) / grid.s_eps0
    return rho


def unknown_index(grid: Grid, j, k, i):
    """Linear index of interior node (j, k, i) with 1 <= k <= nz-2, 1 <= i <= nr-2."""
    return (j * (grid.nz - 2) + (k - 1)) * (grid.nr - 2) + (i - 1)


def assemble(grid: Grid) -> sp.csr_matrix:
    """The undecomposed 3-D matrix A on interior unknowns (Sec. 3.1, App. A).

    Row q: diagonal ``D0 + 2 mu/dtheta^2``; ``-G`` to each interior radial and
    axial neighbour; ``-mu/dtheta^2`` to the two azimuthal neighbours (periodic;
    for ntheta = 1 or 2 they coincide and the entries add).  Couplings to
    boundary nodes are not in A: they go to the right-hand side.
    """
    if grid.dtype is not np.float64:
        raise TypeError("assemble() builds a float64 matrix")
    nt, nz, nr = grid.ntheta, grid.nz, grid.nr
    J, K, I = np.meshgrid(np.arange(nt), np.arange(1, nz - 1), np.arange(1, nr - 1), indexing="ij")
    row = unknown_index(grid, J, K, I)
    gt = grid.theta_coupling()
    bshape = (nt, 1, 1)
    rows, cols, vals = [], [], []

    def add(mask, col, val):
        rows.append(row[mask])
        cols.append(col[mask])
        vals.append(np.broadcast_to(val, row.shape)[mask])

    everywhere = np.ones(row.shape, dtype=bool)
    add(everywhere, row, np.tile((grid.D0 + 2 * gt)[None], bshape))
    add(I > 1, unknown_index(grid, J, K, I - 1), -np.tile(grid.G_rm[None], bshape))
    add(I < nr - 2, unknown_index(grid, J, K, I + 1), -np.tile(grid.G_rp[None], bshape))
    add(K > 1, unknown_index(grid, J, K - 1, I), -np.tile(grid.G_zm[None], bshape))
    add(K < nz - 2, unknown_index(grid, J, K + 1, I), -np.tile(grid.G_zp[None], bshape))
    add(everywhere, unknown_index(grid, (J + 1) % nt, K, I), -np.tile(gt[None], bshape))
    add(everywhere, unknown_index(grid, (J - 1) % nt, K, I), -np.tile(gt[None], bshape))
    n = grid.n_unknowns
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return A.tocsr()  # duplicate (row, col) pairs are summed


def rhs(grid: Grid, rho: np.ndarray, phi_boundary: np.ndarray) -> np.ndarray:
    """Right-hand side ``b = s_q rho_q + b^D_q`` on interior nodes, Eq. (full_finite_volume_row).

    ``rho`` and ``phi_boundary`` are full node arrays; only interior values of
    ``rho`` and only boundary values of ``phi_boundary`` are read.  ``b^D``
    collects ``G * phi`` over the boundary neighbours of each node,
    Eq. (boundary_rhs_appendix).  Shape ``(ntheta, nz-2, nr-2)``.
    """
    t = grid.dtype
    rho = np.asarray(rho, dtype=t)
    pb = np.asarray(phi_boundary, dtype=t)
    b = grid.s_eps0 * rho[:, 1:-1, 1:-1] / t(EPS0)
    b = b.copy()
    b[:, :, 0] += grid.G_rm[:, 0] * pb[:, 1:-1, 0]
    b[:, :, -1] += grid.G_rp[:, -1] * pb[:, 1:-1, -1]
    b[:, 0, :] += grid.G_zm[0, :] * pb[:, 0, 1:-1]
    b[:, -1, :] += grid.G_zp[-1, :] * pb[:, -1, 1:-1]
    return b


def with_boundary(grid: Grid, u_interior: np.ndarray, phi_boundary: np.ndarray) -> np.ndarray:
    """Full potential: interior unknowns plus the boundary node values."""
    phi = np.array(phi_boundary, dtype=grid.dtype, copy=True)
    phi[:, 1:-1, 1:-1] = np.asarray(u_interior).reshape(grid.interior_shape)
    return phi
