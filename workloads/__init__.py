"""Seeded synthetic inputs for the full-spectrum cylindrical Poisson solve.

This module only *generates inputs*: grid descriptions, manufactured
potentials and charge densities drawn from a seed.  It contains none of the
solver's arithmetic (no finite-volume coefficient, operator, transform or
eigenvalue), so that both the CPU oracle and the GPU library can consume the
same arrays without sharing any of the method's code.

Arrays are C-contiguous ``[Ntheta][Nz][Nr]`` float64 (r fastest), node values
of an annular grid:

* ``Nr`` radial nodes ``r_i = r_in + i (r_out - r_in)/(Nr - 1)`` including both
  radial Dirichlet faces,
* ``Nz`` axial nodes ``z_k = k dz`` including both axial Dirichlet faces,
* ``Ntheta`` periodic azimuthal nodes ``theta_j = 2 pi j / Ntheta``.

The paper's production inputs are not published, so these generators stand in
for them (the cylindrical Hall-thruster geometry of Sec. 2 and the grid sizes
of Sec. 5.1 / Table "evaluation matrix").
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem",
    "SMALL",
    "BATCHED",
    "PAPER_SCALE",
    "HIGH_SHIFT",
    "node_coordinates",
    "manufactured_potential",
    "blob_charge",
    "random_problems",
    "stretched_points",
    "mesh_blob_charge",
    "cell_centres",
    "blob_field",
    "sequence_plan",
]


@dataclasses.dataclass(frozen=True)
class Problem:
    """One annular grid with theta-invariant Dirichlet face values (volts)."""

    nr: int
    ntheta: int
    nz: int
    r_in: float
    r_out: float
    dz: float
    phi_r_in: float = 0.0
    phi_r_out: float = 0.0
    phi_z0: float = 0.0
    phi_zL: float = 300.0
    name: str = ""

    @property
    def length(self) -> float:
        return self.dz * (self.nz - 1)

    @property
    def shape(self) -> tuple[int, int, int]:
        return (self.ntheta, self.nz, self.nr)

    @property
    def bc(self) -> tuple[float, float, float, float]:
        return (self.phi_r_in, self.phi_r_out, self.phi_z0, self.phi_zL)

    @property
    def unknowns(self) -> int:
        return self.ntheta * (self.nz - 2) * (self.nr - 2)

    @property
    def nodes(self) -> int:
        return self.ntheta * self.nz * self.nr

    def with_sizes(self, nr: int, ntheta: int, nz: int, name: str = "") -> "Problem":
        """Same physical annulus and boundary values, resampled on another grid."""
        return dataclasses.replace(
            self, nr=nr, ntheta=ntheta, nz=nz, dz=self.length / (nz - 1), name=name or self.name
        )


_R_IN, _R_OUT, _L = 0.02, 0.05, 0.05

#: 33 x 16 x 33 nodes; the sparse direct oracle finishes in about a second.
SMALL = Problem(33, 16, 33, _R_IN, _R_OUT, _L / 32, name="small-33x16x33")
#: 129 x 64 x 129 nodes (33 real-FFT modes).
BATCHED = Problem(129, 64, 129, _R_IN, _R_OUT, _L / 128, name="batched-129x64x129")
#: 400 x 128 x 512 nodes (65 real-FFT modes): the paper-scale grid
#: (26,214,400 nodes, the logical cell count of the paper's fine case).
PAPER_SCALE = Problem(400, 128, 512, _R_IN, _R_OUT, _L / 511, name="paper-400x128x512")
#: A geometry where the azimuthal shift dominates the diagonal near r_in, so a
#: wrong eigenvalue or plane assignment changes the answer visibly.
HIGH_SHIFT = Problem(33, 64, 33, 1e-3, _R_OUT, _L / 32, name="high-shift-33x64x33")


def node_coordinates(p: Problem) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Node coordinates (theta, z, r) of the grid, as 1-D float64 arrays."""
    r = p.r_in + (p.r_out - p.r_in) * np.arange(p.nr, dtype=np.float64) / (p.nr - 1)
    z = p.dz * np.arange(p.nz, dtype=np.float64)
    th = 2.0 * math.pi * np.arange(p.ntheta, dtype=np.float64) / p.ntheta
    return th, z, r


def _boundary_faces(p: Problem, phi: np.ndarray) -> np.ndarray:
    """Overwrite boundary nodes with the face values; axial faces win at corners."""
    phi[:, :, 0] = p.phi_r_in
    phi[:, :, -1] = p.phi_r_out
    phi[:, 0, :] = p.phi_z0
    phi[:, -1, :] = p.phi_zL
    return phi


def _blob_draws(p: Problem, seed: int):
    """The seeded draws of manufactured_potential, in its order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = p.r_out - p.r_in
    length = p.length
    h1 = w / 32.0
    blobs = []
    for _ in range(4):
        a = rng.uniform(-1.0, 1.0)
        rb = rng.uniform(p.r_in + 0.2 * w, p.r_out - 0.2 * w)
        zb = rng.uniform(0.2 * length, 0.8 * length)
        sig = rng.uniform(2.0, 5.0) * h1
        cd = rng.uniform(-1.0, 1.0, size=6)
        blobs.append((a, rb, zb, sig, cd))
    return blobs


def _add_blobs(p: Problem, seed: int, dtype, out: np.ndarray) -> np.ndarray:
    """out + sum_b a_b g_b(r, z) [1 + sum_m (c_bm cos m theta + d_bm sin m theta)]
    at every node, the blobs added to ``out`` one after another."""
    th, z, r = (np.asarray(c, dtype=dtype) for c in node_coordinates(p))
    T = th[:, None, None]
    Z = z[None, :, None]
    R = r[None, None, :]
    for a, rb, zb, sig, cd in _blob_draws(p, seed):
        g = np.exp(-((R - dtype(rb)) ** 2 + (Z - dtype(zb)) ** 2) / dtype(2.0 * sig * sig))
        ang = np.ones_like(T)
        for m in range(1, 4):
            ang = ang + dtype(cd[2 * m - 2]) * np.cos(m * T) + dtype(cd[2 * m - 1]) * np.sin(m * T)
        out = out + dtype(a) * g * ang
    return out


def blob_field(p: Problem, seed: int) -> np.ndarray:
    """The blob part of ``manufactured_potential(p, seed)`` (no axial background)
    on the interior nodes, zero on the boundary nodes, scaled to unit RMS over
    the interior: one seeded drift direction of a time sequence whose exact
    answers stay known (the potential moves by multiples of such fields)."""
    f = _add_blobs(p, seed, np.float64, np.zeros(p.shape))
    f[:, 0, :] = f[:, -1, :] = 0.0
    f[:, :, 0] = f[:, :, -1] = 0.0
    f /= np.sqrt(np.mean(f[:, 1:-1, 1:-1] ** 2))
    return np.ascontiguousarray(f)


def manufactured_potential(p: Problem, seed: int = 12345, dtype=np.float64) -> np.ndarray:
    """A seeded smooth potential phi_true at every node (volts).

    ``phi_true = phi_zL * z / L + sum_b a_b g_b(r, z) [1 + sum_{m=1..3}
    (c_bm cos m theta + d_bm sin m theta)]`` with four Gaussian blobs ``g_b``.
    Draws (``numpy.random.Generator(PCG64(seed))``), per blob in order:
    amplitude ``a ~ U(-1, 1)``, centre ``r_b ~ U(r_in + 0.2 W, r_out - 0.2 W)``,
    ``z_b ~ U(0.2 L, 0.8 L)``, width ``sigma = U(2, 5) * W / 32`` and the six
    harmonic amplitudes ``c_1, d_1, c_2, d_2, c_3, d_3 ~ U(-1, 1)``.  Widths
    are physical (tied to the 33-node radial spacing), so a finer grid samples
    the same function.  Boundary nodes carry the Dirichlet face values.

    ``dtype`` may be ``numpy.longdouble`` to evaluate in extended precision.
    """
    _, z, _ = (np.asarray(c, dtype=dtype) for c in node_coordinates(p))
    Z = z[None, :, None]
    phi = np.zeros(p.shape, dtype=dtype) + dtype(p.phi_zL) * Z / dtype(p.length)
    return _boundary_faces(p, _add_blobs(p, seed, dtype, phi))


def _inside(lo: float, hi: float, margin: float) -> tuple[float, float]:
    """Interval [lo + margin, hi - margin], collapsed to its midpoint on tiny grids."""
    a, b = lo + margin, hi - margin
    if a > b:
        a = b = 0.5 * (lo + hi)
    return a, b


def blob_charge(p: Problem, seed: int = 24680) -> np.ndarray:
    """A seeded particle-like charge density rho (C/m^3) at every node.

    Eight 3-D Gaussian clouds of charge ``q_b ~ U(-1, 1) * 1e-4`` C/m^3 (about
    1% of e * 5e16 m^-3, the paper's reference plasma density), radial and
    axial widths ``U(2, 5)`` cells, azimuthal width ``U(2, 5)`` cells (periodic
    distance), centres at least three widths from the radial and axial faces;
    the sum is modulated by ``1 + sum_{m=1..8} eps_m cos(m theta + psi_m)``
    (``eps_m ~ U(0, 0.1)``, ``psi_m ~ U(0, 2 pi)``) as azimuthal spokes, then
    white noise of relative amplitude 1e-3 (a particle-noise proxy) is added.
    Boundary nodes are zero (they are not read by the solve).
    """
    th, z, r = node_coordinates(p)
    dr = (p.r_out - p.r_in) / (p.nr - 1)
    return _blob_charge(th, z, r, (p.r_in, p.r_out), (0.0, p.length), dr, p.dz, seed)


def _blob_charge(th, z, r, r_span, z_span, dr, dz, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    dth = 2.0 * math.pi / len(th)
    T = th[:, None, None]
    Z = z[None, :, None]
    R = r[None, None, :]
    shape = (len(th), len(z), len(r))
    rho = np.zeros(shape)
    for _ in range(8):
        q = rng.uniform(-1.0, 1.0) * 1e-4
        sr = rng.uniform(2.0, 5.0) * dr
        sz = rng.uniform(2.0, 5.0) * dz
        st = rng.uniform(2.0, 5.0) * dth
        rc = rng.uniform(*_inside(r_span[0], r_span[1], 3 * sr))
        zc = rng.uniform(*_inside(z_span[0], z_span[1], 3 * sz))
        tc = rng.uniform(0.0, 2.0 * math.pi)
        dt = np.angle(np.exp(1j * (T - tc)))  # periodic distance in (-pi, pi]
        rho += q * np.exp(-0.5 * (((R - rc) / sr) ** 2 + (dt / st) ** 2 + ((Z - zc) / sz) ** 2))
    spokes = np.ones_like(T)
    for m in range(1, 9):
        eps_m = rng.uniform(0.0, 0.1)
        psi_m = rng.uniform(0.0, 2.0 * math.pi)
        spokes = spokes + eps_m * np.cos(m * T + psi_m)
    rho = rho * spokes
    rho = rho + 1e-3 * np.abs(rho).max() * rng.standard_normal(shape)
    rho[:, :, 0] = rho[:, :, -1] = 0.0
    rho[:, 0, :] = rho[:, -1, :] = 0.0
    return np.ascontiguousarray(rho)


def stretched_points(a: float, b: float, n: int, beta: float) -> np.ndarray:
    """n + 1 increasing points from a to b whose intervals grow geometrically by
    the factor beta (beta = 1: uniform; beta < 1 refines towards b).  A mesh
    generator for the non-uniform grids of App. A (boundary-layer refinement)."""
    if beta == 1.0:
        return np.linspace(a, b, n + 1)
    w = beta ** np.arange(n)
    x = a + (b - a) * np.concatenate([[0.0], np.cumsum(w) / w.sum()])
    x[-1] = b
    return x


def cell_centres(faces) -> np.ndarray:
    """Node coordinates of a cell-centred direction with the given faces: the
    first face, the cell midpoints, the last face (where the Dirichlet values sit)."""
    f = np.asarray(faces, dtype=np.float64)
    return np.concatenate([f[:1], 0.5 * (f[:-1] + f[1:]), f[-1:]])


def mesh_blob_charge(r, z, ntheta: int, seed: int = 24680) -> np.ndarray:
    """``blob_charge`` on explicit node coordinates r (Nr) and z (Nz): widths in
    units of the median node spacings, centres inside [r[0], r[-1]] x [z[0], z[-1]]."""
    r = np.asarray(r, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    th = 2.0 * math.pi * np.arange(ntheta, dtype=np.float64) / ntheta
    dr = float(np.median(np.diff(r)))
    dz = float(np.median(np.diff(z)))
    return _blob_charge(th, z, r, (float(r[0]), float(r[-1])), (float(z[0]), float(z[-1])), dr, dz, seed)


def random_problems(count: int = 16, seed: int = 24680) -> list[Problem]:
    """Uneven annular grids: Nr ~ U{65..401}, Ntheta in {32, 64, 128}, Nz ~ U{65..513}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        nr = int(rng.integers(65, 402))
        nt = int(rng.choice([32, 64, 128]))
        nz = int(rng.integers(65, 514))
        out.append(SMALL.with_sizes(nr, nt, nz, name=f"uneven-{i}-{nr}x{nt}x{nz}"))
    return out


def drift_fields(p: Problem, count: int = 8, seed: int = 97531) -> list[np.ndarray]:
    """Smooth seeded charge perturbations for a time sequence of solves: each is
    sin(a pi (r - r_in)/W) * sin(b pi z/L) * cos(m theta + psi) with a, b in
    1..4, m in 0..8 and psi in [0, 2 pi), scaled to max |.| = 1, zero on the
    boundary nodes.  Separable, so cheap at any size."""
    rng = np.random.Generator(np.random.PCG64(seed))
    th, z, r = node_coordinates(p)
    W_, L_ = p.r_out - p.r_in, p.length
    out = []
    for _ in range(count):
        a, b = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        m, psi = int(rng.integers(0, 9)), float(rng.uniform(0.0, 2.0 * math.pi))
        fr = np.sin(a * math.pi * (r - p.r_in) / W_)
        fz = np.sin(b * math.pi * z / L_)
        ft = np.cos(m * th + psi)
        f = ft[:, None, None] * fz[None, :, None] * fr[None, None, :]
        f /= np.abs(f).max()
        f[:, :, 0] = f[:, :, -1] = 0.0
        f[:, 0, :] = f[:, -1, :] = 0.0
        out.append(np.ascontiguousarray(f))
    return out


def sequence_plan(steps: int = 200, fields: int = 8, seed: int = 97531) -> tuple[np.ndarray, np.ndarray]:
    """Which of ``fields`` seeded blob fields (seeds seed .. seed + fields - 1)
    drifts the potential at each step of a time sequence, and with which sign:
    step t adds sign[t] * 0.01 * rms(blob part of phi_true) * blob_field(seed + k[t])."""
    rng = np.random.Generator(np.random.PCG64(seed + 2))
    return rng.integers(0, fields, size=steps), rng.choice(np.array([-1.0, 1.0]), size=steps)


def drift_signs(steps: int = 200, seed: int = 97531) -> np.ndarray:
    """Seeded +-1 signs of the per-step perturbations of a time sequence."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return rng.choice(np.array([-1.0, 1.0]), size=steps)
