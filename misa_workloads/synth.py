"""Seeded synthetic inputs for the EAM lattice workloads.

Workload recipe (shared by tests, smoke and bench):

* BCC lattice of ``n x n x n`` cubic cells, lattice constant ``a`` (Angstrom),
  periodic orthorhombic box ``L = n * a`` per axis.  Atom ``i`` of the
  generated arrays has atom id ``i``; corner sites come first (cell order
  x fastest), then body-centre sites.  This order deliberately differs from
  the lattice-id order the method uses internally.
* Gaussian displacements, ``sigma`` Angstrom per component.
* Maxwell velocities at temperature ``T``: each component ~ N(0, kB T C / m),
  centre-of-mass velocity removed, then rescaled so that the kinetic
  temperature with ``3 (N - 1)`` degrees of freedom is exactly ``T``.
* Recoil atoms (primary knock-on atoms): the atom nearest the box centre, or
  ``k`` atoms drawn uniformly; direction uniform on the sphere from three
  seeded normals; speed ``sqrt(2 E C / m)``; the recoil velocity replaces the
  thermal one.
* Random numbers come from ``numpy.random.Generator(PCG64)`` children of one
  ``SeedSequence(seed)``: [displacements, velocities, recoil atoms, recoil
  directions].

Units: Angstrom, eV, fs, amu.  ``C`` converts eV/(Angstrom amu) to
Angstrom/fs^2 and is built from the exact SI elementary charge and the
CODATA-2018 atomic mass unit.

The synthetic potential (a stand-in for a tabulated Fe potential):
``f(r) = exp(-3 (r / 2.47 - 1))``,
``phi(r) = 0.4 [exp(-3.2 (r - 2.5)) - 2 exp(-1.6 (r - 2.5))]`` eV (Morse),
``F(rho) = -sqrt(rho)`` eV, tabulated at 5000 equidistant points:
f and phi on ``[0, rc]`` (last node exactly at rc), F on ``[0, RHO_MAX]``.
The shifted-force variant replaces ``g`` in {f, phi} by
``g(r) - g(rc) - (r - rc) g'(rc)`` so both vanish smoothly at the cut-off.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

A_FE = 2.855            # lattice constant [Angstrom]
RC = 5.0                # cut-off radius [Angstrom]
DELTA = 0.6             # slot tolerance: atoms farther than this from their site leave the lattice [Angstrom]
MASS_FE = 55.845        # [amu]
KB_EV = 8.617333262e-5  # Boltzmann constant [eV/K]
ACC_A_FS2 = (1.602176634e-19 / 1.66053906660e-27) * 1e-10  # 1 eV/(Angstrom amu) in Angstrom/fs^2
N_TABLE = 5000          # samples per potential function
RHO_MAX = 61.8          # upper end of the embedding-function grid (about 4x the perfect-lattice density)

# analytic potential parameters: f(r) = exp(-F_BETA (r / F_RE - 1));
# phi(r) = M_D [exp(-2 M_ALPHA (r - M_R0)) - 2 exp(-M_ALPHA (r - M_R0))];  F(rho) = -EMB_A sqrt(rho)
F_BETA, F_RE = 3.0, 2.47
M_D, M_ALPHA, M_R0 = 0.4, 1.6, 2.5
EMB_A = 1.0


def analytic_potential_params() -> dict:
    """Parameters of the synthetic analytic EAM (same numbers the sample arrays use)."""
    return dict(f_beta=F_BETA, f_re=F_RE, m_d=M_D, m_alpha=M_ALPHA, m_r0=M_R0, emb_a=EMB_A)


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n_cells: int
    precision: str          # "fp64" or "fp32" pair arithmetic
    steps: int
    dt_max: float           # fs
    dx_max: float           # Angstrom per step; 0 = fixed dt
    n_recoils: int
    recoil_ev: float
    recoil_at_centre: bool
    seed: int
    temperature: float = 300.0
    sigma: float = 0.02

    @property
    def n_atoms(self) -> int:
        return 2 * self.n_cells ** 3


CONFIGS = {
    "c1": Config("c1-bcc16-fp64", 16, "fp64", 100, 1.0, 0.0, 0, 0.0, False, 1000),
    "c2": Config("c2-bcc128-recoil1kev", 128, "fp64", 1000, 1.0, 0.05, 1, 1000.0, True, 1001),
    "c3": Config("c3-bcc320-fp32-5recoils", 320, "fp32", 500, 1.0, 0.05, 5, 2000.0, False, 1002),
}


def bcc_positions(n: tuple[int, int, int] | int, a: float = A_FE) -> np.ndarray:
    """Perfect BCC site positions, shape (2 nx ny nz, 3): corners, then body centres."""
    if isinstance(n, int):
        n = (n, n, n)
    nx, ny, nz = n
    gz, gy, gx = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nx, dtype=np.float64), indexing="ij")
    corner = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    pos = np.concatenate([corner, corner + 0.5], axis=0)
    pos *= a
    return pos


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(c)) for c in ss.spawn(4)]


def thermal_state(n, a=A_FE, temperature=300.0, sigma=0.02, mass=MASS_FE, seed=0):
    """Displaced BCC crystal with Maxwell velocities rescaled to exactly ``temperature``.

    Returns (x, v, box) with x, v of shape (N, 3) float64 and box = (Lx, Ly, Lz).
    """
    if isinstance(n, int):
        n = (n, n, n)
    rd, rv, _, _ = _streams(seed)
    x = bcc_positions(n, a)
    N = x.shape[0]
    if sigma > 0:
        x += rd.normal(0.0, sigma, size=x.shape)
    v = np.zeros_like(x)
    if temperature > 0 and N > 1:
        v = rv.normal(0.0, math.sqrt(KB_EV * temperature * ACC_A_FS2 / mass), size=x.shape)
        v -= v.mean(axis=0)
        ke = 0.5 * mass * float(np.einsum("ij,ij->", v, v)) / ACC_A_FS2
        t_now = 2.0 * ke / (3.0 * (N - 1) * KB_EV)
        v *= math.sqrt(temperature / t_now)
    box = tuple(float(k) * a for k in n)
    return x, v, box


def add_recoils(x, v, box, n_recoils, energy_ev, at_centre, mass=MASS_FE, seed=0):
    """Give recoil (knock-on) atoms a speed sqrt(2 E C / m) along seeded random directions.

    Returns the list of recoil atom ids.  ``v`` is modified in place.
    """
    if n_recoils <= 0:
        return []
    _, _, ra, rdir = _streams(seed)
    L = np.asarray(box)
    if at_centre:
        d = x - 0.5 * L
        d -= L * np.rint(d / L)
        ids = [int(np.argmin(np.einsum("ij,ij->i", d, d)))]
    else:
        ids = [int(k) for k in ra.choice(x.shape[0], size=n_recoils, replace=False)]
    speed = math.sqrt(2.0 * energy_ev * ACC_A_FS2 / mass)
    for i in ids:
        u = rdir.normal(size=3)
        u /= np.linalg.norm(u)
        v[i] = speed * u
    return ids


def make_state(cfg: Config, n_cells=None):
    """Initial state of a named configuration (optionally on a smaller box)."""
    n = cfg.n_cells if n_cells is None else n_cells
    x, v, box = thermal_state(n, A_FE, cfg.temperature, cfg.sigma, MASS_FE, cfg.seed)
    rec = add_recoils(x, v, box, cfg.n_recoils, cfg.recoil_ev, cfg.recoil_at_centre, MASS_FE, cfg.seed)
    return x, v, box, rec


def _f(r):
    return np.exp(-F_BETA * (r / F_RE - 1.0))


def _df(r):
    return -(F_BETA / F_RE) * _f(r)


def _phi(r):
    return M_D * (np.exp(-2.0 * M_ALPHA * (r - M_R0)) - 2.0 * np.exp(-M_ALPHA * (r - M_R0)))


def _dphi(r):
    return M_D * (-2.0 * M_ALPHA * np.exp(-2.0 * M_ALPHA * (r - M_R0))
                  + 2.0 * M_ALPHA * np.exp(-M_ALPHA * (r - M_R0)))


def potential_samples(n_points=N_TABLE, rc=RC, rho_max=RHO_MAX, variant="raw"):
    """Equidistant samples of f, phi (on [0, rc]) and F (on [0, rho_max]).

    Returns {"f": (x0, h, y), "phi": (x0, h, y), "F": (x0, h, y)} with float64 y.
    ``variant`` is "raw" (plain truncation at rc) or "shifted" (shifted-force f, phi).
    """
    hr = rc / (n_points - 1)
    r = np.arange(n_points, dtype=np.float64) * hr
    r[-1] = rc
    fy, py = _f(r), _phi(r)
    if variant == "shifted":
        fy = fy - _f(rc) - (r - rc) * _df(rc)
        py = py - _phi(rc) - (r - rc) * _dphi(rc)
    elif variant != "raw":
        raise ValueError(variant)
    he = rho_max / (n_points - 1)
    rho = np.arange(n_points, dtype=np.float64) * he
    Fy = -EMB_A * np.sqrt(rho)
    return {"f": (0.0, hr, fy), "phi": (0.0, hr, py), "F": (0.0, he, Fy)}


@dataclasses.dataclass(frozen=True)
class BatchConfig:
    """Batched uneven replicas: independent periodic cubic boxes, one recoil each."""
    name: str
    n_boxes: int
    n_min: int              # cells per axis drawn uniformly from n_min .. n_max
    n_max: int
    e_min: float            # recoil energy log-uniform in [e_min, e_max] eV
    e_max: float
    steps: int
    dt_max: float
    dx_max: float
    seed: int
    precision: str = "fp32"
    temperature: float = 300.0
    sigma: float = 0.02


BATCH_CONFIGS = {
    "c4": BatchConfig("c4-256-boxes-10to40-recoil0.1to2kev", 256, 10, 40, 100.0, 2000.0, 2000, 1.0, 0.05, 1003),
}


def make_batch(cfg: BatchConfig, n_boxes=None):
    """Per-box (n_cells, x, v, box, recoil ids, recoil energy) of a batch configuration.

    Box k uses seed cfg.seed * 1000 + k for its thermal state and recoil direction;
    sizes and energies come from a stream of cfg.seed.  The recoil atom is the one
    nearest the box centre."""
    nb = cfg.n_boxes if n_boxes is None else n_boxes
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(cfg.seed)))
    sizes = rng.integers(cfg.n_min, cfg.n_max + 1, size=cfg.n_boxes)[:nb]
    energies = np.exp(rng.uniform(math.log(cfg.e_min), math.log(cfg.e_max), size=cfg.n_boxes))[:nb]
    out = []
    for k in range(nb):
        n = int(sizes[k])
        seed = cfg.seed * 1000 + k
        x, v, box = thermal_state(n, A_FE, cfg.temperature, cfg.sigma, MASS_FE, seed)
        rec = add_recoils(x, v, box, 1, float(energies[k]), True, MASS_FE, seed)
        out.append((n, x, v, box, rec, float(energies[k])))
    return out
