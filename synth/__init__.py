"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds workload definitions and input generators only: sizes,
seeds, starting positions and closed-form orbital tables.  It contains none of
the method's arithmetic (no spline evaluation, determinant, Jastrow, update or
energy), so both the HIP path and the CPU oracle can take their inputs from it.

The five workloads are synthetic stand-ins for the paper's NiO supercell runs
(Sec. IV: hundreds to thousands of walkers per GPU; "small/medium" systems of up
to 1000 electrons and larger ones), shaped as:

  C1  4+4 electrons, L=5, 16^3 grid, analytic plane-wave orbitals (prefiltered
      spline), no Jastrow, 16 walkers, 200 VMC sweeps, FP64, Sherman-Morrison.
  C2  32+32, L=10, 48^3, seeded U[-1,1] coefficients, Pade J2, 256 walkers,
      100 sweeps, FP64 and mixed precision.
  C3  256+256, L=20, 64^3 (FP32, 268 MB), J2, 4 crowds x 512 walkers,
      delay rank k in {1,4,8,16,32}, FP64 recompute every 64 sweeps.
  C4  1024+1024, L=32, 96^3 (FP32, 3.62 GB), J2, 128 walkers, k=32, FP64
      recompute every 32 sweeps.
  C5  DMC over three systems at once (the C2/C3/C4 systems), tau=0.01,
      target populations 2000 / 500 / 64.
"""
from dataclasses import dataclass
from typing import Optional

import numpy as np

__all__ = ["Workload", "WORKLOADS", "start_positions", "planewave_table", "workload", "icosahedron_offsets",
           "TRICLINIC", "cell_positions", "complex_table"]


@dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # electrons per spin = orbitals per spin
    L: float               # cubic box edge, bohr
    G: int                 # spline grid points per dimension
    walkers: int           # walkers per crowd
    crowds: int
    sweeps: int
    warmup: int
    precision: str         # "fp64" or "mixed"
    delay_rank: int        # 1 = Sherman-Morrison
    recompute_every: int   # sweeps between FP64 recomputes (0 = never)
    use_j2: bool
    orbitals: str          # "planewave" or "seeded"
    seed: int
    sigma: float = 0.5
    dmc_target: Optional[int] = None

    @property
    def n_e(self) -> int:
        return 2 * self.n

    def table_bytes(self, elem_bytes: int) -> int:
        return self.G ** 3 * self.n * elem_bytes


WORKLOADS = {
    "c1": Workload("c1", 4, 5.0, 16, 16, 1, 200, 0, "fp64", 1, 0, False, "planewave", 1001),
    "c2": Workload("c2", 32, 10.0, 48, 256, 1, 100, 0, "mixed", 1, 32, True, "seeded", 1002),
    "c3": Workload("c3", 256, 20.0, 64, 512, 4, 128, 8, "mixed", 32, 64, True, "seeded", 1003),
    "c4": Workload("c4", 1024, 32.0, 96, 128, 1, 64, 4, "mixed", 32, 32, True, "seeded", 1004),
    # DMC systems of C5 (same boxes and grids as C2-C4), target populations
    "c5s1": Workload("c5s1", 32, 10.0, 48, 2000, 1, 100, 20, "mixed", 1, 0, True, "seeded", 1005, 0.5, 2000),
    "c5s2": Workload("c5s2", 256, 20.0, 64, 500, 1, 100, 20, "mixed", 8, 0, True, "seeded", 1006, 0.5, 500),
    "c5s3": Workload("c5s3", 1024, 32.0, 96, 64, 1, 100, 20, "mixed", 32, 0, True, "seeded", 1007, 0.5, 64),
}

# Pade J2 parameters of the workloads: a = 0.25 (parallel spins), 0.5 (antiparallel), b = 1
J2_A_PAR, J2_A_ANTI, J2_B = 0.25, 0.5, 1.0


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def start_positions(seed: int, n_walkers: int, n_e: int, L: float, first_walker: int = 0) -> np.ndarray:
    """Uniform starting positions in [0, L)^3, shape [W][Ne][3], FP64.

    Walker w's positions depend only on (seed, first_walker + w), so any subset
    of a crowd can be regenerated on its own.
    """
    out = np.empty((n_walkers, n_e, 3))
    for w in range(n_walkers):
        rng = np.random.default_rng([seed, first_walker + w])
        out[w] = rng.uniform(0.0, L, size=(n_e, 3))
    return out


def planewave_table(G: int, L: float) -> np.ndarray:
    """Interpolating cubic-spline coefficients of {1, cos kx, sin kx, cos ky}, k = 2 pi / L.

    For a Fourier mode the periodic interpolation prefilter is closed form:
    control value = f(x_j) / beta(k h) per varying axis, beta(q) = (2 + cos q)/3
    (beta = 1 along axes where the mode is constant).  Shape [G][G][G][4], FP64.
    """
    h = L / G
    k = 2.0 * np.pi / L
    beta = (2.0 + np.cos(k * h)) / 3.0
    x = np.arange(G) * h
    t = np.zeros((G, G, G, 4))
    t[..., 0] = 1.0
    t[..., 1] = (np.cos(k * x) / beta)[:, None, None]
    t[..., 2] = (np.sin(k * x) / beta)[:, None, None]
    t[..., 3] = (np.cos(k * x) / beta)[None, :, None]
    return t


def icosahedron_offsets(radius: float) -> np.ndarray:
    """The 12 vertices of a regular icosahedron on the sphere of the given radius, [12][3]:
    the points of a 12-point spherical quadrature (equal weights, exact for spherical harmonics
    of degree up to 5), a synthetic stand-in for the quadrature points of a non-local
    pseudopotential around an electron."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(v)
    return radius * v / np.linalg.norm(v, axis=1, keepdims=True)


# A general (triclinic) cell for the complex-orbital tests and workload: lattice vectors as rows,
# bohr (edges 10.0, 9.0 and 11.0; angles of about 100 degrees between a1 and a2, 70 between a1
# and a3, 86 between a2 and a3; volume 907 bohr^3).
TRICLINIC = np.array([[10.0, 0.0, 0.0],
                      [-1.5, 8.874119674649425, 0.0],
                      [3.7622215, 1.5, 10.221357245]])


def cell_positions(seed: int, n_walkers: int, n_e: int, lattice, first_walker: int = 0) -> np.ndarray:
    """Uniform starting positions in the cell spanned by the rows of `lattice`: uniform fractional
    coordinates f in [0, 1)^3, r = f @ lattice.  Shape [W][Ne][3], FP64; walker w depends only on
    (seed, first_walker + w)."""
    lat = np.asarray(lattice, dtype=np.float64)
    out = np.empty((n_walkers, n_e, 3))
    for w in range(n_walkers):
        rng = np.random.default_rng([seed, first_walker + w, 7])
        out[w] = rng.uniform(0.0, 1.0, size=(n_e, 3)) @ lat
    return out


def complex_table(seed: int, G: int, n: int) -> np.ndarray:
    """Seeded complex B-spline coefficients, real and imaginary parts U[-1, 1], shape [G][G][G][n]
    complex128 (orbital index fastest)."""
    rng = np.random.default_rng([seed, G, n, 11])
    t = np.empty((G, G, G, n), np.complex128)
    t.real = rng.uniform(-1.0, 1.0, size=t.shape)
    t.imag = rng.uniform(-1.0, 1.0, size=t.shape)
    return t
