"""Seeded synthetic inputs for the transport path.

This module carries none of the method's arithmetic. It produces the data that
the paper's input files hold (neighbour list, hoppings, on-site potentials,
positions, length and volume; Section 4.2), random-phase state vectors
(Section 3.1) and time-step lists (Section 4.2.6). The tests, the benchmark and
the smoke check feed the same arrays to both the HIP path and the CPU oracle.

Lattices: a periodic chain, a square lattice with optional next-nearest
hopping, a simple cubic lattice, and a honeycomb lattice in brick-wall form
with Peierls phases for a uniform perpendicular field.  On-site potentials
follow the Anderson model of Section 5 (uniform in [-W/2, W/2]).

Conventions
-----------
* ``nbr[i, s]`` is the s-th neighbour of site i, valid for ``s < nn[i]``; other
  slots hold -1.
* ``hop[i, s]`` is the matrix element H[i, nbr[i, s]]; ``None`` means the
  paper's default of -1 for every pair (Section 4.2.2).
* ``x`` is the coordinate along the transport direction, ``length_x`` the
  periodic length in that direction (<= 0: open boundary), ``volume`` the
  system volume Omega (Section 4.2.4).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

HBAR_EV_FS = 0.6582119569  # hbar in eV*fs: converts a step in fs to hbar/eV


@dataclasses.dataclass
class Model:
    nn: np.ndarray                      # int32 [n]
    nbr: np.ndarray                     # int32 [n, max_nn]
    hop: Optional[np.ndarray]           # float64 or complex128 [n, max_nn]
    onsite: Optional[np.ndarray]        # float64 [n]
    x: np.ndarray                       # float64 [n]
    length_x: float
    volume: float
    hop_class: Optional[np.ndarray] = None   # int32 [n, max_nn]
    n_class: int = 1
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.nn.shape[0])

    @property
    def max_nn(self) -> int:
        return int(self.nbr.shape[1])


def anderson(n: int, W: float, seed: int) -> np.ndarray:
    """On-site energies uniform in [-W/2, W/2] (Anderson model, Section 5)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.5 * W, 0.5 * W, size=n)


def random_phase(n: int, B: int, seed: int) -> np.ndarray:
    """B random-phase vectors exp(i theta), theta uniform in [0, 2pi).

    Layout [n][B] (B fastest), complex128, so <phi|phi> = n per column.
    """
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * math.pi, size=(n, B))
    return np.ascontiguousarray(np.exp(1j * theta))


def _finish(nbr: np.ndarray) -> np.ndarray:
    nn = np.full(nbr.shape[0], nbr.shape[1], dtype=np.int32)
    return nn


def chain(L: int, t: float = -1.0, W: float = 0.0, seed: int = 0,
          periodic: bool = True, onsite: Optional[np.ndarray] = None) -> Model:
    """1D chain of L sites, lattice constant 1; slots: +1, -1."""
    i = np.arange(L)
    nbr = np.stack([(i + 1) % L, (i - 1) % L], axis=1).astype(np.int32)
    nn = np.full(L, 2, dtype=np.int32)
    if not periodic:
        nbr, nn = _drop_bonds(nbr, nn, np.stack([i == L - 1, i == 0], axis=1))
    hop = None if t == -1.0 else np.full((L, 2), t)
    U = onsite if onsite is not None else (anderson(L, W, seed) if W > 0 else None)
    return Model(nn, nbr, hop, U, i.astype(np.float64),
                 float(L) if periodic else 0.0, float(L), name=f"chain{L}")


def _drop_bonds(nbr, nn, drop):
    """Remove the marked slots and compact each row's neighbour list."""
    n, k = nbr.shape
    out = np.full_like(nbr, -1)
    cnt = np.zeros(n, dtype=np.int32)
    for s in range(k):
        keep = ~drop[:, s]
        rows = np.nonzero(keep)[0]
        out[rows, cnt[rows]] = nbr[rows, s]
        cnt[rows] += 1
    return out, cnt


def square(Lx: int, Ly: int, t1: float = -1.0, t2: Optional[float] = None,
           W: float = 0.0, seed: int = 0, periodic_x: bool = True,
           onsite: Optional[np.ndarray] = None) -> Model:
    """Square lattice, site index ix + Lx*iy, lattice constant 1.

    Slots 0-3: +x, -x, +y, -y (hopping t1).  With t2, slots 4-7 are the
    next-nearest neighbours (+x+y, -x+y, +x-y, -x-y) with hopping t2, and
    ``hop_class`` marks slots 0-3 as class 0 and 4-7 as class 1.  y is always
    periodic; x is periodic unless ``periodic_x`` is False (open in x).
    """
    ix, iy = np.meshgrid(np.arange(Lx), np.arange(Ly), indexing="xy")
    ix = ix.ravel()
    iy = iy.ravel()
    n = Lx * Ly

    def idx(a, b):
        return ((a % Lx) + Lx * (b % Ly)).astype(np.int32)

    cols = [idx(ix + 1, iy), idx(ix - 1, iy), idx(ix, iy + 1), idx(ix, iy - 1)]
    wraps = [ix == Lx - 1, ix == 0, np.zeros(n, bool), np.zeros(n, bool)]
    if t2 is not None:
        cols += [idx(ix + 1, iy + 1), idx(ix - 1, iy + 1),
                 idx(ix + 1, iy - 1), idx(ix - 1, iy - 1)]
        wraps += [ix == Lx - 1, ix == 0, ix == Lx - 1, ix == 0]
    nbr = np.stack(cols, axis=1).astype(np.int32)
    k = nbr.shape[1]
    nn = np.full(n, k, dtype=np.int32)
    hop_vals = np.full((n, k), t1)
    cls = None
    if t2 is not None:
        hop_vals[:, 4:] = t2
        cls = np.zeros((n, k), dtype=np.int32)
        cls[:, 4:] = 1
    if not periodic_x:
        drop = np.stack(wraps, axis=1)
        # compact neighbours, hoppings and classes together
        order = np.argsort(drop, axis=1, kind="stable")
        nbr = np.take_along_axis(nbr, order, axis=1)
        hop_vals = np.take_along_axis(hop_vals, order, axis=1)
        if cls is not None:
            cls = np.take_along_axis(cls, order, axis=1)
        nn = (k - drop.sum(axis=1)).astype(np.int32)
        slot = np.arange(k)[None, :]
        nbr = np.where(slot < nn[:, None], nbr, -1).astype(np.int32)
    default_hop = (t2 is None and t1 == -1.0)
    hop = None if default_hop else hop_vals
    U = onsite if onsite is not None else (anderson(n, W, seed) if W > 0 else None)
    return Model(nn, nbr, hop, U, ix.astype(np.float64),
                 float(Lx) if periodic_x else 0.0, float(Lx * Ly),
                 hop_class=cls, n_class=2 if t2 is not None else 1,
                 name=f"square{Lx}x{Ly}")


def cubic(L: int, t: float = -1.0, W: float = 0.0, seed: int = 0,
          onsite: Optional[np.ndarray] = None) -> Model:
    """Simple cubic L^3, periodic; index ix + L*(iy + L*iz); slots +-x, +-y, +-z."""
    m = box(L, L, L, t=t, W=W, seed=seed, onsite=onsite)
    m.name = f"cubic{L}"
    return m


def box(Lx: int, Ly: int, Lz: int, t: float = -1.0, W: float = 0.0, seed: int = 0,
        onsite: Optional[np.ndarray] = None, slot_seed: Optional[int] = None) -> Model:
    """Simple cubic Lx x Ly x Lz box, periodic in all three directions; index
    ix + Lx*(iy + Ly*iz); slots +-x, +-y, +-z (each row's slots shuffled when slot_seed is
    given)."""
    n = Lx * Ly * Lz
    s = np.arange(n, dtype=np.int64)
    ix = s % Lx
    iy = (s // Lx) % Ly
    iz = s // (Lx * Ly)

    def idx(a, b, c):
        return ((a % Lx) + Lx * ((b % Ly) + Ly * (c % Lz))).astype(np.int32)

    nbr = np.stack([idx(ix + 1, iy, iz), idx(ix - 1, iy, iz),
                    idx(ix, iy + 1, iz), idx(ix, iy - 1, iz),
                    idx(ix, iy, iz + 1), idx(ix, iy, iz - 1)], axis=1)
    if slot_seed is not None:
        order = np.argsort(np.random.default_rng(slot_seed).random((n, 6)), axis=1)
        nbr = np.take_along_axis(nbr, order, axis=1).astype(np.int32)
    nn = np.full(n, 6, dtype=np.int32)
    hop = None if t == -1.0 else np.full((n, 6), t)
    U = onsite if onsite is not None else (anderson(n, W, seed) if W > 0 else None)
    return Model(nn, nbr, hop, U, ix.astype(np.float64), float(Lx), float(n),
                 name=f"box{Lx}x{Ly}x{Lz}")


def honeycomb(nx_cells: int, ny_cells: int, t: float = -2.7, a_cc: float = 0.142,
              flux: float = 0.0, W: float = 0.0, seed: int = 0,
              onsite: Optional[np.ndarray] = None) -> Model:
    """Honeycomb lattice of nx_cells x ny_cells unit cells in brick-wall form.

    Sites (i, j) with i < Nx = 2*nx_cells (zigzag chains along x, the transport
    direction) and j < Ny = ny_cells, index i + Nx*j, periodic in both
    directions.  Slots: 0 -> (i+1, j), 1 -> (i-1, j), 2 -> (i, j+1) when i+j is
    even, else (i, j-1).  x = i * (sqrt(3)/2) a_cc.

    ``flux`` is the magnetic flux per hexagon in flux quanta.  Peierls phases
    (Landau gauge along x): the hop from (i, j) to (i+1, j) carries
    exp(i*theta_j) with theta_j = -pi*flux*j; the vertical bonds that wrap from
    row Ny-1 to row 0 at column i carry exp(i*pi*flux*Ny*i).  Every hexagon then
    encloses 2*pi*flux; this is consistent on the torus when the total flux
    flux*Nx*Ny/2 is an integer.
    """
    Nx, Ny = 2 * nx_cells, ny_cells
    if Ny % 2:
        raise ValueError("brick-wall honeycomb needs an even number of rows")
    n = Nx * Ny
    s = np.arange(n, dtype=np.int64)
    i = s % Nx
    j = s // Nx
    up = ((i + j) % 2) == 0
    jv = np.where(up, j + 1, j - 1)
    nbr = np.stack([((i + 1) % Nx) + Nx * j, ((i - 1) % Nx) + Nx * j,
                    i + Nx * (jv % Ny)], axis=1).astype(np.int32)
    nn = np.full(n, 3, dtype=np.int32)
    if flux != 0.0:
        total = flux * Nx * Ny / 2.0
        if abs(total - round(total)) > 1e-9:
            raise ValueError("total flux through the torus must be integer")
        theta = -math.pi * flux * j
        hop = np.empty((n, 3), dtype=np.complex128)
        hop[:, 0] = t * np.exp(-1j * theta)    # H[(i,j),(i+1,j)] = conj(t e^{i theta})
        hop[:, 1] = t * np.exp(1j * theta)     # H[(i,j),(i-1,j)] = t e^{i theta}
        phv = math.pi * flux * Ny * i
        wrap_up = up & (j == Ny - 1)           # (i, Ny-1) -> (i, 0)
        wrap_dn = (~up) & (j == 0)             # (i, 0) -> (i, Ny-1)
        v = np.full(n, t, dtype=np.complex128)
        v[wrap_up] = t * np.exp(-1j * phv[wrap_up])
        v[wrap_dn] = t * np.exp(1j * phv[wrap_dn])
        hop[:, 2] = v
    else:
        hop = np.full((n, 3), t)
    U = onsite if onsite is not None else (anderson(n, W, seed) if W > 0 else None)
    dxs = math.sqrt(3.0) / 2.0 * a_cc
    return Model(nn, nbr, hop, U, (i * dxs).astype(np.float64), Nx * dxs,
                 Nx * dxs * Ny * 1.5 * a_cc, name=f"honeycomb{nx_cells}x{ny_cells}")


def concat_segments(models: List[Model]) -> Model:
    """Block-diagonal concatenation of independent realisations (row offsets)."""
    off = 0
    nbrs, nns, hops, Us, xs, cls = [], [], [], [], [], []
    k = max(m.max_nn for m in models)
    complex_hop = any(m.hop is not None and np.iscomplexobj(m.hop) for m in models)
    for m in models:
        nb = np.full((m.n, k), -1, dtype=np.int32)
        nb[:, :m.max_nn] = np.where(m.nbr >= 0, m.nbr + off, -1)
        nbrs.append(nb)
        nns.append(m.nn)
        h = np.full((m.n, k), -1.0, dtype=np.complex128 if complex_hop else np.float64)
        if m.hop is not None:
            h[:, :m.max_nn] = m.hop
        hops.append(h)
        Us.append(m.onsite if m.onsite is not None else np.zeros(m.n))
        xs.append(m.x)
        c = np.zeros((m.n, k), dtype=np.int32)           # hopping classes (padding: class 0)
        if m.hop_class is not None:
            c[:, :m.max_nn] = m.hop_class
        cls.append(c)
        off += m.n
    n_class = max(m.n_class for m in models)
    return Model(np.concatenate(nns), np.concatenate(nbrs), np.concatenate(hops),
                 np.concatenate(Us), np.concatenate(xs), -1.0,
                 float(sum(m.volume for m in models)),
                 hop_class=np.concatenate(cls) if n_class > 1 else None, n_class=n_class, name="segments")


def bond_disorder(m: Model, spread: float, seed: int, max_phase: float = 0.0) -> Model:
    """m with every bond's hopping multiplied by (1 + spread * u), u uniform in [-1, 1], and
    (max_phase > 0) a phase exp(i phi), phi uniform in [-max_phase, max_phase], drawn once per
    bond so that H stays Hermitian: the q-th entry of row i pointing to j and the q-th entry
    of row j pointing to i hold h and conj(h)."""
    rng = np.random.default_rng(seed)
    base = dense_hop(m)
    cplx = max_phase > 0 or np.iscomplexobj(base)
    hop = np.array(base, dtype=np.complex128 if cplx else np.float64, copy=True)
    seen = {}
    for i in range(m.n):
        for s in range(int(m.nn[i])):
            j = int(m.nbr[i, s])
            q = sum(1 for t in range(s) if m.nbr[i, t] == j)
            key = (min(i, j), max(i, j), q)
            if key not in seen:
                f = 1.0 + spread * rng.uniform(-1.0, 1.0)
                ph = np.exp(1j * rng.uniform(-max_phase, max_phase)) if max_phase > 0 else 1.0
                seen[key] = (i, f * ph)
            first, g = seen[key]
            hop[i, s] = hop[i, s] * (g if (first == i or not cplx) else np.conj(g))
    return dataclasses.replace(m, hop=hop, name=m.name + "_bond")


def dense_hop(m: Model) -> np.ndarray:
    """The hopping array with the paper's default (-1) filled in."""
    if m.hop is None:
        return np.where(m.nbr >= 0, -1.0, 0.0)
    return m.hop


# --------------------------------------------------------------------------
# Workloads with the shapes of the paper's examples (Section 5) scaled to the
# sizes used by the benchmark and the parity tests.
# --------------------------------------------------------------------------

def workload_square64() -> dict:
    """2D square 64x64 periodic, t=-1, W=1 Anderson; DeltaE=4.5; M=1000;
    1001 energies in [-4.2, 4.2]; VAC and MSD over 10 steps dt=1, Np=100."""
    m = square(64, 64, W=1.0, seed=1001)
    return dict(model=m, phi=random_phase(m.n, 1, 1002), energy_max=4.5, M=1000,
                energies=np.linspace(-4.2, 4.2, 1001), dt=np.ones(10), Np=100,
                name="square64x64")


def workload_honeycomb(nx_cells: int = 1000, ny_cells: int = 1000,
                       n_vectors: int = 10) -> dict:
    """Honeycomb 1000x1000 cells = 2,000,000 orbitals, t=-2.7 eV, Peierls phases
    for flux 1/2000 per hexagon, Anderson W=2 eV (U in [-1,1] eV);
    DeltaE = 1.01 * Gershgorin bound (1 + 3*2.7 eV); M=3000; 20 steps of 15 fs."""
    m = honeycomb(nx_cells, ny_cells, t=-2.7, a_cc=0.142, flux=1.0 / 2000.0,
                  W=2.0, seed=2001)
    phis = [random_phase(m.n, 1, 2002 + r) for r in range(n_vectors)]
    dt = np.full(20, 15.0 / HBAR_EV_FS)
    return dict(model=m, phis=phis, energy_max=1.01 * (1.0 + 3 * 2.7), M=3000,
                dt=dt, Np=0, energies=np.linspace(-9.0, 9.0, 1001),
                name=f"honeycomb{nx_cells}x{ny_cells}")


def segment_sizes(n_seg: int = 8, lo: int = 200, hi: int = 2000) -> List[int]:
    """Square-lattice side lengths spaced geometrically from lo to hi."""
    if n_seg == 1:
        return [lo]
    return [int(round(lo * (hi / lo) ** (r / (n_seg - 1)))) for r in range(n_seg)]


def workload_batched(sides: Optional[List[int]] = None, B: int = 16,
                     M: int = 2000) -> dict:
    """Uneven square-lattice realisations (200^2 .. 2000^2), W_r uniform in
    [0.5, 3]; B random-phase vectors per realisation; per-segment DeltaE =
    1.01 * (4 + W_r/2)."""
    sides = sides or segment_sizes()
    Ws = np.random.default_rng(3001).uniform(0.5, 3.0, size=len(sides))
    models = [square(L, L, W=float(Ws[r]), seed=3002 + r) for r, L in enumerate(sides)]
    phi = np.concatenate([random_phase(mm.n, B, 3100 + r)
                          for r, mm in enumerate(models)], axis=0)
    return dict(models=models, Ws=Ws, phi=phi, B=B, M=M,
                seg_energy_max=1.01 * (4.0 + Ws / 2.0), name="batched_square")


def workload_cubic(L: int = 200, W: float = 16.0, B: int = 4) -> dict:
    """Cubic L^3 (8,000,000 orbitals at L=200), t=-1, Anderson W in {8,16,24};
    B random-phase vectors; MSD over 40 steps dt=2 with 60 terms; M=1000."""
    m = cubic(L, W=W, seed=4000 + int(W))
    return dict(model=m, phi=random_phase(m.n, B, 4100), energy_max=1.01 * (6.0 + W / 2.0),
                M=1000, dt=np.full(40, 2.0), Np=60, name=f"cubic{L}_W{int(W)}")


def workload_paper_diffusive(L: int = 2000) -> dict:
    """The paper's first example (Section 5.1): square L x L (2000 x 2000), periodic, t = -1,
    Anderson W = 4 (seed 6001); one random-phase vector (seed 6002); DeltaE = 6.1, M = 1000
    (default); VAC and MSD over 20 steps of 0.2; energies -6 .. 6 in steps of 0.02."""
    m = square(L, L, W=4.0, seed=6001)
    return dict(model=m, phi=random_phase(m.n, 1, 6002), energy_max=6.1, M=1000,
                dt=np.full(20, 0.2), energies=np.linspace(-6.0, 6.0, 601), vac=True, msd=True,
                name=f"paper_diffusive_square{L}")


def workload_paper_localized(L: int = 4_000_000) -> dict:
    """The paper's second example (Section 5.2): chain of 4,000,000 sites, periodic, t = -1,
    Anderson W = 4 (seed 6101); two random-phase vectors (seeds 6102, 6103); DeltaE = 4.1,
    M = 500; MSD only over 30 non-uniform steps 0.1 .. 1.0, 1 .. 10, 10 .. 100; energies
    -4 .. 4 in steps of 0.02."""
    m = chain(L, W=4.0, seed=6101)
    dt = np.concatenate([np.arange(1, 11) * 0.1, np.arange(1, 11) * 1.0, np.arange(1, 11) * 10.0])
    phi = np.concatenate([random_phase(m.n, 1, 6102 + r) for r in range(2)], axis=1)
    return dict(model=m, phi=phi, energy_max=4.1, M=500, dt=dt,
                energies=np.linspace(-4.0, 4.0, 401), vac=False, msd=True,
                name=f"paper_localized_chain{L}")


def workload_train(L: int = 512) -> dict:
    """Square L x L with trainable on-site energies (uniform in [-1,1]) and two
    hopping classes (t1 nearest, t2 next-nearest); DeltaE fixed at 6.0; M=512."""
    m = square(L, L, t1=-1.0, t2=-0.1, onsite=np.random.default_rng(5001).uniform(-1, 1, L * L))
    target = square(L, L, t1=-1.0, t2=-0.1,
                    onsite=np.random.default_rng(5002).uniform(-1, 1, L * L))
    return dict(model=m, target_model=target, phi=random_phase(m.n, 1, 5003),
                energy_max=6.0, M=512, energies=np.linspace(-5.0, 5.0, 1001),
                dt=np.ones(10), fd_seed=5004, name=f"train_square{L}")
