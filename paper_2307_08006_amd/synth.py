"""Seeded synthetic inputs for the lambda-ABF alchemical nonbonded step.

This module only builds inputs: lattices, parameters, walker batches and the
lambda/ABF settings.  It holds none of the method's arithmetic, so that the
HIP path and the FP64 oracle can both be fed from it without sharing any
computation.

Workloads (stand-ins for the paper's systems, whose structures and force
fields are not available):
  * ``lj_reduced``      -- 512 LJ particles in reduced units at density 0.8,
                           one soft-core-decoupled solute (alpha 0.5, p 1).
  * ``harmonic``        -- 3 non-interacting particles with lambda-switched
                           harmonic restraints k(lambda) = 1 + 3 lambda.
  * ``charged_lj``      -- a charged LJ fluid (sigma 3.15 A, eps 0.15 kcal/mol,
                           charges +-0.4 e) at 0.1 atoms/A^3 with a decoupled
                           solute; the size of the paper's solvated boxes.
  * ``batch``           -- several walkers of a system with independent
                           velocities and initial lambda.
  * ``uneven``          -- walkers of log-uniform sizes, each a solvent box
                           around a restrained dense cluster with a ligand.
Positions are put on the grid the chosen precision represents exactly inside
a box offset by a power of two (see ``quantize``), so that every consumer
starts from bit-identical coordinates.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# unit constants (real units: A, fs, amu, kcal/mol, e)
KB_KCAL = 0.0019872041          # kcal/mol/K
COULOMB_K = 332.0637            # kcal A / (mol e^2)
ACCEL_REAL = 4.184e-4           # (kcal/mol/A/amu) -> A/fs^2

BASE_SEED = 20230717


@dataclasses.dataclass
class SystemSpec:
    """Static description of a batch of walkers and its initial state."""
    atom_offset: np.ndarray          # int64 [W+1]
    box: np.ndarray                  # float64 [W,3]
    pos: np.ndarray                  # float64 [N,3], inside [0, L)
    mass: np.ndarray                 # float64 [N]
    charge: np.ndarray               # float64 [N]
    sigma: np.ndarray                # float64 [N]
    epsilon: np.ndarray              # float64 [N]
    is_solute: np.ndarray            # uint8 [N]
    r_cut: float
    r_skin: float
    kT: float
    gamma: float
    dt: float
    coulomb_k: float
    accel_unit: float
    seed: int
    precision: str = "fp32"          # "fp32" | "fp64"
    vel: Optional[np.ndarray] = None     # float64 [N,3]; None -> Maxwell-Boltzmann
    anchor: Optional[np.ndarray] = None  # float64 [N,3]
    k0: Optional[np.ndarray] = None      # float64 [N]
    k1: Optional[np.ndarray] = None      # float64 [N]
    rebuild_interval: int = 10
    r_skin_alch: float = 0.0             # list buffer of alchemical pairs; 0 -> r_skin
    column_width: Optional[np.ndarray] = None  # float64 [W] cluster column width factor; None -> 1
    prune_buffer: Optional[np.ndarray] = None  # float64 [W] pair-list prune buffer b (A); None/0 -> min(0.5, r_skin / 2)
    pme_dims: Optional[np.ndarray] = None  # int32 [W,3] PME grid (2^a 3^b 5^c, multiples of 8); None -> no PME
    ewald_beta: float = 0.0              # Ewald splitting parameter (1/A) when pme_dims is set
    pme_order: int = 4                   # B-spline order of the PME charge assignment
    name: str = ""

    @property
    def n_walkers(self) -> int:
        return int(self.atom_offset.shape[0] - 1)

    @property
    def n_atoms(self) -> int:
        return int(self.atom_offset[-1])

    def walker_slice(self, w: int) -> slice:
        return slice(int(self.atom_offset[w]), int(self.atom_offset[w + 1]))


@dataclasses.dataclass
class LambdaSpec:
    """Extended-lambda and ABF settings (one set shared by all walkers)."""
    lambda0: np.ndarray              # float64 [W]
    p_lambda0: Optional[np.ndarray]  # float64 [W]; None -> Maxwell-Boltzmann
    m_lambda: float
    gamma_lambda: float
    kT_lambda: float
    elec_start: float = 0.0
    elec_end: float = 0.5
    vdw_start: float = 0.5
    vdw_end: float = 1.0
    direction: str = "decouple"      # "decouple" | "couple"
    sc_alpha: float = 0.5
    sc_power: int = 1
    n_bins: int = 100
    lo: float = 0.0
    hi: float = 1.0
    full_samples: int = 100
    share_interval: int = 1
    fixed_lambda: bool = False
    abf_on: bool = True
    sc_form: str = "beutler"         # "beutler": alpha (1-c)^p + (r/sig)^6; "shifted": r^2 + delta (1-c)
    sc_shift: float = 5.0            # delta of the separation-shifted form (length^2)
    # lambda-dependent distance restraint between two atoms per walker:
    # V = k/2 (d - d_min)^2 for d < d_min = (delta/2)(1 - cos(2 pi n lambda))
    dr_pairs: Optional[np.ndarray] = None   # int [W][2] walker-local atom indices
    dr_delta: float = 20.0
    dr_k: float = 5.0
    dr_freq: int = 1


def _pow2_at_least(x: float) -> float:
    return float(2.0 ** math.ceil(math.log2(x)))


def quantize(pos: np.ndarray, box: np.ndarray, precision: str):
    """Round the box edges and positions (wrapped into [0, L)) to the values
    that ``(B + x) - B`` preserves in the given precision, B being the
    smallest power of two >= 2L (the storage offset of the GPU layout).
    Returns (pos, box) as float64."""
    pos = np.array(pos, dtype=np.float64, copy=True)
    box = np.array(box, dtype=np.float64, copy=True)
    ft = np.float32 if precision == "fp32" else np.float64
    for k in range(3):
        L = float(box[k])
        B = _pow2_at_least(2.0 * L)
        Lq = float(ft(ft(B) + ft(L)) - ft(B))
        box[k] = Lq
        x = pos[:, k] - Lq * np.floor(pos[:, k] / Lq)
        xq = (ft(B) + x.astype(ft)).astype(ft)
        xq = np.where(xq >= ft(B + Lq), xq - ft(Lq), xq)
        pos[:, k] = (xq - ft(B)).astype(np.float64)
    return pos, box


def _lattice_sc(n_side: int, L: float) -> np.ndarray:
    a = L / n_side
    g = (np.arange(n_side) + 0.5) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def _lattice_fcc(n_cell: int, L: float) -> np.ndarray:
    a = L / n_cell
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]], dtype=np.float64)
    g = np.arange(n_cell, dtype=np.float64)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    sites = (cells[:, None, :] + basis[None, :, :] + 0.25).reshape(-1, 3)
    return sites * a


# ----------------------------------------------------------------------------
# reduced-unit LJ fluid with one decoupled solute
# ----------------------------------------------------------------------------
def lj_reduced(n_atoms: int = 512, density: float = 0.8, seed: int = BASE_SEED,
               precision: str = "fp64", r_cut: float = 2.5, r_skin: float = 0.5,
               n_walkers: int = 1, lambda0: float = 0.0, n_bins: int = 50,
               full_samples: int = 100, jitter: float = 0.05, charges: float = 0.0):
    """512 LJ particles (sigma = eps = m = 1), cubic periodic box at the given
    density, seeded simple-cubic lattice with +-jitter, T = 1, gamma = 1,
    dt = 0.005, atom 0 decoupled through soft-core vdW only
    (c_v = 1 - lambda); m_lambda = 10, gamma_lambda = 1."""
    rng = np.random.default_rng(seed)
    L = (n_atoms / density) ** (1.0 / 3.0)
    n_side = int(math.ceil(n_atoms ** (1.0 / 3.0) - 1e-9))
    sites = _lattice_sc(n_side, L)
    if sites.shape[0] > n_atoms:
        sites = sites[np.sort(rng.permutation(sites.shape[0])[:n_atoms])]
    pos1 = sites + rng.uniform(-jitter, jitter, size=sites.shape)
    pos_all, boxes = [], []
    for w in range(n_walkers):
        p, b = quantize(pos1, np.array([L, L, L]), precision)
        pos_all.append(p)
        boxes.append(b)
    N = n_atoms * n_walkers
    q = np.zeros(n_atoms)
    if charges:
        q = np.where(rng.permutation(n_atoms) % 2 == 0, charges, -charges)
    spec = SystemSpec(
        atom_offset=np.arange(n_walkers + 1, dtype=np.int64) * n_atoms,
        box=np.array(boxes), pos=np.concatenate(pos_all),
        mass=np.ones(N), charge=np.tile(q, n_walkers), sigma=np.ones(N), epsilon=np.ones(N),
        is_solute=np.tile((np.arange(n_atoms) == 0).astype(np.uint8), n_walkers),
        r_cut=r_cut, r_skin=r_skin, kT=1.0, gamma=1.0, dt=0.005, coulomb_k=1.0,
        accel_unit=1.0, seed=seed, precision=precision, name="lj_reduced")
    lam = LambdaSpec(lambda0=np.full(n_walkers, float(lambda0)), p_lambda0=None,
                     m_lambda=10.0, gamma_lambda=1.0, kT_lambda=1.0,
                     elec_start=0.0, elec_end=1.0, vdw_start=0.0, vdw_end=1.0,
                     direction="decouple", sc_alpha=0.5, sc_power=1, n_bins=n_bins,
                     lo=0.0, hi=1.0, full_samples=full_samples, share_interval=1)
    return spec, lam


# ----------------------------------------------------------------------------
# lambda-switched harmonic restraints (closed-form free energy)
# ----------------------------------------------------------------------------
def harmonic(n_walkers: int = 1, seed: int = BASE_SEED + 100, precision: str = "fp64",
             k0: float = 1.0, k1: float = 4.0, n_bins: int = 50, full_samples: int = 100,
             L: float = 64.0):
    """3 particles (m = 1) with anchors at the box centre, no pair
    interactions (eps = q = 0), k(lambda) = k0 + lambda (k1 - k0) on every
    Cartesian component, T = 1, gamma = 1, dt = 0.005, m_lambda = 10,
    gamma_lambda = 1.  The box is large enough never to be felt."""
    rng = np.random.default_rng(seed)
    n = 3
    c = np.full((n, 3), L / 2)
    pos = []
    boxes = []
    for w in range(n_walkers):
        p, b = quantize(c + rng.normal(0.0, 0.5, size=(n, 3)), np.array([L, L, L]), precision)
        pos.append(p)
        boxes.append(b)
    anchor, _ = quantize(np.tile(c, (n_walkers, 1)), boxes[0], precision)
    N = n * n_walkers
    spec = SystemSpec(
        atom_offset=np.arange(n_walkers + 1, dtype=np.int64) * n, box=np.array(boxes),
        pos=np.concatenate(pos), mass=np.ones(N), charge=np.zeros(N), sigma=np.ones(N),
        epsilon=np.zeros(N), is_solute=np.zeros(N, np.uint8), r_cut=2.5, r_skin=2.0, kT=1.0,
        gamma=1.0, dt=0.005, coulomb_k=1.0, accel_unit=1.0, seed=seed, precision=precision,
        anchor=anchor, k0=np.full(N, k0), k1=np.full(N, k1), name="harmonic")
    lam = LambdaSpec(lambda0=rng.uniform(0, 1, n_walkers), p_lambda0=None, m_lambda=10.0,
                     gamma_lambda=1.0, kT_lambda=1.0, elec_start=0.0, elec_end=1.0,
                     vdw_start=0.0, vdw_end=1.0, direction="decouple", n_bins=n_bins,
                     full_samples=full_samples, share_interval=1)
    return spec, lam


# ----------------------------------------------------------------------------
# charged LJ fluid in real units with a decoupled solute
# ----------------------------------------------------------------------------
SOLVENT_SIGMA = 3.15        # the literal sigma of the workload description
FLUID_SIGMA = 2.04          # sigma giving rho sigma^3 = 0.85 at 0.1 atoms/A^3
SOLVENT_EPS = 0.15
SOLVENT_Q = 0.4
SOLVENT_MASS = 18.015
SOLUTE_MASS = 12.011


def _solute_params(rng, n_solute: int, scale: float = 1.0):
    sig = rng.uniform(2.5, 3.8, n_solute) * scale
    eps = np.full(n_solute, 0.15)
    q = rng.uniform(-0.8, 0.8, n_solute)
    if n_solute:
        q[-1] = -np.sum(q[:-1])
    return sig, eps, q


SOLUTE_K = 100.0            # kcal/mol/A^2: restraint holding the solute's shape


def charged_lj(n_atoms: int = 30000, n_solute: int = 30, density: float = 0.1,
               seed: int = BASE_SEED + 1, precision: str = "fp32", r_cut: float = 12.0,
               r_skin: float = 1.0, temperature: float = 300.0, dt: float = 2.0,
               gamma_ps: float = 1.0, jitter: float = 0.05, sigma: float = FLUID_SIGMA,
               solute_k: float = SOLUTE_K, r_skin_alch: float = 0.0, lj_spread: float = 0.0):
    """One walker: n_atoms (solvent + solute) of a charged LJ fluid at 0.1
    atoms/A^3 on a seeded FCC lattice (+-jitter A).  Solvent charges are
    +-0.4 e on alternating (001) planes of the FCC basis (8 unlike and 4 like
    nearest neighbours), half of the solvent from each species, vacancies by
    a seeded permutation; the solvent sigma defaults to 2.04 A
    (rho sigma^3 = 0.85, a dense supercritical LJ fluid; with the literal
    3.15 A, rho sigma^3 = 3.1 is a compressed solid whose relaxation heats
    the system to ~10^4 K).  Pair counts depend on density and cutoff only.
    The solute: the n_solute cube-corner sites of the FCC cells (a simple
    cubic sub-lattice, spacing a = 3.42 A at this density) nearest the box
    centre, sigma ~ U(2.5, 3.8) A, eps 0.15, charges ~ U(-0.8, 0.8) summing
    to zero, each atom held to its initial site by a lambda-independent
    harmonic restraint (solute_k) that stands in for the molecule's bonded
    terms: an unbonded charged cluster left alone in vacuum at lambda = 1
    flies apart (~3000 K).
    Lambda: electrostatics removed over [0, 0.5], soft-core vdW over
    [0.5, 1] (decoupling), m_lambda = 150000 kcal/mol fs^2,
    gamma_lambda = 1000 /ps, 100 bins, fullSamples 100.
    lj_spread > 0 gives every solvent atom its own sigma and epsilon, each
    uniform within +-lj_spread (relative) of the defaults (a mixture, so that
    pairs take Lorentz-Berthelot mixed parameters)."""
    rng = np.random.default_rng(seed)
    L = (n_atoms / density) ** (1.0 / 3.0)
    n_cell = int(math.ceil((n_atoms / 4.0) ** (1.0 / 3.0) - 1e-9))
    sites = _lattice_fcc(n_cell, L)
    basis = np.arange(sites.shape[0]) % 4
    species = (basis >= 2).astype(np.int64)      # basis (0,0,0),(1/2,1/2,0): +; the others: -
    dc = np.linalg.norm(sites - L / 2, axis=1)
    corner = np.nonzero(basis == 0)[0]
    sol_sites = corner[np.argsort(dc[corner], kind="stable")[:n_solute]]
    free = np.ones(sites.shape[0], bool)
    free[sol_sites] = False
    n_solv = n_atoms - n_solute
    keep = [sol_sites]
    for p_ in (0, 1):
        idx = np.nonzero(free & (species == p_))[0]
        take = n_solv // 2 + (n_solv % 2 if p_ == 0 else 0)
        keep.append(idx[rng.permutation(idx.size)[:take]])
    keep = np.sort(np.concatenate(keep))
    pos = sites[keep] + rng.uniform(-jitter, jitter, size=(n_atoms, 3))
    pos, box = quantize(pos, np.array([L, L, L]), precision)
    # small boxes: keep r_cut + r_skin_alch inside half the box
    if r_skin_alch:
        r_skin_alch = max(r_skin, min(r_skin_alch, 0.49 * float(box.min()) - r_cut))
    solute = np.isin(keep, sol_sites).astype(np.uint8)
    charge = np.where(species[keep] == 0, SOLVENT_Q, -SOLVENT_Q).astype(np.float64)
    sig = np.full(n_atoms, sigma)
    eps = np.full(n_atoms, SOLVENT_EPS)
    mass = np.full(n_atoms, SOLVENT_MASS)
    s_sig, s_eps, s_q = _solute_params(rng, n_solute)
    idx = np.nonzero(solute)[0]
    if lj_spread > 0.0:
        env = np.nonzero(solute == 0)[0]
        sig[env] *= 1.0 + rng.uniform(-lj_spread, lj_spread, env.size)
        eps[env] *= 1.0 + rng.uniform(-lj_spread, lj_spread, env.size)
    sig[idx], eps[idx], charge[idx], mass[idx] = s_sig, s_eps, s_q, SOLUTE_MASS
    k = np.zeros(n_atoms)
    k[idx] = solute_k
    spec = SystemSpec(
        atom_offset=np.array([0, n_atoms], np.int64), box=box[None, :], pos=pos, mass=mass,
        charge=charge, sigma=sig, epsilon=eps, is_solute=solute, r_cut=r_cut, r_skin=r_skin,
        kT=KB_KCAL * temperature, gamma=gamma_ps * 1e-3, dt=dt, coulomb_k=COULOMB_K,
        accel_unit=ACCEL_REAL, seed=seed, precision=precision, r_skin_alch=r_skin_alch,
        anchor=pos.copy() if solute_k else None, k0=k if solute_k else None,
        k1=k.copy() if solute_k else None, name="charged_lj")
    lam = LambdaSpec(lambda0=np.array([0.0]), p_lambda0=None, m_lambda=150000.0,
                     gamma_lambda=1000.0 * 1e-3, kT_lambda=KB_KCAL * temperature,
                     elec_start=0.0, elec_end=0.5, vdw_start=0.5, vdw_end=1.0,
                     direction="decouple", sc_alpha=0.5, sc_power=1, n_bins=100, lo=0.0,
                     hi=1.0, full_samples=100, share_interval=1)
    return spec, lam


def with_pme(spec: SystemSpec, spacing: float = 1.1, tolerance: float = 1e-6, order: int = 4,
             dims=None, sizes: str = "pow2") -> SystemSpec:
    """The same system with Ewald electrostatics: per walker the smallest PME
    grid with spacing <= `spacing` A on each edge (sizes "pow2": powers of
    two; "235": multiples of 8 with no prime factor above 5), or the given
    dims; the splitting parameter beta with erfc(beta r_cut) = tolerance; and
    B-spline order `order`."""
    if dims is None:
        pick = _grid_pow2 if sizes == "pow2" else _grid_235
        dims = np.array([[pick(L / spacing, order) for L in b] for b in spec.box], np.int32)
    else:
        dims = np.broadcast_to(np.asarray(dims, np.int32), (spec.n_walkers, 3)).copy()
    lo, hi = 0.0, 10.0 / spec.r_cut
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if math.erfc(mid * spec.r_cut) > tolerance else (lo, mid)
    return dataclasses.replace(spec, pme_dims=dims, ewald_beta=0.5 * (lo + hi), pme_order=order,
                               name=spec.name + "_pme")


def _grid_235(x: float, floor: int) -> int:
    k = 16
    while True:
        r = k
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if k >= x and k >= floor and r == 1:
            return k
        k += 8


def _grid_pow2(x: float, floor: int) -> int:
    k = 1
    while k < x or k < floor:
        k *= 2
    return k


def batch(spec: SystemSpec, lam: LambdaSpec, n_walkers: int, seed: int):
    """n_walkers copies of a one-walker system (same coordinates and
    parameters, independent velocity streams through the walker index),
    initial lambda ~ U(0, 1)."""
    assert spec.n_walkers == 1
    rng = np.random.default_rng(seed)
    n = spec.n_atoms
    rep = lambda a: None if a is None else np.concatenate([a] * n_walkers)
    out = dataclasses.replace(
        spec, atom_offset=np.arange(n_walkers + 1, dtype=np.int64) * n,
        box=np.repeat(spec.box, n_walkers, axis=0), pos=rep(spec.pos), mass=rep(spec.mass),
        charge=rep(spec.charge), sigma=rep(spec.sigma), epsilon=rep(spec.epsilon),
        is_solute=rep(spec.is_solute), vel=None, anchor=rep(spec.anchor),
        k0=rep(spec.k0), k1=rep(spec.k1), seed=seed, name=spec.name + f"_x{n_walkers}",
        column_width=None if spec.column_width is None else np.repeat(spec.column_width, n_walkers),
        prune_buffer=None if spec.prune_buffer is None else np.repeat(spec.prune_buffer, n_walkers),
        pme_dims=None if spec.pme_dims is None else np.repeat(spec.pme_dims, n_walkers, axis=0))
    lam2 = dataclasses.replace(lam, lambda0=rng.uniform(0.0, 1.0, n_walkers), p_lambda0=None,
                               dr_pairs=None if lam.dr_pairs is None
                               else np.tile(np.asarray(lam.dr_pairs).reshape(1, 2), (n_walkers, 1)))
    return out, lam2


def ti_windows(spec: SystemSpec, lam: LambdaSpec, n_windows: int, replicas: int, seed: int):
    """Fixed-lambda thermodynamic integration: n_windows x replicas copies of
    a one-walker system, lambda frozen at the centres of n_windows equal bins
    on [lo, hi] (window-major order).  The per-bin mean of dV/dlambda is then
    the window average and the bin readout (Riemann sum) is the midpoint-rule
    TI estimate of the free-energy difference."""
    out, lam2 = batch(spec, lam, n_windows * replicas, seed=seed)
    w = (lam.hi - lam.lo) / n_windows
    centres = lam.lo + (np.arange(n_windows) + 0.5) * w
    lam2 = dataclasses.replace(lam2, lambda0=np.repeat(centres, replicas), n_bins=n_windows,
                               fixed_lambda=True, abf_on=True, p_lambda0=None)
    return out, lam2


def subset(spec: SystemSpec, lam: LambdaSpec, walkers) -> tuple:
    """The given walkers of a batch as a batch of their own."""
    walkers = [int(w) for w in walkers]
    sl = [spec.walker_slice(w) for w in walkers]
    pick = lambda a: None if a is None else np.concatenate([a[s] for s in sl])
    off = np.zeros(len(walkers) + 1, np.int64)
    off[1:] = np.cumsum([s.stop - s.start for s in sl])
    out = dataclasses.replace(
        spec, atom_offset=off, box=spec.box[walkers], pos=pick(spec.pos), vel=pick(spec.vel),
        mass=pick(spec.mass), charge=pick(spec.charge), sigma=pick(spec.sigma),
        epsilon=pick(spec.epsilon), is_solute=pick(spec.is_solute), anchor=pick(spec.anchor),
        k0=pick(spec.k0), k1=pick(spec.k1),
        column_width=None if spec.column_width is None else spec.column_width[walkers],
        prune_buffer=None if spec.prune_buffer is None else spec.prune_buffer[walkers],
        pme_dims=None if spec.pme_dims is None else spec.pme_dims[walkers])
    lam2 = dataclasses.replace(lam, lambda0=np.asarray(lam.lambda0)[walkers],
                               p_lambda0=None if lam.p_lambda0 is None
                               else np.asarray(lam.p_lambda0)[walkers],
                               dr_pairs=None if lam.dr_pairs is None
                               else np.asarray(lam.dr_pairs).reshape(-1, 2)[walkers])
    return out, lam2


def concat(specs, lam: LambdaSpec, lambda0: np.ndarray, seed: int, name: str):
    """Concatenate one-walker systems (which must share r_cut, units and
    precision) into one batch of uneven walkers."""
    W = len(specs)
    off = np.zeros(W + 1, np.int64)
    for w, s in enumerate(specs):
        off[w + 1] = off[w] + s.n_atoms
    cat = lambda f: np.concatenate([getattr(s, f) for s in specs])
    has_r = all(s.anchor is not None for s in specs)
    s0 = specs[0]
    out = dataclasses.replace(
        s0, atom_offset=off, box=np.concatenate([s.box for s in specs]), pos=cat("pos"),
        mass=cat("mass"), charge=cat("charge"), sigma=cat("sigma"), epsilon=cat("epsilon"),
        is_solute=cat("is_solute"), vel=None,
        anchor=cat("anchor") if has_r else None, k0=cat("k0") if has_r else None,
        k1=cat("k1") if has_r else None, seed=seed, name=name,
        column_width=np.concatenate([np.ones(1) if s.column_width is None else s.column_width
                                     for s in specs]),
        prune_buffer=np.concatenate([np.zeros(1) if s.prune_buffer is None else s.prune_buffer
                                     for s in specs]),
        pme_dims=None if s0.pme_dims is None else np.concatenate([s.pme_dims for s in specs]))
    lam2 = dataclasses.replace(lam, lambda0=np.asarray(lambda0, np.float64), p_lambda0=None)
    return out, lam2


def uneven(n_walkers: int = 64, n_min: int = 5000, n_max: int = 60000,
           seed: int = BASE_SEED + 3, precision: str = "fp32", r_cut: float = 12.0,
           r_skin: float = 1.2, r_skin_alch: float = 0.0):
    """Walkers with atom counts log-uniform in [n_min, n_max]: each a charged
    LJ solvent box around a dense cluster (0.12 atoms/A^3, FCC) restrained
    harmonically (k = 1 kcal/mol/A^2, lambda-independent) to its initial
    sites, with a 20-80 atom decoupled ligand just outside the cluster (on
    the cube-corner sub-lattice, restrained to its sites like the solute of
    charged_lj).  Solvent sites start SHELL and the ligand LIG_GAP outside
    the cluster so that no pair starts deep inside the LJ core.  The list
    buffer is 1.2 A: over ~1.4 M atoms the two largest displacements in 10
    steps reach 0.85-1.0 A (ballistic estimate and measurement), too close
    to a 1 A buffer."""
    rng = np.random.default_rng(seed)
    specs = []
    for w in range(n_walkers):
        N = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        n_cl = int(round(math.exp(rng.uniform(math.log(2000), math.log(20000)))))
        n_cl = int(np.clip(n_cl, 2000, N // 2))
        n_lig = int(rng.integers(20, 81))
        specs.append(_cluster_walker(rng, N, n_cl, n_lig, precision, r_cut, r_skin, seed + w,
                                     r_skin_alch))
    _, lam = charged_lj(n_atoms=3000, precision=precision)
    return concat(specs, lam, rng.uniform(0, 1, n_walkers), seed, "uneven")


SHELL = 2.2     # A: solvent sites start this far outside the cluster (about one sigma)
LIG_GAP = 3.5   # A: and the ligand this far (its sigma reaches 3.8 A)


def _cluster_walker(rng, N, n_cl, n_lig, precision, r_cut, r_skin, seed, r_skin_alch=0.0):
    vol = n_cl / 0.12 + (N - n_cl) / 0.1
    L = vol ** (1.0 / 3.0)
    R = (3.0 * n_cl / (4.0 * math.pi * 0.12)) ** (1.0 / 3.0)
    c = np.full(3, L / 2)
    # cluster: FCC at 0.12 inside the sphere (closest sites to the centre)
    a_cl = (4.0 / 0.12) ** (1.0 / 3.0)
    ncl_side = int(math.ceil(2 * R / a_cl)) + 2
    cl_sites = _lattice_fcc(ncl_side, ncl_side * a_cl) - ncl_side * a_cl / 2 + c
    cl_species = (np.arange(cl_sites.shape[0]) % 4) // 2
    dcl = np.linalg.norm(cl_sites - c, axis=1)
    cl_pick = np.argsort(dcl, kind="stable")[:n_cl]
    cl = cl_sites[cl_pick]
    R_eff = np.linalg.norm(cl - c, axis=1).max()
    # ligand: sites in a shell just outside the cluster, along a seeded direction
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    # solvent: FCC sites outside R + 1 A; the 1 A shell costs sites, so the
    # lattice is refined until enough remain (vacancies keep 0.1 atoms/A^3)
    n_solv = N - n_cl - n_lig
    n_side = int(math.ceil(L / (4.0 / 0.1) ** (1.0 / 3.0)))
    while True:
        solv_sites = _lattice_fcc(n_side, L)
        sv_basis = np.arange(solv_sites.shape[0]) % 4
        sv_species = sv_basis // 2
        ds = np.linalg.norm(solv_sites - c, axis=1)
        out_idx = np.nonzero(ds > R_eff + SHELL)[0]
        # ligand: the cube-corner sites (3.42 A apart) nearest a centre placed
        # so that the ligand ball starts LIG_GAP outside the cluster
        r_lig = (3.0 * n_lig * (4.0 / 0.1) / (4.0 * math.pi)) ** (1.0 / 3.0)
        lig_c = c + u * (R_eff + LIG_GAP + r_lig)
        corner = out_idx[(sv_basis[out_idx] == 0) & (ds[out_idx] > R_eff + LIG_GAP)]
        dl = np.linalg.norm(solv_sites[corner] - lig_c, axis=1)
        lig_idx = corner[np.argsort(dl, kind="stable")[:n_lig]]
        lig = solv_sites[lig_idx]
        rest_idx = np.setdiff1d(out_idx, lig_idx)
        if rest_idx.shape[0] >= n_solv:
            break
        n_side += 1
    pick = rest_idx[np.sort(rng.permutation(rest_idx.shape[0])[:n_solv])]
    solv = solv_sites[pick]
    species = np.concatenate([cl_species[cl_pick], np.zeros(n_lig, np.int64), sv_species[pick]])
    pos = np.concatenate([cl, lig, solv]) + rng.uniform(-0.05, 0.05, size=(N, 3))
    pos, box = quantize(pos, np.array([L, L, L]), precision)
    anchor = pos.copy()
    k = np.zeros(N)
    k[:n_cl] = 1.0
    k[n_cl:n_cl + n_lig] = SOLUTE_K
    solute = np.zeros(N, np.uint8)
    solute[n_cl:n_cl + n_lig] = 1
    sig = np.full(N, FLUID_SIGMA)
    eps = np.full(N, SOLVENT_EPS)
    mass = np.full(N, SOLVENT_MASS)
    charge = np.where(species == 0, SOLVENT_Q, -SOLVENT_Q).astype(np.float64)
    charge[solute == 1] = 0.0
    s_sig, s_eps, s_q = _solute_params(rng, n_lig)
    li = np.arange(n_cl, n_cl + n_lig)
    sig[li], eps[li], charge[li], mass[li] = s_sig, s_eps, s_q, SOLUTE_MASS
    return SystemSpec(
        atom_offset=np.array([0, N], np.int64), box=box[None, :], pos=pos, mass=mass,
        charge=charge, sigma=sig, epsilon=eps, is_solute=solute, r_cut=r_cut, r_skin=r_skin,
        kT=KB_KCAL * 300.0, gamma=1e-3, dt=2.0, coulomb_k=COULOMB_K, accel_unit=ACCEL_REAL,
        seed=seed, precision=precision, anchor=anchor, k0=k, k1=k.copy(), r_skin_alch=r_skin_alch,
        name="cluster")
