"""Pins of the oracle's Ewald electrostatics (smooth PME with the reciprocal
term interpolated linearly between the electrostatic end states).

The plain Ewald sum is pinned to the NaCl Madelung constant and to its own
independence of the splitting parameter beta (which holds only when the
real-space, reciprocal, self and neutralising-background terms are all
right).  The smooth-PME reciprocal term is pinned to that exact Ewald sum
as grid and spline order grow, and to finite differences.  The walker-level
evaluation is pinned to exact Ewald sums of the end states and to
finite differences in positions, lambda and charges.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2307_08006_amd import synth

# NaCl (rock salt) Madelung constant referred to the nearest-neighbour
# distance (e.g. Kittel, Introduction to Solid State Physics, ch. 3).
MADELUNG_NACL = 1.747564594633


def _rock_salt():
    x, q = [], []
    for i in range(2):
        for j in range(2):
            for k in range(2):
                x.append([i, j, k])
                q.append(1.0 if (i + j + k) % 2 == 0 else -1.0)
    return np.array(x, float) + 0.25, np.array(q), np.array([2.0, 2.0, 2.0])


@pytest.mark.parametrize("beta", [1.5, 2.5, 3.5])
def test_ewald_reproduces_nacl_madelung_constant(beta):
    x, q, L = _rock_salt()
    e, f = oracle.ewald_exact(x, q, L, beta, 7.0 / beta, int(np.ceil(3.2 * beta)) + 2)
    # 4 ion pairs per cell, nearest-neighbour distance 1: E = -4 M
    assert abs(e / 4 + MADELUNG_NACL) < 1e-10
    assert np.abs(f).max() < 1e-10           # every ion sits at a centre of symmetry


def _random_charges(n=24, seed=5, net=0.0):
    rng = np.random.default_rng(seed)
    L = np.array([3.0, 3.4, 2.8])
    x = rng.uniform(0, 1, (n, 3)) * L
    q = rng.normal(size=n)
    q += net / n - q.mean()
    return x, q, L


@pytest.mark.parametrize("net", [0.0, 1.3])
def test_ewald_is_independent_of_beta(net):
    """Total energy and forces do not depend on the splitting; with a net
    charge this holds only with the neutralising-background term."""
    x, q, L = _random_charges(net=net)
    ref = None
    for beta in (1.6, 2.2, 3.0):
        e, f = oracle.ewald_exact(x, q, L, beta, 7.0 / beta, int(np.ceil(3.3 * beta * L.max() / np.pi)) + 2)
        if ref is None:
            ref = (e, f)
        else:
            assert abs(e - ref[0]) < 1e-9 * abs(ref[0]), (beta, e, ref[0])
            assert np.abs(f - ref[1]).max() < 1e-8 * np.abs(ref[1]).max()


def test_ewald_forces_are_minus_gradient():
    x, q, L = _random_charges(n=10, net=0.4)
    beta, rr, km = 2.0, 3.5, 10
    _, f = oracle.ewald_exact(x, q, L, beta, rr, km)
    h = 1e-6
    for i in (0, 3, 7):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = -(oracle.ewald_exact(xp, q, L, beta, rr, km)[0] - oracle.ewald_exact(xm, q, L, beta, rr, km)[0]) / (2 * h)
            assert abs(f[i, k] - fd) < 1e-6 * max(1.0, abs(fd))


def test_spme_converges_to_exact_reciprocal_sum():
    """SPME + self + background -> the k-space Ewald sum (real space removed
    by a vanishing real-space radius) as grid and order grow."""
    x, q, L = _random_charges(n=30, net=0.7)
    beta = 3.0
    e_ex, f_ex = oracle.ewald_exact(x, q, L, beta, 1e-9, 14)
    V = L.prod()
    rest = -beta / np.sqrt(np.pi) * (q * q).sum() - np.pi * q.sum() ** 2 / (2 * V * beta * beta)
    errs = []
    for dims, p in (((16,) * 3, 4), ((32,) * 3, 6), ((64,) * 3, 8)):
        e, f = oracle.spme_energy(x, q, L, beta, dims, p)
        errs.append((abs(e + rest - e_ex), np.abs(f - f_ex).max()))
    assert errs[0][0] > errs[1][0] > errs[2][0] and errs[0][1] > errs[1][1] > errs[2][1]
    assert errs[2][0] < 1e-8 * abs(e_ex) and errs[2][1] < 1e-6 * np.abs(f_ex).max(), errs


def test_spme_on_the_papers_grid_sizes_converges_to_exact_sum():
    """Grids of 2^a 3^b 5^c points (24^3 and 48^3 as in the paper's Tinker
    runs, and a mixed 40 x 48 x 24): SPME + self + background against the
    exact k-space sum, the error shrinking with grid and order."""
    x, q, L = _random_charges(n=30, net=0.4)
    beta = 3.0
    e_ex, f_ex = oracle.ewald_exact(x, q, L, beta, 1e-9, 14)
    V = L.prod()
    rest = -beta / np.sqrt(np.pi) * (q * q).sum() - np.pi * q.sum() ** 2 / (2 * V * beta * beta)
    errs = []
    for dims, p in (((24,) * 3, 6), ((40, 48, 24), 6), ((48,) * 3, 8)):
        e, f = oracle.spme_energy(x, q, L, beta, dims, p)
        errs.append((abs(e + rest - e_ex), np.abs(f - f_ex).max()))
    assert errs[0][0] > errs[2][0] and errs[0][1] > errs[2][1]
    assert errs[2][0] < 1e-7 * abs(e_ex) and errs[2][1] < 1e-5 * np.abs(f_ex).max(), errs


def test_spme_forces_are_minus_gradient():
    x, q, L = _random_charges(n=12)
    args = (L, 2.0, (16, 16, 16), 4)
    _, f = oracle.spme_energy(x, q, *args)
    h = 1e-6
    for i in (0, 5, 11):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = -(oracle.spme_energy(xp, q, *args)[0] - oracle.spme_energy(xm, q, *args)[0]) / (2 * h)
            assert abs(f[i, k] - fd) < 1e-6 * max(1.0, abs(fd))


def test_spme_is_translation_invariant_on_grid_shifts():
    """Moving every charge by whole grid cells leaves the SPME energy and
    forces unchanged (the B-spline weights are the same, shifted)."""
    x, q, L = _random_charges(n=15)
    dims = (16, 32, 16)
    e0, f0 = oracle.spme_energy(x, q, L, 2.5, dims, 6)
    x1 = x + np.array([3, 5, 15]) * L / np.array(dims)
    e1, f1 = oracle.spme_energy(x1, q, L, 2.5, dims, 6)
    assert abs(e1 - e0) < 1e-12 * abs(e0)
    assert np.abs(f1 - f0).max() < 1e-10 * np.abs(f0).max()


# --------------------------------------------------------------------------
# walker level: real space erfc pairs + reciprocal with the interpolation
# --------------------------------------------------------------------------
def _pme_small(dims=(64, 64, 64), order=8, solute_q=None):
    spec, lam = synth.lj_reduced(n_atoms=125, density=0.5, seed=7, jitter=0.15, charges=0.5,
                                 r_cut=2.5)
    spec.is_solute[:] = 0
    spec.is_solute[:3] = 1
    spec.sigma[:3] = [0.9, 1.2, 1.05]
    spec.epsilon[:3] = [0.8, 1.3, 0.5]
    if solute_q is not None:
        spec.charge[:3] = solute_q
    lam.elec_start, lam.elec_end, lam.vdw_start, lam.vdw_end = 0.0, 0.5, 0.5, 1.0
    return synth.with_pme(spec, dims=dims, order=order), lam


def _coulomb(spec, lam, x, l):
    """Electrostatic part: the evaluation minus the same with no charges."""
    f, u, g = oracle.Oracle(spec, lam).evaluate(0, x, l)
    s0 = dataclasses.replace(spec, charge=np.zeros_like(spec.charge))
    f0, u0, g0 = oracle.Oracle(s0, lam).evaluate(0, x, l)
    return f - f0, u.sum() - u0.sum(), g - g0, u


def _ewald(spec, x, sel):
    return oracle.ewald_exact(x[sel], spec.charge[sel], spec.box[0], spec.ewald_beta, spec.r_cut, 20)


@pytest.mark.parametrize("solute_q", [None, [0.7, -0.2, 0.6]])
def test_pme_walker_end_states_are_exact_ewald_sums(solute_q):
    """ce = 1: the Ewald sum of all charges (pairs cut at r_cut);
    ce = 0: the sum of the environment's and the group's own Ewald sums.
    The second case has a charged group, so the background cross term
    matters."""
    spec, lam = _pme_small(solute_q=solute_q)
    x = spec.pos
    s = spec.is_solute.astype(bool)
    f1, u1, _, _ = _coulomb(spec, lam, x, 0.0)
    e_all, f_all = _ewald(spec, x, np.ones_like(s))
    assert abs(u1 - e_all) < 1e-8 * abs(e_all), (u1, e_all)
    assert np.abs(f1 - f_all).max() < 1e-7 * np.abs(f_all).max()
    f0, u0, _, _ = _coulomb(spec, lam, x, 0.7)
    eE, fE = _ewald(spec, x, ~s)
    eS, fS = _ewald(spec, x, s)
    assert abs(u0 - eE - eS) < 1e-8 * abs(eE + eS), (u0, eE + eS)
    fsep = np.zeros_like(f0)
    fsep[~s], fsep[s] = fE, fS
    assert np.abs(f0 - fsep).max() < 1e-7 * np.abs(fsep).max()


def test_pme_walker_interpolates_linearly_and_dudl_is_the_end_state_gap():
    spec, lam = _pme_small(dims=(16, 16, 16), order=4, solute_q=[0.7, -0.2, 0.6])
    x = spec.pos
    _, v1, _, _ = _coulomb(spec, lam, x, 0.0)     # ce = 1
    _, v0, _, _ = _coulomb(spec, lam, x, 0.5)     # ce = 0
    for l in (0.1, 0.25, 0.4):
        ce = 1.0 - 2.0 * l
        _, v, g, _ = _coulomb(spec, lam, x, l)
        assert abs(v - ((1 - ce) * v0 + ce * v1)) < 1e-12 * abs(v1)
        assert abs(g - (-2.0) * (v1 - v0)) < 1e-11 * abs(v1 - v0)


@pytest.mark.parametrize("l", [0.15, 0.35, 0.8])
def test_pme_walker_forces_and_dudl_are_gradients(l):
    spec, lam = _pme_small(dims=(16, 16, 16), order=4, solute_q=[0.7, -0.2, 0.6])
    o = oracle.Oracle(spec, lam)
    x = spec.pos.copy()
    f, _, g = o.evaluate(0, x, l)
    E = lambda xx, ll: o.evaluate(0, xx, ll)[1].sum()
    h = 1e-6
    for i in (0, 1, 2, 40, 90):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = -(E(xp, l) - E(xm, l)) / (2 * h)
            assert abs(f[i, k] - fd) < 1e-6 * max(1.0, abs(fd)), (i, k, f[i, k], fd)
    hl = 1e-6
    fd = (E(x, l + hl) - E(x, l - hl)) / (2 * hl)
    assert abs(g - fd) < 1e-6 * max(1.0, abs(g)), (g, fd)


def test_pme_walker_charge_gradient_matches_finite_difference():
    spec, lam = _pme_small(dims=(16, 16, 16), order=4, solute_q=[0.7, -0.2, 0.6])
    l = 0.2
    g = oracle.Oracle(spec, lam).param_grad(0, spec.pos, l)
    h = 1e-5
    for i in (0, 2, 10, 77):
        vals = []
        for sgn in (+1, -1):
            sp = dataclasses.replace(spec, charge=spec.charge.copy())
            sp.charge[i] += sgn * h
            vals.append(oracle.Oracle(sp, lam).evaluate(0, spec.pos, l)[1].sum())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(g[i, 2] - fd) < 1e-6 * max(1.0, abs(fd)), (i, g[i, 2], fd)


def test_pme_rejects_bad_grids():
    spec, lam = _pme_small(dims=(16, 16, 16), order=4)
    for dims, order in (((16, 28, 16), 4), ((16, 16, 16), 5), ((16, 16, 16), 10), ((2, 16, 16), 4),
                        ((0, 16, 16), 4), ((16, -8, 16), 4)):
        sp = dataclasses.replace(spec, pme_dims=np.array([dims], np.int32), pme_order=order)
        with pytest.raises(ValueError):
            oracle.Oracle(sp, lam).evaluate(0, sp.pos, 0.1)
