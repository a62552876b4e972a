"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself through a retyped formula: each
test uses a printed value (golden files with citations), a closed form, a
special case that reduces to a textbook expression, a finite difference, a
brute-force enumeration or a conservation law.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2307_08006_amd import synth
from conftest import read_golden


def _sys(direction="decouple", es=0.0, ee=0.5, vs=0.5, ve=1.0, **kw):
    spec, lam = synth.lj_reduced(n_atoms=125, density=0.5, r_cut=2.5, r_skin=0.2, **kw)
    lam.direction, lam.elec_start, lam.elec_end, lam.vdw_start, lam.vdw_end = direction, es, ee, vs, ve
    return spec, lam


# --------------------------------------------------------------------------
# alchemical schedule
# --------------------------------------------------------------------------
def test_schedule_reproduces_si_table():
    spec, lam = _sys(direction="couple", es=0.5, ee=1.0, vs=0.0, ve=0.5)
    o = oracle.Oracle(spec, lam)
    rows = read_golden("si_lambda_schedule.txt")
    assert len(rows) == 24
    for l, le, lv in rows:
        ce, cv, _, _ = o.schedule(float(l))
        assert abs(ce - float(le)) < 1e-12 and abs(cv - float(lv)) < 1e-12, (l, ce, cv)


def test_schedule_decoupling_is_one_minus_clips():
    spec, lam = _sys()
    o = oracle.Oracle(spec, lam)
    for l in np.linspace(0, 1, 101):
        ce, cv, dce, dcv = o.schedule(l)
        assert abs(ce - (1 - np.clip(2 * l, 0, 1))) < 1e-15
        assert abs(cv - (1 - np.clip(2 * l - 1, 0, 1))) < 1e-15


@pytest.mark.parametrize("direction", ["couple", "decouple"])
def test_schedule_derivative_is_one_sided_slope(direction):
    spec, lam = _sys(direction=direction)
    o = oracle.Oracle(spec, lam)
    h = 1e-7
    for l in [0.0, 0.1, 0.3, 0.49, 0.5, 0.51, 0.7, 0.99, 1.0]:
        _, _, dce, dcv = o.schedule(l)
        lo, hi = (l - h, l) if l == 1.0 else (l, l + h)
        a, b = o.schedule(lo), o.schedule(hi)
        assert abs(dce - (b[0] - a[0]) / h) < 1e-6
        assert abs(dcv - (b[1] - a[1]) / h) < 1e-6


# --------------------------------------------------------------------------
# pair terms
# --------------------------------------------------------------------------
def test_softcore_worked_values():
    # alpha 0.5, p 1, unshifted; eps = sigma = 1
    t = oracle.pair_terms(1.0, 1.0, 1.0, 0.0, cv=1.0, ce=1.0)
    assert abs(t[0]) < 1e-15                       # U(sigma) = 0 at full coupling
    t = oracle.pair_terms(2 ** (1 / 6), 1.0, 1.0, 0.0, cv=1.0, ce=1.0)
    assert abs(t[0] + 1.0) < 1e-14 and abs(t[2]) < 1e-13   # minimum: -eps, zero force
    t = oracle.pair_terms(1.0, 1.0, 1.0, 0.0, cv=0.5, ce=1.0)
    assert abs(t[0] + 0.32) < 1e-14 and abs(t[1] + 0.256) < 1e-14  # s = 0.8
    t = oracle.pair_terms(0.0, 1.0, 1.0, 0.0, cv=0.0, ce=1.0)
    assert t[0] == 0.0 and abs(t[1] - 8.0) < 1e-14  # finite soft core at r = 0
    t = oracle.pair_terms(1.0, 1.0, 2.5, 0.0, cv=0.0, ce=1.0)
    assert t[0] == 0.0 and t[2] == 0.0              # fully decoupled: no LJ


def test_softcore_full_coupling_is_textbook_lj():
    for sig, eps in [(1.0, 1.0), (3.15, 0.15), (2.7, 0.3)]:
        for r in np.linspace(0.8 * sig, 3 * sig, 17):
            t = oracle.pair_terms(r, sig, eps, 0.0, 1.0, 1.0, r_cut=4 * sig, shift=True)
            x = (sig / r) ** 6
            xc = (sig / (4 * sig)) ** 6
            u = 4 * eps * (x * x - x) - 4 * eps * (xc * xc - xc)
            f = 24 * eps * (2 * x * x - x) / r          # textbook -dU/dr
            assert abs(t[0] - u) <= 1e-12 * max(1, abs(u))
            assert abs(t[2] * r - f) <= 1e-12 * max(1, abs(f))


def test_shifted_force_coulomb_values():
    rc, qq = 12.0, 332.0637 * 0.4 * -0.4
    t = oracle.pair_terms(rc, 1.0, 0.0, qq, 1.0, 1.0, r_cut=rc)
    assert abs(t[3]) < 1e-12 and abs(t[5]) < 1e-12
    t = oracle.pair_terms(rc / 2, 1.0, 0.0, qq, 1.0, 1.0, r_cut=rc)
    assert abs(t[3] - qq / (2 * rc)) < 1e-12 * abs(qq)
    assert abs(t[5] * (rc / 2) - 3 * qq / rc ** 2) < 1e-12 * abs(qq)
    t = oracle.pair_terms(rc / 2, 1.0, 0.0, qq, 1.0, 0.25, r_cut=rc)
    assert abs(t[3] - 0.25 * qq / (2 * rc)) < 1e-12 * abs(qq) and abs(t[4] - qq / (2 * rc)) < 1e-12 * abs(qq)


@pytest.mark.parametrize("cv,ce", [(1.0, 1.0), (0.3, 0.7), (0.05, 0.0), (0.9, 0.2)])
def test_pair_force_and_coupling_derivative_match_fd(cv, ce):
    sig, eps, qq, rc = 3.0, 0.2, 40.0, 12.0
    h = 1e-6
    for r in [2.0, 2.9, 3.4, 5.0, 9.0]:
        t = oracle.pair_terms(r, sig, eps, qq, cv, ce, r_cut=rc, shift=True)
        up = oracle.pair_terms(r + h, sig, eps, qq, cv, ce, r_cut=rc, shift=True)
        dn = oracle.pair_terms(r - h, sig, eps, qq, cv, ce, r_cut=rc, shift=True)
        dudr = ((up[0] + up[3]) - (dn[0] + dn[3])) / (2 * h)
        assert abs((t[2] + t[5]) * r + dudr) < 1e-6 * max(1, abs(dudr))
        hc = 1e-6
        a = oracle.pair_terms(r, sig, eps, qq, cv + hc, ce, r_cut=rc, shift=True)
        b = oracle.pair_terms(r, sig, eps, qq, cv - hc, ce, r_cut=rc, shift=True)
        assert abs(t[1] - (a[0] - b[0]) / (2 * hc)) < 1e-6 * max(1, abs(t[1]))
        a = oracle.pair_terms(r, sig, eps, qq, cv, ce + hc, r_cut=rc, shift=True)
        b = oracle.pair_terms(r, sig, eps, qq, cv, ce - hc, r_cut=rc, shift=True)
        assert abs(t[4] - (a[3] - b[3]) / (2 * hc)) < 1e-6 * max(1, abs(t[4]))


# --------------------------------------------------------------------------
# neighbour set
# --------------------------------------------------------------------------
def _brute_set(x, L, rl):
    n = x.shape[0]
    out = set()
    for i in range(n):
        for j in range(i + 1, n):
            d = x[j] - x[i]
            d = d - L * np.rint(d / L)
            if float(d @ d) < rl * rl:
                out.add((i, j))
    return out


@pytest.mark.parametrize("n,dens,seed", [(64, 0.5, 1), (200, 0.8, 2), (512, 0.8, 3), (343, 0.3, 4)])
def test_cell_list_equals_brute_force(n, dens, seed):
    spec, lam = synth.lj_reduced(n_atoms=n, density=dens, seed=seed, jitter=0.3)
    o = oracle.Oracle(spec, lam)
    L = spec.box[0]
    rl = 2.8 if L[0] > 3 * 2.8 else L[0] / 3.2
    a = o.neighbor_pairs(0, spec.pos, rl, brute=False)
    b = o.neighbor_pairs(0, spec.pos, rl, brute=True)
    assert np.array_equal(a, b)
    assert set(map(tuple, a.tolist())) == _brute_set(spec.pos, L, rl)


def test_neighbor_boundary_pairs_are_strict():
    # pairs placed at r_list (1 +- k ulp), also across the periodic boundary
    spec, lam = synth.lj_reduced(n_atoms=4, density=4 / 1000.0, seed=5)
    L = 10.0
    spec.box[:] = L
    rl = 3.0
    o = oracle.Oracle(spec, lam)
    for k in [-2, -1, 0, 1, 2]:
        r = rl + k * np.spacing(rl)
        x = np.array([[1.0, 5.0, 5.0], [1.0 + r, 5.0, 5.0], [9.5, 1.0, 1.0], [9.5 - L + L, 1.0, 1.0]])
        x[3] = [(9.5 + r) % L, 1.0, 1.0]
        pairs = set(map(tuple, o.neighbor_pairs(0, x, rl, brute=True).tolist()))
        # the FP64 separation decides; compare with the same definition done by hand
        assert ((0, 1) in pairs) == (((1.0 + r) - 1.0) ** 2 < rl * rl)
        d = x[3, 0] - x[2, 0]
        d -= L * np.rint(d / L)
        assert ((2, 3) in pairs) == (d * d < rl * rl)


# --------------------------------------------------------------------------
# forces, dU/dlambda, endpoints
# --------------------------------------------------------------------------
def _charged_small(seed=7, n_sol=3, form="beutler"):
    spec, lam = synth.lj_reduced(n_atoms=125, density=0.5, seed=seed, jitter=0.15, charges=0.5,
                                 r_cut=2.5)
    lam.sc_form, lam.sc_shift = form, 0.5
    spec.is_solute[:] = 0
    spec.is_solute[:n_sol] = 1
    spec.sigma[:n_sol] = [0.9, 1.2, 1.05][:n_sol]
    spec.epsilon[:n_sol] = [0.8, 1.3, 0.5][:n_sol]
    lam.elec_start, lam.elec_end, lam.vdw_start, lam.vdw_end = 0.0, 0.5, 0.5, 1.0
    return spec, lam


def _energy(o, x, l):
    _, u, _ = o.evaluate(0, x, l)
    return u.sum()


@pytest.mark.parametrize("l", [0.0, 0.2, 0.6, 0.95])
def test_forces_are_minus_energy_gradient(l):
    spec, lam = _charged_small()
    o = oracle.Oracle(spec, lam)
    x = spec.pos.copy()
    f, _, _ = o.evaluate(0, x, l)
    h = 1e-6
    rng = np.random.default_rng(3)
    for i in rng.choice(64, 10, replace=False):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = -(_energy(o, xp, l) - _energy(o, xm, l)) / (2 * h)
            assert abs(f[i, k] - fd) < 1e-6 * max(1.0, abs(fd)), (i, k, f[i, k], fd)


def test_pair_forces_sum_to_zero():
    spec, lam = _charged_small()
    o = oracle.Oracle(spec, lam)
    f, _, _ = o.evaluate(0, spec.pos, 0.3)
    assert np.abs(f.sum(axis=0)).max() < 1e-12 * np.abs(f).sum()


@pytest.mark.parametrize("l", [0.0, 0.15, 0.4, 0.62, 0.8, 1.0])
def test_dudl_matches_energy_finite_difference(l):
    spec, lam = _charged_small()
    o = oracle.Oracle(spec, lam)
    _, _, g = o.evaluate(0, spec.pos, l)
    h = 1e-4
    if l == 0.0:
        fd = (-3 * _energy(o, spec.pos, 0) + 4 * _energy(o, spec.pos, h) - _energy(o, spec.pos, 2 * h)) / (2 * h)
    elif l == 1.0:
        fd = (3 * _energy(o, spec.pos, 1) - 4 * _energy(o, spec.pos, 1 - h) + _energy(o, spec.pos, 1 - 2 * h)) / (2 * h)
    else:
        fd = (_energy(o, spec.pos, l + h) - _energy(o, spec.pos, l - h)) / (2 * h)
    assert abs(g - fd) < 1e-7 * max(1.0, abs(g)), (g, fd)


def test_lambda0_endpoint_is_plain_lj_plus_sf_coulomb():
    spec, lam = _charged_small()
    o = oracle.Oracle(spec, lam)
    _, u, _ = o.evaluate(0, spec.pos, 0.0, brute=True)
    # textbook shifted LJ + shifted-force Coulomb over all pairs, brute force
    x, L, rc = spec.pos, spec.box[0], spec.r_cut
    tot = 0.0
    n = spec.n_atoms
    for i in range(n):
        for j in range(i + 1, n):
            d = x[j] - x[i]
            d -= L * np.rint(d / L)
            r = math.sqrt(d @ d)
            if r >= rc:
                continue
            s = 0.5 * (spec.sigma[i] + spec.sigma[j])
            e = math.sqrt(spec.epsilon[i] * spec.epsilon[j])
            a, ac = (s / r) ** 6, (s / rc) ** 6
            tot += 4 * e * (a * a - a) - 4 * e * (ac * ac - ac)
            qq = spec.charge[i] * spec.charge[j]
            tot += qq * (1 / r - 1 / rc + (r - rc) / rc ** 2)
    assert abs(u.sum() - tot) <= 1e-13 * abs(tot)


def test_lambda1_endpoint_removes_solute_environment_terms():
    spec, lam = _charged_small()
    o = oracle.Oracle(spec, lam)
    f, u, _ = o.evaluate(0, spec.pos, 1.0)
    assert u[2] == 0.0 and u[3] == 0.0
    # same energy as environment-only plus solute-only systems
    env = spec.is_solute == 0
    spec_e, _ = _charged_small()
    spec_e.epsilon[~env] = 0.0
    spec_e.charge[~env] = 0.0
    spec_s, _ = _charged_small()
    spec_s.epsilon[env] = 0.0
    spec_s.charge[env] = 0.0
    ue = oracle.Oracle(spec_e, lam).evaluate(0, spec.pos, 1.0)[1].sum()
    us = oracle.Oracle(spec_s, lam).evaluate(0, spec.pos, 1.0)[1].sum()
    assert abs(u.sum() - (ue + us)) <= 1e-13 * abs(u.sum())


def test_parameter_gradient_matches_fd():
    spec, lam = _charged_small()
    l = 0.7
    o = oracle.Oracle(spec, lam)
    g = o.param_grad(0, spec.pos, l)
    h = 1e-5
    for i in [0, 1, 2, 10]:
        for k, field in enumerate(["epsilon", "sigma", "charge"]):
            vals = []
            for sgn in (+1, -1):
                sp, _ = _charged_small()
                getattr(sp, field)[i] += sgn * h
                vals.append(oracle.Oracle(sp, lam).evaluate(0, spec.pos, l)[1].sum())
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(g[i, k] - fd) < 1e-6 * max(1.0, abs(fd)), (i, field, g[i, k], fd)


def test_restraint_energy_force_and_dudl():
    spec, lam = synth.harmonic(n_walkers=1)
    o = oracle.Oracle(spec, lam)
    x = spec.pos
    for l in [0.0, 0.37, 1.0]:
        f, u, g = o.evaluate(0, x, l)
        d = x - spec.anchor
        k = 1.0 + 3.0 * l
        assert abs(u[4] - 0.5 * k * (d * d).sum()) < 1e-12
        assert np.allclose(f, -k * d, rtol=0, atol=1e-12)
        assert abs(g - 1.5 * (d * d).sum()) < 1e-12


# --------------------------------------------------------------------------
# noise
# --------------------------------------------------------------------------
def test_philox_known_answers():
    for row in read_golden("philox4x32_10_kat.txt"):
        v = [int(t, 16) for t in row]
        assert oracle.philox4x32_10(v[:4], v[4:6]).tolist() == v[6:]


def test_normals_have_unit_moments():
    z = np.array([oracle.normals(12345, a, 7, 3, 0) for a in range(20000)]).ravel()
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.02
    assert abs((z ** 4).mean() - 3.0) < 0.1


def test_normals_invert_to_their_philox_uniforms():
    """Box-Muller maps the uniforms u1 = (a + 1) 2^-32 in (0, 1] and
    u2 = b 2^-32 of the Philox output words (a, b) to a pair whose squared
    radius is -2 ln u1 and whose angle is 2 pi u2: checked by inverting the
    oracle's normals against the known-answer-pinned Philox words, so a
    swapped pair, a dropped +1 or a wrong scale of either uniform fails."""
    seed, w, step = 0x0123456789ABCDEF, 5, 17
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for atom in (0, 1, 2, 77, 4095, 0xFFFFFFFF):
        words = oracle.philox4x32_10([atom, step, w, 0], key)
        z = oracle.normals(seed, atom, step, w, 0)
        for k in range(2):
            a, b = int(words[2 * k]), int(words[2 * k + 1])
            u1 = (a + 1) * 2.0 ** -32
            u2 = b * 2.0 ** -32
            z0, z1 = z[2 * k], z[2 * k + 1]
            assert abs((z0 * z0 + z1 * z1) - (-2.0 * math.log(u1))) <= 1e-12 * max(1.0, -2.0 * math.log(u1))
            ang = math.atan2(z1, z0) % (2.0 * math.pi)
            d = abs(ang - 2.0 * math.pi * u2)
            assert min(d, 2.0 * math.pi - d) <= 1e-9, (atom, k, ang, u2)


def test_initial_velocities_are_maxwell_boltzmann():
    """Initial atom velocities sample exp(-m v^2 / 2kT) per component (in
    units where a force/mass factor a converts kcal/mol/A/amu: variance
    kT a / m), and lambda momenta exp(-p^2 / 2 m_lambda kT): per-walker draws
    differ, and the sample variances of 3 x 30,000 components (two masses)
    and of 4,000 lambda momenta agree with those within 4 standard errors."""
    spec, lam = synth.charged_lj(n_atoms=30000, precision="fp64")
    spec, lamb = synth.batch(spec, lam, 2, seed=3)
    o = oracle.Oracle(spec, lamb)
    st = o.init_state()
    v = st["v"]
    m = np.asarray(spec.mass)
    for mass in np.unique(m):
        sel = v[m == mass]
        want = spec.kT * spec.accel_unit / mass
        got = float((sel * sel).mean())
        se = want * math.sqrt(2.0 / sel.size)
        assert abs(got - want) <= 4 * se + 1e-300, (mass, got, want)
    n0 = spec.walker_slice(0).stop
    assert not np.array_equal(v[:n0], v[n0:])
    # lambda momenta: 4000 walkers of the 3-particle system
    hs, hl = synth.harmonic(n_walkers=4000, seed=5)
    oh = oracle.Oracle(hs, hl)
    sh = oh.init_state()
    p = sh["p_lambda"]
    want = hl.m_lambda * hl.kT_lambda
    assert abs(float((p * p).mean()) - want) <= 4 * want * math.sqrt(2.0 / p.size)
    assert abs(float(p.mean())) <= 4 * math.sqrt(want / p.size)


def test_units_standard_state_correction():
    (t, ratio, val, digits), = read_golden("units_standard_state.txt")
    corr = synth.KB_KCAL * float(t) * math.log(float(ratio))
    assert round(corr, int(digits)) == float(val)


# --------------------------------------------------------------------------
# ABF accumulator and readout
# --------------------------------------------------------------------------
def test_abf_readout_is_riemann_sum_of_bin_means():
    n = 10
    count = np.arange(1, n + 1, dtype=np.int64)
    grad = np.linspace(-3, 5, n)
    g, prof, da, rc = oracle.abf_readout(count, grad * count, 0.0, 1.0)
    assert rc == 0 and np.allclose(g, grad)
    assert abs(da - grad.sum() / n) < 1e-14
    assert np.allclose(prof, np.concatenate([[0], np.cumsum(grad)[:-1]]) / n)
    count[3] = 0
    assert oracle.abf_readout(count, grad * count, 0.0, 1.0)[3] == -7


def _bias_state(n_bins=10, full=100, W=2):
    spec, lam = synth.harmonic(n_walkers=W)
    lam.n_bins, lam.full_samples = n_bins, full
    o = oracle.Oracle(spec, lam)
    o.init_state()
    z = dict(bin_count=np.zeros(n_bins, np.int64), bin_sum=np.zeros(n_bins),
             loc_count=np.zeros((W, n_bins), np.int64), loc_sum=np.zeros((W, n_bins)))
    return o, z


def test_abf_bias_hand_computed_states():
    """The bias force on lambda (the blue term of Eq. lambda-abf) for
    constructed accumulator states, computed by hand: ramp(n) = min(1,
    n / fullSamples) on the bin's combined count (shared + the walker's own
    unshared samples), times that bin's mean; 0 for an empty bin.  A ramp
    fixed at 1, an uncapped n / N_full, a mean over the shared samples only
    or over another walker's deltas each fail one of these values."""
    o, z = _bias_state()
    # bin 3 (lambda in [0.3, 0.4)): 30 shared samples summing to 60
    z["bin_count"][3], z["bin_sum"][3] = 30, 60.0
    # walker 0 holds 20 unshared samples of bin 3 summing to 10; walker 1 none
    z["loc_count"][0, 3], z["loc_sum"][0, 3] = 20, 10.0
    # bin 7: 150 shared samples summing to -300 (beyond full_samples)
    z["bin_count"][7], z["bin_sum"][7] = 150, -300.0
    # bin 8: only walker 1's unshared samples, 250 of them summing to 500
    z["loc_count"][1, 8], z["loc_sum"][1, 8] = 250, 500.0
    o.load_state(**z)
    # walker 1, bin 3: n = 30, ramp 0.3, mean 2        -> 0.6
    assert o.abf_bias(1, 0.35) == pytest.approx(0.6, abs=1e-15)
    # walker 0, bin 3: n = 50, ramp 0.5, mean 70/50    -> 0.7
    assert o.abf_bias(0, 0.35) == pytest.approx(0.7, abs=1e-15)
    # bin 7: n = 150 >= 100, ramp 1, mean -2           -> -2
    assert o.abf_bias(0, 0.75) == pytest.approx(-2.0, abs=1e-15)
    # bin 8: walker 1 sees its own 250 samples (mean 2) -> 2; walker 0 sees nothing -> 0
    assert o.abf_bias(1, 0.85) == pytest.approx(2.0, abs=1e-15)
    assert o.abf_bias(0, 0.85) == 0.0
    # an empty bin, and lambda = hi falling into the last bin (empty)
    assert o.abf_bias(0, 0.05) == 0.0 and o.abf_bias(1, 1.0) == 0.0
    # exactly full_samples: ramp 1
    z["bin_count"][5], z["bin_sum"][5] = 100, 25.0
    o.load_state(**z)
    assert o.abf_bias(0, 0.5) == pytest.approx(0.25, abs=1e-15)


def test_abf_bias_drives_the_first_steps_as_constructed():
    """One oracle step from a constructed accumulator: the lambda momentum
    of a walker with dV/dlambda = 0 (no atoms interact, k0 = k1) and no
    friction changes by exactly dt/2 times the hand-computed bias over the
    opening half-kick, so the step uses the frozen state as constructed."""
    spec, lam = synth.harmonic(n_walkers=1, k0=1.0, k1=1.0)
    lam.n_bins, lam.full_samples, lam.gamma_lambda = 10, 100, 0.0
    lam.lambda0, lam.p_lambda0 = np.array([0.35]), np.array([0.0])
    o = oracle.Oracle(spec, lam)
    o.init_state()
    o.load_state(bin_count=np.array([0, 0, 0, 40, 0, 0, 0, 0, 0, 0], np.int64),
                 bin_sum=np.array([0, 0, 0, 100.0, 0, 0, 0, 0, 0, 0]))
    st = o.run(1)
    bias = 0.4 * (100.0 / 40.0)          # ramp 40/100 times mean 2.5
    assert st["bias"][0] == pytest.approx(bias, abs=1e-15)
    assert st["dudl"][0] == 0.0
    # p after B (h bias) and O with gamma_lambda = 0 (c1 = 1, no noise)
    assert st["p_lambda"][0] == pytest.approx(0.5 * spec.dt * bias, rel=1e-14)


def test_bin_edges():
    spec, lam = synth.lj_reduced()
    o = oracle.Oracle(spec, lam)
    assert o.bin_of(0.0) == 0 and o.bin_of(1.0) == 49 and o.bin_of(0.02) == 1
    assert o.bin_of(0.0199999) == 0 and o.bin_of(0.999) == 49


def test_replay_is_bitwise_deterministic():
    spec, lam = synth.lj_reduced(n_atoms=64, density=0.5, n_walkers=3, lambda0=0.4)
    lam.share_interval = 2
    a = oracle.Oracle(spec, lam)
    a.init_state()
    ra = a.run(30)
    b = oracle.Oracle(spec, lam)
    b.init_state()
    rb = b.run(30)
    for k in ("x", "v", "lam", "p_lambda", "bin_count", "bin_sum", "bin_sum2"):
        assert np.array_equal(ra[k], rb[k]), k
    assert ra["bin_count"].sum() + ra["loc_count"].sum() == 90


# --------------------------------------------------------------------------
# integrator
# --------------------------------------------------------------------------
def test_free_particle_velocity_variance():
    spec, lam = synth.harmonic(n_walkers=16, k0=0.0, k1=0.0)
    spec.gamma = 5.0
    lam.abf_on = False
    lam.fixed_lambda = True
    o = oracle.Oracle(spec, lam)
    o.init_state()
    vs = []
    for _ in range(200):
        o.run(10)
        vs.append(o.full_step()[0].copy())
    v = np.array(vs).ravel()
    assert abs(v.var() - spec.kT) < 0.05


def test_reflection_keeps_momentum_magnitude():
    spec, lam = synth.harmonic(n_walkers=1, k0=2.0, k1=2.0)
    lam.abf_on = False
    lam.gamma_lambda = 0.0
    lam.lambda0 = np.array([0.999])
    lam.p_lambda0 = np.array([3.0])
    lam.m_lambda = 1.0
    o = oracle.Oracle(spec, lam)
    st = o.init_state()
    o.run(1)
    assert st["lam"][0] < 1.0 and st["lam"][0] > 0.98
    assert abs(abs(st["p_lambda"][0]) - 3.0) < 1e-15 and st["p_lambda"][0] < 0


def _nve_cluster(dt):
    rng = np.random.default_rng(11)
    g = np.array([[i, j, k] for i in range(3) for j in range(2) for k in range(2)], float) * 1.12
    pos = g + 20.0 + rng.uniform(-0.03, 0.03, g.shape)
    n = pos.shape[0]
    spec, lam = synth.lj_reduced(n_atoms=n, density=n / 40.0 ** 3, seed=3, r_cut=10.0, r_skin=0.5)
    spec.box[:] = 40.0
    spec.pos = pos
    spec.charge = np.where(np.arange(n) % 2 == 0, 0.3, -0.3)
    spec.vel = rng.normal(0, 0.15, (n, 3))
    spec.gamma = 0.0
    spec.dt = dt
    lam.gamma_lambda = 0.0
    lam.abf_on = False
    lam.m_lambda = 200.0
    lam.lambda0 = np.array([0.5])
    lam.p_lambda0 = np.array([0.5])
    return spec, lam


def _nve_energy_rms(dt, t_total=2.0):
    spec, lam = _nve_cluster(dt)
    o = oracle.Oracle(spec, lam)
    st = o.init_state()
    H = []
    for _ in range(int(round(t_total / dt))):
        o.run(1)
        v, p = o.full_step()
        _, u, _ = o.evaluate(0, st["x"], st["lam"][0])
        H.append(0.5 * (v * v).sum() + p[0] ** 2 / (2 * lam.m_lambda) + u.sum())
        assert 0.3 < st["lam"][0] < 0.7
    H = np.array(H)
    return np.sqrt(np.mean((H - H[0]) ** 2))


def test_nve_energy_error_scales_as_dt_squared():
    e1 = _nve_energy_rms(0.004)
    e2 = _nve_energy_rms(0.002)
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)
    assert e1 < 1e-3


# --------------------------------------------------------------------------
# free energy: lambda-switched harmonic restraints, closed form
# --------------------------------------------------------------------------
@pytest.mark.slow
def test_harmonic_restraint_free_energy_closed_form():
    spec, lam = synth.harmonic(n_walkers=512, seed=909)
    o = oracle.Oracle(spec, lam)
    st = o.init_state()
    o.run(100000)
    cnt = st["bin_count"] + st["loc_count"].sum(0)
    tot = st["bin_sum"] + st["loc_sum"].sum(0)
    g, prof, da, rc = oracle.abf_readout(cnt, tot, 0.0, 1.0)
    assert rc == 0
    exact = 4.5 * spec.kT * math.log(4.0)
    assert abs(exact - 6.2383) < 1e-4
    assert abs(da - exact) < 0.05 * spec.kT, (da, exact)
    # the lambda histogram is flat under the converged bias
    frac = cnt / cnt.sum()
    assert frac.min() > 0.5 / 50 and frac.max() < 1.6 / 50


@pytest.mark.slow
def test_fixed_lambda_ti_harmonic_closed_form():
    """Fixed-lambda TI (lambda frozen at 50 window centres, 16 replicas each):
    the midpoint sum of the window means of dV/dlambda reproduces
    (9/2) kT ln(k1/k0); every sample of a walker lands in its own window."""
    base, lam = synth.harmonic(n_walkers=1, seed=911)
    spec, lamw = synth.ti_windows(base, lam, n_windows=50, replicas=16, seed=912)
    o = oracle.Oracle(spec, lamw)
    st = o.init_state()
    o.run(40000)
    assert np.array_equal(st["lam"], lamw.lambda0)          # frozen
    cnt = st["bin_count"] + st["loc_count"].sum(0)
    tot = st["bin_sum"] + st["loc_sum"].sum(0)
    assert (cnt == 16 * 40000).all()
    g, prof, da, rc = oracle.abf_readout(cnt, tot, 0.0, 1.0)
    assert rc == 0
    exact = 4.5 * spec.kT * math.log(4.0)
    assert abs(da - exact) < 0.05 * spec.kT, (da, exact)
    # window means against the closed form <dV/dlambda> = (9/2)(k1 - k0) kT / k(lambda)
    lc = (np.arange(50) + 0.5) / 50
    want = 4.5 * 3.0 / (1.0 + 3.0 * lc)
    # statistical error of a window mean: dV/dlambda = (3/2) sum of 9 x^2 with
    # var(x^2) = 2 (kT/k)^2 and ~200 independent samples per walker-window
    # (40000 steps of 0.005 over a unit correlation time): sigma ~ 0.11 / k
    sigma = 0.11 / (1.0 + 3.0 * lc)
    assert (np.abs(g - want) < 4.5 * sigma).all(), np.max(np.abs(g - want) / sigma)


# --------------------------------------------------------------------------
# separation-shifted (Zacharias) soft-core variant
# --------------------------------------------------------------------------
def test_shifted_softcore_is_lj_at_the_effective_distance():
    """s = r^2 + delta (1 - c) makes the term c times the plain LJ at distance
    sqrt(s): energy, F/r (times the chain factor) and the shift at r_cut all
    follow from the textbook LJ pinned above."""
    rng = np.random.default_rng(21)
    for _ in range(50):
        r, sig, eps = rng.uniform(0.3, 2.4), rng.uniform(0.8, 1.3), rng.uniform(0.2, 2.0)
        c, delta, rc = rng.uniform(0.0, 1.0), rng.uniform(0.1, 6.0), 2.5
        reff, rceff = math.sqrt(r * r + delta * (1 - c)), math.sqrt(rc * rc + delta * (1 - c))
        z = oracle.pair_terms_shifted(r, sig, eps, 0.0, c, 1.0, delta=delta, r_cut=rc, shift=True)
        lj = oracle.pair_terms(reff, sig, eps, 0.0, 1.0, 1.0)
        ljc = oracle.pair_terms(rceff, sig, eps, 0.0, 1.0, 1.0)
        assert z[0] == pytest.approx(c * (lj[0] - ljc[0]), rel=1e-11, abs=1e-14)
        # -(1/r) dU/dr = c (F/r)_LJ(r_eff), since d r_eff / d r = r / r_eff
        assert z[2] == pytest.approx(c * lj[2], rel=1e-11, abs=1e-14)


def test_shifted_softcore_full_coupling_is_textbook_lj():
    for r in (0.9, 1.12, 1.7, 2.4):
        z = oracle.pair_terms_shifted(r, 1.1, 0.7, 0.0, 1.0, 1.0, delta=3.0, r_cut=2.5, shift=True)
        t = 4 * 0.7 * ((1.1 / r) ** 12 - (1.1 / r) ** 6) - 4 * 0.7 * ((1.1 / 2.5) ** 12 - (1.1 / 2.5) ** 6)
        assert z[0] == pytest.approx(t, rel=1e-12)
    # finite at r = 0 below full coupling
    z0 = oracle.pair_terms_shifted(0.0, 1.0, 1.0, 0.0, 0.5, 1.0, delta=2.0)
    assert z0[0] == pytest.approx(4 * 0.5 * (1.0 / 1.0 ** 6 - 1.0 / 1.0 ** 3), abs=1e-15)


@pytest.mark.parametrize("c", [1.0, 0.7, 0.3, 0.02])
def test_shifted_softcore_pair_fd(c):
    h = 1e-6
    for r in (0.6, 1.0, 1.6, 2.3):
        z = oracle.pair_terms_shifted(r, 1.05, 0.9, 0.0, c, 1.0, delta=0.5, r_cut=2.5, shift=True)
        up = oracle.pair_terms_shifted(r + h, 1.05, 0.9, 0.0, c, 1.0, delta=0.5, r_cut=2.5, shift=True)
        dn = oracle.pair_terms_shifted(r - h, 1.05, 0.9, 0.0, c, 1.0, delta=0.5, r_cut=2.5, shift=True)
        assert z[2] * r == pytest.approx(-(up[0] - dn[0]) / (2 * h), rel=1e-6, abs=1e-9)
        if 0.0 < c < 1.0:
            cp = oracle.pair_terms_shifted(r, 1.05, 0.9, 0.0, c + h, 1.0, delta=0.5, r_cut=2.5, shift=True)
            cm = oracle.pair_terms_shifted(r, 1.05, 0.9, 0.0, c - h, 1.0, delta=0.5, r_cut=2.5, shift=True)
            assert z[1] == pytest.approx((cp[0] - cm[0]) / (2 * h), rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("l", [0.0, 0.3, 0.62, 0.8, 0.97])
def test_shifted_softcore_system_derivatives_match_fd(l):
    """Forces, dV/dlambda and dV/d(eps, sigma, q) of a small charged system
    with the separation-shifted form against central differences."""
    spec, lam = _charged_small(form="shifted")
    o = oracle.Oracle(spec, lam)
    x = spec.pos.copy()
    f, _, g = o.evaluate(0, x, l)
    h = 1e-6
    for i in (0, 1, 2, 40):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = -(_energy(o, xp, l) - _energy(o, xm, l)) / (2 * h)
            assert abs(f[i, k] - fd) < 1e-6 * max(1.0, abs(fd)), (i, k, f[i, k], fd)
    hl = 1e-4
    if l == 0.0:
        fd = (-3 * _energy(o, x, 0) + 4 * _energy(o, x, hl) - _energy(o, x, 2 * hl)) / (2 * hl)
    else:
        fd = (_energy(o, x, l + hl) - _energy(o, x, l - hl)) / (2 * hl)
    assert abs(g - fd) < 1e-7 * max(1.0, abs(g)), (g, fd)
    pg = o.param_grad(0, x, l)
    hp = 1e-5
    for i in (0, 1, 2):
        for k, field in enumerate(["epsilon", "sigma", "charge"]):
            vals = []
            for sgn in (+1, -1):
                sp, _ = _charged_small(form="shifted")
                getattr(sp, field)[i] += sgn * hp
                vals.append(oracle.Oracle(sp, lam).evaluate(0, x, l)[1].sum())
            fd = (vals[0] - vals[1]) / (2 * hp)
            assert abs(pg[i, k] - fd) < 1e-6 * max(1.0, abs(fd)), (i, field, pg[i, k], fd)


# --------------------------------------------------------------------------
# lambda-dependent distance restraint ("Dealing with metastabilities")
# --------------------------------------------------------------------------
def _dr_sys(n=1, delta=2.0, k=5.0, pair=(0, 6)):
    spec, lam = _charged_small()
    lam.dr_pairs = np.array([pair], np.int32)
    lam.dr_delta, lam.dr_k, lam.dr_freq = delta, k, n
    return spec, lam


def _pair_distance(spec, a, b):
    d = spec.pos[b] - spec.pos[a]
    L = spec.box[0]
    d -= L * np.round(d / L)
    return float(np.linalg.norm(d))


def test_dmin_is_zero_at_the_end_states_and_delta_midway():
    """The properties the paper states: d_min(0) = d_min(1) = 0 and
    d_min(0.5) = delta (n = 1); with lambda doubled (n = 2, the SI script)
    the peaks move to 1/4 and 3/4."""
    o1 = oracle.Oracle(*_dr_sys(n=1, delta=20.0))
    assert o1.dmin(0.0)[0] == 0.0 and abs(o1.dmin(1.0)[0]) < 1e-12
    assert o1.dmin(0.5)[0] == pytest.approx(20.0, rel=1e-15)
    o2 = oracle.Oracle(*_dr_sys(n=2, delta=10.0))
    for l, want in [(0.25, 10.0), (0.75, 10.0), (0.5, 0.0), (0.0, 0.0)]:
        assert o2.dmin(l)[0] == pytest.approx(want, abs=1e-12)


def test_distance_restraint_leaves_the_end_states_and_far_pairs_alone():
    spec, lam = _dr_sys(delta=2.0)
    base, lam0 = _charged_small()
    o, o0 = oracle.Oracle(spec, lam), oracle.Oracle(base, lam0)
    for l in (0.0, 1.0):
        f, u, g = o.evaluate(0, spec.pos, l)
        f0, u0, g0 = o0.evaluate(0, spec.pos, l)
        assert np.array_equal(f, f0) and np.array_equal(u, u0) and g == g0
    # midway: acts iff d < delta
    d = _pair_distance(spec, 0, 6)
    f, u, g = o.evaluate(0, spec.pos, 0.5)
    f0, u0, g0 = o0.evaluate(0, spec.pos, 0.5)
    if d < 2.0:
        assert u[4] - u0[4] == pytest.approx(0.5 * 5.0 * (d - 2.0) ** 2, rel=1e-12)
    spec2, lam2 = _dr_sys(delta=0.5 * d)    # d_min(0.5) below d: inert everywhere
    for l in (0.3, 0.5, 0.8):
        f2, u2, g2 = oracle.Oracle(spec2, lam2).evaluate(0, spec.pos, l)
        f0, u0, g0 = o0.evaluate(0, spec.pos, l)
        assert np.array_equal(f2, f0) and g2 == g0


def test_distance_restraint_lambda_force_matches_the_si_expression():
    """With lambda doubled (n = 2) the force on lambda is
    -F_d delta pi sin(2 pi l1) 2 with l1 = 2 lambda and F_d = -k (d - d_min)."""
    spec, lam = _dr_sys(n=2, delta=2.5, k=10.0)
    base, lam0 = _charged_small()
    o, o0 = oracle.Oracle(spec, lam), oracle.Oracle(base, lam0)
    d = _pair_distance(spec, 0, 6)
    hit = 0
    for l in (0.1, 0.2, 0.3, 0.4, 0.6, 0.7):
        l1 = 2.0 * l
        dmin = 2.5 / 2.0 * (1 - math.cos(2 * math.pi * l1))
        g = o.evaluate(0, spec.pos, l)[2] - o0.evaluate(0, spec.pos, l)[2]
        if d < dmin:
            fd = -10.0 * (d - dmin)
            want = -(-fd * 2.5 * math.pi * math.sin(2 * math.pi * l1) * 2.0)   # dV/dlambda
            assert g == pytest.approx(want, rel=1e-12)
            hit += 1
        else:
            assert g == 0.0
    assert hit >= 2


@pytest.mark.parametrize("n", [1, 2])
def test_distance_restraint_derivatives_match_fd(n):
    spec, lam = _dr_sys(n=n, delta=2.5, k=5.0)
    o = oracle.Oracle(spec, lam)
    x = spec.pos.copy()
    for l in (0.2, 0.45, 0.7):
        if o.dmin(l)[0] <= _pair_distance(spec, 0, 6):
            continue
        f, _, g = o.evaluate(0, x, l)
        h = 1e-6
        for i in (0, 6):
            for k in range(3):
                xp, xm = x.copy(), x.copy()
                xp[i, k] += h
                xm[i, k] -= h
                fd = -(_energy(o, xp, l) - _energy(o, xm, l)) / (2 * h)
                assert abs(f[i, k] - fd) < 1e-6 * max(1.0, abs(fd)), (i, k, f[i, k], fd)
        hl = 1e-5
        fd = (_energy(o, x, l + hl) - _energy(o, x, l - hl)) / (2 * hl)
        assert abs(g - fd) < 1e-6 * max(1.0, abs(g)), (l, g, fd)


def test_parallel_evaluation_does_not_depend_on_the_thread_count():
    """Walkers of 2048 atoms or more are evaluated cell column by cell column
    in parallel, each column with its own sums added in column order: one
    thread and eight give bitwise the same forces, energies and dV/dlambda
    (and the per-atom force scale)."""
    import subprocess
    import sys
    code = (
        "import sys, numpy as np; sys.path.insert(0, %r); import oracle; "
        "from paper_2307_08006_amd import synth; "
        "spec, lam = synth.charged_lj(n_atoms=3000, precision='fp64', seed=5, r_cut=8.0); "
        "o = oracle.Oracle(spec, lam); f, u, g = o.evaluate(0, spec.pos, 0.3); "
        "fs = o.force_scale(0, spec.pos, 0.3); "
        "sys.stdout.buffer.write(np.concatenate([f.ravel(), u, [g], fs]).tobytes())"
    ) % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))),)
    out = []
    for nt in ("1", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        out.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                  capture_output=True).stdout)
    assert len(out[0]) > 0 and out[0] == out[1]
