"""GPU parity: the HIP path, called through the C ABI, against the FP64
oracle on identical seeded inputs.

Tolerances (from the arithmetic of each path):
  * neighbour sets: bit-exact (same FP64 decision on identical positions);
  * FP64 systems: forces, energies, dV/dlambda within 1e-10 relative
    (differences only in summation order);
  * FP32 systems: forces ||dF|| / ||F|| <= 1e-5 per walker (FP32 pair terms
    on exact FP32 separations) and, atom by atom, |dF_i| <= 1e-5 s_i with
    s_i the sum of the magnitudes of atom i's force terms (the oracle's force
    scale; robust to cancellation in the net force; 1e-10 in FP64 systems);
    dV/dlambda and every alchemical quantity within 1e-9 relative (computed
    in FP64 on the FP32 positions);
  * short FP64 trajectories with the same noise: lambda, p_lambda, ABF sums
    and positions within 1e-9 relative.
"""
import math

import numpy as np
import pytest

import oracle
from conftest import per_atom_ok
from paper_2307_08006_amd import labf, synth

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _small_charged(precision, n=3000, seed=synth.BASE_SEED + 11, n_solute=30, lj_spread=0.0):
    return synth.charged_lj(n_atoms=n, n_solute=n_solute, precision=precision, seed=seed,
                            lj_spread=lj_spread)


def _mixed(precision):
    """Every solvent atom with its own sigma and epsilon (+-15 %): pairs use
    Lorentz-Berthelot mixing instead of one uniform LJ pair."""
    return _small_charged(precision, lj_spread=0.15)


def _uneven(precision):
    a, lam = _small_charged(precision, n=2600, seed=31)
    b, _ = _small_charged(precision, n=4100, seed=32, n_solute=12)
    c, _ = synth.charged_lj(n_atoms=3300, n_solute=0, precision=precision, seed=33)
    return synth.concat([a, b, c], lam, np.array([0.1, 0.45, 0.8]), seed=34, name="uneven3")


def _shifted(precision):
    """Separation-shifted soft-core (delta = 5 A^2) with the staggered schedule
    of the NAMD setup: electrostatics over [0, 0.5], vdW over [0, 1]."""
    spec, lam = _small_charged(precision)
    lam.sc_form, lam.sc_shift = "shifted", 5.0
    lam.elec_start, lam.elec_end, lam.vdw_start, lam.vdw_end = 0.0, 0.5, 0.0, 1.0
    return spec, lam


def _restrained(precision, freq=1):
    """Distance restraint between the first solute atom and the environment
    atom nearest to 4 A from it (delta = 10 A, k = 5): active at
    intermediate lambda."""
    spec, lam = _small_charged(precision)
    a = int(np.nonzero(spec.is_solute)[0][0])
    d = spec.pos - spec.pos[a]
    d -= spec.box[0] * np.round(d / spec.box[0])
    r = np.linalg.norm(d, axis=1)
    r[spec.is_solute.astype(bool)] = np.inf
    b = int(np.argmin(np.abs(r - 4.0)))
    lam.dr_pairs = np.array([[a, b]], np.int32)
    lam.dr_delta, lam.dr_k, lam.dr_freq = 10.0, 5.0, freq
    return spec, lam


def _pme(precision):
    """Smooth-PME electrostatics (grid spacing <= 1.1 A, order 4,
    erfc(beta r_cut) = 1e-6) with a net-charged group, so that the
    neutralising-background cross term enters dV/dlambda."""
    spec, lam = _small_charged(precision)
    spec = synth.with_pme(spec)
    spec.charge[np.nonzero(spec.is_solute)[0][:3]] += 0.3
    return spec, lam


def _uneven_pme(precision):
    """Three uneven walkers with differently shaped PME grids (order 6)."""
    spec, lam = _uneven(precision)
    return synth.with_pme(spec, dims=[[32, 32, 32], [16, 32, 64], [64, 16, 16]], order=6), lam


def _uneven_pme_mixed(precision):
    """Uneven walkers where one grid's y-z planes exceed the LDS plane limit
    (32 x 128 x 128: transformed line by line) and the others fit (planes)."""
    spec, lam = _uneven(precision)
    return synth.with_pme(spec, dims=[[32, 128, 128], [32, 32, 32], [64, 16, 16]], order=4), lam


def _uneven_pme_235(precision, axes=False):
    """Grids with factors 3 and 5 (24, 40, 48, 80, 96, 120 points): mixed-radix
    transforms, by planes or (axes=True, 96 x 120 planes) line by line, beside
    one walker whose grid lengths are all powers of two (its blocks are
    ordered first and run the radix-2 kernels)."""
    spec, lam = _uneven(precision)
    dims = [[24, 96, 120], [40, 40, 40], [32, 32, 64]] if axes else [[24, 48, 40], [32, 64, 32], [80, 24, 48]]
    return synth.with_pme(spec, dims=dims, order=6), lam


def _pme_everything(precision):
    """PME with the separation-shifted soft-core, the staggered schedule and
    the lambda-dependent distance restraint, all at once."""
    spec, lam = _restrained(precision)
    lam.sc_form, lam.sc_shift = "shifted", 5.0
    lam.elec_start, lam.elec_end, lam.vdw_start, lam.vdw_end = 0.0, 0.5, 0.0, 1.0
    spec = synth.with_pme(spec, order=6)
    spec.charge[np.nonzero(spec.is_solute)[0][:2]] -= 0.25
    return spec, lam


def _pme_axes(precision):
    """A 16 x 128 x 128 grid: y-z planes too large for one LDS block, so the
    transforms run axis by axis."""
    spec, lam = _pme(precision)
    return synth.with_pme(spec, dims=(16, 128, 128), order=4), lam


SYSTEMS = {
    "lj512_fp64": lambda: synth.lj_reduced(),
    "charged3k_fp32": lambda: _small_charged("fp32"),
    "charged3k_fp64": lambda: _small_charged("fp64"),
    "charged3k_fp32_mixedlj": lambda: _mixed("fp32"),
    "charged3k_fp64_mixedlj": lambda: _mixed("fp64"),
    "uneven3_fp32": lambda: _uneven("fp32"),
    "charged3k_fp32_shifted": lambda: _shifted("fp32"),
    "charged3k_fp64_shifted": lambda: _shifted("fp64"),
    "charged3k_fp64_restrained": lambda: _restrained("fp64"),
    "charged3k_fp32_restrained2": lambda: _restrained("fp32", freq=2),
    "charged3k_fp32_pme": lambda: _pme("fp32"),
    "charged3k_fp64_pme": lambda: _pme("fp64"),
    "uneven3_fp32_pme": lambda: _uneven_pme("fp32"),
    "charged3k_fp64_pme_axes": lambda: _pme_axes("fp64"),
    "charged3k_fp32_pme_shifted_restrained": lambda: _pme_everything("fp32"),
    "uneven3_fp64_pme_mixed": lambda: _uneven_pme_mixed("fp64"),
    "uneven3_fp64_pme_235": lambda: _uneven_pme_235("fp64"),
    "uneven3_fp32_pme_235_axes": lambda: _uneven_pme_235("fp32", axes=True),
}


@pytest.fixture(scope="module", params=sorted(SYSTEMS))
def case(request):
    spec, lam = SYSTEMS[request.param]()
    sys_ = labf.System(spec, lam)
    yield request.param, spec, lam, sys_
    sys_.close()


def test_philox_stream_matches_oracle():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, size=(512, 4), dtype=np.uint64).astype(np.uint32)
    key = np.array([0x12345678, 0x9ABCDEF0], np.uint32)
    got = labf.philox(ctr, key)
    for i in range(ctr.shape[0]):
        assert got[i].tolist() == oracle.philox4x32_10(ctr[i], key).tolist()


def test_positions_round_trip(case):
    name, spec, lam, s = case
    pos, _ = s.read_atoms()
    assert np.array_equal(pos, spec.pos), name


def test_neighbour_set_is_bit_exact(case):
    name, spec, lam, s = case
    o = oracle.Oracle(spec, lam)
    pos, _ = s.read_atoms()
    for w in range(spec.n_walkers):
        sl = spec.walker_slice(w)
        got = s.export_pairs(w)
        want = o.neighbor_pairs(w, pos[sl], spec.r_cut + spec.r_skin)
        assert got.shape == want.shape and np.array_equal(got, want), (name, w, got.shape, want.shape)


def test_pair_count_matches_oracle(case):
    name, spec, lam, s = case
    o = oracle.Oracle(spec, lam)
    pos, _ = s.read_atoms()
    got = s.count_pairs()
    for w in range(spec.n_walkers):
        want = o.neighbor_pairs(w, pos[spec.walker_slice(w)], spec.r_cut).shape[0]
        assert got[w] == want, (name, w)


@pytest.mark.parametrize("lam_value", [0.0, 0.3, 0.5, 0.77, 1.0])
def test_forces_energy_dudl_match_oracle(case, lam_value):
    name, spec, lam, s = case
    lam2 = type(lam)(**{**lam.__dict__, "lambda0": np.full(spec.n_walkers, lam_value)})
    s.set_lambda_params(lam2)
    f, e, g = s.compute_forces()
    o = oracle.Oracle(spec, lam2)
    pos, _ = s.read_atoms()
    fp64 = spec.precision == "fp64"
    if name.endswith("mixedlj"):
        assert s.info()["uniform_lj"] == 0, name
    for w in range(spec.n_walkers):
        sl = spec.walker_slice(w)
        fo, uo, go = o.evaluate(w, pos[sl], lam_value)
        ftol = 1e-10 if fp64 else 1e-5
        assert _rel(f[sl], fo) <= ftol, (name, w, _rel(f[sl], fo))
        ok, worst, i = per_atom_ok(f[sl], fo, o.force_scale(w, pos[sl], lam_value), ftol)
        assert ok, (name, w, "per-atom", worst, i)
        assert abs(g[w] - go) <= 1e-9 * max(abs(go), 1e-3), (name, w, g[w], go)
        # alchemical and restraint energies: FP64 on both sides
        for k in (1, 2, 3, 4):
            assert abs(e[w, k] - uo[k]) <= 1e-9 * max(abs(uo[k]), 1e-3), (name, w, k, e[w, k], uo[k])
        etol = 1e-10 if fp64 else 2e-6
        assert abs(e[w, 0] - uo[0]) <= etol * max(abs(uo[0]), 1.0), (name, w, e[w, 0], uo[0])


def _state(s):
    st = s.read_walker_state()
    c, s1, s2 = s.read_abf_bins(True)
    pos, vel = s.read_atoms()
    return st, c, s1, s2, pos, vel


@pytest.mark.parametrize("mode", ["batched", "plain", "fixed_lambda", "pme_batched", "pme_plain",
                                  "pme235_batched"])
def test_short_fp64_trajectory_matches_oracle(mode):
    if mode == "fixed_lambda":
        # fixed-lambda TI windows: lambda frozen at 4 window centres
        base, lam0 = synth.lj_reduced(n_walkers=1)
        spec, lam = synth.ti_windows(base, lam0, n_windows=4, replicas=1, seed=77)
        mode = "batched"
    elif mode.startswith("pme"):
        # charged fluid with Ewald electrostatics on a 16 x 16 x 32 grid, or a
        # 24 x 40 x 16 one (mixed-radix transforms)
        spec, lam = synth.lj_reduced(n_walkers=2, lambda0=0.35, charges=0.5)
        spec = synth.with_pme(spec, dims=(24, 40, 16) if mode.startswith("pme235") else (16, 16, 32))
        mode = mode.split("_", 1)[1]
    else:
        spec, lam = synth.lj_reduced(n_walkers=2, lambda0=0.35)
    lam.share_interval = 2
    s = labf.System(spec, lam)
    o = oracle.Oracle(spec, lam)
    ost = o.init_state()
    for n in (3, 7, 10, 20):
        s.step(n, mode)
        o.run(n)
        st, c, s1, s2, pos, vel = _state(s)
        ref_c = ost["bin_count"] + ost["loc_count"].sum(0)
        ref_s = ost["bin_sum"] + ost["loc_sum"].sum(0)
        assert np.array_equal(c, ref_c)
        assert _rel(s1, ref_s) <= 1e-9
        assert _rel(st["lam"], ost["lam"]) <= 1e-9, (st["lam"], ost["lam"])
        assert _rel(st["p_lambda"], ost["p_lambda"]) <= 1e-9
        assert _rel(st["dudl"], ost["dudl"]) <= 1e-9
        d = pos - ost["x"]
        L = spec.box[0, 0]
        d -= L * np.rint(d / L)
        assert np.abs(d).max() <= 1e-9
        assert _rel(vel, ost["v"]) <= 1e-9
        assert (st["status"] == 0).all()
    s.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_pme_pairs_up_to_the_cutoff_match_oracle(precision):
    """Single charged pairs with Ewald electrostatics from 1 A out to just
    inside r_cut (the last interval of the FP32 real-space table)."""
    import dataclasses
    base, lam = synth.charged_lj(n_atoms=3000, n_solute=0, precision=precision)
    L = 32.0
    for r in (1.0, 4.7, 9.3, 11.99, 11.9995):
        pos = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
        pos, box = synth.quantize(pos, np.array([L, L, L]), precision)
        spec = dataclasses.replace(base, atom_offset=np.array([0, 2]), box=box[None, :], pos=pos,
                                   vel=np.zeros((2, 3)), mass=np.full(2, 20.0),
                                   charge=np.array([0.4, -0.4]), sigma=np.full(2, 2.04),
                                   epsilon=np.zeros(2), is_solute=np.zeros(2, np.uint8),
                                   anchor=None, k0=None, k1=None)
        spec = synth.with_pme(spec)
        s = labf.System(spec, lam)
        f, e, _ = s.compute_forces()
        p, _ = s.read_atoms()
        o = oracle.Oracle(spec, lam)
        fo, uo, _ = o.evaluate(0, p, 0.0)
        s.close()
        ftol = 1e-10 if precision == "fp64" else 1e-6
        assert _rel(f, fo) <= ftol, (r, f, fo)
        assert per_atom_ok(f, fo, o.force_scale(0, p, 0.0), ftol)[0], (r, f, fo)
        assert abs(e[0, 0] - uo[0]) <= ftol * abs(uo[0]), (r, e[0, 0], uo[0])


@pytest.mark.parametrize("pme", [False, True, "mixed", "235"])
def test_batched_and_plain_are_bitwise_identical(pme):
    if pme == "235":
        spec, lam = _uneven_pme_235("fp32", axes=True)
    elif pme:
        spec, lam = _uneven_pme_mixed("fp32") if pme == "mixed" else _uneven_pme("fp32")
    else:
        spec, lam = _uneven("fp32")
    a = labf.System(spec, lam)
    b = labf.System(spec, lam)
    a.step(25, "batched")
    b.step(25, "plain")
    sa, sb = _state(a), _state(b)
    for k in ("lam", "p_lambda", "dudl", "bias"):
        assert np.array_equal(sa[0][k], sb[0][k]), k
    for x, y in zip(sa[1:], sb[1:]):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_repeated_runs_are_bitwise_identical():
    spec, lam = _small_charged("fp32")
    r = []
    for _ in range(2):
        s = labf.System(spec, lam)
        s.step(20)
        r.append(_state(s))
        s.close()
    for x, y in zip(r[0][1:], r[1][1:]):
        assert np.array_equal(x, y)


def test_harmonic_restraint_free_energy_closed_form():
    spec, lam = synth.harmonic(n_walkers=512, seed=909)
    s = labf.System(spec, lam)
    s.step(100000)
    g, prof, da, rc = s.free_energy()
    assert rc == 0
    exact = 4.5 * spec.kT * math.log(4.0)
    assert abs(da - exact) < 0.05 * spec.kT, (da, exact)
    st = s.read_walker_state()
    assert (st["status"] == 0).all()
    s.close()


def test_distance_restraint_energy_at_half_lambda():
    """At lambda = 1/2, d_min = delta: the restraint part of the energy is
    k/2 (d - delta)^2 from the positions read back (the solute carries no
    other restraint)."""
    spec, lam = _restrained("fp64")
    spec.anchor = spec.k0 = spec.k1 = None
    lam.lambda0 = np.array([0.5])
    with labf.System(spec, lam) as s:
        f, e, g = s.compute_forces()
        pos, _ = s.read_atoms()
    a, b = lam.dr_pairs[0]
    d = pos[b] - pos[a]
    d -= spec.box[0] * np.round(d / spec.box[0])
    r = float(np.linalg.norm(d))
    assert r < 10.0
    assert e[0, 4] == pytest.approx(0.5 * 5.0 * (r - 10.0) ** 2, rel=1e-12)
    # forces on the pair include -dV/dx = k (d - delta) (x_b - x_a)/d on a
    o = oracle.Oracle(spec, lam)
    fo, _, _ = o.evaluate(0, pos, 0.5)
    assert _rel(f, fo) <= 1e-10
    assert per_atom_ok(f, fo, o.force_scale(0, pos, 0.5), 1e-10)[0]


def test_fixed_lambda_ti_harmonic_closed_form():
    """Fixed-lambda TI on the GPU: 50 windows x 16 replicas of the 3-particle
    harmonic system, lambda frozen at the window centres; the midpoint sum
    of the window means reproduces (9/2) kT ln(k1/k0) within 0.05 kT."""
    base, lam = synth.harmonic(n_walkers=1, seed=911)
    spec, lamw = synth.ti_windows(base, lam, n_windows=50, replicas=16, seed=912)
    with labf.System(spec, lamw) as s:
        s.step(40000)
        g, prof, da, rc = s.free_energy()
        st = s.read_walker_state()
        cnt, _, _ = s.read_abf_bins()
    assert rc == 0
    assert np.array_equal(st["lam"], lamw.lambda0) and (st["status"] == 0).all()
    assert (cnt == 16 * 40000).all()
    exact = 4.5 * spec.kT * math.log(4.0)
    assert abs(da - exact) < 0.05 * spec.kT, (da, exact)


def test_full_size_single_walker_forces():
    spec, lam = synth.charged_lj(n_atoms=30000, precision="fp32")
    s = labf.System(spec, lam)
    o = oracle.Oracle(spec, lam)
    pos, _ = s.read_atoms()
    for lv in (0.25, 0.75):
        lam2 = type(lam)(**{**lam.__dict__, "lambda0": np.array([lv])})
        s.set_lambda_params(lam2)
        f, e, g = s.compute_forces()
        fo, uo, go = o.evaluate(0, pos, lv)
        assert _rel(f, fo) <= 1e-5, _rel(f, fo)
        ok, worst, i = per_atom_ok(f, fo, o.force_scale(0, pos, lv), 1e-5)
        assert ok, ("per-atom", worst, i)
        assert abs(g[0] - go) <= 1e-9 * abs(go)
    cnt = s.count_pairs()
    assert cnt[0] == o.neighbor_pairs(0, pos, spec.r_cut).shape[0]
    s.close()


def test_full_size_single_walker_pme():
    """The benchmark walker with smooth PME (64^3 grid, order 4): every
    force, dV/dlambda and the energy parts against the oracle."""
    spec, lam = synth.charged_lj(n_atoms=30000, precision="fp32")
    spec = synth.with_pme(spec, spacing=1.1, order=4)
    spec.charge[np.nonzero(spec.is_solute)[0][:3]] += 0.2
    s = labf.System(spec, lam)
    o = oracle.Oracle(spec, lam)
    pos, _ = s.read_atoms()
    for lv in (0.25, 0.75):
        lam2 = type(lam)(**{**lam.__dict__, "lambda0": np.array([lv])})
        s.set_lambda_params(lam2)
        f, e, g = s.compute_forces()
        fo, uo, go = o.evaluate(0, pos, lv)
        assert _rel(f, fo) <= 1e-5, _rel(f, fo)
        ok, worst, i = per_atom_ok(f, fo, o.force_scale(0, pos, lv), 1e-5)
        assert ok, ("per-atom", worst, i)
        assert abs(g[0] - go) <= 1e-9 * max(abs(go), 1e-3), (g[0], go)
        for k in (1, 2, 3, 4):
            assert abs(e[0, k] - uo[k]) <= 1e-9 * max(abs(uo[k]), 1e-3), (k, e[0, k], uo[k])
        assert abs(e[0, 0] - uo[0]) <= 2e-6 * abs(uo[0]), (e[0, 0], uo[0])
    s.close()


def _top2(v):
    v = np.sort(np.asarray(v, float))
    pad = np.concatenate([np.zeros(2), v])
    return pad[-1], pad[-2]


def test_list_validity_check_matches_host_displacements():
    """The rebuild flags a walker (status bit 4) iff its displacements since
    the previous rebuild could have brought an unlisted pair inside r_cut:
    e1 + e2 > r_skin over environment atoms, or a1 + max(e1, a2) > r_skin_alch
    with an alchemical atom.  Walkers get one fast environment atom (walkers
    0-3) or a fast decoupled solute (walkers 4-7) so that both tests fire in
    some walkers and not in others; the expected flags come from the
    positions read back before and after the interval."""
    base, lam = synth.lj_reduced(density=0.3)   # mean free path ~1 sigma
    W, n = 8, base.n_atoms
    spec, lamb = synth.batch(base, lam, W, seed=71)
    rng = np.random.default_rng(72)
    vel = rng.normal(size=(W * n, 3))
    solute = np.nonzero(base.is_solute)[0][0]
    env_atom = (solute + 7) % n
    for w in range(W):
        if w < 4:
            vel[w * n + env_atom] = [2.0 + 2.0 * w, 0.0, 0.0]
        else:
            vel[w * n + solute] = [10.0 + 8.0 * (w - 4), 0.0, 0.0]
    spec.vel = vel
    spec.r_skin, spec.r_skin_alch = 0.5, 1.2
    lamb.lambda0 = np.ones(W)          # solute fully decoupled: it flies freely
    lamb.fixed_lambda = True
    with labf.System(spec, lamb) as s:
        p0, _ = s.read_atoms()
        s.step(spec.rebuild_interval)
        p1, _ = s.read_atoms()
        s.step(1)                      # rebuild: the check runs here
        st = s.read_walker_state()["status"]
    L = spec.box[0]
    d = p1 - p0
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(1)).reshape(W, n)
    alch = base.is_solute.astype(bool)
    want, margin, sums = [], [], []
    for w in range(W):
        e1, e2 = _top2(r[w][~alch])
        a1, a2 = _top2(r[w][alch])
        t_env, t_a = e1 + e2 - spec.r_skin, a1 + max(e1, a2) - spec.r_skin_alch
        want.append(bool(t_env > 0 or t_a > 0))
        margin.append(min(abs(t_env), abs(t_a)))
        sums.append((round(e1 + e2, 4), round(a1 + max(e1, a2), 4)))
    assert min(margin) > 1e-6, margin   # no case decided by rounding
    got = [(int(x) & 4) != 0 for x in st]
    assert got == want, (got, want, sums)
    assert (np.asarray(st) & ~np.uint32(4)).max() == 0
    assert any(want[:4]) and not all(want[:4])
    assert any(want[4:]) and not all(want[4:])


def test_uneven_64_walkers_full_size_sampled():
    """The 64-walker uneven batch (5k-60k atoms per walker, 1.34 M atoms) in
    the launch configuration the benchmark times (autotuned column widths
    from the cache): forces and dV/dlambda of the smallest, the largest and
    two other walkers against the oracle, the pair count of the smallest."""
    from paper_2307_08006_amd import autotune
    spec, lam = synth.uneven(precision="fp32")
    spec.column_width = autotune.cached_widths(spec)
    n = np.diff(spec.atom_offset)
    sample = sorted({int(np.argmin(n)), int(np.argmax(n)), 7, 40})
    with labf.System(spec, lam) as s:
        f, e, g = s.compute_forces()
        pos, _ = s.read_atoms()
        cnt = s.count_pairs()
        st = s.read_walker_state()
    assert (st["status"] & ~np.uint32(4)).max() == 0, st["status"]
    o = oracle.Oracle(spec, lam)
    for w in sample:
        sl = spec.walker_slice(w)
        fo, uo, go = o.evaluate(w, pos[sl], float(lam.lambda0[w]))
        assert _rel(f[sl], fo) <= 1e-5, (w, _rel(f[sl], fo))
        ok, worst, i = per_atom_ok(f[sl], fo, o.force_scale(w, pos[sl], float(lam.lambda0[w])), 1e-5)
        assert ok, (w, "per-atom", worst, i)
        assert abs(g[w] - go) <= 1e-9 * max(abs(go), 1e-12), (w, g[w], go)
    w = int(np.argmin(n))
    sl = spec.walker_slice(w)
    assert cnt[w] == len(o.neighbor_pairs(w, pos[sl], spec.r_cut))
