"""GPU: the error of each result of the mixed-precision path (FP32 pair terms
and FP32 positions on a 2^-23 B grid; FP64 dV/dlambda, lambda, ABF sums)
against the FP64 oracle, on the benchmark workloads, and the effect of the
FP32 position grid on energy conservation.

Each test prints the measured errors; when LABF_PRECISION_REPORT names a
file, the measurements are also written there as JSON (one key per test).
The bounds asserted are the stated tolerances: forces 1e-5 (norm and per
atom against the oracle's force scale), energies 2e-6 relative for the
environment part (FP32 pair terms) and 1e-9 for the parts computed in FP64,
dV/dlambda and ABF samples 1e-9, the free energy 0.05 kT.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2307_08006_amd import labf, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _report(key, value):
    print(key, json.dumps(value, indent=None))
    path = os.environ.get("LABF_PRECISION_REPORT")
    if not path:
        return
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data[key] = value
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


def _force_errors(f, fo, fs):
    d = np.linalg.norm(f - fo, axis=1)
    ratio = d / np.maximum(fs, 1e-300)
    return {"norm_rel": float(np.linalg.norm(f - fo) / np.linalg.norm(fo)),
            "per_atom_max": float(ratio.max()), "per_atom_rms": float(np.sqrt((ratio ** 2).mean()))}


def _rel(a, b, floor=1e-3):
    return float(abs(a - b) / max(abs(b), floor))


def _walker_errors(s, spec, lam, walkers, lam_values=None):
    """Forces, energy parts and dV/dlambda of the given walkers against the
    oracle at each walker's lambda (or at each value of lam_values)."""
    o = oracle.Oracle(spec, lam)
    rows = []
    settings = [None] if lam_values is None else list(lam_values)
    for lv in settings:
        if lv is not None:
            lam2 = type(lam)(**{**lam.__dict__, "lambda0": np.full(spec.n_walkers, lv)})
            s.set_lambda_params(lam2)
        else:
            lam2 = lam
        f, e, g = s.compute_forces()
        pos, _ = s.read_atoms()
        for w in walkers:
            sl = spec.walker_slice(w)
            lw = float(lam2.lambda0[w])
            fo, uo, go = o.evaluate(w, pos[sl], lw)
            fs = o.force_scale(w, pos[sl], lw)
            r = {"walker": int(w), "atoms": int(sl.stop - sl.start), "lambda": lw}
            r.update(_force_errors(f[sl], fo, fs))
            r["energy_rel"] = [_rel(e[w, k], uo[k], 1.0 if k == 0 else 1e-3) for k in range(5)]
            r["dudl_rel"] = _rel(g[w], go)
            rows.append(r)
    return rows


def _check(rows):
    for r in rows:
        assert r["norm_rel"] <= 1e-5 and r["per_atom_max"] <= 1e-5, r
        assert r["energy_rel"][0] <= 2e-6 and max(r["energy_rel"][1:]) <= 1e-9, r
        assert r["dudl_rel"] <= 1e-9, r


def _summary(rows):
    return {"walkers": len(rows),
            "force_norm_rel_max": max(r["norm_rel"] for r in rows),
            "force_per_atom_max": max(r["per_atom_max"] for r in rows),
            "force_per_atom_rms_max": max(r["per_atom_rms"] for r in rows),
            "energy_env_rel_max": max(r["energy_rel"][0] for r in rows),
            "energy_fp64_parts_rel_max": max(max(r["energy_rel"][1:]) for r in rows),
            "dudl_rel_max": max(r["dudl_rel"] for r in rows), "rows": rows}


def test_errors_of_forces_energies_and_dudl():
    """The 30k-atom walker at lambda 0.25, 0.5, 0.75; two walkers of the
    16-walker batch and the smallest and largest walker of the 64-walker
    uneven batch at their own lambda."""
    spec, lam = synth.charged_lj(n_atoms=30000, precision="fp32")
    with labf.System(spec, lam) as s:
        c1 = _walker_errors(s, spec, lam, [0], [0.25, 0.5, 0.75])
    _check(c1)
    base, lam1 = synth.charged_lj(n_atoms=30000, precision="fp32")
    spec2, lam2 = synth.batch(base, lam1, 16, seed=synth.BASE_SEED + 2)
    with labf.System(spec2, lam2) as s:
        c2 = _walker_errors(s, spec2, lam2, [0, 9])
    _check(c2)
    from paper_2307_08006_amd import autotune
    spec3, lam3 = synth.uneven(precision="fp32")
    spec3.column_width = autotune.cached_widths(spec3)
    n = np.diff(spec3.atom_offset)
    with labf.System(spec3, lam3) as s:
        c3 = _walker_errors(s, spec3, lam3, [int(np.argmin(n)), int(np.argmax(n))])
    _check(c3)
    _report("forces_energies_dudl", {"C1_30k": _summary(c1), "C2_16x30k_sample": _summary(c2),
                                     "C3_uneven_sample": _summary(c3)})


def test_errors_of_the_backward_pass():
    """8 x 30k walkers: the position, lambda and solute-parameter gradients
    of two walkers against the oracle's."""
    base, lam = synth.charged_lj(n_atoms=30000, precision="fp32")
    spec, lamb = synth.batch(base, lam, 8, seed=43)
    rows = []
    with labf.System(spec, lamb) as s:
        pos, _ = s.read_atoms()
        dev = torch.device("cuda")
        tp = torch.tensor(pos, device=dev)
        tl = torch.tensor(lamb.lambda0, device=dev)
        tq = torch.tensor(s.solute_params(), device=dev)
        g = torch.ones(8, device=dev, dtype=torch.float64)
        gp, gl, gq = torch.empty_like(tp), torch.empty_like(tl), torch.empty_like(tq)
        s.energy(tp, tl, tq)
        s.energy_backward(g, tp, tl, tq, gp, gl, gq)
        pos, _ = s.read_atoms()
    gp, gl, gq = gp.cpu().numpy(), gl.cpu().numpy(), gq.cpu().numpy()
    o = oracle.Oracle(spec, lamb)
    per = gq.shape[0] // 8
    for w in (0, 5):
        sl = spec.walker_slice(w)
        lw = float(lamb.lambda0[w])
        f, _, dudl = o.evaluate(w, pos[sl], lw)
        pg = o.param_grad(w, pos[sl], lw)[np.asarray(spec.is_solute[sl]).astype(bool)]
        r = {"walker": w, "lambda": lw}
        r.update(_force_errors(-gp[sl], f, o.force_scale(w, pos[sl], lw)))
        r["grad_lambda_rel"] = _rel(gl[w], dudl)
        r["grad_params_rel"] = float(np.linalg.norm(gq[w * per:(w + 1) * per] - pg) / np.linalg.norm(pg))
        rows.append(r)
        assert r["norm_rel"] <= 1e-5 and r["per_atom_max"] <= 1e-5, r
        assert r["grad_lambda_rel"] <= 1e-9 and r["grad_params_rel"] <= 1e-9, r
    _report("backward_8x30k", {"rows": rows})


def test_errors_of_lambda_and_abf_sums_over_a_graph_block():
    """The 30k walker (4 copies at lambda 0.2, 0.4, 0.6, 0.8): one captured
    graph block (rebuild + ten FP32 steps) against the oracle continued from
    the GPU's state.  The first sample of the block is exact to 1e-9 (FP64
    dV/dlambda on identical positions, checked by the stepping tests); the
    later ones inherit the FP32 position rounding, which is what this
    measures: bin sums, lambda, p_lambda and the last dV/dlambda."""
    base, lam = synth.charged_lj(n_atoms=30000, precision="fp32")
    spec, lamb = synth.batch(base, lam, 4, seed=synth.BASE_SEED + 6)
    lamb.lambda0 = np.array([0.2, 0.4, 0.6, 0.8])
    with labf.System(spec, lamb) as s:
        s.step(spec.rebuild_interval)
        st = s.read_walker_state()
        c, s1, s2 = s.read_abf_bins(True)
        pos, vel = s.read_atoms()
        o = oracle.Oracle(spec, lamb)
        o.init_state()
        o.load_state(x=pos, v=vel, lam=st["lam"], p_lambda=st["p_lambda"], bin_count=c, bin_sum=s1,
                     bin_sum2=s2, step=st["step"], pending=1)
        s.step(spec.rebuild_interval)      # one graph block
        o.run(spec.rebuild_interval)
        st2 = s.read_walker_state()
        c2, t1, _ = s.read_abf_bins(True)
    a = o.arr
    ref = a["bin_sum"] + a["loc_sum"].sum(0)
    assert np.array_equal(c2, a["bin_count"] + a["loc_count"].sum(0))
    new = c2 - c
    d_bins = np.abs((t1 - s1) - (ref - s1))[new > 0] / new[new > 0]
    out = {"bin_mean_abs_max": float(d_bins.max()),
           "bin_sum_rel_max": float((np.abs(t1 - ref)[c2 > 0] / np.maximum(np.abs(ref[c2 > 0]), 1e-3)).max()),
           "lambda_abs_max": float(np.abs(st2["lam"] - a["lam"]).max()),
           "p_lambda_abs_max": float(np.abs(st2["p_lambda"] - a["p_lambda"]).max()),
           "dudl_last_rel_max": float(np.max(np.abs(st2["dudl"] - a["dudl"]) /
                                             np.maximum(np.abs(a["dudl"]), 1e-3)))}
    assert out["bin_mean_abs_max"] <= 5e-2 and out["lambda_abs_max"] <= 1e-5, out
    _report("lambda_abf_graph_block_4x30k", out)


def test_free_energy_error_fp32_and_fp64_paths():
    """The 3-particle harmonic system (closed form (9/2) kT ln 4) on both
    paths with the same noise: the FP32 path stores positions in FP32 and
    keeps lambda, dV/dlambda and the bins in FP64; its Delta A differs from
    the FP64 path's only through the position rounding."""
    out = {}
    exact = 4.5 * math.log(4.0)
    for prec in ("fp64", "fp32"):
        spec, lam = synth.harmonic(n_walkers=512, seed=909, precision=prec)
        with labf.System(spec, lam) as s:
            s.step(100000)
            g, prof, da, rc = s.free_energy()
            st = s.read_walker_state()
        assert rc == 0 and (st["status"] == 0).all()
        out[prec] = {"delta_a_kT": da / spec.kT, "error_kT": (da - exact * spec.kT) / spec.kT}
        assert abs(da / spec.kT - exact) < 0.05, out
    out["fp32_minus_fp64_kT"] = out["fp32"]["delta_a_kT"] - out["fp64"]["delta_a_kT"]
    _report("delta_a_harmonic", out)


def _hamiltonian(s, spec):
    """Total energy K + V with full-step velocities (the pending closing
    half-kick applied), and the temperature."""
    f, e, _ = s.compute_forces()
    _, vel = s.read_atoms()
    m = np.asarray(spec.mass)[:, None]
    v = vel + 0.5 * spec.dt * spec.accel_unit * f / m
    ke = 0.5 * float((m * v * v).sum()) / spec.accel_unit
    return ke + float(e.sum()), 2.0 * ke / (3.0 * spec.n_atoms * synth.KB_KCAL)


def test_nve_energy_drift_fp32_vs_fp64():
    """The 30k walker, thermalised (1,000 steps at 1 fs, 20 /ps), then
    1,000 NVE steps at 2 fs (no
    friction, lambda fixed at 0.4, no ABF) in FP32 and in FP64 from the same
    state: the drift and the fluctuation of the total energy, and the mean
    temperature of each.  This measures what the FP32 position grid
    (2^-23 B = 3e-5 A here) does to energy conservation."""
    import dataclasses
    spec, lam = synth.charged_lj(n_atoms=30000, precision="fp32")
    lam.lambda0 = np.array([0.4])
    lam.fixed_lambda, lam.abf_on = True, False
    eq = dataclasses.replace(spec, gamma=20e-3, dt=1.0, rebuild_interval=1)
    with labf.System(eq, lam) as s:
        s.step(1000)
        pos, vel = s.read_atoms()
    # a 1.5 A list buffer: without friction the atoms of the young liquid
    # move farther in ten steps than under the thermostat
    out = {}
    for prec in ("fp64", "fp32"):
        # positions read back from the FP32 system are representable in both
        sp = dataclasses.replace(spec, pos=pos, vel=vel, gamma=0.0, precision=prec, r_skin=1.5)
        hs, ts = [], []
        with labf.System(sp, lam) as s:
            for k in range(21):
                if k:
                    s.step(50)
                h, t = _hamiltonian(s, sp)
                hs.append(h)
                ts.append(t)
            st = s.read_walker_state()
        assert (st["status"] == 0).all(), (prec, st["status"])
        t_ps = np.arange(21) * 50 * spec.dt * 1e-3
        slope = float(np.polyfit(t_ps, hs, 1)[0])
        out[prec] = {"drift_kcal_mol_per_ps": slope,
                     "drift_per_atom_kT_per_ns": slope * 1e3 / (spec.n_atoms * spec.kT),
                     "h_rms_kcal_mol": float(np.std(hs)), "temperature_mean_K": float(np.mean(ts)),
                     "h0_kcal_mol": hs[0]}
        assert np.isfinite(hs).all()
    dt_rel = abs(out["fp32"]["temperature_mean_K"] / out["fp64"]["temperature_mean_K"] - 1.0)
    out["temperature_rel_diff"] = dt_rel
    assert dt_rel < 0.02, out
    _report("nve_30k_fp32_vs_fp64", out)
