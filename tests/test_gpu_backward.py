"""GPU: the differentiable energy and its backward kernels
(labf_energy_forward, labf_energy_backward and the torch.autograd.Function
over them) against the FP64 oracle and against central finite differences.

Tolerances:
  * energies: FP64 systems 1e-10 relative; FP32 systems 2e-6 relative
    (FP32 environment pair terms; alchemical parts are FP64);
  * grad_pos = -g F: FP64 1e-10, FP32 1e-5 (norm-wise, as the forces, and
    atom by atom relative to |g| times the oracle's per-atom force scale);
  * grad_lambda and grad_params: 1e-9 relative (FP64 on the stored
    positions, in FP32 systems too);
  * central differences (h = 1e-4): 1e-6 relative for lambda and the solute
    parameters (FP32 systems too: the environment-only terms cancel
    exactly), 1e-6 of the gradient norm for positions (FP64 systems).
"""
import time

import numpy as np
import pytest

import oracle
from paper_2307_08006_amd import labf, synth
from conftest import per_atom_ok

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _charged(precision, n=3000, seed=synth.BASE_SEED + 11):
    return synth.charged_lj(n_atoms=n, precision=precision, seed=seed)


def _shifted(spec, lam):
    lam.sc_form, lam.sc_shift = "shifted", 5.0
    lam.elec_start, lam.elec_end, lam.vdw_start, lam.vdw_end = 0.0, 0.5, 0.0, 1.0
    return spec, lam


def _restrained(spec, lam):
    a = int(np.nonzero(spec.is_solute)[0][0])
    d = spec.pos - spec.pos[a]
    d -= spec.box[0] * np.round(d / spec.box[0])
    r = np.linalg.norm(d, axis=1)
    r[spec.is_solute.astype(bool)] = np.inf
    b = int(np.argmin(np.abs(r - 4.0)))
    lam.dr_pairs = np.array([[a, b]], np.int32)
    lam.dr_delta, lam.dr_k, lam.dr_freq = 10.0, 5.0, 1
    return spec, lam


def _pme(spec, lam):
    spec = synth.with_pme(spec)
    spec.charge[np.nonzero(spec.is_solute)[0][:3]] += 0.3
    return spec, lam


CASES = {
    "lj512_fp64": lambda: synth.lj_reduced(),
    "charged3k_fp64": lambda: _charged("fp64"),
    "charged3k_fp32": lambda: _charged("fp32"),
    "charged3k_fp32_mixedlj": lambda: synth.charged_lj(n_atoms=3000, precision="fp32",
                                                       seed=synth.BASE_SEED + 11, lj_spread=0.15),
    "charged3k_fp64_mixedlj": lambda: synth.charged_lj(n_atoms=3000, precision="fp64",
                                                       seed=synth.BASE_SEED + 11, lj_spread=0.15),
    "charged3k_fp64_shifted": lambda: _shifted(*_charged("fp64")),
    "charged3k_fp64_restrained": lambda: _restrained(*_charged("fp64")),
    "charged3k_fp64_pme": lambda: _pme(*_charged("fp64")),
    "charged3k_fp32_pme": lambda: _pme(*_charged("fp32")),
}
LAMS = [0.35, 0.75]   # inside the electrostatics and the soft-core vdW ramps


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    base, lam = CASES[request.param]()
    spec, lamb = synth.batch(base, lam, 2, seed=41)
    lamb.lambda0 = np.array(LAMS)
    s = labf.System(spec, lamb)
    pos, _ = s.read_atoms()
    dev = torch.device("cuda")
    t = dict(pos=torch.tensor(pos, device=dev), lam=torch.tensor(LAMS, device=dev, dtype=torch.float64),
             par=torch.tensor(s.solute_params(), device=dev))
    yield request.param, spec, lamb, s, t
    s.close()


def _oracle(spec, lamb, s, t):
    """Oracle evaluation at the positions the library holds (read back)."""
    pos, _ = s.read_atoms()
    o = oracle.Oracle(spec, lamb)
    out = []
    for w in range(spec.n_walkers):
        sl = spec.walker_slice(w)
        lw = float(t["lam"][w])
        f, u, g = o.evaluate(w, pos[sl], lw)
        pg = o.param_grad(w, pos[sl], lw)
        out.append((f, float(np.sum(u)), float(g), pg[np.asarray(spec.is_solute[sl]).astype(bool)],
                    o.force_scale(w, pos[sl], lw)))
    return out


def test_energy_matches_oracle(case):
    name, spec, lamb, s, t = case
    g = torch.empty_like(t["lam"])
    e = s.energy(t["pos"], t["lam"], t["par"], dudl=g).cpu().numpy()
    g = g.cpu().numpy()
    ref = _oracle(spec, lamb, s, t)
    tol = 1e-10 if spec.precision == "fp64" else 2e-6
    for w in range(spec.n_walkers):
        assert abs(e[w] - ref[w][1]) <= tol * abs(ref[w][1]), (name, w, e[w], ref[w][1])
        assert abs(g[w] - ref[w][2]) <= 1e-9 * max(abs(ref[w][2]), 1e-3), (name, w, g[w], ref[w][2])


def test_backward_matches_oracle(case):
    name, spec, lamb, s, t = case
    g = torch.tensor([0.7, -1.3], device="cuda", dtype=torch.float64)
    gp = torch.empty_like(t["pos"])
    gl = torch.empty_like(t["lam"])
    gq = torch.empty_like(t["par"])
    s.energy_backward(g, t["pos"], t["lam"], t["par"], gp, gl, gq)
    gp, gl, gq = gp.cpu().numpy(), gl.cpu().numpy(), gq.cpu().numpy()
    ref = _oracle(spec, lamb, s, t)
    ftol = 1e-10 if spec.precision == "fp64" else 1e-5
    nsol = 0
    for w in range(spec.n_walkers):
        gw = float(g[w])
        f, _, dudl, pg, fs = ref[w]
        sl = spec.walker_slice(w)
        assert _rel(gp[sl], -gw * f) <= ftol, (name, w, _rel(gp[sl], -gw * f))
        ok, worst, i = per_atom_ok(gp[sl], -gw * f, abs(gw) * fs, ftol)
        assert ok, (name, w, "per-atom", worst, i)
        assert abs(gl[w] - gw * dudl) <= 1e-9 * abs(gw * dudl), (name, w, gl[w], gw * dudl)
        k = pg.shape[0]
        assert _rel(gq[nsol:nsol + k], gw * pg) <= 1e-9, (name, w, gq[nsol:nsol + k], gw * pg)
        nsol += k
    assert nsol == gq.shape[0]


def _energy(s, t, **over):
    a = dict(t)
    a.update(over)
    return s.energy(a["pos"], a["lam"], a["par"]).cpu().numpy()


def test_lambda_and_parameter_gradients_match_central_differences(case):
    name, spec, lamb, s, t = case
    h = 1e-4
    g = torch.ones(2, device="cuda", dtype=torch.float64)
    gl = torch.empty_like(t["lam"])
    gq = torch.empty_like(t["par"])
    s.energy_backward(g, t["pos"], t["lam"], t["par"], None, gl, gq)
    gl, gq = gl.cpu().numpy(), gq.cpu().numpy()
    for w in range(2):
        dl = torch.zeros(2, device="cuda", dtype=torch.float64)
        dl[w] = h
        fd = (_energy(s, t, lam=t["lam"] + dl)[w] - _energy(s, t, lam=t["lam"] - dl)[w]) / (2 * h)
        assert abs(fd - gl[w]) <= 1e-6 * max(abs(gl[w]), 1.0), (name, w, fd, gl[w])
    # first two solute atoms of each walker, all three parameters
    per = gq.shape[0] // 2
    for i in sorted({0, min(1, per - 1), per, per + min(1, per - 1)}):
        w = 0 if i < per else 1
        for q in range(3):
            if q == 1 and float(t["par"][i, 0]) == 0.0:
                continue  # sigma is inert without epsilon
            dp = torch.zeros_like(t["par"])
            dp[i, q] = h
            fd = (_energy(s, t, par=t["par"] + dp)[w] - _energy(s, t, par=t["par"] - dp)[w]) / (2 * h)
            assert abs(fd - gq[i, q]) <= 1e-6 * max(abs(gq[i, q]), 1.0), (name, i, q, fd, gq[i, q])


def test_position_gradient_matches_central_differences(case):
    name, spec, lamb, s, t = case
    if spec.precision != "fp64":
        pytest.skip("FP32 positions are stored on a 1.5e-5 A grid; checked against the oracle instead")
    h = 1e-4
    g = torch.ones(2, device="cuda", dtype=torch.float64)
    gp = torch.empty_like(t["pos"])
    s.energy_backward(g, t["pos"], t["lam"], t["par"], gp, None, None)
    gp = gp.cpu().numpy()
    sol = np.nonzero(spec.is_solute)[0]
    n = spec.walker_slice(0).stop
    atoms = [int(sol[0]), int(sol[-1]), 5, n + 17]
    scale = np.abs(gp).max()
    for a in atoms:
        w = 0 if a < n else 1
        for k in range(3):
            dp = torch.zeros_like(t["pos"])
            dp[a, k] = h
            fd = (_energy(s, t, pos=t["pos"] + dp)[w] - _energy(s, t, pos=t["pos"] - dp)[w]) / (2 * h)
            assert abs(fd - gp[a, k]) <= 1e-6 * scale, (name, a, k, fd, gp[a, k])


def test_autograd_function_matches_direct_backward(case):
    from paper_2307_08006_amd.autograd import energy
    name, spec, lamb, s, t = case
    pos = t["pos"].clone().requires_grad_(True)
    lam = t["lam"].clone().requires_grad_(True)
    par = t["par"].clone().requires_grad_(True)
    e = energy(s, pos, lam, par)
    wts = torch.tensor([2.0, -0.5], device="cuda", dtype=torch.float64)
    (e * wts).sum().backward()
    gp = torch.empty_like(t["pos"])
    gl = torch.empty_like(t["lam"])
    gq = torch.empty_like(t["par"])
    s.energy_backward(wts, t["pos"], t["lam"], t["par"], gp, gl, gq)
    assert torch.equal(pos.grad, gp) and torch.equal(lam.grad, gl) and torch.equal(par.grad, gq)
    # only the requested gradients are computed
    lam2 = t["lam"].clone().requires_grad_(True)
    (gl2,) = torch.autograd.grad(energy(s, t["pos"], lam2, t["par"]).sum(), [lam2])
    assert torch.allclose(gl2, gl / wts, rtol=1e-12, atol=0)


def test_invalid_solute_parameters_are_rejected(case):
    name, spec, lamb, s, t = case
    bad = t["par"].clone()
    bad[0, 0] = -1.0
    with pytest.raises(labf.LabfError) as ei:
        s.energy(t["pos"], t["lam"], bad)
    assert ei.value.code == -1
    e = s.energy(t["pos"], t["lam"], t["par"])      # still usable
    assert torch.isfinite(e).all()


def test_full_size_backward_8x30k():
    """Eight 30k-atom FP32 walkers (lambda ~ U(0,1)): forward and backward at
    full size; dV/dlambda and the solute parameter gradients of every walker
    and the position gradient of walker 0 against the oracle."""
    base, lam = synth.charged_lj(n_atoms=30000, precision="fp32")
    spec, lamb = synth.batch(base, lam, 8, seed=43)
    with labf.System(spec, lamb) as s:
        pos, _ = s.read_atoms()
        dev = torch.device("cuda")
        tp = torch.tensor(pos, device=dev)
        tl = torch.tensor(lamb.lambda0, device=dev)
        tq = torch.tensor(s.solute_params(), device=dev)
        g = torch.linspace(0.5, 2.0, 8, device=dev, dtype=torch.float64)
        gp, gl, gq = torch.empty_like(tp), torch.empty_like(tl), torch.empty_like(tq)
        s.energy(tp, tl, tq)
        s.energy_backward(g, tp, tl, tq, gp, gl, gq)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            s.energy(tp, tl, tq)
            s.energy_backward(g, tp, tl, tq, gp, gl, gq)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 5 * 1e3
        print(f"forward + backward, 8 x 30k atoms: {ms:.2f} ms")
        # a forward at new positions, then a backward on the same tensors
        # (which reuses the forward's lists) give the same gradients
        tp2 = tp.clone()
        s.energy(tp2, tl, tq)
        gp2 = torch.empty_like(tp)
        s.energy_backward(g, tp2, tl, tq, gp2, None, None)
        assert torch.equal(gp2, gp)
        pos, _ = s.read_atoms()
    gp, gl, gq = gp.cpu().numpy(), gl.cpu().numpy(), gq.cpu().numpy()
    o = oracle.Oracle(spec, lamb)
    nsol = 0
    for w in range(8):
        sl = spec.walker_slice(w)
        lw = float(lamb.lambda0[w])
        gw = float(g[w])
        if w == 0:
            f, _, dudl = o.evaluate(w, pos[sl], lw)
            assert _rel(gp[sl], -gw * f) <= 1e-5
            ok, worst, i = per_atom_ok(gp[sl], -gw * f, abs(gw) * o.force_scale(w, pos[sl], lw), 1e-5)
            assert ok, ("per-atom", worst, i)
        else:
            _, _, dudl = o.evaluate(w, pos[sl], lw)
        assert abs(gl[w] - gw * dudl) <= 1e-9 * max(abs(gw * dudl), 1e-12), (w, gl[w], gw * dudl)
        pg = o.param_grad(w, pos[sl], lw)[np.asarray(spec.is_solute[sl]).astype(bool)]
        assert _rel(gq[nsol:nsol + pg.shape[0]], gw * pg) <= 1e-9, w
        nsol += pg.shape[0]
