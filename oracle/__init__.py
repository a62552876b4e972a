"""FP64 CPU oracle of the lambda-ABF alchemical nonbonded step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg import this package.  The GPU product path never
imports it, and it shares no code with the HIP path: the arithmetic lives in
``labf_oracle.c`` (plain C, FP64, compiled with ``-ffp-contract=off``); this
module only marshals numpy arrays through ctypes.

Functions follow the lambda-ABF paper (Lagardere et al.); each C routine
names the section or equation it implements.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "labf_oracle.c")
_HDR = os.path.join(_HERE, "labf_oracle.h")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liblabf_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain FP64, no fast-math, no contraction)."""
    os.makedirs(_BUILD, exist_ok=True)
    stale = (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(_HDR)))
    if force or stale:
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcSys(C.Structure):
    _fields_ = [
        ("n_walkers", C.c_int32), ("pad0", C.c_int32),
        ("atom_offset", C.c_void_p), ("box", C.c_void_p), ("mass", C.c_void_p),
        ("charge", C.c_void_p), ("sigma", C.c_void_p), ("epsilon", C.c_void_p),
        ("is_solute", C.c_void_p), ("anchor", C.c_void_p), ("k0", C.c_void_p),
        ("k1", C.c_void_p),
        ("r_cut", C.c_double), ("r_skin", C.c_double), ("kT", C.c_double),
        ("gamma", C.c_double), ("dt", C.c_double), ("coulomb_k", C.c_double),
        ("accel_unit", C.c_double), ("seed", C.c_uint64),
        ("m_lambda", C.c_double), ("gamma_lambda", C.c_double), ("kT_lambda", C.c_double),
        ("elec_start", C.c_double), ("elec_end", C.c_double), ("vdw_start", C.c_double),
        ("vdw_end", C.c_double), ("direction", C.c_int32), ("sc_power", C.c_int32),
        ("sc_alpha", C.c_double), ("n_bins", C.c_int32), ("share_interval", C.c_int32),
        ("lam_lo", C.c_double), ("lam_hi", C.c_double), ("full_samples", C.c_int64),
        ("fixed_lambda", C.c_int32), ("abf_on", C.c_int32),
        ("sc_form", C.c_int32), ("pad1", C.c_int32), ("sc_shift", C.c_double),
        ("dr_pairs", C.c_void_p), ("dr_delta", C.c_double), ("dr_k", C.c_double),
        ("dr_freq", C.c_int32), ("pme_on", C.c_int32), ("pme_dims", C.c_void_p),
        ("ewald_beta", C.c_double), ("pme_order", C.c_int32), ("pad3", C.c_int32),
    ]


class OrcState(C.Structure):
    _fields_ = [
        ("x", C.c_void_p), ("v", C.c_void_p), ("f", C.c_void_p), ("lam", C.c_void_p),
        ("p_lambda", C.c_void_p), ("dudl", C.c_void_p), ("bias", C.c_void_p),
        ("bin_count", C.c_void_p), ("bin_sum", C.c_void_p), ("bin_sum2", C.c_void_p),
        ("loc_count", C.c_void_p), ("loc_sum", C.c_void_p), ("loc_sum2", C.c_void_p),
        ("status", C.c_void_p), ("step", C.c_int64), ("pending", C.c_int32), ("pad0", C.c_int32),
    ]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = C.CDLL(build())
            P, I32, I64, D, U32, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint32, C.c_uint64
            L.orc_schedule.argtypes = [P, D, P]
            L.orc_schedule.restype = None
            L.orc_pair_terms.argtypes = [D, D, D, D, D, D, D, I32, D, I32, P]
            L.orc_pair_terms.restype = None
            L.orc_pair_terms_shifted.argtypes = [D, D, D, D, D, D, D, D, I32, P]
            L.orc_pair_terms_shifted.restype = None
            L.orc_dmin.argtypes = [P, D, P]
            L.orc_dmin.restype = None
            L.orc_neighbor_pairs.argtypes = [P, I32, P, D, I32, I64, P]
            L.orc_neighbor_pairs.restype = I64
            L.orc_evaluate.argtypes = [P, I32, P, D, I32, P, P, P]
            L.orc_evaluate.restype = I32
            L.orc_param_grad.argtypes = [P, I32, P, D, P]
            L.orc_param_grad.restype = I32
            L.orc_force_scale.argtypes = [P, I32, P, D, P]
            L.orc_force_scale.restype = I32
            L.orc_abf_bias.argtypes = [P, P, I32, D]
            L.orc_abf_bias.restype = D
            L.orc_philox4x32_10.argtypes = [P, P, P]
            L.orc_philox4x32_10.restype = None
            L.orc_normals.argtypes = [U64, U32, U32, U32, U32, P]
            L.orc_normals.restype = None
            L.orc_init_velocities.argtypes = [P, P]
            L.orc_init_velocities.restype = I32
            L.orc_run.argtypes = [P, P, I64, I32]
            L.orc_run.restype = I32
            L.orc_full_step.argtypes = [P, P, P, P]
            L.orc_full_step.restype = I32
            L.orc_abf_readout.argtypes = [I32, D, D, P, P, P, P, P]
            L.orc_abf_readout.restype = I32
            L.orc_bin_of.argtypes = [P, D]
            L.orc_bin_of.restype = I32
            L.orc_ewald_exact.argtypes = [I64, P, P, P, D, D, I32, D, P]
            L.orc_ewald_exact.restype = D
            L.orc_spme_energy.argtypes = [I64, P, P, P, D, P, I32, D, P]
            L.orc_spme_energy.restype = D
            _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """Holds an orc_sys built from a SystemSpec + LambdaSpec and, once
    ``init_state`` is called, a full dynamic state."""

    def __init__(self, spec, lam):
        self.spec, self.lam = spec, lam
        self._keep = dict(
            atom_offset=np.ascontiguousarray(spec.atom_offset, np.int64),
            box=_f64(spec.box, (-1, 3)), mass=_f64(spec.mass), charge=_f64(spec.charge),
            sigma=_f64(spec.sigma), epsilon=_f64(spec.epsilon),
            is_solute=np.ascontiguousarray(spec.is_solute, np.uint8),
            anchor=_f64(spec.anchor, (-1, 3)), k0=_f64(spec.k0), k1=_f64(spec.k1))
        k = self._keep
        s = OrcSys()
        s.n_walkers = spec.n_walkers
        for f in ("atom_offset", "box", "mass", "charge", "sigma", "epsilon", "is_solute",
                  "anchor", "k0", "k1"):
            setattr(s, f, _p(k[f]))
        for f in ("r_cut", "r_skin", "kT", "gamma", "dt", "coulomb_k", "accel_unit"):
            setattr(s, f, float(getattr(spec, f)))
        s.seed = int(spec.seed) & 0xFFFFFFFFFFFFFFFF
        s.m_lambda, s.gamma_lambda, s.kT_lambda = lam.m_lambda, lam.gamma_lambda, lam.kT_lambda
        s.elec_start, s.elec_end = lam.elec_start, lam.elec_end
        s.vdw_start, s.vdw_end = lam.vdw_start, lam.vdw_end
        s.direction = 1 if lam.direction == "couple" else 0
        s.sc_alpha, s.sc_power = lam.sc_alpha, lam.sc_power
        s.n_bins, s.lam_lo, s.lam_hi = lam.n_bins, lam.lo, lam.hi
        s.full_samples, s.share_interval = lam.full_samples, lam.share_interval
        s.fixed_lambda, s.abf_on = int(lam.fixed_lambda), int(lam.abf_on)
        s.sc_form = 1 if lam.sc_form == "shifted" else 0
        s.sc_shift = float(lam.sc_shift)
        if lam.dr_pairs is not None:
            self._dr = np.ascontiguousarray(lam.dr_pairs, np.int32).reshape(-1, 2)
            s.dr_pairs = self._dr.ctypes.data
            s.dr_delta, s.dr_k, s.dr_freq = float(lam.dr_delta), float(lam.dr_k), int(lam.dr_freq)
        if getattr(spec, "pme_dims", None) is not None:
            self._pme = np.ascontiguousarray(spec.pme_dims, np.int32).reshape(-1, 3)
            s.pme_on, s.pme_dims = 1, self._pme.ctypes.data
            s.ewald_beta, s.pme_order = float(spec.ewald_beta), int(spec.pme_order)
        self.sys = s
        self.st = None

    # -- pure functions -------------------------------------------------------
    def schedule(self, lam: float):
        out = np.zeros(4)
        lib().orc_schedule(C.byref(self.sys), float(lam), _p(out))
        return out

    def neighbor_pairs(self, w: int, x, r_list: float, brute: bool = False) -> np.ndarray:
        x = _f64(x, (-1, 3))
        n = lib().orc_neighbor_pairs(C.byref(self.sys), w, _p(x), r_list, int(brute), 0, None)
        if n < 0:
            raise ValueError("invalid neighbour request")
        out = np.zeros((max(n, 1), 2), np.int64)
        n2 = lib().orc_neighbor_pairs(C.byref(self.sys), w, _p(x), r_list, int(brute), n, _p(out))
        assert n2 == n
        return out[:n]

    def evaluate(self, w: int, x, lam: float, brute: bool = False):
        """(forces [n,3], energy parts [5], dU/dlambda) of walker w."""
        x = _f64(x, (-1, 3))
        f = np.zeros_like(x)
        u = np.zeros(5)
        g = np.zeros(1)
        rc = lib().orc_evaluate(C.byref(self.sys), w, _p(x), float(lam), int(brute), _p(f), _p(u), _p(g))
        if rc != 0:
            raise ValueError("invalid evaluation request")
        return f, u, float(g[0])

    def param_grad(self, w: int, x, lam: float) -> np.ndarray:
        x = _f64(x, (-1, 3))
        g = np.zeros_like(x)
        rc = lib().orc_param_grad(C.byref(self.sys), w, _p(x), float(lam), _p(g))
        if rc != 0:
            raise ValueError("invalid evaluation request")
        return g

    def force_scale(self, w: int, x, lam: float) -> np.ndarray:
        """Per atom of walker w, the sum of the magnitudes of its force terms
        (|f_ij| over pairs within r_cut, the reciprocal-space and restraint
        forces): the scale against which per-atom force errors are judged."""
        x = _f64(x, (-1, 3))
        fs = np.zeros(x.shape[0])
        rc = lib().orc_force_scale(C.byref(self.sys), w, _p(x), float(lam), _p(fs))
        if rc != 0:
            raise ValueError("invalid evaluation request")
        return fs

    def abf_bias(self, w: int, lam: float) -> float:
        """ABF bias force on lambda that walker w sees at lambda in the
        current state (shared bins plus its own unshared samples)."""
        if self.st is None:
            raise RuntimeError("init_state first")
        return float(lib().orc_abf_bias(C.byref(self.sys), C.byref(self.st), int(w), float(lam)))

    def load_state(self, x=None, v=None, lam=None, p_lambda=None, bin_count=None, bin_sum=None,
                   bin_sum2=None, loc_count=None, loc_sum=None, loc_sum2=None, step=None,
                   pending=None):
        """Overwrite parts of the dynamic state (after init_state), e.g. to
        continue from a state read back from elsewhere."""
        if self.st is None:
            self.init_state()
        a = self.arr
        for k, val in (("x", x), ("v", v), ("lam", lam), ("p_lambda", p_lambda),
                       ("bin_count", bin_count), ("bin_sum", bin_sum), ("bin_sum2", bin_sum2),
                       ("loc_count", loc_count), ("loc_sum", loc_sum), ("loc_sum2", loc_sum2)):
            if val is not None:
                a[k][...] = np.asarray(val).reshape(a[k].shape)
        if step is not None:
            self.st.step = int(step)
        if pending is not None:
            self.st.pending = int(pending)
        return a

    def dmin(self, lam: float):
        """(d_min(lambda), d d_min / d lambda) of the distance restraint."""
        out = np.zeros(2)
        lib().orc_dmin(C.byref(self.sys), float(lam), _p(out))
        return out

    def bin_of(self, lam: float) -> int:
        return int(lib().orc_bin_of(C.byref(self.sys), float(lam)))

    # -- dynamics -------------------------------------------------------------
    def init_state(self):
        spec, lam = self.spec, self.lam
        W, N, B = spec.n_walkers, spec.n_atoms, lam.n_bins
        a = dict(x=_f64(spec.pos, (-1, 3)).copy(), v=np.zeros((N, 3)), f=np.zeros((N, 3)),
                 lam=np.array(lam.lambda0, np.float64).copy(), p_lambda=np.zeros(W),
                 dudl=np.zeros(W), bias=np.zeros(W), bin_count=np.zeros(B, np.int64),
                 bin_sum=np.zeros(B), bin_sum2=np.zeros(B), loc_count=np.zeros((W, B), np.int64),
                 loc_sum=np.zeros((W, B)), loc_sum2=np.zeros((W, B)),
                 status=np.zeros(W, np.uint32))
        st = OrcState()
        for k, v in a.items():
            setattr(st, k, _p(v))
        st.step, st.pending = 0, 0
        self.st, self.arr = st, a
        lib().orc_init_velocities(C.byref(self.sys), C.byref(st))
        if spec.vel is not None:
            a["v"][:] = _f64(spec.vel, (-1, 3))
        if lam.p_lambda0 is not None:
            a["p_lambda"][:] = np.asarray(lam.p_lambda0, np.float64)
        return a

    def run(self, n_steps: int, brute: bool = False):
        rc = lib().orc_run(C.byref(self.sys), C.byref(self.st), int(n_steps), int(brute))
        if rc != 0:
            raise RuntimeError("oracle run failed")
        return self.arr

    @property
    def step(self) -> int:
        return int(self.st.step)

    @property
    def pending(self) -> int:
        return int(self.st.pending)

    def full_step(self):
        """Full-step atom velocities and lambda momenta of the current state."""
        v = np.zeros_like(self.arr["v"])
        p = np.zeros_like(self.arr["p_lambda"])
        rc = lib().orc_full_step(C.byref(self.sys), C.byref(self.st), _p(v), _p(p))
        if rc != 0:
            raise RuntimeError("oracle full_step failed")
        return v, p


def pair_terms(r, sig, eps, qq, cv, ce, alpha=0.5, p=1, r_cut=1e300, shift=False):
    """Single-pair terms: (U_LJ, dU_LJ/dc_v, (F/r)_LJ, U_C, dU_C/dc_e, (F/r)_C)."""
    out = np.zeros(6)
    lib().orc_pair_terms(float(r), float(sig), float(eps), float(qq), float(cv), float(ce),
                         float(alpha), int(p), float(r_cut), int(shift), _p(out))
    return out


def pair_terms_shifted(r, sig, eps, qq, cv, ce, delta=5.0, r_cut=1e300, shift=False):
    """Single-pair terms with the separation-shifted soft-core."""
    out = np.zeros(6)
    lib().orc_pair_terms_shifted(float(r), float(sig), float(eps), float(qq), float(cv), float(ce),
                                 float(delta), float(r_cut), int(shift), _p(out))
    return out


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def normals(seed, atom, step, walker, purpose):
    o = np.zeros(4)
    lib().orc_normals(int(seed) & 0xFFFFFFFFFFFFFFFF, atom & 0xFFFFFFFF, step & 0xFFFFFFFF,
                      walker & 0xFFFFFFFF, purpose & 0xFFFFFFFF, _p(o))
    return o


def abf_readout(count, total, lo, hi):
    """(bin gradients, A at bin left edges, Delta A, status)."""
    count = np.ascontiguousarray(count, np.int64)
    total = np.ascontiguousarray(total, np.float64)
    n = count.shape[0]
    g, prof, da = np.zeros(n), np.zeros(n), np.zeros(1)
    rc = lib().orc_abf_readout(n, float(lo), float(hi), _p(count), _p(total), _p(g), _p(prof), _p(da))
    return g, prof, float(da[0]), int(rc)


def ewald_exact(x, q, box, beta, r_real, kmax, coulomb_k=1.0):
    """Plain Ewald sum (real-space images within r_real, |m_a| <= kmax,
    self and neutralising-background terms): (energy, forces)."""
    x = _f64(x, (-1, 3))
    q = _f64(q)
    L = _f64(box)
    f = np.zeros_like(x)
    e = lib().orc_ewald_exact(x.shape[0], _p(x), _p(q), _p(L), float(beta), float(r_real), int(kmax),
                              float(coulomb_k), _p(f))
    return float(e), f


def spme_energy(x, q, box, beta, dims, order=4, coulomb_k=1.0):
    """Smooth-PME reciprocal energy and forces of one charge set (no self
    or background term)."""
    x = _f64(x, (-1, 3))
    q = _f64(q)
    L = _f64(box)
    K = np.ascontiguousarray(dims, np.int32)
    f = np.zeros_like(x)
    e = lib().orc_spme_energy(x.shape[0], _p(x), _p(q), _p(L), float(beta), _p(K), int(order),
                              float(coulomb_k), _p(f))
    return float(e), f
