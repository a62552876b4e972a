"""Python binding of the lambda-ABF C ABI (include/labf.h).

Argument marshalling only: every step of the method runs in the gfx950 HIP
library ``_build/liblabf.so``.  There is no CPU fallback; if the library is
missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from .synth import LambdaSpec, SystemSpec

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "liblabf.so")

LABF_FP32, LABF_FP64 = 0, 1
LABF_DECOUPLE, LABF_COUPLE = 0, 1
MODE_BATCHED, MODE_PLAIN = 0, 1
WS_NONFINITE, WS_REFLECT, WS_SKIN, WS_CAPACITY = 1, 2, 4, 8
STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_STATE", -3: "E_HIP", -4: "E_NONFINITE",
                -5: "E_SKIN", -6: "E_UNSUPPORTED", -7: "E_EMPTY_BIN", -8: "E_CAPACITY"}

# every symbol include/labf.h declares
EXPORTS = ["labf_workspace_size", "labf_create_system", "labf_set_lambda_params", "labf_step_walkers",
           "labf_read_abf_bins", "labf_free_energy", "labf_read_walker_state",
           "labf_read_atoms", "labf_write_atoms", "labf_compute_forces", "labf_export_pairs",
           "labf_export_pairs_noalloc",
           "labf_count_pairs", "labf_profile_steps", "labf_philox", "labf_get_info",
           "labf_energy_forward", "labf_energy_backward", "labf_set_distance_restraint",
           "labf_probe", "labf_destroy_system",
           "labf_last_error"]


class LabfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class SystemDesc(C.Structure):
    _fields_ = [
        ("n_walkers", C.c_int32), ("precision", C.c_int32),
        ("atom_offset", C.c_void_p), ("box", C.c_void_p), ("pos", C.c_void_p),
        ("vel", C.c_void_p), ("mass", C.c_void_p), ("charge", C.c_void_p),
        ("sigma", C.c_void_p), ("epsilon", C.c_void_p), ("is_solute", C.c_void_p),
        ("anchor", C.c_void_p), ("k0", C.c_void_p), ("k1", C.c_void_p),
        ("r_cut", C.c_double), ("r_skin", C.c_double), ("kT", C.c_double),
        ("gamma", C.c_double), ("dt", C.c_double), ("coulomb_k", C.c_double),
        ("accel_unit", C.c_double), ("seed", C.c_uint64),
        ("rebuild_interval", C.c_int32), ("pme_order", C.c_int32),
        ("r_skin_alch", C.c_double), ("column_width", C.c_void_p),
        ("pme_dims", C.c_void_p), ("ewald_beta", C.c_double),
        ("max_bins", C.c_int32), ("list_capacity", C.c_int32),
        ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
        ("prune_buffer", C.c_void_p),
    ]


class LambdaParams(C.Structure):
    _fields_ = [
        ("lambda0", C.c_void_p), ("p_lambda0", C.c_void_p),
        ("m_lambda", C.c_double), ("gamma_lambda", C.c_double), ("kT_lambda", C.c_double),
        ("elec_start", C.c_double), ("elec_end", C.c_double),
        ("vdw_start", C.c_double), ("vdw_end", C.c_double),
        ("direction", C.c_int32), ("sc_power", C.c_int32), ("sc_alpha", C.c_double),
        ("n_bins", C.c_int32), ("share_interval", C.c_int32),
        ("lo", C.c_double), ("hi", C.c_double), ("full_samples", C.c_int64),
        ("fixed_lambda", C.c_int32), ("abf_on", C.c_int32),
        ("sc_form", C.c_int32), ("reserved2", C.c_int32), ("sc_shift", C.c_double),
    ]


class Info(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("n_slots", C.c_int64), ("n_clusters", C.c_int64),
                ("n_list_entries", C.c_int64), ("n_walkers", C.c_int32), ("list_cap", C.c_int32),
                ("precision", C.c_int32), ("uniform_lj", C.c_int32),
                ("list_max_env", C.c_int32), ("list_max_alch", C.c_int32),
                ("n_solute", C.c_int64)]


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LabfError(-3, f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        # torch carries its own HIP runtime; it must be loaded before this
        # library starts HIP, or torch finds no GPU later in the process
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "labf_workspace_size": ([P, P], I32),
            "labf_create_system": ([P, P, P], I32),
            "labf_set_lambda_params": ([P, P, P], I32),
            "labf_step_walkers": ([P, I64, I32, P], I32),
            "labf_read_abf_bins": ([P, I32, I32, P, P, P, P], I32),
            "labf_free_energy": ([P, P, P, P, P], I32),
            "labf_read_walker_state": ([P, P, P, P, P, P, P, P], I32),
            "labf_read_atoms": ([P, P, P, P], I32),
            "labf_write_atoms": ([P, P, P, P], I32),
            "labf_compute_forces": ([P, P, P, P, P], I32),
            "labf_export_pairs": ([P, I32, I64, P, P, P], I32),
            "labf_export_pairs_noalloc": ([P, I32, I64, P, P, P], I32),
            "labf_count_pairs": ([P, P, P, P], I32),
            "labf_profile_steps": ([P, I64, P, P], I32),
            "labf_philox": ([I64, P, P, P, P], I32),
            "labf_probe": ([I32, I64, P, P], I32),
            "labf_get_info": ([P, P, P], I32),
            "labf_energy_forward": ([P, P, P, P, P, P, P], I32),
            "labf_energy_backward": ([P, P, P, P, P, P, P, P, P], I32),
            "labf_set_distance_restraint": ([P, P, C.c_double, C.c_double, I32, P], I32),
            "labf_destroy_system": ([P], None),
            "labf_last_error": ([P], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def _stream(stream):
    """The HIP stream handle of a call: the given one, else torch's current
    stream (the default stream without a GPU build of torch)."""
    if stream is not None:
        return int(stream)
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream) or None
    except ImportError:
        pass
    return None


def _dev(t, shape, name):
    """Device pointer of a contiguous float64 CUDA (HIP) tensor of the given
    shape, or None."""
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise LabfError(-1, f"{name}: need a contiguous float64 GPU tensor of shape {tuple(shape)}")
    return t.data_ptr()


def _torch_stream(stream):
    import torch
    return int(stream) if stream is not None else torch.cuda.current_stream().cuda_stream


def _desc(spec: SystemSpec, max_bins: int = 0, list_capacity: int = 0):
    """(labf_system_desc, the host arrays it points to) of a SystemSpec."""
    keep = dict(
        atom_offset=np.ascontiguousarray(spec.atom_offset, np.int64), box=_f64(spec.box, (-1, 3)),
        pos=_f64(spec.pos, (-1, 3)), vel=_f64(spec.vel, (-1, 3)), mass=_f64(spec.mass),
        charge=_f64(spec.charge), sigma=_f64(spec.sigma), epsilon=_f64(spec.epsilon),
        is_solute=np.ascontiguousarray(spec.is_solute, np.uint8), anchor=_f64(spec.anchor, (-1, 3)),
        k0=_f64(spec.k0), k1=_f64(spec.k1), column_width=_f64(spec.column_width),
        prune_buffer=_f64(spec.prune_buffer),
        pme_dims=None if spec.pme_dims is None else np.ascontiguousarray(spec.pme_dims, np.int32))
    d = SystemDesc()
    d.n_walkers = spec.n_walkers
    d.precision = LABF_FP64 if spec.precision == "fp64" else LABF_FP32
    for k, v in keep.items():
        setattr(d, k, _p(v))
    for k in ("r_cut", "r_skin", "kT", "gamma", "dt", "coulomb_k", "accel_unit"):
        setattr(d, k, float(getattr(spec, k)))
    d.seed = int(spec.seed) & 0xFFFFFFFFFFFFFFFF
    d.rebuild_interval = int(spec.rebuild_interval)
    d.pme_order = 0 if spec.pme_dims is None else int(spec.pme_order)
    d.ewald_beta = float(spec.ewald_beta) if spec.pme_dims is not None else 0.0
    d.r_skin_alch = float(spec.r_skin_alch)
    d.max_bins = int(max_bins)
    d.list_capacity = int(list_capacity)
    return d, keep


def workspace_size(spec: SystemSpec, max_bins: int = 0, list_capacity: int = 0) -> int:
    """Bytes of device workspace a system of this spec needs (host arithmetic
    in the library, no GPU call)."""
    d, keep = _desc(spec, max_bins, list_capacity)
    n = C.c_size_t(0)
    rc = lib().labf_workspace_size(C.byref(d), C.byref(n))
    if rc != 0:
        raise LabfError(rc, lib().labf_last_error(None).decode())
    return int(n.value)


class System:
    """A batch of walkers living on the GPU (one labf_system handle).  Its
    device memory is a torch uint8 tensor (the workspace) that this object
    owns; every call runs on torch's current stream unless a stream is
    given."""

    def __init__(self, spec: SystemSpec, lam: Optional[LambdaSpec] = None, stream=None,
                 max_bins: Optional[int] = None, list_capacity: int = 0):
        self.spec = spec
        self._stream_arg = stream
        self._h = None
        self._ws = None
        self._last_cfg = {}
        if max_bins is None:
            max_bins = max(1024, int(lam.n_bins) if lam is not None else 0)
        d, keep = _desc(spec, max_bins, list_capacity)
        n = C.c_size_t(0)
        rc = lib().labf_workspace_size(C.byref(d), C.byref(n))
        if rc != 0:
            raise LabfError(rc, lib().labf_last_error(None).decode())
        import torch
        # torch owns the device memory (its caching allocator hands out
        # blocks aligned to at least 512 bytes)
        self._ws = torch.empty(int(n.value), dtype=torch.uint8, device="cuda")
        d.workspace, d.workspace_bytes = self._ws.data_ptr(), int(n.value)
        h = C.c_void_p()
        rc = lib().labf_create_system(C.byref(d), self.stream, C.byref(h))
        if rc != 0:
            self._ws = None
            raise LabfError(rc, lib().labf_last_error(None).decode())
        self._h = h
        self.W, self.N = spec.n_walkers, spec.n_atoms
        self.n_bins = None
        if lam is not None:
            self.set_lambda_params(lam)

    # -- plumbing ---------------------------------------------------------------
    def _chk(self, rc):
        if rc != 0:
            raise LabfError(rc, lib().labf_last_error(self._h).decode())

    def _chk_cfg(self, rc):
        """_chk for the calls that install a configuration: after a failure
        the system's configuration is unknown to the binding."""
        if rc != 0:
            self._last_cfg.clear()
        self._chk(rc)

    @property
    def stream(self):
        """Stream handle of the calls: the one given at creation, else torch's
        current stream."""
        return _stream(self._stream_arg)

    @property
    def workspace_bytes(self) -> int:
        return 0 if self._ws is None else int(self._ws.numel())

    def close(self):
        if self._h is not None:
            lib().labf_destroy_system(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls ------------------------------------------------------------------
    def set_lambda_params(self, lam: LambdaSpec):
        lam0 = np.ascontiguousarray(lam.lambda0, np.float64)
        p0 = None if lam.p_lambda0 is None else np.ascontiguousarray(lam.p_lambda0, np.float64)
        p = LambdaParams()
        p.lambda0, p.p_lambda0 = _p(lam0), _p(p0)
        p.m_lambda, p.gamma_lambda, p.kT_lambda = lam.m_lambda, lam.gamma_lambda, lam.kT_lambda
        p.elec_start, p.elec_end, p.vdw_start, p.vdw_end = (lam.elec_start, lam.elec_end,
                                                            lam.vdw_start, lam.vdw_end)
        p.direction = LABF_COUPLE if lam.direction == "couple" else LABF_DECOUPLE
        p.sc_power, p.sc_alpha = int(lam.sc_power), float(lam.sc_alpha)
        p.n_bins, p.share_interval = int(lam.n_bins), int(lam.share_interval)
        p.lo, p.hi, p.full_samples = float(lam.lo), float(lam.hi), int(lam.full_samples)
        p.fixed_lambda, p.abf_on = int(lam.fixed_lambda), int(lam.abf_on)
        p.sc_form = 1 if lam.sc_form == "shifted" else 0
        p.sc_shift = float(lam.sc_shift)
        self._chk(lib().labf_set_lambda_params(self._h, C.byref(p), self.stream))
        if lam.dr_pairs is not None:
            self.set_distance_restraint(lam.dr_pairs, lam.dr_delta, lam.dr_k, lam.dr_freq)
        self.n_bins = int(lam.n_bins)

    def step(self, n_steps: int, mode: str = "batched"):
        m = MODE_PLAIN if mode == "plain" else MODE_BATCHED
        self._last_cfg.clear()
        self._chk(lib().labf_step_walkers(self._h, int(n_steps), m, self.stream))

    def set_distance_restraint(self, pairs, delta: float, k: float, freq: int = 1):
        """Lambda-dependent distance restraint between two atoms per walker
        (pairs [W][2] walker-local indices, (-1, -1) for none; None removes it)."""
        pr = None if pairs is None else np.ascontiguousarray(pairs, np.int32).reshape(self.W, 2)
        self._chk(lib().labf_set_distance_restraint(self._h, _p(pr), float(delta), float(k), int(freq),
                                                    self.stream))

    def read_abf_bins(self, include_unshared: bool = True):
        c = np.zeros(self.n_bins, np.int64)
        s1 = np.zeros(self.n_bins)
        s2 = np.zeros(self.n_bins)
        self._chk(lib().labf_read_abf_bins(self._h, self.n_bins, int(include_unshared), _p(c), _p(s1),
                                           _p(s2), self.stream))
        return c, s1, s2

    def free_energy(self):
        g, prof, da = np.zeros(self.n_bins), np.zeros(self.n_bins), np.zeros(1)
        rc = lib().labf_free_energy(self._h, _p(g), _p(prof), _p(da), self.stream)
        if rc not in (0, -7):
            self._chk(rc)
        return g, prof, float(da[0]), int(rc)

    def read_walker_state(self):
        W = self.W
        lam, p, g, b = np.zeros(W), np.zeros(W), np.zeros(W), np.zeros(W)
        st = np.zeros(W, np.uint32)
        step = np.zeros(1, np.int64)
        self._chk(lib().labf_read_walker_state(self._h, _p(lam), _p(p), _p(g), _p(b), _p(st),
                                               _p(step), self.stream))
        return dict(lam=lam, p_lambda=p, dudl=g, bias=b, status=st, step=int(step[0]))

    # -- differentiable energy (device tensors; see paper_2307_08006_amd.autograd)
    @property
    def n_solute(self) -> int:
        return int(np.count_nonzero(self.spec.is_solute))

    def solute_params(self):
        """(epsilon, sigma, q) of the solute atoms in increasing atom order, [S][3]."""
        m = np.asarray(self.spec.is_solute).astype(bool)
        return np.stack([np.asarray(self.spec.epsilon)[m], np.asarray(self.spec.sigma)[m],
                         np.asarray(self.spec.charge)[m]], axis=1)

    def _changed(self, name, t):
        """Device pointer of t, or None when t is the tensor (same storage,
        same version) the system was given last time under this name: the
        library then keeps its configuration and the lists built for it."""
        if t is None:
            return None
        key = (t.data_ptr(), t._version, tuple(t.shape))
        last = self._last_cfg.get(name)
        if last is not None and last[1] == key:
            return None
        # the reference keeps that memory from being reused by another
        # tensor, which could otherwise present the same pointer and version
        self._last_cfg[name] = (t, key)
        return t.data_ptr()

    def energy(self, pos=None, lam=None, params=None, out=None, dudl=None, stream=None):
        """Total potential energy per walker [W] at the given configuration
        (float64 GPU tensors, each optional; the configuration replaces the
        system's); dV/dlambda per walker into dudl if given.  Energies only:
        no forces or parameter gradients are computed."""
        import torch
        W, N, S = self.W, self.N, self.n_solute
        if out is None:
            out = torch.empty(W, dtype=torch.float64, device="cuda")
        _dev(pos, (N, 3), "pos"), _dev(params, (S, 3), "params")
        self._chk_cfg(lib().labf_energy_forward(
            self._h, self._changed("pos", pos), _dev(lam, (W,), "lambda"),
            self._changed("params", params), _dev(out, (W,), "energy"), _dev(dudl, (W,), "dudl"),
            _torch_stream(stream)))
        return out

    def energy_backward(self, grad_energy, pos=None, lam=None, params=None, grad_pos=None,
                        grad_lam=None, grad_params=None, stream=None):
        """Recompute the pair terms at the given configuration and write
        g_w dV/dx, g_w dV/dlambda and g_w dV/d(eps, sigma, q) of the solute
        into the given output tensors (each optional).  Positions and
        parameters identical to the last call's (same tensors, unmodified)
        are not installed again, so the neighbour lists are reused."""
        W, N, S = self.W, self.N, self.n_solute
        _dev(pos, (N, 3), "pos"), _dev(params, (S, 3), "params")
        self._chk_cfg(lib().labf_energy_backward(
            self._h, self._changed("pos", pos), _dev(lam, (W,), "lambda"),
            self._changed("params", params), _dev(grad_energy, (W,), "grad_energy"),
            _dev(grad_pos, (N, 3), "grad_pos"), _dev(grad_lam, (W,), "grad_lambda"),
            _dev(grad_params, (S, 3), "grad_params"), _torch_stream(stream)))

    def read_atoms(self):
        pos = np.zeros((self.N, 3))
        vel = np.zeros((self.N, 3))
        self._chk(lib().labf_read_atoms(self._h, _p(pos), _p(vel), self.stream))
        return pos, vel

    def write_atoms(self, pos=None, vel=None):
        pos = _f64(pos, (-1, 3))
        vel = _f64(vel, (-1, 3))
        self._last_cfg.clear()
        self._chk(lib().labf_write_atoms(self._h, _p(pos), _p(vel), self.stream))

    def compute_forces(self):
        f = np.zeros((self.N, 3))
        e = np.zeros((self.W, 5))
        g = np.zeros(self.W)
        self._chk(lib().labf_compute_forces(self._h, _p(f), _p(e), _p(g), self.stream))
        return f, e, g

    def export_pairs(self, walker: int) -> np.ndarray:
        n = np.zeros(1, np.int64)
        self._chk(lib().labf_export_pairs(self._h, int(walker), 0, None, _p(n), self.stream))
        out = np.zeros((max(int(n[0]), 1), 2), np.int64)
        self._chk(lib().labf_export_pairs(self._h, int(walker), out.shape[0], _p(out), _p(n),
                                          self.stream))
        return out[: int(n[0])]

    def count_pairs(self, env_only: bool = False) -> np.ndarray:
        """Pairs with r < r_cut per walker (all pairs, or environment pairs)."""
        out = np.zeros(self.W, np.int64)
        env = np.zeros(self.W, np.int64)
        self._chk(lib().labf_count_pairs(self._h, _p(out), _p(env), self.stream))
        return env if env_only else out

    def profile_steps(self, n_steps: int) -> dict:
        """Per-kernel times (ms) from HIP events around single launches."""
        ms = np.zeros(5)
        self._chk(lib().labf_profile_steps(self._h, int(n_steps), _p(ms), self.stream))
        return dict(rebuild_ms=float(ms[0]), alch_ms=float(ms[1]), env_ms=float(ms[2]),
                    pme_ms=float(ms[3]), prune_ms=float(ms[4]))

    def info(self) -> dict:
        inf = Info()
        self._chk(lib().labf_get_info(self._h, C.byref(inf), self.stream))
        return {k: getattr(inf, k) for k, _ in Info._fields_}


PROBES = {"fp32_fma": 0, "fp64_fma": 1, "fp32_rsq": 2, "triad": 3}


def probe(kind: str, n: int, stream=None) -> float:
    """Achievable-peak probe of the device: lane-operations/s for the FMA and
    rsqrt chains (n iterations), bytes/s for the triad (n floats per array)."""
    rate = np.zeros(1)
    rc = lib().labf_probe(PROBES[kind], int(n), _p(rate), _stream(stream))
    if rc != 0:
        raise LabfError(rc, lib().labf_last_error(None).decode())
    return float(rate[0])


def philox(ctr, key, stream=None) -> np.ndarray:
    """Philox4x32-10 of the device for counters ctr[n,4] and key[2]."""
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, np.uint32).reshape(2)
    out = np.zeros_like(ctr)
    rc = lib().labf_philox(ctr.shape[0], _p(ctr), _p(key), _p(out), _stream(stream))
    if rc != 0:
        raise LabfError(rc, lib().labf_last_error(None).decode())
    return out


def create_error() -> str:
    return lib().labf_last_error(None).decode()
