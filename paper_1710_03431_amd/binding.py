"""ctypes binding of libaqt (include/aqt.h): argument marshalling only.

Every numerical step runs in the HIP library; PyTorch supplies device memory
and the stream.  Importing this module loads the in-tree libaqt.so and raises
if it is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaqt.so")

AQT_OK, AQT_EINVAL, AQT_ENOMEM, AQT_ESTATE, AQT_EHIP, AQT_ENUMERIC, AQT_ECAPACITY = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, BF16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16}
KIND_NAMES = ("relax", "excite", "dephase")

EXPORTED = ("aqt_create", "aqt_destroy", "aqt_last_error", "aqt_version", "aqt_set_hamiltonian",
            "aqt_set_schedule", "aqt_set_bath", "aqt_precompute", "aqt_precompute_ex", "aqt_set_tables", "aqt_get_tables",
            "aqt_get_dims", "aqt_run", "aqt_grad_pgs", "aqt_set_lamb_shift", "aqt_get_lamb_shift",
            "aqt_set_bath_correlation", "aqt_set_bath_terms", "aqt_set_coupling", "aqt_get_channel_count",
            "aqt_set_grid", "aqt_run_fixed_step", "aqt_run_status", "aqt_run_noalloc",
            "aqt_step_bound", "aqt_bound_grid", "aqt_bound_grid_points",
            "aqt_batch_create", "aqt_batch_launch", "aqt_batch_tiles",
            "aqt_batch_last_error", "aqt_batch_destroy")
BATCH_GRAPH, BATCH_AUTOTUNE = 1, 2
RUN_RECORDS_TRUNCATED, RUN_JUMP_LIMIT = 1, 2


class Jump(C.Structure):
    _fields_ = [("t", C.c_double), ("step", C.c_int32), ("qubit", C.c_int16), ("kind", C.c_int16),
                ("from_level", C.c_int32), ("to_level", C.c_int32)]


class RunParams(C.Structure):
    _fields_ = [("precision", C.c_int32), ("record_capacity", C.c_int32), ("n_traj", C.c_int64),
                ("seed", C.c_uint64), ("instance_id", C.c_uint64), ("traj_offset", C.c_uint64),
                ("tile", C.c_int32), ("segment", C.c_int32)]


class Outputs(C.Structure):
    _fields_ = [("pgs_sum", C.c_void_p), ("pgs_sumsq", C.c_void_p), ("jump_totals", C.c_void_p),
                ("jump_count", C.c_void_p), ("jumps", C.c_void_p), ("net_gs", C.c_void_p),
                ("net_hist", C.c_void_p), ("hist_lo", C.c_int32), ("hist_hi", C.c_int32),
                ("final_state", C.c_void_p)]


EIG_METHODS = {"auto": 0, "dense": 1, "iterative": 2}

JUMP_DTYPE = np.dtype([("t", "<f8"), ("step", "<i4"), ("qubit", "<i2"), ("kind", "<i2"),
                       ("from_level", "<i4"), ("to_level", "<i4")])
assert JUMP_DTYPE.itemsize == C.sizeof(Jump) == 24


class AqtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libaqt status {status}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libaqt.so and declare the C signatures (no GPU work happens here)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1710_03431_amd.build`")
    # torch bundles its own HIP runtime under the same soname as /opt/rocm's; load it
    # first so that libaqt and torch share one runtime (streams, allocations).
    import torch  # noqa: F401
    lib = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    ctx = C.c_void_p
    lib.aqt_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]
    lib.aqt_destroy.argtypes = [ctx]
    lib.aqt_destroy.restype = None
    lib.aqt_last_error.argtypes = [ctx]
    lib.aqt_last_error.restype = C.c_char_p
    lib.aqt_version.argtypes = []
    lib.aqt_set_hamiltonian.argtypes = [ctx, C.c_int, dp, dp]
    lib.aqt_set_schedule.argtypes = [ctx, C.c_double, C.c_int, dp, dp]
    lib.aqt_set_bath.argtypes = [ctx, C.c_double, C.c_double, C.c_double]
    lib.aqt_precompute.argtypes = [ctx, C.c_int, C.c_int, C.c_double]
    lib.aqt_precompute_ex.argtypes = [ctx, C.c_int, C.c_int, C.c_double, C.c_int]
    lib.aqt_set_tables.argtypes = [ctx, C.c_int, C.c_int, dp, ip, dp, dp, dp, dp]
    lib.aqt_get_tables.argtypes = [ctx, dp, ip, dp, dp, dp, dp, dp, dp]
    lib.aqt_get_dims.argtypes = [ctx, ip, ip, ip]
    lib.aqt_run.argtypes = [ctx, C.POINTER(RunParams), C.POINTER(Outputs)]
    lib.aqt_grad_pgs.argtypes = [ctx, C.POINTER(RunParams), dp, dp, dp, dp, C.c_void_p]
    lib.aqt_set_lamb_shift.argtypes = [ctx, C.c_int]
    lib.aqt_set_bath_correlation.argtypes = [ctx, dp]
    lib.aqt_set_bath_terms.argtypes = [ctx, C.c_int, dp, dp]
    lib.aqt_set_coupling.argtypes = [ctx, C.c_int, dp, dp, dp]
    lib.aqt_set_grid.argtypes = [ctx, C.c_int, dp]
    lib.aqt_get_channel_count.argtypes = [ctx, ip]
    lib.aqt_run_fixed_step.argtypes = [ctx, C.POINTER(RunParams), C.c_int, C.POINTER(Outputs)]
    lib.aqt_run_status.argtypes = [ctx, ip]
    lib.aqt_run_noalloc.argtypes = [ctx, C.POINTER(RunParams), C.POINTER(Outputs)]
    lib.aqt_step_bound.argtypes = [ctx, C.c_int, dp]
    lib.aqt_bound_grid.argtypes = [ctx, C.c_int, C.c_int, dp]
    lib.aqt_bound_grid_points.argtypes = [ctx, C.c_double, C.c_int, ip]
    lib.aqt_get_lamb_shift.argtypes = [ctx, dp]
    lib.aqt_batch_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int,
                                     C.POINTER(RunParams), C.POINTER(Outputs), C.c_int]
    lib.aqt_batch_launch.argtypes = [C.c_void_p]
    lib.aqt_batch_tiles.argtypes = [C.c_void_p, ip]
    lib.aqt_batch_last_error.argtypes = [C.c_void_p]
    lib.aqt_batch_last_error.restype = C.c_char_p
    lib.aqt_batch_destroy.argtypes = [C.c_void_p]
    lib.aqt_batch_destroy.restype = None
    for name in EXPORTED:
        if name not in ("aqt_destroy", "aqt_last_error", "aqt_batch_last_error", "aqt_batch_destroy"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Engine:
    """One libaqt context bound to a GPU and a stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = self.lib.aqt_create(C.byref(h), device, C.c_void_p(stream.cuda_stream))
        if st != AQT_OK:
            raise AqtError(st, f"aqt_create failed on device {device} (no usable HIP device?)")
        self.ctx = h
        self.n_grid = self.n_levels = self.n_qubits = self.n_channels = None
        self.n_ctrl = 0

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.aqt_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != AQT_OK:
            raise AqtError(st, self.lib.aqt_last_error(self.ctx).decode())

    # ---------------------------------------------------------------- inputs
    def set_hamiltonian(self, h, J):
        h = _f64(h)
        J = _f64(J)
        self._check(self.lib.aqt_set_hamiltonian(self.ctx, len(h), _dptr(h), _dptr(J)))

    def set_schedule(self, t_f, A_ctrl, B_ctrl):
        A = _f64(A_ctrl)
        B = _f64(B_ctrl)
        self._check(self.lib.aqt_set_schedule(self.ctx, float(t_f), len(A), _dptr(A), _dptr(B)))
        self.n_ctrl = len(A)

    def set_bath(self, eta, omega_c, T):
        self._check(self.lib.aqt_set_bath(self.ctx, float(eta), float(omega_c), float(T)))

    def set_bath_correlation(self, C=None):
        """gamma_ab(w) = C_ab gamma(w) between the qubits' baths (None: independent)."""
        self._check(self.lib.aqt_set_bath_correlation(self.ctx, None if C is None else _dptr(_f64(C))))

    def set_bath_terms(self, terms=None):
        """gamma_ab(w) = sum_m C_m[a, b] gamma(w; omega_c_m) for terms ((C_m, omega_c_m), ...)
        (None or empty: independent baths)."""
        if not terms:
            self._check(self.lib.aqt_set_bath_terms(self.ctx, 0, None, None))
            return
        Cs = _f64(np.stack([np.asarray(c, dtype=np.float64) for c, _ in terms]))
        wc = _f64(np.array([float(w) for _, w in terms]))
        self._check(self.lib.aqt_set_bath_terms(self.ctx, len(terms), _dptr(Cs), _dptr(wc)))

    def set_coupling(self, cz=None, cx=None, omega_c=None):
        """Channel k couples through sum_a (cz[k][a] sz_a + cx[k][a] sx_a) with cutoff omega_c[k]
        (None: the bath's); cz and cx [n_channels, n_qubits]; both None: sz of each qubit."""
        if cz is None and cx is None:
            self._check(self.lib.aqt_set_coupling(self.ctx, 0, None, None, None))
            return
        z = None if cz is None else _f64(np.atleast_2d(cz))
        x = None if cx is None else _f64(np.atleast_2d(cx))
        nch = (z if z is not None else x).shape[0]
        w = None if omega_c is None else _f64(np.asarray(omega_c, dtype=np.float64).reshape(nch))
        self._check(self.lib.aqt_set_coupling(self.ctx, nch, None if z is None else _dptr(z),
                                              None if x is None else _dptr(x), None if w is None else _dptr(w)))

    def set_grid(self, s=None):
        """Grid points s_0 = 0 < ... < s_{M-1} = 1 of the anneal (None: equidistant)."""
        if s is None:
            self._check(self.lib.aqt_set_grid(self.ctx, 0, None))
            return
        s = _f64(s)
        self._check(self.lib.aqt_set_grid(self.ctx, len(s), _dptr(s)))

    def step_bound(self, n_probe: int):
        """App. B time-step bound (ns) at n_probe equidistant s points (aqt_step_bound)."""
        out = np.zeros(int(n_probe))
        self._check(self.lib.aqt_step_bound(self.ctx, int(n_probe), _dptr(out)))
        return out

    def bound_grid(self, n_grid: int, n_probe: int = 401):
        """Grid of n_grid points following the App. B bound (aqt_bound_grid); not applied."""
        out = np.zeros(int(n_grid))
        self._check(self.lib.aqt_bound_grid(self.ctx, int(n_grid), int(n_probe), _dptr(out)))
        return out

    def bound_grid_points(self, fraction: float, n_probe: int = 401) -> int:
        """Fewest grid points whose bound-following grid keeps every step within `fraction`
        of the App. B bound (aqt_bound_grid_points)."""
        v = C.c_int32()
        self._check(self.lib.aqt_bound_grid_points(self.ctx, float(fraction), int(n_probe), C.byref(v)))
        return v.value

    def channel_count(self) -> int:
        v = C.c_int32()
        self._check(self.lib.aqt_get_channel_count(self.ctx, C.byref(v)))
        return v.value

    def set_lamb_shift(self, enabled: bool):
        self._check(self.lib.aqt_set_lamb_shift(self.ctx, int(bool(enabled))))

    def get_lamb_shift(self):
        out = np.zeros((self.n_grid, self.n_levels))
        self._check(self.lib.aqt_get_lamb_shift(self.ctx, _dptr(out)))
        return out

    def set_instance(self, inst):
        """Hamiltonian, schedule, bath and Lamb-shift choice of a workloads.Instance."""
        self.set_hamiltonian(inst.h, inst.J)
        self.set_schedule(inst.t_f, inst.A_ctrl, inst.B_ctrl)
        self.set_bath(inst.eta, inst.omega_c, inst.T)
        self.set_bath_correlation(getattr(inst, "bath_corr", None))
        if getattr(inst, "bath_terms", None) is not None:
            self.set_bath_terms(inst.bath_terms)
        if getattr(inst, "coupling", None) is not None:
            self.set_coupling(*inst.coupling)
        self.set_grid(getattr(inst, "s_grid", None))
        self.set_lamb_shift(getattr(inst, "lamb_shift", False))

    def precompute(self, n_grid: int, n_levels: int, deg_tol: float = 1e-8, method: str = "auto"):
        """GPU eigensystem and tables; method "auto", "dense" or "iterative"."""
        m = EIG_METHODS[method]
        self._check(self.lib.aqt_precompute_ex(self.ctx, int(n_grid), int(n_levels), float(deg_tol), m))
        self._dims()

    def set_tables(self, E, gs, O, cinit, R, zdiag):
        E = _f64(E)
        M, n = E.shape
        gs = np.ascontiguousarray(np.asarray(gs, dtype=np.int32))
        O = _f64(O)
        cinit = _f64(cinit)
        R = _f64(R)
        zdiag = _f64(zdiag)
        self._check(self.lib.aqt_set_tables(self.ctx, M, n, _dptr(E), _iptr(gs), _dptr(O), _dptr(cinit),
                                            _dptr(R), _dptr(zdiag)))
        self._dims()

    def _dims(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.aqt_get_dims(self.ctx, C.byref(a), C.byref(b), C.byref(c)))
        self.n_grid, self.n_levels, self.n_qubits = a.value, b.value, c.value
        self.n_channels = self.channel_count()

    def get_tables(self, want=("E", "gs", "O", "cinit", "R", "zdiag", "Gamma", "leak")):
        M, n, nq = self.n_grid, self.n_levels, self.n_channels
        shapes = {"E": (M, n), "gs": (M,), "O": (M, n, n), "cinit": (n,), "R": (M, nq, n, n),
                  "zdiag": (M, nq, n), "Gamma": (M, n), "leak": (M,)}
        out = {k: (np.zeros(shapes[k], dtype=np.int32 if k == "gs" else np.float64) if k in want else None)
               for k in shapes}
        self._check(self.lib.aqt_get_tables(self.ctx, _dptr(out["E"]), _iptr(out["gs"]), _dptr(out["O"]),
                                            _dptr(out["cinit"]), _dptr(out["R"]), _dptr(out["zdiag"]),
                                            _dptr(out["Gamma"]), _dptr(out["leak"])))
        return {k: v for k, v in out.items() if v is not None}

    # ---------------------------------------------------------------- run
    def run_status(self) -> int:
        """AQT_RUN_* flags of the runs since the last call (synchronises the stream).
        Raises if a trajectory hit the per-step jump limit; truncated records are only
        reported in the flags (observables and jump counts stay valid)."""
        v = C.c_int32()
        st = self.lib.aqt_run_status(self.ctx, C.byref(v))
        if st not in (AQT_OK, AQT_ECAPACITY):
            self._check(st)
        return v.value

    def alloc_outputs(self, n_traj: int, record_capacity: int = 0, hist=(-64, 64), final_state=False,
                      per_trajectory=True):
        t = self.torch
        dev = t.device("cuda", self.device)
        M, n = self.n_grid, self.n_levels
        o = {"pgs_sum": t.zeros(M, dtype=t.float64, device=dev),
             "pgs_sumsq": t.zeros(M, dtype=t.float64, device=dev),
             "jump_totals": t.zeros(3, dtype=t.int64, device=dev),
             "net_hist": t.zeros(hist[1] - hist[0] + 1, dtype=t.int64, device=dev),
             "hist": hist}
        if per_trajectory:
            o["jump_count"] = t.zeros(n_traj, dtype=t.int32, device=dev)
            o["net_gs"] = t.zeros(n_traj, dtype=t.int32, device=dev)
        if record_capacity:
            o["jumps"] = t.zeros(n_traj * record_capacity * 24, dtype=t.uint8, device=dev)
        if final_state:
            o["final_state"] = t.zeros(n_traj * n * 2, dtype=t.float64, device=dev)
        return o

    def run_into(self, outs: dict, n_traj: int, precision="fp64", seed=0, instance_id=0, traj_offset=0,
                 record_capacity=0, tile=0):
        """Enqueue one run writing into pre-allocated outputs (no synchronisation)."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        p = RunParams(precision=prec, record_capacity=int(record_capacity), n_traj=int(n_traj),
                      seed=int(seed), instance_id=int(instance_id), traj_offset=int(traj_offset),
                      tile=int(tile), segment=0)

        def ptr(k):
            v = outs.get(k)
            return None if v is None else v.data_ptr()

        o = Outputs(pgs_sum=ptr("pgs_sum"), pgs_sumsq=ptr("pgs_sumsq"), jump_totals=ptr("jump_totals"),
                    jump_count=ptr("jump_count"), jumps=ptr("jumps"), net_gs=ptr("net_gs"),
                    net_hist=ptr("net_hist"), hist_lo=int(outs["hist"][0]), hist_hi=int(outs["hist"][1]),
                    final_state=ptr("final_state"))
        self._check(self.lib.aqt_run(self.ctx, C.byref(p), C.byref(o)))

    def run_noalloc_into(self, outs: dict, n_traj: int, precision="fp64", seed=0, instance_id=0, traj_offset=0,
                         record_capacity=0, tile=0):
        """As run_into, through aqt_run_noalloc (no device allocation by the library)."""
        p = _params(n_traj, precision, seed, instance_id, traj_offset, record_capacity, tile)
        self._check(self.lib.aqt_run_noalloc(self.ctx, C.byref(p), C.byref(_outputs(outs))))

    def run(self, n_traj: int, precision="fp64", seed=0, instance_id=0, traj_offset=0, record_capacity=0,
            tile=0, final_state=False, hist=(-64, 64)):
        """Run K trajectories and return host numpy results (synchronises)."""
        outs = self.alloc_outputs(n_traj, record_capacity, hist, final_state)
        self.run_into(outs, n_traj, precision, seed, instance_id, traj_offset, record_capacity, tile)
        flags = self.run_status()
        res = {k: v.cpu().numpy() for k, v in outs.items() if k not in ("hist", "jumps")}
        res["hist_lo"] = hist[0]
        res["records_truncated"] = bool(flags & RUN_RECORDS_TRUNCATED)
        if record_capacity:
            raw = outs["jumps"].cpu().numpy().view(JUMP_DTYPE).reshape(n_traj, record_capacity)
            res["jumps"] = raw
        if final_state:
            res["final_state"] = res["final_state"].reshape(n_traj, self.n_levels, 2)
        return res


    def run_fixed_step(self, n_traj: int, substeps: int, precision="fp64", seed=0, instance_id=0, traj_offset=0,
                       record_capacity=0, final_state=False):
        """Fixed-step unraveling (aqt_run_fixed_step); host numpy results (synchronises)."""
        outs = self.alloc_outputs(n_traj, record_capacity, (0, 0), final_state)
        outs.pop("net_hist")
        p = _params(n_traj, precision, seed, instance_id, traj_offset, record_capacity, 0)

        def ptr(k):
            v = outs.get(k)
            return None if v is None else v.data_ptr()

        o = Outputs(pgs_sum=ptr("pgs_sum"), pgs_sumsq=ptr("pgs_sumsq"), jump_totals=ptr("jump_totals"),
                    jump_count=ptr("jump_count"), jumps=ptr("jumps"), net_gs=ptr("net_gs"), net_hist=None,
                    hist_lo=0, hist_hi=0, final_state=ptr("final_state"))
        self._check(self.lib.aqt_run_fixed_step(self.ctx, C.byref(p), int(substeps), C.byref(o)))
        flags = self.run_status()
        res = {k: v.cpu().numpy() for k, v in outs.items() if k not in ("hist", "jumps")}
        res["records_truncated"] = bool(flags & RUN_RECORDS_TRUNCATED)
        if record_capacity:
            res["jumps"] = outs["jumps"].cpu().numpy().view(JUMP_DTYPE).reshape(n_traj, record_capacity)
        if final_state:
            res["final_state"] = res["final_state"].reshape(n_traj, self.n_levels, 2)
        return res

    # ---------------------------------------------------------------- gradient
    def grad_pgs(self, n_traj: int, precision="fp32", seed=0, instance_id=0, traj_offset=0, tile=0,
                 per_trajectory=False, segment=0):
        """Gradient of E[P_GS(1)] with respect to (A controls, B controls, eta) (synchronises).
        Returns value, value_se, grad, grad_se and, on request, per_traj [K][2(2m+2)]
        (f, g, then 1, s; see aqt_grad_pgs)."""
        m = self.n_ctrl
        p = _params(n_traj, precision, seed, instance_id, traj_offset, 0, tile)
        p.segment = int(segment)
        v, vse = np.zeros(1), np.zeros(1)
        g, gse = np.zeros(2 * m + 1), np.zeros(2 * m + 1)
        pt = None
        if per_trajectory:
            t = self.torch
            pt = t.zeros((n_traj, 2 * (2 * m + 2)), dtype=t.float64, device=t.device("cuda", self.device))
        self._check(self.lib.aqt_grad_pgs(self.ctx, C.byref(p), _dptr(v), _dptr(vse), _dptr(g), _dptr(gse),
                                          None if pt is None else pt.data_ptr()))
        out = {"value": float(v[0]), "value_se": float(vse[0]), "grad": g, "grad_se": gse}
        if pt is not None:
            out["per_traj"] = pt.cpu().numpy()
        return out


def _params(n_traj, precision, seed, instance_id, traj_offset, record_capacity, tile):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return RunParams(precision=prec, record_capacity=int(record_capacity), n_traj=int(n_traj), seed=int(seed),
                     instance_id=int(instance_id), traj_offset=int(traj_offset), tile=int(tile), segment=0)


def _outputs(outs):
    def ptr(k):
        v = outs.get(k)
        return None if v is None else v.data_ptr()
    return Outputs(pgs_sum=ptr("pgs_sum"), pgs_sumsq=ptr("pgs_sumsq"), jump_totals=ptr("jump_totals"),
                   jump_count=ptr("jump_count"), jumps=ptr("jumps"), net_gs=ptr("net_gs"),
                   net_hist=ptr("net_hist"), hist_lo=int(outs["hist"][0]), hist_hi=int(outs["hist"][1]),
                   final_state=ptr("final_state"))


def _pgs_function():
    """torch.autograd.Function for E[P_GS(1)] of an Engine's instance (built lazily so that
    importing this module does not import torch)."""
    import torch

    class PGS(torch.autograd.Function):
        """value = E[P_GS(1)] estimated from n_traj trajectories; backward multiplies the
        gradient that aqt_grad_pgs returns with the same forward call (controls of A, of B,
        eta; CPU float64 tensors).  The engine's Hamiltonian and bath constants other than
        eta are used as set; the schedule and eta are taken from the inputs."""

        @staticmethod
        def forward(ctx, A_ctrl, B_ctrl, eta, engine, t_f, omega_c, T, n_grid, n_levels, n_traj, precision, seed):
            engine.set_schedule(t_f, A_ctrl.detach().cpu().numpy(), B_ctrl.detach().cpu().numpy())
            engine.set_bath(float(eta), omega_c, T)
            engine.precompute(n_grid, n_levels)
            out = engine.grad_pgs(n_traj, precision, seed=seed)
            m = A_ctrl.numel()
            g = torch.as_tensor(out["grad"], dtype=torch.float64)
            ctx.save_for_backward(g[:m].clone(), g[m:2 * m].clone(), g[2 * m:].clone())
            ctx.value_se = out["value_se"]
            return torch.tensor(out["value"], dtype=torch.float64)

        @staticmethod
        def backward(ctx, grad_out):
            gA, gB, ge = ctx.saved_tensors
            return (grad_out * gA, grad_out * gB, (grad_out * ge).reshape(()), None, None, None, None, None, None,
                    None, None, None)

    return PGS


def pgs(engine, A_ctrl, B_ctrl, eta, *, t_f, omega_c, T, n_grid, n_levels, n_traj, precision="fp32", seed=0):
    """Differentiable E[P_GS(1)] (see _pgs_function): A_ctrl, B_ctrl and eta are CPU float64
    tensors (eta 0-dimensional); gradients flow to them through aqt_grad_pgs."""
    return _pgs_function().apply(A_ctrl, B_ctrl, eta, engine, t_f, omega_c, T, n_grid, n_levels, n_traj,
                                 precision, seed)


class Batch:
    """Many instances (Engines with tables) run by one persistent launch (aqt_batch_*).

    runs: list of dicts with keys n_traj, seed, instance_id, traj_offset, record_capacity, tile.
    Output buffers are allocated here and bound at creation; launch() replays them.
    """

    def __init__(self, engines, runs, precision="bf16", graph=True, autotune=True, hist=(-64, 64)):
        self.engines = list(engines)
        self.lib = load_library()
        n = len(self.engines)
        self.outs = []
        params = (RunParams * n)()
        outs = (Outputs * n)()
        ctxs = (C.c_void_p * n)()
        for i, (eng, r) in enumerate(zip(self.engines, runs)):
            o = eng.alloc_outputs(r["n_traj"], r.get("record_capacity", 0), hist)
            self.outs.append(o)
            params[i] = _params(r["n_traj"], precision, r.get("seed", 0), r.get("instance_id", i),
                                r.get("traj_offset", 0), r.get("record_capacity", 0), r.get("tile", 0))
            outs[i] = _outputs(o)
            ctxs[i] = eng.ctx
        self.runs = list(runs)
        h = C.c_void_p()
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_AUTOTUNE if autotune else 0)
        st = self.lib.aqt_batch_create(C.byref(h), ctxs, n, params, outs, flags)
        if st != AQT_OK:
            msg = self.lib.aqt_batch_last_error(h).decode() if h.value else "aqt_batch_create failed"
            if h.value:
                self.lib.aqt_batch_destroy(h)
            raise AqtError(st, msg)
        self.handle = h
        t = (C.c_int32 * n)()
        self.lib.aqt_batch_tiles(h, t)
        self.tiles = list(t)

    def launch(self):
        st = self.lib.aqt_batch_launch(self.handle)
        if st != AQT_OK:
            raise AqtError(st, self.lib.aqt_batch_last_error(self.handle).decode())

    def results(self):
        """Host copies of every instance's outputs (synchronises the first engine's stream)."""
        self.engines[0].stream.synchronize()
        res = []
        for o, r in zip(self.outs, self.runs):
            d = {k: v.cpu().numpy() for k, v in o.items() if k not in ("hist", "jumps")}
            if r.get("record_capacity", 0):
                d["jumps"] = o["jumps"].cpu().numpy().view(JUMP_DTYPE).reshape(r["n_traj"], r["record_capacity"])
            res.append(d)
        return res

    def close(self):
        if getattr(self, "handle", None):
            self.lib.aqt_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
