"""ctypes binding of libqops (argument marshalling only: every step of the
simulation runs in the library's HIP kernels).  PyTorch supplies device
memory and the stream."""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqops.so")

# enum qops_kind
KINDS = ["h", "x", "y", "z", "s", "sdg", "t", "tdg", "sx", "rx", "ry", "rz", "p", "u3",
         "cx", "cz", "cp", "swap", "rzz", "dense"]
KIND_ID = {k: i for i, k in enumerate(KINDS)}
ARITY = {k: (1 if i <= KIND_ID["u3"] else 2) for k, i in KIND_ID.items() if k != "dense"}

C64, C128 = 0, 1
PLAN_GATEWISE, PLAN_FUSED, PLAN_PROFILED, PLAN_LEARNED = 0, 1, 2, 3
SWAP_VIRTUAL, SWAP_PHYSICAL = 0, 1
ORDER_LOGICAL, ORDER_PHYSICAL = 0, 1

STATUS = {0: "OK", -1: "INVALID_ARG", -2: "QUBIT_RANGE", -3: "DUPLICATE_QUBIT", -4: "UNSUPPORTED",
          -5: "OUT_OF_MEMORY", -6: "HIP_ERROR", -7: "BAD_STATE", -8: "NOT_UNITARY"}


class QopsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint16), ("k", ctypes.c_uint8), ("n_ctrl", ctypes.c_uint8),
                ("q", ctypes.c_int32 * 6), ("ctrl", ctypes.c_int32 * 4), ("param", ctypes.c_double * 3),
                ("mat", ctypes.POINTER(ctypes.c_double))]


class PlanOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("swap_mode", ctypes.c_int32), ("tile_upper", ctypes.c_int32),
                ("max_fuse_k", ctypes.c_int32), ("use_mfma", ctypes.c_int32), ("check_unitary", ctypes.c_int32),
                ("remap", ctypes.c_int32), ("profile", ctypes.c_void_p), ("model", ctypes.c_void_p),
                ("fold_rotations", ctypes.c_int32), ("merge_blocks", ctypes.c_int32)]


class PlanStats(ctypes.Structure):
    _fields_ = [("n_passes", ctypes.c_int32), ("n_tile_passes", ctypes.c_int32),
                ("n_permute_passes", ctypes.c_int32), ("n_ops", ctypes.c_int32), ("n_gates_in", ctypes.c_int32),
                ("n_virtual_swaps", ctypes.c_int32), ("tile_upper", ctypes.c_int32), ("max_fuse_k", ctypes.c_int32),
                ("bytes_alg", ctypes.c_double), ("predicted_s", ctypes.c_double), ("plan_seconds", ctypes.c_double),
                ("n_folded", ctypes.c_int32)]


class PassRecord(ctypes.Structure):
    _fields_ = [("pass_", ctypes.c_int32), ("type", ctypes.c_int32), ("n_ops", ctypes.c_int32),
                ("n_gates", ctypes.c_int32), ("tile_bits", ctypes.c_int32), ("n_mfma", ctypes.c_int32),
                ("max_k", ctypes.c_int32), ("n_remaps", ctypes.c_int32), ("t_begin", ctypes.c_double),
                ("seconds", ctypes.c_double), ("bytes_alg", ctypes.c_double), ("flops", ctypes.c_double),
                ("phys_mask", ctypes.c_uint64)]


class OpInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32), ("t", ctypes.c_int32 * 10),
                ("cmask", ctypes.c_uint64), ("pass_", ctypes.c_int32), ("n_merged", ctypes.c_int32)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("n", ctypes.POINTER(ctypes.c_int32)),
                ("gates", ctypes.POINTER(ctypes.POINTER(Gate))), ("n_gates", ctypes.POINTER(ctypes.c_size_t)),
                ("precision", ctypes.c_int32), ("stream", ctypes.c_void_p), ("small_max_n", ctypes.c_int32),
                ("tile_bits", ctypes.c_int32), ("max_fuse_k", ctypes.c_int32)]


class BatchStats(ctypes.Structure):
    _fields_ = [("small_circuits", ctypes.c_int32), ("tile_circuits", ctypes.c_int32),
                ("graph_nodes", ctypes.c_int32), ("small_max_n", ctypes.c_int32), ("tile_bits", ctypes.c_int32),
                ("max_fuse_k", ctypes.c_int32),
                ("outputs", ctypes.c_int64), ("state_bytes", ctypes.c_double)]


class TierOpts(ctypes.Structure):
    _fields_ = [("remap", ctypes.c_int32), ("reserved", ctypes.c_int32), ("plan", PlanOpts)]


class TierStats(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("groups", ctypes.c_int32), ("exchanges", ctypes.c_int32),
                ("virtual_swaps", ctypes.c_int32), ("gpu_passes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("h2d_bytes", ctypes.c_double), ("d2h_bytes", ctypes.c_double), ("seconds", ctypes.c_double),
                ("plan_seconds", ctypes.c_double)]


class PassInfo(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("tile_bits", ctypes.c_int32), ("n_upper", ctypes.c_int32),
                ("upper", ctypes.c_int32 * 8), ("n_ops", ctypes.c_int32), ("n_remaps", ctypes.c_int32),
                ("n_mfma", ctypes.c_int32), ("bytes_alg", ctypes.c_double), ("flops", ctypes.c_double)]


_lib = None

# name -> (restype, argtypes); every symbol include/qops.h declares
_VP, _I32, _SZ, _U64, _DP = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int32)
SIGNATURES = {
    "qops_last_error": (ctypes.c_char_p, []),
    "qops_version": (_I32, []),
    "qops_create": (_I32, [_I32, _I32, _VP, _SZ, _VP, ctypes.POINTER(_VP)]),
    "qops_destroy": (_I32, [_VP]),
    "qops_set_launch_limit": (_I32, [_VP, _I32]),
    "qops_state_pointer": (_I32, [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_SZ)]),
    "qops_init_basis": (_I32, [_VP, _U64]),
    "qops_init_amplitudes": (_I32, [_VP, _VP]),
    "qops_plan_opts_default": (_I32, [ctypes.POINTER(PlanOpts)]),
    "qops_plan_build": (_I32, [_I32, _I32, _IP, ctypes.POINTER(Gate), _SZ, ctypes.POINTER(PlanOpts), ctypes.POINTER(_VP)]),
    "qops_plan_free": (_I32, [_VP]),
    "qops_plan_stats_get": (_I32, [_VP, ctypes.POINTER(PlanStats)]),
    "qops_plan_final_layout": (_I32, [_VP, _IP]),
    "qops_plan_num_ops": (_I32, [_VP, ctypes.POINTER(_SZ)]),
    "qops_plan_op": (_I32, [_VP, _SZ, ctypes.POINTER(OpInfo), _DP]),
    "qops_plan_pass_info": (_I32, [_VP, _SZ, ctypes.POINTER(PassInfo)]),
    "qops_run_plan": (_I32, [_VP, _VP]),
    "qops_plan_update": (_I32, [_VP, ctypes.POINTER(Gate), _SZ]),
    "qops_apply": (_I32, [_VP, ctypes.POINTER(Gate), _SZ, ctypes.POINTER(PlanOpts)]),
    "qops_profile_run": (_I32, [_VP, _VP, ctypes.POINTER(_VP)]),
    "qops_profile_num_passes": (_I32, [_VP, ctypes.POINTER(_SZ)]),
    "qops_profile_pass": (_I32, [_VP, _SZ, ctypes.POINTER(PassRecord)]),
    "qops_profile_counts": (_I32, [_VP, _IP, _IP]),
    "qops_profile_total": (_I32, [_VP, _DP, _IP]),
    "qops_profile_features": (_I32, [_VP, ctypes.POINTER(ctypes.c_float)]),
    "qops_profile_dump": (_I32, [_VP, ctypes.c_char_p]),
    "qops_profile_trace": (_I32, [_VP, ctypes.c_char_p]),
    "qops_profile_merge": (_I32, [_VP, _VP]),
    "qops_profile_free": (_I32, [_VP]),
    "qops_profile_create": (_I32, [_I32, ctypes.POINTER(_VP)]),
    "qops_profile_compact": (_I32, [_VP, ctypes.POINTER(_VP)]),
    "qops_profile_save": (_I32, [_VP, ctypes.c_char_p]),
    "qops_profile_load": (_I32, [ctypes.c_char_p, ctypes.POINTER(_VP)]),
    "qops_profile_predict_passes": (_I32, [_VP, ctypes.POINTER(PlanOpts), _DP]),
    "qops_plan_predict": (_I32, [_VP, ctypes.POINTER(PlanOpts), _DP]),
    "qops_mlp_num_params": (_I32, [ctypes.POINTER(_SZ)]),
    "qops_mlp_create": (_I32, [ctypes.POINTER(ctypes.c_float), _SZ, ctypes.POINTER(_VP)]),
    "qops_mlp_set_normalization": (_I32, [_VP, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "qops_mlp_get_params": (_I32, [_VP, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                   ctypes.POINTER(ctypes.c_float)]),
    "qops_mlp_grad": (_I32, [_VP, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), _I32,
                             ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "qops_mlp_train": (_I32, [_VP, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), _I32, _I32, _I32,
                              ctypes.c_float, _U64, ctypes.POINTER(ctypes.c_float)]),
    "qops_mlp_predict": (_I32, [_VP, ctypes.POINTER(ctypes.c_float), _I32, ctypes.POINTER(ctypes.c_float)]),
    "qops_model_save": (_I32, [_VP, ctypes.c_char_p]),
    "qops_model_load": (_I32, [ctypes.c_char_p, ctypes.POINTER(_VP)]),
    "qops_model_free": (_I32, [_VP]),
    "qops_batch_create": (_I32, [ctypes.POINTER(BatchDesc), ctypes.POINTER(_VP)]),
    "qops_batch_launch": (_I32, [_VP]),
    "qops_batch_results": (_I32, [_VP, _DP]),
    "qops_batch_time": (_I32, [_VP, _I32, _DP]),
    "qops_batch_update": (_I32, [_VP, ctypes.POINTER(ctypes.POINTER(Gate)), ctypes.POINTER(ctypes.c_size_t)]),
    "qops_batch_info": (_I32, [_VP, ctypes.POINTER(BatchStats)]),
    "qops_batch_free": (_I32, [_VP]),
    "qops_batch_autotune": (_I32, [ctypes.POINTER(BatchDesc), ctypes.c_char_p, _IP, _IP, _IP, _DP]),
    "qops_tier_opts_default": (_I32, [ctypes.POINTER(TierOpts)]),
    "qops_tier_create": (_I32, [_I32, _I32, _I32, _I32, _VP, _SZ, _VP, ctypes.POINTER(_VP)]),
    "qops_tier_destroy": (_I32, [_VP]),
    "qops_tier_segment_pointer": (_I32, [_VP, _I32, ctypes.POINTER(_VP), ctypes.POINTER(_SZ)]),
    "qops_tier_init_basis": (_I32, [_VP, _U64]),
    "qops_tier_run": (_I32, [_VP, ctypes.POINTER(Gate), _SZ, ctypes.POINTER(TierOpts), ctypes.POINTER(TierStats)]),
    "qops_tier_plan": (_I32, [_I32, _I32, _I32, _IP, ctypes.POINTER(Gate), _SZ, _I32, ctypes.POINTER(TierStats), _IP]),
    "qops_tier_get_layout": (_I32, [_VP, _IP]),
    "qops_tier_expect_z": (_I32, [_VP, _DP]),
    "qops_tier_read_state": (_I32, [_VP, _VP, _I32]),
    "qops_swap": (_I32, [_VP, _I32, _I32, _I32]),
    "qops_get_layout": (_I32, [_VP, _IP]),
    "qops_set_layout": (_I32, [_VP, _IP]),
    "qops_read_state": (_I32, [_VP, _VP, _I32]),
    "qops_norm": (_I32, [_VP, _DP]),
    "qops_probabilities": (_I32, [_VP, _IP, _I32, _DP]),
    "qops_expect_z": (_I32, [_VP, _DP]),
    "qops_expect_zz": (_I32, [_VP, _IP, _I32, _DP]),
    "qops_expect_z_noalloc": (_I32, [_VP, _VP]),
    "qops_synchronize": (_I32, [_VP]),
}


def lib():
    """Loads libqops.so; raises if it has not been built (there is no
    fallback implementation)."""
    global _lib
    if _lib is None:
        # PyTorch provides the device memory and streams; loading it first makes
        # the library bind to the same HIP runtime instance (same SONAME).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libqops.so not found at {LIB_PATH}; build it with "
                              f"`python -m paper_2410_09326_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def register(name: str, restype, argtypes) -> None:
    """Declares an additional entry point (used by submodules)."""
    SIGNATURES[name] = (restype, argtypes)
    if _lib is not None:
        f = getattr(_lib, name)
        f.restype = restype
        f.argtypes = argtypes


def check(rc: int) -> None:
    if rc != 0:
        msg = lib().qops_last_error()
        raise QopsError(rc, msg.decode() if msg else "")


# ---------------------------------------------------------------------------
# Gate marshalling
# ---------------------------------------------------------------------------

class GateArray:
    """A gate list laid out as qops_gate structs.  Accepts objects with
    attributes kind/qubits/controls/params/matrix, or tuples
    (kind, qubits[, params[, controls[, matrix]]])."""

    def __init__(self, gates: Iterable) -> None:
        gl = list(gates)
        self.n = len(gl)
        self.arr = (Gate * max(1, self.n))()
        self._mats: List[np.ndarray] = []
        for i, g in enumerate(gl):
            if isinstance(g, tuple):
                kind = g[0]
                qubits = g[1]
                params = g[2] if len(g) > 2 else ()
                controls = g[3] if len(g) > 3 else ()
                matrix = g[4] if len(g) > 4 else None
            else:
                kind, qubits, params, controls, matrix = g.kind, g.qubits, g.params, g.controls, g.matrix
            s = self.arr[i]
            s.kind = KIND_ID[kind]
            s.k = len(qubits)
            s.n_ctrl = len(controls)
            if len(qubits) > 6 or len(controls) > 4:
                raise QopsError(-4, f"gate {i}: too many qubits")
            for j, q in enumerate(qubits):
                s.q[j] = int(q)
            for j, c in enumerate(controls):
                s.ctrl[j] = int(c)
            for j, v in enumerate(params):
                s.param[j] = float(v)
            if kind == "dense":
                m = np.ascontiguousarray(np.asarray(matrix, dtype=np.complex128)).view(np.float64).ravel().copy()
                self._mats.append(m)
                s.mat = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def ptr(self):
        return ctypes.cast(self.arr, ctypes.POINTER(Gate))


def plan_opts_from(**opts) -> PlanOpts:
    return plan_opts(**opts)


def plan_opts(mode: int = PLAN_FUSED, swap_mode: int = SWAP_VIRTUAL, tile_upper: int = 0, max_fuse_k: int = 0,
              use_mfma: int = 1, check_unitary: int = 0, remap: int = 0, profile=None, model=None,
              fold_rotations: int = 0, merge_blocks: int = 0) -> PlanOpts:
    o = PlanOpts()
    check(lib().qops_plan_opts_default(ctypes.byref(o)))
    o.mode, o.swap_mode, o.tile_upper = mode, swap_mode, tile_upper
    o.max_fuse_k, o.use_mfma, o.check_unitary, o.remap = max_fuse_k, use_mfma, check_unitary, remap
    o.profile = profile.handle if profile is not None else None
    o.model = model.handle if model is not None else None
    o.fold_rotations = fold_rotations
    o.merge_blocks = merge_blocks
    return o


# ---------------------------------------------------------------------------
# Plans
# ---------------------------------------------------------------------------

class Plan:
    def __init__(self, n: int, gates, precision: int = C64, l2p: Optional[Sequence[int]] = None, **opts) -> None:
        self.n = n
        self.precision = precision
        self._gates = gates if isinstance(gates, GateArray) else GateArray(gates)
        self._opts = plan_opts(**opts)
        h = ctypes.c_void_p()
        l2p_arr = (ctypes.c_int32 * n)(*l2p) if l2p is not None else None
        check(lib().qops_plan_build(n, precision, l2p_arr, self._gates.ptr(), self._gates.n,
                                    ctypes.byref(self._opts), ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().qops_plan_free(self.handle)
                self.handle = None
        except Exception:
            pass

    def stats(self) -> dict:
        s = PlanStats()
        check(lib().qops_plan_stats_get(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in PlanStats._fields_}

    def final_layout(self) -> np.ndarray:
        out = (ctypes.c_int32 * self.n)()
        check(lib().qops_plan_final_layout(self.handle, out))
        return np.array(out[:], dtype=np.int32)

    def ops(self) -> List[dict]:
        n = ctypes.c_size_t()
        check(lib().qops_plan_num_ops(self.handle, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            info = OpInfo()
            buf = np.zeros(2 * 4 ** 6, dtype=np.float64)
            check(lib().qops_plan_op(self.handle, i, ctypes.byref(info), buf.ctypes.data_as(_DP)))
            k = info.k
            if info.kind == 1:
                m = buf[:2 * 2 ** k].view(np.complex128).copy()
            elif info.kind == 3:
                m = None
            else:
                m = buf[:2 * 4 ** k].view(np.complex128).reshape(2 ** k, 2 ** k).copy()
            out.append({"kind": info.kind, "k": k, "t": list(info.t[:k]), "cmask": int(info.cmask),
                        "pass": info.pass_, "n_merged": info.n_merged, "m": m})
        return out

    def passes(self) -> List[dict]:
        out = []
        i = 0
        while True:
            info = PassInfo()
            if lib().qops_plan_pass_info(self.handle, i, ctypes.byref(info)) != 0:
                break
            out.append({"type": info.type, "L": info.tile_bits, "upper": list(info.upper[:info.n_upper]),
                        "n_ops": info.n_ops, "n_remaps": info.n_remaps, "n_mfma": info.n_mfma,
                        "bytes_alg": info.bytes_alg, "flops": info.flops})
            i += 1
        return out

    def predict(self, **opts) -> float:
        v = ctypes.c_double()
        o = plan_opts(**opts)
        check(lib().qops_plan_predict(self.handle, ctypes.byref(o), ctypes.byref(v)))
        return v.value

    def update(self, gates) -> None:
        self._gates = gates if isinstance(gates, GateArray) else GateArray(gates)
        check(lib().qops_plan_update(self.handle, self._gates.ptr(), self._gates.n))


class Profile:
    """Result of a profiling run: per-pass device times (context records) and
    per-kind, per-qubit gate counters (counter records)."""

    def __init__(self, handle) -> None:
        self.handle = handle

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().qops_profile_free(self.handle)
                self.handle = None
        except Exception:
            pass

    def records(self) -> List[dict]:
        n = ctypes.c_size_t()
        check(lib().qops_profile_num_passes(self.handle, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            r = PassRecord()
            check(lib().qops_profile_pass(self.handle, i, ctypes.byref(r)))
            d = {f: getattr(r, f) for f, _ in PassRecord._fields_}
            d["pass"] = d.pop("pass_")
            out.append(d)
        return out

    def total(self):
        s = ctypes.c_double()
        n = ctypes.c_int32()
        check(lib().qops_profile_total(self.handle, ctypes.byref(s), ctypes.byref(n)))
        return s.value, n.value

    def counts(self):
        _, n = self.total()
        lc = np.zeros(len(KINDS) * n, dtype=np.int32)
        pc = np.zeros(len(KINDS) * n, dtype=np.int32)
        check(lib().qops_profile_counts(self.handle, lc.ctypes.data_as(_IP), pc.ctypes.data_as(_IP)))
        return lc.reshape(len(KINDS), n), pc.reshape(len(KINDS), n)

    def features(self) -> np.ndarray:
        n = ctypes.c_size_t()
        check(lib().qops_profile_num_passes(self.handle, ctypes.byref(n)))
        out = np.zeros((n.value, 64), dtype=np.float32)
        check(lib().qops_profile_features(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def dump(self, path: str) -> None:
        check(lib().qops_profile_dump(self.handle, path.encode()))

    def trace(self, path: str) -> None:
        """Chrome trace-event JSON of the passes and per-qubit gate counts."""
        check(lib().qops_profile_trace(self.handle, path.encode()))

    def merge(self, other: "Profile") -> None:
        check(lib().qops_profile_merge(self.handle, other.handle))

    @classmethod
    def empty(cls, n: int) -> "Profile":
        h = ctypes.c_void_p()
        check(lib().qops_profile_create(n, ctypes.byref(h)))
        return cls(h)

    def save(self, path: str) -> None:
        check(lib().qops_profile_save(self.handle, path.encode()))

    def compact(self) -> "Profile":
        """Per pass shape, the passes at five time percentiles: prices like
        this profile under the plain table."""
        h = ctypes.c_void_p()
        check(lib().qops_profile_compact(self.handle, ctypes.byref(h)))
        return Profile(h)

    @classmethod
    def load(cls, path: str) -> "Profile":
        h = ctypes.c_void_p()
        check(lib().qops_profile_load(path.encode(), ctypes.byref(h)))
        return cls(h)

    def predict_passes(self, **opts) -> np.ndarray:
        """Cost-model prediction (seconds) for every pass recorded here."""
        n = ctypes.c_size_t()
        check(lib().qops_profile_num_passes(self.handle, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.float64)
        o = plan_opts(**opts)
        check(lib().qops_profile_predict_passes(self.handle, ctypes.byref(o), out.ctypes.data_as(_DP)))
        return out


_FP = ctypes.POINTER(ctypes.c_float)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


class CostModel:
    """The learned pass-time model (64 -> 128 -> 128 -> 1 perceptron) whose
    training, gradients and predictions run in the library's GPU kernels."""

    NFEAT = 64

    def __init__(self, params: Optional[np.ndarray] = None, handle=None) -> None:
        if handle is not None:
            self.handle = handle
            return
        h = ctypes.c_void_p()
        if params is None:
            check(lib().qops_mlp_create(None, 0, ctypes.byref(h)))
        else:
            p = _f32(params)
            check(lib().qops_mlp_create(p.ctypes.data_as(_FP), p.size, ctypes.byref(h)))
        self.handle = h

    @staticmethod
    def num_params() -> int:
        n = ctypes.c_size_t()
        check(lib().qops_mlp_num_params(ctypes.byref(n)))
        return n.value

    @classmethod
    def load(cls, path: str) -> "CostModel":
        h = ctypes.c_void_p()
        check(lib().qops_model_load(path.encode(), ctypes.byref(h)))
        return cls(handle=h)

    def save(self, path: str) -> None:
        check(lib().qops_model_save(self.handle, path.encode()))

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().qops_model_free(self.handle)
                self.handle = None
        except Exception:
            pass

    def set_normalization(self, mu, sd) -> None:
        m, s = _f32(mu), _f32(sd)
        check(lib().qops_mlp_set_normalization(self.handle, m.ctypes.data_as(_FP), s.ctypes.data_as(_FP)))

    def params(self):
        p = np.zeros(self.num_params(), dtype=np.float32)
        mu = np.zeros(self.NFEAT, dtype=np.float32)
        sd = np.zeros(self.NFEAT, dtype=np.float32)
        check(lib().qops_mlp_get_params(self.handle, p.ctypes.data_as(_FP), mu.ctypes.data_as(_FP),
                                        sd.ctypes.data_as(_FP)))
        return p, mu, sd

    def grad(self, X, t):
        X, t = _f32(X), _f32(t)
        g = np.zeros(self.num_params(), dtype=np.float32)
        loss = ctypes.c_float()
        check(lib().qops_mlp_grad(self.handle, X.ctypes.data_as(_FP), t.ctypes.data_as(_FP), len(t),
                                  g.ctypes.data_as(_FP), ctypes.byref(loss)))
        return float(loss.value), g

    def train(self, X, t, epochs: int = 20, batch: int = 256, lr: float = 1e-3, seed: int = 0) -> float:
        X, t = _f32(X), _f32(t)
        loss = ctypes.c_float()
        check(lib().qops_mlp_train(self.handle, X.ctypes.data_as(_FP), t.ctypes.data_as(_FP), len(t), epochs, batch,
                                   float(lr), int(seed), ctypes.byref(loss)))
        return float(loss.value)

    def predict(self, X) -> np.ndarray:
        X = _f32(X)
        out = np.zeros(X.shape[0], dtype=np.float32)
        check(lib().qops_mlp_predict(self.handle, X.ctypes.data_as(_FP), X.shape[0], out.ctypes.data_as(_FP)))
        return out


class Batch:
    """Many circuits (each given as (n, gates)) simulated from |0..0> in one
    graph launch; results are <Z_q> per circuit."""

    def __init__(self, circuits, precision: int = C64, small_max_n: int = 0, tile_bits: int = 0,
                 max_fuse_k: int = 0) -> None:
        self.ns = [int(n) for n, _ in circuits]
        self._desc, self._keep = self._describe(circuits, precision, small_max_n, tile_bits, max_fuse_k)
        h = ctypes.c_void_p()
        check(lib().qops_batch_create(ctypes.byref(self._desc), ctypes.byref(h)))
        self.handle = h

    @staticmethod
    def _describe(circuits, precision, small_max_n, tile_bits, max_fuse_k=0):
        arrays = [g if isinstance(g, GateArray) else GateArray(g) for _, g in circuits]
        cnt = len(arrays)
        ns = (ctypes.c_int32 * cnt)(*[int(n) for n, _ in circuits])
        gp = (ctypes.POINTER(Gate) * cnt)(*[a.ptr() for a in arrays])
        ng = (ctypes.c_size_t * cnt)(*[a.n for a in arrays])
        d = BatchDesc(cnt, ns, gp, ng, precision, None, small_max_n, tile_bits, max_fuse_k)
        return d, (arrays, ns, gp, ng)

    @staticmethod
    def autotune(circuits, precision: int = C64, cache: Optional[str] = None):
        d, keep = Batch._describe(circuits, precision, 0, 0)
        sm, tb, kf, sec = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        check(lib().qops_batch_autotune(ctypes.byref(d), cache.encode() if cache else None, ctypes.byref(sm),
                                        ctypes.byref(tb), ctypes.byref(kf), ctypes.byref(sec)))
        return sm.value, tb.value, kf.value, sec.value

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().qops_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def launch(self) -> None:
        check(lib().qops_batch_launch(self.handle))

    def results(self) -> List[np.ndarray]:
        out = np.zeros(sum(self.ns), dtype=np.float64)
        check(lib().qops_batch_results(self.handle, out.ctypes.data_as(_DP)))
        res, o = [], 0
        for n in self.ns:
            res.append(out[o:o + n].copy())
            o += n
        return res

    def time(self, reps: int = 5) -> float:
        v = ctypes.c_double()
        check(lib().qops_batch_time(self.handle, reps, ctypes.byref(v)))
        return v.value

    def update(self, gate_lists) -> None:
        arrays = [g if isinstance(g, GateArray) else GateArray(g) for g in gate_lists]
        cnt = len(arrays)
        gp = (ctypes.POINTER(Gate) * cnt)(*[a.ptr() for a in arrays])
        ng = (ctypes.c_size_t * cnt)(*[a.n for a in arrays])
        check(lib().qops_batch_update(self.handle, gp, ng))
        self._upd = (arrays, gp, ng)

    def info(self) -> dict:
        s = BatchStats()
        check(lib().qops_batch_info(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in BatchStats._fields_}


# ---------------------------------------------------------------------------
# Simulator handle
# ---------------------------------------------------------------------------

class Simulator:
    """A 2^n-amplitude state on the GPU.  The state buffer is a torch tensor
    (device memory) that the library borrows; work goes on torch's current
    stream unless `stream` is given."""

    def __init__(self, n: int, precision: int = C64, device: str = "cuda:0", stream=None, buffer=None) -> None:
        import torch
        self.n = n
        self.precision = precision
        amp = 8 if precision == C64 else 16
        if buffer is None:
            buffer = torch.empty((2 ** n) * amp // 4, dtype=torch.float32, device=device)
        self.buffer = buffer
        if stream is None:
            stream = torch.cuda.current_stream(buffer.device)
        self.stream = stream
        h = ctypes.c_void_p()
        check(lib().qops_create(n, precision, ctypes.c_void_p(buffer.data_ptr()),
                                buffer.numel() * buffer.element_size(), ctypes.c_void_p(stream.cuda_stream),
                                ctypes.byref(h)))
        self.handle = h

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().qops_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch_limit(self, max_workgroups: int) -> None:
        """Caps the work-groups of every state pass (0 = the kernels' own)."""
        check(lib().qops_set_launch_limit(self.handle, int(max_workgroups)))

    def init_basis(self, x: int = 0) -> None:
        check(lib().qops_init_basis(self.handle, int(x)))

    def init_amplitudes(self, psi: np.ndarray) -> None:
        dt = np.complex64 if self.precision == C64 else np.complex128
        a = np.ascontiguousarray(psi, dtype=dt)
        assert a.size == 2 ** self.n
        check(lib().qops_init_amplitudes(self.handle, a.ctypes.data_as(ctypes.c_void_p)))

    def apply(self, gates, **opts) -> None:
        ga = gates if isinstance(gates, GateArray) else GateArray(gates)
        o = plan_opts(**opts)
        check(lib().qops_apply(self.handle, ga.ptr(), ga.n, ctypes.byref(o)))

    def run(self, plan: Plan) -> None:
        check(lib().qops_run_plan(self.handle, plan.handle))

    def profile(self, plan: Plan) -> Profile:
        """Runs `plan` with per-pass HIP-event timing and gate counters."""
        h = ctypes.c_void_p()
        check(lib().qops_profile_run(self.handle, plan.handle, ctypes.byref(h)))
        return Profile(h)

    def swap(self, a: int, b: int, mode: int = SWAP_VIRTUAL) -> None:
        check(lib().qops_swap(self.handle, a, b, mode))

    def layout(self) -> np.ndarray:
        out = (ctypes.c_int32 * self.n)()
        check(lib().qops_get_layout(self.handle, out))
        return np.array(out[:], dtype=np.int32)

    def set_layout(self, l2p: Sequence[int]) -> None:
        arr = (ctypes.c_int32 * self.n)(*[int(v) for v in l2p])
        check(lib().qops_set_layout(self.handle, arr))

    def state(self, order: int = ORDER_LOGICAL) -> np.ndarray:
        dt = np.complex64 if self.precision == C64 else np.complex128
        out = np.empty(2 ** self.n, dtype=dt)
        check(lib().qops_read_state(self.handle, out.ctypes.data_as(ctypes.c_void_p), order))
        return out

    def norm(self) -> float:
        v = ctypes.c_double()
        check(lib().qops_norm(self.handle, ctypes.byref(v)))
        return v.value

    def probabilities(self, qubits: Sequence[int]) -> np.ndarray:
        m = len(qubits)
        q = (ctypes.c_int32 * m)(*[int(v) for v in qubits])
        out = np.empty(2 ** m, dtype=np.float64)
        check(lib().qops_probabilities(self.handle, q, m, out.ctypes.data_as(_DP)))
        return out

    def expect_z(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float64)
        check(lib().qops_expect_z(self.handle, out.ctypes.data_as(_DP)))
        return out

    def expect_z_noalloc(self, out) -> None:
        """<Z_q> into `out`, a float64 device tensor of n entries, on the
        handle's stream, without allocating (asynchronous)."""
        import torch
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < self.n or not out.is_contiguous():
            raise QopsError(-1, "out must be a contiguous float64 device tensor of n entries")
        check(lib().qops_expect_z_noalloc(self.handle, ctypes.c_void_p(out.data_ptr())))

    def expect_zz(self, pairs) -> np.ndarray:
        """<Z_a Z_b> for every pair (a, b) of logical qubits."""
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        out = np.zeros(len(pr), dtype=np.float64)
        check(lib().qops_expect_zz(self.handle, pr.ctypes.data_as(_IP), len(pr), out.ctypes.data_as(_DP)))
        return out

    def synchronize(self) -> None:
        check(lib().qops_synchronize(self.handle))


# ---------------------------------------------------------------------------
# Host-memory state tier
# ---------------------------------------------------------------------------

def _tier_stats(st: TierStats) -> dict:
    return {f: getattr(st, f) for f, _ in TierStats._fields_ if f != "reserved"}


def tier_plan(n: int, gates, global_bits: int, max_active: int = 1, remap: int = 1,
              l2p: Optional[Sequence[int]] = None):
    """Host-only staging of a gate list on a tiered state (no GPU): the
    stages, groups and exchanges a run would use, and the final layout."""
    ga = gates if isinstance(gates, GateArray) else GateArray(gates)
    st = TierStats()
    out = (ctypes.c_int32 * n)()
    l2p_arr = (ctypes.c_int32 * n)(*l2p) if l2p is not None else None
    check(lib().qops_tier_plan(n, global_bits, max_active, l2p_arr, ga.ptr(), ga.n, remap, ctypes.byref(st), out))
    return _tier_stats(st), np.array(out[:], dtype=np.int32)


class TieredSimulator:
    """A 2^n-amplitude state in pinned host memory whose top `global_bits`
    physical bits select segments; runs stream it through the device in
    stages (at most `max_active` segment bits active per device group)."""

    def __init__(self, n: int, precision: int = C64, global_bits: int = 2, max_active: int = 1, stream=None) -> None:
        import torch
        self.n = n
        self.precision = precision
        self.global_bits = global_bits
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        check(lib().qops_tier_create(n, precision, global_bits, max_active, None, 0,
                                     ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().qops_tier_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_basis(self, x: int = 0) -> None:
        check(lib().qops_tier_init_basis(self.handle, int(x)))

    def run(self, gates, remap: int = 1, **plan_opts) -> dict:
        ga = gates if isinstance(gates, GateArray) else GateArray(gates)
        o = TierOpts()
        check(lib().qops_tier_opts_default(ctypes.byref(o)))
        o.remap = remap
        o.plan = plan_opts_from(**plan_opts)
        st = TierStats()
        check(lib().qops_tier_run(self.handle, ga.ptr(), ga.n, ctypes.byref(o), ctypes.byref(st)))
        return _tier_stats(st)

    def layout(self) -> np.ndarray:
        out = (ctypes.c_int32 * self.n)()
        check(lib().qops_tier_get_layout(self.handle, out))
        return np.array(out[:], dtype=np.int32)

    def expect_z(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float64)
        check(lib().qops_tier_expect_z(self.handle, out.ctypes.data_as(_DP)))
        return out

    def state(self, order: int = ORDER_LOGICAL) -> np.ndarray:
        dt = np.complex64 if self.precision == C64 else np.complex128
        out = np.empty(2 ** self.n, dtype=dt)
        check(lib().qops_tier_read_state(self.handle, out.ctypes.data_as(ctypes.c_void_p), order))
        return out

    def segment_view(self, s: int) -> np.ndarray:
        """Segment s of the pinned host state (physical amplitudes
        s * 2^(n-g) onwards, no copy); valid until close()."""
        p = ctypes.c_void_p()
        nb = ctypes.c_size_t()
        check(lib().qops_tier_segment_pointer(self.handle, int(s), ctypes.byref(p), ctypes.byref(nb)))
        dt = np.complex64 if self.precision == C64 else np.complex128
        buf = (ctypes.c_char * nb.value).from_address(p.value)
        return np.frombuffer(buf, dtype=dt)
