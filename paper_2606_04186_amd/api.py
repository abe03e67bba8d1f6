"""ctypes binding of libqflow (argument marshalling only).

Device arrays are torch tensors on a ROCm device (float64 / int32,
contiguous); their data pointers are handed to the library unchanged.  Host
arrays are numpy arrays.  Every function mirrors one entry point of
include/qflow.h and raises QFlowError on a non-zero status.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqflow.so")

FP64, FP32, BF16X3 = 0, 1, 2
UNOWNED_FROZEN = 1 << 4
GRAPH = 1 << 5
DIIS = 1 << 6
SOLVER_VQE = 1 << 7
TRUNC_F, TRUNC_H = 0, 1   # qflow_set_truncation
Z_AUTO, Z_SPACE, Z_DENSE = 0, 1, 2   # qflow_z_mode
STATIC_SCRATCH_BYTES = 128 * 1024 * 1024   # QFLOW_STATIC_SCRATCH_BYTES

SPACE_DTYPE = np.dtype([("n_o", "<i4"), ("n_v", "<i4"), ("orb", "<i4", (8,))])
DAV_PER_CLASS, DAV_PERSISTENT = 0, 1   # qflow_tuning.davidson


class Tuning(ctypes.Structure):
    """qflow_tuning: the context's launch choices."""
    _fields_ = [("davidson", ctypes.c_int32), ("split_target", ctypes.c_int32),
                ("f64_tile", ctypes.c_int32), ("z_mode", ctypes.c_int32),
                ("block_44", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}

_STATUS = {
    0: "QFLOW_OK", -1: "QFLOW_E_INVALID_ARG", -2: "QFLOW_E_SYMMETRY", -3: "QFLOW_E_OOM",
    -4: "QFLOW_E_DEVICE", -5: "QFLOW_E_NOT_CONVERGED", -6: "QFLOW_E_REF_WEIGHT",
    -7: "QFLOW_E_STATE", -8: "QFLOW_E_UNSUPPORTED",
}

_lib = None


class QFlowError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")


def lib() -> ctypes.CDLL:
    """Load libqflow.so from the package directory (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2606_04186_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "qflow_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, vp]),
            "qflow_destroy": (ctypes.c_int, [vp]),
            "qflow_last_error": (ctypes.c_char_p, [vp]),
            "qflow_load_integrals": (ctypes.c_int, [vp, i32, i32, vp, vp, d]),
            "qflow_reference": (ctypes.c_int, [vp, vp, vp, vp]),
            "qflow_mp2_guess": (ctypes.c_int, [vp, vp, vp]),
            "qflow_residual": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, ctypes.c_int]),
            "qflow_heff_size": (i64, [vp]),
            "qflow_amp_size": (i64, [vp]),
            "qflow_ci_size": (i64, [vp]),
            "qflow_build_heff": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, ctypes.c_int]),
            "qflow_solve_active_batch": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, vp,
                                                        vp, vp, vp, vp, d, i32]),
            "qflow_solve_active_batch_static": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp,
                                                               vp, vp, vp, vp, vp, vp, d,
                                                               i32]),
            "qflow_solve_vqe_batch": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp,
                                                     vp, d, i32]),
            "qflow_set_vqe": (ctypes.c_int, [vp, d, i32]),
            "qflow_set_truncation": (ctypes.c_int, [vp, ctypes.c_int]),
            "qflow_flow_step": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, i32]),
            "qflow_flow_sweep_windowed": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, i32, vp,
                                                         vp, i32]),
            "qflow_last_timings": (ctypes.c_int, [vp, vp, ctypes.c_int]),
            "qflow_set_z_mode": (ctypes.c_int, [vp, ctypes.c_int]),
            "qflow_set_solver": (ctypes.c_int, [vp, d, i32]),
            "qflow_last_solve": (ctypes.c_int, [vp, i32, vp, vp]),
            "qflow_set_tuning": (ctypes.c_int, [vp, vp]),
            "qflow_get_tuning": (ctypes.c_int, [vp, vp]),
            "qflow_autotune": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, i32, ctypes.c_char_p,
                                              vp, vp, i32]),
            "qflow_sample_spaces": (ctypes.c_int, [i32, i32, i32, i32, vp, vp, i64, i32, vp, vp,
                                                   i32, vp, vp]),
            "qflow_build_owners": (ctypes.c_int, [i32, i32, i32, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(x):
    """Device pointer of a torch tensor, or host pointer of a numpy array."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        assert x.flags["C_CONTIGUOUS"]
        return x.ctypes.data
    assert x.is_contiguous(), "tensors passed to libqflow must be contiguous"
    return x.data_ptr()


def _spaces(spaces) -> np.ndarray:
    s = np.ascontiguousarray(spaces, dtype=SPACE_DTYPE)
    return s


def make_spaces(lists) -> np.ndarray:
    """[(occ tuple, vir tuple), ...] -> structured array of qflow_space."""
    out = np.zeros(len(lists), dtype=SPACE_DTYPE)
    for k, (occ, vir) in enumerate(lists):
        out[k]["n_o"] = len(occ)
        out[k]["n_v"] = len(vir)
        orb = list(occ) + list(vir)
        out[k]["orb"][: len(orb)] = orb
    return out


def heff_size(space) -> int:
    return int(lib().qflow_heff_size(_ptr(np.ascontiguousarray(space, dtype=SPACE_DTYPE))))


def amp_size(space) -> int:
    return int(lib().qflow_amp_size(_ptr(np.ascontiguousarray(space, dtype=SPACE_DTYPE))))


def ci_size(space) -> int:
    return int(lib().qflow_ci_size(_ptr(np.ascontiguousarray(space, dtype=SPACE_DTYPE))))


def offsets(spaces, size_fn) -> np.ndarray:
    sizes = [size_fn(s) for s in spaces]
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


class Context:
    """One libqflow context bound to a device and a HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        L = lib()
        h = ctypes.c_void_p()
        st = None
        if stream is not None:
            st = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self._check(L.qflow_create(ctypes.byref(h), device, st), None)
        self.h = h
        self.n = self.o = self.v = 0

    def close(self):
        if getattr(self, "h", None):
            lib().qflow_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code, h="self"):
        if code != 0:
            msg = ""
            hh = self.h if h == "self" else h
            if hh:
                msg = lib().qflow_last_error(hh).decode()
            raise QFlowError(code, msg)

    def load_integrals(self, h, eri, n_occ, sym_tol=1e-12):
        """h [n,n] and chemist eri [n,n,n,n]: float64 device tensors."""
        n = h.shape[0]
        self._check(lib().qflow_load_integrals(self.h, n, int(n_occ), _ptr(h), _ptr(eri),
                                               sym_tol))
        self.n, self.o, self.v = n, int(n_occ), n - int(n_occ)

    def reference(self):
        e = ctypes.c_double()
        eps = np.zeros(self.n)
        f = np.zeros((self.n, self.n))
        self._check(lib().qflow_reference(self.h, ctypes.byref(e), _ptr(eps), _ptr(f)))
        return e.value, eps, f

    def mp2_guess(self, t1, t2):
        self._check(lib().qflow_mp2_guess(self.h, _ptr(t1), _ptr(t2)))

    def residual(self, t1, t2, r1, r2, e0, precision=FP64):
        self._check(lib().qflow_residual(self.h, _ptr(t1), _ptr(t2), _ptr(r1), _ptr(r2),
                                         _ptr(e0), precision))

    def build_heff(self, spaces, t1, t2, heff, heff_off, precision=FP64):
        sp = _spaces(spaces)
        self._check(lib().qflow_build_heff(self.h, len(sp), _ptr(sp), _ptr(t1), _ptr(t2),
                                           _ptr(heff), _ptr(heff_off), precision))

    def solve_active_batch(self, spaces, heff, heff_off, energy, c0, amp, amp_off, iters,
                           status, tol=1e-10, max_iter=200, ci=None, ci_off=None):
        """ci / ci_off (optional): start vectors in, eigenvectors out."""
        sp = _spaces(spaces)
        self._check(lib().qflow_solve_active_batch(
            self.h, len(sp), _ptr(sp), _ptr(heff), _ptr(heff_off), _ptr(energy), _ptr(c0),
            _ptr(amp), _ptr(amp_off), _ptr(ci), _ptr(ci_off), _ptr(iters), _ptr(status), tol,
            max_iter))

    def solve_active_batch_static(self, spaces, heff, heff_off, energy, c0, amp, amp_off,
                                  iters, status, tol=1e-10, max_iter=200, ci=None,
                                  ci_off=None):
        """solve_active_batch without device allocation (work memory in the
        library's static scratch of STATIC_SCRATCH_BYTES per device)."""
        sp = _spaces(spaces)
        self._check(lib().qflow_solve_active_batch_static(
            self.h, len(sp), _ptr(sp), _ptr(heff), _ptr(heff_off), _ptr(energy), _ptr(c0),
            _ptr(amp), _ptr(amp_off), _ptr(ci), _ptr(ci_off), _ptr(iters), _ptr(status), tol,
            max_iter))

    def solve_vqe_batch(self, spaces, heff, heff_off, theta0, amp, amp_off, energy, iters,
                        status, gtol=1e-10, max_iter=500):
        """UCCSD-VQE solve of every space from the parameters theta0 (amp
        layout); optimised parameters into amp (may be theta0)."""
        sp = _spaces(spaces)
        self._check(lib().qflow_solve_vqe_batch(
            self.h, len(sp), _ptr(sp), _ptr(heff), _ptr(heff_off), _ptr(theta0), _ptr(amp),
            _ptr(amp_off), _ptr(energy), _ptr(iters), _ptr(status), float(gtol), int(max_iter)))

    def set_truncation(self, truncation):
        """TRUNC_F (DUCC(2F), the default) or TRUNC_H (adds 1/2 [[V_N, s]_2, s]_2)."""
        self._check(lib().qflow_set_truncation(self.h, int(truncation)))

    def set_vqe(self, gtol=1e-10, max_iter=500):
        """Stopping rule of the flow steps' VQE solves (SOLVER_VQE)."""
        self._check(lib().qflow_set_vqe(self.h, float(gtol), int(max_iter)))

    def flow_step(self, spaces, owner1, owner2, t1, t2, energy, flags=FP64):
        sp = _spaces(spaces)
        em, md = ctypes.c_double(), ctypes.c_double()
        self._check(lib().qflow_flow_step(self.h, len(sp), _ptr(sp), _ptr(owner1), _ptr(owner2),
                                          _ptr(t1), _ptr(t2), _ptr(energy), ctypes.byref(em),
                                          ctypes.byref(md), flags))
        return em.value, md.value

    def flow_sweep_windowed(self, spaces, owner1, owner2, t1, t2, energy, window, flags=FP64):
        """One windowed Gauss-Seidel sweep; returns (e_mean, max_dt)."""
        sp = _spaces(spaces)
        em, md = ctypes.c_double(), ctypes.c_double()
        self._check(lib().qflow_flow_sweep_windowed(
            self.h, len(sp), _ptr(sp), _ptr(owner1), _ptr(owner2), _ptr(t1), _ptr(t2),
            _ptr(energy), int(window), ctypes.byref(em), ctypes.byref(md), flags))
        return em.value, md.value

    def set_z_mode(self, mode):
        """How build_heff forms the sigma1 x two-body terms: Z_AUTO, Z_SPACE
        or Z_DENSE (module constants)."""
        self._check(lib().qflow_set_z_mode(self.h, int(mode)))

    def set_tuning(self, davidson=None, split_target=None, f64_tile=None, z_mode=None,
                   block_44=None):
        """Change some of the launch choices (None keeps the current value)."""
        t = self.get_tuning()
        for name, val in (("davidson", davidson), ("split_target", split_target),
                          ("f64_tile", f64_tile), ("z_mode", z_mode), ("block_44", block_44)):
            if val is not None:
                setattr(t, name, int(val))
        self._check(lib().qflow_set_tuning(self.h, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        self._check(lib().qflow_get_tuning(self.h, ctypes.byref(t)))
        return t

    def autotune(self, spaces, owner1, owner2, t1, t2, flags=FP64, cache_path=None):
        """Choose and apply the launch choices by timing flow steps; returns
        (Tuning, report text).  t1, t2 are read, not changed."""
        sp = _spaces(spaces)
        t = Tuning()
        rep = ctypes.create_string_buffer(8192)
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(lib().qflow_autotune(self.h, len(sp), _ptr(sp), _ptr(owner1), _ptr(owner2),
                                         _ptr(t1), _ptr(t2), int(flags), path, ctypes.byref(t),
                                         rep, len(rep)))
        return t, rep.value.decode()

    def last_solve(self, K):
        """(iters, status) of the last flow step's eigensolves, numpy int32."""
        it = np.zeros(K, dtype=np.int32)
        st = np.zeros(K, dtype=np.int32)
        self._check(lib().qflow_last_solve(self.h, int(K), _ptr(it), _ptr(st)))
        return it, st

    def set_solver(self, tol=1e-10, max_iter=200):
        """Stopping rule of the flow steps' eigensolves."""
        self._check(lib().qflow_set_solver(self.h, float(tol), int(max_iter)))

    STAGES = ("yg", "ladder_h", "ladder_yg", "ring_pack", "ring_gemm", "ring_j", "sigma1_x",
              "residual", "heff", "solve", "update", "total")

    def last_timings(self):
        """Device milliseconds of the last flow_step per stage and in total
        (STAGES order; stages are -1 for a graph replay)."""
        ms = np.zeros(len(self.STAGES), dtype=np.float32)
        c = lib().qflow_last_timings(self.h, _ptr(ms), len(self.STAGES))
        return dict(zip(self.STAGES, ms[:c].tolist()))


def sample_spaces(No, Nv, no, nv, eps, uniforms, cap=0, max_out=None):
    """Algorithm 1 on the host library; returns (spaces, delta_eps, used)."""
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    if max_out is None:
        max_out = cap if cap > 0 else len(u)
    out = np.zeros(max_out, dtype=SPACE_DTYPE)
    de = np.zeros(max_out)
    K = ctypes.c_int32()
    used = ctypes.c_int64()
    code = lib().qflow_sample_spaces(No, Nv, no, nv, _ptr(eps), _ptr(u), len(u), cap, _ptr(out),
                                     _ptr(de), max_out, ctypes.byref(K), ctypes.byref(used))
    if code != 0:
        raise QFlowError(code, "qflow_sample_spaces")
    return out[: K.value].copy(), de[: K.value].copy(), used.value


def build_owners(No, Nv, spaces):
    sp = _spaces(spaces)
    o1 = np.zeros((No, Nv), dtype=np.int32)
    o2 = np.zeros((No, No, Nv, Nv), dtype=np.int32)
    code = lib().qflow_build_owners(No, Nv, len(sp), _ptr(sp), _ptr(o1), _ptr(o2))
    if code != 0:
        raise QFlowError(code, "qflow_build_owners")
    return o1, o2
