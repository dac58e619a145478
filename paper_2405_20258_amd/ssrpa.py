"""Thin ctypes binding of libssrpa (the C ABI in include/ssrpa.h).

Argument marshalling only: every step of the computation runs inside the HIP
library.  Device buffers are passed as integer addresses (for example
``tensor.data_ptr()`` of a torch tensor on the GPU) and streams as HIP stream
handles (``torch.cuda.current_stream().cuda_stream``).  The functions keep the
C names; :class:`Context` and :class:`System` are small owners of the opaque
handles.  If the shared library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SSRPA_LIB", os.path.join(_HERE, "libssrpa.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} not found: build it with `python -c 'import "
        f"__graft_entry__ as g; g.build()'` (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

OK, ERR_ARG, ERR_ALIAS, ERR_NOMEM, ERR_HIP, ERR_NUMERIC, ERR_STATE = range(7)
FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}

_p = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_sz = ctypes.c_size_t
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i32p = ctypes.POINTER(ctypes.c_int32)


class ssrpa_system_desc(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_double * 9),
                ("fft", ctypes.c_int32 * 3),
                ("n_pw", ctypes.c_int32),
                ("miller", _i32p),
                ("n_v", ctypes.c_int32),
                ("n_c", ctypes.c_int32),
                ("coeff", _dp),
                ("coeff_on_device", ctypes.c_int32),
                ("energy", _dp),
                ("ecut_chi", ctypes.c_double),
                ("occupation", _dp),
                ("coulomb_truncation", ctypes.c_int32),
                ("real_orbitals", ctypes.c_int32)]
TRUNCATIONS = {None: 0, "slab": 1}


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


ssrpa_status_string = _sig("ssrpa_status_string", ctypes.c_char_p, [_i])
ssrpa_last_error = _sig("ssrpa_last_error", ctypes.c_char_p, [_p])
ssrpa_version = _sig("ssrpa_version", ctypes.c_char_p, [])
ssrpa_context_create = _sig("ssrpa_context_create", _i,
                            [_i, _sz, ctypes.POINTER(_p)])
ssrpa_context_destroy = _sig("ssrpa_context_destroy", _i, [_p])
ssrpa_context_memory = _sig("ssrpa_context_memory", _i,
                            [_p, ctypes.POINTER(_sz), ctypes.POINTER(_sz)])
ssrpa_footprint = _sig("ssrpa_footprint", _i,
                       [ctypes.POINTER(ssrpa_system_desc), _i, _i, _i, _i,
                        ctypes.POINTER(_sz)])
ssrpa_plan_valence_block = _sig("ssrpa_plan_valence_block", _i,
                                [ctypes.POINTER(ssrpa_system_desc), _i, _i, _i,
                                 _sz, _ip])
ssrpa_system_create = _sig("ssrpa_system_create", _i,
                           [_p, ctypes.POINTER(ssrpa_system_desc), _p,
                            ctypes.POINTER(_p)])
ssrpa_system_destroy = _sig("ssrpa_system_destroy", _i, [_p])
ssrpa_system_bands = _sig("ssrpa_system_bands", _i, [_p, _ip, _ip, _ip])
ssrpa_chi_gvectors = _sig("ssrpa_chi_gvectors", _i, [_p, _ip, _i32p])
ssrpa_orbitals_realspace = _sig("ssrpa_orbitals_realspace", _i, [_p, _p, _p])
ssrpa_pair_matrix = _sig("ssrpa_pair_matrix", _i, [_p, _i, _i, _i, _p, _p])
ssrpa_chi0_static = _sig("ssrpa_chi0_static", _i, [_p, _i, _i, _p, _i, _p])
ssrpa_subspace = _sig("ssrpa_subspace", _i, [_p, _i, _dp, _p, _p])
ssrpa_subspace_basis = _sig("ssrpa_subspace_basis", _i,
                            [_p, _i, _i, _dp, _p, _p])
BASES = {"symmetrized": 0, "chi0": 1}
ssrpa_epsilon_inverse = _sig("ssrpa_epsilon_inverse", _i,
                             [_p, _i, _i, _dp, _i, _i, _p, _p])
ssrpa_correlation_energy = _sig("ssrpa_correlation_energy", _i,
                                [_p, _i, _i, _dp, _dp, _i, _i, _d, _dp, _dp,
                                 _p, _p])
ssrpa_trace_log = _sig("ssrpa_trace_log", _i, [_p, _p, _i, _i, _d, _dp, _p])
ssrpa_trace_log_noalloc = _sig("ssrpa_trace_log_noalloc", _i,
                               [_p, _p, _i, _i, _d, _p, _p, _p])
ssrpa_device_copy = _sig("ssrpa_device_copy", _i, [_p, _p, _p, _sz, _p])
ssrpa_frequency_grid = _sig("ssrpa_frequency_grid", _i, [_i, _d, _dp, _dp])
ssrpa_stage_times = _sig("ssrpa_stage_times", _i, [_p, _i, _dp, _ip])
STAGES = ["pair_fft", "chi0_herk", "eigen", "projection", "freq_herk",
          "trace_log"]
ssrpa_correlation_energy_enqueue = _sig(
    "ssrpa_correlation_energy_enqueue", _i,
    [_p, _i, _i, _dp, _dp, _i, _i, _p, ctypes.POINTER(_p)])
ssrpa_ticket_query = _sig("ssrpa_ticket_query", _i, [_p, _ip])
ssrpa_ticket_wait = _sig("ssrpa_ticket_wait", _i, [_p, _dp, _dp])

ssrpa_server_create = _sig("ssrpa_server_create", _i,
                           [_p, _i, _d, ctypes.POINTER(_p)])
ssrpa_server_submit = _sig("ssrpa_server_submit", _i,
                           [_p, ctypes.POINTER(ssrpa_system_desc), _i, _i, _dp,
                            _dp, _i, ctypes.POINTER(ctypes.c_uint64)])
ssrpa_server_poll = _sig("ssrpa_server_poll", _i,
                         [_p, ctypes.c_uint64, _ip, _ip, _dp, _dp, _dp, _dp])
ssrpa_server_device_times = _sig("ssrpa_server_device_times", _i,
                                 [_p, ctypes.c_uint64, _dp, _dp])
ssrpa_server_error = _sig("ssrpa_server_error", ctypes.c_char_p,
                          [_p, ctypes.c_uint64])
ssrpa_server_drain = _sig("ssrpa_server_drain", _i, [_p])
ssrpa_server_memory = _sig("ssrpa_server_memory", _i,
                           [_p, ctypes.POINTER(_sz), ctypes.POINTER(_sz)])
ssrpa_server_destroy = _sig("ssrpa_server_destroy", _i, [_p])
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = range(4)

ssrpa_kmesh_create = _sig("ssrpa_kmesh_create", _i,
                          [_p, _i, ctypes.POINTER(ssrpa_system_desc), _dp, _dp,
                           _p, ctypes.POINTER(_p)])
ssrpa_kmesh_destroy = _sig("ssrpa_kmesh_destroy", _i, [_p])
ssrpa_kmesh_chi_gvectors = _sig("ssrpa_kmesh_chi_gvectors", _i,
                                [_p, _dp, _ip, _i32p])
ssrpa_kmesh_stage_times = _sig("ssrpa_kmesh_stage_times", _i,
                               [_p, _i, _dp, _ip])
ssrpa_kmesh_correlation_energy = _sig(
    "ssrpa_kmesh_correlation_energy", _i,
    [_p, _dp, _i32p, _i32p, _i, _i, _dp, _dp, _dp, _dp, _p, _p])

EXPORTED = [n for n in dir() if n.startswith("ssrpa_") and
            n != "ssrpa_system_desc"]


class SsrpaError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        msg = ssrpa_status_string(status).decode()
        super().__init__(f"{msg} ({status})" + (f": {detail}" if detail else ""))


def _check(status: int, ctx=None):
    if status != OK:
        detail = ssrpa_last_error(ctx).decode() if ctx else ""
        raise SsrpaError(status, detail)


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _addr(x) -> Optional[int]:
    """Device address of a torch tensor / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def frequency_grid(n: int, omega0: float = 1.0):
    om = np.empty(n)
    wt = np.empty(n)
    _check(ssrpa_frequency_grid(n, omega0, _dptr(om), _dptr(wt)))
    return om, wt


def make_desc(a, fft, miller, coeff, energy, n_v, ecut_chi, keep, occ=None,
              truncation=None, real=False):
    """ssrpa_system_desc from host arrays; `keep` holds the buffers alive.
    occ: occupation factors per band (None: insulator); truncation: None or
    "slab"."""
    lattice = np.asarray(a, dtype=np.float64)
    if lattice.ndim == 0:
        lattice = np.eye(3) * float(lattice)
    miller = np.ascontiguousarray(miller, dtype=np.int32)
    energy = np.ascontiguousarray(energy, dtype=np.float64)
    d = ssrpa_system_desc()
    for i, v in enumerate(lattice.reshape(9)):
        d.lattice[i] = float(v)
    for i in range(3):
        d.fft[i] = int(fft[i])
    d.n_pw = int(miller.shape[0])
    d.miller = miller.ctypes.data_as(_i32p)
    d.n_v = int(n_v)
    d.n_c = int(energy.shape[0] - n_v)
    if isinstance(coeff, np.ndarray):
        coeff = np.ascontiguousarray(coeff, dtype=np.complex128)
        d.coeff = ctypes.cast(coeff.ctypes.data, _dp)
        d.coeff_on_device = 0
    else:  # torch complex128 tensor on the device
        d.coeff = ctypes.cast(_addr(coeff), _dp)
        d.coeff_on_device = 1
    d.energy = energy.ctypes.data_as(_dp)
    d.ecut_chi = float(ecut_chi)
    if occ is not None:
        occ = np.ascontiguousarray(occ, dtype=np.float64)
        d.occupation = occ.ctypes.data_as(_dp)
    else:
        d.occupation = None
    d.coulomb_truncation = TRUNCATIONS[truncation]
    d.real_orbitals = 1 if real else 0
    keep.extend([miller, energy, coeff, occ])
    return d


class Context:
    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = _p()
        _check(ssrpa_context_create(device, hbm_budget, ctypes.byref(h)))
        self.handle = h
        self._systems = weakref.WeakSet()

    def close(self):
        """Destroy the context, closing its remaining systems first."""
        if self.handle:
            for s in list(self._systems):
                s.close()
            _check(ssrpa_context_destroy(self.handle), self.handle)
            self.handle = None

    def memory(self):
        a, b = _sz(), _sz()
        _check(ssrpa_context_memory(self.handle, ctypes.byref(a),
                                    ctypes.byref(b)), self.handle)
        return a.value, b.value

    def trace_log(self, x_dev, n: int, n_mat: int, coupling: float = 1.0,
                  stream=None):
        f = np.empty(n_mat)
        _check(ssrpa_trace_log(self.handle, _addr(x_dev), n, n_mat, coupling,
                               _dptr(f), _stream(stream)), self.handle)
        return f

    def device_copy(self, src_dev, dst_dev, nbytes: int, stream=None):
        """Plain 16-byte-wide device copy (reference dispatch for counters)."""
        _check(ssrpa_device_copy(self.handle, _addr(src_dev), _addr(dst_dev),
                                 nbytes, _stream(stream)), self.handle)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class System:
    """A resident system: orbitals on the device plus chi0 / subspace state."""

    def __init__(self, ctx: Context, a, fft, miller, coeff, energy, n_v,
                 ecut_chi, stream=None, occ=None, truncation=None, real=False):
        self.ctx = ctx
        keep = []
        self.desc = make_desc(a, fft, miller, coeff, energy, n_v, ecut_chi,
                              keep, occ, truncation, real)
        h = _p()
        _check(ssrpa_system_create(ctx.handle, ctypes.byref(self.desc),
                                   _stream(stream), ctypes.byref(h)),
               ctx.handle)
        self.handle = h
        ctx._systems.add(self)
        nv, c0, nc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(ssrpa_system_bands(h, ctypes.byref(nv), ctypes.byref(c0),
                                  ctypes.byref(nc)), ctx.handle)
        self.n_v, self.c_first, self.n_c = nv.value, c0.value, nc.value
        self.fft = tuple(int(x) for x in fft)

    @classmethod
    def from_synthetic(cls, ctx: Context, s, stream=None, truncation=None,
                       real=None):
        """real None: the system's own flag (synthetic real orbitals)."""
        if real is None:
            real = bool(getattr(s, "real_orbitals", False))
        return cls(ctx, s.a, s.fft, s.miller, s.coeff, s.energy, s.n_v,
                   s.ecut_chi, stream, getattr(s, "occ", None), truncation,
                   real)

    def close(self):
        if getattr(self, "handle", None):
            if self.ctx.handle:
                ssrpa_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        _check(st, self.ctx.handle)

    def gvectors(self) -> np.ndarray:
        n = ctypes.c_int()
        self._chk(ssrpa_chi_gvectors(self.handle, ctypes.byref(n), None))
        m = np.empty((n.value, 3), dtype=np.int32)
        self._chk(ssrpa_chi_gvectors(self.handle, ctypes.byref(n),
                                     m.ctypes.data_as(_i32p)))
        return m

    @property
    def n_g(self) -> int:
        n = ctypes.c_int()
        self._chk(ssrpa_chi_gvectors(self.handle, ctypes.byref(n), None))
        return n.value

    def orbitals_realspace(self, out_dev, stream=None):
        self._chk(ssrpa_orbitals_realspace(self.handle, _addr(out_dev),
                                           _stream(stream)))

    def pair_matrix(self, v0: int, n_vb: int, out_dev, scaled: bool = True,
                    stream=None):
        self._chk(ssrpa_pair_matrix(self.handle, v0, n_vb, int(scaled),
                                    _addr(out_dev), _stream(stream)))

    def chi0_static(self, precision="fp64", valence_block: int = 0,
                    out_dev=None, symmetrized: bool = True, stream=None):
        self._chk(ssrpa_chi0_static(self.handle, PRECISIONS[precision],
                                    valence_block, _addr(out_dev),
                                    int(symmetrized), _stream(stream)))

    def subspace(self, n_eig: int, basis_dev=None, stream=None,
                 kind: str = "symmetrized") -> np.ndarray:
        ev = np.empty(n_eig)
        self._chk(ssrpa_subspace_basis(self.handle, BASES[kind], n_eig,
                                       _dptr(ev), _addr(basis_dev),
                                       _stream(stream)))
        return ev

    def epsilon_inverse(self, n_eig: int, omega, out_dev, precision="fp64",
                        valence_block: int = 0, stream=None):
        """(I - X_j)^-1 for every frequency into out_dev (device,
        n_freq x n x n complex)."""
        om = np.ascontiguousarray(omega, dtype=np.float64)
        self._chk(ssrpa_epsilon_inverse(self.handle, n_eig, len(om), _dptr(om),
                                        PRECISIONS[precision], valence_block,
                                        _addr(out_dev), _stream(stream)))

    def correlation_energy(self, n_eig: int, omega: Sequence[float],
                           weight: Sequence[float], precision="fp64",
                           valence_block: int = 0, coupling: float = 1.0,
                           chi_sub_dev=None, stream=None):
        om = np.ascontiguousarray(omega, dtype=np.float64)
        wt = np.ascontiguousarray(weight, dtype=np.float64)
        ec = ctypes.c_double()
        f = np.empty(len(om))
        self._chk(ssrpa_correlation_energy(
            self.handle, n_eig, len(om), _dptr(om), _dptr(wt),
            PRECISIONS[precision], valence_block, coupling, ctypes.byref(ec),
            _dptr(f), _addr(chi_sub_dev), _stream(stream)))
        return ec.value, f

    def stage_times(self, enable: bool = True):
        """{stage: (ms, launches)} since the last call; (re)starts timing."""
        ms = np.zeros(len(STAGES))
        n = (ctypes.c_int * len(STAGES))()
        self._chk(ssrpa_stage_times(self.handle, int(enable), _dptr(ms), n))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(STAGES)}

    def enqueue(self, n_eig: int, omega, weight, precision="fp64",
                valence_block: int = 0, stream=None):
        om = np.ascontiguousarray(omega, dtype=np.float64)
        wt = np.ascontiguousarray(weight, dtype=np.float64)
        t = _p()
        self._chk(ssrpa_correlation_energy_enqueue(
            self.handle, n_eig, len(om), _dptr(om), _dptr(wt),
            PRECISIONS[precision], valence_block, _stream(stream),
            ctypes.byref(t)))
        return Ticket(t, len(om))


class KMesh:
    """A resident k mesh (insulator): kpoints is a list of dicts with keys
    miller, coeff, energy, n_v, weight (g_k) and kfrac (k in fractions of the
    reciprocal vectors)."""

    def __init__(self, ctx: Context, a, fft, kpoints, ecut_chi, stream=None):
        self.ctx = ctx
        keep = []
        n = len(kpoints)
        descs = (ssrpa_system_desc * n)()
        for i, k in enumerate(kpoints):
            descs[i] = make_desc(a, fft, k["miller"], k["coeff"], k["energy"],
                                 k["n_v"], ecut_chi, keep)
        kfrac = np.ascontiguousarray([k["kfrac"] for k in kpoints],
                                     dtype=np.float64)
        kw = np.ascontiguousarray([k["weight"] for k in kpoints],
                                  dtype=np.float64)
        h = _p()
        _check(ssrpa_kmesh_create(ctx.handle, n, descs, _dptr(kfrac), _dptr(kw),
                                  _stream(stream), ctypes.byref(h)), ctx.handle)
        self.handle = h
        ctx._systems.add(self)

    def close(self):
        if getattr(self, "handle", None):
            if self.ctx.handle:
                ssrpa_kmesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gvectors(self, q) -> np.ndarray:
        qa = np.ascontiguousarray(q, dtype=np.float64)
        n = ctypes.c_int()
        _check(ssrpa_kmesh_chi_gvectors(self.handle, _dptr(qa), ctypes.byref(n),
                                        None), self.ctx.handle)
        m = np.empty((n.value, 3), dtype=np.int32)
        _check(ssrpa_kmesh_chi_gvectors(self.handle, _dptr(qa), ctypes.byref(n),
                                        m.ctypes.data_as(_i32p)), self.ctx.handle)
        return m

    def stage_times(self, enable: bool = True):
        """{stage: (ms, launches)} since the last call; (re)starts timing."""
        ms = np.zeros(len(STAGES))
        n = (ctypes.c_int * len(STAGES))()
        _check(ssrpa_kmesh_stage_times(self.handle, int(enable), _dptr(ms), n),
               self.ctx.handle)
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(STAGES)}

    def correlation_energy(self, q, kq, g0, n_eig: int, omega, weight,
                           chi0_dev=None, stream=None):
        """E_c(q) and its integrand; kq, g0 with k_i + q = k_kq[i] + g0[i]."""
        qa = np.ascontiguousarray(q, dtype=np.float64)
        kq = np.ascontiguousarray(kq, dtype=np.int32)
        g0 = np.ascontiguousarray(g0, dtype=np.int32).reshape(-1, 3)
        om = np.ascontiguousarray(omega, dtype=np.float64)
        wt = np.ascontiguousarray(weight, dtype=np.float64)
        f = np.empty(len(om))
        ec = ctypes.c_double()
        _check(ssrpa_kmesh_correlation_energy(
            self.handle, _dptr(qa), kq.ctypes.data_as(_i32p),
            g0.ctypes.data_as(_i32p), n_eig, len(om), _dptr(om), _dptr(wt),
            ctypes.byref(ec), _dptr(f), _addr(chi0_dev), _stream(stream)),
            self.ctx.handle)
        return ec.value, f


class Ticket:
    def __init__(self, handle, n_freq):
        self.handle = handle
        self.n_freq = n_freq

    def done(self) -> bool:
        d = ctypes.c_int()
        _check(ssrpa_ticket_query(self.handle, ctypes.byref(d)))
        return bool(d.value)

    def wait(self):
        ec = ctypes.c_double()
        f = np.empty(self.n_freq)
        st = ssrpa_ticket_wait(self.handle, ctypes.byref(ec), _dptr(f))
        self.handle = None
        _check(st)
        return ec.value, f


class Server:
    """Request loop over a context: admission by HBM footprint, overlapping
    solves on separate streams (ssrpa_server_* in the C ABI)."""

    def __init__(self, ctx: Context, max_running: int = 4,
                 max_bypass_s: float = 2.0):
        h = _p()
        _check(ssrpa_server_create(ctx.handle, max_running, max_bypass_s,
                                   ctypes.byref(h)), ctx.handle)
        self.handle = h
        self.ctx = ctx

    def submit(self, s, n_eig: int, omega, weight, precision="fp64") -> int:
        """Queue a synthetic system `s` (host arrays); returns the request id."""
        keep = []
        d = make_desc(s.a, s.fft, s.miller, s.coeff, s.energy, s.n_v,
                      s.ecut_chi, keep, getattr(s, "occ", None), None,
                      bool(getattr(s, "real_orbitals", False)))
        om = np.ascontiguousarray(omega, dtype=np.float64)
        wt = np.ascontiguousarray(weight, dtype=np.float64)
        rid = ctypes.c_uint64()
        _check(ssrpa_server_submit(self.handle, ctypes.byref(d), n_eig,
                                   len(om), _dptr(om), _dptr(wt),
                                   PRECISIONS[precision], ctypes.byref(rid)),
               self.ctx.handle)
        return rid.value

    def poll(self, rid: int) -> dict:
        st, status = ctypes.c_int(), ctypes.c_int()
        ec, t0, t1, t2 = (ctypes.c_double() for _ in range(4))
        _check(ssrpa_server_poll(self.handle, rid, ctypes.byref(st),
                                 ctypes.byref(status), ctypes.byref(ec),
                                 ctypes.byref(t0), ctypes.byref(t1),
                                 ctypes.byref(t2)))
        return dict(state=st.value, status=status.value, ec=ec.value,
                    t_submit=t0.value, t_start=t1.value, t_done=t2.value)

    def device_times(self, rid: int):
        """(start_ms, end_ms) of a finished request on the device clock."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(ssrpa_server_device_times(self.handle, rid, ctypes.byref(a),
                                         ctypes.byref(b)))
        return a.value, b.value

    def error(self, rid: int) -> str:
        """Message of a failed request ("" otherwise)."""
        return ssrpa_server_error(self.handle, rid).decode()

    def drain(self):
        _check(ssrpa_server_drain(self.handle))

    def memory(self):
        a, b = _sz(), _sz()
        _check(ssrpa_server_memory(self.handle, ctypes.byref(a),
                                   ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if self.handle:
            ssrpa_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
