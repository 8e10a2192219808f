"""ctypes binding of the C ABI in ``include/isdf.h`` (argument marshalling only).

Every step of the path runs in the gfx950 library ``libisdf_gfx950.so``; this
module converts numpy arrays / torch tensors to pointers and status codes to
exceptions.  It fails loudly when the library is missing: there is no CPU
fallback.  PyTorch, when given, only supplies device memory and the HIP
stream.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisdf_gfx950.so")

ISDF_OK = 0
STATUS = {0: "ISDF_OK", -1: "ISDF_E_INVALID", -2: "ISDF_E_NOMEM", -3: "ISDF_E_STATE",
          -4: "ISDF_E_NUMERIC", -5: "ISDF_E_DEVICE", -6: "ISDF_E_BUSY",
          -7: "ISDF_E_NOTFOUND", -8: "ISDF_E_CANCELLED"}
ISDF_FP64, ISDF_MIXED_FP32, ISDF_MIXED_BF16X3, ISDF_MIXED_BF16 = 0, 1, 2, 3
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16": 3}
ISDF_INPUT_DEVICE = 0x1
ISDF_NO_PIVOT = 0x2
ISDF_ZETA_ROUTE = 0x4
ISDF_W_PLAIN = 0x8
ISDF_FRAG_DEVICE = 0x1
ISDF_HF_DEVICE = 0x1
ISDF_MP2_DEVICE = 0x1
ISDF_DRPA_DEVICE = 0x1
C_SOS = 1.3
REQ_STATES = {0: "QUEUED", 1: "RUNNING", 2: "DONE", 3: "FAILED", 4: "CANCELLED"}

EXPORTS = ["isdf_create", "isdf_fit", "isdf_coulomb_kernel", "isdf_get_metric",
           "isdf_get_kernel", "isdf_get_ivs", "isdf_get_rhs", "isdf_get_eta_tilde", "isdf_fragment_eri",
           "isdf_serve_start", "isdf_submit", "isdf_submit_n", "isdf_poll", "isdf_cancel",
           "isdf_serve_stop", "isdf_stats", "isdf_stage_ms", "isdf_stage_total", "isdf_stage_reset", "isdf_plan_bytes", "isdf_storage_model_bytes",
           "isdf_graph_create", "isdf_graph_launch", "isdf_graph_destroy", "isdf_autotune", "isdf_set_tiling",
           "isdf_save", "isdf_load", "isdf_fragment_eri_static", "isdf_select_points", "isdf_hf_jk",
           "isdf_sos_mp2", "isdf_drpa", "isdf_destroy", "isdf_last_error", "isdf_version"]


class IsdfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Request(ctypes.Structure):
    _fields_ = [("n_f", ctypes.c_int32), ("C", ctypes.c_void_p), ("eri", ctypes.c_void_p),
                ("prec", ctypes.c_int32), ("flags", ctypes.c_uint32), ("priority", ctypes.c_int32)]


class TuneReport(ctypes.Structure):
    _fields_ = [("eri_qgroup", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("ms", ctypes.c_double),
                ("ms_default", ctypes.c_double), ("n_tried", ctypes.c_int32)]


_lib = None


def load_library(path=LIB_PATH):
    """Load the gfx950 library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libisdf_gfx950.so not found at %s; build it with "
                           "`python -m paper_2601_16379_amd.build`" % path)
    # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7;
    # importing it first makes the library bind to that same runtime (same
    # soname) instead of loading a second copy from /opt/rocm.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I32, U32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_double
    sig = {
        "isdf_create": (I32, [ctypes.POINTER(P), P, P, P, I32, P, P, I32, U32, P]),
        "isdf_fit": (I32, [P, I32]),
        "isdf_coulomb_kernel": (I32, [P, I32]),
        "isdf_get_metric": (I32, [P, I32, P]),
        "isdf_get_kernel": (I32, [P, I32, P]),
        "isdf_get_ivs": (I32, [P, I32, P]),
        "isdf_get_rhs": (I32, [P, I32, P]),
        "isdf_get_eta_tilde": (I32, [P, I32, P]),
        "isdf_fragment_eri": (I32, [P, I32, I32, P, P, P, U32]),
        "isdf_fragment_eri_static": (I32, [P, I32, I32, P, P, P, U32]),
        "isdf_select_points": (I32, [P, P, I32, P, I32, P, P, U32, P]),
        "isdf_hf_jk": (I32, [P, P, P, P, U32]),
        "isdf_sos_mp2": (I32, [P, P, P, I32, I32, I32, P, P, P, P, P, U32]),
        "isdf_drpa": (I32, [P, P, P, I32, I32, I32, P, I32, P, P, P, P, P, P, U32]),
        "isdf_serve_start": (I32, [P, I32, I32, I64]),
        "isdf_submit": (I32, [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
        "isdf_submit_n": (I32, [P, I32, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
        "isdf_stage_total": (I32, [P, ctypes.c_char_p, ctypes.POINTER(D), ctypes.POINTER(I64)]),
        "isdf_stage_reset": (I32, [P]),
        "isdf_poll": (I32, [P, ctypes.c_uint64, ctypes.POINTER(I32), ctypes.POINTER(D)]),
        "isdf_cancel": (I32, [P, ctypes.c_uint64]),
        "isdf_serve_stop": (I32, [P]),
        "isdf_stats": (I32, [P, ctypes.c_char_p, I64]),
        "isdf_stage_ms": (D, [P, ctypes.c_char_p]),
        "isdf_plan_bytes": (I64, [P, P, I32, I32]),
        "isdf_storage_model_bytes": (I64, [I64, I64, I64]),
        "isdf_graph_create": (I32, [P, I32, I32, P, P, P, ctypes.POINTER(P)]),
        "isdf_graph_launch": (I32, [P]),
        "isdf_autotune": (I32, [P, I32, I32, P, P, P, ctypes.POINTER(TuneReport)]),
        "isdf_set_tiling": (I32, [P, I32, I32]),
        "isdf_graph_destroy": (I32, [P]),
        "isdf_save": (I32, [P, ctypes.c_char_p]),
        "isdf_load": (I32, [ctypes.POINTER(P), ctypes.c_char_p, P]),
        "isdf_destroy": (I32, [P]),
        "isdf_last_error": (ctypes.c_char_p, [P]),
        "isdf_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(x):
    """(pointer, is_device) of a numpy array or torch tensor."""
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C contiguous")
        return x.ctypes.data, False
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr(), x.device.type != "cpu"
    raise TypeError("expected numpy array or torch tensor, got %r" % type(x))


def current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return 0


def isdf_plan_bytes(grid, kmesh, n_orb, n_ip):
    lib = load_library()
    g = np.asarray(grid, dtype=np.int32)
    k = np.asarray(kmesh, dtype=np.int32)
    return int(lib.isdf_plan_bytes(g.ctypes.data, k.ctypes.data, int(n_orb), int(n_ip)))


def isdf_storage_model_bytes(n_k, n_ip, n_ao):
    return int(load_library().isdf_storage_model_bytes(int(n_k), int(n_ip), int(n_ao)))


def isdf_version():
    return load_library().isdf_version().decode()


def select_points(grid, kmesh, orbitals, n_ip, stream=None):
    """``isdf_select_points``: the first n_ip pivots of the pivoted Cholesky
    of the pair products of ``orbitals`` ([N_k, n_orb, N_g] c128, numpy or
    torch, host or device).  Returns (ip_index int32 [n_ip] in selection
    order, residual float64 [n_ip]: d(p) of each pivot when chosen)."""
    lib = load_library()
    g = np.ascontiguousarray(np.asarray(grid, dtype=np.int32))
    k = np.ascontiguousarray(np.asarray(kmesh, dtype=np.int32))
    shape = tuple(orbitals.shape)
    if len(shape) != 3 or shape[0] != int(np.prod(k)) or shape[2] != int(np.prod(g)):
        raise ValueError("orbitals must be [N_k, n_orb, N_g]")
    optr, odev = _ptr(orbitals)
    ip = np.zeros(int(n_ip), dtype=np.int32)
    res = np.zeros(int(n_ip), dtype=np.float64)
    st_ = current_stream() if stream is None else stream
    st = lib.isdf_select_points(g.ctypes.data, k.ctypes.data, int(shape[1]), optr, int(n_ip), ip.ctypes.data,
                                res.ctypes.data, ISDF_INPUT_DEVICE if odev else 0, st_)
    if st != ISDF_OK:
        raise IsdfError(st, "isdf_select_points: " + lib.isdf_last_error(None).decode())
    return ip, res


def _n_classes(kmesh):
    """Number of classes {q, -q} of a k mesh (q with -q not smaller)."""
    m = [int(v) for v in kmesh]
    n = 0
    for j1 in range(m[0]):
        for j2 in range(m[1]):
            for j3 in range(m[2]):
                q = (j1 * m[1] + j2) * m[2] + j3
                mq = (((-j1) % m[0]) * m[1] + (-j2) % m[1]) * m[2] + (-j3) % m[2]
                n += mq >= q
    return n


class Isdf:
    """One library context: ``isdf_create`` at construction, the other calls
    as methods with the C names (``fit``, ``coulomb_kernel``, ...)."""

    def __init__(self, lattice, grid, kmesh, orbitals, ip_index, no_pivot=False, stream=None, q_batch=0,
                 zeta_route=False, w_plain=False, _handle=None):
        self.lib = load_library()
        if _handle is not None:             # a context restored by isdf_load
            self.h, (self.grid, self.kmesh, self.n_orb, self.n_ip, self.stream) = _handle
            self.n_k = int(np.prod(self.kmesh))
            self.n_g = int(np.prod(self.grid))
            return
        lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64))
        self.grid = np.ascontiguousarray(np.asarray(grid, dtype=np.int32))
        self.kmesh = np.ascontiguousarray(np.asarray(kmesh, dtype=np.int32))
        self.n_k = int(np.prod(self.kmesh))
        self.n_g = int(np.prod(self.grid))
        optr, odev = _ptr(orbitals)
        if isinstance(ip_index, np.ndarray):
            ip_index = np.ascontiguousarray(ip_index, dtype=np.int32)
        iptr, idev = _ptr(ip_index)
        if odev != idev:
            raise ValueError("orbitals and ip_index must both be host or both device")
        shape = tuple(orbitals.shape)
        if len(shape) != 3 or shape[0] != self.n_k or shape[2] != self.n_g:
            raise ValueError("orbitals must be [N_k, n_orb, N_g]")
        self.n_orb = int(shape[1])
        self.n_ip = int(ip_index.shape[0])
        flags = (ISDF_INPUT_DEVICE if odev else 0) | (ISDF_NO_PIVOT if no_pivot else 0) \
            | (ISDF_ZETA_ROUTE if zeta_route else 0) | (ISDF_W_PLAIN if w_plain else 0) \
            | ((int(q_batch) & 0xFFFF) << 16)
        self.stream = current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        st = self.lib.isdf_create(ctypes.byref(h), lat.ctypes.data, self.grid.ctypes.data,
                                  self.kmesh.ctypes.data, self.n_orb, optr, iptr, self.n_ip,
                                  flags, self.stream)
        if st != ISDF_OK:
            raise IsdfError(st, "isdf_create: " + self.lib.isdf_last_error(None).decode())
        self.h = h

    @classmethod
    def load(cls, path, stream=None):
        """A context restored from a checkpoint written by ``save`` (no
        orbitals: it serves fragment ERIs with the saved W^q)."""
        import struct
        lib = load_library()
        with open(path, "rb") as f:
            head = f.read(144)
        st_ = current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        st = lib.isdf_load(ctypes.byref(h), os.fsencode(path), st_)
        if st != ISDF_OK:
            raise IsdfError(st, "isdf_load: " + lib.isdf_last_error(None).decode())
        grid = np.array(struct.unpack_from("<3i", head, 16), dtype=np.int32)
        kmesh = np.array(struct.unpack_from("<3i", head, 28), dtype=np.int32)
        n_orb, n_ip = struct.unpack_from("<2i", head, 40)
        return cls(None, None, None, None, None, _handle=(h, (grid, kmesh, n_orb, n_ip, st_)))

    def save(self, path):
        self._check(self.lib.isdf_save(self.h, os.fsencode(path)), "isdf_save")

    # -- helpers -------------------------------------------------------------
    def _check(self, st, what):
        if st != ISDF_OK:
            raise IsdfError(st, "%s: %s" % (what, self.lib.isdf_last_error(self.h).decode()))

    def close(self):
        for g in getattr(self, "_graphs", []):
            g.close()                      # graphs go before their context
        if getattr(self, "h", None):
            self.lib.isdf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the path ------------------------------------------------------------
    def fit(self, prec="fp64"):
        """``prec``: precision of the kernel that will consume eta; a mixed
        precision stores eta as complex FP32 where the grid allows it."""
        self._check(self.lib.isdf_fit(self.h, PRECISIONS.get(prec, prec)), "isdf_fit")

    def coulomb_kernel(self, prec="fp64"):
        self._check(self.lib.isdf_coulomb_kernel(self.h, PRECISIONS.get(prec, prec)),
                    "isdf_coulomb_kernel")

    def _get(self, fn, idx, shape):
        out = np.empty(shape, dtype=np.complex128)
        self._check(fn(self.h, int(idx), out.ctypes.data), fn.__name__)
        return out

    def get_metric(self, q):
        return self._get(self.lib.isdf_get_metric, q, (self.n_ip, self.n_ip))

    def get_kernel(self, q):
        return self._get(self.lib.isdf_get_kernel, q, (self.n_ip, self.n_ip))

    def get_ivs(self, k):
        return self._get(self.lib.isdf_get_ivs, k, (self.n_ip, self.n_orb))

    def get_rhs(self, q):
        return self._get(self.lib.isdf_get_rhs, q, (self.n_ip, self.n_g))

    def get_eta_tilde(self, q):
        return self._get(self.lib.isdf_get_eta_tilde, q, (self.n_ip, self.n_g))

    def fragment_eri(self, coeffs, prec="fp64", out=None, pair_blocks=0):
        """ERIs of a batch of fragments in one pass.  ``coeffs``: list of
        [N_k, n_orb, n_f] complex128 arrays (numpy = host, torch cuda tensors =
        device).  ``pair_blocks`` > 1 runs every fragment alone with its pairs
        in that many blocks.  Returns the list of [n_f]^4 outputs (same kind)."""
        n = len(coeffs)
        nfs = np.array([c.shape[2] for c in coeffs], dtype=np.int32)
        dev = [(_ptr(c)[1]) for c in coeffs]
        if any(dev) != all(dev):
            raise ValueError("mixing host and device fragments in one call")
        if out is None:
            if dev[0]:
                import torch
                out = [torch.empty((f, f, f, f), dtype=torch.complex128, device=coeffs[0].device)
                       for f in nfs]
            else:
                out = [np.empty((f, f, f, f), dtype=np.complex128) for f in nfs]
        cptr = (ctypes.c_void_p * n)(*[_ptr(c)[0] for c in coeffs])
        eptr = (ctypes.c_void_p * n)(*[_ptr(e)[0] for e in out])
        flags = (ISDF_FRAG_DEVICE if dev[0] else 0) | ((int(pair_blocks) & 0xFF) << 8)
        self._check(self.lib.isdf_fragment_eri(self.h, PRECISIONS.get(prec, prec), n,
                                               nfs.ctypes.data, cptr, eptr, flags),
                    "isdf_fragment_eri")
        return out

    def hf_jk(self, dm, want_j=True, want_k=True):
        """``isdf_hf_jk``: Coulomb and exchange matrices of the k-point density
        matrices ``dm`` ([N_k, n_orb, n_orb] complex128, numpy = host, torch
        cuda tensor = device).  Returns (J, K) of the same kind (None where not
        asked for)."""
        if tuple(dm.shape) != (self.n_k, self.n_orb, self.n_orb):
            raise ValueError("dm must be [N_k, n_orb, n_orb]")
        dptr, dev = _ptr(dm)
        if dev:
            import torch
            mk = lambda: torch.empty(tuple(dm.shape), dtype=torch.complex128, device=dm.device)  # noqa: E731
        else:
            mk = lambda: np.empty(tuple(dm.shape), dtype=np.complex128)  # noqa: E731
        j = mk() if want_j else None
        k = mk() if want_k else None
        self._check(self.lib.isdf_hf_jk(self.h, dptr, _ptr(j)[0] if j is not None else None,
                                        _ptr(k)[0] if k is not None else None, ISDF_HF_DEVICE if dev else 0),
                    "isdf_hf_jk")
        return j, k

    def sos_mp2(self, mo_coeff, mo_energy, n_occ, tau, weight, per_class=False):
        """``isdf_sos_mp2``: opposite-spin MP2 energy per cell from canonical
        orbitals ``mo_coeff`` ([N_k, n_orb, n_mo] complex128, numpy or torch
        cuda) with energies ``mo_energy`` ([N_k, n_mo]) and the first n_occ
        occupied, on the quadrature (tau, weight) of [0, inf).  Returns a dict:
        e_os, e_sos_mp2 (= 1.3 e_os), integrand (F at every tau) and, with
        per_class, classes ([n_tau, nh] contributions)."""
        cptr, dev = _ptr(mo_coeff)
        nmo = int(mo_coeff.shape[2])
        if tuple(mo_coeff.shape[:2]) != (self.n_k, self.n_orb):
            raise ValueError("mo_coeff must be [N_k, n_orb, n_mo]")
        e = np.ascontiguousarray(np.asarray(mo_energy, dtype=np.float64))
        if e.shape != (self.n_k, nmo):
            raise ValueError("mo_energy must be [N_k, n_mo]")
        t = np.ascontiguousarray(np.asarray(tau, dtype=np.float64))
        w = np.ascontiguousarray(np.asarray(weight, dtype=np.float64))
        if t.shape != w.shape or t.ndim != 1:
            raise ValueError("tau and weight must be matching 1-d arrays")
        f = np.zeros(t.size)
        nh = _n_classes(self.kmesh)
        cls = np.zeros((t.size, nh)) if per_class else None
        eos = ctypes.c_double()
        self._check(self.lib.isdf_sos_mp2(self.h, cptr, e.ctypes.data, nmo, int(n_occ), int(t.size), t.ctypes.data,
                                          w.ctypes.data, f.ctypes.data,
                                          cls.ctypes.data if cls is not None else None, ctypes.byref(eos),
                                          ISDF_MP2_DEVICE if dev else 0), "isdf_sos_mp2")
        out = {"e_os": eos.value, "e_sos_mp2": C_SOS * eos.value, "integrand": f}
        if per_class:
            out["classes"] = cls
        return out

    def drpa(self, mo_coeff, mo_energy, n_occ, tau, omega_weight, transform, per_class=False):
        """``isdf_drpa``: direct RPA correlation energy per cell (eq. (16)) of
        the canonical orbitals: polarisabilities at the times ``tau``, mapped
        to the frequencies by ``transform`` ([n_omega, n_tau] complex128,
        gamma[m, n] ~ the weight of exp(-D tau_n) in 1/(D - i w_m)), the
        frequency quadrature weights ``omega_weight``.  Returns a dict:
        e_drpa, e_second (the second-order term), integrand (F at every
        frequency) and, with per_class, classes ([n_omega, nh])."""
        cptr, dev = _ptr(mo_coeff)
        nmo = int(mo_coeff.shape[2])
        if tuple(mo_coeff.shape[:2]) != (self.n_k, self.n_orb):
            raise ValueError("mo_coeff must be [N_k, n_orb, n_mo]")
        e = np.ascontiguousarray(np.asarray(mo_energy, dtype=np.float64))
        if e.shape != (self.n_k, nmo):
            raise ValueError("mo_energy must be [N_k, n_mo]")
        t = np.ascontiguousarray(np.asarray(tau, dtype=np.float64))
        ow = np.ascontiguousarray(np.asarray(omega_weight, dtype=np.float64))
        g = np.ascontiguousarray(np.asarray(transform, dtype=np.complex128))
        if t.ndim != 1 or ow.ndim != 1 or g.shape != (ow.size, t.size):
            raise ValueError("transform must be [n_omega, n_tau] for tau [n_tau], omega_weight [n_omega]")
        f = np.zeros(ow.size)
        cls = np.zeros((ow.size, _n_classes(self.kmesh))) if per_class else None
        e_r, e_2 = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.isdf_drpa(self.h, cptr, e.ctypes.data, nmo, int(n_occ), int(t.size), t.ctypes.data,
                                       int(ow.size), ow.ctypes.data, g.ctypes.data, f.ctypes.data,
                                       cls.ctypes.data if cls is not None else None, ctypes.byref(e_r),
                                       ctypes.byref(e_2), ISDF_DRPA_DEVICE if dev else 0), "isdf_drpa")
        out = {"e_drpa": e_r.value, "e_second": e_2.value, "integrand": f}
        if per_class:
            out["classes"] = cls
        return out

    def graph(self, coeffs, out, prec="bf16x3"):
        """The fragment pipeline of this batch (device tensors ``coeffs``, ERIs
        into ``out``) captured as a HIP graph; ``.launch()`` replays it."""
        n = len(coeffs)
        if len(out) != n:
            raise ValueError("one output per fragment")
        if not all(_ptr(c)[1] for c in coeffs) or not all(_ptr(e)[1] for e in out):
            raise ValueError("graph fragments must be device tensors")
        nfs = np.array([c.shape[2] for c in coeffs], dtype=np.int32)
        cptr = (ctypes.c_void_p * n)(*[_ptr(c)[0] for c in coeffs])
        eptr = (ctypes.c_void_p * n)(*[_ptr(e)[0] for e in out])
        h = ctypes.c_void_p()
        self._check(self.lib.isdf_graph_create(self.h, PRECISIONS.get(prec, prec), n, nfs.ctypes.data,
                                               cptr, eptr, ctypes.byref(h)), "isdf_graph_create")
        g = FragmentGraph(self, h, list(coeffs), list(out))
        if not hasattr(self, "_graphs"):
            self._graphs = []
        self._graphs.append(g)
        return g

    def autotune(self, coeffs, out, prec="bf16x3"):
        """isdf_autotune on this batch (device tensors); returns the report."""
        n = len(coeffs)
        if not all(_ptr(c)[1] for c in coeffs) or not all(_ptr(e)[1] for e in out):
            raise ValueError("autotune fragments must be device tensors")
        nfs = np.array([c.shape[2] for c in coeffs], dtype=np.int32)
        cptr = (ctypes.c_void_p * n)(*[_ptr(c)[0] for c in coeffs])
        eptr = (ctypes.c_void_p * n)(*[_ptr(e)[0] for e in out])
        r = TuneReport()
        self._check(self.lib.isdf_autotune(self.h, PRECISIONS.get(prec, prec), n, nfs.ctypes.data, cptr, eptr,
                                           ctypes.byref(r)), "isdf_autotune")
        return {"eri_qgroup": r.eri_qgroup, "wg_per_cu": r.wg_per_cu, "ms": r.ms,
                "ms_default": r.ms_default, "n_tried": r.n_tried}

    def set_tiling(self, eri_qgroup, wg_per_cu=0):
        self._check(self.lib.isdf_set_tiling(self.h, int(eri_qgroup), int(wg_per_cu)), "isdf_set_tiling")

    # -- serving -------------------------------------------------------------
    def serve_start(self, max_inflight=2, max_batch=64, budget_bytes=64 << 30):
        self._check(self.lib.isdf_serve_start(self.h, max_inflight, max_batch, budget_bytes),
                    "isdf_serve_start")

    def submit(self, coeffs, eri, prec="fp64", priority=0):
        cp, cdev = _ptr(coeffs)
        ep, edev = _ptr(eri)
        if cdev != edev:
            raise ValueError("C and eri must both be host or both device")
        req = Request(int(coeffs.shape[2]), cp, ep, PRECISIONS.get(prec, prec),
                      ISDF_FRAG_DEVICE if cdev else 0, int(priority))
        t = ctypes.c_uint64()
        self._check(self.lib.isdf_submit(self.h, ctypes.byref(req), ctypes.byref(t)), "isdf_submit")
        return t.value

    def submit_n(self, coeffs, eris, prec="fp64", priority=0):
        """Submit several fragments at one instant; returns their tickets."""
        n = len(coeffs)
        reqs = (Request * n)()
        for i, (c, e) in enumerate(zip(coeffs, eris)):
            cp, cdev = _ptr(c)
            ep, edev = _ptr(e)
            if cdev != edev:
                raise ValueError("C and eri must both be host or both device")
            reqs[i] = Request(int(c.shape[2]), cp, ep, PRECISIONS.get(prec, prec),
                              ISDF_FRAG_DEVICE if cdev else 0, int(priority))
        t = (ctypes.c_uint64 * n)()
        self._check(self.lib.isdf_submit_n(self.h, n, reqs, t), "isdf_submit_n")
        return list(t)

    def poll(self, ticket):
        st = ctypes.c_int32()
        lat = ctypes.c_double()
        self._check(self.lib.isdf_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(st),
                                       ctypes.byref(lat)), "isdf_poll")
        return REQ_STATES[st.value], lat.value

    def cancel(self, ticket):
        self._check(self.lib.isdf_cancel(self.h, ctypes.c_uint64(ticket)), "isdf_cancel")

    def serve_stop(self):
        self._check(self.lib.isdf_serve_stop(self.h), "isdf_serve_stop")

    # -- introspection ---------------------------------------------------------
    def stats(self):
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        self._check(self.lib.isdf_stats(self.h, buf, len(buf)), "isdf_stats")
        return json.loads(buf.value.decode())

    def stage_ms(self, name):
        return float(self.lib.isdf_stage_ms(self.h, name.encode()))

    def stage_total(self, name):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self._check(self.lib.isdf_stage_total(self.h, name.encode(), ctypes.byref(ms),
                                              ctypes.byref(cnt)), "isdf_stage_total")
        return ms.value, cnt.value

    def stage_reset(self):
        self._check(self.lib.isdf_stage_reset(self.h), "isdf_stage_reset")

    def last_error(self):
        return self.lib.isdf_last_error(self.h).decode()


class FragmentGraph:
    """A captured fragment batch (isdf_graph_*); keeps its tensors alive."""

    def __init__(self, ctx, h, coeffs, out):
        self.ctx, self.h, self.coeffs, self.out = ctx, h, coeffs, out

    def launch(self):
        self.ctx._check(self.ctx.lib.isdf_graph_launch(self.h), "isdf_graph_launch")
        return self.out

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.isdf_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
