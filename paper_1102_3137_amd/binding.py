"""ctypes binding of include/dyson.h (argument marshalling only).

Functions keep the C names (dyson_create, dyson_plan_create, dyson_solve, ...).
The `Plan` helper accepts torch tensors that live on the GPU and passes their
data pointers and the current HIP stream; PyTorch provides device memory and
streams, every computation runs in the HIP kernels of the library.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdyson_mi355x.so")

PART_NESTED, PART_SINGLE = 0, 1
PREC_FP64, PREC_MIXED, PREC_MIXED16 = 0, 1, 2
MEM_DEVICE, MEM_HOST = 0, 1
STATUS = {0: "DYSON_OK", 1: "DYSON_EINVAL", 2: "DYSON_ENOMEM", 3: "DYSON_EBREAKDOWN",
          4: "DYSON_ENOCONV", 5: "DYSON_EDEVICE", 6: "DYSON_EUNSUPPORTED", 7: "DYSON_EBUSY",
          8: "DYSON_ECANCELLED", 9: "DYSON_ETIMEOUT"}
OK, EINVAL, ENOMEM, EBREAKDOWN, ENOCONV, EDEVICE, EUNSUPPORTED, EBUSY, ECANCELLED, ETIMEOUT = \
    range(10)


class DysonError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Lattice(C.Structure):
    _fields_ = [("dim", C.c_int), ("L", C.c_int * 3), ("periodic", C.c_int * 3),
                ("t", C.c_double), ("mu", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("leaf_edge", C.c_int), ("partition", C.c_int), ("precision", C.c_int),
                ("max_rank", C.c_int), ("extra_steps", C.c_int), ("max_inner_iters", C.c_int),
                ("inner_tol", C.c_double), ("lanczos_tol", C.c_double), ("seed", C.c_uint64),
                ("profile", C.c_int), ("level_streams", C.c_int), ("check_sites", C.c_int),
                ("fault_step", C.c_int), ("fault_attempts", C.c_int),
                ("breakdown_tol", C.c_double), ("interface_lanczos", C.c_int),
                ("inner_graphs", C.c_int)]


class Report(C.Structure):
    _fields_ = [("t_total_ms", C.c_double), ("levels", C.c_int), ("max_rank_used", C.c_int),
                ("lanczos_steps", C.c_longlong), ("inner_iters", C.c_longlong),
                ("inner_iters_max", C.c_int), ("restarts", C.c_int), ("truncated", C.c_int),
                ("kern_ms", C.c_double * 4), ("kern_launches", C.c_longlong * 4),
                ("kern_bytes", C.c_double * 4), ("t_queue_ms", C.c_double),
                ("batches", C.c_int), ("hbm_bytes", C.c_size_t), ("est_rel_err", C.c_double),
                ("capped_items", C.c_int)]

    def as_dict(self):
        return {"t_total_ms": self.t_total_ms, "levels": self.levels,
                "max_rank_used": self.max_rank_used, "lanczos_steps": self.lanczos_steps,
                "inner_iters": self.inner_iters, "inner_iters_max": self.inner_iters_max,
                "restarts": self.restarts, "truncated": self.truncated,
                "kern_ms": list(self.kern_ms), "kern_launches": list(self.kern_launches),
                "kern_bytes": list(self.kern_bytes), "t_queue_ms": self.t_queue_ms,
                "batches": self.batches, "hbm_bytes": int(self.hbm_bytes),
                "est_rel_err": self.est_rel_err, "capped_items": self.capped_items}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class PlanInfo(C.Structure):
    _fields_ = [("n_sites", C.c_int), ("n_tiles", C.c_int), ("tile_sites", C.c_int),
                ("levels", C.c_int), ("n_nodes", C.c_int * 32), ("max_m", C.c_int * 32),
                ("sum_m", C.c_longlong * 32)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)

# (name, restype, argtypes) for every entry point of include/dyson.h
SIGNATURES = [
    ("dyson_create", C.c_int, [C.POINTER(_P), C.c_int, C.c_size_t, C.POINTER(Allocator)]),
    ("dyson_destroy", C.c_int, [_P]),
    ("dyson_plan_create", C.c_int, [_P, C.POINTER(Lattice), C.POINTER(Opts), C.POINTER(_P)]),
    ("dyson_plan_destroy", C.c_int, [_P]),
    ("dyson_plan_trim", C.c_int, [_P]),
    ("dyson_plan_get_info", C.c_int, [_P, C.POINTER(PlanInfo)]),
    ("dyson_plan_get_maps", C.c_int, [_P, _I, _I, _I]),
    ("dyson_plan_get_domains", C.c_int, [_P, C.c_int, _I, _I]),
    ("dyson_footprint", C.c_int, [_P, C.c_int, C.POINTER(C.c_size_t)]),
    ("dyson_solve", C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P, C.POINTER(Report)]),
    ("dyson_solve_z", C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P, C.POINTER(Report)]),
    ("dyson_solve_host", C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P, C.POINTER(Report)]),
    ("dyson_solve_schur", C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P, C.POINTER(Report)]),
    ("dyson_solve_noalloc", C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P, C.POINTER(Report)]),
    ("dyson_noalloc_bytes", C.c_int, [_P, C.c_int, C.POINTER(C.c_size_t)]),
    ("dyson_noalloc_max_bytes", C.c_size_t, []),
    ("dyson_assemble", C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P]),
    ("dyson_leaf_diag", C.c_int, [_P, C.c_int, _P, _P, _P]),
    ("dyson_xmatvec", C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P]),
    ("dyson_correct_level", C.c_int, [_P, C.c_int, C.c_int, _P, _P, _I, _P]),
    ("dyson_autotune", C.c_int, [_P, C.POINTER(Lattice), C.POINTER(Opts), C.c_int, _P, _P, _P,
                                 C.POINTER(Opts), C.POINTER(C.c_double)]),
    ("dyson_serve_config", C.c_int, [_P, C.c_int, C.c_int]),
    ("dyson_submit", C.c_int, [_P, C.c_int, _P, _P, _P, _P, C.c_int, C.POINTER(_P)]),
    ("dyson_submit_z", C.c_int, [_P, C.c_int, _P, _P, _P, _P, C.c_int, C.POINTER(_P)]),
    ("dyson_poll", C.c_int, [_P, _I]),
    ("dyson_wait", C.c_int, [_P, C.c_double]),
    ("dyson_cancel", C.c_int, [_P]),
    ("dyson_req_report", C.c_int, [_P, C.POINTER(Report)]),
    ("dyson_release", C.c_int, [_P]),
    ("dyson_solve_batch", C.c_int, [C.c_int, C.POINTER(_P), _I, C.POINTER(_P), C.POINTER(_P),
                                    C.POINTER(_P), C.POINTER(_P), _P, C.POINTER(Report)]),
    ("dyson_last_error", C.c_char_p, []),
    ("dyson_version", C.c_char_p, []),
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1102_3137_amd.build`"
                          " (there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != 0:
        raise DysonError(status, load_library().dyson_last_error().decode())


# thin wrappers with the C names --------------------------------------------
def dyson_create(device: int = 0, hbm_budget: int = 0, allocator: Allocator | None = None):
    h = _P()
    _check(load_library().dyson_create(C.byref(h), device, hbm_budget,
                                       C.byref(allocator) if allocator is not None else None))
    return h


def dyson_destroy(ctx):
    _check(load_library().dyson_destroy(ctx))


def dyson_plan_create(ctx, lat: Lattice, opts: Opts | None):
    h = _P()
    _check(load_library().dyson_plan_create(ctx, C.byref(lat),
                                            C.byref(opts) if opts is not None else None,
                                            C.byref(h)))
    return h


def dyson_plan_destroy(plan):
    _check(load_library().dyson_plan_destroy(plan))


def dyson_plan_get_info(plan) -> PlanInfo:
    info = PlanInfo()
    _check(load_library().dyson_plan_get_info(plan, C.byref(info)))
    return info


def dyson_plan_get_maps(plan, n_sites: int):
    import numpy as np
    depth = np.zeros(n_sites, np.int32)
    is_sep = np.zeros(n_sites, np.int32)
    tile = np.zeros(n_sites, np.int32)
    ip = lambda a: a.ctypes.data_as(_I)  # noqa: E731
    _check(load_library().dyson_plan_get_maps(plan, ip(depth), ip(is_sep), ip(tile)))
    return depth, is_sep, tile


def dyson_plan_get_domains(plan, level: int, n_nodes: int):
    import numpy as np
    m = np.zeros(n_nodes, np.int32)
    cap = np.zeros(n_nodes, np.int32)
    _check(load_library().dyson_plan_get_domains(plan, level, m.ctypes.data_as(_I),
                                                 cap.ctypes.data_as(_I)))
    return m, cap


def dyson_footprint(plan, K: int) -> int:
    b = C.c_size_t()
    _check(load_library().dyson_footprint(plan, K, C.byref(b)))
    return int(b.value)


def dyson_solve(plan, K, V_ptr, omega_ptr, sigma_ptr, G_ptr, stream, report: Report | None = None):
    _check(load_library().dyson_solve(plan, K, V_ptr, omega_ptr, sigma_ptr, G_ptr, stream,
                                      C.byref(report) if report is not None else None))


def dyson_solve_host(plan, K, V_ptr, omega_ptr, sigma_ptr, G_ptr, stream,
                     report: Report | None = None):
    _check(load_library().dyson_solve_host(plan, K, V_ptr, omega_ptr, sigma_ptr, G_ptr, stream,
                                           C.byref(report) if report is not None else None))


def dyson_solve_noalloc(plan, K, V_ptr, omega_ptr, sigma_ptr, G_ptr, stream,
                        report: Report | None = None):
    _check(load_library().dyson_solve_noalloc(plan, K, V_ptr, omega_ptr, sigma_ptr, G_ptr, stream,
                                              C.byref(report) if report is not None else None))


def dyson_solve_schur(plan, K, V_ptr, omega_ptr, sigma_ptr, G_ptr, stream,
                      report: Report | None = None):
    _check(load_library().dyson_solve_schur(plan, K, V_ptr, omega_ptr, sigma_ptr, G_ptr, stream,
                                            C.byref(report) if report is not None else None))


def dyson_noalloc_bytes(plan, K: int) -> int:
    b = C.c_size_t()
    _check(load_library().dyson_noalloc_bytes(plan, K, C.byref(b)))
    return int(b.value)


def dyson_noalloc_max_bytes() -> int:
    return int(load_library().dyson_noalloc_max_bytes())


def dyson_solve_z(plan, K, V_ptr, z_ptr, sigma_ptr, G_ptr, stream, report: Report | None = None):
    _check(load_library().dyson_solve_z(plan, K, V_ptr, z_ptr, sigma_ptr, G_ptr, stream,
                                        C.byref(report) if report is not None else None))


def dyson_assemble(plan, K, V_ptr, omega_ptr, sigma_ptr, d_ptr, stream):
    _check(load_library().dyson_assemble(plan, K, V_ptr, omega_ptr, sigma_ptr, d_ptr, stream))


def dyson_leaf_diag(plan, K, d_ptr, G_ptr, stream):
    _check(load_library().dyson_leaf_diag(plan, K, d_ptr, G_ptr, stream))


def dyson_xmatvec(plan, level, K, d_ptr, q_ptr, u_ptr, stream):
    _check(load_library().dyson_xmatvec(plan, level, K, d_ptr, q_ptr, u_ptr, stream))


def dyson_correct_level(plan, level, K, d_ptr, G_ptr, steps_np, stream):
    sp = steps_np.ctypes.data_as(_I) if steps_np is not None else None
    _check(load_library().dyson_correct_level(plan, level, K, d_ptr, G_ptr, sp, stream))


def dyson_serve_config(ctx, slots: int, max_batch_freqs: int):
    _check(load_library().dyson_serve_config(ctx, slots, max_batch_freqs))


def dyson_submit(plan, K, V_ptr, omega_ptr, sigma_ptr, G_ptr, mem, zmode=False):
    h = _P()
    fn = load_library().dyson_submit_z if zmode else load_library().dyson_submit
    _check(fn(plan, K, V_ptr, omega_ptr, sigma_ptr, G_ptr, mem, C.byref(h)))
    return h


def dyson_poll(req) -> bool:
    d = C.c_int()
    _check(load_library().dyson_poll(req, C.byref(d)))
    return bool(d.value)


def dyson_wait(req, timeout_s: float = -1.0) -> int:
    """Returns the request's status code (DYSON_ETIMEOUT if unfinished)."""
    return load_library().dyson_wait(req, float(timeout_s))


def dyson_cancel(req):
    _check(load_library().dyson_cancel(req))


def dyson_req_report(req) -> Report:
    r = Report()
    _check(load_library().dyson_req_report(req, C.byref(r)))
    return r


def dyson_release(req):
    _check(load_library().dyson_release(req))


# torch-facing helper ---------------------------------------------------------
def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Plan:
    """A plan on one GPU.  Inputs and outputs are torch tensors on that GPU:
    V float64 [N], omega float64 [K], sigma complex128 [K, N]; G complex128 [K, N]."""

    def __init__(self, dims, t=-1.0, mu=0.0, leaf_edge=16, partition=PART_NESTED,
                 precision=PREC_FP64, max_rank=0, extra_steps=10, max_inner_iters=2000,
                 inner_tol=1e-14, lanczos_tol=1e-11, seed=0x5EED, profile=False, device=0,
                 ctx: "Context | None" = None, level_streams=4, periodic=None,
                 check_sites=2, fault_step=0, fault_attempts=0, breakdown_tol=1e-4,
                 interface_lanczos=0, inner_graphs=0):
        dims = tuple(int(x) for x in dims)
        lat = Lattice()
        lat.dim = len(dims)
        per = tuple(periodic) if periodic is not None else (0,) * len(dims)
        for a in range(3):
            lat.L[a] = dims[a] if a < len(dims) else 1
            lat.periodic[a] = int(per[a]) if a < len(per) else 0
        lat.t, lat.mu = float(t), float(mu)
        o = Opts(leaf_edge, partition, precision, max_rank, extra_steps, max_inner_iters,
                 inner_tol, lanczos_tol, seed, int(profile), int(level_streams),
                 int(check_sites) if check_sites else -1, int(fault_step), int(fault_attempts),
                 float(breakdown_tol), int(interface_lanczos), int(inner_graphs))
        self.dims = dims
        self.n_sites = 1
        for x in dims:
            self.n_sites *= x
        self._own_ctx = ctx is None
        self.context = ctx if ctx is not None else Context(device)
        self.ctx = self.context.handle
        self.plan = dyson_plan_create(self.ctx, lat, o)
        self.info = dyson_plan_get_info(self.plan)

    def trim(self):
        """dyson_plan_trim: gives back the workspace kept between blocking calls."""
        _check(load_library().dyson_plan_trim(self.plan))

    def close(self):
        if getattr(self, "plan", None):
            dyson_plan_destroy(self.plan)
            self.plan = None
        if getattr(self, "_own_ctx", False) and getattr(self, "context", None):
            self.context.close()
        self.context = None
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def levels(self):
        i = self.info
        return [dict(n_nodes=i.n_nodes[l], max_m=i.max_m[l], sum_m=i.sum_m[l])
                for l in range(i.levels)]

    def maps(self):
        return dyson_plan_get_maps(self.plan, self.n_sites)

    def footprint(self, K):
        return dyson_footprint(self.plan, K)

    def domains(self, level):
        """(m, step cap) of every correction domain of the level."""
        return dyson_plan_get_domains(self.plan, level, self.info.n_nodes[level])

    def solve_host(self, V, omega, sigma, G=None, report=False):
        """Host-to-host solve: numpy arrays in (V float64 [N], omega float64 [K],
        sigma complex128 [K, N]), numpy G complex128 [K, N] out."""
        import numpy as np
        V = np.ascontiguousarray(V, np.float64)
        omega = np.ascontiguousarray(omega, np.float64)
        sigma = np.ascontiguousarray(sigma, np.complex128)
        K = int(omega.shape[0])
        if G is None:
            G = np.empty((K, self.n_sites), np.complex128)
        assert G.dtype == np.complex128 and G.flags.c_contiguous
        cp = lambda a: C.c_void_p(a.ctypes.data)  # noqa: E731
        rep = Report()
        dyson_solve_host(self.plan, K, cp(V), cp(omega), cp(sigma), cp(G), _stream(), rep)
        return (G, rep.as_dict()) if report else G

    @staticmethod
    def _c(x):
        import torch
        assert x.is_cuda and x.is_contiguous(), "device tensors required"
        if x.is_complex():
            assert x.dtype == torch.complex128
        else:
            assert x.dtype == torch.float64
        return x

    def solve(self, V, omega, sigma, G=None, report=False):
        import torch
        K = int(omega.shape[0])
        if G is None:
            G = torch.empty((K, self.n_sites), dtype=torch.complex128, device=V.device)
        rep = Report()
        dyson_solve(self.plan, K, _ptr(self._c(V)), _ptr(self._c(omega)), _ptr(self._c(sigma)),
                    _ptr(self._c(G)), _stream(), rep)
        return (G, rep.as_dict()) if report else G

    def solve_noalloc(self, V, omega, sigma, G, report=False):
        """dyson_solve_noalloc: the workspace comes from the device's fixed
        scratch array; G (complex128 [K, N] on the GPU) is the caller's."""
        K = int(omega.shape[0])
        rep = Report()
        dyson_solve_noalloc(self.plan, K, _ptr(self._c(V)), _ptr(self._c(omega)),
                            _ptr(self._c(sigma)), _ptr(self._c(G)), _stream(), rep)
        return (G, rep.as_dict()) if report else G

    def solve_schur(self, V, omega, sigma, G=None, report=False):
        """dyson_solve_schur: diag(H^{-1}) by the explicit Schur complement of a
        one-level decomposition (eq. (6))."""
        import torch
        K = int(omega.shape[0])
        if G is None:
            G = torch.empty((K, self.n_sites), dtype=torch.complex128, device=V.device)
        rep = Report()
        dyson_solve_schur(self.plan, K, _ptr(self._c(V)), _ptr(self._c(omega)),
                          _ptr(self._c(sigma)), _ptr(self._c(G)), _stream(), rep)
        return (G, rep.as_dict()) if report else G

    def noalloc_bytes(self, K):
        return dyson_noalloc_bytes(self.plan, K)

    def solve_z(self, V, z, sigma, G=None, report=False):
        """The solve at complex energies z (complex128 [K], Im z > 0)."""
        import torch
        K = int(z.shape[0])
        assert z.is_cuda and z.dtype == torch.complex128 and z.is_contiguous()
        if G is None:
            G = torch.empty((K, self.n_sites), dtype=torch.complex128, device=V.device)
        rep = Report()
        dyson_solve_z(self.plan, K, _ptr(self._c(V)), _ptr(z), _ptr(self._c(sigma)),
                      _ptr(self._c(G)), _stream(), rep)
        return (G, rep.as_dict()) if report else G

    def assemble(self, V, omega, sigma):
        import torch
        K = int(omega.shape[0])
        d = torch.empty((K, self.n_sites), dtype=torch.complex128, device=V.device)
        dyson_assemble(self.plan, K, _ptr(self._c(V)), _ptr(self._c(omega)),
                       _ptr(self._c(sigma)), _ptr(d), _stream())
        return d

    def leaf_diag(self, d):
        import torch
        G = torch.empty_like(d)
        dyson_leaf_diag(self.plan, int(d.shape[0]), _ptr(self._c(d)), _ptr(G), _stream())
        return G

    def xmatvec(self, level, d, q):
        import torch
        u = torch.empty_like(q)
        dyson_xmatvec(self.plan, level, int(d.shape[0]), _ptr(self._c(d)), _ptr(self._c(q)),
                      _ptr(u), _stream())
        return u

    def submit(self, V, omega, sigma, G=None, mem=MEM_DEVICE):
        """Queue a solve on the context's server.  mem=MEM_DEVICE: torch tensors on
        the GPU (complete when submitted); mem=MEM_HOST: numpy arrays (V float64 [N],
        omega float64 [K], sigma complex128 [K, N]), G a complex128 [K, N] array.
        A complex omega (complex128) is taken as the energies z_k (dyson_submit_z)."""
        import numpy as np
        K = int(omega.shape[0])
        zmode = bool(omega.is_complex()) if hasattr(omega, "is_complex") else \
            np.iscomplexobj(omega)
        if mem == MEM_DEVICE:
            import torch
            if G is None:
                G = torch.empty((K, self.n_sites), dtype=torch.complex128, device=V.device)
            keep = (self._c(V), self._c(omega), self._c(sigma), self._c(G))
            # the server reads the inputs on its own streams: they must be
            # complete when the request is queued
            torch.cuda.current_stream(V.device).synchronize()
            h = dyson_submit(self.plan, K, _ptr(keep[0]), _ptr(keep[1]), _ptr(keep[2]),
                             _ptr(keep[3]), MEM_DEVICE, zmode)
        else:
            V = np.ascontiguousarray(V, np.float64)
            omega = np.ascontiguousarray(omega, np.complex128 if zmode else np.float64)
            sigma = np.ascontiguousarray(sigma, np.complex128)
            if G is None:
                G = np.empty((K, self.n_sites), np.complex128)
            assert G.dtype == np.complex128 and G.flags.c_contiguous
            keep = (V, omega, sigma, G)
            cp = lambda a: C.c_void_p(a.ctypes.data)  # noqa: E731
            h = dyson_submit(self.plan, K, cp(V), cp(omega), cp(sigma), cp(G), MEM_HOST, zmode)
        return Request(h, G, keep, self)

    def correct_level(self, level, d, Gacc):
        import numpy as np
        K = int(d.shape[0])
        steps = np.zeros(K * self.info.n_nodes[level], np.int32)
        dyson_correct_level(self.plan, level, K, _ptr(self._c(d)), _ptr(self._c(Gacc)), steps,
                            _stream())
        return steps.reshape(K, self.info.n_nodes[level])


class Context:
    """A device context; its server runs the requests of every plan made on it."""

    def __init__(self, device=0, hbm_budget=0, slots=None, max_batch_freqs=None,
                 allocator: Allocator | None = None):
        import weakref
        self._alloc = allocator  # the callbacks must outlive the context
        self._plans = weakref.WeakSet()
        self.handle = dyson_create(device, hbm_budget, allocator)
        if slots is not None or max_batch_freqs is not None:
            dyson_serve_config(self.handle, slots or 3, max_batch_freqs or 256)

    def autotune(self, dims, V, omega, sigma, t=-1.0, mu=0.0, periodic=None, **opts):
        """Measured leaf edge and level-stream count for this lattice on the
        probe inputs (torch tensors on the GPU); returns a dict of options for
        plan() and the probe's site*freq/s."""
        lat = Lattice()
        dims = tuple(int(x) for x in dims)
        lat.dim = len(dims)
        per = tuple(periodic) if periodic is not None else (0,) * len(dims)
        for a in range(3):
            lat.L[a] = dims[a] if a < len(dims) else 1
            lat.periodic[a] = int(per[a]) if a < len(per) else 0
        lat.t, lat.mu = float(t), float(mu)
        base = Opts(0, opts.get("partition", PART_NESTED), opts.get("precision", PREC_FP64),
                    opts.get("max_rank", 0), opts.get("extra_steps", 10),
                    opts.get("max_inner_iters", 2000), opts.get("inner_tol", 1e-14),
                    opts.get("lanczos_tol", 1e-11), opts.get("seed", 0x5EED), 0, 0)
        best, rate = Opts(), C.c_double()
        _check(load_library().dyson_autotune(self.handle, C.byref(lat), C.byref(base),
                                             int(omega.shape[0]), _ptr(Plan._c(V)),
                                             _ptr(Plan._c(omega)), _ptr(Plan._c(sigma)),
                                             C.byref(best), C.byref(rate)))
        return {"leaf_edge": best.leaf_edge, "level_streams": best.level_streams,
                "interface_lanczos": best.interface_lanczos, "rate": rate.value}

    def solve_batch(self, items, report=False):
        """dyson_solve_batch: items = [(plan, V, omega, sigma), ...] with torch
        tensors on the GPU (plans of this context); returns the G tensors (and
        the reports)."""
        import torch
        n = len(items)
        outs = []
        arr = lambda vals: (_P * n)(*vals)  # noqa: E731
        for (p, V, om, sig) in items:
            outs.append(torch.empty((int(om.shape[0]), p.n_sites), dtype=torch.complex128,
                                    device=V.device))
        reps = (Report * n)()
        Ks = (C.c_int * n)(*[int(it[2].shape[0]) for it in items])
        _check(load_library().dyson_solve_batch(
            n, arr([it[0].plan for it in items]), Ks,
            arr([Plan._c(it[1]).data_ptr() for it in items]),
            arr([Plan._c(it[2]).data_ptr() for it in items]),
            arr([Plan._c(it[3]).data_ptr() for it in items]),
            arr([g.data_ptr() for g in outs]), _stream(), reps))
        return (outs, [r.as_dict() for r in reps]) if report else outs

    def plan(self, dims, **kw) -> Plan:
        p = Plan(dims, ctx=self, **kw)
        self._plans.add(p)
        return p

    def close(self):
        """Destroys the context after the plans made on it."""
        if getattr(self, "handle", None):
            for p in list(self._plans):
                p.close()
            dyson_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Request:
    """Handle of a submitted solve; G is filled when it finishes successfully.
    It keeps its plan (and the arrays it borrows) alive until released."""

    def __init__(self, handle, G, keep, plan=None):
        self.handle, self.G, self._keep, self._plan = handle, G, keep, plan

    def done(self) -> bool:
        return dyson_poll(self.handle)

    def wait(self, timeout=None):
        """Wait and return G; raises DysonError on failure or timeout."""
        st = dyson_wait(self.handle, -1.0 if timeout is None else float(timeout))
        _check(st)
        return self.G

    def status(self, timeout=None) -> int:
        return dyson_wait(self.handle, -1.0 if timeout is None else float(timeout))

    def cancel(self):
        dyson_cancel(self.handle)

    def report(self) -> dict:
        return dyson_req_report(self.handle).as_dict()

    def release(self):
        if self.handle is not None:
            dyson_release(self.handle)
            self.handle = None
            self._keep = None
            self._plan = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
