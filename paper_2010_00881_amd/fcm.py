"""ctypes binding of libfcm (argument marshalling only).

Every numerical step runs inside libfcm.so; this module converts problem
descriptors to the C structs of include/fcm.h, passes torch device pointers
and the current HIP stream, and converts results back.  There is no CPU
fallback: if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfcm.so")

FCM_FP64, FCM_MIXED = 0, 1
FCM_SMOOTH_ELEMENTWISE, FCM_SMOOTH_PATCHWISE = 0, 1
FCM_COARSE_BLOCKTRI, FCM_COARSE_HMG = 0, 1
FCM_SPACE_TENSOR, FCM_SPACE_TRUNK = 0, 1
STATUS = {0: "ok", 1: "not converged", -1: "invalid argument", -2: "out of device memory",
          -3: "HIP error", -4: "not SPD", -5: "CG breakdown", -6: "non-finite value", -7: "busy"}


class FcmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libfcm status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("p", ctypes.c_int), ("n_fields", ctypes.c_int), ("refine_levels", ctypes.c_int),
        ("geom", ctypes.c_int), ("n_balls", ctypes.c_int),
        ("ball_c", ctypes.POINTER(ctypes.c_double)), ("ball_r", ctypes.POINTER(ctypes.c_double)),
        ("alpha", ctypes.c_double), ("quad_depth", ctypes.c_int),
        ("kappa", ctypes.c_double), ("E", ctypes.c_double), ("nu", ctypes.c_double),
        ("dirichlet_faces", ctypes.c_uint),
        ("n_traction", ctypes.c_int), ("traction_face", ctypes.POINTER(ctypes.c_int)),
        ("traction_vec", ctypes.POINTER(ctypes.c_double)),
        ("n_gauss", ctypes.c_int), ("gauss", ctypes.POINTER(ctypes.c_double)),
        ("f_const", ctypes.c_double), ("body_force", ctypes.c_double * 3),
        ("beta", ctypes.c_double), ("surf_n", ctypes.c_int * 2), ("space", ctypes.c_int),
        ("psi", ctypes.c_double), ("trig_src", ctypes.c_double * 2),
        ("trig_dir", ctypes.c_double * 2),
    ]


class Options(ctypes.Structure):
    _fields_ = [("smoother", ctypes.c_int), ("omega", ctypes.c_double),
                ("n_pre", ctypes.c_int), ("n_post", ctypes.c_int),
                ("precision", ctypes.c_int), ("rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("use_graphs", ctypes.c_int),
                ("autotune", ctypes.c_int), ("coarse", ctypes.c_int),
                ("coarse_dense_max", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("true_rel_res", ctypes.c_double), ("t_setup_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double),
                ("res_history", ctypes.POINTER(ctypes.c_double)), ("n_history", ctypes.c_int)]

    def to_dict(self):
        hist = [self.res_history[i] for i in range(self.n_history)] if self.res_history else []
        return dict(iterations=self.iterations, rel_res=self.rel_res,
                    true_rel_res=self.true_rel_res, t_setup_ms=self.t_setup_ms,
                    t_solve_ms=self.t_solve_ms, history=hist)


class Stats(ctypes.Structure):
    _fields_ = [("n_elements", ctypes.c_int64), ("n_kept", ctypes.c_int64),
                ("n_cut", ctypes.c_int64), ("n_unique_blocks", ctypes.c_int64),
                ("n_shared_classes", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("coarse_blocks", ctypes.c_int), ("coarse_block_size", ctypes.c_int),
                ("n_fp64_blocks", ctypes.c_int64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("memory_budget_bytes", ctypes.c_int64), ("max_active", ctypes.c_int),
                ("n_streams", ctypes.c_int)]


# exported symbols and their signatures (checked by the CPU test-suite)
_P = ctypes.c_void_p
SIGNATURES = {
    "fcm_setup": ([ctypes.POINTER(Problem), ctypes.POINTER(Options), _P, ctypes.POINTER(_P)], ctypes.c_int),
    "fcm_sizes": ([_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64),
                   ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "fcm_rhs": ([_P, _P, _P], ctypes.c_int),
    "fcm_apply": ([_P, ctypes.c_int, _P, _P, _P], ctypes.c_int),
    "fcm_smooth": ([_P, ctypes.c_int, _P, _P, _P], ctypes.c_int),
    "fcm_coarse_solve": ([_P, _P, _P, _P], ctypes.c_int),
    "fcm_spd_inverse": ([_P, ctypes.c_int, ctypes.c_int, _P, _P], ctypes.c_int),
    "fcm_spd_inverse_noalloc": ([_P, ctypes.c_int, ctypes.c_int, _P, _P], ctypes.c_int),
    "fcm_vcycle": ([_P, _P, _P, _P], ctypes.c_int),
    "fcm_pcg_solve": ([_P, _P, _P, ctypes.POINTER(SolveInfo), _P], ctypes.c_int),
    "fcm_pcg_solve_batched": ([ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(_P),
                               ctypes.POINTER(SolveInfo), ctypes.POINTER(ctypes.c_int), _P],
                              ctypes.c_int),
    "fcm_mg_solve": ([_P, _P, _P, ctypes.POINTER(SolveInfo), ctypes.POINTER(ctypes.c_double), _P],
                     ctypes.c_int),
    "fcm_dof_keys": ([_P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "fcm_local_modes": ([_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "fcm_element": ([_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                     ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "fcm_get_stats": ([_P, ctypes.POINTER(Stats)], ctypes.c_int),
    "fcm_get_tuning": ([_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                        ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "fcm_set_tuning": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "fcm_time_op": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, ctypes.POINTER(ctypes.c_double),
                     ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "fcm_destroy": ([_P], None),
    "fcm_trim_pool": ([], ctypes.c_int),
    "fcm_hlevels": ([_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "fcm_server_create": ([ctypes.POINTER(ServerOpts), ctypes.POINTER(_P)], ctypes.c_int),
    "fcm_serve_submit": ([_P, ctypes.POINTER(Problem), ctypes.POINTER(Options),
                          ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "fcm_serve_poll": ([_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                        ctypes.c_int64, ctypes.POINTER(SolveInfo), ctypes.POINTER(ctypes.c_double)],
                       ctypes.c_int),
    "fcm_server_destroy": ([_P], ctypes.c_int),
    "fcm_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "fcm_last_error": ([], ctypes.c_char_p),
}

_LIB = None


def lib():
    """Load libfcm.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2010_00881_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = L
    return _LIB


def _check(st, allow=(0, 1)):
    if st not in allow:
        raise FcmError(st, lib().fcm_last_error().decode())
    return st


def _dptr(arr):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _ProblemData:
    """Problem struct plus the host arrays it points to (kept alive)."""

    def __init__(self, desc):
        d = int(desc["dim"])
        self.ball_c = np.ascontiguousarray(np.asarray(desc.get("ball_c", []), dtype=np.float64).reshape(-1))
        self.ball_r = np.ascontiguousarray(np.asarray(desc.get("ball_r", []), dtype=np.float64))
        g = []
        for A, w, c in desc.get("gauss", []):
            cc = list(c) + [0.0] * (3 - len(c))
            g.append([A, w] + cc[:3])
        self.gauss = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1))
        tr = desc.get("tractions", [])
        self.tface = np.ascontiguousarray(np.asarray([f for f, _ in tr], dtype=np.int32))
        tv = []
        for _, t in tr:
            tv += list(t) + [0.0] * (3 - len(t))
        self.tvec = np.ascontiguousarray(np.asarray(tv, dtype=np.float64))
        P = Problem()
        P.dim = d
        for ax in range(3):
            P.n[ax] = int(desc["n"][ax]) if ax < d else 1
            P.lo[ax] = float(desc["lo"][ax]) if ax < d else 0.0
            P.hi[ax] = float(desc["hi"][ax]) if ax < d else 1.0
        P.p = int(desc["p"])
        P.n_fields = int(desc.get("n_fields", 1))
        P.refine_levels = int(desc.get("refine_levels", 0))
        P.geom = int(desc.get("geom", 0))
        P.n_balls = int(self.ball_r.size)
        P.ball_c = _dptr(self.ball_c)
        P.ball_r = _dptr(self.ball_r)
        P.alpha = float(desc["alpha"])
        P.quad_depth = int(desc.get("quad_depth", 3))
        P.kappa = float(desc.get("kappa", 1.0))
        P.E = float(desc.get("E", 1.0))
        P.nu = float(desc.get("nu", 0.3))
        P.dirichlet_faces = int(desc.get("dirichlet_faces", 0))
        P.n_traction = int(self.tface.size)
        P.traction_face = self.tface.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        P.traction_vec = _dptr(self.tvec)
        P.n_gauss = len(g)
        P.gauss = _dptr(self.gauss)
        P.f_const = float(desc.get("f_const", 0.0))
        bf = list(desc.get("body_force", [0.0] * d)) + [0.0] * 3
        for i in range(3):
            P.body_force[i] = float(bf[i])
        P.beta = float(desc.get("beta", 0.0))
        sn = desc.get("surface_rule", (0, 0))
        P.surf_n[0], P.surf_n[1] = int(sn[0]), int(sn[1])
        sp = desc.get("space", "tensor")
        if sp not in ("tensor", "trunk"):
            raise ValueError(f"unknown space {sp!r}")
        P.space = 1 if sp == "trunk" else 0
        P.psi = float(desc.get("psi", 0.0))
        for name in ("trig_src", "trig_dir"):
            v = desc.get(name) or (0.0, 0.0)
            getattr(P, name)[0], getattr(P, name)[1] = float(v[0]), float(v[1])
        self.struct = P


def make_options(opts):
    o = Options()
    sm = opts.get("smoother", "elementwise")
    if sm not in ("elementwise", "patchwise"):
        raise ValueError(f"unknown smoother {sm!r}")
    o.smoother = FCM_SMOOTH_PATCHWISE if sm == "patchwise" else FCM_SMOOTH_ELEMENTWISE
    o.omega = float(opts["omega"])
    o.n_pre = int(opts.get("n_pre", 5))
    o.n_post = int(opts.get("n_post", 5))
    prec = opts.get("precision", "fp64")
    o.precision = FCM_MIXED if prec in ("mixed", "fp32", FCM_MIXED) else FCM_FP64
    o.rtol = float(opts.get("rtol", 1e-10))
    o.max_iter = int(opts.get("max_iter", 500))
    o.use_graphs = int(opts.get("use_graphs", 1))
    o.autotune = int(opts.get("autotune", 1))
    co = opts.get("coarse", "blocktri")
    if co not in ("blocktri", "hmg"):
        raise ValueError(f"unknown coarse solve {co!r}")
    o.coarse = FCM_COARSE_HMG if co == "hmg" else FCM_COARSE_BLOCKTRI
    o.coarse_dense_max = int(opts.get("coarse_dense_max", 0))
    return o


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One FCM problem set up on the GPU (owns an fcm_handle)."""

    def __init__(self, desc, opts):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libfcm needs a GPU (torch.cuda.is_available() is False)")
        self.desc = desc
        self._pd = _ProblemData(desc)
        self._opts = make_options(opts)
        h = ctypes.c_void_p()
        _check(lib().fcm_setup(ctypes.byref(self._pd.struct), ctypes.byref(self._opts), _stream(),
                               ctypes.byref(h)), allow=(0,))
        self.h = h
        n = ctypes.c_int()
        npd = (ctypes.c_int64 * 8)()
        _check(lib().fcm_sizes(self.h, ctypes.byref(n), None, npd))
        self.n_levels = n.value
        self.n_padded = [npd[i] for i in range(n.value)]
        self._n_dofs = None

    @property
    def n_dofs(self):
        """Unknowns per level, coarse first (counted on the host on first use)."""
        if self._n_dofs is None:
            n = ctypes.c_int()
            nd = (ctypes.c_int64 * 8)()
            _check(lib().fcm_sizes(self.h, ctypes.byref(n), nd, None))
            self._n_dofs = [nd[i] for i in range(n.value)]
        return self._n_dofs

    def close(self):
        if getattr(self, "h", None):
            # the handle's memory is released in order on its setup stream;
            # work queued with it on other streams must finish first
            import torch
            torch.cuda.synchronize()
            lib().fcm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- data
    def _new(self, level=None):
        import torch
        lv = self.n_levels - 1 if level is None else level
        return torch.zeros(self.n_padded[lv], dtype=torch.float64, device="cuda")

    def rhs(self):
        b = self._new()
        _check(lib().fcm_rhs(self.h, _ptr(b), _stream()))
        return b

    def apply(self, level, x):
        y = self._new(level)
        _check(lib().fcm_apply(self.h, level, _ptr(x), _ptr(y), _stream()))
        return y

    def smooth(self, level, r):
        z = self._new(level)
        _check(lib().fcm_smooth(self.h, level, _ptr(r), _ptr(z), _stream()))
        return z

    def hlevels(self):
        """Cells per axis of the geometric h-levels (h-level 0 = the p = 1 level);
        empty without them."""
        cnt = ctypes.c_int(0)
        cells = (ctypes.c_int * 36)()
        _check(lib().fcm_hlevels(self.h, ctypes.byref(cnt), cells))
        return [tuple(cells[3 * k + a] for a in range(3)) for k in range(cnt.value)]

    def _hnew(self, k):
        import torch
        n = self.hlevels()[k]
        nf = int(self.desc.get("n_fields", 1))
        return torch.zeros(nf * (n[0] + 1) * (n[1] + 1) * (n[2] + 1), dtype=torch.float64,
                           device="cuda")

    def happly(self, k, x):
        """y = A_k x on h-level k >= 1 (Galerkin matrix)."""
        y = self._hnew(k)
        _check(lib().fcm_apply(self.h, -k, _ptr(x), _ptr(y), _stream()))
        return y

    def hsmooth(self, k, r):
        """z = M_k^{-1} r, the patchwise Schwarz operator of h-level k."""
        z = self._hnew(k)
        _check(lib().fcm_smooth(self.h, -k, _ptr(r), _ptr(z), _stream()))
        return z

    def coarse_solve(self, b):
        x = self._new(0)
        _check(lib().fcm_coarse_solve(self.h, _ptr(b), _ptr(x), _stream()))
        return x

    def vcycle(self, r):
        z = self._new()
        _check(lib().fcm_vcycle(self.h, _ptr(r), _ptr(z), _stream()))
        return z

    def pcg(self, b=None, x=None):
        x = self._new() if x is None else x
        info = SolveInfo()
        st = _check(lib().fcm_pcg_solve(self.h, None if b is None else _ptr(b), _ptr(x),
                                        ctypes.byref(info), _stream()))
        d = info.to_dict()
        d["status"] = st
        return x, d

    def mg_solve(self, b=None):
        x = self._new()
        info = SolveInfo()
        rho = ctypes.c_double()
        st = _check(lib().fcm_mg_solve(self.h, None if b is None else _ptr(b), _ptr(x),
                                       ctypes.byref(info), ctypes.byref(rho), _stream()))
        d = info.to_dict()
        d["status"] = st
        d["rho_max"] = rho.value
        return x, d

    # -------------------------------------------------------------- tables
    def dof_keys(self):
        keys = np.empty(self.n_padded[-1], dtype=np.int64)
        _check(lib().fcm_dof_keys(self.h, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return keys

    def local_modes(self):
        m = ctypes.c_int()
        _check(lib().fcm_local_modes(self.h, ctypes.byref(m), None))
        out = np.empty((m.value, 4), dtype=np.int32)
        _check(lib().fcm_local_modes(self.h, ctypes.byref(m),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return out

    def element(self, e):
        m = self.local_modes().shape[0]
        K = np.zeros((m, m))
        be = np.zeros(m)
        st = ctypes.c_int()
        _check(lib().fcm_element(self.h, int(e), ctypes.byref(st), _dptr(K), _dptr(be)))
        return st.value, K, be

    OPS = {"smooth": 0, "residual": 1, "coarse": 2, "vcycle": 3, "smooth_stored": 4}

    def time_op(self, op, level=None, reps=20):
        """(ms per launch, algorithmic bytes per launch) timed with HIP events."""
        lv = self.n_levels - 1 if level is None else level
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(lib().fcm_time_op(self.h, self.OPS[op], lv, int(reps), _stream(), ctypes.byref(ms),
                                 ctypes.byref(by)))
        return ms.value, by.value

    def tuning(self, level):
        """Launch variants of the patchwise smoother of a level (autotuner)."""
        cr, gb, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().fcm_get_tuning(self.h, int(level), ctypes.byref(cr), ctypes.byref(gb),
                                    ctypes.byref(ms)))
        return {"class_rows": cr.value, "gemv_band": gb.value, "tune_ms": ms.value}

    def set_tuning(self, level, class_rows=-1, gemv_band=-1):
        _check(lib().fcm_set_tuning(self.h, int(level), int(class_rows), int(gemv_band)))

    def stats(self):
        s = Stats()
        _check(lib().fcm_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}


class Server:
    """Continuous-batching request loop (fcm_server_*)."""

    def __init__(self, memory_budget_bytes=64 << 30, max_active=16, n_streams=4):
        o = ServerOpts(int(memory_budget_bytes), int(max_active), int(n_streams))
        s = ctypes.c_void_p()
        _check(lib().fcm_server_create(ctypes.byref(o), ctypes.byref(s)), allow=(0,))
        self.s = s
        self._keep = {}

    def submit(self, desc, opts):
        pd = _ProblemData(desc)
        o = make_options(opts)
        rid = ctypes.c_uint64()
        _check(lib().fcm_serve_submit(self.s, ctypes.byref(pd.struct), ctypes.byref(o),
                                      ctypes.byref(rid)), allow=(0,))
        return rid.value

    def poll(self, rid, n_padded=None):
        done = ctypes.c_int()
        info = SolveInfo()
        lat = ctypes.c_double()
        x = None
        xp = None
        if n_padded:
            x = np.zeros(n_padded)
            xp = _dptr(x)
        st = lib().fcm_serve_poll(self.s, ctypes.c_uint64(rid), ctypes.byref(done), xp,
                                  int(n_padded or 0), ctypes.byref(info), ctypes.byref(lat))
        if not done.value:
            return None
        d = info.to_dict()
        d["status"] = st
        d["latency_ms"] = lat.value
        d["x"] = x
        if st < 0:
            d["error"] = lib().fcm_last_error().decode()
        return d

    def close(self):
        if getattr(self, "s", None):
            lib().fcm_server_destroy(self.s)
            self.s = None


def trim_pool():
    """Return the cached, unused device memory of the library's pool."""
    _check(lib().fcm_trim_pool())


def pcg_batched(solvers):
    """MG-PCG of several problems, each CG step of all of them one graph launch
    (fcm_pcg_solve_batched).  Returns [(x, info), ...] in the order given."""
    n = len(solvers)
    xs = [s._new() for s in solvers]
    hs = (_P * n)(*[s.h for s in solvers])
    xp = (_P * n)(*[_ptr(x) for x in xs])
    infos = (SolveInfo * n)()
    sts = (ctypes.c_int * n)()
    _check(lib().fcm_pcg_solve_batched(hs, n, xp, infos, sts, _stream()))
    out = []
    for i in range(n):
        d = infos[i].to_dict()
        d["status"] = sts[i]
        out.append((xs[i], d))
    return out


def spd_inverse(A, kappa=None):
    """In-place batched inverse of SPD matrices on the device (test hook).

    A: CUDA float64 tensor of shape (batch, n, n), contiguous; kappa: optional
    CUDA float64 tensor of shape (batch,) receiving the scaled 1-norm condition
    numbers."""
    assert A.is_cuda and A.dtype.is_floating_point and A.element_size() == 8 and A.is_contiguous()
    b, n, n2 = A.shape
    assert n == n2
    _check(lib().fcm_spd_inverse(_ptr(A), n, b, _ptr(kappa) if kappa is not None else None,
                                 _stream()))
    return A


def spd_inverse_noalloc(A, kappa=None):
    """spd_inverse through the allocation-free entry point (static device
    scratch of 4 Mi doubles; see fcm_spd_inverse_noalloc)."""
    assert A.is_cuda and A.dtype.is_floating_point and A.element_size() == 8 and A.is_contiguous()
    b, n, n2 = A.shape
    assert n == n2
    _check(lib().fcm_spd_inverse_noalloc(_ptr(A), n, b,
                                         _ptr(kappa) if kappa is not None else None, _stream()))
    return A
