"""Python binding of libeifmm.so (include/eifmm.h): argument marshalling only.

Every step of the evaluation runs in the library's HIP kernels; this module
passes device pointers of PyTorch tensors and the current HIP stream.  There is
no fallback: if the built library is missing, loading fails with an error.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeifmm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "eifmm.h")

KERNELS = {"laplace": 0, "yukawa": 1, "gauss": 2, "sqdist": 3, "cosr": 4, "mq": 5,
           "advdiff": 6}
PRECISIONS = {"fp64": 0, "mixed": 1}
FLAG_HOST_ONLY = 1
FLAG_HOST_SETUP = 2
FLAG_TWO_EIM = 4
MAX_DEPTH = 8
NPHASE = 10
PHASES = ["tree", "p2p", "p2m", "m2m", "what", "m2l", "l2l", "lhat", "l2p", "proj"]
STATUS = {0: "OK", -1: "EINVAL", -2: "EDOMAIN", -3: "ESTATE", -4: "EEIM", -5: "ENOMEM",
          -6: "EHIP"}


class EifmmError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)} ({_status_str(code)})")


class Config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("kernel_param", ctypes.c_double), ("lo", ctypes.c_double * 3),
                ("L", ctypes.c_double), ("n", ctypes.c_int64), ("depth", ctypes.c_int32),
                ("max_rhs", ctypes.c_int32), ("eim_tol", ctypes.c_double),
                ("tol_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("dmax", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("compress_tol", ctypes.c_double), ("n_targets", ctypes.c_int64),
                ("compress_tol2", ctypes.c_double), ("scale_level", ctypes.c_int32),
                ("reserved_cfg", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("d", ctypes.c_int32 * (MAX_DEPTH + 1)), ("dpad", ctypes.c_int32 * (MAX_DEPTH + 1)),
                ("rank", ctypes.c_int32 * (MAX_DEPTH + 1)),
                ("eim_err", ctypes.c_double * (MAX_DEPTH + 1)), ("setup_ms", ctypes.c_double),
                ("phase_ms", ctypes.c_double * NPHASE), ("phase_calls", ctypes.c_int64 * NPHASE),
                ("m2l_flops", ctypes.c_double), ("proj_flops", ctypes.c_double),
                ("active_boxes", ctypes.c_int64 * (MAX_DEPTH + 1)),
                ("il_pairs", ctypes.c_int64 * (MAX_DEPTH + 1)), ("near_pairs", ctypes.c_int64),
                ("hip_error", ctypes.c_int32), ("scale_level", ctypes.c_int32),
                ("near_point_pairs", ctypes.c_int64), ("d2", ctypes.c_int32 * (MAX_DEPTH + 1)),
                ("rpad", ctypes.c_int32 * (MAX_DEPTH + 1)), ("near_mode", ctypes.c_int32),
                ("m2l_flops_exec", ctypes.c_double)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("nprob", ctypes.c_int32),
                ("ntables", ctypes.c_int32), ("graph_nodes", ctypes.c_int32),
                ("m2l_rbt", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("m2l_flops", ctypes.c_double), ("tune_ms", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("reserved", ctypes.c_double * 4)]


_lib = None


def lib():
    """Load the built library (no build here: run __graft_entry__.build() first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # PyTorch ships its own HIP runtime and links it by an unversioned name; it
        # has to be loaded first so the library binds to that same runtime instead
        # of a second copy (two runtimes in one process do not share the device).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.eifmm_plan_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(vp)]
        L.eifmm_set_points.argtypes = [vp, vp, vp]
        L.eifmm_set_points_targets.argtypes = [vp, vp, vp, vp]
        L.eifmm_evaluate.argtypes = [vp, vp, i32, i64, vp, i64, vp]
        L.eifmm_evaluate_noalloc.argtypes = [vp, vp, i32, i64, vp, i64, vp]
        L.eifmm_set_timing.argtypes = [vp, i32]
        L.eifmm_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.eifmm_get_level.argtypes = [vp, i32, ctypes.POINTER(i32), vp, vp, vp, vp, vp, vp]
        L.eifmm_get_level2.argtypes = L.eifmm_get_level.argtypes
        L.eifmm_get_compression2.argtypes = [vp, i32, vp]
        L.eifmm_get_compression.argtypes = [vp, i32, ctypes.POINTER(i32), vp, vp]
        L.eifmm_export_tree.argtypes = [vp, vp, vp, vp]
        L.eifmm_export_lists.argtypes = [vp, i32, ctypes.POINTER(i64), vp, vp, vp, vp, vp, vp]
        L.eifmm_export_expansion.argtypes = [vp, i32, i32, i32, vp]
        L.eifmm_plan_destroy.argtypes = [vp]
        L.eifmm_batch_create.argtypes = [ctypes.POINTER(Config), i32, ctypes.POINTER(vp)]
        L.eifmm_batch_set_points.argtypes = [vp, vp, vp]
        L.eifmm_batch_evaluate.argtypes = [vp, vp, vp, vp]
        L.eifmm_batch_evaluate_unfused.argtypes = [vp, vp, vp, vp]
        L.eifmm_batch_export_expansion.argtypes = [vp, i32, i32, i32, vp]
        L.eifmm_batch_get_stats.argtypes = [vp, i32, ctypes.POINTER(Stats)]
        L.eifmm_batch_get_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
        L.eifmm_batch_destroy.argtypes = [vp]
        L.eifmm_status_str.argtypes = [ctypes.c_int]
        L.eifmm_status_str.restype = ctypes.c_char_p
        for f in ("eifmm_plan_create", "eifmm_set_points", "eifmm_set_points_targets",
                  "eifmm_evaluate", "eifmm_evaluate_noalloc", "eifmm_set_timing",
                  "eifmm_get_stats", "eifmm_get_level", "eifmm_get_level2",
                  "eifmm_get_compression", "eifmm_get_compression2",
                  "eifmm_export_tree", "eifmm_export_lists",
                  "eifmm_export_expansion", "eifmm_plan_destroy", "eifmm_batch_create",
                  "eifmm_batch_set_points", "eifmm_batch_evaluate",
                  "eifmm_batch_evaluate_unfused", "eifmm_batch_export_expansion",
                  "eifmm_batch_get_stats",
                  "eifmm_batch_get_info", "eifmm_batch_destroy"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _status_str(code):
    try:
        return lib().eifmm_status_str(code).decode()
    except Exception:  # library not loadable
        return "?"


def _check(code, what):
    if code != 0:
        raise EifmmError(code, what)


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_config(kernel, param, lo, L, n, depth, tau, max_rhs=1, precision="fp64", tol_mode=0,
                dmax=0, host_only=False, compress_tol=0.0, n_targets=0, host_setup=False,
                two_eim=False, compress_tol2=0.0, scale_level=0):
    c = Config()
    c.struct_size = ctypes.sizeof(Config)
    c.kernel = KERNELS[kernel]
    c.kernel_param = float(param)
    for a in range(3):
        c.lo[a] = float(lo[a])
    c.L = float(L)
    c.n = int(n)
    c.depth = int(depth)
    c.max_rhs = int(max_rhs)
    c.eim_tol = float(tau)
    c.tol_mode = int(tol_mode)
    c.precision = PRECISIONS[precision]
    c.dmax = int(dmax)
    c.flags = ((FLAG_HOST_ONLY if host_only else 0) | (FLAG_HOST_SETUP if host_setup else 0)
               | (FLAG_TWO_EIM if two_eim else 0))
    c.compress_tol = float(compress_tol)
    c.n_targets = int(n_targets)
    c.compress_tol2 = float(compress_tol2)
    c.scale_level = int(scale_level)
    return c


def _stats_dict(s, depth):
    lv = range(2, depth + 1)
    return dict(depth=s.depth, d={k: s.d[k] for k in lv}, dpad={k: s.dpad[k] for k in lv},
                rank={k: s.rank[k] for k in lv}, rpad={k: s.rpad[k] for k in lv},
                proj_flops=s.proj_flops, m2l_flops_exec=s.m2l_flops_exec,
                near_mode=s.near_mode,
                scale_level=s.scale_level,
                eim_err={k: s.eim_err[k] for k in lv}, setup_ms=s.setup_ms,
                phase_ms={PHASES[q]: s.phase_ms[q] for q in range(NPHASE)},
                phase_calls={PHASES[q]: s.phase_calls[q] for q in range(NPHASE)},
                m2l_flops=s.m2l_flops,
                active_boxes={k: s.active_boxes[k] for k in range(depth + 1)},
                il_pairs={k: s.il_pairs[k] for k in lv}, near_pairs=s.near_pairs,
                d2={k: s.d2[k] for k in lv},
                near_point_pairs=s.near_point_pairs, hip_error=s.hip_error)


class Plan:
    """One fixed (kernel, domain, N, depth, tau) setting; points and potentials vary.
    n_targets > 0: f is evaluated at that many separate targets (set_points with
    targets=...)."""

    def __init__(self, kernel, param, lo, L, n, depth, tau, max_rhs=1, precision="fp64",
                 tol_mode=0, dmax=0, host_only=False, compress_tol=0.0, n_targets=0,
                 host_setup=False, two_eim=False, compress_tol2=0.0, scale_level=0):
        c = make_config(kernel, param, lo, L, n, depth, tau, max_rhs, precision, tol_mode, dmax,
                        host_only, compress_tol, n_targets, host_setup, two_eim, compress_tol2,
                        scale_level)
        self.cfg = c
        self.n, self.depth, self.max_rhs = int(n), int(depth), int(max_rhs)
        self.n_targets = int(n_targets)
        self.n_out = self.n_targets if self.n_targets else self.n
        self.kernel, self.precision = kernel, precision
        h = ctypes.c_void_p()
        _check(lib().eifmm_plan_create(ctypes.byref(c), ctypes.byref(h)), "eifmm_plan_create")
        self._h = h

    # -- per query -----------------------------------------------------------
    def set_points(self, xyz, targets=None):
        """xyz: CUDA float64 tensor of shape (3, n), contiguous (the sources); targets:
        (3, n_targets) for a plan with separate targets."""
        self.check_in(xyz, (3, self.n), "xyz")
        if targets is None:
            _check(lib().eifmm_set_points(self._h, ctypes.c_void_p(xyz.data_ptr()), _stream()),
                   "eifmm_set_points")
            return
        self.check_in(targets, (3, self.n_targets), "targets")
        _check(lib().eifmm_set_points_targets(self._h, ctypes.c_void_p(xyz.data_ptr()),
                                              ctypes.c_void_p(targets.data_ptr()), _stream()),
               "eifmm_set_points_targets")

    def evaluate(self, sigma, out=None):
        """sigma: CUDA float64 tensor (n,) or (nrhs, n) (column-major n x nrhs).
        Returns f, (m,) or (nrhs, m) with m the target count, in input order."""
        import torch
        nrhs = self.check_sigma(sigma, self.n)
        shape = (self.n_out,) if sigma.dim() == 1 else (nrhs, self.n_out)
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=sigma.device)
        else:
            # the library writes nrhs columns of n_out doubles at out's address
            self.check_out(out, shape, sigma.device)
        _check(lib().eifmm_evaluate(self._h, ctypes.c_void_p(sigma.data_ptr()), nrhs, self.n,
                                    ctypes.c_void_p(out.data_ptr()), self.n_out, _stream()),
               "eifmm_evaluate")
        return out

    def evaluate_noalloc(self, sigma, out):
        """eifmm_evaluate_noalloc: as evaluate, into a caller-allocated `out`, with
        no device allocation inside the call."""
        nrhs = self.check_sigma(sigma, self.n)
        shape = (self.n_out,) if sigma.dim() == 1 else (nrhs, self.n_out)
        self.check_out(out, shape, sigma.device)
        _check(lib().eifmm_evaluate_noalloc(self._h, ctypes.c_void_p(sigma.data_ptr()), nrhs,
                                            self.n, ctypes.c_void_p(out.data_ptr()), self.n_out,
                                            _stream()), "eifmm_evaluate_noalloc")
        return out

    @staticmethod
    def check_in(t, shape, name):
        """A tensor the library reads (or, for a batch's outputs, writes): float64,
        contiguous, of the expected shape, on a GPU (raises ValueError otherwise,
        before any launch)."""
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64:
            raise ValueError(f"{name} must be a float64 tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_cuda:
            raise ValueError(f"{name} must be on a GPU, not {t.device}")

    @staticmethod
    def check_sigma(sigma, n):
        """Checks sigma, (n,) or (nrhs, n), as check_in does; returns nrhs."""
        import torch
        if not isinstance(sigma, torch.Tensor) or sigma.dim() not in (1, 2):
            raise ValueError("sigma must be a tensor of shape (n,) or (nrhs, n)")
        Plan.check_in(sigma, (n,) if sigma.dim() == 1 else (sigma.shape[0], n), "sigma")
        return 1 if sigma.dim() == 1 else int(sigma.shape[0])

    @staticmethod
    def check_out(out, shape, device):
        """An output tensor the library may write: float64, contiguous, on the
        device of sigma, of the expected shape (raises ValueError otherwise)."""
        import torch
        if not isinstance(out, torch.Tensor) or out.dtype != torch.float64:
            raise ValueError("out must be a float64 tensor")
        if not out.is_contiguous():
            raise ValueError("out must be contiguous")
        if out.device != device:
            raise ValueError(f"out is on {out.device}, sigma on {device}")
        if tuple(out.shape) != tuple(shape):
            raise ValueError(f"out has shape {tuple(out.shape)}, expected {tuple(shape)}")

    def evaluate_raw(self, sigma_ptr, nrhs, ld, f_ptr, ldf, stream=None):
        """Direct pass-through of eifmm_evaluate (for tests of the argument checks)."""
        return lib().eifmm_evaluate(self._h, sigma_ptr, nrhs, ld, f_ptr, ldf, stream)

    # -- statistics and exports ------------------------------------------------
    def set_timing(self, on=True):
        """on: True (every phase), False, or "m2l" (the M2L launch only)."""
        mode = 2 if on == "m2l" else (1 if on else 0)
        _check(lib().eifmm_set_timing(self._h, mode), "eifmm_set_timing")

    def stats(self):
        s = Stats()
        s.struct_size = ctypes.sizeof(Stats)
        _check(lib().eifmm_get_stats(self._h, ctypes.byref(s)), "eifmm_get_stats")
        return _stats_dict(s, self.depth)

    def level(self, k, second=False):
        """EIM data of level k (second=True: the second EIM of a two-EIM plan)."""
        fn = lib().eifmm_get_level2 if second else lib().eifmm_get_level
        d = ctypes.c_int32()
        _check(fn(self._h, k, ctypes.byref(d), None, None, None, None, None, None),
               "eifmm_get_level")
        d = d.value
        X, Y = np.empty((d, 3)), np.empty((d, 3))
        ia, ib = np.empty(d, dtype=np.int64), np.empty(d, dtype=np.int64)
        B, G = np.empty((d, d)), np.empty((d, d))
        _check(fn(self._h, k, None, _np_ptr(X), _np_ptr(Y), _np_ptr(ia), _np_ptr(ib),
                  _np_ptr(B), _np_ptr(G)), "eifmm_get_level")
        return dict(d=d, X=X, Y=Y, ia=ia, ib=ib, B=B, G=G)

    def compression2(self, k):
        """Second-stage ranks of level k (316, offset-id order; zeros when off)."""
        out = np.zeros(316, dtype=np.int32)
        _check(lib().eifmm_get_compression2(self._h, k, _np_ptr(out)), "eifmm_get_compression2")
        return out

    def compression(self, k):
        """(r, singular values, U) of level k's M2L compression; U has one row per
        M2L row point (the second EIM's size when there are two EIMs)."""
        d = self.stats()["d2"][k] or self.level(k)["d"]  # d2 is 0 with one EIM
        r = ctypes.c_int32()
        _check(lib().eifmm_get_compression(self._h, k, ctypes.byref(r), None, None),
               "eifmm_get_compression")
        sv, U = np.empty(d), np.empty((d, max(r.value, 0)))
        _check(lib().eifmm_get_compression(self._h, k, None, _np_ptr(sv), _np_ptr(U)),
               "eifmm_get_compression")
        return r.value, sv, U

    def export_tree(self):
        m = self.n + self.n_targets
        perm = np.empty(m, dtype=np.int32)
        keys = np.empty(m, dtype=np.uint32)
        ls = np.empty((1 << (3 * self.depth)) + 1, dtype=np.int64)
        _check(lib().eifmm_export_tree(self._h, _np_ptr(perm), _np_ptr(ls), _np_ptr(keys)),
               "eifmm_export_tree")
        return perm, ls, keys

    def export_lists(self, level):
        nb = 1 << (3 * level)
        na = ctypes.c_int64()
        active = np.empty(nb, dtype=np.uint32)
        near_ptr = np.empty(nb + 1, dtype=np.int64)
        near_src = np.empty(27 * nb, dtype=np.uint32)
        il_ptr = np.empty(nb + 1, dtype=np.int64)
        il_src = np.empty(189 * nb, dtype=np.uint32)
        il_off = np.empty(189 * nb, dtype=np.int16)
        _check(lib().eifmm_export_lists(self._h, level, ctypes.byref(na), _np_ptr(active),
                                        _np_ptr(near_ptr), _np_ptr(near_src), _np_ptr(il_ptr),
                                        _np_ptr(il_src), _np_ptr(il_off)), "eifmm_export_lists")
        a = na.value
        nn, ni = int(near_ptr[a]), int(il_ptr[a])
        return dict(active=active[:a].copy(), near_ptr=near_ptr[:a + 1].copy(),
                    near_src=near_src[:nn].copy(), il_ptr=il_ptr[:a + 1].copy(),
                    il_src=il_src[:ni].copy(), il_off=il_off[:ni].copy())

    def export_expansion(self, which, k, rhs=0):
        """which in ('W', 'What', 'g', 'l', 'lhat'): dense (8^k, d_k) array."""
        w = ["W", "What", "g", "l", "lhat"].index(which)
        d = self.level(k)["d"]
        if w >= 2:  # g, l and lhat have the second EIM's size, if there is one
            d2 = self.stats()["d2"][k]
            d = d2 if d2 else d
        out = np.empty((1 << (3 * k), d))
        _check(lib().eifmm_export_expansion(self._h, w, k, rhs, _np_ptr(out)),
               "eifmm_export_expansion")
        return out

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.eifmm_plan_destroy(h)
        self._h = None

    def __del__(self):
        self.close()


class Batch:
    """Independent problems evaluated together (eifmm_batch_*).

    problems: list of dicts with keys kernel, param, n, tau and optionally depth
    (None or -1: autotuned), tol_mode, compress_tol, lo, L, dmax; precision is
    one for the whole batch."""

    def __init__(self, problems, precision="fp64"):
        n = len(problems)
        arr = (Config * n)()
        for i, q in enumerate(problems):
            depth = q.get("depth")
            arr[i] = make_config(q["kernel"], q.get("param", 0.0), q.get("lo", (0, 0, 0)),
                                 q.get("L", 1.0), q["n"], -1 if depth is None else depth,
                                 q["tau"], 1, precision, q.get("tol_mode", 0), q.get("dmax", 0),
                                 False, q.get("compress_tol", 0.0),
                                 scale_level=q.get("scale_level", 0))
        self.ns = [int(q["n"]) for q in problems]
        self.nprob = n
        h = ctypes.c_void_p()
        _check(lib().eifmm_batch_create(arr, n, ctypes.byref(h)), "eifmm_batch_create")
        self._h = h

    @staticmethod
    def _ptrs(tensors, ns, shape):
        if len(tensors) != len(ns):
            raise ValueError(f"{len(tensors)} tensors for {len(ns)} problems")
        a = (ctypes.c_void_p * len(ns))()
        for i, (t, n) in enumerate(zip(tensors, ns)):
            Plan.check_in(t, shape(n), f"tensor of problem {i}")
            a[i] = t.data_ptr() if n > 0 else None
        return a

    def set_points(self, xyz):
        """xyz: list of CUDA float64 tensors of shape (3, n_p)."""
        self._xyz = list(xyz)  # the library reads them during the call only
        p = self._ptrs(self._xyz, self.ns, lambda n: (3, n))
        _check(lib().eifmm_batch_set_points(self._h, p, _stream()), "eifmm_batch_set_points")

    def evaluate(self, sigma, out=None):
        """sigma: list of CUDA float64 tensors (n_p,); returns the list of f."""
        import torch
        if out is None:
            out = [torch.empty_like(t) for t in sigma]
        ps = self._ptrs(sigma, self.ns, lambda n: (n,))
        pf = self._ptrs(out, self.ns, lambda n: (n,))
        _check(lib().eifmm_batch_evaluate(self._h, ps, pf, _stream()), "eifmm_batch_evaluate")
        return out

    def evaluate_unfused(self, sigma, out=None):
        """Each problem's own pass in sequence (no fusion, no graph)."""
        import torch
        if out is None:
            out = [torch.empty_like(t) for t in sigma]
        ps = self._ptrs(sigma, self.ns, lambda n: (n,))
        pf = self._ptrs(out, self.ns, lambda n: (n,))
        _check(lib().eifmm_batch_evaluate_unfused(self._h, ps, pf, _stream()),
               "eifmm_batch_evaluate_unfused")
        return out

    def export_expansion(self, p, which, k):
        """Expansion of problem p after an evaluation, as Plan.export_expansion."""
        w = ["W", "What", "g", "l", "lhat"].index(which)
        d = self.stats(p)["d"][k]
        out = np.empty((1 << (3 * k), d))
        _check(lib().eifmm_batch_export_expansion(self._h, p, w, k, _np_ptr(out)),
               "eifmm_batch_export_expansion")
        return out

    def stats(self, p):
        s = Stats()
        s.struct_size = ctypes.sizeof(Stats)
        _check(lib().eifmm_batch_get_stats(self._h, p, ctypes.byref(s)), "eifmm_batch_get_stats")
        return _stats_dict(s, s.depth)

    def info(self):
        i = BatchInfo()
        i.struct_size = ctypes.sizeof(BatchInfo)
        _check(lib().eifmm_batch_get_info(self._h, ctypes.byref(i)), "eifmm_batch_get_info")
        return dict(nprob=i.nprob, ntables=i.ntables, graph_nodes=i.graph_nodes,
                    m2l_rbt=i.m2l_rbt, m2l_flops=i.m2l_flops, tune_ms=i.tune_ms,
                    setup_ms=i.setup_ms)

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.eifmm_batch_destroy(h)
        self._h = None

    def __del__(self):
        self.close()


def declared_symbols(header=HEADER):
    """Names of the functions declared in include/eifmm.h."""
    import re
    txt = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(eifmm_\w+)\s*\(", txt, re.M)))
