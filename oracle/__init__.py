"""CPU FP64 oracle for the EIFMM evaluation pass.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product path.  It
shares no code with the HIP library.

The arithmetic lives in ``eifmm_oracle.c`` (plain loops, double precision, one
routine per step of F. Casenave, arXiv:1408.0210); this module only marshals
numpy arrays through ctypes.  Points are SoA arrays of shape (3, n).

parity unpinned: the map from the EIM tolerance tau to the achieved error of the
full pass (the paper prints accuracies without tau), and d_k for the physical
kernels (never printed); both are measured, not asserted.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "eifmm_oracle.c")
LIB_PATH = os.environ.get("ORACLE_LIB_OVERRIDE") or os.path.join(_HERE, "liboracle.so")

KERNELS = {"laplace": 0, "yukawa": 1, "gauss": 2, "sqdist": 3, "cosr": 4, "mq": 5,
           "cosdot": 6, "expdot": 7, "advdiff": 8}
SINGULAR = {"laplace", "yukawa", "cosr", "advdiff"}
NONSYMMETRIC = {"expdot", "advdiff"}  # k(-z) != k(z): two EIMs per level

OK, EINVAL, EDOMAIN, EEIM, ENOMEM = 0, -1, -2, -4, -5


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force=True):
    """Compile the oracle with gcc (no FMA contraction, OpenMP for the loops)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c99",
           "-D_DEFAULT_SOURCE", "-o", LIB_PATH + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        d, i64, i32, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.orc_kernel_eval.argtypes = [i32, vp, i64, vp, vp]
        L.orc_kernel_eval.restype = None
        L.orc_direct.argtypes = [i32, vp, i64, vp, i64, vp, vp, vp, i32]
        L.orc_tree.argtypes = [i64, vp, vp, d, i32, vp, vp, vp]
        L.orc_lists.argtypes = [i32, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.orc_offset_table.argtypes = [vp]
        L.orc_offset_table.restype = None
        L.orc_training_sets.argtypes = [i32, i32, vp, P(i64), vp, P(i64)]
        L.orc_eim.argtypes = [i32, vp, i32, d, d, i32, d, P(i32), vp, vp, vp, vp, vp, vp, vp,
                              P(d)]
        L.orc_eim_swapped.argtypes = L.orc_eim.argtypes
        L.orc_apply_delta.argtypes = [i32, i32, vp, vp, vp, vp, i32]
        L.orc_apply_delta.restype = None
        L.orc_plan_create.argtypes = [i32, vp, vp, d, i32, d, i32, i32, i32, P(i32)]
        L.orc_plan_create.restype = vp
        L.orc_plan_level.argtypes = [vp, i32, i32, P(i32), vp, vp, vp, vp, vp, vp, vp]
        L.orc_plan_eval.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32]
        L.orc_plan_free.argtypes = [vp]
        L.orc_plan_free.restype = None
        L.orc_plan_set_compression.argtypes = [vp, i32, i32, vp, vp]
        L.orc_plan_set_compression2.argtypes = [vp, i32, vp, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _params(param):
    p = np.zeros(3, dtype=np.float64)
    if param is not None:
        v = np.atleast_1d(np.asarray(param, dtype=np.float64))
        p[:v.size] = v
    return p


def _soa(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim != 2 or x.shape[0] != 3:
        raise ValueError("points must have shape (3, n)")
    return x


def kernel_eval(kernel, param, z):
    """k(z) for difference vectors z of shape (n, 3)."""
    z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1, 3)
    out = np.empty(z.shape[0])
    p = _params(param)
    lib().orc_kernel_eval(KERNELS[kernel], _p(p), z.shape[0], _p(z), _p(out))
    return out


def direct(kernel, param, targets, sources, sigma, threads=0):
    """eq. (1): f_i = sum_j sigma_j K(x_i, y_j), r == 0 pairs skipped for singular K."""
    xt, ys = _soa(targets), _soa(sources)
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    assert s.shape == (ys.shape[1],)
    f = np.empty(xt.shape[1])
    p = _params(param)
    st = lib().orc_direct(KERNELS[kernel], _p(p), xt.shape[1], _p(xt), ys.shape[1], _p(ys),
                          _p(s), _p(f), threads)
    if st:
        raise OracleError(st, "direct")
    return f


def tree(xyz, lo, L, depth):
    """Leaf keys per input point, the (key, index) sort permutation and leaf starts."""
    x = _soa(xyz)
    n = x.shape[1]
    keys = np.empty(n, dtype=np.uint32)
    perm = np.empty(n, dtype=np.int32)
    ls = np.empty((1 << (3 * depth)) + 1, dtype=np.int64)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    st = lib().orc_tree(n, _p(x), _p(lo), float(L), depth, _p(keys), _p(perm), _p(ls))
    if st:
        raise OracleError(st, "tree")
    return keys, perm, ls


def lists(leaf_start, depth, level):
    """Active boxes, near lists and interaction lists (with offset ids) at `level`."""
    ls = np.ascontiguousarray(leaf_start, dtype=np.int64)
    nb = 1 << (3 * level)
    na = np.zeros(1, dtype=np.int64)
    active = np.empty(nb, dtype=np.uint32)
    near_ptr = np.empty(nb + 1, dtype=np.int64)
    near_src = np.empty(27 * nb, dtype=np.uint32)
    il_ptr = np.empty(nb + 1, dtype=np.int64)
    il_src = np.empty(189 * nb, dtype=np.uint32)
    il_off = np.empty(189 * nb, dtype=np.int16)
    st = lib().orc_lists(depth, _p(ls), level, _p(na), _p(active), _p(near_ptr), _p(near_src),
                         _p(il_ptr), _p(il_src), _p(il_off))
    if st:
        raise OracleError(st, "lists")
    a = int(na[0])
    nn = int(near_ptr[a])
    ni = int(il_ptr[a])
    return dict(active=active[:a].copy(), near_ptr=near_ptr[:a + 1].copy(),
                near_src=near_src[:nn].copy(), il_ptr=il_ptr[:a + 1].copy(),
                il_src=il_src[:ni].copy(), il_off=il_off[:ni].copy())


def offset_table():
    t = np.empty((316, 3), dtype=np.int32)
    lib().orc_offset_table(_p(t))
    return t


def training_sets(kernel, level):
    """Training points (units of l_k), AoS: (T_x in I_0, T_y in J_0)."""
    L = lib()
    ntx, nty = ctypes.c_int64(), ctypes.c_int64()
    st = L.orc_training_sets(KERNELS[kernel], level, None, ctypes.byref(ntx), None,
                             ctypes.byref(nty))
    if st:
        raise OracleError(st, "training_sets")
    tx = np.empty((ntx.value, 3))
    ty = np.empty((nty.value, 3))
    L.orc_training_sets(KERNELS[kernel], level, _p(tx), ctypes.byref(ntx), _p(ty),
                        ctypes.byref(nty))
    return tx, ty


def eim(kernel, param, level, L, tau, dmax=1024, abs_scale=0.0, swapped=False):
    """Algorithm 1 on the level's training sets; returns the interpolation data.
    swapped: the second EIM of Sec. 3.1, on D_x = J_0 and D_y = I_0 (X then holds
    J_0 points, Y holds I_0 points)."""
    p = _params(param)
    ia = np.empty(dmax, dtype=np.int64)
    ib = np.empty(dmax, dtype=np.int64)
    X = np.empty((dmax, 3))
    Y = np.empty((dmax, 3))
    B = np.empty((dmax, dmax))
    G = np.empty((dmax, dmax))
    eps = np.empty(dmax + 1)
    d = ctypes.c_int()
    sc = ctypes.c_double()
    fn = lib().orc_eim_swapped if swapped else lib().orc_eim
    st = fn(KERNELS[kernel], _p(p), level, float(L), float(tau), dmax, float(abs_scale),
            ctypes.byref(d), _p(ia), _p(ib), _p(X), _p(Y), _p(B), _p(G), _p(eps),
            ctypes.byref(sc))
    dd = d.value
    res = dict(d=dd, ia=ia[:dd].copy(), ib=ib[:dd].copy(), X=X[:dd].copy(), Y=Y[:dd].copy(),
               B=B[:dd, :dd].copy(), G=G[:dd, :dd].copy(), eps=eps[:dd + 1].copy(),
               scale=sc.value, status=st)
    if st not in (OK, EEIM):
        raise OracleError(st, "eim")
    return res


def apply_delta(B, G, v, transpose=False):
    """Delta v = B^{-T} Gamma^{-1} v (or Delta^T v) by triangular solves."""
    d = B.shape[0]
    B = np.ascontiguousarray(B, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty(d)
    lib().orc_apply_delta(d, d, _p(B), _p(G), _p(v), _p(w), 1 if transpose else 0)
    return w


def m2l_matrices(kernel, param, Y, level, L=1.0, X=None):
    """The 316 translation-invariant M2L matrices of a level (Sec. 4.2):
    K^delta[m', l] = K(X_m', Y_l + 2 l_k delta), in offset-id order; the rows X are
    the second EIM's points when there is one, else X = Y."""
    X = Y if X is None else X
    h = L * 2.0 ** (-level)
    dt = offset_table().astype(np.float64)
    z = X[None, :, None, :] - (Y[None, None, :, :] + h * dt[:, None, None, :])
    return kernel_eval(kernel, param, z.reshape(-1, 3)).reshape(316, len(X), len(Y))


def compression_rank(s, eps):
    """Rank kept by the two filters of Sec. 4.2 on singular values s (descending):
    (i) the values with s_j / s_0 > eps, (ii) the shortest prefix whose sum reaches
    (1 - eps) of the total; both are applied and the larger rank is kept."""
    r1 = int((s / s[0] > eps).sum())
    cs = np.cumsum(s) / s.sum()
    r2 = int(min(len(s), np.searchsorted(cs, 1.0 - eps) + 1))
    return max(r1, r2)


def compression_factors(C, eps, ranks=None):
    """Second stage of Sec. 4.2 on each compressed matrix C^delta (r x r): an SVD
    (in place of the bivariate ACA and the two QR decompositions), the two filters
    with eps (or the given ranks), and the split of the kept singular values
    between the factors: C^delta ~ Ut Vt with Ut = P_s sqrt(S_s), Vt = sqrt(S_s) Q_s^T.
    Returns the ranks s_o and the factor lists."""
    s_list, Ut, Vt = [], [], []
    for o, Co in enumerate(C):
        P, sv, Qt = np.linalg.svd(Co)
        so = compression_rank(sv, eps) if ranks is None else int(ranks[o])
        h = np.sqrt(sv[:so])
        Ut.append(np.ascontiguousarray(P[:, :so] * h[None, :]))
        Vt.append(np.ascontiguousarray(h[:, None] * Qt[:so, :]))
        s_list.append(so)
    return np.array(s_list, dtype=np.int32), Ut, Vt


def compression_basis(kernel, param, Y, level, eps, L=1.0, rank=None):
    """Sec. 4.2, first stage, with an exact SVD in place of the bivariate ACA:
    K_fat = [K^delta_1 ... K^delta_316] = U S V^T; keep the leading r columns of U
    (r from the filters, or `rank` when given)."""
    Kd = m2l_matrices(kernel, param, Y, level, L)
    Kfat = np.concatenate(list(Kd), axis=1)
    U, s, _ = np.linalg.svd(Kfat, full_matrices=False)
    r = compression_rank(s, eps) if rank is None else int(rank)
    return np.ascontiguousarray(U[:, :r]), s, r


def compression_bases(kernel, param, X, Y, level, eps, L=1.0, rank=None):
    """Sec. 4.2, first stage, for M2L matrices that are not symmetric (two EIMs):
    U from the SVD of K_fat = [K^delta_1 ... K^delta_316] (its column space, rows X)
    and V from the SVD of K_thin, the matrices stacked (their common row space).
    r is the larger of the two filtered ranks (or `rank`)."""
    Kd = m2l_matrices(kernel, param, Y, level, L, X=X)
    U, su, _ = np.linalg.svd(np.concatenate(list(Kd), axis=1), full_matrices=False)
    _, sv, Vt = np.linalg.svd(np.concatenate(list(Kd), axis=0), full_matrices=False)
    r = max(compression_rank(su, eps), compression_rank(sv, eps)) if rank is None else int(rank)
    return np.ascontiguousarray(U[:, :r]), np.ascontiguousarray(Vt[:r].T), su, sv, r


class Plan:
    """Per-level EIM data (levels 2..depth) and the Algorithm-3 evaluation.
    A kernel that is not symmetric gets the second EIM of Sec. 3.1 on every level
    (levels2); two_eim=True gives it to a symmetric kernel too."""

    def __init__(self, kernel, param, lo, L, depth, tau, dmax=1024, tol_mode=0, compress_tol=0.0,
                 compress_rank=None, two_eim=False, compress_tol2=0.0, compress_rank2=None):
        self.kernel, self.param = kernel, _params(param)
        self.lo = np.ascontiguousarray(lo, dtype=np.float64)
        self.L, self.depth, self.tau = float(L), int(depth), float(tau)
        self.two = bool(two_eim) or kernel in NONSYMMETRIC
        st = ctypes.c_int()
        self._h = lib().orc_plan_create(KERNELS[kernel], _p(self.param), _p(self.lo), self.L,
                                        self.depth, self.tau, dmax, tol_mode,
                                        1 if two_eim else 0, ctypes.byref(st))
        if not self._h:
            raise OracleError(st.value, "plan_create")
        self.levels = {k: self._level(k) for k in range(2, self.depth + 1)}
        self.levels2 = {k: self._level(k, 1) for k in range(2, self.depth + 1)} if self.two else {}
        self.compress_tol = float(compress_tol)
        if compress_tol > 0:
            for k in range(2, self.depth + 1):
                rk = compress_rank.get(k) if isinstance(compress_rank, dict) else compress_rank
                Y = self.levels[k]["Y"]
                X = self.levels2[k]["X"] if self.two else None
                if self.two:
                    U, V, sv, sv2, r = compression_bases(kernel, self.param, X, Y, k,
                                                         compress_tol, self.L, rank=rk)
                    self.levels[k].update(U=U, V=V, sv=sv, sv2=sv2, r=r)
                else:
                    U, sv, r = compression_basis(kernel, self.param, Y, k, compress_tol, self.L,
                                                 rank=rk)
                    V = U
                    self.levels[k].update(U=U, sv=sv, r=r)
                st = lib().orc_plan_set_compression(self._h, k, r, _p(U),
                                                    _p(V) if self.two else None)
                if st:
                    raise OracleError(st, "set_compression")
                if compress_tol2 > 0:
                    # second stage (Sec. 4.2): each C^delta = U^T K^delta V factored
                    Kd = m2l_matrices(kernel, self.param, Y, k, self.L, X=X)
                    C = np.einsum("ia,oij,jb->oab", U, Kd, V, optimize=True)
                    r2 = compress_rank2.get(k) if isinstance(compress_rank2, dict) else None
                    r2 = None if r2 is None else np.asarray(r2)
                    s2, Ut, Vt = compression_factors(C, compress_tol2, r2)
                    self.levels[k].update(s2=s2)
                    # Ut_o (r x s_o) and Vt_o (s_o x r), each row-major, offset after offset
                    up = np.ascontiguousarray(np.concatenate([u.ravel() for u in Ut]))
                    vp = np.ascontiguousarray(np.concatenate([v.ravel() for v in Vt]))
                    st = lib().orc_plan_set_compression2(self._h, k, _p(s2), _p(up), _p(vp))
                    if st:
                        raise OracleError(st, "set_compression2")

    def _level(self, k, which=0):
        d = ctypes.c_int()
        lib().orc_plan_level(self._h, k, which, ctypes.byref(d), None, None, None, None, None,
                             None, None)
        dd = d.value
        X, Y = np.empty((dd, 3)), np.empty((dd, 3))
        B, G = np.empty((dd, dd)), np.empty((dd, dd))
        ia, ib = np.empty(dd, dtype=np.int64), np.empty(dd, dtype=np.int64)
        eps = np.empty(dd + 1)
        lib().orc_plan_level(self._h, k, which, ctypes.byref(d), _p(X), _p(Y), _p(B), _p(G),
                             _p(ia), _p(ib), _p(eps))
        return dict(d=dd, X=X, Y=Y, B=B, G=G, ia=ia, ib=ib, eps=eps)

    def level_offsets(self, second=False):
        """Dump layout: (offset, boxes, values per box) per level; second=True for g,
        l and lhat, which hold the second EIM's d values per box when there is one."""
        lv = self.levels2 if (second and self.two) else self.levels
        off, out = 0, {}
        for k in range(2, self.depth + 1):
            out[k] = (off, (1 << (3 * k)), lv[k]["d"])
            off += (1 << (3 * k)) * lv[k]["d"]
        return out, off

    def evaluate(self, xyz, sigma, dumps=False, threads=0):
        x = _soa(xyz)
        n = x.shape[1]
        s = np.ascontiguousarray(sigma, dtype=np.float64)
        assert s.shape == (n,)
        f = np.empty(n)
        dd = {}
        if dumps:
            offs, tot = self.level_offsets()
            offs2, tot2 = self.level_offsets(second=True)
            lvd = self.levels2 if self.two else self.levels
            dk = lvd[self.depth]["d"] if self.depth >= 2 else 0
            for name in ("W", "What"):
                dd[name] = np.zeros(tot)
            for name in ("g", "l"):
                dd[name] = np.zeros(tot2)
            dd["lhat"] = np.zeros((1 << (3 * self.depth)) * dk)
            dd["fnear"] = np.zeros(n)
            dd["ffar"] = np.zeros(n)
        st = lib().orc_plan_eval(self._h, n, _p(x), _p(s), _p(f), _p(dd.get("W")),
                                 _p(dd.get("What")), _p(dd.get("g")), _p(dd.get("l")),
                                 _p(dd.get("lhat")), _p(dd.get("fnear")), _p(dd.get("ffar")),
                                 threads)
        if st:
            raise OracleError(st, "plan_eval")
        if not dumps:
            return f
        out = {"fnear": dd["fnear"], "ffar": dd["ffar"]}
        for name in ("W", "What", "g", "l"):
            of = offs if name in ("W", "What") else offs2
            out[name] = {k: dd[name][o:o + nb * d].reshape(nb, d) for k, (o, nb, d) in of.items()}
        if self.depth >= 2:
            out["lhat"] = dd["lhat"].reshape(1 << (3 * self.depth), -1)
        return f, out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_plan_free(h)
            self._h = None
