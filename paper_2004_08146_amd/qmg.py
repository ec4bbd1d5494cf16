"""ctypes binding of libqmg.so (argument marshalling only).

Every computation runs in the HIP library; torch provides device memory and
the current stream.  Names mirror the C interface in ``include/qmg.h``
without the ``qmg_`` prefix.  Internal fields are opaque byte tensors on the
GPU (``Lattice.field``); canonical fields are complex128 torch tensors of
shape ``[nrhs, N0, N1, N2, N3, 4, 3]`` (gauge: ``[N0, N1, N2, N3, 4, 3, 3]``).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqmg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libqmg.so is not built: run __graft_entry__.build() (or "
                      "python paper_2004_08146_amd/build.py)")
_lib = ctypes.CDLL(LIB_PATH)

F64, F32, BF16 = 0, 1, 2
_PREC = {"f64": F64, "f32": F32, "bf16": BF16, F64: F64, F32: F32, BF16: BF16}
STATUS = {0: "QMG_OK", 1: "QMG_NOT_CONVERGED", -1: "QMG_E_ARG", -2: "QMG_E_STATE",
          -3: "QMG_E_NOMEM", -4: "QMG_E_HIP", -5: "QMG_E_NUMERIC"}


class QmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("restart", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("n_mr", ctypes.c_int), ("coarse_maxiter", ctypes.c_int),
                ("coarse_tol", ctypes.c_double), ("mg_prec", ctypes.c_int), ("use_coarse", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("q_form", ctypes.c_int), ("smoother", ctypes.c_int),
                ("levels", ctypes.c_int), ("l3_iters", ctypes.c_int), ("l2_smooth", ctypes.c_int),
                ("x0", ctypes.c_int)]


STATS_HIST = 32


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("coarse_iters", ctypes.c_int),
                ("true_relres", ctypes.c_double), ("seconds", ctypes.c_double),
                ("vcycle_seconds", ctypes.c_double), ("apply_seconds", ctypes.c_double),
                ("orth_seconds", ctypes.c_double), ("n_hist", ctypes.c_int),
                ("relres_hist", ctypes.c_double * STATS_HIST)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "relres_hist"}
        d["relres_hist"] = list(self.relres_hist[:self.n_hist])
        return d


class EigParams(ctypes.Structure):
    _fields_ = [("m_min", ctypes.c_int), ("m_max", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxiter", ctypes.c_int), ("inner_tol", ctypes.c_double), ("inner_maxiter", ctypes.c_int),
                ("update_interp", ctypes.c_int), ("block", ctypes.c_int), ("solve", Params),
                ("extraction", ctypes.c_int), ("both_signs", ctypes.c_int)]


class EigStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("interp_updates", ctypes.c_int), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)
_SIG = {
    "qmg_default_params": ([], Params),
    "qmg_create": ([ctypes.POINTER(_vp), ctypes.POINTER(_i), ctypes.POINTER(_i), _i], _i),
    "qmg_destroy": ([_vp], _i),
    "qmg_last_error": ([_vp], ctypes.c_char_p),
    "qmg_field_bytes": ([_vp, _i], ctypes.c_size_t),
    "qmg_coarse_bytes": ([_vp, _i], ctypes.c_size_t),
    "qmg_coarse_site_order": ([_vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64], _i),
    "qmg_pack": ([_vp, _vp, _vp, _i, _i, _vp], _i),
    "qmg_unpack": ([_vp, _vp, _vp, _i, _i, _vp], _i),
    "qmg_field_dot": ([_vp, _dp, _vp, _vp, _i, _i, _vp], _i),
    "qmg_set_gauge": ([_vp, _vp, _d, _d, _vp], _i),
    "qmg_apply_Q": ([_vp, _vp, _vp, _i, _i, _vp], _i),
    "qmg_apply_Q_shifted": ([_vp, _vp, _vp, _dp, _i, _i, _vp], _i),
    "qmg_apply_A": ([_vp, _vp, _vp, _dp, _i, _i, _vp], _i),
    "qmg_sap_smooth": ([_vp, _vp, _vp, _dp, _i, _i, _i, _i, _vp], _i),
    "qmg_set_test_vectors": ([_vp, _vp, _i, _vp], _i),
    "qmg_setup_mg": ([_vp, _vp, _i, _i, _i, _i, _i, _d, _i, _vp], _i),
    "qmg_restrict": ([_vp, _vp, _vp, _i, _i, _vp], _i),
    "qmg_prolong": ([_vp, _vp, _vp, _i, _i, _vp], _i),
    "qmg_apply_coarse": ([_vp, _vp, _vp, _dp, _i, _i, _vp], _i),
    "qmg_coarse_solve": ([_vp, _vp, _vp, _dp, _i, _i, _d, _i, _vp], _i),
    "qmg_vcycle": ([_vp, _vp, _vp, _dp, _i, ctypes.POINTER(Params), _vp], _i),
    "qmg_solve_shifted": ([_vp, _vp, _vp, _dp, _i, ctypes.POINTER(Params), ctypes.POINTER(Stats), _vp], _i),
    "qmg_gauge_force": ([_vp, _vp, _vp, _vp, _vp, _vp], _i),
    "qmg_autotune": ([_vp, ctypes.c_char_p], _i),
    "qmg_local_coherence": ([_vp, _dp, _vp, _i, _vp], _i),
    "qmg_default_eig_params": ([], EigParams),
    "qmg_eigensolve": ([_vp, _i, _dp, _vp, _vp, _i, _vp, ctypes.POINTER(EigParams), ctypes.POINTER(EigStats),
                        _vp], _i),
    "qmg_hermitian_eig": ([_i, _dp, _dp, _dp], _i),
    "qmg_set_level3_vectors": ([_vp, _vp, _i, ctypes.POINTER(_i), _vp], _i),
    "qmg_setup_level3": ([_vp, _vp, _i, ctypes.POINTER(_i), _i, _i, _i, _vp], _i),
    "qmg_restrict_l3": ([_vp, _vp, _vp, _i, _i, _vp], _i),
    "qmg_prolong_l3": ([_vp, _vp, _vp, _i, _i, _vp], _i),
    "qmg_apply_l3": ([_vp, _vp, _vp, _dp, _i, _i, _vp], _i),
    "qmg_level2_solve": ([_vp, _vp, _vp, _dp, _i, _i, _i, _i, _i, _vp], _i),
    "qmg_level3_shape": ([_vp, ctypes.POINTER(_i), ctypes.POINTER(_i)], _i),
    "qmg_stream_copy": ([_vp, _vp, ctypes.c_size_t, _vp], _i),
    "qmg_field_dot_noalloc": ([_vp, _dp, _vp, _vp, _i, _i, _vp], _i),
}
for _name, (_args, _res) in _SIG.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIG)


def default_params(**kw):
    p = _lib.qmg_default_params()
    for k, v in kw.items():
        if k == "mg_prec":
            v = _PREC[v]
        setattr(p, k, v)
    return p


def default_eig_params(**kw):
    """GD-lambdaAMG parameters; keys of the inner solver go in solve={...}."""
    p = _lib.qmg_default_eig_params()
    for k, v in kw.items():
        if k == "solve":
            for kk, vv in v.items():
                setattr(p.solve, kk, _PREC[vv] if kk == "mg_prec" else vv)
        else:
            setattr(p, k, v)
    return p


def hermitian_eig(a):
    """Eigenvalues (ascending) and eigenvectors of a Hermitian matrix with the
    library's host Jacobi solver (the harmonic-Ritz step of the eigensolver)."""
    import numpy as np
    a = np.asarray(a, dtype=np.complex128)
    m = a.shape[0]
    af = np.asfortranarray(a).ravel(order="F").view(np.float64).copy()
    w = np.zeros(m)
    z = np.zeros(2 * m * m)
    st = _lib.qmg_hermitian_eig(m, af.ctypes.data_as(_dp), w.ctypes.data_as(_dp), z.ctypes.data_as(_dp))
    if st != 0:
        raise QmgError(st, "hermitian_eig")
    return w, z.view(np.complex128).reshape(m, m, order="F")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def stream_copy(dst, src):
    """Copy the bytes of device tensor src into dst with the library's streaming
    kernel (a bandwidth probe)."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < n:
        raise ValueError("stream_copy: destination too small")
    st = _lib.qmg_stream_copy(_ptr(dst), _ptr(src), n, _stream())
    if st != 0:
        raise QmgError(st, "stream_copy")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _taus(tau, nrhs):
    if isinstance(tau, (int, float)):
        tau = [float(tau)] * nrhs
    tau = [float(t) for t in tau]
    if len(tau) != nrhs:
        raise ValueError("need one shift per right-hand side")
    return (ctypes.c_double * nrhs)(*tau)


class Lattice:
    """A qmg context: lattice shape, blocking and the device-resident operator."""

    def __init__(self, dims, block=(4, 4, 4, 4), device=0):
        self.dims = tuple(int(d) for d in dims)
        self.block = tuple(int(b) for b in block)
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        st = _lib.qmg_create(ctypes.byref(h), (_i * 4)(*self.dims), (_i * 4)(*self.block), device)
        if st != 0:
            raise QmgError(st, "qmg_create failed for dims %s block %s" % (self.dims, self.block))
        self._h = h
        self.ntv = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.qmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st < 0 or st > 1:
            raise QmgError(st, "%s: %s" % (what, _lib.qmg_last_error(self._h).decode()))
        return st

    # ---------------------------------------------------------- storage --
    def field_bytes(self, prec="f64"):
        return _lib.qmg_field_bytes(self._h, _PREC[prec])

    def coarse_bytes(self, prec="f64"):
        return _lib.qmg_coarse_bytes(self._h, _PREC[prec])

    def field(self, nrhs=1, prec="f64", zero=True):
        n = self.field_bytes(prec) * nrhs
        f = torch.zeros if zero else torch.empty
        return f(n, dtype=torch.uint8, device=self.device)

    def coarse(self, nrhs=1, prec="f64", zero=True):
        n = self.coarse_bytes(prec) * nrhs
        f = torch.zeros if zero else torch.empty
        return f(n, dtype=torch.uint8, device=self.device)

    def coarse_site_order(self):
        nb = 1
        for d, b in zip(self.dims, self.block):
            nb *= d // b
        out = (ctypes.c_int64 * nb)()
        self._check(_lib.qmg_coarse_site_order(self._h, out, nb), "coarse_site_order")
        return list(out)

    def pack(self, canon, prec="f64", out=None):
        canon = canon.to(self.device, torch.complex128).contiguous()
        nrhs = canon.numel() // (12 * _vol(self.dims))
        out = self.field(nrhs, prec, zero=False) if out is None else out
        self._check(_lib.qmg_pack(self._h, _ptr(out), _ptr(canon), nrhs, _PREC[prec], _stream()), "pack")
        return out

    def unpack(self, f, nrhs=1, prec="f64"):
        out = torch.empty((nrhs,) + self.dims + (4, 3), dtype=torch.complex128, device=self.device)
        self._check(_lib.qmg_unpack(self._h, _ptr(out), _ptr(f), nrhs, _PREC[prec], _stream()), "unpack")
        return out

    def field_dot(self, a, b, nrhs=1, prec="f64"):
        res = (ctypes.c_double * (2 * nrhs))()
        self._check(_lib.qmg_field_dot(self._h, res, _ptr(a), _ptr(b), nrhs, _PREC[prec], _stream()),
                    "field_dot")
        return [complex(res[2 * k], res[2 * k + 1]) for k in range(nrhs)]

    def field_dot_noalloc(self, a, b, nrhs=1, prec="f64"):
        """field_dot without any device allocation (fixed library scratch)."""
        res = (ctypes.c_double * (2 * nrhs))()
        self._check(_lib.qmg_field_dot_noalloc(self._h, res, _ptr(a), _ptr(b), nrhs, _PREC[prec], _stream()),
                    "field_dot_noalloc")
        return [complex(res[2 * k], res[2 * k + 1]) for k in range(nrhs)]

    # --------------------------------------------------------- operator --
    def set_gauge(self, U, m0, csw=0.0):
        U = U.to(self.device, torch.complex128).contiguous()
        self._check(_lib.qmg_set_gauge(self._h, _ptr(U), float(m0), float(csw), _stream()), "set_gauge")
        self.ntv = 0

    def apply_Q(self, out, inp, nrhs=1, prec="f64"):
        self._check(_lib.qmg_apply_Q(self._h, _ptr(out), _ptr(inp), nrhs, _PREC[prec], _stream()), "apply_Q")
        return out

    def apply_Q_shifted(self, out, inp, tau, nrhs=1, prec="f64"):
        self._check(_lib.qmg_apply_Q_shifted(self._h, _ptr(out), _ptr(inp), _taus(tau, nrhs), nrhs,
                                             _PREC[prec], _stream()), "apply_Q_shifted")
        return out

    def apply_A(self, out, inp, tau, nrhs=1, prec="f64"):
        self._check(_lib.qmg_apply_A(self._h, _ptr(out), _ptr(inp), _taus(tau, nrhs), nrhs, _PREC[prec],
                                     _stream()), "apply_A")
        return out

    def sap_smooth(self, x, f, tau, nrhs=1, nsweep=3, n_mr=3, prec="f64"):
        self._check(_lib.qmg_sap_smooth(self._h, _ptr(x), _ptr(f), _taus(tau, nrhs), nrhs, nsweep, n_mr,
                                        _PREC[prec], _stream()), "sap_smooth")
        return x

    # ------------------------------------------------------- multigrid --
    def set_test_vectors(self, W, ntv):
        self._check(_lib.qmg_set_test_vectors(self._h, _ptr(W), ntv, _stream()), "set_test_vectors")
        self.ntv = ntv

    def setup_mg(self, W0, ntv, setup_iters=6, smooth=4, n_mr=3, coarse_maxiter=20, coarse_tol=0.5, prec="f32"):
        self._check(_lib.qmg_setup_mg(self._h, _ptr(W0), ntv, setup_iters, smooth, n_mr, coarse_maxiter,
                                      float(coarse_tol), _PREC[prec], _stream()), "setup_mg")
        self.ntv = ntv
        return W0

    def restrict(self, yc, v, nrhs=1, prec="f64"):
        self._check(_lib.qmg_restrict(self._h, _ptr(yc), _ptr(v), nrhs, _PREC[prec], _stream()), "restrict")
        return yc

    def prolong(self, v, yc, nrhs=1, prec="f64"):
        self._check(_lib.qmg_prolong(self._h, _ptr(v), _ptr(yc), nrhs, _PREC[prec], _stream()), "prolong")
        return v

    def apply_coarse(self, out, inp, tau, nrhs=1, prec="f64"):
        self._check(_lib.qmg_apply_coarse(self._h, _ptr(out), _ptr(inp), _taus(tau, nrhs), nrhs,
                                          _PREC[prec], _stream()), "apply_coarse")
        return out

    def coarse_solve(self, y, r, tau, nrhs=1, iters=20, tol=0.0, prec="f64"):
        self._check(_lib.qmg_coarse_solve(self._h, _ptr(y), _ptr(r), _taus(tau, nrhs), nrhs, iters,
                                          float(tol), _PREC[prec], _stream()), "coarse_solve")
        return y

    # ------------------------------------------------------- third level --
    def set_level3_vectors(self, W2, ntv2, block2):
        """W2: ntv2 FP64 level-2 (coarse) vectors on the device, internal site order."""
        b2 = (ctypes.c_int * 4)(*block2)
        self._check(_lib.qmg_set_level3_vectors(self._h, _ptr(W2), ntv2, b2, _stream()), "set_level3_vectors")

    def setup_level3(self, W2, ntv2, block2, setup_iters=3, smooth=2, l3_iters=20):
        """Level-2 test vectors by inverse iteration (W2 updated in place)."""
        b2 = (ctypes.c_int * 4)(*block2)
        self._check(_lib.qmg_setup_level3(self._h, _ptr(W2), ntv2, b2, setup_iters, smooth, l3_iters, _stream()),
                    "setup_level3")
        return W2

    def level2_vectors_from(self, W, ntv2):
        """P^H w_j of the first ntv2 fine FP64 test vectors W (internal layout):
        starting level-2 vectors for setup_level3."""
        fb = self.field_bytes("f64")
        out = self.coarse(ntv2)
        cb = self.coarse_bytes("f64")
        for j in range(ntv2):
            self.restrict(out[j * cb:(j + 1) * cb], W[j * fb:(j + 1) * fb], 1)
        return out

    def level3_shape(self):
        n3, nc3 = ctypes.c_int(), ctypes.c_int()
        self._check(_lib.qmg_level3_shape(self._h, ctypes.byref(n3), ctypes.byref(nc3)), "level3_shape")
        return n3.value, nc3.value

    def l3_vec(self, nrhs=1, prec="f64"):
        n3, nc3 = self.level3_shape()
        itemsize = 16 if prec == "f64" else 8
        return torch.zeros(n3 * nc3 * nrhs * itemsize, dtype=torch.uint8, device=self.device)

    def restrict_l3(self, y3, y2, nrhs=1, prec="f64"):
        self._check(_lib.qmg_restrict_l3(self._h, _ptr(y3), _ptr(y2), nrhs, _PREC[prec], _stream()), "restrict_l3")
        return y3

    def prolong_l3(self, y2, y3, nrhs=1, prec="f64"):
        self._check(_lib.qmg_prolong_l3(self._h, _ptr(y2), _ptr(y3), nrhs, _PREC[prec], _stream()), "prolong_l3")
        return y2

    def apply_l3(self, out, inp, tau, nrhs=1, prec="f64"):
        self._check(_lib.qmg_apply_l3(self._h, _ptr(out), _ptr(inp), _taus(tau, nrhs), nrhs, _PREC[prec],
                                      _stream()), "apply_l3")
        return out

    def level2_solve(self, y, r, tau, nrhs=1, k2=4, k3=20, s2=2, prec="f64"):
        self._check(_lib.qmg_level2_solve(self._h, _ptr(y), _ptr(r), _taus(tau, nrhs), nrhs, k2, k3, s2,
                                          _PREC[prec], _stream()), "level2_solve")
        return y

    def vcycle(self, z, r, tau, nrhs=1, params=None):
        params = params or default_params()
        self._check(_lib.qmg_vcycle(self._h, _ptr(z), _ptr(r), _taus(tau, nrhs), nrhs, ctypes.byref(params),
                                    _stream()), "vcycle")
        return z

    def solve_shifted(self, x, b, tau, nrhs=1, params=None):
        """Returns (status, [per-rhs stats dicts]); status 1 = not converged."""
        params = params or default_params()
        stats = (Stats * nrhs)()
        st = self._check(_lib.qmg_solve_shifted(self._h, _ptr(x), _ptr(b), _taus(tau, nrhs), nrhs,
                                                ctypes.byref(params), stats, _stream()), "solve_shifted")
        return st, [s.as_dict() for s in stats]

    def gauge_force(self, phi, x):
        """(dL/dU, dL/dconj(U)) of L = phi^H Q x as canonical complex128 tensors."""
        shp = self.dims + (4, 3, 3)
        G = torch.empty(shp, dtype=torch.complex128, device=self.device)
        Gb = torch.empty(shp, dtype=torch.complex128, device=self.device)
        self._check(_lib.qmg_gauge_force(self._h, _ptr(G), _ptr(Gb), _ptr(phi), _ptr(x), _stream()),
                    "gauge_force")
        return G, Gb

    def local_coherence(self, v, nrhs=1):
        """lc(v_k) = ||Pi v_k|| / ||v_k|| for nrhs internal F64 fields (numpy array)."""
        import numpy as np
        lc = np.zeros(nrhs)
        self._check(_lib.qmg_local_coherence(self._h, lc.ctypes.data_as(_dp), _ptr(v), nrhs, _stream()),
                    "local_coherence")
        return lc

    def eigensolve(self, nev, X, t0, V0=None, n0=0, params=None):
        """GD-lambdaAMG: returns (status, eigenvalues (numpy, lock order), stats dict);
        X receives nev internal F64 eigenvector fields."""
        import numpy as np
        params = params or default_eig_params()
        lam = np.zeros(nev)
        stats = EigStats()
        st = self._check(_lib.qmg_eigensolve(self._h, nev, lam.ctypes.data_as(_dp), _ptr(X),
                                             _ptr(V0) if V0 is not None else None, n0, _ptr(t0),
                                             ctypes.byref(params), ctypes.byref(stats), _stream()), "eigensolve")
        return st, lam[:stats.converged], stats.as_dict()

    def autotune(self, cache_json_path=None):
        p = cache_json_path.encode() if cache_json_path else None
        self._check(_lib.qmg_autotune(self._h, p), "autotune")


def _vol(dims):
    v = 1
    for d in dims:
        v *= d
    return v


class QuadraticForm(torch.autograd.Function):
    """L = phi^H Q[U] x with gradients for U (gauge force), phi and x.

    Forward and backward run in the HIP library (apply_Q, field_dot,
    gauge_force); the binding only applies the complex chain rule: for the
    upstream gradient g of L, grad_U = conj(g) dL/dconj(U) + g conj(dL/dU),
    grad_phi = conj(g) Q x and grad_x = g Q phi.
    """

    @staticmethod
    def forward(ctx, lat, U, phi, x, m0):
        lat.set_gauge(U.detach(), m0, 0.0)
        pf = lat.pack(phi.detach())
        xf = lat.pack(x.detach())
        qx = lat.apply_Q(lat.field(1), xf)
        L = lat.field_dot(pf, qx)[0]
        ctx.lat = lat
        ctx.save_for_backward(U.detach(), phi.detach(), x.detach())
        ctx.m0 = m0
        return torch.tensor(L, dtype=torch.complex128, device=U.device)

    @staticmethod
    def backward(ctx, g):
        lat = ctx.lat
        U, phi, x = ctx.saved_tensors
        lat.set_gauge(U, ctx.m0, 0.0)
        pf = lat.pack(phi)
        xf = lat.pack(x)
        G, Gb = lat.gauge_force(pf, xf)
        gU = torch.conj(g) * Gb + g * torch.conj(G)
        qx = lat.unpack(lat.apply_Q(lat.field(1), xf)).reshape(phi.shape)
        qphi = lat.unpack(lat.apply_Q(lat.field(1), pf)).reshape(x.shape)
        return None, gU, torch.conj(g) * qx, g * qphi, None
