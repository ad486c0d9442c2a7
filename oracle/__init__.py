"""FP64 CPU oracle for the LDDMM Gauss-Newton-Krylov hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark call it; the product library never does.  numpy arrays in,
numpy arrays out, all float64, grid order [n1][n2][n3] with x3 fastest and
vector fields stacked as [3][n1][n2][n3].

Every function forwards to lddmm_oracle.c, which cites the passage of the
paper (arXiv 2008.12820) each step follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        d, i, l, p = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        sig = {
            "or_set_fft_mode": (None, [i]),
            "or_fft3": (None, [p, i, i, i, i]),
            "or_spectral_grad": (None, [p, p, i, i, i]),
            "or_spectral_div": (None, [p, p, i, i, i]),
            "or_reg_apply": (None, [p, p, i, i, i, i, i]),
            "or_reg_inverse": (None, [p, p, i, i, i, i, i, d]),
            "or_leray": (None, [p, p, i, i, i]),
            "or_interp": (None, [p, i, i, i, i, p, l, p]),
            "or_departure": (None, [p, i, i, i, i, p, p]),
            "or_departure_points": (None, [p, i, i, i, i, p, l, p, p]),
            "or_inner": (d, [p, p, l, d]),
            "or_ctx_create": (p, [i, i, i, i, i, d, i]),
            "or_ctx_destroy": (None, [p]),
            "or_ctx_set_images": (None, [p, p, p]),
            "or_ctx_set_velocity": (None, [p, p]),
            "or_ctx_objective": (None, [p, p]),
            "or_ctx_gradient": (None, [p, p]),
            "or_ctx_adjoint": (None, [p, p, p]),
            "or_ctx_body_force": (None, [p, p, p]),
            "or_ctx_inc_state": (None, [p, p, p]),
            "or_ctx_matvec": (None, [p, p, p]),
            "or_ctx_get": (None, [p, i, i, p]),
            "or_ctx_pcg": (i, [p, p, i, d, p, p]),
            "or_ctx_gn_iterate": (i, [p, i, d, p, p]),
            "or_ctx_h0_apply": (None, [p, p, p]),
            "or_restrict": (None, [p, p, i, i, i, i]),
            "or_fd8_grad": (None, [p, p, i, i, i]),
            "or_fd8_div": (None, [p, p, i, i, i]),
            "or_ctx_set_fd8": (None, [p, i]),
            "or_interp_linear": (None, [p, i, i, i, i, p, l, p]),
            "or_ctx_set_ip_order": (None, [p, i]),
            "or_ctx_set_beta": (None, [p, d]),
            "or_prolong": (None, [p, p, i, i, i, i]),
            "or_ctx_2linvh0": (i, [p, p, d, i, p]),
            "or_ctx_invh0": (i, [p, p, d, i, p]),
            "or_ctx_pcg_pc": (i, [p, p, i, d, i, d, i, p, p]),
            "or_ctx_pcg_hist": (i, [p, p, i, d, i, d, i, p, p, p]),
            "or_ctx_gn_iterate_pc": (i, [p, i, d, i, d, i, p, p]),
            "or_ctx_transport": (None, [p, p, p]),
            "or_ctx_transport_vjp": (None, [p, p, p, p, p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _c(a):
    """float64 C-contiguous copy/view and its pointer."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def set_fft_mode(mode: int):
    """0: naive DFT up to length 32, recursive FFT above; 1: always naive; 2: always FFT."""
    lib().or_set_fft_mode(int(mode))


def fft3(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unnormalised 3D DFT of a complex array, exponent sign*2*pi*i*k.x/n."""
    z = np.ascontiguousarray(a, dtype=np.complex128).copy()
    n1, n2, n3 = z.shape
    lib().or_fft3(z.ctypes.data_as(ctypes.c_void_p), n1, n2, n3, int(sign))
    return z


def spectral_grad(f):
    f, pf = _c(f)
    g = np.empty((3,) + f.shape)
    lib().or_spectral_grad(pf, g.ctypes.data_as(ctypes.c_void_p), *f.shape)
    return g


def spectral_div(v):
    v, pv = _c(v)
    out = np.empty(v.shape[1:])
    lib().or_spectral_div(pv, out.ctypes.data_as(ctypes.c_void_p), *v.shape[1:])
    return out


def reg_apply(v, reg):
    v, pv = _c(v)
    shp = v.shape[-3:]
    nc = 1 if v.ndim == 3 else v.shape[0]
    out = np.empty(v.shape)
    lib().or_reg_apply(pv, out.ctypes.data_as(ctypes.c_void_p), nc, *shp, int(reg))
    return out


def reg_inverse(v, reg, beta):
    v, pv = _c(v)
    shp = v.shape[-3:]
    nc = 1 if v.ndim == 3 else v.shape[0]
    out = np.empty(v.shape)
    lib().or_reg_inverse(pv, out.ctypes.data_as(ctypes.c_void_p), nc, *shp, int(reg),
                         float(beta))
    return out


def leray(v):
    v, pv = _c(v)
    out = np.empty(v.shape)
    lib().or_leray(pv, out.ctypes.data_as(ctypes.c_void_p), *v.shape[1:])
    return out


def _interp_generic(fields, y, fn):
    single = fields.ndim == 3
    f = fields[None] if single else fields
    f, pf = _c(f)
    y, py = _c(y)
    nq = y.shape[1]
    out = np.empty((f.shape[0], nq))
    fn(pf, f.shape[0], *f.shape[1:], py, nq, out.ctypes.data_as(ctypes.c_void_p))
    return out[0] if single else out


def interp(fields, y):
    """fields: [nf][n1][n2][n3] (or one [n1][n2][n3]); y: [3][nq] physical
    coordinates.  Returns [nf][nq] (or [nq])."""
    return _interp_generic(fields, y, lib().or_interp)


def departure(v, nt):
    """Departure points X (state) and Xa (adjoint), [3][n1][n2][n3] physical."""
    v, pv = _c(v)
    X = np.empty(v.shape)
    Xa = np.empty(v.shape)
    lib().or_departure(pv, *v.shape[1:], int(nt), X.ctypes.data_as(ctypes.c_void_p),
                       Xa.ctypes.data_as(ctypes.c_void_p))
    return X, Xa


def departure_points(v, nt, idx):
    """Departure points X, Xa at the grid points idx ([3][nq] integer
    indices) only: [3][nq] physical coordinates each."""
    v, pv = _c(v)
    ii = np.ascontiguousarray(idx, dtype=np.int64)
    nq = ii.shape[1]
    X = np.empty((3, nq))
    Xa = np.empty((3, nq))
    lib().or_departure_points(pv, *v.shape[1:], int(nt), ii.ctypes.data_as(ctypes.c_void_p), nq,
                              X.ctypes.data_as(ctypes.c_void_p), Xa.ctypes.data_as(ctypes.c_void_p))
    return X, Xa


def fd8_grad(f):
    """Eighth-order central-difference gradient (periodic), [3] stack out."""
    a, pa = _c(f)
    out = np.empty((3,) + a.shape)
    lib().or_fd8_grad(pa, out.ctypes.data_as(ctypes.c_void_p), *a.shape)
    return out


def fd8_div(v):
    """Eighth-order central-difference divergence of a [3] stack."""
    a, pa = _c(v)
    out = np.empty(a.shape[1:])
    lib().or_fd8_div(pa, out.ctypes.data_as(ctypes.c_void_p), *a.shape[1:])
    return out


def interp_linear(fields, y):
    """Trilinear interpolation (d = 1), arguments as interp."""
    return _interp_generic(fields, y, lib().or_interp_linear)


def restrict(f):
    """Spectral restriction of a field (or [3] stack) to half the resolution
    (Algorithm "PC", Restrict): coarse Nyquist modes dropped."""
    a, pa = _c(f)
    vec = a.ndim == 4
    shape = a.shape[1:] if vec else a.shape
    out = np.empty(((3,) if vec else ()) + tuple(n // 2 for n in shape))
    lib().or_restrict(pa, out.ctypes.data_as(ctypes.c_void_p), 3 if vec else 1, *shape)
    return out


def prolong(f):
    """Spectral prolongation (zero padding) to twice the resolution (Prolong)."""
    a, pa = _c(f)
    vec = a.ndim == 4
    shape = a.shape[1:] if vec else a.shape
    out = np.empty(((3,) if vec else ()) + tuple(2 * n for n in shape))
    lib().or_prolong(pa, out.ctypes.data_as(ctypes.c_void_p), 3 if vec else 1, *shape)
    return out


def grid_points(shape):
    """Physical coordinates of the grid, [3][n1][n2][n3]."""
    axes = [np.arange(n) * (2 * np.pi / n) for n in shape]
    return np.stack(np.meshgrid(*axes, indexing="ij"))


def inner(a, b, h3):
    a, pa = _c(a)
    b, pb = _c(b)
    return lib().or_inner(pa, pb, a.size, float(h3))


class Problem:
    """One registration problem: grid, N_t, regularisation, images, velocity."""

    def __init__(self, shape, nt, reg=1, beta=1e-2, leray=False, fd8=False, ip=3):
        self.shape = tuple(int(s) for s in shape)
        self.nt = int(nt)
        self.reg = int(reg)
        self.beta = float(beta)
        self.leray = bool(leray)
        self.N = int(np.prod(self.shape))
        self.h3 = float(np.prod([2 * np.pi / n for n in self.shape]))
        self._ctx = lib().or_ctx_create(*self.shape, self.nt, self.reg, self.beta,
                                        int(self.leray))
        self.fd8 = bool(fd8)
        lib().or_ctx_set_fd8(self._ctx, int(self.fd8))
        self.ip = 1 if ip == 1 else 3
        lib().or_ctx_set_ip_order(self._ctx, self.ip)

    def set_beta(self, beta):
        """new regularisation weight; the next gradient is the new ||g0||"""
        self.beta = float(beta)
        lib().or_ctx_set_beta(self._ctx, self.beta)

    def gn_solve(self, v0, beta_target, eps_n=5e-2, max_gn=10, max_pcg=50, rtol=0.0,
                 continuation=True, pc="2linvh0", eps_h0=1e-3, max_inner=50, pc_switch=0.5):
        """Gauss-Newton-Krylov driver (Algorithm "GNK") with beta-continuation
        (Section 2 "Preconditioning", last paragraph): beta = 1, 1e-1, ...
        while above beta_target, then beta_target; per stage, Gauss-Newton
        iterations from the previous stage's velocity until ||g|| <= eps_n ||g0||
        (g0 the stage's first gradient), max_gn iterations or a failed line
        search; InvA while beta > pc_switch, else pc.  Returns (v, report)."""
        betas = []
        if continuation:
            b = 1.0
            while b > beta_target * (1 + 1e-12):
                betas.append(b)
                b /= 10.0
        betas.append(float(beta_target))
        v = np.array(v0, dtype=np.float64)
        rep = {"stages": 0, "gn_iters": 0, "pcg_iters": 0, "inner_iters": 0}
        self.set_velocity(v)
        for beta in betas:
            self.set_beta(beta)
            kind = "inva" if beta > pc_switch else pc
            rep["stages"] += 1
            g0 = None
            for _ in range(max_gn):
                g = self.gradient()
                gn = np.sqrt(inner(g, g, self.h3))
                g0 = gn if g0 is None else g0
                if gn <= eps_n * g0:
                    break
                v, info = self.gn_iterate(max_pcg, rtol, pc=kind, eps_h0=eps_h0, max_inner=max_inner)
                rep["gn_iters"] += 1
                rep["pcg_iters"] += info["pcg_iters"]
                rep["inner_iters"] += int(info["inner_iters"])
                if info["alpha"] == 0.0:
                    break
        g = self.gradient()
        rep["J"] = self.objective()[0]
        rep["gnorm_rel"] = float(np.sqrt(inner(g, g, self.h3)) / g0) if g0 else 0.0
        return v, rep

    def __del__(self):
        if getattr(self, "_ctx", None) and _lib is not None:
            _lib.or_ctx_destroy(self._ctx)
            self._ctx = None

    def set_images(self, m0, m1):
        a, pa = _c(m0)
        b, pb = _c(m1)
        lib().or_ctx_set_images(self._ctx, pa, pb)

    def set_velocity(self, v):
        a, pa = _c(v)
        lib().or_ctx_set_velocity(self._ctx, pa)

    def objective(self):
        out = np.empty(3)
        lib().or_ctx_objective(self._ctx, out.ctypes.data_as(ctypes.c_void_p))
        return float(out[0]), float(out[1]), float(out[2])

    def gradient(self):
        g = np.empty((3,) + self.shape)
        lib().or_ctx_gradient(self._ctx, g.ctypes.data_as(ctypes.c_void_p))
        return g

    def matvec(self, vt):
        a, pa = _c(vt)
        out = np.empty((3,) + self.shape)
        lib().or_ctx_matvec(self._ctx, pa, out.ctypes.data_as(ctypes.c_void_p))
        return out

    def inc_state(self, vt):
        a, pa = _c(vt)
        out = np.empty((self.nt + 1,) + self.shape)
        lib().or_ctx_inc_state(self._ctx, pa, out.ctypes.data_as(ctypes.c_void_p))
        return out

    def adjoint(self, phi):
        a, pa = _c(phi)
        out = np.empty((self.nt + 1,) + self.shape)
        lib().or_ctx_adjoint(self._ctx, pa, out.ctypes.data_as(ctypes.c_void_p))
        return out

    def body_force(self, lam):
        a, pa = _c(lam)
        out = np.empty((3,) + self.shape)
        lib().or_ctx_body_force(self._ctx, pa, out.ctypes.data_as(ctypes.c_void_p))
        return out

    def get(self, what, j=0):
        """'X', 'Xa', 'm', 'G', 'delta', 'delta_a', 'v'."""
        code = {"X": 0, "Xa": 1, "m": 2, "G": 3, "delta": 4, "delta_a": 5, "v": 6}[what]
        vec = what in ("X", "Xa", "G", "v")
        out = np.empty(((3,) if vec else ()) + self.shape)
        lib().or_ctx_get(self._ctx, code, int(j), out.ctypes.data_as(ctypes.c_void_p))
        return out

    def displacement(self, which="X"):
        """(X - x)/h in voxels, the departure points relative to the grid."""
        X = self.get(which)
        x = grid_points(self.shape)
        h = np.array([2 * np.pi / n for n in self.shape]).reshape(3, 1, 1, 1)
        return (X - x) / h

    def h0_apply(self, s):
        """H0 s = beta0 A s + grad m(1) (grad m(1) . s), beta0 = max(beta, 5e-2)
        (Section 2 "Preconditioning", eq. h0-pc)."""
        a, pa = _c(s)
        out = np.empty((3,) + self.shape)
        lib().or_ctx_h0_apply(self._ctx, pa, out.ctypes.data_as(ctypes.c_void_p))
        return out

    def invh0(self, r, tol, max_it):
        """Inner PCG solve of H0 s = r (Algorithm "PC"); returns (s, iterations)."""
        a, pa = _c(r)
        out = np.empty((3,) + self.shape)
        it = lib().or_ctx_invh0(self._ctx, pa, float(tol), int(max_it),
                                out.ctypes.data_as(ctypes.c_void_p))
        return out, int(it)

    def two_level_invh0(self, r, tol, max_it):
        """2LInvH0 (Algorithm "PC", second function); returns (s, coarse iterations)."""
        a, pa = _c(r)
        out = np.empty((3,) + self.shape)
        it = lib().or_ctx_2linvh0(self._ctx, pa, float(tol), int(max_it),
                                  out.ctypes.data_as(ctypes.c_void_p))
        return out, int(it)

    def pcg(self, rhs, max_it, rtol, pc="inva", eps_h0=1e-3, max_inner=50):
        if pc != "inva":
            a, pa = _c(rhs)
            x = np.empty((3,) + self.shape)
            info = np.empty(5)
            lib().or_ctx_pcg_pc(self._ctx, pa, int(max_it), float(rtol), {"invh0": 1, "2linvh0": 2}[pc],
                                float(eps_h0), int(max_inner), x.ctypes.data_as(ctypes.c_void_p),
                                info.ctypes.data_as(ctypes.c_void_p))
            return x, {"iters": int(info[0]), "rel_res": float(info[1]), "flags": int(info[2]),
                       "r0": float(info[3]), "inner": int(info[4])}
        return self._pcg_inva(rhs, max_it, rtol)

    def pcg_history(self, rhs, max_it, rtol, pc="inva", eps_h0=1e-3, max_inner=50):
        """PCG as pcg(), plus the relative residual ||r_k|| / ||r0|| after each
        iteration; returns (x, info, history[iterations])."""
        a, pa = _c(rhs)
        x = np.empty((3,) + self.shape)
        info = np.empty(5)
        hist = np.zeros(max(int(max_it), 1))
        lib().or_ctx_pcg_hist(self._ctx, pa, int(max_it), float(rtol),
                              {"inva": 0, "invh0": 1, "2linvh0": 2}[pc], float(eps_h0), int(max_inner),
                              x.ctypes.data_as(ctypes.c_void_p), info.ctypes.data_as(ctypes.c_void_p),
                              hist.ctypes.data_as(ctypes.c_void_p))
        d = {"iters": int(info[0]), "rel_res": float(info[1]), "flags": int(info[2]),
             "r0": float(info[3]), "inner": int(info[4])}
        return x, d, hist[:d["iters"]]

    def _pcg_inva(self, rhs, max_it, rtol):
        a, pa = _c(rhs)
        x = np.empty((3,) + self.shape)
        info = np.empty(4)
        lib().or_ctx_pcg(self._ctx, pa, int(max_it), float(rtol),
                         x.ctypes.data_as(ctypes.c_void_p), info.ctypes.data_as(ctypes.c_void_p))
        return x, {"iters": int(info[0]), "rel_res": float(info[1]), "flags": int(info[2]),
                   "r0": float(info[3])}

    def gn_iterate(self, max_pcg, rtol, pc="inva", eps_h0=1e-3, max_inner=50):
        v = np.empty((3,) + self.shape)
        info = np.empty(9)
        lib().or_ctx_gn_iterate_pc(self._ctx, int(max_pcg), float(rtol),
                                   {"inva": 0, "invh0": 1, "2linvh0": 2}[pc], float(eps_h0),
                                   int(max_inner),
                                   v.ctypes.data_as(ctypes.c_void_p),
                                   info.ctypes.data_as(ctypes.c_void_p))
        keys = ["pcg_iters", "rel_res", "flags", "alpha", "J_before", "J_after", "gnorm_rel",
                "gnorm", "inner_iters"]
        d = dict(zip(keys, info.tolist()))
        d["pcg_iters"] = int(d["pcg_iters"])
        d["flags"] = int(d["flags"])
        return v, d

    def transport(self, m0):
        a, pa = _c(m0)
        out = np.empty((self.nt + 1,) + self.shape)
        lib().or_ctx_transport(self._ctx, pa, out.ctypes.data_as(ctypes.c_void_p))
        return out

    def transport_vjp(self, m0, gout):
        a, pa = _c(m0)
        b, pb = _c(gout)
        gm0 = np.empty(self.shape)
        gv = np.empty((3,) + self.shape)
        lib().or_ctx_transport_vjp(self._ctx, pa, pb, gm0.ctypes.data_as(ctypes.c_void_p),
                                   gv.ctypes.data_as(ctypes.c_void_p))
        return gm0, gv
