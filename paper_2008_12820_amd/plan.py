"""Plan: owns one lddmm_plan (device workspace for one registration problem)
and marshals torch tensors to the C calls of include/lddmm.h."""
import torch

from . import _lib as L


class Plan:
    def __init__(self, shape, nt, reg=L.REG_H1S, beta=1e-2, leray=False, device=None,
                 stream=None, transport_only=False, fd8=False, linear_ip=False):
        self.shape = tuple(int(s) for s in shape)
        self.nt = int(nt)
        self.reg = int(reg)
        self.beta = float(beta)
        self.leray = bool(leray)
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        self.cfg = L.make_config(self.shape, self.nt, self.reg, self.beta, self.leray,
                                 (L.FLAG_TRANSPORT_ONLY if transport_only else 0) |
                                 (L.FLAG_FD8 if fd8 else 0) |
                                 (L.FLAG_LINEAR_IP if linear_ip else 0))
        with torch.cuda.device(self.device):
            self._h = L.lddmm_plan_create(self.cfg, s.cuda_stream)

    # ---- lifetime ----
    def close(self):
        if getattr(self, "_h", None) is not None:
            L.lddmm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def workspace_bytes(shape, nt, reg=L.REG_H1S, beta=1e-2, leray=False, transport_only=False):
        return L.lddmm_workspace_bytes(L.make_config(
            shape, nt, reg, beta, leray, L.FLAG_TRANSPORT_ONLY if transport_only else 0))

    # ---- helpers ----
    def _scalar(self):
        return torch.empty(self.shape, device=self.device, dtype=torch.float32)

    def _vector(self):
        return torch.empty((3,) + self.shape, device=self.device, dtype=torch.float32)

    def _in(self, t, vec):
        shp = ((3,) if vec else ()) + self.shape
        if tuple(t.shape) != shp:
            raise ValueError(f"expected shape {shp}, got {tuple(t.shape)}")
        if t.device != self.device:
            raise ValueError(f"tensor on {t.device}, plan on {self.device}")
        return t.contiguous().to(torch.float32)

    # ---- calls ----
    def set_images(self, m0, m1):
        L.lddmm_set_images(self._h, self._in(m0, False), self._in(m1, False))

    def set_velocity(self, v):
        L.lddmm_set_velocity(self._h, self._in(v, True))

    def objective(self):
        return L.lddmm_objective(self._h)

    def gradient(self, out=None):
        g = out if out is not None else self._vector()
        gn = L.lddmm_gradient(self._h, g)
        return g, gn

    def hessian_matvec(self, vt, out=None):
        hv = out if out is not None else self._vector()
        L.lddmm_hessian_matvec(self._h, self._in(vt, True), hv)
        return hv

    def apply_inv_reg(self, r, out=None):
        s = out if out is not None else self._vector()
        L.lddmm_apply_inv_reg(self._h, self._in(r, True), s)
        return s

    def set_preconditioner(self, kind, eps_h0=1e-3, max_inner=50):
        """kind "inva" ((beta A)^-1), "invh0" (inner PCG on eq. h0-pc) or
        "2linvh0" (the same on the half grid)"""
        L.lddmm_set_preconditioner(self._h, {"inva": 0, "invh0": 1, "2linvh0": 2}[kind], eps_h0, max_inner)

    def set_beta(self, beta):
        L.lddmm_set_beta(self._h, beta)
        self.beta = float(beta)

    def gn_solve(self, v, beta_target, eps_n=5e-2, max_gn=10, max_pcg=50, rtol=0.0, continuation=True,
                 pc="2linvh0", eps_h0=1e-3, max_inner=50, pc_switch=0.5):
        """Gauss-Newton-Krylov solve with beta-continuation (lddmm_gn_solve);
        v (initial velocity) is overwritten with the result; returns the report."""
        rep = L.lddmm_gn_solve(self._h, v, beta_target, eps_n=eps_n, rtol=rtol, eps_h0=eps_h0,
                               pc_switch=pc_switch, max_gn=max_gn, max_pcg=max_pcg, max_inner=max_inner,
                               continuation=continuation, pc_kind={"inva": 0, "invh0": 1, "2linvh0": 2}[pc])
        self.beta = float(beta_target)
        return rep

    def apply_h0(self, s, out=None):
        o = out if out is not None else self._vector()
        L.lddmm_apply_h0(self._h, self._in(s, True), o)
        return o

    def apply_invh0(self, r, tol, max_inner, out=None):
        s = out if out is not None else self._vector()
        it = L.lddmm_apply_invh0(self._h, self._in(r, True), tol, max_inner, s)
        return s, it

    def apply_2linvh0(self, r, tol, max_inner, out=None):
        s = out if out is not None else self._vector()
        it = L.lddmm_apply_2linvh0(self._h, self._in(r, True), tol, max_inner, s)
        return s, it

    def newton_step(self, max_pcg, rtol=0.0, out=None, allow_notconv=False):
        vt = out if out is not None else self._vector()
        st, info = L.lddmm_newton_step(self._h, max_pcg, rtol, vt, allow_notconv)
        info["status"] = st
        return vt, info

    def pcg_history(self):
        """relative residuals ||r_k|| / ||r0|| of the last PCG solve"""
        return L.lddmm_pcg_history(self._h)

    def gn_iterate(self, v, max_pcg, rtol=0.0):
        """v (updated in place) must equal the plan's current velocity."""
        return L.lddmm_gn_iterate(self._h, max_pcg, rtol, v)

    def transport_forward(self, m0, v, ckpt=None):
        m1 = self._scalar()
        L.lddmm_transport_forward(self._h, self._in(m0, False), self._in(v, True), m1, ckpt)
        return m1

    def transport_vjp(self, ckpt, v, grad_m1, want_m0=True, want_v=True):
        gm0 = self._scalar() if want_m0 else None
        gv = self._vector() if want_v else None
        L.lddmm_transport_vjp(self._h, ckpt, self._in(v, True), self._in(grad_m1, False), gm0, gv)
        return gm0, gv

    def reg_energy(self, v, want_Av=True):
        """(1/2 sum (A v).v, A v) -- plain sums, beta not applied."""
        Av = self._vector() if want_Av else None
        e = L.lddmm_reg_energy(self._h, self._in(v, True), Av)
        return e, Av

    def fft_r2c(self, f):
        n1, n2, n3 = self.shape
        out = torch.empty((n1, n2, n3 // 2 + 1, 2), device=self.device, dtype=torch.float32)
        L.lddmm_fft_r2c(self._h, self._in(f, False), out)
        return torch.view_as_complex(out)

    def fft_c2r(self, fhat):
        n1, n2, n3 = self.shape
        fr = torch.view_as_real(fhat.to(torch.complex64).contiguous()).contiguous()
        out = self._scalar()
        L.lddmm_fft_c2r(self._h, fr, out)
        return out

    def spectral_op(self, op, x):
        nin = 1 if op == L.OP_GRAD else 3
        nout = 1 if op == L.OP_DIV else 3
        x = self._in(x, nin == 3)
        out = self._vector() if nout == 3 else self._scalar()
        L.lddmm_spectral_op(self._h, op, x, out)
        return out

    def interp(self, fields, disp):
        """fields: [nf, n1, n2, n3] (or one scalar field); disp: [3, n1, n2, n3] voxels."""
        single = fields.dim() == 3
        f = (fields[None] if single else fields).contiguous().to(torch.float32)
        out = torch.empty_like(f)
        L.lddmm_interp(self._h, f.shape[0], f, self._in(disp, True), out)
        return out[0] if single else out

    def get_field(self, what, j=0):
        if what in (L.FIELD_PCG_R_HAT, L.FIELD_PCG_P_HAT):  # three half spectra, complex64
            n1, n2, n3 = self.shape
            out = torch.empty((3, n1, n2, n3 // 2 + 1), device=self.device, dtype=torch.complex64)
            L.lddmm_get_field(self._h, what, j, torch.view_as_real(out))
            return out
        vec = what in (L.FIELD_DISP, L.FIELD_DISP_ADJ, L.FIELD_GRAD_STATE, L.FIELD_PCG_R, L.FIELD_PCG_Z,
                       L.FIELD_PCG_P)
        out = self._vector() if vec else self._scalar()
        L.lddmm_get_field(self._h, what, j, out)
        return out

    def autotune(self):
        L.lddmm_autotune(self._h)
        return L.lddmm_tuning(self._h)

    def set_gather_mode(self, mode):
        L.lddmm_set_gather_mode(self._h, mode)

    def set_overlap(self, enable):
        L.lddmm_set_overlap(self._h, enable)

    def tuning(self):
        return L.lddmm_tuning(self._h)

    def set_timing(self, enable, only=None):
        """enable per-kernel HIP-event timing; only: a kernel class name to
        bracket alone (the other launches stay unbracketed)"""
        if enable and only is not None:
            ids = {L.lddmm_kernel_name(k): k for k in range(L.lddmm_num_kernels())}
            L.lddmm_set_timing_only(self._h, ids[only])
        else:
            L.lddmm_set_timing(self._h, enable)

    def timing(self):
        """{kernel name: (total ms, launches)} since the last set_timing."""
        out = {}
        for k in range(L.lddmm_num_kernels()):
            ms, n = L.lddmm_get_timing(self._h, k)
            if n:
                out[L.lddmm_kernel_name(k)] = (ms, n)
        return out
