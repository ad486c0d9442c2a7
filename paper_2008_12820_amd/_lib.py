"""ctypes binding of liblddmm.so (the C ABI declared in include/lddmm.h).

Argument marshalling only: every function here forwards to the C call of the
same name.  Device arrays are passed as torch tensors (float32, contiguous,
on the plan's device) and handed over as raw device pointers.  The library
is never emulated: if liblddmm.so is missing the import fails loudly.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblddmm.so")

# status codes (lddmm_status)
OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOTCONV, EUNSUPPORTED = range(7)
REG_H1S, REG_H2S = 1, 2
OP_GRAD, OP_DIV, OP_REG, OP_INVREG, OP_LERAY = 1, 2, 3, 4, 5
FIELD_DISP, FIELD_DISP_ADJ, FIELD_STATE, FIELD_GRAD_STATE, FIELD_DIV, FIELD_INC_STATE, \
    FIELD_ADJOINT, FIELD_PCG_R, FIELD_PCG_Z, FIELD_PCG_P, FIELD_PCG_R_HAT, FIELD_PCG_P_HAT = \
    1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12


FLAG_TRANSPORT_ONLY = 1
FLAG_FD8 = 2
FLAG_LINEAR_IP = 4


class Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("nt", ctypes.c_int32), ("reg", ctypes.c_int32),
                ("leray", ctypes.c_int32), ("flags", ctypes.c_int32), ("beta", ctypes.c_double)]


class NewtonInfo(ctypes.Structure):
    _fields_ = [("pcg_iters", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("alpha", ctypes.c_double),
                ("J_before", ctypes.c_double), ("J_after", ctypes.c_double),
                ("gnorm", ctypes.c_double), ("gnorm_rel", ctypes.c_double),
                ("inner_iters", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class SolveOpts(ctypes.Structure):
    _fields_ = [("beta_target", ctypes.c_double), ("eps_n", ctypes.c_double), ("rtol", ctypes.c_double),
                ("eps_h0", ctypes.c_double), ("pc_switch", ctypes.c_double), ("max_gn", ctypes.c_int32),
                ("max_pcg", ctypes.c_int32), ("max_inner", ctypes.c_int32), ("continuation", ctypes.c_int32),
                ("pc_kind", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SolveReport(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("gn_iters", ctypes.c_int32), ("pcg_iters", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("J", ctypes.c_double), ("gnorm_rel", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LddmmError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: {status_string(status)} ({detail})")
        self.status = status


_lib = None


def lib():
    """Load liblddmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        p, i32, d, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        st = ctypes.c_int
        P = ctypes.POINTER
        sigs = {
            "lddmm_workspace_bytes": (st, [P(Config), P(sz)]),
            "lddmm_plan_create": (st, [P(Config), p, P(p)]),
            "lddmm_plan_destroy": (st, [p]),
            "lddmm_set_images": (st, [p, p, p]),
            "lddmm_set_velocity": (st, [p, p]),
            "lddmm_objective": (st, [p, P(d), P(d), P(d)]),
            "lddmm_gradient": (st, [p, p, P(d)]),
            "lddmm_hessian_matvec": (st, [p, p, p]),
            "lddmm_apply_inv_reg": (st, [p, p, p]),
            "lddmm_set_preconditioner": (st, [p, i32, d, i32]),
            "lddmm_set_beta": (st, [p, d]),
            "lddmm_set_timing_only": (st, [p, i32]),
            "lddmm_gn_solve": (st, [p, P(SolveOpts), p, P(SolveReport)]),
            "lddmm_apply_h0": (st, [p, p, p]),
            "lddmm_apply_invh0": (st, [p, p, d, i32, p, P(i32)]),
            "lddmm_apply_2linvh0": (st, [p, p, d, i32, p, P(i32)]),
            "lddmm_newton_step": (st, [p, i32, d, p, P(NewtonInfo)]),
            "lddmm_gn_iterate": (st, [p, i32, d, p, P(NewtonInfo)]),
            "lddmm_pcg_history": (st, [p, P(d), i32, P(i32)]),
            "lddmm_transport_forward": (st, [p, p, p, p, p]),
            "lddmm_transport_vjp": (st, [p, p, p, p, p, p]),
            "lddmm_transport_forward_static": (st, [P(Config), p, p, p, p, p]),
            "lddmm_reg_energy": (st, [p, p, p, P(d)]),
            "lddmm_fft_r2c": (st, [p, p, p]),
            "lddmm_fft_c2r": (st, [p, p, p]),
            "lddmm_spectral_op": (st, [p, i32, p, p]),
            "lddmm_interp": (st, [p, i32, p, p, p]),
            "lddmm_get_field": (st, [p, i32, i32, p]),
            "lddmm_batch_create": (st, [i32, P(Config), i32, P(p)]),
            "lddmm_batch_destroy": (st, [p]),
            "lddmm_batch_plan": (st, [p, i32, P(p)]),
            "lddmm_batch_set_images": (st, [p, P(p), P(p)]),
            "lddmm_batch_set_velocity": (st, [p, P(p)]),
            "lddmm_batch_gn_iterate": (st, [p, i32, d, i32, P(p), P(NewtonInfo)]),
            "lddmm_autotune": (st, [p]),
            "lddmm_set_gather_mode": (st, [p, i32]),
            "lddmm_set_overlap": (st, [p, i32]),
            "lddmm_tuning": (st, [p, ctypes.c_char_p, sz]),
            "lddmm_set_timing": (st, [p, i32]),
            "lddmm_get_timing": (st, [p, i32, P(d), P(ctypes.c_int64)]),
            "lddmm_num_kernels": (i32, []),
            "lddmm_kernel_name": (ctypes.c_char_p, [i32]),
            "lddmm_status_string": (ctypes.c_char_p, [st]),
            "lddmm_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(s):
    return lib().lddmm_status_string(s).decode()


def last_error():
    return lib().lddmm_last_error().decode()


def _check(status, where):
    if status != OK:
        raise LddmmError(status, where, last_error())
    return status


def _ptr(t):
    """Raw device pointer of a float32 contiguous tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("expected a contiguous float32 tensor")
    return ctypes.c_void_p(t.data_ptr())


def make_config(n, nt, reg=REG_H1S, beta=1e-2, leray=False, flags=0):
    c = Config()
    c.n[0], c.n[1], c.n[2] = (int(x) for x in n)
    c.nt, c.reg, c.leray, c.beta = int(nt), int(reg), int(bool(leray)), float(beta)
    c.flags = int(flags)
    return c


# ---- one wrapper per C call ------------------------------------------------

def lddmm_workspace_bytes(cfg):
    out = ctypes.c_size_t()
    _check(lib().lddmm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)), "workspace_bytes")
    return out.value


def lddmm_plan_create(cfg, stream):
    h = ctypes.c_void_p()
    _check(lib().lddmm_plan_create(ctypes.byref(cfg), ctypes.c_void_p(stream), ctypes.byref(h)),
           "plan_create")
    return h


def lddmm_plan_destroy(plan):
    _check(lib().lddmm_plan_destroy(plan), "plan_destroy")


def lddmm_set_images(plan, m0, m1):
    _check(lib().lddmm_set_images(plan, _ptr(m0), _ptr(m1)), "set_images")


def lddmm_set_velocity(plan, v):
    _check(lib().lddmm_set_velocity(plan, _ptr(v)), "set_velocity")


def lddmm_objective(plan):
    J, m, r = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().lddmm_objective(plan, ctypes.byref(J), ctypes.byref(m), ctypes.byref(r)),
           "objective")
    return J.value, m.value, r.value


def lddmm_gradient(plan, g):
    gn = ctypes.c_double()
    _check(lib().lddmm_gradient(plan, _ptr(g), ctypes.byref(gn)), "gradient")
    return gn.value


def lddmm_hessian_matvec(plan, vt, hvt):
    _check(lib().lddmm_hessian_matvec(plan, _ptr(vt), _ptr(hvt)), "hessian_matvec")


def lddmm_apply_inv_reg(plan, r, s):
    _check(lib().lddmm_apply_inv_reg(plan, _ptr(r), _ptr(s)), "apply_inv_reg")


def lddmm_set_beta(plan, beta):
    _check(lib().lddmm_set_beta(plan, float(beta)), "set_beta")


def lddmm_gn_solve(plan, v_inout, beta_target, eps_n=5e-2, rtol=0.0, eps_h0=1e-3, pc_switch=0.5, max_gn=10,
                   max_pcg=50, max_inner=50, continuation=True, pc_kind=2):
    o = SolveOpts(beta_target=float(beta_target), eps_n=float(eps_n), rtol=float(rtol), eps_h0=float(eps_h0),
                  pc_switch=float(pc_switch), max_gn=int(max_gn), max_pcg=int(max_pcg), max_inner=int(max_inner),
                  continuation=int(bool(continuation)), pc_kind=int(pc_kind), reserved=0)
    rep = SolveReport()
    _check(lib().lddmm_gn_solve(plan, ctypes.byref(o), _ptr(v_inout), ctypes.byref(rep)), "gn_solve")
    return rep.as_dict()


def lddmm_set_preconditioner(plan, kind, eps_h0=1e-3, max_inner=50):
    _check(lib().lddmm_set_preconditioner(plan, int(kind), float(eps_h0), int(max_inner)),
           "set_preconditioner")


def lddmm_apply_h0(plan, s, out):
    _check(lib().lddmm_apply_h0(plan, _ptr(s), _ptr(out)), "apply_h0")


def lddmm_apply_invh0(plan, r, tol, max_inner, s):
    it = ctypes.c_int32(0)
    _check(lib().lddmm_apply_invh0(plan, _ptr(r), float(tol), int(max_inner), _ptr(s), ctypes.byref(it)),
           "apply_invh0")
    return it.value


def lddmm_apply_2linvh0(plan, r, tol, max_inner, s):
    it = ctypes.c_int32(0)
    _check(lib().lddmm_apply_2linvh0(plan, _ptr(r), float(tol), int(max_inner), _ptr(s), ctypes.byref(it)),
           "apply_2linvh0")
    return it.value


def lddmm_newton_step(plan, max_pcg, rtol, vt_out, allow_notconv=False):
    info = NewtonInfo()
    st = lib().lddmm_newton_step(plan, int(max_pcg), float(rtol), _ptr(vt_out), ctypes.byref(info))
    if not (allow_notconv and st == ENOTCONV):
        _check(st, "newton_step")
    return st, info.as_dict()


def lddmm_pcg_history(plan, maxlen=4096):
    """||r_k|| / ||r0|| after each iteration of the last PCG (a list)"""
    buf = (ctypes.c_double * max(int(maxlen), 1))()
    cnt = ctypes.c_int32(0)
    _check(lib().lddmm_pcg_history(plan, buf, int(maxlen), ctypes.byref(cnt)), "pcg_history")
    return [buf[k] for k in range(min(cnt.value, int(maxlen)))]


def lddmm_gn_iterate(plan, max_pcg, rtol, v_inout):
    info = NewtonInfo()
    _check(lib().lddmm_gn_iterate(plan, int(max_pcg), float(rtol), _ptr(v_inout),
                                  ctypes.byref(info)), "gn_iterate")
    return info.as_dict()


def lddmm_transport_forward(plan, m0, v, m1_out, ckpt=None):
    _check(lib().lddmm_transport_forward(plan, _ptr(m0), _ptr(v), _ptr(m1_out), _ptr(ckpt)),
           "transport_forward")


def lddmm_transport_forward_static(cfg, stream, m0, v, m1_out, ckpt=None):
    _check(lib().lddmm_transport_forward_static(ctypes.byref(cfg), ctypes.c_void_p(stream), _ptr(m0), _ptr(v),
                                                _ptr(m1_out), _ptr(ckpt)), "transport_forward_static")


def lddmm_transport_vjp(plan, ckpt, v, grad_m1, grad_m0=None, grad_v=None):
    _check(lib().lddmm_transport_vjp(plan, _ptr(ckpt), _ptr(v), _ptr(grad_m1), _ptr(grad_m0),
                                     _ptr(grad_v)), "transport_vjp")


def lddmm_reg_energy(plan, v, Av=None):
    e = ctypes.c_double()
    _check(lib().lddmm_reg_energy(plan, _ptr(v), _ptr(Av), ctypes.byref(e)), "reg_energy")
    return e.value


def lddmm_fft_r2c(plan, f, fhat):
    _check(lib().lddmm_fft_r2c(plan, _ptr(f), _ptr(fhat)), "fft_r2c")


def lddmm_fft_c2r(plan, fhat, f):
    _check(lib().lddmm_fft_c2r(plan, _ptr(fhat), _ptr(f)), "fft_c2r")


def lddmm_spectral_op(plan, op, x, out):
    _check(lib().lddmm_spectral_op(plan, int(op), _ptr(x), _ptr(out)), "spectral_op")


def lddmm_interp(plan, nfields, fields, disp, out):
    _check(lib().lddmm_interp(plan, int(nfields), _ptr(fields), _ptr(disp), _ptr(out)), "interp")


def lddmm_get_field(plan, what, j, out):
    _check(lib().lddmm_get_field(plan, int(what), int(j), _ptr(out)), "get_field")


def _ptr_array(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _ptr(t).value
    return arr


def lddmm_batch_create(cfgs, nstreams):
    arr = (Config * len(cfgs))(*cfgs)
    h = ctypes.c_void_p()
    _check(lib().lddmm_batch_create(len(cfgs), arr, int(nstreams), ctypes.byref(h)), "batch_create")
    return h


def lddmm_batch_destroy(batch):
    _check(lib().lddmm_batch_destroy(batch), "batch_destroy")


def lddmm_batch_plan(batch, b):
    h = ctypes.c_void_p()
    _check(lib().lddmm_batch_plan(batch, int(b), ctypes.byref(h)), "batch_plan")
    return h


def lddmm_batch_set_images(batch, m0s, m1s):
    _check(lib().lddmm_batch_set_images(batch, _ptr_array(m0s), _ptr_array(m1s)), "batch_set_images")


def lddmm_batch_set_velocity(batch, vs):
    _check(lib().lddmm_batch_set_velocity(batch, _ptr_array(vs)), "batch_set_velocity")


def lddmm_batch_gn_iterate(batch, max_pcg, rtol, use_graph, vs):
    infos = (NewtonInfo * len(vs))()
    _check(lib().lddmm_batch_gn_iterate(batch, int(max_pcg), float(rtol), int(bool(use_graph)),
                                        _ptr_array(vs), infos), "batch_gn_iterate")
    return [i.as_dict() for i in infos]


def lddmm_autotune(plan):
    _check(lib().lddmm_autotune(plan), "autotune")


def lddmm_set_gather_mode(plan, mode):
    _check(lib().lddmm_set_gather_mode(plan, int(mode)), "set_gather_mode")


def lddmm_set_overlap(plan, enable):
    _check(lib().lddmm_set_overlap(plan, int(bool(enable))), "set_overlap")


def lddmm_tuning(plan):
    buf = ctypes.create_string_buffer(1024)
    _check(lib().lddmm_tuning(plan, buf, 1024), "tuning")
    return buf.value.decode()


def lddmm_set_timing(plan, enable):
    _check(lib().lddmm_set_timing(plan, int(bool(enable))), "set_timing")


def lddmm_set_timing_only(plan, kernel_id):
    _check(lib().lddmm_set_timing_only(plan, int(kernel_id)), "set_timing_only")


def lddmm_get_timing(plan, kernel_id):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().lddmm_get_timing(plan, int(kernel_id), ctypes.byref(ms), ctypes.byref(n)),
           "get_timing")
    return ms.value, n.value


def lddmm_num_kernels():
    return lib().lddmm_num_kernels()


def lddmm_kernel_name(i):
    return lib().lddmm_kernel_name(int(i)).decode()
