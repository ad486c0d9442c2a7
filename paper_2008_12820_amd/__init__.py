"""MI355X (gfx950) Gauss-Newton-Krylov hot path for LDDMM registration
(Brunn et al., arXiv 2008.12820) behind a C ABI (include/lddmm.h).

    from paper_2008_12820_amd import Plan
    plan = Plan((256, 256, 256), nt=4, reg=2, beta=5e-4)
    plan.set_images(m0, m1); plan.set_velocity(v)
    g, gnorm = plan.gradient(); Hv = plan.hessian_matvec(vt)

All tensors are float32 CUDA (HIP) tensors; scalar fields are [n1, n2, n3],
vector fields [3, n1, n2, n3].  Every call runs in liblddmm.so.
"""
from . import _lib
from ._lib import (EDEVICE, EINVAL, ENOMEM, ENOTCONV, ESTATE, EUNSUPPORTED, OK, OP_DIV,  # noqa
                   OP_GRAD, OP_INVREG, OP_LERAY, OP_REG, REG_H1S, REG_H2S, LddmmError)
from .plan import Plan  # noqa: F401

__all__ = ["Plan", "LddmmError"]
