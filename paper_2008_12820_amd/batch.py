"""Batch: many independent registrations of uneven grid sizes advanced one
Gauss-Newton iteration at a time (lddmm_batch_* in include/lddmm.h)."""
import torch

from . import _lib as L


class Batch:
    def __init__(self, shapes, nt, reg=L.REG_H2S, beta=1e-3, leray=False, nstreams=8):
        self.shapes = [tuple(int(x) for x in s) for s in shapes]
        self.nt = int(nt)
        self.cfgs = [L.make_config(s, nt, reg, beta, leray) for s in self.shapes]
        self._h = L.lddmm_batch_create(self.cfgs, nstreams)

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.lddmm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.shapes)

    def set_images(self, m0s, m1s):
        L.lddmm_batch_set_images(self._h, [t.contiguous() for t in m0s], [t.contiguous() for t in m1s])

    def set_velocity(self, vs):
        L.lddmm_batch_set_velocity(self._h, [t.contiguous() for t in vs])

    def gn_iterate(self, vs, max_pcg, rtol=0.0, use_graph=True):
        """vs: list of [3, n, n, n] float32 tensors, updated in place."""
        torch.cuda.synchronize()
        return L.lddmm_batch_gn_iterate(self._h, max_pcg, rtol, use_graph, vs)

    def objective(self, b):
        return L.lddmm_objective(L.lddmm_batch_plan(self._h, b))
