"""MI355X randomized Krylov-Schur (rKS) eigensolver.

The numerical work runs in ``librks.so`` (hand-written HIP kernels for gfx950
plus the host driver), reached through the C-ABI declared in include/rks.h.
This package is the thin Python binding: ``_binding`` mirrors the C names,
``Solver`` bundles create/solve/eigpairs/destroy for convenience.
"""
import numpy as np

from . import _binding as rks
from ._binding import (RksError, RksOpts, RksStats, load, rks_opts_default, rks_create, rks_solve,
                       rks_num_pairs, rks_eigpairs, rks_destroy, rks_strerror, rks_last_error,
                       rks_sketch, rks_sketch_noalloc, rks_spmv_sketch, rks_arnoldi, rks_get_state, rks_rotate,
                       rks_host_schur, rks_host_order, rks_net_conv3x3_forward, rks_net_conv3x3_backward,
                       rks_net_subspace_loss, rks_net_adam, rks_net_upsample, rks_copy_probe, rks_read_probe)

__all__ = ["Solver", "RksError", "RksOpts", "RksStats", "load", "rks_opts_default", "rks_create",
           "rks_solve", "rks_num_pairs", "rks_eigpairs", "rks_destroy", "rks_strerror",
           "rks_last_error", "rks_sketch", "rks_sketch_noalloc", "rks_spmv_sketch", "rks_arnoldi", "rks_get_state",
           "rks_rotate", "rks_host_schur", "rks_host_order", "rks_net_conv3x3_forward",
           "rks_net_conv3x3_backward", "rks_net_subspace_loss", "rks_net_adam", "rks_net_upsample",
           "rks_copy_probe", "rks_read_probe"]


class Solver:
    """create -> solve -> eigpairs on one CSR matrix (host NumPy arrays)."""

    def __init__(self, row_ptr, col, val, n, k, m, d, which="LM", tol=1e-10, **opts):
        self.n, self.k, self.m, self.d = int(n), int(k), int(m), int(d)
        self.opts = rks_opts_default(**opts)
        self.ctx = rks_create(row_ptr, col, val, n, k, m, d, which, tol, self.opts)
        self.stats = RksStats()

    @classmethod
    def from_csr(cls, A, **kw):
        return cls(A.row_ptr, A.col, A.val, A.n, **kw)

    def solve(self, u0=None) -> int:
        self.stats = RksStats()
        return rks_solve(self.ctx, u0, self.stats)

    def eigpairs(self, want_vectors=True, want_resid=True):
        ke = rks_num_pairs(self.ctx)
        lr = np.zeros(ke)
        li = np.zeros(ke)
        X = np.zeros((self.n, ke), order="F") if want_vectors else None
        res = np.zeros(ke) if want_resid else None
        rks_eigpairs(self.ctx, lr, li, X, res)
        return lr + 1j * li, X, res

    def close(self):
        if self.ctx:
            rks_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
