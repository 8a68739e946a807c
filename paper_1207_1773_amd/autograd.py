"""torch.autograd.Function for the differentiable generalized solve.

forward: hgv_zhegvx computes every eigenpair (the reverse mode needs the complement of
the selected pairs), hgv_gauge_fix makes the entry of largest modulus of each eigenvector
real and positive, and the selected pairs il..iu are returned.
backward: hgv_zhegvx_backward turns (dL/dW, dL/dX) into (Abar, Bbar), Hermitian, such that
dL = Re tr(Abar^H dA) + Re tr(Bbar^H dB) for Hermitian perturbations (the solve reads
the lower triangles, i.e. A and B are treated as Hermitian matrices).
All arithmetic runs in the library's kernels; this module only marshals tensors.
"""
import ctypes

import torch

from . import hgv_gauge_fix, hgv_zhegvx_backward, hgv_zhegvx_backward_bufsize
from .tensors import Context, _ptr, colmajor, from_colmajor


class EighGeneralized(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, il, iu, nb=0):
        hc = Context.get(A.device)
        n = A.shape[0]
        lam, Xall, info, _ = hc.zhegvx(A, B, 1, n, "fp64", nb)
        if info != 0:
            raise RuntimeError("hgv_zhegvx failed: info = %d" % info)
        Xc = Xall.mT.contiguous()                 # column-major buffer of Xall (n x n)
        hc._sync_stream()
        hgv_gauge_fix(hc.handle, n, n, _ptr(Xc), max(n, 1))
        Xall = from_colmajor(Xc)
        ctx.save_for_backward(lam, Xc)
        ctx.il, ctx.iu, ctx.n = il, iu, n
        return lam[il - 1:iu].clone(), Xall[:, il - 1:iu].clone()

    @staticmethod
    def backward(ctx, gW, gX):
        lam, Xc = ctx.saved_tensors
        il, iu, n = ctx.il, ctx.iu, ctx.n
        m = iu - il + 1
        dev = lam.device
        hc = Context.get(dev)
        hc._sync_stream()
        Wbar = (gW if gW is not None else torch.zeros(m, dtype=torch.float64, device=dev)).contiguous()
        Gb = gX if gX is not None else torch.zeros((n, m), dtype=torch.complex128, device=dev)
        Gc = colmajor(Gb)
        Ab = torch.empty((n, n), dtype=torch.complex128, device=dev)
        Bb = torch.empty((n, n), dtype=torch.complex128, device=dev)
        w = hc._work(hgv_zhegvx_backward_bufsize(hc.handle, n, il, iu))
        hgv_zhegvx_backward(hc.handle, n, il, iu, _ptr(lam), _ptr(Xc), max(n, 1), _ptr(Wbar), _ptr(Gc), max(n, 1),
                            _ptr(Ab), max(n, 1), _ptr(Bb), max(n, 1), _ptr(w), w.numel())
        # Ab, Bb hold the gradients column-major; from_colmajor views them as matrices
        return from_colmajor(Ab), from_colmajor(Bb), None, None, None


def eigh_differentiable(A, B, il=1, iu=None, nb=0):
    """Selected eigenpairs (W, X) of A x = lambda B x with gradients to A and B."""
    n = A.shape[0]
    return EighGeneralized.apply(A, B, il, n if iu is None else iu, nb)
