"""torch.autograd binding of the contact volumes and their Jacobian.

``contact_volumes(ctx, dscene, x0, x1, d, eps, dt)`` runs the detect on
device tensors x0, x1 ([3, n_vtx] float64) and returns

    V      [n_vol]       contact volumes (differentiable)
    G      [n_jrow, 3]   Jacobian rows dV/dX1 (differentiable)
    index  dict of non-differentiable tensors: vol_pair, j_vol, j_vtx, ...

The backward is the library's hand-written kernel (stiv_backward): the exact
vector-Jacobian product of V and G with respect to x0 and x1, including the
Hessian-vector products of G and the dependence of the contact times on the
positions.  The contact set itself is piecewise constant in the positions.
"""
import torch

from . import stiv


class STIVFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x0, x1, ctx, dscene, d, eps, dt):
        ds = stiv.DeviceScene.__new__(stiv.DeviceScene)
        ds.__dict__.update(dscene.__dict__)
        ds.x0 = x0.detach().contiguous()
        ds.x1 = x1.detach().contiguous()
        res, outs = stiv.detect(ctx, ds, d, eps, dt, outputs=None, to_numpy=False)
        fctx.stiv = (ctx, ds, d, eps, dt, res["_struct"], outs)
        V = res["vol_V"].clone()
        G = res["j_g"].clone()
        idx = {k: res[k].clone() for k in ("vol_pair", "j_vol", "j_vtx", "pair_ab", "pair_shift", "ct_key", "ct_tau")}
        fctx.idx = idx
        return V, G

    @staticmethod
    def backward(fctx, gV, gG):
        ctx, ds, d, eps, dt, r, outs = fctx.stiv
        dX0, dX1 = stiv.backward(ctx, ds, d, eps, dt, r,
                                 gV.contiguous() if gV is not None else None,
                                 gG.contiguous() if gG is not None else None)
        return dX0, dX1, None, None, None, None, None


def contact_volumes(ctx, dscene, x0, x1, d, eps, dt):
    """(V, G, index) with autograd through the library's backward kernel."""
    holder = {}

    class _F(STIVFunction):
        @staticmethod
        def forward(fctx, *args):
            out = STIVFunction.forward(fctx, *args)
            holder["idx"] = fctx.idx
            return out

    V, G = _F.apply(x0, x1, ctx, dscene, d, eps, dt)
    return V, G, holder["idx"]
