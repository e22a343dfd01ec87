"""SFBcast and SFReduce(SUM) as mutually adjoint autograd functions.

Section 4.1 of the paper pairs the two operations: y = M x gathers the
ghost entries with SFBcast, y = M^T x adds them back with SFReduce SUM.  As
linear maps on unit data they are transposes of each other -- Bcast is
leaf = P root, Reduce SUM is root + P^T leaf -- so each one's backward is the
other one on the same star forest:

  SFBcastFn:      leaf = P root            d root = P^T d leaf   (Reduce SUM onto zeros)
  SFReduceSumFn:  out = root + P^T leaf    d leaf = P d out       (Bcast; holes get 0)
                                           d root = d out

Both forward and backward run in the library's kernels on the current
stream; with the SF in deterministic mode every Reduce is bit-reproducible.
"""
import torch
import torch.utils.checkpoint

from . import sf as S


def _leaf_shape(sf_obj, root):
    return (sf_obj.leafspace,) + tuple(root.shape[1:])


class SFBcastFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sfo, root):
        root = root.contiguous()
        leaf = torch.zeros(_leaf_shape(sfo, root), dtype=root.dtype, device=root.device)
        sfo.bcast(root, leaf, "replace")
        ctx.sfo = sfo
        ctx.root_shape = root.shape
        return leaf

    @staticmethod
    def backward(ctx, gleaf):
        groot = torch.zeros(ctx.root_shape, dtype=gleaf.dtype, device=gleaf.device)
        ctx.sfo.reduce(gleaf.contiguous(), groot, "sum")
        return None, groot


class SFReduceSumFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sfo, leaf, root):
        out = root.contiguous().clone()
        sfo.reduce(leaf.contiguous(), out, "sum")
        ctx.sfo = sfo
        ctx.leaf_shape = leaf.shape
        return out

    @staticmethod
    def backward(ctx, gout):
        gout = gout.contiguous()
        gleaf = torch.zeros(ctx.leaf_shape, dtype=gout.dtype, device=gout.device)
        ctx.sfo.bcast(gout, gleaf, "replace")
        return None, gleaf, gout


class DiffSF:
    """A star forest usable inside autograd graphs."""

    def __init__(self, sf_obj, leafspace):
        self.sf = sf_obj
        self.leafspace = int(leafspace)

    def bcast(self, root, leaf, op):
        self.sf.bcast(root, leaf, op, unit=S.unit_of(root))

    def reduce(self, leaf, root, op):
        self.sf.reduce(leaf, root, op, unit=S.unit_of(root))


def sf_bcast(dsf, root):
    return SFBcastFn.apply(dsf, root)


def sf_reduce_sum(dsf, leaf, root):
    return SFReduceSumFn.apply(dsf, leaf, root)


def layer(dsf, h, a):
    """h' = tanh(Reduce_SUM(a * Bcast(h)) onto zeros), a: per-leaf scalars."""
    e = sf_bcast(dsf, h)
    m = e * a.reshape((-1,) + (1,) * (e.dim() - 1))
    z = sf_reduce_sum(dsf, m, torch.zeros_like(h))
    return torch.tanh(z)


def chain_loss(sf_obj, h, a_list, G, checkpoint=True, leafspace=None):
    """<h_K, G> after K layers; each layer recomputed in backward when
    ``checkpoint`` (torch.utils.checkpoint)."""
    dsf = sf_obj if isinstance(sf_obj, DiffSF) else DiffSF(sf_obj, leafspace or sf_obj.nleaves)
    x = h
    for a in a_list:
        if checkpoint:
            x = torch.utils.checkpoint.checkpoint(layer, dsf, x, a, use_reentrant=False)
        else:
            x = layer(dsf, x, a)
    return (x * G).sum()
