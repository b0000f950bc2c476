"""Differentiable wrappers: dL/d(values of A) through the fixed-pattern LS solves.

RSAIFunction.apply(val, A, params) -> (valM, frob):
  valM = values of M = RSAI(tol)(A) (pattern fixed by the forward pass),
  frob = sum_k ||A m_k - e_k||^2.
Its backward calls rsai_backward (the adjoint kernel): the pattern of M is held
fixed, each m_k is the solution of (2.3) on its pattern. The forward build keeps the
R factors of its final solves (keep_factors) so that the adjoint reuses them; the
columns that do not fit the factor budget are refactorised.

RSAIBatchFunction.apply(params, mats, *vals) does the same for several matrices in
one batched build (rsai_build_batched) and one adjoint call per matrix.

SpMV.apply(val, x, A) -> A x, differentiable in the values and in x.
rsai_loss(A, val, b) = sum_k ||A m_k - e_k||^2 + ||A M b - b||^2;
rsai_loss_batched(mats, vals, bs) = the sum of these over the matrices.
"""
from __future__ import annotations

import torch

from . import rsai


class SpMV(torch.autograd.Function):
    @staticmethod
    def forward(ctx, val, x, A):
        ctx.A = A
        ctx.save_for_backward(val, x)
        return rsai.spmv(A, x, val=val.detach())

    @staticmethod
    def backward(ctx, dy):
        val, x = ctx.saved_tensors
        A = ctx.A
        dy = dy.contiguous()
        dval = dx = None
        if ctx.needs_input_grad[0]:
            dval = torch.zeros_like(val)
            rsai.spmv_vjp(A, dy, x.detach(), dval, val=val.detach())
        if ctx.needs_input_grad[1]:
            dx = rsai.spmv(A, dy, transpose=True, val=val.detach())
        return dval, dx, None


class RSAIFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, val, A, params):
        Av = rsai.Matrix(A.colptr, A.rowidx, val.detach())
        Av._max_col_len = A._max_col_len
        # keep the R factors of the final solves for the adjoint unless told not to
        plan = rsai.build(Av, **dict({"keep_factors": True}, **params))
        cp, ri, vm = plan.export()
        rn = plan.stats(fields=("resnorm",))["resnorm"]
        frob = torch.sum(rn * rn)
        ctx.plan = plan
        ctx.Av = Av
        ctx.nnzA = val.numel()
        ctx.mark_non_differentiable(cp, ri)
        return vm, frob, cp, ri

    @staticmethod
    def backward(ctx, g_vm, g_frob, g_cp, g_ri):
        dA = torch.zeros(ctx.nnzA, dtype=torch.float64, device=g_vm.device if g_vm is not None else "cuda")
        w = float(g_frob.item()) if g_frob is not None else 0.0
        ctx.plan.backward(g_vm.contiguous() if g_vm is not None else None, w, dA)
        return dA, None, None


class RSAIBatchFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, mats, *vals):
        Avs = []
        for A, val in zip(mats, vals):
            Av = rsai.Matrix(A.colptr, A.rowidx, val.detach())
            Av._max_col_len = A._max_col_len
            Avs.append(Av)
        plan = rsai.build_batched(Avs, **dict({"keep_factors": True}, **params))
        outs, pattern = [], []
        for i in range(len(Avs)):
            cp, ri, vm = plan.export(i)
            rn = plan.stats(i, fields=("resnorm",))["resnorm"]
            pattern += [cp, ri]
            outs += [vm, torch.sum(rn * rn), cp, ri]
        ctx.mark_non_differentiable(*pattern)
        ctx.plan = plan
        ctx.Avs = Avs
        ctx.nnz = [v.numel() for v in vals]
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        dAs = []
        for i, nz in enumerate(ctx.nnz):
            g_vm, g_frob = grads[4 * i], grads[4 * i + 1]
            dA = torch.zeros(nz, dtype=torch.float64, device=ctx.Avs[i].colptr.device)
            w = float(g_frob.item()) if g_frob is not None else 0.0
            ctx.plan.backward(g_vm.contiguous() if g_vm is not None else None, w, dA, mat=i)
            dAs.append(dA)
        return (None, None, *dAs)


def rsai_loss_batched(mats, vals, bs, **params) -> torch.Tensor:
    """Sum over the matrices of sum_k ||A m_k - e_k||^2 + ||A M b - b||^2, with all
    the M built in one batched build."""
    outs = RSAIBatchFunction.apply(params, list(mats), *vals)
    total = None
    for i, (A, val, b) in enumerate(zip(mats, vals, bs)):
        vm, frob, cp, ri = outs[4 * i:4 * i + 4]
        Mst = rsai.Matrix(cp, ri, vm.detach())
        u = SpMV.apply(vm, b, Mst)
        s = SpMV.apply(val, u, A) - b
        li = frob + torch.dot(s, s)
        total = li if total is None else total + li
    return total


def rsai_loss(A: "rsai.Matrix", val: torch.Tensor, b: torch.Tensor, **params) -> torch.Tensor:
    """L = sum_k ||A m_k - e_k||^2 + ||A M b - b||^2 with M = RSAI(tol)(A(val))."""
    vm, frob, cp, ri = RSAIFunction.apply(val, A, params)
    Mst = rsai.Matrix(cp, ri, vm.detach())
    u = SpMV.apply(vm, b, Mst)
    s = SpMV.apply(val, u, A) - b
    return frob + torch.dot(s, s)
