"""torch.autograd binding of one MAHI evaluation (argument marshalling only).

E(x, lambda-tilde, form charges) is the HI energy of the general formulation
(paper, eq iter_ham_lambda).  One mahi_eval returns E together with its exact
derivatives in all three inputs (forces F = -dE/dx, dE/dlambda-tilde per form
and dE/dq per form charge; paper, section "Calculation of Forces on lambda
Particles" and the mapping K of the appendix), so the forward pass keeps them
and the backward pass only scales them by the incoming gradient: no second
evaluation is needed.

The evaluator must run on torch's current stream (pass
stream=torch.cuda.current_stream().cuda_stream when creating it); forward
then orders itself with the surrounding torch work without synchronising.
"""
from __future__ import annotations

import numpy as np
import torch

from .mahi import Mahi


class MahiEnergy(torch.autograd.Function):
    """energy = MahiEnergy.apply(x, lambda_tilde, form_charges, evaluator).

    x: [N, 3] CUDA tensor of the evaluator's precision (float32 or float64);
    lambda_tilde: [sum forms] float64 tensor; form_charges: flat float64 tensor
    in the evaluator's layout (per site: form-major, atom-minor), or None to
    keep the charges given at creation.  Returns a float64 0-d CUDA tensor.
    """

    @staticmethod
    def forward(ctx, x, lambda_tilde, form_charges, evaluator: Mahi):
        dev = x.device
        want_dtype = torch.float32 if evaluator.precision == 32 else torch.float64
        if x.dtype != want_dtype or not x.is_cuda or x.shape != (evaluator.n, 3):
            raise ValueError("x must be a CUDA tensor of shape (N, 3) in the evaluator's precision")
        if form_charges is not None:
            evaluator.set_form_charges(form_charges.detach().to("cpu", torch.float64).numpy())
        if evaluator.n_forms:
            evaluator.set_lambda(lambda_tilde.detach().to("cpu", torch.float64).numpy())
        xc = x.detach().contiguous()
        E = torch.zeros((), dtype=torch.float64, device=dev)
        F = torch.empty((evaluator.n, 3), dtype=want_dtype, device=dev)
        nf, nq = evaluator.n_forms, evaluator.n_form_charges
        dvdl = torch.empty(max(nf, 1), dtype=torch.float64, device=dev)
        dedq = torch.empty(max(nq, 1), dtype=torch.float64, device=dev)
        evaluator.eval_device(xc.data_ptr(), E.data_ptr(), F.data_ptr(), dvdl.data_ptr() if nf else 0,
                              dedq_ptr=dedq.data_ptr() if nf else 0)
        ctx.save_for_backward(F, dvdl[:nf], dedq[:nq])
        ctx.has_q = form_charges is not None
        ctx.lt_device = lambda_tilde.device
        ctx.fq_device = form_charges.device if form_charges is not None else None
        return E

    @staticmethod
    def backward(ctx, gE):
        F, dvdl, dedq = ctx.saved_tensors
        gx = gl = gq = None
        if ctx.needs_input_grad[0]:
            gx = (-gE.to(F.dtype)) * F
        if ctx.needs_input_grad[1]:
            gl = (gE * dvdl).to(ctx.lt_device)
        if ctx.has_q and ctx.needs_input_grad[2]:
            gq = (gE * dedq).to(ctx.fq_device)
        return gx, gl, gq, None


def mahi_energy(x, lambda_tilde, evaluator: Mahi, form_charges=None):
    """Functional form of MahiEnergy.apply."""
    if lambda_tilde is None:
        lambda_tilde = torch.zeros(0, dtype=torch.float64)
    return MahiEnergy.apply(x, lambda_tilde, form_charges, evaluator)


def flat_form_charges(system) -> np.ndarray:
    """Form charges of a synth-style system in the evaluator's flat layout."""
    return np.concatenate([np.asarray(s.charges, dtype=np.float64).reshape(-1) for s in system.sites]) \
        if system.sites else np.zeros(0)
