"""torch.autograd binding of one MAHI evaluation (argument marshalling only).

E(x, lambda-tilde, form charges) is the HI energy of the general formulation
(paper, eq iter_ham_lambda).  Its derivatives in all three inputs are what a
full evaluation returns: the forces F = -dE/dx, dE/dlambda-tilde per form and
dE/dq per form charge (paper, section "Calculation of Forces on lambda
Particles" and the mapping K of the appendix).

Two modes:

* recompute (default): the forward pass evaluates the energy only (without
  forces the library forms the potential alone: no field in the near field and
  no gradient of the local expansions) and keeps nothing but its inputs; the
  backward pass evaluates again with every derivative requested.  Nothing of
  the expansions or the N x 3 forces lives between the two passes.
* store: the forward pass requests every derivative at once and keeps them
  (F is 12 MB at a million atoms); the backward pass only scales them.  One
  evaluation instead of two when a gradient is always taken.

Both passes order the evaluation with torch's current stream through events
(no host synchronisation): the evaluator's stream waits for the work that
produced the inputs, and torch's stream waits for the outputs.  Both passes set the evaluator's weights (and form charges, when given) to the
forward pass's values, so other evaluations with the same evaluator may run in
between.
"""
from __future__ import annotations

import numpy as np
import torch

from .mahi import Mahi


def _ordered_eval(evaluator: Mahi, dev, *args, **kw):
    """eval_device on the evaluator's stream, ordered after the work on torch's
    current stream and before everything issued there afterwards."""
    cur = torch.cuda.current_stream(dev)
    handle = evaluator.stream_handle()
    if handle == cur.cuda_stream:
        evaluator.eval_device(*args, **kw)
        return
    lib = torch.cuda.ExternalStream(handle, device=dev)
    lib.wait_stream(cur)
    evaluator.eval_device(*args, **kw)
    cur.wait_stream(lib)


def _full_eval(evaluator: Mahi, x, want_dtype):
    dev = x.device
    E = torch.zeros((), dtype=torch.float64, device=dev)
    F = torch.empty((evaluator.n, 3), dtype=want_dtype, device=dev)
    nf, nq = evaluator.n_forms, evaluator.n_form_charges
    dvdl = torch.empty(max(nf, 1), dtype=torch.float64, device=dev)
    dedq = torch.empty(max(nq, 1), dtype=torch.float64, device=dev)
    _ordered_eval(evaluator, dev, x.data_ptr(), E.data_ptr(), F.data_ptr(), dvdl.data_ptr() if nf else 0,
                  dedq_ptr=dedq.data_ptr() if nf else 0)
    return E, F, dvdl[:nf], dedq[:nq]


def _set_state(evaluator: Mahi, lambda_tilde, form_charges):
    if form_charges is not None:
        evaluator.set_form_charges(form_charges.detach().to("cpu", torch.float64).numpy())
    if evaluator.n_forms:
        evaluator.set_lambda(lambda_tilde.detach().to("cpu", torch.float64).numpy())


class MahiEnergy(torch.autograd.Function):
    """energy = MahiEnergy.apply(x, lambda_tilde, form_charges, evaluator, store).

    x: [N, 3] CUDA tensor of the evaluator's precision (float32 or float64);
    lambda_tilde: [sum forms] float64 tensor; form_charges: flat float64 tensor
    in the evaluator's layout (per site: form-major, atom-minor), or None to
    keep the charges given at creation; store: keep the derivatives from the
    forward pass (True) or recompute them in the backward pass (False).
    Returns a float64 0-d CUDA tensor.
    """

    @staticmethod
    def forward(ctx, x, lambda_tilde, form_charges, evaluator: Mahi, store: bool = False):
        want_dtype = torch.float32 if evaluator.precision == 32 else torch.float64
        if x.dtype != want_dtype or not x.is_cuda or x.shape != (evaluator.n, 3):
            raise ValueError("x must be a CUDA tensor of shape (N, 3) in the evaluator's precision")
        _set_state(evaluator, lambda_tilde, form_charges)
        xc = x.detach().contiguous()
        ctx.store = bool(store)
        ctx.evaluator = evaluator
        ctx.want_dtype = want_dtype
        ctx.has_q = form_charges is not None
        ctx.lt_device = lambda_tilde.device
        ctx.fq_device = form_charges.device if form_charges is not None else None
        if ctx.store:
            E, F, dvdl, dedq = _full_eval(evaluator, xc, want_dtype)
            ctx.save_for_backward(F, dvdl, dedq)
            return E
        E = torch.zeros((), dtype=torch.float64, device=x.device)
        _ordered_eval(evaluator, x.device, xc.data_ptr(), E.data_ptr())  # energy only: no forces or derivatives
        lt = lambda_tilde.detach().clone()
        fq = form_charges.detach().clone() if form_charges is not None else torch.zeros(0, dtype=torch.float64)
        ctx.save_for_backward(xc, lt, fq)
        return E

    @staticmethod
    def backward(ctx, gE):
        if ctx.store:
            F, dvdl, dedq = ctx.saved_tensors
        else:
            xc, lt, fq = ctx.saved_tensors
            _set_state(ctx.evaluator, lt, fq if ctx.has_q else None)
            _, F, dvdl, dedq = _full_eval(ctx.evaluator, xc, ctx.want_dtype)
        gx = gl = gq = None
        if ctx.needs_input_grad[0]:
            gx = (-gE.to(F.dtype)) * F
        if ctx.needs_input_grad[1]:
            gl = (gE * dvdl).to(ctx.lt_device)
        if ctx.has_q and ctx.needs_input_grad[2]:
            gq = (gE * dedq).to(ctx.fq_device)
        return gx, gl, gq, None, None


def mahi_energy(x, lambda_tilde, evaluator: Mahi, form_charges=None, store: bool = False):
    """Functional form of MahiEnergy.apply."""
    if lambda_tilde is None:
        lambda_tilde = torch.zeros(0, dtype=torch.float64)
    return MahiEnergy.apply(x, lambda_tilde, form_charges, evaluator, store)


def flat_form_charges(system) -> np.ndarray:
    """Form charges of a synth-style system in the evaluator's flat layout."""
    return np.concatenate([np.asarray(s.charges, dtype=np.float64).reshape(-1) for s in system.sites]) \
        if system.sites else np.zeros(0)
