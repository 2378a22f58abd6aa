"""Softmax-gated ensemble head as a torch.autograd.Function over the library's kernels.

Experts: q_0 = softmax(z + b) (the adaptive-bias head of section 3.7 applied to the LLM logits)
and the n-gram orders P_1..P_K (section 3.5); gate w = softmax(theta); p = sum_j w_j q_j;
loss_r = -log p_r(t*_r).  Forward and backward are the hand-written kernels behind
nc_ensemble_forward / nc_ensemble_backward; the gradients are reduced over rows in a fixed order
(no float atomics).  The logits z and the n-gram experts are inputs, not parameters.
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import check, lib


def _ptr(t, dtype, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on a HIP device")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class EnsembleHead(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z, b, theta, P, target):
        rows, vocab = z.shape
        nexp = theta.shape[0]
        loss = torch.empty(rows, dtype=torch.float32, device=z.device)
        resp = torch.empty((rows, nexp), dtype=torch.float32, device=z.device)
        Pp = _ptr(P, torch.float32, "P") if nexp > 1 else None
        check(lib().nc_ensemble_forward(_ptr(z, torch.float32, "z"), _ptr(b, torch.float32, "b"),
                                        _ptr(theta, torch.float32, "theta"), Pp,
                                        _ptr(target, torch.int32, "target"), rows, vocab, nexp,
                                        _ptr(loss, torch.float32, "loss"), None,
                                        _ptr(resp, torch.float32, "resp"), _stream()))
        ctx.save_for_backward(z, b, theta, resp, target)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        z, b, theta, resp, target = ctx.saved_tensors
        rows, vocab = z.shape
        nexp = theta.shape[0]
        gl = grad_loss.contiguous().to(torch.float32)
        gb = torch.empty_like(b)
        gth = torch.empty_like(theta)
        check(lib().nc_ensemble_backward(_ptr(z, torch.float32, "z"), _ptr(b, torch.float32, "b"),
                                         _ptr(theta, torch.float32, "theta"),
                                         _ptr(resp, torch.float32, "resp"),
                                         _ptr(target, torch.int32, "target"),
                                         _ptr(gl, torch.float32, "grad_loss"), rows, vocab, nexp,
                                         C.c_float(0.0), _ptr(gb, torch.float32, "grad_b"),
                                         _ptr(gth, torch.float32, "grad_theta"), _stream()))
        return None, gb, gth, None, None


def ensemble_loss(z, b, theta, P, target):
    """Per-row -log p(t*) of the gated ensemble; differentiable in b and theta."""
    return EnsembleHead.apply(z, b, theta, P, target)


def ensemble_sgd_step(z, b, theta, P, target, lr: float = 1e-3):
    """One fused SGD step on (b, theta) for the summed loss, in place; returns the losses."""
    rows, vocab = z.shape
    nexp = theta.shape[0]
    loss = torch.empty(rows, dtype=torch.float32, device=z.device)
    resp = torch.empty((rows, nexp), dtype=torch.float32, device=z.device)
    Pp = _ptr(P, torch.float32, "P") if nexp > 1 else None
    check(lib().nc_ensemble_forward(_ptr(z, torch.float32, "z"), _ptr(b, torch.float32, "b"),
                                    _ptr(theta, torch.float32, "theta"), Pp,
                                    _ptr(target, torch.int32, "target"), rows, vocab, nexp,
                                    _ptr(loss, torch.float32, "loss"), None,
                                    _ptr(resp, torch.float32, "resp"), _stream()))
    ones = torch.ones(rows, dtype=torch.float32, device=z.device)
    check(lib().nc_ensemble_backward(_ptr(z, torch.float32, "z"), _ptr(b, torch.float32, "b"),
                                     _ptr(theta, torch.float32, "theta"),
                                     _ptr(resp, torch.float32, "resp"),
                                     _ptr(target, torch.int32, "target"),
                                     _ptr(ones, torch.float32, "grad_loss"), rows, vocab, nexp,
                                     C.c_float(lr), None, None, _stream()))
    return loss
