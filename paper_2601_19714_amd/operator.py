"""The imaging operator as a differentiable PyTorch function (prediction and its transpose).

ImagingOperator(X) is the prediction P X (wsimg_predict: image -> visibilities), and its
backward is the transpose applied to the incoming gradient, A g (wsimg_image with unit
weights and no normalisation), both computed by the HIP kernels of the library.  With
torch's convention for a real loss L of complex y (the gradient is dL/dRe y + i dL/dIm y),
dL/dX = A(dL/dy) exactly, because sum_ij A(z)_ij X_ij = Re sum_m z_m conj((P X)_m).

Both directions use one plane range, fixed when the operator is built (from the rows with
positive weight, as wsimg_image would pick it), and the same kept rows: a row is dropped in
both if its uvw or weight is not finite or its taps leave the grid.
"""

from __future__ import annotations

from typing import Optional, Tuple

import torch

from . import Plan


class ImagingOperator:
    """P: real image [n, n] -> visibilities [M] on one GPU, with P^T as its gradient."""

    def __init__(self, uvw, weights, freq_hz: float, n: int, pixel_rad: float, n_wplanes: int,
                 support: int = 7, beta: Optional[float] = None, precision: str = "f32",
                 w_range: Optional[Tuple[float, float]] = None):
        self.uvw, self.weights, self.freq_hz = uvw, weights, float(freq_hz)
        self.n = int(n)
        rdt = torch.float32 if precision in ("f32", "float32") else torch.float64
        if w_range is None:
            with Plan(n, pixel_rad, n_wplanes, support, beta, precision, max_vis=uvw.shape[0],
                      device=uvw.device) as probe:
                zero = torch.zeros((n, n), dtype=rdt, device=uvw.device)
                _, st = probe.predict(uvw, weights, freq_hz, zero, stats=True)
            w_range = (st["w_lo"], st["w_hi"])
        self.w_range = (float(w_range[0]), float(w_range[1]))
        kw = dict(support=support, beta=beta, precision=precision, max_vis=uvw.shape[0],
                  w_range=self.w_range, device=uvw.device)
        self._pred = Plan(n, pixel_rad, n_wplanes, **kw)
        self._adj = Plan(n, pixel_rad, n_wplanes, normalize=False, **kw)
        # unit weights on the rows the prediction keeps (non-finite weights stay dropped)
        self._unit = torch.where(torch.isfinite(weights), torch.ones_like(weights),
                                 torch.full_like(weights, float("nan")))

    def predict(self, image):
        """P X (no autograd)."""
        return self._pred.predict(self.uvw, self.weights, self.freq_hz, image.contiguous())

    def adjoint(self, vis):
        """A z = P^T z: the unnormalised dirty image of visibilities z with unit weights."""
        return self._adj.image(self.uvw, vis.contiguous(), self._unit, self.freq_hz)

    def __call__(self, image):
        return _Predict.apply(image, self)

    def close(self):
        self._pred.close()
        self._adj.close()


class _Predict(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image, op):
        ctx.op = op
        return op.predict(image.detach())

    @staticmethod
    def backward(ctx, grad_vis):
        return ctx.op.adjoint(grad_vis), None
