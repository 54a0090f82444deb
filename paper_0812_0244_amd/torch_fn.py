"""E_c^nl (or the whole E_xc of Eq. (Exc)) as a differentiable torch
function whose backward is v_nl (v_xc).

Eq. (Vi) defines v_i = (1/dOmega) dE/dn_i, so the gradient of E with
respect to the grid values n_i is dOmega * v_i.  The forward pass runs the
HIP library (which produces E and v together); the backward pass launches
nothing.  PyTorch provides device memory and the stream only.
"""
from __future__ import annotations

import numpy as np
import torch

from .binding import FUNCTIONAL_VDW_DF, VdwNl


class NonlocalCorrelation:
    """A planned grid plus kernel table on one device.

    ``table`` is a mapping with ``qmesh``, ``qc``, ``mc``, ``dk``, ``phi``
    ([nq, nq, nk], radial kernel table) and ``c_soft``.  ``grad_mode`` 0:
    spectral gradient; m = 1..4: central differences with m points a side.
    """

    def __init__(self, shape, cell, table, precision: int = 32, device: int = 0, grad_mode: int = 0):
        self.shape = tuple(int(s) for s in shape)
        c = np.asarray(cell, dtype=np.float64)
        self.cell = tuple(float(x) for x in c) if c.shape == (3,) else c.reshape(3, 3).copy()
        self.precision = precision
        self.device = device
        self.dtype = torch.float64 if precision == 64 else torch.float32
        vol = float(np.prod(c)) if c.shape == (3,) else abs(float(np.linalg.det(c.reshape(3, 3))))
        self.dvol = vol / float(np.prod(self.shape))
        self.lib = VdwNl(device)
        self.grad_mode = grad_mode
        self.lib.set_grid(self.shape, self.cell, grad_mode, precision)
        self.lib.set_kernel_table(table["qmesh"], table["qc"], int(table.get("mc", 12)), table["dk"],
                                  table["phi"], table["c_soft"])

    def energy_potential(self, n: torch.Tensor, v: torch.Tensor | None = None):
        """(E_k, Delta E, v) for a device tensor n of the planned shape and precision."""
        if n.dtype != self.dtype or tuple(n.shape) != self.shape or not n.is_cuda:
            raise ValueError("n must be a %s CUDA tensor of shape %s" % (self.dtype, self.shape))
        n = n.contiguous()
        if v is None:
            v = torch.empty_like(n)
        stream = torch.cuda.current_stream(n.device).cuda_stream
        ek, de = self.lib.energy_potential(n.data_ptr(), v.data_ptr(), stream)
        return ek, de, v

    def total(self, n: torch.Tensor):
        """(E, v): the energy this engine's functional defines and its potential."""
        ek, de, v = self.energy_potential(n)
        return ek + de, v

    def __call__(self, n: torch.Tensor) -> torch.Tensor:
        return VdwNlEnergy.apply(n, self)


class VdwDF(NonlocalCorrelation):
    """The whole functional of Eq. (Exc), E_xc = E_x^GGA + E_c^LDA + E_c^nl
    (revPBE exchange, Perdew-Wang 1992 LDA correlation), with v_xc; the
    arguments are those of NonlocalCorrelation."""

    def __init__(self, shape, cell, table, precision: int = 32, device: int = 0, grad_mode: int = 0):
        super().__init__(shape, cell, table, precision, device, grad_mode)
        self.lib.set_functional(FUNCTIONAL_VDW_DF)

    def energy_potential(self, n: torch.Tensor, v: torch.Tensor | None = None):
        """(E_k, Delta E, E_x, E_c^LDA, v_xc) for a device tensor n."""
        ek, de, v = super().energy_potential(n, v)
        ex, ec = self.lib.semilocal_energies()[0]
        return ek, de, float(ex), float(ec), v

    def total(self, n: torch.Tensor):
        ek, de, ex, ec, v = self.energy_potential(n)
        return ek + de + ex + ec, v


class VdwNlEnergy(torch.autograd.Function):
    """forward(n) = E (FP64 scalar: E_c^nl, or E_xc for a VdwDF engine);
    backward(gE) = gE * dOmega * v."""

    @staticmethod
    def forward(ctx, n, engine: NonlocalCorrelation):
        e, v = engine.total(n.detach())
        ctx.save_for_backward(v)
        ctx.dvol = engine.dvol
        return torch.tensor(e, dtype=torch.float64, device=n.device)

    @staticmethod
    def backward(ctx, gE):
        (v,) = ctx.saved_tensors
        return (gE.to(v.dtype) * ctx.dvol) * v, None
