"""Named limb-darkening laws as radial profile generators.

RoadRunner takes the stellar limb darkening as a radial profile I(mu) and
can be driven by any named law or by a callable (Sect. 3.2.1, Sect. 3.2.2);
this module turns law coefficients into the profile samples that
``Tables`` (rr_prepare_ld), ``Tables.set_profile`` (rr_set_profile) and
``evaluate_ld`` (rr_evaluate_ld, one profile per parameter row) take, and
gives each law's normalisation I_star = 2 pi int_0^1 mu I(mu) dmu in closed
form.  The library itself integrates I_star exactly for the piecewise-linear
interpolant of the samples, which tends to these values as the mu sampling
is refined.

Profiles are normalised to I(1) = 1.  Coefficients have shape (..., ncoef)
and broadcast over leading dimensions; results have shape (..., nmu).  All
functions accept NumPy arrays or torch tensors (on any device) and return
torch tensors in FP64.

Laws (1 - mu written as m):
  uniform                       1
  linear (u)                    1 - u m
  quadratic (a, b)              1 - a m - b m^2
  triangular-quadratic (q1, q2) quadratic with a = 2 sqrt(q1) q2,
                                b = sqrt(q1) (1 - 2 q2)
  general (c_1 .. c_n)          1 - sum_n c_n m^n
  nonlinear (c_1 .. c_4)        1 - sum_n c_n (1 - mu^(n/2))
  logarithmic (a, b)            1 - a m - b mu ln mu
  power-2 (c, alpha)            1 - c (1 - mu^alpha)
  power-2-pm (h1, h2)           power-2 with c = 1 - h1 + h2,
                                alpha = log2(c / h2)
The exponential law diverges at the limb (mu = 0) and cannot be sampled
there; use a callable with ``from_callable`` if it is needed.
"""

import math

import numpy as np
import torch

NCOEF = {"uniform": 0, "linear": 1, "quadratic": 2, "triangular-quadratic": 2,
         "nonlinear": 4, "logarithmic": 2, "power-2": 2, "power-2-pm": 2}


def _t(x):
    if isinstance(x, torch.Tensor):
        return x.to(torch.float64)
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


def _split(coeffs, n, law):
    c = _t(coeffs)
    if n == 0:
        return c, []
    if c.shape[-1] != n:
        raise ValueError(f"{law} takes {n} coefficients per profile")
    return c, [c[..., i:i + 1] for i in range(n)]


def _to_standard(law, coeffs):
    """Reparametrised laws -> their standard form."""
    if law == "triangular-quadratic":
        _, (q1, q2) = _split(coeffs, 2, law)
        s = torch.sqrt(q1)
        return "quadratic", torch.cat([2.0 * s * q2, s * (1.0 - 2.0 * q2)], -1)
    if law == "power-2-pm":
        _, (h1, h2) = _split(coeffs, 2, law)
        c = 1.0 - h1 + h2
        return "power-2", torch.cat([c, torch.log2(c / h2)], -1)
    return law, coeffs


def profile(law, mu, coeffs=()):
    """Profile samples I(mu) of a named law, shape (..., nmu)."""
    law, coeffs = _to_standard(law, coeffs)
    mu = _t(mu)
    if law == "general":
        c = _t(coeffs)
        m = 1.0 - mu
        out = torch.ones(c.shape[:-1] + mu.shape, dtype=torch.float64, device=c.device)
        for n in range(1, c.shape[-1] + 1):
            out = out - c[..., n - 1:n] * m.to(c.device) ** n
        return out
    if law not in NCOEF:
        raise ValueError(f"unknown law {law!r}")
    c, p = _split(coeffs, NCOEF[law], law)
    mu = mu.to(c.device)
    m = 1.0 - mu
    if law == "uniform":
        return torch.ones(c.shape[:-1] + mu.shape if c.dim() else mu.shape,
                          dtype=torch.float64, device=c.device)
    if law == "linear":
        return 1.0 - p[0] * m
    if law == "quadratic":
        return 1.0 - p[0] * m - p[1] * m * m
    if law == "nonlinear":
        out = torch.ones_like(p[0] * mu)
        for n in range(1, 5):
            out = out - p[n - 1] * (1.0 - mu ** (0.5 * n))
        return out
    if law == "logarithmic":
        mlm = torch.where(mu > 0, mu * torch.log(torch.where(mu > 0, mu, torch.ones_like(mu))),
                          torch.zeros_like(mu))
        return 1.0 - p[0] * m - p[1] * mlm
    if law == "power-2":
        return 1.0 - p[0] * (1.0 - mu ** p[1])
    raise ValueError(f"unknown law {law!r}")


def istar(law, coeffs=()):
    """Closed-form I_star = 2 pi int_0^1 mu I(mu) dmu, shape (...)."""
    law, coeffs = _to_standard(law, coeffs)
    pi = math.pi
    if law == "general":
        c = _t(coeffs)
        n = torch.arange(1, c.shape[-1] + 1, dtype=torch.float64, device=c.device)
        return pi * (1.0 - (c * 2.0 / ((n + 1.0) * (n + 2.0))).sum(-1))
    if law not in NCOEF:
        raise ValueError(f"unknown law {law!r}")
    c, p = _split(coeffs, NCOEF[law], law)
    if law == "uniform":
        return torch.full(c.shape[:-1] if c.dim() else (), pi, dtype=torch.float64)
    if law == "linear":
        return pi * (1.0 - p[0][..., 0] / 3.0)
    if law == "quadratic":
        return pi * (1.0 - p[0][..., 0] / 3.0 - p[1][..., 0] / 6.0)
    if law == "nonlinear":
        n = torch.arange(1, 5, dtype=torch.float64, device=c.device)
        return pi * (1.0 - (c * n / (n + 4.0)).sum(-1))
    if law == "logarithmic":
        return pi * (1.0 - p[0][..., 0] / 3.0 + 2.0 * p[1][..., 0] / 9.0)
    if law == "power-2":
        a = p[1][..., 0]
        return pi * (1.0 - p[0][..., 0] * a / (a + 2.0))
    raise ValueError(f"unknown law {law!r}")


def from_callable(fn, mu, params):
    """Profile samples from a callable fn(mu, params) -> I(mu), for laws not
    listed here; I_star then comes from the library's integral of the
    sampled profile."""
    return _t(fn(_t(mu), params))
