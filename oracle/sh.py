"""Real spherical harmonics for the FP64 oracle (test infrastructure only).

Colour model, SH form: the colour seen from view direction v is
sum_{l<=L} sum_{m=-l..l} c_lm Y_lm(v) (paper, Preliminaries, eq. 4).  The paper
does not print the basis; this oracle takes the real basis with the
Condon-Shortley phase (the basis of the 3D-GS family that SG-Splatting plugs
into):

    Y_l^m  = sqrt(2) K_l^m  Re[(x+iy)^m] (-1)^m P_l^(m)(z)     m > 0
    Y_l^-m = sqrt(2) K_l^m  Im[(x+iy)^m] (-1)^m P_l^(m)(z)     m > 0
    Y_l^0  = K_l^0 P_l(z)
    K_l^m  = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)

where P_l^(m) is the m-th derivative of the Legendre polynomial P_l and
(x, y, z) is the unit direction; sin(theta)^m e^{i m phi} = (x+iy)^m removes
the angles.  Coefficients are ordered l-major, then m = -l..l.

Everything is built from these definitions at import time (numpy's Legendre
series for P_l); no constant table is typed in.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


def _legendre_derivative_power_series(l: int, m: int) -> np.ndarray:
    """Power-series coefficients (ascending) of d^m/dz^m P_l(z)."""
    c = np.zeros(l + 1)
    c[l] = 1.0
    power = npleg.leg2poly(c)
    for _ in range(m):
        power = nppoly.polyder(power)
    return np.atleast_1d(power)


def _terms(max_degree: int):
    """[(l, m, norm, zpoly)] with norm including sqrt(2) and (-1)^|m|."""
    out = []
    for l in range(max_degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            k = math.sqrt((2 * l + 1) / (4.0 * math.pi)
                          * math.factorial(l - am) / math.factorial(l + am))
            norm = k if m == 0 else math.sqrt(2.0) * k * (-1.0) ** am
            out.append((l, m, norm, _legendre_derivative_power_series(l, am)))
    return out


_TERMS = _terms(3)


def n_coeffs(degree: int) -> int:
    return (degree + 1) ** 2


def sh_basis(degree: int, d: np.ndarray) -> np.ndarray:
    """Y_lm at unit directions d (3, N) -> (n_coeffs, N), float64."""
    x, y, z = (np.asarray(c, np.float64) for c in d)
    out = []
    for (l, m, norm, zp) in _TERMS[: n_coeffs(degree)]:
        w = (x + 1j * y) ** abs(m)
        ang = w.real if m >= 0 else w.imag
        out.append(norm * ang * nppoly.polyval(z, zp))
    return np.array(out)


def sh_basis_grad(degree: int, d: np.ndarray) -> np.ndarray:
    """d Y_lm / d(x, y, z), treating x, y, z as independent -> (n_coeffs, 3, N).

    Only the component tangent to the sphere is meaningful; callers project
    with (I - d d^T).
    """
    x, y, z = (np.asarray(c, np.float64) for c in d)
    out = []
    for (l, m, norm, zp) in _TERMS[: n_coeffs(degree)]:
        am = abs(m)
        w = (x + 1j * y) ** am
        dw = am * (x + 1j * y) ** (am - 1) if am > 0 else np.zeros_like(w)
        q = nppoly.polyval(z, zp)
        dq = nppoly.polyval(z, nppoly.polyder(zp)) if len(zp) > 1 else np.zeros_like(z)
        if m >= 0:
            ang, dax, day = w.real, dw.real, -dw.imag
        else:
            ang, dax, day = w.imag, dw.imag, dw.real
        out.append(np.stack([norm * dax * q, norm * day * q, norm * ang * dq]))
    return np.array(out)
