"""Fourth-order exponential time differencing (ETD-RK4), oracle.

Test infrastructure only.  The method is the Cox-Matthews scheme (the
paper's reference cox2002exponential; the paper itself runs exponential
Euler and Runge-Kutta methods of order 2 and 3 on the same phi-function
actions, Section 5).  For u' = L u + F(u) with L = -A (A the positive
Kronecker-sum operator) and step h, with phi_k evaluated at h L or h L / 2:

  a  = e^{hL/2} u  + h/2 phi_1(hL/2) F(u)
  b  = e^{hL/2} u  + h/2 phi_1(hL/2) F(a)
  c  = e^{hL/2} a  + h/2 phi_1(hL/2) (2 F(b) - F(u))
  u+ = e^{hL} u + h [ f1 F(u) + 2 f2 (F(a) + F(b)) + f3 F(c) ]

where Cox and Matthews' three coefficient functions, written with the phi
functions of h L, are
  f1 = phi_1 - 3 phi_2 + 4 phi_3,  f2 = phi_2 - 2 phi_3,  f3 = -phi_2 + 4 phi_3.
(Their closed forms h^-2 L^-3 [-4 - hL + e^{hL}(4 - 3hL + (hL)^2)], etc.,
expand to exactly these combinations.)

F(u) = c1 u + c3 u^3 (the cubic reaction of the Allen-Cahn equation has
c1 = 1, c3 = -1).  The phi-function actions come from `phi` (default: the
dense augmented-matrix exponential of phi_exact, for small grids).
"""
from __future__ import annotations

import numpy as np

from .phi_exact import phi_dense_aug


def cubic(u, c1=1.0, c3=-1.0):
    return c1 * u + c3 * u * u * u


def etdrk4_step(mats, h, u, F, phi=phi_dense_aug):
    """One Cox-Matthews step of u' = -A u + F(u); returns the new u."""
    half = h / 2.0
    Fu = F(u)
    pu = phi(mats, half, u, 1)       # e^{hL/2} u (row 0)
    pFu = phi(mats, half, Fu, 1)     # phi_1(hL/2) F(u) (row 1)
    a = pu[0] + half * pFu[1]
    Fa = F(a)
    b = pu[0] + half * phi(mats, half, Fa, 1)[1]
    Fb = F(b)
    c = phi(mats, half, a, 0)[0] + half * phi(mats, half, 2.0 * Fb - Fu, 1)[1]
    Fc = F(c)
    full_u = phi(mats, h, u, 0)[0]
    g1 = phi(mats, h, Fu, 3)
    g2 = phi(mats, h, Fa + Fb, 3)
    g3 = phi(mats, h, Fc, 3)
    f1 = g1[1] - 3.0 * g1[2] + 4.0 * g1[3]
    f2 = g2[2] - 2.0 * g2[3]
    f3 = -g3[2] + 4.0 * g3[3]
    return full_u + h * (f1 + 2.0 * f2 + f3)


def etdrk4(mats, h, u0, steps, F=cubic, phi=phi_dense_aug):
    u = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(steps):
        u = etdrk4_step(mats, h, u, F, phi)
    return u
