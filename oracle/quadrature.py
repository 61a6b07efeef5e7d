"""Quadrature for the square-root integral (float64 results from mpmath at
high precision).  Test infrastructure only.

The integral (Sec. 1, eq. sqrt_rational)
    lambda^(1/2) = (2/pi) int_0^inf lambda / (lambda + z^2) dz
is discretised with the conformal-map rule of Hale, Higham and Trefethen
(SIAM J. Numer. Anal. 46, 2008, their third method for A^(1/2)), derived
here for spectra inside [m, M]:

  with k'^2 = 1 - m/M and K' = K(k'^2) (complete elliptic integral of the
  first kind, parameter convention), substitute z = sqrt(m) sc(v | k'^2)
  for v in (0, K').  The integrand is analytic for |Im v| < K(m/M), and the
  midpoint rule with N nodes v_j = (j - 1/2) K'/N gives
      shifts   s_j = z_j^2 = m sc(v_j)^2
      weights  w_j = (2/pi) (K'/N) sqrt(m) dn(v_j) / cn(v_j)^2
  so that f(A) b ~ sum_j w_j A (A + s_j I)^-1 b.  The error decays like
  exp(-2 pi^2 N / log(16 M/m)).

Also the two elliptic-integral facts used in the proof of Thm. lansq:
eq. ellipticK_eval and Lemma elliptic_k_bd.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np


def sqrt_rule(m: float, M: float, N: int, dps: int = 40):
    """Shifts s_j and weights w_j (float64 arrays of length N) of the rule
    above for the interval [m, M], 0 < m <= M."""
    if not (m > 0 and M >= m):
        raise ValueError("need 0 < m <= M")
    with mp.workdps(dps):
        m_ = mp.mpf(m)
        M_ = mp.mpf(M)
        if M_ == m_:
            M_ = m_ * (1 + mp.mpf(10) ** (-dps // 2))
        kp2 = 1 - m_ / M_                      # parameter k'^2
        Kp = mp.ellipk(kp2)
        s = np.empty(N)
        w = np.empty(N)
        for j in range(N):
            v = (j + mp.mpf(1) / 2) * Kp / N
            sn = mp.ellipfun("sn", v, m=kp2)
            cn = mp.ellipfun("cn", v, m=kp2)
            dn = mp.ellipfun("dn", v, m=kp2)
            z = mp.sqrt(m_) * sn / cn
            s[j] = float(z * z)
            w[j] = float(2 / mp.pi * Kp / N * mp.sqrt(m_) * dn / (cn * cn))
    return s, w


def apply_rule_scalar(lam, shifts, weights):
    """sum_j w_j lam / (lam + s_j): the rule's approximation to sqrt(lam)."""
    lam = np.asarray(lam, dtype=np.float64)
    return sum(w * lam / (lam + s) for s, w in zip(shifts, weights))


def elliptic_integral_eval(l1: float, ld: float):
    """Right-hand side of eq. ellipticK_eval: K(1 - l1/ld) / sqrt(ld),
    the value of int_0^inf ((l1 + z^2)(ld + z^2))^-1/2 dz."""
    with mp.workdps(30):
        return float(mp.ellipk(1 - mp.mpf(l1) / mp.mpf(ld)) / mp.sqrt(ld))


def elliptic_integral_numeric(l1: float, ld: float):
    """The left-hand side of eq. ellipticK_eval by adaptive quadrature."""
    with mp.workdps(30):
        f = lambda z: 1 / mp.sqrt((l1 + z * z) * (ld + z * z))
        return float(mp.quad(f, [0, mp.sqrt(ld), mp.sqrt(l1), mp.inf]))


def lemma_elliptic_sides(x: float):
    """The three members of Lemma elliptic_k_bd's chain for x > 1:
    (2/pi) sqrt(x) K(1 - x),  (5/(4 pi)) log(16 x),  (1/2) log(16 x)."""
    with mp.workdps(30):
        x_ = mp.mpf(x)
        a = 2 / mp.pi * mp.sqrt(x_) * mp.ellipk(1 - x_)
        b = 5 / (4 * mp.pi) * mp.log(16 * x_)
        c = mp.log(16 * x_) / 2
        return float(a), float(b), float(c)
