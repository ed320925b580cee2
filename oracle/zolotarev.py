"""Zolotarev rational approximations of the sign function (oracle, test infrastructure).

Zolo-pd (Sec. 5 of the paper, following Nakatsukasa & Freund) maps every
singular value in [l, 1] to 1 with two iterations of a type (2r+1, 2r)
Zolotarev function, r <= 8 terms per iteration.  The paper only names the
function; the definition used here is the standard one:

    Z(x; l) = M * x * prod_{j=1..r} (x^2 + c_{2j}) / (x^2 + c_{2j-1})
    c_i     = l^2 * sn^2(i K'/(2r+1); l') / cn^2(i K'/(2r+1); l'),  i = 1..2r
    l'      = sqrt(1 - l^2),   K' = K(l')  (complete elliptic integral)

with partial fractions  prod_j (y + c_{2j})/(y + c_{2j-1}) = 1 + sum_j a_j/(y + c_{2j-1}),

    a_j = - prod_{k=1..r} (c_{2j-1} - c_{2k}) / prod_{k != j} (c_{2j-1} - c_{2k-1}).

Normalisation: M is fixed by Z(1; l) = 1, so that 0 <= Z <= 1 on [0, 1]
(Sec. 5.1, the modified Zolo-pd maps [eps, 1] to 1 - O(u) and stays in [0, 1]).
The next lower bound is l_{k+1} = Z(l_k; l_k).  The degree r is the smallest
r <= 8 whose two-step composition leaves 1 - l_2 <= tol (Sec. 5 says p <= 8
suffices in double precision down to eps = 1e-15).

Everything is computed with mpmath at 60 significant digits, straight from
the elliptic-function definition; results are returned as Python floats
(rounded once) plus the mpf values for the tests.
"""
from __future__ import annotations

import mpmath as mp

DPS = 60
U_DOUBLE = 2.0 ** -53


def coeffs_mp(ell, r, dps=DPS):
    """Return (c[1..2r], a[1..r], M, ell_next) as mpf for Z_{2r+1}(.; ell)."""
    if r < 1:
        raise ValueError("r must be >= 1")
    with mp.workdps(dps):
        l = mp.mpf(ell)
        if not (0 < l <= 1):
            raise ValueError("ell must lie in (0, 1]")
        m_comp = 1 - l * l                     # parameter of modulus l' (m = l'^2)
        Kp = mp.ellipk(m_comp)
        c = []
        for i in range(1, 2 * r + 1):
            u = i * Kp / (2 * r + 1)
            sn = mp.ellipfun("sn", u, m=m_comp)
            cn = mp.ellipfun("cn", u, m=m_comp)
            c.append(l * l * sn * sn / (cn * cn))
        # c is 0-based here: c[i-1] == c_i
        odd = [c[2 * j] for j in range(r)]       # c_1, c_3, ..., c_{2r-1}
        even = [c[2 * j + 1] for j in range(r)]  # c_2, c_4, ..., c_{2r}
        a = []
        for j in range(r):
            num = mp.mpf(1)
            for k in range(r):
                num *= odd[j] - even[k]
            den = mp.mpf(1)
            for k in range(r):
                if k != j:
                    den *= odd[j] - odd[k]
            a.append(-num / den)
        prod1 = mp.mpf(1)
        for j in range(r):
            prod1 *= (1 + even[j]) / (1 + odd[j])
        M = 1 / prod1
        ell_next = eval_product(l, c, M)
        return c, a, M, ell_next


def eval_product(x, c, M):
    """Z(x) in product form, M * x * prod (x^2 + c_{2j}) / (x^2 + c_{2j-1})."""
    x = mp.mpf(x)
    r = len(c) // 2
    p = M * x
    for j in range(r):
        p *= (x * x + c[2 * j + 1]) / (x * x + c[2 * j])
    return p


def eval_partial(x, c, a, M):
    """Z(x) in partial-fraction form, M * x * (1 + sum_j a_j / (x^2 + c_{2j-1}))."""
    x = mp.mpf(x)
    r = len(a)
    s = mp.mpf(1)
    for j in range(r):
        s += a[j] / (x * x + c[2 * j])
    return M * x * s


class ZoloStep:
    """One Zolotarev iteration: floats for use with numpy plus the mpf originals."""

    def __init__(self, ell, r, dps=DPS):
        c, a, M, ell_next = coeffs_mp(ell, r, dps)
        self.r = r
        self.ell = float(ell)
        self.c_mp, self.a_mp, self.M_mp, self.ell_next_mp = c, a, M, ell_next
        self.c = [float(v) for v in c]
        self.c_odd = [float(c[2 * j]) for j in range(r)]
        self.c_even = [float(c[2 * j + 1]) for j in range(r)]
        self.a = [float(v) for v in a]
        self.M = float(M)
        self.ell_next = float(ell_next)

    def __call__(self, x):
        return float(eval_product(x, self.c_mp, self.M_mp))


def two_step(ell, r, dps=DPS):
    """The two Zolo-pd iterations for lower bound ell: (step1, step2, 1 - l_2 as mpf)."""
    s1 = ZoloStep(ell, r, dps)
    with mp.workdps(dps):
        l1 = min(s1.ell_next_mp, mp.mpf(1))
    s2 = ZoloStep(l1, r, dps)
    with mp.workdps(dps):
        resid = 1 - s2.ell_next_mp
    return s1, s2, resid


def choose_r(ell, tol=U_DOUBLE, rmax=8, dps=DPS):
    """Smallest r in 1..rmax with 1 - l_2 <= tol after two iterations, or None."""
    for r in range(1, rmax + 1):
        _, _, resid = two_step(ell, r, dps)
        if resid <= tol:
            return r
    return None
