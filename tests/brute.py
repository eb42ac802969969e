"""O(N^2) brute-force line inverse by the method of images (tests only).

Independent of the oracle's recursions and boundary formulas: the discrete
L^{-1}[v](x_j) is written as a sum over cells and over the images of each cell
of (alpha/2) * integral of exp(-alpha*|x_j - x''|) * p(x') dx', integrated with
mpmath at 30 digits.  Images: periodic x'' = x' + nL; Neumann x'' = x' + 2nL
(even reflections 2nL - x' with the same sign); Dirichlet the reflections carry
a minus sign.  The interpolant p of a cell is the one the fast method assigns:
when the kernel grows like exp(+alpha x') across the cell (the image lies to
the left of the target, unreflected, or to the right, reflected) it is the
window centred on the cell's right node (the J^L window); otherwise the window
centred on the cell's left node (the J^R window).  Non-periodic windows are
shifted to the nearest in-range M+1 nodes.
"""
from __future__ import annotations

import mpmath as mp

mp.mp.dps = 30


def _lag(nodes, i, t):
    p = mp.mpf(1)
    for k, xk in enumerate(nodes):
        if k != i:
            p *= (t - xk) / (nodes[i] - xk)
    return p


def _window(bc, n, N, M, centre):
    lo = centre - M // 2
    if bc != "periodic":
        lo = max(0, min(lo, N - M))
    return lo


def line_inverse(v, alpha, L, bc, M, images=60):
    """Brute-force discrete L^{-1} of the node values v (list of floats).

    periodic: len(v) = n unique nodes, h = L/n; neumann/dirichlet: nodes incl.
    both ends, h = L/(n-1).  Returns a list of mpf.
    """
    n = len(v)
    N = n if bc == "periodic" else n - 1
    h = mp.mpf(L) / N
    a = mp.mpf(alpha)
    Lm = mp.mpf(L)

    def val(k):
        return mp.mpf(v[k % n]) if bc == "periodic" else mp.mpf(v[k])

    # per cell c = [x_c, x_{c+1}]: integrals of exp(+a(x'-x_c)) pL and exp(-a(x'-x_c)) pR
    Ip, Im = [], []
    for c in range(N):
        loL = _window(bc, n, N, M, c + 1)
        loR = _window(bc, n, N, M, c)
        nodesL = [(loL + i) * h for i in range(M + 1)]
        nodesR = [(loR + i) * h for i in range(M + 1)]
        xc = c * h

        def pL(x):
            return sum(val(loL + i) * _lag(nodesL, i, x) for i in range(M + 1))

        def pR(x):
            return sum(val(loR + i) * _lag(nodesR, i, x) for i in range(M + 1))

        Ip.append(mp.quad(lambda x: mp.e ** (a * (x - xc)) * pL(x), [xc, xc + h]))
        Im.append(mp.quad(lambda x: mp.e ** (-a * (x - xc)) * pR(x), [xc, xc + h]))

    out = []
    for j in range(n):
        xj = j * h
        s = mp.mpf(0)
        for c in range(N):
            xc, xc1 = c * h, (c + 1) * h
            Kp = mp.mpf(0)
            Km = mp.mpf(0)
            if bc == "periodic":
                for m in range(-images, images + 1):
                    sh = m * Lm
                    if xc1 + sh <= xj:      # left image: exp(-a(xj - x' - sh))
                        Kp += mp.e ** (-a * (xj - xc - sh))
                    else:                   # right image: exp(-a(x' + sh - xj))
                        Km += mp.e ** (-a * (xc + sh - xj))
            else:
                sgn = -1 if bc == "dirichlet" else 1
                for m in range(-images, images + 1):
                    sh = 2 * m * Lm
                    if xc1 + sh <= xj:
                        Kp += mp.e ** (-a * (xj - xc - sh))
                    else:
                        Km += mp.e ** (-a * (xc + sh - xj))
                    # reflected image x'' = sh - x', cell [sh - x_{c+1}, sh - x_c]
                    if sh - xc <= xj:       # left: exp(-a(xj - sh + x'))  ~ exp(-a x')
                        Km += sgn * mp.e ** (-a * (xj - sh + xc))
                    else:                   # right: exp(-a(sh - x' - xj)) ~ exp(+a x')
                        Kp += sgn * mp.e ** (-a * (sh - xc - xj))
            s += Kp * Ip[c] + Km * Im[c]
        out.append(a / 2 * s)
    return out
