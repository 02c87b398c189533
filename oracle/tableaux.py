"""Two-derivative Butcher tableaux of the limiting Hermite-Birkhoff RK methods
(appendix, Eqs. butcher4, butcher6, butcher8), as exact fractions.

Each has nodes c (s of them), and matrices B1, B2 (s x s) so that the
quadrature I_l = dt sum_j B1[l][j] R1(w_j) + dt^2 sum_j B2[l][j] R2(w_j)
integrates over [t_n, t_n + c_l dt] (Sec. 2.1).
"""
from fractions import Fraction as Fr


class Tableau:
    def __init__(self, q, c, B1, B2):
        self.q = q
        self.s = len(c)
        self.c = [Fr(x) for x in c]
        self.B1 = [[Fr(x) for x in row] for row in B1]
        self.B2 = [[Fr(x) for x in row] for row in B2]


def tableau(q):
    if q == 4:
        return Tableau(4, [0, 1],
                       [[0, 0], [Fr(1, 2), Fr(1, 2)]],
                       [[0, 0], [Fr(1, 12), Fr(-1, 12)]])
    if q == 6:
        return Tableau(6, [0, Fr(1, 2), 1],
                       [[0, 0, 0],
                        [Fr(101, 480), Fr(8, 30), Fr(55, 2400)],
                        [Fr(7, 30), Fr(16, 30), Fr(7, 30)]],
                       [[0, 0, 0],
                        [Fr(65, 4800), Fr(-25, 600), Fr(-25, 8000)],
                        [Fr(5, 300), 0, Fr(-5, 300)]])
    if q == 8:
        return Tableau(8, [0, Fr(1, 3), Fr(2, 3), 1],
                       [[0, 0, 0, 0],
                        [Fr(6893, 54432), Fr(313, 2016), Fr(89, 2016), Fr(397, 54432)],
                        [Fr(223, 1701), Fr(20, 63), Fr(13, 63), Fr(20, 1701)],
                        [Fr(31, 224), Fr(81, 224), Fr(81, 224), Fr(31, 224)]],
                       [[0, 0, 0, 0],
                        [Fr(1283, 272160), Fr(-851, 30240), Fr(-269, 30240), Fr(-163, 272160)],
                        [Fr(43, 8505), Fr(-16, 945), Fr(-19, 945), Fr(-8, 8505)],
                        [Fr(19, 3360), Fr(-9, 1120), Fr(9, 1120), Fr(-19, 3360)]])
    raise ValueError("q must be 4, 6 or 8")
