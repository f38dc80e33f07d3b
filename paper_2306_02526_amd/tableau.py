"""ARK4(3)6L[2]SA additive Runge-Kutta tableau (Kennedy & Carpenter, 2003).

The paper integrates with this pair (Sec. 3.1, Table 1 structure: ESDIRK with an
explicit first stage, a_ii = gamma = 1/4, last row equal to b; ERK sharing c).
Values are exact rationals of that publication, evaluated in double precision.
"""
from fractions import Fraction as F

import numpy as np


def _rows():
    s = 6
    A = np.zeros((s, s), dtype=object)
    Ah = np.zeros((s, s), dtype=object)
    A[:] = F(0)
    Ah[:] = F(0)
    b = [F(82889, 524892), F(0), F(15625, 83664), F(69875, 102672), F(-2260, 8211), F(1, 4)]
    A[1, 0] = F(1, 4)
    A[2, :2] = [F(8611, 62500), F(-1743, 31250)]
    A[3, :3] = [F(5012029, 34652500), F(-654441, 2922500), F(174375, 388108)]
    A[4, :4] = [F(15267082809, 155376265600), F(-71443401, 120774400),
                F(730878875, 902184768), F(2285395, 8070912)]
    A[5, :5] = b[:5]
    for i in range(1, s):
        A[i, i] = F(1, 4)
    Ah[1, 0] = F(1, 2)
    Ah[2, :2] = [F(13861, 62500), F(6889, 62500)]
    Ah[3, :3] = [F(-116923316275, 2393684061468), F(-2731218467317, 15368042101831),
                 F(9408046702089, 11113171139209)]
    Ah[4, :4] = [F(-451086348788, 2902428689909), F(-2682348792572, 7519795681897),
                 F(12662868775082, 11960479115383), F(3355817975965, 11060851509271)]
    Ah[5, :5] = [F(647845179188, 3216320057751), F(73281519250, 8382639484533),
                 F(552539513391, 3454668386233), F(3354512671639, 8306763924573), F(4040, 17871)]
    c = [F(0), F(1, 2), F(83, 250), F(31, 50), F(17, 20), F(1)]
    return s, A, b, Ah, list(b), c


def ark436l2sa():
    s, A, b, Ah, bh, c = _rows()
    f = np.vectorize(float)
    return {"s": s, "gamma": 0.25, "A": f(A).astype(np.float64), "b": np.array([float(v) for v in b]),
            "c": np.array([float(v) for v in c]), "Ahat": f(Ah).astype(np.float64),
            "bhat": np.array([float(v) for v in bh])}
