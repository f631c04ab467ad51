"""Writes tridiag3.txt: closed-form rows of the adaptive FSAI factor of A = tridiag(1, 4, 1)
(n = 3) for k_max = 1 and 2, s = 1, eps = 0, derived by hand from eqs. DensSys and diagScal
(Sec. 2 of the paper); only the math module is used.

Derivation.  Row 0 has no lower candidates: G_00 = 4^{-1/2}.  Rows 1 and 2 take their one
lower neighbour at step 1; A[P,P] = [[4,1],[1,4]] = L L^T with L = [[2,0],[1/2, sqrt(15)/2]],
so g = L^{-T} e_2 = (-1/(2 sqrt15), 2/sqrt15).  At step 2 row 2 has the candidate 0 with
gradient v_0 = a_01 g_1 = -1/(2 sqrt15) != 0 (row 1 reaches it), the pattern becomes {0,1,2}
and row 2 equals the last row of chol(A)^{-1}: L22 = sqrt(56/15), x2 = 1/L22,
x1 = -(L21 x2)/L11, x0 = -(L10 x1)/L00 with L10 = 1/2, L11 = sqrt15/2, L21 = 2/sqrt15."""
import math
import os

r15 = math.sqrt(15.0)
L00, L10, L11, L21, L22 = 2.0, 0.5, r15 / 2, 2.0 / r15, math.sqrt(56.0 / 15.0)
x2 = 1 / L22
x1 = -(L21 * x2) / L11
x0 = -(L10 * x1) / L00
rows = [
    (1, 0, 0, 0.5), (1, 1, 0, -1 / (2 * r15)), (1, 1, 1, 2 / r15), (1, 2, 0, 0.0),
    (1, 2, 1, -1 / (2 * r15)), (1, 2, 2, 2 / r15),
    (2, 0, 0, 0.5), (2, 1, 0, -1 / (2 * r15)), (2, 1, 1, 2 / r15),
    (2, 2, 0, x0), (2, 2, 1, x1), (2, 2, 2, x2),
]
out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tridiag3.txt")
with open(out, "w") as f:
    f.write("# Adaptive FSAI factor G of A = tridiag(1,4,1), n = 3, s = 1, eps = 0 (Sec. 2,\n")
    f.write("# eqs. DensSys, diagScal, grapsi); closed forms derived in make_tridiag3.py.\n")
    f.write("# columns: kmax row col G[row,col]\n")
    for k, i, j, v in rows:
        f.write(f"{k} {i} {j} {v!r}\n")
