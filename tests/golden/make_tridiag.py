"""Write tridiag_n8.txt: the closed-form Cholesky factor of tridiag(-1, 2, -1), n = 8.

With 1-based i the pivots of the 1-D Laplacian are (i+1)/i, so
L_ii = sqrt((i+1)/i) and L_{i+1,i} = -sqrt(i/(i+1)).  Evaluated here with
40-digit decimal arithmetic straight from these formulas (no factorization
code is run), then rounded to the nearest double by float().
"""
import decimal
import os

decimal.getcontext().prec = 40
n = 8
out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tridiag_n8.txt")
with open(out, "w") as f:
    f.write("# closed-form Cholesky factor of tridiag(-1,2,-1), n=8; 0-based band column index\n")
    f.write("# kind  column  value  (diag: L(j,j) = sqrt((j+2)/(j+1)); sub: L(j+1,j) = -sqrt((j+1)/(j+2)))\n")
    for j in range(n):
        v = (decimal.Decimal(j + 2) / decimal.Decimal(j + 1)).sqrt()
        f.write("diag %d %s\n" % (j, repr(float(v))))
    for j in range(n - 1):
        v = -(decimal.Decimal(j + 1) / decimal.Decimal(j + 2)).sqrt()
        f.write("sub %d %s\n" % (j, repr(float(v))))
