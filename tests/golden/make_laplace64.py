"""Write laplace64_features.json: closed-form Table 1 quantities of the
5-point Laplacian on a 64 x 64 grid (natural ordering r = i*64 + j).

Derived from the grid geometry alone (which neighbours exist for each grid
point), with exact rationals; it calls neither the oracle nor the library.
Row classes: interior (5 entries, span 128), left/right edges (4 entries,
span 128), top/bottom edges (4 entries, span 65), corners (3 entries, spans
64 or 65).  A "miss" is a gap of more than 16 columns (8-byte x elements,
128-byte line), per the Table 1 caption.
"""
import json
import os
from fractions import Fraction

n = 64
rows = []
for i in range(n):
    for j in range(n):
        r = i * n + j
        cols = sorted(c for c, ok in [(r - n, i > 0), (r - 1, j > 0), (r, True),
                                      (r + 1, j < n - 1), (r + n, i < n - 1)] if ok)
        rows.append(cols)
N = n * n
L = [len(c) for c in rows]
bw = [c[-1] - c[0] for c in rows]
miss = sum(1 for c in rows for a, b in zip(c, c[1:]) if (b - a) * 8 > 128)
avg = Fraction(sum(L), N)
var = sum((Fraction(t) - avg) ** 2 for t in L) / N
bavg = Fraction(sum(bw), N)
bvar = sum((Fraction(t) - bavg) ** 2 for t in bw) / N
disp = sum(Fraction(a, b + 1) for a, b in zip(L, bw)) / N
hist = {}
for b in bw:
    hist[b] = hist.get(b, 0) + 1
out = {
    "source": "Table 1 definitions on the 5-point Laplacian, 64 x 64 grid",
    "N": N, "NNZ": sum(L), "nnz_min": min(L), "nnz_max": max(L),
    "nnz_avg": [avg.numerator, avg.denominator],
    "nnz_var": [var.numerator, var.denominator],
    "S_bw": sum(bw), "bw_avg": float(bavg),
    "bw_var": [bvar.numerator, bvar.denominator],
    "bw_histogram": {str(k): v for k, v in sorted(hist.items())},
    "dispersion_avg": [disp.numerator, disp.denominator],
    "S_miss": miss,
}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       "laplace64_features.json"), "w") as f:
    json.dump(out, f, indent=1)
print(out)
