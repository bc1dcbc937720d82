"""Writes n4_unreg_imag.txt from the closed forms derived in n4_unreg_imag.md."""
import math
import os

rows = []
for J in (0.7, -1.3):
    for beta in (0.0, 2.0, 10.0):
        for s in (0.0, 0.5, 1.0, 3.0, 7.25):
            reF = -math.cos(J * s) / 4.0
            imF = math.sin(J * s) * math.tanh(beta * J / 4.0) / 4.0
            G = math.cosh((2 * s - beta) * J / 4.0) / (2.0 * math.cosh(beta * J / 4.0)) if s <= beta else float("nan")
            rows.append((J, beta, s, reF, imF, G))
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "n4_unreg_imag.txt"), "w") as f:
    f.write("# J beta s ReF_u ImF_u G(tau=s)  (closed forms in n4_unreg_imag.md)\n")
    for r in rows:
        f.write(" ".join(repr(x) for x in r) + "\n")
