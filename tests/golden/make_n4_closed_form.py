"""Writes n4_closed_form.txt from the closed forms derived in n4_closed_form.md."""
import math
import os

rows = []
for J in (0.7, -1.3):
    for beta in (0.0, 2.0, 10.0):
        for t in (0.0, 0.5, 3.0, 7.25):
            F = -math.cos(J * t) / (4.0 * math.cosh(beta * J / 4.0))
            den = 4.0 * math.cosh(beta * J / 4.0)
            re = (math.cos(J * t / 2) * (math.exp(-beta * J / 4) + math.exp(beta * J / 4))) / den
            im = (math.sin(J * t / 2) * (math.exp(-beta * J / 4) - math.exp(beta * J / 4))) / den
            rows.append((J, beta, t, F, re, im))
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "n4_closed_form.txt"), "w") as f:
    f.write("# J beta t F ReG ImG  (closed forms in n4_closed_form.md)\n")
    for r in rows:
        f.write(" ".join(repr(x) for x in r) + "\n")
