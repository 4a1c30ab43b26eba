"""Regenerate the real-shift constants synth.ALPHA_STAR (coarsest grid) and
synth.ALPHA2_STAR (level 2, the second shift of Remark 4.1) with the oracle's
grid-to-grid dispersion analysis (Sec. 4.2, eq. (4.8) and (4.10)).

    python tests/golden/make_alpha.py

Prints the dictionary literal; it calls only oracle/.
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import alpha  # noqa: E402

out = {}
for G in (10.0, 32.0 / 3.0, 34.0 / 3.0, 12.0):
    out[(2, G)] = alpha.alpha_star("p5", "fw", G, lo=1.0, hi=1.3, exhaustive=True)[0]
for G in (10.0, 11.0, 12.0):
    out[(3, G)] = alpha.alpha_star("p7", "fw", G, lo=1.0, hi=1.3)[0]
out2 = {}
for G in (10.0, 32.0 / 3.0, 34.0 / 3.0, 12.0):
    out2[(2, G)] = alpha.alpha2_star("p5", "fw", G)[0]
for G in (10.0, 11.0, 12.0):
    out2[(3, G)] = alpha.alpha2_star("p7", "fw", G)[0]
for name, d in (("ALPHA_STAR", out), ("ALPHA2_STAR", out2)):
    print(name, "= {")
    for k, v in d.items():
        print("    (%d, %r): %.4f," % (k[0], k[1], v))
    print("}")
