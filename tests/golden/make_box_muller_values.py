"""Write tests/golden/box_muller_values.txt: hand-evaluated proposal normals.

    python tests/golden/make_box_muller_values.py

The serving step draws its Metropolis proposals from Philox4x32-10 (Salmon
et al., SC'11) with counter (walker, step, call, 0) and key (seed low word,
seed high word).  Each call's four 32-bit output words give two uniforms
u = ((a >> 5) 2^26 + (b >> 6) + 1/2) / 2^53 and the Box-Muller pair
(Box and Muller, Ann. Math. Stat. 29, 1958)

    xi_0 = sqrt(-2 ln u_1) cos(2 pi u_2),   xi_1 = sqrt(-2 ln u_1) sin(2 pi u_2).

This script evaluates that map in 40-digit arithmetic (mpmath) from the
output words; it shares nothing with the oracle's own Box-Muller code.  The
output words of the first counter are the published known-answer vector
(counter 0, key 0); those of the second come from the oracle's Philox, which
the published vectors pin (test_philox_known_answers).
"""

import os
import sys

import mpmath

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.vmc import philox4x32_10  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
mpmath.mp.dps = 40

# (seed, walker, step, call): the first is the published all-zero vector
CASES = [(0, 0, 0, 0), (0x0123456789ABCDEF, 3, 17, 1)]


def uniform(a, b):
    return (mpmath.mpf(a >> 5) * 2**26 + (b >> 6) + mpmath.mpf(1) / 2) / mpmath.mpf(2) ** 53


def main():
    lines = ["# Box-Muller normals of the serving step's proposal stream, 40-digit evaluation.",
             "# Written by make_box_muller_values.py (mpmath, from the Philox output words).",
             "# Columns: seed walker step call out0 out1 out2 out3 (hex) xi0 xi1"]
    for seed, w, step, call in CASES:
        key = (seed & 0xFFFFFFFF, seed >> 32)
        words = philox4x32_10((w, step, call, 0), key)
        u1, u2 = uniform(words[0], words[1]), uniform(words[2], words[3])
        rad = mpmath.sqrt(-2 * mpmath.log(u1))
        xi0 = rad * mpmath.cos(2 * mpmath.pi * u2)
        xi1 = rad * mpmath.sin(2 * mpmath.pi * u2)
        lines.append(f"{seed:016x} {w} {step} {call} " + " ".join(f"{x:08x}" for x in words)
                     + f" {mpmath.nstr(xi0, 25)} {mpmath.nstr(xi1, 25)}")
    with open(os.path.join(HERE, "box_muller_values.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
