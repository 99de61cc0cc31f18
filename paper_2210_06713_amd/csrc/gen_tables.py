"""Writes the constant tables the PSF kernels compile in.

    python paper_2210_06713_amd/csrc/gen_tables.py

twiddle64.h / twiddle128.h: exp(-2 pi i k / N), k = 0..N-1, rounded to
binary32 (forward-DFT twiddles).  cheb32.h / cheb64.h: Chebyshev T_p(x),
p = 0..10 (phases up to radial order 10), at the pupil-window columns of the pruned DFT input (entry n is
column offset c' = n for n < N/2, else n - N, and x = c' / (N/2)), by the
three-term recurrence in binary64.
"""
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def f32(v):
    return "0.0f" if v == 0.0 else f"{float(np.float32(v)):.9e}f"


def twiddle(n):
    re, im = [], []
    for k in range(n):
        c, s = math.cos(2 * math.pi * k / n), -math.sin(2 * math.pi * k / n)
        re.append(0.0 if abs(c) < 1e-12 else c)
        im.append(0.0 if abs(s) < 1e-12 else s)
    out = ["#pragma once",
           f"// exp(-2 pi i k / {n}), k = 0..{n - 1}, rounded to binary32 (forward DFT twiddles)"]
    for name, vals in (("re", re), ("im", im)):
        out.append(f"constexpr float kW{n}{name}[{n}] = {{")
        for i in range(0, n, 4):
            out.append("    " + " ".join(f32(v) + "," for v in vals[i:i + 4]))
        out.append("};")
    return "\n".join(out) + "\n"


def cheb(n):
    half = n // 2
    name = "kChebCol" if n == 32 else f"kChebCol{n}"
    out = ["#pragma once",
           f"// Chebyshev T_p(x) at the {n} pupil-window columns of the pruned DFT input:",
           f"// entry n is column offset c' = n (n < {half}) or n - {n}, x = c'/{half}, p = 0..10.",
           f"constexpr float {name}[{n}][11] = {{"]
    for i in range(n):
        c = i if i < half else i - n
        x = c / half
        t = [1.0, x]
        for _ in range(9):
            t.append(2 * x * t[-1] - t[-2])
        out.append("    {" + ", ".join(f"{float(np.float32(v)):.9e}f" for v in t) + "},")
    out.append("};")
    return "\n".join(out) + "\n"


def main():
    files = {"twiddle64.h": twiddle(64), "twiddle128.h": twiddle(128),
             "cheb32.h": cheb(32), "cheb64.h": cheb(64)}
    for name, text in files.items():
        with open(os.path.join(HERE, name), "w") as f:
            f.write(text)


if __name__ == "__main__":
    main()
