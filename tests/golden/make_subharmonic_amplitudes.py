"""Writes subharmonic_amplitudes_G4096.txt: the oracle's subharmonic wave
amplitudes (the low-frequency remedy Sec. IV-B names) for the full-size
frame's grid: 4096 x 4096, pixel pitch D/8, aliases
folded to |l| <= 2, three levels.  Calls only ``oracle/``; the full-grid
normalising sum takes minutes, which is why the GPU test reads this file.

    python tests/golden/make_subharmonic_amplitudes.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import spectra  # noqa: E402

G, DS, FOLD, LEVELS = 4096, 0.125, 2, 3


def main():
    amps = spectra.subharmonic_amplitudes(G, G, DS, FOLD, LEVELS)   # (2 modes, levels, 4 cells)
    header = (f"oracle subharmonic amplitudes, grid {G}x{G}, pitch {DS} D, fold {FOLD}, {LEVELS} levels\n"
              "rows: (mode Noll 2, 3) x level 1..3; columns: cells (1,0) (1,1) (0,1) (-1,1)\n"
              "written by tests/golden/make_subharmonic_amplitudes.py from oracle/spectra.py")
    np.savetxt(os.path.join(HERE, f"subharmonic_amplitudes_G{G}.txt"), amps.reshape(-1, 4), fmt="%.17e",
               header=header)


if __name__ == "__main__":
    main()
