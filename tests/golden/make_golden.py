"""Writes the regression fixtures in this folder.  Calls only the CPU oracle
and the seeded input generators; run from the repository root:
    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth   # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    w = synth.bbh_1det_4s(32)
    g = w.grid
    data = oracle.workload_data(w)
    vals = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, w.theta)
    with open(os.path.join(HERE, "bbh_1det_4s_lnl.txt"), "w") as fh:
        fh.write("# oracle lnL of the first 32 samples of the 1-detector 4 s workload (4017 bins),\n")
        fh.write("# data = seeded noise + oracle injection; written by tests/golden/make_golden.py\n")
        for x in vals:
            fh.write(f"{x:.17e}\n")


if __name__ == "__main__":
    main()
