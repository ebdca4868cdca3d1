"""Write the oracle regression fixtures in this folder.

Calls only the FP64 oracle (and the seeded input generators).  The paper prints
no worked numeric example, so these fixtures pin the oracle against its own
earlier output: any later change to its arithmetic shows up as a diff and must
be justified by a passage of the paper.

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle import im  # noqa: E402

COLS = (0, 10, 40, 44, 80)


def main():
    cfg = wl.scao_small()
    F = wl.if_stack(cfg.grid)
    I = im.im_build_misreg(F[list(COLS)], cfg.theta, cfg.pupil, cfg.p, cfg.valid)
    J = im.jacobian(F[[40]], cfg.theta, cfg.pupil, cfg.p, cfg.valid)
    with open(os.path.join(HERE, "scao_8x8_im_columns.txt"), "w") as f:
        f.write("# FP64 oracle IM columns, 8x8 SCAO workload, theta=(0.3,-0.2,0.5deg,1.01)\n")
        f.write("# columns: actuator ids " + " ".join(map(str, COLS)) + "; rows: s_x[0..51], s_y[0..51]\n")
        for r in range(I.shape[1]):
            f.write(" ".join("%.17e" % I[c, r] for c in range(len(COLS))) + "\n")
    with open(os.path.join(HERE, "scao_8x8_jacobian_act40.txt"), "w") as f:
        f.write("# FP64 oracle dIM/d(t_x, t_y, rho, m) of actuator 40, 8x8 SCAO workload\n")
        for r in range(J.shape[2]):
            f.write(" ".join("%.17e" % J[j, 0, r] for j in range(4)) + "\n")


if __name__ == "__main__":
    main()
