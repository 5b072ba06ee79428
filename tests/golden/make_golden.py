"""Writes the golden fixtures of this directory from the oracle alone.

The paper prints no worked numerical example of the DG operators, so these
values are not the paper's: they are the FP64 oracle's results on a tiny
seeded case, stored so that a later change to the oracle's arithmetic shows
up as a difference (and the library can be held to the same numbers).
Inputs come from the seeded generators in paper_2512_17101_amd/workload.py,
which hold none of the method's arithmetic.

Case: periodic box [0, 10]^3 of 3^3 cubes x 6 = 162 tets (Kuhn subdivision,
5 % vertex jitter, seed 7), order p = 1, isentropic vortex (strength 5, free
stream Mach 0.5).  Files:
  ref_p1.txt           reference element of order 1: rst, Dr, Ds, Dt, LIFT, Fmask
  euler_p1_3cubed.txt  the Euler RHS of the whole mesh and the state after
                       one LSRK(5,4) step of dt = 0.05, stored for elements
                       0..15 (layout [5][16][4], row-major)

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import euler as oe, lsrk as olsrk, mesh as om, reference_element as ore  # noqa: E402
from paper_2512_17101_amd import workload as wl  # noqa: E402

P = 1
N = 3
NE = 16  # elements stored
SEED = 7
DT = 0.05


def case():
    xyz, vid = wl.kuhn_box_mesh(N, 10.0, 0.05, SEED)
    ops = ore.operators(P)
    geo = om.geometry(xyz)
    conn = om.connectivity(vid, P)
    q = wl.vortex_state(om.node_coordinates(xyz, ops["rst"]))
    return xyz, vid, ops, geo, conn, q


def _block(name, a):
    a = np.asarray(a)
    lines = [f"# {name} shape {' '.join(str(s) for s in a.shape)}"]
    lines += [f"{v:.17g}" for v in a.ravel()]
    return "\n".join(lines) + "\n"


def read(path):
    """{name: array} of a fixture file written by this script."""
    out, name, shape, vals = {}, None, None, []
    for line in open(path):
        line = line.strip()
        if line.startswith("#"):
            parts = line[1:].split()
            if len(parts) < 2 or parts[1] != "shape":
                continue  # a comment line
            if name is not None:
                out[name] = np.array(vals, dtype=np.float64).reshape(shape)
            name, shape, vals = parts[0], tuple(int(s) for s in parts[2:]), []
        elif line:
            vals.append(float(line))
    if name is not None:
        out[name] = np.array(vals, dtype=np.float64).reshape(shape)
    return out


def main():
    xyz, vid, ops, geo, conn, q = case()
    ref = (_block("rst", ops["rst"]) + _block("Dr", ops["Dr"]) + _block("Ds", ops["Ds"]) + _block("Dt", ops["Dt"])
           + _block("LIFT", ops["LIFT"]) + _block("Fmask", np.asarray(ops["Fmask"], dtype=np.float64)))
    head = ("# reference tetrahedron of order 1 (oracle/reference_element.py), written by make_golden.py\n")
    open(os.path.join(HERE, "ref_p1.txt"), "w").write(head + ref)
    r = oe.rhs(ops, geo, conn, q)
    q1, _ = olsrk.lsrk_step(lambda qq, tt: oe.rhs(ops, geo, conn, qq), q, 0.0, DT)
    head = ("# Euler p = 1 on the periodic 3^3 x 6 Kuhn box (jitter 5 %, seed 7), isentropic vortex:\n"
            "# rhs(q) and q after one LSRK(5,4) step of dt = 0.05 on elements 0..15, from oracle/euler.py and\n"
            "# oracle/lsrk.py, written by make_golden.py\n")
    open(os.path.join(HERE, "euler_p1_3cubed.txt"), "w").write(head + _block("rhs", r[:, :NE]) + _block("q1", q1[:, :NE]))


if __name__ == "__main__":
    main()
